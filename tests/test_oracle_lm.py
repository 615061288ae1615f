"""Pins of the oracle's Levenberg-Marquardt step for Eq. EQHOC (Sec. 5 "Optimization
Algorithm": the J^T J + lambda I update on the sum-of-squares collocation objective).

The step is an iteration, so it is pinned by what its result must satisfy and
by independent routes to the same result: the written-out residual Jacobian
against central differences of the residuals; at order 2 the root of the
residual is the Eq. EQ minimizer (reached by L-BFGS and a Newton polish of the
Alg. 1 gradient); at higher orders L-BFGS reaches the same collocation root
where it converges; the LM result is a fixed point of dense Newton on the
residual equations; and an LM rollout has the convergence order of the
collocation method against an RK4 solution of the continuous equations.
"""
import math

import numpy as np
import pytest

import refkin
from oracle.oracle import Oracle, collocation
from paper_1709_04145_amd import workloads as W


def _tree(n_models=3, seed=3, max_links=5):
    return W.random_tree_models(n_models, seed, max_links=max_links, ball_prob=0.4)


@pytest.mark.parametrize("K", [3, 4])
def test_residual_jacobian_matches_central_differences(K):
    d = _tree(2, seed=60 + K, max_links=4)
    rng = np.random.default_rng(61 + K)
    qp, qc = (rng.uniform(-1, 1, d.n_dofs) for _ in range(2))
    qu = rng.uniform(-1, 1, (K - 1, d.n_dofs))
    tau = rng.uniform(-1, 1, d.n_dofs)
    dt = 0.05
    orc = Oracle(d)
    R, J = orc.eqhoc_residual_jacobian(K, dt, qp, qc, qu, tau)
    E, g = orc.eqhoc_objective_grad(K, dt, qp, qc, qu, tau)
    do = d.dof_offset
    U = K - 1
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        r = R[:, sl].reshape(-1)
        assert abs(E[i] - r @ r) <= 1e-13 * max(1e-300, r @ r)
        # dE/dq = 2 J^T r, the objective's own gradient
        assert np.allclose(2 * J[i].T @ r, g[:, sl].reshape(-1), rtol=0, atol=1e-10 * np.abs(g).max())
    h = 1e-6
    for trial in range(3):
        v = rng.standard_normal((U, d.n_dofs))
        Rp, _ = orc.eqhoc_residual_jacobian(K, dt, qp, qc, qu + h * v, tau, jacobian=False)
        Rm, _ = orc.eqhoc_residual_jacobian(K, dt, qp, qc, qu - h * v, tau, jacobian=False)
        fd = (Rp - Rm) / (2 * h)
        for i in range(d.n_models):
            sl = slice(do[i], do[i + 1])
            jv = J[i] @ v[:, sl].reshape(-1)
            ref = fd[:, sl].reshape(-1)
            assert np.max(np.abs(jv - ref)) <= 1e-6 * max(1.0, np.abs(ref).max()), trial


def test_order_two_lm_reaches_the_eq_minimizer():
    """K = 2: the residual is the Eq. EQ gradient, so LM on its square reaches
    the Eq. EQ minimizer q* that L-BFGS and a Newton polish of the Alg. 1
    gradient find.  The squared objective's relative gradient tolerance leaves
    the residual |grad E(q)| of the result, so the result is within the
    first-order bound |H(q*)^-1| |grad E(q)| of q* (50% margin), and dense Newton
    on the residual equations from it lands on q*."""
    wl = W.config(2, n_models=5)
    orc = Oracle(wl.model)
    dt = wl.step.dt
    qs, _ = orc.rollout(wl.q0, 2, dt)
    qp, qc = qs[-2], qs[-1]
    ql, st = orc.step_lm(2, qp, qc, dt, tol=1e-10)
    assert np.all(st["flag"] == 1), st
    qn, _ = orc.step(qp, qc, dt, tol=1e-11)
    qx, _ = orc.newton_polish(qn, qp, qc, dt)
    _, g, _ = orc.objective_grad(ql[0], qp, qc, dt)
    H = orc.hessian(qx, qp, qc, dt)
    do = wl.model.dof_offset
    for i in range(wl.model.n_models):
        sl = slice(do[i], do[i + 1])
        bound = 1.5 * np.linalg.norm(np.linalg.inv(H[i]), 2) * np.linalg.norm(g[sl])
        assert np.linalg.norm(ql[0][sl] - qx[sl]) <= bound + 1e-12, i
    qr = _newton_on_residual(orc, 2, dt, qp, qc, ql)
    assert np.max(np.abs(qr[0] - qx)) < 1e-10


@pytest.mark.parametrize("K", [3, 4])
def test_lm_and_lbfgs_reach_the_same_collocation_root(K):
    """Small trees at a step size where L-BFGS converges: both optimizers of Sec. 5
    end at the same root of the collocation residual (Eq. HOC)."""
    d = _tree(3, seed=70 + K, max_links=4)
    rng = np.random.default_rng(71 + K)
    q0 = rng.uniform(-0.5, 0.5, d.n_dofs)
    dt = 0.005
    orc = Oracle(d)
    ql, sl_ = orc.step_lm(K, q0, q0, dt, tol=1e-8)
    qb, sb = orc.step_hoc(K, q0, q0, dt, tol=1e-8, max_iter=5000)
    assert np.all(sl_["flag"] == 1) and np.all(sb["flag"] == 1), (sl_, sb)
    # both polished by dense Newton on the residual equations: one root, and
    # each result within its tolerance-implied distance |J^-1| |r| of it
    pl = _newton_on_residual(orc, K, dt, q0, q0, ql)
    pb = _newton_on_residual(orc, K, dt, q0, q0, qb)
    assert np.max(np.abs(pl - pb)) < 1e-11, np.max(np.abs(pl - pb))
    _, J = orc.eqhoc_residual_jacobian(K, dt, q0, q0, pl)
    do = d.dof_offset
    for q in (ql, qb):
        R, _ = orc.eqhoc_residual_jacobian(K, dt, q0, q0, q, jacobian=False)
        for i in range(d.n_models):
            sl = slice(do[i], do[i + 1])
            bound = 1.5 * np.linalg.norm(np.linalg.inv(J[i]), 2) * np.linalg.norm(R[:, sl])
            assert np.linalg.norm(q[:, sl] - pl[:, sl]) <= bound + 1e-13, i


def _newton_on_residual(orc, K, dt, qp, qc, qu, iters=3):
    """Dense Newton on the residual equations r(q) = 0, model by model."""
    do = orc.desc.dof_offset
    U = K - 1
    q = qu.copy()
    for _ in range(iters):
        R, J = orc.eqhoc_residual_jacobian(K, dt, qp, qc, q)
        for i in range(orc.n_models):
            sl = slice(do[i], do[i + 1])
            dx = np.linalg.solve(J[i], -R[:, sl].reshape(-1))
            q[:, sl] += dx.reshape(U, -1)
    return q


def test_lm_converges_on_the_branching_workload_to_a_newton_fixed_point():
    """The 2048-tree workload's trees (30-60 links, ball joints, K = 4, dt = 0.05),
    first two steps from rest for four of them: every LM step converges, and
    dense Newton on the residual equations started at the LM result moves it by
    no more than its tolerance implies; plain LM (no geodesic acceleration)
    reaches the same root where it converges within the cap."""
    wl = W.config(3, n_models=4)
    orc = Oracle(wl.model)
    dt, K = wl.step.dt, 4
    qp = qc = wl.q0
    do = wl.model.dof_offset
    for step in range(2):
        qu, st = orc.step_lm(K, qp, qc, dt, tol=1e-10)
        assert np.all(st["flag"] == 1), st
        qn = _newton_on_residual(orc, K, dt, qp, qc, qu)
        R, _ = orc.eqhoc_residual_jacobian(K, dt, qp, qc, qu, jacobian=False)
        _, J = orc.eqhoc_residual_jacobian(K, dt, qp, qc, qn)
        for i in range(wl.model.n_models):
            sl = slice(do[i], do[i + 1])
            bound = 1.5 * np.linalg.norm(np.linalg.inv(J[i]), 2) * np.linalg.norm(R[:, sl])
            assert np.linalg.norm(qn[:, sl] - qu[:, sl]) <= bound + 1e-12, (step, i)
        if step == 0:
            qpl, stp = orc.step_lm(K, qp, qc, dt, tol=1e-10, geodesic=False, max_iter=600)
            ok = stp["flag"] == 1
            Rp, _ = orc.eqhoc_residual_jacobian(K, dt, qp, qc, qpl, jacobian=False)
            for i in np.nonzero(ok)[0]:
                sl = slice(do[i], do[i + 1])
                bound = 1.5 * np.linalg.norm(np.linalg.inv(J[i]), 2) * (np.linalg.norm(R[:, sl]) +
                                                                        np.linalg.norm(Rp[:, sl]))
                assert np.linalg.norm(qpl[:, sl] - qu[:, sl]) <= bound + 1e-12, i
        qp, qc = qu[K - 3], qu[K - 2]


@pytest.mark.slow
def test_lm_rollout_has_the_collocation_order():
    """An LM rollout tracks the continuous equations (RK4 reference) with error
    O(dt^(K-1)): order ~2 for K = 3, and K = 4 far below K = 3 at the same dt."""
    d = W._assemble([W.chain_model([1.0, 0.8, 0.6], 0.1, [1000.0] * 3, W.alternating_axes(3, "y"))])
    q0 = np.array([0.4, -0.3, 0.2])
    T = 0.2
    ref = refkin.rk4_reference(d, q0, T, 0.001)
    orc = Oracle(d, threads=1)

    def err(K, dt):
        tau, _ = collocation(K)
        s = -tau[0] * dt
        qprev = refkin.rk4_reference(d, q0, s, s / max(1, int(round(s / 0.0005))))
        qs, sts = orc.rollout_lm(K, qprev, q0, int(round(T / dt)), dt, tol=1e-10)
        # converged, or stopped at the float64 floor of the squared residual
        assert all(np.all((st["flag"] == 1) | (st["flag"] == 2)) for st in sts)
        return float(np.max(np.abs(qs[-1] - ref)))

    e3 = [err(3, dt) for dt in (0.01, 0.005)]
    assert 1.7 < math.log2(e3[0] / e3[1]) < 2.4, e3
    e4 = err(4, 0.01)
    assert e4 < 1e-2 * e3[0], (e3[0], e4)


# ---------------------------------------------------------------- order 2 (Eq. EQ)
# Sec. 5 applies Levenberg-Marquardt to Eq. EQ directly: its kinetic term is an
# integral of squares whose Gauss-Newton matrix J^T J is the joint-space inertia
# H_q(q).  step_lm_eq is pinned by the minimizer it must reach (the Newton-polished
# L-BFGS result, within the tolerance-implied distance), by its first step in the
# two limits of lambda (the Gauss-Newton step with the inertia of the test's own
# Jacobian-form kinematics, and a gradient step of length |g| / lambda), and by the
# degenerate start that is already a minimizer.


def _eq_bound_check(orc, d, q, qp, qc, dt, tau=None):
    qn, _ = orc.step(qp, qc, dt, tau, tol=1e-11, max_iter=2000)
    qx, _ = orc.newton_polish(qn, qp, qc, dt, tau)
    _, g, _ = orc.objective_grad(q, qp, qc, dt, tau)
    H = orc.hessian(qx, qp, qc, dt)
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        bound = 1.5 * np.linalg.norm(np.linalg.inv(H[i]), 2) * np.linalg.norm(g[sl])
        assert np.linalg.norm(q[sl] - qx[sl]) <= bound + 1e-12, (i, np.linalg.norm(q[sl] - qx[sl]), bound)


def test_eq_lm_reaches_the_eq_minimizer_on_chains():
    """Chains of the 4096-chain workload, third step of a rollout from rest."""
    wl = W.config(2, n_models=5)
    orc = Oracle(wl.model)
    dt = wl.step.dt
    qs, _ = orc.rollout(wl.q0, 2, dt)
    qp, qc = qs[-2], qs[-1]
    q, st = orc.step_lm_eq(qp, qc, dt, tol=1e-8)
    assert np.all(st["flag"] == 1), st
    # Gauss-Newton on a nearly consistent least-squares problem: few iterations
    assert np.all(st["iterations"] <= 40), st["iterations"]
    _eq_bound_check(orc, wl.model, q, qp, qc, dt)


def test_eq_lm_reaches_the_eq_minimizer_on_trees_with_torques():
    d = _tree(4, seed=140, max_links=6)
    rng = np.random.default_rng(141)
    qc = rng.uniform(-1, 1, d.n_dofs)
    qp = qc - 0.02 * rng.standard_normal(d.n_dofs)
    tau = rng.uniform(-20, 20, d.n_dofs)
    orc = Oracle(d)
    dt = 0.01
    q, st = orc.step_lm_eq(qp, qc, dt, tau, tol=1e-7)  # 1e-8 is below one tree's float64 floor
    assert np.all(st["flag"] == 1), st
    _eq_bound_check(orc, d, q, qp, qc, dt, tau)


def test_eq_lm_at_a_minimizer_start_takes_no_iteration():
    """No gravity, no torque, at rest: the warm start q_0 is the minimizer (E = 0)."""
    d = W.random_tree_models(3, 142, max_links=5, ball_prob=0.4, gravity=[0.0, 0.0, 0.0])
    q0 = np.random.default_rng(143).uniform(-1, 1, d.n_dofs)
    q, st = Oracle(d).step_lm_eq(q0, q0, 0.01)
    assert np.all(st["flag"] == 1) and np.all(st["iterations"] == 0), st
    assert np.array_equal(q, q0)


@pytest.mark.parametrize("lambda0", [1e-20, 1e4])
def test_eq_lm_first_step_in_the_limits_of_lambda(lambda0):
    """One iteration from the warm start: with lambda at its floor (1e-15 max diag)
    the step is the Gauss-Newton step -H_q^-1 g; with lambda = 1e4 max diag it is
    the gradient step -g / lambda up to |H_q| / lambda.  H_q here comes from the test's own kinematics
    (Jacobian form of the inertia), g from the pinned Alg. 1 gradient."""
    d = _tree(3, seed=144, max_links=5)
    rng = np.random.default_rng(145)
    qc = rng.uniform(-1, 1, d.n_dofs)
    qp = qc - 0.01 * rng.standard_normal(d.n_dofs)
    dt = 0.01
    orc = Oracle(d)
    q, st = orc.step_lm_eq(qp, qc, dt, tol=1e-14, max_iter=1, lambda0=lambda0)
    assert np.all(st["iterations"] == 1) and np.all(st["evaluations"] == 2), st
    warm = 2 * qc - qp
    _, g, _ = orc.objective_grad(warm, qp, qc, dt)
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        Hq = refkin.inertia_matrix(d.subset([i]), warm[sl], 0)
        dmax = float(np.max(np.diag(Hq)))
        if lambda0 < 1e-15:
            ref = -np.linalg.solve(Hq, g[sl])
            tol = 1e-9
        else:
            ref = -g[sl] / (lambda0 * dmax)
            tol = 1.01 * np.linalg.norm(Hq, 2) / (lambda0 * dmax) + 1e-8
        assert np.linalg.norm((q[sl] - warm[sl]) - ref) <= tol * np.linalg.norm(ref), i
