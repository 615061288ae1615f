"""Levenberg-Marquardt steps of the order-K collocation objective (Eq. EQHOC,
Sec. 5 "Optimization Algorithm") on the GPU against the FP64 CPU oracle's LM.

A step is determined by its tolerance only (a relative tolerance on the gradient
of a sum of squares leaves the residual r of the result), so the check is what
the tolerance implies: both sides converge, and the GPU's configurations are
within 1.5 |J(q*)^-1| |r(q_gpu)| of the oracle's root q* (the oracle's LM result
polished by dense Newton on the residual equations, J the oracle's written-out
Jacobian, r the oracle's residual at the GPU's configurations).  Where both sides
follow the same iterates (the same Jacobian up to rounding: the GPU assembles it
from composite sums, the oracle from its pose derivatives), the iteration counts
agree, which checks the GPU's Jacobian.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_1709_04145_amd import abd
from paper_1709_04145_amd import workloads as W
from test_gpu_long import hanging_chains
from test_gpu_parity import cu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    abd.load()
    yield


def _gpu_step(d, K, qp, qc, dt, tol, max_iter=300):
    m = abd.Model(d)
    out = torch.zeros((K - 1, d.n_dofs), dtype=torch.float64, device="cuda")
    st = m.new_stats()
    m.step(cu(np.concatenate([qp, qc])), out, abd.StepOptions(dt=dt, order_K=K, tol=tol, max_iter=max_iter,
                                                                solver=abd.SOLVER_LM), stats=st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), m.read_stats(st, d.n_models)


def _newton_root(orc, K, dt, qp, qc, qu, iters=3):
    do = orc.desc.dof_offset
    q = qu.copy()
    for _ in range(iters):
        R, J = orc.eqhoc_residual_jacobian(K, dt, qp, qc, q)
        for i in range(orc.n_models):
            sl = slice(do[i], do[i + 1])
            q[:, sl] += np.linalg.solve(J[i], -R[:, sl].reshape(-1)).reshape(K - 1, -1)
    return q


def _check_against_root(d, K, dt, qp, qc, got, ref):
    orc = Oracle(d)
    root = _newton_root(orc, K, dt, qp, qc, ref)
    _, J = orc.eqhoc_residual_jacobian(K, dt, qp, qc, root)
    R, _ = orc.eqhoc_residual_jacobian(K, dt, qp, qc, got, jacobian=False)
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        dist = float(np.linalg.norm(got[:, sl] - root[:, sl]))
        bound = 1.5 * np.linalg.norm(np.linalg.inv(J[i]), 2) * float(np.linalg.norm(R[:, sl]))
        say(f"  model {i}: |q_gpu - q*| {dist:.2e}, tolerance-implied bound {bound:.2e}")
        assert dist <= bound + 1e-13, (i, dist, bound)
    return root


ORDER4_OFF = ("order 4 with ABD_SOLVER_LM is switched off (ABD_ENOTSUP): its first GPU run faulted "
              "(illegal memory access) and the cause has not been found")


@pytest.mark.parametrize("K", [3, pytest.param(4, marks=pytest.mark.skip(reason=ORDER4_OFF))])
def test_lm_step_small_trees_matches_oracle(K):
    d = W.random_tree_models(6, 80 + K, max_links=6, ball_prob=0.4)
    q0 = np.random.default_rng(81 + K).uniform(-0.5, 0.5, d.n_dofs)
    dt, tol = 0.01, 1e-8
    say(f"lm small trees K={K}")
    ref, rst = Oracle(d).step_lm(K, q0, q0, dt, tol=tol)
    got, st = _gpu_step(d, K, q0, q0, dt, tol)
    assert np.all(rst["flag"] == 1), rst
    assert np.all(st["flag"] == abd.FLAG_CONVERGED), st
    _check_against_root(d, K, dt, q0, q0, got, ref)
    assert np.all(np.abs(st["iterations"] - rst["iterations"]) <= 2), (st["iterations"], rst["iterations"])


def test_lm_step_chains_moving_matches_oracle():
    """Serial chains of 10..40 hinges with a velocity (distinct known points), K = 3."""
    K = 3
    d = W.random_chain_models(5, 91, lo=10, hi=40)
    rng = np.random.default_rng(92)
    qc = rng.uniform(-1, 1, d.n_dofs)
    qp = qc - 0.01 * rng.standard_normal(d.n_dofs)
    dt, tol = 0.01, 1e-8
    say("lm chains K=3")
    ref, rst = Oracle(d).step_lm(K, qp, qc, dt, tol=tol)
    got, st = _gpu_step(d, K, qp, qc, dt, tol)
    assert np.all(rst["flag"] == 1) and np.all(st["flag"] == abd.FLAG_CONVERGED), (rst, st)
    _check_against_root(d, K, dt, qp, qc, got, ref)


@pytest.mark.parametrize("K", [3, pytest.param(4, marks=pytest.mark.skip(reason=ORDER4_OFF))])
def test_lm_branching_workload_two_steps_teacher_forced(K):
    """Four trees of the 2048-tree workload (30..60 links with ball joints, 90..180
    DOFs, dt = 0.05): the first two steps from rest, each started on both sides
    from the oracle's known points; every step converges on both sides."""
    wl = W.config(3, n_models=4)
    d, dt, tol = wl.model, wl.step.dt, wl.step.tol
    orc = Oracle(d)
    qp = qc = wl.q0
    for step in range(2):
        say(f"lm workload trees step {step}")
        ref, rst = orc.step_lm(K, qp, qc, dt, tol=tol)
        got, st = _gpu_step(d, K, qp, qc, dt, tol)
        say(f"  iterations gpu {st['iterations'].tolist()} oracle {rst['iterations'].tolist()}")
        assert np.all(rst["flag"] == 1), rst
        assert np.all(st["flag"] == abd.FLAG_CONVERGED), st
        _check_against_root(d, K, dt, qp, qc, got, ref)
        qp, qc = ref[K - 3], ref[K - 2]


def test_lm_rollout_equals_step_loop_bitwise():
    K = 3
    d = W.random_tree_models(5, 95, max_links=6, ball_prob=0.4)
    q0 = np.random.default_rng(96).uniform(-0.5, 0.5, d.n_dofs)
    opts = abd.StepOptions(dt=0.01, order_K=K, solver=abd.SOLVER_LM)
    say("lm rollout vs step loop")
    m = abd.Model(d)
    traj, _ = m.rollout(cu(np.concatenate([q0, q0])), 3, opts)
    torch.cuda.synchronize()
    traj = traj.cpu().numpy()
    qp = qc = q0
    for k in range(3):
        out = torch.zeros((K - 1, d.n_dofs), dtype=torch.float64, device="cuda")
        m.step(cu(np.concatenate([qp, qc])), out, opts)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert np.array_equal(o, traj[k]), k
        qp, qc = o[K - 3], o[K - 2]


def test_lm_unsupported_cases_are_rejected():
    d = W.random_chain_models(2, 97, lo=3, hi=5)
    m = abd.Model(d)
    q = cu(np.zeros(d.n_dofs))
    out = torch.zeros(d.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(abd.AbdError) as e:  # LM computes in float64 only
        m.step(torch.cat([q, q]), out, abd.StepOptions(dt=0.01, solver=abd.SOLVER_LM, precision=abd.MIXED))
    assert e.value.code == abd.ABD_ENOTSUP
    with pytest.raises(abd.AbdError) as e:
        m.step(torch.cat([q, q]), out, abd.StepOptions(dt=0.01, solver=7))
    assert e.value.code == abd.ABD_EINVAL
    out4 = torch.zeros((3, d.n_dofs), dtype=torch.float64, device="cuda")
    with pytest.raises(abd.AbdError) as e:  # order 4 is switched off: rejected on the host, nothing launched
        m.step(torch.cat([q, q]), out4, abd.StepOptions(dt=0.01, order_K=4, solver=abd.SOLVER_LM))
    assert e.value.code == abd.ABD_ENOTSUP
    out3 = torch.zeros((2, d.n_dofs), dtype=torch.float64, device="cuda")
    st = m.new_rollout_stats(1)
    with pytest.raises(abd.AbdError) as e:
        m.rollout_noalloc(torch.cat([q, q]), 1, abd.StepOptions(dt=0.01, order_K=3, solver=abd.SOLVER_LM), out3, st)
    assert e.value.code == abd.ABD_ENOTSUP
    with pytest.raises(abd.AbdError) as e:  # order 2 too: its matrices are allocated on first use
        m.rollout_noalloc(torch.cat([q, q]), 1, abd.StepOptions(dt=0.01, solver=abd.SOLVER_LM), out, st)
    assert e.value.code == abd.ABD_ENOTSUP


# ---------------------------------------------------------------- order 2 (Eq. EQ)
# Levenberg-Marquardt on Eq. EQ with the joint-space inertia H_q as J^T J, against
# the oracle's step_lm_eq.  The result is fixed by its tolerance: both sides
# converge and the GPU's configuration lies within 1.5 |H(q*)^-1| |grad E(q_gpu)|
# of the minimizer q* (the oracle's LM result polished by dense Newton with the
# oracle's written-out Hessian).  Both sides take the same iterates up to
# rounding (the GPU assembles H_q from composite sums, the oracle from its pose
# derivatives), so the iteration counts agree to within 2.


def _gpu_step_eq(d, qp, qc, dt, tol, tau=None, max_iter=300):
    m = abd.Model(d)
    out = torch.zeros(d.n_dofs, dtype=torch.float64, device="cuda")
    st = m.new_stats()
    m.step(cu(np.concatenate([qp, qc])), out, abd.StepOptions(dt=dt, tol=tol, max_iter=max_iter,
                                                                solver=abd.SOLVER_LM),
           tau=None if tau is None else cu(tau), stats=st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), m.read_stats(st, d.n_models)


def _check_eq_minimizer(d, qp, qc, dt, got, ref, tau=None):
    orc = Oracle(d)
    root, _ = orc.newton_polish(ref, qp, qc, dt, tau)
    H = orc.hessian(root, qp, qc, dt)
    _, g, _ = orc.objective_grad(got, qp, qc, dt, tau)
    do = d.dof_offset
    worst = 0.0
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        dist = float(np.linalg.norm(got[sl] - root[sl]))
        bound = 1.5 * np.linalg.norm(np.linalg.inv(H[i]), 2) * float(np.linalg.norm(g[sl]))
        worst = max(worst, dist / max(bound, 1e-300))
        assert dist <= bound + 1e-13, (i, dist, bound)
    say(f"  max |q_gpu - q*| / bound {worst:.2f}")


def _eq_case(d, qp, qc, dt, tol, tau=None):
    ref, rst = Oracle(d).step_lm_eq(qp, qc, dt, tau, tol=tol)
    got, st = _gpu_step_eq(d, qp, qc, dt, tol, tau)
    say(f"  iterations gpu {st['iterations'].tolist()[:12]} oracle {rst['iterations'].tolist()[:12]}")
    assert np.all(rst["flag"] == 1), rst
    assert np.all(st["flag"] == abd.FLAG_CONVERGED), st
    _check_eq_minimizer(d, qp, qc, dt, got, ref, tau)
    assert np.all(np.abs(st["iterations"] - rst["iterations"]) <= 2), (st["iterations"], rst["iterations"])


def test_lm_eq_chain_workload_matches_oracle():
    """32 chains of the 4096-chain workload (10..50 hinges, dt = 0.01), third step."""
    wl = W.config(2, n_models=32)
    say("lm eq chain workload")
    qs, _ = Oracle(wl.model).rollout(wl.q0, 2, wl.step.dt)
    _eq_case(wl.model, qs[-2], qs[-1], wl.step.dt, 1e-7)  # 1e-8 is below some chains' float64 floor


def test_lm_eq_trees_with_torques_match_oracle():
    d = W.random_tree_models(12, 150, max_links=8, ball_prob=0.4)
    rng = np.random.default_rng(151)
    qc = rng.uniform(-1, 1, d.n_dofs)
    qp = qc - 0.02 * rng.standard_normal(d.n_dofs)
    tau = rng.uniform(-20, 20, d.n_dofs)
    say("lm eq trees with torques")
    _eq_case(d, qp, qc, 0.01, 1e-7, tau)


def test_lm_eq_large_step_chains_match_oracle():
    """Chains of 10 and 40 hinges at dt = 0.05 (the step size of the paper's LM /
    L-BFGS comparison), moving."""
    d = W.random_chain_models(6, 152, lo=10, hi=40)
    rng = np.random.default_rng(153)
    qc = rng.uniform(-1, 1, d.n_dofs)
    qp = qc - 0.05 * rng.standard_normal(d.n_dofs)
    say("lm eq chains dt 0.05")
    _eq_case(d, qp, qc, 0.05, 1e-7)


def test_lm_eq_long_chains_match_oracle():
    """Chains of 65, 300 and 600 hinges: two, eight and sixteen waves per model."""
    d, q0 = hanging_chains([65, 300, 600], 154)
    rng = np.random.default_rng(155)
    qc = q0 + 0.05 * rng.standard_normal(d.n_dofs)
    say("lm eq long chains")
    _eq_case(d, qc, qc, 0.01, 1e-5)  # the 300-hinge chain's float64 floor lies near 2e-5


def test_lm_eq_rollout_equals_step_loop_bitwise():
    d = W.random_tree_models(5, 156, max_links=6, ball_prob=0.4)
    q0 = np.random.default_rng(157).uniform(-0.5, 0.5, d.n_dofs)
    opts = abd.StepOptions(dt=0.01, solver=abd.SOLVER_LM)
    say("lm eq rollout vs step loop")
    m = abd.Model(d)
    traj, _ = m.rollout(cu(np.concatenate([q0, q0])), 3, opts)
    torch.cuda.synchronize()
    traj = traj.cpu().numpy()
    qp = qc = q0
    for k in range(3):
        out = torch.zeros(d.n_dofs, dtype=torch.float64, device="cuda")
        m.step(cu(np.concatenate([qp, qc])), out, opts)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        assert np.array_equal(o, traj[k]), k
        qp, qc = qc, o
