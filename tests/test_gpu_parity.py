"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (stated per quantity):
  * objective and gradient, float64 kernels: 1e-12 relative (objective relative
    to the sum of the magnitudes of its terms, gradient relative to its largest
    component);
  * one time step, float64, teacher-forced (both sides step from the same
    float64 (q_{k-1}, q_k)): 1e-10 relative in q (max |dq| / max(1, max |q|))
    when both sides converge to a relative gradient tolerance of 1e-12: the
    oracle's own results at 1e-12 and 1e-13 differ by at most 3e-11 on these
    cases, while at 1e-11 they differ by up to 1.2e-9, so 1e-12 is the
    tolerance at which 1e-10 is implied rather than a matter of both sides
    taking the same path.  At the configured tolerance (1e-8) the bound is
    1e-7 (two runs of the same method from the same start);
  * one time step, mixed precision: 1e-5 relative pose error against the oracle
    (max link-origin distance over the model's reach, max rotation Frobenius
    distance).
"""
import sys

import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_1709_04145_amd import abd
from paper_1709_04145_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    abd.load()
    yield


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cu(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def rel_q(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b))))) if a.size else 0.0


def mixed_chains(n_models, seed, max_dofs=64):
    """Serial chains mixing hinge and ball joints, ragged, up to max_dofs DOFs."""
    models = []
    for i in range(n_models):
        rng = np.random.default_rng([seed, i])
        target = int(rng.integers(1, max_dofs + 1))
        dofs, axis, lengths = [], [], []
        while sum(dofs) < target:
            k = 3 if (rng.uniform() < 0.3 and sum(dofs) + 3 <= target) else 1
            dofs.append(k)
            if k == 3:
                axis.extend(np.eye(3))
            else:
                v = rng.standard_normal(3)
                axis.append(v / np.linalg.norm(v))
            lengths.append(rng.uniform(0.2, 1.0))
        n = len(dofs)
        offset = np.zeros((n, 3))
        for l in range(1, n):
            offset[l] = [lengths[l - 1], 0.0, 0.0]
        mm = np.stack([W.box_mass_moment(lengths[l], 0.1, rng.uniform(500, 2000)) for l in range(n)])
        models.append(dict(parent=np.arange(-1, n - 1), dofs=np.array(dofs, np.int32), axis=np.array(axis),
                           offset=offset, mm=mm))
    return W._assemble(models)


def pose_error(orc, desc, q, qref):
    A = orc.poses(q)
    Ar = orc.poses(qref)
    lo = desc.link_offset
    err_x, err_R = 0.0, 0.0
    for i in range(desc.n_models):
        sl = slice(lo[i], lo[i + 1])
        reach = np.sum(np.linalg.norm(desc.offset[sl], axis=1)) + 2.0 * np.max(desc.mass_moment[sl, 3] / desc.mass_moment[sl, 9])
        err_x = max(err_x, float(np.max(np.linalg.norm(A[sl, :, 3] - Ar[sl, :, 3], axis=1)) / reach))
        err_R = max(err_R, float(np.max(np.linalg.norm(A[sl, :, :3] - Ar[sl, :, :3], axis=(1, 2)))))
    return err_x, err_R


# ------------------------------------------------------------ evaluation
@pytest.mark.parametrize("seed", [1, 2])
def test_objective_and_gradient_fp64(seed):
    d = mixed_chains(40, seed)
    say(f"objective_grad fp64 seed={seed} models={d.n_models} dofs={d.n_dofs}")
    rng = np.random.default_rng(100 + seed)
    q, qp, qc = (rng.uniform(-2, 2, d.n_dofs) for _ in range(3))
    tau = rng.uniform(-1, 1, d.n_dofs)
    dt = 0.05
    E, g, S = Oracle(d).objective_grad(q, qp, qc, dt, tau)
    m = abd.Model(d)
    Eg, gg = m.objective_grad(cu(q), cu(np.concatenate([qp, qc])), dt, tau=cu(tau))
    Eg, gg = Eg.cpu().numpy(), gg.cpu().numpy()
    assert np.all(np.abs(Eg - E) <= 1e-12 * S)
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        scale = np.max(np.abs(g[sl]))
        assert np.max(np.abs(gg[sl] - g[sl])) <= 1e-12 * scale, i


def test_objective_mixed_is_close():
    d = mixed_chains(20, 7)
    rng = np.random.default_rng(5)
    q, qp, qc = (rng.uniform(-1, 1, d.n_dofs) for _ in range(3))
    say("objective_grad mixed")
    E, g, S = Oracle(d).objective_grad(q, qp, qc, 0.03)
    m = abd.Model(d)
    Eg, gg = m.objective_grad(cu(q), cu(np.concatenate([qp, qc])), 0.03, precision=abd.MIXED)
    assert np.all(np.abs(Eg.cpu().numpy() - E) <= 1e-5 * S)


def test_poses_fp64():
    d = mixed_chains(30, 3)
    q = np.random.default_rng(6).uniform(-3, 3, d.n_dofs)
    say("poses")
    A = Oracle(d).poses(q)
    Ag = abd.Model(d).poses(cu(q)).cpu().numpy()
    assert np.max(np.abs(Ag - A)) <= 1e-13 * max(1.0, np.max(np.abs(A)))


# ------------------------------------------------------------------ steps
def _step_gpu(d, qp, qc, opts, tau=None):
    m = abd.Model(d)
    out = torch.zeros(d.n_dofs, dtype=torch.float64, device="cuda")
    st = m.new_stats()
    m.step(cu(np.concatenate([qp, qc])), out, opts, tau=None if tau is None else cu(tau), stats=st)
    torch.cuda.synchronize()
    return out.cpu().numpy(), m.read_stats(st, d.n_models)


def _replicated(desc, k):
    return desc.subset(np.tile(np.arange(desc.n_models), k))


def test_config1_teacher_forced_fp64():
    wl = W.config(1)
    orc = Oracle(wl.model)
    dt = wl.step.dt
    qs, _ = orc.rollout(wl.q0, wl.step.steps, dt)
    K = wl.step.steps
    rep = _replicated(wl.model, K)
    qp = np.concatenate([qs[max(k - 1, 0)] for k in range(K)])
    qc = np.concatenate([qs[k] for k in range(K)])
    say(f"config1 teacher-forced fp64, {K} steps in one batch")
    ref, rst = Oracle(rep).step(qp, qc, dt)
    out, st = _step_gpu(rep, qp, qc, abd.StepOptions(dt=dt))
    assert rel_q(out, ref) <= 1e-10
    assert np.all(st["flag"] == rst["flag"])
    assert np.all(np.abs(st["iterations"] - rst["iterations"]) <= 1)


@pytest.mark.parametrize("precision", [abd.FP64, abd.MIXED])
def test_config2_subset_teacher_forced(precision):
    wl = W.config(2, n_models=128)
    orc = Oracle(wl.model)
    dt = wl.step.dt
    qs, _ = orc.rollout(wl.q0, 3, dt)
    say(f"config2 subset teacher-forced precision={precision}")
    for k in (0, 3):
        qp, qc = qs[max(k - 1, 0)], qs[k]
        if precision == abd.FP64:
            for tol, bound in ((1e-12, 1e-10), (1e-8, 1e-7)):
                ref, rst = orc.step(qp, qc, dt, tol=tol)
                out, st = _step_gpu(wl.model, qp, qc, abd.StepOptions(dt=dt, tol=tol))
                assert rel_q(out, ref) <= bound, (k, tol, rel_q(out, ref))
                assert np.all(st["flag"] == 1), np.unique(st["flag"], return_counts=True)
        else:
            ref, rst = orc.step(qp, qc, dt)
            out, st = _step_gpu(wl.model, qp, qc, abd.StepOptions(dt=dt, precision=precision))
            ex, eR = pose_error(orc, wl.model, out, ref)
            assert ex <= 1e-5 and eR <= 1e-5, (k, ex, eR)
            assert np.all(st["flag"] == 1), np.unique(st["flag"], return_counts=True)
            _check_float32_phase(st, abd.REFRESH)


def _check_float32_phase(st, refresh):
    """Mixed steps: the float32 phase ends at the step's first re-formation of the
    preconditioner (so at most `refresh` float32 iterations), the warm start is
    evaluated in float32, and float32 evaluations are a subset of all of them."""
    assert np.all(st["f32_iterations"] <= refresh), int(st["f32_iterations"].max())
    assert np.all(st["f32_evaluations"] >= st["f32_iterations"] + 1), "float32 evaluations undercounted"
    assert np.all(st["f32_evaluations"] <= st["evaluations"])


def test_frozen_preconditioner_matches_oracle():
    """refresh = 0 (H_q of the warm start for the whole step) on both sides:
    float64 to 1e-10 at a 1e-12 tolerance, like the default path."""
    wl = W.config(2, n_models=128)
    orc = Oracle(wl.model)
    dt = wl.step.dt
    qs, _ = orc.rollout(wl.q0, 3, dt)
    say("config2 subset, frozen preconditioner")
    ref, rst = orc.step(qs[-2], qs[-1], dt, tol=1e-12, refresh=0, max_iter=2000)
    out, st = _step_gpu(wl.model, qs[-2], qs[-1], abd.StepOptions(dt=dt, tol=1e-12, refresh=0, max_iter=2000))
    assert np.all(st["flag"] == 1) and np.all(rst["flag"] == 1)
    assert rel_q(out, ref) <= 1e-10, rel_q(out, ref)


def test_results_do_not_depend_on_model_order():
    """Each model is solved on its own (workgroups take models in descending
    frame count): a permuted batch gives every model the same result, bit for
    bit, in both precisions."""
    wl = W.config(2, n_models=48)
    d = wl.model
    perm = np.random.default_rng(91).permutation(d.n_models)
    dp = d.subset(perm)
    idx = d.dof_subset_index(perm)
    qs, _ = Oracle(d).rollout(wl.q0, 2, wl.step.dt)
    say("model order independence")
    for precision in (abd.FP64, abd.MIXED):
        opts = abd.StepOptions(dt=wl.step.dt, precision=precision)
        a, sa = _step_gpu(d, qs[-2], qs[-1], opts)
        b, sb = _step_gpu(dp, qs[-2][idx], qs[-1][idx], opts)
        assert np.array_equal(a[idx], b)
        assert np.array_equal(sa["iterations"][perm], sb["iterations"])


def test_ragged_mixed_joint_chains_fp64():
    d = mixed_chains(64, 11, max_dofs=40)
    rng = np.random.default_rng(12)
    qc = rng.uniform(-1, 1, d.n_dofs)
    tau = rng.uniform(-1, 1, d.n_dofs)
    say(f"ragged hinge/ball chains dofs={d.n_dofs}")
    ref, rst = Oracle(d).step(qc, qc, 0.01, tau=tau, tol=1e-12)
    out, st = _step_gpu(d, qc, qc, abd.StepOptions(dt=0.01, tol=1e-12), tau=tau)
    both = (st["flag"] == 1) & (rst["flag"] == 1)
    assert np.mean(both) > 0.9, (np.unique(st["flag"], return_counts=True), np.unique(rst["flag"], return_counts=True))
    do = d.dof_offset
    for i in np.nonzero(both)[0]:
        sl = slice(do[i], do[i + 1])
        assert rel_q(out[sl], ref[sl]) <= 1e-10, i


def test_ragged_mixed_joint_chains_mixed():
    """Mixed precision on ragged hinge/ball chains of 1..64 DOFs (the one-wave
    limit, where the float32 inverse fills its whole LDS region): every step
    converges, and its poses are within 1e-5 relative pose error of the oracle's
    float64 solution."""
    d = mixed_chains(64, 13, max_dofs=64)
    n = np.diff(d.dof_offset)
    assert n.min() == 1 and n.max() == 64
    rng = np.random.default_rng(14)
    qc = rng.uniform(-1, 1, d.n_dofs)
    say(f"ragged hinge/ball chains, mixed, dofs={d.n_dofs}")
    orc = Oracle(d)
    ref, rst = orc.step(qc, qc, 0.01, tol=1e-12, max_iter=3000)
    out, st = _step_gpu(d, qc, qc, abd.StepOptions(dt=0.01, precision=abd.MIXED))
    assert np.all(st["flag"] == abd.FLAG_CONVERGED), np.unique(st["flag"], return_counts=True)
    ok = rst["flag"] == 1
    assert np.mean(ok) > 0.9
    keep = np.nonzero(ok)[0]
    sub = d.subset(keep)
    idx = d.dof_subset_index(keep)
    ex, eR = pose_error(Oracle(sub), sub, out[idx], ref[idx])
    assert ex <= 1e-5 and eR <= 1e-5, (ex, eR)


def test_identity_preconditioner_fp64():
    """Without the inertia preconditioner (H0 = gamma I), both sides solved to a
    1e-12 relative gradient (about 1000 iterations on the 10-link chain): the
    same 1e-10 bound as the preconditioned path."""
    wl = W.config(1)
    q = wl.q0
    say("identity preconditioner")
    ref, rst = Oracle(wl.model).step(q, q, wl.step.dt, precond=0, tol=1e-12, max_iter=20000)
    out, st = _step_gpu(wl.model, q, q, abd.StepOptions(dt=wl.step.dt, precond=abd.PRECOND_IDENTITY, tol=1e-12,
                                                         max_iter=20000))
    assert st["flag"][0] == 1 and rst["flag"][0] == 1, (st["flag"], rst["flag"])
    assert rel_q(out, ref) <= 1e-10, rel_q(out, ref)


def _ill_conditioned_chains(n_models, seed):
    """Hinge chains with link lengths log-uniform in [0.02, 2] m and densities
    log-uniform in [1e-2, 1e5] kg/m^3: joint-space inertias of condition 1e9..1e17."""
    models = []
    for i in range(n_models):
        rng = np.random.default_rng([seed, i])
        n = int(rng.integers(20, 64))
        axis = rng.standard_normal((n, 3))
        axis /= np.linalg.norm(axis, axis=1, keepdims=True)
        L = np.exp(rng.uniform(np.log(0.02), np.log(2.0), n))
        offset = np.zeros((n, 3))
        offset[1:, 0] = L[:-1]
        mm = np.stack([W.box_mass_moment(L[l], 0.1 * min(1.0, L[l]), np.exp(rng.uniform(np.log(1e-2), np.log(1e5))))
                       for l in range(n)])
        models.append(dict(parent=np.arange(-1, n - 1), dofs=np.ones(n, np.int32), axis=axis, offset=offset, mm=mm))
    return W._assemble(models)


def test_mixed_ill_conditioned_chains_converge():
    """Mixed precision keeps a one-wave chain's explicit inverse in float32 only
    while the recursion's pivots span at most 1e5; these chains (pivots spanning
    up to 1e14) must keep the float64 inverse where float32 rounding would make
    it a poor or indefinite preconditioner.  Every step must converge, to a point
    where the oracle's float64 gradient meets the tolerance too."""
    d = _ill_conditioned_chains(32, 77)
    rng = np.random.default_rng(78)
    q = rng.uniform(-1, 1, d.n_dofs)
    dt, tol = 0.03, 1e-8
    say("mixed ill-conditioned chains")
    orc = Oracle(d)
    out, st = _step_gpu(d, q, q, abd.StepOptions(dt=dt, tol=tol, max_iter=5000, precision=abd.MIXED))
    say(f"  flags {np.unique(st['flag'], return_counts=True)}, iterations max {st['iterations'].max()}")
    assert np.all(st["flag"] == abd.FLAG_CONVERGED), st["flag"]
    _, g, _ = orc.objective_grad(out, q, q, dt)
    _, g0, _ = orc.objective_grad(q, q, q, dt)  # warm start 2 q_k - q_{k-1} = q
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        assert np.linalg.norm(g[sl]) <= 1.1 * tol * np.linalg.norm(g0[sl]), (i, np.linalg.norm(g[sl]) / np.linalg.norm(g0[sl]))


def test_full_config2_sampled_fp64_and_mixed():
    wl = W.config(2)
    dt = wl.step.dt
    say(f"config2 full size: {wl.model.n_models} models, {wl.model.n_dofs} dofs")
    sample = np.arange(0, wl.model.n_models, 64)
    sub = wl.model.subset(sample)
    idx = wl.model.dof_subset_index(sample)
    orc = Oracle(sub)
    for precision, tol in ((abd.FP64, 1e-12), (abd.MIXED, 1e-8)):
        ref, rst = orc.step(wl.q0[idx], wl.q0[idx], dt, tol=tol)
        out, st = _step_gpu(wl.model, wl.q0, wl.q0, abd.StepOptions(dt=dt, precision=precision, tol=tol))
        assert np.all(st["flag"] == 1), np.unique(st["flag"], return_counts=True)
        if precision == abd.FP64:
            assert rel_q(out[idx], ref) <= 1e-10
        else:
            ex, eR = pose_error(orc, sub, out[idx], ref)
            assert ex <= 1e-5 and eR <= 1e-5


@pytest.mark.parametrize("precision", [abd.FP64, abd.MIXED])
def test_rollout_equals_step_loop_bitwise(precision):
    """One launch for K steps computes exactly what K single-step launches compute."""
    wl = W.config(2, n_models=64)
    K = 6
    m = abd.Model(wl.model)
    opts = abd.StepOptions(dt=wl.step.dt, precision=precision)
    q0 = cu(wl.q0)
    say(f"rollout vs step loop precision={precision}")
    traj_loop, st_loop = m.step_loop(q0, K, opts)
    st = m.new_rollout_stats(K)
    traj, _ = m.rollout(torch.cat([q0, q0]), K, opts, stats=st)
    torch.cuda.synchronize()
    assert torch.equal(traj, traj_loop[1:])
    st = m.read_rollout_stats(st, K)
    for k in range(K):
        assert np.array_equal(st[k]["iterations"], st_loop[k]["iterations"])
        assert np.array_equal(st[k]["flag"], st_loop[k]["flag"])


def test_rollout_with_torques_matches_oracle():
    """Rollout with per-step joint torques (config 5 chains: 1 m, 10 kg links).
    Every GPU step k is checked against the exact minimizer q* of the step from
    the GPU's own (q_{k-1}, q_k) and torque k (oracle L-BFGS, then Newton), which
    also checks that step k reads torque row k.  These chains are so badly
    conditioned that a relative gradient tolerance of 1e-8 leaves ~1e-6 in q
    (the oracle's own result is 9e-7 from q* on one of these steps), so the
    check is the one the tolerance implies: the gradient at the GPU's q
    (computed by the oracle) is within the tolerance, and the GPU's q is within
    |H(q*)^-1| |g(q)| of q* (first-order bound, 50% margin)."""
    steps = 5
    wl = W.config(5, n_models=32, steps=steps)
    dt = wl.step.dt
    d = wl.model
    say("rollout with torques")
    m = abd.Model(d)
    q0 = cu(wl.q0)
    tol = wl.step.tol
    traj, _ = m.rollout(torch.cat([q0, q0]), steps, abd.StepOptions(dt=dt, tol=tol), torque=cu(wl.torque))
    qg = np.concatenate([wl.q0[None], wl.q0[None], traj.cpu().numpy()])  # q_{-1}, q_0, q_1..
    orc = Oracle(d)
    do = d.dof_offset
    for k in range(steps):
        qp, qc, tau = qg[k], qg[k + 1], wl.torque[k]
        ref, _ = orc.step(qp, qc, dt, tau=tau, tol=1e-11, max_iter=2000)
        qs, _ = orc.newton_polish(ref, qp, qc, dt, tau=tau, iters=3)
        _, g_w, _ = orc.objective_grad(2 * qc - qp, qp, qc, dt, tau)  # gradient at the warm start
        _, g_q, _ = orc.objective_grad(qg[k + 2], qp, qc, dt, tau)     # gradient at the GPU's q
        H = orc.hessian(qs, qp, qc, dt)
        for i in range(d.n_models):
            sl = slice(do[i], do[i + 1])
            gq, gw = np.linalg.norm(g_q[sl]), np.linalg.norm(g_w[sl])
            assert gq <= 2.0 * tol * gw + 1e-13, (k, i, gq, gw)
            hinv = 1.0 / np.min(np.linalg.eigvalsh(H[i]))
            err = np.linalg.norm(qg[k + 2][sl] - qs[sl])
            assert err <= 1.5 * hinv * gq + 1e-12, (k, i, err, hinv * gq)
def test_mixed_rollout_with_torques_bounded_float32_phase():
    """Mixed-precision rollout on the torque workload's chains (1 m, 10 kg links,
    joint forces per step): each step's float32 phase stays within the first
    re-formation interval, and every step's result is within 1e-5 relative pose
    error of the oracle's minimizer of the same step (teacher-forced from the
    GPU's own float64 history, oracle solved to 1e-11 and Newton-polished)."""
    steps = 5
    wl = W.config(5, n_models=32, steps=steps)
    dt = wl.step.dt
    d = wl.model
    say("mixed rollout with torques")
    m = abd.Model(d)
    q0 = cu(wl.q0)
    st = m.new_rollout_stats(steps)
    traj, _ = m.rollout(torch.cat([q0, q0]), steps, abd.StepOptions(dt=dt, precision=abd.MIXED),
                        torque=cu(wl.torque), stats=st)
    st = m.read_rollout_stats(st, steps)
    qg = np.concatenate([wl.q0[None], wl.q0[None], traj.cpu().numpy()])
    orc = Oracle(d)
    for k in range(steps):
        _check_float32_phase(st[k], abd.REFRESH)
        assert np.all(st[k]["flag"] == abd.FLAG_CONVERGED), (k, np.unique(st[k]["flag"]))
        qp, qc, tau = qg[k], qg[k + 1], wl.torque[k]
        ref, _ = orc.step(qp, qc, dt, tau=tau, tol=1e-11, max_iter=2000)
        qs, _ = orc.newton_polish(ref, qp, qc, dt, tau=tau, iters=3)
        ex, eR = pose_error(orc, d, qg[k + 2], qs)
        assert ex <= 1e-5 and eR <= 1e-5, (k, ex, eR)


# ------------------------------------------------------------- edge cases
def test_empty_batch():
    d = W.random_chain_models(0, 1)
    m = abd.Model(d)
    assert m.n_models == 0
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = torch.zeros(2, dtype=torch.float64, device="cuda")
    # zero DOFs: the call is a no-op
    abd.load().abd_step(m._h, abd.StepOptions(dt=0.1).c(), abd._ptr(hist), None, abd._ptr(out), None,
                        abd._stream())


def test_1024_dofs_is_the_limit():
    d = W.random_chain_models(1, 3, lo=1024, hi=1024)
    abd.Model(d)
    d1025 = W.random_chain_models(1, 3, lo=1025, hi=1025)
    with pytest.raises(abd.AbdError) as e:
        abd.Model(d1025)
    assert e.value.code == abd.ABD_ENOTSUP


def test_zero_gravity_rest_is_exact_fixed_point():
    d = mixed_chains(16, 21)
    d.gravity = np.zeros(3)
    q = np.random.default_rng(3).uniform(-1, 1, d.n_dofs)
    out, st = _step_gpu(d, q, q, abd.StepOptions(dt=0.1))
    assert np.array_equal(out, q)
    assert np.all(st["iterations"] == 0) and np.all(st["flag"] == 1)


def test_nonfinite_model_is_isolated():
    d = W.random_chain_models(8, 5, lo=5, hi=40)
    q = np.random.default_rng(4).uniform(-1, 1, d.n_dofs)
    qb = q.copy()
    qb[d.dof_offset[3]] = np.nan
    out, st = _step_gpu(d, q, qb, abd.StepOptions(dt=0.05))
    assert st["flag"][3] == abd.FLAG_NONFINITE
    others = [i for i in range(d.n_models) if i != 3]
    assert np.all(st["flag"][others] == abd.FLAG_CONVERGED)


def test_max_iter_zero_and_one():
    wl = W.config(2, n_models=16)
    q = wl.q0
    out, st = _step_gpu(wl.model, q, q, abd.StepOptions(dt=wl.step.dt, max_iter=0))
    assert np.all(st["flag"] == abd.FLAG_MAX_ITER) and np.all(st["iterations"] == 0)
    assert np.array_equal(out, q)  # warm start with zero velocity is q itself
    ref, rst = Oracle(wl.model).step(q, q, wl.step.dt, max_iter=1)
    out, st = _step_gpu(wl.model, q, q, abd.StepOptions(dt=wl.step.dt, max_iter=1))
    assert np.all(st["flag"] == rst["flag"])
    assert rel_q(out, ref) <= 1e-10


@pytest.mark.parametrize("precision", [abd.FP64, abd.MIXED])
def test_unreachable_tolerance_stops_at_the_minimizer(precision):
    """tol = 0 can never be met: every step must end by the line search (flag 2,
    which includes an accepted point equal to the iterate) or at the cap, and
    hold the oracle's minimizer of a 1e-12 solve to 1e-10 relative."""
    wl = W.config(2, n_models=32)
    q = wl.q0
    say(f"unreachable tolerance precision={precision}")
    ref, rst = Oracle(wl.model).step(q, q, wl.step.dt, tol=1e-12, max_iter=2000)
    out, st = _step_gpu(wl.model, q, q, abd.StepOptions(dt=wl.step.dt, tol=0.0, max_iter=2000, precision=precision))
    assert np.all(rst["flag"] == 1)
    assert np.all(np.isin(st["flag"], [abd.FLAG_LS_FLOOR, abd.FLAG_MAX_ITER])), np.unique(st["flag"])
    do = wl.model.dof_offset
    for i in range(wl.model.n_models):
        sl = slice(do[i], do[i + 1])
        assert np.max(np.abs(out[sl] - ref[sl])) / max(1.0, np.max(np.abs(ref[sl]))) <= 1e-10, i


def test_invalid_options_rejected():
    d = mixed_chains(2, 1)
    m = abd.Model(d)
    hist = torch.zeros(2 * d.n_dofs, dtype=torch.float64, device="cuda")
    out = torch.zeros(d.n_dofs, dtype=torch.float64, device="cuda")
    for bad in (dict(dt=0.0), dict(dt=0.1, lbfgs_m=11), dict(dt=0.1, max_ls=0), dict(dt=0.1, precision=7),
                dict(dt=0.1, precond=1), dict(dt=0.1, refresh=-1)):
        with pytest.raises(abd.AbdError) as e:
            m.step(hist, out, abd.StepOptions(**bad))
        assert e.value.code == abd.ABD_EINVAL
    out5 = torch.zeros(4 * d.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(abd.AbdError) as e:
        m.step(hist, out5, abd.StepOptions(dt=0.1, order_K=5))
    assert e.value.code == abd.ABD_ENOTSUP
    import ctypes
    o1 = abd.StepOptions(dt=0.1, order_K=1).c()
    rc = abd.load().abd_step(m._h, ctypes.byref(o1), ctypes.c_void_p(hist.data_ptr()), None,
                             ctypes.c_void_p(out.data_ptr()), None, None)
    assert rc == abd.ABD_EINVAL


def test_rollout_captured_in_hip_graph_replays_exactly():
    """abd_rollout captured in a HIP graph (through torch's graph capture) and
    replayed several times, with other eager work on the same model in between,
    matches an eager rollout of the same inputs bit for bit on every replay."""
    wl = W.config(2, n_models=64)
    d = wl.model
    m = abd.Model(d)
    opts = abd.StepOptions(dt=wl.step.dt, precision=abd.MIXED)
    steps = 3
    rng = np.random.default_rng(81)
    init = torch.zeros(2 * d.n_dofs, dtype=torch.float64, device="cuda")
    traj = torch.empty((steps, d.n_dofs), dtype=torch.float64, device="cuda")
    stats = m.new_rollout_stats(steps)
    init.copy_(cu(np.concatenate([wl.q0, wl.q0])))
    m.rollout(init, steps, opts, q_traj=traj, stats=stats)  # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.rollout(init, steps, opts, q_traj=traj, stats=stats)
    torch.cuda.synchronize()
    for rep in range(3):
        q0 = wl.q0 + 0.1 * rng.uniform(-1, 1, d.n_dofs)
        init.copy_(cu(np.concatenate([q0, q0])))
        g.replay()
        torch.cuda.synchronize()
        got = traj.clone()
        got_st = m.read_rollout_stats(stats, steps)
        # eager work on the same model between replays
        ref, ref_st = m.rollout(cu(np.concatenate([q0, q0])), steps, opts, stats=m.new_rollout_stats(steps))
        torch.cuda.synchronize()
        assert torch.equal(got, ref), rep
        ref_st = m.read_rollout_stats(ref_st, steps)
        assert np.array_equal(got_st["iterations"], ref_st["iterations"]), rep
