"""Branched models (trees of hinge and ball joints) on the GPU against the FP64
CPU oracle.  Frames are reordered internally to depth-first preorder; the
forward pass runs by pointer jumping along the ancestor paths and the adjoint
sums over the frames below by preorder-range differences.

  * objective and gradient, float64: 1e-12 relative; poses 1e-12 absolute;
  * one step, teacher-forced: 1e-10 relative in q with both sides at a relative
    gradient tolerance of 1e-12 (small trees); mixed precision 1e-5 relative pose
    error;
  * the 2048-tree workload's trees (30..60 ball-jointed links, 90..180 DOFs):
    one step at tolerance 1e-6, checked by what the tolerance implies (gradient
    at the GPU's q within the tolerance, distance to the exact minimizer within
    |H(q*)^-1| |g(q)|);
  * a rollout in one launch equals the loop of single steps bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_1709_04145_amd import abd
from paper_1709_04145_amd import workloads as W
from test_gpu_parity import cu, pose_error, say, _step_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    abd.load()
    yield


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b))))) if a.size else 0.0


@pytest.mark.parametrize("which", ["small", "workload"])
def test_tree_objective_gradient_and_poses(which):
    d = W.random_tree_models(24, 51, max_links=12, ball_prob=0.4) if which == "small" else W.config_models(3, 6)
    say(f"tree objective {which} dofs={d.n_dofs}")
    rng = np.random.default_rng(52)
    q, qp, qc = (rng.uniform(-1, 1, d.n_dofs) for _ in range(3))
    tau = rng.uniform(-1, 1, d.n_dofs)
    dt = 0.05
    orc = Oracle(d)
    E, g, S = orc.objective_grad(q, qp, qc, dt, tau)
    m = abd.Model(d)
    Eg, gg = m.objective_grad(cu(q), cu(np.concatenate([qp, qc])), dt, tau=cu(tau))
    Eg, gg = Eg.cpu().numpy(), gg.cpu().numpy()
    assert np.all(np.abs(Eg - E) <= 1e-12 * S), (Eg - E, S)
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        assert _rel(gg[sl], g[sl]) <= 1e-12, (i, _rel(gg[sl], g[sl]))
    np.testing.assert_allclose(m.poses(cu(q)).cpu().numpy(), orc.poses(q), rtol=0, atol=1e-12)


@pytest.mark.parametrize("precision", [abd.FP64, abd.MIXED])
def test_small_tree_step_teacher_forced(precision):
    d = W.random_tree_models(32, 53, max_links=8, ball_prob=0.4)
    rng = np.random.default_rng(54)
    qc = rng.uniform(-0.6, 0.6, d.n_dofs)
    qp = qc + 0.01 * rng.uniform(-1, 1, d.n_dofs)
    dt = 0.02
    say(f"small tree step precision={precision}")
    orc = Oracle(d)
    if precision == abd.FP64:
        ref, rst = orc.step(qp, qc, dt, tol=1e-12, max_iter=2000)
        out, st = _step_gpu(d, qp, qc, abd.StepOptions(dt=dt, tol=1e-12, max_iter=2000))
        both = (st["flag"] == 1) & (rst["flag"] == 1)
        assert np.mean(both) > 0.9, (st["flag"], rst["flag"])
        do = d.dof_offset
        for i in np.nonzero(both)[0]:
            sl = slice(do[i], do[i + 1])
            err = float(np.max(np.abs(out[sl] - ref[sl]))) / max(1.0, float(np.max(np.abs(ref[sl]))))
            assert err <= 1e-10, (i, err)
    else:
        ref, rst = orc.step(qp, qc, dt)
        out, st = _step_gpu(d, qp, qc, abd.StepOptions(dt=dt, precision=precision))
        assert np.all(st["flag"] == 1), st["flag"]
        ex, eR = pose_error(orc, d, out, ref)
        assert ex <= 1e-5 and eR <= 1e-5, (ex, eR)


def test_workload_trees_step_meets_its_tolerance():
    wl = W.config(3, n_models=4)
    d, q0 = wl.model, wl.q0
    dt, tol = 0.01, 1e-6
    say("workload trees step")
    m = abd.Model(d)
    out = torch.zeros(d.n_dofs, dtype=torch.float64, device="cuda")
    st = m.new_stats()
    m.step(cu(np.concatenate([q0, q0])), out, abd.StepOptions(dt=dt, tol=tol, max_iter=3000), stats=st)
    torch.cuda.synchronize()
    st = m.read_stats(st, d.n_models)
    assert np.all(st["flag"] == abd.FLAG_CONVERGED), st
    qg = out.cpu().numpy()
    orc = Oracle(d)
    ref, _ = orc.step(q0, q0, dt, tol=1e-9, max_iter=5000)
    qs, _ = orc.newton_polish(ref, q0, q0, dt, iters=3)
    _, g_w, _ = orc.objective_grad(q0, q0, q0, dt)
    _, g_q, _ = orc.objective_grad(qg, q0, q0, dt)
    H = orc.hessian(qs, q0, q0, dt)
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        gq, gw = np.linalg.norm(g_q[sl]), np.linalg.norm(g_w[sl])
        assert gq <= 2.0 * tol * gw, (i, gq, gw)
        hinv = 1.0 / np.min(np.linalg.eigvalsh(H[i]))
        assert np.linalg.norm(qg[sl] - qs[sl]) <= 1.5 * hinv * gq + 1e-12, i


@pytest.mark.parametrize("which", ["small", "workload"])
def test_tree_preconditioner_follows_the_oracles_iterations(which):
    """The GPU applies H_q^-1 of a branched model through the explicit L^-1 of its
    articulated-body factorization H_q = L D L^T (with a level-by-level
    recursion); the oracle runs the recursion's sweeps.  The two are the same
    matrix, so at a tight tolerance the float64 L-BFGS iterations are the same:
    the counts agree on at least 90 % of the models and within 2 on all (a wrong
    factorization changes the search directions and the counts)."""
    if which == "small":
        d = W.random_tree_models(32, 53, max_links=8, ball_prob=0.4)
        rng = np.random.default_rng(54)
        qc = rng.uniform(-0.6, 0.6, d.n_dofs)
        qp = qc + 0.01 * rng.uniform(-1, 1, d.n_dofs)
        dt, tol = 0.02, 1e-10
    else:
        wl = W.config(3, n_models=8)
        d, qp, qc = wl.model, wl.q0, wl.q0
        dt, tol = 0.01, 1e-8
    say(f"tree preconditioner iterations {which}")
    _, rst = Oracle(d).step(qp, qc, dt, tol=tol, max_iter=3000)
    _, st = _step_gpu(d, qp, qc, abd.StepOptions(dt=dt, tol=tol, max_iter=3000))
    gi, oi = st["iterations"], rst["iterations"]
    say(f"  gpu {gi.tolist()} oracle {oi.tolist()}")
    assert np.all(st["flag"] == abd.FLAG_CONVERGED) and np.all(rst["flag"] == 1)
    assert np.mean(gi == oi) >= 0.9 and np.all(np.abs(gi - oi) <= 2), (gi, oi)


def test_tree_rollout_equals_step_loop_bitwise():
    d = W.random_tree_models(16, 55, max_links=30, ball_prob=0.5)
    q0 = np.random.default_rng(56).uniform(-0.5, 0.5, d.n_dofs)
    m = abd.Model(d)
    opts = abd.StepOptions(dt=0.02, tol=1e-8, max_iter=800)
    K = 3
    traj_loop, st_loop = m.step_loop(cu(q0), K, opts)
    st = m.new_rollout_stats(K)
    traj, _ = m.rollout(torch.cat([cu(q0), cu(q0)]), K, opts, stats=st)
    torch.cuda.synchronize()
    assert torch.equal(traj, traj_loop[1:])


def test_tree_second_order_calls_rejected():
    d = W._assemble([W.tree_model(np.array([-1, 0, 0, 1]), 0.5, 0.1, 1000.0)])  # branched
    m = abd.Model(d)
    q = cu(np.zeros(d.n_dofs))
    with pytest.raises(abd.AbdError) as e:
        m.hvp(q, torch.cat([q, q]), q, 0.01)
    assert e.value.code == abd.ABD_ENOTSUP
