"""Second-order paths of the HIP library against the FP64 CPU oracle.

  * Hessian-vector product (abd_hvp) against the oracle's dense Hessian
    (second derivatives of the poses written out, pinned by central differences
    of the Alg. 1 gradient): 1e-10 relative to the largest component;
  * rollout VJP (abd_rollout_vjp, implicit differentiation with CG) against the
    oracle's dense implicit differentiation of the SAME trajectory (pinned by
    central differences of whole rollouts): CG is run to a 1e-13 relative
    residual, and the bound is 1e-8 relative to the largest component (the
    residual is amplified by at most the condition number of the step Hessian);
  * the autograd functions built on them.
"""
import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_1709_04145_amd import abd
from paper_1709_04145_amd import workloads as W
from test_gpu_parity import cu, mixed_chains, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    abd.load()
    yield


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b))))) if a.size else 0.0


@pytest.mark.parametrize("seed", [3, 4])
def test_hvp_matches_oracle_hessian(seed):
    d = mixed_chains(24, seed, max_dofs=64)
    say(f"hvp seed={seed} dofs={d.n_dofs}")
    rng = np.random.default_rng(50 + seed)
    q, qp, qc, v = (rng.uniform(-1.5, 1.5, d.n_dofs) for _ in range(4))
    dt = 0.04
    H = Oracle(d).hessian(q, qp, qc, dt)
    m = abd.Model(d)
    hv = m.hvp(cu(q), cu(np.concatenate([qp, qc])), cu(v), dt).cpu().numpy()
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        ref = H[i] @ v[sl]
        assert _rel(hv[sl], ref) <= 1e-10, (i, _rel(hv[sl], ref))


def _config5_rollout(n_models, steps):
    wl = W.config(5, n_models=n_models, steps=steps)
    m = abd.Model(wl.model)
    q0 = cu(wl.q0)
    init = torch.cat([q0, q0]).contiguous()
    opts = abd.StepOptions(dt=wl.step.dt, tol=1e-11)
    traj, _ = m.rollout(init, steps, opts, torque=cu(wl.torque))
    torch.cuda.synchronize()
    return wl, m, init, traj, opts


def test_rollout_vjp_matches_oracle():
    steps = 5
    wl, m, init, traj, opts = _config5_rollout(16, steps)
    d = wl.model
    rng = np.random.default_rng(61)
    w = rng.normal(size=(steps, d.n_dofs))
    say(f"rollout vjp models={d.n_models} dofs={d.n_dofs} steps={steps}")
    st = m.new_rollout_stats(steps)
    g_init, g_tau = m.rollout_vjp(init, traj, cu(w), opts.dt, tol=1e-13, max_iter=500, stats=st)
    torch.cuda.synchronize()
    stats = m.read_rollout_stats(st, steps)
    assert np.all(stats["flag"] == abd.FLAG_CONVERGED), np.unique(stats["flag"], return_counts=True)
    qi = init.cpu().numpy()
    n = d.n_dofs
    ref_m1, ref_0, ref_tau = Oracle(d).rollout_vjp(qi[:n], qi[n:], traj.cpu().numpy(), opts.dt, w)
    gi = g_init.cpu().numpy()
    assert _rel(gi[:n], ref_m1) <= 1e-8, _rel(gi[:n], ref_m1)
    assert _rel(gi[n:], ref_0) <= 1e-8, _rel(gi[n:], ref_0)
    assert _rel(g_tau.cpu().numpy(), ref_tau) <= 1e-8, _rel(g_tau.cpu().numpy(), ref_tau)
    say(f"cg iterations per step: mean {stats['iterations'].mean():.1f} max {stats['iterations'].max()}")


def test_rollout_vjp_identity_preconditioner_agrees():
    steps = 3
    wl, m, init, traj, opts = _config5_rollout(8, steps)
    rng = np.random.default_rng(62)
    w = cu(rng.normal(size=(steps, wl.model.n_dofs)))
    a, ta = m.rollout_vjp(init, traj, w, opts.dt, tol=1e-13, max_iter=3000)
    b, tb = m.rollout_vjp(init, traj, w, opts.dt, tol=1e-13, max_iter=3000, precond=abd.PRECOND_IDENTITY)
    torch.cuda.synchronize()
    assert _rel(b.cpu().numpy(), a.cpu().numpy()) <= 1e-6
    assert _rel(tb.cpu().numpy(), ta.cpu().numpy()) <= 1e-6


def test_autograd_rollout_end_effector_loss():
    """Config 5's loss |x_ee(q_T) - target|^2 through the differentiable rollout:
    the gradients to q_0 (q_{-1} tied to q_0) and to the torques equal the
    oracle's implicit differentiation of the same trajectory."""
    steps = 4
    wl = W.config(5, n_models=6, steps=steps)
    d = wl.model
    m = abd.Model(d)
    opts = abd.StepOptions(dt=wl.step.dt, tol=1e-11)
    q0 = cu(wl.q0).requires_grad_(True)
    tau = cu(wl.torque).requires_grad_(True)
    traj = abd.rollout(m, torch.cat([q0, q0]), steps, opts, torque=tau, vjp_tol=1e-13, vjp_max_iter=500)
    poses = m.poses(traj[-1].detach().contiguous()).cpu().numpy()
    # end effector of each chain: (L, 0, 0) of its last link; dL/dq_T from the
    # world-frame Jacobian of that point, dx/dq_n = w_n x (x - p_n) (one DOF per link)
    lo, do = d.link_offset, d.dof_offset
    dL_dqT = np.zeros(d.n_dofs)
    for i in range(d.n_models):
        last = lo[i + 1] - 1
        L_last = 2.0 * d.mass_moment[last, 3] / d.mass_moment[last, 9]
        x = poses[last, :, 3] + poses[last, :, :3] @ np.array([L_last, 0.0, 0.0])
        r = x - wl.target[i]
        for l in range(lo[i], lo[i + 1]):
            n_ = do[i] + (l - lo[i])
            wv = poses[l, :, :3] @ d.axis[n_]
            dL_dqT[n_] = 2.0 * r @ np.cross(wv, x - poses[l, :, 3])
    g_traj = torch.zeros_like(traj)
    g_traj[-1] = cu(dL_dqT)
    traj.backward(g_traj)
    torch.cuda.synchronize()
    w = np.zeros((steps, d.n_dofs))
    w[-1] = dL_dqT
    ref_m1, ref_0, ref_tau = Oracle(d).rollout_vjp(wl.q0, wl.q0, traj.detach().cpu().numpy(), opts.dt, w)
    assert _rel(q0.grad.cpu().numpy(), ref_m1 + ref_0) <= 1e-8
    assert _rel(tau.grad.cpu().numpy(), ref_tau) <= 1e-8


def test_objective_autograd():
    d = mixed_chains(8, 7, max_dofs=30)
    rng = np.random.default_rng(71)
    q, qp, qc, tau = (rng.uniform(-1, 1, d.n_dofs) for _ in range(4))
    dt = 0.03
    m = abd.Model(d)
    qt = cu(q).requires_grad_(True)
    tt = cu(tau).requires_grad_(True)
    E = abd.objective(m, qt, cu(np.concatenate([qp, qc])), dt, tau=tt)
    wts = torch.arange(1, d.n_models + 1, dtype=torch.float64, device="cuda")
    (E * wts).sum().backward()
    _, g, _ = Oracle(d).objective_grad(q, qp, qc, dt, tau)
    per_dof = np.repeat(np.arange(1, d.n_models + 1), np.diff(d.dof_offset)).astype(np.float64)
    assert _rel(qt.grad.cpu().numpy(), per_dof * g) <= 1e-12
    assert _rel(tt.grad.cpu().numpy(), -dt * dt * per_dof * q) <= 1e-15
