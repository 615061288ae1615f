"""abd_rollout_noalloc (the entry point for callers that cannot allocate device
memory) against abd_rollout through the C ABI: the same kernels with the step
scratch in the library's fixed device array instead of the model's buffers, so
trajectories and per-step stats must agree bit for bit.  Two calls in a row,
the second on a smaller batch, for each case; a model whose step scratch
exceeds the array is rejected before anything is enqueued."""
import numpy as np
import pytest
import torch

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


def _both(d, q_init, steps, opts, torque=None):
    """(trajectory, stats bytes) of abd_rollout and of abd_rollout_noalloc."""
    m = abd.Model(d)
    qi = cu(q_init)
    tq = None if torque is None else cu(torque)
    U = opts.order_K - 1
    shape = (steps, d.n_dofs) if U == 1 else (steps, U, d.n_dofs)
    ref, st_ref = m.rollout(qi, steps, opts, torque=tq, stats=m.new_rollout_stats(steps))
    out = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    st = m.new_rollout_stats(steps)
    m.rollout_noalloc(qi, steps, opts, out, st, torque=tq)
    torch.cuda.synchronize()
    return (ref.cpu().numpy(), st_ref.cpu().numpy().view(np.uint8)[:abd.STATS_BYTES * steps * d.n_models],
            out.cpu().numpy(), st.cpu().numpy().view(np.uint8)[:abd.STATS_BYTES * steps * d.n_models])


def _check(d, q_init, steps, opts, torque=None):
    ref, sref, got, sgot = _both(d, q_init, steps, opts, torque)
    assert np.array_equal(ref, got), float(np.nanmax(np.abs(ref - got)))
    assert np.array_equal(sref, sgot)


@pytest.mark.parametrize("precision", [abd.FP64, abd.MIXED])
def test_noalloc_rollout_equals_rollout_then_smaller_batch(precision):
    wl = W.config(2, n_models=256)
    q0 = wl.q0
    say(f"noalloc chains 256 then 40, precision={precision}")
    opts = abd.StepOptions(dt=wl.step.dt, precision=precision)
    _check(wl.model, np.concatenate([q0, q0]), 4, opts)
    small = W.config(2, n_models=40)
    _check(small.model, np.concatenate([small.q0, small.q0]), 3, opts)


def test_noalloc_long_chains_and_torques_then_smaller():
    """Models of more than 64 DOFs (the L-BFGS ring and preconditioner scratch
    live in the array too), with joint forces."""
    d, q0 = hanging_chains([65, 300, 140], 11)
    rng = np.random.default_rng(5)
    steps = 3
    tau = rng.uniform(-1, 1, (steps, d.n_dofs))
    say("noalloc long chains 65/300/140 then 90")
    opts = abd.StepOptions(dt=0.01, tol=1e-6)
    _check(d, np.concatenate([q0, q0]), steps, opts, torque=tau)
    d2, q2 = hanging_chains([90], 12)
    _check(d2, np.concatenate([q2, q2]), 2, opts)


def test_noalloc_order3_and_trees_then_smaller():
    """Order K = 3 (known-point seeds in the array) on branched models, then a
    smaller chain batch."""
    d = W.random_tree_models(12, 77, max_links=8)
    rng = np.random.default_rng(3)
    q0 = rng.uniform(-0.5, 0.5, d.n_dofs)
    say("noalloc order 3 trees then chains")
    opts = abd.StepOptions(dt=0.005, order_K=3, tol=1e-10)
    _check(d, np.concatenate([q0, q0]), 2, opts)
    c = W.random_chain_models(5, 8, lo=3, hi=10)
    qc = rng.uniform(-0.5, 0.5, c.n_dofs)
    _check(c, np.concatenate([qc, qc]), 2, opts)


def test_noalloc_rejects_models_beyond_the_array():
    """256 ropes of 1000 links need about 98 MB of step scratch: rejected with
    ABD_ENOTSUP before any work is enqueued (the outputs keep their contents)."""
    wl = W.config(4)
    m = abd.Model(wl.model)
    say("noalloc rejects the 256-rope batch")
    out = torch.full((1, wl.model.n_dofs), 7.0, dtype=torch.float64, device="cuda")
    st = m.new_rollout_stats(1)
    with pytest.raises(abd.AbdError) as e:
        m.rollout_noalloc(cu(np.concatenate([wl.q0, wl.q0])), 1, abd.StepOptions(dt=wl.step.dt), out, st)
    assert e.value.code == abd.ABD_ENOTSUP
    assert "static buffer" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
