"""The 1000-link rope workload (ropes of 5 cm links, 5 g each, dt = 0.1, L-BFGS
history 10): teacher-forced steps against the FP64 oracle's, both precisions.

The reference (tests/golden/rope_steps.npz, written by
tests/golden/make_rope_reference.py from the oracle only) holds the oracle's first
three steps of four ropes, solved to a relative gradient tolerance of 1e-5 within
3000 iterations (the float64 floor of the gradient of these ropes lies near
1e-6..1e-7; from the fourth step on the oracle itself reaches the cap).  The step
objective is not convex at these step sizes: the oracle's Hessian at its own
results has negative eigenvalues (stored as lambda_min), so a result is not an
isolated minimizer.  The oracle restarted from a start perturbed by 1e-13 ends
up to 6 rad away in some joints after 0.5x..2x the iterations, at an objective
within 7.3e-7 of the step's decrease from the warm start of its unperturbed
result.  What is compared is therefore what the tolerance fixes: every step
converges on the GPU (iteration cap 6000: the count is as sensitive to rounding
as the path), the oracle's gradient at the GPU's configuration meets the
tolerance, and the objective there equals the oracle's to 1e-5 of the step's
decrease.
"""
import os

import numpy as np
import pytest
import torch

from oracle.oracle import Oracle
from paper_1709_04145_amd import abd
from paper_1709_04145_amd import workloads as W
from test_gpu_parity import cu, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rope_steps.npz")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    abd.load()
    yield


@pytest.mark.parametrize("precision", [abd.FP64, abd.MIXED])
def test_rope_steps_teacher_forced(precision):
    ref = np.load(GOLDEN, allow_pickle=False)
    nm, tol, max_iter = int(ref["models"]), float(ref["tol"]), int(ref["max_iter"])
    qs = ref["q"]  # [q_{-1}, q_0, q_1, ...] of the oracle
    wl = W.config(4, n_models=nm)
    d, dt = wl.model, wl.step.dt
    assert np.array_equal(qs[1], wl.q0)
    orc = Oracle(d)
    m = abd.Model(d)
    opts = abd.StepOptions(dt=dt, lbfgs_m=wl.step.lbfgs_m, tol=tol, max_iter=2 * max_iter, precision=precision)
    do = d.dof_offset
    for k in range(qs.shape[0] - 2):
        qp, qc, qr = qs[k], qs[k + 1], qs[k + 2]
        say(f"rope step {k} precision {precision}")
        out = torch.zeros(d.n_dofs, dtype=torch.float64, device="cuda")
        st = m.new_stats()
        m.step(cu(np.concatenate([qp, qc])), out, opts, stats=st)
        torch.cuda.synchronize()
        st = m.read_stats(st, nm)
        q = out.cpu().numpy()
        assert np.all(ref["flag"][k] == 1)
        assert np.all(st["flag"] == abd.FLAG_CONVERGED), (k, st["flag"], st["iterations"])
        warm = 2 * qc - qp
        Ew, gw, _ = orc.objective_grad(warm, qp, qc, dt)
        Eg, gg, Sg = orc.objective_grad(q, qp, qc, dt)
        Er, _, _ = orc.objective_grad(qr, qp, qc, dt)
        for i in range(nm):
            sl = slice(do[i], do[i + 1])
            gn, g0 = np.linalg.norm(gg[sl]), np.linalg.norm(gw[sl])
            gap = abs(Eg[i] - Er[i]) / (Ew[i] - Er[i])
            say(f"  rope {i}: iterations gpu {st['iterations'][i]} oracle {ref['iterations'][k][i]}, "
                f"|g|/|g0| {gn / g0:.2e}, objective gap / decrease {gap:.2e}, "
                f"max |q - q_oracle| {np.max(np.abs(q[sl] - qr[sl])):.2e}")
            assert gn <= 2.0 * tol * g0 + 1e-12 * Sg[i], (k, i, gn / g0)
            assert gap <= 1e-5, (k, i, gap)
