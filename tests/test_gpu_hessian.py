"""Explicit Hessian of the step objective (abd_hessian) against the FP64 oracle's
written-out second derivatives (orc_hessian, itself pinned by central
differences of the Alg. 1 gradient) and against the GPU's Hessian-vector
product: serial chains, branched models with ball joints (the 2048-tree
workload's trees among them) and chains of up to 600 DOFs (16 waves).
Tolerance: 1e-10 of the block's largest entry (the entries are sums of
products of poses; both sides round differently)."""
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


def _compare(d, q, qp, qc, dt, tol=1e-10):
    m = abd.Model(d)
    Hg = [h.cpu().numpy() for h in m.hessian(cu(q), cu(np.concatenate([qp, qc])), dt)]
    Ho = Oracle(d).hessian(q, qp, qc, dt)
    worst = 0.0
    for i, (a, b) in enumerate(zip(Hg, Ho)):
        if b.size == 0:
            continue
        err = float(np.max(np.abs(a - b)) / max(1e-300, float(np.max(np.abs(b)))))
        worst = max(worst, err)
        assert err <= tol, (i, err)
    say(f"  max rel error {worst:.2e} over {d.n_models} models")
    return m, Hg


@pytest.mark.parametrize("which", ["chains", "trees", "workload_trees"])
def test_hessian_matches_oracle(which):
    if which == "chains":
        d = W.config(2, n_models=32).model
    elif which == "trees":
        d = W.random_tree_models(12, 131, max_links=8, ball_prob=0.4)
    else:
        d = W.config_models(3, 3)
    say(f"hessian {which} dofs={d.n_dofs}")
    rng = np.random.default_rng(132)
    q, qp, qc = (rng.uniform(-1, 1, d.n_dofs) for _ in range(3))
    _compare(d, q, qp, qc, 0.03)


def test_hessian_long_chains_match_oracle():
    d, q0 = hanging_chains([65, 300, 600], 133)
    rng = np.random.default_rng(134)
    q = q0 + 0.05 * rng.standard_normal(d.n_dofs)
    say(f"hessian long chains dofs={d.n_dofs}")
    _compare(d, q, q0, q0, 0.01)


def test_hessian_times_vector_is_the_hvp():
    """H v from the explicit blocks equals abd_hvp (forward-mode Alg. 1) on chains
    of up to 64 DOFs; H is symmetric."""
    d = W.config(2, n_models=16).model
    rng = np.random.default_rng(135)
    q, qp, qc, v = (rng.uniform(-1, 1, d.n_dofs) for _ in range(4))
    dt = 0.03
    m = abd.Model(d)
    hist = cu(np.concatenate([qp, qc]))
    Hg = [h.cpu().numpy() for h in m.hessian(cu(q), hist, dt)]
    Hv = m.hvp(cu(q), hist, cu(v), dt).cpu().numpy()
    do = d.dof_offset
    for i in range(d.n_models):
        sl = slice(do[i], do[i + 1])
        H = Hg[i]
        assert np.max(np.abs(H - H.T)) <= 1e-12 * np.max(np.abs(H))
        hv = H @ v[sl]
        assert np.max(np.abs(hv - Hv[sl])) <= 1e-11 * max(1e-300, np.max(np.abs(Hv[sl]))), i
