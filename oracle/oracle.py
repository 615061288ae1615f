"""ctypes front end of the FP64 CPU oracle (abd_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product path (the HIP library and its
Python binding) never imports this module.

Besides marshalling, this module holds two plain numerical helpers that use
the C routines as their only source of objective values and gradients:
``newton_polish`` (Newton iterations with a central-difference Hessian of the
Alg. 1 gradient, used to pin the L-BFGS result to the exact minimizer) and
``rollout`` (a loop of steps).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abd_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

FLAG_CONVERGED, FLAG_LS_FLOOR, FLAG_MAX_ITER, FLAG_NONFINITE = 1, 2, 4, 8
EPS64 = 2.0 ** -53
EPS32 = 2.0 ** -24
# default period (accepted iterations) at which a step re-forms H_q at the
# current iterate (the value the GPU library's step options default to)
REFRESH = 10


class OrcOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("order_K", C.c_int), ("lbfgs_m", C.c_int),
                ("tol", C.c_double), ("max_iter", C.c_int), ("max_ls", C.c_int),
                ("eps_w", C.c_double), ("precond", C.c_int), ("refresh", C.c_int)]


class OrcLmOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("order_K", C.c_int), ("max_iter", C.c_int), ("tol", C.c_double),
                ("lambda0", C.c_double), ("geodesic", C.c_int), ("geo_h", C.c_double),
                ("geo_alpha", C.c_double)]


class OrcStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("evaluations", C.c_int), ("flag", C.c_int),
                ("pad", C.c_int), ("grad_norm", C.c_double), ("energy", C.c_double)]


STATS_DTYPE = np.dtype([("iterations", np.int32), ("evaluations", np.int32), ("flag", np.int32),
                        ("pad", np.int32), ("grad_norm", np.float64), ("energy", np.float64)])


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE arithmetic, OpenMP over models)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unknown-pragmas", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        _lib.orc_create.restype = C.c_void_p
        _lib.orc_create.argtypes = [C.c_int, ip, ip, ip, dp, dp, dp, dp]
        _lib.orc_free.argtypes = [C.c_void_p]
        _lib.orc_set_extras.argtypes = [C.c_void_p, ip, dp, C.c_int, ip, dp, dp, C.c_double, C.c_double]
        _lib.orc_set_extras.restype = C.c_int
        _lib.orc_poses.argtypes = [C.c_void_p, dp, dp, C.c_int]
        _lib.orc_objective_grad.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, dp, dp, dp, C.c_int]
        _lib.orc_objective_Iform.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, dp, C.c_int]
        _lib.orc_alg1_I.argtypes = [C.c_void_p, dp, dp, dp, dp, C.c_int]
        _lib.orc_inertia_diag.argtypes = [C.c_void_p, dp, dp, C.c_int]
        _lib.orc_inertia_matrix.argtypes = [C.c_void_p, dp, dp, C.c_int]
        _lib.orc_hessian.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, C.c_int]
        _lib.orc_collocation.argtypes = [C.c_int, dp, dp]
        _lib.orc_collocation.restype = C.c_int
        _lib.orc_eqhoc_objective_grad.argtypes = [C.c_void_p, C.c_int, C.c_double, dp, dp, dp, dp, dp, C.c_int]
        _lib.orc_eqhoc_residual_jacobian.argtypes = [C.c_void_p, C.c_int, C.c_double, dp, dp, dp, dp, dp,
                                                     C.c_int]
        _lib.orc_step_hoc.argtypes = [C.c_void_p, C.POINTER(OrcOpts), dp, dp, dp, C.c_void_p, C.c_int]
        _lib.orc_step_hoc.restype = C.c_int
        _lib.orc_step_lm_hoc.argtypes = [C.c_void_p, C.POINTER(OrcLmOpts), dp, dp, dp, C.c_void_p, C.c_int]
        _lib.orc_step_lm_hoc.restype = C.c_int
        _lib.orc_cross_hessian.argtypes = [C.c_void_p, dp, dp, C.c_double, dp, C.c_int]
        _lib.orc_step.argtypes = [C.c_void_p, C.POINTER(OrcOpts), dp, dp, dp, C.c_void_p, C.c_int]
        _lib.orc_step.restype = C.c_int
        _lib.orc_energy_report.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, C.c_int]
    return _lib


def _d(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def collocation(K: int):
    """(tau [K+1], w [K-1, K+1]) of the order-K position-based collocation (Eq. HOC)."""
    tau = np.zeros(K + 1)
    w = np.zeros((K - 1) * (K + 1))
    if lib().orc_collocation(K, _d(tau), _d(w)) != 0:
        raise ValueError(f"order {K} out of range")
    return tau, w.reshape(K - 1, K + 1)


class Oracle:
    """FP64 oracle bound to one batch of models (a ``workloads.ModelDesc``)."""

    def __init__(self, desc, threads: Optional[int] = None):
        self.desc = desc
        self.threads = threads or default_threads()
        self._keep = [np.ascontiguousarray(desc.link_offset, dtype=np.int32),
                      np.ascontiguousarray(desc.parent, dtype=np.int32),
                      np.ascontiguousarray(desc.dofs_per_link, dtype=np.int32),
                      _f64(desc.axis), _f64(desc.offset), _f64(desc.mass_moment),
                      _f64(desc.gravity)]
        k = self._keep
        self._h = lib().orc_create(desc.n_models, _i(k[0]), _i(k[1]), _i(k[2]),
                                   _d(k[3]), _d(k[4]), _d(k[5]), _d(k[6]))
        self.n_models, self.n_dofs, self.n_links = desc.n_models, desc.n_dofs, desc.n_links
        self.extras = bool(getattr(desc, "has_extras", False))
        if self.extras:
            kind = None if desc.dof_kind is None else np.ascontiguousarray(desc.dof_kind, dtype=np.int32)
            drag = None if desc.drag is None else _f64(desc.drag)
            nc = desc.n_contacts
            cl = np.ascontiguousarray(desc.contact_link if nc else np.zeros(1), dtype=np.int32)
            cp = _f64(desc.contact_point if nc else np.zeros(3))
            plane = _f64(desc.contact_plane)
            self._keep += [kind, drag, cl, cp, plane]
            rc = lib().orc_set_extras(self._h, None if kind is None else _i(kind), _d(drag), nc, _i(cl), _d(cp),
                                      _d(plane), float(desc.contact_d1), float(desc.contact_d2))
            if rc != 0:
                raise ValueError("invalid slide / drag / contact description")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    def _no_extras(self, what):
        if self.extras:
            raise NotImplementedError(f"{what}: slide, drag and contact terms enter the order-2 objective "
                                      f"(Eq. EQ) and its L-BFGS step only")

    # ---------------------------------------------------------------- queries
    def poses(self, q) -> np.ndarray:
        out = np.zeros((self.n_links, 3, 4))
        lib().orc_poses(self._h, _d(_f64(q)), _d(out), self.threads)
        return out

    def objective_grad(self, q, q_prev, q_curr, dt, tau=None):
        E = np.zeros(self.n_models)
        g = np.zeros(self.n_dofs)
        S = np.zeros(self.n_models)
        hist = _f64(np.concatenate([q_prev, q_curr]))
        tau = None if tau is None else _f64(tau)
        lib().orc_objective_grad(self._h, dt, _d(_f64(q)), _d(hist), _d(tau), _d(E), _d(g), _d(S),
                                 self.threads)
        return E, g, S

    def objective_Iform(self, q, q_prev, q_curr, dt, tau=None):
        E = np.zeros(self.n_models)
        hist = _f64(np.concatenate([q_prev, q_curr]))
        tau = None if tau is None else _f64(tau)
        lib().orc_objective_Iform(self._h, dt, _d(_f64(q)), _d(hist), _d(tau), _d(E), self.threads)
        return E

    def alg1_I(self, q_a, q_b):
        I = np.zeros(self.n_models)
        g = np.zeros(self.n_dofs)
        lib().orc_alg1_I(self._h, _d(_f64(q_a)), _d(_f64(q_b)), _d(I), _d(g), self.threads)
        return I, g

    def inertia_diag(self, q) -> np.ndarray:
        h = np.zeros(self.n_dofs)
        lib().orc_inertia_diag(self._h, _d(_f64(q)), _d(h), self.threads)
        return h

    def inertia_matrix(self, q):
        """List of dense per-model joint-space inertia matrices at q."""
        nd = np.diff(self.desc.dof_offset).astype(np.int64)
        buf = np.zeros(int(np.sum(nd * nd)))
        lib().orc_inertia_matrix(self._h, _d(_f64(q)), _d(buf), self.threads)
        out, o = [], 0
        for n in nd:
            out.append(buf[o:o + n * n].reshape(n, n))
            o += n * n
        return out

    def _blocks(self, buf):
        nd = np.diff(self.desc.dof_offset).astype(np.int64)
        out, o = [], 0
        for n in nd:
            out.append(buf[o:o + n * n].reshape(n, n))
            o += n * n
        return out

    def _block_buffer(self):
        nd = np.diff(self.desc.dof_offset).astype(np.int64)
        return np.zeros(max(1, int(np.sum(nd * nd))))

    def hessian(self, q, q_prev, q_curr, dt):
        """List of dense per-model Hessians d2E/dq dq of the step objective at q."""
        buf = self._block_buffer()
        hist = _f64(np.concatenate([q_prev, q_curr]))
        lib().orc_hessian(self._h, dt, _d(_f64(q)), _d(hist), _d(buf), self.threads)
        return self._blocks(buf)

    def cross_hessian(self, q, q_other, scale):
        """List of per-model C[a][b] = scale sum_l <dA_l(q)/dq_a M_l, dA_l(q_o)/dq_o,b>."""
        self._no_extras("cross_hessian")
        buf = self._block_buffer()
        lib().orc_cross_hessian(self._h, _d(_f64(q)), _d(_f64(q_other)), scale, _d(buf), self.threads)
        return self._blocks(buf)

    def energy_report(self, q_prev, q_curr, dt) -> np.ndarray:
        H = np.zeros(self.n_models)
        lib().orc_energy_report(self._h, dt, _d(_f64(q_prev)), _d(_f64(q_curr)), _d(H), self.threads)
        return H

    # ------------------------------------------------------------------- step
    def step(self, q_prev, q_curr, dt, tau=None, lbfgs_m=5, tol=1e-8, max_iter=500, max_ls=40,
             eps_w=EPS64, order_K=2, precond=2, refresh=REFRESH):
        opts = OrcOpts(dt, order_K, lbfgs_m, tol, max_iter, max_ls, eps_w, precond, refresh)
        hist = _f64(np.concatenate([q_prev, q_curr]))
        out = np.zeros(self.n_dofs)
        stats = np.zeros(self.n_models, dtype=STATS_DTYPE)
        tau = None if tau is None else _f64(tau)
        rc = lib().orc_step(self._h, C.byref(opts), _d(hist), _d(tau), _d(out),
                            stats.ctypes.data_as(C.c_void_p), self.threads)
        if rc != 0:
            raise ValueError(f"orc_step failed ({rc})")
        return out, stats

    def rollout(self, q0, steps, dt, q_init_prev=None, torque=None, **kw):
        """States q_0..q_steps (zero initial velocity unless q_init_prev is given)."""
        qs = [np.array(q0, dtype=np.float64)]
        prev = qs[0].copy() if q_init_prev is None else np.array(q_init_prev, dtype=np.float64)
        stats = []
        for k in range(steps):
            tau = None if torque is None else torque[k]
            nxt, st = self.step(prev, qs[-1], dt, tau=tau, **kw)
            prev = qs[-1]
            qs.append(nxt)
            stats.append(st)
        return np.stack(qs), stats

    def eqhoc_objective_grad(self, K, dt, q_prev, q_curr, q_unknown, tau=None):
        """Eq. EQHOC per model and its gradient [K-1, n] w.r.t. the unknown points."""
        self._no_extras("eqhoc_objective_grad")
        E = np.zeros(self.n_models)
        g = np.zeros((K - 1) * self.n_dofs)
        known = _f64(np.concatenate([q_prev, q_curr]))
        unk = _f64(np.asarray(q_unknown).reshape(-1))
        tau = None if tau is None else _f64(tau)
        lib().orc_eqhoc_objective_grad(self._h, K, dt, _d(known), _d(unk), _d(tau), _d(E), _d(g), self.threads)
        return E, g.reshape(K - 1, self.n_dofs)

    def eqhoc_residual_jacobian(self, K, dt, q_prev, q_curr, q_unknown, tau=None, jacobian=True):
        """Residuals dt^2 r_u of Eq. HOC ([K-1, n]) at the unknown points and, with
        jacobian, the list of dense per-model Jacobians ([(K-1) nd]^2, unknown-major)."""
        self._no_extras("eqhoc_residual_jacobian")
        U = K - 1
        R = np.zeros(U * self.n_dofs)
        known = _f64(np.concatenate([q_prev, q_curr]))
        unk = _f64(np.asarray(q_unknown).reshape(-1))
        tau = None if tau is None else _f64(tau)
        nd = np.diff(self.desc.dof_offset).astype(np.int64)
        J = np.zeros(max(1, int(np.sum((U * nd) ** 2)))) if jacobian else None
        lib().orc_eqhoc_residual_jacobian(self._h, K, dt, _d(known), _d(unk), _d(tau), _d(R), _d(J),
                                          self.threads)
        R = R.reshape(U, self.n_dofs)
        if not jacobian:
            return R, None
        out, o = [], 0
        for n in nd:
            N = int(U * n)
            out.append(J[o:o + N * N].reshape(N, N))
            o += N * N
        return R, out

    def step_hoc(self, K, q_prev, q_curr, dt, tau=None, lbfgs_m=5, tol=1e-8, max_iter=500, max_ls=40,
                 eps_w=EPS64, precond=2):
        """One Eq. EQHOC step: returns the K-1 unknown configurations [K-1, n] and stats.
        q_prev is the previous step's alpha_{K-2} point, q_curr = q_k."""
        self._no_extras("step_hoc")
        opts = OrcOpts(dt, K, lbfgs_m, tol, max_iter, max_ls, eps_w, precond, 0)
        known = _f64(np.concatenate([q_prev, q_curr]))
        out = np.zeros((K - 1) * self.n_dofs)
        stats = np.zeros(self.n_models, dtype=STATS_DTYPE)
        tau = None if tau is None else _f64(tau)
        rc = lib().orc_step_hoc(self._h, C.byref(opts), _d(known), _d(tau), _d(out),
                                stats.ctypes.data_as(C.c_void_p), self.threads)
        if rc != 0:
            raise ValueError(f"orc_step_hoc failed ({rc})")
        return out.reshape(K - 1, self.n_dofs), stats

    def step_lm(self, K, q_prev, q_curr, dt, tau=None, tol=1e-8, max_iter=300, lambda0=1e-3, geodesic=True,
                geo_h=0.1, geo_alpha=0.75):
        """One Eq. EQHOC step (order K >= 2) by Levenberg-Marquardt (orc_step_lm_hoc):
        returns the K-1 unknown configurations [K-1, n] and stats (iterations =
        LM iterations, accepted or rejected; evaluations = residual evaluations)."""
        self._no_extras("step_lm")
        opts = OrcLmOpts(dt, K, max_iter, tol, lambda0, 1 if geodesic else 0, geo_h, geo_alpha)
        known = _f64(np.concatenate([q_prev, q_curr]))
        out = np.zeros((K - 1) * self.n_dofs)
        stats = np.zeros(self.n_models, dtype=STATS_DTYPE)
        tau = None if tau is None else _f64(tau)
        rc = lib().orc_step_lm_hoc(self._h, C.byref(opts), _d(known), _d(tau), _d(out),
                                   stats.ctypes.data_as(C.c_void_p), self.threads)
        if rc != 0:
            raise ValueError(f"orc_step_lm_hoc failed ({rc})")
        return out.reshape(K - 1, self.n_dofs), stats

    def step_lm_eq(self, q_prev, q_curr, dt, tau=None, tol=1e-8, max_iter=300, lambda0=1e-3):
        """One step of Eq. EQ (order 2) by Levenberg-Marquardt (Sec. 5): the kinetic
        term is an integral of squares whose J^T J is the joint-space inertia
        H_q(q) = sum_l tr(dA_l/dq_i M_l dA_l/dq_j^T) (orc_inertia_matrix); each
        iteration solves (H_q + lambda I) v = -grad E by a dense Cholesky and
        accepts v if it decreases E.  lambda starts at lambda0 max diag(H_q), stays
        >= 1e-15 max diag(H_q), and follows Nielsen's rule with the gain ratio
        against the model decrease -g.v - v.H_q v / 2.  Warm start 2 q_k - q_{k-1}.
        Stops when |grad E| <= tol |grad E(warm start)| (flag 1), when lambda
        overflows or an accepted point equals the iterate (flag 2), or after max_iter
        iterations, accepted or rejected (flag 4).  Returns (q, stats); stats
        count iterations and objective evaluations."""
        self._no_extras("step_lm_eq")
        qp, qc = _f64(q_prev), _f64(q_curr)
        do = self.desc.dof_offset
        nm = self.n_models
        q = 2.0 * qc - qp
        stats = np.zeros(nm, dtype=STATS_DTYPE)
        E, g, _ = self.objective_grad(q, qp, qc, dt, tau)
        stats["evaluations"] = 1
        g0 = np.array([np.linalg.norm(g[do[i]:do[i + 1]]) for i in range(nm)])
        lam = np.full(nm, -1.0)
        nu = np.full(nm, 2.0)
        active = np.ones(nm, bool)
        for i in range(nm):
            if not np.isfinite(E[i]) or not np.all(np.isfinite(g[do[i]:do[i + 1]])):
                stats["flag"][i] = FLAG_NONFINITE
                active[i] = False
            elif g0[i] == 0.0:
                stats["flag"][i] = FLAG_CONVERGED
                active[i] = False
        for _ in range(max_iter):
            if not active.any():
                break
            H = self.inertia_matrix(q)
            qt = q.copy()
            pred = np.zeros(nm)
            tried = np.zeros(nm, bool)
            for i in np.nonzero(active)[0]:
                sl = slice(do[i], do[i + 1])
                stats["iterations"][i] += 1
                dmax = float(np.max(np.diag(H[i])))
                if lam[i] < 0.0:
                    lam[i] = lambda0 * dmax
                lam[i] = max(lam[i], 1e-15 * dmax)
                if not lam[i] <= 1e300:
                    stats["flag"][i] = FLAG_LS_FLOOR
                    active[i] = False
                    continue
                try:
                    L = np.linalg.cholesky(H[i] + lam[i] * np.eye(H[i].shape[0]))
                except np.linalg.LinAlgError:
                    lam[i] *= nu[i]
                    nu[i] *= 2.0
                    continue
                v = -np.linalg.solve(L.T, np.linalg.solve(L, g[sl]))
                qt[sl] = q[sl] + v
                pred[i] = -(g[sl] @ v) - 0.5 * (v @ (H[i] @ v))
                tried[i] = True
            if not tried.any():
                continue
            Et, gt, _ = self.objective_grad(qt, qp, qc, dt, tau)
            for i in np.nonzero(tried)[0]:
                sl = slice(do[i], do[i + 1])
                stats["evaluations"][i] += 1
                if not (np.isfinite(Et[i]) and Et[i] < E[i]):
                    lam[i] *= nu[i]
                    nu[i] *= 2.0
                    continue
                if np.array_equal(qt[sl], q[sl]):
                    stats["flag"][i] = FLAG_LS_FLOOR
                    active[i] = False
                    continue
                rho = min(1.0, (E[i] - Et[i]) / max(pred[i], 1e-300))
                lam[i] *= max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)
                nu[i] = 2.0
                q[sl] = qt[sl]
                g[sl] = gt[sl]
                E[i] = Et[i]
                if np.linalg.norm(g[sl]) <= tol * g0[i]:
                    stats["flag"][i] = FLAG_CONVERGED
                    active[i] = False
        stats["flag"][active] = FLAG_MAX_ITER
        for i in range(nm):
            stats["grad_norm"][i] = np.linalg.norm(g[do[i]:do[i + 1]])
            stats["energy"][i] = E[i]
        return q, stats

    def rollout_lm(self, K, q_prev, q0, steps, dt, **kw):
        """Order-K rollout by Levenberg-Marquardt steps: q_0..q_steps and the stats."""
        qs = [np.array(q0, dtype=np.float64)]
        prev = np.array(q_prev, dtype=np.float64)
        stats = []
        for _ in range(steps):
            pts, st = self.step_lm(K, prev, qs[-1], dt, **kw)
            prev = pts[K - 3] if K >= 3 else qs[-1]
            qs.append(pts[K - 2].copy())
            stats.append(st)
        return np.stack(qs), stats

    def rollout_hoc(self, K, q_prev, q0, steps, dt, **kw):
        """Order-K rollout from the known points (q_{-1+alpha_{K-2}}, q_0): returns
        q_0..q_steps at whole steps and the per-step stats."""
        qs = [np.array(q0, dtype=np.float64)]
        prev = np.array(q_prev, dtype=np.float64)
        stats = []
        for _ in range(steps):
            pts, st = self.step_hoc(K, prev, qs[-1], dt, **kw)
            prev = pts[K - 3] if K >= 3 else qs[-1]
            qs.append(pts[K - 2].copy())
            stats.append(st)
        return np.stack(qs), stats

    def rollout_vjp(self, q_init_prev, q0, traj, dt, dL_dtraj):
        """Reverse-mode derivative of a rollout by the implicit function theorem.

        Step k defines q_{k+1} through the stationarity condition of its objective
        (Eq. PBAD): g(q_{k+1}; q_k, q_{k-1}, tau_k) = 0.  Differentiating it,
            H dq_{k+1} + C_k dq_k + C_{k-1} dq_{k-1} - dt^2 dtau_k = 0,
        with H the Hessian at q_{k+1} and C_k, C_{k-1} the mixed second
        derivatives (scales -2 and +1).  Given lambda = dL/dq_{k+1} (complete once
        every later step has been processed), mu = H^{-1} lambda and
            dL/dq_k += -C_k^T mu,  dL/dq_{k-1} += -C_{k-1}^T mu,  dL/dtau_k = dt^2 mu.
        traj = [q_1..q_T] (T x n); dL_dtraj = dL/dq_1..q_T (T x n, the explicit
        dependence of the loss).  Returns (dL/dq_{-1}, dL/dq_0, dL/dtau [T x n]).
        Dense solves, model by model."""
        self._no_extras("rollout_vjp")
        traj = np.asarray(traj, dtype=np.float64)
        T = traj.shape[0]
        n = self.n_dofs
        qs = [np.asarray(q_init_prev, np.float64), np.asarray(q0, np.float64)] + [traj[k] for k in range(T)]
        lam = [np.zeros(n), np.zeros(n)] + [np.array(dL_dtraj[k], dtype=np.float64) for k in range(T)]
        dtau = np.zeros((T, n))
        do = self.desc.dof_offset
        for k in range(T - 1, -1, -1):
            q, qc, qp = qs[k + 2], qs[k + 1], qs[k]
            H = self.hessian(q, qp, qc, dt)
            Cc = self.cross_hessian(q, qc, -2.0)
            Cp = self.cross_hessian(q, qp, 1.0)
            for i in range(self.n_models):
                sl = slice(do[i], do[i + 1])
                if do[i + 1] == do[i]:
                    continue
                mu = np.linalg.solve(H[i], lam[k + 2][sl])
                lam[k + 1][sl] -= Cc[i].T @ mu
                lam[k][sl] -= Cp[i].T @ mu
                dtau[k, sl] = dt * dt * mu
        return lam[0], lam[1], dtau

    # ---------------------------------------------------------------- helpers
    def newton_polish(self, q, q_prev, q_curr, dt, tau=None, iters=8, h=1e-6):
        """Newton on grad E = 0 with a central-difference Hessian of the Alg. 1
        gradient, model by model.  Returns the polished q and the final |g| per model."""
        q = _f64(q).copy()
        do = self.desc.dof_offset
        gnorm = np.zeros(self.n_models)
        for _ in range(iters):
            E, g, _ = self.objective_grad(q, q_prev, q_curr, dt, tau)
            nmax = int(np.max(np.diff(do))) if self.n_models else 0
            Hs = [np.zeros((do[i + 1] - do[i],) * 2) for i in range(self.n_models)]
            for j in range(nmax):
                qp, qm = q.copy(), q.copy()
                idx = [do[i] + j for i in range(self.n_models) if do[i] + j < do[i + 1]]
                qp[idx] += h
                qm[idx] -= h
                _, gp, _ = self.objective_grad(qp, q_prev, q_curr, dt, tau)
                _, gm, _ = self.objective_grad(qm, q_prev, q_curr, dt, tau)
                col = (gp - gm) / (2 * h)
                for i in range(self.n_models):
                    if do[i] + j < do[i + 1]:
                        Hs[i][:, j] = col[do[i]:do[i + 1]]
            for i in range(self.n_models):
                sl = slice(do[i], do[i + 1])
                if do[i + 1] == do[i]:
                    continue
                H = 0.5 * (Hs[i] + Hs[i].T)
                q[sl] -= np.linalg.solve(H, g[sl])
        _, g, _ = self.objective_grad(q, q_prev, q_curr, dt, tau)
        for i in range(self.n_models):
            gnorm[i] = np.linalg.norm(g[do[i]:do[i + 1]])
        return q, gnorm
