"""Python binding of the C ABI in include/abd.h (ctypes; argument marshalling only).

Every step of the computation runs in the HIP library ``libabd.so`` built from
the sources under ``csrc/``.  PyTorch is used for device memory and streams.  There is no
fallback: if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabd.so")

ABD_OK, ABD_EINVAL, ABD_ENOMEM, ABD_EDEVICE, ABD_ENOTSUP = 0, -1, -2, -3, -4
FP64, MIXED = 0, 1
PRECOND_IDENTITY, PRECOND_INERTIA = 0, 2
# default period (accepted iterations) at which a step re-forms its inertia
# preconditioner at the current iterate
REFRESH = 10
FLAG_CONVERGED, FLAG_LS_FLOOR, FLAG_MAX_ITER, FLAG_NONFINITE = 1, 2, 4, 8
SCHEDULE_AUTO, SCHEDULE_WAVE, SCHEDULE_TILE = 0, 1, 2
SOLVER_LBFGS, SOLVER_LM = 0, 1


class ModelDescC(C.Structure):
    _fields_ = [("n_models", C.c_int),
                ("link_offset", C.POINTER(C.c_int)),
                ("parent", C.POINTER(C.c_int)),
                ("dofs_per_link", C.POINTER(C.c_int)),
                ("axis", C.POINTER(C.c_double)),
                ("offset", C.POINTER(C.c_double)),
                ("mass_moment", C.POINTER(C.c_double)),
                ("gravity", C.c_double * 3),
                ("dof_kind", C.POINTER(C.c_int)),
                ("drag", C.POINTER(C.c_double)),
                ("n_contacts", C.c_int),
                ("contact_link", C.POINTER(C.c_int)),
                ("contact_point", C.POINTER(C.c_double)),
                ("contact_plane", C.c_double * 4),
                ("contact_d1", C.c_double),
                ("contact_d2", C.c_double)]

DOF_HINGE, DOF_SLIDE = 0, 1


class StepOptsC(C.Structure):
    _fields_ = [("dt", C.c_double), ("order_K", C.c_int), ("lbfgs_m", C.c_int),
                ("tol", C.c_double), ("max_iter", C.c_int), ("max_ls", C.c_int),
                ("precision", C.c_int), ("precond", C.c_int), ("refresh", C.c_int),
                ("schedule", C.c_int), ("solver", C.c_int)]


STATS_DTYPE = np.dtype([("iterations", np.int32), ("evaluations", np.int32), ("flag", np.int32),
                        ("f32_iterations", np.int32), ("f32_evaluations", np.int32), ("reserved", np.int32),
                        ("grad_norm", np.float64), ("energy", np.float64)])
STATS_BYTES = 40
assert STATS_DTYPE.itemsize == STATS_BYTES

# every exported entry point and its prototype
_PROTOS = {
    "abd_create_model": (C.c_int, [C.POINTER(ModelDescC), C.POINTER(C.c_void_p)]),
    "abd_destroy_model": (None, [C.c_void_p]),
    "abd_model_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "abd_step": (C.c_int, [C.c_void_p, C.POINTER(StepOptsC), C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p]),
    "abd_rollout": (C.c_int, [C.c_void_p, C.POINTER(StepOptsC), C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_int, C.c_void_p]),
    "abd_rollout_noalloc": (C.c_int, [C.c_void_p, C.POINTER(StepOptsC), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_int, C.c_void_p]),
    "abd_objective_grad": (C.c_int, [C.c_void_p, C.POINTER(StepOptsC), C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "abd_hvp": (C.c_int, [C.c_void_p, C.POINTER(StepOptsC), C.c_void_p, C.c_void_p, C.c_void_p,
                          C.c_void_p, C.c_void_p]),
    "abd_hessian": (C.c_int, [C.c_void_p, C.POINTER(StepOptsC), C.c_void_p, C.c_void_p, C.c_void_p,
                              C.c_void_p]),
    "abd_rollout_vjp": (C.c_int, [C.c_void_p, C.POINTER(StepOptsC), C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "abd_poses": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "abd_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libabd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no non-HIP fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class AbdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"abd error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != ABD_OK:
        raise AbdError(rc, load().abd_last_error().decode())


@dataclass
class StepOptions:
    dt: float
    order_K: int = 2
    lbfgs_m: int = 5
    tol: float = 1e-8
    max_iter: int = 500
    max_ls: int = 40
    precision: int = FP64
    precond: int = PRECOND_INERTIA
    refresh: int = REFRESH
    schedule: int = SCHEDULE_AUTO
    solver: int = SOLVER_LBFGS

    def c(self) -> StepOptsC:
        return StepOptsC(self.dt, self.order_K, self.lbfgs_m, self.tol, self.max_iter, self.max_ls,
                         self.precision, self.precond, self.refresh, self.schedule, self.solver)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t, n, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return t


class Model:
    """A batch of articulated models resident on the current HIP device."""

    def __init__(self, desc):
        lib = load()
        self.desc = desc
        self._keep = [np.ascontiguousarray(desc.link_offset, dtype=np.int32),
                      np.ascontiguousarray(desc.parent, dtype=np.int32),
                      np.ascontiguousarray(desc.dofs_per_link, dtype=np.int32),
                      np.ascontiguousarray(desc.axis, dtype=np.float64),
                      np.ascontiguousarray(desc.offset, dtype=np.float64),
                      np.ascontiguousarray(desc.mass_moment, dtype=np.float64)]
        k = self._keep
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        cd = ModelDescC(int(desc.n_models), ip(k[0]), ip(k[1]), ip(k[2]), dp(k[3]), dp(k[4]), dp(k[5]),
                        (C.c_double * 3)(*[float(x) for x in desc.gravity]))
        # optional terms (slides, drag, contact points)
        kind = getattr(desc, "dof_kind", None)
        drag = getattr(desc, "drag", None)
        nc = int(getattr(desc, "n_contacts", 0))
        if kind is not None:
            self._keep.append(np.ascontiguousarray(kind, dtype=np.int32))
            cd.dof_kind = ip(self._keep[-1])
        if drag is not None:
            self._keep.append(np.ascontiguousarray(drag, dtype=np.float64))
            cd.drag = dp(self._keep[-1])
        if nc > 0:
            self._keep += [np.ascontiguousarray(desc.contact_link, dtype=np.int32),
                           np.ascontiguousarray(desc.contact_point, dtype=np.float64)]
            cd.n_contacts = nc
            cd.contact_link = ip(self._keep[-2])
            cd.contact_point = dp(self._keep[-1])
            cd.contact_plane = (C.c_double * 4)(*[float(x) for x in desc.contact_plane])
            cd.contact_d1 = float(desc.contact_d1)
            cd.contact_d2 = float(desc.contact_d2)
        h = C.c_void_p()
        _check(lib.abd_create_model(C.byref(cd), C.byref(h)))
        self._h = h
        nm, nl, nd = C.c_int(), C.c_int(), C.c_int()
        _check(lib.abd_model_info(h, C.byref(nm), C.byref(nl), C.byref(nd)))
        self.n_models, self.n_links, self.n_dofs = nm.value, nl.value, nd.value

    def close(self):
        if getattr(self, "_h", None):
            load().abd_destroy_model(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------------- calls
    def step(self, q_hist: torch.Tensor, q_out: torch.Tensor, opts: StepOptions,
             tau: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None, stream=None):
        """Enqueue one time step.  q_hist = [q_{k-1}; q_k] (2*n_dofs contiguous); for
        order_K > 2, q_hist = [q_{k-1+alpha_{K-2}}; q_k] and q_out receives the K-1
        unknown configurations ([K-1, n_dofs], the last one is q_{k+1})."""
        _dev_f64(q_hist, 2 * self.n_dofs, "q_hist")
        _dev_f64(q_out, (opts.order_K - 1) * self.n_dofs, "q_out")
        if tau is not None:
            _dev_f64(tau, self.n_dofs, "tau")
        if stats is not None and (not stats.is_cuda or stats.numel() * stats.element_size() < STATS_BYTES * self.n_models):
            raise ValueError(f"stats must be a CUDA buffer of {STATS_BYTES} bytes per model")
        o = opts.c()
        _check(load().abd_step(self._h, C.byref(o), _ptr(q_hist), _ptr(tau), _ptr(q_out), _ptr(stats),
                               _stream(stream)))

    def new_stats(self) -> torch.Tensor:
        return torch.zeros((max(1, self.n_models), STATS_BYTES // 8), dtype=torch.float64, device="cuda")

    @staticmethod
    def read_stats(stats: torch.Tensor, n_models: int) -> np.ndarray:
        raw = stats.detach().cpu().numpy().reshape(-1).view(np.uint8)[:STATS_BYTES * n_models]
        return raw.view(STATS_DTYPE).copy()

    def objective_grad(self, q, q_hist, dt, tau=None, precision=FP64, order_K=2, want_tau_grad=False,
                       stream=None):
        """Objective per model and gradient.  order_K > 2: Eq. EQHOC with q the K-1
        unknown configurations ([K-1, n_dofs]); the gradient has the same shape.
        With want_tau_grad, also returns dE/dtau [n_dofs] (computed by the library)."""
        U = order_K - 1
        _dev_f64(q, U * self.n_dofs, "q")
        _dev_f64(q_hist, 2 * self.n_dofs, "q_hist")
        if tau is not None:
            _dev_f64(tau, self.n_dofs, "tau")
        E = torch.zeros(max(1, self.n_models), dtype=torch.float64, device="cuda")
        g = torch.zeros(max(1, U * self.n_dofs), dtype=torch.float64, device="cuda")
        gt = torch.zeros(max(1, self.n_dofs), dtype=torch.float64, device="cuda") if want_tau_grad else None
        o = StepOptions(dt=dt, precision=precision, order_K=order_K).c()
        _check(load().abd_objective_grad(self._h, C.byref(o), _ptr(q), _ptr(q_hist), _ptr(tau), _ptr(E),
                                         _ptr(g), _ptr(gt), _stream(stream)))
        g = g[:U * self.n_dofs]
        out = (E[:self.n_models], (g if order_K == 2 else g.view(U, self.n_dofs)))
        return out + (gt[:self.n_dofs],) if want_tau_grad else out

    def hvp(self, q, q_hist, v, dt, stream=None):
        """Hessian-vector product of the step objective at q (float64)."""
        _dev_f64(q, self.n_dofs, "q")
        _dev_f64(q_hist, 2 * self.n_dofs, "q_hist")
        _dev_f64(v, self.n_dofs, "v")
        Hv = torch.zeros(max(1, self.n_dofs), dtype=torch.float64, device="cuda")
        o = StepOptions(dt=dt).c()
        _check(load().abd_hvp(self._h, C.byref(o), _ptr(q), _ptr(q_hist), _ptr(v), _ptr(Hv), _stream(stream)))
        return Hv[:self.n_dofs]

    def hessian(self, q, q_hist, dt, stream=None):
        """Explicit Hessian of the step objective at q (abd_hessian): a list of dense
        per-model [n_i, n_i] blocks (views of one device buffer)."""
        _dev_f64(q, self.n_dofs, "q")
        _dev_f64(q_hist, 2 * self.n_dofs, "q_hist")
        per = np.diff(np.asarray(self.desc.dof_offset)).astype(np.int64)
        H = torch.zeros(max(1, int(np.sum(per * per))), dtype=torch.float64, device="cuda")
        o = StepOptions(dt=dt).c()
        _check(load().abd_hessian(self._h, C.byref(o), _ptr(q), _ptr(q_hist), _ptr(H), _stream(stream)))
        out, off = [], 0
        for nd in per:
            out.append(H[off:off + nd * nd].view(int(nd), int(nd)))
            off += int(nd * nd)
        return out

    def rollout_vjp(self, q_init, q_traj, dL_dq_traj, dt, tol=1e-10, max_iter=200, precond=PRECOND_INERTIA,
                    want_tau=True, stats=None, stream=None):
        """Reverse-mode derivative of a rollout (abd_rollout_vjp).

        q_init [2n] = q_{-1}, q_0; q_traj [T, n] = q_1..q_T; dL_dq_traj [T, n].
        Returns (dL/dq_init [2n], dL/dtau [T, n] or None)."""
        n = self.n_dofs
        T = q_traj.shape[0] if q_traj.dim() == 2 else q_traj.numel() // max(1, n)
        _dev_f64(q_init, 2 * n, "q_init")
        _dev_f64(q_traj, T * n, "q_traj")
        _dev_f64(dL_dq_traj, T * n, "dL_dq_traj")
        if stats is not None and stats.numel() * stats.element_size() < STATS_BYTES * self.n_models * T:
            raise ValueError(f"stats must hold {STATS_BYTES} bytes per model and step")
        g_init = torch.zeros(max(1, 2 * n), dtype=torch.float64, device="cuda")
        g_tau = torch.zeros((max(1, T), max(1, n)), dtype=torch.float64, device="cuda") if want_tau else None
        o = StepOptions(dt=dt, tol=tol, max_iter=max_iter, precond=precond).c()
        _check(load().abd_rollout_vjp(self._h, C.byref(o), _ptr(q_init), _ptr(q_traj), _ptr(dL_dq_traj),
                                      _ptr(g_init), _ptr(g_tau), _ptr(stats), int(T), _stream(stream)))
        return g_init[:2 * n], (g_tau[:T, :n] if want_tau else None)

    def poses(self, q, stream=None):
        _dev_f64(q, self.n_dofs, "q")
        out = torch.zeros((max(1, self.n_links), 3, 4), dtype=torch.float64, device="cuda")
        _check(load().abd_poses(self._h, _ptr(q), _ptr(out), _stream(stream)))
        return out[:self.n_links]

    def rollout(self, q_init: torch.Tensor, steps: int, opts: StepOptions, torque=None,
                q_traj: Optional[torch.Tensor] = None, stats: Optional[torch.Tensor] = None, stream=None):
        """Enqueue `steps` time steps in one launch (abd_rollout).

        q_init = [q_{-1}; q_0] (2*n_dofs); torque [steps, n_dofs] or None.
        Returns (q_traj [steps, n_dofs] = q_1..q_steps, stats buffer [steps*n_models] or None).
        order_K > 2: q_init = [q_{-1+alpha_{K-2}}; q_0] and q_traj is [steps, K-1, n_dofs]
        (every step's unknown configurations)."""
        n = self.n_dofs
        U = opts.order_K - 1
        _dev_f64(q_init, 2 * n, "q_init")
        if q_traj is None:
            shape = (max(1, steps), n) if U == 1 else (max(1, steps), U, n)
            q_traj = torch.empty(shape, dtype=torch.float64, device="cuda")
        _dev_f64(q_traj, max(1, steps) * U * n, "q_traj")
        if torque is not None:
            _dev_f64(torque, steps * n, "torque")
        if stats is not None and stats.numel() * stats.element_size() < STATS_BYTES * self.n_models * steps:
            raise ValueError(f"stats must hold {STATS_BYTES} bytes per model and step")
        o = opts.c()
        _check(load().abd_rollout(self._h, C.byref(o), _ptr(q_init), _ptr(torque), _ptr(q_traj), _ptr(stats),
                                  int(steps), _stream(stream)))
        return q_traj[:steps], stats

    def rollout_noalloc(self, q_init: torch.Tensor, steps: int, opts: StepOptions, q_traj: torch.Tensor,
                        stats: torch.Tensor, torque=None, stream=None):
        """abd_rollout_noalloc: as rollout, with caller-provided outputs (q_traj, stats)
        and the step scratch in the library's fixed device array (no allocation)."""
        n = self.n_dofs
        _dev_f64(q_init, 2 * n, "q_init")
        _dev_f64(q_traj, max(1, steps) * (opts.order_K - 1) * n, "q_traj")
        if torque is not None:
            _dev_f64(torque, steps * n, "torque")
        if stats is None or stats.numel() * stats.element_size() < STATS_BYTES * self.n_models * steps:
            raise ValueError(f"stats must hold {STATS_BYTES} bytes per model and step")
        o = opts.c()
        _check(load().abd_rollout_noalloc(self._h, C.byref(o), _ptr(q_init), _ptr(torque), _ptr(q_traj),
                                          _ptr(stats), int(steps), _stream(stream)))
        return q_traj, stats

    def new_rollout_stats(self, steps: int) -> torch.Tensor:
        return torch.zeros((max(1, steps * self.n_models), STATS_BYTES // 8), dtype=torch.float64, device="cuda")

    def read_rollout_stats(self, stats: torch.Tensor, steps: int) -> np.ndarray:
        return self.read_stats(stats, steps * self.n_models).reshape(steps, self.n_models)

    def step_loop(self, q0: torch.Tensor, steps: int, opts: StepOptions, q_init_prev=None, torque=None):
        """Trajectory q_0..q_steps from one abd_step call per step (zero initial velocity
        unless q_init_prev is given); the buffer holds [q_{-1}, q_0, q_1, ...] so every
        step reads [q_{k-1}; q_k] in place."""
        n = self.n_dofs
        buf = torch.empty((steps + 2, n), dtype=torch.float64, device="cuda")
        buf[1] = q0
        buf[0] = q0 if q_init_prev is None else q_init_prev
        stats = []
        for k in range(steps):
            st = self.new_stats()
            tau = None if torque is None else torque[k]
            self.step(buf[k:k + 2].reshape(-1), buf[k + 2], opts, tau=tau, stats=st)
            stats.append(st)
        torch.cuda.synchronize()
        return buf[1:], [self.read_stats(s, self.n_models) for s in stats]


# ------------------------------------------------------------------ autograd
class ObjectiveFunction(torch.autograd.Function):
    """E(q) per model (abd_objective_grad) as a differentiable function of q and
    tau.  Backward: dE/dq (the Alg. 1 gradient) and dE/dtau, both computed by
    the library in the forward call; the backward only scales them by the
    incoming per-model weights.  q_hist is treated as a constant."""

    @staticmethod
    def forward(ctx, q, tau, model, q_hist, dt):
        E, g, gt = model.objective_grad(q.detach().contiguous(), q_hist.detach().contiguous(), dt,
                                        tau=None if tau is None else tau.detach().contiguous(),
                                        want_tau_grad=True)
        ctx.has_tau = tau is not None
        dof_model = _dof_model_index(model)
        ctx.save_for_backward(g, gt, dof_model)
        return E

    @staticmethod
    def backward(ctx, gE):
        g, gt, dof_model = ctx.saved_tensors
        w = gE[dof_model]
        return w * g, (w * gt if ctx.has_tau else None), None, None, None


def _dof_model_index(model):
    """Model index of every DOF (cached on the model)."""
    idx = getattr(model, "_dof_model", None)
    if idx is None:
        per_model = np.diff(np.asarray(model.desc.dof_offset)).astype(np.int64)
        idx = torch.as_tensor(np.repeat(np.arange(model.n_models), per_model), device="cuda")
        model._dof_model = idx
    return idx


def objective(model, q, q_hist, dt, tau=None):
    """Differentiable per-model objective E(q) (see ObjectiveFunction)."""
    return ObjectiveFunction.apply(q, tau, model, q_hist, dt)


class RolloutFunction(torch.autograd.Function):
    """q_1..q_T = rollout(q_{-1}, q_0, tau) (abd_rollout, float64) with its
    reverse-mode derivative by implicit differentiation (abd_rollout_vjp)."""

    @staticmethod
    def forward(ctx, q_init, torque, model, steps, opts, vjp_opts):
        traj, _ = model.rollout(q_init.detach().contiguous(), steps, opts,
                                torque=None if torque is None else torque.detach().contiguous())
        ctx.model, ctx.opts, ctx.vjp_opts, ctx.has_tau = model, opts, vjp_opts, torque is not None
        ctx.save_for_backward(q_init.detach(), traj)
        return traj.clone()

    @staticmethod
    def backward(ctx, g_traj):
        q_init, traj = ctx.saved_tensors
        g_init, g_tau = ctx.model.rollout_vjp(q_init.contiguous(), traj.contiguous(), g_traj.contiguous(),
                                              ctx.opts.dt, want_tau=ctx.has_tau, **ctx.vjp_opts)
        return g_init, g_tau, None, None, None, None


def rollout(model, q_init, steps, opts, torque=None, vjp_tol=1e-10, vjp_max_iter=200):
    """Differentiable rollout: returns q_1..q_steps [steps, n_dofs]; gradients flow
    to q_init = [q_{-1}; q_0] and to torque [steps, n_dofs]."""
    if opts.precision != FP64:
        raise ValueError("the differentiable rollout runs in float64 (precision=FP64)")
    if opts.order_K != 2:
        raise ValueError("the differentiable rollout is defined for order_K = 2 (Eq. EQ); "
                         "abd_rollout_vjp has no order-K derivative")
    return RolloutFunction.apply(q_init, torque, model, steps, opts,
                                 dict(tol=vjp_tol, max_iter=vjp_max_iter))
