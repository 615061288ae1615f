// second_order.hip -- Hessian-vector products and the rollout derivative (implicit
// differentiation of Eq. PBAD).
#include "abd_device.h"

namespace {

struct HvpArgs {
  DevModel d;
  double dt2;
  const double* q;
  const double* q_prev;
  const double* q_curr;
  const double* v;
  double* Hv;
};

__global__ void __launch_bounds__(kWave) k_hvp(HvpArgs a) {
  const DevModel& d = a.d;
  const int model = blockIdx.x, lane = threadIdx.x;
  const int f0 = d.f0[model], nf = d.f0[model + 1] - f0;
  if (nf == 0) return;
  const bool valid = lane < nf;
  const int f = f0 + (valid ? lane : 0);
  const FrameGeo geo = load_geo(d, f, valid);
  WaveScan ws;
  write_B(ws, d, geo, f, valid, valid ? a.q_prev[f] : 0.0, valid ? a.q_curr[f] : 0.0);
  // the B rows of this lane were written by this lane: no barrier needed
  const double hv = hess_vec(ws, d, geo, f, valid, valid ? a.q[f] : 0.0, valid ? a.v[f] : 0.0, a.dt2);
  if (valid) a.Hv[f] = hv;
}

// Reverse-mode derivative of a rollout by implicit differentiation.  Step k
// defines q_{k+1} by the stationarity of its objective (Eq. PBAD),
// g(q_{k+1}; q_k, q_{k-1}, tau_k) = 0, so with lambda = dL/dq_{k+1} (complete
// once the later steps are done) and H mu = lambda (H = Hessian at q_{k+1}):
//   dL/dq_k     += adjoint at q_k     of the seed  2 dA(mu) M,
//   dL/dq_{k-1} += adjoint at q_{k-1} of the seed   -dA(mu) M,
//   dL/dtau_k    = dt^2 mu,
// dA(mu) the tangent poses at q_{k+1} along mu.  H mu = lambda is solved by
// conjugate gradients preconditioned with the inverse joint-space inertia at
// q_{k+1} (the same operator as the step's initial inverse Hessian).
struct VjpArgs {
  DevModel d;
  double dt2, tol;
  int max_iter, n_steps, use_aba;
  const double* q_init;  // [2][n]: q_{-1}, q_0
  const double* q_traj;  // [n_steps][n]: q_1 .. q_T
  const double* dL_dq;   // [n_steps][n]: explicit dL/dq_1 .. dL/dq_T
  double* dL_dinit;      // [2][n]
  double* dL_dtau;       // [n_steps][n] or NULL
  abd_step_stats* stats; // [n_steps][n_models] or NULL
};

__global__ void __launch_bounds__(kWave) k_rollout_vjp(VjpArgs args) {
  __shared__ ModelLds L;
  extern __shared__ double hl[];  // packed explicit inverse (inverse_lds_doubles(max frames))
  const DevModel& d = args.d;
  const int n = d.n_dofs, T = args.n_steps;
  const int model = blockIdx.x, lane = threadIdx.x;
  const int f0 = d.f0[model], nf = d.f0[model + 1] - f0;
  if (nf == 0) {
    if (lane == 0 && args.stats)
      for (int k = 0; k < T; ++k) {
        abd_step_stats st = {0, 0, ABD_FLAG_CONVERGED, 0, 0, 0, 0.0, 0.0};
        args.stats[(size_t)k * d.n_models + model] = st;
      }
    return;
  }
  const bool valid = lane < nf;
  const int f = f0 + (valid ? lane : 0);
  const FrameGeo geo = load_geo(d, f, valid);
  const bool use_aba = args.use_aba != 0;
  WaveScan ws;
  // q_j and the explicit dL/dq_j of this lane's DOF, j >= -1
  auto qat = [&](int j) -> double {
    if (!valid) return 0.0;
    return j >= 1 ? args.q_traj[(size_t)(j - 1) * n + f] : args.q_init[(size_t)(j + 1) * n + f];
  };
  auto dl = [&](int j) -> double { return (valid && j >= 1) ? args.dL_dq[(size_t)(j - 1) * n + f] : 0.0; };
  double lam_next = dl(T), lam_cur = dl(T - 1), lam_prev = dl(T - 2);
  for (int k = T - 1; k >= 0; --k) {
    const double q = qat(k + 1), qc = qat(k), qp = qat(k - 1);
    double mu = 0.0, rn = 0.0;
    int it = 0, hv_count = 0, flag = ABD_FLAG_CONVERGED;
    if (nf > 0) {
      step_setup(ws, d, hl + 10 * lane, L.tab[lane], geo, f, valid, qp, qc, q, use_aba);
      if (use_aba) {
        __syncthreads();
        aba_setup_rows(hl, L.tab, nf, lane);
        __syncthreads();
        aba_inverse(L.tab, nf, lane, hl);  // overwrites the inertias
        __syncthreads();  // every lane reads the other lanes' columns
      }
      // ---- preconditioned conjugate gradients on H mu = lambda
      const double b = valid ? lam_next : 0.0;
      const double bn = uniform(sqrt(wave_sum(b * b)));
      double r = b;
      double z = use_aba ? apply_inverse(hl, &L.tab[0][0], nf, lane, r) : r;
      double p = z;
      double rz = uniform(wave_sum(r * z));
      rn = bn;
      if (!isfinite(bn)) {
        flag = ABD_FLAG_NONFINITE;
      } else if (bn > 0.0) {
        flag = ABD_FLAG_MAX_ITER;
        while (it < args.max_iter) {
          const double hp = hess_vec(ws, d, geo, f, valid, q, p, args.dt2);
          ++hv_count;
          const double php = uniform(wave_sum(p * hp));
          if (!(php > 0.0)) {
            flag = ABD_FLAG_LS_FLOOR;  // not positive definite along p
            break;
          }
          const double al = rz / php;
          mu += al * p;
          r -= al * hp;
          ++it;
          rn = uniform(sqrt(wave_sum(r * r)));
          if (rn <= args.tol * bn) {
            flag = ABD_FLAG_CONVERGED;
            break;
          }
          z = use_aba ? apply_inverse(hl, &L.tab[0][0], nf, lane, r) : r;
          const double rz1 = uniform(wave_sum(r * z));
          p = z + (rz1 / rz) * p;
          rz = rz1;
        }
      }
      // ---- propagate to the two past configurations
      double M[10];
      const double* rec = d.fr64 + (size_t)f * 16;
#pragma unroll
      for (int i = 0; i < 10; ++i) M[i] = valid ? rec[6 + i] : 0.0;
      double S[12];
      {
        const Xf<double> A = fk_geo<double>(ws, geo, valid, q);
        double dA[12], W[3], w[3];
        tangent_pose(ws, A, geo.a, valid, mu, dA, W, w);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double s = 0.0;
#pragma unroll
            for (int x = 0; x < 4; ++x) s += dA[4 * r + x] * M[sym4(x, c)];
            S[4 * r + c] = s;
          }
      }
      {
        const Xf<double> Ac = fk_geo<double>(ws, geo, valid, qc);
        double S2[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) S2[i] = 2.0 * S[i];
        lam_cur += adjoint_of_seed(ws, Ac, S2, geo.a, valid);
      }
      {
        const Xf<double> Ap = fk_geo<double>(ws, geo, valid, qp);
#pragma unroll
        for (int i = 0; i < 12; ++i) S[i] = -S[i];
        lam_prev += adjoint_of_seed(ws, Ap, S, geo.a, valid);
      }
    }
    if (args.dL_dtau && valid) args.dL_dtau[(size_t)k * n + f] = args.dt2 * mu;
    if (args.stats && lane == 0) {
      abd_step_stats st;
      st.iterations = it;
      st.evaluations = hv_count;
      st.flag = flag;
      st.f32_iterations = 0;
      st.f32_evaluations = 0;
      st.reserved = 0;
      st.grad_norm = rn;
      st.energy = 0.0;
      args.stats[(size_t)k * d.n_models + model] = st;
    }
    lam_next = lam_cur;
    lam_cur = lam_prev;
    lam_prev = dl(k - 2);
  }
  if (valid) {
    args.dL_dinit[f] = lam_cur;        // q_{-1}
    args.dL_dinit[(size_t)n + f] = lam_next;  // q_0
  }
}

}  // namespace

namespace abd_impl {

int launch_hvp(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist, const double* v,
               double* Hv, void* stream) {
  HvpArgs a;
  a.d = dev_view(m);
  a.dt2 = o->dt * o->dt;
  a.q = q;
  a.q_prev = q_hist;
  a.q_curr = q_hist + m->n_dofs;
  a.v = v;
  a.Hv = Hv;
  hipLaunchKernelGGL(k_hvp, dim3(m->n_models), dim3(kWave), 0, static_cast<hipStream_t>(stream), a);
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

int launch_rollout_vjp(abd_model* m, const abd_step_opts* o, const double* q_init, const double* q_traj,
                       const double* dL_dq_traj, double* dL_dq_init, double* dL_dtau, abd_step_stats* stats,
                       int n_steps, void* stream) {
  VjpArgs a;
  a.d = dev_view(m);
  a.dt2 = o->dt * o->dt;
  a.tol = o->tol;
  a.max_iter = o->max_iter;
  a.n_steps = n_steps;
  a.use_aba = o->precond == ABD_PRECOND_INERTIA;
  a.q_init = q_init;
  a.q_traj = q_traj;
  a.dL_dq = dL_dq_traj;
  a.dL_dinit = dL_dq_init;
  a.dL_dtau = dL_dtau;
  a.stats = stats;
  hipLaunchKernelGGL(k_rollout_vjp, dim3(m->n_models), dim3(kWave),
                     (size_t)inverse_lds_doubles(m->max_frames) * sizeof(double), static_cast<hipStream_t>(stream), a);
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

}  // namespace abd_impl
