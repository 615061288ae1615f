// eval.hip -- objective/gradient (Eq. EQ, Alg. 1) and pose kernels and their launches.
#include "abd_device.h"

namespace {

// ---------------------------------------------------- objective / poses --
struct EvalArgs {
  DevModel d;
  double dt2;
  int precision;
  const double* q;
  const double* q_prev;
  const double* q_curr;
  const double* tau;
  double* E;
  double* grad;
  double* grad_tau;
};

template <int NW, bool TREE, bool FX = false>
__global__ void __launch_bounds__(NW* kWave) k_objective_grad(EvalArgs a) {
  __shared__ ScanLds<NW, TREE> L;
  const DevModel& d = a.d;
  const int model = blockIdx.x, j = threadIdx.x;
  const int f0 = d.f0[model], nf = d.f0[model + 1] - f0;
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);
  if (nf == 0) {
    if (j == 0) a.E[model] = 0.0;
    return;
  }
  typename ModelScan<NW, TREE>::type sc = ModelScan<NW, TREE>::make(L, d, j / kWave, j % kWave, j, f, valid);
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;
  const double qkm1 = valid ? a.q_prev[io] : 0.0, qk = valid ? a.q_curr[io] : 0.0;
  const FrameGeo geo = load_geo<FX>(d, f, valid);
  write_B<FX>(sc, d, geo, f, valid, qkm1, qk);
  // the B (and A(q_k)) rows of this thread were written by this thread: no barrier needed
  const double q = valid ? a.q[io] : 0.0;
  const double tau = (valid && a.tau) ? a.tau[io] : 0.0;
  const EvalResult r = a.precision == ABD_MIXED ? evaluate<float, FX>(sc, d, geo, f, valid, q, tau, a.dt2)
                                                : evaluate<double, FX>(sc, d, geo, f, valid, q, tau, a.dt2);
  if (j == 0) a.E[model] = r.E;
  if (a.grad && valid) a.grad[io] = r.g;
  // E contains -dt^2 tau.q
  if (a.grad_tau && valid) a.grad_tau[io] = -a.dt2 * q;
}

template <int NW, bool TREE, bool FX = false>
__global__ void __launch_bounds__(NW* kWave) k_poses(DevModel d, const double* q, double* poses) {
  __shared__ ScanLds<NW, TREE> L;
  const int model = blockIdx.x, j = threadIdx.x;
  const int f0 = d.f0[model], nf = d.f0[model + 1] - f0;
  if (nf == 0) return;
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);
  typename ModelScan<NW, TREE>::type sc = ModelScan<NW, TREE>::make(L, d, j / kWave, j % kWave, j, f, valid);
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;
  const Xf<double> A = fk_geo<double, FX>(sc, load_geo<FX>(d, f, valid), valid, valid ? q[io] : 0.0);
  if (valid) {
    const int l = d.pose_link[f];
    if (l >= 0)
#pragma unroll
      for (int k = 0; k < 12; ++k) poses[12 * (size_t)l + k] = A.m[k];
  }
}

}  // namespace

namespace abd_impl {

int launch_objective(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist,
                     const double* tau, double* E, double* grad, double* grad_tau, void* stream) {
  EvalArgs a;
  a.d = dev_view(m);
  a.dt2 = o->dt * o->dt;
  a.precision = o->precision;
  a.q = q;
  a.q_prev = q_hist;
  a.q_curr = q_hist + m->n_dofs;
  a.tau = tau;
  a.E = E;
  a.grad = grad;
  a.grad_tau = grad_tau;
  const int nw = waves_for(m->max_frames);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(m->n_models), block(nw * kWave);
  if (m->fx) {  // at most 256 frames per model
    if (m->tree) {
      if (nw == 1) hipLaunchKernelGGL((k_objective_grad<1, true, true>), grid, block, 0, s, a);
      else if (nw == 2) hipLaunchKernelGGL((k_objective_grad<2, true, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_objective_grad<4, true, true>), grid, block, 0, s, a);
    } else {
      if (nw == 1) hipLaunchKernelGGL((k_objective_grad<1, false, true>), grid, block, 0, s, a);
      else if (nw == 2) hipLaunchKernelGGL((k_objective_grad<2, false, true>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_objective_grad<4, false, true>), grid, block, 0, s, a);
    }
  } else if (m->tree) {
    switch (nw) {
      case 1: hipLaunchKernelGGL((k_objective_grad<1, true>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_objective_grad<2, true>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((k_objective_grad<4, true>), grid, block, 0, s, a); break;
    }
  } else {
    switch (nw) {
      case 1: hipLaunchKernelGGL((k_objective_grad<1, false>), grid, block, 0, s, a); break;
      case 2: hipLaunchKernelGGL((k_objective_grad<2, false>), grid, block, 0, s, a); break;
      case 4: hipLaunchKernelGGL((k_objective_grad<4, false>), grid, block, 0, s, a); break;
      case 8: hipLaunchKernelGGL((k_objective_grad<8, false>), grid, block, 0, s, a); break;
      default: hipLaunchKernelGGL((k_objective_grad<16, false>), grid, block, 0, s, a); break;
    }
  }
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

int launch_poses(abd_model* m, const double* q, double* poses, void* stream) {
  const int nw = waves_for(m->max_frames);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid(m->n_models), block(nw * kWave);
  const DevModel d = dev_view(m);
  if (m->fx) {  // at most 256 frames per model
    if (m->tree) {
      if (nw == 1) hipLaunchKernelGGL((k_poses<1, true, true>), grid, block, 0, s, d, q, poses);
      else if (nw == 2) hipLaunchKernelGGL((k_poses<2, true, true>), grid, block, 0, s, d, q, poses);
      else hipLaunchKernelGGL((k_poses<4, true, true>), grid, block, 0, s, d, q, poses);
    } else {
      if (nw == 1) hipLaunchKernelGGL((k_poses<1, false, true>), grid, block, 0, s, d, q, poses);
      else if (nw == 2) hipLaunchKernelGGL((k_poses<2, false, true>), grid, block, 0, s, d, q, poses);
      else hipLaunchKernelGGL((k_poses<4, false, true>), grid, block, 0, s, d, q, poses);
    }
  } else if (m->tree) {
    switch (nw) {
      case 1: hipLaunchKernelGGL((k_poses<1, true>), grid, block, 0, s, d, q, poses); break;
      case 2: hipLaunchKernelGGL((k_poses<2, true>), grid, block, 0, s, d, q, poses); break;
      default: hipLaunchKernelGGL((k_poses<4, true>), grid, block, 0, s, d, q, poses); break;
    }
  } else {
    switch (nw) {
      case 1: hipLaunchKernelGGL((k_poses<1, false>), grid, block, 0, s, d, q, poses); break;
      case 2: hipLaunchKernelGGL((k_poses<2, false>), grid, block, 0, s, d, q, poses); break;
      case 4: hipLaunchKernelGGL((k_poses<4, false>), grid, block, 0, s, d, q, poses); break;
      case 8: hipLaunchKernelGGL((k_poses<8, false>), grid, block, 0, s, d, q, poses); break;
      default: hipLaunchKernelGGL((k_poses<16, false>), grid, block, 0, s, d, q, poses); break;
    }
  }
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

}  // namespace abd_impl
