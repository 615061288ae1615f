// hoc_common.h -- what the order-K collocation solvers share (Sec. 4 Eq. HOC /
// Eq. EQHOC): the step arguments, the collocation points and weights, and the
// host-side filling of the arguments.
#pragma once
#include "abd_device.h"

#include <cmath>

namespace {

// ------------------------------------------ high-order collocation (K>2) --
// Sec. 4, Eq. HOC / Eq. EQHOC for one-wave models.  The K-1 unknown
// configurations q_u of a step sit in registers of the lane that owns the frame
// (U = K-1 values per lane).  With the known seed part
// Bk_u = w_u0 A(q_prev) + w_u1 A(q_k) (per step) and the poses A_a = A(q_a):
//   seed      G_u = (Bk_u + sum_a w_u,2+a A_a) M - dt^2 g (M e4)^T
//   residual  rho_u = adjoint of G_u at q_u (- dt^2 tau)          [= dt^2 r_u]
//   objective E = sum_u |rho_u|^2
//   gradient  dE/dq_a = 2 (T_a + C_a), where, with dA_u the tangent poses at
//             q_u along rho_u,
//             T_a = derivative of the adjoint of the FIXED seed G_a at q_a along
//                   rho_a (the second derivatives of the poses, S(q_a; G_a) rho_a),
//             C_a = adjoint at q_a of the seed sum_u w_u,2+a dA_u M
//                   (the mixed second derivatives, C(q_u, q_a)^T rho_u).
template <int U>
struct HocArgs {
  DevModel d;
  double dt2, tol;
  int m, max_iter, max_ls, precond, n_steps;
  double w[U][U + 2];   // dt^2 Pddot(tau_{2+u}) = sum_p w[u][p] P_p over the K+1 points
  double vscale;        // 1 / (tau_1 - tau_0): warm-start velocity from the known points
  double tau_u[U];      // the unknown points (units of dt from t_k)
  double minv[U][U];    // (W_uu^T W_uu)^-1, W_uu = weights among the unknown points
  const double* q_prev; // q_{-1+alpha_{K-2}}
  const double* q_curr; // q_0
  const double* tau;    // [n_steps][n_dofs] or NULL
  double* q_out;        // [n_steps][U][n_dofs]
  abd_step_stats* stats;
  double* Bk;           // scratch [n_dofs][U][12]
  double* hist3;        // models of more than 64 DOFs: L-BFGS pairs [n_dofs][2][kMaxHist][3]
};

}  // namespace

namespace abd_impl {

// Points tau[K+1] of a step (units of dt from t_k) and second-derivative
// weights w[(K-1)(K+1)] at the K-1 unknown points, K = 3, 4.
void hoc_collocation(int K, double* tau, double* w);

template <int U>
int fill_hoc_args(abd_model* m, const abd_step_opts* o, HocArgs<U>& a, const StepScratch* sc = nullptr) {
  const int K = U + 1, np = K + 1;
  double tau[5], w[3 * 5];
  hoc_collocation(K, tau, w);
  a.d = dev_view(m);
  if (sc) {
    a.d.B64 = sc->B64;
    a.d.B32 = sc->B32;
    a.d.hist = sc->hist;
    a.d.hinv = sc->hinv;
  }
  a.dt2 = o->dt * o->dt;
  a.tol = o->tol;
  a.m = o->lbfgs_m;
  a.max_iter = o->max_iter;
  a.max_ls = o->max_ls;
  a.precond = o->precond;
  for (int u = 0; u < U; ++u) {
    for (int p = 0; p < np; ++p) a.w[u][p] = w[u * np + p];
    a.tau_u[u] = tau[2 + u];
  }
  a.vscale = 1.0 / (tau[1] - tau[0]);
  // (W_uu^T W_uu)^-1 by Gauss-Jordan
  double g[U][2 * U];
  for (int r = 0; r < U; ++r)
    for (int c = 0; c < U; ++c) {
      double t = 0.0;
      for (int k = 0; k < U; ++k) t += w[k * np + 2 + r] * w[k * np + 2 + c];
      g[r][c] = t;
      g[r][U + c] = r == c ? 1.0 : 0.0;
    }
  for (int c = 0; c < U; ++c) {
    int piv = c;
    for (int r = c + 1; r < U; ++r)
      if (std::fabs(g[r][c]) > std::fabs(g[piv][c])) piv = r;
    for (int k = 0; k < 2 * U; ++k) std::swap(g[c][k], g[piv][k]);
    const double d = g[c][c];
    for (int k = 0; k < 2 * U; ++k) g[c][k] /= d;
    for (int r = 0; r < U; ++r) {
      if (r == c) continue;
      const double fct = g[r][c];
      for (int k = 0; k < 2 * U; ++k) g[r][k] -= fct * g[c][k];
    }
  }
  for (int r = 0; r < U; ++r)
    for (int c = 0; c < U; ++c) a.minv[r][c] = g[r][U + c];
  if (sc) {  // caller-placed scratch: nothing is allocated
    a.Bk = sc->Bk;
    a.hist3 = sc->hist3;
    return ABD_OK;
  }
  if (!m->Bk) {
    int rc = model_alloc(m, reinterpret_cast<void**>(&m->Bk), 36 * (size_t)m->n_dofs * sizeof(double));
    if (rc) return rc;
  }
  if (!m->hist3 && m->max_frames > kMaxFrames) {
    int rc = model_alloc(m, reinterpret_cast<void**>(&m->hist3), 2 * kMaxHist * 3 * (size_t)m->n_dofs * sizeof(double));
    if (rc) return rc;
  }
  a.Bk = m->Bk;
  a.hist3 = m->hist3;
  return ABD_OK;
}

}  // namespace abd_impl
