// lm.hip -- Levenberg-Marquardt solver of the order-K collocation step (Sec. 5
// "Optimization Algorithm" with the sum-of-squares objective Eq. EQHOC):
// kernel and launch.
//
// Per iteration of a step the workgroup of a model
//   1. evaluates the residuals r = (dt^2 r_u) at the K-1 unknown configurations
//      (Alg. 1 forward pass per configuration, seeded adjoint pass per unknown);
//   2. after an accepted step, assembles the Jacobian J = dr/dq* explicitly
//      (N = (K-1) n, dense N x N in the model's device scratch):
//        J_ua = delta_ua S(q_u; G_u) + w_ua C(q_u, q_a),
//      both from sums over the frames below the deeper of the two frames of an
//      entry ("composite" tensors, as in the composite-rigid-body algorithm), so
//      the entries cost O(1) each after O(n) scans;
//   3. forms A = J^T J (tiled in LDS) and factors A + lambda I = U^T U
//      (blocked Cholesky, row blocks of 32);
//   4. solves for the step v = -(A + lambda I)^-1 J^T r, adds half the geodesic
//      acceleration a = -(A + lambda I)^-1 J^T r_vv (r_vv from one more residual
//      evaluation at q + h v), and accepts the step if it decreases E = |r|^2,
//      with Nielsen's lambda update.
// The composite forms.  For frames b above or equal to c (c the deeper) and
// configurations q_u, q_a, with world axes w, joint points p:
//   dA_l(q)/dq_b = [w_b]x (A_l - p_b e4^T)  for every link l below b,
//   d2A_l/dq_b dq_c = [w_b]x [w_c]x (A_l - p_c e4^T),
// so, summing over the links l below c,
//   C(q_u, q_a)_bc = (w_b . w'_c) tr X - w'_c^T X w_b,
//       X = N_c - h_c p'_c^T - p_b h'_c^T + m_c p_b p'_c^T,
//       N_c = sum_l A_l(q_u) M_l A_l(q_a)^T, h_c = sum_l A_l(q_u) M_l e4,
//       h'_c the same at q_a, m_c = sum_l mass_l   (primes: at q_a);
//   S(q_u; G_u)_bc = w_b^T Y_c w_c - (w_b . w_c) tr Y_c,
//       Y_c = sum_l A_l G_l^T - p_c (sum_l G_l e4)^T   (all at q_u).
// (When the deeper frame is the residual's frame b the roles swap.)

#include "hoc_common.h"

namespace {

constexpr double kLmLambda0 = 1e-3;     // initial lambda relative to max diag(J^T J)
constexpr double kLmLambdaMin = 1e-15;  // lambda floor relative to max diag(J^T J)
constexpr double kLmGeoH = 0.1;         // finite-difference step of the geodesic acceleration
constexpr double kLmGeoAlpha = 0.75;    // steps with 2 |a| > alpha |v| are rejected
constexpr int kTM = 32, kTN = 64, kTK = 16;  // GEMM tile (rows x columns x depth)

template <int U>
struct LmArgs {
  HocArgs<U> h;
  double* mat;            // per model: J, A = J^T J (upper), U factor (upper, mirrored below)
  const long long* moff;  // [n_models+1] start of every model's block (doubles)
  int nfmax;              // frames of the batch's largest model
};

// Residuals of the unknown points at q (per lane: rho[u] of this frame) and the
// objective E (wave-uniform).  Same arithmetic as the evaluation of the L-BFGS
// path (hoc_evaluate), without the gradient.
template <int U, typename Sc>
__device__ double lm_residual(Sc& sc, const HocArgs<U>& args, const FrameGeo& geo, int f, bool valid,
                              const double q[U], double tau, double rho[U]) {
  const DevModel& d = args.d;
  asm volatile("" ::: "memory");
  double M[10];
  const double* rec = d.fr64 + (size_t)f * 16;
#pragma unroll
  for (int k = 0; k < 10; ++k) M[k] = ld_if(rec + 6 + k, valid);
  const double* Bk = args.Bk + (size_t)f * (12 * U);
  const double gv[3] = {d.gx, d.gy, d.gz};
  Xf<double> A[U];
#pragma unroll
  for (int u = 0; u < U; ++u) A[u] = fk_geo<double>(sc, geo, valid, q[u]);
  double E = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    double G[12];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          double bx = ld_if(Bk + 12 * u + 4 * r + x, valid);
#pragma unroll
          for (int a = 0; a < U; ++a) bx += args.w[u][2 + a] * A[a].m[4 * r + x];
          s += bx * M[sym4(x, c)];
        }
        G[4 * r + c] = s - args.dt2 * gv[r] * M[sym4(c, 3)];
      }
    const double res = adjoint_of_seed(sc, A[u], G, geo.a, valid);
    rho[u] = valid ? res - args.dt2 * tau : 0.0;
    E += rho[u] * rho[u];
  }
  return sc.sum(E);
}

// Explicit Jacobian of the residuals at q into J (row (u, b), column (a, c),
// row-major, leading dimension N = U nf; J must be zero where no entry is
// written: entries of frames that are not above one another).  wp: LDS table
// [U][nfmax][6] of the world axes and joint points of every frame.  oidx (may
// be null: the frame order) gives the row/column position of every frame of
// the model.  With U = 1, weights (1, -2, 1) and Bk = A(q_{k-1}) - 2 A(q_k), the
// residual is the gradient of Eq. EQ and J its Hessian.
template <int U, typename Sc, bool WITH_S = true>
__device__ void lm_jacobian(Sc& sc, const HocArgs<U>& args, const FrameGeo& geo, int f, bool valid, int j,
                            int nf, int nfmax, const double q[U], double* J, double* wp,
                            const int* oidx = nullptr) {
  const DevModel& d = args.d;
  const int N = U * nf;
  asm volatile("" ::: "memory");
  double M[10];
  const double* rec = d.fr64 + (size_t)f * 16;
#pragma unroll
  for (int k = 0; k < 10; ++k) M[k] = ld_if(rec + 6 + k, valid);
  const double* Bk = args.Bk + (size_t)f * (12 * U);
  const double gv[3] = {d.gx, d.gy, d.gz};
  Xf<double> A[U];
#pragma unroll
  for (int u = 0; u < U; ++u) A[u] = fk_geo<double>(sc, geo, valid, q[u]);
  // world axis and joint point of this frame at every unknown point
  double w[U][3], p[U][3];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      w[u][i] = A[u].m[4 * i] * geo.a[0] + A[u].m[4 * i + 1] * geo.a[1] + A[u].m[4 * i + 2] * geo.a[2];
      p[u][i] = A[u].m[4 * i + 3];
    }
  if (valid)
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        wp[((size_t)u * nfmax + j) * 6 + i] = w[u][i];
        wp[((size_t)u * nfmax + j) * 6 + 3 + i] = p[u][i];
      }
  // AM_u = A_u M (3x4): its last column is h_u, and N(u,a) = AM_u A_a^T
  double AM[U][12];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x) s += A[u].m[4 * r + x] * M[sym4(x, c)];
        AM[u][4 * r + c] = s;
      }
  // composite h_u (every unknown point) and mass below this frame
  double hs[U][3], ms;
  {
    double v[6], t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      v[i] = valid ? AM[0][4 * i + 3] : 0.0;
      v[3 + i] = (valid && U > 1) ? AM[U > 1 ? 1 : 0][4 * i + 3] : 0.0;
    }
    sc.suffix6_total2(v, t0, t1);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      hs[0][i] = v[i];
      if (U > 1) hs[U > 1 ? 1 : 0][i] = v[3 + i];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = (valid && U > 2) ? AM[U > 2 ? 2 : 1][4 * i + 3] : 0.0;
    v[3] = valid ? M[9] : 0.0;
    v[4] = 0.0;
    v[5] = 0.0;
    sc.suffix6_total2(v, t0, t1);
    if (U > 2)
#pragma unroll
      for (int i = 0; i < 3; ++i) hs[U > 2 ? 2 : 1][i] = v[i];
    ms = v[3];
  }
  // ancestors of this frame (this frame first), walked for every pair of points
  const int* fpar = d.fpar + (f - j);  // parent frames of the model (local indices)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // seed G_u and the composite Y_u, F_u below this frame (for the S block)
    double Y[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Fv[3];
    if (WITH_S) {
      double G[12];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double s = 0.0;
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            double bx = ld_if(Bk + 12 * u + 4 * r + x, valid);
#pragma unroll
            for (int a = 0; a < U; ++a) bx += args.w[u][2 + a] * A[a].m[4 * r + x];
            s += bx * M[sym4(x, c)];
          }
          G[4 * r + c] = s - args.dt2 * gv[r] * M[sym4(c, 3)];
        }
      double v[6], t0 = 0.0, t1 = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          double acc = 0.0;
#pragma unroll
          for (int x = 0; x < 4; ++x) acc += A[u].m[4 * r + x] * G[4 * s2 + x];
          v[2 * r + s2] = valid ? acc : 0.0;
        }
      sc.suffix6_total2(v, t0, t1);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Y[3 * r + 0] = v[2 * r + 0];
        Y[3 * r + 1] = v[2 * r + 1];
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x) acc += A[u].m[4 * r + x] * G[8 + x];
        v[r] = valid ? acc : 0.0;
        v[3 + r] = valid ? G[4 * r + 3] : 0.0;
      }
      sc.suffix6_total2(v, t0, t1);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Y[3 * r + 2] = v[r];
        Fv[r] = v[3 + r];
      }
      // Y <- Y - p_c F^T at this (deeper) frame
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) Y[3 * r + c] -= p[u][r] * Fv[c];
    }
    const double trY = Y[0] + Y[4] + Y[8];
    double Yw[3];  // Y w_b (this frame at q_u)
#pragma unroll
    for (int r = 0; r < 3; ++r) Yw[r] = Y[3 * r] * w[u][0] + Y[3 * r + 1] * w[u][1] + Y[3 * r + 2] * w[u][2];
#pragma unroll
    for (int a = 0; a < U; ++a) {
      // composite N(u, a) below this frame
      double Nc[9];
      {
        double v[6], t0 = 0.0, t1 = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int s2 = 0; s2 < 2; ++s2) {
            double acc = 0.0;
#pragma unroll
            for (int x = 0; x < 4; ++x) acc += AM[u][4 * r + x] * A[a].m[4 * s2 + x];
            v[2 * r + s2] = valid ? acc : 0.0;
          }
        sc.suffix6_total2(v, t0, t1);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          Nc[3 * r + 0] = v[2 * r + 0];
          Nc[3 * r + 1] = v[2 * r + 1];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          double acc = 0.0;
#pragma unroll
          for (int x = 0; x < 4; ++x) acc += AM[u][4 * r + x] * A[a].m[8 + x];
          v[r] = valid ? acc : 0.0;
          v[3 + r] = 0.0;
        }
        sc.suffix6_total2(v, t0, t1);
#pragma unroll
        for (int r = 0; r < 3; ++r) Nc[3 * r + 2] = v[r];
      }
      sc.sync();  // every frame has written its axes and points
      if (!valid) continue;
      const double wuu = args.w[u][2 + a];
      const double tN = Nc[0] + Nc[4] + Nc[8];
      const double* hu = hs[u];
      const double* ha = hs[a];
      // this frame b as the residual's frame (row entries: DOF frame x at q_a)
      const double* wb = w[u];
      const double* pb = p[u];
      double Nw[3];  // N w_b
#pragma unroll
      for (int r = 0; r < 3; ++r) Nw[r] = Nc[3 * r] * wb[0] + Nc[3 * r + 1] * wb[1] + Nc[3 * r + 2] * wb[2];
      const double pb_ha = pb[0] * ha[0] + pb[1] * ha[1] + pb[2] * ha[2];
      const double ha_wb = ha[0] * wb[0] + ha[1] * wb[1] + ha[2] * wb[2];
      // this frame b as the DOF frame (column entries: residual frame x at q_u)
      const double* wba = w[a];
      const double* pba = p[a];
      double Ntw[3];  // N^T w_b(q_a)
#pragma unroll
      for (int c = 0; c < 3; ++c) Ntw[c] = Nc[c] * wba[0] + Nc[3 + c] * wba[1] + Nc[6 + c] * wba[2];
      const double wba_hu = wba[0] * hu[0] + wba[1] * hu[1] + wba[2] * hu[2];
      const double hu_pba = hu[0] * pba[0] + hu[1] * pba[1] + hu[2] * pba[2];
      const int ob = oidx ? oidx[j] : j;                                  // position of this frame
      double* row = J + ((size_t)u * nf + ob) * N + (size_t)a * nf;      // J[(u, b)][(a, .)]
      double* col = J + (size_t)a * nf + ob;                              // J[(u, .)][(a, b)]
      for (int x = j; x >= 0; x = fpar[x]) {
        const int ox = oidx ? oidx[x] : x;
        // row entry J[(u,b),(a,x)]: X = N - h_u p'^T - p_b h_a^T + m p_b p'^T
        const double* wx = wp + ((size_t)a * nfmax + x) * 6;
        const double wq[3] = {wx[0], wx[1], wx[2]}, pq[3] = {wx[3], wx[4], wx[5]};
        const double hu_pq = hu[0] * pq[0] + hu[1] * pq[1] + hu[2] * pq[2];
        const double pb_pq = pb[0] * pq[0] + pb[1] * pq[1] + pb[2] * pq[2];
        const double trX = tN - hu_pq - pb_ha + ms * pb_pq;
        const double wq_wb = wq[0] * wb[0] + wq[1] * wb[1] + wq[2] * wb[2];
        const double wq_Nw = wq[0] * Nw[0] + wq[1] * Nw[1] + wq[2] * Nw[2];
        const double wq_hu = wq[0] * hu[0] + wq[1] * hu[1] + wq[2] * hu[2];
        const double pq_wb = pq[0] * wb[0] + pq[1] * wb[1] + pq[2] * wb[2];
        const double wq_pb = wq[0] * pb[0] + wq[1] * pb[1] + wq[2] * pb[2];
        const double wXw = wq_Nw - wq_hu * pq_wb - wq_pb * ha_wb + ms * wq_pb * pq_wb;
        double e = wuu * (wq_wb * trX - wXw);
        // S block (u == a): frame x above b, both at q_u
        const double* wu = wp + ((size_t)u * nfmax + x) * 6;
        double sv = 0.0;
        if (WITH_S && u == a) {
          const double wxu[3] = {wu[0], wu[1], wu[2]};
          sv = (wxu[0] * Yw[0] + wxu[1] * Yw[1] + wxu[2] * Yw[2]) -
               (wxu[0] * wb[0] + wxu[1] * wb[1] + wxu[2] * wb[2]) * trY;
          e += sv;
        }
        row[ox] = e;
        if (x != j) {
          // column entry J[(u,x),(a,b)]: X' = N - h_u p_b(a)^T - p_x(u) h_a^T + m p_x(u) p_b(a)^T
          const double wxu[3] = {wu[0], wu[1], wu[2]}, pxu[3] = {wu[3], wu[4], wu[5]};
          const double px_ha = pxu[0] * ha[0] + pxu[1] * ha[1] + pxu[2] * ha[2];
          const double px_pba = pxu[0] * pba[0] + pxu[1] * pba[1] + pxu[2] * pba[2];
          const double trXc = tN - hu_pba - px_ha + ms * px_pba;
          const double wx_wba = wxu[0] * wba[0] + wxu[1] * wba[1] + wxu[2] * wba[2];
          const double Ntw_wx = Ntw[0] * wxu[0] + Ntw[1] * wxu[1] + Ntw[2] * wxu[2];
          const double pba_wx = pba[0] * wxu[0] + pba[1] * wxu[1] + pba[2] * wxu[2];
          const double wba_px = wba[0] * pxu[0] + wba[1] * pxu[1] + wba[2] * pxu[2];
          const double ha_wx = ha[0] * wxu[0] + ha[1] * wxu[1] + ha[2] * wxu[2];
          const double wXwc = Ntw_wx - wba_hu * pba_wx - wba_px * ha_wx + ms * wba_px * pba_wx;
          col[((size_t)u * nf + ox) * N] = wuu * (wx_wba * trXc - wXwc) + sv;
        }
      }
    }
  }
}


// ------------------------------------------------------------ dense algebra --
// One tile of C = X^T X restricted to rows [i0, i0 + kTM) and columns
// [j0, j0 + kTN), summed over k in [k0, k1): acc[r] = sum_k X[k][i] X[k][jc] for
// this thread's rows i = i0 + (tid / kTN) * RT + r and column jc = j0 + tid % kTN.
// X is row-major with leading dimension ld; indices at or beyond n read as 0.
// xs: LDS [kTK][kTM], ys: LDS [kTK][kTN].  Every thread of the workgroup calls it.
template <int NW>
__device__ void gemm_tn_tile(const double* X, int ld, int n, int k0, int k1, int i0, int j0, double* xs,
                             double* ys, double* acc) {
  constexpr int T = NW * kWave, RT = kTM / NW;
  const int tid = threadIdx.x, tj = tid % kTN, ti = tid / kTN;
#pragma unroll
  for (int r = 0; r < RT; ++r) acc[r] = 0.0;
  for (int kk = k0; kk < k1; kk += kTK) {
    for (int e = tid; e < kTK * kTM; e += T) {
      const int k = kk + e / kTM, i = i0 + e % kTM;
      xs[e] = (k < k1 && i < n) ? X[(size_t)k * ld + i] : 0.0;
    }
    for (int e = tid; e < kTK * kTN; e += T) {
      const int k = kk + e / kTN, jc = j0 + e % kTN;
      ys[e] = (k < k1 && jc < n) ? X[(size_t)k * ld + jc] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kTK; ++k) {
      const double y = ys[k * kTN + tj];
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[r] += xs[k * kTM + ti * RT + r] * y;
    }
    __syncthreads();
  }
}

// A = J^T J (upper triangle and the diagonal tiles), N x N row-major.
template <int NW>
__device__ void form_normal(const double* J, double* A, int N, double* xs, double* ys) {
  constexpr int RT = kTM / NW;
  const int tj = threadIdx.x % kTN, ti = threadIdx.x / kTN;
  double acc[RT];
  for (int i0 = 0; i0 < N; i0 += kTM)
    for (int j0 = (i0 / kTN) * kTN; j0 < N; j0 += kTN) {
      gemm_tn_tile<NW>(J, N, N, 0, N, i0, j0, xs, ys, acc);
      const int jc = j0 + tj;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const int i = i0 + ti * RT + r;
        if (i < N && jc < N && jc >= i) A[(size_t)i * N + jc] = acc[r];
      }
    }
  __threadfence_block();
  __syncthreads();
}

// Cholesky factor of B = A + lam I (A: upper triangle, N x N row-major):
// B = U^T U with U upper, written to Uf (upper triangle, then mirrored into the
// lower triangle so that both U's rows and columns are contiguous rows of Uf).
// Left-looking by blocks of kTM rows; the diagonal block is factored in LDS (D).
// Returns false (uniform) if a pivot is not positive.
template <int NW>
__device__ bool factor(const double* A, double* Uf, int N, double lam, double* xs, double* ys, double* D,
                       int* bad) {
  constexpr int T = NW * kWave, RT = kTM / NW;
  const int tid = threadIdx.x, tj = tid % kTN, ti = tid / kTN;
  for (int e = tid; e < N * N; e += T) {
    const int i = e / N, jc = e % N;
    if (jc >= i) Uf[e] = A[e] + (jc == i ? lam : 0.0);
  }
  if (tid == 0) *bad = 0;
  __threadfence_block();
  __syncthreads();
  double acc[RT];
  for (int r0 = 0; r0 < N; r0 += kTM) {
    const int rn = N - r0 < kTM ? N - r0 : kTM;
    // 1. the block's rows minus the contribution of the rows above
    if (r0 > 0) {
      for (int j0 = r0; j0 < N; j0 += kTN) {
        gemm_tn_tile<NW>(Uf, N, N, 0, r0, r0, j0, xs, ys, acc);
        const int jc = j0 + tj;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const int i = r0 + ti * RT + r;
          if (i < N && jc < N && jc >= i) Uf[(size_t)i * N + jc] -= acc[r];
        }
      }
      __threadfence_block();
      __syncthreads();
    }
    // 2. the diagonal block, unblocked, in LDS
    for (int e = tid; e < kTM * kTM; e += T) {
      const int x = e / kTM, y = e % kTM;
      D[e] = (x < rn && y < rn && y >= x) ? Uf[(size_t)(r0 + x) * N + r0 + y] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < rn; ++c) {
      const double piv = D[c * kTM + c];
      const double dc = piv > 0.0 ? sqrt(piv) : 1.0;
      __syncthreads();
      if (tid == 0) {
        if (!(piv > 0.0)) *bad = 1;
        D[c * kTM + c] = dc;
      }
      for (int y = c + 1 + tid; y < rn; y += T) D[c * kTM + y] /= dc;
      __syncthreads();
      for (int e = tid; e < kTM * kTM; e += T) {
        const int x = e / kTM, y = e % kTM;
        if (x > c && x < rn && y >= x && y < rn) D[e] -= D[c * kTM + x] * D[c * kTM + y];
      }
      __syncthreads();
    }
    for (int e = tid; e < kTM * kTM; e += T) {
      const int x = e / kTM, y = e % kTM;
      if (x < rn && y < rn && y >= x) Uf[(size_t)(r0 + x) * N + r0 + y] = D[e];
    }
    // 3. the block's rows right of the diagonal block: solve D^T Z = W per column
    for (int jc = r0 + rn + tid; jc < N; jc += T) {
      double z[kTM];
#pragma unroll
      for (int c = 0; c < kTM; ++c) z[c] = c < rn ? Uf[(size_t)(r0 + c) * N + jc] : 0.0;
#pragma unroll
      for (int c = 0; c < kTM; ++c) {
        if (c < rn) {
          double t = z[c];
#pragma unroll
          for (int k = 0; k < c; ++k) t -= D[k * kTM + c] * z[k];
          z[c] = t / D[c * kTM + c];
        }
      }
#pragma unroll
      for (int c = 0; c < kTM; ++c)
        if (c < rn) Uf[(size_t)(r0 + c) * N + jc] = z[c];
    }
    __threadfence_block();
    __syncthreads();
  }
  // mirror the upper triangle into the lower one
  for (int e = tid; e < N * N; e += T) {
    const int i = e / N, jc = e % N;
    if (jc < i) Uf[e] = Uf[(size_t)jc * N + i];
  }
  __threadfence_block();
  __syncthreads();
  return *bad == 0;
}

// x <- (U^T U)^-1 x for the factor of factor(); x: LDS vector of N.
template <int NW>
__device__ void chol_solve_lds(const double* Uf, int N, double* x) {
  constexpr int T = NW * kWave;
  const int tid = threadIdx.x;
  // U^T y = b: column j of U^T is row j of U (right of the diagonal)
  for (int jr = 0; jr < N; ++jr) {
    const double yj = x[jr] / Uf[(size_t)jr * N + jr];
    __syncthreads();
    for (int i = jr + 1 + tid; i < N; i += T) x[i] -= Uf[(size_t)jr * N + i] * yj;
    if (tid == 0) x[jr] = yj;
    __syncthreads();
  }
  // U x = y: column j of U above the diagonal is the mirrored row j
  for (int jr = N - 1; jr >= 0; --jr) {
    const double xj = x[jr] / Uf[(size_t)jr * N + jr];
    __syncthreads();
    for (int i = tid; i < jr; i += T) x[i] -= Uf[(size_t)jr * N + i] * xj;
    if (tid == 0) x[jr] = xj;
    __syncthreads();
  }
}

// chol_solve_lds for a workgroup of one wave and N <= 64 NS: the vector in
// registers (lane i holds entries i, i + 64, ...), each row of the factor read
// as one coalesced run while the previous row is used, and no barrier; the
// same arithmetic per entry as chol_solve_lds (bitwise the same result).
template <int NS>
__device__ void chol_solve_wave(const double* Uf, int N, double* x) {
  const int lane = threadIdx.x;
  double v[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) v[s] = lane + kWave * s < N ? x[lane + kWave * s] : 0.0;
  // U^T y = b: column j of U^T is row j of U (right of the diagonal)
  double rn[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) rn[s] = lane + kWave * s < N ? Uf[lane + kWave * s] : 0.0;
  for (int jr = 0; jr < N; ++jr) {
    double r[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) r[s] = rn[s];
    if (jr + 1 < N)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = lane + kWave * s;
        rn[s] = i < N ? Uf[(size_t)(jr + 1) * N + i] : 0.0;
      }
    const int so = jr / kWave, lo = jr % kWave;
    double xj = 0.0, dj = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (s == so) {
        xj = readlane(v[s], lo);
        dj = readlane(r[s], lo);
      }
    const double yj = xj / dj;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + kWave * s;
      if (i > jr && i < N) v[s] -= r[s] * yj;
      if (s == so && lane == lo) v[s] = yj;
    }
  }
  // U x = y: column j of U above the diagonal is the mirrored row j
#pragma unroll
  for (int s = 0; s < NS; ++s) rn[s] = lane + kWave * s < N ? Uf[(size_t)(N - 1) * N + lane + kWave * s] : 0.0;
  for (int jr = N - 1; jr >= 0; --jr) {
    double r[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) r[s] = rn[s];
    if (jr > 0)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int i = lane + kWave * s;
        rn[s] = i < N ? Uf[(size_t)(jr - 1) * N + i] : 0.0;
      }
    const int so = jr / kWave, lo = jr % kWave;
    double xj = 0.0, dj = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s)
      if (s == so) {
        xj = readlane(v[s], lo);
        dj = readlane(r[s], lo);
      }
    const double xv = xj / dj;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int i = lane + kWave * s;
      if (i < jr) v[s] -= r[s] * xv;
      if (s == so && lane == lo) v[s] = xv;
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s)
    if (lane + kWave * s < N) x[lane + kWave * s] = v[s];
  __syncthreads();
}

// out = M^T v (out[c] = sum_k M[k][c] v[k]); v, out: LDS vectors of N.
template <int NW>
__device__ void matvec_t(const double* Mx, int N, const double* v, double* out, double scale) {
  constexpr int T = NW * kWave;
  for (int c = threadIdx.x; c < N; c += T) {
    double s = 0.0;
    for (int k = 0; k < N; ++k) s += Mx[(size_t)k * N + c] * v[k];
    out[c] = scale * s;
  }
  __syncthreads();
}

// out = M v (row dot products, one wavefront per row); v, out: LDS vectors of N.
template <int NW>
__device__ void matvec(const double* Mx, int N, const double* v, double* out) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  for (int k = wave; k < N; k += NW) {
    double s = 0.0;
    for (int c = lane; c < N; c += kWave) s += Mx[(size_t)k * N + c] * v[c];
    s = wave_sum(s);
    if (lane == 0) out[k] = s;
  }
  __syncthreads();
}

// sum over an LDS vector of f(i) (every thread calls; uniform result)
template <typename Sc, typename F>
__device__ __forceinline__ double vsum(Sc& sc, int N, F f) {
  double s = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) s += f(i);
  return sc.sum(s);
}

}  // namespace

namespace {

// After an accepted step: J at q (zeroed first: entries of frames that are not
// above one another stay 0), g = J^T r (r in rv), A = J^T J.  Returns this
// thread's largest diagonal entry of A.
template <int NW, int U, typename Sc>
__device__ __forceinline__ double lm_linearize(Sc& ws, const HocArgs<U>& args, const FrameGeo& geo, int f,
                                               bool valid, int j, int nf, int nfmax, const double q[U], int N,
                                               double* Jm, double* Am, const double* rv, double* gv,
                                               double* work, double* xs, double* ys) {
  for (int e = j; e < N * N; e += NW * kWave) Jm[e] = 0.0;
  __threadfence_block();
  __syncthreads();
  lm_jacobian<U>(ws, args, geo, f, valid, j, nf, nfmax, q, Jm, work);
  __threadfence_block();
  __syncthreads();
  matvec_t<NW>(Jm, N, rv, gv, 1.0);
  form_normal<NW>(Jm, Am, N, xs, ys);
  double dm = 0.0;
  for (int i = j; i < N; i += NW * kWave) dm = fmax(dm, Am[(size_t)i * N + i]);
  return dm;
}

// Maximum of v over the workgroup (uniform); red: LDS [NW].
template <int NW>
__device__ __forceinline__ double block_max(double* red, double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) m = fmax(m, red[w]);
  return m;
}

// This lane's U values into an LDS vector of the model (element u nf + j).
template <int U>
__device__ __forceinline__ void put_lane(double* vec, const double x[U], int nf, int j, bool valid) {
  if (valid)
#pragma unroll
    for (int u = 0; u < U; ++u) vec[u * nf + j] = x[u];
}

// LDS of the LM kernel: the scan buffers; the dynamic area holds six vectors of
// the batch's largest N and one work area (the frames' axes and joint points
// during a Jacobian assembly, the GEMM tiles and the diagonal block otherwise).
template <int NW, bool TREE, int U>
__global__ void __launch_bounds__(NW* kWave, 1) k_rollout_lm(LmArgs<U> la) {
  __shared__ ScanLds<NW, TREE> L;
  __shared__ int bad;
  extern __shared__ double dyn[];
  const HocArgs<U>& args = la.h;
  const DevModel& d = args.d;
  const int n = d.n_dofs;
  const int j = threadIdx.x;
  const bool lead = j == 0;
  if (blockIdx.x >= d.n_models) return;
  const int model = d.order[blockIdx.x];
  const int f0 = d.f0[model];
  const int nf = d.f0[model + 1] - f0;
  if (nf == 0) {
    if (lead && args.stats)
      for (int k = 0; k < args.n_steps; ++k) {
        abd_step_stats st = {0, 0, ABD_FLAG_CONVERGED, 0, 0, 0, 0.0, 0.0};
        args.stats[(size_t)k * d.n_models + model] = st;
      }
    return;
  }
  const int N = U * nf;
  const int nmax = U * la.nfmax;
  double* const rv = dyn;             // residuals r
  double* const gv = rv + nmax;       // J^T r
  double* const vv = gv + nmax;       // velocity v, then the step s
  double* const av = vv + nmax;       // acceleration a
  double* const t1 = av + nmax;       // J v, then J s
  double* const t2 = t1 + nmax;       // r_vv
  double* const work = t2 + nmax;
  double* const xs = work;            // GEMM tiles [kTK][kTM] + [kTK][kTN]
  double* const ys = work + kTK * kTM;
  double* const Dd = ys + kTK * kTN;  // diagonal block [kTM][kTM]
  double* const Jm = la.mat + la.moff[model];
  double* const Am = Jm + (size_t)N * N;
  double* const Um = Am + (size_t)N * N;
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);
  typename ModelScan<NW, TREE>::type ws = ModelScan<NW, TREE>::make(L, d, j / kWave, j % kWave, j, f, valid);
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;
  const FrameGeo geo = load_geo(d, f, valid);
  double qprev = valid ? args.q_prev[io] : 0.0;
  double qk = valid ? args.q_curr[io] : 0.0;

  __shared__ double red[NW];
  for (int step = 0; step < args.n_steps; ++step) {
    double q[U], rho[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = valid ? qk + args.tau_u[u] * args.vscale * (qk - qprev) : 0.0;
    const double tau = (valid && args.tau) ? args.tau[(size_t)step * n + io] : 0.0;
    int iters = 0, evals = 0, flag = 0;
    double E = 0.0, g0 = 0.0, gn = 0.0;
    // known seed parts of the step
    {
      const Xf<double> Ap = fk_geo<double>(ws, geo, valid, qprev);
      const Xf<double> Ak = fk_geo<double>(ws, geo, valid, qk);
      if (valid)
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int k = 0; k < 12; ++k)
            args.Bk[(size_t)f * (12 * U) + 12 * u + k] = args.w[u][0] * Ap.m[k] + args.w[u][1] * Ak.m[k];
    }
    __threadfence_block();
    __syncthreads();
    E = lm_residual<U>(ws, args, geo, f, valid, q, tau, rho);
    ++evals;
    put_lane<U>(rv, rho, nf, j, valid);
    double dmax = 0.0, lambda = 0.0, nu = 2.0;
    {
      bool fin = isfinite(E);
#pragma unroll
      for (int u = 0; u < U; ++u) fin = fin && isfinite(rho[u]);
      if (!ws.all_finite(fin ? 0.0 : NAN)) {
        flag = ABD_FLAG_NONFINITE;
      } else {
        dmax = block_max<NW>(red, lm_linearize<NW, U>(ws, args, geo, f, valid, j, nf, la.nfmax, q, N, Jm, Am, rv, gv, work,
                                              xs, ys));
        g0 = 2.0 * sqrt(vsum(ws, N, [&](int i) { return gv[i] * gv[i]; }));
        gn = g0;
        if (!isfinite(g0)) flag = ABD_FLAG_NONFINITE;
        else if (g0 == 0.0) flag = ABD_FLAG_CONVERGED;
        lambda = kLmLambda0 * dmax;
      }
    }
    while (flag == 0) {
      if (iters >= args.max_iter) {
        flag = ABD_FLAG_MAX_ITER;
        break;
      }
      ++iters;
      const double lam = fmax(lambda, kLmLambdaMin * dmax);
      if (!(lam <= 1e300)) {
        flag = ABD_FLAG_LS_FLOOR;
        break;
      }
      if (!factor<NW>(Am, Um, N, lam, xs, ys, Dd, &bad)) {
        lambda = lam * nu;
        nu *= 2.0;
        continue;
      }
      // velocity v = -(A + lam I)^-1 J^T r
      for (int i = j; i < N; i += NW * kWave) vv[i] = -gv[i];
      __syncthreads();
      chol_solve_lds<NW>(Um, N, vv);
      matvec<NW>(Jm, N, vv, t1);  // J v
      // geodesic acceleration from the residuals at q + h v
      double qh[U], rh[U];
#pragma unroll
      for (int u = 0; u < U; ++u) qh[u] = valid ? q[u] + kLmGeoH * vv[u * nf + j] : 0.0;
      lm_residual<U>(ws, args, geo, f, valid, qh, tau, rh);
      ++evals;
      if (valid)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k = u * nf + j;
          t2[k] = (2.0 / kLmGeoH) * ((rh[u] - rho[u]) / kLmGeoH - t1[k]);
        }
      __syncthreads();
      matvec_t<NW>(Jm, N, t2, av, -1.0);
      chol_solve_lds<NW>(Um, N, av);
      const double na = sqrt(vsum(ws, N, [&](int i) { return av[i] * av[i]; }));
      const double nv = sqrt(vsum(ws, N, [&](int i) { return vv[i] * vv[i]; }));
      if (!(2.0 * na <= kLmGeoAlpha * nv)) {
        lambda = lam * nu;
        nu *= 2.0;
        continue;
      }
      for (int i = j; i < N; i += NW * kWave) vv[i] += 0.5 * av[i];  // the step s
      __syncthreads();
      matvec<NW>(Jm, N, vv, t1);  // J s
      const double pred = vsum(ws, N, [&](int i) { const double x = rv[i] + t1[i]; return x * x; });
      double qt[U], rt[U];
#pragma unroll
      for (int u = 0; u < U; ++u) qt[u] = valid ? q[u] + vv[u * nf + j] : 0.0;
      const double Et = lm_residual<U>(ws, args, geo, f, valid, qt, tau, rt);
      ++evals;
      if (!(isfinite(Et) && Et < E)) {
        lambda = lam * nu;
        nu *= 2.0;
        continue;
      }
      double moved = 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u) moved += (valid && qt[u] != q[u]) ? 1.0 : 0.0;
      if (ws.sum(moved) == 0.0) {
        flag = ABD_FLAG_LS_FLOOR;
        break;
      }
      double gain = (E - Et) / fmax(E - pred, 1e-300);
      if (gain > 1.0) gain = 1.0;
      const double c3 = 2.0 * gain - 1.0;
      lambda = lam * fmax(1.0 / 3.0, 1.0 - c3 * c3 * c3);
      nu = 2.0;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        q[u] = qt[u];
        rho[u] = rt[u];
      }
      E = Et;
      put_lane<U>(rv, rho, nf, j, valid);
      dmax = block_max<NW>(red, lm_linearize<NW, U>(ws, args, geo, f, valid, j, nf, la.nfmax, q, N, Jm, Am, rv, gv, work, xs,
                                           ys));
      gn = 2.0 * sqrt(vsum(ws, N, [&](int i) { return gv[i] * gv[i]; }));
      if (gn <= args.tol * g0) flag = ABD_FLAG_CONVERGED;
    }
    if (valid)
#pragma unroll
      for (int u = 0; u < U; ++u) args.q_out[((size_t)step * U + u) * n + io] = q[u];
    if (args.stats && lead) {
      abd_step_stats st;
      st.iterations = iters;
      st.evaluations = evals;
      st.flag = flag;
      st.f32_iterations = 0;
      st.f32_evaluations = 0;
      st.reserved = 0;
      st.grad_norm = gn;
      st.energy = E;
      args.stats[(size_t)step * d.n_models + model] = st;
    }
    qprev = valid ? q[U - 2] : 0.0;
    qk = valid ? q[U - 1] : 0.0;
    __syncthreads();
  }
}

}  // namespace

namespace {

struct HessArgs {
  HocArgs<1> h;           // model, dt^2, weights (1, -2, 1), Bk = the model's per-step B
  const double* q;        // [n_dofs]
  double* H;              // per model a dense n_i x n_i row-major block
  const long long* hoff;  // [n_models+1] start of every model's block
  int nfmax;
};

// Hessian of the step objective (Eq. EQ scaled by dt^2) at q, explicitly: the
// Jacobian of its gradient, assembled like the order-K Jacobian with one point.
template <int NW, bool TREE>
__global__ void __launch_bounds__(NW* kWave) k_hessian(HessArgs a) {
  __shared__ ScanLds<NW, TREE> L;
  __shared__ int oidx[kMaxFrames * NW];
  extern __shared__ double wp[];  // [nfmax][6]
  const HocArgs<1>& args = a.h;
  const DevModel& d = args.d;
  const int j = threadIdx.x;
  const int model = blockIdx.x;
  const int f0 = d.f0[model];
  const int nf = d.f0[model + 1] - f0;
  if (nf == 0) return;
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);
  typename ModelScan<NW, TREE>::type ws = ModelScan<NW, TREE>::make(L, d, j / kWave, j % kWave, j, f, valid);
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;
  if (valid) oidx[j] = io - f0;  // the model's DOFs are contiguous from f0 in the caller's order too
  const FrameGeo geo = load_geo(d, f, valid);
  const double q = valid ? a.q[io] : 0.0;
  {
    const Xf<double> Ap = fk_geo<double>(ws, geo, valid, valid ? args.q_prev[io] : 0.0);
    const Xf<double> Ak = fk_geo<double>(ws, geo, valid, valid ? args.q_curr[io] : 0.0);
    if (valid)
#pragma unroll
      for (int k = 0; k < 12; ++k) args.Bk[(size_t)f * 12 + k] = Ap.m[k] - 2.0 * Ak.m[k];
  }
  double* Hm = a.H + a.hoff[model];
  for (int e = j; e < nf * nf; e += NW * kWave) Hm[e] = 0.0;
  __threadfence_block();
  __syncthreads();
  const double qq[1] = {q};
  lm_jacobian<1>(ws, args, geo, f, valid, j, nf, a.nfmax, qq, Hm, wp, oidx);
}

}  // namespace

namespace {

struct Lm2Args {
  DevModel d;
  double dt2, tol;
  int max_iter, n_steps;
  const double* q_prev;   // q_{-1}
  const double* q_curr;   // q_0
  const double* tau;      // [n_steps][n_dofs] or NULL
  double* q_out;          // [n_steps][n_dofs]
  abd_step_stats* stats;  // [n_steps][n_models] or NULL
  double* mat;            // per model: A = H_q (n_i x n_i), factor U
  const long long* moff;  // [n_models+1] start of every model's matrices
  int nfmax;
};

// Order 2 (Eq. EQ) by Levenberg-Marquardt (Sec. 5): the kinetic term is an
// integral of squares whose J^T J is the joint-space inertia H_q = C(q, q)
// (the Gauss-Newton part of the explicit Hessian, from composite sums); each
// iteration solves (H_q + lambda I) v = -grad E by the per-model Cholesky and
// accepts v if it decreases E (Nielsen's lambda rule against the model decrease
// -g.v - v.H_q v / 2).  One evaluation per iteration, no line search.
template <int NW, bool TREE>
__global__ void __launch_bounds__(NW* kWave, 1) k_rollout_lm2(Lm2Args la) {
  __shared__ ScanLds<NW, TREE> L;
  __shared__ int bad;
  __shared__ double red[NW];
  extern __shared__ double dyn[];
  const DevModel& d = la.d;
  const int n = d.n_dofs;
  const int j = threadIdx.x;
  const bool lead = j == 0;
  if (blockIdx.x >= d.n_models) return;
  const int model = d.order[blockIdx.x];
  const int f0 = d.f0[model];
  const int nf = d.f0[model + 1] - f0;
  if (nf == 0) {
    if (lead && la.stats)
      for (int k = 0; k < la.n_steps; ++k) {
        abd_step_stats st = {0, 0, ABD_FLAG_CONVERGED, 0, 0, 0, 0.0, 0.0};
        la.stats[(size_t)k * d.n_models + model] = st;
      }
    return;
  }
  const int N = nf;
  double* const vv = dyn;                 // step
  double* const hv = vv + la.nfmax;       // H_q v
  double* const work = hv + la.nfmax;
  double* const xs = work;
  double* const ys = work + kTK * kTM;
  double* const Dd = ys + kTK * kTN;
  double* const Am = la.mat + la.moff[model];
  double* const Um = Am + (size_t)N * N;
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);
  typename ModelScan<NW, TREE>::type ws = ModelScan<NW, TREE>::make(L, d, j / kWave, j % kWave, j, f, valid);
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;
  const FrameGeo geo = load_geo(d, f, valid);
  HocArgs<1> h;  // what the Gauss-Newton assembly reads: the model and C's weight 1
  h.d = d;
  h.dt2 = la.dt2;
  h.w[0][0] = 1.0;
  h.w[0][1] = -2.0;
  h.w[0][2] = 1.0;
  h.Bk = d.B64;
  double qkm1 = valid ? la.q_prev[io] : 0.0;
  double qk = valid ? la.q_curr[io] : 0.0;
  for (int step = 0; step < la.n_steps; ++step) {
    double q = valid ? 2.0 * qk - qkm1 : 0.0;
    const double tau = (valid && la.tau) ? la.tau[(size_t)step * n + io] : 0.0;
    int iters = 0, evals = 0, flag = 0;
    write_B(ws, d, geo, f, valid, qkm1, qk);
    __threadfence_block();
    __syncthreads();
    EvalResult r = evaluate<double>(ws, d, geo, f, valid, q, tau, la.dt2);
    ++evals;
    double E = r.E, g = r.g, gn = 0.0, g0 = 0.0, lambda = -1.0, nu = 2.0, dmax = 0.0;
    bool fresh = false;  // H_q assembled at the current q
    if (!isfinite(E) || !ws.all_finite(g)) {
      flag = ABD_FLAG_NONFINITE;
    } else {
      g0 = uniform(sqrt(ws.sum(g * g)));
      gn = g0;
      if (g0 == 0.0) flag = ABD_FLAG_CONVERGED;
    }
    while (flag == 0) {
      if (iters >= la.max_iter) {
        flag = ABD_FLAG_MAX_ITER;
        break;
      }
      ++iters;
      if (!fresh) {
        for (int e = j; e < N * N; e += NW * kWave) Am[e] = 0.0;
        __threadfence_block();
        __syncthreads();
        const double qq[1] = {q};
        lm_jacobian<1, decltype(ws), false>(ws, h, geo, f, valid, j, nf, la.nfmax, qq, Am, work);
        __threadfence_block();
        __syncthreads();
        double dm = 0.0;
        for (int i = j; i < N; i += NW * kWave) dm = fmax(dm, Am[(size_t)i * N + i]);
        dmax = block_max<NW>(red, dm);
        fresh = true;
        if (lambda < 0.0) lambda = kLmLambda0 * dmax;
      }
      const double lam = fmax(lambda, kLmLambdaMin * dmax);
      if (!(lam <= 1e300)) {
        flag = ABD_FLAG_LS_FLOOR;
        break;
      }
      if (!factor<NW>(Am, Um, N, lam, xs, ys, Dd, &bad)) {
        lambda = lam * nu;
        nu *= 2.0;
        continue;
      }
      if (valid) vv[j] = -g;
      __syncthreads();
      if constexpr (NW == 1) {
        chol_solve_wave<1>(Um, N, vv);
        matvec_t<NW>(Am, N, vv, hv, 1.0);  // H_q v (the assembled H_q is symmetric)
      } else {
        chol_solve_lds<NW>(Um, N, vv);
        matvec<NW>(Am, N, vv, hv);
      }
      const double v = valid ? vv[j] : 0.0;
      const double pred = -ws.sum(g * v + 0.5 * v * (valid ? hv[j] : 0.0));
      const double x = q + v;
      const EvalResult rt = evaluate<double>(ws, d, geo, f, valid, x, tau, la.dt2);
      ++evals;
      if (!(isfinite(rt.E) && ws.all_finite(rt.g) && rt.E < E)) {
        lambda = lam * nu;
        nu *= 2.0;
        continue;
      }
      if (uniform(ws.sum(valid && x != q ? 1.0 : 0.0)) == 0.0) {
        flag = ABD_FLAG_LS_FLOOR;
        break;
      }
      double gain = (E - rt.E) / fmax(pred, 1e-300);
      if (gain > 1.0) gain = 1.0;
      const double c3 = 2.0 * gain - 1.0;
      lambda = lam * fmax(1.0 / 3.0, 1.0 - c3 * c3 * c3);
      nu = 2.0;
      q = x;
      g = rt.g;
      E = rt.E;
      fresh = false;
      gn = uniform(sqrt(ws.sum(g * g)));
      if (gn <= la.tol * g0) flag = ABD_FLAG_CONVERGED;
    }
    if (valid) la.q_out[(size_t)step * n + io] = q;
    if (la.stats && lead) {
      abd_step_stats st;
      st.iterations = iters;
      st.evaluations = evals;
      st.flag = flag;
      st.f32_iterations = 0;
      st.f32_evaluations = 0;
      st.reserved = 0;
      st.grad_norm = gn;
      st.energy = E;
      la.stats[(size_t)step * d.n_models + model] = st;
    }
    qkm1 = qk;
    qk = q;
    __syncthreads();
  }
}

}  // namespace

namespace abd_impl {

// Per-model dense matrices of the LM solvers, sized for three unknown points
// (3 (3 n_i)^2 doubles per model), allocated on a model's first LM call.
static int lm_matrices(abd_model* m) {
  if (m->lm_mat) return ABD_OK;
  std::vector<long long> off(m->n_models + 1, 0);
  for (int i = 0; i < m->n_models; ++i) {
    const long long nmat = 3LL * (m->f0_host[i + 1] - m->f0_host[i]);
    off[i + 1] = off[i] + 3 * nmat * nmat;
  }
  void* p = nullptr;
  int rc;
  if ((rc = model_alloc(m, &p, std::max<long long>(1, off[m->n_models]) * sizeof(double)))) return rc;
  m->lm_mat = static_cast<double*>(p);
  if ((rc = model_alloc(m, &p, off.size() * sizeof(long long)))) return rc;
  m->lm_off = static_cast<long long*>(p);
  HIP_TRY(hipMemcpy(m->lm_off, off.data(), off.size() * sizeof(long long), hipMemcpyHostToDevice));
  return ABD_OK;
}

int launch_lm_hoc(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
                  const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream) {
  int rc = check_hoc(m, o);
  if (rc) return rc;
  if (o->precision != ABD_FP64) return fail(ABD_ENOTSUP, "ABD_SOLVER_LM runs in ABD_FP64 only in this library");
  const int U = o->order_K - 1;
  if (U != 2)
    return fail(ABD_ENOTSUP, "ABD_SOLVER_LM handles order_K = 3 in this library (order 4 is switched off)");
  // per-model dense matrices (J, J^T J, factor)
  if ((rc = lm_matrices(m))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nw = waves_for(m->max_frames);
  const int nfmax = m->max_frames;
  const size_t work = std::max<size_t>((size_t)U * 6 * nfmax, (size_t)kTK * (kTM + kTN) + kTM * kTM);
  const size_t lds = (6 * (size_t)U * nfmax + work) * sizeof(double);
  const dim3 grid(m->n_models), block(nw * kWave);
#define ABD_LM(NW, TREE, UU)                                                                   \
  do {                                                                                         \
    LmArgs<UU> a;                                                                              \
    if ((rc = fill_hoc_args<UU>(m, o, a.h))) return rc;                                        \
    a.h.n_steps = n_steps; a.h.q_prev = q_prev; a.h.q_curr = q_curr; a.h.tau = tau;            \
    a.h.q_out = q_out; a.h.stats = stats;                                                      \
    a.mat = m->lm_mat; a.moff = m->lm_off; a.nfmax = nfmax;                                    \
    if (lds > 65536)                                                                           \
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rollout_lm<NW, TREE, UU>),  \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));      \
    hipLaunchKernelGGL((k_rollout_lm<NW, TREE, UU>), grid, block, lds, s, a);                  \
  } while (0)
#define ABD_LM_U(NW, TREE) ABD_LM(NW, TREE, 2)
  if (m->tree) {
    if (nw == 1) ABD_LM_U(1, true);
    else if (nw == 2) ABD_LM_U(2, true);
    else ABD_LM_U(4, true);
  } else {
    if (nw == 1) ABD_LM_U(1, false);
    else if (nw == 2) ABD_LM_U(2, false);
    else ABD_LM_U(4, false);
  }
#undef ABD_LM_U
#undef ABD_LM
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

int launch_hessian(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist, double* H,
                   void* stream) {
  int rc;
  if (!m->sq_off) {
    std::vector<long long> off(m->n_models + 1, 0);
    for (int i = 0; i < m->n_models; ++i) {
      const long long nfi = m->f0_host[i + 1] - m->f0_host[i];
      off[i + 1] = off[i] + nfi * nfi;
    }
    void* p = nullptr;
    if ((rc = model_alloc(m, &p, off.size() * sizeof(long long)))) return rc;
    m->sq_off = static_cast<long long*>(p);
    HIP_TRY(hipMemcpy(m->sq_off, off.data(), off.size() * sizeof(long long), hipMemcpyHostToDevice));
  }
  HessArgs a;
  a.h.d = dev_view(m);
  a.h.dt2 = o->dt * o->dt;
  a.h.w[0][0] = 1.0;
  a.h.w[0][1] = -2.0;
  a.h.w[0][2] = 1.0;
  a.h.q_prev = q_hist;
  a.h.q_curr = q_hist + m->n_dofs;
  a.h.Bk = m->B64;  // the model's per-step constant, rewritten here for this q_hist
  a.q = q;
  a.H = H;
  a.hoff = m->sq_off;
  a.nfmax = m->max_frames;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nw = waves_for(m->max_frames);
  const size_t lds = (size_t)6 * m->max_frames * sizeof(double);
  const dim3 grid(m->n_models), block(nw * kWave);
#define ABD_HESS(NW, TREE) hipLaunchKernelGGL((k_hessian<NW, TREE>), grid, block, lds, s, a)
  if (m->tree) {
    if (nw == 1) ABD_HESS(1, true);
    else if (nw == 2) ABD_HESS(2, true);
    else ABD_HESS(4, true);
  } else {
    switch (nw) {
      case 1: ABD_HESS(1, false); break;
      case 2: ABD_HESS(2, false); break;
      case 4: ABD_HESS(4, false); break;
      case 8: ABD_HESS(8, false); break;
      default: ABD_HESS(16, false); break;
    }
  }
#undef ABD_HESS
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

int launch_lm2(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
               const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream) {
  if (o->precision != ABD_FP64) return fail(ABD_ENOTSUP, "ABD_SOLVER_LM runs in ABD_FP64 only in this library");
  int rc = lm_matrices(m);
  if (rc) return rc;
  Lm2Args a;
  a.d = dev_view(m);
  a.dt2 = o->dt * o->dt;
  a.tol = o->tol;
  a.max_iter = o->max_iter;
  a.n_steps = n_steps;
  a.q_prev = q_prev;
  a.q_curr = q_curr;
  a.tau = tau;
  a.q_out = q_out;
  a.stats = stats;
  a.mat = m->lm_mat;
  a.moff = m->lm_off;
  a.nfmax = m->max_frames;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nw = waves_for(m->max_frames);
  const size_t work = std::max<size_t>((size_t)6 * m->max_frames, (size_t)kTK * (kTM + kTN) + kTM * kTM);
  const size_t lds = (2 * (size_t)m->max_frames + work) * sizeof(double);
  const dim3 grid(m->n_models), block(nw * kWave);
#define ABD_LM2(NW, TREE)                                                                       \
  do {                                                                                          \
    if (lds > 65536)                                                                            \
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_rollout_lm2<NW, TREE>),      \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));       \
    hipLaunchKernelGGL((k_rollout_lm2<NW, TREE>), grid, block, lds, s, a);                      \
  } while (0)
  if (m->tree) {
    if (nw == 1) ABD_LM2(1, true);
    else if (nw == 2) ABD_LM2(2, true);
    else ABD_LM2(4, true);
  } else {
    switch (nw) {
      case 1: ABD_LM2(1, false); break;
      case 2: ABD_LM2(2, false); break;
      case 4: ABD_LM2(4, false); break;
      case 8: ABD_LM2(8, false); break;
      default: ABD_LM2(16, false); break;
    }
  }
#undef ABD_LM2
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

}  // namespace abd_impl
