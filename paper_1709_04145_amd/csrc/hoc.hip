// hoc.hip -- high-order collocation (Sec. 4, Eq. HOC / Eq. EQHOC): kernels and launches.
#include "hoc_common.h"

namespace {


// Derivative along a tangent (dA, W) of the adjoint pass at poses A with a FIXED
// seed G (K, F = its suffix sums at these poses):
//   dk = sum_c dR[:,c] x G[:,c] + dt x G[:,3],  dF = 0,
//   result_n = dw_n . (K_n - p_n x F_n) + w_n . (dK_n - dp_n x F_n).
template <typename Sc>
__device__ double adjoint_fixed_seed_tangent(Sc& sc, const Xf<double>& A, const double dA[12], const double W[3],
                                             const double w[3], const double G[12], const double K[3],
                                             const double F[3], bool valid) {
  double dk[3] = {0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double dcol[3] = {dA[c], dA[4 + c], dA[8 + c]};
    const double gc[3] = {G[c], G[4 + c], G[8 + c]};
    double x[3];
    cross3(dcol, gc, x);
#pragma unroll
    for (int i = 0; i < 3; ++i) dk[i] += x[i];
  }
  double dK6[6] = {valid ? dk[0] : 0.0, valid ? dk[1] : 0.0, valid ? dk[2] : 0.0, 0.0, 0.0, 0.0};
  double ua = 0.0, ub = 0.0;
  sc.suffix6_total2(dK6, ua, ub);
  const double p[3] = {A.m[3], A.m[7], A.m[11]};
  const double dp[3] = {dA[3], dA[7], dA[11]};
  double dw[3], pF[3], dpF[3];
  cross3(W, w, dw);
  cross3(p, F, pF);
  cross3(dp, F, dpF);
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) r += dw[i] * (K[i] - pF[i]) + w[i] * (dK6[i] - dpF[i]);
  return valid ? r : 0.0;
}

// One EQHOC evaluation: E (wave-uniform) and the gradient g[U] of this lane.
// R: precision of the forward kinematics (float for the float32 phase of a
// mixed step: the poses are then widened and everything after them, seeds,
// residuals, tangents and adjoint sums, runs in float64).
template <int U, typename R = double, typename Sc>
__device__ double hoc_evaluate(Sc& sc, const HocArgs<U>& args, const FrameGeo& geo, int f, bool valid,
                               const double q[U], double tau, double g[U], double* rho_sum = nullptr) {
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
  for (int u = 0; u < U; ++u) {
    const Xf<R> Ar = fk_geo<R>(sc, geo, valid, q[u]);
#pragma unroll
    for (int k = 0; k < 12; ++k) A[u].m[k] = (double)Ar.m[k];
  }
  // seeds, residuals and their suffix sums
  double rho[U], KF[U][6];
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
    double k[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double col[3] = {A[u].m[c], A[u].m[4 + c], A[u].m[8 + c]};
      const double gc[3] = {G[c], G[4 + c], G[8 + c]};
      double x[3];
      cross3(col, gc, x);
#pragma unroll
      for (int i = 0; i < 3; ++i) k[i] += x[i];
    }
    KF[u][0] = valid ? k[0] : 0.0; KF[u][1] = valid ? k[1] : 0.0; KF[u][2] = valid ? k[2] : 0.0;
    KF[u][3] = valid ? G[3] : 0.0; KF[u][4] = valid ? G[7] : 0.0; KF[u][5] = valid ? G[11] : 0.0;
    double ua = 0.0, ub = 0.0;
    sc.suffix6_total2(KF[u], ua, ub);
    double w[3], pF[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = A[u].m[4 * i] * geo.a[0] + A[u].m[4 * i + 1] * geo.a[1] + A[u].m[4 * i + 2] * geo.a[2];
    const double p[3] = {A[u].m[3], A[u].m[7], A[u].m[11]};
    const double F[3] = {KF[u][3], KF[u][4], KF[u][5]};
    cross3(p, F, pF);
    const double r = w[0] * (KF[u][0] - pF[0]) + w[1] * (KF[u][1] - pF[1]) + w[2] * (KF[u][2] - pF[2]);
    rho[u] = valid ? r - args.dt2 * tau : 0.0;
    E += rho[u] * rho[u];
  }
  if (rho_sum) {
    double t = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) t += rho[u];
    *rho_sum = t;
  }
  E = sc.sum(E);
  // tangents along the residuals; fixed-seed terms; mixed-seed accumulation
  double S[U][12];
#pragma unroll
  for (int a = 0; a < U; ++a)
#pragma unroll
    for (int i = 0; i < 12; ++i) S[a][i] = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    double dA[12], W[3], w[3];
    tangent_pose(sc, A[u], geo.a, valid, rho[u], dA, W, w);
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
    const double K3[3] = {KF[u][0], KF[u][1], KF[u][2]}, F3[3] = {KF[u][3], KF[u][4], KF[u][5]};
    g[u] = adjoint_fixed_seed_tangent(sc, A[u], dA, W, w, G, K3, F3, valid);
    // dA_u M, accumulated into the mixed seeds of every unknown a
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int x = 0; x < 4; ++x) s += dA[4 * r + x] * M[sym4(x, c)];
#pragma unroll
        for (int a = 0; a < U; ++a) S[a][4 * r + c] += args.w[u][2 + a] * s;
      }
  }
#pragma unroll
  for (int a = 0; a < U; ++a) g[a] = 2.0 * (g[a] + adjoint_of_seed(sc, A[a], S[a], geo.a, valid));
  return E;
}

// A mixed step (PREC = ABD_MIXED) evaluates with float32 kinematics until its
// gradient has dropped to kHocF32Drop of the warm start's (the residuals are
// sums of poses whose weights, up to 82 at K = 4, cancel to O(dt^2), so float32
// poses resolve the gradient only to about that), float32 claims convergence,
// its line search meets float32 rounding or fails, or its direction is no
// descent; it then re-evaluates at the iterate in float64, drops the pairs and
// goes on in float64.
constexpr double kHocF32Drop = 1e-3;

template <int NW, bool TREE, int U, int PREC = ABD_FP64>
__global__ void __launch_bounds__(NW* kWave, 1) k_rollout_hoc(HocArgs<U> args) {
  __shared__ RollLds<NW, TREE> L;
  // one-wave models: s ring [m][U][64], then y ring; one-wave chains: then the
  // packed explicit inverse (inverse_lds_doubles(max frames))
  extern __shared__ double pairs[];
  double* const hl = pairs + 2 * args.m * U * kWave;
  const DevModel& d = args.d;
  const int n = d.n_dofs;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int j = threadIdx.x;
  const bool lead = threadIdx.x == 0;
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
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);
  typename ModelScan<NW, TREE>::type ws = ModelScan<NW, TREE>::make(L, d, wave, lane, j, f, valid);
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;
  const bool use_aba = args.precond == ABD_PRECOND_INERTIA;
  const bool explicit_inverse = NW == 1 && !TREE;
  double* Hi = d.hinv + d.hoff[model];
  const int fend_j = TREE && valid ? d.fend[f] : j;  // the last frame below this one
  __shared__ double inert_sink[10];  // written by lanes without a frame, never read
  const FrameGeo geo = load_geo(d, f, valid);
  const double c1 = 1e-4, dlt = 0.1;
  double qprev = valid ? args.q_prev[io] : 0.0;
  double qk = valid ? args.q_curr[io] : 0.0;
  // pairs: s of slot k, unknown u at sp[(k * U + u) * stride], y likewise at yp
  double *sp, *yp;
  int stride;
  if (NW == 1) {
    sp = pairs + lane;
    yp = pairs + args.m * U * kWave + lane;
    stride = kWave;
  } else {
    sp = args.hist3 + (size_t)f * (2 * kMaxHist * 3);
    yp = sp + kMaxHist * 3;
    stride = 1;
  }
  for (int step = 0; step < args.n_steps; ++step) {
    double q[U], g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = valid ? qk + args.tau_u[u] * args.vscale * (qk - qprev) : 0.0;
    const double tau = (valid && args.tau) ? args.tau[(size_t)step * n + io] : 0.0;
    int iters = 0, evals = 0, flag = 0, count = 0, head = 0, f32_iters = 0, f32_evals = 0;
    double E = 0.0, g0 = 0.0, gn = 0.0, gam = 1.0;
    bool reset = false, f32 = PREC == ABD_MIXED, to64 = false;
    // one evaluation at the precision of the step's current phase
    auto evaluate_hoc = [&](const double* qq, double* gg) -> double {
      ++evals;
      if (PREC == ABD_MIXED && f32) {
        ++f32_evals;
        return hoc_evaluate<U, float>(ws, args, geo, f, valid, qq, tau, gg);
      }
      return hoc_evaluate<U, double>(ws, args, geo, f, valid, qq, tau, gg);
    };
    if (nf == 0) {
      flag = ABD_FLAG_CONVERGED;
    } else {
      // known seed parts and the preconditioner at q_k
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
      if (use_aba) {
        // lanes without a frame of a multi-wave model: a sink, not frame 0's slot
        double* inert = NW == 1 ? (TREE ? L.inert[lane] : hl + 10 * lane) : (valid ? Hi + (size_t)j * 10 : inert_sink);
        step_setup(ws, d, inert, L.tab[j], geo, f, valid, qprev, qk, qk, true);
        if (NW > 1) __threadfence_block();
        __syncthreads();
        if (TREE) {
          if (PREC == ABD_FP64)
            aba_setup_tree_levels(NW == 1 ? &L.inert[0][0] : Hi, L.tab, d.fend + f0, Hi + 10 * (size_t)nf, j, valid,
                                  valid ? d.fheight[f] : 0, d.mheight[model]);
          else if (lead)
            aba_setup_tree(NW == 1 ? &L.inert[0][0] : Hi, L.tab, L.tpar, Hi + 10 * (size_t)nf, nf);
        } else if (wave == 0) {
          aba_setup_rows(NW == 1 ? hl : Hi, L.tab, nf, lane);
        }
        __syncthreads();
        if (explicit_inverse) {
          aba_inverse(L.tab, nf, lane, hl);  // overwrites the inertias
          __syncthreads();  // every lane reads the other lanes' columns
        }
        if (TREE && PREC == ABD_FP64) {
          // the explicit L^-1 of the recursion, one column per frame's thread
          tree_inverse_factor(L.tab, L.tpar, d.wrow + f0, Hi + 31 * (size_t)nf, j, valid);
          __threadfence_block();
          __syncthreads();
        }
      }
      E = evaluate_hoc(q, g);
      bool fin = isfinite(E);
#pragma unroll
      for (int u = 0; u < U; ++u) fin = fin && ws.all_finite(g[u]);
      if (!fin) {
        flag = ABD_FLAG_NONFINITE;
      } else {
        double gg = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) gg += g[u] * g[u];
        g0 = uniform(sqrt(ws.sum(gg)));
        gn = g0;
        if (g0 == 0.0) flag = ABD_FLAG_CONVERGED;
        else if (args.max_iter <= 0) flag = ABD_FLAG_MAX_ITER;
      }
      while (flag == 0) {
        if (PREC == ABD_MIXED && to64) {
          // leave float32: re-evaluate at q in float64 and restart the history
          to64 = false;
          f32 = false;
          count = 0;
          reset = false;
          E = evaluate_hoc(q, g);
          bool fin64 = isfinite(E);
          double gg = 0.0;
#pragma unroll
          for (int u = 0; u < U; ++u) {
            fin64 = fin64 && ws.all_finite(g[u]);
            gg += g[u] * g[u];
          }
          if (!fin64) {
            flag = ABD_FLAG_NONFINITE;
            break;
          }
          gn = uniform(sqrt(ws.sum(gg)));
          if (gn <= args.tol * g0) {
            flag = ABD_FLAG_CONVERGED;
            break;
          }
          if (iters >= args.max_iter) {
            flag = ABD_FLAG_MAX_ITER;
            break;
          }
        }
        if (reset) count = 0;
        // ---- two-loop recursion, newest pair first
        double qv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) qv[u] = g[u];
        for (int k = 0; k < count; ++k) {
          const int slot = (head - k + args.m) % args.m;
          double sq = 0.0;
#pragma unroll
          for (int u = 0; u < U; ++u) sq += ld_if(sp + (slot * U + u) * stride, valid) * qv[u];
          const double sqs = ws.sum(sq);  // reduction (a barrier for several waves) before the rho read
          const double a_k = uniform(L.rho[k] * sqs);
          if (lead) L.alp[k] = a_k;
#pragma unroll
          for (int u = 0; u < U; ++u) qv[u] -= a_k * ld_if(yp + (slot * U + u) * stride, valid);
        }
        // ---- initial inverse Hessian: (W^T W)^-1 (x) H_q^-2, or gamma I
        double r[U];
        if (use_aba) {
          double y[U];
          if (explicit_inverse) {
#pragma unroll
            for (int u = 0; u < U; ++u)
              y[u] = apply_inverse(hl, &L.tab[0][0], nf, lane, apply_inverse(hl, &L.tab[0][0], nf, lane, qv[u]));
          } else if (TREE && PREC == ABD_FP64) {
            const double* W = Hi + 31 * (size_t)nf;
#pragma unroll
            for (int u = 0; u < U; ++u)
              y[u] = tree_apply_inverse(L.tab, L.tpar, d.wrow + f0, W, L.xb, &L.acc[0][0], j, fend_j, valid,
                                        tree_apply_inverse(L.tab, L.tpar, d.wrow + f0, W, L.xb, &L.acc[0][0], j,
                                                           fend_j, valid, qv[u]));
          } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
              L.xb[j] = valid ? qv[u] : 0.0;
              __syncthreads();
              // (the mixed kernels of branched models keep the one-thread sweeps)
              if (lead)
                for (int rep = 0; rep < 2; ++rep) {
                  if (TREE)
                    aba_solve_tree(L.tab, L.xb, L.tpar, L.acc, nf);
                  else
                    aba_solve(L.tab, L.xb, nf);
                }
              __syncthreads();
              y[u] = valid ? L.xb[j] : 0.0;
              __syncthreads();
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < U; ++a) t += args.minv[u][a] * y[a];
            r[u] = t;
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) r[u] = (count > 0 ? gam : 1.0) * qv[u];
        }
        // ---- oldest pair first
        for (int k = count - 1; k >= 0; --k) {
          const int slot = (head - k + args.m) % args.m;
          double yr = 0.0;
#pragma unroll
          for (int u = 0; u < U; ++u) yr += ld_if(yp + (slot * U + u) * stride, valid) * r[u];
          const double yrs = ws.sum(yr);
          const double b = uniform(L.rho[k] * yrs);
#pragma unroll
          for (int u = 0; u < U; ++u) r[u] += (L.alp[k] - b) * ld_if(sp + (slot * U + u) * stride, valid);
        }
        double dir[U], gdl = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          dir[u] = valid ? -r[u] : 0.0;
          gdl += g[u] * dir[u];
        }
        const double gd = uniform(ws.sum(gdl));
        if (!(gd < 0.0)) {
          if (!reset && count > 0) {
            reset = true;
            continue;
          }
          if (PREC == ABD_MIXED && f32) {
            to64 = true;  // the float32 gradient gives no descent direction
            continue;
          }
          flag = ABD_FLAG_LS_FLOOR;
          break;
        }
        reset = false;
        const double eps_w = (PREC == ABD_MIXED && f32) ? 5.9604644775390625e-8 : 1.1102230246251565e-16;
        double alpha = 1.0, Et = 0.0, qt[U], gt[U];
        bool ok = false, noisy = false;
        for (int ls = 0; ls < args.max_ls; ++ls) {
#pragma unroll
          for (int u = 0; u < U; ++u) qt[u] = q[u] + alpha * dir[u];
          Et = evaluate_hoc(qt, gt);
          bool fin = isfinite(Et);
#pragma unroll
          for (int u = 0; u < U; ++u) fin = fin && ws.all_finite(gt[u]);
          if (fin) {
            if (Et <= E + c1 * alpha * gd) {
              ok = true;
            } else if (fabs(Et - E) <= 10.0 * eps_w * Et) {
              noisy = true;
              double gtdl = 0.0;
#pragma unroll
              for (int u = 0; u < U; ++u) gtdl += gt[u] * dir[u];
              if (ws.sum(gtdl) <= (2.0 * dlt - 1.0) * gd) ok = true;
            }
          }
          if (ok) break;
          alpha = next_alpha(alpha, E, Et, gd);
        }
        if (!ok) {
          if (PREC == ABD_MIXED && f32) {
            to64 = true;  // float32 stalls the search: continue in float64 from q
            continue;
          }
          flag = ABD_FLAG_LS_FLOOR;
          break;
        }
        {
          // an accepted point equal to q in every coordinate is no progress
          double mv = 0.0;
#pragma unroll
          for (int u = 0; u < U; ++u) mv += (valid && qt[u] != q[u]) ? 1.0 : 0.0;
          if (uniform(ws.sum(mv)) == 0.0) {
            if (PREC == ABD_MIXED && f32) {
              to64 = true;
              continue;
            }
            flag = ABD_FLAG_LS_FLOOR;
            break;
          }
        }
        double syl = 0.0, ssl = 0.0, yyl = 0.0, ggl = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double sv = qt[u] - q[u], yv = gt[u] - g[u];
          syl += sv * yv;
          ssl += sv * sv;
          yyl += yv * yv;
          ggl += gt[u] * gt[u];
        }
        ws.sum2(syl, ssl);
        ws.sum2(yyl, ggl);
        if (syl > 1e-12 * sqrt(ssl) * sqrt(yyl)) {
          if (lead) {
            for (int k = args.m - 1; k > 0; --k) L.rho[k] = L.rho[k - 1];
            L.rho[0] = 1.0 / syl;
          }
          gam = uniform(syl / yyl);
          head = count == 0 ? 0 : (head + 1) % args.m;
          if (valid)
#pragma unroll
            for (int u = 0; u < U; ++u) {
              sp[(head * U + u) * stride] = qt[u] - q[u];
              yp[(head * U + u) * stride] = gt[u] - g[u];
            }
          if (count < args.m) ++count;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          q[u] = qt[u];
          g[u] = gt[u];
        }
        E = Et;
        ++iters;
        if (PREC == ABD_MIXED && f32) ++f32_iters;
        gn = uniform(sqrt(ggl));
        if (PREC == ABD_MIXED && f32 && (gn <= fmax(args.tol, kHocF32Drop) * g0 || noisy)) {
          to64 = true;  // float32 has done what it can: confirm / continue in float64
          continue;
        }
        if (gn <= args.tol * g0) flag = ABD_FLAG_CONVERGED;
        else if (iters >= args.max_iter) flag = ABD_FLAG_MAX_ITER;
      }
    }
    if (valid)
#pragma unroll
      for (int u = 0; u < U; ++u) args.q_out[((size_t)step * U + u) * n + io] = q[u];
    if (args.stats && lead) {
      abd_step_stats st;
      st.iterations = iters;
      st.evaluations = evals;
      st.flag = flag;
      st.f32_iterations = f32_iters;
      st.f32_evaluations = f32_evals;
      st.reserved = 0;
      st.grad_norm = gn;
      st.energy = E;
      args.stats[(size_t)step * d.n_models + model] = st;
    }
    qprev = valid ? q[U - 2] : 0.0;
    qk = valid ? q[U - 1] : 0.0;
  }
}

struct HocObjArgs {
  DevModel d;
  double dt2;
  double w[3][5];
  const double* q_prev;
  const double* q_curr;
  const double* q;     // [U][n]
  const double* tau;
  double* E;
  double* grad;        // [U][n] or NULL
  double* grad_tau;    // [n] or NULL
  double* Bk;
};

template <int NW, bool TREE, int U, typename R = double>
__global__ void __launch_bounds__(NW* kWave) k_hoc_objective(HocObjArgs a) {
  __shared__ ScanLds<NW, TREE> L;
  const DevModel& d = a.d;
  const int model = blockIdx.x, j = threadIdx.x;
  const int f0 = d.f0[model], nf = d.f0[model + 1] - f0;
  if (nf == 0) {
    if (j == 0) a.E[model] = 0.0;
    return;
  }
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);
  const int n = d.n_dofs;
  typename ModelScan<NW, TREE>::type ws = ModelScan<NW, TREE>::make(L, d, j / kWave, j % kWave, j, f, valid);
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;
  const FrameGeo geo = load_geo(d, f, valid);
  HocArgs<U> h;
  h.d = d;
  h.dt2 = a.dt2;
  for (int u = 0; u < U; ++u)
    for (int p = 0; p < U + 2; ++p) h.w[u][p] = a.w[u][p];
  h.Bk = a.Bk;
  {
    const Xf<double> Ap = fk_geo<double>(ws, geo, valid, valid ? a.q_prev[io] : 0.0);
    const Xf<double> Ak = fk_geo<double>(ws, geo, valid, valid ? a.q_curr[io] : 0.0);
    if (valid)
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < 12; ++k)
          a.Bk[(size_t)f * (12 * U) + 12 * u + k] = h.w[u][0] * Ap.m[k] + h.w[u][1] * Ak.m[k];
  }
  double q[U], g[U];
#pragma unroll
  for (int u = 0; u < U; ++u) q[u] = valid ? a.q[(size_t)u * n + io] : 0.0;
  const double tau = (valid && a.tau) ? a.tau[io] : 0.0;
  double rsum = 0.0;
  const double E = hoc_evaluate<U, R>(ws, h, geo, f, valid, q, tau, g, &rsum);
  if (j == 0) a.E[model] = E;
  // rho_u = (adjoint term) - dt^2 tau, so dE/dtau = -2 dt^2 sum_u rho_u
  if (a.grad_tau && valid) a.grad_tau[io] = -2.0 * a.dt2 * rsum;
  if (a.grad && valid)
#pragma unroll
    for (int u = 0; u < U; ++u) a.grad[(size_t)u * n + io] = g[u];
}

}  // namespace

namespace abd_impl {

// Collocation of order K = 3, 4 (Eq. HOC): the interior points are the roots of
// the Legendre polynomial L_{K-2}(2 alpha - 1) (closed forms for K <= 4) and
// alpha_{K-1} = 1; the K+1 points of a step are tau = (alpha_{K-2} - 1, 0,
// alpha_1, ..., alpha_{K-1}).  The weights of the second derivative at an
// unknown point x solve the moment conditions sum_j w_j tau_j^p = p (p-1) x^(p-2),
// p = 0..K (exact for polynomials of degree <= K), by Gaussian elimination.
void hoc_collocation(int K, double* tau, double* w) {
  double alpha[4] = {0, 0, 0, 0};
  if (K == 3) {
    alpha[1] = 0.5;
  } else {
    alpha[1] = 0.5 * (1.0 - 1.0 / std::sqrt(3.0));
    alpha[2] = 0.5 * (1.0 + 1.0 / std::sqrt(3.0));
  }
  alpha[K - 1] = 1.0;
  tau[0] = alpha[K - 2] - 1.0;
  tau[1] = 0.0;
  for (int u = 1; u <= K - 1; ++u) tau[1 + u] = alpha[u];
  const int np = K + 1;
  for (int u = 0; u < K - 1; ++u) {
    const double x = tau[2 + u];
    double a[5][6];
    for (int p = 0; p < np; ++p) {
      for (int j = 0; j < np; ++j) a[p][j] = std::pow(tau[j], p);
      a[p][np] = p >= 2 ? p * (p - 1) * std::pow(x, p - 2) : 0.0;
    }
    for (int c = 0; c < np; ++c) {
      int piv = c;
      for (int r = c + 1; r < np; ++r)
        if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
      for (int k = 0; k <= np; ++k) std::swap(a[c][k], a[piv][k]);
      for (int r = 0; r < np; ++r) {
        if (r == c) continue;
        const double fct = a[r][c] / a[c][c];
        for (int k = c; k <= np; ++k) a[r][k] -= fct * a[c][k];
      }
    }
    for (int j = 0; j < np; ++j) w[u * np + j] = a[j][np] / a[j][j];
  }
}

int check_hoc(const abd_model* m, const abd_step_opts* o) {
  if (m->max_frames > 4 * kMaxFrames)
    return fail(ABD_ENOTSUP, "order_K > 2 handles models of at most 256 DOFs in this library");
  return ABD_OK;
}

int launch_hoc(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
               const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream,
               const StepScratch* sc) {
  int rc = check_hoc(m, o);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int U = o->order_K - 1;
  const int nw = waves_for(m->max_frames);
  size_t pair_bytes = nw == 1 ? 2 * (size_t)o->lbfgs_m * U * kWave * sizeof(double) : 0;
  if (nw == 1 && !m->tree) pair_bytes += (size_t)inverse_lds_doubles(m->max_frames) * sizeof(double);
  const dim3 grid(m->n_models), block(nw * kWave);
#define ABD_HOC(NW, TREE, UU)                                                                  \
  do {                                                                                         \
    HocArgs<UU> a;                                                                             \
    if ((rc = fill_hoc_args<UU>(m, o, a, sc))) return rc;                                      \
    a.n_steps = n_steps; a.q_prev = q_prev; a.q_curr = q_curr; a.tau = tau; a.q_out = q_out;   \
    a.stats = stats;                                                                           \
    if (o->precision == ABD_MIXED)                                                             \
      hipLaunchKernelGGL((k_rollout_hoc<NW, TREE, UU, ABD_MIXED>), grid, block, pair_bytes, s, a); \
    else                                                                                       \
      hipLaunchKernelGGL((k_rollout_hoc<NW, TREE, UU>), grid, block, pair_bytes, s, a);        \
  } while (0)
#define ABD_HOC_U(NW, TREE) \
  do {                      \
    if (U == 2)             \
      ABD_HOC(NW, TREE, 2); \
    else                    \
      ABD_HOC(NW, TREE, 3); \
  } while (0)
  if (m->tree) {
    if (nw == 1) ABD_HOC_U(1, true);
    else if (nw == 2) ABD_HOC_U(2, true);
    else ABD_HOC_U(4, true);
  } else {
    if (nw == 1) ABD_HOC_U(1, false);
    else if (nw == 2) ABD_HOC_U(2, false);
    else ABD_HOC_U(4, false);
  }
#undef ABD_HOC_U
#undef ABD_HOC
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

int launch_hoc_objective(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist,
                         const double* tau, double* E, double* grad, double* grad_tau, void* stream) {
  int rc = check_hoc(m, o);
  if (rc) return rc;
  const int U = o->order_K - 1;
  HocObjArgs h;
  HocArgs<3> tmp;
  if ((rc = fill_hoc_args<3>(m, o, tmp))) return rc;  // allocates the scratch
  double tau_pts[5], w[15];
  hoc_collocation(o->order_K, tau_pts, w);
  h.d = dev_view(m);
  h.dt2 = o->dt * o->dt;
  for (int u = 0; u < 3; ++u)
    for (int p = 0; p < 5; ++p) h.w[u][p] = (u < U && p < U + 2) ? w[u * (U + 2) + p] : 0.0;
  h.q_prev = q_hist;
  h.q_curr = q_hist + m->n_dofs;
  h.q = q;
  h.tau = tau;
  h.E = E;
  h.grad = grad;
  h.grad_tau = grad_tau;
  h.Bk = m->Bk;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nw = waves_for(m->max_frames);
  const dim3 grid(m->n_models), block(nw * kWave);
  const bool f32 = o->precision == ABD_MIXED;  // float32 kinematics
#define ABD_HOCOBJ(NW, TREE)                                                              \
  do {                                                                                    \
    if (U == 2 && f32)                                                                    \
      hipLaunchKernelGGL((k_hoc_objective<NW, TREE, 2, float>), grid, block, 0, s, h);    \
    else if (U == 2)                                                                      \
      hipLaunchKernelGGL((k_hoc_objective<NW, TREE, 2>), grid, block, 0, s, h);           \
    else if (f32)                                                                         \
      hipLaunchKernelGGL((k_hoc_objective<NW, TREE, 3, float>), grid, block, 0, s, h);    \
    else                                                                                  \
      hipLaunchKernelGGL((k_hoc_objective<NW, TREE, 3>), grid, block, 0, s, h);           \
  } while (0)
  if (m->tree) {
    if (nw == 1) ABD_HOCOBJ(1, true);
    else if (nw == 2) ABD_HOCOBJ(2, true);
    else ABD_HOCOBJ(4, true);
  } else {
    if (nw == 1) ABD_HOCOBJ(1, false);
    else if (nw == 2) ABD_HOCOBJ(2, false);
    else ABD_HOCOBJ(4, false);
  }
#undef ABD_HOCOBJ
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

}  // namespace abd_impl
