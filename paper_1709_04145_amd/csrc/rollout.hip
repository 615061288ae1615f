// rollout.hip -- the order-2 step kernel (Sec. 4 Eq. EQ, Sec. 5 L-BFGS) and its launch.
#include "abd_device.h"

namespace {

// FX: models with slides, drag or contact points (the terms of Sec. 6's
// applications; a separate instantiation, so that the others carry none of it).
// SEG < 64: one-wave chains packed kWave / SEG per wavefront, model b of the
// dispatch order in segment b % (kWave / SEG) of workgroup b / (kWave / SEG);
// each segment runs its model's steps on its own (the segments branch apart).
template <int NW, int PREC, bool TREE, bool FX = false, int SEG = kWave>
__global__ void __launch_bounds__(NW* kWave, (NW >= 4 ? 1 : kWavesPerSimd)) k_rollout(StepArgs args) {
  static_assert(SEG == kWave || (NW == 1 && !TREE), "packed models are one-wave chains");
  constexpr int SEGS = kWave / SEG;  // models per wavefront
  // chains of one wavefront each: the recursion's table in the dynamic LDS, so
  // that all of it is sized to the batch's largest model
  constexpr bool kDynTab = NW == 1 && !TREE && SEGS == 1;
  __shared__ RollLds<NW, TREE, SEGS, !kDynTab> L;
  __shared__ ChainLds<(NW > 1 && !TREE)> CL;
  // one-wave models: L-BFGS pairs of the current step, s in ring slots [0, m),
  // y in [m, 2m), ps doubles per slot (one per frame of the batch's largest
  // model for chains of one wavefront each, else one per lane); one-wave
  // chains: then the explicit inverse (chain_lds_doubles(nfmax); packed
  // float64, or the full float32 matrix for MIXED) and the recursion's table
  // (nfmax rows, at least 64 doubles), or per segment of packed models
  // tile_inverse_doubles(SEG) each
  extern __shared__ double pairs[];
  const DevModel& d = args.d;
  const int n = d.n_dofs;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int seg = SEGS > 1 ? lane / SEG : 0;
  const int j = SEGS > 1 ? lane % SEG : (int)threadIdx.x;  // frame of this thread within its model
  const int jl = SEGS > 1 ? j : lane;                       // its lane in the one-wave helpers
  const int ps = kDynTab ? args.nfmax : kWave;
  double* const hl = pairs + 2 * args.m * ps + (SEGS > 1 ? seg * tile_inverse_doubles(SEG) : 0);
  double* const rho = L.rho + seg * kMaxHist;
  double* const alp = L.alp + seg * kMaxHist;
  double (*const tab)[kTab] =
      kDynTab ? reinterpret_cast<double (*)[kTab]>(hl + chain_lds_doubles(args.nfmax)) : L.tab + seg * SEG;
  const bool lead = j == 0;
  const int mslot = blockIdx.x * SEGS + seg;
  const bool has_model = mslot < d.n_models;
  if (!has_model) return;
  const int model = d.order[mslot];
  const int f0 = d.f0[model];
  const int nf = d.f0[model + 1] - f0;
  if (nf == 0) {  // a model without frames: every step is trivially converged
    if (lead && args.stats)
      for (int k = 0; k < args.n_steps; ++k) {
        abd_step_stats st = {0, 0, ABD_FLAG_CONVERGED, 0, 0, 0, 0.0, 0.0};
        args.stats[(size_t)k * d.n_models + model] = st;
      }
    return;
  }
  const bool valid = j < nf;
  const int f = f0 + (valid ? j : 0);  // invalid lanes alias frame 0 of the model (loads stay in bounds)
  auto sc = [&]() {
    if constexpr (SEGS > 1) return SegScan<SEG>{j};
    else return ModelScan<NW, TREE>::make(L, d, wave, lane, j, f, valid);
  }();
  const int io = TREE ? (valid ? d.uidx[f] : 0) : f;  // index of this frame's DOF in the caller's vectors
  const bool use_aba = args.precond == ABD_PRECOND_INERTIA;
  // one-wave chains: explicit inverse; otherwise inertias [nf][10] (then, for
  // branched models, the recursion's accumulators [nf][21])
  double* Hi = d.hinv + d.hoff[model];
  const int fend_j = TREE && valid ? d.fend[f] : j;  // the last frame below this one
  const int hj = TREE && valid ? d.fheight[f] : 0;    // the longest path below this frame
  const FrameGeo geo = load_geo<FX>(d, f, valid);
  const double eps_w = PREC == ABD_MIXED ? 5.9604644775390625e-8 : 1.1102230246251565e-16;
  const double c1 = 1e-4, dlt = 0.1;

  // q_{k-1} and q_k of the current step
  double qkm1 = ld_if(args.q_prev + io, valid);
  double qk = ld_if(args.q_curr + io, valid);
  int step = 0;
  int state = args.n_steps > 0 ? kSetup : kDone;

  // per-step solver state
  double* hs;
  int hstride, ys;
  if (NW == 1) {
    hs = pairs + lane;
    hstride = ps;
    ys = args.m * ps;
  } else {
    hs = d.hist + (size_t)f * (2 * kMaxHist);
    hstride = 1;
    ys = kMaxHist;
  }
  bool f32 = false, reset = false;
  // set when the float32 inverse is no descent preconditioner at the iterate:
  // the step then continues with H0 = gamma I until the next formation
  bool h0_plain = false;
  // MIXED: re-evaluate at the iterate in float64 before the next direction (set
  // when float32 has done what it can, and at the step's first re-formation)
  bool to64 = false;
  int iters = 0, evals = 0, flag = 0, f32_iters = 0, f32_evals = 0, count = 0, head = 0, refreshed = 0;
  double q = 0.0, tau = 0.0, E = 0.0, g = 0.0, g0 = 0.0, gn = 0.0, gam = 1.0;
#ifdef ABD_PROFILE
  if (lead && abd_prof) abd_prof[(size_t)model * 16 + 10] = __builtin_amdgcn_s_memrealtime();
#endif
  bool inv32 = false;  // MIXED, one-wave chains: the explicit inverse is the float32 matrix
  // the recursion's tables (and, for one-wave chains, the explicit inverse) once
  // every frame has written its inputs
  auto factor_precond = [&]() {
    if (NW > 1) __threadfence_block();  // inertias go through device memory
    __syncthreads();
    PROF_T(t_r);
    if constexpr (TREE) {
      aba_setup_tree_levels(NW == 1 ? &L.inert[0][0] : Hi, tab, d.fend + f0, Hi + 10 * (size_t)nf, j, valid, hj,
                            d.mheight[model]);
    } else if constexpr (NW > 1) {
      aba_setup_rows_staged<NW>(Hi, tab, nf, j, CL.stg);
    } else {
      if (wave == 0) aba_setup_rows<SEG>(hl, tab, nf, jl);
    }
    __syncthreads();
    if (TREE) {
      // the explicit L^-1 of the recursion, one column per frame's thread
      tree_inverse_factor(tab, L.tpar, d.wrow + f0, Hi + 31 * (size_t)nf, j, valid);
      __threadfence_block();
      __syncthreads();
    }
    PROF_ADD(2, t_r);
    PROF_T(t_i);
    if (NW == 1 && !TREE) {
      if (PREC == ABD_MIXED) {
        // float32 inverse only while the pivots D_f span at most kInv32MaxRatio
        float lo = (float)tab[jl < nf ? jl : 0][12], hi = lo;  // 1/D_f
#pragma unroll
        for (int o = SEG / 2; o > 0; o >>= 1) {
          lo = fminf(lo, __shfl_xor(lo, o));
          hi = fmaxf(hi, __shfl_xor(hi, o));
        }
        if (SEGS > 1)
          inv32 = hi <= kInv32MaxRatio * lo;
        else
          inv32 = __builtin_amdgcn_readfirstlane((int)(hi <= kInv32MaxRatio * lo)) != 0;
      }
      // overwrites the inertias
      if (inv32)
        aba_inverse_f32<SEG>(tab, nf, jl, reinterpret_cast<float*>(hl));
      else
        aba_inverse<SEG>(tab, nf, jl, hl);
      __syncthreads();  // every lane reads the other lanes' columns
    }
    PROF_ADD(3, t_i);
  };
  // frames' inertias: lanes without a frame of a multi-wave model write their
  // (zero) record to a sink, never to frame 0's slot, which lane 0 fills; so do
  // the lanes past the model's frames of chains of one wavefront each, with
  // their table rows, which have no place in the LDS sized to the batch (the
  // recursion reads the model's frames only)
  __shared__ double inert_sink[10];
  __shared__ double tab_sink[kTab];
  double* const inert = NW == 1 ? (TREE ? L.inert[lane] : ((kDynTab && !valid) ? inert_sink : hl + 10 * jl))
                                : (valid ? Hi + (size_t)j * 10 : inert_sink);
  double* const tab_j = (kDynTab && !valid) ? tab_sink : tab[j];

  while (state != kDone) {
    bool step_done = false;
    if (state == kSetup) {
      PROF_T(t_s);
      q = valid ? 2.0 * qk - qkm1 : 0.0;  // warm start: constant-velocity extrapolation
      tau = (valid && args.tau) ? args.tau[(size_t)step * n + io] : 0.0;
      f32 = PREC == ABD_MIXED;
      iters = 0; evals = 0; flag = 0; f32_iters = 0; f32_evals = 0; count = 0; head = 0; refreshed = 0;
      reset = false; gam = 1.0;
      h0_plain = false;
      to64 = false;
      if (nf == 0) {
        flag = ABD_FLAG_CONVERGED;
        step_done = true;
      } else {
        step_setup<FX>(sc, d, inert, tab_j, geo, f, valid, qkm1, qk, q, use_aba);
        if (use_aba) factor_precond();
        PROF_ADD(0, t_s);
        const EvalResult r = (PREC == ABD_MIXED) ? evaluate<float, FX>(sc, d, geo, f, valid, q, tau, args.dt2)
                                                  : evaluate<double, FX>(sc, d, geo, f, valid, q, tau, args.dt2);
        ++evals;
        if (PREC == ABD_MIXED) ++f32_evals;
        E = r.E;
        g = r.g;
        gn = 0.0;
        if (!isfinite(E) || !sc.all_finite(g)) {
          flag = ABD_FLAG_NONFINITE;
          step_done = true;
        } else {
          g0 = sc.uniform(sqrt(sc.sum(g * g)));
          gn = g0;
          if (g0 == 0.0) {
            flag = ABD_FLAG_CONVERGED;
            step_done = true;
          } else if (args.max_iter <= 0) {
            flag = ABD_FLAG_MAX_ITER;
            step_done = true;
          } else {
            state = kIterate;
          }
        }
      }
    } else {
      if (use_aba && args.refresh > 0 && iters > 0 && iters % args.refresh == 0 && iters != refreshed) {
        // the inertia of the warm start no longer describes the iterate: re-form
        // the preconditioner at q and restart the curvature history
        refreshed = iters;
        PROF_T(t_f);
        precond_frame<FX>(sc, d, inert, tab_j, geo, f, valid, q);
        factor_precond();
        count = 0;
        head = 0;
        h0_plain = false;
        if (PREC == ABD_MIXED && f32) to64 = true;
        PROF_ADD(4, t_f);
#ifdef ABD_PROFILE
        if (lead && abd_prof) abd_prof[(size_t)model * 16 + 8] += 1;
#endif
      }
      if (PREC == ABD_MIXED && to64) {
        // leave float32: re-evaluate at q in float64 (right after a re-formation,
        // or where float32 converged, met its rounding or stalled the search)
        to64 = false;
        f32 = false;
        const EvalResult r = evaluate<double, FX>(sc, d, geo, f, valid, q, tau, args.dt2);
        ++evals;
        E = r.E;
        g = r.g;
        gn = sc.uniform(sqrt(sc.sum(g * g)));
        if (gn <= args.tol * g0) {
          flag = ABD_FLAG_CONVERGED;
          step_done = true;
        } else if (iters >= args.max_iter) {
          flag = ABD_FLAG_MAX_ITER;
          step_done = true;
        }
      }
      PROF_T(t_a);
      if (!step_done) {
        // ---- two-loop recursion: newest pair first; the next pair is requested
        // while the current one is used
        if (reset) count = 0;
        double qv = g;
        {
          double sk = ld_if(hs + head * hstride, valid && count > 0);
          double yk = ld_if(hs + ys + head * hstride, valid && count > 0);
          for (int k = 0; k < count; ++k) {
            const int nxt = (head - k - 1 + args.m) % args.m;
            const double sn = ld_if(hs + nxt * hstride, valid && k + 1 < count);
            const double yn = ld_if(hs + ys + nxt * hstride, valid && k + 1 < count);
            // the reduction (a barrier for several waves) before the LDS read of
            // rho, which the lead lane writes when the pair is accepted
            const double sq = sc.sum(sk * qv);
            const double a_k = sc.uniform(rho[(head - k + args.m) % args.m] * sq);
            if (lead) alp[k] = a_k;
            qv -= a_k * yk;
            sk = sn;
            yk = yn;
          }
        }
        // ---- initial inverse Hessian
        double r;
        if (!use_aba || h0_plain) {
          r = (count > 0 ? gam : 1.0) * qv;
        } else if (NW == 1 && !TREE) {
          PROF_T(t_h);
          // the recursion's table is free between formations
          // the vector goes through the recursion's table, which is free between
          // formations (packed models: through an area of its own per segment)
          double* const vb = SEGS > 1 ? L.vb + seg * SEG : &tab[0][0];
          r = inv32 ? apply_inverse_f32<SEG>(reinterpret_cast<const float*>(hl), reinterpret_cast<float*>(vb), nf, jl, qv)
                    : apply_inverse<SEG>(hl, vb, nf, jl, qv);
          PROF_ADD(14, t_h);
        } else if (TREE) {
          r = tree_apply_inverse(tab, L.tpar, d.wrow + f0, Hi + 31 * (size_t)nf, L.xb, &L.acc[0][0], j, fend_j, valid,
                                 qv);
        } else {
          L.xb[j] = valid ? qv : 0.0;
          __syncthreads();
          chain_solve<NW>(tab, L.xb, CL.sgm, CL.sgin, nf, j);
          r = ld_if(&L.xb[j], valid);
        }
        PROF_ADD(1, t_a);
        PROF_T(t_c);
        PROF_T(t_l);
        // ---- oldest pair first
        {
          int slot = (head - (count - 1) + args.m) % args.m;
          double sk = ld_if(hs + slot * hstride, valid && count > 0);
          double yk = ld_if(hs + ys + slot * hstride, valid && count > 0);
          for (int k = count - 1; k >= 0; --k) {
            const int nxt = (slot + 1) % args.m;
            const double sn = ld_if(hs + nxt * hstride, valid && k > 0);
            const double yn = ld_if(hs + ys + nxt * hstride, valid && k > 0);
            const double yr = sc.sum(yk * r);
            const double b = sc.uniform(rho[slot] * yr);
            r += (alp[k] - b) * sk;
            sk = sn;
            yk = yn;
            slot = nxt;
          }
        }
        const double dir = valid ? -r : 0.0;
        const double gd = sc.uniform(sc.sum(g * dir));
        PROF_ADD(12, t_l);
        if (!(gd < 0.0)) {
          if (!reset) {
            reset = true;  // redo the direction with an empty history
          } else if (inv32 && !h0_plain) {
            h0_plain = true;  // -H0 g is no descent direction either
          } else if (PREC == ABD_MIXED && f32) {
            to64 = true;  // the float32 gradient gives no descent direction: go on in float64
            reset = false;
            h0_plain = false;
          } else {
            flag = ABD_FLAG_LS_FLOOR;
            step_done = true;
          }
        } else {
          reset = false;
          double alpha = 1.0;
          int ls = 0;
          bool noisy = false;
          for (;;) {
            const double x = q + alpha * dir;
            EvalResult rt;
            PROF_T(t_e);
            // the first trial of an iteration (usually accepted) is evaluated
            // with its gradient, later ones with it only where an acceptance
            // test below reads it (the same values either way)
            const bool full = ls == 0;
            const double bound = E + c1 * alpha * gd, tol_s = 10.0 * eps_w;
            if (PREC == ABD_MIXED && f32) {
              rt = full ? evaluate<float, FX>(sc, d, geo, f, valid, x, tau, args.dt2)
                        : evaluate<float, FX, true>(sc, d, geo, f, valid, x, tau, args.dt2, bound, E, tol_s);
              ++f32_evals;
            } else {
              rt = full ? evaluate<double, FX>(sc, d, geo, f, valid, x, tau, args.dt2)
                        : evaluate<double, FX, true>(sc, d, geo, f, valid, x, tau, args.dt2, bound, E, tol_s);
            }
            PROF_ADD(6, t_e);
  #ifdef ABD_PROFILE
            if (lead && abd_prof) abd_prof[(size_t)model * 16 + 7] += 1;
  #endif
            ++evals;
            int ok = 0;
            if (isfinite(rt.E) && sc.all_finite(rt.g)) {
              if (rt.E <= E + c1 * alpha * gd) {
                ok = 1;
              } else if (fabs(rt.E - E) <= 10.0 * eps_w * rt.S) {
                noisy = true;
                const double gtd = sc.sum(rt.g * dir);
                if (gtd <= (2.0 * dlt - 1.0) * gd) ok = 1;
              }
            }
            if (!ok) {
              alpha = next_alpha(alpha, E, rt.E, gd);
              if (++ls < args.max_ls) continue;
              if (PREC == ABD_MIXED && f32) {
                to64 = true;  // float32 rounding stalls the search: continue in float64 from q
                break;
              }
              flag = ABD_FLAG_LS_FLOOR;
              step_done = true;
              break;
            }
            // an accepted trial point that equals q in every coordinate is no
            // progress: at this precision the iteration cannot move any more
            if (sc.uniform(sc.sum(valid && x != q ? 1.0 : 0.0)) == 0.0) {
              if (PREC == ABD_MIXED && f32) {
                to64 = true;
                break;
              }
              flag = ABD_FLAG_LS_FLOOR;
              step_done = true;
              break;
            }
            // accepted: curvature pair (the step actually taken) and update
            PROF_T(t_u);
            const double sv = x - q;
            const double y = rt.g - g;
            double sy = sv * y, ss = sv * sv, yy = y * y, gg = rt.g * rt.g;
            sc.sum2(sy, ss);
            sc.sum2(yy, gg);
            if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
              gam = sc.uniform(sy / yy);
              head = count == 0 ? 0 : (head + 1) % args.m;
              if (lead) rho[head] = 1.0 / sy;  // rho lives in the ring slot of its pair
              if (valid) {
                hs[head * hstride] = sv;
                hs[ys + head * hstride] = y;
              }
              if (count < args.m) ++count;
            }
            q = x;
            g = rt.g;
            E = rt.E;
            ++iters;
            if (PREC == ABD_MIXED && f32) ++f32_iters;
            gn = sc.uniform(sqrt(gg));
            PROF_ADD(13, t_u);
            const bool conv = gn <= args.tol * g0;
            if (PREC == ABD_MIXED && f32 && (conv || noisy)) {
              to64 = true;  // float32 has done what it can: confirm / continue in float64
              break;
            }
            if (conv) {
              flag = ABD_FLAG_CONVERGED;
              step_done = true;
            } else if (iters >= args.max_iter) {
              flag = ABD_FLAG_MAX_ITER;
              step_done = true;
            }
            break;
          }
        }
        PROF_ADD(5, t_c);
      }
#ifdef ABD_PROFILE
      if (lead && abd_prof) abd_prof[(size_t)model * 16 + 9] += 1;
#endif
    }
    if (step_done) {
      if (valid) args.q_out[(size_t)step * n + io] = q;
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
      qkm1 = qk;
      qk = q;
      ++step;
      state = step < args.n_steps ? kSetup : kDone;
    }
  }
#ifdef ABD_PROFILE
  if (lead && abd_prof) abd_prof[(size_t)model * 16 + 11] = __builtin_amdgcn_s_memrealtime();
#endif
}

}  // namespace

namespace abd_impl {

// Segment width of the packed (TILE) schedule for this batch: serial chains of
// at most 16 or 32 DOFs; 0 where the batch cannot be packed.
static int tile_segment(const abd_model* m) {
  if (m->tree || m->max_frames <= 0 || m->max_frames > 32) return 0;
  return m->max_frames <= 16 ? 16 : 32;
}

// One launch of the order-2 rollout: seg = 0 one model per workgroup (WAVE),
// 16 or 32 packed models of that many lanes (TILE).
static int dispatch_rollout(const abd_model* m, const abd_step_opts* o, const StepArgs& a, int seg,
                            hipStream_t s) {
  const int nw = waves_for(m->max_frames);
  const bool f64 = o->precision == ABD_FP64;
  if (seg > 0) {
    const int segs = kWave / seg;
    const dim3 grid((m->n_models + segs - 1) / segs), block(kWave);
    const size_t bytes = (2 * (size_t)o->lbfgs_m * kWave + (size_t)segs * tile_inverse_doubles(seg)) * sizeof(double);
#define ABD_TILE(S, FXV)                                                                              \
  do {                                                                                                \
    if (f64)                                                                                          \
      hipLaunchKernelGGL((k_rollout<1, ABD_FP64, false, FXV, S>), grid, block, bytes, s, a);         \
    else                                                                                              \
      hipLaunchKernelGGL((k_rollout<1, ABD_MIXED, false, FXV, S>), grid, block, bytes, s, a);        \
  } while (0)
    if (m->fx) {
      if (seg == 16) ABD_TILE(16, true);
      else ABD_TILE(32, true);
    } else {
      if (seg == 16) ABD_TILE(16, false);
      else ABD_TILE(32, false);
    }
#undef ABD_TILE
    HIP_TRY(hipGetLastError());
    return ABD_OK;
  }
  const dim3 grid(m->n_models), block(nw * kWave);
  // one-wave models: the L-BFGS pairs; chains: per frame of the largest model,
  // then the explicit inverse and the recursion's table (at least 64 doubles:
  // it also carries the vector of the inverse product)
  size_t pair_bytes = 0;
  if (nw == 1 && m->tree) pair_bytes = 2 * (size_t)o->lbfgs_m * kWave * sizeof(double);
  if (nw == 1 && !m->tree) {
    const int nf = m->max_frames;
    pair_bytes = (2 * (size_t)o->lbfgs_m * nf + chain_lds_doubles(nf) + (kTab * nf > kWave ? kTab * nf : kWave)) *
                 sizeof(double);
  }
#define ABD_LAUNCH(NW, TREE)                                                                \
  do {                                                                                      \
    if (f64)                                                                                \
      hipLaunchKernelGGL((k_rollout<NW, ABD_FP64, TREE>), grid, block, pair_bytes, s, a);   \
    else                                                                                    \
      hipLaunchKernelGGL((k_rollout<NW, ABD_MIXED, TREE>), grid, block, pair_bytes, s, a);  \
  } while (0)
#define ABD_LAUNCH_FX(NW, TREE)                                                                   \
  do {                                                                                            \
    if (f64)                                                                                      \
      hipLaunchKernelGGL((k_rollout<NW, ABD_FP64, TREE, true>), grid, block, pair_bytes, s, a);   \
    else                                                                                          \
      hipLaunchKernelGGL((k_rollout<NW, ABD_MIXED, TREE, true>), grid, block, pair_bytes, s, a);  \
  } while (0)
  if (m->fx) {  // at most 256 frames per model (checked when the model is created)
    if (m->tree) {
      if (nw == 1) ABD_LAUNCH_FX(1, true);
      else if (nw == 2) ABD_LAUNCH_FX(2, true);
      else ABD_LAUNCH_FX(4, true);
    } else {
      if (nw == 1) ABD_LAUNCH_FX(1, false);
      else if (nw == 2) ABD_LAUNCH_FX(2, false);
      else ABD_LAUNCH_FX(4, false);
    }
  } else if (m->tree) {
    switch (nw) {
      case 1: ABD_LAUNCH(1, true); break;
      case 2: ABD_LAUNCH(2, true); break;
      default: ABD_LAUNCH(4, true); break;
    }
  } else {
    switch (nw) {
      case 1: ABD_LAUNCH(1, false); break;
      case 2: ABD_LAUNCH(2, false); break;
      case 4: ABD_LAUNCH(4, false); break;
      case 8: ABD_LAUNCH(8, false); break;
      default: ABD_LAUNCH(16, false); break;
    }
  }
#undef ABD_LAUNCH
#undef ABD_LAUNCH_FX
  HIP_TRY(hipGetLastError());
  return ABD_OK;
}

// The schedule autotuner: times the first steps (up to 8) of this very call
// under WAVE and under TILE (each run three times, the best of the last two
// counted, outputs into the model's scratch trajectory, no stats),
// synchronizing the stream, and keeps the faster for the model handle and
// precision.  Both schedules give the same bits, so the choice changes only the
// time.
static int autotune_schedule(abd_model* m, const abd_step_opts* o, const StepArgs& a, hipStream_t s, int& choice) {
  const int T = a.n_steps < 8 ? a.n_steps : 8;
  const size_t need = (size_t)T * m->n_dofs;
  if (m->tune_len < need) {
    void* p = nullptr;
    int rc = model_alloc(m, &p, need * sizeof(double));
    if (rc) return rc;
    m->tune_buf = static_cast<double*>(p);
    m->tune_len = need;
  }
  StepArgs t = a;
  t.n_steps = T;
  t.q_out = m->tune_buf;
  t.stats = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(ABD_EDEVICE, "hipEventCreate failed");
  }
  const int cands[2] = {0, tile_segment(m)};
  float best_ms = 0.0f;
  int best = 0, rc = ABD_OK;
  for (int c = 0; c < 2 && rc == ABD_OK; ++c)
    for (int rep = 0; rep < 3 && rc == ABD_OK; ++rep) {
      float ms = 0.0f;
      if (hipEventRecord(e0, s) != hipSuccess || (rc = dispatch_rollout(m, o, t, cands[c], s)) != ABD_OK ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        if (rc == ABD_OK) rc = fail(ABD_EDEVICE, "timing the schedules failed");
        break;
      }
      if (rep > 0 && ((c == 0 && rep == 1) || ms < best_ms)) {
        best_ms = ms;
        best = cands[c];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == ABD_OK) choice = best;
  return rc;
}

int launch_rollout(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
                   const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream,
                   const StepScratch* sc) {
  StepArgs a;
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
  a.refresh = o->refresh;
  a.n_steps = n_steps;
  a.nfmax = m->max_frames;
  a.q_prev = q_prev;
  a.q_curr = q_curr;
  a.tau = tau;
  a.q_out = q_out;
  a.stats = stats;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int seg = 0;
  if (o->schedule == ABD_SCHEDULE_TILE) {
    seg = tile_segment(m);
    if (!seg) return fail(ABD_ENOTSUP, "ABD_SCHEDULE_TILE packs serial chains of at most 32 DOFs");
  } else if (o->schedule == ABD_SCHEDULE_AUTO && tile_segment(m)) {
    int& choice = m->tile_choice[o->precision == ABD_MIXED ? 1 : 0];
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    // callers that cannot allocate or synchronize (a given scratch, graph
    // capture) take the decision already made, else WAVE
    if (choice < 0 && !sc && cs == hipStreamCaptureStatusNone) {
      int rc = autotune_schedule(m, o, a, s, choice);
      if (rc) return rc;
    }
    seg = choice > 0 ? choice : 0;
  }
  return dispatch_rollout(m, o, a, seg, s);
}

}  // namespace abd_impl

#ifdef ABD_PROFILE
// Profiling builds only: device buffer of 16 counters per model.
extern "C" int abd_debug_set_profile_buffer(unsigned long long* dev_ptr) {
  HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(abd_prof), &dev_ptr, sizeof(dev_ptr)));
  return ABD_OK;
}
#endif
