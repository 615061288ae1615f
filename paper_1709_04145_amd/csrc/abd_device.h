// abd_device.h -- device code shared by the kernels of the library (gfx950).
//
// Position-based articulated dynamics (Pan & Manocha): every time step solves
// q_{k+1} = argmin E(q) (Sec. 4, Eq. EQ, scaled by dt^2) with a quasi-Newton
// method (Sec. 5).  Per evaluation the hot path is
//   1. forward kinematics A_l = A_parent T_l(q_l)      (Alg. 1 forward pass)
//   2. per-link energy terms and the seed dE/dA_l      (Eq. EQ with Eq. ATOM)
//   3. the adjoint backward pass giving dE/dq          (Alg. 1 backward pass)
// and per iteration the two-loop L-BFGS direction and a backtracking line search.
//
// Layout on the GPU.  A model is a tree (usually a serial chain) of elementary
// hinge "frames" (one per DOF; a ball joint is three consecutive hinges with
// massless intermediate frames).  One workgroup owns one model (one wavefront
// up to 64 frames, 2..16 beyond) and lane j owns frame j:
//   * FK is an inclusive prefix scan of 3x4 rigid transforms over the lanes
//     (DPP row shifts + row broadcasts: 6 levels for 64 lanes);
//   * the adjoint backward pass is evaluated in the world frame: with
//     G_l = dE/dA_l, k_l = sum_c R_l[:,c] x G_l[:,c] + t_l x G_l[:,3] and
//     f_l = G_l[:,3], the derivative is g_n = w_n . (K_n - p_n x F_n) where
//     (K_n, F_n) are suffix sums over the frames below n, w_n the world hinge
//     axis and p_n the world joint point.  This is the same quantity as the
//     4x4 body-frame recursion of Alg. 1 (A <- (A + dI/dT) t^T), rewritten as
//     a plain sum so that it becomes a float64 suffix scan;
//   * L-BFGS dot products are float64 wave reductions.
// The initial inverse Hessian of L-BFGS is the inverse joint-space inertia,
// formed at the warm start and again at the iterate every `refresh` iterations.
// The articulated-body recursion factors it (sequential along the chain, its
// 6x6 algebra spread over six lanes, tables in LDS) and, for one-wave chains,
// the 64 lanes solve for the columns of the explicit inverse at once and keep
// it in LDS (a packed float64 triangle; the full matrix in float32 for mixed
// precision); every iteration then applies it as a matrix-vector product, so
// the iteration has no sequential sweep.  Models never
// wait for each other, and the L-BFGS pairs live in LDS.
//
// No MFMA: nothing on this path is a dense contraction.

#pragma once
#include "abd_internal.h"

#include <cmath>
#include <cstdint>

namespace {

constexpr int kWave = 64;
constexpr int kMaxFrames = 64;  // frames (DOFs) per wavefront
constexpr int kMaxWaves = 16;   // wavefronts per model (at most 1024 frames)
constexpr int kMaxHist = 10;    // longest L-BFGS history
constexpr int kTab = 13;        // recursion record per frame: s (6), U (6), 1/D

// Optional per-phase cycle counters (build with -DABD_PROFILE): lane 0 of every
// model wave accumulates s_memtime deltas into abd_prof[model][slot]; nothing is
// recorded while no buffer is set (abd_prof null).
#ifdef ABD_PROFILE
__device__ unsigned long long* abd_prof;
#define PROF_T(var) unsigned long long var = __builtin_readcyclecounter()
#define PROF_ADD(slot, t0)                                                          \
  do {                                                                              \
    if (threadIdx.x == 0 && has_model && abd_prof)                                  \
      abd_prof[(size_t)model * 16 + (slot)] += __builtin_readcyclecounter() - (t0); \
  } while (0)
#else
#define PROF_T(var)
#define PROF_ADD(slot, t0)
#endif

// ------------------------------------------------------------------ DPP --
// update_dpp keeps `old` in lanes whose source is out of the row (bound_ctrl
// off) or whose row is masked off.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp(double old, double v) {
  const long long o = __double_as_longlong(old), x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(x & 0xffffffffll), CTRL,
                                             ROW_MASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(x >> 32), CTRL, ROW_MASK, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Zero-filling row shift (all rows enabled): lanes whose source lies outside the
// row read 0, so no "old" value has to be materialised.
template <int CTRL>
__device__ __forceinline__ float dpp0(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp0(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffll), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Keep a wave-uniform double in scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(x & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_uniform(double v) { return uniform(v); }

// Inclusive prefix sum over the 64 lanes (row shifts 1,2,4,8, then the
// row-15 and row-31 broadcasts).  Every lane ends with its inclusive prefix.
__device__ __forceinline__ double wave_prefix_sum(double v) {
  v += dpp0<0x111>(v);
  v += dpp0<0x112>(v);
  v += dpp0<0x114>(v);
  v += dpp0<0x118>(v);
  v += dpp<0x142, 0xA>(0.0, v);
  v += dpp<0x143, 0xC>(0.0, v);
  return v;
}
__device__ __forceinline__ double wave_sum(double v) { return readlane(wave_prefix_sum(v), 63); }

// Two independent sums in one pass (interleaved for latency hiding).
__device__ __forceinline__ void wave_sum2(double& a, double& b) {
  a += dpp0<0x111>(a); b += dpp0<0x111>(b);
  a += dpp0<0x112>(a); b += dpp0<0x112>(b);
  a += dpp0<0x114>(a); b += dpp0<0x114>(b);
  a += dpp0<0x118>(a); b += dpp0<0x118>(b);
  a += dpp<0x142, 0xA>(0.0, a); b += dpp<0x142, 0xA>(0.0, b);
  a += dpp<0x143, 0xC>(0.0, a); b += dpp<0x143, 0xC>(0.0, b);
  a = readlane(a, 63);
  b = readlane(b, 63);
}

// Load *p on every lane and keep it where c holds (0 elsewhere).  The address
// must be valid on every lane (callers clamp indices to the model's frames), so
// the load is unconditional and needs no execution-mask branch.
template <typename T>
__device__ __forceinline__ T ld_if(const T* p, bool c) {
  const T x = *p;
  return c ? x : T(0);
}

// ------------------------------------------------------------ transforms --
// 3x4 rigid transform [R|t], row-major: m[4r+c].
template <typename R>
struct Xf {
  R m[12];
};

// Unit quaternion (w, x, y, z) of a rotation.
template <typename R>
struct Quat {
  R w, x, y, z;
};

// a (x) b : rotation b followed, in the frame of a, i.e. R(a) R(b)
template <typename R>
__device__ __forceinline__ Quat<R> qmul(const Quat<R>& a, const Quat<R>& b) {
  Quat<R> c;
  c.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
  c.x = a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y;
  c.y = a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x;
  c.z = a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w;
  return c;
}

template <typename R, int CTRL, int ROW_MASK>
__device__ __forceinline__ Quat<R> dpp_quat(const Quat<R>& v) {
  Quat<R> y;
  y.w = dpp<CTRL, ROW_MASK>(R(1), v.w);
  if constexpr (ROW_MASK == 0xF) {
    // every row enabled: only lanes without a source take the identity, whose
    // vector part the zero fill supplies without a materialised old value
    y.x = dpp0<CTRL>(v.x);
    y.y = dpp0<CTRL>(v.y);
    y.z = dpp0<CTRL>(v.z);
  } else {
    y.x = dpp<CTRL, ROW_MASK>(R(0), v.x);
    y.y = dpp<CTRL, ROW_MASK>(R(0), v.y);
    y.z = dpp<CTRL, ROW_MASK>(R(0), v.z);
  }
  return y;
}

// Q_j = r_0 (x) r_1 (x) ... (x) r_j over the lanes: the rotation part of Alg. 1's
// forward pass T^j = T^{j-1} t_j as an inclusive prefix scan (row shifts 1,2,4,8,
// then row broadcasts 15 and 31; the identity fills lanes without a source).
template <typename R>
__device__ __forceinline__ Quat<R> wave_prefix_quat(Quat<R> v) {
  v = qmul(dpp_quat<R, 0x111, 0xF>(v), v);
  v = qmul(dpp_quat<R, 0x112, 0xF>(v), v);
  v = qmul(dpp_quat<R, 0x114, 0xF>(v), v);
  v = qmul(dpp_quat<R, 0x118, 0xF>(v), v);
  v = qmul(dpp_quat<R, 0x142, 0xA>(v), v);
  v = qmul(dpp_quat<R, 0x143, 0xC>(v), v);
  return v;
}

// Inclusive prefix sum in precision R (row shifts + row broadcasts).
template <typename R>
__device__ __forceinline__ R wave_prefix_sum_r(R v) {
  v += dpp0<0x111>(v);
  v += dpp0<0x112>(v);
  v += dpp0<0x114>(v);
  v += dpp0<0x118>(v);
  v += dpp<0x142, 0xA>(R(0), v);
  v += dpp<0x143, 0xC>(R(0), v);
  return v;
}

// rotate v by the unit quaternion Q: v + 2w (u x v) + 2 u x (u x v), u = (x, y, z)
template <typename R>
__device__ __forceinline__ void qrotate(const Quat<R>& Q, const R v[3], R out[3]) {
  const R c0 = Q.y * v[2] - Q.z * v[1], c1 = Q.z * v[0] - Q.x * v[2], c2 = Q.x * v[1] - Q.y * v[0];
  const R d0 = Q.y * c2 - Q.z * c1, d1 = Q.z * c0 - Q.x * c2, d2 = Q.x * c1 - Q.y * c0;
  out[0] = v[0] + R(2) * (Q.w * c0 + d0);
  out[1] = v[1] + R(2) * (Q.w * c1 + d1);
  out[2] = v[2] + R(2) * (Q.w * c2 + d2);
}

// sin and cos of half the joint angle without the math library's general
// argument path: Cody-Waite reduction of x = q/2 by pi/2 (pi/2 split into a
// 30-bit, a 30-bit and a 53-bit part, exact products for |k| < 2^23, i.e.
// |q| < ~1e7 rad), then Taylor series of sin and cos on [-pi/4, pi/4]
// (float64: through r^17 and r^16; float32: through r^11 and r^10, evaluated
// in float32 after the float64 reduction).
constexpr double kTwoOverPi = 0.6366197723675814;
constexpr double kPio2Hi = 0x1.921fb54800000p+0;
constexpr double kPio2Mid = -0x1.de973dc800000p-31;
constexpr double kPio2Lo = -0x1.9d9cceba3f91fp-62;

constexpr double inv_fact(int n) { return n <= 1 ? 1.0 : inv_fact(n - 1) / n; }
// 1/n!, forced to compile-time constants
template <int N>
struct InvFact {
  static constexpr double value = inv_fact(N);
};

__device__ __forceinline__ double reduce_pio2(double x, int& quadrant) {
  const double k = rint(x * kTwoOverPi);
  double r = fma(-k, kPio2Hi, x);
  r = fma(-k, kPio2Mid, r);
  r = fma(-k, kPio2Lo, r);
  quadrant = ((int)k) & 3;
  return r;
}

template <typename R>
__device__ __forceinline__ void sincos_poly(R r, R& sr, R& cr);
template <>
__device__ __forceinline__ void sincos_poly<double>(double r, double& sr, double& cr) {
  const double z = r * r;
  double ps = -InvFact<17>::value;
  ps = fma(ps, z, InvFact<15>::value);
  ps = fma(ps, z, -InvFact<13>::value);
  ps = fma(ps, z, InvFact<11>::value);
  ps = fma(ps, z, -InvFact<9>::value);
  ps = fma(ps, z, InvFact<7>::value);
  ps = fma(ps, z, -InvFact<5>::value);
  ps = fma(ps, z, InvFact<3>::value);
  sr = fma(-r * z, ps, r);  // r - r^3/3! + ...
  double pc = InvFact<16>::value;
  pc = fma(pc, z, -InvFact<14>::value);
  pc = fma(pc, z, InvFact<12>::value);
  pc = fma(pc, z, -InvFact<10>::value);
  pc = fma(pc, z, InvFact<8>::value);
  pc = fma(pc, z, -InvFact<6>::value);
  pc = fma(pc, z, InvFact<4>::value);
  pc = fma(pc, z, -0.5);
  cr = fma(z, pc, 1.0);
}
template <>
__device__ __forceinline__ void sincos_poly<float>(float r, float& sr, float& cr) {
  const float z = r * r;
  float ps = -(float)InvFact<11>::value;
  ps = fmaf(ps, z, (float)InvFact<9>::value);
  ps = fmaf(ps, z, -(float)InvFact<7>::value);
  ps = fmaf(ps, z, (float)InvFact<5>::value);
  ps = fmaf(ps, z, -(float)InvFact<3>::value);
  sr = fmaf(r * z, ps, r);
  float pc = -(float)InvFact<10>::value;
  pc = fmaf(pc, z, (float)InvFact<8>::value);
  pc = fmaf(pc, z, -(float)InvFact<6>::value);
  pc = fmaf(pc, z, (float)InvFact<4>::value);
  pc = fmaf(pc, z, -0.5f);
  cr = fmaf(z, pc, 1.0f);
}

template <typename R>
__device__ __forceinline__ void half_sincos(double q, R& s, R& c) {
  int quadrant;
  const double r = reduce_pio2(0.5 * q, quadrant);
  R sr, cr;
  sincos_poly<R>((R)r, sr, cr);
  // x = k pi/2 + r
  const R s0 = (quadrant & 1) ? cr : sr;
  const R c0 = (quadrant & 1) ? sr : cr;
  s = (quadrant & 2) ? -s0 : s0;
  c = ((quadrant + 1) & 2) ? -c0 : c0;
}

// Hinge rotation by q about the unit axis a: the quaternion (cos q/2, sin q/2 a).
template <typename R>
__device__ __forceinline__ Quat<R> hinge_quat(const R a[3], double q) {
  R sh, ch;
  half_sincos(q, sh, ch);
  Quat<R> r;
  r.w = ch;
  r.x = sh * a[0];
  r.y = sh * a[1];
  r.z = sh * a[2];
  return r;
}

// Index of S[x][y] in the 6-entry upper triangle of a symmetric 3x3
// (00 01 02 11 12 22), and of M[x][y] in the 10-entry upper triangle of a
// symmetric 4x4.  Written without recursion so that, with unrolled constant
// arguments, the index folds to a constant (a recursive form is turned into a
// loop before inlining and leaves a run-time register index).
__device__ __forceinline__ constexpr int sym3_ordered(int x, int y) { return x == 0 ? y : x == 1 ? 2 + y : 5; }
__device__ __forceinline__ constexpr int sym3(int x, int y) {
  return x <= y ? sym3_ordered(x, y) : sym3_ordered(y, x);
}
__device__ __forceinline__ constexpr int sym4_ordered(int x, int y) {
  return x == 0 ? y : x == 1 ? 3 + y : x == 2 ? 5 + y : 9;
}
__device__ __forceinline__ constexpr int sym4(int x, int y) {
  return x <= y ? sym4_ordered(x, y) : sym4_ordered(y, x);
}

// ------------------------------------------------------------- model data --
struct DevModel {
  int n_models, n_dofs;
  const int* f0;            // [n_models+1] first frame (= DOF) of every model
  const int* order;         // [n_models] model of every workgroup of a rollout: most frames
                            // first, so the longest solves start first and the dispatcher's
                            // round robin spreads them over the XCDs
  // per-frame records (array of structures: one pointer per lane, immediate offsets)
  //   fr: axis (3), joint offset (3, nonzero only on a link's first frame),
  //       mass moment upper triangle (10, nonzero only on a link's last frame)
  const double* fr64;       // [n_dofs][16]
  const float* fr32;        // [n_dofs][16]
  const int* pose_link;     // [n_dofs] link whose pose frame this is, -1 otherwise
  double* B64;              // [n_dofs][12] per-step constant -2 A(q_k) + A(q_{k-1})
  float* B32;               // [n_dofs][12]
  const long long* hoff;    // [n_models+1] start of every model's block in hinv
  double* hinv;             // per model: chains of more than 64 frames, the frames' spatial
                            // inertias [nf][10]; branched models, those and the recursion's
                            // accumulators [nf][31], then the explicit L^-1 of the
                            // preconditioner (rows over the frames below: sum of
                            // (fend - f + 1)); nothing for one-wave chains (their
                            // explicit inverse lives in LDS)
  double* hist;             // models of more than 64 frames: [n_dofs][2*kMaxHist] L-BFGS
                            // pairs, s ring then y ring
  // frames are stored in depth-first preorder of the links (the identity for chains)
  const int* uidx;          // [n_dofs] index of the frame's DOF in the caller's vectors
  const int* fpar;          // [n_dofs] parent frame within the model, -1 = world
  const int* fend;          // [n_dofs] last frame below this one (within the model)
  const int* wrow;          // branched models: [n_dofs] start of the frame's row of the
                            // preconditioner's explicit L^-1 within the model's block
  const int* fheight;       // branched models: [n_dofs] longest path down to a leaf
  const int* mheight;       // branched models: [n_models] largest height of the model
  int jump_rounds;          // ceil(log2(deepest frame path)) of the batch
  double gx, gy, gz;
  // optional terms (models with slides, drag or contact points; NULL otherwise)
  const signed char* fkind; // [n_dofs] 1 = slide (translation along the axis), 0 = hinge
  const double* fdrag;      // [n_dofs] drag coefficient of the link whose mass the frame carries
  const int* coff;          // [n_dofs+1] contact points of frame f: coff[f] .. coff[f+1]-1
  const double* cpt;        // [n_contacts][3] point in the frame of its link
  double* Ak64;             // [n_dofs][12] per-step A(q_k) (drag and friction)
  float* Ak32;              // [n_dofs][12]
  double plane[4];          // contact half-space n.x < h: n (unit, world), h
  double cd1, cd2;          // normal and friction penalties of Eq. FRI
};

inline DevModel dev_view(const abd_model* m) {
  DevModel d;
  d.n_models = m->n_models;
  d.n_dofs = m->n_dofs;
  d.f0 = m->f0;
  d.order = m->order;
  d.fr64 = m->fr64;
  d.fr32 = m->fr32;
  d.pose_link = m->pose_link;
  d.B64 = m->B64; d.B32 = m->B32;
  d.hoff = m->hoff;
  d.hinv = m->hinv;
  d.hist = m->hist;
  d.uidx = m->uidx;
  d.fpar = m->fpar;
  d.fend = m->fend;
  d.wrow = m->wrow;
  d.fheight = m->fheight;
  d.mheight = m->mheight;
  d.jump_rounds = m->jump_rounds;
  d.gx = m->g[0]; d.gy = m->g[1]; d.gz = m->g[2];
  d.fkind = m->fkind;
  d.fdrag = m->fdrag;
  d.coff = m->coff;
  d.cpt = m->cpt;
  d.Ak64 = m->Ak64;
  d.Ak32 = m->Ak32;
  for (int k = 0; k < 4; ++k) d.plane[k] = m->plane[k];
  d.cd1 = m->cd1;
  d.cd2 = m->cd2;
  return d;
}

// wavefronts per model workgroup: the power of two covering the longest model
inline int waves_for(int max_frames) {
  int nw = 1;
  while (nw * kMaxFrames < max_frames) nw *= 2;
  return nw;
}

template <typename R>
struct Arr;
template <>
struct Arr<double> {
  static __device__ __forceinline__ const double* fr(const DevModel& d) { return d.fr64; }
  static __device__ __forceinline__ const double* B(const DevModel& d) { return d.B64; }
  static __device__ __forceinline__ const double* Ak(const DevModel& d) { return d.Ak64; }
};
template <>
struct Arr<float> {
  static __device__ __forceinline__ const float* fr(const DevModel& d) { return d.fr32; }
  static __device__ __forceinline__ const float* B(const DevModel& d) { return d.B32; }
  static __device__ __forceinline__ const float* Ak(const DevModel& d) { return d.Ak32; }
};

// ----------------------------------------------------------- scan policies --
// Scans and reductions over the frames of one model.  Frame j of a model lives
// in lane j % 64 of wave j / 64 of its workgroup.
//   WaveScan:     one wavefront per model (DPP only);
//   BlockScan<NW>: NW wavefronts per model: DPP inside each wave, then the wave
//                 totals are exchanged through LDS (one barrier per scan).  Two
//                 exchange areas alternate: a wave can only write an area again
//                 after the barrier of the next scan, which every wave reaches
//                 after reading the area.
struct WaveScan {
  template <typename R>
  __device__ __forceinline__ Quat<R> prefix_quat(const Quat<R>& v) { return wave_prefix_quat(v); }
  // the predecessor's inclusive prefix (identity for frame 0)
  template <typename R>
  __device__ __forceinline__ Quat<R> parent_quat(const Quat<R>& incl) { return dpp_quat<R, 0x138, 0xF>(incl); }
  template <typename R>
  __device__ __forceinline__ void prefix_sum3(R v[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_prefix_sum_r(v[k]);
  }
  // v[k] <- sum over the frames at and below this one; a, b <- model totals
  __device__ __forceinline__ void suffix6_total2(double v[6], double& a, double& b) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double pre = wave_prefix_sum(v[k]);
      v[k] = (readlane(pre, 63) - pre) + v[k];
    }
    wave_sum2(a, b);
  }
  __device__ __forceinline__ double suffix(double v) {
    const double pre = wave_prefix_sum(v);
    return (readlane(pre, 63) - pre) + v;
  }
  __device__ __forceinline__ double sum(double v) { return wave_sum(v); }
  __device__ __forceinline__ void sum2(double& a, double& b) { wave_sum2(a, b); }
  __device__ __forceinline__ bool all_finite(double x) { return !__any(!isfinite(x)); }
  __device__ __forceinline__ void sync() {}
  // a model-uniform value kept in scalar registers
  __device__ __forceinline__ double uniform(double v) { return wave_uniform(v); }
};

// Models packed S lanes apart in one wavefront (S = 16: one DPP row per model,
// S = 32: two rows), frame j of the model in lane j of its segment.  The scans
// are the wave scans without the steps that cross a segment (S = 16: no row
// broadcasts; S = 32: the row-15 broadcast into rows 1 and 3 only), the totals
// are read from the segment's last lane, and nothing is made wave-uniform: the
// models of a wavefront branch independently.  Lanes past a model's last frame
// hold identities and zeros exactly as in the wave scans, so every sum and
// product takes the same operands in the same order as there (a model gets the
// same results in either layout).
template <int S>
struct SegScan {
  static_assert(S == 16 || S == 32, "segments of one or two DPP rows");
  int fl;  // lane within the segment
  template <typename R>
  __device__ __forceinline__ Quat<R> prefix_quat(Quat<R> v) {
    v = qmul(dpp_quat<R, 0x111, 0xF>(v), v);
    v = qmul(dpp_quat<R, 0x112, 0xF>(v), v);
    v = qmul(dpp_quat<R, 0x114, 0xF>(v), v);
    v = qmul(dpp_quat<R, 0x118, 0xF>(v), v);
    if (S == 32) v = qmul(dpp_quat<R, 0x142, 0xA>(v), v);
    return v;
  }
  template <typename R>
  __device__ __forceinline__ Quat<R> parent_quat(const Quat<R>& incl) {
    const Quat<R> sh = dpp_quat<R, 0x138, 0xF>(incl);
    return fl == 0 ? Quat<R>{R(1), R(0), R(0), R(0)} : sh;
  }
  template <typename R>
  static __device__ __forceinline__ R prefix(R v) {
    v += dpp0<0x111>(v);
    v += dpp0<0x112>(v);
    v += dpp0<0x114>(v);
    v += dpp0<0x118>(v);
    if (S == 32) v += dpp<0x142, 0xA>(R(0), v);
    return v;
  }
  static __device__ __forceinline__ double last(double v) { return __shfl(v, S - 1, S); }
  template <typename R>
  __device__ __forceinline__ void prefix_sum3(R v[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = prefix(v[k]);
  }
  __device__ __forceinline__ void suffix6_total2(double v[6], double& a, double& b) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double pre = prefix(v[k]);
      v[k] = (last(pre) - pre) + v[k];
    }
    sum2(a, b);
  }
  __device__ __forceinline__ double suffix(double v) {
    const double pre = prefix(v);
    return (last(pre) - pre) + v;
  }
  __device__ __forceinline__ double sum(double v) { return last(prefix(v)); }
  __device__ __forceinline__ void sum2(double& a, double& b) {
    a = prefix(a);
    b = prefix(b);
    a = last(a);
    b = last(b);
  }
  __device__ __forceinline__ bool all_finite(double x) {
    const unsigned long long bad = __ballot(!isfinite(x));
    const int base = (int)(threadIdx.x % kWave) - fl;
    return ((bad >> base) & ((1ull << S) - 1)) == 0;
  }
  __device__ __forceinline__ void sync() {}
  __device__ __forceinline__ double uniform(double v) { return v; }
};

template <int NW>
struct BlockScan {
  double* xch;  // LDS [2][NW][8]
  int wave, lane, area;
  double cq[4];  // carry of the last prefix_quat: product of the earlier waves' totals

  __device__ __forceinline__ double* next_area() {
    double* a = xch + area * (NW * 8);
    area ^= 1;
    return a;
  }
  __device__ __forceinline__ void sync() { __syncthreads(); }
  __device__ __forceinline__ double uniform(double v) { return wave_uniform(v); }

  template <typename R>
  __device__ __forceinline__ Quat<R> prefix_quat(const Quat<R>& v0) {
    const Quat<R> v = wave_prefix_quat(v0);
    double* a = next_area();
    if (lane == 63) {
      a[wave * 8 + 0] = v.w; a[wave * 8 + 1] = v.x; a[wave * 8 + 2] = v.y; a[wave * 8 + 3] = v.z;
    }
    __syncthreads();
    Quat<R> c{R(1), R(0), R(0), R(0)};
    for (int w = 0; w < wave; ++w)
      c = qmul(c, Quat<R>{(R)a[w * 8 + 0], (R)a[w * 8 + 1], (R)a[w * 8 + 2], (R)a[w * 8 + 3]});
    cq[0] = c.w; cq[1] = c.x; cq[2] = c.y; cq[3] = c.z;
    return qmul(c, v);
  }
  template <typename R>
  __device__ __forceinline__ Quat<R> parent_quat(const Quat<R>& incl) {
    const Quat<R> sh = dpp_quat<R, 0x138, 0xF>(incl);
    const Quat<R> c{(R)cq[0], (R)cq[1], (R)cq[2], (R)cq[3]};
    return lane == 0 ? c : sh;
  }
  template <typename R>
  __device__ __forceinline__ void prefix_sum3(R v[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = wave_prefix_sum_r(v[k]);
    double* a = next_area();
    if (lane == 63)
#pragma unroll
      for (int k = 0; k < 3; ++k) a[wave * 8 + k] = v[k];
    __syncthreads();
    double c[3] = {0, 0, 0};
    for (int w = 0; w < wave; ++w)
#pragma unroll
      for (int k = 0; k < 3; ++k) c[k] += a[w * 8 + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] += (R)c[k];
  }
  __device__ __forceinline__ void suffix6_total2(double v[6], double& ta, double& tb) {
    double pre[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pre[k] = wave_prefix_sum(v[k]);
    wave_sum2(ta, tb);
    double* a = next_area();
    if (lane == 63) {
#pragma unroll
      for (int k = 0; k < 6; ++k) a[wave * 8 + k] = pre[k];
      a[wave * 8 + 6] = ta;
      a[wave * 8 + 7] = tb;
    }
    __syncthreads();
    double before[6] = {0, 0, 0, 0, 0, 0}, all[6] = {0, 0, 0, 0, 0, 0};
    ta = 0.0;
    tb = 0.0;
    for (int w = 0; w < NW; ++w) {
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double x = a[w * 8 + k];
        all[k] += x;
        if (w < wave) before[k] += x;
      }
      ta += a[w * 8 + 6];
      tb += a[w * 8 + 7];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = (all[k] - (before[k] + pre[k])) + v[k];
  }
  __device__ __forceinline__ double suffix(double v) {
    const double pre = wave_prefix_sum(v);
    double* a = next_area();
    if (lane == 63) a[wave * 8] = pre;
    __syncthreads();
    double before = 0.0, all = 0.0;
    for (int w = 0; w < NW; ++w) {
      const double x = a[w * 8];
      all += x;
      if (w < wave) before += x;
    }
    return (all - (before + pre)) + v;
  }
  __device__ __forceinline__ double sum(double v) {
    v = wave_sum(v);
    double* a = next_area();
    if (lane == 0) a[wave * 8] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += a[w * 8];
    return t;
  }
  __device__ __forceinline__ bool all_finite(double x) { return sum(isfinite(x) ? 0.0 : 1.0) == 0.0; }
  __device__ __forceinline__ void sum2(double& x, double& y) {
    wave_sum2(x, y);
    double* a = next_area();
    if (lane == 0) {
      a[wave * 8] = x;
      a[wave * 8 + 1] = y;
    }
    __syncthreads();
    x = 0.0;
    y = 0.0;
    for (int w = 0; w < NW; ++w) {
      x += a[w * 8];
      y += a[w * 8 + 1];
    }
  }
};

// TreeScan<NW>: branched models.  Frames are stored in depth-first preorder,
// so the frames below frame j form the contiguous range [j, end_j].
//   * prefixes along the ancestor path (the rotation and translation parts of
//     Alg. 1's forward pass) by pointer jumping through LDS: every frame keeps
//     the partial result over its path up to a current ancestor and replaces it
//     by the ancestor's partial result composed with its own, then jumps to the
//     ancestor's ancestor (`rounds` = ceil(log2(depth)) rounds);
//   * sums over the frames below (the adjoint pass) as differences of the
//     preorder prefix sum: P(end_j) - P(j - 1);
//   * model-wide reductions as in BlockScan.
template <int NW>
struct TreeScan : BlockScan<NW> {
  double (*tq)[4];  // LDS [64 NW][4]: partial rotations, then prefix sums
  double (*tv)[6];  // LDS [64 NW][6]
  int* tanc;        // LDS [64 NW]: current ancestor
  int j, parent, send, rounds;

  template <typename R>
  __device__ __forceinline__ Quat<R> prefix_quat(const Quat<R>& r) {
    Quat<R> x = r;
    int a = parent;
    for (int k = 0; k < rounds; ++k) {
      tq[j][0] = x.w; tq[j][1] = x.x; tq[j][2] = x.y; tq[j][3] = x.z;
      tanc[j] = a;
      __syncthreads();
      if (a >= 0) {
        const Quat<R> y{(R)tq[a][0], (R)tq[a][1], (R)tq[a][2], (R)tq[a][3]};
        const int aa = tanc[a];
        x = qmul(y, x);
        a = aa;
      }
      __syncthreads();
    }
    return x;
  }
  template <typename R>
  __device__ __forceinline__ Quat<R> parent_quat(const Quat<R>& incl) {
    tq[j][0] = incl.w; tq[j][1] = incl.x; tq[j][2] = incl.y; tq[j][3] = incl.z;
    __syncthreads();
    Quat<R> p{R(1), R(0), R(0), R(0)};
    if (parent >= 0) p = Quat<R>{(R)tq[parent][0], (R)tq[parent][1], (R)tq[parent][2], (R)tq[parent][3]};
    __syncthreads();
    return p;
  }
  template <typename R>
  __device__ __forceinline__ void prefix_sum3(R v[3]) {
    double x[3] = {v[0], v[1], v[2]};
    int a = parent;
    for (int k = 0; k < rounds; ++k) {
      tv[j][0] = x[0]; tv[j][1] = x[1]; tv[j][2] = x[2];
      tanc[j] = a;
      __syncthreads();
      if (a >= 0) {
        const int aa = tanc[a];
        x[0] += tv[a][0]; x[1] += tv[a][1]; x[2] += tv[a][2];
        a = aa;
      }
      __syncthreads();
    }
    v[0] = (R)x[0]; v[1] = (R)x[1]; v[2] = (R)x[2];
  }
  __device__ __forceinline__ void suffix6_total2(double v[6], double& ta, double& tb) {
    // inclusive preorder prefix of the 6 values (waves + carries), model totals of ta, tb
    double pre[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) pre[k] = wave_prefix_sum(v[k]);
    wave_sum2(ta, tb);
    double* a = this->next_area();
    if (this->lane == 63) {
#pragma unroll
      for (int k = 0; k < 6; ++k) a[this->wave * 8 + k] = pre[k];
      a[this->wave * 8 + 6] = ta;
      a[this->wave * 8 + 7] = tb;
    }
    __syncthreads();
    double before[6] = {0, 0, 0, 0, 0, 0};
    ta = 0.0;
    tb = 0.0;
    for (int w = 0; w < NW; ++w) {
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if (w < this->wave) before[k] += a[w * 8 + k];
      ta += a[w * 8 + 6];
      tb += a[w * 8 + 7];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) tv[j][k] = before[k] + pre[k];
    __syncthreads();
    // sum over [j, end_j] = P(end_j) - P(j) + own
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = (tv[send][k] - tv[j][k]) + v[k];
    __syncthreads();
  }
  __device__ __forceinline__ double suffix(double v) {
    double w6[6] = {v, 0, 0, 0, 0, 0};
    double ua = 0.0, ub = 0.0;
    suffix6_total2(w6, ua, ub);
    return w6[0];
  }
};

// World pose A_j = [R_j | t_j] of every frame of this wave's model (Alg. 1
// forward pass; frame j's joint is at its origin, offset o_j in the parent frame):
//   R_j = R_{j-1} Rot(a_j, q_j)  -> prefix scan of hinge quaternions,
//   t_j = t_{j-1} + R_{j-1} o_j  -> prefix sum of the parent-rotated offsets.
// A slide frame (slide = true) does not rotate and moves its offset along its
// axis: R_j = R_{j-1}, t_j = t_{j-1} + R_{j-1} (o_j + q_j a_j).
template <typename R, typename S>
__device__ __forceinline__ Xf<R> forward_kinematics(S& sc, const R a[3], const R o[3], bool valid, double q,
                                                    bool slide = false) {
  Quat<R> Q = hinge_quat(a, valid && !slide ? q : 0.0);
  if (!valid || slide) Q = Quat<R>{R(1), R(0), R(0), R(0)};
  Q = sc.prefix_quat(Q);
  // parent rotation: the predecessor's prefix (identity for the root frame)
  const Quat<R> Qp = sc.parent_quat(Q);
  R v[3];
  if (slide) {
    const R os[3] = {o[0] + R(q) * a[0], o[1] + R(q) * a[1], o[2] + R(q) * a[2]};
    qrotate(Qp, os, v);
  } else {
    qrotate(Qp, o, v);
  }
  sc.prefix_sum3(v);
  Xf<R> A;
  A.m[3] = v[0];
  A.m[7] = v[1];
  A.m[11] = v[2];
  const R xx = Q.x * Q.x, yy = Q.y * Q.y, zz = Q.z * Q.z;
  const R xy = Q.x * Q.y, xz = Q.x * Q.z, yz = Q.y * Q.z;
  const R wx = Q.w * Q.x, wy = Q.w * Q.y, wz = Q.w * Q.z;
  A.m[0] = R(1) - R(2) * (yy + zz);
  A.m[1] = R(2) * (xy - wz);
  A.m[2] = R(2) * (xz + wy);
  A.m[4] = R(2) * (xy + wz);
  A.m[5] = R(1) - R(2) * (xx + zz);
  A.m[6] = R(2) * (yz - wx);
  A.m[8] = R(2) * (xz - wy);
  A.m[9] = R(2) * (yz + wx);
  A.m[10] = R(1) - R(2) * (xx + yy);
  return A;
}

// axis and joint offset of this lane's frame (float64, kept in registers), and
// whether it is a slide (only read by the FX instantiations: models with slides,
// drag or contact points)
struct FrameGeo {
  double a[3], o[3];
  bool slide;
};
template <bool FX = false>
__device__ __forceinline__ FrameGeo load_geo(const DevModel& d, int f, bool valid) {
  FrameGeo g;
  const double* rec = d.fr64 + (size_t)f * 16;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g.a[k] = ld_if(rec + k, valid);
    g.o[k] = ld_if(rec + 3 + k, valid);
  }
  g.slide = FX && valid && d.fkind && d.fkind[f] == 1;
  return g;
}
template <typename R, bool FX = false, typename S>
__device__ __forceinline__ Xf<R> fk_geo(S& sc, const FrameGeo& g, bool valid, double q) {
  const R a[3] = {(R)g.a[0], (R)g.a[1], (R)g.a[2]};
  const R o[3] = {(R)g.o[0], (R)g.o[1], (R)g.o[2]};
  return forward_kinematics<R>(sc, a, o, valid, q, FX && g.slide);
}

// Eq. FRI at one contact point, world position x (xk at q_k), times dt^2:
//   V = dt^2 D1 d^2 + D2 d^2 |P (x - xk)|^2,  d = max(0, h - n.x),  P = I - n n^T.
// Returns V and the force f = dV/dx.
__device__ __forceinline__ double contact_force(const DevModel& d, double dt2, const double x[3],
                                                const double xk[3], double f[3]) {
  const double* n = d.plane;
  const double pen = d.plane[3] - (n[0] * x[0] + n[1] * x[1] + n[2] * x[2]);
  if (!(pen > 0.0)) {
    f[0] = f[1] = f[2] = 0.0;
    return 0.0;
  }
  const double v0 = x[0] - xk[0], v1 = x[1] - xk[1], v2 = x[2] - xk[2];
  const double nv = n[0] * v0 + n[1] * v1 + n[2] * v2;
  const double u0 = v0 - nv * n[0], u1 = v1 - nv * n[1], u2 = v2 - nv * n[2];
  const double a = dt2 * d.cd1 + d.cd2 * (u0 * u0 + u1 * u1 + u2 * u2);
  const double fn = -2.0 * pen * a, ft = 2.0 * d.cd2 * pen * pen;
  f[0] = fn * n[0] + ft * u0;
  f[1] = fn * n[1] + ft * u1;
  f[2] = fn * n[2] + ft * u2;
  return pen * pen * a;
}

struct EvalResult {
  double E;  // objective of the model (wave-uniform)
  double S;  // sum of |per-frame terms| (rounding scale of E; wave-uniform)
  double g;  // dE/dq of this lane's DOF (0 on lanes without a frame)
};

// One objective + gradient evaluation for the model of this wave.  FX: the
// model may have slides, drag and contact points.  TRIAL (a line-search trial
// that is likely rejected): the model totals E, S first, by the same sums in
// the same order (bitwise the same values), and the adjoint scan and the
// gradient only where an acceptance test will read them: sufficient decrease
// (E <= bound) or a change within the objective's rounding (|E - E0| <=
// tol_s S); g = 0 otherwise.
template <typename R, bool FX = false, bool TRIAL = false, typename S>
__device__ EvalResult evaluate(S& sc, const DevModel& d, const FrameGeo& geo, int f, bool valid, double q,
                               double tau, double dt2, double bound = 0.0, double E0 = 0.0, double tol_s = 0.0) {
  // keep the per-frame loads inside the evaluation (no hoisting across calls,
  // which would pin them in registers for the whole solve); they are issued
  // first so that their latency overlaps the kinematics scan
  asm volatile("" ::: "memory");
  R M[10], Bn[4];
  const R* rec = Arr<R>::fr(d) + (size_t)f * 16;
  const R* Bp = Arr<R>::B(d) + (size_t)f * 12;
#pragma unroll
  for (int k = 0; k < 10; ++k) M[k] = ld_if(rec + 6 + k, valid);
#pragma unroll
  for (int k = 0; k < 4; ++k) Bn[k] = Bp[k];  // lanes without a frame: M = 0 zeroes every term
  const Xf<R> A = fk_geo<R, FX>(sc, geo, valid, q);
  const R a[3] = {(R)geo.a[0], (R)geo.a[1], (R)geo.a[2]};

  // Row r of D = A + B (= A(q) - 2A(q_k) + A(q_{k-1})), of D M and of the seed
  // G = dE/dA = D M - dt^2 g (M e4)^T; e = 1/2 tr(D M D^T) - dt^2 g^T A M e4.
  // The world-frame adjoint term k = sum_c R[:,c] x G[:,c] + t x G[:,3]
  // is accumulated as each row of G appears (float64).
  const R dt2r = R(dt2);
  R e = R(0), pot = R(0);
  double k0 = 0.0, k1 = 0.0, k2 = 0.0, fv[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const R gr = R(r == 0 ? d.gx : r == 1 ? d.gy : d.gz);
    R D[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) D[c] = A.m[4 * r + c] + Bn[c];
    if (r < 2)
#pragma unroll
      for (int c = 0; c < 4; ++c) Bn[c] = Bp[4 * (r + 1) + c];
    R AMe4 = R(0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      R dm = R(0);
#pragma unroll
      for (int x = 0; x < 4; ++x) dm += D[x] * M[sym4(x, c)];
      e += R(0.5) * dm * D[c];
      AMe4 += A.m[4 * r + c] * M[sym4(c, 3)];
      const double Grc = (double)(dm - dt2r * gr * M[sym4(c, 3)]);
      // (u x w) with u = column c of A, w = column c of G; row r of w is Grc
      const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
      const double u1 = A.m[4 * r1 + c], u2 = A.m[4 * r2 + c];
      // component r1 gets +u2*w_r, component r2 gets -u1*w_r
      if (r == 0) { k1 += u2 * Grc; k2 -= u1 * Grc; }
      if (r == 1) { k2 += u2 * Grc; k0 -= u1 * Grc; }
      if (r == 2) { k0 += u2 * Grc; k1 -= u1 * Grc; }
      if (c == 3) fv[r] = Grc;
    }
    pot -= gr * AMe4;
  }
  // drag c tr(dA M dA^T), dA = A - A(q_k), seed 2 c dA M; contact points (Eq. FRI):
  // a point force f at x adds x x f to the moment sum and f to the force sum
  double efx = 0.0;
  if (FX && valid) {
    const R* Akp = Arr<R>::Ak(d) + (size_t)f * 12;
    const double c = d.fdrag ? d.fdrag[f] : 0.0;
    if (c != 0.0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        R dA[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) dA[x] = A.m[4 * r + x] - Akp[4 * r + x];
        const int r1 = (r + 1) % 3, r2 = (r + 2) % 3;
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
          R dm = R(0);
#pragma unroll
          for (int x = 0; x < 4; ++x) dm += dA[x] * M[sym4(x, cc)];
          efx += c * (double)dm * (double)dA[cc];
          const double Grc = 2.0 * c * (double)dm;
          const double u1 = A.m[4 * r1 + cc], u2 = A.m[4 * r2 + cc];
          if (r == 0) { k1 += u2 * Grc; k2 -= u1 * Grc; }
          if (r == 1) { k2 += u2 * Grc; k0 -= u1 * Grc; }
          if (r == 2) { k0 += u2 * Grc; k1 -= u1 * Grc; }
          if (cc == 3) fv[r] += Grc;
        }
      }
    }
    if (d.coff)
      for (int p = d.coff[f]; p < d.coff[f + 1]; ++p) {
        const double pt[3] = {d.cpt[3 * p], d.cpt[3 * p + 1], d.cpt[3 * p + 2]};
        double x[3], xk[3], fc[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          x[r] = (double)A.m[4 * r] * pt[0] + (double)A.m[4 * r + 1] * pt[1] + (double)A.m[4 * r + 2] * pt[2] +
                 (double)A.m[4 * r + 3];
          xk[r] = (double)Akp[4 * r] * pt[0] + (double)Akp[4 * r + 1] * pt[1] + (double)Akp[4 * r + 2] * pt[2] +
                  (double)Akp[4 * r + 3];
        }
        efx += contact_force(d, dt2, x, xk, fc);
        k0 += x[1] * fc[2] - x[2] * fc[1];
        k1 += x[2] * fc[0] - x[0] * fc[2];
        k2 += x[0] * fc[1] - x[1] * fc[0];
        fv[0] += fc[0];
        fv[1] += fc[1];
        fv[2] += fc[2];
      }
  }
  const double tq = dt2 * tau * q;
  const double elane = (double)e + dt2 * (double)pot + efx;
  double Ev = elane - (valid ? tq : 0.0);
  double Sv = fabs(elane) + (valid ? fabs(tq) : 0.0);

  // suffix sums over the frames below (inclusive prefix, then total - prefix +
  // own) and the model totals of E and S
  double suf[6] = {k0, k1, k2, fv[0], fv[1], fv[2]};
  if constexpr (TRIAL) {
    sc.sum2(Ev, Sv);
    if (!(isfinite(Ev) && (Ev <= bound || fabs(Ev - E0) <= tol_s * Sv))) {
      EvalResult res;
      res.g = 0.0;
      res.E = Ev;
      res.S = Sv;
      return res;
    }
    double ta = 0.0, tb = 0.0;  // totals formed again, not needed
    sc.suffix6_total2(suf, ta, tb);
  } else {
    sc.suffix6_total2(suf, Ev, Sv);
  }

  // world axis w = R a, joint point p = t
  const double w0 = (double)A.m[0] * a[0] + (double)A.m[1] * a[1] + (double)A.m[2] * a[2];
  const double w1 = (double)A.m[4] * a[0] + (double)A.m[5] * a[1] + (double)A.m[6] * a[2];
  const double w2 = (double)A.m[8] * a[0] + (double)A.m[9] * a[1] + (double)A.m[10] * a[2];
  const double p0 = A.m[3], p1 = A.m[7], p2 = A.m[11];
  // hinge: dE/dq = w.(K - p x F); slide: dE/dq = w.F
  const bool sl = FX && geo.slide;
  const double m0 = sl ? suf[3] : suf[0] - (p1 * suf[5] - p2 * suf[4]);
  const double m1 = sl ? suf[4] : suf[1] - (p2 * suf[3] - p0 * suf[5]);
  const double m2 = sl ? suf[5] : suf[2] - (p0 * suf[4] - p1 * suf[3]);
  EvalResult res;
  res.g = valid ? (w0 * m0 + w1 * m1 + w2 * m2 - dt2 * tau) : 0.0;
  res.E = Ev;
  res.S = Sv;
  return res;
}


// ------------------------------------------------------------ step kernel --
struct StepArgs {
  DevModel d;
  double dt2, tol;
  int m, max_iter, max_ls, precond;
  int refresh;                // re-form the inertia preconditioner every `refresh` iterations (0: never)
  int n_steps;                // time steps in this launch
  int nfmax;                  // frames of the batch's largest model (sizes the LDS of one-wave chains)
  const double* q_prev;       // q_{-1}
  const double* q_curr;       // q_0
  const double* tau;          // [n_steps][n_dofs] or NULL
  double* q_out;              // [n_steps][n_dofs]: q_1 .. q_{n_steps}
  abd_step_stats* stats;      // [n_steps][n_models] or NULL
};

// Largest number of segments of chain_solve (chains of more than one wave).
constexpr int kSolveSegs = 32;

// Per-model LDS of the rollout kernel (one model per workgroup of NW waves):
//   tab:   per frame s (6 = world hinge motion (w; p x w)), U (6 = I^A s), 1/D
//   inert: per frame world spatial inertia about the origin (J 6, h 3, m), for
//          one-wave trees; one-wave chains keep it in the LDS of their explicit
//          inverse, NW > 1 in the model's device scratch
//   xb:    NW > 1: the vector swept by the recursion; branched models: the
//          vector of the preconditioner's product
//   xch:   scan exchange areas of BlockScan
//   branched models (TREE): pointer-jumping buffers of TreeScan (tq, tv, tanc),
//   frame parents (tpar) and the middle vector of the preconditioner's product
//   (acc, first nf doubles)
// SEGS: models per wavefront (packed one-wave chains): the per-model scalars of
// the two-loop recursion are kept per segment, and the vector of the inverse
// product has its own area (vb) instead of the recursion's table.
// TAB false: the table lives in dynamic LDS sized to the batch (k_rollout's
// one-model-per-wavefront chains), and this struct keeps a placeholder row.
template <int NW, bool TREE = false, int SEGS = 1, bool TAB = true>
struct RollLds {
  double tab[TAB ? kMaxFrames * NW : 1][kTab];
  double inert[(NW == 1 && TREE) ? kMaxFrames : 1][10];  // one-wave chains: in the inverse's LDS
  double rho[kMaxHist * SEGS];  // 1/(s_i.y_i): k_rollout by ring slot of the pair, others newest first
  double alp[kMaxHist * SEGS];  // two-loop coefficients
  double vb[SEGS > 1 ? kWave : 1];
  double xb[(NW == 1 && !TREE) ? 1 : kMaxFrames * NW];
  double xch[2][NW][8];
  double tq[TREE ? kMaxFrames * NW : 1][4];
  double tv[TREE ? kMaxFrames * NW : 1][6];
  double acc[TREE ? kMaxFrames * NW : 1][6];
  int tanc[TREE ? kMaxFrames * NW : 1];
  int tpar[TREE ? kMaxFrames * NW : 1];
};
using ModelLds = RollLds<1, false>;

// LDS of chains of more than one wave in k_rollout (a variable of its own, so
// that the kernels without it allocate none): the segment maps and entry
// states of chain_solve and the staged inertia records of aba_setup_rows_staged.
template <bool ON>
struct ChainLds {
  double sgm[kSolveSegs][7][6];
  double sgin[kSolveSegs][6];
  double stg[2][kWave * 10];
};
template <>
struct ChainLds<false> {
  double sgm[1][7][6];
  double sgin[1][6];
  double stg[1][kWave * 10];
};

// 1/x for x > 0 from the hardware reciprocal and one Newton step (a few ulp;
// used where the value only shapes a preconditioner).
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

// Articulated inertias of a chain at the configuration of the preconditioner,
// tip to root:
//   I^A_f = I_f + P_{f+1},  U_f = I^A_f s_f,  D_f = s_f.U_f,
//   P_f = I^A_f - U_f U_f^T / D_f  (passed to the parent frame),
// with the 6x6 algebra spread over lanes: lane
// r < 6 holds row r of P (full rows), computes U_r = P_r . s, the six U_r are
// broadcast through scalar registers, D and 1/D are formed on every lane, and
// each lane updates its row, P_rc <- P_rc - U_r U_c / D.  Entry c of row r of
// the frame inertia [[J, [h]x], [[h]x^T, m 1]] is a signed pick from the
// 10-entry record (J 00 01 02 11 12 22, h, m).  The whole wave runs; lanes >= 6
// shadow row 5 and store nothing.  The next frame's inputs are read while the
// current one is processed.
// Lane r's picks of row r of the frame inertia from the 10-entry record:
// entry c = sgn[c] * record[idx[c]].
__device__ __forceinline__ void rows_pick(int r, int idx[6], float sgn[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int a = r < 3 ? r : c, b = r < 3 ? c : r;  // (3x3 block row, column) of the pick
    if (r < 3 && c < 3) {  // J
      const int lo = a < b ? a : b, hi = a < b ? b : a;
      idx[c] = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
      sgn[c] = 1.0f;
    } else if (r >= 3 && c >= 3) {  // m 1
      idx[c] = 9;
      sgn[c] = (r == c) ? 1.0f : 0.0f;
    } else {  // [h]x (row block 0) or its transpose (row block 1): ([h]x)_{a, b - 3}
      const int ra = a, cb = b - 3;
      if (ra == cb) {
        idx[c] = 9;
        sgn[c] = 0.0f;
      } else {
        idx[c] = 6 + (3 - ra - cb);                 // the remaining component of h
        sgn[c] = (cb == (ra + 2) % 3) ? 1.0f : -1.0f;  // (0,2) (1,0) (2,1) positive
      }
    }
  }
}

// One frame of the recursion on the rows: P += in (this lane's row of the frame
// inertia), U_r = P_r . s, broadcast, D, 1/D, table row f, P -= U U^T / D.
template <int SEG>
__device__ __forceinline__ void rows_step(double P[6], const double in[6], const double s[6], double* tabf,
                                          int lane) {
#pragma unroll
  for (int c = 0; c < 6; ++c) P[c] += in[c];
  const double U = (P[0] * s[0] + P[1] * s[1]) + (P[2] * s[2] + P[3] * s[3]) + (P[4] * s[4] + P[5] * s[5]);
  double Uc[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) Uc[c] = SEG == kWave ? readlane(U, c) : __shfl(U, c, SEG);
  const double D = (s[0] * Uc[0] + s[1] * Uc[1]) + (s[2] * Uc[2] + s[3] * Uc[3]) + (s[4] * Uc[4] + s[5] * Uc[5]);
  const double iD = (D > 0.0) ? recip(D) : 0.0;
  if (lane < 6) tabf[6 + lane] = U;
  if (lane == 0) tabf[12] = iD;
  const double V = U * iD;
#pragma unroll
  for (int c = 0; c < 6; ++c) P[c] -= V * Uc[c];
}

template <int SEG = kWave>
__device__ void aba_setup_rows(const double* inert, double (*tab)[kTab], int nf_in, int lane) {
  // wave-uniform frame loop (segments of packed models: each its own)
  const int nf = SEG == kWave ? __builtin_amdgcn_readfirstlane(nf_in) : nf_in;
  if (nf <= 0) return;
  const int r = lane < 6 ? lane : 5;
  int idx[6];
  float sgn[6];  // -1, 0, +1
  rows_pick(r, idx, sgn);
  double P[6] = {0, 0, 0, 0, 0, 0};
  double in[6], s[6], inn[6], sn[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    inn[c] = (double)sgn[c] * inert[(nf - 1) * 10 + idx[c]];
    sn[c] = tab[nf - 1][c];
  }
  for (int f = nf - 1; f >= 0; --f) {
    const int fn = f > 0 ? f - 1 : 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      in[c] = inn[c];
      s[c] = sn[c];
      inn[c] = (double)sgn[c] * inert[fn * 10 + idx[c]];
      sn[c] = tab[fn][c];
    }
    rows_step<SEG>(P, in, s, tab[f], lane);
  }
}

// The same recursion for a chain of more than one wave, whose inertia records
// live in device memory: they are staged into LDS 64 frames at a time (buf, two
// chunks of 640 doubles), the waves other than wave 0 loading the next chunk
// while wave 0 runs the current one.  Every thread of the workgroup calls it.
template <int NW>
__device__ void aba_setup_rows_staged(const double* inert, double (*tab)[kTab], int nf, int tid,
                                      double (*buf)[kWave * 10]) {
  static_assert(NW > 1, "one-wave chains keep their inertias in LDS");
  const int wave = tid / kWave, lane = tid % kWave;
  const int ktop = (nf - 1) / kWave;
  auto stage = [&](int k, int t0, int stride) {
    const int base = k * kWave, cnt = (nf - base < kWave ? nf - base : kWave) * 10;
    for (int e = t0; e < cnt; e += stride) buf[k & 1][e] = inert[(size_t)base * 10 + e];
  };
  stage(ktop, tid, NW * kWave);
  __syncthreads();
  const int r = lane < 6 ? lane : 5;
  int idx[6];
  float sgn[6];
  rows_pick(r, idx, sgn);
  double P[6] = {0, 0, 0, 0, 0, 0};
  for (int k = ktop; k >= 0; --k) {
    if (wave > 0 && k > 0) stage(k - 1, tid - kWave, (NW - 1) * kWave);
    if (wave == 0) {
      const int lo = k * kWave, hi = (lo + kWave < nf ? lo + kWave : nf) - 1;
      const double* ib = buf[k & 1];
      double in[6], s[6], inn[6], sn[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        inn[c] = (double)sgn[c] * ib[(hi - lo) * 10 + idx[c]];
        sn[c] = tab[hi][c];
      }
      for (int f = hi; f >= lo; --f) {
        const int fn = f > lo ? f - 1 : lo;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          in[c] = inn[c];
          s[c] = sn[c];
          inn[c] = (double)sgn[c] * ib[(fn - lo) * 10 + idx[c]];
          sn[c] = tab[fn][c];
        }
        rows_step<kWave>(P, in, s, tab[f], lane);
      }
    }
    __syncthreads();
  }
}

// Explicit inverse of the joint-space inertia of a one-wave chain, kept in LDS
// as the packed upper triangle: entry (i, j), i <= j, at tri(j) + i, so column
// j of the triangle is contiguous.  Lane j solves H x = e_j with the two sweeps
//   backward  u_f = b_f - s_f.p,   p <- p + U_f u_f / D_f,
//   forward   x_f = (u_f - U_f.a) / D_f,  a <- a + s_f x_f,
// all lanes walking the frames together (the records are LDS broadcasts).  The
// right-hand side vanishes beyond frame j, so p stays zero there and u_f = 0
// for f > j: lane j's nonzero u_f are exactly its own packed column, where they
// are parked and then overwritten by x_f (f <= j); the entries x_f, f > j, are
// those of the columns of the other lanes (H^-1 is symmetric).
__device__ __forceinline__ int tri(int j) { return (j * (j + 1)) >> 1; }

// LDS doubles of the packed inverse, which also holds the per-frame inertia
// inputs of the recursion (10 per frame) before the inverse is formed.
__host__ __device__ constexpr int inverse_lds_doubles(int nf) {
  return (nf * (nf + 1) / 2 > 10 * kMaxFrames) ? nf * (nf + 1) / 2 : 10 * kMaxFrames;
}
// k_rollout's area for chains of at most nf frames, one per wavefront: only
// the lanes of frames write inertia inputs there (the others write to a sink).
__host__ __device__ constexpr int chain_lds_doubles(int nf) {
  return (nf * (nf + 1) / 2 > 10 * nf) ? nf * (nf + 1) / 2 : 10 * nf;
}
// The same area for one model of a wavefront packed with models of at most s
// frames (the float32 full inverse, s^2 floats, fits in the triangle too).
__host__ __device__ constexpr int tile_inverse_doubles(int s) {
  return (s * (s + 1) / 2 > 10 * s) ? s * (s + 1) / 2 : 10 * s;
}

template <int SEG = kWave>
__device__ void aba_inverse(const double (*tab)[kTab], int nf_in, int lane, double* P) {
  const int nf = SEG == kWave ? __builtin_amdgcn_readfirstlane(nf_in) : nf_in;  // wave-uniform frame loops
  const bool act = lane < nf;
  const int col = act ? lane : nf - 1;
  const int base = tri(col);  // lanes without a frame address the last column (in bounds, never stored)
  // the record of the next frame is read while the current one is used
  double t[kTab], tn[kTab];
#pragma unroll
  for (int k = 0; k < kTab; ++k) tn[k] = tab[nf - 1][k];
  double p[6] = {0, 0, 0, 0, 0, 0};
  for (int f = nf - 1; f >= 0; --f) {
#pragma unroll
    for (int k = 0; k < kTab; ++k) t[k] = tn[k];
    const int fn = f > 0 ? f - 1 : 0;
#pragma unroll
    for (int k = 0; k < kTab; ++k) tn[k] = tab[fn][k];
    const double sp = (t[0] * p[0] + t[1] * p[1]) + (t[2] * p[2] + t[3] * p[3]) + (t[4] * p[4] + t[5] * p[5]);
    const double u = (f == lane ? 1.0 : 0.0) - sp;
    if (act && f <= lane) P[base + f] = u;
    const double w = u * t[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] += t[6 + k] * w;
  }
  // tn holds frame 0's record now
  double a[6] = {0, 0, 0, 0, 0, 0};
  double un = ld_if(P + base, act);
  for (int f = 0; f < nf; ++f) {
#pragma unroll
    for (int k = 0; k < kTab; ++k) t[k] = tn[k];
    const double uf = un;
    const int fn = f + 1 < nf ? f + 1 : f;
#pragma unroll
    for (int k = 0; k < kTab; ++k) tn[k] = tab[fn][k];
    un = ld_if(P + base + (fn <= col ? fn : col), act && fn <= lane);
    const double Ua = (t[6] * a[0] + t[7] * a[1]) + (t[8] * a[2] + t[9] * a[3]) + (t[10] * a[4] + t[11] * a[5]);
    const double x = ((act && f <= lane ? uf : 0.0) - Ua) * t[12];
    if (act && f <= lane) P[base + f] = x;
#pragma unroll
    for (int i = 0; i < 6; ++i) a[i] += t[i] * x;
  }
}

// r_j = sum_i (H^-1)_ij v_i: the preconditioner applied to the wave's vector v
// (lane i holds v_i), reading the packed triangle: (i, j) from column j for
// i <= j, from column i (symmetry) otherwise.  v goes through LDS (vb, 64
// doubles) and is read back as broadcasts; eight matrix entries are requested
// at a time.  The row index is wave-uniform (scalar registers), so each entry
// costs a select between two precomputed indices and no branch; rows past the
// model's last (the batch tail) re-read its last row with weight zero.  One
// wave per workgroup.
constexpr int kMvBatch = 8;

template <int SEG = kWave>
__device__ __forceinline__ double apply_inverse(const double* P, double* vb, int nf_in, int lane, double v) {
  const int nf = SEG == kWave ? __builtin_amdgcn_readfirstlane(nf_in) : nf_in;
  const bool act = lane < nf;
  const int col = act ? lane : nf - 1;
  const int base = tri(col);
  vb[lane] = act ? v : 0.0;
  __syncthreads();
  double r0 = 0.0, r1 = 0.0;
  for (int i0 = 0; i0 < nf; i0 += kMvBatch) {
    double h[kMvBatch], x[kMvBatch];
#pragma unroll
    for (int k = 0; k < kMvBatch; ++k) {
      const int i = i0 + k < nf ? i0 + k : nf - 1;
      const int upper = base + i, lower = tri(i) + col;
      h[k] = P[i <= col ? upper : lower];
      x[k] = vb[i];
    }
    // all reads of the batch are issued before the first is used (otherwise
    // the scheduler pairs each read with its use and waits for every pair)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kMvBatch; k += 2) {
      r0 += h[k] * (i0 + k < nf ? x[k] : 0.0);
      r1 += h[k + 1] * (i0 + k + 1 < nf ? x[k + 1] : 0.0);
    }
  }
  __syncthreads();  // vb is reused by the next product
  return act ? r0 + r1 : 0.0;
}

// The same inverse as aba_inverse (float64 sweeps), stored for the mixed
// kernel as the full symmetric matrix in float32, row-major with row stride nf:
// entry (f, j) at F[f * nf + j].  Lane j's u_f (f <= j) are parked at its own
// entries of rows f and read back, then overwritten by x_f, by the same lane
// (no other lane touches column j), so the sweeps need no barrier; u_f = 0 for
// f > j is not stored.  The matrix is only a preconditioner: float32 rounding
// of u and of the entries changes the search directions, not the solution the
// iteration converges to.  nf^2 floats fit in the packed triangle's tri(nf)
// doubles.
// The float32 inverse is formed while the recursion's pivots D_f span at most
// kInv32MaxRatio: uneven chains of 10..50 box links span up to ~1e4, and there
// the eigenvalues of (float32 inverse) x H stay within [0.97, 1.04]; chains
// whose pivots span 1e6 and more can leave it a poor or indefinite
// preconditioner, and they keep the packed float64 inverse.
constexpr float kInv32MaxRatio = 1e5f;

template <int SEG = kWave>
__device__ void aba_inverse_f32(const double (*tab)[kTab], int nf_in, int lane, float* F) {
  const int nf = SEG == kWave ? __builtin_amdgcn_readfirstlane(nf_in) : nf_in;
  const bool act = lane < nf;
  const int col = act ? lane : nf - 1;
  double t[kTab], tn[kTab];
#pragma unroll
  for (int k = 0; k < kTab; ++k) tn[k] = tab[nf - 1][k];
  double p[6] = {0, 0, 0, 0, 0, 0};
  for (int f = nf - 1; f >= 0; --f) {
#pragma unroll
    for (int k = 0; k < kTab; ++k) t[k] = tn[k];
    const int fn = f > 0 ? f - 1 : 0;
#pragma unroll
    for (int k = 0; k < kTab; ++k) tn[k] = tab[fn][k];
    const double sp = (t[0] * p[0] + t[1] * p[1]) + (t[2] * p[2] + t[3] * p[3]) + (t[4] * p[4] + t[5] * p[5]);
    const double u = (f == lane ? 1.0 : 0.0) - sp;
    if (act && f <= lane) F[f * nf + col] = (float)u;
    const double w = u * t[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] += t[6 + k] * w;
  }
  double a[6] = {0, 0, 0, 0, 0, 0};
  float un = ld_if(F + col, act);
  for (int f = 0; f < nf; ++f) {
#pragma unroll
    for (int k = 0; k < kTab; ++k) t[k] = tn[k];
    const float uf = un;
    const int fn = f + 1 < nf ? f + 1 : f;
#pragma unroll
    for (int k = 0; k < kTab; ++k) tn[k] = tab[fn][k];
    un = ld_if(F + fn * nf + col, act && fn <= lane);
    const double Ua = (t[6] * a[0] + t[7] * a[1]) + (t[8] * a[2] + t[9] * a[3]) + (t[10] * a[4] + t[11] * a[5]);
    const double x = ((act && f <= lane ? (double)uf : 0.0) - Ua) * t[12];
    if (act) F[f * nf + col] = (float)x;
#pragma unroll
    for (int i = 0; i < 6; ++i) a[i] += t[i] * x;
  }
}

// r_j = sum_i F_ij v_i with the float32 full inverse of aba_inverse_f32: row i
// is read by the wave as one contiguous run (lane j takes entry (i, j)), v goes
// through LDS as float32 (vb, 64 floats, zero past the model's last frame) and
// is read back as broadcasts, products and sums in float32.  Rows past the last
// (the batch tail) re-read the last row with weight zero.  One wave per
// workgroup.
template <int SEG = kWave>
__device__ __forceinline__ double apply_inverse_f32(const float* F, float* vb, int nf_in, int lane, double v) {
  const int nf = SEG == kWave ? __builtin_amdgcn_readfirstlane(nf_in) : nf_in;
  const bool act = lane < nf;
  const float* Fc = F + (act ? lane : nf - 1);
  vb[lane] = act ? (float)v : 0.0f;
  __syncthreads();
  float r0 = 0.0f, r1 = 0.0f;
  for (int i0 = 0; i0 < nf; i0 += kMvBatch) {
    float h[kMvBatch], x[kMvBatch];
#pragma unroll
    for (int k = 0; k < kMvBatch; ++k) {
      const int i = i0 + k < nf ? i0 + k : nf - 1;
      h[k] = Fc[i * nf];
      x[k] = vb[i0 + k];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kMvBatch; k += 2) {
      r0 = fmaf(h[k], x[k], r0);
      r1 = fmaf(h[k + 1], x[k + 1], r1);
    }
  }
  __syncthreads();  // vb is reused by the next product
  return act ? (double)(r0 + r1) : 0.0;
}

// x = H^{-1} b for a chain of more than one wave, in place in xb (LDS), by
// segments instead of one thread's two sweeps.  Each sweep is an affine
// recurrence in a 6-vector: backward (tip to root) p <- p + w_f (b_f - s_f.p),
// w_f = U_f / D_f, giving u_f = b_f - s_f.p; forward (root to tip)
// a <- a + s_f (u_f - U_f.a) / D_f, giving x_f = (u_f - U_f.a) / D_f.  The
// frames split into S segments of L (L = max(16, ceil(n / kSolveSegs))); per
// sweep:
//   1. seven threads per segment run its frames on the unit vectors (the map's
//      columns) and on zero with the right-hand side (its offset) at once;
//   2. one wave chains the segment maps from the sweep's first segment on,
//      giving every segment's entry state;
//   3. one thread per segment re-runs its frames from its entry state and
//      writes u (or x).
// The arithmetic of a segment's frames in step 3 is the sweep's own; only the
// entry states are composed differently (the preconditioner's rounding).
// Every thread of the workgroup calls it; xb must hold b and be visible.
template <int NW>
__device__ void chain_solve(const double (*tab)[kTab], double* xb, double (*sgm)[7][6], double (*sgin)[6], int n,
                            int tid) {
  const int L = n > 16 * kSolveSegs ? (n + kSolveSegs - 1) / kSolveSegs : 16;
  const int S = (n + L - 1) / L;
  const int g = tid / 7, c = tid % 7;
  const bool grp = g < S;
  const int lo = g * L, hi = (lo + L < n ? lo + L : n) - 1;
  // ---- backward sweep
  if (grp) {
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (c < 6) v[c] = 1.0;
    for (int f = hi; f >= lo; --f) {
      const double* r = tab[f];
      const double sv = (r[0] * v[0] + r[1] * v[1]) + (r[2] * v[2] + r[3] * v[3]) + (r[4] * v[4] + r[5] * v[5]);
      const double w = ((c == 6 ? xb[f] : 0.0) - sv) * r[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] += r[6 + k] * w;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) sgm[g][c][k] = v[k];
  }
  __syncthreads();
  if (tid < kWave) {  // entry states from the tip segment down
    const int cc = tid < 6 ? tid : 5;
    double p = 0.0;
    for (int gg = S - 1; gg >= 0; --gg) {
      if (tid < 6) sgin[gg][tid] = p;
      double pk[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) pk[k] = __shfl(p, k);
      double np = sgm[gg][6][cc];
#pragma unroll
      for (int k = 0; k < 6; ++k) np += sgm[gg][k][cc] * pk[k];
      p = np;
    }
  }
  __syncthreads();
  if (grp && c == 0) {
    double p[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = sgin[g][k];
    for (int f = hi; f >= lo; --f) {
      const double* r = tab[f];
      const double sp = (r[0] * p[0] + r[1] * p[1]) + (r[2] * p[2] + r[3] * p[3]) + (r[4] * p[4] + r[5] * p[5]);
      const double u = xb[f] - sp;
      xb[f] = u;
      const double w = u * r[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) p[k] += r[6 + k] * w;
    }
  }
  __syncthreads();
  // ---- forward sweep
  if (grp) {
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (c < 6) v[c] = 1.0;
    for (int f = lo; f <= hi; ++f) {
      const double* r = tab[f];
      const double Uv = (r[6] * v[0] + r[7] * v[1]) + (r[8] * v[2] + r[9] * v[3]) + (r[10] * v[4] + r[11] * v[5]);
      const double x = ((c == 6 ? xb[f] : 0.0) - Uv) * r[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) v[k] += r[k] * x;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) sgm[g][c][k] = v[k];
  }
  __syncthreads();
  if (tid < kWave) {  // entry states from the root segment up
    const int cc = tid < 6 ? tid : 5;
    double a = 0.0;
    for (int gg = 0; gg < S; ++gg) {
      if (tid < 6) sgin[gg][tid] = a;
      double ak[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) ak[k] = __shfl(a, k);
      double na = sgm[gg][6][cc];
#pragma unroll
      for (int k = 0; k < 6; ++k) na += sgm[gg][k][cc] * ak[k];
      a = na;
    }
  }
  __syncthreads();
  if (grp && c == 0) {
    double a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] = sgin[g][k];
    for (int f = lo; f <= hi; ++f) {
      const double* r = tab[f];
      const double Ua = (r[6] * a[0] + r[7] * a[1]) + (r[8] * a[2] + r[9] * a[3]) + (r[10] * a[4] + r[11] * a[5]);
      const double x = (xb[f] - Ua) * r[12];
      xb[f] = x;
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] += r[k] * x;
    }
  }
  __syncthreads();
}

// x = H^{-1} b in O(n) by one thread (models of more than one wave): backward
// sweep u_f = b_f - s_f.p, p <- p + U_f u_f / D_f; forward sweep
// x_f = (u_f - U_f.a) / D_f, a <- a + s_f x_f; in place in xb (LDS).  The
// record of the next frame is read while the current one is used.
__device__ void aba_solve(const double (*tab)[kTab], double* xb, int nf) {
  if (nf <= 0) return;
  double p[6] = {0, 0, 0, 0, 0, 0};
  double t[13], b;
#pragma unroll
  for (int k = 0; k < 13; ++k) t[k] = tab[nf - 1][k];
  b = xb[nf - 1];
  for (int f = nf - 1; f >= 0; --f) {
    const int fn = f > 0 ? f - 1 : 0;
    double tn[13];
#pragma unroll
    for (int k = 0; k < 13; ++k) tn[k] = tab[fn][k];
    const double bn = xb[fn];
    const double sp = (t[0] * p[0] + t[1] * p[1]) + (t[2] * p[2] + t[3] * p[3]) + (t[4] * p[4] + t[5] * p[5]);
    const double u = b - sp;
    xb[f] = u;
    const double w = u * t[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] += t[6 + k] * w;
#pragma unroll
    for (int k = 0; k < 13; ++k) t[k] = tn[k];
    b = bn;
  }
  double a[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 13; ++k) t[k] = tab[0][k];
  b = xb[0];
  for (int f = 0; f < nf; ++f) {
    const int fn = f + 1 < nf ? f + 1 : f;
    double tn[13];
#pragma unroll
    for (int k = 0; k < 13; ++k) tn[k] = tab[fn][k];
    const double bn = xb[fn];
    const double Ua = (t[6] * a[0] + t[7] * a[1]) + (t[8] * a[2] + t[9] * a[3]) + (t[10] * a[4] + t[11] * a[5]);
    const double x = (b - Ua) * t[12];
    xb[f] = x;
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] += t[k] * x;
#pragma unroll
    for (int k = 0; k < 13; ++k) t[k] = tn[k];
    b = bn;
  }
}

// Branched models (one thread, frames in depth-first preorder, parent[f] < f):
// the articulated inertias accumulate the children's P_c into the parent,
//   I^A_f = I_f + sum_children P_c,  U_f = I^A_f s_f,  D_f = s_f.U_f,
//   P_f = I^A_f - U_f U_f^T / D_f;
// pacc [nf][21] (device scratch) holds the accumulated children's P.
__device__ void aba_setup_tree(const double* inert, double (*tab)[kTab], const int* parent, double* pacc, int nf) {
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k < 21; ++k) pacc[f * 21 + k] = 0.0;
  for (int f = nf - 1; f >= 0; --f) {
    double P[21], s[6], in[10];
#pragma unroll
    for (int k = 0; k < 21; ++k) P[k] = pacc[f * 21 + k];
#pragma unroll
    for (int k = 0; k < 10; ++k) in[k] = inert[f * 10 + k];
#pragma unroll
    for (int k = 0; k < 6; ++k) s[k] = tab[f][k];
#pragma unroll
    for (int k = 0; k < 6; ++k) P[k] += in[k];
    P[7] -= in[8]; P[8] += in[7]; P[9] += in[8]; P[11] -= in[6]; P[12] -= in[7]; P[13] += in[6];
    P[15] += in[9]; P[18] += in[9]; P[20] += in[9];
    double U[6];
    U[0] = P[0] * s[0] + P[1] * s[1] + P[2] * s[2] + P[6] * s[3] + P[7] * s[4] + P[8] * s[5];
    U[1] = P[1] * s[0] + P[3] * s[1] + P[4] * s[2] + P[9] * s[3] + P[10] * s[4] + P[11] * s[5];
    U[2] = P[2] * s[0] + P[4] * s[1] + P[5] * s[2] + P[12] * s[3] + P[13] * s[4] + P[14] * s[5];
    U[3] = P[6] * s[0] + P[9] * s[1] + P[12] * s[2] + P[15] * s[3] + P[16] * s[4] + P[17] * s[5];
    U[4] = P[7] * s[0] + P[10] * s[1] + P[13] * s[2] + P[16] * s[3] + P[18] * s[4] + P[19] * s[5];
    U[5] = P[8] * s[0] + P[11] * s[1] + P[14] * s[2] + P[17] * s[3] + P[19] * s[4] + P[20] * s[5];
    const double D = (s[0] * U[0] + s[1] * U[1]) + (s[2] * U[2] + s[3] * U[3]) + (s[4] * U[4] + s[5] * U[5]);
    const double iD = (D > 0.0) ? 1.0 / D : 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) tab[f][6 + k] = U[k];
    tab[f][12] = iD;
    const int p = parent[f];
    if (p >= 0) {
      double V[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) V[k] = U[k] * iD;
      P[0] -= U[0] * V[0]; P[1] -= U[0] * V[1]; P[2] -= U[0] * V[2];
      P[3] -= U[1] * V[1]; P[4] -= U[1] * V[2]; P[5] -= U[2] * V[2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) P[6 + 3 * r + c] -= U[r] * V[3 + c];
      P[15] -= U[3] * V[3]; P[16] -= U[3] * V[4]; P[17] -= U[3] * V[5];
      P[18] -= U[4] * V[4]; P[19] -= U[4] * V[5]; P[20] -= U[5] * V[5];
#pragma unroll
      for (int k = 0; k < 21; ++k) pacc[p * 21 + k] += P[k];
    }
  }
}

// The same recursion with a thread per frame, level by level: a frame of
// height h (the longest path down to a leaf) runs at round h, once every frame
// below it has passed its articulated inertia up.  Thread j (frame j, valid)
// sums the passed-up inertias of its children (c = j + 1, then the frame after
// each child's range), adds its own, forms U, D and 1/D into tab[j] and leaves
// P - U U^T / D at pacc[j] for its parent.  levels: the model's largest height;
// every thread of the workgroup calls it.
__device__ void aba_setup_tree_levels(const double* inert, double (*tab)[kTab], const int* fend, double* pacc, int j,
                                      bool valid, int hj, int levels) {
  for (int h = 0; h <= levels; ++h) {
    if (valid && hj == h) {
      double P[21];
#pragma unroll
      for (int k = 0; k < 21; ++k) P[k] = 0.0;
      for (int c = j + 1; c <= fend[j]; c = fend[c] + 1)
#pragma unroll
        for (int k = 0; k < 21; ++k) P[k] += pacc[c * 21 + k];
      double in[10], s[6];
#pragma unroll
      for (int k = 0; k < 10; ++k) in[k] = inert[j * 10 + k];
#pragma unroll
      for (int k = 0; k < 6; ++k) s[k] = tab[j][k];
#pragma unroll
      for (int k = 0; k < 6; ++k) P[k] += in[k];
      P[7] -= in[8]; P[8] += in[7]; P[9] += in[8]; P[11] -= in[6]; P[12] -= in[7]; P[13] += in[6];
      P[15] += in[9]; P[18] += in[9]; P[20] += in[9];
      double U[6];
      U[0] = P[0] * s[0] + P[1] * s[1] + P[2] * s[2] + P[6] * s[3] + P[7] * s[4] + P[8] * s[5];
      U[1] = P[1] * s[0] + P[3] * s[1] + P[4] * s[2] + P[9] * s[3] + P[10] * s[4] + P[11] * s[5];
      U[2] = P[2] * s[0] + P[4] * s[1] + P[5] * s[2] + P[12] * s[3] + P[13] * s[4] + P[14] * s[5];
      U[3] = P[6] * s[0] + P[9] * s[1] + P[12] * s[2] + P[15] * s[3] + P[16] * s[4] + P[17] * s[5];
      U[4] = P[7] * s[0] + P[10] * s[1] + P[13] * s[2] + P[16] * s[3] + P[18] * s[4] + P[19] * s[5];
      U[5] = P[8] * s[0] + P[11] * s[1] + P[14] * s[2] + P[17] * s[3] + P[19] * s[4] + P[20] * s[5];
      const double D = (s[0] * U[0] + s[1] * U[1]) + (s[2] * U[2] + s[3] * U[3]) + (s[4] * U[4] + s[5] * U[5]);
      const double iD = (D > 0.0) ? 1.0 / D : 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) tab[j][6 + k] = U[k];
      tab[j][12] = iD;
      double V[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) V[k] = U[k] * iD;
      P[0] -= U[0] * V[0]; P[1] -= U[0] * V[1]; P[2] -= U[0] * V[2];
      P[3] -= U[1] * V[1]; P[4] -= U[1] * V[2]; P[5] -= U[2] * V[2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) P[6 + 3 * r + c] -= U[r] * V[3 + c];
      P[15] -= U[3] * V[3]; P[16] -= U[3] * V[4]; P[17] -= U[3] * V[5];
      P[18] -= U[4] * V[4]; P[19] -= U[4] * V[5]; P[20] -= U[5] * V[5];
#pragma unroll
      for (int k = 0; k < 21; ++k) pacc[j * 21 + k] = P[k];
    }
    __threadfence_block();  // pacc goes through device memory
    __syncthreads();
  }
}

// x = H^{-1} b on a branched model (one thread, in place in xb): backward sweep
// in reverse preorder u_f = b_f - s_f.p_f, p_parent += p_f + U_f u_f / D_f;
// forward sweep in preorder x_f = (u_f - U_f.a_parent) / D_f, a_f = a_parent + s_f x_f.
// acc [nf][6] (LDS) holds p, then a.
__device__ void aba_solve_tree(const double (*tab)[kTab], double* xb, const int* parent, double (*acc)[6], int nf) {
  for (int f = 0; f < nf; ++f)
    for (int k = 0; k < 6; ++k) acc[f][k] = 0.0;
  for (int f = nf - 1; f >= 0; --f) {
    const double* t = tab[f];
    double p[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] = acc[f][k];
    const double sp = (t[0] * p[0] + t[1] * p[1]) + (t[2] * p[2] + t[3] * p[3]) + (t[4] * p[4] + t[5] * p[5]);
    const double u = xb[f] - sp;
    xb[f] = u;
    const double w = u * t[12];
    const int pa = parent[f];
    if (pa >= 0)
#pragma unroll
      for (int k = 0; k < 6; ++k) acc[pa][k] += p[k] + t[6 + k] * w;
  }
  for (int f = 0; f < nf; ++f) {
    const double* t = tab[f];
    const int pa = parent[f];
    double a[6] = {0, 0, 0, 0, 0, 0};
    if (pa >= 0)
#pragma unroll
      for (int k = 0; k < 6; ++k) a[k] = acc[pa][k];
    const double Ua = (t[6] * a[0] + t[7] * a[1]) + (t[8] * a[2] + t[9] * a[3]) + (t[10] * a[4] + t[11] * a[5]);
    const double x = (xb[f] - Ua) * t[12];
    xb[f] = x;
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[f][k] = a[k] + t[k] * x;
  }
}

// The recursion's two sweeps are the factorization H = L D L^T of a branched
// model's joint-space inertia in the world frame: with p_f summed over the
// frames below f, the backward sweep solves (I + N) u = b, N_fg = s_f.U_g / D_g
// for g below f, so u = L^-1 b with L = I + N; the forward sweep solves
// (D + N') x = u with N'_fg = U_f.s_g = D_f N_gf for g above f, i.e.
// D L^T x = u.  Hence H^-1 = L^-T D^-1 L^-1, and column j of L^-1 (the
// backward sweep of e_j) is nonzero on j and the frames above it only:
//   u_j = 1, then up the path  p <- p + U_g u_g / D_g,  u_a = -s_a.p.
// W holds row a of L^-1 over the frames below a (a contiguous preorder range
// [a, fend_a]) from wrow[a] on: entry (a, j) at W[wrow[a] + j - a].
// tree_inverse_factor: this thread's column j of L^-1 into W (every frame's
// thread at once; tab must hold s, U, 1/D of every frame of the model).
__device__ __forceinline__ void tree_inverse_factor(const double (*tab)[kTab], const int* parent, const int* wrow,
                                                    double* W, int j, bool valid) {
  if (!valid) return;
  double p[6] = {0, 0, 0, 0, 0, 0};
  double u = 1.0;
  int g = j;
  for (;;) {
    const double* t = tab[g];
    W[wrow[g] + (j - g)] = u;
    const double w = u * t[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) p[k] += t[6 + k] * w;
    g = parent[g];
    if (g < 0) break;
    const double* s = tab[g];
    u = -((s[0] * p[0] + s[1] * p[1]) + (s[2] * p[2] + s[3] * p[3]) + (s[4] * p[4] + s[5] * p[5]));
  }
}

// r = H^-1 v on a branched model from W (tree_inverse_factor): z = L^-1 v, row a
// of L^-1 times v over the frames below a; y = D^-1 z; r_j = sum over the
// frames a on the path from j up of (L^-1)_aj y_a.  Every thread of the
// workgroup calls it (lane j's frame: valid; fend_j: the last frame below it);
// xb, yb: LDS vectors of the model's frames.
__device__ __forceinline__ double tree_apply_inverse(const double (*tab)[kTab], const int* parent, const int* wrow,
                                                     const double* W, double* xb, double* yb, int j, int fend_j,
                                                     bool valid, double v) {
  if (valid) xb[j] = v;
  __syncthreads();
  if (valid) {
    // eight entries of the row requested before the first is used
    const double* row = W + wrow[j] - j;
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    int i = j;
    for (; i + 7 <= fend_j; i += 8) {
      double w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) w[k] = row[i + k];
#pragma unroll
      for (int k = 0; k < 8; ++k) z[k & 3] += w[k] * xb[i + k];
    }
    for (; i <= fend_j; ++i) z[0] += row[i] * xb[i];
    yb[j] = ((z[0] + z[1]) + (z[2] + z[3])) * tab[j][12];
  }
  __syncthreads();
  double r = 0.0;
  if (valid)
    for (int a = j; a >= 0; a = parent[a]) r += W[wrow[a] + (j - a)] * yb[a];
  __syncthreads();  // xb, yb are reused by the next product
  return r;
}

// Inputs of the inertia preconditioner at configuration q (float64): this
// frame's world spatial inertia about the origin and its joint motion (FX: a
// slide's motion is the pure translation (0; w), and a link's inertia is
// weighted by 1 + 2c, the Gauss-Newton weight of its kinetic and drag terms).
template <bool FX = false, typename S>
__device__ __forceinline__ void precond_frame(S& sc, const DevModel& d, double* inert, double* tab,
                                              const FrameGeo& geo, int f, bool valid, double q0);

// Setup of one step for this wave's model (float64): the per-step constant
// B = -2 A(q_k) + A(q_{k-1}) of every frame (FX: and A(q_k) itself where the
// model has drag or contact points), and for the inertia preconditioner its
// inputs at the warm start.
template <bool FX = false, typename S>
__device__ __forceinline__ void step_setup(S& sc, const DevModel& d, double* inert, double* tab, const FrameGeo& geo,
                                           int f, bool valid, double qkm1, double qk, double q0, bool use_aba) {
  double* B64 = d.B64 + (size_t)f * 12;
  float* B32 = d.B32 + (size_t)f * 12;
  {
    const Xf<double> Akm1 = fk_geo<double, FX>(sc, geo, valid, qkm1);
    if (valid)
#pragma unroll
      for (int k = 0; k < 12; ++k) B64[k] = Akm1.m[k];
  }
  {
    const Xf<double> Ak = fk_geo<double, FX>(sc, geo, valid, qk);
    if (valid)
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const double b = B64[k] - 2.0 * Ak.m[k];
        B64[k] = b;
        B32[k] = (float)b;
      }
    if (FX && valid && d.Ak64)
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        d.Ak64[(size_t)f * 12 + k] = Ak.m[k];
        d.Ak32[(size_t)f * 12 + k] = (float)Ak.m[k];
      }
  }
  if (use_aba) precond_frame<FX>(sc, d, inert, tab, geo, f, valid, q0);
}

template <bool FX, typename S>
__device__ __forceinline__ void precond_frame(S& sc, const DevModel& d, double* inert, double* tab,
                                              const FrameGeo& geo, int f, bool valid, double q0) {
  const double* a = geo.a;
  const Xf<double> A = fk_geo<double, FX>(sc, geo, valid, q0);
  double M[10];
  const double* rec = d.fr64 + (size_t)f * 16;
#pragma unroll
  for (int k = 0; k < 10; ++k) M[k] = ld_if(rec + 6 + k, valid);
  if (FX && valid && d.fdrag) {
    const double wgt = 1.0 + 2.0 * d.fdrag[f];
#pragma unroll
    for (int k = 0; k < 10; ++k) M[k] *= wgt;
  }
  const double ms = M[9];
  // world moment tensor: h = R (m c) + m t ; Sigma = R S R^T + R mc t^T + t (R mc)^T + m t t^T
  double Rmc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) Rmc[r] = A.m[4 * r] * M[3] + A.m[4 * r + 1] * M[6] + A.m[4 * r + 2] * M[8];
  const double t[3] = {A.m[3], A.m[7], A.m[11]};
  double Sw[6];  // 00 01 02 11 12 22
  {
    int k = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = r; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          const double RS = A.m[4 * r] * M[sym4(0, x)] + A.m[4 * r + 1] * M[sym4(1, x)] + A.m[4 * r + 2] * M[sym4(2, x)];
          acc += RS * A.m[4 * c + x];
        }
        Sw[k++] = acc + Rmc[r] * t[c] + t[r] * Rmc[c] + ms * t[r] * t[c];
      }
  }
  const double tr = Sw[0] + Sw[3] + Sw[5];
  double* in = inert;
  in[0] = valid ? tr - Sw[0] : 0.0;
  in[1] = valid ? -Sw[1] : 0.0;
  in[2] = valid ? -Sw[2] : 0.0;
  in[3] = valid ? tr - Sw[3] : 0.0;
  in[4] = valid ? -Sw[4] : 0.0;
  in[5] = valid ? tr - Sw[5] : 0.0;
  in[6] = valid ? Rmc[0] + ms * t[0] : 0.0;
  in[7] = valid ? Rmc[1] + ms * t[1] : 0.0;
  in[8] = valid ? Rmc[2] + ms * t[2] : 0.0;
  in[9] = valid ? ms : 0.0;
  const double w0 = A.m[0] * a[0] + A.m[1] * a[1] + A.m[2] * a[2];
  const double w1 = A.m[4] * a[0] + A.m[5] * a[1] + A.m[6] * a[2];
  const double w2 = A.m[8] * a[0] + A.m[9] * a[1] + A.m[10] * a[2];
  double* ts = tab;
  if (FX && geo.slide) {
    ts[0] = 0.0;
    ts[1] = 0.0;
    ts[2] = 0.0;
    ts[3] = w0;
    ts[4] = w1;
    ts[5] = w2;
    return;
  }
  ts[0] = valid ? w0 : 0.0;
  ts[1] = valid ? w1 : 0.0;
  ts[2] = valid ? w2 : 0.0;
  ts[3] = valid ? t[1] * w2 - t[2] * w1 : 0.0;
  ts[4] = valid ? t[2] * w0 - t[0] * w2 : 0.0;
  ts[5] = valid ? t[0] * w1 - t[1] * w0 : 0.0;
}

// Next trial step after a rejected one: backtracking with quadratic
// interpolation (the minimizer of the parabola through E(0), E'(0) = gd and
// E(alpha)), kept within [0.1, 0.5] alpha; halving when E(alpha) is not finite
// or the parabola has no interior minimum.  All values are wave-uniform.
__device__ __forceinline__ double next_alpha(double alpha, double E, double Et, double gd) {
  if (!isfinite(Et)) return 0.5 * alpha;
  const double den = 2.0 * (Et - E - gd * alpha);
  if (!(den > 0.0)) return 0.5 * alpha;
  const double aq = -gd * alpha * alpha / den;
  return aq < 0.1 * alpha ? 0.1 * alpha : (aq > 0.5 * alpha ? 0.5 * alpha : aq);
}

// Per-model state of the rollout kernel.
enum ModelState { kSetup = 0, kIterate = 1, kDone = 2 };

// A rollout of n_steps time steps, one model per workgroup of NW wavefronts
// (frame j in lane j % 64 of wave j / 64).  Every model advances through the
// steps at its own pace and a workgroup ends when its model has finished the
// last step, so the hardware dispatcher starts the next model in its place (the
// per-iteration interleaving of Sec. 5's GPU scheme, done by the dispatcher
// instead of a software queue).
// A step is: setup (B, and for the inertia preconditioner the recursion and,
// for one-wave chains, the explicit inverse in LDS), the warm-start evaluation,
// then iterations of two-loop L-BFGS direction + backtracking line search +
// update; every `refresh` accepted iterations the preconditioner is formed again
// at the iterate and the pairs are dropped.  The initial inverse Hessian is
// applied as a matrix-vector product from the explicit inverse (one-wave chains)
// or by the two sweeps of the recursion on one thread (longer chains, trees).
// The L-BFGS pairs live in LDS (one wave) or in the per-frame device ring.
// Workgroup b takes the b-th model in descending frame count (d.order).
// Every branch is uniform over the workgroup (all decisions use reduced values).
// MIXED: float32 evaluations until the line search meets float32 rounding,
// float32 claims convergence or the step's first preconditioner re-formation
// comes (a long float32 phase can leave a hard step far slower to finish in
// float64), then float64 to the end of the step.
// Two waves per SIMD: one-wave workgroups use up to 256 VGPRs (3 per SIMD
// needed <= 168 and spilled, and was slower).
constexpr int kWavesPerSimd = 2;
template <int NW>
struct ScanOf {
  using type = BlockScan<NW>;
  static __device__ __forceinline__ type make(double* xch, int wave, int lane) {
    type t;
    t.xch = xch;
    t.wave = wave;
    t.lane = lane;
    t.area = 0;
    return t;
  }
};
template <>
struct ScanOf<1> {
  using type = WaveScan;
  static __device__ __forceinline__ type make(double*, int, int) { return WaveScan{}; }
};

// LDS of the kernels that only evaluate (objective, poses): the scan buffers.
template <int NW, bool TREE>
struct ScanLds {
  double xch[2][NW][8];
  double tq[TREE ? kMaxFrames * NW : 1][4];
  double tv[TREE ? kMaxFrames * NW : 1][6];
  int tanc[TREE ? kMaxFrames * NW : 1];
  int tpar[TREE ? kMaxFrames * NW : 1];
};

// The scan policy of a model workgroup: DPP (+ LDS carries) for chains,
// pointer jumping and preorder ranges for branched models.
template <int NW, bool TREE>
struct ModelScan {
  using type = typename ScanOf<NW>::type;
  template <typename Lds>
  static __device__ __forceinline__ type make(Lds& L, const DevModel&, int wave, int lane, int, int, bool) {
    return ScanOf<NW>::make(&L.xch[0][0][0], wave, lane);
  }
};
template <int NW>
struct ModelScan<NW, true> {
  using type = TreeScan<NW>;
  template <typename Lds>
  static __device__ __forceinline__ type make(Lds& L, const DevModel& d, int wave, int lane, int j, int f,
                                              bool valid) {
    type t;
    t.xch = &L.xch[0][0][0];
    t.wave = wave;
    t.lane = lane;
    t.area = 0;
    t.tq = L.tq;
    t.tv = L.tv;
    t.tanc = L.tanc;
    t.j = j;
    t.parent = valid ? d.fpar[f] : -1;
    t.send = valid ? d.fend[f] : j;
    t.rounds = d.jump_rounds;
    L.tpar[j] = t.parent;
    __syncthreads();
    return t;
  }
};


// ------------------------------------------------------- second order --
__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Suffix sum over the frames at and below each lane (chain order = lane order).
__device__ __forceinline__ double wave_suffix_sum(double v) {
  const double pre = wave_prefix_sum(v);
  return (readlane(pre, 63) - pre) + v;
}

// Adjoint backward pass of Alg. 1 for a given seed S_l = dF/dA_l (3x4 per frame)
// at the configuration whose poses are A (world-frame form): returns
// dF/dq_n = w_n . (K_n - p_n x F_n) with the suffix sums of
// k = sum_c R[:,c] x S[:,c] + t x S[:,3] and f = S[:,3].
template <typename Sc>
__device__ double adjoint_of_seed(Sc& sc, const Xf<double>& A, const double S[12], const double a[3], bool valid) {
  const double t[3] = {A.m[3], A.m[7], A.m[11]};
  double k[3] = {0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double col[3] = {c < 3 ? A.m[c] : t[0], c < 3 ? A.m[4 + c] : t[1], c < 3 ? A.m[8 + c] : t[2]};
    const double s[3] = {S[c], S[4 + c], S[8 + c]};
    double x[3];
    cross3(col, s, x);
#pragma unroll
    for (int i = 0; i < 3; ++i) k[i] += x[i];
  }
  double KF[6] = {valid ? k[0] : 0.0, valid ? k[1] : 0.0, valid ? k[2] : 0.0,
                  valid ? S[3] : 0.0, valid ? S[7] : 0.0, valid ? S[11] : 0.0};
  double unused_a = 0.0, unused_b = 0.0;
  sc.suffix6_total2(KF, unused_a, unused_b);
  const double K[3] = {KF[0], KF[1], KF[2]}, F[3] = {KF[3], KF[4], KF[5]};
  double w[3], pF[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = A.m[4 * i] * a[0] + A.m[4 * i + 1] * a[1] + A.m[4 * i + 2] * a[2];
  cross3(t, F, pF);
  const double r = w[0] * (K[0] - pF[0]) + w[1] * (K[1] - pF[1]) + w[2] * (K[2] - pF[2]);
  return valid ? r : 0.0;
}

// Tangent of the poses along a DOF direction v (forward-mode Alg. 1):
// dA_j/dq_n = [[w_n]x R_j | w_n x (t_j - p_n)] for every frame n at or above j,
// so with the prefix sums W_j = sum v_n w_n and Z_j = sum v_n (w_n x p_n)
//   dR_j = [W_j]x R_j,   dt_j = W_j x t_j - Z_j.
template <typename Sc>
__device__ void tangent_pose(Sc& sc, const Xf<double>& A, const double a[3], bool valid, double v, double dA[12],
                             double W[3], double w[3]) {
  const double t[3] = {A.m[3], A.m[7], A.m[11]};
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = A.m[4 * i] * a[0] + A.m[4 * i + 1] * a[1] + A.m[4 * i + 2] * a[2];
  double wp[3];
  cross3(w, t, wp);
  const double vv = valid ? v : 0.0;
  double Z[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    W[i] = vv * w[i];
    Z[i] = vv * wp[i];
  }
  sc.prefix_sum3(W);
  sc.prefix_sum3(Z);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double col[3] = {A.m[c], A.m[4 + c], A.m[8 + c]};
    double x[3];
    cross3(W, col, x);
    dA[c] = x[0];
    dA[4 + c] = x[1];
    dA[8 + c] = x[2];
  }
  double Wt[3];
  cross3(W, t, Wt);
  dA[3] = Wt[0] - Z[0];
  dA[7] = Wt[1] - Z[1];
  dA[11] = Wt[2] - Z[2];
}

// Hessian-vector product of the step objective at q (float64): the derivative
// of the gradient g_n = w_n . (K_n - p_n x F_n) along v.  With the tangent
// poses dA and the tangent seed dG = dA M (the gravity part of the seed is
// constant),
//   dk = sum_c (dR[:,c] x G[:,c] + R[:,c] x dG[:,c]) + dt x G[:,3] + t x dG[:,3],
//   (Hv)_n = dw_n . (K_n - p_n x F_n) + w_n . (dK_n - dp_n x F_n - p_n x dF_n),
// dw_n = W_n x w_n, dp_n = dt_n.  Needs B of the step in the model scratch.
template <typename Sc>
__device__ double hess_vec(Sc& sc, const DevModel& d, const FrameGeo& geo, int f, bool valid, double q, double v,
                           double dt2) {
  asm volatile("" ::: "memory");
  double M[10], B[12];
  const double* rec = d.fr64 + (size_t)f * 16;
  const double* Bp = d.B64 + (size_t)f * 12;
#pragma unroll
  for (int k = 0; k < 10; ++k) M[k] = ld_if(rec + 6 + k, valid);
#pragma unroll
  for (int k = 0; k < 12; ++k) B[k] = ld_if(Bp + k, valid);
  const Xf<double> A = fk_geo<double>(sc, geo, valid, q);
  double dA[12], W[3], w[3];
  tangent_pose(sc, A, geo.a, valid, v, dA, W, w);
  const double g[3] = {d.gx, d.gy, d.gz};
  double G[12], dG[12];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double s = 0.0, ds = 0.0;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        s += (A.m[4 * r + x] + B[4 * r + x]) * M[sym4(x, c)];
        ds += dA[4 * r + x] * M[sym4(x, c)];
      }
      G[4 * r + c] = s - dt2 * g[r] * M[sym4(c, 3)];
      dG[4 * r + c] = ds;
    }
  double k[3] = {0, 0, 0}, dk[3] = {0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double col[3] = {A.m[c], A.m[4 + c], A.m[8 + c]};
    const double dcol[3] = {dA[c], dA[4 + c], dA[8 + c]};
    const double gc[3] = {G[c], G[4 + c], G[8 + c]};
    const double dgc[3] = {dG[c], dG[4 + c], dG[8 + c]};
    double x[3], y[3], z[3];
    cross3(col, gc, x);
    cross3(dcol, gc, y);
    cross3(col, dgc, z);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      k[i] += x[i];
      dk[i] += y[i] + z[i];
    }
  }
  double KF[6] = {valid ? k[0] : 0.0, valid ? k[1] : 0.0, valid ? k[2] : 0.0,
                  valid ? G[3] : 0.0, valid ? G[7] : 0.0, valid ? G[11] : 0.0};
  double dKF[6] = {valid ? dk[0] : 0.0, valid ? dk[1] : 0.0, valid ? dk[2] : 0.0,
                   valid ? dG[3] : 0.0, valid ? dG[7] : 0.0, valid ? dG[11] : 0.0};
  double unused_a = 0.0, unused_b = 0.0;
  sc.suffix6_total2(KF, unused_a, unused_b);
  sc.suffix6_total2(dKF, unused_a, unused_b);
  const double K[3] = {KF[0], KF[1], KF[2]}, F[3] = {KF[3], KF[4], KF[5]};
  const double dK[3] = {dKF[0], dKF[1], dKF[2]}, dF[3] = {dKF[3], dKF[4], dKF[5]};
  const double p[3] = {A.m[3], A.m[7], A.m[11]};
  const double dp[3] = {dA[3], dA[7], dA[11]};
  double dw[3], pF[3], dpF[3], pdF[3];
  cross3(W, w, dw);
  cross3(p, F, pF);
  cross3(dp, F, dpF);
  cross3(p, dF, pdF);
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) r += dw[i] * (K[i] - pF[i]) + w[i] * (dK[i] - dpF[i] - pdF[i]);
  return valid ? r : 0.0;
}

// B = A(q_{k-1}) - 2 A(q_k) of this lane's frame into the model scratch (FX:
// and A(q_k) where the model has drag or contact points).
template <bool FX = false, typename Sc>
__device__ __forceinline__ void write_B(Sc& sc, const DevModel& d, const FrameGeo& geo, int f, bool valid,
                                        double qkm1, double qk) {
  const Xf<double> Ak = fk_geo<double, FX>(sc, geo, valid, qk);
  const Xf<double> Akm1 = fk_geo<double, FX>(sc, geo, valid, qkm1);
  if (valid) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double b = Akm1.m[k] - 2.0 * Ak.m[k];
      d.B64[(size_t)f * 12 + k] = b;
      d.B32[(size_t)f * 12 + k] = (float)b;
    }
    if (FX && d.Ak64)
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        d.Ak64[(size_t)f * 12 + k] = Ak.m[k];
        d.Ak32[(size_t)f * 12 + k] = (float)Ak.m[k];
      }
  }
}

}  // namespace
