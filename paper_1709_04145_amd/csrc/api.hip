// api.hip -- host side of the C ABI in include/abd.h: model creation, argument checks,
// dispatch to the kernel launches.
#include "abd_device.h"

#include <algorithm>
#include <mutex>

namespace abd_impl {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int model_alloc(abd_model* m, void** dst, size_t bytes) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(1, bytes)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ABD_ENOMEM, "hipMalloc failed");
  }
  m->allocs.push_back(p);
  *dst = p;
  return ABD_OK;
}

}  // namespace abd_impl

using abd_impl::fail;
using abd_impl::g_err;

namespace {

template <typename T>
int upload(abd_model* m, T** dst, const std::vector<T>& src) {
  size_t bytes = std::max<size_t>(1, src.size()) * sizeof(T);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ABD_ENOMEM, "hipMalloc failed");
  }
  m->allocs.push_back(p);
  if (!src.empty() && hipMemcpy(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ABD_EDEVICE, "hipMemcpy to device failed");
  }
  *dst = static_cast<T*>(p);
  return ABD_OK;
}

template <typename T>
int alloc(abd_model* m, T** dst, size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ABD_ENOMEM, "hipMalloc failed");
  }
  m->allocs.push_back(p);
  *dst = static_cast<T*>(p);
  return ABD_OK;
}

void free_model(abd_model* m) {
  for (void* p : m->allocs) (void)hipFree(p);
  m->allocs.clear();
}

bool psd4(const double* u) {
  // symmetric 4x4 from the upper triangle; PSD test by pivoted LDL^T with tolerance
  static const int idx[16] = {0, 1, 2, 3, 1, 4, 5, 6, 2, 5, 7, 8, 3, 6, 8, 9};
  double A[4][4];
  double scale = 0.0;
  for (int i = 0; i < 16; ++i) {
    A[i / 4][i % 4] = u[idx[i]];
    scale = std::fmax(scale, std::fabs(u[idx[i]]));
  }
  const double tol = 1e-12 * (scale > 0 ? scale : 1.0);
  for (int k = 0; k < 4; ++k) {
    if (A[k][k] < -tol) return false;
    if (A[k][k] <= tol) {
      for (int j = k + 1; j < 4; ++j)
        if (std::fabs(A[k][j]) > 1e-6 * std::sqrt(scale) * std::sqrt(std::fabs(A[j][j]) + tol)) return false;
      continue;
    }
    for (int i = k + 1; i < 4; ++i) {
      const double l = A[i][k] / A[k][k];
      for (int j = k + 1; j < 4; ++j) A[i][j] -= l * A[k][j];
    }
  }
  return true;
}


int check_device(const abd_model* m) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != m->device) return fail(ABD_EINVAL, "current HIP device differs from the model's device");
  return ABD_OK;
}

int check_opts(const abd_step_opts* o, bool for_step) {
  if (!o) return fail(ABD_EINVAL, "opts is NULL");
  if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(ABD_EINVAL, "dt must be finite and > 0");
  if (o->precision != ABD_FP64 && o->precision != ABD_MIXED)
    return fail(ABD_EINVAL, "precision must be ABD_FP64 or ABD_MIXED");
  if (!for_step) return ABD_OK;
  if (o->order_K < 2) return fail(ABD_EINVAL, "order_K must be >= 2");
  if (o->order_K > 4) return fail(ABD_ENOTSUP, "order_K > 4 is not handled by this library");
  if (o->lbfgs_m < 1 || o->lbfgs_m > 10) return fail(ABD_EINVAL, "lbfgs_m must be in 1..10");
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(ABD_EINVAL, "tol must be finite and >= 0");
  if (o->max_iter < 0) return fail(ABD_EINVAL, "max_iter must be >= 0");
  if (o->max_ls < 1 || o->max_ls > 60) return fail(ABD_EINVAL, "max_ls must be in 1..60");
  if (o->precond != ABD_PRECOND_IDENTITY && o->precond != ABD_PRECOND_INERTIA)
    return fail(ABD_EINVAL, "precond must be ABD_PRECOND_IDENTITY or ABD_PRECOND_INERTIA");
  if (o->refresh < 0) return fail(ABD_EINVAL, "refresh must be >= 0");
  if (o->schedule != ABD_SCHEDULE_AUTO && o->schedule != ABD_SCHEDULE_WAVE && o->schedule != ABD_SCHEDULE_TILE)
    return fail(ABD_EINVAL, "schedule must be ABD_SCHEDULE_AUTO, ABD_SCHEDULE_WAVE or ABD_SCHEDULE_TILE");
  if (o->solver != ABD_SOLVER_LBFGS && o->solver != ABD_SOLVER_LM)
    return fail(ABD_EINVAL, "solver must be ABD_SOLVER_LBFGS or ABD_SOLVER_LM");

  return ABD_OK;
}

int check_rollout_args(const abd_model* m, const abd_step_opts* o, const double* q_init, const double* q_traj,
                       int n_steps) {
  int rc = check_opts(o, true);  // options first: they are checked without a device
  if (rc) return rc;
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  if (n_steps < 0) return fail(ABD_EINVAL, "n_steps must be >= 0");
  if (m->n_models == 0 || n_steps == 0) return ABD_OK;
  if (!q_init || !q_traj) return fail(ABD_EINVAL, "q_init and q_traj must not be NULL");
  const size_t nd = m->n_dofs;
  if (q_traj < q_init + 2 * nd && q_init < q_traj + (size_t)n_steps * (o->order_K - 1) * nd)
    return fail(ABD_EINVAL, "q_traj overlaps q_init");
  return check_device(m);
}

// Step scratch of abd_rollout_noalloc: one fixed array per device, held until the
// process ends.  Host code never uses the array's name as an address: the device
// address comes from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device).
int scratch_base(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(ABD_ENOTSUP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(ABD_EDEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[device];
  return ABD_OK;
}

// Zero the first n doubles of the scratch (a kernel, so that the clear is an
// ordinary node when a caller captures the stream in a graph).
__global__ void k_zero_scratch(double* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

}  // namespace

extern "C" {



const char* abd_last_error(void) { return g_err.c_str(); }

int abd_create_model(const abd_model_desc* desc, abd_model** out) {
  g_err.clear();
  if (!desc || !out) return fail(ABD_EINVAL, "desc and out must not be NULL");
  *out = nullptr;
  const int nm = desc->n_models;
  if (nm < 0) return fail(ABD_EINVAL, "n_models < 0");
  if (!desc->link_offset) return fail(ABD_EINVAL, "link_offset is NULL");
  if (desc->link_offset[0] != 0) return fail(ABD_EINVAL, "link_offset[0] must be 0");
  for (int i = 0; i < nm; ++i)
    if (desc->link_offset[i + 1] < desc->link_offset[i]) return fail(ABD_EINVAL, "link_offset must be non-decreasing");
  const int nl = desc->link_offset[nm];
  if (nl > 0 && (!desc->parent || !desc->dofs_per_link || !desc->axis || !desc->offset || !desc->mass_moment))
    return fail(ABD_EINVAL, "model arrays must not be NULL");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(desc->gravity[k])) return fail(ABD_EINVAL, "gravity must be finite");
  long long nd_ll = 0;
  for (int l = 0; l < nl; ++l) {
    const int k = desc->dofs_per_link[l];
    if (k < 1 || k > 6) return fail(ABD_EINVAL, "dofs_per_link must be in 1..6 (link " + std::to_string(l) + ")");
    nd_ll += k;
  }
  if (nd_ll > (1ll << 30)) return fail(ABD_EINVAL, "too many DOFs");
  const int nd = (int)nd_ll;

  std::vector<int> f0(nm + 1, 0), pose_link(nd, -1), link_dof(nl + 1, 0);
  for (int l = 0; l < nl; ++l) link_dof[l + 1] = link_dof[l] + desc->dofs_per_link[l];
  for (int i = 0; i <= nm; ++i) f0[i] = link_dof[desc->link_offset[i]];
  std::vector<double> fr64(16 * (size_t)nd, 0.0);
  bool chain = true;
  int max_frames = 0;
  for (int i = 0; i < nm; ++i) {
    const int lo = desc->link_offset[i], hi = desc->link_offset[i + 1];
    max_frames = std::max(max_frames, f0[i + 1] - f0[i]);
    for (int l = lo; l < hi; ++l) {
      const int p = desc->parent[l];
      if (p < -1 || p >= l - lo) return fail(ABD_EINVAL, "parent of link " + std::to_string(l) + " must precede it");
      if (p != l - lo - 1) chain = false;
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(desc->offset[3 * l + k])) return fail(ABD_EINVAL, "offset not finite");
      const double* u = desc->mass_moment + 10 * (size_t)l;
      for (int k = 0; k < 10; ++k)
        if (!std::isfinite(u[k])) return fail(ABD_EINVAL, "mass_moment not finite");
      if (!(u[9] > 0.0)) return fail(ABD_EINVAL, "mass of link " + std::to_string(l) + " must be > 0");
      if (!psd4(u)) return fail(ABD_EINVAL, "mass_moment of link " + std::to_string(l) + " is not PSD");
      const int d0 = link_dof[l], k = desc->dofs_per_link[l];
      for (int j = 0; j < k; ++j) {
        const double* a = desc->axis + 3 * (size_t)(d0 + j);
        const double nrm = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        if (!std::isfinite(nrm) || std::fabs(nrm - 1.0) > 1e-9)
          return fail(ABD_EINVAL, "axis of DOF " + std::to_string(d0 + j) + " must be a unit vector");
        for (int c = 0; c < 3; ++c) fr64[16 * (size_t)(d0 + j) + c] = a[c];
      }
      for (int c = 0; c < 3; ++c) fr64[16 * (size_t)d0 + 3 + c] = desc->offset[3 * (size_t)l + c];
      for (int c = 0; c < 10; ++c) fr64[16 * (size_t)(d0 + k - 1) + 6 + c] = u[c];
      pose_link[d0 + k - 1] = l;
    }
  }
  if (max_frames > kMaxFrames * kMaxWaves)
    return fail(ABD_ENOTSUP, "models with more than 1024 DOFs are not handled by this library");
  // optional terms: slides, drag, contact points
  bool any_slide = false, any_drag = false;
  if (desc->dof_kind)
    for (int f = 0; f < nd; ++f) {
      if (desc->dof_kind[f] != ABD_DOF_HINGE && desc->dof_kind[f] != ABD_DOF_SLIDE)
        return fail(ABD_EINVAL, "dof_kind of DOF " + std::to_string(f) + " must be ABD_DOF_HINGE or ABD_DOF_SLIDE");
      any_slide |= desc->dof_kind[f] == ABD_DOF_SLIDE;
    }
  if (desc->drag)
    for (int l = 0; l < nl; ++l) {
      if (!(desc->drag[l] >= 0.0) || !std::isfinite(desc->drag[l]))
        return fail(ABD_EINVAL, "drag of link " + std::to_string(l) + " must be finite and >= 0");
      any_drag |= desc->drag[l] != 0.0;
    }
  const int nc = desc->n_contacts;
  if (nc < 0) return fail(ABD_EINVAL, "n_contacts < 0");
  if (nc > 0) {
    if (!desc->contact_link || !desc->contact_point) return fail(ABD_EINVAL, "contact arrays must not be NULL");
    for (int c = 0; c < nc; ++c) {
      if (desc->contact_link[c] < 0 || desc->contact_link[c] >= nl)
        return fail(ABD_EINVAL, "contact_link of point " + std::to_string(c) + " out of range");
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(desc->contact_point[3 * (size_t)c + k])) return fail(ABD_EINVAL, "contact_point not finite");
    }
    const double* pl = desc->contact_plane;
    const double nrm = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
    if (!std::isfinite(nrm) || std::fabs(nrm - 1.0) > 1e-9 || !std::isfinite(pl[3]))
      return fail(ABD_EINVAL, "contact_plane must be a unit normal and a finite offset");
    if (!(desc->contact_d1 >= 0.0) || !std::isfinite(desc->contact_d1) || !(desc->contact_d2 >= 0.0) ||
        !std::isfinite(desc->contact_d2))
      return fail(ABD_EINVAL, "contact_d1 and contact_d2 must be finite and >= 0");
  }
  const bool fx = any_slide || any_drag || nc > 0;
  if (fx && max_frames > 4 * kMaxFrames)
    return fail(ABD_ENOTSUP, "models with slides, drag or contact points of more than 256 DOFs are not handled "
                             "by this library");
  if (!chain && max_frames > 4 * kMaxFrames)
    return fail(ABD_ENOTSUP, "branched models of more than 256 DOFs are not handled by this library");
  // Internal frame order: depth-first preorder of each model's links (children
  // in index order), the frames of a link consecutive, so that the frames below
  // any frame form a contiguous range.  For chains this is the caller's order.
  std::vector<int> uidx(nd), fpar(nd), fend(nd), fdepth(nd, 0);
  int max_depth = 1;
  for (int i = 0; i < nm; ++i) {
    const int lo = desc->link_offset[i], hi = desc->link_offset[i + 1], nlk = hi - lo;
    std::vector<std::vector<int>> kids(nlk);
    std::vector<int> stack, first(nlk), last(nlk), subend(nlk);
    for (int l = nlk - 1; l >= 0; --l) {
      const int p = desc->parent[lo + l];
      if (p < 0) stack.push_back(l);
      else kids[p].push_back(l);
    }
    for (auto& k : kids) std::reverse(k.begin(), k.end());  // pushed in reverse: pop in index order
    std::vector<int> order;
    while (!stack.empty()) {
      const int l = stack.back();
      stack.pop_back();
      order.push_back(l);
      for (int c : kids[l]) stack.push_back(c);
    }
    int pos = f0[i];
    for (int l : order) {
      const int k = desc->dofs_per_link[lo + l], p = desc->parent[lo + l];
      first[l] = pos;
      for (int jj = 0; jj < k; ++jj, ++pos) {
        uidx[pos] = link_dof[lo + l] + jj;
        fpar[pos] = jj > 0 ? pos - 1 - f0[i] : (p < 0 ? -1 : last[p] - f0[i]);
        fdepth[pos] = (fpar[pos] < 0 ? 0 : fdepth[f0[i] + fpar[pos]]) + 1;
        max_depth = std::max(max_depth, fdepth[pos]);
      }
      last[l] = pos - 1;
    }
    for (int t = (int)order.size() - 1; t >= 0; --t) {
      const int l = order[t];
      subend[l] = last[l];
      for (int c : kids[l]) subend[l] = std::max(subend[l], subend[c]);
      for (int fr = first[l]; fr <= last[l]; ++fr) fend[fr] = subend[l] - f0[i];
    }
  }
  int jump_rounds = 0;
  while ((1 << jump_rounds) < max_depth) ++jump_rounds;
  // per-frame records in internal order
  {
    std::vector<double> r(fr64.size());
    std::vector<int> pl(nd);
    for (int fr = 0; fr < nd; ++fr) {
      std::copy(fr64.begin() + 16 * (size_t)uidx[fr], fr64.begin() + 16 * (size_t)uidx[fr] + 16, r.begin() + 16 * (size_t)fr);
      pl[fr] = pose_link[uidx[fr]];
    }
    fr64.swap(r);
    pose_link.swap(pl);
  }
  // per-model preconditioner scratch: the per-frame spatial inertias (10 nf) of
  // a chain longer than one wave; inertias and recursion accumulators (31 nf) of
  // a branched model, then its explicit L^-1 by rows, row f over the frames
  // below f (wrow: where each row starts); one-wave chains keep theirs in LDS
  std::vector<long long> hoff(nm + 1, 0);
  std::vector<int> wrow(chain ? 0 : nd), fheight(chain ? 0 : nd, 0), mheight(chain ? 0 : nm, 0);
  if (!chain)
    for (int i = 0; i < nm; ++i)
      for (int fr = f0[i + 1] - 1; fr >= f0[i]; --fr) {
        if (fpar[fr] >= 0) fheight[f0[i] + fpar[fr]] = std::max(fheight[f0[i] + fpar[fr]], fheight[fr] + 1);
        mheight[i] = std::max(mheight[i], fheight[fr]);
      }
  for (int i = 0; i < nm; ++i) {
    const long long k = f0[i + 1] - f0[i];
    long long w = 0;
    if (!chain)
      for (int fr = f0[i]; fr < f0[i + 1]; ++fr) {
        wrow[fr] = (int)w;
        w += fend[fr] - (fr - f0[i]) + 1;
      }
    hoff[i + 1] = hoff[i] + (!chain ? 31 * k + w : k <= kMaxFrames ? 0 : 10 * k);
  }

  std::vector<int> order(nm);
  for (int i = 0; i < nm; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return f0[a + 1] - f0[a] > f0[b + 1] - f0[b]; });

  abd_model* m = new abd_model();
  HIP_TRY(hipGetDevice(&m->device));
  m->n_models = nm;
  m->n_links = nl;
  m->n_dofs = nd;
  m->max_frames = max_frames;
  m->tree = !chain;
  m->jump_rounds = jump_rounds;
  m->hinv_len = hoff[nm];
  m->f0_host = f0;
  for (int k = 0; k < 3; ++k) m->g[k] = desc->gravity[k];
  m->fx = fx;
  if (nc > 0) {
    for (int k = 0; k < 4; ++k) m->plane[k] = desc->contact_plane[k];
    m->cd1 = desc->contact_d1;
    m->cd2 = desc->contact_d2;
  }
  std::vector<float> fr32(fr64.begin(), fr64.end());
  // optional terms in internal frame order: slide flags, drag per frame (the link's
  // coefficient on the frame carrying its mass), contact points grouped by frame
  std::vector<signed char> fkind;
  std::vector<double> fdrag, cpt;
  std::vector<int> coff;
  if (any_slide) {
    fkind.assign(nd, 0);
    for (int fr = 0; fr < nd; ++fr) fkind[fr] = desc->dof_kind[uidx[fr]] == ABD_DOF_SLIDE ? 1 : 0;
  }
  if (any_drag) {
    fdrag.assign(nd, 0.0);
    for (int fr = 0; fr < nd; ++fr)
      if (pose_link[fr] >= 0) fdrag[fr] = desc->drag[pose_link[fr]];
  }
  if (nc > 0) {
    std::vector<int> frame_of_link(nl, 0);
    for (int fr = 0; fr < nd; ++fr)
      if (pose_link[fr] >= 0) frame_of_link[pose_link[fr]] = fr;
    coff.assign(nd + 1, 0);
    for (int c = 0; c < nc; ++c) coff[frame_of_link[desc->contact_link[c]] + 1]++;
    for (int fr = 0; fr < nd; ++fr) coff[fr + 1] += coff[fr];
    std::vector<int> fill(nd, 0);
    cpt.assign(3 * (size_t)nc, 0.0);
    for (int c = 0; c < nc; ++c) {
      const int fr = frame_of_link[desc->contact_link[c]], at = coff[fr] + fill[fr]++;
      for (int k = 0; k < 3; ++k) cpt[3 * (size_t)at + k] = desc->contact_point[3 * (size_t)c + k];
    }
  }
  int rc = ABD_OK;
  if ((rc = upload(m, &m->f0, f0)) || (rc = upload(m, &m->order, order)) ||
      (rc = upload(m, &m->pose_link, pose_link)) ||
      (rc = upload(m, &m->fr64, fr64)) || (rc = upload(m, &m->fr32, fr32)) ||
      (rc = alloc(m, &m->B64, 12 * (size_t)nd)) || (rc = alloc(m, &m->B32, 12 * (size_t)nd)) ||
      (rc = upload(m, &m->hoff, hoff)) || (rc = upload(m, &m->uidx, uidx)) ||
      (rc = upload(m, &m->fpar, fpar)) || (rc = upload(m, &m->fend, fend)) ||
      (!chain && ((rc = upload(m, &m->wrow, wrow)) || (rc = upload(m, &m->fheight, fheight)) ||
                  (rc = upload(m, &m->mheight, mheight)))) ||
      (rc = alloc(m, &m->hist, max_frames > kMaxFrames ? 2 * kMaxHist * (size_t)nd : 1)) ||
      (rc = alloc(m, &m->hinv, (size_t)hoff[nm])) ||
      (any_slide && (rc = upload(m, &m->fkind, fkind))) || (any_drag && (rc = upload(m, &m->fdrag, fdrag))) ||
      (nc > 0 && ((rc = upload(m, &m->coff, coff)) || (rc = upload(m, &m->cpt, cpt)))) ||
      ((any_drag || nc > 0) &&
       ((rc = alloc(m, &m->Ak64, 12 * (size_t)nd)) || (rc = alloc(m, &m->Ak32, 12 * (size_t)nd))))) {
    free_model(m);
    delete m;
    return rc;
  }
  // lanes without a frame read frame 0's B of their model (times a zero mass
  // moment): keep the buffers finite from the start
  if (nd > 0 && (hipMemset(m->B64, 0, 12 * (size_t)nd * sizeof(double)) != hipSuccess ||
                 hipMemset(m->B32, 0, 12 * (size_t)nd * sizeof(float)) != hipSuccess)) {
    (void)hipGetLastError();
    free_model(m);
    delete m;
    return fail(ABD_EDEVICE, "hipMemset failed");
  }
  *out = m;
  return ABD_OK;
}

void abd_destroy_model(abd_model* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  free_model(m);
  delete m;
}

int abd_model_info(const abd_model* m, int* n_models, int* n_links, int* n_dofs) {
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  if (n_models) *n_models = m->n_models;
  if (n_links) *n_links = m->n_links;
  if (n_dofs) *n_dofs = m->n_dofs;
  return ABD_OK;
}


int abd_step(abd_model* m, const abd_step_opts* o, const double* q_hist, const double* tau, double* q_out,
             abd_step_stats* stats, void* stream) {
  g_err.clear();
  int rc = check_opts(o, true);  // options first: they are checked without a device
  if (rc) return rc;
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  if (m->n_models == 0) return ABD_OK;
  if (!q_hist || !q_out) return fail(ABD_EINVAL, "q_hist and q_out must not be NULL");
  const size_t out_len = (size_t)(o->order_K - 1) * m->n_dofs;
  if (q_out < q_hist + 2 * (size_t)m->n_dofs && q_hist < q_out + out_len)
    return fail(ABD_EINVAL, "q_out overlaps q_hist");
  if ((rc = check_device(m))) return rc;
  if (m->fx && (o->order_K > 2 || o->solver == ABD_SOLVER_LM)) return fail(ABD_ENOTSUP, "models with slides, drag or contact points take order_K = 2 with ABD_SOLVER_LBFGS in this library");
  if (o->order_K > 2 && o->solver == ABD_SOLVER_LM)
    return abd_impl::launch_lm_hoc(m, o, q_hist, q_hist + m->n_dofs, tau, q_out, stats, 1, stream);
  if (o->order_K > 2) return abd_impl::launch_hoc(m, o, q_hist, q_hist + m->n_dofs, tau, q_out, stats, 1, stream);
  if (o->solver == ABD_SOLVER_LM)
    return abd_impl::launch_lm2(m, o, q_hist, q_hist + m->n_dofs, tau, q_out, stats, 1, stream);
  return abd_impl::launch_rollout(m, o, q_hist, q_hist + m->n_dofs, tau, q_out, stats, 1, stream);
}

int abd_rollout(abd_model* m, const abd_step_opts* o, const double* q_init, const double* tau, double* q_traj,
                abd_step_stats* stats, int n_steps, void* stream) {
  g_err.clear();
  int rc = check_rollout_args(m, o, q_init, q_traj, n_steps);
  if (rc || m->n_models == 0 || n_steps == 0) return rc;
  const size_t nd = m->n_dofs;
  if (m->fx && (o->order_K > 2 || o->solver == ABD_SOLVER_LM)) return fail(ABD_ENOTSUP, "models with slides, drag or contact points take order_K = 2 with ABD_SOLVER_LBFGS in this library");
  if (o->order_K > 2 && o->solver == ABD_SOLVER_LM)
    return abd_impl::launch_lm_hoc(m, o, q_init, q_init + nd, tau, q_traj, stats, n_steps, stream);
  if (o->order_K > 2) return abd_impl::launch_hoc(m, o, q_init, q_init + nd, tau, q_traj, stats, n_steps, stream);
  if (o->solver == ABD_SOLVER_LM)
    return abd_impl::launch_lm2(m, o, q_init, q_init + nd, tau, q_traj, stats, n_steps, stream);
  return abd_impl::launch_rollout(m, o, q_init, q_init + nd, tau, q_traj, stats, n_steps, stream);
}

int abd_rollout_noalloc(abd_model* m, const abd_step_opts* o, const double* q_init, const double* tau,
                        double* q_traj, abd_step_stats* stats, int n_steps, void* stream) {
  g_err.clear();
  int rc = check_rollout_args(m, o, q_init, q_traj, n_steps);
  if (rc || m->n_models == 0 || n_steps == 0) return rc;
  if (o->order_K > 2 && (rc = abd_impl::check_hoc(m, o))) return rc;
  if (o->solver == ABD_SOLVER_LM)
    return fail(ABD_ENOTSUP, "abd_rollout_noalloc: ABD_SOLVER_LM keeps dense per-model matrices (use abd_rollout)");
  if (m->fx)
    return fail(ABD_ENOTSUP, "abd_rollout_noalloc: models with slides, drag or contact points keep per-step "
                             "poses in model memory (use abd_rollout)");
  // carve the step scratch out of this device's static array
  unsigned char* base = nullptr;
  if ((rc = scratch_base(m->device, &base))) return rc;
  const size_t nd = m->n_dofs;
  const bool ring = m->max_frames > kMaxFrames;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  abd_impl::StepScratch sc;
  sc.B64 = reinterpret_cast<double*>(take(12 * nd * sizeof(double)));
  sc.B32 = reinterpret_cast<float*>(take(12 * nd * sizeof(float)));
  const size_t cleared = off;  // the per-frame constants start finite (zero)
  sc.hist = reinterpret_cast<double*>(take((ring ? 2 * kMaxHist * nd : 1) * sizeof(double)));
  sc.hinv = reinterpret_cast<double*>(take(std::max<long long>(1, m->hinv_len) * sizeof(double)));
  sc.Bk = nullptr;
  sc.hist3 = nullptr;
  if (o->order_K > 2) {
    sc.Bk = reinterpret_cast<double*>(take(36 * nd * sizeof(double)));
    if (ring) sc.hist3 = reinterpret_cast<double*>(take(2 * kMaxHist * 3 * nd * sizeof(double)));
  }
  if (off > kScratchBytes)
    return fail(ABD_ENOTSUP, "abd_rollout_noalloc: this model needs " + std::to_string(off) +
                                 " bytes of step scratch; the static buffer holds " +
                                 std::to_string(kScratchBytes) + " (use abd_rollout)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t words = cleared / sizeof(double);
  const int blocks = (int)std::min<size_t>(1024, (words + 255) / 256);
  hipLaunchKernelGGL(k_zero_scratch, dim3(std::max(1, blocks)), dim3(256), 0, s,
                     reinterpret_cast<double*>(base), words);
  HIP_TRY(hipGetLastError());
  if (o->order_K > 2)
    return abd_impl::launch_hoc(m, o, q_init, q_init + nd, tau, q_traj, stats, n_steps, stream, &sc);
  return abd_impl::launch_rollout(m, o, q_init, q_init + nd, tau, q_traj, stats, n_steps, stream, &sc);
}

int abd_objective_grad(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist,
                       const double* tau, double* E, double* grad, double* grad_tau, void* stream) {
  g_err.clear();
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  int rc = check_opts(o, false);
  if (rc) return rc;
  if (m->n_models == 0) return ABD_OK;
  if (!q || !q_hist || !E) return fail(ABD_EINVAL, "q, q_hist and E must not be NULL");
  if ((rc = check_device(m))) return rc;
  if (o->order_K < 2) return fail(ABD_EINVAL, "order_K must be >= 2");
  if (o->order_K > 4) return fail(ABD_ENOTSUP, "order_K > 4 is not handled by this library");
  if (m->fx && o->order_K > 2)
    return fail(ABD_ENOTSUP, "slides, drag and contact points enter the order-2 objective (Eq. EQ) only");
  if (o->order_K > 2) return abd_impl::launch_hoc_objective(m, o, q, q_hist, tau, E, grad, grad_tau, stream);
  return abd_impl::launch_objective(m, o, q, q_hist, tau, E, grad, grad_tau, stream);
}

int abd_hvp(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist, const double* v,
            double* Hv, void* stream) {
  g_err.clear();
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  int rc = check_opts(o, false);
  if (rc) return rc;
  if (m->n_models == 0) return ABD_OK;
  if (!q || !q_hist || !v || !Hv) return fail(ABD_EINVAL, "q, q_hist, v and Hv must not be NULL");
  if (m->max_frames > kMaxFrames || m->tree || m->fx)
    return fail(ABD_ENOTSUP, "abd_hvp handles serial hinge chains of at most 64 DOFs without drag or contact "
                             "points in this library");
  if ((rc = check_device(m))) return rc;
  return abd_impl::launch_hvp(m, o, q, q_hist, v, Hv, stream);
}

int abd_hessian(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist, double* H,
                void* stream) {
  g_err.clear();
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  int rc = check_opts(o, false);
  if (rc) return rc;
  if (m->n_models == 0) return ABD_OK;
  if (!q || !q_hist || !H) return fail(ABD_EINVAL, "q, q_hist and H must not be NULL");
  if (m->fx) return fail(ABD_ENOTSUP, "abd_hessian handles models without slides, drag or contact points");
  if ((rc = check_device(m))) return rc;
  return abd_impl::launch_hessian(m, o, q, q_hist, H, stream);
}

int abd_rollout_vjp(abd_model* m, const abd_step_opts* o, const double* q_init, const double* q_traj,
                    const double* dL_dq_traj, double* dL_dq_init, double* dL_dtau, abd_step_stats* stats,
                    int n_steps, void* stream) {
  g_err.clear();
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  int rc = check_opts(o, false);
  if (rc) return rc;
  if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(ABD_EINVAL, "tol must be finite and >= 0");
  if (o->max_iter < 0) return fail(ABD_EINVAL, "max_iter must be >= 0");
  if (o->precond != ABD_PRECOND_IDENTITY && o->precond != ABD_PRECOND_INERTIA)
    return fail(ABD_EINVAL, "precond must be ABD_PRECOND_IDENTITY or ABD_PRECOND_INERTIA");
  if (n_steps < 1) return fail(ABD_EINVAL, "n_steps must be >= 1");
  if (m->n_models == 0) return ABD_OK;
  if (!q_init || !q_traj || !dL_dq_traj || !dL_dq_init)
    return fail(ABD_EINVAL, "q_init, q_traj, dL_dq_traj and dL_dq_init must not be NULL");
  if (m->max_frames > kMaxFrames || m->tree || m->fx)
    return fail(ABD_ENOTSUP, "abd_rollout_vjp handles serial hinge chains of at most 64 DOFs without drag or "
                             "contact points in this library");
  if ((rc = check_device(m))) return rc;
  return abd_impl::launch_rollout_vjp(m, o, q_init, q_traj, dL_dq_traj, dL_dq_init, dL_dtau, stats, n_steps,
                                      stream);
}

int abd_poses(abd_model* m, const double* q, double* poses, void* stream) {
  g_err.clear();
  if (!m) return fail(ABD_EINVAL, "model is NULL");
  if (m->n_models == 0) return ABD_OK;
  if (!q || !poses) return fail(ABD_EINVAL, "q and poses must not be NULL");
  int rc = check_device(m);
  if (rc) return rc;
  return abd_impl::launch_poses(m, q, poses, stream);
}

}  // extern "C"
