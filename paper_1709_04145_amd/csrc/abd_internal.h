// abd_internal.h -- declarations shared by the translation units of the library:
// the model handle behind the opaque abd_model of include/abd.h, error reporting
// and the kernel launches each unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/abd.h"

struct abd_model {
  int device = 0;
  int n_models = 0, n_links = 0, n_dofs = 0, max_frames = 0, jump_rounds = 0;
  bool tree = false;
  double g[3] = {0, 0, 0};
  // device buffers
  int* f0 = nullptr;
  int* order = nullptr;
  int* pose_link = nullptr;
  double* fr64 = nullptr;
  float* fr32 = nullptr;
  double* B64 = nullptr;
  float* B32 = nullptr;
  long long* hoff = nullptr;
  double* hinv = nullptr;
  double* hist = nullptr;
  double* Bk = nullptr;  // known seed parts of order-K steps, allocated on first use
  double* hist3 = nullptr;  // order-K pairs of models of more than 64 DOFs, on first use
  long long hinv_len = 0;  // doubles of preconditioner scratch (hinv) the model needs
  std::vector<int> f0_host; // [n_models+1] first frame of every model
  double* lm_mat = nullptr;     // Levenberg-Marquardt matrices per model, on first use
  long long* lm_off = nullptr;  // [n_models+1] start of every model's matrices
  long long* sq_off = nullptr;  // [n_models+1] start of every model's n_i x n_i block, on first use
  int* uidx = nullptr;
  int* fpar = nullptr;
  int* fend = nullptr;
  int* wrow = nullptr;  // branched models: row offsets of the explicit L^-1 of the preconditioner
  int* fheight = nullptr;  // branched models: frame heights (longest path down to a leaf)
  int* mheight = nullptr;  // branched models: largest frame height of each model
  // optional terms (slides, drag, contact points); fx = any of them present
  bool fx = false;
  signed char* fkind = nullptr;  // [n_dofs] 1 = slide, internal frame order; NULL: all hinges
  double* fdrag = nullptr;       // [n_dofs] drag coefficient per frame; NULL: no drag
  int* coff = nullptr;           // [n_dofs+1] contact points per frame; NULL: none
  double* cpt = nullptr;         // [n_contacts][3]
  double* Ak64 = nullptr;        // [n_dofs][12] per-step A(q_k) (drag, friction)
  float* Ak32 = nullptr;
  double plane[4] = {0, 0, 1, 0};
  double cd1 = 0.0, cd2 = 0.0;
  // ABD_SCHEDULE_AUTO: the schedule the autotuner chose per precision (FP64,
  // MIXED): -1 not yet timed, 0 WAVE, 16 or 32 TILE; its scratch trajectory
  int tile_choice[2] = {-1, -1};
  double* tune_buf = nullptr;
  size_t tune_len = 0;
  std::vector<void*> allocs;
};

namespace abd_impl {

// Record msg as the calling thread's last error and return code.
int fail(int code, const std::string& msg);

// Device allocation owned by the model (freed with it); ABD_ENOMEM on failure.
int model_alloc(abd_model* m, void** dst, size_t bytes);

// Where the kernels of a step or rollout keep the buffers they write besides their
// inputs and outputs.  Without one (nullptr) they use the model's own buffers, the
// order-K ones allocated on first use.
struct StepScratch {
  double* B64;    // [n_dofs][12]
  float* B32;     // [n_dofs][12]
  double* hist;   // models of more than 64 frames: [n_dofs][2*kMaxHist]
  double* hinv;   // [hinv_len]
  double* Bk;     // order K > 2: [n_dofs][3][12]
  double* hist3;  // order K > 2, models of more than 64 frames: [n_dofs][2][kMaxHist][3]
};

// Kernel launches (stream-ordered; arguments already validated by the caller).
int launch_rollout(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
                   const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream,
                   const StepScratch* sc = nullptr);
int launch_hoc(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
               const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream,
               const StepScratch* sc = nullptr);
int launch_lm_hoc(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
                  const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream);
int launch_lm2(abd_model* m, const abd_step_opts* o, const double* q_prev, const double* q_curr,
               const double* tau, double* q_out, abd_step_stats* stats, int n_steps, void* stream);
int launch_hessian(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist, double* H,
                   void* stream);
int launch_hoc_objective(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist,
                         const double* tau, double* E, double* grad, double* grad_tau, void* stream);
int launch_objective(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist,
                     const double* tau, double* E, double* grad, double* grad_tau, void* stream);
int launch_poses(abd_model* m, const double* q, double* poses, void* stream);
int launch_hvp(abd_model* m, const abd_step_opts* o, const double* q, const double* q_hist, const double* v,
               double* Hv, void* stream);
int launch_rollout_vjp(abd_model* m, const abd_step_opts* o, const double* q_init, const double* q_traj,
                       const double* dL_dq_traj, double* dL_dq_init, double* dL_dtau, abd_step_stats* stats,
                       int n_steps, void* stream);
int check_hoc(const abd_model* m, const abd_step_opts* o);

}  // namespace abd_impl

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      (void)hipGetLastError(); /* reported here: do not leave it for the caller */ \
      return abd_impl::fail(ABD_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    }                                                                              \
  } while (0)
