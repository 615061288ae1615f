/*
 * abd.h -- C ABI of the MI355X (gfx950) library for position-based articulated
 * dynamics (Pan & Manocha, "Time Integrating Articulated Body Dynamics Using
 * Position-Based Collocation Methods").
 *
 * One time step of a batch of articulated models solves, per model,
 *     q_{k+1} = argmin_q  E(q)                                  (Sec. 4, Eq. EQ)
 *     E(q) = sum_l 1/2 tr(D_l M_l D_l^T) - dt^2 sum_l g^T A_l(q) M_l e4 - dt^2 tau.q
 *     D_l  = A_l(q) - 2 A_l(q_k) + A_l(q_{k-1})
 * i.e. dt^2 times the paper's energy: the kinetic term of the second-order
 * position-based discretisation integrated exactly over each body through its
 * mass moment tensor M_l = int rho (p;1)(p;1)^T dp (Eq. ATOM), plus gravity and
 * an optional generalized joint force tau.  A_l = [R_l | t_l] is the world pose
 * of link l (forward kinematics, Alg. 1 forward pass).  The minimizer satisfies
 * the stationarity condition Eq. PBAD.  The solver is a quasi-Newton method
 * (L-BFGS, Sec. 5) whose gradient is the adjoint backward pass of Alg. 1.
 *
 * Conventions common to every call
 * - All pointers passed to abd_step / abd_objective_grad are DEVICE pointers on
 *   the device the model was created on; the caller owns them.  Work is enqueued
 *   on `stream` (a hipStream_t; NULL = the default stream) and the call returns
 *   after enqueueing; results are valid once the stream reaches that point.
 * - DOF vectors are float64 [n_dofs] in the model's DOF order (link-major, the
 *   DOFs of link l in the order of its axes).
 * - Return value: ABD_OK, or a negative code; abd_last_error() then describes it.
 *   Argument errors are detected on the host before anything is enqueued.
 *   Per-model numerical outcomes are reported in abd_step_stats.flag, never in
 *   the return code.
 * - Concurrent calls on one model from several host threads are not supported:
 *   a model owns per-step scratch memory.
 */
#ifndef ABD_H
#define ABD_H

#ifdef __cplusplus
extern "C" {
#endif

#define ABD_OK 0
#define ABD_EINVAL (-1)   /* invalid argument */
#define ABD_ENOMEM (-2)   /* device allocation failed */
#define ABD_EDEVICE (-3)  /* HIP runtime error */
#define ABD_ENOTSUP (-4)  /* valid input that this library does not handle */

#define ABD_FP64 0        /* every operation in double precision */
#define ABD_MIXED 1       /* kinematics and energy terms in float32 until the
                             line search reaches float32 rounding (at most until
                             the step's first preconditioner re-formation), then
                             double;
                             for one-wave chains whose articulated pivots span at
                             most 1e5, the inertia preconditioner's explicit
                             inverse is kept in float32 (it shapes the search
                             directions only, not the converged solution).
                             order_K > 2: the forward kinematics in float32 (the
                             seeds, residuals and gradient from the widened poses
                             in double) until the gradient has dropped to 1e-3 of
                             the warm start's, float32 claims convergence, meets
                             its rounding or gives no descent, then double with
                             the L-BFGS history restarted */

/* schedules (abd_step_opts.schedule): how models are mapped onto the GPU */
#define ABD_SCHEDULE_AUTO 0 /* the library picks: for the order-2 L-BFGS step of a
                               batch of serial chains of at most 32 DOFs, the faster
                               of WAVE and TILE, timed on the first (up to 8) steps of
                               the model handle's first call at each precision (that call
                               then synchronizes its stream once; under graph capture,
                               and in abd_rollout_noalloc before a first timed call,
                               WAVE is taken); otherwise WAVE */
#define ABD_SCHEDULE_WAVE 1 /* one model per workgroup of the fewest wavefronts (64
                               frames each) that hold the batch's longest model,
                               models dispatched longest first (Sec. 5 "GPU
                               Parallelization": one workgroup per trajectory) */
#define ABD_SCHEDULE_TILE 2 /* serial chains of at most 32 DOFs packed 4 (<= 16 DOFs)
                               or 2 per wavefront, each model in its own lanes and
                               branching on its own; other batches: ABD_ENOTSUP.
                               Every schedule gives the same results, bit for bit;
                               solvers other than order-2 L-BFGS ignore the choice. */

/* optimizers (abd_step_opts.solver), Sec. 5 "Optimization Algorithm" */
#define ABD_SOLVER_LBFGS 0  /* L-BFGS (two-loop recursion) with a backtracking line search */
#define ABD_SOLVER_LM 1     /* Levenberg-Marquardt (Sec. 5), ABD_FP64 only (ABD_ENOTSUP
                               otherwise): (J^T J + lambda I) v = -grad E with a
                               per-model Cholesky factorization; lambda by
                               Nielsen's gain-ratio rule (initial 1e-3 max diag(J^T J), at
                               least 1e-15 of it); a step is accepted when it decreases E.
                               Order 2 (Eq. EQ, an integral of squares): J^T J is the
                               joint-space inertia H_q(q), one objective evaluation per
                               iteration.  Order 3 (Eq. EQHOC, a sum of squares of the
                               residuals r): the explicit Jacobian of r, plus half the
                               geodesic acceleration of Transtrum & Sethna's variant
                               (finite-difference step 0.1, steps with 2|a| > 0.75|v|
                               rejected); order 4 is rejected (ABD_ENOTSUP).  max_iter
                               counts iterations, accepted or rejected; stats evaluations
                               count objective (order 2) or residual evaluations; flag 2 =
                               lambda overflow or an accepted point equal to the iterate.
                               lbfgs_m, max_ls, precond and refresh are ignored.  Device
                               memory: 27 n_i^2 doubles per model, on first use. */

#define ABD_PRECOND_IDENTITY 0 /* L-BFGS initial inverse Hessian gamma*I */
#define ABD_PRECOND_INERTIA 2  /* initial inverse Hessian = inverse joint-space
                                  inertia, formed at the warm start and re-formed
                                  at the iterate every opts->refresh iterations */

/* per-model outcome flags */
#define ABD_FLAG_CONVERGED 1   /* |g| <= tol * |g(q0)| */
#define ABD_FLAG_LS_FLOOR 2    /* no step accepted by the line search, or the accepted point
                                  equals the iterate in every coordinate (no progress possible
                                  at float64 precision) */
#define ABD_FLAG_MAX_ITER 4    /* max_iter iterations done */
#define ABD_FLAG_NONFINITE 8   /* objective or gradient not finite at the warm start */

typedef struct abd_model abd_model;

/* Host-side description of a batch of models (copied by abd_create_model). */
typedef struct {
  int n_models;
  const int* link_offset;     /* [n_models+1], link_offset[0]=0; links of model i are
                                 link_offset[i] .. link_offset[i+1]-1 */
  const int* parent;          /* [n_links] parent link index within the model, -1 =
                                 fixed world frame; a parent precedes its children */
  const int* dofs_per_link;   /* [n_links] 1..6 consecutive elementary DOFs per joint */
  const double* axis;         /* [3*n_dofs] unit axis of each DOF, expressed in the frame
                                 it moves (link-major DOF order) */
  const double* offset;       /* [3*n_links] joint origin in the parent link frame */
  const double* mass_moment;  /* [10*n_links] upper triangle (row-major) of the symmetric
                                 positive semi-definite 4x4 M_l with M_l[3][3] = mass > 0 */
  double gravity[3];          /* gravitational acceleration (world frame) */
  /* Optional terms of Sec. 6's applications (NULL / 0: absent).  A model that
     uses any of them ("extras") takes abd_step / abd_rollout at order_K = 2
     with ABD_SOLVER_LBFGS, abd_objective_grad and abd_poses; every other entry
     point returns ABD_ENOTSUP for it, and it may have at most 256 DOFs. */
  const int* dof_kind;        /* [n_dofs] ABD_DOF_HINGE (rotation about the axis) or
                                 ABD_DOF_SLIDE (translation along it; the frame does
                                 not rotate); NULL = all hinges.  A 6-DOF floating root
                                 is a root link with three slides and three hinges. */
  const double* drag;         /* [n_links] drag coefficient c_l >= 0 (finite): adds
                                 c_l tr((A_l(q) - A_l(q_k)) M_l (A_l(q) - A_l(q_k))^T), which
                                 is dt^2 times the drag potential D |(P(q) - P(q_k))/dt|^2
                                 of Sec. 6 integrated over the body, c_l = D / rho_l;
                                 NULL = none */
  int n_contacts;             /* discrete contact points (>= 0) */
  const int* contact_link;    /* [n_contacts] global link index of each point */
  const double* contact_point;/* [3*n_contacts] point in its link's frame */
  double contact_plane[4];    /* n (unit, world) and h: the obstacle is n.x < h */
  double contact_d1;          /* D1 >= 0, normal penalty of Eq. FRI */
  double contact_d2;          /* D2 >= 0, friction penalty of Eq. FRI: each point adds
                                 dt^2 D1 d^2 + D2 d^2 |(I - n n^T)(x(q) - x(q_k))|^2,
                                 d = max(0, h - n.x) its penetration depth */
} abd_model_desc;

#define ABD_DOF_HINGE 0
#define ABD_DOF_SLIDE 1

typedef struct {
  double dt;         /* time step > 0 */
  int order_K;       /* collocation order K: 2 = Eq. EQ (one unknown configuration per
                        step); 3, 4 = Eq. EQHOC with K-1 unknown configurations per
                        step (models of <= 256 DOFs); other values are
                        rejected (EINVAL below 2, ENOTSUP above 4) */
  int lbfgs_m;       /* L-BFGS history length, 1..10 */
  double tol;        /* stop when |grad| <= tol * |grad at the warm start| */
  int max_iter;      /* L-BFGS iterations per step, >= 0 */
  int max_ls;        /* line-search halvings per iteration, 1..60 */
  int precision;     /* ABD_FP64 or ABD_MIXED */
  int precond;       /* ABD_PRECOND_IDENTITY or ABD_PRECOND_INERTIA */
  int refresh;       /* ABD_PRECOND_INERTIA, order_K = 2: every `refresh` accepted
                        iterations of a step, re-form the preconditioner at the
                        current iterate and drop the L-BFGS pairs; 0 = keep the
                        warm start's for the whole step.  >= 0 (EINVAL otherwise) */
  int schedule;      /* ABD_SCHEDULE_* (EINVAL for other values) */
  int solver;        /* ABD_SOLVER_* (EINVAL for other values) */
} abd_step_opts;

typedef struct {
  int iterations;    /* accepted iterations */
  int evaluations;   /* objective+gradient evaluations (incl. the warm start) */
  int flag;          /* ABD_FLAG_* */
  int f32_iterations;/* iterations whose evaluations ran in float32 (ABD_MIXED) */
  int f32_evaluations;/* evaluations that ran in float32 (ABD_MIXED) */
  int reserved;      /* 0 */
  double grad_norm;  /* |grad| at the returned q */
  double energy;     /* E at the returned q */
} abd_step_stats;    /* 40 bytes */

/* Validate a description and upload it to the current HIP device.  The
 * description is the model of Sec. 5: bodies with a parent relation, joint axes
 * and offsets, and the precomputed per-body integrals of Eq. ATOM (mass_moment:
 * int rho (p;1)(p;1)^T dp over the body, in its own frame), which turn every
 * body integral of Eq. EQ into a contraction with the pose.  Checks
 * topology, finite values, unit axes, positive mass and positive semi-definite
 * moment tensors (ABD_EINVAL).  Synchronous.  *out receives the handle.
 * Limits of this library (ABD_ENOTSUP): serial chains of up to 1024 DOFs per
 * model, branched models (trees) of up to 256 DOFs per model, models with
 * slides, drag or contact points of up to 256 DOFs.  abd_hvp and
 * abd_rollout_vjp take serial chains of up to 64 DOFs; order_K > 2 takes models
 * of up to 256 DOFs. */
int abd_create_model(const abd_model_desc* desc, abd_model** out);

/* Release the model's device memory (synchronizes the device first). */
void abd_destroy_model(abd_model* model);

/* Sizes of a created model (any pointer may be NULL). */
int abd_model_info(const abd_model* model, int* n_models, int* n_links, int* n_dofs);

/* One time step for every model (Sec. 4 and 5): warm start 2 q_k - q_{k-1},
 * then preconditioned L-BFGS with a backtracking line search on E.  Results do
 * not depend on the order of the models in the batch (each model is solved on
 * its own; workgroups take the models with the most frames first).
 *   q_hist : [2*n_dofs] = q_{k-1} followed by q_k
 *   tau    : [n_dofs] generalized joint forces held over the step, or NULL
 *   q_out  : [n_dofs] receives q_{k+1}; must not overlap q_hist
 *   stats  : [n_models] per-model outcome, or NULL
 * Order K > 2 (Eq. HOC): the step has K-1 unknown configurations at the
 * collocation points t_k + alpha_u dt (alpha_1..alpha_{K-2} the roots of the
 * Legendre polynomial L_{K-2}(2 alpha - 1), alpha_{K-1} = 1).  Then q_hist =
 * q_{k-1+alpha_{K-2}} followed by q_k, q_out is [(K-1)*n_dofs] (all unknown
 * configurations, the last one is q_{k+1}), the objective is Eq. EQHOC (sum of
 * squared residuals, each scaled by dt^2), the warm start extrapolates the known
 * points at constant velocity, and the initial inverse Hessian is
 * (W^T W)^-1 (x) H_q(q_k)^-2 (W: collocation weights among the unknown points). */
int abd_step(abd_model* model, const abd_step_opts* opts, const double* q_hist,
             const double* tau, double* q_out, abd_step_stats* stats, void* stream);

/* n_steps consecutive time steps in one launch (a rollout).  Every model
 * advances through the steps at its own pace, so a model whose step needs many
 * iterations does not hold back the others between steps (the anti-starvation
 * scheme of Sec. 5's GPU implementation: work is interleaved per iteration).
 *   q_init : [2*n_dofs] = q_{-1} followed by q_0
 *   tau    : [n_steps*n_dofs] joint forces of every step, or NULL
 *   q_traj : [n_steps*n_dofs] receives q_1 .. q_{n_steps}; must not overlap q_init
 *   stats  : [n_steps*n_models] per-step outcome, or NULL
 * abd_step is the n_steps = 1 case.  Order K > 2: q_init = q_{-1+alpha_{K-2}}
 * followed by q_0, and q_traj is [n_steps][K-1][n_dofs] (every step's unknown
 * configurations). */
int abd_rollout(abd_model* model, const abd_step_opts* opts, const double* q_init,
                const double* tau, double* q_traj, abd_step_stats* stats, int n_steps,
                void* stream);

/* abd_rollout for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as abd_rollout, but every buffer the kernels write
 * besides the caller's inputs and outputs (per-frame step constants, L-BFGS
 * rings of models of more than 64 DOFs, preconditioner work space, order-K
 * known-point seeds) lives in one fixed 64 MiB device array per GPU, held
 * until the process ends; the call never allocates (abd_rollout allocates the
 * order-K buffers on a model's first order-K call).  The array is cleared as
 * needed by a kernel enqueued on `stream`.
 *   Arguments and results as abd_rollout.  A model whose step scratch exceeds
 *   64 MiB (about 144 bytes per DOF for serial chains of <= 64 DOFs, more for
 *   longer or branched models and for order K > 2) is rejected with
 *   ABD_ENOTSUP before anything is enqueued.
 *   All calls on one GPU share its array: calls that overlap on one device
 *   (different streams, or different host threads) race and give undefined
 *   results; order them on one stream. */
int abd_rollout_noalloc(abd_model* model, const abd_step_opts* opts, const double* q_init,
                        const double* tau, double* q_traj, abd_step_stats* stats, int n_steps,
                        void* stream);

/* Objective and gradient without optimization (Eq. EQ scaled by dt^2; gradient by
 * the adjoint backward pass of Alg. 1).
 *   q        : [n_dofs] configuration to evaluate
 *   q_hist   : [2*n_dofs] = q_{k-1} followed by q_k
 *   tau      : [n_dofs] or NULL
 *   E        : [n_models] objective per model
 *   grad     : [n_dofs] gradient dE/dq, or NULL
 *   grad_tau : [n_dofs] dE/dtau (= -dt^2 q for order 2; for order K > 2 the
 *              derivative of Eq. EQHOC with respect to the joint forces held over
 *              the step, -2 dt^2 sum_u rho_u), or NULL
 * opts->precision selects float64 or float32 kinematics; opts->order_K > 2
 * evaluates Eq. EQHOC with q and grad of [(K-1)*n_dofs] (the unknown
 * configurations) and q_hist = q_{k-1+alpha_{K-2}}, q_k; other fields but dt are
 * ignored. */
int abd_objective_grad(abd_model* model, const abd_step_opts* opts, const double* q,
                       const double* q_hist, const double* tau, double* E, double* grad,
                       double* grad_tau, void* stream);

/* Hessian-vector product of the step objective at q (float64): Hv = (d2E/dq dq) v,
 * the derivative of the Alg. 1 gradient along v, computed by forward-mode
 * differentiation of the forward and backward passes (O(n) per model).
 *   q, v, Hv : [n_dofs]     q_hist : [2*n_dofs] = q_{k-1} followed by q_k
 * opts->dt is used; the other fields are ignored. */
int abd_hvp(abd_model* model, const abd_step_opts* opts, const double* q, const double* q_hist,
            const double* v, double* Hv, void* stream);

/* Hessian d2E/dq dq of the step objective (Eq. EQ scaled by dt^2) at q, as
 * explicit dense blocks (float64): the Jacobian of the Alg. 1 gradient, i.e.
 * the inertial term's Gauss-Newton part sum_l <dA_l/dq_b M_l, dA_l/dq_c> plus
 * the seed's second-derivative part sum_l <G_l, d2A_l/dq_b dq_c> (the blocks
 * that Alg. 2/3 of the paper compute), each entry from sums over the links
 * below the deeper of its two joints, so one workgroup assembles a model's
 * n_i^2 entries after O(n_i) scans.
 *   q      : [n_dofs]       q_hist : [2*n_dofs] = q_{k-1} followed by q_k
 *   H      : [sum_i n_i^2] one row-major n_i x n_i block per model (the model's
 *            DOFs in the caller's order), model after model
 * opts->dt is used; the other fields are ignored.  Serial chains of up to 1024
 * DOFs and branched models of up to 256 DOFs.  Uses the model's per-step scratch
 * (calls on one model must be ordered on one stream). */
int abd_hessian(abd_model* model, const abd_step_opts* opts, const double* q, const double* q_hist,
                double* H, void* stream);

/* Reverse-mode derivative of a rollout (float64).  Every step's result is
 * defined by the stationarity condition of its objective (Eq. PBAD), so by the
 * implicit function theorem, with lambda = dL/dq_{k+1} and H mu = lambda (H the
 * Hessian at q_{k+1}, solved by conjugate gradients preconditioned with the
 * inverse joint-space inertia):
 *   dL/dq_k += -(d2E/dq dq_k)^T mu,  dL/dq_{k-1} += -(d2E/dq dq_{k-1})^T mu,
 *   dL/dtau_k = dt^2 mu.
 *   q_init     : [2*n_dofs] = q_{-1}, q_0 of the forward rollout
 *   q_traj     : [n_steps*n_dofs] = q_1 .. q_{n_steps} it produced
 *   dL_dq_traj : [n_steps*n_dofs] explicit dL/dq_1 .. dL/dq_{n_steps}
 *   dL_dq_init : [2*n_dofs] receives dL/dq_{-1}, dL/dq_0
 *   dL_dtau    : [n_steps*n_dofs] receives dL/dtau_0 .. dL/dtau_{n_steps-1}, or NULL
 *   stats      : [n_steps*n_models] per solve: iterations = CG iterations,
 *                evaluations = Hessian-vector products, grad_norm = final residual,
 *                flag 1 converged / 2 H not positive definite along a CG direction /
 *                4 max_iter / 8 non-finite; or NULL
 * opts: dt; tol = relative CG residual; max_iter = CG iterations per step;
 * precond selects the CG preconditioner.  The torques of the forward rollout are
 * not needed (the objective is linear in them). */
int abd_rollout_vjp(abd_model* model, const abd_step_opts* opts, const double* q_init, const double* q_traj,
                    const double* dL_dq_traj, double* dL_dq_init, double* dL_dtau, abd_step_stats* stats,
                    int n_steps, void* stream);

/* World poses [R|t] (3x4 row-major, 12 doubles per link) of every link at q
 * (forward kinematics of Alg. 1).  poses: device [12*n_links]. */
int abd_poses(abd_model* model, const double* q, double* poses, void* stream);

/* Text of the last error raised on the calling host thread ("" if none). */
const char* abd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
