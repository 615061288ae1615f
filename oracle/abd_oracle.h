/*
 * FP64 CPU oracle for position-based articulated dynamics (Pan & Manocha,
 * "Time Integrating Articulated Body Dynamics Using Position-Based Collocation
 * Methods").  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
 * CPU-baseline leg of the benchmark call it; the product path never does.
 * It shares no code, header or table with the HIP library.
 *
 * Every routine is a plain, slow, sequential restatement of the paper:
 *   - link poses by the sequential transform product of Alg. 1 (forward pass),
 *   - the objective of Eq. EQ scaled by dt^2, with the body integral done
 *     exactly through the per-link mass moment tensor (Eq. ATOM),
 *   - its gradient by the literal 4x4 adjoint backward pass of Alg. 1,
 *   - the quasi-Newton solve of Sec. 5 (L-BFGS with a backtracking line search
 *     that enforces decrease, as the paper requires of the optimizer).
 * All arithmetic is double precision.
 */
#ifndef ABD_ORACLE_H
#define ABD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_model orc_model;

typedef struct {
  double dt;
  int order_K;     /* 2 = Eq. EQ; >2 = Eq. EQHOC (collocation) */
  int lbfgs_m;     /* history length */
  double tol;      /* stop when |g| <= tol*|g(q0)| */
  int max_iter;
  int max_ls;      /* line-search halvings before giving up */
  double eps_w;    /* working-precision epsilon used by the noise test */
  int precond;     /* initial inverse Hessian H0: 0 gamma*I, 1 gamma*diag(H_q)^-1,
                      2 H_q^-1 (joint-space inertia at the warm start) */
  int refresh;     /* precond 2, K = 2: every `refresh` iterations re-form H_q at the
                      current iterate and drop the curvature pairs (0 = never) */
} orc_opts;

/* Levenberg-Marquardt options (order K >= 2 collocation, Eq. EQHOC). */
typedef struct {
  double dt;
  int order_K;
  int max_iter;      /* iterations, accepted or rejected */
  double tol;        /* stop when |dE/dq| <= tol * |dE/dq at the warm start| */
  double lambda0;    /* initial lambda relative to max diag(J^T J) */
  int geodesic;      /* 1: add half the geodesic acceleration (Transtrum & Sethna) */
  double geo_h;      /* finite-difference step of the second directional derivative */
  double geo_alpha;  /* reject steps with 2|a| > geo_alpha |v| */
} orc_lm_opts;

typedef struct {
  int iterations;
  int evaluations;
  int flag;        /* 1 converged, 2 line-search floor, 4 max-iter, 8 non-finite */
  int pad;
  double grad_norm;
  double energy;
} orc_stats;

orc_model* orc_create(int n_models, const int* link_offset, const int* parent,
                      const int* dofs_per_link, const double* axis, const double* offset,
                      const double* mass_moment, const double* gravity);
void orc_free(orc_model* m);

/* Optional terms of the step objective (Sec. 6 applications), replacing any set
 * before.  dof_kind [n_dofs] (NULL: all hinges): 0 = hinge (rotation about the
 * DOF's axis), 1 = slide (translation along it), so that a 6-DOF floating root
 * is three slides and three hinges on one link.  drag [n_links] (NULL: none):
 * per link c_l >= 0, adding c_l tr((A_l(q) - A_l(q_k)) M_l (...)^T) = dt^2 times
 * the paper's drag potential D |(P(q) - P(q_k))/dt|^2 integrated over the body
 * with c_l = D / rho_l.  n_contacts points (contact_link: global link index,
 * contact_point [3*n_contacts] in the link frame) with the penalty potential of
 * Eq. FRI against the half-space n.x < h (plane = n[3], h):
 *   dt^2 D1 d^2 + D2 d^2 |(I - n n^T)(x(q) - x(q_k))|^2,  d = max(0, h - n.x).
 * Returns 0, or -1 on invalid input (the model is then left without extras). */
int orc_set_extras(orc_model* m, const int* dof_kind, const double* drag, int n_contacts,
                   const int* contact_link, const double* contact_point, const double* plane, double d1,
                   double d2);

/* World poses A = [R|t] (3x4 row-major, 12 doubles) of every link at q. */
void orc_poses(const orc_model* m, const double* q, double* poses, int n_threads);

/* Objective (dt^2-scaled Eq. EQ, D-form) and gradient (Alg. 1) for every model.
 * q_hist = [q_{k-1} ; q_k] (2*n_dofs).  tau may be NULL.  grad may be NULL.
 * S (may be NULL) receives sum_l |e_l| (the noise scale of the line search). */
void orc_objective_grad(const orc_model* m, double dt, const double* q, const double* q_hist,
                        const double* tau, double* E, double* grad, double* S, int n_threads);

/* Objective of the same step assembled from the pairwise integrals of
 * Appendix A: 1/2 I(q,q) - 2 I(q,q_k) + I(q,q_{k-1}) + potential - dt^2 tau.q.
 * Differs from orc_objective_grad's E by a q-independent constant. */
void orc_objective_Iform(const orc_model* m, double dt, const double* q, const double* q_hist,
                         const double* tau, double* E, int n_threads);

/* Eq. ATOM and Alg. 1: I(q_a,q_b) per model and dI/dq_b (n_dofs). */
void orc_alg1_I(const orc_model* m, const double* q_a, const double* q_b, double* I,
                double* dI_dqb, int n_threads);

/* Diagonal of the joint-space inertia sum_l tr(dA_l/dq_n M_l dA_l/dq_n^T) at q. */
void orc_inertia_diag(const orc_model* m, const double* q, double* h, int n_threads);

/* Joint-space inertia H_ij = sum_l tr(dA_l/dq_i M_l dA_l/dq_j^T) at q, one dense
 * row-major block per model, packed model after model (sum of n_i^2 doubles). */
void orc_inertia_matrix(const orc_model* m, const double* q, double* H, int n_threads);

/* Hessian d2E/dq dq of the step objective at q (second derivatives of the
 * poses written out), one dense row-major block per model, packed like
 * orc_inertia_matrix.  q_hist = [q_{k-1}; q_k]. */
void orc_hessian(const orc_model* m, double dt, const double* q, const double* q_hist, double* H,
                 int n_threads);

/* C_ab = scale * sum_l <dA_l(q)/dq_a M_l, dA_l(q_o)/dq_o,b>: the mixed second
 * derivative of E with respect to q and a past configuration (scale -2 for q_k,
 * +1 for q_{k-1}).  Packed dense blocks. */
void orc_cross_hessian(const orc_model* m, const double* q, const double* q_o, double scale, double* C,
                       int n_threads);

/* Collocation of order K (2..8) for Eq. HOC: tau[K+1] = the points of one step
 * in units of dt from t_k (alpha_{K-2}-1, 0, alpha_1..alpha_{K-1}), and
 * w[(K-1)*(K+1)] = second derivatives of the Lagrange basis at the K-1 unknown
 * points (dt^2 Pddot(tau_{2+u}) = sum_j w[u][j] P_j).  Returns 0, or -1 for K
 * out of range. */
int orc_collocation(int K, double* tau, double* w);

/* Eq. EQHOC objective per model and its gradient ([K-1][n_dofs]) with respect to
 * the K-1 unknown configurations q_unknown ([K-1][n_dofs]), given the two known
 * configurations q_known = [q_{k-1+alpha_{K-2}}; q_k].  tau may be NULL. */
void orc_eqhoc_objective_grad(const orc_model* m, int K, double dt, const double* q_known,
                              const double* q_unknown, const double* tau, double* E, double* grad,
                              int n_threads);

/* Residuals dt^2 r_u of Eq. HOC ([K-1][n_dofs]) at the unknown configurations
 * and, if J is not NULL, their Jacobian: per model one dense row-major block of
 * ((K-1) nd)^2 doubles (row (u, b), column (a, c)), packed model after model. */
void orc_eqhoc_residual_jacobian(const orc_model* m, int K, double dt, const double* q_known,
                                 const double* q_unknown, const double* tau, double* R, double* J,
                                 int n_threads);

/* One time step for every model: q_out = argmin of the step objective,
 * reached by preconditioned L-BFGS from the warm start 2 q_k - q_{k-1}. */
int orc_step(const orc_model* m, const orc_opts* o, const double* q_hist, const double* tau,
             double* q_out, orc_stats* stats, int n_threads);

/* One Eq. EQHOC step (order_K = 3..8) for every model: q_known = [q_{k-1+alpha_{K-2}};
 * q_k] ([2][n_dofs]), q_out receives the K-1 unknown configurations ([K-1][n_dofs],
 * the last one is q_{k+1}).  Returns 0, or -1 for an order out of range. */
int orc_step_hoc(const orc_model* m, const orc_opts* o, const double* q_known, const double* tau,
                 double* q_out, orc_stats* stats, int n_threads);

/* One Eq. EQHOC step (order_K = 2..8) for every model by Levenberg-Marquardt
 * (Sec. 5): (J^T J + lambda I) v = -J^T r with the written-out Jacobian of the
 * residuals and a dense Cholesky solve, Nielsen's lambda rule, optional
 * geodesic acceleration.  Arguments as orc_step_hoc; stats count LM iterations
 * (accepted or rejected) and residual evaluations.  Returns 0, or -1 for an
 * order out of range. */
int orc_step_lm_hoc(const orc_model* m, const orc_lm_opts* o, const double* q_known, const double* tau,
                    double* q_out, orc_stats* stats, int n_threads);

/* Reported total energy at step k: (1/2dt^2) sum tr(dA M dA^T) + V(q_k),
 * dA = A(q_k) - A(q_{k-1}). */
void orc_energy_report(const orc_model* m, double dt, const double* q_prev, const double* q_curr,
                       double* H, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
