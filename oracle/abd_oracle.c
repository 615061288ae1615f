/*
 * FP64 CPU oracle -- test infrastructure only (see abd_oracle.h).
 *
 * Kinematic representation.  Every DOF is one elementary hinge "frame".  A
 * link with d DOFs is d consecutive frames: the first is translated by the
 * joint offset and rotates about the first axis, the others have zero offset
 * and rotate about the following axes; only the link's last frame carries its
 * mass moment tensor.  A ball joint is thus three consecutive hinges with
 * massless zero-length intermediate frames.  With one DOF per frame, Alg. 1
 * applies verbatim: T^f = T^{parent(f)} t_f(q_f) in the forward pass, and in
 * the backward pass  A <- A + dE/dT^f ;  g_f += (T^{parent(f)} dt_f/dq_f) : A ;
 * A_parent <- A_parent + A t_f^T  (the tree form of "A <- A t^T").
 *
 * Objective (Sec. 4, Eq. EQ, multiplied by dt^2 so the minimizer is unchanged):
 *   E(q) = sum_l 1/2 tr(D_l M_l D_l^T) - dt^2 sum_l g^T A_l(q) M_l e4 - dt^2 tau.q
 *   D_l  = A_l(q) - 2 A_l(q_k) + A_l(q_{k-1}),  A = [R|t] (3x4)
 * since  int rho |P_a - 2P_b + P_c|^2 / 2 dp = 1/2 tr(D M D^T)  exactly when
 * M = int rho (p;1)(p;1)^T dp (Eq. ATOM), and the gravity potential density
 * -rho g.P integrates to -g^T A M e4.
 */
#include "abd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc_model {
  int n_models, n_links, n_dofs;
  int *link_offset, *parent, *dofs_per_link;
  double *axis, *offset, *mm;
  double g[3];
  int *link_dof;     /* [n_links] first global dof of the link */
  int *model_dof;    /* [n_models+1] */
  int *frame_parent; /* [n_dofs] parent frame (global dof index), -1 = world */
  int *frame_link;   /* [n_dofs] link owning the frame */
  int *frame_first;  /* [n_dofs] 1 if first frame of its link */
  int *frame_mass;   /* [n_dofs] link whose mass the frame carries, -1 = massless */
  /* optional terms (orc_set_extras) */
  int *dof_kind;     /* [n_dofs] 0 hinge, 1 slide; NULL = every DOF a hinge */
  double *drag;      /* [n_links] drag coefficient of every link; NULL = no drag */
  int *c_off;        /* [n_links+1] contact points of link l: c_off[l] .. c_off[l+1]-1; NULL = none */
  double *c_pt;      /* [3*n_contacts] point in its link's frame, grouped by link */
  double plane[4];   /* contact plane: unit normal n (world) and offset h */
  double c_d1, c_d2; /* normal and friction penalties of Eq. FRI */
};

static int is_slide(const orc_model* m, int f) { return m->dof_kind && m->dof_kind[f] == 1; }

/* ------------------------------------------------------------------ 4x4 -- */
static void m4_eye(double* A) {
  memset(A, 0, 16 * sizeof(double));
  A[0] = A[5] = A[10] = A[15] = 1.0;
}
static void m4_mul(const double* A, const double* B, double* C) {
  double t[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += A[4 * i + k] * B[4 * k + j];
      t[4 * i + j] = s;
    }
  memcpy(C, t, sizeof t);
}
/* C += A B^T */
static void m4_add_mul_bt(const double* A, const double* B, double* C) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += A[4 * i + k] * B[4 * j + k];
      C[4 * i + j] += s;
    }
}
static double m4_frob(const double* A, const double* B) {
  double s = 0.0;
  for (int i = 0; i < 16; ++i) s += A[i] * B[i];
  return s;
}
/* inverse of a rigid transform [R t; 0 1] */
static void m4_rigid_inv(const double* T, double* Ti) {
  memset(Ti, 0, 16 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ti[4 * i + j] = T[4 * j + i];
  for (int i = 0; i < 3; ++i)
    Ti[4 * i + 3] = -(Ti[4 * i + 0] * T[3] + Ti[4 * i + 1] * T[7] + Ti[4 * i + 2] * T[11]);
  Ti[15] = 1.0;
}
/* symmetric 4x4 from its upper triangle (00 01 02 03 11 12 13 22 23 33) */
static void mm_full(const double* u, double* M) {
  static const int idx[16] = {0, 1, 2, 3, 1, 4, 5, 6, 2, 5, 7, 8, 3, 6, 8, 9};
  for (int i = 0; i < 16; ++i) M[i] = u[idx[i]];
}

/* Local transform of one DOF frame.  Hinge (Rodrigues): R = I + sin(th) K +
 * (1-cos(th)) K^2, K = [a]x, t = [R o; 0 1].  Slide: t = [I, o + th a; 0 1]. */
static void local_tf(const double* a, const double* o, double th, double* t, int slide) {
  if (slide) {
    m4_eye(t);
    for (int i = 0; i < 3; ++i) t[4 * i + 3] = (o ? o[i] : 0.0) + th * a[i];
    return;
  }
  double K[9] = {0, -a[2], a[1], a[2], 0, -a[0], -a[1], a[0], 0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += K[3 * i + k] * K[3 * k + j];
      K2[3 * i + j] = s;
    }
  double s = sin(th), c = 1.0 - cos(th);
  memset(t, 0, 16 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[4 * i + j] = (i == j ? 1.0 : 0.0) + s * K[3 * i + j] + c * K2[3 * i + j];
  for (int i = 0; i < 3; ++i) t[4 * i + 3] = o ? o[i] : 0.0;
  t[15] = 1.0;
}
/* dt/dth: hinge [cos(th) K + sin(th) K^2, 0; 0 0]; slide [0, a; 0 0] */
static void local_dtf(const double* a, double th, double* dt, int slide) {
  if (slide) {
    memset(dt, 0, 16 * sizeof(double));
    for (int i = 0; i < 3; ++i) dt[4 * i + 3] = a[i];
    return;
  }
  double K[9] = {0, -a[2], a[1], a[2], 0, -a[0], -a[1], a[0], 0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += K[3 * i + k] * K[3 * k + j];
      K2[3 * i + j] = s;
    }
  double c = cos(th), s = sin(th);
  memset(dt, 0, 16 * sizeof(double));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) dt[4 * i + j] = c * K[3 * i + j] + s * K2[3 * i + j];
}

/* --------------------------------------------------------------- model -- */
orc_model* orc_create(int n_models, const int* link_offset, const int* parent,
                      const int* dofs_per_link, const double* axis, const double* offset,
                      const double* mass_moment, const double* gravity) {
  orc_model* m = (orc_model*)calloc(1, sizeof(orc_model));
  m->n_models = n_models;
  m->n_links = link_offset[n_models];
  int L = m->n_links;
  m->link_offset = (int*)malloc((n_models + 1) * sizeof(int));
  memcpy(m->link_offset, link_offset, (n_models + 1) * sizeof(int));
  m->parent = (int*)malloc((L > 0 ? L : 1) * sizeof(int));
  m->dofs_per_link = (int*)malloc((L > 0 ? L : 1) * sizeof(int));
  memcpy(m->parent, parent, L * sizeof(int));
  memcpy(m->dofs_per_link, dofs_per_link, L * sizeof(int));
  m->link_dof = (int*)malloc((L > 0 ? L : 1) * sizeof(int));
  int nd = 0;
  for (int l = 0; l < L; ++l) {
    m->link_dof[l] = nd;
    nd += dofs_per_link[l];
  }
  m->n_dofs = nd;
  m->model_dof = (int*)malloc((n_models + 1) * sizeof(int));
  for (int i = 0; i <= n_models; ++i)
    m->model_dof[i] = (link_offset[i] < L) ? m->link_dof[link_offset[i]] : nd;
  m->axis = (double*)malloc((nd > 0 ? 3 * nd : 1) * sizeof(double));
  memcpy(m->axis, axis, 3 * nd * sizeof(double));
  m->offset = (double*)malloc((L > 0 ? 3 * L : 1) * sizeof(double));
  memcpy(m->offset, offset, 3 * L * sizeof(double));
  m->mm = (double*)malloc((L > 0 ? 10 * L : 1) * sizeof(double));
  memcpy(m->mm, mass_moment, 10 * L * sizeof(double));
  memcpy(m->g, gravity, 3 * sizeof(double));
  int nd1 = nd > 0 ? nd : 1;
  m->frame_parent = (int*)malloc(nd1 * sizeof(int));
  m->frame_link = (int*)malloc(nd1 * sizeof(int));
  m->frame_first = (int*)malloc(nd1 * sizeof(int));
  m->frame_mass = (int*)malloc(nd1 * sizeof(int));
  for (int i = 0; i < n_models; ++i) {
    int lo = link_offset[i];
    for (int l = lo; l < link_offset[i + 1]; ++l) {
      int d = m->link_dof[l], k = dofs_per_link[l];
      for (int j = 0; j < k; ++j) {
        int f = d + j;
        m->frame_link[f] = l;
        m->frame_first[f] = (j == 0);
        m->frame_mass[f] = (j == k - 1) ? l : -1;
        if (j > 0)
          m->frame_parent[f] = f - 1;
        else if (parent[l] < 0)
          m->frame_parent[f] = -1;
        else {
          int pl = lo + parent[l];
          m->frame_parent[f] = m->link_dof[pl] + dofs_per_link[pl] - 1;
        }
      }
    }
  }
  return m;
}

void orc_free(orc_model* m) {
  if (!m) return;
  free(m->link_offset); free(m->parent); free(m->dofs_per_link); free(m->axis);
  free(m->offset); free(m->mm); free(m->link_dof); free(m->model_dof);
  free(m->frame_parent); free(m->frame_link); free(m->frame_first); free(m->frame_mass);
  free(m->dof_kind); free(m->drag); free(m->c_off); free(m->c_pt);
  free(m);
}

int orc_set_extras(orc_model* m, const int* dof_kind, const double* drag, int n_contacts,
                   const int* contact_link, const double* contact_point, const double* plane, double d1,
                   double d2) {
  int L = m->n_links, nd = m->n_dofs;
  free(m->dof_kind); free(m->drag); free(m->c_off); free(m->c_pt);
  m->dof_kind = NULL; m->drag = NULL; m->c_off = NULL; m->c_pt = NULL;
  if (n_contacts < 0 || !(d1 >= 0.0) || !(d2 >= 0.0)) return -1;
  if (dof_kind)
    for (int f = 0; f < nd; ++f)
      if (dof_kind[f] != 0 && dof_kind[f] != 1) return -1;
  if (drag)
    for (int l = 0; l < L; ++l)
      if (!(drag[l] >= 0.0) || !isfinite(drag[l])) return -1;
  for (int c = 0; c < n_contacts; ++c)
    if (contact_link[c] < 0 || contact_link[c] >= L) return -1;
  if (dof_kind) {
    m->dof_kind = (int*)malloc((nd > 0 ? nd : 1) * sizeof(int));
    for (int f = 0; f < nd; ++f) m->dof_kind[f] = dof_kind[f];
  }
  if (drag) {
    m->drag = (double*)malloc((L > 0 ? L : 1) * sizeof(double));
    for (int l = 0; l < L; ++l) m->drag[l] = drag[l];
  }
  if (n_contacts > 0) {
    m->c_off = (int*)calloc(L + 1, sizeof(int));
    m->c_pt = (double*)malloc(3 * (size_t)n_contacts * sizeof(double));
    for (int c = 0; c < n_contacts; ++c) m->c_off[contact_link[c] + 1]++;
    for (int l = 0; l < L; ++l) m->c_off[l + 1] += m->c_off[l];
    int* fill = (int*)calloc(L > 0 ? L : 1, sizeof(int));
    for (int c = 0; c < n_contacts; ++c) {
      int l = contact_link[c], at = m->c_off[l] + fill[l]++;
      for (int k = 0; k < 3; ++k) m->c_pt[3 * at + k] = contact_point[3 * c + k];
    }
    free(fill);
    for (int k = 0; k < 4; ++k) m->plane[k] = plane[k];
    m->c_d1 = d1;
    m->c_d2 = d2;
  }
  return 0;
}

static int model_nd(const orc_model* m, int i) { return m->model_dof[i + 1] - m->model_dof[i]; }

/* Eq. FRI for one contact point at world position x (xk at q_k), scaled by dt^2
 * like the rest of the objective:
 *   V = dt^2 D1 d^2 + D2 d^2 |P (x - xk)|^2,  d = max(0, h - n.x),  P = I - n n^T
 * (penetration depth d of the half-space n.x < h, tangential displacement over
 * the step).  Returns V; f = dV/dx; Hx (if not NULL) = d2V/dx2, 3x3 row-major. */
static double contact_term(const orc_model* m, double dt2, const double* x, const double* xk, double* f,
                           double* Hx) {
  const double* n = m->plane;
  double d = m->plane[3] - (n[0] * x[0] + n[1] * x[1] + n[2] * x[2]);
  for (int k = 0; k < 3; ++k) f[k] = 0.0;
  if (Hx) memset(Hx, 0, 9 * sizeof(double));
  if (!(d > 0.0)) return 0.0;
  double v[3], u[3], nv = 0.0;
  for (int k = 0; k < 3; ++k) v[k] = x[k] - xk[k];
  for (int k = 0; k < 3; ++k) nv += n[k] * v[k];
  for (int k = 0; k < 3; ++k) u[k] = v[k] - nv * n[k];
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double a = dt2 * m->c_d1 + m->c_d2 * uu;
  /* d/dx: dd/dx = -n, d|u|^2/dx = 2u */
  for (int k = 0; k < 3; ++k) f[k] = -2.0 * d * a * n[k] + 2.0 * m->c_d2 * d * d * u[k];
  if (Hx)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        Hx[3 * r + c] = 2.0 * a * n[r] * n[c] - 4.0 * m->c_d2 * d * (n[r] * u[c] + u[r] * n[c]) +
                        2.0 * m->c_d2 * d * d * ((r == c ? 1.0 : 0.0) - n[r] * n[c]);
  return d * d * a;
}

/* world position of the point p (link frame) under the pose T (rows 0..2) */
static void point_at(const double* T, const double* p, double* x) {
  for (int r = 0; r < 3; ++r) x[r] = T[4 * r] * p[0] + T[4 * r + 1] * p[1] + T[4 * r + 2] * p[2] + T[4 * r + 3];
}

/* Mass moment tensor of link l as a full 4x4; scaled: times 1 + 2 c_l (c_l the
 * link's drag coefficient), the Gauss-Newton weight of the kinetic and drag
 * terms together, which the step's inertia preconditioner uses.  (Contact
 * stiffness is not represented: as an isotropic point mass it slows the
 * sliding modes more than it helps the normal ones.) */
static void link_mm(const orc_model* m, int l, double* M, int scaled) {
  mm_full(m->mm + 10 * l, M);
  if (scaled && m->drag)
    for (int k = 0; k < 16; ++k) M[k] *= 1.0 + 2.0 * m->drag[l];
}

/* The drag and contact terms of link l (pose A at q, Ak at q_k) added to its
 * energy e and seed G = dE/dA (3 rows of 4): drag c tr(dA M dA^T) with
 * dA = A - Ak (the paper's drag potential D |(P - P_k)/dt|^2 integrated over
 * the body, times dt^2, with c = D / rho), and Eq. FRI at the link's points. */
static double extra_terms(const orc_model* m, int l, double dt2, const double* M, const double* A,
                          const double* Ak, double* G) {
  double e = 0.0;
  if (m->drag && m->drag[l] != 0.0) {
    double c = m->drag[l];
    for (int r = 0; r < 3; ++r) {
      double dA[4];
      for (int k = 0; k < 4; ++k) dA[k] = A[4 * r + k] - Ak[4 * r + k];
      for (int k = 0; k < 4; ++k) {
        double dm = 0.0;
        for (int x = 0; x < 4; ++x) dm += dA[x] * M[4 * x + k];
        e += c * dm * dA[k];
        G[4 * r + k] += 2.0 * c * dm;
      }
    }
  }
  if (m->c_off)
    for (int p = m->c_off[l]; p < m->c_off[l + 1]; ++p) {
      const double* pt = m->c_pt + 3 * p;
      double x[3], xk[3], f[3];
      point_at(A, pt, x);
      point_at(Ak, pt, xk);
      e += contact_term(m, dt2, x, xk, f, NULL);
      for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) G[4 * r + k] += f[r] * pt[k];
        G[4 * r + 3] += f[r];
      }
    }
  return e;
}

/* Forward pass of Alg. 1 for model i: T[j] (world) and tl[j] (local), j local frame index. */
static void fk_model(const orc_model* m, int i, const double* q, double* T, double* tl) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  double I4[16];
  m4_eye(I4);
  for (int j = 0; j < nd; ++j) {
    int f = d0 + j;
    const double* o = m->frame_first[f] ? m->offset + 3 * m->frame_link[f] : NULL;
    double* t = tl + 16 * j;
    local_tf(m->axis + 3 * f, o, q[f], t, is_slide(m, f));
    int p = m->frame_parent[f];
    m4_mul(p >= 0 ? T + 16 * (p - d0) : I4, t, T + 16 * j);
  }
}

typedef struct {
  double *Tk, *Tkm1, *T, *tl, *Adj;
} eval_ws;

static void ws_alloc(eval_ws* w, int nd) {
  size_t n = (size_t)(nd > 0 ? nd : 1) * 16;
  w->Tk = (double*)malloc(n * sizeof(double));
  w->Tkm1 = (double*)malloc(n * sizeof(double));
  w->T = (double*)malloc(n * sizeof(double));
  w->tl = (double*)malloc(n * sizeof(double));
  w->Adj = (double*)malloc(n * sizeof(double));
}
static void ws_free(eval_ws* w) {
  free(w->Tk); free(w->Tkm1); free(w->T); free(w->tl); free(w->Adj);
}

/* Backward pass of Alg. 1 over the frames of model i.  Adj holds the per-frame
 * seeds dE/dT^f on entry (accumulated with child contributions as it runs).
 * g (global indexing) receives dE/dq_f. */
static void alg1_backward(const orc_model* m, int i, const double* T, const double* tl,
                          double* Adj, const double* q, double* g) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  double I4[16], dt[16], W[16];
  m4_eye(I4);
  for (int j = nd - 1; j >= 0; --j) {
    int f = d0 + j;
    int p = m->frame_parent[f];
    local_dtf(m->axis + 3 * f, q[f], dt, is_slide(m, f));
    m4_mul(p >= 0 ? T + 16 * (p - d0) : I4, dt, W);
    g[f] = m4_frob(W, Adj + 16 * j);
    if (p >= 0) m4_add_mul_bt(Adj + 16 * j, tl + 16 * j, Adj + 16 * (p - d0));
  }
}

/* Objective and gradient of model i at q.  Tk, Tkm1 = frame poses at q_k, q_{k-1}. */
static double eval_model(const orc_model* m, int i, double dt, const double* q, const double* tau,
                         eval_ws* w, double* g, double* S) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  fk_model(m, i, q, w->T, w->tl);
  memset(w->Adj, 0, (size_t)nd * 16 * sizeof(double));
  double E = 0.0, Ssum = 0.0, dt2 = dt * dt;
  for (int l = m->link_offset[i]; l < m->link_offset[i + 1]; ++l) {
    int j = m->link_dof[l] + m->dofs_per_link[l] - 1 - d0;
    double M[16];
    mm_full(m->mm + 10 * l, M);
    const double *A = w->T + 16 * j, *Ak = w->Tk + 16 * j, *Akm1 = w->Tkm1 + 16 * j;
    double e = 0.0;
    for (int r = 0; r < 3; ++r) {
      double D[4], DM[4];
      for (int c = 0; c < 4; ++c) D[c] = A[4 * r + c] - 2.0 * Ak[4 * r + c] + Akm1[4 * r + c];
      for (int c = 0; c < 4; ++c) {
        DM[c] = 0.0;
        for (int k = 0; k < 4; ++k) DM[c] += D[k] * M[4 * k + c];
      }
      for (int c = 0; c < 4; ++c) e += 0.5 * DM[c] * D[c];
      /* potential row r: -dt^2 g_r (A_r . M e4) */
      double AMe4 = 0.0;
      for (int k = 0; k < 4; ++k) AMe4 += A[4 * r + k] * M[4 * k + 3];
      e -= dt2 * m->g[r] * AMe4;
      /* seed row r of dE/dA: D M - dt^2 g (M e4)^T */
      for (int c = 0; c < 4; ++c) w->Adj[16 * j + 4 * r + c] += DM[c] - dt2 * m->g[r] * M[4 * c + 3];
    }
    e += extra_terms(m, l, dt2, M, A, Ak, w->Adj + 16 * j);
    E += e;
    Ssum += fabs(e);
  }
  if (tau)
    for (int j = 0; j < nd; ++j) {
      double t = dt2 * tau[d0 + j] * q[d0 + j];
      E -= t;
      Ssum += fabs(t);
    }
  if (g) {
    alg1_backward(m, i, w->T, w->tl, w->Adj, q, g);
    if (tau)
      for (int j = 0; j < nd; ++j) g[d0 + j] -= dt2 * tau[d0 + j];
  }
  if (S) *S = Ssum;
  return E;
}

/* ------------------------------------------------------------ queries -- */
void orc_poses(const orc_model* m, const double* q, double* poses, int n_threads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i), d0 = m->model_dof[i];
    eval_ws w;
    ws_alloc(&w, nd);
    fk_model(m, i, q, w.T, w.tl);
    for (int l = m->link_offset[i]; l < m->link_offset[i + 1]; ++l) {
      int j = m->link_dof[l] + m->dofs_per_link[l] - 1 - d0;
      memcpy(poses + 12 * (size_t)l, w.T + 16 * j, 12 * sizeof(double));
    }
    ws_free(&w);
  }
}

void orc_objective_grad(const orc_model* m, double dt, const double* q, const double* q_hist,
                        const double* tau, double* E, double* grad, double* S, int n_threads) {
  const double* qkm1 = q_hist;
  const double* qk = q_hist + m->n_dofs;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    eval_ws w;
    ws_alloc(&w, model_nd(m, i));
    fk_model(m, i, qk, w.Tk, w.tl);
    fk_model(m, i, qkm1, w.Tkm1, w.tl);
    double s;
    E[i] = eval_model(m, i, dt, q, tau, &w, grad, &s);
    if (S) S[i] = s;
    ws_free(&w);
  }
}

/* Eq. ATOM's pairing of one link: int rho P_a . P_b dp = sum_r row_r(A) M row_r(B)^T
 * over the three pose rows. */
static double link_I(const orc_model* m, int l, const double* A, const double* B) {
  double M[16], s = 0.0;
  mm_full(m->mm + 10 * l, M);
  for (int r = 0; r < 3; ++r)
    for (int x = 0; x < 4; ++x)
      for (int y = 0; y < 4; ++y) s += A[4 * r + x] * M[4 * x + y] * B[4 * r + y];
  return s;
}

/* I(q_a,q_b) of Eq. ATOM for model i with the homogeneous 4x4 transforms:
 * [T_a^T T_b] : M minus the homogeneous 1*1 entry (the body mass). */
static double atom_I(const orc_model* m, int i, const double* Ta, const double* Tb) {
  int d0 = m->model_dof[i];
  double I = 0.0;
  for (int l = m->link_offset[i]; l < m->link_offset[i + 1]; ++l) {
    int j = m->link_dof[l] + m->dofs_per_link[l] - 1 - d0;
    double M[16];
    mm_full(m->mm + 10 * l, M);
    const double *A = Ta + 16 * j, *B = Tb + 16 * j;
    double s = 0.0; /* tr((Ta^T Tb)^T M) = sum_k row_k(Ta) M row_k(Tb)^T */
    for (int k = 0; k < 4; ++k)
      for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) s += A[4 * k + x] * M[4 * x + y] * B[4 * k + y];
    I += s - M[15];
  }
  return I;
}

void orc_alg1_I(const orc_model* m, const double* q_a, const double* q_b, double* I,
                double* dI_dqb, int n_threads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i), d0 = m->model_dof[i];
    eval_ws w;
    ws_alloc(&w, nd);
    fk_model(m, i, q_a, w.Tk, w.tl);
    fk_model(m, i, q_b, w.T, w.tl);
    I[i] = atom_I(m, i, w.Tk, w.T);
    /* seed dI^f/dT^f(q_b) = T^f(q_a) M on mass-carrying frames */
    memset(w.Adj, 0, (size_t)nd * 16 * sizeof(double));
    for (int l = m->link_offset[i]; l < m->link_offset[i + 1]; ++l) {
      int j = m->link_dof[l] + m->dofs_per_link[l] - 1 - d0;
      double M[16];
      mm_full(m->mm + 10 * l, M);
      m4_mul(w.Tk + 16 * j, M, w.Adj + 16 * j);
    }
    alg1_backward(m, i, w.T, w.tl, w.Adj, q_b, dI_dqb);
    ws_free(&w);
  }
}

static double potential(const orc_model* m, int i, const double* T) {
  int d0 = m->model_dof[i];
  double V = 0.0;
  for (int l = m->link_offset[i]; l < m->link_offset[i + 1]; ++l) {
    int j = m->link_dof[l] + m->dofs_per_link[l] - 1 - d0;
    const double* u = m->mm + 10 * l;
    const double Me4[4] = {u[3], u[6], u[8], u[9]};
    for (int r = 0; r < 3; ++r) {
      double s = 0.0;
      for (int k = 0; k < 4; ++k) s += T[16 * j + 4 * r + k] * Me4[k];
      V -= m->g[r] * s;
    }
  }
  return V;
}

void orc_objective_Iform(const orc_model* m, double dt, const double* q, const double* q_hist,
                         const double* tau, double* E, int n_threads) {
  const double* qkm1 = q_hist;
  const double* qk = q_hist + m->n_dofs;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i), d0 = m->model_dof[i];
    eval_ws w;
    ws_alloc(&w, nd);
    fk_model(m, i, qk, w.Tk, w.tl);
    fk_model(m, i, qkm1, w.Tkm1, w.tl);
    fk_model(m, i, q, w.T, w.tl);
    double e = 0.5 * atom_I(m, i, w.T, w.T) - 2.0 * atom_I(m, i, w.T, w.Tk) + atom_I(m, i, w.T, w.Tkm1);
    e += dt * dt * potential(m, i, w.T);
    /* drag of App. A: c (I(q,q) - 2 I(q,q_k) + I(q_k,q_k)) per link; contact points */
    for (int l = m->link_offset[i]; l < m->link_offset[i + 1]; ++l) {
      int j = m->link_dof[l] + m->dofs_per_link[l] - 1 - d0;
      if (m->drag && m->drag[l] != 0.0)
        e += m->drag[l] * (link_I(m, l, w.T + 16 * j, w.T + 16 * j) - 2.0 * link_I(m, l, w.T + 16 * j, w.Tk + 16 * j) +
                           link_I(m, l, w.Tk + 16 * j, w.Tk + 16 * j));
      if (m->c_off)
        for (int p = m->c_off[l]; p < m->c_off[l + 1]; ++p) {
          double x[3], xk[3], f[3];
          point_at(w.T + 16 * j, m->c_pt + 3 * p, x);
          point_at(w.Tk + 16 * j, m->c_pt + 3 * p, xk);
          e += contact_term(m, dt * dt, x, xk, f, NULL);
        }
    }
    if (tau)
      for (int j = 0; j < nd; ++j) e -= dt * dt * tau[d0 + j] * q[d0 + j];
    E[i] = e;
    ws_free(&w);
  }
}

/* Joint-space inertia diagonal of model i by the plain definition:
 * h_n = sum over mass frames f below DOF n of tr(dA_f M dA_f^T),
 * dT^f/dq_n = T^{parent(n)} dt_n (T^n)^{-1} T^f. */
static void inertia_diag_model(const orc_model* m, int i, const double* q, eval_ws* w, double* h,
                               char* desc, int scaled) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  fk_model(m, i, q, w->T, w->tl);
  double I4[16], dtl[16], W[16], Ti[16], tmp[16], dA[16], M[16];
  m4_eye(I4);
  for (int j = 0; j < nd; ++j) {
    int f = d0 + j, p = m->frame_parent[f];
    local_dtf(m->axis + 3 * f, q[f], dtl, is_slide(m, f));
    m4_mul(p >= 0 ? w->T + 16 * (p - d0) : I4, dtl, tmp);
    m4_rigid_inv(w->T + 16 * j, Ti);
    m4_mul(tmp, Ti, W);
    double s = 0.0;
    for (int k = j; k < nd; ++k) {
      int pk = m->frame_parent[d0 + k];
      desc[k] = (k == j) || (pk >= d0 + j && desc[pk - d0]);
      int l = m->frame_mass[d0 + k];
      if (!desc[k] || l < 0) continue;
      link_mm(m, l, M, scaled);
      m4_mul(W, w->T + 16 * k, dA);
      for (int r = 0; r < 3; ++r)
        for (int x = 0; x < 4; ++x)
          for (int y = 0; y < 4; ++y) s += dA[4 * r + x] * M[4 * x + y] * dA[4 * r + y];
    }
    h[f] = s;
  }
}

void orc_inertia_diag(const orc_model* m, const double* q, double* h, int n_threads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i);
    eval_ws w;
    ws_alloc(&w, nd);
    char* desc = (char*)malloc(nd > 0 ? nd : 1);
    inertia_diag_model(m, i, q, &w, h, desc, 0);
    free(desc);
    ws_free(&w);
  }
}

void orc_energy_report(const orc_model* m, double dt, const double* q_prev, const double* q_curr,
                       double* H, int n_threads) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i), d0 = m->model_dof[i];
    eval_ws w;
    ws_alloc(&w, nd);
    fk_model(m, i, q_curr, w.Tk, w.tl);
    fk_model(m, i, q_prev, w.Tkm1, w.tl);
    double ke = 0.0;
    for (int l = m->link_offset[i]; l < m->link_offset[i + 1]; ++l) {
      int j = m->link_dof[l] + m->dofs_per_link[l] - 1 - d0;
      double M[16];
      mm_full(m->mm + 10 * l, M);
      for (int r = 0; r < 3; ++r) {
        double D[4];
        for (int c = 0; c < 4; ++c) D[c] = w.Tk[16 * j + 4 * r + c] - w.Tkm1[16 * j + 4 * r + c];
        for (int x = 0; x < 4; ++x)
          for (int y = 0; y < 4; ++y) ke += 0.5 * D[x] * M[4 * x + y] * D[y];
      }
    }
    H[i] = ke / (dt * dt) + potential(m, i, w.Tk);
    ws_free(&w);
  }
}

/* Joint-space inertia of model i at q by its plain definition
 *   H_ij = sum_l tr(dA_l/dq_i M_l dA_l/dq_j^T),   dT^l/dq_n = W_n T^l,
 *   W_n  = T^{parent(n)} (dt_n/dq_n) (T^n)^{-1},
 * grouped by the distributive law: only links below both DOFs contribute, so
 * for i an ancestor-or-self of j,  H_ij = tr(W_i C_j W_j^T)  with
 * C_j = sum_{l below j} T^l M_l T^{lT}  (world moment tensor of the subtree). */
static void inertia_matrix_model(const orc_model* m, int i, const double* q, eval_ws* w, double* H,
                                 double* Wb, double* Cb, int scaled) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  fk_model(m, i, q, w->T, w->tl);
  double I4[16], dtl[16], tmp[16], Ti[16], M[16];
  m4_eye(I4);
  for (int j = 0; j < nd; ++j) {
    int f = d0 + j, p = m->frame_parent[f];
    local_dtf(m->axis + 3 * f, q[f], dtl, is_slide(m, f));
    m4_mul(p >= 0 ? w->T + 16 * (p - d0) : I4, dtl, tmp);
    m4_rigid_inv(w->T + 16 * j, Ti);
    m4_mul(tmp, Ti, Wb + 16 * j);
    memset(Cb + 16 * j, 0, 16 * sizeof(double));
    int l = m->frame_mass[f];
    if (l >= 0) {
      link_mm(m, l, M, scaled);
      m4_mul(w->T + 16 * j, M, tmp);
      m4_add_mul_bt(tmp, w->T + 16 * j, Cb + 16 * j);
    }
  }
  for (int j = nd - 1; j >= 0; --j) {
    int p = m->frame_parent[d0 + j];
    if (p >= 0)
      for (int k = 0; k < 16; ++k) Cb[16 * (p - d0) + k] += Cb[16 * j + k];
  }
  memset(H, 0, (size_t)nd * nd * sizeof(double));
  for (int j = 0; j < nd; ++j) {
    for (int a = j; a >= 0; a = m->frame_parent[d0 + a] >= 0 ? m->frame_parent[d0 + a] - d0 : -1) {
      m4_mul(Wb + 16 * a, Cb + 16 * j, tmp);
      double v = m4_frob(tmp, Wb + 16 * j);
      H[(size_t)a * nd + j] = v;
      H[(size_t)j * nd + a] = v;
    }
  }
}

void orc_inertia_matrix(const orc_model* m, const double* q, double* H, int n_threads) {
  size_t* off = (size_t*)malloc((m->n_models + 1) * sizeof(size_t));
  off[0] = 0;
  for (int i = 0; i < m->n_models; ++i) off[i + 1] = off[i] + (size_t)model_nd(m, i) * model_nd(m, i);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i);
    eval_ws w;
    ws_alloc(&w, nd);
    double* Wb = (double*)malloc((size_t)(nd > 0 ? nd : 1) * 32 * sizeof(double));
    inertia_matrix_model(m, i, q, &w, H + off[i], Wb, Wb + 16 * (size_t)(nd > 0 ? nd : 1), 0);
    free(Wb);
    ws_free(&w);
  }
  free(off);
}

/* ------------------------------------------------ second derivatives -- */
/* FK of model i at q (into w->T, w->tl) and the world derivative generator of
 * every frame, W_n = T^{parent(n)} (dt_n/dq_n) (T^n)^{-1}, so that
 * dT^f/dq_n = W_n T^f for every frame f below DOF n. */
static void generators_model(const orc_model* m, int i, const double* q, eval_ws* w, double* Wb) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  fk_model(m, i, q, w->T, w->tl);
  double I4[16], dtl[16], tmp[16], Ti[16];
  m4_eye(I4);
  for (int j = 0; j < nd; ++j) {
    int f = d0 + j, p = m->frame_parent[f];
    local_dtf(m->axis + 3 * f, q[f], dtl, is_slide(m, f));
    m4_mul(p >= 0 ? w->T + 16 * (p - d0) : I4, dtl, tmp);
    m4_rigid_inv(w->T + 16 * j, Ti);
    m4_mul(tmp, Ti, Wb + 16 * j);
  }
}

/* below[a*nd+b] = 1 when frame b is frame a or one of its descendants. */
static void below_model(const orc_model* m, int i, char* below) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  memset(below, 0, (size_t)nd * nd);
  for (int b = 0; b < nd; ++b)
    for (int a = b; a >= 0; a = m->frame_parent[d0 + a] >= 0 ? m->frame_parent[d0 + a] - d0 : -1)
      below[(size_t)a * nd + b] = 1;
}

static size_t* block_offsets(const orc_model* m) {
  size_t* off = (size_t*)malloc((m->n_models + 1) * sizeof(size_t));
  off[0] = 0;
  for (int i = 0; i < m->n_models; ++i) off[i + 1] = off[i] + (size_t)model_nd(m, i) * model_nd(m, i);
  return off;
}

/* Hessian of the step objective of model i at q by its plain definition
 *   d2E/dq_a dq_b = sum_l <dA_l/dq_a M_l, dA_l/dq_b> + <G_l, d2A_l/dq_a dq_b>,
 * with dT^l/dq_n = W_n T^l and, for a an ancestor-or-self of b (both above l),
 * d2T^l/dq_a dq_b = W_a W_b T^l;  G_l = D_l M_l - dt^2 g (M_l e4)^T is the
 * derivative of E with respect to A_l (the seed of Alg. 1's backward pass).
 * Only the three pose rows enter (the last row of every derivative is zero). */
static void hessian_model(const orc_model* m, int i, double dt, const double* q, const double* qk,
                          const double* qkm1, eval_ws* w, double* H, double* Wb, double* Gb, char* below) {
  int d0 = m->model_dof[i], nd = model_nd(m, i);
  double dt2 = dt * dt;
  fk_model(m, i, qk, w->Tk, w->tl);
  fk_model(m, i, qkm1, w->Tkm1, w->tl);
  generators_model(m, i, q, w, Wb);
  below_model(m, i, below);
  memset(Gb, 0, (size_t)nd * 16 * sizeof(double));
  for (int j = 0; j < nd; ++j) {
    int l = m->frame_mass[d0 + j];
    if (l < 0) continue;
    double M[16];
    mm_full(m->mm + 10 * l, M);
    const double *A = w->T + 16 * j, *Ak = w->Tk + 16 * j, *Akm1 = w->Tkm1 + 16 * j;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 4; ++c) {
        double dm = 0.0;
        for (int k = 0; k < 4; ++k) dm += (A[4 * r + k] - 2.0 * Ak[4 * r + k] + Akm1[4 * r + k]) * M[4 * k + c];
        Gb[16 * j + 4 * r + c] = dm - dt2 * m->g[r] * M[4 * c + 3];
      }
    extra_terms(m, l, dt2, M, A, Ak, Gb + 16 * j);
  }
  memset(H, 0, (size_t)nd * nd * sizeof(double));
  double dAa[16], dAb[16], dAaM[16], WW[16], d2A[16], M[16];
  for (int a = 0; a < nd; ++a)
    for (int b = a; b < nd; ++b) {
      if (!below[(size_t)a * nd + b]) continue;
      m4_mul(Wb + 16 * a, Wb + 16 * b, WW);
      double v = 0.0;
      for (int j = b; j < nd; ++j) {
        int l = m->frame_mass[d0 + j];
        if (l < 0 || !below[(size_t)b * nd + j]) continue;
        mm_full(m->mm + 10 * l, M);
        if (m->drag) /* the drag term adds 2 c_l tr(dA M dA'^T) */
          for (int k = 0; k < 16; ++k) M[k] *= 1.0 + 2.0 * m->drag[l];
        m4_mul(Wb + 16 * a, w->T + 16 * j, dAa);
        m4_mul(Wb + 16 * b, w->T + 16 * j, dAb);
        m4_mul(dAa, M, dAaM);
        m4_mul(WW, w->T + 16 * j, d2A);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 4; ++c) v += dAaM[4 * r + c] * dAb[4 * r + c] + Gb[16 * j + 4 * r + c] * d2A[4 * r + c];
        /* contact points: (dx/dq_a)^T d2V/dx2 (dx/dq_b), dx/dq = dA (p;1) */
        if (m->c_off)
          for (int p = m->c_off[l]; p < m->c_off[l + 1]; ++p) {
            const double* pt = m->c_pt + 3 * p;
            double x[3], xk[3], f[3], Hx[9], xa[3], xb[3];
            point_at(w->T + 16 * j, pt, x);
            point_at(w->Tk + 16 * j, pt, xk);
            contact_term(m, dt2, x, xk, f, Hx);
            for (int r = 0; r < 3; ++r) {
              xa[r] = dAa[4 * r] * pt[0] + dAa[4 * r + 1] * pt[1] + dAa[4 * r + 2] * pt[2] + dAa[4 * r + 3];
              xb[r] = dAb[4 * r] * pt[0] + dAb[4 * r + 1] * pt[1] + dAb[4 * r + 2] * pt[2] + dAb[4 * r + 3];
            }
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) v += xa[r] * Hx[3 * r + c] * xb[c];
          }
      }
      H[(size_t)a * nd + b] = v;
      H[(size_t)b * nd + a] = v;
    }
}

void orc_hessian(const orc_model* m, double dt, const double* q, const double* q_hist, double* H,
                 int n_threads) {
  size_t* off = block_offsets(m);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i), n1 = nd > 0 ? nd : 1;
    eval_ws w;
    ws_alloc(&w, nd);
    double* Wb = (double*)malloc((size_t)n1 * 32 * sizeof(double));
    char* below = (char*)malloc((size_t)n1 * n1);
    hessian_model(m, i, dt, q, q_hist + m->n_dofs, q_hist, &w, H + off[i], Wb, Wb + 16 * (size_t)n1, below);
    free(below);
    free(Wb);
    ws_free(&w);
  }
  free(off);
}

/* Mixed second derivative of a pairing  scale * sum_l <A_l(q) M_l, A_l(q_o)>
 * (the form in which E depends on a past configuration: scale -2 for q_k,
 * +1 for q_{k-1}):
 *   C_ab = scale * sum_l <dA_l(q)/dq_a M_l, dA_l(q_o)/dq_o,b>  over links l
 * below both DOFs.  C[a][b] row-major, one block per model. */
void orc_cross_hessian(const orc_model* m, const double* q, const double* q_o, double scale, double* C,
                       int n_threads) {
  size_t* off = block_offsets(m);
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int d0 = m->model_dof[i], nd = model_nd(m, i), n1 = nd > 0 ? nd : 1;
    eval_ws w, wo;
    ws_alloc(&w, nd);
    ws_alloc(&wo, nd);
    double* Wb = (double*)malloc((size_t)n1 * 32 * sizeof(double));
    double* Wo = Wb + 16 * (size_t)n1;
    char* below = (char*)malloc((size_t)n1 * n1);
    generators_model(m, i, q, &w, Wb);
    generators_model(m, i, q_o, &wo, Wo);
    below_model(m, i, below);
    double* Ci = C + off[i];
    double dA[16], dAM[16], dAo[16], M[16];
    for (int a = 0; a < nd; ++a)
      for (int b = 0; b < nd; ++b) {
        double v = 0.0;
        for (int j = 0; j < nd; ++j) {
          int l = m->frame_mass[d0 + j];
          if (l < 0 || !below[(size_t)a * nd + j] || !below[(size_t)b * nd + j]) continue;
          mm_full(m->mm + 10 * l, M);
          m4_mul(Wb + 16 * a, w.T + 16 * j, dA);
          m4_mul(dA, M, dAM);
          m4_mul(Wo + 16 * b, wo.T + 16 * j, dAo);
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 4; ++c) v += dAM[4 * r + c] * dAo[4 * r + c];
        }
        Ci[(size_t)a * nd + b] = scale * v;
      }
    free(below);
    free(Wb);
    ws_free(&wo);
    ws_free(&w);
  }
  free(off);
}

/* Dense Cholesky H = L L^T in place (lower triangle); 0 on success. */
static int cholesky(double* A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(s > 0.0)) return -1;
    double ljj = sqrt(s);
    A[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / ljj;
    }
  }
  return 0;
}
/* x <- (L L^T)^{-1} x */
static void chol_solve(const double* L, int n, double* x) {
  for (int i = 0; i < n; ++i) {
    double t = x[i];
    for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * x[k];
    x[i] = t / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double t = x[i];
    for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * x[k];
    x[i] = t / L[(size_t)i * n + i];
  }
}

/* ------------------------------------------------------------- L-BFGS -- */
static double dotv(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}
static int finitev(const double* a, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

/* Next trial step after a rejected one (backtracking with quadratic
 * interpolation, Nocedal & Wright Sec. 3.5): the minimizer of the parabola
 * through E(0), E'(0) = gd and E(alpha), kept within [0.1, 0.5] alpha; plain
 * halving when E(alpha) is not finite or the parabola has no interior minimum. */
static double next_alpha(double alpha, double E, double Et, double gd) {
  if (!isfinite(Et)) return 0.5 * alpha;
  double den = 2.0 * (Et - E - gd * alpha);
  if (!(den > 0.0)) return 0.5 * alpha;
  double aq = -gd * alpha * alpha / den;
  return aq < 0.1 * alpha ? 0.1 * alpha : (aq > 0.5 * alpha ? 0.5 * alpha : aq);
}

/* v <- gamma * H0 v for the chosen initial inverse Hessian. */
static void apply_H0(int mode, const double* P, const double* L, int nd, double gamma, double* v) {
  if (mode == 2) {
    chol_solve(L, nd, v);
  } else {
    for (int j = 0; j < nd; ++j) v[j] *= gamma * P[j];
  }
}

/* One step of model i (K = 2): preconditioned L-BFGS (two-loop recursion,
 * Liu & Nocedal) from the warm start 2 q_k - q_{k-1}, with a backtracking line
 * search that requires decrease of E (Sec. 4); when the change of E is below
 * the evaluation's own rounding level the sign of the directional derivative
 * decides instead.  Local vectors have length nd; the objective routine uses
 * global DOF indexing, so trial points live in full-length scratch copies. */
static void step_model(const orc_model* m, int i, const orc_opts* o, const double* qkm1,
                       const double* qk, const double* tau, double* qfull, double* gfull,
                       double* q_out, orc_stats* st) {
  const int d0 = m->model_dof[i], nd = model_nd(m, i), M = o->lbfgs_m > 0 ? o->lbfgs_m : 1;
  int mode = o->precond;
  orc_stats s = {0, 0, 0, 0, 0.0, 0.0};
  if (nd == 0) {
    s.flag = 1;
    *st = s;
    return;
  }
  eval_ws w;
  ws_alloc(&w, nd);
  double* buf = (double*)calloc((size_t)nd * (6 + 2 * M) + 3 * M, sizeof(double));
  double *q = buf, *g = q + nd, *d = g + nd, *qt = d + nd, *gt = qt + nd, *P = gt + nd;
  double *Sv = P + nd, *Yv = Sv + (size_t)M * nd, *rho = Yv + (size_t)M * nd, *alp = rho + M,
         *gam = alp + M;
  double* L = NULL;
  char* desc = (char*)malloc(nd);

  fk_model(m, i, qk, w.Tk, w.tl);
  fk_model(m, i, qkm1, w.Tkm1, w.tl);
  /* warm start: constant-velocity extrapolation */
  for (int j = 0; j < nd; ++j) q[j] = 2.0 * qk[d0 + j] - qkm1[d0 + j];
  for (int j = 0; j < nd; ++j) qfull[d0 + j] = q[j];
  for (int j = 0; j < nd; ++j) P[j] = 1.0;
  if (mode == 2) {
    L = (double*)malloc(((size_t)nd * nd + 32 * (size_t)nd) * sizeof(double));
    inertia_matrix_model(m, i, qfull, &w, L, L + (size_t)nd * nd, L + (size_t)nd * nd + 16 * nd, 1);
    if (cholesky(L, nd) != 0) mode = 1; /* not positive definite: fall back to the diagonal */
  }
  if (mode == 1) {
    inertia_diag_model(m, i, qfull, &w, gfull, desc, 1);
    for (int j = 0; j < nd; ++j) {
      double h = gfull[d0 + j];
      P[j] = (h > 0.0 && isfinite(h)) ? 1.0 / h : 1.0;
    }
  }
  double Sn;
  double E = eval_model(m, i, o->dt, qfull, tau, &w, gfull, &Sn);
  for (int j = 0; j < nd; ++j) g[j] = gfull[d0 + j];
  s.evaluations = 1;
  if (!isfinite(E) || !finitev(g, nd)) {
    s.flag = 8;
    s.energy = E;
    s.grad_norm = NAN;
    goto done;
  }
  double g0 = sqrt(dotv(g, g, nd)), gn = g0;
  if (g0 == 0.0) {
    s.flag = 1;
    goto finish;
  }
  int head = 0, count = 0;
  const double c1 = 1e-4, dlt = 0.1;
  for (int it = 0; it < o->max_iter; ++it) {
    if (mode == 2 && o->refresh > 0 && it > 0 && it % o->refresh == 0) {
      /* H_q of the warm start no longer describes the iterate: re-form it at q
       * (qfull holds q after an accepted step) and restart the history */
      inertia_matrix_model(m, i, qfull, &w, L, L + (size_t)nd * nd, L + (size_t)nd * nd + 16 * nd, 1);
      if (cholesky(L, nd) != 0) {
        s.flag = 2;
        break;
      }
      count = 0;
      head = 0;
    }
    /* two-loop recursion, newest pair first */
    for (int j = 0; j < nd; ++j) d[j] = g[j];
    for (int t = 0; t < count; ++t) {
      int k = (head + count - 1 - t) % M;
      alp[k] = rho[k] * dotv(Sv + (size_t)k * nd, d, nd);
      for (int j = 0; j < nd; ++j) d[j] -= alp[k] * Yv[(size_t)k * nd + j];
    }
    double gamma = (count > 0 && mode != 2) ? gam[(head + count - 1) % M] : 1.0;
    apply_H0(mode, P, L, nd, gamma, d);
    for (int t = count - 1; t >= 0; --t) {
      int k = (head + count - 1 - t) % M;
      double b = rho[k] * dotv(Yv + (size_t)k * nd, d, nd);
      for (int j = 0; j < nd; ++j) d[j] += (alp[k] - b) * Sv[(size_t)k * nd + j];
    }
    for (int j = 0; j < nd; ++j) d[j] = -d[j];
    double gd = dotv(g, d, nd);
    if (!(gd < 0.0)) { /* not a descent direction: drop the history */
      count = 0;
      for (int j = 0; j < nd; ++j) d[j] = g[j];
      apply_H0(mode, P, L, nd, 1.0, d);
      for (int j = 0; j < nd; ++j) d[j] = -d[j];
      gd = dotv(g, d, nd);
      if (!(gd < 0.0)) { /* H0 not positive definite along g: give up */
        s.flag = 2;
        break;
      }
    }
    /* backtracking line search */
    double alpha = 1.0, Et = 0.0, St = 0.0;
    int ok = 0;
    for (int ls = 0; ls < o->max_ls; ++ls) {
      for (int j = 0; j < nd; ++j) qt[j] = q[j] + alpha * d[j];
      for (int j = 0; j < nd; ++j) qfull[d0 + j] = qt[j];
      Et = eval_model(m, i, o->dt, qfull, tau, &w, gfull, &St);
      for (int j = 0; j < nd; ++j) gt[j] = gfull[d0 + j];
      s.evaluations++;
      if (isfinite(Et) && finitev(gt, nd)) {
        if (Et <= E + c1 * alpha * gd)
          ok = 1;
        else if (fabs(Et - E) <= 10.0 * o->eps_w * St) {
          /* change of E within rounding: accept unless the slope shows overshoot */
          double gtd = dotv(gt, d, nd);
          if (gtd <= (2.0 * dlt - 1.0) * gd) ok = 1;
        }
      }
      if (ok) break;
      alpha = next_alpha(alpha, E, Et, gd);
    }
    if (!ok) {
      s.flag = 2;
      break;
    }
    /* an accepted point equal to q in every coordinate is no progress: the
     * iteration cannot move at this precision */
    int moved = 0;
    for (int j = 0; j < nd; ++j) moved |= qt[j] != q[j];
    if (!moved) {
      s.flag = 2;
      break;
    }
    /* curvature pair */
    for (int j = 0; j < nd; ++j) qt[j] -= q[j]; /* s = accepted point - q */
    double sy = 0.0, ss = 0.0, yy = 0.0, yPy = 0.0;
    for (int j = 0; j < nd; ++j) {
      double yj = gt[j] - g[j];
      sy += qt[j] * yj;
      ss += qt[j] * qt[j];
      yy += yj * yj;
      yPy += yj * P[j] * yj;
    }
    if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
      int k;
      if (count < M) {
        k = (head + count) % M;
        count++;
      } else {
        k = head;
        head = (head + 1) % M;
      }
      for (int j = 0; j < nd; ++j) {
        Sv[(size_t)k * nd + j] = qt[j];
        Yv[(size_t)k * nd + j] = gt[j] - g[j];
      }
      rho[k] = 1.0 / sy;
      gam[k] = sy / yPy;
    }
    for (int j = 0; j < nd; ++j) {
      q[j] = qfull[d0 + j];
      g[j] = gt[j];
    }
    E = Et;
    s.iterations++;
    gn = sqrt(dotv(g, g, nd));
    if (gn <= o->tol * g0) {
      s.flag = 1;
      break;
    }
  }
  if (s.flag == 0) s.flag = 4;
finish:
  s.grad_norm = gn;
  s.energy = E;
done:
  for (int j = 0; j < nd; ++j) q_out[d0 + j] = q[j];
  *st = s;
  free(L);
  free(desc);
  free(buf);
  ws_free(&w);
}

int orc_step(const orc_model* m, const orc_opts* o, const double* q_hist, const double* tau,
             double* q_out, orc_stats* stats, int n_threads) {
  if (o->order_K != 2) return -1;
  const double* qkm1 = q_hist;
  const double* qk = q_hist + m->n_dofs;
  int nd = m->n_dofs > 0 ? m->n_dofs : 1;
  int nt = n_threads > 0 ? n_threads : 1;
  double* scratch = (double*)malloc((size_t)nt * 2 * nd * sizeof(double));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int i = 0; i < m->n_models; ++i) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* qfull = scratch + (size_t)tid * 2 * nd;
    double* gfull = qfull + nd;
    step_model(m, i, o, qkm1, qk, tau, qfull, gfull, q_out, stats + i);
  }
  free(scratch);
  return 0;
}

/* ------------------------------------------ high-order collocation (K>2) -- */
/* Sec. 4, Eq. HOC / Eq. EQHOC.  Collocation points of order K: alpha_1 < ... <
 * alpha_{K-2} are the roots of the Legendre polynomial L_{K-2}(2 alpha - 1) and
 * alpha_{K-1} = 1.  The K+1 points of one step, in units of dt from t_k, are
 *   tau = (alpha_{K-2} - 1, 0, alpha_1, ..., alpha_{K-1})
 * (the first is the previous step's alpha_{K-2} point; alpha_0 = 0 for K = 2).
 * Every body point follows the polynomial through its positions at these
 * points, so dt^2 Pddot(tau_i) = sum_j w_ij P_j with w_ij = L_j''(tau_i) for the
 * Lagrange basis L_j through the points. */
#define ORC_KMAX 8

/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence. */
static double legendre(int n, double x, double* dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *dp = 0.0;
    return 1.0;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *dp = n * (x * p1 - p0) / (x * x - 1.0);
  return p1;
}

int orc_collocation(int K, double* tau, double* w) {
  if (K < 2 || K > ORC_KMAX) return -1;
  int n = K - 2;
  double alpha[ORC_KMAX + 1];
  /* roots of P_n by Newton from the usual cosine guesses, ascending in alpha */
  for (int r = 0; r < n; ++r) {
    double x = cos(acos(-1.0) * (r + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double dp, p = legendre(n, x, &dp);
      double dx = p / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    alpha[n - r] = 0.5 * (x + 1.0); /* index 1..n ascending */
  }
  alpha[0] = 0.0;
  alpha[K - 1] = 1.0;
  tau[0] = alpha[K - 2] - 1.0;
  tau[1] = 0.0;
  for (int u = 1; u <= K - 1; ++u) tau[1 + u] = alpha[u];
  /* w[u][j] = L_j''(tau_{1+u}), u = 0..K-2 (the unknown points), j = 0..K */
  int np = K + 1;
  for (int u = 0; u < K - 1; ++u) {
    double x = tau[2 + u];
    for (int j = 0; j < np; ++j) {
      double den = 1.0;
      for (int a = 0; a < np; ++a)
        if (a != j) den *= tau[j] - tau[a];
      double num = 0.0;
      for (int a = 0; a < np; ++a) {
        if (a == j) continue;
        for (int b = 0; b < np; ++b) {
          if (b == j || b == a) continue;
          double prod = 1.0;
          for (int c = 0; c < np; ++c)
            if (c != j && c != a && c != b) prod *= x - tau[c];
          num += prod;
        }
      }
      w[u * np + j] = num / den;
    }
  }
  return 0;
}

/* Per-model work space of the EQHOC evaluation: poses T (and local transforms
 * tl) of all K+1 points, derivative generators of the K-1 unknown points, the
 * seeds and residuals of the unknown points. */
typedef struct {
  int K, nd;
  double *T, *tl, *Wg, *G, *res, *Adj, *blk;
  char* below;
} hoc_ws;

static void hoc_alloc(hoc_ws* h, int K, int nd) {
  int n1 = nd > 0 ? nd : 1;
  h->K = K;
  h->nd = nd;
  h->T = (double*)malloc((size_t)(K + 1) * n1 * 16 * sizeof(double));
  h->tl = (double*)malloc((size_t)(K + 1) * n1 * 16 * sizeof(double));
  h->Wg = (double*)malloc((size_t)(K + 1) * n1 * 16 * sizeof(double));
  h->G = (double*)malloc((size_t)(K - 1) * n1 * 16 * sizeof(double));
  h->res = (double*)malloc((size_t)(K - 1) * n1 * sizeof(double));
  h->Adj = (double*)malloc((size_t)n1 * 16 * sizeof(double));
  h->blk = (double*)malloc((size_t)n1 * n1 * sizeof(double));
  h->below = (char*)malloc((size_t)n1 * n1);
}
static void hoc_free(hoc_ws* h) {
  free(h->T); free(h->tl); free(h->Wg); free(h->G); free(h->res); free(h->Adj); free(h->blk);
  free(h->below);
}

/* EQHOC objective of model i and its gradient with respect to the K-1 unknown
 * configurations.  pts[p] (p = 0..K) are full-length DOF vectors: the two known
 * points and the unknowns.  Per unknown u (point p = 2+u):
 *   dt^2 r_u = sum_p w_up dI(q_u, q_p)/dq_u - dt^2 dV/dq... as the Alg. 1
 *   backward pass at q_u of the seed G_u = sum_p w_up A(q_p) M - dt^2 g (M e4)^T,
 *   minus dt^2 tau (generalized force);
 *   E = sum_u |dt^2 r_u|^2.
 * Gradient dE/dq_a = 2 sum_u J_ua^T (dt^2 r_u) with the blocks
 *   J_uu = S(q_u; G_u) + w_u,(2+u) C(q_u, q_u),   J_ua = w_u,(2+a) C(q_u, q_a),
 *   S(q; G)_bc = sum_l <G_l, d2A_l(q)/dq_b dq_c>,
 *   C(q, q')_bc = sum_l <dA_l(q)/dq_b M_l, dA_l(q')/dq'_c>,
 * written out from the pose derivatives (dT/dq_n = W_n T, d2T/dq_b dq_c = W_b W_c T).
 * grad (may be NULL) receives [K-1][nd] local values; res_out (may be NULL) the
 * scaled residuals dt^2 r_u ([K-1][nd]); jac_out (may be NULL) the Jacobian of
 * those residuals, row (u, b), column (a, c), row-major [(K-1) nd]^2. */
static double hoc_eval_model(const orc_model* m, int i, int K, const double* w, double dt,
                             const double* const* pts, const double* tau, hoc_ws* h, double* grad,
                             double* res_out, double* jac_out) {
  const int d0 = m->model_dof[i], nd = model_nd(m, i), np = K + 1, U = K - 1;
  const double dt2 = dt * dt;
  eval_ws ew;
  ws_alloc(&ew, nd);
  for (int p = 0; p < np; ++p) {
    if (p >= 2) {
      generators_model(m, i, pts[p], &ew, h->Wg + (size_t)p * nd * 16);
    } else {
      fk_model(m, i, pts[p], ew.T, ew.tl);
    }
    memcpy(h->T + (size_t)p * nd * 16, ew.T, (size_t)nd * 16 * sizeof(double));
    memcpy(h->tl + (size_t)p * nd * 16, ew.tl, (size_t)nd * 16 * sizeof(double));
  }
  below_model(m, i, h->below);
  double E = 0.0;
  for (int u = 0; u < U; ++u) {
    double* G = h->G + (size_t)u * nd * 16;
    memset(G, 0, (size_t)nd * 16 * sizeof(double));
    for (int j = 0; j < nd; ++j) {
      int l = m->frame_mass[d0 + j];
      if (l < 0) continue;
      double M[16], TM[16];
      mm_full(m->mm + 10 * l, M);
      for (int p = 0; p < np; ++p) {
        m4_mul(h->T + ((size_t)p * nd + j) * 16, M, TM);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 4; ++c) G[16 * j + 4 * r + c] += w[u * np + p] * TM[4 * r + c];
      }
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 4; ++c) G[16 * j + 4 * r + c] -= dt2 * m->g[r] * M[4 * c + 3];
    }
    /* residual: Alg. 1 backward pass at q_u with the seed G_u */
    memcpy(h->Adj, G, (size_t)nd * 16 * sizeof(double));
    double* r = h->res + (size_t)u * nd;
    double* gfull = (double*)calloc((size_t)m->n_dofs > 0 ? m->n_dofs : 1, sizeof(double));
    alg1_backward(m, i, h->T + (size_t)(2 + u) * nd * 16, h->tl + (size_t)(2 + u) * nd * 16, h->Adj,
                  pts[2 + u], gfull);
    for (int j = 0; j < nd; ++j) r[j] = gfull[d0 + j] - (tau ? dt2 * tau[d0 + j] : 0.0);
    free(gfull);
    for (int j = 0; j < nd; ++j) E += r[j] * r[j];
  }
  if (res_out) memcpy(res_out, h->res, (size_t)U * nd * sizeof(double));
  if (grad || jac_out) {
    if (grad) memset(grad, 0, (size_t)U * nd * sizeof(double));
    double WW[16], d2A[16], dA[16], dAM[16], dAo[16], M[16];
    for (int u = 0; u < U; ++u) {
      const double* Tu = h->T + (size_t)(2 + u) * nd * 16;
      const double* Wu = h->Wg + (size_t)(2 + u) * nd * 16;
      const double* G = h->G + (size_t)u * nd * 16;
      const double* r = h->res + (size_t)u * nd;
      for (int a = 0; a < U; ++a) {
        const double* Ta = h->T + (size_t)(2 + a) * nd * 16;
        const double* Wa = h->Wg + (size_t)(2 + a) * nd * 16;
        const double wua = w[u * np + 2 + a];
        /* block J_ua (rows: residual components b, columns: DOFs c of q_a) */
        for (int b = 0; b < nd; ++b)
          for (int c = 0; c < nd; ++c) {
            double v = 0.0;
            if (a == u) {
              /* S(q_u; G_u)_bc, b or c the ancestor */
              int lo = b < c ? b : c, hi = b < c ? c : b;
              if (h->below[(size_t)lo * nd + hi]) {
                m4_mul(Wu + 16 * lo, Wu + 16 * hi, WW);
                for (int j = hi; j < nd; ++j) {
                  if (m->frame_mass[d0 + j] < 0 || !h->below[(size_t)hi * nd + j]) continue;
                  m4_mul(WW, Tu + 16 * j, d2A);
                  for (int x = 0; x < 12; ++x) v += G[16 * j + x] * d2A[x];
                }
              }
            }
            if (wua != 0.0) {
              double cv = 0.0;
              for (int j = 0; j < nd; ++j) {
                int l = m->frame_mass[d0 + j];
                if (l < 0 || !h->below[(size_t)b * nd + j] || !h->below[(size_t)c * nd + j]) continue;
                mm_full(m->mm + 10 * l, M);
                m4_mul(Wu + 16 * b, Tu + 16 * j, dA);
                m4_mul(dA, M, dAM);
                m4_mul(Wa + 16 * c, Ta + 16 * j, dAo);
                for (int x = 0; x < 12; ++x) cv += dAM[x] * dAo[x];
              }
              v += wua * cv;
            }
            h->blk[(size_t)b * nd + c] = v;
          }
        if (jac_out)
          for (int b = 0; b < nd; ++b)
            memcpy(jac_out + ((size_t)u * nd + b) * U * nd + (size_t)a * nd, h->blk + (size_t)b * nd,
                   (size_t)nd * sizeof(double));
        if (grad)
          for (int c = 0; c < nd; ++c) {
            double s = 0.0;
            for (int b = 0; b < nd; ++b) s += h->blk[(size_t)b * nd + c] * r[b];
            grad[(size_t)a * nd + c] += 2.0 * s;
          }
      }
    }
  }
  ws_free(&ew);
  return E;
}

void orc_eqhoc_objective_grad(const orc_model* m, int K, double dt, const double* q_known,
                              const double* q_unknown, const double* tau, double* E, double* grad,
                              int n_threads) {
  double tauv[ORC_KMAX + 1], w[(ORC_KMAX - 1) * (ORC_KMAX + 1)];
  orc_collocation(K, tauv, w);
  const int n = m->n_dofs, U = K - 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i), d0 = m->model_dof[i];
    const double* pts[ORC_KMAX + 1];
    pts[0] = q_known;
    pts[1] = q_known + n;
    for (int u = 0; u < U; ++u) pts[2 + u] = q_unknown + (size_t)u * n;
    hoc_ws h;
    hoc_alloc(&h, K, nd);
    double* g = grad ? (double*)malloc((size_t)U * (nd > 0 ? nd : 1) * sizeof(double)) : NULL;
    E[i] = hoc_eval_model(m, i, K, w, dt, pts, tau, &h, g, NULL, NULL);
    if (grad)
      for (int u = 0; u < U; ++u)
        for (int j = 0; j < nd; ++j) grad[(size_t)u * n + d0 + j] = g[(size_t)u * nd + j];
    free(g);
    hoc_free(&h);
  }
}

/* Residuals dt^2 r_u of Eq. HOC at the K-1 unknown configurations ([K-1][n_dofs],
 * global DOF order) and, if J is not NULL, their Jacobian with respect to the
 * unknowns: one dense row-major block of ((K-1) nd)^2 doubles per model, packed
 * model after model, row (u, b) and column (a, c) in unknown-major order. */
void orc_eqhoc_residual_jacobian(const orc_model* m, int K, double dt, const double* q_known,
                                 const double* q_unknown, const double* tau, double* R, double* J,
                                 int n_threads) {
  double tauv[ORC_KMAX + 1], w[(ORC_KMAX - 1) * (ORC_KMAX + 1)];
  orc_collocation(K, tauv, w);
  const int n = m->n_dofs, U = K - 1;
  size_t* joff = (size_t*)malloc(((size_t)m->n_models + 1) * sizeof(size_t));
  joff[0] = 0;
  for (int i = 0; i < m->n_models; ++i) {
    size_t N = (size_t)U * model_nd(m, i);
    joff[i + 1] = joff[i] + N * N;
  }
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads > 0 ? n_threads : 1)
  for (int i = 0; i < m->n_models; ++i) {
    int nd = model_nd(m, i), d0 = m->model_dof[i];
    const double* pts[ORC_KMAX + 1];
    pts[0] = q_known;
    pts[1] = q_known + n;
    for (int u = 0; u < U; ++u) pts[2 + u] = q_unknown + (size_t)u * n;
    hoc_ws h;
    hoc_alloc(&h, K, nd);
    double* r = (double*)malloc((size_t)U * (nd > 0 ? nd : 1) * sizeof(double));
    hoc_eval_model(m, i, K, w, dt, pts, tau, &h, NULL, r, J ? J + joff[i] : NULL);
    for (int u = 0; u < U; ++u)
      for (int j = 0; j < nd; ++j) R[(size_t)u * n + d0 + j] = r[(size_t)u * nd + j];
    free(r);
    hoc_free(&h);
  }
  free(joff);
}

/* Dense inverse of a small matrix by Gauss-Jordan with partial pivoting; 0 on success. */
static int small_inverse(const double* A, int n, double* X) {
  double a[ORC_KMAX * ORC_KMAX * 2];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) a[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(a[r * 2 * n + c]) > fabs(a[p * 2 * n + c])) p = r;
    if (a[p * 2 * n + c] == 0.0) return -1;
    for (int k = 0; k < 2 * n; ++k) {
      double t = a[c * 2 * n + k];
      a[c * 2 * n + k] = a[p * 2 * n + k];
      a[p * 2 * n + k] = t;
    }
    double piv = a[c * 2 * n + c];
    for (int k = 0; k < 2 * n; ++k) a[c * 2 * n + k] /= piv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * 2 * n + c];
      for (int k = 0; k < 2 * n; ++k) a[r * 2 * n + k] -= f * a[c * 2 * n + k];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) X[r * n + c] = a[r * 2 * n + n + c];
  return 0;
}

/* One EQHOC step of model i (Sec. 4-5): L-BFGS over the K-1 unknown
 * configurations with the same line search and termination as the K = 2 step.
 * Warm start: constant velocity from the two known points,
 * q_u = q_k + alpha_u (q_k - q_prev) / (1 - alpha_{K-2}).  Initial inverse
 * Hessian (precond 2): E is a sum of squares whose Jacobian is close to
 * W_uu (x) H_q (W_uu: weights among the unknown points, H_q: joint-space
 * inertia at q_k), so H0 = (W_uu^T W_uu)^-1 (x) H_q^-2; precond 0: gamma I. */
static void step_model_hoc(const orc_model* m, int i, const orc_opts* o, const double* qprev, const double* qk,
                           const double* tau, double* qunk_full, double* q_out, orc_stats* st) {
  const int K = o->order_K, U = K - 1, np = K + 1, n = m->n_dofs;
  const int d0 = m->model_dof[i], nd = model_nd(m, i), N = U * nd, Mh = o->lbfgs_m > 0 ? o->lbfgs_m : 1;
  orc_stats s = {0, 0, 0, 0, 0.0, 0.0};
  if (nd == 0) {
    s.flag = 1;
    *st = s;
    return;
  }
  double tauv[ORC_KMAX + 1], w[(ORC_KMAX - 1) * (ORC_KMAX + 1)];
  orc_collocation(K, tauv, w);
  int mode = o->precond == 2 ? 2 : 0;
  double* buf = (double*)calloc((size_t)N * (6 + 2 * Mh) + 3 * Mh, sizeof(double));
  double *q = buf, *g = q + N, *d = g + N, *qt = d + N, *gt = qt + N, *tmp = gt + N;
  double *Sv = tmp + N, *Yv = Sv + (size_t)Mh * N, *rho = Yv + (size_t)Mh * N, *alp = rho + Mh, *gam = alp + Mh;
  double* L = NULL;
  double Minv[ORC_KMAX * ORC_KMAX];
  hoc_ws h;
  hoc_alloc(&h, K, nd);
  const double* pts[ORC_KMAX + 1];
  pts[0] = qprev;
  pts[1] = qk;
  for (int u = 0; u < U; ++u) pts[2 + u] = qunk_full + (size_t)u * n;

  const double vscale = 1.0 / (tauv[1] - tauv[0]);
  for (int u = 0; u < U; ++u)
    for (int j = 0; j < nd; ++j)
      q[u * nd + j] = qk[d0 + j] + tauv[2 + u] * vscale * (qk[d0 + j] - qprev[d0 + j]);
  if (mode == 2) {
    double Wuu[ORC_KMAX * ORC_KMAX], WtW[ORC_KMAX * ORC_KMAX];
    for (int u = 0; u < U; ++u)
      for (int a = 0; a < U; ++a) Wuu[u * U + a] = w[u * np + 2 + a];
    for (int a = 0; a < U; ++a)
      for (int b = 0; b < U; ++b) {
        double t = 0.0;
        for (int u = 0; u < U; ++u) t += Wuu[u * U + a] * Wuu[u * U + b];
        WtW[a * U + b] = t;
      }
    eval_ws ew;
    ws_alloc(&ew, nd);
    L = (double*)malloc(((size_t)nd * nd + 32 * (size_t)nd) * sizeof(double));
    inertia_matrix_model(m, i, qk, &ew, L, L + (size_t)nd * nd, L + (size_t)nd * nd + 16 * nd, 0);
    ws_free(&ew);
    if (cholesky(L, nd) != 0 || small_inverse(WtW, U, Minv) != 0) mode = 0;
  }
#define HOC_EVAL(X, GRAD, EOUT)                                                     \
  do {                                                                              \
    for (int u_ = 0; u_ < U; ++u_)                                                  \
      for (int j_ = 0; j_ < nd; ++j_) qunk_full[(size_t)u_ * n + d0 + j_] = (X)[u_ * nd + j_]; \
    EOUT = hoc_eval_model(m, i, K, w, o->dt, pts, tau, &h, GRAD, NULL, NULL);       \
  } while (0)
  double E;
  HOC_EVAL(q, g, E);
  s.evaluations = 1;
  if (!isfinite(E) || !finitev(g, N)) {
    s.flag = 8;
    s.energy = E;
    s.grad_norm = NAN;
    goto done;
  }
  double g0 = sqrt(dotv(g, g, N)), gn = g0;
  if (g0 == 0.0) {
    s.flag = 1;
    goto finish;
  }
  int head = 0, count = 0;
  const double c1 = 1e-4, dlt = 0.1;
  for (int it = 0; it < o->max_iter; ++it) {
    for (int j = 0; j < N; ++j) d[j] = g[j];
    for (int t = 0; t < count; ++t) {
      int k = (head + count - 1 - t) % Mh;
      alp[k] = rho[k] * dotv(Sv + (size_t)k * N, d, N);
      for (int j = 0; j < N; ++j) d[j] -= alp[k] * Yv[(size_t)k * N + j];
    }
    /* initial inverse Hessian */
    if (mode == 2) {
      for (int u = 0; u < U; ++u) {
        chol_solve(L, nd, d + (size_t)u * nd);
        chol_solve(L, nd, d + (size_t)u * nd);
      }
      for (int u = 0; u < U; ++u)
        for (int j = 0; j < nd; ++j) {
          double t = 0.0;
          for (int a = 0; a < U; ++a) t += Minv[u * U + a] * d[(size_t)a * nd + j];
          tmp[(size_t)u * nd + j] = t;
        }
      memcpy(d, tmp, (size_t)N * sizeof(double));
    } else {
      double gamma = count > 0 ? gam[(head + count - 1) % Mh] : 1.0;
      for (int j = 0; j < N; ++j) d[j] *= gamma;
    }
    for (int t = count - 1; t >= 0; --t) {
      int k = (head + count - 1 - t) % Mh;
      double b = rho[k] * dotv(Yv + (size_t)k * N, d, N);
      for (int j = 0; j < N; ++j) d[j] += (alp[k] - b) * Sv[(size_t)k * N + j];
    }
    for (int j = 0; j < N; ++j) d[j] = -d[j];
    double gd = dotv(g, d, N);
    if (!(gd < 0.0)) {
      if (count > 0) {
        count = 0;
        --it;
        continue; /* redo the direction with an empty history */
      }
      s.flag = 2;
      break;
    }
    double alpha = 1.0, Et = 0.0;
    int ok = 0;
    for (int ls = 0; ls < o->max_ls; ++ls) {
      for (int j = 0; j < N; ++j) qt[j] = q[j] + alpha * d[j];
      HOC_EVAL(qt, gt, Et);
      s.evaluations++;
      if (isfinite(Et) && finitev(gt, N)) {
        if (Et <= E + c1 * alpha * gd)
          ok = 1;
        else if (fabs(Et - E) <= 10.0 * o->eps_w * Et) {
          double gtd = dotv(gt, d, N);
          if (gtd <= (2.0 * dlt - 1.0) * gd) ok = 1;
        }
      }
      if (ok) break;
      alpha = next_alpha(alpha, E, Et, gd);
    }
    if (!ok) {
      s.flag = 2;
      break;
    }
    int moved = 0; /* an accepted point equal to q is no progress (as for order 2) */
    for (int j = 0; j < N; ++j) moved |= qt[j] != q[j];
    if (!moved) {
      s.flag = 2;
      break;
    }
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int j = 0; j < N; ++j) {
      double sj = qt[j] - q[j], yj = gt[j] - g[j];
      sy += sj * yj;
      ss += sj * sj;
      yy += yj * yj;
    }
    if (sy > 1e-12 * sqrt(ss) * sqrt(yy)) {
      int k;
      if (count < Mh) {
        k = (head + count) % Mh;
        count++;
      } else {
        k = head;
        head = (head + 1) % Mh;
      }
      for (int j = 0; j < N; ++j) {
        Sv[(size_t)k * N + j] = qt[j] - q[j];
        Yv[(size_t)k * N + j] = gt[j] - g[j];
      }
      rho[k] = 1.0 / sy;
      gam[k] = sy / yy;
    }
    memcpy(q, qt, (size_t)N * sizeof(double));
    memcpy(g, gt, (size_t)N * sizeof(double));
    E = Et;
    s.iterations++;
    gn = sqrt(dotv(g, g, N));
    if (gn <= o->tol * g0) {
      s.flag = 1;
      break;
    }
  }
  if (s.flag == 0) s.flag = 4;
finish:
  s.grad_norm = gn;
  s.energy = E;
done:
  for (int u = 0; u < U; ++u)
    for (int j = 0; j < nd; ++j) q_out[(size_t)u * n + d0 + j] = q[u * nd + j];
  *st = s;
#undef HOC_EVAL
  free(L);
  free(buf);
  hoc_free(&h);
}

/* One Eq. EQHOC step of model i by Levenberg-Marquardt (Sec. 5 "Optimization
 * Algorithm"): each iteration forms the residuals r = (dt^2 r_u) and their
 * Jacobian J (written out, hoc_eval_model), and solves
 *     (J^T J + lambda I) v = -J^T r              (the paper's update; dense Cholesky)
 * E = |r|^2, dE/dq = 2 J^T r.  lambda starts at lambda0 * max diag(J^T J) and is
 * adapted by the gain ratio rho = (E - E(q+s)) / (E - |r + J s|^2) of the step s
 * (Nielsen's rule: accepted steps scale lambda by max(1/3, 1 - (2 rho - 1)^3),
 * rejected ones by nu, nu doubling while steps are rejected).  A step is
 * accepted when it decreases E.  With `geodesic`, the step adds half the
 * geodesic acceleration of Transtrum & Sethna's LM variant: with the second
 * directional derivative of the residuals along v from a finite difference of
 * step h, r_vv = (2/h) ((r(q + h v) - r)/h - J v), a = (J^T J + lambda I)^-1
 * (-J^T r_vv) and s = v + a/2; a step whose acceleration is large against its
 * velocity (2|a| > alpha |v|) is rejected like one that increases E.
 * lambda is kept at least 1e-15 max diag(J^T J) so that the Cholesky factor
 * exists.  Stop when |dE/dq| <= tol |dE/dq at the warm start| (flag 1), when an
 * accepted point equals the iterate or lambda overflows (flag 2), or after
 * max_iter iterations, accepted or not (flag 4).  Warm start as orc_step_hoc. */
static void step_model_lm(const orc_model* m, int i, const orc_lm_opts* o, const double* qprev,
                          const double* qk, const double* tau, double* qunk_full, double* q_out,
                          orc_stats* st) {
  const int K = o->order_K, U = K - 1, n = m->n_dofs;
  const int d0 = m->model_dof[i], nd = model_nd(m, i), N = U * nd;
  orc_stats s = {0, 0, 0, 0, 0.0, 0.0};
  if (nd == 0) {
    s.flag = 1;
    *st = s;
    return;
  }
  double tauv[ORC_KMAX + 1], w[(ORC_KMAX - 1) * (ORC_KMAX + 1)];
  orc_collocation(K, tauv, w);
  hoc_ws h;
  hoc_alloc(&h, K, nd);
  const double* pts[ORC_KMAX + 1];
  pts[0] = qprev;
  pts[1] = qk;
  for (int u = 0; u < U; ++u) pts[2 + u] = qunk_full + (size_t)u * n;
  double* buf = (double*)calloc((size_t)N * 11, sizeof(double));
  double *q = buf, *r = q + N, *g = r + N, *v = g + N, *a = v + N, *qt = a + N, *rt = qt + N, *Jv = rt + N,
         *rvv = Jv + N, *sv = rvv + N, *tmp = sv + N;
  double* J = (double*)malloc((size_t)N * N * sizeof(double));
  double* JTJ = (double*)malloc((size_t)N * N * sizeof(double));
  double* L = (double*)malloc((size_t)N * N * sizeof(double));
#define LM_RES(X, ROUT, JOUT, EOUT)                                                 \
  do {                                                                              \
    for (int u_ = 0; u_ < U; ++u_)                                                  \
      for (int j_ = 0; j_ < nd; ++j_) qunk_full[(size_t)u_ * n + d0 + j_] = (X)[u_ * nd + j_]; \
    EOUT = hoc_eval_model(m, i, K, w, o->dt, pts, tau, &h, NULL, ROUT, JOUT);       \
    ++s.evaluations;                                                                \
  } while (0)
  const double vscale = 1.0 / (tauv[1] - tauv[0]);
  for (int u = 0; u < U; ++u)
    for (int j = 0; j < nd; ++j) q[u * nd + j] = qk[d0 + j] + tauv[2 + u] * vscale * (qk[d0 + j] - qprev[d0 + j]);
  double E;
  LM_RES(q, r, J, E);
  /* g = J^T r */
  for (int c = 0; c < N; ++c) {
    double t = 0.0;
    for (int k = 0; k < N; ++k) t += J[(size_t)k * N + c] * r[k];
    g[c] = t;
  }
  if (!isfinite(E) || !finitev(g, N)) {
    s.flag = 8;
    s.energy = E;
    s.grad_norm = NAN;
    goto out;
  }
  const double g0 = 2.0 * sqrt(dotv(g, g, N));
  double gn = g0, lambda = -1.0, nu = 2.0;
  if (g0 == 0.0) {
    s.flag = 1;
    goto fin;
  }
  for (int it = 0; it < o->max_iter; ++it) {
    s.iterations++;
    double dmax = 0.0;
    for (int x = 0; x < N; ++x)
      for (int y = 0; y <= x; ++y) {
        double t = 0.0;
        for (int k = 0; k < N; ++k) t += J[(size_t)k * N + x] * J[(size_t)k * N + y];
        JTJ[(size_t)x * N + y] = t;
        JTJ[(size_t)y * N + x] = t;
      }
    for (int x = 0; x < N; ++x) dmax = fmax(dmax, JTJ[(size_t)x * N + x]);
    if (lambda < 0.0) lambda = o->lambda0 * dmax;
    if (lambda < 1e-15 * dmax) lambda = 1e-15 * dmax;
    if (!(lambda <= 1e300)) {
      s.flag = 2;
      break;
    }
    memcpy(L, JTJ, (size_t)N * N * sizeof(double));
    for (int x = 0; x < N; ++x) L[(size_t)x * N + x] += lambda;
    if (cholesky(L, N) != 0) {
      lambda *= nu;
      nu *= 2.0;
      continue;
    }
    for (int x = 0; x < N; ++x) v[x] = -g[x];
    chol_solve(L, N, v);
    /* J v */
    for (int k = 0; k < N; ++k) {
      double t = 0.0;
      for (int c = 0; c < N; ++c) t += J[(size_t)k * N + c] * v[c];
      Jv[k] = t;
    }
    memcpy(sv, v, (size_t)N * sizeof(double));
    if (o->geodesic) {
      const double hh = o->geo_h;
      double Eh;
      for (int x = 0; x < N; ++x) qt[x] = q[x] + hh * v[x];
      LM_RES(qt, rt, NULL, Eh);
      (void)Eh;
      for (int k = 0; k < N; ++k) rvv[k] = (2.0 / hh) * ((rt[k] - r[k]) / hh - Jv[k]);
      for (int c = 0; c < N; ++c) {
        double t = 0.0;
        for (int k = 0; k < N; ++k) t += J[(size_t)k * N + c] * rvv[k];
        a[c] = -t;
      }
      chol_solve(L, N, a);
      const double na = sqrt(dotv(a, a, N)), nv = sqrt(dotv(v, v, N));
      if (!(2.0 * na <= o->geo_alpha * nv)) {
        lambda *= nu;
        nu *= 2.0;
        continue;
      }
      for (int x = 0; x < N; ++x) sv[x] = v[x] + 0.5 * a[x];
    }
    /* predicted objective |r + J s|^2 */
    double pred = 0.0;
    for (int k = 0; k < N; ++k) {
      double t = r[k];
      for (int c = 0; c < N; ++c) t += J[(size_t)k * N + c] * sv[c];
      pred += t * t;
    }
    for (int x = 0; x < N; ++x) qt[x] = q[x] + sv[x];
    double Et;
    LM_RES(qt, rt, NULL, Et);
    if (!(isfinite(Et) && Et < E)) {
      lambda *= nu;
      nu *= 2.0;
      continue;
    }
    int moved = 0;
    for (int x = 0; x < N; ++x) moved |= qt[x] != q[x];
    if (!moved) {
      s.flag = 2;
      break;
    }
    double rho = (E - Et) / fmax(E - pred, 1e-300);
    if (rho > 1.0) rho = 1.0;
    const double c3 = 2.0 * rho - 1.0;
    lambda *= fmax(1.0 / 3.0, 1.0 - c3 * c3 * c3);
    nu = 2.0;
    memcpy(q, qt, (size_t)N * sizeof(double));
    LM_RES(q, r, J, E);
    for (int c = 0; c < N; ++c) {
      double t = 0.0;
      for (int k = 0; k < N; ++k) t += J[(size_t)k * N + c] * r[k];
      g[c] = t;
    }
    gn = 2.0 * sqrt(dotv(g, g, N));
    if (gn <= o->tol * g0) {
      s.flag = 1;
      break;
    }
  }
  if (s.flag == 0) s.flag = 4;
fin:
  s.grad_norm = gn;
  s.energy = E;
out:
  for (int u = 0; u < U; ++u)
    for (int j = 0; j < nd; ++j) q_out[(size_t)u * n + d0 + j] = q[u * nd + j];
  *st = s;
#undef LM_RES
  (void)tmp;
  free(J);
  free(JTJ);
  free(L);
  free(buf);
  hoc_free(&h);
}

int orc_step_lm_hoc(const orc_model* m, const orc_lm_opts* o, const double* q_known, const double* tau,
                    double* q_out, orc_stats* stats, int n_threads) {
  if (o->order_K < 2 || o->order_K > ORC_KMAX) return -1;
  const int n = m->n_dofs > 0 ? m->n_dofs : 1, U = o->order_K - 1;
  int nt = n_threads > 0 ? n_threads : 1;
  double* scratch = (double*)malloc((size_t)nt * U * n * sizeof(double));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int i = 0; i < m->n_models; ++i) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* qunk = scratch + (size_t)tid * U * n;
    step_model_lm(m, i, o, q_known, q_known + m->n_dofs, tau, qunk, q_out, stats + i);
  }
  free(scratch);
  return 0;
}

int orc_step_hoc(const orc_model* m, const orc_opts* o, const double* q_known, const double* tau,
                 double* q_out, orc_stats* stats, int n_threads) {
  if (o->order_K < 3 || o->order_K > ORC_KMAX) return -1;
  const int n = m->n_dofs > 0 ? m->n_dofs : 1, U = o->order_K - 1;
  int nt = n_threads > 0 ? n_threads : 1;
  double* scratch = (double*)malloc((size_t)nt * U * n * sizeof(double));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int i = 0; i < m->n_models; ++i) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    double* qunk = scratch + (size_t)tid * U * n;
    step_model_hoc(m, i, o, q_known, q_known + m->n_dofs, tau, qunk, q_out, stats + i);
  }
  free(scratch);
  return 0;
}
