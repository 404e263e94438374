/*
 * ipc_oracle.h -- C interface of the CPU oracle (test infrastructure only).
 *
 * The oracle is a plain, single-threaded FP64 implementation of one implicit
 * time step of Incremental Potential Contact as used by the paper's grasp
 * simulator (Sec. III-A, solver constants of Sec. III-D): projected Newton on
 * inertia + Neo-Hookean elasticity + log-barrier contact + lagged friction,
 * with a CCD-bounded backtracking line search.  It exists to check the GPU
 * library; nothing outside tests/, the smoke check and the benchmark's CPU
 * baseline may call it.  It shares no source with the GPU library.
 */
#ifndef IPC_ORACLE_H
#define IPC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_verts;
  const double *rest_pos;   /* [n_verts*3] */
  const double *init_pos;   /* [n_verts*3] or NULL (= rest_pos) */
  const double *init_vel;   /* [n_verts*3] or NULL (= 0) */
  int32_t n_tets;
  const int32_t *tets;      /* [n_tets*4] */
  const double *E, *nu, *rho; /* [n_tets] */
  int32_t n_tris;
  const int32_t *tris;      /* [n_tris*3] kinematic-only surface triangles */
  const int32_t *kin_group; /* [n_verts], -1 free */
  int32_t n_groups, n_motion_steps;
  const double *motion;     /* [n_motion_steps][n_groups][12] */
  const double *gravity;    /* [n_motion_steps][3] */
  double dt, dhat, kappa, mu, eps_v, newton_tol;
  int32_t newton_max_iter;
  double pcg_rel_tol;       /* relative residual for the linear solve */
  int32_t linear_solver;    /* 0 = block-Jacobi PCG, 1 = dense Cholesky */
  /* solver variants (0 = off; see the step-by-step description in ipc_oracle.cpp) */
  double newton_rel_tol;    /* > 0: stop at |p|_inf <= newton_rel_tol * L * dt, L = bbox diagonal
                               of the free vertices at creation (replaces newton_tol)          */
  int32_t friction_iters;   /* lagged friction updates per step (0 or 1: one, at x^n)        */
  int32_t inversion_filter; /* 1: the line search starts at most at 0.8 x the first root of
                               det F(alpha) = 0 over all tets                                 */
  int32_t adaptive_kappa;   /* 1: kappa doubles (up to 100 kappa) when the least active-pair
                               distance falls below 1e-2 dhat and keeps decreasing            */
} ipco_desc;

typedef struct {
  int32_t steps_done;
  int32_t status;
  int32_t fail_reason;      /* 0 none, 1 max iterations, 2 non-finite, 3 line-search stall, 4 DBC */
  int32_t newton_iters;
  int32_t max_newton_iters;
  int32_t ls_halvings;
  int64_t pcg_iters;
  int64_t n_active_last;
  double min_dist_last;
  double energy_last;
  double kappa_last;        /* barrier stiffness after the last step */
} ipco_info;

int ipco_create(const ipco_desc *d, void **out);
void ipco_destroy(void *s);
const char *ipco_last_error(void);
int ipco_step(void *s, int32_t n_steps, ipco_info *info);
int ipco_get_state(void *s, double *pos, double *vel, double *cauchy, double *von_mises);
int ipco_set_state(void *s, const double *pos, const double *vel, int32_t step);
int ipco_get_step(void *s);

/* scene-level checks */
int ipco_surface_sizes(void *s, int32_t out[3]);
int ipco_surface(void *s, int32_t *tris, int32_t *edges, int32_t *verts);
int ipco_mass(void *s, double *mass);
int64_t ipco_candidates(void *s, const double *x, const double *p, int32_t *out, int64_t cap);
int64_t ipco_active(void *s, const double *x, int32_t *out, double *d2, int64_t cap);
int ipco_begin_step(void *s, double *x_start);
double ipco_energy(void *s, const double *x);
int ipco_gradient(void *s, const double *x, double *g, double *gabs);
int ipco_hessian_dense(void *s, const double *x, double *H);
int ipco_newton_dir(void *s, const double *x, double *p, int64_t *pcg_iters);
double ipco_ccd_bound(void *s, const double *x, const double *p);
int64_t ipco_friction_pairs(void *s, int32_t *verts, double *lambda_, double *normal, double *w, int64_t cap);

/* element-level routines */
int ipco_pt_classify(const double *x12, double *d2);
int ipco_ee_classify(const double *x12, double *d2);
int ipco_barrier_scalar(double d, double dhat, double *out3);
int ipco_pair_barrier(int kind, int type, const double *x12, double dhat, double kappa,
                      double eps_x, int project, double *energy, double *g12, double *H144);
int ipco_tet_elastic(const double *X12, const double *x12, double E, double nu, int project,
                     double *energy, double *g12, double *H144);
int ipco_psd_project(int n, double *A);
double ipco_accd(int kind, const double *x12, const double *p12, double s);
int ipco_friction_f0(double y, double eps, double *out3);
/* One lagged friction element (energy mu*lambda*f0(|u|), gradient, Hessian). */
int ipco_friction_elem(const double *x12, const double *xn12, const double *w4, const double *n3, double lambda,
                       double mu, double eps, double *energy, double *g12, double *H144);
/* Newton record of the last step: rows (Phi before, Phi accepted, alpha, halvings). */
int64_t ipco_iter_log(void *s, double *out, int64_t cap);
/* Inversion filter of one tet: the first t in (0, tmax] with det(Ds(x + t p)) <= 0, or +inf
 * (x12, p12: the four vertices and their displacements).  Also the cubic's coefficients k[4]. */
double ipco_tet_first_root(const double *x12, const double *p12, double tmax, double *k4);
/* Step bound of the inversion filter over a scene's tets at x along p. */
double ipco_inversion_bound(void *s, const double *x, const double *p);
/* Current barrier stiffness of a scene. */
double ipco_kappa(void *s);
/* Grasp-validation controls (Sec. III-D).  Contact force between tagged bodies at x:
 * out[(a*ntags + b)*3 + k] = force on the vertices tagged a exerted by those tagged b. */
int ipco_contact_forces(void *s, const double *x, const int32_t *tags, int32_t ntags, double *out);
/* Hold kinematic group `group` at motion row `row` from the next step on (-1 releases it). */
int ipco_hold_group(void *s, int32_t group, int32_t row);
/* Gravity override for the following steps (NULL: back to the schedule). */
int ipco_set_gravity(void *s, const double *g);
/* Test-only planted fault: delta added to every line-search trial energy. */
int ipco_debug_ls_offset(void *s, double delta);

#ifdef __cplusplus
}
#endif
#endif
