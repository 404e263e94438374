/*
 * ipc.h -- C-ABI of the MI355X (gfx950) incremental-potential contact solver.
 *
 * What the library computes: the implicit time step of the paper's IPC grasp
 * simulator (GRIP, Sec. III-A "IPC Simulator with Parallel Environment"):
 * for every environment, x^{n+1} = argmin of the incremental potential
 *
 *   Phi(x) = sum_i m_i |x_i - xhat_i|^2 / (2 dt^2)         inertia, xhat = x^n + dt v^n + dt^2 g
 *          + sum_e V_e Psi_NH(F_e)                         Neo-Hookean tetrahedra
 *          + kappa sum_k e_k b(d_k),  b(d) = -(d-dhat)^2 ln(d/dhat)  point-triangle / edge-edge barrier
 *          + sum_k mu lambda_k f0(|u_k|)                   lagged smoothed friction (eps_v dt)
 *
 * solved by projected Newton with an additive-CCD step bound and a
 * backtracking line search ("barrier augmentation, CCD and projected Newton
 * with a step-size filter", Sec. II-C).  Environments are isolated: no
 * contact pairs across environments, each has its own CCD step size and line
 * search, its own stopping test, and a failure (no convergence within
 * newton_max_iter = 100, Sec. III-D) freezes only that environment
 * (problems (i)-(iv) of Sec. III-A).  Solver constants default to those of
 * Sec. III-D: dt = 0.01 s, kappa = 3e6 kg/s^2, dhat = 1e-3 m, eps_v = 1e-3 m/s,
 * FP64.
 *
 * Conventions
 *   - All floating-point data are FP64, SI units.  Positions and velocities
 *     are row-major [n][3]; indices are int32.
 *   - Pointers passed in are host pointers unless stated; the library copies
 *     every input at create time and never keeps a caller pointer.  Output
 *     buffers are owned by the caller.
 *   - Return value: 0 on success, a negative IPC_E_* code on error; the
 *     message of the last error on the calling thread is ipc_last_error().
 *   - One scene handle must not be used from two threads at once; distinct
 *     handles may.  All scenes live on the current HIP device at creation.
 */
#ifndef IPC_MI355X_H
#define IPC_MI355X_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPC_OK 0
#define IPC_E_ARG (-1)          /* bad sizes, indices, NaN/Inf, dt <= 0, dhat <= 0, ...          */
#define IPC_E_INVERTED (-2)     /* a tet has det(Dm) <= 0 at rest or J <= 0 initially            */
#define IPC_E_INTERSECTING (-3) /* initial configuration intersects (IPC precondition, Sec. III-C) */
#define IPC_E_NOMEM (-4)        /* device allocation failed / memory budget exceeded             */
#define IPC_E_FAILED (-5)       /* environment failed (Sec. III-A, III-D); scene is frozen       */
#define IPC_E_DEVICE (-6)       /* HIP runtime error                                             */

/* fail_reason values reported in ipc_step_info */
#define IPC_FAIL_NONE 0
#define IPC_FAIL_MAXIT 1     /* Newton did not converge in newton_max_iter iterations (Sec. III-D) */
#define IPC_FAIL_NONFINITE 2 /* non-finite gradient or search direction                          */
#define IPC_FAIL_LS 3        /* more than 40 line-search halvings                                 */
#define IPC_FAIL_DBC 4       /* prescribed kinematic move is not CCD-safe / inverts a tet         */

#define IPC_FP64 0  /* every step in FP64 */
#define IPC_MIXED 1 /* PCG matrix, preconditioner and vectors in FP32, dot products in FP64 */

typedef struct ipc_scene_s *ipc_scene;

typedef struct {
  int32_t n_verts;
  const double *rest_pos;   /* [n_verts*3] rest positions                                   */
  const double *init_pos;   /* [n_verts*3] or NULL (= rest_pos)                             */
  const double *init_vel;   /* [n_verts*3] or NULL (= 0)                                    */
  int32_t n_tets;
  const int32_t *tets;      /* [n_tets*4], positively oriented: det[X1-X0,X2-X0,X3-X0] > 0  */
  const double *E, *nu, *rho; /* [n_tets] Young's modulus (Pa), Poisson ratio, density      */
  int32_t n_tris;
  const int32_t *tris;      /* [n_tris*3] kinematic-only surfaces (ground, rigid links)     */
  const int32_t *kin_group; /* [n_verts] -1 = free vertex, g >= 0 = driven by group g        */
  int32_t n_groups, n_motion_steps;
  const double *motion;     /* [n_motion_steps][n_groups][12] row-major 3x4 [R|t]: the target
                               of a group-g vertex at step n is R X + t, X = its rest position;
                               step n uses row min(n, n_motion_steps-1)                      */
  const double *gravity;    /* [n_motion_steps][3]; the step n -> n+1 uses row min(n, last)   */
  double dt, dhat, kappa, mu, eps_v; /* 0.01, 1e-3, 3e6, friction coefficient, 1e-3          */
  double newton_tol;        /* converged when |p|_inf <= newton_tol * dt (p = Newton step)   */
  int32_t newton_max_iter;  /* 100 (Sec. III-D)                                             */
  double pcg_rel_tol;       /* PCG stops at |r|_2 <= pcg_rel_tol |g|_2 (1e-4 default, 1e-8 for parity) */
  int32_t precision;        /* IPC_FP64 or IPC_MIXED                                        */
  /* Solver variants (0 = off).  Each follows a passage of the paper that
   * leaves the exact rule open; the rule taken is stated here. */
  double newton_rel_tol;    /* > 0: the paper's relative Newton tolerance eps_r (Sec. III-D, 1e-3):
                               converged when |p|_inf <= eps_r * L * dt, L = diagonal of the
                               bounding box of the free vertices at creation; replaces newton_tol */
  int32_t friction_iters;   /* lagged friction updates per time step (0 or 1: one, at x^n; the
                               paper leaves the count open, Sec. III-D).  With k > 1, once an
                               environment's Newton solve converges its friction data are taken
                               again at the converged iterate (the tangential displacement is still
                               measured from x^n) and the solve is repeated, k solves in all, each
                               with its own newton_max_iter budget                           */
  int32_t inversion_filter; /* 1: step-size filter against inversion (Sec. II-C): the line search
                               starts at most at 0.8 t*, t* the first root in (0, 1.25] of
                               det(Ds(x + t p)) over every tet (a cubic in t), besides the CCD bound */
  int32_t adaptive_kappa;   /* 1: at each Newton iterate, if the least active-pair distance is below
                               1e-2 dhat and smaller than at the previous iterate, kappa doubles, up
                               to 100 times its given value (the paper fixes kappa = 3e6, Sec.
                               III-D; this is the variant that adapts it)                     */
} ipc_scene_desc;

typedef struct {
  int32_t steps_done;       /* time steps completed by this call                             */
  int32_t status;           /* IPC_OK or IPC_E_FAILED                                        */
  int32_t fail_reason;      /* IPC_FAIL_*                                                    */
  int32_t newton_iters;     /* total Newton iterations (search directions computed)          */
  int32_t max_newton_iters; /* largest per-step count                                        */
  int32_t ls_halvings;      /* total line-search halvings                                    */
  int64_t pcg_iters;        /* total PCG iterations                                          */
  int64_t n_active_last;    /* active contact pairs (d^2 < dhat^2) at the last accepted iterate */
  double min_dist_last;     /* least distance among those pairs (+inf if none): the contact
                               gap of Table I's D2, zero penetration when > 0               */
  double energy_last;       /* Phi at the last accepted iterate                              */
  double kappa_last;        /* barrier stiffness after the last step (kappa unless adaptive)  */
} ipc_step_info;

/* Create a scene from host data (copied).  Validates sizes, finiteness,
 * orientation (IPC_E_INVERTED) and that the initial configuration is free of
 * intersections (IPC_E_INTERSECTING): the IPC precondition of Sec. III-C.
 * Allocates device memory on the current device (IPC_E_NOMEM on failure). */
int ipc_create_scene(const ipc_scene_desc *desc, ipc_scene *out);

/* Advance one scene by n_steps time steps (Sec. III-A).  info may be NULL.
 * Returns IPC_E_FAILED if the scene fails; it is then frozen at its last
 * accepted step and later calls return IPC_E_FAILED without changing it. */
int ipc_step(ipc_scene s, int32_t n_steps, ipc_step_info *info);

/* Advance n scenes together: every kernel covers all of them, while each
 * keeps its own CCD bound, line search, stopping test and failure state
 * (Sec. III-A).  infos may be NULL or point to n records.  Returns IPC_OK if
 * every scene completed all steps, else IPC_E_FAILED (see infos). */
int ipc_step_batch(ipc_scene *scenes, int32_t n, int32_t n_steps, ipc_step_info *infos);

/* Copy the current state to host buffers: pos [n_verts*3]; vel [n_verts*3]
 * or NULL; cauchy [n_tets*6] (xx,yy,zz,yz,xz,xy) or NULL; von_mises
 * [n_tets] or NULL (per-tet stress output, Sec. IV-D). */
int ipc_get_state(ipc_scene s, double *pos, double *vel, double *cauchy, double *von_mises);

/* Utility, not a step of the method: overwrite positions/velocities (vel
 * NULL = 0) and the step index, and clear a failed flag, for checkpoint /
 * resume.  The caller vouches for the state: it is not checked for
 * intersection or inversion here (the next step's line search would reject
 * an infeasible iterate).  The barrier stiffness and augmented-Lagrangian
 * state are kept.  IPC_E_ARG for a NULL pos, a negative step or non-finite
 * values. */
int ipc_set_state(ipc_scene s, const double *pos, const double *vel, int32_t step);

void ipc_destroy_scene(ipc_scene s);
const char *ipc_last_error(void);

/* Sizes of a scene: out[0] verts, out[1] tets, out[2] surface triangles,
 * out[3] surface edges, out[4] surface vertices, out[5] current step index,
 * out[6] failed flag. */
int ipc_scene_sizes(ipc_scene s, int64_t out[7]);

/* Measurement on the current device (sums over its lanes).  When enabled,
 * every 16th PCG iteration of each solve (iterations 5, 21, 37, ...) has its
 * matrix-vector product and its update each timed from kernel start to
 * kernel end by HIP events carried in their dispatches (hipExtLaunchKernel),
 * and a separate launch between the two kernels (outside both timings) adds
 * the iteration's algorithmic bytes to device counters:
 * for the product the stored 3x3 blocks and column indices (sliced ELL and
 * merged contact blocks) plus one read of u and one write of w per row; for
 * the whole iteration the same blocks plus per row the preconditioner block
 * and eight vector accesses of three values (N (9 s + 4) + n 9 s + 24 n s);
 * with the two-level PCG (m = 6 x bodies) the product adds per row its 3 m
 * entries of H Z, its body index and, in a body, its position (3 m s + 4 +
 * 24), and the iteration adds the update's body index and position reads and
 * its m partials per tile.
 * Every assembly pass (elasticity, inertia, gradient and stored blocks) is
 * timed too, from the start of its first kernel to the end of its last, its
 * algorithmic bytes (per tet 208 B of inputs, per row
 * 80 B, 9 s per stored block) counted the same way.  ipc_prof_read writes
 * out[12]: out[0] product milliseconds, out[1] timed iterations, out[2] their
 * product bytes; out[3..5] the same three for the timed products over more
 * than 64 tiles; out[6] milliseconds of product + update of the timed
 * iterations, out[7] their count, out[8] their whole-iteration bytes;
 * out[9] assembly milliseconds, out[10] assembly passes, out[11] their bytes.
 * ipc_prof_enable(2) instead counts the bytes of every iteration and times
 * none (out[0] stays 0, out[1] counts every iteration): the algorithmic
 * bytes of the same launches that a hardware counter run over the whole
 * program sees.  ipc_prof_enable(0) turns measurement off. */
int ipc_prof_enable(int32_t on);
int ipc_prof_reset(void);
int ipc_prof_read(double *out);
/* Contact work since the last reset while measurement is enabled (sums over
 * the device's lanes), counted per assembly pass of a Newton iteration
 * (Sec. II-C: the barrier and friction terms of the incremental potential):
 * out[0] candidate pairs classified (closest-point type and distance),
 * out[1] active barrier pair elements evaluated (energy gradient and
 * PSD-projected Hessian), out[2] lagged friction elements evaluated.
 * Line-search energy passes are not counted. */
int ipc_prof_pairs(double *out);

/* Execution knobs of the current device's solver.  They change how work is
 * scheduled, never a result: the tiled PCG kernels and the per-environment
 * PCG kernel reduce in the same order and produce the same bits.
 *   IPC_TUNE_TAIL_TILES: once at most this many vertex tiles (256 rows each)
 *     of a batch are still iterating their PCG, the remaining environments
 *     are finished by one workgroup each in a single launch (default 0 =
 *     never: one CU's bandwidth makes that slower than the tiled launches on
 *     environments of a few thousand rows; initial value from the environment
 *     variable IPC_TAIL_TILES).
 *   IPC_TUNE_FUSED_PCG: 1 = every environment of up to 8192 rows runs its
 *     whole PCG in one workgroup from the start (default 0; IPC_FUSED_PCG).
 *   IPC_TUNE_NARROW: 1 = once at most half of a batch still iterates its
 *     Newton loop, the batch is laid out again with those environments only
 *     (default), 0 = never (IPC_NARROW).
 *   IPC_TUNE_LANES: number of lanes per device (1..16; default: the
 *     process's hardware queues minus the one the runtime's null stream
 *     holds, at most 4 -- GPU_MAX_HW_QUEUES, 4 unless set, gives 3; IPC_LANES).
 *     A lane is an independent set of device buffers with its own stream;
 *     ipc_create_scene places a scene in the lane with the fewest tets, and
 *     ipc_step_batch steps the scenes of each lane together, the lanes
 *     concurrently from one host thread each, so that one lane's
 *     latency-bound tail overlaps with the others' work.  Applies to scenes
 *     created afterwards.
 * Returns IPC_OK, or IPC_E_ARG for an unknown key or a negative value (other
 * than -1 for IPC_TUNE_WIDE_TILES). */
/* Further execution settings, read from the environment when a device's
 * first lane is created (none changes a result):
 *   IPC_BP_STASH    broad phase: pairs per query kept by the counting pass
 *                   (default 64); queries with more are traversed again
 *   IPC_BP_COOP     1 (default): the counting pass walks each query's cells
 *                   with a group of 8 lanes; 0: one lane per query
 *   IPC_PIPELINE    1 (default): the next block of PCG iterations is queued
 *                   before the host polls the previous one
 *   IPC_POLL_BLOCK  PCG iterations per poll (default 8 mixed, 4 FP64)
 *   IPC_NARROW_PCT  the batch is laid out again once at most this percentage
 *                   of it still iterates its Newton loop (default 50)
 *   IPC_WIDE_TILES  PCG product launches over at most this many tiles issue
 *                   four slots per lane and round (default: every launch in
 *                   FP64, none in the mixed path) */
#define IPC_TUNE_TAIL_TILES 1
#define IPC_TUNE_FUSED_PCG 2
#define IPC_TUNE_NARROW 4
#define IPC_TUNE_LANES 5
/* Test hook, not an execution knob: the next `value` scene placements on
 * each lane of the current device fail as if the device were out of memory
 * (ipc_create_scene returns IPC_E_NOMEM; a server retires the request with
 * IPC_FAIL_ADMIT and goes on).  Lets the failure path be tested without
 * exhausting the GPU. */
#define IPC_TUNE_ADMIT_FAULTS 6
/* IPC_TUNE_ASYNC: 1 (default; IPC_ASYNC) = decoupled schedule: within a
 * lane, an environment that finishes a time step begins its next one while
 * the others are still iterating theirs, each round being one Newton
 * iteration of every environment with work; 0 = lock-step time steps (every
 * environment of the batch finishes step n before any begins step n+1).  The
 * same results bit for bit (every environment runs the same sequence). */
#define IPC_TUNE_ASYNC 7
/* IPC_TUNE_WIDE_TILES: PCG product launches over at most this many tiles
 * issue each lane's slots four at a time (0 = none; -1 = the default: every
 * FP64 launch and no mixed one; initial value from IPC_WIDE_TILES, else -1).
 * IPC_TUNE_POLL_BLOCK: PCG iterations queued per host poll, 1..1024, or -1 =
 * the default: 8 in mixed precision, 4 in FP64 (initial value IPC_POLL_BLOCK,
 * else -1).  Neither changes a result. */
#define IPC_TUNE_WIDE_TILES 8
#define IPC_TUNE_POLL_BLOCK 9
/* IPC_TUNE_COARSE: 1 (default; IPC_COARSE) = two-level PCG: block Jacobi plus
 * an exact solve on the rigid motions (3 translations, 3 rotations) of each
 * body of an environment (its connected sets of free vertices, the 4 largest
 * with at least 4 vertices; while one of the 4 slots is left, the largest set,
 * if it has at least 64 vertices, in two halves along its longest axis);
 * 0 = block Jacobi alone.  Unlike the other knobs
 * it changes the PCG's iterates, within its stopping tolerance; results stay
 * the same alone and in any batch.  While it is on, IPC_TUNE_FUSED_PCG and
 * IPC_TUNE_TAIL_TILES have no effect (those kernels are block Jacobi only).
 * Applies from the next step. */
#define IPC_TUNE_COARSE 10
int ipc_set_tuning(int32_t key, int64_t value);
int ipc_get_tuning(int32_t key, int64_t *value);

/* Per-workload tuning of IPC_TUNE_WIDE_TILES and IPC_TUNE_POLL_BLOCK on the
 * current device.  With cache_path (nullable) naming a text file that holds
 * a line for this workload (key: scene count, total tets to three significant
 * digits, precisions, lane count), its values are applied and out[2] = 1.
 * Otherwise the current setting and each of the candidates {0, 64, all
 * tiles} x {4, 8, 16} are timed (twice each, the faster run counting) over
 * `steps` (1..64) time steps of copies of the n scenes set to their current
 * state (the copies take device memory alongside the scenes while the call
 * runs; the scenes themselves are not stepped); the fastest candidate
 * replaces the current setting only if it is at least 3% faster; the result
 * is applied, out[2] = 0, and a line "key<TAB>wide poll ms_per_step" is
 * appended to the file.  out[0], out[1] = the values applied.  The knobs change no result,
 * so results stay bitwise those of any other setting.  IPC_E_ARG for bad
 * arguments or an unwritable cache file; a device error as any stepping call. */
int ipc_autotune(const ipc_scene *scenes, int32_t n, int32_t steps, const char *cache_path, int64_t out[3]);

/* CCD step bound over a caller's list of contact pairs (Sec. II-C: the
 * projected-Newton step is filtered by continuous collision detection; the
 * bound is the additive-CCD time of impact, mean displacement removed,
 * conservative rescaling s).  n pairs of one kind (0 point-triangle: point,
 * then the triangle's three vertices; 1 edge-edge: the two vertices of each
 * edge), positions x12 [n*12] and displacements p12 [n*12], host pointers.
 * *alpha = min(1, min over the pairs of the time of impact), 1 for n = 0.
 * IPC_E_ARG for a bad kind, n < 0, NULL pointers, non-finite data or s
 * outside (0, 1).  Uses a per-call device buffer of per-block minima. */
int ipc_ccd_bound_pairs(int32_t kind, int64_t n, const double *x12, const double *p12, double s, double *alpha);

/* The same bound for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * it calls no allocating routine.  x12, p12 [n*12] and alpha [1] are DEVICE
 * pointers on the current device; the two kernels are queued on `stream`
 * (a hipStream_t, NULL = the null stream) and the call returns without
 * waiting: *alpha holds the bound once the stream has reached it.  The
 * per-block minima live in a fixed device array of 65536 doubles (512 KiB)
 * that each GPU the library runs on holds until the process ends, so
 * n <= 8388608 (128 pairs per entry); larger n is rejected with IPC_E_ARG
 * before anything is queued.  Every call on one GPU shares that array and
 * overwrites the entries it uses (nothing needs to start at zero): calls
 * that overlap on one GPU (different streams, or threads) race; calls on
 * one stream are ordered.  Errors: IPC_E_ARG as above, IPC_E_DEVICE if the
 * launch fails; the message is in ipc_last_error(). */
int ipc_ccd_bound_pairs_noalloc(int32_t kind, int64_t n, const double *x12, const double *p12, double s,
                                double *alpha, void *stream);

/* Grasp-quality metrics of Sec. IV-C, Eq. (2)-(3), at the scene's current
 * positions.  The manipuland is given by its closed boundary triangle mesh
 * obj_tris [n_obj_tris*3] (scene vertex ids, outward oriented); its signed
 * distance field d_o(p) is the distance from p to the nearest of those
 * triangles, positive inside (generalised winding number above 1/2),
 * negative outside.  The sample set S_h on the gripper's surface is given as
 * n_samples points on the triangles hand_tris [n_hand_tris*3]: point k lies
 * on triangle sample_tri[k] at barycentric (u, v) = sample_uv[2k..2k+1],
 * p = (1-u-v) x0 + u x1 + v x2 (the paper samples 50,000 points; the caller
 * draws them).  D[0] = D1 = max(0, max_p d_o(p)) (penetration depth), D[1] =
 * D2 = |max_p d_o(p)| (gripper-manipuland gap, or the depth when they
 * interpenetrate).  sdf [n_samples] receives every d_o(p) (may be NULL).
 * IPC_E_ARG for indices out of range, u or v negative or u + v > 1, empty
 * sets.  Host pointers; per-call device buffers. */
int ipc_grasp_metrics(ipc_scene s, int32_t n_obj_tris, const int32_t *obj_tris, int32_t n_hand_tris,
                      const int32_t *hand_tris, int32_t n_samples, const int32_t *sample_tri, const double *sample_uv,
                      double *D, double *sdf);

/* ---------------------------------------------------------------------------
 * Grasp validation (Sec. III-D): gravity is off while the fingers close, a
 * finger's motion is halted once its contact force exceeds 50 N, then gravity
 * of 9.8 m/s^2 is applied along the six axis directions for 0.1 s each; the
 * grasp is stable if the manipuland is still in contact with the gripper at
 * the end and its centre of mass moves less than a threshold proportional to
 * eps_v dt.  The controls below act on the following time steps.
 * ------------------------------------------------------------------------- */

/* Holds kinematic group `group` at motion row `row`: from the next step on
 * its targets are those of row min(scheduled row, row); row = -1 releases it.
 * IPC_E_ARG for a bad group or row < -1. */
int ipc_hold_group(ipc_scene s, int32_t group, int32_t row);

/* Overrides the gravity schedule with g [3] (m/s^2) for the following steps;
 * g = NULL returns to the schedule. */
int ipc_set_gravity(ipc_scene s, const double *g);

/* Contact forces between tagged bodies at the scene's current positions:
 * tags [n_verts] gives each vertex a body tag in [0, ntags) (others: ignored),
 * out [ntags*ntags*3]: out[(a*ntags + b)*3 + k] is the force on the vertices
 * tagged a exerted by those tagged b through the barrier: every active pair
 * pushes its first side (the point, or the first edge) with lambda n and its
 * second side with -lambda n, lambda = -kappa e b'(d), n the unit normal of
 * the closest-point difference.  1 <= ntags <= 64. */
int ipc_contact_forces(ipc_scene s, const int32_t *tags, int32_t ntags, double *out);

#define IPC_MAX_FINGERS 8
typedef struct {
  const int32_t *vertex_tag;      /* [n_verts]: 0 the manipuland, f = 1..n_fingers finger f, -1 other */
  int32_t n_fingers;              /* 1..IPC_MAX_FINGERS                                             */
  const int32_t *finger_of_group; /* [n_groups]: the finger (1..n_fingers) a kinematic group drives,
                                     0 none (ground, ...)                                          */
  double force_limit;             /* 50 N: a finger halts once |force on it from the manipuland|
                                     exceeds this                                                  */
  int32_t max_close_steps;        /* closing steps at most (the motion schedule's rows drive them)   */
  int32_t settle_steps;           /* steps with gravity off after closing                           */
  int32_t phase_steps;            /* steps per gravity direction (0.1 s / dt = 10)                   */
  double gravity;                 /* 9.8 m/s^2                                                      */
  double com_factor;              /* threshold = com_factor * eps_v * dt on the centre-of-mass
                                     displacement in each phase's last step                         */
} ipc_grasp_protocol;

typedef struct {
  int32_t stable;                          /* in contact at the end and every phase below threshold */
  int32_t in_contact;                      /* a finger touches the manipuland at the final step     */
  int32_t failed, fail_reason;             /* the simulation failed (IPC_FAIL_*); stable = 0        */
  int32_t steps_run;
  int32_t halt_step[IPC_MAX_FINGERS];      /* step index at which finger f+1 halted, -1 never       */
  double finger_force[IPC_MAX_FINGERS];    /* its contact force then (N)                            */
  double com_shift[6];                     /* |COM displacement| over each gravity phase (m):
                                              +x, -x, +y, -y, +z, -z                               */
  double com_drift[6];                     /* |COM displacement| in each phase's last step (m)       */
} ipc_grasp_result;

/* Runs the protocol on a scene from its current state (the reading taken
 * where the paper is brief): gravity off; up to max_close_steps steps of the
 * motion schedule, after each the contact force of every finger from the
 * manipuland, a finger whose force exceeds force_limit holding its groups at
 * the row just reached; every finger still moving is then held where it is;
 * settle_steps steps; then for +x, -x, +y, -y, +z, -z in turn gravity of that
 * magnitude for phase_steps steps.  The scene is left at the final state with
 * its holds and the last gravity override in place (release with
 * ipc_hold_group(.., -1) / ipc_set_gravity(s, NULL)).  A simulation failure
 * ends the protocol with r->failed set and IPC_OK returned. */
int ipc_validate_grasp(ipc_scene s, const ipc_grasp_protocol *p, ipc_grasp_result *r);

/* ---------------------------------------------------------------------------
 * Inspection entry points.  Each runs the same device kernels the step uses,
 * on host-supplied positions, so callers can check individual stages.
 * Pair rows are (kind, v0, v1, v2, v3): kind 0 = point-triangle (v0 the
 * point, v1<v2<v3 the triangle), kind 1 = edge-edge (v0<v1 and v2<v3 the
 * edges, (v0,v1) < (v2,v3)).
 * ------------------------------------------------------------------------- */

/* Candidate pairs whose d-hat-widened boxes overlap at x (p == NULL) or over
 * the sweep x -> x+p.  Writes min(count, cap) rows to out [cap*5]; returns
 * the count or a negative error. */
int64_t ipc_debug_candidates(ipc_scene s, const double *x, const double *p, int32_t *out, int64_t cap);

/* Active pairs (d^2 < dhat^2) at x: rows (kind, v0..v3, type) into out
 * [cap*6], squared distances into d2 [cap] (may be NULL). */
int64_t ipc_debug_active(ipc_scene s, const double *x, int32_t *out, double *d2, int64_t cap);

/* Prepare the step n -> n+1 at the current state (kinematic targets,
 * predicted positions, lagged friction, Dirichlet move) without advancing;
 * the starting iterate is written to x_start [n_verts*3] (may be NULL). */
int ipc_debug_begin_step(ipc_scene s, double *x_start);

/* Gradient of Phi at x (kinematic rows 0) for the prepared step. */
int ipc_debug_gradient(ipc_scene s, const double *x, double *g);

/* Phi at x for the prepared step (+inf if infeasible). */
double ipc_debug_energy(ipc_scene s, const double *x);

/* y = H v with H the PSD-projected Hessian at x (kinematic rows: identity). */
int ipc_debug_hessian_apply(ipc_scene s, const double *x, const double *v, double *y);

/* Newton search direction at x (solves H p = -g with the world's PCG: the
 * two-level one unless IPC_TUNE_COARSE is 0, then block Jacobi alone). */
int ipc_debug_newton_dir(ipc_scene s, const double *x, double *p, int64_t *pcg_iters);

/* Coarse space of the two-level PCG as built at creation (a utility for tests;
 * no passage of the paper defines it): vbody[n_verts] receives each vertex's
 * body (0 .. nbody-1, a split largest set taking 0 and 1; -1 for kinematic
 * vertices and free vertices outside the bodies), frame[4 * nbody] each body's reference point and size (x, y, z, s:
 * the rest centroid of its vertices, summed in vertex order, and the largest
 * rest distance from it).  Either pointer may be null; frame must hold
 * 4 * IPC_COARSE_BODIES doubles.  Returns nbody (0 .. IPC_COARSE_BODIES) or
 * a negative error code. */
#define IPC_COARSE_BODIES 4
int ipc_debug_bodies(ipc_scene s, int32_t *vbody, double *frame);

/* CCD step bound min(1, additive-CCD time of impact) over the sweep x -> x+p. */
double ipc_debug_ccd_bound(ipc_scene s, const double *x, const double *p);

/* Inversion filter's step bound min(1, min over tets of 0.8 t*) along x + t p
 * (t* the first root of det(Ds(x + t p)), Sec. II-C step-size filter),
 * whether or not the scene enables the filter. */
double ipc_debug_inversion_bound(ipc_scene s, const double *x, const double *p);

/* Element routines evaluated by device code (one element per call). */
int ipc_debug_classify(int32_t kind, int64_t n, const double *x12, int32_t *types, double *d2);
int ipc_debug_pair_barrier(int32_t kind, int32_t type, const double *x12, double dhat, double kappa,
                           double eps_x, int32_t project, double *energy, double *g12, double *H144);
int ipc_debug_tet_elastic(const double *X12, const double *x12, double E, double nu, int32_t project,
                          double *energy, double *g12, double *H144);
int64_t ipc_debug_accd(int32_t kind, int64_t n, const double *x12, const double *p12, double s, double *t);
/* Per tet (x12, p12: its four vertices and their displacements): the
 * coefficients k4 [n*4] of det(Ds(x + t p)) = k0 + k1 t + k2 t^2 + k3 t^3 and
 * its first root t [n] in (0, tmax] (+inf if none, 0 if det <= 0 at t = 0). */
int64_t ipc_debug_tet_first_root(int64_t n, const double *x12, const double *p12, double tmax, double *t, double *k4);

/* ===========================================================================
 * Serving: continuous batching of simulation requests on one device.
 *
 * A server owns one worker thread per lane of the device (IPC_TUNE_LANES).
 * Each worker, tick after tick: (1) admits queued requests into its lane, in
 * submission order, while fewer than max_slots requests run in all, its lane
 * holds less than its share (max_slots / lanes, rounded up) and the request's
 * admission charge fits in budget_bytes; (2) advances the requests running in
 * its lane, all of them in one batch through the same kernels as
 * ipc_step_batch; (3) retires the requests that completed their steps or
 * failed, keeping their final state for ipc_server_result and freeing their
 * slot and memory.  Under the decoupled schedule (IPC_TUNE_ASYNC = 1, the
 * default) a tick is one round of it: every running request takes one Newton
 * iteration, or ends its step and begins the next, so requests join and leave
 * between Newton iterations; with IPC_TUNE_ASYNC = 0 a tick is one time step
 * of every running request.  Lanes run concurrently, and a request's result
 * is bitwise the same as when it runs alone.  The admission charge
 * (ipc_request_info.bytes) is the resident state (positions and velocities,
 * meshes, sparsity pattern, PCG vectors) plus half again for the arenas'
 * growth, plus an estimate of the request's share of the lane's per-step
 * contact and candidate lists, which scales with its surface; denser contact
 * than the estimate grows those lists beyond the charge.
 *
 * The paper (Sec. IV) runs its grasp pipeline as many independent
 * environments; this interface serves such environments as they arrive.
 * =========================================================================== */
typedef struct ipc_server_s *ipc_server;

#define IPC_REQ_QUEUED 0
#define IPC_REQ_RUNNING 1
#define IPC_REQ_DONE 2
#define IPC_REQ_FAILED 3

typedef struct {
  int32_t status;       /* IPC_REQ_*                                                       */
  int32_t steps_done;   /* converged time steps                                             */
  int32_t n_steps;      /* steps requested                                                  */
  int32_t fail_reason;  /* IPC_FAIL_* once FAILED (IPC_FAIL_DEVICE: the server stopped)     */
  double t_submit;      /* seconds since the server was created, at entry to submit        */
  double t_admit;       /* -1 while queued                                                 */
  double t_done;        /* -1 until DONE / FAILED; latency = t_done - t_submit             */
  int64_t newton_iters; /* summed over the request's steps                                  */
  int64_t pcg_iters;
  int64_t bytes;        /* resident device bytes of the request's scene                     */
} ipc_request_info;

#define IPC_FAIL_DEVICE 5 /* the server's worker hit a device error and stopped */
#define IPC_FAIL_ADMIT 6  /* the request could not be placed on the device (out of memory);
                             the server goes on with the others                          */

/* Creates a server on the current device.  budget_bytes > 0; max_slots >= 1
 * fixes the slot cap, max_slots = 0 lets the server tune it: starting at 8
 * per lane, while requests are waiting it doubles the cap after every window
 * of 8 ticks per lane (64 under the decoupled schedule), unless that window's seconds per converged step exceed
 * 1.5x the best window's, in which case it settles on the best window's cap. */
int ipc_server_create(int64_t budget_bytes, int32_t max_slots, ipc_server *out);
/* Validates and copies the scene (as ipc_create_scene; same error codes, and
 * IPC_E_NOMEM if it alone exceeds the budget) and queues it for n_steps >= 1
 * time steps; *id identifies the request. */
int ipc_server_submit(ipc_server srv, const ipc_scene_desc *desc, int32_t n_steps, int64_t *id);
/* Current record of a request (IPC_E_ARG for an unknown id). */
int ipc_server_poll(ipc_server srv, int64_t id, ipc_request_info *info);
/* Waits up to timeout_s seconds for the request to be DONE or FAILED, then
 * fills *info (nullable) as ipc_server_poll does. */
int ipc_server_wait(ipc_server srv, int64_t id, double timeout_s, ipc_request_info *info);
/* Positions [n_verts*3] and velocities (nullable) of a finished request: the
 * last converged step (IPC_E_ARG if it has not finished). */
int ipc_server_result(ipc_server srv, int64_t id, double *pos, double *vel);
/* Forgets a finished request and its stored result. */
int ipc_server_release(ipc_server srv, int64_t id);
/* Fixes the slot cap (takes effect at the next admission; ends tuning). */
int ipc_server_set_slots(ipc_server srv, int32_t max_slots);
/* Totals: out[0] requests finished, out[1] failed, out[2] converged steps,
 * out[3] ticks, out[4] running now, out[5] queued now, out[6] resident bytes
 * in use, out[7] seconds since creation, out[8] current slot cap. */
int ipc_server_stats(ipc_server srv, double *out);
/* Stops the worker after its current tick; unfinished requests are dropped. */
void ipc_server_destroy(ipc_server srv);

#ifdef __cplusplus
}
#endif
#endif
