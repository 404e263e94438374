// ipc_world.h -- device-side data layout shared by the host driver and kernels.
//
// All scenes on a device live in one "world": every per-vertex, per-tet and
// per-surface-primitive array is one flat device allocation, and each scene
// (environment) owns a contiguous range in each of them.  Vertex ranges are
// aligned to 64 so that a 64-row slice of the sliced-ELL Hessian never mixes
// environments.  Kernels walk per-environment tiles, so every reduction is
// taken in an order relative to the environment's own start: an environment
// produces the same bits alone or in any batch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipcw {

constexpr int kTile = 256;     // elements per work tile (one 256-thread block)
constexpr int kSlice = 64;     // rows per sliced-ELL slice (one wavefront)
constexpr int kFusedRows = 8192;  // environments up to this many rows solve in one workgroup
// Two-level PCG: the rigid motions (3 translations, 3 rotations) of up to
// kCoarseBodies bodies per environment span the coarse space
constexpr int kCoarseBodies = 4;
constexpr int kCoarseM = 6 * kCoarseBodies;

enum Status { ST_IDLE = 0, ST_ACTIVE = 1, ST_CONVERGED = 2, ST_FAILED = 3 };
// Phase of an environment in one round of the decoupled schedule: PH_ITER
// (iterating, or not in the round), PH_BEGIN (starts a time step: targets,
// predicted positions, lagged friction, Dirichlet move), PH_RELAG (takes its
// friction data again at its converged iterate), PH_FINISH (ends its step),
// PH_FINISH_BEGIN (ends its step and starts the next).
enum Phase { PH_ITER = 0, PH_BEGIN = 1, PH_RELAG = 2, PH_FINISH = 3, PH_FINISH_BEGIN = 4 };
enum Fail { FAIL_NONE = 0, FAIL_MAXIT = 1, FAIL_NONFINITE = 2, FAIL_LS = 3, FAIL_DBC = 4 };

// vertex kind codes in kin[]: >= 0 kinematic group, -1 free, -2 padding row
constexpr int KIN_FREE = -1;
constexpr int KIN_PAD = -2;

struct Tile {
  int env;    // environment slot
  int start;  // first global element index
  int count;  // elements in this tile (<= kTile)
  int rel;    // tile index relative to the environment's first tile
};

// Static description of one environment (device copy, indexed by slot).
struct EnvDev {
  int v_off, nv, nv_pad;
  int t_off, nt;
  int tri_off, ntri;
  int e_off, ne;
  int sv_off, nsv;
  int pos_off, npos;
  int mo_off, n_groups, n_motion;
  int step;
  int maxit, precision;
  int vtile_first, vtile_count;  // this env's tiles in the batch vertex-tile list
  int item_off;                  // first broad-phase query item (surface verts, then edges) in the batch
  int bitem_off;                 // first broad-phase grid item (surface tris, then edges) in the batch
  int fused;                     // 1: the PCG solve runs in one workgroup (nv_pad <= kFusedRows)
  double dt, dhat, kappa, mu, eps_v, tol, pcg_tol;
  double cell;                   // hash-grid cell size of this environment
  double mbar;                   // mean free-vertex mass (augmented-Lagrangian weight mbar / dt^2)
  // solver variants
  int fric_iters;                // lagged friction updates per step (>= 1)
  int inv_filter;                // 1: the inversion filter bounds the line search
  int adapt_kappa;               // 1: kappa adapts to the least active-pair distance
  int nnzb;                      // stored 3x3 blocks of the elastic pattern (measurement)
  // coarse space of the PCG: bodies (connected sets of free vertices), each
  // with a reference point and a length that scales its rotation columns
  int nbody;
  double cb[kCoarseBodies][3];
  double cscale[kCoarseBodies];
};

// Per-environment solver state (device arrays indexed by slot).
struct EnvState {
  int *status, *reason, *iters, *halvings, *ls_done, *ls_cnt, *pcg_done, *pcg_it, *dbc_bad;
  long long *pcg_total;
  double *alpha, *E0, *E1, *pinf;
  unsigned long long *amax_bits;  // CCD bound as ordered bits of a non-negative double
  int *cand_beg, *cand_end, *act_beg, *act_end, *fric_beg, *fric_end, *big_beg, *big_end;
  int *in_step;                   // 1 if the env takes part in the current step
  // augmented-Lagrangian Dirichlet mode: al = 1 while the kinematic vertices
  // are unknowns; al_action per Newton iteration: 0 line search, 1 multiplier
  // update, 2 snap attempt, 3 snap accepted
  int *al, *al_action, *snap_bad;
  double *kA, *viol, *viol_prev;
  double *pcg_bb;                 // |g|^2 of the current solve
  // barrier stiffness (adapted per iterate with adapt_kappa), its given value,
  // and the least active-pair distance at the previous Newton iterate
  double *kappa, *kappa0, *dmin_prev;
  // active pairs and least squared distance among them at the last
  // classified iterate; friction lag rounds done this step; the Newton
  // iteration count at which the current round fails
  int *nact, *lag, *iter_cap;
  double *dmin2;
  // what the environment does in the current round of work (PH_*)
  int *phase;
  // PCG step length and r.u of the last two iterations (slot = iteration & 1)
  double *cg_a0, *cg_a1, *cg_g0, *cg_g1;
  // two-level PCG: E^-1 of the coarse matrix Z^T H Z [kCoarseM^2 per env],
  // the current coarse correction c = E^-1 Z^T r [kCoarseM per env], its
  // contribution (Z^T r).c to r.u, and whether the factorisation succeeded
  double *cinv, *cc, *cgam;
  int *cok;
};

// Flat device arrays of the world (element-indexed).
struct WorldDev {
  // per vertex
  double *X, *x, *v, *xn, *xh, *p, *g, *r, *z, *pp, *w, *q, *mass, *Minv, *e_v, *lam;
  float *r32, *z32, *pp32, *w32, *q32, *p32, *Minv32;
  int *kin, *venv, *vt_beg, *vt_end, *row_nnz;
  int *vbody;  // coarse body of a free vertex within its environment, -1 for others
  // (H Z)_i of the two-level PCG, 3 x kCoarseM per vertex, FP64 and FP32
  // copies, sliced like the ELL values: entry (r, k) of row i at
  // ((i / kSlice) 3 kCoarseM + r kCoarseM + k) kSlice + i % kSlice
  double *hz;
  float *hz32;
  // per slice (vertex / 64)
  int *slice_pos, *slice_w;
  // per sliced-ELL position
  int *col, *cb_beg, *cb_end;
  double *val;   // [pos/64][9][64]
  float *val32;  // same layout
  // contributor entries and vertex->tet incidence
  int *contrib, *vt_ent;
  // per tet
  int4 *tet;
  double *Dinv, *vol, *mu, *la, *tg, *tH, *e_t;
  int *tenv;
  // surface primitives
  int4 *tri;    // x,y,z vertex ids (ascending), w = env
  int4 *edge;   // x,y vertex ids (ascending), z = env
  double *elen2;
  int *sv;      // vertex id
  int *sv_env;
  double *box_sv, *box_tri, *box_edge;  // [6] lo.xyz hi.xyz
  // motion / gravity (per env ranges)
  double *motion;
};

}  // namespace ipcw
