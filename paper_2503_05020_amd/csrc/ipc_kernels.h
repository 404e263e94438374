// ipc_kernels.h -- launchers of the device kernels (host-callable).
#pragma once
#include <hip/hip_runtime.h>

#include "ipc_world.h"

namespace ipck {
using ipcw::EnvDev;
using ipcw::EnvState;
using ipcw::Tile;
using ipcw::WorldDev;

// Work lists of one batch (device pointers) and their sizes.
struct Batch {
  const Tile *vtiles, *ttiles, *svtiles, *tritiles, *etiles, *itiles, *btiles;
  int n_vt, n_tt, n_svt, n_trit, n_et, n_it, n_bt;
  int n_bitems;     // grid items (surface tris + edges of all envs)
  const int *envs;  // env slots in the batch
  int n_envs;
  int n_items;      // broad-phase work items (surface verts + edges of all envs)
};

// Dynamic per-iteration lists.
// one hash-grid entry: a surface primitive registered in one cell, with its
// box rounded outward to float for a quick rejection test
struct GridEnt {
  int code, cx, cy, cz;  // triangle id (>= 0) or ~edge id; cell coordinates
  float lo[3], hi[3];
  int env, pad;
};

// PCG product launches over more than this many tiles are measured as a
// class of their own (the rest are the latency-bound tails)
constexpr int kWideTiles = 64;

struct Lists {
  int *counts, *offs, *scan_tmp;  // item counts, exclusive scan (n_items+1)
  int2 *cand;                     // candidate pairs: PT (sv, tri) or EE (~ea, eb)
  int *cand_type, *cand_flag, *cand_offs;
  double *cand_d2, *e_c;
  int2 *act;                      // active pairs (same encoding)
  int *act_type;
  double *act_d2;                 // their squared distances
  // friction (lagged at x^n)
  int4 *fv;
  double *fw, *fn, *flam, *e_f;
  int *fenv;
  // contact elements (barrier then friction)
  int4 *ce_v;
  double *ce_g, *ce_H;
  // incidence
  int *inc_cnt, *inc_off, *inc_cur, *inc_ent;
  // contact blocks per row merged by column: from 4 * inc_off[i], cr_cnt[i] of them
  int *cr_col, *cr_cnt;
  int *cr_key, *cr_scol, *cr_ssrc;           // expanded pairs: columns, sorted columns, sorted sources
  int *cr_flag, *cr_pos, *cr_rows;           // rows with contact: flags, scan, list
  double *cr_val;
  float *cr_val32;
  // reduction partials per vertex tile (PCG: a = u.Hu, b0/b1 = r.u, c0/c1 = r.r)
  double *part_a, *part_b0, *part_b1, *part_c0, *part_c1;
  // two-level PCG: per tile, Z^T r [kCoarseM] and the tile's part of Z^T H Z [kCoarseM^2]
  double *part_z, *e_tile;
  int coarse;  // 1: the PCG uses the coarse correction
  int *counter;  // device scratch counters [16]
  int *bar_slow;  // barrier pairs that take the full 12x12 element (k_barrier_elems_full)
  // hash grid
  int *g_ncell, *g_big, *g_eoff, *g_bigoff, *g_ebucket, *g_bcnt, *g_boff, *g_bcur, *g_bigl;
  GridEnt *g_ent, *g_sorted;
  int2 *bp_stash;  // first pairs of each query, from the counting pass
  int stash_n;     // pairs per query the stash holds
  int bp_coop;     // 1: the counting pass walks each query's cells with a group of lanes
  int wide_tiles;  // PCG products over at most this many tiles use the latency variant
  unsigned long long *prof;  // algorithmic bytes moved by profiled kernels (nullptr = off)
};

void begin_step(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B);
void apply_dbc(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B);
void dbc_check_J(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B);
void env_begin(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B);
void env_dbc(hipStream_t s, const EnvState &S, const Batch &B);

// broad phase over the state positions x (+ p if swept)
void boxes(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, const double *x,
           const double *p);
void scan_int(hipStream_t s, const int *in, int *out, int n, int *tmp);  // out[n+1] exclusive
void grid_count(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L);
void grid_fill(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
               int n_ent, unsigned nbuckets);
void bp_grid_count(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
                   unsigned nbuckets);
void bp_grid_write(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
                   unsigned nbuckets, bool overflow);
void cand_segments(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L);

void classify_cands(hipStream_t s, const WorldDev &W, const EnvDev *E, const Lists &L, int n, const double *x);
void compact_active(hipStream_t s, const Lists &L, int n);
void act_segments(hipStream_t s, const EnvState &S, const Batch &B, const Lists &L);
// per environment: active-pair count, least squared distance; with adapt = 1
// (a Newton iterate) the adaptive barrier stiffness update
void act_stats(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L, int adapt);
void barrier_elems(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_act,
                   const double *x);
void friction_setup(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_act);
void friction_elems(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_fric,
                    int ce_off, const double *x);
void incidence(hipStream_t s, const WorldDev &W, const EnvState &S, Lists &L, int n_ce, int nv_world);
void incidence_fill(hipStream_t s, const WorldDev &W, const EnvState &S, Lists &L, int n_ce, int nv_world);

// merged contact blocks of every row (after incidence_fill)
void contact_rows(hipStream_t s, Lists &L, int nv_world, int n_inc, int mixed);
// start / stop (nullable): events recorded by the dispatches themselves at the
// start of k_elastic and the end of k_assemble_sell (the assembly pass timing)
void elastic(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B,
             hipEvent_t start = nullptr);
void assemble(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L,
              int mixed, hipEvent_t stop = nullptr);

// the coarse matrix E = Z^T H Z of the two-level PCG and E^-1, per environment
// of the batch, at the assembled H
void coarse_setup(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B,
                  const Lists &L, int mixed);
void pcg_init(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
              int *pending, int mixed);
// one tiled PCG iteration (product with its dot product, then the update with
// the stopping test) over the listed tiles; `it` = iterations done so far
// ev (nullable): four events recorded before and after the product and
// before and after the update; count: add the iteration's algorithmic bytes
// to L.prof[0 or 1] (product, by launch size) and L.prof[2] (whole iteration)
void pcg_iter(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, Lists &L, int it, int *pending,
              int mixed, const hipEvent_t *ev, bool count, const Tile *tiles, int n_tiles);
// algorithmic bytes of one assembly pass over the environments still iterating -> *prof
void asm_bytes(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, int mixed,
               unsigned long long *prof);
// tiles of environments whose PCG still iterates -> out (count at offs[B.n_vt])
void live_tiles(hipStream_t s, const EnvState &S, const Batch &B, Lists &L, Tile *out, int *flag, int *offs);
// continues the PCG of the environments whose tiles are listed (one workgroup
// each) to convergence; `it` = tiled iterations done so far
void pcg_resume(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, Lists &L, const Tile *tiles,
                int n_tiles, int it, int mixed);
void pcg_finish(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B, int mixed);
// one workgroup per environment for the environments flagged `fused`
void pcg_fused(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const int *fenv, int n_fenv,
               Lists &L, int mixed);
void spmv_debug(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
                const double *in, double *out);

void conv_check(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
                int *n_active);
// augmented-Lagrangian Dirichlet mode: after the convergence test, set the
// displacement to check (snap) / zero (multiplier update); after the swept CCD
// pass, accept the snap or update multipliers and kA
void al_prepare(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B);
void snap_J(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B);
void al_finish(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B);
void ccd_init(hipStream_t s, const EnvState &S, const Batch &B);
void accd(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n,
          const double *x, const double *p);
// inversion filter: lowers each line-searching environment's step bound to
// 0.8 x the first root of det F along the direction, over its tets
// (force = 1: every listed environment, whatever its variant flag and AL action)
void inv_bound(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, int force);
// friction lag rounds: reactivates converged environments that take another
// lagged friction update this step; *n_relag = their number
// sel = 0: every converged environment with lag rounds left; sel = 1: those
// in phase PH_RELAG (decoupled schedule)
void relag(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, int sel, int *n_relag);
// decoupled schedule: phase of every batch environment; the phase step after k_step_end
void set_phase(hipStream_t s, const EnvState &S, const Batch &B, int ph);
void phase_advance(hipStream_t s, const EnvState &S, const Batch &B);
// friction merge: clear the active flags of candidates whose environment keeps
// its friction; plan the new per-environment ranges (total -> *total); copy
// the kept pairs and set up the new ones into the second buffers
void cand_restrict(hipStream_t s, const WorldDev &W, const EnvState &S, const Lists &L, int n);
void fric_plan(hipStream_t s, const EnvState &S, const Batch &B, int *nb, int *ne, int *total);
void fric_merge(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L,
                int n_old, int n_act, const int *nb, const int *ne, int4 *fv2, double *fw2, double *fn2, double *flam2,
                int *fenv2);
void ls_init(hipStream_t s, const EnvState &S, const Batch &B);
void energy(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L, int n_cand,
            int n_fric, int zero_alpha, double *E_out);
void ls_decide(hipStream_t s, const EnvState &S, const Batch &B, int *pending);
void update_x(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B);
void iter_end(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, int *n_active);
// sel = 0: every environment in the step; sel = 1: those whose phase ends it
void step_end(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, int sel);

void stress(hipStream_t s, const WorldDev &W, int t_off, int nt, double *cauchy, double *vm);

// element-level debug kernels
void dbg_classify(hipStream_t s, int kind, int n, const double *x12, int *types, double *d2);
void dbg_pair(hipStream_t s, int kind, int type, const double *x12, double dhat, double kappa, double eps_x,
              int project, double *out /*1+12+144*/);
void dbg_tet(hipStream_t s, const double *X12, const double *x12, double mu, double la, double *out /*1+12+144*/);
void dbg_accd(hipStream_t s, int kind, int n, const double *x12, const double *p12, double sfac, double *t);
// CCD bound over n pairs of one kind: out[0] = min(1, min_k ACCD_k); part
// holds pairs_ccd_parts(n) per-block minima (no clearing needed)
int pairs_ccd_parts(int64_t n);
void pairs_ccd_bound(hipStream_t s, int kind, int n, const double *x12, const double *p12, double sfac, double *part,
                     double *out);
// the allocation-free variant's per-block minima: a static device array
// (*ptr: the current device's copy) holding pairs for up to
// noalloc_max_pairs() pairs
int64_t noalloc_max_pairs();
hipError_t noalloc_scratch(double **ptr);
// grasp-quality metrics over n_samples points on the gripper (triangle index +
// barycentric (u, v) into hand_tris) against the manipuland's triangles, at
// positions x (world vertex ids): sdf [n_samples], part [sdf_parts(n)] block
// maxima, out[0] = D1, out[1] = D2
// contact forces between tagged bodies over the active pairs in L (positions
// W.x): out [ntags*ntags*3]; f [n_act*3], fab [n_act] scratch
void contact_forces(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_act,
                    const int *tag, int v_off, int ntags, double *f, int *fab, double *out);
int sdf_parts(int n_samples);
void grasp_metrics(hipStream_t s, const double *x, const int *obj_tris, int n_obj, const int *hand_tris,
                   const int *sample_tri, const double *sample_uv, int n_samples, double *sdf, double *part,
                   double *out);
void dbg_tet_root(hipStream_t s, int n, const double *x12, const double *p12, double tmax, double *t, double *k4);

}  // namespace ipck
