// ipc_kernels.hip -- gfx950 kernels of the batched IPC Newton step.
//
// Layout: SoA-by-element world arrays (see ipc_world.h); positions are [n][3]
// FP64.  Every kernel over vertices / tets / primitives walks a tile list of
// 256-element tiles that never straddle two environments; an environment
// whose status is not ACTIVE is skipped at tile entry, which is how converged
// and failed environments drop out of the computation (Sec. III-A, problems
// (iii) and (iv)).  Reductions use fixed shared-memory trees over tiles and a
// fixed order over an environment's tiles, so no floating-point atomics are
// used anywhere.
#include <hip/hip_ext.h>

#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>

#include "device_math.h"
#include "ipc_kernels.h"

#ifndef IPC_LAUNCH
#define IPC_LAUNCH(kernel, grid, block, stream) kernel<<<(grid), (block), 0, (stream)>>>
#endif

using namespace ipcw;
using namespace ipcdev;
using ipck::GridEnt;

namespace {

constexpr int TB = kTile;

DEV double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

DEV double block_max(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double a = sh[threadIdx.x], b = sh[threadIdx.x + s];
      sh[threadIdx.x] = (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
    }
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// sum of the per-tile partials of one environment, in tile order
DEV double env_tiles_sum(const double *part, const EnvDev &e) {
  double s = 0.0;
  for (int i = 0; i < e.vtile_count; ++i) s += part[e.vtile_first + i];
  return s;
}

DEV void pair_info(const WorldDev &W, int2 c, int &kind, int v[4], int &env, double &eps_x) {
  if (c.x >= 0) {
    kind = 0;
    int4 tr = W.tri[c.y];
    v[0] = W.sv[c.x];
    v[1] = tr.x;
    v[2] = tr.y;
    v[3] = tr.z;
    env = tr.w;
    eps_x = 0.0;
  } else {
    kind = 1;
    int a = ~c.x, b = c.y;
    int4 A = W.edge[a], Bq = W.edge[b];
    v[0] = A.x;
    v[1] = A.y;
    v[2] = Bq.x;
    v[3] = Bq.y;
    env = A.z;
    eps_x = 1e-3 * W.elen2[a] * W.elen2[b];
  }
}

DEV void gather12(const double *x, const int v[4], double *out) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[3 * i + k] = x[3 * v[i] + k];
}

DEV void gather12_trial(const double *x, const double *p, double a, const int v[4], double *out) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) out[3 * i + k] = x[3 * v[i] + k] + a * p[3 * v[i] + k];
}

DEV bool active_env(const EnvState &S, int env) { return S.status[env] == ST_ACTIVE; }

// unknowns of the Newton solve: free vertices, plus the kinematic vertices of
// an environment in augmented-Lagrangian Dirichlet mode
DEV bool is_dof(const WorldDev &W, const EnvState &S, int i, int env) {
  int k = W.kin[i];
  return k == KIN_FREE || (k >= 0 && S.al[env]);
}

// ---------------------------------------------------------------------------
// step set-up: kinematic targets, predicted positions, Dirichlet displacement
// ---------------------------------------------------------------------------
DEV bool begins(const EnvState &S, int env) { return S.status[env] == ST_ACTIVE && S.phase[env] == PH_BEGIN; }

__global__ void k_begin_step(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !begins(S, t.env)) return;
  const EnvDev &E = envs[t.env];
  int i = t.start + threadIdx.x;
  int k = W.kin[i];
  double xi[3] = {W.x[3 * i], W.x[3 * i + 1], W.x[3 * i + 2]};
  for (int c = 0; c < 3; ++c) W.xn[3 * i + c] = xi[c];
  if (k == KIN_PAD) {
    for (int c = 0; c < 3; ++c) {
      W.xh[3 * i + c] = xi[c];
      W.p[3 * i + c] = 0.0;
    }
    return;
  }
  // after the schedule's motion and gravity rows: per group its hold row
  // (-1: none), then the gravity override (flag, g)
  const double *ctl = W.motion + E.mo_off + (12 * E.n_groups + 3) * E.n_motion;
  if (k >= 0) {
    int row = min(E.step + 1, E.n_motion - 1);
    if (ctl[k] >= 0.0) row = min(row, (int)ctl[k]);
    const double *T = W.motion + E.mo_off + 12 * (row * E.n_groups + k);
    const double *X = W.X + 3 * i;
    for (int r = 0; r < 3; ++r) {
      double xb = T[4 * r] * X[0] + T[4 * r + 1] * X[1] + T[4 * r + 2] * X[2] + T[4 * r + 3];
      W.xh[3 * i + r] = xb;
      W.p[3 * i + r] = xb - xi[r];
    }
  } else {
    int grow = min(E.step, E.n_motion - 1);
    const double *g = W.motion + E.mo_off + 12 * E.n_motion * E.n_groups + 3 * grow;
    if (ctl[E.n_groups] != 0.0) g = ctl + E.n_groups + 1;
    double h = E.dt;
    for (int c = 0; c < 3; ++c) {
      W.xh[3 * i + c] = xi[c] + h * W.v[3 * i + c] + h * h * g[c];
      W.p[3 * i + c] = 0.0;
    }
  }
}

__global__ void k_dbc_J(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !begins(S, t.env)) return;
  int e = t.start + threadIdx.x;
  int4 q = W.tet[e];
  int v[4] = {q.x, q.y, q.z, q.w};
  double x[12];
  gather12_trial(W.xn, W.p, 1.0, v, x);
  double F[9];
  nh_F(x, W.Dinv + 9 * e, F);
  if (!(det33(F) > 0.0)) S.dbc_bad[t.env] = 1;
}

__global__ void k_apply_dbc(WorldDev W, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !begins(S, t.env)) return;
  int i = t.start + threadIdx.x;
  if (W.kin[i] < 0) return;
  if (S.al[t.env]) {
    for (int c = 0; c < 3; ++c) W.lam[3 * i + c] = 0.0;  // multipliers start at zero
    return;
  }
  for (int c = 0; c < 3; ++c) W.x[3 * i + c] = W.xh[3 * i + c];
}

__global__ void k_env_begin(const EnvDev *envs, EnvState S, const int *benv, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (S.phase[e] != PH_BEGIN) return;
  S.in_step[e] = 0;
  if (S.status[e] == ST_FAILED) return;
  S.in_step[e] = 1;
  S.status[e] = ST_ACTIVE;
  S.reason[e] = FAIL_NONE;
  S.iters[e] = 0;
  S.iter_cap[e] = envs[e].maxit;
  S.lag[e] = 0;
  S.halvings[e] = 0;
  S.pcg_total[e] = 0;
  S.dbc_bad[e] = 0;
  S.al[e] = 0;
  S.al_action[e] = 0;
  S.amax_bits[e] = (unsigned long long)__double_as_longlong(1.0);
}

__global__ void k_env_dbc(EnvState S, const int *envs, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = envs[j];
  if (!begins(S, e)) return;
  double a = __longlong_as_double((long long)S.amax_bits[e]);
  if (a < 1.0 || S.dbc_bad[e]) {
    // the prescribed move is not feasible in one go: the kinematic vertices
    // become unknowns pulled to their targets by an augmented Lagrangian
    S.al[e] = 1;
    S.kA[e] = 1e3;
    S.viol_prev[e] = kInf;
  }
}

// ---------------------------------------------------------------------------
// broad phase: dhat-widened boxes, brute-force overlap per environment
// ---------------------------------------------------------------------------
__global__ void k_boxes(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, int which, const double *x,
                        const double *p) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  const EnvDev &E = envs[t.env];
  int j = t.start + threadIdx.x;
  int v[3];
  int n;
  double *out;
  if (which == 0) {
    v[0] = W.sv[j];
    n = 1;
    out = W.box_sv + 6 * j;
  } else if (which == 1) {
    int4 q = W.tri[j];
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    n = 3;
    out = W.box_tri + 6 * j;
  } else {
    int4 q = W.edge[j];
    v[0] = q.x;
    v[1] = q.y;
    n = 2;
    out = W.box_edge + 6 * j;
  }
  double lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      double a = x[3 * v[i] + k];
      lo[k] = fmin(lo[k], a);
      hi[k] = fmax(hi[k], a);
      if (p) {
        double b = a + p[3 * v[i] + k];
        lo[k] = fmin(lo[k], b);
        hi[k] = fmax(hi[k], b);
      }
    }
  for (int k = 0; k < 3; ++k) {
    out[k] = lo[k] - E.dhat;
    out[3 + k] = hi[k] + E.dhat;
  }
}

// ---------------------------------------------------------------------------
// hash-grid broad phase.  Each environment's triangles and edges are binned
// into cubic cells of size E.cell (their dhat-widened boxes cover at most 4
// cells per axis; larger boxes go to a per-environment "big" list).  A query
// primitive visits the cells its box covers and reports a pair only from the
// cell that holds the lower corner of the two boxes' intersection, so every
// overlapping pair is found exactly once; each query sorts its own hits, so
// the order of the output is deterministic.  The result is the same set as
// testing all pairs.
// ---------------------------------------------------------------------------
constexpr int kMaxSpan = 4;

DEV bool cell_range(const double *box, double h, int lo[3], int hi[3]) {
  bool big = false;
  for (int k = 0; k < 3; ++k) {
    double a = floor(box[k] / h), b = floor(box[3 + k] / h);
    if (!(a > -1e9 && b < 1e9)) {  // also catches NaN
      big = true;
      lo[k] = hi[k] = 0;
      continue;
    }
    lo[k] = (int)a;
    hi[k] = (int)b;
    if (hi[k] - lo[k] >= kMaxSpan) big = true;
  }
  return big;
}

DEV unsigned cell_hash(int kind, int env, int cx, int cy, int cz, unsigned mask) {
  unsigned h = (unsigned)cx * 73856093u ^ (unsigned)cy * 19349663u ^ (unsigned)cz * 83492791u ^
               (unsigned)env * 2654435761u ^ (unsigned)kind * 0x9E3779B9u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return h & mask;
}

// float bounds that enclose a double interval
DEV float f_down(double v) {
  float f = (float)v;
  return ((double)f > v) ? nextafterf(f, -INFINITY) : f;
}
DEV float f_up(double v) {
  float f = (float)v;
  return ((double)f < v) ? nextafterf(f, INFINITY) : f;
}

DEV int bitem_index(const EnvDev &E, int kind, int b) {
  return E.bitem_off + (kind == 0 ? (b - E.tri_off) : (E.ntri + b - E.e_off));
}

__global__ void k_grid_count(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, int *ncell, int *isbig) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count) return;
  const EnvDev &E = envs[t.env];
  int kind = t.rel, b = t.start + threadIdx.x;
  int it = bitem_index(E, kind, b);
  if (!active_env(S, t.env)) {
    ncell[it] = 0;
    isbig[it] = 0;
    return;
  }
  const double *box = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
  int lo[3], hi[3];
  bool big = cell_range(box, E.cell, lo, hi);
  isbig[it] = big ? 1 : 0;
  ncell[it] = big ? 0 : (hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
}

__global__ void k_grid_fill(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, const int *eoff,
                            const int *bigoff, GridEnt *ent, int *ebucket, int *bcnt, int *bigl, unsigned mask) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  const EnvDev &E = envs[t.env];
  int kind = t.rel, b = t.start + threadIdx.x;
  int it = bitem_index(E, kind, b);
  int code = (kind == 0) ? b : ~b;
  const double *box = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
  int lo[3], hi[3];
  if (cell_range(box, E.cell, lo, hi)) {
    bigl[bigoff[it]] = code;
    return;
  }
  int o = eoff[it];
  GridEnt g;
  g.code = code;
  g.env = t.env;
  g.pad = 0;
  for (int k = 0; k < 3; ++k) {
    g.lo[k] = f_down(box[k]);
    g.hi[k] = f_up(box[3 + k]);
  }
  for (int cx = lo[0]; cx <= hi[0]; ++cx)
    for (int cy = lo[1]; cy <= hi[1]; ++cy)
      for (int cz = lo[2]; cz <= hi[2]; ++cz) {
        unsigned h = cell_hash(kind, t.env, cx, cy, cz, mask);
        g.cx = cx;
        g.cy = cy;
        g.cz = cz;
        ent[o] = g;
        ebucket[o] = (int)h;
        atomicAdd(&bcnt[h], 1);
        ++o;
      }
}

__global__ void k_grid_place(const GridEnt *ent, const int *ebucket, int n, const int *boff, int *bcur,
                             GridEnt *sorted) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int h = ebucket[k];
  sorted[boff[h] + atomicAdd(&bcur[h], 1)] = ent[k];
}


__global__ void k_big_seg(const EnvDev *envs, EnvState S, const int *benv, int n, const int *bigoff) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  const EnvDev &E = envs[e];
  S.big_beg[e] = bigoff[E.bitem_off];
  S.big_end[e] = bigoff[E.bitem_off + E.ntri + E.ne];
}

struct QueryPrim {
  double lo[3], hi[3];
  float flo[3], fhi[3];
  int v0, v1;
  bool akin;
};

// exclusions + emission of one candidate pair (a query, b candidate)
DEV bool accept_pair(const WorldDev &W, int kind, const QueryPrim &A, int b) {
  if (kind == 0) {
    int4 q = W.tri[b];
    if (A.v0 == q.x || A.v0 == q.y || A.v0 == q.z) return false;
    if (A.akin && W.kin[q.x] >= 0 && W.kin[q.y] >= 0 && W.kin[q.z] >= 0) return false;
  } else {
    int4 q = W.edge[b];
    if (A.v0 == q.x || A.v0 == q.y || A.v1 == q.x || A.v1 == q.y) return false;
    if (A.akin && W.kin[q.x] >= 0 && W.kin[q.y] >= 0) return false;
  }
  return true;
}

DEV bool boxes_overlap(const QueryPrim &A, const double *bx) {
  return A.lo[0] <= bx[3] && bx[0] <= A.hi[0] && A.lo[1] <= bx[4] && bx[1] <= A.hi[1] && A.lo[2] <= bx[5] &&
         bx[2] <= A.hi[2];
}

// WRITE = false: count each query's pairs and keep the first stash_n of them,
// in their final order, in stash[item * stash_n ...]; queries with more are
// counted in *n_over.  WRITE = true: write the pairs of those queries only
// (the others are copied from the stash by k_bp_gather).
template <bool WRITE>
__global__ void __launch_bounds__(256) k_bp_grid(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles,
                                                 int *counts, const int *offs, int2 *out, const GridEnt *sorted,
                                                 const int *boff, const int *bigl, unsigned mask, int2 *stash,
                                                 int stash_n, int *n_over) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count) return;
  const EnvDev &E = envs[t.env];
  int kind = t.rel;
  int a = t.start + threadIdx.x;
  int item = E.item_off + (kind == 0 ? (a - E.sv_off) : (E.nsv + a - E.e_off));
  if (!active_env(S, t.env)) {
    if (!WRITE) counts[item] = 0;
    return;
  }
  if (WRITE && counts[item] <= stash_n) return;
  int2 *st = stash + (size_t)item * stash_n;
  QueryPrim A;
  const double *bx = (kind == 0 ? W.box_sv : W.box_edge) + 6 * a;
  for (int k = 0; k < 3; ++k) {
    A.lo[k] = bx[k];
    A.hi[k] = bx[3 + k];
    A.flo[k] = f_down(bx[k]);
    A.fhi[k] = f_up(bx[3 + k]);
  }
  if (kind == 0) {
    A.v0 = W.sv[a];
    A.v1 = -1;
    A.akin = W.kin[A.v0] >= 0;
  } else {
    int4 q = W.edge[a];
    A.v0 = q.x;
    A.v1 = q.y;
    A.akin = W.kin[q.x] >= 0 && W.kin[q.y] >= 0;
  }
  const double h = E.cell;
  int cnt = 0;
  int pos = WRITE ? offs[item] : 0;
  int lo[3], hi[3];
  bool big = cell_range(bx, h, lo, hi);
  if (big) {
    // every candidate of the environment, like an all-pairs test
    int bbeg = (kind == 0) ? E.tri_off : a + 1;
    int bend = (kind == 0) ? E.tri_off + E.ntri : E.e_off + E.ne;
    for (int b = bbeg; b < bend; ++b) {
      const double *bb = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
      if (!boxes_overlap(A, bb) || !accept_pair(W, kind, A, b)) continue;
      const int2 hit = kind == 0 ? make_int2(a, b) : make_int2(~a, b);
      if (WRITE)
        out[pos++] = hit;
      else if (cnt < stash_n)
        st[cnt] = hit;
      ++cnt;
    }
  } else {
    for (int cx = lo[0]; cx <= hi[0]; ++cx)
      for (int cy = lo[1]; cy <= hi[1]; ++cy)
        for (int cz = lo[2]; cz <= hi[2]; ++cz) {
          unsigned hh = cell_hash(kind, t.env, cx, cy, cz, mask);
          for (int e = boff[hh]; e < boff[hh + 1]; ++e) {
            const GridEnt &en = sorted[e];
            if (en.cx != cx || en.cy != cy || en.cz != cz || en.env != t.env) continue;
            if ((kind == 0) != (en.code >= 0)) continue;
            // outward-rounded float boxes: no overlap here means none in FP64
            if (A.flo[0] > en.hi[0] || en.lo[0] > A.fhi[0] || A.flo[1] > en.hi[1] || en.lo[1] > A.fhi[1] ||
                A.flo[2] > en.hi[2] || en.lo[2] > A.fhi[2])
              continue;
            int b = (kind == 0) ? en.code : ~en.code;
            if (kind == 1 && b <= a) continue;
            const double *bb = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
            if (!boxes_overlap(A, bb)) continue;
            // owner cell: the one holding the lower corner of the intersection
            if ((int)floor(fmax(A.lo[0], bb[0]) / h) != cx || (int)floor(fmax(A.lo[1], bb[1]) / h) != cy ||
                (int)floor(fmax(A.lo[2], bb[2]) / h) != cz)
              continue;
            if (!accept_pair(W, kind, A, b)) continue;
            const int2 hit = kind == 0 ? make_int2(a, b) : make_int2(~a, b);
            if (WRITE)
              out[pos++] = hit;
            else if (cnt < stash_n)
              st[cnt] = hit;
            ++cnt;
          }
        }
    // bucket order depends on atomics: put this query's cell hits in
    // candidate-index order so the output is deterministic
    int2 *o = WRITE ? out + offs[item] : st;
    const int nc = WRITE ? pos - offs[item] : (cnt <= stash_n ? cnt : 0);
    for (int j = 1; j < nc; ++j) {
      int2 key = o[j];
      int m = j - 1;
      while (m >= 0 && o[m].y > key.y) {
        o[m + 1] = o[m];
        --m;
      }
      o[m + 1] = key;
    }
    for (int j = S.big_beg[t.env]; j < S.big_end[t.env]; ++j) {
      int code = bigl[j];
      if ((kind == 0) != (code >= 0)) continue;
      int b = (kind == 0) ? code : ~code;
      if (kind == 1 && b <= a) continue;
      const double *bb = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
      if (!boxes_overlap(A, bb) || !accept_pair(W, kind, A, b)) continue;
      const int2 hit = kind == 0 ? make_int2(a, b) : make_int2(~a, b);
      if (WRITE)
        out[pos++] = hit;
      else if (cnt < stash_n)
        st[cnt] = hit;
      ++cnt;
    }
  }
  if (!WRITE) {
    counts[item] = cnt;
    if (cnt > stash_n) atomicAdd(n_over, 1);
  }
}

// Counting pass with kBpGroup lanes per query (launch: kBpGroup blocks per
// query tile).  The lanes of a group take every kBpGroup-th entry of each
// bucket (and of the big list or the all-pairs range), so that a group's loads
// are adjacent; each round's hits are placed by a ballot prefix count in the
// order one lane walking the entries would find them, and the group's first
// lane sorts the cell hits.  Same output as k_bp_grid<false>.
constexpr int kBpGroup = 8;
__global__ void __launch_bounds__(256) k_bp_coop(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles,
                                                 int *counts, const GridEnt *sorted, const int *boff,
                                                 const int *bigl, unsigned mask, int2 *stash, int stash_n,
                                                 int *n_over) {
  constexpr int G = kBpGroup, QPB = TB / G;
  Tile t = tiles[blockIdx.x / G];
  const int qi = (int)(blockIdx.x % G) * QPB + (int)threadIdx.x / G;  // query within the tile
  if (qi >= t.count) return;  // the whole group
  const int gl = threadIdx.x % G, gbase = (threadIdx.x & 63) & ~(G - 1);
  const unsigned long long below = (1ull << gl) - 1;
  const EnvDev &E = envs[t.env];
  const int kind = t.rel;
  const int a = t.start + qi;
  const int item = E.item_off + (kind == 0 ? (a - E.sv_off) : (E.nsv + a - E.e_off));
  if (!active_env(S, t.env)) {
    if (gl == 0) counts[item] = 0;
    return;
  }
  int2 *st = stash + (size_t)item * stash_n;
  QueryPrim A;
  const double *bx = (kind == 0 ? W.box_sv : W.box_edge) + 6 * a;
  for (int k = 0; k < 3; ++k) {
    A.lo[k] = bx[k];
    A.hi[k] = bx[3 + k];
    A.flo[k] = f_down(bx[k]);
    A.fhi[k] = f_up(bx[3 + k]);
  }
  if (kind == 0) {
    A.v0 = W.sv[a];
    A.v1 = -1;
    A.akin = W.kin[A.v0] >= 0;
  } else {
    int4 q = W.edge[a];
    A.v0 = q.x;
    A.v1 = q.y;
    A.akin = W.kin[q.x] >= 0 && W.kin[q.y] >= 0;
  }
  const double h = E.cell;
  int cnt = 0;
  // one round of the group: every lane with a hit stores it at its place
  auto emit = [&](bool hit, int b) {
    const unsigned long long m = (__ballot(hit) >> gbase) & ((1ull << G) - 1);
    if (hit) {
      const int pos = cnt + __popcll(m & below);
      if (pos < stash_n) st[pos] = kind == 0 ? make_int2(a, b) : make_int2(~a, b);
    }
    cnt += __popcll(m);
  };
  int lo[3], hi[3];
  if (cell_range(bx, h, lo, hi)) {
    // every candidate of the environment, like an all-pairs test
    const int bbeg = (kind == 0) ? E.tri_off : a + 1;
    const int bend = (kind == 0) ? E.tri_off + E.ntri : E.e_off + E.ne;
    for (int b0 = bbeg; b0 < bend; b0 += G) {
      const int b = b0 + gl;
      bool hit = false;
      if (b < bend) {
        const double *bb = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
        hit = boxes_overlap(A, bb) && accept_pair(W, kind, A, b);
      }
      emit(hit, b);
    }
  } else {
    for (int cx = lo[0]; cx <= hi[0]; ++cx)
      for (int cy = lo[1]; cy <= hi[1]; ++cy)
        for (int cz = lo[2]; cz <= hi[2]; ++cz) {
          const unsigned hh = cell_hash(kind, t.env, cx, cy, cz, mask);
          const int e0 = boff[hh], e1 = boff[hh + 1];
          for (int eb = e0; eb < e1; eb += G) {
            const int e = eb + gl;
            bool hit = false;
            int b = 0;
            if (e < e1) {
              const GridEnt &en = sorted[e];
              b = (kind == 0) ? en.code : ~en.code;
              // outward-rounded float boxes: no overlap here means none in FP64
              hit = en.cx == cx && en.cy == cy && en.cz == cz && en.env == t.env && (kind == 0) == (en.code >= 0) &&
                    !(A.flo[0] > en.hi[0] || en.lo[0] > A.fhi[0] || A.flo[1] > en.hi[1] || en.lo[1] > A.fhi[1] ||
                      A.flo[2] > en.hi[2] || en.lo[2] > A.fhi[2]) &&
                    !(kind == 1 && b <= a);
              if (hit) {
                const double *bb = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
                // owner cell: the one holding the lower corner of the intersection
                hit = boxes_overlap(A, bb) && (int)floor(fmax(A.lo[0], bb[0]) / h) == cx &&
                      (int)floor(fmax(A.lo[1], bb[1]) / h) == cy && (int)floor(fmax(A.lo[2], bb[2]) / h) == cz &&
                      accept_pair(W, kind, A, b);
              }
            }
            emit(hit, b);
          }
        }
    // bucket order depends on atomics: the first lane puts the query's cell
    // hits in candidate-index order so the output is deterministic
    if (gl == 0 && cnt <= stash_n)
      for (int j = 1; j < cnt; ++j) {
        int2 key = st[j];
        int m = j - 1;
        while (m >= 0 && st[m].y > key.y) {
          st[m + 1] = st[m];
          --m;
        }
        st[m + 1] = key;
      }
    const int jb = S.big_beg[t.env], je = S.big_end[t.env];
    for (int j0 = jb; j0 < je; j0 += G) {
      const int j = j0 + gl;
      bool hit = false;
      int b = 0;
      if (j < je) {
        const int code = bigl[j];
        b = (kind == 0) ? code : ~code;
        hit = (kind == 0) == (code >= 0) && !(kind == 1 && b <= a);
        if (hit) {
          const double *bb = (kind == 0 ? W.box_tri : W.box_edge) + 6 * b;
          hit = boxes_overlap(A, bb) && accept_pair(W, kind, A, b);
        }
      }
      emit(hit, b);
    }
  }
  if (gl == 0) {
    counts[item] = cnt;
    if (cnt > stash_n) atomicAdd(n_over, 1);
  }
}

// pairs of the queries that fit the stash, copied to their place in the list
__global__ void k_bp_gather(const int *counts, const int *offs, const int2 *stash, int stash_n, int n_items,
                            int2 *out) {
  int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= n_items) return;
  const int c = counts[item];
  if (c > stash_n) return;
  const int2 *st = stash + (size_t)item * stash_n;
  int2 *o = out + offs[item];
  for (int j = 0; j < c; ++j) o[j] = st[j];
}

// ---------------------------------------------------------------------------
// exclusive scan of int counts: out[0..n], out[n] = total
// ---------------------------------------------------------------------------
constexpr int SCAN_PER_BLOCK = 1024;

__global__ void k_scan1(const int *in, int *out, int n, int *bsum) {
  __shared__ int sh[TB];
  int base = blockIdx.x * SCAN_PER_BLOCK;
  int v[4], s = 0;
  for (int k = 0; k < 4; ++k) {
    int i = base + threadIdx.x * 4 + k;
    v[k] = (i < n) ? in[i] : 0;
    s += v[k];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < TB; off <<= 1) {
    int add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - s;
  for (int k = 0; k < 4; ++k) {
    int i = base + threadIdx.x * 4 + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == TB - 1) bsum[blockIdx.x] = sh[TB - 1];
}

__global__ void k_scan2(int *bsum, int nb, int *total_out) {
  __shared__ int sh[TB];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += TB) {
    int i = c0 + threadIdx.x;
    int v = (i < nb) ? bsum[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < TB; off <<= 1) {
      int add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
    int tot = sh[TB - 1];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan3(int *out, int n, const int *bsum) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += bsum[i / SCAN_PER_BLOCK];
}

// per-env candidate segments [beg, end) from the scanned item offsets
__global__ void k_cand_seg(const EnvDev *envs, EnvState S, const int *benv, int n, const int *offs) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  const EnvDev &E = envs[e];
  S.cand_beg[e] = offs[E.item_off];
  S.cand_end[e] = offs[E.item_off + E.nsv + E.ne];
}

// ---------------------------------------------------------------------------
// narrow phase: type, d^2, active flag (d^2 < dhat^2)
// ---------------------------------------------------------------------------
__global__ void k_classify(WorldDev W, const EnvDev *envs, const int2 *cand, int n, const double *x, int *type,
                           double *d2o, int *flag) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int kind, v[4], env;
  double ex;
  pair_info(W, cand[k], kind, v, env, ex);
  double xx[12];
  gather12(x, v, xx);
  double d2;
  int ty = classify(kind, xx, &d2);
  double dh = envs[env].dhat;
  type[k] = ty;
  d2o[k] = d2;
  flag[k] = (d2 < dh * dh) ? 1 : 0;
}

__global__ void k_compact(const int2 *cand, const int *type, const double *d2, const int *flag, const int *offs,
                          int n, int2 *act, int *act_type, double *act_d2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || !flag[k]) return;
  int o = offs[k];
  act[o] = cand[k];
  act_type[o] = type[k];
  act_d2[o] = d2[k];
}

__global__ void k_act_seg(EnvState S, const int *benv, int n, const int *offs) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  S.act_beg[e] = offs[S.cand_beg[e]];
  S.act_end[e] = offs[S.cand_end[e]];
}

// Contact statistics of the iterate just classified, one block per
// environment still iterating: the number of active pairs and the least
// squared distance among them.  With `adapt` (a Newton iterate) and the
// adaptive-stiffness variant, kappa doubles, up to 100 times its given value,
// when the least distance is below 1e-2 dhat and smaller than at the
// previous iterate.
__global__ void k_act_stats(const EnvDev *envs, EnvState S, const int *benv, const double *act_d2, int adapt) {
  __shared__ double sh[TB];
  int e = benv[blockIdx.x];
  if (S.status[e] != ST_ACTIVE) return;
  const int b = S.act_beg[e], n = S.act_end[e] - b;
  double m = kInf;
  for (int i = threadIdx.x; i < n; i += TB) m = fmin(m, act_d2[b + i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  m = sh[0];
  S.nact[e] = n;
  S.dmin2[e] = m;
  const EnvDev &E = envs[e];
  if (adapt && E.adapt_kappa) {
    const double d = sqrt(m);
    if (d < 1e-2 * E.dhat && d < S.dmin_prev[e]) S.kappa[e] = fmin(2.0 * S.kappa[e], 100.0 * S.kappa0[e]);
    S.dmin_prev[e] = d;
  }
}

// ---------------------------------------------------------------------------
// contact elements
// ---------------------------------------------------------------------------
DEV void store_blocks(const double *H, double *out) {
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b) {
      double *B = out + 9 * blk_index(a, b);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) B[3 * r + c] = H[(3 * a + r) * 12 + 3 * b + c];
    }
}

// Barrier contact elements.  The unmollified, non-degenerate pairs (nearly
// all) are formed without the 12x12 matrix (pair_barrier_fast: no per-lane
// scratch memory); the others are listed in slow (count in *n_slow) for
// k_barrier_elems_full.  Each pair writes only its own slot, so the split
// changes no result.
__global__ void __launch_bounds__(128) k_barrier_elems(WorldDev W, const EnvDev *envs, const double *kap,
                                                       const int2 *act, const int *act_type, int n, const double *x,
                                                       int4 *ce_v, double *ce_g, double *ce_H, int *n_slow,
                                                       int *slow) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int kind, v[4], env;
  double ex;
  pair_info(W, act[k], kind, v, env, ex);
  const EnvDev &E = envs[env];
  double xx[12], g[12];
  gather12(x, v, xx);
  if (pair_barrier_fast(kind, act_type[k], xx, E.dhat, kap[env], ex, g, ce_H + 90 * (size_t)k) < 0.0) {
    slow[atomicAdd(n_slow, 1)] = k;
    return;
  }
  ce_v[k] = make_int4(v[0], v[1], v[2], v[3]);
  for (int i = 0; i < 12; ++i) ce_g[12 * k + i] = g[i];
}

// the listed pairs: mollified edge-edge pairs and degenerate ones, through
// the full 12x12 element and its Jacobi projection (grid-stride over the
// list, whose length only the device knows).  Each thread's 12x12 matrix and
// Jacobi workspace sit in LDS (kFullStride doubles per thread: bank-spread
// rows) rather than in per-lane scratch memory.
constexpr int kFullThreads = 32, kFullStride = 321;
__global__ void __launch_bounds__(kFullThreads)
    k_barrier_elems_full(WorldDev W, const EnvDev *envs, const double *kap, const int2 *act, const int *act_type,
                         const double *x, int4 *ce_v, double *ce_g, double *ce_H, const int *n_slow, const int *slow) {
  __shared__ double lds[kFullThreads * kFullStride];
  double *H = lds + threadIdx.x * kFullStride, *scr = H + 144;
  const int m = *n_slow;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    const int k = slow[j];
    int kind, v[4], env;
    double ex;
    pair_info(W, act[k], kind, v, env, ex);
    const EnvDev &E = envs[env];
    double xx[12], g[12];
    gather12(x, v, xx);
    pair_barrier_full(kind, act_type[k], xx, E.dhat, kap[env], ex, true, g, H, scr);
    ce_v[k] = make_int4(v[0], v[1], v[2], v[3]);
    for (int i = 0; i < 12; ++i) ce_g[12 * k + i] = g[i];
    store_blocks(H, ce_H + 90 * (size_t)k);
  }
}

// lagged friction data at x^n (positions in W.x at set-up time)
// (nb != nullptr: the pair of environment env goes to position nb[env] + its
// index within the environment's active pairs, act_beg the first of those)
__global__ void k_friction_setup(WorldDev W, const EnvDev *envs, const double *kap, const int2 *act,
                                 const int *act_type, int n, int4 *fv, double *fw, double *fn, double *flam,
                                 int *fenv, const int *nb, const int *act_beg) {
  int kk = blockIdx.x * blockDim.x + threadIdx.x;
  if (kk >= n) return;
  int kind, v[4], env;
  double ex;
  pair_info(W, act[kk], kind, v, env, ex);
  const int k = nb ? nb[env] + (kk - act_beg[env]) : kk;
  const EnvDev &E = envs[env];
  double xx[12], w[4];
  gather12(W.x, v, xx);
  int ty = act_type[kk];
  closest_weights(kind, ty, xx, w);
  double dv[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 3; ++c) dv[c] += w[i] * xx[3 * i + c];
  double dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  double d2;
  classify(kind, xx, &d2);
  double d = sqrt(d2), b0, b1, b2;
  barrier_b(d, E.dhat, &b0, &b1, &b2);
  double e = 1.0;
  if (kind == 1) {
    d3 nn = cross3(sub3(ld3(xx + 3), ld3(xx)), sub3(ld3(xx + 9), ld3(xx + 6)));
    double c = dot3(nn, nn);
    if (c < ex) e = (c / ex) * (2.0 - c / ex);
  }
  fv[k] = make_int4(v[0], v[1], v[2], v[3]);
  for (int i = 0; i < 4; ++i) fw[4 * k + i] = w[i];
  for (int c = 0; c < 3; ++c) fn[3 * k + c] = dv[c] / dn;
  flam[k] = -kap[env] * e * b1;
  fenv[k] = env;
}

// Contact force of every active pair (grasp validation, Sec. III-D): the
// barrier pushes the pair's first side (the point / first edge) along the unit
// normal n of the closest-point difference with lambda = -kappa e b'(d), the
// second side with the opposite force.  f[k] = lambda n; fab[k] = the tag pair
// (first side's tag) * ntags + (second side's tag), -1 if either is untagged.
__global__ void k_pair_force(WorldDev W, const EnvDev *envs, const double *kap, const int2 *act, const int *act_type,
                             int n, const int *tag, int v_off, int ntags, double *f, int *fab) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int kind, v[4], env;
  double ex;
  pair_info(W, act[k], kind, v, env, ex);
  const EnvDev &E = envs[env];
  double xx[12], w[4];
  gather12(W.x, v, xx);
  closest_weights(kind, act_type[k], xx, w);
  // closest_weights gives the closest-point difference up to orientation:
  // make it point from the second side to the first (the first side's
  // weights sum to +1)
  const double first = kind == 0 ? w[0] : w[0] + w[1];
  const double sg = first < 0.0 ? -1.0 : 1.0;
  double dv[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 3; ++c) dv[c] += sg * w[i] * xx[3 * i + c];
  const double dn = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
  double d2;
  classify(kind, xx, &d2);
  double b0, b1, b2;
  barrier_b(sqrt(d2), E.dhat, &b0, &b1, &b2);
  double e = 1.0;
  if (kind == 1) {
    d3 nn = cross3(sub3(ld3(xx + 3), ld3(xx)), sub3(ld3(xx + 9), ld3(xx + 6)));
    double c = dot3(nn, nn);
    if (c < ex) e = (c / ex) * (2.0 - c / ex);
  }
  const double lam = -kap[env] * e * b1;
  for (int c = 0; c < 3; ++c) f[3 * k + c] = lam * dv[c] / dn;
  const int ta = tag[v[0] - v_off], tb = tag[v[kind == 0 ? 1 : 2] - v_off];
  fab[k] = (ta >= 0 && ta < ntags && tb >= 0 && tb < ntags) ? ta * ntags + tb : -1;
}

// out[(a ntags + b) 3 + c]: force on the vertices tagged a from those tagged b,
// one block per (a, b): the pairs of tag pair (a, b) add their force, those of
// (b, a) subtract it; each thread sums a fixed stride, then a fixed tree
__global__ void k_tag_force_sum(const double *f, const int *fab, int n, int ntags, double *out) {
  __shared__ double sh[3 * TB];
  const int a = blockIdx.x / ntags, b = blockIdx.x % ntags;
  const int ab = a * ntags + b, ba = b * ntags + a;
  double s[3] = {0, 0, 0};
  for (int k = threadIdx.x; k < n; k += TB) {
    const double sg = fab[k] == ab ? 1.0 : (fab[k] == ba ? -1.0 : 0.0);
    if (sg != 0.0 && ab != ba)
      for (int c = 0; c < 3; ++c) s[c] += sg * f[3 * k + c];
  }
  for (int c = 0; c < 3; ++c) sh[c * TB + threadIdx.x] = s[c];
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 3; ++c) sh[c * TB + threadIdx.x] += sh[c * TB + threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) out[3 * ab + c] = sh[c * TB];
}

// friction potential mu lambda f0(|u|), u = (I - n n^T) sum_i w_i (x_i - x^n_i):
// grad_i = mu lambda w_i (f1(y)/y) u,  hess_ij = mu lambda w_i w_j [a (I - n n^T) + c u u^T]
// with a = f1/y, c = (f1' - f1/y) / y^2 (closed form, PSD).
__global__ void k_friction_elems(WorldDev W, const EnvDev *envs, EnvState S, const int4 *fv, const double *fw,
                                 const double *fn, const double *flam, const int *fenv, int n, const double *x,
                                 int4 *ce_v, double *ce_g, double *ce_H) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int env = fenv[k];
  const EnvDev &E = envs[env];
  int4 q = fv[k];
  int v[4] = {q.x, q.y, q.z, q.w};
  double w[4] = {fw[4 * k], fw[4 * k + 1], fw[4 * k + 2], fw[4 * k + 3]};
  double nr[3] = {fn[3 * k], fn[3 * k + 1], fn[3 * k + 2]};
  double u[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 3; ++c) u[c] += w[i] * (x[3 * v[i] + c] - W.xn[3 * v[i] + c]);
  double un = u[0] * nr[0] + u[1] * nr[1] + u[2] * nr[2];
  for (int c = 0; c < 3; ++c) u[c] -= un * nr[c];
  double y = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double eps = E.eps_v * E.dt;
  double f1y, a, cc;
  if (y < eps) {
    f1y = 2.0 / eps - y / (eps * eps);
    a = f1y;
    cc = (y > 0.0) ? -1.0 / (eps * eps * y) : 0.0;
  } else {
    f1y = 1.0 / y;
    a = 1.0 / y;
    cc = -1.0 / (y * y * y);
  }
  bool on = S.status[env] == ST_ACTIVE;
  double sc = on ? E.mu * flam[k] : 0.0;
  double K[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) K[3 * r + c] = a * ((r == c ? 1.0 : 0.0) - nr[r] * nr[c]) + cc * u[r] * u[c];
  ce_v[k] = make_int4(v[0], v[1], v[2], v[3]);
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 3; ++c) ce_g[12 * (size_t)k + 3 * i + c] = sc * w[i] * f1y * u[c];
  for (int i = 0; i < 4; ++i)
    for (int j = i; j < 4; ++j) {
      double *B = ce_H + 90 * (size_t)k + 9 * blk_index(i, j);
      double s = sc * w[i] * w[j];
      for (int r = 0; r < 9; ++r) B[r] = s * K[r];
    }
}

// ---------------------------------------------------------------------------
// vertex -> contact element incidence (free vertices only), sorted per vertex
// ---------------------------------------------------------------------------
__global__ void k_inc_count(WorldDev W, EnvState S, const int4 *ce_v, int n, int *cnt) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int4 q = ce_v[k];
  int v[4] = {q.x, q.y, q.z, q.w};
  for (int a = 0; a < 4; ++a)
    if (is_dof(W, S, v[a], W.venv[v[a]])) atomicAdd(&cnt[v[a]], 1);
}

__global__ void k_inc_fill(WorldDev W, EnvState S, const int4 *ce_v, int n, const int *off, int *cur, int *ent) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int4 q = ce_v[k];
  int v[4] = {q.x, q.y, q.z, q.w};
  for (int a = 0; a < 4; ++a)
    if (is_dof(W, S, v[a], W.venv[v[a]])) {
      int pos = atomicAdd(&cur[v[a]], 1);
      ent[off[v[a]] + pos] = 4 * k + a;
    }
}

__global__ void k_inc_sort(const int *off, int *ent, int nv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  int b = off[i], e = off[i + 1];
  for (int j = b + 1; j < e; ++j) {
    int key = ent[j], m = j - 1;
    while (m >= b && ent[m] > key) {
      ent[m + 1] = ent[m];
      --m;
    }
    ent[m + 1] = key;
  }
}

// Contact blocks per row, merged by column: row i's incidence entries (element,
// local vertex a, in element order) give the blocks (a, b), b = 0..3, at
// column v_b, numbered k = 4 * entry + b.  They are ordered by (column, k) and
// the blocks of one column are summed in that order (FP64, plus an FP32 copy
// for mixed precision).  Output starts at 4 * inc_off[i]; cr_cnt[i] = number
// of distinct columns.  One 64-lane wavefront per row with contact; the rows
// are listed by k_contact_row_list.
__global__ void k_contact_row_flags(const int *inc_off, int nv, int *flag, int *cr_cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  flag[i] = inc_off[i + 1] > inc_off[i] ? 1 : 0;
  cr_cnt[i] = 0;
}

__global__ void k_contact_row_list(const int *flag, const int *pos, int nv, int *rows) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nv && flag[i]) rows[pos[i]] = i;
}

__global__ void __launch_bounds__(64) k_contact_rows(const int *rows, const int *n_rows, const int *inc_off,
                                                     const int *inc_ent, const int4 *ce_v, const double *ce_H,
                                                     int *cr_key, int *cr_scol, int *cr_ssrc, int *cr_col, int *cr_cnt,
                                                     double *cr_val, float *cr_val32, int mixed) {
  if ((int)blockIdx.x >= *n_rows) return;
  const int i = rows[blockIdx.x];
  const int lane = threadIdx.x;
  const int b0 = inc_off[i], n = 4 * (inc_off[i + 1] - b0), base = 4 * b0;
  // columns of the expanded pairs
  for (int k = lane; k < n; k += 64) {
    const int4 q = ce_v[inc_ent[b0 + k / 4] >> 2];
    const int vv[4] = {q.x, q.y, q.z, q.w};
    cr_key[base + k] = vv[k & 3];
  }
  __syncthreads();
  // stable order by column: the rank of pair k
  for (int k = lane; k < n; k += 64) {
    const int c = cr_key[base + k];
    int r = 0;
    for (int m = 0; m < n; ++m) {
      const int cm = cr_key[base + m];
      r += (cm < c || (cm == c && m < k)) ? 1 : 0;
    }
    cr_scol[base + r] = c;
    cr_ssrc[base + r] = k;
  }
  __syncthreads();
  // runs of equal columns: the first pair of each run sums the run's blocks
  int heads = 0;
  for (int k0 = 0; k0 < n; k0 += 64) {  // same trip count in every lane
    const int k = k0 + lane;
    const bool head = k < n && (k == 0 || cr_scol[base + k] != cr_scol[base + k - 1]);
    const unsigned long long mask = __ballot(head);
    if (head) {
      const int out = heads + __builtin_popcountll(mask & ((1ull << lane) - 1ull));
      const int c = cr_scol[base + k];
      double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (int m = k; m < n && cr_scol[base + m] == c; ++m) {
        const int src = cr_ssrc[base + m];
        const int ent = inc_ent[b0 + src / 4];
        const int a = ent & 3, bb = src & 3;
        const double *B = ce_H + 90 * (size_t)(ent >> 2) + 9 * (a <= bb ? blk_index(a, bb) : blk_index(bb, a));
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) acc[3 * r + cc] += (a <= bb) ? B[3 * r + cc] : B[3 * cc + r];
      }
      cr_col[base + out] = c;
      for (int r = 0; r < 9; ++r) cr_val[9 * (size_t)(base + out) + r] = acc[r];
      if (mixed)
        for (int r = 0; r < 9; ++r) cr_val32[9 * (size_t)(base + out) + r] = (float)acc[r];
    }
    heads += __builtin_popcountll(mask);
  }
  if (lane == 0) cr_cnt[i] = heads;
}

// ---------------------------------------------------------------------------
// elasticity per tet: gradient (12) and projected Hessian blocks (10 x 9)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_elastic(WorldDev W, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  int e = t.start + threadIdx.x;
  int4 q = W.tet[e];
  int v[4] = {q.x, q.y, q.z, q.w};
  double x[12], g[12], en;
  gather12(W.x, v, x);
  // the Hessian blocks are written straight to their place
  double *blocks = W.tH + 90 * (size_t)e;
  const bool ok = nh_element(x, W.Dinv + 9 * e, W.vol[e], W.mu[e], W.la[e], &en, g, blocks);
  if (!ok) {
    for (int i = 0; i < 12; ++i) g[i] = __builtin_nan("");
    for (int i = 0; i < 90; ++i) blocks[i] = 0.0;
  }
  for (int i = 0; i < 12; ++i) W.tg[12 * (size_t)e + i] = g[i];
}

// ---------------------------------------------------------------------------
// assembly: gradient, block-Jacobi preconditioner, sliced-ELL values
// ---------------------------------------------------------------------------
DEV void add_block(double *D, const double *B, bool tr) {
  if (!tr)
    for (int r = 0; r < 9; ++r) D[r] += B[r];
  else
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) D[3 * r + c] += B[3 * c + r];
}

__global__ void k_assemble_rows(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, const int *inc_off,
                                const int *inc_ent, const double *ce_g, const double *ce_H, int mixed) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  const EnvDev &E = envs[t.env];
  int i = t.start + threadIdx.x;
  int k = W.kin[i];
  double g[3] = {0, 0, 0};
  double D[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Mi[9];
  if (is_dof(W, S, i, t.env)) {
    if (k == KIN_FREE) {  // inertia
      double w = W.mass[i] / (E.dt * E.dt);
      for (int c = 0; c < 3; ++c) g[c] = w * (W.x[3 * i + c] - W.xh[3 * i + c]);
      for (int r = 0; r < 9; ++r) D[r] = (r % 4 == 0) ? w : 0.0;
    } else {  // AL penalty kA w/2 |x - xbar|^2 - sqrt(w) lam.(x - xbar), w = mbar/dt^2
      double w0 = E.mbar / (E.dt * E.dt), w = S.kA[t.env] * w0, sw = sqrt(w0);
      for (int c = 0; c < 3; ++c) g[c] = w * (W.x[3 * i + c] - W.xh[3 * i + c]) - sw * W.lam[3 * i + c];
      for (int r = 0; r < 9; ++r) D[r] = (r % 4 == 0) ? w : 0.0;
    }
    for (int j = W.vt_beg[i]; j < W.vt_end[i]; ++j) {
      int ent = W.vt_ent[j];
      int te = ent >> 2, a = ent & 3;
      for (int c = 0; c < 3; ++c) g[c] += W.tg[12 * (size_t)te + 3 * a + c];
      add_block(D, W.tH + 90 * (size_t)te + 9 * blk_index(a, a), false);
    }
    for (int j = inc_off[i]; j < inc_off[i + 1]; ++j) {
      int ent = inc_ent[j];
      int ce = ent >> 2, a = ent & 3;
      for (int c = 0; c < 3; ++c) g[c] += ce_g[12 * (size_t)ce + 3 * a + c];
      add_block(D, ce_H + 90 * (size_t)ce + 9 * blk_index(a, a), false);
    }
    inv33(D, Mi);
  } else {
    for (int r = 0; r < 9; ++r) Mi[r] = D[r];
  }
  for (int c = 0; c < 3; ++c) W.g[3 * i + c] = g[c];
  for (int r = 0; r < 9; ++r) W.Minv[9 * (size_t)i + r] = Mi[r];
  if (mixed)
    for (int r = 0; r < 9; ++r) W.Minv32[9 * (size_t)i + r] = (float)Mi[r];
}

__global__ void k_assemble_sell(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, int mixed) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  const EnvDev &E = envs[t.env];
  int i = t.start + threadIdx.x;
  int sl = i / kSlice, lane = i % kSlice;
  int base = W.slice_pos[sl], wdt = W.slice_w[sl];
  int kr = W.kin[i];
  bool rdof = is_dof(W, S, i, t.env);
  double w = (kr == KIN_FREE) ? W.mass[i] / (E.dt * E.dt)
                              : (rdof ? S.kA[t.env] * E.mbar / (E.dt * E.dt) : 0.0);
  for (int k = 0; k < wdt; ++k) {
    int pos = base + k * kSlice + lane;
    int col = W.col[pos];
    double B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (!rdof) {
      if (k == 0)
        for (int r = 0; r < 9; ++r) B[r] = (r % 4 == 0) ? 1.0 : 0.0;
    } else if (is_dof(W, S, col, t.env)) {
      for (int j = W.cb_beg[pos]; j < W.cb_end[pos]; ++j) {
        int c = W.contrib[j];
        int te = c >> 5, bi = (c >> 1) & 15, tr = c & 1;
        add_block(B, W.tH + 90 * (size_t)te + 9 * bi, tr != 0);
      }
      if (k == 0)
        for (int r = 0; r < 3; ++r) B[4 * r] += w;
    }
    size_t vb = (size_t)(pos / kSlice) * (9 * kSlice) + lane;
    for (int r = 0; r < 9; ++r) W.val[vb + r * kSlice] = B[r];
    if (mixed)
      for (int r = 0; r < 9; ++r) W.val32[vb + r * kSlice] = (float)B[r];
  }
}

// ---------------------------------------------------------------------------
// block-Jacobi PCG, one independent solve per environment
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Two-level PCG.  The coarse space spans the rigid motions of each body of an
// environment (its connected sets of free vertices): for a free vertex i of
// body b, Z_i = [I | R_i] with R_i = -[d_i]x / s_b, d_i = x_i - cb_b (cb_b a
// reference point, s_b the body's size, so that the six columns have like
// magnitudes); Z_i = 0 for every other row.  The preconditioner is
//   M^-1 r = D^-1 r + Z E^-1 Z^T r,  E = Z^T H Z
// (block Jacobi plus an exact solve on the coarse space).  Z_i [t; w] =
// t + (w x d_i) / s_b and Z_i^T r = [r; (d_i x r) / s_b].
// ---------------------------------------------------------------------------
// tiles whose Z^T r partials a 1024-thread product stages in LDS at once
constexpr int kZChunk = 1024 / kCoarseM;
// position of entry k (of 3 kCoarseM) of (H Z)_i in the sliced layout: the
// 64 rows of a slice side by side for each entry
DEV size_t hz_index(int i, int k) {
  return ((size_t)(i / kSlice) * (3 * kCoarseM) + k) * kSlice + (size_t)(i % kSlice);
}
// coarse correction (Z c)_i of a row at position xi in body b; c holds
// (t, w) per body.  The one routine every kernel uses for it (same bits).
DEV void coarse_corr_x(const EnvDev &E, int b, const double xi[3], const double *c, double out[3]) {
  const double is = 1.0 / E.cscale[b];
  const double d0 = xi[0] - E.cb[b][0], d1 = xi[1] - E.cb[b][1], d2 = xi[2] - E.cb[b][2];
  const double *t = c + 6 * b, *w = c + 6 * b + 3;
  out[0] = t[0] + (w[1] * d2 - w[2] * d1) * is;
  out[1] = t[1] + (w[2] * d0 - w[0] * d2) * is;
  out[2] = t[2] + (w[0] * d1 - w[1] * d0) * is;
}
DEV void coarse_corr(const EnvDev &E, int b, const double *x, int i, const double *c, double out[3]) {
  const double xi[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
  coarse_corr_x(E, b, xi, c, out);
}
// Z_i^T r of a row at position xi in body b (six values)
DEV void coarse_zt_x(const EnvDev &E, int b, const double xi[3], const double r[3], double q[6]) {
  const double is = 1.0 / E.cscale[b];
  const double d0 = xi[0] - E.cb[b][0], d1 = xi[1] - E.cb[b][1], d2 = xi[2] - E.cb[b][2];
  q[0] = r[0];
  q[1] = r[1];
  q[2] = r[2];
  q[3] = (d1 * r[2] - d2 * r[1]) * is;
  q[4] = (d2 * r[0] - d0 * r[2]) * is;
  q[5] = (d0 * r[1] - d1 * r[0]) * is;
}

// sums of v[0..N) over the 256 threads of a tile (one row each): the
// butterfly over each wavefront, then the four wavefront sums as
// (w0 + w1) + (w2 + w3); thread k < N gets sum k (others 0).  Every thread of
// the block calls it.  sh: 4 * N doubles.
template <int N>
DEV double tile_sums(double v[N], double *sh) {
#pragma unroll
  for (int k = 0; k < N; ++k)
    for (int m = 32; m > 0; m >>= 1) v[k] += __shfl_xor(v[k], m, 64);
  const int wv = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0 && wv < 4)
#pragma unroll
    for (int k = 0; k < N; ++k) sh[wv * N + k] = v[k];
  __syncthreads();
  double out = 0.0;
  if ((int)threadIdx.x < N) {
    const int k = threadIdx.x;
    out = (sh[k] + sh[N + k]) + (sh[2 * N + k] + sh[3 * N + k]);
  }
  __syncthreads();
  return out;
}

// sums of v[0..8) over the 256 threads of a tile (one row each): a
// transposed butterfly over each wavefront (at the exchanges 32, 16 and 8
// each lane keeps half of its values, adds its partner's copies of them and
// hands over the other half; the one value left goes through the exchanges
// 4, 2, 1), then the four wavefront sums as (w0 + w1) + (w2 + w3).  Thread
// k < 8 gets sum k (others 0).  10 exchanges instead of the full butterfly's
// 48.  Every thread of the block calls it.  sh: 32 doubles.
DEV double tile_sums8(const double v[8], double *sh) {
  const int ln = threadIdx.x & 63;
  const bool h32 = ln & 32, h16 = ln & 16, h8 = ln & 8;
  double a[4], b[2];
#pragma unroll
  for (int j = 0; j < 4; ++j) a[j] = (h32 ? v[j + 4] : v[j]) + __shfl_xor(h32 ? v[j] : v[j + 4], 32, 64);
#pragma unroll
  for (int j = 0; j < 2; ++j) b[j] = (h16 ? a[j + 2] : a[j]) + __shfl_xor(h16 ? a[j] : a[j + 2], 16, 64);
  double c = (h8 ? b[1] : b[0]) + __shfl_xor(h8 ? b[0] : b[1], 8, 64);
  for (int m = 4; m > 0; m >>= 1) c += __shfl_xor(c, m, 64);
  const int wv = threadIdx.x / 64;
  if ((ln & 7) == 0) sh[wv * 8 + (h32 ? 4 : 0) + (h16 ? 2 : 0) + (h8 ? 1 : 0)] = c;
  __syncthreads();
  double out = 0.0;
  if (threadIdx.x < 8) {
    const int k = threadIdx.x;
    out = (sh[k] + sh[8 + k]) + (sh[16 + k] + sh[24 + k]);
  }
  __syncthreads();
  return out;
}

// sums of v[0..P) over the 256 threads of a tile (one row each), P = 8, 16,
// 32 or 64: the transposed butterfly of tile_sums8 with log2 P halving
// exchanges (32, 16, ...) and the full butterfly over the exchanges left,
// then the four wavefront sums as (w0 + w1) + (w2 + w3).  Thread k < P gets
// sum k (others 0).  Every thread of the block calls it.  sh: 4 P doubles.
template <int P>
DEV double tile_sums_tr(const double v[P], double *sh) {
  static_assert(P == 8 || P == 16 || P == 32 || P == 64, "P");
  const int ln = threadIdx.x & 63;
  double a[P];
#pragma unroll
  for (int k = 0; k < P; ++k) a[k] = v[k];
  int idx = 0;
#pragma unroll
  for (int m = 32, h = P / 2; h >= 1; m >>= 1, h >>= 1) {
    const bool hi = ln & m;
#pragma unroll
    for (int j = 0; j < h; ++j) a[j] = (hi ? a[j + h] : a[j]) + __shfl_xor(hi ? a[j] : a[j + h], m, 64);
    idx += hi ? h : 0;
  }
  constexpr int group = 64 / P;  // lanes left holding the same value
#pragma unroll
  for (int m = group / 2; m > 0; m >>= 1) a[0] += __shfl_xor(a[0], m, 64);
  const int wv = threadIdx.x / 64;
  if (ln % group == 0) sh[wv * P + idx] = a[0];
  __syncthreads();
  double out = 0.0;
  if ((int)threadIdx.x < P) {
    const int k = threadIdx.x;
    out = (sh[k] + sh[P + k]) + (sh[2 * P + k] + sh[3 * P + k]);
  }
  __syncthreads();
  return out;
}

// the vector a product reads: stored, or the next direction formed on the fly
template <typename T>
struct StoredVec {
  const T *v;
  DEV double operator[](int k) const { return (double)v[k]; }
};

// One row of the matrix-vector product by kLPR = 4 lanes: lane l takes the
// sliced-ELL slots l, l+4, ... and the row's merged contact blocks l, l+4, ...
// (the four lanes' loads are in flight together); the four lane sums
// are combined by two xor exchanges, which leaves the same bits in all four
// lanes.  Every lane of the group must call it (invalid rows pass valid =
// false and contribute zeros).
constexpr int kLPR = 4;

// one slot of a row: a += B x_c (B = the 3x3 block at b, components kSlice apart)
template <typename T, typename V>
DEV void slot_acc(const T *b, const V &v, int c, double &a0, double &a1, double &a2) {
  const double x0 = v[3 * c], x1 = v[3 * c + 1], x2 = v[3 * c + 2];
  a0 += (double)b[0] * x0 + (double)b[kSlice] * x1 + (double)b[2 * kSlice] * x2;
  a1 += (double)b[3 * kSlice] * x0 + (double)b[4 * kSlice] * x1 + (double)b[5 * kSlice] * x2;
  a2 += (double)b[6 * kSlice] * x0 + (double)b[7 * kSlice] * x1 + (double)b[8 * kSlice] * x2;
}

// one contact block of a row: a += B x_c (B row-major, 9 contiguous values)
template <typename T, typename V>
DEV void block_acc(const T *b, const V &v, int c, double &a0, double &a1, double &a2) {
  const double x0 = v[3 * c], x1 = v[3 * c + 1], x2 = v[3 * c + 2];
  a0 += (double)b[0] * x0 + (double)b[1] * x1 + (double)b[2] * x2;
  a1 += (double)b[3] * x0 + (double)b[4] * x1 + (double)b[5] * x2;
  a2 += (double)b[6] * x0 + (double)b[7] * x1 + (double)b[8] * x2;
}

// Where a row's stored blocks are: its slice's offset and width in the
// sliced-ELL arrays, and the offset and count of its merged contact blocks.
// Loaded apart from the product so that kernels can issue these loads with
// their other first loads.
struct RowHead {
  int base, wdt, cb, cn;
};
DEV RowHead row_head(const WorldDev &W, int i, const int *inc_off, const int *cr_cnt) {
  const int sl = i / kSlice;
  return {W.slice_pos[sl], W.slice_w[sl], 4 * inc_off[i], cr_cnt[i]};
}

// WIDE: the lane's slots are processed four per round (their loads in
// flight together: fewer round trips, for launches of a few tiles where
// latency dominates), and the columns of its first four contact blocks are
// loaded with the first slots; otherwise one per round (fewer registers,
// more waves for launches over the whole batch).  Same additions in the
// same order.
template <typename T, typename V, bool WIDE>
DEV void row_product(const WorldDev &W, int i, bool valid, int l, const RowHead &h, const V &v, const T *val,
                     const int *cr_col, const T *cr_val, double y[3]) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (valid) {
    const int lane = i % kSlice;
    const int *colp = W.col + h.base + lane;
    const T *vp = val + (size_t)(h.base / kSlice) * (9 * kSlice) + lane;
    int k = l, j = l;
    if (WIDE) {
      int cc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cc[u] = l + u * kLPR < h.cn ? cr_col[h.cb + l + u * kLPR] : 0;
      for (; k + 3 * kLPR < h.wdt; k += 4 * kLPR) {
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = colp[(k + u * kLPR) * kSlice];
#pragma unroll
        for (int u = 0; u < 4; ++u) slot_acc<T>(vp + (size_t)(k + u * kLPR) * (9 * kSlice), v, c[u], a0, a1, a2);
      }
#pragma unroll 1
      for (; k < h.wdt; k += kLPR) slot_acc<T>(vp + (size_t)k * (9 * kSlice), v, colp[k * kSlice], a0, a1, a2);
      // contact blocks of the row, merged by column (k_contact_rows): the
      // first four from the columns loaded above, then four per round
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (j + u * kLPR < h.cn) block_acc<T>(cr_val + 9 * (size_t)(h.cb + j + u * kLPR), v, cc[u], a0, a1, a2);
      j += 4 * kLPR;
      for (; j + 3 * kLPR < h.cn; j += 4 * kLPR) {
        int c[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) c[u] = cr_col[h.cb + j + u * kLPR];
#pragma unroll
        for (int u = 0; u < 4; ++u) block_acc<T>(cr_val + 9 * (size_t)(h.cb + j + u * kLPR), v, c[u], a0, a1, a2);
      }
    } else {
#pragma unroll 1
      for (; k < h.wdt; k += kLPR) slot_acc<T>(vp + (size_t)k * (9 * kSlice), v, colp[k * kSlice], a0, a1, a2);
    }
    // contact blocks of the row, merged by column (k_contact_rows)
#pragma unroll 1
    for (; j < h.cn; j += kLPR) block_acc<T>(cr_val + 9 * (size_t)(h.cb + j), v, cr_col[h.cb + j], a0, a1, a2);
  }
  a0 += __shfl_xor(a0, 1, 64);
  a1 += __shfl_xor(a1, 1, 64);
  a2 += __shfl_xor(a2, 1, 64);
  a0 += __shfl_xor(a0, 2, 64);
  a1 += __shfl_xor(a1, 2, 64);
  a2 += __shfl_xor(a2, 2, 64);
  y[0] = a0;
  y[1] = a1;
  y[2] = a2;
}

// Fixed-order sums of the PCG (the tiled and the per-environment kernels use
// the same ones, so both give the same bits).  A butterfly over the lanes of
// a wavefront leaves the same bits in every lane: each step adds the same two
// operands, only their order differs.
//
// quarter_sum2: a and b summed over each 256-thread quarter of the block (a
// whole 256-thread block, or one tile's quarter of a 1024-thread block): the
// butterfly over each wavefront, then the quarter's four wavefront sums as
// (w0 + w1) + (w2 + w3); every thread gets its quarter's sums.  sh: 32 doubles.
DEV void quarter_sum2(double &a, double &b, double *sh) {
  for (int m = 32; m > 0; m >>= 1) {
    a += __shfl_xor(a, m, 64);
    b += __shfl_xor(b, m, 64);
  }
  const int wv = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    sh[wv] = a;
    sh[16 + wv] = b;
  }
  __syncthreads();
  const int q = wv & ~3;
  a = (sh[q] + sh[q + 1]) + (sh[q + 2] + sh[q + 3]);
  b = (sh[16 + q] + sh[17 + q]) + (sh[18 + q] + sh[19 + q]);
  __syncthreads();
}

// rows_sum: the sum over the 256 rows of a tile in a 1024-thread block with
// kLPR lanes per row, every lane of a row holding the row's value: the
// butterfly over the 16 rows of each wavefront, then the 16 wavefront sums
// pairwise; every thread gets it.  sh: 16 doubles.
DEV double rows_sum(double v, double *sh) {
  for (int m = 32; m >= kLPR; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = v;
  __syncthreads();
  double t[8];
  for (int k = 0; k < 8; ++k) t[k] = sh[2 * k] + sh[2 * k + 1];
  for (int k = 0; k < 4; ++k) t[k] = t[2 * k] + t[2 * k + 1];
  const double r = (t[0] + t[1]) + (t[2] + t[3]);
  __syncthreads();
  return r;
}

// env_sums3: the per-tile partials pa, pb, pc of one environment summed in
// tile order (the additions of env_tiles_sum), with up to 256 partials of
// each loaded at once by the block's first 256 threads and added up from LDS
// by every thread.  sh: 768 doubles; every thread of the block calls it.
DEV void env_sums3(const double *pa, const double *pb, const double *pc, const EnvDev &E, double *sh, double &a,
                   double &b, double &c) {
  a = 0.0;
  b = 0.0;
  c = 0.0;
  for (int base = 0; base < E.vtile_count; base += TB) {
    const int j = base + (int)threadIdx.x;
    if ((int)threadIdx.x < TB && j < E.vtile_count) {
      sh[threadIdx.x] = pa[E.vtile_first + j];
      sh[TB + threadIdx.x] = pb[E.vtile_first + j];
      sh[2 * TB + threadIdx.x] = pc[E.vtile_first + j];
    }
    __syncthreads();
    const int n = min(TB, E.vtile_count - base);
    for (int k = 0; k < n; ++k) {
      a += sh[k];
      b += sh[TB + k];
      c += sh[2 * TB + k];
    }
    __syncthreads();
  }
}

DEV bool pcg_env_live(const EnvState &S, int env) { return S.status[env] == ST_ACTIVE && !S.pcg_done[env]; }

// slot of a vertex tile in the per-tile partial arrays: its index in the
// batch's full tile list (kernels may run over a compacted copy of the list)
DEV int tile_slot(const EnvDev *envs, const Tile &t) { return envs[t.env].vtile_first + t.rel; }

// ---------------------------------------------------------------------------
// Block-Jacobi PCG in the Chronopoulos-Gear form: alongside the direction p
// it updates s = H p, so that both dot products of an iteration (gamma = r.u
// and delta = w.u, with u = M r and w = H u) come from one product launch and
// one update launch.  Per iteration i:
//   beta = gamma_i / gamma_{i-1},  alpha = gamma_i / (delta_i - beta gamma_i / alpha_{i-1})
//   (beta = 0, alpha = gamma/delta at i = 0)
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,  u = M r
// Vectors: x in p (the solution), r, u in z, p in pp, s in q, w in w.
// The per-row pieces are shared by the tiled kernels (one 256-row tile per
// workgroup, two launches per iteration) and the per-environment kernels
// (one 1024-thread workgroup iterating a whole environment); both reduce dot
// products per 256-row tile with the same tree and then over the
// environment's tiles in order, and take the same scalar steps, so the two
// paths produce the same bits and where the tiled solve hands over to the
// per-environment kernel changes no result.
// ---------------------------------------------------------------------------
template <typename T>
DEV void row_init(const WorldDev &W, bool fr, int i, T *x, T *r, T *u, T *pp, T *q, const T *Minv, double &g,
                  double &rr) {
  T rv[3], uv[3];
  for (int c = 0; c < 3; ++c) rv[c] = fr ? (T)(-W.g[3 * i + c]) : (T)0;
  const T *M = Minv + 9 * (size_t)i;
  for (int c = 0; c < 3; ++c) uv[c] = fr ? M[3 * c] * rv[0] + M[3 * c + 1] * rv[1] + M[3 * c + 2] * rv[2] : (T)0;
  for (int c = 0; c < 3; ++c) {
    r[3 * i + c] = rv[c];
    u[3 * i + c] = uv[c];
    pp[3 * i + c] = (T)0;
    q[3 * i + c] = (T)0;
    x[3 * i + c] = (T)0;
    g += (double)rv[c] * (double)uv[c];
    rr += (double)rv[c] * (double)rv[c];
  }
}

// w_i = (H u)_i by the row's 4 lanes; returns u_i . w_i (same in all four
// lanes, 0 for an invalid row)
template <typename T, bool WIDE, typename V>
DEV double row_spmv_v(const WorldDev &W, int i, bool valid, int l, const RowHead &h, const int *cr_col,
                      const T *cr_val, const V &v, T *w, const T *val) {
  double y[3];
  row_product<T, V, WIDE>(W, i, valid, l, h, v, val, cr_col, cr_val, y);
  if (!valid) return 0.0;
  double d = 0.0;
  for (int c = 0; c < 3; ++c) {
    if (l == c) w[3 * i + c] = (T)y[c];
    d += v[3 * i + c] * (double)(T)y[c];
  }
  return d;
}
template <typename T, bool WIDE>
DEV double row_spmv(const WorldDev &W, int i, bool valid, int l, const RowHead &h, const int *cr_col,
                    const T *cr_val, const T *u, T *w, const T *val) {
  return row_spmv_v<T, WIDE>(W, i, valid, l, h, cr_col, cr_val, StoredVec<T>{u}, w, val);
}

// one row's vectors and preconditioner block, loaded ahead of the scalars
template <typename T>
struct RowVals {
  T x[3], r[3], u[3], p[3], s[3], w[3], M[9];
};
template <typename T>
DEV void row_load(int i, const T *x, const T *r, const T *u, const T *pp, const T *q, const T *w, const T *Minv,
                  RowVals<T> &v) {
  for (int c = 0; c < 3; ++c) {
    v.x[c] = x[3 * i + c];
    v.r[c] = r[3 * i + c];
    v.u[c] = u[3 * i + c];
    v.p[c] = pp[3 * i + c];
    v.s[c] = q[3 * i + c];
    v.w[c] = w[3 * i + c];
  }
  for (int k = 0; k < 9; ++k) v.M[k] = Minv[9 * (size_t)i + k];
}

// the update of one row; adds r.u and r.r of the new residual
// uc: the coarse correction of the row's preconditioned residual (zeros for
// block Jacobi alone): the direction is updated with u + uc
template <typename T>
DEV void row_step(int i, double alpha, double beta, const RowVals<T> &v, T *x, T *r, T *u, T *pp, T *q, double &g,
                  double &rr, const double uc[3], double rn[3]) {
  T rv[3], uv[3];
  for (int c = 0; c < 3; ++c) {
    const T pn = (T)fma(beta, (double)v.p[c], (double)v.u[c] + uc[c]);
    const T sn = (T)fma(beta, (double)v.s[c], (double)v.w[c]);
    pp[3 * i + c] = pn;
    q[3 * i + c] = sn;
    x[3 * i + c] = (T)((double)v.x[c] + alpha * (double)pn);
    rv[c] = (T)((double)v.r[c] - alpha * (double)sn);
    r[3 * i + c] = rv[c];
  }
  for (int c = 0; c < 3; ++c) uv[c] = v.M[3 * c] * rv[0] + v.M[3 * c + 1] * rv[1] + v.M[3 * c + 2] * rv[2];
  for (int c = 0; c < 3; ++c) {
    u[3 * i + c] = uv[c];
    g += (double)rv[c] * (double)uv[c];
    rr += (double)rv[c] * (double)rv[c];
    rn[c] = (double)rv[c];
  }
}

// Scalars of iteration `it` from the environment's sums (gamma, delta, r.r)
// and the previous iteration's alpha and gamma; returns 1 if the solve stops:
// relative residual reached, non-finite values, the cap of 30 n_v + 10
// iterations, or a non-positive curvature.
DEV int cg_step(const EnvDev &E, double bb, int it, double gam, double del, double rr, double a_prev, double g_prev,
                double &alpha, double &beta) {
  if (rr <= E.pcg_tol * E.pcg_tol * bb || !(rr == rr) || it >= 30 * E.nv + 10 || !(gam > 0.0)) return 1;
  beta = it == 0 ? 0.0 : gam / g_prev;
  const double den = it == 0 ? del : del - beta * gam / a_prev;
  if (!(den > 0.0)) return 1;
  alpha = gam / den;
  return 0;
}

// per-tile Z^T r of the rows' residual rv (row in body bi at xi; bi < 0 for
// rows outside the bodies): per body, the butterfly of its six values over
// each wavefront, then the four wavefront sums as (w0 + w1) + (w2 + w3):
// part_z[slot * kCoarseM + 6 b + k].  Every thread of the 256-thread block
// calls it.  sh: 4 * kCoarseM doubles.
DEV void tile_zt(const EnvDev &E, int bi, const double xi[3], const double rv[3], double *sh, double *out) {
  double q[6] = {0, 0, 0, 0, 0, 0};
  if (bi >= 0) coarse_zt_x(E, bi, xi, rv, q);
  const int wv = threadIdx.x / 64;
  for (int b = 0; b < E.nbody; ++b) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double v = (bi == b) ? q[k] : 0.0;
      for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
      if ((threadIdx.x & 63) == 0) sh[wv * kCoarseM + 6 * b + k] = v;
    }
  }
  __syncthreads();
  const int n = 6 * E.nbody;
  if ((int)threadIdx.x < n) {
    const int k = threadIdx.x;
    out[k] = (sh[k] + sh[kCoarseM + k]) + (sh[2 * kCoarseM + k] + sh[3 * kCoarseM + k]);
  }
}

template <typename T>
__global__ void k_pcg_init(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, T *x, T *r, T *u, T *pp,
                           T *q, const T *Minv, double *part_g, double *part_rr, double *part_z, int coarse) {
  __shared__ double sh[4 * kCoarseM];
  Tile t = tiles[blockIdx.x];
  if (!active_env(S, t.env) || envs[t.env].fused) return;
  int i = t.start + threadIdx.x;
  const bool mine = (int)threadIdx.x < t.count;
  double g = 0.0, rr = 0.0;
  if (mine) row_init<T>(W, is_dof(W, S, i, t.env), i, x, r, u, pp, q, Minv, g, rr);
  quarter_sum2(g, rr, sh);
  if (threadIdx.x == 0) {
    part_g[tile_slot(envs, t)] = g;
    part_rr[tile_slot(envs, t)] = rr;
  }
  const EnvDev &E = envs[t.env];
  if (coarse && E.nbody > 0) {
    const int bi = mine ? W.vbody[i] : -1;
    double xi[3] = {0.0, 0.0, 0.0}, rv[3] = {0.0, 0.0, 0.0};
    if (bi >= 0)
      for (int c = 0; c < 3; ++c) {
        xi[c] = W.x[3 * (size_t)i + c];
        rv[c] = (double)r[3 * (size_t)i + c];
      }
    tile_zt(E, bi, xi, rv, sh, part_z + (size_t)tile_slot(envs, t) * kCoarseM);
  }
}

__global__ void k_pcg_env_init(const EnvDev *envs, EnvState S, const int *benv, int n, const double *part_rr,
                               int *pending) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (envs[e].fused) return;  // solved by the fused kernel
  S.pcg_it[e] = 0;
  if (S.status[e] != ST_ACTIVE) {
    S.pcg_done[e] = 1;
    return;
  }
  double bb = env_tiles_sum(part_rr, envs[e]);
  S.pcg_bb[e] = bb;
  if (bb == 0.0 || !(bb == bb)) {
    S.pcg_done[e] = 1;
    return;
  }
  S.pcg_done[e] = 0;
  atomicAdd(pending, 1);
}

// w = H u for live environments, partial u.w (delta) per tile
// CO: the two-level PCG is on (environments with a coarse factor take u + Z c)
template <typename T, bool WIDE, bool CO>
__global__ void __launch_bounds__(1024) k_spmv(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles,
                                               const int *inc_off, const int *cr_cnt, const int *cr_col,
                                               const T *cr_val, const T *u, T *w, const T *val, double *part_d,
                                               const double *part_z) {
  __shared__ double sh[16];
  // two-level PCG: the tiles' Z^T r (kZChunk tiles), E^-1, Z^T r and c
  __shared__ double zs[CO ? kZChunk * kCoarseM : 1], es[CO ? kCoarseM * kCoarseM : 1];
  __shared__ double zq[CO ? kCoarseM : 1], zc[CO ? kCoarseM : 1];
  Tile t = tiles[blockIdx.x];
  const int row = threadIdx.x / kLPR, l = threadIdx.x % kLPR;
  const int i = t.start + row;
  const bool valid = row < t.count;
  // the row's head (row t.start for lanes past the tile's rows) is loaded
  // together with the environment's state; the empty asm keeps the compiler
  // from moving these loads after the test
  int st = S.status[t.env], dn = S.pcg_done[t.env];
  RowHead h = row_head(W, valid ? i : t.start, inc_off, cr_cnt);
  asm volatile("" : "+v"(h.base), "+v"(h.wdt), "+v"(h.cb), "+v"(h.cn), "+v"(st), "+v"(dn));
  if (st != ST_ACTIVE || dn) return;
  const EnvDev &E = envs[t.env];
  double d;
  if (CO && E.nbody > 0 && S.cok[t.env]) {
    // c = E^-1 Z^T r from the tiles' Z^T r (tile order), then w = H u +
    // (H Z) c at this row (H Z stored by k_coarse_hz; lane l < 3 takes
    // component l, exchanged among the row's lanes) and delta with u + Z c.
    // The tiles' Z^T r, E^-1, the row's body and its H Z entries of the
    // first body are loaded ahead of the product and used after it.
    const int m = 6 * E.nbody;
    const int nz = min(E.vtile_count, kZChunk);
    const int tz = threadIdx.x / kCoarseM, jz = threadIdx.x % kCoarseM;
    const double pz = (tz < nz && jz < m) ? part_z[(size_t)(E.vtile_first + tz) * kCoarseM + jz] : 0.0;
    const double pe =
        (int)threadIdx.x < m * kCoarseM ? S.cinv[(size_t)t.env * (kCoarseM * kCoarseM) + threadIdx.x] : 0.0;
    const int ri = valid ? i : t.start;
    const int b = W.vbody[ri];
    const T *hzp = (sizeof(T) == 4 ? (const T *)(const void *)W.hz32 : (const T *)(const void *)W.hz) +
                   hz_index(ri, (l < 3 ? l : 0) * kCoarseM);
    T hz0[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) hz0[k] = hzp[(size_t)k * kSlice];
    double y[3];
    row_product<T, StoredVec<T>, WIDE>(W, i, valid, l, h, StoredVec<T>{u}, val, cr_col, cr_val, y);
    if (tz < kZChunk) zs[threadIdx.x] = pz;
    if ((int)threadIdx.x < kCoarseM * kCoarseM) es[threadIdx.x] = pe;
    __syncthreads();
    if ((int)threadIdx.x < m) {
      double q = 0.0;
      for (int k = 0; k < nz; ++k) q += zs[k * kCoarseM + threadIdx.x];
      for (int k = nz; k < E.vtile_count; ++k) q += part_z[(size_t)(E.vtile_first + k) * kCoarseM + threadIdx.x];
      zq[threadIdx.x] = q;
    }
    __syncthreads();
    if ((int)threadIdx.x < m) {
      double c = 0.0;
      for (int j = 0; j < m; ++j) c += es[threadIdx.x * kCoarseM + j] * zq[j];
      zc[threadIdx.x] = c;
      if (t.rel == 0) S.cc[(size_t)t.env * kCoarseM + threadIdx.x] = c;
    }
    __syncthreads();
    if (t.rel == 0 && threadIdx.x == 0) {
      double gz = 0.0;
      for (int j = 0; j < m; ++j) gz += zq[j] * zc[j];
      S.cgam[t.env] = gz;
    }
    double hc = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) hc += (double)hz0[k] * zc[k];
    for (int k = 6; k < m; ++k) hc += (double)hzp[(size_t)k * kSlice] * zc[k];
    const int base = threadIdx.x & 63 & ~3;
    const double h0 = __shfl(hc, base, 64), h1 = __shfl(hc, base + 1, 64), h2 = __shfl(hc, base + 2, 64);
    d = 0.0;
    if (valid) {
      double uf[3] = {(double)u[3 * i], (double)u[3 * i + 1], (double)u[3 * i + 2]};
      if (b >= 0) {
        double o[3];
        coarse_corr(E, b, W.x, i, zc, o);
        for (int c = 0; c < 3; ++c) uf[c] = uf[c] + o[c];
      }
      const double hcc[3] = {h0, h1, h2};
      for (int c = 0; c < 3; ++c) {
        const double yc = y[c] + hcc[c];
        if (l == c) w[3 * i + c] = (T)yc;
        d += uf[c] * (double)(T)yc;
      }
    }
  } else {
    d = row_spmv<T, WIDE>(W, i, valid, l, h, cr_col, cr_val, u, w, val);
  }
  d = rows_sum(d, sh);
  if (threadIdx.x == 0) part_d[tile_slot(envs, t)] = d;
}

// Algorithmic bytes of a PCG iteration over the listed tiles, counted by a
// launch of its own right after the product (outside its timing, before the
// update changes which environments iterate): *spmv += the product's
// (stored 3x3 blocks and column indices of the sliced ELL and the merged
// contact blocks, one read of u and one write of w per row), *iter += the
// whole iteration's: the product's blocks plus per row the preconditioner
// block and eight vector accesses of three values, N (9 s + 4) + n 9 s +
// 24 n s for N blocks, n rows, s bytes per value.  With the two-level PCG
// (m = 6 bodies) the product also reads per row its 3 m entries of H Z and
// its body (3 m s + 4) and per row of a body its position (24); the update
// reads body and position again (4 + 24) and writes m partials per tile (8 m).
template <typename T>
__global__ void k_pcg_bytes(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, const int *cr_cnt,
                            int coarse, unsigned long long *spmv, unsigned long long *iter) {
  __shared__ double sh[2 * TB];
  Tile t = tiles[blockIdx.x];
  if (S.status[t.env] != ST_ACTIVE || S.pcg_done[t.env]) return;
  const int m = coarse && S.cok[t.env] ? 6 * envs[t.env].nbody : 0;
  double b = 0.0, c = threadIdx.x == 0 ? 8.0 * m : 0.0;
  if ((int)threadIdx.x < t.count) {
    const int i = t.start + threadIdx.x;
    const double blk = (double)(W.row_nnz[i] + cr_cnt[i]) * (9.0 * sizeof(T) + 4.0);
    b = blk + 6.0 * sizeof(T);
    c += blk + 9.0 * sizeof(T) + 24.0 * sizeof(T);
    if (m) {
      const double pos = W.vbody[i] >= 0 ? 24.0 : 0.0;
      b += 3.0 * m * sizeof(T) + 4.0 + pos;
      c += 3.0 * m * sizeof(T) + 8.0 + 2.0 * pos;
    }
  }
  sh[threadIdx.x] = b;
  sh[TB + threadIdx.x] = c;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[threadIdx.x] += sh[threadIdx.x + w];
      sh[TB + threadIdx.x] += sh[TB + threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(spmv, (unsigned long long)sh[0]);
    atomicAdd(iter, (unsigned long long)sh[TB]);
  }
}

// Algorithmic bytes of one assembly pass (elasticity, inertia, gradient and
// the stored 3x3 blocks) over the environments still iterating: per tet its
// vertex ids, gathered positions, inverse rest shape, volume and Lame
// parameters (208 B); per row mass, position, predicted position and the
// gradient written (80 B); the N stored blocks written once (9 s each).
__global__ void k_asm_bytes(const EnvDev *envs, EnvState S, const int *benv, int n, int mixed,
                            unsigned long long *prof) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (S.status[e] != ST_ACTIVE) return;
  const EnvDev &E = envs[e];
  const double b = 208.0 * E.nt + 80.0 * E.nv + 9.0 * (mixed ? 4.0 : 8.0) * E.nnzb;
  atomicAdd(prof, (unsigned long long)b);
}

// Stopping test, scalars and the update of iteration `it` (the host's count:
// every live environment started its solve with the others).  The first tile
// of an environment keeps alpha and gamma for the next iteration (slot it&1;
// this launch reads slot (it-1)&1 only) and, when the solve stops, the
// bookkeeping.
template <typename T>
__global__ void k_pcg_update(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, int it,
                             const double *part_d, const double *part_g, const double *part_rr, double *part_g_new,
                             double *part_rr_new, T *x, T *r, T *u, T *pp, T *q, const T *w, const T *Minv,
                             int *pending, double *part_z, int coarse) {
  __shared__ double sh[3 * TB];
  __shared__ double s_ab[2];
  __shared__ int s_done;
  __shared__ double zc[kCoarseM];
  Tile t = tiles[blockIdx.x];
  // The row's vectors (row t.start for threads past the tile's rows) are
  // loaded together with the environment's state and are in flight while the
  // environment's sums are formed; an environment no longer iterating takes
  // the same path and stops at the test below, so that no branch stands
  // between these loads.
  const int i = t.start + threadIdx.x;
  const bool mine = (int)threadIdx.x < t.count;
  RowVals<T> v;
  row_load<T>(mine ? i : t.start, x, r, u, pp, q, w, Minv, v);
  const int st = S.status[t.env], dn = S.pcg_done[t.env];
  const bool live = st == ST_ACTIVE && !dn;
  const EnvDev &E = envs[t.env];
  // two-level PCG: the correction c of this iteration's u (stored by the
  // product), r.u's share (Z^T r).c, the row's body and position, loaded
  // with the rest
  double cgam = 0.0, cpre = 0.0, xi[3] = {0.0, 0.0, 0.0};
  int bi = -1;
  if (coarse) {
    cgam = S.cgam[t.env];
    if ((int)threadIdx.x < kCoarseM) cpre = S.cc[(size_t)t.env * kCoarseM + threadIdx.x];
    const int ri = mine ? i : t.start;
    bi = mine ? W.vbody[ri] : -1;
    for (int c = 0; c < 3; ++c) xi[c] = W.x[3 * (size_t)ri + c];
  }
  const bool co = coarse && E.nbody > 0 && S.cok[t.env];
  if (!co) bi = -1;
  double gam, del, rr;
  env_sums3(part_g, part_d, part_rr, E, sh, gam, del, rr);
  if (co) gam += cgam;
  if (co && (int)threadIdx.x < kCoarseM) zc[threadIdx.x] = cpre;  // read after the barrier below
  if (threadIdx.x == 0 && !live) s_done = 1;
  if (threadIdx.x == 0 && live) {
    const int e = t.env, k = (it + 1) & 1;  // slot of iteration it - 1
    double alpha = 0.0, beta = 0.0;
    s_done = cg_step(E, S.pcg_bb[e], it, gam, del, rr, k ? S.cg_a1[e] : S.cg_a0[e], k ? S.cg_g1[e] : S.cg_g0[e],
                     alpha, beta);
    s_ab[0] = alpha;
    s_ab[1] = beta;
    if (t.rel == 0) {
      if (s_done) {
        S.pcg_done[e] = 1;
        S.pcg_it[e] = it;
        S.pcg_total[e] += it;
        atomicSub(pending, 1);
      } else if (it & 1) {
        S.cg_a1[e] = alpha;
        S.cg_g1[e] = gam;
      } else {
        S.cg_a0[e] = alpha;
        S.cg_g0[e] = gam;
      }
    }
  }
  __syncthreads();
  if (s_done) return;
  double g = 0.0, rr2 = 0.0;
  double uc[3] = {0.0, 0.0, 0.0}, rn[3] = {0.0, 0.0, 0.0};
  if (bi >= 0) coarse_corr_x(E, bi, xi, zc, uc);
  if (mine) row_step<T>(i, s_ab[0], s_ab[1], v, x, r, u, pp, q, g, rr2, uc, rn);
  const int slot = tile_slot(envs, t);
  if (!co) {
    quarter_sum2(g, rr2, sh);
    if (threadIdx.x == 0) {
      part_g_new[slot] = g;
      part_rr_new[slot] = rr2;
    }
    return;
  }
  // two-level PCG: Z^T r of the new residual (six values per body) reduced
  // together with r.u and r.r in one pass of P = 8, 16 or 32 values
  double zr[6] = {0, 0, 0, 0, 0, 0};
  if (bi >= 0) coarse_zt_x(E, bi, xi, rn, zr);
  const int m = 6 * E.nbody;
  auto reduce = [&](auto tag) {
    constexpr int P = decltype(tag)::value;
    double vals[P];
#pragma unroll
    for (int k = 0; k < P; ++k) vals[k] = 0.0;
#pragma unroll
    for (int k = 0; k < P - 2; ++k) vals[k] = (bi >= 0 && k / 6 == bi) ? zr[k % 6] : 0.0;
    vals[P - 2] = g;
    vals[P - 1] = rr2;
    const double sum = tile_sums_tr<P>(vals, sh);
    if ((int)threadIdx.x < m) part_z[(size_t)slot * kCoarseM + threadIdx.x] = sum;
    if (threadIdx.x == P - 2) part_g_new[slot] = sum;
    if (threadIdx.x == P - 1) part_rr_new[slot] = sum;
  };
  if (m <= 6)
    reduce(std::integral_constant<int, 8>());
  else if (m <= 14)
    reduce(std::integral_constant<int, 16>());
  else
    reduce(std::integral_constant<int, 32>());
}

// ---------------------------------------------------------------------------
// Coarse matrix E = Z^T H Z of the two-level PCG, at the assembled H: per tile
// (one row per thread) and per column body bb, Y = (H Z)_i restricted to the
// columns of bb (3 x 6, over the row's sliced-ELL slots and merged contact
// blocks, FP64), then Z_i^T Y (6 x 6) summed over the tile's rows of each body
// b2 into e_tile[slot][6 b2 + r][6 bb + c].  Rows outside the bodies add zero.
// ---------------------------------------------------------------------------
DEV void coarse_block_acc(const double *B, int stride, const EnvDev &E, int b, const double *x, int j,
                          double Y[3][6]) {
  const double is = 1.0 / E.cscale[b];
  const double d[3] = {x[3 * j] - E.cb[b][0], x[3 * j + 1] - E.cb[b][1], x[3 * j + 2] - E.cb[b][2]};
  // columns of R_j = -[d]x / s: e_0 x d, e_1 x d, e_2 x d, over s
  const double R[3][3] = {{0.0, d[2] * is, -d[1] * is}, {-d[2] * is, 0.0, d[0] * is}, {d[1] * is, -d[0] * is, 0.0}};
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double b0 = B[(3 * r) * stride], b1 = B[(3 * r + 1) * stride], b2 = B[(3 * r + 2) * stride];
    Y[r][0] += b0;
    Y[r][1] += b1;
    Y[r][2] += b2;
#pragma unroll
    for (int c = 0; c < 3; ++c) Y[r][3 + c] += b0 * R[0][c] + b1 * R[1][c] + b2 * R[2][c];
  }
}

__global__ void __launch_bounds__(256) k_coarse_hz(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles,
                                                   const int *inc_off, const int *cr_cnt, const int *cr_col,
                                                   const double *cr_val, double *e_tile, int mixed) {
  __shared__ double sh[4 * 36];
  Tile t = tiles[blockIdx.x];
  const EnvDev &E = envs[t.env];
  if (!active_env(S, t.env) || E.nbody == 0) return;
  const int i = t.start + threadIdx.x;
  const bool mine = (int)threadIdx.x < t.count;
  const int bi = mine ? W.vbody[i] : -1;
  RowHead h{0, 0, 0, 0};
  if (mine) h = row_head(W, i, inc_off, cr_cnt);
  double di[3] = {0, 0, 0}, isi = 0.0;
  if (bi >= 0) {
    isi = 1.0 / E.cscale[bi];
    for (int k = 0; k < 3; ++k) di[k] = W.x[3 * i + k] - E.cb[bi][k];
  }
  double *out = e_tile + (size_t)tile_slot(envs, t) * (kCoarseM * kCoarseM);
  for (int bb = 0; bb < E.nbody; ++bb) {
    double Y[3][6] = {{0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}, {0, 0, 0, 0, 0, 0}};
    if (mine) {
      const int lane = i % kSlice;
      const double *vp = W.val + (size_t)(h.base / kSlice) * (9 * kSlice) + lane;
      for (int k = 0; k < h.wdt; ++k) {
        const int j = W.col[h.base + lane + k * kSlice];
        if (W.vbody[j] == bb) coarse_block_acc(vp + (size_t)k * (9 * kSlice), kSlice, E, bb, W.x, j, Y);
      }
      for (int k = 0; k < h.cn; ++k) {
        const int j = cr_col[h.cb + k];
        if (W.vbody[j] == bb) coarse_block_acc(cr_val + 9 * (size_t)(h.cb + k), 1, E, bb, W.x, j, Y);
      }
      // (H Z)_i for the product of the two-level PCG (every row: a dof row
      // outside the bodies may neighbour them)
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 6; ++c) {
          const size_t o = hz_index(i, r * kCoarseM + 6 * bb + c);
          W.hz[o] = Y[r][c];
          if (mixed) W.hz32[o] = (float)Y[r][c];
        }
    }
    // C = Z_i^T Y: the rows of Y, then (d_i x Y_c) / s for each column c
    double C[36];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double y0 = Y[0][c], y1 = Y[1][c], y2 = Y[2][c];
      C[c] = y0;
      C[6 + c] = y1;
      C[12 + c] = y2;
      C[18 + c] = (di[1] * y2 - di[2] * y1) * isi;
      C[24 + c] = (di[2] * y0 - di[0] * y2) * isi;
      C[30 + c] = (di[0] * y1 - di[1] * y0) * isi;
    }
    for (int b2 = 0; b2 < E.nbody; ++b2) {
      double v[36];
#pragma unroll
      for (int k = 0; k < 36; ++k) v[k] = (bi == b2) ? C[k] : 0.0;
      const double sum = tile_sums<36>(v, sh);
      if ((int)threadIdx.x < 36) {
        const int r = threadIdx.x / 6, c = threadIdx.x % 6;
        out[(6 * b2 + r) * kCoarseM + 6 * bb + c] = sum;
      }
    }
  }
}

// E from the tiles (tile order), symmetrised, Cholesky-factored and inverted
// (E^-1 = L^-T L^-1) in LDS by one 64-thread block per environment; cok = 0
// when a pivot is below 1e-10 of E's largest diagonal entry (the environment
// then runs block Jacobi alone)
__global__ void __launch_bounds__(64) k_coarse_factor(const EnvDev *envs, EnvState S, const int *benv,
                                                      const double *e_tile) {
  constexpr int M = kCoarseM;
  __shared__ double A[M * M], Li[M * M];
  __shared__ int bad;
  __shared__ double tiny;
  const int e = benv[blockIdx.x];
  const EnvDev &E = envs[e];
  const int m = 6 * E.nbody, tid = threadIdx.x;
  if (S.status[e] != ST_ACTIVE || m == 0) {
    if (tid == 0) S.cok[e] = 0;
    return;
  }
  for (int qd = tid; qd < m * m; qd += 64) {
    const int r = qd / m, c = qd % m;
    double a = 0.0;
    for (int k = 0; k < E.vtile_count; ++k) a += e_tile[(size_t)(E.vtile_first + k) * (M * M) + r * M + c];
    A[r * M + c] = a;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int qd = tid; qd < m * m; qd += 64) {
    const int r = qd / m, c = qd % m;
    if (r < c) {
      const double a = 0.5 * (A[r * M + c] + A[c * M + r]);
      A[r * M + c] = a;
      A[c * M + r] = a;
    }
  }
  // a pivot below 1e-10 of E's largest diagonal entry (a body whose rigid
  // motions are not independent, e.g. collinear free vertices) counts as a
  // failed factorisation: the environment then runs block Jacobi alone
  if (tid == 0) {
    double dmax = 0.0;
    for (int k = 0; k < m; ++k) dmax = fmax(dmax, A[k * M + k]);
    tiny = 1e-10 * dmax;
  }
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    if (tid == 0) {
      const double p = A[k * M + k];
      if (!(p > tiny)) bad = 1;
      A[k * M + k] = p > tiny ? sqrt(p) : 1.0;
    }
    __syncthreads();
    for (int r = k + 1 + tid; r < m; r += 64) A[r * M + k] /= A[k * M + k];
    __syncthreads();
    for (int qd = tid; qd < m * m; qd += 64) {
      const int r = qd / m, c = qd % m;
      if (c > k && c <= r) A[r * M + c] -= A[r * M + k] * A[c * M + k];
    }
    __syncthreads();
  }
  // L^-1 column by column (forward substitution of e_j)
  for (int j = tid; j < m; j += 64)
    for (int r = 0; r < m; ++r) {
      if (r < j) {
        Li[r * M + j] = 0.0;
        continue;
      }
      double a = (r == j) ? 1.0 : 0.0;
      for (int k = j; k < r; ++k) a -= A[r * M + k] * Li[k * M + j];
      Li[r * M + j] = a / A[r * M + r];
    }
  __syncthreads();
  double *inv = S.cinv + (size_t)e * (M * M);
  for (int qd = tid; qd < m * m; qd += 64) {
    const int r = qd / m, c = qd % m;
    double a = 0.0;
    for (int k = (r > c ? r : c); k < m; ++k) a += Li[k * M + r] * Li[k * M + c];
    inv[r * M + c] = a;
  }
  if (tid == 0) S.cok[e] = bad ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Per-environment PCG: one 1024-thread workgroup iterates a whole
// environment inside one launch.  The product runs one 256-row tile per pass
// (4 lanes per row, as k_spmv); the update runs four tiles per pass, each
// 256-thread quarter reducing its tile with the tiled kernels' tree.  Tile
// partials go to the same per-tile arrays and are summed in tile order.
// ---------------------------------------------------------------------------
constexpr int FB = 1024;

// sums of a and b over each 256-thread quarter (quarter_sum2); thread 0 of
// each quarter stores them for tile `tile0 + quarter` if that tile exists
DEV void tile_sums2(double a, double b, double *sh, const EnvDev &E, int tile0, double *pa, double *pb) {
  quarter_sum2(a, b, sh);
  const int qd = threadIdx.x / TB;
  if (threadIdx.x % TB == 0 && tile0 + qd < E.vtile_count) {
    if (pa) pa[E.vtile_first + tile0 + qd] = a;
    if (pb) pb[E.vtile_first + tile0 + qd] = b;
  }
  __syncthreads();
}

// Iterations of one environment from iteration `it` (u, r, x, p, s current;
// gamma and r.r partials in part_g[it&1], part_rr[it&1]; alpha, gamma of
// iteration it-1 in a_prev, g_prev) until the stopping rule; returns the
// iteration count
template <typename T>
DEV int env_iterate(const WorldDev &W, const EnvDev &E, double bb, int it, double a_prev, double g_prev,
                    const int *inc_off, const int *cr_cnt, const int *cr_col, const T *cr_val, T *x, T *r, T *u, T *pp,
                    T *q, T *w, const T *val, const T *Minv, double *part_d, double *const part_g[2],
                    double *const part_rr[2], double (*sh)[FB]) {
  const int r0 = E.v_off, r1 = E.v_off + E.nv_pad;
  for (;;) {
    for (int base = r0; base < r1; base += TB) {
      const int row = threadIdx.x / kLPR, l = threadIdx.x % kLPR;
      const int i = base + row;
      const bool valid = i < r1;
      RowHead h{0, 0, 0, 0};
      if (valid) h = row_head(W, i, inc_off, cr_cnt);
      double d = row_spmv<T, true>(W, i, valid, l, h, cr_col, cr_val, u, w, val);
      d = rows_sum(d, sh[0]);
      if (threadIdx.x == 0) part_d[E.vtile_first + (base - r0) / TB] = d;
    }
    __syncthreads();  // the last tile's partial
    double gam, del, rr;
    env_sums3(part_g[it & 1], part_d, part_rr[it & 1], E, sh[0], gam, del, rr);
    double alpha = 0.0, beta = 0.0;
    if (cg_step(E, bb, it, gam, del, rr, a_prev, g_prev, alpha, beta)) break;
    for (int base = r0; base < r1; base += FB) {
      int i = base + threadIdx.x;
      double g = 0.0, rri = 0.0;
      if (i < r1) {
        RowVals<T> v;
        row_load<T>(i, x, r, u, pp, q, w, Minv, v);
        const double zero3[3] = {0.0, 0.0, 0.0};
        double rn[3];
        row_step<T>(i, alpha, beta, v, x, r, u, pp, q, g, rri, zero3, rn);
      }
      tile_sums2(g, rri, sh[1], E, (base - r0) / TB, part_g[(it + 1) & 1], part_rr[(it + 1) & 1]);
    }
    a_prev = alpha;
    g_prev = gam;
    ++it;
  }
  return it;
}

template <typename T>
__global__ void __launch_bounds__(1024) k_pcg_fused(WorldDev W, const EnvDev *envs, EnvState S, const int *fenv,
                                                    const int *inc_off, const int *cr_cnt, const int *cr_col,
                                                    const T *cr_val, T *x, T *r, T *u, T *pp, T *q, T *w,
                                                    const T *val, const T *Minv, double *part_d, double *part_g0,
                                                    double *part_g1, double *part_rr0, double *part_rr1) {
  __shared__ double sh[2][FB];
  int e = fenv[blockIdx.x];
  if (S.status[e] != ST_ACTIVE) return;
  const EnvDev &E = envs[e];
  const int r0 = E.v_off, r1 = E.v_off + E.nv_pad;
  double *const pg[2] = {part_g0, part_g1}, *const prr[2] = {part_rr0, part_rr1};
  for (int base = r0; base < r1; base += FB) {
    int i = base + threadIdx.x;
    double g = 0.0, rr = 0.0;
    if (i < r1) row_init<T>(W, is_dof(W, S, i, e), i, x, r, u, pp, q, Minv, g, rr);
    tile_sums2(g, rr, sh[1], E, (base - r0) / TB, part_g0, part_rr0);
  }
  const double bb = env_tiles_sum(part_rr0, E);
  int it = 0;
  if (!(bb == 0.0 || !(bb == bb)))
    it = env_iterate<T>(W, E, bb, 0, 0.0, 0.0, inc_off, cr_cnt, cr_col, cr_val, x, r, u, pp, q, w, val, Minv, part_d,
                        pg, prr, sh);
  if (threadIdx.x == 0) {
    S.pcg_it[e] = it;
    S.pcg_total[e] += it;
    S.pcg_done[e] = 1;
  }
}

// Tail of the tiled PCG: once few tiles are still iterating, the first tile
// of each live environment continues its solve in one workgroup from the
// state the tiled kernels left after `it` iterations.
template <typename T>
__global__ void __launch_bounds__(1024) k_pcg_resume(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles,
                                                     int it, const int *inc_off, const int *cr_cnt, const int *cr_col,
                                                     const T *cr_val, T *x, T *r, T *u, T *pp, T *q, T *w,
                                                     const T *val, const T *Minv, double *part_d, double *part_g0,
                                                     double *part_g1, double *part_rr0, double *part_rr1) {
  __shared__ double sh[2][FB];
  Tile t = tiles[blockIdx.x];
  if (t.rel != 0 || !pcg_env_live(S, t.env)) return;
  const int e = t.env;
  const EnvDev &E = envs[e];
  double *const pg[2] = {part_g0, part_g1}, *const prr[2] = {part_rr0, part_rr1};
  const int k = (it + 1) & 1;  // slot of iteration it - 1
  const int n = env_iterate<T>(W, E, S.pcg_bb[e], it, k ? S.cg_a1[e] : S.cg_a0[e], k ? S.cg_g1[e] : S.cg_g0[e],
                               inc_off, cr_cnt, cr_col, cr_val, x, r, u, pp, q, w, val, Minv, part_d, pg, prr, sh);
  if (threadIdx.x == 0) {
    S.pcg_it[e] = n;
    S.pcg_total[e] += n;
    S.pcg_done[e] = 1;
  }
}

// flags of the vertex tiles whose environment still iterates its PCG
__global__ void k_live_flags(EnvState S, const Tile *tiles, int n, int *flag) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) flag[j] = pcg_env_live(S, tiles[j].env) ? 1 : 0;
}

__global__ void k_live_compact(const Tile *tiles, int n, const int *flag, const int *offs, Tile *out) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && flag[j]) out[offs[j]] = tiles[j];
}

__global__ void k_p32_to_p(WorldDev W, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  int i = t.start + threadIdx.x;
  for (int c = 0; c < 3; ++c) W.p[3 * i + c] = (double)W.p32[3 * i + c];
}

// debug: out = H in over the batch (all vertices of ACTIVE envs), one
// 256-row tile per 1024-thread workgroup as in k_spmv
__global__ void __launch_bounds__(1024) k_spmv_dbg(WorldDev W, EnvState S, const Tile *tiles, const int *inc_off,
                                                   const int *cr_cnt, const int *cr_col, const double *cr_val,
                                                   const double *in, double *out) {
  Tile t = tiles[blockIdx.x];
  if (!active_env(S, t.env)) return;
  const int row = threadIdx.x / kLPR, l = threadIdx.x % kLPR;
  const int i = t.start + row;
  const bool valid = row < t.count;
  double y[3];
  RowHead h{0, 0, 0, 0};
  if (valid) h = row_head(W, i, inc_off, cr_cnt);
  row_product<double, StoredVec<double>, false>(W, i, valid, l, h, StoredVec<double>{in}, W.val, cr_col, cr_val, y);
  if (valid && l < 3) out[3 * i + l] = y[l];
}

// ---------------------------------------------------------------------------
// convergence test |p|_inf <= tol * dt (per environment)
// ---------------------------------------------------------------------------
__global__ void k_pinf(WorldDev W, EnvState S, const Tile *tiles, double *part, double *part_viol) {
  __shared__ double sh[TB];
  Tile t = tiles[blockIdx.x];
  if (!active_env(S, t.env)) return;
  int i = t.start + threadIdx.x;
  double m = 0.0, v = 0.0;
  if ((int)threadIdx.x < t.count && is_dof(W, S, i, t.env))
    for (int c = 0; c < 3; ++c) {
      double a = W.p[3 * i + c];
      m = (a != a) ? a : fmax(m, fabs(a));
    }
  if ((int)threadIdx.x < t.count && W.kin[i] >= 0 && S.al[t.env])
    for (int c = 0; c < 3; ++c) v = fmax(v, fabs(W.x[3 * i + c] - W.xh[3 * i + c]));
  m = block_max(m, sh);
  v = block_max(v, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = m;
    part_viol[blockIdx.x] = v;
  }
}

__global__ void k_env_conv(const EnvDev *envs, EnvState S, const int *benv, int n, const double *part,
                           const double *part_viol, int *n_active) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (S.status[e] != ST_ACTIVE) return;
  const EnvDev &E = envs[e];
  double m = 0.0;
  bool nan = false;
  for (int i = 0; i < E.vtile_count; ++i) {
    double a = part[E.vtile_first + i];
    if (!(a == a) || a == kInf) nan = true;
    m = fmax(m, a);
  }
  S.pinf[e] = m;
  S.iters[e] += 1;
  S.al_action[e] = 0;
  if (nan) {
    S.status[e] = ST_FAILED;
    S.reason[e] = FAIL_NONFINITE;
  } else if (m <= E.tol * E.dt && !S.al[e]) {
    S.status[e] = ST_CONVERGED;
  } else {
    if (m <= E.tol * E.dt) {
      // AL mode, inner problem converged: snap to the targets once within
      // 1e-2 dhat (if CCD-safe), otherwise update the multipliers
      double v = 0.0;
      for (int i = 0; i < E.vtile_count; ++i) v = fmax(v, part_viol[E.vtile_first + i]);
      S.viol[e] = v;
      S.al_action[e] = (v <= 1e-2 * E.dhat) ? 2 : 1;
    }
    atomicAdd(n_active, 1);
  }
}

// AL actions: the displacement the swept CCD pass must check (snap) or none
__global__ void k_al_prepare(WorldDev W, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  int act = S.al_action[t.env];
  if (act == 0) return;
  int i = t.start + threadIdx.x;
  bool snap = (act == 2) && W.kin[i] >= 0;
  for (int c = 0; c < 3; ++c) W.p[3 * i + c] = snap ? W.xh[3 * i + c] - W.x[3 * i + c] : 0.0;
  if (threadIdx.x == 0 && t.rel == 0) S.snap_bad[t.env] = 0;
}

__global__ void k_snap_J(WorldDev W, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env) || S.al_action[t.env] != 2) return;
  int e = t.start + threadIdx.x;
  int4 q = W.tet[e];
  int v[4] = {q.x, q.y, q.z, q.w};
  double x[12];
  gather12_trial(W.x, W.p, 1.0, v, x);
  double F[9];
  nh_F(x, W.Dinv + 9 * e, F);
  if (!(det33(F) > 0.0)) S.snap_bad[t.env] = 1;
}

__global__ void k_al_decide(EnvState S, const int *benv, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (S.status[e] != ST_ACTIVE || S.al_action[e] != 2) return;
  double a = __longlong_as_double((long long)S.amax_bits[e]);
  S.al_action[e] = (a >= 1.0 && !S.snap_bad[e]) ? 3 : 1;
}

__global__ void k_al_vertex(const EnvDev *envs, WorldDev W, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  int act = S.al_action[t.env];
  int i = t.start + threadIdx.x;
  if (W.kin[i] < 0 || (act != 1 && act != 3)) return;
  if (act == 3) {
    for (int c = 0; c < 3; ++c) W.x[3 * i + c] = W.xh[3 * i + c];
  } else {
    const EnvDev &E = envs[t.env];
    double sw = sqrt(E.mbar / (E.dt * E.dt)), kA = S.kA[t.env];
    for (int c = 0; c < 3; ++c) W.lam[3 * i + c] -= kA * sw * (W.x[3 * i + c] - W.xh[3 * i + c]);
  }
}

__global__ void k_al_env(EnvState S, const int *benv, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (S.status[e] != ST_ACTIVE) return;
  int act = S.al_action[e];
  if (act == 3) {
    S.al[e] = 0;
  } else if (act == 1) {
    if (S.viol[e] > 0.1 * S.viol_prev[e]) S.kA[e] *= 2.0;
    S.viol_prev[e] = S.viol[e];
  }
}

// ---------------------------------------------------------------------------
// additive CCD step bound (per environment minimum via ordered-bit atomicMin)
// ---------------------------------------------------------------------------
__global__ void k_ccd_init(EnvState S, const int *benv, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  S.amax_bits[benv[j]] = (unsigned long long)__double_as_longlong(1.0);
}

__global__ void __launch_bounds__(128) k_accd(WorldDev W, EnvState S, const int2 *cand, int n, const double *x,
                                              const double *p) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int kind, v[4], env;
  double ex;
  pair_info(W, cand[k], kind, v, env, ex);
  if (S.status[env] != ST_ACTIVE) return;
  double xx[12], pp[12];
  gather12(x, v, xx);
  gather12(p, v, pp);
  double tt = accd(kind, xx, pp, 0.1);
  if (tt < 1.0) atomicMin(&S.amax_bits[env], (unsigned long long)__double_as_longlong(tt));
}

// inversion filter: every tet of an environment in its line search lowers the
// environment's step bound to min(1, 0.8 t*), t* the first root of
// det(Ds(x + t p)) (ordered-bit atomicMin, as for the CCD bound)
__global__ void k_inv_bound(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, int force) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !active_env(S, t.env)) return;
  if (!force && (S.al_action[t.env] != 0 || !envs[t.env].inv_filter || S.phase[t.env] != PH_ITER)) return;
  int e = t.start + threadIdx.x;
  int4 q = W.tet[e];
  int v[4] = {q.x, q.y, q.z, q.w};
  double xx[12], pp[12];
  gather12(W.x, v, xx);
  gather12(W.p, v, pp);
  double a = tet_inversion_bound(xx, pp);
  if (a < 1.0) atomicMin(&S.amax_bits[t.env], (unsigned long long)__double_as_longlong(a));
}

// friction lag round: an environment whose Newton solve converged and that
// takes more lagged friction updates this step solves again (friction data
// are then taken at its converged iterate), with a fresh iteration budget
__global__ void k_relag(const EnvDev *envs, EnvState S, const int *benv, int n, int sel, int *n_relag) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (sel ? S.phase[e] != PH_RELAG
          : (!S.in_step[e] || S.status[e] != ST_CONVERGED || S.lag[e] + 1 >= envs[e].fric_iters))
    return;
  S.lag[e] += 1;
  S.status[e] = ST_ACTIVE;
  S.iter_cap[e] = S.iters[e] + envs[e].maxit;
  S.al_action[e] = 0;
  atomicAdd(n_relag, 1);
}

__global__ void k_ls_init(EnvState S, const int *benv, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  S.alpha[e] = __longlong_as_double((long long)S.amax_bits[e]);
  S.ls_done[e] = (S.status[e] == ST_ACTIVE && S.al_action[e] == 0 && S.phase[e] == PH_ITER) ? 0 : 1;
  S.ls_cnt[e] = 0;
}

// ---------------------------------------------------------------------------
// line-search energies at x + alpha_env p (alpha = 0 for the reference value)
// ---------------------------------------------------------------------------
DEV bool ls_live(const EnvState &S, int env) { return S.status[env] == ST_ACTIVE && !S.ls_done[env]; }

__global__ void k_energy_v(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, int zero_alpha) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !ls_live(S, t.env)) return;
  const EnvDev &E = envs[t.env];
  int i = t.start + threadIdx.x;
  double a = zero_alpha ? 0.0 : S.alpha[t.env];
  double e = 0.0;
  if (W.kin[i] == KIN_FREE) {
    double q = 0.0;
    for (int c = 0; c < 3; ++c) {
      double r = W.x[3 * i + c] + a * W.p[3 * i + c] - W.xh[3 * i + c];
      q += r * r;
    }
    e = W.mass[i] * q / (2.0 * E.dt * E.dt);
  } else if (W.kin[i] >= 0 && S.al[t.env]) {
    double w0 = E.mbar / (E.dt * E.dt), q = 0.0, l = 0.0;
    for (int c = 0; c < 3; ++c) {
      double r = W.x[3 * i + c] + a * W.p[3 * i + c] - W.xh[3 * i + c];
      q += r * r;
      l += W.lam[3 * i + c] * r;
    }
    e = 0.5 * S.kA[t.env] * w0 * q - sqrt(w0) * l;
  }
  W.e_v[i] = e;
}

__global__ void k_energy_t(WorldDev W, EnvState S, const Tile *tiles, int zero_alpha) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !ls_live(S, t.env)) return;
  int e = t.start + threadIdx.x;
  double a = zero_alpha ? 0.0 : S.alpha[t.env];
  int4 q = W.tet[e];
  int v[4] = {q.x, q.y, q.z, q.w};
  double x[12];
  gather12_trial(W.x, W.p, a, v, x);
  W.e_t[e] = nh_energy(x, W.Dinv + 9 * e, W.vol[e], W.mu[e], W.la[e]);
}

__global__ void k_energy_c(WorldDev W, const EnvDev *envs, EnvState S, const int2 *cand, int n, int zero_alpha,
                           double *e_c) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int kind, v[4], env;
  double ex;
  pair_info(W, cand[k], kind, v, env, ex);
  if (!ls_live(S, env)) return;
  const EnvDev &E = envs[env];
  double a = zero_alpha ? 0.0 : S.alpha[env];
  double xx[12], d2;
  gather12_trial(W.x, W.p, a, v, xx);
  classify(kind, xx, &d2);
  double e = 0.0;
  if (!(d2 > 0.0))
    e = kInf;
  else if (d2 < E.dhat * E.dhat)
    e = pair_barrier_energy(kind, xx, d2, E.dhat, S.kappa[env], ex);
  e_c[k] = e;
}

__global__ void k_energy_f(WorldDev W, const EnvDev *envs, EnvState S, const int4 *fv, const double *fw,
                           const double *fn, const double *flam, const int *fenv, int n, int zero_alpha, double *e_f) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int env = fenv[k];
  if (!ls_live(S, env)) return;
  const EnvDev &E = envs[env];
  double a = zero_alpha ? 0.0 : S.alpha[env];
  int4 q = fv[k];
  int v[4] = {q.x, q.y, q.z, q.w};
  double u[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int c = 0; c < 3; ++c)
      u[c] += fw[4 * k + i] * (W.x[3 * v[i] + c] + a * W.p[3 * v[i] + c] - W.xn[3 * v[i] + c]);
  double un = u[0] * fn[3 * k] + u[1] * fn[3 * k + 1] + u[2] * fn[3 * k + 2];
  for (int c = 0; c < 3; ++c) u[c] -= un * fn[3 * k + c];
  double y = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  e_f[k] = E.mu * flam[k] * friction_f0(y, E.eps_v * E.dt);
}

// one block per environment: Phi = inertia + elastic + barrier + friction
__global__ void k_env_energy(WorldDev W, const EnvDev *envs, EnvState S, const int *benv, const double *e_c,
                             const double *e_f, double *E_out) {
  __shared__ double sh[TB];
  int e = benv[blockIdx.x];
  if (!ls_live(S, e)) return;
  const EnvDev &E = envs[e];
  double s = 0.0;
  for (int i = threadIdx.x; i < E.nv_pad; i += TB) s += W.e_v[E.v_off + i];
  for (int i = threadIdx.x; i < E.nt; i += TB) s += W.e_t[E.t_off + i];
  for (int i = S.cand_beg[e] + threadIdx.x; i < S.cand_end[e]; i += TB) s += e_c[i];
  for (int i = S.fric_beg[e] + threadIdx.x; i < S.fric_end[e]; i += TB) s += e_f[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) E_out[e] = (s == s) ? s : kInf;
}

__global__ void k_ls_decide(EnvState S, const int *benv, int n, int *pending) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (S.status[e] != ST_ACTIVE || S.ls_done[e]) return;
  if (S.E1[e] <= S.E0[e]) {
    S.ls_done[e] = 1;
    return;
  }
  S.alpha[e] *= 0.5;
  S.halvings[e] += 1;
  if (++S.ls_cnt[e] > 40) {
    S.status[e] = ST_FAILED;
    S.reason[e] = FAIL_LS;
    return;
  }
  atomicAdd(pending, 1);
}

__global__ void k_update_x(WorldDev W, EnvState S, const Tile *tiles) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || S.status[t.env] != ST_ACTIVE || S.al_action[t.env] != 0 ||
      S.phase[t.env] != PH_ITER)
    return;
  int i = t.start + threadIdx.x;
  double a = S.alpha[t.env];
  for (int c = 0; c < 3; ++c) W.x[3 * i + c] += a * W.p[3 * i + c];
}

__global__ void k_iter_end(const EnvDev *envs, EnvState S, const int *benv, int n, int *n_active) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  if (S.status[e] != ST_ACTIVE) return;
  if (S.iters[e] >= S.iter_cap[e]) {
    S.status[e] = ST_FAILED;
    S.reason[e] = FAIL_MAXIT;
    return;
  }
  atomicAdd(n_active, 1);
}

// sel = 0: every environment that took part in the step; sel = 1: those
// whose phase ends a step (the decoupled schedule)
__global__ void k_step_end(WorldDev W, const EnvDev *envs, EnvState S, const Tile *tiles, int sel) {
  Tile t = tiles[blockIdx.x];
  if ((int)threadIdx.x >= t.count || !S.in_step[t.env]) return;
  if (sel && S.phase[t.env] != PH_FINISH && S.phase[t.env] != PH_FINISH_BEGIN) return;
  int st = S.status[t.env];
  int i = t.start + threadIdx.x;
  if (st == ST_CONVERGED) {
    double h = envs[t.env].dt;
    for (int c = 0; c < 3; ++c) W.v[3 * i + c] = (W.x[3 * i + c] - W.xn[3 * i + c]) / h;
  } else if (st == ST_FAILED) {
    for (int c = 0; c < 3; ++c) W.x[3 * i + c] = W.xn[3 * i + c];
  }
}

// after k_step_end of the decoupled schedule: an environment that ended its
// step rests (converged) or stays failed, and one that goes on begins
__global__ void k_phase_advance(EnvState S, const int *benv, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  int e = benv[j];
  const int ph = S.phase[e];
  if (ph == PH_FINISH || ph == PH_FINISH_BEGIN) {
    if (S.status[e] == ST_CONVERGED) S.status[e] = ST_IDLE;
    S.phase[e] = ph == PH_FINISH_BEGIN ? PH_BEGIN : PH_ITER;
  }
}

__global__ void k_set_phase(EnvState S, const int *benv, int n, int ph) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) S.phase[benv[j]] = ph;
}

// ---------------------------------------------------------------------------
// friction merge of the decoupled schedule: environments that begin a step or
// re-lag take new friction data from the active pairs of this round's list;
// the others keep theirs.  Pairs are stored per environment in batch order.
// ---------------------------------------------------------------------------
DEV bool new_friction(const EnvState &S, int env) {
  return S.status[env] == ST_ACTIVE && (S.phase[env] == PH_BEGIN || S.phase[env] == PH_RELAG);
}
DEV bool keeps_friction(const EnvState &S, int env) { return S.status[env] == ST_ACTIVE && S.phase[env] == PH_ITER; }

// candidates of environments that keep their friction are not active here
__global__ void k_cand_restrict(WorldDev W, EnvState S, const int2 *cand, int n, int *flag) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  int kind, v[4], env;
  double ex;
  pair_info(W, cand[k], kind, v, env, ex);
  if (!new_friction(S, env)) flag[k] = 0;
}

// new friction ranges in batch order (one thread: a few hundred environments);
// nb[e] = -1 for environments whose friction is dropped
__global__ void k_fric_plan(EnvState S, const int *benv, int n, int *nb, int *ne, int *total) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int off = 0;
  for (int j = 0; j < n; ++j) {
    const int e = benv[j];
    int c = -1;
    if (new_friction(S, e))
      c = S.act_end[e] - S.act_beg[e];
    else if (keeps_friction(S, e))
      c = S.fric_end[e] - S.fric_beg[e];
    nb[e] = c < 0 ? -1 : off;
    ne[e] = c < 0 ? -1 : off + c;
    off += c < 0 ? 0 : c;
  }
  *total = off;
}

__global__ void k_fric_copy(EnvState S, int n_old, const int4 *fv, const double *fw, const double *fn,
                            const double *flam, const int *fenv, const int *nb, int4 *fv2, double *fw2, double *fn2,
                            double *flam2, int *fenv2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_old) return;
  const int e = fenv[k];
  if (!keeps_friction(S, e) || nb[e] < 0) return;
  const int o = nb[e] + (k - S.fric_beg[e]);
  fv2[o] = fv[k];
  for (int i = 0; i < 4; ++i) fw2[4 * o + i] = fw[4 * k + i];
  for (int c = 0; c < 3; ++c) fn2[3 * o + c] = fn[3 * k + c];
  flam2[o] = flam[k];
  fenv2[o] = e;
}

__global__ void k_fric_commit(EnvState S, const int *benv, int n, const int *nb, const int *ne) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int e = benv[j];
  S.fric_beg[e] = nb[e] < 0 ? 0 : nb[e];
  S.fric_end[e] = nb[e] < 0 ? 0 : ne[e];
}

// ---------------------------------------------------------------------------
// Cauchy stress sigma = J^-1 P F^T and von Mises
// ---------------------------------------------------------------------------
__global__ void k_stress(WorldDev W, int t_off, int nt, double *cauchy, double *vm) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nt) return;
  int e = t_off + k;
  int4 q = W.tet[e];
  int v[4] = {q.x, q.y, q.z, q.w};
  double x[12], F[9], FiT[9];
  gather12(W.x, v, x);
  nh_F(x, W.Dinv + 9 * e, F);
  double J = inv_T33(F, FiT);
  double mu = W.mu[e], la = W.la[e], lJ = log(J);
  double P[9], S[9];
  for (int i = 0; i < 9; ++i) P[i] = mu * F[i] + (la * lJ - mu) * FiT[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      S[3 * i + j] = (P[3 * i] * F[3 * j] + P[3 * i + 1] * F[3 * j + 1] + P[3 * i + 2] * F[3 * j + 2]) / J;
  double *o = cauchy + 6 * (size_t)k;
  o[0] = S[0];
  o[1] = S[4];
  o[2] = S[8];
  o[3] = S[5];
  o[4] = S[2];
  o[5] = S[1];
  double a = S[0] - S[4], b = S[4] - S[8], c = S[8] - S[0];
  vm[k] = sqrt(0.5 * (a * a + b * b + c * c) + 3.0 * (S[1] * S[1] + S[5] * S[5] + S[2] * S[2]));
}

// ---------------------------------------------------------------------------
// element-level debug kernels
// ---------------------------------------------------------------------------
__global__ void k_dbg_classify(int kind, int n, const double *x12, int *types, double *d2) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  types[k] = classify(kind, x12 + 12 * (size_t)k, &d2[k]);
}

__global__ void k_dbg_pair(int kind, int type, const double *x12, double dhat, double kappa, double eps_x, int project,
                           double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double x[12], g[12], H[144], scr[168];
  for (int i = 0; i < 12; ++i) x[i] = x12[i];
  out[0] = pair_barrier_full(kind, type, x, dhat, kappa, eps_x, project != 0, g, H, scr);
  for (int i = 0; i < 12; ++i) out[1 + i] = g[i];
  for (int i = 0; i < 144; ++i) out[13 + i] = H[i];
}

__global__ void k_dbg_tet(const double *X12, const double *x12, double mu, double la, double *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double Dm[9], Dinv[9];
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) Dm[i * 3 + a] = X12[3 * (a + 1) + i] - X12[i];
  inv33(Dm, Dinv);
  double vol = det33(Dm) / 6.0;
  double x[12], g[12], blocks[90], en;
  for (int i = 0; i < 12; ++i) x[i] = x12[i];
  if (!nh_element(x, Dinv, vol, mu, la, &en, g, blocks)) {
    out[0] = kInf;
    return;
  }
  out[0] = en;
  for (int i = 0; i < 12; ++i) out[1 + i] = g[i];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          const double *B = blocks + 9 * (a <= b ? blk_index(a, b) : blk_index(b, a));
          out[13 + (3 * a + r) * 12 + 3 * b + c] = (a <= b) ? B[3 * r + c] : B[3 * c + r];
        }
}

__global__ void k_dbg_tet_root(int n, const double *x12, const double *p12, double tmax, double *t, double *k4) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double c[4];
  det_line_cubic(x12 + 12 * k, p12 + 12 * k, c);
  t[k] = cubic_first_root(c, tmax);
  for (int i = 0; i < 4; ++i) k4[4 * k + i] = c[i];
}

__global__ void k_dbg_accd(int kind, int n, const double *x12, const double *p12, double sfac, double *t) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  t[k] = accd(kind, x12 + 12 * (size_t)k, p12 + 12 * (size_t)k, sfac);
}

// CCD step bound over a list of pairs of one kind (Sec. II-C: CCD bounds the
// Newton step): min(1, min_k ACCD_k).  Pass 1 writes each block's minimum to
// part[block]; pass 2 (one block) takes the minimum over the partials.  Both
// minima are exact, so the result does not depend on the block count.
constexpr int kCcdBlock = 128;
__global__ void __launch_bounds__(kCcdBlock) k_pairs_ccd_min(int kind, int n, const double *x12, const double *p12,
                                                            double sfac, double *part) {
  __shared__ double sh[kCcdBlock];
  const int k = blockIdx.x * kCcdBlock + threadIdx.x;
  double t = 1.0;
  if (k < n) t = fmin(1.0, accd(kind, x12 + 12 * (size_t)k, p12 + 12 * (size_t)k, sfac));
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int w = kCcdBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(TB) k_min_reduce(const double *part, int n_part, double *out) {
  __shared__ double sh[TB];
  double m = 1.0;
  for (int i = threadIdx.x; i < n_part; i += TB) m = fmin(m, part[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Per-block minima of the allocation-free CCD bound: a file-scope device
// array, one copy per GPU (its storage comes with the code object and lives
// until the process ends).  Host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
constexpr int kNoAllocParts = 1 << 16;
static __device__ __align__(256) double ccd_scratch[kNoAllocParts];

// Grasp-quality metrics (Sec. IV-C, Eq. (2)-(3)): one thread per sample point
// on the gripper's surface, the manipuland's boundary triangles streamed
// through LDS in tiles of 256; each thread keeps its least squared distance
// and its winding sum (solid angles / 4 pi).  d_o(p) = +distance inside
// (winding > 1/2), -distance outside.  part[block] = the block's largest d_o.
constexpr int kSdfTile = 256;
__global__ void __launch_bounds__(kSdfTile) k_sdf_samples(const double *x, const int *obj_tris, int n_obj,
                                                          const int *hand_tris, const int *sample_tri,
                                                          const double *sample_uv, int n_samples, double *sdf,
                                                          double *part) {
  __shared__ double tv[kSdfTile * 9];
  __shared__ double red[kSdfTile];
  const int i = blockIdx.x * kSdfTile + threadIdx.x;
  d3 p = {0.0, 0.0, 0.0};
  if (i < n_samples) {
    const int t = sample_tri[i];
    const double u = sample_uv[2 * i], v = sample_uv[2 * i + 1], w = 1.0 - u - v;
    const int a = hand_tris[3 * t], b = hand_tris[3 * t + 1], c = hand_tris[3 * t + 2];
    p = {w * x[3 * a] + u * x[3 * b] + v * x[3 * c], w * x[3 * a + 1] + u * x[3 * b + 1] + v * x[3 * c + 1],
         w * x[3 * a + 2] + u * x[3 * b + 2] + v * x[3 * c + 2]};
  }
  double best = kInf, wind = 0.0;
  for (int base = 0; base < n_obj; base += kSdfTile) {
    const int m = min(kSdfTile, n_obj - base);
    __syncthreads();
    for (int k = threadIdx.x; k < 9 * m; k += kSdfTile) {
      const int tri = k / 9, r = k % 9;
      tv[k] = x[3 * obj_tris[3 * (base + tri) + r / 3] + r % 3];
    }
    __syncthreads();
    if (i < n_samples)
      for (int j = 0; j < m; ++j) {
        const double *q = tv + 9 * j;
        const d3 A = {q[0], q[1], q[2]}, B = {q[3], q[4], q[5]}, C = {q[6], q[7], q[8]};
        best = fmin(best, point_tri_dist2(p, A, B, C));
        wind += tri_solid_angle(p, A, B, C);
      }
  }
  double d = -kInf;
  if (i < n_samples) {
    d = sqrt(best);
    if (!(wind > 2.0 * M_PI)) d = -d;  // winding number wind / 4 pi <= 1/2: outside
    sdf[i] = d;
  }
  red[threadIdx.x] = d;
  __syncthreads();
  for (int s = kSdfTile / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_max_reduce(const double *part, int n, double *out) {
  __shared__ double red[TB];
  double m = -kInf;
  for (int k = threadIdx.x; k < n; k += TB) m = fmax(m, part[k]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = fmax(0.0, red[0]);  // D1
    out[1] = fabs(red[0]);       // D2
  }
}

__global__ void k_fill_int(int *p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline int nblk(int n, int b) { return (n + b - 1) / b; }

}  // namespace

// ===========================================================================
// launchers
// ===========================================================================
namespace ipck {

void begin_step(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B) {
  if (B.n_vt) IPC_LAUNCH(k_begin_step, B.n_vt, TB, s)(W, E, S, B.vtiles);
}
void dbc_check_J(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B) {
  if (B.n_tt) IPC_LAUNCH(k_dbc_J, B.n_tt, TB, s)(W, E, S, B.ttiles);
}
void apply_dbc(hipStream_t s, const WorldDev &W, const EnvDev *, const EnvState &S, const Batch &B) {
  if (B.n_vt) IPC_LAUNCH(k_apply_dbc, B.n_vt, TB, s)(W, S, B.vtiles);
}
void env_begin(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B) {
  IPC_LAUNCH(k_env_begin, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs);
}
void env_dbc(hipStream_t s, const EnvState &S, const Batch &B) {
  IPC_LAUNCH(k_env_dbc, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs);
}

void boxes(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, const double *x,
           const double *p) {
  if (B.n_svt) IPC_LAUNCH(k_boxes, B.n_svt, TB, s)(W, E, S, B.svtiles, 0, x, p);
  if (B.n_trit) IPC_LAUNCH(k_boxes, B.n_trit, TB, s)(W, E, S, B.tritiles, 1, x, p);
  if (B.n_et) IPC_LAUNCH(k_boxes, B.n_et, TB, s)(W, E, S, B.etiles, 2, x, p);
}

void grid_count(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L) {
  if (B.n_bt) IPC_LAUNCH(k_grid_count, B.n_bt, TB, s)(W, E, S, B.btiles, L.g_ncell, L.g_big);
}
void grid_fill(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
               int n_ent, unsigned nbuckets) {
  IPC_LAUNCH(k_fill_int, nblk(nbuckets + 1, TB), TB, s)(L.g_bcnt, nbuckets + 1, 0);
  IPC_LAUNCH(k_fill_int, nblk(nbuckets + 1, TB), TB, s)(L.g_bcur, nbuckets + 1, 0);
  if (B.n_bt)
    IPC_LAUNCH(k_grid_fill, B.n_bt, TB, s)(W, E, S, B.btiles, L.g_eoff, L.g_bigoff, L.g_ent, L.g_ebucket, L.g_bcnt,
                                          L.g_bigl, nbuckets - 1);
  IPC_LAUNCH(k_big_seg, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs, L.g_bigoff);
  scan_int(s, L.g_bcnt, L.g_boff, (int)nbuckets, L.scan_tmp);
  if (n_ent) IPC_LAUNCH(k_grid_place, nblk(n_ent, TB), TB, s)(L.g_ent, L.g_ebucket, n_ent, L.g_boff, L.g_bcur, L.g_sorted);
}
void bp_grid_count(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
                   unsigned nbuckets) {
  IPC_LAUNCH(k_fill_int, 1, 64, s)(L.counter + 4, 1, 0);
  if (B.n_it && L.bp_coop)
    IPC_LAUNCH(k_bp_coop, B.n_it * kBpGroup, TB, s)(W, E, S, B.itiles, L.counts, L.g_sorted, L.g_boff, L.g_bigl,
                                                    nbuckets - 1, L.bp_stash, L.stash_n, L.counter + 4);
  else if (B.n_it)
    IPC_LAUNCH(k_bp_grid<false>, B.n_it, TB, s)(W, E, S, B.itiles, L.counts, nullptr, nullptr, L.g_sorted, L.g_boff,
                                               L.g_bigl, nbuckets - 1, L.bp_stash, L.stash_n, L.counter + 4);
}
void bp_grid_write(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
                   unsigned nbuckets, bool overflow) {
  if (B.n_items) IPC_LAUNCH(k_bp_gather, nblk(B.n_items, TB), TB, s)(L.counts, L.offs, L.bp_stash, L.stash_n, B.n_items,
                                                                   L.cand);
  if (overflow && B.n_it)
    IPC_LAUNCH(k_bp_grid<true>, B.n_it, TB, s)(W, E, S, B.itiles, L.counts, L.offs, L.cand, L.g_sorted, L.g_boff,
                                              L.g_bigl, nbuckets - 1, L.bp_stash, L.stash_n, nullptr);
}

void scan_int(hipStream_t s, const int *in, int *out, int n, int *tmp) {
  int nb = nblk(n, SCAN_PER_BLOCK);
  if (nb > 0) IPC_LAUNCH(k_scan1, nb, TB, s)(in, out, n, tmp);
  IPC_LAUNCH(k_scan2, 1, TB, s)(tmp, nb, out + n);
  if (n > 0) IPC_LAUNCH(k_scan3, nblk(n, TB), TB, s)(out, n, tmp);
}

void cand_segments(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L) {
  IPC_LAUNCH(k_cand_seg, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs, L.offs);
}

void classify_cands(hipStream_t s, const WorldDev &W, const EnvDev *E, const Lists &L, int n, const double *x) {
  if (n) IPC_LAUNCH(k_classify, nblk(n, TB), TB, s)(W, E, L.cand, n, x, L.cand_type, L.cand_d2, L.cand_flag);
}
void compact_active(hipStream_t s, const Lists &L, int n) {
  if (n)
    IPC_LAUNCH(k_compact, nblk(n, TB), TB, s)(L.cand, L.cand_type, L.cand_d2, L.cand_flag, L.cand_offs, n, L.act,
                                              L.act_type, L.act_d2);
}
void act_segments(hipStream_t s, const EnvState &S, const Batch &B, const Lists &L) {
  IPC_LAUNCH(k_act_seg, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs, L.cand_offs);
}
void act_stats(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L, int adapt) {
  if (B.n_envs) IPC_LAUNCH(k_act_stats, B.n_envs, TB, s)(E, S, B.envs, L.act_d2, adapt);
}
void barrier_elems(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_act,
                   const double *x) {
  if (!n_act) return;
  int *n_slow = L.counter + 8;
  IPC_LAUNCH(k_fill_int, 1, 64, s)(n_slow, 1, 0);
  IPC_LAUNCH(k_barrier_elems, nblk(n_act, 128), 128, s)(W, E, S.kappa, L.act, L.act_type, n_act, x, L.ce_v, L.ce_g,
                                                        L.ce_H, n_slow, L.bar_slow);
  // few pairs take the full path: a small grid strides over them
  IPC_LAUNCH(k_barrier_elems_full, std::min(nblk(n_act, kFullThreads), 256), kFullThreads, s)(
      W, E, S.kappa, L.act, L.act_type, x, L.ce_v, L.ce_g, L.ce_H, n_slow, L.bar_slow);
}
void friction_setup(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_act) {
  if (n_act)
    IPC_LAUNCH(k_friction_setup, nblk(n_act, TB), TB, s)(W, E, S.kappa, L.act, L.act_type, n_act, L.fv, L.fw, L.fn,
                                                         L.flam, L.fenv, nullptr, nullptr);
}
void cand_restrict(hipStream_t s, const WorldDev &W, const EnvState &S, const Lists &L, int n) {
  if (n) IPC_LAUNCH(k_cand_restrict, nblk(n, TB), TB, s)(W, S, L.cand, n, L.cand_flag);
}
void fric_plan(hipStream_t s, const EnvState &S, const Batch &B, int *nb, int *ne, int *total) {
  IPC_LAUNCH(k_fric_plan, 1, 64, s)(S, B.envs, B.n_envs, nb, ne, total);
}
void fric_merge(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L,
                int n_old, int n_act, const int *nb, const int *ne, int4 *fv2, double *fw2, double *fn2, double *flam2,
                int *fenv2) {
  if (n_old)
    IPC_LAUNCH(k_fric_copy, nblk(n_old, TB), TB, s)(S, n_old, L.fv, L.fw, L.fn, L.flam, L.fenv, nb, fv2, fw2, fn2,
                                                    flam2, fenv2);
  if (n_act)
    IPC_LAUNCH(k_friction_setup, nblk(n_act, TB), TB, s)(W, E, S.kappa, L.act, L.act_type, n_act, fv2, fw2, fn2,
                                                         flam2, fenv2, nb, S.act_beg);
  IPC_LAUNCH(k_fric_commit, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs, nb, ne);
}
void set_phase(hipStream_t s, const EnvState &S, const Batch &B, int ph) {
  IPC_LAUNCH(k_set_phase, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs, ph);
}
void phase_advance(hipStream_t s, const EnvState &S, const Batch &B) {
  IPC_LAUNCH(k_phase_advance, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs);
}
void friction_elems(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_fric,
                    int ce_off, const double *x) {
  if (n_fric)
    IPC_LAUNCH(k_friction_elems, nblk(n_fric, TB), TB, s)(W, E, S, L.fv, L.fw, L.fn, L.flam, L.fenv, n_fric, x,
                                                      L.ce_v + ce_off, L.ce_g + 12 * (size_t)ce_off,
                                                      L.ce_H + 90 * (size_t)ce_off);
}

void incidence(hipStream_t s, const WorldDev &W, const EnvState &S, Lists &L, int n_ce, int nv_world) {
  IPC_LAUNCH(k_fill_int, nblk(nv_world + 1, TB), TB, s)(L.inc_cnt, nv_world + 1, 0);
  IPC_LAUNCH(k_fill_int, nblk(nv_world + 1, TB), TB, s)(L.inc_cur, nv_world + 1, 0);
  if (n_ce) IPC_LAUNCH(k_inc_count, nblk(n_ce, TB), TB, s)(W, S, L.ce_v, n_ce, L.inc_cnt);
  scan_int(s, L.inc_cnt, L.inc_off, nv_world, L.scan_tmp);
}
void incidence_fill(hipStream_t s, const WorldDev &W, const EnvState &S, Lists &L, int n_ce, int nv_world) {
  if (n_ce) {
    IPC_LAUNCH(k_inc_fill, nblk(n_ce, TB), TB, s)(W, S, L.ce_v, n_ce, L.inc_off, L.inc_cur, L.inc_ent);
    IPC_LAUNCH(k_inc_sort, nblk(nv_world, TB), TB, s)(L.inc_off, L.inc_ent, nv_world);
  }
}

void contact_rows(hipStream_t s, Lists &L, int nv_world, int n_inc, int mixed) {
  IPC_LAUNCH(k_contact_row_flags, nblk(nv_world, TB), TB, s)(L.inc_off, nv_world, L.cr_flag, L.cr_cnt);
  scan_int(s, L.cr_flag, L.cr_pos, nv_world, L.scan_tmp);
  IPC_LAUNCH(k_contact_row_list, nblk(nv_world, TB), TB, s)(L.cr_flag, L.cr_pos, nv_world, L.cr_rows);
  // at most one listed row per incidence entry; blocks past the list's length exit
  const int grid = std::min(n_inc, nv_world);
  if (grid > 0)
    IPC_LAUNCH(k_contact_rows, grid, 64, s)(L.cr_rows, L.cr_pos + nv_world, L.inc_off, L.inc_ent, L.ce_v, L.ce_H,
                                           L.cr_key, L.cr_scol, L.cr_ssrc, L.cr_col, L.cr_cnt, L.cr_val, L.cr_val32,
                                           mixed);
}

void elastic(hipStream_t s, const WorldDev &W, const EnvDev *, const EnvState &S, const Batch &B, hipEvent_t start) {
  if (B.n_tt)
    hipExtLaunchKernelGGL(k_elastic, dim3(B.n_tt), dim3(TB), 0, s, start, nullptr, 0, W, S, B.ttiles);
  else if (start)
    (void)hipEventRecord(start, s);
}

void assemble(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, const Lists &L,
              int mixed, hipEvent_t stop) {
  if (!B.n_vt) {
    if (stop) (void)hipEventRecord(stop, s);
    return;
  }
  IPC_LAUNCH(k_assemble_rows, B.n_vt, TB, s)(W, E, S, B.vtiles, L.inc_off, L.inc_ent, L.ce_g, L.ce_H, mixed);
  hipExtLaunchKernelGGL(k_assemble_sell, dim3(B.n_vt), dim3(TB), 0, s, nullptr, stop, 0, W, E, S,
                        (const Tile *)B.vtiles, mixed);
}

void pcg_init(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
              int *pending, int mixed) {
  IPC_LAUNCH(k_fill_int, 1, 64, s)(pending, 1, 0);
  if (B.n_vt && !mixed)
    IPC_LAUNCH(k_pcg_init<double>, B.n_vt, TB, s)(W, E, S, B.vtiles, W.p, W.r, W.z, W.pp, W.q, W.Minv, L.part_b0,
                                                  L.part_c0, L.part_z, L.coarse);
  if (B.n_vt && mixed)
    IPC_LAUNCH(k_pcg_init<float>, B.n_vt, TB, s)(W, E, S, B.vtiles, W.p32, W.r32, W.z32, W.pp32, W.q32, W.Minv32,
                                                 L.part_b0, L.part_c0, L.part_z, L.coarse);
  IPC_LAUNCH(k_pcg_env_init, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs, L.part_c0, pending);
}

void coarse_setup(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B,
                  const Lists &L, int mixed) {
  if (!B.n_vt) return;
  IPC_LAUNCH(k_coarse_hz, B.n_vt, TB, s)(W, E, S, B.vtiles, L.inc_off, L.cr_cnt, L.cr_col, L.cr_val, L.e_tile,
                                         mixed);
  IPC_LAUNCH(k_coarse_factor, B.n_envs, 64, s)(E, S, B.envs, L.e_tile);
}

void live_tiles(hipStream_t s, const EnvState &S, const Batch &B, Lists &L, Tile *out, int *flag, int *offs) {
  if (!B.n_vt) return;
  IPC_LAUNCH(k_live_flags, nblk(B.n_vt, TB), TB, s)(S, B.vtiles, B.n_vt, flag);
  scan_int(s, flag, offs, B.n_vt, L.scan_tmp);
  IPC_LAUNCH(k_live_compact, nblk(B.n_vt, TB), TB, s)(B.vtiles, B.n_vt, flag, offs, out);
}

template <typename T>
const T *cr_vals(const Lists &L);
template <>
const double *cr_vals<double>(const Lists &L) {
  return L.cr_val;
}
template <>
const float *cr_vals<float>(const Lists &L) {
  return L.cr_val32;
}

// the vectors of one precision: solution, residual, preconditioned residual,
// direction, H times direction, H times preconditioned residual
template <typename T>
struct PcgVecs {
  T *x, *r, *u, *pp, *q, *w;
  const T *val, *Minv, *cr_val;
};
PcgVecs<double> vecs64(const WorldDev &W, const Lists &L) {
  return {W.p, W.r, W.z, W.pp, W.q, W.w, W.val, W.Minv, L.cr_val};
}
PcgVecs<float> vecs32(const WorldDev &W, const Lists &L) {
  return {W.p32, W.r32, W.z32, W.pp32, W.q32, W.w32, W.val32, W.Minv32, L.cr_val32};
}

template <typename T>
void pcg_iter_t(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, Lists &L, int it, int *pending,
                const hipEvent_t *ev, bool count, const Tile *tiles, int n_tiles, const PcgVecs<T> &v) {
  // per-tile partials of gamma and r.r: slot it & 1 holds this iteration's,
  // the update writes the next iteration's into the other slot
  double *g_cur = (it & 1) ? L.part_b1 : L.part_b0, *g_new = (it & 1) ? L.part_b0 : L.part_b1;
  double *rr_cur = (it & 1) ? L.part_c1 : L.part_c0, *rr_new = (it & 1) ? L.part_c0 : L.part_c1;
  const int nt = kLPR * TB;
  // a timed launch carries its events in its dispatch (start and end of the
  // kernel itself, as a profiler sees them; no event packets around it)
  hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr, e2 = ev ? ev[2] : nullptr,
             e3 = ev ? ev[3] : nullptr;
  // launches of a few tiles are latency-bound: issue each lane's slots four
  // at a time (not with the two-level PCG, whose loads ahead of the product
  // leave no registers for it)
  const bool wide = n_tiles <= L.wide_tiles;
  auto spmv = [&](auto kern) {
    hipExtLaunchKernelGGL(kern, dim3(n_tiles), dim3(nt), 0, s, e0, e1, 0, W, E, S, tiles, L.inc_off, L.cr_cnt,
                          L.cr_col, v.cr_val, (const T *)v.u, v.w, v.val, L.part_a, (const double *)L.part_z);
  };
  if (L.coarse)
    spmv(k_spmv<T, false, true>);
  else
    wide ? spmv(k_spmv<T, true, false>) : spmv(k_spmv<T, false, false>);
  if (ev) {
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) throw std::runtime_error(std::string("timed product launch: ") + hipGetErrorString(le));
  }
  // the iteration's algorithmic bytes (product: counter 0 for launches of at
  // most kWideTiles tiles, 1 for larger ones; whole iteration: counter 2),
  // counted between the two kernels, outside both timings
  if (count)
    IPC_LAUNCH(k_pcg_bytes<T>, n_tiles, TB, s)(W, E, S, tiles, L.cr_cnt, L.coarse,
                                               L.prof + (n_tiles > kWideTiles ? 1 : 0), L.prof + 2);
  hipExtLaunchKernelGGL(k_pcg_update<T>, dim3(n_tiles), dim3(TB), 0, s, e2, e3, 0, W, E, S, tiles, it,
                        (const double *)L.part_a, (const double *)g_cur, (const double *)rr_cur, g_new, rr_new, v.x,
                        v.r, v.u, v.pp, v.q, (const T *)v.w, v.Minv, pending, L.part_z, L.coarse);
}

void pcg_iter(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, Lists &L, int it, int *pending,
              int mixed, const hipEvent_t *ev, bool count, const Tile *tiles, int n_tiles) {
  if (!n_tiles) return;
  if (!mixed)
    pcg_iter_t<double>(s, W, E, S, L, it, pending, ev, count, tiles, n_tiles, vecs64(W, L));
  else
    pcg_iter_t<float>(s, W, E, S, L, it, pending, ev, count, tiles, n_tiles, vecs32(W, L));
}
void asm_bytes(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, int mixed,
               unsigned long long *prof) {
  IPC_LAUNCH(k_asm_bytes, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs, mixed, prof);
}

void pcg_fused(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const int *fenv, int n_fenv,
               Lists &L, int mixed) {
  if (!n_fenv) return;
  auto go = [&](auto v) {
    using T = std::remove_pointer_t<decltype(v.x)>;
    IPC_LAUNCH(k_pcg_fused<T>, n_fenv, FB, s)(W, E, S, fenv, L.inc_off, L.cr_cnt, L.cr_col, v.cr_val, v.x, v.r, v.u,
                                              v.pp, v.q, v.w, v.val, v.Minv, L.part_a, L.part_b0, L.part_b1,
                                              L.part_c0, L.part_c1);
  };
  if (!mixed)
    go(vecs64(W, L));
  else
    go(vecs32(W, L));
}

void pcg_resume(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, Lists &L, const Tile *tiles,
                int n_tiles, int it, int mixed) {
  if (!n_tiles) return;
  auto go = [&](auto v) {
    using T = std::remove_pointer_t<decltype(v.x)>;
    IPC_LAUNCH(k_pcg_resume<T>, n_tiles, FB, s)(W, E, S, tiles, it, L.inc_off, L.cr_cnt, L.cr_col, v.cr_val, v.x, v.r,
                                                v.u, v.pp, v.q, v.w, v.val, v.Minv, L.part_a, L.part_b0, L.part_b1,
                                                L.part_c0, L.part_c1);
  };
  if (!mixed)
    go(vecs64(W, L));
  else
    go(vecs32(W, L));
}

void pcg_finish(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B, int mixed) {
  if (mixed && B.n_vt) IPC_LAUNCH(k_p32_to_p, B.n_vt, TB, s)(W, S, B.vtiles);
}

void spmv_debug(hipStream_t s, const WorldDev &W, const EnvDev *, const EnvState &S, const Batch &B, Lists &L,
                const double *in, double *out) {
  if (B.n_vt) IPC_LAUNCH(k_spmv_dbg, B.n_vt, kLPR * TB, s)(W, S, B.vtiles, L.inc_off, L.cr_cnt, L.cr_col, L.cr_val, in, out);
}

void conv_check(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L,
                int *n_active) {
  IPC_LAUNCH(k_fill_int, 1, 64, s)(n_active, 1, 0);
  if (B.n_vt) IPC_LAUNCH(k_pinf, B.n_vt, TB, s)(W, S, B.vtiles, L.part_a, L.part_b0);
  IPC_LAUNCH(k_env_conv, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs, L.part_a, L.part_b0, n_active);
}

void al_prepare(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B) {
  if (B.n_vt) IPC_LAUNCH(k_al_prepare, B.n_vt, TB, s)(W, S, B.vtiles);
}
void snap_J(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B) {
  if (B.n_tt) IPC_LAUNCH(k_snap_J, B.n_tt, TB, s)(W, S, B.ttiles);
}
void al_finish(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B) {
  IPC_LAUNCH(k_al_decide, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs);
  if (B.n_vt) IPC_LAUNCH(k_al_vertex, B.n_vt, TB, s)(E, W, S, B.vtiles);
  IPC_LAUNCH(k_al_env, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs);
}

void ccd_init(hipStream_t s, const EnvState &S, const Batch &B) {
  IPC_LAUNCH(k_ccd_init, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs);
}
void accd(hipStream_t s, const WorldDev &W, const EnvDev *, const EnvState &S, const Lists &L, int n, const double *x,
          const double *p) {
  if (n) IPC_LAUNCH(k_accd, nblk(n, 128), 128, s)(W, S, L.cand, n, x, p);
}
void inv_bound(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, int force) {
  if (B.n_tt) IPC_LAUNCH(k_inv_bound, B.n_tt, TB, s)(W, E, S, B.ttiles, force);
}
void relag(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, int sel, int *n_relag) {
  IPC_LAUNCH(k_fill_int, 1, 64, s)(n_relag, 1, 0);
  IPC_LAUNCH(k_relag, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs, sel, n_relag);
}
void ls_init(hipStream_t s, const EnvState &S, const Batch &B) {
  IPC_LAUNCH(k_ls_init, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs);
}

void energy(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, Lists &L, int n_cand,
            int n_fric, int zero_alpha, double *E_out) {
  if (B.n_vt) IPC_LAUNCH(k_energy_v, B.n_vt, TB, s)(W, E, S, B.vtiles, zero_alpha);
  if (B.n_tt) IPC_LAUNCH(k_energy_t, B.n_tt, TB, s)(W, S, B.ttiles, zero_alpha);
  if (n_cand) IPC_LAUNCH(k_energy_c, nblk(n_cand, TB), TB, s)(W, E, S, L.cand, n_cand, zero_alpha, L.e_c);
  if (n_fric)
    IPC_LAUNCH(k_energy_f, nblk(n_fric, TB), TB, s)(W, E, S, L.fv, L.fw, L.fn, L.flam, L.fenv, n_fric, zero_alpha, L.e_f);
  IPC_LAUNCH(k_env_energy, B.n_envs, TB, s)(W, E, S, B.envs, L.e_c, L.e_f, E_out);
}

void ls_decide(hipStream_t s, const EnvState &S, const Batch &B, int *pending) {
  IPC_LAUNCH(k_fill_int, 1, 64, s)(pending, 1, 0);
  IPC_LAUNCH(k_ls_decide, nblk(B.n_envs, 64), 64, s)(S, B.envs, B.n_envs, pending);
}
void update_x(hipStream_t s, const WorldDev &W, const EnvState &S, const Batch &B) {
  if (B.n_vt) IPC_LAUNCH(k_update_x, B.n_vt, TB, s)(W, S, B.vtiles);
}
void iter_end(hipStream_t s, const EnvDev *E, const EnvState &S, const Batch &B, int *n_active) {
  IPC_LAUNCH(k_fill_int, 1, 64, s)(n_active, 1, 0);
  IPC_LAUNCH(k_iter_end, nblk(B.n_envs, 64), 64, s)(E, S, B.envs, B.n_envs, n_active);
}
void step_end(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Batch &B, int sel) {
  if (B.n_vt) IPC_LAUNCH(k_step_end, B.n_vt, TB, s)(W, E, S, B.vtiles, sel);
}

void stress(hipStream_t s, const WorldDev &W, int t_off, int nt, double *cauchy, double *vm) {
  if (nt) IPC_LAUNCH(k_stress, nblk(nt, TB), TB, s)(W, t_off, nt, cauchy, vm);
}

void dbg_classify(hipStream_t s, int kind, int n, const double *x12, int *types, double *d2) {
  if (n) IPC_LAUNCH(k_dbg_classify, nblk(n, TB), TB, s)(kind, n, x12, types, d2);
}
void dbg_pair(hipStream_t s, int kind, int type, const double *x12, double dhat, double kappa, double eps_x,
              int project, double *out) {
  IPC_LAUNCH(k_dbg_pair, 1, 64, s)(kind, type, x12, dhat, kappa, eps_x, project, out);
}
void dbg_tet(hipStream_t s, const double *X12, const double *x12, double mu, double la, double *out) {
  IPC_LAUNCH(k_dbg_tet, 1, 64, s)(X12, x12, mu, la, out);
}
int pairs_ccd_parts(int64_t n) { return (int)((n + kCcdBlock - 1) / kCcdBlock); }

int64_t noalloc_max_pairs() { return (int64_t)kNoAllocParts * kCcdBlock; }

// Address of the current device's copy of ccd_scratch, looked up once per
// device and kept (no allocation: a fixed table indexed by device ordinal).
hipError_t noalloc_scratch(double **ptr) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static double *addr[kMaxDev] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(ccd_scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double *>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}
void pairs_ccd_bound(hipStream_t s, int kind, int n, const double *x12, const double *p12, double sfac, double *part,
                     double *out) {
  const int nb = pairs_ccd_parts(n);
  if (nb) IPC_LAUNCH(k_pairs_ccd_min, nb, kCcdBlock, s)(kind, n, x12, p12, sfac, part);
  IPC_LAUNCH(k_min_reduce, 1, TB, s)(part, nb, out);
}
void contact_forces(hipStream_t s, const WorldDev &W, const EnvDev *E, const EnvState &S, const Lists &L, int n_act,
                    const int *tag, int v_off, int ntags, double *f, int *fab, double *out) {
  if (n_act)
    IPC_LAUNCH(k_pair_force, nblk(n_act, TB), TB, s)(W, E, S.kappa, L.act, L.act_type, n_act, tag, v_off, ntags, f,
                                                     fab);
  IPC_LAUNCH(k_tag_force_sum, ntags * ntags, TB, s)(f, fab, n_act, ntags, out);
}
int sdf_parts(int n_samples) { return (n_samples + kSdfTile - 1) / kSdfTile; }
void grasp_metrics(hipStream_t s, const double *x, const int *obj_tris, int n_obj, const int *hand_tris,
                   const int *sample_tri, const double *sample_uv, int n_samples, double *sdf, double *part,
                   double *out) {
  const int nb = sdf_parts(n_samples);
  if (nb)
    IPC_LAUNCH(k_sdf_samples, nb, kSdfTile, s)(x, obj_tris, n_obj, hand_tris, sample_tri, sample_uv, n_samples, sdf,
                                               part);
  IPC_LAUNCH(k_max_reduce, 1, TB, s)(part, nb, out);
}
void dbg_tet_root(hipStream_t s, int n, const double *x12, const double *p12, double tmax, double *t, double *k4) {
  if (n) IPC_LAUNCH(k_dbg_tet_root, nblk(n, 64), 64, s)(n, x12, p12, tmax, t, k4);
}
void dbg_accd(hipStream_t s, int kind, int n, const double *x12, const double *p12, double sfac, double *t) {
  if (n) IPC_LAUNCH(k_dbg_accd, nblk(n, 128), 128, s)(kind, n, x12, p12, sfac, t);
}

}  // namespace ipck
