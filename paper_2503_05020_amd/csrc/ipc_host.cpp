// ipc_host.cpp -- scene preprocessing, the device world, the batched Newton
// driver and the C-ABI of include/ipc.h.
//
// The driver follows the per-environment solver structure of Sec. III-A:
// all environments of a batch share every kernel launch, while each keeps
// its own contact set (no cross-environment pairs), CCD step bound, line
// search, convergence flag and failure flag; converged and failed
// environments are skipped by every later launch of the step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <cstring>
#include <map>
#include <memory>
#include <condition_variable>
#include <deque>
#include <exception>
#include <mutex>
#include <thread>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ipc.h"
#include "device_math.h"
#include "ipc_kernels.h"
#include "ipc_world.h"

using ipcw::EnvDev;
using ipcw::EnvState;
using ipcw::Tile;
using ipcw::WorldDev;

namespace {

// message of the last error on this thread (fixed storage: setting it never allocates)
thread_local char g_err[512];
void set_err(const char *m) {
  std::strncpy(g_err, m ? m : "", sizeof g_err - 1);
  g_err[sizeof g_err - 1] = 0;
}

struct ApiError : std::runtime_error {
  int code;
  ApiError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw ApiError(IPC_E_NOMEM, std::string("out of device memory in ") + what);
    throw ApiError(IPC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define HC(x) hip_check((x), #x)

// ---------------------------------------------------------------------------
// growable device buffers and range allocators
// ---------------------------------------------------------------------------
struct RawBuf {
  void **slot;
  size_t elem;
};

// Element-range allocator with a first-fit free list; all arrays registered
// with an arena share its index space and grow together.
struct Arena {
  size_t cap = 0, top = 0, align = 1;
  std::vector<std::pair<size_t, size_t>> free_list;  // (offset, length), sorted
  std::vector<RawBuf> bufs;

  size_t alloc(size_t n) {
    n = (n + align - 1) / align * align;
    if (n == 0) return top;
    for (size_t i = 0; i < free_list.size(); ++i)
      if (free_list[i].second >= n) {
        size_t off = free_list[i].first;
        free_list[i].first += n;
        free_list[i].second -= n;
        if (free_list[i].second == 0) free_list.erase(free_list.begin() + i);
        return off;
      }
    size_t off = top;
    top += n;
    return off;
  }
  void release(size_t off, size_t n) {
    n = (n + align - 1) / align * align;
    if (n == 0) return;
    free_list.push_back({off, n});
    std::sort(free_list.begin(), free_list.end());
    std::vector<std::pair<size_t, size_t>> merged;
    for (auto &f : free_list) {
      if (!merged.empty() && merged.back().first + merged.back().second == f.first)
        merged.back().second += f.second;
      else
        merged.push_back(f);
    }
    if (!merged.empty() && merged.back().first + merged.back().second == top) {
      top = merged.back().first;
      merged.pop_back();
    }
    free_list = merged;
  }
  // make room for top elements; existing contents are preserved
  void reserve(hipStream_t s) {
    if (top <= cap) return;
    size_t nc = std::max(top, cap + cap / 2);
    nc = (nc + 255) / 256 * 256;
    HC(hipStreamSynchronize(s));
    for (RawBuf &b : bufs) {
      void *q = nullptr;
      HC(hipMalloc(&q, nc * b.elem));
      if (*b.slot && cap) HC(hipMemcpy(q, *b.slot, cap * b.elem, hipMemcpyDeviceToDevice));
      if (*b.slot) HC(hipFree(*b.slot));
      *b.slot = q;
    }
    cap = nc;
  }
};

template <class T>
struct DBuf {
  T *p = nullptr;
  size_t cap = 0;
  // grows to hold at least n elements (contents are not kept); returns true
  // if the buffer moved
  bool ensure(size_t n) {
    if (n <= cap) return false;
    size_t nc = std::max(n, cap + cap / 2);
    nc = std::max<size_t>(nc, 64);
    if (p) HC(hipFree(p));
    p = nullptr;
    HC(hipMalloc(&p, nc * sizeof(T)));
    cap = nc;
    return true;
  }
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
};

// ---------------------------------------------------------------------------
// host-side preprocessing of one scene
// ---------------------------------------------------------------------------
struct HostScene {
  int nv = 0, nv_pad = 0, nt = 0, ntri = 0, ne = 0, nsv = 0, npos = 0, n_free = 0;
  std::vector<double> X, x0, v0, mass, Dinv, vol, mu, la;
  std::vector<int> kin, tets;
  std::vector<std::array<int, 3>> tris;
  std::vector<std::array<int, 2>> edges;
  std::vector<int> sverts;
  std::vector<double> elen2;
  std::vector<int> vt_beg, vt_end, vt_ent;  // local tet*4+slot
  std::vector<int> row_nnz;                  // stored blocks per row (without ELL padding)
  std::vector<int> slice_pos, slice_w;       // per local slice (positions local)
  std::vector<int> col, cb_beg, cb_end, contrib;
  std::vector<double> motion;  // motion rows then gravity rows
  int n_groups = 0, n_motion = 0;
  double cell = 0.0;  // hash-grid cell size
  double mbar = 1.0;  // mean free-vertex mass
  double dt, dhat, kappa, mu_f, eps_v, tol, pcg_tol;
  int maxit, precision;
  int fric_iters = 1, inv_filter = 0, adapt_kappa = 0;
  // coarse space of the PCG: body of each free vertex (-1: none), bodies'
  // reference points and lengths
  std::vector<int> vbody;
  int nbody = 0;
  double cb[ipcw::kCoarseBodies][3] = {}, cscale[ipcw::kCoarseBodies] = {};
};

bool finite_all(const double *p, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

double det3h(const double *M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) + M[2] * (M[3] * M[7] - M[4] * M[6]);
}

void inv3h(const double *M, double *R) {
  double id = 1.0 / det3h(M);
  R[0] = (M[4] * M[8] - M[5] * M[7]) * id;
  R[1] = (M[2] * M[7] - M[1] * M[8]) * id;
  R[2] = (M[1] * M[5] - M[2] * M[4]) * id;
  R[3] = (M[5] * M[6] - M[3] * M[8]) * id;
  R[4] = (M[0] * M[8] - M[2] * M[6]) * id;
  R[5] = (M[2] * M[3] - M[0] * M[5]) * id;
  R[6] = (M[3] * M[7] - M[4] * M[6]) * id;
  R[7] = (M[1] * M[6] - M[0] * M[7]) * id;
  R[8] = (M[0] * M[4] - M[1] * M[3]) * id;
}

// signed volume factor of (a, b, c, d)
double orient(const double *a, const double *b, const double *c, const double *d) {
  double u[3], v[3], w[3];
  for (int k = 0; k < 3; ++k) {
    u[k] = b[k] - a[k];
    v[k] = c[k] - a[k];
    w[k] = d[k] - a[k];
  }
  return u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) + u[2] * (v[0] * w[1] - v[1] * w[0]);
}

// Segment (a, b) crosses triangle (t0, t1, t2): strict opposite sides of the
// plane and strictly inside the triangle, each by more than 1e-9 L^3 with L
// the longest distance among the five points, so that coplanar or touching
// neighbours of a valid mesh (orientations at rounding level) are not flagged.
bool seg_tri_cross(const double *a, const double *b, const double *t0, const double *t1, const double *t2) {
  const double *P[5] = {a, b, t0, t1, t2};
  double L2 = 0.0;
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += (P[i][k] - P[j][k]) * (P[i][k] - P[j][k]);
      L2 = std::max(L2, s);
    }
  double eps = 1e-9 * L2 * std::sqrt(L2);
  double da = orient(t0, t1, t2, a), db = orient(t0, t1, t2, b);
  if (!((da > eps && db < -eps) || (da < -eps && db > eps))) return false;
  double s0 = orient(a, b, t0, t1), s1 = orient(a, b, t1, t2), s2 = orient(a, b, t2, t0);
  return (s0 > eps && s1 > eps && s2 > eps) || (s0 < -eps && s1 < -eps && s2 < -eps);
}

struct Box {
  double lo[3], hi[3];
};

// sweep-and-prune over x of two box lists: calls f(i, j) for every
// overlapping pair (i from A, j from B); same=true enumerates i<j within A.
template <class F>
void sweep_pairs(const std::vector<Box> &A, const std::vector<Box> &B, bool same, F f) {
  std::vector<int> ia(A.size()), ib(B.size());
  for (size_t i = 0; i < A.size(); ++i) ia[i] = (int)i;
  for (size_t i = 0; i < B.size(); ++i) ib[i] = (int)i;
  auto cmpA = [&](int p, int q) { return A[p].lo[0] < A[q].lo[0]; };
  auto cmpB = [&](int p, int q) { return B[p].lo[0] < B[q].lo[0]; };
  std::sort(ia.begin(), ia.end(), cmpA);
  if (same) {
    for (size_t s = 0; s < ia.size(); ++s) {
      const Box &a = A[ia[s]];
      for (size_t t = s + 1; t < ia.size(); ++t) {
        const Box &b = A[ia[t]];
        if (b.lo[0] > a.hi[0]) break;
        if (a.lo[1] <= b.hi[1] && b.lo[1] <= a.hi[1] && a.lo[2] <= b.hi[2] && b.lo[2] <= a.hi[2])
          f(std::min(ia[s], ia[t]), std::max(ia[s], ia[t]));
      }
    }
    return;
  }
  std::sort(ib.begin(), ib.end(), cmpB);
  size_t start = 0;
  for (size_t s = 0; s < ia.size(); ++s) {
    const Box &a = A[ia[s]];
    while (start < ib.size() && B[ib[start]].hi[0] < a.lo[0] - 1e30) ++start;
    for (size_t t = 0; t < ib.size(); ++t) {
      const Box &b = B[ib[t]];
      if (b.lo[0] > a.hi[0]) break;
      if (b.hi[0] < a.lo[0]) continue;
      if (a.lo[1] <= b.hi[1] && b.lo[1] <= a.hi[1] && a.lo[2] <= b.hi[2] && b.lo[2] <= a.hi[2]) f(ia[s], ib[t]);
    }
  }
}

Box make_box(const std::vector<double> &x, const int *v, int n, double pad) {
  Box b;
  for (int k = 0; k < 3; ++k) {
    b.lo[k] = ipcdev::kInf;
    b.hi[k] = -ipcdev::kInf;
  }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      b.lo[k] = std::min(b.lo[k], x[3 * v[i] + k]);
      b.hi[k] = std::max(b.hi[k], x[3 * v[i] + k]);
    }
  for (int k = 0; k < 3; ++k) {
    b.lo[k] -= pad;
    b.hi[k] += pad;
  }
  return b;
}

std::unique_ptr<HostScene> preprocess(const ipc_scene_desc *d) {
  if (!d) throw ApiError(IPC_E_ARG, "null descriptor");
  if (d->n_verts <= 0 || !d->rest_pos || !d->kin_group) throw ApiError(IPC_E_ARG, "no vertices");
  if (d->n_tets < 0 || (d->n_tets > 0 && (!d->tets || !d->E || !d->nu || !d->rho)))
    throw ApiError(IPC_E_ARG, "tet arrays missing");
  if (d->n_tris < 0 || (d->n_tris > 0 && !d->tris)) throw ApiError(IPC_E_ARG, "triangle array missing");
  if (d->n_motion_steps < 1 || d->n_groups < 0 || !d->gravity || (d->n_groups > 0 && !d->motion))
    throw ApiError(IPC_E_ARG, "motion schedule missing");
  if (!(d->dt > 0) || !(d->dhat > 0) || !(d->kappa > 0) || !(d->mu >= 0) || !(d->eps_v > 0) ||
      !(d->newton_tol > 0) || d->newton_max_iter < 1 || !(d->pcg_rel_tol > 0) || !std::isfinite(d->dt) ||
      !std::isfinite(d->dhat) || !std::isfinite(d->kappa) || !std::isfinite(d->mu))
    throw ApiError(IPC_E_ARG, "bad solver parameter");
  if (d->precision != IPC_FP64 && d->precision != IPC_MIXED) throw ApiError(IPC_E_ARG, "bad precision flag");
  if (!(d->newton_rel_tol >= 0) || !std::isfinite(d->newton_rel_tol) || d->friction_iters < 0 ||
      d->inversion_filter < 0 || d->adaptive_kappa < 0)
    throw ApiError(IPC_E_ARG, "bad solver variant");
  if ((long)d->n_tets * 32 >= (1L << 31)) throw ApiError(IPC_E_ARG, "too many tets for one scene");
  auto S = std::make_unique<HostScene>();
  HostScene &H = *S;
  H.nv = d->n_verts;
  H.nt = d->n_tets;
  long nv3 = 3L * H.nv;
  if (!finite_all(d->rest_pos, nv3) || (d->init_pos && !finite_all(d->init_pos, nv3)) ||
      (d->init_vel && !finite_all(d->init_vel, nv3)))
    throw ApiError(IPC_E_ARG, "non-finite vertex data");
  H.X.assign(d->rest_pos, d->rest_pos + nv3);
  H.x0 = d->init_pos ? std::vector<double>(d->init_pos, d->init_pos + nv3) : H.X;
  H.v0 = d->init_vel ? std::vector<double>(d->init_vel, d->init_vel + nv3) : std::vector<double>(nv3, 0.0);
  H.kin.assign(d->kin_group, d->kin_group + H.nv);
  H.n_groups = d->n_groups;
  H.n_motion = d->n_motion_steps;
  for (int k : H.kin)
    if (k < -1 || k >= H.n_groups) throw ApiError(IPC_E_ARG, "kin_group out of range");
  if (H.n_groups > 0) H.motion.assign(d->motion, d->motion + 12L * H.n_groups * H.n_motion);
  H.motion.insert(H.motion.end(), d->gravity, d->gravity + 3L * H.n_motion);
  if (!finite_all(H.motion.data(), (long)H.motion.size())) throw ApiError(IPC_E_ARG, "non-finite motion");
  // controls of the grasp-validation protocol after the schedule: per group
  // the motion row it is held at (-1: none), then the gravity override
  // (flag, g); see ipc_hold_group / ipc_set_gravity
  H.motion.insert(H.motion.end(), (size_t)H.n_groups, -1.0);
  H.motion.insert(H.motion.end(), 4, 0.0);
  H.dt = d->dt;
  H.dhat = d->dhat;
  H.kappa = d->kappa;
  H.mu_f = d->mu;
  H.eps_v = d->eps_v;
  H.tol = d->newton_tol;
  H.maxit = d->newton_max_iter;
  H.pcg_tol = d->pcg_rel_tol;
  H.precision = d->precision;
  H.tets.assign(d->tets, d->tets + 4L * H.nt);
  for (int v : H.tets)
    if (v < 0 || v >= H.nv) throw ApiError(IPC_E_ARG, "tet index out of range");
  H.Dinv.resize(9L * H.nt);
  H.vol.resize(H.nt);
  H.mu.resize(H.nt);
  H.la.resize(H.nt);
  H.mass.assign(H.nv, 0.0);
  for (int e = 0; e < H.nt; ++e) {
    double E = d->E[e], nu = d->nu[e], rho = d->rho[e];
    if (!(E > 0) || !(nu > -1.0 && nu < 0.5) || !(rho > 0) || !std::isfinite(E) || !std::isfinite(rho))
      throw ApiError(IPC_E_ARG, "bad material");
    const int *t = &H.tets[4 * e];
    double Dm[9];
    for (int i = 0; i < 3; ++i)
      for (int a = 0; a < 3; ++a) Dm[i * 3 + a] = H.X[3 * t[a + 1] + i] - H.X[3 * t[0] + i];
    double det = det3h(Dm);
    if (!(det > 0.0)) throw ApiError(IPC_E_INVERTED, "tet with non-positive rest volume");
    inv3h(Dm, &H.Dinv[9 * e]);
    H.vol[e] = det / 6.0;
    H.mu[e] = E / (2.0 * (1.0 + nu));
    H.la[e] = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    for (int k = 0; k < 4; ++k) H.mass[t[k]] += rho * H.vol[e] / 4.0;
    // initial J > 0
    double Ds[9], F[9];
    for (int i = 0; i < 3; ++i)
      for (int a = 0; a < 3; ++a) Ds[i * 3 + a] = H.x0[3 * t[a + 1] + i] - H.x0[3 * t[0] + i];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        F[i * 3 + j] = Ds[i * 3] * H.Dinv[9 * e + j] + Ds[i * 3 + 1] * H.Dinv[9 * e + 3 + j] +
                       Ds[i * 3 + 2] * H.Dinv[9 * e + 6 + j];
    if (!(det3h(F) > 0.0)) throw ApiError(IPC_E_INVERTED, "inverted tet in the initial configuration");
  }
  double msum = 0.0;
  for (int i = 0; i < H.nv; ++i) {
    if (H.kin[i] < 0 && !(H.mass[i] > 0.0)) throw ApiError(IPC_E_ARG, "free vertex without mass");
    if (H.kin[i] < 0) {
      ++H.n_free;
      msum += H.mass[i];
    }
  }
  H.mbar = H.n_free > 0 ? msum / H.n_free : 1.0;
  H.fric_iters = std::max(1, (int)d->friction_iters);
  H.inv_filter = d->inversion_filter != 0;
  H.adapt_kappa = d->adaptive_kappa != 0;
  if (d->newton_rel_tol > 0) {
    // the paper's relative Newton tolerance (Sec. III-D): eps_r times the
    // diagonal of the free vertices' bounding box at creation
    double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int i = 0; i < H.nv; ++i)
      if (H.kin[i] < 0)
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], H.x0[3 * i + k]);
          hi[k] = std::max(hi[k], H.x0[3 * i + k]);
        }
    double diag2 = 0.0;
    if (H.n_free > 0)
      for (int k = 0; k < 3; ++k) diag2 += (hi[k] - lo[k]) * (hi[k] - lo[k]);
    H.tol = d->newton_rel_tol * std::sqrt(diag2);
  }
  // surface: boundary faces (used by one tet) + kinematic triangles, each with
  // ascending vertex ids, list sorted lexicographically; edges (min,max) sorted
  {
    std::vector<std::array<int, 3>> faces;
    faces.reserve(4L * H.nt);
    for (int e = 0; e < H.nt; ++e) {
      const int *t = &H.tets[4 * e];
      const int F[4][3] = {{t[0], t[1], t[2]}, {t[0], t[1], t[3]}, {t[0], t[2], t[3]}, {t[1], t[2], t[3]}};
      for (auto &f : F) {
        std::array<int, 3> k = {f[0], f[1], f[2]};
        std::sort(k.begin(), k.end());
        faces.push_back(k);
      }
    }
    std::sort(faces.begin(), faces.end());
    for (size_t i = 0; i < faces.size();) {
      size_t j = i;
      while (j < faces.size() && faces[j] == faces[i]) ++j;
      if (j - i == 1) H.tris.push_back(faces[i]);
      i = j;
    }
    for (int i = 0; i < d->n_tris; ++i) {
      std::array<int, 3> k = {d->tris[3 * i], d->tris[3 * i + 1], d->tris[3 * i + 2]};
      for (int c = 0; c < 3; ++c)
        if (k[c] < 0 || k[c] >= H.nv || H.kin[k[c]] < 0)
          throw ApiError(IPC_E_ARG, "kinematic triangle with bad or free vertex");
      std::sort(k.begin(), k.end());
      H.tris.push_back(k);
    }
    std::sort(H.tris.begin(), H.tris.end());
    H.tris.erase(std::unique(H.tris.begin(), H.tris.end()), H.tris.end());
    for (auto &t : H.tris) {
      H.edges.push_back({t[0], t[1]});
      H.edges.push_back({t[1], t[2]});
      H.edges.push_back({t[0], t[2]});
      H.sverts.push_back(t[0]);
      H.sverts.push_back(t[1]);
      H.sverts.push_back(t[2]);
    }
    std::sort(H.edges.begin(), H.edges.end());
    H.edges.erase(std::unique(H.edges.begin(), H.edges.end()), H.edges.end());
    std::sort(H.sverts.begin(), H.sverts.end());
    H.sverts.erase(std::unique(H.sverts.begin(), H.sverts.end()), H.sverts.end());
    H.ntri = (int)H.tris.size();
    H.ne = (int)H.edges.size();
    H.nsv = (int)H.sverts.size();
    H.elen2.resize(H.ne);
    for (int i = 0; i < H.ne; ++i) {
      double s = 0;
      for (int k = 0; k < 3; ++k) {
        double a = H.X[3 * H.edges[i][1] + k] - H.X[3 * H.edges[i][0] + k];
        s += a * a;
      }
      H.elen2[i] = s;
    }
    // grid cell: median surface edge length plus the two dhat margins, so a
    // typical widened edge box spans at most two cells per axis
    if (H.ne > 0) {
      std::vector<double> len(H.elen2);
      std::nth_element(len.begin(), len.begin() + len.size() / 2, len.end());
      H.cell = std::sqrt(len[len.size() / 2]) + 2.0 * H.dhat;
    } else {
      H.cell = 1.0;
    }
  }
  // the initial configuration must be free of intersections: no candidate
  // pair at zero distance and no surface edge crossing a surface triangle
  {
    std::vector<Box> bv(H.nsv), bt(H.ntri), be(H.ne);
    for (int i = 0; i < H.nsv; ++i) bv[i] = make_box(H.x0, &H.sverts[i], 1, H.dhat);
    for (int i = 0; i < H.ntri; ++i) bt[i] = make_box(H.x0, H.tris[i].data(), 3, H.dhat);
    for (int i = 0; i < H.ne; ++i) be[i] = make_box(H.x0, H.edges[i].data(), 2, H.dhat);
    auto allkin = [&](const int *v, int n) {
      for (int i = 0; i < n; ++i)
        if (H.kin[v[i]] < 0) return false;
      return true;
    };
    bool bad = false;
    sweep_pairs(bv, bt, false, [&](int i, int j) {
      int p = H.sverts[i];
      const auto &t = H.tris[j];
      if (p == t[0] || p == t[1] || p == t[2]) return;
      int all[4] = {p, t[0], t[1], t[2]};
      if (allkin(all, 4)) return;
      double xx[12], d2;
      for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 3; ++k) xx[3 * a + k] = H.x0[3 * all[a] + k];
      ipcdev::classify(0, xx, &d2);
      if (!(d2 > 0.0)) bad = true;
    });
    sweep_pairs(be, be, true, [&](int i, int j) {
      const auto &A = H.edges[i], &B = H.edges[j];
      if (A[0] == B[0] || A[0] == B[1] || A[1] == B[0] || A[1] == B[1]) return;
      int all[4] = {A[0], A[1], B[0], B[1]};
      if (allkin(all, 4)) return;
      double xx[12], d2;
      for (int a = 0; a < 4; ++a)
        for (int k = 0; k < 3; ++k) xx[3 * a + k] = H.x0[3 * all[a] + k];
      ipcdev::classify(1, xx, &d2);
      if (!(d2 > 0.0)) bad = true;
    });
    sweep_pairs(be, bt, false, [&](int i, int j) {
      const auto &E = H.edges[i];
      const auto &t = H.tris[j];
      for (int a = 0; a < 2; ++a)
        if (E[a] == t[0] || E[a] == t[1] || E[a] == t[2]) return;
      int all[5] = {E[0], E[1], t[0], t[1], t[2]};
      if (allkin(all, 5)) return;
      if (seg_tri_cross(&H.x0[3 * E[0]], &H.x0[3 * E[1]], &H.x0[3 * t[0]], &H.x0[3 * t[1]], &H.x0[3 * t[2]]))
        bad = true;
    });
    if (bad) throw ApiError(IPC_E_INTERSECTING, "intersecting initial configuration");
  }
  // vertex -> (tet, slot) incidence, ascending tet id
  H.nv_pad = (H.nv + ipcw::kSlice - 1) / ipcw::kSlice * ipcw::kSlice;
  H.vt_beg.assign(H.nv_pad, 0);
  H.vt_end.assign(H.nv_pad, 0);
  {
    std::vector<int> cnt(H.nv_pad + 1, 0);
    for (int e = 0; e < H.nt; ++e)
      for (int a = 0; a < 4; ++a) cnt[H.tets[4 * e + a] + 1]++;
    for (int i = 0; i < H.nv_pad; ++i) cnt[i + 1] += cnt[i];
    H.vt_ent.resize(4L * H.nt);
    std::vector<int> cur(cnt.begin(), cnt.end() - 1);
    for (int e = 0; e < H.nt; ++e)
      for (int a = 0; a < 4; ++a) H.vt_ent[cur[H.tets[4 * e + a]]++] = 4 * e + a;
    for (int i = 0; i < H.nv_pad; ++i) {
      H.vt_beg[i] = cnt[i];
      H.vt_end[i] = cnt[i + 1];
    }
  }
  // sliced-ELL pattern: row i holds itself (slot 0) and the vertices sharing
  // a tet with it, ascending; contributors per slot in ascending tet order
  {
    std::vector<std::vector<int>> nbr(H.nv_pad);
    for (int i = 0; i < H.nv_pad; ++i) nbr[i].push_back(i);
    for (int e = 0; e < H.nt; ++e)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          if (a != b) nbr[H.tets[4 * e + a]].push_back(H.tets[4 * e + b]);
    for (int i = 0; i < H.nv_pad; ++i) {
      std::sort(nbr[i].begin() + 1, nbr[i].end());
      nbr[i].erase(std::unique(nbr[i].begin() + 1, nbr[i].end()), nbr[i].end());
      nbr[i].erase(std::remove(nbr[i].begin() + 1, nbr[i].end(), i), nbr[i].end());
    }
    H.row_nnz.resize(H.nv_pad);
    for (int i = 0; i < H.nv_pad; ++i) H.row_nnz[i] = (int)nbr[i].size();
    int nsl = H.nv_pad / ipcw::kSlice;
    H.slice_pos.resize(nsl);
    H.slice_w.resize(nsl);
    int pos = 0;
    for (int s = 0; s < nsl; ++s) {
      int w = 0;
      for (int l = 0; l < ipcw::kSlice; ++l) w = std::max(w, (int)nbr[s * ipcw::kSlice + l].size());
      H.slice_pos[s] = pos;
      H.slice_w[s] = w;
      pos += w * ipcw::kSlice;
    }
    H.npos = pos;
    H.col.assign(pos, 0);
    H.cb_beg.assign(pos, 0);
    H.cb_end.assign(pos, 0);
    // (row, col) -> position
    std::vector<std::map<int, int>> where(H.nv_pad);
    for (int s = 0; s < nsl; ++s)
      for (int l = 0; l < ipcw::kSlice; ++l) {
        int i = s * ipcw::kSlice + l;
        for (int k = 0; k < H.slice_w[s]; ++k) {
          int p = H.slice_pos[s] + k * ipcw::kSlice + l;
          int c = (k < (int)nbr[i].size()) ? nbr[i][k] : i;
          H.col[p] = c;
          if (k < (int)nbr[i].size()) where[i][c] = p;
        }
      }
    std::vector<std::vector<int>> lists(pos);
    for (int e = 0; e < H.nt; ++e)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          int r = H.tets[4 * e + a], c = H.tets[4 * e + b];
          int p = where[r].at(c);
          int blk = (a <= b) ? ipcdev::blk_index(a, b) : ipcdev::blk_index(b, a);
          lists[p].push_back(e * 32 + blk * 2 + (a > b ? 1 : 0));
        }
    for (int p = 0; p < pos; ++p) {
      H.cb_beg[p] = (int)H.contrib.size();
      H.contrib.insert(H.contrib.end(), lists[p].begin(), lists[p].end());
      H.cb_end[p] = (int)H.contrib.size();
    }
  }
  // coarse space of the two-level PCG: the connected sets of free vertices
  // (joined through tets), the kCoarseBodies largest with at least 4
  // vertices (ties: lowest vertex id); while a slot is left and the largest
  // set has at least 64 vertices, that set is split in two halves at the
  // median of its rest positions along the longest axis of their box (ties:
  // vertex order), which then take the first two slots.  Each piece has its
  // rest centroid and the largest rest distance from it.
  {
    std::vector<int> par(H.nv);
    for (int i = 0; i < H.nv; ++i) par[i] = i;
    auto find = [&](int i) {
      while (par[i] != i) i = par[i] = par[par[i]];
      return i;
    };
    for (int e = 0; e < H.nt; ++e)
      for (int a = 1; a < 4; ++a) {
        const int u = H.tets[4 * e], v = H.tets[4 * e + a];
        if (H.kin[u] >= 0 || H.kin[v] >= 0) continue;
        const int ru = find(u), rv = find(v);
        if (ru != rv) par[std::max(ru, rv)] = std::min(ru, rv);
      }
    std::map<int, std::vector<int>> comp;  // root (lowest id of the set) -> free vertices, ascending
    for (int i = 0; i < H.nv; ++i)
      if (H.kin[i] < 0) comp[find(i)].push_back(i);
    std::vector<const std::vector<int> *> order;
    for (auto &c : comp)
      if (c.second.size() >= 4) order.push_back(&c.second);
    std::stable_sort(order.begin(), order.end(),
                     [](const std::vector<int> *a, const std::vector<int> *b) { return a->size() > b->size(); });
    H.vbody.assign(H.nv_pad, -1);
    std::vector<std::vector<int>> pieces;
    for (size_t k = 0; k < std::min<size_t>(order.size(), ipcw::kCoarseBodies); ++k) pieces.push_back(*order[k]);
    if (!pieces.empty() && pieces.size() < (size_t)ipcw::kCoarseBodies && pieces[0].size() >= 64) {
      std::vector<int> vs = pieces[0];
      double lo[3] = {HUGE_VAL, HUGE_VAL, HUGE_VAL}, hi[3] = {-HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
      for (int i : vs)
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], H.X[3 * i + k]);
          hi[k] = std::max(hi[k], H.X[3 * i + k]);
        }
      int ax = 0;
      for (int k = 1; k < 3; ++k)
        if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
      std::stable_sort(vs.begin(), vs.end(), [&](int u, int v) { return H.X[3 * u + ax] < H.X[3 * v + ax]; });
      std::vector<int> first(vs.begin(), vs.begin() + vs.size() / 2), second(vs.begin() + vs.size() / 2, vs.end());
      std::sort(first.begin(), first.end());
      std::sort(second.begin(), second.end());
      pieces[0] = first;
      pieces.insert(pieces.begin() + 1, second);
    }
    H.nbody = (int)pieces.size();
    for (int b = 0; b < H.nbody; ++b) {
      const std::vector<int> &vs = pieces[b];
      double c[3] = {0, 0, 0};
      for (int i : vs)
        for (int k = 0; k < 3; ++k) c[k] += H.X[3 * i + k];
      for (int k = 0; k < 3; ++k) H.cb[b][k] = c[k] / (double)vs.size();
      double r2 = 0.0;
      for (int i : vs) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) d2 += (H.X[3 * i + k] - H.cb[b][k]) * (H.X[3 * i + k] - H.cb[b][k]);
        r2 = std::max(r2, d2);
        H.vbody[i] = b;
      }
      H.cscale[b] = std::max(std::sqrt(r2), 1e-12);
    }
  }
  return S;
}

// ---------------------------------------------------------------------------
// the device world
// ---------------------------------------------------------------------------
struct EnvRec {
  bool used = false;
  size_t v_off, t_off, tri_off, e_off, sv_off, pos_off, contrib_off, vt_off, mo_off;
  size_t v_n, t_n, tri_n, e_n, sv_n, pos_n, contrib_n, vt_n, mo_n;
};

struct World {
  int device = 0;
  hipStream_t stream = nullptr;
  WorldDev W{};
  Arena aV, aT, aTri, aE, aSV, aPos, aContrib, aVT, aMo, aSlice;
  std::vector<EnvDev> envs_h;
  std::vector<EnvRec> recs;
  EnvDev *envs_d = nullptr;
  size_t env_cap = 0;
  EnvState S{};
  std::vector<void **> state_int, state_ll, state_dbl;
  std::vector<std::pair<void **, size_t>> state_wide;  // per-environment arrays of several values
  // batch
  std::vector<int> batch_envs;
  DBuf<Tile> vt_d, tt_d, svt_d, trit_d, et_d, it_d, bt_d;
  DBuf<int> benv_d, fenv_d, live_flag, live_offs;
  DBuf<Tile> live_d;
  std::vector<int> fused_h;  // batch envs whose PCG runs in one workgroup
  ipck::Batch B{};
  ipck::Lists L{};
  DBuf<int> counts, offs, scan_tmp, cand_type, cand_flag, cand_offs, act_type, fenv, inc_cnt, inc_off, inc_cur,
      inc_ent, counter, cr_col, cr_cnt, cr_key, cr_scol, cr_ssrc, cr_flag, cr_pos, cr_rows;
  DBuf<double> cr_val;
  DBuf<float> cr_val32;
  DBuf<int2> cand, act;
  DBuf<int> g_ncell, g_big, g_eoff, g_bigoff, g_ebucket, g_bcnt, g_boff, g_bcur, g_bigl;
  DBuf<ipck::GridEnt> g_ent, g_sorted;
  DBuf<int2> bp_stash;
  DBuf<double> act_d2, cand_d2, e_c, fw, fn, flam, e_f, ce_g, ce_H, part_a, part_z, e_tile, part_b0, part_b1, part_c0, part_c1;
  DBuf<int4> fv, ce_v;
  // decoupled schedule: second friction buffers (merged into, then swapped),
  // per-environment plans of the new friction ranges, host copy of the phases
  DBuf<int4> fv2;
  DBuf<double> fw2, fn2, flam2;
  DBuf<int> fenv2, fplan_b, fplan_e;
  DBuf<int> bar_slow;  // barrier pairs for the full element kernel
  int *phase_h = nullptr;  // pinned, env_cap entries
  size_t phase_cap = 0;
  int *pinned = nullptr;  // host mirror of counters
  hipEvent_t poll_ev[2] = {nullptr, nullptr};  // PCG polls in flight (copies into pinned[8], pinned[9])
  // profiling of the PCG matrix product (HIP events on this stream)
  bool prof_on = false;
  bool prof_all = false;  // bytes of every product launch, none timed
  DBuf<unsigned long long> prof_bytes;
  std::vector<hipEvent_t> ev_pool;
  double prof_ms = 0.0, prof_ms_big = 0.0;  // big: launches over more than kWideTiles tiles
  long long prof_launches = 0, prof_launches_big = 0;
  double prof_ms_iter = 0.0, prof_ms_asm = 0.0;
  long long prof_skipped = 0;  // timed samples whose events were not recorded
  long long prof_asm = 0;      // assembly passes
  // contact work of the assembly passes: candidate pairs classified, barrier
  // pair elements and friction elements evaluated (gradient and projected Hessian)
  long long prof_cands = 0, prof_bar = 0, prof_fric = 0;
  std::vector<hipEvent_t> asm_ev;  // event pairs around the assembly passes of the current step
  int n_fric = 0;
  std::mutex mu;

  World(int dev) : device(dev) {
    HC(hipSetDevice(dev));
    HC(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
    HC(hipHostMalloc((void **)&pinned, 64 * sizeof(int), hipHostMallocDefault));
    for (hipEvent_t &e : poll_ev) HC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    aV.align = ipcw::kSlice;
    aPos.align = ipcw::kSlice;
    auto reg = [](Arena &a, void **slot, size_t elem) { a.bufs.push_back({slot, elem}); };
    reg(aV, (void **)&W.X, 24);
    reg(aV, (void **)&W.x, 24);
    reg(aV, (void **)&W.v, 24);
    reg(aV, (void **)&W.xn, 24);
    reg(aV, (void **)&W.xh, 24);
    reg(aV, (void **)&W.p, 24);
    reg(aV, (void **)&W.g, 24);
    reg(aV, (void **)&W.r, 24);
    reg(aV, (void **)&W.z, 24);
    reg(aV, (void **)&W.pp, 24);
    reg(aV, (void **)&W.w, 24);
    reg(aV, (void **)&W.q, 24);
    reg(aV, (void **)&W.mass, 8);
    reg(aV, (void **)&W.Minv, 72);
    reg(aV, (void **)&W.e_v, 8);
    reg(aV, (void **)&W.lam, 24);
    reg(aV, (void **)&W.r32, 12);
    reg(aV, (void **)&W.z32, 12);
    reg(aV, (void **)&W.pp32, 12);
    reg(aV, (void **)&W.w32, 12);
    reg(aV, (void **)&W.q32, 12);
    reg(aV, (void **)&W.p32, 12);
    reg(aV, (void **)&W.Minv32, 36);
    reg(aV, (void **)&W.kin, 4);
    reg(aV, (void **)&W.venv, 4);
    reg(aV, (void **)&W.vt_beg, 4);
    reg(aV, (void **)&W.vt_end, 4);
    reg(aV, (void **)&W.row_nnz, 4);
    reg(aV, (void **)&W.vbody, 4);
    reg(aV, (void **)&W.hz, 8 * 3 * ipcw::kCoarseM);
    reg(aV, (void **)&W.hz32, 4 * 3 * ipcw::kCoarseM);
    reg(aSlice, (void **)&W.slice_pos, 4);
    reg(aSlice, (void **)&W.slice_w, 4);
    reg(aPos, (void **)&W.col, 4);
    reg(aPos, (void **)&W.cb_beg, 4);
    reg(aPos, (void **)&W.cb_end, 4);
    reg(aPos, (void **)&W.val, 72);
    reg(aPos, (void **)&W.val32, 36);
    reg(aContrib, (void **)&W.contrib, 4);
    reg(aVT, (void **)&W.vt_ent, 4);
    reg(aT, (void **)&W.tet, 16);
    reg(aT, (void **)&W.Dinv, 72);
    reg(aT, (void **)&W.vol, 8);
    reg(aT, (void **)&W.mu, 8);
    reg(aT, (void **)&W.la, 8);
    reg(aT, (void **)&W.tg, 96);
    reg(aT, (void **)&W.tH, 720);
    reg(aT, (void **)&W.e_t, 8);
    reg(aT, (void **)&W.tenv, 4);
    reg(aTri, (void **)&W.tri, 16);
    reg(aTri, (void **)&W.box_tri, 48);
    reg(aE, (void **)&W.edge, 16);
    reg(aE, (void **)&W.elen2, 8);
    reg(aE, (void **)&W.box_edge, 48);
    reg(aSV, (void **)&W.sv, 4);
    reg(aSV, (void **)&W.sv_env, 4);
    reg(aSV, (void **)&W.box_sv, 48);
    reg(aMo, (void **)&W.motion, 8);
    state_int = {(void **)&S.status,   (void **)&S.reason,   (void **)&S.iters,   (void **)&S.halvings,
                 (void **)&S.ls_done,  (void **)&S.ls_cnt,   (void **)&S.pcg_done, (void **)&S.pcg_it,
                 (void **)&S.dbc_bad,  (void **)&S.cand_beg, (void **)&S.cand_end, (void **)&S.act_beg,
                 (void **)&S.act_end,  (void **)&S.fric_beg, (void **)&S.fric_end, (void **)&S.in_step,
                 (void **)&S.big_beg,  (void **)&S.big_end,  (void **)&S.al,       (void **)&S.al_action,
                 (void **)&S.snap_bad, (void **)&S.nact,     (void **)&S.lag,      (void **)&S.iter_cap,
                 (void **)&S.phase};
    state_ll = {(void **)&S.pcg_total, (void **)&S.amax_bits};
    state_dbl = {(void **)&S.alpha, (void **)&S.E0,  (void **)&S.E1,       (void **)&S.pinf,
                 (void **)&S.pcg_bb, (void **)&S.kA, (void **)&S.viol, (void **)&S.viol_prev,
                 (void **)&S.cg_a0,  (void **)&S.cg_a1, (void **)&S.cg_g0, (void **)&S.cg_g1,
                 (void **)&S.kappa,  (void **)&S.kappa0, (void **)&S.dmin_prev, (void **)&S.dmin2,
                 (void **)&S.cgam};
    state_int.push_back((void **)&S.cok);
    state_wide = {{(void **)&S.cinv, 8 * ipcw::kCoarseM * ipcw::kCoarseM}, {(void **)&S.cc, 8 * ipcw::kCoarseM}};
  }

  void ensure_envs(size_t n) {
    if (n <= env_cap) return;
    size_t nc = std::max<size_t>(n, std::max<size_t>(64, env_cap * 2));
    HC(hipStreamSynchronize(stream));
    auto grow = [&](void **slot, size_t elem) {
      void *q = nullptr;
      HC(hipMalloc(&q, nc * elem));
      HC(hipMemset(q, 0, nc * elem));
      if (*slot && env_cap) HC(hipMemcpy(q, *slot, env_cap * elem, hipMemcpyDeviceToDevice));
      if (*slot) HC(hipFree(*slot));
      *slot = q;
    };
    grow((void **)&envs_d, sizeof(EnvDev));
    for (void **s : state_int) grow(s, 4);
    for (void **s : state_ll) grow(s, 8);
    for (void **s : state_dbl) grow(s, 8);
    for (auto &s : state_wide) grow(s.first, s.second);
    env_cap = nc;
  }

  void upload_env(int e) {
    HC(hipMemcpyAsync(envs_d + e, &envs_h[e], sizeof(EnvDev), hipMemcpyHostToDevice, stream));
  }
  // every environment record in one copy
  void upload_envs() {
    if (!envs_h.empty())
      HC(hipMemcpyAsync(envs_d, envs_h.data(), envs_h.size() * sizeof(EnvDev), hipMemcpyHostToDevice, stream));
  }

  template <class T>
  void up(T *dst, const T *src, size_t n) {
    if (n) HC(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, stream));
  }

  // device bytes of a scene's resident state (every array registered with
  // the arenas, at the scene's element counts)
  size_t resident_bytes(const HostScene &H) const {
    auto ab = [](const Arena &a, size_t n) {
      size_t e = 0;
      for (const RawBuf &b : a.bufs) e += b.elem;
      return (n + a.align - 1) / a.align * a.align * e;
    };
    return ab(aV, H.nv_pad) + ab(aT, H.nt) + ab(aTri, H.ntri) + ab(aE, H.ne) + ab(aSV, H.nsv) + ab(aPos, H.npos) +
           ab(aContrib, H.contrib.size()) + ab(aVT, H.vt_ent.size()) + ab(aMo, H.motion.size()) +
           ab(aSlice, (H.nv_pad + ipcw::kSlice - 1) / ipcw::kSlice);
  }
  // The serving admission charge of a scene: its resident bytes, half again
  // for the arenas' growth slack (they grow by 1.5x), and an estimate of its
  // share of the lane's per-step work buffers, which scale with the scene's
  // surface: per broad-phase query the counts, offsets and pair stash; per
  // grid item its entries (a box spans at most 8 cells before it goes to the
  // per-environment list, 2 on average); 16 candidate pairs per query with
  // their type, flags, squared distance and energy; one contact element per
  // surface vertex (4 blocks per row in the merged contact rows); the
  // vertex-tile partials.  Lists longer than that grow the lane's buffers
  // beyond the charge.
  size_t work_bytes(const HostScene &H) const {
    const size_t items = (size_t)H.nsv + H.ne, grid = (size_t)H.ntri + H.ne;
    size_t b = items * (8 + 8 * (size_t)stash_n);
    b += grid * (2 * 2 * sizeof(ipck::GridEnt) + 6 * 4);
    b += items * 16 * (8 + 4 + 4 + 4 + 8 + 8 + 8 + 4 + 8);
    b += (size_t)H.nsv * ((16 + 96 + 720) + 4 * 4 * (4 * 4 + 36 + 72));
    b += (size_t)H.nv_pad * 4 * 7 + (H.nv_pad / ipcw::kTile + 1) * 40;
    return b;
  }
  size_t scene_bytes(const HostScene &H) const { return resident_bytes(H) * 3 / 2 + work_bytes(H); }

  int add_scene(const HostScene &H) {
    int slot = -1;
    for (size_t i = 0; i < recs.size(); ++i)
      if (!recs[i].used) {
        slot = (int)i;
        break;
      }
    if (slot < 0) {
      slot = (int)recs.size();
      recs.push_back({});
      envs_h.push_back({});
    }
    ensure_envs(recs.size());
    EnvRec &R = recs[slot];
    R.used = true;
    live_tets += H.nt;
    R.v_n = H.nv_pad;
    R.t_n = H.nt;
    R.tri_n = H.ntri;
    R.e_n = H.ne;
    R.sv_n = H.nsv;
    R.pos_n = H.npos;
    R.contrib_n = H.contrib.size();
    R.vt_n = H.vt_ent.size();
    R.mo_n = H.motion.size();
    R.v_off = aV.alloc(R.v_n);
    R.t_off = aT.alloc(R.t_n);
    R.tri_off = aTri.alloc(R.tri_n);
    R.e_off = aE.alloc(R.e_n);
    R.sv_off = aSV.alloc(R.sv_n);
    R.pos_off = aPos.alloc(R.pos_n);
    R.contrib_off = aContrib.alloc(R.contrib_n);
    R.vt_off = aVT.alloc(R.vt_n);
    R.mo_off = aMo.alloc(R.mo_n);
    const size_t slice_top = aSlice.top;
    aSlice.top = std::max(aSlice.top, aV.top / ipcw::kSlice);
    try {
      if (admit_faults > 0) {
        --admit_faults;
        throw ApiError(IPC_E_NOMEM, "admission fault planted by IPC_TUNE_ADMIT_FAULTS");
      }
      if ((aT.top + 1) * 32 >= (size_t)1 << 31) throw ApiError(IPC_E_NOMEM, "world tet index space exhausted");
      for (Arena *a : {&aV, &aT, &aTri, &aE, &aSV, &aPos, &aContrib, &aVT, &aMo, &aSlice}) a->reserve(stream);
      upload_scene(H, slot);
    } catch (...) {
      // leave the world as it was: ranges released, slot free
      remove_scene(slot);
      aSlice.top = std::max(slice_top, aV.top / ipcw::kSlice);
      throw;
    }
    batch_envs.clear();  // tile lists must be rebuilt
    return slot;
  }

  // copies a scene into its allocated ranges (slot's record filled in)
  void upload_scene(const HostScene &H, int slot) {
    EnvRec &R = recs[slot];
    size_t vo = R.v_off, to = R.t_off;
    // vertices (padded rows: zero position, kin = PAD)
    std::vector<double> X(3 * R.v_n, 0.0), x(3 * R.v_n, 0.0), v(3 * R.v_n, 0.0), m(R.v_n, 0.0);
    std::vector<int> kin(R.v_n, ipcw::KIN_PAD), venv(R.v_n, slot), vb(R.v_n), ve(R.v_n);
    for (int i = 0; i < H.nv; ++i) {
      for (int k = 0; k < 3; ++k) {
        X[3 * i + k] = H.X[3 * i + k];
        x[3 * i + k] = H.x0[3 * i + k];
        v[3 * i + k] = H.v0[3 * i + k];
      }
      m[i] = H.mass[i];
      kin[i] = H.kin[i] < 0 ? ipcw::KIN_FREE : H.kin[i];
    }
    for (size_t i = 0; i < R.v_n; ++i) {
      vb[i] = H.vt_beg[i] + (int)R.vt_off;
      ve[i] = H.vt_end[i] + (int)R.vt_off;
    }
    up(W.X + 3 * vo, X.data(), X.size());
    up(W.x + 3 * vo, x.data(), x.size());
    up(W.v + 3 * vo, v.data(), v.size());
    up(W.mass + vo, m.data(), m.size());
    up(W.kin + vo, kin.data(), kin.size());
    up(W.venv + vo, venv.data(), venv.size());
    up(W.vt_beg + vo, vb.data(), vb.size());
    up(W.vt_end + vo, ve.data(), ve.size());
    up(W.row_nnz + vo, H.row_nnz.data(), H.row_nnz.size());
    up(W.vbody + vo, H.vbody.data(), H.vbody.size());
    HC(hipMemsetAsync(W.p + 3 * vo, 0, 24 * R.v_n, stream));
    HC(hipMemsetAsync(W.pp + 3 * vo, 0, 24 * R.v_n, stream));
    HC(hipMemsetAsync(W.pp32 + 3 * vo, 0, 12 * R.v_n, stream));
    HC(hipMemsetAsync(W.lam + 3 * vo, 0, 24 * R.v_n, stream));
    std::vector<int> vt(H.vt_ent.size());
    for (size_t i = 0; i < vt.size(); ++i) vt[i] = (H.vt_ent[i] >> 2) * 4 + (int)to * 4 + (H.vt_ent[i] & 3);
    up(W.vt_ent + R.vt_off, vt.data(), vt.size());
    // sliced ELL
    std::vector<int> sp(H.slice_pos.size()), col(H.col.size()), cb(H.cb_beg.size()), ce(H.cb_end.size());
    for (size_t s = 0; s < sp.size(); ++s) sp[s] = H.slice_pos[s] + (int)R.pos_off;
    for (size_t p = 0; p < col.size(); ++p) {
      col[p] = H.col[p] + (int)vo;
      cb[p] = H.cb_beg[p] + (int)R.contrib_off;
      ce[p] = H.cb_end[p] + (int)R.contrib_off;
    }
    up(W.slice_pos + vo / ipcw::kSlice, sp.data(), sp.size());
    up(W.slice_w + vo / ipcw::kSlice, H.slice_w.data(), H.slice_w.size());
    up(W.col + R.pos_off, col.data(), col.size());
    up(W.cb_beg + R.pos_off, cb.data(), cb.size());
    up(W.cb_end + R.pos_off, ce.data(), ce.size());
    std::vector<int> cn(H.contrib.size());
    for (size_t i = 0; i < cn.size(); ++i) cn[i] = H.contrib[i] + (int)to * 32;
    up(W.contrib + R.contrib_off, cn.data(), cn.size());
    // tets
    std::vector<int4> tet(H.nt);
    std::vector<int> tenv(H.nt, slot);
    for (int e = 0; e < H.nt; ++e)
      tet[e] = make_int4(H.tets[4 * e] + (int)vo, H.tets[4 * e + 1] + (int)vo, H.tets[4 * e + 2] + (int)vo,
                         H.tets[4 * e + 3] + (int)vo);
    up(W.tet + to, tet.data(), tet.size());
    up(W.Dinv + 9 * to, H.Dinv.data(), H.Dinv.size());
    up(W.vol + to, H.vol.data(), H.vol.size());
    up(W.mu + to, H.mu.data(), H.mu.size());
    up(W.la + to, H.la.data(), H.la.size());
    up(W.tenv + to, tenv.data(), tenv.size());
    // surface
    std::vector<int4> tri(H.ntri), edge(H.ne);
    for (int i = 0; i < H.ntri; ++i)
      tri[i] = make_int4(H.tris[i][0] + (int)vo, H.tris[i][1] + (int)vo, H.tris[i][2] + (int)vo, slot);
    for (int i = 0; i < H.ne; ++i) edge[i] = make_int4(H.edges[i][0] + (int)vo, H.edges[i][1] + (int)vo, slot, 0);
    std::vector<int> sv(H.nsv), svenv(H.nsv, slot);
    for (int i = 0; i < H.nsv; ++i) sv[i] = H.sverts[i] + (int)vo;
    up(W.tri + R.tri_off, tri.data(), tri.size());
    up(W.edge + R.e_off, edge.data(), edge.size());
    up(W.elen2 + R.e_off, H.elen2.data(), H.elen2.size());
    up(W.sv + R.sv_off, sv.data(), sv.size());
    up(W.sv_env + R.sv_off, svenv.data(), svenv.size());
    up(W.motion + R.mo_off, H.motion.data(), H.motion.size());
    // env record
    EnvDev &E = envs_h[slot];
    std::memset(&E, 0, sizeof(E));
    E.v_off = (int)vo;
    E.nv = H.nv;
    E.nv_pad = H.nv_pad;
    E.t_off = (int)to;
    E.nt = H.nt;
    E.tri_off = (int)R.tri_off;
    E.ntri = H.ntri;
    E.e_off = (int)R.e_off;
    E.ne = H.ne;
    E.sv_off = (int)R.sv_off;
    E.nsv = H.nsv;
    E.pos_off = (int)R.pos_off;
    E.npos = H.npos;
    E.mo_off = (int)R.mo_off;
    E.n_groups = H.n_groups;
    E.n_motion = H.n_motion;
    E.step = 0;
    E.maxit = H.maxit;
    E.precision = H.precision;
    E.dt = H.dt;
    E.dhat = H.dhat;
    E.kappa = H.kappa;
    E.mu = H.mu_f;
    E.eps_v = H.eps_v;
    E.tol = H.tol;
    E.pcg_tol = H.pcg_tol;
    E.cell = H.cell;
    E.mbar = H.mbar;
    E.fric_iters = H.fric_iters;
    E.nnzb = 0;
    for (int r : H.row_nnz) E.nnzb += r;
    E.inv_filter = H.inv_filter;
    E.adapt_kappa = H.adapt_kappa;
    E.nbody = H.nbody;
    for (int b = 0; b < ipcw::kCoarseBodies; ++b) {
      for (int k = 0; k < 3; ++k) E.cb[b][k] = H.cb[b][k];
      E.cscale[b] = H.cscale[b] > 0.0 ? H.cscale[b] : 1.0;
    }
    upload_env(slot);
    int zero = 0;
    HC(hipMemcpyAsync(S.status + slot, &zero, 4, hipMemcpyHostToDevice, stream));
    // barrier stiffness as given; no previous iterate yet
    const double kap = H.kappa, inf = HUGE_VAL;
    HC(hipMemcpyAsync(S.kappa + slot, &kap, 8, hipMemcpyHostToDevice, stream));
    HC(hipMemcpyAsync(S.kappa0 + slot, &kap, 8, hipMemcpyHostToDevice, stream));
    HC(hipMemcpyAsync(S.dmin_prev + slot, &inf, 8, hipMemcpyHostToDevice, stream));
    HC(hipStreamSynchronize(stream));
  }

  void remove_scene(int slot) {
    EnvRec &R = recs[slot];
    if (!R.used) return;
    aV.release(R.v_off, R.v_n);
    aT.release(R.t_off, R.t_n);
    aTri.release(R.tri_off, R.tri_n);
    aE.release(R.e_off, R.e_n);
    aSV.release(R.sv_off, R.sv_n);
    aPos.release(R.pos_off, R.pos_n);
    aContrib.release(R.contrib_off, R.contrib_n);
    aVT.release(R.vt_off, R.vt_n);
    aMo.release(R.mo_off, R.mo_n);
    live_tets -= (long long)R.t_n;
    R.used = false;
    batch_envs.clear();
  }

  // ---- batch set-up -------------------------------------------------------
  void set_batch(const std::vector<int> &envs) {
    if (envs == batch_envs) return;
    swept_n = -1;  // candidate lists follow the batch layout
    std::vector<Tile> vt, tt, svt, trit, et, it, bt;
    int item_off = 0, bitem_off = 0;
    fused_h.clear();
    for (int e : envs) {
      EnvDev &E = envs_h[e];
      E.vtile_first = (int)vt.size();
      for (int s = 0, r = 0; s < E.nv_pad; s += ipcw::kTile, ++r)
        vt.push_back({e, E.v_off + s, std::min(ipcw::kTile, E.nv_pad - s), r});
      E.vtile_count = (int)vt.size() - E.vtile_first;
      for (int s = 0, r = 0; s < E.nt; s += ipcw::kTile, ++r)
        tt.push_back({e, E.t_off + s, std::min(ipcw::kTile, E.nt - s), r});
      for (int s = 0; s < E.nsv; s += ipcw::kTile) svt.push_back({e, E.sv_off + s, std::min(ipcw::kTile, E.nsv - s), 0});
      for (int s = 0; s < E.ntri; s += ipcw::kTile)
        trit.push_back({e, E.tri_off + s, std::min(ipcw::kTile, E.ntri - s), 0});
      for (int s = 0; s < E.ne; s += ipcw::kTile) et.push_back({e, E.e_off + s, std::min(ipcw::kTile, E.ne - s), 0});
      for (int s = 0; s < E.nsv; s += ipcw::kTile) it.push_back({e, E.sv_off + s, std::min(ipcw::kTile, E.nsv - s), 0});
      for (int s = 0; s < E.ne; s += ipcw::kTile) it.push_back({e, E.e_off + s, std::min(ipcw::kTile, E.ne - s), 1});
      for (int s = 0; s < E.ntri; s += ipcw::kTile) bt.push_back({e, E.tri_off + s, std::min(ipcw::kTile, E.ntri - s), 0});
      for (int s = 0; s < E.ne; s += ipcw::kTile) bt.push_back({e, E.e_off + s, std::min(ipcw::kTile, E.ne - s), 1});
      E.item_off = item_off;
      item_off += E.nsv + E.ne;
      E.bitem_off = bitem_off;
      bitem_off += E.ntri + E.ne;
      E.fused = (E.nv_pad <= ipcw::kFusedRows && use_fused()) ? 1 : 0;
      if (E.fused) fused_h.push_back(e);
    }
    upload_envs();
    auto put = [&](DBuf<Tile> &d, const std::vector<Tile> &h) {
      d.ensure(h.size() + 1);
      up(d.p, h.data(), h.size());
    };
    put(vt_d, vt);
    put(tt_d, tt);
    put(svt_d, svt);
    put(trit_d, trit);
    put(et_d, et);
    put(it_d, it);
    put(bt_d, bt);
    benv_d.ensure(envs.size() + 1);
    up(benv_d.p, envs.data(), envs.size());
    fenv_d.ensure(fused_h.size() + 1);
    up(fenv_d.p, fused_h.data(), fused_h.size());
    live_d.ensure(vt.size() + 1);
    live_flag.ensure(vt.size() + 1);
    live_offs.ensure(vt.size() + 2);
    B.vtiles = vt_d.p;
    B.ttiles = tt_d.p;
    B.svtiles = svt_d.p;
    B.tritiles = trit_d.p;
    B.etiles = et_d.p;
    B.itiles = it_d.p;
    B.btiles = bt_d.p;
    B.n_bt = (int)bt.size();
    B.n_bitems = bitem_off;
    B.n_vt = (int)vt.size();
    B.n_tt = (int)tt.size();
    B.n_svt = (int)svt.size();
    B.n_trit = (int)trit.size();
    B.n_et = (int)et.size();
    B.n_it = (int)it.size();
    B.envs = benv_d.p;
    B.n_envs = (int)envs.size();
    B.n_items = item_off;
    counts.ensure(item_off + 1);
    offs.ensure(item_off + 2);
    bp_stash.ensure((size_t)stash_n * item_off + 1);
    g_ncell.ensure(bitem_off + 1);
    g_big.ensure(bitem_off + 1);
    g_eoff.ensure(bitem_off + 2);
    g_bigoff.ensure(bitem_off + 2);
    g_bigl.ensure(bitem_off + 1);
    size_t nvw = aV.cap + 2;
    inc_cnt.ensure(nvw);
    inc_off.ensure(nvw);
    inc_cur.ensure(nvw);
    cr_cnt.ensure(nvw);
    cr_flag.ensure(nvw);
    cr_pos.ensure(nvw + 1);
    cr_rows.ensure(nvw);
    size_t nvt = vt.size() + 1;
    part_a.ensure(nvt);
    part_z.ensure(nvt * ipcw::kCoarseM);
    e_tile.ensure(nvt * ipcw::kCoarseM * ipcw::kCoarseM);
    part_b0.ensure(nvt);
    part_b1.ensure(nvt);
    part_c0.ensure(nvt);
    part_c1.ensure(nvt);
    counter.ensure(16);
    scan_tmp.ensure(std::max<size_t>(std::max<size_t>(item_off, bitem_off), nvw) / 1024 + 64);
    HC(hipStreamSynchronize(stream));
    batch_envs = envs;
    refresh_lists();
  }

  void refresh_lists() {
    L.counts = counts.p;
    L.offs = offs.p;
    L.scan_tmp = scan_tmp.p;
    L.cand = cand.p;
    L.cand_type = cand_type.p;
    L.cand_flag = cand_flag.p;
    L.cand_offs = cand_offs.p;
    L.cand_d2 = cand_d2.p;
    L.e_c = e_c.p;
    L.act = act.p;
    L.act_type = act_type.p;
    L.act_d2 = act_d2.p;
    L.fv = fv.p;
    L.fw = fw.p;
    L.fn = fn.p;
    L.flam = flam.p;
    L.e_f = e_f.p;
    L.fenv = fenv.p;
    L.ce_v = ce_v.p;
    L.ce_g = ce_g.p;
    L.ce_H = ce_H.p;
    L.inc_cnt = inc_cnt.p;
    L.inc_off = inc_off.p;
    L.inc_cur = inc_cur.p;
    L.inc_ent = inc_ent.p;
    L.cr_col = cr_col.p;
    L.cr_cnt = cr_cnt.p;
    L.cr_key = cr_key.p;
    L.cr_scol = cr_scol.p;
    L.cr_ssrc = cr_ssrc.p;
    L.cr_flag = cr_flag.p;
    L.cr_pos = cr_pos.p;
    L.cr_rows = cr_rows.p;
    L.cr_val = cr_val.p;
    L.cr_val32 = cr_val32.p;
    L.part_a = part_a.p;
    L.part_z = part_z.p;
    L.e_tile = e_tile.p;
    L.part_b0 = part_b0.p;
    L.part_b1 = part_b1.p;
    L.part_c0 = part_c0.p;
    L.part_c1 = part_c1.p;
    L.counter = counter.p;
    L.bar_slow = bar_slow.p;
    L.prof = prof_on ? prof_bytes.p : nullptr;
    L.g_ncell = g_ncell.p;
    L.g_big = g_big.p;
    L.g_eoff = g_eoff.p;
    L.g_bigoff = g_bigoff.p;
    L.g_ebucket = g_ebucket.p;
    L.g_bcnt = g_bcnt.p;
    L.g_boff = g_boff.p;
    L.g_bcur = g_bcur.p;
    L.g_bigl = g_bigl.p;
    L.g_ent = g_ent.p;
    L.g_sorted = g_sorted.p;
    L.bp_stash = bp_stash.p;
    L.stash_n = stash_n;
    L.bp_coop = bp_coop;
  }

  void set_prof(int mode) {
    prof_on = mode != 0;
    prof_all = mode == 2;
    const bool on = prof_on;
    if (on && !prof_bytes.p) {
      prof_bytes.ensure(8);
      HC(hipMemsetAsync(prof_bytes.p, 0, 8 * prof_bytes.cap, stream));
      HC(hipStreamSynchronize(stream));
    }
    refresh_lists();
  }

  void prof_reset() {
    prof_ms = prof_ms_big = prof_ms_iter = prof_ms_asm = 0.0;
    prof_skipped = 0;
    prof_launches = prof_launches_big = prof_asm = 0;
    prof_cands = prof_bar = prof_fric = 0;
    if (prof_bytes.p) {
      HC(hipMemsetAsync(prof_bytes.p, 0, 32, stream));
      HC(hipStreamSynchronize(stream));
    }
  }

  std::vector<hipEvent_t> asm_pool;
  hipEvent_t asm_event(size_t i) {
    while (asm_pool.size() <= i) {
      hipEvent_t e;
      HC(hipEventCreate(&e));
      asm_pool.push_back(e);
    }
    return asm_pool[i];
  }
  // adds the assembly passes timed since the last call (stream idle)
  void collect_asm() {
    for (size_t k = 0; k + 1 < asm_ev.size(); k += 2) {
      float ms = 0.f;
      HC(hipEventElapsedTime(&ms, asm_ev[k], asm_ev[k + 1]));
      prof_ms_asm += ms;
      prof_asm += 1;
    }
    asm_ev.clear();
  }

  hipEvent_t pool_event(size_t i) {
    while (ev_pool.size() <= i) {
      hipEvent_t e;
      HC(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
    return ev_pool[i];
  }

  int read_int(const int *dptr) {
    HC(hipMemcpyAsync(pinned, dptr, sizeof(int), hipMemcpyDeviceToHost, stream));
    HC(hipStreamSynchronize(stream));
    return pinned[0];
  }
  // two device ints read with one synchronisation
  void read_int2(const int *a, const int *b, int &va, int &vb) {
    HC(hipMemcpyAsync(pinned, a, sizeof(int), hipMemcpyDeviceToHost, stream));
    HC(hipMemcpyAsync(pinned + 1, b, sizeof(int), hipMemcpyDeviceToHost, stream));
    HC(hipStreamSynchronize(stream));
    va = pinned[0];
    vb = pinned[1];
  }

  // ---- broad phase: candidate list at x (p == nullptr) or over x -> x+p ----
  int broad_phase(const double *x, const double *p) {
    ipck::boxes(stream, W, envs_d, S, B, x, p);
    // bin triangles and edges into the per-environment hash grids
    ipck::grid_count(stream, W, envs_d, S, B, L);
    ipck::scan_int(stream, L.g_ncell, L.g_eoff, B.n_bitems, L.scan_tmp);
    ipck::scan_int(stream, L.g_big, L.g_bigoff, B.n_bitems, L.scan_tmp);
    int n_ent = read_int(L.g_eoff + B.n_bitems);
    unsigned nb = 1024;
    while (nb < 2u * (unsigned)n_ent) nb <<= 1;
    bool moved = g_ent.ensure(n_ent + 1);
    moved |= g_sorted.ensure(n_ent + 1);
    moved |= g_ebucket.ensure(n_ent + 1);
    moved |= g_bcnt.ensure(nb + 1);
    moved |= g_boff.ensure(nb + 2);
    moved |= g_bcur.ensure(nb + 1);
    moved |= scan_tmp.ensure(nb / 1024 + 64);
    if (moved) refresh_lists();
    ipck::grid_fill(stream, W, envs_d, S, B, L, n_ent, nb);
    // query: count, scan, write
    ipck::bp_grid_count(stream, W, envs_d, S, B, L, nb);
    ipck::scan_int(stream, L.counts, L.offs, B.n_items, L.scan_tmp);
    int n = 0, n_over = 0;
    read_int2(L.offs + B.n_items, L.counter + 4, n, n_over);
    const bool overflow = n_over > 0;
    if (tracing())
      std::fprintf(stderr, "[ipc]   broad phase: %d queries, %d pairs, %d queries over the stash of %d\n", B.n_items, n,
                   n_over, stash_n);
    // each list is sized on its own: capacities are rounded independently
    moved = cand.ensure(n + 1);
    moved |= cand_type.ensure(n + 1);
    moved |= cand_flag.ensure(n + 1);
    moved |= cand_offs.ensure(n + 2);
    moved |= cand_d2.ensure(n + 1);
    moved |= e_c.ensure(n + 1);
    if (moved) refresh_lists();
    ipck::bp_grid_write(stream, W, envs_d, S, B, L, nb, overflow);
    ipck::cand_segments(stream, envs_d, S, B, L);
    return n;
  }

  // classify + compact the active pairs of the current candidate list
  // adapt = 1 at a Newton iterate: the adaptive barrier stiffness update
  int active_pairs(int n_cand, const double *x, int adapt = 0) {
    if (scan_tmp.ensure(n_cand / 1024 + 64)) refresh_lists();
    ipck::classify_cands(stream, W, envs_d, L, n_cand, x);
    ipck::scan_int(stream, L.cand_flag, L.cand_offs, n_cand, L.scan_tmp);
    int n = read_int(L.cand_offs + n_cand);
    bool moved = act.ensure(n + 1);
    moved |= act_type.ensure(n + 1);
    moved |= act_d2.ensure(n + 1);
    if (moved) refresh_lists();
    ipck::compact_active(stream, L, n_cand);
    ipck::act_segments(stream, S, B, L);
    ipck::act_stats(stream, envs_d, S, B, L, adapt);
    return n;
  }

  void ensure_ce(int n) {
    bool moved = ce_v.ensure(n + 1);
    moved |= ce_g.ensure(12L * (n + 1));
    moved |= ce_H.ensure(90L * (n + 1));
    if (moved) refresh_lists();
  }

  // friction pairs = active pairs at x^n (positions in W.x)
  // lagged friction set from the active pairs at W.x (= xn at step start),
  // classified from a candidate list of nc pairs whose boxes contain W.x
  void friction_setup(int nc) {
    int na = active_pairs(nc, W.x);
    bool moved = fv.ensure(na + 1);
    moved |= fw.ensure(4L * (na + 1));
    moved |= fn.ensure(3L * (na + 1));
    moved |= flam.ensure(na + 1);
    moved |= e_f.ensure(na + 1);
    moved |= fenv.ensure(na + 1);
    if (moved) refresh_lists();
    ipck::friction_setup(stream, W, envs_d, S, L, na);
    // the friction segments are the active segments of this list
    copy_state_int(S.fric_beg, S.act_beg);
    copy_state_int(S.fric_end, S.act_end);
    n_fric = na;
  }

  // Decoupled schedule: environments in phase PH_BEGIN / PH_RELAG take new
  // lagged friction data from the active pairs at W.x of the current
  // candidate list (nc pairs, whose boxes contain W.x); environments still
  // iterating keep theirs; the others drop theirs.  Pairs stay grouped per
  // environment in batch order and in candidate order within one, the order
  // a full friction set-up gives.
  void friction_merge(int nc) {
    bool moved = scan_tmp.ensure(nc / 1024 + 64);
    moved |= act.ensure(nc + 1);
    moved |= act_type.ensure(nc + 1);
    moved |= act_d2.ensure(nc + 1);
    if (moved) refresh_lists();
    ipck::classify_cands(stream, W, envs_d, L, nc, W.x);
    ipck::cand_restrict(stream, W, S, L, nc);
    ipck::scan_int(stream, L.cand_flag, L.cand_offs, nc, L.scan_tmp);
    ipck::compact_active(stream, L, nc);
    ipck::act_segments(stream, S, B, L);
    fplan_b.ensure(env_cap + 1);
    fplan_e.ensure(env_cap + 1);
    ipck::fric_plan(stream, S, B, fplan_b.p, fplan_e.p, L.counter + 6);
    int na = 0, total = 0;
    read_int2(L.cand_offs + nc, L.counter + 6, na, total);
    fv2.ensure(total + 1);
    fw2.ensure(4L * (total + 1));
    fn2.ensure(3L * (total + 1));
    flam2.ensure(total + 1);
    fenv2.ensure(total + 1);
    ipck::fric_merge(stream, W, envs_d, S, B, L, n_fric, na, fplan_b.p, fplan_e.p, fv2.p, fw2.p, fn2.p, flam2.p,
                     fenv2.p);
    auto swp = [](auto &a, auto &b) {
      std::swap(a.p, b.p);
      std::swap(a.cap, b.cap);
    };
    swp(fv, fv2);
    swp(fw, fw2);
    swp(fn, fn2);
    swp(flam, flam2);
    swp(fenv, fenv2);
    e_f.ensure(total + 1);
    n_fric = total;
    refresh_lists();
  }

  // host phases of every environment slot -> device (pinned staging)
  void upload_phases(const std::vector<int> &ph) {
    if (phase_cap < ph.size()) {
      HC(hipStreamSynchronize(stream));
      if (phase_h) HC(hipHostFree(phase_h));
      phase_cap = std::max<size_t>(ph.size(), 256);
      HC(hipHostMalloc((void **)&phase_h, phase_cap * sizeof(int), hipHostMallocDefault));
    }
    HC(hipStreamSynchronize(stream));  // the previous upload has been read
    std::memcpy(phase_h, ph.data(), ph.size() * sizeof(int));
    HC(hipMemcpyAsync(S.phase, phase_h, ph.size() * sizeof(int), hipMemcpyHostToDevice, stream));
  }

  void copy_state_int(int *dst, const int *src) {
    HC(hipMemcpyAsync(dst, src, sizeof(int) * env_cap, hipMemcpyDeviceToDevice, stream));
  }

  // Candidate list left by the last swept pass (x -> x + p, d̂-widened) when
  // every environment of the batch has since moved to x + a p with a in
  // [0, 1] (or kept x): the boxes of a static pass at the new x lie inside
  // those swept boxes, so the list holds every pair a static pass would find,
  // and the exact d² < d̂² test picks the same active set.  -1: none.
  int swept_n = -1;
  long long live_tets = 0;  // tets of the scenes living here (lane placement)
  int admit_faults = 0;     // test hook: the next add_scene calls fail as out of memory

  // gradient, contact elements, incidence, assembled Hessian at W.x
  int assemble_system(int mixed) {
    int nc = swept_n >= 0 ? swept_n : broad_phase(W.x, nullptr);
    swept_n = -1;
    int na = active_pairs(nc, W.x, 1);
    ensure_ce(na + n_fric);
    if (bar_slow.ensure(na + 1)) L.bar_slow = bar_slow.p;
    ipck::barrier_elems(stream, W, envs_d, S, L, na, W.x);
    ipck::friction_elems(stream, W, envs_d, S, L, n_fric, na, W.x);
    int nce = na + n_fric;
    if (prof_on) {
      prof_cands += nc;
      prof_bar += na;
      prof_fric += n_fric;
    }
    int nvw = (int)aV.cap;
    ipck::incidence(stream, W, S, L, nce, nvw);
    int ntot = read_int(L.inc_off + nvw);
    bool moved = inc_ent.ensure(ntot + 1);
    moved |= cr_col.ensure(4L * ntot + 1);
    moved |= cr_key.ensure(4L * ntot + 1);
    moved |= cr_scol.ensure(4L * ntot + 1);
    moved |= cr_ssrc.ensure(4L * ntot + 1);
    moved |= scan_tmp.ensure(nvw / 1024 + 64);
    moved |= cr_val.ensure(36L * ntot + 1);
    moved |= cr_val32.ensure(36L * ntot + 1);
    if (moved) refresh_lists();
    ipck::incidence_fill(stream, W, S, L, nce, nvw);
    ipck::contact_rows(stream, L, nvw, ntot, mixed);
    // measurement: the assembly pass (elasticity, inertia, gradient, stored
    // blocks) from the start of its first kernel to the end of its last
    // (events carried by the two dispatches), its algorithmic bytes counted
    // after it
    hipEvent_t a0 = nullptr, a1 = nullptr;
    if (prof_on && !prof_all) {
      a0 = asm_event(asm_ev.size());
      a1 = asm_event(asm_ev.size() + 1);
      asm_ev.push_back(a0);
      asm_ev.push_back(a1);
    }
    ipck::elastic(stream, W, envs_d, S, B, a0);
    ipck::assemble(stream, W, envs_d, S, B, L, mixed, a1);
    if (coarse) ipck::coarse_setup(stream, W, envs_d, S, B, L, mixed);
    if (prof_on) ipck::asm_bytes(stream, envs_d, S, B, mixed, prof_bytes.p + 3);
    return na;
  }

  // execution knobs (ipc_set_tuning); initial values from the environment
public:
  static int env_knob(const char *name, int dflt) {
    const char *e = std::getenv(name);
    return (e && e[0]) ? std::max(0, std::atoi(e)) : dflt;
  }
  // 1: environments of up to kFusedRows rows run their whole PCG in one
  // workgroup each (default 0: tiled, faster on the batched grasp workload
  // because large solves then spread over several CUs)
  int fused_pcg = env_knob("IPC_FUSED_PCG", 0) ? 1 : 0;
  // live vertex tiles at or below which the tiled PCG hands the remaining
  // environments to one workgroup each (0 = never)
  int tail_tiles = env_knob("IPC_TAIL_TILES", 0);
  // 1: the next block of PCG iterations is queued before the host polls the
  // previous one (0: after it)
  const int pipeline = env_knob("IPC_PIPELINE", 1) ? 1 : 0;
  // PCG iterations per block between polls of the pending count (-1: 8 in
  // mixed precision, 4 in FP64)
  int poll_block = env_knob("IPC_POLL_BLOCK", -1) > 0 ? env_knob("IPC_POLL_BLOCK", -1) : -1;
  // the batch is laid out again once at most this percentage of it still
  // iterates its Newton loop
  const int narrow_pct = std::min(100, env_knob("IPC_NARROW_PCT", 50));
  // broad phase: pairs per query that the counting pass keeps (queries with
  // more are traversed a second time to write them)
  const int stash_n = std::max(1, env_knob("IPC_BP_STASH", 64));
  // 1: the counting pass walks each query's cells with a group of 8 lanes
  // (adjacent loads), 0: one lane per query
  const int bp_coop = env_knob("IPC_BP_COOP", 1) ? 1 : 0;
  // PCG product launches over at most this many tiles issue each lane's
  // slots four at a time, larger ones one at a time.  Default (-1): every
  // launch in FP64 and none in the mixed path, where the one-slot variant (44
  // VGPRs against 86) measured faster also in the latency-bound tails.
  int wide_tiles = [] {
    const char *e = std::getenv("IPC_WIDE_TILES");
    return (e && e[0]) ? std::max(0, std::atoi(e)) : -1;
  }();
  // 1: re-lay the batch out with the still-iterating environments once at
  // most half of it iterates (narrow_batch)
  int narrow = env_knob("IPC_NARROW", 1) ? 1 : 0;
  // 1: the decoupled schedule (run_steps_lane_async): environments begin
  // their next step as soon as they finish one; 0: lock-step time steps
  int async_mode = env_knob("IPC_ASYNC", 1) ? 1 : 0;
  // 1: the two-level PCG (block Jacobi plus the bodies' rigid motions as a
  // coarse space); the per-environment PCG kernels are block Jacobi only, so
  // they are not used while it is on
  int coarse = env_knob("IPC_COARSE", 1) ? 1 : 0;
  bool use_fused() const { return fused_pcg == 1 && !coarse; }
  void set_fused(int on) {
    if ((on != 0) == (fused_pcg == 1)) return;
    fused_pcg = on ? 1 : 0;
    batch_envs.clear();  // E.fused is decided when a batch is laid out
  }
  void set_coarse(int on) {
    if ((on != 0) == (coarse == 1)) return;
    coarse = on ? 1 : 0;
    batch_envs.clear();
  }
  void copy_knobs(const World &o) {
    set_fused(o.fused_pcg);
    set_coarse(o.coarse);
    wide_tiles = o.wide_tiles;
    poll_block = o.poll_block;
    tail_tiles = o.tail_tiles;
    narrow = o.narrow;
    async_mode = o.async_mode;
    set_prof(o.prof_all ? 2 : o.prof_on ? 1 : 0);
  }

  long long solve(int mixed) {
    int *pending = L.counter;
    ipck::pcg_fused(stream, W, envs_d, S, fenv_d.p, (int)fused_h.size(), L, mixed);
    if (fused_h.size() == batch_envs.size()) {
      ipck::pcg_finish(stream, W, S, B, mixed);
      HC(hipStreamSynchronize(stream));
      if (!tracing()) return 0;
      std::vector<int> its(env_cap);
      HC(hipMemcpyAsync(its.data(), S.pcg_it, 4 * env_cap, hipMemcpyDeviceToHost, stream));
      HC(hipStreamSynchronize(stream));
      int mx = 0;
      for (int e : fused_h) mx = std::max(mx, its[e]);
      return mx;
    }
    L.wide_tiles = wide_tiles >= 0 ? wide_tiles : mixed ? 0 : 1 << 30;
    L.coarse = coarse;
    ipck::pcg_init(stream, W, envs_d, S, B, L, pending, mixed);
    // an environment's solve stops at the latest in the iteration whose index
    // reaches its cap of 30 n_v + 10 (that iteration only takes the test)
    int cap = 0;
    for (int e : batch_envs) cap = std::max(cap, 30 * envs_h[e].nv + 11);
    int it = 0;
    size_t nev = 0;
    // iterate over the tiles of environments still solving; the list is
    // compacted whenever an environment has converged since the last poll
    const Tile *tl = B.vtiles;
    int ntl = B.n_vt, last_pending = -1;
    std::vector<char> ev_big;  // per timed launch: over more than kWideTiles tiles
    const bool tr = tracing();
    double t_launch = 0.0, t_wait = 0.0;
    auto now = []() { return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count(); };
    // Blocks of poll_block iterations, pipelined: block k+1 is queued before the host
    // waits for the count of environments still iterating after block k, so
    // the device does not idle while the host polls.  A block queued after
    // every solve has stopped costs only launches whose tiles exit at once.
    const int pb = poll_block > 0 ? poll_block : mixed ? 8 : 4;
    auto launch_block = [&](int slot) {
      for (int j = 0; j < pb; ++j) {
        // every 16th iteration is timed (the product and the update carry
        // start and end events in their dispatches) and counts its
        // algorithmic bytes in a launch of its own between the two kernels;
        // with prof_all every iteration counts its bytes and none is timed
        const hipEvent_t *ev = nullptr;
        bool count = false;
        if (prof_all) {
          count = true;
          prof_launches += 1;
        } else if (prof_on && (it & 15) == 5) {
          for (int q = 0; q < 4; ++q) pool_event(nev + q);
          ev = &ev_pool[nev];
          nev += 4;
          count = true;
          ev_big.push_back(ntl > ipck::kWideTiles ? 1 : 0);
        }
        ipck::pcg_iter(stream, W, envs_d, S, L, it++, pending, mixed, ev, count, tl, ntl);
      }
      HC(hipMemcpyAsync(pinned + 8 + slot, pending, sizeof(int), hipMemcpyDeviceToHost, stream));
      HC(hipEventRecord(poll_ev[slot], stream));
    };
    int slot = 0;
    launch_block(slot);
    while (true) {
      double t0 = tr ? now() : 0.0;
      const bool queued = pipeline && it < cap;
      if (queued) launch_block(1 - slot);
      double t1 = tr ? now() : 0.0;
      HC(hipEventSynchronize(poll_ev[slot]));
      const int pend = pinned[8 + slot];
      if (tr) {
        t_launch += t1 - t0;
        t_wait += now() - t1;
      }
      if (pend <= 0 || it >= cap) break;
      if (pend != last_pending) {
        ipck::live_tiles(stream, S, B, L, live_d.p, live_flag.p, live_offs.p);
        ntl = read_int(live_offs.p + B.n_vt);
        tl = live_d.p;
        last_pending = pend;
        if (ntl <= tail_tiles && !coarse) {
          // few tiles left: their launches would be latency-bound, so one
          // workgroup per environment finishes the solves in one launch
          ipck::pcg_resume(stream, W, envs_d, S, L, tl, ntl, it, mixed);
          break;
        }
      }
      if (!queued) launch_block(1 - slot);
      slot = 1 - slot;
    }
    ipck::pcg_finish(stream, W, S, B, mixed);
    if (tr)
      std::fprintf(stderr, "[ipc]   pcg %d iterations: host launching %.0f us, waiting %.0f us\n", it, t_launch, t_wait);
    if (prof_on) {
      HC(hipStreamSynchronize(stream));
      for (size_t k = 0; k + 3 < nev; k += 4) {
        float ms = 0.f, mu = 0.f;
        // a sample whose events were not both recorded is left out (counted)
        if (hipEventElapsedTime(&ms, ev_pool[k], ev_pool[k + 1]) != hipSuccess ||
            hipEventElapsedTime(&mu, ev_pool[k + 2], ev_pool[k + 3]) != hipSuccess) {
          (void)hipGetLastError();
          ++prof_skipped;
          continue;
        }
        prof_ms += ms;
        prof_ms_iter += ms + mu;
        prof_launches += 1;
        if (ev_big[k / 4]) {
          prof_ms_big += ms;
          prof_launches_big += 1;
        }
      }
      collect_asm();
    }
    return it;
  }

  // ---- one time step of every environment in the current batch -------------
  // IPC_TRACE=1 prints one line per Newton iteration to stderr.
  static bool tracing() {
    static int t = -1;
    if (t < 0) {
      const char *e = std::getenv("IPC_TRACE");
      t = (e && e[0] && e[0] != '0') ? 1 : 0;
    }
    return t == 1;
  }

  // Newton iterations of the current batch until every environment has
  // converged or failed (at most maxit iterations per environment and round)
  template <class Clock>
  void newton_loop(int maxit, int mixed, bool inv, Clock &ms) {
    for (int it = 0; it < maxit; ++it) {
      int na = assemble_system(mixed);
      long long pit = solve(mixed);
      ipck::conv_check(stream, W, envs_d, S, B, L, L.counter + 1);
      int still = read_int(L.counter + 1);
      if (tracing())
        std::fprintf(stderr, "[ipc] newton %d: active pairs %d friction %d pcg %lld envs-left %d  %.1f ms\n", it, na,
                     n_fric, pit, still, ms());
      if (still == 0) break;
      if (narrow && 100 * still <= narrow_pct * (int)batch_envs.size()) narrow_batch();
      ipck::al_prepare(stream, W, S, B);
      int ns = broad_phase(W.x, W.p);
      ipck::ccd_init(stream, S, B);
      ipck::accd(stream, W, envs_d, S, L, ns, W.x, W.p);
      if (inv) ipck::inv_bound(stream, W, envs_d, S, B, 0);
      ipck::snap_J(stream, W, S, B);
      ipck::ls_init(stream, S, B);
      ipck::energy(stream, W, envs_d, S, B, L, ns, n_fric, 1, S.E0);
      int trials = 0;
      for (int trial = 0; trial < 64; ++trial) {
        ipck::energy(stream, W, envs_d, S, B, L, ns, n_fric, 0, S.E1);
        ipck::ls_decide(stream, S, B, L.counter + 2);
        ++trials;
        if (read_int(L.counter + 2) == 0) break;
      }
      if (tracing()) std::fprintf(stderr, "[ipc]   swept %d line-search trials %d  %.1f ms\n", ns, trials, ms());
      ipck::al_finish(stream, W, envs_d, S, B);
      ipck::update_x(stream, W, S, B);
      swept_n = ns;  // x moved by a p with a <= 1, snapped inside the swept boxes, or stayed
      ipck::iter_end(stream, envs_d, S, B, L.counter + 3);
      if (read_int(L.counter + 3) == 0) break;
    }
  }

  void step_batch() {
    auto t0 = std::chrono::steady_clock::now();
    auto ms = [&]() {
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    swept_n = -1;
    ipck::set_phase(stream, S, B, ipcw::PH_BEGIN);
    ipck::env_begin(stream, envs_d, S, B);
    ipck::begin_step(stream, W, envs_d, S, B);
    // one swept pass over the Dirichlet move (free vertices stay at xn): its
    // boxes contain xn, so it also yields the friction set's pairs at xn
    int nc = broad_phase(W.xn, W.p);
    friction_setup(nc);
    ipck::ccd_init(stream, S, B);
    ipck::accd(stream, W, envs_d, S, L, nc, W.xn, W.p);
    ipck::dbc_check_J(stream, W, envs_d, S, B);
    ipck::env_dbc(stream, S, B);
    ipck::apply_dbc(stream, W, envs_d, S, B);
    ipck::set_phase(stream, S, B, ipcw::PH_ITER);
    swept_n = nc;  // x is xn, or the targets on kinematic rows: inside these boxes
    int maxit = 0, rounds = 1;
    bool inv = false;
    int mixed = 0;
    for (int e : batch_envs) {
      maxit = std::max(maxit, envs_h[e].maxit);
      rounds = std::max(rounds, envs_h[e].fric_iters);
      inv |= envs_h[e].inv_filter != 0;
      mixed |= envs_h[e].precision == IPC_MIXED;
    }
    const std::vector<int> step_envs = batch_envs;
    for (int lag = 0; lag < rounds; ++lag) {
      if (lag > 0) {
        // another lagged friction update: environments that converged and
        // take one solve again, with friction data taken at their iterate
        set_batch(step_envs);
        ipck::relag(stream, envs_d, S, B, 0, L.counter + 5);
        if (read_int(L.counter + 5) == 0) break;
        int nc = broad_phase(W.x, nullptr);
        friction_setup(nc);
        swept_n = nc;  // the static list at x serves the first iteration
      }
      newton_loop(maxit, mixed, inv, ms);
    }
    swept_n = -1;
    set_batch(step_envs);
    ipck::step_end(stream, W, envs_d, S, B, 0);
    HC(hipStreamSynchronize(stream));
    if (prof_on) collect_asm();
  }

  // Once at most half of the batch is still iterating, lay the batch out
  // again with those environments only, so that every per-iteration launch
  // covers their tiles alone.  Each environment's sums run over its own tiles
  // in their own order, so this changes no result.
  void narrow_batch() {
    std::vector<int> st(env_cap);
    HC(hipMemcpyAsync(st.data(), S.status, 4 * env_cap, hipMemcpyDeviceToHost, stream));
    HC(hipStreamSynchronize(stream));
    std::vector<int> live;
    for (int e : batch_envs)
      if (st[e] == ipcw::ST_ACTIVE) live.push_back(e);
    set_batch(live);
  }
};

// Each device holds `g_lanes` worlds ("lanes"), each with its own
// stream, buffers and host thread while stepping.  A batch whose scenes live
// in several lanes is stepped lane by lane concurrently, so the tail of one
// lane's Newton and PCG loops (few environments, latency-bound launches)
// overlaps with the other lanes' work on the same GPU.
std::mutex g_worlds_mu;
std::map<int, std::vector<std::unique_ptr<World>>> g_worlds;
int g_lanes = -1;

int lanes_setting() {
  // By default one lane per hardware queue of the process beside the one the
  // runtime's null stream holds (GPU_MAX_HW_QUEUES, 4 unless set: 3 lanes),
  // and at most 4: on the batched grasp workload 4 lanes on 5 queues measured
  // 7% above 3 lanes, while 5 to 8 lanes, on 8 or 16 queues, ran slower.
  if (g_lanes < 0) {
    const int queues = World::env_knob("GPU_MAX_HW_QUEUES", 4);
    g_lanes = std::max(1, std::min(16, World::env_knob("IPC_LANES", std::max(1, std::min(4, queues - 1)))));
  }
  return g_lanes;
}

// every lane of the current device, creating them up to the lane count
std::vector<World *> worlds_for_current_device() {
  int dev = 0;
  HC(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_worlds_mu);
  auto &v = g_worlds[dev];
  int n = lanes_setting();
  while ((int)v.size() < n) {
    v.push_back(std::make_unique<World>(dev));
    if (v.size() > 1) v.back()->copy_knobs(*v.front());
  }
  std::vector<World *> out;
  for (auto &w : v) out.push_back(w.get());
  return out;
}

World &world_for_current_device() { return *worlds_for_current_device().front(); }

// lane for a new scene: the one with the fewest live tets (first on ties)
World &world_for_new_scene() {
  auto ws = worlds_for_current_device();
  int n = std::min<int>(lanes_setting(), (int)ws.size());
  World *best = ws[0];
  for (int i = 1; i < n; ++i) {
    std::lock_guard<std::mutex> lk(ws[i]->mu);
    if (ws[i]->live_tets < best->live_tets) best = ws[i];
  }
  return *best;
}

}  // namespace

struct ipc_scene_s {
  World *world;
  int slot;
  std::unique_ptr<HostScene> host;
  int step = 0;
  bool failed = false;
  int fail_reason = 0;
};

namespace {

int api_error(const std::exception &e) {
  if (auto *a = dynamic_cast<const ApiError *>(&e)) {
    set_err(a->what());
    return a->code;
  }
  set_err(e.what());
  return IPC_E_DEVICE;
}

template <class F>
int guarded(F f) {
  try {
    return f();
  } catch (const std::exception &e) {
    return api_error(e);
  }
}

template <class T>
void down(World &w, T *dst, const T *src, size_t n) {
  if (n) HC(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, w.stream));
}

// per-env scalar state readback
struct EnvSnapshot {
  int status, reason, iters, halvings;
  long long pcg_total;
  double E0;
};

// all env slots at once (one copy per field)
struct EnvSnapshots {
  std::vector<int> status, reason, iters, halvings, nact, lag;
  std::vector<long long> pcg_total;
  std::vector<double> E0, dmin2, kappa;
  void fetch(World &w) {
    size_t n = w.env_cap;
    status.resize(n);
    reason.resize(n);
    iters.resize(n);
    halvings.resize(n);
    nact.resize(n);
    pcg_total.resize(n);
    E0.resize(n);
    dmin2.resize(n);
    kappa.resize(n);
    lag.resize(n);
    HC(hipMemcpyAsync(lag.data(), w.S.lag, 4 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(nact.data(), w.S.nact, 4 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(dmin2.data(), w.S.dmin2, 8 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(kappa.data(), w.S.kappa, 8 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(status.data(), w.S.status, 4 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(reason.data(), w.S.reason, 4 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(iters.data(), w.S.iters, 4 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(halvings.data(), w.S.halvings, 4 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(pcg_total.data(), w.S.pcg_total, 8 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipMemcpyAsync(E0.data(), w.S.E0, 8 * n, hipMemcpyDeviceToHost, w.stream));
    HC(hipStreamSynchronize(w.stream));
  }
};

EnvSnapshot snapshot(World &w, int e) {
  EnvSnapshot s{};
  down(w, &s.status, w.S.status + e, 1);
  down(w, &s.reason, w.S.reason + e, 1);
  down(w, &s.iters, w.S.iters + e, 1);
  down(w, &s.halvings, w.S.halvings + e, 1);
  down(w, &s.pcg_total, w.S.pcg_total + e, 1);
  down(w, &s.E0, w.S.E0 + e, 1);
  HC(hipStreamSynchronize(w.stream));
  return s;
}

void set_status(World &w, int e, int st) {
  HC(hipMemcpyAsync(w.S.status + e, &st, 4, hipMemcpyHostToDevice, w.stream));
  HC(hipStreamSynchronize(w.stream));
}

// positions of one scene (real rows only)
void put_x(World &w, ipc_scene s, double *dev_arr, const double *host) {
  HC(hipMemcpyAsync(dev_arr + 3L * w.envs_h[s->slot].v_off, host, 24L * s->host->nv, hipMemcpyHostToDevice,
                    w.stream));
}
void get_x(World &w, ipc_scene s, const double *dev_arr, double *host) {
  HC(hipMemcpyAsync(host, dev_arr + 3L * w.envs_h[s->slot].v_off, 24L * s->host->nv, hipMemcpyDeviceToHost,
                    w.stream));
  HC(hipStreamSynchronize(w.stream));
}

// Decoupled schedule of one lane: every round, the environments in the middle
// of a time step take one Newton iteration (assembly, solve, convergence
// test, then CCD and line search), while an environment whose step ended in
// the round's convergence test ends it at once and begins its next step in
// the same round (targets, predicted positions, lagged friction and the
// Dirichlet move), or re-lags its friction.  No environment waits for the
// others to finish a step, so a round's launches cover every environment
// that still has work, and the lane's rounds number about the largest total
// of Newton iterations of one environment instead of the sum over steps of
// each step's largest.  Each environment goes through exactly the sequence of
// the lock-step schedule (same lists, same order of every sum), so its
// results are bitwise those of World::step_batch.
//
// LaneRounds holds the schedule's state so that environments can join between
// rounds (the server admits requests there) and leave once their steps are
// done or they fail.  A batch layout change between rounds only makes the
// next assembly search its candidates afresh: an environment's active pairs,
// their order and every sum over them are the same either way.
struct LaneRounds {
  struct Item {
    ipc_scene s = nullptr;
    int remaining = 0;
    bool stepping = false;  // in the middle of a time step
    bool fresh = true;      // added, not begun yet
    ipc_step_info info{};
  };
  World &w;
  std::vector<Item> items;
  std::vector<int> ph;
  EnvSnapshots snap;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double t_asm = 0, t_pcg = 0, t_state = 0, t_begin = 0, t_ls = 0;
  long rounds = 0;
  long long steps_converged = 0;  // over all items, since creation
  explicit LaneRounds(World &lane) : w(lane) {}
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  void add(ipc_scene s, int n_steps, const ipc_step_info &init) {
    Item it;
    it.s = s;
    it.remaining = s->failed ? 0 : n_steps;
    it.info = init;
    items.push_back(it);
  }
  bool has_work() const {
    for (const Item &it : items)
      if (it.stepping || (it.fresh && it.remaining > 0)) return true;
    return false;
  }
  // items with no steps left (done or failed), removed from the schedule
  std::vector<Item> take_done() {
    std::vector<Item> done, keep;
    for (Item &it : items) (it.stepping || (it.fresh && it.remaining > 0) ? keep : done).push_back(it);
    items.swap(keep);
    return done;
  }

  // One round.  Returns false when no item had work.
  bool round() {
    using namespace ipcw;
    // batch: the items with work; laid out again when items joined or left
    // it, or once at most narrow_pct% of it still has work
    std::vector<int> live;
    bool joined = false;
    for (const Item &it : items)
      if (it.stepping || (it.fresh && it.remaining > 0)) {
        live.push_back(it.s->slot);
        joined |= it.fresh;
      }
    if (live.empty()) return false;
    {
      std::vector<int> have = w.batch_envs;
      std::sort(have.begin(), have.end());
      bool covered = true;
      for (int e : live) covered &= std::binary_search(have.begin(), have.end(), e);
      const bool shrink = w.narrow && 100 * (int)live.size() <= w.narrow_pct * (int)w.batch_envs.size();
      if (!covered || joined || shrink) w.set_batch(live);
    }
    if (ph.size() < w.env_cap) ph.assign(w.env_cap, PH_ITER);
    int mixed = 0;
    bool inv = false, any_stepping = false;
    for (const Item &it : items) {
      const EnvDev &E = w.envs_h[it.s->slot];
      inv |= E.inv_filter != 0;
      mixed |= E.precision == IPC_MIXED;
      any_stepping |= it.stepping;
    }
    // 1. one Newton iteration of the environments in the middle of a step
    double t = ms();
    if (any_stepping) {
      int na = w.assemble_system(mixed);
      double t1 = ms();
      t_asm += t1 - t;
      long long pit = w.solve(mixed);
      ipck::conv_check(w.stream, w.W, w.envs_d, w.S, w.B, w.L, w.L.counter + 1);
      t_pcg += ms() - t1;
      if (World::tracing())
        std::fprintf(stderr, "[ipc] round %ld: active pairs %d friction %d pcg %lld  %.1f ms\n", rounds, na,
                     w.n_fric, pit, ms());
    }
    // 2. states; steps that ended, steps that begin, friction re-lags
    t = ms();
    snap.fetch(w);
    t_state += ms() - t;
    ++rounds;
    std::fill(ph.begin(), ph.end(), (int)PH_ITER);
    bool begin = false, relag = false, iterate = false, finish = false;
    for (Item &it : items) {
      ipc_scene s = it.s;
      const int e = s->slot;
      if (it.fresh) {
        if (it.remaining > 0) {
          ph[e] = PH_BEGIN;
          it.stepping = true;
          begin = true;
          w.envs_h[e].step = s->step;
          w.upload_env(e);
        }
        it.fresh = false;
        continue;
      }
      if (!it.stepping) continue;
      const int st = snap.status[e];
      if (st == ST_ACTIVE) {
        iterate = true;
        continue;
      }
      if (st == ST_CONVERGED && snap.lag[e] + 1 < w.envs_h[e].fric_iters) {
        ph[e] = PH_RELAG;
        relag = true;
        continue;
      }
      // the step is over
      ipc_step_info &inf = it.info;
      inf.newton_iters += snap.iters[e];
      inf.max_newton_iters = std::max(inf.max_newton_iters, snap.iters[e]);
      inf.ls_halvings += snap.halvings[e];
      inf.pcg_iters += snap.pcg_total[e];
      inf.energy_last = snap.E0[e];
      inf.kappa_last = snap.kappa[e];
      finish = true;
      if (st == ST_CONVERGED) {
        s->step += 1;
        it.remaining -= 1;
        inf.steps_done += 1;
        ++steps_converged;
        inf.n_active_last = snap.nact[e];
        inf.min_dist_last = std::sqrt(snap.dmin2[e]);
        if (it.remaining > 0) {
          ph[e] = PH_FINISH_BEGIN;
          begin = true;
          w.envs_h[e].step = s->step;
          w.upload_env(e);
        } else {
          ph[e] = PH_FINISH;
          it.stepping = false;
        }
      } else {
        s->failed = true;
        s->fail_reason = (st == ST_FAILED) ? snap.reason[e] : IPC_FAIL_MAXIT;
        inf.status = IPC_E_FAILED;
        inf.fail_reason = s->fail_reason;
        ph[e] = PH_FINISH;
        it.stepping = false;
        it.remaining = 0;
      }
    }
    if (!begin && !relag && !iterate && !finish) return false;
    // 3. the round's device work
    w.upload_phases(ph);
    if (finish) {
      ipck::step_end(w.stream, w.W, w.envs_d, w.S, w.B, 1);
      ipck::phase_advance(w.stream, w.S, w.B);
    }
    if (begin) {
      ipck::env_begin(w.stream, w.envs_d, w.S, w.B);
      ipck::begin_step(w.stream, w.W, w.envs_d, w.S, w.B);
    }
    if (relag) ipck::relag(w.stream, w.envs_d, w.S, w.B, 1, w.L.counter + 5);
    if (!begin && !relag && !iterate) {  // only step ends this round
      w.swept_n = -1;
      HC(hipStreamSynchronize(w.stream));
      return true;
    }
    t = ms();
    if (iterate) ipck::al_prepare(w.stream, w.W, w.S, w.B);
    // one swept pass: the Newton directions of the iterating environments and
    // the Dirichlet moves of the beginning ones (their free vertices stay)
    int ns = w.broad_phase(w.W.x, w.W.p);
    if (begin || relag) w.friction_merge(ns);
    ipck::ccd_init(w.stream, w.S, w.B);
    ipck::accd(w.stream, w.W, w.envs_d, w.S, w.L, ns, w.W.x, w.W.p);
    if (begin) {
      ipck::dbc_check_J(w.stream, w.W, w.envs_d, w.S, w.B);
      ipck::env_dbc(w.stream, w.S, w.B);
      ipck::apply_dbc(w.stream, w.W, w.envs_d, w.S, w.B);
    }
    t_begin += ms() - t;
    t = ms();
    if (iterate) {
      if (inv) ipck::inv_bound(w.stream, w.W, w.envs_d, w.S, w.B, 0);
      ipck::snap_J(w.stream, w.W, w.S, w.B);
      ipck::ls_init(w.stream, w.S, w.B);
      ipck::energy(w.stream, w.W, w.envs_d, w.S, w.B, w.L, ns, w.n_fric, 1, w.S.E0);
      for (int trial = 0; trial < 64; ++trial) {
        ipck::energy(w.stream, w.W, w.envs_d, w.S, w.B, w.L, ns, w.n_fric, 0, w.S.E1);
        ipck::ls_decide(w.stream, w.S, w.B, w.L.counter + 2);
        if (w.read_int(w.L.counter + 2) == 0) break;
      }
      ipck::al_finish(w.stream, w.W, w.envs_d, w.S, w.B);
      ipck::update_x(w.stream, w.W, w.S, w.B);
    }
    ipck::iter_end(w.stream, w.envs_d, w.S, w.B, w.L.counter + 3);
    w.swept_n = ns;
    t_ls += ms() - t;
    return true;
  }

  void trace_summary() const {
    if (World::tracing())
      std::fprintf(stderr,
                   "[ipc] lane %p: %zu envs, %ld rounds, %.1f ms: assembly %.1f, pcg %.1f, states %.1f, "
                   "begin+broad phase+ccd %.1f, line search %.1f\n",
                   (void *)&w, items.size(), rounds, ms(), t_asm, t_pcg, t_state, t_begin, t_ls);
  }
};

void run_steps_lane_async(World &w, std::vector<ipc_scene> &scenes, int n_steps, ipc_step_info *infos) {
  LaneRounds R(w);
  std::vector<int> batch;
  for (size_t i = 0; i < scenes.size(); ++i) {
    R.add(scenes[i], n_steps, infos ? infos[i] : ipc_step_info{});
    batch.push_back(scenes[i]->slot);
  }
  std::vector<LaneRounds::Item> all = R.items;  // item order = scene order
  w.swept_n = -1;
  while (R.round()) {
  }
  R.trace_summary();
  if (infos)
    for (size_t i = 0; i < scenes.size(); ++i)
      for (const LaneRounds::Item &it : R.items)
        if (it.s == scenes[i]) infos[i] = it.info;
  w.swept_n = -1;
  w.set_batch(batch);
  HC(hipStreamSynchronize(w.stream));
  if (w.prof_on) w.collect_asm();
}

// steps scenes that all live in one lane
void run_steps_lane(std::vector<ipc_scene> scenes, int n_steps, ipc_step_info *infos) {
  if (scenes.empty()) return;
  World &w = *scenes[0]->world;
  std::lock_guard<std::mutex> lk(w.mu);
  std::vector<int> slots;
  for (auto s : scenes) slots.push_back(s->slot);
  {
    std::vector<int> sorted = slots;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      throw ApiError(IPC_E_ARG, "a scene appears twice in the batch");
  }
  HC(hipSetDevice(w.device));
  w.set_batch(slots);
  for (size_t i = 0; i < scenes.size(); ++i)
    if (infos) {
      std::memset(&infos[i], 0, sizeof(ipc_step_info));
      infos[i].status = scenes[i]->failed ? IPC_E_FAILED : IPC_OK;
      infos[i].fail_reason = scenes[i]->fail_reason;
    }
  if (w.async_mode) {
    run_steps_lane_async(w, scenes, n_steps, infos);
    return;
  }
  EnvSnapshots snap;
  for (int st = 0; st < n_steps; ++st) {
    bool any = false;
    for (auto s : scenes) any |= !s->failed;
    if (!any) break;
    // the motion row follows each env's own step index
    for (auto s : scenes) w.envs_h[s->slot].step = s->step;
    w.upload_envs();
    w.step_batch();
    snap.fetch(w);
    for (size_t i = 0; i < scenes.size(); ++i) {
      ipc_scene s = scenes[i];
      if (s->failed) continue;
      int e = s->slot;
      if (infos) {
        infos[i].newton_iters += snap.iters[e];
        infos[i].max_newton_iters = std::max(infos[i].max_newton_iters, snap.iters[e]);
        infos[i].ls_halvings += snap.halvings[e];
        infos[i].pcg_iters += snap.pcg_total[e];
        infos[i].energy_last = snap.E0[e];
        infos[i].kappa_last = snap.kappa[e];
      }
      if (snap.status[e] == ipcw::ST_CONVERGED) {
        s->step += 1;
        if (infos) {
          infos[i].steps_done += 1;
          // contact statistics of the accepted iterate (its last classification)
          infos[i].n_active_last = snap.nact[e];
          infos[i].min_dist_last = std::sqrt(snap.dmin2[e]);
        }
        snap.status[e] = ipcw::ST_IDLE;
      } else {
        s->failed = true;
        s->fail_reason = (snap.status[e] == ipcw::ST_FAILED) ? snap.reason[e] : IPC_FAIL_MAXIT;
        snap.status[e] = ipcw::ST_FAILED;
        if (infos) {
          infos[i].status = IPC_E_FAILED;
          infos[i].fail_reason = s->fail_reason;
        }
      }
    }
    HC(hipMemcpyAsync(w.S.status, snap.status.data(), 4 * w.env_cap, hipMemcpyHostToDevice, w.stream));
    HC(hipStreamSynchronize(w.stream));
  }
}

// steps a batch: the scenes of each lane are stepped together, lanes
// concurrently (one host thread per extra lane)
void run_steps(const std::vector<ipc_scene> &scenes, int n_steps, ipc_step_info *infos) {
  if (scenes.empty()) return;
  int dev = scenes[0]->world->device;
  std::vector<World *> lanes;
  std::vector<std::vector<size_t>> idx;
  for (size_t i = 0; i < scenes.size(); ++i) {
    World *w = scenes[i]->world;
    if (w->device != dev) throw ApiError(IPC_E_ARG, "scenes of one batch must live on the same device");
    size_t k = std::find(lanes.begin(), lanes.end(), w) - lanes.begin();
    if (k == lanes.size()) {
      lanes.push_back(w);
      idx.emplace_back();
    }
    idx[k].push_back(i);
  }
  if (lanes.size() == 1) {
    run_steps_lane(scenes, n_steps, infos);
    return;
  }
  std::vector<std::vector<ipc_step_info>> part(lanes.size());
  std::vector<std::exception_ptr> err(lanes.size());
  auto work = [&](size_t k) {
    try {
      HC(hipSetDevice(dev));
      std::vector<ipc_scene> sub;
      for (size_t i : idx[k]) sub.push_back(scenes[i]);
      part[k].assign(sub.size(), ipc_step_info{});
      run_steps_lane(sub, n_steps, infos ? part[k].data() : nullptr);
    } catch (...) {
      err[k] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  for (size_t k = 1; k < lanes.size(); ++k) th.emplace_back(work, k);
  work(0);
  for (auto &t : th) t.join();
  for (auto &e : err)
    if (e) std::rethrow_exception(e);
  if (infos)
    for (size_t k = 0; k < lanes.size(); ++k)
      for (size_t j = 0; j < idx[k].size(); ++j) infos[idx[k][j]] = part[k][j];
}

// ---------------------------------------------------------------------------
// serving: a worker thread per lane admits queued requests by slot count and
// memory, advances all running ones together one tick at a time (a round of
// the decoupled schedule, or a time step under the lock-step one), retires
// finished ones between ticks
// ---------------------------------------------------------------------------
struct Request {
  int64_t id = 0;
  std::unique_ptr<HostScene> host;  // until admitted
  ipc_scene scene = nullptr;        // while running
  int32_t n_steps = 0, status = IPC_REQ_QUEUED, steps_done = 0, fail_reason = 0;
  double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
  int64_t newton = 0, pcg = 0, bytes = 0;
  int nv = 0;
  std::vector<double> pos, vel;  // once finished
};

}  // namespace

struct ipc_server_s {
  std::vector<World *> lanes;  // one worker thread per lane
  int64_t budget = 0;
  int32_t max_slots = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::vector<std::vector<Request *>> running;  // per lane
  // per lane: requests taken off the queue and being placed on the device
  // (their bytes and slot are already counted); a device error retires them
  // with the running ones
  std::vector<std::vector<Request *>> admitting;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  int64_t next_id = 1, used = 0;
  int n_running = 0;  // over all lanes, admitted requests included
  bool stop = false, dead = false;
  std::string error;
  long long finished = 0, failed = 0, conv_steps = 0, ticks = 0;
  // slot-cap autotuner (max_slots = 0 at creation): starting from 8 slots per
  // lane, while requests wait, double the cap after every window of 8 ticks
  // per lane (64 rounds per lane under the decoupled schedule, where a round
  // is one Newton iteration), unless the window's seconds per converged step exceed 1.5x the
  // best window's: then settle on the best window's cap.  A tick costs about
  // its slowest environment's step, so more slots raise throughput until the
  // device saturates.
  bool auto_slots = false, settled = false;
  int32_t best_cap = 0;
  double best_cost = 0.0, win_t0 = 0.0;
  long long win_ticks = 0, win_steps = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  std::vector<std::thread> workers;
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

void retire(ipc_server_s *sv, Request *r, bool failed, int reason) {
  // caller holds sv->mu
  r->status = failed ? IPC_REQ_FAILED : IPC_REQ_DONE;
  r->fail_reason = failed ? reason : IPC_FAIL_NONE;
  r->t_done = sv->now();
  sv->used -= r->bytes;
  if (failed)
    ++sv->failed;
  else
    ++sv->finished;
}

// caller holds sv->mu; `mine` = requests the asking lane runs or is admitting
// (each lane takes at most its share of the slot cap)
bool can_admit(const ipc_server_s *sv, size_t mine) {
  const size_t share = (sv->max_slots + sv->lanes.size() - 1) / sv->lanes.size();
  return !sv->queue.empty() && sv->n_running < sv->max_slots && mine < share &&
         sv->used + sv->queue.front()->bytes <= sv->budget;
}

void autotune_tick(ipc_server_s *sv, long long tick_steps) {
  // caller holds sv->mu
  if (!sv->auto_slots || sv->settled) return;
  sv->win_steps += tick_steps;
  const long long window = sv->lanes[0]->async_mode ? 64 : 8;
  if (++sv->win_ticks < window * (long long)sv->lanes.size()) return;
  double t = sv->now();
  double cost = (t - sv->win_t0) / std::max<long long>(sv->win_steps, 1);
  if (!sv->queue.empty()) {  // demand above the cap: the cap is what limits
    if (sv->best_cost > 0.0 && cost > 1.5 * sv->best_cost) {
      sv->max_slots = sv->best_cap;
      sv->settled = true;
    } else {
      if (sv->best_cost == 0.0 || cost < sv->best_cost) {
        sv->best_cost = cost;
        sv->best_cap = sv->max_slots;
      }
      sv->max_slots = std::min(1024, 2 * sv->max_slots);
      sv->cv_work.notify_all();
    }
  }
  sv->win_ticks = 0;
  sv->win_steps = 0;
  sv->win_t0 = t;
}

// the worker of lane k: admit into this lane, advance its running requests
// one tick, retire the finished ones
void server_loop(ipc_server_s *sv, size_t k) {
  World *w = sv->lanes[k];
  std::vector<Request *> &mine = sv->running[k];
  std::vector<Request *> &admitting = sv->admitting[k];
  std::vector<ipc_step_info> infos;
  LaneRounds R(*w);  // the lane's decoupled schedule (w->async_mode)
  try {
    HC(hipSetDevice(w->device));
    while (true) {
      std::vector<Request *> admit;
      {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_work.wait(lk, [&]() { return sv->stop || sv->dead || !mine.empty() || can_admit(sv, mine.size()); });
        if (sv->stop || sv->dead) return;
        while (can_admit(sv, mine.size() + admitting.size())) {
          Request *r = sv->queue.front();
          sv->queue.pop_front();
          sv->used += r->bytes;
          ++sv->n_running;
          admitting.push_back(r);
        }
        admit = admitting;
      }
      bool freed = false;
      for (Request *r : admit) {
        auto *sc = new ipc_scene_s();
        sc->world = w;
        bool placed = false;
        {
          std::lock_guard<std::mutex> lk(w->mu);
          try {
            sc->slot = w->add_scene(*r->host);
            placed = true;
          } catch (const ApiError &e) {
            // out of device memory for this request alone: it fails, the
            // others go on (add_scene left the lane as it was)
            if (e.code != IPC_E_NOMEM) {
              delete sc;
              throw;
            }
          } catch (...) {
            delete sc;
            throw;
          }
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        auto at = std::find(admitting.begin(), admitting.end(), r);
        if (at != admitting.end()) admitting.erase(at);
        if (sv->dead) {
          // another lane's device error retired every request meanwhile
          if (placed) {
            std::lock_guard<std::mutex> wl(w->mu);
            w->remove_scene(sc->slot);
          }
          delete sc;
          return;
        }
        if (!placed) {
          delete sc;
          r->t_admit = sv->now();
          retire(sv, r, true, IPC_FAIL_ADMIT);
          --sv->n_running;
          freed = true;
          continue;
        }
        sc->host = std::move(r->host);
        r->scene = sc;
        r->status = IPC_REQ_RUNNING;
        r->t_admit = sv->now();
        mine.push_back(r);
      }
      if (freed) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
      }
      std::vector<Request *> run;
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        run = mine;
      }
      if (run.empty()) continue;
      std::vector<Request *> done;
      long long tick_steps = 0;
      if (w->async_mode) {
        // one round of the decoupled schedule: the admitted requests begin
        // their first step in it, the others take a Newton iteration or move
        // on to their next step
        for (Request *r : run)
          if (std::none_of(R.items.begin(), R.items.end(),
                           [&](const LaneRounds::Item &it) { return it.s == r->scene; })) {
            ipc_step_info init{};
            init.status = r->scene->failed ? IPC_E_FAILED : IPC_OK;
            R.add(r->scene, r->n_steps - r->steps_done, init);
          }
        const long long before = R.steps_converged;
        {
          std::lock_guard<std::mutex> wl(w->mu);
          R.round();
        }
        tick_steps = R.steps_converged - before;
        std::vector<LaneRounds::Item> fin = R.take_done();
        for (const LaneRounds::Item &it : fin) {
          Request *r = *std::find_if(run.begin(), run.end(), [&](Request *q) { return q->scene == it.s; });
          r->pos.resize(3 * (size_t)r->nv);
          r->vel.resize(3 * (size_t)r->nv);
          std::lock_guard<std::mutex> wl(w->mu);
          get_x(*w, it.s, w->W.x, r->pos.data());
          get_x(*w, it.s, w->W.v, r->vel.data());
          w->remove_scene(it.s->slot);
          done.push_back(r);
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->dead) return;
        // progress of the lane's requests (counts since admission)
        auto progress = [&](const LaneRounds::Item &it) {
          auto at = std::find_if(run.begin(), run.end(), [&](Request *q) { return q->scene == it.s; });
          if (at == run.end()) return;
          Request *r = *at;
          r->steps_done = it.info.steps_done;
          r->newton = it.info.newton_iters;
          r->pcg = it.info.pcg_iters;
        };
        for (const LaneRounds::Item &it : R.items) progress(it);
        for (const LaneRounds::Item &it : fin) progress(it);
      } else {
        std::vector<ipc_scene> scenes;
        for (Request *r : run) scenes.push_back(r->scene);
        infos.assign(run.size(), ipc_step_info{});
        run_steps_lane(scenes, 1, infos.data());
        {
          // another lane's device error retires every request: leave them alone
          std::lock_guard<std::mutex> lk(sv->mu);
          if (sv->dead) return;
        }
        for (size_t i = 0; i < run.size(); ++i) {
          Request *r = run[i];
          ipc_scene sc = scenes[i];
          bool fin = sc->failed || r->steps_done + infos[i].steps_done >= r->n_steps;
          if (fin) {
            r->pos.resize(3 * (size_t)r->nv);
            r->vel.resize(3 * (size_t)r->nv);
            std::lock_guard<std::mutex> lk(w->mu);
            get_x(*w, sc, w->W.x, r->pos.data());
            get_x(*w, sc, w->W.v, r->vel.data());
            w->remove_scene(sc->slot);
            done.push_back(r);
          }
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->dead) return;
        for (size_t i = 0; i < run.size(); ++i) {
          Request *r = run[i];
          r->steps_done += infos[i].steps_done;
          r->newton += infos[i].newton_iters;
          r->pcg += infos[i].pcg_iters;
          tick_steps += infos[i].steps_done;
        }
      }
      std::lock_guard<std::mutex> lk(sv->mu);
      if (sv->dead) return;
      sv->conv_steps += tick_steps;
      autotune_tick(sv, tick_steps);
      for (Request *r : done) {
        retire(sv, r, r->scene->failed, r->scene->fail_reason);
        delete r->scene;
        r->scene = nullptr;
        mine.erase(std::find(mine.begin(), mine.end(), r));
        --sv->n_running;
      }
      ++sv->ticks;
      sv->cv_done.notify_all();
      if (!done.empty()) sv->cv_work.notify_all();  // freed slots and memory
    }
  } catch (const std::exception &e) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->dead = true;
    sv->error = e.what();
    for (auto &lane : sv->running) {
      for (Request *r : lane) {
        retire(sv, r, true, IPC_FAIL_DEVICE);
        r->scene = nullptr;  // left with the device's world
      }
      lane.clear();
    }
    for (auto &lane : sv->admitting) {
      for (Request *r : lane) retire(sv, r, true, IPC_FAIL_DEVICE);
      lane.clear();
    }
    for (Request *r : sv->queue) {
      sv->used += r->bytes;  // retire() subtracts it again
      retire(sv, r, true, IPC_FAIL_DEVICE);
    }
    sv->queue.clear();
    sv->n_running = 0;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

void fill_info(const Request &r, ipc_request_info *info) {
  info->status = r.status;
  info->steps_done = r.steps_done;
  info->n_steps = r.n_steps;
  info->fail_reason = r.fail_reason;
  info->t_submit = r.t_submit;
  info->t_admit = r.t_admit;
  info->t_done = r.t_done;
  info->newton_iters = r.newton;
  info->pcg_iters = r.pcg;
  info->bytes = r.bytes;
}

Request &find_req(ipc_server srv, int64_t id) {
  auto it = srv->reqs.find(id);
  if (it == srv->reqs.end()) throw ApiError(IPC_E_ARG, "unknown request id");
  return *it->second;
}

bool finished(const Request &r) { return r.status == IPC_REQ_DONE || r.status == IPC_REQ_FAILED; }

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

const char *ipc_last_error(void) { return g_err; }

int ipc_create_scene(const ipc_scene_desc *desc, ipc_scene *out) {
  return guarded([&]() {
    if (!out) throw ApiError(IPC_E_ARG, "null output handle");
    auto host = preprocess(desc);
    World &w = world_for_new_scene();
    std::lock_guard<std::mutex> lk(w.mu);
    int slot = w.add_scene(*host);
    auto *s = new ipc_scene_s();
    s->world = &w;
    s->slot = slot;
    s->host = std::move(host);
    *out = s;
    return IPC_OK;
  });
}

void ipc_destroy_scene(ipc_scene s) {
  if (!s) return;
  try {
    std::lock_guard<std::mutex> lk(s->world->mu);
    s->world->remove_scene(s->slot);
  } catch (...) {
  }
  delete s;
}

int ipc_step(ipc_scene s, int32_t n_steps, ipc_step_info *info) { return ipc_step_batch(&s, 1, n_steps, info); }

int ipc_step_batch(ipc_scene *scenes, int32_t n, int32_t n_steps, ipc_step_info *infos) {
  return guarded([&]() {
    if (!scenes || n < 0 || n_steps < 0) throw ApiError(IPC_E_ARG, "bad arguments");
    std::vector<ipc_scene> v(scenes, scenes + n);
    for (auto s : v)
      if (!s) throw ApiError(IPC_E_ARG, "null scene");
    bool failed_before = false;
    for (auto s : v) failed_before |= s->failed;
    run_steps(v, n_steps, infos);
    for (auto s : v)
      if (s->failed) {
        set_err(failed_before ? "scene already failed" : "environment failed");
        return IPC_E_FAILED;
      }
    return IPC_OK;
  });
}

int ipc_get_state(ipc_scene s, double *pos, double *vel, double *cauchy, double *von_mises) {
  return guarded([&]() {
    if (!s || !pos) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = *s->world;
    std::lock_guard<std::mutex> lk(w.mu);
    HC(hipSetDevice(w.device));
    get_x(w, s, w.W.x, pos);
    if (vel) get_x(w, s, w.W.v, vel);
    if (cauchy || von_mises) {
      const EnvDev &E = w.envs_h[s->slot];
      DBuf<double> c, m;
      c.ensure(6L * E.nt + 1);
      m.ensure(E.nt + 1);
      ipck::stress(w.stream, w.W, E.t_off, E.nt, c.p, m.p);
      if (cauchy) down(w, cauchy, c.p, 6L * E.nt);
      if (von_mises) down(w, von_mises, m.p, E.nt);
      HC(hipStreamSynchronize(w.stream));
    }
    return IPC_OK;
  });
}

int ipc_set_state(ipc_scene s, const double *pos, const double *vel, int32_t step) {
  return guarded([&]() {
    if (!s || !pos || step < 0) throw ApiError(IPC_E_ARG, "bad arguments");
    if (!finite_all(pos, 3L * s->host->nv) || (vel && !finite_all(vel, 3L * s->host->nv)))
      throw ApiError(IPC_E_ARG, "non-finite state");
    World &w = *s->world;
    std::lock_guard<std::mutex> lk(w.mu);
    HC(hipSetDevice(w.device));
    put_x(w, s, w.W.x, pos);
    std::vector<double> z(3L * s->host->nv, 0.0);
    put_x(w, s, w.W.v, vel ? vel : z.data());
    HC(hipStreamSynchronize(w.stream));
    s->step = step;
    s->failed = false;
    s->fail_reason = 0;
    set_status(w, s->slot, ipcw::ST_IDLE);
    return IPC_OK;
  });
}

int ipc_prof_enable(int32_t on) {
  return guarded([&]() {
    for (World *w : worlds_for_current_device()) {
      std::lock_guard<std::mutex> lk(w->mu);
      w->set_prof(on == 2 ? 2 : on != 0 ? 1 : 0);
    }
    return IPC_OK;
  });
}

int ipc_set_tuning(int32_t key, int64_t value) {
  return guarded([&]() {
    if (value < 0 && !((key == IPC_TUNE_WIDE_TILES || key == IPC_TUNE_POLL_BLOCK) && value == -1))
      throw ApiError(IPC_E_ARG, "tuning value must be >= 0");
    if (key == IPC_TUNE_LANES) {
      if (value < 1 || value > 16) throw ApiError(IPC_E_ARG, "lanes must be in [1, 16]");
      std::lock_guard<std::mutex> lk(g_worlds_mu);
      g_lanes = (int)value;
      return IPC_OK;
    }
    if (key != IPC_TUNE_TAIL_TILES && key != IPC_TUNE_FUSED_PCG && key != IPC_TUNE_NARROW &&
        key != IPC_TUNE_ADMIT_FAULTS && key != IPC_TUNE_ASYNC && key != IPC_TUNE_WIDE_TILES &&
        key != IPC_TUNE_POLL_BLOCK && key != IPC_TUNE_COARSE)
      throw ApiError(IPC_E_ARG, "unknown tuning key");
    if (key == IPC_TUNE_POLL_BLOCK && value != -1 && (value < 1 || value > 1024))
      throw ApiError(IPC_E_ARG, "poll block must be -1 or in [1, 1024]");
    for (World *pw : worlds_for_current_device()) {
      World &w = *pw;
      std::lock_guard<std::mutex> lk(w.mu);
      if (key == IPC_TUNE_TAIL_TILES)
        w.tail_tiles = (int)std::min<int64_t>(value, 1 << 30);
      else if (key == IPC_TUNE_FUSED_PCG)
        w.set_fused(value != 0);
      else if (key == IPC_TUNE_ADMIT_FAULTS)
        w.admit_faults = (int)std::min<int64_t>(value, 1 << 30);
      else if (key == IPC_TUNE_ASYNC)
        w.async_mode = value != 0;
      else if (key == IPC_TUNE_WIDE_TILES)
        w.wide_tiles = (int)std::min<int64_t>(value, 1 << 30);  // -1: the default
      else if (key == IPC_TUNE_POLL_BLOCK)
        w.poll_block = (int)value;
      else if (key == IPC_TUNE_COARSE)
        w.set_coarse(value != 0);
      else
        w.narrow = value != 0;
    }
    return IPC_OK;
  });
}

int ipc_get_tuning(int32_t key, int64_t *value) {
  return guarded([&]() {
    if (!value) throw ApiError(IPC_E_ARG, "null output");
    if (key == IPC_TUNE_LANES) {
      *value = lanes_setting();
      return IPC_OK;
    }
    World &w = world_for_current_device();
    std::lock_guard<std::mutex> lk(w.mu);
    if (key == IPC_TUNE_TAIL_TILES)
      *value = w.tail_tiles;
    else if (key == IPC_TUNE_FUSED_PCG)
      *value = w.fused_pcg;
    else if (key == IPC_TUNE_NARROW)
      *value = w.narrow;
    else if (key == IPC_TUNE_ADMIT_FAULTS)
      *value = w.admit_faults;
    else if (key == IPC_TUNE_ASYNC)
      *value = w.async_mode;
    else if (key == IPC_TUNE_WIDE_TILES)
      *value = w.wide_tiles;  // -1: the default (every FP64 launch, no mixed one)
    else if (key == IPC_TUNE_POLL_BLOCK)
      *value = w.poll_block;  // -1: the default (8 mixed, 4 FP64)
    else if (key == IPC_TUNE_COARSE)
      *value = w.coarse;
    else
      throw ApiError(IPC_E_ARG, "unknown tuning key");
    return IPC_OK;
  });
}

// an entry point of this library called from another one: its error code
// and message are passed on
#define HC_API(call)                                       \
  do {                                                     \
    const int rc_ = (call);                                \
    if (rc_ != IPC_OK) throw ApiError(rc_, ipc_last_error()); \
  } while (0)

// Per-workload tuning of the scheduling knobs that change no result (the
// four-slot product variant's tile threshold and the PCG poll block): every
// candidate pair is timed on copies of the caller's scenes set to their
// current state, the fastest is applied to the device and recorded in the
// cache file under the workload's key (scene count, total tets to three
// significant digits, precisions, lane count), so a later call with the same
// key applies it without timing.
int ipc_autotune(const ipc_scene *scenes, int32_t n, int32_t steps, const char *cache_path, int64_t out[3]) {
  return guarded([&]() {
    if (!scenes || n <= 0 || steps <= 0 || steps > 64 || !out) throw ApiError(IPC_E_ARG, "bad arguments");
    std::vector<ipc_scene> orig(scenes, scenes + n);
    long long tets = 0;
    int prec_mask = 0;
    for (ipc_scene s : orig) {
      if (!s) throw ApiError(IPC_E_ARG, "null scene");
      tets += s->host->nt;
      prec_mask |= 1 << (s->host->precision == IPC_MIXED ? 1 : 0);
    }
    long long mag = 1;
    while (tets / mag >= 1000) mag *= 10;
    char key[160];
    std::snprintf(key, sizeof key, "envs=%d tets=%lld prec=%d lanes=%d", n, (tets + mag / 2) / mag * mag, prec_mask,
                  lanes_setting());
    auto apply = [&](int64_t wide, int64_t poll) {
      for (World *pw : worlds_for_current_device()) {
        std::lock_guard<std::mutex> lk(pw->mu);
        pw->wide_tiles = (int)wide;
        pw->poll_block = (int)poll;
      }
    };
    if (cache_path) {
      std::ifstream in(cache_path);
      std::string line;
      while (std::getline(in, line)) {
        const size_t tab = line.find('\t');
        if (tab == std::string::npos || line.compare(0, tab, key) != 0 || tab != std::strlen(key)) continue;
        long long wide = 0, poll = 0;
        double ms = 0.0;
        if (std::sscanf(line.c_str() + tab + 1, "%lld %lld %lf", &wide, &poll, &ms) == 3 &&
            (poll == -1 || (poll >= 1 && poll <= 1024))) {
          apply(wide, poll);
          out[0] = wide;
          out[1] = poll;
          out[2] = 1;
          return IPC_OK;
        }
      }
    }
    // copies of the scenes at their current state
    std::vector<ipc_scene> copies;
    std::vector<std::vector<double>> pos(n), vel(n);
    auto destroy = [&]() {
      for (ipc_scene c : copies) ipc_destroy_scene(c);
      copies.clear();
    };
    try {
      for (int i = 0; i < n; ++i) {
        ipc_scene s = orig[i];
        pos[i].resize(3L * s->host->nv);
        vel[i].resize(3L * s->host->nv);
        HC_API(ipc_get_state(s, pos[i].data(), vel[i].data(), nullptr, nullptr));
        World &w = world_for_new_scene();
        std::lock_guard<std::mutex> lk(w.mu);
        int slot = w.add_scene(*s->host);
        auto *c = new ipc_scene_s();
        c->world = &w;
        c->slot = slot;
        c->host = std::make_unique<HostScene>(*s->host);
        copies.push_back(c);
      }
      auto reset = [&]() {
        for (int i = 0; i < n; ++i) HC_API(ipc_set_state(copies[i], pos[i].data(), vel[i].data(), orig[i]->step));
      };
      // the current setting first: a candidate replaces it only when it is
      // at least 3% faster (each timed twice, the faster run counts)
      World &w0 = world_for_current_device();
      std::vector<std::pair<int64_t, int64_t>> cand = {{w0.wide_tiles, w0.poll_block}};
      for (int64_t wd : {int64_t(0), int64_t(64), int64_t(1) << 30})
        for (int64_t pl : {int64_t(4), int64_t(8), int64_t(16)})
          if (!(wd == cand[0].first && pl == cand[0].second)) cand.push_back({wd, pl});
      double best = HUGE_VAL, current = HUGE_VAL;
      int64_t bw = cand[0].first, bp = cand[0].second;
      for (size_t k = 0; k < cand.size(); ++k) {
        apply(cand[k].first, cand[k].second);
        if (k == 0) {  // buffers grow to this workload's sizes once, untimed
          reset();
          run_steps(copies, steps, nullptr);
        }
        double ms = HUGE_VAL;
        for (int rep = 0; rep < 2; ++rep) {
          reset();
          const auto t0 = std::chrono::steady_clock::now();
          run_steps(copies, steps, nullptr);
          ms = std::min(ms, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        if (k == 0) current = ms;
        if (ms < best && (k == 0 || ms < 0.97 * current)) {
          best = ms;
          bw = cand[k].first;
          bp = cand[k].second;
        }
      }
      destroy();
      apply(bw, bp);
      out[0] = bw;
      out[1] = bp;
      out[2] = 0;
      if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        if (!o) throw ApiError(IPC_E_ARG, "cannot write the tuning cache file");
        o << key << '\t' << bw << ' ' << bp << ' ' << best / steps << '\n';
      }
    } catch (...) {
      destroy();
      throw;
    }
    return IPC_OK;
  });
}

int ipc_prof_reset(void) {
  return guarded([&]() {
    for (World *w : worlds_for_current_device()) {
      std::lock_guard<std::mutex> lk(w->mu);
      w->prof_reset();
    }
    return IPC_OK;
  });
}

int ipc_prof_read(double *out) {
  return guarded([&]() {
    if (!out) throw ApiError(IPC_E_ARG, "null output");
    for (int k = 0; k < 12; ++k) out[k] = 0.0;
    for (World *pw : worlds_for_current_device()) {
      World &w = *pw;
      std::lock_guard<std::mutex> lk(w.mu);
      unsigned long long b[4] = {0, 0, 0, 0};
      if (w.prof_bytes.p) {
        HC(hipMemcpyAsync(b, w.prof_bytes.p, 32, hipMemcpyDeviceToHost, w.stream));
        HC(hipStreamSynchronize(w.stream));
      }
      out[0] += w.prof_ms;
      out[1] += (double)w.prof_launches;
      out[2] += (double)(b[0] + b[1]);
      out[3] += w.prof_ms_big;
      out[4] += (double)w.prof_launches_big;
      out[5] += (double)b[1];
      out[6] += w.prof_ms_iter;
      out[7] += (double)w.prof_launches;
      out[8] += (double)b[2];
      if (w.prof_skipped) std::fprintf(stderr, "[ipc] %lld timed PCG samples left out: events not recorded\n", w.prof_skipped);
      out[9] += w.prof_ms_asm;
      out[10] += (double)w.prof_asm;
      out[11] += (double)b[3];
    }
    return IPC_OK;
  });
}

int ipc_prof_pairs(double *out) {
  return guarded([&]() {
    if (!out) throw ApiError(IPC_E_ARG, "null output");
    for (int k = 0; k < 3; ++k) out[k] = 0.0;
    for (World *pw : worlds_for_current_device()) {
      std::lock_guard<std::mutex> lk(pw->mu);
      out[0] += (double)pw->prof_cands;
      out[1] += (double)pw->prof_bar;
      out[2] += (double)pw->prof_fric;
    }
    return IPC_OK;
  });
}

int ipc_scene_sizes(ipc_scene s, int64_t out[7]) {
  if (!s || !out) return IPC_E_ARG;
  out[0] = s->host->nv;
  out[1] = s->host->nt;
  out[2] = s->host->ntri;
  out[3] = s->host->ne;
  out[4] = s->host->nsv;
  out[5] = s->step;
  out[6] = s->failed ? 1 : 0;
  return IPC_OK;
}

// ---------------------------------------------------------------------------
// inspection entry points
// ---------------------------------------------------------------------------
namespace {

struct DebugScope {
  World &w;
  ipc_scene s;
  std::vector<double> saved_x;
  std::lock_guard<std::mutex> lk;
  DebugScope(ipc_scene sc) : w(*sc->world), s(sc), lk(sc->world->mu) {
    HC(hipSetDevice(w.device));
    saved_x.resize(3L * s->host->nv);
    get_x(w, s, w.W.x, saved_x.data());
    w.set_batch({s->slot});
    set_status(w, s->slot, ipcw::ST_ACTIVE);
  }
  ~DebugScope() {
    try {
      put_x(w, s, w.W.x, saved_x.data());
      set_status(w, s->slot, s->failed ? ipcw::ST_FAILED : ipcw::ST_IDLE);
    } catch (...) {
    }
  }
};

}  // namespace

int64_t ipc_debug_candidates(ipc_scene s, const double *x, const double *p, int32_t *out, int64_t cap) {
  try {
    if (!s || !x) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    if (p) put_x(w, s, w.W.p, p);
    int n = w.broad_phase(w.W.x, p ? w.W.p : nullptr);
    std::vector<int2> c(n);
    down(w, c.data(), w.cand.p, n);
    HC(hipStreamSynchronize(w.stream));
    const HostScene &H = *s->host;
    const EnvDev &E = w.envs_h[s->slot];
    for (int64_t i = 0; i < n && i < cap; ++i) {
      int32_t *r = out + 5 * i;
      if (c[i].x >= 0) {
        const auto &t = H.tris[c[i].y - E.tri_off];
        r[0] = 0;
        r[1] = H.sverts[c[i].x - E.sv_off];
        r[2] = t[0];
        r[3] = t[1];
        r[4] = t[2];
      } else {
        const auto &A = H.edges[~c[i].x - E.e_off], &Bq = H.edges[c[i].y - E.e_off];
        r[0] = 1;
        r[1] = A[0];
        r[2] = A[1];
        r[3] = Bq[0];
        r[4] = Bq[1];
      }
    }
    return n;
  } catch (const std::exception &e) {
    return api_error(e);
  }
}

int64_t ipc_debug_active(ipc_scene s, const double *x, int32_t *out, double *d2, int64_t cap) {
  try {
    if (!s || !x) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    int n = w.broad_phase(w.W.x, nullptr);
    w.active_pairs(n, w.W.x);
    std::vector<int2> c(n);
    std::vector<int> ty(n), fl(n);
    std::vector<double> dd(n);
    down(w, c.data(), w.cand.p, n);
    down(w, ty.data(), w.cand_type.p, n);
    down(w, fl.data(), w.cand_flag.p, n);
    down(w, dd.data(), w.cand_d2.p, n);
    HC(hipStreamSynchronize(w.stream));
    const HostScene &H = *s->host;
    const EnvDev &E = w.envs_h[s->slot];
    int64_t k = 0;
    for (int i = 0; i < n; ++i) {
      if (!fl[i]) continue;
      if (k < cap) {
        int32_t *r = out + 6 * k;
        if (c[i].x >= 0) {
          const auto &t = H.tris[c[i].y - E.tri_off];
          r[0] = 0;
          r[1] = H.sverts[c[i].x - E.sv_off];
          r[2] = t[0];
          r[3] = t[1];
          r[4] = t[2];
        } else {
          const auto &A = H.edges[~c[i].x - E.e_off], &Bq = H.edges[c[i].y - E.e_off];
          r[0] = 1;
          r[1] = A[0];
          r[2] = A[1];
          r[3] = Bq[0];
          r[4] = Bq[1];
        }
        r[5] = ty[i];
        if (d2) d2[k] = dd[i];
      }
      ++k;
    }
    return k;
  } catch (const std::exception &e) {
    return api_error(e);
  }
}

int ipc_debug_bodies(ipc_scene s, int32_t *vbody, double *frame) {
  return guarded([&]() {
    if (!s) throw ApiError(IPC_E_ARG, "bad arguments");
    static_assert(ipcw::kCoarseBodies == IPC_COARSE_BODIES, "coarse body count");
    const HostScene &H = *s->host;
    if (vbody)
      for (int i = 0; i < H.nv; ++i) vbody[i] = H.vbody[i];
    if (frame)
      for (int b = 0; b < H.nbody; ++b) {
        for (int k = 0; k < 3; ++k) frame[4 * b + k] = H.cb[b][k];
        frame[4 * b + 3] = H.cscale[b];
      }
    return H.nbody;
  });
}

int ipc_debug_begin_step(ipc_scene s, double *x_start) {
  return guarded([&]() {
    if (!s) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = *s->world;
    std::vector<double> saved_x, saved_v;
    {
      DebugScope D(s);
      w.envs_h[s->slot].step = s->step;
      w.upload_env(s->slot);
      ipck::set_phase(w.stream, w.S, w.B, ipcw::PH_BEGIN);
      ipck::env_begin(w.stream, w.envs_d, w.S, w.B);
      ipck::begin_step(w.stream, w.W, w.envs_d, w.S, w.B);
      int nc = w.broad_phase(w.W.xn, w.W.p);
      w.friction_setup(nc);
      ipck::ccd_init(w.stream, w.S, w.B);
      ipck::accd(w.stream, w.W, w.envs_d, w.S, w.L, nc, w.W.xn, w.W.p);
      ipck::dbc_check_J(w.stream, w.W, w.envs_d, w.S, w.B);
      ipck::env_dbc(w.stream, w.S, w.B);
      ipck::apply_dbc(w.stream, w.W, w.envs_d, w.S, w.B);
      ipck::set_phase(w.stream, w.S, w.B, ipcw::PH_ITER);
      if (x_start) get_x(w, s, w.W.x, x_start);
    }
    return IPC_OK;
  });
}

int ipc_debug_gradient(ipc_scene s, const double *x, double *g) {
  return guarded([&]() {
    if (!s || !x || !g) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    w.assemble_system(0);
    get_x(w, s, w.W.g, g);
    return IPC_OK;
  });
}

double ipc_debug_energy(ipc_scene s, const double *x) {
  try {
    if (!s || !x) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    std::vector<double> z(3L * s->host->nv, 0.0);
    put_x(w, s, w.W.p, z.data());
    int n = w.broad_phase(w.W.x, nullptr);
    ipck::ccd_init(w.stream, w.S, w.B);
    ipck::ls_init(w.stream, w.S, w.B);
    ipck::energy(w.stream, w.W, w.envs_d, w.S, w.B, w.L, n, w.n_fric, 1, w.S.E0);
    double E0;
    down(w, &E0, w.S.E0 + s->slot, 1);
    HC(hipStreamSynchronize(w.stream));
    return E0;
  } catch (const std::exception &e) {
    api_error(e);
    return std::nan("");
  }
}

int ipc_debug_hessian_apply(ipc_scene s, const double *x, const double *v, double *y) {
  return guarded([&]() {
    if (!s || !x || !v || !y) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    w.assemble_system(0);
    put_x(w, s, w.W.r, v);
    ipck::spmv_debug(w.stream, w.W, w.envs_d, w.S, w.B, w.L, w.W.r, w.W.q);
    get_x(w, s, w.W.q, y);
    return IPC_OK;
  });
}

int ipc_debug_newton_dir(ipc_scene s, const double *x, double *p, int64_t *pcg_iters) {
  return guarded([&]() {
    if (!s || !x || !p) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    int mixed = s->host->precision == IPC_MIXED;
    w.assemble_system(mixed);
    w.solve(mixed);
    get_x(w, s, w.W.p, p);
    if (pcg_iters) {
      int it;
      down(w, &it, w.S.pcg_it + s->slot, 1);
      HC(hipStreamSynchronize(w.stream));
      *pcg_iters = it;
    }
    return IPC_OK;
  });
}

double ipc_debug_ccd_bound(ipc_scene s, const double *x, const double *p) {
  try {
    if (!s || !x || !p) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    put_x(w, s, w.W.p, p);
    int n = w.broad_phase(w.W.x, w.W.p);
    ipck::ccd_init(w.stream, w.S, w.B);
    ipck::accd(w.stream, w.W, w.envs_d, w.S, w.L, n, w.W.x, w.W.p);
    unsigned long long bits;
    down(w, &bits, w.S.amax_bits + s->slot, 1);
    HC(hipStreamSynchronize(w.stream));
    double a;
    std::memcpy(&a, &bits, 8);
    return a;
  } catch (const std::exception &e) {
    api_error(e);
    return std::nan("");
  }
}

double ipc_debug_inversion_bound(ipc_scene s, const double *x, const double *p) {
  try {
    if (!s || !x || !p) throw ApiError(IPC_E_ARG, "bad arguments");
    DebugScope D(s);
    World &w = D.w;
    put_x(w, s, w.W.x, x);
    put_x(w, s, w.W.p, p);
    ipck::ccd_init(w.stream, w.S, w.B);
    ipck::inv_bound(w.stream, w.W, w.envs_d, w.S, w.B, 1);
    unsigned long long bits;
    down(w, &bits, w.S.amax_bits + s->slot, 1);
    HC(hipStreamSynchronize(w.stream));
    double a;
    std::memcpy(&a, &bits, 8);
    return a;
  } catch (const std::exception &e) {
    api_error(e);
    return std::nan("");
  }
}

int ipc_ccd_bound_pairs(int32_t kind, int64_t n, const double *x12, const double *p12, double s, double *alpha) {
  return guarded([&]() {
    if ((kind != 0 && kind != 1) || n < 0 || n > INT32_MAX || (n > 0 && (!x12 || !p12)) || !alpha ||
        !(s > 0.0 && s < 1.0))
      throw ApiError(IPC_E_ARG, "bad arguments");
    if (!finite_all(x12, 12 * n) || !finite_all(p12, 12 * n)) throw ApiError(IPC_E_ARG, "non-finite pair data");
    World &w = world_for_current_device();
    std::lock_guard<std::mutex> lk(w.mu);
    DBuf<double> X, P, part, out;
    X.ensure(12 * n + 1);
    P.ensure(12 * n + 1);
    part.ensure(ipck::pairs_ccd_parts(n) + 1);
    out.ensure(1);
    w.up(X.p, x12, 12 * n);
    w.up(P.p, p12, 12 * n);
    ipck::pairs_ccd_bound(w.stream, kind, (int)n, X.p, P.p, s, part.p, out.p);
    HC(hipGetLastError());
    down(w, alpha, out.p, 1);
    HC(hipStreamSynchronize(w.stream));
    return IPC_OK;
  });
}

int ipc_ccd_bound_pairs_noalloc(int32_t kind, int64_t n, const double *x12, const double *p12, double s,
                                double *alpha, void *stream) {
  // no allocation anywhere on this path: no exceptions, no containers
  if ((kind != 0 && kind != 1) || n < 0 || (n > 0 && (!x12 || !p12)) || !alpha || !(s > 0.0 && s < 1.0)) {
    set_err("ipc_ccd_bound_pairs_noalloc: bad arguments");
    return IPC_E_ARG;
  }
  if (n > ipck::noalloc_max_pairs()) {
    set_err("ipc_ccd_bound_pairs_noalloc: more pairs than the fixed scratch holds (8388608)");
    return IPC_E_ARG;
  }
  double *part = nullptr;
  hipError_t e = ipck::noalloc_scratch(&part);
  if (e == hipSuccess) {
    ipck::pairs_ccd_bound(static_cast<hipStream_t>(stream), kind, (int)n, x12, p12, s, part, alpha);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    set_err(hipGetErrorString(e));
    return IPC_E_DEVICE;
  }
  return IPC_OK;
}

int ipc_grasp_metrics(ipc_scene s, int32_t n_obj_tris, const int32_t *obj_tris, int32_t n_hand_tris,
                      const int32_t *hand_tris, int32_t n_samples, const int32_t *sample_tri, const double *sample_uv,
                      double *D, double *sdf) {
  return guarded([&]() {
    if (!s || n_obj_tris < 1 || !obj_tris || n_hand_tris < 1 || !hand_tris || n_samples < 1 || !sample_tri ||
        !sample_uv || !D)
      throw ApiError(IPC_E_ARG, "bad arguments");
    const int nv = s->host->nv;
    for (int64_t k = 0; k < 3L * n_obj_tris; ++k)
      if (obj_tris[k] < 0 || obj_tris[k] >= nv) throw ApiError(IPC_E_ARG, "manipuland triangle index out of range");
    for (int64_t k = 0; k < 3L * n_hand_tris; ++k)
      if (hand_tris[k] < 0 || hand_tris[k] >= nv) throw ApiError(IPC_E_ARG, "gripper triangle index out of range");
    for (int k = 0; k < n_samples; ++k) {
      const double u = sample_uv[2 * k], v = sample_uv[2 * k + 1];
      if (sample_tri[k] < 0 || sample_tri[k] >= n_hand_tris || !(u >= 0.0) || !(v >= 0.0) || !(u + v <= 1.0 + 1e-12))
        throw ApiError(IPC_E_ARG, "bad sample (triangle index or barycentric coordinates)");
    }
    World &w = *s->world;
    std::lock_guard<std::mutex> lk(w.mu);
    HC(hipSetDevice(w.device));
    const int vo = w.envs_h[s->slot].v_off;
    std::vector<int> ot(obj_tris, obj_tris + 3L * n_obj_tris), ht(hand_tris, hand_tris + 3L * n_hand_tris);
    for (int &v : ot) v += vo;
    for (int &v : ht) v += vo;
    DBuf<int> OT, HT, ST;
    DBuf<double> UV, SDF, part, out;
    OT.ensure(ot.size());
    HT.ensure(ht.size());
    ST.ensure(n_samples);
    UV.ensure(2L * n_samples);
    SDF.ensure(n_samples);
    part.ensure(ipck::sdf_parts(n_samples) + 1);
    out.ensure(2);
    w.up(OT.p, ot.data(), ot.size());
    w.up(HT.p, ht.data(), ht.size());
    w.up(ST.p, sample_tri, n_samples);
    w.up(UV.p, sample_uv, 2L * n_samples);
    ipck::grasp_metrics(w.stream, w.W.x, OT.p, n_obj_tris, HT.p, ST.p, UV.p, n_samples, SDF.p, part.p, out.p);
    HC(hipGetLastError());
    down(w, D, out.p, 2);
    if (sdf) down(w, sdf, SDF.p, n_samples);
    HC(hipStreamSynchronize(w.stream));
    return IPC_OK;
  });
}

// ---- grasp validation (Sec. III-D) -------------------------------------------
namespace {
// where a scene's protocol controls sit in the world's motion array
size_t ctl_offset(World &w, ipc_scene s) {
  const EnvDev &E = w.envs_h[s->slot];
  return w.recs[s->slot].mo_off + (12L * E.n_groups + 3) * E.n_motion;
}

// force on every tag from every tag at the scene's positions (caller holds w.mu)
void contact_forces_locked(World &w, ipc_scene s, const int32_t *tags, int ntags, double *out) {
  DBuf<int> T, fab;
  DBuf<double> f, o;
  const int nv = s->host->nv;
  T.ensure(nv);
  o.ensure(3L * ntags * ntags);
  w.up(T.p, tags, nv);
  w.set_batch({s->slot});
  set_status(w, s->slot, ipcw::ST_ACTIVE);
  try {
    int nc = w.broad_phase(w.W.x, nullptr);
    int na = w.active_pairs(nc, w.W.x);
    f.ensure(3L * na + 3);
    fab.ensure(na + 1);
    ipck::contact_forces(w.stream, w.W, w.envs_d, w.S, w.L, na, T.p, w.envs_h[s->slot].v_off, ntags, f.p, fab.p, o.p);
    HC(hipGetLastError());
    down(w, out, o.p, 3L * ntags * ntags);
    HC(hipStreamSynchronize(w.stream));
  } catch (...) {
    set_status(w, s->slot, s->failed ? ipcw::ST_FAILED : ipcw::ST_IDLE);
    throw;
  }
  set_status(w, s->slot, s->failed ? ipcw::ST_FAILED : ipcw::ST_IDLE);
}

double com_of(const std::vector<double> &pos, const HostScene &H, const int32_t *tags, int k) {
  double m = 0.0, c = 0.0;
  for (int i = 0; i < H.nv; ++i)
    if (tags[i] == 0) {
      m += H.mass[i];
      c += H.mass[i] * pos[3 * i + k];
    }
  return m > 0 ? c / m : 0.0;
}
}  // namespace

int ipc_hold_group(ipc_scene s, int32_t group, int32_t row) {
  return guarded([&]() {
    if (!s || group < 0 || group >= s->host->n_groups || row < -1) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = *s->world;
    std::lock_guard<std::mutex> lk(w.mu);
    HC(hipSetDevice(w.device));
    const double v = row;
    HC(hipMemcpyAsync(w.W.motion + ctl_offset(w, s) + group, &v, 8, hipMemcpyHostToDevice, w.stream));
    HC(hipStreamSynchronize(w.stream));
    return IPC_OK;
  });
}

int ipc_set_gravity(ipc_scene s, const double *g) {
  return guarded([&]() {
    if (!s || (g && !finite_all(g, 3))) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = *s->world;
    std::lock_guard<std::mutex> lk(w.mu);
    HC(hipSetDevice(w.device));
    const double v[4] = {g ? 1.0 : 0.0, g ? g[0] : 0.0, g ? g[1] : 0.0, g ? g[2] : 0.0};
    HC(hipMemcpyAsync(w.W.motion + ctl_offset(w, s) + s->host->n_groups, v, 32, hipMemcpyHostToDevice, w.stream));
    HC(hipStreamSynchronize(w.stream));
    return IPC_OK;
  });
}

int ipc_contact_forces(ipc_scene s, const int32_t *tags, int32_t ntags, double *out) {
  return guarded([&]() {
    if (!s || !tags || ntags < 1 || ntags > 64 || !out) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = *s->world;
    std::lock_guard<std::mutex> lk(w.mu);
    HC(hipSetDevice(w.device));
    contact_forces_locked(w, s, tags, ntags, out);
    return IPC_OK;
  });
}

int ipc_validate_grasp(ipc_scene s, const ipc_grasp_protocol *p, ipc_grasp_result *r) {
  return guarded([&]() {
    if (!s || !p || !r || !p->vertex_tag || p->n_fingers < 1 || p->n_fingers > IPC_MAX_FINGERS ||
        !p->finger_of_group || !(p->force_limit > 0) || p->max_close_steps < 0 || p->settle_steps < 0 ||
        p->phase_steps < 1 || !(p->gravity >= 0) || !(p->com_factor > 0))
      throw ApiError(IPC_E_ARG, "bad protocol");
    const HostScene &H = *s->host;
    for (int g = 0; g < H.n_groups; ++g)
      if (p->finger_of_group[g] < 0 || p->finger_of_group[g] > p->n_fingers)
        throw ApiError(IPC_E_ARG, "finger_of_group out of range");
    const int nt = p->n_fingers + 1;
    std::memset(r, 0, sizeof(*r));
    for (int f = 0; f < IPC_MAX_FINGERS; ++f) r->halt_step[f] = -1;
    World &w = *s->world;
    std::vector<double> F(3L * nt * nt), pos(3L * H.nv);
    auto step1 = [&]() {
      if (s->failed) return false;
      ipc_step_info info{};
      run_steps_lane({s}, 1, &info);
      r->steps_run += 1;
      if (s->failed) {
        r->failed = 1;
        r->fail_reason = s->fail_reason;
        return false;
      }
      return true;
    };
    auto forces = [&]() {
      std::lock_guard<std::mutex> lk(w.mu);
      contact_forces_locked(w, s, p->vertex_tag, nt, F.data());
    };
    auto finger_force = [&](int f) {  // |force on finger f from the manipuland|
      const double *v = &F[3L * (f * nt + 0)];
      return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    };
    auto com = [&](double c[3]) {
      {
        std::lock_guard<std::mutex> lk(w.mu);
        get_x(w, s, w.W.x, pos.data());
      }
      for (int k = 0; k < 3; ++k) c[k] = com_of(pos, H, p->vertex_tag, k);
    };
    HC(hipSetDevice(w.device));
    const double zero[3] = {0, 0, 0};
    int rc = ipc_set_gravity(s, zero);  // gravity off while the fingers close
    if (rc != IPC_OK) return rc;
    // closing: each finger is halted once its contact force exceeds the limit
    int halted = 0;
    for (int n = 0; n < p->max_close_steps && halted < p->n_fingers; ++n) {
      if (!step1()) return IPC_OK;
      forces();
      for (int f = 1; f <= p->n_fingers; ++f) {
        if (r->halt_step[f - 1] >= 0 || !(finger_force(f) > p->force_limit)) continue;
        r->halt_step[f - 1] = s->step;
        r->finger_force[f - 1] = finger_force(f);
        ++halted;
        // the finger's groups keep the targets they have now reached
        const int row = std::min(s->step, H.n_motion - 1);
        for (int g = 0; g < H.n_groups; ++g)
          if (p->finger_of_group[g] == f && (rc = ipc_hold_group(s, g, row)) != IPC_OK) return rc;
      }
    }
    // fingers still moving stop where they are after the closing phase
    {
      const int row = std::min(s->step, H.n_motion - 1);
      for (int g = 0; g < H.n_groups; ++g)
        if (p->finger_of_group[g] > 0 && r->halt_step[p->finger_of_group[g] - 1] < 0 &&
            (rc = ipc_hold_group(s, g, row)) != IPC_OK)
          return rc;
    }
    for (int n = 0; n < p->settle_steps; ++n)
      if (!step1()) return IPC_OK;
    // six axis-aligned gravity phases
    for (int ph = 0; ph < 6; ++ph) {
      double g[3] = {0, 0, 0};
      g[ph / 2] = (ph % 2 == 0 ? 1.0 : -1.0) * p->gravity;
      if ((rc = ipc_set_gravity(s, g)) != IPC_OK) return rc;
      double c0[3], cp[3], c1[3];
      com(c0);
      for (int n = 0; n < p->phase_steps; ++n) {
        if (n == p->phase_steps - 1) com(cp);
        if (!step1()) return IPC_OK;
      }
      com(c1);
      double sh = 0.0, dr = 0.0;
      for (int k = 0; k < 3; ++k) {
        sh += (c1[k] - c0[k]) * (c1[k] - c0[k]);
        dr += (c1[k] - cp[k]) * (c1[k] - cp[k]);
      }
      r->com_shift[ph] = std::sqrt(sh);
      r->com_drift[ph] = std::sqrt(dr);
    }
    forces();
    double fsum = 0.0;
    for (int f = 1; f <= p->n_fingers; ++f) fsum += finger_force(f);
    r->in_contact = fsum > 0.0;
    const double limit = p->com_factor * H.eps_v * H.dt;
    bool still = true;
    for (int ph = 0; ph < 6; ++ph) still &= r->com_drift[ph] <= limit;
    r->stable = (r->in_contact && still) ? 1 : 0;
    return IPC_OK;
  });
}

// element-level routines on the device
int64_t ipc_debug_tet_first_root(int64_t n, const double *x12, const double *p12, double tmax, double *t, double *k4) {
  try {
    if (n < 0 || (n > 0 && (!x12 || !p12 || !t || !k4)) || !(tmax > 0)) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = world_for_current_device();
    std::lock_guard<std::mutex> lk(w.mu);
    DBuf<double> X, P, T, K;
    X.ensure(12 * n + 1);
    P.ensure(12 * n + 1);
    T.ensure(n + 1);
    K.ensure(4 * n + 1);
    w.up(X.p, x12, 12 * n);
    w.up(P.p, p12, 12 * n);
    ipck::dbg_tet_root(w.stream, (int)n, X.p, P.p, tmax, T.p, K.p);
    down(w, t, T.p, n);
    down(w, k4, K.p, 4 * n);
    HC(hipStreamSynchronize(w.stream));
    return n;
  } catch (const std::exception &e) {
    return api_error(e);
  }
}

int ipc_debug_classify(int32_t kind, int64_t n, const double *x12, int32_t *types, double *d2) {
  return guarded([&]() {
    if (n < 0 || (n > 0 && (!x12 || !types || !d2))) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = world_for_current_device();
    std::lock_guard<std::mutex> lk(w.mu);
    DBuf<double> X, D2;
    DBuf<int> T;
    X.ensure(12 * n + 1);
    D2.ensure(n + 1);
    T.ensure(n + 1);
    w.up(X.p, x12, 12 * n);
    ipck::dbg_classify(w.stream, kind, (int)n, X.p, T.p, D2.p);
    down(w, types, T.p, n);
    down(w, d2, D2.p, n);
    HC(hipStreamSynchronize(w.stream));
    return IPC_OK;
  });
}

int ipc_debug_pair_barrier(int32_t kind, int32_t type, const double *x12, double dhat, double kappa, double eps_x,
                           int32_t project, double *energy, double *g12, double *H144) {
  return guarded([&]() {
    if (!x12) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = world_for_current_device();
    std::lock_guard<std::mutex> lk(w.mu);
    DBuf<double> X, O;
    X.ensure(12);
    O.ensure(157);
    w.up(X.p, x12, 12);
    ipck::dbg_pair(w.stream, kind, type, X.p, dhat, kappa, eps_x, project, O.p);
    double o[157];
    down(w, o, O.p, 157);
    HC(hipStreamSynchronize(w.stream));
    if (energy) *energy = o[0];
    if (g12) std::memcpy(g12, o + 1, 12 * 8);
    if (H144) std::memcpy(H144, o + 13, 144 * 8);
    return IPC_OK;
  });
}

int ipc_debug_tet_elastic(const double *X12, const double *x12, double E, double nu, int32_t project, double *energy,
                          double *g12, double *H144) {
  return guarded([&]() {
    if (!X12 || !x12) throw ApiError(IPC_E_ARG, "bad arguments");
    (void)project;
    World &w = world_for_current_device();
    std::lock_guard<std::mutex> lk(w.mu);
    DBuf<double> XR, X, O;
    XR.ensure(12);
    X.ensure(12);
    O.ensure(157);
    w.up(XR.p, X12, 12);
    w.up(X.p, x12, 12);
    double mu = E / (2.0 * (1.0 + nu)), la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    ipck::dbg_tet(w.stream, XR.p, X.p, mu, la, O.p);
    double o[157];
    down(w, o, O.p, 157);
    HC(hipStreamSynchronize(w.stream));
    if (energy) *energy = o[0];
    if (g12) std::memcpy(g12, o + 1, 12 * 8);
    if (H144) std::memcpy(H144, o + 13, 144 * 8);
    return std::isfinite(o[0]) ? IPC_OK : IPC_E_INVERTED;
  });
}

int64_t ipc_debug_accd(int32_t kind, int64_t n, const double *x12, const double *p12, double sfac, double *t) {
  try {
    if (n < 0 || (n > 0 && (!x12 || !p12 || !t))) throw ApiError(IPC_E_ARG, "bad arguments");
    World &w = world_for_current_device();
    std::lock_guard<std::mutex> lk(w.mu);
    DBuf<double> X, P, T;
    X.ensure(12 * n + 1);
    P.ensure(12 * n + 1);
    T.ensure(n + 1);
    w.up(X.p, x12, 12 * n);
    w.up(P.p, p12, 12 * n);
    ipck::dbg_accd(w.stream, kind, (int)n, X.p, P.p, sfac, T.p);
    down(w, t, T.p, n);
    HC(hipStreamSynchronize(w.stream));
    return n;
  } catch (const std::exception &e) {
    return api_error(e);
  }
}

int ipc_server_create(int64_t budget_bytes, int32_t max_slots, ipc_server *out) {
  return guarded([&]() {
    if (!out || budget_bytes <= 0 || max_slots < 0) throw ApiError(IPC_E_ARG, "bad server arguments");
    auto sv = std::make_unique<ipc_server_s>();
    sv->lanes = worlds_for_current_device();
    sv->lanes.resize(std::min<size_t>(sv->lanes.size(), (size_t)lanes_setting()));
    sv->running.resize(sv->lanes.size());
    sv->admitting.resize(sv->lanes.size());
    sv->budget = budget_bytes;
    sv->auto_slots = max_slots == 0;
    sv->max_slots = sv->auto_slots ? 8 * (int32_t)std::max<size_t>(1, sv->lanes.size()) : max_slots;
    sv->best_cap = sv->max_slots;
    for (size_t k = 0; k < sv->lanes.size(); ++k) sv->workers.emplace_back(server_loop, sv.get(), k);
    *out = sv.release();
    return IPC_OK;
  });
}

int ipc_server_submit(ipc_server srv, const ipc_scene_desc *desc, int32_t n_steps, int64_t *id) {
  return guarded([&]() {
    if (!srv || !id || n_steps < 1) throw ApiError(IPC_E_ARG, "bad arguments");
    const double t_arrival = srv->now();  // validation and copying count toward latency
    auto host = preprocess(desc);
    auto r = std::make_unique<Request>();
    r->bytes = (int64_t)srv->lanes[0]->scene_bytes(*host);
    if (r->bytes > srv->budget) throw ApiError(IPC_E_NOMEM, "scene exceeds the server's memory budget");
    r->nv = host->nv;
    r->n_steps = n_steps;
    r->host = std::move(host);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->dead) throw ApiError(IPC_E_DEVICE, "server stopped: " + srv->error);
    r->id = srv->next_id++;
    r->t_submit = t_arrival;
    *id = r->id;
    srv->queue.push_back(r.get());
    srv->reqs[r->id] = std::move(r);
    srv->cv_work.notify_all();
    return IPC_OK;
  });
}

int ipc_server_poll(ipc_server srv, int64_t id, ipc_request_info *info) {
  return guarded([&]() {
    if (!srv || !info) throw ApiError(IPC_E_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(srv->mu);
    fill_info(find_req(srv, id), info);
    return IPC_OK;
  });
}

int ipc_server_wait(ipc_server srv, int64_t id, double timeout_s, ipc_request_info *info) {
  return guarded([&]() {
    if (!srv || !(timeout_s >= 0)) throw ApiError(IPC_E_ARG, "bad arguments");
    std::unique_lock<std::mutex> lk(srv->mu);
    Request &r = find_req(srv, id);
    srv->cv_done.wait_for(lk, std::chrono::duration<double>(std::min(timeout_s, 1e7)), [&]() { return finished(r); });
    if (info) fill_info(r, info);
    return IPC_OK;
  });
}

int ipc_server_result(ipc_server srv, int64_t id, double *pos, double *vel) {
  return guarded([&]() {
    if (!srv || !pos) throw ApiError(IPC_E_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(srv->mu);
    Request &r = find_req(srv, id);
    if (!finished(r)) throw ApiError(IPC_E_ARG, "request has not finished");
    if (r.pos.empty() && r.nv > 0) throw ApiError(IPC_E_DEVICE, "no state kept: the server stopped");
    std::memcpy(pos, r.pos.data(), r.pos.size() * sizeof(double));
    if (vel) std::memcpy(vel, r.vel.data(), r.vel.size() * sizeof(double));
    return IPC_OK;
  });
}

int ipc_server_release(ipc_server srv, int64_t id) {
  return guarded([&]() {
    if (!srv) throw ApiError(IPC_E_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(srv->mu);
    Request &r = find_req(srv, id);
    if (!finished(r)) throw ApiError(IPC_E_ARG, "request has not finished");
    srv->reqs.erase(id);
    return IPC_OK;
  });
}

int ipc_server_set_slots(ipc_server srv, int32_t max_slots) {
  return guarded([&]() {
    if (!srv || max_slots < 1) throw ApiError(IPC_E_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->max_slots = max_slots;
    srv->auto_slots = false;
    srv->cv_work.notify_all();
    return IPC_OK;
  });
}

int ipc_server_stats(ipc_server srv, double *out) {
  return guarded([&]() {
    if (!srv || !out) throw ApiError(IPC_E_ARG, "bad arguments");
    std::lock_guard<std::mutex> lk(srv->mu);
    out[0] = (double)srv->finished;
    out[1] = (double)srv->failed;
    out[2] = (double)srv->conv_steps;
    out[3] = (double)srv->ticks;
    out[4] = (double)srv->n_running;
    out[5] = (double)srv->queue.size();
    out[6] = (double)srv->used;
    out[7] = srv->now();
    out[8] = (double)srv->max_slots;
    return IPC_OK;
  });
}

void ipc_server_destroy(ipc_server srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto &t : srv->workers)
    if (t.joinable()) t.join();
  try {
    for (auto &lane : srv->running)
      for (Request *r : lane)
        if (r->scene) {
          std::lock_guard<std::mutex> lk(r->scene->world->mu);
          r->scene->world->remove_scene(r->scene->slot);
          delete r->scene;
          r->scene = nullptr;
        }
  } catch (...) {
  }
  delete srv;
}

}  // extern "C"
