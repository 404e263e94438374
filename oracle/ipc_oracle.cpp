// ipc_oracle.cpp -- CPU oracle for the incremental-potential time step.
//
// TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded FP64
// restatement of what one implicit time step of the paper's IPC grasp
// simulator computes (Sec. III-A "IPC Simulator with Parallel Environment",
// constants of Sec. III-D "Grasp Validation"; the IPC ingredients -- barrier
// augmentation, CCD, projected Newton with a step-size filter -- are the ones
// the paper lists in Sec. II-C).  The paper does not print the IPC formulas;
// the ones used here are the standard IPC definitions, and every choice the
// paper leaves open is taken as documented next to the code.
//
// Independence from the GPU library: per-element first and second
// derivatives are obtained by forward-mode second-order automatic
// differentiation of the energy expressions (type Dual below), whereas the
// GPU library uses hand-derived closed forms.  Candidate and active sets are
// found by brute force over all primitive pairs.  PSD projection is plain
// cyclic Jacobi.  The linear solve is textbook block-Jacobi PCG (or a dense
// Cholesky factorisation for tiny systems).
//
// Every per-element routine is pinned by the CPU tests (closed forms, finite
// differences, brute force, special cases).  Parity unpinned: the
// whole-trajectory result, which has no closed form; it is checked only
// through the invariants (no intersection, J > 0, energy decrease) and the
// physics cases in the tests.
#include "ipc_oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <vector>

namespace {

constexpr double kInf = std::numeric_limits<double>::infinity();
thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

enum { OK = 0, E_ARG = -1, E_INVERTED = -2, E_INTERSECTING = -3, E_NOMEM = -4, E_FAILED = -5 };
enum { FAIL_NONE = 0, FAIL_MAXIT = 1, FAIL_NONFINITE = 2, FAIL_LS = 3, FAIL_DBC = 4 };

// ---------------------------------------------------------------------------
// small vector helpers (fixed evaluation order, no fused multiply-add)
// ---------------------------------------------------------------------------
struct V3 {
  double x, y, z;
};
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline V3 ld(const double *p) { return {p[0], p[1], p[2]}; }

// ---------------------------------------------------------------------------
// Forward-mode second-order dual number over N variables.
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double g[N];
  double h[N][N];
};
template <int N>
Dual<N> dconst(double c) {
  Dual<N> r;
  std::memset(&r, 0, sizeof(r));
  r.v = c;
  return r;
}
template <int N>
Dual<N> dvar(double c, int i) {
  Dual<N> r = dconst<N>(c);
  r.g[i] = 1.0;
  return r;
}
template <int N>
Dual<N> operator+(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] + b.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] + b.h[i][j];
  return r;
}
template <int N>
Dual<N> operator-(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] - b.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] - b.h[i][j];
  return r;
}
template <int N>
Dual<N> operator*(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      r.h[i][j] = a.v * b.h[i][j] + b.v * a.h[i][j] + a.g[i] * b.g[j] + b.g[i] * a.g[j];
  return r;
}
template <int N>
Dual<N> operator*(double s, const Dual<N> &a) {
  Dual<N> r;
  r.v = s * a.v;
  for (int i = 0; i < N; ++i) r.g[i] = s * a.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = s * a.h[i][j];
  return r;
}
// f(u) given f, f', f''
template <int N>
Dual<N> chain(const Dual<N> &u, double f, double f1, double f2) {
  Dual<N> r;
  r.v = f;
  for (int i = 0; i < N; ++i) r.g[i] = f1 * u.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = f1 * u.h[i][j] + f2 * u.g[i] * u.g[j];
  return r;
}
template <int N>
Dual<N> recip(const Dual<N> &u) {
  double iv = 1.0 / u.v;
  return chain(u, iv, -iv * iv, 2.0 * iv * iv * iv);
}
template <int N>
Dual<N> operator/(const Dual<N> &a, const Dual<N> &b) {
  return a * recip(b);
}
template <int N>
Dual<N> dsqrt(const Dual<N> &u) {
  double s = std::sqrt(u.v);
  return chain(u, s, 0.5 / s, -0.25 / (s * u.v));
}
template <int N>
Dual<N> dlog(const Dual<N> &u) {
  return chain(u, std::log(u.v), 1.0 / u.v, -1.0 / (u.v * u.v));
}

template <class T>
struct TV3 {
  T x, y, z;
};
template <class T>
TV3<T> tsub(const TV3<T> &a, const TV3<T> &b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class T>
T tdot(const TV3<T> &a, const TV3<T> &b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class T>
TV3<T> tcross(const TV3<T> &a, const TV3<T> &b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// ---------------------------------------------------------------------------
// Distance classification (fixed operation sequence; see the pair-type table
// in the design notes).  PT pairs are (p, t0, t1, t2); EE pairs are
// (a0, a1, b0, b1).
//   PT types: 0 interior, 1..3 point-edge on (t0,t1),(t1,t2),(t2,t0),
//             4..6 point-point with t0, t1, t2.
//   EE types: 0 interior, 1 a0-edge b, 2 a1-edge b, 3 b0-edge a, 4 b1-edge a,
//             5 a0-b0, 6 a0-b1, 7 a1-b0, 8 a1-b1.
// ---------------------------------------------------------------------------
enum { PS_PP_A = 0, PS_PP_B = 1, PS_PE = 2 };

int point_segment(V3 p, V3 a, V3 b, double *d2, double *s_out) {
  V3 e = sub(b, a);
  V3 w = sub(p, a);
  double ee = dot(e, e);
  if (!(ee > 0.0)) {
    *d2 = dot(w, w);
    *s_out = 0.0;
    return PS_PP_A;
  }
  double s = dot(w, e) / ee;
  if (s <= 0.0) {
    *d2 = dot(w, w);
    *s_out = 0.0;
    return PS_PP_A;
  }
  if (s >= 1.0) {
    V3 q = sub(p, b);
    *d2 = dot(q, q);
    *s_out = 1.0;
    return PS_PP_B;
  }
  V3 c = cross(w, e);
  *d2 = dot(c, c) / ee;
  *s_out = s;
  return PS_PE;
}

int pt_classify(const double *x, double *d2_out) {
  V3 p = ld(x), t0 = ld(x + 3), t1 = ld(x + 6), t2 = ld(x + 9);
  V3 e1 = sub(t1, t0), e2 = sub(t2, t0), w = sub(p, t0);
  double a = dot(e1, e1), b = dot(e1, e2), c = dot(e2, e2), d = dot(e1, w), e = dot(e2, w);
  double det = a * c - b * b;
  if (det > 0.0) {
    double b1 = (c * d - b * e) / det;
    double b2 = (a * e - b * d) / det;
    if (b1 >= 0.0 && b2 >= 0.0 && b1 + b2 <= 1.0) {
      V3 n = cross(e1, e2);
      double wn = dot(w, n);
      *d2_out = wn * wn / dot(n, n);
      return 0;
    }
  }
  V3 T[3] = {t0, t1, t2};
  double best = kInf;
  int type = -1;
  for (int j = 0; j < 3; ++j) {
    double d2, s;
    int k = point_segment(p, T[j], T[(j + 1) % 3], &d2, &s);
    if (d2 < best) {
      best = d2;
      type = (k == PS_PE) ? 1 + j : (k == PS_PP_A ? 4 + j : 4 + (j + 1) % 3);
    }
  }
  *d2_out = best;
  return type;
}

int ee_classify(const double *x, double *d2_out) {
  V3 a0 = ld(x), a1 = ld(x + 3), b0 = ld(x + 6), b1 = ld(x + 9);
  V3 ea = sub(a1, a0), eb = sub(b1, b0), w = sub(a0, b0);
  V3 n = cross(ea, eb);
  double nn = dot(n, n);
  double A = dot(ea, ea), B = dot(ea, eb), C = dot(eb, eb), D = dot(ea, w), E = dot(eb, w);
  if (nn > 1e-12 * A * C) {
    double det = A * C - B * B;
    double s = (B * E - C * D) / det;
    double t = (A * E - B * D) / det;
    if (s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0) {
      double wn = dot(w, n);
      *d2_out = wn * wn / nn;
      return 0;
    }
  }
  // point-segment fall-backs, first strict minimum wins
  static const int pp_map[4][2] = {{5, 6}, {7, 8}, {5, 7}, {6, 8}};
  V3 P[4] = {a0, a1, b0, b1};
  V3 SA[4] = {b0, b0, a0, a0}, SB[4] = {b1, b1, a1, a1};
  double best = kInf;
  int type = -1;
  for (int k = 0; k < 4; ++k) {
    double d2, s;
    int r = point_segment(P[k], SA[k], SB[k], &d2, &s);
    if (d2 < best) {
      best = d2;
      type = (r == PS_PE) ? 1 + k : pp_map[k][r];
    }
  }
  *d2_out = best;
  return type;
}

// Vertex slots (into the 4 pair vertices) that a given type involves, and for
// the point-edge / point-point cases which role each plays.
struct TypeSlots {
  int n;        // 2 (PP), 3 (PE), 4 (interior)
  int s[4];     // slots: PP -> (point, other); PE -> (point, edge a, edge b); interior -> 0..3
};
TypeSlots type_slots(int kind, int type) {
  TypeSlots t{};
  if (type == 0) {
    t.n = 4;
    for (int i = 0; i < 4; ++i) t.s[i] = i;
    return t;
  }
  if (kind == 0) {  // PT
    if (type <= 3) {
      int j = type - 1;
      t.n = 3;
      t.s[0] = 0;
      t.s[1] = 1 + j;
      t.s[2] = 1 + (j + 1) % 3;
    } else {
      t.n = 2;
      t.s[0] = 0;
      t.s[1] = 1 + (type - 4);
    }
    return t;
  }
  // EE
  static const int pe[4][3] = {{0, 2, 3}, {1, 2, 3}, {2, 0, 1}, {3, 0, 1}};
  static const int pp[4][2] = {{0, 2}, {0, 3}, {1, 2}, {1, 3}};
  if (type <= 4) {
    t.n = 3;
    for (int i = 0; i < 3; ++i) t.s[i] = pe[type - 1][i];
  } else {
    t.n = 2;
    for (int i = 0; i < 2; ++i) t.s[i] = pp[type - 5][i];
  }
  return t;
}

// Squared distance of a given type as a differentiable expression.
template <class T>
T d2_expr(int kind, int type, const TV3<T> P[4]) {
  TypeSlots ts = type_slots(kind, type);
  if (ts.n == 2) {
    TV3<T> w = tsub(P[ts.s[0]], P[ts.s[1]]);
    return tdot(w, w);
  }
  if (ts.n == 3) {
    TV3<T> e = tsub(P[ts.s[2]], P[ts.s[1]]);
    TV3<T> w = tsub(P[ts.s[0]], P[ts.s[1]]);
    TV3<T> c = tcross(w, e);
    return tdot(c, c) / tdot(e, e);
  }
  if (kind == 0) {
    TV3<T> e1 = tsub(P[2], P[1]), e2 = tsub(P[3], P[1]), w = tsub(P[0], P[1]);
    TV3<T> n = tcross(e1, e2);
    T wn = tdot(w, n);
    return wn * wn / tdot(n, n);
  }
  TV3<T> ea = tsub(P[1], P[0]), eb = tsub(P[3], P[2]), w = tsub(P[0], P[2]);
  TV3<T> n = tcross(ea, eb);
  T wn = tdot(w, n);
  return wn * wn / tdot(n, n);
}

// ---------------------------------------------------------------------------
// Barrier b(d) = -(d - dhat)^2 ln(d / dhat) for 0 < d < dhat, 0 otherwise.
// ---------------------------------------------------------------------------
void barrier_scalar(double d, double dhat, double out[3]) {
  if (d >= dhat) {
    out[0] = out[1] = out[2] = 0.0;
    return;
  }
  double r = d - dhat, L = std::log(d / dhat);
  out[0] = -r * r * L;
  out[1] = -2.0 * r * L - r * r / d;
  out[2] = -2.0 * L - 4.0 * r / d + r * r / (d * d);
}

// Edge-edge mollifier as a function of c = |ea x eb|^2.
template <int N>
Dual<N> mollifier(const Dual<N> &c, double eps_x) {
  if (c.v >= eps_x) return dconst<N>(1.0);
  Dual<N> q = (1.0 / eps_x) * c;
  return q * (dconst<N>(2.0) - q);
}

// ---------------------------------------------------------------------------
// PSD projection: cyclic Jacobi eigen-decomposition, negative eigenvalues
// clamped to zero.  Stops when the off-diagonal Frobenius norm is at most
// 1e-15 of the matrix norm, or after 50 sweeps.
// ---------------------------------------------------------------------------
void psd_project(int n, double *A) {
  std::vector<double> M(A, A + n * n), V(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  double fro = 0.0;
  for (int i = 0; i < n * n; ++i) fro += M[i] * M[i];
  fro = std::sqrt(fro);
  if (fro == 0.0) return;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if (i != j) off += M[i * n + j] * M[i * n + j];
    if (std::sqrt(off) <= 1e-15 * fro) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = M[p * n + q];
        if (apq == 0.0) continue;
        double theta = (M[q * n + q] - M[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          double mkp = M[k * n + p], mkq = M[k * n + q];
          M[k * n + p] = c * mkp - s * mkq;
          M[k * n + q] = s * mkp + c * mkq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          double mpk = M[p * n + k], mqk = M[q * n + k];
          M[p * n + k] = c * mpk - s * mqk;
          M[q * n + k] = s * mpk + c * mqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) {
        double lam = M[k * n + k];
        if (lam > 0.0) acc += V[i * n + k] * lam * V[j * n + k];
      }
      A[i * n + j] = acc;
    }
}

// ---------------------------------------------------------------------------
// Pair barrier energy kappa * e * b(d) with AD derivatives over 12 variables.
// ---------------------------------------------------------------------------
double pair_barrier(int kind, int type, const double *x, double dhat, double kappa, double eps_x,
                    bool want_derivs, bool project, double *g, double *H) {
  if (!want_derivs) {
    TV3<double> P[4];
    for (int i = 0; i < 4; ++i) P[i] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};
    double z = d2_expr<double>(kind, type, P);
    double d = std::sqrt(z);
    double b[3];
    barrier_scalar(d, dhat, b);
    double e = 1.0;
    if (kind == 1) {
      TV3<double> c3 = tcross(tsub(P[1], P[0]), tsub(P[3], P[2]));
      double c = tdot(c3, c3);
      if (c < eps_x) {
        double q = c / eps_x;
        e = q * (2.0 - q);
      }
    }
    return kappa * e * b[0];
  }
  typedef Dual<12> D;
  TV3<D> P[4];
  for (int i = 0; i < 4; ++i)
    P[i] = {dvar<12>(x[3 * i], 3 * i), dvar<12>(x[3 * i + 1], 3 * i + 1), dvar<12>(x[3 * i + 2], 3 * i + 2)};
  D z = d2_expr<D>(kind, type, P);
  D d = dsqrt(z);
  double b[3];
  barrier_scalar(d.v, dhat, b);
  D bd = chain(d, b[0], b[1], b[2]);
  D E = bd;
  if (kind == 1) {
    TV3<D> c3 = tcross(tsub(P[1], P[0]), tsub(P[3], P[2]));
    D c = tdot(c3, c3);
    E = mollifier(c, eps_x) * bd;
  }
  E = kappa * E;
  for (int i = 0; i < 12; ++i) g[i] = E.g[i];
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j) H[i * 12 + j] = E.h[i][j];
  if (project) psd_project(12, H);
  return E.v;
}

// ---------------------------------------------------------------------------
// Neo-Hookean: Psi = mu/2 (tr F^T F - 3) - mu ln J + lambda/2 (ln J)^2,
// J = det F; Psi = +inf when J <= 0.  Derivatives by AD over the 9 entries
// of F (row-major), PSD projection at the 9x9 level, then mapped to the 12
// vertex coordinates through F = Ds Dm^-1.
// ---------------------------------------------------------------------------
template <class T>
T det3(const T F[9]) {
  return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]);
}

bool inv3(const double M[9], double R[9]) {
  double det = det3<double>(M);
  if (det == 0.0) return false;
  double id = 1.0 / det;
  R[0] = (M[4] * M[8] - M[5] * M[7]) * id;
  R[1] = (M[2] * M[7] - M[1] * M[8]) * id;
  R[2] = (M[1] * M[5] - M[2] * M[4]) * id;
  R[3] = (M[5] * M[6] - M[3] * M[8]) * id;
  R[4] = (M[0] * M[8] - M[2] * M[6]) * id;
  R[5] = (M[2] * M[3] - M[0] * M[5]) * id;
  R[6] = (M[3] * M[7] - M[4] * M[6]) * id;
  R[7] = (M[1] * M[6] - M[0] * M[7]) * id;
  R[8] = (M[0] * M[4] - M[1] * M[3]) * id;
  return true;
}

void lame(double E, double nu, double *mu, double *la) {
  *mu = E / (2.0 * (1.0 + nu));
  *la = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
}

// Ds (columns x1-x0, x2-x0, x3-x0), row-major.
void build_Ds(const double *x, double Ds[9]) {
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) Ds[i * 3 + a] = x[3 * (a + 1) + i] - x[i];
}

void matmul3(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
}

// energy density with derivatives wrt F (AD).  Returns false if J <= 0.
bool nh_density(const double F[9], double mu, double la, bool derivs, bool project, double *psi,
                double gF[9], double HF[81]) {
  double J = det3<double>(F);
  if (!(J > 0.0)) return false;
  if (!derivs) {
    double tr = 0.0;
    for (int i = 0; i < 9; ++i) tr += F[i] * F[i];
    double lJ = std::log(J);
    *psi = 0.5 * mu * (tr - 3.0) - mu * lJ + 0.5 * la * lJ * lJ;
    return true;
  }
  typedef Dual<9> D;
  D Fd[9];
  for (int i = 0; i < 9; ++i) Fd[i] = dvar<9>(F[i], i);
  D tr = dconst<9>(0.0);
  for (int i = 0; i < 9; ++i) tr = tr + Fd[i] * Fd[i];
  D lJ = dlog(det3<D>(Fd));
  D P = (0.5 * mu) * (tr - dconst<9>(3.0)) - mu * lJ + (0.5 * la) * (lJ * lJ);
  *psi = P.v;
  for (int i = 0; i < 9; ++i) gF[i] = P.g[i];
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) HF[i * 9 + j] = P.h[i][j];
  if (project) psd_project(9, HF);
  return true;
}

// dF/dx as a 9x12 matrix for F = Ds Dm^-1.
void dFdx(const double Dinv[9], double B[9 * 12]) {
  std::memset(B, 0, sizeof(double) * 108);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      int row = i * 3 + j;
      double s0 = 0.0;
      for (int a = 0; a < 3; ++a) {
        B[row * 12 + 3 * (a + 1) + i] = Dinv[a * 3 + j];
        s0 += Dinv[a * 3 + j];
      }
      B[row * 12 + i] = -s0;
    }
}

// Elastic energy of one tet (V * Psi) with gradient / projected Hessian in x.
bool tet_elastic(const double *x, const double Dinv[9], double vol, double mu, double la, bool derivs,
                 bool project, double *energy, double g[12], double H[144]) {
  double Ds[9], F[9];
  build_Ds(x, Ds);
  matmul3(Ds, Dinv, F);
  double psi, gF[9], HF[81];
  if (!nh_density(F, mu, la, derivs, project, &psi, gF, HF)) return false;
  *energy = vol * psi;
  if (!derivs) return true;
  double B[108];
  dFdx(Dinv, B);
  for (int c = 0; c < 12; ++c) {
    double s = 0.0;
    for (int r = 0; r < 9; ++r) s += B[r * 12 + c] * gF[r];
    g[c] = vol * s;
  }
  double HB[9 * 12];
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 12; ++c) {
      double s = 0.0;
      for (int k = 0; k < 9; ++k) s += HF[r * 9 + k] * B[k * 12 + c];
      HB[r * 12 + c] = s;
    }
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j) {
      double s = 0.0;
      for (int r = 0; r < 9; ++r) s += B[r * 12 + i] * HB[r * 12 + j];
      H[i * 12 + j] = vol * s;
    }
  return true;
}

// ---------------------------------------------------------------------------
// Lagged friction (one lag per step, taken at x^n):
//   D_k(x) = mu * lambda_k * f0(|u_k|),  u_k = (I - n n^T) sum_i w_i (x_i - x^n_i)
//   f0(y) = -y^3/(3 eps^2) + y^2/eps + eps/3 for y < eps, y otherwise; eps = eps_v dt.
// ---------------------------------------------------------------------------
void friction_f0(double y, double eps, double out[3]) {
  if (y < eps) {
    out[0] = -y * y * y / (3.0 * eps * eps) + y * y / eps + eps / 3.0;
    out[1] = -y * y / (eps * eps) + 2.0 * y / eps;
    out[2] = -2.0 * y / (eps * eps) + 2.0 / eps;
  } else {
    out[0] = y;
    out[1] = 1.0;
    out[2] = 0.0;
  }
}

struct FricPair {
  int v[4];
  double w[4];
  double n[3];
  double lambda;
};

// One lagged friction element: energy mu*lambda*f0(|u|) with
// u = (I - n n^T) sum_i w_i (x_i - x^n_i), its gradient and its Hessian.
// With y = |u|, the gradient is mu*lambda*w_i*(f1(y)/y)*u for vertex i and the
// Hessian block (i, j) is mu*lambda*w_i*w_j*[a (I - n n^T) + c u u^T]:
//   y < eps:  a = f1/y = 2/eps - y/eps^2,  c = (d/dy)(f1/y)/y = -1/(eps^2 y)  (c = 0 at y = 0)
//   y >= eps: a = 1/y,                     c = -1/y^3
// (the exact second derivatives of f0(|u|); a + c y^2 >= 0 in both branches,
// so the matrix is PSD without projection).
double friction_elem(const double x12[12], const double xn12[12], const double w[4], const double n[3],
                     double lambda, double mu, double eps, double *g, double *H) {
  double u[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 3; ++k) u[k] += w[i] * (x12[3 * i + k] - xn12[3 * i + k]);
  double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
  for (int k = 0; k < 3; ++k) u[k] -= un * n[k];
  double y = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double f0[3];
  friction_f0(y, eps, f0);
  double E = mu * lambda * f0[0];
  if (!g && !H) return E;
  double f1y, a, c;
  if (y < eps) {
    f1y = 2.0 / eps - y / (eps * eps);
    a = f1y;
    c = (y > 0.0) ? -1.0 / (eps * eps * y) : 0.0;
  } else {
    f1y = 1.0 / y;
    a = 1.0 / y;
    c = -1.0 / (y * y * y);
  }
  double sc = mu * lambda;
  if (g)
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 3; ++k) g[3 * i + k] = sc * w[i] * f1y * u[k];
  if (H) {
    double K[9];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) K[r * 3 + q] = a * ((r == q ? 1.0 : 0.0) - n[r] * n[q]) + c * u[r] * u[q];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) H[(3 * i + r) * 12 + 3 * j + q] = sc * w[i] * w[j] * K[r * 3 + q];
  }
  return E;
}

// Closest-point weights of a classified pair: sum_i w_i x_i is the vector
// from the closest point of the second primitive to that of the first.
void closest_weights(int kind, int type, const double *x, double w[4]) {
  for (int i = 0; i < 4; ++i) w[i] = 0.0;
  V3 P[4] = {ld(x), ld(x + 3), ld(x + 6), ld(x + 9)};
  if (type == 0) {
    if (kind == 0) {
      V3 e1 = sub(P[2], P[1]), e2 = sub(P[3], P[1]), q = sub(P[0], P[1]);
      double a = dot(e1, e1), b = dot(e1, e2), c = dot(e2, e2), d = dot(e1, q), e = dot(e2, q);
      double det = a * c - b * b;
      double b1 = (c * d - b * e) / det, b2 = (a * e - b * d) / det;
      w[0] = 1.0;
      w[1] = -(1.0 - b1 - b2);
      w[2] = -b1;
      w[3] = -b2;
    } else {
      V3 ea = sub(P[1], P[0]), eb = sub(P[3], P[2]), q = sub(P[0], P[2]);
      double A = dot(ea, ea), B = dot(ea, eb), C = dot(eb, eb), D = dot(ea, q), E = dot(eb, q);
      double det = A * C - B * B;
      double s = (B * E - C * D) / det, t = (A * E - B * D) / det;
      w[0] = 1.0 - s;
      w[1] = s;
      w[2] = -(1.0 - t);
      w[3] = -t;
    }
    return;
  }
  TypeSlots ts = type_slots(kind, type);
  // orientation: first primitive minus second primitive
  double sign = 1.0;
  if (kind == 1 && ts.s[0] >= 2) sign = -1.0;  // the point belongs to edge b
  if (ts.n == 2) {
    w[ts.s[0]] = sign;
    w[ts.s[1]] = -sign;
    return;
  }
  V3 p = P[ts.s[0]], a = P[ts.s[1]], b = P[ts.s[2]];
  V3 e = sub(b, a);
  double s = dot(sub(p, a), e) / dot(e, e);
  w[ts.s[0]] = sign;
  w[ts.s[1]] = -sign * (1.0 - s);
  w[ts.s[2]] = -sign * s;
}

// ---------------------------------------------------------------------------
// Additive CCD (conservative time of impact along x + t p, t in [0,1]).
// ---------------------------------------------------------------------------
double pair_dist(int kind, const double *x) {
  double d2;
  if (kind == 0)
    pt_classify(x, &d2);
  else
    ee_classify(x, &d2);
  return std::sqrt(d2);
}

double accd(int kind, const double *x, const double *p, double s) {
  double pm[12], mean[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 3; ++k) mean[k] += p[3 * i + k];
  for (int k = 0; k < 3; ++k) mean[k] *= 0.25;
  double nrm[4];
  for (int i = 0; i < 4; ++i) {
    double s2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      pm[3 * i + k] = p[3 * i + k] - mean[k];
      s2 += pm[3 * i + k] * pm[3 * i + k];
    }
    nrm[i] = std::sqrt(s2);
  }
  double l = (kind == 0) ? nrm[0] + std::max(nrm[1], std::max(nrm[2], nrm[3]))
                         : std::max(nrm[0], nrm[1]) + std::max(nrm[2], nrm[3]);
  if (l == 0.0) return 1.0;
  double d0 = pair_dist(kind, x);
  double t = 0.0;
  double xt[12];
  for (long it = 0; it < 1000000; ++it) {
    for (int i = 0; i < 12; ++i) xt[i] = x[i] + t * pm[i];
    double d = pair_dist(kind, xt);
    if (t > 0.0 && d <= s * d0) return t;
    double tau = (1.0 - s) * d / l;
    if (t + tau >= 1.0) return 1.0;
    t += tau;
  }
  return t;
}

// ---------------------------------------------------------------------------
// Scene
// ---------------------------------------------------------------------------
struct Pair {
  int kind;  // 0 PT, 1 EE
  int v[4];
  int edge_a, edge_b;  // EE: surface edge ids (for the mollifier threshold)
};

struct Scene {
  int nv = 0, nt = 0;
  std::vector<double> X, x, v;
  std::vector<int> tet;
  std::vector<double> vol, mu_l, la_l, Dinv, mass;
  std::vector<int> kin;
  int ngroups = 0, nmotion = 0;
  std::vector<double> motion, gravity;
  double dt, dhat, kappa, mu, eps_v, tol, pcg_tol;
  int maxit, solver;
  // solver variants (off by default)
  int friction_iters = 1;     // lagged friction updates per step
  bool inv_filter = false;    // per-tet det F root bounds the line search
  bool adaptive_kappa = false;
  double kappa0 = 0.0;        // kappa as given (adaptive kappa stays in [kappa0, 100 kappa0])
  double dmin_prev = 0.0;     // least active-pair distance at the previous Newton iterate
  std::vector<std::array<int, 3>> stri;
  std::vector<std::array<int, 2>> sedge;
  std::vector<int> svert;
  std::vector<double> edge_len2;  // rest squared length per surface edge
  int step = 0;
  bool failed = false;
  int fail_reason = 0;
  // per-step context
  bool ctx = false;
  std::vector<double> xn, xhat, xbar;
  std::vector<FricPair> fric;
  // augmented-Lagrangian Dirichlet mode (kinematic vertices are unknowns)
  double mbar = 0.0;  // mean free-vertex mass
  bool al = false;
  double kA = 0.0, w_al = 0.0, viol_prev = 0.0;
  std::vector<double> Lam;
  // Newton record of the last step: per accepted iterate (Phi before, Phi
  // after, step size, halvings)
  std::vector<double> iter_log;
  // test-only planted fault: added to every line-search trial energy
  double debug_ls_offset = 0.0;
  // grasp-validation controls (Sec. III-D): a held kinematic group keeps the
  // target of motion row hold[g] from then on (-1: follows its schedule); a
  // gravity override replaces the schedule's gravity rows
  std::vector<int> hold;
  bool g_over = false;
  double g_ovr[3] = {0, 0, 0};
};

bool is_kin(const Scene &s, int i) { return s.kin[i] >= 0; }
// unknowns of the Newton solve: free vertices, plus kinematic ones in AL mode
bool is_dof(const Scene &s, int i) { return !is_kin(s, i) || s.al; }

void gather12(const std::vector<double> &x, const int v[4], double out[12]) {
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 3; ++k) out[3 * i + k] = x[3 * v[i] + k];
}

// AABB overlap of two vertex sets (optionally swept by p), widened by dhat.
void vbox(const Scene &s, const std::vector<double> &x, const double *p, const int *vs, int n, double lo[3],
          double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = kInf;
    hi[k] = -kInf;
  }
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      double a = x[3 * vs[i] + k];
      lo[k] = std::min(lo[k], a);
      hi[k] = std::max(hi[k], a);
      if (p) {
        double b = a + p[3 * vs[i] + k];
        lo[k] = std::min(lo[k], b);
        hi[k] = std::max(hi[k], b);
      }
    }
  for (int k = 0; k < 3; ++k) {
    lo[k] = lo[k] - s.dhat;
    hi[k] = hi[k] + s.dhat;
  }
}

bool overlap(const double alo[3], const double ahi[3], const double blo[3], const double bhi[3]) {
  for (int k = 0; k < 3; ++k)
    if (!(alo[k] <= bhi[k] && blo[k] <= ahi[k])) return false;
  return true;
}

// Candidate set by brute force over all PT and EE pairs.
std::vector<Pair> candidates(const Scene &s, const std::vector<double> &x, const double *p) {
  std::vector<Pair> out;
  int nsv = (int)s.svert.size(), nst = (int)s.stri.size(), nse = (int)s.sedge.size();
  std::vector<double> vlo(nsv * 3), vhi(nsv * 3), tlo(nst * 3), thi(nst * 3), elo(nse * 3), ehi(nse * 3);
  for (int i = 0; i < nsv; ++i) vbox(s, x, p, &s.svert[i], 1, &vlo[3 * i], &vhi[3 * i]);
  for (int i = 0; i < nst; ++i) vbox(s, x, p, s.stri[i].data(), 3, &tlo[3 * i], &thi[3 * i]);
  for (int i = 0; i < nse; ++i) vbox(s, x, p, s.sedge[i].data(), 2, &elo[3 * i], &ehi[3 * i]);
  for (int i = 0; i < nsv; ++i) {
    int vi = s.svert[i];
    for (int t = 0; t < nst; ++t) {
      const auto &T = s.stri[t];
      if (T[0] == vi || T[1] == vi || T[2] == vi) continue;
      if (is_kin(s, vi) && is_kin(s, T[0]) && is_kin(s, T[1]) && is_kin(s, T[2])) continue;
      if (!overlap(&vlo[3 * i], &vhi[3 * i], &tlo[3 * t], &thi[3 * t])) continue;
      out.push_back({0, {vi, T[0], T[1], T[2]}, -1, -1});
    }
  }
  for (int a = 0; a < nse; ++a)
    for (int b = a + 1; b < nse; ++b) {
      const auto &A = s.sedge[a], &B = s.sedge[b];
      if (A[0] == B[0] || A[0] == B[1] || A[1] == B[0] || A[1] == B[1]) continue;
      if (is_kin(s, A[0]) && is_kin(s, A[1]) && is_kin(s, B[0]) && is_kin(s, B[1])) continue;
      if (!overlap(&elo[3 * a], &ehi[3 * a], &elo[3 * b], &ehi[3 * b])) continue;
      out.push_back({1, {A[0], A[1], B[0], B[1]}, a, b});
    }
  return out;
}

struct ActivePair {
  Pair p;
  int type;
  double d2;
};

std::vector<ActivePair> active_set(const Scene &s, const std::vector<double> &x, const std::vector<Pair> &cand) {
  std::vector<ActivePair> out;
  double dh2 = s.dhat * s.dhat;
  for (const Pair &c : cand) {
    double xx[12], d2;
    gather12(x, c.v, xx);
    int type = c.kind == 0 ? pt_classify(xx, &d2) : ee_classify(xx, &d2);
    if (d2 < dh2) out.push_back({c, type, d2});
  }
  return out;
}

double eps_cross(const Scene &s, const Pair &p) {
  if (p.kind != 1) return 0.0;
  return 1e-3 * s.edge_len2[p.edge_a] * s.edge_len2[p.edge_b];
}

// ---------------------------------------------------------------------------
// Scene construction
// ---------------------------------------------------------------------------
// Orientation of d relative to the plane through a, b, c (sign of the triple product).
double orient3d(V3 a, V3 b, V3 c, V3 d) { return dot(sub(b, a), cross(sub(c, a), sub(d, a))); }

// True if segment (a, b) crosses triangle (t0, t1, t2) with a margin: the
// endpoints lie strictly on opposite sides of the triangle's plane and the
// segment's line passes strictly inside the triangle, each test beyond
// 1e-9 L^3 (L = longest edge involved).  Touching and coplanar configurations
// (orientations at rounding level) do not count as crossings.
bool segment_crosses_triangle(V3 a, V3 b, V3 t0, V3 t1, V3 t2) {
  V3 P[5] = {a, b, t0, t1, t2};
  double L2 = 0.0;
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) {
      V3 d = sub(P[i], P[j]);
      L2 = std::max(L2, dot(d, d));
    }
  double eps = 1e-9 * L2 * std::sqrt(L2);
  double da = orient3d(t0, t1, t2, a), db = orient3d(t0, t1, t2, b);
  if (!((da > eps && db < -eps) || (da < -eps && db > eps))) return false;
  double s0 = orient3d(a, b, t0, t1), s1 = orient3d(a, b, t1, t2), s2 = orient3d(a, b, t2, t0);
  return (s0 > eps && s1 > eps && s2 > eps) || (s0 < -eps && s1 < -eps && s2 < -eps);
}

bool finite(const double *p, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

int build_scene(const ipco_desc *d, Scene **out) {
  if (!d) return fail(E_ARG, "null descriptor");
  if (d->n_verts <= 0 || !d->rest_pos || !d->kin_group) return fail(E_ARG, "no vertices");
  if (d->n_tets < 0 || (d->n_tets > 0 && (!d->tets || !d->E || !d->nu || !d->rho)))
    return fail(E_ARG, "tet arrays missing");
  if (d->n_tris < 0 || (d->n_tris > 0 && !d->tris)) return fail(E_ARG, "triangle array missing");
  if (d->n_motion_steps < 1 || d->n_groups < 0 || !d->gravity || (d->n_groups > 0 && !d->motion))
    return fail(E_ARG, "motion schedule missing");
  if (!(d->dt > 0) || !(d->dhat > 0) || !(d->kappa > 0) || !(d->mu >= 0) || !(d->eps_v > 0) ||
      !(d->newton_tol > 0) || d->newton_max_iter < 1 || !(d->pcg_rel_tol > 0))
    return fail(E_ARG, "bad solver parameter");
  Scene *s = new Scene();
  s->nv = d->n_verts;
  s->nt = d->n_tets;
  long nv3 = 3L * s->nv;
  if (!finite(d->rest_pos, nv3) || (d->init_pos && !finite(d->init_pos, nv3)) ||
      (d->init_vel && !finite(d->init_vel, nv3))) {
    delete s;
    return fail(E_ARG, "non-finite vertex data");
  }
  s->X.assign(d->rest_pos, d->rest_pos + nv3);
  s->x = d->init_pos ? std::vector<double>(d->init_pos, d->init_pos + nv3) : s->X;
  s->v = d->init_vel ? std::vector<double>(d->init_vel, d->init_vel + nv3) : std::vector<double>(nv3, 0.0);
  s->kin.assign(d->kin_group, d->kin_group + s->nv);
  s->ngroups = d->n_groups;
  s->nmotion = d->n_motion_steps;
  for (int i = 0; i < s->nv; ++i)
    if (s->kin[i] < -1 || s->kin[i] >= s->ngroups) {
      delete s;
      return fail(E_ARG, "kin_group out of range");
    }
  if (s->ngroups > 0) s->motion.assign(d->motion, d->motion + 12L * s->ngroups * s->nmotion);
  s->gravity.assign(d->gravity, d->gravity + 3L * s->nmotion);
  if (!finite(s->motion.data(), (long)s->motion.size()) || !finite(s->gravity.data(), (long)s->gravity.size())) {
    delete s;
    return fail(E_ARG, "non-finite motion");
  }
  if (d->newton_rel_tol < 0 || d->friction_iters < 0 || d->inversion_filter < 0 || d->adaptive_kappa < 0) {
    delete s;
    return fail(E_ARG, "bad solver variant");
  }
  s->dt = d->dt;
  s->dhat = d->dhat;
  s->kappa = d->kappa;
  s->kappa0 = d->kappa;
  s->dmin_prev = kInf;
  s->friction_iters = std::max(1, (int)d->friction_iters);
  s->inv_filter = d->inversion_filter != 0;
  s->adaptive_kappa = d->adaptive_kappa != 0;
  s->mu = d->mu;
  s->eps_v = d->eps_v;
  s->tol = d->newton_tol;
  s->maxit = d->newton_max_iter;
  s->pcg_tol = d->pcg_rel_tol;
  s->solver = d->linear_solver;
  s->tet.assign(d->tets, d->tets + 4L * s->nt);
  for (int i = 0; i < 4 * s->nt; ++i)
    if (s->tet[i] < 0 || s->tet[i] >= s->nv) {
      delete s;
      return fail(E_ARG, "tet index out of range");
    }
  s->vol.resize(s->nt);
  s->mu_l.resize(s->nt);
  s->la_l.resize(s->nt);
  s->Dinv.resize(9L * s->nt);
  s->mass.assign(s->nv, 0.0);
  for (int e = 0; e < s->nt; ++e) {
    if (!(d->E[e] > 0) || !(d->nu[e] > -1.0 && d->nu[e] < 0.5) || !(d->rho[e] > 0)) {
      delete s;
      return fail(E_ARG, "bad material");
    }
    double Xe[12], Dm[9];
    gather12(s->X, &s->tet[4 * e], Xe);
    build_Ds(Xe, Dm);
    double det = det3<double>(Dm);
    if (!(det > 0.0)) {
      delete s;
      return fail(E_INVERTED, "tet with non-positive rest volume");
    }
    inv3(Dm, &s->Dinv[9 * e]);
    s->vol[e] = det / 6.0;
    lame(d->E[e], d->nu[e], &s->mu_l[e], &s->la_l[e]);
    double m = d->rho[e] * s->vol[e] / 4.0;
    for (int k = 0; k < 4; ++k) s->mass[s->tet[4 * e + k]] += m;
  }
  int nfree = 0;
  for (int i = 0; i < s->nv; ++i) {
    if (!is_kin(*s, i) && !(s->mass[i] > 0.0)) {
      delete s;
      return fail(E_ARG, "free vertex without mass");
    }
    if (!is_kin(*s, i)) {
      s->mbar += s->mass[i];
      ++nfree;
    }
  }
  s->mbar = nfree > 0 ? s->mbar / nfree : 1.0;
  if (d->newton_rel_tol > 0) {
    // the paper's relative Newton tolerance (Sec. III-D), read as a fraction
    // of the free vertices' bounding-box diagonal per time step
    double lo[3] = {kInf, kInf, kInf}, hi[3] = {-kInf, -kInf, -kInf};
    for (int i = 0; i < s->nv; ++i)
      if (!is_kin(*s, i))
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], s->x[3 * i + k]);
          hi[k] = std::max(hi[k], s->x[3 * i + k]);
        }
    double L2 = 0.0;
    for (int k = 0; k < 3; ++k) L2 += nfree > 0 ? (hi[k] - lo[k]) * (hi[k] - lo[k]) : 0.0;
    s->tol = d->newton_rel_tol * std::sqrt(L2);
  }
  // Surface: tet faces used by exactly one tet, plus the kinematic triangles.
  // Canonical form: triangle vertices ascending, list sorted; edges (min,max).
  std::map<std::array<int, 3>, int> faces;
  for (int e = 0; e < s->nt; ++e) {
    const int *t = &s->tet[4 * e];
    int F[4][3] = {{t[0], t[2], t[1]}, {t[0], t[1], t[3]}, {t[0], t[3], t[2]}, {t[1], t[2], t[3]}};
    for (auto &f : F) {
      std::array<int, 3> k = {f[0], f[1], f[2]};
      std::sort(k.begin(), k.end());
      faces[k] += 1;
    }
  }
  std::vector<std::array<int, 3>> tris;
  for (auto &kv : faces)
    if (kv.second == 1) tris.push_back(kv.first);
  for (int i = 0; i < d->n_tris; ++i) {
    std::array<int, 3> k = {d->tris[3 * i], d->tris[3 * i + 1], d->tris[3 * i + 2]};
    for (int c = 0; c < 3; ++c)
      if (k[c] < 0 || k[c] >= s->nv || !is_kin(*s, k[c])) {
        delete s;
        return fail(E_ARG, "kinematic triangle with bad or free vertex");
      }
    std::sort(k.begin(), k.end());
    tris.push_back(k);
  }
  std::sort(tris.begin(), tris.end());
  tris.erase(std::unique(tris.begin(), tris.end()), tris.end());
  s->stri = tris;
  std::vector<std::array<int, 2>> edges;
  std::vector<int> verts;
  for (auto &t : tris) {
    edges.push_back({t[0], t[1]});
    edges.push_back({t[1], t[2]});
    edges.push_back({t[0], t[2]});
    verts.insert(verts.end(), t.begin(), t.end());
  }
  std::sort(edges.begin(), edges.end());
  edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
  std::sort(verts.begin(), verts.end());
  verts.erase(std::unique(verts.begin(), verts.end()), verts.end());
  s->sedge = edges;
  s->svert = verts;
  s->edge_len2.resize(edges.size());
  for (size_t i = 0; i < edges.size(); ++i) {
    V3 a = ld(&s->X[3 * edges[i][0]]), b = ld(&s->X[3 * edges[i][1]]);
    V3 e = sub(b, a);
    s->edge_len2[i] = dot(e, e);
  }
  // Initial configuration must be inversion- and intersection-free.
  for (int e = 0; e < s->nt; ++e) {
    double xe[12], Ds[9], F[9];
    gather12(s->x, &s->tet[4 * e], xe);
    build_Ds(xe, Ds);
    matmul3(Ds, &s->Dinv[9 * e], F);
    if (!(det3<double>(F) > 0.0)) {
      delete s;
      return fail(E_INVERTED, "inverted tet in the initial configuration");
    }
  }
  for (const Pair &c : candidates(*s, s->x, nullptr)) {
    double xx[12], d2;
    gather12(s->x, c.v, xx);
    if (c.kind == 0)
      pt_classify(xx, &d2);
    else
      ee_classify(xx, &d2);
    if (!(d2 > 0.0)) {
      delete s;
      return fail(E_INTERSECTING, "intersecting initial configuration");
    }
  }
  // Intersection also shows as a surface edge piercing a surface triangle
  // (the pair distances can all stay positive when bodies pass through).
  for (const auto &e : s->sedge)
    for (const auto &t : s->stri) {
      if (e[0] == t[0] || e[0] == t[1] || e[0] == t[2] || e[1] == t[0] || e[1] == t[1] || e[1] == t[2]) continue;
      if (is_kin(*s, e[0]) && is_kin(*s, e[1]) && is_kin(*s, t[0]) && is_kin(*s, t[1]) && is_kin(*s, t[2])) continue;
      if (segment_crosses_triangle(ld(&s->x[3 * e[0]]), ld(&s->x[3 * e[1]]), ld(&s->x[3 * t[0]]),
                                   ld(&s->x[3 * t[1]]), ld(&s->x[3 * t[2]]))) {
        delete s;
        return fail(E_INTERSECTING, "intersecting initial configuration");
      }
    }
  *out = s;
  return OK;
}

// ---------------------------------------------------------------------------
// Energy, gradient, Hessian at x (step context must be set)
// ---------------------------------------------------------------------------
double energy(const Scene &s, const std::vector<double> &x) {
  double h2 = s.dt * s.dt;
  double Ein = 0.0;
  for (int i = 0; i < s.nv; ++i) {
    if (is_kin(s, i)) continue;
    double q = 0.0;
    for (int k = 0; k < 3; ++k) {
      double r = x[3 * i + k] - s.xhat[3 * i + k];
      q += r * r;
    }
    Ein += s.mass[i] * q / (2.0 * h2);
  }
  // AL penalty on the prescribed vertices:
  //   sum_K  kA w/2 |x - xbar|^2 - sqrt(w) Lam . (x - xbar)
  if (s.al)
    for (int i = 0; i < s.nv; ++i) {
      if (!is_kin(s, i)) continue;
      double q = 0.0, l = 0.0;
      for (int k = 0; k < 3; ++k) {
        double r = x[3 * i + k] - s.xbar[3 * i + k];
        q += r * r;
        l += s.Lam[3 * i + k] * r;
      }
      Ein += 0.5 * s.kA * s.w_al * q - std::sqrt(s.w_al) * l;
    }
  double Eel = 0.0;
  for (int e = 0; e < s.nt; ++e) {
    double xe[12], en;
    gather12(x, &s.tet[4 * e], xe);
    if (!tet_elastic(xe, &s.Dinv[9 * e], s.vol[e], s.mu_l[e], s.la_l[e], false, false, &en, nullptr, nullptr))
      return kInf;
    Eel += en;
  }
  double Eb = 0.0;
  std::vector<Pair> cand = candidates(s, x, nullptr);
  for (const Pair &c : cand) {
    double xx[12], d2;
    gather12(x, c.v, xx);
    int type = c.kind == 0 ? pt_classify(xx, &d2) : ee_classify(xx, &d2);
    if (!(d2 > 0.0)) return kInf;
    if (d2 < s.dhat * s.dhat)
      Eb += pair_barrier(c.kind, type, xx, s.dhat, s.kappa, eps_cross(s, c), false, false, nullptr, nullptr);
  }
  double Ef = 0.0, eps = s.eps_v * s.dt;
  for (const FricPair &f : s.fric) {
    double xx[12], xxn[12];
    gather12(x, f.v, xx);
    gather12(s.xn, f.v, xxn);
    Ef += friction_elem(xx, xxn, f.w, f.n, f.lambda, s.mu, eps, nullptr, nullptr);
  }
  double E = Ein + Eel + Eb + Ef;
  return std::isfinite(E) ? E : kInf;
}

// Sparse symmetric block matrix over all vertices (kinematic rows dropped).
struct BlockMat {
  std::map<std::pair<int, int>, std::array<double, 9>> b;
  void add(int i, int j, const double *blk, double scale) {
    auto &B = b[{i, j}];
    for (int k = 0; k < 9; ++k) B[k] += scale * blk[k];
  }
};

void add_element(const Scene &s, const int v[4], const double g[12], const double H[144], std::vector<double> &G,
                 std::vector<double> *Gabs, BlockMat *M) {
  for (int a = 0; a < 4; ++a) {
    if (!is_dof(s, v[a])) continue;
    for (int k = 0; k < 3; ++k) {
      G[3 * v[a] + k] += g[3 * a + k];
      if (Gabs) (*Gabs)[3 * v[a] + k] += std::fabs(g[3 * a + k]);
    }
    if (!M) continue;
    for (int b = 0; b < 4; ++b) {
      if (!is_dof(s, v[b])) continue;
      double blk[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) blk[r * 3 + c] = H[(3 * a + r) * 12 + 3 * b + c];
      M->add(v[a], v[b], blk, 1.0);
    }
  }
}

// Returns false on a non-finite or infeasible state.
bool grad_hess(const Scene &s, const std::vector<double> &x, std::vector<double> &G, std::vector<double> *Gabs,
               BlockMat *M) {
  G.assign(3 * s.nv, 0.0);
  if (Gabs) Gabs->assign(3 * s.nv, 0.0);
  double h2 = s.dt * s.dt;
  for (int i = 0; i < s.nv; ++i) {
    if (is_kin(s, i)) continue;
    double w = s.mass[i] / h2;
    for (int k = 0; k < 3; ++k) {
      double gi = w * (x[3 * i + k] - s.xhat[3 * i + k]);
      G[3 * i + k] += gi;
      if (Gabs) (*Gabs)[3 * i + k] += std::fabs(gi);
    }
    if (M) {
      double blk[9] = {w, 0, 0, 0, w, 0, 0, 0, w};
      M->add(i, i, blk, 1.0);
    }
  }
  if (s.al)
    for (int i = 0; i < s.nv; ++i) {
      if (!is_kin(s, i)) continue;
      double w = s.kA * s.w_al, sw = std::sqrt(s.w_al);
      for (int k = 0; k < 3; ++k) {
        double gi = w * (x[3 * i + k] - s.xbar[3 * i + k]) - sw * s.Lam[3 * i + k];
        G[3 * i + k] += gi;
        if (Gabs) (*Gabs)[3 * i + k] += std::fabs(gi);
      }
      if (M) {
        double blk[9] = {w, 0, 0, 0, w, 0, 0, 0, w};
        M->add(i, i, blk, 1.0);
      }
    }
  for (int e = 0; e < s.nt; ++e) {
    double xe[12], en, g[12], H[144];
    gather12(x, &s.tet[4 * e], xe);
    if (!tet_elastic(xe, &s.Dinv[9 * e], s.vol[e], s.mu_l[e], s.la_l[e], true, true, &en, g, H)) return false;
    add_element(s, &s.tet[4 * e], g, H, G, Gabs, M);
  }
  std::vector<Pair> cand = candidates(s, x, nullptr);
  for (const ActivePair &a : active_set(s, x, cand)) {
    if (!(a.d2 > 0.0)) return false;
    double xx[12], g[12], H[144];
    gather12(x, a.p.v, xx);
    pair_barrier(a.p.kind, a.type, xx, s.dhat, s.kappa, eps_cross(s, a.p), true, true, g, H);
    add_element(s, a.p.v, g, H, G, Gabs, M);
  }
  double eps = s.eps_v * s.dt;
  for (const FricPair &f : s.fric) {
    double xx[12], xxn[12], g[12], H[144];
    gather12(x, f.v, xx);
    gather12(s.xn, f.v, xxn);
    friction_elem(xx, xxn, f.w, f.n, f.lambda, s.mu, eps, g, H);
    add_element(s, f.v, g, H, G, Gabs, M);
  }
  for (double gv : G)
    if (!std::isfinite(gv)) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Linear solves on the free vertices
// ---------------------------------------------------------------------------
struct Csr {
  int n;  // block rows
  std::vector<int> rp, ci;
  std::vector<double> val;  // 9 per block
};

Csr to_csr(const Scene &s, const BlockMat &M, std::vector<int> &dof_of, std::vector<int> &vert_of) {
  dof_of.assign(s.nv, -1);
  vert_of.clear();
  for (int i = 0; i < s.nv; ++i)
    if (is_dof(s, i)) {
      dof_of[i] = (int)vert_of.size();
      vert_of.push_back(i);
    }
  Csr C;
  C.n = (int)vert_of.size();
  C.rp.assign(C.n + 1, 0);
  for (auto &kv : M.b) C.rp[dof_of[kv.first.first] + 1]++;
  for (int i = 0; i < C.n; ++i) C.rp[i + 1] += C.rp[i];
  C.ci.resize(M.b.size());
  C.val.resize(9 * M.b.size());
  std::vector<int> fill(C.rp.begin(), C.rp.end() - 1);
  for (auto &kv : M.b) {  // map order = row-major, column ascending
    int r = dof_of[kv.first.first];
    int k = fill[r]++;
    C.ci[k] = dof_of[kv.first.second];
    for (int q = 0; q < 9; ++q) C.val[9 * k + q] = kv.second[q];
  }
  return C;
}

void spmv(const Csr &C, const std::vector<double> &x, std::vector<double> &y) {
  y.assign(3 * C.n, 0.0);
  for (int i = 0; i < C.n; ++i)
    for (int k = C.rp[i]; k < C.rp[i + 1]; ++k) {
      const double *B = &C.val[9 * k];
      int j = C.ci[k];
      for (int r = 0; r < 3; ++r)
        y[3 * i + r] += B[3 * r] * x[3 * j] + B[3 * r + 1] * x[3 * j + 1] + B[3 * r + 2] * x[3 * j + 2];
    }
}

double vdot(const std::vector<double> &a, const std::vector<double> &b) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// Block-Jacobi preconditioned CG: solve C z = b to |r| <= tol |b|.
long pcg(const Csr &C, const std::vector<double> &b, std::vector<double> &z, double tol, long maxit) {
  int n = C.n;
  std::vector<double> Minv(9 * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = C.rp[i]; k < C.rp[i + 1]; ++k)
      if (C.ci[k] == i) {
        double Bi[9];
        std::copy(&C.val[9 * k], &C.val[9 * k] + 9, Bi);
        inv3(Bi, &Minv[9 * i]);
      }
  z.assign(3 * n, 0.0);
  std::vector<double> r = b, s(3 * n), p(3 * n), q;
  double bn = std::sqrt(vdot(b, b));
  if (bn == 0.0) return 0;
  auto prec = [&](const std::vector<double> &in, std::vector<double> &out) {
    for (int i = 0; i < n; ++i)
      for (int rr = 0; rr < 3; ++rr)
        out[3 * i + rr] = Minv[9 * i + 3 * rr] * in[3 * i] + Minv[9 * i + 3 * rr + 1] * in[3 * i + 1] +
                          Minv[9 * i + 3 * rr + 2] * in[3 * i + 2];
  };
  prec(r, s);
  p = s;
  double rs = vdot(r, s);
  long it = 0;
  while (it < maxit && std::sqrt(vdot(r, r)) > tol * bn) {
    spmv(C, p, q);
    double alpha = rs / vdot(p, q);
    for (int i = 0; i < 3 * n; ++i) {
      z[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    prec(r, s);
    double rs2 = vdot(r, s);
    double beta = rs2 / rs;
    rs = rs2;
    for (int i = 0; i < 3 * n; ++i) p[i] = s[i] + beta * p[i];
    ++it;
  }
  return it;
}

// Dense Cholesky solve (tiny systems).
bool dense_solve(const Csr &C, const std::vector<double> &b, std::vector<double> &z) {
  int N = 3 * C.n;
  std::vector<double> A((size_t)N * N, 0.0);
  for (int i = 0; i < C.n; ++i)
    for (int k = C.rp[i]; k < C.rp[i + 1]; ++k)
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) A[(size_t)(3 * i + r) * N + 3 * C.ci[k] + c] = C.val[9 * k + 3 * r + c];
  for (int j = 0; j < N; ++j) {
    double dsum = A[(size_t)j * N + j];
    for (int k = 0; k < j; ++k) dsum -= A[(size_t)j * N + k] * A[(size_t)j * N + k];
    if (!(dsum > 0.0)) return false;
    double L = std::sqrt(dsum);
    A[(size_t)j * N + j] = L;
    for (int i = j + 1; i < N; ++i) {
      double sacc = A[(size_t)i * N + j];
      for (int k = 0; k < j; ++k) sacc -= A[(size_t)i * N + k] * A[(size_t)j * N + k];
      A[(size_t)i * N + j] = sacc / L;
    }
  }
  z = b;
  for (int i = 0; i < N; ++i) {
    double sacc = z[i];
    for (int k = 0; k < i; ++k) sacc -= A[(size_t)i * N + k] * z[k];
    z[i] = sacc / A[(size_t)i * N + i];
  }
  for (int i = N - 1; i >= 0; --i) {
    double sacc = z[i];
    for (int k = i + 1; k < N; ++k) sacc -= A[(size_t)k * N + i] * z[k];
    z[i] = sacc / A[(size_t)i * N + i];
  }
  return true;
}

// Newton direction p (all vertices, kinematic entries 0).  Returns false if
// the state is not finite.
bool newton_dir(const Scene &s, const std::vector<double> &x, std::vector<double> &p, long *iters) {
  std::vector<double> G;
  BlockMat M;
  if (!grad_hess(s, x, G, nullptr, &M)) return false;
  std::vector<int> dof_of, vert_of;
  Csr C = to_csr(s, M, dof_of, vert_of);
  std::vector<double> b(3 * C.n), z;
  for (int i = 0; i < C.n; ++i)
    for (int k = 0; k < 3; ++k) b[3 * i + k] = -G[3 * vert_of[i] + k];
  long it = 0;
  if (s.solver == 1) {
    if (!dense_solve(C, b, z)) return false;
  } else {
    it = pcg(C, b, z, s.pcg_tol, 10L * 3 * C.n + 10);
  }
  if (iters) *iters = it;
  p.assign(3 * s.nv, 0.0);
  for (int i = 0; i < C.n; ++i)
    for (int k = 0; k < 3; ++k) p[3 * vert_of[i] + k] = z[3 * i + k];
  for (double v : p)
    if (!std::isfinite(v)) return false;
  return true;
}

double ccd_bound(const Scene &s, const std::vector<double> &x, const std::vector<double> &p) {
  double alpha = 1.0;
  for (const Pair &c : candidates(s, x, p.data())) {
    double xx[12], pp[12];
    gather12(x, c.v, xx);
    gather12(p, c.v, pp);
    alpha = std::min(alpha, accd(c.kind, xx, pp, 0.1));
  }
  return alpha;
}

// ---------------------------------------------------------------------------
// Inversion filter (a step-size filter that keeps every tet inversion-free
// along the search line, Sec. II-C).  Along x + t p the volume factor of a
// tet, J(t) = det(Ds(x) + t Ds(p)), is a cubic in t with J(0) > 0: expanding
// the determinant column by column,
//   J(t) = k0 + k1 t + k2 t^2 + k3 t^3,
//   k0 = |a0 a1 a2|,  k1 = |b0 a1 a2| + |a0 b1 a2| + |a0 a1 b2|,
//   k2 = |a0 b1 b2| + |b0 a1 b2| + |b0 b1 a2|,  k3 = |b0 b1 b2|,
// with a_c, b_c the columns of Ds(x), Ds(p).  Its first positive root t*
// bounds the step: every tet keeps J > 0 on [0, 0.8 t*] (the factor 0.8 is
// a reading; the paper gives no constant).
// ---------------------------------------------------------------------------
double det_cols(const double *c0, const double *c1, const double *c2) {
  return c0[0] * (c1[1] * c2[2] - c1[2] * c2[1]) - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1]) +
         c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]);
}

void det_cubic(const double *x12, const double *p12, double k[4]) {
  double a[3][3], b[3][3];
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) {
      a[c][r] = x12[3 * (c + 1) + r] - x12[r];
      b[c][r] = p12[3 * (c + 1) + r] - p12[r];
    }
  k[0] = det_cols(a[0], a[1], a[2]);
  k[1] = det_cols(b[0], a[1], a[2]) + det_cols(a[0], b[1], a[2]) + det_cols(a[0], a[1], b[2]);
  k[2] = det_cols(a[0], b[1], b[2]) + det_cols(b[0], a[1], b[2]) + det_cols(b[0], b[1], a[2]);
  k[3] = det_cols(b[0], b[1], b[2]);
}

double cubic_at(const double k[4], double t) { return ((k[3] * t + k[2]) * t + k[1]) * t + k[0]; }

// First t in (0, tmax] with J(t) <= 0 (+inf if J stays positive there).  The
// stationary points of J (roots of J' = k1 + 2 k2 t + 3 k3 t^2) split
// [0, tmax] into pieces on which J is monotone; the first piece whose right
// end has J <= 0 holds the root, found by bisection.
double first_root(const double k[4], double tmax) {
  if (!(k[0] > 0.0)) return 0.0;
  std::vector<double> cut = {0.0};
  double A = 3.0 * k[3], B = 2.0 * k[2], C = k[1];
  if (A != 0.0) {
    double disc = B * B - 4.0 * A * C;
    if (disc >= 0.0) {
      double sq = std::sqrt(disc);
      double r1 = (-B - sq) / (2.0 * A), r2 = (-B + sq) / (2.0 * A);
      for (double r : {std::min(r1, r2), std::max(r1, r2)})
        if (r > 0.0 && r < tmax) cut.push_back(r);
    }
  } else if (B != 0.0) {
    double r = -C / B;
    if (r > 0.0 && r < tmax) cut.push_back(r);
  }
  cut.push_back(tmax);
  for (size_t i = 0; i + 1 < cut.size(); ++i) {
    double lo = cut[i], hi = cut[i + 1];
    if (cubic_at(k, hi) > 0.0) continue;
    // J(lo) > 0 >= J(hi): bisect to the interval's resolution
    for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
      double mid = 0.5 * (lo + hi);
      if (cubic_at(k, mid) > 0.0)
        lo = mid;
      else
        hi = mid;
    }
    return hi;
  }
  return kInf;
}

constexpr double kInvSafety = 0.8;

// min over tets of 0.8 t* (capped at 1), the inversion filter's step bound
double inversion_bound(const Scene &s, const std::vector<double> &x, const std::vector<double> &p) {
  double alpha = 1.0;
  for (int e = 0; e < s.nt; ++e) {
    double xe[12], pe[12], k[4];
    gather12(x, &s.tet[4 * e], xe);
    gather12(p, &s.tet[4 * e], pe);
    det_cubic(xe, pe, k);
    double t = first_root(k, 1.0 / kInvSafety);
    alpha = std::min(alpha, kInvSafety * t);
  }
  return alpha;
}

bool all_tets_positive(const Scene &s, const std::vector<double> &x) {
  for (int e = 0; e < s.nt; ++e) {
    double xe[12], Ds[9], F[9];
    gather12(x, &s.tet[4 * e], xe);
    build_Ds(xe, Ds);
    matmul3(Ds, &s.Dinv[9 * e], F);
    if (!(det3<double>(F) > 0.0)) return false;
  }
  return true;
}

// Lagged friction data (lambda, n, closest-point weights) of the active
// pairs at xl; the tangential displacement is always measured from x^n.
// The first lag of a step is taken at x^n; with friction_iters > 1 it is
// taken again at each converged iterate and the step is solved again.
void lag_friction(Scene &s, const std::vector<double> &xl) {
  s.fric.clear();
  std::vector<Pair> cand = candidates(s, xl, nullptr);
  for (const ActivePair &a : active_set(s, xl, cand)) {
    double xx[12];
    gather12(xl, a.p.v, xx);
    FricPair f;
    std::copy(a.p.v, a.p.v + 4, f.v);
    closest_weights(a.p.kind, a.type, xx, f.w);
    double dv[3] = {0, 0, 0};
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 3; ++k) dv[k] += f.w[i] * xx[3 * i + k];
    double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    for (int k = 0; k < 3; ++k) f.n[k] = dv[k] / dn;
    double d = std::sqrt(a.d2), b[3];
    barrier_scalar(d, s.dhat, b);
    double e = 1.0;
    if (a.p.kind == 1) {
      V3 ea = sub(ld(xx + 3), ld(xx)), eb = sub(ld(xx + 9), ld(xx + 6));
      V3 c3 = cross(ea, eb);
      double c = dot(c3, c3), ex = eps_cross(s, a.p);
      if (c < ex) e = (c / ex) * (2.0 - c / ex);
    }
    f.lambda = -s.kappa * e * b[1];
    if (f.lambda > 0.0 && s.mu > 0.0) s.fric.push_back(f);
  }
}

// Kinematic targets, predicted positions, lagged friction and the direct
// Dirichlet move for the step n -> n+1.  Returns the starting iterate in x0.
int begin_step(Scene &s, std::vector<double> &x0) {
  int n = s.step;
  int mrow = std::min(n + 1, s.nmotion - 1);
  int grow = std::min(n, s.nmotion - 1);
  const double *g = s.g_over ? s.g_ovr : &s.gravity[3 * grow];
  double h = s.dt;
  s.xn = s.x;
  s.xhat = s.x;
  s.xbar = s.x;
  for (int i = 0; i < s.nv; ++i) {
    if (is_kin(s, i)) {
      int row = mrow;
      if (!s.hold.empty() && s.hold[s.kin[i]] >= 0) row = std::min(row, s.hold[s.kin[i]]);
      const double *T = &s.motion[12L * (row * s.ngroups + s.kin[i])];
      const double *X = &s.X[3 * i];
      for (int r = 0; r < 3; ++r)
        s.xbar[3 * i + r] = T[4 * r] * X[0] + T[4 * r + 1] * X[1] + T[4 * r + 2] * X[2] + T[4 * r + 3];
    } else {
      for (int k = 0; k < 3; ++k) s.xhat[3 * i + k] = s.x[3 * i + k] + h * s.v[3 * i + k] + h * h * g[k];
    }
  }
  // lagged friction set at x^n
  lag_friction(s, s.xn);
  // direct Dirichlet move if CCD-safe and inversion-free
  std::vector<double> y = s.xn, dp(3 * s.nv, 0.0);
  bool any = false;
  for (int i = 0; i < s.nv; ++i)
    if (is_kin(s, i))
      for (int k = 0; k < 3; ++k) {
        y[3 * i + k] = s.xbar[3 * i + k];
        dp[3 * i + k] = y[3 * i + k] - s.xn[3 * i + k];
        if (dp[3 * i + k] != 0.0) any = true;
      }
  s.ctx = true;
  s.al = false;
  if (any && (ccd_bound(s, s.xn, dp) < 1.0 || !all_tets_positive(s, y))) {
    // the prescribed move is not feasible in one go: the kinematic vertices
    // become unknowns pulled to their targets by an augmented Lagrangian
    s.al = true;
    s.kA = 1e3;
    s.w_al = s.mbar / (h * h);
    s.viol_prev = kInf;
    s.Lam.assign(3 * s.nv, 0.0);
    x0 = s.xn;
    return FAIL_NONE;
  }
  x0 = y;
  return FAIL_NONE;
}

// Largest distance of a prescribed vertex from its target (AL mode).
double dbc_violation(const Scene &s, const std::vector<double> &x) {
  double v = 0.0;
  for (int i = 0; i < s.nv; ++i)
    if (is_kin(s, i))
      for (int k = 0; k < 3; ++k) v = std::max(v, std::fabs(x[3 * i + k] - s.xbar[3 * i + k]));
  return v;
}

// Contact statistics of an accepted iterate: the number of active pairs
// (d^2 < dhat^2) and the least distance among them (+inf if there are none).
void min_dist(const Scene &s, const std::vector<double> &x, double *dmin, long *nact) {
  std::vector<Pair> cand = candidates(s, x, nullptr);
  double m = kInf;
  long na = 0;
  for (const Pair &c : cand) {
    double xx[12], d2;
    gather12(x, c.v, xx);
    if (c.kind == 0)
      pt_classify(xx, &d2);
    else
      ee_classify(xx, &d2);
    if (d2 < s.dhat * s.dhat) {
      m = std::min(m, d2);
      ++na;
    }
  }
  *dmin = std::sqrt(m);
  *nact = na;
}

// Adaptive barrier stiffness (variant): at each Newton iterate, if the least
// active-pair distance is below 1e-2 dhat and smaller than at the previous
// iterate, kappa doubles, up to 100 times its given value (a reading of IPC's
// adaptive stiffness; the paper fixes kappa = 3e6, Sec. III-D).
void adapt_kappa(Scene &s, const std::vector<double> &x) {
  double d;
  long na;
  min_dist(s, x, &d, &na);
  if (d < 1e-2 * s.dhat && d < s.dmin_prev) s.kappa = std::min(2.0 * s.kappa, 100.0 * s.kappa0);
  s.dmin_prev = d;
}

// One projected-Newton solve from x (Sec. II-C): direction from the
// PSD-projected Hessian, stop on |p|_inf <= tol dt, CCD (and optionally
// inversion) step bound, backtracking line search on Phi.  Returns FAIL_NONE
// when converged, else the failure reason; *n_dirs counts the directions.
int newton_solve(Scene &s, std::vector<double> &x, ipco_info *info, int *n_dirs) {
  double tolh = s.tol * s.dt;
  std::vector<double> p, xt(3 * s.nv);
  int it = 0;
  *n_dirs = 0;
  for (; it < s.maxit; ++it) {
    if (s.adaptive_kappa) adapt_kappa(s, x);
    long pit = 0;
    if (!newton_dir(s, x, p, &pit)) return FAIL_NONFINITE;
    *n_dirs = it + 1;
    if (info) info->pcg_iters += pit;
    double pinf = 0.0;
    for (double v : p) pinf = std::max(pinf, std::fabs(v));
    if (pinf <= tolh) {
      if (!s.al) return FAIL_NONE;
      // AL mode: the inner problem converged.  Snap to the targets once they
      // are within 1e-2 dhat and the move is CCD-safe; otherwise update the
      // multipliers (and double kA unless the violation fell tenfold).
      double viol = dbc_violation(s, x);
      if (viol <= 1e-2 * s.dhat) {
        std::vector<double> dp(3 * s.nv, 0.0), y = x;
        for (int i = 0; i < s.nv; ++i)
          if (is_kin(s, i))
            for (int k = 0; k < 3; ++k) {
              dp[3 * i + k] = s.xbar[3 * i + k] - x[3 * i + k];
              y[3 * i + k] = s.xbar[3 * i + k];
            }
        if (ccd_bound(s, x, dp) >= 1.0 && all_tets_positive(s, y)) {
          x = y;
          s.al = false;
          continue;
        }
      }
      double sw = std::sqrt(s.w_al);
      for (int i = 0; i < s.nv; ++i)
        if (is_kin(s, i))
          for (int k = 0; k < 3; ++k) s.Lam[3 * i + k] -= s.kA * sw * (x[3 * i + k] - s.xbar[3 * i + k]);
      if (viol > 0.1 * s.viol_prev) s.kA *= 2.0;
      s.viol_prev = viol;
      continue;
    }
    double alpha = ccd_bound(s, x, p);
    if (s.inv_filter) alpha = std::min(alpha, inversion_bound(s, x, p));
    double E0 = energy(s, x);
    int halvings = 0;
    for (;;) {
      for (int i = 0; i < 3 * s.nv; ++i) xt[i] = x[i] + alpha * p[i];
      double E1 = energy(s, xt) + s.debug_ls_offset;
      if (E1 <= E0) {
        s.iter_log.insert(s.iter_log.end(), {E0, E1, alpha, (double)halvings});
        break;
      }
      alpha *= 0.5;
      if (++halvings > 40) return FAIL_LS;
    }
    if (info) info->ls_halvings += halvings;
    x = xt;
  }
  return FAIL_MAXIT;
}

int step_one(Scene &s, ipco_info *info) {
  std::vector<double> x;
  int fr = begin_step(s, x);
  s.iter_log.clear();
  int dirs_total = 0;
  // friction lagged at x^n, then (variant) re-lagged at each converged iterate
  for (int lag = 0; fr == FAIL_NONE && lag < s.friction_iters; ++lag) {
    if (lag > 0) lag_friction(s, x);
    int dirs = 0;
    fr = newton_solve(s, x, info, &dirs);
    dirs_total += dirs;
  }
  if (info) {
    info->newton_iters += dirs_total;
    info->max_newton_iters = std::max(info->max_newton_iters, dirs_total);
    info->kappa_last = s.kappa;
  }
  if (fr != FAIL_NONE) {
    s.failed = true;
    s.fail_reason = fr;
    return E_FAILED;
  }
  for (int i = 0; i < 3 * s.nv; ++i) s.v[i] = (x[i] - s.xn[i]) / s.dt;
  s.x = x;
  s.step += 1;
  s.ctx = false;
  if (info) {
    double dm;
    long na;
    min_dist(s, s.x, &dm, &na);
    info->min_dist_last = dm;
    info->n_active_last = na;
  }
  return OK;
}

void cauchy_stress(const Scene &s, int e, double out[6], double *vm) {
  double xe[12], Ds[9], F[9];
  gather12(s.x, &s.tet[4 * e], xe);
  build_Ds(xe, Ds);
  matmul3(Ds, &s.Dinv[9 * e], F);
  double J = det3<double>(F);
  double Finv[9];
  inv3(F, Finv);
  double mu = s.mu_l[e], la = s.la_l[e], lJ = std::log(J);
  double P[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i * 3 + j] = mu * F[i * 3 + j] + (la * lJ - mu) * Finv[j * 3 + i];
  double S[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += P[i * 3 + k] * F[j * 3 + k];
      S[i * 3 + j] = acc / J;
    }
  out[0] = S[0];
  out[1] = S[4];
  out[2] = S[8];
  out[3] = S[5];
  out[4] = S[2];
  out[5] = S[1];
  double a = S[0] - S[4], b = S[4] - S[8], c = S[8] - S[0];
  *vm = std::sqrt(0.5 * (a * a + b * b + c * c) + 3.0 * (S[1] * S[1] + S[5] * S[5] + S[2] * S[2]));
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

int ipco_create(const ipco_desc *d, void **out) {
  if (!out) return fail(E_ARG, "null output handle");
  Scene *s = nullptr;
  int rc = build_scene(d, &s);
  if (rc != OK) return rc;
  *out = s;
  return OK;
}

void ipco_destroy(void *s) { delete static_cast<Scene *>(s); }

const char *ipco_last_error(void) { return g_err.c_str(); }

int ipco_step(void *h, int32_t n_steps, ipco_info *info) {
  Scene *s = static_cast<Scene *>(h);
  if (!s || n_steps < 0) return fail(E_ARG, "bad arguments");
  if (info) std::memset(info, 0, sizeof(*info));
  if (s->failed) {
    if (info) {
      info->status = E_FAILED;
      info->fail_reason = s->fail_reason;
    }
    return fail(E_FAILED, "scene already failed");
  }
  for (int k = 0; k < n_steps; ++k) {
    int rc = step_one(*s, info);
    if (rc != OK) {
      if (info) {
        info->status = rc;
        info->fail_reason = s->fail_reason;
      }
      return fail(rc, "step failed");
    }
    if (info) info->steps_done += 1;
  }
  if (info) info->energy_last = 0.0;
  return OK;
}

int ipco_get_state(void *h, double *pos, double *vel, double *cauchy, double *vm) {
  Scene *s = static_cast<Scene *>(h);
  if (!s || !pos) return fail(E_ARG, "bad arguments");
  std::copy(s->x.begin(), s->x.end(), pos);
  if (vel) std::copy(s->v.begin(), s->v.end(), vel);
  if (cauchy || vm)
    for (int e = 0; e < s->nt; ++e) {
      double c[6], v;
      cauchy_stress(*s, e, c, &v);
      if (cauchy) std::copy(c, c + 6, cauchy + 6L * e);
      if (vm) vm[e] = v;
    }
  return OK;
}

int ipco_set_state(void *h, const double *pos, const double *vel, int32_t step) {
  Scene *s = static_cast<Scene *>(h);
  if (!s || !pos || step < 0) return fail(E_ARG, "bad arguments");
  s->x.assign(pos, pos + 3 * s->nv);
  if (vel)
    s->v.assign(vel, vel + 3 * s->nv);
  else
    s->v.assign(3 * s->nv, 0.0);
  s->step = step;
  s->failed = false;
  s->fail_reason = 0;
  s->ctx = false;
  return OK;
}

int ipco_get_step(void *h) { return static_cast<Scene *>(h)->step; }

int ipco_surface_sizes(void *h, int32_t out[3]) {
  Scene *s = static_cast<Scene *>(h);
  out[0] = (int)s->stri.size();
  out[1] = (int)s->sedge.size();
  out[2] = (int)s->svert.size();
  return OK;
}

int ipco_surface(void *h, int32_t *tris, int32_t *edges, int32_t *verts) {
  Scene *s = static_cast<Scene *>(h);
  for (size_t i = 0; i < s->stri.size(); ++i)
    for (int k = 0; k < 3; ++k) tris[3 * i + k] = s->stri[i][k];
  for (size_t i = 0; i < s->sedge.size(); ++i)
    for (int k = 0; k < 2; ++k) edges[2 * i + k] = s->sedge[i][k];
  for (size_t i = 0; i < s->svert.size(); ++i) verts[i] = s->svert[i];
  return OK;
}

int ipco_mass(void *h, double *mass) {
  Scene *s = static_cast<Scene *>(h);
  std::copy(s->mass.begin(), s->mass.end(), mass);
  return OK;
}

int64_t ipco_candidates(void *h, const double *x, const double *p, int32_t *out, int64_t cap) {
  Scene *s = static_cast<Scene *>(h);
  std::vector<double> xv(x, x + 3 * s->nv);
  std::vector<Pair> c = candidates(*s, xv, p);
  for (size_t i = 0; i < c.size() && (int64_t)i < cap; ++i) {
    out[5 * i] = c[i].kind;
    for (int k = 0; k < 4; ++k) out[5 * i + 1 + k] = c[i].v[k];
  }
  return (int64_t)c.size();
}

int64_t ipco_active(void *h, const double *x, int32_t *out, double *d2, int64_t cap) {
  Scene *s = static_cast<Scene *>(h);
  std::vector<double> xv(x, x + 3 * s->nv);
  std::vector<ActivePair> a = active_set(*s, xv, candidates(*s, xv, nullptr));
  for (size_t i = 0; i < a.size() && (int64_t)i < cap; ++i) {
    out[6 * i] = a[i].p.kind;
    for (int k = 0; k < 4; ++k) out[6 * i + 1 + k] = a[i].p.v[k];
    out[6 * i + 5] = a[i].type;
    if (d2) d2[i] = a[i].d2;
  }
  return (int64_t)a.size();
}

int ipco_begin_step(void *h, double *x_start) {
  Scene *s = static_cast<Scene *>(h);
  std::vector<double> x0;
  int fr = begin_step(*s, x0);
  if (fr != FAIL_NONE) return fail(E_FAILED, "direct Dirichlet move is not feasible");
  if (x_start) std::copy(x0.begin(), x0.end(), x_start);
  return OK;
}

double ipco_energy(void *h, const double *x) {
  Scene *s = static_cast<Scene *>(h);
  if (!s->ctx) return std::nan("");
  return energy(*s, std::vector<double>(x, x + 3 * s->nv));
}

int ipco_gradient(void *h, const double *x, double *g, double *gabs) {
  Scene *s = static_cast<Scene *>(h);
  if (!s->ctx) return fail(E_ARG, "call ipco_begin_step first");
  std::vector<double> G, Ga;
  if (!grad_hess(*s, std::vector<double>(x, x + 3 * s->nv), G, &Ga, nullptr)) return fail(E_FAILED, "non-finite");
  std::copy(G.begin(), G.end(), g);
  if (gabs) std::copy(Ga.begin(), Ga.end(), gabs);
  return OK;
}

int ipco_hessian_dense(void *h, const double *x, double *H) {
  Scene *s = static_cast<Scene *>(h);
  if (!s->ctx) return fail(E_ARG, "call ipco_begin_step first");
  std::vector<double> G;
  BlockMat M;
  if (!grad_hess(*s, std::vector<double>(x, x + 3 * s->nv), G, nullptr, &M)) return fail(E_FAILED, "non-finite");
  long N = 3L * s->nv;
  std::fill(H, H + N * N, 0.0);
  for (int i = 0; i < s->nv; ++i)
    if (!is_dof(*s, i))
      for (int k = 0; k < 3; ++k) H[(3 * i + k) * N + 3 * i + k] = 1.0;
  for (auto &kv : M.b)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) H[(3L * kv.first.first + r) * N + 3L * kv.first.second + c] = kv.second[3 * r + c];
  return OK;
}

int ipco_newton_dir(void *h, const double *x, double *p, int64_t *pcg_iters) {
  Scene *s = static_cast<Scene *>(h);
  if (!s->ctx) return fail(E_ARG, "call ipco_begin_step first");
  std::vector<double> P;
  long it = 0;
  if (!newton_dir(*s, std::vector<double>(x, x + 3 * s->nv), P, &it)) return fail(E_FAILED, "non-finite");
  std::copy(P.begin(), P.end(), p);
  if (pcg_iters) *pcg_iters = it;
  return OK;
}

double ipco_ccd_bound(void *h, const double *x, const double *p) {
  Scene *s = static_cast<Scene *>(h);
  return ccd_bound(*s, std::vector<double>(x, x + 3 * s->nv), std::vector<double>(p, p + 3 * s->nv));
}

int64_t ipco_friction_pairs(void *h, int32_t *verts, double *lambda_, double *normal, double *w, int64_t cap) {
  Scene *s = static_cast<Scene *>(h);
  for (size_t i = 0; i < s->fric.size() && (int64_t)i < cap; ++i) {
    const FricPair &f = s->fric[i];
    for (int k = 0; k < 4; ++k) {
      if (verts) verts[4 * i + k] = f.v[k];
      if (w) w[4 * i + k] = f.w[k];
    }
    if (lambda_) lambda_[i] = f.lambda;
    if (normal)
      for (int k = 0; k < 3; ++k) normal[3 * i + k] = f.n[k];
  }
  return (int64_t)s->fric.size();
}

int ipco_pt_classify(const double *x12, double *d2) { return pt_classify(x12, d2); }
int ipco_ee_classify(const double *x12, double *d2) { return ee_classify(x12, d2); }

int ipco_barrier_scalar(double d, double dhat, double *out3) {
  barrier_scalar(d, dhat, out3);
  return OK;
}

int ipco_pair_barrier(int kind, int type, const double *x12, double dhat, double kappa, double eps_x, int project,
                      double *energy_out, double *g12, double *H144) {
  double g[12], H[144];
  double e = pair_barrier(kind, type, x12, dhat, kappa, eps_x, true, project != 0, g, H);
  if (energy_out) *energy_out = e;
  if (g12) std::copy(g, g + 12, g12);
  if (H144) std::copy(H, H + 144, H144);
  return OK;
}

int ipco_tet_elastic(const double *X12, const double *x12, double E, double nu, int project, double *energy_out,
                     double *g12, double *H144) {
  double Dm[9], Dinv[9], mu, la;
  build_Ds(X12, Dm);
  double det = det3<double>(Dm);
  if (!(det > 0.0) || !inv3(Dm, Dinv)) return fail(E_INVERTED, "bad rest tet");
  lame(E, nu, &mu, &la);
  double en, g[12], H[144];
  if (!tet_elastic(x12, Dinv, det / 6.0, mu, la, true, project != 0, &en, g, H)) {
    if (energy_out) *energy_out = kInf;
    return E_INVERTED;
  }
  if (energy_out) *energy_out = en;
  if (g12) std::copy(g, g + 12, g12);
  if (H144) std::copy(H, H + 144, H144);
  return OK;
}

int ipco_psd_project(int n, double *A) {
  if (n <= 0 || n > 64) return fail(E_ARG, "bad size");
  psd_project(n, A);
  return OK;
}

double ipco_accd(int kind, const double *x12, const double *p12, double s) { return accd(kind, x12, p12, s); }

int64_t ipco_iter_log(void *h, double *out, int64_t cap) {
  Scene *s = static_cast<Scene *>(h);
  int64_t n = (int64_t)s->iter_log.size() / 4;
  for (int64_t i = 0; i < 4 * std::min(n, cap); ++i) out[i] = s->iter_log[i];
  return n;
}

double ipco_tet_first_root(const double *x12, const double *p12, double tmax, double *k4) {
  double k[4];
  det_cubic(x12, p12, k);
  if (k4)
    for (int i = 0; i < 4; ++i) k4[i] = k[i];
  return first_root(k, tmax);
}

double ipco_inversion_bound(void *h, const double *x, const double *p) {
  Scene *s = static_cast<Scene *>(h);
  return inversion_bound(*s, std::vector<double>(x, x + 3 * s->nv), std::vector<double>(p, p + 3 * s->nv));
}

double ipco_kappa(void *h) { return static_cast<Scene *>(h)->kappa; }

// Contact force between tagged bodies at x (Sec. III-D halts a finger once its
// contact force exceeds 50 N).  For every active pair the barrier pushes its
// two sides apart along the unit normal n of the closest-point difference
// (from the triangle / second edge toward the point / first edge) with
// magnitude lambda = -kappa e b'(d): the first side receives +lambda n, the
// second -lambda n.  out[(a ntags + b) 3 + k] sums, over the pairs whose first
// side is tagged a and second side b (and the reverse, with the sign
// flipped), the force exerted on a by b.  Vertices tagged outside [0, ntags)
// are ignored.
int ipco_contact_forces(void *h, const double *x, const int32_t *tags, int32_t ntags, double *out) {
  Scene *s = static_cast<Scene *>(h);
  if (!s || !x || !tags || ntags < 1 || !out) return fail(E_ARG, "bad arguments");
  std::vector<double> xv(x, x + 3 * s->nv);
  for (int k = 0; k < 3 * ntags * ntags; ++k) out[k] = 0.0;
  std::vector<Pair> cand = candidates(*s, xv, nullptr);
  for (const ActivePair &a : active_set(*s, xv, cand)) {
    double xx[12], w[4];
    gather12(xv, a.p.v, xx);
    closest_weights(a.p.kind, a.type, xx, w);
    double dv[3] = {0, 0, 0};
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 3; ++k) dv[k] += w[i] * xx[3 * i + k];
    double dn = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    double d = std::sqrt(a.d2), b[3];
    barrier_scalar(d, s->dhat, b);
    double e = 1.0;
    if (a.p.kind == 1) {
      V3 ea = sub(ld(xx + 3), ld(xx)), eb = sub(ld(xx + 9), ld(xx + 6));
      V3 c3 = cross(ea, eb);
      double c = dot(c3, c3), ex = eps_cross(*s, a.p);
      if (c < ex) e = (c / ex) * (2.0 - c / ex);
    }
    double lambda = -s->kappa * e * b[1];
    int ta = tags[a.p.v[0]], tb = tags[a.p.v[a.p.kind == 0 ? 1 : 2]];
    if (ta < 0 || ta >= ntags || tb < 0 || tb >= ntags) continue;
    for (int k = 0; k < 3; ++k) {
      out[(ta * ntags + tb) * 3 + k] += lambda * dv[k] / dn;
      out[(tb * ntags + ta) * 3 + k] -= lambda * dv[k] / dn;
    }
  }
  return OK;
}

int ipco_hold_group(void *h, int32_t group, int32_t row) {
  Scene *s = static_cast<Scene *>(h);
  if (!s || group < 0 || group >= s->ngroups || row < -1) return fail(E_ARG, "bad arguments");
  if (s->hold.empty()) s->hold.assign(s->ngroups, -1);
  s->hold[group] = row;
  return OK;
}

int ipco_set_gravity(void *h, const double *g) {
  Scene *s = static_cast<Scene *>(h);
  if (!s) return fail(E_ARG, "bad arguments");
  s->g_over = g != nullptr;
  if (g)
    for (int k = 0; k < 3; ++k) s->g_ovr[k] = g[k];
  return OK;
}

int ipco_debug_ls_offset(void *h, double delta) {
  static_cast<Scene *>(h)->debug_ls_offset = delta;
  return OK;
}

int ipco_friction_elem(const double *x12, const double *xn12, const double *w4, const double *n3, double lambda,
                       double mu, double eps, double *energy, double *g12, double *H144) {
  double e = friction_elem(x12, xn12, w4, n3, lambda, mu, eps, g12, H144);
  if (energy) *energy = e;
  return OK;
}

int ipco_friction_f0(double y, double eps, double *out3) {
  friction_f0(y, eps, out3);
  return OK;
}

}  // extern "C"
