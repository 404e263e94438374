// device_math.h -- per-element device routines of the IPC time step.
//
// Distances, barrier, mollifier, friction, Neo-Hookean elasticity, PSD
// projection and additive CCD for one element.  The derivative formulas here
// are derived by hand (see the comments); they are independent of the CPU
// oracle, which differentiates the energies automatically.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEV __host__ __device__ inline
#define HD __host__ __device__ inline

namespace ipcdev {

constexpr double kInf = __builtin_huge_val();

struct d3 {
  double x, y, z;
};
HD d3 ld3(const double *p) { return {p[0], p[1], p[2]}; }

// -- exact-sequence vector ops (no contraction: the classification and the
//    active test must reproduce the host's rounding bit for bit) -------------
HD d3 sub3(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
HD double dot3(d3 a, d3 b) {
#pragma clang fp contract(off)
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
HD d3 cross3(d3 a, d3 b) {
#pragma clang fp contract(off)
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// -- pair classification ------------------------------------------------------
// PT pair (p, t0, t1, t2): 0 interior, 1..3 point-edge (t0,t1),(t1,t2),(t2,t0),
// 4..6 point-point t0,t1,t2.  EE pair (a0, a1, b0, b1): 0 interior, 1 a0|b,
// 2 a1|b, 3 b0|a, 4 b1|a, 5 a0-b0, 6 a0-b1, 7 a1-b0, 8 a1-b1.
enum { PS_A = 0, PS_B = 1, PS_E = 2 };

HD int point_seg(d3 p, d3 a, d3 b, double *d2) {
#pragma clang fp contract(off)
  d3 e = sub3(b, a);
  d3 w = sub3(p, a);
  double ee = dot3(e, e);
  if (!(ee > 0.0)) {
    *d2 = dot3(w, w);
    return PS_A;
  }
  double s = dot3(w, e) / ee;
  if (s <= 0.0) {
    *d2 = dot3(w, w);
    return PS_A;
  }
  if (s >= 1.0) {
    d3 q = sub3(p, b);
    *d2 = dot3(q, q);
    return PS_B;
  }
  d3 c = cross3(w, e);
  *d2 = dot3(c, c) / ee;
  return PS_E;
}

HD int classify_pt(d3 p, d3 t0, d3 t1, d3 t2, double *d2out) {
#pragma clang fp contract(off)
  d3 e1 = sub3(t1, t0), e2 = sub3(t2, t0), w = sub3(p, t0);
  double a = dot3(e1, e1), b = dot3(e1, e2), c = dot3(e2, e2), d = dot3(e1, w), e = dot3(e2, w);
  double det = a * c - b * b;
  if (det > 0.0) {
    double b1 = (c * d - b * e) / det;
    double b2 = (a * e - b * d) / det;
    if (b1 >= 0.0 && b2 >= 0.0 && b1 + b2 <= 1.0) {
      d3 n = cross3(e1, e2);
      double wn = dot3(w, n);
      *d2out = wn * wn / dot3(n, n);
      return 0;
    }
  }
  double best = kInf;
  int type = -1;
  d3 T[3] = {t0, t1, t2};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double d2;
    int k = point_seg(p, T[j], T[j == 2 ? 0 : j + 1], &d2);
    if (d2 < best) {
      best = d2;
      type = (k == PS_E) ? 1 + j : (k == PS_A ? 4 + j : 4 + (j == 2 ? 0 : j + 1));
    }
  }
  *d2out = best;
  return type;
}

HD int classify_ee(d3 a0, d3 a1, d3 b0, d3 b1, double *d2out) {
#pragma clang fp contract(off)
  d3 ea = sub3(a1, a0), eb = sub3(b1, b0), w = sub3(a0, b0);
  d3 n = cross3(ea, eb);
  double nn = dot3(n, n);
  double A = dot3(ea, ea), B = dot3(ea, eb), C = dot3(eb, eb), D = dot3(ea, w), E = dot3(eb, w);
  if (nn > 1e-12 * A * C) {
    double det = A * C - B * B;
    double s = (B * E - C * D) / det;
    double t = (A * E - B * D) / det;
    if (s > 0.0 && s < 1.0 && t > 0.0 && t < 1.0) {
      double wn = dot3(w, n);
      *d2out = wn * wn / nn;
      return 0;
    }
  }
  const int ppA[4] = {5, 7, 5, 6}, ppB[4] = {6, 8, 7, 8};
  d3 P[4] = {a0, a1, b0, b1};
  double best = kInf;
  int type = -1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double d2;
    int r = (k < 2) ? point_seg(P[k], b0, b1, &d2) : point_seg(P[k], a0, a1, &d2);
    if (d2 < best) {
      best = d2;
      type = (r == PS_E) ? 1 + k : (r == PS_A ? ppA[k] : ppB[k]);
    }
  }
  *d2out = best;
  return type;
}

HD int classify(int kind, const double *x, double *d2) {
  return kind == 0 ? classify_pt(ld3(x), ld3(x + 3), ld3(x + 6), ld3(x + 9), d2)
                   : classify_ee(ld3(x), ld3(x + 3), ld3(x + 6), ld3(x + 9), d2);
}

// -- squared distance of a classified pair with derivatives --------------------
// Every type is d^2(x) = min_beta |r(x, beta)|^2 with r = sum_i c_i(beta) x_i
// and c affine in the parameters beta (none for point-point, the segment
// parameter for point-edge, the barycentric pair for point-triangle, the two
// segment parameters for edge-edge).  At the minimiser (envelope theorem):
//   grad_i d^2   = 2 c_i r
//   hess_ij d^2  = 2 c_i c_j I - 2 sum_kl Ginv_kl u_ik u_jl^T,
//   q_k = sum_i (dc_i/dbeta_k) x_i,  G_kl = q_k . q_l,  u_ik = c_i q_k + (dc_i/dbeta_k) r.
struct TypeGeo {
  int nb;           // number of parameters
  double c[4];      // coefficient of each pair slot
  double dc[2][4];  // d c / d beta_k
  int n_involved;
  int involved[4];
};

DEV void type_geometry(int kind, int type, const double *x, TypeGeo &T) {
  for (int i = 0; i < 4; ++i) {
    T.c[i] = 0.0;
    T.dc[0][i] = 0.0;
    T.dc[1][i] = 0.0;
  }
  d3 P[4] = {ld3(x), ld3(x + 3), ld3(x + 6), ld3(x + 9)};
  if (type == 0) {
    T.n_involved = 4;
    for (int i = 0; i < 4; ++i) T.involved[i] = i;
    T.nb = 2;
    if (kind == 0) {  // r = p - t0 - b1 (t1 - t0) - b2 (t2 - t0)
      d3 e1 = sub3(P[2], P[1]), e2 = sub3(P[3], P[1]), w = sub3(P[0], P[1]);
      double a = dot3(e1, e1), b = dot3(e1, e2), c = dot3(e2, e2), d = dot3(e1, w), e = dot3(e2, w);
      double det = a * c - b * b;
      double b1 = (c * d - b * e) / det, b2 = (a * e - b * d) / det;
      T.c[0] = 1.0;
      T.c[1] = -(1.0 - b1 - b2);
      T.c[2] = -b1;
      T.c[3] = -b2;
      T.dc[0][1] = 1.0;
      T.dc[0][2] = -1.0;
      T.dc[1][1] = 1.0;
      T.dc[1][3] = -1.0;
    } else {  // r = a0 + s (a1 - a0) - b0 - t (b1 - b0)
      d3 ea = sub3(P[1], P[0]), eb = sub3(P[3], P[2]), w = sub3(P[0], P[2]);
      double A = dot3(ea, ea), B = dot3(ea, eb), C = dot3(eb, eb), D = dot3(ea, w), E = dot3(eb, w);
      double det = A * C - B * B;
      double s = (B * E - C * D) / det, t = (A * E - B * D) / det;
      T.c[0] = 1.0 - s;
      T.c[1] = s;
      T.c[2] = -(1.0 - t);
      T.c[3] = -t;
      T.dc[0][0] = -1.0;
      T.dc[0][1] = 1.0;
      T.dc[1][2] = 1.0;
      T.dc[1][3] = -1.0;
    }
    return;
  }
  // sub-types: point-edge (point, a, b) or point-point (point, other); the
  // slots are picked with selects, not by indexing, so that the arrays stay
  // in registers
  int sp, sa, sb = -1;
  if (kind == 0) {
    sp = 0;
    if (type <= 3) {
      sa = type;
      sb = (type == 3) ? 1 : type + 1;
    } else {
      sa = type - 3;
    }
  } else if (type <= 4) {  // point-edge: (0; 2, 3), (1; 2, 3), (2; 0, 1), (3; 0, 1)
    sp = type - 1;
    sa = (type <= 2) ? 2 : 0;
    sb = sa + 1;
  } else {  // point-point: (0, 2), (0, 3), (1, 2), (1, 3)
    sp = (type <= 6) ? 0 : 1;
    sa = (type == 5 || type == 7) ? 2 : 3;
  }
  if (sb < 0) {  // r = p - q
    T.nb = 0;
    T.n_involved = 2;
    T.involved[0] = sp;
    T.involved[1] = sa;
#pragma unroll
    for (int i = 0; i < 4; ++i) T.c[i] = (i == sp) ? 1.0 : (i == sa) ? -1.0 : 0.0;
    return;
  }
  // r = p - a - s (b - a).  e = b - a and w = p - a are formed as sums with
  // coefficients in {-1, 0, 1} (exact products, zeros added exactly: the
  // same bits as the differences) rather than by picking points with a
  // run-time index, which would put the points in scratch memory.
  double ce[4], cw[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ce[i] = (i == sb) ? 1.0 : (i == sa) ? -1.0 : 0.0;
    cw[i] = (i == sp) ? 1.0 : (i == sa) ? -1.0 : 0.0;
  }
  d3 e = {0.0, 0.0, 0.0}, w = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    e.x += ce[i] * P[i].x;
    e.y += ce[i] * P[i].y;
    e.z += ce[i] * P[i].z;
    w.x += cw[i] * P[i].x;
    w.y += cw[i] * P[i].y;
    w.z += cw[i] * P[i].z;
  }
  double s = dot3(w, e) / dot3(e, e);
  T.nb = 1;
  T.n_involved = 3;
  T.involved[0] = sp;
  T.involved[1] = sa;
  T.involved[2] = sb;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T.c[i] = (i == sp) ? 1.0 : (i == sa) ? -(1.0 - s) : (i == sb) ? -s : 0.0;
    T.dc[0][i] = (i == sa) ? 1.0 : (i == sb) ? -1.0 : 0.0;
  }
}

// z = d^2, gz[12], Hz[144] (row-major, zero outside the involved slots).
DEV void d2_derivs(const double *x, const TypeGeo &T, double *z, double *gz, double *Hz) {
  double r[3] = {0, 0, 0}, q[2][3] = {{0, 0, 0}, {0, 0, 0}};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 3; ++k) {
      r[k] += T.c[i] * x[3 * i + k];
      q[0][k] += T.dc[0][i] * x[3 * i + k];
      q[1][k] += T.dc[1][i] * x[3 * i + k];
    }
  *z = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 3; ++k) gz[3 * i + k] = 2.0 * T.c[i] * r[k];
  double Gi[2][2] = {{0, 0}, {0, 0}};
  if (T.nb == 1) {
    Gi[0][0] = 1.0 / (q[0][0] * q[0][0] + q[0][1] * q[0][1] + q[0][2] * q[0][2]);
  } else if (T.nb == 2) {
    double g00 = q[0][0] * q[0][0] + q[0][1] * q[0][1] + q[0][2] * q[0][2];
    double g01 = q[0][0] * q[1][0] + q[0][1] * q[1][1] + q[0][2] * q[1][2];
    double g11 = q[1][0] * q[1][0] + q[1][1] * q[1][1] + q[1][2] * q[1][2];
    double id = 1.0 / (g00 * g11 - g01 * g01);
    Gi[0][0] = g11 * id;
    Gi[1][1] = g00 * id;
    Gi[0][1] = Gi[1][0] = -g01 * id;
  }
  double u[4][2][3];
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 2; ++k)
      for (int m = 0; m < 3; ++m) u[i][k][m] = T.c[i] * q[k][m] + T.dc[k][i] * r[m];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double v = (a == b) ? 2.0 * T.c[i] * T.c[j] : 0.0;
          for (int k = 0; k < T.nb; ++k)
            for (int l = 0; l < T.nb; ++l) v -= 2.0 * Gi[k][l] * u[i][k][a] * u[j][l][b];
          Hz[(3 * i + a) * 12 + 3 * j + b] = v;
        }
}

// -- barrier ----------------------------------------------------------------
DEV void barrier_b(double d, double dhat, double *b0, double *b1, double *b2) {
  if (d >= dhat) {
    *b0 = *b1 = *b2 = 0.0;
    return;
  }
  double r = d - dhat, L = log(d / dhat);
  *b0 = -r * r * L;
  *b1 = -2.0 * r * L - r * r / d;
  *b2 = -2.0 * L - 4.0 * r / d + r * r / (d * d);
}

// c = |ea x eb|^2 and its derivatives in the 12 pair coordinates:
//   grad_ea c = 2 eb x n, grad_eb c = 2 n x ea;
//   Hess over (ea, eb) = 2 M^T M + [[0, -2[n]x], [2[n]x, 0]],  M = [-[eb]x, [ea]x].
DEV void cross_norm2_derivs(const double *x, double *c, double *gc, double *Hc) {
  d3 ea = sub3(ld3(x + 3), ld3(x)), eb = sub3(ld3(x + 9), ld3(x + 6));
  d3 n = cross3(ea, eb);
  *c = dot3(n, n);
  d3 ga = cross3(eb, n), gb = cross3(n, ea);
  double GA[3] = {2 * ga.x, 2 * ga.y, 2 * ga.z}, GB[3] = {2 * gb.x, 2 * gb.y, 2 * gb.z};
  for (int k = 0; k < 3; ++k) {
    gc[k] = -GA[k];
    gc[3 + k] = GA[k];
    gc[6 + k] = -GB[k];
    gc[9 + k] = GB[k];
  }
  // M = [-[eb]x, [ea]x] (3x6); [v]x w = v x w
  double EA[3] = {ea.x, ea.y, ea.z}, EB[3] = {eb.x, eb.y, eb.z}, N[3] = {n.x, n.y, n.z};
  double M[3][6];
  auto skew = [](const double *v, double S[3][3]) {
    S[0][0] = 0;
    S[0][1] = -v[2];
    S[0][2] = v[1];
    S[1][0] = v[2];
    S[1][1] = 0;
    S[1][2] = -v[0];
    S[2][0] = -v[1];
    S[2][1] = v[0];
    S[2][2] = 0;
  };
  double SA[3][3], SB[3][3], SN[3][3];
  skew(EA, SA);
  skew(EB, SB);
  skew(N, SN);
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      M[r][k] = -SB[r][k];
      M[r][3 + k] = SA[r][k];
    }
  double H6[6][6];
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      double s = 0.0;
      for (int r = 0; r < 3; ++r) s += M[r][a] * M[r][b];
      H6[a][b] = 2.0 * s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      H6[a][3 + b] += -2.0 * SN[a][b];
      H6[3 + a][b] += 2.0 * SN[a][b];
    }
  // map (ea, eb) -> (a0, a1, b0, b1): ea = a1 - a0, eb = b1 - b0
  const double sgn[4] = {-1.0, 1.0, -1.0, 1.0};
  const int grp[4] = {0, 0, 1, 1};
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          Hc[(3 * i + a) * 12 + 3 * j + b] = sgn[i] * sgn[j] * H6[3 * grp[i] + a][3 * grp[j] + b];
}

// -- PSD projection: cyclic Jacobi, negative eigenvalues clamped to 0 ----------
// A is n x n row-major with leading dimension ld; V is scratch of n*n.
DEV void psd_project(int n, double *A, int ld, double *V) {
  double fro = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) fro += A[i * ld + j] * A[i * ld + j];
  if (fro == 0.0) return;
  fro = sqrt(fro);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += 2.0 * A[i * ld + j] * A[i * ld + j];
    if (sqrt(off) <= 1e-15 * fro) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * ld + q];
        if (apq == 0.0) continue;
        double theta = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * ld + p], akq = A[k * ld + q];
          A[k * ld + p] = c * akp - s * akq;
          A[k * ld + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * ld + k], aqk = A[q * ld + k];
          A[p * ld + k] = c * apk - s * aqk;
          A[q * ld + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  double lam[12];
  for (int k = 0; k < n; ++k) lam[k] = fmax(A[k * ld + k], 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc += V[i * n + k] * lam[k] * V[j * n + k];
      A[i * ld + j] = acc;
      A[j * ld + i] = acc;
    }
}

// -- exact PSD projection of a barrier Hessian on its range -----------------------
// Without the mollifier, H = kappa (B2 gz gz^T + B1 Hz) with gz = 2 c (x) r and
// Hz = 2 (c c^T) (x) I - 2 sum Ginv_kl u_k u_l^T, u_k = c (x) q_k + dc_k (x) r.
// Writing dc_k = w_k + c (c.dc_k)/|c|^2 with w_k orthogonal to c gives
// u_k = c (x) (q_k + ...) + w_k (x) r, so range(H) lies in
//   span{ c (x) e_1, c (x) e_2, c (x) e_3, w_k (x) r }   (dimension 3 + nb <= 5).
// With Q an orthonormal basis of that span, Proj(H) = Q Proj(Q^T H Q) Q^T.
DEV bool subspace_project(const TypeGeo &T, const double *x, double *H) {
  double r[3] = {0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 3; ++k) r[k] += T.c[i] * x[3 * i + k];
  double cn2 = T.c[0] * T.c[0] + T.c[1] * T.c[1] + T.c[2] * T.c[2] + T.c[3] * T.c[3];
  double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(cn2 > 0.0) || !(rn > 0.0)) return false;
  double Q[5][12];
  int D = 0;
  double ci = 1.0 / sqrt(cn2);
  for (int m = 0; m < 3; ++m, ++D)
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 3; ++k) Q[D][3 * i + k] = (k == m) ? T.c[i] * ci : 0.0;
  double om[2][4];
  int nw = 0;
  for (int kk = 0; kk < T.nb; ++kk) {
    double w[4], cd = 0.0, dn = 0.0;
    for (int i = 0; i < 4; ++i) {
      cd += T.c[i] * T.dc[kk][i];
      dn += T.dc[kk][i] * T.dc[kk][i];
    }
    for (int i = 0; i < 4; ++i) w[i] = T.dc[kk][i] - T.c[i] * cd / cn2;
    for (int j = 0; j < nw; ++j) {
      double pr = 0.0;
      for (int i = 0; i < 4; ++i) pr += w[i] * om[j][i];
      for (int i = 0; i < 4; ++i) w[i] -= pr * om[j][i];
    }
    double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    if (!(wn > 1e-12 * sqrt(dn))) continue;
    for (int i = 0; i < 4; ++i) om[nw][i] = w[i] / wn;
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 3; ++k) Q[D][3 * i + k] = om[nw][i] * r[k] / rn;
    ++nw;
    ++D;
  }
  // M = Q^T H Q
  double HQ[12][5], M[25], V[25];
  for (int a = 0; a < 12; ++a)
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int b = 0; b < 12; ++b) s += H[a * 12 + b] * Q[j][b];
      HQ[a][j] = s;
    }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int a = 0; a < 12; ++a) s += Q[i][a] * HQ[a][j];
      M[i * D + j] = s;
    }
  for (int i = 0; i < D; ++i)  // symmetrise rounding
    for (int j = i + 1; j < D; ++j) M[i * D + j] = M[j * D + i] = 0.5 * (M[i * D + j] + M[j * D + i]);
  psd_project(D, M, D, V);
  for (int a = 0; a < 12; ++a)
    for (int b = a; b < 12; ++b) {
      double s = 0.0;
      for (int i = 0; i < D; ++i) {
        double t = 0.0;
        for (int j = 0; j < D; ++j) t += M[i * D + j] * Q[j][b];
        s += Q[i][a] * t;
      }
      H[a * 12 + b] = s;
      H[b * 12 + a] = s;
    }
  return true;
}

// -- pair barrier element ------------------------------------------------------
// Energy kappa * e(c) * b(d) with gradient and (optionally projected) Hessian.
// b as a function of z = d^2: db/dz = b'/(2d), d2b/dz2 = (b'' - b'/d) / (4 z).
// Returns the energy; H is 12x12 row-major.
DEV double pair_barrier_full(int kind, int type, const double *x, double dhat, double kappa, double eps_x,
                             bool project, double *g, double *H, double *scratch /*144*/) {
  TypeGeo T;
  type_geometry(kind, type, x, T);
  double z;
  d2_derivs(x, T, &z, g, H);
  double d = sqrt(z);
  double b0, b1, b2;
  barrier_b(d, dhat, &b0, &b1, &b2);
  double B1 = b1 / (2.0 * d);
  double B2 = (b2 - b1 / d) / (4.0 * z);
  // H <- B2 gz gz^T + B1 Hz ; g <- B1 gz   (H holds Hz, g holds gz on entry)
  for (int i = 0; i < 12; ++i)
    for (int j = 0; j < 12; ++j) H[i * 12 + j] = B2 * g[i] * g[j] + B1 * H[i * 12 + j];
  for (int i = 0; i < 12; ++i) g[i] *= B1;
  double e = 1.0;
  bool all4 = (T.n_involved == 4), mollified = false;
  if (kind == 1) {
    double c, gc[12];
    double *Hc = scratch;
    cross_norm2_derivs(x, &c, gc, Hc);
    if (c < eps_x) {
      double q = c / eps_x;
      e = q * (2.0 - q);
      double e1 = (2.0 / eps_x) * (1.0 - q), e2 = -2.0 / (eps_x * eps_x);
      // E = e b : H = e Hb + b (e2 gc gc^T + e1 Hc) + e1 (gc gb^T + gb gc^T)
      for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j)
          H[i * 12 + j] = e * H[i * 12 + j] + b0 * (e2 * gc[i] * gc[j] + e1 * Hc[i * 12 + j]) +
                          e1 * (gc[i] * g[j] + g[i] * gc[j]);
      for (int i = 0; i < 12; ++i) g[i] = e * g[i] + b0 * e1 * gc[i];
      all4 = true;
      mollified = true;
    }
  }
  for (int i = 0; i < 12; ++i) g[i] *= kappa;
  for (int i = 0; i < 144; ++i) H[i] *= kappa;
  if (project) {
    if (!mollified && subspace_project(T, x, H)) {
      // exact projection on the (3 + nb)-dimensional range, see above
    } else if (all4) {
      psd_project(12, H, 12, scratch);
    } else {
      // project on the involved coordinates only (the rest of H is zero)
      int n = 3 * T.n_involved;
      double *S = scratch, *V = scratch + 81;  // n <= 9 here
      int idx[9];
      for (int a = 0; a < T.n_involved; ++a)
        for (int k = 0; k < 3; ++k) idx[3 * a + k] = 3 * T.involved[a] + k;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) S[i * 9 + j] = H[idx[i] * 12 + idx[j]];
      psd_project(n, S, 9, V);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) H[idx[i] * 12 + idx[j]] = S[i * 9 + j];
    }
  }
  return kappa * e * b0;
}

// -- PSD projection of a fixed-size symmetric matrix ----------------------------
// The cyclic Jacobi of psd_project with the size known at compile time, so
// that A and V stay in registers (no per-lane scratch memory).
template <int N>
DEV void psd_project_n(double A[N * N], double V[N * N]) {
  double fro = 0.0;
#pragma unroll
  for (int i = 0; i < N * N; ++i) fro += A[i] * A[i];
  if (fro == 0.0) return;
  fro = sqrt(fro);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) V[i * N + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += 2.0 * A[i * N + j] * A[i * N + j];
    if (sqrt(off) <= 1e-15 * fro) break;
#pragma unroll
    for (int p = 0; p < N - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p * N + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * N + q] - A[p * N + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double akp = A[k * N + p], akq = A[k * N + q];
          A[k * N + p] = c * akp - s * akq;
          A[k * N + q] = s * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double apk = A[p * N + k], aqk = A[q * N + k];
          A[p * N + k] = c * apk - s * aqk;
          A[q * N + k] = s * apk + c * aqk;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double vkp = V[k * N + p], vkq = V[k * N + q];
          V[k * N + p] = c * vkp - s * vkq;
          V[k * N + q] = s * vkp + c * vkq;
        }
      }
  }
  double lam[N];
#pragma unroll
  for (int k = 0; k < N; ++k) lam[k] = fmax(A[k * N + k], 0.0);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += V[i * N + k] * lam[k] * V[j * N + k];
      A[i * N + j] = acc;
      A[j * N + i] = acc;
    }
}

// -- pair barrier element without the 12x12 matrix ---------------------------------
// The unmollified element (e = 1): H = kappa (B2 gz gz^T + B1 Hz) lies in the
// span of the orthonormal Q_m = c (x) e_m / |c| (m < 3) and
// Q_{3+j} = om_j (x) r / |r| (subspace_project), so its projection is
// Q Proj(M) Q^T with M = Q^T H Q, formed here from coordinates in that basis
// instead of from H:
//   c (x) v -> |c| v in coordinates 0..2;  w (x) r -> |r| (w . om_j) in
//   coordinate 3 + j, for w orthogonal to c;
//   gz = 2 c (x) r;  u_k = c (x) (q_k + (c . dc_k) / |c|^2 r) + w_k (x) r with
//   w_k = dc_k - c (c . dc_k) / |c|^2;
//   Hz = 2 sum_m (c (x) e_m)(c (x) e_m)^T - 2 sum_kl Ginv_kl u_k u_l^T.
// M is padded to 5 x 5 with zero rows and columns, which the Jacobi rotations
// leave alone.  The projected blocks are then
//   H[3a + r][3b + s] = sum_ij phi_a(r, i) P_ij phi_b(s, j),
//   phi_a(r, m) = c_a [r = m] / |c|,  phi_a(r, 3 + j) = om_j[a] r_r / |r|.
// Writes the gradient g[12] and the ten 3x3 blocks (a <= b, blk_index order)
// of the projected Hessian to blocks[90] and returns the energy; returns -1
// with nothing written for an edge-edge pair in its mollified range
// (|ea x eb|^2 < eps_x) or a degenerate pair (|c| or |r| zero), which
// pair_barrier_full handles.
DEV double pair_barrier_fast(int kind, int type, const double *x, double dhat, double kappa, double eps_x,
                             double *g, double *blocks) {
  if (kind == 1) {
    d3 n = cross3(sub3(ld3(x + 3), ld3(x)), sub3(ld3(x + 9), ld3(x + 6)));
    if (dot3(n, n) < eps_x) return -1.0;
  }
  TypeGeo T;
  type_geometry(kind, type, x, T);
  double r[3] = {0, 0, 0}, q[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      r[k] += T.c[i] * x[3 * i + k];
      q[0][k] += T.dc[0][i] * x[3 * i + k];
      q[1][k] += T.dc[1][i] * x[3 * i + k];
    }
  const double z = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double cn2 = T.c[0] * T.c[0] + T.c[1] * T.c[1] + T.c[2] * T.c[2] + T.c[3] * T.c[3];
  if (!(cn2 > 0.0) || !(z > 0.0)) return -1.0;
  const double d = sqrt(z), cn = sqrt(cn2);
  double b0, b1, b2;
  barrier_b(d, dhat, &b0, &b1, &b2);
  const double B1 = b1 / (2.0 * d), B2 = (b2 - b1 / d) / (4.0 * z);
  double Gi[2][2] = {{0, 0}, {0, 0}};
  if (T.nb == 1) {
    Gi[0][0] = 1.0 / (q[0][0] * q[0][0] + q[0][1] * q[0][1] + q[0][2] * q[0][2]);
  } else if (T.nb == 2) {
    const double g00 = q[0][0] * q[0][0] + q[0][1] * q[0][1] + q[0][2] * q[0][2];
    const double g01 = q[0][0] * q[1][0] + q[0][1] * q[1][1] + q[0][2] * q[1][2];
    const double g11 = q[1][0] * q[1][0] + q[1][1] * q[1][1] + q[1][2] * q[1][2];
    const double id = 1.0 / (g00 * g11 - g01 * g01);
    Gi[0][0] = g11 * id;
    Gi[1][1] = g00 * id;
    Gi[0][1] = Gi[1][0] = -g01 * id;
  }
  // w_k and their orthonormalisation om_j (Gram-Schmidt, as subspace_project)
  double w[2][4], om[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, cd[2] = {0, 0};
  int nw = 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    double dn = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      cd[k] += T.c[i] * T.dc[k][i];
      dn += T.dc[k][i] * T.dc[k][i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) w[k][i] = T.dc[k][i] - T.c[i] * cd[k] / cn2;
    if (k >= T.nb) continue;
    double o[4] = {w[k][0], w[k][1], w[k][2], w[k][3]};
    if (nw == 1) {
      const double pr = o[0] * om[0][0] + o[1] * om[0][1] + o[2] * om[0][2] + o[3] * om[0][3];
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] -= pr * om[0][i];
    }
    const double on = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2] + o[3] * o[3]);
    if (!(on > 1e-12 * sqrt(dn))) continue;
    if (nw == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) om[0][i] = o[i] / on;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) om[1][i] = o[i] / on;
    }
    ++nw;
  }
  // coordinates of gz and u_k
  double G5[5] = {2.0 * cn * r[0], 2.0 * cn * r[1], 2.0 * cn * r[2], 0.0, 0.0};
  double U[2][5];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int m = 0; m < 3; ++m) U[k][m] = cn * (q[k][m] + cd[k] / cn2 * r[m]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      U[k][3 + j] = d * (w[k][0] * om[j][0] + w[k][1] * om[j][1] + w[k][2] * om[j][2] + w[k][3] * om[j][3]);
  }
  double M[25], V[25];
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = i; j < 5; ++j) {
      double h = B2 * G5[i] * G5[j] + ((i == j && i < 3) ? B1 * 2.0 * cn2 : 0.0);
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int l = 0; l < 2; ++l) h -= B1 * 2.0 * Gi[k][l] * U[k][i] * U[l][j];
      M[i * 5 + j] = M[j * 5 + i] = kappa * h;
    }
  psd_project_n<5>(M, V);
  // blocks: for each b, T_b = P phi_b^T (5 x 3), then block (a, b) = phi_a T_b
  double ca[4], oa[2][4], rh[3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    ca[a] = T.c[a] / cn;
    oa[0][a] = om[0][a];
    oa[1][a] = om[1][a];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) rh[k] = r[k] / d;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double Tb[5][3];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int s2 = 0; s2 < 3; ++s2)
        Tb[i][s2] = M[i * 5 + s2] * ca[b] + (M[i * 5 + 3] * oa[0][b] + M[i * 5 + 4] * oa[1][b]) * rh[s2];
#pragma unroll
    for (int a = 0; a <= b; ++a) {
      double *B = blocks + 9 * (a * 4 - (a * (a - 1)) / 2 + (b - a));  // blk_index(a, b)
#pragma unroll
      for (int r2 = 0; r2 < 3; ++r2)
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2)
          B[3 * r2 + s2] = ca[a] * Tb[r2][s2] + (oa[0][a] * Tb[3][s2] + oa[1][a] * Tb[4][s2]) * rh[r2];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) g[3 * i + k] = kappa * (B1 * (2.0 * T.c[i] * r[k]));
  return kappa * b0;
}

// Energy only, from the classified squared distance.
DEV double pair_barrier_energy(int kind, const double *x, double d2, double dhat, double kappa, double eps_x) {
  double d = sqrt(d2);
  double b0, b1, b2;
  barrier_b(d, dhat, &b0, &b1, &b2);
  double e = 1.0;
  if (kind == 1) {
    d3 n = cross3(sub3(ld3(x + 3), ld3(x)), sub3(ld3(x + 9), ld3(x + 6)));
    double c = dot3(n, n);
    if (c < eps_x) {
      double q = c / eps_x;
      e = q * (2.0 - q);
    }
  }
  return kappa * e * b0;
}

// Closest-point weights of a classified pair: sum_i w_i x_i is the vector
// between the two closest points (first primitive minus second).
DEV void closest_weights(int kind, int type, const double *x, double *w) {
  TypeGeo T;
  type_geometry(kind, type, x, T);
  // r = sum c_i x_i is exactly that difference, up to orientation
  for (int i = 0; i < 4; ++i) w[i] = T.c[i];
}

// -- Neo-Hookean tetrahedron ---------------------------------------------------
// Psi = mu/2 (|F|^2 - 3) - mu ln J + lambda/2 ln^2 J,  F = Ds Dm^-1.
//   P = mu F + (lambda ln J - mu) F^-T
//   dP/dF[(i,j),(k,l)] = mu d_ik d_jl + (mu - lambda ln J) Finv^T_il Finv^T_kj + lambda Finv^T_ij Finv^T_kl
// Gradient wrt vertex a: V P d_a, with d_0 = -(sum of Dm^-1 rows), d_a = row a-1 of Dm^-1.
// Hessian block (a,b)_{k,m} = V sum_{j,l} d_a[j] d_b[l] dP/dF[(k,j),(m,l)], after PSD projection of dP/dF.
DEV bool nh_F(const double *x, const double *Dinv, double F[9]) {
  double Ds[9];
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) Ds[i * 3 + a] = x[3 * (a + 1) + i] - x[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[i * 3 + j] = Ds[i * 3] * Dinv[j] + Ds[i * 3 + 1] * Dinv[3 + j] + Ds[i * 3 + 2] * Dinv[6 + j];
  return true;
}

DEV double det33(const double *M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) + M[2] * (M[3] * M[7] - M[4] * M[6]);
}

// inverse transpose of a 3x3 (row-major); returns det
DEV double inv_T33(const double *F, double *FiT) {
  double J = det33(F);
  double iJ = 1.0 / J;
  // cofactor matrix / det = F^-T
  FiT[0] = (F[4] * F[8] - F[5] * F[7]) * iJ;
  FiT[1] = (F[5] * F[6] - F[3] * F[8]) * iJ;
  FiT[2] = (F[3] * F[7] - F[4] * F[6]) * iJ;
  FiT[3] = (F[2] * F[7] - F[1] * F[8]) * iJ;
  FiT[4] = (F[0] * F[8] - F[2] * F[6]) * iJ;
  FiT[5] = (F[1] * F[6] - F[0] * F[7]) * iJ;
  FiT[6] = (F[1] * F[5] - F[2] * F[4]) * iJ;
  FiT[7] = (F[2] * F[3] - F[0] * F[5]) * iJ;
  FiT[8] = (F[0] * F[4] - F[1] * F[3]) * iJ;
  return J;
}

DEV double nh_energy(const double *x, const double *Dinv, double vol, double mu, double la) {
  double F[9];
  nh_F(x, Dinv, F);
  double J = det33(F);
  if (!(J > 0.0)) return kInf;
  double tr = 0.0;
  for (int i = 0; i < 9; ++i) tr += F[i] * F[i];
  double lJ = log(J);
  return vol * (0.5 * mu * (tr - 3.0) - mu * lJ + 0.5 * la * lJ * lJ);
}

// Unique 3x3 blocks (a <= b) of a symmetric 12x12 element matrix, in the order
// (0,0),(0,1),(0,2),(0,3),(1,1),(1,2),(1,3),(2,2),(2,3),(3,3).
HD int blk_index(int a, int b) { return a * 4 - (a * (a - 1)) / 2 + (b - a); }

// One Jacobi rotation of a symmetric 3x3 A (row-major) in the (p, q) plane,
// accumulated into the columns of V (the rotation of psd_project).
template <int p, int q>
DEV void jacobi3_rot(double A[9], double V[9]) {
  const double apq = A[3 * p + q];
  if (apq == 0.0) return;
  const double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
  const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double akp = A[3 * k + p], akq = A[3 * k + q];
    A[3 * k + p] = c * akp - s * akq;
    A[3 * k + q] = s * akp + c * akq;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double apk = A[3 * p + k], aqk = A[3 * q + k];
    A[3 * p + k] = c * apk - s * aqk;
    A[3 * q + k] = s * apk + c * aqk;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vkp = V[3 * k + p], vkq = V[3 * k + q];
    V[3 * k + p] = c * vkp - s * vkq;
    V[3 * k + q] = s * vkp + c * vkq;
  }
}

// Eigen-decomposition of a symmetric 3x3 by cyclic Jacobi (fixed indices, so
// everything stays in registers): A ends diagonal with the eigenvalues, the
// columns of V are the eigenvectors.
DEV void jacobi3(double A[9], double V[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    const double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (!(off > 1e-34 * dia)) break;
    jacobi3_rot<0, 1>(A, V);
    jacobi3_rot<0, 2>(A, V);
    jacobi3_rot<1, 2>(A, V);
  }
}

// index of (r, c), r <= c, in the packed upper triangle of a symmetric 9x9
HD int tri9(int r, int c) { return r * 9 - (r * (r - 1)) / 2 + (c - r); }

// PSD projection of the Neo-Hookean dP/dF in closed form, packed upper
// triangle of the 9x9 (row-major (i,j),(k,l) indexing as in nh_element).
// dP/dF maps a 3x3 X to mu X + c1 G X^T G + la (G:X) G with G = F^-T and
// c1 = mu - la ln J.  With the singular value decomposition F = U diag(sig) V^T
// (U, V orthogonal, sig > 0 as J > 0), G = U diag(s) V^T with s = 1/sig, and for
// X = U Y V^T the image is U (mu Y + c1 S Y^T S + la (s . diag Y) S) V^T.  Hence
// the nine eigenpairs, all in closed form but one 3x3 block:
//   Y = (E_ab + E_ba)/sqrt2, a < b:  mu + c1 s_a s_b
//   Y = (E_ab - E_ba)/sqrt2, a < b:  mu - c1 s_a s_b
//   Y diagonal: the symmetric 3x3 block  mu I + c1 diag(s_a^2) + la s s^T.
// The projection sums the modes with their eigenvalues clamped at 0.
DEV void nh_dPdF_projected(const double F[9], double lJ, double mu, double la, double Hs[45]) {
  // right singular vectors and singular values from F^T F
  double C[9], V[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
  jacobi3(C, V);
  // left singular vectors: u_a = F v_a / |F v_a| for the two largest singular
  // values (the second orthogonalised against the first), the third
  // completing an orthonormal basis with the sign of F v_3
  double ev[3] = {C[0], C[4], C[8]}, v[3][3], u[3][3], sg[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) v[a][i] = V[3 * i + a];
  // descending order (fixed indices: the swaps stay in registers)
  auto order = [&](int p, int q) {
    if (ev[p] < ev[q]) {
      const double t = ev[p];
      ev[p] = ev[q];
      ev[q] = t;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double w = v[p][i];
        v[p][i] = v[q][i];
        v[q][i] = w;
      }
    }
  };
  order(0, 1);
  order(1, 2);
  order(0, 1);
  double Fv[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) Fv[a][i] = F[3 * i] * v[a][0] + F[3 * i + 1] * v[a][1] + F[3 * i + 2] * v[a][2];
  {
    double n0 = sqrt(Fv[0][0] * Fv[0][0] + Fv[0][1] * Fv[0][1] + Fv[0][2] * Fv[0][2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) u[0][i] = Fv[0][i] / n0;
    double d = u[0][0] * Fv[1][0] + u[0][1] * Fv[1][1] + u[0][2] * Fv[1][2];
    double w[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) w[i] = Fv[1][i] - d * u[0][i];
    double n1 = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
#pragma unroll
    for (int i = 0; i < 3; ++i) u[1][i] = w[i] / n1;
    double c3[3] = {u[0][1] * u[1][2] - u[0][2] * u[1][1], u[0][2] * u[1][0] - u[0][0] * u[1][2],
                    u[0][0] * u[1][1] - u[0][1] * u[1][0]};
    const double sgn = (c3[0] * Fv[2][0] + c3[1] * Fv[2][1] + c3[2] * Fv[2][2]) >= 0.0 ? 1.0 : -1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) u[2][i] = sgn * c3[i];
    // singular values as u_a . F v_a (more accurate for the small ones than
    // the square roots of the eigenvalues of F^T F)
    sg[0] = n0;
    sg[1] = n1;
    sg[2] = u[2][0] * Fv[2][0] + u[2][1] * Fv[2][1] + u[2][2] * Fv[2][2];
  }
  double sv[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) sv[a] = 1.0 / sg[a];
  const double c1 = mu - la * lJ;
#pragma unroll
  for (int k = 0; k < 45; ++k) Hs[k] = 0.0;
  // adds lam+ vec(Q) vec(Q)^T for Q = sum_m coef_m u_{a_m} v_{b_m}^T
  auto add_mode = [&](double lam, const double Q[9]) {
    if (!(lam > 0.0)) return;
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int c = r; c < 9; ++c) Hs[tri9(r, c)] += lam * Q[r] * Q[c];
  };
  // the diagonal block
  double A[9], Wd[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) A[3 * a + b] = (a == b ? mu + c1 * sv[a] * sv[a] : 0.0) + la * sv[a] * sv[b];
  jacobi3(A, Wd);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double Q[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Q[3 * i + j] = Wd[k] * u[0][i] * v[0][j] + Wd[3 + k] * u[1][i] * v[1][j] + Wd[6 + k] * u[2][i] * v[2][j];
    add_mode(A[4 * k], Q);
  }
  // twist and flip pairs
  const double r2 = 0.70710678118654752440;
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int a = pr == 2 ? 1 : 0, b = pr == 0 ? 1 : 2;
    double Qp[9], Qm[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double x1 = u[a][i] * v[b][j], x2 = u[b][i] * v[a][j];
        Qp[3 * i + j] = r2 * (x1 + x2);
        Qm[3 * i + j] = r2 * (x1 - x2);
      }
    add_mode(mu + c1 * sv[a] * sv[b], Qp);
    add_mode(mu - c1 * sv[a] * sv[b], Qm);
  }
}

// Returns false if J <= 0.  g[12]; blocks[90] (10 blocks x 9, row-major),
// from the projected dP/dF (nh_dPdF_projected).
DEV bool nh_element(const double *x, const double *Dinv, double vol, double mu, double la, double *energy, double *g,
                    double *blocks) {
  double F[9], FiT[9];
  nh_F(x, Dinv, F);
  double J = inv_T33(F, FiT);
  if (!(J > 0.0)) return false;
  double lJ = log(J);
  double tr = 0.0;
  for (int i = 0; i < 9; ++i) tr += F[i] * F[i];
  *energy = vol * (0.5 * mu * (tr - 3.0) - mu * lJ + 0.5 * la * lJ * lJ);
  double P[9];
  for (int i = 0; i < 9; ++i) P[i] = mu * F[i] + (la * lJ - mu) * FiT[i];
  double dvec[4][3];
  for (int j = 0; j < 3; ++j) {
    dvec[1][j] = Dinv[j];
    dvec[2][j] = Dinv[3 + j];
    dvec[3][j] = Dinv[6 + j];
    dvec[0][j] = -(Dinv[j] + Dinv[3 + j] + Dinv[6 + j]);
  }
  for (int a = 0; a < 4; ++a)
    for (int k = 0; k < 3; ++k)
      g[3 * a + k] = vol * (P[k * 3] * dvec[a][0] + P[k * 3 + 1] * dvec[a][1] + P[k * 3 + 2] * dvec[a][2]);
  if (!blocks) return true;
  double Hs[45];
  nh_dPdF_projected(F, lJ, mu, la, Hs);
  // block (a,b)_{k,m} = vol sum_{j,l} d_a[j] H[(k,j),(m,l)] d_b[l]
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      double *B = blocks + 9 * blk_index(a, b);
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            double t = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l) {
              const int r = k * 3 + j, c = m * 3 + l;
              t += Hs[r <= c ? tri9(r, c) : tri9(c, r)] * dvec[b][l];
            }
            s += dvec[a][j] * t;
          }
          B[k * 3 + m] = vol * s;
        }
    }
  return true;
}

// -- friction smoothing ----------------------------------------------------------
DEV double friction_f0(double y, double eps) {
  return (y < eps) ? (-y * y * y / (3.0 * eps * eps) + y * y / eps + eps / 3.0) : y;
}

// -- additive CCD ---------------------------------------------------------------
DEV double pair_distance(int kind, const double *x) {
  double d2;
  classify(kind, x, &d2);
  return sqrt(d2);
}

DEV double accd(int kind, const double *x, const double *p, double s) {
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
    nrm[i] = sqrt(s2);
  }
  double l = (kind == 0) ? nrm[0] + fmax(nrm[1], fmax(nrm[2], nrm[3])) : fmax(nrm[0], nrm[1]) + fmax(nrm[2], nrm[3]);
  if (l == 0.0) return 1.0;
  double d0 = pair_distance(kind, x);
  double t = 0.0, xt[12];
  for (int it = 0; it < 1000000; ++it) {
    for (int i = 0; i < 12; ++i) xt[i] = x[i] + t * pm[i];
    double d = pair_distance(kind, xt);
    if (t > 0.0 && d <= s * d0) return t;
    double tau = (1.0 - s) * d / l;
    if (t + tau >= 1.0) return 1.0;
    t += tau;
  }
  return t;
}

// -- inversion filter (the step-size filter of Sec. II-C that keeps every tet
//    inversion-free along the search line) ---------------------------------------
// Along x + t p the edge matrix of a tet is Ds(x) + t Ds(p), with columns
// a_c + t b_c (a_c = x_{c+1} - x_0, b_c = p_{c+1} - p_0).  Its determinant is
// multilinear in the columns, so det = c0 + c1 t + c2 t^2 + c3 t^3 with
//   c0 = [a0 a1 a2],  c1 = [b0 a1 a2] + [a0 b1 a2] + [a0 a1 b2],
//   c2 = [a0 b1 b2] + [b0 a1 b2] + [b0 b1 a2],  c3 = [b0 b1 b2],
// [u v w] = u . (v x w).  J = det Ds / det Dm has the same sign (det Dm > 0).
DEV void det_line_cubic(const double *x, const double *p, double c[4]) {
  d3 a[3], b[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = sub3(ld3(x + 3 * (k + 1)), ld3(x));
    b[k] = sub3(ld3(p + 3 * (k + 1)), ld3(p));
  }
  c[0] = dot3(a[0], cross3(a[1], a[2]));
  c[1] = dot3(b[0], cross3(a[1], a[2])) + dot3(a[0], cross3(b[1], a[2])) + dot3(a[0], cross3(a[1], b[2]));
  c[2] = dot3(a[0], cross3(b[1], b[2])) + dot3(b[0], cross3(a[1], b[2])) + dot3(b[0], cross3(b[1], a[2]));
  c[3] = dot3(b[0], cross3(b[1], b[2]));
}

DEV double cubic_eval(const double c[4], double t) { return c[0] + t * (c[1] + t * (c[2] + t * c[3])); }

// Smallest t in (0, tmax] with det <= 0, +inf if there is none (0 if det <= 0
// already at t = 0).  The real roots of the derivative c1 + 2 c2 t + 3 c3 t^2
// cut [0, tmax] into pieces on which the cubic is monotone; the first piece
// whose right end is not positive holds the root, which bisection brackets
// down to adjacent doubles (the returned end has det <= 0).
DEV double cubic_first_root(const double c[4], double tmax) {
  if (!(c[0] > 0.0)) return 0.0;
  double cut[4];
  int nc = 0;
  cut[nc++] = 0.0;
  const double qa = 3.0 * c[3], qb = 2.0 * c[2], qc = c[1];
  double r0 = -1.0, r1 = -1.0;
  if (qa != 0.0) {
    const double disc = qb * qb - 4.0 * qa * qc;
    if (disc >= 0.0) {
      const double sq = sqrt(disc);
      r0 = (-qb - sq) / (2.0 * qa);
      r1 = (-qb + sq) / (2.0 * qa);
      if (r1 < r0) {
        const double t = r0;
        r0 = r1;
        r1 = t;
      }
    }
  } else if (qb != 0.0) {
    r0 = -qc / qb;
  }
  if (r0 > 0.0 && r0 < tmax) cut[nc++] = r0;
  if (r1 > 0.0 && r1 < tmax && r1 > cut[nc - 1]) cut[nc++] = r1;
  cut[nc++] = tmax;
  for (int i = 0; i + 1 < nc; ++i) {
    double lo = cut[i], hi = cut[i + 1];
    if (cubic_eval(c, hi) > 0.0) continue;
    for (int it = 0; it < 128; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      if (cubic_eval(c, mid) > 0.0)
        lo = mid;
      else
        hi = mid;
    }
    return hi;
  }
  return kInf;
}

// the filter's step bound for one tet: min(1, 0.8 t*) (0.8: safety factor)
constexpr double kInvSafety = 0.8;
DEV double tet_inversion_bound(const double *x, const double *p) {
  double c[4];
  det_line_cubic(x, p, c);
  const double t = cubic_first_root(c, 1.0 / kInvSafety);
  return fmin(1.0, kInvSafety * t);
}

// -- grasp-quality metrics (Sec. IV-C): distance and solid angle of a triangle
//    seen from a point -----------------------------------------------------------
// Squared distance from p to the triangle (a, b, c) by the region of the
// closest point: the barycentric coordinates of p's projection decide whether
// the closest point is a vertex, a point on an edge, or interior.
DEV double point_tri_dist2(d3 p, d3 a, d3 b, d3 c) {
  const d3 ab = sub3(b, a), ac = sub3(c, a), ap = sub3(p, a);
  const double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
  auto n2 = [](d3 v) { return v.x * v.x + v.y * v.y + v.z * v.z; };
  auto at = [](d3 o, d3 e, double t) { return d3{o.x + t * e.x, o.y + t * e.y, o.z + t * e.z}; };
  if (d1 <= 0.0 && d2 <= 0.0) return n2(ap);  // vertex a
  const d3 bp = sub3(p, b);
  const double d3_ = dot3(ab, bp), d4 = dot3(ac, bp);
  if (d3_ >= 0.0 && d4 <= d3_) return n2(bp);  // vertex b
  const double vc = d1 * d4 - d3_ * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3_ <= 0.0) {  // edge ab
    const double t = d1 / (d1 - d3_);
    return n2(sub3(p, at(a, ab, t)));
  }
  const d3 cp = sub3(p, c);
  const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) return n2(cp);  // vertex c
  const double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {  // edge ac
    const double t = d2 / (d2 - d6);
    return n2(sub3(p, at(a, ac, t)));
  }
  const double va = d3_ * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3_) >= 0.0 && (d5 - d6) >= 0.0) {  // edge bc
    const d3 bc = sub3(c, b);
    const double t = (d4 - d3_) / ((d4 - d3_) + (d5 - d6));
    return n2(sub3(p, at(b, bc, t)));
  }
  const double den = 1.0 / (va + vb + vc);  // interior: project onto the plane
  const double v = vb * den, w = vc * den;
  const d3 q = {a.x + ab.x * v + ac.x * w, a.y + ab.y * v + ac.y * w, a.z + ab.z * v + ac.z * w};
  return n2(sub3(p, q));
}

// Signed solid angle of the oriented triangle (a, b, c) seen from p
// (Van Oosterom and Strackee, 1983); the sum over a closed outward surface is
// 4 pi inside and 0 outside.
DEV double tri_solid_angle(d3 p, d3 a, d3 b, d3 c) {
  const d3 u = sub3(a, p), v = sub3(b, p), w = sub3(c, p);
  const double lu = sqrt(dot3(u, u)), lv = sqrt(dot3(v, v)), lw = sqrt(dot3(w, w));
  const double num = dot3(u, cross3(v, w));
  const double den = lu * lv * lw + dot3(u, v) * lw + dot3(u, w) * lv + dot3(v, w) * lu;
  return 2.0 * atan2(num, den);
}

DEV void inv33(const double *M, double *R) {
  double det = det33(M);
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
}

}  // namespace ipcdev
