// Macromodel generation on the device (section II, section III), one element kind at a
// time, plus current recovery on the original scatterers (eq. JABE).
//
// For a kind with PEC surface S (RWG functions Lambda, N of them) inside the op's box
// S^ (RWG functions Lambda^, N^ of them; Buffa-Christiansen dual functions Lambda^' on
// its barycentric refinement; n the inward normal):
//   L-type blocks  G^(X,Y)_ab = -j k eta int int [f_a . g_b - k^-2 div f_a div' g_b] G,
//                  for (X, Y) = (E, J), (E, H^), (E^, J), (E^, H^)  (eq. Gm_EJ_1, Gm_EJ_2, G1, G2)
//   K-type blocks  G^(X,E^)_ab = < f_a, int grad G x Lambda^'_b dS' >  (eq. Gm_EJ_3, G3), with
//                  the principal value on S^ itself (faces in one plane give 0) plus D / 2
//   D_ab = < Lambda^_a, n x Lambda^'_b >                              (section IV)
// and then, by Gauss-Jordan elimination and complex GEMMs on the FP64 matrix cores,
//   [T | Y] = G^(E^,H^)^-1 [G^(E^,J) | G^(E^,E^)]                     (eq. Hdiscretized1)
//   [A | B] = [G^(E,J) | G^(E,E^)] - G^(E,H^) [T | Y]                  (eq. JM)
//   R = A^-1 B,  M = T R                                              (eq. JABE, eq. Tm1)
// M goes to the op as the kind's block (section III), R stays on the device for
// J = -R E^ on every element of the kind.
//
// Quadrature (the paper does not give one): the symmetric 7-point degree-5 rule on test
// and source triangles; the static part of the kernel (1/(4 pi R) for L, its gradient
// for K) is integrated in closed form over the source triangle (Wilton et al. 1984,
// Graglia 1993; the gradient's normal part is the triangle's signed solid angle, van
// Oosterom and Strackee 1983), the rest by the rule.  A K-type pair whose centroids are
// closer than 1.5 times the sum of the triangles' radii uses the rule on the four
// midpoint sub-triangles of both triangles.
//
// Work is organised per triangle pair (one thread each): for an L pair the nine
// products of the three local half-RWG functions on each side; for a K pair the two
// vectors U = int_T W, V = int_T W x r with W(r) = int_t grad G dS' (grad_r G is parallel
// to r - r', so grad G x (s r' - q) = grad G x (s r - q) and every dual-function piece
// (s r - q) / (2 A_t) contracts with U and V alone).  Assembly kernels then sum the pairs
// of each RWG function's two triangles (and of each dual function's pieces) in a fixed
// order, so the blocks are run-to-run identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/aimm.h"
#include "op.hpp"

namespace aimm {
namespace {

constexpr double kPiD = 3.14159265358979323846;

struct TriD {
  double v[9];    // vertices
  double n[3];    // unit normal (right hand of the vertex order)
  double area;
  double le[3];   // length of the edge opposite vertex i
  double cen[3];  // centroid
  double rad;     // largest centroid-to-vertex distance
};

// Radon's 7-point rule (barycentric points, weights summing to 1), and the same rule on
// the four midpoint sub-triangles (a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca).
struct Rules {
  double b7[7][3], w7[7];
  double b28[28][3], w28[28];
};
__constant__ Rules c_rules;

Rules make_rules() {
  Rules r{};
  const double s15 = std::sqrt(15.0);
  const double a1 = (9.0 - 2.0 * s15) / 21.0, c1 = (6.0 + s15) / 21.0;
  const double a2 = (9.0 + 2.0 * s15) / 21.0, c2 = (6.0 - s15) / 21.0;
  const double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, c1, c1}, {c1, a1, c1}, {c1, c1, a1},
                            {a2, c2, c2},             {c2, a2, c2}, {c2, c2, a2}};
  const double ws[7] = {9.0 / 40.0, (155.0 + s15) / 1200.0, (155.0 + s15) / 1200.0, (155.0 + s15) / 1200.0,
                        (155.0 - s15) / 1200.0, (155.0 - s15) / 1200.0, (155.0 - s15) / 1200.0};
  for (int q = 0; q < 7; ++q) {
    for (int i = 0; i < 3; ++i) r.b7[q][i] = pts[q][i];
    r.w7[q] = ws[q];
  }
  const double E[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double sub[4][3][3];
  for (int i = 0; i < 3; ++i) {
    const double ab = 0.5 * (E[0][i] + E[1][i]), bc = 0.5 * (E[1][i] + E[2][i]), ca = 0.5 * (E[2][i] + E[0][i]);
    const double s4[4][3] = {{E[0][i], ab, ca}, {ab, E[1][i], bc}, {ca, bc, E[2][i]}, {ab, bc, ca}};
    for (int m = 0; m < 4; ++m)
      for (int c = 0; c < 3; ++c) sub[m][c][i] = s4[m][c];
  }
  for (int m = 0; m < 4; ++m)
    for (int q = 0; q < 7; ++q) {
      for (int i = 0; i < 3; ++i)
        r.b28[7 * m + q][i] = pts[q][0] * sub[m][0][i] + pts[q][1] * sub[m][1][i] + pts[q][2] * sub[m][2][i];
      r.w28[7 * m + q] = ws[q] / 4.0;
    }
  return r;
}

__device__ __forceinline__ void bary_point(const TriD& t, const double* b, double* p) {
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = b[0] * t.v[c] + b[1] * t.v[3 + c] + b[2] * t.v[6 + c];
}

__device__ __forceinline__ double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// edge term int_edge dl / R = asinh(s+/r0) - asinh(s-/r0); 0 when r lies on the edge's line
// (every use multiplies it by a factor that vanishes there, or the case cannot occur)
__device__ __forceinline__ double edge_log(double sm, double sp, double r0, double le) {
  return r0 > 1e-14 * le ? asinh(sp / r0) - asinh(sm / r0) : 0.0;
}

// Closed forms over source triangle t at point r: I1 = int 1/R dS', Ivec = int r'/R dS'.
__device__ void static_potential(const double* r, const TriD& t, double& I1, double* Iv) {
  const double d = (r[0] - t.v[0]) * t.n[0] + (r[1] - t.v[1]) * t.n[1] + (r[2] - t.v[2]) * t.n[2];
  const double rho[3] = {r[0] - d * t.n[0], r[1] - d * t.n[1], r[2] - d * t.n[2]};
  const double ad = fabs(d);
  double s1 = 0.0, w[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double* va = t.v + 3 * i;
    const double* vb = t.v + 3 * ((i + 1) % 3);
    double e[3] = {vb[0] - va[0], vb[1] - va[1], vb[2] - va[2]};
    const double le = sqrt(dot3(e, e));
    const double lh[3] = {e[0] / le, e[1] / le, e[2] / le};
    const double uh[3] = {lh[1] * t.n[2] - lh[2] * t.n[1], lh[2] * t.n[0] - lh[0] * t.n[2],
                          lh[0] * t.n[1] - lh[1] * t.n[0]};
    const double a[3] = {va[0] - rho[0], va[1] - rho[1], va[2] - rho[2]};
    const double b[3] = {vb[0] - rho[0], vb[1] - rho[1], vb[2] - rho[2]};
    const double sm = dot3(a, lh), sp = dot3(b, lh), t0 = dot3(a, uh);
    const double r0sq = t0 * t0 + d * d;
    const double rp = sqrt(r0sq + sp * sp), rm = sqrt(r0sq + sm * sm);
    const double f = edge_log(sm, sp, sqrt(r0sq), le);
    s1 += t0 * f - ad * (atan2(t0 * sp, r0sq + ad * rp) - atan2(t0 * sm, r0sq + ad * rm));
    const double c = 0.5 * (r0sq * f + sp * rp - sm * rm);
#pragma unroll
    for (int x = 0; x < 3; ++x) w[x] += c * uh[x];
  }
  I1 = s1;
#pragma unroll
  for (int x = 0; x < 3; ++x) Iv[x] = w[x] + rho[x] * s1;
}

// (exp(-j k R) - 1) / (4 pi R) and its R -> 0 limit -j k / (4 pi)
__device__ __forceinline__ cplx<double> smooth_kernel(double R, double k) {
  if (!(R > 0.0)) return cmk<double>(0.0, -k / (4.0 * kPiD));
  double s, c;
  sincos(k * R, &s, &c);
  const double h = sin(0.5 * k * R);
  const double den = 4.0 * kPiD * R;
  (void)c;
  return cmk<double>(-2.0 * h * h / den, -s / den);
}

// d/dR of (exp(-j k R) - 1) / (4 pi R), divided by R:
// [1 - (1 + j k R) exp(-j k R)] / (4 pi R^3); series -k^2 / (8 pi R) + j k^3 / (12 pi) for small k R
__device__ __forceinline__ cplx<double> smooth_grad_over_R(double R, double k) {
  const double x = k * R;
  if (x < 1e-3) return cmk<double>(-k * k / (8.0 * kPiD * R), k * k * k / (12.0 * kPiD));
  double s, c;
  sincos(x, &s, &c);
  const double h = sin(0.5 * x);
  const double den = 4.0 * kPiD * R * R * R;
  return cmk<double>((2.0 * h * h - x * s) / den, (s - x * c) / den);
}

// grad_r int_t 1/R dS': signed solid angle times the normal, minus the edge terms
__device__ void static_gradient(const double* r, const TriD& t, double* g) {
  const double a[3] = {t.v[0] - r[0], t.v[1] - r[1], t.v[2] - r[2]};
  const double b[3] = {t.v[3] - r[0], t.v[4] - r[1], t.v[5] - r[2]};
  const double c[3] = {t.v[6] - r[0], t.v[7] - r[1], t.v[8] - r[2]};
  const double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b)), lc = sqrt(dot3(c, c));
  const double bxc[3] = {b[1] * c[2] - b[2] * c[1], b[2] * c[0] - b[0] * c[2], b[0] * c[1] - b[1] * c[0]};
  const double num = dot3(a, bxc);
  const double den = la * lb * lc + dot3(a, b) * lc + dot3(a, c) * lb + dot3(b, c) * la;
  const double om = 2.0 * atan2(num, den);
#pragma unroll
  for (int x = 0; x < 3; ++x) g[x] = om * t.n[x];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double* va = t.v + 3 * i;
    const double* vb = t.v + 3 * ((i + 1) % 3);
    const double e[3] = {vb[0] - va[0], vb[1] - va[1], vb[2] - va[2]};
    const double le = sqrt(dot3(e, e));
    const double lh[3] = {e[0] / le, e[1] / le, e[2] / le};
    const double uh[3] = {lh[1] * t.n[2] - lh[2] * t.n[1], lh[2] * t.n[0] - lh[0] * t.n[2],
                          lh[0] * t.n[1] - lh[1] * t.n[0]};
    const double ra[3] = {va[0] - r[0], va[1] - r[1], va[2] - r[2]};
    const double sm = dot3(ra, lh);
    const double sp = (vb[0] - r[0]) * lh[0] + (vb[1] - r[1]) * lh[1] + (vb[2] - r[2]) * lh[2];
    const double r0 = sqrt(fmax(dot3(ra, ra) - sm * sm, 0.0));
    const double f = edge_log(sm, sp, r0, le);
#pragma unroll
    for (int x = 0; x < 3; ++x) g[x] -= f * uh[x];
  }
}

// ---- L-type pairs ---------------------------------------------------------------------
// out[(i * nb + j) * 9 + 3 a + b] = (l_a l_b / (4 A_T A_t)) int int (r - p_a).(r' - p_b) G
//                                  - (l_a l_b / (A_T A_t k^2)) int int G
// for test triangle i (local edge a opposite vertex p_a) and source triangle j.
__global__ void __launch_bounds__(256) k_lpair(const TriD* __restrict__ ta, int na, const TriD* __restrict__ tb,
                                               int nb, double k, cplx<double>* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= nb || i >= na) return;
  const TriD T = ta[i];
  const TriD t = tb[j];
  double rs[7][3];
#pragma unroll
  for (int s = 0; s < 7; ++s) bary_point(t, c_rules.b7[s], rs[s]);
  cplx<double> S0 = cmk<double>(0, 0);
  cplx<double> P[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) P[a][b] = cmk<double>(0, 0);
  for (int q = 0; q < 7; ++q) {
    double r[3];
    bary_point(T, c_rules.b7[q], r);
    double I1, Iv[3];
    static_potential(r, t, I1, Iv);
    cplx<double> I0 = cmk<double>(I1 / (4.0 * kPiD), 0.0);
    cplx<double> J[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) J[x] = cmk<double>(Iv[x] / (4.0 * kPiD), 0.0);
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      const double dx = r[0] - rs[s][0], dy = r[1] - rs[s][1], dz = r[2] - rs[s][2];
      const cplx<double> g = cscale(smooth_kernel(sqrt(dx * dx + dy * dy + dz * dz), k), c_rules.w7[s] * t.area);
      I0 = cadd(I0, g);
#pragma unroll
      for (int x = 0; x < 3; ++x) cfmas(J[x], rs[s][x], g);
    }
    const double aw = c_rules.w7[q] * T.area;
    cfmas(S0, aw, I0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double dq[3] = {r[0] - T.v[3 * a], r[1] - T.v[3 * a + 1], r[2] - T.v[3 * a + 2]};
      cplx<double> dJ = cmk<double>(0, 0);
#pragma unroll
      for (int x = 0; x < 3; ++x) cfmas(dJ, dq[x], J[x]);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double dp = dq[0] * t.v[3 * b] + dq[1] * t.v[3 * b + 1] + dq[2] * t.v[3 * b + 2];
        cfmas(P[a][b], aw, csub(dJ, cscale(I0, dp)));
      }
    }
  }
  cplx<double>* o = out + (int64_t(i) * nb + j) * 9;
  const double inv = 1.0 / (T.area * t.area);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double ll = T.le[a] * t.le[b] * inv;
      o[3 * a + b] = csub(cscale(P[a][b], 0.25 * ll), cscale(S0, ll / (k * k)));
    }
}

struct RwgD {
  int tp, tm;   // triangles
  int ep, em;   // local edge index (opposite the free vertex) in tp and tm
  double len;
  double pp[3], pm[3];  // free vertices
};

// out[a + b * ld] = -j k eta sum over the two triangles of a and of b of the signed pair values
__global__ void k_lassemble(const cplx<double>* __restrict__ V, int nbt, const RwgD* __restrict__ ra, int Na,
                            const RwgD* __restrict__ rb, int Nb, double keta, cplx<double>* __restrict__ out,
                            int64_t ld) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (a >= Na || b >= Nb) return;
  const RwgD A = ra[a], B = rb[b];
  const int TA[2] = {A.tp, A.tm}, EA[2] = {A.ep, A.em};
  const int TB[2] = {B.tp, B.tm}, EB[2] = {B.ep, B.em};
  cplx<double> s = cmk<double>(0, 0);
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const cplx<double> val = V[(int64_t(TA[u]) * nbt + TB[v]) * 9 + 3 * EA[u] + EB[v]];
      s = (u == v) ? cadd(s, val) : csub(s, val);
    }
  // -j k eta (x + j y) = k eta y - j k eta x
  out[a + int64_t(b) * ld] = cmk<double>(keta * s.im, -keta * s.re);
}

// ---- K-type pairs ---------------------------------------------------------------------
// out[(i * nb + j) * 6 + 0..2] = U = int_T W dS, [3..5] = V = int_T W x r dS,
// W(r) = int_t grad_r G dS' (closed-form static part plus the rule on the remainder).
__global__ void __launch_bounds__(128) k_kpair(const TriD* __restrict__ ta, int na, const TriD* __restrict__ tb,
                                               int nb, double k, int skip_coplanar, cplx<double>* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= nb || i >= na) return;
  const TriD T = ta[i];
  const TriD t = tb[j];
  cplx<double> U[3], V[3];
#pragma unroll
  for (int x = 0; x < 3; ++x) U[x] = V[x] = cmk<double>(0, 0);
  cplx<double>* o = out + (int64_t(i) * nb + j) * 6;
  if (skip_coplanar) {
    double dmax = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      dmax = fmax(dmax, fabs((T.v[3 * c] - t.v[0]) * t.n[0] + (T.v[3 * c + 1] - t.v[1]) * t.n[1] +
                             (T.v[3 * c + 2] - t.v[2]) * t.n[2]));
    if (dmax < 1e-12 && fabs(dot3(T.n, t.n)) > 1.0 - 1e-12) {
#pragma unroll
      for (int x = 0; x < 6; ++x) o[x] = cmk<double>(0, 0);
      return;
    }
  }
  const double dc[3] = {T.cen[0] - t.cen[0], T.cen[1] - t.cen[1], T.cen[2] - t.cen[2]};
  const bool near = sqrt(dot3(dc, dc)) < 1.5 * (T.rad + t.rad);
  const int nq = near ? 28 : 7;
  const double* bq = near ? &c_rules.b28[0][0] : &c_rules.b7[0][0];
  const double* wq = near ? c_rules.w28 : c_rules.w7;
  for (int q = 0; q < nq; ++q) {
    double r[3];
    bary_point(T, bq + 3 * q, r);
    double g[3];
    static_gradient(r, t, g);
    cplx<double> W[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) W[x] = cmk<double>(g[x] / (4.0 * kPiD), 0.0);
    for (int s = 0; s < nq; ++s) {
      double rs[3];
      bary_point(t, bq + 3 * s, rs);
      const double d[3] = {r[0] - rs[0], r[1] - rs[1], r[2] - rs[2]};
      const double R = sqrt(dot3(d, d));
      const cplx<double> h = cscale(smooth_grad_over_R(R, k), wq[s] * t.area);
#pragma unroll
      for (int x = 0; x < 3; ++x) cfmas(W[x], d[x], h);
    }
    const double aw = wq[q] * T.area;
#pragma unroll
    for (int x = 0; x < 3; ++x) cfmas(U[x], aw, W[x]);
    // W x r
    cfmas(V[0], aw, csub(cscale(W[1], r[2]), cscale(W[2], r[1])));
    cfmas(V[1], aw, csub(cscale(W[2], r[0]), cscale(W[0], r[2])));
    cfmas(V[2], aw, csub(cscale(W[0], r[1]), cscale(W[1], r[0])));
  }
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    o[x] = U[x];
    o[3 + x] = V[x];
  }
}

// out[a + b * ld] = sum over the two triangles T of test RWG a and the pieces (t, s, q) of dual
// function b of  sigma l_a / (2 A_T) [-s p . V + q . V + q . (p x U)]  (s, q already / (2 A_t))
__global__ void k_kassemble(const cplx<double>* __restrict__ UV, int nbt, const RwgD* __restrict__ ra, int Na,
                            const int* __restrict__ bptr, const int* __restrict__ btri,
                            const double* __restrict__ bsq, int Nb, const double* __restrict__ tri_area,
                            cplx<double>* __restrict__ out, int64_t ld) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (a >= Na || b >= Nb) return;
  const RwgD A = ra[a];
  cplx<double> acc = cmk<double>(0, 0);
  for (int u = 0; u < 2; ++u) {
    const int T = u == 0 ? A.tp : A.tm;
    const double* p = u == 0 ? A.pp : A.pm;
    const double c = (u == 0 ? 1.0 : -1.0) * A.len / (2.0 * tri_area[T]);
    for (int e = bptr[b]; e < bptr[b + 1]; ++e) {
      const cplx<double>* w = UV + (int64_t(T) * nbt + btri[e]) * 6;
      const double s = bsq[4 * e], q[3] = {bsq[4 * e + 1], bsq[4 * e + 2], bsq[4 * e + 3]};
      cplx<double> val = cmk<double>(0, 0);
#pragma unroll
      for (int x = 0; x < 3; ++x) cfmas(val, q[x] - s * p[x], w[3 + x]);
      // q . (p x U)
      const double pxq[3] = {p[1] * q[2] - p[2] * q[1], p[2] * q[0] - p[0] * q[2], p[0] * q[1] - p[1] * q[0]};
      // q . (p x U) = U . (q x p) = -U . (p x q)
#pragma unroll
      for (int x = 0; x < 3; ++x) cfmas(val, -pxq[x], w[x]);
      cfmas(acc, c, val);
    }
  }
  out[a + int64_t(b) * ld] = acc;
}

// out[a + b * ld] += scale * D[a + b * N] (D real, column-major)
__global__ void k_add_real(cplx<double>* __restrict__ out, int64_t ld, const double* __restrict__ D, int N,
                           double scale) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (a >= N) return;
  out[a + int64_t(b) * ld].re += scale * D[a + int64_t(b) * N];
}

// ---- Gauss-Jordan elimination with partial pivoting ------------------------------------
// On the n x ncol column-major system [A | B] (ld >= n): step k picks the largest |a_ik|
// (i >= k, first one on ties), swaps rows k and p over columns k.., scales row k past
// column k by 1 / a_kk, and k_gj_elim removes column k from every other row past column
// k.  After n steps columns n.. hold A^-1 B.
__global__ void __launch_bounds__(256) k_gj_pivot(cplx<double>* __restrict__ A, int64_t ld, int n, int ncol, int k,
                                                  int* __restrict__ info) {
  __shared__ double best[256];
  __shared__ int bidx[256];
  const int tid = threadIdx.x;
  double m = -1.0;
  int mi = n;
  for (int i = k + tid; i < n; i += 256) {
    const cplx<double> v = A[i + int64_t(k) * ld];
    const double a2 = v.re * v.re + v.im * v.im;
    if (a2 > m) {
      m = a2;
      mi = i;
    }
  }
  best[tid] = m;
  bidx[tid] = mi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      const double o = best[tid + off];
      const int oi = bidx[tid + off];
      if (o > best[tid] || (o == best[tid] && oi < bidx[tid])) {
        best[tid] = o;
        bidx[tid] = oi;
      }
    }
    __syncthreads();
  }
  const int p = bidx[0];
  if (!(best[0] > 0.0)) {
    if (tid == 0 && *info == 0) *info = k + 1;
    return;
  }
  const cplx<double> piv = A[p + int64_t(k) * ld];
  const double d2 = piv.re * piv.re + piv.im * piv.im;
  const cplx<double> inv = cmk<double>(piv.re / d2, -piv.im / d2);
  __syncthreads();
  for (int j = k + tid; j < ncol; j += 256) {
    cplx<double>* ck = A + int64_t(j) * ld;
    cplx<double> vk = ck[k], vp = ck[p];
    if (p != k) {
      ck[p] = vk;
      vk = vp;
    }
    ck[k] = j > k ? cmul(vk, inv) : vk;
  }
}

__global__ void __launch_bounds__(256) k_gj_elim(cplx<double>* __restrict__ A, int64_t ld, int n, int ncol, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i == k) return;
  const cplx<double> m = A[i + int64_t(k) * ld];
  const int j0 = k + 1 + blockIdx.y * 8;
  const int j1 = min(j0 + 8, ncol);
  for (int j = j0; j < j1; ++j) {
    cplx<double>* c = A + int64_t(j) * ld;
    c[i] = csub(c[i], cmul(m, c[k]));
  }
}

// ---- complex FP64 GEMM on the matrix cores ---------------------------------------------
// C = alpha A B + beta C, A (M x K, column-major, lda), B (K x N), C (M x N); column j of
// B and of C starts at boff[j] / coff[j] elements when given, else at j * ldb / j * ldc.
// 32 x 32 tiles, four waves of 16 x 16, K chunks of 16 staged in LDS; four real
// v_mfma_f64_16x16x4f64 per complex step (A lane l holds A[l % 16][l / 16], B lane l
// holds B[l / 16][l % 16]; output register r of lane l is row l / 16 + 4 r, column l % 16).
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct ZgemmArgs {
  int M, N, K;
  double alpha, beta;
  const cplx<double>* A;
  int64_t lda;
  const cplx<double>* B;
  int64_t ldb;
  const int64_t* boff;
  cplx<double>* C;
  int64_t ldc;
  const int64_t* coff;
};

__global__ void __launch_bounds__(256) k_zgemm(ZgemmArgs g) {
  __shared__ cplx<double> As[32][17];
  __shared__ cplx<double> Bs[32][17];  // Bs[col][k]
  const int m0 = blockIdx.x * 32, n0 = blockIdx.y * 32;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  f64x4 accR = {0, 0, 0, 0}, accI = {0, 0, 0, 0};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    for (int e = threadIdx.x; e < 32 * 16; e += 256) {
      const int r = e & 31, kk = e >> 5;
      const int row = m0 + r, kg = k0 + kk;
      As[r][kk] = (row < g.M && kg < g.K) ? g.A[row + int64_t(kg) * g.lda] : cmk<double>(0, 0);
      const int c = e >> 4, kb = e & 15;
      const int col = n0 + c, kgb = k0 + kb;
      cplx<double> bv = cmk<double>(0, 0);
      if (col < g.N && kgb < g.K) {
        const int64_t base = g.boff ? g.boff[col] : int64_t(col) * g.ldb;
        bv = g.B[base + kgb];
      }
      Bs[c][kb] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const cplx<double> av = As[wm * 16 + li][kk + lk];
      const cplx<double> bv = Bs[wn * 16 + li][kk + lk];
      accR = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.re, accR, 0, 0, 0);
      accR = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.im, bv.im, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.im, accI, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f64_16x16x4f64(av.im, bv.re, accI, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = m0 + wm * 16 + lk + 4 * q, col = n0 + wn * 16 + li;
    if (row < g.M && col < g.N) {
      const int64_t base = g.coff ? g.coff[col] : int64_t(col) * g.ldc;
      cplx<double>* c = g.C + base + row;
      cplx<double> v = cmk<double>(g.alpha * accR[q], g.alpha * accI[q]);
      if (g.beta != 0.0) v = cadd(v, cscale(*c, g.beta));
      *c = v;
    }
  }
}

hipError_t zgemm(const ZgemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zgemm, dim3((g.M + 31) / 32, (g.N + 31) / 32), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---- host: geometry, dual functions and D ---------------------------------------------

struct P3 {
  double x, y, z;
};
inline P3 operator-(P3 a, P3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline P3 operator+(P3 a, P3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline P3 operator*(double s, P3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double pdot(P3 a, P3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline P3 pcross(P3 a, P3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

TriD make_trid(P3 a, P3 b, P3 c) {
  TriD t{};
  const P3 v[3] = {a, b, c};
  for (int i = 0; i < 3; ++i) {
    t.v[3 * i] = v[i].x;
    t.v[3 * i + 1] = v[i].y;
    t.v[3 * i + 2] = v[i].z;
  }
  const P3 cr = pcross(b - a, c - a);
  const double n2 = std::sqrt(pdot(cr, cr));
  t.area = 0.5 * n2;
  t.n[0] = cr.x / n2;
  t.n[1] = cr.y / n2;
  t.n[2] = cr.z / n2;
  for (int i = 0; i < 3; ++i) {
    const P3 e = v[(i + 2) % 3] - v[(i + 1) % 3];
    t.le[i] = std::sqrt(pdot(e, e));
  }
  const P3 ce = (1.0 / 3.0) * (a + b + c);
  t.cen[0] = ce.x;
  t.cen[1] = ce.y;
  t.cen[2] = ce.z;
  t.rad = 0.0;
  for (int i = 0; i < 3; ++i) t.rad = std::max(t.rad, std::sqrt(pdot(v[i] - ce, v[i] - ce)));
  return t;
}

struct HostMesh {
  std::vector<P3> vert;
  std::vector<int> tri;  // [n_tri][3]
  std::vector<int> rwg;  // [n_rwg][4]
  std::vector<TriD> tris;
  std::vector<RwgD> rwgs;
  int nt = 0, nr = 0;
};

HostMesh host_mesh(const double* vert, int n_vert, const int32_t* tri, int n_tri, const int32_t* rwg, int n_rwg) {
  HostMesh m;
  m.vert.resize(n_vert);
  for (int i = 0; i < n_vert; ++i) m.vert[i] = {vert[3 * i], vert[3 * i + 1], vert[3 * i + 2]};
  m.tri.assign(tri, tri + 3 * n_tri);
  m.rwg.assign(rwg, rwg + 4 * n_rwg);
  m.nt = n_tri;
  m.nr = n_rwg;
  for (int t = 0; t < n_tri; ++t) {
    for (int c = 0; c < 3; ++c)
      if (tri[3 * t + c] < 0 || tri[3 * t + c] >= n_vert) throw std::invalid_argument("triangle vertex out of range");
    m.tris.push_back(make_trid(m.vert[tri[3 * t]], m.vert[tri[3 * t + 1]], m.vert[tri[3 * t + 2]]));
    if (!(m.tris.back().area > 0.0)) throw std::invalid_argument("degenerate triangle in a scatterer mesh");
  }
  for (int n = 0; n < n_rwg; ++n) {
    const int va = rwg[4 * n], vb = rwg[4 * n + 1], tp = rwg[4 * n + 2], tm = rwg[4 * n + 3];
    if (tp < 0 || tp >= n_tri || tm < 0 || tm >= n_tri || tp == tm)
      throw std::invalid_argument("RWG triangle index out of range");
    RwgD r{};
    r.tp = tp;
    r.tm = tm;
    int idx[2] = {-1, -1};
    for (int u = 0; u < 2; ++u) {
      const int T = u == 0 ? tp : tm;
      int cnt = 0;
      for (int c = 0; c < 3; ++c) {
        const int v = tri[3 * T + c];
        if (v != va && v != vb) {
          idx[u] = c;
          ++cnt;
        }
      }
      if (cnt != 1) throw std::invalid_argument("an RWG triangle does not contain its edge");
    }
    r.ep = idx[0];
    r.em = idx[1];
    const P3 e = m.vert[vb] - m.vert[va];
    r.len = std::sqrt(pdot(e, e));
    const P3 pp = m.vert[tri[3 * tp + idx[0]]], pm = m.vert[tri[3 * tm + idx[1]]];
    r.pp[0] = pp.x;
    r.pp[1] = pp.y;
    r.pp[2] = pp.z;
    r.pm[0] = pm.x;
    r.pm[1] = pm.y;
    r.pm[2] = pm.z;
    m.rwgs.push_back(r);
  }
  return m;
}

// Buffa-Christiansen functions of a closed surface as pieces on its barycentric refinement.
// Refined triangles of coarse triangle T = (v0, v1, v2), barycentre b, midpoints m_ij:
// slot 0 (v0, m01, b), 1 (m01, v1, b), 2 (v1, m12, b), 3 (m12, v2, b), 4 (v2, m20, b), 5 (m20, v0, b).
// The function of edge e carries flux l_e from the cell of one end vertex to the other:
// half through each of the refined edges (m_e, b) of its two triangles, the rest around
// each end vertex so that every refined triangle of the cell gets charge l_e / (2 N_v).
struct Duals {
  std::vector<TriD> rtris;        // refined triangles
  std::vector<int> parent;        // coarse triangle of each
  std::vector<int> ptr, rt;       // pieces of dual function b: ptr[b] .. ptr[b+1]
  std::vector<double> s, q;       // s and q (3 per piece), unscaled
};

Duals build_duals(const HostMesh& m) {
  Duals D;
  std::map<std::pair<int, int>, int> mid;  // sorted vertex pair -> refined point
  std::vector<P3> pts(m.vert.begin(), m.vert.end());
  auto key = [](int a, int b) { return std::make_pair(std::min(a, b), std::max(a, b)); };
  std::map<std::pair<int, int>, std::vector<int>> edge_tris;
  for (int t = 0; t < m.nt; ++t)
    for (int c = 0; c < 3; ++c) {
      const int a = m.tri[3 * t + c], b = m.tri[3 * t + (c + 1) % 3];
      auto kk = key(a, b);
      if (!mid.count(kk)) {
        mid[kk] = int(pts.size());
        pts.push_back(0.5 * (m.vert[a] + m.vert[b]));
      }
      edge_tris[kk].push_back(t);
    }
  for (auto& e : edge_tris)
    if (e.second.size() != 2) throw std::invalid_argument("the equivalent surface is not closed");
  std::vector<int> bar(m.nt);
  for (int t = 0; t < m.nt; ++t) {
    bar[t] = int(pts.size());
    pts.push_back((1.0 / 3.0) * (m.vert[m.tri[3 * t]] + m.vert[m.tri[3 * t + 1]] + m.vert[m.tri[3 * t + 2]]));
  }
  // refined triangles, and the slot of (coarse triangle, corner vertex, edge at that corner)
  for (int t = 0; t < m.nt; ++t) {
    const int v0 = m.tri[3 * t], v1 = m.tri[3 * t + 1], v2 = m.tri[3 * t + 2];
    const int m01 = mid[key(v0, v1)], m12 = mid[key(v1, v2)], m20 = mid[key(v2, v0)];
    const int sl[6][2] = {{v0, m01}, {m01, v1}, {v1, m12}, {m12, v2}, {v2, m20}, {m20, v0}};
    for (int k = 0; k < 6; ++k) {
      D.rtris.push_back(make_trid(pts[sl[k][0]], pts[sl[k][1]], pts[bar[t]]));
      D.parent.push_back(t);
    }
  }
  auto slot = [&](int t, int v, std::pair<int, int> e) {
    const int v0 = m.tri[3 * t], v1 = m.tri[3 * t + 1], v2 = m.tri[3 * t + 2];
    if (v == v0) return e == key(v0, v1) ? 0 : 5;
    if (v == v1) return e == key(v0, v1) ? 1 : 2;
    return e == key(v1, v2) ? 3 : 4;
  };
  auto other_edge = [&](int t, int v, std::pair<int, int> e) {
    for (int c = 0; c < 3; ++c) {
      const int u = m.tri[3 * t + c];
      if (u != v && u != e.first && u != e.second) return key(u, v);
    }
    throw std::invalid_argument("degenerate triangle in the equivalent surface");
  };
  D.ptr.push_back(0);
  for (int n = 0; n < m.nr; ++n) {
    const int va = m.rwg[4 * n], vb = m.rwg[4 * n + 1], tp = m.rwg[4 * n + 2], tm = m.rwg[4 * n + 3];
    const auto e = key(va, vb);
    const P3 ev = m.vert[vb] - m.vert[va];
    const double le = std::sqrt(pdot(ev, ev));
    const P3 ehat = (1.0 / le) * ev;
    const TriD& Tp = m.tris[tp];
    const P3 n_in = {-Tp.n[0], -Tp.n[1], -Tp.n[2]};
    const P3 cp = {Tp.cen[0], Tp.cen[1], Tp.cen[2]};
    const P3 me = 0.5 * (m.vert[va] + m.vert[vb]);
    // n x Lambda' along Lambda^ (from T+ across the edge): the source cell is chosen so
    const int src = pdot(pcross(n_in, ehat), me - cp) > 0.0 ? va : vb;
    const int snk = src == va ? vb : va;
    std::map<int, std::pair<double, P3>> acc;  // refined triangle -> (s, q)
    for (int side = 0; side < 2; ++side) {
      const int v = side == 0 ? src : snk;
      const double sign = side == 0 ? 1.0 : -1.0;
      // fan around v from T+ (edge e) to T- (edge e): (coarse triangle, edge of its first
      // refined triangle, edge of its second)
      std::vector<std::pair<int, std::pair<int, int>>> chain;
      int t = tp;
      auto ed = e;
      for (int guard = 0;; ++guard) {
        if (guard > 4 * m.nt) throw std::invalid_argument("open fan around a vertex");
        const auto ed2 = other_edge(t, v, ed);
        chain.push_back({t, ed});
        chain.push_back({t, ed2});
        if (t == tm) {
          if (ed2 != e) throw std::invalid_argument("fan around a vertex does not close");
          break;
        }
        const auto& ts = edge_tris[ed2];
        t = ts[0] == t ? ts[1] : ts[0];
        ed = ed2;
      }
      const int n2 = int(chain.size()), N = n2 / 2;
      for (int k = 1; k <= n2; ++k) {
        const int T = chain[k - 1].first;
        const auto ek = chain[k - 1].second;
        const P3 pv = m.vert[v], pm = pts[mid[ek]], pb = pts[bar[T]];
        const int r = 6 * T + slot(T, v, ek);
        // outflows: odd k leaves to k+1 over (v, b) [opposite m] and came over (v, m)
        // [opposite b]; even k the reverse; the two ends also exit over (m_e, b) [opposite v]
        const P3 opp_next = (k % 2 == 1) ? pm : pb;
        const P3 opp_prev = (k % 2 == 1) ? pb : pm;
        double s = 0.0;
        P3 q = {0, 0, 0};
        if (k < n2) {
          const double f = -le * double(N - k) / (2.0 * N);
          s += f;
          q = q + f * opp_next;
        }
        if (k > 1) {
          const double f = le * double(N - k + 1) / (2.0 * N);
          s += f;
          q = q + f * opp_prev;
        }
        if (k == 1 || k == n2) {
          s += 0.5 * le;
          q = q + (0.5 * le) * pv;
        }
        auto& a = acc[r];
        a.first += sign * s;
        a.second = a.second + (sign * 1.0) * q;
      }
    }
    for (auto& kv : acc) {
      D.rt.push_back(kv.first);
      D.s.push_back(kv.second.first);
      D.q.push_back(kv.second.second.x);
      D.q.push_back(kv.second.second.y);
      D.q.push_back(kv.second.second.z);
    }
    D.ptr.push_back(int(D.rt.size()));
  }
  return D;
}

// D_ab = < Lambda^_a, n x Lambda^'_b >, n = inward normal; exact by the centroid of each
// refined triangle (the integrand is quadratic there).  Dense, column-major N x N.
std::vector<double> dual_gram(const HostMesh& m, const Duals& d) {
  const int N = m.nr;
  std::vector<double> D(size_t(N) * N, 0.0);
  std::vector<std::vector<int>> rwg_of(m.nt);
  for (int a = 0; a < N; ++a) {
    rwg_of[m.rwgs[a].tp].push_back(a);
    rwg_of[m.rwgs[a].tm].push_back(a);
  }
  for (int b = 0; b < N; ++b)
    for (int e = d.ptr[b]; e < d.ptr[b + 1]; ++e) {
      const TriD& t = d.rtris[d.rt[e]];
      const int T = d.parent[d.rt[e]];
      const TriD& Tc = m.tris[T];
      const P3 n_in = {-Tc.n[0], -Tc.n[1], -Tc.n[2]};
      const P3 c = {t.cen[0], t.cen[1], t.cen[2]};
      const P3 q = {d.q[3 * e], d.q[3 * e + 1], d.q[3 * e + 2]};
      const double s = d.s[e];
      for (int a : rwg_of[T]) {
        const RwgD& r = m.rwgs[a];
        const bool plus = r.tp == T;
        const P3 p = plus ? P3{r.pp[0], r.pp[1], r.pp[2]} : P3{r.pm[0], r.pm[1], r.pm[2]};
        const double val = -s * pdot(p, pcross(n_in, c)) + pdot(p - c, pcross(n_in, q));
        D[a + size_t(b) * N] += (plus ? 1.0 : -1.0) * r.len / (4.0 * Tc.area) * val;
      }
    }
  return D;
}

#define MM_HIP(expr)                                                                    \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      throw std::runtime_error(std::string("macromodel: ") + #expr + ": " + hipGetErrorString(_e)); \
  } while (0)

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  explicit DevBuf(size_t count) : n(count) {
    if (hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) throw std::bad_alloc();
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

template <typename T>
void to_dev(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) {
  MM_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

struct MeshDev {
  DevBuf<TriD> tris;
  DevBuf<RwgD> rwgs;
  DevBuf<double> area;
  MeshDev(const HostMesh& m, hipStream_t s) : tris(m.tris.size()), rwgs(m.rwgs.size()), area(m.tris.size()) {
    to_dev(tris, m.tris, s);
    to_dev(rwgs, m.rwgs, s);
    std::vector<double> a(m.tris.size());
    for (size_t i = 0; i < a.size(); ++i) a[i] = m.tris[i].area;
    to_dev(area, a, s);
    MM_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope with the caller
  }
};

void l_block(const HostMesh& ma, const MeshDev& da, const HostMesh& mb, const MeshDev& db, double k, double eta,
             cplx<double>* pairs, cplx<double>* out, int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(k_lpair, dim3((mb.nt + 255) / 256, ma.nt), dim3(256), 0, s, da.tris.p, ma.nt, db.tris.p,
                     mb.nt, k, pairs);
  MM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_lassemble, dim3((ma.nr + 255) / 256, mb.nr), dim3(256), 0, s, pairs, mb.nt, da.rwgs.p,
                     ma.nr, db.rwgs.p, mb.nr, k * eta, out, ld);
  MM_HIP(hipGetLastError());
}

void k_block(const HostMesh& ma, const MeshDev& da, int n_rt, const TriD* rtris, const int* bptr, const int* btri,
             const double* bsq, int nbf, double k, int skip_coplanar, cplx<double>* pairs, cplx<double>* out,
             int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(k_kpair, dim3((n_rt + 127) / 128, ma.nt), dim3(128), 0, s, da.tris.p, ma.nt, rtris, n_rt, k,
                     skip_coplanar, pairs);
  MM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_kassemble, dim3((ma.nr + 255) / 256, nbf), dim3(256), 0, s, pairs, n_rt, da.rwgs.p, ma.nr,
                     bptr, btri, bsq, nbf, da.area.p, out, ld);
  MM_HIP(hipGetLastError());
}

// In-place Gauss-Jordan on [A | B] (n x ncol, ld); throws on a zero pivot.
void gauss_jordan(cplx<double>* A, int64_t ld, int n, int ncol, int* info_dev, hipStream_t s) {
  MM_HIP(hipMemsetAsync(info_dev, 0, sizeof(int), s));
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(256), 0, s, A, ld, n, ncol, k, info_dev);
    const int cols = ncol - k - 1;
    if (cols > 0) hipLaunchKernelGGL(k_gj_elim, dim3((n + 255) / 256, (cols + 7) / 8), dim3(256), 0, s, A, ld, n, ncol, k);
  }
  MM_HIP(hipGetLastError());
  int info = 0;
  MM_HIP(hipMemcpyAsync(&info, info_dev, sizeof(int), hipMemcpyDeviceToHost, s));
  MM_HIP(hipStreamSynchronize(s));
  if (info != 0) throw std::invalid_argument("singular matrix in the macromodel elimination (step " +
                                             std::to_string(info) + "); the box may be at an interior resonance");
}

}  // namespace
}  // namespace aimm

using namespace aimm;

// Per-op storage of the generated recovery blocks and scatterer layout.
struct MacroStore {
  std::vector<int> n_scat;                 // RWG functions per kind
  std::vector<cplx<double>*> R;            // device [kind] N_t x N column-major
  std::vector<int64_t> elem_off;           // [n_elem + 1] scatterer unknown offsets
  std::vector<std::vector<cd>> M_host, R_host;
  std::vector<double> D_dense;
  aimm::DeviceMem mem;
};

namespace {
std::map<const aim_op*, MacroStore*>& stores() {
  static std::map<const aim_op*, MacroStore*> s;
  return s;
}
std::mutex g_store_mu;
}  // namespace

void aimm_release_macro_store(const aim_op* op) {
  std::lock_guard<std::mutex> lk(g_store_mu);
  auto it = stores().find(op);
  if (it != stores().end()) {
    delete it->second;
    stores().erase(it);
  }
}

void aimm_macro_store_elem_types(const aim_op* op) {
  std::lock_guard<std::mutex> lk(g_store_mu);
  auto it = stores().find(op);
  if (it == stores().end()) return;
  MacroStore* st = it->second;
  st->elem_off.assign(size_t(op->ne) + 1, 0);
  for (int e = 0; e < op->ne; ++e) st->elem_off[e + 1] = st->elem_off[e] + st->n_scat[op->elem_type[e]];
}

static MacroStore* store_of(const aim_op* op) {
  std::lock_guard<std::mutex> lk(g_store_mu);
  auto it = stores().find(op);
  return it == stores().end() ? nullptr : it->second;
}

extern "C" int aim_build_macromodels(aim_op* op, const aim_surface* scatterers, void* stream) {
  if (!op || !scatterers) {
    set_error("macromodels: op and scatterers must not be NULL");
    return AIM_EINVAL;
  }
  if (!op->device_ready) {
    set_error("macromodels: the op has no device data (host-only op)");
    return AIM_ESTATE;
  }
  if (op->d_set) {
    set_error("macromodels: D is already set on this op; build the macromodels on a fresh op");
    return AIM_ESTATE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nk = op->n_types, Nh = op->N;
  const double k = op->arr.k, eta = op->arr.eta;
  MacroStore* st = new MacroStore();
  try {
    {
      const Rules r = make_rules();  // this device's copy of the quadrature tables
      MM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rules), &r, sizeof(Rules)));
    }
    const HostMesh box = host_mesh(op->vert.data(), int(op->vert.size() / 3), op->tri.data(),
                                   int(op->tri.size() / 3), op->rwg.data(), int(op->rwg.size() / 4));
    const Duals du = build_duals(box);
    st->D_dense = dual_gram(box, du);
    std::vector<HostMesh> sc;
    for (int t = 0; t < nk; ++t) {
      const aim_surface& a = scatterers[t];
      if (a.n_vert < 3 || a.n_tri < 1 || a.n_rwg < 1 || !a.vert || !a.tri || !a.rwg)
        throw std::invalid_argument("macromodels: scatterer " + std::to_string(t) + " is empty");
      sc.push_back(host_mesh(a.vert, a.n_vert, a.tri, a.n_tri, a.rwg, a.n_rwg));
      st->n_scat.push_back(a.n_rwg);
    }
    const int n_rt = int(du.rtris.size());
    // device copies of the box, its refinement and the dual-function pieces (s, q / (2 A_t))
    MeshDev boxd(box, s);
    DevBuf<TriD> rtd(du.rtris.size());
    to_dev(rtd, du.rtris, s);
    DevBuf<int> bptr(du.ptr.size()), btri(du.rt.size());
    to_dev(bptr, du.ptr, s);
    to_dev(btri, du.rt, s);
    std::vector<double> sq(4 * du.rt.size());
    for (size_t e = 0; e < du.rt.size(); ++e) {
      const double inv = 1.0 / (2.0 * du.rtris[du.rt[e]].area);
      sq[4 * e] = du.s[e] * inv;
      for (int c = 0; c < 3; ++c) sq[4 * e + 1 + c] = du.q[3 * e + c] * inv;
    }
    DevBuf<double> bsq(sq.size());
    to_dev(bsq, sq, s);
    DevBuf<double> Dd(st->D_dense.size());
    to_dev(Dd, st->D_dense, s);
    DevBuf<int> info(1);
    std::vector<cd> Mall(size_t(nk) * Nh * Nh);
    for (int t = 0; t < nk; ++t) {
      const HostMesh& m = sc[t];
      const int N = m.nr;
      MeshDev md(m, s);
      // pair scratch: the largest of the L (9 values) and K (6 values) pair tables of this kind
      size_t pmax = 0;
      pmax = std::max(pmax, size_t(m.nt) * m.nt * 9);
      pmax = std::max(pmax, size_t(m.nt) * box.nt * 9);
      pmax = std::max(pmax, size_t(box.nt) * box.nt * 9);
      pmax = std::max(pmax, size_t(m.nt) * n_rt * 6);
      pmax = std::max(pmax, size_t(box.nt) * n_rt * 6);
      DevBuf<cplx<double>> pairs(pmax);
      // [G^(E^,H^) | G^(E^,J) | G^(E^,E^)]  (Nh x (Nh + N + Nh))
      const int c1 = Nh + N + Nh;
      DevBuf<cplx<double>> aug1(size_t(Nh) * c1);
      l_block(box, boxd, box, boxd, k, eta, pairs.p, aug1.p, Nh, s);
      l_block(box, boxd, m, md, k, eta, pairs.p, aug1.p + size_t(Nh) * Nh, Nh, s);
      k_block(box, boxd, n_rt, rtd.p, bptr.p, btri.p, bsq.p, Nh, k, 1, pairs.p, aug1.p + size_t(Nh) * (Nh + N), Nh,
              s);
      hipLaunchKernelGGL(k_add_real, dim3((Nh + 255) / 256, Nh), dim3(256), 0, s, aug1.p + size_t(Nh) * (Nh + N),
                         int64_t(Nh), Dd.p, Nh, 0.5);
      MM_HIP(hipGetLastError());
      // [G^(E,J) | G^(E,E^)]  (N x (N + Nh)) and G^(E,H^) (N x Nh)
      const int c2 = N + Nh;
      DevBuf<cplx<double>> aug2(size_t(N) * c2);
      DevBuf<cplx<double>> geh(size_t(N) * Nh);
      l_block(m, md, m, md, k, eta, pairs.p, aug2.p, N, s);
      k_block(m, md, n_rt, rtd.p, bptr.p, btri.p, bsq.p, Nh, k, 0, pairs.p, aug2.p + size_t(N) * N, N, s);
      l_block(m, md, box, boxd, k, eta, pairs.p, geh.p, N, s);
      // [T | Y] = G^(E^,H^)^-1 [G^(E^,J) | G^(E^,E^)]
      gauss_jordan(aug1.p, Nh, Nh, c1, info.p, s);
      // [A | B] -= G^(E,H^) [T | Y]
      ZgemmArgs g{};
      g.M = N;
      g.N = c2;
      g.K = Nh;
      g.alpha = -1.0;
      g.beta = 1.0;
      g.A = geh.p;
      g.lda = N;
      g.B = aug1.p + size_t(Nh) * Nh;
      g.ldb = Nh;
      g.C = aug2.p;
      g.ldc = N;
      MM_HIP(zgemm(g, s));
      // R = A^-1 B
      gauss_jordan(aug2.p, N, N, c2, info.p, s);
      // M = T R
      DevBuf<cplx<double>> Md(size_t(Nh) * Nh);
      ZgemmArgs h{};
      h.M = Nh;
      h.N = Nh;
      h.K = N;
      h.alpha = 1.0;
      h.beta = 0.0;
      h.A = aug1.p + size_t(Nh) * Nh;
      h.lda = Nh;
      h.B = aug2.p + size_t(N) * N;
      h.ldb = N;
      h.C = Md.p;
      h.ldc = Nh;
      MM_HIP(zgemm(h, s));
      cplx<double>* Rk = st->mem.alloc<cplx<double>>(size_t(N) * Nh);
      MM_HIP(hipMemcpyAsync(Rk, aug2.p + size_t(N) * N, size_t(N) * Nh * sizeof(cplx<double>),
                            hipMemcpyDeviceToDevice, s));
      st->R.push_back(Rk);
      std::vector<cplx<double>> mh(size_t(Nh) * Nh), rh(size_t(N) * Nh);
      MM_HIP(hipMemcpyAsync(mh.data(), Md.p, mh.size() * sizeof(cplx<double>), hipMemcpyDeviceToHost, s));
      MM_HIP(hipMemcpyAsync(rh.data(), Rk, rh.size() * sizeof(cplx<double>), hipMemcpyDeviceToHost, s));
      MM_HIP(hipStreamSynchronize(s));
      st->M_host.emplace_back(mh.size());
      st->R_host.emplace_back(rh.size());
      for (size_t e = 0; e < mh.size(); ++e) {
        st->M_host.back()[e] = cd(mh[e].re, mh[e].im);
        Mall[size_t(t) * Nh * Nh + e] = st->M_host.back()[e];
      }
      for (size_t e = 0; e < rh.size(); ++e) st->R_host.back()[e] = cd(rh[e].re, rh[e].im);
    }
    // scatterer unknown offsets, element-major
    st->elem_off.assign(size_t(op->ne) + 1, 0);
    for (int e = 0; e < op->ne; ++e) st->elem_off[e + 1] = st->elem_off[e] + st->n_scat[op->elem_type[e]];
    // hand M and D to the op through the public setters (device layouts and host copies)
    const int rc = aim_set_macromodels(op, reinterpret_cast<const double*>(Mall.data()));
    if (rc != AIM_OK) throw std::runtime_error(std::string("macromodels: ") + aim_last_error());
    std::vector<int32_t> rows, cols;
    std::vector<double> vals;
    for (int b = 0; b < Nh; ++b)
      for (int a = 0; a < Nh; ++a) {
        const double v = st->D_dense[a + size_t(b) * Nh];
        if (v != 0.0) {
          rows.push_back(a);
          cols.push_back(b);
          vals.push_back(v);
          vals.push_back(0.0);
        }
      }
    const int rd = aim_set_dmatrix(op, int64_t(rows.size()), rows.data(), cols.data(), vals.data());
    if (rd != AIM_OK) throw std::runtime_error(std::string("macromodels: ") + aim_last_error());
  } catch (const std::bad_alloc&) {
    delete st;
    set_error("macromodels: device allocation failed");
    return AIM_ENOMEM;
  } catch (const std::invalid_argument& e) {
    delete st;
    set_error(e.what());
    return AIM_EINVAL;
  } catch (const std::exception& e) {
    delete st;
    set_error(e.what());
    return AIM_EDEVICE;
  }
  aimm_release_macro_store(op);
  std::lock_guard<std::mutex> lk(g_store_mu);
  stores()[op] = st;
  return AIM_OK;
}

extern "C" int aim_get_macromodel(const aim_op* op, int32_t kind, double* M, double* R, double* D) {
  MacroStore* st = store_of(op);
  if (!op || !st) {
    set_error("macromodels: not generated on this op");
    return AIM_ESTATE;
  }
  if (kind < 0 || kind >= int(st->n_scat.size())) {
    set_error("macromodels: kind out of range");
    return AIM_EINVAL;
  }
  if (M) std::copy(st->M_host[kind].begin(), st->M_host[kind].end(), reinterpret_cast<cd*>(M));
  if (R) std::copy(st->R_host[kind].begin(), st->R_host[kind].end(), reinterpret_cast<cd*>(R));
  if (D) std::copy(st->D_dense.begin(), st->D_dense.end(), D);
  return AIM_OK;
}

extern "C" int64_t aim_scatterer_unknowns(const aim_op* op, int32_t kind) {
  MacroStore* st = store_of(op);
  if (!op || !st) return -1;
  if (kind >= 0) return kind < int(st->n_scat.size()) ? st->n_scat[kind] : -1;
  return st->elem_off.back();
}

extern "C" int aim_recover_currents(aim_op* op, const void* x, void* J, int32_t nrhs, void* stream) {
  MacroStore* st = store_of(op);
  if (!op || !x || !J) {
    set_error("recover currents: op, x and J must not be NULL");
    return AIM_EINVAL;
  }
  if (!st) {
    set_error("recover currents: macromodels not generated on this op");
    return AIM_ESTATE;
  }
  if (nrhs < 1) {
    set_error("recover currents: nrhs must be >= 1");
    return AIM_EINVAL;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ne = op->ne, Nh = op->N;
  const int64_t ntot = st->elem_off.back();
  try {
    for (int t = 0; t < int(st->n_scat.size()); ++t) {
      std::vector<int64_t> bo, co;
      for (int r = 0; r < nrhs; ++r)
        for (int m = 0; m < ne; ++m)
          if (op->elem_type[m] == t) {
            bo.push_back((int64_t(r) * ne + m) * Nh);
            co.push_back(int64_t(r) * ntot + st->elem_off[m]);
          }
      if (bo.empty()) continue;
      DevBuf<int64_t> bd(bo.size()), cdv(co.size());
      to_dev(bd, bo, s);
      to_dev(cdv, co, s);
      ZgemmArgs g{};
      g.M = st->n_scat[t];
      g.N = int(bo.size());
      g.K = Nh;
      g.alpha = -1.0;
      g.beta = 0.0;
      g.A = st->R[t];
      g.lda = st->n_scat[t];
      g.B = static_cast<const cplx<double>*>(x);
      g.boff = bd.p;
      g.C = static_cast<cplx<double>*>(J);
      g.coff = cdv.p;
      MM_HIP(zgemm(g, s));
      MM_HIP(hipStreamSynchronize(s));  // the offset tables are freed on return
    }
  } catch (const std::bad_alloc&) {
    set_error("recover currents: device allocation failed");
    return AIM_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return AIM_EDEVICE;
  }
  return AIM_OK;
}
