// Restarted GMRES on the final system (section V, eq. finalsystem), one Krylov
// space per right-hand side, all right-hand sides advanced together.
//
// Per cycle: FP64 true residual r = b - A x (FP64 product; none from the zero
// start), v_0 = r / ||r||; then for j = 0 .. m-1: w = A v_j, classical Gram-Schmidt
// applied twice (CGS2, in the Gram-matrix form described below) with FP64 sums,
// v_{j+1} = w' / ||w'||, Givens rotations on the FP64 Hessenberg column; finally
// x += V y with y from the triangular least-squares system.  AIM_MIXED runs the
// products in complex FP32 and stores the basis in complex FP32; all dot products,
// norms, the Gram and Hessenberg matrices, rotations and x stay FP64.
// Reductions are split into fixed chunks summed in a fixed order, and no value
// mixes right-hand sides, so each solution is independent of the batch it ran in.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/aimm.h"
#include "op.hpp"

namespace aimm {

template <typename T>
int matvec_impl(aim_op* op, const cplx<T>* x, cplx<T>* y, int R, int flags, hipStream_t s, hipEvent_t* ev = nullptr);
template <typename T>
int precond_impl(aim_op* op, const cplx<T>* x, cplx<T>* y, int R, hipStream_t s);

namespace {
void drop_graphs(KrylovWork& K);


constexpr int kBS = 256;
constexpr int kE = 4;
constexpr int kChunk = kBS * kE;

template <typename T>
__device__ __forceinline__ cplx<double> up(cplx<T> v) {
  return cmk<double>(double(v.re), double(v.im));
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block sum of (a, b) pairs; result valid in thread 0
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    sh[2 * w] = a;
    sh[2 * w + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0;
    b = 0;
    for (int i = 0; i < kBS / 64; ++i) {
      a += sh[2 * i];
      b += sh[2 * i + 1];
    }
  }
}

constexpr int kIV = 4;  // basis vectors loaded together (independent loads in flight)
constexpr int kMaxRestart = 96;

// ---- one Arnoldi step in Gram form ------------------------------------------------
// The basis is stored unnormalised: u_{j+1} = w - V c holds the orthogonalised
// product itself and v_i = s_i u_i with s_i = 1 / ||u_i|| (kept in FP64, s_0 = 1).
// Classical Gram-Schmidt applied twice gives, with p = V^H w and the Gram matrix
// S = V^H V, the coefficients c = p + V^H (w - V p) = 2 p - S p; so one pass over the
// basis computes p and the new column of S (the dots of every v_i with v_j, the
// product's input), a small per-right-hand-side kernel forms c, and one more pass
// writes u_{j+1} = w - V c and the partial sums of its norm.  Every dot product and
// norm is summed in FP64 in a fixed order.

// v[u][e] = V_{min(i0+u, nv-1)}[r][base + e kBS + tid] (zero past n)
template <typename Tb>
__device__ __forceinline__ void load_batch(const cplx<Tb>* __restrict__ V, int i0, int nv, int r, int R, int64_t n,
                                           int64_t base, cplx<Tb> (&v)[kIV][kE]) {
#pragma unroll
  for (int u = 0; u < kIV; ++u) {
    const int i = min(i0 + u, nv - 1);
    const cplx<Tb>* vi = V + (int64_t(i) * R + r) * n;
#pragma unroll
    for (int e = 0; e < kE; ++e) {
      const int64_t k = base + e * kBS + threadIdx.x;
      v[u][e] = k < n ? vi[k] : cmk<Tb>(0, 0);
    }
  }
}

// Lane exchanges without the LDS crossbar.  fold32(a, b): lanes 0-31 receive
// a[l] + a[l + 32] and lanes 32-63 receive b[l - 32] + b[l]; fold16(a, b): in each
// 32-lane half, lanes with bit 4 clear receive a[l] + a[l + 16] and lanes with it set
// b[l - 16] + b[l].  v_permlane32_swap (v_permlane16_swap) exchanges the upper lanes
// (odd rows of 16) of its first operand with the lower lanes (even rows) of its second,
// so one swap of (a, b) leaves each lane holding both terms of its sum.  dpp<CTRL>: a
// DPP lane permutation on the vector ALU (row_mirror: lane l <-> 15 - l in each row of
// 16; row_half_mirror: l <-> 7 - l in each group of 8; quad permutations).
__device__ __forceinline__ double fold32(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double fold16(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
constexpr int kRowMirror = 0x140, kHalfMirror = 0x141, kQuadSwap2 = 0x4E, kQuadSwap1 = 0xB1;

// Sums of 8 values over the 64 lanes of a wave by recursive halving: at each of the
// first three steps a lane keeps half of its values and adds the partner's copy of
// them (partners differ in bit 5, then 4, then 3), so value q = 4 b5 + 2 b4 + b3 ends
// in the lanes whose bits 5..3 spell q; three more exchanges within each group of 8
// lanes finish the sum.  The summation order is fixed.
__device__ __forceinline__ double wave_sum8(double (&x)[8], int lane) {
  const bool b3 = lane & 8;
  double y[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) y[q] = fold32(x[q], x[q + 4]);
  double z[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) z[q] = fold16(y[q], y[q + 2]);
  double t;
  {
    const double send = b3 ? z[0] : z[1], keep = b3 ? z[1] : z[0];
    t = keep + dpp<kRowMirror>(send);
  }
  t += dpp<kHalfMirror>(t);
  t += dpp<kQuadSwap2>(t);
  t += dpp<kQuadSwap1>(t);
  return t;  // the sum of value lane >> 3
}

// x = thread partials, for basis vectors i0 and i0 + 1, of (re, im) conj(u_i) . a and
// (re, im) conj(u_i) . b.  Wave sums go to wsum[((kind * nv + i) * 4 + wave) * 2 + part],
// kind 0 for a, 1 for b.
__device__ __forceinline__ void store_pair_sums(double (&x)[8], int i0, int nv, double* wsum) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double t = wave_sum8(x, lane);
  const int q = lane >> 3, i = i0 + (q >> 2), kind = (q >> 1) & 1;
  if ((lane & 7) == 0 && i < nv) wsum[((kind * nv + i) * 4 + wave) * 2 + (q & 1)] = t;
}

__device__ __forceinline__ void pair_terms(cplx<double> v, cplx<double> a, cplx<double> b, double* x) {
  x[0] = v.re * a.re + v.im * a.im;
  x[1] = v.re * a.im - v.im * a.re;
  x[2] = v.re * b.re + v.im * b.im;
  x[3] = v.re * b.im - v.im * b.re;
}

// block sums of the wave partials, in wave order, into the chunk slots of part
__device__ __forceinline__ void store_dots(const double* wsum, double* __restrict__ part, int nvals, int r, int c,
                                           int nch) {
  __syncthreads();
  for (int i = threadIdx.x; i < nvals; i += blockDim.x) {
    double a = 0, b = 0;
    for (int q = 0; q < 4; ++q) {
      a += wsum[(i * 4 + q) * 2];
      b += wsum[(i * 4 + q) * 2 + 1];
    }
    part[((int64_t(r) * nvals + i) * nch + c) * 2] = a;
    part[((int64_t(r) * nvals + i) * nch + c) * 2 + 1] = b;
  }
}

// the product A v_j = s_j A u_j at element idx, from its FP32 or FP64 copy
__device__ __forceinline__ cplx<double> product_value(const cplx<float>* __restrict__ wlo,
                                                      const cplx<double>* __restrict__ w, int64_t idx, double s) {
  const cplx<double> a = wlo ? up(wlo[idx]) : w[idx];
  return cmk<double>(a.re * s, a.im * s);
}

// acc -= sum_{i < nv} u_i coef_i over this thread's elements, in order of i
template <typename Tb>
__device__ __forceinline__ void subtract_batched(const cplx<Tb>* __restrict__ V, const cplx<double>* __restrict__ cf,
                                                 cplx<double> (&acc)[kE], int nv, int r, int R, int64_t n,
                                                 int64_t base) {
  for (int i0 = 0; i0 < nv; i0 += kIV) {
    cplx<Tb> v[kIV][kE];
    load_batch(V, i0, nv, r, R, n, base, v);
#pragma unroll
    for (int u = 0; u < kIV; ++u) {
      if (i0 + u >= nv) break;
      const cplx<double> h = cf[i0 + u];
#pragma unroll
      for (int e = 0; e < kE; ++e) {
        const cplx<double> vv = up(v[u][e]);
        acc[e].re -= vv.re * h.re - vv.im * h.im;
        acc[e].im -= vv.re * h.im + vv.im * h.re;
      }
    }
  }
}

// Projection pass, any span: chunk partials (kChunk elements) of conj(u_i) . A v_j
// (values 0 .. nv-1) and conj(u_i) . u_j (values nv .. 2nv-1).
template <typename Tb>
__global__ void __launch_bounds__(kBS) k_proj(const cplx<Tb>* __restrict__ V, const cplx<float>* __restrict__ wlo,
                                              const cplx<double>* __restrict__ w, const double* __restrict__ sc,
                                              int ldsc, double* __restrict__ part, int64_t n, int nv, int R) {
  extern __shared__ double wsum[];  // [2 nv][4 waves][2]
  const int c = blockIdx.x, r = blockIdx.y, nch = gridDim.x;
  const int64_t base = int64_t(c) * kChunk;
  const double sj = sc[int64_t(r) * ldsc + nv - 1];
  const cplx<Tb>* uj = V + (int64_t(nv - 1) * R + r) * n;
  cplx<double> a[kE], b[kE];
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int64_t k = base + e * kBS + threadIdx.x;
    a[e] = k < n ? product_value(wlo, w, int64_t(r) * n + k, sj) : cmk<double>(0, 0);
    b[e] = k < n ? up(uj[k]) : cmk<double>(0, 0);
  }
  for (int i0 = 0; i0 < nv; i0 += kIV) {
    cplx<Tb> v[kIV][kE];
    load_batch(V, i0, nv, r, R, n, base, v);
#pragma unroll
    for (int h = 0; h < kIV; h += 2) {
      if (i0 + h < nv) {
        double x[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int e = 0; e < kE; ++e) {
            double t[4];
            pair_terms(up(v[h + u][e]), a[e], b[e], t);
#pragma unroll
            for (int q = 0; q < 4; ++q) x[4 * u + q] += t[q];
          }
        store_pair_sums(x, i0 + h, nv, wsum);
      }
    }
  }
  store_dots(wsum, part, 2 * nv, r, c, nch);
}

// Update pass, any span: u_{j+1} = A v_j - sum_i u_i cr_i, and chunk partials of its
// squared norm.
template <typename Tb>
__global__ void __launch_bounds__(kBS) k_next(const cplx<Tb>* __restrict__ V, const cplx<float>* __restrict__ wlo,
                                              const cplx<double>* __restrict__ w, const double* __restrict__ sc,
                                              int ldsc, const cplx<double>* __restrict__ cr, int ldc,
                                              cplx<Tb>* __restrict__ unext, double* __restrict__ part, int64_t n,
                                              int nv, int R) {
  __shared__ double sh[2 * kBS / 64];
  const int c = blockIdx.x, r = blockIdx.y, nch = gridDim.x;
  const int64_t base = int64_t(c) * kChunk;
  const double sj = sc[int64_t(r) * ldsc + nv - 1];
  cplx<double> acc[kE];
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int64_t k = base + e * kBS + threadIdx.x;
    acc[e] = k < n ? product_value(wlo, w, int64_t(r) * n + k, sj) : cmk<double>(0, 0);
  }
  subtract_batched(V, cr + int64_t(r) * ldc, acc, nv, r, R, n, base);
  double nn = 0, dummy = 0;
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int64_t k = base + e * kBS + threadIdx.x;
    if (k < n) {
      unext[int64_t(r) * n + k] = cmk<Tb>(Tb(acc[e].re), Tb(acc[e].im));
      nn += acc[e].re * acc[e].re + acc[e].im * acc[e].im;
    }
  }
  block_sum2(nn, dummy, sh);
  if (threadIdx.x == 0) part[int64_t(r) * nch + c] = nn;
}

// ---- register-resident variants: one element per thread, the thread's values of all
// nv <= NVB basis vectors loaded at once and kept in registers, so every load of a
// thread is in flight together.  Chunks are kBS elements.

// An empty asm that claims to modify v: the conversion of a held FP32 value to FP64
// cannot be hoisted above it, so the span stays in registers at its own width.
template <typename Tb>
__device__ __forceinline__ cplx<Tb> keep(cplx<Tb> v) {
  asm volatile("" : "+v"(v.re), "+v"(v.im));
  return v;
}

template <typename Tb, int NVB>
__device__ __forceinline__ void load_span(const cplx<Tb>* __restrict__ V, int nv, int r, int R, int64_t n, int64_t k,
                                          cplx<Tb> (&v)[NVB]) {
#pragma unroll
  for (int i = 0; i < NVB; ++i) v[i] = (i < nv && k < n) ? V[(int64_t(i) * R + r) * n + k] : cmk<Tb>(0, 0);
}

template <typename Tb, int NVB>
__global__ void __launch_bounds__(kBS) k_proj_span(const cplx<Tb>* __restrict__ V, const cplx<float>* __restrict__ wlo,
                                                   const cplx<double>* __restrict__ w, const double* __restrict__ sc,
                                                   int ldsc, double* __restrict__ part, int64_t n, int nv, int R) {
  static_assert(NVB % 2 == 0, "span");
  extern __shared__ double wsum[];  // [2 nv][4 waves][2]
  const int c = blockIdx.x, r = blockIdx.y, nch = gridDim.x;
  const int64_t k = int64_t(c) * kBS + threadIdx.x;
  cplx<Tb> v[NVB];
  load_span<Tb, NVB>(V, nv, r, R, n, k, v);
  const double sj = sc[int64_t(r) * ldsc + nv - 1];
  const cplx<double> a = k < n ? product_value(wlo, w, int64_t(r) * n + k, sj) : cmk<double>(0, 0);
  // u_j = v[nv - 1], picked without indexing the register array at run time
  cplx<Tb> ul = v[0];
#pragma unroll
  for (int i = 1; i < NVB; ++i)
    if (i == nv - 1) ul = v[i];
  const cplx<double> b = up(ul);
#pragma unroll
  for (int i0 = 0; i0 < NVB; i0 += 2) {
    if (i0 < nv) {
      double x[8];
      pair_terms(up(keep(v[i0])), a, b, x);
      pair_terms(up(keep(v[i0 + 1])), a, b, x + 4);
      store_pair_sums(x, i0, nv, wsum);
    }
  }
  store_dots(wsum, part, 2 * nv, r, c, nch);
}

// a -= sum_{i < nv} v_i cf_i, in order of i.  Slots i >= nv hold v_i = 0 and take the
// last coefficient, so they subtract exact zeros and the loop has no branches.
template <typename Tb, int NVB>
__device__ __forceinline__ void span_subtract(const cplx<Tb> (&v)[NVB], const cplx<double>* __restrict__ cf, int nv,
                                              cplx<double>& a) {
#pragma unroll
  for (int i = 0; i < NVB; ++i) {
    const cplx<double> h = cf[min(i, nv - 1)], vv = up(keep(v[i]));
    a.re -= vv.re * h.re - vv.im * h.im;
    a.im -= vv.re * h.im + vv.im * h.re;
  }
}

template <typename Tb, int NVB>
__global__ void __launch_bounds__(kBS) k_next_span(const cplx<Tb>* __restrict__ V, const cplx<float>* __restrict__ wlo,
                                                   const cplx<double>* __restrict__ w, const double* __restrict__ sc,
                                                   int ldsc, const cplx<double>* __restrict__ cr, int ldc,
                                                   cplx<Tb>* __restrict__ unext, double* __restrict__ part, int64_t n,
                                                   int nv, int R) {
  __shared__ double sh[2 * kBS / 64];
  const int c = blockIdx.x, r = blockIdx.y, nch = gridDim.x;
  const int64_t k = int64_t(c) * kBS + threadIdx.x;
  cplx<Tb> v[NVB];
  load_span<Tb, NVB>(V, nv, r, R, n, k, v);
  const double sj = sc[int64_t(r) * ldsc + nv - 1];
  cplx<double> a = k < n ? product_value(wlo, w, int64_t(r) * n + k, sj) : cmk<double>(0, 0);
  span_subtract<Tb, NVB>(v, cr + int64_t(r) * ldc, nv, a);
  double nn = 0, dummy = 0;
  if (k < n) {
    unext[int64_t(r) * n + k] = cmk<Tb>(Tb(a.re), Tb(a.im));
    nn = a.re * a.re + a.im * a.im;
  }
  block_sum2(nn, dummy, sh);
  if (threadIdx.x == 0) part[int64_t(r) * nch + c] = nn;
}

// Thread partial of sum_c p[c * stride] over c = tid, tid + kBS, ... (in that order),
// loads issued in batches of 16 so they are in flight together.
__device__ __forceinline__ void thread_partials(const double* __restrict__ p, int nch, int stride, double& a,
                                                double* b) {
  constexpr int kU = 16;
  for (int c0 = 0; c0 < nch; c0 += kU * kBS) {
    double va[kU], vb[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int c = min(c0 + u * kBS + int(threadIdx.x), nch - 1);
      va[u] = p[int64_t(c) * stride];
      if (b) vb[u] = p[int64_t(c) * stride + 1];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const bool in = c0 + u * kBS + int(threadIdx.x) < nch;
      a += in ? va[u] : 0.0;
      if (b) *b += in ? vb[u] : 0.0;
    }
  }
}

// h[r][i] (+)= sum_c part ; one block per (r, i), fixed summation order
__global__ void __launch_bounds__(kBS) k_reduce_dots(const double* __restrict__ part, cplx<double>* h, int nch, int nv,
                                                     int R, int ldh, int accumulate) {
  __shared__ double sh[2 * kBS / 64];
  const int t = blockIdx.x;
  if (t >= nv * R) return;
  const int r = t / nv, i = t - r * nv;
  const double* p = part + int64_t(t) * nch * 2;
  double a = 0, b = 0;
  thread_partials(p, nch, 2, a, &b);
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    cplx<double>& o = h[int64_t(r) * ldh + i];
    if (accumulate) {
      o.re += a;
      o.im += b;
    } else {
      o.re = a;
      o.im = b;
    }
  }
}

// Per right-hand side: p_i = s_i pq_i, new Gram column S_ij = s_i s_j pq_{nv+i}
// (i <= j), c = 2 p - S p.  hcol <- c (the Hessenberg column above the diagonal),
// cr <- s_i c_i (coefficients of the stored u_i).  S: [R][m+1][m+1] column-major,
// Hermitian, so (S p)_i = sum_k conj(S_ki) p_k reads column i contiguously; one wave
// per row i, lanes over k, a fixed-order lane sum.
__global__ void __launch_bounds__(kBS) k_gram(const cplx<double>* __restrict__ pq, int ldpq, cplx<double>* S,
                                              const double* __restrict__ sc, cplx<double>* __restrict__ hcol,
                                              cplx<double>* __restrict__ cr, int m, int j, int R) {
  __shared__ cplx<double> ps[kMaxRestart], qs[kMaxRestart];
  const int r = blockIdx.x;
  if (r >= R) return;
  const int nv = j + 1, ld = m + 1;
  const double* s = sc + int64_t(r) * ld;
  const double sj = s[j];
  cplx<double>* Sr = S + int64_t(r) * ld * ld;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    const cplx<double> pv = pq[int64_t(r) * ldpq + i], qv = pq[int64_t(r) * ldpq + nv + i];
    ps[i] = cmk<double>(pv.re * s[i], pv.im * s[i]);
    qs[i] = cmk<double>(qv.re * s[i] * sj, qv.im * s[i] * sj);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    Sr[i + int64_t(j) * ld] = qs[i];
    Sr[j + int64_t(i) * ld] = cmk<double>(qs[i].re, -qs[i].im);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = wave; i < nv; i += kBS / 64) {
    // S_ki for k < nv: column i of the stored matrix, except row j (conj q_i) and,
    // for i = j, the new column (q_k); both come from qs
    double a = 0, b = 0;
    for (int k0 = 0; k0 < nv; k0 += 64) {
      const int k = k0 + lane;
      if (k < nv) {
        cplx<double> ski;
        if (i == j)
          ski = qs[k];
        else if (k == j)
          ski = cmk<double>(qs[i].re, -qs[i].im);
        else
          ski = Sr[k + int64_t(i) * ld];
        // conj(S_ki) p_k
        a += ski.re * ps[k].re + ski.im * ps[k].im;
        b += ski.re * ps[k].im - ski.im * ps[k].re;
      }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      const cplx<double> cv = cmk<double>(2 * ps[i].re - a, 2 * ps[i].im - b);
      hcol[int64_t(r) * ld + i] = cv;
      cr[int64_t(r) * ld + i] = cmk<double>(cv.re * s[i], cv.im * s[i]);
    }
  }
}

// Per right-hand side, after the update pass: beta = ||u_{j+1}|| from the chunk
// partials (fixed order), s_{j+1} = 1 / beta, then the Givens step on column j:
//   H[r]: (m+1) x m column-major (ld m+1); hcol: the column above the diagonal;
//   scal[4r] <- beta, scal[4r+1] = stop threshold on |g|, scal[4r+2] = iteration
//   budget of this cycle; jused[r] = 0 while running, set to j+1 when the residual
//   estimate passes the threshold or the budget runs out, negative for right-hand
//   sides that are already finished.
// The rotations are staged in LDS and applied in order by one thread, carrying the
// running entry in registers.
__global__ void __launch_bounds__(kBS) k_finish_step(const double* __restrict__ part, int nch, double* sc,
                                                     double* scal, cplx<double>* H, cplx<double>* cs,
                                                     cplx<double>* sn, cplx<double>* g,
                                                     const cplx<double>* __restrict__ hcol, int* jused, int m, int j,
                                                     int R) {
  __shared__ double sh[2 * kBS / 64];
  __shared__ cplx<double> hc[kMaxRestart + 1], cc[kMaxRestart], ss[kMaxRestart];
  __shared__ double beta_s;
  const int r = blockIdx.x;
  if (r >= R) return;
  double sum = 0, dummy = 0;
  thread_partials(part + int64_t(r) * nch, nch, 1, sum, nullptr);
  block_sum2(sum, dummy, sh);
  if (threadIdx.x == 0) {
    const double beta = sqrt(sum);
    sc[int64_t(r) * (m + 1) + j + 1] = beta > 0 ? 1.0 / beta : 0.0;
    scal[4 * r] = beta;
    beta_s = beta;
  }
  __syncthreads();
  if (jused[r] != 0) return;
  cplx<double>* Hc = H + (int64_t(r) * m + j) * (m + 1);
  cplx<double>* c = cs + int64_t(r) * m;
  cplx<double>* s = sn + int64_t(r) * m;
  cplx<double>* gg = g + int64_t(r) * (m + 1);
  for (int i = threadIdx.x; i <= j; i += blockDim.x) {
    hc[i] = hcol[int64_t(r) * (m + 1) + i];
    if (i < j) {
      cc[i] = c[i];
      ss[i] = s[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    cplx<double> p = hc[0];
    for (int i = 0; i < j; ++i) {
      const cplx<double> q = hc[i + 1], ci = cc[i], si = ss[i];
      hc[i] = cadd(cmulc(p, ci), cmulc(q, si));  // conj(c) p + conj(s) q
      p = csub(cmul(ci, q), cmul(si, p));        // -s p + c q
    }
    const cplx<double> a = p, b = cmk<double>(beta_s, 0.0);
    const double den = sqrt(a.re * a.re + a.im * a.im + b.re * b.re + b.im * b.im);
    cplx<double> cj, sj;
    if (den > 0) {
      cj = cmk<double>(a.re / den, a.im / den);
      sj = cmk<double>(b.re / den, b.im / den);
    } else {
      cj = cmk<double>(1.0, 0.0);
      sj = cmk<double>(0.0, 0.0);
    }
    c[j] = cj;
    s[j] = sj;
    hc[j] = cmk<double>(den, 0.0);
    hc[j + 1] = cmk<double>(0.0, 0.0);
    const cplx<double> gj = gg[j];
    const cplx<double> gn = cmk<double>(-(sj.re * gj.re - sj.im * gj.im), -(sj.re * gj.im + sj.im * gj.re));
    gg[j + 1] = gn;
    gg[j] = cmulc(gj, cj);  // conj(c) g_j
    const double est = sqrt(gn.re * gn.re + gn.im * gn.im);
    if (est <= scal[4 * r + 1] || double(j + 1) >= scal[4 * r + 2]) jused[r] = j + 1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) Hc[i] = hc[i];
}

// chunk partials of ||a - b||^2 (b may be null) and of the difference into out
__global__ void __launch_bounds__(kBS) k_residual(const cplx<double>* __restrict__ a, const cplx<double>* __restrict__ b,
                                                  cplx<double>* __restrict__ out, double* part, int64_t n) {
  __shared__ double sh[2 * kBS / 64];
  const int c = blockIdx.x, r = blockIdx.y, nch = gridDim.x;
  const int64_t base = int64_t(c) * kChunk;
  double nn = 0, dummy = 0;
#pragma unroll
  for (int e = 0; e < kE; ++e) {
    const int64_t k = base + e * kBS + threadIdx.x;
    if (k >= n) continue;
    const int64_t idx = int64_t(r) * n + k;
    cplx<double> v = a[idx];
    if (b) v = csub(v, b[idx]);
    if (out) out[idx] = v;
    nn += v.re * v.re + v.im * v.im;
  }
  block_sum2(nn, dummy, sh);
  if (threadIdx.x == 0) part[int64_t(r) * nch + c] = nn;
}

// out[r] = sqrt(sum_c part[r][c]); one block per r, fixed summation order
__global__ void __launch_bounds__(kBS) k_finish_norm(const double* part, double* out, int nch, int R, int stride) {
  __shared__ double sh[2 * kBS / 64];
  const int r = blockIdx.x;
  if (r >= R) return;
  double s = 0, dummy = 0;
#pragma unroll 4
  for (int c = threadIdx.x; c < nch; c += kBS) s += part[int64_t(r) * nch + c];
  block_sum2(s, dummy, sh);
  if (threadIdx.x == 0) out[r * stride] = sqrt(s);
}

// v[r] = w[r] / nrm[r] (zero if nrm = 0), stored in the basis precision
template <typename Tb>
__global__ void k_scale(const cplx<double>* __restrict__ w, cplx<Tb>* __restrict__ v, const double* nrm, int stride,
                        int64_t n, int R) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * R) return;
  const int r = int(t / n);
  const double d = nrm[r * stride];
  const double s = d > 0 ? 1.0 / d : 0.0;
  v[t] = cmk<Tb>(Tb(w[t].re * s), Tb(w[t].im * s));
}

// y = H^-1 g on the leading k columns (back substitution); k = jused[r] if set,
// j_end if still running, 0 for finished right-hand sides.  One wave per right-hand
// side; the triangle is staged in LDS and each step's sum is a lane reduction.
__global__ void __launch_bounds__(64) k_lsq(const cplx<double>* H, const cplx<double>* g, cplx<double>* y,
                                            const int* jused, int m, int R, int j_end) {
  extern __shared__ cplx<double> Hs[];  // [m][m+1] column-major, then y[m+1]
  const int r = blockIdx.x;
  if (r >= R) return;
  const int k = jused[r] > 0 ? jused[r] : (jused[r] == 0 ? j_end : 0);
  const cplx<double>* Hr = H + int64_t(r) * m * (m + 1);
  cplx<double>* ys = Hs + m * (m + 1);
  for (int t = threadIdx.x; t < k * (m + 1); t += 64) Hs[t] = Hr[t];
  for (int t = threadIdx.x; t <= m; t += 64) ys[t] = cmk<double>(0, 0);
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    double a = 0, b = 0;
    for (int l = i + 1 + threadIdx.x; l < k; l += 64) {
      const cplx<double> p = cmul(Hs[l * (m + 1) + i], ys[l]);
      a += p.re;
      b += p.im;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (threadIdx.x == 0) {
      const cplx<double> gi = g[int64_t(r) * (m + 1) + i];
      const cplx<double> acc = cmk<double>(gi.re - a, gi.im - b);
      const cplx<double> d = Hs[i * (m + 1) + i];
      const double dd = d.re * d.re + d.im * d.im;
      ys[i] = dd > 0 ? cmk<double>((acc.re * d.re + acc.im * d.im) / dd, (acc.im * d.re - acc.re * d.im) / dd)
                     : cmk<double>(0, 0);
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t <= m; t += 64) y[int64_t(r) * (m + 1) + t] = ys[t];
}

// x[r] += sum_i v_i[r] y[r][i] = sum_i u_i[r] (s_i y_i)  (y is zero beyond the used columns)
template <typename Tb>
__global__ void k_update_x(const cplx<Tb>* __restrict__ V, cplx<double>* __restrict__ x,
                           const cplx<double>* __restrict__ y, const double* __restrict__ sc, int64_t n, int nv, int R,
                           int m) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * R) return;
  const int r = int(t / n);
  const int64_t k = t - int64_t(r) * n;
  cplx<double> acc = x[t];
  const cplx<double>* yr = y + int64_t(r) * (m + 1);
  const double* sr = sc + int64_t(r) * (m + 1);
  for (int i = 0; i < nv; ++i) {
    const cplx<double> yi = cmk<double>(yr[i].re * sr[i], yr[i].im * sr[i]);
    cfma(acc, up(V[(int64_t(i) * R + r) * n + k]), yi);
  }
  x[t] = acc;
}

__global__ void k_add(cplx<double>* __restrict__ x, const cplx<double>* __restrict__ d, int64_t n) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  cplx<double> v = x[t];
  v.re += d[t].re;
  v.im += d[t].im;
  x[t] = v;
}

inline unsigned nblk(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// largest Krylov span the register-resident passes hold (two VGPRs per FP32 value)
template <typename Tb>
constexpr int kSpanMax = sizeof(Tb) == sizeof(float) ? 64 : 32;

// pass 0: projections, 1: update; register-resident when the span fits
template <typename Tb, int NVB>
void launch_step_n(int pass, const cplx<Tb>* V, const cplx<float>* wlo, const cplx<double>* w, const double* sc,
                   int ldsc, const cplx<double>* cr, int ldc, cplx<Tb>* unext, double* part, int64_t n, int nv, int R,
                   hipStream_t s) {
  const dim3 g(nblk(n, kBS), R), b(kBS);
  if (pass == 0)
    hipLaunchKernelGGL((k_proj_span<Tb, NVB>), g, b, sizeof(double) * 16 * nv, s, V, wlo, w, sc, ldsc, part, n, nv,
                       R);
  else
    hipLaunchKernelGGL((k_next_span<Tb, NVB>), g, b, 0, s, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R);
}

// returns the number of chunk partials per right-hand side the pass wrote
template <typename Tb>
int launch_step(int pass, const cplx<Tb>* V, const cplx<float>* wlo, const cplx<double>* w, const double* sc, int ldsc,
                const cplx<double>* cr, int ldc, cplx<Tb>* unext, double* part, int64_t n, int nv, int R,
                hipStream_t s) {
  if (nv > kSpanMax<Tb>) {
    const dim3 g(nblk(n, kChunk), R), b(kBS);
    if (pass == 0)
      hipLaunchKernelGGL(k_proj<Tb>, g, b, sizeof(double) * 16 * nv, s, V, wlo, w, sc, ldsc, part, n, nv, R);
    else
      hipLaunchKernelGGL(k_next<Tb>, g, b, 0, s, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R);
    return int(g.x);
  }
  if (nv <= 8)
    launch_step_n<Tb, 8>(pass, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R, s);
  else if (nv <= 16)
    launch_step_n<Tb, 16>(pass, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R, s);
  else if (nv <= 24)
    launch_step_n<Tb, 24>(pass, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R, s);
  else if (nv <= 32 || kSpanMax<Tb> <= 32)
    launch_step_n<Tb, 32>(pass, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R, s);
  else if constexpr (kSpanMax<Tb> >= 64) {
    if (nv <= 40)
      launch_step_n<Tb, 40>(pass, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R, s);
    else if (nv <= 48)
      launch_step_n<Tb, 48>(pass, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R, s);
    else
      launch_step_n<Tb, 64>(pass, V, wlo, w, sc, ldsc, cr, ldc, unext, part, n, nv, R, s);
  }
  return int(nblk(n, kBS));
}

#define GM_HIP(expr)                                                              \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess) {                                                       \
      set_error(std::string("gmres: ") + #expr + ": " + hipGetErrorString(_e));  \
      return AIM_EDEVICE;                                                         \
    }                                                                             \
  } while (0)

#define GM_LAUNCH(...)                      \
  do {                                      \
    hipLaunchKernelGGL(__VA_ARGS__);        \
    GM_HIP(hipGetLastError());              \
  } while (0)

template <typename Tb>
int gmres_impl(aim_op* op, const cplx<double>* b, cplx<double>* x, int R, const gmres_opts& o, gmres_stat* st,
               hipStream_t s) {
  KrylovWork& K = op->kw;
  const int64_t n = int64_t(op->ne) * op->N;
  const int m = o.restart;
  const bool pre = o.precond == AIM_PRECOND_BLOCK_JACOBI;
  const int sys = o.system;  // AIM_FULL: the final system; AIM_G_ONLY: G x = b
  const int nch = int((n + kChunk - 1) / kChunk);
  const int nchs = int((n + kBS - 1) / kBS);  // chunks of the register-resident passes
  const dim3 gch(nch, R), bs(kBS), b64(64);
  cplx<Tb>* V = static_cast<cplx<Tb>*>(K.V);
  // ||b|| (and, for the zero start, the first residual r = b into K.r)
  GM_LAUNCH(k_residual, gch, bs, 0, s, b, (const cplx<double>*)nullptr, o.x0_given ? (cplx<double>*)nullptr : K.r,
            K.part, n);
  GM_LAUNCH(k_finish_norm, dim3(R), bs, 0, s, K.part, K.scal + 3, nch, R, 4);
  if (!o.x0_given) GM_HIP(hipMemsetAsync(x, 0, sizeof(cplx<double>) * n * R, s));
  // host sides of the small transfers live in pinned memory (K.h_*); the host writes a
  // staging array only after a stream synchronisation that follows its last transfer
  std::vector<double> bnorm(R), relres(R, 1.0);
  std::vector<int> active(R, 1), iters(R, 0), restarts(R, 0), matvecs(R, 0);
  double* hs = K.h_scal;
  int *jused = K.h_jused, *jinit = K.h_jinit;
  cplx<double>*g0 = K.h_g0, *gh = K.h_gh;
  double* ib0 = K.h_ib0;
  const size_t gl = size_t(R) * (m + 1);
  GM_HIP(hipMemcpyAsync(hs, K.scal, sizeof(double) * 4 * R, hipMemcpyDeviceToHost, s));
  GM_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < R; ++r) bnorm[r] = hs[4 * r + 3];
  for (size_t i = 0; i < gl; ++i) {
    g0[i] = cplx<double>{0.0, 0.0};
    ib0[i] = 0.0;
  }
  for (int r = 0; r < R; ++r) ib0[size_t(r) * (m + 1)] = 1.0;  // s_0 = 1: v_0 is stored normalised
  const int check = std::max(1, o.check_every);
  // Host checks of the stop flags: a check costs a round trip, a late one costs the
  // iterations run past convergence.  Each check extrapolates every running residual
  // estimate geometrically from the previous check and places the next check where
  // the slowest is predicted to pass its threshold (at most check_every ahead).
  // The first check of a later cycle is placed from the rate the previous cycle
  // reached (its restart usually sits just above the threshold).
  std::vector<double> est_prev(R), rate_last(R, 0.0);
  std::vector<int> j_prev(R);
  bool x_zero = !o.x0_given;
  // the launches of inner iteration j: (preconditioner,) product, two Gram-Schmidt passes
  // with their reductions, and the Hessenberg / Givens step; no host synchronisation
  auto inner = [&](int j, hipStream_t s) -> int {
    const cplx<Tb>* uj = V + int64_t(j) * R * n;
    cplx<Tb>* unext = V + int64_t(j + 1) * R * n;
    const int nv = j + 1;
    const cplx<float>* wlo = nullptr;
    int irc;
    if (pre) {
      // right preconditioning: the product acts on z = P v_j (the residual buffer is free in a cycle)
      irc = precond_impl<Tb>(op, uj, reinterpret_cast<cplx<Tb>*>(K.r), R, s);
      if (irc) return irc;
      uj = reinterpret_cast<const cplx<Tb>*>(K.r);
    }
    if (sizeof(Tb) == sizeof(double)) {
      irc = matvec_impl<double>(op, reinterpret_cast<const cplx<double>*>(uj), K.w, R, sys, s);
      if (irc) return irc;
    } else {
      irc = matvec_impl<float>(op, reinterpret_cast<const cplx<float>*>(uj), static_cast<cplx<float>*>(K.ylow), R,
                               sys, s);
      if (irc) return irc;
      wlo = static_cast<const cplx<float>*>(K.ylow);
    }
    // classical Gram-Schmidt twice, in Gram form
    int np = launch_step<Tb>(0, V, wlo, K.w, K.ib, m + 1, nullptr, 0, nullptr, K.part, n, nv, R, s);
    GM_HIP(hipGetLastError());
    GM_LAUNCH(k_reduce_dots, dim3(2 * nv * R), bs, 0, s, K.part, K.pq, np, 2 * nv, R, 2 * (m + 1), 0);
    GM_LAUNCH(k_gram, dim3(R), bs, 0, s, K.pq, 2 * (m + 1), K.S, K.ib, K.hcol, K.cr, m, j, R);
    np = launch_step<Tb>(1, V, wlo, K.w, K.ib, m + 1, K.cr, m + 1, unext, K.part, n, nv, R, s);
    GM_HIP(hipGetLastError());
    GM_LAUNCH(k_finish_step, dim3(R), bs, 0, s, K.part, np, K.ib, K.scal, K.H, K.cs, K.sn, K.g, K.hcol, K.active, m,
              j, R);
    return AIM_OK;
  };
  const bool use_graphs = o.graphs != 0;
  if (K.graph_epoch != op->graph_epoch) {
    drop_graphs(K);
    K.graph_epoch = op->graph_epoch;
  }
  const int graph_key = (m << 4) | (sys << 1) | int(pre);
  // the launches of iteration j, captured as a graph or kernel by kernel
  auto launch_iter = [&](int j) -> int {
    if (!use_graphs) return inner(j, s);
    // one captured graph per iteration index: replays the same launches with no
    // per-kernel host overhead (captured on first use, replayed in later cycles and solves)
    std::vector<hipGraphExec_t>& gv = K.graphs[graph_key];
    if (gv.size() < size_t(m)) gv.resize(size_t(m), nullptr);
    if (!gv[j]) {
      if (!K.cap) GM_HIP(hipStreamCreateWithFlags(&K.cap, hipStreamNonBlocking));
      GM_HIP(hipStreamBeginCapture(K.cap, hipStreamCaptureModeThreadLocal));
      const int crc = inner(j, K.cap);
      hipGraph_t graph = nullptr;
      const hipError_t ce = hipStreamEndCapture(K.cap, &graph);
      if (crc) {
        if (graph) (void)hipGraphDestroy(graph);
        return crc;
      }
      GM_HIP(ce);
      const hipError_t ie = hipGraphInstantiate(&gv[j], graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      GM_HIP(ie);
    }
    GM_HIP(hipGraphLaunch(gv[j], s));
    return AIM_OK;
  };
  for (;;) {
    // FP64 true residual r = b - A x; for the zero start r = b is already in K.r and its
    // norm on the host
    int rc = AIM_OK;
    if (x_zero) {
      for (int r = 0; r < R; ++r) hs[4 * r] = bnorm[r];
    } else {
      rc = matvec_impl<double>(op, x, K.w, R, sys, s);
      if (rc) return rc;
      GM_LAUNCH(k_residual, gch, bs, 0, s, b, K.w, K.r, K.part, n);
      GM_LAUNCH(k_finish_norm, dim3(R), bs, 0, s, K.part, K.scal, nch, R, 4);
      GM_HIP(hipMemcpyAsync(hs, K.scal, sizeof(double) * 4 * R, hipMemcpyDeviceToHost, s));
      GM_HIP(hipStreamSynchronize(s));
    }
    bool any = false;
    int budget_max = 0;
    for (int r = 0; r < R; ++r) {
      if (!active[r]) continue;
      if (!x_zero) matvecs[r] += 1;
      relres[r] = bnorm[r] > 0 ? hs[4 * r] / bnorm[r] : 0.0;
      if (relres[r] <= o.tol || iters[r] >= o.max_iters) {
        active[r] = 0;
        continue;
      }
      any = true;
      budget_max = std::max(budget_max, std::min(m, o.max_iters - iters[r]));
    }
    if (!any) break;
    for (int r = 0; r < R; ++r) {
      hs[4 * r + 1] = o.tol * bnorm[r];
      hs[4 * r + 2] = active[r] ? double(std::min(m, o.max_iters - iters[r])) : 0.0;
      jinit[r] = active[r] ? 0 : -1;
      g0[size_t(r) * (m + 1)] = cplx<double>{active[r] ? hs[4 * r] : 0.0, 0.0};
    }
    GM_HIP(hipMemcpyAsync(K.scal, hs, sizeof(double) * 4 * R, hipMemcpyHostToDevice, s));
    GM_HIP(hipMemcpyAsync(K.active, jinit, sizeof(int) * R, hipMemcpyHostToDevice, s));
    GM_HIP(hipMemcpyAsync(K.g, g0, sizeof(cplx<double>) * gl, hipMemcpyHostToDevice, s));
    GM_HIP(hipMemcpyAsync(K.ib, ib0, sizeof(double) * gl, hipMemcpyHostToDevice, s));
    GM_LAUNCH(k_scale<Tb>, dim3(nblk(n * R, 256)), dim3(256), 0, s, K.r, V, K.scal, 4, n, R);
    x_zero = false;
    for (int r = 0; r < R; ++r) {
      est_prev[r] = hs[4 * r];
      j_prev[r] = 0;
    }
    // predicted_stop: every running right-hand side is predicted to pass its threshold
    // by the next check (then no iteration is enqueued ahead of that check)
    int j_end = 0, next_check = std::min(check, budget_max);
    bool predicted_stop = false;
    {
      bool known = true;
      int need_max = 1;
      for (int r = 0; r < R; ++r) {
        if (!active[r]) continue;
        if (!(rate_last[r] < 0)) {
          known = false;
          break;
        }
        const int need = int(std::ceil(std::log(hs[4 * r + 1] / hs[4 * r]) / rate_last[r]));
        if (need > check) known = false;
        need_max = std::max(need_max, std::min(std::max(need, 1), check));
      }
      if (known) next_check = std::min(next_check, need_max);
      predicted_stop = known;
    }
    int launched = 0;  // iterations of this cycle already enqueued
    for (int j = 0; j < budget_max; ++j) {
      if (j >= launched) {
        rc = launch_iter(j);
        if (rc) return rc;
        launched = j + 1;
      }
      j_end = j + 1;
      if (j_end >= next_check || j_end == budget_max) {
        GM_HIP(hipMemcpyAsync(jused, K.active, sizeof(int) * R, hipMemcpyDeviceToHost, s));
        GM_HIP(hipMemcpyAsync(gh, K.g, sizeof(cplx<double>) * gl, hipMemcpyDeviceToHost, s));
        GM_HIP(hipEventRecord(K.ev_check, s));
        // The device goes on with the next iteration while the host reads the flags.
        // Should every right-hand side have stopped, that iteration changes nothing the
        // solution uses: the Givens step leaves stopped right-hand sides alone, and its
        // other outputs (u_{j+2}, s_{j+2}, scratch) lie past the columns the update reads.
        if (!predicted_stop && j_end < budget_max) {
          rc = launch_iter(j_end);
          if (rc) return rc;
          launched = j_end + 1;
        }
        GM_HIP(hipEventSynchronize(K.ev_check));
        bool all = true;
        int ahead = 1;
        predicted_stop = true;
        for (int r = 0; r < R; ++r) {
          if (jused[r] != 0) continue;
          all = false;
          const cplx<double> gv = gh[size_t(r) * (m + 1) + j_end];
          const double est = std::sqrt(gv.re * gv.re + gv.im * gv.im), thr = hs[4 * r + 1];
          int need = check;
          bool known = false;
          if (est > 0 && est < est_prev[r] && thr > 0) {
            const double rate = std::log(est / est_prev[r]) / double(j_end - j_prev[r]);
            need = int(std::ceil(std::log(thr / est) / rate));
            rate_last[r] = rate;
            known = need <= check;
          }
          if (!known) predicted_stop = false;
          ahead = std::max(ahead, std::min(std::max(need, 1), check));
          est_prev[r] = est;
          j_prev[r] = j_end;
        }
        if (all) break;
        next_check = j_end + ahead;
      }
    }
    GM_LAUNCH(k_lsq, dim3(R), b64, sizeof(cplx<double>) * (size_t(m) * (m + 1) + m + 1), s, K.H, K.g, K.h2,
              K.active, m, R, j_end);
    if (pre) {
      // x += P (V y), P applied in FP64
      GM_HIP(hipMemsetAsync(K.w, 0, sizeof(cplx<double>) * n * R, s));
      GM_LAUNCH(k_update_x<Tb>, dim3(nblk(n * R, 256)), dim3(256), 0, s, V, K.w, K.h2, K.ib, n, j_end, R, m);
      rc = precond_impl<double>(op, K.w, K.r, R, s);
      if (rc) return rc;
      GM_LAUNCH(k_add, dim3(nblk(n * R, 256)), dim3(256), 0, s, x, K.r, n * R);
    } else {
      GM_LAUNCH(k_update_x<Tb>, dim3(nblk(n * R, 256)), dim3(256), 0, s, V, x, K.h2, K.ib, n, j_end, R, m);
    }
    GM_HIP(hipMemcpyAsync(jused, K.active, sizeof(int) * R, hipMemcpyDeviceToHost, s));
    GM_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < R; ++r) {
      if (!active[r]) continue;
      const int k = jused[r] > 0 ? jused[r] : j_end;
      iters[r] += k;
      matvecs[r] += k;
      restarts[r] += 1;
    }
  }
  bool all_conv = true;
  for (int r = 0; r < R; ++r) {
    st[r].iters = iters[r];
    st[r].restarts = restarts[r];
    st[r].matvecs = matvecs[r];
    st[r].true_relres = relres[r];
    st[r].converged = relres[r] <= o.tol ? 1 : 0;
    if (!st[r].converged) all_conv = false;
  }
  return all_conv ? AIM_OK : AIM_ENOCONV;
}

void drop_graphs(KrylovWork& K) {
  for (auto& kv : K.graphs)
    for (hipGraphExec_t g : kv.second)
      if (g) (void)hipGraphExecDestroy(g);
  K.graphs.clear();
}

void free_krylov(KrylovWork& K) {
  drop_graphs(K);
  void* ps[] = {K.V,  K.w,  K.wlow, K.ylow, K.r,    K.H,    K.cs,     K.sn, K.g,
                K.hcol, K.h2, K.part, K.scal, K.active, K.S, K.ib, K.pq, K.cr};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  if (K.hpin) (void)hipHostFree(K.hpin);
  if (K.cap) (void)hipStreamDestroy(K.cap);
  if (K.ev_check) (void)hipEventDestroy(K.ev_check);
  K = KrylovWork{};
}

int ensure_krylov(aim_op* op, int R, int m, int prec) {
  KrylovWork& K = op->kw;
  if (K.V && K.R == R && K.restart >= m && K.prec == prec) return AIM_OK;
  free_krylov(K);
  const int64_t n = int64_t(op->ne) * op->N;
  const int nch = int((n + kChunk - 1) / kChunk);
  const size_t vb = prec == AIM_FP64 ? sizeof(cplx<double>) : sizeof(cplx<float>);
  bool ok = true;
  auto al = [&](void** p, size_t bytes) {
    if (ok && hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
      *p = nullptr;
      ok = false;
    }
  };
  al(&K.V, size_t(m + 1) * R * n * vb);
  al(reinterpret_cast<void**>(&K.w), sizeof(cplx<double>) * R * n);
  al(reinterpret_cast<void**>(&K.r), sizeof(cplx<double>) * R * n);
  if (prec != AIM_FP64) al(&K.ylow, sizeof(cplx<float>) * R * n);
  al(reinterpret_cast<void**>(&K.H), sizeof(cplx<double>) * R * m * (m + 1));
  al(reinterpret_cast<void**>(&K.cs), sizeof(cplx<double>) * R * m);
  al(reinterpret_cast<void**>(&K.sn), sizeof(cplx<double>) * R * m);
  al(reinterpret_cast<void**>(&K.g), sizeof(cplx<double>) * R * (m + 1));
  al(reinterpret_cast<void**>(&K.hcol), sizeof(cplx<double>) * R * (m + 1));
  al(reinterpret_cast<void**>(&K.h2), sizeof(cplx<double>) * R * (m + 1));
  al(reinterpret_cast<void**>(&K.S), sizeof(cplx<double>) * R * (m + 1) * (m + 1));
  al(reinterpret_cast<void**>(&K.ib), sizeof(double) * R * (m + 1));
  al(reinterpret_cast<void**>(&K.pq), sizeof(cplx<double>) * R * 2 * (m + 1));
  al(reinterpret_cast<void**>(&K.cr), sizeof(cplx<double>) * R * (m + 1));
  const int nchs = int((n + kBS - 1) / kBS);
  // chunk partials of up to 2 (m + 1) complex values per right-hand side
  K.part_len = size_t(R) * 2 * (m + 1) * std::max(nch, nchs) * 2;
  al(reinterpret_cast<void**>(&K.part), sizeof(double) * K.part_len);
  al(reinterpret_cast<void**>(&K.scal), sizeof(double) * 4 * R);
  al(reinterpret_cast<void**>(&K.active), sizeof(int) * R);
  {
    // pinned staging: [R][4] doubles, 2 x [R] ints, 2 x [R][m+1] complex, [R][m+1] doubles
    const size_t gl = size_t(R) * (m + 1);
    auto up8 = [](size_t b) { return (b + 15) / 16 * 16; };
    const size_t o1 = up8(sizeof(double) * 4 * R), o2 = o1 + up8(sizeof(int) * R), o3 = o2 + up8(sizeof(int) * R),
                 o4 = o3 + sizeof(cplx<double>) * gl, o5 = o4 + sizeof(cplx<double>) * gl,
                 end = o5 + sizeof(double) * gl;
    if (ok && hipHostMalloc(&K.hpin, end, hipHostMallocDefault) != hipSuccess) {
      K.hpin = nullptr;
      ok = false;
    }
    if (ok) {
      unsigned char* h = static_cast<unsigned char*>(K.hpin);
      K.h_scal = reinterpret_cast<double*>(h);
      K.h_jinit = reinterpret_cast<int*>(h + o1);
      K.h_jused = reinterpret_cast<int*>(h + o2);
      K.h_g0 = reinterpret_cast<cplx<double>*>(h + o3);
      K.h_gh = reinterpret_cast<cplx<double>*>(h + o4);
      K.h_ib0 = reinterpret_cast<double*>(h + o5);
    }
  }
  if (ok && hipEventCreateWithFlags(&K.ev_check, hipEventDisableTiming) != hipSuccess) {
    K.ev_check = nullptr;
    ok = false;
  }
  if (!ok) {
    free_krylov(K);
    set_error("gmres: device allocation of the Krylov workspace failed");
    return AIM_ENOMEM;
  }
  K.R = R;
  K.restart = m;
  K.prec = prec;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_lsq), hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(sizeof(cplx<double>) * (size_t(m) * (m + 1) + m + 1)));
  return AIM_OK;
}

}  // namespace
}  // namespace aimm

using namespace aimm;

extern "C" int gmres_solve(aim_op* op, const void* b, void* x, int32_t nrhs, const gmres_opts* opts,
                           gmres_stat* stats, void* stream) {
  if (!op || !b || !x || !opts || !stats) {
    set_error("gmres: NULL argument");
    return AIM_EINVAL;
  }
  if (nrhs < 1 || nrhs > op->R_max) {
    set_error("gmres: nrhs must be in [1, max_rhs]");
    return AIM_EINVAL;
  }
  if (opts->restart < 1 || opts->restart > kMaxRestart || opts->max_iters < 0 || !(opts->tol > 0) ||
      (opts->precision != AIM_FP64 && opts->precision != AIM_MIXED)) {
    set_error("gmres: bad options (restart in [1,96], max_iters >= 0, tol > 0, precision)");
    return AIM_EINVAL;
  }
  if (b == x) {
    set_error("gmres: b and x must not alias");
    return AIM_EINVAL;
  }
  if (opts->precond != AIM_PRECOND_NONE && opts->precond != AIM_PRECOND_BLOCK_JACOBI) {
    set_error("gmres: unknown preconditioner");
    return AIM_EINVAL;
  }
  if (opts->precond == AIM_PRECOND_BLOCK_JACOBI && !op->p_set) {
    set_error("gmres: block-Jacobi preconditioner not built (aim_build_preconditioner)");
    return AIM_ESTATE;
  }
  if (opts->system != AIM_FULL && opts->system != AIM_G_ONLY) {
    set_error("gmres: system must be AIM_FULL or AIM_G_ONLY");
    return AIM_EINVAL;
  }
  if (!op->device_ready || (opts->system == AIM_FULL && (!op->m_set || !op->d_set))) {
    set_error("gmres: device data, macromodels and D must be set");
    return AIM_ESTATE;
  }
  int rc = ensure_krylov(op, nrhs, opts->restart, opts->precision);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (opts->precision == AIM_FP64)
    return gmres_impl<double>(op, static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), nrhs, *opts,
                              stats, s);
  return gmres_impl<float>(op, static_cast<const cplx<double>*>(b), static_cast<cplx<double>*>(x), nrhs, *opts, stats,
                           s);
}

namespace aimm {
void release_krylov(aim_op* op) { free_krylov(op->kw); }
}  // namespace aimm
