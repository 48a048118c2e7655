// In-place mixed-radix (2, 3, 4, 5) FFT of lines held in LDS, run cooperatively by
// one workgroup.
//
// Forward transform: decimation in frequency.  Stage s works on blocks of size B_s
// (B_0 = L) with stride S_s = B_s / r_s: for every block b and j < S_s it takes the
// r_s values at b B_s + j + i S_s, applies the length-r_s DFT, multiplies output q by
// exp(-2 pi i j q / B_s) and writes it back to b B_s + j + q S_s.  Butterflies of a
// stage touch disjoint slots, so the stage runs in place.  The result is in mixed-
// radix digit-reversed order: slot p = sum_s q_s S_s holds frequency
// k = q_0 + r_0 (q_1 + r_1 (q_2 + ...)).
// Inverse transform: the stages undone in reverse order with conjugate twiddles and
// the inverse DFT; it reads digit-reversed input and returns natural order, scaled
// by L.  A convolution therefore never needs a permutation pass.
//
// Every stage is compiled for its radix (values stay in registers); integer
// divisions by the per-stage counts use precomputed multipliers: for n d < 2^32,
// n / d = umulhi(n, floor((2^32 - 1) / d) + 1).
#pragma once

#include "device_common.hpp"

namespace aimm {

constexpr int kMaxStages = 12;

struct FftPlan {
  int L;
  int nst;
  int radix[kMaxStages];
  int stride[kMaxStages];     // S_s
  int tw_step[kMaxStages];    // L / B_s
  unsigned div_nb[kMaxStages];  // multiplier for division by L / r_s
  unsigned div_S[kMaxStages];   // multiplier for division by S_s
};

__host__ __device__ inline unsigned magic_div(unsigned d) { return d == 1 ? 0u : 0xFFFFFFFFu / d + 1u; }
__device__ __forceinline__ int fast_div(int n, unsigned magic) {
  return magic == 0u ? n : int(__umulhi(unsigned(n), magic));
}

template <typename T, int R>
__device__ __forceinline__ void dft_r(cplx<T>* x, T sgn) {
  // sgn = +1: forward (exp(-2 pi i / R)), sgn = -1: inverse.
  if constexpr (R == 2) {
    cplx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 4) {
    cplx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    cplx<T> b0 = cadd(x[1], x[3]), b1 = cmul_mi(csub(x[1], x[3]), sgn);
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  } else if constexpr (R == 3) {
    const T s3 = T(0.86602540378443864676);
    cplx<T> t1 = cadd(x[1], x[2]);
    cplx<T> t2 = cscale(cmul_mi(csub(x[1], x[2]), sgn), s3);
    cplx<T> m = cmk<T>(x[0].re - T(0.5) * t1.re, x[0].im - T(0.5) * t1.im);
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, t2);
    x[2] = csub(m, t2);
  } else {
    static_assert(R == 5, "radix");
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
    cplx<T> a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    cplx<T> a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    cplx<T> x0 = x[0];
    cplx<T> p1 = cmk<T>(x0.re + c1 * a1.re + c2 * a2.re, x0.im + c1 * a1.im + c2 * a2.im);
    cplx<T> p2 = cmk<T>(x0.re + c2 * a1.re + c1 * a2.re, x0.im + c2 * a1.im + c1 * a2.im);
    cplx<T> q1 = cmul_mi(cmk<T>(s1 * b1.re + s2 * b2.re, s1 * b1.im + s2 * b2.im), sgn);
    cplx<T> q2 = cmul_mi(cmk<T>(s2 * b1.re - s1 * b2.re, s2 * b1.im - s1 * b2.im), sgn);
    x[0] = cadd(x0, cadd(a1, a2));
    x[1] = cadd(p1, q1);
    x[4] = csub(p1, q1);
    x[2] = cadd(p2, q2);
    x[3] = csub(p2, q2);
  }
}

template <typename T, int R, bool FWD>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int ld, int nlines, const FftPlan& P, int s,
                                          const cplx<T>* tw) {
  const int S = P.stride[s], step = P.tw_step[s];
  const unsigned mnb = P.div_nb[s], mS = P.div_S[s];
  const int nb = P.L / R;
  const int items = nb * nlines;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int line = fast_div(it, mnb);
    const int t = it - line * nb;
    const int blk = fast_div(t, mS);
    const int j = t - blk * S;
    cplx<T>* base = buf + line * ld + blk * S * R + j;
    cplx<T> x[R];
    if constexpr (FWD) {
#pragma unroll
      for (int i = 0; i < R; ++i) x[i] = base[i * S];
      dft_r<T, R>(x, T(1));
      base[0] = x[0];
#pragma unroll
      for (int qo = 1; qo < R; ++qo) base[qo * S] = cmul(x[qo], tw[j * qo * step]);
    } else {
      x[0] = base[0];
#pragma unroll
      for (int qo = 1; qo < R; ++qo) x[qo] = cmulc(base[qo * S], tw[j * qo * step]);
      dft_r<T, R>(x, T(-1));
#pragma unroll
      for (int i = 0; i < R; ++i) base[i * S] = x[i];
    }
  }
}

template <typename T, bool FWD>
__device__ __forceinline__ void fft_stage_any(cplx<T>* buf, int ld, int nlines, const FftPlan& P, int s,
                                              const cplx<T>* tw) {
  switch (P.radix[s]) {
    case 2: fft_stage<T, 2, FWD>(buf, ld, nlines, P, s, tw); break;
    case 3: fft_stage<T, 3, FWD>(buf, ld, nlines, P, s, tw); break;
    case 4: fft_stage<T, 4, FWD>(buf, ld, nlines, P, s, tw); break;
    default: fft_stage<T, 5, FWD>(buf, ld, nlines, P, s, tw); break;
  }
}

// Forward (DIF) transform of nlines lines at buf + line * ld, in place.
// tw[t] = exp(-2 pi i t / L).  Ends with a barrier.
template <typename T>
__device__ void lds_fft_fwd(cplx<T>* buf, int ld, int nlines, const FftPlan& P, const cplx<T>* tw) {
  for (int s = 0; s < P.nst; ++s) {
    fft_stage_any<T, true>(buf, ld, nlines, P, s, tw);
    __syncthreads();
  }
}

// Inverse (DIT) transform, digit-reversed in, natural out, scaled by L.
template <typename T>
__device__ void lds_fft_inv(cplx<T>* buf, int ld, int nlines, const FftPlan& P, const cplx<T>* tw) {
  for (int s = P.nst - 1; s >= 0; --s) {
    fft_stage_any<T, false>(buf, ld, nlines, P, s, tw);
    __syncthreads();
  }
}

}  // namespace aimm
