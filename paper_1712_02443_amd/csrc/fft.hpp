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
#pragma once

#include "device_common.hpp"

namespace aimm {

constexpr int kMaxStages = 12;

struct FftPlan {
  int L;
  int nst;
  int radix[kMaxStages];
  int stride[kMaxStages];  // S_s
  int tw_step[kMaxStages]; // L / B_s
};

template <typename T>
__device__ __forceinline__ void dft_small(cplx<T>* x, int r, T sgn) {
  // sgn = +1: forward (exp(-2 pi i / r)), sgn = -1: inverse.
  if (r == 2) {
    cplx<T> a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if (r == 4) {
    cplx<T> a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    cplx<T> b0 = cadd(x[1], x[3]), b1 = cmul_mi(csub(x[1], x[3]), sgn);
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    x[1] = cadd(a1, b1);
    x[3] = csub(a1, b1);
  } else if (r == 3) {
    const T s3 = T(0.86602540378443864676);
    cplx<T> t1 = cadd(x[1], x[2]);
    cplx<T> t2 = cscale(cmul_mi(csub(x[1], x[2]), sgn), s3);
    cplx<T> m = cmk<T>(x[0].re - T(0.5) * t1.re, x[0].im - T(0.5) * t1.im);
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, t2);
    x[2] = csub(m, t2);
  } else {  // 5
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

// Forward (DIF) transform of nlines lines at buf + line * ld, in place.
// tw[t] = exp(-2 pi i t / L).  Ends with a barrier.
template <typename T>
__device__ void lds_fft_fwd(cplx<T>* buf, int ld, int nlines, const FftPlan& P, const cplx<T>* tw) {
  const int L = P.L;
  for (int s = 0; s < P.nst; ++s) {
    const int r = P.radix[s], S = P.stride[s], step = P.tw_step[s];
    const int nb = L / r;
    const int items = nb * nlines;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
      const int line = it / nb, t = it - line * nb;
      const int blk = t / S, j = t - blk * S;
      cplx<T>* base = buf + line * ld + blk * S * r + j;
      cplx<T> x[5];
      for (int i = 0; i < r; ++i) x[i] = base[i * S];
      dft_small(x, r, T(1));
      base[0] = x[0];
      for (int qo = 1; qo < r; ++qo) base[qo * S] = cmul(x[qo], tw[j * qo * step]);
    }
    __syncthreads();
  }
}

// Inverse (DIT) transform, digit-reversed in, natural out, scaled by L.
template <typename T>
__device__ void lds_fft_inv(cplx<T>* buf, int ld, int nlines, const FftPlan& P, const cplx<T>* tw) {
  const int L = P.L;
  for (int s = P.nst - 1; s >= 0; --s) {
    const int r = P.radix[s], S = P.stride[s], step = P.tw_step[s];
    const int nb = L / r;
    const int items = nb * nlines;
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
      const int line = it / nb, t = it - line * nb;
      const int blk = t / S, j = t - blk * S;
      cplx<T>* base = buf + line * ld + blk * S * r + j;
      cplx<T> x[5];
      x[0] = base[0];
      for (int qo = 1; qo < r; ++qo) x[qo] = cmulc(base[qo * S], tw[j * qo * step]);
      dft_small(x, r, T(-1));
      for (int i = 0; i < r; ++i) base[i * S] = x[i];
    }
    __syncthreads();
  }
}

}  // namespace aimm
