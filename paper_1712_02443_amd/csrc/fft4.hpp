// Length-L FFT of lines held in LDS as two passes of register DFTs (the four-step
// factorisation L = L1 L2), run cooperatively by one workgroup.
//
// With x = L2 x1 + x2 and k = k1 + L1 k2,
//   X[k1 + L1 k2] = sum_{x2} W_{L2}^{x2 k2} W_L^{x2 k1} sum_{x1} a[L2 x1 + x2] W_{L1}^{x1 k1},
// so pass A gives each of L2 threads a line's stride-L2 subsequence for one length-L1
// DFT in registers followed by the twiddle W_L^{x2 k1}, and pass B gives each of L1
// threads L2 consecutive results for one length-L2 DFT.  Input and output are in
// natural order.  Element i of a line sits at LDS slot i + i / L2 (one pad slot per
// L2 values), which makes both passes read and write consecutive slots across lanes.
// The register DFTs recurse on the same factorisation down to radix 2, 3, 4 and 5,
// with their twiddles folded to constants at compile time.
#pragma once

#include <type_traits>
#include <utility>

#include "fft.hpp"

namespace aimm {
namespace fft4 {

// (cos, sin) of 2 pi m / n in double, evaluated at compile time: the angle is reduced
// to [0, pi/4] by quadrant and octant symmetry and fed to Taylor series.
struct CS {
  double c, s;
};
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int k = 1; k <= 12; ++k) {
    t *= -x * x / double((2 * k) * (2 * k + 1));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1, s = 1;
  for (int k = 1; k <= 12; ++k) {
    t *= -x * x / double((2 * k - 1) * (2 * k));
    s += t;
  }
  return s;
}
constexpr CS cs_frac(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n;       // quadrant
  long r = 4 * m - q * n;           // angle within the quadrant = (pi / 2) r / n
  const double half_pi = 1.57079632679489661923;
  double c = 1, s = 0;
  if (2 * r <= n) {
    const double b = half_pi * double(r) / double(n);
    c = taylor_cos(b);
    s = taylor_sin(b);
  } else {
    const double b = half_pi * double(n - r) / double(n);
    c = taylor_sin(b);
    s = taylor_cos(b);
  }
  if (r == 0) {
    c = 1;
    s = 0;
  }
  switch (q) {
    case 0: return CS{c, s};
    case 1: return CS{-s, c};
    case 2: return CS{-c, -s};
    default: return CS{s, -c};
  }
}

template <int I, int END, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < END) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, END>(f);
  }
}

template <int N>
constexpr int first_factor() {
  return N % 4 == 0 ? 4 : N % 5 == 0 ? 5 : N % 3 == 0 ? 3 : N % 2 == 0 ? 2 : N;
}

// In-register DFT of compile-time length N (5-smooth), natural order in and out.
// FWD: exp(-2 pi i / N) kernel; otherwise the conjugate (unscaled inverse).
template <typename T, int N, bool FWD>
struct RegDft {
  static __device__ __forceinline__ void run(cplx<T>* x) {
    if constexpr (N == 1) {
      return;
    } else if constexpr (N == 2 || N == 3 || N == 4 || N == 5) {
      dft_r<T, N>(x, FWD ? T(1) : T(-1));
    } else {
      constexpr int R = first_factor<N>(), M = N / R;
      static_assert(R > 1 && R < N, "length must be 5-smooth");
      cplx<T> b[N];
      static_for<0, M>([&](auto x2c) {
        constexpr int x2 = decltype(x2c)::value;
        cplx<T> t[R];
        static_for<0, R>([&](auto x1c) {
          constexpr int x1 = decltype(x1c)::value;
          t[x1] = x[M * x1 + x2];
        });
        RegDft<T, R, FWD>::run(t);
        static_for<0, R>([&](auto k1c) {
          constexpr int k1 = decltype(k1c)::value;
          if constexpr ((x2 * k1) % N == 0) {
            b[x2 * R + k1] = t[k1];
          } else {
            constexpr CS w = cs_frac(x2 * k1, N);
            b[x2 * R + k1] = cmul(t[k1], cmk<T>(T(w.c), FWD ? T(-w.s) : T(w.s)));
          }
        });
      });
      static_for<0, R>([&](auto k1c) {
        constexpr int k1 = decltype(k1c)::value;
        cplx<T> u[M];
        static_for<0, M>([&](auto x2c) {
          constexpr int x2 = decltype(x2c)::value;
          u[x2] = b[x2 * R + k1];
        });
        RegDft<T, M, FWD>::run(u);
        static_for<0, M>([&](auto k2c) {
          constexpr int k2 = decltype(k2c)::value;
          x[k1 + R * k2] = u[k2];
        });
      });
    }
  }
};

}  // namespace fft4

// LDS slot of element i of a line
template <int L2>
__device__ __forceinline__ int f4_slot(int i) {
  return i + i / L2;
}
// slots per line
template <int L1, int L2>
constexpr int f4_ld() {
  return L1 * (L2 + 1);
}

// Transform nlines lines at buf + line * f4_ld in place.  tw[t] = exp(-2 pi i t / L)
// for t < L (LDS).  Needs blockDim.x >= nlines * max(L1, L2); ends with a barrier.
// Pruning: ZERO_TAIL declares the input zero beyond index L / 2 (a line zero-padded
// from at most L / 2 + 1 values), so pass A keeps only rows x1 <= L1 / 2 and the DFTs
// fold the zeros away; HALF_OUT keeps only outputs up to index L / 2 (the unpadded
// part), so pass B stores, and computes, outputs k2 <= L2 / 2 only.
template <typename T, int L1, int L2, bool FWD, bool ZERO_TAIL = false, bool HALF_OUT = false>
__device__ __forceinline__ void fft4_lines(cplx<T>* buf, int nlines, const cplx<T>* tw) {
  constexpr int P = L2 + 1, LD = f4_ld<L1, L2>();
  constexpr int NA = ZERO_TAIL ? L1 / 2 + 1 : L1, NB = HALF_OUT ? L2 / 2 + 1 : L2;
  // pass A: one length-L1 DFT per (line, x2), then the twiddles W_L^{x2 k1}
  if (int(threadIdx.x) < nlines * L2) {
    const int line = threadIdx.x / L2, x2 = threadIdx.x - line * L2;
    __builtin_assume(x2 >= 0 && x2 < L2);
    cplx<T>* b = buf + line * LD;
    cplx<T> v[L1];
#pragma unroll
    for (int x1 = 0; x1 < L1; ++x1) v[x1] = x1 < NA ? b[x1 * P + x2] : cmk<T>(0, 0);
    fft4::RegDft<T, L1, FWD>::run(v);
#pragma unroll
    for (int k1 = 1; k1 < L1; ++k1) v[k1] = FWD ? cmul(v[k1], tw[x2 * k1]) : cmulc(v[k1], tw[x2 * k1]);
#pragma unroll
    for (int k1 = 0; k1 < L1; ++k1) b[k1 * P + x2] = v[k1];
  }
  __syncthreads();
  // pass B: one length-L2 DFT per (line, k1); results go to the slots of k1 + L1 k2
  const bool act = int(threadIdx.x) < nlines * L1;
  const int line = threadIdx.x / L1, k1 = threadIdx.x - line * L1;
  __builtin_assume(k1 >= 0 && k1 < L1);
  cplx<T> u[L2];
  if (act) {
    const cplx<T>* b = buf + line * LD + k1 * P;
#pragma unroll
    for (int x2 = 0; x2 < L2; ++x2) u[x2] = b[x2];
  }
  __syncthreads();
  if (act) {
    fft4::RegDft<T, L2, FWD>::run(u);
    cplx<T>* o = buf + line * LD;
#pragma unroll
    for (int k2 = 0; k2 < NB; ++k2) o[f4_slot<L2>(k1 + L1 * k2)] = u[k2];
  }
  __syncthreads();
}

}  // namespace aimm
