// Complex arithmetic and small helpers shared by the device kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace aimm {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmk(T r, T i) {
  cplx<T> c;
  c.re = r;
  c.im = i;
  return c;
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return cmk<T>(a.re + b.re, a.im + b.im);
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return cmk<T>(a.re - b.re, a.im - b.im);
}
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return cmk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return cmk<T>(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) {
  return cmk<T>(a.re * s, a.im * s);
}
// acc += a * b
template <typename T>
__device__ __forceinline__ void cfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
// acc += s * b  (real s)
template <typename T>
__device__ __forceinline__ void cfmas(cplx<T>& acc, T s, cplx<T> b) {
  acc.re = fma(s, b.re, acc.re);
  acc.im = fma(s, b.im, acc.im);
}
// multiply by -i (sign = +1) or +i (sign = -1): (-i)(u + iv) = v - iu
template <typename T>
__device__ __forceinline__ cplx<T> cmul_mi(cplx<T> a, T sign) {
  return cmk<T>(sign * a.im, -sign * a.re);
}

}  // namespace aimm
