// Argument blocks and launchers of the AIM product kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "fft.hpp"

namespace aimm {

constexpr int kMaxNz = 16;     // grid nodes along z (direct aperiodic sum in the spectrum pass)
constexpr int kMaxTypes = 16;  // distinct element kinds

struct ProjArgs {
  int R, ne, N, px, py, pitch;
  int ex, ey, ez;
  int nx, ny, nz, q3;
  const int* node_ptr;
  const int* node_ent;
};

struct ConvArgs {
  int R, nx, ny, nz, B;
  FftPlan Px, Py;
  const void* tw_x;
  const void* tw_y;
  const void* gt;
  const int* rev_x;
  const int* rev_y;
};

struct CombineArgs {
  int R, ne, N, px, pitch;
  int nx, ny, nz, q, q3;
  int n_off;
  double keta, sig_phi;
  const int* sloc;
  const int* near_ptr;
  const int* near_col;
  const int* nbr;
  const int* d_ptr;
  const int* d_col;
};

struct GemmArgs {
  int N, R, n_types;
  int tile_start[kMaxTypes + 1];
  int type_count[kMaxTypes];
  int col_start[kMaxTypes];
  const int* col_list;
};

template <typename T>
hipError_t launch_project(const cplx<T>* u, cplx<T>* Q, const ProjArgs& a, const T* Wp, hipStream_t s);
template <typename T>
hipError_t launch_convolve(const cplx<T>* Q, cplx<T>* Phi, cplx<T>* S, const ConvArgs& a, hipStream_t s,
                           hipEvent_t* ev = nullptr);
template <typename T>
hipError_t launch_combine(int mode, const cplx<T>* Phi, const cplx<T>* u, const cplx<T>* x, cplx<T>* y,
                          const CombineArgs& a, const T* Wt, const cplx<T>* near_val, const cplx<T>* d_val,
                          hipStream_t s);
template <typename T>
hipError_t launch_macro(const cplx<T>* M, const cplx<T>* X, cplx<T>* U, const GemmArgs& a, hipStream_t s);
hipError_t launch_spectrum(cplx<double>* raw, int Lx, int Ly, int nz, double k, double h, const FftPlan& Px,
                           const FftPlan& Py, const cplx<double>* tw_x, const cplx<double>* tw_y, int B,
                           hipStream_t s);
template <typename T>
hipError_t launch_extract(const cplx<double>* raw, cplx<T>* gt, int Lx, int Ly, int nz, const int* pos_x,
                          const int* pos_y, hipStream_t s);
hipError_t launch_expand_rhs(const cplx<double>* loc, const double* kinc, cplx<double>* b, int R, int ne, int N,
                             int px, double pitch_len, double k, hipStream_t s);
// Raise the dynamic LDS limit of the FFT kernels to `bytes` (device maximum).
hipError_t configure_lds(size_t bytes);
template <typename Tin, typename Tout>
hipError_t launch_convert(const cplx<Tin>* in, cplx<Tout>* out, int64_t n, hipStream_t s);

}  // namespace aimm
