// Argument blocks and launchers of the AIM product kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "fft.hpp"

namespace aimm {

constexpr int kMaxNz = 16;     // grid nodes along z (direct aperiodic sum in the spectrum pass)
constexpr int kMaxTypes = 16;  // distinct element kinds

constexpr int kMaxOffsets = 25;  // lattice offsets carrying near-field pairs

struct ProjArgs {
  int R, ne, N, px, py, pitch;
  int ex, ey, ez;
  int nx, ny, nz, q3;
  const int* node_ptr;
  const int* node_n;  // per gather entry: n * ne (offset of basis n in the element-fastest u)
  const void* zero;  // one zero complex value (read for absent neighbours)
};

// FFT lengths L = L1 L2 with register-DFT (four-step) passes
#define AIM_F4_LENGTHS(X) X(3, 9) X(5, 8) X(6, 9) X(8, 8) X(10, 20) X(16, 24) X(20, 20) X(25, 32)
bool fft4_supported(int L);
// whether the three FFT passes launch for padded lengths Lx, Ly, nz z nodes, B ky lines
// per x-pass workgroup and the register-DFT (f4) or radix-stage passes, with elem-byte
// complex values and lds_limit bytes of LDS per workgroup
bool conv_fits(int Lx, int Ly, int nz, int B, bool f4, size_t elem, size_t lds_limit);

struct ConvArgs {
  int R, nx, ny, nz, B;
  int f4;  // 1: register-DFT passes (natural-order spectra), 0: radix-stage passes
  FftPlan Px, Py;
  const void* tw_x;
  const void* tw_y;
  const void* gt;
  const int* rev_x;
  const int* rev_y;
  int passes;        // bit 0: forward y, bit 1: x with the spectrum product, bit 2: inverse y
  void* x_out;       // target of the x pass; nullptr: in place in S
};

constexpr int kNearGroupDev = 16;  // rows per matrix-core near-field group
constexpr int kNearColTailDev = 32;  // zero columns after the last group
constexpr int kXcds = 8;           // accelerator complex dies; workgroups are dealt to them round-robin

struct NearArgs {
  int R, ne, N, px, py;
  const int* offsets;  // [n_off][2] (dx, dy)
  const int* near_ptr;
  const int* near_col;
  const int* grp_ptr;  // row-group tables (matrix-core path); grp_A == nullptr selects the CSR path
  const int* grp_col;
  const int* grp_row;  // [groups][kNearGroupDev] row of each group slot, -1 for none
  const int* slot_of;  // [N] group slot of each row
  const void* grp_A;
  const void* zero;    // one zero complex value (read for absent neighbours)
  int grp_max_cols;    // largest column count of a group (LDS staging of its columns)
  int ld_nf;           // slots per element of the output (groups x kNearGroupDev)
  int eb;              // matrix-core path: blocks of 16 elements per workgroup (1 or 2)
};

struct InterpArgs {
  int R, ne, N, px, py, pitch;
  int nx, ny, nz, q, q3, ex, ey;
  int TX, TY;  // elements per workgroup tile
  double keta, sig_phi;
  const int* sloc;
  // D block, padded to dmax slots per row and stored slot-major: entry s of row n at
  // s * N + n (padding: column n, value 0)
  const int* d_colT;
  int dmax;
  // near-field input, slot-ordered: row n of element m at m * ld_nf + slot_of[n]
  const int* slot_of;
  int ld_nf;
};

inline size_t interp_lds_bytes(const InterpArgs& a, size_t elem) {
  const size_t bx = size_t(a.pitch) * (a.TX - 1) + a.ex, by = size_t(a.pitch) * (a.TY - 1) + a.ey;
  // the tile's potential box (4 psi), then the tile's input rows for the D product
  return (4 * bx * by * a.nz + size_t(a.TX) * a.TY * a.N) * elem;
}

constexpr int kGemmColsHost = 32;  // output columns per macromodel GEMM workgroup

// Macromodel rows on the device: per kind, Krows = 4 Kq + kGemmKTail columns of M
// (column-major), zero past N; Kq is the per-wave K range, a multiple of 16.
constexpr int kGemmKTail = 16;  // one prefetch batch past the last wave's range
inline int gemm_kq(int N) { return (N + 63) / 64 * 16; }
inline int gemm_krows(int N) { return 4 * gemm_kq(N) + kGemmKTail; }

struct GemmArgs {
  int N, R, n_types, ne;
  int Kq, Krows;
  const void* Mb;  // split-BF16 planes of M (FP32 path), or null for the FP32 MFMA kernel
  int tile_start[kMaxTypes + 1];
  int type_count[kMaxTypes];
  int col_start[kMaxTypes];
  const int* col_list;
};

template <typename T>
hipError_t launch_project(const cplx<T>* uT, cplx<T>* Q, const ProjArgs& a, const T* Wp, hipStream_t s);
template <typename T>
hipError_t launch_convolve(const cplx<T>* Q, cplx<T>* Phi, cplx<T>* S, const ConvArgs& a, hipStream_t s,
                           hipEvent_t* ev = nullptr);
template <typename T>
hipError_t launch_near(const cplx<T>* uT, cplx<T>* nf, const NearArgs& a, const cplx<T>* near_val, hipStream_t s);
template <typename T>
hipError_t launch_interp(int mode, const cplx<T>* Phi, const cplx<T>* nf, const cplx<T>* x, cplx<T>* y,
                         const InterpArgs& a, const T* Wt, const cplx<T>* d_val, hipStream_t s);
template <typename T>
hipError_t launch_transpose(const cplx<T>* x, cplx<T>* xT, int R, int ne, int N, hipStream_t s);
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
