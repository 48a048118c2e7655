// Far field of the array's equivalent currents for many directions at once: the
// directivity patterns and bistatic RCS that section VI reports for the solved arrays.
//
// With J = -M x the equivalent electric currents of every element (section III, eq.
// Toperator with eq. JABE: J^ = T J = -T A^-1 B E^; x the solution E^ of eq.
// finalsystem) and element m centred at c_m on the lattice,
//   E(r^) = -(j k eta / 4 pi) (I - r^ r^) . sum_n F_n(r^) S(r^, n),
//   S(r^, n) = sum_m exp(j k r^ . c_m) J[m][n],
//   F_n(r^) = int Lambda_n(r) exp(j k r^ . r) dS   (element-local r),
// the far-zone field E r exp(j k r) for unit incident amplitude.  S is a complex GEMM
// over the elements (directions x elements times elements x RWG functions) on the FP64
// matrix cores; its left operand is never stored: c_m = (p h ix, p h iy, 0), so
// exp(j k r^ . c_m) = X[d][ix] Y[d][iy] with two small tables.  Each workgroup contracts
// its S tile with F (seven-point rule on both triangles, evaluated on the fly) and
// writes one partial per tile of RWG functions; a last kernel sums the partials in a
// fixed order, projects out the radial part and forms 10 log10(4 pi |E|^2).
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/aimm.h"
#include "op.hpp"

namespace aimm {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kFfD = 32;  // directions per tile
constexpr int kFfN = 32;  // RWG functions per tile
constexpr int kFfK = 32;  // elements per staged chunk
constexpr int kFfQ = 14;  // quadrature points per RWG function

__global__ void k_ff_tables(const double* __restrict__ rhat, cplx<double>* __restrict__ X,
                            cplx<double>* __restrict__ Y, int D, int px, int py, double kp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = px + py;
  if (t >= D * w) return;
  const int d = t / w, i = t - d * w;
  double s, c;
  if (i < px) {
    sincos(kp * rhat[3 * d] * i, &s, &c);
    X[int64_t(d) * px + i] = cmk<double>(c, s);
  } else {
    sincos(kp * rhat[3 * d + 1] * (i - px), &s, &c);
    Y[int64_t(d) * py + (i - px)] = cmk<double>(c, s);
  }
}

struct FfArgs {
  int D, N, ne, px, py, R;
  double k;
  const double* rhat;        // [D][3]
  const cplx<double>* X;     // [D][px]
  const cplx<double>* Y;     // [D][py]
  const double* quad;        // [N][14][6]
  cplx<double>* part;        // [N tiles][R][D][3]
};

// v_mfma_f64_16x16x4f64: A lane l holds A[l % 16][l / 16], B lane l holds B[l / 16][l % 16];
// output register r of lane l is row l / 16 + 4 r, column l % 16 (measured on gfx950)
__global__ void __launch_bounds__(256) k_ff_gemm(const cplx<double>* __restrict__ uT, FfArgs a) {
  __shared__ cplx<double> ph[kFfD][kFfK + 1];
  __shared__ cplx<double> js[kFfN][kFfK + 1];
  const int d0 = blockIdx.x * kFfD, n0 = blockIdx.y * kFfN, r = blockIdx.z;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wd = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;
  const cplx<double>* u = uT + int64_t(r) * a.N * a.ne;
  f64x4 accR = {}, accI = {};
  for (int m0 = 0; m0 < a.ne; m0 += kFfK) {
    // stage the chunk: phases of 32 directions and currents of 32 RWG functions over 32 elements
    for (int e = threadIdx.x; e < kFfD * kFfK; e += blockDim.x) {
      const int i = e / kFfK, k = e - i * kFfK;
      const int d = d0 + i, m = m0 + k;
      cplx<double> p = cmk<double>(0, 0);
      if (d < a.D && m < a.ne) {
        const int iy = m / a.px, ix = m - iy * a.px;
        p = cmul(a.X[int64_t(d) * a.px + ix], a.Y[int64_t(d) * a.py + iy]);
      }
      ph[i][k] = p;
      const int n = n0 + i;
      js[i][k] = (n < a.N && m < a.ne) ? u[int64_t(n) * a.ne + m] : cmk<double>(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kFfK; kk += 4) {
      const cplx<double> av = ph[wd * 16 + li][kk + lk];
      const cplx<double> bv = js[wn * 16 + li][kk + lk];
      accR = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.re, accR, 0, 0, 0);
      accR = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.im, bv.im, accR, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.im, accI, 0, 0, 0);
      accI = __builtin_amdgcn_mfma_f64_16x16x4f64(av.im, bv.re, accI, 0, 0, 0);
    }
    __syncthreads();
  }
  // S tile into LDS (reusing the phase buffer): row = direction, column = RWG function
#pragma unroll
  for (int q = 0; q < 4; ++q) ph[wd * 16 + lk + 4 * q][wn * 16 + li] = cmk<double>(accR[q], accI[q]);
  __syncthreads();
  // contraction with F: thread = (direction, group of four RWG functions)
  const int di = threadIdx.x >> 3, ng = threadIdx.x & 7;
  const int d = d0 + di;
  cplx<double> acc[3] = {cmk<double>(0, 0), cmk<double>(0, 0), cmk<double>(0, 0)};
  if (d < a.D) {
    const double rx = a.rhat[3 * d], ry = a.rhat[3 * d + 1], rz = a.rhat[3 * d + 2];
    for (int j = 0; j < 4; ++j) {
      const int nl = ng * 4 + j, n = n0 + nl;
      if (n >= a.N) break;
      const double* q = a.quad + int64_t(n) * kFfQ * 6;
      cplx<double> f[3] = {cmk<double>(0, 0), cmk<double>(0, 0), cmk<double>(0, 0)};
      for (int p = 0; p < kFfQ; ++p) {
        double s, c;
        sincos(a.k * (rx * q[6 * p] + ry * q[6 * p + 1] + rz * q[6 * p + 2]), &s, &c);
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          f[x].re += q[6 * p + 3 + x] * c;
          f[x].im += q[6 * p + 3 + x] * s;
        }
      }
      const cplx<double> sv = ph[di][nl];
#pragma unroll
      for (int x = 0; x < 3; ++x) cfma(acc[x], f[x], sv);
    }
  }
  // sum over the eight threads of one direction (consecutive lanes)
#pragma unroll
  for (int off = 1; off < 8; off <<= 1)
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      acc[x].re += __shfl_xor(acc[x].re, off);
      acc[x].im += __shfl_xor(acc[x].im, off);
    }
  if (ng == 0 && d < a.D) {
    cplx<double>* o = a.part + ((int64_t(blockIdx.y) * a.R + r) * a.D + d) * 3;
#pragma unroll
    for (int x = 0; x < 3; ++x) o[x] = acc[x];
  }
}

__global__ void k_ff_finish(const cplx<double>* __restrict__ part, const double* __restrict__ rhat,
                            cplx<double>* __restrict__ E, double* __restrict__ rcs, int D, int R, int ntiles,
                            double keta) {
  // keta carries the sign of the current: -k eta for J = -M x
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R * D) return;
  const int r = t / D, d = t - r * D;
  cplx<double> v[3] = {cmk<double>(0, 0), cmk<double>(0, 0), cmk<double>(0, 0)};
  for (int tl = 0; tl < ntiles; ++tl) {
    const cplx<double>* p = part + ((int64_t(tl) * R + r) * D + d) * 3;
#pragma unroll
    for (int x = 0; x < 3; ++x) v[x] = cadd(v[x], p[x]);
  }
  const double rh[3] = {rhat[3 * d], rhat[3 * d + 1], rhat[3 * d + 2]};
  cplx<double> dot = cmk<double>(0, 0);
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    dot.re += rh[x] * v[x].re;
    dot.im += rh[x] * v[x].im;
  }
  const double g = keta / (4.0 * M_PI);
  double p2 = 0;
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const double tr = v[x].re - rh[x] * dot.re, ti = v[x].im - rh[x] * dot.im;
    // -(j g)(tr + j ti) = g ti - j g tr
    const cplx<double> e = cmk<double>(g * ti, -g * tr);
    E[(int64_t(r) * D + d) * 3 + x] = e;
    p2 += e.re * e.re + e.im * e.im;
  }
  if (rcs) rcs[int64_t(r) * D + d] = 10.0 * log10(fmax(4.0 * M_PI * p2, 1e-300));
}

// bytes of the direction block at the head of the workspace (256-byte aligned tail)
inline size_t ff_dir_bytes(int ndir) { return (size_t(ndir) * 3 * sizeof(double) + 255) / 256 * 256; }

// Workspace bytes of one far-field call: directions, phase tables and per-tile partials.
inline size_t ff_need_bytes(int ndir, int px, int py, int ntiles, int nrhs) {
  return ff_dir_bytes(ndir) + size_t(ndir) * (px + py) * sizeof(cplx<double>) +
         size_t(ntiles) * nrhs * ndir * 3 * sizeof(cplx<double>);
}

// Workspace of the allocation-free entry point aim_far_field_noalloc: one copy per GPU,
// kept until the process ends.  Host code never uses this name as an address: the
// device address of each GPU's copy is looked up once per device (ff_scratch_ptr).
constexpr size_t kFfScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kFfScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), resolved on first use.
hipError_t ff_scratch_ptr(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// The address resolved for `device` by ff_scratch_ptr, or NULL (no HIP call).
void* ff_scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace
}  // namespace aimm

using namespace aimm;

#define FF_HIP(expr)                                                                     \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      set_error(std::string("far field: ") + #expr + ": " + hipGetErrorString(_e));     \
      return AIM_EDEVICE;                                                                \
    }                                                                                    \
  } while (0)

namespace aimm {

// Set-up of the far field at op build time, on the op's device (current): the
// quadrature table of the RWG radiation integrals, and the device address of this
// GPU's scratch array.  Throws std::bad_alloc or std::runtime_error.
void ff_prepare(aim_op* op) {
  if (!op->ff_quad) {
    SurfaceIn sf;
    sf.n_vert = int(op->vert.size() / 3);
    sf.n_tri = int(op->tri.size() / 3);
    sf.n_rwg = int(op->rwg.size() / 4);
    sf.vert = op->vert.data();
    sf.tri = op->tri.data();
    sf.rwg = op->rwg.data();
    std::vector<double> q;
    far_quadrature(sf, q);
    op->ff_quad = op->mem.alloc<double>(q.size());
    if (hipMemcpyAsync(op->ff_quad, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice,
                       op->build_stream) != hipSuccess ||
        hipStreamSynchronize(op->build_stream) != hipSuccess)
      throw std::runtime_error("far field: hipMemcpy of the quadrature table failed");
  }
  void* p = nullptr;
  const hipError_t e = ff_scratch_ptr(op->device, &p);
  if (e != hipSuccess)
    throw std::runtime_error(std::string("far field: hipGetSymbolAddress(scratch) failed: ") +
                             hipGetErrorString(e));
}

}  // namespace aimm

namespace {

// Argument checks shared by both entry points (nothing is modified on failure).
int ff_check(aim_op* op, const void* x, int32_t nrhs, int32_t ndir, const double* rhat, void* E,
             int32_t system) {
  if (!op || !x || !rhat || !E || ndir < 1) {
    set_error("far field: op, x, rhat and E must not be NULL and ndir >= 1");
    return AIM_EINVAL;
  }
  if (nrhs < 1 || nrhs > op->R_max) {
    set_error("far field: nrhs must be in [1, max_rhs]");
    return AIM_EINVAL;
  }
  for (int64_t i = 0; i < 3 * int64_t(ndir); ++i)
    if (!std::isfinite(rhat[i])) {
      set_error("far field: directions must be finite");
      return AIM_EINVAL;
    }
  if (system != AIM_FULL && system != AIM_G_ONLY) {
    set_error("far field: system must be AIM_FULL or AIM_G_ONLY");
    return AIM_EINVAL;
  }
  if (!op->device_ready || (system == AIM_FULL && !op->m_set) || !op->ff_quad) {
    set_error("far field: device data and macromodels must be set");
    return AIM_ESTATE;
  }
  return AIM_OK;
}

// The far-field launches on the workspace ws (at least ff_need_bytes of the call).
int ff_run(aim_op* op, const void* x, int32_t nrhs, int32_t ndir, const double* rhat, void* E, void* rcs_db,
           int32_t system, hipStream_t s, unsigned char* ws) {
  const int N = op->N, ne = op->ne, px = op->arr.px, py = op->arr.py;
  const int ntiles = (N + kFfN - 1) / kFfN;
  double* rd = reinterpret_cast<double*>(ws);
  cplx<double>* X = reinterpret_cast<cplx<double>*>(ws + ff_dir_bytes(ndir));
  cplx<double>* Y = X + size_t(ndir) * px;
  cplx<double>* part = Y + size_t(ndir) * py;
  FF_HIP(hipMemcpyAsync(rd, rhat, size_t(ndir) * 3 * sizeof(double), hipMemcpyHostToDevice, s));
  // currents M x (negated in the last kernel) or x itself, element-fastest
  cplx<double>* uT = static_cast<cplx<double>*>(op->u);
  if (system == AIM_FULL) {
    GemmArgs ga = gemm_args_of(op, nrhs);
    FF_HIP(launch_macro<double>(op->p64.M, static_cast<const cplx<double>*>(x), uT, ga, s));
  } else {
    FF_HIP(launch_transpose<double>(static_cast<const cplx<double>*>(x), uT, nrhs, ne, N, s));
  }
  const double kp = op->arr.k * op->arr.pitch * op->arr.h;
  const int nt = ndir * (px + py);
  hipLaunchKernelGGL(k_ff_tables, dim3((nt + 255) / 256), dim3(256), 0, s, rd, X, Y, ndir, px, py, kp);
  FF_HIP(hipGetLastError());
  FfArgs a{};
  a.D = ndir;
  a.N = N;
  a.ne = ne;
  a.px = px;
  a.py = py;
  a.R = nrhs;
  a.k = op->arr.k;
  a.rhat = rd;
  a.X = X;
  a.Y = Y;
  a.quad = op->ff_quad;
  a.part = part;
  hipLaunchKernelGGL(k_ff_gemm, dim3((ndir + kFfD - 1) / kFfD, ntiles, nrhs), dim3(256), 0, s, uT, a);
  FF_HIP(hipGetLastError());
  const double keta = (system == AIM_FULL ? -1.0 : 1.0) * op->arr.k * op->arr.eta;
  hipLaunchKernelGGL(k_ff_finish, dim3((nrhs * ndir + 255) / 256), dim3(256), 0, s, part, rd,
                     static_cast<cplx<double>*>(E), static_cast<double*>(rcs_db), ndir, nrhs, ntiles, keta);
  FF_HIP(hipGetLastError());
  return AIM_OK;
}

}  // namespace

extern "C" int aim_far_field(aim_op* op, const void* x, int32_t nrhs, int32_t ndir, const double* rhat, void* E,
                             void* rcs_db, int32_t system, void* stream) {
  const int rc = ff_check(op, x, nrhs, ndir, rhat, E, system);
  if (rc != AIM_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ntiles = (op->N + kFfN - 1) / kFfN;
  try {
    // workspace: directions, phase tables and per-tile partials, grown on demand
    const size_t need = ff_need_bytes(ndir, op->arr.px, op->arr.py, ntiles, op->R_max);
    if (need > op->ff_bytes) {
      if (op->ff_ws) {
        FF_HIP(hipStreamSynchronize(s));
        op->mem.release(op->ff_ws, op->ff_bytes);
        op->ff_ws = nullptr;
        op->ff_bytes = 0;
      }
      op->ff_ws = op->mem.alloc<unsigned char>(need);
      op->ff_bytes = need;
    }
  } catch (const std::bad_alloc&) {
    set_error("far field: device allocation failed");
    return AIM_ENOMEM;
  }
  return ff_run(op, x, nrhs, ndir, rhat, E, rcs_db, system, s, static_cast<unsigned char*>(op->ff_ws));
}

extern "C" int aim_far_field_noalloc(aim_op* op, const void* x, int32_t nrhs, int32_t ndir, const double* rhat,
                                     void* E, void* rcs_db, int32_t system, void* stream) {
  const int rc = ff_check(op, x, nrhs, ndir, rhat, E, system);
  if (rc != AIM_OK) return rc;
  const int ntiles = (op->N + kFfN - 1) / kFfN;
  const size_t need = ff_need_bytes(ndir, op->arr.px, op->arr.py, ntiles, nrhs);
  if (need > kFfScratchBytes) {
    set_error("far field (no allocation): the call needs " + std::to_string(need) +
              " bytes of workspace, more than the " + std::to_string(kFfScratchBytes) +
              "-byte scratch array; use fewer directions or right-hand sides per call");
    return AIM_EINVAL;
  }
  void* ws = ff_scratch_lookup(op->device);  // resolved when the op was built
  if (!ws) {
    set_error("far field (no allocation): scratch address of the op's device is not set");
    return AIM_ESTATE;
  }
  return ff_run(op, x, nrhs, ndir, rhat, E, rcs_db, system, static_cast<hipStream_t>(stream),
                static_cast<unsigned char*>(ws));
}
