// C ABI of the library: operator construction, the final-system product of
// eq. MV_product1 and its parts.  GMRES lives in gmres.hip.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>

#include "../../include/aimm.h"
#include "op.hpp"
#include "precond.hpp"

namespace aimm {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }

#define AIM_HIP(expr)                                                                    \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      set_error(std::string(#expr) + ": " + hipGetErrorString(_e));                      \
      return AIM_EDEVICE;                                                                \
    }                                                                                    \
  } while (0)

static FftPlan make_plan(int L, std::vector<int>& rev, std::vector<int>& pos) {
  std::vector<int> f = radix_plan(L);
  if (f.empty() || int(f.size()) > kMaxStages) throw std::invalid_argument("FFT length not 5-smooth");
  FftPlan P{};
  P.L = L;
  P.nst = int(f.size());
  int B = L;
  for (int s = 0; s < P.nst; ++s) {
    P.radix[s] = f[s];
    P.stride[s] = B / f[s];
    P.tw_step[s] = L / B;
    P.div_nb[s] = magic_div(unsigned(L / f[s]));
    P.div_S[s] = magic_div(unsigned(P.stride[s]));
    B = P.stride[s];
  }
  rev.assign(L, 0);
  pos.assign(L, 0);
  for (int p = 0; p < L; ++p) {
    int rem = p, k = 0, mult = 1;
    for (int s = 0; s < P.nst; ++s) {
      const int qd = rem / P.stride[s];
      rem -= qd * P.stride[s];
      k += qd * mult;
      mult *= P.radix[s];
    }
    rev[p] = k;
    pos[k] = p;
  }
  return P;
}

template <typename T>
static void twiddles(int L, std::vector<cplx<T>>& out) {
  out.resize(L);
  for (int t = 0; t < L; ++t) {
    const long double a = -2.0L * 3.141592653589793238462643383279502884L * (long double)t / (long double)L;
    out[t].re = T(std::cos(a));
    out[t].im = T(std::sin(a));
  }
}

// Copy of host data to new device memory, on the stream the op is built on (the copy has
// completed on return).
template <typename T>
static T* upload(aim_op* op, const T* host, size_t n) {
  T* d = op->mem.alloc<T>(n);
  if (n && (hipMemcpyAsync(d, host, n * sizeof(T), hipMemcpyHostToDevice, op->build_stream) != hipSuccess ||
            hipStreamSynchronize(op->build_stream) != hipSuccess))
    throw std::runtime_error("hipMemcpy upload failed");
  return d;
}

// bf16 round-to-nearest-even of a finite float, and v = h + m + l in bf16 terms (each
// remainder is exact in FP32)
static uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
static float bf16_to_float(uint16_t b) {
  const uint32_t u = uint32_t(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
static void split_bf16(float v, uint16_t out[3]) {
  out[0] = bf16_rne(v);
  const float r1 = v - bf16_to_float(out[0]);
  out[1] = bf16_rne(r1);
  out[2] = bf16_rne(r1 - bf16_to_float(out[1]));
}

template <typename T>
static void fill_prec(aim_op* op, PrecData<T>& P) {
  const Setup& st = op->st;
  const int N = st.N, q3 = st.q3;
  std::vector<T> Wp(st.W.size()), Wt(st.W.size());
  for (int p = 0; p < 4; ++p)
    for (int n = 0; n < N; ++n)
      for (int s = 0; s < q3; ++s) Wt[(size_t(p) * q3 + s) * N + n] = T(st.W[(size_t(p) * N + n) * q3 + s]);
  // projection: the four weights of each gather entry, in gather-table order
  for (size_t e = 0; e < st.node_ent.size(); ++e)
    for (int p = 0; p < 4; ++p) Wp[e * 4 + p] = T(st.W[size_t(p) * N * q3 + st.node_ent[e]]);
  P.Wp = upload(op, Wp.data(), Wp.size());
  P.Wt = upload(op, Wt.data(), Wt.size());
  std::vector<cplx<T>> nv(st.near_val.size());
  for (size_t i = 0; i < nv.size(); ++i) {
    nv[i].re = T(st.near_val[i].real());
    nv[i].im = T(st.near_val[i].imag());
  }
  P.near = upload(op, nv.data(), nv.size());
  std::vector<cplx<T>> ga(st.grp_A.size());
  for (size_t i = 0; i < ga.size(); ++i) {
    ga[i].re = T(st.grp_A[i].real());
    ga[i].im = T(st.grp_A[i].imag());
  }
  P.grpA = upload(op, ga.data(), ga.size());
  std::vector<cplx<T>> tw;
  twiddles<T>(op->Lx, tw);
  P.tw_x = upload(op, tw.data(), tw.size());
  twiddles<T>(op->Ly, tw);
  P.tw_y = upload(op, tw.data(), tw.size());
  P.gt = op->mem.alloc<cplx<T>>(size_t(op->Lx / 2 + 1) * (op->Ly / 2 + 1) * st.nz);
  // ky lines per workgroup in the spectrum pass: the widest allowed value whose
  // workgroup fits LDS.  One line block (B = 1) measured fastest on the 400 x 400 grid
  // (more workgroups in flight); AIMM_FFT_B raises the maximum.
  int bmax = 1;
  if (const char* env = std::getenv("AIMM_FFT_B")) bmax = std::max(1, std::atoi(env));
  P.B = 1;
  for (int B = bmax; B >= 2; --B) {
    if (conv_fits(op->Lx, op->Ly, st.nz, B, op->fft4, sizeof(cplx<T>), std::min<size_t>(op->lds_max, 160 * 1024))) {
      P.B = B;
      break;
    }
  }
}

template <typename T>
static ConvArgs conv_args(aim_op* op, const PrecData<T>& P, int R) {
  ConvArgs a{};
  a.R = R;
  a.nx = op->st.nx;
  a.ny = op->st.ny;
  a.nz = op->st.nz;
  a.B = P.B;
  a.f4 = op->fft4 ? 1 : 0;
  a.Px = op->Px;
  a.Py = op->Py;
  a.tw_x = P.tw_x;
  a.tw_y = P.tw_y;
  a.gt = P.gt;
  a.rev_x = op->rev_x;
  a.rev_y = op->rev_y;
  a.passes = 7;
  a.x_out = nullptr;
  return a;
}

static ProjArgs proj_args(aim_op* op, int R) {
  const Setup& st = op->st;
  ProjArgs a{};
  a.R = R;
  a.ne = op->ne;
  a.N = st.N;
  a.px = op->arr.px;
  a.py = op->arr.py;
  a.pitch = op->arr.pitch;
  a.ex = st.ex;
  a.ey = st.ey;
  a.ez = st.ez;
  a.nx = st.nx;
  a.ny = st.ny;
  a.nz = st.nz;
  a.q3 = st.q3;
  a.node_ptr = op->node_ptr;
  a.node_n = op->node_n;
  a.zero = op->zero;
  return a;
}

static NearArgs near_args(aim_op* op, int R) {
  const Setup& st = op->st;
  NearArgs a{};
  a.R = R;
  a.ne = op->ne;
  a.N = st.N;
  a.px = op->arr.px;
  a.py = op->arr.py;
  a.offsets = op->offsets_d;
  a.grp_ptr = op->grp_ptr;
  a.grp_col = op->grp_col;
  a.grp_row = op->grp_row;
  a.slot_of = op->slot_of;
  a.grp_A = nullptr;
  a.zero = op->zero;
  a.grp_max_cols = op->st.grp_max_cols;
  a.ld_nf = int(op->st.grp_row.size());
  a.near_ptr = op->near_ptr;
  a.near_col = op->near_col;
  return a;
}

template <typename T>
static InterpArgs interp_args(aim_op* op, int R) {
  const Setup& st = op->st;
  InterpArgs a{};
  a.R = R;
  a.ne = op->ne;
  a.N = st.N;
  a.px = op->arr.px;
  a.py = op->arr.py;
  a.pitch = op->arr.pitch;
  a.nx = st.nx;
  a.ny = st.ny;
  a.nz = st.nz;
  a.q = st.q;
  a.q3 = st.q3;
  a.ex = st.ex;
  a.ey = st.ey;
  a.keta = op->arr.k * op->arr.eta;
  a.sig_phi = -1.0 / (op->arr.k * op->arr.k);
  a.sloc = op->sloc;
  a.d_colT = op->d_colT;
  a.dmax = op->d_max;
  a.slot_of = op->slot_of;
  a.ld_nf = int(op->st.grp_row.size());
  // element tile of the interpolation workgroup: the projection weights are loaded
  // once per tile, the tile's box of potentials must fit LDS
  // (one element per workgroup measured fastest on the 32 x 32 array)
  a.TX = op->interp_tx > 0 ? op->interp_tx : 1;
  a.TY = op->interp_ty > 0 ? op->interp_ty : 1;
  while (a.TX * a.TY > 4 || interp_lds_bytes(a, sizeof(cplx<T>)) > op->lds_max) {
    if (a.TY > 1)
      a.TY = 1;
    else if (a.TX > 1)
      a.TX = 1;
    else
      break;
  }
  return a;
}

static GemmArgs gemm_args(aim_op* op, int R) {
  GemmArgs a{};
  a.N = op->N;
  a.ne = op->ne;
  a.R = R;
  a.n_types = op->n_types;
  a.Kq = gemm_kq(op->N);
  a.Krows = gemm_krows(op->N);
  a.Mb = op->gemm_bf16 ? op->Mb : nullptr;
  a.col_list = op->col_list;
  a.tile_start[0] = 0;
  for (int t = 0; t < op->n_types; ++t) {
    a.type_count[t] = op->type_count[t];
    a.col_start[t] = op->col_start[t];
    a.tile_start[t + 1] = a.tile_start[t] + (R * op->type_count[t] + kGemmColsHost - 1) / kGemmColsHost;
  }
  return a;
}

GemmArgs gemm_args_of(aim_op* op, int R) { return gemm_args(op, R); }

template <typename T>
PrecData<T>& prec_data(aim_op* op);
template <>
PrecData<double>& prec_data<double>(aim_op* op) {
  return op->p64;
}
template <>
PrecData<float>& prec_data<float>(aim_op* op) {
  return op->p32;
}

static int check_common(aim_op* op, const void* a, const void* b, int32_t nrhs, int32_t precision) {
  if (!op) {
    set_error("op is NULL");
    return AIM_EINVAL;
  }
  if (!op->device_ready) {
    set_error("op was built without device data (aim_build_host)");
    return AIM_ESTATE;
  }
  if (!a || !b) {
    set_error("device pointers must not be NULL");
    return AIM_EINVAL;
  }
  if (nrhs < 1 || nrhs > op->R_max) {
    set_error("nrhs must be in [1, max_rhs]");
    return AIM_EINVAL;
  }
  if (precision != AIM_FP64 && precision != AIM_MIXED) {
    set_error("precision must be AIM_FP64 or AIM_MIXED");
    return AIM_EINVAL;
  }
  return AIM_OK;
}

// ev (optional): 8 events, recorded before the first kernel and after each of the
// seven (GEMM or transpose, projection, three FFT passes, near field, interpolation).
template <typename T>
int matvec_impl(aim_op* op, const cplx<T>* x, cplx<T>* y, int R, int flags, hipStream_t s, hipEvent_t* ev = nullptr) {
  PrecData<T>& P = prec_data<T>(op);
  cplx<T>* uT = static_cast<cplx<T>*>(op->u);
  cplx<T>* nf = static_cast<cplx<T>*>(op->nf);
  cplx<T>* grid = static_cast<cplx<T>*>(op->grid);
  cplx<T>* S = static_cast<cplx<T>*>(op->S);
  if (ev) AIM_HIP(hipEventRecord(ev[0], s));
  if (flags == AIM_FULL)
    AIM_HIP(launch_macro<T>(P.M, x, uT, gemm_args(op, R), s));
  else
    AIM_HIP(launch_transpose<T>(x, uT, R, op->ne, op->N, s));
  if (ev) AIM_HIP(hipEventRecord(ev[1], s));
  // the near field depends on u only: it runs on the op's second stream, concurrently
  // with the projection and the FFT passes (in order on one stream when timing kernels)
  NearArgs na = near_args(op, R);
  if (op->near_mfma) na.grp_A = P.grpA;
  na.eb = op->near_eb[sizeof(T) == sizeof(double) ? 0 : 1];
  const bool fork = !ev && op->s_aux && flags != AIM_FAR_ONLY;
  // the near field leaves the caller's stream at fork point fp (0 after the macromodel
  // product, 1 after the projection, 2 after the y pass), so that it overlaps the kernels
  // that follow; the results do not depend on the point
  const int fp = fork ? op->near_fork[sizeof(T) == sizeof(double) ? 0 : 1] : -1;
  auto fork_near = [&]() -> hipError_t {
    hipError_t e = hipEventRecord(op->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(op->s_aux, op->ev_fork, 0);
    if (e == hipSuccess) e = launch_near<T>(uT, nf, na, P.near, op->s_aux);
    if (e == hipSuccess) e = hipEventRecord(op->ev_join, op->s_aux);
    return e;
  };
  if (fp == 0) AIM_HIP(fork_near());
  AIM_HIP(launch_project<T>(uT, grid, proj_args(op, R), P.Wp, s));
  if (ev) AIM_HIP(hipEventRecord(ev[2], s));
  if (fp <= 1) {
    if (fp == 1) AIM_HIP(fork_near());
    AIM_HIP(launch_convolve<T>(grid, grid, S, conv_args(op, P, R), s, ev ? ev + 3 : nullptr));
  } else {
    ConvArgs ca = conv_args(op, P, R);
    ca.passes = 1;  // y pass
    AIM_HIP(launch_convolve<T>(grid, grid, S, ca, s, nullptr));
    AIM_HIP(fork_near());
    ca.passes = 2 | 4;  // x pass with the spectrum product, inverse y pass
    AIM_HIP(launch_convolve<T>(grid, grid, S, ca, s, nullptr));
  }
  if (ev) AIM_HIP(hipEventRecord(ev[5], s));
  if (fork)
    AIM_HIP(hipStreamWaitEvent(s, op->ev_join, 0));
  else if (flags != AIM_FAR_ONLY)
    AIM_HIP(launch_near<T>(uT, nf, na, P.near, s));
  if (ev) AIM_HIP(hipEventRecord(ev[6], s));
  AIM_HIP(launch_interp<T>(flags, grid, nf, x, y, interp_args<T>(op, R), P.Wt, P.dval, s));
  if (ev) AIM_HIP(hipEventRecord(ev[7], s));
  return AIM_OK;
}

template int matvec_impl<double>(aim_op*, const cplx<double>*, cplx<double>*, int, int, hipStream_t, hipEvent_t*);
template int matvec_impl<float>(aim_op*, const cplx<float>*, cplx<float>*, int, int, hipStream_t, hipEvent_t*);

// y = blockdiag(P_t(m)) x, element-major in and out (grouped product, then the
// transpose from its element-fastest output)
template <typename T>
int precond_impl(aim_op* op, const cplx<T>* x, cplx<T>* y, int R, hipStream_t s) {
  cplx<T>* uT = static_cast<cplx<T>*>(op->u);
  GemmArgs a = gemm_args(op, R);
  a.Mb = op->gemm_bf16 ? op->Pb : nullptr;
  const cplx<T>* P;
  if constexpr (sizeof(T) == sizeof(double))
    P = op->P64;
  else
    P = op->P32;
  AIM_HIP(launch_macro<T>(P, x, uT, a, s));
  AIM_HIP(launch_transpose<T>(uT, y, R, op->N, op->ne, s));
  return AIM_OK;
}
template int precond_impl<double>(aim_op*, const cplx<double>*, cplx<double>*, int, hipStream_t);
template int precond_impl<float>(aim_op*, const cplx<float>*, cplx<float>*, int, hipStream_t);

// Per-kernel durations: after one full product (so every intermediate buffer holds
// its real data), each of the seven kernels is launched once untimed and then reps
// times back to back between two events on s.  Each launch rewrites only its own
// output from inputs that no launch of the loop changes, so the repetitions are
// identical; the in-place x pass writes to a temporary buffer instead of its input.
// A last full product leaves y valid.
template <typename T>
static int time_kernels(aim_op* op, const cplx<T>* x, cplx<T>* y, int R, int reps, double* ms, hipStream_t s) {
  PrecData<T>& P = prec_data<T>(op);
  cplx<T>* uT = static_cast<cplx<T>*>(op->u);
  cplx<T>* nf = static_cast<cplx<T>*>(op->nf);
  cplx<T>* grid = static_cast<cplx<T>*>(op->grid);
  cplx<T>* S = static_cast<cplx<T>*>(op->S);
  const size_t spec = size_t(R) * 4 * op->st.nx * op->Ly * op->st.nz;
  cplx<T>* Sx = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&Sx), spec * sizeof(cplx<T>)) != hipSuccess) {
    set_error("out of device memory for the timing buffer");
    return AIM_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = AIM_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("event creation failed");
    rc = AIM_EDEVICE;
  }
  NearArgs na = near_args(op, R);
  if (op->near_mfma) na.grp_A = P.grpA;
  na.eb = op->near_eb[sizeof(T) == sizeof(double) ? 0 : 1];
  const GemmArgs ga = gemm_args(op, R);
  const ProjArgs pa = proj_args(op, R);
  const InterpArgs ia = interp_args<T>(op, R);
  auto stage = [&](int k) -> hipError_t {
    ConvArgs ca = conv_args(op, P, R);
    switch (k) {
      case 0: return launch_macro<T>(P.M, x, uT, ga, s);
      case 1: return launch_project<T>(uT, grid, pa, P.Wp, s);
      case 2: ca.passes = 1; return launch_convolve<T>(grid, nullptr, S, ca, s, nullptr);
      case 3: ca.passes = 2; ca.x_out = Sx; return launch_convolve<T>(nullptr, nullptr, S, ca, s, nullptr);
      case 4: ca.passes = 4; return launch_convolve<T>(nullptr, grid, S, ca, s, nullptr);
      case 5: return launch_near<T>(uT, nf, na, P.near, s);
      default: return launch_interp<T>(AIM_FULL, grid, nf, x, y, ia, P.Wt, P.dval, s);
    }
  };
  if (rc == AIM_OK) rc = matvec_impl<T>(op, x, y, R, AIM_FULL, s, nullptr);
  for (int k = 0; k < 7 && rc == AIM_OK; ++k) {
    hipError_t he = stage(k);
    if (he == hipSuccess) he = hipEventRecord(e0, s);
    for (int it = 0; it < reps && he == hipSuccess; ++it) he = stage(k);
    if (he == hipSuccess) he = hipEventRecord(e1, s);
    if (he == hipSuccess) he = hipEventSynchronize(e1);
    float t = 0;
    if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    if (he != hipSuccess) {
      set_error(std::string("kernel timing failed: ") + hipGetErrorString(he));
      rc = AIM_EDEVICE;
      break;
    }
    ms[k] = double(t) / reps;
  }
  if (rc == AIM_OK) rc = matvec_impl<T>(op, x, y, R, AIM_FULL, s, nullptr);
  if (hipStreamSynchronize(s) != hipSuccess && rc == AIM_OK) {
    set_error("stream synchronisation failed");
    rc = AIM_EDEVICE;
  }
  (void)hipFree(Sx);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace aimm

using namespace aimm;

extern "C" {

const char* aim_last_error(void) { return aimm::g_err.c_str(); }

static int build_op(const aim_surface* surface, const aim_array* array, aim_op** out, bool device,
                    hipStream_t stream) {
  if (!surface || !array || !out) {
    set_error("surface, array and out must not be NULL");
    return AIM_EINVAL;
  }
  SurfaceIn s;
  s.n_vert = surface->n_vert;
  s.n_tri = surface->n_tri;
  s.n_rwg = surface->n_rwg;
  s.vert = surface->vert;
  s.tri = surface->tri;
  s.rwg = surface->rwg;
  ArrayIn a;
  a.k = array->k;
  a.eta = array->eta;
  a.h = array->h;
  a.r_near = array->r_near;
  a.order = array->order;
  a.px = array->px;
  a.py = array->py;
  a.pitch = array->pitch_cells;
  a.n_types = array->n_types;
  a.elem_type = array->elem_type;
  a.max_rhs = array->max_rhs;
  aim_op* op = nullptr;
  try {
    validate(s, a);
    if (a.n_types > kMaxTypes) throw std::invalid_argument("n_types exceeds 16");
    op = new aim_op();
    op->build_stream = stream;
    op->vert.assign(s.vert, s.vert + 3 * s.n_vert);
    op->tri.assign(s.tri, s.tri + 3 * s.n_tri);
    op->rwg.assign(s.rwg, s.rwg + 4 * s.n_rwg);
    op->elem_type.assign(a.elem_type, a.elem_type + a.px * a.py);
    s.vert = op->vert.data();
    s.tri = op->tri.data();
    s.rwg = op->rwg.data();
    a.elem_type = op->elem_type.data();
    op->arr = a;
    build_setup(s, a, op->st);
    Setup& st = op->st;
    if (st.nz > kMaxNz) throw std::invalid_argument("grid extent along z exceeds 16 nodes");
    if (st.offsets.size() / 2 > size_t(kMaxOffsets)) throw std::invalid_argument("too many near-field offsets");
    op->ne = a.px * a.py;
    op->N = st.N;
    op->R_max = a.max_rhs;
    op->n_types = a.n_types;
    op->Lx = smooth_length(std::max(2 * st.nx - 2, st.nx));
    op->Ly = smooth_length(std::max(2 * st.ny - 2, st.ny));
    std::vector<int> rx, px_, ry, py_;
    op->Px = make_plan(op->Lx, rx, px_);
    op->Py = make_plan(op->Ly, ry, py_);
    if (!device) {
      *out = op;
      return AIM_OK;
    }
    op->device_ready = true;
    // a default-priority stream for the near field, joined back by events; they order
    // work between two streams of this device only, so a device-scope release and
    // acquire suffice (no system-scope cache write-back and invalidation)
    if (hipStreamCreateWithFlags(&op->s_aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess)
      throw std::runtime_error("stream or event creation failed");
    if (const char* env = std::getenv("AIMM_SERIAL")) {
      if (std::atoi(env) != 0) {
        (void)hipStreamDestroy(op->s_aux);
        op->s_aux = nullptr;
      }
    }
    if (hipGetDevice(&op->device) != hipSuccess) throw std::runtime_error("no HIP device");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, op->device) != hipSuccess) throw std::runtime_error("device query failed");
    op->lds_max = prop.sharedMemPerBlock;
    // integer tables
    op->sloc = upload(op, st.sloc.data(), st.sloc.size());
    op->node_ptr = upload(op, st.node_ptr.data(), st.node_ptr.size());
    // projection gather entries as offsets n * n_elem into the element-fastest u
    if (int64_t(st.N) * op->ne > INT32_MAX) throw std::invalid_argument("n_rwg * n_elem exceeds 2^31");
    std::vector<int32_t> noff(st.node_n.size());
    for (size_t e = 0; e < noff.size(); ++e) noff[e] = st.node_n[e] * op->ne;
    op->node_n = upload(op, noff.data(), noff.size());
    op->near_ptr = upload(op, st.near_ptr.data(), st.near_ptr.size());
    op->near_col = upload(op, st.near_col.data(), st.near_col.size());
    op->rev_x = upload(op, rx.data(), rx.size());
    op->rev_y = upload(op, ry.data(), ry.size());
    const int n_off = int(st.offsets.size() / 2);
    std::vector<int> nbr(size_t(op->ne) * std::max(n_off, 1), -1);
    for (int m = 0; m < op->ne; ++m) {
      const int ix = m % a.px, iy = m / a.px;
      for (int o = 0; o < n_off; ++o) {
        const int jx = ix + st.offsets[2 * o], jy = iy + st.offsets[2 * o + 1];
        if (jx >= 0 && jx < a.px && jy >= 0 && jy < a.py) nbr[size_t(m) * n_off + o] = jy * a.px + jx;
      }
    }
    op->nbr = upload(op, nbr.data(), nbr.size());
    op->offsets_d = upload(op, st.offsets.data(), st.offsets.size());
    op->grp_ptr = upload(op, st.grp_ptr.data(), st.grp_ptr.size());
    {
      // matrix-core near-field columns as (n' ne + dx + dy px) << 5 | (dy + 2) 5 + (dx + 2):
      // the offset of the neighbour's u from the element's own and a 5 x 5 validity slot
      std::vector<int32_t> gc(st.grp_col.size());
      const int64_t lim = int64_t(1) << 25;
      for (size_t i = 0; i < gc.size(); ++i) {
        const int c = st.grp_col[i];
        const int np_ = c & 0xFFFF, dx = ((c >> 16) & 0xFF) - 8, dy = ((c >> 24) & 0xFF) - 8;
        const int64_t off = int64_t(np_) * op->ne + dx + int64_t(dy) * a.px;
        if (std::abs(dx) > 2 || std::abs(dy) > 2 || off >= lim || off <= -lim) op->near_mfma = false;
        gc[i] = int32_t(off * 32 + (dy + 2) * 5 + (dx + 2));
      }
      op->grp_col = upload(op, gc.data(), gc.size());
    }
    op->grp_row = upload(op, st.grp_row.data(), st.grp_row.size());
    op->slot_of = upload(op, st.slot_of.data(), st.slot_of.size());
    {
      const cplx<double> z{0.0, 0.0};
      op->zero = upload(op, &z, 1);
    }
    if (const char* env = std::getenv("AIMM_NEAR_CSR")) op->near_mfma = op->near_mfma && std::atoi(env) == 0;
    // register-DFT FFT passes where both padded lengths have a compiled factorisation
    op->fft4 = fft4_supported(op->Lx) && fft4_supported(op->Ly);
    if (const char* env = std::getenv("AIMM_FFT4")) op->fft4 = op->fft4 && std::atoi(env) != 0;
    // the matrix-core kernel stages a group's columns in LDS
    if (size_t(st.grp_max_cols) * sizeof(int) > 32768) op->near_mfma = false;
    // split-BF16 macromodel product in the mixed path (AIMM_GEMM=fp32 selects the FP32 kernel)
    op->gemm_bf16 = op->N % 8 == 0;
    if (const char* env = std::getenv("AIMM_GEMM")) op->gemm_bf16 = op->gemm_bf16 && std::strcmp(env, "fp32") != 0;
    if (const char* env = std::getenv("AIMM_INTERP_TILE")) std::sscanf(env, "%dx%d", &op->interp_tx, &op->interp_ty);
    // macromodel column lists, r-major within each kind
    op->type_count.assign(a.n_types, 0);
    op->col_start.assign(a.n_types, 0);
    std::vector<int> cols;
    for (int t = 0; t < a.n_types; ++t) {
      op->col_start[t] = int(cols.size());
      std::vector<int> el;
      for (int m = 0; m < op->ne; ++m)
        if (a.elem_type[m] == t) el.push_back(m);
      op->type_count[t] = int(el.size());
      for (int r = 0; r < a.max_rhs; ++r)
        for (int m : el) cols.push_back(r * op->ne + m);
    }
    op->col_list = upload(op, cols.data(), cols.size());
    fill_prec(op, op->p64);
    fill_prec(op, op->p32);
    // FFT workgroups may need more than the default dynamic LDS
    const size_t lmax = std::min<size_t>(op->lds_max, 160 * 1024);
    (void)configure_lds(lmax);
    // kernel spectrum on the device (FP64), then stored in both precisions
    {
      const size_t lds_y = sizeof(cplx<double>) * size_t(op->Ly) * (1 + st.nz);
      const size_t lds_x = sizeof(cplx<double>) * size_t(op->Lx) * (1 + st.nz);
      if (lds_y > op->lds_max || lds_x > op->lds_max)
        throw std::invalid_argument("padded grid too large for one workgroup's LDS in FP64");
      cplx<double>* raw = op->mem.alloc<cplx<double>>(size_t(op->Lx) * op->Ly * st.nz);
      int* pxd = upload(op, px_.data(), px_.size());
      int* pyd = upload(op, py_.data(), py_.size());
      hipError_t e = launch_spectrum(raw, op->Lx, op->Ly, st.nz, a.k, a.h, op->Px, op->Py, op->p64.tw_x,
                                     op->p64.tw_y, 1, op->build_stream);
      if (e == hipSuccess)
        e = launch_extract<double>(raw, op->p64.gt, op->Lx, op->Ly, st.nz, pxd, pyd, op->build_stream);
      if (e == hipSuccess)
        e = launch_extract<float>(raw, op->p32.gt, op->Lx, op->Ly, st.nz, pxd, pyd, op->build_stream);
      if (e == hipSuccess) e = hipStreamSynchronize(op->build_stream);
      if (e != hipSuccess) throw std::runtime_error(std::string("spectrum build: ") + hipGetErrorString(e));
      op->mem.release(raw, sizeof(cplx<double>) * size_t(op->Lx) * op->Ly * st.nz);
      op->mem.release(pxd, sizeof(int) * px_.size());
      op->mem.release(pyd, sizeof(int) * py_.size());
    }
    // workspaces, sized for complex128
    const size_t n_unk = size_t(op->ne) * op->N * a.max_rhs;
    op->u = op->mem.alloc<cplx<double>>(n_unk);
    op->nf = op->mem.alloc<cplx<double>>(size_t(op->ne) * st.grp_row.size() * a.max_rhs);
    op->grid = op->mem.alloc<cplx<double>>(size_t(a.max_rhs) * 4 * st.nx * st.ny * st.nz);
    op->S = op->mem.alloc<cplx<double>>(size_t(a.max_rhs) * 4 * st.nx * op->Ly * st.nz);
    ff_prepare(op);
    // later uploads (operator data, preconditioner) run on the null stream: the build
    // stream may not outlive this call
    op->build_stream = nullptr;
  } catch (const std::bad_alloc&) {
    delete op;
    set_error("device or host allocation failed");
    return AIM_ENOMEM;
  } catch (const std::invalid_argument& e) {
    delete op;
    set_error(e.what());
    return AIM_EINVAL;
  } catch (const std::exception& e) {
    delete op;
    set_error(e.what());
    return AIM_EDEVICE;
  }
  *out = op;
  return AIM_OK;
}

int aim_build_grid(const aim_surface* surface, const aim_array* array, void* stream, aim_op** out) {
  return build_op(surface, array, out, true, static_cast<hipStream_t>(stream));
}

int aim_build_host(const aim_surface* surface, const aim_array* array, aim_op** out) {
  return build_op(surface, array, out, false, nullptr);
}

int aim_get_tuning(const aim_op* op, aim_tuning* t) {
  if (!op || !t) {
    set_error("op and tuning must not be NULL");
    return AIM_EINVAL;
  }
  t->fft_b[0] = op->p64.B;
  t->fft_b[1] = op->p32.B;
  t->interp_tx = op->interp_tx > 0 ? op->interp_tx : 1;
  t->interp_ty = op->interp_ty > 0 ? op->interp_ty : 1;
  t->gemm_bf16 = op->gemm_bf16 ? 1 : 0;
  t->fft_register = op->fft4 ? 1 : 0;
  t->near_block[0] = op->near_eb[0];
  t->near_block[1] = op->near_eb[1];
  t->near_fork[0] = op->near_fork[0];
  t->near_fork[1] = op->near_fork[1];
  return AIM_OK;
}

int aim_set_tuning(aim_op* op, const aim_tuning* t) {
  if (!op || !t) {
    set_error("op and tuning must not be NULL");
    return AIM_EINVAL;
  }
  if (!op->device_ready) {
    set_error("tuning: host-only op");
    return AIM_ESTATE;
  }
  if (t->fft_register == 1 && !(fft4_supported(op->Lx) && fft4_supported(op->Ly))) {
    set_error("tuning: no register-DFT FFT pass for these padded lengths");
    return AIM_EINVAL;
  }
  // the FFT passes must launch with the line blocks and pass kind in force afterwards
  const int nz = op->st.nz;
  const size_t lmax = std::min<size_t>(op->lds_max, 160 * 1024);
  const bool f4 = t->fft_register >= 0 ? t->fft_register == 1 : op->fft4;
  for (int p = 0; p < 2; ++p) {
    if (t->fft_b[p] < 0) {
      set_error("tuning: fft_b must be >= 0 (0 keeps the current value)");
      return AIM_EINVAL;
    }
    const int B = t->fft_b[p] > 0 ? t->fft_b[p] : (p == 0 ? op->p64.B : op->p32.B);
    const size_t elem = p == 0 ? sizeof(cplx<double>) : sizeof(cplx<float>);
    if (!conv_fits(op->Lx, op->Ly, nz, B, f4, elem, lmax)) {
      set_error("tuning: fft_b must divide the padded y length and its x-pass workgroup must fit (threads, LDS)");
      return AIM_EINVAL;
    }
  }
  if (t->interp_tx != 0 || t->interp_ty != 0) {
    if (t->interp_tx < 1 || t->interp_ty < 1 || t->interp_tx * t->interp_ty > 4) {
      set_error("tuning: interpolation tile must be tx x ty >= 1 with tx ty <= 4");
      return AIM_EINVAL;
    }
    // checked in FP32; FP64 launches use the largest tile at most this size that fits
    InterpArgs ia = interp_args<float>(op, 1);
    ia.TX = t->interp_tx;
    ia.TY = t->interp_ty;
    if (interp_lds_bytes(ia, sizeof(cplx<float>)) > op->lds_max) {
      set_error("tuning: the interpolation tile's potentials do not fit one workgroup's LDS");
      return AIM_EINVAL;
    }
  }
  for (int p = 0; p < 2; ++p)
    if (t->near_block[p] < 0 || t->near_block[p] > 2) {
      set_error("tuning: near_block must be 1 or 2 element blocks per workgroup (0 keeps the current value)");
      return AIM_EINVAL;
    }
  for (int p = 0; p < 2; ++p)
    if (t->near_fork[p] < -1 || t->near_fork[p] > 2) {
      set_error("tuning: near_fork must be 0 (after the GEMM), 1 (after the projection) or 2 (after the y pass); "
                "-1 keeps the current value");
      return AIM_EINVAL;
    }
  if (t->gemm_bf16 == 1 && op->N % 8 != 0) {
    set_error("tuning: the split-BF16 product needs N % 8 == 0");
    return AIM_EINVAL;
  }
  if (t->fft_b[0] > 0) op->p64.B = t->fft_b[0];
  if (t->fft_b[1] > 0) op->p32.B = t->fft_b[1];
  if (t->interp_tx > 0) {
    op->interp_tx = t->interp_tx;
    op->interp_ty = t->interp_ty;
  }
  if (t->gemm_bf16 >= 0) op->gemm_bf16 = t->gemm_bf16 == 1;
  if (t->fft_register >= 0) op->fft4 = t->fft_register == 1;
  for (int p = 0; p < 2; ++p)
    if (t->near_block[p] > 0) op->near_eb[p] = t->near_block[p];
  for (int p = 0; p < 2; ++p)
    if (t->near_fork[p] >= 0) op->near_fork[p] = t->near_fork[p];
  ++op->graph_epoch;  // captured GMRES iterations carry the old launch arguments
  return AIM_OK;
}

int aim_set_elem_type(aim_op* op, const int32_t* elem_type, void* stream) {
  if (!op || !elem_type) {
    set_error("op and elem_type must not be NULL");
    return AIM_EINVAL;
  }
  for (int m = 0; m < op->ne; ++m)
    if (elem_type[m] < 0 || elem_type[m] >= op->n_types) {
      set_error("element kind out of range");
      return AIM_EINVAL;
    }
  std::vector<int> count(op->n_types, 0), start(op->n_types, 0), cols;
  cols.reserve(size_t(op->ne) * op->R_max);
  for (int t = 0; t < op->n_types; ++t) {
    start[t] = int(cols.size());
    std::vector<int> el;
    for (int m = 0; m < op->ne; ++m)
      if (elem_type[m] == t) el.push_back(m);
    count[t] = int(el.size());
    for (int r = 0; r < op->R_max; ++r)
      for (int m : el) cols.push_back(r * op->ne + m);
  }
  if (op->device_ready) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(op->col_list, cols.data(), cols.size() * sizeof(int), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("element kinds: device copy failed");
      return AIM_EDEVICE;
    }
  }
  op->type_count.swap(count);
  op->col_start.swap(start);
  ++op->graph_epoch;  // captured GMRES iterations carry the old kind counts
  std::copy(elem_type, elem_type + op->ne, op->elem_type.begin());
  aimm_macro_store_elem_types(op);
  return AIM_OK;
}


// Device copies of one set of per-kind N x N blocks (host complex128 [n_types][N][N],
// column-major): complex128 and complex64 with gemm_krows(N) columns per kind (zero
// past N), and, for N % 8 == 0, the split-BF16 planes
// [h, m, l of re; of im][k / 8][row][k % 8] of the complex64 values.
// Allocates on first use; throws std::bad_alloc or std::runtime_error.
static void upload_blocks(aim_op* op, const cd* M, cplx<double>*& d64, cplx<float>*& d32, void*& db) {
  const size_t N = size_t(op->N), kr = size_t(gemm_krows(op->N));
  const size_t n = size_t(op->n_types) * kr * N;
  if (!d64) {
    d64 = op->mem.alloc<cplx<double>>(n);
    d32 = op->mem.alloc<cplx<float>>(n);
  }
  std::vector<cplx<double>> m64(n, cplx<double>{0.0, 0.0});
  std::vector<cplx<float>> m32(n, cplx<float>{0.0f, 0.0f});
  for (size_t t = 0; t < size_t(op->n_types); ++t)
    for (size_t e = 0; e < N * N; ++e) {
      const size_t src = t * N * N + e, dst = t * kr * N + e;
      m64[dst].re = M[src].real();
      m64[dst].im = M[src].imag();
      m32[dst].re = float(M[src].real());
      m32[dst].im = float(M[src].imag());
    }
  if (hipMemcpy(d64, m64.data(), n * sizeof(cplx<double>), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d32, m32.data(), n * sizeof(cplx<float>), hipMemcpyHostToDevice) != hipSuccess)
    throw std::runtime_error("hipMemcpy of the block set failed");
  if (op->N % 8 != 0) return;
  const size_t KB = kr / 8, per = 6 * KB * N * 8;
  std::vector<uint16_t> mb(size_t(op->n_types) * per, 0);
  for (size_t t = 0; t < size_t(op->n_types); ++t)
    for (size_t k = 0; k < kr; ++k)
      for (size_t i = 0; i < N; ++i) {
        const cplx<float> v = m32[t * kr * N + k * N + i];
        const float comp[2] = {v.re, v.im};
        for (int c = 0; c < 2; ++c) {
          uint16_t part3[3];
          split_bf16(comp[c], part3);
          for (int q = 0; q < 3; ++q) mb[t * per + ((size_t(3 * c + q) * KB + k / 8) * N + i) * 8 + k % 8] = part3[q];
        }
      }
  if (!db) db = op->mem.alloc<uint16_t>(mb.size());
  if (hipMemcpy(db, mb.data(), mb.size() * sizeof(uint16_t), hipMemcpyHostToDevice) != hipSuccess)
    throw std::runtime_error("hipMemcpy of the split-BF16 planes failed");
}

int aim_set_macromodels(aim_op* op, const double* M) {
  if (!op || !M) {
    set_error("op and M must not be NULL");
    return AIM_EINVAL;
  }
  const size_t nn = size_t(op->n_types) * op->N * op->N;
  std::vector<cd> host(nn);
  for (size_t e = 0; e < nn; ++e) host[e] = cd(M[2 * e], M[2 * e + 1]);
  if (op->device_ready) {
    try {
      upload_blocks(op, host.data(), op->p64.M, op->p32.M, op->Mb);
    } catch (const std::bad_alloc&) {
      set_error("device allocation failed");
      return AIM_ENOMEM;
    } catch (const std::exception& e) {
      set_error(e.what());
      return AIM_EDEVICE;
    }
  }
  op->m_host.swap(host);
  op->m_set = true;
  op->p_set = false;  // a preconditioner built from the previous blocks is stale
  return AIM_OK;
}

int aim_set_dmatrix(aim_op* op, int64_t nnz, const int32_t* rows, const int32_t* cols, const double* vals) {
  if (!op || nnz < 0 || (nnz > 0 && (!rows || !cols || !vals))) {
    set_error("bad D arguments");
    return AIM_EINVAL;
  }
  const int N = op->N;
  for (int64_t i = 0; i < nnz; ++i)
    if (rows[i] < 0 || rows[i] >= N || cols[i] < 0 || cols[i] >= N) {
      set_error("D index out of range");
      return AIM_EINVAL;
    }
  if (op->d_set) {
    set_error("D is already set");
    return AIM_ESTATE;
  }
  op->d_rows.assign(rows, rows + nnz);
  op->d_cols.assign(cols, cols + nnz);
  op->d_vals.resize(size_t(nnz));
  for (int64_t i = 0; i < nnz; ++i) op->d_vals[size_t(i)] = cd(vals[2 * i], vals[2 * i + 1]);
  if (!op->device_ready) {
    op->d_nnz = nnz;
    op->d_set = true;
    return AIM_OK;
  }
  // padded row layout, slot-major: slot s of row n at s * N + n; entries keep their
  // input order within a row, padding slots point at column n with value 0
  std::vector<int> cnt(N, 0);
  for (int64_t i = 0; i < nnz; ++i) cnt[rows[i]]++;
  const int dmax = nnz > 0 ? *std::max_element(cnt.begin(), cnt.end()) : 0;
  std::vector<int> colT(size_t(dmax) * N), fill(N, 0);
  std::vector<cplx<double>> v64(size_t(dmax) * N, cplx<double>{0.0, 0.0});
  std::vector<cplx<float>> v32(size_t(dmax) * N, cplx<float>{0.0f, 0.0f});
  for (int sl = 0; sl < dmax; ++sl)
    for (int n = 0; n < N; ++n) colT[size_t(sl) * N + n] = n;
  for (int64_t i = 0; i < nnz; ++i) {
    const size_t at = size_t(fill[rows[i]]++) * N + rows[i];
    colT[at] = cols[i];
    v64[at].re = vals[2 * i];
    v64[at].im = vals[2 * i + 1];
    v32[at].re = float(vals[2 * i]);
    v32[at].im = float(vals[2 * i + 1]);
  }
  try {
    if (dmax > 0) {
      op->d_colT = upload(op, colT.data(), colT.size());
      op->p64.dval = upload(op, v64.data(), v64.size());
      op->p32.dval = upload(op, v32.data(), v32.size());
    }
  } catch (const std::bad_alloc&) {
    set_error("device allocation failed");
    return AIM_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return AIM_EDEVICE;
  }
  op->d_max = dmax;
  op->d_nnz = nnz;
  op->d_set = true;
  return AIM_OK;
}

int macro_apply(aim_op* op, const void* x, void* u, int32_t nrhs, int32_t precision, void* stream) {
  int c = check_common(op, x, u, nrhs, precision);
  if (c) return c;
  if (!op->m_set) {
    set_error("macromodels not set");
    return AIM_ESTATE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the GEMM writes element-fastest; transposing [N][ne] back is the same kernel with
  // the two extents swapped
  if (precision == AIM_FP64) {
    cplx<double>* uT = static_cast<cplx<double>*>(op->u);
    AIM_HIP(launch_macro<double>(op->p64.M, static_cast<const cplx<double>*>(x), uT, gemm_args(op, nrhs), s));
    AIM_HIP(launch_transpose<double>(uT, static_cast<cplx<double>*>(u), nrhs, op->N, op->ne, s));
  } else {
    cplx<float>* uT = static_cast<cplx<float>*>(op->u);
    AIM_HIP(launch_macro<float>(op->p32.M, static_cast<const cplx<float>*>(x), uT, gemm_args(op, nrhs), s));
    AIM_HIP(launch_transpose<float>(uT, static_cast<cplx<float>*>(u), nrhs, op->N, op->ne, s));
  }
  return AIM_OK;
}

int aim_build_preconditioner(aim_op* op) {
  if (!op) {
    set_error("op is NULL");
    return AIM_EINVAL;
  }
  if (!op->m_set || !op->d_set) {
    set_error("macromodels and D must be set before the preconditioner");
    return AIM_ESTATE;
  }
  const size_t NN = size_t(op->N) * op->N;
  try {
    std::vector<cd> G, Pt, P(size_t(op->n_types) * NN);
    self_block(op->st, op->arr, G);
    for (int t = 0; t < op->n_types; ++t) {
      block_inverse(G, op->m_host.data() + t * NN, op->d_rows.data(), op->d_cols.data(), op->d_vals.data(),
                    int64_t(op->d_rows.size()), op->N, Pt);
      std::copy(Pt.begin(), Pt.end(), P.begin() + t * NN);
    }
    if (op->device_ready) upload_blocks(op, P.data(), op->P64, op->P32, op->Pb);
    op->p_host.swap(P);
  } catch (const std::bad_alloc&) {
    set_error("allocation failed");
    return AIM_ENOMEM;
  } catch (const std::runtime_error& e) {
    set_error(e.what());
    return op->device_ready && std::string(e.what()).find("hipMemcpy") != std::string::npos ? AIM_EDEVICE
                                                                                               : AIM_EINVAL;
  }
  op->p_set = true;
  return AIM_OK;
}

int aim_get_preconditioner(const aim_op* op, double* P) {
  if (!op || !P) {
    set_error("op and P must not be NULL");
    return AIM_EINVAL;
  }
  if (!op->p_set) {
    set_error("preconditioner not built (or stale after aim_set_macromodels)");
    return AIM_ESTATE;
  }
  for (size_t e = 0; e < op->p_host.size(); ++e) {
    P[2 * e] = op->p_host[e].real();
    P[2 * e + 1] = op->p_host[e].imag();
  }
  return AIM_OK;
}

int precond_apply(aim_op* op, const void* x, void* y, int32_t nrhs, int32_t precision, void* stream) {
  int c = check_common(op, x, y, nrhs, precision);
  if (c) return c;
  if (!op->p_set) {
    set_error("preconditioner not built (or stale after aim_set_macromodels)");
    return AIM_ESTATE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == AIM_FP64)
    return precond_impl<double>(op, static_cast<const cplx<double>*>(x), static_cast<cplx<double>*>(y), nrhs, s);
  return precond_impl<float>(op, static_cast<const cplx<float>*>(x), static_cast<cplx<float>*>(y), nrhs, s);
}

int aim_matvec(aim_op* op, const void* x, void* y, int32_t nrhs, int32_t precision, int32_t flags, void* stream) {
  int c = check_common(op, x, y, nrhs, precision);
  if (c) return c;
  if (flags < AIM_FULL || flags > AIM_FAR_ONLY) {
    set_error("unknown flags");
    return AIM_EINVAL;
  }
  if (x == y) {
    set_error("x and y must not alias");
    return AIM_EINVAL;
  }
  if (flags == AIM_FULL && (!op->m_set || !op->d_set)) {
    set_error("macromodels and D must be set for the full product");
    return AIM_ESTATE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == AIM_FP64)
    return matvec_impl<double>(op, static_cast<const cplx<double>*>(x), static_cast<cplx<double>*>(y), nrhs, flags, s);
  return matvec_impl<float>(op, static_cast<const cplx<float>*>(x), static_cast<cplx<float>*>(y), nrhs, flags, s);
}

int aim_time_kernels(aim_op* op, const void* x, void* y, int32_t nrhs, int32_t precision, int32_t reps, double* ms,
                     void* stream) {
  int c = check_common(op, x, y, nrhs, precision);
  if (c) return c;
  if (!ms || reps < 1 || x == y) {
    set_error("ms must not be NULL, reps >= 1, x and y must not alias");
    return AIM_EINVAL;
  }
  if (!op->m_set || !op->d_set) {
    set_error("macromodels and D must be set");
    return AIM_ESTATE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == AIM_FP64)
    return time_kernels<double>(op, static_cast<const cplx<double>*>(x), static_cast<cplx<double>*>(y), nrhs, reps,
                                ms, s);
  return time_kernels<float>(op, static_cast<const cplx<float>*>(x), static_cast<cplx<float>*>(y), nrhs, reps, ms, s);
}

int aim_project(aim_op* op, const void* u, void* Q, int32_t nrhs, int32_t precision, void* stream) {
  int c = check_common(op, u, Q, nrhs, precision);
  if (c) return c;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == AIM_FP64) {
    cplx<double>* uT = static_cast<cplx<double>*>(op->u);
    AIM_HIP(launch_transpose<double>(static_cast<const cplx<double>*>(u), uT, nrhs, op->ne, op->N, s));
    AIM_HIP(launch_project<double>(uT, static_cast<cplx<double>*>(Q), proj_args(op, nrhs), op->p64.Wp, s));
  } else {
    cplx<float>* uT = static_cast<cplx<float>*>(op->u);
    AIM_HIP(launch_transpose<float>(static_cast<const cplx<float>*>(u), uT, nrhs, op->ne, op->N, s));
    AIM_HIP(launch_project<float>(uT, static_cast<cplx<float>*>(Q), proj_args(op, nrhs), op->p32.Wp, s));
  }
  return AIM_OK;
}

int aim_convolve(aim_op* op, const void* Q, void* Phi, int32_t nrhs, int32_t precision, void* stream) {
  int c = check_common(op, Q, Phi, nrhs, precision);
  if (c) return c;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (precision == AIM_FP64)
    AIM_HIP(launch_convolve<double>(static_cast<const cplx<double>*>(Q), static_cast<cplx<double>*>(Phi),
                                    static_cast<cplx<double>*>(op->S), conv_args(op, op->p64, nrhs), s));
  else
    AIM_HIP(launch_convolve<float>(static_cast<const cplx<float>*>(Q), static_cast<cplx<float>*>(Phi),
                                   static_cast<cplx<float>*>(op->S), conv_args(op, op->p32, nrhs), s));
  return AIM_OK;
}

int aim_plane_wave_rhs(aim_op* op, const double* theta, const double* phi, const int32_t* pol, int32_t nrhs,
                       void* b, void* stream) {
  if (!op || !theta || !phi || !pol || !b || nrhs < 1 || nrhs > op->R_max) {
    set_error("bad plane-wave arguments");
    return AIM_EINVAL;
  }
  if (!op->device_ready) {
    set_error("op was built without device data (aim_build_host)");
    return AIM_ESTATE;
  }
  for (int r = 0; r < nrhs; ++r)
    if (pol[r] != 0 && pol[r] != 1) {
      set_error("pol must be 0 or 1");
      return AIM_EINVAL;
    }
  SurfaceIn s;
  s.n_vert = int(op->vert.size() / 3);
  s.n_tri = int(op->tri.size() / 3);
  s.n_rwg = int(op->rwg.size() / 4);
  s.vert = op->vert.data();
  s.tri = op->tri.data();
  s.rwg = op->rwg.data();
  std::vector<cplx<double>> loc(size_t(nrhs) * op->N);
  std::vector<double> kinc(3 * nrhs);
  std::vector<cd> l;
  for (int r = 0; r < nrhs; ++r) {
    plane_wave_local(s, op->arr.k, theta[r], phi[r], pol[r], l, &kinc[3 * r]);
    for (int n = 0; n < op->N; ++n) {
      loc[size_t(r) * op->N + n].re = l[n].real();
      loc[size_t(r) * op->N + n].im = l[n].imag();
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  void *dl = nullptr, *dk = nullptr;
  AIM_HIP(hipMalloc(&dl, loc.size() * sizeof(cplx<double>)));
  if (hipMalloc(&dk, kinc.size() * sizeof(double)) != hipSuccess) {
    (void)hipFree(dl);
    set_error("hipMalloc failed");
    return AIM_ENOMEM;
  }
  hipError_t e = hipMemcpyAsync(dl, loc.data(), loc.size() * sizeof(cplx<double>), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(dk, kinc.data(), kinc.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = launch_expand_rhs(static_cast<cplx<double>*>(dl), static_cast<double*>(dk), static_cast<cplx<double>*>(b),
                          nrhs, op->ne, op->N, op->arr.px, op->arr.pitch * op->arr.h, op->arr.k, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dl);
  (void)hipFree(dk);
  if (e != hipSuccess) {
    set_error(std::string("plane-wave rhs: ") + hipGetErrorString(e));
    return AIM_EDEVICE;
  }
  return AIM_OK;
}

int aim_get_info(const aim_op* op, aim_info* info) {
  if (!op || !info) {
    set_error("op and info must not be NULL");
    return AIM_EINVAL;
  }
  info->n_rwg = op->N;
  info->n_elem = op->ne;
  info->n_types = op->n_types;
  info->nx = op->st.nx;
  info->ny = op->st.ny;
  info->nz = op->st.nz;
  info->lx = op->Lx;
  info->ly = op->Ly;
  info->n_offsets = int(op->st.offsets.size() / 2);
  info->near_nnz = int64_t(op->st.near_val.size());
  info->d_nnz = op->d_nnz;
  info->device_bytes = int64_t(op->mem.bytes);
  info->paths = op->device_ready ? ((op->fft4 ? AIM_PATH_FFT_REGISTER : 0) | (op->near_mfma ? AIM_PATH_NEAR_MFMA : 0) |
                                    (op->gemm_bf16 ? AIM_PATH_GEMM_BF16X3 : 0))
                                 : 0;
  return AIM_OK;
}

int aim_get_near(const aim_op* op, int32_t* rows, int32_t* offs, int32_t* cols, double* vals, int32_t* offsets) {
  if (!op || !rows || !offs || !cols || !vals || !offsets) {
    set_error("NULL argument");
    return AIM_EINVAL;
  }
  const Setup& st = op->st;
  for (int n = 0; n < st.N; ++n)
    for (int e = st.near_ptr[n]; e < st.near_ptr[n + 1]; ++e) {
      rows[e] = n;
      offs[e] = st.near_col[e] >> 16;
      cols[e] = st.near_col[e] & 0xFFFF;
      vals[2 * e] = st.near_val[e].real();
      vals[2 * e + 1] = st.near_val[e].imag();
    }
  for (size_t i = 0; i < st.offsets.size(); ++i) offsets[i] = st.offsets[i];
  return AIM_OK;
}

size_t aim_footprint_bytes(const aim_surface* surface, const aim_array* array, int32_t nrhs, int32_t restart,
                           int32_t precision) {
  if (!surface || !array || nrhs < 1 || restart < 1) return 0;
  // stencil extent from the edge midpoints, as in the build
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int n = 0; n < surface->n_rwg; ++n)
    for (int ax = 0; ax < 3; ++ax) {
      const double c = 0.5 * (surface->vert[3 * surface->rwg[4 * n] + ax] + surface->vert[3 * surface->rwg[4 * n + 1] + ax]);
      const double v = std::floor(c / array->h - 0.5 * array->order + 0.5 + 1e-9);
      lo[ax] = std::min(lo[ax], v);
      hi[ax] = std::max(hi[ax], v);
    }
  const int q = array->order + 1;
  const size_t ex = size_t(hi[0] - lo[0]) + q, ey = size_t(hi[1] - lo[1]) + q, ez = size_t(hi[2] - lo[2]) + q;
  const size_t nx = size_t(array->pitch_cells) * (array->px - 1) + ex;
  const size_t ny = size_t(array->pitch_cells) * (array->py - 1) + ey;
  const size_t Ly = size_t(smooth_length(int(std::max(2 * ny - 2, ny))));
  const size_t Lx = size_t(smooth_length(int(std::max(2 * nx - 2, nx))));
  const size_t N = size_t(surface->n_rwg), ne = size_t(array->px) * array->py, R = size_t(array->max_rhs);
  const size_t n = ne * N;
  size_t b = 0;
  b += n * R * 16;                                   // u
  b += (N + 15) / 16 * 16 * ne * R * 16;             // near-field output (group-slot order)
  b += R * 4 * nx * ny * ez * 16;                    // grid
  b += R * 4 * nx * Ly * ez * 16;                    // spectrum pass
  b += (Lx / 2 + 1) * (Ly / 2 + 1) * ez * 24;        // kernel spectrum, both precisions
  b += size_t(array->n_types) * N * N * 24;          // macromodels
  b += size_t(array->n_types) * 6 * (4 * ((N + 63) / 64 * 16) + 16) * N * 2;  // their split-BF16 planes
  b += N * 600 * 28 + N * q * q * q * 4 * 24;        // near field (upper estimate) and weights
  const size_t vec = precision == AIM_FP64 ? 16 : 8;
  b += size_t(restart + 1) * size_t(nrhs) * n * vec;  // Krylov basis
  b += size_t(nrhs) * n * (16 * 3 + 2 * vec);         // GMRES vectors
  b += size_t(nrhs) * size_t(restart + 1) * (restart + 1) * 16;  // Gram matrices
  b += size_t(nrhs) * 2 * size_t(restart + 1) * (n / 256 + 1) * 16;  // reduction partials
  return b;
}

void aim_destroy(aim_op* op) {
  if (!op) return;
  if (op->device_ready) {
    (void)hipDeviceSynchronize();
    aimm::release_krylov(op);
    if (op->s_aux) (void)hipStreamDestroy(op->s_aux);
    if (op->ev_fork) (void)hipEventDestroy(op->ev_fork);
    if (op->ev_join) (void)hipEventDestroy(op->ev_join);
  }
  aimm_release_macro_store(op);
  delete op;
}

}  // extern "C"
