// The operator object behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "aim_kernels.hpp"
#include "setup.hpp"

struct aim_op;

namespace aimm {

void set_error(const std::string& msg);
struct KrylovWork;

struct DeviceMem {
  std::vector<void*> ptrs;
  size_t bytes = 0;
  template <typename T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    void* p = nullptr;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    ptrs.push_back(p);
    bytes += count * sizeof(T);
    return static_cast<T*>(p);
  }
  void release(void* p, size_t nbytes) {
    for (auto& q : ptrs)
      if (q == p) {
        (void)hipFree(q);
        q = nullptr;
        bytes -= nbytes;
      }
  }
  ~DeviceMem() {
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
};

// Per-precision copies of the real and complex operator data.
template <typename T>
struct PrecData {
  T* Wp = nullptr;           // [N * q3][4] projection weights per gather entry, in gather-table order
  T* Wt = nullptr;           // [4][q3][N] interpolation weights
  cplx<T>* near = nullptr;   // pre-corrected near field
  cplx<T>* grpA = nullptr;   // near field as dense row-group blocks
  cplx<T>* gt = nullptr;     // kernel spectrum, [Lx/2+1][Ly/2+1][nz]
  cplx<T>* tw_x = nullptr;
  cplx<T>* tw_y = nullptr;
  cplx<T>* M = nullptr;      // [n_types][N][N] column-major
  cplx<T>* dval = nullptr;   // D values
  int B = 1;                 // ky lines per workgroup in the spectrum pass
};

struct KrylovWork {
  int R = 0, restart = 0, prec = -1;
  void* V = nullptr;         // [restart+1][R][n] basis (complex128 or complex64)
  size_t V_bytes = 0;
  cplx<double>* w = nullptr; // [R][n] working vector (FP64)
  void* wlow = nullptr;      // [R][n] low-precision product input/output
  void* ylow = nullptr;
  cplx<double>* r = nullptr; // [R][n] residual
  cplx<double>* H = nullptr; // [R][restart+1][restart]
  cplx<double>* cs = nullptr;
  cplx<double>* sn = nullptr;
  cplx<double>* g = nullptr;  // [R][restart+1]
  cplx<double>* hcol = nullptr;  // [R][restart+1] first Gram-Schmidt pass
  cplx<double>* h2 = nullptr;    // [R][restart+1] least-squares solution
  double* part = nullptr;     // reduction partials
  size_t part_len = 0;
  double* scal = nullptr;     // [R][4] norms / flags
  cplx<double>* S = nullptr;  // [R][restart+1][restart+1] Gram matrix of the basis
  double* ib = nullptr;       // [R][restart+1] v_i = ib_i u_i (stored u_i unnormalised)
  cplx<double>* pq = nullptr; // [R][2 (restart+1)] projections and new Gram column
  cplx<double>* cr = nullptr; // [R][restart+1] update coefficients of the stored u_i
  int* active = nullptr;      // [R] per-cycle stop column
  // pinned host staging for the per-cycle and per-check transfers (asynchronous DMA)
  void* hpin = nullptr;
  double* h_scal = nullptr;        // [R][4]
  int* h_jinit = nullptr;          // [R]
  int* h_jused = nullptr;          // [R]
  cplx<double>* h_g0 = nullptr;    // [R][restart+1]
  cplx<double>* h_gh = nullptr;    // [R][restart+1]
  double* h_ib0 = nullptr;         // [R][restart+1]
  // captured inner iterations: key (precond, system, restart) -> one executable graph per
  // iteration index j, valid for this workspace and the op's graph epoch
  std::map<int, std::vector<hipGraphExec_t>> graphs;
  int graph_epoch = -1;
  // stream the iterations are captured on (the caller's stream may be the null stream,
  // which cannot be captured); the graphs are then launched on the caller's stream
  hipStream_t cap = nullptr;
  // recorded after a check's flag transfers: the host waits for it while the device
  // runs the iteration enqueued after it
  hipEvent_t ev_check = nullptr;
};

void release_krylov(aim_op* op);
// far-field set-up at op build time (quadrature table, scratch address of the device)
void ff_prepare(aim_op* op);
// grouped-product arguments of the op's macromodel layout for R right-hand sides
GemmArgs gemm_args_of(aim_op* op, int R);

}  // namespace aimm

// frees the generated macromodel data of an op (R blocks, host copies); called by aim_destroy
void aimm_release_macro_store(const aim_op* op);
// recomputes the generated data's per-element scatterer offsets after the element kinds change
void aimm_macro_store_elem_types(const aim_op* op);

struct aim_op {
  aimm::Setup st;
  aimm::ArrayIn arr{};
  std::vector<int32_t> elem_type;
  std::vector<double> vert;
  std::vector<int32_t> tri, rwg;
  int device = 0;
  int graph_epoch = 0;  // bumped when captured launch arguments change (element kinds)
  hipStream_t build_stream = nullptr;  // stream of aim_build_grid's uploads and kernels (during the call)
  int ne = 0, N = 0, R_max = 0, n_types = 0;
  int Lx = 0, Ly = 0;
  aimm::FftPlan Px{}, Py{};
  std::vector<int> type_count, col_start;
  bool m_set = false, d_set = false;
  bool device_ready = false;  // false for ops from aim_build_host
  int64_t d_nnz = 0;
  int d_max = 0;  // slots per row of the padded D layout
  size_t lds_max = 65536;
  aimm::DeviceMem mem;
  int *sloc = nullptr, *node_ptr = nullptr, *node_n = nullptr, *near_ptr = nullptr,
      *near_col = nullptr;
  int* offsets_d = nullptr;  // [n_off][2] lattice offsets of the near-field blocks
  int *grp_ptr = nullptr, *grp_col = nullptr, *grp_row = nullptr, *slot_of = nullptr;
  aimm::cplx<double>* zero = nullptr;  // one zero value (16 bytes; also read as complex64)
  bool near_mfma = true;
  bool fft4 = false;  // register-DFT FFT passes
  bool gemm_bf16 = false;  // mixed-path macromodel product on the bf16 matrix cores (split in three)
  void* Mb = nullptr;      // [n_types][6 planes][Krows / 8][N][8] bf16
  int interp_tx = 0, interp_ty = 0;  // interpolation tile (0 = automatic)
  int near_eb[2] = {1, 1};  // near field: blocks of 16 elements per workgroup [FP64, mixed]
  int near_fork[2] = {0, 0};  // near field forked after: 0 the GEMM, 1 the projection, 2 the y pass [FP64, mixed]
  int *nbr = nullptr, *d_colT = nullptr, *rev_x = nullptr, *rev_y = nullptr, *col_list = nullptr;
  aimm::PrecData<double> p64;
  aimm::PrecData<float> p32;
  // host copies of the operator data, for the preconditioner's diagonal blocks
  std::vector<aimm::cd> m_host;                 // [n_types][N][N] column-major
  std::vector<int32_t> d_rows, d_cols;
  std::vector<aimm::cd> d_vals;
  // block-Jacobi preconditioner P_t = (D - G_self M_t)^-1, same device layouts as M
  bool p_set = false;
  std::vector<aimm::cd> p_host;                 // [n_types][N][N] column-major
  aimm::cplx<double>* P64 = nullptr;
  aimm::cplx<float>* P32 = nullptr;
  void* Pb = nullptr;                           // split-BF16 planes of P (as Mb)
  void* u = nullptr;      // [R][N][n_elem] macromodel output, element-fastest (sized for complex128)
  void* nf = nullptr;     // [R][n_elem][N] near-field product (sized for complex128)
  void* grid = nullptr;   // Q / Phi (sized for complex128)
  void* S = nullptr;      // spectrum pass buffer (sized for complex128)
  // the near field runs on a second stream, beside step (i) and the FFT passes
  hipStream_t s_aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* ff_quad = nullptr;  // far-field quadrature table [N][14][6], built on first use
  void* ff_ws = nullptr;      // far-field workspace (directions, phase tables, partials)
  size_t ff_bytes = 0;
  aimm::KrylovWork kw;
};
