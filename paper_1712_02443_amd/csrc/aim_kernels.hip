// Device kernels of the AIM matrix-vector product (section V, steps (i)-(iii)) plus
// the near-field pre-correction and the block-diagonal D term of eq. MV_product1.
//
// Layouts (complex values interleaved):
//   vectors  x, u, y : [R][n_elem][N]          (element-major unknowns)
//   grids    Q, Phi  : [R][4][nx][ny][nz]      (psi = x, y, z, phi)
//   spectrum S       : [R][4][nx][Ly][nz]      (y transformed, ky in digit-reversed slots)
#include "aim_kernels.hpp"
#include "fft.hpp"
#include "fft4.hpp"

namespace aimm {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Strided copy global -> LDS with U loads in flight per thread (a plain strided loop
// waits for each load before its store).  f(e) -> value, g(e, value) stores it.
template <int U, typename T, typename Load, typename Store>
__device__ __forceinline__ void batched_copy(int n, Load f, Store g) {
  for (int base = threadIdx.x; base < n; base += U * blockDim.x) {
    cplx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * blockDim.x;
      if (e < n) v[u] = f(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + u * blockDim.x;
      if (e < n) g(e, v[u]);
    }
  }
}

// ---- step (i): projection, owner-computes gather --------------------------------
// Grid node g is written by exactly one element (its owner: the element whose
// pitch-wide home cell contains g, the last row/column owning the tail).  The owner
// gathers every basis of itself and of the neighbours whose stencil box covers g.

// Node (lx, ly, lz) of element (ix, iy), its owner: sum over the covering cells.
// Wp holds the four weights (psi = x, y, z, phi) of every gather entry in the order of
// the gather table and node_n the entry's offset n * ne, so an entry costs two
// wave-uniform loads and one coalesced load of u, with no dependent index load; eight
// entries' loads are issued before their arithmetic.  A covering cell of a neighbour
// outside the lattice reads the lane's own element instead and its sum is scaled by
// zero (u is finite).
template <typename T>
__device__ __forceinline__ void project_cell(const cplx<T>* __restrict__ us, const ProjArgs& a,
                                             const T* __restrict__ Wp, int e, int e1, cplx<T> (&acc)[4]) {
  for (; e + 8 <= e1; e += 8) {
    cplx<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = us[a.node_n[e + u]];
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int p = 0; p < 4; ++p) cfmas(acc[p], Wp[int64_t(e + u) * 4 + p], v[u]);
  }
  if (e + 4 <= e1) {
    cplx<T> v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = us[a.node_n[e + u]];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int p = 0; p < 4; ++p) cfmas(acc[p], Wp[int64_t(e + u) * 4 + p], v[u]);
    e += 4;
  }
  for (; e < e1; ++e) {
    const cplx<T> v = us[a.node_n[e]];
#pragma unroll
    for (int p = 0; p < 4; ++p) cfmas(acc[p], Wp[int64_t(e) * 4 + p], v);
  }
}

template <typename T>
__device__ __forceinline__ void project_node(const cplx<T>* __restrict__ ur, cplx<T>* __restrict__ Qr,
                                             const ProjArgs& a, const T* __restrict__ Wp, int ix, int iy, int lx,
                                             int ly, int lz) {
  const int gx = ix * a.pitch + lx, gy = iy * a.pitch + ly;
  if (gx >= a.nx || gy >= a.ny) return;  // home cell of the last column / row past the grid
  const int m = iy * a.px + ix;
  cplx<T> acc[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) acc[p] = cmk<T>(0, 0);
  for (int dy = 0; ly + a.pitch * dy < a.ey; ++dy) {
    for (int dx = 0; lx + a.pitch * dx < a.ex; ++dx) {
      const int node = ((lx + a.pitch * dx) * a.ey + (ly + a.pitch * dy)) * a.ez + lz;
      const int e0 = a.node_ptr[node], e1 = a.node_ptr[node + 1];
      if (dx == 0 && dy == 0) {
        project_cell(ur + m, a, Wp, e0, e1, acc);
      } else {
        const bool ok = ix - dx >= 0 && iy - dy >= 0;
        cplx<T> c[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) c[p] = cmk<T>(0, 0);
        project_cell(ur + (ok ? m - dx - dy * a.px : m), a, Wp, e0, e1, c);
        const T f = ok ? T(1) : T(0);
#pragma unroll
        for (int p = 0; p < 4; ++p) cfmas(acc[p], f, c[p]);
      }
    }
  }
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t g = (int64_t(gx) * a.ny + gy) * a.nz + lz;
#pragma unroll
  for (int p = 0; p < 4; ++p) Qr[p * nodes + g] = acc[p];
}

// Home cells (lx, ly < pitch): every element owns them.  Lanes of a wave are 64
// consecutive elements at the same element-local node, so the gather table row is
// wave-uniform and u is read from its element-fastest copy.
template <typename T>
__device__ __forceinline__ void project_tail(const cplx<T>* __restrict__ uT, cplx<T>* __restrict__ Q,
                                             const ProjArgs& a, const T* __restrict__ Wp, int w, int lane);
__device__ __forceinline__ int project_tail_waves(const ProjArgs& a);

// One wave per workgroup: the tail waves (fewer, with longer gathers) come first.
template <typename T>
__global__ void __launch_bounds__(64) k_project(const cplx<T>* __restrict__ uT, cplx<T>* __restrict__ Q,
                                                ProjArgs a, const T* __restrict__ Wp) {
  const int ntail = project_tail_waves(a) * a.R;
  if (int(blockIdx.x) < ntail) {
    project_tail(uT, Q, a, Wp, blockIdx.x, threadIdx.x);
    return;
  }
  const int ne64 = (a.ne + 63) & ~63;
  const int nloc = a.pitch * a.pitch * a.ez;
  const int64_t gid = int64_t(blockIdx.x - ntail) * 64 + threadIdx.x;
  const int m = int(gid % ne64);
  const int64_t rest = gid / ne64;
  const int L = __builtin_amdgcn_readfirstlane(int(rest % nloc));
  const int r = __builtin_amdgcn_readfirstlane(int(rest / nloc));
  if (r >= a.R || m >= a.ne) return;
  const int lz = L % a.ez, ly = (L / a.ez) % a.pitch, lx = L / (a.ez * a.pitch);
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  project_node(uT + int64_t(r) * a.N * a.ne, Q + int64_t(r) * 4 * nodes, a, Wp, m % a.px, m / a.px, lx, ly, lz);
}

// Nodes beyond the last home cells: the right strip (owned by the last column of
// elements), the top strip (last row) and their corner (last element), wx = ex - pitch
// and wy = ey - pitch nodes wide.  One wave per (strip, local node), lanes over the
// strip's elements, so the gather table row stays wave-uniform.
__device__ __forceinline__ int project_tail_waves(const ProjArgs& a) {
  const int wx = max(a.ex - a.pitch, 0), wy = max(a.ey - a.pitch, 0);
  return wx * a.pitch * a.ez * ((a.py + 63) / 64) + a.pitch * wy * a.ez * ((a.px + 63) / 64) + wx * wy * a.ez;
}

template <typename T>
__device__ __forceinline__ void project_tail(const cplx<T>* __restrict__ uT, cplx<T>* __restrict__ Q,
                                             const ProjArgs& a, const T* __restrict__ Wp, int w, int lane) {
  const int wx = max(a.ex - a.pitch, 0), wy = max(a.ey - a.pitch, 0);
  const int cy = (a.py + 63) / 64, cx = (a.px + 63) / 64;  // lane chunks per strip node
  const int na = wx * a.pitch * a.ez * cy, nb = a.pitch * wy * a.ez * cx, nc = wx * wy * a.ez;
  const int per_r = na + nb + nc;
  const int r = w / per_r;
  if (r >= a.R) return;
  w -= r * per_r;
  int ix, iy, lx, ly, lz;
  if (w < na) {
    const int L = w / cy;
    iy = (w % cy) * 64 + lane;
    ix = a.px - 1;
    if (iy >= a.py) return;
    lz = L % a.ez;
    ly = (L / a.ez) % a.pitch;
    lx = a.pitch + L / (a.pitch * a.ez);
  } else if (w < na + nb) {
    w -= na;
    const int L = w / cx;
    ix = (w % cx) * 64 + lane;
    iy = a.py - 1;
    if (ix >= a.px) return;
    lz = L % a.ez;
    ly = a.pitch + (L / a.ez) % wy;
    lx = L / (wy * a.ez);
  } else {
    const int L = w - na - nb;
    if (lane != 0) return;
    ix = a.px - 1;
    iy = a.py - 1;
    lz = L % a.ez;
    ly = a.pitch + (L / a.ez) % wy;
    lx = a.pitch + L / (wy * a.ez);
  }
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  project_node(uT + int64_t(r) * a.N * a.ne, Q + int64_t(r) * 4 * nodes, a, Wp, ix, iy, lx, ly, lz);
}

// [R][ne][N] -> [R][N][ne] (element-fastest copy of a vector); with the extents
// swapped it maps [R][N][ne] back to [R][ne][N]
template <typename T>
__global__ void __launch_bounds__(256) k_transpose(const cplx<T>* __restrict__ x, cplx<T>* __restrict__ xT, int ne,
                                                   int N) {
  __shared__ cplx<T> tile[32][33];
  const int r = blockIdx.z;
  const int n0 = blockIdx.x * 32, m0 = blockIdx.y * 32;
  const cplx<T>* src = x + int64_t(r) * ne * N;
  cplx<T>* dst = xT + int64_t(r) * ne * N;
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int k = ty; k < 32; k += 8) {
    const int m = m0 + k, n = n0 + tx;
    if (m < ne && n < N) tile[k][tx] = src[int64_t(m) * N + n];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int n = n0 + k, m = m0 + tx;
    if (m < ne && n < N) dst[int64_t(n) * ne + m] = tile[tx][k];
  }
}

// ---- step (ii), pass 1: forward FFT along y of every (r, psi, x) plane ------------
template <typename T>
__global__ void __launch_bounds__(256) k_fft_y_fwd(const cplx<T>* in, cplx<T>* out, int ny_in, int nz,
                                                   FftPlan P, const cplx<T>* __restrict__ twg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  const int L = P.L;
  cplx<T>* buf = tw + L;
  const int ld = L;
  const int64_t plane = blockIdx.x;
  const cplx<T>* src = in + plane * int64_t(ny_in) * nz;
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twg[i];
  batched_copy<8, T>(
      ny_in * nz, [&](int e) { return src[e]; },
      [&](int e, cplx<T> v) {
        const int y = e / nz, z = e - y * nz;
        buf[z * ld + y] = v;
      });
  for (int e = threadIdx.x; e < (L - ny_in) * nz; e += blockDim.x) {
    const int z = e / (L - ny_in), y = ny_in + (e - z * (L - ny_in));
    buf[z * ld + y] = cmk<T>(0, 0);
  }
  __syncthreads();
  lds_fft_fwd(buf, ld, nz, P, tw);
  cplx<T>* dst = out + plane * int64_t(L) * nz;
  for (int e = threadIdx.x; e < L * nz; e += blockDim.x) {
    const int y = e / nz, z = e - y * nz;
    dst[e] = buf[z * ld + y];
  }
}

// ---- step (ii), pass 2: along x, forward FFT, product with the kernel spectrum ----
// (2-D transform in x, y; direct aperiodic sum along z), inverse FFT.  MODE 1 only
// transforms forward and keeps all Lx slots (used to build the spectrum).
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_fft_x(const cplx<T>* in, cplx<T>* out, int nx_in, int Ly, int nz,
                                               int B, FftPlan P, const cplx<T>* __restrict__ twg,
                                               const cplx<T>* __restrict__ gt, const int* __restrict__ rev_x,
                                               const int* __restrict__ rev_y) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  const int L = P.L;
  cplx<T>* buf = tw + L;
  const int ld = L;
  const int nkb = Ly / B;
  const int64_t plane = blockIdx.x / nkb;
  const int kb = blockIdx.x - int(plane) * nkb;
  const int lines = B * nz;
  const int64_t row = int64_t(Ly) * nz;  // stride between x rows
  const cplx<T>* src = in + plane * int64_t(nx_in) * row + int64_t(kb) * lines;
  cplx<T>* dst = out + plane * int64_t(nx_in) * row + int64_t(kb) * lines;
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twg[i];
  batched_copy<8, T>(
      nx_in * lines,
      [&](int e) {
        const int x = e / lines, l = e - x * lines;
        return src[int64_t(x) * row + l];
      },
      [&](int e, cplx<T> v) {
        const int x = e / lines, l = e - x * lines;
        buf[l * ld + x] = v;
      });
  for (int e = threadIdx.x; e < (L - nx_in) * lines; e += blockDim.x) {
    const int l = e / (L - nx_in), x = nx_in + (e - l * (L - nx_in));
    buf[l * ld + x] = cmk<T>(0, 0);
  }
  __syncthreads();
  lds_fft_fwd(buf, ld, lines, P, tw);
  if (MODE == 0) {
    const int half_y = Ly / 2 + 1;
    for (int it = threadIdx.x; it < L * B; it += blockDim.x) {
      const int b = it / L, kp = it - b * L;
      int kx = rev_x[kp];
      kx = min(kx, L - kx);
      int ky = rev_y[kb * B + b];
      ky = min(ky, Ly - ky);
      const cplx<T>* g = gt + (int64_t(kx) * half_y + ky) * nz;
      cplx<T> gv[kMaxNz], v[kMaxNz];
#pragma unroll
      for (int z = 0; z < kMaxNz; ++z) {
        gv[z] = z < nz ? g[z] : cmk<T>(0, 0);
        v[z] = z < nz ? buf[(b * nz + z) * ld + kp] : cmk<T>(0, 0);
      }
#pragma unroll
      for (int z = 0; z < kMaxNz; ++z) {
        if (z < nz) {
          cplx<T> acc = cmk<T>(0, 0);
#pragma unroll
          for (int zp = 0; zp < kMaxNz; ++zp) cfma(acc, gv[z > zp ? z - zp : zp - z], v[zp]);
          buf[(b * nz + z) * ld + kp] = acc;
        }
      }
    }
    __syncthreads();
    lds_fft_inv(buf, ld, lines, P, tw);
  }
  for (int e = threadIdx.x; e < nx_in * lines; e += blockDim.x) {
    const int x = e / lines, l = e - x * lines;
    dst[int64_t(x) * row + l] = buf[l * ld + x];
  }
}

// ---- step (ii), pass 3: inverse FFT along y, keep the unpadded nodes -------------
template <typename T>
__global__ void __launch_bounds__(256) k_fft_y_inv(const cplx<T>* in, cplx<T>* out, int ny, int nz,
                                                   FftPlan P, const cplx<T>* __restrict__ twg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  const int L = P.L;
  cplx<T>* buf = tw + L;
  const int ld = L;
  const int64_t plane = blockIdx.x;
  const cplx<T>* src = in + plane * int64_t(L) * nz;
  for (int i = threadIdx.x; i < L; i += blockDim.x) tw[i] = twg[i];
  batched_copy<8, T>(
      L * nz, [&](int e) { return src[e]; },
      [&](int e, cplx<T> v) {
        const int y = e / nz, z = e - y * nz;
        buf[z * ld + y] = v;
      });
  __syncthreads();
  lds_fft_inv(buf, ld, nz, P, tw);
  cplx<T>* dst = out + plane * int64_t(ny) * nz;
  for (int e = threadIdx.x; e < ny * nz; e += blockDim.x) {
    const int y = e / nz, z = e - y * nz;
    dst[e] = buf[z * ld + y];
  }
}

// tw[0, L) <- twg, every load issued before the first LDS store
template <typename T, int L>
__device__ __forceinline__ void load_twiddles(cplx<T>* tw, const cplx<T>* __restrict__ twg) {
  constexpr int kMaxPer = 8;
  const int per = (L + int(blockDim.x) - 1) / int(blockDim.x);
  cplx<T> v[kMaxPer];
#pragma unroll
  for (int u = 0; u < kMaxPer; ++u) {
    const int i = min(int(threadIdx.x) + u * int(blockDim.x), L - 1);
    v[u] = twg[i];
  }
#pragma unroll
  for (int u = 0; u < kMaxPer; ++u) {
    const int i = int(threadIdx.x) + u * int(blockDim.x);
    if (u < per && i < L) tw[i] = v[u];
  }
  for (int i = int(threadIdx.x) + kMaxPer * int(blockDim.x); i < L; i += blockDim.x) tw[i] = twg[i];
}

// ---- step (ii) with register DFTs (four-step, natural order) for L = L1 L2 --------
// Same three passes as above; lines are held at the padded slots of fft4_lines, and
// spectra are in natural order, so no digit-reversal tables are involved.
template <typename T, int L1, int L2, int NZ>
__global__ void __launch_bounds__(512) k_fft4_y_fwd(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                    int ny_in, int nz_rt, const cplx<T>* __restrict__ twg) {
  constexpr int L = L1 * L2, LD = f4_ld<L1, L2>();
  const int nz = NZ > 0 ? NZ : nz_rt;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf = tw + L;
  const int64_t plane = blockIdx.x;
  const cplx<T>* src = in + plane * int64_t(ny_in) * nz;
  load_twiddles<T, L>(tw, twg);
  batched_copy<8, T>(
      ny_in * nz, [&](int e) { return src[e]; },
      [&](int e, cplx<T> v) {
        const int y = e / nz, z = e - y * nz;
        buf[z * LD + f4_slot<L2>(y)] = v;
      });
  // zero padding, up to the last row the pruned first pass reads
  constexpr int kRead = (L1 / 2 + 1) * L2;
  for (int e = threadIdx.x; e < (kRead - ny_in) * nz; e += blockDim.x) {
    const int y = ny_in + e / nz, z = e - (y - ny_in) * nz;
    buf[z * LD + f4_slot<L2>(y)] = cmk<T>(0, 0);
  }
  __syncthreads();
  fft4_lines<T, L1, L2, true, true, false>(buf, nz, tw);
  cplx<T>* dst = out + plane * int64_t(L) * nz;
  for (int e = threadIdx.x; e < L * nz; e += blockDim.x) {
    const int y = e / nz, z = e - y * nz;
    dst[e] = buf[z * LD + f4_slot<L2>(y)];
  }
}

template <typename T, int L1, int L2, int NZ>
__global__ void __launch_bounds__(512) k_fft4_x(const cplx<T>* in, cplx<T>* out, int nx_in, int Ly, int nz_rt, int B,
                                                int n_blocks, const cplx<T>* __restrict__ twg,
                                                const cplx<T>* __restrict__ gt) {
  constexpr int L = L1 * L2, LD = f4_ld<L1, L2>();
  constexpr int ZM = NZ > 0 ? NZ : kMaxNz;  // unrolled z extent
  const int nz = NZ > 0 ? NZ : nz_rt;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf = tw + L;
  const int nkb = Ly / B;
  // Workgroups go to the XCDs round-robin by index; this numbering gives each XCD a
  // contiguous run of line blocks, so the neighbouring blocks that share cache lines
  // (a block's rows are only B nz values long) are read through the same L2.
  const int nblk = int(gridDim.x), per_xcd = (nblk + kXcds - 1) / kXcds;
  const int lb = int(blockIdx.x % kXcds) * per_xcd + int(blockIdx.x / kXcds);
  if (lb >= n_blocks) return;
  const int64_t plane = lb / nkb;
  const int kb = lb - int(plane) * nkb;
  const int lines = B * nz;
  const int64_t row = int64_t(Ly) * nz;  // stride between x rows
  const cplx<T>* src = in + plane * int64_t(nx_in) * row + int64_t(kb) * lines;
  cplx<T>* dst = out + plane * int64_t(nx_in) * row + int64_t(kb) * lines;
  load_twiddles<T, L>(tw, twg);
  // thread -> (row phase x0, line l); rows x0, x0 + rpp, ... up to the last row the
  // pruned first pass reads (zero beyond nx_in)
  constexpr int kRead = (L1 / 2 + 1) * L2;
  const int rpp = int(blockDim.x) / lines;
  const int l = int(threadIdx.x) % lines, x0 = int(threadIdx.x) / lines;
  if (x0 < rpp) {
    constexpr int U = 8;
    for (int xb = x0; xb < kRead; xb += U * rpp) {
      cplx<T> v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int x = xb + u * rpp;
        v[u] = x < nx_in ? src[int64_t(x) * row + l] : cmk<T>(0, 0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int x = xb + u * rpp;
        if (x < kRead) buf[l * LD + f4_slot<L2>(x)] = v[u];
      }
    }
  }
  __syncthreads();
  fft4_lines<T, L1, L2, true, true, false>(buf, lines, tw);
  const int half_y = Ly / 2 + 1;
  for (int it = threadIdx.x; it < L * B; it += blockDim.x) {
    const int b = it / L, k = it - b * L;
    const int kx = min(k, L - k);
    int ky = kb * B + b;
    ky = min(ky, Ly - ky);
    const cplx<T>* g = gt + (int64_t(kx) * half_y + ky) * nz;
    cplx<T> gv[ZM], v[ZM];
    const int slot = f4_slot<L2>(k);
#pragma unroll
    for (int z = 0; z < ZM; ++z) {
      gv[z] = z < nz ? g[z] : cmk<T>(0, 0);
      v[z] = z < nz ? buf[(b * nz + z) * LD + slot] : cmk<T>(0, 0);
    }
#pragma unroll
    for (int z = 0; z < ZM; ++z) {
      if (z < nz) {
        cplx<T> acc = cmk<T>(0, 0);
#pragma unroll
        for (int zp = 0; zp < ZM; ++zp) cfma(acc, gv[z > zp ? z - zp : zp - z], v[zp]);
        buf[(b * nz + z) * LD + slot] = acc;
      }
    }
  }
  __syncthreads();
  fft4_lines<T, L1, L2, false, false, true>(buf, lines, tw);
  if (x0 < rpp)
    for (int x = x0; x < nx_in; x += rpp) dst[int64_t(x) * row + l] = buf[l * LD + f4_slot<L2>(x)];
}

template <typename T, int L1, int L2, int NZ>
__global__ void __launch_bounds__(512) k_fft4_y_inv(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, int ny,
                                                    int nz_rt, const cplx<T>* __restrict__ twg) {
  constexpr int L = L1 * L2, LD = f4_ld<L1, L2>();
  const int nz = NZ > 0 ? NZ : nz_rt;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* buf = tw + L;
  const int64_t plane = blockIdx.x;
  const cplx<T>* src = in + plane * int64_t(L) * nz;
  load_twiddles<T, L>(tw, twg);
  batched_copy<8, T>(
      L * nz, [&](int e) { return src[e]; },
      [&](int e, cplx<T> v) {
        const int y = e / nz, z = e - y * nz;
        buf[z * LD + f4_slot<L2>(y)] = v;
      });
  __syncthreads();
  fft4_lines<T, L1, L2, false, false, true>(buf, nz, tw);
  cplx<T>* dst = out + plane * int64_t(ny) * nz;
  for (int e = threadIdx.x; e < ny * nz; e += blockDim.x) {
    const int y = e / nz, z = e - y * nz;
    dst[e] = buf[z * LD + f4_slot<L2>(y)];
  }
}

// ---- pre-corrected near field: nf = C u ----------------------------------------
// Lanes are 64 consecutive elements, a wave walks one CSR row n of the shared
// near-field block (wave-uniform entries), u is read element-fastest.  Results are
// staged in LDS and written element-major.
constexpr int kNearRows = 16;
template <typename T>
__global__ void __launch_bounds__(256) k_near(const cplx<T>* __restrict__ uT, cplx<T>* __restrict__ nf, NearArgs a,
                                              const cplx<T>* __restrict__ near_val) {
  __shared__ cplx<T> tile[kNearRows][65];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n0 = blockIdx.x * kNearRows, m0 = blockIdx.y * 64, r = blockIdx.z;
  const int m = m0 + lane;
  const bool valid = m < a.ne;
  const int ix = m % a.px, iy = m / a.px;
  const cplx<T>* ur = uT + int64_t(r) * a.N * a.ne;
  constexpr int U = 8;  // entries in flight per lane
  for (int rr = wave; rr < kNearRows; rr += 4) {
    const int n = __builtin_amdgcn_readfirstlane(n0 + rr);
    cplx<T> acc = cmk<T>(0, 0);
    if (n < a.N) {
      const int e0 = a.near_ptr[n], e1 = a.near_ptr[n + 1];
      int e = e0;
      for (; e + U <= e1; e += U) {
        cplx<T> uv[U], cv[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const int c = a.near_col[e + k];
          const int o = c >> 16, np_ = c & 0xFFFF;
          const int jx = ix + a.offsets[2 * o], jy = iy + a.offsets[2 * o + 1];
          const bool ok = valid && jx >= 0 && jx < a.px && jy >= 0 && jy < a.py;
          cv[k] = near_val[e + k];
          uv[k] = ok ? ur[int64_t(np_) * a.ne + jy * a.px + jx] : cmk<T>(0, 0);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) cfma(acc, cv[k], uv[k]);
      }
      for (; e < e1; ++e) {
        const int c = a.near_col[e];
        const int o = c >> 16, np_ = c & 0xFFFF;
        const int jx = ix + a.offsets[2 * o], jy = iy + a.offsets[2 * o + 1];
        if (valid && jx >= 0 && jx < a.px && jy >= 0 && jy < a.py)
          cfma(acc, near_val[e], ur[int64_t(np_) * a.ne + jy * a.px + jx]);
      }
    }
    tile[rr][lane] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * kNearRows; idx += 256) {
    const int mm = idx / kNearRows, nn = idx - mm * kNearRows;
    if (m0 + mm < a.ne && n0 + nn < a.N) nf[(int64_t(r) * a.ne + m0 + mm) * a.ld_nf + a.slot_of[n0 + nn]] = tile[nn][mm];
  }
}

// ---- pre-corrected near field on the matrix cores ---------------------------------
// Rows are clustered into groups of kNearGroup (16); a group's coefficients form a
// dense 16 x K block over the union of its columns (o, n').  One wave computes 16 rows x 16
// elements: A (16 x 4) straight from the block, B (4 x 16) = u of the 16 elements'
// neighbours at offset o, column n' (element-fastest, so each k reads 16 consecutive
// values).  Four real MFMAs per complex step.
template <typename T>
struct NearMfma;
template <>
struct NearMfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct NearMfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
// output row of register r in lane l: v_mfma_f32_16x16x4f32 keeps four consecutive
// rows per lane group, v_mfma_f64_16x16x4f64 interleaves them (measured on gfx950)
template <typename T>
__device__ __forceinline__ int mfma16_row(int lane, int r) {
  return sizeof(T) == 4 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

template <typename T, int EB>
__global__ void __launch_bounds__(256) k_near_mfma(const cplx<T>* __restrict__ uT, cplx<T>* __restrict__ nf,
                                                   NearArgs a, const cplx<T>* __restrict__ grp_A) {
  // four waves, one per quarter of the union columns, over EB blocks of 16 elements
  // (EB blocks share every coefficient operand load); the group's column list is
  // staged in LDS so the operand gathers wait on LDS only
  using M = NearMfma<T>;
  __shared__ cplx<T> tile[EB][4][kNearGroupDev][17];
  extern __shared__ int cols_s[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kh = wave;
  const int mblk = blockIdx.x * 16 * EB, g = blockIdx.y, r = blockIdx.z;
  const int jcol = lane & 15, kq = lane >> 4;
  // bit (dy + 2) 5 + (dx + 2): the neighbour at lattice offset (dx, dy) exists
  unsigned vmask[EB];
  const cplx<T>* ur[EB];
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    const int mb = mblk + 16 * e + jcol;
    const int ix = mb % a.px, iy = mb / a.px;
    unsigned vm = 0;
    if (mb < a.ne)
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx)
          if (ix + dx >= 0 && ix + dx < a.px && iy + dy >= 0 && iy + dy < a.py) vm |= 1u << ((dy + 2) * 5 + dx + 2);
    vmask[e] = vm;
    ur[e] = uT + int64_t(r) * a.N * a.ne + mb;
  }
  const cplx<T>* zero = static_cast<const cplx<T>*>(a.zero);
  // the group's columns plus one prefetch batch past them (the next group's or the
  // zero tail): every load below is unconditional, so the prefetch stays in flight
  const int g0 = a.grp_ptr[g], ncols = a.grp_ptr[g + 1] - g0;
  for (int t = threadIdx.x; t < ncols + kNearColTailDev; t += blockDim.x) cols_s[t] = a.grp_col[g0 + t];
  __syncthreads();
  const int quarter = ncols / 4;  // column counts are multiples of four K quarters of whole batches
  const int k0 = kh * quarter, k1 = k0 + quarter;
  const cplx<T>* Ag = grp_A + int64_t(g0) * kNearGroupDev;
  // three real products per complex step: re.re, im.im and (re + im).(re + im)
  typename M::acc_t accRR[EB] = {}, accII[EB] = {}, accSS[EB] = {};
  constexpr int P = 4;  // K-steps per batch; the next batch is loaded ahead (8 measured 2% slower in FP32)
  auto fetch = [&](int k, cplx<T>& av, cplx<T>(&bv)[EB]) {
    const int col = cols_s[k + kq];
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const bool ok = (vmask[e] >> (col & 31)) & 1u;
      bv[e] = *(ok ? ur[e] + (col >> 5) : zero);  // absent neighbours read a zero
    }
    av = Ag[int64_t(k + kq) * kNearGroupDev + jcol];
  };
  cplx<T> ca[P], cb[P][EB];
#pragma unroll
  for (int u = 0; u < P; ++u) fetch(k0 + 4 * u, ca[u], cb[u]);
  for (int k = k0; k < k1; k += 4 * P) {
    cplx<T> na[P], nb[P][EB];
#pragma unroll
    for (int u = 0; u < P; ++u) fetch(k + 4 * P + 4 * u, na[u], nb[u]);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const T as = ca[u].re + ca[u].im;
#pragma unroll
      for (int e = 0; e < EB; ++e) {
        accRR[e] = M::mma(ca[u].re, cb[u][e].re, accRR[e]);
        accII[e] = M::mma(ca[u].im, cb[u][e].im, accII[e]);
        accSS[e] = M::mma(as, cb[u][e].re + cb[u][e].im, accSS[e]);
      }
    }
#pragma unroll
    for (int u = 0; u < P; ++u) {
      ca[u] = na[u];
#pragma unroll
      for (int e = 0; e < EB; ++e) cb[u][e] = nb[u][e];
    }
  }
#pragma unroll
  for (int e = 0; e < EB; ++e)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
      tile[e][kh][mfma16_row<T>(lane, rr)][jcol] =
          cmk<T>(accRR[e][rr] - accII[e][rr], accSS[e][rr] - accRR[e][rr] - accII[e][rr]);
  __syncthreads();
  // output in group-slot order: 16 consecutive slots per element
  const int s0 = g * kNearGroupDev;
  for (int idx = threadIdx.x; idx < 16 * EB * kNearGroupDev; idx += 256) {
    const int mm = idx / kNearGroupDev, nn = idx - mm * kNearGroupDev;
    const int e = mm >> 4, me = mm & 15;
    if (mblk + mm < a.ne)
      nf[(int64_t(r) * a.ne + mblk + mm) * a.ld_nf + s0 + nn] =
          cadd(cadd(tile[e][0][nn][me], tile[e][1][nn][me]), cadd(tile[e][2][nn][me], tile[e][3][nn][me]));
  }
}

// ---- step (iii) + combine: one workgroup per tile of elements ---------------------
// The tile's box of grid potentials (4 psi) and, in MODE 0, the tile's input rows are
// staged in LDS; every basis gathers its (N_O+1)^3 nodes per psi from LDS.  MODE 0: y = D x - (v + nf); 1: y = v + nf;
// 2: y = v, with v = -j k eta0 [sum_{x,y,z} I_psi Phi_psi - k^-2 I_phi Phi_phi].
template <typename T, int MODE, int QS>
__global__ void __launch_bounds__(sizeof(T) == sizeof(float) ? 1024 : 512)
    k_interp(const cplx<T>* __restrict__ Phi, const cplx<T>* __restrict__ nf, const cplx<T>* __restrict__ x,
             cplx<T>* __restrict__ y, InterpArgs a, const T* __restrict__ Wt, const cplx<T>* __restrict__ d_val) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cplx<T>* box = reinterpret_cast<cplx<T>*>(smem_raw);
  const int ntx = (a.px + a.TX - 1) / a.TX;
  const int tile = blockIdx.x, r = blockIdx.y;
  const int ix0 = (tile % ntx) * a.TX, iy0 = (tile / ntx) * a.TY;
  const int gx0 = ix0 * a.pitch, gy0 = iy0 * a.pitch;
  const int bx = min(a.pitch * (a.TX - 1) + a.ex, a.nx - gx0);
  const int by = min(a.pitch * (a.TY - 1) + a.ey, a.ny - gy0);
  const int bz = a.nz;
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const cplx<T>* ph = Phi + int64_t(r) * 4 * nodes;
  const int run = by * bz;  // contiguous run per (psi, x)
  batched_copy<12, T>(
      4 * bx * run,
      [&](int idx) {
        const int p = idx / (bx * run);
        const int rem = idx - p * bx * run;
        const int lx = rem / run, k = rem - lx * run;
        return ph[p * nodes + (int64_t(gx0 + lx) * a.ny + gy0) * a.nz + k];
      },
      [&](int idx, cplx<T> v) { box[idx] = v; });
  constexpr int kMaxTile = 4;
  const int64_t rows = int64_t(a.ne) * a.N;
  // elements of this tile, in order
  int ne_t = 0;
  int tm[kMaxTile], tox[kMaxTile], toy[kMaxTile];
  for (int ty = 0; ty < a.TY; ++ty)
    for (int tx = 0; tx < a.TX; ++tx) {
      const int ix = ix0 + tx, iy = iy0 + ty;
      if (ix < a.px && iy < a.py && ne_t < kMaxTile) {
        tm[ne_t] = iy * a.px + ix;
        tox[ne_t] = tx * a.pitch;
        toy[ne_t] = ty * a.pitch;
        ++ne_t;
      }
    }
  // the tile's input rows, for the D product
  cplx<T>* xs = box + 4 * bx * run;
  if constexpr (MODE == 0) {
    for (int e = 0; e < ne_t; ++e) {
      const cplx<T>* xr = x + int64_t(r) * rows + int64_t(tm[e]) * a.N;
      batched_copy<4, T>(
          a.N, [&](int idx) { return xr[idx]; }, [&](int idx, cplx<T> v) { xs[e * a.N + idx] = v; });
    }
  }
  __syncthreads();
  constexpr int q = QS, q3 = QS * QS * QS;
#pragma unroll 1
  for (int n = threadIdx.x; n < a.N; n += blockDim.x) {
    const int sx = a.sloc[3 * n], sy = a.sloc[3 * n + 1], oz = a.sloc[3 * n + 2];
    cplx<T> acc[kMaxTile];
#pragma unroll
    for (int e = 0; e < kMaxTile; ++e) acc[e] = cmk<T>(0, 0);
#pragma unroll(sizeof(T) == 4 ? 4 : 2)
    for (int p = 0; p < 4; ++p) {
      T w[q3];
#pragma unroll
      for (int t = 0; t < q3; ++t) w[t] = Wt[(int64_t(p) * q3 + t) * a.N + n];
      const T sg = p < 3 ? T(1) : T(a.sig_phi);
      const cplx<T>* f = box + p * bx * run;
#pragma unroll
      for (int e = 0; e < kMaxTile; ++e) {
        if (e < ne_t) {
          cplx<T> sacc = cmk<T>(0, 0);
#pragma unroll
          for (int i = 0; i < q; ++i)
#pragma unroll
            for (int j = 0; j < q; ++j) {
              const cplx<T>* fr = f + ((tox[e] + sx + i) * by + (toy[e] + sy + j)) * bz + oz;
#pragma unroll
              for (int l = 0; l < q; ++l) cfmas(sacc, w[(i * q + j) * q + l], fr[l]);
            }
          cfmas(acc[e], sg, sacc);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < kMaxTile; ++e) {
      if (e < ne_t) {
        const int64_t rowbase = int64_t(r) * rows + int64_t(tm[e]) * a.N;
        cplx<T> out = cmk<T>(T(a.keta) * acc[e].im, -T(a.keta) * acc[e].re);  // -j k eta0 * acc
        if (MODE != 2) out = cadd(out, nf[(int64_t(r) * a.ne + tm[e]) * a.ld_nf + a.slot_of[n]]);
        if (MODE == 0) {
          // D row n: slot-major padded layout, so every slot's loads are independent
          const cplx<T>* xe = xs + e * a.N;
          cplx<T> dx = cmk<T>(0, 0);
#pragma unroll 4
          for (int sl = 0; sl < a.dmax; ++sl) {
            const int64_t at = int64_t(sl) * a.N + n;
            cfma(dx, d_val[at], xe[a.d_colT[at]]);
          }
          out = csub(dx, out);
        }
        y[rowbase + n] = out;
      }
    }
  }
}

// ---- section III: block-diagonal macromodel product, grouped complex GEMM --------
// U[:, c] = M_t X[:, c] for every column c = r * n_elem + m of an element of kind t,
// on the matrix cores: each complex step is three real products (re.re, im.im and
// (re + im).(re + im)), combined after the K loop; the output is written
// element-fastest, uT[r][i][m].

// Tile: 32 rows x kGemmCols columns per workgroup; its four waves split K in four
// contiguous ranges and read their MFMA operands straight from global memory (A:
// two 32-value row segments per step, B: per-column runs that stay in L1); the four
// partial tiles are summed in LDS in a fixed order.
constexpr int kGemmCols = 32;
constexpr int kGemmRows = 32;

__device__ __forceinline__ void gemm_tile_setup(const GemmArgs& a, int& t, int* cols, int64_t* colbase) {
  t = 0;
  int tile = blockIdx.x;
  while (t + 1 < a.n_types && tile >= a.tile_start[t + 1]) ++t;
  tile -= a.tile_start[t];
  const int c0 = tile * kGemmCols;
  const int ncols = a.R * a.type_count[t];
  if (threadIdx.x < kGemmCols) {
    const int c = c0 + threadIdx.x;
    const int col = c < ncols ? a.col_list[a.col_start[t] + c] : -1;
    cols[threadIdx.x] = col;
    colbase[threadIdx.x] = col < 0 ? -1 : int64_t(col / a.ne) * a.N * a.ne + (col % a.ne);
  }
}

// sum the four partial tiles and write rows i0 .. i0+31 element-fastest
template <typename T>
__device__ __forceinline__ void gemm_reduce_store(const cplx<T>* part, cplx<T>* U, const int64_t* colbase, int N, int ne,
                                                  int i0) {
  for (int idx = threadIdx.x; idx < kGemmRows * kGemmCols; idx += blockDim.x) {
    const int row = idx / kGemmCols, col = idx % kGemmCols;
    cplx<T> acc = part[row * (kGemmCols + 1) + col];
#pragma unroll
    for (int w = 1; w < 4; ++w) acc = cadd(acc, part[(w * kGemmRows + row) * (kGemmCols + 1) + col]);
    const int64_t cb = colbase[col];
    if (cb >= 0 && i0 + row < N) U[cb + int64_t(i0 + row) * ne] = acc;
  }
}

__global__ void __launch_bounds__(256) k_gemm_f32(const cplx<float>* __restrict__ M, const cplx<float>* __restrict__ X,
                                                  cplx<float>* __restrict__ U, GemmArgs a) {
  __shared__ cplx<float> part[4 * kGemmRows * (kGemmCols + 1)];
  __shared__ int cols[kGemmCols];
  __shared__ int64_t colbase[kGemmCols];
  int t;
  gemm_tile_setup(a, t, cols, colbase);
  __syncthreads();
  const int N = a.N, i0 = blockIdx.y * kGemmRows;
  const cplx<float>* Mt = M + int64_t(t) * a.Krows * N;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 31, kk = lane >> 5;
  const int colj = cols[lane & 31];
  // Every operand load is unconditional, so the prefetched batch stays in flight:
  // rows past N and padding columns read valid data whose outputs are discarded, and
  // the K range of each wave runs over M's zero rows past N (X is clamped there).
  const int ir = min(i0 + i, N - 1);
  const int kq = a.Kq, kb = w * kq, ke = kb + kq;
  const cplx<float>* xc = X + int64_t(max(colj, 0)) * N;
  auto fetch = [&](int k, cplx<float>& av, cplx<float>& bv) {
    const int kk2 = k + kk;
    av = Mt[int64_t(kk2) * N + ir];
    bv = xc[min(kk2, N - 1)];
  };
  // three real products per complex step: re.re, im.im and (re + im).(re + im)
  f32x16 accRR = {}, accII = {}, accSS = {};
  constexpr int P = 8;
  cplx<float> ca[P], cb[P];
#pragma unroll
  for (int u = 0; u < P; ++u) fetch(kb + 2 * u, ca[u], cb[u]);
  for (int k = kb; k < ke; k += 2 * P) {
    cplx<float> na[P], nb[P];
#pragma unroll
    for (int u = 0; u < P; ++u) fetch(k + 2 * P + 2 * u, na[u], nb[u]);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      accRR = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[u].re, cb[u].re, accRR, 0, 0, 0);
      accII = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[u].im, cb[u].im, accII, 0, 0, 0);
      accSS = __builtin_amdgcn_mfma_f32_32x32x2f32(ca[u].re + ca[u].im, cb[u].re + cb[u].im, accSS, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < P; ++u) {
      ca[u] = na[u];
      cb[u] = nb[u];
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);  // v_mfma_f32_32x32x2f32 output row
    part[(w * kGemmRows + row) * (kGemmCols + 1) + (lane & 31)] =
        cmk<float>(accRR[r] - accII[r], accSS[r] - accRR[r] - accII[r]);
  }
  __syncthreads();
  gemm_reduce_store<float>(part, U, colbase, N, a.ne, i0);
}

// ---- split-BF16 macromodel product (the mixed path's bf16 matrix cores) -------------
// Every FP32 value v is carried as three bfloat16 terms v = h + m + l (h = bf16(v),
// m = bf16(v - h), l = bf16(v - h - m); each difference is exact in FP32), and a real
// product uses the six bf16 products h.h + h.m + m.h + h.l + l.h + m.m, accumulated
// in FP32 by v_mfma_f32_32x32x16_bf16 (the dropped terms are below 2^-24 relative).
// Complex steps take the four real products re.re - im.im and re.im + im.re (four
// rather than the FP32 kernel's three: the kernel is bound by the bytes of M it
// streams, and the (re + im) planes would add half of them again).  M is pre-split on
// the host into 6 planes (h, m, l of re, then of im) laid out [plane][k / 8][row][8]
// so a lane's 8 consecutive k of one row are one 16-byte load; X is split on the fly
// (8 consecutive k of one column, 64 contiguous bytes, per lane).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split3(float v, __bf16& h, __bf16& m, __bf16& l) {
  h = __bf16(v);
  const float r1 = v - float(h);
  m = __bf16(r1);
  l = __bf16(r1 - float(m));
}

__global__ void __launch_bounds__(256) k_gemm_bf16x3(const u32x4* __restrict__ Mb, const cplx<float>* __restrict__ X,
                                                     cplx<float>* __restrict__ U, GemmArgs a) {
  __shared__ cplx<float> part[4 * kGemmRows * (kGemmCols + 1)];
  __shared__ int cols[kGemmCols];
  __shared__ int64_t colbase[kGemmCols];
  int t;
  gemm_tile_setup(a, t, cols, colbase);
  __syncthreads();
  const int N = a.N, i0 = blockIdx.y * kGemmRows;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 31, hk = lane >> 5;
  const int ir = min(i0 + i, N - 1);  // rows past N: any valid row, outputs discarded
  const int colj = max(cols[lane & 31], 0);
  const int kq = a.Kq, kb = w * kq, ke = kb + kq;
  const int KB = a.Krows / 8;
  const u32x4* Mt = Mb + int64_t(t) * 6 * KB * N;
  const cplx<float>* xc = X + int64_t(colj) * N;
  // lane's 8 k of the chunk at k0: A rows ir, k0 + 8 hk .. + 7 (6 planes); B column colj
  auto load_a = [&](int k0, u32x4* av) {
#pragma unroll
    for (int p = 0; p < 6; ++p) av[p] = Mt[(int64_t(p) * KB + (k0 >> 3) + hk) * N + ir];
  };
  auto load_b = [&](int k0, cplx<float>* bv) {
    const int kk = k0 + 8 * hk;
    const cplx<float>* src = xc + (kk + 8 <= N ? kk : 0);  // past N: any finite values (M rows are zero)
#pragma unroll
    for (int u = 0; u < 8; ++u) bv[u] = src[u];
  };
  f32x16 accRe = {}, accIm = {};
  auto mma6 = [](f32x16 acc, const bf16x8* a3, const bf16x8* b3) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[0], b3[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[0], b3[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[1], b3[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[0], b3[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[2], b3[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3[1], b3[1], acc, 0, 0, 0);
    return acc;
  };
  u32x4 ca[6], na[6];
  cplx<float> cb[8], nb[8];
  load_a(kb, ca);
  load_b(kb, cb);
  for (int k0 = kb; k0 < ke; k0 += 16) {
    if (k0 + 16 < ke) {
      load_a(k0 + 16, na);
      load_b(k0 + 16, nb);
    }
    bf16x8 br[3], bi[3], bn[3];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      __bf16 h, m, l;
      split3(cb[u].re, h, m, l);
      br[0][u] = h;
      br[1][u] = m;
      br[2][u] = l;
      split3(cb[u].im, h, m, l);
      bi[0][u] = h;
      bi[1][u] = m;
      bi[2][u] = l;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {  // -im, exactly: the sign bits of its split terms flipped
      u32x4 t = __builtin_bit_cast(u32x4, bi[q]);
#pragma unroll
      for (int c = 0; c < 4; ++c) t[c] ^= 0x80008000u;
      bn[q] = __builtin_bit_cast(bf16x8, t);
    }
    bf16x8 ar[3], ai[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      ar[p] = __builtin_bit_cast(bf16x8, ca[p]);
      ai[p] = __builtin_bit_cast(bf16x8, ca[3 + p]);
    }
    accRe = mma6(accRe, ar, br);
    accRe = mma6(accRe, ai, bn);
    accIm = mma6(accIm, ar, bi);
    accIm = mma6(accIm, ai, br);
#pragma unroll
    for (int p = 0; p < 6; ++p) ca[p] = na[p];
#pragma unroll
    for (int u = 0; u < 8; ++u) cb[u] = nb[u];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);  // 32 x 32 MFMA output row
    part[(w * kGemmRows + row) * (kGemmCols + 1) + (lane & 31)] =
        cmk<float>(accRe[r], accIm[r]);
  }
  __syncthreads();
  gemm_reduce_store<float>(part, U, colbase, N, a.ne, i0);
}

__global__ void __launch_bounds__(256) k_gemm_f64(const cplx<double>* __restrict__ M,
                                                  const cplx<double>* __restrict__ X, cplx<double>* __restrict__ U,
                                                  GemmArgs a) {
  __shared__ cplx<double> part[4 * kGemmRows * (kGemmCols + 1)];
  __shared__ int cols[kGemmCols];
  __shared__ int64_t colbase[kGemmCols];
  int t;
  gemm_tile_setup(a, t, cols, colbase);
  __syncthreads();
  const int N = a.N, i0 = blockIdx.y * kGemmRows;
  const cplx<double>* Mt = M + int64_t(t) * a.Krows * N;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l16 = lane & 15, kk = lane >> 4;
  int colq[2], rowq[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    colq[q] = max(cols[q * 16 + l16], 0);  // padding columns: any valid column, outputs discarded
    rowq[q] = min(i0 + q * 16 + l16, N - 1);
  }
  // unconditional loads over M's zero rows past N, as in the FP32 kernel
  const int kq = a.Kq, kb = w * kq, ke = kb + kq;
  auto fetch = [&](int k, cplx<double>* av, cplx<double>* bv) {
    const int kk2 = k + kk;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      av[q] = Mt[int64_t(kk2) * N + rowq[q]];
      bv[q] = X[int64_t(colq[q]) * N + min(kk2, N - 1)];
    }
  };
  f64x4 accR[2][2] = {}, accI[2][2] = {};
  constexpr int P = 4;
  cplx<double> ca[P][2], cb[P][2];
#pragma unroll
  for (int u = 0; u < P; ++u) fetch(kb + 4 * u, ca[u], cb[u]);
  for (int k = kb; k < ke; k += 4 * P) {
    cplx<double> na[P][2], nb[P][2];
#pragma unroll
    for (int u = 0; u < P; ++u) fetch(k + 4 * P + 4 * u, na[u], nb[u]);
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          accR[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u][ti].re, cb[u][tj].re, accR[ti][tj], 0, 0, 0);
          accR[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ca[u][ti].im, cb[u][tj].im, accR[ti][tj], 0, 0, 0);
          accI[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u][ti].re, cb[u][tj].im, accI[ti][tj], 0, 0, 0);
          accI[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(ca[u][ti].im, cb[u][tj].re, accI[ti][tj], 0, 0, 0);
        }
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        ca[u][q] = na[u][q];
        cb[u][q] = nb[u][q];
      }
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = ti * 16 + (lane >> 4) + 4 * r;  // v_mfma_f64_16x16x4f64 output row
        part[(w * kGemmRows + row) * (kGemmCols + 1) + tj * 16 + l16] = cmk<double>(accR[ti][tj][r], accI[ti][tj][r]);
      }
  __syncthreads();
  gemm_reduce_store<double>(part, U, colbase, N, a.ne, i0);
}

// ---- setup helpers -----------------------------------------------------------------
// Periodic samples of the grid Green's function on Lx x Ly x nz, layout [x][y][z]:
// G(d) = exp(-j k h |d|) / (4 pi h |d|) with the x, y separations folded to min(d, L - d).
__global__ void k_kernel_samples(cplx<double>* out, int Lx, int Ly, int nz, double kh, double h) {
  const int64_t n = int64_t(Lx) * Ly * nz;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int z = int(i % nz);
  const int y = int((i / nz) % Ly);
  const int x = int(i / (int64_t(nz) * Ly));
  const int dx = min(x, Lx - x), dy = min(y, Ly - y);
  const double d = sqrt(double(dx) * dx + double(dy) * dy + double(z) * z);
  if (d == 0.0) {
    out[i] = cmk<double>(0.0, 0.0);
    return;
  }
  double s, c;
  sincos(kh * d, &s, &c);
  const double f = 1.0 / (4.0 * 3.14159265358979323846 * h * d);
  out[i] = cmk<double>(c * f, -s * f);
}

// Natural-order spectrum on kx <= Lx/2, ky <= Ly/2, scaled by 1 / (Lx Ly).
template <typename T>
__global__ void k_extract_spectrum(const cplx<double>* raw, cplx<T>* gt, int Lx, int Ly, int nz,
                                   const int* pos_x, const int* pos_y) {
  const int hx = Lx / 2 + 1, hy = Ly / 2 + 1;
  const int64_t n = int64_t(hx) * hy * nz;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int z = int(i % nz);
  const int ky = int((i / nz) % hy);
  const int kx = int(i / (int64_t(nz) * hy));
  const cplx<double> v = raw[(int64_t(pos_x[kx]) * Ly + pos_y[ky]) * nz + z];
  const double s = 1.0 / (double(Lx) * double(Ly));
  gt[i] = cmk<T>(T(v.re * s), T(v.im * s));
}

// b[r][m][n] = exp(-j k kinc_r . c_m) * loc[r][n]
__global__ void k_expand_rhs(const cplx<double>* loc, const double* kinc, cplx<double>* b, int R, int ne, int N,
                             int px, double pitch_len, double k) {
  const int64_t rows = int64_t(ne) * N;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * R) return;
  const int r = int(i / rows);
  const int64_t mn = i - int64_t(r) * rows;
  const int m = int(mn / N), n = int(mn - int64_t(m) * N);
  const double cx = (m % px) * pitch_len, cy = (m / px) * pitch_len;
  const double ph = -k * (kinc[3 * r] * cx + kinc[3 * r + 1] * cy);
  double s, c;
  sincos(ph, &s, &c);
  b[i] = cmul(loc[int64_t(r) * N + n], cmk<double>(c, s));
}

template <typename Tin, typename Tout>
__global__ void k_convert(const cplx<Tin>* in, cplx<Tout>* out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cmk<Tout>(Tout(in[i].re), Tout(in[i].im));
}

// ---- launchers -------------------------------------------------------------------
static inline unsigned blocks_for(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

template <typename T>
hipError_t launch_project(const cplx<T>* uT, cplx<T>* Q, const ProjArgs& a, const T* Wp, hipStream_t s) {
  const int64_t ne64 = (a.ne + 63) / 64 * 64;
  const int64_t n = ne64 * a.pitch * a.pitch * a.ez * a.R;
  const int wx = std::max(a.ex - a.pitch, 0), wy = std::max(a.ey - a.pitch, 0);
  const int64_t tail_waves = int64_t(wx * a.pitch * a.ez * ((a.py + 63) / 64) + a.pitch * wy * a.ez * ((a.px + 63) / 64) +
                                     wx * wy * a.ez) * a.R;
  hipLaunchKernelGGL(k_project<T>, dim3(unsigned(tail_waves + blocks_for(n, 64))), dim3(64), 0, s, uT, Q, a, Wp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transpose(const cplx<T>* x, cplx<T>* xT, int R, int ne, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose<T>, dim3((N + 31) / 32, (ne + 31) / 32, R), dim3(256), 0, s, x, xT, ne, N);
  return hipGetLastError();
}

// the three passes with register DFTs: (LX1, LX2) along x, (LY1, LY2) along y; NZ > 0
// fixes the node count along z at compile time
template <typename T, int LX1, int LX2, int LY1, int LY2, int NZ>
hipError_t launch_convolve4_z(const cplx<T>* Q, cplx<T>* Phi, cplx<T>* S, const ConvArgs& a, hipStream_t s,
                              hipEvent_t* ev) {
  const int planes = a.R * 4 * a.nx;
  constexpr int Ly = LY1 * LY2, Lx = LX1 * LX2;
  auto threads = [](int lines, int l1, int l2) { return unsigned((lines * std::max(l1, l2) + 63) / 64 * 64); };
  if (threads(a.B * a.nz, LX1, LX2) > 512 || threads(a.nz, LY1, LY2) > 512) return hipErrorInvalidConfiguration;
  size_t lds = sizeof(cplx<T>) * (size_t(Ly) + size_t(a.nz) * f4_ld<LY1, LY2>());
  hipError_t e = hipSuccess;
  if (a.passes & 1) {
    hipLaunchKernelGGL((k_fft4_y_fwd<T, LY1, LY2, NZ>), dim3(planes), dim3(threads(a.nz, LY1, LY2)), lds, s, Q, S,
                       a.ny, a.nz, reinterpret_cast<const cplx<T>*>(a.tw_y));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev) (void)hipEventRecord(ev[0], s);
  if (a.passes & 2) {
    const int nkb = Ly / a.B, nblocks = a.R * 4 * nkb;
    cplx<T>* xo = a.x_out ? static_cast<cplx<T>*>(a.x_out) : S;
    lds = sizeof(cplx<T>) * (size_t(Lx) + size_t(a.B) * a.nz * f4_ld<LX1, LX2>());
    hipLaunchKernelGGL((k_fft4_x<T, LX1, LX2, NZ>), dim3((nblocks + kXcds - 1) / kXcds * kXcds),
                       dim3(threads(a.B * a.nz, LX1, LX2)), lds, s, S, xo, a.nx, Ly, a.nz, a.B, nblocks,
                       reinterpret_cast<const cplx<T>*>(a.tw_x), reinterpret_cast<const cplx<T>*>(a.gt));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (a.passes & 4) {
    lds = sizeof(cplx<T>) * (size_t(Ly) + size_t(a.nz) * f4_ld<LY1, LY2>());
    hipLaunchKernelGGL((k_fft4_y_inv<T, LY1, LY2, NZ>), dim3(planes), dim3(threads(a.nz, LY1, LY2)), lds, s, S, Phi,
                       a.ny, a.nz, reinterpret_cast<const cplx<T>*>(a.tw_y));
    e = hipGetLastError();
  }
  return e;
}

template <typename T, int LX1, int LX2, int LY1, int LY2>
hipError_t launch_convolve4(const cplx<T>* Q, cplx<T>* Phi, cplx<T>* S, const ConvArgs& a, hipStream_t s,
                            hipEvent_t* ev) {
  if (a.nz == 8) return launch_convolve4_z<T, LX1, LX2, LY1, LY2, 8>(Q, Phi, S, a, s, ev);
  if (a.nz == 9) return launch_convolve4_z<T, LX1, LX2, LY1, LY2, 9>(Q, Phi, S, a, s, ev);
  return launch_convolve4_z<T, LX1, LX2, LY1, LY2, 0>(Q, Phi, S, a, s, ev);
}

template <typename T, int LX1, int LX2>
hipError_t launch_convolve4_y(const cplx<T>* Q, cplx<T>* Phi, cplx<T>* S, const ConvArgs& a, hipStream_t s,
                              hipEvent_t* ev) {
#define AIM_F4(LY1, LY2) \
  if (a.Py.L == LY1 * LY2) return launch_convolve4<T, LX1, LX2, LY1, LY2>(Q, Phi, S, a, s, ev);
  AIM_F4_LENGTHS(AIM_F4)
#undef AIM_F4
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_convolve(const cplx<T>* Q, cplx<T>* Phi, cplx<T>* S, const ConvArgs& a, hipStream_t s,
                           hipEvent_t* ev) {
  if (a.f4) {
#define AIM_F4(LX1, LX2) \
  if (a.Px.L == LX1 * LX2) return launch_convolve4_y<T, LX1, LX2>(Q, Phi, S, a, s, ev);
    AIM_F4_LENGTHS(AIM_F4)
#undef AIM_F4
    return hipErrorInvalidValue;
  }
  const int planes = a.R * 4 * a.nx;
  size_t lds = sizeof(cplx<T>) * size_t(a.Py.L) * (1 + a.nz);
  hipError_t e = hipSuccess;
  if (a.passes & 1) {
    hipLaunchKernelGGL(k_fft_y_fwd<T>, dim3(planes), dim3(256), lds, s, Q, S, a.ny, a.nz, a.Py,
                       reinterpret_cast<const cplx<T>*>(a.tw_y));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev) (void)hipEventRecord(ev[0], s);
  if (a.passes & 2) {
    const int nkb = a.Py.L / a.B;
    cplx<T>* xo = a.x_out ? static_cast<cplx<T>*>(a.x_out) : S;
    lds = sizeof(cplx<T>) * size_t(a.Px.L) * (1 + a.B * a.nz);
    hipLaunchKernelGGL((k_fft_x<T, 0>), dim3(a.R * 4 * nkb), dim3(256), lds, s, S, xo, a.nx, a.Py.L, a.nz, a.B,
                       a.Px, reinterpret_cast<const cplx<T>*>(a.tw_x), reinterpret_cast<const cplx<T>*>(a.gt),
                       a.rev_x, a.rev_y);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (a.passes & 4) {
    lds = sizeof(cplx<T>) * size_t(a.Py.L) * (1 + a.nz);
    hipLaunchKernelGGL(k_fft_y_inv<T>, dim3(planes), dim3(256), lds, s, S, Phi, a.ny, a.nz, a.Py,
                       reinterpret_cast<const cplx<T>*>(a.tw_y));
    e = hipGetLastError();
  }
  return e;
}

template <typename T>
hipError_t launch_near(const cplx<T>* uT, cplx<T>* nf, const NearArgs& a, const cplx<T>* near_val, hipStream_t s) {
  if (a.grp_A) {
    // element blocks fastest, so consecutive workgroups (spread over the XCDs) share
    // the rows of u they read
    const size_t lds = sizeof(int) * size_t(a.grp_max_cols + kNearColTailDev);
    if (a.eb == 2) {
      const dim3 g((a.ne + 31) / 32, (a.N + kNearGroupDev - 1) / kNearGroupDev, a.R);
      hipLaunchKernelGGL((k_near_mfma<T, 2>), g, dim3(256), lds, s, uT, nf, a,
                         reinterpret_cast<const cplx<T>*>(a.grp_A));
    } else {
      const dim3 g((a.ne + 15) / 16, (a.N + kNearGroupDev - 1) / kNearGroupDev, a.R);
      hipLaunchKernelGGL((k_near_mfma<T, 1>), g, dim3(256), lds, s, uT, nf, a,
                         reinterpret_cast<const cplx<T>*>(a.grp_A));
    }
  } else {
    const dim3 g((a.N + kNearRows - 1) / kNearRows, (a.ne + 63) / 64, a.R);
    hipLaunchKernelGGL(k_near<T>, g, dim3(256), 0, s, uT, nf, a, near_val);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(int mode, const cplx<T>* Phi, const cplx<T>* nf, const cplx<T>* x, cplx<T>* y,
                         const InterpArgs& a, const T* Wt, const cplx<T>* d_val, hipStream_t s) {
  const int tiles = ((a.px + a.TX - 1) / a.TX) * ((a.py + a.TY - 1) / a.TY);
  const size_t lds = interp_lds_bytes(a, sizeof(cplx<T>));
  // one thread per basis function in FP32 (no serial loop over a tile's rows); FP64,
  // with twice the registers and LDS per block, ran fastest at 512 (measured, N = 648)
  const int bs = std::min(sizeof(T) == sizeof(float) ? 1024 : 512, (a.N + 63) / 64 * 64);
  const dim3 g(tiles, a.R), b(bs);
#define AIM_INTERP(M, QQ) hipLaunchKernelGGL((k_interp<T, M, QQ>), g, b, lds, s, Phi, nf, x, y, a, Wt, d_val)
#define AIM_INTERP_Q(M)                  \
  switch (a.q) {                        \
    case 2: AIM_INTERP(M, 2); break;    \
    case 3: AIM_INTERP(M, 3); break;    \
    default: AIM_INTERP(M, 4); break;   \
  }
  if (mode == 0) {
    AIM_INTERP_Q(0)
  } else if (mode == 1) {
    AIM_INTERP_Q(1)
  } else {
    AIM_INTERP_Q(2)
  }
#undef AIM_INTERP_Q
#undef AIM_INTERP
  return hipGetLastError();
}

template <typename T>
hipError_t launch_macro(const cplx<T>* M, const cplx<T>* X, cplx<T>* U, const GemmArgs& a, hipStream_t s) {
  const int tiles = a.tile_start[a.n_types];  // host copy of the tile prefix sums
  if (tiles == 0) return hipSuccess;
  const dim3 g(tiles, (a.N + kGemmRows - 1) / kGemmRows), b(256);
  if constexpr (sizeof(T) == sizeof(float)) {
    if (a.Mb)
      hipLaunchKernelGGL(k_gemm_bf16x3, g, b, 0, s, static_cast<const u32x4*>(a.Mb),
                         reinterpret_cast<const cplx<float>*>(X), reinterpret_cast<cplx<float>*>(U), a);
    else
      hipLaunchKernelGGL(k_gemm_f32, g, b, 0, s, reinterpret_cast<const cplx<float>*>(M),
                         reinterpret_cast<const cplx<float>*>(X), reinterpret_cast<cplx<float>*>(U), a);
  } else {
    hipLaunchKernelGGL(k_gemm_f64, g, b, 0, s, reinterpret_cast<const cplx<double>*>(M),
                       reinterpret_cast<const cplx<double>*>(X), reinterpret_cast<cplx<double>*>(U), a);
  }
  return hipGetLastError();
}

hipError_t launch_spectrum(cplx<double>* raw, int Lx, int Ly, int nz, double k, double h, const FftPlan& Px,
                           const FftPlan& Py, const cplx<double>* tw_x, const cplx<double>* tw_y, int B,
                           hipStream_t s) {
  const int64_t n = int64_t(Lx) * Ly * nz;
  hipLaunchKernelGGL(k_kernel_samples, dim3(blocks_for(n, 256)), dim3(256), 0, s, raw, Lx, Ly, nz, k * h, h);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  size_t lds = sizeof(cplx<double>) * size_t(Ly) * (1 + nz);
  hipLaunchKernelGGL(k_fft_y_fwd<double>, dim3(Lx), dim3(256), lds, s, raw, raw, Ly, nz, Py, tw_y);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  lds = sizeof(cplx<double>) * size_t(Lx) * (1 + B * nz);
  hipLaunchKernelGGL((k_fft_x<double, 1>), dim3(Ly / B), dim3(256), lds, s, raw, raw, Lx, Ly, nz, B, Px, tw_x,
                     (const cplx<double>*)nullptr, (const int*)nullptr, (const int*)nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_extract(const cplx<double>* raw, cplx<T>* gt, int Lx, int Ly, int nz, const int* pos_x,
                          const int* pos_y, hipStream_t s) {
  const int64_t n = int64_t(Lx / 2 + 1) * (Ly / 2 + 1) * nz;
  hipLaunchKernelGGL(k_extract_spectrum<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, raw, gt, Lx, Ly, nz, pos_x,
                     pos_y);
  return hipGetLastError();
}

hipError_t launch_expand_rhs(const cplx<double>* loc, const double* kinc, cplx<double>* b, int R, int ne, int N,
                             int px, double pitch_len, double k, hipStream_t s) {
  const int64_t n = int64_t(ne) * N * R;
  hipLaunchKernelGGL(k_expand_rhs, dim3(blocks_for(n, 256)), dim3(256), 0, s, loc, kinc, b, R, ne, N, px,
                     pitch_len, k);
  return hipGetLastError();
}

template <typename Tin, typename Tout>
hipError_t launch_convert(const cplx<Tin>* in, cplx<Tout>* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

bool fft4_supported(int L) {
#define AIM_F4(L1, L2) \
  if (L == L1 * L2) return true;
  AIM_F4_LENGTHS(AIM_F4)
#undef AIM_F4
  return false;
}

static bool f4_factors(int L, int& l1, int& l2) {
#define AIM_F4(A, B) \
  if (L == A * B) {  \
    l1 = A;          \
    l2 = B;          \
    return true;     \
  }
  AIM_F4_LENGTHS(AIM_F4)
#undef AIM_F4
  return false;
}

bool conv_fits(int Lx, int Ly, int nz, int B, bool f4, size_t elem, size_t lds_limit) {
  if (B < 1 || Ly % B != 0) return false;
  const size_t zb = size_t(B) * nz;
  if (!f4) return elem * Lx * (1 + zb) <= lds_limit && elem * Ly * (1 + size_t(nz)) <= lds_limit;
  int x1, x2, y1, y2;
  if (!f4_factors(Lx, x1, x2) || !f4_factors(Ly, y1, y2)) return false;
  // the same thread counts and LDS layouts as launch_convolve4_z
  auto threads = [](size_t lines, int l1, int l2) { return (lines * std::max(l1, l2) + 63) / 64 * 64; };
  if (threads(zb, x1, x2) > 512 || threads(nz, y1, y2) > 512) return false;
  return elem * (Lx + zb * x1 * (x2 + 1)) <= lds_limit && elem * (Ly + size_t(nz) * y1 * (y2 + 1)) <= lds_limit;
}

hipError_t configure_lds(size_t bytes) {
  const int b = int(bytes);
  hipError_t e = hipSuccess, t;
#define AIM_ATTR(f)                                                                   \
  t = hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize, b); \
  if (t != hipSuccess) e = t;
#define AIM_F4_ATTR_Z(L1, L2, NZ)                \
  AIM_ATTR((k_fft4_y_fwd<float, L1, L2, NZ>))   \
  AIM_ATTR((k_fft4_y_fwd<double, L1, L2, NZ>))  \
  AIM_ATTR((k_fft4_y_inv<float, L1, L2, NZ>))   \
  AIM_ATTR((k_fft4_y_inv<double, L1, L2, NZ>))  \
  AIM_ATTR((k_fft4_x<float, L1, L2, NZ>))       \
  AIM_ATTR((k_fft4_x<double, L1, L2, NZ>))
#define AIM_F4_ATTR(L1, L2) AIM_F4_ATTR_Z(L1, L2, 0) AIM_F4_ATTR_Z(L1, L2, 8) AIM_F4_ATTR_Z(L1, L2, 9)
  AIM_F4_LENGTHS(AIM_F4_ATTR)
#undef AIM_F4_ATTR_Z
#undef AIM_F4_ATTR
  AIM_ATTR(k_fft_y_fwd<float>)
  AIM_ATTR(k_fft_y_fwd<double>)
  AIM_ATTR(k_fft_y_inv<float>)
  AIM_ATTR(k_fft_y_inv<double>)
  AIM_ATTR((k_fft_x<float, 0>))
  AIM_ATTR((k_fft_x<double, 0>))
  AIM_ATTR((k_fft_x<double, 1>))
  AIM_ATTR((k_interp<float, 0, 2>))
  AIM_ATTR((k_interp<float, 0, 3>))
  AIM_ATTR((k_interp<float, 0, 4>))
  AIM_ATTR((k_interp<float, 1, 2>))
  AIM_ATTR((k_interp<float, 1, 3>))
  AIM_ATTR((k_interp<float, 1, 4>))
  AIM_ATTR((k_interp<float, 2, 2>))
  AIM_ATTR((k_interp<float, 2, 3>))
  AIM_ATTR((k_interp<float, 2, 4>))
  AIM_ATTR((k_interp<double, 0, 2>))
  AIM_ATTR((k_interp<double, 0, 3>))
  AIM_ATTR((k_interp<double, 0, 4>))
  AIM_ATTR((k_interp<double, 1, 2>))
  AIM_ATTR((k_interp<double, 1, 3>))
  AIM_ATTR((k_interp<double, 1, 4>))
  AIM_ATTR((k_interp<double, 2, 2>))
  AIM_ATTR((k_interp<double, 2, 3>))
  AIM_ATTR((k_interp<double, 2, 4>))
#undef AIM_ATTR
  return e;
}

template hipError_t launch_project<float>(const cplx<float>*, cplx<float>*, const ProjArgs&, const float*, hipStream_t);
template hipError_t launch_project<double>(const cplx<double>*, cplx<double>*, const ProjArgs&, const double*,
                                           hipStream_t);
template hipError_t launch_convolve<float>(const cplx<float>*, cplx<float>*, cplx<float>*, const ConvArgs&, hipStream_t,
                                           hipEvent_t*);
template hipError_t launch_convolve<double>(const cplx<double>*, cplx<double>*, cplx<double>*, const ConvArgs&,
                                            hipStream_t, hipEvent_t*);
template hipError_t launch_near<float>(const cplx<float>*, cplx<float>*, const NearArgs&, const cplx<float>*,
                                       hipStream_t);
template hipError_t launch_near<double>(const cplx<double>*, cplx<double>*, const NearArgs&, const cplx<double>*,
                                        hipStream_t);
template hipError_t launch_interp<float>(int, const cplx<float>*, const cplx<float>*, const cplx<float>*, cplx<float>*,
                                         const InterpArgs&, const float*, const cplx<float>*, hipStream_t);
template hipError_t launch_interp<double>(int, const cplx<double>*, const cplx<double>*, const cplx<double>*,
                                          cplx<double>*, const InterpArgs&, const double*, const cplx<double>*,
                                          hipStream_t);
template hipError_t launch_transpose<float>(const cplx<float>*, cplx<float>*, int, int, int, hipStream_t);
template hipError_t launch_transpose<double>(const cplx<double>*, cplx<double>*, int, int, int, hipStream_t);
template hipError_t launch_macro<float>(const cplx<float>*, const cplx<float>*, cplx<float>*, const GemmArgs&,
                                        hipStream_t);
template hipError_t launch_macro<double>(const cplx<double>*, const cplx<double>*, cplx<double>*, const GemmArgs&,
                                         hipStream_t);
template hipError_t launch_extract<float>(const cplx<double>*, cplx<float>*, int, int, int, const int*, const int*,
                                          hipStream_t);
template hipError_t launch_extract<double>(const cplx<double>*, cplx<double>*, int, int, int, const int*, const int*,
                                           hipStream_t);
template hipError_t launch_convert<double, float>(const cplx<double>*, cplx<float>*, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const cplx<float>*, cplx<double>*, int64_t, hipStream_t);

}  // namespace aimm
