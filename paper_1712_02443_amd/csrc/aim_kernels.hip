// Device kernels of the AIM matrix-vector product (section V, steps (i)-(iii)) plus
// the near-field pre-correction and the block-diagonal D term of eq. MV_product1.
//
// Layouts (complex values interleaved):
//   vectors  x, u, y : [R][n_elem][N]          (element-major unknowns)
//   grids    Q, Phi  : [R][4][nx][ny][nz]      (psi = x, y, z, phi)
//   spectrum S       : [R][4][nx][Ly][nz]      (y transformed, ky in digit-reversed slots)
#include "aim_kernels.hpp"
#include "fft.hpp"

namespace aimm {

// ---- step (i): projection, one thread per grid node, deterministic gather --------
template <typename T>
__global__ void __launch_bounds__(256) k_project(const cplx<T>* __restrict__ u, cplx<T>* __restrict__ Q,
                                                 ProjArgs a, const T* __restrict__ Wp) {
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= nodes * a.R) return;
  const int r = int(gid / nodes);
  const int64_t g = gid - int64_t(r) * nodes;
  const int gz = int(g % a.nz);
  const int gy = int((g / a.nz) % a.ny);
  const int gx = int(g / (int64_t(a.nz) * a.ny));
  cplx<T> acc[4];
  for (int p = 0; p < 4; ++p) acc[p] = cmk<T>(0, 0);
  const int tx = gx - (a.ex - 1), ty = gy - (a.ey - 1);
  const int ix_lo = tx <= 0 ? 0 : (tx + a.pitch - 1) / a.pitch;
  const int iy_lo = ty <= 0 ? 0 : (ty + a.pitch - 1) / a.pitch;
  const int ix_hi = min(a.px - 1, gx / a.pitch);
  const int iy_hi = min(a.py - 1, gy / a.pitch);
  const int64_t NQ = int64_t(a.N) * a.q3;
  for (int iy = iy_lo; iy <= iy_hi; ++iy) {
    for (int ix = ix_lo; ix <= ix_hi; ++ix) {
      const int lx = gx - ix * a.pitch, ly = gy - iy * a.pitch;
      const int node = (lx * a.ey + ly) * a.ez + gz;
      const int e0 = a.node_ptr[node], e1 = a.node_ptr[node + 1];
      const cplx<T>* ue = u + (int64_t(r) * a.ne + int64_t(iy) * a.px + ix) * a.N;
      for (int e = e0; e < e1; ++e) {
        const int ent = a.node_ent[e];
        const cplx<T> v = ue[ent / a.q3];
        for (int p = 0; p < 4; ++p) cfmas(acc[p], Wp[p * NQ + ent], v);
      }
    }
  }
  cplx<T>* out = Q + int64_t(r) * 4 * nodes + g;
  for (int p = 0; p < 4; ++p) out[p * nodes] = acc[p];
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
  for (int e = threadIdx.x; e < ny_in * nz; e += blockDim.x) {
    const int y = e / nz, z = e - y * nz;
    buf[z * ld + y] = src[e];
  }
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
  for (int e = threadIdx.x; e < nx_in * lines; e += blockDim.x) {
    const int x = e / lines, l = e - x * lines;
    buf[l * ld + x] = src[int64_t(x) * row + l];
  }
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
  for (int e = threadIdx.x; e < L * nz; e += blockDim.x) {
    const int y = e / nz, z = e - y * nz;
    buf[z * ld + y] = src[e];
  }
  __syncthreads();
  lds_fft_inv(buf, ld, nz, P, tw);
  cplx<T>* dst = out + plane * int64_t(ny) * nz;
  for (int e = threadIdx.x; e < ny * nz; e += blockDim.x) {
    const int y = e / nz, z = e - y * nz;
    dst[e] = buf[z * ld + y];
  }
}

// ---- step (iii) + near field + D: one thread per (r, element, RWG) row -----------
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_interp_combine(const cplx<T>* __restrict__ Phi,
                                                        const cplx<T>* __restrict__ u,
                                                        const cplx<T>* __restrict__ x, cplx<T>* __restrict__ y,
                                                        CombineArgs a, const T* __restrict__ Wt,
                                                        const cplx<T>* __restrict__ near_val,
                                                        const cplx<T>* __restrict__ d_val) {
  const int64_t rows = int64_t(a.ne) * a.N;
  const int64_t gid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= rows * a.R) return;
  const int r = int(gid / rows);
  const int64_t mn = gid - int64_t(r) * rows;
  const int m = int(mn / a.N), n = int(mn - int64_t(m) * a.N);
  const int ix = m % a.px, iy = m / a.px;
  const int gx = ix * a.pitch + a.sloc[3 * n], gy = iy * a.pitch + a.sloc[3 * n + 1], gz = a.sloc[3 * n + 2];
  const int64_t nodes = int64_t(a.nx) * a.ny * a.nz;
  const cplx<T>* ph = Phi + int64_t(r) * 4 * nodes;
  cplx<T> acc = cmk<T>(0, 0);
  for (int p = 0; p < 4; ++p) {
    cplx<T> s = cmk<T>(0, 0);
    const T* w = Wt + int64_t(p) * a.q3 * a.N + n;
    const cplx<T>* f = ph + p * nodes;
    int idx = 0;
    for (int i = 0; i < a.q; ++i)
      for (int j = 0; j < a.q; ++j) {
        const cplx<T>* fr = f + (int64_t(gx + i) * a.ny + (gy + j)) * a.nz + gz;
        for (int l = 0; l < a.q; ++l, ++idx) cfmas(s, w[int64_t(idx) * a.N], fr[l]);
      }
    cfmas(acc, p < 3 ? T(1) : T(a.sig_phi), s);
  }
  // far field: -j k eta * acc
  cplx<T> out = cmk<T>(T(a.keta) * acc.im, -T(a.keta) * acc.re);
  if (MODE != 2) {  // + C u (pre-corrected near field)
    const cplx<T>* ur = u + int64_t(r) * rows;
    const int* nb = a.nbr + int64_t(m) * a.n_off;
    cplx<T> nf = cmk<T>(0, 0);
    for (int e = a.near_ptr[n]; e < a.near_ptr[n + 1]; ++e) {
      const int c = a.near_col[e];
      const int o = c / a.N, np_ = c - o * a.N;
      const int mm = nb[o];
      if (mm >= 0) cfma(nf, near_val[e], ur[int64_t(mm) * a.N + np_]);
    }
    out = cadd(out, nf);
  }
  if (MODE == 0) {  // y = D x - G u
    const cplx<T>* xr = x + int64_t(r) * rows + int64_t(m) * a.N;
    cplx<T> dx = cmk<T>(0, 0);
    for (int e = a.d_ptr[n]; e < a.d_ptr[n + 1]; ++e) cfma(dx, d_val[e], xr[a.d_col[e]]);
    out = csub(dx, out);
  }
  y[gid] = out;
}

// ---- section III: block-diagonal macromodel product, grouped complex GEMM --------
// U[:, c] = M_t X[:, c] for every column c = r * n_elem + m of an element of kind t.
template <typename T>
__global__ void __launch_bounds__(256) k_macro_gemm(const cplx<T>* __restrict__ M, const cplx<T>* __restrict__ X,
                                                    cplx<T>* __restrict__ U, GemmArgs a) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ cplx<T> As[TK][TM];
  __shared__ cplx<T> Bs[TK][TN + 1];
  __shared__ int cols[TN];
  // which kind and which column tile
  int t = 0, tile = blockIdx.x;
  while (t + 1 < a.n_types && tile >= a.tile_start[t + 1]) ++t;
  tile -= a.tile_start[t];
  const int ncols = a.R * a.type_count[t];
  const int c0 = tile * TN;
  const int i0 = blockIdx.y * TM;
  const int N = a.N;
  const cplx<T>* Mt = M + int64_t(t) * N * N;
  if (threadIdx.x < TN) {
    const int c = c0 + threadIdx.x;
    cols[threadIdx.x] = c < ncols ? a.col_list[a.col_start[t] + c] : -1;
  }
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  cplx<T> acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = cmk<T>(0, 0);
  __syncthreads();
  for (int k0 = 0; k0 < N; k0 += TK) {
    for (int e = threadIdx.x; e < TK * TM; e += 256) {
      const int kk = e / TM, ii = e - kk * TM;
      const int gi = i0 + ii, gk = k0 + kk;
      As[kk][ii] = (gi < N && gk < N) ? Mt[int64_t(gk) * N + gi] : cmk<T>(0, 0);
    }
    for (int e = threadIdx.x; e < TK * TN; e += 256) {
      const int jj = e / TK, kk = e - jj * TK;
      const int c = cols[jj], gk = k0 + kk;
      Bs[kk][jj] = (c >= 0 && gk < N) ? X[int64_t(c) * N + gk] : cmk<T>(0, 0);
    }
    __syncthreads();
    for (int kk = 0; kk < TK; ++kk) {
      cplx<T> av[4], bv[4];
      for (int i = 0; i < 4; ++i) av[i] = As[kk][tx + 16 * i];
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][ty + 16 * j];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) cfma(acc[i][j], av[i], bv[j]);
    }
    __syncthreads();
  }
  for (int j = 0; j < 4; ++j) {
    const int c = cols[ty + 16 * j];
    if (c < 0) continue;
    for (int i = 0; i < 4; ++i) {
      const int gi = i0 + tx + 16 * i;
      if (gi < N) U[int64_t(c) * N + gi] = acc[i][j];
    }
  }
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
hipError_t launch_project(const cplx<T>* u, cplx<T>* Q, const ProjArgs& a, const T* Wp, hipStream_t s) {
  const int64_t n = int64_t(a.nx) * a.ny * a.nz * a.R;
  hipLaunchKernelGGL(k_project<T>, dim3(blocks_for(n, 256)), dim3(256), 0, s, u, Q, a, Wp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_convolve(const cplx<T>* Q, cplx<T>* Phi, cplx<T>* S, const ConvArgs& a, hipStream_t s,
                           hipEvent_t* ev) {
  const int planes = a.R * 4 * a.nx;
  size_t lds = sizeof(cplx<T>) * size_t(a.Py.L) * (1 + a.nz);
  hipLaunchKernelGGL(k_fft_y_fwd<T>, dim3(planes), dim3(256), lds, s, Q, S, a.ny, a.nz, a.Py,
                     reinterpret_cast<const cplx<T>*>(a.tw_y));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev) (void)hipEventRecord(ev[0], s);
  const int nkb = a.Py.L / a.B;
  lds = sizeof(cplx<T>) * size_t(a.Px.L) * (1 + a.B * a.nz);
  hipLaunchKernelGGL((k_fft_x<T, 0>), dim3(a.R * 4 * nkb), dim3(256), lds, s, S, S, a.nx, a.Py.L, a.nz, a.B,
                     a.Px, reinterpret_cast<const cplx<T>*>(a.tw_x), reinterpret_cast<const cplx<T>*>(a.gt),
                     a.rev_x, a.rev_y);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev) (void)hipEventRecord(ev[1], s);
  lds = sizeof(cplx<T>) * size_t(a.Py.L) * (1 + a.nz);
  hipLaunchKernelGGL(k_fft_y_inv<T>, dim3(planes), dim3(256), lds, s, S, Phi, a.ny, a.nz, a.Py,
                     reinterpret_cast<const cplx<T>*>(a.tw_y));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(int mode, const cplx<T>* Phi, const cplx<T>* u, const cplx<T>* x, cplx<T>* y,
                          const CombineArgs& a, const T* Wt, const cplx<T>* near_val, const cplx<T>* d_val,
                          hipStream_t s) {
  const int64_t n = int64_t(a.ne) * a.N * a.R;
  const dim3 g(blocks_for(n, 256)), b(256);
  if (mode == 0)
    hipLaunchKernelGGL((k_interp_combine<T, 0>), g, b, 0, s, Phi, u, x, y, a, Wt, near_val, d_val);
  else if (mode == 1)
    hipLaunchKernelGGL((k_interp_combine<T, 1>), g, b, 0, s, Phi, u, x, y, a, Wt, near_val, d_val);
  else
    hipLaunchKernelGGL((k_interp_combine<T, 2>), g, b, 0, s, Phi, u, x, y, a, Wt, near_val, d_val);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_macro(const cplx<T>* M, const cplx<T>* X, cplx<T>* U, const GemmArgs& a, hipStream_t s) {
  const int tiles = a.tile_start[a.n_types];  // host copy of the tile prefix sums
  if (tiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_macro_gemm<T>, dim3(tiles, (a.N + 63) / 64), dim3(256), 0, s, M, X, U, a);
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

hipError_t configure_lds(size_t bytes) {
  const int b = int(bytes);
  hipError_t e = hipSuccess, t;
#define AIM_ATTR(f)                                                                   \
  t = hipFuncSetAttribute(reinterpret_cast<const void*>(f), hipFuncAttributeMaxDynamicSharedMemorySize, b); \
  if (t != hipSuccess) e = t;
  AIM_ATTR(k_fft_y_fwd<float>)
  AIM_ATTR(k_fft_y_fwd<double>)
  AIM_ATTR(k_fft_y_inv<float>)
  AIM_ATTR(k_fft_y_inv<double>)
  AIM_ATTR((k_fft_x<float, 0>))
  AIM_ATTR((k_fft_x<double, 0>))
  AIM_ATTR((k_fft_x<double, 1>))
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
template hipError_t launch_combine<float>(int, const cplx<float>*, const cplx<float>*, const cplx<float>*, cplx<float>*,
                                          const CombineArgs&, const float*, const cplx<float>*, const cplx<float>*,
                                          hipStream_t);
template hipError_t launch_combine<double>(int, const cplx<double>*, const cplx<double>*, const cplx<double>*,
                                           cplx<double>*, const CombineArgs&, const double*, const cplx<double>*,
                                           const cplx<double>*, hipStream_t);
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
