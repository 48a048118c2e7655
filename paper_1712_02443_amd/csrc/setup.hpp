// Host-side construction of the AIM operator for one array (section V): stencils,
// projection weights, near-field pattern and pre-corrected near-field values.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace aimm {

using cd = std::complex<double>;

struct SurfaceIn {
  int n_vert = 0, n_tri = 0, n_rwg = 0;
  const double* vert = nullptr;
  const int32_t* tri = nullptr;
  const int32_t* rwg = nullptr;
};

struct ArrayIn {
  double k = 0, eta = 0, h = 0, r_near = 0;
  int order = 2;
  int px = 0, py = 0, pitch = 0, n_types = 0;
  const int32_t* elem_type = nullptr;
  int max_rhs = 1;
};

// Everything the device path needs that depends only on the surface and the lattice.
struct Setup {
  int N = 0;          // RWG functions per surface
  int q = 0, q3 = 0;  // stencil nodes per axis and per stencil
  int ex = 0, ey = 0, ez = 0;        // extent of one element's stencils (nodes)
  int nx = 0, ny = 0, nz = 0;        // unpadded grid
  std::vector<int32_t> sloc;         // [N][3] stencil origin relative to the element's extent box
  std::vector<double> W;             // [4][N][q3] projection weights, psi = x, y, z, phi
  std::vector<int32_t> offsets;      // [n_off][2] lattice offsets (dx, dy) carrying near pairs
  std::vector<int32_t> near_ptr;     // [N + 1] CSR rows of the pre-corrected near field
  std::vector<int32_t> near_col;     // packed (o << 16) | n'
  std::vector<cd> near_val;          // pre-corrected values C = G_exact - G_grid
  // near field regrouped for the matrix cores: rows clustered in groups of kNearGroup, each group
  // with the union of its columns (padded to a multiple of 4) and a dense coefficient
  // block A[k][i] = C[group row i][union column k]
  std::vector<int32_t> grp_ptr;      // [n_groups + 1] offsets into grp_col / grp_A (in columns)
  std::vector<int32_t> grp_col;      // packed n' | (dx + 8) << 16 | (dy + 8) << 24
  std::vector<cd> grp_A;             // [total columns][kNearGroup]
  std::vector<int32_t> grp_row;      // [n_groups][kNearGroup] row n of each group slot (-1: none)
  std::vector<int32_t> slot_of;      // [N] group slot of row n (the near-field output is slot-ordered)
  int grp_max_cols = 0;              // largest padded column count of a group
  std::vector<int32_t> node_ptr;     // [ex*ey*ez + 1] projection gather table by local node
  std::vector<int32_t> node_ent;     // packed n * q3 + p
  std::vector<int32_t> node_n;       // n of the same entries
  std::vector<double> cent;          // [N][3] RWG edge midpoints (element-local)
};

constexpr int kNearGroup = 16;
// group column counts are padded to a multiple of this: four K quarters of whole 16-column prefetch batches
constexpr int kNearColAlign = 64;
constexpr int kNearColTail = 32;   // zero columns after the last group (one prefetch batch)

// Throws std::invalid_argument with a message on bad input.
void validate(const SurfaceIn& s, const ArrayIn& a);
void build_setup(const SurfaceIn& s, const ArrayIn& a, Setup& out);

// Element-local part of the plane-wave excitation (eq. V1): for each RWG n,
// loc[n] = -sum_T sum_q A w_q (Lambda_n(r_q) . e) exp(-j k kinc . r_q).
void plane_wave_local(const SurfaceIn& s, double k, double theta, double phi, int pol,
                      std::vector<cd>& loc, double kinc[3]);

// Quadrature of the radiation integral F_n(r^) = int Lambda_n(r) exp(j k r^ . r) dS
// (element-local r): per RWG n, 14 points (7 per triangle, T+ then T-) as
// (x, y, z, c_x, c_y, c_z) with c = weight * area * Lambda_n(point).
void far_quadrature(const SurfaceIn& s, std::vector<double>& q);

// Smallest length >= n whose prime factors are 2, 3 and 5 only.
int smooth_length(int n);
// Radix factorisation (4, 2, 3, 5 preferred in that order); empty if not 5-smooth.
std::vector<int> radix_plan(int L);

}  // namespace aimm
