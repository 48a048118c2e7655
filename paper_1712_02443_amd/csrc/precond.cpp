// Block-Jacobi preconditioner of the final system (section IV eq. finalsystem).
//
// The diagonal block of the operator D - G T A^-1 B for element m is
//     A_mm = D - G_mm M_t(m),
// where G_mm is the AIM operator of section V restricted to the RWG functions of one
// element.  The grid part of G is translation invariant and the pre-corrected near
// field of lattice offset (0, 0) is the same block for every element, so G_mm is one
// N x N matrix for the whole array, and A_mm depends only on the kind t(m).  The
// preconditioner is blockdiag(P_t(m)) with P_t = (D - G_self M_t)^-1, one inverse per
// distinct element, the same reuse that section III makes of T A^-1 B.  The paper
// preconditions its solves with an incomplete factorisation of the near-field
// matrix (section VI); this block form keeps the per-kind sharing of the method and
// is applied by the same grouped product as the macromodels.
//
// Everything here is host FP64: G_self from the stencil weights and the sampled
// Green's function (the same grid approximation the pre-correction subtracts) plus
// the offset-(0, 0) pre-corrected entries, then a partially pivoted LU.
#include "precond.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace aimm {
namespace {

constexpr double kPi = 3.14159265358979323846;

// f(i) for i in [0, n) over the host threads
template <typename F>
void parallel_for(int n, F&& f) {
  const unsigned nth = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) f(i);
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nth; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

}  // namespace

void self_block(const Setup& st, const ArrayIn& a, std::vector<cd>& G) {
  const int N = st.N, q = st.q, q3 = st.q3;
  const int ex = st.ex, ey = st.ey, ez = st.ez;
  const double k = a.k, h = a.h;
  // sampled Green's function on every node separation inside one element's box
  const int sx = 2 * ex - 1, sy = 2 * ey - 1, sz = 2 * ez - 1;
  std::vector<cd> Gt(size_t(sx) * sy * sz);
  for (int dx = -(ex - 1); dx < ex; ++dx)
    for (int dy = -(ey - 1); dy < ey; ++dy)
      for (int dz = -(ez - 1); dz < ez; ++dz) {
        const double r = h * std::sqrt(double(dx * dx + dy * dy + dz * dz));
        Gt[(size_t(dx + ex - 1) * sy + (dy + ey - 1)) * sz + (dz + ez - 1)] =
            r > 0 ? std::exp(cd(0.0, -k * r)) / (4.0 * kPi * r) : cd(0.0);
      }
  auto node = [&](int n, int p, int ax) {
    const int c[3] = {p / (q * q), (p / q) % q, p % q};
    return st.sloc[3 * n + ax] + c[ax];
  };
  const double sig[4] = {1.0, 1.0, 1.0, -1.0 / (k * k)};
  const cd scale(0.0, -k * a.eta);
  G.assign(size_t(N) * N, cd(0.0));
  // column nb: the potential of basis nb on the element's box, then its moments
  const size_t box = size_t(ex) * ey * ez;
  parallel_for(N, [&](int nb) {
    std::vector<cd> F(box);
    std::vector<cd> col(N, cd(0.0));
    for (int psi = 0; psi < 4; ++psi) {
      const double* wb = &st.W[(size_t(psi) * N + nb) * q3];
      std::fill(F.begin(), F.end(), cd(0.0));
      for (int pp = 0; pp < q3; ++pp) {
        if (wb[pp] == 0.0) continue;
        const int bx = node(nb, pp, 0), by = node(nb, pp, 1), bz = node(nb, pp, 2);
        for (int x = 0; x < ex; ++x)
          for (int y = 0; y < ey; ++y) {
            const cd* g = &Gt[(size_t(x - bx + ex - 1) * sy + (y - by + ey - 1)) * sz + (ez - 1 - bz)];
            cd* f = &F[(size_t(x) * ey + y) * ez];
            for (int z = 0; z < ez; ++z) f[z] += wb[pp] * g[z];
          }
      }
      for (int na = 0; na < N; ++na) {
        const double* wa = &st.W[(size_t(psi) * N + na) * q3];
        cd acc = 0.0;
        for (int p = 0; p < q3; ++p)
          acc += wa[p] * F[(size_t(node(na, p, 0)) * ey + node(na, p, 1)) * ez + node(na, p, 2)];
        col[na] += sig[psi] * acc;
      }
    }
    for (int na = 0; na < N; ++na) G[size_t(nb) * N + na] = scale * col[na];
  });
  // pre-corrected near field of the element on itself
  int o0 = -1;
  for (size_t o = 0; 2 * o < st.offsets.size(); ++o)
    if (st.offsets[2 * o] == 0 && st.offsets[2 * o + 1] == 0) o0 = int(o);
  if (o0 < 0) return;
  for (int na = 0; na < N; ++na)
    for (int e = st.near_ptr[na]; e < st.near_ptr[na + 1]; ++e)
      if ((st.near_col[e] >> 16) == o0) G[size_t(st.near_col[e] & 0xFFFF) * N + na] += st.near_val[e];
}

void block_inverse(const std::vector<cd>& Gself, const cd* M, const int32_t* drow, const int32_t* dcol,
                   const cd* dval, int64_t dnnz, int N, std::vector<cd>& P) {
  // A = D - G_self M (column-major)
  std::vector<cd> A(size_t(N) * N);
  parallel_for(N, [&](int j) {
    cd* aj = &A[size_t(j) * N];
    std::fill(aj, aj + N, cd(0.0));
    const cd* mj = M + size_t(j) * N;
    for (int l = 0; l < N; ++l) {
      const cd m = mj[l];
      if (m == cd(0.0)) continue;
      const cd* gl = &Gself[size_t(l) * N];
      for (int i = 0; i < N; ++i) aj[i] -= gl[i] * m;
    }
  });
  for (int64_t e = 0; e < dnnz; ++e) A[size_t(dcol[e]) * N + drow[e]] += dval[e];
  // LU with partial pivoting, right-looking; the trailing update runs over columns
  std::vector<int> piv(N);
  for (int c = 0; c < N; ++c) {
    int p = c;
    double best = std::abs(A[size_t(c) * N + c]);
    for (int i = c + 1; i < N; ++i) {
      const double v = std::abs(A[size_t(c) * N + i]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    if (!(best > 0.0)) throw std::runtime_error("the diagonal block D - G_self M_t is singular");
    piv[c] = p;
    if (p != c)
      for (int j = 0; j < N; ++j) std::swap(A[size_t(j) * N + c], A[size_t(j) * N + p]);
    const cd inv = 1.0 / A[size_t(c) * N + c];
    cd* ac = &A[size_t(c) * N];
    for (int i = c + 1; i < N; ++i) ac[i] *= inv;
    const int rest = N - c - 1;
    if (rest == 0) break;
    auto upd = [&](int jj) {
      cd* aj = &A[size_t(c + 1 + jj) * N];
      const cd f = aj[c];
      if (f == cd(0.0)) return;
      for (int i = c + 1; i < N; ++i) aj[i] -= ac[i] * f;
    };
    if (size_t(rest) * rest < 65536) {
      for (int jj = 0; jj < rest; ++jj) upd(jj);
    } else {
      parallel_for(rest, upd);
    }
  }
  // P = A^-1: solve L U P = Pi for each column of the identity
  P.assign(size_t(N) * N, cd(0.0));
  parallel_for(N, [&](int j) {
    std::vector<cd> y(N, cd(0.0));
    y[j] = 1.0;
    for (int c = 0; c < N; ++c)
      if (piv[c] != c) std::swap(y[c], y[piv[c]]);
    for (int c = 0; c < N; ++c) {
      const cd v = y[c];
      if (v == cd(0.0)) continue;
      const cd* ac = &A[size_t(c) * N];
      for (int i = c + 1; i < N; ++i) y[i] -= ac[i] * v;
    }
    for (int c = N - 1; c >= 0; --c) {
      const cd* ac = &A[size_t(c) * N];
      y[c] /= ac[c];
      const cd v = y[c];
      for (int i = 0; i < c; ++i) y[i] -= ac[i] * v;
    }
    std::copy(y.begin(), y.end(), &P[size_t(j) * N]);
  });
}

}  // namespace aimm
