// Host construction of the AIM operator (section V) for one array.
//
// Stencils: one per RWG function, anchored at the edge midpoint c, origin
// s = floor(c / h - N_O / 2 + 1/2 + 1e-9) per axis, (N_O + 1)^3 nodes.
// Projection weights (step (i)): W_psi[n][p] = int f_psi(r) l_i(x) l_j(y) l_l(z) dS
// over the two triangles of RWG n, f = Lambda . x_hat, Lambda . y_hat, Lambda . z_hat,
// div Lambda; l = Lagrange polynomials of order N_O on the stencil nodes; 7-point
// degree-5 triangle rule.  Interpolation (step (iii)) is the transpose.
// Near field: pairs with |c_a - c_b| <= r_near or overlapping stencils keep the
// exact Galerkin entry of eq. Gouter1, through the pre-correction
// C_ab = G_exact_ab - G_grid_ab.  Exact entries use the same 7-point rule on both
// triangles with the static 1/(4 pi R) part of the kernel integrated in closed form
// over the source triangle (Wilton et al. 1984; Graglia 1993).
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <thread>

namespace aimm {
namespace {

struct V3 {
  double x = 0, y = 0, z = 0;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

struct CV3 {
  cd x, y, z;
};

constexpr double kPi = 3.14159265358979323846;

// Radon's 7-point rule, weights normalised to sum 1 (integral = area * sum w f).
struct Rule7 {
  double b[7][3];
  double w[7];
  Rule7() {
    const double s15 = std::sqrt(15.0);
    const double a1 = (9.0 - 2.0 * s15) / 21.0, b1 = (6.0 + s15) / 21.0;
    const double a2 = (9.0 + 2.0 * s15) / 21.0, b2 = (6.0 - s15) / 21.0;
    const double w0 = 9.0 / 40.0, w1 = (155.0 + s15) / 1200.0, w2 = (155.0 - s15) / 1200.0;
    const double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a1, b1, b1}, {b1, a1, b1}, {b1, b1, a1},
                              {a2, b2, b2},             {b2, a2, b2}, {b2, b2, a2}};
    const double ws[7] = {w0, w1, w1, w1, w2, w2, w2};
    for (int q = 0; q < 7; ++q) {
      for (int i = 0; i < 3; ++i) b[q][i] = pts[q][i];
      w[q] = ws[q];
    }
  }
};
const Rule7 R7;

struct Tri {
  V3 v[3];
  double area;
  V3 nrm;
  V3 pts[7];
};

Tri make_tri(V3 a, V3 b, V3 c) {
  Tri t;
  t.v[0] = a;
  t.v[1] = b;
  t.v[2] = c;
  V3 cr = cross(b - a, c - a);
  double n2 = norm(cr);
  t.area = 0.5 * n2;
  t.nrm = (1.0 / n2) * cr;
  for (int q = 0; q < 7; ++q)
    t.pts[q] = R7.b[q][0] * a + R7.b[q][1] * b + R7.b[q][2] * c;
  return t;
}

Tri shifted(const Tri& t, V3 s) {
  Tri o = t;
  for (int i = 0; i < 3; ++i) o.v[i] = t.v[i] + s;
  for (int q = 0; q < 7; ++q) o.pts[q] = t.pts[q] + s;
  return o;
}

// Closed-form int_T 1/R dS' (I1) and int_T (r' - rho)/R dS' (Iv), rho = projection of r.
void static_pot(const V3& r, const Tri& t, double& I1, V3& Iv) {
  const double d = dot(r - t.v[0], t.nrm);
  const V3 rho = r - d * t.nrm;
  const double ad = std::fabs(d);
  I1 = 0.0;
  Iv = V3{};
  for (int i = 0; i < 3; ++i) {
    const V3 va = t.v[i], vb = t.v[(i + 1) % 3];
    const V3 e = vb - va;
    const double le = norm(e);
    const V3 lh = (1.0 / le) * e;
    const V3 uh = cross(lh, t.nrm);
    const double sm = dot(va - rho, lh);
    const double sp = dot(vb - rho, lh);
    const double t0 = dot(va - rho, uh);
    const double r0sq = t0 * t0 + d * d;
    const double rp = std::sqrt(r0sq + sp * sp);
    const double rm = std::sqrt(r0sq + sm * sm);
    const double r0 = std::sqrt(r0sq);
    double f = 0.0;
    if (r0 > 1e-14 * le) f = std::asinh(sp / r0) - std::asinh(sm / r0);
    const double beta = std::atan2(t0 * sp, r0sq + ad * rp) - std::atan2(t0 * sm, r0sq + ad * rm);
    I1 += t0 * f - ad * beta;
    const double c = 0.5 * (r0sq * f + sp * rp - sm * rm);
    Iv = Iv + c * uh;
  }
}

// (exp(-jkR) - 1) / (4 pi R) with its R -> 0 limit.
inline cd smooth_g(double R, double k) {
  if (!(R > 0.0)) return cd(0.0, -k / (4.0 * kPi));
  const double s = std::sin(0.5 * k * R);
  return cd(-2.0 * s * s, -std::sin(k * R)) / (4.0 * kPi * R);
}

// Moments over the test triangle's rule of K0 = int_Tb G and K1 = int_Tb G r':
// m0 = sum w K0, m1 = sum w K1, m2 = sum w r K0, m3 = sum w r . K1.
void pair_moments(const Tri& ta, const Tri& tb, double k, cd& m0, CV3& m1, CV3& m2, cd& m3) {
  m0 = 0.0;
  m3 = 0.0;
  m1 = CV3{};
  m2 = CV3{};
  for (int q = 0; q < 7; ++q) {
    const V3 r = ta.pts[q];
    cd K0 = 0.0;
    CV3 K1{};
    for (int s = 0; s < 7; ++s) {
      const V3 rs = tb.pts[s];
      const double R = norm(r - rs);
      const cd g = smooth_g(R, k) * (R7.w[s] * tb.area);
      K0 += g;
      K1.x += g * rs.x;
      K1.y += g * rs.y;
      K1.z += g * rs.z;
    }
    double I1;
    V3 Iv;
    static_pot(r, tb, I1, Iv);
    const double d = dot(r - tb.v[0], tb.nrm);
    const V3 rho = r - d * tb.nrm;
    const double c = 1.0 / (4.0 * kPi);
    K0 += c * I1;
    K1.x += c * (Iv.x + rho.x * I1);
    K1.y += c * (Iv.y + rho.y * I1);
    K1.z += c * (Iv.z + rho.z * I1);
    const double w = R7.w[q];
    m0 += w * K0;
    m1.x += w * K1.x;
    m1.y += w * K1.y;
    m1.z += w * K1.z;
    m2.x += w * r.x * K0;
    m2.y += w * r.y * K0;
    m2.z += w * r.z * K0;
    m3 += w * (r.x * K1.x + r.y * K1.y + r.z * K1.z);
  }
}

struct Rwg {
  int tp, tm;
  V3 pp, pm, c;
  double len;
};

struct Mesh {
  std::vector<Tri> tri;
  std::vector<Rwg> rwg;
};

Mesh make_mesh(const SurfaceIn& s) {
  Mesh m;
  auto vert = [&](int i) { return V3{s.vert[3 * i], s.vert[3 * i + 1], s.vert[3 * i + 2]}; };
  m.tri.reserve(s.n_tri);
  for (int t = 0; t < s.n_tri; ++t)
    m.tri.push_back(make_tri(vert(s.tri[3 * t]), vert(s.tri[3 * t + 1]), vert(s.tri[3 * t + 2])));
  m.rwg.resize(s.n_rwg);
  for (int n = 0; n < s.n_rwg; ++n) {
    const int va = s.rwg[4 * n], vb = s.rwg[4 * n + 1], tp = s.rwg[4 * n + 2], tm = s.rwg[4 * n + 3];
    auto free_v = [&](int t) {
      for (int i = 0; i < 3; ++i) {
        const int v = s.tri[3 * t + i];
        if (v != va && v != vb) return vert(v);
      }
      throw std::invalid_argument("RWG triangle does not contain its edge");
    };
    Rwg& r = m.rwg[n];
    r.tp = tp;
    r.tm = tm;
    r.pp = free_v(tp);
    r.pm = free_v(tm);
    r.len = norm(vert(vb) - vert(va));
    r.c = 0.5 * (vert(va) + vert(vb));
  }
  return m;
}

// Exact Galerkin entry G_ab of eq. Gouter1: test RWG a at the origin, source RWG b
// translated by sb.
cd efie_entry(const Mesh& M, int a, int b, V3 sb, double k, double eta) {
  const Rwg& A = M.rwg[a];
  const Rwg& B = M.rwg[b];
  cd acc = 0.0;
  for (int ia = 0; ia < 2; ++ia) {
    const Tri& ta = M.tri[ia == 0 ? A.tp : A.tm];
    const V3 pa = ia == 0 ? A.pp : A.pm;
    const double sga = ia == 0 ? 1.0 : -1.0;
    for (int ib = 0; ib < 2; ++ib) {
      const Tri tb = shifted(M.tri[ib == 0 ? B.tp : B.tm], sb);
      const V3 pb = (ib == 0 ? B.pp : B.pm) + sb;
      const double sgb = ib == 0 ? 1.0 : -1.0;
      cd m0, m3;
      CV3 m1, m2;
      pair_moments(ta, tb, k, m0, m1, m2, m3);
      const cd d = m3 - (pb.x * m2.x + pb.y * m2.y + pb.z * m2.z) -
                   (pa.x * m1.x + pa.y * m1.y + pa.z * m1.z) + dot(pa, pb) * m0;
      const double fa = A.len / (2.0 * ta.area), fb = B.len / (2.0 * tb.area);
      const cd vec = ta.area * fa * fb * d;
      const cd sca = ta.area * (A.len / ta.area) * (B.len / tb.area) * m0;
      acc += sga * sgb * (vec - sca / (k * k));
    }
  }
  return cd(0.0, -k * eta) * acc;
}

double lagrange(int i, double t, int order) {
  double v = 1.0;
  for (int m = 0; m <= order; ++m)
    if (m != i) v *= (t - m) / double(i - m);
  return v;
}

}  // namespace

int smooth_length(int n) {
  for (int m = std::max(n, 1);; ++m) {
    int r = m;
    for (int p : {2, 3, 5})
      while (r % p == 0) r /= p;
    if (r == 1) return m;
  }
}

std::vector<int> radix_plan(int L) {
  std::vector<int> f;
  int r = L;
  while (r % 4 == 0) {
    f.push_back(4);
    r /= 4;
  }
  while (r % 2 == 0) {
    f.push_back(2);
    r /= 2;
  }
  while (r % 3 == 0) {
    f.push_back(3);
    r /= 3;
  }
  while (r % 5 == 0) {
    f.push_back(5);
    r /= 5;
  }
  if (r != 1) return {};
  return f;
}

void validate(const SurfaceIn& s, const ArrayIn& a) {
  auto bad = [](const std::string& m) { throw std::invalid_argument(m); };
  if (!s.vert || !s.tri || !s.rwg) bad("surface arrays must not be NULL");
  if (s.n_vert < 3 || s.n_tri < 2 || s.n_rwg < 1) bad("surface needs >= 3 vertices, >= 2 triangles, >= 1 RWG");
  if (s.n_rwg > 65535) bad("at most 65535 RWG functions per surface");
  for (int t = 0; t < 3 * s.n_tri; ++t)
    if (s.tri[t] < 0 || s.tri[t] >= s.n_vert) bad("triangle vertex index out of range");
  for (int n = 0; n < s.n_rwg; ++n) {
    for (int i = 0; i < 2; ++i)
      if (s.rwg[4 * n + i] < 0 || s.rwg[4 * n + i] >= s.n_vert) bad("RWG vertex index out of range");
    for (int i = 2; i < 4; ++i)
      if (s.rwg[4 * n + i] < 0 || s.rwg[4 * n + i] >= s.n_tri) bad("RWG triangle index out of range");
    if (s.rwg[4 * n + 2] == s.rwg[4 * n + 3]) bad("RWG with T+ == T-");
  }
  if (!(a.k > 0) || !(a.eta > 0) || !(a.h > 0) || !(a.r_near >= 0)) bad("k, eta, h must be > 0 and r_near >= 0");
  if (a.order < 1 || a.order > 3) bad("order must be 1, 2 or 3");
  if (a.px < 1 || a.py < 1 || a.pitch < 1) bad("px, py, pitch_cells must be >= 1");
  if (a.n_types < 1 || !a.elem_type) bad("n_types >= 1 and elem_type required");
  for (int m = 0; m < a.px * a.py; ++m)
    if (a.elem_type[m] < 0 || a.elem_type[m] >= a.n_types) bad("elem_type out of range");
  if (a.max_rhs < 1 || a.max_rhs > 4096) bad("max_rhs must be in [1, 4096]");
  if (int64_t(a.px) * a.py * s.n_rwg * a.max_rhs > (int64_t(1) << 31) - 1) bad("problem exceeds 2^31 unknowns x rhs");
}

void build_setup(const SurfaceIn& s, const ArrayIn& a, Setup& out) {
  validate(s, a);
  const Mesh M = make_mesh(s);
  const int N = s.n_rwg, q = a.order + 1, q3 = q * q * q;
  out.N = N;
  out.q = q;
  out.q3 = q3;
  // stencil origins
  std::vector<int> sg(3 * N);
  int smin[3] = {1 << 30, 1 << 30, 1 << 30}, smax[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
  out.cent.resize(3 * N);
  for (int n = 0; n < N; ++n) {
    const double c[3] = {M.rwg[n].c.x, M.rwg[n].c.y, M.rwg[n].c.z};
    for (int ax = 0; ax < 3; ++ax) {
      out.cent[3 * n + ax] = c[ax];
      const int v = int(std::floor(c[ax] / a.h - 0.5 * a.order + 0.5 + 1e-9));
      sg[3 * n + ax] = v;
      smin[ax] = std::min(smin[ax], v);
      smax[ax] = std::max(smax[ax], v);
    }
  }
  out.ex = smax[0] - smin[0] + q;
  out.ey = smax[1] - smin[1] + q;
  out.ez = smax[2] - smin[2] + q;
  out.nx = a.pitch * (a.px - 1) + out.ex;
  out.ny = a.pitch * (a.py - 1) + out.ey;
  out.nz = out.ez;
  out.sloc.resize(3 * N);
  for (int n = 0; n < N; ++n)
    for (int ax = 0; ax < 3; ++ax) out.sloc[3 * n + ax] = sg[3 * n + ax] - smin[ax];

  // projection weights
  out.W.assign(size_t(4) * N * q3, 0.0);
  for (int n = 0; n < N; ++n) {
    const Rwg& R = M.rwg[n];
    for (int side = 0; side < 2; ++side) {
      const Tri& t = M.tri[side == 0 ? R.tp : R.tm];
      const V3 p = side == 0 ? R.pp : R.pm;
      const double sgn = side == 0 ? 1.0 : -1.0;
      const double f = sgn * R.len / (2.0 * t.area);
      const double dv = sgn * R.len / t.area;
      for (int qq = 0; qq < 7; ++qq) {
        const V3 r = t.pts[qq];
        const double wq = t.area * R7.w[qq];
        const V3 lam = f * (r - p);
        const double tx = r.x / a.h - sg[3 * n], ty = r.y / a.h - sg[3 * n + 1], tz = r.z / a.h - sg[3 * n + 2];
        double lx[4], ly[4], lz[4];
        for (int i = 0; i < q; ++i) {
          lx[i] = lagrange(i, tx, a.order);
          ly[i] = lagrange(i, ty, a.order);
          lz[i] = lagrange(i, tz, a.order);
        }
        const double fv[4] = {lam.x, lam.y, lam.z, dv};
        for (int i = 0; i < q; ++i)
          for (int j = 0; j < q; ++j)
            for (int l = 0; l < q; ++l) {
              const double b = lx[i] * ly[j] * lz[l] * wq;
              const int pidx = (i * q + j) * q + l;
              for (int psi = 0; psi < 4; ++psi) out.W[(size_t(psi) * N + n) * q3 + pidx] += fv[psi] * b;
            }
      }
    }
  }

  // projection gather table: local node -> (basis, stencil point)
  const int nloc = out.ex * out.ey * out.ez;
  std::vector<int> cnt(nloc + 1, 0);
  auto node_of = [&](int n, int p) {
    const int i = p / (q * q), j = (p / q) % q, l = p % q;
    return ((out.sloc[3 * n] + i) * out.ey + (out.sloc[3 * n + 1] + j)) * out.ez + (out.sloc[3 * n + 2] + l);
  };
  for (int n = 0; n < N; ++n)
    for (int p = 0; p < q3; ++p) cnt[node_of(n, p) + 1]++;
  out.node_ptr.assign(nloc + 1, 0);
  for (int i = 0; i < nloc; ++i) out.node_ptr[i + 1] = out.node_ptr[i] + cnt[i + 1];
  out.node_ent.assign(size_t(N) * q3, 0);
  out.node_n.assign(size_t(N) * q3, 0);
  std::vector<int> fill(out.node_ptr.begin(), out.node_ptr.end() - 1);
  for (int n = 0; n < N; ++n)
    for (int p = 0; p < q3; ++p) {
      const int at = fill[node_of(n, p)]++;
      out.node_ent[at] = n * q3 + p;
      out.node_n[at] = n;
    }

  // grid Green's function on the separations near pairs can reach
  const double k = a.k, eta = a.eta, h = a.h;
  const int R = std::max(out.ex, out.ey) + 4 * a.pitch + q;  // generous bound for 3 lattice steps
  const int DZ = out.ez + q;
  auto gidx = [&](int dx, int dy, int dz) { return (size_t(dx + R) * (2 * R + 1) + (dy + R)) * (2 * DZ + 1) + (dz + DZ); };
  std::vector<cd> Gt(size_t(2 * R + 1) * (2 * R + 1) * (2 * DZ + 1));
  for (int dx = -R; dx <= R; ++dx)
    for (int dy = -R; dy <= R; ++dy)
      for (int dz = -DZ; dz <= DZ; ++dz) {
        const double r = h * std::sqrt(double(dx * dx + dy * dy + dz * dz));
        Gt[gidx(dx, dy, dz)] = r > 0 ? std::exp(cd(0.0, -k * r)) / (4.0 * kPi * r) : cd(0.0);
      }

  // near field, one block per lattice offset (translation invariance)
  const int reach = 3;
  struct Ent {
    int o, col;
    cd v;
  };
  std::vector<std::vector<Ent>> rows(N);
  std::vector<std::array<int, 2>> offs;
  for (int dy = -std::min(reach, a.py - 1); dy <= std::min(reach, a.py - 1); ++dy)
    for (int dx = -std::min(reach, a.px - 1); dx <= std::min(reach, a.px - 1); ++dx) offs.push_back({dx, dy});
  const double sig[4] = {1.0, 1.0, 1.0, -1.0 / (k * k)};
  std::vector<std::vector<std::vector<Ent>>> per_off(offs.size(), std::vector<std::vector<Ent>>(N));
  std::atomic<int> next{0};
  const int total = int(offs.size()) * N;
  auto worker = [&]() {
    std::vector<cd> T(size_t(4) * q3);
    for (;;) {
      const int job = next.fetch_add(1);
      if (job >= total) break;
      const int oi = job / N, na = job % N;
      const int dx = offs[oi][0], dy = offs[oi][1];
      const V3 sb{double(dx * a.pitch) * h, double(dy * a.pitch) * h, 0.0};
      const int gsh[3] = {dx * a.pitch, dy * a.pitch, 0};
      const V3 ca = M.rwg[na].c;
      for (int nb = 0; nb < N; ++nb) {
        const V3 cb = M.rwg[nb].c + sb;
        const V3 dd = ca - cb;
        bool near = std::sqrt(dot(dd, dd)) <= a.r_near + 1e-12;
        int dg[3];
        bool ovl = true;
        for (int ax = 0; ax < 3; ++ax) {
          dg[ax] = sg[3 * na + ax] - (sg[3 * nb + ax] + gsh[ax]);
          if (std::abs(dg[ax]) > a.order) ovl = false;
        }
        if (!(near || ovl)) continue;
        if (std::abs(dg[0]) + q > R || std::abs(dg[1]) + q > R || std::abs(dg[2]) + q > DZ)
          throw std::runtime_error("near pair beyond the precomputed separation table");
        const cd ex = efie_entry(M, na, nb, sb, k, eta);
        // grid approximation of the same entry
        cd gg = 0.0;
        for (int psi = 0; psi < 4; ++psi) {
          const double* wa = &out.W[(size_t(psi) * N + na) * q3];
          const double* wb = &out.W[(size_t(psi) * N + nb) * q3];
          cd acc = 0.0;
          for (int p = 0; p < q3; ++p) {
            if (wa[p] == 0.0) continue;
            const int i = p / (q * q), j = (p / q) % q, l = p % q;
            cd inner = 0.0;
            for (int pp = 0; pp < q3; ++pp) {
              const int ii = pp / (q * q), jj = (pp / q) % q, ll = pp % q;
              inner += Gt[gidx(dg[0] + i - ii, dg[1] + j - jj, dg[2] + l - ll)] * wb[pp];
            }
            acc += wa[p] * inner;
          }
          gg += sig[psi] * acc;
        }
        gg *= cd(0.0, -k * eta);
        per_off[oi][na].push_back({oi, nb, ex - gg});
      }
    }
  };
  unsigned nth = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  std::exception_ptr err;
  std::mutex emu;
  for (unsigned t = 0; t < nth; ++t)
    th.emplace_back([&]() {
      try {
        worker();
      } catch (...) {
        std::lock_guard<std::mutex> g(emu);
        err = std::current_exception();
        next = total;
      }
    });
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
  // keep offsets with pairs; the outermost searched ring must be empty
  std::vector<int> remap(offs.size(), -1);
  for (size_t oi = 0; oi < offs.size(); ++oi) {
    bool any = false;
    for (int n = 0; n < N && !any; ++n) any = !per_off[oi][n].empty();
    if (!any) continue;
    if (std::max(std::abs(offs[oi][0]), std::abs(offs[oi][1])) >= reach)
      throw std::invalid_argument("near field reaches 3 lattice steps; pitch too small for r_near");
    remap[oi] = int(out.offsets.size() / 2);
    out.offsets.push_back(offs[oi][0]);
    out.offsets.push_back(offs[oi][1]);
  }
  out.near_ptr.assign(N + 1, 0);
  for (int n = 0; n < N; ++n) {
    for (size_t oi = 0; oi < offs.size(); ++oi) {
      if (remap[oi] < 0) continue;
      for (const Ent& e : per_off[oi][n]) {
        out.near_col.push_back((remap[oi] << 16) | e.col);
        out.near_val.push_back(e.v);
      }
    }
    out.near_ptr[n + 1] = int32_t(out.near_col.size());
  }
  // Row groups for the matrix-core near field.  Every group's coefficient block is
  // dense over the union of its rows' columns, so rows are clustered greedily: a
  // group starts at the unassigned row with the smallest edge midpoint (x, then y,
  // then z) and repeatedly takes the unassigned row that adds the fewest new columns
  // (lowest index on ties).
  const int ng = (N + kNearGroup - 1) / kNearGroup;
  int max_col = 0;
  for (int32_t c : out.near_col) max_col = std::max(max_col, int(c >> 16) * 65536 + (c & 0xFFFF));
  std::vector<char> in_union(size_t(max_col) + 1, 0), taken(N, 0);
  out.grp_row.assign(size_t(ng) * kNearGroup, -1);
  for (int g = 0; g < ng; ++g) {
    std::vector<int32_t> ucols;
    auto add_row = [&](int n, int slot) {
      taken[n] = 1;
      out.grp_row[size_t(g) * kNearGroup + slot] = n;
      for (int e = out.near_ptr[n]; e < out.near_ptr[n + 1]; ++e) {
        const int32_t c = out.near_col[e];
        const size_t key = size_t(c >> 16) * 65536 + (c & 0xFFFF);
        if (!in_union[key]) {
          in_union[key] = 1;
          ucols.push_back(c);
        }
      }
    };
    int seed = -1;
    for (int n = 0; n < N; ++n) {
      if (taken[n]) continue;
      if (seed < 0) {
        seed = n;
        continue;
      }
      const double* cn = &out.cent[3 * n];
      const double* cs = &out.cent[3 * seed];
      if (cn[0] < cs[0] || (cn[0] == cs[0] && (cn[1] < cs[1] || (cn[1] == cs[1] && cn[2] < cs[2])))) seed = n;
    }
    if (seed < 0) break;
    add_row(seed, 0);
    for (int slot = 1; slot < kNearGroup; ++slot) {
      int best = -1, best_new = 0;
      for (int n = 0; n < N; ++n) {
        if (taken[n]) continue;
        int added = 0;
        for (int e = out.near_ptr[n]; e < out.near_ptr[n + 1]; ++e) {
          const int32_t c = out.near_col[e];
          added += !in_union[size_t(c >> 16) * 65536 + (c & 0xFFFF)];
        }
        if (best < 0 || added < best_new) {
          best = n;
          best_new = added;
        }
      }
      if (best < 0) break;
      add_row(best, slot);
    }
    for (int32_t c : ucols) in_union[size_t(c >> 16) * 65536 + (c & 0xFFFF)] = 0;
  }
  out.slot_of.assign(N, -1);
  for (int t = 0; t < ng * kNearGroup; ++t)
    if (out.grp_row[t] >= 0) out.slot_of[out.grp_row[t]] = t;
  out.grp_ptr.assign(ng + 1, 0);
  out.grp_col.clear();
  out.grp_A.clear();
  out.grp_max_cols = 0;
  for (int g = 0; g < ng; ++g) {
    std::map<int32_t, int> col_index;
    for (int i = 0; i < kNearGroup; ++i) {
      const int n = out.grp_row[size_t(g) * kNearGroup + i];
      if (n < 0) continue;
      for (int e = out.near_ptr[n]; e < out.near_ptr[n + 1]; ++e) col_index.emplace(out.near_col[e], 0);
    }
    int k = 0;
    for (auto& kv : col_index) kv.second = k++;
    // a multiple of two K halves of whole prefetch batches, so the kernel needs no bounds tests
    const int kpad = (k + kNearColAlign - 1) / kNearColAlign * kNearColAlign;
    const size_t base = out.grp_col.size();
    // device form of a column: n' | (dx + 8) << 16 | (dy + 8) << 24 (lattice offset inline)
    auto dev_col = [&](int32_t c) {
      const int o = c >> 16, np_ = c & 0xFFFF;
      return int32_t(np_ | ((out.offsets[2 * o] + 8) << 16) | ((out.offsets[2 * o + 1] + 8) << 24));
    };
    for (auto& kv : col_index) out.grp_col.push_back(dev_col(kv.first));
    // padding columns repeat a real column with zero coefficients
    for (int p = k; p < kpad; ++p) out.grp_col.push_back(col_index.empty() ? int32_t((8 << 16) | (8 << 24))
                                                                           : dev_col(col_index.begin()->first));
    out.grp_A.resize(out.grp_col.size() * kNearGroup, cd(0.0));
    for (int i = 0; i < kNearGroup; ++i) {
      const int n = out.grp_row[size_t(g) * kNearGroup + i];
      if (n < 0) continue;
      for (int e = out.near_ptr[n]; e < out.near_ptr[n + 1]; ++e)
        out.grp_A[(base + col_index[out.near_col[e]]) * kNearGroup + i] = out.near_val[e];
    }
    out.grp_ptr[g + 1] = int32_t(out.grp_col.size());
    out.grp_max_cols = std::max(out.grp_max_cols, kpad);
  }
  // one more batch of zero columns after the last group: the final prefetch reads it
  const int32_t self_col = int32_t((8 << 16) | (8 << 24));
  for (int p = 0; p < kNearColTail; ++p) out.grp_col.push_back(self_col);
  out.grp_A.resize(out.grp_col.size() * kNearGroup, cd(0.0));
}

void far_quadrature(const SurfaceIn& s, std::vector<double>& q) {
  const Mesh M = make_mesh(s);
  q.assign(size_t(s.n_rwg) * 14 * 6, 0.0);
  for (int n = 0; n < s.n_rwg; ++n) {
    const Rwg& R = M.rwg[n];
    for (int side = 0; side < 2; ++side) {
      const Tri& t = M.tri[side == 0 ? R.tp : R.tm];
      const V3 p = side == 0 ? R.pp : R.pm;
      const double f = (side == 0 ? 1.0 : -1.0) * R.len / (2.0 * t.area);
      for (int k = 0; k < 7; ++k) {
        const V3 r = t.pts[k];
        const V3 c = (f * R7.w[k] * t.area) * (r - p);
        double* o = &q[(size_t(n) * 14 + side * 7 + k) * 6];
        o[0] = r.x;
        o[1] = r.y;
        o[2] = r.z;
        o[3] = c.x;
        o[4] = c.y;
        o[5] = c.z;
      }
    }
  }
}

void plane_wave_local(const SurfaceIn& s, double k, double theta, double phi, int pol,
                      std::vector<cd>& loc, double kinc[3]) {
  const Mesh M = make_mesh(s);
  const double st = std::sin(theta), ct = std::cos(theta), sp = std::sin(phi), cp = std::cos(phi);
  kinc[0] = -st * cp;
  kinc[1] = -st * sp;
  kinc[2] = -ct;
  const V3 kv{kinc[0], kinc[1], kinc[2]};
  const V3 e = pol == 0 ? V3{ct * cp, ct * sp, -st} : V3{-sp, cp, 0.0};
  loc.assign(s.n_rwg, cd(0.0));
  for (int n = 0; n < s.n_rwg; ++n) {
    const Rwg& R = M.rwg[n];
    cd acc = 0.0;
    for (int side = 0; side < 2; ++side) {
      const Tri& t = M.tri[side == 0 ? R.tp : R.tm];
      const V3 p = side == 0 ? R.pp : R.pm;
      const double f = (side == 0 ? 1.0 : -1.0) * R.len / (2.0 * t.area);
      for (int qq = 0; qq < 7; ++qq) {
        const V3 r = t.pts[qq];
        acc += t.area * R7.w[qq] * f * dot(r - p, e) * std::exp(cd(0.0, -k * dot(kv, r)));
      }
    }
    loc[n] = -acc;
  }
}

}  // namespace aimm
