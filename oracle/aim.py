"""The adaptive integral method, step by step (section V).

Readings of points the paper leaves open:
  * grid: uniform spacing h; an element's lattice offset is an exact number of
    cells, so every element-local quantity is shared by identical surfaces;
  * stencil: one per basis function, (N_O + 1) nodes per axis, anchored at the
    RWG edge midpoint c: origin s = floor(c / h - N_O / 2 + 1/2 + 1e-9) per axis
    (the 1e-9 breaks ties on faces that sit on half-integer node positions);
  * projection weights (step (i)): tensor-product Lagrange interpolation of order
    N_O on the stencil, integrated against Lambda . x_hat, Lambda . y_hat,
    Lambda . z_hat and div Lambda with the same 7-point rule as the Galerkin
    entries; interpolation (step (iii)) uses the transposed weights (Galerkin
    testing), so I_psi = P_psi^T;
  * grid kernel (step (ii)): the free-space Green's function sampled at node
    separations, G(d) = exp(-j k h |d|) / (4 pi h |d|), with G(0) = 0 (the value
    never reaches a far pair, see the near rule below); the same kernel serves all
    four potentials, the scalar potential entering with weight -1/k^2 and the
    whole product with -j k eta0;
  * near field: pair (a, b) is near when |c_a - c_b| <= r_near or their stencils
    share a node; near entries are the exact Galerkin values, i.e. the sparse
    pre-correction is C_ab = G_exact_ab - G_grid_ab (section V, near-field
    matrix "with some pre-correction").
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.fft

from .geometry import RwgGeom, seven_point_rule

_BARY, _W = seven_point_rule()


def stencil_origin(center: np.ndarray, h: float, order: int) -> np.ndarray:
    """Integer stencil origin per axis for element-local anchor points (n, 3)."""
    return np.floor(center / h - 0.5 * order + 0.5 + 1e-9).astype(np.int64)


def lagrange(t: np.ndarray, order: int) -> np.ndarray:
    """l_i(t), i = 0..order, the Lagrange basis on nodes 0..order; shape t.shape + (order+1,)."""
    out = np.ones(t.shape + (order + 1,))
    for i in range(order + 1):
        for m in range(order + 1):
            if m != i:
                out[..., i] *= (t - m) / (i - m)
    return out


def projection_weights(geo: RwgGeom, h: float, order: int):
    """Stencil origins s (n, 3) and weights W (4, n, N_O+1, N_O+1, N_O+1) for psi = x, y, z, phi.

    W[psi, a, i, j, l] = sum_{T in a} sum_q A_T w_q f_psi(r_q) l_i(tx) l_j(ty) l_l(tz),
    with t = r_q / h - s_a, f_{x,y,z} = Lambda_a components, f_phi = div Lambda_a.
    """
    s = stencil_origin(geo.center, h, order)
    n = geo.n_rwg
    p = order + 1
    W = np.zeros((4, n, p, p, p))
    for sgn, tidx, free in ((1.0, geo.tp, geo.pp), (-1.0, geo.tm, geo.pm)):
        tv = geo.tri_vert[tidx]                               # (n, 3, 3)
        A = geo.tri_area[tidx]
        rq = np.einsum("qi,nik->nqk", _BARY, tv)              # (n, 7, 3)
        lam = sgn * (geo.length / (2.0 * A))[:, None, None] * (rq - free[:, None, :])
        div = sgn * geo.length / A
        t = rq / h - s[:, None, :]
        lx, ly, lz = (lagrange(t[..., ax], order) for ax in range(3))   # (n, 7, p)
        basis = np.einsum("nqi,nqj,nql->nqijl", lx, ly, lz)
        wq = A[:, None] * _W[None, :]
        for psi in range(3):
            W[psi] += np.einsum("nq,nqijl->nijl", wq * lam[..., psi], basis)
        W[3] += np.einsum("nq,nqijl->nijl", wq * div[:, None], basis)
    return s, W


@dataclass
class Grid:
    """The global AIM grid of one array."""
    shape: tuple            # (Nx, Ny, Nz) nodes
    origin_cell: np.ndarray  # integer node index of global node 0 in element-(0,0) cells
    g: np.ndarray           # (n_elem * n_rwg, 3) global stencil origin of every unknown


def build_grid(s_local: np.ndarray, offsets: np.ndarray, order: int) -> Grid:
    """Place every element's stencils on one grid; offsets (n_elem, 3) in cells."""
    smin = s_local.min(axis=0)
    smax = s_local.max(axis=0)
    ext = smax - smin + order + 1
    shape = tuple(int(offsets[:, a].max() - offsets[:, a].min() + ext[a]) for a in range(3))
    base = offsets.min(axis=0) + smin
    g = (offsets[:, None, :] + s_local[None, :, :] - base).reshape(-1, 3)
    return Grid(shape, base, g)


def green_samples(shape, h: float, k: float, g0: complex = 0.0) -> np.ndarray:
    """G(d) on separations d in [-(N-1), N-1]^3, as an array indexed by d + N - 1."""
    ax = [np.arange(-(n - 1), n) for n in shape]
    dx, dy, dz = np.meshgrid(*ax, indexing="ij")
    r = h * np.sqrt(dx * dx + dy * dy + dz * dz).astype(np.float64)
    rs = np.where(r > 0, r, 1.0)
    G = np.exp(-1j * k * rs) / (4.0 * np.pi * rs)
    return np.where(r > 0, G, g0)


def project(grid: Grid, W: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Step (i): Q_psi[g] = sum_a W_psi[a, g - g_a] u_a.  u (n_unk,), returns (4, Nx, Ny, Nz)."""
    nb = W.shape[1]
    p = W.shape[2]
    Q = np.zeros((4,) + grid.shape, dtype=np.complex128)
    flat = np.zeros((4, int(np.prod(grid.shape))), dtype=np.complex128)
    Ny, Nz = grid.shape[1], grid.shape[2]
    local = np.arange(u.shape[0]) % nb
    for i in range(p):
        for j in range(p):
            for l in range(p):
                node = (grid.g[:, 0] + i) * Ny * Nz + (grid.g[:, 1] + j) * Nz + (grid.g[:, 2] + l)
                for psi in range(4):
                    flat[psi] += np.bincount(node, weights=(W[psi, local, i, j, l] * u).real,
                                             minlength=flat.shape[1])
                    flat[psi] += 1j * np.bincount(node, weights=(W[psi, local, i, j, l] * u).imag,
                                                  minlength=flat.shape[1])
    Q[:] = flat.reshape(Q.shape)
    return Q


def convolve_direct(Q: np.ndarray, Gs: np.ndarray) -> np.ndarray:
    """Step (ii) by definition: Phi[g] = sum_g' G(g - g') Q[g'] (aperiodic); small grids only."""
    shape = Q.shape[1:]
    N = int(np.prod(shape))
    idx = np.stack(np.meshgrid(*[np.arange(n) for n in shape], indexing="ij"), -1).reshape(N, 3)
    off = np.array([n - 1 for n in shape])
    d = idx[:, None, :] - idx[None, :, :] + off
    H = Gs[d[..., 0], d[..., 1], d[..., 2]]               # (N, N) dense Toeplitz operator
    return np.stack([(H @ Q[p].reshape(N)).reshape(shape) for p in range(Q.shape[0])])


def convolve_fft(Q: np.ndarray, Gs: np.ndarray, pad=None) -> np.ndarray:
    """Step (ii) with the FFT: circular convolution on a padded grid L >= 2N - 1 per axis."""
    shape = Q.shape[1:]
    L = tuple(2 * n - 1 for n in shape) if pad is None else tuple(pad)
    # wrap the kernel: separation d sits at index d mod L
    K = np.zeros(L, dtype=np.complex128)
    ax = [np.arange(-(n - 1), n) % l for n, l in zip(shape, L)]
    K[np.ix_(*ax)] = Gs
    Kf = scipy.fft.fftn(K)
    out = np.empty_like(Q)
    for p in range(Q.shape[0]):
        F = scipy.fft.fftn(Q[p], s=L)
        out[p] = scipy.fft.ifftn(F * Kf)[tuple(slice(0, n) for n in shape)]
    return out


def interpolate(grid: Grid, W: np.ndarray, Phi: np.ndarray, k: float, eta: float) -> np.ndarray:
    """Step (iii) plus the sum over psi:
    v_a = -j k eta0 [ sum_{psi=x,y,z} <W_psi[a], Phi_psi> - k^-2 <W_phi[a], Phi_phi> ]."""
    nb = W.shape[1]
    p = W.shape[2]
    n = grid.g.shape[0]
    local = np.arange(n) % nb
    v = np.zeros(n, dtype=np.complex128)
    sig = (1.0, 1.0, 1.0, -1.0 / (k * k))
    for i in range(p):
        for j in range(p):
            for l in range(p):
                gx, gy, gz = grid.g[:, 0] + i, grid.g[:, 1] + j, grid.g[:, 2] + l
                for psi in range(4):
                    v += sig[psi] * W[psi, local, i, j, l] * Phi[psi, gx, gy, gz]
    return -1j * k * eta * v


def interpolate_rows(grid: Grid, W: np.ndarray, Phi: np.ndarray, k: float, eta: float,
                     rows: np.ndarray) -> np.ndarray:
    """Step (iii) for the listed unknowns only (same sum as `interpolate`)."""
    nb = W.shape[1]
    p = W.shape[2]
    local = rows % nb
    g = grid.g[rows]
    v = np.zeros(rows.size, dtype=np.complex128)
    sig = (1.0, 1.0, 1.0, -1.0 / (k * k))
    for i in range(p):
        for j in range(p):
            for l in range(p):
                for psi in range(4):
                    v += sig[psi] * W[psi, local, i, j, l] * Phi[psi, g[:, 0] + i, g[:, 1] + j, g[:, 2] + l]
    return -1j * k * eta * v


def near_pairs(center_a, g_a, center_b, g_b, r_near: float, order: int) -> np.ndarray:
    """Boolean (na, nb) near-field mask between two sets of basis functions."""
    d = center_a[:, None, :] - center_b[None, :, :]
    close = np.sqrt((d * d).sum(-1)) <= r_near + 1e-12
    overlap = np.all(np.abs(g_a[:, None, :] - g_b[None, :, :]) <= order, axis=-1)
    return close | overlap


def grid_pair_values(Wa, ga, Wb, gb, Gs, Gshape, k: float, eta: float) -> np.ndarray:
    """G_grid_ab = -j k eta0 sum_psi sigma_psi sum_{p,p'} W_psi[a,p] G(g_a+p-g_b-p') W_psi[b,p'].

    Wa, Wb: (4, P, q, q, q) per pair; ga, gb: (P, 3); Gs indexed by d + N - 1 on the
    full grid of shape Gshape.
    """
    q = Wa.shape[2]
    P = ga.shape[0]
    off = np.array([n - 1 for n in Gshape])
    pts = np.stack(np.meshgrid(np.arange(q), np.arange(q), np.arange(q), indexing="ij"), -1).reshape(-1, 3)
    rel = pts[:, None, :] - pts[None, :, :]                       # (q^3, q^3, 3)
    sig = (1.0, 1.0, 1.0, -1.0 / (k * k))
    out = np.zeros(P, dtype=np.complex128)
    for s in range(0, P, 2048):
        sl = slice(s, min(s + 2048, P))
        d = (ga[sl] - gb[sl])[:, None, None, :] + rel[None] + off
        K = Gs[d[..., 0], d[..., 1], d[..., 2]]                    # (p, q^3, q^3)
        for psi in range(4):
            wa = Wa[psi, sl].reshape(-1, q ** 3)
            wb = Wb[psi, sl].reshape(-1, q ** 3)
            out[sl] += sig[psi] * np.einsum("pi,pij,pj->p", wa, K, wb)
    return -1j * k * eta * out
