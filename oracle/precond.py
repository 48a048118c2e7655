"""Block-Jacobi preconditioner of the final system (section IV eq. finalsystem).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The diagonal block of D - G T A^-1 B belonging to element m is D - G_mm M_t(m),
with G_mm the AIM operator (section V: grid far field plus pre-corrected near
field) between the RWG functions of element m itself.  The grid part depends only
on node separations and the near field of an element on itself is the same for
every site, so G_mm equals the AIM operator of a one-element array of the same
surface and grid; the oracle takes it from there, column by column, and inverts
each kind's block with a library routine.  The paper's own solves use an
incomplete factorisation of the near-field matrix (section VI); this per-kind
block form is the reading implemented by the device library.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from synth import Workload

from .system import OracleOperator


def one_element(wl: Workload) -> Workload:
    """The same surface, grid and operator data on a 1 x 1 lattice."""
    return replace(wl, px=1, py=1, elem_type=np.zeros(1, dtype=np.int32))


def self_block(wl: Workload) -> np.ndarray:
    """G_self (N x N): G of a one-element array applied to each unit vector."""
    op = OracleOperator(one_element(wl))
    n = op.nb
    G = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        G[:, j] = op.g_apply(e)
    return G


def diagonal_blocks(wl: Workload, G_self: np.ndarray | None = None) -> np.ndarray:
    """(n_types, N, N): D - G_self M_t for each kind t."""
    G = self_block(wl) if G_self is None else G_self
    n = G.shape[0]
    r, c, v = wl.d_matrix()
    D = np.zeros((n, n), dtype=np.complex128)
    np.add.at(D, (r, c), v)
    M = wl.macromodels()
    return np.stack([D - G @ M[t] for t in range(wl.n_types)])


def block_jacobi(wl: Workload, G_self: np.ndarray | None = None) -> np.ndarray:
    """(n_types, N, N): P_t = (D - G_self M_t)^-1."""
    return np.stack([np.linalg.inv(A) for A in diagonal_blocks(wl, G_self)])


def apply(P: np.ndarray, elem_type: np.ndarray, x: np.ndarray) -> np.ndarray:
    """blockdiag(P_t(m)) x for one element-major vector."""
    n = P.shape[1]
    X = x.reshape(-1, n)
    out = np.empty_like(X)
    for m in range(X.shape[0]):
        out[m] = P[elem_type[m]] @ X[m]
    return out.reshape(-1)
