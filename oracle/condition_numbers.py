"""Condition numbers of the standard EFIE and of the macromodel system on 2 x 2 arrays
(the conditioning comparison of section VI), from the oracle's dense matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Run: python -m oracle.condition_numbers
"""
from __future__ import annotations

import numpy as np

from synth import make_workload, standard_mom_workload

from .galerkin import efie_dense
from .geometry import rwg_geometry
from .system import OracleOperator


def standard_efie(cell: float) -> np.ndarray:
    """Dense G of a 2 x 2 array of PEC Jerusalem crosses meshed on `cell` squares."""
    wl = standard_mom_workload(px=2, py=2, cell=cell)
    m = wl.surface
    return efie_dense(rwg_geometry(m.vert, m.tri, m.rwg), wl.elem_center(), wl.k, wl.eta)


def macromodel_system() -> np.ndarray:
    """Dense D - G M of the 2 x 2 slice of the 32 x 32 array (648-RWG boxes)."""
    return OracleOperator(make_workload(1, px=2, py=2)).dense()


def main() -> None:
    for cell in (0.02, 0.01):
        G = standard_efie(cell)
        print(f"standard EFIE, 2x2 crosses, cell {cell}: {G.shape[0]} unknowns, cond {np.linalg.cond(G):.1f}")
    A = macromodel_system()
    print(f"macromodel system, 2x2 boxes: {A.shape[0]} unknowns, cond {np.linalg.cond(A):.1f}")


if __name__ == "__main__":
    main()
