"""Plane-wave excitation vector (section IV eq. V1) and radiated far field.

V_n = < Lambda_n, n x n x E_inc > = -< Lambda_n, E_inc > for a tangential testing
function (the paper writes the un-hatted Lambda there; the testing functions are
the RWG functions of the equivalent surface, as in eq. EFIEDiscretized_Outer).

Plane wave arriving from direction (theta, phi) (not in the paper, which uses
feeds): propagation k_inc = -(sin t cos p, sin t sin p, cos t), polarisation
TM = theta_hat = (cos t cos p, cos t sin p, -sin t), TE = phi_hat = (-sin p, cos p, 0),
E_inc(r) = e_hat exp(-j k k_inc . r), unit amplitude.
"""
from __future__ import annotations

import numpy as np

from .geometry import RwgGeom, seven_point_rule

_BARY, _W = seven_point_rule()


def incidence(theta: float, phi: float, pol: int):
    st, ct, sp_, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    kinc = -np.array([st * cp, st * sp_, ct])
    e = np.array([ct * cp, ct * sp_, -st]) if pol == 0 else np.array([-sp_, cp, 0.0])
    return kinc, e


def plane_wave_rhs(geo: RwgGeom, centers: np.ndarray, theta: float, phi: float, pol: int,
                   k: float) -> np.ndarray:
    """V for every (element, RWG), element-major; centers (n_elem, 3)."""
    kinc, e = incidence(theta, phi, pol)
    out = np.zeros((centers.shape[0], geo.n_rwg), dtype=np.complex128)
    for sgn, tidx, free in ((1.0, geo.tp, geo.pp), (-1.0, geo.tm, geo.pm)):
        tv = geo.tri_vert[tidx]
        A = geo.tri_area[tidx]
        rq = np.einsum("qi,nik->nqk", _BARY, tv)                       # (n, 7, 3) local
        lam_e = sgn * (geo.length / (2.0 * A))[:, None] * np.einsum("nqk,k->nq", rq - free[:, None, :], e)
        phase_local = np.exp(-1j * k * np.einsum("nqk,k->nq", rq, kinc))
        phase_elem = np.exp(-1j * k * centers @ kinc)                   # (n_elem,)
        s = np.einsum("q,nq,nq->n", _W, lam_e, phase_local) * A
        out += phase_elem[:, None] * s[None, :]
    return -out.reshape(-1)


def radiated_field(geo: RwgGeom, centers: np.ndarray, J: np.ndarray, rhat: np.ndarray,
                   k: float, eta: float) -> np.ndarray:
    """Far-zone E r exp(j k r) of equivalent currents J (element-major) along unit rhat (D, 3).

    E_far = -(j k eta / 4 pi) (I - rhat rhat) . sum_a J_a int Lambda_a exp(j k rhat . r') dS'.
    """
    Jm = J.reshape(centers.shape[0], geo.n_rwg)
    acc = np.zeros((rhat.shape[0], 3), dtype=np.complex128)
    for sgn, tidx, free in ((1.0, geo.tp, geo.pp), (-1.0, geo.tm, geo.pm)):
        tv = geo.tri_vert[tidx]
        A = geo.tri_area[tidx]
        rq = np.einsum("qi,nik->nqk", _BARY, tv)
        lam = sgn * (geo.length / (2.0 * A))[:, None, None] * (rq - free[:, None, :])  # (n, 7, 3)
        ph_loc = np.exp(1j * k * np.einsum("nqk,dk->dnq", rq, rhat))                 # (D, n, 7)
        ph_el = np.exp(1j * k * rhat @ centers.T)                                     # (D, n_elem)
        per_basis = np.einsum("q,n,nqk,dnq->dnk", _W, A, lam, ph_loc)               # (D, n, 3)
        acc += np.einsum("dm,mn,dnk->dk", ph_el, Jm, per_basis)
    proj = acc - rhat * np.einsum("dk,dk->d", rhat, acc)[:, None]
    return -(1j * k * eta / (4.0 * np.pi)) * proj


def rcs_db(E: np.ndarray) -> np.ndarray:
    """Bistatic RCS 10 log10(4 pi |E_far|^2 / |E0|^2) in dB relative to lambda^2 (E0 = 1)."""
    return 10.0 * np.log10(4.0 * np.pi * np.maximum((np.abs(E) ** 2).sum(-1), 1e-300))


def radiated_near_field(geo: RwgGeom, centers: np.ndarray, J: np.ndarray, points: np.ndarray,
                        k: float, eta: float) -> np.ndarray:
    """E(r) of surface currents J (element-major) at points (P, 3) away from the surfaces:
    E = -j k eta int J G dS' - j (eta / k) grad int (div' J) G dS'  (G = exp(-j k R) / (4 pi R)),
    the 7-point rule on every source triangle (points must be well separated from them)."""
    Jm = J.reshape(centers.shape[0], geo.n_rwg)
    out = np.zeros((points.shape[0], 3), dtype=np.complex128)
    for sgn, tidx, free in ((1.0, geo.tp, geo.pp), (-1.0, geo.tm, geo.pm)):
        tv = geo.tri_vert[tidx]
        A = geo.tri_area[tidx]
        rq = np.einsum("qi,nik->nqk", _BARY, tv)
        lam = sgn * (geo.length / (2.0 * A))[:, None, None] * (rq - free[:, None, :])  # (n, 7, 3)
        div = sgn * geo.length / A                                                     # (n,)
        for m in range(centers.shape[0]):
            src = rq + centers[m]
            d = points[:, None, None, :] - src[None]                                  # (P, n, 7, 3)
            R = np.sqrt((d * d).sum(-1))
            G = np.exp(-1j * k * R) / (4.0 * np.pi * R)
            dG = -(1.0 + 1j * k * R) * G / R                                          # dG/dR
            w = _W[None, None, :] * A[None, :, None] * Jm[m][None, :, None]           # (P, n, 7)
            out += -1j * k * eta * np.einsum("pnq,nqk->pk", w * G, lam)
            out += -1j * (eta / k) * np.einsum("pnq,n,pnqk->pk", w * dG / R, div, d)
    return out
