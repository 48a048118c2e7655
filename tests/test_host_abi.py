"""Host-side checks of the C-ABI library (no GPU): exports, host setup vs the oracle, argument errors."""
import ctypes
import os
import re

import numpy as np
import pytest

from synth import make_workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1712_02443_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1712_02443_amd.build import build
        build()
    return _lib.load()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "aimm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([a-z_][a-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_1712_02443_amd import _lib
    assert set(names) == set(_lib.EXPORTS), set(names) ^ set(_lib.EXPORTS)


def _host_op(wl):
    from paper_1712_02443_amd import AimOperator
    return AimOperator.from_workload(wl, host_only=True)


@pytest.mark.parametrize("case", [(0, {}), (2, dict(px=3, py=2, nrhs=1)), (1, dict(px=2, py=3, nrhs=1))])
def test_host_near_field_matches_oracle(lib, case):
    """Pre-corrected near field computed by the library's C++ setup vs the oracle's per-offset blocks."""
    from oracle.system import OracleOperator
    idx, kw = case
    wl = make_workload(idx, **kw)
    op = _host_op(wl)
    inf = op.info()
    o = OracleOperator(wl)
    assert (inf["nx"], inf["ny"], inf["nz"]) == tuple(o.grid.shape)
    rows, offs, cols, vals, offsets = op.near()
    assert len(offsets) == len(o.blocks)
    mx = max(np.abs(v[2]).max() for v in o.blocks.values())
    for oi, (dx, dy) in enumerate(offsets):
        ba, bb, bv = o.blocks[(int(dx), int(dy))]
        sel = offs == oi
        ours = {(int(a), int(b)): v for a, b, v in zip(rows[sel], cols[sel], vals[sel])}
        theirs = {(int(a), int(b)): v for a, b, v in zip(ba, bb, bv)}
        assert set(ours) == set(theirs)
        err = max(abs(ours[k] - theirs[k]) for k in theirs)
        assert err <= 1e-13 * mx
    op.close()


def test_host_near_field_exact_entries_against_independent_quadrature(lib):
    """The library's exact near-field entries (its pre-corrected values plus the grid part,
    whose weights the oracle's pins fix by moment identities) against references that
    share nothing with either Galerkin implementation: a 24 x 24 Gauss product rule of
    the full kernel for pairs in different boxes (0.1 wavelength apart; the 7-point
    rule is within 2e-3 there), and the pair rule on 64 sub-triangles of both triangles
    for pairs in one box (the 7-point rule is within 3e-2 of it on touching pairs)."""
    from galerkin_refs import plain_entry, refined_entry
    from oracle import aim
    from oracle.system import OracleOperator
    wl = make_workload(0)
    op = _host_op(wl)
    rows, offs, cols, vals, offsets = op.near()
    o = OracleOperator(wl, near=False)
    rng = np.random.default_rng(0)
    worst = {True: 0.0, False: 0.0}
    for oi, (dx, dy) in enumerate(offsets):
        pick = rng.choice(np.flatnonzero(offs == oi), 3, replace=False)
        sh = np.array([dx, dy, 0]) * wl.pitch_cells
        a, b = rows[pick], cols[pick]
        grid = aim.grid_pair_values(o.W[:, a], o.s_local[a], o.W[:, b], (o.s_local + sh)[b], o.Gs, o.grid.shape,
                                    wl.k, wl.eta)
        exact = vals[pick] + grid
        same_box = (int(dx), int(dy)) == (0, 0)
        for i in range(len(pick)):
            if same_box:
                ref = refined_entry(o.geo, a[i], b[i], wl.k, wl.eta, levels=3)
            else:
                ref = plain_entry(o.geo, a[i], np.zeros(3), b[i], sh * wl.h, wl.k, wl.eta, n=24)
            worst[same_box] = max(worst[same_box], abs(exact[i] - ref) / abs(ref))
    assert worst[False] < 5e-3
    assert worst[True] < 3e-2
    op.close()


def test_padded_lengths_are_5_smooth_and_long_enough(lib):
    for idx, kw in ((0, {}), (1, {}), (2, {}), (4, dict(px=64))):
        wl = make_workload(idx, **kw)
        inf = _host_op(wl).info() if wl.n_elem <= 1024 else None
        if inf is None:
            continue
        for n, L in ((inf["nx"], inf["lx"]), (inf["ny"], inf["ly"])):
            assert L >= 2 * n - 2
            r = L
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            assert r == 1
    inf = _host_op(make_workload(1)).info()
    assert (inf["nx"], inf["ny"], inf["nz"], inf["lx"], inf["ly"]) == (195, 195, 9, 400, 400)


def test_invalid_arguments_are_rejected(lib):
    from paper_1712_02443_amd import AimError, AimOperator
    wl = make_workload(0)
    m = wl.surface
    base = dict(k=wl.k, eta=wl.eta, h=wl.h, r_near=wl.r_near, order=2, px=2, py=2, pitch_cells=6,
                elem_type=wl.elem_type, n_types=1, max_rhs=1, host_only=True)
    for bad in (dict(order=5), dict(h=-1.0), dict(px=0), dict(elem_type=np.array([0, 0, 0, 3])),
                dict(max_rhs=0)):
        kw = dict(base, **bad)
        with pytest.raises(AimError) as e:
            AimOperator(m.vert, m.tri, m.rwg, **kw)
        assert e.value.code == -1
    rwg = m.rwg.copy()
    rwg[0, 2] = 10_000
    with pytest.raises(AimError):
        AimOperator(m.vert, m.tri, rwg, **base)


def test_device_calls_on_host_op_report_state(lib):
    from paper_1712_02443_amd import _lib
    wl = make_workload(0)
    op = _host_op(wl)
    buf = ctypes.c_void_p(1)
    code = lib.aim_matvec(op._op, buf, ctypes.c_void_p(2), 1, 0, 0, None)
    assert code == _lib.AIM_ESTATE
    assert b"aim_build_host" in lib.aim_last_error()
    # operator data is accepted (kept on the host for the preconditioner); products are not
    M = np.zeros(2 * 288 * 288)
    assert lib.aim_set_macromodels(op._op, M.ctypes.data_as(_lib._f64p)) == _lib.AIM_OK
    assert lib.macro_apply(op._op, buf, ctypes.c_void_p(2), 1, 0, None) == _lib.AIM_ESTATE
    assert lib.aim_matvec(None, buf, buf, 1, 0, 0, None) == _lib.AIM_EINVAL
    rh = np.array([0.0, 0.0, 1.0])
    assert lib.aim_far_field(op._op, buf, 1, 1, rh.ctypes.data_as(_lib._f64p), buf, None, 0, None) == _lib.AIM_ESTATE
    assert lib.aim_far_field(op._op, buf, 1, 0, rh.ctypes.data_as(_lib._f64p), buf, None, 0, None) == _lib.AIM_EINVAL
    rh[0] = np.nan
    assert lib.aim_far_field(op._op, buf, 1, 1, rh.ctypes.data_as(_lib._f64p), buf, None, 0, None) == _lib.AIM_EINVAL
    op.close()


def test_tuning_calls_check_their_arguments(lib):
    """aim_get_tuning / aim_set_tuning: null arguments are refused, a host-only op reports
    its build-time configuration and refuses a new one (it has no device kernels), and
    the Python struct has the layout the header declares (10 int32 fields)."""
    from paper_1712_02443_amd import _lib
    assert ctypes.sizeof(_lib.AimTuning) == 10 * 4
    wl = make_workload(0)
    op = _host_op(wl)
    t = _lib.AimTuning()
    assert lib.aim_get_tuning(None, ctypes.byref(t)) == _lib.AIM_EINVAL
    assert lib.aim_get_tuning(op._op, None) == _lib.AIM_EINVAL
    assert lib.aim_get_tuning(op._op, ctypes.byref(t)) == _lib.AIM_OK
    assert list(t.near_block) == [1, 1] and list(t.near_fork) == [0, 0] and t.interp_tx >= 1 and t.interp_ty >= 1
    assert lib.aim_set_tuning(None, ctypes.byref(t)) == _lib.AIM_EINVAL
    assert lib.aim_set_tuning(op._op, ctypes.byref(t)) == _lib.AIM_ESTATE
    assert b"host-only" in lib.aim_last_error()
    op.close()


def test_footprint_grows_with_rhs_and_restart(lib):
    from paper_1712_02443_amd import footprint_bytes
    wl = make_workload(1)
    m = wl.surface
    kw = dict(k=wl.k, eta=wl.eta, h=wl.h, r_near=wl.r_near, order=2, px=32, py=32, pitch_cells=6,
              elem_type=wl.elem_type, n_types=1, max_rhs=1)
    a = footprint_bytes(m.vert, m.tri, m.rwg, nrhs=1, restart=50, precision=0, **kw)
    b = footprint_bytes(m.vert, m.tri, m.rwg, nrhs=1, restart=80, precision=0, **kw)
    c = footprint_bytes(m.vert, m.tri, m.rwg, nrhs=1, restart=50, precision=1, **kw)
    n = 663552
    assert a > 51 * n * 16          # at least the FP64 Krylov basis
    # basis vectors, Gram matrix and per-chunk reduction partials of the 30 more columns
    assert b - a == 30 * n * 16 + (81 ** 2 - 51 ** 2) * 16 + 2 * 30 * (n // 256 + 1) * 16
    assert c < a
