"""CPU checks of the C ABI library: every declared symbol is exported, the
host planner's geometry equals the oracle's, and argument errors are
reported before any device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle

from oracle_cases import leaf_nodes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _H():
    import paper_1612_02736_amd as H
    try:
        H.lib()
    except ImportError as e:
        pytest.fail(f"libhps.so not built: {e}")
    return H


def _declared(header):
    txt = open(os.path.join(ROOT, "include", header)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hps_[a-z0-9_]+)\s*\(", txt)))


@pytest.mark.parametrize("header", ["hps.h", "hps_debug.h"])
def test_every_declared_symbol_is_exported(header):
    L = ctypes.CDLL(_H().LIB_PATH)
    names = _declared(header)
    assert len(names) >= 5
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("nx,ny,nprob,refine,bc", [
    (4, 4, 1, None, None), (3, 5, 1, None, None), (2, 2, 3, None, None),
    (4, 4, 1, (0, 0.25, 0.75, 1), None), (4, 4, 1, (0, 0.37, 0.61, 3), None),
    (2, 2, 2, (1, 0.8, 0.3, 2), None),
    (4, 4, 1, None, "NPNP"), (5, 4, 1, None, "PPPP"), (4, 6, 2, None, "PNPN"),
    (3, 4, 1, (0, 0.4, 0.5, 2), "NNNN"), (4, 4, 1, (0, 0.5, 0.5, 1), "DPDP")])
def test_geometry_matches_oracle(nx, ny, nprob, refine, bc):
    """Leaf grids, Gauss node numbering and the canonical boundary list agree
    with the oracle's, including trees with Neumann and periodic sides (a
    problem with a Neumann side has one more box in the library: the closure
    above its root)."""
    H = _H()
    t = H.Tree(0.0, 1.0, 0.0, 1.0, nx, ny, nprob)
    ot = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, nx, ny, nprob)
    if bc:
        t.set_bc(bc)
        ot.set_bc(bc)
    if refine:
        t.refine_point(*refine)
        ot.refine_point(*refine)
    assert t.n_leaves == len(ot.leaves)
    closures = nprob if bc and "N" in bc else 0
    assert t.info()["n_boxes"] == len(ot.boxes) + closures
    for p in (8, 16):
        np.testing.assert_allclose(t.leaf_cheb_nodes(p), leaf_nodes(ot, p), atol=2e-16)
    q = 7
    xy, bd = ot.gauss(q)
    ng, nb = t.counts(q)
    assert (ng, nb) == (xy.shape[0], bd.size)
    np.testing.assert_allclose(t.gauss_nodes(q), xy, atol=2e-16)
    np.testing.assert_allclose(t.bdry_gauss_nodes(q), xy[bd], atol=2e-16)


def test_argument_errors_before_device_work():
    H = _H()
    L = H.lib()
    h = ctypes.c_void_p()
    assert L.hps_tree_uniform(0.0, 1.0, 0.0, 1.0, 0, 4, 1, ctypes.byref(h)) == -1
    assert L.hps_tree_uniform(1.0, 1.0, 0.0, 1.0, 4, 4, 1, ctypes.byref(h)) == -1
    t = H.Tree(0, 1, 0, 1, 2, 2)
    assert L.hps_tree_refine_point(t._h, 5, 0.5, 0.5, 1, 1.4) == -2
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)          # never dereferenced: arguments fail first
    for (p, q) in [(8, 8), (8, 9), (3, 2), (7, 6)]:
        o = H.hps.BuildOpts(q=q, stream=None, keep_fp32=0)
        rc = L.hps_build(t._h, fake, p, ctypes.byref(o), ctypes.byref(out))
        assert rc == -1, (p, q, rc)
        assert not out.value
    assert "p must" in L.hps_last_error().decode() or "need p" in L.hps_last_error().decode()


def test_workspace_size_grows_with_tree():
    H = _H()
    a = H.Tree(0, 1, 0, 1, 4, 4).workspace_bytes(16)
    b = H.Tree(0, 1, 0, 1, 8, 8).workspace_bytes(16)
    assert 0 < a < b
    # leaves alone: F, S_ci, H, T in FP64
    mi, g4 = 14 * 14, 60
    assert b >= 64 * 8 * (mi * (mi + g4) + g4 * mi + g4 * g4)


def test_economic_workspace_drops_exactly_the_leaf_inverses():
    """The storage-efficient version (Sec. 5.4 remark) keeps no leaf F: each
    leaf's [S_ci | F] block (mi x (4q + mi) doubles) shrinks to S_ci (mi x 4q),
    blocks being padded to 32 doubles, on uniform and refined trees and for
    several p."""
    H = _H()
    pad = lambda n: (n + 31) // 32 * 32
    for (nx, p, refine) in [(4, 16, None), (8, 12, None), (4, 10, (0.3, 0.6, 2))]:
        t = H.Tree(0, 1, 0, 1, nx, nx)
        if refine:
            t.refine_point(0, *refine)
        mi, g4 = (p - 2) ** 2, 4 * (p - 1)
        full, econ = t.workspace_bytes(p), t.workspace_bytes(p, economic=True)
        assert full - econ == 8 * t.n_leaves * (pad(mi * (g4 + mi)) - pad(mi * g4)), \
            (nx, p, full, econ)
        assert full - econ >= 8 * t.n_leaves * (mi * mi - 32)


def test_economic_build_rejects_fp32_copies():
    H = _H()
    L = H.lib()
    t = H.Tree(0, 1, 0, 1, 2, 2)
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)          # never dereferenced: arguments fail first
    o = H.hps.BuildOpts(q=0, stream=None, keep_fp32=1, economic=1)
    assert L.hps_build(t._h, fake, 8, ctypes.byref(o), ctypes.byref(out)) == -1
    assert not out.value
    assert "economic" in L.hps_last_error().decode()


def test_translation_invariant_workspace():
    """One operator copy per distinct box: far below the full build on
    uniform trees, never above it, and not offered on refined trees."""
    H = _H()
    for (nx, p) in [(4, 16), (16, 12), (64, 16)]:
        t = H.Tree(0, 1, 0, 1, nx, nx)
        full, ded = t.workspace_bytes(p), t.workspace_bytes(p, translation_invariant=True)
        assert 0 < ded <= full, (nx, p, ded, full)
        if nx >= 16:
            assert ded < full / 4, (nx, p, ded, full)
    t = H.Tree(0, 1, 0, 1, 4, 4).refine_point(0, 0.3, 0.6, 2)
    assert t.workspace_bytes(12, translation_invariant=True) == 0
    assert t.workspace_bytes(12, economic=True, translation_invariant=True) == 0
