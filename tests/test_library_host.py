"""CPU tests of the native library: it loads, exports every declared entry
point, validates its arguments, and its host construction (cluster tree,
partition, ACA in C++) agrees with the independent oracle.  No GPU work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.greens import CoplanarRectGeometry
from oracle.hmatrix import HMatrix as OracleH
from synth import WORKLOADS, config_fault, planar_rect_fault
from synth.faults import MU, NU

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2110_12165_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "hmat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:hmat_status|void|const char\*|int64_t)\s+(\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert {"hmat_build", "hmat_matvec", "hmat_matvec_T", "rs_rhs"} <= set(names)
    so = lib.load()
    for name in names:
        assert hasattr(so, name), name
        assert name in lib.SIGNATURES, name


def _host_build(lib, f, w, **over):
    so = lib.load()
    verts = np.ascontiguousarray(f.verts)
    sd = np.ascontiguousarray(f.slip_dir)
    mesh = lib.HmatMesh(f.n, 4, verts.ctypes.data_as(C.POINTER(C.c_double)),
                        sd.ctypes.data_as(C.POINTER(C.c_double)))
    green = lib.HmatGreen(lib.GF_FS_RECT_COPLANAR, over.pop("component", 0), MU, NU)
    o = lib.HmatOpts()
    so.hmat_default_opts(C.byref(o))
    o.aca_eps, o.eta, o.leaf, o.lattice = w["aca_eps"], w["eta"], w["leaf"], w["lattice"]
    for k, v in over.items():
        setattr(o, k, v)
    h = C.c_void_p()
    st = so.hmat_build_host(C.byref(mesh), C.byref(green), C.byref(o), C.byref(h))
    return st, h


def _export(lib, h):
    so = lib.load()
    hb = lib.HmatHostBlocks()
    lib.check(so.hmat_export(h, C.byref(hb)))
    nb = hb.nblocks
    return dict(perm=np.ctypeslib.as_array(hb.perm, shape=(hb.n,)).copy(),
                desc=np.ctypeslib.as_array(hb.desc, shape=(6 * nb,)).reshape(nb, 6).copy(),
                off=np.ctypeslib.as_array(hb.off, shape=(nb,)).copy(),
                values=np.ctypeslib.as_array(hb.values, shape=(hb.nvalues,)).copy())


@pytest.mark.parametrize("name", ["planar64x32", "dip30_48x24", "strike_37x23"])
def test_host_build_matches_oracle(lib, name):
    w = WORKLOADS[name]
    f = config_fault(name)
    st, h = _host_build(lib, f, w)
    assert st == 0, lib.load().hmat_last_error()
    ex = _export(lib, h)
    lib.load().hmat_destroy(h)
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    H = OracleH.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
    assert np.array_equal(ex["perm"], H.perm)
    od = np.array([[1 if b.kind == "lr" else 0, b.r0, b.m, b.c0, b.n, b.rank] for b in H.blocks])
    assert np.array_equal(od, ex["desc"])
    # the factors represent the same blocks to rounding
    for k, b in enumerate(H.blocks):
        o, (kind, r0, m, c0, n, r) = ex["off"][k], ex["desc"][k]
        if kind == 0:
            D = ex["values"][o:o + m * n].reshape(n, m).T
            np.testing.assert_allclose(D, b.D, rtol=0, atol=1e-12 * np.abs(b.D).max())
        elif r:
            U = ex["values"][o:o + m * r].reshape(r, m).T
            V = ex["values"][o + m * r:o + (m + n) * r].reshape(r, n).T
            ref = b.U @ b.V.T
            assert np.abs(U @ V.T - ref).max() <= 1e-10 * np.abs(ref).max()


def test_normal_component_of_coplanar_fault_is_zero(lib):
    w = WORKLOADS["dip30_48x24"]
    st, h = _host_build(lib, config_fault("dip30_48x24"), w, component=1)
    assert st == 0
    ex = _export(lib, h)
    lib.load().hmat_destroy(h)
    assert np.all(ex["values"] == 0.0)


def test_invalid_arguments_rejected(lib):
    so = lib.load()
    f = planar_rect_fault(8, 8, 100.0, 90.0, "strike")
    w = dict(aca_eps=1e-6, eta=2.0, leaf=4, lattice=1)
    for bad in (dict(aca_eps=0.0), dict(eta=-1.0), dict(leaf=0), dict(lattice=3), dict(prec=7), dict(kernel=9),
                dict(wg_waves=5), dict(wg_waves_p1=2), dict(mm_groups=4), dict(mm_groups=-1), dict(transpose=2),
                dict(build_device=2), dict(max_nrhs=-1), dict(n_threads=-1)):
        st, h = _host_build(lib, f, dict(w, **{k: v for k, v in bad.items() if k in w}),
                            **{k: v for k, v in bad.items() if k not in w})
        assert st == -1, bad
        assert so.hmat_last_error()
    # lattice deeper than the tree
    st, h = _host_build(lib, f, dict(w, leaf=64, lattice=4))
    assert st == -1 and b"complete" in so.hmat_last_error()
    # non-coplanar mesh
    g = planar_rect_fault(4, 4, 100.0, 90.0, "strike")
    g.verts[3, :, 1] += 1.0
    st, h = _host_build(lib, g, w)
    assert st == -1
    # non-finite coordinate
    g = planar_rect_fault(4, 4, 100.0, 90.0, "strike")
    g.verts[0, 0, 0] = np.nan
    st, h = _host_build(lib, g, w)
    assert st == -1
    # products on a host-only handle report a state error, not a crash
    st, h = _host_build(lib, f, w)
    assert st == 0
    assert so.hmat_matvec(h, C.c_void_p(16), C.c_void_p(1 << 20), 1, 64, 1.0, 0.0, None) == -4
    # the frozen-step integration and its adjoint check the handle first
    prm = lib.RsParams(64, 1e-6, 0.6, 4.6e6, 1e-9, 16, 16, 16)
    dts = (C.c_double * 3)(1.0, 2.0, 4.0)
    assert so.rs_rk45_replay(h, None, C.byref(prm), C.c_void_p(16), None, dts, 3, None, 1, C.c_void_p(16), None) == -4
    assert so.rs_rk45_adjoint(h, None, C.byref(prm), C.c_void_p(16), 2, dts, 3, None, C.c_void_p(16),
                              C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), 1 << 30, None) == -4
    so.hmat_destroy(h)
    # workspace of the adjoint: 8 (36 n K + 31 n + 32) bytes
    assert so.rs_rk45_adjoint_workspace_bytes(1000, 50) == 8 * (36 * 1000 * 50 + 31 * 1000 + 32)
    assert so.rs_rk45_adjoint_workspace_bytes(-1, 50) == -1
    assert so.rs_rk45_adjoint_workspace_bytes(10, 0) == -1
    assert so.rs_rk45_adjoint_workspace_bytes(1 << 30, 1 << 30) == -1


def test_import_validates_tiling(lib):
    so = lib.load()
    o = lib.HmatOpts()
    so.hmat_default_opts(C.byref(o))
    perm = np.arange(4, dtype=np.int32)
    desc = np.array([[0, 0, 4, 0, 3, 0]], dtype=np.int64)     # leaves a gap
    off = np.zeros(1, dtype=np.int64)
    vals = np.zeros(12)
    hb = lib.HmatHostBlocks(4, 1, 12, perm.ctypes.data_as(C.POINTER(C.c_int32)),
                            desc.ctypes.data_as(C.POINTER(C.c_int64)),
                            off.ctypes.data_as(C.POINTER(C.c_int64)),
                            vals.ctypes.data_as(C.POINTER(C.c_double)))
    h = C.c_void_p()
    assert so.hmat_import(C.byref(hb), C.byref(o), None, C.byref(h)) == -1
    perm2 = np.array([0, 1, 1, 3], dtype=np.int32)
    desc2 = np.array([[0, 0, 4, 0, 4, 0]], dtype=np.int64)
    vals2 = np.zeros(16)
    hb2 = lib.HmatHostBlocks(4, 1, 16, perm2.ctypes.data_as(C.POINTER(C.c_int32)),
                             desc2.ctypes.data_as(C.POINTER(C.c_int64)),
                             off.ctypes.data_as(C.POINTER(C.c_int64)),
                             vals2.ctypes.data_as(C.POINTER(C.c_double)))
    assert so.hmat_import(C.byref(hb2), C.byref(o), None, C.byref(h)) == -1


def test_integration_entry_points_reject_bad_arguments(lib):
    """Argument checks of the replay, adjoint and ensemble entry points run
    before any device work (host-only handle or null pointers)."""
    so = lib.load()
    f = planar_rect_fault(8, 8, 100.0, 90.0, "strike")
    st, h = _host_build(lib, f, dict(aca_eps=1e-6, eta=2.0, leaf=4, lattice=1))
    assert st == 0
    prm = lib.RsParams(64, 1e-6, 0.6, 4.6e6, 1e-9, 16, 16, 16)
    dts = (C.c_double * 2)(1.0, 2.0)
    # null parameters / handle
    assert so.rs_rk45_replay(None, None, C.byref(prm), C.c_void_p(16), None, dts, 2, None, 1, C.c_void_p(16), None) == -1
    assert so.rs_rk45_replay(h, None, None, C.c_void_p(16), None, dts, 2, None, 1, C.c_void_p(16), None) == -1
    # ensemble: host-only handle, bad member counts, bad mode
    ep = lib.RsEnsParams(64, 8, 2, 1e-6, 0.6, 4.6e6, 1e-9, 16, 16, 16)
    es = lib.RsEnsState()
    for r in range(64):
        es.dt[r] = 1.0
    assert so.rs_ens_rk45_run(h, None, C.byref(ep), C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), C.byref(es),
                              1, 0, 0, None) == -4
    so.hmat_destroy(h)
    assert so.rs_ens_workspace_bytes(100, 0) == -1
    assert so.rs_ens_workspace_bytes(100, 65) == -1
    assert so.rs_ens_workspace_bytes(-1, 8) == -1
    assert so.rs_ens_workspace_bytes(100, 8) >= 8 * 28 * 100 * 8
    # kernel entries: out-of-range index
    verts = np.ascontiguousarray(f.verts)
    sd = np.ascontiguousarray(f.slip_dir)
    mesh = lib.HmatMesh(f.n, 4, verts.ctypes.data_as(C.POINTER(C.c_double)), sd.ctypes.data_as(C.POINTER(C.c_double)))
    green = lib.HmatGreen(lib.GF_FS_RECT_COPLANAR, 0, 32e9, 0.25)
    rows = (C.c_int64 * 1)(f.n)
    cols = (C.c_int64 * 1)(0)
    out = (C.c_double * 1)()
    assert so.hmat_kernel_entries(C.byref(mesh), C.byref(green), 1, rows, cols, out) == -1
    assert b"range" in so.hmat_last_error()
