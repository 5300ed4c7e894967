"""GPU parity of the H-matrix product (eq. 20) against the FP64 oracle.

Tolerances:
* shared factors (oracle-built blocks imported into the library): the GPU
  sums the same terms in another order, FP64 storage and FP64 accumulation
  -> relative error <= 1e-13; FP32 storage rounds every stored entry once
  (unit roundoff 6e-8) and accumulates in FP64 -> <= 2e-5 required, about
  1e-7 expected;
* independent build (C++ construction on the library side): the same rules
  give the same blocks, so the FP64 product is held to 1e-6 against the
  oracle's H product, and both are held to 10 * eps_ACA against the plain
  product y = A x.
"""
import numpy as np
import pytest

from _util import oracle_blocks, rel, say
from oracle.dense import dense_matrix, fft_grid_product
from oracle.greens import CoplanarRectGeometry
from oracle.hmatrix import HMatrix as OracleH
from synth import WORKLOADS, config_fault, loguniform_rates
from synth.faults import MU, NU

pytestmark = pytest.mark.gpu

CASES = ["planar64x32", "dip30_48x24", "strike_37x23", "dip30_150x70"]
KERNELS = ["plain", "split", "persistent"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def hm():
    import paper_2110_12165_amd as hm
    hm.library()
    return hm


_cache = {}


def oracle_case(name):
    if name not in _cache:
        w = WORKLOADS[name]
        f = config_fault(name)
        g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
        H = OracleH.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
        _cache[name] = (w, f, g, H)
    return _cache[name]


def _opts(w):
    return dict(aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"])


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kernel", KERNELS)
def test_shared_factor_parity(torch_dev, hm, name, prec, kernel):
    torch, dev = torch_dev
    w, f, g, H = oracle_case(name)
    say(f"[shared] {name} N={f.n} {prec} {kernel}")
    B = oracle_blocks(H)
    Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec=prec, kernel=kernel)
    x = loguniform_rates(f.n, w["seed"])
    y_ref = H.matvec(x)
    y = Hg.matvec(torch.tensor(x, device=dev)).cpu().numpy()
    tol = 1e-13 if prec == "f64" else 2e-5
    r = rel(y, y_ref)
    say(f"    rel {r:.3e}")
    assert r <= tol
    assert np.max(np.abs(y - y_ref)) <= 10 * tol * np.max(np.abs(y_ref))
    if prec == "f32":
        assert r <= 1e-6          # FP64 accumulation keeps FP32 storage error near unit roundoff
    # transpose product against the oracle's transpose
    yt = Hg.matvec_T(torch.tensor(x, device=dev)).cpu().numpy()
    assert rel(yt, H.matvec_T(x)) <= tol
    Hg.close()


@pytest.mark.parametrize("name", CASES)
def test_independent_build_parity(torch_dev, hm, name):
    torch, dev = torch_dev
    w, f, g, H = oracle_case(name)
    say(f"[build] {name} N={f.n}")
    x = loguniform_rates(f.n, w["seed"])
    y_h = H.matvec(x)
    y_exact = fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, x)
    for prec, kernel in (("f64", "plain"), ("f64", "persistent"), ("f32", "persistent"), ("f32", "split")):
        Hg = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, prec=prec, kernel=kernel, **_opts(w))
        y = Hg.matvec(torch.tensor(x, device=dev)).cpu().numpy()
        info = Hg.info()
        Hg.close()
        st = H.stats()
        assert info["n_dense"] == st["n_dense"] and info["n_lr"] == st["n_lr"]
        assert info["dense_entries"] + info["lr_entries"] == st["entries"]
        r_h, r_x = rel(y, y_h), rel(y, y_exact)
        say(f"    {prec}/{kernel}: vs oracle H {r_h:.2e}, vs exact {r_x:.2e}")
        assert r_h <= (1e-6 if prec == "f64" else 2e-5)
        assert r_x <= 10 * w["aca_eps"]


def test_alpha_beta_multi_rhs_and_ld(torch_dev, hm):
    """Seven columns with a leading dimension beyond n: with the split
    schedule a pass of four vectors, one of two, then one vector (each panel
    entry read once per pass); every column against the oracle."""
    torch, dev = torch_dev
    w, f, g, H = oracle_case("dip30_48x24")
    B = oracle_blocks(H)
    rng = np.random.default_rng(21)
    n, k, ld = f.n, 7, f.n + 5
    X = rng.standard_normal((n, k))
    Y0 = rng.standard_normal((n, k))
    for kernel in KERNELS:
        Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec="f64", kernel=kernel)
        xbuf = torch.zeros(k * ld, dtype=torch.float64, device=dev)
        ybuf = torch.zeros(k * ld, dtype=torch.float64, device=dev)
        for c in range(k):
            xbuf[c * ld:c * ld + n] = torch.tensor(X[:, c], device=dev)
            ybuf[c * ld:c * ld + n] = torch.tensor(Y0[:, c], device=dev)
        ybuf[n:ld] = 7.0                              # padding must stay untouched
        Hg.matvec_raw(xbuf.data_ptr(), ybuf.data_ptr(), nrhs=k, ld=ld, alpha=-2.0, beta=0.5,
                      stream_ptr=torch.cuda.current_stream().cuda_stream)
        out = ybuf.cpu().numpy()
        for c in range(k):
            ref = -2.0 * H.matvec(X[:, c]) + 0.5 * Y0[:, c]
            assert rel(out[c * ld:c * ld + n], ref) <= 1e-13
        assert np.all(out[n:ld] == 7.0)
        # beta = 0 ignores NaN in y
        y = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
        Hg.matvec(torch.tensor(X[:, 0], device=dev), y=y, beta=0.0)
        assert torch.isfinite(y).all()
        # nrhs = 0 is a no-op
        Hg.matvec_raw(xbuf.data_ptr(), ybuf.data_ptr(), nrhs=0, ld=ld)
        Hg.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_multi_vector_passes(torch_dev, hm, prec):
    """The multi-vector product of the split schedule (passes of 4 and 2
    vectors, forward and transposed, several wave counts) against the
    oracle's products column by column, and against single-vector calls of
    the same handle to rounding."""
    torch, dev = torch_dev
    w, f, g, H = oracle_case("dip30_150x70")
    B = oracle_blocks(H)
    rng = np.random.default_rng(22)
    n, k = f.n, 6
    X = 10.0 ** rng.uniform(-12, -9, (n, k))
    tol = 1e-13 if prec == "f64" else 1e-6
    for wg, wg1 in ((8, 4), (4, 16)):
        Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec=prec, kernel="split",
                                    wg_waves=wg, wg_waves_p1=wg1)
        Xd = torch.tensor(X, device=dev)
        for tr in (False, True):
            Y = (Hg.matvec_T(Xd) if tr else Hg.matvec(Xd)).cpu().numpy()
            for c in range(k):
                ref = H.matvec_T(X[:, c]) if tr else H.matvec(X[:, c])
                assert rel(Y[:, c], ref) <= tol, (wg, wg1, tr, c)
                y1 = (Hg.matvec_T(Xd[:, c].contiguous()) if tr else Hg.matvec(Xd[:, c].contiguous())).cpu().numpy()
                assert rel(Y[:, c], y1) <= 1e-14
        Hg.close()


def test_bitwise_reproducible_and_schedule_independent(torch_dev, hm):
    torch, dev = torch_dev
    w, f, g, H = oracle_case("dip30_150x70")
    B = oracle_blocks(H)
    x = torch.tensor(loguniform_rates(f.n, 5), device=dev)
    for kernel in ("split", "persistent"):
        Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec="f64", kernel=kernel)
        ys = [Hg.matvec(x).cpu().numpy() for _ in range(5)]
        for y in ys[1:]:
            assert np.array_equal(y, ys[0])
        Hg.close()
    # other workgroup shapes and unit sizes change only the summation order
    ref = H.matvec(x.cpu().numpy())
    for wg in (4, 16):
        for ukib in (64, 1024):
            Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec="f64",
                                        kernel="persistent", wg_waves=wg, unit_kib=ukib)
            assert rel(Hg.matvec(x).cpu().numpy(), ref) <= 1e-13
            Hg.close()


def test_degenerate_sizes(torch_dev, hm):
    torch, dev = torch_dev
    from synth import planar_rect_fault
    for nx, ny, leaf in ((1, 1, 4), (2, 1, 4), (3, 2, 1), (5, 3, 64)):
        f = planar_rect_fault(nx, ny, 100.0, 90.0, "strike")
        g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
        A = dense_matrix(g)
        x = loguniform_rates(f.n, 3)
        X = loguniform_rates(f.n, 4, nrhs=6)
        for kernel in KERNELS:
            Hg = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, leaf=leaf, kernel=kernel)
            y = Hg.matvec(torch.tensor(x, device=dev)).cpu().numpy()
            assert rel(y, A @ x) <= 1e-6, (nx, ny, kernel)
            # six vectors (passes of 4 and 2 on the split schedule), forward and transposed
            Xd = torch.tensor(X, device=dev)
            Y, YT = Hg.matvec(Xd).cpu().numpy(), Hg.matvec_T(Xd).cpu().numpy()
            for c in range(X.shape[1]):
                assert rel(Y[:, c], A @ X[:, c]) <= 1e-6, (nx, ny, kernel, c)
                assert rel(YT[:, c], A.T @ X[:, c]) <= 1e-6, (nx, ny, kernel, c)
            Hg.close()


def test_zero_matrix_keeps_beta_y(torch_dev, hm):
    torch, dev = torch_dev
    w, f, g, H = oracle_case("dip30_48x24")
    for kernel in KERNELS:
        Hb = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=1, kernel=kernel, **_opts(w))
        y0 = torch.arange(f.n, dtype=torch.float64, device=dev)
        y = y0.clone()
        Hb.matvec(torch.ones(f.n, dtype=torch.float64, device=dev), y=y, alpha=1.0, beta=2.0)
        assert torch.equal(y, 2.0 * y0)
        Hb.close()


def test_autotune_and_profile(torch_dev, hm):
    """hmat_autotune picks a schedule among the candidates and keeps the
    products (and the transposed ones) within rounding of the oracle;
    hmat_profile reports one timing and byte count per launch (factors of
    the launch plus the vectors it reads and writes)."""
    torch, dev = torch_dev
    w, f, g, H = oracle_case("dip30_150x70")
    B = oracle_blocks(H)
    x = loguniform_rates(f.n, 9)
    xd = torch.tensor(x, device=dev)
    ref, ref_t = H.matvec(x), H.matvec_T(x)
    Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec="f64", kernel="auto")
    info = Hg.autotune(reps=3)
    say(f"[autotune] dip30_150x70: kernel {info['kernel']}, waves {info['wg_waves']} / {info['wg_waves_p1']}")
    assert info["kernel"] in ("plain", "split", "persistent")
    assert rel(Hg.matvec(xd).cpu().numpy(), ref) <= 1e-13
    assert rel(Hg.matvec_T(xd).cpu().numpy(), ref_t) <= 1e-13
    y = torch.empty_like(xd)
    pr = Hg.profile(xd, y, reps=5)
    assert pr["n_launches"] in (1, 2) and pr["reps"] == 5
    assert all(m > 0.0 for m in pr["ms"]) and pr["ms_product"] > 0.0
    st = Hg.info()
    if pr["n_launches"] == 2:   # phase 1 and phase 2 each count the vectors they touch
        assert sum(pr["alg_bytes"]) == st["factor_bytes"] + 40 * st["n"] + 16 * st["sum_rank"]
    else:
        assert pr["alg_bytes"][0] == st["alg_bytes"]
    assert rel(y.cpu().numpy(), ref) <= 1e-13
    Hg.close()


def test_autotune_choice_is_remembered(torch_dev, hm):
    """A second handle on the same blocks (same storage, options and
    device) takes the schedule the first one timed, without timing the
    candidates again: the same choice in a fraction of the time, and the
    same products bit for bit."""
    import time
    torch, dev = torch_dev
    w, f, g, H = oracle_case("dip30_150x70")
    B = oracle_blocks(H)
    xd = torch.tensor(loguniform_rates(f.n, 10), device=dev)
    picks, secs, ys = [], [], []
    for _ in range(2):
        Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec="f32", kernel="auto",
                                    unit_kib=128)
        t0 = time.perf_counter()
        info = Hg.autotune(reps=5)
        secs.append(time.perf_counter() - t0)
        picks.append((info["kernel"], info["wg_waves"], info["wg_waves_p1"]))
        ys.append(Hg.matvec(xd).cpu().numpy())
        Hg.close()
    say(f"[autotune cache] {picks[0]}: first {secs[0]:.3f} s, second {secs[1]:.3f} s")
    assert picks[1] == picks[0]
    assert secs[1] <= 0.5 * secs[0]
    assert np.array_equal(ys[0], ys[1])


@pytest.mark.parametrize("wg,wg1", [(8, 4), (4, 4), (8, 8)])
def test_row_split_layouts(torch_dev, hm, wg, wg1):
    """Small matrices split their oversized phase-1 units by rows, with the
    partial intermediate values added by phase 2: parity with the oracle on
    shared factors (FP64 to 1e-13, FP32 to 2e-5) and with the same handle
    built whole (ensemble buffers keep units whole), forward and transposed,
    bitwise reproducible."""
    torch, dev = torch_dev
    w, f, g, H = oracle_case("dip30_150x70")
    B = oracle_blocks(H)
    x = loguniform_rates(f.n, 21)
    xd = torch.tensor(x, device=dev)
    ref, ref_t = H.matvec(x), H.matvec_T(x)
    for prec, tol in (("f64", 1e-13), ("f32", 2e-5)):
        Hs = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec=prec, kernel="split",
                                    wg_waves=wg, wg_waves_p1=wg1)
        ys = [Hs.matvec(xd).cpu().numpy() for _ in range(3)]
        yt = Hs.matvec_T(xd).cpu().numpy()
        n_split = Hs.info()["n_units_p1"]
        Hs.close()
        assert all(np.array_equal(y, ys[0]) for y in ys[1:])
        assert rel(ys[0], ref) <= tol and rel(yt, ref_t) <= tol
        if prec == "f32":   # the ensemble buffers need FP32 storage
            Hw = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec=prec,
                                        kernel="split", wg_waves=wg, wg_waves_p1=wg1, max_nrhs=8)
            yw = Hw.matvec(xd).cpu().numpy()
            n_whole = Hw.info()["n_units_p1"]
            Hw.close()
            say(f"[row split] waves {wg}/{wg1}: phase-1 units {n_split} split, {n_whole} whole")
            assert rel(yw, ref) <= tol
            if wg1 == 4:
                assert n_split > n_whole   # the layout did split units


def test_binding_rejects_host_and_misshaped_tensors(torch_dev, hm):
    """Tensors whose addresses would reach the kernels unchecked (outputs on
    the host, wrong shapes, non-contiguous views) are refused by the binding
    before any launch."""
    torch, dev = torch_dev
    from synth import planar_rect_fault
    f = planar_rect_fault(8, 4, 100.0, 90.0, "strike")
    n = f.n
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, leaf=4, prec="f32", kernel="split", max_nrhs=8)
    x = torch.ones(n, dtype=torch.float64, device=dev)
    X = torch.ones((n, 3), dtype=torch.float64, device=dev)
    bad_y = (torch.empty(n, dtype=torch.float64), torch.empty(n + 1, dtype=torch.float64, device=dev),
             torch.empty(n, dtype=torch.float32, device=dev), torch.empty(2 * n, dtype=torch.float64, device=dev)[::2])
    for y in bad_y:
        with pytest.raises(ValueError):
            H.matvec(x, y=y)
        with pytest.raises(ValueError):
            H.profile(x, y, reps=1)
    with pytest.raises(ValueError):
        H.matvec(X, y=torch.empty((n, 2), dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):
        H.matvec(X, y=torch.empty((n, 3), dtype=torch.float64))
    with pytest.raises(ValueError):
        H.matmat(X, Y=torch.empty((n, 3), dtype=torch.float64))
    with pytest.raises(ValueError):
        H.matmat(X, Y=torch.empty((3, n), dtype=torch.float64, device=dev).t())
    a = torch.full((n,), 0.01, dtype=torch.float64, device=dev)
    strided = torch.full((2 * n,), 0.01, dtype=torch.float64, device=dev)[::2]
    with pytest.raises(ValueError):
        hm.RK45(H, None, strided, a, a, 1e-6, 0.6, 4.6e6, 1e-9)
    rk = hm.RK45(H, None, a, a, a, 1e-6, 0.6, 4.6e6, 1e-9)
    y = torch.ones(3 * n, dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):
        rk.run(y, torch.zeros(n, dtype=torch.float64), 1)
    with pytest.raises(ValueError):
        hm.rs_rhs(H, None, y, a, a, a, 1e-6, 0.6, 4.6e6, 1e-9, dydt=torch.empty(3 * n, dtype=torch.float64))
    with pytest.raises(ValueError):
        hm.rs_rhs(H, None, y, a, a, a, 1e-6, 0.6, 4.6e6, 1e-9, V_out=torch.empty(n + 1, dtype=torch.float64,
                                                                                      device=dev))
    # the valid calls still run
    assert H.matvec(x).shape == (n,) and H.matmat(X).shape == (n, 3)
    H.close()
