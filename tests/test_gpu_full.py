"""GPU parity at the full benchmark size: planar 30-degree dipping thrust,
480 x 256 squares of 50 m (N = 122880), ACA eps 1e-5, leaf 64, eta 2,
lattice 32 x 32, in the launch configurations that bench.py times.

The oracle cannot rebuild an H-matrix of this size in test time, so the
GPU products are compared with the exact product y = A x, which the oracle
computes by FFT (translation invariance of the planar grid) and, for
sampled rows, one row at a time straight from the entries.  The
requirement: relative error <= 1e-6 for FP64 storage and <= 2e-5 for FP32
storage (the compression error of this matrix is about 3e-8).  The
stiffness of equal coplanar squares is symmetric (A_ij = A_ji), so the same
exact product checks the transposed products H^T x.

The integration at this size is checked against the oracle itself: the
oracle builds the H-matrix and integrates with its own step control through
the sparse form of its product (eq. 20 on all blocks at once, row chunks on
the host's threads); the GPU takes the oracle's blocks and replays its
steps.  Nothing the GPU computes is fed to the oracle.
"""
import os

import numpy as np
import pytest

from _util import rel, say
from oracle.dense import dense_rows, fft_grid_product
from oracle.greens import CoplanarRectGeometry
from synth import WORKLOADS, config_fault, loguniform_rates
from synth.faults import MU, NU

pytestmark = pytest.mark.gpu

NAME = "dip30_480x256"


@pytest.fixture(scope="module")
def setup():
    import torch

    import paper_2110_12165_amd as hm
    from paper_2110_12165_amd.tuning import bench_options
    assert torch.cuda.is_available()
    w = WORKLOADS[NAME]
    f = config_fault(NAME)
    x = loguniform_rates(f.n, w["seed"])
    y_exact = fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, x)
    return torch, hm, bench_options, w, f, x, y_exact


@pytest.mark.parametrize("variant", ["batched_f32", "plain_f64", "batched_f64"])
def test_full_size_against_exact_product(setup, variant):
    torch, hm, bench_options, w, f, x, y_exact = setup
    opts = bench_options(NAME, variant)
    say(f"[full] {NAME} N={f.n} {variant} {opts}")
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, **opts)
    dev = torch.device("cuda:0")
    xd = torch.tensor(x, device=dev)
    y1 = H.matvec(xd).cpu().numpy()
    y2 = H.matvec(xd).cpu().numpy()
    yT = H.matvec_T(xd).cpu().numpy()             # the same handle's H^T x (A is symmetric)
    tol = 1e-6 if opts["prec"] == "f64" else 2e-5
    if variant != "plain_f64":
        # six vectors: a pass of 4 and a pass of 2 through the factors (the
        # multi-vector product bench.py times), forward and transposed, each
        # column against its exact product
        Xm = np.stack([x] + [loguniform_rates(f.n, 40 + c) for c in range(5)], axis=1)
        Xd = torch.tensor(Xm, device=dev)
        Ym = H.matvec(Xd).cpu().numpy()
        YmT = H.matvec_T(Xd).cpu().numpy()
        for c in range(Xm.shape[1]):
            yc = y_exact if c == 0 else fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, Xm[:, c])
            rc, rcT = rel(Ym[:, c], yc), rel(YmT[:, c], yc)
            say(f"    vector {c} of 6: rel vs exact {rc:.3e}, transposed {rcT:.3e}")
            assert rc <= tol and rcT <= tol, c
        assert rel(Ym[:, 0], y1) <= 1e-14 and rel(YmT[:, 0], yT) <= 1e-14
    info = H.info()
    H.close()
    r = rel(y1, y_exact)
    say(f"    rel vs exact {r:.3e}  entries {info['dense_entries'] + info['lr_entries']}")
    assert r <= tol
    assert np.array_equal(y1, y2)                 # run-to-run reproducible
    rT = rel(yT, y_exact)
    say(f"    transposed product: rel vs exact {rT:.3e}")
    assert rT <= tol
    # sampled rows, evaluated one by one from the entries
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    rows = np.random.default_rng(99).choice(f.n, 48, replace=False)
    ref = dense_rows(g, rows, x)
    assert np.max(np.abs(y1[rows] - ref)) <= 1e-5 * np.max(np.abs(y_exact))
    assert info["max_rank"] <= 64 and info["n_lr"] > 40000


@pytest.mark.parametrize("groups", [1, 2, 3])
def test_full_size_ensemble_against_exact_product(setup, groups):
    """The ensemble product (BF16x6 and BF16x3 on MFMA) with one and with
    two wave groups per 64-output slice, and with phase 2 on pairs of row
    intervals, against exact products."""
    torch, hm, bench_options, w, f, x, y_exact = setup
    opts = dict(bench_options(NAME, "batched_f32"), max_nrhs=64, mm_groups=groups)
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, **opts)
    dev = torch.device("cuda:0")
    X = loguniform_rates(f.n, 3, nrhs=4)
    ref = np.stack([fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, X[:, c]) for c in range(4)], axis=1)
    Xd = torch.tensor(X, device=dev)
    Y6 = H.matmat(Xd, mode="x6").cpu().numpy()
    Y3 = H.matmat(Xd, mode="x3").cpu().numpy()
    info = H.info()
    H.close()
    r6, r3 = rel(Y6, ref), rel(Y3, ref)
    say(f"[full] {NAME} ensemble groups {groups}: rel x6 {r6:.3e} x3 {r3:.3e}")
    want = (1, 3) if groups == 3 else (groups, groups)
    assert info["mm_groups"] == {"x3": want, "x6": want}
    # BF16x3 keeps 16 significant bits of each operand (two bf16 parts) and
    # of each stored intermediate value: about 2^-16 = 1.5e-5 per term,
    # averaging down over a sum; 5e-5 bounds it with room (measured 4.5e-6)
    assert r6 <= 2e-5 and r3 <= 5e-5


def test_aca_tolerance_controls_the_product_error():
    """The ACA tolerance of eq. (19) sets the product's error: at N = 30720
    (the benchmark fault at a quarter of its size) and eps from 1e-3 to
    1e-8, the FP64 product (matrix built on the device) stays within 3 eps
    of the exact product, the error falls with eps and the stored entries
    grow — the one-GPU analogue of the paper's tolerance study."""
    import torch

    import paper_2110_12165_amd as hm
    name = "dip30_240x128"
    w = WORKLOADS[name]
    f = config_fault(name)
    x = loguniform_rates(f.n, w["seed"])
    y_exact = fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, x)
    xd = torch.tensor(x, device="cuda:0")
    errs, stored = [], []
    for eps in (1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
        H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, aca_eps=eps, eta=w["eta"], leaf=w["leaf"],
                             lattice=w["lattice"], prec="f64", kernel="split", build_device=1, transpose=0)
        y = H.matvec(xd).cpu().numpy()
        info = H.info()
        H.close()
        errs.append(rel(y, y_exact))
        stored.append((info["dense_entries"] + info["lr_entries"]) / float(f.n) ** 2)
        say(f"[eps] {name} N={f.n} eps {eps:.0e}: rel error {errs[-1]:.2e}, stored {100 * stored[-1]:.2f} %, "
            f"max rank {info['max_rank']}")
        assert errs[-1] <= 3 * eps
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert all(b > a for a, b in zip(stored, stored[1:]))


def test_integration_against_oracle(setup):
    """The benchmark simulation at its own size against the oracle's.  The
    oracle builds its H-matrix (its own tree, partition and ACA; lattice
    block-rows in parallel processes) and integrates 100 accepted steps
    from steady state at the benchmark slip rates with its own step control
    (eqs. 14-16), through the sparse form of its product.  The GPU, on the
    oracle's blocks (hmat_import) in the launch configuration bench.py
    times:
    * replays the oracle's accepted steps (rs_rk45_replay) with FP64
      factors: state and slip within 1e-8 of each component's largest
      magnitude; with FP32 factors within 1e-5 (storage rounding of 3.7e-8
      in every product, carried through the steps), the figure reported;
    * runs its own step control (graph-replayed attempts, FP64 factors):
      the same number of rejected attempts and every accepted step within
      1e-3 of the oracle's (error ratios are differences of nearly equal
      solutions, so the two controllers' choices drift apart by rounding)."""
    torch, hm, bench_options, w, f, x, y_exact = setup
    from _util import oracle_blocks, oracle_build_parallel
    from oracle import friction as fr
    from oracle import rk45
    from oracle.hmatrix import SparseHMatrix
    from synth import friction_params
    n, n_steps = f.n, 100
    p = friction_params(f)
    y0 = fr.initial_state(x, p, p["sigma"])
    say(f"[full] {NAME}: oracle build (parallel lattice rows)")
    H = oracle_build_parallel(NAME)
    Bk = oracle_blocks(H)
    threads = min(16, len(os.sched_getaffinity(0)))
    S = SparseHMatrix(H, threads=threads)
    del H
    calls = [0]

    def apply_A(v):
        calls[0] += 1
        if calls[0] % 120 == 0:
            say(f"    oracle integration: attempt {calls[0] // 6}")
        return S.matvec(v)
    sr = lambda z: fr.slip_rate(z[:n], z[n:2 * n], z[2 * n:], p["a"], p["V0"])  # noqa: E731
    ref = rk45.integrate(lambda z: fr.rhs(z, p, apply_A), y0, 1.0, n_steps, slip_rate=sr)
    S.close()
    del S
    dts = np.array([dt for (_, dt, _, ok) in ref["log"] if ok])
    rej = sum(1 for e in ref["log"] if not e[3])
    say(f"    oracle: {n_steps} steps ({rej} rejected) to t = {ref['t']:.4e} s, dt {dts[0]:.3g} .. {dts[-1]:.3g} s")
    dev = torch.device("cuda:0")
    dp = {k: torch.tensor(p[k], device=dev) for k in ("a", "b", "dc")}
    errs = {}
    for variant in ("batched_f64", "batched_f32"):
        Hg = hm.HMatrix.from_blocks(Bk["n"], Bk["perm"], Bk["desc"], Bk["off"], Bk["values"],
                                    **bench_options(NAME, variant))
        rk = hm.RK45(Hg, None, dp["a"], dp["b"], dp["dc"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
        y = torch.tensor(y0, device=dev)
        D = torch.zeros(n, dtype=torch.float64, device=dev)
        rk.replay(y, D, dts)
        torch.cuda.synchronize()
        yy, DD = y.cpu().numpy(), D.cpu().numpy()
        e_y = max(np.max(np.abs(yy[c * n:(c + 1) * n] - ref["y"][c * n:(c + 1) * n]))
                  / np.max(np.abs(ref["y"][c * n:(c + 1) * n])) for c in range(3))
        errs[variant] = (e_y, np.max(np.abs(DD - ref["D"])) / np.max(np.abs(ref["D"])))
        if variant == "batched_f64":
            # the GPU's own step control from the same state
            y = torch.tensor(y0, device=dev)
            D = torch.zeros(n, dtype=torch.float64, device=dev)
            dt_log = torch.zeros(n_steps, dtype=torch.float64, device=dev)
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                rk.run(y, D, n_steps, use_graph=True, stream=s, dt_log=dt_log)
            s.synchronize()
            drift = float(np.max(np.abs(dt_log.cpu().numpy() - dts) / dts))
            gpu_rej = rk.state.rejected
        Hg.close()
    say(f"    GPU replay of the oracle's steps: FP64 factors state {errs['batched_f64'][0]:.2e} slip "
        f"{errs['batched_f64'][1]:.2e}; FP32 factors state {errs['batched_f32'][0]:.2e} slip "
        f"{errs['batched_f32'][1]:.2e}; GPU step control: {gpu_rej} rejected, steps within {drift:.1e}")
    assert max(errs["batched_f64"]) <= 1e-8
    assert max(errs["batched_f32"]) <= 1e-5
    assert gpu_rej == rej and drift <= 1e-3


@pytest.mark.parametrize("name,lattice", [("dip30_120x64", 32), ("dip30_240x128", 32), ("dip30_960x512", 32),
                                          ("dip30_480x256", 1), ("dip30_480x256", 8)])
def test_sweep_configurations_against_exact_product(setup, name, lattice):
    """The size and lattice sweeps bench.py times (N = 7680 ... 491520 at
    lattice 32, the largest being the maximum size measured; lattice 1, the
    normal H-matrix, and 8 at N = 122880), in their launch configuration
    (device construction, FP32 split schedule), against the oracle's exact
    product of each grid."""
    torch, hm = setup[0], setup[1]
    w = WORKLOADS[name]
    f = config_fault(name)
    say(f"[sweep] {name} N={f.n} lattice {lattice}")
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"],
                         lattice=lattice, prec="f32", kernel="split", transpose=0, build_device=1)
    x = loguniform_rates(f.n, w["seed"])
    y = H.matvec(torch.tensor(x, device=torch.device("cuda:0"))).cpu().numpy()
    H.close()
    torch.cuda.empty_cache()
    r = rel(y, fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, x))
    say(f"    rel vs exact {r:.3e}")
    assert r <= 2e-5
