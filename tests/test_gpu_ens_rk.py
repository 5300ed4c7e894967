"""GPU ensemble integration (rs_ens_rk45_run): many rate-and-state
simulations advanced together, against the FP64 oracle integrating each
member on its own (oracle.friction.rhs, oracle.rk45.integrate) on shared
H-matrix factors.

Members: per-element a - b ~ U[-0.006, 0.004] (b = 0.015) and d_c
log-uniform in [0.005, 0.05] m (synth.ensemble_params), initial states at
steady state at log-uniform slip rates, state variable kicked by
U(-0.05, 0.05).

Tolerances.  One step: the increments y1 - y0 and the slip are linear
combinations of stage derivatives whose product part carries the ensemble
product's error (BF16x6: FP32 storage and FP32-exact operands, ~1e-6
relative; BF16x3: ~5e-6, amplified by cancellation in row sums): 2e-5 and
2e-4 of the largest increment of each component.  The next step depends on
the error estimate, a difference of two solutions (cancellation), so it is
compared at 1e-3.  Several steps: controller decisions identical (counts),
times and states within 1e-3 relative.
"""
import numpy as np
import pytest

from _util import oracle_blocks, say
from oracle import friction as fr
from oracle import rk45
from oracle.greens import CoplanarRectGeometry
from oracle.hmatrix import HMatrix as OracleH
from synth import WORKLOADS, config_fault, ensemble_params, loguniform_rates
from synth.faults import MU, NU

pytestmark = pytest.mark.gpu

M = 8


@pytest.fixture(scope="module")
def case():
    import torch

    import paper_2110_12165_amd as hm
    name = "dip30_48x24"
    w = WORKLOADS[name]
    f = config_fault(name)
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    H = OracleH.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
    Bk = oracle_blocks(H)
    Hg = hm.HMatrix.from_blocks(Bk["n"], Bk["perm"], Bk["desc"], Bk["off"], Bk["values"], prec="f32",
                                kernel="split", max_nrhs=64)
    p = ensemble_params(f, M, 3)
    V = loguniform_rates(f.n, 5, nrhs=M)
    kick = np.random.default_rng(105).uniform(-0.05, 0.05, (f.n, M))
    y0 = np.empty((3, f.n, M))
    members = []
    for r in range(M):
        pr = dict(p, a=p["a"][:, r], b=p["b"][:, r], dc=p["dc"][:, r])
        yr = fr.initial_state(V[:, r], pr, p["sigma"])
        yr[:f.n] += kick[:, r]
        y0[:, :, r] = yr.reshape(3, f.n)
        members.append(pr)
    yield torch, hm, f, H, Hg, p, y0, members
    Hg.close()


def _gpu(torch, hm, Hg, p, y0, n_accept, mode, B=None, dt0=1.0, use_graph=False, split=None):
    dev = torch.device("cuda:0")
    a, b, dc = (torch.tensor(np.ascontiguousarray(p[k]), device=dev) for k in ("a", "b", "dc"))
    ens = hm.EnsembleRK45(Hg, B, a, b, dc, p["V0"], p["f0"], p["eta_rad"], p["V_pl"], mode=mode, dt0=dt0)
    y = torch.tensor(np.ascontiguousarray(y0), device=dev)
    D = torch.zeros(y0.shape[1:], dtype=torch.float64, device=dev)
    s = torch.cuda.Stream() if use_graph else None
    for k in (split or [n_accept]):
        if s is not None:
            with torch.cuda.stream(s):
                ens.run(y, D, k, use_graph=True, stream=s)
            s.synchronize()
        else:
            ens.run(y, D, k, use_graph=False)
    torch.cuda.synchronize()
    return ens, y.cpu().numpy(), D.cpu().numpy()


def _oracle(f, H, pr, y0r, n_accept, dt0=1.0, with_B=False):
    Vf = lambda y: fr.slip_rate(y[:f.n], y[f.n:2 * f.n], y[2 * f.n:], pr["a"], pr["V0"])
    return rk45.integrate(lambda y: fr.rhs(y, pr, H.matvec, H.matvec if with_B else None), y0r, dt0, n_accept,
                          slip_rate=Vf)


@pytest.mark.parametrize("mode,tol", [("x6", 2e-5), ("x3", 2e-4)])
def test_one_step_matches_oracle(case, mode, tol):
    torch, hm, f, H, Hg, p, y0, members = case
    say(f"[ensemble rk45] dip30_48x24, {M} members, one step, {mode}")
    ens, y, D = _gpu(torch, hm, Hg, p, y0, 1, mode, dt0=100.0)
    n = f.n
    for r in range(M):
        ref = _oracle(f, H, members[r], y0[:, :, r].reshape(-1), 1, dt0=100.0)
        assert ens.accepted[r] == 1 and ens.rejected[r] == sum(1 for e in ref["log"] if not e[3])
        dy, dref = (y[:, :, r] - y0[:, :, r]), (ref["y"].reshape(3, n) - y0[:, :, r])
        for c in range(2):        # phi, tau (sigma does not move: B = 0)
            assert np.max(np.abs(dy[c] - dref[c])) <= tol * np.max(np.abs(dref[c])), (r, c)
        assert np.all(y[2, :, r] == y0[2, :, r])
        assert np.max(np.abs(D[:, r] - ref["D"])) <= tol * np.max(np.abs(ref["D"]))
        assert ens.t[r] == pytest.approx(ref["t"], rel=1e-15)
        assert ens.dt[r] == pytest.approx(ref["dt"], rel=1e-3)


def test_normal_stress_path_one_step(case):
    """B = A (sigma evolves) on five members."""
    torch, hm, f, H, Hg, p, y0, members = case
    m5 = {k: (v[:, :5] if isinstance(v, np.ndarray) and v.ndim == 2 else v) for k, v in p.items()}
    ens, y, D = _gpu(torch, hm, Hg, m5, y0[:, :, :5], 1, "x6", B=Hg, dt0=100.0)
    n = f.n
    for r in range(5):
        ref = _oracle(f, H, members[r], y0[:, :, r].reshape(-1), 1, dt0=100.0, with_B=True)
        dy, dref = (y[:, :, r] - y0[:, :, r]), (ref["y"].reshape(3, n) - y0[:, :, r])
        for c in range(3):
            assert np.max(np.abs(dy[c] - dref[c])) <= 2e-5 * np.max(np.abs(dref[c])), (r, c)


def test_several_steps_match_oracle(case):
    torch, hm, f, H, Hg, p, y0, members = case
    say(f"[ensemble rk45] dip30_48x24, {M} members, 15 steps, x6")
    ens, y, D = _gpu(torch, hm, Hg, p, y0, 15, "x6")
    n = f.n
    for r in range(M):
        ref = _oracle(f, H, members[r], y0[:, :, r].reshape(-1), 15)
        yr = ref["y"].reshape(3, n)
        assert ens.accepted[r] == 15
        assert ens.rejected[r] == sum(1 for e in ref["log"] if not e[3])
        assert ens.t[r] == pytest.approx(ref["t"], rel=1e-3)
        for c in range(2):
            assert np.max(np.abs(y[c, :, r] - yr[c])) <= 1e-3 * np.max(np.abs(yr[c] - y0[c, :, r])), (r, c)
        assert np.max(np.abs(D[:, r] - ref["D"])) <= 1e-3 * np.max(np.abs(ref["D"]))


def test_graph_batches_and_direct_agree_bitwise(case):
    torch, hm, f, H, Hg, p, y0, members = case
    e1, y1, D1 = _gpu(torch, hm, Hg, p, y0, 10, "x3")
    e2, y2, D2 = _gpu(torch, hm, Hg, p, y0, 10, "x3", use_graph=True, split=[4, 6])
    assert np.array_equal(y1, y2) and np.array_equal(D1, D2)
    assert np.array_equal(e1.t, e2.t) and np.array_equal(e1.rejected, e2.rejected)
    assert np.all(e1.accepted == 10)


def test_triangle_fault_with_normal_stress_one_step():
    """Curved thrust of 384 triangles with its own shear (A) and normal-stress
    (B) matrices, sigma rising with depth: one step of four members (BF16x6
    ensemble products with A and with B per stage) against the oracle on the
    dense FP64 matrices."""
    import torch

    import paper_2110_12165_amd as hm
    from oracle.triangles import TriangleGeometry
    from synth import config_triangle_fault
    f = config_triangle_fault("thrust_16x12")
    n, m = f.n, 4
    A, B = TriangleGeometry(f.verts, f.slip_dir, MU, NU).blocks(np.arange(n), np.arange(n))
    p = ensemble_params(f, m, 3)
    V = loguniform_rates(n, 5, nrhs=m)
    kick = np.random.default_rng(105).uniform(-0.05, 0.05, (n, m))
    y0 = np.empty((3, n, m))
    members = []
    for r in range(m):
        pr = dict(p, a=p["a"][:, r], b=p["b"][:, r], dc=p["dc"][:, r])
        yr = fr.initial_state(V[:, r], pr, p["sigma"])
        yr[:n] += kick[:, r]
        y0[:, :, r] = yr.reshape(3, n)
        members.append(pr)
    # the oracle's dense matrices as single dense blocks, FP32 storage
    perm = np.arange(n, dtype=np.int32)
    desc = np.array([[0, 0, n, 0, n, 0]], dtype=np.int64)
    HA, HB = (hm.HMatrix.from_blocks(n, perm, desc, np.array([0]), M.T.reshape(-1).copy(), prec="f32",
                                     kernel="split", max_nrhs=64) for M in (A, B))
    ens, y, D = _gpu(torch, hm, HA, p, y0, 1, "x6", B=HB, dt0=100.0)
    HA.close()
    HB.close()
    say(f"[ensemble rk45] thrust_16x12 N={n}, {m} members, A and B, one step: sigma moved by up to "
        f"{np.max(np.abs(y[2] - y0[2])):.3e} Pa")
    for r in range(m):
        pr = members[r]
        Vf = lambda yy: fr.slip_rate(yy[:n], yy[n:2 * n], yy[2 * n:], pr["a"], pr["V0"])
        with np.errstate(over="ignore", invalid="ignore"):   # rejected trial steps may overflow eq. (7)
            ref = rk45.integrate(lambda yy: fr.rhs(yy, pr, lambda v: A @ v, lambda v: B @ v),
                                 y0[:, :, r].reshape(-1), 100.0, 1, slip_rate=Vf)
        assert ens.accepted[r] == 1 and ens.rejected[r] == sum(1 for e in ref["log"] if not e[3])
        assert ens.t[r] == pytest.approx(ref["t"], rel=1e-15)
        dy, dref = (y[:, :, r] - y0[:, :, r]), (ref["y"].reshape(3, n) - y0[:, :, r])
        for c in range(3):
            assert np.max(np.abs(dref[c])) > 0.0
            assert np.max(np.abs(dy[c] - dref[c])) <= 2e-5 * np.max(np.abs(dref[c])), (r, c)
        assert np.max(np.abs(D[:, r] - ref["D"])) <= 2e-5 * np.max(np.abs(ref["D"]))
