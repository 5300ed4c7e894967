"""GPU discrete adjoint of the frozen-step integration (rs_rk45_replay /
rs_rk45_adjoint) against the FP64 oracle adjoint (oracle.adjoint, itself
pinned by complex-step derivatives and finite differences), and against
central finite differences of the GPU forward map at the size of the
paper-scale ensemble mesh.

Loss: L = 1/2 |D_M - D_target|^2, D_target from a perturbed by
U(-1e-3, 1e-3) (seed 4): on the same frozen steps for the small case, by
its own controlled integration to the same final time for the paper-scale
case; gradients for a (b fixed: also the gradient for a - b), d_c and the
initial state.

Gradient checks of the benchmark's kind (curved thrust with A and B): the
oracle integrates with its own step control and its own target, the GPU
replays the oracle's steps on the same blocks.  The window is the 80 steps
before the first event (CONFIG4_WINDOW, with the measurements that set
it): on 384 triangles with everything the oracle's own, on 1920 triangles
and on the 21000-triangle mesh of the benchmark with the library's FP64
blocks, the last plus central differences for 20 elements of seed 4.

Tolerances.  Shared FP64 factors: the products agree with the oracle's to
1e-13 and the element-wise functions to a few ulp; over 20 steps the
trajectories agree to ~1e-10, and the gradients (a smooth function of the
trajectory) are compared at 1e-7 of their largest entry.  FP32-stored
factors change the operator by ~1e-7 relative, which the gradients inherit:
1e-4.  Finite differences (h = 1e-6 on a and d_c, central): truncation
O(h^2) and cancellation ~1e-16 L / h, compared at 1e-4 relative plus 1e-6 of
the largest entry.
"""
import os

import numpy as np
import pytest

from _util import oracle_blocks, oracle_triangle_matrices, rel, say
from oracle import adjoint as adj
from oracle import friction as fr
from oracle import rk45
from oracle.greens import CoplanarRectGeometry
from oracle.hmatrix import HMatrix as OracleH
from synth import WORKLOADS, config_fault, friction_params, loguniform_rates
from synth.faults import MU, NU

pytestmark = pytest.mark.gpu

N_STEPS = 20
CKPT = 7            # 20 steps = segments of 7, 7 and 6


def _state(f, p, seed, kick=0.05):
    y = fr.initial_state(loguniform_rates(f.n, seed), p, p["sigma"])
    y[:f.n] += np.random.default_rng(100 + seed).uniform(-kick, kick, f.n)
    return y


@pytest.fixture(scope="module")
def small():
    import torch

    import paper_2110_12165_amd as hm
    name = "dip30_48x24"
    w = WORKLOADS[name]
    f = config_fault(name)
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    H = OracleH.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
    p = friction_params(f)
    dev = torch.device("cuda:0")
    Bk = oracle_blocks(H)
    hg = {prec: hm.HMatrix.from_blocks(Bk["n"], Bk["perm"], Bk["desc"], Bk["off"], Bk["values"], prec=prec,
                                       kernel="split")
          for prec in ("f64", "f32")}
    dp = {k: torch.tensor(p[k], device=dev) for k in ("a", "b", "dc")}
    y0 = _state(f, p, 0)
    Vfun = lambda y: fr.slip_rate(y[:f.n], y[f.n:2 * f.n], y[2 * f.n:], p["a"], p["V0"])
    out = {}
    for with_B in (False, True):
        apply_B = H.matvec if with_B else None
        run = rk45.integrate(lambda y: fr.rhs(y, p, H.matvec, apply_B), y0, 1.0, N_STEPS, slip_rate=Vfun)
        dts = [dt for (_, dt, _, ok) in run["log"] if ok]
        pt = dict(p, a=p["a"] + np.random.default_rng(4).uniform(-1e-3, 1e-3, f.n))
        D_t = adj.replay(pt, H.matvec, apply_B, y0, dts)[2]
        ref = adj.slip_misfit_gradient(p, H.matvec, H.matvec_T, y0, dts, D_t, apply_B,
                                       H.matvec_T if with_B else None)
        D_ref = adj.replay(p, H.matvec, apply_B, y0, dts)[2]
        out[with_B] = dict(dts=dts, D_t=D_t, ref=ref, D_ref=D_ref)
    yield torch, hm, f, p, hg, dp, y0, out
    for h in hg.values():
        h.close()


def _gpu_gradient(torch, hm, Hg, with_B, p, dp, y0, dts, D_t, ckpt_every=CKPT):
    dev = dp["a"].device
    rk = hm.RK45(Hg, Hg if with_B else None, dp["a"], dp["b"], dp["dc"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    y = torch.tensor(y0, device=dev)
    D = torch.zeros(len(y0) // 3, dtype=torch.float64, device=dev)
    ckpt = rk.replay(y, D, dts, ckpt_every=ckpt_every)
    Dbar = D - torch.tensor(D_t, device=dev)
    ybar = torch.zeros_like(y)
    _, ga, gdc = rk.adjoint(ckpt, dts, ckpt_every, ybar, Dbar)
    torch.cuda.synchronize()
    L = 0.5 * float((Dbar * Dbar).sum())
    return L, ga.cpu().numpy(), gdc.cpu().numpy(), ybar.cpu().numpy(), D.cpu().numpy()


def _close(got, want):
    return float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


@pytest.mark.parametrize("with_B", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_matches_oracle(small, prec, with_B):
    torch, hm, f, p, hg, dp, y0, out = small
    say(f"[adjoint vs oracle] dip30_48x24 {prec} B={'A' if with_B else 0}, {N_STEPS} steps, ckpt {CKPT}")
    o = out[with_B]
    L, ga, gdc, gy, D = _gpu_gradient(torch, hm, hg[prec], with_B, p, dp, y0, o["dts"], o["D_t"])
    Lr, ga_r, gdc_r, gy_r = o["ref"]
    tol = 1e-7 if prec == "f64" else 1e-4
    n = f.n
    errs = dict(D=rel(D, o["D_ref"]), a=_close(ga, ga_r), dc=_close(gdc, gdc_r),
                phi=_close(gy[:n], gy_r[:n]), tau=_close(gy[n:2 * n], gy_r[n:2 * n]))
    if with_B:
        errs["sigma"] = _close(gy[2 * n:], gy_r[2 * n:])
    say("   max error / max entry:", {k: f"{v:.2e}" for k, v in errs.items()})
    assert L == pytest.approx(Lr, rel=100 * tol)
    for k, v in errs.items():
        assert v <= tol, k


def test_checkpoint_interval_does_not_change_the_gradient(small):
    torch, hm, f, p, hg, dp, y0, out = small
    o = out[False]
    r1 = _gpu_gradient(torch, hm, hg["f64"], False, p, dp, y0, o["dts"], o["D_t"], ckpt_every=1)
    r2 = _gpu_gradient(torch, hm, hg["f64"], False, p, dp, y0, o["dts"], o["D_t"], ckpt_every=50)
    for a, b in zip(r1[1:4], r2[1:4]):
        np.testing.assert_array_equal(a, b)


def test_replay_reproduces_the_controlled_run(small):
    """rs_rk45_run's step log replayed by rs_rk45_replay gives the same state
    and slip, bit for bit (same stage and update arithmetic)."""
    torch, hm, f, p, hg, dp, y0, out = small
    dev = dp["a"].device
    rk = hm.RK45(hg["f64"], None, dp["a"], dp["b"], dp["dc"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    y = torch.tensor(y0, device=dev)
    D = torch.zeros(f.n, dtype=torch.float64, device=dev)
    log = torch.zeros(30, dtype=torch.float64, device=dev)
    rk.run(y, D, 30, use_graph=False, dt_log=log)
    assert rk.state.rejected >= 0 and rk.state.accepted == 30
    y2 = torch.tensor(y0, device=dev)
    D2 = torch.zeros_like(D)
    rk.replay(y2, D2, log.cpu().numpy())
    torch.cuda.synchronize()
    assert torch.equal(y, y2) and torch.equal(D, D2)
    assert rk.t == pytest.approx(float(log.sum()), rel=1e-14)


def test_autograd_function(small):
    torch, hm, f, p, hg, dp, y0, out = small
    from paper_2110_12165_amd.autograd import rk45_replay
    o = out[False]
    a = dp["a"].clone().requires_grad_(True)
    dc = dp["dc"].clone().requires_grad_(True)
    y0t = torch.tensor(y0, device=a.device, requires_grad=True)
    yM, DM = rk45_replay(hg["f64"], None, a, dp["b"], dc, y0t, o["dts"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"],
                         ckpt_every=CKPT)
    D_t = torch.tensor(o["D_t"], device=a.device)
    loss = 0.5 * ((DM - D_t) ** 2).sum() + 1e-3 * yM[f.n:2 * f.n].sum() / 1e6
    loss.backward()
    Lr, ga_r, gdc_r, gy_r = o["ref"]
    # the y_M term adds the adjoint of <c, y_M>: the library's adjoint with
    # D_bar = 0 and y_bar = c, subtracted, leaves the oracle's slip gradient
    rk = hm.RK45(hg["f64"], None, dp["a"], dp["b"], dp["dc"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    y = torch.tensor(y0, device=a.device)
    ckpt = rk.replay(y, None, o["dts"], ckpt_every=CKPT)
    c = torch.zeros(3 * f.n, dtype=torch.float64, device=a.device)
    c[f.n:2 * f.n] = 1e-3 / 1e6
    _, ga_c, gdc_c = rk.adjoint(ckpt, o["dts"], CKPT, c.clone())
    tol = 1e-7
    assert _close(a.grad.cpu().numpy() - ga_c.cpu().numpy(), ga_r) <= tol
    assert _close(dc.grad.cpu().numpy() - gdc_c.cpu().numpy(), gdc_r) <= tol


def _target_at(hm, Hg, p, a, b, dc, y0, T, HB=None):
    """Slip at time T of the controlled integration with parameters (a, b,
    dc): steps while they end before T, then one forced step to T."""
    import torch
    rk = hm.RK45(Hg, HB, a, b, dc, p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    y = torch.tensor(y0, device=a.device)
    D = torch.zeros(len(y0) // 3, dtype=torch.float64, device=a.device)
    while rk.t + rk.dt < T:
        rk.step(y, D)
    rk.dt = T - rk.t
    rk.attempt(y, D, force=1)
    return D, rk.state.accepted


WINDOW = 80   # steps of the controlled run before nucleation (slip rates stay below 1e-8 m/s)


@pytest.fixture(scope="module")
def paper_scale():
    """N = 21000 planar stand-in of the paper-scale mesh, FP32 factors, built
    by the library; the first WINDOW steps of the controlled run from a kicked
    steady state, their steps logged.  Later steps of this run nucleate and
    host a seismic event, through which the final slip is so sensitive to a
    (gradients ~1e10) that a central difference of one element's a by 1e-6
    already leaves the frozen steps' stability region.  The target slip comes
    from the perturbed a at the same final time, by its own controlled
    integration: the frozen steps of the base run sit at the explicit
    stability limit, which a 10 % change of a moves."""
    import torch

    import paper_2110_12165_amd as hm
    name = "dip30_150x140"
    w = WORKLOADS[name]
    f = config_fault(name)
    p = friction_params(f)
    dev = torch.device("cuda:0")
    Hg = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"],
                          lattice=w["lattice"], prec="f32", kernel="split")
    dp = {k: torch.tensor(p[k], device=dev) for k in ("a", "b", "dc")}
    y0 = _state(f, p, 3)
    rk = hm.RK45(Hg, None, dp["a"], dp["b"], dp["dc"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    y = torch.tensor(y0, device=dev)
    D = torch.zeros(f.n, dtype=torch.float64, device=dev)
    log = torch.zeros(WINDOW, dtype=torch.float64, device=dev)
    rk.run(y, D, WINDOW, use_graph=False, dt_log=log)
    dts = log.cpu().numpy()
    n = f.n
    yn = y.cpu().numpy()
    vmax = float(np.max(fr.slip_rate(yn[:n], yn[n:2 * n], yn[2 * n:], p["a"], p["V0"])))
    at = dp["a"] + torch.tensor(np.random.default_rng(4).uniform(-1e-3, 1e-3, n), device=dev)
    D_t, steps_t = _target_at(hm, Hg, p, at, dp["b"], dp["dc"], y0, rk.t)
    say(f"[paper scale] N={n}, {WINDOW} steps to t={rk.t:.4e} s ({rk.state.rejected} rejected), largest slip "
        f"{float(D.max()):.3e} m, largest slip rate {vmax:.2e} m/s; target: {steps_t} steps, "
        f"largest slip {float(D_t.max()):.3e} m")
    assert vmax < 1e-8 and torch.isfinite(D_t).all()
    yield torch, hm, f, p, Hg, dp, y0, dts, D_t
    Hg.close()


def test_adjoint_against_central_differences_paper_scale(paper_scale):
    torch, hm, f, p, Hg, dp, y0, dts, D_t = paper_scale
    dev = dp["a"].device
    say(f"[adjoint vs FD] dip30_150x140 f32, {WINDOW} steps, ckpt 50, 20 elements")
    rk = hm.RK45(Hg, None, dp["a"], dp["b"], dp["dc"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    y = torch.tensor(y0, device=dev)
    D = torch.zeros(f.n, dtype=torch.float64, device=dev)
    ckpt = rk.replay(y, D, dts, ckpt_every=50)
    Dbar = D - D_t
    _, ga, gdc = rk.adjoint(ckpt, dts, 50, torch.zeros_like(y), Dbar)
    ga, gdc = ga.cpu().numpy(), gdc.cpu().numpy()

    def loss(a, dc):
        r = hm.RK45(Hg, None, a, dp["b"], dc, p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
        yy = torch.tensor(y0, device=dev)
        DD = torch.zeros(f.n, dtype=torch.float64, device=dev)
        r.replay(yy, DD, dts)
        return 0.5 * float(((DD - D_t) ** 2).sum())

    h = 1e-6
    idx = np.random.default_rng(4).choice(f.n, 20, replace=False)
    worst = 0.0
    for key, g in (("a", ga), ("dc", gdc)):
        scale = np.max(np.abs(g))
        for i in idx:
            tp, tm = dp[key].clone(), dp[key].clone()
            tp[i] += h
            tm[i] -= h
            args_p = (tp, dp["dc"]) if key == "a" else (dp["a"], tp)
            args_m = (tm, dp["dc"]) if key == "a" else (dp["a"], tm)
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            err = abs(fd - g[i]) / (abs(g[i]) + 1e-2 * scale)
            worst = max(worst, err)
            say(f"   {key}[{int(i)}]: adjoint {g[i]: .6e}  central difference {fd: .6e}")
            assert abs(fd - g[i]) <= 1e-4 * abs(g[i]) + 1e-6 * scale, (key, int(i), fd, g[i])
    say(f"   worst FD mismatch (relative): {worst:.2e}")


class _DenseGeom:
    """A dense matrix seen through the interface the oracle's H-matrix
    construction reads (centres for the tree, entries on demand)."""

    def __init__(self, centres, M):
        self.centres, self.M = centres, M

    def block(self, rows, cols):
        return self.M[np.ix_(rows, cols)]

    def entry_row(self, i, cols):
        return self.M[i, cols]

    def entry_col(self, rows, j):
        return self.M[rows, j]


def _oracle_slip_at(p, A, B, y0, T):
    """Slip at time T of the oracle's controlled integration: each trial
    step is the controller's (eqs. 14-15) cut to end at T at the latest,
    and every attempt, the last one too, passes the error test."""
    n = len(y0) // 3
    f = lambda y: fr.rhs(y, p, A, B)  # noqa: E731
    V = lambda y: fr.slip_rate(y[:n], y[n:2 * n], y[2 * n:], p["a"], p["V0"])  # noqa: E731
    y, D, t, dt = np.array(y0), np.zeros(n), 0.0, 1.0
    while True:
        last = t + dt >= T
        h = T - t if last else dt
        y5, y4, _, _ = rk45.attempt(f, y, h)
        r = rk45.error_ratio(y5, y4)
        ok = bool(np.isfinite(r) and r <= 1.0)
        if ok:
            D = D + 0.5 * h * (V(y) + V(y5))                                   # eq. (16)
            y, t = y5, t + h
            if last:
                return D
        dt = rk45.next_dt(h, r, ok)


def _oracle_gradient_case(p, ops, y0, n_steps):
    """The oracle's side of a gradient check on a fault with A and B: its
    controlled run of n_steps accepted steps from y0; the target slip from
    a + U(-1e-3, 1e-3) (seed 4) by its own controlled run to the same final
    time; its discrete adjoint on the frozen steps.  ops = (A, A^T, B, B^T)
    products.  Returns (dts, D_target, (L, dL/da, dL/d d_c, dL/dy0), D_M)."""
    A, AT, B, BT = ops
    n = len(y0) // 3
    V = lambda y: fr.slip_rate(y[:n], y[n:2 * n], y[2 * n:], p["a"], p["V0"])  # noqa: E731
    with np.errstate(over="ignore", invalid="ignore"):
        run = rk45.integrate(lambda y: fr.rhs(y, p, A, B), y0, 1.0, n_steps, slip_rate=V)
        dts = [dt for (_, dt, _, ok) in run["log"] if ok]
        pt = dict(p, a=p["a"] + np.random.default_rng(4).uniform(-1e-3, 1e-3, n))
        D_t = _oracle_slip_at(pt, A, B, y0, run["t"])
    ref = adj.slip_misfit_gradient(p, A, AT, y0, dts, D_t, B, BT)
    return dts, D_t, ref, run["D"]


def _gpu_gradient_ab(torch, hm, HA, HB, p, dp, y0, dts, D_t, ckpt_every=50):
    dev = dp["a"].device
    rk = hm.RK45(HA, HB, dp["a"], dp["b"], dp["dc"], p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
    y = torch.tensor(y0, device=dev)
    D = torch.zeros(len(y0) // 3, dtype=torch.float64, device=dev)
    ckpt = rk.replay(y, D, dts, ckpt_every=ckpt_every)
    Dbar = D - torch.tensor(D_t, device=dev)
    ybar = torch.zeros_like(y)
    _, ga, gdc = rk.adjoint(ckpt, dts, ckpt_every, ybar, Dbar)
    torch.cuda.synchronize()
    return 0.5 * float((Dbar * Dbar).sum()), ga.cpu().numpy(), gdc.cpu().numpy(), ybar.cpu().numpy(), D.cpu().numpy()


def _gradient_errors(n, got, ref, D_ref):
    L, ga, gdc, gy, D = got
    Lr, ga_r, gdc_r, gy_r = ref
    return dict(L=abs(L - Lr) / Lr, D=rel(D, D_ref), a=_close(ga, ga_r), dc=_close(gdc, gdc_r),
                phi=_close(gy[:n], gy_r[:n]), tau=_close(gy[n:2 * n], gy_r[n:2 * n]),
                sigma=_close(gy[2 * n:], gy_r[2 * n:]))


def _thrust_state(f, p, seed=3):
    y0 = fr.initial_state(loguniform_rates(f.n, seed), p, p["sigma"])
    y0[:f.n] += np.random.default_rng(100 + seed).uniform(-0.05, 0.05, f.n)
    return y0


# Window of a gradient check on the curved thrust: the 80 steps before the
# first event.  Through an event the final slip is so sensitive to the
# parameters that no two correct computations agree: on 1920 triangles the
# oracle's own gradient with its block-loop product and with its sparse
# product (the same blocks, sums in another order) differ by 1.2e-10 of the
# largest entry after 80 steps and by 5e-7 after 120 (the first event, slip
# rates up to 8e-2 m/s), and FP32-rounded factors move it by 1.4e-4 and by
# 2.3 (230 %); on 384 triangles by 1e-10 after 80 steps, 4e-8 after 100,
# 1.5e-2 after 200.
CONFIG4_WINDOW = 80


def test_adjoint_window_oracle_matrices():
    """The gradient window on a curved thrust of 384 triangles, everything
    on the oracle's side its own: dense A and B by its cubature, its
    H-matrix of them (tree, partition, ACA), its controlled run, target and
    adjoint.  The GPU takes the oracle's blocks (FP64 storage) and steps and
    must give the oracle's gradients to 1e-7 of their largest entry."""
    import torch

    import paper_2110_12165_amd as hm
    from synth import TRIANGLE_WORKLOADS, config_triangle_fault, triangle_friction_params
    name = "thrust_16x12"
    w = TRIANGLE_WORKLOADS[name]
    f = config_triangle_fault(name)
    n = f.n
    p = triangle_friction_params(f)
    say(f"[adjoint vs oracle] {name} N={n}: oracle cubature of A and B")
    A, B = oracle_triangle_matrices(f.verts, f.slip_dir)
    centres = f.verts.sum(axis=1) / 3.0
    HA = OracleH.build(_DenseGeom(centres, A), w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
    HB = OracleH.build(_DenseGeom(centres, B), w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
    y0 = _thrust_state(f, p)
    dts, D_t, ref, D_ref = _oracle_gradient_case(p, (HA.matvec, HA.matvec_T, HB.matvec, HB.matvec_T), y0,
                                                 CONFIG4_WINDOW)
    dev = torch.device("cuda:0")
    dp = {k: torch.tensor(p[k], device=dev) for k in ("a", "b", "dc")}
    ga, gb = oracle_blocks(HA), oracle_blocks(HB)
    GA = hm.HMatrix.from_blocks(ga["n"], ga["perm"], ga["desc"], ga["off"], ga["values"], prec="f64", kernel="split")
    GB = hm.HMatrix.from_blocks(gb["n"], gb["perm"], gb["desc"], gb["off"], gb["values"], prec="f64", kernel="split")
    errs = _gradient_errors(n, _gpu_gradient_ab(torch, hm, GA, GB, p, dp, y0, dts, D_t), ref, D_ref)
    GA.close()
    GB.close()
    say(f"   {len(dts)} steps to t = {sum(dts):.4e} s; max error / max entry:",
        {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= 1e-7, k


@pytest.fixture(scope="module")
def exported_thrust():
    """Curved thrust meshes with the library's FP64 blocks (host build) read
    by the oracle through hmat_export: the oracle's cubature of every entry
    at these sizes takes CPU hours, and the library's entries are pinned to
    it separately (3e-15 of the largest entry at N = 1920, rows at
    N = 21000)."""
    import torch

    import paper_2110_12165_amd as hm
    from oracle.hmatrix import SparseHMatrix
    from synth import TRIANGLE_WORKLOADS, config_triangle_fault, triangle_friction_params
    cache = {}

    def get(name):
        if name not in cache:
            w = TRIANGLE_WORKLOADS[name]
            f = config_triangle_fault(name)
            opts = dict(aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"], kernel="split")
            gpu, ops, sparse = {}, [], []
            for c in (0, 1):
                H64 = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=c, prec="f64", **opts)
                e = H64.export()
                H32 = hm.HMatrix.from_blocks(e["n"], e["perm"], e["desc"].reshape(-1), e["off"], e["values"],
                                             prec="f32", **opts)
                S = SparseHMatrix(OracleH.from_arrays(e["n"], e["perm"], e["desc"], e["off"], e["values"]),
                                  threads=min(16, len(os.sched_getaffinity(0))))
                gpu[c] = (H64, H32)
                ops += [S.matvec, S.matvec_T]
                sparse.append(S)
            cache[name] = (f, triangle_friction_params(f), gpu, tuple(ops), sparse)
        return cache[name][:4]
    dev = torch.device("cuda:0")
    yield torch, hm, dev, get
    for f, p, gpu, ops, sparse in cache.values():
        for H64, H32 in gpu.values():
            H64.close()
            H32.close()
        for S in sparse:
            S.close()


def test_adjoint_window_exported_blocks(exported_thrust):
    """The gradient window on the curved thrust of 1920 triangles: the
    oracle's controlled run, target and adjoint on the library's FP64
    blocks, the GPU's gradient on the oracle's steps and target with FP64
    storage (1e-7 of the largest entry) and FP32 storage (1e-3: rounding the
    factors to FP32 moves the oracle's own gradient by 1.4e-4)."""
    torch, hm, dev, get = exported_thrust
    f, p, gpu, ops = get("thrust_40x24")
    n = f.n
    y0 = _thrust_state(f, p)
    say(f"[adjoint vs oracle] thrust_40x24 N={n}, {CONFIG4_WINDOW} steps, A and B")
    dts, D_t, ref, D_ref = _oracle_gradient_case(p, ops, y0, CONFIG4_WINDOW)
    dp = {k: torch.tensor(p[k], device=dev) for k in ("a", "b", "dc")}
    for prec, k, tol in (("f64", 0, 1e-7), ("f32", 1, 1e-3)):
        errs = _gradient_errors(n, _gpu_gradient_ab(torch, hm, gpu[0][k], gpu[1][k], p, dp, y0, dts, D_t), ref,
                                D_ref)
        say(f"   {prec}: {len(dts)} steps to t = {sum(dts):.4e} s; max error / max entry:",
            {kk: f"{v:.2e}" for kk, v in errs.items()})
        for kk, v in errs.items():
            assert v <= tol, (prec, kk)


def test_adjoint_paper_scale_triangles(exported_thrust):
    """The curved thrust of 21000 triangles (the gradient benchmark's mesh)
    over the WINDOW steps before nucleation: the oracle's controlled run,
    target and adjoint on the library's FP64 blocks against the GPU's
    gradient on the oracle's steps and target (FP64 storage 1e-7, FP32
    storage 1e-4 of the largest entry); then the FP32 gradient against
    central differences of the GPU's replay for 20 elements of seed 4
    (h = 1e-6)."""
    torch, hm, dev, get = exported_thrust
    f, p, gpu, ops = get("thrust_150x70")
    n = f.n
    y0 = _thrust_state(f, p)
    say(f"[adjoint vs oracle] thrust_150x70 N={n}, {WINDOW} steps, A and B")
    dts, D_t, ref, D_ref = _oracle_gradient_case(p, ops, y0, WINDOW)
    dp = {k: torch.tensor(p[k], device=dev) for k in ("a", "b", "dc")}
    got32 = None
    for prec, k, tol in (("f64", 0, 1e-7), ("f32", 1, 1e-4)):
        got = _gpu_gradient_ab(torch, hm, gpu[0][k], gpu[1][k], p, dp, y0, dts, D_t)
        errs = _gradient_errors(n, got, ref, D_ref)
        say(f"   {prec}: {len(dts)} steps to t = {sum(dts):.4e} s; max error / max entry:",
            {kk: f"{v:.2e}" for kk, v in errs.items()})
        for kk, v in errs.items():
            assert v <= tol, (prec, kk)
        got32 = got
    HA, HB = gpu[0][1], gpu[1][1]
    _, ga, gdc = got32[:3]
    D_td = torch.tensor(D_t, device=dev)

    def loss(a, dc):
        r = hm.RK45(HA, HB, a, dp["b"], dc, p["V0"], p["f0"], p["eta_rad"], p["V_pl"])
        yy = torch.tensor(y0, device=dev)
        DD = torch.zeros(n, dtype=torch.float64, device=dev)
        r.replay(yy, DD, dts)
        return 0.5 * float(((DD - D_td) ** 2).sum())

    h = 1e-6
    idx = np.random.default_rng(4).choice(n, 20, replace=False)
    worst = 0.0
    for key, g in (("a", ga), ("dc", gdc)):
        scale = np.max(np.abs(g))
        for i in idx:
            tp, tm = dp[key].clone(), dp[key].clone()
            tp[i] += h
            tm[i] -= h
            args_p = (tp, dp["dc"]) if key == "a" else (dp["a"], tp)
            args_m = (tm, dp["dc"]) if key == "a" else (dp["a"], tm)
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            worst = max(worst, abs(fd - g[i]) / (abs(g[i]) + 1e-2 * scale))
            assert abs(fd - g[i]) <= 1e-4 * abs(g[i]) + 1e-6 * scale, (key, int(i), fd, g[i])
    say(f"   FP32 gradient vs central differences, 20 elements (seed 4): worst {worst:.2e}")
