"""GPU parity of the ensemble product Y = H X on MFMA (eq. 20 for a block
of members) against the FP64 oracle, on shared factors.

Tolerances from the arithmetic: FP32 storage (unit roundoff 6e-8) and FP32
accumulation on MFMA over up to a few thousand inputs per row:
* BF16x6 (three bf16 parts represent each FP32 operand exactly; the dropped
  cross products are O(2^-24)): relative error <= 2e-5, as the FP32 path;
* BF16x3 (two parts, 16 significant bits: each operand and each stored
  intermediate value within 2^-17 relative, so a term within about
  3 * 2^-17 = 2.3e-5 of its size, and sums of many such terms with mixed
  rounding far closer): relative error <= 5e-5 on log-uniform members; on
  the degenerate sizes with signed members, 4 * 2^-17 times the
  cancellation factor |A| |X| / |A X| of the case.
"""
import numpy as np
import pytest

from _util import oracle_blocks, rel, say
from oracle.greens import CoplanarRectGeometry
from oracle.hmatrix import HMatrix as OracleH
from synth import WORKLOADS, config_fault, loguniform_rates
from synth.faults import MU, NU

pytestmark = pytest.mark.gpu


_oracles = {}


# (workload, schedule: 0 = timed choice, 1 or 2 wave groups per slice forced,
# 3 phase 2 on pairs of row intervals sharing their common inputs)
@pytest.fixture(scope="module", params=[("dip30_150x70", 0), ("dip30_150x70", 1), ("dip30_150x70", 2),
                                        ("dip30_150x70", 3), ("planar64x32", 1), ("planar64x32", 2),
                                        ("planar64x32", 3)],
                ids=lambda p: f"{p[0]}-g{p[1]}")
def case(request):
    import torch

    import paper_2110_12165_amd as hm
    name, groups = request.param
    w = WORKLOADS[name]
    f = config_fault(name)
    if name not in _oracles:
        g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
        H = OracleH.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
        _oracles[name] = (H, oracle_blocks(H))
    H, B = _oracles[name]
    Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec="f32", kernel="split",
                                wg_waves=8, wg_waves_p1=4, max_nrhs=64, mm_groups=groups)
    mg = Hg.info()["mm_groups"]
    say(f"[ensemble] {name} wave groups {mg}")
    if groups:
        want = (1, 3) if groups == 3 else (groups, groups)
        assert mg == {"x3": want, "x6": want}
    else:
        assert all(m[0] in (1, 2) and m[1] in (1, 2, 3) for m in mg.values())
    yield torch, hm, f"{name}-g{groups}", f, H, Hg
    Hg.close()


# BF16x3 keeps 16 significant bits of each operand and of each stored
# intermediate value (two bf16 parts: relative error <= 2^-17 each), so a
# term carries at most ~3 * 2^-17 = 2.3e-5 of its size and a sum of many
# terms of mixed rounding far less: 5e-5 bounds it (measured 3e-6 to 5e-6).
@pytest.mark.parametrize("mode,tol", [("x6", 2e-5), ("x3", 5e-5)])
def test_ensemble_parity(case, mode, tol):
    torch, hm, name, f, H, Hg = case
    dev = torch.device("cuda:0")
    X = loguniform_rates(f.n, 3, nrhs=64)
    ref = H.matvec(X)
    Y = Hg.matmat(torch.tensor(X, device=dev), mode=mode).cpu().numpy()
    r = rel(Y, ref)
    say(f"[ensemble] {name} N={f.n} {mode}: rel {r:.3e}")
    assert r <= tol
    # every member separately within the same bound
    per = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert per.max() <= 2 * tol


def test_ensemble_partial_groups_alpha_beta(case):
    torch, hm, name, f, H, Hg = case
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(8)
    for k in (1, 5, 70):
        X = rng.standard_normal((f.n, k))
        Y0 = rng.standard_normal((f.n, k))
        Y = torch.tensor(Y0, device=dev)
        Hg.matmat(torch.tensor(X, device=dev), Y=Y, alpha=-0.5, beta=2.0, mode="x6")
        ref = -0.5 * H.matvec(X) + 2.0 * Y0
        assert rel(Y.cpu().numpy(), ref) <= 2e-5, k


def test_ensemble_matches_single_vector_products(case):
    torch, hm, name, f, H, Hg = case
    dev = torch.device("cuda:0")
    X = torch.tensor(loguniform_rates(f.n, 4, nrhs=16), device=dev)
    Ym = Hg.matmat(X, mode="x6").cpu().numpy()
    Yv = np.stack([Hg.matvec(X[:, c].contiguous()).cpu().numpy() for c in range(16)], axis=1)
    assert rel(Ym, Yv) <= 2e-5


@pytest.mark.parametrize("groups", [0, 1, 2, 3])
def test_ensemble_degenerate_sizes(groups):
    """Tiny meshes (one element, no low-rank block, a single leaf) and a
    matrix of zeros (the normal component of a planar fault): the ensemble
    product against the dense oracle matrix, and beta * Y kept."""
    import torch

    import paper_2110_12165_amd as hm
    from oracle.dense import dense_matrix
    from synth import planar_rect_fault
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(17)
    for nx, ny, leaf in ((1, 1, 4), (2, 1, 4), (3, 2, 1), (5, 3, 64)):
        f = planar_rect_fault(nx, ny, 100.0, 90.0, "strike")
        A = dense_matrix(CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU))
        Hg = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, leaf=leaf, prec="f32", kernel="split", max_nrhs=64,
                              mm_groups=groups)
        X = rng.standard_normal((f.n, 3))
        # few terms per row and signed members: the BF16x3 bound per term
        # (3 * 2^-17) times the cancellation in A X, with room
        kappa = np.linalg.norm(np.abs(A) @ np.abs(X)) / np.linalg.norm(A @ X)
        for mode, tol in (("x6", 2e-5), ("x3", 4 * 2.0 ** -17 * kappa)):
            Y = Hg.matmat(torch.tensor(X, device=dev), mode=mode).cpu().numpy()
            assert rel(Y, A @ X) <= tol, (nx, ny, leaf, mode)
        Hg.close()
    f = planar_rect_fault(16, 8, 100.0, 90.0, "strike")
    Hb = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, component=1, leaf=8, lattice=2, prec="f32", kernel="split",
                          max_nrhs=64, mm_groups=groups)
    Y0 = torch.tensor(rng.standard_normal((f.n, 5)), device=dev)
    Y = Y0.clone()
    Hb.matmat(torch.ones((f.n, 5), dtype=torch.float64, device=dev), Y=Y, alpha=1.0, beta=2.0, mode="x6")
    assert torch.equal(Y, 2.0 * Y0)
    Hb.close()


def test_autotune_keeps_the_ensemble_product():
    """hmat_autotune on a handle with ensemble buffers re-lays it out and
    re-times the wave groups; the ensemble product still agrees with the
    single-vector products on the new layout."""
    import torch

    import paper_2110_12165_amd as hm
    name = "dip30_150x70"
    w = WORKLOADS[name]
    f = config_fault(name)
    Hg = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"],
                          lattice=w["lattice"], prec="f32", kernel="split", max_nrhs=64)
    info = Hg.autotune(reps=3)
    say(f"[ensemble] autotune picked {info['kernel']} {info['wg_waves']}/{info['wg_waves_p1']}, "
        f"wave groups {info['mm_groups']}")
    assert info["kernel"] in ("split", "persistent")
    assert all(m[0] in (1, 2) and m[1] in (1, 2, 3) for m in info["mm_groups"].values())
    dev = torch.device("cuda:0")
    X = torch.tensor(loguniform_rates(f.n, 6, nrhs=16), device=dev)
    Ym = Hg.matmat(X, mode="x6").cpu().numpy()
    Yv = np.stack([Hg.matvec(X[:, c].contiguous()).cpu().numpy() for c in range(16)], axis=1)
    Hg.close()
    assert rel(Ym, Yv) <= 2e-5
