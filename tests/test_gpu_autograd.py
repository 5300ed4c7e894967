"""Transpose product and autograd backward against the oracle (eq. 20 and
its transpose, shared factors).  The product is linear, so the gradient of
<w, H x> with respect to x is exactly H^T w."""
import numpy as np
import pytest

from _util import oracle_blocks, rel, say
from oracle.greens import CoplanarRectGeometry
from oracle.hmatrix import HMatrix as OracleH
from synth import WORKLOADS, config_fault, loguniform_rates
from synth.faults import MU, NU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    import torch

    import paper_2110_12165_amd as hm
    name = "dip30_150x70"
    w = WORKLOADS[name]
    f = config_fault(name)
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    H = OracleH.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
    return torch, hm, f, H, oracle_blocks(H)


@pytest.mark.parametrize("kernel,prec,tol", [("split", "f64", 1e-13), ("persistent", "f64", 1e-13),
                                             ("split", "f32", 2e-5), ("plain", "f64", 1e-13)])
def test_backward_is_transpose_product(case, kernel, prec, tol):
    torch, hm, f, H, B = case
    from paper_2110_12165_amd.autograd import hmatvec
    say(f"[autograd] dip30_150x70 {kernel} {prec}")
    Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec=prec, kernel=kernel)
    dev = torch.device("cuda:0")
    x = torch.tensor(loguniform_rates(f.n, 7), device=dev, requires_grad=True)
    wv = np.random.default_rng(9).standard_normal(f.n)
    y = hmatvec(Hg, x)
    loss = (torch.tensor(wv, device=dev) * y).sum()
    loss.backward()
    assert rel(y.detach().cpu().numpy(), H.matvec(x.detach().cpu().numpy())) <= tol
    assert rel(x.grad.cpu().numpy(), H.matvec_T(wv)) <= tol
    Hg.close()


def test_gradcheck_small(case):
    torch, hm, f, H, B = case
    from paper_2110_12165_amd.autograd import hmatvec
    from synth import planar_rect_fault
    small = planar_rect_fault(12, 6, 100.0, 30.0, "dip")
    Hs = hm.HMatrix.build(small.verts, small.slip_dir, MU, NU, leaf=8, lattice=2, kernel="split")
    x = torch.randn(small.n, dtype=torch.float64, device="cuda:0", requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: hmatvec(Hs, v) * 1e-9, (x,), eps=1e-3, atol=1e-9, rtol=1e-6)
    Hs.close()


def test_transpose_requires_layout(case):
    torch, hm, f, H, B = case
    Hg = hm.HMatrix.from_blocks(B["n"], B["perm"], B["desc"], B["off"], B["values"], prec="f64", kernel="split",
                                transpose=0)
    with pytest.raises(hm.HmatError):
        Hg.matvec_T(torch.ones(f.n, dtype=torch.float64, device="cuda:0"))
    Hg.close()
