"""Construction on the device (hmat_opts.build_device = 1): ACA and entries
on the GPU with the host construction's rules, against the host
construction and the dense products of the closed-form entries.

The pivots of the two ACAs are chosen from values computed in different
summation orders, so a near-tie can pick another (equally valid) pivot;
the block structure must be identical, the ranks nearly so, and both
products within the ACA tolerance of the dense product."""
import numpy as np
import pytest

from _util import rel, say
from synth import (TRIANGLE_WORKLOADS, WORKLOADS, config_fault, config_triangle_fault, loguniform_rates)
from synth.faults import MU, NU

pytestmark = pytest.mark.gpu


def _export_arrays(H):
    ex = H.export()
    return ex


CASES = [("dip30_48x24", 0), ("strike_37x23", 0), ("thrust_40x24", 0), ("thrust_40x24", 1)]


@pytest.mark.parametrize("name,component", CASES)
def test_device_build_matches_host_build(name, component):
    import torch

    import paper_2110_12165_amd as hm
    tri = name.startswith("thrust")
    w = (TRIANGLE_WORKLOADS if tri else WORKLOADS)[name]
    f = config_triangle_fault(name) if tri else config_fault(name)
    say(f"[device build] {name} N={f.n} component {component}")
    opts = dict(aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"], prec="f64",
                kernel="split", component=component)
    Hh = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, build_device=0, **opts)
    Hd = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, build_device=1, **opts)
    Hd2 = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, build_device=1, **opts)
    eh, ed, ed2 = Hh.export(), Hd.export(), Hd2.export()
    # identical block structure (kind may differ only by a dense fallback; positions identical)
    assert np.array_equal(eh["perm"], ed["perm"])
    assert np.array_equal(eh["desc"][:, 1:5], ed["desc"][:, 1:5])
    rh, rd = eh["desc"][:, 5].sum(), ed["desc"][:, 5].sum()
    same = np.mean(eh["desc"][:, 5] == ed["desc"][:, 5])
    say(f"   ranks: host {rh}, device {rd}; identical in {100 * same:.1f} % of the blocks")
    assert abs(int(rd) - int(rh)) <= 0.02 * max(int(rh), 1) + 2
    # reproducible
    assert np.array_equal(ed["desc"], ed2["desc"]) and np.array_equal(ed["values"], ed2["values"])
    x = loguniform_rates(f.n, 3)
    xd = torch.tensor(x, device="cuda:0")
    yh = Hh.matvec(xd).cpu().numpy()
    yd = Hd.matvec(xd).cpu().numpy()
    for H in (Hh, Hd, Hd2):
        H.close()
    n = f.n
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    D = hm.kernel_entries(f.verts, f.slip_dir, MU, NU, rows.ravel(), cols.ravel(), component).reshape(n, n)
    y = D @ x
    if np.linalg.norm(y) == 0.0:
        assert np.all(yd == 0.0)
        return
    say(f"   rel vs dense: host {rel(yh, y):.2e}, device {rel(yd, y):.2e}")
    assert rel(yd, y) <= 10 * w["aca_eps"]
    assert rel(yd, yh) <= 20 * w["aca_eps"]


@pytest.mark.parametrize("nx,ny,lattice,leaf", [(3, 2, 1, 1), (1, 1, 1, 1), (9, 7, 2, 4)])
def test_device_build_small_and_transpose(nx, ny, lattice, leaf):
    """Degenerate sizes (a single element, all-dense matrices, ragged
    leaves) and the FP32 transposed layout of a device-built matrix: H x and
    H^T x against the dense products of the closed-form entries."""
    import torch

    import paper_2110_12165_amd as hm
    from synth import planar_rect_fault
    f = planar_rect_fault(nx, ny, 100.0, 30.0, "dip")
    say(f"[device build] {nx}x{ny} lattice {lattice} leaf {leaf}")
    H = hm.HMatrix.build(f.verts, f.slip_dir, MU, NU, aca_eps=1e-8, eta=2.0, leaf=leaf, lattice=lattice,
                         prec="f32", kernel="split", build_device=1)
    n = f.n
    x = loguniform_rates(n, 5)
    xd = torch.tensor(x, device="cuda:0")
    y = H.matvec(xd).cpu().numpy()
    yt = H.matvec_T(xd).cpu().numpy()
    H.close()
    rows, cols = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    D = hm.kernel_entries(f.verts, f.slip_dir, MU, NU, rows.ravel(), cols.ravel(), 0).reshape(n, n)
    assert rel(y, D @ x) <= 1e-6
    assert rel(yt, D.T @ x) <= 1e-6
