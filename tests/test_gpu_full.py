"""GPU parity at the full benchmark size: planar 30-degree dipping thrust,
480 x 256 squares of 50 m (N = 122880), ACA eps 1e-5, leaf 64, eta 2,
lattice 32 x 32, in the launch configurations that bench.py times.

The oracle cannot rebuild an H-matrix of this size in test time, so the
GPU products are compared with the exact product y = A x, which the oracle
computes by FFT (translation invariance of the planar grid) and, for
sampled rows, one row at a time straight from the entries.  The
requirement: relative error <= 1e-6 for FP64 storage and <= 2e-5 for FP32
storage (the compression error of this matrix is about 3e-8).
"""
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
    info = H.info()
    H.close()
    r = rel(y1, y_exact)
    say(f"    rel vs exact {r:.3e}  entries {info['dense_entries'] + info['lr_entries']}")
    assert r <= (1e-6 if opts["prec"] == "f64" else 2e-5)
    assert np.array_equal(y1, y2)                 # run-to-run reproducible
    # sampled rows, evaluated one by one from the entries
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    rows = np.random.default_rng(99).choice(f.n, 48, replace=False)
    ref = dense_rows(g, rows, x)
    assert np.max(np.abs(y1[rows] - ref)) <= 1e-5 * np.max(np.abs(y_exact))
    assert info["max_rank"] <= 64 and info["n_lr"] > 40000
