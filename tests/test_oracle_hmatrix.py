"""Pins for oracle.hmatrix and oracle.dense (eqs. 5-6 and eq. 20)."""
import numpy as np
import pytest

from oracle.dense import dense_matrix, dense_rows, fft_grid_product
from oracle.greens import CoplanarRectGeometry
from oracle.hmatrix import HMatrix
from synth import WORKLOADS, config_fault, loguniform_rates
from synth.faults import MU, NU


def _build(name):
    w = WORKLOADS[name]
    f = config_fault(name)
    g = CoplanarRectGeometry(f.verts, f.slip_dir, MU, NU)
    H = HMatrix.build(g, w["leaf"], w["eta"], w["aca_eps"], w["lattice"])
    return f, g, H, w


@pytest.fixture(scope="module", params=["planar64x32", "dip30_48x24", "strike_37x23"])
def built(request):
    return _build(request.param)


def test_fft_and_rows_match_explicit_matrix(built):
    f, g, H, w = built
    A = dense_matrix(g)
    x = loguniform_rates(f.n, 7)
    yd = A @ x
    yf = fft_grid_product(f.nx, f.ny, f.h, f.slip, MU, NU, x)
    assert np.linalg.norm(yf - yd) <= 1e-13 * np.linalg.norm(yd)
    rows = np.array([0, f.n // 3, f.n - 1])
    np.testing.assert_allclose(dense_rows(g, rows, x), yd[rows], rtol=1e-12)


def test_hmatvec_close_to_plain_product(built):
    f, g, H, w = built
    x = loguniform_rates(f.n, w["seed"])
    y = H.matvec(x)
    yd = dense_matrix(g) @ x
    rel = np.linalg.norm(y - yd) / np.linalg.norm(yd)
    assert rel <= 10.0 * w["aca_eps"]
    # the represented matrix itself is close in Frobenius norm
    A = dense_matrix(g)
    assert np.linalg.norm(H.to_dense() - A) <= 10.0 * w["aca_eps"] * np.linalg.norm(A)


def test_hmatvec_linear_and_transpose_identity(built):
    f, g, H, w = built
    rng = np.random.default_rng(3)
    x1, x2, yv = rng.standard_normal((3, f.n))
    assert np.all(H.matvec(np.zeros(f.n)) == 0.0)
    lhs = H.matvec(2.0 * x1 - 3.0 * x2)
    rhs = 2.0 * H.matvec(x1) - 3.0 * H.matvec(x2)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)
    a = yv @ H.matvec(x1)
    b = H.matvec_T(yv) @ x1
    assert abs(a - b) <= 1e-12 * np.linalg.norm(yv) * np.linalg.norm(H.matvec(x1))
    # the kernel is symmetric, so H^T x ~ H x up to the compression error
    assert np.linalg.norm(H.matvec_T(x1) - H.matvec(x1)) <= 20 * w["aca_eps"] * np.linalg.norm(H.matvec(x1))
    # multi right-hand side equals column by column
    X = rng.standard_normal((f.n, 3))
    Y = H.matvec(X)
    for c in range(3):
        np.testing.assert_allclose(Y[:, c], H.matvec(X[:, c]), rtol=0, atol=1e-12 * np.abs(Y).max())


def test_storage_is_compressed():
    f, g, H, w = _build("planar64x32")
    st = H.stats()
    assert st["entries"] < 0.6 * f.n ** 2
    assert st["n_lr"] > 0 and st["n_dense"] > 0


def _as_arrays(H):
    """An oracle H-matrix in the array layout HMatrix.from_arrays reads
    (dense blocks column-major; U then V, column-major)."""
    desc, off, vals, at = [], [], [], 0
    for b in H.blocks:
        if b.kind == "dense":
            v = b.D.T.reshape(-1)
            desc.append([0, b.r0, b.m, b.c0, b.n, 0])
        else:
            v = np.concatenate([b.U.T.reshape(-1), b.V.T.reshape(-1)])
            desc.append([1, b.r0, b.m, b.c0, b.n, b.rank])
        off.append(at)
        vals.append(v)
        at += v.size
    return np.array(desc), np.array(off), np.concatenate(vals)


def test_arrays_read_back_block_for_block(built):
    f, g, H, w = built
    desc, off, vals = _as_arrays(H)
    H2 = HMatrix.from_arrays(H.n, H.perm, desc, off, vals)
    assert len(H2.blocks) == len(H.blocks)
    for a, b in zip(H.blocks, H2.blocks):
        assert (a.kind, a.r0, a.m, a.c0, a.n, a.rank) == (b.kind, b.r0, b.m, b.c0, b.n, b.rank)
        if a.kind == "dense":
            assert np.array_equal(a.D, b.D)
        else:
            assert np.array_equal(a.U, b.U) and np.array_equal(a.V, b.V)


def test_sparse_form_matches_block_loop(built):
    """H = D + U V^T as sparse matrices: both products agree with the block
    loop to rounding (the sums of a row are taken in another order), and
    the threaded row chunks give the same bits as one thread."""
    from oracle.hmatrix import SparseHMatrix
    f, g, H, w = built
    x = loguniform_rates(f.n, 3)
    S1 = SparseHMatrix(H)
    S4 = SparseHMatrix(H, threads=4)
    assert S1.nnz == H.stats()["entries"]
    for mv, mv1, mv4 in ((H.matvec, S1.matvec, S4.matvec), (H.matvec_T, S1.matvec_T, S4.matvec_T)):
        y = mv(x)
        y1 = mv1(x)
        assert np.linalg.norm(y1 - y) <= 1e-14 * np.linalg.norm(y)
        assert np.array_equal(mv4(x), y1)
    S4.close()
