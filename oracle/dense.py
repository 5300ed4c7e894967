"""The plain product y = A x (eqs. 5-6), without any compression (FP64).

Three forms of the same definition:

* ``dense_matrix``  — the explicit N x N matrix (small N).
* ``dense_rows``    — y_i = sum_j A_ij x_j for selected rows, one row at a
                      time (any N; O(N) per row).
* ``fft_grid_product`` — for a planar grid of equal squares the entries
  depend only on the in-plane offset between elements (translation
  invariance), so A is block-Toeplitz with Toeplitz blocks and A x is a
  2D linear convolution of the offset table with x, evaluated exactly
  (up to rounding) with zero-padded FFTs.  The grid is indexed
  k = iy * nx + ix as in ``synth``.

Pins (tests/test_oracle_hmatrix.py): the FFT form against the explicit
matrix, the row form against the explicit matrix.
"""
from __future__ import annotations

import numpy as np

from .greens import rect_traction


def dense_matrix(geom):
    idx = np.arange(geom.n)
    return geom.block(idx, idx)


def dense_rows(geom, rows, x):
    x = np.asarray(x, dtype=np.float64)
    cols = np.arange(geom.n)
    out = np.empty((len(rows),) + x.shape[1:])
    for k, i in enumerate(rows):
        out[k] = geom.entry_row(int(i), cols) @ x
    return out


def offset_table(nx, ny, h, slip, mu, nu):
    """K[dy + ny - 1, dx + nx - 1] = A between elements whose grid offset
    (receiver minus source) is (dx, dy)."""
    dx = np.arange(-(nx - 1), nx) * h
    dy = np.arange(-(ny - 1), ny) * h
    DX, DY = np.meshgrid(dx, dy)          # (2ny-1, 2nx-1)
    if slip == "strike":                  # slip axis along strike (x)
        u, v = DX, DY
    else:                                 # slip axis down dip
        u, v = DY, DX
    half = 0.5 * h
    return rect_traction(u, v, -half, half, -half, half, mu, nu)


def fft_grid_product(nx, ny, h, slip, mu, nu, x):
    """y = A x for the nx x ny grid, x in grid order (length nx*ny, or
    (nx*ny, k))."""
    x = np.asarray(x, dtype=np.float64)
    multi = x.ndim == 2
    X = x.reshape(ny, nx, -1)
    K = offset_table(nx, ny, h, slip, mu, nu)
    P = (2 * ny - 1, 2 * nx - 1)
    Kf = np.fft.rfft2(K, s=P)
    out = np.empty_like(X)
    for c in range(X.shape[2]):
        full = np.fft.irfft2(Kf * np.fft.rfft2(X[:, :, c], s=P), s=P)
        out[:, :, c] = full[ny - 1:2 * ny - 1, nx - 1:2 * nx - 1]
    out = out.reshape(nx * ny, -1)
    return out if multi else out[:, 0]
