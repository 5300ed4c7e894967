"""Adaptive cross approximation with partial pivoting (FP64).

Paper: section 3.1.2, eqs. (18)-(19).  An admissible block A_LM (m x n) is
approximated by sum_k g_k h_k^T, built one rank at a time from single rows
and columns of the block, so only O((m + n) r) entries are ever evaluated.
The rank grows until the newest rank-one term is small against the
running Frobenius-norm estimate of the approximation (the paper notes that
eq. 19 cannot be checked exactly because the full block is never formed).

Steps as implemented (a reading of the method; the paper does not spell out
the variant, the first pivot, ties or the rank-control method it cites):

1. Start from the first row of the block; no row used yet; S2 = 0.
2. Residual row r = a(i, :) - sum_l U[i, l] V[:, l]; mark row i used.
3. Column pivot j = argmax |r| (lowest index on ties).  If |r_j| is zero
   (<= 1e-300) take the lowest unused row and go back to 2; stop when no
   row is left.
4. v = r / r_j; residual column u = a(:, j) - sum_l V[j, l] U[:, l].
5. Append (u, v).  Update the squared norm estimate
   S2 += 2 sum_{l<k} (u_l . u)(v_l . v) + |u|^2 |v|^2.
6. Stop when |u| |v| <= eps * sqrt(S2).
7. Dense fallback (in place of the cited rank-control method): if
   k (m + n) >= m n or k reaches max_rank, the block is stored dense.
8. Next row = argmax over unused rows of |u_i| (lowest index on ties).

The factors returned are U (m x k) and V (n x k) with A ~ U V^T, i.e. the
paper's g = U^T and h = V^T.

Pins (tests/test_oracle_aca.py): exact recovery of exactly low-rank blocks
at their rank; Frobenius error of kernel blocks measured against the
explicit block, compared with the tolerance; rank compared with the
optimal (SVD) rank at the same error.
"""
from __future__ import annotations

import numpy as np


def aca(row_fn, col_fn, m, n, eps, max_rank=0):
    """Return (U, V) or None when the dense fallback applies.

    row_fn(i) -> block row i (length n); col_fn(j) -> block column j (length m).
    """
    if max_rank <= 0:
        max_rank = min(m, n) // 2
    max_rank = max(1, min(max_rank, min(m, n)))
    us, vs = [], []
    used = np.zeros(m, dtype=bool)
    i = 0
    s2 = 0.0
    while True:
        r = np.array(row_fn(i), dtype=np.float64)
        for ul, vl in zip(us, vs):
            r -= ul[i] * vl
        used[i] = True
        j = int(np.argmax(np.abs(r)))
        if abs(r[j]) <= 1e-300:
            free = np.flatnonzero(~used)
            if free.size == 0:
                break
            i = int(free[0])
            continue
        v = r / r[j]
        u = np.array(col_fn(j), dtype=np.float64)
        for ul, vl in zip(us, vs):
            u -= vl[j] * ul
        cross = 0.0
        for ul, vl in zip(us, vs):
            cross += float(ul @ u) * float(vl @ v)
        nu2 = float(u @ u)
        nv2 = float(v @ v)
        s2 += 2.0 * cross + nu2 * nv2
        us.append(u)
        vs.append(v)
        k = len(us)
        if np.sqrt(nu2) * np.sqrt(nv2) <= eps * np.sqrt(s2):
            break
        if k * (m + n) >= m * n or k >= max_rank:
            return None
        cand = np.where(used, -1.0, np.abs(u))
        i = int(np.argmax(cand))
        if cand[i] < 0.0:
            break
    k = len(us)
    if k * (m + n) >= m * n:
        return None
    U = np.array(us).T.reshape(m, k) if k else np.zeros((m, 0))
    V = np.array(vs).T.reshape(n, k) if k else np.zeros((n, 0))
    return U, V
