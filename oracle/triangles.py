"""Element stiffness entries for triangular elements in an unbounded medium
(FP64, NumPy).  Test infrastructure, like the rest of this package.

Paper: section 2.1, eqs. (5)-(6), with piecewise-constant slip on triangles
and collocation at the centroids.  With s_i the slip direction and n_i the
unit normal of element i (vertices counter-clockwise seen from +n_i),

    A_ij =  s_i . sigma^(j)(c_i) . n_i      (shear traction along s_i)
    B_ij = -n_i . sigma^(j)(c_i) . n_i      (normal traction, compression > 0)

where sigma^(j) is the stress of unit uniform slip s_j on triangle j and
c_i the centroid of triangle i.  The paper uses half-space solutions; the
workloads here use a full space (isotropic, mu, nu).

Route (independent of the library's closed form):

* point dislocation: per unit area and slip, the displacement is
  u_k = -m_pq d_q G_kp(r), r = x - x', with Kelvin's tensor
  G_kp = [(3 - 4 nu) delta_kp / R + r_k r_p / R^3] / (16 pi mu (1 - nu))
  and the moment density m = mu (s n^T + n s^T); its stress is
  sigma_ij = lambda delta_ij u_k,k + mu (u_i,j + u_j,i), lambda = 2 mu nu / (1 - 2 nu);
* i != j: the point stress integrated over triangle j by adaptive cubature
  (Gauss-Legendre on the collapsed square, the triangle split into four
  until the stress changes by less than 1e-10 relative);
* i == j (the receiver at its own centroid, in the source plane): the
  normal traction of in-plane slip vanishes on the plane, and the shear
  traction is the Hadamard finite part of the in-plane kernel
  G_ss = mu / (4 pi) [1/(1-nu) d_1^2 + d_2^2] (1/rho) (axis 1 along s) over
  the triangle; by the divergence theorem
  f.p. int_T d_a d_b (1/rho) dA = sum over edges of int (x_b - x'_b)/rho^3 nu_a dl
  (nu the outward in-plane edge normal; the small circle around the
  receiver contributes only the divergent part that the finite part drops),
  the edge integrals taken by adaptive quadrature.

Pins (tests/test_oracle_triangles.py): the point stress against symbolic
differentiation of Kelvin's solution for random slip and normal vectors;
the coplanar case against oracle.greens' point kernel; a rectangle equals
the sum of its two triangles, receiver inside (one self-type and one
off-element triangle) and outside, against oracle.greens' closed form;
the far field against the point dislocation.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate

_GL = {k: np.polynomial.legendre.leggauss(k) for k in (6, 8)}


def point_stress(r, s, n, mu, nu):
    """Stress (..., 3, 3) at offsets r (..., 3) from a point dislocation with
    unit slip s across a plane of unit normal n, per unit area."""
    r = np.asarray(r, dtype=np.float64)
    m = mu * (np.outer(s, n) + np.outer(n, s))
    R2 = np.einsum("...i,...i->...", r, r)
    R = np.sqrt(R2)
    iR3, iR5, iR7 = 1.0 / (R2 * R), 1.0 / (R2 * R2 * R), 1.0 / (R2 * R2 * R2 * R)
    C = 1.0 / (16.0 * np.pi * mu * (1.0 - nu))
    d = np.eye(3)
    # grad u: g_kl = -m_pq d_l d_q G_kp
    #   d_l d_q G_kp / C = -(3-4nu) d_kp (d_ql/R^3 - 3 r_q r_l/R^5)
    #                      + (d_kq d_pl + d_pq d_kl)/R^3
    #                      - 3 (d_kq r_p + d_pq r_k) r_l / R^5
    #                      - 3 (d_kl r_p r_q + d_pl r_k r_q + d_ql r_k r_p) / R^5
    #                      + 15 r_k r_p r_q r_l / R^7
    tr_m = np.trace(m)
    mr = np.einsum("pq,...q->...p", m, r)             # m_pq r_q
    rmr = np.einsum("...p,...p->...", r, mr)          # r_p m_pq r_q
    # term by term, contracted with m_pq:
    # -(3-4nu) d_kp (d_ql/R^3 - 3 r_q r_l/R^5) m_pq = -(3-4nu) (m_kl/R^3 - 3 (m r)_k r_l / R^5)
    a = -(3.0 - 4.0 * nu) * (m * iR3[..., None, None] - 3.0 * mr[..., :, None] * r[..., None, :] * iR5[..., None, None])
    # (d_kq d_pl + d_pq d_kl)/R^3 m_pq = (m_lk + tr(m) d_kl) / R^3
    b = (m.T + tr_m * d) * iR3[..., None, None]
    # -3 (d_kq r_p + d_pq r_k) r_l / R^5 m_pq = -3 ((m^T r)_k + tr(m) r_k) r_l / R^5
    mtr = np.einsum("pq,...p->...q", m, r)
    c = -3.0 * (mtr + tr_m * r)[..., :, None] * r[..., None, :] * iR5[..., None, None]
    # -3 (d_kl r_p r_q + d_pl r_k r_q + d_ql r_k r_p) / R^5 m_pq
    #   = -3 (d_kl rmr + r_k (m r)_l + r_k (m^T r)_l) / R^5
    e = -3.0 * (rmr[..., None, None] * d + r[..., :, None] * mr[..., None, :]
                + r[..., :, None] * mtr[..., None, :]) * iR5[..., None, None]
    # 15 r_k r_p r_q r_l / R^7 m_pq = 15 rmr r_k r_l / R^7
    f = 15.0 * rmr[..., None, None] * r[..., :, None] * r[..., None, :] * iR7[..., None, None]
    g = -C * (a + b + c + e + f)                       # g[..., k, l] = du_k / dx_l
    lam = 2.0 * mu * nu / (1.0 - 2.0 * nu)
    div = np.einsum("...kk->...", g)
    return lam * div[..., None, None] * d + mu * (g + np.swapaxes(g, -1, -2))


def _rule(k):
    """Gauss-Legendre rule of k^2 points on the collapsed unit square:
    (xi, eta, weight * jacobian factor xi) for the map
    x = v0 + xi (v1 - v0) + xi eta (v2 - v1), dA = 2 area xi dxi deta."""
    t, w = _GL[k]
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    xi, eta = np.meshgrid(t, t, indexing="ij")
    wt = np.outer(w, w) * xi
    return xi.ravel(), eta.ravel(), wt.ravel()


def _tri_rule(v, k=8):
    xi, eta, wt = _rule(k)
    pts = v[0] + xi[:, None] * (v[1] - v[0]) + (xi * eta)[:, None] * (v[2] - v[1])
    area2 = np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    return pts, wt * area2


def _split4(v):
    m01, m12, m20 = 0.5 * (v[0] + v[1]), 0.5 * (v[1] + v[2]), 0.5 * (v[2] + v[0])
    return [np.array([v[0], m01, m20]), np.array([m01, v[1], m12]),
            np.array([m20, m12, v[2]]), np.array([m12, m20, m01])]


def _integrate(x, v, s, n, mu, nu, tol, depth, max_depth):
    """Stress (M, 3, 3) at receivers x (M, 3) from unit slip on triangle v,
    adaptive: each piece is accepted where splitting it in four changes the
    stress by less than tol relative."""
    pts, w = _tri_rule(v)
    coarse = np.einsum("q,mqij->mij", w, point_stress(x[:, None, :] - pts[None], s, n, mu, nu))
    kids = _split4(v)
    fine = np.zeros_like(coarse)
    for c in kids:
        pc, wc = _tri_rule(c)
        fine += np.einsum("q,mqij->mij", wc, point_stress(x[:, None, :] - pc[None], s, n, mu, nu))
    err = np.linalg.norm((fine - coarse).reshape(len(x), -1), axis=1)
    ref = np.linalg.norm(fine.reshape(len(x), -1), axis=1)
    bad = err > tol * ref + 1e-300
    if not np.any(bad) or depth >= max_depth:
        return fine
    out = fine.copy()
    idx = np.nonzero(bad)[0]
    acc = np.zeros((len(idx), 3, 3))
    for c in kids:
        acc += _integrate(x[idx], c, s, n, mu, nu, tol, depth + 1, max_depth)
    out[idx] = acc
    return out


def _edge_integral(p, a, b, comp):
    """int over the segment a->b of (p - x')_comp / |p - x'|^3 dl (2D)."""
    L = np.hypot(b[0] - a[0], b[1] - a[1])

    def f(t):
        q = a + t * (b - a)
        d = p - q
        return d[comp] / np.hypot(d[0], d[1]) ** 3 * L

    val, _ = integrate.quad(f, 0.0, 1.0, epsabs=0.0, epsrel=1e-13, limit=200)
    return val


class TriangleGeometry:
    """Per-element data of a triangle mesh and its A or B entries.

    verts (N, 3, 3), counter-clockwise seen from +normal; slip_dir (N, 3)
    unit vectors in the element planes.
    """

    def __init__(self, verts, slip_dir, mu, nu, tol=1e-10, max_depth=10):
        self.verts = np.asarray(verts, dtype=np.float64)
        if self.verts.ndim != 3 or self.verts.shape[1:] != (3, 3):
            raise ValueError("verts must have shape (N, 3, 3)")
        self.n = self.verts.shape[0]
        self.mu, self.nu, self.tol, self.max_depth = float(mu), float(nu), tol, max_depth
        self.centres = self.verts.sum(axis=1) / 3.0
        nrm = np.cross(self.verts[:, 1] - self.verts[:, 0], self.verts[:, 2] - self.verts[:, 0])
        self.normals = nrm / np.linalg.norm(nrm, axis=1)[:, None]
        self.slip = np.asarray(slip_dir, dtype=np.float64)
        self._self = {}

    def _self_shear(self, j):
        """Finite-part shear traction of triangle j at its own centroid."""
        if j not in self._self:
            v, s, n = self.verts[j], self.slip[j], self.normals[j]
            e1 = s / np.linalg.norm(s)
            e2 = np.cross(n, e1)
            c = self.centres[j]
            q = np.stack([[(vv - c) @ e1, (vv - c) @ e2] for vv in v])   # in-plane coordinates
            J11 = J22 = 0.0
            for k in range(3):
                a, b = q[k], q[(k + 1) % 3]
                t = (b - a) / np.hypot(*(b - a))
                nu_out = np.array([t[1], -t[0]])        # outward for counter-clockwise edges
                # f.p. int d_a d_b (1/rho) = sum_edges int (p - x')_b / rho^3 nu_a dl, p = 0 here
                J11 += nu_out[0] * _edge_integral(np.zeros(2), a, b, 0)
                J22 += nu_out[1] * _edge_integral(np.zeros(2), a, b, 1)
            self._self[j] = self.mu / (4.0 * np.pi) * (J11 / (1.0 - self.nu) + J22)
        return self._self[j]

    def stress(self, rows, j):
        """Stress tensors (len(rows), 3, 3) at the centroids of rows from unit slip on j (rows != j)."""
        x = self.centres[np.asarray(rows)]
        return _integrate(x, self.verts[j], self.slip[j], self.normals[j], self.mu, self.nu,
                          self.tol, 0, self.max_depth)

    def blocks(self, rows, cols):
        """Dense blocks (A, B) from one stress evaluation per source."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        A = np.empty((len(rows), len(cols)))
        B = np.empty((len(rows), len(cols)))
        for jj, j in enumerate(cols):
            other = rows != j
            if np.any(other):
                sig = self.stress(rows[other], j)
                s, nr = self.slip[rows[other]], self.normals[rows[other]]
                A[other, jj] = np.einsum("mi,mij,mj->m", s, sig, nr)
                B[other, jj] = -np.einsum("mi,mij,mj->m", nr, sig, nr)
            if np.any(~other):
                A[~other, jj] = self._self_shear(j)
                B[~other, jj] = 0.0
        return A, B

    def block(self, rows, cols, component="A"):
        """Dense block of A (component "A") or B ("B")."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        out = np.empty((len(rows), len(cols)))
        for jj, j in enumerate(cols):
            other = rows != j
            if np.any(other):
                sig = self.stress(rows[other], j)
                s, nr = self.slip[rows[other]], self.normals[rows[other]]
                if component == "A":
                    out[other, jj] = np.einsum("mi,mij,mj->m", s, sig, nr)
                else:
                    out[other, jj] = -np.einsum("mi,mij,mj->m", nr, sig, nr)
            if np.any(~other):
                out[~other, jj] = self._self_shear(j) if component == "A" else 0.0
        return out
