// Closed-form stiffness entries (section 2.1, eqs. (5)-(6)) shared by the
// host construction and the device construction: the same source compiles
// for the CPU (g++) and for gfx950 (hipcc), so both builds evaluate the same
// formulas.  The derivations are in build_entries.cpp (coplanar rectangles)
// and build_triangles.cpp (triangular dislocation loops).
#pragma once

#include <cmath>

#ifdef __HIPCC__
#define HM_HD __host__ __device__
#else
#define HM_HD
#endif

namespace hm {

// Traction along axis 1 at in-plane point (x1, x2) from unit slip along axis
// 1 on the rectangle [a1, b1] x [a2, b2] of the same plane (full space).
HM_HD inline double rect_traction(double x1, double x2, double a1, double b1, double a2, double b2, double mu,
                                  double nu) {
  const double ua = x1 - a1, ub = x1 - b1, va = x2 - a2, vb = x2 - b2;
  const double raa = sqrt(ua * ua + va * va), rba = sqrt(ub * ub + va * va);
  const double rab = sqrt(ua * ua + vb * vb), rbb = sqrt(ub * ub + vb * vb);
  const double j1 = -(va / (ua * raa) - va / (ub * rba) - vb / (ua * rab) + vb / (ub * rbb));
  const double j2 = -(ua / (va * raa) - ub / (va * rba) - ua / (vb * rab) + ub / (vb * rbb));
  return mu / (4.0 * M_PI) * (j1 / (1.0 - nu) + j2);
}

struct V3 {
  double x, y, z;
};
HM_HD inline V3 v3sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
HM_HD inline V3 v3add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
HM_HD inline V3 v3scale(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
HM_HD inline double v3dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
HM_HD inline V3 v3cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
HM_HD inline double v3norm(V3 a) { return sqrt(v3dot(a, a)); }

// u . sigma . v at x from unit slip b on the triangular dislocation loop
// t[0] -> t[1] -> t[2] in a full space (Peach-Koehler line integral, each
// edge in closed form; see build_triangles.cpp).
HM_HD inline double tri_traction(V3 x, const V3* t, V3 b, V3 u, V3 v, double mu, double nu) {
  const double k1 = mu / (4.0 * M_PI), k2 = mu / (4.0 * M_PI * (1.0 - nu));
  const double uv = v3dot(u, v);
  double out = 0.0;
  for (int e = 0; e < 3; ++e) {
    const V3 A = t[e], B = t[(e + 1) % 3];
    const V3 AB = v3sub(B, A);
    const double L = v3norm(AB);
    const V3 tt = v3scale(1.0 / L, AB);
    const V3 rA = v3sub(x, A), rB = v3sub(x, B);
    const double zA = v3dot(rA, tt), zB = v3dot(rB, tt);
    const V3 p = v3sub(rA, v3scale(zA, tt));
    const double rho2 = v3dot(p, p);
    const double RA = v3norm(rA), RB = v3norm(rB);
    const double cA = zA / RA, cB = zB / RB;
    const double J30 = zA * zB > 0.0 ? (zA * zA - zB * zB) / ((zA * RB + zB * RA) * RA * RB) : (cA - cB) / rho2;
    const double J31 = -1.0 / RA + 1.0 / RB;
    const double K =
        1.0 / (RA * RA) + 1.0 / (RB * RB) + (zA * zA + zB * zB + rho2) / ((RA * RB + zA * zB) * RA * RB);
    const double J50 = J30 * K / 3.0;
    const double J51 = -1.0 / (3.0 * RA * RA * RA) + 1.0 / (3.0 * RB * RB * RB);
    const double J52 = J30 * (cA * cA + cA * cB + cB * cB) / 3.0;
    const V3 I3 = v3add(v3scale(J30, p), v3scale(J31, tt));  // int r / R^3 ds
    const V3 dPsi = v3scale(-1.0, I3);
    const V3 c = v3cross(dPsi, b);
    const V3 beta = v3cross(b, tt);
    const double bp = v3dot(beta, p), up = v3dot(u, p), vp = v3dot(v, p), ut = v3dot(u, tt), vt = v3dot(v, tt);
    const double D = 3.0 * (bp * up * vp * J50 + J51 * bp * (up * vt + ut * vp) + J52 * bp * ut * vt) -
                     (v3dot(beta, u) * v3dot(I3, v) + v3dot(beta, v) * v3dot(I3, u) + uv * v3dot(beta, I3));
    out += -k1 * (v3dot(c, u) * vt + v3dot(c, v) * ut) - k2 * (D - 2.0 * uv * v3dot(beta, dPsi));
  }
  return out;
}

// Per-element data of either kernel, packed in one array (kind 1: p1, p2,
// lo1, hi1, lo2, hi2 of n each; kind 2: vertices 9n, centroids 3n, normals
// 3n, unit slip directions 3n), and the entry A_ij (component 0) or B_ij (1).
struct EntryView {
  int kind;        // hmat_green_kind
  int component;   // 0 shear (A), 1 normal (B)
  double mu, nu;
  long long n;
  const double* a;
};

HM_HD inline double entry_of(const EntryView& E, long long i, long long j) {
  const long long n = E.n;
  if (E.kind == 1) {
    if (E.component == 1) return 0.0;
    const double* a = E.a;
    return rect_traction(a[i], a[n + i], a[2 * n + j], a[3 * n + j], a[4 * n + j], a[5 * n + j], E.mu, E.nu);
  }
  const double* vt = E.a + 9 * j;
  const V3 t[3] = {{vt[0], vt[1], vt[2]}, {vt[3], vt[4], vt[5]}, {vt[6], vt[7], vt[8]}};
  const double* c = E.a + 9 * n + 3 * i;
  const double* nr = E.a + 12 * n + 3 * i;
  const double* si = E.a + 15 * n + 3 * i;
  const double* sj = E.a + 15 * n + 3 * j;
  const V3 x{c[0], c[1], c[2]}, nv{nr[0], nr[1], nr[2]}, bj{sj[0], sj[1], sj[2]};
  if (E.component == 1) {
    if (i == j) return 0.0;  // in-plane slip: no normal traction on its own plane
    return -tri_traction(x, t, bj, nv, nv, E.mu, E.nu);
  }
  return tri_traction(x, t, bj, V3{si[0], si[1], si[2]}, nv, E.mu, E.nu);
}

}  // namespace hm
