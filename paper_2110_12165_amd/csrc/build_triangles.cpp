// Stiffness entries of triangular elements in an unbounded isotropic solid
// (section 2.1, eqs. (5)-(6): piecewise-constant slip, collocation at the
// centroids), for nonplanar faults:
//
//   A_ij =  s_i . sigma^(j)(c_i) . n_i    (shear traction along s_i)
//   B_ij = -n_i . sigma^(j)(c_i) . n_i    (normal traction, compression > 0)
//
// sigma^(j) is the stress of unit uniform slip b = s_j on triangle j.  A
// uniform displacement discontinuity on a planar triangle is a triangular
// dislocation loop, whose stress is a line integral over the loop
// (Peach & Koehler 1950, isotropic form):
//
//   sigma_ab = sum over the three edges of
//     -mu/(4 pi) (c_a t_b + c_b t_a)
//     -mu/(4 pi (1-nu)) (beta_i D_iab - 2 delta_ab beta . dPsi),
//   c = dPsi x b,  beta = b x t,
//
// for an edge from A to B (unit direction t, length L), with
//   dPsi_i = d_i int_0^L ds / R = -int r_i / R^3 ds,
//   D_ijk  = d_i d_j d_k int_0^L R ds = int (3 r_i r_j r_k / R^5
//            - (delta_ij r_k + delta_ik r_j + delta_jk r_i) / R^3) ds,
// r = x - x'(s), R = |r|.  Writing r = p + z t (p the part normal to the
// edge line, rho = |p|, z = r . t, from z_A = (x - A) . t to z_B = (x - B) . t),
// the edge integrals are J3_m = int z^m / R^3 and J5_m = int z^m / R^5:
//   J3_0 = [z / (rho^2 R)],  J3_1 = [-1 / R],
//   J5_0 = [z (2 z^2 + 3 rho^2) / (3 rho^4 R^3)],  J5_1 = [-1 / (3 R^3)],
//   J5_2 = [z^3 / (3 rho^2 R^3)]                       ([f] = f(z_A) - f(z_B)),
// evaluated in forms without cancellation when the receiver lies near the
// extension of the edge line (z_A z_B > 0): with c = z / R,
//   J3_0 = (z_A^2 - z_B^2) / ((z_A R_B + z_B R_A) R_A R_B),
//   J5_0 = J3_0 / 3 [1/R_A^2 + 1/R_B^2 + (z_A^2 + z_B^2 + rho^2) / ((R_A R_B + z_A z_B) R_A R_B)],
//   J5_2 = J3_0 (c_A^2 + c_A c_B + c_B^2) / 3.
// Since beta . t = 0 the t t t part of D drops out of every contraction.
// At its own centroid (in the source plane, inside the loop) the line
// integral gives the finite-part self term; the normal traction of the self
// term is 0.  A triangle's orientation follows its vertex order
// (counter-clockwise seen from +n); the loop is traversed in that order.
//
// Compiled without floating-point contraction so the entries are
// reproducible across builds.
#include <cmath>
#include <memory>
#include <string>

#include "hmat_internal.hpp"

namespace hm {
namespace {

struct V3 {
  double x, y, z;
};
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }

// u . sigma . v at x for unit slip b on the loop verts[0] -> verts[1] -> verts[2].
double loop_traction(V3 x, const V3* verts, V3 b, V3 u, V3 v, double mu, double nu) {
  const double k1 = mu / (4.0 * M_PI), k2 = mu / (4.0 * M_PI * (1.0 - nu));
  const double uv = dot(u, v);
  double out = 0.0;
  for (int e = 0; e < 3; ++e) {
    const V3 A = verts[e], B = verts[(e + 1) % 3];
    const V3 AB = B - A;
    const double L = norm(AB);
    const V3 t = (1.0 / L) * AB;
    const V3 rA = x - A, rB = x - B;
    const double zA = dot(rA, t), zB = dot(rB, t);
    const V3 p = rA - zA * t;
    const double rho2 = dot(p, p);
    const double RA = norm(rA), RB = norm(rB);
    const double cA = zA / RA, cB = zB / RB;
    const double J30 = zA * zB > 0.0 ? (zA * zA - zB * zB) / ((zA * RB + zB * RA) * RA * RB) : (cA - cB) / rho2;
    const double J31 = -1.0 / RA + 1.0 / RB;
    const double K = 1.0 / (RA * RA) + 1.0 / (RB * RB) + (zA * zA + zB * zB + rho2) / ((RA * RB + zA * zB) * RA * RB);
    const double J50 = J30 * K / 3.0;
    const double J51 = -1.0 / (3.0 * RA * RA * RA) + 1.0 / (3.0 * RB * RB * RB);
    const double J52 = J30 * (cA * cA + cA * cB + cB * cB) / 3.0;
    const V3 I3 = J30 * p + J31 * t;  // int r / R^3 ds
    const V3 dPsi = -1.0 * I3;
    const V3 c = cross(dPsi, b);
    const V3 beta = cross(b, t);
    const double bp = dot(beta, p), up = dot(u, p), vp = dot(v, p), ut = dot(u, t), vt = dot(v, t);
    const double D = 3.0 * (bp * up * vp * J50 + J51 * bp * (up * vt + ut * vp) + J52 * bp * ut * vt) -
                     (dot(beta, u) * dot(I3, v) + dot(beta, v) * dot(I3, u) + uv * dot(beta, I3));
    out += -k1 * (dot(c, u) * vt + dot(c, v) * ut) - k2 * (D - 2.0 * uv * dot(beta, dPsi));
  }
  return out;
}

class TriangleEntries final : public EntryFn {
 public:
  double mu, nu;
  bool normal;                          // B (normal traction) instead of A
  std::vector<V3> verts, cen, nrm, slip;  // 3 n, n, n, n

  double entry(int64_t i, int64_t j) const override {
    const V3 n = nrm[i];
    if (normal) {
      if (i == j) return 0.0;  // in-plane slip: no normal traction on its own plane
      return -loop_traction(cen[i], &verts[3 * j], slip[j], n, n, mu, nu);
    }
    return loop_traction(cen[i], &verts[3 * j], slip[j], slip[i], n, mu, nu);
  }
};

}  // namespace

EntryFn* make_triangle_entry_fn(const hmat_mesh& mesh, const hmat_green& green, Geometry& geo) {
  if (mesh.nvert != 3) fail(HMAT_EINVAL, "the triangle kernel needs nvert = 3");
  const int64_t n = mesh.n;
  const double* Vp = mesh.verts;
  for (int64_t k = 0; k < n * 9; ++k)
    if (!std::isfinite(Vp[k])) fail(HMAT_EINVAL, "non-finite vertex coordinate");
  for (int64_t k = 0; k < n * 3; ++k)
    if (!std::isfinite(mesh.slip_dir[k])) fail(HMAT_EINVAL, "non-finite slip direction");
  auto E = std::make_unique<TriangleEntries>();
  E->mu = green.mu;
  E->nu = green.nu;
  E->normal = green.component == 1;
  E->verts.resize(3 * n);
  E->cen.resize(n);
  E->nrm.resize(n);
  E->slip.resize(n);
  geo.n = n;
  geo.centres.resize(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double* v = Vp + 9 * i;
    const V3 a{v[0], v[1], v[2]}, b{v[3], v[4], v[5]}, c{v[6], v[7], v[8]};
    E->verts[3 * i] = a;
    E->verts[3 * i + 1] = b;
    E->verts[3 * i + 2] = c;
    const V3 cr = cross(b - a, c - a);
    const double area2 = norm(cr);
    const double lmax = std::fmax(norm(b - a), std::fmax(norm(c - b), norm(a - c)));
    if (!(area2 > 1e-12 * lmax * lmax)) fail(HMAT_EINVAL, "degenerate element " + std::to_string(i));
    const V3 nn = (1.0 / area2) * cr;
    const V3 s{mesh.slip_dir[3 * i], mesh.slip_dir[3 * i + 1], mesh.slip_dir[3 * i + 2]};
    const double sn = norm(s);
    if (!(sn > 0.0)) fail(HMAT_EINVAL, "zero slip direction at element " + std::to_string(i));
    if (std::fabs(dot(s, nn)) > 1e-6 * sn)
      fail(HMAT_EINVAL, "element " + std::to_string(i) + ": slip direction not in the element plane");
    E->nrm[i] = nn;
    E->slip[i] = (1.0 / sn) * s;
    const V3 ce = (1.0 / 3.0) * ((a + b) + c);
    E->cen[i] = ce;
    geo.centres[3 * i] = ce.x;
    geo.centres[3 * i + 1] = ce.y;
    geo.centres[3 * i + 2] = ce.z;
  }
  return E.release();
}

}  // namespace hm
