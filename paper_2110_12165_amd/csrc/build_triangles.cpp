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

class TriangleEntries final : public EntryFn {
 public:
  int64_t n;
  double mu, nu;
  int component;            // 0: A (shear), 1: B (normal)
  std::vector<double> a;    // vertices 9n, centroids 3n, unit normals 3n, unit slips 3n

  EntryView view() const override { return EntryView{HMAT_GF_FS_TRIANGLE, component, mu, nu, n, a.data()}; }
  double entry(int64_t i, int64_t j) const override { return entry_of(view(), i, j); }
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
  E->n = n;
  E->mu = green.mu;
  E->nu = green.nu;
  E->component = green.component;
  E->a.resize(18 * n);
  double* pv = E->a.data();
  double* pc = pv + 9 * n;
  double* pn = pc + 3 * n;
  double* ps = pn + 3 * n;
  geo.n = n;
  geo.centres.resize(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double* v = Vp + 9 * i;
    const V3 a{v[0], v[1], v[2]}, b{v[3], v[4], v[5]}, c{v[6], v[7], v[8]};
    for (int k = 0; k < 9; ++k) pv[9 * i + k] = v[k];
    const V3 cr = v3cross(v3sub(b, a), v3sub(c, a));
    const double area2 = v3norm(cr);
    const double lmax = std::fmax(v3norm(v3sub(b, a)), std::fmax(v3norm(v3sub(c, b)), v3norm(v3sub(a, c))));
    if (!(area2 > 1e-12 * lmax * lmax)) fail(HMAT_EINVAL, "degenerate element " + std::to_string(i));
    const V3 nn = v3scale(1.0 / area2, cr);
    const V3 s{mesh.slip_dir[3 * i], mesh.slip_dir[3 * i + 1], mesh.slip_dir[3 * i + 2]};
    const double sn = v3norm(s);
    if (!(sn > 0.0)) fail(HMAT_EINVAL, "zero slip direction at element " + std::to_string(i));
    if (std::fabs(v3dot(s, nn)) > 1e-6 * sn)
      fail(HMAT_EINVAL, "element " + std::to_string(i) + ": slip direction not in the element plane");
    const V3 su = v3scale(1.0 / sn, s);
    const V3 ce = v3scale(1.0 / 3.0, v3add(v3add(a, b), c));
    pc[3 * i] = ce.x; pc[3 * i + 1] = ce.y; pc[3 * i + 2] = ce.z;
    pn[3 * i] = nn.x; pn[3 * i + 1] = nn.y; pn[3 * i + 2] = nn.z;
    ps[3 * i] = su.x; ps[3 * i + 1] = su.y; ps[3 * i + 2] = su.z;
    geo.centres[3 * i] = ce.x;
    geo.centres[3 * i + 1] = ce.y;
    geo.centres[3 * i + 2] = ce.z;
  }
  return E.release();
}

}  // namespace hm
