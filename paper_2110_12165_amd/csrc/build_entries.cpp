// Mesh validation and stiffness entries A_ij (section 2.1, eqs. (5)-(6)).
//
// Full-space kernel for rectangles lying in one plane with a common in-plane
// slip direction e1.  With e2 = n x e1 and in-plane coordinates along
// (e1, e2), the traction along e1 at the centre (x1, x2) of element i due to
// unit slip along e1 on the rectangle [a1,b1] x [a2,b2] of element j is
//
//   tau = mu / (4 pi) * ( J1 / (1 - nu) + J2 ),
//   J1 = -( F(ua,va) - F(ub,va) - F(ua,vb) + F(ub,vb) ),  F(u,v) = v / (u r),
//   J2 = -( G(ua,va) - G(ub,va) - G(ua,vb) + G(ub,vb) ),  G(u,v) = u / (v r),
//
// with ua = x1 - a1, ub = x1 - b1, va = x2 - a2, vb = x2 - b2, r = |(u, v)|:
// the integral over the rectangle of the in-plane traction kernel
// mu/(4 pi) [ 1/(1-nu) d1^2 + d2^2 ](1/r) of a planar dislocation in an
// unbounded isotropic solid (Hadamard finite part on the element itself).
// The normal traction of coplanar in-plane slip vanishes, so B = 0.
//
// This file is compiled without floating-point contraction so the entries
// are reproducible across builds.
#include <cmath>
#include <memory>

#include "hmat_internal.hpp"

namespace hm {
namespace {

inline double dot3(const double* a, const double* e) { return (a[0] * e[0] + a[1] * e[1]) + a[2] * e[2]; }

inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

inline double norm3(const double* a) { return std::sqrt((a[0] * a[0] + a[1] * a[1]) + a[2] * a[2]); }

class CoplanarRectEntries final : public EntryFn {
 public:
  int64_t n;
  double mu, nu;
  int component;              // 1: normal traction, identically 0
  std::vector<double> a;      // p1, p2, lo1, hi1, lo2, hi2 (n each)

  EntryView view() const override { return EntryView{HMAT_GF_FS_RECT_COPLANAR, component, mu, nu, n, a.data()}; }
  double entry(int64_t i, int64_t j) const override { return entry_of(view(), i, j); }
};

}  // namespace

EntryFn* make_entry_fn(const hmat_mesh& mesh, const hmat_green& green, Geometry& geo) {
  if (green.kind != HMAT_GF_FS_RECT_COPLANAR && green.kind != HMAT_GF_FS_TRIANGLE)
    fail(HMAT_EUNSUPPORTED, "unknown Green's function kind");
  if (green.component != 0 && green.component != 1) fail(HMAT_EINVAL, "component must be 0 (shear) or 1 (normal)");
  if (!(green.mu > 0.0) || !std::isfinite(green.mu)) fail(HMAT_EINVAL, "mu must be positive and finite");
  if (!(green.nu > -1.0 && green.nu < 0.5)) fail(HMAT_EINVAL, "nu must lie in (-1, 0.5)");
  if (mesh.n < 1) fail(HMAT_EINVAL, "mesh.n must be >= 1");
  if (mesh.n > (int64_t)INT32_MAX / 2) fail(HMAT_EINVAL, "mesh.n too large");
  if (!mesh.verts || !mesh.slip_dir) fail(HMAT_EINVAL, "mesh.verts and mesh.slip_dir must be non-null");
  if (green.kind == HMAT_GF_FS_TRIANGLE) return make_triangle_entry_fn(mesh, green, geo);
  if (mesh.nvert != 4) fail(HMAT_EINVAL, "the coplanar rectangle kernel needs nvert = 4");

  const int64_t n = mesh.n;
  const double* V = mesh.verts;
  for (int64_t k = 0; k < n * 12; ++k)
    if (!std::isfinite(V[k])) fail(HMAT_EINVAL, "non-finite vertex coordinate");
  for (int64_t k = 0; k < n * 3; ++k)
    if (!std::isfinite(mesh.slip_dir[k])) fail(HMAT_EINVAL, "non-finite slip direction");

  auto E = std::make_unique<CoplanarRectEntries>();
  E->n = n;
  E->mu = green.mu;
  E->nu = green.nu;
  E->component = green.component;

  // Plane and in-plane axes from element 0.
  double d1[3], d3[3], nrm[3], e1[3], e2[3];
  for (int c = 0; c < 3; ++c) {
    d1[c] = V[3 + c] - V[c];
    d3[c] = V[9 + c] - V[c];
  }
  cross3(d1, d3, nrm);
  const double nn = norm3(nrm);
  if (!(nn > 0.0)) fail(HMAT_EINVAL, "degenerate element 0");
  for (int c = 0; c < 3; ++c) nrm[c] = nrm[c] / nn;
  const double sn = norm3(mesh.slip_dir);
  if (!(sn > 0.0)) fail(HMAT_EINVAL, "zero slip direction");
  for (int c = 0; c < 3; ++c) e1[c] = mesh.slip_dir[c] / sn;
  cross3(nrm, e1, e2);

  geo.n = n;
  geo.centres.resize(3 * n);
  E->a.resize(6 * n);
  double* p1 = E->a.data();
  double* p2 = p1 + n;
  double* lo1 = p2 + n;
  double* hi1 = lo1 + n;
  double* lo2 = hi1 + n;
  double* hi2 = lo2 + n;

  // Tolerances relative to the element size scale.
  double scale = 0.0;
  for (int c = 0; c < 3; ++c) scale = std::fmax(scale, std::fabs(d1[c]) + std::fabs(d3[c]));
  double extent = 0.0;
  for (int64_t k = 0; k < n * 12; ++k) extent = std::fmax(extent, std::fabs(V[k]));
  const double tol_ang = 1e-9;
  const double tol_len = 1e-9 * std::fmax(scale, extent);

  for (int64_t i = 0; i < n; ++i) {
    const double* v = V + 12 * i;
    double* c = &geo.centres[3 * i];
    for (int a = 0; a < 3; ++a) c[a] = (((v[a] + v[3 + a]) + v[6 + a]) + v[9 + a]) * 0.25;

    // rectangle: opposite edges equal, adjacent edges orthogonal, planar
    double ea[3], eb[3], ec[3], ed[3];
    for (int a = 0; a < 3; ++a) {
      ea[a] = v[3 + a] - v[a];
      eb[a] = v[9 + a] - v[a];
      ec[a] = v[6 + a] - v[9 + a];
      ed[a] = v[6 + a] - v[3 + a];
    }
    const double la = norm3(ea), lb = norm3(eb);
    if (!(la > 0.0 && lb > 0.0)) fail(HMAT_EINVAL, "degenerate element " + std::to_string(i));
    double diff1 = 0.0, diff2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      diff1 = std::fmax(diff1, std::fabs(ea[a] - ec[a]));
      diff2 = std::fmax(diff2, std::fabs(eb[a] - ed[a]));
    }
    if (diff1 > tol_len || diff2 > tol_len || std::fabs(dot3(ea, eb)) > tol_ang * la * lb)
      fail(HMAT_EINVAL, "element " + std::to_string(i) + " is not a rectangle");
    double ni[3];
    cross3(ea, eb, ni);
    const double nni = norm3(ni);
    double cr[3];
    cross3(ni, nrm, cr);
    if (norm3(cr) > tol_ang * nni || dot3(ni, nrm) <= 0.0)
      fail(HMAT_EINVAL, "element " + std::to_string(i) + " is not parallel to element 0 (coplanar kernel)");
    double off[3] = {c[0] - geo.centres[0], c[1] - geo.centres[1], c[2] - geo.centres[2]};
    if (std::fabs(dot3(off, nrm)) > tol_len)
      fail(HMAT_EINVAL, "element " + std::to_string(i) + " lies off the plane of element 0");
    const double* s = mesh.slip_dir + 3 * i;
    double sc[3];
    cross3(s, e1, sc);
    if (norm3(sc) > tol_ang * norm3(s))
      fail(HMAT_EINVAL, "element " + std::to_string(i) + ": the coplanar kernel needs one common slip direction");

    double q1[4], q2[4];
    for (int k = 0; k < 4; ++k) {
      q1[k] = dot3(v + 3 * k, e1);
      q2[k] = dot3(v + 3 * k, e2);
    }
    double l1 = q1[0], h1 = q1[0], l2 = q2[0], h2 = q2[0];
    for (int k = 1; k < 4; ++k) {
      l1 = std::fmin(l1, q1[k]); h1 = std::fmax(h1, q1[k]);
      l2 = std::fmin(l2, q2[k]); h2 = std::fmax(h2, q2[k]);
    }
    for (int k = 0; k < 4; ++k) {
      const bool ok1 = std::fabs(q1[k] - l1) <= tol_len || std::fabs(q1[k] - h1) <= tol_len;
      const bool ok2 = std::fabs(q2[k] - l2) <= tol_len || std::fabs(q2[k] - h2) <= tol_len;
      if (!ok1 || !ok2)
        fail(HMAT_EINVAL, "element " + std::to_string(i) + ": edges must be parallel and normal to the slip direction");
    }
    p1[i] = dot3(c, e1);
    p2[i] = dot3(c, e2);
    lo1[i] = l1; hi1[i] = h1; lo2[i] = l2; hi2[i] = h2;
  }
  return E.release();
}

}  // namespace hm
