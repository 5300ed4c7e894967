// Cluster tree and lattice block partition (section 3.1.1, eq. (17);
// section 3.2).
//
// Tree: binary geometric bisection of the element centres.  A cluster with
// more than `leaf` members is cut across the longest side of the bounding
// box of its centres (ties: lowest axis) at the box midpoint; members below
// the midpoint go to the first child, the rest to the second, each keeping
// their order.  If one side would be empty the members are stably sorted
// along that axis and split floor(size/2) : ceil(size/2).
//
// Partition: the tree is cut at depth L = log2(lattice); every pair of
// depth-L clusters (a lattice block) is refined on its own: an admissible
// pair, min(diam) < eta * dist with boxes of the centres, becomes one
// low-rank block; two inadmissible leaves become a dense block; otherwise
// the non-leaf side(s) are split.
#include <algorithm>
#include <cmath>

#include "hmat_internal.hpp"

namespace hm {
namespace {

struct Builder {
  const Geometry& geo;
  int32_t leaf;
  ClusterTree& t;
  std::vector<int64_t> tmp;

  int32_t make(int64_t start, int64_t size, int32_t depth) {
    TreeNode nd;
    nd.start = start;
    nd.size = size;
    nd.depth = depth;
    const double* c = geo.centres.data();
    for (int a = 0; a < 3; ++a) {
      nd.lo[a] = c[3 * t.perm[start] + a];
      nd.hi[a] = nd.lo[a];
    }
    for (int64_t k = start + 1; k < start + size; ++k)
      for (int a = 0; a < 3; ++a) {
        const double v = c[3 * t.perm[k] + a];
        nd.lo[a] = std::fmin(nd.lo[a], v);
        nd.hi[a] = std::fmax(nd.hi[a], v);
      }
    const int32_t id = (int32_t)t.nodes.size();
    t.nodes.push_back(nd);
    t.max_depth = std::max(t.max_depth, depth);
    if (size <= leaf) return id;

    int axis = 0;
    double best = nd.hi[0] - nd.lo[0];
    for (int a = 1; a < 3; ++a) {
      const double e = nd.hi[a] - nd.lo[a];
      if (e > best) { best = e; axis = a; }
    }
    const double mid = 0.5 * (nd.lo[axis] + nd.hi[axis]);
    int64_t nl = 0;
    tmp.clear();
    for (int64_t k = start; k < start + size; ++k)
      if (c[3 * t.perm[k] + axis] < mid) tmp.push_back(t.perm[k]);
    nl = (int64_t)tmp.size();
    for (int64_t k = start; k < start + size; ++k)
      if (!(c[3 * t.perm[k] + axis] < mid)) tmp.push_back(t.perm[k]);
    if (nl == 0 || nl == size) {
      tmp.assign(t.perm.begin() + start, t.perm.begin() + start + size);
      std::stable_sort(tmp.begin(), tmp.end(), [&](int64_t p, int64_t q) {
        return c[3 * p + axis] < c[3 * q + axis];
      });
      nl = size / 2;
    }
    std::copy(tmp.begin(), tmp.end(), t.perm.begin() + start);
    const int32_t a = make(start, nl, depth + 1);
    const int32_t b = make(start + nl, size - nl, depth + 1);
    t.nodes[id].child[0] = a;
    t.nodes[id].child[1] = b;
    return id;
  }
};

double diam(const TreeNode& a) {
  const double d0 = a.hi[0] - a.lo[0], d1 = a.hi[1] - a.lo[1], d2 = a.hi[2] - a.lo[2];
  return std::sqrt((d0 * d0 + d1 * d1) + d2 * d2);
}

double dist(const TreeNode& a, const TreeNode& b) {
  double g[3];
  for (int k = 0; k < 3; ++k) g[k] = std::fmax(0.0, std::fmax(b.lo[k] - a.hi[k], a.lo[k] - b.hi[k]));
  return std::sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
}

bool admissible(const TreeNode& a, const TreeNode& b, double eta) {
  return std::fmin(diam(a), diam(b)) < eta * dist(a, b);
}

}  // namespace

ClusterTree build_tree(const Geometry& geo, int32_t leaf) {
  if (leaf < 1) fail(HMAT_EINVAL, "leaf must be >= 1");
  ClusterTree t;
  t.perm.resize(geo.n);
  for (int64_t k = 0; k < geo.n; ++k) t.perm[k] = k;
  t.nodes.reserve(2 * (geo.n / std::max(1, leaf / 2) + 1));
  Builder b{geo, leaf, t, {}};
  b.make(0, geo.n, 0);
  return t;
}

std::vector<BlockSpec> partition(const ClusterTree& t, int32_t lattice, double eta) {
  if (lattice < 1 || (lattice & (lattice - 1)) != 0) fail(HMAT_EINVAL, "lattice must be a power of two");
  if (!(eta > 0.0) || !std::isfinite(eta)) fail(HMAT_EINVAL, "eta must be positive");
  int depth = 0;
  while ((1 << depth) < lattice) ++depth;
  std::vector<int32_t> level{0};
  for (int d = 0; d < depth; ++d) {
    std::vector<int32_t> nxt;
    for (int32_t id : level) {
      const TreeNode& nd = t.nodes[id];
      if (nd.leaf())
        fail(HMAT_EINVAL, "cluster tree is not complete to the lattice depth " + std::to_string(depth) +
                              " (a leaf of size " + std::to_string(nd.size) + " at depth " + std::to_string(d) + ")");
      nxt.push_back(nd.child[0]);
      nxt.push_back(nd.child[1]);
    }
    level.swap(nxt);
  }
  std::vector<BlockSpec> out;
  // explicit stack keeps the depth-first, first-child-first order
  struct Item { int32_t a, b; };
  std::vector<Item> stack;
  for (size_t li = 0; li < level.size(); ++li)
    for (size_t lj = 0; lj < level.size(); ++lj) {
      stack.push_back({level[li], level[lj]});
      while (!stack.empty()) {
        const Item it = stack.back();
        stack.pop_back();
        const TreeNode& a = t.nodes[it.a];
        const TreeNode& b = t.nodes[it.b];
        if (admissible(a, b, eta)) {
          out.push_back({1, a.start, a.size, b.start, b.size, (int32_t)li, (int32_t)lj});
        } else if (a.leaf() && b.leaf()) {
          out.push_back({0, a.start, a.size, b.start, b.size, (int32_t)li, (int32_t)lj});
        } else if (a.leaf()) {
          stack.push_back({it.a, b.child[1]});
          stack.push_back({it.a, b.child[0]});
        } else if (b.leaf()) {
          stack.push_back({a.child[1], it.b});
          stack.push_back({a.child[0], it.b});
        } else {
          stack.push_back({a.child[1], b.child[1]});
          stack.push_back({a.child[1], b.child[0]});
          stack.push_back({a.child[0], b.child[1]});
          stack.push_back({a.child[0], b.child[0]});
        }
      }
    }
  return out;
}

}  // namespace hm
