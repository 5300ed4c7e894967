// Adaptive cross approximation and assembly of the block list
// (section 3.1.2, eqs. (18)-(19)).
//
// Partial pivoting: start at the first row of the block; the residual row
// gives the column pivot (largest magnitude, lowest index on ties); the
// residual column scaled by the pivot gives the new rank-one term; the next
// row is the unused row with the largest entry of the new column.  A zero
// residual row moves on to the lowest unused row.  The rank stops growing
// when |u| |v| <= eps * ||U V^T||_F, with the Frobenius norm updated
// incrementally.  Blocks whose factors would not be smaller than the dense
// block, or that reach max_rank, are stored dense.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

#include "hmat_internal.hpp"

namespace hm {

bool aca_block(const EntryFn& A, const int64_t* rows, int64_t m, const int64_t* cols, int64_t n,
               double eps, int32_t max_rank, std::vector<double>& U, std::vector<double>& V,
               int64_t& rank) {
  int64_t kmax = max_rank > 0 ? max_rank : std::min(m, n) / 2;
  kmax = std::max<int64_t>(1, std::min<int64_t>(kmax, std::min(m, n)));
  U.clear();
  V.clear();
  std::vector<char> used(m, 0);
  std::vector<double> r(n), u(m);
  int64_t k = 0;
  int64_t i = 0;
  double s2 = 0.0;
  for (;;) {
    for (int64_t j = 0; j < n; ++j) r[j] = A.entry(rows[i], cols[j]);
    for (int64_t l = 0; l < k; ++l) {
      const double ul = U[l * m + i];
      const double* vl = &V[l * n];
      for (int64_t j = 0; j < n; ++j) r[j] -= ul * vl[j];
    }
    used[i] = 1;
    int64_t jp = 0;
    double best = std::fabs(r[0]);
    for (int64_t j = 1; j < n; ++j)
      if (std::fabs(r[j]) > best) { best = std::fabs(r[j]); jp = j; }
    if (best <= 1e-300) {
      int64_t nxt = -1;
      for (int64_t q = 0; q < m; ++q)
        if (!used[q]) { nxt = q; break; }
      if (nxt < 0) break;
      i = nxt;
      continue;
    }
    const double piv = r[jp];
    for (int64_t j = 0; j < n; ++j) r[j] = r[j] / piv;  // v
    for (int64_t q = 0; q < m; ++q) u[q] = A.entry(rows[q], cols[jp]);
    for (int64_t l = 0; l < k; ++l) {
      const double vl = V[l * n + jp];
      const double* ul = &U[l * m];
      for (int64_t q = 0; q < m; ++q) u[q] -= vl * ul[q];
    }
    double cross = 0.0;
    for (int64_t l = 0; l < k; ++l) {
      double du = 0.0, dv = 0.0;
      for (int64_t q = 0; q < m; ++q) du += U[l * m + q] * u[q];
      for (int64_t j = 0; j < n; ++j) dv += V[l * n + j] * r[j];
      cross += du * dv;
    }
    double nu2 = 0.0, nv2 = 0.0;
    for (int64_t q = 0; q < m; ++q) nu2 += u[q] * u[q];
    for (int64_t j = 0; j < n; ++j) nv2 += r[j] * r[j];
    s2 += 2.0 * cross + nu2 * nv2;
    U.insert(U.end(), u.begin(), u.end());
    V.insert(V.end(), r.begin(), r.end());
    ++k;
    if (std::sqrt(nu2) * std::sqrt(nv2) <= eps * std::sqrt(s2)) break;
    if (k * (m + n) >= m * n || k >= kmax) return false;
    int64_t ip = -1;
    double bu = -1.0;
    for (int64_t q = 0; q < m; ++q)
      if (!used[q] && std::fabs(u[q]) > bu) { bu = std::fabs(u[q]); ip = q; }
    if (ip < 0) break;
    i = ip;
  }
  if (k * (m + n) >= m * n) return false;
  rank = k;
  return true;
}

HostMatrix assemble(const EntryFn& A, const ClusterTree& tree, const std::vector<BlockSpec>& blocks,
                    double eps, int32_t max_rank, int32_t n_threads) {
  if (!(eps > 0.0) || !std::isfinite(eps)) fail(HMAT_EINVAL, "aca_eps must be positive");
  if (max_rank < 0) fail(HMAT_EINVAL, "max_rank must be >= 0");
  const int64_t nb = (int64_t)blocks.size();
  struct Result {
    int kind = 0;
    int64_t rank = 0;
    std::vector<double> a, b;
  };
  std::vector<Result> res(nb);
  const int64_t* perm = tree.perm.data();
  std::atomic<int64_t> next{0};
  std::atomic<bool> failed{false};
  std::string err;
  auto work = [&]() {
    try {
      std::vector<double> U, V;
      for (;;) {
        const int64_t b = next.fetch_add(1);
        if (b >= nb || failed.load()) break;
        const BlockSpec& s = blocks[b];
        const int64_t* rows = perm + s.r0;
        const int64_t* cols = perm + s.c0;
        Result& R = res[b];
        int64_t rank = 0;
        if (s.kind == 1 && aca_block(A, rows, s.m, cols, s.n, eps, max_rank, U, V, rank)) {
          R.kind = 1;
          R.rank = rank;
          R.a = U;
          R.b = V;
        } else {
          R.kind = 0;
          R.a.resize(s.m * s.n);
          for (int64_t j = 0; j < s.n; ++j)
            for (int64_t i = 0; i < s.m; ++i) R.a[j * s.m + i] = A.entry(rows[i], cols[j]);
        }
      }
    } catch (const std::exception& e) {
      failed.store(true);
      err = e.what();
    }
  };
  int nt = n_threads > 0 ? n_threads : host_threads();
  nt = (int)std::min<int64_t>(nt, std::max<int64_t>(1, nb));
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  if (failed.load()) fail(HMAT_ENOMEM, "block construction failed: " + err);

  HostMatrix H;
  H.n = (int64_t)tree.perm.size();
  H.perm.resize(H.n);
  for (int64_t k = 0; k < H.n; ++k) H.perm[k] = (int32_t)tree.perm[k];
  H.desc.resize(6 * nb);
  H.off.resize(nb);
  int64_t total = 0;
  for (int64_t b = 0; b < nb; ++b) {
    H.off[b] = total;
    total += (int64_t)(res[b].a.size() + res[b].b.size());
  }
  H.values.resize(total);
  parallel_for(nb, n_threads, [&](int64_t b) {
    const BlockSpec& s = blocks[b];
    int64_t* d = &H.desc[6 * b];
    d[0] = res[b].kind;
    d[1] = s.r0; d[2] = s.m; d[3] = s.c0; d[4] = s.n; d[5] = res[b].rank;
    std::copy(res[b].a.begin(), res[b].a.end(), H.values.begin() + H.off[b]);
    std::copy(res[b].b.begin(), res[b].b.end(), H.values.begin() + H.off[b] + res[b].a.size());
    std::vector<double>().swap(res[b].a);
    std::vector<double>().swap(res[b].b);
  });
  H.tree_depth = tree.max_depth;
  return H;
}

void validate_host_matrix(const HostMatrix& H) {
  const int64_t n = H.n;
  if (n < 1) fail(HMAT_EINVAL, "n must be >= 1");
  if ((int64_t)H.perm.size() != n) fail(HMAT_EINVAL, "perm has the wrong length");
  std::vector<char> seen(n, 0);
  for (int64_t k = 0; k < n; ++k) {
    const int32_t p = H.perm[k];
    if (p < 0 || p >= n || seen[p]) fail(HMAT_EINVAL, "perm is not a permutation");
    seen[p] = 1;
  }
  // Tiling check: every block inside the matrix; total area n^2; rows of
  // each block row-interval covered by column ranges without overlap is
  // verified by sorting blocks per row interval.
  const int64_t nb = H.nblocks();
  long double area = 0.0L;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t* d = &H.desc[6 * b];
    const int64_t kind = d[0], r0 = d[1], m = d[2], c0 = d[3], nn = d[4], r = d[5];
    if ((kind != 0 && kind != 1) || m < 1 || nn < 1 || r0 < 0 || c0 < 0 || r0 + m > n || c0 + nn > n || r < 0 ||
        (kind == 0 && r != 0) || (kind == 1 && r > std::min(m, nn)))
      fail(HMAT_EINVAL, "bad block descriptor " + std::to_string(b));
    const int64_t need = kind == 0 ? m * nn : r * (m + nn);
    if (H.off[b] < 0 || H.off[b] + need > (int64_t)H.values.size())
      fail(HMAT_EINVAL, "block " + std::to_string(b) + " values out of range");
    area += (long double)m * (long double)nn;
  }
  if (area != (long double)n * (long double)n) fail(HMAT_EINVAL, "blocks do not tile the matrix");
  // Overlap check on the finest row refinement.
  std::vector<int64_t> cuts;
  cuts.reserve(2 * nb + 2);
  for (int64_t b = 0; b < nb; ++b) {
    cuts.push_back(H.desc[6 * b + 1]);
    cuts.push_back(H.desc[6 * b + 1] + H.desc[6 * b + 2]);
  }
  std::sort(cuts.begin(), cuts.end());
  cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
  std::vector<std::vector<std::pair<int64_t, int64_t>>> spans(cuts.size());
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t* d = &H.desc[6 * b];
    auto lo = std::lower_bound(cuts.begin(), cuts.end(), d[1]) - cuts.begin();
    auto hi = std::lower_bound(cuts.begin(), cuts.end(), d[1] + d[2]) - cuts.begin();
    for (auto s = lo; s < hi; ++s) spans[s].push_back({d[3], d[3] + d[4]});
  }
  for (size_t s = 0; s + 1 < cuts.size(); ++s) {
    auto& v = spans[s];
    std::sort(v.begin(), v.end());
    int64_t at = 0;
    for (auto& p : v) {
      if (p.first != at) fail(HMAT_EINVAL, "blocks overlap or leave a gap");
      at = p.second;
    }
    if (at != n) fail(HMAT_EINVAL, "blocks leave a gap");
  }
}

}  // namespace hm
