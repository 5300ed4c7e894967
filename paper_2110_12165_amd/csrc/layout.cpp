// Host-side packing of a block list into the device layouts.
#include "layout.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>

namespace hm {
namespace {

template <typename T>
int64_t align_elems(int64_t off) {
  const int64_t a = 256 / (int64_t)sizeof(T);
  return (off + a - 1) / a * a;
}

// Block b of H, or of H^T with tr set (rows and columns exchanged, the dense
// part transposed, U and V exchanged), read in place.
struct BlockView {
  const HostMatrix& H;
  bool tr;
  const int64_t* d(int64_t b) const { return &H.desc[6 * b]; }
  int64_t kind(int64_t b) const { return d(b)[0]; }
  int64_t r0(int64_t b) const { return d(b)[tr ? 3 : 1]; }
  int64_t m(int64_t b) const { return d(b)[tr ? 4 : 2]; }
  int64_t c0(int64_t b) const { return d(b)[tr ? 1 : 3]; }
  int64_t n(int64_t b) const { return d(b)[tr ? 2 : 4]; }
  int64_t rank(int64_t b) const { return d(b)[5]; }
  // Column j of the dense block as (first entry, stride between rows).
  std::pair<const double*, int64_t> dense_col(int64_t b, int64_t j) const {
    const double* v = &H.values[H.off[b]];
    const int64_t mh = d(b)[2];
    return tr ? std::make_pair(v + j, mh) : std::make_pair(v + j * mh, (int64_t)1);
  }
  // Column kk of U (length m) and of V (length n), contiguous.
  const double* u_col(int64_t b, int64_t kk) const {
    const double* v = &H.values[H.off[b]];
    return tr ? v + d(b)[2] * d(b)[5] + kk * d(b)[4] : v + kk * d(b)[2];
  }
  const double* v_col(int64_t b, int64_t kk) const {
    const double* v = &H.values[H.off[b]];
    return tr ? v + kk * d(b)[2] : v + d(b)[2] * d(b)[5] + kk * d(b)[4];
  }
};

inline int32_t to_i32(int64_t v, const char* what) {
  if (v < 0 || v > INT32_MAX) fail(HMAT_EUNSUPPORTED, std::string(what) + " exceeds the 32-bit range of the layout");
  return (int32_t)v;
}

// For each refined interval, the blocks that contain it (block order) and
// the interval's offset inside each block.
struct Incidence {
  std::vector<std::pair<int64_t, int64_t>> iv;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> members;  // (block, offset)
};

Incidence incidence(const HostMatrix& H, bool columns, int64_t cap) {
  Incidence I;
  I.iv = refine_ranges(H, columns, cap);
  I.members.resize(I.iv.size());
  std::vector<int64_t> starts(I.iv.size());
  for (size_t k = 0; k < I.iv.size(); ++k) starts[k] = I.iv[k].first;
  const int64_t nb = H.nblocks();
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t* d = &H.desc[6 * b];
    const int64_t lo = columns ? d[3] : d[1];
    const int64_t len = columns ? d[4] : d[2];
    size_t k = std::lower_bound(starts.begin(), starts.end(), lo) - starts.begin();
    for (; k < I.iv.size() && I.iv[k].first < lo + len; ++k)
      I.members[k].push_back({(int32_t)b, (int32_t)(I.iv[k].first - lo)});
  }
  return I;
}

}  // namespace

std::vector<std::pair<int64_t, int64_t>> refine_ranges(const HostMatrix& H, bool columns, int64_t cap) {
  std::vector<int64_t> cuts{0, H.n};
  for (int64_t b = 0; b < H.nblocks(); ++b) {
    const int64_t* d = &H.desc[6 * b];
    const int64_t lo = columns ? d[3] : d[1];
    const int64_t len = columns ? d[4] : d[2];
    cuts.push_back(lo);
    cuts.push_back(lo + len);
  }
  std::sort(cuts.begin(), cuts.end());
  cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
  std::vector<std::pair<int64_t, int64_t>> out;
  for (size_t k = 0; k + 1 < cuts.size(); ++k) {
    const int64_t a = cuts[k], b = cuts[k + 1];
    const int64_t parts = (b - a + cap - 1) / cap;
    for (int64_t p = 0; p < parts; ++p) out.push_back({a + (b - a) * p / parts, a + (b - a) * (p + 1) / parts});
  }
  return out;
}

HostMatrix transpose_host(const HostMatrix& H) {
  HostMatrix T;
  T.n = H.n;
  T.perm = H.perm;
  T.lattice = H.lattice;
  T.tree_depth = H.tree_depth;
  const int64_t nb = H.nblocks();
  T.desc.resize(6 * nb);
  T.off = H.off;
  T.values.resize(H.values.size());
  parallel_for(nb, 0, [&](int64_t b) {
    const int64_t* d = &H.desc[6 * b];
    int64_t* e = &T.desc[6 * b];
    const int64_t m = d[2], n = d[4], r = d[5];
    e[0] = d[0];
    e[1] = d[3];
    e[2] = n;
    e[3] = d[1];
    e[4] = m;
    e[5] = r;
    const double* v = &H.values[H.off[b]];
    double* w = &T.values[H.off[b]];
    if (d[0] == 0) {
      for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) w[i * n + j] = v[j * m + i];  // D^T, column-major n x m
    } else {
      std::copy(v + m * r, v + (m + n) * r, w);      // U' = V (n x r)
      std::copy(v, v + m * r, w + n * r);            // V' = U (m x r)
    }
  });
  return T;
}

template <typename T>
PlainLayout<T> make_plain(const HostMatrix& H, bool transpose, int32_t n_threads) {
  PlainLayout<T> L;
  const int64_t nb = H.nblocks();
  L.blocks.resize(nb);
  int64_t off = 0, tslot = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t* d = &H.desc[6 * b];
    PlainBlock& p = L.blocks[b];
    p.kind = (int32_t)d[0];
    p.r0 = to_i32(d[1], "row");
    p.m = to_i32(d[2], "block rows");
    p.c0 = to_i32(d[3], "column");
    p.n = to_i32(d[4], "block columns");
    p.rank = to_i32(d[5], "rank");
    p.pad = 0;
    p.tslot = to_i32(tslot, "total rank");
    if (p.kind == 0) {
      p.offA = off = align_elems<T>(off);
      p.offB = 0;
      off += d[2] * d[4];
    } else {
      p.offA = off = align_elems<T>(off);
      off += d[2] * d[5];
      p.offB = off = align_elems<T>(off);
      off += d[4] * d[5];
      tslot += d[5];
      if (d[5] > 0) L.lr_list.push_back((int32_t)b);
    }
  }
  L.sum_rank = tslot;
  L.pool.resize(align_elems<T>(off) + 256 / sizeof(T));
  parallel_zero(L.pool.data(), (int64_t)L.pool.size(), n_threads);
  parallel_for(nb, n_threads, [&](int64_t b) {
    const int64_t* d = &H.desc[6 * b];
    const double* v = &H.values[H.off[b]];
    const PlainBlock& p = L.blocks[b];
    if (p.kind == 0) {
      for (int64_t k = 0; k < d[2] * d[4]; ++k) L.pool[p.offA + k] = (T)v[k];
    } else {
      for (int64_t k = 0; k < d[2] * d[5]; ++k) L.pool[p.offA + k] = (T)v[k];
      for (int64_t k = 0; k < d[4] * d[5]; ++k) L.pool[p.offB + k] = (T)v[d[2] * d[5] + k];
    }
  });
  for (int pass = 0; pass < (transpose ? 2 : 1); ++pass) {
    Incidence I = incidence(H, pass == 1, 64);
    auto& units = pass == 0 ? L.row_units : L.col_units;
    auto& ents = pass == 0 ? L.row_entries : L.col_entries;
    for (size_t k = 0; k < I.iv.size(); ++k) {
      RowUnit u;
      u.row0 = (int32_t)I.iv[k].first;
      u.m = (int32_t)(I.iv[k].second - I.iv[k].first);
      u.begin = to_i32((int64_t)ents.size(), "unit entries");
      for (auto& e : I.members[k]) {
        const PlainBlock& p = L.blocks[e.first];
        if (p.kind == 1 && p.rank == 0) continue;
        ents.push_back({e.first, e.second});
      }
      u.end = to_i32((int64_t)ents.size(), "unit entries");
      units.push_back(u);
    }
  }
  return L;
}

template <typename T>
BatchedLayout<T> make_batched(const HostMatrix& H, int32_t wg_waves, int64_t unit_bytes, int32_t wg_waves_p1,
                              bool transpose, int32_t n_threads, int64_t split_slots, bool pair_inputs) {
  constexpr int W = 16 / (int)sizeof(T);
  BatchedLayout<T> L;
  L.wg_waves = wg_waves;
  L.wg_waves_p1 = wg_waves_p1;
  L.unit_bytes = unit_bytes;
  const int64_t nb = H.nblocks();
  const BlockView B{H, transpose};

  // ---- phase 1: group low-rank blocks by their column cluster -------------
  // A unit covers the rows of its cluster (all of them, or with split_rows
  // one of P <= 4 row ranges of a cluster whose units would be far larger
  // than the others: each part then writes its own partial intermediate
  // values, added by phase 2).  Waves of a unit split its rows into RG
  // groups (at least kMinQuads input groups each) and the outputs into S
  // groups of 64.
  constexpr int64_t kMinQuads = 16;
  constexpr int kMaxParts = 4;
  struct Group {
    int64_t c0, n;
    std::vector<int32_t> blocks;
    int64_t R = 0, base = 0;
    int S = 1, RG = 1, P = 1;
    int64_t nq_part = 0;           // input groups per row part
    int64_t xbase[kMaxParts] = {};  // first slot of each part's values (part 0: base)
  };
  std::vector<Group> groups;
  std::map<std::pair<int64_t, int64_t>, size_t> gid;
  for (int64_t b = 0; b < nb; ++b) {
    if (B.kind(b) != 1 || B.rank(b) == 0) continue;
    auto key = std::make_pair(B.c0(b), B.n(b));
    auto it = gid.find(key);
    if (it == gid.end()) {
      it = gid.emplace(key, groups.size()).first;
      Group g;
      g.c0 = B.c0(b);
      g.n = B.n(b);
      groups.push_back(g);
    }
    groups[it->second].blocks.push_back((int32_t)b);
    groups[it->second].R += B.rank(b);
  }
  // Row parts (small matrices only): a 64-output unit of a group is split
  // when it is more than twice the mean 64-output unit.  Measured: N = 21000
  // 58.6 -> 49.0 us per product; at N = 122880 (5.6 units per slot) the
  // extra units and partial values cost more than the shorter tail gains.
  double mean64 = 0.0;
  bool split_rows = false;
  {
    double tot = 0.0, cnt = 0.0;
    for (const auto& g : groups) {
      const double u64 = (double)((g.R + 63) / 64);
      tot += u64 * 64.0 * (double)((g.n + W - 1) / W);
      cnt += u64;
    }
    mean64 = cnt > 0 ? tot / cnt : 0.0;
    split_rows = split_slots > 0 && cnt < 2.0 * (double)split_slots;
  }
  std::vector<int64_t> slot_of_block(nb, -1);  // t index of (block, column 0)
  int64_t t = 1;                                // t[0] is the zero pad
  for (auto& g : groups) {
    // Row groups first (at least kMinQuads input groups per wave), then as
    // many output groups as the remaining waves allow.  Measured on the
    // benchmark fault: more, shorter per-wave loops beat fewer, fuller units.
    const int64_t nq = (g.n + W - 1) / W;
    int P = 1;
    if (split_rows && mean64 > 0.0) {
      const double ratio = 64.0 * (double)nq / (2.0 * mean64);
      if (ratio > 1.0) P = (int)std::min<double>(kMaxParts, std::ceil(ratio));
      while (P > 1 && nq / P < kMinQuads) --P;
    }
    g.P = P;
    g.nq_part = (nq + P - 1) / P;
    g.RG = (int)std::max<int64_t>(1, std::min<int64_t>(wg_waves_p1, g.nq_part / kMinQuads));
    const int64_t need = (g.R + 63) / 64;
    g.S = (int)std::max<int64_t>(1, std::min<int64_t>(need, wg_waves_p1 / g.RG));
    while (g.S > 1 && 64LL * g.S * g.nq_part * W * (int64_t)sizeof(T) > unit_bytes) --g.S;
    g.base = t;
    g.xbase[0] = t;
    for (int32_t b : g.blocks) {
      slot_of_block[b] = t;
      t += B.rank(b);
    }
  }
  const int64_t t_main = t;
  for (auto& g : groups)
    for (int p = 1; p < g.P; ++p) {
      g.xbase[p] = t;
      t += g.R;
    }
  L.t_size = t;
  to_i32(t + 1, "intermediate values");
  // partial values of each split intermediate value, added in part order
  std::vector<int32_t> sum_of_slot(t_main, -1);
  for (const auto& g : groups) {
    if (g.P == 1) continue;
    for (int64_t k = 0; k < g.R; ++k) {
      sum_of_slot[g.base + k] = (int32_t)(L.sums.size() / 4);
      for (int p = 0; p < kMaxParts; ++p) L.sums.push_back(p < g.P ? (int32_t)(g.xbase[p] + k) : 0);
    }
  }
  to_i32(L.t_size + (int64_t)L.sums.size() / 4 + 1, "intermediate values and their sums");

  struct Pending { Unit u; int kind; size_t g; int64_t s0; int64_t r0; };
  int64_t off = 0;
  std::vector<Pending> pend;
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    const Group& g = groups[gi];
    const int64_t NS = 64LL * g.S;
    for (int64_t s0 = 0; s0 < g.R; s0 += NS) {
      const int64_t ns = std::min(NS, g.R - s0);
      for (int p = 0; p < g.P; ++p) {
        const int64_t r0 = (int64_t)p * g.nq_part * W;
        const int64_t rows = std::min(g.n - r0, g.nq_part * W);
        if (rows <= 0) continue;
        Unit u{};
        u.kind = 1;
        u.nout = (int32_t)ns;
        u.nq = to_i32((rows + W - 1) / W, "unit inputs");
        u.S = (int32_t)((ns + 63) / 64);
        u.RG = g.RG;
        u.in0 = to_i32(g.c0 + r0, "row");
        u.nin = (int32_t)rows;
        u.out0 = to_i32(g.xbase[p] + s0, "intermediate index");
        u.off = 0;
        pend.push_back({u, 1, gi, s0, r0});
      }
    }
  }
  // ---- phase 2: one unit per refined row interval --------------------------
  // Inputs of an interval: the columns of every dense block meeting it, then
  // the rank columns of every low-rank block meeting it (Col: block, column
  // or rank index, the interval's first row inside the block, source).
  struct Col {
    int32_t b, j, i0, src;
  };
  Incidence I = incidence(H, transpose, 64);
  std::vector<std::vector<Col>> cols(I.iv.size());
  for (size_t k = 0; k < I.iv.size(); ++k)
    for (int pass = 0; pass < 2; ++pass)
      for (auto& e : I.members[k]) {
        const int64_t b = e.first;
        if (pass == 0 && B.kind(b) == 0) {
          for (int64_t j = 0; j < B.n(b); ++j)
            cols[k].push_back({(int32_t)b, (int32_t)j, e.second, H.perm[B.c0(b) + j]});
        } else if (pass == 1 && B.kind(b) == 1 && B.rank(b) > 0) {
          for (int64_t kk = 0; kk < B.rank(b); ++kk) {
            const int64_t slot = slot_of_block[b] + kk;
            const int64_t j = sum_of_slot[slot];
            cols[k].push_back({(int32_t)b, (int32_t)kk, e.second,
                               j < 0 ? -(int32_t)slot - 1 : -(int32_t)(L.t_size + j) - 1});
          }
        }
      }
  // pairs of consecutive intervals: the inputs both use first, in the order
  // of the first interval's list, then each interval's own
  std::vector<int32_t> ncom(I.iv.size(), 0);
  if (pair_inputs) {
    parallel_for((int64_t)I.iv.size() / 2, n_threads, [&](int64_t pj) {
      std::vector<Col>& a = cols[2 * pj];
      std::vector<Col>& b = cols[2 * pj + 1];
      std::map<int32_t, size_t> in_b;
      for (size_t i = 0; i < b.size(); ++i) in_b.emplace(b[i].src, i);
      std::vector<Col> na, nb, ra;
      std::vector<char> taken(b.size(), 0);
      for (const Col& c : a) {
        auto it = in_b.find(c.src);
        if (it == in_b.end()) {
          ra.push_back(c);
        } else {
          na.push_back(c);
          nb.push_back(b[it->second]);
          taken[it->second] = 1;
        }
      }
      ncom[2 * pj] = ncom[2 * pj + 1] = (int32_t)na.size();
      na.insert(na.end(), ra.begin(), ra.end());
      for (size_t i = 0; i < b.size(); ++i)
        if (!taken[i]) nb.push_back(b[i]);
      a.swap(na);
      b.swap(nb);
    });
  }
  for (size_t k = 0; k < I.iv.size(); ++k) {
    const int64_t a = I.iv[k].first, m = I.iv[k].second - I.iv[k].first;
    Unit u{};
    u.kind = 2;
    u.nout = (int32_t)m;
    u.S = 1;
    u.RG = wg_waves;
    u.in0 = to_i32((int64_t)L.src.size(), "input list");
    u.out0 = (int32_t)a;
    u.ncom = ncom[k];
    int64_t K = 0;
    for (const Col& c : cols[k]) {
      L.src.push_back(c.src);
      ++K;
    }
    while (K % W) {
      L.src.push_back(-1);
      ++K;
    }
    u.nq = to_i32(K / W, "unit inputs");
    u.nin = (int32_t)K;
    u.off = 0;
    pend.push_back({u, 2, k, 0, 0});
  }
  to_i32((int64_t)L.src.size(), "input list");
  // Dispatch order: phase 1 before phase 2, larger units first.  Panels are
  // laid out in that same order, so workgroups running at the same time
  // stream neighbouring regions of the pool.
  auto bytes = [](const Unit& u) { return (int64_t)u.nq * u.nout; };
  std::stable_sort(pend.begin(), pend.end(), [&](const Pending& a, const Pending& b) {
    if (a.kind != b.kind) return a.kind < b.kind;
    return bytes(a.u) > bytes(b.u);
  });
  for (auto& p : pend) {
    p.u.off = off = align_elems<T>(off);
    off += (int64_t)p.u.nq * W * p.u.nout;
  }
  L.pool.resize(align_elems<T>(off) + 256 / sizeof(T));
  parallel_zero(L.pool.data(), (int64_t)L.pool.size(), n_threads);

  // ---- fill panels (units own disjoint pool ranges) -------------------------
  parallel_for((int64_t)pend.size(), n_threads, [&](int64_t pi) {
    const Pending& p = pend[pi];
    const Unit& u = p.u;
    T* dst = &L.pool[u.off];
    if (p.kind == 1) {
      const Group& g = groups[p.g];
      // local output slot o of this unit -> column of V of one block
      std::vector<const double*> sl(u.nout);
      {
        int64_t s = 0, o = 0;
        for (int32_t b : g.blocks)
          for (int64_t kk = 0; kk < B.rank(b); ++kk, ++s)
            if (s >= p.s0 && s < p.s0 + u.nout) sl[o++] = B.v_col(b, kk);
      }
      for (int64_t q = 0; q < u.nq; ++q)
        for (int64_t o = 0; o < u.nout; ++o) {
          const double* V = sl[o] + p.r0;  // rows of this part
          for (int c = 0; c < W; ++c) {
            const int64_t j = q * W + c;
            dst[(q * u.nout + o) * W + c] = j < u.nin ? (T)V[j] : T(0);
          }
        }
    } else {
      const int64_t m = u.nout;
      int64_t col = 0;
      // colv[i * stride] = coefficient of row i of this unit
      auto put = [&](const double* colv, int64_t stride) {
        const int64_t q = col / W, c = col % W;
        for (int64_t o = 0; o < m; ++o) dst[(q * m + o) * W + c] = colv ? (T)colv[o * stride] : T(0);
        ++col;
      };
      for (const Col& c : cols[p.g]) {
        if (B.kind(c.b) == 0) {
          const auto cs = B.dense_col(c.b, c.j);
          put(cs.first + (int64_t)c.i0 * cs.second, cs.second);
        } else {
          put(B.u_col(c.b, c.j) + c.i0, 1);
        }
      }
      while (col % W) put(nullptr, 0);
    }
  });
  std::vector<Unit> p1, p2;
  std::vector<int32_t> unit_of_interval(I.iv.size(), -1);
  for (auto& p : pend) {
    if (p.kind == 2) unit_of_interval[p.g] = (int32_t)p2.size();
    (p.kind == 1 ? p1 : p2).push_back(p.u);
  }
  L.n1 = (int32_t)p1.size();
  L.n2 = (int32_t)p2.size();
  if (pair_inputs) {
    std::vector<std::pair<int64_t, std::pair<int32_t, int32_t>>> pr;
    for (size_t k = 0; k < I.iv.size(); k += 2) {
      const int32_t ua = unit_of_interval[k];
      const int32_t ub = k + 1 < I.iv.size() ? unit_of_interval[k + 1] : -1;
      const int64_t sz = (int64_t)p2[ua].nq * p2[ua].nout + (ub >= 0 ? (int64_t)p2[ub].nq * p2[ub].nout : 0);
      pr.push_back({sz, {ua, ub}});
    }
    std::stable_sort(pr.begin(), pr.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    for (const auto& e : pr) {
      L.pairs.push_back(e.second.first);
      L.pairs.push_back(e.second.second);
    }
  }
  L.units = std::move(p1);
  L.units.insert(L.units.end(), p2.begin(), p2.end());
  return L;
}

template PlainLayout<float> make_plain<float>(const HostMatrix&, bool, int32_t);
template PlainLayout<double> make_plain<double>(const HostMatrix&, bool, int32_t);
template BatchedLayout<float> make_batched<float>(const HostMatrix&, int32_t, int64_t, int32_t, bool, int32_t,
                                                  int64_t, bool);
template BatchedLayout<double> make_batched<double>(const HostMatrix&, int32_t, int64_t, int32_t, bool, int32_t,
                                                    int64_t, bool);

}  // namespace hm
