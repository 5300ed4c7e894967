// CPU replay of the batched product's indexing (test infrastructure).
//
// Builds the blocks of a planar grid with the library's host construction,
// packs them with make_batched for several workgroup shapes, then walks
// every unit exactly as the HIP kernel does (same stage rounds, waves,
// lanes, input groups and reduction slots), asserting that every access
// stays inside its buffer, and compares the result with a direct product
// over the blocks.  Also checks that every panel entry is read exactly once.
//
// usage: layout_check nx ny h dip slip(0 strike,1 dip) leaf lattice eps
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

#include "hmat_internal.hpp"
#include "layout.hpp"

using namespace hm;

static void die(const char* m, long a = 0, long b = 0) {
  std::fprintf(stderr, "FAIL: %s (%ld, %ld)\n", m, a, b);
  std::exit(1);
}

// Pairs of a layout built with paired inputs: every phase-2 unit in exactly
// one pair, partners covering adjacent row intervals, equal common counts
// and identical leading sources.
template <typename T>
static void check_pairs(const BatchedLayout<T>& L) {
  std::vector<int> seen(L.n2, 0);
  if (L.pairs.size() % 2) die("pairs list of odd length");
  for (size_t i = 0; i < L.pairs.size(); i += 2) {
    const int32_t a = L.pairs[i], b = L.pairs[i + 1];
    if (a < 0 || a >= L.n2 || b < -1 || b >= L.n2) die("pair index", a, b);
    if (seen[a]++ || (b >= 0 && seen[b]++)) die("unit in two pairs", a, b);
    const Unit& ua = L.units[L.n1 + a];
    if (b < 0) {
      if (ua.ncom != 0) die("lone interval with common inputs", a, ua.ncom);
      continue;
    }
    const Unit& ub = L.units[L.n1 + b];
    if (ua.out0 + ua.nout != ub.out0) die("pair not adjacent", ua.out0, ub.out0);
    if (ua.ncom != ub.ncom || ua.ncom > ua.nin || ub.ncom > ub.nin) die("common count", ua.ncom, ub.ncom);
    for (int k = 0; k < ua.ncom; ++k)
      if (L.src[ua.in0 + k] != L.src[ub.in0 + k] || L.src[ua.in0 + k] == -1) die("common source differs", a, k);
  }
  for (int32_t k = 0; k < L.n2; ++k)
    if (!seen[k]) die("unit in no pair", k);
}

// kStage: inputs staged per round (2048 for one vector; the multi-vector
// product stages 1024 inputs of each of its R vectors).
template <typename T>
static double replay(const HostMatrix& H, int NW, int NW1, int64_t unit_bytes, const std::vector<double>& x,
                     const std::vector<double>& yref, int64_t split_slots = 0, int64_t* n_sums = nullptr,
                     bool pairs = false, int kStage = 2048) {
  constexpr int W = 16 / (int)sizeof(T);
  BatchedLayout<T> L = make_batched<T>(H, NW, unit_bytes, NW1, false, 0, split_slots, pairs);
  if (n_sums) *n_sums = (int64_t)L.sums.size() / 4;
  if (pairs) check_pairs(L);
  else if (!L.pairs.empty()) die("pairs without paired inputs");
  if (L.sums.size() % 4) die("sums not in groups of 4", (long)L.sums.size());
  // every partial slot belongs to exactly one sum; the main slot comes first
  std::vector<int> in_sum(L.t_size, 0);
  for (size_t j = 0; j < L.sums.size(); ++j) {
    const int32_t k = L.sums[j];
    if (k < 0 || k >= L.t_size) die("sum slot", (long)j, k);
    if (k > 0 && in_sum[k]++) die("slot in two sums", k);
    if (j % 4 == 0 && k == 0) die("sum without its main slot", (long)j);
  }
  const int64_t n = H.n;
  std::vector<double> t(L.t_size, 0.0), y(n, 0.0);
  std::vector<unsigned char> touched(L.pool.size(), 0);
  std::vector<int> y_written(n, 0);
  std::vector<int> t_written(L.t_size, 0);
  for (int pass = 1; pass <= 2; ++pass) {
    for (int32_t ui = 0; ui < L.n1 + L.n2; ++ui) {
      const Unit& u = L.units[ui];
      if (u.kind != pass) continue;
      if (ui < L.n1 && u.kind != 1) die("phase-2 unit among phase-1 units", ui);
      const int NWu = u.kind == 1 ? NW1 : NW;
      if (u.S < 1 || u.RG < 1 || u.S * u.RG > NWu) die("bad S/RG", u.S, u.RG);
      if (u.nout < 1 || u.nout > 64 * u.S) die("bad nout", u.nout, u.S);
      const int nin_pad = u.nq * W;
      std::vector<double> zs(kStage), red((size_t)NWu * 64, 0.0);
      std::vector<double> acc((size_t)NWu * 64, 0.0);
      if (u.kind == 2 && u.nin != nin_pad) die("phase-2 input list not padded to its groups", u.nin, nin_pad);
      for (int c0 = 0; c0 < nin_pad; c0 += kStage) {
        const int cl = std::min(kStage, nin_pad - c0);
        if (cl % W) die("stage not a multiple of W", cl);
        {
          // the kernels stage in batches of B inputs per thread (single vector:
          // up to 4; multi-vector: 2, or 1 when a round has one input per
          // thread): index loads clamped to the unit's list, LDS slots below kStage
          const int NT = NWu * 64;
          const int B = kStage == 2048 ? std::min(4, kStage / NT) : (kStage / NT >= 2 ? 2 : 1);
          if (B < 1 || kStage % (B * NT) != 0) die("staging batch", B, NT);
          for (int i0 = 0; i0 < cl; i0 += B * NT)
            for (int i = i0; i < i0 + B * NT; ++i) {
              if (i >= kStage) die("stage slot", i);
              const int gi = c0 + i;
              const int64_t idx = (int64_t)u.in0 + std::max(0, std::min(gi, u.nin - 1));
              if (u.kind == 1 ? idx >= n : idx >= (int64_t)L.src.size()) die("clamped index load", (long)idx);
            }
        }
        for (int i = 0; i < cl; ++i) {
          const int gi = c0 + i;
          double v = 0.0;
          if (u.kind == 1) {
            if (gi < u.nin) {
              if (u.in0 + gi >= n) die("perm index", u.in0 + gi);
              v = x[H.perm[u.in0 + gi]];
            }
          } else {
            if ((int64_t)u.in0 + gi >= (int64_t)L.src.size()) die("src index", u.in0 + gi);
            const int s = L.src[u.in0 + gi];
            if (s >= 0) {
              if (s >= n) die("x index", s);
              v = x[s];
            } else if (-s - 1 < L.t_size) {
              if (-s - 1 > 0 && in_sum[-s - 1]) die("split value read as a whole", -s - 1);
              if (-s - 1 > 0 && !t_written[-s - 1]) die("t read before written", -s - 1);
              v = t[-s - 1];
            } else {
              const int64_t j = -(int64_t)s - 1 - L.t_size;
              if (j >= (int64_t)L.sums.size() / 4) die("sum index", (long)j);
              v = 0.0;
              for (int p = 0; p < 4; ++p) {
                const int32_t k = L.sums[4 * j + p];
                if (k > 0 && !t_written[k]) die("partial read before written", k);
                v += t[k];
              }
            }
          }
          zs[i] = v;
        }
        for (int wave = 0; wave < NWu; ++wave) {
          const bool working = wave < u.S * u.RG;
          const int sg = wave % u.S, rg = wave / u.S;
          for (int lane = 0; lane < 64; ++lane) {
            const int o = sg * 64 + lane;
            if (!(working && o < u.nout)) continue;
            const int q0 = c0 / W, q1 = q0 + cl / W;
            for (int q = q0 + rg; q < q1; q += u.RG) {
              for (int c = 0; c < W; ++c) {
                const int64_t e = u.off + ((int64_t)q * u.nout + o) * W + c;
                if (e < 0 || e >= (int64_t)L.pool.size()) die("pool index", (long)e);
                if (touched[e]++) die("panel entry read twice", (long)e);
                const int zi = (q - q0) * W + c;
                if (zi < 0 || zi >= cl) die("stage index", zi);
                acc[wave * 64 + lane] += (double)L.pool[e] * zs[zi];
              }
            }
          }
        }
      }
      for (int wave = 0; wave < NWu; ++wave) {
        const int sg = wave % u.S, rg = wave / u.S;
        if (rg != 0) continue;
        for (int lane = 0; lane < 64; ++lane) {
          const int o = sg * 64 + lane;
          if (o >= u.nout) continue;
          double sum = 0.0;
          for (int r = 0; r < u.RG; ++r) {
            const int idx = (r * u.S + sg) * 64 + lane;
            if (idx >= NWu * 64) die("reduction index", idx);
            sum += acc[idx];
          }
          if (u.kind == 1) {
            const int64_t ti = (int64_t)u.out0 + o;
            if (ti < 1 || ti >= L.t_size) die("t output index", (long)ti);
            if (t_written[ti]++) die("t written twice", (long)ti);
            t[ti] = sum;
          } else {
            const int64_t row = (int64_t)u.out0 + o;
            if (row < 0 || row >= n) die("row index", (long)row);
            if (y_written[row]++) die("row written twice", (long)row);
            y[H.perm[row]] = sum;
          }
        }
      }
    }
  }
  for (int64_t i = 0; i < n; ++i)
    if (y_written[i] != 1) die("row not written once", (long)i, y_written[i]);
  for (int64_t k = 1; k < L.t_size; ++k)
    if (t_written[k] != 1) die("intermediate value not written once", (long)k, t_written[k]);
  // every non-padding panel entry must have been read (padding entries are 0)
  for (size_t e = 0; e < L.pool.size(); ++e)
    if (!touched[e] && L.pool[e] != T(0)) die("nonzero panel entry never read", (long)e);
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    num += (y[i] - yref[i]) * (y[i] - yref[i]);
    den += yref[i] * yref[i];
  }
  return std::sqrt(num / den);
}

int main(int argc, char** argv) {
  if (argc != 9) die("usage");
  const int nx = std::atoi(argv[1]), ny = std::atoi(argv[2]);
  const double h = std::atof(argv[3]), dip = std::atof(argv[4]);
  const int slip = std::atoi(argv[5]), leaf = std::atoi(argv[6]), lattice = std::atoi(argv[7]);
  const double eps = std::atof(argv[8]);
  const int64_t n = (int64_t)nx * ny;
  // planar grid of squares, as the synthetic workloads build it
  const double c = dip == 90.0 ? 0.0 : std::cos(dip * M_PI / 180.0);
  const double s = dip == 90.0 ? 1.0 : std::sin(dip * M_PI / 180.0);
  std::vector<double> verts(n * 12), sd(n * 3);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t iy = k / nx, ix = k % nx;
    const double xs[4] = {ix * h, (ix + 1) * h, (ix + 1) * h, ix * h};
    const double ds[4] = {iy * h, iy * h, (iy + 1) * h, (iy + 1) * h};
    for (int v = 0; v < 4; ++v) {
      verts[k * 12 + 3 * v] = xs[v];
      verts[k * 12 + 3 * v + 1] = ds[v] * c;
      verts[k * 12 + 3 * v + 2] = -ds[v] * s;
    }
    if (slip == 0) { sd[3 * k] = 1; sd[3 * k + 1] = 0; sd[3 * k + 2] = 0; }
    else { sd[3 * k] = 0; sd[3 * k + 1] = -c; sd[3 * k + 2] = s; }
  }
  hmat_mesh mesh{n, 4, verts.data(), sd.data()};
  hmat_green green{HMAT_GF_FS_RECT_COPLANAR, 0, 32e9, 0.25};
  Geometry geo;
  std::unique_ptr<EntryFn> E(make_entry_fn(mesh, green, geo));
  ClusterTree tree = build_tree(geo, leaf);
  HostMatrix H = assemble(*E, tree, partition(tree, lattice, 2.0), eps, 0, 0);
  std::vector<double> x(n), yref(n, 0.0), yc(n, 0.0);
  for (int64_t i = 0; i < n; ++i) x[i] = std::pow(10.0, -12.0 + 3.0 * std::fmod(0.6180339887 * (i + 1), 1.0));
  for (int64_t b = 0; b < H.nblocks(); ++b) {  // direct product over the blocks
    const int64_t* d = &H.desc[6 * b];
    const double* v = &H.values[H.off[b]];
    if (d[0] == 0) {
      for (int64_t j = 0; j < d[4]; ++j)
        for (int64_t i = 0; i < d[2]; ++i) yc[d[1] + i] += v[j * d[2] + i] * x[H.perm[d[3] + j]];
    } else {
      for (int64_t k = 0; k < d[5]; ++k) {
        double tk = 0.0;
        for (int64_t j = 0; j < d[4]; ++j) tk += v[d[2] * d[5] + k * d[4] + j] * x[H.perm[d[3] + j]];
        for (int64_t i = 0; i < d[2]; ++i) yc[d[1] + i] += v[k * d[2] + i] * tk;
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) yref[H.perm[i]] = yc[i];
  // transpose: direct product with H^T over the original blocks
  std::vector<double> yrefT(n, 0.0), ycT(n, 0.0);
  for (int64_t b = 0; b < H.nblocks(); ++b) {
    const int64_t* d = &H.desc[6 * b];
    const double* v = &H.values[H.off[b]];
    if (d[0] == 0) {
      for (int64_t j = 0; j < d[4]; ++j)
        for (int64_t i = 0; i < d[2]; ++i) ycT[d[3] + j] += v[j * d[2] + i] * x[H.perm[d[1] + i]];
    } else {
      for (int64_t k = 0; k < d[5]; ++k) {
        double sk = 0.0;
        for (int64_t i = 0; i < d[2]; ++i) sk += v[k * d[2] + i] * x[H.perm[d[1] + i]];
        for (int64_t j = 0; j < d[4]; ++j) ycT[d[3] + j] += v[d[2] * d[5] + k * d[4] + j] * sk;
      }
    }
  }
  for (int64_t i = 0; i < n; ++i) yrefT[H.perm[i]] = ycT[i];
  const HostMatrix HT = transpose_host(H);
  // packing H^T in place gives the same layout as packing the transposed copy
  for (int NW1 : {4, 8}) {
    const BatchedLayout<float> a = make_batched<float>(HT, 8, 256 << 10, NW1);
    const BatchedLayout<float> b = make_batched<float>(H, 8, 256 << 10, NW1, true, 3);
    if (a.pool != b.pool || a.src != b.src || a.n1 != b.n1 || a.n2 != b.n2 || a.t_size != b.t_size ||
        a.units.size() != b.units.size())
      die("in-place transpose packing differs", NW1);
    for (size_t k = 0; k < a.units.size(); ++k)
      if (std::memcmp(&a.units[k], &b.units[k], sizeof(Unit)) != 0) die("in-place transpose unit differs", (long)k);
  }
  for (int NW : {4, 8}) {
    const double r64 = replay<double>(HT, NW, 4, 256 << 10, x, yrefT);
    const double r32 = replay<float>(HT, NW, 4, 256 << 10, x, yrefT);
    std::printf("transpose NW=%d rel64=%.3e rel32=%.3e\n", NW, r64, r32);
    if (!(r64 < 1e-13) || !(r32 < 1e-6)) die("replayed transpose product differs");
  }
  for (int NW : {4, 8, 16})
    for (int NW1 : {4, 8, 16})
    for (int64_t ub : {64 << 10, 4 << 20}) {
      const double r64 = replay<double>(H, NW, NW1, ub, x, yref);
      const double r32 = replay<float>(H, NW, NW1, ub, x, yref);
      std::printf("NW=%d NW1=%d unit=%ld rel64=%.3e rel32=%.3e\n", NW, NW1, (long)ub, r64, r32);
      if (!(r64 < 1e-13) || !(r32 < 1e-6)) die("replayed product differs");
    }
  // phase-1 units split by rows (partial values added by phase 2)
  for (int NW1 : {4, 8}) {
    int64_t ns64 = 0, ns32 = 0;
    const double r64 = replay<double>(H, 8, NW1, 256 << 10, x, yref, 1 << 20, &ns64);
    const double r32 = replay<float>(H, 8, NW1, 256 << 10, x, yref, 1 << 20, &ns32);
    std::printf("split NW1=%d sums %ld/%ld rel64=%.3e rel32=%.3e\n", NW1, (long)ns64, (long)ns32, r64, r32);
    if (!(r64 < 1e-13) || !(r32 < 1e-6)) die("replayed split product differs");
  }
  // staging rounds of the multi-vector product (1024 inputs per vector), and shorter
  for (int ks : {1024, 512}) {
    const double r64 = replay<double>(H, 8, 4, 256 << 10, x, yref, 0, nullptr, false, ks);
    const double r32 = replay<float>(H, 8, 4, 256 << 10, x, yref, 1 << 20, nullptr, false, ks);
    std::printf("rounds of %d inputs rel64=%.3e rel32=%.3e\n", ks, r64, r32);
    if (!(r64 < 1e-13) || !(r32 < 1e-6)) die("replayed product with shorter rounds differs");
  }
  // inputs ordered in pairs of intervals (layouts of handles with ensemble buffers)
  for (int NW : {4, 8}) {
    const double r64 = replay<double>(H, NW, 4, 256 << 10, x, yref, 0, nullptr, true);
    const double r32 = replay<float>(H, NW, 4, 256 << 10, x, yref, 0, nullptr, true);
    std::printf("pairs NW=%d rel64=%.3e rel32=%.3e\n", NW, r64, r32);
    if (!(r64 < 1e-13) || !(r32 < 1e-6)) die("replayed product with paired inputs differs");
  }
  std::printf("OK\n");
  return 0;
}
