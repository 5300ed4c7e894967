// Construction of the block list on the device (section 3.1.2, eqs.
// (18)-(19); entries of eqs. (5)-(6)).
//
// The cluster tree and the block partition come from the host; the GPU then
//   * runs the adaptive cross approximation of every admissible block, one
//     workgroup per block, with the host's rules (build_aca.cpp): partial
//     pivoting from the first row, column pivot = largest residual (lowest
//     index on ties), zero residual row -> lowest unused row, incremental
//     Frobenius estimate, stop when |u| |v| <= eps ||U V^T||_F, dense
//     fallback when k (m + n) >= m n or k reaches max_rank;
//   * evaluates every dense block (and every block that fell back to dense);
//   * packs the factors of each low-rank block (U then V, column-major).
// Reductions combine wave sums in a fixed order, so a build is reproducible.
// Entries come from entries.hpp, the formulas of the host construction.
// A block whose rank would pass kAcaCap, or whose rows do not fit the LDS
// row mask, is approximated on the host instead (same rules).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <string>

#include "hmat_internal.hpp"

namespace hm {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kAcaCap = 64;          // ranks kept on the device per block
constexpr int kMaxMaskRows = 49152;  // rows of the LDS used-row mask

struct AcaBlock {
  long long r0, m, c0, n, off;  // off: scratch offset (U: kAcaCap m, then V: kAcaCap n)
  int kmax, pad;
};

struct FillBlock {
  long long r0, m, c0, n, off;  // off: output offset (m n, column-major)
};

struct PackBlock {
  long long m, n, src, dst;  // src: scratch offset, dst: packed offset
  int k, pad;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// largest value, lowest index on ties
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const double ov = __shfl_xor(v, d, 64);
    const int oi = __shfl_xor(i, d, 64);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
  return v;
}

// Workgroup argmax (uniform result); sv/si: LDS scratch of kWaves entries.
__device__ __forceinline__ void block_argmax(double& v, int& i, double* sv, int* si) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  wave_argmax(v, i);
  if (lane == 0) {
    sv[wave] = v;
    si[wave] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
  for (int w = 1; w < kWaves; ++w)
    if (sv[w] > v || (sv[w] == v && si[w] < i)) {
      v = sv[w];
      i = si[w];
    }
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_aca(EntryView E, const long long* __restrict__ perm,
                                                   const AcaBlock* __restrict__ blocks, double* __restrict__ scratch,
                                                   double eps, int* __restrict__ rank_out,
                                                   int* __restrict__ status_out) {
  extern __shared__ double dyn[];
  double* red = dyn;                          // kWaves x (2 kAcaCap + 2)
  double* ui = red + kWaves * (2 * kAcaCap + 2);  // U[i, l], l < k
  double* vj = ui + kAcaCap;                  // V[jp, l], l < k
  unsigned char* used = reinterpret_cast<unsigned char*>(vj + kAcaCap);
  __shared__ double sv[kWaves];
  __shared__ int si[kWaves];
  const AcaBlock B = blocks[blockIdx.x];
  const int m = (int)B.m, n = (int)B.n;
  const long long* rows = perm + B.r0;
  const long long* cols = perm + B.c0;
  double* U = scratch + B.off;                 // column l at U + l m
  double* V = U + (long long)kAcaCap * m;      // column l at V + l n
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int ld = 2 * kAcaCap + 2;
  for (int q = tid; q < m; q += kThreads) used[q] = 0;
  __syncthreads();
  int k = 0, i = 0, status = 0;
  double s2 = 0.0;
  for (;;) {
    for (int l = tid; l < k; l += kThreads) ui[l] = U[(long long)l * m + i];
    __syncthreads();
    // residual row i -> candidate column k of V
    double* vk = V + (long long)k * n;
    double bv = -1.0;
    int bj = INT_MAX;
    for (int j = tid; j < n; j += kThreads) {
      double r = entry_of(E, rows[i], cols[j]);
      for (int l = 0; l < k; ++l) r -= ui[l] * V[(long long)l * n + j];
      vk[j] = r;
      const double a = fabs(r);
      if (a > bv) {
        bv = a;
        bj = j;
      }
    }
    if (tid == 0) used[i] = 1;
    block_argmax(bv, bj, sv, si);
    if (!(bv > 1e-300)) {
      // zero residual row: the lowest unused row
      int nxt = INT_MAX;
      for (int q = tid; q < m; q += kThreads)
        if (!used[q]) {
          nxt = q;
          break;
        }
      nxt = wave_min(nxt);
      if (lane == 0) si[wave] = nxt;
      __syncthreads();
      nxt = si[0];
      for (int w = 1; w < kWaves; ++w) nxt = min(nxt, si[w]);
      __syncthreads();
      if (nxt >= m) break;
      i = nxt;
      continue;
    }
    const int jp = bj;
    const double piv = vk[jp];
    __syncthreads();  // every thread holds the pivot before its owner rescales it
    for (int j = tid; j < n; j += kThreads) vk[j] = vk[j] / piv;
    for (int l = tid; l < k; l += kThreads) vj[l] = V[(long long)l * n + jp];
    __syncthreads();
    // residual column jp -> column k of U
    double* uk = U + (long long)k * m;
    for (int q = tid; q < m; q += kThreads) {
      double u = entry_of(E, rows[q], cols[jp]);
      for (int l = 0; l < k; ++l) u -= vj[l] * U[(long long)l * m + q];
      uk[q] = u;
    }
    __syncthreads();
    // U_l . u and V_l . v for l < k; |u|^2 and |v|^2 at l = k
    for (int l = 0; l <= k; ++l) {
      const double* Ul = U + (long long)l * m;
      const double* Vl = V + (long long)l * n;
      double du = 0.0, dv = 0.0;
      for (int q = tid; q < m; q += kThreads) du += Ul[q] * uk[q];
      for (int j = tid; j < n; j += kThreads) dv += Vl[j] * vk[j];
      du = wave_sum(du);
      dv = wave_sum(dv);
      if (lane == 0) {
        red[wave * ld + 2 * l] = du;
        red[wave * ld + 2 * l + 1] = dv;
      }
    }
    __syncthreads();
    double cross = 0.0, nu2 = 0.0, nv2 = 0.0;
    for (int l = 0; l <= k; ++l) {
      double du = 0.0, dv = 0.0;
      for (int w = 0; w < kWaves; ++w) {
        du += red[w * ld + 2 * l];
        dv += red[w * ld + 2 * l + 1];
      }
      if (l < k) cross += du * dv;
      else {
        nu2 = du;
        nv2 = dv;
      }
    }
    s2 += 2.0 * cross + nu2 * nv2;
    ++k;
    if (sqrt(nu2) * sqrt(nv2) <= eps * sqrt(s2)) break;
    if ((long long)k * (m + n) >= (long long)m * n || k >= B.kmax) {
      status = 1;
      break;
    }
    if (k >= kAcaCap) {
      status = 2;
      break;
    }
    // next row: the unused row with the largest |u|
    double bu = -1.0;
    int bq = INT_MAX;
    for (int q = tid; q < m; q += kThreads)
      if (!used[q] && fabs(uk[q]) > bu) {
        bu = fabs(uk[q]);
        bq = q;
      }
    block_argmax(bu, bq, sv, si);
    if (bq >= m) break;
    i = bq;
  }
  if (status == 0 && (long long)k * (m + n) >= (long long)m * n) status = 1;
  if (tid == 0) {
    rank_out[blockIdx.x] = k;
    status_out[blockIdx.x] = status;
  }
}

// Entries of whole blocks, column-major, over a flat index space of
// `total` entries (block b owns [starts[b], starts[b+1])).
__global__ __launch_bounds__(kThreads) void k_fill(EntryView E, const long long* __restrict__ perm,
                                                    const FillBlock* __restrict__ blocks,
                                                    const long long* __restrict__ starts, int nb, long long total,
                                                    double* __restrict__ out) {
  const long long chunk = (long long)kThreads * 64;
  const long long e0 = (long long)blockIdx.x * chunk;
  if (e0 >= total) return;
  // block holding e0 (last b with starts[b] <= e0)
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (starts[mid] <= e0) lo = mid;
    else hi = mid - 1;
  }
  int b = lo;
  const long long e1 = min(total, e0 + chunk);
  for (long long e = e0 + threadIdx.x; e < e1; e += kThreads) {
    while (b + 1 < nb && starts[b + 1] <= e) ++b;
    const FillBlock B = blocks[b];
    const long long loc = e - starts[b];
    const long long j = loc / B.m, i = loc - j * B.m;
    out[B.off + loc] = entry_of(E, perm[B.r0 + i], perm[B.c0 + j]);
  }
}

// U[:, :k] then V[:, :k] of each block, contiguous, into the packed buffer.
__global__ __launch_bounds__(kThreads) void k_pack(const PackBlock* __restrict__ blocks,
                                                    const double* __restrict__ scratch, double* __restrict__ out) {
  const PackBlock B = blocks[blockIdx.x];
  const long long nu = (long long)B.k * B.m, nv = (long long)B.k * B.n;
  const double* U = scratch + B.src;
  const double* V = U + (long long)kAcaCap * B.m;
  for (long long e = threadIdx.x; e < nu; e += kThreads) out[B.dst + e] = U[e];
  for (long long e = threadIdx.x; e < nv; e += kThreads) out[B.dst + nu + e] = V[e];
}

void hip_ok(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(HMAT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device buffer released on scope exit.
struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { reset(bytes); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(0); }
  void reset(size_t bytes) {
    if (p) (void)hipFree(p);
    p = nullptr;
    if (bytes) hip_ok(hipMalloc(&p, bytes), "hipMalloc");
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

template <typename T>
void upload(DevBuf& d, const std::vector<T>& v, hipStream_t s) {
  d.reset(v.size() * sizeof(T));
  if (!v.empty()) hip_ok(hipMemcpyAsync(d.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
}

// Pinned host buffer released on scope exit.
struct PinnedBuf {
  void* p = nullptr;
  explicit PinnedBuf(size_t bytes) { hip_ok(hipHostMalloc(&p, bytes, hipHostMallocDefault), "hipHostMalloc"); }
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() { (void)hipHostFree(p); }
};

struct Event {
  hipEvent_t e = nullptr;
  Event() { hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate"); }
  Event(const Event&) = delete;
  Event& operator=(const Event&) = delete;
  ~Event() { (void)hipEventDestroy(e); }
};

// A run of `len` doubles at offset soff of a device buffer, bound for dst.
struct Segment {
  long long soff, len;
  double* dst;
};

// Device-to-host copy of the segments (sorted by soff, disjoint) of the
// buffer src through two pinned staging halves: the DMA of one chunk runs
// while host threads scatter the previous one to the destinations.
class Downloader {
 public:
  static constexpr long long kChunk = 1 << 22;  // doubles per staging half (32 MiB)
  Downloader(hipStream_t s, int32_t n_threads) : s_(s), nt_(n_threads), stage_(2 * kChunk * sizeof(double)) {}

  void run(const double* src, long long total, const std::vector<Segment>& segs) {
    if (total <= 0 || segs.empty()) return;
    double* stage = static_cast<double*>(stage_.p);
    const long long nch = (total + kChunk - 1) / kChunk;
    auto enqueue = [&](long long c) {
      const long long a = c * kChunk, len = std::min(kChunk, total - a);
      hip_ok(hipMemcpyAsync(stage + (c & 1) * kChunk, src + a, len * sizeof(double), hipMemcpyDeviceToHost, s_),
             "download");
      hip_ok(hipEventRecord(ev_[c & 1].e, s_), "hipEventRecord");
    };
    enqueue(0);
    size_t first = 0;
    for (long long c = 0; c < nch; ++c) {
      // the other half was scattered in the previous iteration
      if (c + 1 < nch) enqueue(c + 1);
      hip_ok(hipEventSynchronize(ev_[c & 1].e), "download");
      const long long a = c * kChunk, b = std::min(total, a + kChunk);
      const double* st = stage + (c & 1) * kChunk;
      while (first < segs.size() && segs[first].soff + segs[first].len <= a) ++first;
      size_t last = first;
      while (last < segs.size() && segs[last].soff < b) ++last;
      parallel_for((int64_t)(last - first), nt_, [&](int64_t k) {
        const Segment& g = segs[first + k];
        const long long lo = std::max(a, g.soff), hi = std::min(b, g.soff + g.len);
        if (hi > lo) std::memcpy(g.dst + (lo - g.soff), st + (lo - a), (hi - lo) * sizeof(double));
      });
    }
  }

 private:
  hipStream_t s_;
  int32_t nt_;
  PinnedBuf stage_;
  Event ev_[2];
};

}  // namespace

HostMatrix assemble_device(const EntryFn& A, const ClusterTree& tree, const std::vector<BlockSpec>& blocks,
                           double eps, int32_t max_rank, int32_t n_threads, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (!(eps > 0.0) || !std::isfinite(eps)) fail(HMAT_EINVAL, "aca_eps must be positive");
  if (max_rank < 0) fail(HMAT_EINVAL, "max_rank must be >= 0");
  const EntryView V = A.view();
  const int64_t n = (int64_t)tree.perm.size();
  const int64_t nb = (int64_t)blocks.size();
  const size_t npacked = V.kind == HMAT_GF_FS_RECT_COPLANAR ? 6 * (size_t)n : 18 * (size_t)n;
  DevBuf d_entries(npacked * sizeof(double));
  hip_ok(hipMemcpyAsync(d_entries.p, V.a, npacked * sizeof(double), hipMemcpyHostToDevice, s), "upload");
  EntryView Ed = V;
  Ed.a = d_entries.as<double>();
  std::vector<long long> perm(tree.perm.begin(), tree.perm.end());
  DevBuf d_perm;
  upload(d_perm, perm, s);

  // Where each block's values are: a packed device buffer (buf, boff) or
  // own storage (host fallback); len = k (m + n) or m n doubles.
  struct Result {
    int kind = 0;
    int64_t rank = 0;
    long long len = 0;
    int buf = -1;
    long long boff = 0;
    std::vector<double> own;
  };
  std::vector<Result> res(nb);
  std::deque<DevBuf> packed_bufs;  // packed factors, one per ACA batch
  std::vector<int64_t> dense_list, host_list;

  // --- low-rank candidates, in batches whose scratch fits a share of free memory
  std::vector<int64_t> lr;
  for (int64_t b = 0; b < nb; ++b) {
    if (blocks[b].kind != 1) dense_list.push_back(b);
    else if (blocks[b].m > kMaxMaskRows) host_list.push_back(b);
    else lr.push_back(b);
  }
  size_t free_b = 0, total_b = 0;
  hip_ok(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
  const long long budget = std::max<long long>(1ll << 28, (long long)(free_b / 4 / sizeof(double)));
  for (size_t p0 = 0; p0 < lr.size();) {
    std::vector<AcaBlock> ab;
    long long off = 0;
    size_t p1 = p0;
    for (; p1 < lr.size(); ++p1) {
      const BlockSpec& s0 = blocks[lr[p1]];
      const long long need = (long long)kAcaCap * (s0.m + s0.n);
      if (!ab.empty() && off + need > budget) break;
      int64_t kmax = max_rank > 0 ? max_rank : std::min(s0.m, s0.n) / 2;
      kmax = std::max<int64_t>(1, std::min<int64_t>(kmax, std::min(s0.m, s0.n)));
      ab.push_back(AcaBlock{s0.r0, s0.m, s0.c0, s0.n, off, (int)std::min<int64_t>(kmax, INT_MAX), 0});
      off += need;
    }
    long long mmax = 1;
    for (const AcaBlock& q : ab) mmax = std::max(mmax, q.m);
    const size_t lds = sizeof(double) * (kWaves * (2 * kAcaCap + 2) + 2 * kAcaCap) + (size_t)((mmax + 7) / 8 * 8);
    DevBuf d_ab, d_rank((p1 - p0) * sizeof(int)), d_status((p1 - p0) * sizeof(int)), d_scratch(off * sizeof(double));
    upload(d_ab, ab, s);
    hipLaunchKernelGGL(k_aca, dim3((unsigned)ab.size()), dim3(kThreads), lds, s, Ed, d_perm.as<long long>(),
                       d_ab.as<AcaBlock>(), d_scratch.as<double>(), eps, d_rank.as<int>(), d_status.as<int>());
    hip_ok(hipGetLastError(), "ACA launch");
    std::vector<int> rank(ab.size()), status(ab.size());
    hip_ok(hipMemcpyAsync(rank.data(), d_rank.p, rank.size() * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_ok(hipMemcpyAsync(status.data(), d_status.p, status.size() * sizeof(int), hipMemcpyDeviceToHost, s), "copy");
    hip_ok(hipStreamSynchronize(s), "ACA");
    // pack the accepted factors; they stay on the device until the layout is known
    std::vector<PackBlock> pk;
    long long packed = 0;
    for (size_t q = 0; q < ab.size(); ++q) {
      const int64_t b = lr[p0 + q];
      if (status[q] == 1) dense_list.push_back(b);
      else if (status[q] == 2) host_list.push_back(b);
      else {
        pk.push_back(PackBlock{ab[q].m, ab[q].n, ab[q].off, packed, rank[q], 0});
        Result& R = res[b];
        R.kind = 1;
        R.rank = rank[q];
        R.len = (long long)rank[q] * (ab[q].m + ab[q].n);
        R.buf = R.len > 0 ? (int)packed_bufs.size() : -1;
        R.boff = packed;
        packed += R.len;
      }
    }
    if (packed > 0) {
      DevBuf d_pk;
      upload(d_pk, pk, s);
      packed_bufs.emplace_back((size_t)packed * sizeof(double));
      hipLaunchKernelGGL(k_pack, dim3((unsigned)pk.size()), dim3(kThreads), 0, s, d_pk.as<PackBlock>(),
                         d_scratch.as<double>(), packed_bufs.back().as<double>());
      hip_ok(hipGetLastError(), "pack launch");
      hip_ok(hipStreamSynchronize(s), "pack");
    }
    p0 = p1;
  }

  // --- blocks the device left to the host (rank beyond the device cap, or too many rows)
  {
    std::vector<double> U, W;
    for (int64_t b : host_list) {
      const BlockSpec& sp = blocks[b];
      int64_t rank = 0;
      if (aca_block(A, tree.perm.data() + sp.r0, sp.m, tree.perm.data() + sp.c0, sp.n, eps, max_rank, U, W, rank)) {
        Result& R = res[b];
        R.kind = 1;
        R.rank = rank;
        R.own = U;
        R.own.insert(R.own.end(), W.begin(), W.end());
        R.len = (long long)R.own.size();
      } else {
        dense_list.push_back(b);
      }
    }
  }
  for (int64_t b : dense_list) {
    res[b] = Result{};
    res[b].len = blocks[b].m * blocks[b].n;
  }

  // --- the block list, laid out as the host construction does
  HostMatrix H;
  H.n = n;
  H.perm.resize(n);
  for (int64_t k = 0; k < n; ++k) H.perm[k] = (int32_t)tree.perm[k];
  H.desc.resize(6 * nb);
  H.off.resize(nb);
  int64_t total = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const BlockSpec& sp = blocks[b];
    int64_t* d = &H.desc[6 * b];
    d[0] = res[b].kind;
    d[1] = sp.r0; d[2] = sp.m; d[3] = sp.c0; d[4] = sp.n; d[5] = res[b].rank;
    H.off[b] = total;
    total += res[b].len;
  }
  H.values.resize(total);
  Downloader down(s, n_threads);

  // --- packed factors to their places
  {
    std::vector<std::vector<Segment>> segs(packed_bufs.size());
    for (int64_t b = 0; b < nb; ++b)
      if (res[b].buf >= 0) segs[res[b].buf].push_back(Segment{res[b].boff, res[b].len, H.values.data() + H.off[b]});
    for (size_t i = 0; i < packed_bufs.size(); ++i) {
      const long long tot = segs[i].empty() ? 0 : segs[i].back().soff + segs[i].back().len;
      down.run(packed_bufs[i].as<double>(), tot, segs[i]);
      packed_bufs[i].reset(0);
    }
  }
  parallel_for(nb, n_threads, [&](int64_t b) {
    if (!res[b].own.empty()) std::copy(res[b].own.begin(), res[b].own.end(), H.values.begin() + H.off[b]);
  });

  // --- dense blocks, in batches, evaluated on the device and copied to their places
  std::sort(dense_list.begin(), dense_list.end());
  for (size_t p0 = 0; p0 < dense_list.size();) {
    std::vector<FillBlock> fb;
    std::vector<long long> starts;
    std::vector<Segment> segs;
    long long tot = 0;
    size_t p1 = p0;
    for (; p1 < dense_list.size(); ++p1) {
      const int64_t b = dense_list[p1];
      const BlockSpec& sp = blocks[b];
      const long long need = (long long)sp.m * sp.n;
      if (!fb.empty() && tot + need > budget) break;
      fb.push_back(FillBlock{sp.r0, sp.m, sp.c0, sp.n, tot});
      starts.push_back(tot);
      segs.push_back(Segment{tot, need, H.values.data() + H.off[b]});
      tot += need;
    }
    DevBuf d_fb, d_starts, d_out(tot * sizeof(double));
    upload(d_fb, fb, s);
    upload(d_starts, starts, s);
    const long long chunk = (long long)kThreads * 64;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((tot + chunk - 1) / chunk)), dim3(kThreads), 0, s, Ed,
                       d_perm.as<long long>(), d_fb.as<FillBlock>(), d_starts.as<long long>(), (int)fb.size(), tot,
                       d_out.as<double>());
    hip_ok(hipGetLastError(), "fill launch");
    down.run(d_out.as<double>(), tot, segs);
    hip_ok(hipStreamSynchronize(s), "fill");
    p0 = p1;
  }
  H.tree_depth = tree.max_depth;
  return H;
}

}  // namespace hm
