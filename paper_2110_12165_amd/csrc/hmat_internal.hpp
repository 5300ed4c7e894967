// Internal declarations of the lattice H-matrix library (host side).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <exception>
#include <mutex>
#include <new>
#include <sched.h>
#include <stdexcept>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "entries.hpp"
#include "hmat.h"

namespace hm {

// Error carrying a status code; converted to hmat_status at the C boundary.
struct Error : std::runtime_error {
  hmat_status code;
  Error(hmat_status c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

[[noreturn]] inline void fail(hmat_status c, const std::string& msg) { throw Error(c, msg); }

// Allocator whose value-less construction leaves arithmetic elements
// uninitialised: large host buffers that are written in full afterwards
// (by several threads) skip a serial zero fill.
template <typename T>
struct NoInitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <typename U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... Args>
  void construct(U* p, Args&&... args) {
    ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
  }
};
template <typename T>
using HostVec = std::vector<T, NoInitAlloc<T>>;

// Threads this process may run on (its CPU affinity mask), at least 1.
inline int32_t host_threads() {
  cpu_set_t set;
  CPU_ZERO(&set);
  if (sched_getaffinity(0, sizeof(set), &set) == 0) return std::max(1, CPU_COUNT(&set));
  return (int32_t)std::max(1u, std::thread::hardware_concurrency());
}

// Runs f(0 .. count-1) on up to n_threads threads (0: host_threads()),
// items handed out one at a time.  If f throws, the remaining items are
// skipped and the first exception is rethrown after all threads joined.
template <typename F>
void parallel_for(int64_t count, int32_t n_threads, F&& f) {
  int64_t nt = n_threads > 0 ? n_threads : host_threads();
  nt = std::max<int64_t>(1, std::min<int64_t>(nt, count));
  std::atomic<int64_t> next{0};
  std::atomic<bool> failed{false};
  std::exception_ptr err;
  std::mutex err_mu;
  auto work = [&] {
    try {
      for (int64_t k; !failed.load(std::memory_order_relaxed) && (k = next.fetch_add(1)) < count;) f(k);
    } catch (...) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (!err) err = std::current_exception();
      failed.store(true);
    }
  };
  std::vector<std::thread> th;
  th.reserve((size_t)nt);
  try {
    for (int64_t t = 1; t < nt; ++t) th.emplace_back(work);
  } catch (...) {  // no more threads: stop the started ones and report
    failed.store(true);
    for (auto& t : th) t.join();
    throw;
  }
  work();
  for (auto& t : th) t.join();
  if (err) std::rethrow_exception(err);
}

// Sets v[0 .. size) to zero in chunks spread over threads.
template <typename T>
void parallel_zero(T* v, int64_t size, int32_t n_threads) {
  constexpr int64_t kChunk = 1 << 18;
  parallel_for((size + kChunk - 1) / kChunk, n_threads, [&](int64_t c) {
    const int64_t a = c * kChunk, b = std::min(size, a + kChunk);
    std::fill(v + a, v + b, T(0));
  });
}

// ---------------------------------------------------------------------------
// Geometry and stiffness entries (eqs. (5)-(6)).
// ---------------------------------------------------------------------------
class EntryFn {
 public:
  virtual ~EntryFn() = default;
  // A(i, j) in user element order.
  virtual double entry(int64_t i, int64_t j) const = 0;
  // The packed per-element data behind entry() (see entries.hpp), valid
  // while this object lives; used to evaluate entries on the device.
  virtual EntryView view() const = 0;
};

struct Geometry {
  int64_t n = 0;
  std::vector<double> centres;  // n * 3
};

// Validates the mesh and Green's function and returns the entry function;
// fills geo.centres.
EntryFn* make_entry_fn(const hmat_mesh& mesh, const hmat_green& green, Geometry& geo);
// The triangle kernel (called by make_entry_fn after the common checks).
EntryFn* make_triangle_entry_fn(const hmat_mesh& mesh, const hmat_green& green, Geometry& geo);

// ---------------------------------------------------------------------------
// Cluster tree and block partition (section 3.1.1, eq. (17); section 3.2).
// ---------------------------------------------------------------------------
struct TreeNode {
  int64_t start = 0, size = 0;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  int32_t child[2] = {-1, -1};
  int32_t depth = 0;
  bool leaf() const { return child[0] < 0; }
};

struct ClusterTree {
  std::vector<int64_t> perm;     // cluster position -> user element
  std::vector<TreeNode> nodes;   // nodes[0] = root
  int32_t max_depth = 0;
};

ClusterTree build_tree(const Geometry& geo, int32_t leaf);

struct BlockSpec {
  int kind;  // 0 dense, 1 admissible (low-rank candidate)
  int64_t r0, m, c0, n;
  int32_t lat_row, lat_col;
};

std::vector<BlockSpec> partition(const ClusterTree& tree, int32_t lattice, double eta);

// ---------------------------------------------------------------------------
// Blocks in FP64 on the host (the export format of hmat.h).
// ---------------------------------------------------------------------------
struct HostMatrix {
  int64_t n = 0;
  std::vector<int32_t> perm;
  std::vector<int64_t> desc;    // 6 per block: kind, r0, m, c0, n, rank
  std::vector<int64_t> off;     // per block
  HostVec<double> values;
  int32_t lattice = 1;
  int32_t tree_depth = 0;
  int64_t nblocks() const { return (int64_t)off.size(); }
};

// Adaptive cross approximation of the block rows x cols (user indices).
// Returns false when the dense fallback applies; U is m x k, V is n x k,
// column-major.
bool aca_block(const EntryFn& A, const int64_t* rows, int64_t m, const int64_t* cols, int64_t n,
               double eps, int32_t max_rank, std::vector<double>& U, std::vector<double>& V,
               int64_t& rank);

HostMatrix assemble(const EntryFn& A, const ClusterTree& tree, const std::vector<BlockSpec>& blocks,
                    double eps, int32_t max_rank, int32_t n_threads);

// The same block list built on the device (build_gpu.hip): ACA of the
// admissible blocks and entries of the dense ones on the GPU, with the rules
// of assemble(); blocks beyond the device rank cap go through aca_block().
// n_threads: threads of the host-side steps (0: all); stream: a
// hipStream_t (or null).
HostMatrix assemble_device(const EntryFn& A, const ClusterTree& tree, const std::vector<BlockSpec>& blocks,
                           double eps, int32_t max_rank, int32_t n_threads, void* stream);

// Checks that blocks tile the matrix once and perm is a permutation.
void validate_host_matrix(const HostMatrix& H);

}  // namespace hm
