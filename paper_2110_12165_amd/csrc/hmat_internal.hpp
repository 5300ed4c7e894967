// Internal declarations of the lattice H-matrix library (host side).
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
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
  std::vector<double> values;
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
// stream: a hipStream_t (or null).
HostMatrix assemble_device(const EntryFn& A, const ClusterTree& tree, const std::vector<BlockSpec>& blocks,
                           double eps, int32_t max_rank, void* stream);

// Checks that blocks tile the matrix once and perm is a permutation.
void validate_host_matrix(const HostMatrix& H);

}  // namespace hm
