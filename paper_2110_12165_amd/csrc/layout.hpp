// Device layouts of a block list (host-side packing).
#pragma once

#include <cstdint>
#include <vector>

#include "device_types.hpp"
#include "hmat_internal.hpp"

namespace hm {

// Natural layout: blocks as built, each starting on a 256-byte boundary.
template <typename T>
struct PlainLayout {
  HostVec<T> pool;
  std::vector<PlainBlock> blocks;
  std::vector<int32_t> lr_list;        // low-rank blocks with rank > 0
  std::vector<RowUnit> row_units;      // owners of output rows (product)
  std::vector<UnitEntry> row_entries;
  std::vector<RowUnit> col_units;      // owners of output rows of the transpose
  std::vector<UnitEntry> col_entries;
  int64_t sum_rank = 0;
};

template <typename T>
PlainLayout<T> make_plain(const HostMatrix& H, bool transpose, int32_t n_threads = 0);

// Batched layout: every product becomes a list of work units over packed
// panels (see Unit in device_types.hpp).
template <typename T>
struct BatchedLayout {
  HostVec<T> pool;
  std::vector<Unit> units;             // n1 phase-1 units, then n2 phase-2 units
  int32_t n1 = 0, n2 = 0;
  std::vector<int32_t> src;
  int64_t t_size = 0;                  // intermediate values, entry 0 = zero pad
  // Phase-1 units split by rows write partial intermediate values; entry j
  // (4 slots, unused ones 0) lists the partials of one value, which phase 2
  // adds in that order when a source reads -(t_size + j) - 1.
  std::vector<int32_t> sums;
  // pair_inputs: phase-2 units in pairs of consecutive row intervals, (a, b)
  // indices relative to the first phase-2 unit (b = -1 for an interval
  // without a partner), largest pairs first
  std::vector<int32_t> pairs;
  int32_t wg_waves = 8;                // waves per workgroup of phase-2 units
  int32_t wg_waves_p1 = 8;             // waves per workgroup of phase-1 units
  int64_t unit_bytes = 0;
};

// wg_waves: waves per workgroup of phase-2 units; wg_waves_p1: of phase-1
// units (equal for the persistent schedule, which runs both in one launch).
// transpose: pack H^T (read in place; the same layout as packing
// transpose_host(H)).  n_threads: panel-filling threads, 0 for all.
// split_slots > 0: phase-1 workgroups resident on the device at once; when
// phase 1 has fewer than two 64-output units per such slot (small
// matrices, where the largest units run alone at the end of the phase),
// units more than twice the mean are split by rows into up to 4 units with
// partial intermediate values (see sums).  0: no splitting.
// pair_inputs: consecutive row intervals 2j, 2j + 1 form pairs; the inputs the
// two share (the same x element or intermediate value) lead both input
// lists in the same order (Unit::ncom), so that the ensemble product can
// stage them once for the pair (pairs).
template <typename T>
BatchedLayout<T> make_batched(const HostMatrix& H, int32_t wg_waves, int64_t unit_bytes, int32_t wg_waves_p1,
                              bool transpose = false, int32_t n_threads = 0, int64_t split_slots = 0,
                              bool pair_inputs = false);

// The blocks of H^T (dense blocks transposed, U and V exchanged), same
// permutation: packing them gives the layouts of the transpose product.
HostMatrix transpose_host(const HostMatrix& H);

// Row intervals of the finest common refinement of the blocks' row (or
// column) ranges, each split into pieces of at most `cap` rows.
std::vector<std::pair<int64_t, int64_t>> refine_ranges(const HostMatrix& H, bool columns, int64_t cap);

}  // namespace hm
