// Launch interface of the product kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace hm {

// Device pointers of a natural-layout product.
struct PlainArgs {
  const PlainBlock* blocks;
  const int32_t* lr_list;
  int32_t n_lr;
  const RowUnit* rows;
  int32_t n_rows;
  const UnitEntry* row_ents;
  const RowUnit* cols;
  int32_t n_cols;
  const UnitEntry* col_ents;
  const void* pool;
  const int32_t* perm;
  double* t;  // scratch: sum of ranks
};

// Device pointers of a batched-layout product.
struct BatchedArgs {
  const Unit* units;
  int32_t n1, n2;
  const int32_t* src;
  double* t;  // scratch: intermediate values t = V^T x, t[0] = 0
  const int32_t* sums;  // 4 partial-value slots per split intermediate value (or null)
  int32_t t_size;       // intermediate values (main and partial); src -(t_size + j) - 1 reads sums[4 j ..]
  const void* pool;
  const int32_t* perm;
  QueueCounters* ctr;
  int32_t wg_waves;     // waves per workgroup, phase-2 units (and the persistent launch)
  int32_t wg_waves_p1;  // waves per workgroup, phase-1 units
  double* tm;           // intermediate values of the multi-vector product: kMultiMax segments of t_size
};

// Vectors a multi-vector product applies per pass over the factors.
constexpr int kMultiMax = 4;

// ev (optional): events recorded before the first launch, between the
// launches and after the last one (plain and split: 3; persistent: 2).
template <typename T>
hipError_t launch_plain(const PlainArgs& a, bool transpose, const double* x, double* y, double alpha, double beta,
                        hipStream_t s, hipEvent_t* ev = nullptr);

template <typename T>
hipError_t launch_batched(const BatchedArgs& a, bool persistent, int grid, const double* x, double* y, double alpha,
                          double beta, hipStream_t s, hipEvent_t* ev = nullptr);

// Split schedule for nvec = 2 or 4 vectors at once: each panel entry is read
// once for all of them.  x + r ldx -> y + r ldy (r < nvec).
template <typename T>
hipError_t launch_batched_multi(const BatchedArgs& a, int nvec, const double* x, int64_t ldx, double* y, int64_t ldy,
                                double alpha, double beta, hipStream_t s);

template <typename T>
int persistent_blocks_per_cu(int wg_waves);

// Phase-1 workgroups of wg_waves_p1 waves resident per compute unit.
template <typename T>
int phase1_blocks_per_cu(int wg_waves_p1);

}  // namespace hm
