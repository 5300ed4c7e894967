// Launch interface of the ensemble (multi-RHS) product on MFMA.
#pragma once

#include <hip/hip_runtime.h>

#include "device_types.hpp"

namespace hm {

struct MMArgs {
  const Unit* units;       // batched units (phase 1 then phase 2); every nout <= 1024
  int32_t n1, n2;
  const int32_t* slices1;  // 64-output slices of the phase-1 units: 16 * unit + slice
  int32_t ns1;             // number of slices
  const int32_t* src;      // phase-2 input sources (user index of x, or -t-1)
  const void* pool;        // FP32 panels
  const int32_t* perm;     // cluster position -> user element
  const int32_t* invperm;  // user element -> cluster position
  int64_t n, t_size;
  void* Xs;                // bf16 [3][n][64]: split member values, cluster order
  void* Ts;                // bf16 [3][t_size][64]: split intermediate values
  const double* X;         // user order, element-major: X[i * ldx + r]
  int64_t ldx;
  double* Y;               // user order, element-major: Y[i * ldy + r]
  int64_t ldy;
  int32_t nrhs;            // 1..64
  int32_t cus;             // compute units of the device
  int32_t groups1, groups2;  // wave groups (1 or 2) sharing a 64-output slice in phase 1, phase 2;
                             // groups2 == kGroupsPairs: phase 2 on pairs of row intervals
  const int32_t* pairs;      // pairs of phase-2 units (a, b; b = -1 alone), or null
  int32_t npairs;
};

// Phase-2 schedule value of MMArgs::groups2 (and of the handle's choice)
// that runs the pairs of row intervals sharing their common inputs.
constexpr int32_t kGroupsPairs = 3;

// parts = 2 (3 bf16 products, "BF16x3") or 3 (6 products, "BF16x6").
// ev (optional): 3 events, before / between the phases / after.
hipError_t launch_mm(const MMArgs& a, int parts, double alpha, double beta, hipStream_t s, hipEvent_t* ev = nullptr);

}  // namespace hm
