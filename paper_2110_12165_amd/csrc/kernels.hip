// HIP kernels of the H-matrix-vector product (section 3.1.3, eq. (20)) for
// gfx950.
//
// The product y = H x is taken in two phases:
//   phase 1: t_b = V_b^T x_M for every low-rank block b (the inner sum of
//            eq. (20));
//   phase 2: for every output row, the sum of the dense-block products and
//            of the U_b t_b terms of the low-rank blocks meeting that row
//            (the outer sum of eq. (20) and the summation of all block
//            contributions).  Each row has exactly one owner, so y is written
//            once, without atomics, and FP64 results are reproducible.
//
// Two layouts are supported:
//   plain:   blocks in their natural column-major form; phase 1 has one
//            workgroup per low-rank block, phase 2 one wave per row unit.
//   batched: every phase is a list of work units over packed panels in
//            which each lane (one output) reads 16 contiguous bytes per
//            input group, so every wave load is a contiguous, fully used
//            segment of HBM; inputs of a unit are staged once in LDS (FP64).
//            Run as two launches (split) or one persistent launch in which
//            phase-2 units wait for a completion counter of phase 1.
// Products accumulate in FP64 whatever the storage precision.
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels.hpp"

namespace hm {
namespace {

constexpr int kStage = 2048;  // inputs staged in LDS per round (FP64)

template <typename T>
struct Pack;
template <>
struct Pack<float> {
  typedef float vec __attribute__((ext_vector_type(4)));
  static constexpr int W = 4;
};
template <>
struct Pack<double> {
  typedef double vec __attribute__((ext_vector_type(2)));
  static constexpr int W = 2;
};

template <typename T>
__device__ __forceinline__ typename Pack<T>::vec load_stream(const typename Pack<T>::vec* p) {
  return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// ------------------------------------------------------------------------
// batched layout
// ------------------------------------------------------------------------
// Stages inputs [c0, c0 + cl) of unit u in zs (FP64).  Each thread takes
// inputs tid + k NW 64 in batches of kStageBatch: first every index (perm
// or src), then every value, with no branch between the loads, so a batch
// costs two memory round trips rather than two per input.  A padding input
// (past nin in phase 1) reads t[0], the zero pad; an input whose value was
// split over row parts adds the partials in part order, after the batch.
constexpr int kStageBatch = 4;

template <int NW, bool COHERENT>
__device__ __forceinline__ void stage_inputs(const Unit& u, int c0, int cl, const double* __restrict__ x,
                                             const int32_t* __restrict__ perm, const int32_t* __restrict__ src,
                                             const double* t, const int32_t* __restrict__ sums, int t_size,
                                             double* zs) {
  constexpr int NT = NW * 64;
  // inputs per thread per batch: every slot of a batch lies inside zs
  // (kStage entries), so its values are stored without a bounds test
  constexpr int B = kStageBatch * NT <= kStage ? kStageBatch : kStage / NT;
  static_assert(B >= 1 && kStage % (B * NT) == 0, "staging batch");
  const int tid = threadIdx.x;
  // index list of the unit: phase 1 its rows (nin of them, then padding),
  // phase 2 its input list (nin entries, padding included)
  const int32_t* ip = (u.kind == 1 ? perm : src) + u.in0;
  const int lim = u.nin;
  for (int i0 = 0; i0 < cl; i0 += B * NT) {
    int s[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int gi = c0 + i0 + k * NT + tid;
      s[k] = ip[max(0, min(gi, lim - 1))];
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int gi = c0 + i0 + k * NT + tid;
      if (gi >= lim) s[k] = -1;  // t[0]
    }
    double v[B];
    bool split = false;
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int j = -s[k] - 1;
      split |= j >= t_size;
      const double* p = s[k] >= 0 ? x + s[k] : t + (j < t_size ? j : 0);
      v[k] = COHERENT ? load_agent(p) : *p;
    }
    if (split) {  // a value split over row parts: partials added in part order
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int j = -s[k] - 1;
        if (j >= t_size) {
          const int* e = sums + 4 * (j - t_size);
          if (COHERENT)
            v[k] = ((load_agent(t + e[0]) + load_agent(t + e[1])) + load_agent(t + e[2])) + load_agent(t + e[3]);
          else
            v[k] = ((t[e[0]] + t[e[1]]) + t[e[2]]) + t[e[3]];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < B; ++k) zs[i0 + k * NT + tid] = v[k];  // past cl: never read
  }
}

template <typename T, int NW, bool COHERENT>
__device__ __forceinline__ void run_unit(const Unit& u, const T* __restrict__ pool, const double* __restrict__ x,
                                         double* __restrict__ y, const int32_t* __restrict__ perm,
                                         const int32_t* __restrict__ src, double* t,
                                         const int32_t* __restrict__ sums, int t_size, double alpha, double beta,
                                         double* zs, double* red) {
  using V = typename Pack<T>::vec;
  constexpr int W = Pack<T>::W;
  constexpr int U = 8;  // loads in flight per lane
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int S = u.S, RG = u.RG;
  const bool working = wave < S * RG;
  const int sg = wave % S, rg = wave / S;
  const int o = sg * 64 + lane;
  const bool active = working && o < u.nout;
  const int nin_pad = u.nq * W;
  const size_t stride = (size_t)u.nout;
  const V* base = reinterpret_cast<const V*>(pool + u.off) + o;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};

  for (int c0 = 0; c0 < nin_pad; c0 += kStage) {
    const int cl = min(kStage, nin_pad - c0);
    stage_inputs<NW, COHERENT>(u, c0, cl, x, perm, src, t, sums, t_size, zs);
    __syncthreads();
    if (active) {
      const int q0 = c0 / W;
      const int q1 = q0 + cl / W;
      int q = q0 + rg;
      for (; q + (U - 1) * RG < q1; q += U * RG) {
        V v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = load_stream<T>(base + (size_t)(q + k * RG) * stride);
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const double* z = zs + (q + k * RG - q0) * W;
#pragma unroll
          for (int c = 0; c < W; ++c) acc[k & 3] = fma((double)v[k][c], z[c], acc[k & 3]);
        }
      }
      for (; q < q1; q += RG) {
        const V v0 = load_stream<T>(base + (size_t)q * stride);
        const double* z = zs + (q - q0) * W;
#pragma unroll
        for (int c = 0; c < W; ++c) acc[0] = fma((double)v0[c], z[c], acc[0]);
      }
    }
    __syncthreads();
  }
  double sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if (RG > 1) {
    if (working) red[wave * 64 + lane] = sum;
    __syncthreads();
    if (rg == 0) {
      sum = 0.0;
      for (int r = 0; r < RG; ++r) sum += red[(r * S + sg) * 64 + lane];
    }
  }
  if (rg == 0 && active) {
    if (u.kind == 1) {
      t[u.out0 + o] = sum;
    } else {
      const int row = perm[u.out0 + o];
      y[row] = beta == 0.0 ? alpha * sum : fma(alpha, sum, beta * y[row]);
    }
  }
  __syncthreads();
}

// run_unit for R vectors at once (R = 2 or 4; split schedule): every panel
// entry is read once and applied to the R vectors' inputs, which are staged
// in LDS rounds of kStageMulti inputs per vector (vector r at
// zs[r * kStageMulti]; 1024 inputs, so that a typical phase-2 unit of
// ~1700 inputs takes two rounds, not four as with 512).  Vector r reads
// x + r ldx, writes y + r ldy, and its intermediate values are t + r ldt.
// The sums of a row are taken in the same order as run_unit's except for
// the shorter staging rounds.
constexpr int kStageMulti = 1024;
template <typename T, int NW, int R>
__device__ __forceinline__ void run_unit_multi(const Unit& u, const T* __restrict__ pool, const double* __restrict__ x,
                                               int64_t ldx, double* __restrict__ y, int64_t ldy,
                                               const int32_t* __restrict__ perm, const int32_t* __restrict__ src,
                                               double* t, int64_t ldt, const int32_t* __restrict__ sums, int t_size,
                                               double alpha, double beta, double* zs, double* red) {
  using V = typename Pack<T>::vec;
  constexpr int W = Pack<T>::W;
  constexpr int U = 8;
  constexpr int KSR = kStageMulti;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int S = u.S, RG = u.RG;
  const bool working = wave < S * RG;
  const int sg = wave % S, rg = wave / S;
  const int o = sg * 64 + lane;
  const bool active = working && o < u.nout;
  const int nin_pad = u.nq * W;
  const size_t stride = (size_t)u.nout;
  const V* base = reinterpret_cast<const V*>(pool + u.off) + o;
  double acc[R][4];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;

  // staging as in stage_inputs, B inputs per thread and batch
  constexpr int NT = NW * 64;
  constexpr int B = KSR / NT >= 2 ? 2 : 1;
  static_assert(KSR % (B * NT) == 0, "staging batch");
  const int32_t* ip = (u.kind == 1 ? perm : src) + u.in0;
  for (int c0 = 0; c0 < nin_pad; c0 += KSR) {
    const int cl = min(KSR, nin_pad - c0);
    for (int i0 = 0; i0 < cl; i0 += B * NT) {
      int s[B];
#pragma unroll
      for (int k = 0; k < B; ++k) s[k] = ip[max(0, min(c0 + i0 + k * NT + tid, u.nin - 1))];
#pragma unroll
      for (int k = 0; k < B; ++k)
        if (c0 + i0 + k * NT + tid >= u.nin) s[k] = -1;  // t[0]
      double v[B][R];
      bool split = false;
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int j = -s[k] - 1;
        split |= j >= t_size;
#pragma unroll
        for (int r = 0; r < R; ++r) v[k][r] = s[k] >= 0 ? x[r * ldx + s[k]] : t[r * ldt + (j < t_size ? j : 0)];
      }
      if (split) {
#pragma unroll
        for (int k = 0; k < B; ++k) {
          const int j = -s[k] - 1;
          if (j >= t_size) {
            const int* e = sums + 4 * (j - t_size);
#pragma unroll
            for (int r = 0; r < R; ++r)
              v[k][r] = ((t[r * ldt + e[0]] + t[r * ldt + e[1]]) + t[r * ldt + e[2]]) + t[r * ldt + e[3]];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < B; ++k)
#pragma unroll
        for (int r = 0; r < R; ++r) zs[r * KSR + i0 + k * NT + tid] = v[k][r];  // past cl: never read
    }
    __syncthreads();
    if (active) {
      const int q0 = c0 / W;
      const int q1 = q0 + cl / W;
      int q = q0 + rg;
      for (; q + (U - 1) * RG < q1; q += U * RG) {
        V v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = load_stream<T>(base + (size_t)(q + k * RG) * stride);
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const double* z = zs + (q + k * RG - q0) * W;
#pragma unroll
          for (int c = 0; c < W; ++c) {
            const double a = (double)v[k][c];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r][k & 3] = fma(a, z[r * KSR + c], acc[r][k & 3]);
          }
        }
      }
      for (; q < q1; q += RG) {
        const V v0 = load_stream<T>(base + (size_t)q * stride);
        const double* z = zs + (q - q0) * W;
#pragma unroll
        for (int c = 0; c < W; ++c) {
          const double a = (double)v0[c];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r][0] = fma(a, z[r * KSR + c], acc[r][0]);
        }
      }
    }
    __syncthreads();
  }
  double sum[R];
#pragma unroll
  for (int r = 0; r < R; ++r) sum[r] = (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]);
  if (RG > 1) {
    if (working)
#pragma unroll
      for (int r = 0; r < R; ++r) red[(r * NW + wave) * 64 + lane] = sum[r];
    __syncthreads();
    if (rg == 0)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sum[r] = 0.0;
        for (int g = 0; g < RG; ++g) sum[r] += red[(r * NW + g * S + sg) * 64 + lane];
      }
  }
  if (rg == 0 && active) {
    if (u.kind == 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) t[r * ldt + u.out0 + o] = sum[r];
    } else {
      const int row = perm[u.out0 + o];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double* yp = y + r * ldy + row;
        *yp = beta == 0.0 ? alpha * sum[r] : fma(alpha, sum[r], beta * *yp);
      }
    }
  }
  __syncthreads();
}

template <typename T, int NW, int PHASE, int R>
__global__ __launch_bounds__(NW * 64) void k_phase_multi(BatchedArgs a, const double* __restrict__ x, int64_t ldx,
                                                         double* __restrict__ y, int64_t ldy, double alpha,
                                                         double beta) {
  __shared__ double zs[kStageMulti * R];
  __shared__ double red[R * NW * 64];
  const Unit u = a.units[(PHASE == 1 ? 0 : a.n1) + blockIdx.x];
  run_unit_multi<T, NW, R>(u, static_cast<const T*>(a.pool), x, ldx, y, ldy, a.perm, a.src, a.tm, a.t_size, a.sums,
                           a.t_size, alpha, beta, zs, red);
}

// Split schedule: one launch per phase (distinct symbols), one workgroup per
// unit, units in decreasing size.
template <typename T, int NW, int PHASE>
__global__ __launch_bounds__(NW * 64) void k_phase(BatchedArgs a, const double* __restrict__ x,
                                                   double* __restrict__ y, double alpha, double beta) {
  __shared__ double zs[kStage];
  __shared__ double red[NW * 64];
  const Unit u = a.units[(PHASE == 1 ? 0 : a.n1) + blockIdx.x];
  run_unit<T, NW, false>(u, static_cast<const T*>(a.pool), x, y, a.perm, a.src, a.t, a.sums, a.t_size, alpha, beta,
                         zs, red);
}

// Persistent schedule: one launch of resident workgroups that take units by
// ticket until none is left, phase 1 before phase 2.
//   * Tickets are sharded: shard s hands out units s, s + kShards, ...; a
//     workgroup draws from its own shard (blockIdx % kShards) and, once that
//     is exhausted, from the others in turn, one ticket after each unit
//     (drawing the next one early made workgroups hold two of the largest
//     units at once and ran slower).
//   * A workgroup that finds no phase-1 unit left in any shard adds the
//     number of phase-1 units it finished to its shard's done1 (after a
//     release fence) and waits until the done1 counts sum to n1; it then
//     acquires and goes on with phase 2.  Every phase-1 unit was claimed by a
//     running workgroup before any workgroup waits, so the wait ends; it is
//     bounded all the same (kSpinLimit polls, then the error counter is set
//     and the workgroup skips phase 2).
//   * The last workgroup of each shard to exit counts the shard in
//     exited_all; the last shard resets every counter for the next launch.
constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ unsigned atomic_add_agent(uint32_t* p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned load_agent_u(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int shard_units(int n, int s) { return n > s ? (n - s + kShards - 1) / kShards : 0; }

// Thread 0 only: the unit of ticket tk drawn on shard sh, or a ticket of the
// next shards once sh is exhausted; -1 when every shard is.
__device__ int resolve_ticket(PaddedCounter* tick, int n, int& sh, int& tried, unsigned tk) {
  for (;;) {
    if (tk < (unsigned)shard_units(n, sh)) return sh + kShards * (int)tk;
    if (++tried >= kShards) return -1;
    sh = (sh + 1) % kShards;
    tk = load_agent_u(&tick[sh].v) >= (unsigned)shard_units(n, sh) ? 0xffffffffu : atomic_add_agent(&tick[sh].v, 1u);
  }
}

template <typename T, int NW>
__global__ __launch_bounds__(NW * 64) void k_persistent(BatchedArgs a, const double* __restrict__ x,
                                                        double* __restrict__ y, double alpha, double beta) {
  __shared__ double zs[kStage];
  __shared__ double red[NW * 64];
  __shared__ int s_unit;
  QueueCounters* q = a.ctr;
  const int own = (int)(blockIdx.x % kShards);
  const T* pool = static_cast<const T*>(a.pool);
  bool ok = true;
  for (int phase = 1; phase <= 2 && ok; ++phase) {
    PaddedCounter* tick = phase == 1 ? q->tick1 : q->tick2;
    const int n = phase == 1 ? a.n1 : a.n2;
    const int base = phase == 1 ? 0 : a.n1;
    int sh = own, tried = 0, done = 0;
    for (;;) {
      if (threadIdx.x == 0) s_unit = resolve_ticket(tick, n, sh, tried, atomic_add_agent(&tick[sh].v, 1u));
      __syncthreads();
      const int cur = __builtin_amdgcn_readfirstlane(s_unit);
      __syncthreads();
      if (cur < 0) break;
      run_unit<T, NW, true>(a.units[base + cur], pool, x, y, a.perm, a.src, a.t, a.sums, a.t_size, alpha, beta, zs,
                            red);
      ++done;
    }
    if (phase == 1) {
      // publish, then wait for every phase-1 unit
      if (threadIdx.x == 0 && done > 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        atomic_add_agent(&q->done1[own].v, (unsigned)done);
      }
      if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        for (unsigned spins = 0;; ++spins) {
          unsigned v = lane < kShards ? load_agent_u(&q->done1[lane].v) : 0u;
#pragma unroll
          for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
          if (__builtin_amdgcn_readfirstlane(v) >= (unsigned)a.n1) break;
          if (spins >= kSpinLimit) {
            if (lane == 0) atomic_add_agent(&q->error.v, 1u);
            ok = false;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      if (threadIdx.x == 0) s_unit = ok ? 1 : 0;
      __syncthreads();
      ok = __builtin_amdgcn_readfirstlane(s_unit) != 0;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    const int in_shard = (int)((gridDim.x - own + kShards - 1) / kShards);
    const unsigned prev = __hip_atomic_fetch_add(&q->exited[own].v, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if ((int)prev == in_shard - 1) {
      const unsigned shards = gridDim.x < (unsigned)kShards ? gridDim.x : (unsigned)kShards;
      const unsigned p2 = __hip_atomic_fetch_add(&q->exited_all.v, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (p2 == shards - 1) {
        for (int s = 0; s < kShards; ++s) {
          __hip_atomic_store(&q->tick1[s].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&q->tick2[s].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&q->done1[s].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&q->exited[s].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __hip_atomic_store(&q->exited_all.v, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// ------------------------------------------------------------------------
// plain layout
// ------------------------------------------------------------------------
// Phase 1 (or its transpose): one workgroup of 256 per low-rank block;
// t[k] = sum_j F[k*len + j] x[perm[start + j]], F = V (forward) or U (transpose).
template <typename T>
__global__ __launch_bounds__(256) void k_plain_p1(PlainArgs a, const double* __restrict__ x, bool transpose) {
  __shared__ double part[4];
  const PlainBlock b = a.blocks[a.lr_list[blockIdx.x]];
  const T* pool = static_cast<const T*>(a.pool);
  const T* F = pool + (transpose ? b.offA : b.offB);
  const int len = transpose ? b.m : b.n;
  const int start = transpose ? b.r0 : b.c0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = 0; k < b.rank; ++k) {
    double acc = 0.0;
    for (int j = threadIdx.x; j < len; j += 256) acc += (double)F[(size_t)k * len + j] * x[a.perm[start + j]];
    acc = wave_sum(acc);
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a.t[b.tslot + k] = (part[0] + part[1]) + (part[2] + part[3]);
    __syncthreads();
  }
}

// Phase 2: one wave per row unit; lane i owns row row0 + i.
template <typename T>
__global__ __launch_bounds__(64) void k_plain_p2(PlainArgs a, const double* __restrict__ x, double* __restrict__ y,
                                                 double alpha, double beta) {
  const RowUnit u = a.rows[blockIdx.x];
  const int i = threadIdx.x;
  if (i >= u.m) return;
  const T* pool = static_cast<const T*>(a.pool);
  double acc = 0.0;
  for (int e = u.begin; e < u.end; ++e) {
    const UnitEntry en = a.row_ents[e];
    const PlainBlock b = a.blocks[en.block];
    const T* F = pool + b.offA + en.off + i;
    if (b.kind == 0) {
      for (int j = 0; j < b.n; ++j) acc += (double)F[(size_t)j * b.m] * x[a.perm[b.c0 + j]];
    } else {
      for (int k = 0; k < b.rank; ++k) acc += (double)F[(size_t)k * b.m] * a.t[b.tslot + k];
    }
  }
  const int row = a.perm[u.row0 + i];
  y[row] = beta == 0.0 ? alpha * acc : fma(alpha, acc, beta * y[row]);
}

// Phase 2 of the transpose: one wave per column unit; lane j owns column
// col0 + j of H, i.e. row col0 + j of H^T.
template <typename T>
__global__ __launch_bounds__(64) void k_plain_p2t(PlainArgs a, const double* __restrict__ x, double* __restrict__ y,
                                                  double alpha, double beta) {
  const RowUnit u = a.cols[blockIdx.x];
  const int j = threadIdx.x;
  if (j >= u.m) return;
  const T* pool = static_cast<const T*>(a.pool);
  double acc = 0.0;
  for (int e = u.begin; e < u.end; ++e) {
    const UnitEntry en = a.col_ents[e];
    const PlainBlock b = a.blocks[en.block];
    if (b.kind == 0) {
      const T* D = pool + b.offA + (size_t)(en.off + j) * b.m;
      for (int i = 0; i < b.m; ++i) acc += (double)D[i] * x[a.perm[b.r0 + i]];
    } else {
      const T* Vf = pool + b.offB + en.off + j;
      for (int k = 0; k < b.rank; ++k) acc += (double)Vf[(size_t)k * b.n] * a.t[b.tslot + k];
    }
  }
  const int row = a.perm[u.row0 + j];
  y[row] = beta == 0.0 ? alpha * acc : fma(alpha, acc, beta * y[row]);
}

template <typename T, int PHASE>
void launch_phase(const BatchedArgs& a, int nw, unsigned grid, const double* x, double* y, double alpha, double beta,
                  hipStream_t s) {
  switch (nw) {
    case 4: hipLaunchKernelGGL((k_phase<T, 4, PHASE>), dim3(grid), dim3(4 * 64), 0, s, a, x, y, alpha, beta); break;
    case 8: hipLaunchKernelGGL((k_phase<T, 8, PHASE>), dim3(grid), dim3(8 * 64), 0, s, a, x, y, alpha, beta); break;
    default: hipLaunchKernelGGL((k_phase<T, 16, PHASE>), dim3(grid), dim3(16 * 64), 0, s, a, x, y, alpha, beta);
  }
}

template <typename T>
void launch_persistent(const BatchedArgs& a, int nw, int grid, const double* x, double* y, double alpha, double beta,
                       hipStream_t s) {
  switch (nw) {
    case 4: hipLaunchKernelGGL((k_persistent<T, 4>), dim3(grid), dim3(4 * 64), 0, s, a, x, y, alpha, beta); break;
    case 8: hipLaunchKernelGGL((k_persistent<T, 8>), dim3(grid), dim3(8 * 64), 0, s, a, x, y, alpha, beta); break;
    default: hipLaunchKernelGGL((k_persistent<T, 16>), dim3(grid), dim3(16 * 64), 0, s, a, x, y, alpha, beta);
  }
}

template <typename T, int PHASE, int R>
void launch_phase_multi(const BatchedArgs& a, int nw, unsigned grid, const double* x, int64_t ldx, double* y,
                        int64_t ldy, double alpha, double beta, hipStream_t s) {
  switch (nw) {
    case 4:
      hipLaunchKernelGGL((k_phase_multi<T, 4, PHASE, R>), dim3(grid), dim3(4 * 64), 0, s, a, x, ldx, y, ldy, alpha,
                         beta);
      break;
    case 8:
      hipLaunchKernelGGL((k_phase_multi<T, 8, PHASE, R>), dim3(grid), dim3(8 * 64), 0, s, a, x, ldx, y, ldy, alpha,
                         beta);
      break;
    default:
      hipLaunchKernelGGL((k_phase_multi<T, 16, PHASE, R>), dim3(grid), dim3(16 * 64), 0, s, a, x, ldx, y, ldy, alpha,
                         beta);
  }
}

template <typename T, int NW>
int occupancy_nw() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<T, NW>, NW * 64, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace

template <typename T>
hipError_t launch_batched(const BatchedArgs& a, bool persistent, int grid, const double* x, double* y, double alpha,
                          double beta, hipStream_t s, hipEvent_t* ev) {
  const auto ok = [](int w) { return w == 4 || w == 8 || w == 16; };
  if (!ok(a.wg_waves) || !ok(a.wg_waves_p1)) return hipErrorInvalidValue;
  if (persistent) {
    if (a.wg_waves_p1 != a.wg_waves) return hipErrorInvalidValue;
    if (ev) (void)hipEventRecord(ev[0], s);
    if (a.n1 + a.n2 > 0) launch_persistent<T>(a, a.wg_waves, grid, x, y, alpha, beta, s);
    if (ev) (void)hipEventRecord(ev[1], s);
    return hipGetLastError();
  }
  if (ev) (void)hipEventRecord(ev[0], s);
  if (a.n1 > 0) launch_phase<T, 1>(a, a.wg_waves_p1, (unsigned)a.n1, x, y, alpha, beta, s);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (a.n2 > 0) launch_phase<T, 2>(a, a.wg_waves, (unsigned)a.n2, x, y, alpha, beta, s);
  if (ev) (void)hipEventRecord(ev[2], s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batched_multi(const BatchedArgs& a, int nvec, const double* x, int64_t ldx, double* y, int64_t ldy,
                                double alpha, double beta, hipStream_t s) {
  const auto ok = [](int w) { return w == 4 || w == 8 || w == 16; };
  if (!ok(a.wg_waves) || !ok(a.wg_waves_p1) || !a.tm || (nvec != 2 && nvec != 4)) return hipErrorInvalidValue;
  if (nvec == 2) {
    if (a.n1 > 0) launch_phase_multi<T, 1, 2>(a, a.wg_waves_p1, (unsigned)a.n1, x, ldx, y, ldy, alpha, beta, s);
    if (a.n2 > 0) launch_phase_multi<T, 2, 2>(a, a.wg_waves, (unsigned)a.n2, x, ldx, y, ldy, alpha, beta, s);
  } else {
    if (a.n1 > 0) launch_phase_multi<T, 1, 4>(a, a.wg_waves_p1, (unsigned)a.n1, x, ldx, y, ldy, alpha, beta, s);
    if (a.n2 > 0) launch_phase_multi<T, 2, 4>(a, a.wg_waves, (unsigned)a.n2, x, ldx, y, ldy, alpha, beta, s);
  }
  return hipGetLastError();
}

template <typename T>
int phase1_blocks_per_cu(int wg_waves_p1) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (wg_waves_p1) {
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phase<T, 4, 1>, 4 * 64, 0); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phase<T, 8, 1>, 8 * 64, 0); break;
    case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_phase<T, 16, 1>, 16 * 64, 0); break;
    default: break;
  }
  return e == hipSuccess && nb > 0 ? nb : 1;
}

template <typename T>
int persistent_blocks_per_cu(int wg_waves) {
  switch (wg_waves) {
    case 4: return occupancy_nw<T, 4>();
    case 8: return occupancy_nw<T, 8>();
    case 16: return occupancy_nw<T, 16>();
    default: return 1;
  }
}

template <typename T>
hipError_t launch_plain(const PlainArgs& a, bool transpose, const double* x, double* y, double alpha, double beta,
                        hipStream_t s, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], s);
  if (a.n_lr > 0) hipLaunchKernelGGL(k_plain_p1<T>, dim3(a.n_lr), dim3(256), 0, s, a, x, transpose);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (!transpose) {
    if (a.n_rows > 0) hipLaunchKernelGGL(k_plain_p2<T>, dim3(a.n_rows), dim3(64), 0, s, a, x, y, alpha, beta);
  } else {
    if (a.n_cols > 0) hipLaunchKernelGGL(k_plain_p2t<T>, dim3(a.n_cols), dim3(64), 0, s, a, x, y, alpha, beta);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  return hipGetLastError();
}

template hipError_t launch_batched<float>(const BatchedArgs&, bool, int, const double*, double*, double, double,
                                          hipStream_t, hipEvent_t*);
template hipError_t launch_batched<double>(const BatchedArgs&, bool, int, const double*, double*, double, double,
                                           hipStream_t, hipEvent_t*);
template hipError_t launch_batched_multi<float>(const BatchedArgs&, int, const double*, int64_t, double*, int64_t,
                                                double, double, hipStream_t);
template hipError_t launch_batched_multi<double>(const BatchedArgs&, int, const double*, int64_t, double*, int64_t,
                                                 double, double, hipStream_t);
template int persistent_blocks_per_cu<float>(int);
template int persistent_blocks_per_cu<double>(int);
template int phase1_blocks_per_cu<float>(int);
template int phase1_blocks_per_cu<double>(int);
template hipError_t launch_plain<float>(const PlainArgs&, bool, const double*, double*, double, double, hipStream_t,
                                        hipEvent_t*);
template hipError_t launch_plain<double>(const PlainArgs&, bool, const double*, double*, double, double, hipStream_t,
                                         hipEvent_t*);

}  // namespace hm
