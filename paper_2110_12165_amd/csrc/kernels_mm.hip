// Ensemble product Y = H X for up to 64 right-hand sides on MFMA (gfx950).
//
// Eq. (20) applied to a block of slip-rate vectors: phase 1 forms
// T = V^T X per column cluster, phase 2 forms Y_I = D X_J + U T per row
// interval, over the same work units and packed panels as the single-vector
// product.  Each unit is now a small matrix product (outputs x inputs times
// inputs x 64 members) computed with v_mfma_f32_16x16x32_bf16.  Operands
// are split into bf16 parts (x = p0 + p1 + p2, each part the bf16 rounding
// of the remainder; three parts represent an FP32 value exactly) and the
// cross products with i + j < NS are accumulated in FP32:
//   NS = 2: p0q0 + p0q1 + p1q0              (3 products, "BF16x3")
//   NS = 3: ... + p0q2 + p1q1 + p2q0         (6 products, "BF16x6")
// The members' values are kept split, in cluster order, member-contiguous
// ([part][input][64]), and are staged into LDS unchanged (16-byte copies):
// one LDS row per input, 64 members.  The MFMA B operand wants 8 consecutive
// inputs of one member per lane; gfx950's transposing LDS read
// (ds_read_b64_tr_b16) delivers exactly that from member-contiguous rows.
// The panels are split on the fly as they stream from HBM.
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels_mm.hpp"

namespace hm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

constexpr int kNR = 64;       // members per product (N)
// Inputs staged per round (KS, 32 or 64, a template argument of the kernel).
// Measured (per phase, N = 122880 / 21000): BF16x3 runs faster with rounds
// of 64 in both phases; BF16x6 phase 2 with rounds of 32 (340 against 367 us
// / 101 against 125 us: its 3-part LDS rows then need 12 KB, not 24, and
// more workgroups fit), BF16x6 phase 1 with 32 when it has many slices
// (N = 122880: 260 against 281 us) and with 64 when it has few (N = 21000:
// 90 against 108 us).
constexpr int kWaves = 4;

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

// Physical 16-byte chunk (8 members) of member chunk ch in LDS row r.  The
// XOR with row bits 1 and 3 makes both the staging writes (two rows of eight
// chunks per 16 lanes) and the transposing reads (four rows of two chunks per
// 16 lanes, two such groups per half-wave) free of bank conflicts.
__device__ __forceinline__ int zchunk(int r, int ch) { return ch ^ (r & 2) ^ ((r >> 1) & 4); }

// B fragment of v_mfma_f32_16x16x32_bf16 for inputs k0 + [0, 32) and members
// m0 + [0, 16) from member-contiguous LDS rows: lane l receives inputs
// k0 + 8 (l / 16) + [0, 8) of member m0 + l % 16.  ds_read_b64_tr_b16 gives
// lane i of a 16-lane group element i % 4 of the 4-element vectors addressed
// by lanes 4e + i / 4 (e = 0..3, one per result element), so lane j of the
// group addresses input row (j / 4) and members 4 (j % 4) + [0, 4).
__device__ __forceinline__ s16x8 b_fragment(const unsigned short (*z)[kNR], int k0, int m0, int lane) {
  const int g = lane >> 4, j = lane & 15;
  const int col = m0 + 4 * (j & 3);
  s16x4 h[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int row = k0 + 8 * g + 4 * t + (j >> 2);
    const unsigned short* p = &z[row][8 * zchunk(row, col >> 3) + (col & 7)];
    h[t] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4*)(p));
  }
  return s16x8{h[0][0], h[0][1], h[0][2], h[0][3], h[1][0], h[1][1], h[1][2], h[1][3]};
}

template <int NS>
__device__ __forceinline__ void split(float x, __bf16* p) {
  float r = x;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const __bf16 h = (__bf16)r;
    p[i] = h;
    r = r - (float)h;
  }
}

// Member values of the inputs, split: Xs[p][k][r] (cluster order k < n).
// One thread per input and four members (8-byte stores per part); VEC: X and
// ldx allow 16-byte loads.
template <int NS, bool VEC>
__global__ __launch_bounds__(256) void k_split_members(int64_t n, int nrhs, const double* __restrict__ X,
                                                       int64_t ldx, const int32_t* __restrict__ perm,
                                                       __bf16* __restrict__ Xs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (k, members 4 j + [0, 4))
  if (e >= n * (kNR / 4)) return;
  const int64_t k = e / (kNR / 4);
  const int r0 = 4 * (int)(e % (kNR / 4));
  const double* xr = X + (int64_t)perm[k] * ldx + r0;
  float v[4];
  if (VEC && r0 + 4 <= nrhs) {
    typedef double f64x2 __attribute__((ext_vector_type(2)));
    const f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(xr));
    const f64x2 b = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(xr) + 1);
    v[0] = (float)a[0];
    v[1] = (float)a[1];
    v[2] = (float)b[0];
    v[3] = (float)b[1];
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = r0 + j < nrhs ? (float)xr[j] : 0.f;
  }
  __bf16 p[4][NS];
#pragma unroll
  for (int j = 0; j < 4; ++j) split<NS>(v[j], p[j]);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    *reinterpret_cast<bf16x4*>(Xs + ((int64_t)i * n + k) * kNR + r0) = bf16x4{p[0][i], p[1][i], p[2][i], p[3][i]};
  }
}

// 16-byte staging items per thread and part
template <int KS>
constexpr int items_of() { return KS * 8 / (kWaves * 64); }

// Workgroups are dealt to the 8 XCDs round-robin in dispatch order, and each
// XCD has its own L2.  The 64-output slices of one phase-1 unit stage the
// same inputs; this maps workgroup b to a logical item so that chunks of
// kChunk consecutive items (a unit's slices) run on one XCD at nearly the
// same time, while the chunks still rotate over the XCDs.  A bijection of
// [0, G); the last G mod (8 kChunk) items keep their index.  Measured at
// N = 122880: phase 1 -5 %; phase 2 (one unit per row interval, no shared
// slices) gains nothing from it, nor from dispatching its units in row
// order, and keeps the identity (largest units first).
constexpr int kXcds = 8;
constexpr int kChunk = 4;
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int full = G / (kXcds * kChunk) * (kXcds * kChunk);
  if (b >= full) return b;
  const int xcd = b % kXcds, rest = b / kXcds;
  return ((rest / kChunk) * kXcds + xcd) * kChunk + rest % kChunk;
}

// Members of inputs c0 + [0, K_S) of a unit, split parts, read into registers
// (item e = tid + 256 i: input e / 8, 8-member chunk e % 8); zero beyond the
// unit's inputs and for the zero pad of the intermediate vector.
template <int NS, int PHASE, int KS>
__device__ __forceinline__ void stage_load(const MMArgs& a, const Unit& u, int c0, int K, int tid,
                                           s16x8 (&sr)[NS][items_of<KS>()]) {
  const __bf16* __restrict__ Xs = static_cast<const __bf16*>(a.Xs);
  const __bf16* Ts = static_cast<const __bf16*>(a.Ts);
#pragma unroll
  for (int it = 0; it < items_of<KS>(); ++it) {
    const int e = tid + it * kWaves * 64;
    const int ch = e & 7, k = c0 + (e >> 3);
    const __bf16* row = nullptr;
    int64_t part = 0;
    if (k < K) {
      if (PHASE == 1) {
        if (k < u.nin) {
          row = Xs + ((int64_t)u.in0 + k) * kNR;
          part = a.n * kNR;
        }
      } else {
        const int sx = a.src[u.in0 + k];
        if (sx >= 0) {
          row = Xs + (int64_t)a.invperm[sx] * kNR;
          part = a.n * kNR;
        } else if (sx < -1) {
          row = Ts + (int64_t)(-sx - 1) * kNR;
          part = a.t_size * kNR;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < NS; ++p)
      sr[p][it] = row ? *reinterpret_cast<const s16x8*>(row + p * part + 8 * ch) : s16x8{0, 0, 0, 0, 0, 0, 0, 0};
  }
}

template <int NS, int KS>
__device__ __forceinline__ void stage_store(unsigned short (*zs)[KS][kNR], int tid,
                                            const s16x8 (&sr)[NS][items_of<KS>()]) {
#pragma unroll
  for (int it = 0; it < items_of<KS>(); ++it) {
    const int e = tid + it * kWaves * 64;
    const int ch = e & 7, kk = e >> 3;
#pragma unroll
    for (int p = 0; p < NS; ++p) *reinterpret_cast<s16x8*>(&zs[p][kk][8 * zchunk(kk, ch)]) = sr[p][it];
  }
}

// Panel quads of output o for the NST 32-input steps of the round at c0:
// step s, half h = quad (c0 + 32 s) / 4 + 2 lk + h.
template <int NST>
__device__ __forceinline__ void load_a(const float* pool, const Unit& u, int c0, int o, bool orow, int lk,
                                       f32x4 (&ar)[NST][2]) {
#pragma unroll
  for (int st = 0; st < NST; ++st)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = (c0 + 32 * st) / 4 + 2 * lk + h;
      ar[st][h] = (orow && q < u.nq) ? __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(
                                           pool + u.off + ((size_t)q * u.nout + o) * 4))
                                     : f32x4{0.f, 0.f, 0.f, 0.f};
    }
}

// One workgroup per 64-output slice of a unit (phase-1 units with more than
// 64 outputs are split into slices that stage the same inputs); wave w owns
// the 16 outputs 16 (w % 4) + [0, 16) of the slice and all 64 members.
// G2 groups of four waves share a slice: group g takes rounds g, g + G2, ...
// into its own LDS rows, and the groups' sums are added in group order at
// the end.  G2 = 2 halves the path of every workgroup and the workgroups
// resident per compute unit; the caller chooses per phase (MMArgs groups).
// Rounds are software-pipelined: the members and panel quads of a group's
// next round are loaded into registers while the MFMAs of its current round
// run, and written to LDS after it.
template <int NS, int PHASE, int KS, int G2>
__global__ __launch_bounds__(kWaves * 64 * G2) void k_mm(MMArgs a, double alpha, double beta) {
  __bf16* Ts = static_cast<__bf16*>(a.Ts);
  // bf16 bit patterns as 16-bit integers (whole vectors are bit-cast to bf16);
  // row = input of the round, 64 members, chunks swizzled by zchunk
  __shared__ __attribute__((aligned(16))) unsigned short zs[G2][NS][KS][kNR];
  static_assert(sizeof(zs) >= (G2 > 1 ? kWaves * 64 * 16 * sizeof(float) : 0), "LDS too small for the group sums");
  int ui, ob = 0;
  if (PHASE == 1) {
    const int code = a.slices1[xcd_remap((int)blockIdx.x, (int)gridDim.x)];
    ui = code >> 4;
    ob = 64 * (code & 15);
  } else {
    ui = a.n1 + blockIdx.x;
  }
  const Unit u = a.units[ui];
  const float* pool = static_cast<const float*>(a.pool);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int grp = wave / kWaves, gw = wave % kWaves, gtid = tid % (kWaves * 64);
  const int lm = lane & 15, lk = lane >> 4;  // MFMA lane: row/col within 16, k group of 8
  const int ntiles = (min(u.nout, ob + 64) - ob + 15) >> 4;
  const int K = u.nq * 4;
  const int rounds = (K + KS - 1) / KS;
  const int iters = (rounds + G2 - 1) / G2;  // rounds of one group (the last ones may be empty)
  const int o = ob + gw * 16 + lm;
  const bool work = gw < ntiles, orow = work && o < u.nout;
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  s16x8 sr[NS][items_of<KS>()];
  f32x4 ar[KS / 32][2], an[KS / 32][2];
  stage_load<NS, PHASE, KS>(a, u, grp * KS, K, gtid, sr);
  if (work) load_a(pool, u, grp * KS, o, orow, lk, ar);
  stage_store<NS, KS>(zs[grp], gtid, sr);
  __syncthreads();

  for (int it = 0; it < iters; ++it) {
    const bool more = it + 1 < iters;
    const int next = ((it + 1) * G2 + grp) * KS;  // first input of this group's next round
    if (more) {
      stage_load<NS, PHASE, KS>(a, u, next, K, gtid, sr);
      if (work) load_a(pool, u, next, o, orow, lk, an);
    }
    if (work) {
#pragma unroll
      for (int st = 0; st < KS / 32; ++st) {
        // A fragment: output o, inputs 32 st + 8 lk + [0, 8) of the round
        bf16x8 ap[NS];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 pp[NS];
          split<NS>(ar[st][j >> 2][j & 3], pp);
#pragma unroll
          for (int i = 0; i < NS; ++i) ap[i][j] = pp[i];
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          bf16x8 bp[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i)
            bp[i] = __builtin_bit_cast(bf16x8, b_fragment(zs[grp][i], 32 * st, nt * 16, lane));
#pragma unroll
          for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = 0; j < NS - i; ++j)
              acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i], bp[j], acc[nt], 0, 0, 0);
        }
        // keep the scheduler from hoisting the LDS reads of later steps
        // (their fragments would all be live at once)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
    if (more) {
      stage_store<NS, KS>(zs[grp], gtid, sr);
#pragma unroll
      for (int st = 0; st < KS / 32; ++st) {
        ar[st][0] = an[st][0];
        ar[st][1] = an[st][1];
      }
      __syncthreads();
    }
  }
  if (G2 > 1) {
    // groups 1.. hand their sums to group 0 through LDS (the rows are no
    // longer read: every group passed the barrier after its last MFMAs)
    float* red = reinterpret_cast<float*>(&zs[0][0][0][0]);
    for (int g = 1; g < G2; ++g) {
      if (grp == g && work)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) red[(gw * 64 + lane) * 16 + nt * 4 + i] = acc[nt][i];
      __syncthreads();
      if (grp == 0 && work)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[nt][i] += red[(gw * 64 + lane) * 16 + nt * 4 + i];
      __syncthreads();
    }
    if (grp != 0) return;
  }
  if (!work) return;
  // write: lane holds outputs ob + 16 gw + 4 lk + [0, 4), member 16 nt + lm
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int r = nt * 16 + lm;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int oo = ob + gw * 16 + 4 * lk + i;
      if (oo >= u.nout) continue;
      const float v = acc[nt][i];
      if (PHASE == 1) {
        __bf16 pp[NS];
        split<NS>(v, pp);
        const int64_t slot = (int64_t)u.out0 + oo;
#pragma unroll
        for (int p = 0; p < NS; ++p) Ts[((int64_t)p * a.t_size + slot) * kNR + r] = pp[p];
      } else if (r < a.nrhs) {
        double* yp = a.Y + (int64_t)a.perm[u.out0 + oo] * a.ldy + r;
        *yp = beta == 0.0 ? alpha * (double)v : fma(alpha, (double)v, beta * *yp);
      }
    }
  }
}

// Phase 2 on pairs of row intervals (layouts built with paired inputs:
// Unit::ncom leading inputs are common to both intervals of a pair, in the
// same order).  Eight waves: group g (four waves) owns interval g of the
// pair, 16 rows per wave and all 64 members, over its own panel.  Round r
// (inputs r KS + [0, KS) of a group's list) lies wholly inside the common
// inputs for r < ncom / KS: those rounds are staged once, by all eight
// waves, into shared LDS rows that both groups read; every later round each
// group stages from its own list into its own rows.  A pair stages its
// common inputs once instead of twice (at N = 122880: 0.53 GB of staging
// demand instead of 0.88 GB).  Rounds are software-pipelined like k_mm's.
constexpr int kPairWaves = 2 * kWaves;

template <int NS, int KS>
__device__ __forceinline__ void pair_stage_load(const MMArgs& a, const int32_t* __restrict__ src, int c0, int K,
                                                int e0, int estep, s16x8 (&sr)[NS][KS * 8 / (kWaves * 64)]) {
  const __bf16* __restrict__ Xs = static_cast<const __bf16*>(a.Xs);
  const __bf16* Ts = static_cast<const __bf16*>(a.Ts);
  constexpr int kItems = KS * 8 / (kWaves * 64);
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int e = e0 + it * estep;
    const int ch = e & 7, k = c0 + (e >> 3);
    const __bf16* row = nullptr;
    int64_t part = 0;
    if (e < KS * 8 && k < K) {
      const int sx = src[k];
      if (sx >= 0) {
        row = Xs + (int64_t)a.invperm[sx] * kNR;
        part = a.n * kNR;
      } else if (sx < -1) {
        row = Ts + (int64_t)(-sx - 1) * kNR;
        part = a.t_size * kNR;
      }
    }
#pragma unroll
    for (int p = 0; p < NS; ++p)
      sr[p][it] = row ? *reinterpret_cast<const s16x8*>(row + p * part + 8 * ch) : s16x8{0, 0, 0, 0, 0, 0, 0, 0};
  }
}

template <int NS, int KS>
__device__ __forceinline__ void pair_stage_store(unsigned short (*zs)[KS][kNR], int e0, int estep,
                                                 const s16x8 (&sr)[NS][KS * 8 / (kWaves * 64)]) {
  constexpr int kItems = KS * 8 / (kWaves * 64);
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int e = e0 + it * estep;
    if (e >= KS * 8) continue;
    const int ch = e & 7, kk = e >> 3;
#pragma unroll
    for (int p = 0; p < NS; ++p) *reinterpret_cast<s16x8*>(&zs[p][kk][8 * zchunk(kk, ch)]) = sr[p][it];
  }
}

template <int NS, int KS>
__global__ __launch_bounds__(kPairWaves * 64) void k_mm_pair(MMArgs a, double alpha, double beta) {
  // [0]: shared rows of the common rounds; [1 + g]: rows of group g
  __shared__ __attribute__((aligned(16))) unsigned short zs[3][NS][KS][kNR];
  const int ia = a.pairs[2 * blockIdx.x], ib = a.pairs[2 * blockIdx.x + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int grp = wave / kWaves, gw = wave % kWaves, gtid = tid % (kWaves * 64);
  const int mine = grp == 0 ? ia : ib;  // -1: interval without a partner, group 1 idle
  Unit u{};
  if (mine >= 0) u = a.units[a.n1 + mine];
  const float* pool = static_cast<const float*>(a.pool);
  const int lm = lane & 15, lk = lane >> 4;
  const int K = u.nq * 4;
  const int rounds = (K + KS - 1) / KS;
  const Unit ua = a.units[a.n1 + ia];
  const int rounds_a = (ua.nq * 4 + KS - 1) / KS;
  const int rounds_b = ib >= 0 ? (a.units[a.n1 + ib].nq * 4 + KS - 1) / KS : 0;
  const int total = max(rounds_a, rounds_b);
  const int nsh = ib >= 0 ? ua.ncom / KS : 0;  // rounds inside the common inputs
  const int32_t* src_a = a.src + ua.in0;        // the common inputs, as listed by interval a
  const int32_t* src_me = a.src + u.in0;
  const int ntiles = (u.nout + 15) >> 4;
  const int o = gw * 16 + lm;
  const bool work = gw < ntiles, orow = work && o < u.nout;
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  constexpr int kItems = KS * 8 / (kWaves * 64);
  s16x8 sr[NS][kItems];
  f32x4 ar[KS / 32][2], an[KS / 32][2];
  // staging of round r: shared rounds by all eight waves (items tid, tid + 512,
  // ...), the others by each group for itself (gtid, gtid + 256, ...)
  auto load_round = [&](int r) {
    if (r < nsh) pair_stage_load<NS, KS>(a, src_a, r * KS, ua.nq * 4, tid, kPairWaves * 64, sr);
    else if (r < rounds) pair_stage_load<NS, KS>(a, src_me, r * KS, K, gtid, kWaves * 64, sr);
  };
  auto store_round = [&](int r) {
    if (r < nsh) pair_stage_store<NS, KS>(zs[0], tid, kPairWaves * 64, sr);
    else if (r < rounds) pair_stage_store<NS, KS>(zs[1 + grp], gtid, kWaves * 64, sr);
  };
  load_round(0);
  if (work && rounds > 0) load_a(pool, u, 0, o, orow, lk, ar);
  store_round(0);
  __syncthreads();
  for (int r = 0; r < total; ++r) {
    const bool more = r + 1 < total;
    if (more) {
      load_round(r + 1);
      if (work && r + 1 < rounds) load_a(pool, u, (r + 1) * KS, o, orow, lk, an);
    }
    if (work && r < rounds) {
      const int region = r < nsh ? 0 : 1 + grp;
#pragma unroll
      for (int st = 0; st < KS / 32; ++st) {
        bf16x8 ap[NS];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 pp[NS];
          split<NS>(ar[st][j >> 2][j & 3], pp);
#pragma unroll
          for (int i = 0; i < NS; ++i) ap[i][j] = pp[i];
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          bf16x8 bp[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i)
            bp[i] = __builtin_bit_cast(bf16x8, b_fragment(zs[region][i], 32 * st, nt * 16, lane));
#pragma unroll
          for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = 0; j < NS - i; ++j)
              acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i], bp[j], acc[nt], 0, 0, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __syncthreads();
    if (more) {
      store_round(r + 1);
#pragma unroll
      for (int st = 0; st < KS / 32; ++st) {
        ar[st][0] = an[st][0];
        ar[st][1] = an[st][1];
      }
      __syncthreads();
    }
  }
  if (!work) return;
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int r = nt * 16 + lm;
    if (r >= a.nrhs) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int oo = gw * 16 + 4 * lk + i;
      if (oo >= u.nout) continue;
      double* yp = a.Y + (int64_t)a.perm[u.out0 + oo] * a.ldy + r;
      const float v = acc[nt][i];
      *yp = beta == 0.0 ? alpha * (double)v : fma(alpha, (double)v, beta * *yp);
    }
  }
}

constexpr int kManySlices = 16;  // phase-1 slices per compute unit from which BF16x6 stages 32 inputs

template <int NS>
hipError_t launch_ns(const MMArgs& a, double alpha, double beta, hipStream_t s, hipEvent_t* ev) {
  const int64_t n = a.n;
  if (ev) (void)hipEventRecord(ev[0], s);
  const dim3 gs((unsigned)((n * (kNR / 4) + 255) / 256));
  if (reinterpret_cast<uintptr_t>(a.X) % 16 == 0 && a.ldx % 2 == 0)
    hipLaunchKernelGGL((k_split_members<NS, true>), gs, dim3(256), 0, s, n, a.nrhs, a.X, a.ldx, a.perm,
                       static_cast<__bf16*>(a.Xs));
  else
    hipLaunchKernelGGL((k_split_members<NS, false>), gs, dim3(256), 0, s, n, a.nrhs, a.X, a.ldx, a.perm,
                       static_cast<__bf16*>(a.Xs));
  const dim3 g1((unsigned)a.ns1), g2((unsigned)a.n2);
  const bool two1 = a.groups1 == 2, two2 = a.groups2 == 2;
  if (a.ns1 > 0) {
    if (NS == 3 && a.ns1 >= kManySlices * a.cus) {
      if (two1) hipLaunchKernelGGL((k_mm<NS, 1, 32, 2>), g1, dim3(2 * kWaves * 64), 0, s, a, alpha, beta);
      else hipLaunchKernelGGL((k_mm<NS, 1, 32, 1>), g1, dim3(kWaves * 64), 0, s, a, alpha, beta);
    } else if (two1) {
      hipLaunchKernelGGL((k_mm<NS, 1, 64, 2>), g1, dim3(2 * kWaves * 64), 0, s, a, alpha, beta);
    } else {
      hipLaunchKernelGGL((k_mm<NS, 1, 64, 1>), g1, dim3(kWaves * 64), 0, s, a, alpha, beta);
    }
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (a.n2 > 0) {
    constexpr int KS2 = NS == 3 ? 32 : 64;
    if (a.groups2 == kGroupsPairs && a.npairs > 0)
      hipLaunchKernelGGL((k_mm_pair<NS, KS2>), dim3((unsigned)a.npairs), dim3(kPairWaves * 64), 0, s, a, alpha, beta);
    else if (two2) hipLaunchKernelGGL((k_mm<NS, 2, KS2, 2>), g2, dim3(2 * kWaves * 64), 0, s, a, alpha, beta);
    else hipLaunchKernelGGL((k_mm<NS, 2, KS2, 1>), g2, dim3(kWaves * 64), 0, s, a, alpha, beta);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mm(const MMArgs& a, int parts, double alpha, double beta, hipStream_t s, hipEvent_t* ev) {
  if (a.nrhs < 1 || a.nrhs > kNR) return hipErrorInvalidValue;
  if (parts == 2) return launch_ns<2>(a, alpha, beta, s, ev);
  if (parts == 3) return launch_ns<3>(a, alpha, beta, s, ev);
  return hipErrorInvalidValue;
}

}  // namespace hm
