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
// ([part][input][64]), so staging one input moves 16-byte chunks of 8
// members; LDS holds them input-contiguous per member ([part][member][k]),
// the order the MFMA operand wants.  The panels are split on the fly as they
// stream from HBM.
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels_mm.hpp"

namespace hm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

constexpr int kNR = 64;       // members per product (N)
constexpr int kKS = 128;      // inputs staged per round (K)
constexpr int kLd = kKS + 8;  // LDS row pitch in bf16 (pad against bank conflicts)
constexpr int kWaves = 4;

// LDS column of input kk in member row r: 16-byte chunks of 8 inputs are
// XOR-swizzled by the row group (r / 8) so that the eight rows written by one
// staged 16-byte load fall into different banks; an MFMA operand read (8
// consecutive inputs of one row) stays one aligned 16-byte chunk.
__device__ __forceinline__ int zcol(int r, int kk) { return (((kk >> 3) ^ ((r >> 3) & 7)) << 3) | (kk & 7); }

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
template <int NS>
__global__ __launch_bounds__(256) void k_split_members(int64_t n, int nrhs, const double* __restrict__ X,
                                                       int64_t ldx, const int32_t* __restrict__ perm,
                                                       __bf16* __restrict__ Xs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (k, r)
  if (e >= n * kNR) return;
  const int64_t k = e / kNR;
  const int r = (int)(e % kNR);
  const float v = r < nrhs ? (float)X[(int64_t)perm[k] * ldx + r] : 0.f;
  __bf16 p[NS];
  split<NS>(v, p);
#pragma unroll
  for (int i = 0; i < NS; ++i) Xs[((int64_t)i * n + k) * kNR + r] = p[i];
}

// MT: output tiles of 16 per wave (phase-2 units have at most 64 outputs: 1).
template <int NS, int PHASE, int MT>
__global__ __launch_bounds__(kWaves * 64) void k_mm(MMArgs a, double alpha, double beta) {
  const __bf16* __restrict__ Xs = static_cast<const __bf16*>(a.Xs);
  __bf16* Ts = static_cast<__bf16*>(a.Ts);
  // bf16 bit patterns as 16-bit integers (whole vectors are bit-cast to bf16)
  __shared__ __attribute__((aligned(16))) unsigned short zs[NS][kNR][kLd];
  const Unit u = a.units[(PHASE == 1 ? 0 : a.n1) + blockIdx.x];
  const float* pool = static_cast<const float*>(a.pool);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int lm = lane & 15, lk = lane >> 4;  // MFMA lane: row/col within 16, k group of 8
  const int ntiles = (u.nout + 15) >> 4;     // 16-output tiles, up to MT per wave
  const int K = u.nq * 4;
  f32x4 acc[MT][4];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int c0 = 0; c0 < K; c0 += kKS) {
    // stage inputs c0 .. c0+kKS: items (part, input, 8-member chunk), one
    // 16-byte load each, scattered into LDS input-contiguous per member
    for (int e = tid; e < NS * kKS * 8; e += kWaves * 64) {
      const int ch = e & 7, kk = (e >> 3) % kKS, p = e / (8 * kKS);
      const int k = c0 + kk;
      s16x8 v = s16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (k < K) {
        const s16x8* srcp = nullptr;
        if (PHASE == 1) {
          if (k < u.nin) srcp = reinterpret_cast<const s16x8*>(Xs + (((int64_t)p * a.n + u.in0 + k) * kNR + 8 * ch));
        } else {
          const int s = a.src[u.in0 + k];
          if (s >= 0)
            srcp = reinterpret_cast<const s16x8*>(Xs + (((int64_t)p * a.n + a.invperm[s]) * kNR + 8 * ch));
          else if (s < -1)
            srcp = reinterpret_cast<const s16x8*>(Ts + (((int64_t)p * a.t_size + (-s - 1)) * kNR + 8 * ch));
        }
        if (srcp) v = *srcp;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) zs[p][8 * ch + j][zcol(8 * ch + j, kk)] = (unsigned short)v[j];
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      const int mt = wave + kWaves * t;
      if (mt >= ntiles) break;
      const int o = mt * 16 + lm;
      const bool orow = o < u.nout;
#pragma unroll 2
      for (int ks = 0; ks < kKS; ks += 32) {
        // A fragment: output o, inputs c0 + ks + 8 lk + [0, 8): two panel quads
        const int q = (c0 + ks) / 4 + 2 * lk;
        float av[8];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
          if (orow && q + h < u.nq) v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(
                                        pool + u.off + ((size_t)(q + h) * u.nout + o) * 4));
          av[4 * h + 0] = v[0];
          av[4 * h + 1] = v[1];
          av[4 * h + 2] = v[2];
          av[4 * h + 3] = v[3];
        }
        bf16x8 ap[NS];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 pp[NS];
          split<NS>(av[j], pp);
#pragma unroll
          for (int i = 0; i < NS; ++i) ap[i][j] = pp[i];
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          bf16x8 bp[NS];
#pragma unroll
          for (int i = 0; i < NS; ++i)
            bp[i] = __builtin_bit_cast(
                bf16x8, *reinterpret_cast<const s16x8*>(&zs[i][nt * 16 + lm][zcol(nt * 16 + lm, ks + 8 * lk)]));
#pragma unroll
          for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int j = 0; j < NS - i; ++j)
              acc[t][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[i], bp[j], acc[t][nt], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // write: lane holds rows mt*16 + 4 lk + [0,4), member nt*16 + lm
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    const int mt = wave + kWaves * t;
    if (mt >= ntiles) break;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int r = nt * 16 + lm;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = mt * 16 + 4 * lk + i;
        if (o >= u.nout) continue;
        const float v = acc[t][nt][i];
        if (PHASE == 1) {
          __bf16 pp[NS];
          split<NS>(v, pp);
          const int64_t slot = (int64_t)u.out0 + o;
#pragma unroll
          for (int p = 0; p < NS; ++p) Ts[((int64_t)p * a.t_size + slot) * kNR + r] = pp[p];
        } else if (r < a.nrhs) {
          double* yp = a.Y + (int64_t)a.perm[u.out0 + o] * a.ldy + r;
          *yp = beta == 0.0 ? alpha * (double)v : fma(alpha, (double)v, beta * *yp);
        }
      }
    }
  }
}

template <int NS>
hipError_t launch_ns(const MMArgs& a, double alpha, double beta, hipStream_t s, hipEvent_t* ev) {
  const int64_t n = a.n;
  if (ev) (void)hipEventRecord(ev[0], s);
  hipLaunchKernelGGL((k_split_members<NS>), dim3((unsigned)((n * kNR + 255) / 256)), dim3(256), 0, s, n, a.nrhs, a.X,
                     a.ldx, a.perm, static_cast<__bf16*>(a.Xs));
  if (a.n1 > 0) hipLaunchKernelGGL((k_mm<NS, 1, 4>), dim3(a.n1), dim3(kWaves * 64), 0, s, a, alpha, beta);
  if (ev) (void)hipEventRecord(ev[1], s);
  if (a.n2 > 0) hipLaunchKernelGGL((k_mm<NS, 2, 1>), dim3(a.n2), dim3(kWaves * 64), 0, s, a, alpha, beta);
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
