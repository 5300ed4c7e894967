// Plain structs shared by the host packer and the HIP kernels.
#pragma once

#include <cstdint>

namespace hm {

// Block of the natural layout: dense block column-major m x n at offA;
// low-rank block U (m x rank, column-major) at offA and V (n x rank,
// column-major) at offB.  Rows and columns in cluster order.  tslot: first
// entry of the block's intermediate vector t = V^T x (and s = U^T x for the
// transpose).
struct PlainBlock {
  int32_t kind, r0, m, c0, n, rank, tslot, pad;
  int64_t offA, offB;
};

// Row-owned unit of the natural layout: rows [row0, row0 + m) (m <= 64) and
// the blocks meeting them, entries [begin, end) of the entry list.
struct RowUnit {
  int32_t row0, m, begin, end;
};

// (block, first row of this unit inside the block) — or first column for the
// column-owned units of the transpose.
struct UnitEntry {
  int32_t block, off;
};

// Work unit of the batched layout.  Its panel holds nq input groups; each
// group stores, for every output lane, W consecutive inputs (16 bytes):
//   panel[(q * nout + o) * W + c] = coefficient of input q*W + c for output o.
// kind 1 (phase 1, t = V^T x): outputs are intermediate values of one column
//   cluster, inputs are its rows in0 + [0, nin) (gathered from x through the
//   permutation; rows beyond nin are zero padding); result o goes to
//   t[out0 + o].
// kind 2 (phase 2, y = D x + U t): outputs are rows out0 + [0, nout) in
//   cluster order, inputs are described by src[in0 + i] (>= 0: element of x
//   in user order; < 0: entry -src-1 of t, entry 0 being a zero pad).
// Waves w < S*RG work: output group w % S (outputs 64*(w % S) + lane), input
//   groups q = w / S (mod RG); partial sums of the RG input groups are added
//   in LDS in a fixed order.
// ncom (kind 2, layouts for the ensemble product): the first ncom inputs are
//   the ones this interval shares with the other interval of its pair, in
//   the same order in both lists (0 otherwise).
struct Unit {
  int32_t nout, nq, S, RG, in0, nin, out0, kind;
  int32_t ncom, pad;
  int64_t off;
};

// Counters of the persistent schedule, each in its own 128-byte line and
// sharded over kShards addresses (workgroup b uses shard b % kShards), so
// that no single address takes an atomic from every workgroup: on this GPU
// device-scope atomics on one address are served one at a time.  Reset by
// the last workgroup to exit.
constexpr int kShards = 8;
struct alignas(128) PaddedCounter {
  uint32_t v;
  uint32_t pad[31];
};
struct QueueCounters {
  PaddedCounter tick1[kShards];   // phase-1 tickets; shard s hands out units s, s + kShards, ...
  PaddedCounter tick2[kShards];   // phase-2 tickets (unit indices relative to n1)
  PaddedCounter done1[kShards];   // phase-1 units finished, counted by the finishing workgroup's shard
  PaddedCounter exited[kShards];  // workgroups of the shard that have exited
  PaddedCounter exited_all;       // shards whose workgroups have all exited
  PaddedCounter error;            // set if a wait gave up (results of that launch invalid)
};

}  // namespace hm
