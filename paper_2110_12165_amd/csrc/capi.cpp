// C entry points of the lattice H-matrix library (include/hmat.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <atomic>
#include <cstdint>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hmat.h"
#include "hmat_internal.hpp"
#include "kernels.hpp"
#include "kernels_mm.hpp"
#include "layout.hpp"
#include "rs.hpp"
#include "rs_adjoint.hpp"
#include "rs_ens.hpp"

namespace {

thread_local std::string g_err;

hmat_status set_err(hmat_status c, const std::string& m) {
  g_err = m;
  return c;
}

void check_hip(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) hm::fail(HMAT_ENOMEM, std::string(what) + ": out of device memory");
  if (e != hipSuccess) hm::fail(HMAT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    check_hip(hipGetDevice(&prev), "hipGetDevice");
    if (prev != dev) check_hip(hipSetDevice(dev), "hipSetDevice");
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename F>
hmat_status guarded(F&& f) {
  try {
    f();
    g_err.clear();
    return HMAT_OK;
  } catch (const hm::Error& e) {
    return set_err(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_err(HMAT_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_err(HMAT_EINVAL, e.what());
  }
}

}  // namespace

// One captured stream sequence, replayed while its key (the pointers and
// constants it was captured with) stays the same.
struct GraphCache {
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;

  template <typename F>
  void ensure(const std::vector<const void*>& k, hipStream_t s, F&& enqueue) {
    if (exec && k == key) return;
    drop();
    check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      enqueue(s);
    } catch (...) {
      hipGraph_t tmp = nullptr;
      (void)hipStreamEndCapture(s, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      throw;
    }
    check_hip(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
    check_hip(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    key = k;
  }

  void drop() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (g) (void)hipGraphDestroy(g);
    exec = nullptr;
    g = nullptr;
    key.clear();
  }
};

void push_u64(std::vector<const void*>& key, uint64_t v) {
  key.push_back(reinterpret_cast<const void*>(static_cast<uintptr_t>(v)));
}

void push_double(std::vector<const void*>& key, double c) {
  const void* v;
  std::memcpy(&v, &c, sizeof(v));
  key.push_back(v);
}

// Identity of a handle for the graph caches of other handles: never reused
// within the process (a new handle may land at a freed handle's address).
std::atomic<uint64_t> g_next_uid{1};

struct hmat_s {
  int device = 0;
  bool on_device = false;  // false: host blocks only (hmat_build_host)
  const uint64_t uid = g_next_uid.fetch_add(1);
  // Bumped whenever the product's buffers or schedule change (drop_batched,
  // setup_batched, tune_mm, hmat_autotune): a graph captured with this
  // handle's kernels is valid only for the generation it was captured at.
  uint64_t gen = 0;
  hm::HostMatrix H;
  hmat_opts opts{};
  int32_t kernel = HMAT_KERNEL_BATCHED_SPLIT;  // resolved
  std::vector<void*> allocs;                  // everything except the batched set
  std::vector<void*> batched_allocs;
  int64_t bytes_fixed = 0, bytes_batched = 0;
  int32_t* d_perm = nullptr;
  hm::PlainArgs plain{};
  hm::BatchedArgs batched{};
  hm::BatchedArgs batched_t{};       // layout of H^T (hmat_matvec_T), if built
  bool has_plain = false, has_batched_t = false;
  int grid_t = 0;
  int grid = 0;
  int cus = 0;
  int32_t* d_invperm = nullptr;  // ensemble product: user element -> cluster position
  void* mm_xs = nullptr;         // ensemble product: bf16 [3][64][n]
  void* mm_ts = nullptr;         // ensemble product: bf16 [3][64][t_size]
  int64_t t_size = 0;
  int32_t max_nout_p1 = 0;
  int32_t* mm_slices1 = nullptr;  // ensemble product: 64-output slices of the phase-1 units
  int32_t mm_ns1 = 0;
  int32_t* mm_pairs = nullptr;    // ensemble product: pairs of phase-2 units sharing common inputs
  int32_t mm_npairs = 0;
  // ensemble product: wave groups per 64-output slice, [mode - BF16X3][phase - 1]
  int32_t mm_groups[2][2] = {{1, 1}, {1, 1}};
  double* rs_x = nullptr;  // n doubles: slip rate minus plate rate (rs_rhs scratch)
  double* rs_ax = nullptr;  // n doubles: A (V - V_pl)
  double* rs_bx = nullptr;  // n doubles: B (V - V_pl)
  hmat_stats st{};
  // side stream and fork/join events: this handle's product runs beside
  // another handle's in the same stage (with_pair)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // Creates them on the first call (never during a graph capture: the
  // entry points call this before they capture).
  void ensure_side() {
    if (side) return;
    check_hip(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming), "hipEventCreateWithFlags");
    check_hip(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming), "hipEventCreateWithFlags");
    check_hip(hipStreamCreateWithFlags(&side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  }
  // captured Runge-Kutta attempts (rs_rk45_run, rs_ens_rk45_run), each keyed
  // by everything it reads
  GraphCache rk_cache, rk_timed_cache, ens_cache;

  void drop_graph() {
    rk_cache.drop();
    rk_timed_cache.drop();
    ens_cache.drop();
  }

  ~hmat_s() {
    if (!on_device) return;
    (void)hipDeviceSynchronize();
    drop_graph();
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    for (void* p : batched_allocs) (void)hipFree(p);
    for (void* p : allocs) (void)hipFree(p);
  }

  template <typename V, typename Alloc>
  V* upload(const std::vector<V, Alloc>& v, hipStream_t s, bool batched_set = false) {
    const size_t bytes = std::max<size_t>(sizeof(V), v.size() * sizeof(V));
    void* p = nullptr;
    check_hip(hipMalloc(&p, bytes), "hipMalloc");
    (batched_set ? batched_allocs : allocs).push_back(p);
    (batched_set ? bytes_batched : bytes_fixed) += (int64_t)bytes;
    if (!v.empty()) check_hip(hipMemcpyAsync(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    return static_cast<V*>(p);
  }

  template <typename V>
  V* alloc_zero(size_t count, hipStream_t s, bool batched_set = false) {
    const size_t bytes = std::max<size_t>(sizeof(V), count * sizeof(V));
    void* p = nullptr;
    check_hip(hipMalloc(&p, bytes), "hipMalloc");
    (batched_set ? batched_allocs : allocs).push_back(p);
    (batched_set ? bytes_batched : bytes_fixed) += (int64_t)bytes;
    check_hip(hipMemsetAsync(p, 0, bytes, s), "hipMemsetAsync");
    return static_cast<V*>(p);
  }

  void drop_batched() {
    (void)hipDeviceSynchronize();
    ++gen;
    drop_graph();
    for (void* p : batched_allocs) (void)hipFree(p);
    batched_allocs.clear();
    bytes_batched = 0;
    batched = {};
    mm_ts = nullptr;
    mm_slices1 = nullptr;
    mm_ns1 = 0;
    mm_pairs = nullptr;
    mm_npairs = 0;
  }

  template <typename T>
  void setup_plain(bool transpose, hipStream_t s) {
    hm::PlainLayout<T> L = hm::make_plain<T>(H, transpose, opts.n_threads);
    plain.blocks = upload(L.blocks, s);
    plain.lr_list = upload(L.lr_list, s);
    plain.n_lr = (int32_t)L.lr_list.size();
    plain.rows = upload(L.row_units, s);
    plain.n_rows = (int32_t)L.row_units.size();
    plain.row_ents = upload(L.row_entries, s);
    plain.cols = upload(L.col_units, s);
    plain.n_cols = (int32_t)L.col_units.size();
    plain.col_ents = upload(L.col_entries, s);
    plain.pool = upload(L.pool, s);
    plain.perm = d_perm;
    plain.t = alloc_zero<double>((size_t)std::max<int64_t>(1, L.sum_rank), s);
    st.sum_rank = L.sum_rank;
    st.n_leaves = (int64_t)L.row_units.size();
    has_plain = true;
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  }

  // Batched layout of H^T, kept for the life of the handle (fixed set).
  template <typename T>
  void setup_batched_t(int32_t wg, int64_t unit_bytes, int32_t wg1, hipStream_t s) {
    hm::BatchedLayout<T> L = hm::make_batched<T>(H, wg, unit_bytes, wg1, true, opts.n_threads, split_slots<T>(wg1));
    batched_t.units = upload(L.units, s);
    batched_t.n1 = L.n1;
    batched_t.n2 = L.n2;
    batched_t.src = upload(L.src, s);
    batched_t.t = alloc_zero<double>((size_t)L.t_size, s);
    batched_t.tm = alloc_zero<double>((size_t)hm::kMultiMax * L.t_size, s);
    batched_t.sums = L.sums.empty() ? nullptr : upload(L.sums, s);
    batched_t.t_size = (int32_t)L.t_size;
    batched_t.pool = upload(L.pool, s);
    batched_t.perm = d_perm;
    batched_t.ctr = alloc_zero<hm::QueueCounters>(1, s);
    batched_t.wg_waves = wg;
    batched_t.wg_waves_p1 = wg1;
    grid_t = hm::persistent_blocks_per_cu<T>(wg) * cus;
    has_batched_t = true;
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  }

  // Row splitting of oversized phase-1 units (make_batched's split_slots):
  // -1 where phase 1 has few units per resident workgroup, 0 never, 1
  // wherever a unit is far above the mean.  Never for handles with ensemble
  // buffers: the ensemble product stages intermediate values split into bf16
  // parts and cannot add partial ones.
  int32_t split_mode = -1;
  template <typename T>
  int64_t split_slots(int32_t wg1) const {
    if (opts.max_nrhs > 0 || split_mode == 0) return 0;
    if (split_mode == 1) return INT32_MAX;
    return (int64_t)hm::phase1_blocks_per_cu<T>(wg1) * cus;
  }

  // Mean duration of `reps` products (after two untimed ones) on stream s.
  double time_product(hipStream_t s, int reps) {
    struct Ev {
      hipEvent_t e = nullptr;
      Ev() { check_hip(hipEventCreate(&e), "hipEventCreate"); }
      ~Ev() { (void)hipEventDestroy(e); }
    } e0, e1;
    for (int w = 0; w < 2; ++w) check_hip(product(false, rs_x, rs_ax, 1.0, 0.0, s, kernel), "product launch");
    check_hip(hipEventRecord(e0.e, s), "hipEventRecord");
    for (int r = 0; r < reps; ++r) check_hip(product(false, rs_x, rs_ax, 1.0, 0.0, s, kernel), "product launch");
    check_hip(hipEventRecord(e1.e, s), "hipEventRecord");
    check_hip(hipEventSynchronize(e1.e), "hipEventSynchronize");
    float ms = 0.f;
    check_hip(hipEventElapsedTime(&ms, e0.e, e1.e), "hipEventElapsedTime");
    return (double)ms / reps;
  }

  hm::MMArgs mm_args(const double* X, int64_t ldx, double* Y, int64_t ldy, int32_t nrhs, int32_t mode) const {
    hm::MMArgs a{};
    a.units = batched.units;
    a.n1 = batched.n1;
    a.n2 = batched.n2;
    a.slices1 = mm_slices1;
    a.ns1 = mm_ns1;
    a.cus = cus;
    a.groups1 = mm_groups[mode - HMAT_MM_BF16X3][0];
    a.groups2 = mm_groups[mode - HMAT_MM_BF16X3][1];
    a.pairs = mm_pairs;
    a.npairs = mm_npairs;
    a.src = batched.src;
    a.pool = batched.pool;
    a.perm = d_perm;
    a.invperm = d_invperm;
    a.n = H.n;
    a.t_size = t_size;
    a.Xs = mm_xs;
    a.Ts = mm_ts;
    a.X = X;
    a.ldx = ldx;
    a.Y = Y;
    a.ldy = ldy;
    a.nrhs = nrhs;
    return a;
  }

  template <typename T>
  void setup_batched(int32_t wg, int64_t unit_bytes, int32_t wg1, hipStream_t s) {
    // Row-split phase-1 units write partial intermediate values that the
    // ensemble product cannot add (it stages them split into bf16 parts):
    // handles with ensemble buffers keep whole units.
    hm::BatchedLayout<T> L =
        hm::make_batched<T>(H, wg, unit_bytes, wg1, false, opts.n_threads, split_slots<T>(wg1), opts.max_nrhs > 0);
    batched.units = upload(L.units, s, true);
    batched.n1 = L.n1;
    batched.n2 = L.n2;
    batched.src = upload(L.src, s, true);
    batched.t = alloc_zero<double>((size_t)L.t_size, s, true);
    batched.tm = alloc_zero<double>((size_t)hm::kMultiMax * L.t_size, s, true);
    batched.sums = L.sums.empty() ? nullptr : upload(L.sums, s, true);
    batched.t_size = (int32_t)L.t_size;
    batched.pool = upload(L.pool, s, true);
    batched.perm = d_perm;
    batched.ctr = alloc_zero<hm::QueueCounters>(1, s, true);
    batched.wg_waves = wg;
    batched.wg_waves_p1 = wg1;
    t_size = L.t_size;
    max_nout_p1 = 0;
    for (int32_t i = 0; i < L.n1; ++i) max_nout_p1 = std::max(max_nout_p1, L.units[i].nout);
    if (opts.max_nrhs > 0) {
      if (!L.sums.empty()) hm::fail(HMAT_EINVAL, "internal: ensemble layout with split units");
      if (opts.prec != HMAT_F32) hm::fail(HMAT_EUNSUPPORTED, "the ensemble product needs FP32 storage");
      if (max_nout_p1 > 1024) hm::fail(HMAT_EUNSUPPORTED, "the ensemble product needs wg_waves_p1 <= 16");
      mm_ts = alloc_zero<uint16_t>((size_t)3 * 64 * L.t_size, s, true);
      std::vector<int32_t> sl;
      for (int32_t i = 0; i < L.n1; ++i)
        for (int32_t k = 0; 64 * k < L.units[i].nout; ++k) sl.push_back(16 * i + k);
      mm_ns1 = (int32_t)sl.size();
      if (!sl.empty()) mm_slices1 = upload(sl, s, true);
      mm_npairs = (int32_t)(L.pairs.size() / 2);
      if (mm_npairs > 0) mm_pairs = upload(L.pairs, s, true);
    }
    grid = hm::persistent_blocks_per_cu<T>(wg) * cus;
    st.n_units_p1 = L.n1;
    st.n_units_p2 = L.n2;
    opts.wg_waves = wg;
    opts.wg_waves_p1 = wg1;
    opts.unit_kib = (int32_t)(unit_bytes / 1024);
    ++gen;
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  }

  bool f32() const { return opts.prec == HMAT_F32; }

  // The persistent schedule runs both phases in one launch: one wave count.
  void setup_batched_any(int32_t wg, int64_t unit_bytes, int32_t wg1, hipStream_t s) {
    if (kernel == HMAT_KERNEL_BATCHED_PERSISTENT || wg1 == 0) wg1 = wg;
    if (f32()) setup_batched<float>(wg, unit_bytes, wg1, s);
    else setup_batched<double>(wg, unit_bytes, wg1, s);
  }

  // nrhs vectors (column-major, leading dimension ld): with the split
  // schedule, passes of kMultiMax and then 2 vectors read each panel entry
  // once per pass; the rest (and the other schedules) one vector at a time.
  hipError_t products(bool transpose, const double* x, double* y, int64_t nrhs, int64_t ld, double alpha,
                      double beta, hipStream_t s, int32_t kern) const {
    int64_t c = 0;
    const bool multi = kern == HMAT_KERNEL_BATCHED_SPLIT && (!transpose || has_batched_t);
    if (multi) {
      const hm::BatchedArgs& a = transpose ? batched_t : batched;
      for (int nv : {hm::kMultiMax, 2})
        for (; c + nv <= nrhs; c += nv) {
          const hipError_t e = f32() ? hm::launch_batched_multi<float>(a, nv, x + c * ld, ld, y + c * ld, ld, alpha,
                                                                       beta, s)
                                     : hm::launch_batched_multi<double>(a, nv, x + c * ld, ld, y + c * ld, ld, alpha,
                                                                        beta, s);
          if (e != hipSuccess) return e;
        }
    }
    for (; c < nrhs; ++c) {
      const hipError_t e = product(transpose, x + c * ld, y + c * ld, alpha, beta, s, kern);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // transpose: H^T, through its batched layout when built, else the natural
  // layout's column units.
  hipError_t product(bool transpose, const double* x, double* y, double alpha, double beta, hipStream_t s,
                     int32_t kern, hipEvent_t* ev = nullptr) const {
    const bool pers = kern == HMAT_KERNEL_BATCHED_PERSISTENT;
    if (transpose && has_batched_t)
      return f32() ? hm::launch_batched<float>(batched_t, pers, grid_t, x, y, alpha, beta, s, ev)
                   : hm::launch_batched<double>(batched_t, pers, grid_t, x, y, alpha, beta, s, ev);
    if (transpose || kern == HMAT_KERNEL_PLAIN) {
      if (!has_plain || (transpose && plain.n_cols == 0)) return hipErrorInvalidValue;
      return f32() ? hm::launch_plain<float>(plain, transpose, x, y, alpha, beta, s, ev)
                   : hm::launch_plain<double>(plain, transpose, x, y, alpha, beta, s, ev);
    }
    return f32() ? hm::launch_batched<float>(batched, pers, grid, x, y, alpha, beta, s, ev)
                 : hm::launch_batched<double>(batched, pers, grid, x, y, alpha, beta, s, ev);
  }
};

namespace {

void check_opts(const hmat_opts& o, bool build) {
  if (build) {
    if (!(o.aca_eps > 0.0) || !std::isfinite(o.aca_eps)) hm::fail(HMAT_EINVAL, "aca_eps must be positive and finite");
    if (!(o.eta > 0.0) || !std::isfinite(o.eta)) hm::fail(HMAT_EINVAL, "eta must be positive and finite");
    if (o.leaf < 1) hm::fail(HMAT_EINVAL, "leaf must be >= 1");
    if (o.lattice < 1 || (o.lattice & (o.lattice - 1)) != 0) hm::fail(HMAT_EINVAL, "lattice must be a power of two");
    if (o.max_rank < 0) hm::fail(HMAT_EINVAL, "max_rank must be >= 0");
    if (o.n_threads < 0) hm::fail(HMAT_EINVAL, "n_threads must be >= 0");
  }
  if (o.prec != HMAT_F64 && o.prec != HMAT_F32) hm::fail(HMAT_EINVAL, "prec must be HMAT_F64 or HMAT_F32");
  if (o.kernel < HMAT_KERNEL_PLAIN || o.kernel > HMAT_KERNEL_AUTO) hm::fail(HMAT_EINVAL, "unknown kernel");
  if (o.wg_waves != 0 && o.wg_waves != 4 && o.wg_waves != 8 && o.wg_waves != 16)
    hm::fail(HMAT_EINVAL, "wg_waves must be 0, 4, 8 or 16");
  if (o.wg_waves_p1 != 0 && o.wg_waves_p1 != 4 && o.wg_waves_p1 != 8 && o.wg_waves_p1 != 16)
    hm::fail(HMAT_EINVAL, "wg_waves_p1 must be 0, 4, 8 or 16");
  if (o.unit_kib < 0) hm::fail(HMAT_EINVAL, "unit_kib must be >= 0");
  if (o.max_nrhs < 0) hm::fail(HMAT_EINVAL, "max_nrhs must be >= 0");
  if (o.transpose != 0 && o.transpose != 1) hm::fail(HMAT_EINVAL, "transpose must be 0 or 1");
  if (o.build_device != 0 && o.build_device != 1) hm::fail(HMAT_EINVAL, "build_device must be 0 or 1");
  if (o.mm_groups < 0 || o.mm_groups > 3) hm::fail(HMAT_EINVAL, "mm_groups must be 0, 1, 2 or 3");
}

// Default schedule of the batched product (fastest measured on MI355X for
// the planar benchmark fault; hmat_autotune can pick another).
constexpr int32_t kAutoKernel = HMAT_KERNEL_BATCHED_SPLIT;
constexpr int32_t kDefaultWaves = 8;
constexpr int32_t kDefaultWavesP1 = 4;
constexpr int32_t kSmallWavesP1 = 8;
constexpr int32_t kSmallP1UnitsPerCU = 8;
constexpr int kSmallTuneReps = 10;  // timed products per small-matrix layout candidate
constexpr int32_t kSmallWavesP2 = 4;
constexpr int32_t kDefaultUnitKiB = 256;
constexpr int kMMTuneReps = 5;  // timed ensemble products per mode and wave-group count

// Choices made by timing (the small-matrix layout at creation, the ensemble
// wave groups, hmat_autotune's schedule), remembered for the life of the
// process: a handle whose block list, storage, options and device model
// match one timed before takes the same choice without timing again.  The
// key is a 64-bit FNV-1a hash of all of these (a collision only costs a
// choice timed for another matrix: results stay correct either way).
enum TuneKind { kTuneSmallLayout = 1, kTuneMMGroups = 2, kTuneAutotune = 3 };

struct TuneCache {
  std::mutex mu;
  std::map<std::pair<uint64_t, int>, std::array<int32_t, 4>> picks;
};
TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t bytes) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

uint64_t tune_key(const hmat_s* h) {
  uint64_t k = 1469598103934665603ull;
  const hm::HostMatrix& H = h->H;
  k = fnv1a(k, &H.n, sizeof(H.n));
  k = fnv1a(k, H.desc.data(), H.desc.size() * sizeof(int64_t));
  k = fnv1a(k, H.perm.data(), H.perm.size() * sizeof(int32_t));
  const int32_t o[7] = {h->opts.prec, h->opts.wg_waves, h->opts.wg_waves_p1, h->opts.unit_kib,
                        h->opts.max_nrhs > 0, h->opts.mm_groups, h->opts.kernel};
  k = fnv1a(k, o, sizeof(o));
  hipDeviceProp_t prop{};
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) {
    k = fnv1a(k, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
    k = fnv1a(k, &prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
  }
  return k;
}

bool tune_lookup(uint64_t key, int kind, std::array<int32_t, 4>& out) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.picks.find({key, kind});
  if (it == c.picks.end()) return false;
  out = it->second;
  return true;
}

void tune_store(uint64_t key, int kind, const std::array<int32_t, 4>& v) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.picks[{key, kind}] = v;
}

// Wave groups of the ensemble product.  Two groups per slice halve the
// path of each workgroup and the workgroups resident per compute unit;
// which wins depends on the unit sizes and counts in a way no simple rule
// caught (measured, us per 64-member BF16x6 product, one / two groups in
// phase 2: N = 7680 85 / 69, N = 21000 193 / 200, N = 30720 178 / 156;
// phase 1, BF16x3: N = 21000 137 / 115, N = 122880 435 / 471).  Unless
// hmat_opts.mm_groups forces a value, this times kMMTuneReps products of each
// mode with one and with two groups, with events around each phase, and
// keeps per phase and mode the faster (fixed for the handle, so its
// products stay reproducible).  The timed products read zeros from a
// temporary buffer.
void tune_mm(hmat_s* h, hipStream_t s) {
  if (h->opts.mm_groups) {
    for (auto& m : h->mm_groups) {
      m[0] = h->opts.mm_groups == hm::kGroupsPairs ? 1 : h->opts.mm_groups;
      m[1] = h->opts.mm_groups;
    }
    ++h->gen;
    return;
  }
  // the groups depend on the layout the handle has now: its schedule joins the key
  const uint64_t key = fnv1a(tune_key(h), &h->batched.wg_waves, sizeof(int32_t)) ^
                       (uint64_t)(uint32_t)h->batched.wg_waves_p1 * 0x9e3779b97f4a7c15ull;
  std::array<int32_t, 4> hit{};
  if (tune_lookup(key, kTuneMMGroups, hit)) {
    h->mm_groups[0][0] = hit[0];
    h->mm_groups[0][1] = hit[1];
    h->mm_groups[1][0] = hit[2];
    h->mm_groups[1][1] = hit[3];
    ++h->gen;
    return;
  }
  struct Buf {
    void* p = nullptr;
    ~Buf() { (void)hipFree(p); }
  } bx, by;
  struct Ev {
    hipEvent_t e = nullptr;
    Ev() { check_hip(hipEventCreate(&e), "hipEventCreate"); }
    ~Ev() { (void)hipEventDestroy(e); }
  } e[3];
  const size_t bytes = (size_t)h->H.n * 64 * sizeof(double);
  check_hip(hipMalloc(&bx.p, bytes), "hipMalloc");
  check_hip(hipMalloc(&by.p, bytes), "hipMalloc");
  check_hip(hipMemsetAsync(bx.p, 0, bytes, s), "hipMemsetAsync");
  hipEvent_t ev[3] = {e[0].e, e[1].e, e[2].e};
  for (int m = 0; m < 2; ++m) {
    const int32_t mode = HMAT_MM_BF16X3 + m;
    double ms[3][2] = {};  // [choice][phase - 1]: one group, two groups, pairs (phase 2 only)
    const int nchoice = h->mm_npairs > 0 ? 3 : 2;
    for (int g = 0; g < nchoice; ++g) {
      h->mm_groups[m][0] = g == 2 ? 1 : g + 1;
      h->mm_groups[m][1] = g == 2 ? hm::kGroupsPairs : g + 1;
      const hm::MMArgs a = h->mm_args(static_cast<const double*>(bx.p), 64, static_cast<double*>(by.p), 64, 64, mode);
      for (int r = 0; r < 2 + kMMTuneReps; ++r) {
        check_hip(hm::launch_mm(a, mode, 1.0, 0.0, s, ev), "ensemble launch");
        check_hip(hipEventSynchronize(ev[2]), "hipEventSynchronize");
        if (r < 2) continue;  // untimed
        float t1 = 0.f, t2 = 0.f;
        check_hip(hipEventElapsedTime(&t1, ev[0], ev[1]), "hipEventElapsedTime");
        check_hip(hipEventElapsedTime(&t2, ev[1], ev[2]), "hipEventElapsedTime");
        ms[g][0] += t1;
        ms[g][1] += t2;
      }
    }
    h->mm_groups[m][0] = ms[1][0] < ms[0][0] ? 2 : 1;
    int best = 0;
    for (int g = 1; g < nchoice; ++g)
      if (ms[g][1] < ms[best][1]) best = g;
    h->mm_groups[m][1] = best == 2 ? hm::kGroupsPairs : best + 1;
  }
  tune_store(key, kTuneMMGroups, {h->mm_groups[0][0], h->mm_groups[0][1], h->mm_groups[1][0], h->mm_groups[1][1]});
  ++h->gen;
}

// The persistent schedule's wait for phase 1 is bounded: a workgroup that
// gives up (about 0.4 s of polling against a phase of ~0.1 ms; never seen)
// skips phase 2 and counts itself in the error counter, so that launch's
// results are invalid.  Calls that synchronise anyway (profile, autotune,
// the Runge-Kutta attempt, step and run) read the counter of the handles
// they used and fail instead of returning such results.
void check_wait_flag(hmat_t h, hipStream_t s) {
  if (!h || !h->on_device || h->kernel != HMAT_KERNEL_BATCHED_PERSISTENT) return;
  for (hm::QueueCounters* q : {h->batched.ctr, h->has_batched_t ? h->batched_t.ctr : nullptr}) {
    if (!q) continue;
    uint32_t e = 0;
    check_hip(hipMemcpyAsync(&e, &q->error.v, sizeof(e), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (e) {
      check_hip(hipMemsetAsync(&q->error.v, 0, sizeof(e), s), "hipMemsetAsync");
      hm::fail(HMAT_EDEVICE, "a persistent product gave up waiting for its phase 1; results since the last "
                             "check are invalid");
    }
  }
}

void fill_stats(hmat_s* h);

// The handles a captured attempt runs kernels of: identity, generation and
// schedule of A and of B (B's buffers are baked into A's graph; a B that
// was re-laid out or destroyed, even if a new handle took its address,
// no longer matches and the attempt is captured again).
void push_handle_key(std::vector<const void*>& key, hmat_t A, hmat_t B) {
  for (hmat_t h : {A, B}) {
    push_u64(key, h ? h->uid : 0);
    push_u64(key, h ? h->gen : 0);
    push_u64(key, h ? (uint64_t)h->kernel : 0);
  }
}

hmat_t create_handle(hm::HostMatrix&& H, const hmat_opts& o, hipStream_t s, bool on_device = true) {
  auto h = std::make_unique<hmat_s>();
  h->H = std::move(H);
  h->opts = o;
  h->kernel = o.kernel == HMAT_KERNEL_AUTO ? kAutoKernel : o.kernel;
  if (!on_device) {
    fill_stats(h.get());
    return h.release();
  }
  h->on_device = true;
  check_hip(hipGetDevice(&h->device), "hipGetDevice");
  int cus = 0;
  check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device), "hipDeviceGetAttribute");
  h->cus = std::max(1, cus);
  const int64_t n = h->H.n;
  h->d_perm = h->upload(h->H.perm, s);
  if (o.max_nrhs > 0) {
    if (h->kernel == HMAT_KERNEL_PLAIN) hm::fail(HMAT_EUNSUPPORTED, "the ensemble product needs a BATCHED kernel");
    std::vector<int32_t> inv(n);
    for (int64_t k = 0; k < n; ++k) inv[h->H.perm[k]] = (int32_t)k;
    h->d_invperm = h->upload(inv, s);
    h->mm_xs = h->alloc_zero<uint16_t>((size_t)3 * 64 * n, s);
  }
  h->rs_x = h->alloc_zero<double>((size_t)n, s);
  h->rs_ax = h->alloc_zero<double>((size_t)n, s);
  h->rs_bx = h->alloc_zero<double>((size_t)n, s);
  if (h->kernel == HMAT_KERNEL_PLAIN) {
    if (h->f32()) h->setup_plain<float>(o.transpose != 0, s);
    else h->setup_plain<double>(o.transpose != 0, s);
  } else {
    int32_t wg = o.wg_waves ? o.wg_waves : kDefaultWaves;
    int32_t wg1 = o.wg_waves_p1 ? o.wg_waves_p1 : kDefaultWavesP1;
    const int64_t ub = (int64_t)(o.unit_kib ? o.unit_kib : kDefaultUnitKiB) * 1024;
    h->setup_batched_any(wg, ub, wg1, s);
    // Small matrices: with fewer than kSmallP1UnitsPerCU phase-1 units per
    // compute unit the largest units run alone at the end of phase 1.  Two
    // remedies, each best on some matrices (measured, us per product):
    // splitting them by rows with four waves per unit (planar N = 21000:
    // 49.3, against 51.0 with eight waves; triangles B: 61.4 against 63.7)
    // or eight waves per unit, which shortens every unit (triangles A: 59.2
    // against 65.2); phase 2 with four waves per unit also wins on some
    // (planar N = 21000: 47.5 against 48.9) and loses on others (N = 7680:
    // 21.3 against 18.1).  The handle times a few products of each layout
    // and keeps the fastest (one choice per handle; its products stay
    // reproducible).
    if (!o.wg_waves_p1 && h->kernel == HMAT_KERNEL_BATCHED_SPLIT && h->batched.n1 < kSmallP1UnitsPerCU * h->cus) {
      struct Cand {
        int32_t wg, wg1, split;
      };
      std::vector<Cand> cands{{wg, kDefaultWavesP1, 1}, {wg, kSmallWavesP1, 0}, {wg, kSmallWavesP1, 1}};
      if (!o.wg_waves) cands.push_back({kSmallWavesP2, kDefaultWavesP1, 1});
      if (o.max_nrhs > 0) cands = {{wg, kDefaultWavesP1, 0}, {wg, kSmallWavesP1, 0}};
      double best = 1e300;
      Cand pick = cands[0], cur{wg, wg1, h->split_mode};
      const uint64_t key = tune_key(h.get());
      std::array<int32_t, 4> hit{};
      if (tune_lookup(key, kTuneSmallLayout, hit)) {
        pick = {hit[0], hit[1], hit[2]};
      } else {
        for (const Cand& c : cands) {
          h->drop_batched();
          h->split_mode = c.split;
          h->setup_batched_any(c.wg, ub, c.wg1, s);
          cur = c;
          const double ms = h->time_product(s, kSmallTuneReps);
          if (ms < best) {
            best = ms;
            pick = c;
          }
        }
        tune_store(key, kTuneSmallLayout, {pick.wg, pick.wg1, pick.split, 0});
      }
      if (pick.wg != cur.wg || pick.wg1 != cur.wg1 || pick.split != cur.split) {
        h->drop_batched();
        h->split_mode = pick.split;
        h->setup_batched_any(pick.wg, ub, pick.wg1, s);
      }
      wg = pick.wg;
      wg1 = pick.wg1;
    }
    if (h->mm_xs) tune_mm(h.get(), s);
    if (o.transpose) {
      const int32_t w1 = h->kernel == HMAT_KERNEL_BATCHED_PERSISTENT ? wg : wg1;
      if (h->f32()) h->setup_batched_t<float>(wg, ub, w1, s);
      else h->setup_batched_t<double>(wg, ub, w1, s);
    }
    // intermediate-vector length and row units of the product (statistics)
    int64_t sr = 0;
    for (int64_t b = 0; b < h->H.nblocks(); ++b) sr += h->H.desc[6 * b + 5];
    h->st.sum_rank = sr;
    h->st.n_leaves = (int64_t)hm::refine_ranges(h->H, false, 64).size();
  }
  fill_stats(h.get());
  return h.release();
}

void fill_stats(hmat_s* h) {
  const int64_t n = h->H.n;
  hmat_stats& st = h->st;
  const int64_t keep_sum_rank = st.sum_rank, keep_leaves = st.n_leaves, keep_u1 = st.n_units_p1,
                keep_u2 = st.n_units_p2;
  st = hmat_stats{};
  st.sum_rank = keep_sum_rank;
  st.n_leaves = keep_leaves;
  st.n_units_p1 = keep_u1;
  st.n_units_p2 = keep_u2;
  st.n = n;
  const int64_t sz = h->f32() ? 4 : 8;
  for (int64_t b = 0; b < h->H.nblocks(); ++b) {
    const int64_t* d = &h->H.desc[6 * b];
    if (d[0] == 0) {
      ++st.n_dense;
      st.dense_entries += d[2] * d[4];
    } else {
      ++st.n_lr;
      st.lr_entries += d[5] * (d[2] + d[4]);
      st.max_rank = std::max(st.max_rank, d[5]);
    }
  }
  st.tree_depth = h->H.tree_depth;
  st.factor_bytes = sz * (st.dense_entries + st.lr_entries);
  st.alg_bytes = st.factor_bytes + 8 * n + 16 * n + 4 * n;
  st.prec = h->opts.prec;
  st.lattice = h->H.lattice;
}

void refresh_stats(hmat_s* h) {
  h->st.device_bytes = h->bytes_fixed + h->bytes_batched;
  h->st.kernel = h->kernel;
  h->st.wg_waves = h->kernel == HMAT_KERNEL_PLAIN ? 0 : h->opts.wg_waves;
  h->st.wg_waves_p1 = h->kernel == HMAT_KERNEL_PLAIN ? 0 : h->opts.wg_waves_p1;
  h->st.mm_groups = 0;
  if (h->mm_xs)
    for (int m = 0; m < 2; ++m)
      for (int p = 0; p < 2; ++p) h->st.mm_groups |= h->mm_groups[m][p] << (4 * (2 * m + p));
}

void check_vectors(hmat_t h, const double* x, const double* y, int64_t nrhs, int64_t ld) {
  if (!h) hm::fail(HMAT_EINVAL, "null handle");
  if (!h->on_device) hm::fail(HMAT_ESTATE, "handle holds host blocks only (hmat_build_host)");
  if (nrhs < 0) hm::fail(HMAT_EINVAL, "nrhs must be >= 0");
  if (nrhs == 0) return;
  if (!x || !y) hm::fail(HMAT_EINVAL, "x and y must be non-null");
  if (ld < h->H.n) hm::fail(HMAT_EINVAL, "ld must be >= n");
  const char* xa = reinterpret_cast<const char*>(x);
  const char* ya = reinterpret_cast<const char*>(y);
  const int64_t span = ((nrhs - 1) * ld + h->H.n) * (int64_t)sizeof(double);
  if (xa < ya + span && ya < xa + span) hm::fail(HMAT_EINVAL, "x and y must not overlap");
}

}  // namespace

extern "C" {

void hmat_default_opts(hmat_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->aca_eps = 1e-6;
  o->eta = 2.0;
  o->leaf = 32;
  o->lattice = 1;
  o->max_rank = 0;
  o->prec = HMAT_F64;
  o->kernel = HMAT_KERNEL_AUTO;
  o->transpose = 1;
}

hmat_status hmat_build(const hmat_mesh* mesh, const hmat_green* green, const hmat_opts* opts, void* stream,
                       hmat_t* out) {
  return guarded([&] {
    if (!mesh || !green || !opts || !out) hm::fail(HMAT_EINVAL, "null argument");
    check_opts(*opts, true);
    hm::Geometry geo;
    std::unique_ptr<hm::EntryFn> E(hm::make_entry_fn(*mesh, *green, geo));
    hm::ClusterTree tree = hm::build_tree(geo, opts->leaf);
    std::vector<hm::BlockSpec> blocks = hm::partition(tree, opts->lattice, opts->eta);
    hm::HostMatrix H =
        opts->build_device
            ? hm::assemble_device(*E, tree, blocks, opts->aca_eps, opts->max_rank, opts->n_threads, stream)
            : hm::assemble(*E, tree, blocks, opts->aca_eps, opts->max_rank, opts->n_threads);
    H.lattice = opts->lattice;
    hmat_t h = create_handle(std::move(H), *opts, static_cast<hipStream_t>(stream));
    refresh_stats(h);
    *out = h;
  });
}

hmat_status hmat_build_host(const hmat_mesh* mesh, const hmat_green* green, const hmat_opts* opts, hmat_t* out) {
  return guarded([&] {
    if (!mesh || !green || !opts || !out) hm::fail(HMAT_EINVAL, "null argument");
    check_opts(*opts, true);
    hm::Geometry geo;
    std::unique_ptr<hm::EntryFn> E(hm::make_entry_fn(*mesh, *green, geo));
    hm::ClusterTree tree = hm::build_tree(geo, opts->leaf);
    std::vector<hm::BlockSpec> blocks = hm::partition(tree, opts->lattice, opts->eta);
    hm::HostMatrix H = hm::assemble(*E, tree, blocks, opts->aca_eps, opts->max_rank, opts->n_threads);
    H.lattice = opts->lattice;
    hmat_t h = create_handle(std::move(H), *opts, nullptr, false);
    refresh_stats(h);
    *out = h;
  });
}

hmat_status hmat_import(const hmat_host_blocks* b, const hmat_opts* opts, void* stream, hmat_t* out) {
  return guarded([&] {
    if (!b || !opts || !out) hm::fail(HMAT_EINVAL, "null argument");
    check_opts(*opts, false);
    if (b->n < 1 || b->nblocks < 1 || b->nvalues < 0) hm::fail(HMAT_EINVAL, "bad sizes");
    if (!b->perm || !b->desc || !b->off || (b->nvalues > 0 && !b->values)) hm::fail(HMAT_EINVAL, "null array");
    if (b->n > (int64_t)INT32_MAX / 2) hm::fail(HMAT_EINVAL, "n too large");
    hm::HostMatrix H;
    H.n = b->n;
    H.perm.assign(b->perm, b->perm + b->n);
    H.desc.assign(b->desc, b->desc + 6 * b->nblocks);
    H.off.assign(b->off, b->off + b->nblocks);
    H.values.assign(b->values, b->values + b->nvalues);
    hm::validate_host_matrix(H);
    H.lattice = 0;
    H.tree_depth = 0;
    hmat_t h = create_handle(std::move(H), *opts, static_cast<hipStream_t>(stream));
    refresh_stats(h);
    *out = h;
  });
}

hmat_status hmat_export(hmat_t h, hmat_host_blocks* out) {
  return guarded([&] {
    if (!h || !out) hm::fail(HMAT_EINVAL, "null argument");
    out->n = h->H.n;
    out->nblocks = h->H.nblocks();
    out->nvalues = (int64_t)h->H.values.size();
    out->perm = h->H.perm.data();
    out->desc = h->H.desc.data();
    out->off = h->H.off.data();
    out->values = h->H.values.data();
  });
}

hmat_status hmat_matvec(hmat_t h, const double* x, double* y, int64_t nrhs, int64_t ld, double alpha, double beta,
                        void* stream) {
  return guarded([&] {
    check_vectors(h, x, y, nrhs, ld);
    if (nrhs == 0) return;
    DeviceGuard g(h->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    check_hip(h->products(false, x, y, nrhs, ld, alpha, beta, s, h->kernel), "product launch");
  });
}

hmat_status hmat_matvec_T(hmat_t h, const double* x, double* y, int64_t nrhs, int64_t ld, double alpha, double beta,
                          void* stream) {
  return guarded([&] {
    check_vectors(h, x, y, nrhs, ld);
    if (nrhs == 0) return;
    DeviceGuard g(h->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (!h->has_batched_t && !(h->has_plain && h->plain.n_cols > 0))
      hm::fail(HMAT_ESTATE, "handle created without opts.transpose");
    const int32_t kt = h->kernel == HMAT_KERNEL_PLAIN ? HMAT_KERNEL_PLAIN : h->kernel;
    check_hip(h->products(true, x, y, nrhs, ld, alpha, beta, s, kt), "transpose launch");
  });
}

namespace {

// Ensemble product of up to 64 right-hand sides (X, Y element-major).
void enqueue_mm(hmat_t h, const double* X, int64_t ldx, double* Y, int64_t ldy, int32_t nrhs, double alpha,
                double beta, int32_t mode, hipStream_t s) {
  const hm::MMArgs a = h->mm_args(X, ldx, Y, ldy, nrhs, mode);
  check_hip(hm::launch_mm(a, mode, alpha, beta, s), "ensemble launch");
}

}  // namespace

hmat_status hmat_matmat(hmat_t h, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t nrhs, double alpha,
                        double beta, int32_t mode, void* stream) {
  return guarded([&] {
    if (!h) hm::fail(HMAT_EINVAL, "null handle");
    if (!h->on_device) hm::fail(HMAT_ESTATE, "handle holds host blocks only (hmat_build_host)");
    if (nrhs < 0) hm::fail(HMAT_EINVAL, "nrhs must be >= 0");
    if (nrhs == 0) return;
    if (!h->mm_xs || !h->mm_ts) hm::fail(HMAT_ESTATE, "handle created without max_nrhs");
    if (mode != HMAT_MM_BF16X3 && mode != HMAT_MM_BF16X6) hm::fail(HMAT_EINVAL, "unknown mode");
    if (!X || !Y) hm::fail(HMAT_EINVAL, "X and Y must be non-null");
    if (ldx < nrhs || ldy < nrhs) hm::fail(HMAT_EINVAL, "ldx and ldy must be >= nrhs");
    const int64_t n = h->H.n;
    const char* xa = reinterpret_cast<const char*>(X);
    const char* ya = reinterpret_cast<const char*>(Y);
    const int64_t sx = ((n - 1) * ldx + nrhs) * 8, sy = ((n - 1) * ldy + nrhs) * 8;
    if (xa < ya + sy && ya < xa + sx) hm::fail(HMAT_EINVAL, "X and Y must not overlap");
    DeviceGuard g(h->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    for (int64_t c0 = 0; c0 < nrhs; c0 += 64)
      enqueue_mm(h, X + c0, ldx, Y + c0, ldy, (int32_t)std::min<int64_t>(64, nrhs - c0), alpha, beta, mode, s);
  });
}

hmat_status hmat_info(hmat_t h, hmat_stats* out) {
  return guarded([&] {
    if (!h || !out) hm::fail(HMAT_EINVAL, "null argument");
    refresh_stats(h);
    *out = h->st;
  });
}

hmat_status hmat_autotune(hmat_t h, int32_t reps, void* stream) {
  return guarded([&] {
    if (!h) hm::fail(HMAT_EINVAL, "null handle");
    if (!h->on_device) hm::fail(HMAT_ESTATE, "handle holds host blocks only (hmat_build_host)");
    if (reps < 1) hm::fail(HMAT_EINVAL, "reps must be >= 1");
    DeviceGuard g(h->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = h->H.n;
    double *x = nullptr, *y = nullptr;
    check_hip(hipMalloc(&x, n * sizeof(double)), "hipMalloc");
    struct Free { void* p; ~Free() { (void)hipFree(p); } } fx{x};
    check_hip(hipMalloc(&y, n * sizeof(double)), "hipMalloc");
    Free fy{y};
    std::vector<double> ones(n, 1e-9);
    check_hip(hipMemcpy(x, ones.data(), n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
    struct Ev {
      hipEvent_t e = nullptr;
      Ev() { check_hip(hipEventCreate(&e), "hipEventCreate"); }
      ~Ev() { (void)hipEventDestroy(e); }
    } ev0, ev1;
    const hipEvent_t e0 = ev0.e, e1 = ev1.e;
    auto time_it = [&](int32_t kern) {
      for (int w = 0; w < 2; ++w) check_hip(h->product(false, x, y, 1.0, 0.0, s, kern), "product launch");
      check_hip(hipEventRecord(e0, s), "hipEventRecord");
      for (int r = 0; r < reps; ++r) check_hip(h->product(false, x, y, 1.0, 0.0, s, kern), "product launch");
      check_hip(hipEventRecord(e1, s), "hipEventRecord");
      check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      return (double)ms / reps;
    };
    int32_t best_k = h->has_plain ? HMAT_KERNEL_PLAIN : h->kernel, best_w = h->opts.wg_waves,
            best_u = kDefaultUnitKiB;
    int32_t best_w1 = h->opts.wg_waves_p1;
    const int32_t saved_kernel = h->kernel;
    const uint64_t key = tune_key(h) ^ (uint64_t)h->has_plain;
    std::array<int32_t, 4> hit{};
    if (tune_lookup(key, kTuneAutotune, hit)) {
      best_k = hit[0];
      best_w = hit[1];
      best_w1 = hit[2];
    } else {
      double best = h->has_plain ? time_it(HMAT_KERNEL_PLAIN) : 1e300;
      for (int32_t k : {HMAT_KERNEL_BATCHED_SPLIT, HMAT_KERNEL_BATCHED_PERSISTENT})
        for (int32_t wg : {4, 8, 16})
          for (int32_t wg1 : {4, 8, 16}) {
            if (k == HMAT_KERNEL_BATCHED_PERSISTENT && wg1 != wg) continue;
            h->drop_batched();
            h->kernel = k;
            h->setup_batched_any(wg, (int64_t)kDefaultUnitKiB * 1024, wg1, s);
            const double t = time_it(k);
            if (t < best) {
              best = t;
              best_k = k;
              best_w = wg;
              best_w1 = wg1;
              best_u = kDefaultUnitKiB;
            }
          }
      tune_store(key, kTuneAutotune, {best_k, best_w, best_w1, 0});
    }
    h->kernel = saved_kernel;
    h->drop_batched();
    h->kernel = best_k;
    if (best_k != HMAT_KERNEL_PLAIN) h->setup_batched_any(best_w, (int64_t)best_u * 1024, best_w1, s);
    if (best_k != HMAT_KERNEL_PLAIN && h->mm_xs) tune_mm(h, s);
    ++h->gen;
    h->drop_graph();
    refresh_stats(h);
  });
}

hmat_status hmat_profile(hmat_t h, const double* x, double* y, int32_t reps, void* stream, hmat_profile_t* out) {
  return guarded([&] {
    check_vectors(h, x, y, 1, h ? h->H.n : 0);
    if (!out) hm::fail(HMAT_EINVAL, "null output");
    if (reps < 1) hm::fail(HMAT_EINVAL, "reps must be >= 1");
    DeviceGuard g(h->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const bool pers = h->kernel == HMAT_KERNEL_BATCHED_PERSISTENT;
    const int nl = pers ? 1 : 2;
    std::vector<hipEvent_t> ev(3 * (size_t)reps, nullptr);
    struct Destroy {
      std::vector<hipEvent_t>& e;
      ~Destroy() { for (auto v : e) if (v) (void)hipEventDestroy(v); }
    } destroy{ev};
    for (auto& e : ev) check_hip(hipEventCreate(&e), "hipEventCreate");
    check_hip(h->product(false, x, y, 1.0, 0.0, s, h->kernel), "product launch");  // warm-up
    for (int r = 0; r < reps; ++r) check_hip(h->product(false, x, y, 1.0, 0.0, s, h->kernel, &ev[3 * r]), "product launch");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    double sum[2] = {0.0, 0.0}, tot = 0.0;
    for (int r = 0; r < reps; ++r) {
      float a = 0.f, b = 0.f;
      check_hip(hipEventElapsedTime(&a, ev[3 * r], ev[3 * r + 1]), "hipEventElapsedTime");
      sum[0] += a;
      if (nl == 2) {
        check_hip(hipEventElapsedTime(&b, ev[3 * r + 1], ev[3 * r + 2]), "hipEventElapsedTime");
        sum[1] += b;
      }
      tot += (double)a + (double)b;
    }
    const hmat_stats& st = h->st;
    const int64_t n = st.n, sz = h->f32() ? 4 : 8;
    // algorithmic bytes of each launch: its factors plus the vectors it must touch
    int64_t lr_cols = 0, lr_rows = 0;  // sum r*n and sum r*m over low-rank blocks
    for (int64_t b = 0; b < h->H.nblocks(); ++b) {
      const int64_t* d = &h->H.desc[6 * b];
      if (d[0] == 1) { lr_cols += d[5] * d[4]; lr_rows += d[5] * d[2]; }
    }
    const int64_t p1 = sz * lr_cols + 12 * n + 8 * st.sum_rank;
    const int64_t p2 = sz * (st.dense_entries + lr_rows) + 8 * st.sum_rank + 28 * n;
    out->n_launches = nl;
    out->reps = reps;
    out->ms[0] = sum[0] / reps;
    out->ms[1] = nl == 2 ? sum[1] / reps : 0.0;
    out->ms_product = tot / reps;
    out->alg_bytes[0] = nl == 2 ? p1 : st.alg_bytes;
    out->alg_bytes[1] = nl == 2 ? p2 : 0;
    check_wait_flag(h, s);
  });
}

hmat_status rs_rhs(hmat_t A, hmat_t B, const rs_params* p, const double* y, double* dydt, double* V_out,
                   void* stream) {
  return guarded([&] {
    if (!A || !p || !y || !dydt) hm::fail(HMAT_EINVAL, "null argument");
    if (!A->on_device || (B && !B->on_device)) hm::fail(HMAT_ESTATE, "handle holds host blocks only");
    if (B && B->device != A->device) hm::fail(HMAT_EINVAL, "A and B live on different devices");
    if (p->n != A->H.n || (B && B->H.n != A->H.n)) hm::fail(HMAT_EINVAL, "n does not match the handles");
    if (!p->a || !p->b || !p->dc) hm::fail(HMAT_EINVAL, "null friction parameter array");
    if (!(p->V0 > 0.0) || !(p->eta_rad >= 0.0) || !std::isfinite(p->f0) || !std::isfinite(p->V_pl))
      hm::fail(HMAT_EINVAL, "bad friction constants");
    DeviceGuard g(A->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = A->H.n;
    // 1) V from eq. (7) and x = V - V_pl
    check_hip(hm::launch_rs_slip_rate(n, p->V0, p->V_pl, p->a, y, A->rs_x, V_out, s), "slip-rate launch");
    // 2) A x (and B x), eqs. (9)-(10) with the backslip loading of eqs. (21)-(22)
    check_hip(A->product(false, A->rs_x, A->rs_ax, 1.0, 0.0, s, A->kernel), "product launch");
    const double* bx = nullptr;
    if (B) {
      check_hip(B->product(false, A->rs_x, A->rs_bx, 1.0, 0.0, s, B->kernel), "product launch");
      bx = A->rs_bx;
    }
    // 3) element-wise right-hand side, eqs. (8), (12), (13)
    check_hip(hm::launch_rs_rhs(n, *p, y, A->rs_ax, bx, dydt, s), "rhs launch");
  });
}

int64_t rs_rk45_workspace_bytes(int64_t n) { return n < 0 ? -1 : 8 * (28 * n + hm::kRkStateDoubles); }

namespace {

struct RkWs {
  double *k, *ys, *y5, *Vs, *xv, *ax, *bx;
  hm::RkDevState* st;
};

RkWs rk_workspace(void* workspace, int64_t n) {
  RkWs w;
  double* base = static_cast<double*>(workspace);
  w.k = base;
  w.ys = w.k + 18 * n;
  w.y5 = w.ys + 3 * n;
  w.Vs = w.y5 + 3 * n;
  w.xv = w.Vs + n;
  w.ax = w.xv + n;
  w.bx = w.ax + n;
  w.st = reinterpret_cast<hm::RkDevState*>(w.bx + n);
  return w;
}

void check_rk_args(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                   const rs_rk45_state* st) {
  static_assert(sizeof(hm::RkDevState) <= hm::kRkStateDoubles * sizeof(double), "device state must fit the workspace tail");
  if (!A || !p || !y || !D || !workspace || !st) hm::fail(HMAT_EINVAL, "null argument");
  if (!A->on_device || (B && !B->on_device)) hm::fail(HMAT_ESTATE, "handle holds host blocks only");
  if (p->n != A->H.n || (B && B->H.n != A->H.n)) hm::fail(HMAT_EINVAL, "n does not match the handles");
  if (B && B->device != A->device) hm::fail(HMAT_EINVAL, "A and B live on different devices");
  if (!p->a || !p->b || !p->dc) hm::fail(HMAT_EINVAL, "null friction parameter array");
  if (!(p->V0 > 0.0) || !(p->eta_rad >= 0.0) || !std::isfinite(p->f0) || !std::isfinite(p->V_pl))
    hm::fail(HMAT_EINVAL, "bad friction constants");
  if (!(st->dt > 0.0) || !std::isfinite(st->dt)) hm::fail(HMAT_EINVAL, "dt must be positive and finite");
  if (reinterpret_cast<uintptr_t>(workspace) % 8) hm::fail(HMAT_EINVAL, "workspace must be 8-byte aligned");
}

// The products with A and with B of one stage: fa(s), and fb on B's side
// stream, forked from s and joined back before anything later on s.  On
// small matrices each product is a few short launches whose ramp and tail
// leave most of the GPU idle, and the two overlap (under graph capture the
// fork and the join become dependencies of the graph).  Each handle has
// its own scratch, so the two are independent and their results do not
// depend on the overlap; A == B (shared scratch) runs both on s.
extern "C++" template <class FA, class FB>
void with_pair(hmat_t A, hmat_t B, hipStream_t s, FA&& fa, FB&& fb) {
  if (!B) {
    fa(s);
    return;
  }
  if (B == A) {
    fa(s);
    fb(s);
    return;
  }
  if (!B->side) {
    // first pair of this handle: no stream is created while the caller
    // captures s into a graph of its own (both products then go on s)
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;  // the null stream is never captured
    if (s) check_hip(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) {
      fa(s);
      fb(s);
      return;
    }
    B->ensure_side();
  }
  check_hip(hipEventRecord(B->ev_fork, s), "hipEventRecord");
  check_hip(hipStreamWaitEvent(B->side, B->ev_fork, 0), "hipStreamWaitEvent");
  fb(B->side);
  check_hip(hipEventRecord(B->ev_join, B->side), "hipEventRecord");
  fa(s);
  check_hip(hipStreamWaitEvent(s, B->ev_join, 0), "hipStreamWaitEvent");
}

// Enqueue one attempt: every kernel reads the step from the device state.
void enqueue_attempt(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, const RkWs& w, double* dt_log,
                     hipStream_t s, bool timed = false) {
  const int64_t n = A->H.n, n3 = 3 * n;
  if (timed) check_hip(hm::launch_rk_stamp(w.st, 0, s), "stamp launch");
  check_hip(hm::launch_rk_begin(w.st, s), "rk begin launch");
  for (int stage = 0; stage < 6; ++stage) {
    const double* yin = y;
    if (stage > 0) {
      check_hip(hm::launch_rk_stage_slip(n, stage, w.st, 0.0, y, w.k, w.ys, p->V0, p->V_pl, p->a, w.xv, s),
                "stage launch");
      yin = w.ys;
    } else {
      check_hip(hm::launch_rs_slip_rate(n, p->V0, p->V_pl, p->a, y, w.xv, w.Vs, s), "slip-rate launch");
    }
    if (timed) check_hip(hm::launch_rk_stamp(w.st, 1, s), "stamp launch");
    with_pair(
        A, B, s, [&](hipStream_t q) { check_hip(A->product(false, w.xv, w.ax, 1.0, 0.0, q, A->kernel), "product launch"); },
        [&](hipStream_t q) { check_hip(B->product(false, w.xv, w.bx, 1.0, 0.0, q, B->kernel), "product launch"); });
    if (timed) check_hip(hm::launch_rk_stamp(w.st, 2, s), "stamp launch");
    check_hip(hm::launch_rs_rhs(n, *p, yin, w.ax, B ? w.bx : nullptr, w.k + stage * n3, s), "rhs launch");
  }
  check_hip(hm::launch_rk_finish_control(n3, w.st, y, w.k, w.y5, s), "error launch");
  check_hip(hm::launch_rk_accept(n, w.st, p->V0, p->a, w.y5, w.Vs, y, D, dt_log, s), "accept launch");
  if (timed) check_hip(hm::launch_rk_stamp(w.st, 3, s), "stamp launch");
}

void put_state(const RkWs& w, const rs_rk45_state* st, long long target, int force, hipStream_t s) {
  hm::RkDevState d{};
  d.t = st->t;
  d.dt = st->dt;
  d.eps = st->eps_rk > 0.0 ? st->eps_rk : 1e-4;
  d.accepted = st->accepted;
  d.rejected = st->rejected;
  d.target = target;
  d.force = force;
  d.log_base = st->accepted;
  check_hip(hipMemcpyAsync(w.st, &d, sizeof(d), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

void get_state(const RkWs& w, rs_rk45_state* st, hipStream_t s) {
  hm::RkDevState d{};
  check_hip(hipMemcpyAsync(&d, w.st, sizeof(d), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  st->t = d.t;
  st->dt = d.dt;
  st->last_err = d.r;
  st->accepted = d.accepted;
  st->rejected = d.rejected;
}

}  // namespace

hmat_status rs_rk45_attempt(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                            rs_rk45_state* st, int32_t force, void* stream) {
  return guarded([&] {
    check_rk_args(A, B, p, y, D, workspace, st);
    if (force < -1 || force > 1) hm::fail(HMAT_EINVAL, "force must be -1, 0 or 1");
    DeviceGuard g(A->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const RkWs w = rk_workspace(workspace, A->H.n);
    put_state(w, st, st->accepted + 1, force, s);
    enqueue_attempt(A, B, p, y, D, w, nullptr, s);
    get_state(w, st, s);
    check_wait_flag(A, s);
    if (B != A) check_wait_flag(B, s);
  });
}

namespace {

// rs_rk45_run, and with `timing` its timed form (stamps in every attempt;
// the totals are read back into *timing).
void run_rk(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace, rs_rk45_state* st,
            int64_t n_accept, int64_t max_attempts, double* dt_log, int32_t use_graph, void* stream,
            rs_rk45_timing* timing) {
  check_rk_args(A, B, p, y, D, workspace, st);
  if (n_accept < 0 || max_attempts < 0) hm::fail(HMAT_EINVAL, "counts must be >= 0");
  if (n_accept == 0) return;
  DeviceGuard g(A->device);
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const RkWs w = rk_workspace(workspace, A->H.n);
  const long long target = st->accepted + n_accept;
  put_state(w, st, target, -1, s);
  const bool timed = timing != nullptr;
  const bool graph = use_graph && s != nullptr;
  GraphCache& cache = timed ? A->rk_timed_cache : A->rk_cache;
  if (B && B != A) B->ensure_side();  // not during the capture
  if (graph) {
    std::vector<const void*> key{p->a, p->b, p->dc, y, D, workspace, dt_log, s};
    for (double c : {p->V0, p->f0, p->eta_rad, p->V_pl}) push_double(key, c);
    push_handle_key(key, A, B);
    cache.ensure(key, s, [&](hipStream_t cs) { enqueue_attempt(A, B, p, y, D, w, dt_log, cs, timed); });
  }
  int64_t launched = 0;
  for (;;) {
    int64_t batch = target - st->accepted;
    if (max_attempts > 0) batch = std::min(batch, max_attempts - launched);
    if (batch <= 0) break;
    for (int64_t k = 0; k < batch; ++k) {
      if (graph) check_hip(hipGraphLaunch(cache.exec, s), "hipGraphLaunch");
      else enqueue_attempt(A, B, p, y, D, w, dt_log, s, timed);
    }
    launched += batch;
    get_state(w, st, s);
    if (st->accepted >= target) break;
  }
  check_wait_flag(A, s);
  if (B != A) check_wait_flag(B, s);
  if (timed) {
    hm::RkDevState d{};
    check_hip(hipMemcpyAsync(&d, w.st, sizeof(d), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    int rate_khz = 0;
    check_hip(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, A->device), "hipDeviceGetAttribute");
    if (rate_khz <= 0) hm::fail(HMAT_EDEVICE, "device reports no wall-clock rate");
    timing->product_ms = (double)d.prof_prod / rate_khz;
    timing->attempt_ms = (double)d.prof_att / rate_khz;
    timing->attempts = launched;
  }
  if (st->accepted < target) hm::fail(HMAT_ESTATE, "target not reached within max_attempts");
}

}  // namespace

hmat_status rs_rk45_run(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                        rs_rk45_state* st, int64_t n_accept, int64_t max_attempts, double* dt_log, int32_t use_graph,
                        void* stream) {
  return guarded([&] {
    run_rk(A, B, p, y, D, workspace, st, n_accept, max_attempts, dt_log, use_graph, stream, nullptr);
  });
}

hmat_status rs_rk45_run_timed(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                              rs_rk45_state* st, int64_t n_accept, int64_t max_attempts, double* dt_log,
                              int32_t use_graph, void* stream, rs_rk45_timing* timing) {
  return guarded([&] {
    if (!timing) hm::fail(HMAT_EINVAL, "null timing output");
    *timing = rs_rk45_timing{};
    run_rk(A, B, p, y, D, workspace, st, n_accept, max_attempts, dt_log, use_graph, stream, timing);
  });
}

hmat_status rs_rk45_step(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, void* workspace,
                         rs_rk45_state* st, int32_t max_attempts, void* stream) {
  if (max_attempts < 1) return set_err(HMAT_EINVAL, "max_attempts must be >= 1");
  return rs_rk45_run(A, B, p, y, D, workspace, st, 1, max_attempts, nullptr, 0, stream);
}

namespace {

void check_replay_args(hmat_t A, hmat_t B, const rs_params* p, const double* dts, int64_t n_steps,
                       int64_t ckpt_every) {
  if (!A || !p) hm::fail(HMAT_EINVAL, "null argument");
  if (!A->on_device || (B && !B->on_device)) hm::fail(HMAT_ESTATE, "handle holds host blocks only");
  if (p->n != A->H.n || (B && B->H.n != A->H.n)) hm::fail(HMAT_EINVAL, "n does not match the handles");
  if (B && B->device != A->device) hm::fail(HMAT_EINVAL, "A and B live on different devices");
  if (!p->a || !p->b || !p->dc) hm::fail(HMAT_EINVAL, "null friction parameter array");
  if (!(p->V0 > 0.0) || !(p->eta_rad >= 0.0) || !std::isfinite(p->f0) || !std::isfinite(p->V_pl))
    hm::fail(HMAT_EINVAL, "bad friction constants");
  if (n_steps < 0) hm::fail(HMAT_EINVAL, "n_steps must be >= 0");
  if (ckpt_every < 1) hm::fail(HMAT_EINVAL, "ckpt_every must be >= 1");
  if (n_steps > 0 && !dts) hm::fail(HMAT_EINVAL, "null step list");
  for (int64_t m = 0; m < n_steps; ++m)
    if (!(dts[m] > 0.0) || !std::isfinite(dts[m])) hm::fail(HMAT_EINVAL, "steps must be positive and finite");
}

// One step of the frozen-step integration from y_in to y_out (may alias):
// the six stages write their derivatives to K (6 blocks of 3n) and, when
// Ystore is given, their inputs for stages 1..5 to Ystore (5 blocks of 3n);
// otherwise the stage input goes to ys.  x, ax, bx: n-vectors.
void enqueue_frozen_step(hmat_t A, hmat_t B, const rs_params* p, const double* y_in, double* y_out, double* D,
                         double dt, double* K, double* Ystore, double* ys, double* x, double* ax, double* bx,
                         hipStream_t s) {
  const int64_t n = A->H.n, n3 = 3 * n;
  for (int stage = 0; stage < 6; ++stage) {
    const double* yin = y_in;
    if (stage > 0) {
      double* dst = Ystore ? Ystore + (stage - 1) * n3 : ys;
      check_hip(hm::launch_rk_stage_slip(n, stage, nullptr, dt, y_in, K, dst, p->V0, p->V_pl, p->a, x, s),
                "stage launch");
      yin = dst;
    } else {
      check_hip(hm::launch_rs_slip_rate(n, p->V0, p->V_pl, p->a, y_in, x, nullptr, s), "slip-rate launch");
    }
    with_pair(
        A, B, s, [&](hipStream_t q) { check_hip(A->product(false, x, ax, 1.0, 0.0, q, A->kernel), "product launch"); },
        [&](hipStream_t q) { check_hip(B->product(false, x, bx, 1.0, 0.0, q, B->kernel), "product launch"); });
    check_hip(hm::launch_rs_rhs(n, *p, yin, ax, B ? bx : nullptr, K + stage * n3, s), "rhs launch");
  }
  check_hip(hm::launch_rk_update_dt(n, dt, p->V0, p->a, K, y_in, y_out, D, s), "update launch");
}

bool transposable(hmat_t h) { return h->has_batched_t || (h->has_plain && h->plain.n_cols > 0); }

}  // namespace

namespace {

// The frozen-step integration of rs_rk45_replay on a workspace of at least
// replay_doubles(n) doubles (stage derivatives 18n, stage input 3n, x, A x,
// B x); every part is written before it is read.
int64_t replay_doubles(int64_t n) { return 24 * n; }

void enqueue_replay(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, const double* dts,
                    int64_t n_steps, double* ckpt, int64_t ckpt_every, double* ws, hipStream_t s) {
  const int64_t n = A->H.n, n3 = 3 * n;
  double* K = ws;  // 18n, then ys 3n, x, ax, bx
  double* ys = K + 6 * n3;
  double* x = ys + n3;
  double* ax = x + n;
  double* bx = ax + n;
  for (int64_t m = 0; m < n_steps; ++m) {
    if (ckpt && m % ckpt_every == 0)
      check_hip(hipMemcpyAsync(ckpt + (m / ckpt_every) * n3, y, n3 * sizeof(double), hipMemcpyDeviceToDevice, s),
                "checkpoint copy");
    enqueue_frozen_step(A, B, p, y, y, D, dts[m], K, nullptr, ys, x, ax, bx, s);
  }
}

// Scratch of rs_rk45_replay_noalloc (the workspace rs_rk45_replay takes from
// its caller), for callers that cannot allocate.  One copy per device,
// held until the process ends; calls on one device share it.
constexpr int64_t kStaticScratchBytes = (int64_t)32 << 20;
__device__ __align__(256) double scratch[kStaticScratchBytes / 8];

// Device address of `scratch` on device `dev` (which must be current),
// looked up once per device.  In host code the array's name is only a
// stand-in: kernels get this address.
double* static_scratch(int dev) {
  static std::mutex mu;
  static std::vector<void*> ptrs;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)ptrs.size() <= dev) ptrs.resize((size_t)dev + 1, nullptr);
  if (!ptrs[dev]) {
    void* ptr = nullptr;
    check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) hm::fail(HMAT_EDEVICE, "hipGetSymbolAddress(scratch) returned a null address");
    ptrs[dev] = ptr;
  }
  return static_cast<double*>(ptrs[dev]);
}

}  // namespace

hmat_status rs_rk45_replay(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, const double* dts,
                           int64_t n_steps, double* ckpt, int64_t ckpt_every, void* workspace, void* stream) {
  return guarded([&] {
    check_replay_args(A, B, p, dts, n_steps, ckpt_every);
    if (!y || !workspace) hm::fail(HMAT_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(workspace) % 8) hm::fail(HMAT_EINVAL, "workspace must be 8-byte aligned");
    if (n_steps == 0) return;
    DeviceGuard g(A->device);
    enqueue_replay(A, B, p, y, D, dts, n_steps, ckpt, ckpt_every, static_cast<double*>(workspace),
                   static_cast<hipStream_t>(stream));
  });
}

int64_t rs_rk45_replay_noalloc_max_n(void) { return kStaticScratchBytes / (8 * replay_doubles(1)); }

hmat_status rs_rk45_replay_noalloc(hmat_t A, hmat_t B, const rs_params* p, double* y, double* D, const double* dts,
                                   int64_t n_steps, double* ckpt, int64_t ckpt_every, void* stream) {
  return guarded([&] {
    check_replay_args(A, B, p, dts, n_steps, ckpt_every);
    if (!y) hm::fail(HMAT_EINVAL, "null argument");
    if (A->H.n > rs_rk45_replay_noalloc_max_n())
      hm::fail(HMAT_EINVAL, "n = " + std::to_string(A->H.n) + " exceeds the static scratch of " +
                                std::to_string(kStaticScratchBytes >> 20) + " MiB (at most " +
                                std::to_string(rs_rk45_replay_noalloc_max_n()) + " elements)");
    if (n_steps == 0) return;
    DeviceGuard g(A->device);
    enqueue_replay(A, B, p, y, D, dts, n_steps, ckpt, ckpt_every, static_scratch(A->device),
                   static_cast<hipStream_t>(stream));
  });
}

hmat_status hmat_check(hmat_t h, void* stream) {
  return guarded([&] {
    if (!h) hm::fail(HMAT_EINVAL, "null handle");
    if (!h->on_device) return;
    DeviceGuard g(h->device);
    check_wait_flag(h, static_cast<hipStream_t>(stream));
  });
}

int64_t rs_rk45_adjoint_workspace_bytes(int64_t n, int64_t ckpt_every) {
  if (n < 0 || ckpt_every < 1) return -1;
  if (n > 0 && ckpt_every > (INT64_MAX / 8 - 64) / (36 * n) - 1) return -1;
  return 8 * (36 * n * ckpt_every + 31 * n + 32);
}

hmat_status rs_rk45_adjoint(hmat_t A, hmat_t B, const rs_params* p, const double* ckpt, int64_t ckpt_every,
                            const double* dts, int64_t n_steps, const double* D_bar, double* y_bar, double* a_bar,
                            double* dc_bar, void* workspace, int64_t workspace_bytes, void* stream) {
  return guarded([&] {
    check_replay_args(A, B, p, dts, n_steps, ckpt_every);
    if (!y_bar || !a_bar || !dc_bar || !workspace || (n_steps > 0 && !ckpt)) hm::fail(HMAT_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(workspace) % 8) hm::fail(HMAT_EINVAL, "workspace must be 8-byte aligned");
    const int64_t n = A->H.n, n3 = 3 * n;
    const int64_t K = std::min<int64_t>(ckpt_every, std::max<int64_t>(n_steps, 1));
    const int64_t need = rs_rk45_adjoint_workspace_bytes(n, K);
    if (need < 0 || workspace_bytes < need) hm::fail(HMAT_EINVAL, "workspace too small");
    if (!transposable(A) || (B && !transposable(B)))
      hm::fail(HMAT_ESTATE, "handle created without opts.transpose");
    if (n_steps == 0) return;
    DeviceGuard g(A->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    double* states = static_cast<double*>(workspace);  // (K + 1) 3n
    double* Ys = states + (K + 1) * n3;                // K x 5 x 3n stage inputs 1..5
    double* Ks = Ys + K * 5 * n3;                      // K x 6 x 3n stage derivatives
    double* Ybar = Ks + K * 6 * n3;                    // 6 x 3n
    double* kbar = Ybar + 6 * n3;                      // 3n
    double* gbar = kbar + n3;
    double* sbar = gbar + n;
    double* xa = sbar + n;
    double* xb = xa + n;
    double* x = xb + n;
    double* ax = x + n;
    double* bx = ax + n;
    const int64_t nseg = (n_steps + ckpt_every - 1) / ckpt_every;
    for (int64_t seg = nseg - 1; seg >= 0; --seg) {
      const int64_t m0 = seg * ckpt_every, L = std::min(ckpt_every, n_steps - m0);
      // recompute the segment from its checkpoint, keeping every stage
      check_hip(hipMemcpyAsync(states, ckpt + seg * n3, n3 * sizeof(double), hipMemcpyDeviceToDevice, s),
                "checkpoint copy");
      for (int64_t l = 0; l < L; ++l)
        enqueue_frozen_step(A, B, p, states + l * n3, states + (l + 1) * n3, nullptr, dts[m0 + l], Ks + l * 6 * n3,
                            Ys + l * 5 * n3, nullptr, x, ax, bx, s);
      // reverse sweep over the segment
      for (int64_t l = L - 1; l >= 0; --l) {
        const double dt = dts[m0 + l];
        if (D_bar)
          check_hip(hm::launch_adj_dterm(n, 0.5 * dt, p->V0, p->a, states + (l + 1) * n3, D_bar, y_bar, a_bar, s),
                    "slip-term launch");
        for (int r = 5; r >= 0; --r) {
          const double* Yr = r == 0 ? states + l * n3 : Ys + (l * 5 + r - 1) * n3;
          const double* Kr = Ks + (l * 6 + r) * n3;
          check_hip(hm::launch_adj_vjp_pre(n, r, dt, *p, Yr, y_bar, Ybar, kbar, gbar, B ? sbar : nullptr, s),
                    "adjoint stage launch");
          with_pair(
              A, B, s,
              [&](hipStream_t q) { check_hip(A->product(true, gbar, xa, 1.0, 0.0, q, A->kernel), "transpose launch"); },
              [&](hipStream_t q) { check_hip(B->product(true, sbar, xb, 1.0, 0.0, q, B->kernel), "transpose launch"); });
          check_hip(hm::launch_adj_vjp_post(n, *p, Yr, Kr, kbar, xa, B ? xb : nullptr, Ybar + r * n3, a_bar, dc_bar,
                                            s),
                    "adjoint stage launch");
        }
        check_hip(hm::launch_adj_combine(n3, y_bar, Ybar, s), "adjoint combine launch");
        if (D_bar)
          check_hip(hm::launch_adj_dterm(n, 0.5 * dt, p->V0, p->a, states + l * n3, D_bar, y_bar, a_bar, s),
                    "slip-term launch");
      }
    }
  });
}

int64_t rs_ens_workspace_bytes(int64_t n, int32_t members) {
  if (n < 0 || members < 1 || members > hm::kEnsMax) return -1;
  return 8 * 28 * n * members + (int64_t)((sizeof(hm::EnsDevState) + 255) / 256 * 256);
}

namespace {

struct EnsWs {
  double *k, *ys, *y5, *Vs, *x, *ax, *bx;
  hm::EnsDevState* st;
};

EnsWs ens_workspace(void* workspace, int64_t n, int32_t M) {
  EnsWs w;
  const int64_t nm = n * M;
  double* base = static_cast<double*>(workspace);
  w.k = base;
  w.ys = w.k + 18 * nm;
  w.y5 = w.ys + 3 * nm;
  w.Vs = w.y5 + 3 * nm;
  w.x = w.Vs + nm;
  w.ax = w.x + nm;
  w.bx = w.ax + nm;
  w.st = reinterpret_cast<hm::EnsDevState*>(w.bx + nm);
  return w;
}

void enqueue_ens_attempt(hmat_t A, hmat_t B, const rs_ens_params* p, double* y, double* D, const EnsWs& w,
                         hipStream_t s) {
  const int64_t n = A->H.n, n3 = 3 * n;
  const int M = p->members;
  check_hip(hm::launch_ens_begin(w.st, s), "ensemble begin launch");
  for (int stage = 0; stage < 6; ++stage) {
    const double* yin = y;
    if (stage > 0) {
      check_hip(hm::launch_ens_stage_slip(n, M, stage, w.st, y, w.k, w.ys, p->V0, p->V_pl, p->a, w.x, s),
                "ensemble stage launch");
      yin = w.ys;
    } else {
      check_hip(hm::launch_ens_slip(n, M, p->V0, p->V_pl, p->a, y, w.x, w.Vs, s), "ensemble slip-rate launch");
    }
    with_pair(
        A, B, s, [&](hipStream_t q) { enqueue_mm(A, w.x, M, w.ax, M, M, 1.0, 0.0, p->mode, q); },
        [&](hipStream_t q) { enqueue_mm(B, w.x, M, w.bx, M, M, 1.0, 0.0, p->mode, q); });
    check_hip(hm::launch_ens_rhs(n, M, p->V0, p->f0, p->eta_rad, p->a, p->b, p->dc, yin, w.ax, B ? w.bx : nullptr,
                                 w.k + stage * n3 * M, s),
              "ensemble rhs launch");
  }
  check_hip(hm::launch_ens_finish_control(n3, M, w.st, y, w.k, w.y5, s), "ensemble error launch");
  check_hip(hm::launch_ens_accept(n, M, w.st, p->V0, p->a, w.y5, w.Vs, y, D, s), "ensemble accept launch");
}

}  // namespace

hmat_status rs_ens_rk45_run(hmat_t A, hmat_t B, const rs_ens_params* p, double* y, double* D, void* workspace,
                            rs_ens_state* st, int64_t n_accept, int64_t max_attempts, int32_t use_graph,
                            void* stream) {
  return guarded([&] {
    if (!A || !p || !y || !D || !workspace || !st) hm::fail(HMAT_EINVAL, "null argument");
    if (!A->on_device || (B && !B->on_device)) hm::fail(HMAT_ESTATE, "handle holds host blocks only");
    if (B && B->device != A->device) hm::fail(HMAT_EINVAL, "A and B live on different devices");
    if (p->n != A->H.n || (B && B->H.n != A->H.n)) hm::fail(HMAT_EINVAL, "n does not match the handles");
    if (p->members < 1 || p->members > hm::kEnsMax) hm::fail(HMAT_EINVAL, "members must be 1..64");
    if (p->mode != HMAT_MM_BF16X3 && p->mode != HMAT_MM_BF16X6) hm::fail(HMAT_EINVAL, "unknown mode");
    if (!p->a || !p->b || !p->dc) hm::fail(HMAT_EINVAL, "null friction parameter array");
    if (!(p->V0 > 0.0) || !(p->eta_rad >= 0.0) || !std::isfinite(p->f0) || !std::isfinite(p->V_pl))
      hm::fail(HMAT_EINVAL, "bad friction constants");
    for (hmat_t h : {A, B})
      if (h && (!h->mm_xs || !h->mm_ts || h->opts.max_nrhs < p->members))
        hm::fail(HMAT_ESTATE, "handle created without max_nrhs >= members");
    for (int r = 0; r < p->members; ++r)
      if (!(st->dt[r] > 0.0) || !std::isfinite(st->dt[r])) hm::fail(HMAT_EINVAL, "dt must be positive and finite");
    if (reinterpret_cast<uintptr_t>(workspace) % 8) hm::fail(HMAT_EINVAL, "workspace must be 8-byte aligned");
    if (n_accept < 0 || max_attempts < 0) hm::fail(HMAT_EINVAL, "counts must be >= 0");
    if (n_accept == 0) return;
    DeviceGuard g(A->device);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int M = p->members;
    const EnsWs w = ens_workspace(workspace, A->H.n, M);
    hm::EnsDevState d{};
    d.eps = st->eps_rk > 0.0 ? st->eps_rk : 1e-4;
    d.members = M;
    for (int r = 0; r < M; ++r) {
      d.t[r] = st->t[r];
      d.dt[r] = st->dt[r];
      d.accepted[r] = st->accepted[r];
      d.rejected[r] = st->rejected[r];
      d.target[r] = st->accepted[r] + n_accept;
    }
    check_hip(hipMemcpyAsync(w.st, &d, sizeof(d), hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    const bool graph = use_graph && s != nullptr;
    if (B && B != A) B->ensure_side();  // not during the capture
    if (graph) {
      std::vector<const void*> key{p->a, p->b, p->dc, y, D, workspace, s};
      for (double c : {p->V0, p->f0, p->eta_rad, p->V_pl}) push_double(key, c);
      key.push_back(reinterpret_cast<const void*>((intptr_t)(M * 16 + p->mode)));
      push_handle_key(key, A, B);
      A->ens_cache.ensure(key, s, [&](hipStream_t cs) { enqueue_ens_attempt(A, B, p, y, D, w, cs); });
    }
    int64_t launched = 0;
    for (;;) {
      int64_t batch = 0;
      for (int r = 0; r < M; ++r) batch = std::max<int64_t>(batch, d.target[r] - d.accepted[r]);
      if (max_attempts > 0) batch = std::min(batch, max_attempts - launched);
      if (batch <= 0) break;
      for (int64_t k = 0; k < batch; ++k) {
        if (graph) check_hip(hipGraphLaunch(A->ens_cache.exec, s), "hipGraphLaunch");
        else enqueue_ens_attempt(A, B, p, y, D, w, s);
      }
      launched += batch;
      check_hip(hipMemcpyAsync(&d, w.st, sizeof(d), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
      check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
      bool done = true;
      for (int r = 0; r < M; ++r) done = done && d.accepted[r] >= d.target[r];
      if (done) break;
    }
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    bool done = true;
    for (int r = 0; r < M; ++r) {
      st->t[r] = d.t[r];
      st->dt[r] = d.dt[r];
      st->last_err[r] = d.r[r];
      st->accepted[r] = d.accepted[r];
      st->rejected[r] = d.rejected[r];
      done = done && d.accepted[r] >= d.target[r];
    }
    if (!done) hm::fail(HMAT_ESTATE, "a member missed its target within max_attempts");
  });
}

hmat_status hmat_kernel_entries(const hmat_mesh* mesh, const hmat_green* green, int64_t count, const int64_t* rows,
                                const int64_t* cols, double* out) {
  return guarded([&] {
    if (!mesh || !green || (count > 0 && (!rows || !cols || !out))) hm::fail(HMAT_EINVAL, "null argument");
    if (count < 0) hm::fail(HMAT_EINVAL, "count must be >= 0");
    hm::Geometry geo;
    std::unique_ptr<hm::EntryFn> E(hm::make_entry_fn(*mesh, *green, geo));
    for (int64_t k = 0; k < count; ++k) {
      if (rows[k] < 0 || rows[k] >= mesh->n || cols[k] < 0 || cols[k] >= mesh->n)
        hm::fail(HMAT_EINVAL, "entry index out of range");
      out[k] = E->entry(rows[k], cols[k]);
    }
  });
}

void hmat_destroy(hmat_t h) { delete h; }

const char* hmat_last_error(void) { return g_err.c_str(); }

}  // extern "C"
