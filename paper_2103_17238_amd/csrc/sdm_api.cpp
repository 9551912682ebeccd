// sdm_api.cpp -- host driver behind include/sdm.h: validation, launch
// planning (cell-size classes, big-cell buckets), workspace carving, batches
// of simulations sharing launches, statistics and the autotuner.
//
// The mapping to the PySDM v1 paper's API ("API in brief"): sdm_init plays
// Builder(n_sd, backend) + Box(dt, dv) + Coalescence(kernel) + build(attributes),
// sdm_coalescence_step plays Particulator.run(n_steps) with the step counter
// n_steps, and sdm_moments the product registry (dv/dlnr spectrum).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/sdm.h"
#include "sdm_internal.hpp"
#include "sdm_refresh.hpp"

using sdm::BigAdapt;
using sdm::BigBucket;
using sdm::BigPairBlock;
using sdm::BigChunk;
using sdm::BigTask;
using sdm::PlanDev;
using sdm::SimDesc;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int ceil_log2(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x) ++b;
  return b;
}

// The automatic mid-size limit (mid_max_slots = -1).  A step over a few
// cells is latency-bound: the big-cell path's two launches take about 15 us
// for one cell of 4 096 to 16 384 slots, the mid-size kernel 13 us at 4 096,
// 21 at 8 192 and 36 at 16 384.  Over many cells throughput decides, and
// there the mid-size kernel is ahead (1 024 cells of 8 192 slots: 184 us per
// step against 375).  So plain cells above kPlainMidMaxDefault slots take the
// big-cell path when a plan has at most kAutoBigCells of them, and then (or
// with cells above 16384 slots) so do at most kAutoBigCells plain cells of
// 513 to 4096 slots: in the serving mix (a few requests per size range in a
// batch) that took the served p50 from 12.6-16.0 to 10.4 ms and p99 from
// 30-34 to 17 ms, fewer launches and no concurrent mid-size kernels beside
// the big-cell chain.  A lone mid-size cell keeps the mid-size kernel.
// Adaptive cells keep the mid-size kernel up to its limit (adaptive big
// cells read one word back per four substep rounds).
constexpr int32_t kPlainMidMaxDefault = 4096;
constexpr int64_t kAutoBigCells = 32;

sdm_tuning default_tuning() {
  sdm_tuning t;
  t.wave_class_mask = sdm::kClassAll;
  t.waves_per_cell = 1;
  t.big_bucket_target = 0;  // automatic
  t.lpt_order = 1;
  t.mid_max_slots = -1;  // automatic
  t.big_bucket_cap = 0;
  return t;
}

bool tuning_ok(const sdm_tuning& t) {
  const int w = t.waves_per_cell;
  return (w == 1 || w == 2 || w == 4 || w == 8) &&
         (t.big_bucket_target == 0 || t.big_bucket_target >= sdm::kMinBucketTarget) &&
         t.big_bucket_target <= 1024 && (t.wave_class_mask & ~sdm::kClassAll) == 0 &&
         t.mid_max_slots >= -1 && t.mid_max_slots <= sdm::kMidCapMax && t.big_bucket_cap >= 0 &&
         t.big_bucket_cap <= 1024;
}

// The chunking and bucketing of a big cell of n slots: at most kBigMaxChunks
// key blocks of a multiple of kBigChunkUnit slots, at most kBigMaxBuckets
// buckets.
struct BigShape {
  int32_t nb, n_chunks, chunk_slots;
};
// The automatic bucket target (big_bucket_target = 0), from one cell's step
// time on the big-cell path: 128 SDs per bucket fastest up to 32768 slots
// (15.1-15.8 us against 15.6-16.4 at 256), 256 at 65536 (17.8 us), 512
// above (21.8 us against 22.6 at 2^17, 31.8 against 35.0 at 2^18).
static int64_t auto_bucket_target(int64_t n) { return n <= 32768 ? 128 : n <= 65536 ? 256 : 512; }

BigShape big_shape(int64_t n, const sdm_tuning& t) {
  BigShape b;
  const int64_t tgt = t.big_bucket_target > 0 ? t.big_bucket_target : auto_bucket_target(n);
  b.nb = (int32_t)std::min<int64_t>(sdm::kBigMaxBuckets, std::max<int64_t>(1, (n + tgt - 1) / tgt));
  const int64_t unit = (int64_t)sdm::kBigChunkUnit * sdm::kBigMaxChunks;
  b.chunk_slots = (int32_t)(sdm::kBigChunkUnit * std::max<int64_t>(1, (n + unit - 1) / unit));
  b.n_chunks = (int32_t)std::max<int64_t>(1, (n + b.chunk_slots - 1) / b.chunk_slots);
  return b;
}

}  // namespace

struct Plan;

// The last stream a simulation's steps were enqueued on, and an event
// recorded there after them.  A plan records one event per step call and
// every member points at it, so the check in plan_step costs nothing for
// members stepped on the same stream.
struct Busy {
  hipEvent_t ev = nullptr;
  hipStream_t st = nullptr;
  Busy() = default;
  Busy(const Busy&) = delete;
  Busy& operator=(const Busy&) = delete;
  ~Busy() {
    if (ev) (void)hipEventDestroy(ev);
  }
};

struct sdm_sim {
  sdm_config cfg{};
  int64_t* xi = nullptr;
  double* v = nullptr;
  double* attrs = nullptr;
  const int64_t* cell_off = nullptr;
  // host copy of cell_off; stale after a device-side rebind until a host
  // path needs it (fresh_offsets)
  mutable std::vector<int64_t> off;
  mutable bool off_stale = false;
  uint32_t step = 0;
  uint32_t limit = 0xFFFFFFFFu;
  sdm_tuning tuning = default_tuning();
  int64_t* sink = nullptr;
  int64_t sink_cap = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  uint32_t* d_status = nullptr;
  unsigned long long* d_stats = nullptr;
  int64_t* d_pair_base = nullptr;
  unsigned long long* d_rebind = nullptr;  // two result words of the device-side rebind
  uint32_t layout_gen = 0;                 // bumped by every sdm_rebind
  bool broken = false;  // a failed re-plan left the launch tables unusable
  std::shared_ptr<Busy> last;  // where the last step of this simulation was enqueued
  Plan* plan = nullptr;
};

static sdm_status rebind_host(sdm_sim* s, int64_t* xi, double* v, double* attrs,
                              const int64_t* cell_off, hipStream_t st);

// Pinned host memory for the device-to-host reads of the set-up calls (cell
// offsets, the validation flag): a copy into pageable memory goes through
// the runtime's staging buffer, which can make it wait for work on other
// streams.  One buffer per process, grown as needed, guarded by a mutex;
// growing it (a pinned allocation) is the only step that may synchronise.
struct PinnedReadback {
  std::mutex mu;
  void* buf = nullptr;
  size_t bytes = 0;
  ~PinnedReadback() {
    if (buf) (void)hipHostFree(buf);
  }
};
static PinnedReadback g_pinned;

// Copies `bytes` from device `src` to host `dst` through the pinned buffer,
// ordered on `st`, and synchronises `st`.
static bool read_back(void* dst, const void* src, size_t bytes, hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_pinned.mu);
  if (g_pinned.bytes < bytes) {
    if (g_pinned.buf) (void)hipHostFree(g_pinned.buf);
    g_pinned.buf = nullptr;
    g_pinned.bytes = 0;
    const size_t want = std::max<size_t>(bytes, 1 << 16);
    if (hipHostMalloc(&g_pinned.buf, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    g_pinned.bytes = want;
  }
  if (hipMemcpyAsync(g_pinned.buf, src, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  std::memcpy(dst, g_pinned.buf, bytes);
  return true;
}

// Refreshes the host copy of the offsets after device-side rebinds.  The
// device offsets are final once sdm_rebind returned (it synchronised the
// stream that wrote them), so a blocking copy suffices; no device-wide
// synchronisation.
static bool fresh_offsets(const sdm_sim* s) {
  if (!s->off_stale) return true;
  if (hipMemcpy(s->off.data(), s->cell_off, sizeof(int64_t) * s->off.size(),
                hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  s->off_stale = false;
  return true;
}

// ---------------------------------------------------------------------------
// Launch plan over a list of simulations
// ---------------------------------------------------------------------------
struct Tables {
  std::vector<sdm::CellTask> wave[sdm::kNumClasses];  // plain-mode cells first, then adaptive
  int n_plain[sdm::kNumClasses] = {};
  std::vector<sdm::CellTask> mid[sdm::kNumMid];  // plain-mode cells first, then adaptive
  int n_mid_plain[sdm::kNumMid] = {0, 0, 0, 0};
  std::vector<BigTask> big;
  std::vector<BigChunk> chunks;  // plain-mode big cells
  std::vector<BigBucket> buckets;
  std::vector<int> abig;  // adaptive big cells: their tasks, chunks, buckets, pair blocks
  std::vector<BigChunk> achunks;
  std::vector<BigBucket> abuckets;
  std::vector<BigPairBlock> apblocks;
  int64_t tmp_total = 0;  // slots of big cells (entries, order)
  int64_t off_total = 0;  // words of the chunks' bucket offsets
  int64_t n_wave_total() const {
    int64_t n = 0;
    for (auto& w : wave) n += (int64_t)w.size();
    return n;
  }
};

static void build_tables(const std::vector<sdm_sim*>& ms, const sdm_tuning& tu, Tables& T) {
  struct Item {
    int64_t n;
    int sim, cell, adaptive;
  };
  std::vector<Item> items[sdm::kNumClasses];
  std::vector<Item> mids[sdm::kNumMid];
  const int mask = tu.wave_class_mask | sdm::kClassTop;
  // the mid-size limit of plain and of adaptive cells (automatic: see
  // kAutoBigCells)
  int64_t mid_plain = tu.mid_max_slots, mid_adapt = tu.mid_max_slots;
  if (tu.mid_max_slots < 0) {
    // plain cells the automatic rule may move: of 4097..16384 slots (upper),
    // of 513..4096 (lower), and any above 16384 (on the big-cell path anyway)
    int64_t upper = 0, lower = 0, above = 0;
    for (auto* s : ms)
      if (!s->cfg.adaptive)
        for (int c = 0; c < s->cfg.n_cells; ++c) {
          const int64_t n = s->off[c + 1] - s->off[c];
          upper += (n > kPlainMidMaxDefault && n <= sdm::kMidCapMax) ? 1 : 0;
          lower += (n > sdm::kWaveCapMax && n <= kPlainMidMaxDefault) ? 1 : 0;
          above += n > sdm::kMidCapMax ? 1 : 0;
        }
    mid_plain = upper <= kAutoBigCells ? kPlainMidMaxDefault : sdm::kMidCapMax;
    // a few smaller ones join a big-cell path the plan runs anyway: extra
    // blocks in its two launches instead of mid-size launches beside them
    const bool big_path = above > 0 || (upper > 0 && upper <= kAutoBigCells);
    if (big_path && upper <= kAutoBigCells && lower <= kAutoBigCells) mid_plain = sdm::kWaveCapMax;
    mid_adapt = sdm::kMidCapMax;
  }
  for (int i = 0; i < (int)ms.size(); ++i) {
    const int64_t mid_max = ms[i]->cfg.adaptive ? mid_adapt : mid_plain;
    const auto& off = ms[i]->off;
    const int C = ms[i]->cfg.n_cells;
    for (int c = 0; c < C; ++c) {
      const int64_t n = off[c + 1] - off[c];
      if (n <= 0) continue;
      if (n <= sdm::kWaveCapMax) {
        int k = 0;
        while (!((mask >> k) & 1) || n > sdm::class_cap(k)) ++k;
        items[k].push_back({n, i, c, ms[i]->cfg.adaptive});
        continue;
      }
      if (n <= mid_max) {
        int k = 0;
        while (n > sdm::mid_cap(k)) ++k;
        mids[k].push_back({n, i, c, ms[i]->cfg.adaptive});
        continue;
      }
      BigTask t{};
      t.xi = ms[i]->xi + off[c];
      t.v = ms[i]->v + off[c];
      t.sim = i;
      t.cell = c;
      t.n_slots = (int32_t)n;
      const BigShape bs = big_shape(n, tu);
      t.nb = bs.nb;
      t.n_chunks = bs.n_chunks;
      t.chunk_slots = bs.chunk_slots;
      t.sort_cap = tu.big_bucket_cap > 0 ? tu.big_bucket_cap : 1024;
      t.pad = 0;
      t.tmp_base = T.tmp_total;
      T.tmp_total += n;
      t.off_base = T.off_total;
      T.off_total += (int64_t)t.n_chunks * (t.nb + 1);
      const int ti = (int)T.big.size();
      T.big.push_back(t);
      const bool ad = ms[i]->cfg.adaptive != 0;
      for (int32_t f = 0; f < t.n_chunks; ++f)
        (ad ? T.achunks : T.chunks).push_back({ti, f, t.sim, 0});
      for (int32_t b = 0; b < t.nb; ++b) (ad ? T.abuckets : T.buckets).push_back({ti, b, t.sim, 0});
      if (ad) {
        T.abig.push_back(ti);
        for (int64_t m = 0; m < n / 2; m += sdm::kAbigPairs)
          T.apblocks.push_back({ti, (int32_t)m});
      }
    }
  }
  // plain-mode cells first (one kernel each), largest first within a mode
  auto order = [&](std::vector<Item>& v, std::vector<sdm::CellTask>& out, int& n_plain) {
    std::stable_sort(v.begin(), v.end(), [&](const Item& a, const Item& b) {
      if (a.adaptive != b.adaptive) return a.adaptive < b.adaptive;
      return tu.lpt_order ? a.n > b.n : false;
    });
    n_plain = 0;
    for (auto& it : v) n_plain += it.adaptive ? 0 : 1;
    out.resize(v.size());
    for (size_t j = 0; j < v.size(); ++j) {
      const sdm_sim* m = ms[v[j].sim];
      sdm::CellTask& ct = out[j];
      ct.xi = m->xi + m->off[v[j].cell];
      ct.v = m->v + m->off[v[j].cell];
      ct.n = (int32_t)v[j].n;
      ct.sim = v[j].sim;
      ct.cell = v[j].cell;
      ct.pad = 0;
    }
  };
  for (int k = 0; k < sdm::kNumClasses; ++k) order(items[k], T.wave[k], T.n_plain[k]);
  for (int k = 0; k < sdm::kNumMid; ++k) order(mids[k], T.mid[k], T.n_mid_plain[k]);
}

struct Layout {
  size_t desc, wave[sdm::kNumClasses], wave_alt[sdm::kNumClasses], order_flag[sdm::kNumClasses],
      order_cnt[sdm::kNumClasses], mid[sdm::kNumMid], big, chunks, buckets, ekey, exi, ev, offs,
      skey, ord, abig, achunks, abuckets, apblocks, astate[2], apmax[2], apre, apair,
      aactive, total;
};

static Layout layout_of(int n_members, const Tables& T) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  L.desc = take(sizeof(SimDesc) * std::max(n_members, 1));
  for (int k = 0; k < sdm::kNumClasses; ++k) {
    const size_t na = T.wave[k].size() - (size_t)T.n_plain[k];
    L.wave[k] = take(sizeof(sdm::CellTask) * std::max<size_t>(T.wave[k].size(), 1));
    L.wave_alt[k] = take(sizeof(sdm::CellTask) * std::max<size_t>(na, 1));
    L.order_flag[k] = take(sizeof(uint32_t) * std::max<size_t>(na, 1));
    L.order_cnt[k] = take(sizeof(uint32_t) * sdm::kOrderGroups * (na / sdm::kOrderBlock + 1));
  }
  for (int k = 0; k < sdm::kNumMid; ++k)
    L.mid[k] = take(sizeof(sdm::CellTask) * std::max<size_t>(T.mid[k].size(), 1));
  L.big = take(sizeof(BigTask) * std::max<size_t>(T.big.size(), 1));
  L.chunks = take(sizeof(BigChunk) * std::max<size_t>(T.chunks.size(), 1));
  L.buckets = take(sizeof(BigBucket) * std::max<size_t>(T.buckets.size(), 1));
  const size_t nt = (size_t)std::max<int64_t>(T.tmp_total, 1);
  L.ekey = take(sizeof(unsigned long long) * nt);
  L.exi = take(sizeof(long long) * nt);
  L.ev = take(sizeof(double) * nt);
  L.offs = take(sizeof(uint32_t) * (size_t)std::max<int64_t>(T.off_total, 1));
  L.skey = take(sizeof(unsigned long long) * nt);
  L.ord = take(sizeof(uint32_t) * nt);
  const bool ad = !T.abig.empty();
  L.abig = take(sizeof(int) * std::max<size_t>(T.abig.size(), 1));
  L.achunks = take(sizeof(BigChunk) * std::max<size_t>(T.achunks.size(), 1));
  L.abuckets = take(sizeof(BigBucket) * std::max<size_t>(T.abuckets.size(), 1));
  L.apblocks = take(sizeof(BigPairBlock) * std::max<size_t>(T.apblocks.size(), 1));
  for (int k = 0; k < 2; ++k) {
    L.astate[k] = take(sizeof(BigAdapt) * (ad ? T.big.size() : 1));
    L.apmax[k] = take(sizeof(unsigned long long) * (ad ? T.big.size() : 1));
  }
  L.apre = take(sizeof(double) * (size_t)(ad ? T.tmp_total : 1));
  L.apair = take(sizeof(unsigned long long) * (size_t)(ad ? T.tmp_total : 1));
  L.aactive = take(sizeof(uint32_t));
  L.total = o;
  return L;
}

// plan bytes for the worst-case tuning: every cell above 512 slots may go to
// the big-cell path (smallest bucket target) or to a mid-size list, and the
// class masks split the same cells differently (one alignment pad per list)
static size_t plan_bytes_worst(const std::vector<sdm_sim*>& ms) {
  sdm_tuning t = default_tuning();
  t.big_bucket_target = sdm::kMinBucketTarget;
  t.mid_max_slots = 0;
  Tables T;
  build_tables(ms, t, T);
  size_t n_mid = 0;
  for (auto* s : ms)
    for (int c = 0; c < s->cfg.n_cells; ++c) {
      const int64_t n = s->off[c + 1] - s->off[c];
      n_mid += (n > sdm::kWaveCapMax && n <= sdm::kMidCapMax) ? 1 : 0;
    }
  // the smallest target gives the most buckets, so the most offsets
  return layout_of((int)ms.size(), T).total + align_up(sizeof(sdm::CellTask) * n_mid) +
         (4 * sdm::kNumClasses + sdm::kNumMid) * kAlign;
}

struct Plan {
  std::vector<sdm_sim*> members;
  sdm_tuning tuning = default_tuning();
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Tables T;
  PlanDev dev{};
  std::vector<SimDesc> desc;  // host copy of the device descriptors
  uint32_t counter = 0;       // launch step of the next step
  uint32_t flip = 0;          // launches since the tables were built
  sdm::SideStream side;       // created at the first step
  std::shared_ptr<Busy> busy;  // event recorded after each step call, created at the first
  Plan() = default;
  Plan(const Plan&) = delete;
  Plan& operator=(const Plan&) = delete;
  ~Plan() {
    if (side.fork) (void)hipEventDestroy(side.fork);
    if (side.join) (void)hipEventDestroy(side.join);
    if (side.join2) (void)hipEventDestroy(side.join2);
    if (side.stream) (void)hipStreamDestroy(side.stream);
    if (side.stream2) (void)hipStreamDestroy(side.stream2);
  }
};

static SimDesc make_desc(const sdm_sim* s, uint32_t delta) {
  SimDesc d{};
  d.xi = s->xi;
  d.v = s->v;
  d.attrs = s->attrs;
  d.cell_off = s->cell_off;
  d.status = s->d_status;
  d.stats = s->d_stats;
  d.sink = s->sink;
  d.pair_base = s->d_pair_base;
  d.n_slots = s->cfg.n_slots;
  d.q = s->cfg.dt_s / s->cfg.dv_m3;
  d.dt = s->cfg.dt_s;
  d.dv = s->cfg.dv_m3;
  d.b = s->cfg.golovin_b_per_s;
  d.seed_lo = (uint32_t)(s->cfg.seed & 0xFFFFFFFFull);
  d.seed_hi = (uint32_t)(s->cfg.seed >> 32);
  d.step_delta = delta;
  d.step_limit = s->limit;
  d.n_attr = s->cfg.n_attr;
  d.kernel = s->cfg.kernel;
  d.adaptive = s->cfg.adaptive;
  d.max_substeps = s->cfg.max_substeps > 0 ? s->cfg.max_substeps : 1024;
  return d;
}

#define HIP_TRY(x)                        \
  do {                                    \
    if ((x) != hipSuccess) {              \
      (void)hipGetLastError();            \
      return SDM_EDEVICE;                 \
    }                                     \
  } while (0)

// stream-ordered upload; src must stay alive until `st` is synchronised
template <typename T>
static hipError_t upload(T* dst, const std::vector<T>& src, hipStream_t st) {
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, st);
}

// LDS one workgroup may use on the current device
static size_t lds_block_limit() {
  int dev = 0, a = 0, b = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    a = 64 * 1024;
  if (hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) b = 0;
  (void)hipGetLastError();
  return (size_t)std::max(a, b);
}

// (Re)build the plan tables for its members and upload them on `st`.  Syncs
// `st` before (the old tables may be in use) and, with sync_end, after (the
// host tables then need not outlive the call's caller; sdm_init instead
// covers the uploads with its own later synchronisation).  No device-wide
// synchronisation: work on other streams keeps running.
static sdm_status plan_setup(Plan* p, hipStream_t st, bool sync_end = true) {
  for (auto* m : p->members)
    if (!fresh_offsets(m)) return SDM_EDEVICE;
  p->T = Tables();
  build_tables(p->members, p->tuning, p->T);
  for (int k = 0; k < sdm::kNumClasses; ++k)  // every used class must fit one workgroup's LDS
    if (!p->T.wave[k].empty() && sdm::cell_lds_bytes(k) > lds_block_limit()) return SDM_EINVAL;
  for (int k = 0; k < sdm::kNumMid; ++k)
    if (!p->T.mid[k].empty() && sdm::mid_lds_bytes(k) > lds_block_limit()) return SDM_EINVAL;
  const Layout L = layout_of((int)p->members.size(), p->T);
  if (L.total > p->ws_bytes) return SDM_ENOMEM;
  char* w = p->ws;
  PlanDev& d = p->dev;
  d.geo = 0;
  for (auto* s : p->members) d.geo |= (s->cfg.kernel == SDM_GEOMETRIC) ? 1 : 0;
  d.desc = reinterpret_cast<const SimDesc*>(w + L.desc);
  for (int k = 0; k < sdm::kNumClasses; ++k) {
    d.wave_tasks[k] = reinterpret_cast<sdm::CellTask*>(w + L.wave[k]);
    d.wave_alt[k] = reinterpret_cast<sdm::CellTask*>(w + L.wave_alt[k]);
    d.order_flag[k] = reinterpret_cast<uint32_t*>(w + L.order_flag[k]);
    d.order_cnt[k] = reinterpret_cast<uint32_t*>(w + L.order_cnt[k]);
    d.n_wave[k] = (int)p->T.wave[k].size();
    d.n_plain[k] = p->T.n_plain[k];
  }
  for (int k = 0; k < sdm::kNumMid; ++k) {
    d.mid_tasks[k] = reinterpret_cast<const sdm::CellTask*>(w + L.mid[k]);
    d.n_mid[k] = (int)p->T.mid[k].size();
    d.n_mid_plain[k] = p->T.n_mid_plain[k];
  }
  d.big = reinterpret_cast<const BigTask*>(w + L.big);
  d.n_big = (int)p->T.big.size();
  d.chunks = reinterpret_cast<const BigChunk*>(w + L.chunks);
  d.n_chunks = (int)p->T.chunks.size();
  int nb_max = 1;
  for (const auto& t : p->T.big) nb_max = std::max(nb_max, (int)t.nb);
  d.big_hist_bytes = (unsigned)(sizeof(uint32_t) * (size_t)(nb_max + 1));
  d.buckets = reinterpret_cast<const BigBucket*>(w + L.buckets);
  d.n_buckets = (int)p->T.buckets.size();
  d.ekey = reinterpret_cast<unsigned long long*>(w + L.ekey);
  d.exi = reinterpret_cast<long long*>(w + L.exi);
  d.ev = reinterpret_cast<double*>(w + L.ev);
  d.offs = reinterpret_cast<uint32_t*>(w + L.offs);
  d.skey = reinterpret_cast<unsigned long long*>(w + L.skey);
  d.ord = reinterpret_cast<uint32_t*>(w + L.ord);
  d.abig = reinterpret_cast<const int*>(w + L.abig);
  d.n_abig = (int)p->T.abig.size();
  d.achunks = reinterpret_cast<const BigChunk*>(w + L.achunks);
  d.n_achunks = (int)p->T.achunks.size();
  d.abuckets = reinterpret_cast<const BigBucket*>(w + L.abuckets);
  d.n_abuckets = (int)p->T.abuckets.size();
  d.apblocks = reinterpret_cast<const BigPairBlock*>(w + L.apblocks);
  d.n_apblocks = (int)p->T.apblocks.size();
  for (int k = 0; k < 2; ++k) {
    d.astate[k] = reinterpret_cast<BigAdapt*>(w + L.astate[k]);
    d.apmax[k] = reinterpret_cast<unsigned long long*>(w + L.apmax[k]);
  }
  d.apre = reinterpret_cast<double*>(w + L.apre);
  d.apair = reinterpret_cast<unsigned long long*>(w + L.apair);
  d.aactive = reinterpret_cast<uint32_t*>(w + L.aactive);

  // the old tables may still be read by steps enqueued on `st`
  HIP_TRY(hipStreamSynchronize(st));
  p->desc.clear();
  for (auto* s : p->members) p->desc.push_back(make_desc(s, s->step - p->counter));
  HIP_TRY(upload(const_cast<SimDesc*>(d.desc), p->desc, st));
  for (int k = 0; k < sdm::kNumClasses; ++k) {
    HIP_TRY(upload(d.wave_tasks[k], p->T.wave[k], st));
    const size_t na = p->T.wave[k].size() - (size_t)p->T.n_plain[k];
    if (na > 0)
      HIP_TRY(hipMemcpyAsync(d.wave_alt[k], p->T.wave[k].data() + p->T.n_plain[k],
                             sizeof(sdm::CellTask) * na, hipMemcpyHostToDevice, st));
    p->flip = 0;
  }
  for (int k = 0; k < sdm::kNumMid; ++k)
    HIP_TRY(upload(const_cast<sdm::CellTask*>(d.mid_tasks[k]), p->T.mid[k], st));
  HIP_TRY(upload(const_cast<BigTask*>(d.big), p->T.big, st));
  HIP_TRY(upload(const_cast<BigChunk*>(d.chunks), p->T.chunks, st));
  HIP_TRY(upload(const_cast<BigBucket*>(d.buckets), p->T.buckets, st));
  HIP_TRY(upload(const_cast<int*>(d.abig), p->T.abig, st));
  HIP_TRY(upload(const_cast<BigChunk*>(d.achunks), p->T.achunks, st));
  HIP_TRY(upload(const_cast<BigBucket*>(d.abuckets), p->T.abuckets, st));
  HIP_TRY(upload(const_cast<BigPairBlock*>(d.apblocks), p->T.apblocks, st));
  if (sync_end) HIP_TRY(hipStreamSynchronize(st));
  return SDM_OK;
}

// descriptors must follow member step counters, limits and sinks
static sdm_status plan_refresh(Plan* p, hipStream_t st) {
  bool changed = false;
  for (size_t i = 0; i < p->members.size(); ++i) {
    const SimDesc want = make_desc(p->members[i], p->members[i]->step - p->counter);
    if (std::memcmp(&want, &p->desc[i], sizeof(SimDesc)) != 0) {
      p->desc[i] = want;
      changed = true;
    }
  }
  if (!changed) return SDM_OK;
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(upload(const_cast<SimDesc*>(p->dev.desc), p->desc, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SDM_OK;
}

// One outer step of the plan's adaptive big cells: substep rounds until every
// cell is done, reading the count of cells still stepping every
// kAbigRoundsPerCheck rounds (a synchronisation of `st`).
static sdm_status abig_step(Plan* p, uint32_t k_abs, hipStream_t st) {
  uint32_t umax = 0;
  for (auto* m : p->members)
    if (m->cfg.adaptive)
      umax = std::max<uint32_t>(umax, (uint32_t)(m->cfg.max_substeps > 0 ? m->cfg.max_substeps
                                                                         : 1024));
  if (sdm::launch_abig_init(p->dev, k_abs, st) != hipSuccess) return SDM_EDEVICE;
  // a capped substep ends a cell's step: umax + 1 rounds always suffice
  for (uint32_t r = 0; r <= umax;) {
    for (int i = 0; i < sdm::kAbigRoundsPerCheck && r <= umax; ++i, ++r)
      if (sdm::launch_abig_round(p->dev, k_abs, r, st) != hipSuccess)
        return SDM_EDEVICE;
    uint32_t active = 0;
    if (sdm::launch_abig_active(p->dev, r, p->dev.aactive, st) != hipSuccess ||
        !read_back(&active, p->dev.aactive, sizeof(uint32_t), st))
      return SDM_EDEVICE;
    if (active == 0) break;
  }
  return SDM_OK;
}

static sdm_status plan_step(Plan* p, int32_t n_steps, hipStream_t st) {
  if (n_steps < 0) return SDM_EINVAL;
  for (auto* m : p->members)
    if (m->broken) return SDM_ESTATE;
  // a member whose last steps were enqueued on another stream and still run
  for (auto* m : p->members)
    if (m->last && m->last->st != st) {
      const hipError_t q = hipEventQuery(m->last->ev);
      if (q == hipErrorNotReady) {
        (void)hipGetLastError();
        return SDM_EAGAIN;
      }
      if (q != hipSuccess) {
        (void)hipGetLastError();
        return SDM_EDEVICE;
      }
    }
  if (n_steps == 0) return SDM_OK;
  sdm_status r = plan_refresh(p, st);
  if (r != SDM_OK) return r;
  // steps any member still takes
  int64_t active = 0;
  for (auto* s : p->members) {
    const int64_t left = s->step < s->limit ? (int64_t)(s->limit - s->step) : 0;
    active = std::max<int64_t>(active, std::min<int64_t>(left, n_steps));
  }
  if (active > 0 && !p->side.stream) {
    if (hipStreamCreateWithFlags(&p->side.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->side.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->side.join, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return SDM_EDEVICE;
    }
  }
  // a second side stream once the plan has cells of the 8192- or 4096-slot class
  if (active > 0 && (p->dev.n_mid[2] > 0 || p->dev.n_mid[1] > 0) && !p->side.stream2) {
    if (hipStreamCreateWithFlags(&p->side.stream2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->side.join2, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return SDM_EDEVICE;
    }
  }
  for (int64_t k = 0; k < active;) {  // up to kFuseMax steps per launch
    const int f = (int)std::min<int64_t>(sdm::kFuseMax, active - k);
    if (sdm::launch_step(p->dev, p->counter + (uint32_t)k, p->flip++, f,
                         p->tuning.waves_per_cell, st, p->side) != hipSuccess)
      return SDM_EDEVICE;
    for (int t = 0; t < f && p->dev.n_abig > 0; ++t) {  // adaptive big cells: substep rounds
      const sdm_status r2 = abig_step(p, p->counter + (uint32_t)(k + t), st);
      if (r2 != SDM_OK) return r2;
    }
    k += f;
  }
  p->counter += (uint32_t)n_steps;
  for (auto* s : p->members) {
    const int64_t left = s->step < s->limit ? (int64_t)(s->limit - s->step) : 0;
    s->step += (uint32_t)std::min<int64_t>(left, n_steps);
  }
  if (active > 0) {  // members are busy on `st` until this event
    if (!p->busy) {
      p->busy = std::make_shared<Busy>();
      if (hipEventCreateWithFlags(&p->busy->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        p->busy.reset();
        return SDM_EDEVICE;
      }
    }
    if (hipEventRecord(p->busy->ev, st) != hipSuccess) {
      (void)hipGetLastError();
      return SDM_EDEVICE;
    }
    p->busy->st = st;
    for (auto* s : p->members) s->last = p->busy;
  }
  // keep descriptors consistent: members that hit their limit get re-synced lazily
  return SDM_OK;
}

// ---------------------------------------------------------------------------
// Simulation handle
// ---------------------------------------------------------------------------
static size_t sim_region_bytes(int32_t n_cells) {
  return align_up(sizeof(uint32_t)) + align_up(2 * sizeof(unsigned long long)) +
         align_up(sizeof(unsigned long long) * sdm::kStatSlots * sdm::kStatFields) +
         align_up(sizeof(int64_t) * ((size_t)n_cells + 1));
}

static bool cfg_ok(const sdm_config* c) {
  if (!c) return false;
  if (c->n_slots < 0 || c->n_cells < 1 || c->n_attr < 0 || c->n_attr > 16) return false;
  if (!(c->dt_s > 0.0) || !(c->dv_m3 > 0.0) || !std::isfinite(c->dt_s) ||
      !std::isfinite(c->dv_m3))
    return false;
  if (c->kernel != SDM_GOLOVIN && c->kernel != SDM_GEOMETRIC) return false;
  if (!(c->golovin_b_per_s >= 0.0) || !std::isfinite(c->golovin_b_per_s)) return false;
  if (c->adaptive != 0 && c->adaptive != 1) return false;
  if (c->max_substeps < 0 || c->reserved != 0) return false;
  if (c->n_slots > 0x7FFFFFFFLL) return false;
  return true;
}

static bool offsets_ok(const sdm_config* c, const int64_t* off) {
  if (off[0] != 0 || off[c->n_cells] != c->n_slots) return false;
  for (int i = 0; i < c->n_cells; ++i)
    if (off[i + 1] < off[i] || off[i + 1] - off[i] > sdm::kBigMaxSlots) return false;
  return true;
}

static size_t plan_bytes_for(const sdm_config* cfg, const int64_t* off) {
  sdm_sim tmp;
  tmp.cfg = *cfg;
  tmp.off.assign(off, off + cfg->n_cells + 1);
  std::vector<sdm_sim*> ms{&tmp};
  return plan_bytes_worst(ms);
}

static size_t plan_bytes_bound(const sdm_config* c) {
  const int64_t ns = c->n_slots, C = c->n_cells;
  const int64_t nbig = std::min<int64_t>(C, ns / (sdm::kWaveCapMax + 1));
  Tables T;  // sizes only
  size_t o = 0;
  auto take = [&](size_t b) { o += align_up(b); };
  take(sizeof(SimDesc));
  for (int k = 0; k < sdm::kNumClasses + sdm::kNumMid; ++k)
    take(sizeof(sdm::CellTask) * (size_t)std::max<int64_t>(C, 1));
  for (int k = 0; k < sdm::kNumClasses; ++k) {  // second lists, order flags and counts
    take(sizeof(sdm::CellTask) * (size_t)std::max<int64_t>(C, 1));
    take(sizeof(uint32_t) * (size_t)std::max<int64_t>(C, 1));
    take(sizeof(uint32_t) * sdm::kOrderGroups * (size_t)(C / sdm::kOrderBlock + 1));
  }
  take(sizeof(BigTask) * (size_t)std::max<int64_t>(nbig, 1));
  const int64_t nchk = ns / sdm::kBigChunkUnit + nbig + 1;
  take(sizeof(BigChunk) * (size_t)nchk);
  const int64_t nbk = ns / sdm::kMinBucketTarget + nbig + 1;
  take(sizeof(BigBucket) * (size_t)nbk);
  const size_t nt = (size_t)std::max<int64_t>(ns, 1);
  take(sizeof(unsigned long long) * nt);  // entries: keys, multiplicities, volumes
  take(sizeof(long long) * nt);
  take(sizeof(double) * nt);
  // offsets: n_chunks (nb + 1) <= 8 n + 1024 words for a cell of n slots
  take(sizeof(uint32_t) * (size_t)(8 * ns + 1024 * nbig + 1));
  take(sizeof(unsigned long long) * nt);  // slow-path keys and order
  take(sizeof(uint32_t) * nt);
  // adaptive big cells: task list, chunks and buckets (counted above once),
  // pair blocks, per-cell state and largest p, per-pair pre-products and slots
  const bool ad = c->adaptive != 0;
  take(sizeof(int) * (size_t)std::max<int64_t>(nbig, 1));
  take(sizeof(BigChunk) * (size_t)(ad ? nchk : 1));
  take(sizeof(BigBucket) * (size_t)(ad ? nbk : 1));
  take(sizeof(BigPairBlock) * (size_t)(ad ? ns / (2 * sdm::kAbigPairs) + nbig + 1 : 1));
  for (int k = 0; k < 2; ++k) {
    take(sizeof(BigAdapt) * (size_t)std::max<int64_t>(nbig, 1));
    take(sizeof(unsigned long long) * (size_t)std::max<int64_t>(nbig, 1));
  }
  take(sizeof(double) * (size_t)(ad ? std::max<int64_t>(ns, 1) : 1));
  take(sizeof(unsigned long long) * (size_t)(ad ? std::max<int64_t>(ns, 1) : 1));
  take(sizeof(uint32_t));
  (void)T;
  return o;
}

extern "C" {

size_t sdm_workspace_bytes(const sdm_config* cfg, const int64_t* host_cell_off) {
  if (!cfg_ok(cfg)) return 0;
  const size_t plan = host_cell_off ? (offsets_ok(cfg, host_cell_off)
                                           ? plan_bytes_for(cfg, host_cell_off)
                                           : 0)
                                    : plan_bytes_bound(cfg);
  if (host_cell_off && plan == 0) return 0;
  return sim_region_bytes(cfg->n_cells) + plan;
}

sdm_status sdm_init(sdm_sim** out, const sdm_config* cfg, int64_t* xi, double* v, double* attrs,
                    const int64_t* cell_off, void* workspace, size_t workspace_bytes,
                    void* stream) {
  if (!out) return SDM_EINVAL;
  *out = nullptr;
  if (!cfg_ok(cfg) || !cell_off || !workspace) return SDM_EINVAL;
  if (cfg->n_slots > 0 && (!xi || !v)) return SDM_EINVAL;
  if (cfg->n_attr > 0 && cfg->n_slots > 0 && !attrs) return SDM_EINVAL;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return SDM_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  sdm::set_lds_limits();

  sdm_sim* s = new (std::nothrow) sdm_sim();
  if (!s) return SDM_ENOMEM;
  s->cfg = *cfg;
  if (s->cfg.max_substeps == 0) s->cfg.max_substeps = 1024;
  s->xi = xi;
  s->v = v;
  s->attrs = cfg->n_attr > 0 ? attrs : nullptr;
  s->cell_off = cell_off;
  s->off.resize((size_t)cfg->n_cells + 1);
  if (!read_back(s->off.data(), cell_off, sizeof(int64_t) * s->off.size(), st)) {
    delete s;
    return SDM_EDEVICE;
  }
  if (!offsets_ok(cfg, s->off.data())) {
    delete s;
    return SDM_EINVAL;
  }
  const size_t need = sim_region_bytes(cfg->n_cells) + plan_bytes_for(cfg, s->off.data());
  if (workspace_bytes < need) {
    delete s;
    return SDM_ENOMEM;
  }
  char* w = static_cast<char*>(workspace);
  s->ws = w;
  s->ws_bytes = workspace_bytes;
  s->d_status = reinterpret_cast<uint32_t*>(w);
  w += align_up(sizeof(uint32_t));
  s->d_rebind = reinterpret_cast<unsigned long long*>(w);
  w += align_up(2 * sizeof(unsigned long long));
  s->d_stats = reinterpret_cast<unsigned long long*>(w);
  w += align_up(sizeof(unsigned long long) * sdm::kStatSlots * sdm::kStatFields);
  s->d_pair_base = reinterpret_cast<int64_t*>(w);
  w += align_up(sizeof(int64_t) * ((size_t)cfg->n_cells + 1));

  s->plan = new (std::nothrow) Plan();
  if (!s->plan) {
    delete s;
    return SDM_ENOMEM;
  }
  s->plan->members = {s};
  s->plan->ws = w;
  s->plan->ws_bytes = workspace_bytes - (size_t)(w - static_cast<char*>(workspace));
  s->plan->tuning = s->tuning;
  // Everything below is ordered on `st` and covered by one synchronisation
  // of `st` (no device-wide one): counters, pair bases, the plan's tables,
  // the validation kernel and the read-back of its flag.
  std::vector<int64_t> pb((size_t)cfg->n_cells + 1, 0);
  for (int c = 0; c < cfg->n_cells; ++c) pb[c + 1] = pb[c] + (s->off[c + 1] - s->off[c]) / 2;
  uint32_t flags = 0;
  bool ok = hipMemsetAsync(s->d_status, 0, sizeof(uint32_t), st) == hipSuccess &&
            hipMemsetAsync(s->d_stats, 0,
                           sizeof(unsigned long long) * sdm::kStatSlots * sdm::kStatFields,
                           st) == hipSuccess &&
            hipMemcpyAsync(s->d_pair_base, pb.data(), sizeof(int64_t) * pb.size(),
                           hipMemcpyHostToDevice, st) == hipSuccess;
  const sdm_status r = ok ? plan_setup(s->plan, st, false) : SDM_EDEVICE;
  ok = ok && r == SDM_OK &&
       sdm::launch_validate(xi, v, cfg->n_slots, s->d_status, st) == hipSuccess;
  // the flag read-back synchronises st: pb and the plan's host tables are
  // alive until here
  const bool synced = ok ? read_back(&flags, s->d_status, sizeof(uint32_t), st)
                        : hipStreamSynchronize(st) == hipSuccess && false;
  if (!ok || !synced) {
    (void)hipGetLastError();
    delete s->plan;
    delete s;
    return r != SDM_OK ? r : SDM_EDEVICE;
  }
  if (flags & sdm::kFlagInvalid) {
    delete s->plan;
    delete s;
    return SDM_EINVAL;
  }
  *out = s;
  return SDM_OK;
}

sdm_status sdm_coalescence_step(sdm_sim* s, int32_t n_steps, void* stream) {
  if (!s || n_steps < 0) return SDM_EINVAL;
  s->plan->counter = s->step;
  return plan_step(s->plan, n_steps, reinterpret_cast<hipStream_t>(stream));
}

sdm_status sdm_condensation_step(sdm_sim* s, const sdm_cond_config* cc, const double* temperature,
                                 const double* pressure, const double* saturation, void* stream) {
  if (!s || !cc || !temperature || !pressure || !saturation) return SDM_EINVAL;
  const int A = s->cfg.n_attr;
  if (!(cc->dt_s > 0.0) || !std::isfinite(cc->dt_s) || cc->reserved != 0 ||
      cc->dry_volume_attr < 0 || cc->dry_volume_attr >= A || cc->kappa_attr < 0 ||
      cc->kappa_attr >= A || cc->dry_volume_attr == cc->kappa_attr || cc->max_iter < 0 ||
      cc->max_iter > 64)
    return SDM_EINVAL;
  if (s->broken) return SDM_ESTATE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (s->last && s->last->st != st) {  // busy on another stream: enqueue nothing
    const hipError_t q = hipEventQuery(s->last->ev);
    if (q == hipErrorNotReady) {
      (void)hipGetLastError();
      return SDM_EAGAIN;
    }
    if (q != hipSuccess) {
      (void)hipGetLastError();
      return SDM_EDEVICE;
    }
  }
  if (!fresh_offsets(s)) return SDM_EDEVICE;
  int64_t max_cell = 0;
  for (int c = 0; c < s->cfg.n_cells; ++c)
    max_cell = std::max<int64_t>(max_cell, s->off[c + 1] - s->off[c]);
  if (max_cell == 0) return SDM_OK;
  const int64_t ns = s->cfg.n_slots;
  if (sdm::launch_condense(s->xi, s->v, s->attrs + (int64_t)cc->dry_volume_attr * ns,
                           s->attrs + (int64_t)cc->kappa_attr * ns, s->cell_off, s->cfg.n_cells,
                           ns, temperature, pressure, saturation, cc->dt_s,
                           cc->max_iter > 0 ? cc->max_iter : 32, st) != hipSuccess)
    return SDM_EDEVICE;
  // the simulation is busy on `st` until this event (its plan's token)
  Plan* p = s->plan;
  if (!p->busy) {
    p->busy = std::make_shared<Busy>();
    if (hipEventCreateWithFlags(&p->busy->ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      p->busy.reset();
      return SDM_EDEVICE;
    }
  }
  if (hipEventRecord(p->busy->ev, st) != hipSuccess) {
    (void)hipGetLastError();
    return SDM_EDEVICE;
  }
  p->busy->st = st;
  s->last = p->busy;
  return SDM_OK;
}

sdm_status sdm_moments(sdm_sim* s, int64_t* m0, double* m12, double* attr_sums,
                       const double* vol_edges, int32_t n_bins, double* spectrum, void* stream) {
  if (!s || n_bins < 0) return SDM_EINVAL;
  if (spectrum && (!vol_edges || n_bins < 1 || n_bins > sdm::kMomentsMaxBins)) return SDM_EINVAL;
  const SimDesc d = make_desc(s, 0);
  // one wave per cell when cells hold 256 slots or fewer on average
  const int waves = s->cfg.n_slots <= 256 * (int64_t)s->cfg.n_cells ? 1 : 4;
  if (sdm::launch_moments(d, s->cfg.n_cells, waves, m0, m12, attr_sums, vol_edges,
                          spectrum ? n_bins : 0, spectrum,
                          reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return SDM_EDEVICE;
  return SDM_OK;
}

sdm_status sdm_status_word(sdm_sim* s, uint32_t* flags, void* stream) {
  if (!s || !flags) return SDM_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(flags, s->d_status, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SDM_OK;
}

sdm_status sdm_reset_status(sdm_sim* s, void* stream) {
  if (!s) return SDM_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipMemsetAsync(s->d_status, 0, sizeof(uint32_t), st));
  HIP_TRY(hipMemsetAsync(s->d_stats, 0,
                         sizeof(unsigned long long) * sdm::kStatSlots * sdm::kStatFields, st));
  return SDM_OK;
}

sdm_status sdm_stats(sdm_sim* s, uint64_t out[4], void* stream) {
  if (!s || !out) return SDM_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<unsigned long long> h((size_t)sdm::kStatSlots * sdm::kStatFields);
  HIP_TRY(hipMemcpyAsync(h.data(), s->d_stats, sizeof(unsigned long long) * h.size(),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int f = 0; f < 4; ++f) out[f] = 0;
  for (int i = 0; i < sdm::kStatSlots; ++i)
    for (int f = 0; f < sdm::kStatFields; ++f) out[f] += h[(size_t)i * sdm::kStatFields + f];
  return SDM_OK;
}

uint32_t sdm_get_step(const sdm_sim* s) { return s ? s->step : 0u; }

sdm_status sdm_set_step(sdm_sim* s, uint32_t step) {
  if (!s) return SDM_EINVAL;
  s->step = step;
  return SDM_OK;
}

sdm_status sdm_set_step_limit(sdm_sim* s, uint32_t limit) {
  if (!s) return SDM_EINVAL;
  s->limit = limit;
  return SDM_OK;
}

sdm_status sdm_debug_gamma_sink(sdm_sim* s, int64_t* dev_buf, int64_t capacity) {
  if (!s) return SDM_EINVAL;
  if (dev_buf && s->off_stale) {  // the pair bases follow the current layout
    if (!fresh_offsets(s)) return SDM_EDEVICE;
    std::vector<int64_t> pb((size_t)s->cfg.n_cells + 1, 0);
    for (int c = 0; c < s->cfg.n_cells; ++c) pb[c + 1] = pb[c] + (s->off[c + 1] - s->off[c]) / 2;
    if (hipMemcpy(s->d_pair_base, pb.data(), sizeof(int64_t) * pb.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      return SDM_EDEVICE;
    }
  }
  if (dev_buf) {
    int64_t pairs = 0;
    for (int c = 0; c < s->cfg.n_cells; ++c) pairs += (s->off[c + 1] - s->off[c]) / 2;
    if (capacity < 2 * pairs) return SDM_EINVAL;
  }
  s->sink = dev_buf;
  s->sink_cap = dev_buf ? capacity : 0;
  return SDM_OK;
}

sdm_status sdm_get_tuning(const sdm_sim* s, sdm_tuning* t) {
  if (!s || !t) return SDM_EINVAL;
  *t = s->tuning;
  return SDM_OK;
}

sdm_status sdm_set_tuning(sdm_sim* s, const sdm_tuning* t, void* stream) {
  if (!s || !t || !tuning_ok(*t)) return SDM_EINVAL;
  s->tuning = *t;
  s->tuning.wave_class_mask |= sdm::kClassTop;
  s->plan->tuning = s->tuning;
  s->plan->counter = s->step;
  return plan_setup(s->plan, reinterpret_cast<hipStream_t>(stream));
}

sdm_status sdm_rebind(sdm_sim* s, int64_t* xi, double* v, double* attrs, const int64_t* cell_off,
                      void* stream) {
  if (!s || !cell_off) return SDM_EINVAL;
  const sdm_config& cfg = s->cfg;
  if (cfg.n_slots > 0 && (!xi || !v)) return SDM_EINVAL;
  if (cfg.n_attr > 0 && cfg.n_slots > 0 && !attrs) return SDM_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // Device-side refresh when the plan has only workgroup-per-cell tasks and
  // no gamma sink: rewrite the tasks from the new offsets, then read back
  // two words; if a cell outgrew its class or slots sit in a cell without a
  // task, fall through to the host re-plan below.
  const sdm::PlanDev& pd = s->plan->dev;
  bool only_wave = pd.n_big == 0 && !s->sink;
  for (int k = 0; k < sdm::kNumMid; ++k) only_wave = only_wave && pd.n_mid[k] == 0;
  if (only_wave) {
    unsigned long long w[2] = {1ull, 0ull};
    // the descriptor for the new buffers goes with the same synchronisation
    // (a failed check re-plans, which rewrites it)
    Plan* p = s->plan;
    p->desc[0].xi = xi;
    p->desc[0].v = v;
    p->desc[0].attrs = cfg.n_attr > 0 ? attrs : nullptr;
    p->desc[0].cell_off = cell_off;
    if (sdm::launch_refresh(pd, cell_off, cfg.n_cells, cfg.n_slots, xi, v, s->d_rebind, st) !=
            hipSuccess ||
        hipMemcpyAsync(const_cast<SimDesc*>(pd.desc), p->desc.data(), sizeof(SimDesc),
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(w, s->d_rebind, sizeof(w), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      // the tables may be half rewritten for the new buffers while the
      // handle still names the old ones: re-plan the old layout, or refuse
      // further steps if that fails too
      (void)hipGetLastError();
      if (plan_setup(s->plan, st) != SDM_OK) s->broken = true;
      return SDM_EDEVICE;
    }
    if (w[0] == 0 && w[1] == (unsigned long long)cfg.n_slots) {
      s->xi = xi;
      s->v = v;
      s->attrs = cfg.n_attr > 0 ? attrs : nullptr;
      s->cell_off = cell_off;
      s->off_stale = true;
      s->plan->counter = s->step;
      s->layout_gen += 1;
      return SDM_OK;
    }
  }
  // host re-plan; the device pass above may have rewritten part of the
  // tables, so a rejected layout re-plans the old one before returning
  const sdm_status r = rebind_host(s, xi, v, attrs, cell_off, st);
  if (r != SDM_OK && only_wave) {
    const sdm_status r2 = plan_setup(s->plan, st);
    if (r2 != SDM_OK) {
      s->broken = true;
      return r2;
    }
  }
  return r;
}

static sdm_status rebind_host(sdm_sim* s, int64_t* xi, double* v, double* attrs,
                              const int64_t* cell_off, hipStream_t st) {
  const sdm_config& cfg = s->cfg;
  std::vector<int64_t> off((size_t)cfg.n_cells + 1);
  if (hipMemcpyAsync(off.data(), cell_off, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost,
                     st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return SDM_EDEVICE;
  }
  if (!offsets_ok(&cfg, off.data())) return SDM_EINVAL;
  if (s->ws_bytes < sim_region_bytes(cfg.n_cells) + plan_bytes_for(&cfg, off.data()))
    return SDM_ENOMEM;
  std::vector<int64_t> pb((size_t)cfg.n_cells + 1, 0);
  for (int c = 0; c < cfg.n_cells; ++c) pb[c + 1] = pb[c] + (off[c + 1] - off[c]) / 2;
  if (hipMemcpyAsync(s->d_pair_base, pb.data(), sizeof(int64_t) * pb.size(),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    (void)hipGetLastError();
    return SDM_EDEVICE;
  }
  s->xi = xi;
  s->v = v;
  s->attrs = cfg.n_attr > 0 ? attrs : nullptr;
  s->cell_off = cell_off;
  s->off.swap(off);
  s->off_stale = false;
  s->plan->counter = s->step;
  s->layout_gen += 1;
  return plan_setup(s->plan, st);
}

void sdm_free(sdm_sim* s) {
  if (!s) return;
  delete s->plan;
  delete s;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct sdm_batch {
  Plan plan;
  std::vector<uint32_t> gens;  // members' layout generations the tables were built for
};

size_t sdm_batch_workspace_bytes(sdm_sim* const* sims, int32_t n) {
  if (!sims || n < 1) return 0;
  std::vector<sdm_sim*> ms(sims, sims + n);
  for (auto* s : ms)
    if (!s || !fresh_offsets(s)) return 0;
  return plan_bytes_worst(ms);
}

sdm_status sdm_batch_create(sdm_batch** out, sdm_sim* const* sims, int32_t n, void* workspace,
                            size_t workspace_bytes, void* stream) {
  if (!out || !sims || n < 1 || !workspace) return SDM_EINVAL;
  *out = nullptr;
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return SDM_EINVAL;
  sdm_batch* b = new (std::nothrow) sdm_batch();
  if (!b) return SDM_ENOMEM;
  b->plan.members.assign(sims, sims + n);
  for (auto* s : b->plan.members)
    if (!s) {
      delete b;
      return SDM_EINVAL;
    }
  b->plan.ws = static_cast<char*>(workspace);
  b->plan.ws_bytes = workspace_bytes;
  b->plan.tuning = b->plan.members[0]->tuning;
  b->plan.counter = 0;
  const sdm_status r = plan_setup(&b->plan, reinterpret_cast<hipStream_t>(stream));
  if (r != SDM_OK) {
    delete b;
    return r;
  }
  for (auto* s : b->plan.members) b->gens.push_back(s->layout_gen);
  *out = b;
  return SDM_OK;
}

sdm_status sdm_batch_step(sdm_batch* b, int32_t n_steps, void* stream) {
  if (!b) return SDM_EINVAL;
  for (size_t i = 0; i < b->gens.size(); ++i)  // a member was re-pointed since
    if (b->plan.members[i]->layout_gen != b->gens[i]) return SDM_ESTATE;
  return plan_step(&b->plan, n_steps, reinterpret_cast<hipStream_t>(stream));
}

void sdm_batch_free(sdm_batch* b) { delete b; }

const char* sdm_strerror(sdm_status st) {
  switch (st) {
    case SDM_OK: return "ok";
    case SDM_EINVAL: return "invalid argument, configuration or state";
    case SDM_ENOMEM: return "workspace too small";
    case SDM_EDEVICE: return "HIP runtime error";
    case SDM_ESTATE: return "call not valid in this state";
    case SDM_EAGAIN: return "resource busy";
  }
  return "unknown status";
}

sdm_status sdm_philox_fill(uint32_t* out, int64_t n, uint32_t c0, uint32_t c1, uint32_t c2,
                           uint32_t c3, uint64_t seed, void* stream) {
  if (n < 0 || (n > 0 && !out)) return SDM_EINVAL;
  if (sdm::launch_philox_fill(out, n, c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32),
                              reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return SDM_EDEVICE;
  return SDM_OK;
}

sdm_status sdm_kernel_values(int32_t kernel, double golovin_b, const double* v1, const double* v2,
                             int64_t n, double* out, void* stream) {
  if (n < 0 || (n > 0 && (!v1 || !v2 || !out))) return SDM_EINVAL;
  if (kernel != SDM_GOLOVIN && kernel != SDM_GEOMETRIC) return SDM_EINVAL;
  if (sdm::launch_kernel_values(kernel, golovin_b, v1, v2, n, out,
                                reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
    return SDM_EDEVICE;
  return SDM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner (sdm_autotune): times candidate launch shapes on a scratch copy
// of the state.  Results never depend on the tuning, only speed does.
// ---------------------------------------------------------------------------
static std::string tune_key(const sdm_sim* s) {
  hipDeviceProp_t prop{};
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&prop, dev);
  // share of slots per size class (<=64, <=128, <=256, <=512, >512), in 5 % steps
  int64_t cls[5] = {0, 0, 0, 0, 0};
  int64_t big_max = 0;
  for (int c = 0; c < s->cfg.n_cells; ++c) {
    const int64_t n = s->off[c + 1] - s->off[c];
    int k = n <= 64 ? 0 : n <= 128 ? 1 : n <= 256 ? 2 : n <= 512 ? 3 : 4;
    cls[k] += n;
    big_max = std::max(big_max, n);
  }
  const double tot = (double)std::max<int64_t>(s->cfg.n_slots, 1);
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s/cu%d/k%d/a%d/ad%d/l2n%d/c%d-%d-%d-%d-%d/b%d",
                prop.gcnArchName, prop.multiProcessorCount, s->cfg.kernel, s->cfg.n_attr,
                s->cfg.adaptive, ceil_log2(std::max<int64_t>(s->cfg.n_slots, 1)),
                (int)std::lround(20 * cls[0] / tot), (int)std::lround(20 * cls[1] / tot),
                (int)std::lround(20 * cls[2] / tot), (int)std::lround(20 * cls[3] / tot),
                (int)std::lround(20 * cls[4] / tot), ceil_log2(std::max<int64_t>(big_max, 1)));
  return buf;
}

static bool cache_lookup(const char* path, const std::string& key, sdm_tuning* t) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char k[512];
    sdm_tuning x{};
    double ms = 0;
    if (std::sscanf(line,
                    "{\"key\": \"%511[^\"]\", \"wave_class_mask\": %d, \"waves_per_cell\": %d, "
                    "\"big_bucket_target\": %d, \"lpt_order\": %d, \"mid_max_slots\": %d, "
                    "\"big_bucket_cap\": %d, \"ms_per_step\": %lf}",
                    k, &x.wave_class_mask, &x.waves_per_cell, &x.big_bucket_target,
                    &x.lpt_order, &x.mid_max_slots, &x.big_bucket_cap, &ms) == 8 &&
        key == k && tuning_ok(x)) {
      *t = x;  // the last matching line wins
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

static void cache_store(const char* path, const std::string& key, const sdm_tuning& t, double ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"key\": \"%s\", \"wave_class_mask\": %d, \"waves_per_cell\": %d, "
               "\"big_bucket_target\": %d, \"lpt_order\": %d, \"mid_max_slots\": %d, "
               "\"big_bucket_cap\": %d, \"ms_per_step\": %.6f}\n",
               key.c_str(), t.wave_class_mask, t.waves_per_cell, t.big_bucket_target,
               t.lpt_order, t.mid_max_slots, t.big_bucket_cap, ms);
  std::fclose(f);
}

extern "C" size_t sdm_autotune_scratch_bytes(const sdm_sim* s) {
  if (!s || !fresh_offsets(s)) return 0;
  const size_t ns = (size_t)s->cfg.n_slots;
  return align_up(ns * 8) + align_up(ns * 8) + align_up(ns * 8 * (size_t)s->cfg.n_attr) +
         sim_region_bytes(s->cfg.n_cells) + plan_bytes_for(&s->cfg, s->off.data());
}

extern "C" sdm_status sdm_autotune(sdm_sim* s, void* scratch, size_t scratch_bytes,
                                   int32_t trial_steps, const char* cache_path,
                                   sdm_tuning* chosen, void* stream) {
  if (!s || trial_steps < 1) return SDM_EINVAL;
  if (!fresh_offsets(s)) return SDM_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const std::string key = tune_key(s);
  sdm_tuning best{};
  if (!cache_path) {  // the environment may name a cache for callers that pass none
    const char* env = std::getenv("SDM_TUNE_CACHE");
    if (env && *env) cache_path = env;
  }
  if (cache_path && cache_lookup(cache_path, key, &best)) {
    const sdm_status r = sdm_set_tuning(s, &best, stream);
    if (r == SDM_OK && chosen) *chosen = s->tuning;
    return r;
  }
  if (!scratch || scratch_bytes < sdm_autotune_scratch_bytes(s) ||
      reinterpret_cast<uintptr_t>(scratch) % kAlign)
    return SDM_ENOMEM;
  const size_t ns = (size_t)s->cfg.n_slots;
  char* w = static_cast<char*>(scratch);
  int64_t* xi2 = reinterpret_cast<int64_t*>(w);
  w += align_up(ns * 8);
  double* v2 = reinterpret_cast<double*>(w);
  w += align_up(ns * 8);
  double* a2 = s->cfg.n_attr ? reinterpret_cast<double*>(w) : nullptr;
  w += align_up(ns * 8 * (size_t)s->cfg.n_attr);
  const size_t ws_left = scratch_bytes - (size_t)(w - static_cast<char*>(scratch));

  auto restore = [&]() {
    bool ok = hipMemcpyAsync(xi2, s->xi, ns * 8, hipMemcpyDeviceToDevice, st) == hipSuccess &&
              hipMemcpyAsync(v2, s->v, ns * 8, hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (a2)
      ok = ok && hipMemcpyAsync(a2, s->attrs, ns * 8 * (size_t)s->cfg.n_attr,
                                hipMemcpyDeviceToDevice, st) == hipSuccess;
    return ok;
  };

  // candidate shapes
  bool has_small[sdm::kNumClasses] = {}, has_big = false, has_mid = false;
  for (int c = 0; c < s->cfg.n_cells; ++c) {
    const int64_t n = s->off[c + 1] - s->off[c];
    if (n > sdm::kMidCapMax) {
      has_big = true;
    } else if (n > sdm::kWaveCapMax) {
      has_mid = true;
    } else if (n > 0) {
      int k = 0;
      while (n > sdm::class_cap(k)) ++k;
      has_small[k] = true;
    }
  }
  std::vector<int> masks = {sdm::kClassTop};
  for (int m : {0x18, 0x14, 0x1C, 0x1E, 0x1F, 0x12, 0x11}) {  // masks that split populated classes
    bool useful = false;
    for (int k = 0; k < sdm::kNumClasses - 1; ++k)
      if (((m >> k) & 1) && has_small[k]) useful = true;
    if (useful) masks.push_back(m);
  }
  std::vector<int> mids = has_mid && !s->cfg.adaptive
                              ? std::vector<int>{sdm::kMidCapMax, kPlainMidMaxDefault, 0}
                              : std::vector<int>{-1};
  std::vector<sdm_tuning> cands;
  for (int mm : mids) {
    // the bucket size matters only when some cell takes the big-cell path
    const bool bigs = has_big || (has_mid && mm >= 0 && mm < sdm::kMidCapMax);
    const std::vector<int> targets =
        bigs ? std::vector<int>{0, 64, 128, 256, 512} : std::vector<int>{0};
    bool any_small = false;
    for (bool h : has_small) any_small = any_small || h;
    const std::vector<int> waves = any_small ? std::vector<int>{1, 2, 4, 8} : std::vector<int>{1};
    for (int m : masks)
      for (int wpb : waves)
        for (int tg : targets) cands.push_back({m, wpb, tg, 1, mm, 0});
  }

  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best_ms = 1e300;
  bool any = false;
  for (const auto& cand : cands) {
    if (!restore()) return SDM_EDEVICE;
    sdm_sim* t = nullptr;
    sdm_config cfg = s->cfg;
    if (sdm_init(&t, &cfg, xi2, v2, a2, s->cell_off, w, ws_left, stream) != SDM_OK) continue;
    t->step = s->step;
    if (sdm_set_tuning(t, &cand, stream) != SDM_OK) {
      sdm_free(t);
      continue;
    }
    bool ok = sdm_coalescence_step(t, 1, stream) == SDM_OK;  // warm-up
    ok = ok && hipEventRecord(e0, st) == hipSuccess;
    ok = ok && sdm_coalescence_step(t, trial_steps, stream) == SDM_OK;
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
    float ms = 0.f;
    ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    sdm_free(t);
    if (!ok) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return SDM_EDEVICE;
    }
    const double per = ms / trial_steps;
    if (per < best_ms) {
      best_ms = per;
      best = cand;
      any = true;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!any) return SDM_EDEVICE;
  const sdm_status r = sdm_set_tuning(s, &best, stream);
  if (r != SDM_OK) return r;
  if (cache_path) cache_store(cache_path, key, s->tuning, best_ms);
  if (chosen) *chosen = s->tuning;
  return SDM_OK;
}
