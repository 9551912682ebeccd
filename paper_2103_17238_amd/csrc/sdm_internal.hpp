// sdm_internal.hpp -- types shared by the HIP kernels and the host driver of
// libsdm (not part of the public ABI, see include/sdm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sdm {

constexpr int kStatSlots = 256;   // spread of the statistics counters (fewer atomics per address)
constexpr int kStatFields = 4;    // live SD-steps, colliding pairs, cell substeps, cell steps
constexpr int kNumClasses = 5;    // workgroup-per-cell capacities 64, 128, 256, 384, 512 slots
constexpr int kWaveCapMax = 512;  // cells above this go to the mid-size or big-cell path
constexpr int kNumMid = 4;        // mid-size capacities 2048, 4096, 8192, 16384 slots
constexpr int kMidCapMax = 16384;
constexpr int kBigChunkUnit = 1024;   // slots per Philox round of a big-cell key block
constexpr int kBigMaxChunks = 256;    // key blocks per big cell, at most
constexpr int kBigMaxBuckets = 16384;  // buckets per big cell, at most (one LDS histogram)
constexpr int64_t kBigMaxSlots = 8388608;  // slots per cell, at most (kBigMaxBuckets x 512)
constexpr int kAbigPairs = 256;   // pairs per block of the adaptive big-cell pair pass
constexpr int kAbigRoundsPerCheck = 4;  // adaptive big-cell substep rounds between host checks
constexpr int kMinBucketTarget = 32;
constexpr int kOrderBlock = 1024;  // tasks per block of the dispatch-order partition
constexpr int kOrderGroups = 4;    // dispatch-order groups by substeps taken
constexpr int kFuseMax = 8;        // steps of a multi-step call fused in one launch
constexpr int kMomentsMaxBins = 1024;  // spectrum bins of sdm_moments, at most

constexpr uint32_t kFlagSubstepCap = 1u;
constexpr uint32_t kFlagGammaCap = 2u;
constexpr uint32_t kFlagBucketOverflow = 4u;
constexpr uint32_t kFlagInvalid = 8u;

inline int class_cap(int k) { return k < 3 ? 64 << k : (k == 3 ? 384 : 512); }
constexpr int kClassAll = 0x1F;  // every class enabled
constexpr int kClassTop = 0x10;  // the 512-slot class, always enabled
inline int mid_cap(int k) { return 2048 << k; }

// Per-simulation parameters read by every step kernel (device array, one per member).
struct SimDesc {
  int64_t* xi;
  double* v;
  double* attrs;  // [n_attr][n_slots]
  const int64_t* cell_off;
  uint32_t* status;
  unsigned long long* stats;  // [kStatSlots][kStatFields]
  int64_t* sink;              // optional gamma sink
  const int64_t* pair_base;   // per-cell first pair index of the sink
  int64_t n_slots;
  double q;   // dt / dV
  double dt;  // s
  double dv;  // m^3
  double b;   // Golovin b [1/s]
  uint32_t seed_lo, seed_hi;
  uint32_t step_delta;  // member step = launch step + step_delta
  uint32_t step_limit;  // member steps >= limit are skipped
  int32_t n_attr;
  int32_t kernel;
  int32_t adaptive;
  int32_t max_substeps;
};

// A cell of at most kWaveCapMax slots, processed by one workgroup; the entry
// carries the cell's own xi / v pointers so that fetching it takes one hop.
struct CellTask {
  int64_t* xi;  // first slot of the cell
  double* v;
  int32_t n;  // slots
  int32_t sim;
  int32_t cell;
  int32_t pad;
};

// A cell above the mid-size limit.  Its slots are split into n_chunks
// chunks of chunk_slots; the key pass writes each chunk's live entries into
// the chunk's own segment of the entry arrays, grouped by bucket (nb key
// ranges), with nb + 1 offsets per chunk; each bucket is then gathered,
// ordered and paired by one workgroup.
struct BigTask {
  int64_t* xi;  // first slot of the cell
  double* v;
  int64_t tmp_base;  // first entry of the cell in the entry and order arrays (n_slots)
  int64_t off_base;  // first word of the cell's offsets (n_chunks x (nb + 1))
  int32_t sim;
  int32_t cell;
  int32_t nb;           // buckets, 1..kBigMaxBuckets
  int32_t n_chunks;     // 1..kBigMaxChunks
  int32_t chunk_slots;  // a multiple of kBigChunkUnit
  int32_t sort_cap;     // longest bucket ordered in LDS (longer: ranked in global memory)
  int32_t n_slots;
  int32_t pad;
};

struct BigChunk {  // chunk_slots consecutive slots of one big cell
  int32_t task;
  int32_t index;  // chunk of the cell: slots [index chunk_slots, (index + 1) chunk_slots)
  int32_t sim;    // the task's simulation (read beside the task)
  int32_t pad;
};

struct BigBucket {  // one bucket of one big cell
  int32_t task;
  int32_t bucket;
  int32_t sim;  // the task's simulation (read beside the task)
  int32_t pad;
};

struct BigPairBlock {  // consecutive pairs of one adaptive big cell
  int32_t task;
  int32_t first;
};

// An adaptive big cell within one outer step (two copies alternate by round).
struct BigAdapt {
  double dt_left;  // time left in the step [s]
  uint32_t u;      // substeps taken
  uint32_t done;   // 1: nothing left to do in this step
  int32_t nlive;   // live SDs at the start of the substep (set by the pre-product pass)
  uint32_t pad;
};

// Device view of a launch plan (all pointers carved from a workspace).
struct PlanDev {
  const SimDesc* desc;
  int geo;  // 1 if any member uses the geometric kernel
  CellTask* wave_tasks[kNumClasses];  // per class: plain-mode cells first, then adaptive
  // adaptive cells of each class: a second copy of their task list; each
  // step writes the next step's order into the other list (a stable
  // partition by substeps taken, most first), the lists alternating from step
  // to step; per task its group, per block of tasks a count per group
  CellTask* wave_alt[kNumClasses];
  uint32_t* order_flag[kNumClasses];
  uint32_t* order_cnt[kNumClasses];
  int n_wave[kNumClasses];
  int n_plain[kNumClasses];
  const CellTask* mid_tasks[kNumMid];  // per mid class: plain-mode cells first
  int n_mid[kNumMid];
  int n_mid_plain[kNumMid];
  const BigTask* big;
  int n_big;
  const BigChunk* chunks;
  int n_chunks;
  unsigned big_hist_bytes;  // LDS of a key block: the largest bucket count + 1 words
  const BigBucket* buckets;
  int n_buckets;
  // entries of every big cell, by chunk, grouped by bucket: (key << 32 |
  // slot), multiplicity and volume; the chunks' bucket offsets; a bucket
  // ranked in global memory (longer than the LDS stage): its keys and order
  unsigned long long* ekey;
  long long* exi;
  double* ev;
  uint32_t* offs;
  unsigned long long* skey;
  uint32_t* ord;
  // adaptive big cells: their tasks, key chunks, buckets and pair blocks;
  // per-cell state and largest p (two copies alternating by round); per
  // pair pre-products and slots
  const int* abig;
  int n_abig;
  const BigChunk* achunks;
  int n_achunks;
  const BigBucket* abuckets;
  int n_abuckets;
  const BigPairBlock* apblocks;
  int n_apblocks;
  BigAdapt* astate[2];
  unsigned long long* apmax[2];
  double* apre;
  unsigned long long* apair;
  uint32_t* aactive;  // device word: cells still stepping
};

// the plan's side streams (and fork/join events) for concurrent class launches
struct SideStream {
  hipStream_t stream = nullptr, stream2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, join2 = nullptr;
};

// launches (sdm_kernels.hip)
// Enqueues nsteps (1..kFuseMax) steps starting at launch step k_abs: the
// workgroup-per-cell classes in one launch each (several steps fused), the
// mid-size and big cells one step per launch.  flip: launches made on this
// plan since its tables were built (selects which of the two adaptive task
// lists is read).
hipError_t launch_step(const PlanDev& p, uint32_t k_abs, uint32_t flip, int nsteps,
                       int waves_per_cell, hipStream_t st, const SideStream& side);
// Diffusional growth of every live super-droplet of one simulation
// (sdm_condense.hip): one block per 256 consecutive slots.
hipError_t launch_condense(const int64_t* xi, double* v, const double* vdry, const double* kvdry,
                           const int64_t* cell_off, int n_cells, int64_t n_slots,
                           const double* temp, const double* pres, const double* sat, double dt,
                           int max_iter, hipStream_t st);
// Adaptive big cells: the start of an outer step (every cell's state
// reset), one substep round (keys, order and pre-products, pairs), and the
// count of cells still stepping after a round, into a device word.
hipError_t launch_abig_init(const PlanDev& p, uint32_t k_abs, hipStream_t st);
hipError_t launch_abig_round(const PlanDev& p, uint32_t k_abs, uint32_t round, hipStream_t st);
hipError_t launch_abig_active(const PlanDev& p, uint32_t round, uint32_t* count, hipStream_t st);
// Per-cell moments, one workgroup of `waves` (1 or 4) wavefronts per cell;
// n_bins <= kMomentsMaxBins.
hipError_t launch_moments(const SimDesc& d, int n_cells, int waves, int64_t* m0, double* m12,
                          double* attr_sums, const double* edges, int n_bins, double* spectrum,
                          hipStream_t st);
hipError_t launch_validate(const int64_t* xi, const double* v, int64_t n, uint32_t* status,
                           hipStream_t st);
hipError_t launch_philox_fill(uint32_t* out, int64_t n, uint32_t c0, uint32_t c1, uint32_t c2,
                              uint32_t c3, uint32_t k0, uint32_t k1, hipStream_t st);
hipError_t launch_kernel_values(int kind, double b, const double* v1, const double* v2, int64_t n,
                                double* out, hipStream_t st);
size_t cell_lds_bytes(int cls);
size_t mid_lds_bytes(int cls);
void set_lds_limits();

}  // namespace sdm
