// sdm_displace.hip -- super-droplet displacement in a prescribed 2D flow and
// re-segmentation of the slots by their new cell (libsdm).
//
// The PySDM v1 paper lists particle displacement among the dynamics beside
// coalescence (section "API in brief") and couples the particles to a
// prescribed single-eddy flow in its kinematic 2D example (section
// "Kinematic (prescribed-flow) examples"); it gives no scheme.  This file
// takes one explicit first-order step per call: along each axis the Courant
// number is interpolated linearly between the two faces of the droplet's cell
// at its position inside the cell, d = (1 - w) c_low + w c_high (two products
// and a sum, no contraction), w' = w + d, the cell shifts by floor(w') with
// periodic wrap, and the fraction w' - floor(w') stays (a fraction that
// rounds to 1 becomes 0 one cell up).  The slots are then re-ordered stably
// by new cell, so every cell's slots keep their old relative order (old cell,
// then old slot): the per-slot random numbers of the coalescence step are tied
// to that order.
//
// Data path (cells c = ix * nz + iz, one wavefront per cell):
//   k_disp_count    per cell, droplets leaving towards each of the 9
//                   neighbour directions (|d| < 1, so at most one cell per
//                   axis); a cell whose offsets do not fit a valid layout is
//                   marked instead
//   k_disp_offsets  per new cell: its size, and where each of its 9 source
//                   cells' droplets start (sources in old cell order); block
//                   prefix sums of the sizes; per block, whether a marked
//                   cell was seen
//   k_disp_scan     prefix over the blocks; the error word (nothing below
//                   writes if it is set)
//   k_disp_scatter  per old cell: each droplet's new slot = start of its new
//                   cell + start of its source cell there + its rank among the
//                   cell's droplets going the same way; copies xi, v, attrs and
//                   the new position
// The arithmetic of the displacement is repeated in the scatter pass rather
// than stored: it is a few flops against 16 bytes per droplet.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/sdm.h"

namespace sdm {

constexpr int kDispWaves = 4;    // cells per workgroup, one wavefront each
constexpr int kOffBlock = 256;   // new cells per block of the size prefix sum
constexpr int kScanThreads = 1024;
constexpr int kDispUnroll = 4;    // 64-slot chunks per round of loads
constexpr int kDispAttrRegs = 8;  // attributes staged in registers per slot
constexpr uint32_t kBadCell = 0xFFFFFFFFu;  // count entry of a cell with invalid offsets

struct DispState {
  int nx, nz, n_attr;
  int64_t n_slots;
  const double* cx;
  const double* cz;
  const int64_t* xi;
  const double* v;
  const double* attrs;
  const double* pos;
  const int64_t* off;
  int64_t* xi_out;
  double* v_out;
  double* attrs_out;
  double* pos_out;
  int64_t* off_out;
  uint32_t* status;
  // workspace
  uint32_t* err;        // 1 word: the offsets are not a valid layout (set by k_disp_scan)
  uint32_t* blk_err;    // [ceil(C / kOffBlock)] a block saw a marked cell
  uint32_t* cnt;        // [C][9] droplets of old cell c moving in direction d
  uint32_t* base;       // [C][9] start of source k's droplets inside new cell c
  uint32_t* local_off;  // [C] start of new cell c inside its block
  uint32_t* blk_sum;    // [ceil(C / kOffBlock)]
  int64_t* blk_off;     // [ceil(C / kOffBlock)]
};

// One axis: new fraction and cell shift (clamped to [-1, 1]); bad when the
// displacement is not below one cell or the old fraction is not in [0, 1).
static __device__ __forceinline__ double axis_step(double w, double lo, double hi, int& shift,
                                            bool& bad) {
  const double d = (1.0 - w) * lo + w * hi;
  bad = !(fabs(d) < 1.0) || !(w >= 0.0 && w < 1.0);
  const double wn = w + d;
  const double f = floor(wn);
  double frac = wn - f;
  double s = f;
  if (frac >= 1.0) {
    frac = 0.0;
    s = f + 1.0;
  }
  shift = (int)fmin(fmax(s, -1.0), 1.0);  // clamp to one cell; NaN -> -1
  return frac;
}

static __device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Along an axis of one cell a move re-enters the same cell; along an axis of
// two both directions reach the one neighbour, taken as +1.  So the groups
// (source cell, direction) that can be non-empty stay distinct for every
// destination, even where a destination's nine neighbours repeat cells.
static __device__ __forceinline__ int periodic_shift(int s, int n_axis) {
  return n_axis == 1 ? 0 : (n_axis == 2 ? (s != 0 ? 1 : 0) : s);
}

static __device__ __forceinline__ int wave_rank_below(uint64_t m, int lane) {
  return __popcll(m & ((1ull << lane) - 1ull));
}

// The droplet j of cell (ix, iz): new fractions and direction (sx + 1) * 3 + (sz + 1).
struct Move {
  double wx, wz;
  int d;
  bool bad;
};

static __device__ __forceinline__ Move move_of(const DispState& S, int64_t j, double cxl, double cxh,
                                        double czl, double czh) {
  Move m;
  int sx, sz;
  bool bx, bz;
  m.wx = axis_step(S.pos[j], cxl, cxh, sx, bx);
  m.wz = axis_step(S.pos[S.n_slots + j], czl, czh, sz, bz);
  sx = periodic_shift(sx, S.nx);
  sz = periodic_shift(sz, S.nz);
  m.d = (sx + 1) * 3 + (sz + 1);
  m.bad = bx || bz;
  return m;
}

__global__ void __launch_bounds__(64 * kDispWaves) k_disp_count(DispState S) {
  const int C = S.nx * S.nz;
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * kDispWaves + (threadIdx.x >> 6);
  if (c >= C) return;  // uniform over the wavefront
  const int ix = c / S.nz, iz = c - ix * S.nz;
  const int64_t a = S.off[c], b = S.off[c + 1];
  const double cxl = S.cx[ix * S.nz + iz], cxh = S.cx[(ix + 1) * S.nz + iz];
  const double czl = S.cz[ix * (S.nz + 1) + iz], czh = S.cz[ix * (S.nz + 1) + iz + 1];
  // every cell checks its own offsets: together they check the whole layout
  const bool valid = a >= 0 && a <= b && b <= S.n_slots && (c != 0 || a == 0) &&
                     (c != C - 1 || b == S.n_slots);
  if (!valid) {
    if (lane < 9) S.cnt[(int64_t)c * 9 + lane] = kBadCell;
    if (lane == 0) atomicOr(S.status, (uint32_t)SDM_FLAG_INVALID_STATE);
    return;
  }
  uint32_t mine = 0;  // lane d < 9: droplets moving in direction d
  bool bad = false;
  for (int64_t j0 = a; j0 < b; j0 += 64 * kDispUnroll) {
    int dir[kDispUnroll];
#pragma unroll
    for (int u = 0; u < kDispUnroll; ++u) {  // the chunks' loads in flight together
      const int64_t j = j0 + 64 * u + lane;
      dir[u] = -1;
      if (j < b) {
        const Move m = move_of(S, j, cxl, cxh, czl, czh);
        dir[u] = m.d;
        bad = bad || m.bad;
      }
    }
#pragma unroll
    for (int u = 0; u < kDispUnroll; ++u)
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const uint64_t bm = __ballot(dir[u] == q);
        if (lane == q) mine += (uint32_t)__popcll(bm);
      }
  }
  if (lane < 9) S.cnt[(int64_t)c * 9 + lane] = mine;
  if (__any(bad) && lane == 0) atomicOr(S.status, (uint32_t)SDM_FLAG_COURANT);
}

// Source k of new cell (ix, iz) sits at offset (k / 3 - 1, k % 3 - 1); its
// droplets reach the cell by moving in direction 8 - k.  Sources are placed
// in old cell order.  Along an axis of one or two cells several k name the
// same cell; of those only one group can hold droplets (periodic_shift), and
// a source's start counts strictly smaller cells only, so it is the same.
__global__ void __launch_bounds__(kOffBlock) k_disp_offsets(DispState S) {
  const int C = S.nx * S.nz;
  const int c = blockIdx.x * kOffBlock + threadIdx.x;
  uint32_t total = 0;
  bool marked = false;
  if (c < C) {
    const int ix = c / S.nz, iz = c - ix * S.nz;
    int src[9];
    uint32_t n[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int jx = wrap(ix + k / 3 - 1, S.nx), jz = wrap(iz + k % 3 - 1, S.nz);
      src[k] = jx * S.nz + jz;
      n[k] = S.cnt[(int64_t)src[k] * 9 + (8 - k)];
      marked = marked || n[k] == kBadCell;  // the cell itself is source k = 4
      total += n[k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      uint32_t before = 0;
#pragma unroll
      for (int k2 = 0; k2 < 9; ++k2) before += src[k2] < src[k] ? n[k2] : 0u;
      S.base[(int64_t)c * 9 + k] = before;
    }
  }
  // exclusive prefix of the new sizes inside the block
  __shared__ uint32_t sh[kOffBlock];
  sh[threadIdx.x] = total;
  __syncthreads();
  for (int o = 1; o < kOffBlock; o <<= 1) {
    const uint32_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0u;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  if (c < C) S.local_off[c] = sh[threadIdx.x] - total;
  if (threadIdx.x == kOffBlock - 1) S.blk_sum[blockIdx.x] = sh[threadIdx.x];
  const int any = __syncthreads_or(marked ? 1 : 0);
  if (threadIdx.x == 0) S.blk_err[blockIdx.x] = any ? 1u : 0u;
}

// One workgroup: exclusive prefix over the block sums; the new n_slots end.
__global__ void __launch_bounds__(kScanThreads) k_disp_scan(DispState S, int nblk) {
  __shared__ int64_t sh[kScanThreads];
  int64_t carry = 0;
  int bad = 0;
  for (int b0 = 0; b0 < nblk; b0 += kScanThreads) {
    const int b = b0 + threadIdx.x;
    if (b < nblk && S.blk_err[b]) bad = 1;
    const int64_t x = b < nblk ? (int64_t)S.blk_sum[b] : 0;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
      const int64_t add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (b < nblk) S.blk_off[b] = carry + sh[threadIdx.x] - x;
    carry += sh[kScanThreads - 1];
    __syncthreads();
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    *S.err = bad ? 1u : 0u;  // read by k_disp_scatter, the next kernel
    if (!bad) S.off_out[S.nx * S.nz] = carry;
  }
}

__global__ void __launch_bounds__(64 * kDispWaves) k_disp_scatter(DispState S) {
  const int C = S.nx * S.nz;
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * kDispWaves + (threadIdx.x >> 6);
  if (c >= C) return;  // uniform over the wavefront
  const uint32_t err = *S.err;
  const int ix = c / S.nz, iz = c - ix * S.nz;
  const int64_t a = S.off[c], b = S.off[c + 1];
  const double cxl = S.cx[ix * S.nz + iz], cxh = S.cx[(ix + 1) * S.nz + iz];
  const double czl = S.cz[ix * (S.nz + 1) + iz], czh = S.cz[ix * (S.nz + 1) + iz + 1];
  if (err) return;
  if (lane == 0) S.off_out[c] = S.blk_off[c / kOffBlock] + S.local_off[c];
  // lane q < 9: next free slot of direction q (its new cell's start, plus
  // this cell's start inside it, plus the droplets already placed)
  int64_t next = 0;
  if (lane < 9) {
    const int jx = wrap(ix + lane / 3 - 1, S.nx), jz = wrap(iz + lane % 3 - 1, S.nz);
    const int t = jx * S.nz + jz;
    next = S.blk_off[t / kOffBlock] + (int64_t)S.local_off[t] + S.base[(int64_t)t * 9 + (8 - lane)];
  }
  const int64_t n = S.n_slots;
  const int A = S.n_attr;
  // kDispUnroll chunks of 64 slots per round: every load of the round is
  // issued before the first store (the bandwidth comes from loads in flight)
  for (int64_t j0 = a; j0 < b; j0 += 64 * kDispUnroll) {
    long long xr[kDispUnroll];
    double vr[kDispUnroll];
    double ar[kDispUnroll][kDispAttrRegs];
    Move mr[kDispUnroll];
#pragma unroll
    for (int u = 0; u < kDispUnroll; ++u) {
      const int64_t j = j0 + 64 * u + lane;
      mr[u] = Move{0.0, 0.0, -1, false};
      xr[u] = 0;
      vr[u] = 0.0;
      if (j < b) {
        xr[u] = S.xi[j];
        vr[u] = S.v[j];
#pragma unroll
        for (int e = 0; e < kDispAttrRegs; ++e)
          if (e < A) ar[u][e] = S.attrs[(int64_t)e * n + j];
        mr[u] = move_of(S, j, cxl, cxh, czl, czh);
      }
    }
#pragma unroll
    for (int u = 0; u < kDispUnroll; ++u) {
      const int64_t j = j0 + 64 * u + lane;
      const bool on = j < b;
      const Move m = mr[u];
      int rank = 0;  // among this chunk's droplets going the same way
      uint32_t adv = 0;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const uint64_t bm = __ballot(m.d == q);
        if (m.d == q) rank = wave_rank_below(bm, lane);
        if (lane == q) adv = (uint32_t)__popcll(bm);
      }
      const long long start = __shfl((long long)next, on ? m.d : 0);
      next += adv;
      if (on) {
        const int64_t dst = start + rank;
        S.xi_out[dst] = xr[u];
        S.v_out[dst] = vr[u];
        S.pos_out[dst] = m.wx;
        S.pos_out[n + dst] = m.wz;
#pragma unroll
        for (int e = 0; e < kDispAttrRegs; ++e)
          if (e < A) S.attrs_out[(int64_t)e * n + dst] = ar[u][e];
        for (int q = kDispAttrRegs; q < A; ++q)  // attributes beyond the staged ones
          S.attrs_out[(int64_t)q * n + dst] = S.attrs[(int64_t)q * n + j];
      }
    }
  }
}

}  // namespace sdm

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

using sdm::kDispWaves;
using sdm::kOffBlock;
using sdm::kScanThreads;
constexpr size_t kAlignD = 256;
constexpr size_t up(size_t x) { return (x + kAlignD - 1) / kAlignD * kAlignD; }

constexpr size_t ws_bytes(int64_t C) {
  const int64_t nblk = (C + kOffBlock - 1) / kOffBlock;
  return up(sizeof(uint32_t)) + 2 * up(sizeof(uint32_t) * 9 * (size_t)C) +
         up(sizeof(uint32_t) * (size_t)C) + 2 * up(sizeof(uint32_t) * (size_t)nblk) +
         up(sizeof(int64_t) * (size_t)nblk);
}


bool disjoint(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return na == 0 || nb == 0 || x + na <= y || y + nb <= x;
}

// Argument checks shared by both entry points; returns SDM_OK or the error.
sdm_status check_args(const sdm_displace_args* g) {
  if (!g || g->nx < 1 || g->nz < 1 || (int64_t)g->nx * g->nz > (int64_t)0x7FFFFFFF / 9 ||
      g->n_attr < 0 || g->n_attr > 16 || g->reserved != 0 || g->n_slots < 0 ||
      g->n_slots >= 0xFFFFFFFFLL)
    return SDM_EINVAL;
  const int64_t C = (int64_t)g->nx * g->nz, n = g->n_slots, A = g->n_attr;
  if (!g->courant_x || !g->courant_z || !g->cell_off || !g->cell_off_out || !g->status)
    return SDM_EINVAL;
  if (n > 0 && (!g->xi || !g->v || !g->pos || !g->xi_out || !g->v_out || !g->pos_out))
    return SDM_EINVAL;
  if (n > 0 && A > 0 && (!g->attrs || !g->attrs_out)) return SDM_EINVAL;
  // outputs must not overlap the inputs (the pass reads and writes in one go)
  const void* ins[5] = {g->xi, g->v, g->attrs, g->pos, g->cell_off};
  const size_t nin[5] = {8 * (size_t)n, 8 * (size_t)n, 8 * (size_t)(A * n), 16 * (size_t)n,
                         8 * (size_t)(C + 1)};
  const void* outs[5] = {g->xi_out, g->v_out, g->attrs_out, g->pos_out, g->cell_off_out};
  for (int i = 0; i < 5; ++i)
    for (int k = 0; k < 5; ++k)
      if (ins[i] && outs[k] && !disjoint(ins[i], nin[i], outs[k], nin[k])) return SDM_EINVAL;
  return SDM_OK;
}

// The four kernels of one call over the workspace at w (ws_bytes(C) bytes,
// every word written before it is read, so it needs no clearing).
sdm_status launch_displace(const sdm_displace_args* g, char* w, hipStream_t st) {
  const int64_t C = (int64_t)g->nx * g->nz, n = g->n_slots;
  sdm::DispState S{};
  S.nx = g->nx;
  S.nz = g->nz;
  S.n_attr = g->n_attr;
  S.n_slots = n;
  S.cx = g->courant_x;
  S.cz = g->courant_z;
  S.xi = g->xi;
  S.v = g->v;
  S.attrs = g->attrs;
  S.pos = g->pos;
  S.off = g->cell_off;
  S.xi_out = g->xi_out;
  S.v_out = g->v_out;
  S.attrs_out = g->attrs_out;
  S.pos_out = g->pos_out;
  S.off_out = g->cell_off_out;
  S.status = g->status;
  const int64_t nblk = (C + kOffBlock - 1) / kOffBlock;
  S.err = reinterpret_cast<uint32_t*>(w);
  w += up(sizeof(uint32_t));
  S.cnt = reinterpret_cast<uint32_t*>(w);
  w += up(sizeof(uint32_t) * 9 * (size_t)C);
  S.base = reinterpret_cast<uint32_t*>(w);
  w += up(sizeof(uint32_t) * 9 * (size_t)C);
  S.local_off = reinterpret_cast<uint32_t*>(w);
  w += up(sizeof(uint32_t) * (size_t)C);
  S.blk_sum = reinterpret_cast<uint32_t*>(w);
  w += up(sizeof(uint32_t) * (size_t)nblk);
  S.blk_err = reinterpret_cast<uint32_t*>(w);
  w += up(sizeof(uint32_t) * (size_t)nblk);
  S.blk_off = reinterpret_cast<int64_t*>(w);

  const unsigned cells_grid = (unsigned)((C + kDispWaves - 1) / kDispWaves);
  hipLaunchKernelGGL(sdm::k_disp_count, dim3(cells_grid), dim3(64 * kDispWaves), 0, st, S);
  hipLaunchKernelGGL(sdm::k_disp_offsets, dim3((unsigned)nblk), dim3(kOffBlock), 0, st, S);
  hipLaunchKernelGGL(sdm::k_disp_scan, dim3(1), dim3(kScanThreads), 0, st, S, (int)nblk);
  hipLaunchKernelGGL(sdm::k_disp_scatter, dim3(cells_grid), dim3(64 * kDispWaves), 0, st, S);
  return hipGetLastError() == hipSuccess ? SDM_OK : SDM_EDEVICE;
}

// Scratch of the allocation-free entry point: the workspace of a domain of up
// to kScratchCells cells, in a file-scope device array.  Each GPU the library
// runs on holds its own copy until the process ends; every call on one GPU
// reuses it, so calls that overlap on one GPU race.  Host code never passes
// the array's name to a kernel (in host code it only stands for the symbol):
// its device address, per device, comes from hipGetSymbolAddress.
constexpr int64_t kScratchCells = int64_t(1) << 17;
constexpr size_t kScratchBytes = ws_bytes(kScratchCells);  // 9.5 MiB
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// the current device's address of `scratch` (looked up once per device)
char* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

size_t sdm_displace_workspace_bytes(int32_t nx, int32_t nz) {
  if (nx < 1 || nz < 1 || (int64_t)nx * nz > (int64_t)0x7FFFFFFF / 9) return 0;
  return ws_bytes((int64_t)nx * nz);
}

sdm_status sdm_displace(const sdm_displace_args* g, void* workspace, size_t workspace_bytes,
                        void* stream) {
  const sdm_status r = check_args(g);
  if (r != SDM_OK) return r;
  const int64_t C = (int64_t)g->nx * g->nz;
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % kAlignD) return SDM_EINVAL;
  if (workspace_bytes < ws_bytes(C)) return SDM_ENOMEM;
  return launch_displace(g, static_cast<char*>(workspace), reinterpret_cast<hipStream_t>(stream));
}

sdm_status sdm_displace_noalloc(const sdm_displace_args* g, void* stream) {
  const sdm_status r = check_args(g);
  if (r != SDM_OK) return r;
  const int64_t C = (int64_t)g->nx * g->nz;
  if (C > kScratchCells) return SDM_ENOMEM;  // ws_bytes grows with C: it fits
  char* w = scratch_address();
  if (!w) return SDM_EDEVICE;
  return launch_displace(g, w, reinterpret_cast<hipStream_t>(stream));
}

int64_t sdm_displace_noalloc_max_cells(void) { return kScratchCells; }

}  // extern "C"
