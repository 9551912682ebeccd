// sdm_refresh.hip -- device-side refresh of a launch plan after the cell
// layout changed (for instance after displacement and re-segmentation).
//
// A plan lists, per workgroup-per-cell class, one task per populated cell:
// the cell's first slot in xi and v and its size.  When only the layout
// changes (same cells, same number of slots, new offsets and new state
// buffers) and every cell still fits the class its task is in, the tables
// stay valid once each task's pointers and size are rewritten, which takes
// one small kernel per list instead of a host-side re-plan.  The host checks
// the two result words and re-plans on the host otherwise.
#include "sdm_refresh.hpp"

namespace sdm {

constexpr int kRefreshBlock = 256;

__global__ void __launch_bounds__(64) k_refresh_zero(unsigned long long* w) {
  if (threadIdx.x < 2) w[threadIdx.x] = 0ull;
}

__global__ void __launch_bounds__(kRefreshBlock) k_refresh_check(const int64_t* off, int C,
                                                                 int64_t n,
                                                                 unsigned long long* w) {
  const int c = blockIdx.x * kRefreshBlock + threadIdx.x;
  if (c > C) return;
  const int64_t a = off[c];
  bool bad = (c == 0 && a != 0) || (c == C && a != n) || (c < C && off[c + 1] < a);
  if (bad) atomicOr(&w[0], 1ull);
}

// count: add the new sizes to w[1] (only for the primary list of a class,
// so that cells listed twice count once)
__global__ void __launch_bounds__(kRefreshBlock) k_refresh_tasks(CellTask* list, int nt, int cap,
                                                                 const int64_t* off, int C,
                                                                 int64_t n_slots, int64_t* xi,
                                                                 double* v, unsigned long long* w,
                                                                 int count) {
  const int i = blockIdx.x * kRefreshBlock + threadIdx.x;
  unsigned long long size = 0;
  if (i < nt) {
    CellTask t = list[i];
    if (t.cell >= 0 && t.cell < C) {
      const int64_t a = off[t.cell], b = off[t.cell + 1];
      // a cell that grew past its class, or offsets out of range (the check
      // kernel flags those too): the host re-plans, these tasks are not used
      if (b - a > cap || a < 0 || b > n_slots || b < a) {
        atomicOr(&w[0], 2ull);
      } else {
        t.xi = xi + a;
        t.v = v + a;
        t.n = (int32_t)(b - a);
        list[i] = t;
        size = (unsigned long long)(b - a);
      }
    } else {
      atomicOr(&w[0], 2ull);
    }
  }
  if (!count) return;
  // workgroup sum, one atomic per workgroup
  __shared__ unsigned long long part[kRefreshBlock / 64];
  for (int o = 32; o > 0; o >>= 1) size += __shfl_down(size, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = size;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int k = 0; k < kRefreshBlock / 64; ++k) s += part[k];
    if (s) atomicAdd(&w[1], s);
  }
}

hipError_t launch_refresh(const PlanDev& p, const int64_t* off, int n_cells, int64_t n_slots,
                          int64_t* xi, double* v, unsigned long long* w, hipStream_t st) {
  const int C = n_cells;
  hipLaunchKernelGGL(k_refresh_zero, dim3(1), dim3(64), 0, st, w);
  hipLaunchKernelGGL(k_refresh_check, dim3((unsigned)((C + kRefreshBlock) / kRefreshBlock)),
                     dim3(kRefreshBlock), 0, st, off, C, n_slots, w);
  for (int k = 0; k < kNumClasses; ++k) {
    const int cap = class_cap(k);
    const int nw = p.n_wave[k], na = p.n_wave[k] - p.n_plain[k];
    const unsigned gw = (unsigned)((nw + kRefreshBlock - 1) / kRefreshBlock);
    const unsigned ga = (unsigned)((na + kRefreshBlock - 1) / kRefreshBlock);
    if (nw > 0)
      hipLaunchKernelGGL(k_refresh_tasks, dim3(gw), dim3(kRefreshBlock), 0, st, p.wave_tasks[k],
                         nw, cap, off, C, n_slots, xi, v, w, 1);
    if (na > 0)
      hipLaunchKernelGGL(k_refresh_tasks, dim3(ga), dim3(kRefreshBlock), 0, st, p.wave_alt[k], na,
                         cap, off, C, n_slots, xi, v, w, 0);
  }
  return hipGetLastError();
}

}  // namespace sdm
