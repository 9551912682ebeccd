// sdm_kernels.hip -- gfx950 kernels of the SDM collision-coalescence step.
//
// One outer step of one cell (Shima et al. 2009, the method the PySDM v1
// paper names as its core, "Introduction"; box set-up of "API in brief"):
//   1. live SDs (xi > 0) of the cell, n of them; nothing happens if n < 2;
//   2. a 32-bit key per live cell-local slot j: word (j mod 4) of
//      Philox4x32-10(counter = (j/4, cell, step, 2 substep), key = seed);
//   3. the live slots ordered by (key, slot);
//   4. candidate pairs (l_2m, l_2m+1), m < floor(n/2); an odd last SD idles;
//   5. p = ((max(xi_a, xi_b) K(v_a, v_b)) S) dt/dV with S = n(n-1)/2 / floor(n/2);
//   6. gamma = floor(p) + [phi < p - floor(p)], phi = 53-bit uniform from
//      words 2(m mod 2), 2(m mod 2)+1 of Philox((m/2, cell, step, 2 substep + 1));
//   7. g = min(gamma, floor(xi_j / xi_k)) (j = larger xi, ties to the first
//      member); either xi_j -= g xi_k and X_k = fma(g, X_j, X_k), or, when
//      xi_j is used up exactly, the equal split xi_j = floor(xi_k / 2),
//      xi_k -= that, X_j = X_k = fma(g, X_j, X_k), for X in {v, attributes}.
// Adaptive mode repeats 2-7 with substeps whose length keeps every p <= 1.
//
// Work mapping.  Cells of <= 512 slots: one wavefront per cell, everything in
// LDS (the sort is a one-pass bucket scatter on the top ceil(log2 n) key bits
// followed by an exact rank inside each bucket, both by the same wave), one
// launch per capacity class covering all cells of all simulations of a plan.
// Larger cells: global bucket counts, scan, scatter, per-bucket rank by one
// wave in LDS, then a pair kernel over the global order.
//
// Floating point: fp64 throughout, built with -ffp-contract=off; the only
// fused operation is the explicit fma of the update.

#include "sdm_internal.hpp"

namespace sdm {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011): 10 rounds of two 32x32
// multiplies (0xD2511F53, 0xCD9E8D57) with a Weyl key schedule
// (0x9E3779B9, 0xBB67AE85).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 x, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * x.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, x.x);
    const uint32_t lo1 = 0xCD9E8D57u * x.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x.z);
    x = make_uint4(hi1 ^ x.y ^ k0, lo1, hi0 ^ x.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return x;
}

// 53-bit uniform in [0, 1) from the high and low words
__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
  const unsigned long long bits = ((unsigned long long)hi << 32) | lo;
  return (double)(bits >> 11) * 0x1p-53;
}

// ---------------------------------------------------------------------------
// Collision kernels
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;
constexpr double kVolToR3 = 3.0 / (4.0 * kPi);  // r^3 = 3 v / (4 pi)
// terminal velocity regimes (Rogers & Yau 1989): u = min(k1 r^2, k2 r, k3 sqrt r)
constexpr double kU1 = 1.19e8;
constexpr double kU2 = 8.0e3;
constexpr double kU3 = 201.0;

__device__ __forceinline__ double fall_speed(double r) {
  const double u1 = kU1 * r * r;
  const double u2 = kU2 * r;
  const double u3 = kU3 * sqrt(r);
  return fmin(fmin(u1, u2), u3);
}

__device__ __forceinline__ double coal_kernel(int kind, double b, double va, double vb) {
  if (kind == 0) return b * (va + vb);  // Golovin additive kernel
  const double ra = cbrt(kVolToR3 * va);
  const double rb = cbrt(kVolToR3 * vb);
  const double rs = ra + rb;
  return kPi * (rs * rs) * fabs(fall_speed(ra) - fall_speed(rb));  // geometric sweep-out, E = 1
}

__device__ __forceinline__ long long collisions(double p, double phi, uint32_t* status) {
  if (!(p < 0x1p62)) {
    atomicOr(status, kFlagGammaCap);
    return 1LL << 62;
  }
  const double f = floor(p);
  return (long long)f + (phi < p - f ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
  return x;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x = fmax(x, __shfl_xor(x, d, 64));
  return x;
}

// exclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_excl_scan(int x, int lane) {
  int inc = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  return inc - x;
}

__device__ __forceinline__ void add_stats(unsigned long long* stats, unsigned long long live,
                                          unsigned long long coll, unsigned long long substeps) {
  unsigned long long* s = stats + (blockIdx.x % kStatSlots) * kStatFields;
  if (live) atomicAdd(s + 0, live);
  if (coll) atomicAdd(s + 1, coll);
  if (substeps) atomicAdd(s + 2, substeps);
  atomicAdd(s + 3, 1ull);
}

// ---------------------------------------------------------------------------
// Update of one colliding pair.  ia/ib index xs/vs (LDS or global) and ga/gb
// the global slots of the attributes.
// ---------------------------------------------------------------------------
template <typename XI, typename VV>
__device__ __forceinline__ void update_pair(XI* xs, VV* vs, int ia, int ib, long long xa,
                                            long long xb, double va, double vb, long long gamma,
                                            double* attrs, int64_t n_slots, int n_attr,
                                            int64_t ga, int64_t gb) {
  const bool a_is_j = xa >= xb;
  const int ij = a_is_j ? ia : ib, ik = a_is_j ? ib : ia;
  const int64_t gj = a_is_j ? ga : gb, gk = a_is_j ? gb : ga;
  const long long xj = a_is_j ? xa : xb, xk = a_is_j ? xb : xa;
  const double vj = a_is_j ? va : vb, vk = a_is_j ? vb : va;
  long long g = gamma;
  if (g > 1) {
    const long long ratio = xj / xk;
    g = g < ratio ? g : ratio;
  }
  const double gd = (double)g;
  const long long rest = xj - g * xk;
  if (rest > 0) {
    xs[ij] = rest;
    vs[ik] = fma(gd, vj, vk);
    for (int q = 0; q < n_attr; ++q) {
      double* a = attrs + (int64_t)q * n_slots;
      a[gk] = fma(gd, a[gj], a[gk]);
    }
  } else {  // equal-multiplicity split
    const long long h = xk >> 1;
    xs[ij] = h;
    xs[ik] = xk - h;
    const double t = fma(gd, vj, vk);
    vs[ij] = t;
    vs[ik] = t;
    for (int q = 0; q < n_attr; ++q) {
      double* a = attrs + (int64_t)q * n_slots;
      const double ta = fma(gd, a[gj], a[gk]);
      a[gj] = ta;
      a[gk] = ta;
    }
  }
}

// ---------------------------------------------------------------------------
// One wavefront per cell (cells of <= CAP slots).
// ---------------------------------------------------------------------------
template <int CAP>
struct WaveLds {
  long long xs[CAP];  // multiplicities of the cell (slot order)
  double vs[CAP];     // volumes (slot order)
  uint32_t keys[CAP];
  uint32_t tmp[CAP];  // bucketed (key << nbits | slot); reused for pair pre-products
  uint32_t cnt[CAP + 4];
  uint16_t ord[CAP];  // live slots in permuted order
  uint8_t dirty[CAP];
};

// keys, bucket count, scan, scatter, rank: L.ord[0..nlive) = permutation
template <int CAP>
__device__ __forceinline__ void wave_sort(WaveLds<CAP>& L, int n, int nlive, int lane, int c,
                                          uint32_t s, uint32_t u, uint32_t k0, uint32_t k1) {
  constexpr int IT = CAP / 64;
  for (int g0 = 0; 4 * g0 < n; g0 += 64) {
    const int g = g0 + lane;
    if (4 * g < n) {
      const uint4 w = philox(make_uint4((uint32_t)g, (uint32_t)c, s, 2u * u), k0, k1);
      *reinterpret_cast<uint4*>(&L.keys[4 * g]) = w;
    }
  }
  const int nbits = 32 - __clz(n - 1);  // n >= 2
  const int nb = 1 << nbits;
  for (int i = lane; i <= nb; i += 64) L.cnt[i] = 0;
  wave_sync();

  uint32_t kr[IT], pos[IT];
  bool lv[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = it * 64 + lane;
    lv[it] = false;
    if (it * 64 < n) {
      lv[it] = j < n && L.xs[j] > 0;
      if (lv[it]) {
        kr[it] = L.keys[j];
        pos[it] = atomicAdd(&L.cnt[kr[it] >> (32 - nbits)], 1u);
      }
    }
  }
  wave_sync();
  {  // exclusive scan of the nb bucket counts
    const int per = nb >= 64 ? nb / 64 : 1;
    const int first = lane * per;
    int local = 0;
    if (first < nb)
      for (int i = 0; i < per; ++i) local += (int)L.cnt[first + i];
    int run = wave_excl_scan(local, lane);
    if (first < nb)
      for (int i = 0; i < per; ++i) {
        const int cv = (int)L.cnt[first + i];
        L.cnt[first + i] = (uint32_t)run;
        run += cv;
      }
    if (lane == 0) L.cnt[nb] = (uint32_t)nlive;
  }
  wave_sync();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    if (lv[it]) {
      const int j = it * 64 + lane;
      L.tmp[L.cnt[kr[it] >> (32 - nbits)] + pos[it]] = (kr[it] << nbits) | (uint32_t)j;
    }
  }
  wave_sync();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    if (lv[it]) {
      const int j = it * 64 + lane;
      const uint32_t b = kr[it] >> (32 - nbits);
      const int st = (int)L.cnt[b], en = (int)L.cnt[b + 1];
      const uint32_t me = (kr[it] << nbits) | (uint32_t)j;
      int r = st;
      for (int qq = st; qq < en; ++qq) r += (L.tmp[qq] < me) ? 1 : 0;
      L.ord[r] = (uint16_t)j;
    }
  }
  wave_sync();
}

enum PassMode { kPassPlain = 0, kPassPmax = 1, kPassAdapt = 2 };

// Candidate pairs of one (sub)step.  kPassPlain updates global memory;
// kPassPmax stores the pre-products (max xi K) S and returns the largest p at
// q; kPassAdapt reads them back, clamps p to 1 if asked and updates LDS.
template <int CAP, int MODE>
__device__ __forceinline__ double wave_pairs(WaveLds<CAP>& L, const SimDesc* dp, int n, int nlive,
                                             int lane, int c, uint32_t s, uint32_t u, double q,
                                             bool clamp, int64_t o0, int* ncoll) {
  const int P = nlive >> 1;
  const double S = (double)((nlive & 1) ? nlive : nlive - 1);
  double* pre = reinterpret_cast<double*>(L.tmp);  // CAP/2 doubles fit in tmp
  double pmax = 0.0;
  const int kind = dp->kernel;
  const double bgol = dp->b;
  int64_t* sink = (MODE == kPassPmax) ? nullptr : dp->sink;
  int64_t sink_base = 0;
  if (sink) sink_base = 2 * dp->pair_base[c];
  for (int h0 = 0; 2 * h0 < P; h0 += 64) {
    const int h = h0 + lane;
    if (2 * h >= P) continue;
    uint4 w = make_uint4(0, 0, 0, 0);
    if (MODE != kPassPmax) w = philox(make_uint4((uint32_t)h, (uint32_t)c, s, 2u * u + 1u),
                                      dp->seed_lo, dp->seed_hi);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int m = 2 * h + e;
      if (m >= P) break;
      const int a = L.ord[2 * m], bb = L.ord[2 * m + 1];
      const long long xa = L.xs[a], xb = L.xs[bb];
      const double va = L.vs[a], vb = L.vs[bb];
      double p;
      if (MODE == kPassAdapt) {
        p = pre[m] * q;
      } else {
        const double kv = coal_kernel(kind, bgol, va, vb);
        const double pp = ((double)(xa > xb ? xa : xb) * kv) * S;
        if (MODE == kPassPmax) {
          pre[m] = pp;
          pmax = fmax(pmax, pp * q);
          continue;
        }
        p = pp * q;
      }
      if (clamp && p > 1.0) p = 1.0;
      const double phi = e == 0 ? uniform53(w.x, w.y) : uniform53(w.z, w.w);
      const long long gamma = collisions(p, phi, dp->status);
      if (sink) {
        sink[sink_base + 2 * m] = (int64_t)((uint64_t)a | ((uint64_t)bb << 32));
        sink[sink_base + 2 * m + 1] = gamma;
      }
      if (gamma > 0) {
        *ncoll += 1;
        if (MODE == kPassPlain) {
          update_pair(dp->xi + o0, dp->v + o0, a, bb, xa, xb, va, vb, gamma, dp->attrs,
                      dp->n_slots, dp->n_attr, o0 + a, o0 + bb);
        } else {
          update_pair(L.xs, L.vs, a, bb, xa, xb, va, vb, gamma, dp->attrs, dp->n_slots,
                      dp->n_attr, o0 + a, o0 + bb);
          L.dirty[a] = 1;
          L.dirty[bb] = 1;
        }
      }
    }
  }
  if (sink && MODE != kPassPmax) {  // unused pair entries of the cell
    for (int m = P + lane; m < (n >> 1); m += 64) {
      sink[sink_base + 2 * m] = -1;
      sink[sink_base + 2 * m + 1] = -1;
    }
  }
  wave_sync();
  return pmax;
}

template <int CAP>
__device__ __forceinline__ int wave_count_live(WaveLds<CAP>& L, int n, int lane) {
  int nl = 0;
  for (int base = 0; base < n; base += 64) {
    const int j = base + lane;
    nl += __popcll(__ballot(j < n && L.xs[j] > 0));
  }
  return nl;
}

template <int CAP>
__global__ void __launch_bounds__(512) k_wave_cells(const SimDesc* __restrict__ descs,
                                                    const int2* __restrict__ tasks, int n_tasks,
                                                    uint32_t k_abs) {
  constexpr int IT = CAP / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int t = blockIdx.x * (blockDim.x >> 6) + wv;
  if (t >= n_tasks) return;
  WaveLds<CAP>& L = reinterpret_cast<WaveLds<CAP>*>(smem)[wv];
  const int2 task = tasks[t];
  const int sim = __builtin_amdgcn_readfirstlane(task.x);
  const int c = __builtin_amdgcn_readfirstlane(task.y);
  const SimDesc* dp = descs + sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  const int64_t o0 = dp->cell_off[c];
  const int n = (int)(dp->cell_off[c + 1] - o0);
  const int64_t* gxi = dp->xi + o0;
  const double* gv = dp->v + o0;

  // stage the cell: all loads first, then the LDS stores
  long long xr[IT];
  double vr[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = it * 64 + lane;
    xr[it] = 0;
    vr[it] = 0.0;
    if (it * 64 < n && j < n) {
      xr[it] = gxi[j];
      vr[it] = gv[j];
    }
  }
  int nlive = 0;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    if (it * 64 < n) {
      const int j = it * 64 + lane;
      if (j < n) {
        L.xs[j] = xr[it];
        L.vs[j] = vr[it];
        L.dirty[j] = 0;
      }
      nlive += __popcll(__ballot(j < n && xr[it] > 0));
    }
  }
  wave_sync();

  int ncoll = 0;
  int nsub = 1;
  if (!dp->adaptive) {
    if (nlive >= 2) {
      wave_sort(L, n, nlive, lane, c, s, 0u, dp->seed_lo, dp->seed_hi);
      wave_pairs<CAP, kPassPlain>(L, dp, n, nlive, lane, c, s, 0u, dp->q, false, o0, &ncoll);
    } else if (dp->sink) {
      const int64_t base = 2 * dp->pair_base[c];
      for (int m = lane; m < (n >> 1); m += 64) {
        dp->sink[base + 2 * m] = -1;
        dp->sink[base + 2 * m + 1] = -1;
      }
    }
  } else {
    // per-cell substepping: every p <= 1 (clamped), so gamma <= 1
    const double dv = dp->dv;
    double dt_left = dp->dt;
    uint32_t u = 0;
    int nl = nlive;
    const uint32_t umax = (uint32_t)dp->max_substeps;
    while (dt_left > 0.0 && u < umax) {
      if (u > 0) nl = wave_count_live(L, n, lane);
      if (nl < 2) break;
      wave_sort(L, n, nl, lane, c, s, u, dp->seed_lo, dp->seed_hi);
      double pmax = wave_pairs<CAP, kPassPmax>(L, dp, n, nl, lane, c, s, u, dt_left / dv, false,
                                               o0, &ncoll);
      pmax = wave_max(pmax);
      const double dt_sub = (pmax <= 1.0) ? dt_left : dt_left / pmax;
      wave_pairs<CAP, kPassAdapt>(L, dp, n, nl, lane, c, s, u, dt_sub / dv, true, o0, &ncoll);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");  // attribute stores before next reads
      dt_left = (dt_sub == dt_left) ? 0.0 : dt_left - dt_sub;
      u += 1;
    }
    if (dt_left > 0.0 && u >= umax) {  // cap: the rest in one unclamped substep
      if (lane == 0) atomicOr(dp->status, kFlagSubstepCap);
      nl = wave_count_live(L, n, lane);
      if (nl >= 2) {
        wave_sort(L, n, nl, lane, c, s, u, dp->seed_lo, dp->seed_hi);
        wave_pairs<CAP, kPassPmax>(L, dp, n, nl, lane, c, s, u, dt_left / dv, false, o0, &ncoll);
        wave_pairs<CAP, kPassAdapt>(L, dp, n, nl, lane, c, s, u, dt_left / dv, false, o0,
                                    &ncoll);
      } else if (dp->sink) {
        const int64_t base = 2 * dp->pair_base[c];
        for (int m = lane; m < (n >> 1); m += 64) {
          dp->sink[base + 2 * m] = -1;
          dp->sink[base + 2 * m + 1] = -1;
        }
      }
      u += 1;
    }
    if (u == 0 && dp->sink) {
      const int64_t base = 2 * dp->pair_base[c];
      for (int m = lane; m < (n >> 1); m += 64) {
        dp->sink[base + 2 * m] = -1;
        dp->sink[base + 2 * m + 1] = -1;
      }
    }
    nsub = (int)u;
    // write back the slots that changed
    int64_t* wxi = dp->xi + o0;
    double* wv2 = dp->v + o0;
    for (int j = lane; j < n; j += 64) {
      if (L.dirty[j]) {
        wxi[j] = L.xs[j];
        wv2[j] = L.vs[j];
      }
    }
  }
  ncoll = wave_sum(ncoll);
  if (lane == 0) add_stats(dp->stats, (unsigned long long)nlive, (unsigned long long)ncoll,
                           (unsigned long long)nsub);
}

// ---------------------------------------------------------------------------
// Big cells (> 512 slots): global bucket sort by the top key bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bucket_of(uint32_t key, int bbits) {
  return bbits ? (key >> (32 - bbits)) : 0u;
}

// B1: bucket counts and live count; 256 threads x 4 slots per block
__global__ void __launch_bounds__(256) k_big_count(const SimDesc* __restrict__ descs,
                                                   const BigTask* __restrict__ big,
                                                   const BigChunk* __restrict__ chunks,
                                                   uint32_t* __restrict__ bucket_cnt,
                                                   uint32_t* __restrict__ task_live,
                                                   uint32_t k_abs) {
  __shared__ int red[4];
  const BigChunk ch = chunks[blockIdx.x];
  const BigTask tk = big[ch.task];
  const SimDesc* dp = descs + tk.sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  const int64_t o0 = dp->cell_off[tk.cell];
  const int g = ch.first / 4 + threadIdx.x;
  const int j0 = 4 * g;
  int live = 0;
  if (j0 < tk.n_slots) {
    const uint4 w = philox(make_uint4((uint32_t)g, (uint32_t)tk.cell, s, 0u), dp->seed_lo,
                           dp->seed_hi);
    const uint32_t kk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = j0 + e;
      if (j < tk.n_slots && dp->xi[o0 + j] > 0) {
        atomicAdd(&bucket_cnt[tk.bucket_base + bucket_of(kk[e], tk.bbits)], 1u);
        ++live;
      }
    }
  }
  live = wave_sum(live);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = live;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = red[0] + red[1] + red[2] + red[3];
    if (tot) atomicAdd(&task_live[ch.task], (uint32_t)tot);
  }
}

// B2: exclusive scan of each big cell's bucket counts
__global__ void __launch_bounds__(256) k_big_scan(const SimDesc* __restrict__ descs,
                                                  const BigTask* __restrict__ big,
                                                  const uint32_t* __restrict__ bucket_cnt,
                                                  uint32_t* __restrict__ bucket_start,
                                                  uint32_t* __restrict__ task_live,
                                                  uint32_t* __restrict__ task_nlive,
                                                  uint32_t k_abs) {
  __shared__ int part[256];
  const BigTask tk = big[blockIdx.x];
  const SimDesc* dp = descs + tk.sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  const int nb = 1 << tk.bbits;
  const int per = (nb + 255) / 256;
  const int first = threadIdx.x * per;
  int local = 0;
  for (int i = 0; i < per; ++i)
    if (first + i < nb) local += (int)bucket_cnt[tk.bucket_base + first + i];
  part[threadIdx.x] = local;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {  // inclusive scan in LDS
    const int t = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int run = part[threadIdx.x] - local;
  for (int i = 0; i < per; ++i) {
    if (first + i < nb) {
      const int cv = (int)bucket_cnt[tk.bucket_base + first + i];
      bucket_start[tk.bucket_base + first + i] = (uint32_t)run;
      run += cv;
    }
  }
  if (threadIdx.x == 0) {
    const uint32_t live = task_live[blockIdx.x];
    bucket_start[tk.bucket_base + nb] = live;
    task_nlive[blockIdx.x] = live;
    task_live[blockIdx.x] = 0;
  }
}

// B3: scatter (key << 32 | slot) into the buckets; leaves the counts at zero
__global__ void __launch_bounds__(256) k_big_scatter(const SimDesc* __restrict__ descs,
                                                     const BigTask* __restrict__ big,
                                                     const BigChunk* __restrict__ chunks,
                                                     uint32_t* __restrict__ bucket_cnt,
                                                     const uint32_t* __restrict__ bucket_start,
                                                     unsigned long long* __restrict__ tmp,
                                                     uint32_t k_abs) {
  const BigChunk ch = chunks[blockIdx.x];
  const BigTask tk = big[ch.task];
  const SimDesc* dp = descs + tk.sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  const int64_t o0 = dp->cell_off[tk.cell];
  const int g = ch.first / 4 + threadIdx.x;
  const int j0 = 4 * g;
  if (j0 >= tk.n_slots) return;
  const uint4 w = philox(make_uint4((uint32_t)g, (uint32_t)tk.cell, s, 0u), dp->seed_lo,
                         dp->seed_hi);
  const uint32_t kk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int j = j0 + e;
    if (j < tk.n_slots && dp->xi[o0 + j] > 0) {
      const uint32_t b = bucket_of(kk[e], tk.bbits);
      const uint32_t pos = atomicSub(&bucket_cnt[tk.bucket_base + b], 1u) - 1u;
      tmp[tk.tmp_base + bucket_start[tk.bucket_base + b] + pos] =
          ((unsigned long long)kk[e] << 32) | (unsigned)j;
    }
  }
}

// B4: exact rank inside each bucket, one wave per bucket
__global__ void __launch_bounds__(512) k_big_rank(const SimDesc* __restrict__ descs,
                                                  const BigTask* __restrict__ big,
                                                  const BigBucket* __restrict__ buckets,
                                                  int n_buckets,
                                                  const uint32_t* __restrict__ bucket_start,
                                                  const unsigned long long* __restrict__ tmp,
                                                  uint32_t* __restrict__ ord, uint32_t k_abs) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int gbk = blockIdx.x * (blockDim.x >> 6) + wv;
  if (gbk >= n_buckets) return;
  unsigned long long* e = reinterpret_cast<unsigned long long*>(smem) + wv * kBucketCap;
  const BigBucket bk = buckets[gbk];
  const BigTask tk = big[bk.task];
  const SimDesc* dp = descs + tk.sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  const int st = (int)bucket_start[tk.bucket_base + bk.bucket];
  const int en = (int)bucket_start[tk.bucket_base + bk.bucket + 1];
  const int len = en - st;
  const unsigned long long* src = tmp + tk.tmp_base + st;
  uint32_t* dst = ord + tk.tmp_base + st;
  if (len <= kBucketCap) {
    for (int i = lane; i < len; i += 64) e[i] = src[i];
    wave_sync();
    for (int i0 = 0; i0 < len; i0 += 64) {
      const int i = i0 + lane;
      const unsigned long long me = i < len ? e[i] : 0ull;
      int r = 0;
      for (int qq = 0; qq < len; ++qq) r += (e[qq] < me) ? 1 : 0;
      if (i < len) dst[r] = (uint32_t)(me & 0xFFFFFFFFull);
    }
  } else {  // rare: bucket larger than the LDS stage, rank from global memory
    if (lane == 0) atomicOr(dp->status, kFlagBucketOverflow);
    for (int i0 = 0; i0 < len; i0 += 64) {
      const int i = i0 + lane;
      const unsigned long long me = i < len ? src[i] : 0ull;
      int r = 0;
      for (int qq = 0; qq < len; ++qq) r += (src[qq] < me) ? 1 : 0;
      if (i < len) dst[r] = (uint32_t)(me & 0xFFFFFFFFull);
    }
  }
}

// B5: pairs over the global order; one thread per pair group (pairs 2h, 2h+1)
__global__ void __launch_bounds__(256) k_big_pairs(const SimDesc* __restrict__ descs,
                                                   const BigTask* __restrict__ big,
                                                   const BigPairBlock* __restrict__ pblocks,
                                                   const uint32_t* __restrict__ task_nlive,
                                                   const uint32_t* __restrict__ ord,
                                                   uint32_t k_abs) {
  __shared__ int red[4];
  const BigPairBlock pb = pblocks[blockIdx.x];
  const BigTask tk = big[pb.task];
  const SimDesc* dp = descs + tk.sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  const int64_t o0 = dp->cell_off[tk.cell];
  const int h = pb.first_group + threadIdx.x;
  const int nlive = (int)task_nlive[pb.task];
  const int P = nlive >> 1;
  int ncoll = 0;
  int64_t* sink = dp->sink;
  const int64_t sink_base = sink ? 2 * dp->pair_base[tk.cell] : 0;
  if (sink) {
    for (int e = 0; e < 2; ++e) {
      const int m = 2 * h + e;
      if (m >= P && m < (tk.n_slots >> 1)) {
        sink[sink_base + 2 * m] = -1;
        sink[sink_base + 2 * m + 1] = -1;
      }
    }
  }
  if (2 * h < P) {
    const double S = (double)((nlive & 1) ? nlive : nlive - 1);
    const uint4 w = philox(make_uint4((uint32_t)h, (uint32_t)tk.cell, s, 1u), dp->seed_lo,
                           dp->seed_hi);
    const uint32_t* o = ord + tk.tmp_base;
    int64_t* xi = dp->xi + o0;
    double* v = dp->v + o0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int m = 2 * h + e;
      if (m >= P) break;
      const int a = (int)o[2 * m], bb = (int)o[2 * m + 1];
      const long long xa = xi[a], xb = xi[bb];
      const double va = v[a], vb = v[bb];
      const double kv = coal_kernel(dp->kernel, dp->b, va, vb);
      const double p = (((double)(xa > xb ? xa : xb) * kv) * S) * dp->q;
      const double phi = e == 0 ? uniform53(w.x, w.y) : uniform53(w.z, w.w);
      const long long gamma = collisions(p, phi, dp->status);
      if (sink) {
        sink[sink_base + 2 * m] = (int64_t)((uint64_t)a | ((uint64_t)bb << 32));
        sink[sink_base + 2 * m + 1] = gamma;
      }
      if (gamma > 0) {
        ++ncoll;
        update_pair(xi, v, a, bb, xa, xb, va, vb, gamma, dp->attrs, dp->n_slots, dp->n_attr,
                    o0 + a, o0 + bb);
      }
    }
  }
  ncoll = wave_sum(ncoll);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ncoll;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long* st = dp->stats + (blockIdx.x % kStatSlots) * kStatFields;
    const int tot = red[0] + red[1] + red[2] + red[3];
    if (tot) atomicAdd(st + 1, (unsigned long long)tot);
    if (pb.first_group == 0) {  // once per cell and step
      atomicAdd(st + 0, (unsigned long long)nlive);
      atomicAdd(st + 2, 1ull);
      atomicAdd(st + 3, 1ull);
    }
  }
}

// ---------------------------------------------------------------------------
// Moments: one block of 256 per cell, fixed-order tree reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double x, double* red) {
  red[threadIdx.x] = x;
  __syncthreads();
  for (int st = 128; st >= 1; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256) k_moments(SimDesc d, int64_t* m0, double* m12,
                                                 double* attr_sums, const double* edges,
                                                 int n_bins, double* spectrum) {
  __shared__ double red[256];
  __shared__ unsigned long long ired[256];
  const int c = blockIdx.x;
  const int64_t o0 = d.cell_off[c];
  const int64_t n = d.cell_off[c + 1] - o0;
  unsigned long long cnt = 0;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const long long x = d.xi[o0 + j];
    if (x > 0) {
      const double w1 = (double)x * d.v[o0 + j];
      cnt += (unsigned long long)x;
      s1 += w1;
      s2 += w1 * d.v[o0 + j];
    }
  }
  ired[threadIdx.x] = cnt;
  __syncthreads();
  for (int st = 128; st >= 1; st >>= 1) {
    if ((int)threadIdx.x < st) ired[threadIdx.x] += ired[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0 && m0) m0[c] = (int64_t)ired[0];
  s1 = block_sum(s1, red);
  s2 = block_sum(s2, red);
  if (threadIdx.x == 0 && m12) {
    m12[2 * c] = s1;
    m12[2 * c + 1] = s2;
  }
  if (attr_sums) {
    for (int q = 0; q < d.n_attr; ++q) {
      const double* a = d.attrs + (int64_t)q * d.n_slots + o0;
      double sa = 0.0;
      for (int64_t j = threadIdx.x; j < n; j += 256) {
        const long long x = d.xi[o0 + j];
        if (x > 0) sa += (double)x * a[j];
      }
      sa = block_sum(sa, red);
      if (threadIdx.x == 0) attr_sums[(int64_t)c * d.n_attr + q] = sa;
    }
  }
  if (spectrum) {
    for (int k = 0; k < n_bins; ++k) {
      const double lo = edges[k], hi = edges[k + 1];
      double sb = 0.0;
      for (int64_t j = threadIdx.x; j < n; j += 256) {
        const long long x = d.xi[o0 + j];
        const double vv = d.v[o0 + j];
        if (x > 0 && lo <= vv && vv < hi) sb += (double)x * vv;
      }
      sb = block_sum(sb, red);
      if (threadIdx.x == 0) spectrum[(int64_t)c * n_bins + k] = sb;
    }
  }
}

// ---------------------------------------------------------------------------
// Validation and test hooks
// ---------------------------------------------------------------------------
__global__ void k_validate(const int64_t* __restrict__ xi, const double* __restrict__ v,
                           int64_t n, uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long long x = xi[i];
  bool bad = x < 0 || x >= (1LL << 53);
  if (x > 0) {
    const double vv = v[i];
    bad = bad || !(vv > 0.0) || !(vv < 1e300);
  }
  if (bad) atomicOr(status, kFlagInvalid);
}

__global__ void k_philox_fill(uint32_t* out, int64_t n, uint32_t c0, uint32_t c1, uint32_t c2,
                              uint32_t c3, uint32_t k0, uint32_t k1) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 w = philox(make_uint4(c0 + (uint32_t)i, c1, c2, c3), k0, k1);
  *reinterpret_cast<uint4*>(out + 4 * i) = w;
}

__global__ void k_kernel_values(int kind, double b, const double* v1, const double* v2, int64_t n,
                                double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = coal_kernel(kind, b, v1[i], v2[i]);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t wave_lds_bytes(int cls) {
  switch (cls) {
    case 0: return sizeof(WaveLds<64>);
    case 1: return sizeof(WaveLds<128>);
    case 2: return sizeof(WaveLds<256>);
    default: return sizeof(WaveLds<512>);
  }
}

void set_lds_limits() {
  static bool done = false;
  if (done) return;
  done = true;
  const int lim = 160 * 1024;
  (void)hipFuncSetAttribute((const void*)k_wave_cells<64>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_wave_cells<128>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_wave_cells<256>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_wave_cells<512>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_big_rank, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lim);
  (void)hipGetLastError();
}

template <int CAP>
static void launch_class(const PlanDev& p, int cls, uint32_t k_abs, int wpb, hipStream_t st) {
  const int n = p.n_wave[cls];
  if (n <= 0) return;
  const int grid = (n + wpb - 1) / wpb;
  hipLaunchKernelGGL(k_wave_cells<CAP>, dim3(grid), dim3(64 * wpb),
                     (unsigned)(wpb * sizeof(WaveLds<CAP>)), st, p.desc, p.wave_tasks[cls], n,
                     k_abs);
}

hipError_t launch_step(const PlanDev& p, uint32_t k_abs, int wpb, hipStream_t st) {
  launch_class<512>(p, 3, k_abs, wpb, st);
  launch_class<256>(p, 2, k_abs, wpb, st);
  launch_class<128>(p, 1, k_abs, wpb, st);
  launch_class<64>(p, 0, k_abs, wpb, st);
  if (p.n_big > 0) {
    hipLaunchKernelGGL(k_big_count, dim3(p.n_chunks), dim3(256), 0, st, p.desc, p.big, p.chunks,
                       p.bucket_cnt, p.task_live, k_abs);
    hipLaunchKernelGGL(k_big_scan, dim3(p.n_big), dim3(256), 0, st, p.desc, p.big, p.bucket_cnt,
                       p.bucket_start, p.task_live, p.task_nlive, k_abs);
    hipLaunchKernelGGL(k_big_scatter, dim3(p.n_chunks), dim3(256), 0, st, p.desc, p.big,
                       p.chunks, p.bucket_cnt, p.bucket_start, p.tmp, k_abs);
    const int rw = 4;
    hipLaunchKernelGGL(k_big_rank, dim3((p.n_buckets + rw - 1) / rw), dim3(64 * rw),
                       (unsigned)(rw * kBucketCap * sizeof(unsigned long long)), st, p.desc,
                       p.big, p.buckets, p.n_buckets, p.bucket_start, p.tmp, p.ord, k_abs);
    hipLaunchKernelGGL(k_big_pairs, dim3(p.n_pblocks), dim3(256), 0, st, p.desc, p.big,
                       p.pblocks, p.task_nlive, p.ord, k_abs);
  }
  return hipGetLastError();
}

hipError_t launch_moments(const SimDesc& d, int n_cells, int64_t* m0, double* m12,
                          double* attr_sums, const double* edges, int n_bins, double* spectrum,
                          hipStream_t st) {
  if (n_cells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_moments, dim3(n_cells), dim3(256), 0, st, d, m0, m12, attr_sums, edges,
                     n_bins, spectrum);
  return hipGetLastError();
}

hipError_t launch_validate(const int64_t* xi, const double* v, int64_t n, uint32_t* status,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xi, v, n,
                     status);
  return hipGetLastError();
}

hipError_t launch_philox_fill(uint32_t* out, int64_t n, uint32_t c0, uint32_t c1, uint32_t c2,
                              uint32_t c3, uint32_t k0, uint32_t k1, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n,
                     c0, c1, c2, c3, k0, k1);
  return hipGetLastError();
}

hipError_t launch_kernel_values(int kind, double b, const double* v1, const double* v2, int64_t n,
                                double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kernel_values, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, kind,
                     b, v1, v2, n, out);
  return hipGetLastError();
}

}  // namespace sdm
