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

#include <algorithm>

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
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * x.x;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * x.z;
    x = make_uint4((uint32_t)(p1 >> 32) ^ x.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ x.w ^ k1,
                   (uint32_t)p0);
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
  const double u12 = fmin(kU1 * r * r, kU2 * r);
  // Up to 600 um the square-root regime lies at least 2.6 % above the linear
  // one (it crosses at (k3/k2)^2 = 631 um), so it cannot be the minimum and
  // its square root is skipped: the result is the same bits.
  if (r <= 6.0e-4) return u12;
  return fmin(u12, kU3 * sqrt(r));
}



// The per-SD quantity the kernel is built from ("size"): the radius for the
// geometric kernel, the volume itself for Golovin's.  A cell kernel keeps it
// in LDS and recomputes it only for SDs whose volume changed, so the cube
// root is taken once per SD and step instead of once per SD and substep.
// pair_kernel(kind, b, size_of(kind, va), size_of(kind, vb)) is bitwise
// coal_kernel(kind, b, va, vb).
__device__ __forceinline__ double size_of(int kind, double v) {
  return kind == 0 ? v : cbrt(kVolToR3 * v);
}

// fall_speed for the cell kernels: the square-root regime is taken only when
// some lane of the wavefront has a radius above 600 um (a wave-uniform
// branch), so that the compiler cannot turn it into a select that computes
// the square root for every SD.  Same bits as fall_speed.
__device__ __forceinline__ double fall_speed_w(double r) {
  double u = fmin(kU1 * r * r, kU2 * r);
  if (__builtin_amdgcn_ballot_w64(r > 6.0e-4) != 0) {
    // an empty volatile statement makes this block non-speculatable: without
    // it the compiler computes the square root for every lane and selects
    __asm__ volatile("");
    if (r > 6.0e-4) u = fmin(u, kU3 * sqrt(r));
  }
  return u;
}

__device__ __forceinline__ double pair_kernel(int kind, double b, double sa, double sb) {
  if (kind == 0) return b * (sa + sb);
  const double rs = sa + sb;
  return kPi * (rs * rs) * fabs(fall_speed_w(sa) - fall_speed_w(sb));
}

// the kernel from two volumes (Golovin additive; geometric sweep-out, E = 1)
__device__ __forceinline__ double coal_kernel(int kind, double b, double va, double vb) {
  return pair_kernel(kind, b, size_of(kind, va), size_of(kind, vb));
}

__device__ __forceinline__ long long collisions(double p, double phi, uint32_t* status) {
  if (p < 1.0) return phi < p ? 1 : 0;  // floor(p) = 0 and p - floor(p) = p
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

// Wave-wide reductions and scans on DPP row operations (VALU lane moves)
// and four readlanes, instead of LDS-routed shuffles: after the two quad
// permutes, the half-row mirror and the row mirror every lane holds its
// 16-lane row's result; lanes 15, 31, 47 and 63 then carry the four rows.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
constexpr int kDppQuad1032 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppQuad2301 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kDppRowMirror = 0x140;  // lane i <- lane 15 - i within a row
constexpr int kDppHalfMirror = 0x141; // lane i <- lane 7 - i within a half row
constexpr int kDppRowShr = 0x110;     // + n: lane i <- lane i - n within a row, 0 below

__device__ __forceinline__ int wave_sum(int x) {
  x += dpp_i<kDppQuad1032>(x);
  x += dpp_i<kDppQuad2301>(x);
  x += dpp_i<kDppHalfMirror>(x);
  x += dpp_i<kDppRowMirror>(x);
  return __builtin_amdgcn_readlane(x, 15) + __builtin_amdgcn_readlane(x, 31) +
         __builtin_amdgcn_readlane(x, 47) + __builtin_amdgcn_readlane(x, 63);
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_i<CTRL>((int)(b & 0xFFFFFFFFll));
  const int hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_max(double x) {
  x = fmax(x, dpp_d<kDppQuad1032>(x));
  x = fmax(x, dpp_d<kDppQuad2301>(x));
  x = fmax(x, dpp_d<kDppHalfMirror>(x));
  x = fmax(x, dpp_d<kDppRowMirror>(x));
  return fmax(fmax(readlane_d(x, 15), readlane_d(x, 31)),
              fmax(readlane_d(x, 47), readlane_d(x, 63)));
}

// exclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_excl_scan(int x, int lane) {
  int v = x;  // inclusive scan within each 16-lane row (shifts 1, 2, 4, 8) ...
  v += dpp_i<kDppRowShr + 1>(v);
  v += dpp_i<kDppRowShr + 2>(v);
  v += dpp_i<kDppRowShr + 4>(v);
  v += dpp_i<kDppRowShr + 8>(v);
  // ... plus the totals of the rows before
  const int r0 = __builtin_amdgcn_readlane(v, 15), r1 = __builtin_amdgcn_readlane(v, 31),
            r2 = __builtin_amdgcn_readlane(v, 47);
  const int row = lane >> 4;
  v += row == 0 ? 0 : row == 1 ? r0 : row == 2 ? r0 + r1 : r0 + r1 + r2;
  return v - x;
}

__device__ __forceinline__ void add_stats(unsigned long long* stats, unsigned long long live,
                                          unsigned long long coll, unsigned long long substeps,
                                          unsigned long long steps = 1) {
  unsigned long long* s = stats + (blockIdx.x % kStatSlots) * kStatFields;
  if (live) atomicAdd(s + 0, live);
  if (coll) atomicAdd(s + 1, coll);
  if (substeps) atomicAdd(s + 2, substeps);
  if (steps) atomicAdd(s + 3, steps);
}

// ---------------------------------------------------------------------------
// Update of one colliding pair.  ia/ib index xs/vs (LDS or global) and ga/gb
// the global slots of the attributes.  Returns 1 if a slot was left empty
// (an equal split of a multiplicity-1 pair), else 0.
// ---------------------------------------------------------------------------
template <typename XI, typename VV>
__device__ __forceinline__ int update_pair(XI* xs, VV* vs, int ia, int ib, long long xa,
                                            long long xb, double va, double vb, long long gamma,
                                            double* attrs, int64_t n_slots, int n_attr,
                                            int64_t ga, int64_t gb, double* nva = nullptr,
                                            double* nvb = nullptr) {
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
    const double t = fma(gd, vj, vk);
    vs[ik] = t;
    if (nva) {  // new volumes of a and b
      *nva = a_is_j ? vj : t;
      *nvb = a_is_j ? t : vj;
    }
    for (int q = 0; q < n_attr; ++q) {
      double* a = attrs + (int64_t)q * n_slots;
      a[gk] = fma(gd, a[gj], a[gk]);
    }
    return 0;
  } else {  // equal-multiplicity split
    const long long h = xk >> 1;
    xs[ij] = h;
    xs[ik] = xk - h;
    const double t = fma(gd, vj, vk);
    vs[ij] = t;
    vs[ik] = t;
    if (nva) {
      *nva = t;
      *nvb = t;
    }
    for (int q = 0; q < n_attr; ++q) {
      double* a = attrs + (int64_t)q * n_slots;
      const double ta = fma(gd, a[gj], a[gk]);
      a[gj] = ta;
      a[gk] = ta;
    }
    return h == 0 ? 1 : 0;  // xk = 1: slot j is left empty
  }
}

// Dispatch-order group of an adaptive cell by the substeps it took (8 or
// more, 4-7, 2-3, at most 1): the next step dispatches the groups in order.
__device__ __forceinline__ uint32_t order_group(uint32_t substeps) {
  return substeps >= 8 ? 0u : substeps >= 4 ? 1u : substeps >= 2 ? 2u : 3u;
}

// A thread's share of the bucket-counter scan: `per` consecutive counters
// from `first` (16-byte LDS accesses when per is a multiple of 4).
__device__ __forceinline__ int scan_load(const uint32_t* cnt, int first, int per, int nb) {
  int local = 0;
  if (first >= nb) return 0;
  if ((per & 3) == 0) {
    for (int i = 0; i < per; i += 4) {
      const uint4 q = *reinterpret_cast<const uint4*>(&cnt[first + i]);
      local += (int)(q.x + q.y + q.z + q.w);
    }
  } else {
    for (int i = 0; i < per; ++i) local += (int)cnt[first + i];
  }
  return local;
}

// replace the counters by their exclusive prefix sums starting at `run`
__device__ __forceinline__ void scan_store(uint32_t* cnt, int first, int per, int nb, int run) {
  if (first >= nb) return;
  if ((per & 3) == 0) {
    for (int i = 0; i < per; i += 4) {
      uint4 q = *reinterpret_cast<const uint4*>(&cnt[first + i]);
      const uint32_t a = (uint32_t)run, b = a + q.x, c2 = b + q.y, d = c2 + q.z;
      run = (int)(d + q.w);
      q = make_uint4(a, b, c2, d);
      *reinterpret_cast<uint4*>(&cnt[first + i]) = q;
    }
  } else {
    for (int i = 0; i < per; ++i) {
      const int cv = (int)cnt[first + i];
      cnt[first + i] = (uint32_t)run;
      run += cv;
    }
  }
}

// ---------------------------------------------------------------------------
// One workgroup ("team" of W wavefronts) per cell of <= CAP slots.
//
// Every phase spreads its work over the W*64 threads.  LDS per slot: the
// multiplicity (8 B) and the SD's kernel size (8 B: radius or volume, see
// size_of) in slot order, one 32-bit word that first holds the bucketed
// (key, slot) entries and then the 16-bit permutation, and one 32-bit bucket
// counter.  Volumes stay in global memory: they are read and written only
// for colliding pairs, like the extra attributes.  In the sort a thread owns
// 4 consecutive slots, i.e. exactly the 4 words of one Philox call, so keys
// never go through LDS; in the pair passes thread h owns pairs 2h and 2h+1,
// whose two uniforms are the 4 words of one Philox call.
//
// Latency: every phase first issues all of a thread's LDS reads, then waits
// once; reads that would be conditional are made unconditional on clamped,
// in-bounds addresses and their results masked, so that no read waits inside
// a per-entry branch.
// ---------------------------------------------------------------------------
constexpr int pow2_ceil(int x) { return x <= 1 ? 1 : 2 * pow2_ceil((x + 1) / 2); }

// One colliding pair of a (sub)step.  The pair pass lists (a, b, gamma);
// the multiplicity phase rewrites the entry as (j, k, split, g): j the
// member with the larger multiplicity, k the other, split = 1 for an equal
// split; the volume and attribute phase then sets X_k = fma(g, X_j, X_k) for
// every extensive X, and X_j = X_k too when the pair split equally.
struct alignas(16) Coll {
  uint16_t j, k;
  uint32_t split;
  long long g;
};

template <int CAP>
struct alignas(16) CellLds {
  // multiplicities as doubles: every multiplicity is an integer below 2^53
  // (sdm_init checks it, and the update only lowers them), so the doubles
  // are exact and compare and convert exactly
  double xd[CAP];
  double rs[CAP];     // kernel sizes (slot order)
  // tmp: bucketed (key << nbits | slot), then the uint16 permutation; cnt:
  // bucket counters / starts.  Once a pair pass has the permutation in
  // registers, tmp and cnt together hold the list of colliding pairs.
  uint32_t tmp[CAP];
  uint32_t cnt[pow2_ceil(CAP) + 4];
  uint32_t dirty[CAP / 32];  // LDS-resident steps: multiplicities to write back
  int nlist;                 // colliding pairs listed in this (sub)step
  int red_i[8];              // cross-wave reductions
  double red_d[8];
};

template <int CAP>
__device__ __forceinline__ Coll* coll_list(CellLds<CAP>& L) {
  static_assert(sizeof(L.tmp) % 16 == 0, "the list starts 16-byte aligned");
  static_assert((sizeof(L.tmp) + sizeof(L.cnt)) / sizeof(Coll) >= CAP / 2,
                "every pair of a full cell can be listed");
  return reinterpret_cast<Coll*>(L.tmp);
}

template <int W>
__device__ __forceinline__ void team_sync() {
  if (W == 1)
    wave_sync();
  else
    __syncthreads();
}

// team-wide sum / max; red points to >= W LDS slots
template <int W>
__device__ __forceinline__ int team_sum_r(int* red, int x, int lane, int wv) {
  x = wave_sum(x);
  if (W == 1) return x;
  if (lane == 0) red[wv] = x;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) t += red[k];
  __syncthreads();
  return t;
}

template <int W>
__device__ __forceinline__ double team_max_r(double* red, double x, int lane, int wv) {
  x = wave_max(x);
  if (W == 1) return x;
  if (lane == 0) red[wv] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < W; ++k) t = fmax(t, red[k]);
  __syncthreads();
  return t;
}

template <int W, int CAP>
__device__ __forceinline__ int team_sum(CellLds<CAP>& L, int x, int lane, int wv) {
  return team_sum_r<W>(L.red_i, x, lane, wv);
}

template <int W, int CAP>
__device__ __forceinline__ double team_max(CellLds<CAP>& L, double x, int lane, int wv) {
  return team_max_r<W>(L.red_d, x, lane, wv);
}

template <int CAP>
__device__ __forceinline__ uint16_t* perm_of(CellLds<CAP>& L) {
  return reinterpret_cast<uint16_t*>(L.tmp);
}

// Slots a thread owns in the sort and pair phases of a workgroup-per-cell
// class: 4, the words of one Philox call, or 6 for one-wave 384-slot cells.
// The work a wave issues per phase is (rounds x slots per thread): 2 x 4 = 8
// slot-works for a 384-slot capacity, 1 x 6 = 6 with six (still two Philox
// calls per thread: six consecutive slots from an even start lie in two
// groups of 4).  For 512 slots 2 x 4 = 1 x 8, so four stay.
template <int CAP, int W>
constexpr int slots_per_thread() {
  return (CAP == 384 && W == 1) ? 6 : 4;
}
template <int CAP, int W>
constexpr int sort_rounds() {
  return (CAP + slots_per_thread<CAP, W>() * 64 * W - 1) / (slots_per_thread<CAP, W>() * 64 * W);
}

// the 32-bit keys of slots j0 .. j0 + SPT - 1 (j0 a multiple of SPT): word
// j mod 4 of Philox((j / 4, c, s, 2u))
template <int SPT>
__device__ __forceinline__ void slot_keys(int j0, int c, uint32_t s, uint32_t u, uint32_t k0,
                                          uint32_t k1, uint32_t (&kr)[SPT]) {
  const uint32_t ga = (uint32_t)j0 >> 2;
  const uint4 wa = philox(make_uint4(ga, (uint32_t)c, s, 2u * u), k0, k1);
  if constexpr (SPT == 4) {
    kr[0] = wa.x;
    kr[1] = wa.y;
    kr[2] = wa.z;
    kr[3] = wa.w;
  } else {
    static_assert(SPT == 6, "4 or 6 slots per thread");
    const uint4 wb = philox(make_uint4(ga + 1u, (uint32_t)c, s, 2u * u), k0, k1);
    const bool odd = (j0 & 3) != 0;  // j0 mod 4 is 0 or 2
    kr[0] = odd ? wa.z : wa.x;
    kr[1] = odd ? wa.w : wa.y;
    kr[2] = odd ? wb.x : wa.z;
    kr[3] = odd ? wb.y : wa.w;
    kr[4] = odd ? wb.z : wb.x;
    kr[5] = odd ? wb.w : wb.y;
  }
}

// keys, bucket count, scan, scatter, rank: permutation of the nlive live slots
template <int CAP, int W>
__device__ __forceinline__ void team_sort(CellLds<CAP>& L, int n, int nlive, int tid, int lane,
                                          int wv, int c, uint32_t s, uint32_t u, uint32_t k0,
                                          uint32_t k1) {
  constexpr int T = 64 * W;
  constexpr int SPT = slots_per_thread<CAP, W>();
  constexpr int I4 = sort_rounds<CAP, W>();  // rounds of SPT slots per thread
  const int nbits = 32 - __clz(n - 1);        // n >= 2
  const int nb = 1 << nbits;
  const int sh = 32 - nbits;
  for (int i = 4 * tid; i < nb + 4; i += 4 * T)  // counters 0..nb, 16 bytes at a time
    *reinterpret_cast<uint4*>(&L.cnt[i]) = make_uint4(0u, 0u, 0u, 0u);
  team_sync<W>();

  // keys of live slots (registers) and their place in their bucket (atomics)
  uint32_t me[I4][SPT], pos[I4][SPT], bk[I4][SPT];
  uint32_t live[I4];
#pragma unroll
  for (int i = 0; i < I4; ++i) {
    const int j0 = SPT * (T * i + tid);
    live[i] = 0;
#pragma unroll
    for (int e = 0; e < SPT; ++e) {
      me[i][e] = 0;
      pos[i][e] = 0;
      bk[i][e] = 0;
    }
    if (j0 < n) {
      uint32_t kr[SPT];
      slot_keys<SPT>(j0, c, s, u, k0, k1, kr);
      double xv[SPT];
#pragma unroll
      for (int e = 0; e < SPT; e += 2) {  // j0 is even: 16-byte LDS reads
        const double2 x2 = *reinterpret_cast<const double2*>(&L.xd[j0 + e]);
        xv[e] = x2.x;
        xv[e + 1] = x2.y;
      }
#pragma unroll
      for (int e = 0; e < SPT; ++e) {
        const bool lv = j0 + e < n && xv[e] > 0.0;
        live[i] |= lv ? 1u << e : 0u;
        bk[i][e] = kr[e] >> sh;
        me[i][e] = (kr[e] << nbits) | (uint32_t)(j0 + e);
        if (lv) pos[i][e] = atomicAdd(&L.cnt[bk[i][e]], 1u);
      }
    }
  }
  team_sync<W>();
  {  // exclusive scan of the nb bucket counts over the team
    const int per = nb >= T ? nb / T : 1;
    const int first = tid * per;
    int local = scan_load(L.cnt, first, per, nb);
    int run = wave_excl_scan(local, lane);
    if (W > 1) {
      if (lane == 63) L.red_i[wv] = run + local;  // this wave's total
      __syncthreads();
      for (int k = 0; k < wv; ++k) run += L.red_i[k];
      __syncthreads();
    }
    scan_store(L.cnt, first, per, nb, run);
    if (tid == 0) L.cnt[nb] = (uint32_t)nlive;
  }
  team_sync<W>();
  // scatter: every bucket range is read before the first store
  uint32_t st[I4][SPT], len[I4][SPT];
#pragma unroll
  for (int i = 0; i < I4; ++i)
#pragma unroll
    for (int e = 0; e < SPT; ++e) {
      const uint32_t b = ((live[i] >> e) & 1) ? bk[i][e] : 0u;  // counters 0..nb are valid
      st[i][e] = L.cnt[b];
      len[i][e] = L.cnt[b + 1];
    }
  int maxlen = 0;
#pragma unroll
  for (int i = 0; i < I4; ++i)
#pragma unroll
    for (int e = 0; e < SPT; ++e) {
      const bool lv = (live[i] >> e) & 1;
      len[i][e] = lv ? len[i][e] - st[i][e] : 0u;
      st[i][e] = lv ? st[i][e] : 0u;
      if (lv) L.tmp[st[i][e] + pos[i][e]] = me[i][e];
      maxlen = max(maxlen, (int)len[i][e]);
    }
  team_sync<W>();
  // exact rank inside the bucket: each round reads one entry of every
  // bucket of the thread (clamped into the array; masked beyond the bucket)
  uint32_t rk[I4][SPT];
#pragma unroll
  for (int i = 0; i < I4; ++i)
#pragma unroll
    for (int e = 0; e < SPT; ++e) rk[i][e] = st[i][e];
  for (int k = 0; k < maxlen; ++k) {
    uint32_t x[I4][SPT];
#pragma unroll
    for (int i = 0; i < I4; ++i)
#pragma unroll
      for (int e = 0; e < SPT; ++e)
        x[i][e] = L.tmp[min(st[i][e] + (uint32_t)k, (uint32_t)CAP - 1u)];
#pragma unroll
    for (int i = 0; i < I4; ++i)
#pragma unroll
      for (int e = 0; e < SPT; ++e)
        rk[i][e] += ((uint32_t)k < len[i][e] && x[i][e] < me[i][e]) ? 1u : 0u;
  }
  team_sync<W>();
  uint16_t* perm = perm_of(L);
#pragma unroll
  for (int i = 0; i < I4; ++i)
#pragma unroll
    for (int e = 0; e < SPT; ++e)
      if ((live[i] >> e) & 1) perm[rk[i][e]] = (uint16_t)(SPT * (T * i + tid) + e);
  if (tid == 0) L.nlist = 0;
  team_sync<W>();
}

enum PassMode { kPassPlain = 0, kPassPmax = 1, kPassAdapt = 2, kPassPlainLds = 3 };

// Registers a thread carries between the two passes of an adaptive substep:
// the slots of its pairs (from the permutation) and their pre-products
// (max xi K) S.
template <int I4, int SPT>
struct PairRegs {
  uint32_t o[I4][SPT / 2];  // permutation entries, two 16-bit slots per word
  double pre[I4][SPT / 2];
};

// The uniforms of pairs NP h .. NP h + NP - 1 (NP = SPT / 2): pair m takes
// words 2 (m mod 2) and 2 (m mod 2) + 1 of Philox((m / 2, c, s, 2u + 1)) as
// the high and low halves; 4 slots per thread need one call, 6 need two.
template <int SPT>
__device__ __forceinline__ void pair_uniforms(int h, int c, uint32_t s, uint32_t u, uint32_t k0,
                                              uint32_t k1, double (&phi)[SPT / 2]) {
  if constexpr (SPT == 4) {
    const uint4 w = philox(make_uint4((uint32_t)h, (uint32_t)c, s, 2u * u + 1u), k0, k1);
    phi[0] = uniform53(w.x, w.y);
    phi[1] = uniform53(w.z, w.w);
  } else {
    const uint32_t ca = (uint32_t)(3 * h) >> 1;
    const uint4 wa = philox(make_uint4(ca, (uint32_t)c, s, 2u * u + 1u), k0, k1);
    const uint4 wb = philox(make_uint4(ca + 1u, (uint32_t)c, s, 2u * u + 1u), k0, k1);
    if ((h & 1) == 0) {  // pairs 3h, 3h + 1 in call ca, 3h + 2 in ca + 1
      phi[0] = uniform53(wa.x, wa.y);
      phi[1] = uniform53(wa.z, wa.w);
      phi[2] = uniform53(wb.x, wb.y);
    } else {  // pair 3h in call ca, 3h + 1 and 3h + 2 in ca + 1
      phi[0] = uniform53(wa.z, wa.w);
      phi[1] = uniform53(wb.x, wb.y);
      phi[2] = uniform53(wb.z, wb.w);
    }
  }
}

// Candidate pairs of one (sub)step; thread h takes sorted positions
// SPT h .. SPT h + SPT - 1, i.e. pairs NP h .. NP h + NP - 1 (NP = SPT / 2),
// whose uniforms come from one or two Philox calls.  kPassPlain updates
// global memory; kPassPlainLds computes p the same way and updates the
// LDS-resident multiplicities (steps fused in one launch); kPassPmax keeps
// the pre-products in registers and returns this thread's largest p at q;
// kPassAdapt takes them back, clamps p to 1 if asked and updates.  Volumes
// and attributes are always updated in global memory (vg: the cell's
// volumes); LDS-resident modes refresh the sizes of the updated SDs.
template <int CAP, int W, int MODE>
__device__ __forceinline__ double team_pairs(CellLds<CAP>& L, const SimDesc* dp, double* vg,
                                             int n, int nlive, int tid, int c, uint32_t s,
                                             uint32_t u, double q, bool clamp, int64_t o0,
                                             int* ncoll,
                                             PairRegs<sort_rounds<CAP, W>(),
                                                      slots_per_thread<CAP, W>()>& R,
                                             int* ndead = nullptr) {
  constexpr int T = 64 * W;
  constexpr int SPT = slots_per_thread<CAP, W>();
  constexpr int NP = SPT / 2;  // pairs per thread and round
  constexpr int I4 = sort_rounds<CAP, W>();
  const int P = nlive >> 1;
  const double S = (double)((nlive & 1) ? nlive : nlive - 1);
  const uint16_t* perm = perm_of(L);
  double pmax = 0.0;
  const int kind = dp->kernel;
  const double bgol = dp->b;
  int64_t* sink = (MODE == kPassPmax) ? nullptr : dp->sink;
  int64_t sink_base = 0;
  if (sink) sink_base = 2 * dp->pair_base[c];
  if (MODE != kPassAdapt) {
    // every pair's slots and sizes first (slots past the pairs clamped into
    // the cell and masked), then the arithmetic
    double xv[I4][SPT];
    double sv[I4][SPT];
#pragma unroll
    for (int i = 0; i < I4; ++i) {
      const int h = T * i + tid;
#pragma unroll
      for (int k = 0; k < NP; ++k) R.o[i][k] = 0u;
      if (NP * h >= P) continue;
      // positions SPT h ..: 4-byte aligned (8-byte with 4 slots per thread),
      // inside the permutation array's 2 CAP entries
      if constexpr (SPT == 4) {
        const uint2 o2 = *reinterpret_cast<const uint2*>(&perm[4 * h]);
        R.o[i][0] = o2.x;
        R.o[i][1] = o2.y;
      } else {
        const uint32_t* pw = reinterpret_cast<const uint32_t*>(&perm[SPT * h]);
#pragma unroll
        for (int k = 0; k < NP; ++k) R.o[i][k] = pw[k];
      }
#pragma unroll
      for (int e = 0; e < SPT; ++e) {
        const uint32_t sl = (e & 1) ? (R.o[i][e >> 1] >> 16) : (R.o[i][e >> 1] & 0xFFFFu);
        const uint32_t j = min(sl, (uint32_t)CAP - 1u);
        xv[i][e] = L.xd[j];
        sv[i][e] = L.rs[j];
      }
    }
#pragma unroll
    for (int i = 0; i < I4; ++i) {
      const int h = T * i + tid;
#pragma unroll
      for (int e = 0; e < NP; ++e) R.pre[i][e] = 0.0;
      if (NP * h >= P) continue;
#pragma unroll
      for (int e = 0; e < NP; ++e) {
        const double kv = pair_kernel(kind, bgol, sv[i][2 * e], sv[i][2 * e + 1]);
        const double pp = (fmax(xv[i][2 * e], xv[i][2 * e + 1]) * kv) * S;
        R.pre[i][e] = (NP * h + e < P) ? pp : 0.0;
        if (MODE == kPassPmax && NP * h + e < P) pmax = fmax(pmax, pp * q);
      }
    }
    if (MODE == kPassPmax) return pmax;
  }
  const bool in_lds = MODE != kPassPlain;
  // every thread's permutation reads are done before the list overwrites it
  team_sync<W>();
  Coll* list = coll_list(L);
  long long* xi_g = reinterpret_cast<long long*>(dp->xi + o0);
#pragma unroll
  for (int i = 0; i < I4; ++i) {
    const int h = T * i + tid;
    if (NP * h >= P) continue;
    double phis[NP];
    pair_uniforms<SPT>(h, c, s, u, dp->seed_lo, dp->seed_hi, phis);
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const int m = NP * h + e;
      if (m >= P) break;
      const int a = (int)(R.o[i][e] & 0xFFFFu);
      const int bb = (int)(R.o[i][e] >> 16);
      double p = R.pre[i][e] * q;
      if (clamp && p > 1.0) p = 1.0;
      const double phi = phis[e];
      const long long gamma = collisions(p, phi, dp->status);
      if (sink) {
        sink[sink_base + 2 * m] = (int64_t)((uint64_t)a | ((uint64_t)bb << 32));
        sink[sink_base + 2 * m + 1] = gamma;
      }
      if (gamma > 0) {  // listed; the updates follow in two dense phases
        *ncoll += 1;
        const int at = atomicAdd(&L.nlist, 1);
        Coll cl;
        cl.j = (uint16_t)a;
        cl.k = (uint16_t)bb;
        cl.split = 0;
        cl.g = gamma;
        list[at] = cl;
      }
    }
  }
  team_sync<W>();
  const int nl = L.nlist;
  // multiplicities: one thread per listed pair
  for (int li = tid; li < nl; li += T) {
    Coll cl = list[li];
    const int a = cl.j, bb = cl.k;
    const double xa = L.xd[a], xb = L.xd[bb];
    const bool a_is_j = xa >= xb;  // ties: the pair's first member
    const int j = a_is_j ? a : bb, k = a_is_j ? bb : a;
    const long long xj = (long long)(a_is_j ? xa : xb), xk = (long long)(a_is_j ? xb : xa);
    long long g = cl.g;
    if (g > 1) {
      const long long ratio = xj / xk;
      g = g < ratio ? g : ratio;
    }
    const long long rest = xj - g * xk;
    long long nj = rest, nk = xk;
    cl.split = 0;
    if (rest <= 0) {  // equal-multiplicity split; xk = 1 leaves slot j empty
      nj = xk >> 1;
      nk = xk - nj;
      cl.split = 1;
      if (in_lds) *ndead += nj == 0 ? 1 : 0;
    }
    if (in_lds) {
      L.xd[j] = (double)nj;
      L.xd[k] = (double)nk;
      atomicOr(&L.dirty[j >> 5], 1u << (j & 31));
      atomicOr(&L.dirty[k >> 5], 1u << (k & 31));
    } else {
      xi_g[j] = nj;
      if (cl.split) xi_g[k] = nk;
    }
    cl.j = (uint16_t)j;
    cl.k = (uint16_t)k;
    cl.g = g;
    list[li] = cl;
  }
  team_sync<W>();
  {  // volumes and attributes of every listed pair, spread over the team:
     // one round of independent global loads for up to T (pair, field) tasks
    const int F = 1 + dp->n_attr;
    const int ntask = nl * F;
    for (int t = tid; t < ntask; t += T) {
      const int li = t / F, f = t - li * F;
      const Coll cl = list[li];
      double* X = f == 0 ? vg : dp->attrs + (int64_t)(f - 1) * dp->n_slots + o0;
      const double val = fma((double)cl.g, X[cl.j], X[cl.k]);
      X[cl.k] = val;
      if (cl.split) X[cl.j] = val;
      if (in_lds && f == 0) {  // the size of an SD follows its volume
        const double sz = size_of(kind, val);
        L.rs[cl.k] = sz;
        if (cl.split) L.rs[cl.j] = sz;
      }
    }
  }
  if (sink) {  // unused pair entries of the cell
    for (int m = P + tid; m < (n >> 1); m += T) {
      sink[sink_base + 2 * m] = -1;
      sink[sink_base + 2 * m + 1] = -1;
    }
  }
  team_sync<W>();
  return pmax;
}

__device__ __forceinline__ void sink_clear_cell(const SimDesc* dp, int c, int n, int tid, int T) {
  if (!dp->sink) return;
  const int64_t base = 2 * dp->pair_base[c];
  for (int m = tid; m < (n >> 1); m += T) {
    dp->sink[base + 2 * m] = -1;
    dp->sink[base + 2 * m + 1] = -1;
  }
}

// One workgroup per cell of the (size-ordered) task list.  The task entry
// carries the cell's data pointers, so the loads of xi and v depend on one
// lookup only; the hardware dispatcher starts the next cell's workgroup as
// soon as one finishes (largest cells first).
template <int CAP, int W, bool ADAPT>
__global__ void __launch_bounds__(64 * W) k_cells(const SimDesc* __restrict__ descs,
                                                  const CellTask* __restrict__ tasks,
                                                  uint32_t k_abs, int nsteps,
                                                  uint32_t* __restrict__ order_flag) {
  constexpr int T = 64 * W;
  constexpr int IT = (CAP + T - 1) / T;
  __shared__ CellLds<CAP> L;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const CellTask cur = tasks[blockIdx.x];
  const int n = cur.n;
  // all loads first (coalesced, slot = T it + tid)
  long long xr[IT];
  double vr[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = it * T + tid;
    xr[it] = 0;
    vr[it] = 0.0;
    if (it * T < n && j < n) {
      xr[it] = cur.xi[j];
      vr[it] = cur.v[j];
    }
  }
  const int c = cur.cell;
  const SimDesc* dp = descs + cur.sim;
  const int64_t o0 = cur.xi - dp->xi;
  const uint32_t s0 = k_abs + dp->step_delta;
  if (s0 >= dp->step_limit) {  // uniform over the block
    if (ADAPT && tid == 0) order_flag[blockIdx.x] = order_group(0);
    return;
  }
  const int kind = dp->kernel;
  // Several steps in one launch (nsteps > 1) keep the cell in LDS from step
  // to step; each step is exactly the single step it replaces.
  const bool in_lds = ADAPT || nsteps > 1;
  if (in_lds)
    for (int k = tid; k < CAP / 32; k += T) L.dirty[k] = 0;
  int mylive = 0;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = it * T + tid;
    if (it * T < n && j < n) {
      L.xd[j] = (double)xr[it];
      L.rs[j] = xr[it] > 0 ? size_of(kind, vr[it]) : 0.0;
      mylive += xr[it] > 0 ? 1 : 0;
    }
  }
  const int nlive = team_sum<W>(L, mylive, lane, wv);  // also orders the LDS stores

  PairRegs<sort_rounds<CAP, W>(), slots_per_thread<CAP, W>()> R;
  int ncoll = 0;
  unsigned long long live_sum = 0, nsub = 0, steps_done = 0;
  if (!in_lds) {  // one plain step: updates go straight to global memory
    if (nlive >= 2) {
      team_sort<CAP, W>(L, n, nlive, tid, lane, wv, c, s0, 0u, dp->seed_lo, dp->seed_hi);
      team_pairs<CAP, W, kPassPlain>(L, dp, cur.v, n, nlive, tid, c, s0, 0u, dp->q, false, o0,
                                     &ncoll, R);
    } else {
      sink_clear_cell(dp, c, n, tid, T);
    }
    live_sum = (unsigned long long)nlive;
    nsub = 1;
    steps_done = 1;
  } else {
    int nl = nlive;  // live SDs: a step only empties slots by multiplicity-1 splits
    for (int t = 0; t < nsteps; ++t) {
      const uint32_t s = s0 + (uint32_t)t;
      if (s >= dp->step_limit) break;  // uniform over the block
      live_sum += (unsigned long long)nl;
      steps_done += 1;
      if (!ADAPT) {
        if (nl >= 2) {
          team_sort<CAP, W>(L, n, nl, tid, lane, wv, c, s, 0u, dp->seed_lo, dp->seed_hi);
          int ndead = 0;
          team_pairs<CAP, W, kPassPlainLds>(L, dp, cur.v, n, nl, tid, c, s, 0u, dp->q, false, o0,
                                            &ncoll, R, &ndead);
          nl -= team_sum<W>(L, ndead, lane, wv);
        } else {
          sink_clear_cell(dp, c, n, tid, T);
        }
        nsub += 1;
      } else {
        // Per-cell substepping: the substep length keeps every p <= 1 (p is
        // clamped to 1), so gamma <= 1.  After max_substeps substeps the rest
        // of the step is done in one unclamped substep and SUBSTEP_CAP is
        // raised.
        const double dv = dp->dv;
        double dt_left = dp->dt;
        uint32_t u = 0;
        const uint32_t umax = (uint32_t)dp->max_substeps;
        while (dt_left > 0.0) {
          const bool capped = u >= umax;
          if (capped && tid == 0) atomicOr(dp->status, kFlagSubstepCap);
          if (nl < 2) {
            if (capped) {
              sink_clear_cell(dp, c, n, tid, T);
              u += 1;
            }
            break;
          }
          team_sort<CAP, W>(L, n, nl, tid, lane, wv, c, s, u, dp->seed_lo, dp->seed_hi);
          double pmax = team_pairs<CAP, W, kPassPmax>(L, dp, cur.v, n, nl, tid, c, s, u,
                                                      dt_left / dv, false, o0, &ncoll, R);
          pmax = team_max<W>(L, pmax, lane, wv);
          const double dt_sub = (capped || pmax <= 1.0) ? dt_left : dt_left / pmax;
          int ndead = 0;
          team_pairs<CAP, W, kPassAdapt>(L, dp, cur.v, n, nl, tid, c, s, u, dt_sub / dv, !capped,
                                         o0, &ncoll, R, &ndead);
          nl -= team_sum<W>(L, ndead, lane, wv);
          // the next substep's volume and attribute loads come from this
          // same workgroup: one CU, one vector L1, so ordering the stores
          // before them is all it takes
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
          team_sync<W>();
          dt_left = (dt_sub == dt_left) ? 0.0 : dt_left - dt_sub;
          u += 1;
          if (capped) break;
        }
        if (u == 0) sink_clear_cell(dp, c, n, tid, T);
        nsub += u;
      }
      // this step's volume and attribute updates before the next step's
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      team_sync<W>();
    }
    if (ADAPT && tid == 0)  // next launch's dispatch order: substeps per step
      order_flag[blockIdx.x] =
          order_group((uint32_t)((nsub + steps_done - 1) / (steps_done ? steps_done : 1)));
    team_sync<W>();
    // write back the multiplicities that changed (volumes are already there)
    for (int j = tid; j < n; j += T)
      if ((L.dirty[j >> 5] >> (j & 31)) & 1u) cur.xi[j] = (long long)L.xd[j];
  }
  ncoll = team_sum<W>(L, ncoll, lane, wv);
  if (tid == 0) add_stats(dp->stats, live_sum, (unsigned long long)ncoll, nsub, steps_done);
}

// ---------------------------------------------------------------------------
// Mid-size cells (512 < n <= CAP, CAP up to 16384 slots): one workgroup of W
// waves per cell.  Only the sort scratch lives in LDS (8 B per slot); xi and
// v stay in global memory, where the pair gathers hit the caches that the
// sort pass has just filled, and updates are written in place.  Adaptive
// substeps re-read the cell after a workgroup-scope fence.
// ---------------------------------------------------------------------------
template <int CAP>
struct alignas(16) MidLds {
  uint32_t tmp[CAP];      // bucketed (key << nbits | slot), then uint16 permutation
  uint32_t cnt[CAP + 4];  // bucket counters / starts, then double pre-products
  int red_i[16];
  double red_d[16];
};

constexpr int mid_waves(int cap) { return cap / 256 < 16 ? cap / 256 : 16; }

// keys, liveness (from global xi), count, scan, scatter, rank; returns the
// number of live SDs (uniform); the permutation is valid when it is >= 2
template <int CAP, int W>
__device__ __forceinline__ int mid_sort(MidLds<CAP>& L, const int64_t* xi, int n, int tid,
                                        int lane, int wv, int c, uint32_t s, uint32_t u,
                                        uint32_t k0, uint32_t k1) {
  constexpr int T = 64 * W;
  constexpr int I4 = (CAP + 4 * T - 1) / (4 * T);
  const int nbits = 32 - __clz(n - 1);
  const int nb = 1 << nbits;
  const int sh = 32 - nbits;
  for (int i = 4 * tid; i < nb + 4; i += 4 * T)  // counters 0..nb, 16 bytes at a time
    *reinterpret_cast<uint4*>(&L.cnt[i]) = make_uint4(0u, 0u, 0u, 0u);
  __syncthreads();
  uint32_t kr[I4][4], pos[I4][4];
  uint32_t live[I4];
  int mylive = 0;
#pragma unroll
  for (int i = 0; i < I4; ++i) {
    const int g = T * i + tid;
    live[i] = 0;
    if (4 * g < n) {
      long long xv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) xv[e] = (4 * g + e < n) ? xi[4 * g + e] : 0;
      const uint4 w = philox(make_uint4((uint32_t)g, (uint32_t)c, s, 2u * u), k0, k1);
      kr[i][0] = w.x;
      kr[i][1] = w.y;
      kr[i][2] = w.z;
      kr[i][3] = w.w;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (xv[e] > 0) {
          live[i] |= 1u << e;
          pos[i][e] = atomicAdd(&L.cnt[kr[i][e] >> sh], 1u);
          ++mylive;
        }
      }
    }
  }
  const int nlive = team_sum_r<W>(L.red_i, mylive, lane, wv);  // also a barrier
  if (nlive < 2) return nlive;
  {  // exclusive scan of the nb counters over the workgroup
    const int per = nb >= T ? nb / T : 1;
    const int first = tid * per;
    int local = scan_load(L.cnt, first, per, nb);
    int run = wave_excl_scan(local, lane);
    if (lane == 63) L.red_i[wv] = run + local;
    __syncthreads();
    for (int k = 0; k < wv; ++k) run += L.red_i[k];
    __syncthreads();
    scan_store(L.cnt, first, per, nb, run);
    if (tid == 0) L.cnt[nb] = (uint32_t)nlive;
  }
  __syncthreads();
  uint32_t st[I4][4], len[I4][4];
  int maxlen = 0;
#pragma unroll
  for (int i = 0; i < I4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      len[i][e] = 0;
      if ((live[i] >> e) & 1) {
        const uint32_t b = kr[i][e] >> sh;
        st[i][e] = L.cnt[b];
        len[i][e] = L.cnt[b + 1] - st[i][e];
        L.tmp[st[i][e] + pos[i][e]] = (kr[i][e] << nbits) | (uint32_t)(4 * (T * i + tid) + e);
        maxlen = max(maxlen, (int)len[i][e]);
      }
    }
  __syncthreads();
  uint32_t rk[I4][4];
#pragma unroll
  for (int i = 0; i < I4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) rk[i][e] = st[i][e];
  for (int k = 0; k < maxlen; ++k) {
#pragma unroll
    for (int i = 0; i < I4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if ((uint32_t)k < len[i][e]) {
          const uint32_t me = (kr[i][e] << nbits) | (uint32_t)(4 * (T * i + tid) + e);
          rk[i][e] += (L.tmp[st[i][e] + k] < me) ? 1u : 0u;
        }
      }
  }
  __syncthreads();
  uint16_t* perm = reinterpret_cast<uint16_t*>(L.tmp);
#pragma unroll
  for (int i = 0; i < I4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if ((live[i] >> e) & 1) perm[rk[i][e]] = (uint16_t)(4 * (T * i + tid) + e);
  __syncthreads();
  return nlive;
}

template <int CAP, int W, int MODE>
__device__ __forceinline__ double mid_pairs(MidLds<CAP>& L, const SimDesc* dp, int64_t* xi,
                                            double* v, int n, int nlive, int tid, int c,
                                            uint32_t s, uint32_t u, double q, bool clamp,
                                            int64_t o0, int* ncoll) {
  constexpr int T = 64 * W;
  constexpr int I4 = (CAP + 4 * T - 1) / (4 * T);
  const int P = nlive >> 1;
  const double S = (double)((nlive & 1) ? nlive : nlive - 1);
  double* pre = reinterpret_cast<double*>(L.cnt);
  const uint16_t* perm = reinterpret_cast<const uint16_t*>(L.tmp);
  double pmax = 0.0;
  int64_t* sink = (MODE == kPassPmax) ? nullptr : dp->sink;
  const int64_t sink_base = sink ? 2 * dp->pair_base[c] : 0;
#pragma unroll
  for (int i = 0; i < I4; ++i) {
    const int h = T * i + tid;
    if (2 * h >= P) continue;
    const uint2 o4 = *reinterpret_cast<const uint2*>(&perm[4 * h]);
    const int aa[2] = {(int)(o4.x & 0xFFFFu), (int)(o4.y & 0xFFFFu)};
    const int bs[2] = {(int)(o4.x >> 16), (int)(o4.y >> 16)};
    uint4 w = make_uint4(0, 0, 0, 0);
    if (MODE != kPassPmax) w = philox(make_uint4((uint32_t)h, (uint32_t)c, s, 2u * u + 1u),
                                      dp->seed_lo, dp->seed_hi);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int m = 2 * h + e;
      if (m >= P) break;
      const int a = aa[e], bb = bs[e];
      const long long xa = xi[a], xb = xi[bb];
      const double va = v[a], vb = v[bb];
      double p;
      if (MODE == kPassAdapt) {
        p = pre[m] * q;
      } else {
        const double kv = coal_kernel(dp->kernel, dp->b, va, vb);
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
        update_pair(xi, v, a, bb, xa, xb, va, vb, gamma, dp->attrs, dp->n_slots, dp->n_attr,
                    o0 + a, o0 + bb);
      }
    }
  }
  if (sink && MODE != kPassPmax) {
    for (int m = P + tid; m < (n >> 1); m += T) {
      sink[sink_base + 2 * m] = -1;
      sink[sink_base + 2 * m + 1] = -1;
    }
  }
  __syncthreads();
  return pmax;
}

template <int CAP, int W, bool ADAPT>
__global__ void __launch_bounds__(64 * W) k_cells_mid(const SimDesc* __restrict__ descs,
                                                      const CellTask* __restrict__ tasks,
                                                      uint32_t k_abs) {
  constexpr int T = 64 * W;
  extern __shared__ __align__(16) unsigned char smem[];
  MidLds<CAP>& L = *reinterpret_cast<MidLds<CAP>*>(smem);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const CellTask ct = tasks[blockIdx.x];
  const SimDesc* dp = descs + ct.sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;  // uniform over the block
  const int n = ct.n;
  const int c = ct.cell;
  int64_t* xi = ct.xi;
  double* v = ct.v;
  const int64_t o0 = xi - dp->xi;
  int ncoll = 0;
  int nsub = 1;
  int nlive0 = 0;
  if (!ADAPT) {
    const int nl = mid_sort<CAP, W>(L, xi, n, tid, lane, wv, c, s, 0u, dp->seed_lo, dp->seed_hi);
    nlive0 = nl;
    if (nl >= 2)
      mid_pairs<CAP, W, kPassPlain>(L, dp, xi, v, n, nl, tid, c, s, 0u, dp->q, false, o0,
                                    &ncoll);
    else
      sink_clear_cell(dp, c, n, tid, T);
  } else {
    const double dv = dp->dv;
    double dt_left = dp->dt;
    uint32_t u = 0;
    const uint32_t umax = (uint32_t)dp->max_substeps;
    while (dt_left > 0.0) {
      const bool capped = u >= umax;
      if (capped && tid == 0) atomicOr(dp->status, kFlagSubstepCap);
      const int nl = mid_sort<CAP, W>(L, xi, n, tid, lane, wv, c, s, u, dp->seed_lo,
                                      dp->seed_hi);
      if (u == 0) nlive0 = nl;
      if (nl < 2) {
        if (capped) {
          sink_clear_cell(dp, c, n, tid, T);
          u += 1;
        }
        break;
      }
      double pmax = mid_pairs<CAP, W, kPassPmax>(L, dp, xi, v, n, nl, tid, c, s, u,
                                                 dt_left / dv, false, o0, &ncoll);
      pmax = team_max_r<W>(L.red_d, pmax, lane, wv);
      const double dt_sub = (capped || pmax <= 1.0) ? dt_left : dt_left / pmax;
      mid_pairs<CAP, W, kPassAdapt>(L, dp, xi, v, n, nl, tid, c, s, u, dt_sub / dv, !capped, o0,
                                    &ncoll);
      // updates of this substep are read by other threads of this workgroup next
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __syncthreads();
      dt_left = (dt_sub == dt_left) ? 0.0 : dt_left - dt_sub;
      u += 1;
      if (capped) break;
    }
    if (u == 0) sink_clear_cell(dp, c, n, tid, T);
    nsub = (int)u;
  }
  ncoll = team_sum_r<W>(L.red_i, ncoll, lane, wv);
  if (tid == 0) add_stats(dp->stats, (unsigned long long)nlive0, (unsigned long long)ncoll,
                          (unsigned long long)nsub);
}

// ---------------------------------------------------------------------------
// Big cells (above the mid-size limit): two launches per step.
//
// k_big_keys: one block per chunk of a cell's slots.  Every live slot's key
// goes to bucket floor(key nb / 2^32) of its cell (nb buckets, a monotone
// map of the key, so buckets are key ranges in order).  The block counts its
// chunk per bucket in LDS, turns the counts into the chunk's own bucket
// offsets (stored: nb + 1 words, the last one the chunk's live count) and
// writes each entry (key << 32 | slot), with the slot's multiplicity and
// volume, at its place in the chunk's segment of the entry arrays.  No
// global atomics and no capacity: a segment holds exactly its chunk's live
// slots.
// k_big_bucket: one workgroup per bucket.  From the offsets of every chunk it
// takes the bucket's first position in the cell's permutation (the entries
// of all chunks in the buckets before it), its length and the cell's live
// count; it gathers the bucket's entries from the chunk segments, orders
// them in LDS (a sub-bucket scatter on the key's position inside the bucket
// range, then an exact rank inside each sub-bucket), and takes every pair
// whose first member sits at an even position of the permutation: the
// partner is the next entry, or, for the last one, the smallest entry of
// the next non-empty bucket, gathered in the same pass.  Multiplicities and
// volumes travel with the entries, so the pairs need no state reads (only
// attributes are read back).  A bucket longer than the LDS stage is ranked in
// global memory instead (exact, slow, flagged).
// ---------------------------------------------------------------------------
constexpr int kBigKeyThreads = 256;
constexpr int kBigThreads = 256;
constexpr int kBigSortCap = 1024;  // entries one workgroup orders in LDS
constexpr int kBigPer = kBigSortCap / kBigThreads;
static_assert(kBigChunkUnit == 4 * kBigKeyThreads, "a Philox round covers one chunk unit");
static_assert(kBigMaxChunks == kBigThreads, "one chunk per thread of a bucket workgroup");

__device__ __forceinline__ uint32_t key_bucket(uint32_t key, uint32_t nb) {
  return (uint32_t)(((unsigned long long)key * nb) >> 32);
}

// exclusive scan of h[0, n) in place (n <= kBigMaxBuckets), h[n] = total;
// each thread a contiguous run, fixed order
__device__ void chunk_scan(uint32_t* h, int n, int* red) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int R = (n + kBigKeyThreads - 1) / kBigKeyThreads;
  const int a = min(tid * R, n), e = min(a + R, n);
  int local = 0;
  for (int i = a; i < e; ++i) local += (int)h[i];
  int run = wave_excl_scan(local, lane);
  if (lane == 63) red[wv] = run + local;
  __syncthreads();
  for (int k = 0; k < wv; ++k) run += red[k];
  if (tid == kBigKeyThreads - 1) h[n] = (uint32_t)(run + local);
  for (int i = a; i < e; ++i) {
    const uint32_t c = h[i];
    h[i] = (uint32_t)run;
    run += (int)c;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBigKeyThreads) k_big_keys(
    const SimDesc* __restrict__ descs, const BigTask* __restrict__ big,
    const BigChunk* __restrict__ chunks, uint32_t* __restrict__ offs,
    unsigned long long* __restrict__ ekey, long long* __restrict__ exi,
    double* __restrict__ ev, uint32_t k_abs, const BigAdapt* __restrict__ astate) {
  // the bucket histogram: nb + 1 words, nb the largest bucket count of the
  // launch's cells (dynamic LDS, up to kBigMaxBuckets + 1 words)
  extern __shared__ uint32_t hist[];
  __shared__ int red[kBigKeyThreads / 64];
  const BigChunk ch = chunks[blockIdx.x];
  const BigTask tk = big[ch.task];
  const SimDesc* dp = descs + ch.sim;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  uint32_t u = 0;  // substep (adaptive cells: this round's, from the cell's state)
  if (astate) {
    const BigAdapt as = astate[ch.task];
    if (as.done) return;
    u = as.u;
  }
  const int tid = threadIdx.x;
  const uint32_t nb = (uint32_t)tk.nb;
  const int first = ch.index * tk.chunk_slots;
  const int last = min(first + tk.chunk_slots, tk.n_slots);
  for (uint32_t i = tid; i <= nb; i += kBigKeyThreads) hist[i] = 0;
  __syncthreads();
  const int64_t seg = tk.tmp_base + first;  // this chunk's segment
  uint32_t* o = offs + tk.off_base + (int64_t)ch.index * (nb + 1u);
  if (tk.chunk_slots == kBigChunkUnit) {
    // one Philox group of 4 slots per thread: places and values in registers
    const int j0 = first + 4 * tid;
    long long xv[4] = {0, 0, 0, 0};
    double vv[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t kk[4] = {0u, 0u, 0u, 0u}, bkt[4] = {0u, 0u, 0u, 0u};
    uint32_t pos[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    if (j0 < last) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (j0 + e < last) {
          xv[e] = tk.xi[j0 + e];
          vv[e] = tk.v[j0 + e];
        }
      const uint4 w = philox(make_uint4((uint32_t)(j0 >> 2), (uint32_t)tk.cell, s, 2u * u),
                             dp->seed_lo, dp->seed_hi);
      kk[0] = w.x;
      kk[1] = w.y;
      kk[2] = w.z;
      kk[3] = w.w;
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (xv[e] > 0) {
          bkt[e] = key_bucket(kk[e], nb);
          pos[e] = atomicAdd(&hist[bkt[e]], 1u);
        }
    }
    __syncthreads();
    chunk_scan(hist, (int)nb, red);
    for (uint32_t i = tid; i <= nb; i += kBigKeyThreads) o[i] = hist[i];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (pos[e] != 0xFFFFFFFFu) {
        const int64_t at = seg + hist[bkt[e]] + pos[e];
        ekey[at] = ((unsigned long long)kk[e] << 32) | (uint32_t)(j0 + e);
        exi[at] = xv[e];
        ev[at] = vv[e];
      }
    return;
  }
  // several groups per thread: count, then recompute the keys and place
  for (int j0 = first + 4 * tid; j0 < last; j0 += 4 * kBigKeyThreads) {
    long long xv[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (j0 + e < last) xv[e] = tk.xi[j0 + e];
    const uint4 w = philox(make_uint4((uint32_t)(j0 >> 2), (uint32_t)tk.cell, s, 2u * u),
                           dp->seed_lo, dp->seed_hi);
    const uint32_t kk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (xv[e] > 0) atomicAdd(&hist[key_bucket(kk[e], nb)], 1u);
  }
  __syncthreads();
  chunk_scan(hist, (int)nb, red);
  for (uint32_t i = tid; i <= nb; i += kBigKeyThreads) o[i] = hist[i];
  __syncthreads();  // the starts are read before they turn into cursors
  for (int j0 = first + 4 * tid; j0 < last; j0 += 4 * kBigKeyThreads) {
    long long xv[4] = {0, 0, 0, 0};
    double vv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (j0 + e < last) {
        xv[e] = tk.xi[j0 + e];
        vv[e] = tk.v[j0 + e];
      }
    const uint4 w = philox(make_uint4((uint32_t)(j0 >> 2), (uint32_t)tk.cell, s, 2u * u),
                           dp->seed_lo, dp->seed_hi);
    const uint32_t kk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (xv[e] > 0) {
        const int64_t at = seg + atomicAdd(&hist[key_bucket(kk[e], nb)], 1u);
        ekey[at] = ((unsigned long long)kk[e] << 32) | (uint32_t)(j0 + e);
        exi[at] = xv[e];
        ev[at] = vv[e];
      }
  }
}

struct alignas(16) BigLds {
  unsigned long long ent[kBigSortCap];  // keys in sub-bucket order
  long long exi[kBigSortCap];           // gathered multiplicities, volumes, slots
  double ev[kBigSortCap];
  uint32_t slot[kBigSortCap];
  uint32_t sc[kBigSortCap + 4];  // sub-bucket counters / starts
  uint32_t ord[kBigSortCap];     // gathered entries in permutation order
  // gathered index -> chunk, for this bucket and for the partner's bucket
  uint16_t own[kBigSortCap], own1[kBigSortCap];
  // per chunk: first gathered index (exclusive scan) and segment start, of
  // this bucket (cs, cb) and of the bucket that holds the partner (cs1, cb1)
  uint32_t cs[kBigMaxChunks + 1], cb[kBigMaxChunks];
  uint32_t cs1[kBigMaxChunks + 1], cb1[kBigMaxChunks];
  // colliding pairs of one round of kBigThreads pairs (attribute updates):
  // slots j, k (the larger multiplicity first), g, equal split
  uint32_t lj[kBigThreads], lk[kBigThreads], lsplit[kBigThreads];
  long long lg[kBigThreads];
  int nlist;
  int red[kBigThreads / 64][4];
  unsigned long long red64[kBigThreads / 64];
  unsigned long long pkey;  // partner of the last entry: the next bucket's smallest entry
  long long pxi;
  double pv;
};

// exclusive scan of one value per thread over the workgroup (fixed order)
__device__ __forceinline__ int block_excl_scan(BigLds& L, int x, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int e = wave_excl_scan(x, lane);
  if (lane == 63) L.red[wv][0] = e + x;
  __syncthreads();
  total = 0;
#pragma unroll
  for (int k = 0; k < kBigThreads / 64; ++k) {
    e += k < wv ? L.red[k][0] : 0;
    total += L.red[k][0];
  }
  __syncthreads();
  return e;
}

// workgroup sums of two values (fixed order)
__device__ __forceinline__ void block_sum2(BigLds& L, int& a, int& b) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    L.red[wv][1] = a;
    L.red[wv][2] = b;
  }
  __syncthreads();
  a = b = 0;
#pragma unroll
  for (int k = 0; k < kBigThreads / 64; ++k) {
    a += L.red[k][1];
    b += L.red[k][2];
  }
  __syncthreads();
}

// chunk of gathered index t: the last chunk i with cs[i] <= t (cs[0] = 0 <= t
// < cs[n])
__device__ __forceinline__ int chunk_of(const uint32_t* cs, int n, int t) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int)cs[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ADAPT: the first pass of an adaptive substep; instead of drawing the
// collisions it stores every pair's slots and pre-product (max xi K) S and
// raises the cell's largest p at the remaining time (k_abig_pairs draws).
template <bool ADAPT>
__global__ void __launch_bounds__(kBigThreads) k_big_bucket(
    const SimDesc* __restrict__ descs, const BigTask* __restrict__ big,
    const BigBucket* __restrict__ buckets, const uint32_t* __restrict__ offs,
    const unsigned long long* __restrict__ ekey, const long long* __restrict__ exi,
    const double* __restrict__ ev, unsigned long long* __restrict__ skey,
    uint32_t* __restrict__ gord, uint32_t k_abs, BigAdapt* __restrict__ astate,
    unsigned long long* __restrict__ apmax, double* __restrict__ apre,
    unsigned long long* __restrict__ apair) {
  __shared__ BigLds L;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const BigBucket bk = buckets[blockIdx.x];
  const BigTask tk = big[bk.task];
  const SimDesc* dp = descs + bk.sim;
  const int b = bk.bucket;
  const uint32_t s = k_abs + dp->step_delta;
  if (s >= dp->step_limit) return;
  double q_left = 0.0;
  if (ADAPT) {
    const BigAdapt as = astate[bk.task];
    if (as.done) return;
    q_left = as.dt_left / dp->dv;
  }
  const int nb = tk.nb, nch = tk.n_chunks;
  const int64_t tb = tk.tmp_base;
  // this thread's chunk: its offsets of buckets b, b + 1, b + 2 and its live count
  uint32_t o_b = 0, o_b1 = 0, o_b2 = 0;
  int before = 0, tot = 0;
  if (tid < nch) {
    const uint32_t* oc = offs + tk.off_base + (int64_t)tid * (nb + 1);
    o_b = oc[b];
    o_b1 = oc[b + 1];
    o_b2 = oc[min(b + 2, nb)];
    tot = (int)oc[nb];
    before = (int)o_b;
  }
  const int lb = (int)(o_b1 - o_b);
  int len = 0;
  const int e0 = block_excl_scan(L, lb, len);
  block_sum2(L, before, tot);
  const int start = before, nlive = tot;
  const int P = nlive >> 1;
  const int c = tk.cell;
  if (ADAPT && b == 0 && tid == 0) astate[bk.task].nlive = nlive;
  int64_t* sink = ADAPT ? nullptr : dp->sink;
  const int64_t sink_base = sink ? 2 * dp->pair_base[c] : 0;
  if (sink && b == 0)  // unused pair entries of the cell
    for (int m = P + tid; m < (tk.n_slots >> 1); m += kBigThreads) {
      sink[sink_base + 2 * m] = -1;
      sink[sink_base + 2 * m + 1] = -1;
    }
  // first entry whose pair this bucket takes, and whether any pair is taken
  const int i0 = start & 1;
  const bool any_pair = len > i0 && (start + i0) / 2 < P;
  const bool need_next = any_pair && ((start + len) & 1) && (start + len - 1) / 2 < P;
  const bool fast = len <= min(tk.sort_cap, kBigSortCap);
  uint32_t* gsorted = gord + tb + start;  // slow path: slots in order
  if (tid == 0) L.nlist = 0;
  if (any_pair) {
    // the partner's bucket: b + 1, else the next non-empty one
    int len1 = 0, e1 = 0;
    uint32_t p_lo = o_b1;
    int l1 = tid < nch ? (int)(o_b2 - o_b1) : 0;
    if (need_next) {
      e1 = block_excl_scan(L, l1, len1);
      for (int nbk = b + 2; len1 == 0 && nbk < nb; ++nbk) {
        uint32_t hi = 0;
        p_lo = 0;
        if (tid < nch) {
          const uint32_t* oc = offs + tk.off_base + (int64_t)tid * (nb + 1);
          p_lo = oc[nbk];
          hi = oc[nbk + 1];
        }
        l1 = (int)(hi - p_lo);
        e1 = block_excl_scan(L, l1, len1);
      }
    }
    // per chunk: where its entries start, and which gathered indices it holds
    if (tid < nch) {
      L.cs[tid] = (uint32_t)e0;
      L.cb[tid] = o_b;
      L.cs1[tid] = (uint32_t)e1;
      L.cb1[tid] = p_lo;
      if (fast)
        for (int k = 0; k < lb; ++k) L.own[e0 + k] = (uint16_t)tid;
      if (need_next)
        for (int k = 0; k < l1 && e1 + k < kBigSortCap; ++k) L.own1[e1 + k] = (uint16_t)tid;
    }
    if (tid == 0) {
      L.cs[nch] = (uint32_t)len;
      L.cs1[nch] = (uint32_t)len1;
    }
    __syncthreads();
    // one round of loads: the bucket's entries (fast path) and the partner
    // bucket's first kBigSortCap entries
    unsigned long long me[kBigPer], pk[kBigPer];
    long long mx[kBigPer], px[kBigPer];
    double mv[kBigPer], pv[kBigPer];
#pragma unroll
    for (int r = 0; r < kBigPer; ++r) {
      const int t = r * kBigThreads + tid;
      me[r] = 0;
      mx[r] = 0;
      mv[r] = 0.0;
      if (fast && t < len) {
        const int i = L.own[t];
        const int64_t src = tb + (int64_t)i * tk.chunk_slots + L.cb[i] + (t - (int)L.cs[i]);
        me[r] = ekey[src];
        mx[r] = exi[src];
        mv[r] = ev[src];
      }
      pk[r] = ~0ull;
      px[r] = 0;
      pv[r] = 0.0;
      if (need_next && t < len1) {
        const int i = L.own1[t];
        const int64_t src = tb + (int64_t)i * tk.chunk_slots + L.cb1[i] + (t - (int)L.cs1[i]);
        pk[r] = ekey[src];
        px[r] = exi[src];
        pv[r] = ev[src];
      }
    }
    if (need_next) {  // the partner: the smallest entry of its bucket
      unsigned long long m = ~0ull;
      long long mxx = 0;
      double mvv = 0.0;
#pragma unroll
      for (int r = 0; r < kBigPer; ++r)
        if (pk[r] < m) {
          m = pk[r];
          mxx = px[r];
          mvv = pv[r];
        }
      for (int t = kBigSortCap + tid; t < len1; t += kBigThreads) {  // a long partner bucket
        const int i = chunk_of(L.cs1, nch, t);
        const int64_t src = tb + (int64_t)i * tk.chunk_slots + L.cb1[i] + (t - (int)L.cs1[i]);
        const unsigned long long k = ekey[src];
        if (k < m) {
          m = k;
          mxx = exi[src];
          mvv = ev[src];
        }
      }
      unsigned long long w = m;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) w = min(w, (unsigned long long)__shfl_xor(w, o));
      if (lane == 0) L.red64[wv] = w;
      __syncthreads();
      unsigned long long r = ~0ull;
#pragma unroll
      for (int k = 0; k < kBigThreads / 64; ++k) r = min(r, L.red64[k]);
      if (m == r && r != ~0ull) {  // entries are distinct: one thread holds it
        L.pkey = m;
        L.pxi = mxx;
        L.pv = mvv;
      }
    }
    if (fast) {
      // order in LDS: sub-buckets on the key's place inside this bucket's key
      // range, then an exact rank inside each sub-bucket
      const int sbits = len <= 1 ? 0 : 32 - __clz(len - 1);
      const int nsb = 1 << sbits;
      // scale < 2^(31 + 10): the product with a 32-bit key needs 128 bits
      const unsigned long long scale = (unsigned long long)(uint32_t)nb << sbits;
      for (int i = tid; i < nsb + 1; i += kBigThreads) L.sc[i] = 0;
      uint32_t sub[kBigPer], pos[kBigPer];
#pragma unroll
      for (int r = 0; r < kBigPer; ++r) {
        const int t = r * kBigThreads + tid;
        if (t < len) {
          L.exi[t] = mx[r];
          L.ev[t] = mv[r];
          L.slot[t] = (uint32_t)(me[r] & 0xFFFFFFFFull);
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kBigPer; ++r) {
        const int t = r * kBigThreads + tid;
        if (t < len) {
          // monotone in the key: (key nb 2^sbits) >> 32 = b 2^sbits + sub
          const unsigned long long key = me[r] >> 32;
          const unsigned long long lo = key * scale, hi = __umul64hi(key, scale);
          sub[r] = (uint32_t)((hi << 32) | (lo >> 32)) - ((uint32_t)b << sbits);
          pos[r] = atomicAdd(&L.sc[sub[r]], 1u);
        }
      }
      __syncthreads();
      int tot_sc = 0;
      {  // exclusive scan of the sub-bucket counters (4 per thread)
        const int f = 4 * tid;
        uint32_t c4[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) c4[e] = f + e < nsb ? L.sc[f + e] : 0u;
        int run = block_excl_scan(L, (int)(c4[0] + c4[1] + c4[2] + c4[3]), tot_sc);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (f + e < nsb) L.sc[f + e] = (uint32_t)run;
          run += (int)c4[e];
        }
        if (tid == 0) L.sc[nsb] = (uint32_t)tot_sc;
      }
      __syncthreads();
      uint32_t st[kBigPer], ln[kBigPer];
#pragma unroll
      for (int r = 0; r < kBigPer; ++r) {
        const int t = r * kBigThreads + tid;
        st[r] = ln[r] = 0;
        if (t < len) {
          st[r] = L.sc[sub[r]];
          ln[r] = L.sc[sub[r] + 1] - st[r];
          L.ent[st[r] + pos[r]] = me[r];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kBigPer; ++r) {
        const int t = r * kBigThreads + tid;
        if (t < len) {
          uint32_t rk = st[r];
          for (uint32_t k = 0; k < ln[r]; ++k) rk += L.ent[st[r] + k] < me[r] ? 1u : 0u;
          L.ord[rk] = (uint32_t)t;
        }
      }
    } else {  // slow path: rank every entry against the whole bucket in global memory
      if (tid == 0) atomicOr(dp->status, kFlagBucketOverflow);
      unsigned long long* sk = skey + tb + start;
      for (int t = tid; t < len; t += kBigThreads) {
        const int i = chunk_of(L.cs, nch, t);
        sk[t] = ekey[tb + (int64_t)i * tk.chunk_slots + L.cb[i] + (t - (int)L.cs[i])];
      }
      __threadfence_block();
      __syncthreads();
      for (int t = tid; t < len; t += kBigThreads) {
        const unsigned long long e = sk[t];
        uint32_t rk = 0;
        for (int k = 0; k < len; ++k) rk += sk[k] < e ? 1u : 0u;
        gsorted[rk] = (uint32_t)(e & 0xFFFFFFFFull);
      }
      __threadfence_block();
    }
  }
  __syncthreads();
  // the i-th entry of the bucket's order (i == len: the partner)
  int64_t* xi = tk.xi;
  double* v = tk.v;
  auto fetch = [&](int i, int& slot, long long& x, double& vol) {
    if (i == len) {
      slot = (int)(uint32_t)(L.pkey & 0xFFFFFFFFull);
      x = L.pxi;
      vol = L.pv;
    } else if (fast) {
      const int g = (int)L.ord[i];
      slot = (int)L.slot[g];
      x = L.exi[g];
      vol = L.ev[g];
    } else {
      slot = (int)gsorted[i];
      x = xi[slot];
      vol = v[slot];
    }
  };
  // pairs: positions start + i with i = i0, i0 + 2, ...; rounds of
  // kBigThreads pairs, each followed by the attribute updates of its collisions
  int ncoll = 0;
  const double S = (double)((nlive & 1) ? nlive : nlive - 1);
  const int64_t o0 = tk.xi - dp->xi;
  const int npairs = any_pair ? min((len - i0 + 1) >> 1, P - ((start + i0) >> 1)) : 0;
  if (ADAPT) {  // pre-products, pairs and this bucket's largest p at the remaining time
    double pm = 0.0;
    for (int t = tid; t < npairs; t += kBigThreads) {
      const int i = i0 + 2 * t;
      const int m = (start + i) >> 1;
      int a, bb;
      long long xa, xb;
      double va, vb;
      fetch(i, a, xa, va);
      fetch(i + 1, bb, xb, vb);
      const double kv = coal_kernel(dp->kernel, dp->b, va, vb);
      const double pp = ((double)(xa > xb ? xa : xb) * kv) * S;
      apre[tb + m] = pp;
      apair[tb + m] = (unsigned long long)(uint32_t)a | ((unsigned long long)bb << 32);
      pm = fmax(pm, pp * q_left);
    }
    // largest p of the block; p >= 0, so its bits order like the values
    unsigned long long pb = (unsigned long long)__double_as_longlong(pm);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) pb = max(pb, (unsigned long long)__shfl_xor(pb, o));
    if (lane == 0) L.red64[wv] = pb;
    __syncthreads();
    if (tid == 0) {
      unsigned long long r = 0;
#pragma unroll
      for (int k = 0; k < kBigThreads / 64; ++k) r = max(r, L.red64[k]);
      if (r) atomicMax(&apmax[bk.task], r);
    }
    return;
  }
  const int A = dp->n_attr;
  for (int base = 0; base < npairs; base += kBigThreads) {
    const int t = base + tid;
    if (t < npairs) {
      const int i = i0 + 2 * t;
      const int m = (start + i) >> 1;
      int a, bb;
      long long xa, xb;
      double va, vb;
      fetch(i, a, xa, va);
      fetch(i + 1, bb, xb, vb);
      const double kv = coal_kernel(dp->kernel, dp->b, va, vb);
      const double p = (((double)(xa > xb ? xa : xb) * kv) * S) * dp->q;
      const uint4 w = philox(make_uint4((uint32_t)(m >> 1), (uint32_t)c, s, 1u), dp->seed_lo,
                             dp->seed_hi);
      const double phi = (m & 1) == 0 ? uniform53(w.x, w.y) : uniform53(w.z, w.w);
      const long long gamma = collisions(p, phi, dp->status);
      if (sink) {
        sink[sink_base + 2 * m] = (int64_t)((uint64_t)a | ((uint64_t)bb << 32));
        sink[sink_base + 2 * m + 1] = gamma;
      }
      if (gamma > 0) {  // multiplicities and volumes now, attributes listed
        ++ncoll;
        const bool a_is_j = xa >= xb;  // ties: the pair's first member
        const long long xj = a_is_j ? xa : xb, xk = a_is_j ? xb : xa;
        const double vj = a_is_j ? va : vb, vk = a_is_j ? vb : va;
        long long g = gamma;
        if (g > 1) {
          const long long ratio = xj / xk;
          g = g < ratio ? g : ratio;
        }
        const int j = a_is_j ? a : bb, k = a_is_j ? bb : a;
        const long long rest = xj - g * xk;
        const double vn = fma((double)g, vj, vk);
        uint32_t split = 0;
        v[k] = vn;
        if (rest > 0) {
          xi[j] = rest;
        } else {  // equal-multiplicity split
          const long long h = xk >> 1;
          xi[j] = h;
          xi[k] = xk - h;
          v[j] = vn;
          split = 1;
        }
        if (A > 0) {
          const int at = atomicAdd(&L.nlist, 1);
          L.lj[at] = (uint32_t)j;
          L.lk[at] = (uint32_t)k;
          L.lsplit[at] = split;
          L.lg[at] = g;
        }
      }
    }
    if (A > 0) {  // attributes of the listed pairs: one round of loads
      __syncthreads();
      const int nl = L.nlist;
      for (int q = tid; q < nl * A; q += kBigThreads) {
        const int li = q / A, f = q - li * A;
        const int j = (int)L.lj[li], k = (int)L.lk[li];
        double* X = dp->attrs + (int64_t)f * dp->n_slots + o0;
        const double val = fma((double)L.lg[li], X[j], X[k]);
        X[k] = val;
        if (L.lsplit[li]) X[j] = val;
      }
      __syncthreads();
      if (tid == 0) L.nlist = 0;
      __syncthreads();
    }
  }
  ncoll = wave_sum(ncoll);
  if ((tid & 63) == 0) L.red[tid >> 6][3] = ncoll;
  __syncthreads();
  if (tid == 0) {
    int tc = 0;
#pragma unroll
    for (int k = 0; k < kBigThreads / 64; ++k) tc += L.red[k][3];
    unsigned long long* stt = dp->stats + (blockIdx.x % kStatSlots) * kStatFields;
    if (tc) atomicAdd(stt + 1, (unsigned long long)tc);
    if (b == 0) {  // once per cell and step
      atomicAdd(stt + 0, (unsigned long long)nlive);
      atomicAdd(stt + 2, 1ull);
      atomicAdd(stt + 3, 1ull);
    }
  }
}

// ---------------------------------------------------------------------------
// Adaptive substeps of big cells.  One outer step of the adaptive big cells
// is a sequence of rounds, each one substep of every cell not yet done:
// k_big_keys (keys of substep u), k_big_bucket<true> (order, pairs,
// pre-products, the cell's largest p at the remaining time dt_left) and
// k_abig_pairs (the substep length dt_left / pmax, or dt_left when pmax <= 1
// or the substep cap is reached; p at the substep clamped to 1 unless
// capped; gamma; updates; the cell's next state).  A cell's state has two
// copies: round r reads copy r mod 2 and writes the other (a cell already done
// copies its state over unchanged).
// ---------------------------------------------------------------------------
__global__ void k_abig_init(const SimDesc* __restrict__ descs, const BigTask* __restrict__ big,
                            const int* __restrict__ atask, int n, BigAdapt* __restrict__ st0,
                            unsigned long long* __restrict__ pm0,
                            unsigned long long* __restrict__ pm1, uint32_t k_abs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = atask[i];
  const SimDesc* dp = descs + big[t].sim;
  BigAdapt a;
  a.dt_left = dp->dt;
  a.u = 0;
  a.done = (k_abs + dp->step_delta >= dp->step_limit) ? 1u : 0u;
  a.nlive = 0;
  a.pad = 0;
  st0[t] = a;
  pm0[t] = 0;
  pm1[t] = 0;
}

__global__ void __launch_bounds__(kAbigPairs) k_abig_pairs(
    const SimDesc* __restrict__ descs, const BigTask* __restrict__ big,
    const BigPairBlock* __restrict__ pblocks, const BigAdapt* __restrict__ cur,
    BigAdapt* __restrict__ nxt, const unsigned long long* __restrict__ pm_cur,
    unsigned long long* __restrict__ pm_nxt, const double* __restrict__ apre,
    const unsigned long long* __restrict__ apair, uint32_t k_abs) {
  __shared__ uint32_t lj[kAbigPairs], lk[kAbigPairs], lsplit[kAbigPairs];
  __shared__ long long lg[kAbigPairs];
  __shared__ int nlist, red[kAbigPairs / 64];
  const int tid = threadIdx.x;
  const BigPairBlock pb = pblocks[blockIdx.x];
  const BigTask tk = big[pb.task];
  const BigAdapt as = cur[pb.task];
  if (as.done) {  // carried into the other copy, which the next round reads
    if (pb.first == 0 && tid == 0) {
      nxt[pb.task] = as;
      pm_nxt[pb.task] = 0;
    }
    return;
  }
  const SimDesc* dp = descs + tk.sim;
  const uint32_t s = k_abs + dp->step_delta;
  const uint32_t u = as.u;
  const bool capped = u >= (uint32_t)dp->max_substeps;
  if (capped && tid == 0 && pb.first == 0) atomicOr(dp->status, kFlagSubstepCap);
  const int nlive = as.nlive;
  const int P = nlive >> 1;
  const int c = tk.cell;
  const int m = pb.first + tid;
  int64_t* sink = dp->sink;
  const int64_t sink_base = sink ? 2 * dp->pair_base[c] : 0;
  if (tid == 0) nlist = 0;
  __syncthreads();
  double dt_sub = as.dt_left;
  int ncoll = 0;
  if (nlive >= 2) {
    const double pmax = __longlong_as_double((long long)pm_cur[pb.task]);
    dt_sub = (capped || pmax <= 1.0) ? as.dt_left : as.dt_left / pmax;
    const double q = dt_sub / dp->dv;
    if (m < P) {
      const unsigned long long pr = apair[tk.tmp_base + m];
      const int a = (int)(uint32_t)(pr & 0xFFFFFFFFull), bb = (int)(uint32_t)(pr >> 32);
      double p = apre[tk.tmp_base + m] * q;
      if (!capped && p > 1.0) p = 1.0;
      const uint4 w = philox(make_uint4((uint32_t)(m >> 1), (uint32_t)c, s, 2u * u + 1u),
                             dp->seed_lo, dp->seed_hi);
      const double phi = (m & 1) == 0 ? uniform53(w.x, w.y) : uniform53(w.z, w.w);
      const long long gamma = collisions(p, phi, dp->status);
      if (sink) {
        sink[sink_base + 2 * m] = (int64_t)((uint64_t)a | ((uint64_t)bb << 32));
        sink[sink_base + 2 * m + 1] = gamma;
      }
      if (gamma > 0) {
        ++ncoll;
        int64_t* xi = tk.xi;
        const long long xa = xi[a], xb = xi[bb];
        const bool a_is_j = xa >= xb;  // ties: the pair's first member
        const long long xj = a_is_j ? xa : xb, xk = a_is_j ? xb : xa;
        long long g = gamma;
        if (g > 1) {
          const long long ratio = xj / xk;
          g = g < ratio ? g : ratio;
        }
        const int j = a_is_j ? a : bb, k = a_is_j ? bb : a;
        const long long rest = xj - g * xk;
        uint32_t split = 0;
        if (rest > 0) {
          xi[j] = rest;
        } else {  // equal-multiplicity split
          const long long h = xk >> 1;
          xi[j] = h;
          xi[k] = xk - h;
          split = 1;
        }
        const int at = atomicAdd(&nlist, 1);
        lj[at] = (uint32_t)j;
        lk[at] = (uint32_t)k;
        lsplit[at] = split;
        lg[at] = g;
      }
    }
  }
  if (sink && m >= P && m < (tk.n_slots >> 1)) {  // no pair this substep
    sink[sink_base + 2 * m] = -1;
    sink[sink_base + 2 * m + 1] = -1;
  }
  __syncthreads();
  {  // volumes and attributes of the listed pairs: one round of loads
    const int nl = nlist;
    const int F = 1 + dp->n_attr;
    const int64_t o0 = tk.xi - dp->xi;
    for (int t = tid; t < nl * F; t += kAbigPairs) {
      const int li = t / F, f = t - li * F;
      const int j = (int)lj[li], k = (int)lk[li];
      double* X = f == 0 ? tk.v : dp->attrs + (int64_t)(f - 1) * dp->n_slots + o0;
      const double val = fma((double)lg[li], X[j], X[k]);
      X[k] = val;
      if (lsplit[li]) X[j] = val;
    }
  }
  ncoll = wave_sum(ncoll);
  if ((tid & 63) == 0) red[tid >> 6] = ncoll;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
#pragma unroll
    for (int k = 0; k < kAbigPairs / 64; ++k) tot += red[k];
    unsigned long long* stt = dp->stats + (blockIdx.x % kStatSlots) * kStatFields;
    if (tot) atomicAdd(stt + 1, (unsigned long long)tot);
    if (pb.first == 0) {  // the cell's next state, once
      BigAdapt na = as;
      if (nlive < 2) {  // no pairs: the step ends here (a capped substep still counts)
        na.u = u + (capped ? 1u : 0u);
        na.done = 1;
      } else {
        na.dt_left = (dt_sub == as.dt_left) ? 0.0 : as.dt_left - dt_sub;
        na.u = u + 1;
        na.done = (na.dt_left > 0.0 && !capped) ? 0u : 1u;
      }
      nxt[pb.task] = na;
      pm_nxt[pb.task] = 0;
      if (u == 0) {
        atomicAdd(stt + 0, (unsigned long long)nlive);
        atomicAdd(stt + 3, 1ull);
      }
      if (na.u > u) atomicAdd(stt + 2, (unsigned long long)(na.u - u));
    }
  }
}

// adaptive big cells still stepping after a round: *count (host-read)
__global__ void k_abig_active(const BigAdapt* __restrict__ st, const int* __restrict__ atask,
                              int n, uint32_t* __restrict__ count) {
  __shared__ int red[4];
  int live = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) live += st[atask[i]].done ? 0 : 1;
  live = wave_sum(live);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = live;
  __syncthreads();
  if (threadIdx.x == 0) *count = (uint32_t)(red[0] + red[1] + red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// Moments: one workgroup of W waves per cell, one pass over the cell's slots.
// Each thread accumulates its slots (strided by the workgroup) in order; the
// spectrum bin of a slot is found by bisection of the edges staged in LDS,
// and each wave adds its slots of one tile into per-wave bin sums in LDS,
// bin by bin (a wave reduction per bin present in the tile).  Waves are
// combined in a fixed order, so every sum has a fixed reduction order.
// ---------------------------------------------------------------------------
constexpr int kMomentsMaxAttr = 16;

__device__ __forceinline__ double wave_sum_d(double x) {
  x += dpp_d<kDppQuad1032>(x);
  x += dpp_d<kDppQuad2301>(x);
  x += dpp_d<kDppHalfMirror>(x);
  x += dpp_d<kDppRowMirror>(x);
  return ((readlane_d(x, 15) + readlane_d(x, 31)) + readlane_d(x, 47)) + readlane_d(x, 63);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += (unsigned long long)__shfl_xor(x, o);
  return x;
}

template <int W>
__global__ void __launch_bounds__(64 * W) k_moments(SimDesc d, int64_t* m0, double* m12,
                                                    double* attr_sums, const double* edges,
                                                    int n_bins, double* spectrum) {
  extern __shared__ double mom_lds[];  // edges[n_bins + 1], then W x n_bins bin sums
  __shared__ double red_d[W][2 + kMomentsMaxAttr];
  __shared__ unsigned long long red_u[W];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c = blockIdx.x;
  const int64_t o0 = d.cell_off[c];
  const int n = (int)(d.cell_off[c + 1] - o0);
  const int A = d.n_attr;
  const bool spec = spectrum != nullptr && n_bins > 0;
  double* e = mom_lds;
  double* bins = mom_lds + (n_bins + 1);
  if (spec) {
    for (int k = tid; k <= n_bins; k += 64 * W) e[k] = edges[k];
    for (int k = tid; k < W * n_bins; k += 64 * W) bins[k] = 0.0;
    __syncthreads();
  }
  unsigned long long cnt = 0;
  double s1 = 0.0, s2 = 0.0;
  double sa[kMomentsMaxAttr];
#pragma unroll
  for (int q = 0; q < kMomentsMaxAttr; ++q) sa[q] = 0.0;
  const double lo = spec ? e[0] : 0.0, hi = spec ? e[n_bins] : 0.0;
  // tiles of 64 W slots; every wave runs every tile (uniform trip count)
  for (int base = 0; base < n; base += 64 * W) {
    const int j = base + tid;
    long long x = 0;
    double vv = 0.0;
    if (j < n) x = d.xi[o0 + j];
    if (x > 0) vv = d.v[o0 + j];
    const double w1 = (double)x * vv;
    if (x > 0) {
      cnt += (unsigned long long)x;
      s1 += w1;
      s2 += w1 * vv;
#pragma unroll
      for (int q = 0; q < kMomentsMaxAttr; ++q)
        if (q < A) sa[q] += (double)x * d.attrs[(int64_t)q * d.n_slots + o0 + j];
    }
    if (spec) {
      int k = -1;
      if (x > 0 && lo <= vv && vv < hi) {  // e[k] <= vv < e[k + 1]
        int a = 0, b = n_bins;
        while (b - a > 1) {
          const int m = (a + b) >> 1;
          if (e[m] <= vv) a = m;
          else b = m;
        }
        k = a;
      }
      unsigned long long act = __ballot(k >= 0);
      while (act) {
        const int kk = __builtin_amdgcn_readlane(k, __ffsll((long long)act) - 1);
        const bool mine = k == kk;
        const double s = wave_sum_d(mine ? w1 : 0.0);
        if (lane == 0) bins[wv * n_bins + kk] += s;
        act &= ~__ballot(mine);
      }
    }
  }
  cnt = wave_sum_u64(cnt);
  s1 = wave_sum_d(s1);
  s2 = wave_sum_d(s2);
#pragma unroll
  for (int q = 0; q < kMomentsMaxAttr; ++q)
    if (q < A) sa[q] = wave_sum_d(sa[q]);
  if (lane == 0) {
    red_u[wv] = cnt;
    red_d[wv][0] = s1;
    red_d[wv][1] = s2;
#pragma unroll
    for (int q = 0; q < kMomentsMaxAttr; ++q)
      if (q < A) red_d[wv][2 + q] = sa[q];
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long tc = red_u[0];
    double t1 = red_d[0][0], t2 = red_d[0][1];
    for (int w = 1; w < W; ++w) {
      tc += red_u[w];
      t1 += red_d[w][0];
      t2 += red_d[w][1];
    }
    if (m0) m0[c] = (int64_t)tc;
    if (m12) {
      m12[2 * c] = t1;
      m12[2 * c + 1] = t2;
    }
  }
  if (attr_sums && tid < A) {
    double t = red_d[0][2 + tid];
    for (int w = 1; w < W; ++w) t += red_d[w][2 + tid];
    attr_sums[(int64_t)c * A + tid] = t;
  }
  if (spec)
    for (int k = tid; k < n_bins; k += 64 * W) {
      double t = bins[k];
      for (int w = 1; w < W; ++w) t += bins[w * n_bins + k];
      spectrum[(int64_t)c * n_bins + k] = t;
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
// Dispatch order of the adaptive cells of a class for the next step: a stable
// partition of this step's list into kOrderGroups groups by the substeps each
// cell took (8 or more, 4-7, 2-3, at most 1), longest first, so that the long
// cells start early instead of stretching the end of the launch (results do
// not depend on the order).  k_order_count counts each group in each block of
// kOrderBlock tasks; k_order_scatter places every task from the counts of the
// groups and blocks before it and its rank among its group in its block.
// ---------------------------------------------------------------------------
// exclusive count of pred over the block's threads before this one; *total:
// over the whole block
__device__ __forceinline__ uint32_t block_excl_count(bool pred, int tid, uint32_t* red,
                                                     uint32_t* total) {
  const int lane = tid & 63, wv = tid >> 6;
  const unsigned long long m = __ballot(pred);
  const uint32_t in_wave = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) red[wv] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kOrderBlock / 64; ++k) {
    const uint32_t c = red[k];
    before += k < wv ? c : 0u;
    all += c;
  }
  __syncthreads();  // red is reused by the next call
  *total = all;
  return before + in_wave;
}

__global__ void __launch_bounds__(kOrderBlock) k_order_count(const uint32_t* __restrict__ group,
                                                             uint32_t* __restrict__ cnt, int n) {
  __shared__ uint32_t red[kOrderBlock / 64];
  const int i = blockIdx.x * kOrderBlock + threadIdx.x;
  const uint32_t g = i < n ? group[i] : kOrderGroups;
#pragma unroll
  for (int q = 0; q < kOrderGroups; ++q) {
    uint32_t total;
    (void)block_excl_count(g == (uint32_t)q, threadIdx.x, red, &total);
    if (threadIdx.x == 0) cnt[blockIdx.x * kOrderGroups + q] = total;
  }
}

__global__ void __launch_bounds__(kOrderBlock) k_order_scatter(
    const CellTask* __restrict__ in, const uint32_t* __restrict__ group,
    const uint32_t* __restrict__ cnt, CellTask* __restrict__ out, int n, int nblocks) {
  __shared__ uint32_t red[kOrderBlock / 64];
  __shared__ uint32_t base[kOrderGroups];  // first slot of the group's tasks of this block
  const int tid = threadIdx.x;
  if (tid < 64) {
    uint32_t before[kOrderGroups], all[kOrderGroups];
#pragma unroll
    for (int q = 0; q < kOrderGroups; ++q) before[q] = all[q] = 0;
    for (int b = tid; b < nblocks; b += 64)
#pragma unroll
      for (int q = 0; q < kOrderGroups; ++q) {
        const uint32_t c = cnt[b * kOrderGroups + q];
        before[q] += b < (int)blockIdx.x ? c : 0u;
        all[q] += c;
      }
    uint32_t run = 0;
#pragma unroll
    for (int q = 0; q < kOrderGroups; ++q) {
      const uint32_t bq = (uint32_t)wave_sum((int)before[q]);
      const uint32_t aq = (uint32_t)wave_sum((int)all[q]);
      if (tid == 0) base[q] = run + bq;
      run += aq;
    }
  }
  __syncthreads();
  const int i = blockIdx.x * kOrderBlock + tid;
  const uint32_t g = i < n ? group[i] : kOrderGroups;
  uint32_t pos = 0;
#pragma unroll
  for (int q = 0; q < kOrderGroups; ++q) {
    uint32_t total;
    const uint32_t r = block_excl_count(g == (uint32_t)q, tid, red, &total);
    if (g == (uint32_t)q) pos = base[q] + r;
  }
  if (i < n) out[pos] = in[i];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t cell_lds_bytes(int cls) {
  switch (cls) {
    case 0: return sizeof(CellLds<64>);
    case 1: return sizeof(CellLds<128>);
    case 2: return sizeof(CellLds<256>);
    case 3: return sizeof(CellLds<384>);
    default: return sizeof(CellLds<512>);
  }
}

void set_lds_limits() {
  static bool done = false;
  if (done) return;
  done = true;
  const int lim = 160 * 1024;
  (void)hipFuncSetAttribute((const void*)k_big_keys, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sizeof(uint32_t) * (kBigMaxBuckets + 1));
  (void)hipFuncSetAttribute((const void*)k_cells_mid<2048, mid_waves(2048), false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_cells_mid<2048, mid_waves(2048), true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_cells_mid<4096, mid_waves(4096), false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_cells_mid<4096, mid_waves(4096), true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_cells_mid<8192, mid_waves(8192), false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_cells_mid<8192, mid_waves(8192), true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_cells_mid<16384, mid_waves(16384), false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipFuncSetAttribute((const void*)k_cells_mid<16384, mid_waves(16384), true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  (void)hipGetLastError();
}

template <int CAP, int W>
static void launch_class_w(const PlanDev& p, int cls, uint32_t k_abs, uint32_t flip, int nsteps,
                           hipStream_t st) {
  const int np = p.n_plain[cls], na = p.n_wave[cls] - p.n_plain[cls];
  if (np > 0)
    hipLaunchKernelGGL((k_cells<CAP, W, false>), dim3(np), dim3(64 * W), 0, st, p.desc,
                       p.wave_tasks[cls], k_abs, nsteps, nullptr);
  if (na > 0) {
    // the adaptive list of this step, and the one the next step will use
    const uint32_t par = flip & 1u;
    CellTask* cur = par ? p.wave_alt[cls] : p.wave_tasks[cls] + np;
    CellTask* nxt = par ? p.wave_tasks[cls] + np : p.wave_alt[cls];
    hipLaunchKernelGGL((k_cells<CAP, W, true>), dim3(na), dim3(64 * W), 0, st, p.desc, cur,
                       k_abs, nsteps, p.order_flag[cls]);
    const int nb = (na + kOrderBlock - 1) / kOrderBlock;
    hipLaunchKernelGGL(k_order_count, dim3(nb), dim3(kOrderBlock), 0, st, p.order_flag[cls],
                       p.order_cnt[cls], na);
    hipLaunchKernelGGL(k_order_scatter, dim3(nb), dim3(kOrderBlock), 0, st, cur,
                       p.order_flag[cls], p.order_cnt[cls], nxt, na, nb);
  }
}

template <int CAP>
static void launch_class(const PlanDev& p, int cls, uint32_t k_abs, uint32_t flip, int nsteps,
                         int w, hipStream_t st) {
  switch (w) {
    case 1: launch_class_w<CAP, 1>(p, cls, k_abs, flip, nsteps, st); break;
    case 2: launch_class_w<CAP, 2>(p, cls, k_abs, flip, nsteps, st); break;
    case 4: launch_class_w<CAP, 4>(p, cls, k_abs, flip, nsteps, st); break;
    default: launch_class_w<CAP, 8>(p, cls, k_abs, flip, nsteps, st); break;
  }
}

size_t mid_lds_bytes(int cls) {
  switch (cls) {
    case 0: return sizeof(MidLds<2048>);
    case 1: return sizeof(MidLds<4096>);
    case 2: return sizeof(MidLds<8192>);
    default: return sizeof(MidLds<16384>);
  }
}

template <int CAP>
static void launch_mid(const PlanDev& p, int cls, uint32_t k_abs, hipStream_t st) {
  constexpr int W = mid_waves(CAP);
  const int np = p.n_mid_plain[cls], na = p.n_mid[cls] - p.n_mid_plain[cls];
  const unsigned lds = (unsigned)sizeof(MidLds<CAP>);
  if (np > 0)
    hipLaunchKernelGGL((k_cells_mid<CAP, W, false>), dim3(np), dim3(64 * W), lds, st, p.desc,
                       p.mid_tasks[cls], k_abs);
  if (na > 0)
    hipLaunchKernelGGL((k_cells_mid<CAP, W, true>), dim3(na), dim3(64 * W), lds, st, p.desc,
                       p.mid_tasks[cls] + np, k_abs);
}

hipError_t launch_step(const PlanDev& p, uint32_t k_abs, uint32_t flip, int nsteps,
                       int waves_per_cell, hipStream_t st, const SideStream& side) {
  // Up to three independent groups of launches run on their own streams and
  // fill each other's tails: A, the cells of up to 256 slots and the
  // 16384- and 2048-slot mid-size classes, on a side stream; B, the 8192-
  // and 4096-slot mid-size classes, on a second side stream; L, the 384-
  // and 512-slot classes and the big-cell chain, on the caller's stream.
  // A group runs on the caller's stream when nothing runs beside it there;
  // the side streams wait for the caller's stream (one event) and are
  // joined back into it (an event each).
  const bool ga = p.n_wave[0] > 0 || p.n_wave[1] > 0 || p.n_wave[2] > 0 || p.n_mid[3] > 0 ||
                  p.n_mid[0] > 0;
  const bool gb = p.n_mid[2] > 0 || p.n_mid[1] > 0;
  const bool gl = p.n_wave[3] > 0 || p.n_wave[4] > 0 || p.n_big > 0;
  const bool fa = side.stream && ga && gl;
  const bool fb = side.stream2 && gb && (ga || gl);
  const hipStream_t sa = fa ? side.stream : st;
  const hipStream_t sb = fb ? side.stream2 : st;
  if (fa || fb) {
    if (hipEventRecord(side.fork, st) != hipSuccess ||
        (fa && hipStreamWaitEvent(sa, side.fork, 0) != hipSuccess) ||
        (fb && hipStreamWaitEvent(sb, side.fork, 0) != hipSuccess))
      return hipErrorUnknown;
  }
  launch_class<256>(p, 2, k_abs, flip, nsteps, waves_per_cell, sa);
  launch_class<128>(p, 1, k_abs, flip, nsteps, waves_per_cell, sa);
  launch_class<64>(p, 0, k_abs, flip, nsteps, waves_per_cell, sa);
  for (int t = 0; t < nsteps; ++t) {  // mid-size cells: one launch per step
    launch_mid<16384>(p, 3, k_abs + t, sa);
    launch_mid<8192>(p, 2, k_abs + t, sb);
    launch_mid<4096>(p, 1, k_abs + t, sb);
    launch_mid<2048>(p, 0, k_abs + t, sa);
  }
  launch_class<512>(p, 4, k_abs, flip, nsteps, waves_per_cell, st);
  launch_class<384>(p, 3, k_abs, flip, nsteps, waves_per_cell, st);
  for (int t = 0; t < nsteps && p.n_chunks > 0; ++t) {  // big cells: two launches per step
    hipLaunchKernelGGL(k_big_keys, dim3(p.n_chunks), dim3(kBigKeyThreads), p.big_hist_bytes, st,
                       p.desc, p.big, p.chunks, p.offs, p.ekey, p.exi, p.ev, k_abs + t,
                       (const BigAdapt*)nullptr);
    hipLaunchKernelGGL(k_big_bucket<false>, dim3(p.n_buckets), dim3(kBigThreads), 0, st, p.desc,
                       p.big, p.buckets, (const uint32_t*)p.offs,
                       (const unsigned long long*)p.ekey, (const long long*)p.exi,
                       (const double*)p.ev, p.skey, p.ord, k_abs + t, (BigAdapt*)nullptr,
                       (unsigned long long*)nullptr, (double*)nullptr,
                       (unsigned long long*)nullptr);
  }
  if (fa && (hipEventRecord(side.join, sa) != hipSuccess ||
             hipStreamWaitEvent(st, side.join, 0) != hipSuccess))
    return hipErrorUnknown;
  if (fb && (hipEventRecord(side.join2, sb) != hipSuccess ||
             hipStreamWaitEvent(st, side.join2, 0) != hipSuccess))
    return hipErrorUnknown;
  return hipGetLastError();
}

hipError_t launch_abig_init(const PlanDev& p, uint32_t k_abs, hipStream_t st) {
  hipLaunchKernelGGL(k_abig_init, dim3((p.n_abig + 255) / 256), dim3(256), 0, st, p.desc, p.big,
                     p.abig, p.n_abig, p.astate[0], p.apmax[0], p.apmax[1], k_abs);
  return hipGetLastError();
}

hipError_t launch_abig_round(const PlanDev& p, uint32_t k_abs, uint32_t round, hipStream_t st) {
  const uint32_t q = round & 1u;
  hipLaunchKernelGGL(k_big_keys, dim3(p.n_achunks), dim3(kBigKeyThreads), p.big_hist_bytes, st,
                     p.desc, p.big, p.achunks, p.offs, p.ekey, p.exi, p.ev, k_abs,
                     (const BigAdapt*)p.astate[q]);
  hipLaunchKernelGGL(k_big_bucket<true>, dim3(p.n_abuckets), dim3(kBigThreads), 0, st, p.desc,
                     p.big, p.abuckets, (const uint32_t*)p.offs,
                     (const unsigned long long*)p.ekey, (const long long*)p.exi,
                     (const double*)p.ev, p.skey, p.ord, k_abs, p.astate[q], p.apmax[q], p.apre,
                     p.apair);
  hipLaunchKernelGGL(k_abig_pairs, dim3(p.n_apblocks), dim3(kAbigPairs), 0, st, p.desc, p.big,
                     p.apblocks, (const BigAdapt*)p.astate[q], p.astate[q ^ 1u],
                     (const unsigned long long*)p.apmax[q], p.apmax[q ^ 1u],
                     (const double*)p.apre, (const unsigned long long*)p.apair, k_abs);
  return hipGetLastError();
}

hipError_t launch_abig_active(const PlanDev& p, uint32_t round, uint32_t* count,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_abig_active, dim3(1), dim3(256), 0, st,
                     (const BigAdapt*)p.astate[round & 1u], p.abig, p.n_abig, count);
  return hipGetLastError();
}

hipError_t launch_moments(const SimDesc& d, int n_cells, int waves, int64_t* m0, double* m12,
                          double* attr_sums, const double* edges, int n_bins, double* spectrum,
                          hipStream_t st) {
  if (n_cells <= 0) return hipSuccess;
  const size_t lds = spectrum && n_bins > 0
                         ? sizeof(double) * ((size_t)n_bins + 1 + (size_t)waves * n_bins)
                         : 0;
  if (waves == 1)
    hipLaunchKernelGGL(k_moments<1>, dim3(n_cells), dim3(64), lds, st, d, m0, m12, attr_sums,
                       edges, n_bins, spectrum);
  else
    hipLaunchKernelGGL(k_moments<4>, dim3(n_cells), dim3(256), lds, st, d, m0, m12, attr_sums,
                       edges, n_bins, spectrum);
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
