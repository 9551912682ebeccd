// sdm_condense.hip -- diffusional growth (condensation / evaporation) of the
// super-droplets of a simulation on gfx950.
//
// The PySDM v1 paper lists condensational growth among its dynamics
// ("Introduction", "API in brief") and uses it with ambient thermodynamics
// in its parcel examples ("Adiabatic parcel examples": activation of aerosol
// by supersaturation, modes of different hygroscopicity) without fixing the
// physics.  Per super-droplet this computes one implicit Euler step in
// x = r^2 of the Maxwell-Mason growth law (Rogers & Yau 1989, ch. 7)
//     r dr/dt = (S - S_eq(r)) / (F_k + F_d),
// with the kappa-Koehler equilibrium saturation (Petters & Kreidenweis 2007)
//     S_eq(r) = (r^3 - r_d^3) / (r^3 - r_d^3 (1 - kappa)) exp(A / r),
// A = 2 sigma / (rho_w R_v T), F_k = (L / (R_v T) - 1) L rho_w / (K T),
// F_d = rho_w R_v T / (D e_s), D = 2.11e-5 (T / 273.15)^1.94 (101325 / p),
// e_s = 611.2 exp(17.67 (T - 273.15) / (T - 29.65)) (Bolton 1980), the
// ambient T, p, S of each cell held over the step.  The implicit equation
// g(x) = x - x0 - c (S - S_eq) = 0, c = 2 dt / (F_k + F_d), is solved by
// Newton's method inside the bracket [r_d^2, max(r_d^2, x0 + c S)]: a step
// that leaves the bracket, or a non-positive slope, becomes the midpoint;
// the bracket closes in on the iterate by the sign of g; the iteration stops
// when a step is at most 1e-14 of x, or after max_iter iterations.
//
// Data: each thread takes one slot, blocks of 256 consecutive slots across
// cell boundaries (every wavefront but the last full), so the reads of xi,
// v and the two attributes are coalesced; each cell's ambient terms are
// computed once per block that holds its slots.  One slot per thread keeps
// the registers low and the occupancy high: the Newton iteration is a chain
// of dependent fp64 operations, and it is the other wavefronts of the SIMD
// that hide its latency.  Bound: HBM for the state (40 B per live slot: xi,
// v, dry volume and kappa dry volume read, v written), fp64 ALU for the exp
// / sqrt / cbrt of the Newton iterations.
#include "sdm_internal.hpp"

namespace sdm {

constexpr double kCondPi = 3.14159265358979323846;
constexpr double kFourPi3 = 4.0 * kCondPi / 3.0;
constexpr double kSigma = 0.072;   // N/m
constexpr double kRhoW = 1000.0;   // kg/m^3
constexpr double kRv = 461.5;      // J/(kg K)
constexpr double kLv = 2.5e6;      // J/kg
constexpr double kKair = 2.4e-2;   // W/(m K)
constexpr double kD0 = 2.11e-5;    // m^2/s at 273.15 K, 101325 Pa
constexpr double kCondTol = 1e-14;
constexpr int kCondThreads = 256;
constexpr int kCondPart = kCondThreads;  // slots per block (one per thread)

// equilibrium saturation ratio and its derivative in x = r^2 (0 at or below
// the dry size)
__device__ __forceinline__ void s_eq_and_slope(double x, double rd3, double kappa, double a,
                                               double& s, double& ds) {
  const double r = sqrt(x);
  const double r3 = x * r;
  if (!(r3 > rd3)) {
    s = 0.0;
    ds = 0.0;
    return;
  }
  const double den = r3 - rd3 * (1.0 - kappa);
  const double f1 = (r3 - rd3) / den;
  const double f2 = exp(a / r);
  s = f1 * f2;
  ds = f2 * ((rd3 * kappa) * (1.5 * r) / (den * den) - f1 * a / (2.0 * r3));
}

// ambient terms of a cell: c = 2 dt / (F_k + F_d), A, S
__device__ __forceinline__ void cell_terms(double T, double p, double S, double dt, double& c,
                                           double& a, double& s) {
  const double es = 611.2 * exp(17.67 * (T - 273.15) / (T - 29.65));
  const double D = kD0 * pow(T / 273.15, 1.94) * (101325.0 / p);
  const double fk = (kLv / (kRv * T) - 1.0) * kLv * kRhoW / (kKair * T);
  const double fd = kRhoW * kRv * T / (D * es);
  c = 2.0 * dt / (fk + fd);
  a = 2.0 * kSigma / (kRhoW * kRv * T);
  s = S;
}

// last cell c with cell_off[c] <= j (cell_off[n_cells] = n_slots > j)
__device__ __forceinline__ int cell_of(const int64_t* __restrict__ off, int n_cells, int64_t j) {
  int lo = 0, hi = n_cells;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= j) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One block per kCondPart consecutive slots, across cell boundaries, so that
// every wavefront but the last is full.  The block finds the cell of its
// first slot (one binary search), reads the offsets of the next kCondPart
// cells into LDS, and lane t computes the ambient terms of cell c0 + t when
// that cell has slots in the block; a thread finds its cell by a binary
// search in that window (a global one, and its own terms, only when more
// than kCondPart cells, most of them empty, lie inside the block).
__global__ void __launch_bounds__(kCondThreads) k_condense(
    const int64_t* __restrict__ xi, double* __restrict__ v, const double* __restrict__ vdry,
    const double* __restrict__ kvdry, const int64_t* __restrict__ cell_off, int n_cells,
    int64_t n_slots, const double* __restrict__ temp, const double* __restrict__ pres,
    const double* __restrict__ sat, double dt, int max_iter) {
  __shared__ int64_t woff[kCondPart + 1];
  __shared__ double wc[kCondPart], wa[kCondPart], ws[kCondPart];
  __shared__ int c0s;
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kCondPart;
  const int64_t j = s0 + tid;
  long long x_ = 0;
  double v_ = 0.0, vd = 0.0, kv = 0.0;
  if (j < n_slots) x_ = xi[j];
  if (x_ > 0) {  // the state first (coalesced), then the solve
    v_ = v[j];
    vd = vdry[j];
    kv = kvdry[j];
  }
  if (tid == 0) c0s = cell_of(cell_off, n_cells, s0);
  __syncthreads();
  const int c0 = c0s;
  woff[tid] = cell_off[min(c0 + tid, n_cells)];
  if (tid == 0) woff[kCondPart] = cell_off[min(c0 + kCondPart, n_cells)];
  __syncthreads();
  {  // lane t: the terms of cell c0 + t if it has slots in this block
    const int c = c0 + tid;
    if (c < n_cells && woff[tid] < s0 + kCondPart && woff[tid + 1] > s0 &&
        woff[tid + 1] > woff[tid])
      cell_terms(temp[c], pres[c], sat[c], dt, wc[tid], wa[tid], ws[tid]);
  }
  __syncthreads();
  if (x_ <= 0) return;
  double cc, a, S;
  if (j < woff[kCondPart]) {  // the cell inside the window
    int lo = 0, hi = kCondPart;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (woff[mid] <= j) lo = mid;
      else hi = mid;
    }
    cc = wc[lo];
    a = wa[lo];
    S = ws[lo];
  } else {
    const int c = cell_of(cell_off, n_cells, j);
    cell_terms(temp[c], pres[c], sat[c], dt, cc, a, S);
  }
  const double kappa = vd > 0.0 ? kv / vd : 0.0;
  const double rd3 = vd / kFourPi3;
  const double rd = cbrt(rd3);
  const double xd = rd * rd;
  const double r0 = cbrt(fmax(v_, vd) / kFourPi3);
  const double x0 = fmax(r0 * r0, xd);
  double lo = xd, hi = fmax(xd, x0 + cc * S);
  double x = fmin(fmax(x0, lo), hi);
  for (int it = 0; it < max_iter; ++it) {
    double se, dse;
    s_eq_and_slope(x, rd3, kappa, a, se, dse);
    const double g = x - x0 - cc * (S - se);
    const double gp = 1.0 + cc * dse;
    if (g == 0.0) break;
    if (g < 0.0) lo = x;
    else if (g > 0.0) hi = x;
    double xn = x - g / gp;
    if (!(gp > 0.0) || !(xn >= lo) || !(xn <= hi)) xn = 0.5 * (lo + hi);
    const bool done = fabs(xn - x) <= kCondTol * xn;
    x = xn;
    if (done) break;
  }
  const double r1 = sqrt(x);
  v[j] = kFourPi3 * (x * r1);
}

hipError_t launch_condense(const int64_t* xi, double* v, const double* vdry, const double* kvdry,
                           const int64_t* cell_off, int n_cells, int64_t n_slots,
                           const double* temp, const double* pres, const double* sat, double dt,
                           int max_iter, hipStream_t st) {
  if (n_cells <= 0 || n_slots <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n_slots + kCondPart - 1) / kCondPart);
  hipLaunchKernelGGL(k_condense, dim3(blocks), dim3(kCondThreads), 0, st, xi, v, vdry, kvdry,
                     cell_off, n_cells, n_slots, temp, pres, sat, dt, max_iter);
  return hipGetLastError();
}

}  // namespace sdm
