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
// Data: each thread takes slot j = part 256 + tid of one cell (blockIdx.x
// the cell, blockIdx.y the 256-slot part), so the reads of xi, v and the two
// attributes are coalesced; the cell's ambient terms are computed once per
// block.  One slot per thread keeps the registers low and the occupancy high:
// the Newton iteration is a chain of dependent fp64 operations, and it is the
// other wavefronts of the SIMD that hide its latency.  Bound: HBM for the state (40 B per live slot:
// xi, v, dry volume and kappa dry volume read, v written), fp64 ALU for the
// exp / sqrt / cbrt of the Newton iterations.
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

__global__ void __launch_bounds__(kCondThreads) k_condense(
    const int64_t* __restrict__ xi, double* __restrict__ v, const double* __restrict__ vdry,
    const double* __restrict__ kvdry, const int64_t* __restrict__ cell_off,
    const double* __restrict__ temp, const double* __restrict__ pres,
    const double* __restrict__ sat, double dt, int max_iter) {
  const int c = blockIdx.x;
  const int64_t o0 = cell_off[c];
  const int64_t n = cell_off[c + 1] - o0;
  const int64_t base = (int64_t)blockIdx.y * kCondPart;
  if (base >= n) return;
  const int64_t j = base + threadIdx.x;
  long long x_ = 0;
  double v_ = 0.0, vd = 0.0, kv = 0.0;
  if (j < n) x_ = xi[o0 + j];
  if (x_ > 0) {  // the state first (coalesced), then the solve
    v_ = v[o0 + j];
    vd = vdry[o0 + j];
    kv = kvdry[o0 + j];
  }
  // the cell's ambient terms, by one thread for the block (a pow and an exp
  // would otherwise cost each wavefront as much as its droplets)
  __shared__ double amb[3];
  if (threadIdx.x == 0) {
    const double T = temp[c], p = pres[c];
    const double es = 611.2 * exp(17.67 * (T - 273.15) / (T - 29.65));
    const double D = kD0 * pow(T / 273.15, 1.94) * (101325.0 / p);
    const double fk = (kLv / (kRv * T) - 1.0) * kLv * kRhoW / (kKair * T);
    const double fd = kRhoW * kRv * T / (D * es);
    amb[0] = 2.0 * dt / (fk + fd);
    amb[1] = 2.0 * kSigma / (kRhoW * kRv * T);
    amb[2] = sat[c];
  }
  __syncthreads();
  if (x_ <= 0) return;
  const double cc = amb[0], a = amb[1], S = amb[2];
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
  v[o0 + j] = kFourPi3 * (x * r1);
}

hipError_t launch_condense(const int64_t* xi, double* v, const double* vdry, const double* kvdry,
                           const int64_t* cell_off, int n_cells, int64_t max_cell,
                           const double* temp, const double* pres, const double* sat, double dt,
                           int max_iter, hipStream_t st) {
  if (n_cells <= 0 || max_cell <= 0) return hipSuccess;
  const unsigned parts = (unsigned)((max_cell + kCondPart - 1) / kCondPart);
  hipLaunchKernelGGL(k_condense, dim3((unsigned)n_cells, parts), dim3(kCondThreads), 0, st, xi,
                     v, vdry, kvdry, cell_off, temp, pres, sat, dt, max_iter);
  return hipGetLastError();
}

}  // namespace sdm
