/*
 * sdm_oracle.c -- plain, slow CPU reference of the Super-Droplet Method (SDM)
 * Monte-Carlo collision-coalescence step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP library; it was written separately from the method's
 * published description.
 *
 * What it follows.
 *   - The PySDM v1 paper (arXiv 2103.17238), sections "Introduction" and
 *     "API in brief": SDM is the package core; a super-droplet (SD) carries a
 *     multiplicity xi (number of real droplets it stands for) and a volume;
 *     the Box environment is a single cell of volume dV advanced with step dt;
 *     the Golovin additive kernel K = b (v1 + v2) with b = 1.5e3 1/s.
 *     Section "Box environment examples": the Berry (1966) example uses the
 *     geometric sweep-out kernel.
 *   - Shima et al. (2009), the paper the SDM was introduced in (cited by the
 *     PySDM paper): per cell, draw a random permutation of the SDs, pair
 *     neighbours, scale each pair's collision probability
 *     max(xi_j, xi_k) K dt / dV by n(n-1)/2 / floor(n/2), turn it into an
 *     integer collision count gamma with one uniform deviate, and update the
 *     multiplicities and extensive attributes, splitting equally when the
 *     larger multiplicity is used up exactly.
 *   - Philox4x32-10 from Salmon, Moraes, Dror & Shaw (2011), "Parallel random
 *     numbers: as easy as 1, 2, 3" (SC'11): 10 rounds, multipliers
 *     0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
 *
 * Readings where the papers are silent (each one is listed in the design
 * notes): the permutation is the order of the live SDs by (32-bit Philox key,
 * slot); the uniform has 53 bits in [0, 1); gamma = floor(p) + [phi < p -
 * floor(p)]; ties in xi give the pair's first member the larger role; dead SDs
 * (xi = 0) keep their slot; radius from volume assumes spheres; the terminal
 * velocity is the continuous three-regime power law
 * u = min(k1 r^2, k2 r, k3 sqrt r) of Rogers & Yau (1989) without air-density
 * correction; collision efficiency E = 1.
 *
 * Floating point: IEEE binary64; build with -O2 -ffp-contract=off and no
 * fast-math.  The only fused operation is the explicit fma() of the
 * attribute update.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_GOLOVIN 0
#define ORC_GEOMETRIC 1

#define ORC_ST_SUBSTEP_CAP 1u
#define ORC_ST_GAMMA_CAP 2u

/* geometric kernel constants (terminal velocity, Rogers & Yau 1989) */
#define ORC_K1 1.19e8 /* 1/(m s), Stokes regime u = k1 r^2 */
#define ORC_K2 8.0e3  /* 1/s,     linear regime u = k2 r   */
#define ORC_K3 201.0  /* m^0.5/s, sqrt regime u = k3 r^0.5 */

typedef struct {
  int64_t n_slots;
  int32_t n_cells;
  int32_t n_attr;
  double dt;
  double dv;
  double b; /* Golovin b [1/s] */
  int32_t kernel;
  int32_t adaptive;
  int32_t max_substeps;
  int32_t n_threads; /* OpenMP threads over cells; <= 1 means serial */
  uint64_t seed;
} orc_cfg;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. 2011).                                 */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { /* key schedule: add the Weyl constants between rounds */
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)prod1;
    uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)prod0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* bulk form for tests: out[4 i + w] = Philox((c0 + i, c1, c2, c3), key)[w] */
void orc_philox_fill(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                     int64_t n, uint32_t* out) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t i = 0; i < n; ++i) {
    uint32_t ctr[4] = {c0 + (uint32_t)i, c1, c2, c3};
    orc_philox4x32_10(ctr, key, out + 4 * i);
  }
}

/* ------------------------------------------------------------------ */
/* Random numbers the step draws.                                      */
/* ------------------------------------------------------------------ */

/* sort key of cell-local slot j: word (j mod 4) of Philox((j/4, c, s, 2u)) */
static uint32_t sort_key(uint64_t seed, int64_t j, int32_t c, uint32_t s, uint32_t u) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)(j / 4), (uint32_t)c, s, 2u * u};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return w[j % 4];
}

/* uniform deviate in [0, 1) with 53 bits from two 32-bit words */
double orc_phi(uint32_t hi, uint32_t lo) {
  uint64_t bits = ((uint64_t)hi << 32) | (uint64_t)lo;
  return (double)(bits >> 11) * (1.0 / 9007199254740992.0); /* 2^-53 */
}

/* uniform of candidate pair m: words 2(m mod 2), 2(m mod 2)+1 of Philox((m/2, c, s, 2u+1)) */
static double pair_uniform(uint64_t seed, int64_t m, int32_t c, uint32_t s, uint32_t u) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)(m / 2), (uint32_t)c, s, 2u * u + 1u};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  int64_t h = 2 * (m % 2);
  return orc_phi(w[h], w[h + 1]);
}

/* ------------------------------------------------------------------ */
/* Coalescence kernels.                                                */
/* ------------------------------------------------------------------ */

/* radius of a sphere of volume v */
double orc_radius(double v) { return cbrt((3.0 / (4.0 * M_PI)) * v); }

/* terminal fall speed: continuous three-regime power law (Rogers & Yau 1989) */
double orc_terminal_velocity(double r) {
  double u1 = ORC_K1 * r * r;
  double u2 = ORC_K2 * r;
  double u3 = ORC_K3 * sqrt(r);
  return fmin(fmin(u1, u2), u3);
}

/* K(v1, v2) in m^3/s */
double orc_kernel(int32_t kind, double b, double v1, double v2) {
  if (kind == ORC_GOLOVIN) return b * (v1 + v2); /* Golovin additive kernel */
  /* geometric sweep-out, E = 1: pi (r1 + r2)^2 |u1 - u2| */
  double r1 = orc_radius(v1), r2 = orc_radius(v2);
  double u1 = orc_terminal_velocity(r1), u2 = orc_terminal_velocity(r2);
  double rs = r1 + r2;
  return M_PI * (rs * rs) * fabs(u1 - u2);
}

/* scale factor n(n-1)/2 / floor(n/2), written as an integer */
int64_t orc_scale_factor(int64_t n) { return (n % 2 == 1) ? n : n - 1; }

/* scaled probability of one candidate pair: ((max xi * K) * S) * q, q = dt/dV */
double orc_pair_probability(int32_t kind, double b, double q, int64_t xi_a, int64_t xi_b,
                            double v_a, double v_b, int64_t scale) {
  int64_t xmax = xi_a > xi_b ? xi_a : xi_b;
  double k = orc_kernel(kind, b, v_a, v_b);
  return (((double)xmax * k) * (double)scale) * q;
}

/* integer number of collisions from probability p and uniform phi */
int64_t orc_gamma(double p, double phi) {
  if (!(p < 4611686018427387904.0)) return (int64_t)4611686018427387904LL; /* cap 2^62 */
  double f = floor(p);
  return (int64_t)f + ((phi < p - f) ? 1 : 0);
}

/*
 * Multiplicity / extensive-attribute update of one pair after gamma > 0
 * collisions.  a is the pair's first member, b the second; X arrays are
 * [n_ext][stride] with attribute q of slot i at X[q * stride + i] (volume is
 * passed as its own array so it need not be contiguous with the others).
 * Returns the number of real droplets removed (g * xi_k).
 */
static int64_t update_pair(int64_t* xi, double* v, double* attrs, int64_t stride, int32_t n_attr,
                           int64_t ia, int64_t ib, int64_t gamma) {
  int64_t j = (xi[ia] >= xi[ib]) ? ia : ib; /* tie: first member of the pair */
  int64_t k = (j == ia) ? ib : ia;
  int64_t ratio = xi[j] / xi[k];
  int64_t g = gamma < ratio ? gamma : ratio;
  double gd = (double)g;
  int64_t removed = g * xi[k];
  int64_t rest = xi[j] - removed;
  if (rest > 0) {
    xi[j] = rest;
    v[k] = fma(gd, v[j], v[k]);
    for (int32_t q = 0; q < n_attr; ++q) {
      double* a = attrs + (int64_t)q * stride;
      a[k] = fma(gd, a[j], a[k]);
    }
  } else { /* equal-multiplicity split */
    int64_t h = xi[k] / 2;
    xi[j] = h;
    xi[k] = xi[k] - h;
    double t = fma(gd, v[j], v[k]);
    v[j] = t;
    v[k] = t;
    for (int32_t q = 0; q < n_attr; ++q) {
      double* a = attrs + (int64_t)q * stride;
      double ta = fma(gd, a[j], a[k]);
      a[j] = ta;
      a[k] = ta;
    }
  }
  return removed;
}

/* test hook: the update rule on one pair of plain values */
void orc_update_pair(int64_t* xi2, double* v2, double* attrs /* [n_attr][2] */, int32_t n_attr,
                     int64_t gamma) {
  if (gamma > 0) update_pair(xi2, v2, attrs, 2, n_attr, 0, 1, gamma);
}

/* ------------------------------------------------------------------ */
/* Permutation: live slots ordered by (key, slot).                     */
/* ------------------------------------------------------------------ */
typedef struct {
  uint32_t key;
  int64_t slot;
} keyed_slot;

static int cmp_keyed(const void* pa, const void* pb) {
  const keyed_slot* a = (const keyed_slot*)pa;
  const keyed_slot* b = (const keyed_slot*)pb;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  if (a->slot != b->slot) return a->slot < b->slot ? -1 : 1;
  return 0;
}

/* order[0..n) = cell-local slots of the live SDs in permuted order; returns n */
static int64_t cell_order(const int64_t* xi_cell, int64_t n_slots, uint64_t seed, int32_t c,
                          uint32_t s, uint32_t u, keyed_slot* scratch, int64_t* order) {
  int64_t n = 0;
  for (int64_t j = 0; j < n_slots; ++j) {
    if (xi_cell[j] > 0) {
      scratch[n].key = sort_key(seed, j, c, s, u);
      scratch[n].slot = j;
      ++n;
    }
  }
  qsort(scratch, (size_t)n, sizeof(keyed_slot), cmp_keyed);
  for (int64_t i = 0; i < n; ++i) order[i] = scratch[i].slot;
  return n;
}

/* test hook: permutation of one cell (xi_cell holds that cell's slots only) */
int64_t orc_cell_order(const int64_t* xi_cell, int64_t n_slots, uint64_t seed, int32_t c,
                       uint32_t s, uint32_t u, int64_t* order) {
  keyed_slot* scratch = (keyed_slot*)malloc(sizeof(keyed_slot) * (size_t)(n_slots > 0 ? n_slots : 1));
  int64_t n = cell_order(xi_cell, n_slots, seed, c, s, u, scratch, order);
  free(scratch);
  return n;
}

/* test hook: scaled probabilities of the pairs an explicit order produces */
void orc_pairs_for_order(int32_t kind, double b, double q, const int64_t* xi, const double* v,
                         const int64_t* order, int64_t n, double* p_out) {
  int64_t scale = orc_scale_factor(n);
  for (int64_t m = 0; m < n / 2; ++m) {
    int64_t a = order[2 * m], bb = order[2 * m + 1];
    p_out[m] = orc_pair_probability(kind, b, q, xi[a], xi[bb], v[a], v[bb], scale);
  }
}

/* ------------------------------------------------------------------ */
/* One cell, one (sub)step.                                            */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t n_live;
  int64_t n_pairs;
  int64_t n_colliding;
} cell_tally;

/*
 * pair_log (optional): per candidate pair m of this cell,
 *   log[2m] = a | (b << 32) (cell-local slots), log[2m+1] = gamma.
 * q_prob: dt/dV used for p; clamp_one: adaptive substeps clamp p <= 1.
 */
static void cell_substep(const orc_cfg* cfg, int64_t* xi, double* v, double* attrs, int64_t off,
                         int64_t n_slots, int32_t c, uint32_t s, uint32_t u, double q_prob,
                         int clamp_one, keyed_slot* scratch, int64_t* order, int64_t* log,
                         cell_tally* tally, uint32_t* status) {
  if (log)
    for (int64_t i = 0; i < 2 * (n_slots / 2); ++i) log[i] = -1;
  int64_t n = cell_order(xi + off, n_slots, cfg->seed, c, s, u, scratch, order);
  tally->n_live = n;
  tally->n_pairs = n / 2;
  if (n < 2) return;
  int64_t scale = orc_scale_factor(n);
  for (int64_t m = 0; m < n / 2; ++m) {
    int64_t a = off + order[2 * m], bb = off + order[2 * m + 1];
    double p = orc_pair_probability(cfg->kernel, cfg->b, q_prob, xi[a], xi[bb], v[a], v[bb], scale);
    if (clamp_one && p > 1.0) p = 1.0;
    double phi = pair_uniform(cfg->seed, m, c, s, u);
    int64_t gamma = orc_gamma(p, phi);
    if (gamma >= 4611686018427387904LL) *status |= ORC_ST_GAMMA_CAP;
    if (log) {
      log[2 * m] = (int64_t)((uint64_t)order[2 * m] | ((uint64_t)order[2 * m + 1] << 32));
      log[2 * m + 1] = gamma;
    }
    if (gamma > 0) {
      tally->n_colliding += 1;
      update_pair(xi, v, attrs, cfg->n_slots, cfg->n_attr, a, bb, gamma);
    }
  }
}

/* largest scaled probability over this cell's candidate pairs at q_prob */
static double cell_pmax(const orc_cfg* cfg, const int64_t* xi, const double* v, int64_t off,
                        const int64_t* order, int64_t n, double q_prob) {
  double pmax = 0.0;
  int64_t scale = orc_scale_factor(n);
  for (int64_t m = 0; m < n / 2; ++m) {
    int64_t a = off + order[2 * m], bb = off + order[2 * m + 1];
    double p = orc_pair_probability(cfg->kernel, cfg->b, q_prob, xi[a], xi[bb], v[a], v[bb], scale);
    if (p > pmax) pmax = p;
  }
  return pmax;
}

/*
 * Adaptive substepping of one cell (keeps gamma <= 1): at each substep u the
 * permutation is redrawn, the largest probability pmax at the remaining time
 * dt_left is found, the substep length is dt_left if pmax <= 1 and
 * dt_left / pmax otherwise, and the pairs are tested with probabilities at
 * that length clamped to 1.  After max_substeps substeps the remainder is
 * done in one unclamped substep and the SUBSTEP_CAP status bit is raised.
 */
/*
 * Optional record of every substep of one cell (test hook): for substep k,
 * dt_left[k] and dt_sub[k] (seconds), n_live[k], clamped[k] (1 if p was
 * clamped to 1, 0 for the unclamped remainder after the substep cap) and the
 * pair log of that substep at log + k * 2 floor(n_slots / 2).
 */
typedef struct {
  int32_t cap;
  int32_t count;
  double* dt_left;
  double* dt_sub;
  int64_t* n_live;
  int32_t* clamped;
  int64_t* log;
} orc_trace;

static int64_t* trace_slot(orc_trace* tr, int64_t n_slots, double dt_left, double dt_sub,
                           int64_t n, int32_t clamped) {
  if (!tr || tr->count >= tr->cap) return NULL;
  int32_t k = tr->count++;
  tr->dt_left[k] = dt_left;
  tr->dt_sub[k] = dt_sub;
  tr->n_live[k] = n;
  tr->clamped[k] = clamped;
  return tr->log + (int64_t)k * 2 * (n_slots / 2);
}

static int32_t cell_adaptive(const orc_cfg* cfg, int64_t* xi, double* v, double* attrs,
                             int64_t off, int64_t n_slots, int32_t c, uint32_t s,
                             keyed_slot* scratch, int64_t* order, int64_t* log, cell_tally* tally,
                             uint32_t* status, orc_trace* tr) {
  double dt_left = cfg->dt;
  uint32_t u = 0;
  int64_t n_live0 = -1;
  while (dt_left > 0.0 && (int32_t)u < cfg->max_substeps) {
    int64_t n = cell_order(xi + off, n_slots, cfg->seed, c, s, u, scratch, order);
    if (n_live0 < 0) n_live0 = n;
    if (n < 2) break;
    double pmax = cell_pmax(cfg, xi, v, off, order, n, dt_left / cfg->dv);
    double dt_sub = (pmax <= 1.0) ? dt_left : dt_left / pmax;
    cell_tally t = {0, 0, 0};
    int64_t* tlog = trace_slot(tr, n_slots, dt_left, dt_sub, n, 1);
    cell_substep(cfg, xi, v, attrs, off, n_slots, c, s, u, dt_sub / cfg->dv, 1, scratch, order,
                 log, &t, status);
    if (tlog && log)
      for (int64_t i = 0; i < 2 * (n_slots / 2); ++i) tlog[i] = log[i];
    tally->n_colliding += t.n_colliding;
    dt_left = (dt_sub == dt_left) ? 0.0 : dt_left - dt_sub;
    u += 1;
  }
  if (dt_left > 0.0 && (int32_t)u >= cfg->max_substeps) {
    /* cap reached with time left: one unclamped substep for the remainder */
    *status |= ORC_ST_SUBSTEP_CAP;
    cell_tally t = {0, 0, 0};
    int64_t* tlog = trace_slot(tr, n_slots, dt_left, dt_left, -1, 0);
    cell_substep(cfg, xi, v, attrs, off, n_slots, c, s, u, dt_left / cfg->dv, 0, scratch, order,
                 log, &t, status);
    if (tlog) {
      tr->n_live[tr->count - 1] = t.n_live;
      if (log)
        for (int64_t i = 0; i < 2 * (n_slots / 2); ++i) tlog[i] = log[i];
    }
    tally->n_colliding += t.n_colliding;
    u += 1;
  }
  if (n_live0 < 0) n_live0 = 0;
  tally->n_live = n_live0;
  return (int32_t)u;
}

/*
 * One outer coalescence step of every cell.
 *   cell_off[C+1]: slots of cell c are [cell_off[c], cell_off[c+1]).
 *   attrs: [n_attr][n_slots].
 *   pair_log (optional): 2 int64 per candidate pair slot; cell c's pairs start
 *     at sum over c' < c of floor(n_slots(c') / 2); unused entries are -1.
 *   substeps (optional): per cell, substeps taken (adaptive mode) or 1.
 *   tallies (optional, 3 int64): sum of live SDs, candidate pairs, colliding pairs.
 * Returns the status bits.
 */
uint32_t orc_step(const orc_cfg* cfg, int64_t* xi, double* v, double* attrs,
                  const int64_t* cell_off, uint32_t step, int64_t* pair_log, int32_t* substeps,
                  int64_t* tallies) {
  int64_t C = cfg->n_cells;
  int64_t max_slots = 1;
  for (int64_t c = 0; c < C; ++c) {
    int64_t ns = cell_off[c + 1] - cell_off[c];
    if (ns > max_slots) max_slots = ns;
  }
  int64_t* pair_base = (int64_t*)malloc(sizeof(int64_t) * (size_t)(C + 1));
  pair_base[0] = 0;
  for (int64_t c = 0; c < C; ++c) pair_base[c + 1] = pair_base[c] + (cell_off[c + 1] - cell_off[c]) / 2;
  if (pair_log)
    for (int64_t i = 0; i < 2 * pair_base[C]; ++i) pair_log[i] = -1;

  double q = cfg->dt / cfg->dv;
  uint32_t status = 0;
  int64_t sum_live = 0, sum_pairs = 0, sum_coll = 0;
  int nthreads = cfg->n_threads > 1 ? cfg->n_threads : 1;
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads) reduction(| : status) \
    reduction(+ : sum_live, sum_pairs, sum_coll)
#endif
  {
    keyed_slot* scratch = (keyed_slot*)malloc(sizeof(keyed_slot) * (size_t)max_slots);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)max_slots);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
    for (int64_t c = 0; c < C; ++c) {
      int64_t off = cell_off[c];
      int64_t ns = cell_off[c + 1] - off;
      int64_t* log = pair_log ? pair_log + 2 * pair_base[c] : NULL;
      cell_tally t = {0, 0, 0};
      int32_t nsub = 1;
      if (cfg->adaptive) {
        nsub = cell_adaptive(cfg, xi, v, attrs, off, ns, (int32_t)c, step, scratch, order, log, &t,
                             &status, NULL);
      } else {
        cell_substep(cfg, xi, v, attrs, off, ns, (int32_t)c, step, 0, q, 0, scratch, order, log, &t,
                     &status);
      }
      if (substeps) substeps[c] = nsub;
      sum_live += t.n_live;
      sum_pairs += t.n_live / 2;
      sum_coll += t.n_colliding;
    }
    free(scratch);
    free(order);
  }
  (void)nthreads;
  if (tallies) {
    tallies[0] = sum_live;
    tallies[1] = sum_pairs;
    tallies[2] = sum_coll;
  }
  free(pair_base);
  return status;
}

/*
 * Test hook: one adaptive outer step of one cell (slots [0, n_slots) of the
 * given arrays, cell index c, step s), recording every substep in the trace
 * arrays (capacity cap substeps; the log holds cap x 2 floor(n_slots / 2)
 * int64).  attrs: [n_attr][n_slots] with cfg->n_slots == n_slots.  Returns
 * the number of substeps recorded; *status_out receives the status bits.
 */
int32_t orc_cell_adaptive_trace(const orc_cfg* cfg, int64_t* xi, double* v, double* attrs,
                                int64_t n_slots, int32_t c, uint32_t s, int32_t cap,
                                double* dt_left, double* dt_sub, int64_t* n_live,
                                int32_t* clamped, int64_t* log, uint32_t* status_out) {
  keyed_slot* scratch = (keyed_slot*)malloc(sizeof(keyed_slot) * (size_t)(n_slots > 0 ? n_slots : 1));
  int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_slots > 0 ? n_slots : 1));
  int64_t* one = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * (n_slots / 2) + 1));
  orc_trace tr = {cap, 0, dt_left, dt_sub, n_live, clamped, log};
  cell_tally t = {0, 0, 0};
  uint32_t status = 0;
  cell_adaptive(cfg, xi, v, attrs, 0, n_slots, c, s, scratch, order, one, &t, &status, &tr);
  free(scratch);
  free(order);
  free(one);
  if (status_out) *status_out = status;
  return tr.count;
}

/* ------------------------------------------------------------------ */
/* Moments and mass spectrum.                                          */
/* ------------------------------------------------------------------ */

/* Neumaier-compensated running sum */
typedef struct {
  double s, c;
} comp_sum;

static void comp_add(comp_sum* acc, double x) {
  double t = acc->s + x;
  if (fabs(acc->s) >= fabs(x))
    acc->c += (acc->s - t) + x;
  else
    acc->c += (x - t) + acc->s;
  acc->s = t;
}

static double comp_value(const comp_sum* acc) { return acc->s + acc->c; }

/*
 * Per cell, over live SDs: m0[c] = sum xi; m12[2c] = sum xi v; m12[2c+1] =
 * sum (xi v) v; attr_sums[c A + q] = sum xi a_q; spectrum[c B + k] = sum xi v
 * over SDs with vol_edges[k] <= v < vol_edges[k+1] (others dropped).  Any
 * output pointer may be NULL.
 */
void orc_moments(const orc_cfg* cfg, const int64_t* xi, const double* v, const double* attrs,
                 const int64_t* cell_off, int64_t* m0, double* m12, double* attr_sums,
                 const double* vol_edges, int32_t n_bins, double* spectrum) {
  int32_t A = cfg->n_attr;
  comp_sum* bins = (comp_sum*)malloc(sizeof(comp_sum) * (size_t)(n_bins > 0 ? n_bins : 1));
  comp_sum* as = (comp_sum*)malloc(sizeof(comp_sum) * (size_t)(A > 0 ? A : 1));
  for (int64_t c = 0; c < cfg->n_cells; ++c) {
    int64_t count = 0;
    comp_sum s1 = {0, 0}, s2 = {0, 0};
    for (int32_t k = 0; k < n_bins; ++k) bins[k].s = bins[k].c = 0.0;
    for (int32_t q = 0; q < A; ++q) as[q].s = as[q].c = 0.0;
    for (int64_t i = cell_off[c]; i < cell_off[c + 1]; ++i) {
      if (xi[i] <= 0) continue;
      double xd = (double)xi[i];
      double w1 = xd * v[i];
      count += xi[i];
      comp_add(&s1, w1);
      comp_add(&s2, w1 * v[i]);
      for (int32_t q = 0; q < A; ++q) comp_add(&as[q], xd * attrs[(int64_t)q * cfg->n_slots + i]);
      for (int32_t k = 0; k < n_bins; ++k) {
        if (vol_edges[k] <= v[i] && v[i] < vol_edges[k + 1]) {
          comp_add(&bins[k], w1);
          break;
        }
      }
    }
    if (m0) m0[c] = count;
    if (m12) {
      m12[2 * c] = comp_value(&s1);
      m12[2 * c + 1] = comp_value(&s2);
    }
    if (attr_sums)
      for (int32_t q = 0; q < A; ++q) attr_sums[c * A + q] = comp_value(&as[q]);
    if (spectrum)
      for (int32_t k = 0; k < n_bins; ++k) spectrum[c * n_bins + k] = comp_value(&bins[k]);
  }
  free(bins);
  free(as);
}

/* probe: a * b + c evaluated in this translation unit's FP mode (no contraction expected) */
double orc_probe_mul_add(double a, double b, double c) { return a * b + c; }

/* number of OpenMP threads available (1 without OpenMP) */
int32_t orc_max_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}
