/* Test driver: runs the CPU oracle (oracle/sdm_oracle.c, linked in) on inputs
 * read from a file and writes every output, so that a build of the oracle
 * under AddressSanitizer and UndefinedBehaviorSanitizer can be compared with
 * the regular build.  Test infrastructure only.
 *
 * Input file (native endianness): int64 n_slots, n_cells, n_attr, kernel,
 * adaptive, max_substeps, n_threads, n_steps, n_bins; uint64 seed; double dt,
 * dv, b; then int64 xi[n_slots], double v[n_slots], double
 * attrs[n_attr * n_slots], int64 cell_off[n_cells + 1], double
 * edges[n_bins + 1].
 *
 * Output file: per step, uint32 status, int64 tallies[3], int32
 * substeps[n_cells], int64 pair_log[2 * pairs]; then int64 xi, double v,
 * double attrs, int64 m0[n_cells], double m12[2 n_cells], double
 * attr_sums[n_cells n_attr], double spectrum[n_cells n_bins].
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int64_t n_slots;
  int32_t n_cells;
  int32_t n_attr;
  double dt;
  double dv;
  double b;
  int32_t kernel;
  int32_t adaptive;
  int32_t max_substeps;
  int32_t n_threads;
  uint64_t seed;
} orc_cfg;

uint32_t orc_step(const orc_cfg* cfg, int64_t* xi, double* v, double* attrs,
                  const int64_t* cell_off, uint32_t step, int64_t* pair_log, int32_t* substeps,
                  int64_t* tallies);
void orc_moments(const orc_cfg* cfg, const int64_t* xi, const double* v, const double* attrs,
                 const int64_t* cell_off, int64_t* m0, double* m12, double* attr_sums,
                 const double* vol_edges, int32_t n_bins, double* spectrum);

static void* take(FILE* f, size_t bytes) {
  void* p = malloc(bytes ? bytes : 1);
  if (!p || (bytes && fread(p, 1, bytes, f) != bytes)) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
  return p;
}

static void put(FILE* f, const void* p, size_t bytes) {
  if (bytes && fwrite(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short write\n");
    exit(2);
  }
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE* in = fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t* h = (int64_t*)take(in, 9 * sizeof(int64_t));
  uint64_t* seed = (uint64_t*)take(in, sizeof(uint64_t));
  double* fl = (double*)take(in, 3 * sizeof(double));
  orc_cfg cfg;
  cfg.n_slots = h[0];
  cfg.n_cells = (int32_t)h[1];
  cfg.n_attr = (int32_t)h[2];
  cfg.kernel = (int32_t)h[3];
  cfg.adaptive = (int32_t)h[4];
  cfg.max_substeps = (int32_t)h[5];
  cfg.n_threads = (int32_t)h[6];
  const int64_t n_steps = h[7], n_bins = h[8];
  cfg.seed = *seed;
  cfg.dt = fl[0];
  cfg.dv = fl[1];
  cfg.b = fl[2];
  const size_t N = (size_t)cfg.n_slots, C = (size_t)cfg.n_cells, A = (size_t)cfg.n_attr;
  int64_t* xi = (int64_t*)take(in, N * sizeof(int64_t));
  double* v = (double*)take(in, N * sizeof(double));
  double* attrs = (double*)take(in, A * N * sizeof(double));
  int64_t* off = (int64_t*)take(in, (C + 1) * sizeof(int64_t));
  double* edges = (double*)take(in, (size_t)(n_bins + 1) * sizeof(double));
  fclose(in);

  int64_t pairs = 0;
  for (size_t c = 0; c < C; ++c) pairs += (off[c + 1] - off[c]) / 2;
  int64_t* log = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * pairs + 1));
  int32_t* sub = (int32_t*)malloc(sizeof(int32_t) * (C + 1));
  FILE* out = fopen(argv[2], "wb");
  if (!out) return 2;
  for (int64_t s = 0; s < n_steps; ++s) {
    int64_t tallies[3] = {0, 0, 0};
    const uint32_t st = orc_step(&cfg, xi, v, A ? attrs : NULL, off, (uint32_t)s, log, sub, tallies);
    put(out, &st, sizeof st);
    put(out, tallies, sizeof tallies);
    put(out, sub, C * sizeof(int32_t));
    put(out, log, (size_t)(2 * pairs) * sizeof(int64_t));
  }
  put(out, xi, N * sizeof(int64_t));
  put(out, v, N * sizeof(double));
  put(out, attrs, A * N * sizeof(double));
  int64_t* m0 = (int64_t*)malloc(sizeof(int64_t) * (C + 1));
  double* m12 = (double*)malloc(sizeof(double) * (2 * C + 1));
  double* as = (double*)malloc(sizeof(double) * (C * A + 1));
  double* spec = (double*)malloc(sizeof(double) * (C * (size_t)n_bins + 1));
  orc_moments(&cfg, xi, v, A ? attrs : NULL, off, m0, m12, as, edges, (int32_t)n_bins, spec);
  put(out, m0, C * sizeof(int64_t));
  put(out, m12, 2 * C * sizeof(double));
  put(out, as, C * A * sizeof(double));
  put(out, spec, C * (size_t)n_bins * sizeof(double));
  fclose(out);
  free(h);
  free(seed);
  free(fl);
  free(xi);
  free(v);
  free(attrs);
  free(off);
  free(edges);
  free(log);
  free(sub);
  free(m0);
  free(m12);
  free(as);
  free(spec);
  return 0;
}
