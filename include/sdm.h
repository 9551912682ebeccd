/*
 * sdm.h -- C ABI of libsdm: the Super-Droplet Method (SDM) Monte-Carlo
 * collision-coalescence step on AMD Instinct MI355X (gfx950).
 *
 * The operation.  The PySDM v1 paper (arXiv 2103.17238) builds a simulation
 * from a super-droplet count and a backend ("API in brief": Builder(n_sd,
 * backend)), a Box environment of time step dt and volume dV, the
 * Coalescence dynamic with a collision kernel such as Golovin(b), and the
 * initial attributes 'volume' and 'n' (multiplicity); it is advanced with
 * run(n_steps) and read through products such as the dv/dlnr spectrum.  The
 * coalescence step is the SDM of Shima et al. (2009), which the paper names as
 * the package core ("Introduction").  Here:
 *   sdm_init             <-> Builder + Box + Coalescence + build(attributes)
 *   sdm_coalescence_step <-> run(n_steps)
 *   sdm_moments          <-> the dv/dlnr product (and total moments)
 * Per step and per cell: a random permutation of the live super-droplets (SDs)
 * from 32-bit Philox4x32-10 keys ordered by (key, slot); neighbour pairs;
 * the pair probability p = max(xi_a, xi_b) K(v_a, v_b) dt/dV scaled by
 * n(n-1)/2 / floor(n/2); gamma = floor(p) + [phi < p - floor(p)] from a 53-bit
 * uniform phi; and the multiplicity / extensive-attribute update with the
 * equal-multiplicity split.  Kernels: Golovin K = b (v1 + v2) ("API in
 * brief") and geometric sweep-out K = pi (r1 + r2)^2 |u1 - u2| with the
 * continuous three-regime terminal velocity of Rogers & Yau (1989) ("Box
 * environment examples", the Berry 1966 example).  Every random number is a
 * function of (seed, cell, step, substep, index) only, so results do not
 * depend on launch shape, batching or tuning.
 *
 * Memory and ownership.
 *   - Every pointer argument named dev_* or documented as "device" is device
 *     memory owned by the caller (e.g. torch tensors).  The library borrows
 *     the state arrays (xi, v, attrs, cell_off) and the workspace for the
 *     lifetime of the handle; it never allocates or frees device memory.
 *   - The library allocates only the host-side handle and, at the first step
 *     of a simulation or batch, one more HIP stream (default priority) and two
 *     events, plus a second stream and one more event at the first step with
 *     cells in the 4096- or 8192-slot mid-size classes (see mid_max_slots);
 *     sdm_free / sdm_batch_free release them.
 *   - Layout is structure-of-arrays: xi[n_slots] (int64), v[n_slots] (float64,
 *     m^3), attrs[n_attr][n_slots] (float64, extra extensive attributes summed
 *     on coalescence like volume), cell_off[n_cells + 1] (int64, slots of cell
 *     c are [cell_off[c], cell_off[c+1]), cell_off[0] = 0, cell_off[n_cells] =
 *     n_slots, at most 8 388 608 slots per cell: a layout with a larger cell
 *     is invalid).  An SD with xi = 0 is dead and keeps its slot.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *
 * Errors.  Every call returns an sdm_status; nothing aborts and no exception
 * crosses the ABI.  Device-side conditions set bits of a per-simulation status
 * word (sdm_status_word).
 *
 * Threading.  Step and moments calls only enqueue work on `stream` and return.
 * Parts of a step may run on the library's own streams, which wait for
 * `stream` (an event) and are joined back into it before the call returns, so
 * work enqueued on `stream` afterwards sees the step complete.  One handle
 * must not be stepped on two streams at once: a step call (alone or in a
 * batch) on another stream than the one its last steps were enqueued on,
 * while those still run, returns SDM_EAGAIN and enqueues nothing.
 *
 * Synchronisation.  No call synchronises the whole device.  Calls that set
 * up launch tables (sdm_init, sdm_batch_create, sdm_set_tuning, sdm_rebind,
 * sdm_autotune) synchronise their `stream`; sdm_status_word and sdm_stats
 * synchronise `stream` to read back.  Calls without a stream argument
 * (sdm_debug_gamma_sink, sdm_batch_workspace_bytes,
 * sdm_autotune_scratch_bytes) are host-only, except right after a
 * device-side sdm_rebind, when they first copy the new offsets to the host
 * with a blocking copy.  The HIP runtime maps streams onto a few hardware
 * queues (GPU_MAX_HW_QUEUES, 4 by default); streams that share a queue run
 * in order, so synchronising `stream` then also waits for work enqueued
 * earlier on the streams it shares a queue with.
 */
#ifndef SDM_H
#define SDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sdm_sim sdm_sim;     /* opaque host handle of one simulation */
typedef struct sdm_batch sdm_batch; /* opaque group of simulations stepped by shared launches */

typedef enum {
  SDM_OK = 0,
  SDM_EINVAL = -1,  /* bad argument, configuration or initial state */
  SDM_ENOMEM = -2,  /* workspace too small */
  SDM_EDEVICE = -3, /* a HIP call failed */
  SDM_ESTATE = -4,  /* call not valid in the handle's current state */
  SDM_EAGAIN = -5   /* resource busy */
} sdm_status;

typedef enum { SDM_GOLOVIN = 0, SDM_GEOMETRIC = 1 } sdm_kernel_kind;

/* bits of the device status word */
#define SDM_FLAG_SUBSTEP_CAP 1u     /* adaptive: max_substeps reached, remainder done unclamped */
#define SDM_FLAG_GAMMA_CAP 2u       /* some p >= 2^62: gamma capped at 2^62 */
#define SDM_FLAG_BUCKET_OVERFLOW 4u /* big-cell sort used its slow path (still exact) */
#define SDM_FLAG_INVALID_STATE 8u   /* validation found xi < 0, xi >= 2^53 or a bad volume */
#define SDM_FLAG_COURANT 16u        /* displacement: some |d| >= 1 cell or a position outside [0, 1) */

typedef struct {
  int64_t n_slots;        /* SD slots (live and dead), >= 0 */
  int32_t n_cells;        /* >= 1 */
  int32_t n_attr;         /* extra extensive attributes, 0..16 */
  double dt_s;            /* time step [s], > 0 (Box dt) */
  double dv_m3;           /* cell volume [m^3], > 0 (Box dv) */
  int32_t kernel;         /* sdm_kernel_kind */
  int32_t adaptive;       /* 1: per-cell substepping keeping gamma <= 1 */
  double golovin_b_per_s; /* Golovin b [1/s] (volume-based kernel), >= 0 */
  uint64_t seed;          /* Philox key */
  int32_t max_substeps;   /* adaptive substep cap per step (0 = 1024) */
  int32_t reserved;       /* must be 0 */
} sdm_config;

/* Launch-shape knobs.  They change speed only, never results. */
typedef struct {
  int32_t wave_class_mask;   /* bit k (k = 0..4) enables the workgroup-per-cell class of
                                64, 128, 256, 384, 512 slots; a cell goes to the smallest
                                enabled class that fits; bit 4 (512) is always on.  Classes
                                up to 256 slots and the mid-size cells run on the library's
                                side streams beside the larger classes and the big-cell
                                kernels */
  int32_t waves_per_cell;    /* 1, 2, 4 or 8: wavefronts in the workgroup of one cell */
  int32_t big_bucket_target; /* cells on the big-cell path: expected SDs per bucket (a key
                                range ordered by one workgroup), 32..1024; 0 (the default)
                                chooses per cell: 128 up to 32768 slots, 256 up to 65536,
                                512 above */
  int32_t lpt_order;         /* 1: dispatch cells by descending size (adaptive cells: at the
                                first step; after it they go by the substeps they took in
                                the step before, most first) */
  int32_t mid_max_slots;     /* cells of 513..mid_max_slots slots (<= 16384) get one workgroup
                                each (mid-size kernel); larger ones take the big-cell path
                                (two launches per step); 0 sends every cell above 512 there.
                                -1 (the default) chooses: adaptive cells up to 16384 slots
                                get the mid-size kernel; plain cells of 4097..16384 slots
                                too when a plan (or batch) has more than 32 of them, else
                                the big-cell path (faster for a few cells, slower for many);
                                plain cells of 513..4096 slots the mid-size kernel, or the
                                big-cell path when the plan uses it anyway and has at most
                                32 of them */
  int32_t big_bucket_cap;    /* big-cell path: longest bucket one workgroup orders in LDS;
                                longer ones are ranked in global memory (still exact,
                                slower, SDM_FLAG_BUCKET_OVERFLOW); 0 = 1024, else 1..1024 */
} sdm_tuning;

/*
 * Workspace bytes sdm_init needs.  host_cell_off (optional, host memory,
 * n_cells + 1 entries) gives the exact size for that cell layout; with NULL
 * the result is an upper bound valid for any layout.  Returns 0 on a bad cfg.
 */
size_t sdm_workspace_bytes(const sdm_config* cfg, const int64_t* host_cell_off);

/*
 * Create a simulation over caller-owned device state (see "Memory and
 * ownership").  attrs may be NULL when n_attr = 0.  workspace: device memory
 * of at least sdm_workspace_bytes bytes, 256-byte aligned.  Copies cell_off
 * to the host, validates cfg, plans the launches and uploads the tables,
 * and validates the state (one kernel), all ordered on `stream`, which it
 * synchronises (twice; work on other streams keeps running).  The step
 * counter starts at 0.
 * Returns SDM_EINVAL for a bad cfg/state, SDM_ENOMEM if the workspace is
 * too small.
 */
sdm_status sdm_init(sdm_sim** out, const sdm_config* cfg, int64_t* xi, double* v, double* attrs,
                    const int64_t* cell_off, void* workspace, size_t workspace_bytes,
                    void* stream);

/* Advance n_steps >= 0 outer steps (enqueue only, except below). Steps beyond the step limit
 * are skipped.  SDM_EAGAIN: the simulation's last steps were enqueued on another stream and
 * still run.  Adaptive mode with cells on the big-cell path (above the mid-size limit): the
 * number of substeps is found on the device, so the call synchronises `stream` once every
 * 4 substep rounds of each step. */
sdm_status sdm_coalescence_step(sdm_sim* s, int32_t n_steps, void* stream);

/*
 * Per-cell moments of the live SDs, written to device buffers (any may be
 * NULL): m0[C] = sum xi (int64, exact); m12[C][2] = (sum xi v, sum xi v^2);
 * attr_sums[C][A] = sum xi a_q; spectrum[C][n_bins] = sum xi v over SDs with
 * vol_edges[k] <= v < vol_edges[k+1] (vol_edges: device, n_bins + 1 increasing
 * volumes [m^3], 1 <= n_bins <= 1024; SDs outside are dropped).  One pass over
 * each cell's slots.  dm/dlnr of bin k is
 * rho_w spectrum / dV / ln(r_{k+1} / r_k).  Sums use a fixed reduction order,
 * so a cell's moments do not depend on the rest of the state.
 */
sdm_status sdm_moments(sdm_sim* s, int64_t* m0, double* m12, double* attr_sums,
                       const double* vol_edges, int32_t n_bins, double* spectrum, void* stream);

/*
 * Diffusional growth (condensation / evaporation).  The paper lists
 * condensational growth among the dynamics beside coalescence ("API in
 * brief") and pairs it with ambient thermodynamics in its parcel examples
 * ("Adiabatic parcel examples": activation of aerosol by supersaturation,
 * hygroscopicity), without fixing the physics; the readings are:
 * kappa-Koehler equilibrium saturation (Petters & Kreidenweis 2007), the
 * Maxwell-Mason growth law r dr/dt = (S - S_eq) / (F_k + F_d) (Rogers & Yau
 * 1989) with Bolton's saturation pressure and Pruppacher & Klett's
 * diffusivity, and one implicit Euler step in r^2 solved by bracketed
 * Newton iterations; the ambient state of each cell is held over the step.
 * A super-droplet's dry volume and kappa x dry volume are two of its
 * extensive attributes (summed on coalescence).  Only live wet volumes v
 * change; the condensed mass of a cell follows from sdm_moments (M1) before
 * and after.
 */
typedef struct {
  double dt_s;             /* time step [s], > 0 */
  int32_t dry_volume_attr; /* attribute holding the dry volume [m^3] */
  int32_t kappa_attr;      /* attribute holding kappa x dry volume [m^3] (another one) */
  int32_t max_iter;        /* Newton iterations per super-droplet, at most 64 (0: 32) */
  int32_t reserved;        /* must be 0 */
} sdm_cond_config;

/* One condensation step of every live super-droplet (enqueue only, except that
 * right after a device-side sdm_rebind the host copy of the offsets is
 * refreshed with a blocking copy).  temperature [K], pressure [Pa] and
 * saturation (saturation ratio, e.g. 1.002 for 0.2 % supersaturation):
 * device arrays of n_cells values each, read on `stream`.  SDM_EINVAL for a
 * bad config (attribute indices outside 0..n_attr-1 or equal); SDM_EAGAIN
 * as for a step when the simulation is busy on another stream. */
sdm_status sdm_condensation_step(sdm_sim* s, const sdm_cond_config* cc, const double* temperature,
                                 const double* pressure, const double* saturation, void* stream);

/* Device status word (SDM_FLAG_* bits); synchronises `stream`. */
sdm_status sdm_status_word(sdm_sim* s, uint32_t* flags, void* stream);
/* Clear the status word and the statistics counters (enqueue). */
sdm_status sdm_reset_status(sdm_sim* s, void* stream);

/*
 * Statistics accumulated since init / reset (synchronises `stream`):
 * out[0] live SD-steps (live SDs at the start of each outer step, summed),
 * out[1] colliding pairs (gamma > 0), out[2] cell substeps, out[3] cell steps.
 */
sdm_status sdm_stats(sdm_sim* s, uint64_t out[4], void* stream);

/* Step counter (outer steps taken; the Philox counter word). */
uint32_t sdm_get_step(const sdm_sim* s);
sdm_status sdm_set_step(sdm_sim* s, uint32_t step);
/* Steps at or beyond `limit` are skipped (UINT32_MAX = no limit). */
sdm_status sdm_set_step_limit(sdm_sim* s, uint32_t limit);

/*
 * Test hook: per candidate pair of the last (sub)step, dev_buf[2 i] =
 * a | (b << 32) (cell-local slots of the pair), dev_buf[2 i + 1] = gamma,
 * where cell c's pairs start at i = sum over c' < c of floor(slots(c') / 2);
 * unused entries are -1.  capacity is in int64 elements (>= 2 x that total).
 * NULL turns the sink off.
 */
sdm_status sdm_debug_gamma_sink(sdm_sim* s, int64_t* dev_buf, int64_t capacity);

/* Launch-shape knobs: get, set (re-plans; same results), and an autotuner. */
sdm_status sdm_get_tuning(const sdm_sim* s, sdm_tuning* t);
sdm_status sdm_set_tuning(sdm_sim* s, const sdm_tuning* t, void* stream);
/*
 * Time candidate tunings on a scratch copy of the state (scratch: device,
 * >= sdm_autotune_scratch_bytes) for trial_steps steps each, apply the
 * fastest to s and, if cache_path is not NULL, record it in that JSON file
 * keyed by device, kernel, n_attr, mode and a cell-size histogram; a cached
 * entry is reused without timing.  cache_path NULL takes the file named by
 * the environment variable SDM_TUNE_CACHE, when set and not empty (no cache
 * otherwise).  s's own state and step counter are not touched.  chosen
 * (optional) receives the tuning.
 */
size_t sdm_autotune_scratch_bytes(const sdm_sim* s);
sdm_status sdm_autotune(sdm_sim* s, void* scratch, size_t scratch_bytes, int32_t trial_steps,
                        const char* cache_path, sdm_tuning* chosen, void* stream);

/*
 * Batches: simulations stepped together by shared launches (one launch per
 * step covers every member's cells).  Members keep their own state, seed,
 * kernel, counters and status.  workspace: device, >= sdm_batch_workspace_bytes.
 * Members must stay alive while the batch exists.  sdm_batch_create builds the
 * launch tables on the host, uploads them on `stream` and synchronises `stream`.
 */
size_t sdm_batch_workspace_bytes(sdm_sim* const* sims, int32_t n);
sdm_status sdm_batch_create(sdm_batch** out, sdm_sim* const* sims, int32_t n, void* workspace,
                            size_t workspace_bytes, void* stream);
/* Advance every member n_steps (each member honours its own step limit).
 * SDM_ESTATE if a member was re-pointed by sdm_rebind since the batch was made.
 * SDM_EAGAIN (nothing enqueued) if a member's last steps were enqueued on another
 * stream (alone or in another batch) and still run. */
sdm_status sdm_batch_step(sdm_batch* b, int32_t n_steps, void* stream);
void sdm_batch_free(sdm_batch* b);

void sdm_free(sdm_sim* s);
const char* sdm_strerror(sdm_status st);

/*
 * Re-point a simulation at new state arrays of the same n_slots and n_cells
 * (for instance the output of sdm_displace, whose cell sizes differ) and
 * re-plan its launches.  The step counter, tuning, statistics and status are
 * kept.  When the plan holds only cells of up to 512 slots and no gamma sink
 * is set, a few kernels rewrite the launch tables from the new offsets on the
 * device and the call synchronises `stream` once to read back two words;
 * if a cell outgrew its size class, slots landed in a cell that had none, or
 * the offsets are not a valid layout, it falls back to the host re-plan:
 * cell_off is copied to the host and validated like in sdm_init.  If a HIP
 * call fails on the way, the old layout is re-planned (SDM_EDEVICE); if that
 * fails too, later step calls return SDM_ESTATE.  Returns
 * SDM_EINVAL for an invalid layout (the handle keeps its old one), SDM_ENOMEM
 * if the new layout needs more workspace than the handle was given (size it
 * with sdm_workspace_bytes(cfg, NULL) to allow any layout).  A batch
 * containing s must be re-created afterwards: sdm_batch_step returns
 * SDM_ESTATE for a batch whose members were re-pointed after it was made.
 */
sdm_status sdm_rebind(sdm_sim* s, int64_t* xi, double* v, double* attrs, const int64_t* cell_off,
                      void* stream);

/*
 * Displacement and re-segmentation.  The paper lists particle displacement
 * among the dynamics beside coalescence ("API in brief") and couples the
 * particles to a prescribed single-eddy flow in its kinematic 2D example
 * ("Kinematic (prescribed-flow) examples") without giving a scheme; this is
 * one explicit first-order step:
 *   - cells c = ix * nz + iz of an nx x nz domain, periodic in x and z,
 *     nx, nz >= 1 (along an axis of one cell a droplet that crosses a face
 *     re-enters its cell; along an axis of two, both directions lead to the
 *     other cell: a 1D column is nx = 1);
 *   - pos[2][n_slots] (float64): each droplet's position inside its cell as
 *     fractions wx = pos[0][j], wz = pos[1][j] in [0, 1);
 *   - Courant numbers on cell faces: courant_x[(nx + 1) * nz], entry
 *     ix * nz + iz on the face between cells ix - 1 and ix of row iz;
 *     courant_z[nx * (nz + 1)], entry ix * (nz + 1) + iz on the face between
 *     cells iz - 1 and iz of column ix;
 *   - per axis d = (1 - w) c_low + w c_high (two products and a sum), w' = w + d,
 *     the cell moves by floor(w') (wrapped), the new fraction is w' - floor(w')
 *     (one that rounds to 1 becomes 0 in the next cell up);
 *   - |d| < 1 is required: a droplet with |d| >= 1, or whose fraction is not
 *     in [0, 1), raises SDM_FLAG_COURANT in *status (its move is clamped to one
 *     cell per axis; the result is defined but not meaningful);
 *   - the output state holds every slot (dead ones too) ordered by new cell;
 *     inside a new cell the slots keep their old relative order (old cell,
 *     then old slot).  cell_off_out is the new layout.
 * All pointers are device memory owned by the caller; outputs must not
 * overlap inputs.  An input cell_off that is not a valid layout of n_slots
 * raises SDM_FLAG_INVALID_STATE and leaves the outputs unwritten.  Enqueue
 * only (four kernels, no allocation, no synchronisation).
 */
typedef struct {
  int32_t nx, nz;          /* cells per axis, >= 1 each */
  int32_t n_attr;          /* extra attributes, 0..16 */
  int32_t reserved;        /* must be 0 */
  int64_t n_slots;         /* 0 .. 2^32 - 2 */
  const double* courant_x; /* [(nx + 1) * nz] */
  const double* courant_z; /* [nx * (nz + 1)] */
  const int64_t* xi;       /* input state, layout as in sdm_init */
  const double* v;
  const double* attrs; /* [n_attr][n_slots] */
  const double* pos;   /* [2][n_slots] */
  const int64_t* cell_off;
  int64_t* xi_out; /* output state, same shapes */
  double* v_out;
  double* attrs_out;
  double* pos_out;
  int64_t* cell_off_out;
  uint32_t* status; /* device word; SDM_FLAG_COURANT / SDM_FLAG_INVALID_STATE or-ed in */
} sdm_displace_args;

/* Workspace bytes of sdm_displace for an nx x nz domain (0 if invalid). */
size_t sdm_displace_workspace_bytes(int32_t nx, int32_t nz);
/* workspace: device, 256-byte aligned, >= sdm_displace_workspace_bytes. */
sdm_status sdm_displace(const sdm_displace_args* args, void* workspace, size_t workspace_bytes,
                        void* stream);

/*
 * sdm_displace without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, checks, kernels and
 * results as sdm_displace; the workspace is instead a file-scope device array
 * of the library (9.5 MiB, held on each GPU the library runs on until the
 * process ends), big enough for nx * nz <= sdm_displace_noalloc_max_cells()
 * (2^17) cells: larger domains return SDM_ENOMEM and enqueue nothing.  The
 * call allocates nothing (the array's device address is looked up once per
 * device at the first call there).  Every call on one GPU uses the same
 * array, whose contents are rewritten before they are read, so calls that
 * overlap on one GPU (other streams, other host threads) race: serialise
 * them.  Enqueue only.
 */
sdm_status sdm_displace_noalloc(const sdm_displace_args* args, void* stream);
int64_t sdm_displace_noalloc_max_cells(void);

/*
 * Test hook for the generator: out[4 i + w] = word w of Philox4x32-10 with
 * counter (c0 + i, c1, c2, c3) and key (seed mod 2^32, seed / 2^32), for
 * i < n (device buffer of 4 n uint32).  Enqueue only.
 */
sdm_status sdm_philox_fill(uint32_t* out, int64_t n, uint32_t c0, uint32_t c1, uint32_t c2,
                           uint32_t c3, uint64_t seed, void* stream);

/* Test hook: K(v1[i], v2[i]) for n pairs of device volumes into device out. */
sdm_status sdm_kernel_values(int32_t kernel, double golovin_b, const double* v1, const double* v2,
                             int64_t n, double* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SDM_H */
