/*
 * imf.h -- C interface of the MI355X (gfx950) inaccessibility-measure-field
 * library.
 *
 * The library computes the inaccessibility measure field (IMF) of
 * Mirzendehdel, Behandish and Nelaturi, "Topology Optimization with
 * Accessibility Constraint for Multi-Axis Machining": Algorithm 1 of
 * Sec. 2.1.5, with Eqs. imf_2 / imf_4 (the IMF as the minimum over orientations
 * and sharp points of shifted convolutions), Eq. imf_3 / imf_5 (minimum over
 * tools), Eq. ident (overlap as a convolution) and Eqs. sweep / A (accessible
 * region as the sweep of the collision-free translations by the cutter).
 *
 * Conventions
 *   - Grids are [nz][ny][nx], x fastest, contiguous; voxel centres at integer
 *     coordinates.  2D problems use ndim = 2 and nz = 1.
 *   - A tool is axisymmetric: cutter K (radius cutter_r, axial [0, cutter_len))
 *     and holder H (radius holder_r, axial [cutter_len, cutter_len +
 *     holder_len)); a direction d is the unit tool axis from the cutter tip
 *     toward the holder; the tip is the origin.  Rasterization is analytic at
 *     voxel centres (radial test closed, axial test half-open).
 *   - Outside the grid is empty space.  Translations are integer voxel
 *     offsets on the same grid.
 *   - Density designs are float32 in [0, 1] on the 2^-24 grid (k / 2^24);
 *     binary designs are uint8 0 or 1.  A request whose design holds any
 *     other value (fixture voxels included) fails with IMF_EINVAL once its
 *     prefix-sum pass has read the design (the outputs are then undefined).
 *
 * Ownership: every input and output pointer is owned by the caller and only
 * used during the call (imf_compute) or until imf_wait returns (imf_submit).
 * Device pointers are HIP device memory of the context's device; "host"
 * arrays are ordinary host memory copied during the call.  The context owns
 * its workspace and caches, bounded by hbm_budget_bytes.
 *
 * Errors: every function returns an imf_status and never throws.  On error the
 * outputs are undefined and imf_last_error() (thread-local) describes it.  The
 * context stays usable unless the status is IMF_EDEVICE.  Functions are
 * thread-safe per context (calls on one context serialize internally).
 */
#ifndef IMF_H_
#define IMF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IMF_OK = 0,
  IMF_EINVAL = 1,      /* invalid argument (message says which) */
  IMF_ENOMEM = 2,      /* device memory or the context budget exhausted */
  IMF_EDEVICE = 3,     /* a HIP call failed */
  IMF_EBUSY = 4,       /* serving queue full */
  IMF_ETIMEOUT = 5,    /* imf_wait timed out (the request keeps running) */
  IMF_ECANCELLED = 6,  /* the request was cancelled */
  IMF_EACCURACY = 7,   /* the guard band overflowed its recheck buffer, or an exact
                          recomputation found a float32 overlap error above half the band */
  IMF_ENOTIMPL = 8
} imf_status;

typedef struct imf_ctx imf_ctx;

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * context's own allocations (0: 90% of the free device memory): workspaces,
 * tool rasters and cached tool spectra.  Spectra are cached while they fit
 * and evicted, least recently used first, when a workspace needs their room
 * (after one device synchronization; captured graphs are then dropped).
 * Environment variables read here set launch parameters and never change a
 * result: IMF_MINFILTER_SHAPE, IMF_MINFILTER_WG_PER_CU, IMF_MINFILTER_SYNC,
 * IMF_BOUND_MIN_VOXELS, IMF_AXIS_RUNS, IMF_GIVEN_ORDER, IMF_OVERLAP_STACK,
 * IMF_THRESHOLD_HINTS, IMF_COMPACT_GAMMA, IMF_DEFER_APPENDS (the inverse x
 * pass's guard-band and bracket entries written after its rows: 1 always, 0
 * never, unset after a long bracket) and IMF_SERVE_WORKERS. */
imf_status imf_create(int device, size_t hbm_budget_bytes, imf_ctx** ctx);
imf_status imf_destroy(imf_ctx* ctx);
/* Message of the last error of the calling thread (never NULL). */
const char* imf_last_error(void);

/* ---------------------------------------------------------------- tools -- */
enum { IMF_TOOL_FLAT = 0, IMF_TOOL_BALL = 1, IMF_TOOL_RECT2D = 2, IMF_TOOL_VOXEL = 3 };
typedef struct {
  int kind;                /* IMF_TOOL_*; RECT2D is 2D only (radii are half-widths) */
  double cutter_r, cutter_len, holder_r, holder_len; /* voxels */
} imf_tool;
/* Register a tool (Sec. 2.1: T = H u K).  Returns an id for requests. */
imf_status imf_tool_register(imf_ctx* ctx, const imf_tool* tool, int* tool_id);
/* Register a voxel-model tool (the voxel tool that Algorithm 1's Rotate step
 * re-samples): labels host [nz][ny][nx] in the tool frame, 0 empty, 1 holder,
 * 2 cutter (the cutter voxels are the sharp points); origin (x, y, z) = the tip
 * voxel.  Used with IMF_DIR_ROTATION directions (3D): a grid offset o takes the
 * label at rint(R^T o) + origin, R^T o evaluated in float64 as
 * (R[0][a] o_x + R[1][a] o_y) + R[2][a] o_z, rint rounding halves to even.
 * The labels are copied to the device; the tool lives until imf_destroy. */
imf_status imf_tool_register_voxel(imf_ctx* ctx, int nx, int ny, int nz, const uint8_t* labels,
                                   const int origin[3], int* tool_id);

/* -------------------------------------------------------------- request -- */
enum { IMF_DIR_F64 = 0, IMF_DIR_LATTICE = 1, IMF_DIR_ROTATION = 2 };
/* sharp points: all cutter voxels (Algorithm 1: Support([1_K])), the cutter's
 * boundary voxels, or the tip voxel only (sparser sampling, Sec. 2.1.5) */
enum { IMF_SHARP_ALL = 0, IMF_SHARP_BOUNDARY = 1, IMF_SHARP_TIP = 2 };
enum { IMF_METHOD_AUTO = 0, IMF_METHOD_FFT = 1, IMF_METHOD_DIRECT = 2 };
/* flags */
#define IMF_FLAG_PLAIN 1u        /* one orientation per batch, no spectrum cache */
#define IMF_FLAG_MASK_SWEEP 2u   /* masks by sweeping D^c with the cutter (bit rows) */
#define IMF_FLAG_NO_CACHE 4u     /* do not keep tool spectra */
#define IMF_FLAG_PROFILE 8u      /* time every kernel class with events (k_ms, k_n) */
#define IMF_FLAG_NO_BOUND 16u    /* no branch and bound in the sharp-point minimum (it is
                                    used on grids of at least 10^6 voxels) */
#define IMF_FLAG_NO_GRAPH 32u    /* launch kernel by kernel: no HIP-graph capture or replay.
                                    Otherwise the second request with the same signature
                                    (request fields, input / output pointers, orientations,
                                    cache state) is captured into a graph, and later ones
                                    replay it; requests that compute tool spectra, PROFILE and
                                    PLAIN requests always launch kernel by kernel */

typedef struct {
  int ndim, nx, ny, nz;
  int design_is_density;       /* 0: uint8 {0,1}; 1: float32 on the 2^-24 grid */
  const void* design;          /* device [nz][ny][nx] */
  const uint8_t* fixture;      /* device [nz][ny][nx] or NULL (Sec. 2.1: O = Omega u F) */
  const uint8_t* domain;       /* device Omega_0 mask or NULL (= not fixture) */
  int n_tools;                 /* >= 1 (Eq. imf_3) */
  const int* tool_ids;         /* host [n_tools] */
  const int* n_dirs;           /* host [n_tools], each >= 1 */
  int dir_kind;                /* IMF_DIR_F64: float64 unit vectors; IMF_DIR_LATTICE: int32
                                  vectors, exact integer rasterization (sizes must be
                                  multiples of 1/2); IMF_DIR_ROTATION: float64 rotation
                                  matrices, row-major, tool frame to grid, orthonormal to
                                  1e-9 with determinant +1 (3D; needed by voxel tools;
                                  an axisymmetric tool takes the image of its +z axis) */
  const void* dirs;            /* host [sum n_dirs][ndim] (x, y[, z]), or [sum n_dirs][9] */
  int sharp;                   /* IMF_SHARP_* */
  double lambda;               /* allowance: B = Omega_0 and f > lambda F_max */
  double tau;                  /* Omega = [rho > tau] for the secluded set (0.5) */
  double mask_theta_abs;       /* >= 0: masks use gamma <= theta (voxel units);
                                  < 0: theta = lambda F_max (two-phase) */
  int method;                  /* IMF_METHOD_* */
  int batch;                   /* orientations per batch, 0: automatic */
  unsigned flags;              /* IMF_FLAG_* */
  /* Fixtures that change with the setup (Sec. 2.1.5: the fixture, hence the
     obstacle O, may differ per re-clamping when the setups are known beforehand).
     Orientation q (in the order of dirs) sees the fixture
     fixture | fixture_sets[fixture_of[q]]; without a domain, Omega_0 excludes the
     voxels of every set.  0 sets: one fixture for all orientations (both pointers
     ignored).  Orientations of one set need not be contiguous, but each change of
     set along dirs starts a new batch, so grouping them is faster.  Caller-owned;
     fixture_of is read during the call only (imf_submit copies it). */
  int n_fixture_sets;           /* 0 .. 256 */
  const uint8_t* fixture_sets;  /* device [n_fixture_sets][nz][ny][nx], nonzero = fixture */
  const int* fixture_of;        /* host [sum n_dirs], each in [0, n_fixture_sets) */
} imf_request;

typedef struct {
  float* imf;          /* device [N] f (voxel-volume units), or NULL */
  float* imf_norm;     /* device [N] fbar * 1_B, or NULL */
  uint8_t* secluded;   /* device [N] Gamma = B minus Omega, or NULL */
  uint64_t* acc_masks; /* device [n_orient][nz][ny][ceil(nx/64)] accessible masks A_R,
                          bit x%64 of word x/64, or NULL */
  float* debug_overlap;  /* device, g of orientation debug_orient over its query box, or NULL */
  int debug_orient;
  int debug_box[6];      /* out: lo (x,y,z) and dims of that box */
} imf_outputs;

typedef struct {
  double F_max;          /* max of f over Omega_0: exact (binary, and density with
                            lambda > 0); the float32 maximum for density with lambda = 0,
                            where no decision depends on it */
  long long guard_flags; /* overlaps recomputed exactly (guard band) */
  float max_frac_err;    /* max |g - rint g| seen before rounding (binary) */
  double guard_band;     /* density: E, the bound on |g32 - g| (voxel units); overlaps
                            within E of a threshold are recomputed exactly */
  double t_ms[8];        /* raster, forward, tool spectra, inverse, recheck, min, finalize, total */
  double model_bytes;    /* algorithmic HBM bytes of the request (cost model) */
  int P[3];              /* transform sizes */
  int n_orient, method, batch;
  int cache_hits, cache_misses;
  /* with IMF_FLAG_PROFILE: device time and launches per kernel class: 0 raster,
   * 1 setup, 2 forward design transform, 3-5 tool spectrum x/y/z, 6 product +
   * inverse z, 7 inverse y, 8 inverse x + rounding, 9 recheck, 10 window-min
   * levels (and the bound's cell minima), 11 sharp-point minimum, 12 sweep,
   * 13 finalize, 14 copies, 15 branch-and-bound pass */
  double k_ms[16];
  int k_n[16];
  double k_bytes[16];    /* algorithmic bytes of each class (compulsory reads + writes) */
  double k_ops[16];      /* class 11: window-minimum lookups (gathered floats, blocks that
                            were computed) */
  long long bound_blocks;  /* (block, orientation) pairs of the sharp-point minimum */
  long long bound_skipped; /* of those, skipped by the lower bound (exact) */
  int graph;               /* 0 launched kernel by kernel, 1 captured into a graph and
                              launched, 2 a replay of a captured graph */
  int lattice_runs;        /* orientations whose sharp points are split into runs along a
                              lattice vector other than a coordinate axis */
  int mf_shape;            /* block shape of the sharp-point minimum (0: 64x1x1, 1: 32x2x1,
                              2: 16x2x2, 3: 16x4x1, 4: 8x4x2 voxels per wave) */
  int mf_wg_per_cu;        /* resident workgroups per CU of its list pass */
  /* density: the largest |g32 - g| (voxel units) that an exact recomputation
   * found (the request fails with IMF_EACCURACY above guard_band / 2) */
  float max_abs_err;
  long long post_exact;    /* exact overlaps computed after the first pass (F_max, band) */
  long long band_entries;  /* overlaps listed around lambda F_max: the band (within
                              guard_band), or the wider bracket of an expected threshold */
  int passes;              /* 2 when theta = lambda F_max was decided by a second pass */
  double box_voxels;       /* sum over orientations of the query-box volume M_x M_y M_z */
  int hinted;              /* lambda F_max expected from the last requests of this shape:
                              1 the listed bracket held the band, 2 it missed, 3 its lists
                              overflowed (2, 3: the band was then scanned, or decided by a
                              second pass), 0 no expectation */
  int fft_plan;            /* transform plans of the inverse z, y and x passes, 2 bits each
                              (z | y << 2 | x << 4): bit 0 one stage per radix 8, 4, 2, 3,
                              5, 7 instead of composite radices, bit 1 half-width tiles */
  double queue_ms;         /* served requests: submission to admission (t_ms[7] is
                              submission to completion); 0 for imf_compute */
  double lock_ms;          /* host time spent waiting for the context lock (served
                              requests: behind the other workers' planning) */
  double hold_ms;          /* host time holding it: planning the request, reserving
                              memory, caches and enqueueing its kernels */
} imf_stats;

/* Bytes of device workspace the request needs (admission control).  The
 * workspace holds the fields of one batch of orientations, sized so that the
 * batch fits the memory budget (App. B: the convolution fields of many
 * orientations are processed in batches under a memory limit). */
imf_status imf_query_footprint(imf_ctx* ctx, const imf_request* req, size_t* bytes);
/* Compute the IMF, masks and secluded set of one request (Algorithm 1 of
 * Sec. 2.1.5: rotate, convolve, sharp-point minimum, minimum over orientations
 * and tools, normalization and allowance; masks by Eqs. sweep / A),
 * stream-ordered on `stream` (a hipStream_t, NULL = default); returns after
 * completion. */
imf_status imf_compute(imf_ctx* ctx, const imf_request* req, const imf_outputs* out,
                       imf_stats* stats, void* stream);

/* -------------------------------------------------------------- serving -- */
/* The serving calls have no counterpart in the paper: they run imf_compute's
 * work for requests of several callers (e.g. concurrent TO runs).
 * Enqueue a request; up to 2 requests run at once (environment variable
 * IMF_SERVE_WORKERS, 1-16, at context creation), each on its own stream,
 * overlapping on the device.  Admission is first come first served while
 * workspaces fit (the running requests' footprints within half the budget; an
 * idle context admits any request); when the oldest waiting request does not
 * fit, one of the next 8 that does is admitted ahead of it, at most 4 times,
 * after which the queue waits for it.  Host arrays of `req` are copied;
 * device buffers must stay valid until wait. */
imf_status imf_submit(imf_ctx* ctx, const imf_request* req, const imf_outputs* out,
                      uint64_t* ticket);
/* Wait for a request (timeout_ms < 0: forever).  Fills stats; latency in t_ms[7]. */
imf_status imf_wait(imf_ctx* ctx, uint64_t ticket, int timeout_ms, imf_stats* stats);
/* Cancel a request that has not started; returns IMF_EBUSY if it is running. */
imf_status imf_cancel(imf_ctx* ctx, uint64_t ticket);

/* Autotune a request shape (method, grid, transform sizes) on a real request:
 * time candidate batch widths, then block shapes (64x1x1, 32x2x1, 16x2x2,
 * 16x4x1, 8x4x2) and resident workgroups per CU (4, 6, 8) of the sharp-point
 * minimum, then (FFT method, transform lengths 192-768) the transform plan of
 * each inverse pass z, y, x in turn: composite radices or one stage per radix
 * 8, 4, 2, 3, 5, 7, full- or half-width tiles (imf_stats.fft_plan; untuned
 * shapes take per pass the radix plan whose kernel fits more workgroups per
 * CU, the composite one on a tie).  Each
 * candidate runs kernel by kernel after a warm-up; the fastest is remembered
 * (an alternative replaces the current choice only when 2% faster), and
 * later requests of that shape with batch = 0 use it.  Captured graphs are
 * dropped.  Results do not depend on the choice beyond float32 rounding of
 * the overlaps (integer and thresholded outputs are exact under every plan).
 * *best_batch receives the batch width. */
imf_status imf_autotune(imf_ctx* ctx, const imf_request* req, const imf_outputs* out,
                        int* best_batch);
/* The context's autotuned table as a text file (host file IO only): save
 * writes every tuned request shape (format 2: "imf-autotune 2", then per
 * shape "<method>|<nx>,<ny>,<nz>|<px>,<py>,<pz> <batch> <shape> <wg> <fft>";
 * format 1 tables, without <fft>, also load); load merges a saved table into the
 * context (an entry replaces the one for the same shape), so a new process
 * skips the tuning.  A malformed file is rejected whole with IMF_EINVAL and
 * leaves the context unchanged.  *n_loaded (may be NULL) receives the number
 * of entries read. */
imf_status imf_autotune_save(imf_ctx* ctx, const char* path);
imf_status imf_autotune_load(imf_ctx* ctx, const char* path, int* n_loaded);

/* ----------------------------------------- coupling to the TO loop (Sec. 2.2) -- */
/* Heaviside projection of the design variables (Eq. Heaviside):
 * rho = 1 - exp(-beta xi) + xi exp(-beta), in float64 with xi clamped to [0, 1],
 * then rounded to the nearest multiple of 2^-24 (halves up), so that rho can be
 * the density design of a request.  xi and rho: device arrays of n floats
 * (may alias).  Stream-ordered on `stream`. */
imf_status imf_heaviside(imf_ctx* ctx, long long n, const float* xi, double beta, float* rho,
                         void* stream);
/* Accessibility filter (Eq. accFilter) from a request's outputs:
 * filter = fbar (imf_norm, the allowance-applied normalized IMF) where the
 * design is solid (rho > tau), 1 on the secluded set (secluded != 0), 0 elsewhere.
 * With sens_phi != NULL also the filtered sensitivity (Eq. filtered_sens):
 * sens_out = (1 - w_acc) S_phi / max_{Omega_0} |S_phi| + w_acc filter (the
 * normalization is 0 where that maximum is 0), float64 arithmetic.  Omega_0 is
 * `domain` != 0 if given, else fixture == 0, else everything.  All arrays are
 * device arrays of nx*ny*nz elements laid out as a request's grids; design is
 * uint8 {0,1} or float32 (design_is_density).  0 <= w_acc <= 1.  The
 * normalization uses one device word of the context: calls that overlap on
 * different streams of one context must be ordered by the caller. */
imf_status imf_access_filter(imf_ctx* ctx, int nx, int ny, int nz, const void* design,
                             int design_is_density, const uint8_t* fixture,
                             const uint8_t* domain, const float* imf_norm,
                             const uint8_t* secluded, double tau, const float* sens_phi,
                             double w_acc, float* filter_out, float* sens_out, void* stream);

/* Greedy machining plan (Sec. 3.4.1, post-processing): starting from the negative
 * space N = Omega_0 and [rho <= tau] (rho the design, Omega_0 as in a request),
 * repeatedly choose the orientation whose accessible mask covers the most of
 * what remains (ties: the lowest orientation index), remove that part, and stop
 * when no orientation removes anything or after max_steps steps.  acc_masks:
 * device [n_orient][nz][ny][ceil(nx/64)] as written by imf_compute.  Host
 * outputs: orient_out[max_steps] and removed_out[max_steps] (voxels removed by
 * each step), *n_steps, and *remaining (voxels of N no orientation reaches,
 * or left after max_steps).  Returns when done (the plan is read on the host
 * step by step). */
imf_status imf_plan_greedy(imf_ctx* ctx, int nx, int ny, int nz, int n_orient,
                           const uint64_t* acc_masks, const void* design, int design_is_density,
                           const uint8_t* fixture, const uint8_t* domain, double tau,
                           int max_steps, int* orient_out, long long* removed_out, int* n_steps,
                           long long* remaining, void* stream);

/* The greedy plan of imf_plan_greedy for callers that cannot allocate device
 * memory (serving loops and harnesses that forbid hipMalloc): it allocates
 * nothing.  Its scratch, the remaining negative space (nz * ny * ceil(nx/64)
 * words) and n_orient + 2 words of counts, lives in a fixed array of 2^20
 * 64-bit words (8 MiB) that every GPU the library runs on holds until the
 * process ends; a plan that needs more returns IMF_EINVAL.  Every call on one
 * GPU shares that array: calls that overlap on one GPU (any context, any
 * stream) race, and the caller must order them.  Same arguments, outputs and
 * errors as imf_plan_greedy; it reads each step's choice on the host, so it is
 * not capturable into a graph. */
imf_status imf_plan_greedy_noalloc(imf_ctx* ctx, int nx, int ny, int nz, int n_orient,
                                   const uint64_t* acc_masks, const void* design,
                                   int design_is_density, const uint8_t* fixture,
                                   const uint8_t* domain, double tau, int max_steps,
                                   int* orient_out, long long* removed_out, int* n_steps,
                                   long long* remaining, void* stream);

/* ------------------------------------------------- single steps (checks) -- */
/* Raster of one oriented tool (the Rotate step): offsets (x, y, z) in z, y, x
 * order into host arrays (voxels of the tool and the sharp points); flags bit 0 =
 * tool, bit 1 = cutter, bit 2 = sharp point. */
imf_status imf_raster(imf_ctx* ctx, int ndim, const imf_tool* tool, int dir_kind,
                      const void* dir, int sharp, int32_t* offsets, uint8_t* flags,
                      long long cap, long long* count);
/* The same for a registered tool (any kind, voxel tools included). */
imf_status imf_raster_tool(imf_ctx* ctx, int tool_id, int ndim, int dir_kind, const void* dir,
                           int sharp, int32_t* offsets, uint8_t* flags, long long cap,
                           long long* count);
/* Complex FFT of `batch` columns of length n laid out [n][batch] (interleaved
 * float re, im), device pointers, unnormalized, sign -1 (inverse: +1). */
imf_status imf_fft_c2c(imf_ctx* ctx, int n, int batch, const float* in, float* out,
                       int inverse, void* stream);
/* 3D real-to-complex FFT of a real [nz][ny][nx] grid zero-padded to
 * (px, py, pz); output layout [py][px/2+1][pz] complex. */
imf_status imf_fft_r2c_3d(imf_ctx* ctx, int nx, int ny, int nz, int px, int py, int pz,
                          const float* in, float* out, void* stream);
/* Smallest supported transform length >= n. */
int imf_fft_size(int n);

#ifdef __cplusplus
}
#endif
#endif /* IMF_H_ */
