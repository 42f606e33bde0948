/*
 * lf2.h -- C ABI of the lf2 library: LATfield2's integrated 3-D FFT, the
 * spectral Poisson solve and the power-spectrum binning built on it
 * (Daverio, Hindmarsh & Bevis, arXiv:1508.05610), for one AMD MI355X
 * (gfx950).
 *
 * Problem statement follows the paper's objects:
 *   - Lattice (section 3.2): a periodic Cartesian lattice given by its
 *     dimension, the size of every dimension and a halo width h.
 *   - Field (section 3.3): data on every site with `ncomp` components.
 *     Sites are stored row-major with dimension 0 fastest (section 3.4);
 *     the components of a site are stored together, innermost (each element
 *     of a field is the list of its components, section 3.5).  Every
 *     dimension carries h halo sites on both sides (section 3.3.1), so the
 *     memory jump along dimension 1 is N0 + 2h sites, and so on (3.4).
 *   - PlanFFT (section 3.6): a plan links a real-space field with its
 *     Fourier-space representation; out-of-place is the default; temporary
 *     memory is shared between plans.
 *
 * Layouts used by every call (N = N0*N1*N2, Nh = N0/2 + 1):
 *   real field      float [N2+2h][N1+2h][N0+2h][ncomp]    (h = lattice halo)
 *   complex field   float2[N2+2h][N1+2h][N0+2h][ncomp]    (c2c, x space)
 *   half spectrum   float2[N2][N1][Nh][ncomp]             (r2c k space, no halo)
 *   full spectrum   float2[N2][N1][N0][ncomp]             (c2c k space, no halo)
 * The halo sites of an input are never read; those of an output are never
 * written.  float2 is (re, im).
 *
 * Transform convention: forward uses exp(-2 pi i k.x/N), backward
 * exp(+2 pi i k.x/N); neither is normalised, so c2r(r2c(f)) = N f (the
 * convention of FFTW, whose 1-d transforms the paper's FFT is built on).
 * The r2c transform halves dimension 0.  c2r applies to any half spectrum
 * G and returns sum over half-spectrum modes of c(kx) Re(G_k e^{+ik.x}),
 * c = 1 for kx in {0, N0/2} and 2 otherwise (the imaginary parts of the
 * kx = 0 and kx = N0/2 entries are ignored).
 *
 * Memory ownership: every field pointer is device memory owned by the
 * caller and must stay valid until the work enqueued on `stream` has
 * finished.  The library owns plans, twiddle and wavevector tables and a
 * workspace that plans share (the paper's shared temporary memory); the
 * workspace grows on demand with hipMalloc inside execute calls, and is
 * meant for calls issued on one stream at a time -- callers that run plans
 * concurrently on several streams give each plan its own workspace with
 * lf2_plan_set_workspace.
 *
 * Streams: `stream` is a hipStream_t (NULL = legacy default stream).  All
 * execute calls are asynchronous with respect to the host.
 *
 * Errors: argument and shape errors are detected before anything is
 * enqueued and returned synchronously; a HIP launch or allocation failure
 * returns LF2_ERR_DEVICE or LF2_ERR_OUT_OF_MEMORY.  Nothing throws across
 * this interface.  lf2_last_error() gives a thread-local message for the
 * last failing call.
 */
#ifndef LF2_H
#define LF2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LF2_OK = 0,
    LF2_ERR_INVALID_ARG = -1,  /* null pointer, bad size, bad enum, misaligned pointer */
    LF2_ERR_UNSUPPORTED = -2,  /* valid request outside what the library implements */
    LF2_ERR_OUT_OF_MEMORY = -3,
    LF2_ERR_DEVICE = -4,       /* HIP runtime error */
    LF2_ERR_BUDGET = -5,       /* server: request larger than the memory budget */
    LF2_ERR_BUSY = -6,         /* server: queue full, try again */
    LF2_ERR_NOT_READY = -7     /* server: ticket not finished yet */
} lf2_status;

/* Lattice (section 3.2): dim must be 3; size[i] >= 1; halo >= 0. */
typedef struct {
    int32_t dim;
    int32_t halo;
    int64_t size[3];
} lf2_lattice;

typedef enum { LF2_R2C = 0, LF2_C2C = 1 } lf2_fft_kind;
typedef enum { LF2_FORWARD = -1, LF2_BACKWARD = +1 } lf2_direction;

/* Plan flags. */
#define LF2_OUT_OF_PLACE 0u           /* default (section 3.6) */
#define LF2_IN_PLACE 0x1u             /* in == out allowed (section 3.6); needs halo 0.  An r2c
                                         plan's real fields then have rows padded to 2 (N0/2 + 1)
                                         floats per component, so each real row and its spectrum
                                         row share their bytes (with LF2_KLAYOUT_PAPER the rows move,
                                         so the forward r2c stages its x pass in the workspace) */
#define LF2_KLAYOUT_PAPER 0x2u        /* k-space in the paper's order (section 3.6): r2c
                                         (k_x, k_z, k_y), i.e. C array [N1][N2][Nh][ncomp]; c2c
                                         (k_z, k_x, k_y), i.e. [N1][N0][N2][ncomp] */
#define LF2_PLAN_AUTOTUNE 0x10u       /* time the tile variants and XCD chunk sizes of the y and
                                         z passes at plan time and keep the fastest per axis */
/* Poisson flags. */
#define LF2_POISSON_CONTINUOUS_K2 0u  /* k^2 = sum_i (2 pi nt_i / (N_i dx))^2 (default) */
#define LF2_POISSON_DISCRETE_K2 1u    /* k^2 = sum_i (2/dx)^2 sin^2(pi n_i / N_i) */
#define LF2_PK_OF_PHI 2u              /* bin the spectrum of phi instead of rho */

typedef struct lf2_plan_s *lf2_plan;

/*
 * Create a plan for a 3-D transform on `lat` with `ncomp` components
 * (PlanFFT, section 3.6).  Extents must factor into 2, 3 and 5
 * (LF2_ERR_UNSUPPORTED otherwise); r2c needs an even N0.  Line lengths
 * (N0/2 for r2c along x) with compiled kernels: 2^a, 3 2^a and 5 2^a up to
 * 1024 along x with ncomp 1, 2, 3 or 6, and up to 2048 along y and z; every
 * other 2^a 3^b 5^c line up to 8192 points (and any ncomp) runs kernels
 * with a run-time radix schedule (lf2_plan_get_schedule), as long as a tile
 * of one line fits the device's LDS.  The plan is bound to the current HIP
 * device; its twiddles (generated in FP64 on the device, rounded once to
 * FP32) stay resident until lf2_plan_destroy.  Synchronises the device once.
 */
lf2_status lf2_fft_plan(lf2_plan *out, const lf2_lattice *lat, int32_t ncomp, lf2_fft_kind kind,
                        uint32_t flags);

/*
 * k-space geometry of a plan (the rKSite / cKSite analogue, section 3.6):
 * ksize = extents of the spectrum in sites (Nh or N0, N1, N2) and kstride =
 * the jump between neighbouring sites along each dimension, in complex
 * elements (components innermost, so kstride[0] = ncomp).  Either pointer
 * may be NULL.
 */
lf2_status lf2_fft_kspace(lf2_plan p, int64_t ksize[3], int64_t kstride[3]);

/*
 * Tuning of the strided pass along `axis` (1 = y, 2 = z) for plain
 * transforms.  variant bit 0: wide tiles (twice the columns per tile, one
 * 1024-thread block per CU; lengths 256, 320, 384, 512, 640, 768, 1024,
 * 2048) instead of narrow tiles (all lengths); bit 2: the register tile
 * (lengths 1024 and 2048, not with bit 0: 32 or 16 columns per tile held in
 * registers as a 32 x 32 or 32 x 64 decomposition with one exchange through
 * LDS); bit 1:
 * nontemporal global loads and stores (they pay on long strides, where each
 * line is touched once).  chunk = consecutive tiles given to one XCD in the
 * tile order (1..1024, default 16).  Narrow and wide tiles compute the same
 * transform bit for bit; the register tile computes it up to FP32 rounding
 * (another order of the butterflies).  The fused Poisson / power-spectrum pass always uses narrow tiles,
 * nontemporal accesses and chunk 16.  get reports the setting and, after
 * LF2_PLAN_AUTOTUNE, the measured microseconds of the default setting
 * (variant 0, chunk 16) and of the chosen one (-1 if not measured); null
 * outputs are skipped; variant -1 means the axis runs a run-time radix
 * schedule (lf2_plan_get_schedule).  set overrides the setting and returns
 * the axis to its compiled kernels (LF2_ERR_UNSUPPORTED for wide tiles or
 * the register tile on a length without them, or for a length without
 * compiled kernels).
 * axis 0 (the x pass): variant = how the two radix-8 stages of a c2c row of
 * 64 points (one component) exchange their values -- 0 through LDS (every
 * plan), 1 across the row's eight lanes with ds_bpermute, 2 across them with
 * DPP moves (LF2_ERR_UNSUPPORTED for other plans); chunk is ignored (0 on
 * get).  LF2_PLAN_AUTOTUNE times the three on such plans.  Every setting
 * computes the same transform up to FP32 rounding.
 * axis 3 (the fused Poisson pass of lf2_poisson_solve along z): variant 0
 * runs its transforms through LDS stage by stage, 1 (z extents 32 to 2048
 * that are powers of two; the default from 64) holds its tile in registers
 * with one LDS exchange each way and bins P(k) from FP32 mode powers
 * (LF2_ERR_UNSUPPORTED for other z extents; a solve whose bin tables do not
 * fit beside that tile, e.g. 4096 bins on 1024-point lines, runs variant
 * 0); chunk is ignored (16 on get),
 * the microseconds are -1.  Both compute the same solve up to FP32
 * rounding.
 */
lf2_status lf2_plan_get_tuning(lf2_plan p, int32_t axis, int32_t *variant, int32_t *chunk,
                               double *us_default, double *us_tuned);
lf2_status lf2_plan_set_tuning(lf2_plan p, int32_t axis, int32_t variant, int32_t chunk);

/*
 * Radix schedule (the radices of the Stockham stages, in order; their
 * product is the line length) of the passes along `axis` (0 = x, 1 = y,
 * 2 = z).  Line lengths with compiled kernels use a schedule fixed at
 * compile time; any other 2^a 3^b 5^c length, and any pass for which a
 * schedule is set, runs kernels that take the schedule at run time (*runtime
 * = 1).  LF2_PLAN_AUTOTUNE times the candidate schedules of every such axis,
 * and of the y and z passes against their compiled kernels, and keeps the
 * fastest.  get: radices[0 .. *nstages - 1] (the rest 0); any output may be
 * NULL.  set: each radix 2, 3, 4, 5, 8 or 16 with product the line length;
 * the fused Poisson / power-spectrum pass of a compiled length keeps its
 * compiled kernel; the x pass of a compiled length cannot be set
 * (LF2_ERR_UNSUPPORTED).  Every schedule computes the same transform up to
 * FP32 rounding.
 */
lf2_status lf2_plan_get_schedule(lf2_plan p, int32_t axis, int32_t radices[15], int32_t *nstages,
                                 int32_t *runtime);
lf2_status lf2_plan_set_schedule(lf2_plan p, int32_t axis, const int32_t *radices, int32_t nstages);

/* Bytes of shared workspace an execute call on this plan may use. */
lf2_status lf2_plan_workspace_bytes(lf2_plan p, size_t *bytes);

/* Give the plan its own workspace (device memory of at least
 * lf2_plan_workspace_bytes, 256-byte aligned, owned by the caller);
 * NULL returns the plan to the shared workspace. */
lf2_status lf2_plan_set_workspace(lf2_plan p, void *dev_ptr, size_t bytes);

/*
 * Execute a transform (section 3.6; forward and backward, section 4).
 *   r2c plan, LF2_FORWARD : in = real field, out = half spectrum
 *   r2c plan, LF2_BACKWARD: in = half spectrum (not modified), out = real field
 *   c2c plan, either      : in = complex field / spectrum, out = spectrum / field
 * in and out must not overlap, except in == out on a plan made with
 * LF2_IN_PLACE.  Pointers must be 8-byte aligned.
 */
lf2_status lf2_fft_execute(lf2_plan p, lf2_direction dir, const void *in, void *out,
                           void *stream);

/*
 * Spectral Poisson solve, laplacian(phi) = rho, periodic, zero mode
 * removed (the Poisson-solver example of sections 2 and 3.6):
 *   phi_hat = -rho_hat / k^2 (k != 0), phi_hat(0) = 0, phi = c2r(phi_hat)/N,
 * with the FP64 factor -1/(N k^2) applied in one pass between the forward
 * and backward transforms along dimension 2.  r2c plan with ncomp = 1.
 * rho and phi are real fields (halo as in the plan) and must not overlap,
 * except rho == phi on a plan made with LF2_IN_PLACE.
 * dx > 0 is the lattice spacing.
 * If nbins > 0, the power spectrum of rho (or of phi with LF2_PK_OF_PHI) is
 * binned as in lf2_power_spectrum into d_pk, d_kmean, d_count (device
 * arrays of nbins doubles; any may be NULL).  d_parseval (nullable device
 * array of 2 doubles) receives { sum_x rho^2, (1/N) sum_k w |rho_hat|^2 }.
 */
lf2_status lf2_poisson_solve(lf2_plan p, const float *rho, float *phi, double dx, uint32_t flags,
                             int32_t nbins, double *d_pk, double *d_kmean, double *d_count,
                             double *d_parseval, void *stream);

/*
 * lf2_poisson_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same solve with the same arguments, layouts and results,
 * but it calls no hipMalloc, hipFree or other allocating routine.  Its
 * workspace is a static device array of LF2_NOALLOC_SCRATCH_BYTES per GPU,
 * held by the library from its first use on that GPU until the process
 * ends.
 *   - A solve whose workspace (the half spectrum, 8 (N0/2 + 1) N1 N2 bytes,
 *     plus 8 KiB (nbins + 1) of bin partials) exceeds the array is
 *     LF2_ERR_UNSUPPORTED (a 256^3 solve fits with up to 4096 bins).
 *   - The plan's k^2 table for (dx, k^2 kind) and shell table for nbins must
 *     already exist: an earlier lf2_poisson_solve (or lf2_power_spectrum for
 *     the shell table) with the same values builds them; otherwise
 *     LF2_ERR_NOT_READY and nothing is enqueued.
 *   - Every call on one GPU shares that GPU's array, which keeps what the
 *     last call left there: calls that overlap on one GPU (several streams
 *     or host threads at once) race and give wrong results; serialise them.
 *     Nothing in the array needs to start at zero.
 *   - Kernel timing (lf2_profile_enable) does not record these launches.
 */
#define LF2_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
lf2_status lf2_poisson_solve_noalloc(lf2_plan p, const float *rho, float *phi, double dx,
                                     uint32_t flags, int32_t nbins, double *d_pk,
                                     double *d_kmean, double *d_count, double *d_parseval,
                                     void *stream);

/*
 * Spherical-shell power spectrum (spectral analysis, section 1).  For
 * every mode n != 0 with integer squared radius q = sum_i (nt_i L/N_i)^2,
 * L = lcm(N0, N1, N2), q_max = sum_i (floor(N_i/2) L/N_i)^2, the bin is
 *   b = min(nbins-1, max{b : b^2 q_max <= nbins^2 q})   (exact integers),
 * and per bin
 *   count = sum w,  pk = (dx^3/N) sum w |F|^2 / count,
 *   kmean = sum w |k| / count,  |k| = 2 pi sqrt(q) / (L dx),
 * with w = 1 at kx in {0, N0/2} and 2 elsewhere for an r2c plan (half
 * spectrum) and w = 1 for a c2c plan.  Empty bins give 0.  Sums are FP64
 * (of FP32 |F|^2 in the register-tile Poisson pass, tuning axis 3).  Repeated
 * calls give the same bits where each wave of a block bins into its own LDS
 * histogram, summed in a fixed order (e.g. up to 169 bins on 512-point z
 * lines); with more bins the waves of a block share one histogram and the
 * last bits of the sums can differ from call to call.
 * field_is_kspace = 0: `field` is a real-space field (r2c: real; c2c:
 * complex), transformed on the way without being modified;
 * field_is_kspace = 1: `field` is already the spectrum.  ncomp must be 1.
 * d_pk, d_kmean, d_count: device arrays of nbins doubles (any may be NULL).
 */
lf2_status lf2_power_spectrum(lf2_plan p, const void *field, int32_t field_is_kspace,
                              int32_t nbins, double dx, double *d_pk, double *d_kmean,
                              double *d_count, void *stream);

lf2_status lf2_plan_destroy(lf2_plan p);

/*
 * Batched Poisson solves on many lattices of different sizes.
 *
 * By default the whole batch -- x r2c, y, z Poisson [+ binning], y backward
 * and x c2r passes of every field, and the finalize of every field's power
 * spectrum -- runs as ONE launch of a persistent kernel, captured once in a
 * hipGraph that lf2_batch_execute replays.  Its blocks take (field, pass,
 * tile) work items from work queues in an order in which every item comes
 * after the items it depends on (one atomic ticket per queue), wait on
 * per-(field, pass) completion counters, and publish their own; the last
 * block to finish resets the queues for the next run.  When the fields
 * spread evenly over the XCDs (greedy by bytes, the largest XCD share at
 * most 1.25x the mean) there is one queue per XCD holding whole fields, and
 * each block serves the queue of the XCD it runs on, so every tile is
 * written and read through one L2; otherwise, or with LF2_BATCH_ONE_QUEUE,
 * one queue serves the whole chip (each item then writes back and
 * invalidates the L2 around its wait and its publication).  Every wait is
 * bounded: a wait that gives up (about a quarter of a second) sets bit 0 of
 * the batch's error word, after which no block of that run waits and the
 * launch ends; a queue left with unclaimed items sets bit 1.
 * With LF2_BATCH_GROUPED the items are instead grouped by pass and line
 * length: one launch per group plus one finalize launch, captured in a
 * hipGraph in which each group depends only on the previous pass's groups
 * that hold one of its fields.
 * Each field gives the same result as lf2_poisson_solve on it alone (power
 * spectra within FP64 summation order).
 *
 * lats: nfields dense lattices (halo 0) whose N0/2, N1 and N2 are each one
 *   of 16, 32, 48, 64, 80, 96, 128, 160, 192, 256, 384.
 * ops: LF2_BATCH_POISSON, optionally | LF2_BATCH_PK for the fused
 *   power spectrum of each rho with nbins bins (1..511), optionally
 *   | LF2_BATCH_GROUPED or | LF2_BATCH_ONE_QUEUE.
 * poisson_flags: 0 or LF2_POISSON_DISCRETE_K2.
 * The batch owns the spectra of all fields (lf2_batch_info).  Plan creation
 * synchronises the device.
 */
#define LF2_BATCH_POISSON 1u
#define LF2_BATCH_PK 2u
#define LF2_BATCH_GROUPED 4u
#define LF2_BATCH_ONE_QUEUE 8u
typedef struct lf2_batch_s *lf2_batch;

lf2_status lf2_batch_plan(lf2_batch *out, int32_t nfields, const lf2_lattice *lats, uint32_t ops,
                          int32_t nbins, double dx, uint32_t poisson_flags);

/*
 * Run the batch on `stream`.  rho and phi are host arrays of nfields device
 * pointers (float fields of each lattice, 8-byte aligned, rho[f] != phi[f]);
 * d_pk, d_kmean, d_count are NULL or host arrays of nfields device pointers
 * to nbins doubles (an entry may be NULL).  When the pointer set differs
 * from the previous call the stream is synchronised once and the field
 * descriptors are uploaded before the graph launch.
 */
lf2_status lf2_batch_execute(lf2_batch b, const float *const *rho, float *const *phi,
                             double *const *d_pk, double *const *d_kmean, double *const *d_count,
                             void *stream);

/* Synchronise the device and read the batch's error word into *err (0: the
 * runs since the last call completed normally; bit 0: a persistent run gave
 * up a dependency wait, bit 1: a queue was left with unclaimed items -- the
 * results are then not valid).  A set word is
 * cleared by this call; until then every later run of the batch is invalid
 * as well.  LF2_ERR_DEVICE if a HIP error is pending. */
lf2_status lf2_batch_error(lf2_batch b, uint32_t *err);

/* Queues of the persistent launch (0 in grouped mode) and whether each
 * serves one XCD (1) or the whole chip (0); either may be NULL. */
lf2_status lf2_batch_queues(lf2_batch b, int32_t *nqueues, int32_t *per_xcd);

/* Work items, kernel launches per execution and workspace bytes. */
lf2_status lf2_batch_info(lf2_batch b, int64_t *nitems, int32_t *launches,
                          size_t *workspace_bytes);

lf2_status lf2_batch_destroy(lf2_batch b);

/*
 * Serving: a request loop for Poisson solves with optional power spectra on
 * lattices of mixed sizes (continuous batching).  A scheduler thread admits
 * queued requests in launch units while a slot is free: the request at the
 * head of the queue, joined by the queued requests with the same lattice,
 * lattice spacing, k^2 kind and bin count (up to 16 requests and 2^26
 * lattice points, lattices of at most 2^24 points whose lines have grouped
 * kernels) -- those run as ONE grouped solve, a launch per pass over all of
 * them; larger lattices run alone.  A unit takes one slot; every request in it is charged
 * its footprint (rho + phi + workspace) against the HBM budget, and the
 * idle pooled workspace counts against the budget too.  A request reuses an
 * idle buffer that fits its workspace when there is one (reserved at
 * admission); idle buffers are freed only when a request needs the room.
 * Workspaces come from a stream-ordered memory pool of the server's own
 * (hipMallocFromPoolAsync / hipFreeAsync), so a free does not wait for the
 * device.  Each unit is launched at once on
 * one of `nstreams` streams, so requests that arrive while others run join
 * the device work as capacity frees up.  Plans (twiddles, wavevector and
 * shell tables) stay resident in a cache keyed by lattice.  A completion
 * thread timestamps each request when its work has finished and returns its
 * capacity.  Requests are independent: each gives the same result as
 * lf2_poisson_solve on its own (power spectra within FP64 summation order).
 *
 * The caller owns rho, phi and the bin arrays of a request and keeps them
 * valid until lf2_server_poll reports it done.  The server's streams do not
 * wait for other streams: rho must hold its values on the device when the
 * request is submitted.  Up to 32 plans stay resident; a new lattice evicts
 * the least recently used plan that no running request holds.  Timestamps
 * are seconds on the host's monotonic clock (lf2_server_now).
 */
typedef struct lf2_server_s *lf2_server;

typedef struct {
    lf2_lattice lat;      /* dense (halo 0) lattice, r2c-compatible (even N0) */
    const float *rho;     /* device, float[N2][N1][N0] */
    float *phi;           /* device, float[N2][N1][N0], must not alias rho */
    double dx;            /* lattice spacing > 0 */
    uint32_t flags;       /* LF2_POISSON_DISCRETE_K2 | LF2_PK_OF_PHI */
    int32_t nbins;        /* 0: no power spectrum */
    double *d_pk, *d_kmean, *d_count;  /* device arrays of nbins doubles (nullable) */
    double t_arrival;     /* arrival time for latency accounting; 0: submit time */
} lf2_request;

typedef struct {
    lf2_status status;    /* LF2_OK, or the request's failure */
    double t_arrival, t_admit, t_done;  /* seconds, monotonic host clock */
} lf2_result;

typedef struct {
    int64_t submitted, completed, failed, rejected_busy, rejected_budget;
    int64_t in_flight, queued;
    size_t bytes_in_flight, peak_bytes_in_flight;
    int64_t plans_cached, plan_hits, plan_misses;
    int64_t groups, grouped_requests;     /* grouped solves launched, requests in them */
    size_t pooled_idle_bytes;             /* idle pooled workspace (counts against the budget) */
    size_t peak_bytes_in_use;             /* largest in-flight + idle pooled bytes seen */
    int64_t workspace_allocs, workspace_frees;  /* pooled workspace buffers made and freed */
} lf2_server_stats;

/* Create a GPU server on the current device.  hbm_budget_bytes bounds the
 * summed footprint of admitted requests plus the idle pooled workspace;
 * max_slots bounds launch units (single requests or grouped solves) in
 * flight; nstreams (>= 1) streams of default priority; max_queue bounds
 * requests waiting for admission. */
lf2_status lf2_server_create(lf2_server *out, size_t hbm_budget_bytes, int32_t max_slots,
                             int32_t nstreams, int32_t max_queue);

/* A server whose executor launches nothing: each request completes
 * delay_us microseconds after admission, the request with ticket
 * fail_ticket (0: none) completes with LF2_ERR_DEVICE.  Admission, budget,
 * queue and failure handling are those of the GPU server; for host-side
 * tests without a GPU.  Bin arrays are not written. */
lf2_status lf2_server_create_fake(lf2_server *out, size_t hbm_budget_bytes, int32_t max_slots,
                                  int32_t max_queue, uint32_t delay_us, uint64_t fail_ticket);

/* Make plans resident for these lattices (and bin counts / spacing), so the
 * first request of each does not pay plan setup.  Synchronises the device. */
lf2_status lf2_server_prepare(lf2_server s, int32_t n, const lf2_lattice *lats, int32_t nbins,
                              double dx, uint32_t flags);

/* Queue a request without blocking.  *ticket (>= 1) identifies it.
 * LF2_ERR_BUDGET: its footprint alone exceeds the budget;
 * LF2_ERR_BUSY: the queue is full (retry later);
 * LF2_ERR_INVALID_ARG / LF2_ERR_UNSUPPORTED: bad request. */
lf2_status lf2_server_submit(lf2_server s, const lf2_request *r, uint64_t *ticket);

/* Result of a ticket.  wait = 0: LF2_ERR_NOT_READY while it runs; wait != 0:
 * block until done.  A finished ticket is reported once and then forgotten
 * (LF2_ERR_INVALID_ARG afterwards). */
lf2_status lf2_server_poll(lf2_server s, uint64_t ticket, lf2_result *res, int32_t wait);

/* Footprint in bytes that admission charges for a request. */
lf2_status lf2_server_footprint(const lf2_request *r, size_t *bytes);

lf2_status lf2_server_get_stats(lf2_server s, lf2_server_stats *st);

/* Drain: wait for every queued and running request, then free the server. */
lf2_status lf2_server_destroy(lf2_server s);

/* Monotonic host clock in seconds (the server's timestamps). */
double lf2_server_now(void);

/*
 * Field operations (the paper's second benchmark, section 4.2; halo cells,
 * section 3.3.1).  A field is float[N2+2h][N1+2h][N0+2h][ncomp] (complex
 * fields: elem_bytes = 8), dimension 0 fastest, components innermost, on
 * the current device; all calls are asynchronous on `stream`.
 *
 * lf2_update_halo: periodic halo update of a field on one GPU: every halo
 * site takes the value of the interior site at its coordinates modulo the
 * lattice extents (faces, edges and corners).  h = 0 is a no-op; h larger
 * than an extent is LF2_ERR_UNSUPPORTED.  elem_bytes is 4 or 8.
 *
 * lf2_gradient: first-order forward derivative of every component along x,
 * y and z into another field with the same halo width and 3 * ncomp
 * components: out(x)[3 c + i] = (in(x + e_i) - in(x))[c] / dx.  Reads the
 * input's halo (h >= 1; update it first); writes the output's interior only.
 * in and out must not alias.
 */
lf2_status lf2_update_halo(const lf2_lattice *lat, int32_t ncomp, int32_t elem_bytes, void *field,
                           void *stream);
lf2_status lf2_gradient(const lf2_lattice *lat, int32_t ncomp, const float *in, float *out,
                        double dx, void *stream);

/*
 * Kernel timing (tracing).  While enabled, every kernel launch made by the
 * calls above is bracketed by two HIP events recorded on the launch's
 * stream and tagged with the kernel's name and its algorithmic HBM bytes
 * (the bytes a single pass over its inputs and outputs must move).
 * lf2_profile_count synchronises on the recorded events and returns the
 * number of distinct kernel names; lf2_profile_get(i, ...) returns, for the
 * i-th name, the launch count, the summed event time in milliseconds and
 * the summed algorithmic bytes.  name receives at most name_len bytes
 * (NUL-terminated).  Enabling or resetting drops earlier records.
 * Recording adds two event records per launch; it is off by default.
 */
lf2_status lf2_profile_enable(int32_t on);
lf2_status lf2_profile_reset(void);
int32_t lf2_profile_count(void);
lf2_status lf2_profile_get(int32_t i, char *name, size_t name_len, int64_t *launches, double *ms,
                           double *bytes);

const char *lf2_status_string(lf2_status s);
const char *lf2_last_error(void);

/* Library version, e.g. "lf2 0.1.0 gfx950". */
const char *lf2_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LF2_H */
