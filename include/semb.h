/*
 * semb.h -- C ABI of the MI355X (gfx950) semblance parameter-scan library.
 *
 * The operations are those of Hu, Yang, Luan and Qian, "Massively Scaling
 * Seismic Processing on Sunway TaihuLight Supercomputer":
 *
 *   cmp_scan        exhaustive CMP velocity scan (section 2.1 and the grid
 *                   search of section 3.2): for every output sample t0 of a
 *                   gather and every candidate q = 4/v^2, the semblance of
 *                   Eq. (1) over a w-sample window centred on each trace's
 *                   intersection with the traveltime curve, linearly
 *                   interpolated (Algorithm 1); then the most coherent
 *                   parameter per sample and the stacked amplitude along it.
 *   crs_scan        the same for the 2D CRS method (section 2.2): the traces
 *                   of the neighbouring gathers join the central gather's and
 *                   the curve becomes a surface in (A, B, q).
 *   stack           semblance and stack at one given parameter per output
 *                   sample (the same sums as above, evaluated once).
 *   semblance_grad  gradient of sum_rows g_s[row] * S(row) with respect to
 *                   each row's parameter and to every input sample.
 *
 * Definitions shared by every call (readings of the paper that it does not
 * spell out):
 *   t0 = s * dt for output sample s = 0 .. ns[central]-1;
 *   CMP traveltime  T = t0^2 + q h^2;
 *   CRS traveltime  T = (t0 + 2 A dm)^2 + 2 t0 B dm^2 + q h^2, dm = midpoint of
 *                   the trace - central_x of the job's central gather;
 *   tau = sqrt(T)/dt, k = floor(tau), x = tau - k, window start a = k - (w-1)/2,
 *   window sample j = f[a+j] + x (f[a+j+1] - f[a+j]), j = 0 .. w-1;
 *   a trace contributes only if T >= 0, a >= 0 and a + w <= ns - 1 (its own ns);
 *   S = sum_j U_j^2 / (M D), U_j = sum of window sample j over contributing
 *   traces, D = sum of their squares, M = number of contributing traces;
 *   S = 0 when M = 0 or D = 0;  stack = (sum_j U_j) / (M w), 0 when M = 0;
 *   pick = smallest flat parameter index reaching the maximum S, with
 *   flat = (iA * nB + iB) * nq + iq  (CMP: flat = iq).
 *
 * Conventions:
 *   - Every pointer is DEVICE memory unless marked [host].  The caller owns
 *     every buffer; the library never allocates or frees device memory and
 *     never synchronises: each call only enqueues work on `stream` and
 *     returns.  Results are valid once the stream has reached that point.
 *   - Arguments are validated on the host before anything is enqueued;
 *     invalid ones return SEMB_EINVAL, a too small workspace
 *     SEMB_EWORKSPACE, and a failed launch SEMB_EHIP.  semb_last_error()
 *     then holds a message (per thread).  Data-dependent conditions (T < 0,
 *     windows off the trace, M = 0, D = 0) are not errors: they have the
 *     results defined above.
 *   - Device contents are not inspected on the host.  The host-side bounds
 *     in semb_gathers (ns_max, nsamples) must hold for the device arrays;
 *     rows beyond ns_max are not computed, and the kernels never read
 *     outside [0, nsamples) or outside a trace.
 */
#ifndef SEMB_H
#define SEMB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SEMB_OK = 0,
    SEMB_EINVAL = 1,     /* invalid argument; nothing was enqueued            */
    SEMB_EWORKSPACE = 2, /* workspace missing or smaller than required        */
    SEMB_EHIP = 3        /* a HIP launch failed; see semb_last_error()        */
} semb_status;

enum { SEMB_KIND_CMP = 0, SEMB_KIND_CRS = 1 };

/* Seismic gathers (the CDP data structure of section 3.2, Fig. 5a): gather g
 * owns traces trace_ptr[g] .. trace_ptr[g+1]-1, stored consecutively from
 * element sample_off[g] of `samples`, each ns[g] samples long (sample n at
 * time n*dt).  The struct itself is [host]; its array pointers are device
 * pointers. */
typedef struct semb_gathers {
    const float *samples;     /* FP32 [nsamples]                                     */
    const int64_t *sample_off; /* [ngathers] first element of gather g              */
    const int32_t *trace_ptr; /* [ngathers + 1], trace_ptr[0] = 0                    */
    const int32_t *ns;        /* [ngathers] samples per trace of gather g, >= 1       */
    const float *half_offset; /* [ntraces] h, metres (the paper's "halfpoints")      */
    const float *midpoint;    /* [ntraces] midpoint coordinate, metres (CRS only;
                                 may be NULL for CMP calls)                          */
    const float *central_x;   /* [ngathers] coordinate of gather g's midpoint, metres
                                 (CRS only; may be NULL for CMP calls)               */
    int32_t ngathers;
    int32_t ntraces;
    int32_t ns_max;           /* [host] upper bound of ns[]; 1 .. SEMB_NS_LIMIT      */
    int64_t nsamples;         /* [host] number of elements of samples                */
    float dt;                 /* [host] sampling interval, seconds, > 0              */
} semb_gathers;

/* Scan jobs.  Job j stacks at gather central[j]; its traces are those of the
 * gathers apert_gather[apert_ptr[j] .. apert_ptr[j+1]-1] in that order (for a
 * CMP job just the central gather; apert_ptr/apert_gather may then be NULL).
 * Output row of (job j, sample s) is out_off[j] + s. */
typedef struct semb_jobs {
    const int32_t *central;      /* [njobs]                                           */
    const int32_t *apert_ptr;    /* [njobs + 1] or NULL (CMP)                          */
    const int32_t *apert_gather; /* [apert_ptr[njobs]] or NULL (CMP)                   */
    const int64_t *out_off;      /* [njobs]                                           */
    int32_t njobs;               /* [host] >= 0                                       */
    int32_t max_apert;           /* [host] upper bound of gathers per aperture
                                    (1 for CMP), 1 .. SEMB_APERT_LIMIT.  A CRS job
                                    whose aperture lists more gathers is not
                                    computed by any call: its rows get the marker
                                    best = -1, s_best = -1, stack = 0 (panel cells
                                    -1; stack and semb_refine: S = -1, stack = 0,
                                    theta kept; semblance_grad: zero gradient;
                                    corrected gathers: zeros).                         */
    int64_t n_out;               /* [host] number of output rows (>= every
                                    out_off[j] + ns[central[j]])                      */
} semb_jobs;

/* Outputs of a scan, one element per output row (panel: n_params per row,
 * row-major).  All are fully overwritten for the rows the jobs cover. */
typedef struct semb_outputs {
    int32_t *best;  /* [n_out] flat index of the picked parameter                  */
    float *s_best;  /* [n_out] its semblance                                        */
    float *stack;   /* [n_out] its stacked amplitude                                */
    float *panel;   /* [n_out * n_params] every semblance, or NULL                  */
    void *panel_f16; /* [n_out * n_params] the same in IEEE FP16 (round to nearest
                        even): half the bytes of the FP32 panel; or NULL          */
} semb_outputs;

#define SEMB_W_MAX 31          /* largest window; w must be odd, 1 .. SEMB_W_MAX */
#define SEMB_NS_LIMIT 2048     /* largest samples per trace (LDS stage capacity)  */
#define SEMB_APERT_LIMIT 64    /* largest number of gathers in one aperture        */

/* Workspace (device bytes) that cmp_scan / crs_scan need for gathers with
 * `nsamples` elements.  [host] */
size_t semb_workspace_bytes(int64_t nsamples);

/* CMP scan (section 2.1; grid search of section 3.2).  q[nq]: candidates
 * q = 4/v^2 in s^2/m^2.  w: window length in samples (odd).  ws: workspace of
 * at least semb_workspace_bytes(g->nsamples) bytes, 256-byte aligned; its
 * contents are scratch. */
semb_status cmp_scan(const semb_gathers *g, const semb_jobs *jobs, const float *q, int32_t nq,
                     int32_t w, const semb_outputs *out, void *ws, size_t ws_bytes,
                     hipStream_t stream);

/* 2D CRS scan (section 2.2 with the same grid search).  A[nA] in s/m, B[nB]
 * in s/m^2, q[nq] in s^2/m^2; n_params = nA * nB * nq, flat index
 * (iA * nB + iB) * nq + iq.  Requires g->midpoint and g->central_x. */
semb_status crs_scan(const semb_gathers *g, const semb_jobs *jobs, const float *A, int32_t nA,
                     const float *B, int32_t nB, const float *q, int32_t nq, int32_t w,
                     const semb_outputs *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* The scan for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * cmp_scan (kind SEMB_KIND_CMP; A, B ignored) or crs_scan (SEMB_KIND_CRS)
 * with the same arguments and the same outputs, bit for bit, but no
 * workspace.  The window-energy planes go to a scratch array of
 * SEMB_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * (until the process ends); the call allocates nothing and frees nothing.
 * The gathers must fit it: semb_workspace_bytes(g->nsamples) <=
 * SEMB_NOALLOC_SCRATCH_BYTES (about 5.5 million samples), else SEMB_EINVAL
 * before anything is enqueued.  All calls on one GPU share its scratch, which
 * keeps the last call's contents (nothing in it needs to start at zero):
 * calls that overlap on one GPU (two streams, two threads) race. */
#define SEMB_NOALLOC_SCRATCH_BYTES (64u << 20)
semb_status semb_scan_noalloc(int32_t kind, const semb_gathers *g, const semb_jobs *jobs, const float *A,
                              int32_t nA, const float *B, int32_t nB, const float *q, int32_t nq, int32_t w,
                              const semb_outputs *out, hipStream_t stream);

/* Semblance and stack of every output row at its own parameter theta[row] =
 * (A, B, q) (FP32 [n_out][3]; CMP ignores A and B).  s_out, stack_out:
 * [n_out], overwritten. */
semb_status stack(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, const float *theta,
                  int32_t w, float *s_out, float *stack_out, hipStream_t stream);

/* Gradient of L = sum_rows g_s[row] * S(row, theta[row]).  g_theta [n_out][3]
 * is overwritten with dL/dA, dL/dB, dL/dq (zero for CMP's A and B).
 * g_samples (nullable, [nsamples]) is ACCUMULATED into (+=), as autograd
 * accumulates gradients; the caller clears it.  With every contributing set
 * and window start held fixed (they are piecewise constant): dS/dv_ij =
 * 2 (U_j - S M v_ij) / (M D), dv_ij/dtau = f[a+j+1] - f[a+j],
 * dtau/dT = 1 / (2 dt sqrt T), dT/dA = 4 dm (t0 + 2 A dm), dT/dB = 2 t0 dm^2,
 * dT/dq = h^2, dv_ij/df[a+j] = 1 - x, dv_ij/df[a+j+1] = x.  Rows with
 * M = 0 or D = 0 and traces with T = 0 contribute nothing. */
semb_status semblance_grad(const semb_gathers *g, const semb_jobs *jobs, int32_t kind,
                           const float *theta, const float *g_s, int32_t w, float *g_theta,
                           float *g_samples, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Continuous refinement of coarse picks with the backward pass.
 * ------------------------------------------------------------------------- */
typedef struct semb_refine_opts {
    int32_t steps;    /* ascent steps, >= 0                                        */
    float eta0;       /* initial step length of every component in normalised
                         units (grid cells), >= 0                                  */
    float grow;       /* growth of a component's step while the sign of its
                         derivative repeats, >= 1 (e.g. 1.2)                       */
    float scale[3];   /* unit of the normalised coordinates per component (A, B, q),
                         e.g. the coarse grid spacing                              */
    float lo[3];      /* the parameters stay inside [lo, hi] per component         */
    float hi[3];
} semb_refine_opts;

/* Gradient-ascent refinement of each output row's parameter theta[row] =
 * (A, B, q) (FP32 [n_out][3], read and overwritten; CMP keeps A = B = 0).  In
 * coordinates u = theta / scale every component k takes its own step: u_k
 * moves eta_k in the direction of the sign of dS/du_k (dS/dtheta as in
 * semblance_grad), clamped to [lo, hi].  eta_k starts at eta0, grows by the
 * factor `grow` while the sign of its derivative repeats from the last
 * accepted step and halves when it flips.  A step is kept only if S
 * increases; otherwise every eta_k halves and the sign memory is cleared.
 * Writes the final S and stack to s_out, stack_out [n_out].  Rows are
 * independent; the whole loop runs on the device in one launch. */
semb_status semb_refine(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, float *theta,
                        const semb_refine_opts *o, int32_t w, float *s_out, float *stack_out,
                        hipStream_t stream);

/* theta[row] = (A[iA], B[iB], q[iq]) for the flat index best[row] =
 * (iA * nB + iB) * nq + iq (A, B may be NULL: 0 is written; indices outside
 * the grid are clamped).  Turns a scan's picks into refine's starting point
 * without a host round trip. */
semb_status semb_theta_from_best(const int32_t *best, int64_t n_out, const float *A, int32_t nA,
                                 const float *B, int32_t nB, const float *q, int32_t nq, float *theta,
                                 hipStream_t stream);

/* theta[row][k] = min(max(theta[row][k] + d[k], lo[k]), hi[k]) for n rows of
 * theta [n][3] (device FP32, in place); d, lo, hi: host [3].  Places further
 * starts of a multi-start refinement beside a coarse peak: the continuous
 * ascent that replaces section 3.2's fine grid climbs the maximum of its
 * start's basin, and a coarse grid can put a side lobe of the wavelet and
 * the main lobe in one cell.  SEMB_EINVAL if lo > hi or d is not finite. */
semb_status semb_theta_shift(float *theta, int64_t n, const float *d, const float *lo, const float *hi,
                             hipStream_t stream);

/* Gathers corrected along each output row's parameter theta[row] = (A, B, q)
 * (the NMO / CRS correction at the picks, for quality control): for job j,
 * aperture trace r (gathers as listed, traces in order) and output sample
 * s < ns[central[j]],
 *   out[corr_off[j] + r * ns[central[j]] + s] = f[k] + x (f[k+1] - f[k]),
 * the trace read at the intersection tau of row out_off[j] + s's traveltime
 * (k = floor(tau), x = tau - k; sections 2.1 / 2.2, Algorithm 1's
 * interpolation), and 0 where T < 0 or samples k and k+1 are not both on the
 * trace.  corr_off [njobs] (device int64) places each job's corrected traces;
 * out (FP32) must hold them all.  CMP ignores A and B. */
semb_status semb_corrected_gathers(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, const float *theta,
                                   const int64_t *corr_off, float *out, hipStream_t stream);

/* Starting points for a multi-start refinement: for each of n_rows rows of a
 * semblance panel (FP32 [n_rows][nA * nB * nq], as a scan writes it), the K
 * (1 .. 8) largest local maxima over the nA x nB x nq grid, best first (flat
 * index (iA * nB + iB) * nq + iq).  A cell is a local maximum when each of
 * its up to 26 neighbours is smaller, or equal with a larger flat index.  A
 * row with fewer than K maxima repeats its best.  best_k [K][n_rows] (int32)
 * and s_k [K][n_rows] (FP32), start-major, so that column k feeds
 * semb_theta_from_best directly. */
semb_status semb_panel_peaks(const float *panel, int64_t n_rows, int32_t nA, int32_t nB, int32_t nq, int32_t K,
                             int32_t *best_k, float *s_k, hipStream_t stream);

/* The best of K refined candidates per row: for each of n rows, the k with
 * the largest s_k[k][row] (the first on ties); writes its S, stack and theta
 * (theta_k [K][n][3]) to s_out, stack_out, theta_out [n][3]. */
semb_status semb_best_of(int32_t K, int64_t n, const float *s_k, const float *stack_k, const float *theta_k,
                         float *s_out, float *stack_out, float *theta_out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batched scan: CMP and CRS jobs of uneven fold and length in ONE persistent
 * launch (the paper processes CDPs as independent tasks, section 3.5; here
 * they are balanced across the GPU instead of across core groups).
 *
 * Work is cut into tiles = (job, block of 64 output samples, range of flat
 * parameter indices).  semb_batch_plan builds the tile list on the host,
 * longest first by estimated cost (samples x parameters x traces); tiles of
 * one (job, sample block) that split its parameter range form a group whose
 * partial picks the last-finishing tile merges.  scan_batch runs the list:
 * workgroups take tiles from an atomic counter until none is left.
 * ------------------------------------------------------------------------- */
typedef struct semb_tile {
    int32_t job;        /* job index                                             */
    int32_t sblk;       /* output samples 64*sblk .. 64*sblk+63 of the job       */
    int32_t p_begin;    /* flat parameter indices p_begin .. p_end-1             */
    int32_t p_end;
    int32_t group;      /* group id (tiles of one job/sample block), -1 if alone */
    int32_t split;      /* position within the group                             */
    int32_t nsplit;     /* tiles in the group (1 if alone)                       */
    int32_t part_base;  /* first partial slot of the group                       */
} semb_tile;

/* Host description of a batch, for planning.  [host] arrays. */
typedef struct semb_batch_host {
    int32_t njobs;
    const int32_t *kind;          /* [njobs] SEMB_KIND_CMP or SEMB_KIND_CRS          */
    const int32_t *central;       /* [njobs]                                         */
    const int32_t *apert_ptr;     /* [njobs + 1] aperture CSR (CMP jobs may list only
                                     the central gather; their aperture is ignored)  */
    const int32_t *apert_gather;
    int32_t ngathers;
    const int32_t *ns;            /* [ngathers]                                      */
    const int32_t *trace_ptr;     /* [ngathers + 1]                                  */
    int32_t npar_cmp;             /* parameters of a CMP job                         */
    int32_t npar_crs;             /* parameters of a CRS job                         */
} semb_batch_host;

/* Build the tile list (at most split_params parameters per tile, rounded up to
 * a multiple of 32).  tiles may be NULL to query the count.  On success
 * returns the number of tiles and sets *ngroups and *nparts (partial slots);
 * returns -1 (see semb_last_error) on invalid input or if max_tiles is too
 * small.  [host] */
int64_t semb_batch_plan(const semb_batch_host *h, int32_t split_params, semb_tile *tiles,
                        int64_t max_tiles, int32_t *ngroups, int32_t *nparts);

/* Device-side parameters of a batch. */
typedef struct semb_batch {
    const int32_t *kind;          /* [njobs] device                                  */
    const float *q_cmp;           /* CMP grid [nq_cmp]                               */
    int32_t nq_cmp;
    int32_t w_cmp;                /* CMP window: 9, 11 or 15                         */
    const float *A;               /* CRS grid, flat (iA * nB + iB) * nq_crs + iq     */
    int32_t nA;
    const float *B;
    int32_t nB;
    const float *q_crs;
    int32_t nq_crs;
    int32_t w_crs;                /* CRS window: 9, 11 or 15                         */
} semb_batch;

/* Workspace for scan_batch. [host] */
size_t semb_batch_workspace_bytes(int64_t nsamples, int32_t w_cmp, int32_t w_crs, int32_t ngroups,
                                  int32_t nparts);

/* Tile shapes of the batched scan: the CRS tile of the persistent kernel comes
 * in SEMB_BATCH_SHAPES shapes (windows behind a branch or branch-free, LDS
 * stage of 2048 or 2560 samples; CMP tiles are the same in every shape, and
 * every shape gives bit-identical outputs).  scan_batch uses the shape
 * recorded for its key (w_cmp, w_crs and the traces-per-job and
 * samples-per-trace buckets of semb_tune_scan), shape 0 without an entry.
 * The entry also holds the split_params the recorded plan was built with
 * (semb_batch_choice returns it, 256 without an entry), so that a caller can
 * plan with the tuned split.  The paper tunes its tile to the local store
 * (section 3.3.2); these are the batch kernel's counterpart. */
#define SEMB_BATCH_SHAPES 3

/* Human-readable description of a batch shape, NULL if out of range. [host] */
const char *semb_batch_shape_name(int32_t shape);

/* Record (shape, split_params) for the key of (w_cmp, w_crs, g, jobs); shape -1
 * removes the entry.  Reads only host fields. [host] */
semb_status semb_set_batch_choice(int32_t w_cmp, int32_t w_crs, const semb_gathers *g, const semb_jobs *jobs,
                                  int32_t shape, int32_t split_params);

/* The batch shape and split_params recorded for this key (defaults 0 and 256);
 * either output may be NULL. [host] */
void semb_batch_choice(int32_t w_cmp, int32_t w_crs, const semb_gathers *g, const semb_jobs *jobs, int32_t *shape,
                       int32_t *split_params);

/* Times every batch shape on a planned batch (arguments as for scan_batch; the
 * plan built with split_params), one warm-up and `reps` timed launches each,
 * compares each shape's best / s_best / stack over all n_out rows with shape
 * 0's, and records the fastest shape whose outputs are bit-identical,
 * together with split_params, for this key (another shape must beat shape 0
 * by 2%).  *shape receives it, ms[SEMB_BATCH_SHAPES] (nullable, host) each
 * shape's mean time in milliseconds, or -1 for a shape whose outputs differed.
 * The outputs are overwritten.  Synchronizes `stream`: not for graph capture. */
semb_status semb_tune_batch(const semb_gathers *g, const semb_jobs *jobs, const semb_batch *b, const semb_tile *tiles,
                            int64_t ntiles, int32_t ngroups, int32_t nparts, int32_t split_params, int32_t reps,
                            const semb_outputs *out, void *ws, size_t ws_bytes, int32_t *shape, float *ms,
                            hipStream_t stream);

/* Run a planned batch (tiles: device copy of the plan).  Outputs as for the
 * scans (panel must be NULL); best indexes the job's own grid.  The workspace
 * holds the window-energy planes, the tile and group counters (reset by a
 * kernel on `stream`, so the call can be captured in a HIP graph and
 * replayed) and the partial picks.  Calls that overlap on one workspace race.
 * ngroups and nparts must be the plan's; a device tile that no such plan
 * could hold (job, sample block, parameter range, group or partial slot out
 * of range) is skipped and leaves its rows unwritten. */
semb_status scan_batch(const semb_gathers *g, const semb_jobs *jobs, const semb_batch *b,
                       const semb_tile *tiles, int64_t ntiles, int32_t ngroups, int32_t nparts,
                       const semb_outputs *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Tile shapes of the exhaustive scan and their tuner.  cmp_scan and crs_scan
 * are built in SEMB_SCAN_SHAPES tile shapes (waves per workgroup, parameters
 * per lane, LDS stage size, windows behind a branch or branch-free; every
 * shape gives bit-identical results).  Which one a call uses is looked up
 * per (kind, w, traces per job, samples per trace), the two sizes rounded up
 * to powers of two from the host fields ntraces / ngathers (times max_apert
 * for CRS) and ns_max; without an entry the kind's default is used (shape 0
 * for CMP, 2 for CRS).  The table is process-wide and guarded by a mutex.
 * Tuned tile shapes are the counterpart of the paper's tuning of its tile and
 * prefetch sizes to the local store (section 3.3, Eq. (2)).
 * ------------------------------------------------------------------------- */
#define SEMB_SCAN_SHAPES 6

/* Human-readable description of a shape, NULL if out of range. [host] */
const char *semb_shape_name(int32_t shape);

/* Times every shape on the first min(sample_jobs, njobs) jobs (one warm-up
 * and `reps` timed calls each), compares each shape's best / s_best / stack
 * rows of those jobs with the default shape's, and records the fastest shape
 * whose rows are bit-identical for this call's key (another shape must beat
 * the default by 2%).  The sample is raised to at least 8 tiles (jobs times
 * ceil(ns_max / 64)) per compute unit when the workload has them: a sample
 * that does not fill the GPU several times is decided by tail effects; *shape receives it,
 * ms[SEMB_SCAN_SHAPES] (nullable, host) each shape's mean time per call in
 * milliseconds, or -1 for a shape whose outputs differed.  Arguments as for
 * cmp_scan (kind CMP; A, B ignored) or crs_scan; the sampled jobs' output
 * rows are overwritten.  Synchronizes `stream`: not for graph capture. */
semb_status semb_tune_scan(const semb_gathers *g, const semb_jobs *jobs, int32_t kind, const float *A,
                           int32_t nA, const float *B, int32_t nB, const float *q, int32_t nq, int32_t w,
                           int32_t sample_jobs, int32_t reps, const semb_outputs *out, void *ws,
                           size_t ws_bytes, int32_t *shape, float *ms, hipStream_t stream);

/* Record `shape` for the key of (kind, w, g, jobs); -1 removes the entry.
 * Reads only host fields of g and jobs. [host] */
semb_status semb_set_scan_shape(int32_t kind, int32_t w, const semb_gathers *g, const semb_jobs *jobs,
                                int32_t shape);

/* The shape a scan with these arguments uses (-1 for invalid arguments). [host] */
int32_t semb_scan_shape(int32_t kind, int32_t w, const semb_gathers *g, const semb_jobs *jobs);

/* Forget every recorded shape (exhaustive scans and batches). [host] */
void semb_clear_tuning(void);

/* The tuning table on disk, so that tuned choices outlive the process.  Text,
 * one entry per line: "scan <kind> <w> <traces bucket> <ns bucket> <shape>"
 * and "batch <w_cmp> <w_crs> <traces bucket> <ns bucket> <shape>
 * <split_params>" ('#' lines are comments).  semb_tuning_save writes every
 * recorded entry; semb_tuning_load merges a file's entries into the table
 * (an entry replaces the one with its key) only if every line is valid.
 * Both return the number of entries, or -1 (semb_last_error) if the file
 * cannot be opened or holds a line that is not an entry. [host] */
int32_t semb_tuning_save(const char *path);
int32_t semb_tuning_load(const char *path);

/* CRS apertures by radius: for every central gather, the gathers whose
 * midpoint (x, y) lies within `radius` of the central's (the paper's
 * neighbourhood of a central CDP, section 2.2, Fig. 2b), central included, in
 * increasing gather index.  x, y: [ngathers] midpoint coordinates in m (y may
 * be NULL for a line); centrals: [ncentrals]; all host memory.  Fills
 * apert_ptr[ncentrals + 1] and, when apert_gather is non-NULL, apert_gather
 * [apert_ptr[ncentrals]] (call once with NULL to size it); *max_apert
 * (nullable) receives the longest list, which crs_scan accepts up to
 * SEMB_APERT_LIMIT.  Returns the number of entries, -1 on invalid input
 * (semb_last_error).  A uniform grid hash with cells of the radius's size
 * keeps each query to 3 x 3 cells.  The CRS operator of crs_scan is the 2D
 * one (section 2.2): its dm is the difference of the single coordinates in
 * semb_gathers.midpoint and .central_x.  With y given, the apertures are 2D
 * but the traveltime still sees only that coordinate: the caller chooses it
 * (e.g. the inline position), and the crossline distance enters nothing.  [host] */
int64_t semb_radius_apertures(const double *x, const double *y, int32_t ngathers, const int32_t *centrals,
                              int32_t ncentrals, double radius, int32_t *apert_ptr, int32_t *apert_gather,
                              int32_t *max_apert);

/* Kernel timing for measurement.  After semb_kernel_timer_start(capacity),
 * the next `capacity` launches of a call's main kernel made by this thread
 * (the scan kernel of cmp_scan / crs_scan, the persistent kernel of
 * scan_batch, the kernels of stack, semblance_grad and semb_refine; not the
 * window-energy pre-pass) are bracketed by a pair of HIP events recorded on
 * the call's stream.  Launches on a stream that is being captured into a
 * graph are not timed.  semb_kernel_timer_stop waits for the recorded
 * events, writes the number of timed launches to *count and the first
 * min(count, ms_len) durations in milliseconds to ms, then releases the
 * events.  The events belong to the device current at start.  [host] */
semb_status semb_kernel_timer_start(int32_t capacity);
semb_status semb_kernel_timer_stop(int32_t *count, float *ms, int32_t ms_len);

/* Microbenchmarks: the ceilings the scan kernels are measured against, taken
 * on the device current for the calling thread (the roofline analysis of
 * section 4.3 divides by such peaks).  Each probe launches 8 workgroups per
 * CU of independent work (a warm-up launch, then `reps` timed launches, HIP
 * events on a stream of its own) and writes *rate (work per second) and *ms
 * (mean milliseconds per launch):
 *   SEMB_PROBE_FMA_F32  plain FP32 FMAs (packed FP32 is not used): flops/s,
 *                       2 per FMA lane
 *   SEMB_PROBE_FMA_F64  FP64 FMAs: flops/s, 2 per FMA lane
 *   SEMB_PROBE_RSQ_F64  v_rsq_f64, the start of every traveltime: lane
 *                       results per second
 *   SEMB_PROBE_LDS_READ 16-byte LDS reads without bank conflicts: bytes/s
 *   SEMB_PROBE_LDS_READ2 paired 4-byte LDS reads (ds_read2_b32) of 16
 *                       consecutive words per lane, neighbouring lanes one
 *                       word apart, as a scan window reads them: bytes/s
 * Allocates and frees a small device buffer; synchronizes its own stream.
 * SEMB_EINVAL for an unknown probe or reps outside 1..100.  [host] */
#define SEMB_PROBE_FMA_F32 0
#define SEMB_PROBE_FMA_F64 1
#define SEMB_PROBE_RSQ_F64 2
#define SEMB_PROBE_LDS_READ 3
#define SEMB_PROBE_LDS_READ2 4
semb_status semb_probe(int32_t probe, int32_t reps, double *rate, double *ms);

/* Message describing the last non-OK status returned on this thread. [host] */
const char *semb_last_error(void);

/* Library version string. [host] */
const char *semb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SEMB_H */
