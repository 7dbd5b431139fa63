// internal.h -- declarations shared by the host API and the kernel
// translation units of the semblance library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "semb.h"

namespace semb {

// The gathers as the kernels see them.
struct GatherView {
    const float *samples;
    const int64_t *sample_off;
    const int32_t *trace_ptr;
    const int32_t *ns;
    const float *half_offset;
    const float *midpoint;
    const float *central_x;
    float dt;
};

// Jobs: central gather, aperture (CSR; NULL = the central gather alone) and
// output row offset; n_sblk = output-sample blocks per job (ceil(ns_max/64)).
struct JobView {
    const int32_t *central;
    const int32_t *apert_ptr;
    const int32_t *apert_gather;
    const int64_t *out_off;
    int32_t njobs;
    int32_t n_sblk;
    int32_t max_apert;  // the caller's bound on gathers per aperture (<= SEMB_APERT_LIMIT)
};

// Does job `job`'s aperture list more gathers than the caller declared?  Such a
// job is not computed by any kernel; its rows get the marker the ABI documents
// (scan: best = -1, s_best = -1, stack = 0; point evaluation: S = -1).
__device__ __forceinline__ bool apert_over(const int32_t *apert_ptr, int32_t max_apert, int job)
{
    return apert_ptr != nullptr && apert_ptr[job + 1] - apert_ptr[job] > max_apert;
}

// One parameter grid (flat index (iA * nB + iB) * nq + iq) with the window
// and the window-energy planes for that window (workspace, one per sample).
struct ParamView {
    const float *A;
    const float *B;
    const float *q;
    int32_t nA, nB, nq, npar;
    int32_t w;
    const float *u0;
    const float *u1;
    const float *u2sq;
};

struct ScanArgs {
    GatherView g;
    JobView j;
    ParamView p;
    int32_t *best;
    float *s_best;
    float *stack;
    float *panel;
    void *panel16;
};

// One partial pick of a split tile: best S, its flat index, its stack.
struct Partial {
    float S;
    int32_t I;
    float stack;
    float pad;
};

struct BatchArgs {
    GatherView g;
    JobView j;
    const int32_t *kind;      // [njobs]
    ParamView pc;             // CMP jobs
    ParamView pr;             // CRS jobs
    const semb_tile *tiles;   // [ntiles], processed in this order
    int64_t ntiles;
    unsigned int *counters;   // [1 + ngroups]: tile counter, then finished splits per group
    Partial *partials;        // [nparts * 64]
    int32_t ngroups, nparts;  // the plan's sizes; a tile outside them is skipped
    int32_t *best;
    float *s_best;
    float *stack;
};

struct PointArgs {
    const float *samples;
    const int64_t *sample_off;
    const int32_t *trace_ptr;
    const int32_t *ns;
    const float *half_offset;
    const float *midpoint;
    const float *central_x;
    float dt;
    const int32_t *central;
    const int32_t *apert_ptr;
    const int32_t *apert_gather;
    const int64_t *out_off;
    int32_t njobs;
    int32_t n_sblk;
    int32_t max_apert;
    const float *theta;   // [n_out][3]
    const float *g_s;     // [n_out] (gradient only)
    float *s_out;
    float *stack_out;
    float *g_theta;       // [n_out][3]
    float *g_samples;     // nullable
    int32_t w;
};

// Options of the gradient-ascent refinement (see semb_refine).
struct RefineArgs {
    float *theta;  // [n_out][3], read and overwritten
    int32_t steps;
    float eta0;
    float grow;
    float scale[3];
    float lo[3];
    float hi[3];
};

// Records the message semb_last_error() returns on this thread.
void set_last_error(const char *msg);

// Launchers (return the hipError_t of the launch).
hipError_t launch_window_energy(const float *samples, const int64_t *sample_off,
                                const int32_t *trace_ptr, const int32_t *ns, int32_t ngathers,
                                int32_t ntraces, int32_t w, float *u0, float *u1, float *u2sq,
                                hipStream_t stream);
// Exhaustive scan in tile shape `shape` (0 .. kScanShapes - 1).
constexpr int kScanShapes = 6;
hipError_t launch_scan(int kind, const ScanArgs &a, int shape, hipStream_t stream);
hipError_t launch_scan_cmp(const ScanArgs &a, int shape, hipStream_t stream);
hipError_t launch_scan_crs(const ScanArgs &a, int shape, hipStream_t stream);
// Batched scan in batch tile shape `shape` (0 .. kBatchShapes - 1).
constexpr int kBatchShapes = 3;
hipError_t launch_batch(const BatchArgs &a, int ngroups, int shape, hipStream_t stream);
hipError_t launch_point(int kind, const PointArgs &a, hipStream_t stream);
hipError_t launch_grad(int kind, const PointArgs &a, hipStream_t stream);
hipError_t launch_refine(int kind, const PointArgs &a, const RefineArgs &o, hipStream_t stream);
hipError_t launch_corrected(int kind, const PointArgs &a, const int64_t *corr_off, float *out, hipStream_t stream);
hipError_t launch_panel_peaks(const float *panel, int64_t n_rows, int nA, int nB, int nq, int K, int32_t *best_k,
                              float *s_k, hipStream_t stream);
hipError_t launch_best_of(int K, int64_t n, const float *s_k, const float *stack_k, const float *theta_k,
                          float *s_out, float *stack_out, float *theta_out, hipStream_t stream);
hipError_t launch_theta_from_best(const int32_t *best, int64_t n, const float *A, int nA, const float *B, int nB,
                                  const float *q, int nq, float *theta, hipStream_t stream);

}  // namespace semb
