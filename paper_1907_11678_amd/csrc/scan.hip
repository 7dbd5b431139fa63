// scan.hip -- gfx950 kernels around the scan tile: the window-energy pass that
// every scan call starts with, and the batched persistent scan of mixed
// CMP / CRS jobs.  The exhaustive scan kernels are built in scan_cmp.hip and
// scan_crs.hip; the tile they share, and its mapping onto CDNA4, is in tile.h.

#include "tile.h"

namespace semb {
namespace {

// ---------------------------------------------------------------------------
// Window energy in Gram form.  For window start n of a trace (n + w <= ns-1)
// let a_j = f[n+j], b_j = f[n+j+1] - f[n+j] (j < w); the interpolated window
// energy sum_j (a_j + x b_j)^2 = aa + 2 x ab + x^2 bb equals
//   (u0 + u1 x)^2 + u2sq,  u1 = sqrt(bb), u0 = ab / u1, u2sq = aa - ab^2 / bb
// (u1 = u0 = 0, u2sq = aa when bb = 0).  The sums are formed in FP64, where
// products of FP32 samples are exact; 1/sqrt(bb) comes from the hardware
// reciprocal square root plus one Newton step (relative error ~1e-15), so
// u0, u1 and u2sq are the FP32 roundings of their exact values up to a few
// units in the last place of FP64.  One block per trace: the trace is staged
// in LDS 2048 positions at a time (coalesced loads), each thread then forms
// the sums of its positions from LDS, and the three planes are written
// coalesced.
// ---------------------------------------------------------------------------
constexpr int ENERGY_PIECE = 2048;

template <int W>
__global__ void __launch_bounds__(256)
window_energy_kernel(const float *__restrict__ samples, const int64_t *__restrict__ sample_off,
                     const int32_t *__restrict__ trace_ptr, const int32_t *__restrict__ ns,
                     int ngathers, float *__restrict__ u0, float *__restrict__ u1, float *__restrict__ u2sq)
{
    __shared__ float sf[ENERGY_PIECE + 32];
    const int t = blockIdx.x;
    int lo = 0, hi = ngathers;  // largest g with trace_ptr[g] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (trace_ptr[mid] <= t) lo = mid; else hi = mid;
    }
    const int n = ns[lo];
    const int64_t base = sample_off[lo] + (int64_t)(t - trace_ptr[lo]) * n;
    for (int p0 = 0; p0 < n; p0 += ENERGY_PIECE) {
        const int nload = min(n - p0, ENERGY_PIECE + W + 1);  // <= ENERGY_PIECE + 32
        __syncthreads();  // the previous piece is done with sf
        for (int i = threadIdx.x; i < nload; i += blockDim.x) sf[i] = samples[base + p0 + i];
        __syncthreads();
        const int pend = min(n, p0 + ENERGY_PIECE);
        for (int p = p0 + (int)threadIdx.x; p < pend; p += blockDim.x) {
            float r0 = 0.f, r1 = 0.f, r2 = 0.f;
            if (p + W <= n - 1) {  // then all W + 1 samples are staged
                const float *f = sf + (p - p0);
                double aa = 0.0, ab = 0.0, bb = 0.0;
                double prev = f[0];
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    const double nxt = f[j + 1];
                    const double d = nxt - prev;  // exact: both are FP32 values
                    aa = fma(prev, prev, aa);
                    ab = fma(prev, d, ab);
                    bb = fma(d, d, bb);
                    prev = nxt;
                }
                if (bb > 0.0) {
                    double y = __builtin_amdgcn_rsq(bb);
                    y = fma(fma(-bb * y, y, 1.0), 0.5 * y, y);  // one Newton step
                    const double c0 = ab * y;
                    r1 = (float)(bb * y);
                    r0 = (float)c0;
                    r2 = (float)fmax(fma(-c0, c0, aa), 0.0);
                } else {
                    r2 = (float)aa;
                }
            }
            u0[base + p] = r0;
            u1[base + p] = r1;
            u2sq[base + p] = r2;
        }
    }
}

template <int W>
hipError_t launch_energy_w(const float *samples, const int64_t *sample_off, const int32_t *trace_ptr,
                           const int32_t *ns, int32_t ngathers, int32_t ntraces, float *u0, float *u1,
                           float *u2sq, hipStream_t stream)
{
    hipLaunchKernelGGL((window_energy_kernel<W>), dim3((unsigned)ntraces), dim3(256), 0, stream, samples,
                       sample_off, trace_ptr, ns, ngathers, u0, u1, u2sq);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The batched scan: a persistent grid takes tiles of a mixed CMP/CRS job list
// from an atomic counter (longest tiles first, as planned on the host).  A
// tile that covers all parameters of its (job, sample block) writes the
// outputs; otherwise it stores a partial pick, and the last tile of its group
// to finish (counted with an atomic, after a release fence) merges the
// group's partials in split order.  Both kinds use 8 waves; CMP tiles give
// each wave 2 parameters, CRS tiles 4 for windows up to 9 samples (each
// trace's loop work is then shared by 4 parameters) and 2 for longer ones,
// whose 4 x (w + 2) accumulators would not fit the 128-VGPR budget of 4
// waves per SIMD.  The CRS tile comes in the batch shapes below (BatchShape);
// CMP tiles are the same in every shape.  The LDS union of the two kinds'
// layouts keeps two workgroups per CU.
//   0: CRS windows behind a branch, 2048-sample stage;
//   1: CRS windows branch-free, 2560-sample stage (the exhaustive CRS
//      scan's default tile);
//   2: CRS windows branch-free, 2048-sample stage.
// Every shape sums each cell's traces in the same order (bit-identical).
// ---------------------------------------------------------------------------
constexpr int BATCH_NW = 8;
constexpr int BATCH_P_CMP = 2;
constexpr int batch_p_crs(int wr) { return wr <= 9 ? 4 : 2; }
constexpr int BATCH_CAP = 2048;
constexpr int BATCH_TMAX = 128;

template <int BS>
struct BatchShape;
template <>
struct BatchShape<0> {
    static constexpr int CAP_CRS = 2048;
    static constexpr bool BRANCHY_CRS = true;
};
template <>
struct BatchShape<1> {
    static constexpr int CAP_CRS = 2560;
    static constexpr bool BRANCHY_CRS = false;
};
template <>
struct BatchShape<2> {
    static constexpr int CAP_CRS = 2048;
    static constexpr bool BRANCHY_CRS = false;
};

__global__ void reset_counters_kernel(unsigned int *c, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0u;
}

template <int WC, int WR, int BS>
__global__ void __launch_bounds__(BATCH_NW * WAVE) __attribute__((amdgpu_waves_per_eu(4)))
batch_kernel(BatchArgs b)
{
    constexpr int CAP_R = BatchShape<BS>::CAP_CRS;
    using LC = StageLds<SEMB_KIND_CMP, WC, BATCH_P_CMP, BATCH_NW, BATCH_CAP, BATCH_TMAX>;
    using LR = StageLds<SEMB_KIND_CRS, WR, batch_p_crs(WR), BATCH_NW, CAP_R, BATCH_TMAX>;
    __shared__ union U {
        LC c;
        LR r;
    } L;
    __shared__ long long sh_tile;
    __shared__ int sh_last;
    const int lane = threadIdx.x & (WAVE - 1);

    for (;;) {
        __syncthreads();  // everyone has read the previous tile index
        if (threadIdx.x == 0) sh_tile = (long long)atomicAdd(&b.counters[0], 1u);
        __syncthreads();
        const long long t = sh_tile;
        if (t >= b.ntiles) break;  // uniform: every workgroup leaves once the list is drained
        const semb_tile tl = b.tiles[t];
        // A tile that no plan of these jobs and sizes could contain is skipped
        // (its rows stay unwritten) rather than read or write out of bounds.
        if (tl.job < 0 || tl.job >= b.j.njobs || tl.sblk < 0 || tl.sblk >= b.j.n_sblk) continue;
        const int kind = b.kind[tl.job];
        if (kind != SEMB_KIND_CMP && kind != SEMB_KIND_CRS) continue;
        if (tl.p_begin < 0 || tl.p_begin >= tl.p_end || tl.p_end > (kind == SEMB_KIND_CMP ? b.pc.npar : b.pr.npar))
            continue;
        if (tl.nsplit > 1 && (tl.group < 0 || tl.group >= b.ngroups || tl.split < 0 || tl.split >= tl.nsplit ||
                              tl.part_base < 0 || (int64_t)tl.part_base + tl.nsplit > b.nparts))
            continue;
        if (kind == SEMB_KIND_CRS && apert_over(b.j.apert_ptr, b.j.max_apert, tl.job)) {
            // every split of the group writes the same marker rows
            write_apert_marker(b.j, tl.job, tl.sblk, b.g.ns[b.j.central[tl.job]], b.pr.npar, b.best, b.s_best,
                               b.stack, nullptr, nullptr);
            continue;
        }
        float bS, bSt;
        int bI;
        if (kind == SEMB_KIND_CMP)
            scan_tile<SEMB_KIND_CMP, WC, BATCH_P_CMP, BATCH_NW, BATCH_CAP, BATCH_TMAX, true>(
                b.g, b.j, b.pc, L.c, tl.job, tl.sblk, tl.p_begin, tl.p_end, nullptr, nullptr, bS, bI, bSt);
        else
            scan_tile<SEMB_KIND_CRS, WR, batch_p_crs(WR), BATCH_NW, CAP_R, BATCH_TMAX, BatchShape<BS>::BRANCHY_CRS>(
                b.g, b.j, b.pr, L.r, tl.job, tl.sblk, tl.p_begin, tl.p_end, nullptr, nullptr, bS, bI, bSt);
        const int64_t row = b.j.out_off[tl.job] + tl.sblk * WAVE + lane;
        if (tl.nsplit <= 1) {
            if (threadIdx.x < WAVE && bS >= 0.f) {
                b.best[row] = bI;
                b.s_best[row] = bS;
                b.stack[row] = bSt;
            }
            continue;
        }
        Partial *part = b.partials + (int64_t)tl.part_base * WAVE;
        if (threadIdx.x < WAVE) {
            Partial pt;
            pt.S = bS;
            pt.I = bI;
            pt.stack = bSt;
            pt.pad = 0.f;
            part[(int64_t)tl.split * WAVE + lane] = pt;
            __threadfence();  // release the partial before counting this split done
        }
        __syncthreads();
        if (threadIdx.x == 0) sh_last = (atomicAdd(&b.counters[1 + tl.group], 1u) == (unsigned)(tl.nsplit - 1));
        __syncthreads();
        if (sh_last && threadIdx.x < WAVE) {
            __threadfence();  // acquire the other splits' partials
            float mS = -2.f, mT = 0.f;
            int mI = 0;
            for (int sp = 0; sp < tl.nsplit; ++sp) {
                const Partial q = part[(int64_t)sp * WAVE + lane];
                if (q.S > mS) {  // splits cover increasing index ranges: first max wins
                    mS = q.S;
                    mI = q.I;
                    mT = q.stack;
                }
            }
            if (mS >= 0.f) {
                b.best[row] = mI;
                b.s_best[row] = mS;
                b.stack[row] = mT;
            }
        }
    }
}

template <int WC, int WR, int BS>
int batch_blocks_per_cu()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<WC, WR, BS>, BATCH_NW * WAVE, 0) !=
        hipSuccess)
        n = 1;
    return n < 1 ? 1 : n;
}

// The persistent grid: as many workgroups as fit on the GPU at once (never
// more than there are tiles).
template <int WC, int WR, int BS>
hipError_t launch_batch_k(const BatchArgs &a, int cus, hipStream_t stream)
{
    const long long want = (long long)cus * batch_blocks_per_cu<WC, WR, BS>();
    const dim3 grid((unsigned)(want < a.ntiles ? want : a.ntiles));
    hipLaunchKernelGGL((batch_kernel<WC, WR, BS>), grid, dim3(BATCH_NW * WAVE), 0, stream, a);
    return hipGetLastError();
}

template <int WC, int WR>
hipError_t launch_batch_s(const BatchArgs &a, int shape, int cus, hipStream_t stream)
{
    switch (shape) {
    case 0: return launch_batch_k<WC, WR, 0>(a, cus, stream);
    case 1: return launch_batch_k<WC, WR, 1>(a, cus, stream);
    case 2: return launch_batch_k<WC, WR, 2>(a, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int WC>
hipError_t launch_batch_wc(const BatchArgs &a, int shape, int cus, hipStream_t stream)
{
    switch (a.pr.w) {
    case 9: return launch_batch_s<WC, 9>(a, shape, cus, stream);
    case 11: return launch_batch_s<WC, 11>(a, shape, cus, stream);
    case 15: return launch_batch_s<WC, 15>(a, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_window_energy(const float *samples, const int64_t *sample_off,
                                const int32_t *trace_ptr, const int32_t *ns, int32_t ngathers,
                                int32_t ntraces, int32_t w, float *u0, float *u1, float *u2sq,
                                hipStream_t stream)
{
    if (ntraces <= 0) return hipSuccess;
#define SEMB_ENERGY(WW) \
    case WW: return launch_energy_w<WW>(samples, sample_off, trace_ptr, ns, ngathers, ntraces, u0, u1, u2sq, stream);
    switch (w) {
        SEMB_ENERGY(1) SEMB_ENERGY(3) SEMB_ENERGY(5) SEMB_ENERGY(7) SEMB_ENERGY(9) SEMB_ENERGY(11)
        SEMB_ENERGY(13) SEMB_ENERGY(15) SEMB_ENERGY(17) SEMB_ENERGY(19) SEMB_ENERGY(21) SEMB_ENERGY(23)
        SEMB_ENERGY(25) SEMB_ENERGY(27) SEMB_ENERGY(29) SEMB_ENERGY(31)
    default: return hipErrorInvalidValue;
    }
#undef SEMB_ENERGY
}

hipError_t launch_scan(int kind, const ScanArgs &a, int shape, hipStream_t stream)
{
    return kind == SEMB_KIND_CMP ? launch_scan_cmp(a, shape, stream) : launch_scan_crs(a, shape, stream);
}

hipError_t launch_batch(const BatchArgs &a, int ngroups, int shape, hipStream_t stream)
{
    const int ncount = 1 + ngroups;
    hipLaunchKernelGGL(reset_counters_kernel, dim3((ncount + 255) / 256 < 1024 ? (ncount + 255) / 256 : 1024),
                       dim3(256), 0, stream, a.counters, ncount);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.ntiles == 0) return e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    switch (a.pc.w) {
    case 9: return launch_batch_wc<9>(a, shape, cus, stream);
    case 11: return launch_batch_wc<11>(a, shape, cus, stream);
    case 15: return launch_batch_wc<15>(a, shape, cus, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace semb
