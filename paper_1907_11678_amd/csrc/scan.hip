// scan.hip -- gfx950 kernels of the exhaustive CMP / 2D-CRS semblance scan.
//
// What is computed (Hu, Yang, Luan, Qian, "Massively Scaling Seismic
// Processing on Sunway TaihuLight Supercomputer"): the grid search of
// section 3.2 -- for every output sample t0 of a job and every candidate
// parameter, the semblance of Eq. (1) over a w-sample window centred on each
// trace's intersection with the traveltime curve (CMP, section 2.1) or
// surface (CRS, section 2.2), each window sample linearly interpolated with
// the intersection's fraction x (Algorithm 1); then the most coherent
// parameter per sample and the stack along it.
//
// How it maps to CDNA4 (the paper's Sunway design is prior art, not copied):
//   * one workgroup = (job, block of 64 consecutive output samples); lane l
//     of every wave owns output sample s0 + l, and wave v owns P parameters of
//     each parameter block.  All lanes of a wave therefore share the
//     parameter and the trace, so the per-(parameter, trace) terms are
//     wave-uniform, and neighbouring lanes read neighbouring (or equal) LDS
//     words -- no bank conflicts;
//   * like the re-designed procedure of section 3.3.2 (Algorithm 2), traces
//     are the outer loop and the per-pair sums U[w], D, M live in registers
//     across all traces; for a chunk of traces the union [lo, hi] of the
//     sample ranges the tile can touch (the paper's min_la..max_lb) is staged
//     once into LDS with coalesced loads, which is also the paper's tiling of
//     the merged intersections to fit local memory;
//   * the window energy D_i = sum_j v_ij^2 is not accumulated sample by
//     sample.  With the shared fraction x, v_ij = f[a+j] + x (f[a+j+1] -
//     f[a+j]), so D_i is a quadratic in x whose coefficients depend only on
//     the window start; window_energy_kernel writes it once per sample as a
//     sum of two squares, D_i = (u0 + u1 x)^2 + u2^2 (Gram form of the two
//     window vectors, computed in FP64), whose terms are never negative and so
//     never cancel.  U_j costs two FMAs per window sample, so a window costs
//     2w + 3 VALU operations and w + 4 LDS words;
//   * the intersection is computed in FP64 (traveltime.h), so the set of
//     contributing traces and the fraction x are those of an exact
//     evaluation;
//   * the blockIdx -> tile map keeps consecutive tiles (one job) on one XCD so
//     that the job's traces stay in that XCD's L2.
//
// Readings where the paper is silent are stated with the ABI in semb.h.

#include "internal.h"
#include "traveltime.h"

namespace semb {
namespace {

constexpr int WAVE = 64;

typedef __attribute__((address_space(3))) void lds_void;

// One dword per lane from global memory straight into LDS: lane l writes LDS
// word (lds_base + l); lds_base must be the same for the whole wave.
__device__ __forceinline__ void lds_dma(const float *g, float *lds_base)
{
    __builtin_amdgcn_global_load_lds((void *)g, (lds_void *)lds_base, 4, 0, 0);
}

// A wave-uniform double moved into scalar registers (frees two VGPRs).
__device__ __forceinline__ double to_sgpr(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// The dispatcher deals workgroups round-robin over the 8 XCDs.  Map the k-th
// workgroup of XCD x to a contiguous range of tiles so that the tiles of one
// job share an L2.  A bijection of [0, nblk).
__device__ __forceinline__ int xcd_tile(int bid, int nblk)
{
    const int per = nblk >> 3, rem = nblk & 7;
    const int x = bid & 7, local = bid >> 3;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + local;
}

// ---------------------------------------------------------------------------
// Window energy in Gram form.  For window start n of a trace (n + w <= ns-1)
// let a_j = f[n+j], b_j = f[n+j+1] - f[n+j] (j < w); the interpolated window
// energy sum_j (a_j + x b_j)^2 = aa + 2 x ab + x^2 bb equals
//   (u0 + u1 x)^2 + u2sq,  u1 = sqrt(bb), u0 = ab / u1, u2sq = aa - ab^2 / bb
// (u1 = u0 = 0, u2sq = aa when bb = 0).  The sums are formed in FP64, where
// products of FP32 samples are exact.  One block per trace.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
window_energy_kernel(const float *__restrict__ samples, const int64_t *__restrict__ sample_off,
                     const int32_t *__restrict__ trace_ptr, const int32_t *__restrict__ ns,
                     int ngathers, int w, float *__restrict__ u0, float *__restrict__ u1,
                     float *__restrict__ u2sq)
{
    const int t = blockIdx.x;
    int lo = 0, hi = ngathers;  // largest g with trace_ptr[g] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (trace_ptr[mid] <= t) lo = mid; else hi = mid;
    }
    const int n = ns[lo];
    const int64_t base = sample_off[lo] + (int64_t)(t - trace_ptr[lo]) * n;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
        if (p + w <= n - 1) {
            const float *f = samples + base + p;
            double aa = 0.0, ab = 0.0, bb = 0.0;
            double prev = f[0];
            for (int j = 0; j < w; ++j) {
                const double nxt = f[j + 1];
                const double d = nxt - prev;  // exact: both are FP32 values
                aa = fma(prev, prev, aa);
                ab = fma(prev, d, ab);
                bb = fma(d, d, bb);
                prev = nxt;
            }
            if (bb > 0.0) {
                const double s1 = sqrt(bb);
                r1 = (float)s1;
                r0 = (float)(ab / s1);
                r2 = (float)fmax(aa - ab * ab / bb, 0.0);
            } else {
                r2 = (float)aa;
            }
        }
        u0[base + p] = r0;
        u1[base + p] = r1;
        u2sq[base + p] = r2;
    }
}

// ---------------------------------------------------------------------------
// The scan.  KIND: SEMB_KIND_CMP / SEMB_KIND_CRS.  W: window.  P: parameters
// per lane.  NW: waves per workgroup.  CAP: LDS sample positions per stage.
// ---------------------------------------------------------------------------
// WPE: minimum waves per SIMD the register allocation must allow.
template <int KIND, int W, int P, int NW, int CAP, int WPE>
__global__ void __launch_bounds__(NW * WAVE) __attribute__((amdgpu_waves_per_eu(WPE)))
scan_kernel(ScanArgs a)
{
    constexpr int HW = (W - 1) / 2;
    constexpr int NT = NW * P;  // parameters per block
    constexpr int RMAX = WAVE;  // traces per stage (one per lane of wave 0)
    constexpr bool CRS = KIND == SEMB_KIND_CRS;

    __shared__ float lf[CAP];                    // staged samples
    __shared__ float lu0[CAP], lu1[CAP], lu2[CAP];  // their window energy (Gram form)
    __shared__ double2 tab[CRS ? NT : 1][RMAX];  // CRS: (2 alpha + beta, alpha^2 + gamma)
    __shared__ double t_cc[RMAX];                // h^2/dt^2 per staged trace
    __shared__ int2 tinfo[RMAX];                 // (base - lo, ns - 1 - W)
    __shared__ long long t_src[RMAX];            // element of the first staged sample
    __shared__ int t_len[RMAX], t_base[RMAX];
    __shared__ float t_dm[RMAX];
    __shared__ double pq[NT], pA[NT], pB[NT];    // this block's parameters
    __shared__ int ag_s[SEMB_APERT_LIMIT];
    __shared__ int ag_cum[SEMB_APERT_LIMIT + 1];
    __shared__ int sh_nfit;

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);

    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int job = tile / a.n_sblk;
    const int sblk = tile - job * a.n_sblk;
    if (job >= a.njobs) return;
    const int c = a.central[job];
    const int nsc = a.ns[c];
    const int s0 = sblk * WAVE;
    if (s0 >= nsc) return;  // uniform over the workgroup, before any barrier
    const int s1 = min(s0 + WAVE, nsc) - 1;
    const int s = s0 + lane;
    const bool lane_on = s < nsc;

    // ---- the job's aperture: gathers and cumulative trace counts ----------
    int na = 1, afirst = -1;
    if (CRS && a.apert_ptr != nullptr) {
        afirst = a.apert_ptr[job];
        na = min(a.apert_ptr[job + 1] - afirst, SEMB_APERT_LIMIT);
        na = max(na, 0);
    }
    if (tid < na) ag_s[tid] = (afirst < 0) ? c : a.apert_gather[afirst + tid];
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        ag_cum[0] = 0;
        for (int k = 0; k < na; ++k) {
            const int g = ag_s[k];
            acc += a.trace_ptr[g + 1] - a.trace_ptr[g];
            ag_cum[k + 1] = acc;
        }
    }
    __syncthreads();
    const int ntr = ag_cum[na];
    const double xc = CRS ? (double)a.central_x[c] : 0.0;
    const double inv_dt = 1.0 / (double)a.dt;

    const double sd = (double)s;
    const double s2 = sd * sd;

    float bS = -1.f, bSt = 0.f;
    int bI = 0;

    for (int pb = 0; pb < a.npar; pb += NT) {
        const int pe = min(pb + NT, a.npar);
        // bounds of this block's parameters (wave-uniform)
        // ---- this block's parameters, decoded once by wave 0 (one per lane) into
        // LDS, with their bounds reduced across the wave.  The previous block
        // ended with a barrier, so the parameter arrays are free.
        double qlo = 0.0, qhi = 0.0, Alo = 0.0, Ahi = 0.0, Blo = 0.0, Bhi = 0.0;
        if (wv == 0) {
            const int th = pb + lane;
            const bool on = lane < NT && th < a.npar;
            double qv = 0.0, Av = 0.0, Bv = 0.0;
            if (on) {
                const int iq = th % a.nq;
                qv = a.q[iq];
                if (CRS) {
                    const int rest = th / a.nq;
                    Bv = a.B[rest % a.nB];
                    Av = a.A[rest / a.nB];
                }
            }
            if (lane < NT) {
                pq[lane] = qv;
                pA[lane] = Av;
                pB[lane] = Bv;
            }
            qlo = wave_min(on ? qv : 1e300);
            qhi = wave_max(on ? qv : -1e300);
            if (CRS) {
                Alo = wave_min(on ? Av : 1e300);
                Ahi = wave_max(on ? Av : -1e300);
                Blo = wave_min(on ? Bv : 1e300);
                Bhi = wave_max(on ? Bv : -1e300);
            }
        }

        float U[P][W], D[P], Mc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int j = 0; j < W; ++j) U[p][j] = 0.f;
            D[p] = 0.f;
            Mc[p] = 0.f;
        }

        for (int t0 = 0; t0 < ntr;) {
            // ---- wave 0: sample range of the next traces, packed into LDS ----
            if (wv == 0) {
                const int t = t0 + lane;
                int len = 0, lo = 0, nsg = 0;
                long long src = 0;
                double cc = 0.0, dm = 0.0;
                if (t < ntr) {
                    int k = 0;
                    while (k + 1 < na && ag_cum[k + 1] <= t) ++k;
                    const int g = ag_s[k];
                    const int li = t - ag_cum[k];
                    const int i = a.trace_ptr[g] + li;
                    nsg = a.ns[g];
                    src = a.sample_off[g] + (long long)li * nsg;
                    const double h = a.half_offset[i];
                    cc = h * h * inv_dt * inv_dt;
                    // the displacement as the kernels use it: rounded to FP32
                    dm = CRS ? (double)(float)((double)a.midpoint[i] - xc) : 0.0;
                    // bounds of tau^2 over the tile (interval arithmetic, FP64)
                    double Tlo, Thi;
                    const double gl = fmin(qlo * cc, qhi * cc), gh = fmax(qlo * cc, qhi * cc);
                    if (!CRS) {
                        Tlo = (double)s0 * s0 + gl;
                        Thi = (double)s1 * s1 + gh;
                    } else {
                        const double ai = 2.0 * dm * inv_dt, bi = 2.0 * dm * dm * inv_dt;
                        const double al = fmin(Alo * ai, Ahi * ai), ah = fmax(Alo * ai, Ahi * ai);
                        const double bl = Blo * bi, bh = Bhi * bi;  // bi >= 0
                        const double yl = s0 + al, yh = s1 + ah;
                        const double y2l = yl > 0.0 ? yl * yl : (yh < 0.0 ? yh * yh : 0.0);
                        const double y2h = fmax(yl * yl, yh * yh);
                        const double sbl = fmin(fmin(s0 * bl, s0 * bh), fmin(s1 * bl, s1 * bh));
                        const double sbh = fmax(fmax(s0 * bl, s0 * bh), fmax(s1 * bl, s1 * bh));
                        Tlo = y2l + sbl + gl;
                        Thi = y2h + sbh + gh;
                    }
                    if (Thi >= 0.0) {
                        // one sample of margin on each side absorbs rounding
                        const long long klo = (long long)floor(sqrt_refined(Tlo)) - 1;
                        const long long khi = (long long)floor(sqrt_refined(Thi)) + 1;
                        const long long l0 = max(0LL, klo - HW);
                        const long long l1 = min((long long)nsg - 1, khi - HW + W);
                        if (l1 >= l0) {
                            lo = (int)l0;
                            len = (int)(l1 - l0 + 1);
                        }
                    }
                }
                int incl = len;
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    const int v = __shfl_up(incl, o, WAVE);
                    if (lane >= o) incl += v;
                }
                const bool fits = (t < ntr) && incl <= CAP;
                const unsigned long long nf = __ballot(!fits);
                int nfit = nf ? (__ffsll((long long)nf) - 1) : WAVE;
                nfit = min(nfit, ntr - t0);
                if (nfit == 0) {  // a single range larger than CAP: the host keeps ns_max <= CAP
                    nfit = 1;
                    if (lane == 0) len = min(len, CAP), incl = len;
                }
                if (lane < nfit) {
                    t_src[lane] = src + lo;
                    t_len[lane] = len;
                    t_base[lane] = incl - len;
                    // a trace without staged samples gets lim = -1: none of its windows count
                    tinfo[lane] = make_int2(incl - len - lo, len > 0 ? nsg - 1 - W : -1);
                    t_cc[lane] = cc;
                    t_dm[lane] = (float)dm;
                }
                if (lane == 0) sh_nfit = nfit;
            }
            __syncthreads();
            const int nfit = sh_nfit;

            // ---- stage the samples and their window energy -------------------
            // Direct global->LDS loads (global_load_lds_dword): lane l of a wave
            // fetches element p0 + l of the trace's range into LDS word
            // base + p0 + l without passing through registers, so every load of
            // the chunk is in flight at once; the barrier below waits for them.
            for (int r = wv; r < nfit; r += NW) {
                const long long src = t_src[r];
                const int len = t_len[r], base = t_base[r];
                for (int p0 = 0; p0 < len; p0 += WAVE) {
                    if (p0 + lane < len) {
                        const long long gi = src + p0 + lane;
                        lds_dma(a.samples + gi, &lf[base + p0]);
                        lds_dma(a.u0 + gi, &lu0[base + p0]);
                        lds_dma(a.u1 + gi, &lu1[base + p0]);
                        lds_dma(a.u2sq + gi, &lu2[base + p0]);
                    }
                }
            }
            if (CRS) {
                // per (parameter, trace): num = s u1 + u0 with
                //   u1 = 2 alpha + beta, u0 = alpha^2 + gamma (FP64)
                for (int pl = wv; pl < NT; pl += NW) {
                    if (lane < nfit) {
                        const double dmr = t_dm[lane];
                        const double al = pA[pl] * 2.0 * dmr * inv_dt;
                        const double be = pB[pl] * 2.0 * dmr * dmr * inv_dt;
                        tab[pl][lane] = make_double2(2.0 * al + be, fma(al, al, pq[pl] * t_cc[lane]));
                    }
                }
            }
            __syncthreads();

            // ---- the hot loop: traces outer, this lane's P parameters inner ----
            // First the P intersections (independent FP64 chains), then the P
            // windows without branches: a window that is off the trace reads a
            // harmless in-range LDS word with zero weights, so the loads of all
            // P windows can be in flight together.
            double qd[P];  // this wave's parameters (CMP), held in scalar registers
#pragma unroll
            for (int p = 0; p < P; ++p) qd[p] = to_sgpr(pq[wv * P + p]);
            if (lane_on) {
                for (int r = 0; r < nfit; ++r) {
                    const int2 ti = tinfo[r];
                    if (ti.y < 0) continue;  // uniform: no staged window on this trace
                    const double cc = t_cc[r];
                    int idx[P];
                    float xw[P], uw[P], vm[P];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        double num;
                        if (CRS) {
                            const double2 tv = tab[wv * P + p][r];
                            num = fma(sd, tv.x, tv.y);
                        } else {
                            num = qd[p] * cc;
                        }
                        const double T = s2 + num;
                        const Hit hit = hit_from_tau(sqrt_refined(T), HW);
                        const bool ok = on_trace(hit.a, ti.y) && T >= 0.0;
                        idx[p] = ok ? hit.a + ti.x : 0;
                        xw[p] = ok ? hit.x : 0.f;
                        vm[p] = ok ? 1.f : 0.f;
                        uw[p] = vm[p] - xw[p];
                    }
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const int id = idx[p];
                        float fw[W + 1];
#pragma unroll
                        for (int j = 0; j <= W; ++j) fw[j] = lf[id + j];
#pragma unroll
                        for (int j = 0; j < W; ++j) {
                            U[p][j] = fmaf(uw[p], fw[j], U[p][j]);
                            U[p][j] = fmaf(xw[p], fw[j + 1], U[p][j]);
                        }
                        const float tq = fmaf(xw[p], lu1[id], lu0[id]);
                        D[p] = fmaf(vm[p], fmaf(tq, tq, lu2[id]), D[p]);
                        Mc[p] += vm[p];
                    }
                }
            }
            __syncthreads();
            t0 += nfit;
        }

        // ---- semblance of this block's parameters; running pick --------------
        if (lane_on) {
            const int64_t row = a.out_off[job] + s;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int th = pb + wv * P + p;
                if (th < a.npar) {
                    float N = 0.f, L = 0.f;
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        N = fmaf(U[p][j], U[p][j], N);
                        L += U[p][j];
                    }
                    const float S = (Mc[p] > 0.f && D[p] > 0.f) ? N / (Mc[p] * D[p]) : 0.f;
                    const float st = (Mc[p] > 0.f) ? L / (Mc[p] * (float)W) : 0.f;
                    if (a.panel) a.panel[row * a.npar + th] = S;
                    if (S > bS) {  // parameters visited in increasing index: first max wins
                        bS = S;
                        bI = th;
                        bSt = st;
                    }
                }
            }
        }
    }

    // ---- pick across the waves (largest S, then smallest index) --------------
    float *rS = lf;  // reuse the stage buffers
    int *rI = reinterpret_cast<int *>(lu0);
    float *rT = lu1;
    __syncthreads();
    rS[wv * WAVE + lane] = bS;
    rI[wv * WAVE + lane] = bI;
    rT[wv * WAVE + lane] = bSt;
    __syncthreads();
    if (wv == 0 && lane_on) {
#pragma unroll
        for (int v = 1; v < NW; ++v) {
            const float S = rS[v * WAVE + lane];
            const int I = rI[v * WAVE + lane];
            if (S > bS || (S == bS && I < bI)) {
                bS = S;
                bI = I;
                bSt = rT[v * WAVE + lane];
            }
        }
        const int64_t row = a.out_off[job] + s;
        a.best[row] = bI;
        a.s_best[row] = bS < 0.f ? 0.f : bS;
        a.stack[row] = bSt;
    }
}

// Tile shape per kind (measured on MI355X, see the design notes): CMP keeps 4
// parameters per lane in 4 waves at <= 128 VGPRs (4 waves per SIMD); CRS, whose
// per-eval table read and larger apertures favour occupancy, uses 2
// parameters per lane in 8 waves.  Stage capacity: 2048 positions (CMP, four
// workgroups per CU), 3072 (CRS, two workgroups per CU).
template <int KIND, int W>
hipError_t launch_w(const ScanArgs &a, hipStream_t stream)
{
    constexpr bool CRS = KIND == SEMB_KIND_CRS;
    constexpr int NW = CRS ? 8 : 4;
    constexpr int P = CRS ? 2 : (W <= 15 ? 4 : 2);
    constexpr int WPE = CRS ? 1 : 4;
    constexpr int CAP = CRS ? 3072 : 2048;
    const long long nblk = (long long)a.njobs * a.n_sblk;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL((scan_kernel<KIND, W, P, NW, CAP, WPE>), dim3((unsigned)nblk), dim3(NW * WAVE), 0,
                       stream, a);
    return hipGetLastError();
}

template <int KIND>
hipError_t launch_kind(const ScanArgs &a, hipStream_t stream)
{
    switch (a.w) {
    case 1: return launch_w<KIND, 1>(a, stream);
    case 3: return launch_w<KIND, 3>(a, stream);
    case 5: return launch_w<KIND, 5>(a, stream);
    case 7: return launch_w<KIND, 7>(a, stream);
    case 9: return launch_w<KIND, 9>(a, stream);
    case 11: return launch_w<KIND, 11>(a, stream);
    case 13: return launch_w<KIND, 13>(a, stream);
    case 15: return launch_w<KIND, 15>(a, stream);
    case 17: return launch_w<KIND, 17>(a, stream);
    case 19: return launch_w<KIND, 19>(a, stream);
    case 21: return launch_w<KIND, 21>(a, stream);
    case 23: return launch_w<KIND, 23>(a, stream);
    case 25: return launch_w<KIND, 25>(a, stream);
    case 27: return launch_w<KIND, 27>(a, stream);
    case 29: return launch_w<KIND, 29>(a, stream);
    case 31: return launch_w<KIND, 31>(a, stream);
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
    hipLaunchKernelGGL(window_energy_kernel, dim3((unsigned)ntraces), dim3(256), 0, stream, samples,
                       sample_off, trace_ptr, ns, ngathers, w, u0, u1, u2sq);
    return hipGetLastError();
}

hipError_t launch_scan(int kind, const ScanArgs &a, hipStream_t stream)
{
    return kind == SEMB_KIND_CMP ? launch_kind<SEMB_KIND_CMP>(a, stream)
                                 : launch_kind<SEMB_KIND_CRS>(a, stream);
}

}  // namespace semb
