// tile.h -- device code of one tile of the CMP / 2D-CRS semblance scan, shared
// by the exhaustive scan kernels (one translation unit per kind) and the
// batched kernel, and the tile shapes the scan kernels are built in.
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

#pragma once

#include <hip/hip_fp16.h>

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

// The LDS word `byte` bytes into a tile's stage, as one address that the
// optimiser cannot re-derive, so the window's w + 1 samples and its three
// energy words are all read from this address plus immediate offsets.
__device__ __forceinline__ const float *stage_at(const float *stage, unsigned byte)
{
    asm("" : "+v"(byte));
    return reinterpret_cast<const float *>(reinterpret_cast<const char *>(stage) + byte);
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
// One tile of the scan: output samples 64*sblk .. 64*sblk+63 of a job and
// flat parameter indices [pbeg, pend).  KIND: SEMB_KIND_CMP / SEMB_KIND_CRS.
// W: window.  P: parameters per lane.  NW: waves per workgroup.  CAP: LDS
// sample positions per stage.  TMAX: traces whose metadata is held in LDS at
// once.  BRANCHY: windows behind a per-parameter branch (skips off-trace
// windows) instead of the branch-free form (keeps every window's loads in
// flight).
//
// Per parameter block the tile makes three kinds of pass:
//   * the trace pass (all threads, one trace each): the sample range every
//     trace can be touched in by the block, bounded by interval arithmetic
//     over the block's parameter box (the paper's min/max of the k1 indices);
//   * per chunk, the stage: every wave packs the next traces whose ranges fit
//     in CAP (the same prefix scan in every wave, so no wave waits for
//     another to decide), then the waves move the ranges into LDS with direct
//     global->LDS loads;
//   * the hot loop over the staged traces.
// The traces' metadata (first sample, length, h^2/dt^2, dm) is loaded into
// LDS once per tile when the aperture has at most TMAX traces, else once per
// TMAX-trace part of it.
// ---------------------------------------------------------------------------
// What the hot loop needs of one trace, read with one LDS load (all 16 bytes
// for CMP; CRS takes its traveltime terms from the parameter table and reads
// the first 8): the last valid window start (-1: nothing staged), the byte
// offset in the stage such that the window of an intersection with floor k
// starts at byte 4 k + off, and h^2/dt^2.
struct __align__(16) TraceRun {
    int lim;
    int off;
    double cc;
};

// Positions of one LDS plane: a block of zeros (at least the W + 1 words a
// window reads) that windows off their trace read in the branch-free tile
// shapes, then the CAP staged positions.  For CMP the block is 64 words, so
// that the plane stride stays a multiple of 64 words (CAP is one) and one
// ds_read2st64 fetches a window's u0 and u1 (measured 0.9% faster on the
// CMP-large scan); for CRS it is W + 1 rounded up to 4 words, which keeps the
// 8 x 4 tile within 128 VGPRs without spills (the wider block measured 0.9%
// slower on the CRS line).
template <int KIND, int W, int CAP>
struct Plane {
    static_assert(W + 1 <= 64 && CAP % 64 == 0, "zero block and stage sizes");
    static constexpr int ZP = KIND == SEMB_KIND_CMP ? 64 : (W + 1 + 3) & ~3;  // words of the zero block
    static constexpr int STRIDE = ZP + CAP;                                    // words per plane
};

template <int KIND, int W, int P, int NW, int CAP, int TMAX>
struct StageLds {
    float st[4][Plane<KIND, W, CAP>::STRIDE];             // staged samples, then their window energy
                                                    // (Gram form): u0, u1, u2^2; each plane
                                                    // starts with the zero block
    double2 tab[KIND == SEMB_KIND_CRS ? NW * P : 1][WAVE];  // CRS: (2 alpha + beta, alpha^2 + gamma)
    // the traces of the current part: fixed per tile ...
    long long t_base[TMAX];                         // element of the trace's sample 0
    int t_ns[TMAX];
    float t_dm[TMAX];                               // midpoint displacement (CRS)
    // ... and per parameter block
    int t_lo[TMAX], t_len[TMAX];                    // staged range [lo, lo + len)
    TraceRun run[TMAX];                             // what the hot loop reads per trace
    double pq[NW * P], pA[NW * P], pB[NW * P];      // the current parameter block
    double box[6];                                  // its bounds: q, A, B (lo, hi)
    int ag_s[SEMB_APERT_LIMIT];
    int ag_cum[SEMB_APERT_LIMIT + 1];
};

// Metadata of traces [tA, tA + nt) of the aperture into L.t_* (all threads).
template <int KIND, class LDS>
__device__ __forceinline__ void load_traces(const GatherView &g, LDS &L, int na, int tA, int nt, double xc,
                                            double inv_dt, int nthreads)
{
    for (int e = threadIdx.x; e < nt; e += nthreads) {
        const int t = tA + e;
        int k = 0;
        while (k + 1 < na && L.ag_cum[k + 1] <= t) ++k;
        const int gg = L.ag_s[k];
        const int li = t - L.ag_cum[k];
        const int i = g.trace_ptr[gg] + li;
        const int nsg = g.ns[gg];
        L.t_base[e] = g.sample_off[gg] + (long long)li * nsg;
        L.t_ns[e] = nsg;
        const double h = g.half_offset[i];
        L.run[e].cc = h * h * inv_dt * inv_dt;
        // the displacement as the kernels use it: rounded to FP32
        L.t_dm[e] = KIND == SEMB_KIND_CRS ? (float)((double)g.midpoint[i] - xc) : 0.f;
    }
}

// All threads of the workgroup call this together.  On return, lane l of
// wave 0 holds the pick of output sample 64*sblk + l over [pbeg, pend):
// bS (negative if the lane's sample lies beyond the job's trace length), bI,
// bSt.  panel / panel16: optional [row][npar] semblance of every cell, FP32
// and FP16 (round to nearest even).
template <int KIND, int W, int P, int NW, int CAP, int TMAX, bool BRANCHY>
__device__ __forceinline__ void scan_tile(const GatherView &g, const JobView &jv, const ParamView &pv,
                                          StageLds<KIND, W, P, NW, CAP, TMAX> &L, int job, int sblk, int pbeg,
                                          int pend, float *panel, __half *panel16, float &bS, int &bI,
                                          float &bSt)
{
    constexpr int HW = (W - 1) / 2;
    constexpr int NT = NW * P;  // parameters per block
    constexpr int NTH = NW * WAVE;
    constexpr bool CRS = KIND == SEMB_KIND_CRS;

    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wv = __builtin_amdgcn_readfirstlane(tid / WAVE);

    const int c = jv.central[job];
    const int nsc = g.ns[c];
    const int s0 = sblk * WAVE;
    const int s1 = min(s0 + WAVE, nsc) - 1;
    const int s = s0 + lane;
    const bool lane_on = s < nsc;

    bS = -1.f;
    bSt = 0.f;
    bI = pbeg;

    __syncthreads();  // the previous tile (persistent loop) is done with L
    // ---- the job's aperture: gathers and cumulative trace counts ----------
    // (a CRS aperture longer than jv.max_apert never reaches this point: the
    // kernels write the documented marker instead, see apert_over)
    int na = 1, afirst = -1;
    if (CRS && jv.apert_ptr != nullptr) {
        afirst = jv.apert_ptr[job];
        na = max(min(jv.apert_ptr[job + 1] - afirst, jv.max_apert), 0);
    }
    if (tid < na) L.ag_s[tid] = (afirst < 0) ? c : jv.apert_gather[afirst + tid];
    // the zero block at the start of every plane (read by off-trace windows;
    // the previous tile's pick may have reused it)
    constexpr int ZW = Plane<KIND, W, CAP>::ZP;
    if (tid < 4 * ZW) L.st[tid / ZW][tid % ZW] = 0.f;
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        L.ag_cum[0] = 0;
        for (int k = 0; k < na; ++k) {
            const int gg = L.ag_s[k];
            acc += g.trace_ptr[gg + 1] - g.trace_ptr[gg];
            L.ag_cum[k + 1] = acc;
        }
    }
    __syncthreads();
    const int ntr = L.ag_cum[na];
    const double xc = CRS ? (double)g.central_x[c] : 0.0;
    const double inv_dt = 1.0 / (double)g.dt;
    const bool resident = ntr <= TMAX;  // one part: metadata loaded once per tile
    if (resident) load_traces<KIND>(g, L, na, 0, ntr, xc, inv_dt, NTH);

    const double sd = (double)s;
    // s^2, but 1e-300 at s = 0, so that T = 0 from a zero offset and zero
    // displacement stays positive (tau ~ 1e-150: window start -hw, fraction 0)
    const double s2e = s > 0 ? sd * sd : 1e-300;

    for (int pb = pbeg; pb < pend; pb += NT) {
        // ---- this block's parameters, decoded once by wave 0 (one per lane) into
        // LDS, with their bounds reduced across the wave.  The previous block
        // ended with a barrier, so the parameter arrays are free.
        if (wv == 0) {
            const int th = pb + lane;
            const bool on = lane < NT && th < pend;
            double qv = 0.0, Av = 0.0, Bv = 0.0;
            if (on) {
                const int iq = th % pv.nq;
                qv = pv.q[iq];
                if (CRS) {
                    const int rest = th / pv.nq;
                    Bv = pv.B[rest % pv.nB];
                    Av = pv.A[rest / pv.nB];
                }
            }
            if (lane < NT) {
                L.pq[lane] = qv;
                L.pA[lane] = Av;
                L.pB[lane] = Bv;
            }
            const double qlo = wave_min(on ? qv : 1e300), qhi = wave_max(on ? qv : -1e300);
            double Alo = 0.0, Ahi = 0.0, Blo = 0.0, Bhi = 0.0;
            if (CRS) {
                Alo = wave_min(on ? Av : 1e300);
                Ahi = wave_max(on ? Av : -1e300);
                Blo = wave_min(on ? Bv : 1e300);
                Bhi = wave_max(on ? Bv : -1e300);
            }
            if (lane == 0) {
                L.box[0] = qlo;
                L.box[1] = qhi;
                L.box[2] = Alo;
                L.box[3] = Ahi;
                L.box[4] = Blo;
                L.box[5] = Bhi;
            }
        }

        float U[P][W], D[P];
        int Mi[P];  // contributing traces
#pragma unroll
        for (int p = 0; p < P; ++p) {
#pragma unroll
            for (int j = 0; j < W; ++j) U[p][j] = 0.f;
            D[p] = 0.f;
            Mi[p] = 0;
        }

        for (int tA = 0; tA < ntr; tA += TMAX) {
            const int nt = min(TMAX, ntr - tA);
            __syncthreads();  // parameters and box visible; the previous part is done with L.t_*
            if (!resident) load_traces<KIND>(g, L, na, tA, nt, xc, inv_dt, NTH);
            // ---- trace pass: the range of samples the block can touch --------
            {
                const double qlo = L.box[0], qhi = L.box[1];
                for (int e = tid; e < nt; e += NTH) {
                    const double cc = L.run[e].cc;
                    const int nsg = L.t_ns[e];
                    int len = 0, lo = 0;
                    double Tlo, Thi;
                    const double gl = fmin(qlo * cc, qhi * cc), gh = fmax(qlo * cc, qhi * cc);
                    if (!CRS) {
                        Tlo = (double)s0 * s0 + gl;
                        Thi = (double)s1 * s1 + gh;
                    } else {
                        const double Alo = L.box[2], Ahi = L.box[3], Blo = L.box[4], Bhi = L.box[5];
                        const double dm = L.t_dm[e];
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
                    L.t_lo[e] = lo;
                    L.t_len[e] = len;
                    // a trace without staged samples gets lim = -1: none of its windows count
                    L.run[e].lim = len > 0 ? nsg - 1 - W : -1;
                }
            }
            __syncthreads();

            for (int cb = 0; cb < nt;) {
                // ---- pack the next traces into one stage (every wave alike) -----
                const int e = cb + lane;
                int len = e < nt ? L.t_len[e] : 0;
                int incl = len;
#pragma unroll
                for (int o = 1; o < WAVE; o <<= 1) {
                    const int v = __shfl_up(incl, o, WAVE);
                    if (lane >= o) incl += v;
                }
                const bool fits = e < nt && incl <= CAP;
                const unsigned long long nf = __ballot(!fits);
                int nfit = nf ? (__ffsll((long long)nf) - 1) : WAVE;
                nfit = min(nfit, nt - cb);
                if (nfit == 0) {  // a range larger than CAP: excluded by the host (ns_max <= CAP)
                    nfit = 1;
                    len = min(len, CAP);
                    incl = len;
                }
                // window start a = k - HW sits at stage position ZP + (incl - len) + a - lo
                if (wv == 0 && lane < nfit) L.run[e].off = 4 * (Plane<KIND, W, CAP>::ZP + incl - len - L.t_lo[e] - HW);

                // ---- stage the samples and their window energy -------------------
                // Direct global->LDS loads (global_load_lds_dword): lane l of a wave
                // fetches element p0 + l of the trace's range into LDS word
                // base + p0 + l without passing through registers, so every load of
                // the chunk is in flight at once; the barrier below waits for them.
                for (int r = wv; r < nfit; r += NW) {
                    const int rl = __builtin_amdgcn_readlane(len, r);
                    const int rb = __builtin_amdgcn_readlane(incl, r) - rl;
                    const long long src = L.t_base[cb + r] + L.t_lo[cb + r];
                    for (int p0 = 0; p0 < rl; p0 += WAVE) {
                        if (p0 + lane < rl) {
                            const long long gi = src + p0 + lane;
                            const int at = Plane<KIND, W, CAP>::ZP + rb + p0;
                            lds_dma(g.samples + gi, &L.st[0][at]);
                            lds_dma(pv.u0 + gi, &L.st[1][at]);
                            lds_dma(pv.u1 + gi, &L.st[2][at]);
                            lds_dma(pv.u2sq + gi, &L.st[3][at]);
                        }
                    }
                }
                if (CRS) {
                    // per (parameter, trace): num = s u1 + u0 with
                    //   u1 = 2 alpha + beta, u0 = alpha^2 + gamma (FP64)
                    for (int pl = wv; pl < NT; pl += NW) {
                        if (lane < nfit) {
                            const double dmr = L.t_dm[e];
                            const double al = L.pA[pl] * 2.0 * dmr * inv_dt;
                            const double be = L.pB[pl] * 2.0 * dmr * dmr * inv_dt;
                            L.tab[pl][lane] = make_double2(2.0 * al + be, fma(al, al, L.pq[pl] * L.run[e].cc));
                        }
                    }
                }
                __syncthreads();

                // ---- the hot loop: traces outer, this lane's P parameters inner ----
                // A trace counts iff T > 0 and its window lies on the trace; T = 0
                // only arises from s = 0 with nothing else (handled by s2e above)
                // or exactly on a CRS surface's edge, a set of measure zero.
                double qd[P];  // this wave's parameters (CMP), held in scalar registers
#pragma unroll
                for (int p = 0; p < P; ++p) qd[p] = to_sgpr(L.pq[wv * P + p]);
                // CMP: a wave whose parameters all lie past the block's end (the
                // last block of a ragged grid) has nothing to add; it only keeps
                // the barriers, and its SIMD slots go to the other workgroups
                // (measured 1.1% on the CMP-large scan and 2.5% on CMP plain; the
                // CRS grids' last blocks are a negligible share, and there the
                // test cost more than it saved)
                const bool wave_on = CRS || pb + wv * P < pend;
                if (lane_on && wave_on) {
                    for (int r = 0; r < nfit; ++r) {
                        // one LDS load per trace: lim and off, and for CMP cc (the
                        // empty asm keeps the optimiser from splitting the load
                        // around the test below)
                        int lim, off;
                        double cc = 0.0;
                        if (CRS) {
                            typedef int v2i __attribute__((ext_vector_type(2)));
                            v2i tr = *reinterpret_cast<const v2i *>(&L.run[cb + r]);
                            asm("" : "+v"(tr));
                            lim = tr.x;
                            off = tr.y;
                        } else {
                            typedef int v4i __attribute__((ext_vector_type(4)));
                            v4i tr = *reinterpret_cast<const v4i *>(&L.run[cb + r]);
                            asm("" : "+v"(tr));
                            lim = tr.x;
                            off = tr.y;
                            cc = __hiloint2double(tr.w, tr.z);
                        }
                        if (lim < 0) continue;  // uniform: no staged window on this trace
                        if (BRANCHY) {
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                double T;
                                if (CRS) {
                                    const double2 tv = L.tab[wv * P + p][r];
                                    T = s2e + fma(sd, tv.x, tv.y);
                                } else {
                                    T = fma(qd[p], cc, s2e);
                                }
                                // k = floor(tau) for 0 <= tau < 2^31.  T <= 0 gives a
                                // NaN or an infinity, which the range test below must
                                // reject without a test on T.  For HW >= 1 the
                                // hardware conversion does it: it saturates (+inf and
                                // tau >= 2^31 give INT_MAX) and turns NaN into 0, and
                                // both lie outside [HW, lim + HW].  For HW = 0 a NaN
                                // would give the valid start 0, so tau is first
                                // clamped to 2^30 (fmin drops the NaN).
                                double tau = sqrt_newton(T);
                                int k;
                                if (HW >= 1) {
                                    asm("v_cvt_i32_f64 %0, %1" : "=v"(k) : "v"(tau));
                                } else {
                                    tau = fmin(tau, 1073741824.0);
                                    k = (int)tau;
                                }
                                if (!((unsigned)(k - HW) <= (unsigned)lim)) continue;
                                const float x = (float)__builtin_amdgcn_fract(tau);
                                const float u = 1.f - x;
                                const float *sp = stage_at(&L.st[0][0], ((unsigned)k << 2) + (unsigned)off);
                                constexpr int PS = Plane<KIND, W, CAP>::STRIDE;
                                float fw[W + 1];
#pragma unroll
                                for (int j = 0; j <= W; ++j) fw[j] = sp[j];
#pragma unroll
                                for (int j = 0; j < W; ++j) {
                                    U[p][j] = fmaf(u, fw[j], U[p][j]);
                                    U[p][j] = fmaf(x, fw[j + 1], U[p][j]);
                                }
                                const float tq = fmaf(x, sp[2 * PS], sp[PS]);
                                D[p] += fmaf(tq, tq, sp[3 * PS]);
                                Mi[p] += 1;
                            }
                        } else {
                            // every window is read: one that is off its trace reads
                            // the zero block at byte 0 of each plane, and adds exact
                            // zeros whatever its (finite) weights, so the loads of all
                            // P windows can be in flight together
                            unsigned addr[P];
                            float xw[P], uw[P];
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                double T;
                                if (CRS) {
                                    const double2 tv = L.tab[wv * P + p][r];
                                    T = s2e + fma(sd, tv.x, tv.y);
                                } else {
                                    T = fma(qd[p], cc, s2e);
                                }
                                const double tau = fmin(sqrt_newton(T), 1073741824.0);
                                const int k = (int)tau;
                                const bool ok = (unsigned)(k - HW) <= (unsigned)lim;
                                addr[p] = ok ? ((unsigned)k << 2) + (unsigned)off : 0u;
                                xw[p] = (float)__builtin_amdgcn_fract(tau);  // tau <= 2^30: finite
                                uw[p] = 1.f - xw[p];
                                Mi[p] += ok ? 1 : 0;
                            }
#pragma unroll
                            for (int p = 0; p < P; ++p) {
                                const float *sp = stage_at(&L.st[0][0], addr[p]);
                                constexpr int PS = Plane<KIND, W, CAP>::STRIDE;
                                float fw[W + 1];
#pragma unroll
                                for (int j = 0; j <= W; ++j) fw[j] = sp[j];
#pragma unroll
                                for (int j = 0; j < W; ++j) {
                                    U[p][j] = fmaf(uw[p], fw[j], U[p][j]);
                                    U[p][j] = fmaf(xw[p], fw[j + 1], U[p][j]);
                                }
                                const float tq = fmaf(xw[p], sp[2 * PS], sp[PS]);
                                D[p] += fmaf(tq, tq, sp[3 * PS]);
                            }
                        }
                    }
                }
                __syncthreads();
                cb += nfit;
            }
        }

        // ---- semblance of this block's parameters; running pick --------------
        if (lane_on) {
            const int64_t row = jv.out_off[job] + s;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int th = pb + wv * P + p;
                if (th < pend) {
                    float N = 0.f, Ls = 0.f;
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        N = fmaf(U[p][j], U[p][j], N);
                        Ls += U[p][j];
                    }
                    const float Mc = (float)Mi[p];
                    const float S = (Mc > 0.f && D[p] > 0.f) ? N / (Mc * D[p]) : 0.f;
                    const float st = (Mc > 0.f) ? Ls / (Mc * (float)W) : 0.f;
                    if (panel) panel[row * pv.npar + th] = S;
                    if (panel16) panel16[row * pv.npar + th] = __float2half(S);
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
    float *rS = L.st[0];  // reuse the stage buffers
    int *rI = reinterpret_cast<int *>(L.st[1]);
    float *rT = L.st[2];
    __syncthreads();
    rS[wv * WAVE + lane] = bS;
    rI[wv * WAVE + lane] = bI;
    rT[wv * WAVE + lane] = bSt;
    __syncthreads();
    if (wv == 0) {
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
    }
}

// ---------------------------------------------------------------------------
// Tile shapes.  A scan kernel is built for every (kind, window, shape); the
// library's tuner times the shapes on a sample of the caller's jobs and keeps
// the fastest whose outputs equal the default shape's bit for bit (every
// shape sums each cell's traces in the same order, and a branch-free window
// that is off the trace adds exact zeros, so they do).
//   0: 4 waves x 4 parameters per lane (2 for w > 15) at <= 128 VGPRs (4 waves
//      per SIMD), 2048-position stage, windows behind a branch -- the CMP
//      default;
//   1: 8 waves x 2 parameters, 3072-position stage, branch-free windows;
//   2: 8 waves x 4 parameters (2 for w > 9), 2560-position stage,
//      branch-free windows -- the CRS default: 4 parameters share each
//      trace's loop work, the loads of all 4 windows are in flight together,
//      and the stage and 128 VGPRs still leave two workgroups per CU;
//   3: 4 waves x 4 parameters (2 for w > 15), 2048-position stage,
//      branch-free windows;
//   4: 8 waves x 4 parameters (2 for w > 15), 2048-position stage, windows
//      behind a branch: twice the parameters per staged chunk;
//   5: 16 waves x 4 parameters (2 for w > 15), 2048-position stage, windows
//      behind a branch: four times the parameters per staged chunk.
// ---------------------------------------------------------------------------
template <int SID, int W>
struct ShapeT;
template <int W>
struct ShapeT<0, W> {
    static constexpr int NW = 4, P = W <= 15 ? 4 : 2, CAP = 2048, TMAX = 128, WPE = 4;
    static constexpr bool BRANCHY = true;
};
template <int W>
struct ShapeT<1, W> {
    static constexpr int NW = 8, P = 2, CAP = 3072, TMAX = 256, WPE = 1;
    static constexpr bool BRANCHY = false;
};
template <int W>
struct ShapeT<2, W> {
    static constexpr int NW = 8, P = W <= 9 ? 4 : 2, CAP = 2560, TMAX = 128, WPE = 2;
    static constexpr bool BRANCHY = false;
};
template <int W>
struct ShapeT<3, W> {
    static constexpr int NW = 4, P = W <= 15 ? 4 : 2, CAP = 2048, TMAX = 128, WPE = 4;
    static constexpr bool BRANCHY = false;
};

template <int W>
struct ShapeT<4, W> {
    static constexpr int NW = 8, P = W <= 15 ? 4 : 2, CAP = 2048, TMAX = 128, WPE = 4;
    static constexpr bool BRANCHY = true;
};
template <int W>
struct ShapeT<5, W> {
    static constexpr int NW = 16, P = W <= 15 ? 4 : 2, CAP = 2048, TMAX = 128, WPE = 4;
    static constexpr bool BRANCHY = true;
};

// Rows 64*sblk .. of a job whose aperture is longer than the caller declared:
// best = -1, s_best = -1, stack = 0 and (if requested) panel cells of -1.
__device__ __forceinline__ void write_apert_marker(const JobView &jv, int job, int sblk, int nsc, int npar,
                                                   int32_t *best, float *s_best, float *stack, float *panel,
                                                   __half *panel16)
{
    const int s0 = sblk * WAVE;
    const int nr = min(WAVE, nsc - s0);
    const int64_t row0 = jv.out_off[job] + s0;
    if ((int)threadIdx.x < nr) {
        best[row0 + threadIdx.x] = -1;
        s_best[row0 + threadIdx.x] = -1.f;
        stack[row0 + threadIdx.x] = 0.f;
    }
    if (panel || panel16) {
        const int64_t ncell = (int64_t)nr * npar;
        for (int64_t e = threadIdx.x; e < ncell; e += blockDim.x) {
            if (panel) panel[row0 * npar + e] = -1.f;
            if (panel16) panel16[row0 * npar + e] = __float2half(-1.f);
        }
    }
}

// The exhaustive scan: one workgroup per (job, sample block), all parameters.
template <int KIND, int W, int SID>
__global__ void __launch_bounds__((ShapeT<SID, W>::NW * WAVE))
__attribute__((amdgpu_waves_per_eu(ShapeT<SID, W>::WPE)))
scan_kernel(ScanArgs a)
{
    using S = ShapeT<SID, W>;
    __shared__ StageLds<KIND, W, S::P, S::NW, S::CAP, S::TMAX> L;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int job = tile / a.j.n_sblk;
    const int sblk = tile - job * a.j.n_sblk;
    if (job >= a.j.njobs) return;
    const int nsc = a.g.ns[a.j.central[job]];
    if (sblk * WAVE >= nsc) return;  // uniform, before any barrier
    if (KIND == SEMB_KIND_CRS && apert_over(a.j.apert_ptr, a.j.max_apert, job)) {
        write_apert_marker(a.j, job, sblk, nsc, a.p.npar, a.best, a.s_best, a.stack, a.panel,
                           static_cast<__half *>(a.panel16));
        return;
    }
    float bS, bSt;
    int bI;
    scan_tile<KIND, W, S::P, S::NW, S::CAP, S::TMAX, S::BRANCHY>(a.g, a.j, a.p, L, job, sblk, 0, a.p.npar,
                                                                   a.panel, static_cast<__half *>(a.panel16), bS, bI,
                                                                   bSt);
    const int lane = threadIdx.x & (WAVE - 1);
    if (threadIdx.x < WAVE && bS >= 0.f) {
        const int64_t row = a.j.out_off[job] + sblk * WAVE + lane;
        a.best[row] = bI;
        a.s_best[row] = bS;
        a.stack[row] = bSt;
    }
}

template <int KIND, int W, int SID>
hipError_t launch_ws(const ScanArgs &a, hipStream_t stream)
{
    const long long nblk = (long long)a.j.njobs * a.j.n_sblk;
    if (nblk == 0) return hipSuccess;
    hipLaunchKernelGGL((scan_kernel<KIND, W, SID>), dim3((unsigned)nblk), dim3(ShapeT<SID, W>::NW * WAVE), 0,
                       stream, a);
    return hipGetLastError();
}

template <int KIND, int SID>
hipError_t launch_s(const ScanArgs &a, hipStream_t stream)
{
    switch (a.p.w) {
    case 1: return launch_ws<KIND, 1, SID>(a, stream);
    case 3: return launch_ws<KIND, 3, SID>(a, stream);
    case 5: return launch_ws<KIND, 5, SID>(a, stream);
    case 7: return launch_ws<KIND, 7, SID>(a, stream);
    case 9: return launch_ws<KIND, 9, SID>(a, stream);
    case 11: return launch_ws<KIND, 11, SID>(a, stream);
    case 13: return launch_ws<KIND, 13, SID>(a, stream);
    case 15: return launch_ws<KIND, 15, SID>(a, stream);
    case 17: return launch_ws<KIND, 17, SID>(a, stream);
    case 19: return launch_ws<KIND, 19, SID>(a, stream);
    case 21: return launch_ws<KIND, 21, SID>(a, stream);
    case 23: return launch_ws<KIND, 23, SID>(a, stream);
    case 25: return launch_ws<KIND, 25, SID>(a, stream);
    case 27: return launch_ws<KIND, 27, SID>(a, stream);
    case 29: return launch_ws<KIND, 29, SID>(a, stream);
    case 31: return launch_ws<KIND, 31, SID>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int KIND>
hipError_t launch_scan_kind(const ScanArgs &a, int sid, hipStream_t stream)
{
    switch (sid) {
    case 0: return launch_s<KIND, 0>(a, stream);
    case 1: return launch_s<KIND, 1>(a, stream);
    case 2: return launch_s<KIND, 2>(a, stream);
    case 3: return launch_s<KIND, 3>(a, stream);
    case 4: return launch_s<KIND, 4>(a, stream);
    case 5: return launch_s<KIND, 5>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace semb
