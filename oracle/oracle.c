/*
 * oracle.c -- FP64 CPU oracle of the CMP / 2D-CRS semblance parameter scan.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP implementation and must never be used
 * as a fallback for it.
 *
 * What it computes (Hu, Yang, Luan, Qian, "Massively Scaling Seismic
 * Processing on Sunway TaihuLight Supercomputer"):
 *
 *  - the grid search of section 3.2 (Fig. 5b): for every output sample t0 of a
 *    central gather and every candidate parameter theta, the semblance of the
 *    traces along the traveltime curve (CMP, section 2.1) or surface (CRS,
 *    section 2.2, where the traces of the neighbouring gathers join in);
 *  - the semblance of Eq. (1) over a window of w samples centred on each
 *    trace's intersection, each sample linearly interpolated with the one
 *    fraction x of the intersection (Algorithm 1, the accumulation of _num,
 *    _den and _ac_linear; Algorithm 2 performs the same sums trace-outer);
 *  - the pick of the most coherent parameter per sample (section 3.2) and the
 *    stacked amplitude along it.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *  - traveltime, CMP:  T = t0^2 + q h^2, q = 4/v^2, h = half-offset;
 *    CRS: T = (t0 + 2 A dm)^2 + 2 t0 B dm^2 + q h^2, dm = trace midpoint -
 *    central midpoint (the paper names the curve and the surface but prints
 *    neither formula);
 *  - tau = sqrt(T)/dt samples, k = floor(tau), x = tau - k, window start
 *    a = k - (w-1)/2; sample j of the window is f[a+j] + x (f[a+j+1] - f[a+j]);
 *  - a trace contributes only if T >= 0 and 0 <= a and a + w <= ns - 1 (all
 *    w+1 samples the window reads lie on the trace);
 *  - S = sum_j U_j^2 / (M * D) with U_j the sum over contributing traces of
 *    window sample j, D the sum of the squares, M the number of contributing
 *    traces (Eq. (1) with the 1/M that makes S lie in [0, 1]); S = 0 if M = 0
 *    or D = 0;
 *  - stack = L / (M w), L the sum of all window samples (the _ac_linear sum);
 *    stack = 0 if M = 0;
 *  - the pick is the smallest flat parameter index reaching the maximum S;
 *    flat index = (iA * nB + iB) * nq + iq.
 *
 * Pins (tests that fix this code against something other than itself):
 * closed forms at zero moveout, ramp traces, integer-aligned single-event
 * Ricker gathers, invariants (0 <= S <= 1, scale and permutation invariance,
 * CRS with A = B = 0 equals CMP), an independent brute force on tiny
 * gathers, and finite differences for the gradient.  The stack formula, the
 * window-edge rule and the tie-break are readings: the tests pin the code to
 * those readings, the paper does not fix them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_CMP 0
#define ORACLE_CRS 1

/* Perturbations used to flag cells whose set of contributing traces could
 * differ between this FP64 evaluation and another correct evaluation of the
 * same definition in a different arithmetic: a trace is "near a boundary" if
 * moving its intersection by FRAGILE_TAU samples, or its squared traveltime
 * by FRAGILE_T_REL times the magnitude of its terms, changes whether it
 * contributes.  The defaults suit an FP32 traveltime; a caller comparing with
 * an implementation whose traveltime is exact to ~1e-10 samples can narrow
 * them with oracle_set_fragility(). */
static double FRAGILE_TAU = 1e-3;    /* samples */
static double FRAGILE_T_REL = 1e-6;  /* relative */

void oracle_set_fragility(double tau_samples, double t_rel)
{
    FRAGILE_TAU = tau_samples;
    FRAGILE_T_REL = t_rel;
}

/* A contributing intersection within KINK_TAU samples of an integer marks its
 * cell as a kink of the gradient: the window's interpolation segments, and so
 * the slopes dv/dtau, change there.  The default suits a gradient compared
 * with central differences whose step moves tau by less than 1e-4 samples. */
static double KINK_TAU = 1e-4;

void oracle_set_kink(double tau_samples)
{
    KINK_TAU = tau_samples;
}

typedef struct {
    const float *samples;
    const int64_t *sample_off;
    const int32_t *trace_ptr;
    const int32_t *ns;
    const float *half_offset;
    const float *midpoint;
    const float *central_x;
    double dt;
} gset;

typedef struct {
    double A, B, q;
} theta_t;

/* Squared traveltime (s^2) of trace i of the aperture for parameter th.  Also
 * returns the sum of the magnitudes of its terms (for the fragility test). */
static double traveltime_sq(int kind, double t0, theta_t th, double dm, double h, double *mag)
{
    if (kind == ORACLE_CMP) {
        *mag = t0 * t0 + fabs(th.q * h * h);
        return t0 * t0 + th.q * h * h;
    }
    double y = t0 + 2.0 * th.A * dm;
    double b = 2.0 * t0 * th.B * dm * dm;
    double c = th.q * h * h;
    *mag = y * y + fabs(b) + fabs(c);
    return y * y + b + c;
}

/* Is a window starting at sample a = floor(tau) - hw entirely on a trace of
 * ns samples? */
static int window_on_trace(double tau, int w, int ns)
{
    int hw = (w - 1) / 2;
    double kf = floor(tau);
    double a = kf - hw;
    return a >= 0.0 && a + w <= (double)(ns - 1);
}

typedef struct {
    double S, stack, D, N, L;
    int M;
    int fragile;
    int kink;
} cell_t;

/* The accumulators of one (job, t0, theta) cell, traces in ascending order:
 * U[w], D, L and M (Algorithm 1's _num, _den, _ac_linear plus the trace count). */
static cell_t eval_cell(const gset *g, int kind, int central, const int32_t *ag, int na,
                        int s, theta_t th, int w, double *U)
{
    cell_t c = {0};
    const int hw = (w - 1) / 2;
    const double t0 = s * g->dt;
    const double xc = (kind == ORACLE_CRS) ? (double)g->central_x[central] : 0.0;
    for (int j = 0; j < w; j++) U[j] = 0.0;
    c.kink = 0;

    for (int p = 0; p < na; p++) {
        const int gg = ag[p];
        const int nsg = g->ns[gg];
        for (int i = g->trace_ptr[gg]; i < g->trace_ptr[gg + 1]; i++) {
            const float *f = g->samples + g->sample_off[gg] + (int64_t)(i - g->trace_ptr[gg]) * nsg;
            const double h = g->half_offset[i];
            const double dm = (kind == ORACLE_CRS) ? (double)g->midpoint[i] - xc : 0.0;
            double mag;
            const double T = traveltime_sq(kind, t0, th, dm, h, &mag);

            /* fragility: would a tiny change of T or tau change whether this
             * trace contributes? */
            const double dT = FRAGILE_T_REL * mag;
            if (fabs(T) <= dT) {
                int v_lo = (T - dT >= 0.0) && window_on_trace(sqrt(T - dT) / g->dt, w, nsg);
                int v_hi = (T + dT >= 0.0) && window_on_trace(sqrt(T + dT) / g->dt, w, nsg);
                if (v_lo != v_hi) c.fragile = 1;
            }
            if (T < 0.0) continue;
            const double tau = sqrt(T) / g->dt;
            const int valid = window_on_trace(tau, w, nsg);
            if (window_on_trace(tau - FRAGILE_TAU, w, nsg) != valid ||
                window_on_trace(tau + FRAGILE_TAU, w, nsg) != valid)
                c.fragile = 1;
            if (!valid) continue;

            const double kf = floor(tau);
            const double x = tau - kf;
            const int64_t a = (int64_t)kf - hw;
            /* a kink: moving the intersection by KINK_TAU samples would read the
             * window from the neighbouring interpolation segments, whose slopes
             * differ (the derivative in theta jumps there) */
            if (x < KINK_TAU || x > 1.0 - KINK_TAU) c.kink = 1;
            for (int j = 0; j < w; j++) {
                const double f0 = f[a + j], f1 = f[a + j + 1];
                const double v = f0 + x * (f1 - f0);
                U[j] += v;
                c.D += v * v;
                c.L += v;
            }
            c.M += 1;
        }
    }
    for (int j = 0; j < w; j++) c.N += U[j] * U[j];
    c.S = (c.M > 0 && c.D > 0.0) ? c.N / ((double)c.M * c.D) : 0.0;
    c.stack = (c.M > 0) ? c.L / ((double)c.M * (double)w) : 0.0;
    return c;
}

/* Condition number of S at one cell, for the tolerance of a comparison with
 * an FP32 evaluation of the same definition.  S = N / (M D) is formed from two
 * separate sums, N = sum_j U_j^2 and D, whose roundings are independent, so
 * each is perturbed on its own: every term of U_j by the magnitude of the two
 * samples it is interpolated from, and every trace's energy D_i = sum_j v_ij^2
 * by 2 sqrt(D_i) (|A_i| + |A'_i|), A_i and A'_i the norms of the window's
 * samples f[a..a+w-1] and f[a+1..a+w]:
 *   kappa = sum_i [ sum_j |dS/dU_j| (|f[a+j]| + |f[a+j+1]|)
 *                   + |dS/dD| 2 sqrt(D_i) (|A_i| + |A'_i|) ],
 * dS/dU_j = 2 U_j / (M D), dS/dD = -S / D.  Rounding the samples, the
 * interpolation and the energies to FP32 (relative error ~2^-24) moves S by
 * about 2^-24 kappa.  U holds the cell's window sums (eval_cell); 0 when S is
 * identically 0. */
static double cell_cond(const gset *g, int kind, int central, const int32_t *ag, int na, int s,
                        theta_t th, int w, const double *U, cell_t cl)
{
    if (!(cl.M > 0 && cl.D > 0.0)) return 0.0;
    const int hw = (w - 1) / 2;
    const double t0 = s * g->dt;
    const double xc = (kind == ORACLE_CRS) ? (double)g->central_x[central] : 0.0;
    const double MD = (double)cl.M * cl.D;
    double kappa = 0.0;
    for (int p = 0; p < na; p++) {
        const int gg = ag[p];
        const int nsg = g->ns[gg];
        for (int i = g->trace_ptr[gg]; i < g->trace_ptr[gg + 1]; i++) {
            const float *f = g->samples + g->sample_off[gg] + (int64_t)(i - g->trace_ptr[gg]) * nsg;
            const double h = g->half_offset[i];
            const double dm = (kind == ORACLE_CRS) ? (double)g->midpoint[i] - xc : 0.0;
            double mag;
            const double T = traveltime_sq(kind, t0, th, dm, h, &mag);
            if (T < 0.0) continue;
            const double tau = sqrt(T) / g->dt;
            if (!window_on_trace(tau, w, nsg)) continue;
            const double kf = floor(tau);
            const double x = tau - kf;
            const int64_t a = (int64_t)kf - hw;
            double Di = 0.0, nA = 0.0, nA1 = 0.0;
            for (int j = 0; j < w; j++) {
                const double f0 = f[a + j], f1 = f[a + j + 1];
                const double v = f0 + x * (f1 - f0);
                kappa += fabs(2.0 * U[j] / MD) * (fabs(f0) + fabs(f1));
                Di += v * v;
                nA += f0 * f0;
                nA1 += f1 * f1;
            }
            kappa += cl.S / cl.D * 2.0 * sqrt(Di) * (sqrt(nA) + sqrt(nA1));
        }
    }
    return kappa;
}

/* Row r of the output -> (job, sample). */
typedef struct {
    int32_t job, s;
} row_t;

static row_t *make_rows(const gset *g, int32_t njobs, const int32_t *job_central, int64_t *nrows)
{
    int64_t n = 0;
    for (int j = 0; j < njobs; j++) n += g->ns[job_central[j]];
    row_t *rows = (row_t *)malloc(sizeof(row_t) * (size_t)(n > 0 ? n : 1));
    int64_t r = 0;
    for (int j = 0; j < njobs; j++)
        for (int s = 0; s < g->ns[job_central[j]]; s++) {
            rows[r].job = j;
            rows[r].s = s;
            r++;
        }
    *nrows = n;
    return rows;
}

static int check_args(int kind, const gset *g, int w, int nA, int nB, int nq)
{
    if (kind != ORACLE_CMP && kind != ORACLE_CRS) return 1;
    if (w < 1 || (w % 2) == 0) return 1;
    if (nA < 1 || nB < 1 || nq < 1) return 1;
    if (!(g->dt > 0.0)) return 1;
    if (kind == ORACLE_CRS && (!g->midpoint || !g->central_x)) return 1;
    return 0;
}

/* kappa (cell_cond) of the picked cell p of a row; flat p = (iA nB + iB) nq + iq. */
static double pick_cond(const gset *g, int kind, int c, const int32_t *ag, int na, int s, const float *A,
                        int32_t nA, const float *B, int32_t nB, const float *q, int32_t nq, int64_t p, int w,
                        double *U)
{
    (void)nA;
    theta_t th;
    th.q = q[p % nq];
    th.B = (kind == ORACLE_CRS) ? (double)B[(p / nq) % nB] : 0.0;
    th.A = (kind == ORACLE_CRS) ? (double)A[p / ((int64_t)nq * nB)] : 0.0;
    cell_t cl = eval_cell(g, kind, c, ag, na, s, th, w, U);
    return cell_cond(g, kind, c, ag, na, s, th, w, U, cl);
}

/*
 * Exhaustive scan (section 3.2): for every job, output sample and flat
 * parameter index, the semblance; then per output row the pick, its
 * semblance and its stack.  Optional outputs: panel (row-major [row][param]),
 * gap (best S minus the best S of any other parameter), fragile (1 if any
 * cell of the row is fragile), cond (cell_cond of the picked cell) and
 * panel_cond (cell_cond of every cell, laid out like panel).  Output row of
 * (job j, sample s) is out_off[j] + s.  Returns 0, or 1 for invalid
 * arguments.
 */
int oracle_scan(int kind, const float *samples, const int64_t *sample_off, const int32_t *trace_ptr,
                const int32_t *ns, const float *half_offset, const float *midpoint,
                const float *central_x, double dt, int32_t njobs, const int32_t *job_central,
                const int32_t *apert_ptr, const int32_t *apert_gather, const int64_t *out_off,
                const float *A, int32_t nA, const float *B, int32_t nB, const float *q, int32_t nq,
                int32_t w, int32_t *best, double *s_best, double *stack, double *panel, double *gap,
                uint8_t *fragile, double *cond, double *panel_cond, int nthreads)
{
    gset g = {samples, sample_off, trace_ptr, ns, half_offset, midpoint, central_x, dt};
    if (check_args(kind, &g, w, nA, nB, nq)) return 1;
    if (kind == ORACLE_CMP) nA = nB = 1;
    const int64_t npar = (int64_t)nA * nB * nq;
    int64_t nrows;
    row_t *rows = make_rows(&g, njobs, job_central, &nrows);
    if (nthreads < 1) nthreads = 1;

#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int64_t r = 0; r < nrows; r++) {
        double U[64];
        double *Ub = (w <= 64) ? U : (double *)malloc(sizeof(double) * (size_t)w);
        const int j = rows[r].job, s = rows[r].s;
        const int64_t orow = out_off[j] + s;
        const int c = job_central[j];
        const int32_t *ag = apert_gather + apert_ptr[j];
        const int na = apert_ptr[j + 1] - apert_ptr[j];
        double s1 = -1.0, s2 = -1.0, st1 = 0.0;
        int64_t p1 = 0;
        int frag = 0;
        for (int iA = 0; iA < nA; iA++)
            for (int iB = 0; iB < nB; iB++)
                for (int iq = 0; iq < nq; iq++) {
                    theta_t th;
                    th.A = (kind == ORACLE_CRS) ? (double)A[iA] : 0.0;
                    th.B = (kind == ORACLE_CRS) ? (double)B[iB] : 0.0;
                    th.q = q[iq];
                    const int64_t p = ((int64_t)iA * nB + iB) * nq + iq;
                    cell_t cl = eval_cell(&g, kind, c, ag, na, s, th, w, Ub);
                    frag |= cl.fragile;
                    if (panel) panel[orow * npar + p] = cl.S;
                    if (panel_cond)
                        panel_cond[orow * npar + p] = cell_cond(&g, kind, c, ag, na, s, th, w, Ub, cl);
                    if (cl.S > s1) { /* strict: the first index wins ties */
                        s2 = s1;
                        s1 = cl.S;
                        st1 = cl.stack;
                        p1 = p;
                    } else if (cl.S > s2) {
                        s2 = cl.S;
                    }
                }
        best[orow] = (int32_t)p1;
        s_best[orow] = s1;
        stack[orow] = st1;
        if (gap) gap[orow] = (npar > 1) ? s1 - s2 : INFINITY;
        if (fragile) fragile[orow] = (uint8_t)frag;
        if (cond) cond[orow] = pick_cond(&g, kind, c, ag, na, s, A, nA, B, nB, q, nq, p1, w, Ub);
        if (Ub != U) free(Ub);
    }
    free(rows);
    return 0;
}

/*
 * The same exhaustive scan restricted to an explicit list of output rows
 * (row r = sample row_s[r] of job row_job[r]); outputs are indexed by r.
 * Lets a test check sampled rows of a workload too large to scan in full.
 */
int oracle_scan_rows(int kind, const float *samples, const int64_t *sample_off, const int32_t *trace_ptr,
                     const int32_t *ns, const float *half_offset, const float *midpoint,
                     const float *central_x, double dt, int32_t nrows, const int32_t *row_job,
                     const int32_t *row_s, const int32_t *job_central, const int32_t *apert_ptr,
                     const int32_t *apert_gather, const float *A, int32_t nA, const float *B, int32_t nB,
                     const float *q, int32_t nq, int32_t w, int32_t *best, double *s_best, double *stack,
                     double *gap, uint8_t *fragile, double *cond, int nthreads)
{
    gset g = {samples, sample_off, trace_ptr, ns, half_offset, midpoint, central_x, dt};
    if (check_args(kind, &g, w, nA, nB, nq)) return 1;
    if (kind == ORACLE_CMP) nA = nB = 1;
    const int64_t npar = (int64_t)nA * nB * nq;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t r = 0; r < nrows; r++) {
        double U[64];
        double *Ub = (w <= 64) ? U : (double *)malloc(sizeof(double) * (size_t)w);
        const int j = row_job[r], s = row_s[r];
        const int c = job_central[j];
        const int32_t *ag = apert_gather + apert_ptr[j];
        const int na = apert_ptr[j + 1] - apert_ptr[j];
        double s1 = -1.0, s2 = -1.0, st1 = 0.0;
        int64_t p1 = 0;
        int frag = 0;
        for (int64_t p = 0; p < npar; p++) {
            theta_t th;
            th.q = q[p % nq];
            th.B = (kind == ORACLE_CRS) ? (double)B[(p / nq) % nB] : 0.0;
            th.A = (kind == ORACLE_CRS) ? (double)A[p / ((int64_t)nq * nB)] : 0.0;
            cell_t cl = eval_cell(&g, kind, c, ag, na, s, th, w, Ub);
            frag |= cl.fragile;
            if (cl.S > s1) {
                s2 = s1;
                s1 = cl.S;
                st1 = cl.stack;
                p1 = p;
            } else if (cl.S > s2) {
                s2 = cl.S;
            }
        }
        best[r] = (int32_t)p1;
        s_best[r] = s1;
        stack[r] = st1;
        if (gap) gap[r] = (npar > 1) ? s1 - s2 : INFINITY;
        if (fragile) fragile[r] = (uint8_t)frag;
        if (cond) cond[r] = pick_cond(&g, kind, c, ag, na, s, A, nA, B, nB, q, nq, p1, w, Ub);
        if (Ub != U) free(Ub);
    }
    return 0;
}

/*
 * Point evaluation: semblance and stack of every output row at its own
 * parameter theta[row] = (A, B, q) (CMP ignores A and B).  Optional per-row
 * contributing-trace count M and fragility flag.
 */
int oracle_point(int kind, const float *samples, const int64_t *sample_off, const int32_t *trace_ptr,
                 const int32_t *ns, const float *half_offset, const float *midpoint,
                 const float *central_x, double dt, int32_t njobs, const int32_t *job_central,
                 const int32_t *apert_ptr, const int32_t *apert_gather, const int64_t *out_off,
                 const double *theta, int32_t w, double *s_out, double *stack_out, int32_t *m_out,
                 uint8_t *fragile, int nthreads)
{
    gset g = {samples, sample_off, trace_ptr, ns, half_offset, midpoint, central_x, dt};
    if (check_args(kind, &g, w, 1, 1, 1)) return 1;
    int64_t nrows;
    row_t *rows = make_rows(&g, njobs, job_central, &nrows);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int64_t r = 0; r < nrows; r++) {
        double U[64];
        double *Ub = (w <= 64) ? U : (double *)malloc(sizeof(double) * (size_t)w);
        const int j = rows[r].job, s = rows[r].s;
        const int64_t orow = out_off[j] + s;
        theta_t th = {theta[3 * orow + 0], theta[3 * orow + 1], theta[3 * orow + 2]};
        if (kind == ORACLE_CMP) th.A = th.B = 0.0;
        cell_t cl = eval_cell(&g, kind, job_central[j], apert_gather + apert_ptr[j],
                              apert_ptr[j + 1] - apert_ptr[j], s, th, w, Ub);
        s_out[orow] = cl.S;
        stack_out[orow] = cl.stack;
        if (m_out) m_out[orow] = cl.M;
        if (fragile) fragile[orow] = (uint8_t)cl.fragile;
        if (Ub != U) free(Ub);
    }
    free(rows);
    return 0;
}

/* Gathers corrected along each output row's parameter, for quality control:
 * the traces of a job's aperture read at the intersection of the row's
 * traveltime curve (CMP, section 2.1) or surface (CRS, section 2.2), by the
 * linear interpolation of Algorithm 1 with a one-sample window.  For job j,
 * aperture trace r (gathers as listed, traces in order) and output sample s:
 *   out[corr_off[j] + r * ns_c + s] = f[k] + x (f[k+1] - f[k]),
 * tau = sqrt(T(s dt, theta[out_off[j] + s])) / dt, k = floor(tau), x = tau - k,
 * and 0 where T < 0 or samples k and k+1 are not both on the trace (the
 * window rule with w = 1).  ns_c = samples of the central gather. */
int oracle_corrected(int kind, const float *samples, const int64_t *sample_off, const int32_t *trace_ptr,
                     const int32_t *ns, const float *half_offset, const float *midpoint,
                     const float *central_x, double dt, int32_t njobs, const int32_t *job_central,
                     const int32_t *apert_ptr, const int32_t *apert_gather, const int64_t *out_off,
                     const double *theta, const int64_t *corr_off, double *out, int nthreads)
{
    gset g = {samples, sample_off, trace_ptr, ns, half_offset, midpoint, central_x, dt};
    if (check_args(kind, &g, 1, 1, 1, 1)) return 1;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int j = 0; j < njobs; j++) {
        const int c = job_central[j];
        const int nsc = g.ns[c];
        const double xc = (kind == ORACLE_CRS) ? (double)g.central_x[c] : 0.0;
        int64_t r = 0;
        for (int p = apert_ptr[j]; p < apert_ptr[j + 1]; p++) {
            const int gg = apert_gather[p];
            const int nsg = g.ns[gg];
            for (int i = g.trace_ptr[gg]; i < g.trace_ptr[gg + 1]; i++, r++) {
                const float *f = g.samples + g.sample_off[gg] + (int64_t)(i - g.trace_ptr[gg]) * nsg;
                const double h = g.half_offset[i];
                const double dm = (kind == ORACLE_CRS) ? (double)g.midpoint[i] - xc : 0.0;
                double *o = out + corr_off[j] + r * nsc;
                for (int s = 0; s < nsc; s++) {
                    const int64_t row = out_off[j] + s;
                    theta_t th = {theta[3 * row + 0], theta[3 * row + 1], theta[3 * row + 2]};
                    if (kind == ORACLE_CMP) th.A = th.B = 0.0;
                    double mag;
                    const double T = traveltime_sq(kind, s * dt, th, dm, h, &mag);
                    double v = 0.0;
                    if (T >= 0.0) {
                        const double tau = sqrt(T) / dt;
                        if (window_on_trace(tau, 1, nsg)) {
                            const double kf = floor(tau);
                            const double frac = tau - kf;
                            const int64_t k = (int64_t)kf;
                            v = (double)f[k] + frac * ((double)f[k + 1] - (double)f[k]);
                        }
                    }
                    o[s] = v;
                }
            }
        }
    }
    return 0;
}

/*
 * Gradient of L = sum_rows g_s[row] * S(row, theta[row]) with respect to
 * theta (overwritten, [row][3] = dL/dA, dL/dB, dL/dq) and, if g_samples is
 * not NULL, with respect to every sample (ACCUMULATED into g_samples, same
 * layout as samples).
 *
 * With the contributing set and every window start a held fixed (they are
 * piecewise constant in theta and the samples):
 *   dS/dv_ij   = 2 (U_j - S M v_ij) / (M D)
 *   dv_ij/dtau = f[a+j+1] - f[a+j]            (slope of the segment used)
 *   dtau/dT    = 1 / (2 dt sqrt(T))
 *   dT/dA = 4 dm (t0 + 2 A dm),  dT/dB = 2 t0 dm^2,  dT/dq = h^2
 *   dv_ij/df[a+j] = 1 - x,  dv_ij/df[a+j+1] = x.
 * Rows with M = 0 or D = 0 (S identically 0) and traces with T = 0 (tau has
 * no derivative there) contribute nothing.
 *
 * Optional outputs for comparisons with an FP32 evaluation:
 *  - g_theta_mag [row][3], g_samples_mag (ACCUMULATED): the same sums with
 *    every term replaced by its magnitude and dS/dv_ij by its size before
 *    the subtraction cancels, 2 (sum_i |v_ij| + S M |v_ij|) / (M D); the
 *    weight 1 - x of a window's first sample enters as 1, the size of the
 *    rounding it inherits from x.  An evaluation whose every term carries a
 *    relative error e differs by at most about e times these;
 *  - rough [row]: 1 if the row's cell is a kink (a contributing intersection
 *    within KINK_TAU samples of an integer) or fragile (its contributing set
 *    could change, as in oracle_scan);
 *  - samples_rough: 1 on every sample a rough row's windows could read.
 */
int oracle_grad(int kind, const float *samples, const int64_t *sample_off, const int32_t *trace_ptr,
                const int32_t *ns, const float *half_offset, const float *midpoint,
                const float *central_x, double dt, int32_t njobs, const int32_t *job_central,
                const int32_t *apert_ptr, const int32_t *apert_gather, const int64_t *out_off,
                const double *theta, const double *g_s, int32_t w, double *g_theta,
                double *g_samples, double *g_theta_mag, double *g_samples_mag, uint8_t *rough,
                uint8_t *samples_rough, int nthreads)
{
    gset g = {samples, sample_off, trace_ptr, ns, half_offset, midpoint, central_x, dt};
    if (check_args(kind, &g, w, 1, 1, 1)) return 1;
    int64_t nrows;
    row_t *rows = make_rows(&g, njobs, job_central, &nrows);
    if (nthreads < 1) nthreads = 1;
    const int hw = (w - 1) / 2;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads)
    for (int64_t r = 0; r < nrows; r++) {
        double U[64];
        double *Ub = (w <= 64) ? U : (double *)malloc(sizeof(double) * (size_t)w);
        const int j = rows[r].job, s = rows[r].s;
        const int64_t orow = out_off[j] + s;
        const int c = job_central[j];
        const int32_t *ag = apert_gather + apert_ptr[j];
        const int na = apert_ptr[j + 1] - apert_ptr[j];
        theta_t th = {theta[3 * orow + 0], theta[3 * orow + 1], theta[3 * orow + 2]};
        if (kind == ORACLE_CMP) th.A = th.B = 0.0;
        double gA = 0.0, gB = 0.0, gq = 0.0;
        double mA = 0.0, mB = 0.0, mq = 0.0;
        cell_t cl = eval_cell(&g, kind, c, ag, na, s, th, w, Ub);
        const double gs = g_s[orow];
        const int is_rough = cl.kink || cl.fragile;
        if (rough) rough[orow] = (uint8_t)is_rough;
        const double t0 = s * dt;
        const double xc = (kind == ORACLE_CRS) ? (double)central_x[c] : 0.0;
        if (is_rough && samples_rough) {
            /* every sample a window of this row could read, on any trace whose
             * intersection exists, one sample of margin each side */
            for (int p = 0; p < na; p++) {
                const int gg = ag[p];
                const int nsg = ns[gg];
                for (int i = trace_ptr[gg]; i < trace_ptr[gg + 1]; i++) {
                    const int64_t base = sample_off[gg] + (int64_t)(i - trace_ptr[gg]) * nsg;
                    const double dm = (kind == ORACLE_CRS) ? (double)midpoint[i] - xc : 0.0;
                    double mag;
                    const double T = traveltime_sq(kind, t0, th, dm, half_offset[i], &mag);
                    if (T < -FRAGILE_T_REL * mag) continue;
                    const int64_t a = (int64_t)floor(sqrt(fmax(T, 0.0)) / dt) - hw;
                    for (int64_t n = a - 1; n <= a + w + 1; n++)
                        if (n >= 0 && n < nsg) samples_rough[base + n] = 1;
                }
            }
        }
        /* sum over contributing traces of |v_ij| per window sample j: the size
         * of U_j before any cancellation (for the magnitudes below) */
        double Ua[64];
        double *Uab = (w <= 64) ? Ua : (double *)malloc(sizeof(double) * (size_t)w);
        for (int jj = 0; jj < w; jj++) Uab[jj] = 0.0;
        if (g_theta_mag || g_samples_mag) {
            for (int p = 0; p < na; p++) {
                const int gg = ag[p];
                const int nsg = ns[gg];
                for (int i = trace_ptr[gg]; i < trace_ptr[gg + 1]; i++) {
                    const float *f = samples + sample_off[gg] + (int64_t)(i - trace_ptr[gg]) * nsg;
                    const double dm = (kind == ORACLE_CRS) ? (double)midpoint[i] - xc : 0.0;
                    double mag;
                    const double T = traveltime_sq(kind, t0, th, dm, half_offset[i], &mag);
                    if (T < 0.0) continue;
                    const double tau = sqrt(T) / dt;
                    if (!window_on_trace(tau, w, nsg)) continue;
                    const double kf = floor(tau);
                    const double x = tau - kf;
                    const int64_t a = (int64_t)kf - hw;
                    for (int jj = 0; jj < w; jj++)
                        Uab[jj] += fabs(f[a + jj] + x * ((double)f[a + jj + 1] - f[a + jj]));
                }
            }
        }
        if (cl.M > 0 && cl.D > 0.0 && gs != 0.0) {
            const double MD = (double)cl.M * cl.D;
            for (int p = 0; p < na; p++) {
                const int gg = ag[p];
                const int nsg = ns[gg];
                for (int i = trace_ptr[gg]; i < trace_ptr[gg + 1]; i++) {
                    const int64_t base = sample_off[gg] + (int64_t)(i - trace_ptr[gg]) * nsg;
                    const float *f = samples + base;
                    const double h = half_offset[i];
                    const double dm = (kind == ORACLE_CRS) ? (double)midpoint[i] - xc : 0.0;
                    double mag;
                    const double T = traveltime_sq(kind, t0, th, dm, h, &mag);
                    if (T < 0.0) continue;
                    const double tau = sqrt(T) / dt;
                    if (!window_on_trace(tau, w, nsg)) continue;
                    const double kf = floor(tau);
                    const double x = tau - kf;
                    const int64_t a = (int64_t)kf - hw;
                    double dS_dtau = 0.0, m_tau = 0.0;
                    for (int jj = 0; jj < w; jj++) {
                        const double f0 = f[a + jj], f1 = f[a + jj + 1];
                        const double v = f0 + x * (f1 - f0);
                        const double dS_dv = 2.0 * (Ub[jj] - cl.S * cl.M * v) / MD;
                        /* its size before the subtraction cancels */
                        const double m_dv = 2.0 * (Uab[jj] + cl.S * cl.M * fabs(v)) / MD;
                        dS_dtau += dS_dv * (f1 - f0);
                        m_tau += m_dv * fabs(f1 - f0);
                        if (g_samples) {
#pragma omp atomic
                            g_samples[base + a + jj] += gs * (1.0 - x) * dS_dv;
#pragma omp atomic
                            g_samples[base + a + jj + 1] += gs * x * dS_dv;
                        }
                        if (g_samples_mag) {
                            /* the weight 1 - x, formed from an x rounded to FP32,
                             * carries that rounding (of size x, not 1 - x): its
                             * magnitude is (1 - x) + x = 1 */
#pragma omp atomic
                            g_samples_mag[base + a + jj] += fabs(gs) * m_dv;
#pragma omp atomic
                            g_samples_mag[base + a + jj + 1] += fabs(gs) * x * m_dv;
                        }
                    }
                    if (T > 0.0) {
                        const double dtau_dT = 1.0 / (2.0 * dt * sqrt(T));
                        if (kind == ORACLE_CRS) {
                            gA += dS_dtau * dtau_dT * 4.0 * dm * (t0 + 2.0 * th.A * dm);
                            gB += dS_dtau * dtau_dT * 2.0 * t0 * dm * dm;
                            mA += m_tau * dtau_dT * 4.0 * fabs(dm) * (fabs(t0) + fabs(2.0 * th.A * dm));
                            mB += m_tau * dtau_dT * 2.0 * t0 * dm * dm;
                        }
                        gq += dS_dtau * dtau_dT * h * h;
                        mq += m_tau * dtau_dT * h * h;
                    }
                }
            }
        }
        g_theta[3 * orow + 0] = gs * gA;
        g_theta[3 * orow + 1] = gs * gB;
        g_theta[3 * orow + 2] = gs * gq;
        if (g_theta_mag) {
            g_theta_mag[3 * orow + 0] = fabs(gs) * mA;
            g_theta_mag[3 * orow + 1] = fabs(gs) * mB;
            g_theta_mag[3 * orow + 2] = fabs(gs) * mq;
        }
        if (Uab != Ua) free(Uab);
        if (Ub != U) free(Ub);
    }
    free(rows);
    return 0;
}

/* Number of OpenMP threads a parallel region would get (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
