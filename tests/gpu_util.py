"""Helpers for the GPU parity tests: run the HIP path through the C ABI on
host-generated inputs and compare its outputs with the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle

# The HIP kernels compute every intersection in FP64 with a Newton-refined
# square root (tau exact to ~1e-10 samples at tau ~ 2000), so the set of
# contributing traces can differ from the oracle's only for intersections
# within that distance of a window boundary: the oracle flags cells within
# 1e-8 samples (or 1e-13 of T) of one as fragile.
FRAGILE_TAU = 1e-8
FRAGILE_T_REL = 1e-13

# Tolerances:
S_TOL = 1e-5           # |S_gpu - S_oracle| on rows whose contributing set is not fragile
PICK_GAP = 1e-4        # picks must be identical where best and runner-up differ by more
STACK_TOL = 2e-5       # |stack_gpu - stack_oracle| relative to the row's sample scale

# Ill-conditioned cells.  The oracle returns per cell a condition number kappa
# (oracle.c, cell_cond): FP32 rounding of the samples, the interpolation and
# the window energies moves S by about 2^-24 kappa.  A cell whose K_COND *
# 2^-24 * kappa exceeds S_TOL is ill-conditioned -- it happens with one-sample
# windows (w = 1) next to zero crossings, where every interpolated value is
# small against the samples it comes from -- and is held to that bound
# instead; every other cell is held to S_TOL.
EPS32 = 2.0 ** -24
K_COND = 4.0


def s_bound(cond) -> np.ndarray:
    """Per-cell |dS| bound: S_TOL, or K_COND * 2^-24 * kappa where that is larger."""
    return np.maximum(S_TOL, K_COND * EPS32 * np.asarray(cond, np.float64))


def device_inputs(gs, jobs):
    import paper_1907_11678_amd as semb
    dg = semb.upload_gathers(gs.samples, gs.sample_off, gs.trace_ptr, gs.ns, gs.half_offset,
                             gs.midpoint, gs.central_x, gs.dt)
    dj = semb.upload_jobs(jobs.central, jobs.apert_ptr, jobs.apert_gather, jobs.out_off, jobs.n_out)
    return dg, dj


def run_scan(kind, gs, jobs, grid, w, panel=False, dg=None, dj=None):
    import torch
    import paper_1907_11678_amd as semb
    if dg is None:
        dg, dj = device_inputs(gs, jobs)
    n = jobs.n_out
    best = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    sb = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    st = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    npar = grid.n if kind == "crs" else grid.q.size
    pan = torch.full((n, npar), float("nan"), dtype=torch.float32, device="cuda") if panel else None
    ws = semb.alloc_workspace(dg.nsamples)
    q = torch.from_numpy(grid.q).cuda()
    if kind == "cmp":
        semb.cmp_scan(dg, dj, q, w, best, sb, st, ws, panel=pan)
    else:
        semb.crs_scan(dg, dj, torch.from_numpy(grid.A).cuda(), torch.from_numpy(grid.B).cuda(), q, w,
                      best, sb, st, ws, panel=pan)
    torch.cuda.synchronize()
    return (best.cpu().numpy(), sb.cpu().numpy().astype(np.float64),
            st.cpu().numpy().astype(np.float64),
            None if pan is None else pan.cpu().numpy().astype(np.float64))


def sample_scale(gs, jobs):
    """Per output row: max |sample| over the job's aperture (stack tolerance scale)."""
    out = np.zeros(jobs.n_out)
    for j in range(jobs.njobs):
        m = 0.0
        for g in jobs.apert_gather[jobs.apert_ptr[j]:jobs.apert_ptr[j + 1]]:
            gg = gs.gather(int(g))
            if gg.size:
                m = max(m, float(np.abs(gg).max()))
        c = int(jobs.central[j])
        out[jobs.out_off[j]:jobs.out_off[j] + int(gs.ns[c])] = m
    return out


def compare(name, gpu, ref, scale=None, rows=None):
    """Assert parity of (best, s_best, stack[, panel]) against an oracle result.
    rows: optional output-row indices the oracle result refers to."""
    best, sb, st, pan = gpu
    if rows is not None:
        best, sb, st = best[rows], sb[rows], st[rows]
        if scale is not None:
            scale = scale[rows]
    ok = ~ref.fragile
    assert np.isfinite(sb).all() and (best >= 0).all(), f"{name}: unwritten outputs"
    # Where the two picks differ, the largest S of one panel differs from the
    # largest of the other by at most the larger of the two picked cells'
    # errors (the maximum is 1-Lipschitz), so the row is held to the larger
    # of their bounds; without the oracle's panel only its own pick is known.
    cond = ref.cond
    if ref.panel_cond is not None:
        r_ = np.arange(best.size)
        cond = np.maximum(cond, ref.panel_cond[r_, np.clip(best, 0, ref.panel_cond.shape[1] - 1)])
    bound = s_bound(cond)[ok]
    dS = np.abs(sb - ref.s_best)[ok]
    worst = float(dS.max()) if dS.size else 0.0
    excess = dS > bound
    assert not excess.any(), (f"{name}: |dS| at the pick {float(dS[excess].max()):.3g} above its bound "
                              f"on {int(excess.sum())} rows")
    ill = int((bound > S_TOL).sum())
    sure = ok & (ref.gap > PICK_GAP)
    nbad = int((best[sure] != ref.best[sure]).sum())
    assert nbad == 0, f"{name}: {nbad} of {int(sure.sum())} decisive picks differ"
    same = ok & (best == ref.best)
    sc = np.maximum(scale if scale is not None else 1.0, 1e-30)
    dst = (np.abs(st - ref.stack) / sc)[same] if np.ndim(sc) else np.abs(st - ref.stack)[same] / sc
    wst = float(dst.max()) if dst.size else 0.0
    assert wst <= STACK_TOL, f"{name}: max relative |d stack| {wst:.3g} > {STACK_TOL}"
    if pan is not None and ref.panel is not None:
        assert np.isfinite(pan).all(), f"{name}: panel not fully written"
        dP = np.abs(pan - ref.panel)[ok]
        pb = s_bound(ref.panel_cond)[ok]
        over = dP > pb
        assert not over.any(), (f"{name}: |dS| over the panel {float(dP[over].max()):.3g} above its bound "
                                f"on {int(over.sum())} cells")
        ill += int((pb > S_TOL).sum())
        cond_ratio = dP[pb > S_TOL] / (EPS32 * ref.panel_cond[ok][pb > S_TOL])
        worst_ratio = float(cond_ratio.max()) if cond_ratio.size else 0.0
    else:
        worst_ratio = None
    return {"rows": int(ref.s_best.size), "fragile": int((~ok).sum()), "max_dS": worst,
            "decisive": int(sure.sum()), "max_dstack": wst, "ill_conditioned": ill,
            "max_dS_over_eps_kappa_ill": worst_ratio}


# Gradients.  The kernels form dS/dtheta and dS/dsample in FP32 from the same
# terms as the oracle (oracle.c, oracle_grad), and the sums cancel heavily near
# a maximum of S.  The oracle also returns, per row and per sample, the same
# sums with every term replaced by its magnitude ("mag"); an evaluation whose
# terms each carry a few FP32 roundings, summed over an aperture's traces,
# differs from the exact sums by a small multiple of 2^-24 * mag.  Every row
# and every sample is held to K_GRAD * 2^-24 * mag, except rows the oracle
# flags as rough (an intersection within FRAGILE_TAU samples of an integer or
# of a validity boundary, where the derivative jumps) and the samples their
# windows read.
K_GRAD = 64.0


def assert_grad_parity(name, kind, gs, jobs, theta, g_s, w, g_theta, g_samples=None):
    """g_theta [n_out, 3] and g_samples (or None) from the GPU, for
    L = sum g_s * S(theta), against the oracle's FP64 gradient."""
    oracle.set_kink(FRAGILE_TAU)
    try:
        gt_ref, gsm_ref, d = oracle.grad(kind, gs, jobs, np.asarray(theta, np.float64),
                                         np.asarray(g_s, np.float64), w, detail=True)
    finally:
        oracle.set_kink(oracle.KINK_DEFAULT)
    smooth = ~d.rough
    out = {"rows": int(smooth.size), "rough": int(d.rough.sum())}
    comps = [2] if kind in ("cmp", 0) else [0, 1, 2]
    for k in comps:
        err = np.abs(g_theta[:, k] - gt_ref[:, k])[smooth]
        mag = d.g_theta_mag[smooth, k]
        bound = K_GRAD * EPS32 * mag
        over = err > bound
        assert not over.any(), (f"{name}: dS/dtheta[{k}] above K_GRAD 2^-24 mag on {int(over.sum())} rows; "
                                f"worst ratio {float((err / np.maximum(EPS32 * mag, 1e-300)).max()):.3g}")
        live = mag > 0
        out[f"max_ratio_{k}"] = float((err[live] / (EPS32 * mag[live])).max()) if live.any() else 0.0
        out[f"median_rel_{k}"] = float(np.median(err[live] / np.maximum(np.abs(gt_ref[smooth, k][live]),
                                                                          1e-300))) if live.any() else 0.0
    if g_samples is not None:
        keep = ~d.samples_rough
        err = np.abs(g_samples - gsm_ref)[keep]
        mag = d.g_samples_mag[keep]
        over = err > K_GRAD * EPS32 * mag
        assert not over.any(), (f"{name}: dS/dsample above K_GRAD 2^-24 mag on {int(over.sum())} samples; "
                                f"worst ratio {float((err / np.maximum(EPS32 * mag, 1e-300)).max()):.3g}")
        live = mag > 0
        out["samples_checked"] = int(keep.sum())
        out["max_ratio_samples"] = float((err[live] / (EPS32 * mag[live])).max()) if live.any() else 0.0
    return out
