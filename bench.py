#!/usr/bin/env python3
"""Throughput of the D3Q27 central-moment collide-stream update on one MI355X.

Workload: 256^3 periodic decaying turbulence (seeded solenoidal field with a
k^-5/3 spectrum over k = 2..32, u_rms = 0.04 per component, rho = 1),
nu = 1e-5, adaptive relaxation on, FP32 shifted populations.  A step is one
fused pull-stream + collide launch over all cells.  Inputs are resident in
HBM before the timed region starts.

Prints ONE JSON line: MLUPS, the HBM roofline of the collide-stream kernel
(algorithmic bytes per launch / average launch time from HIP events on the
stream the kernels run on), the FP16-storage variant on the same workload,
and the FP64 CPU oracle timed on a bounded slab of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q27 MLUPS + % HBM roofline; FP16-store and adjoint vs FP32 plain step"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {"f32": 216, "f16s": 108}   # 27 reads + 27 writes per update
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_traffic.json")
REPS = 5          # timed windows per measurement; the median is reported
STEP_KERNEL_SOURCES = ("step.hip", "brick.hpp", "cm_collide.hpp", "internal.hpp", "lattice.hpp",
                       "wall.hpp")


def kernel_source_hash() -> str:
    """Hash of the sources that make up the collide-stream kernel (the
    kernel the counter file describes); other kernels do not change it."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1807_02284_amd", "csrc")
    for name in STEP_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, n: int):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = rec.get(f"{storage}_{n}")
    if not entry or rec.get("source_hash") != kernel_source_hash():
        return None
    return entry.get("bytes_per_launch")


def timed_windows(enqueue, reps: int = REPS):
    """Durations (ms) of `reps` consecutive windows of GPU work on the stream
    the library launches on (torch's current stream): a device
    synchronisation, an event, then per window `enqueue()` (one window of
    work) followed by an event, and a synchronisation at the end.  The
    windows run back to back, so none but the first starts from an idle
    GPU; the median over them is reported."""
    import torch
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for r in range(reps):
        enqueue()
        ev[r + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[r].elapsed_time(ev[r + 1]) for r in range(reps)]


def per_unit(windows, units: int):
    """Median window time per unit of work (step, launch, reference step)
    and the spread over the windows."""
    return statistics.median(windows) / units, {
        "repetitions": len(windows), "statistic": "median",
        "min": min(windows) / units, "max": max(windows) / units}


def time_steps(lev, steps: int, warmup: int, reps: int = REPS):
    """`warmup` untimed steps, then `reps` timed windows of `steps` steps
    (one C call each: `steps` kernel launches on the current stream).
    Returns (median ms per step, spread)."""
    lev.step(warmup)
    return per_unit(timed_windows(lambda: lev.step(steps), reps), steps)


def kinetic_energy(lev) -> float:
    """E = sum over cells of rho |u|^2 / 2 of the stored state (FP64 sum)."""
    rho, u, _ = lev.read_macro()
    return float(0.5 * (rho.double() * (u.double() ** 2).sum(0)).sum())


def run_gpu(n: int, storage: str, steps: int, warmup: int):
    import numpy as np
    import torch
    from paper_1807_02284_amd import inputs
    from paper_1807_02284_amd.level import F16S, F32, Level, Params

    rho, u = inputs.turbulence(n, 2, 32, 0.04, seed=1807)
    p = Params(nu=1e-5, g_max=0.1, adaptive=True)
    lev = Level(n, n, n, p, storage=F32 if storage == "f32" else F16S)
    lev.init_equilibrium(rho, u)
    c0 = lev.conserved()
    e0 = kinetic_energy(lev)
    ms_step, spread = time_steps(lev, steps, warmup)
    c1 = lev.conserved()
    e1 = kinetic_energy(lev)
    bad = lev.count_nonfinite()
    cells = n ** 3
    mlups = cells / (ms_step * 1e-3) / 1e6
    bytes_launch = cells * BYTES_PER_LUP[storage]
    achieved = bytes_launch / (ms_step * 1e-3) / 1e9
    out = {
        "ms_per_step": ms_step,
        "timing": spread,
        "mlups": mlups,
        "achieved_gbs": achieved,
        "bytes_per_launch": bytes_launch,
        "mass_drift_rel": abs(c1[0] - c0[0]) / c0[0],
        "momentum_drift_abs": float(np.max(np.abs(c1[1:4] - c0[1:4]))),
        "kinetic_energy_ratio": e1 / e0,
        "nonfinite": bad,
    }
    del lev
    torch.cuda.empty_cache()
    return out


def run_precision(n: int, steps: int, ref_slice=None):
    """Taylor-Green (2D vortex extruded in z, u0 = 0.05, tau = 0.6, adaptive
    on) at n^3: FP16 storage against FP32 storage after `steps` steps, both
    against the closed-form decay and, when `ref_slice` (the FP64 oracle's
    velocity [3][n*n] of one z-slice after the same steps; the field does
    not vary along z) is given, against the FP64 oracle; MLUPS of both."""
    import numpy as np
    import torch
    from paper_1807_02284_amd import inputs
    from paper_1807_02284_amd.level import F16S, F32, Level, Params

    rho, u = inputs.taylor_green_2d(n, n, n, 0.05)
    p = Params(nu=0.1 / 3.0, g_max=0.1)
    out = {}
    fields = {}
    for name, st in (("f32", F32), ("f16s", F16S)):
        lev = Level(n, n, n, p, storage=st)
        lev.init_equilibrium(rho, u)
        assert steps % REPS == 0
        ms, spread = time_steps(lev, steps // REPS, 0)      # exactly `steps` steps in all
        _, ug, _ = lev.read_macro()
        fields[name] = ug.double()
        out[name] = {"ms_per_step": ms, "timing": spread, "mlups": n ** 3 / (ms * 1e-3) / 1e6,
                     "achieved_gbs": n ** 3 * BYTES_PER_LUP[name] / (ms * 1e-3) / 1e9}
        del lev
        torch.cuda.empty_cache()

    def vort(uu):
        U = uu.reshape(3, n, n, n)          # [comp, z, y, x]
        def d(a, axis):
            return (torch.roll(a, -1, axis) - torch.roll(a, 1, axis)) / 2
        return torch.stack([d(U[2], 1) - d(U[1], 0), d(U[0], 0) - d(U[2], 2), d(U[1], 2) - d(U[0], 1)])

    k = 2 * np.pi / n
    amp = np.exp(-2 * (0.1 / 3.0) * k * k * steps)
    exact = torch.tensor(u * amp, device=fields["f32"].device)
    rl2 = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    out["f16s_vs_f32_velocity_rel_l2"] = rl2(fields["f16s"], fields["f32"])
    out["f16s_vs_f32_vorticity_rel_l2"] = rl2(vort(fields["f16s"]), vort(fields["f32"]))
    out["f32_vs_closed_form_velocity_rel_l2"] = rl2(fields["f32"], exact)
    out["f16s_vs_closed_form_velocity_rel_l2"] = rl2(fields["f16s"], exact)
    # amplitude of the vortex mode (projection; filters the acoustic waves of
    # the uniform-density start) against the closed-form decay
    u0 = torch.tensor(u, device=fields["f32"].device)
    for name in ("f32", "f16s"):
        a = float((fields[name] * u0).sum() / (u0 * u0).sum())
        out[f"{name}_mode_amplitude_rel_err"] = abs(a - amp) / amp
    if ref_slice is not None:
        ref = torch.tensor(ref_slice, dtype=torch.float64, device=fields["f32"].device)
        ref = ref.reshape(3, 1, n * n).expand(3, n, n * n).reshape(3, n ** 3)
        wref = vort(ref)
        for name in ("f32", "f16s"):
            out[f"{name}_vs_fp64_oracle_velocity_rel_l2"] = rl2(fields[name], ref)
            out[f"{name}_vs_fp64_oracle_vorticity_rel_l2"] = rl2(vort(fields[name]), wref)
        out["fp64_oracle"] = (f"{n}x{n}x1 periodic slice, {steps} steps; the extruded vortex "
                              "does not vary along z, so it equals every z-slice of the 3D run")
    return out


def oracle_tgv_slice(n: int, steps: int):
    """FP64 oracle velocity [3][n*n] of the extruded Taylor-Green vortex after
    `steps` steps, on one periodic z-slice (n x n x 1: the pull from z +- 1
    wraps onto the slice itself, which is exact for a field constant in z)."""
    import oracle
    from paper_1807_02284_amd import inputs

    rho, u = inputs.taylor_green_2d(n, n, 1, 0.05)
    dom = oracle.Domain(n, n, 1)
    p = oracle.Params(nu=0.1 / 3.0, g_max=0.1)
    f, _ = oracle.init(dom, rho, u)
    f, _ = oracle.step(dom, p, f, n_steps=steps)
    _, uo, _ = oracle.macro(dom, p, f)
    return uo


def run_adjoint(n: int, steps: int, every: int):
    """Differentiable buoyant smoke at n^3 (periodic; blob sigma = n/16 at
    (n/2, n/2, n/4); beta = 1e-4, s_ref = initial mean): the target is the
    final smoke scalar of a seeded target run (the same scene driven by a
    seeded smooth random body force of amplitude 1e-5); the differentiated
    run starts from theta = 0, goes forward `steps` steps keeping every
    `every`-th state, then the checkpointed backward (recompute + adjoint)
    gives dL/dtheta of L = 1/2 sum (s - s_target)^2.  Reports ms per step of
    the plain forward step and of the adjoint kernel."""
    import numpy as np
    import torch
    from paper_1807_02284_amd import inputs
    from paper_1807_02284_amd.level import Level, Params
    from paper_1807_02284_amd.rollout import rollout

    s0 = inputs.gaussian_blob(n, n, n, (n / 2, n / 2, n / 4), n / 16.0)
    p = Params(nu=1e-3, g_max=0.1, tau_s=0.51, beta=1e-4, s_ref=float(s0.mean()))
    theta_target = inputs.smooth_random_field(n, n, n, 1e-5, 1835, k_max=4)
    lev = Level(n, n, n, p, scalar=True, force=theta_target)
    lev.init_equilibrium(None, np.zeros((3, n ** 3)), s0)
    h0, g0 = lev.get_populations(shifted=True)
    h0, g0 = h0.clone(), g0.clone()
    lev.step(steps)                              # the seeded target run
    _, _, target = lev.read_macro()
    target = target.clone()
    theta = torch.zeros(3, n ** 3, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    s = rollout(lev, theta, h0, g0, steps, every)
    e[1].record()
    loss = 0.5 * ((s - target) ** 2).sum()
    loss.backward()
    e[2].record()
    torch.cuda.synchronize()
    fwd_ms, bwd_ms = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    # adjoint kernel alone, timed on the same state
    lam = torch.zeros(27 * lev.plane, device="cuda")
    lam2 = torch.zeros_like(lam)
    mu = torch.zeros(7 * lev.plane, device="cuda")
    mu2 = torch.zeros_like(mu)
    dth = torch.zeros(3 * lev.plane, device="cuda")
    for _ in range(3):
        lev.adjoint_step(lev.f, lev.g, lam, mu, lam2, mu2, dth)
    reps = 20

    def adjoint_window():
        for _ in range(reps):
            lev.adjoint_step(lev.f, lev.g, lam, mu, lam2, mu2, dth)

    adj_ms, adj_spread = per_unit(timed_windows(adjoint_window), reps)
    step_ms, step_spread = time_steps(lev, reps, 2)
    cells = n ** 3
    out = {
        "forward_ms_per_step": fwd_ms / steps,
        "backward_ms_per_step": bwd_ms / steps,
        "plain_step_ms": step_ms,
        "plain_step_timing": step_spread,
        "adjoint_kernel_ms": adj_ms,
        "adjoint_kernel_timing": adj_spread,
        "adjoint_vs_plain_step_time": adj_ms / step_ms,
        "backward_vs_forward_time": bwd_ms / fwd_ms,
        "adjoint_mlups": cells / (adj_ms * 1e-3) / 1e6,
        "adjoint_achieved_gbs": cells * 444 / (adj_ms * 1e-3) / 1e9,
        "plain_step_achieved_gbs": cells * 284 / (step_ms * 1e-3) / 1e9,
        "bytes_per_lup": {"plain_step_scalar_force": 284, "adjoint": 444},
        "target": "final smoke scalar of a run driven by a seeded smooth random force "
                  "(amplitude 1e-5, seed 1835)",
        "loss": float(loss.detach()),
        "grad_theta_norm": float(theta.grad.norm()),
    }
    del lev
    torch.cuda.empty_cache()
    return out


def run_plume(nx: int, ny: int, nz: int, spinup: int, n_ref: int):
    """Multi-scale smoke plume: nx*ny*nz reference box, bounce-back walls,
    inflow u = 0.05 with smoke s = 1 at a disk on the x = 0 face, outflow at
    x = nx-1, solid sphere of radius 24 (scaled); passive FP32 scalar; nu0 =
    1e-4 (tau0 = 0.5003), tau_s0 = 0.51.  The jet cylinder starts at
    u = 0.05.  After `spinup` reference-scale steps, two finer scales
    (spacing ratios 1.5 and 2) are placed on the vorticity thresholds 2e-3
    and 8e-3 (with speed thresholds 0.01 and 0.02), then `n_ref` reference
    steps of Algorithm 1 are timed."""
    import numpy as np
    import torch
    from paper_1807_02284_amd import hierarchy, inputs
    from paper_1807_02284_amd.level import Level, Params

    sc = nx / 512.0
    flags = inputs.plume_flags(nx, ny, nz)
    p0 = Params(nu=1e-4, g_max=0.1, tau_s=0.51, u_in=(0.05, 0.0, 0.0), s_in=1.0)
    lev0 = Level(nx, ny, nz, p0, scalar=True, periodic=0, flags=flags)
    x, y, z = inputs.grid_coords(nx, ny, nz)
    jet = ((y + 0.5 - ny / 2) ** 2 + (z + 0.5 - nz / 2) ** 2 <= (32 * sc) ** 2) & (flags == 0)
    u = np.zeros((3, x.size), np.float32)
    u[0, jet] = 0.05
    s0 = np.where(jet & (x < 64 * sc), 1.0, 0.0).astype(np.float32)
    lev0.init_equilibrium(None, u, s0)
    del x, y, z, u, s0, jet
    # reference-scale collide-stream alone (flags + scalar: 273 B/LUP), over
    # the spin-up: REPS windows of spinup / REPS steps
    ms0, spread0 = time_steps(lev0, spinup // REPS, 10)
    n0 = nx * ny * nz
    centre = (160.0 * sc, ny / 2.0, nz / 2.0)
    r = 24.0 * sc

    def sphere(px, py, pz):
        return (px + 0.5 - centre[0]) ** 2 + (py + 0.5 - centre[1]) ** 2 + (pz + 0.5 - centre[2]) ** 2 <= r * r

    H, boxes = hierarchy.dynamic_hierarchy(lev0, flags, ((2e-3, 0.01), (8e-3, 0.02)), (1.5, 2.0),
                                           solid_fn=sphere)
    alphas = [1.0] + [1.0 / lv.c.dx for lv in H.levels[1:]]
    # sub-steps per reference step: l = floor(alpha) + 1 (Algorithm 1); at
    # integer alpha the last one has weight 0 in the time interpolation and
    # the driver does not compute it, so it is not counted either
    literal = [1] + [int(np.floor(a + 1e-12)) + 1 for a in alphas[1:]]
    subs = [1] + [k - 1 if (k - 1) / a == 1.0 else k for k, a in zip(literal[1:], alphas[1:])]
    cells = [lv.n for lv in H.levels]
    lups = sum(c * k for c, k in zip(cells, subs))
    H.step(2)
    win = max(1, n_ref // REPS)
    ms, spread = per_unit(timed_windows(lambda: H.step(win)), win)
    # adjoint of one reference step (forward recompute into the workspace,
    # then the reverse schedule) from the current states, arbitrary adjoints
    ws = torch.empty(H.adjoint_workspace_bytes(), dtype=torch.uint8, device="cuda")
    f_in = [lv.f.clone() for lv in H.levels]
    g_in = [lv.g.clone() for lv in H.levels]
    gen = torch.Generator(device="cuda").manual_seed(11)
    lam = [1e-3 * torch.randn(27 * lv.plane, device="cuda", generator=gen) for lv in H.levels]
    mu = [1e-3 * torch.randn(7 * lv.plane, device="cuda", generator=gen) for lv in H.levels]
    H.adjoint_step(f_in, g_in, lam, mu, ws)
    adj_ms, adj_spread = per_unit(timed_windows(lambda: H.adjoint_step(f_in, g_in, lam, mu, ws)), 1)
    adj_finite = bool(all(torch.isfinite(x).all() for x in lam + mu))
    ws_gb = ws.numel() / 1e9
    del ws, f_in, g_in, lam, mu
    torch.cuda.empty_cache()
    # the dynamic construction repeats every 40 reference steps: rebuild the
    # regions from the current flow (new cells mapped from the parent,
    # shared cells kept), timed on its own (host construction + GPU fill)
    t0 = time.perf_counter()
    H, boxes2 = hierarchy.dynamic_hierarchy(lev0, flags, ((2e-3, 0.01), (8e-3, 0.02)), (1.5, 2.0),
                                            solid_fn=sphere, previous=H)
    rebuild_s = time.perf_counter() - t0
    H.step(2)
    torch.cuda.synchronize()
    bad = sum(lv.count_nonfinite() for lv in H.levels)
    n_scales = len(H.levels)
    del H
    torch.cuda.empty_cache()
    # the same thresholds with the finer scales stored in 8x8x8 bricks of
    # their regions instead of the regions' bounding boxes
    Hb, _ = hierarchy.dynamic_hierarchy(lev0, flags, ((2e-3, 0.01), (8e-3, 0.02)), (1.5, 2.0),
                                        solid_fn=sphere, bricks=True)
    cells_b = [lv.n for lv in Hb.levels]
    subs_b = subs[: len(cells_b)]
    Hb.step(2)
    ms_b, spread_b = per_unit(timed_windows(lambda: Hb.step(win)), win)
    bad_b = sum(lv.count_nonfinite() for lv in Hb.levels)
    lups_b = sum(c * k for c, k in zip(cells_b, subs_b))
    # the brick regions rebuilt from the current flow, timed like the boxes'
    t0 = time.perf_counter()
    Hb2, _ = hierarchy.dynamic_hierarchy(lev0, flags, ((2e-3, 0.01), (8e-3, 0.02)), (1.5, 2.0),
                                         solid_fn=sphere, bricks=True, previous=Hb)
    rebuild_b = time.perf_counter() - t0
    del Hb, Hb2
    torch.cuda.empty_cache()
    out = {
        "reference_box": [nx, ny, nz],
        "scales": n_scales,
        "spacing_ratios": alphas,
        "cells_per_scale": cells,
        "substeps_per_scale": subs,
        "substeps_per_scale_algorithm": literal,
        "boxes_level0_units": [[list(map(int, lo)), list(map(int, hi))] for lo, hi in boxes],
        "coverage_of_reference_volume": [
            float(np.prod([hi[a] - lo[a] + 1 for a in range(3)]) / n0) for lo, hi in boxes],
        "ms_per_reference_step": ms,
        "timing": spread,
        "region_rebuild_s": rebuild_s,
        "boxes_after_rebuild_level0_units": [[list(map(int, lo)), list(map(int, hi))]
                                             for lo, hi in boxes2],
        "ms_per_reference_step_with_rebuild_every_40": ms + rebuild_s * 1e3 / 40,
        "lattice_updates_per_reference_step": lups,
        "mlups_all_scales": lups / (ms * 1e-3) / 1e6,
        "adjoint_ms_per_reference_step": adj_ms,
        "adjoint_timing": adj_spread,
        "adjoint_vs_forward_reference_step": adj_ms / ms,
        "adjoint_workspace_gb": ws_gb,
        "adjoint_finite": adj_finite,
        "reference_scale_step_ms": ms0,
        "reference_scale_timing": spread0,
        "reference_scale_mlups": n0 / (ms0 * 1e-3) / 1e6,
        "reference_scale_achieved_gbs": n0 * 273 / (ms0 * 1e-3) / 1e9,
        "bytes_per_lup_collide_stream": 273,
        "nonfinite": bad,
        "bricks": {"cells_per_scale": cells_b, "ms_per_reference_step": ms_b, "timing": spread_b,
                   "lattice_updates_per_reference_step": lups_b,
                   "mlups_all_scales": lups_b / (ms_b * 1e-3) / 1e6,
                   "speedup_vs_boxes": ms / ms_b, "region_rebuild_s": rebuild_b,
                   "ms_per_reference_step_with_rebuild_every_40": ms_b + rebuild_b * 1e3 / 40,
                   "nonfinite": bad_b},
    }
    del lev0
    torch.cuda.empty_cache()
    return out


def run_gradient_mode(n: int, steps: int, compare_steps: int):
    """The 256^3 turbulence workload with the adaptive factor driven by the
    finite-difference |grad u|_F of the stored velocity (grad_mode 1, one
    step lagged; +24 B/LUP for the velocity field) instead of the local
    strain-rate estimate: MLUPS, and after `compare_steps` steps from the
    same start the velocity-field and kinetic-energy differences between
    the two modes."""
    import numpy as np
    import torch
    from paper_1807_02284_amd import inputs
    from paper_1807_02284_amd.level import Level, Params

    rho, u = inputs.turbulence(n, 2, 32, 0.04, seed=1807)
    fields = {}
    out = {}
    for mode in (1, 0):
        lev = Level(n, n, n, Params(nu=1e-5, g_max=0.1, adaptive=True, grad_mode=mode))
        lev.init_equilibrium(rho, u)
        if mode == 1:
            ms, spread = time_steps(lev, steps // REPS, 10)
            out["ms_per_step"] = ms
            out["timing"] = spread
            out["mlups"] = n ** 3 / (ms * 1e-3) / 1e6
            out["achieved_gbs"] = n ** 3 * 240 / (ms * 1e-3) / 1e9
            lev.init_equilibrium(rho, u)
        lev.step(compare_steps)
        _, ug, _ = lev.read_macro()
        torch.cuda.synchronize()
        fields[mode] = ug.double()
        del lev
        torch.cuda.empty_cache()
    # the running-maximum option: the field maximum is reduced before each step
    lev = Level(n, n, n, Params(nu=1e-5, g_max=0.1, adaptive=True, grad_mode=1, gmax_running=True))
    lev.init_equilibrium(rho, u)
    ms, spread = time_steps(lev, steps // REPS, 10)
    out["running_max_ms_per_step"] = ms
    out["running_max_timing"] = spread
    out["running_max_mlups"] = n ** 3 / (ms * 1e-3) / 1e6
    out["running_max_last_gmax"] = float(lev.gmax_buf[-1])
    del lev
    torch.cuda.empty_cache()
    d = fields[1] - fields[0]
    out["bytes_per_lup"] = 240
    out["compare_steps"] = compare_steps
    out["velocity_rel_l2_fd_vs_local"] = float(torch.linalg.norm(d) / torch.linalg.norm(fields[0]))
    e1, e0 = float((fields[1] ** 2).sum()), float((fields[0] ** 2).sum())
    out["kinetic_energy_ratio_fd_vs_local"] = e1 / e0
    out["kinetic_energy_decay_local"] = e0 / float(np.sum(u.astype(np.float64) ** 2))
    return out


def run_far_field(nx: int, ny: int, nz: int, pad: int, spinup: int, n_ref: int):
    """Open jet with a far field: the plume's reference box (inflow disk on
    the x = 0 face, solid sphere, FP32 scalar, nu0 = 1e-4, tau_s0 = 0.51)
    with its walls and outflow plane replaced by a ghost shell, inside a
    far-field scale of spacing 2 (alpha_c = 0.5) that reaches `pad`
    reference cells beyond the box on every side and has Neumann faces.
    `spinup` reference steps, then `n_ref` timed reference steps of the
    two-scale schedule."""
    import numpy as np
    import torch
    from paper_1807_02284_amd import _capi, hierarchy, inputs
    from paper_1807_02284_amd.level import Level, Params

    sc = nx / 512.0
    x, y, z = inputs.grid_coords(nx, ny, nz)
    kinds = hierarchy.shell_flags(nx, ny, nz)
    disk = (x == 0) & ((y + 0.5 - ny / 2) ** 2 + (z + 0.5 - nz / 2) ** 2 <= (32 * sc) ** 2)
    kinds[disk & (y > 0) & (y < ny - 1) & (z > 0) & (z < nz - 1)] = _capi.INLET
    r = 24.0 * sc
    centre = (160.0 * sc, ny / 2.0, nz / 2.0)

    def sphere(px, py, pz):
        return (px + 0.5 - centre[0]) ** 2 + (py + 0.5 - centre[1]) ** 2 + (pz + 0.5 - centre[2]) ** 2 <= r * r

    kinds[sphere(x, y, z)] = _capi.SOLID
    p0 = Params(nu=1e-4, g_max=0.1, tau_s=0.51, u_in=(0.05, 0.0, 0.0), s_in=1.0)
    lev0 = Level(nx, ny, nz, p0, scalar=True, periodic=0, flags=kinds)
    jet = ((y + 0.5 - ny / 2) ** 2 + (z + 0.5 - nz / 2) ** 2 <= (32 * sc) ** 2) & (kinds == 0)
    u = np.zeros((3, x.size), np.float32)
    u[0, jet] = 0.05
    s0 = np.where(jet & (x < 64 * sc), 1.0, 0.0).astype(np.float32)
    lev0.init_equilibrium(None, u, s0)
    del x, y, z, u, s0, jet
    dxc = 2.0
    shape_c = tuple(int(np.ceil((m - 1 + 2 * pad) / dxc)) + 1 for m in (nx, ny, nz))
    origin_c = (-float(pad),) * 3
    far, kinds_c = hierarchy.far_field_scale(lev0, kinds, dxc, origin_c, shape_c, solid_fn=sphere)
    far.init_equilibrium(None, np.zeros((3, far.n), np.float32), np.zeros(far.n, np.float32))
    H = hierarchy.Hierarchy([lev0, far], [kinds, kinds_c])
    H.step(spinup)
    win = max(1, n_ref // REPS)
    ms, spread = per_unit(timed_windows(lambda: H.step(win)), win)
    # the reference scale alone (flags + scalar), for the share of the exchange
    ms0, spread0 = time_steps(lev0, 20, 2)
    cells = [lev0.n, far.n]
    bad = lev0.count_nonfinite() + far.count_nonfinite()
    out = {
        "reference_box": [nx, ny, nz],
        "far_field_shape": list(shape_c),
        "far_field_spacing": dxc,
        "far_field_shared_cells": int(np.count_nonzero(kinds_c == _capi.GHOST)),
        "reference_shell_cells": int(np.count_nonzero(kinds == _capi.GHOST)),
        "cells_per_scale": cells,
        "ms_per_reference_step": ms,
        "timing": spread,
        "mlups_all_scales": sum(cells) / (ms * 1e-3) / 1e6,
        "reference_scale_step_ms": ms0,
        "reference_scale_timing": spread0,
        "nonfinite": int(bad),
    }
    del H, lev0, far
    torch.cuda.empty_cache()
    return out


def cpu_baseline(n: int, target_s: float = 12.0):
    """The FP64 oracle (as is) on a bounded sample of the workload: a periodic
    n x n x nz_s slab cut from the same seeded turbulence field, one or more
    steps, about target_s seconds of wall clock."""
    import numpy as np
    import oracle
    from paper_1807_02284_amd import inputs

    nz_s = 4
    rho, u = inputs.turbulence(n, 2, 32, 0.04, seed=1807)
    cut = n * n * nz_s
    dom = oracle.Domain(n, n, nz_s)
    p = oracle.Params(nu=1e-5, g_max=0.1, adaptive=True)
    f, _ = oracle.init(dom, rho[:cut], np.ascontiguousarray(u[:, :cut]))
    steps, elapsed = 0, 0.0
    while elapsed < target_s and steps < 400:
        t0 = time.perf_counter()
        f, _ = oracle.step(dom, p, f)
        elapsed += time.perf_counter() - t0
        steps += 1
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": cut * steps / elapsed / 1e6,
        "unit": "MLUPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{steps} step(s) of a periodic {n}x{n}x{nz_s} slab of the {n}^3 turbulence "
                  f"field ({cut} cells), FP64, LU back-transform per cell; {elapsed:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 384^3 FP16-vs-FP32 Taylor-Green variant")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the 128^3 differentiable buoyant-smoke variant")
    ap.add_argument("--no-plume", action="store_true",
                    help="skip the 512x256x256 three-scale plume variant")
    ap.add_argument("--no-gradient-mode", action="store_true",
                    help="skip the finite-difference gradient-mode variant")
    ap.add_argument("--plume-spinup", type=int, default=300,
                    help="reference-scale steps before the plume's finer scales are placed")
    ap.add_argument("--plume-steps", type=int, default=40,
                    help="timed reference steps of the plume's multi-scale runs")
    ap.add_argument("--no-far-field", action="store_true",
                    help="skip the open-jet variant with a far-field scale")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the runs, copy a 1 GiB float32 tensor 3 times (reference "
                         "kernel of known traffic for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: only --gpus 1 is supported (asked for {args.gpus}); this build runs "
              "on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    main_run = run_gpu(args.n, "f32", args.steps, args.warmup)
    t = main_run["timing"]
    print(f"[bench] f32 {args.n}^3: {main_run['mlups']:.0f} MLUPS, "
          f"{main_run['ms_per_step']:.4f} ms/step (median of {t['repetitions']} windows of "
          f"{args.steps} steps; {t['min']:.4f}-{t['max']:.4f})", file=sys.stderr, flush=True)
    variants = {}
    if not args.no_variants:
        v = run_gpu(args.n, "f16s", args.steps, args.warmup)
        variants["f16s"] = {
            "value": v["mlups"], "unit": "MLUPS", "ms_per_step": v["ms_per_step"],
            "timing": v["timing"],
            "vs_f32_plain_step": v["mlups"] / main_run["mlups"],
            "roofline_frac": v["achieved_gbs"] / HBM_PEAK_GBS,
            "achieved_gbs": v["achieved_gbs"], "bytes_per_lup": BYTES_PER_LUP["f16s"],
        }
        print(f"[bench] f16s {args.n}^3: {v['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)

    if not args.no_precision:
        # the FP64 oracle's field for the precision comparison (oracle leg of
        # the benchmark, skipped with the CPU baseline)
        ref_slice = None if args.no_cpu_baseline else oracle_tgv_slice(384, 100)
        pr = run_precision(384, 100, ref_slice)
        variants["precision_tgv_384"] = pr
        print(f"[bench] 384^3 TGV: f32 {pr['f32']['mlups']:.0f} MLUPS, f16s {pr['f16s']['mlups']:.0f} "
              f"MLUPS, f16s vs f32 velocity rel L2 {pr['f16s_vs_f32_velocity_rel_l2']:.2e}"
              + ("" if ref_slice is None else
                 f", vs FP64 oracle: f32 {pr['f32_vs_fp64_oracle_velocity_rel_l2']:.2e}, "
                 f"f16s {pr['f16s_vs_fp64_oracle_velocity_rel_l2']:.2e}"),
              file=sys.stderr, flush=True)
    if not args.no_adjoint:
        ad = run_adjoint(128, 200, 20)
        variants["adjoint_smoke_128"] = ad
        print(f"[bench] 128^3 adjoint: {ad['adjoint_kernel_ms']:.3f} ms/step vs plain "
              f"{ad['plain_step_ms']:.3f} ms ({ad['adjoint_vs_plain_step_time']:.2f}x)",
              file=sys.stderr, flush=True)

    if not args.no_plume:
        pl = run_plume(512, 256, 256, args.plume_spinup, args.plume_steps)
        variants["plume_multiscale_512x256x256"] = pl
        print(f"[bench] plume: {pl['scales']} scales, cells {pl['cells_per_scale']}, "
              f"{pl['ms_per_reference_step']:.2f} ms/reference step, "
              f"{pl['mlups_all_scales']:.0f} MLUPS over all scales; reference scale alone "
              f"{pl['reference_scale_mlups']:.0f} MLUPS", file=sys.stderr, flush=True)

    if not args.no_gradient_mode:
        gm = run_gradient_mode(args.n, 200, 500)
        variants["gradient_mode_fd_256"] = gm
        print(f"[bench] gradient mode: {gm['mlups']:.0f} MLUPS; after {gm['compare_steps']} steps "
              f"velocity rel L2 vs local mode {gm['velocity_rel_l2_fd_vs_local']:.2e}, energy ratio "
              f"{gm['kinetic_energy_ratio_fd_vs_local']:.5f}", file=sys.stderr, flush=True)

    if not args.no_far_field:
        ff = run_far_field(512, 256, 256, 128, 100, 40)
        variants["far_field_open_jet_512x256x256"] = ff
        print(f"[bench] far field: cells {ff['cells_per_scale']}, {ff['ms_per_reference_step']:.2f} "
              f"ms/reference step ({ff['reference_scale_step_ms']:.2f} ms reference scale alone)",
              file=sys.stderr, flush=True)

    if args.copy_calibration:
        x = torch.rand(1 << 28, device="cuda")      # 1 GiB
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("[bench] copy calibration: 3 x (1 GiB read + 1 GiB write)", file=sys.stderr, flush=True)
        del x, y
        torch.cuda.empty_cache()

    traffic = measured_traffic("f32", args.n)
    result = {
        "metric": METRIC,
        "value": main_run["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "timing": {**main_run["timing"], "window_steps": args.steps},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"decaying turbulence {args.n}^3 periodic, D3Q27 central-moment "
                        "collision, adaptive relaxation on",
            "grid": [args.n] * 3,
            "cells": args.n ** 3,
            "nu": 1e-5,
            "spectrum": "E(k) ~ k^-5/3 over integer |k| in [2, 32], seed 1807",
            "u_rms_per_component": 0.04,
            "storage": "f32 shifted populations f_i - w_i",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_step<float> (fused pull-stream + collide)",
            "achieved": main_run["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": main_run["achieved_gbs"] / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": main_run["bytes_per_launch"],
        },
        "checks": {"mass_drift_rel": main_run["mass_drift_rel"],
                   "momentum_drift_abs": main_run["momentum_drift_abs"],
                   "kinetic_energy_ratio_after_warmup_and_steps": main_run["kinetic_energy_ratio"],
                   "nonfinite": main_run["nonfinite"]},
        "variants": variants,
        "source_hash": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.n)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
