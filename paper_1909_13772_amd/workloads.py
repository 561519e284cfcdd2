"""Timed workloads on one GPU (the benchmark configurations besides the
headline channel): batched uneven blocks in a porous medium, the precision
ladder on decaying turbulence, and the cost of the relaxation-time closures.

Each function returns a dict with throughput (MLUPS), the sweep kernel's
achieved bandwidth (algorithmic bytes / HIP-event kernel time) and the
accuracy figures of that configuration.
"""
from __future__ import annotations

import time

import numpy as np

from . import inputs

HBM_PEAK_GBS = 8000.0


def _timed_steps(B, steps, warmup, kernel_steps=None):
    """Wall-clock time of `steps` steps as they normally run (graph replay;
    with the interior/frontier overlap when chosen), then per-kernel HIP-event
    times from `kernel_steps` further steps, which launch every kernel in turn
    on the bound stream (kernel_steps None: the same steps are timed both
    ways, which keeps the sequential order)."""
    import torch

    B.step(warmup)
    B.synchronize()
    if kernel_steps is None:
        B.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(steps)
    B.synchronize()
    t1 = time.perf_counter()
    if kernel_steps is not None:
        B.set_kernel_timing(True)
        B.step(kernel_steps)
        B.synchronize()
    ms, cnt = B.kernel_times()
    B.set_kernel_timing(False)
    return t1 - t0, ms, cnt


def porous(wlb, steps=500, warmup=10, storage=None, autotune=True, seed_blocks=0, seed_spheres=1, overlap=None,
           tiles=None, nt=None, geometry="spheres"):
    """512 uneven blocks (rectilinear 8x8x8, edges from {16,24,32,48,64}),
    random spheres (radius 3-8, solid fraction >= 0.3), D3Q27 MRT, tau 0.8,
    density faces on x (1.0005 / 0.9995), periodic y/z, FP32 storage.
    geometry "empty": the same blocks without spheres; "one_block": the same
    domain without spheres in one block (the cost of the spheres and of the
    decomposition, measured apart)."""
    storage = wlb.F32 if storage is None else storage
    eb = wlb.ELEM_BYTES[storage]
    blocks, dom = inputs.uneven_blocks(seed_blocks)
    if geometry == "spheres":
        solid, frac, nsph = inputs.spheres(dom, seed=seed_spheres, rmin=3.0, rmax=8.0, solid_fraction=0.3,
                                           periodic=(0, 1, 1), clear_x=4)
    else:
        solid, frac, nsph = None, 0.0, 0
        if geometry == "one_block":
            blocks = wlb.single_block(dom)
    rho, u = inputs.uniform_state(dom)
    p = wlb.make_params(tau=0.8, omega_bulk=1.0, omega_higher=1.0, pressure_axis=0, rho_in=1.0005,
                        rho_out=0.9995, autotune=1 if autotune else 0)
    B = wlb.Blocks(blocks, dom, (0, 1, 1), stencil=27, storage=storage)
    try:
        B.init(wlb.MRT, p, rho, u, solid)
        if overlap is not None:  # override the autotuner's choice
            B.set_overlap(overlap)
        if tiles is not None:  # fixed launch configuration (profiler runs without the autotuner)
            B.set_tiles(*tiles)
        if nt is not None:
            B.set_nontemporal(*nt)
        # per-kernel events over the timed steps, as for the channel, unless
        # the sweep parts run concurrently (then timed in a separate run)
        secs, ms, cnt = _timed_steps(B, steps, warmup, kernel_steps=50 if B.info().overlap else None)
        info = B.info()
        force = B.force()  # momentum exchanged with the spheres in the last step
        r, uu, tot = B.moments()
    finally:
        B.close()
    ncell = dom[0] * dom[1] * dom[2]
    # Pressure drop across the medium and the drag it drives: at steady state
    # the drag on the spheres balances c_s^2 (rho_in - rho_out) A (no walls);
    # before that the ratio shows how far the flow has developed.  Darcy
    # permeability from the superficial velocity q = mean mass flux / A,
    # k = nu q L / (c_s^2 (rho_in - rho_out)), lattice units.
    area = dom[1] * dom[2]
    dp_force = (1.0005 - 0.9995) / 3.0 * area
    nfl = int(tot[6])
    sweep_ms = (ms[0] + ms[1]) / max(1, cnt[0] + cnt[1])
    xchg_ms = (ms[2] + ms[3]) / max(1, cnt[2] + cnt[3])
    bytes_launch = nfl * 2 * 27 * eb + ncell * 4
    flux = (r * uu[0]).sum(axis=(0, 1))
    return {
        "workload": "porous medium, 512 uneven blocks, D3Q27 MRT" if geometry == "spheres" else
                    f"porous-medium domain without spheres ({'512 uneven blocks' if geometry == 'empty' else 'one block'}), D3Q27 MRT",
        "domain": list(dom), "cells": ncell, "fluid_cells": nfl, "solid_fraction": float(frac),
        "spheres": int(nsph), "storage": wlb.STORAGE_NAMES[storage], "steps": steps,
        "mlups": ncell * steps / secs / 1e6, "mflups": nfl * steps / secs / 1e6,
        "ms_per_step": secs * 1e3 / steps, "sweep_ms": sweep_ms, "exchange_ms": xchg_ms,
        "even_ms": ms[0] / max(1, cnt[0]), "odd_ms": ms[1] / max(1, cnt[1]),
        "achieved_gbs": bytes_launch / (sweep_ms * 1e-3) / 1e9,
        "roofline_frac": bytes_launch / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "tile": list(info.tile), "grid": info.grid, "n_tiles": info.n_tiles, "xchg_elems": info.xchg_elems,
        "overlap": int(info.overlap), "lds_staging": int(info.lds_staging),
        "nontemporal": [int(info.nt_even), int(info.nt_odd)], "class_tiles": int(info.n_class_tiles),
        "flux_x_mean": float(flux.mean()), "flux_x_spread": float((flux.max() - flux.min()) / abs(flux.mean())),
        "max_u": float(tot[5]),
        "drag_on_spheres": [float(v) for v in force[:3]], "solid_links": int(force[6]),
        "drag_over_pressure_force": float(force[0] / dp_force),
        "permeability_lattice": float((0.8 - 0.5) / 3.0 * (flux.mean() / area) * dom[0] / ((1.0005 - 0.9995) / 3.0)),
    }


def _spectrum(u):
    from .les import shell_spectrum
    return shell_spectrum(u)


def turbulence_precision(wlb, n=384, steps=1000, every=100, seed=0, storages=None, tau=0.5005, umax=0.5):
    """Decaying turbulence (E(k) ~ k^4 exp(-2 (k/4)^2), u_rms 0.05) on n^3,
    D3Q19 TRT (Lambda 3/16).  Every storage type advances in lockstep with the
    FP64 run; every `every` steps each is compared with it (velocity relative
    L2 error; shell-spectrum error per shell for k <= 16 and relative to the
    peak for k <= 64) for as long as the
    FP64 run stays healthy (finite, max |u| < umax), and the step at which a
    run first fails that check is recorded.  At tau = 0.5005 (nu = 1.7e-4)
    the flow is far from resolved at any of these sizes and the plain
    collision operators do not survive 1000 steps in any precision, so the
    ladder is reported up to the reference's breakdown."""
    storages = storages or [wlb.F64, wlb.F32, wlb.F16DEV, wlb.BF16DEV]
    rho, u = inputs.turbulence_bandlimited(n, seed)
    p = wlb.make_params(tau=tau, magic=3.0 / 16.0, autotune=1)
    runs, secs, out = {}, {}, {}
    try:
        for st in storages:
            name = wlb.STORAGE_NAMES[st]
            B = wlb.Blocks(wlb.single_block((n, n, n)), (n, n, n), (1, 1, 1), stencil=19, storage=st)
            B.init(wlb.TRT, p, rho, u)
            runs[name], secs[name] = B, 0.0
            out[name] = {"diverged_at": None, "checkpoints": []}
        del rho, u
        ref_alive = True
        for step in range(every, steps + 1, every):
            fields = {}
            for name, B in list(runs.items()):
                t0 = time.perf_counter()
                B.step(every)
                B.synchronize()
                secs[name] += time.perf_counter() - t0
                _, uu, tot = B.moments()
                vmax = float(np.abs(uu).max())
                if not np.isfinite(vmax) or vmax >= umax:
                    out[name]["diverged_at"] = step
                    B.close()
                    del runs[name]
                    continue
                fields[name] = (uu, float(tot[4]), float(tot[0]))
            ref = fields.get("f64")
            if ref is None:
                ref_alive = False
            if not ref_alive:
                if not runs:
                    break
                continue
            e_ref = _spectrum(ref[0])
            k = np.arange(1, min(64, len(e_ref) - 1) + 1)
            k16 = np.arange(1, min(16, len(e_ref) - 1) + 1)
            peak = float(e_ref[k].max())
            for name, (uu, energy, mass) in fields.items():
                rec = {"step": step, "energy": energy, "mass_rel_drift": abs(mass - n ** 3) / n ** 3,
                       "max_u": float(np.abs(uu).max())}
                if name != "f64":
                    e = _spectrum(uu)
                    rec["u_rel_l2_vs_f64"] = float(np.linalg.norm(uu - ref[0]) / np.linalg.norm(ref[0]))
                    # per-shell relative error over the energy-containing range, and the
                    # error up to k = 64 relative to the spectrum's peak (far shells hold
                    # energies many orders below it, where any rounding is a large
                    # relative change)
                    rec["spectrum_rel_err_max_k16"] = float(np.max(np.abs(e[k16] - e_ref[k16]) / e_ref[k16]))
                    rec["spectrum_err_vs_peak_k64"] = float(np.max(np.abs(e[k] - e_ref[k])) / peak)
                out[name]["checkpoints"].append(rec)
    finally:
        for B in runs.values():
            B.close()
    for name, rec in out.items():
        done = rec["checkpoints"][-1]["step"] if rec["checkpoints"] else 0
        rec["steps_timed"] = rec["diverged_at"] or steps
        rec["mlups"] = n ** 3 * rec["steps_timed"] / secs[name] / 1e6 if secs[name] > 0 else None
        rec["last_compared_step"] = done
    return {"workload": f"decaying turbulence {n}^3, D3Q19 TRT, tau {tau}", "steps": steps, "every": every,
            "storage": out}


def entropic_stability(wlb, n=384, steps=1000, every=100, seed=0, tau=0.5005, umax=0.5):
    """The decaying-turbulence start of the precision ladder (n^3, u_rms 0.05,
    tau 0.5005: far from resolved) advanced in FP32 with D3Q19 TRT, D3Q27 MRT
    (all non-hydrodynamic rates 1), D3Q27 KBC, whose per-cell higher-order
    rate is the entropic stabiliser, and the D3Q27 cumulant collision (bulk
    rate 1, higher cumulants to zero).  Every `every` steps: kinetic energy,
    max |u|, mass drift; the step at which a run first leaves the healthy
    range (non-finite, max |u| >= umax) is recorded."""
    rho, u = inputs.turbulence_bandlimited(n, seed)
    cases = [("d3q19_trt", 19, wlb.TRT), ("d3q27_mrt", 27, wlb.MRT), ("d3q27_kbc", 27, wlb.KBC),
             ("d3q27_cumulant", 27, wlb.CUMULANT)]
    out = {}
    for name, q, coll in cases:
        p = wlb.make_params(tau=tau, magic=3.0 / 16.0, omega_bulk=1.0, omega_higher=1.0, autotune=1)
        B = wlb.Blocks(wlb.single_block((n, n, n)), (n, n, n), (1, 1, 1), stencil=q, storage=wlb.F32)
        rec = {"diverged_at": None, "checkpoints": []}
        secs = 0.0
        try:
            B.init(coll, p, rho, u)
            for step in range(every, steps + 1, every):
                t0 = time.perf_counter()
                B.step(every)
                B.synchronize()
                secs += time.perf_counter() - t0
                _, _, tot = B.moments(fields=False)
                vmax = float(tot[5])
                rec["checkpoints"].append({"step": step, "energy": float(tot[4]), "max_u": vmax,
                                           "mass_rel_drift": abs(float(tot[0]) - n ** 3) / n ** 3})
                if not np.isfinite(vmax) or not np.isfinite(tot[4]) or vmax >= umax:
                    rec["diverged_at"] = step
                    break
        finally:
            B.close()
        done = rec["checkpoints"][-1]["step"] if rec["checkpoints"] else 0
        rec["mlups"] = n ** 3 * done / secs / 1e6 if secs > 0 else None
        out[name] = rec
    return {"workload": f"decaying turbulence {n}^3, FP32, tau {tau}: plain vs entropic collision",
            "steps": steps, "every": every, "runs": out}


def matrix(wlb, n=384, steps=200, warmup=10, params=None):
    """The six forms on one shape: D3Q19 TRT (Lambda 3/16, tau 0.8) on the
    decaying-turbulence state of an n^3 periodic box, FP64 / FP32 / FP16 /
    BF16 deviation storage and FP32 with the Smagorinsky and MLP closures,
    each autotuned; MLUPS, the sweep kernel's achieved bandwidth and roofline
    fraction, and the velocity error against the FP64 run after `steps`."""
    rho, u = inputs.turbulence_bandlimited(n, 0)
    if params is None:
        params = inputs.mlp_params(0, inv_std=[300.0] * 6 + [100.0], out_bias=-4.0)
    forms = (("f64", wlb.F64, 8, wlb.CLOSURE_NONE), ("f32", wlb.F32, 4, wlb.CLOSURE_NONE),
             ("f16dev", wlb.F16DEV, 2, wlb.CLOSURE_NONE), ("bf16dev", wlb.BF16DEV, 2, wlb.CLOSURE_NONE),
             ("f32_smagorinsky", wlb.F32, 4, wlb.CLOSURE_SMAG), ("f32_mlp_closure", wlb.F32, 4, wlb.CLOSURE_MLP))
    out, u64 = {}, None
    for name, st, eb, cl in forms:
        kw = dict(tau=0.8, magic=3 / 16, closure=cl, cs_smag=0.1, autotune=1)
        if cl == wlb.CLOSURE_MLP:
            kw["mlp"] = params
        B = wlb.Blocks(wlb.single_block((n, n, n)), (n, n, n), (1, 1, 1), stencil=19, storage=st)
        try:
            B.init(wlb.TRT, wlb.make_params(**kw), rho, u)
            secs, ms, cnt = _timed_steps(B, steps, warmup)
            _, uu, _ = B.moments()
        finally:
            B.close()
        uu = uu.reshape(3, -1)
        if u64 is None:
            u64 = uu
        sweep_ms = (ms[0] + ms[1]) / max(1, cnt[0] + cnt[1])
        bl = n ** 3 * 2 * 19 * eb
        out[name] = {"mlups": n ** 3 * steps / secs / 1e6, "sweep_ms": sweep_ms,
                     "achieved_gbs": bl / (sweep_ms * 1e-3) / 1e9,
                     "roofline_frac": bl / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "u_rel_err_vs_f64": float(np.linalg.norm(uu - u64) / np.linalg.norm(u64))}
    return {"workload": f"D3Q19 TRT decaying turbulence {n}^3, tau 0.8, every storage and closure",
            "steps": steps, "warmup": warmup, "forms": out}


def closure_cost(wlb, n=128, steps=500, warmup=10, params=None):
    """D3Q19 SRT FP32 on a periodic turbulent n^3 box with no closure,
    Smagorinsky and the MLP closure (tau0 = 0.5025, the coarse relaxation
    time of the learned-closure runs)."""
    rho, u = inputs.turbulence_bandlimited(n, 0)
    if params is None:
        params = inputs.mlp_params(0, inv_std=[300.0] * 6 + [100.0], out_bias=-4.0)
    out = {}
    for name, cl in (("none", wlb.CLOSURE_NONE), ("smagorinsky", wlb.CLOSURE_SMAG), ("mlp", wlb.CLOSURE_MLP)):
        kw = dict(tau=0.5025, closure=cl, cs_smag=0.1, autotune=1)
        if cl == wlb.CLOSURE_MLP:
            kw["mlp"] = params
        B = wlb.Blocks(wlb.single_block((n, n, n)), (n, n, n), (1, 1, 1), stencil=19, storage=wlb.F32)
        try:
            B.init(wlb.SRT, wlb.make_params(**kw), rho, u)
            secs, ms, cnt = _timed_steps(B, steps, warmup)
        finally:
            B.close()
        sweep_ms = (ms[0] + ms[1]) / max(1, cnt[0] + cnt[1])
        bl = n ** 3 * 2 * 19 * 4
        out[name] = {"mlups": n ** 3 * steps / secs / 1e6, "sweep_ms": sweep_ms,
                     "achieved_gbs": bl / (sweep_ms * 1e-3) / 1e9,
                     "roofline_frac": bl / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return {"workload": f"LES closures, D3Q19 SRT FP32 {n}^3", "steps": steps, "closure": out}
