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


def _timed_steps(B, steps, warmup):
    import torch

    B.step(warmup)
    B.synchronize()
    B.set_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(steps)
    B.synchronize()
    t1 = time.perf_counter()
    ms, cnt = B.kernel_times()
    B.set_kernel_timing(False)
    return t1 - t0, ms, cnt


def porous(wlb, steps=500, warmup=10, storage=None, autotune=True, seed_blocks=0, seed_spheres=1):
    """512 uneven blocks (rectilinear 8x8x8, edges from {16,24,32,48,64}),
    random spheres (radius 3-8, solid fraction >= 0.3), D3Q27 MRT, tau 0.8,
    density faces on x (1.0005 / 0.9995), periodic y/z, FP32 storage."""
    storage = wlb.F32 if storage is None else storage
    eb = wlb.ELEM_BYTES[storage]
    blocks, dom = inputs.uneven_blocks(seed_blocks)
    solid, frac, nsph = inputs.spheres(dom, seed=seed_spheres, rmin=3.0, rmax=8.0, solid_fraction=0.3,
                                       periodic=(0, 1, 1), clear_x=4)
    rho, u = inputs.uniform_state(dom)
    p = wlb.make_params(tau=0.8, omega_bulk=1.0, omega_higher=1.0, pressure_axis=0, rho_in=1.0005,
                        rho_out=0.9995, autotune=1 if autotune else 0)
    B = wlb.Blocks(blocks, dom, (0, 1, 1), stencil=27, storage=storage)
    try:
        B.init(wlb.MRT, p, rho, u, solid)
        secs, ms, cnt = _timed_steps(B, steps, warmup)
        info = B.info()
        r, uu, tot = B.moments()
    finally:
        B.close()
    ncell = dom[0] * dom[1] * dom[2]
    nfl = int(tot[6])
    sweep_ms = (ms[0] + ms[1]) / max(1, cnt[0] + cnt[1])
    xchg_ms = (ms[2] + ms[3]) / max(1, cnt[2] + cnt[3])
    bytes_launch = nfl * 2 * 27 * eb + ncell * 4
    flux = (r * uu[0]).sum(axis=(0, 1))
    return {
        "workload": "porous medium, 512 uneven blocks, D3Q27 MRT",
        "domain": list(dom), "cells": ncell, "fluid_cells": nfl, "solid_fraction": float(frac),
        "spheres": int(nsph), "storage": wlb.STORAGE_NAMES[storage], "steps": steps,
        "mlups": ncell * steps / secs / 1e6, "mflups": nfl * steps / secs / 1e6,
        "ms_per_step": secs * 1e3 / steps, "sweep_ms": sweep_ms, "exchange_ms": xchg_ms,
        "achieved_gbs": bytes_launch / (sweep_ms * 1e-3) / 1e9,
        "roofline_frac": bytes_launch / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "tile": list(info.tile), "grid": info.grid, "n_tiles": info.n_tiles, "xchg_elems": info.xchg_elems,
        "flux_x_mean": float(flux.mean()), "flux_x_spread": float((flux.max() - flux.min()) / abs(flux.mean())),
        "max_u": float(tot[5]),
    }


def _spectrum(u):
    from .les import shell_spectrum
    return shell_spectrum(u)


def turbulence_precision(wlb, n=384, steps=1000, warmup=0, seed=0, storages=None):
    """Decaying turbulence (E(k) ~ k^4 exp(-2 (k/4)^2), u_rms 0.05) on n^3,
    D3Q19 TRT (Lambda 3/16), tau 0.5005; each storage type against the FP64
    run: velocity relative L2 error and the worst shell-spectrum error for
    k <= 64 after `steps` steps."""
    storages = storages or [wlb.F64, wlb.F32, wlb.F16DEV, wlb.BF16DEV]
    rho, u = inputs.turbulence_bandlimited(n, seed)
    p = wlb.make_params(tau=0.5005, magic=3.0 / 16.0, autotune=1, health_every=100, health_umax=0.5)
    ref_u, ref_e, out = None, None, {}
    for st in storages:
        B = wlb.Blocks(wlb.single_block((n, n, n)), (n, n, n), (1, 1, 1), stencil=19, storage=st)
        name = wlb.STORAGE_NAMES[st]
        try:
            B.init(wlb.TRT, p, rho, u)
            try:
                secs, ms, cnt = _timed_steps(B, steps, warmup)
            except wlb.WlbError as e:
                out[name] = {"diverged": True, "error": str(e)}
                continue
            _, uu, tot = B.moments()
        finally:
            B.close()
        sweep_ms = (ms[0] + ms[1]) / max(1, cnt[0] + cnt[1])
        bl = n ** 3 * 2 * 19 * wlb.ELEM_BYTES[st]
        e = _spectrum(uu)
        rec = {"mlups": n ** 3 * steps / secs / 1e6, "sweep_ms": sweep_ms,
               "achieved_gbs": bl / (sweep_ms * 1e-3) / 1e9,
               "roofline_frac": bl / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "energy": float(tot[4]),
               "mass_rel_drift": float(abs(tot[0] - n ** 3) / n ** 3)}
        if ref_u is None:
            ref_u, ref_e = uu, e
        else:
            rec["u_rel_l2_vs_f64"] = float(np.linalg.norm(uu - ref_u) / np.linalg.norm(ref_u))
            k = np.arange(1, min(64, len(e) - 1) + 1)
            rec["spectrum_rel_err_max_vs_f64"] = float(np.max(np.abs(e[k] - ref_e[k]) / ref_e[k]))
        out[name] = rec
    return {"workload": f"decaying turbulence {n}^3, D3Q19 TRT, tau 0.5005", "steps": steps, "storage": out}


def closure_cost(wlb, n=128, steps=500, warmup=10, params=None):
    """D3Q19 SRT FP32 on a periodic turbulent n^3 box with no closure,
    Smagorinsky and the MLP closure (tau0 = 0.5075)."""
    rho, u = inputs.turbulence_bandlimited(n, 0)
    if params is None:
        params = inputs.mlp_params(0, inv_std=[300.0] * 6 + [100.0], out_bias=-4.0)
    out = {}
    for name, cl in (("none", wlb.CLOSURE_NONE), ("smagorinsky", wlb.CLOSURE_SMAG), ("mlp", wlb.CLOSURE_MLP)):
        kw = dict(tau=0.5075, closure=cl, cs_smag=0.1, autotune=1)
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
