"""Benchmark: lattice Boltzmann stream-collide on one MI355X.

Workload (headline): D3Q19 TRT (Lambda = 3/16), single block 256^3, FP64
deviation storage, channel with half-way bounce-back walls in y, periodic
x/z, Guo body force f_x = 1e-6, tau = 0.8, starting from rest; one step is
one AA sweep over all cells plus the ghost-layer exchange.  The same
configuration is also timed with FP32, FP16 and BF16 deviation storage,
with the Smagorinsky and learned closures, with D3Q27 MRT / KBC / cumulant
collisions and with the D3Q15 and D2Q9 velocity sets (D2Q9: 256 independent
xy planes) -- the "variants".

Prints ONE JSON line with MLUPS, the HBM roofline fraction of the sweep
kernel (algorithmic bytes / measured kernel time, HIP events on the
library's stream), and the CPU oracle timed on a bounded sample.

Timing: `value` (MLUPS, ms_per_step) is the wall time of the timed steps
run the way wlb_lbm_step runs them in production, as replays of the
captured HIP graph of [even sweep, exchange, odd sweep, exchange].  The
per-kernel times behind `roofline` come from a second run of the same
number of steps with per-kernel HIP events on the library's stream (which
launches the kernels one by one).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 256
TAU, MAGIC, FX = 0.8, 3.0 / 16.0, 1e-6
# the sweep kernels and the arena layout (runtime.hip) decide the HBM traffic
SWEEP_SOURCES = ["paper_1909_13772_amd/csrc/sweep_impl.hpp", "paper_1909_13772_amd/csrc/lattice.hpp",
                 "paper_1909_13772_amd/csrc/wlb_internal.hpp", "paper_1909_13772_amd/csrc/runtime.hip"]


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(storage_name: str, odd_sweep: str):
    """HBM bytes per sweep launch from a committed rocprofv3 counter summary,
    only if it was taken on the current sweep source with the same odd-sweep
    kernel and non-temporal choices."""
    path = os.path.join(ROOT, "profiles", "sweep_channel256_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != sweep_source_hash() or t.get("odd_sweep") != odd_sweep:
        return None
    e = t.get("storage", {}).get(storage_name)
    return None if e is None else e.get("hbm_bytes_per_launch")


def closure_weights(inputs):
    """Trained closure weights if present (paper_1909_13772_amd/mlp_closure.npy),
    else seeded weights of the same shape (the sweep's cost does not depend on
    the values)."""
    import numpy as np
    path = os.path.join(ROOT, "paper_1909_13772_amd", "mlp_closure.npy")
    if os.path.exists(path):
        return np.load(path).astype(np.float32)
    return inputs.mlp_params(0, inv_std=[300.0] * 6 + [100.0], out_bias=-4.0)


def VARIANTS(wlb):
    """(name, storage, element bytes, closure, velocity set, collision) of the
    variants timed on the headline channel."""
    return (("f32", wlb.F32, 4, 0, 19, None), ("f16dev", wlb.F16DEV, 2, 0, 19, None),
            ("bf16dev", wlb.BF16DEV, 2, 0, 19, None), ("f32_smagorinsky", wlb.F32, 4, 1, 19, None),
            ("f32_mlp_closure", wlb.F32, 4, 2, 19, None), ("f32_d3q27_mrt", wlb.F32, 4, 0, 27, wlb.MRT),
            ("f32_d3q27_kbc", wlb.F32, 4, 0, 27, wlb.KBC), ("f32_d3q27_cumulant", wlb.F32, 4, 0, 27, wlb.CUMULANT),
            ("f32_d3q15", wlb.F32, 4, 0, 15, None), ("f32_d2q9_planes", wlb.F32, 4, 0, 9, None))


def poiseuille_series(H, nu, g, T, s):
    u = g * s * (H - s) / (2 * nu)
    for n in range(1, 4000, 2):
        u -= 4 * g * H * H / (nu * math.pi ** 3 * n ** 3) * __import__("numpy").sin(n * math.pi * s / H) * \
            math.exp(-n * n * math.pi ** 2 * nu * T / (H * H))
    return u


def run_config(wlb, inputs, storage, steps, warmup, closure=0, check=False, autotune=True, q=19, coll=None, lds=None,
               nt=None, slot_round=None):
    import numpy as np
    import torch

    shape = (N, N, N)
    rho, u = inputs.uniform_state(shape)
    mlp = None
    if closure == 2:
        mlp = closure_weights(inputs)
    p = wlb.make_params(tau=TAU, magic=MAGIC, force=(FX, 0.0, 0.0), closure=closure, cs_smag=0.1 if closure else 0.0,
                        mlp=mlp, autotune=1 if autotune else 0)
    B = wlb.Blocks(wlb.single_block(shape), shape, (1, 0, 1), stencil=q, storage=storage)
    try:
        if slot_round is not None:  # fixed slot stride (profiler runs without the autotuner)
            B.set_slot_round(slot_round)
        B.init(wlb.TRT if coll is None else coll, p, rho, u)
        if lds is not None:  # fixed odd-sweep choice (profiler runs without the autotuner)
            B.set_lds_staging(int(lds))
        if nt is not None:  # fixed non-temporal choice per parity (profiler runs)
            B.set_nontemporal(*nt)
        B.step(warmup)
        B.synchronize()
        torch.cuda.synchronize()
        # timed region: graph replay (wlb_lbm_step as in production)
        t0 = time.perf_counter()
        B.step(steps)
        B.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = B.info()
        res = {"seconds": t1 - t0, "tile": list(info.tile), "grid": info.grid,
               "n_tiles": info.n_tiles, "xchg_elems": info.xchg_elems, "lds_staging": int(info.lds_staging),
               "nt": [int(info.nt_even), int(info.nt_odd)], "slot_round_kib": int(info.slot_round_kib)}
        if check:
            r, uu, tot = B.moments()
            nu = (TAU - 0.5) / 3
            s = np.arange(N) + 0.5
            # the Guo velocity (j + F/2)/rho after n steps from rest is the
            # continuous flow at time n + 1/2
            ref = poiseuille_series(N, nu, FX, warmup + steps + 0.5, s)
            prof = uu[0].mean(axis=(0, 2))
            res["profile"] = prof
            res["poiseuille_err"] = float(np.abs(prof - ref).max() / ref.max())
            res["mass_drift"] = float(abs(tot[0] - N ** 3) / N ** 3)
        # per-kernel times: a separate run of as many steps with HIP events
        # around every launch
        B.set_kernel_timing(True)
        B.step(steps)
        B.synchronize()
        ms, cnt = B.kernel_times()
        B.set_kernel_timing(False)
        res["kernel_ms"], res["launches"] = ms, cnt
        return res
    finally:
        B.close()


def summarize(res, storage, steps, elem_bytes, q=19):
    cells = N ** 3
    sweeps = res["launches"][0] + res["launches"][1]
    sweep_ms = (res["kernel_ms"][0] + res["kernel_ms"][1]) / max(1, sweeps)
    xchg_ms = (res["kernel_ms"][2] + res["kernel_ms"][3]) / max(1, res["launches"][2] + res["launches"][3])
    bytes_per_launch = cells * 2 * q * elem_bytes
    achieved = bytes_per_launch / (sweep_ms * 1e-3) / 1e9
    ms, cnt = res["kernel_ms"], res["launches"]
    return {
        "even_ms": ms[0] / max(1, cnt[0]),
        "odd_ms": ms[1] / max(1, cnt[1]),
        "mlups": cells * steps / res["seconds"] / 1e6,
        "ms_per_step": res["seconds"] * 1e3 / steps,
        "sweep_ms": sweep_ms,
        "exchange_ms": xchg_ms,
        "achieved_gbs": achieved,
        "frac": achieved / HBM_PEAK_GBS,
        "bytes_per_launch": bytes_per_launch,
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """OpenMP threads for the oracle: OMP_NUM_THREADS when set (the GPU
    host's share of cores for one GPU), else every core this process may
    run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return (int(env) if env and env.isdigit() and int(env) > 0 else avail), avail


def cpu_baseline(inputs):
    """The FP64 oracle on the host: the full 256^3 channel for a few steps on
    the host's OpenMP threads (the value), and one thread on a 64^3 crop."""
    import oracle as O

    nthreads, avail = host_threads()
    shape = (N, N, N)
    steps = 12
    rho, u = inputs.uniform_state(shape)
    p = O.Params(q=19, collision=O.TRT, tau=TAU, magic=MAGIC, force=(FX, 0, 0), periodic=(1, 0, 1))
    d = O.init(19, shape, rho, u)
    t0 = time.perf_counter()
    O.run(p, shape, d, steps, nthreads=nthreads)
    dt = time.perf_counter() - t0
    del d
    small = (64, 64, 64)
    rs, us = inputs.uniform_state(small)
    d1 = O.init(19, small, rs, us)
    t1 = time.perf_counter()
    O.run(p, small, d1, 4, nthreads=1)
    dt1 = time.perf_counter() - t1
    return {"value": N ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": nthreads, "kind": "oracle",
            "sample": f"full 256^3 channel, D3Q19 TRT FP64, {steps} steps ({dt:.1f} s), OpenMP threads={nthreads}",
            "single_thread_mlups": 64 ** 3 * 4 / dt1 / 1e6, "single_thread_sample": "64^3 channel crop, 4 steps",
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(), "cpus_available": avail}


def copy_probe(wlb):
    import torch

    nbytes = 4 << 30
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    ms = wlb.wlb_copy_probe(b.data_ptr(), a.data_ptr(), nbytes, 10, s.cuda_stream)
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def host_io_probe(wlb, inputs, steps, ms_per_step):
    """Host-buffer hand-over of the headline configuration: wlb_lbm_init from
    host rho / u (upload plus initialisation, no autotuner) and
    wlb_moments_get of rho / u to host, each timed as the best of two, and
    the whole-job rate of `steps` steps including both transfers."""
    shape = (N, N, N)
    rho, u = inputs.uniform_state(shape)
    p = wlb.make_params(tau=TAU, magic=MAGIC, force=(FX, 0.0, 0.0))
    B = wlb.Blocks(wlb.single_block(shape), shape, (1, 0, 1), stencil=19, storage=wlb.F64)
    try:
        t_init = t_mom = float("inf")
        for _ in range(2):
            t0 = time.perf_counter()
            B.init(wlb.TRT, p, rho, u)
            B.synchronize()
            t_init = min(t_init, time.perf_counter() - t0)
            t0 = time.perf_counter()
            B.moments()
            t_mom = min(t_mom, time.perf_counter() - t0)
    finally:
        B.close()
    job = t_init + steps * ms_per_step * 1e-3 + t_mom
    return {"init_s": round(t_init, 4), "moments_s": round(t_mom, 4), "steps": steps,
            "mlups_including_host_io": round(N ** 3 * steps / job / 1e6, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variant-steps", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the default tile shape (for profiler runs that should hold only the timed launches)")
    ap.add_argument("--lds-staging", type=int, choices=[0, 1, 2], default=None,
                    help="with --no-autotune: odd sweep direct (0), staged in LDS (1) or over row vectors (2)")
    ap.add_argument("--slot-round", type=int, choices=[16384, 2048, 0], default=None,
                    help="with --no-autotune: slot stride rounding in KiB of the population slots of 64 MiB or more "
                         "(headline and variant runs)")
    ap.add_argument("--nontemporal", type=str, default=None,
                    help="with --no-autotune: 'E,O' non-temporal accesses (1) or cached (0) in the even / odd sweep "
                         "(headline and variant runs)")
    ap.add_argument("--tiles", type=str, default=None,
                    help="with --no-autotune: 'tx,ty,tz,grid' launch configuration of the porous workload")
    ap.add_argument("--variant", type=str, default="f32_mlp_closure",
                    help="with --workload variant: the variant configuration to run alone")
    ap.add_argument("--porous-geometry", choices=["spheres", "empty", "one_block"], default="spheres",
                    help="with --workload porous: spheres (default), the blocks without spheres, or one block")
    ap.add_argument("--workload", choices=["channel", "porous", "turbulence", "closures", "entropic", "matrix",
                                           "variant"],
                    default="channel",
                    help="channel = the headline configuration; variant = one of its variants alone (for "
                         "profiler runs); the others print their own JSON line")
    ap.add_argument("--tau", type=float, default=0.5005, help="relaxation time of the turbulence workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (blocks would shard over GPUs "
              "by exchanging face slabs; not built).", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1909_13772_amd import inputs, wlb

    torch.cuda.set_device(0)
    print(f"[bench] device {torch.cuda.get_device_name(0)}", file=sys.stderr, flush=True)
    if args.workload == "variant":
        cfg = {v[0]: v[1:] for v in VARIANTS(wlb)}
        if args.variant not in cfg:
            print(f"unknown variant {args.variant}; one of {sorted(cfg)}", file=sys.stderr)
            sys.exit(2)
        st, eb, cl, q, coll = cfg[args.variant]
        nt = None if args.nontemporal is None else [int(v) for v in args.nontemporal.split(",")]
        r = run_config(wlb, inputs, st, args.steps, args.warmup, closure=cl, autotune=not args.no_autotune, q=q,
                       coll=coll, lds=args.lds_staging, nt=nt if args.no_autotune else None,
                       slot_round=args.slot_round if args.no_autotune else None)
        sm = summarize(r, st, args.steps, eb, q=q)
        print(json.dumps({"workload": f"channel 256^3 variant {args.variant}", "steps": args.steps,
                          "mlups": sm["mlups"], "even_ms": sm["even_ms"], "odd_ms": sm["odd_ms"],
                          "achieved_gbs": sm["achieved_gbs"], "roofline_frac": sm["frac"], "tile": r["tile"],
                          "grid": r["grid"], "nt": r["nt"], "odd_sweep": r["lds_staging"]}))
        return
    if args.workload != "channel":
        from paper_1909_13772_amd import workloads
        if args.workload == "porous":
            tiles = None if args.tiles is None else [int(v) for v in args.tiles.split(",")]
            nt = None if args.nontemporal is None else [int(v) for v in args.nontemporal.split(",")]
            r = workloads.porous(wlb, steps=args.steps, warmup=args.warmup, autotune=not args.no_autotune,
                                 tiles=tiles if args.no_autotune else None, nt=nt if args.no_autotune else None,
                                 geometry=args.porous_geometry)
        elif args.workload == "turbulence":
            r = workloads.turbulence_precision(wlb, steps=args.steps, tau=args.tau)
        elif args.workload == "entropic":
            r = workloads.entropic_stability(wlb, steps=args.steps, tau=args.tau)
        elif args.workload == "matrix":
            r = workloads.matrix(wlb, steps=args.steps, warmup=args.warmup, params=closure_weights(inputs))
        else:
            r = workloads.closure_cost(wlb, steps=args.steps, warmup=args.warmup)
        print(json.dumps(r))
        return
    head_nt = None if args.nontemporal is None else [int(v) for v in args.nontemporal.split(",")]
    res = run_config(wlb, inputs, wlb.F64, args.steps, args.warmup, check=True, autotune=not args.no_autotune,
                     lds=args.lds_staging, nt=head_nt, slot_round=args.slot_round if args.no_autotune else None)
    head = summarize(res, wlb.F64, args.steps, 8)
    print(f"[bench] f64: {head['mlups']:.0f} MLUPS, sweep {head['sweep_ms']:.3f} ms, "
          f"{head['achieved_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
    variants = {}
    if not args.no_variants:
        # FP64 reference profile after the variants' step count (accuracy of each variant)
        import numpy as np
        r64 = run_config(wlb, inputs, wlb.F64, args.variant_steps, args.warmup, check=True, autotune=False)
        p64 = r64["profile"]
        for name, st, eb, cl, q, coll in VARIANTS(wlb):
            r = run_config(wlb, inputs, st, args.variant_steps, args.warmup, closure=cl, autotune=not args.no_autotune,
                           q=q, coll=coll, check=True, nt=head_nt if args.no_autotune else None,
                           slot_round=args.slot_round if args.no_autotune else None)
            sm = summarize(r, st, args.variant_steps, eb, q=q)
            variants[name] = {"mlups": round(sm["mlups"], 1), "roofline_frac": round(sm["frac"], 4),
                              "achieved_gbs": round(sm["achieved_gbs"], 1), "sweep_ms": round(sm["sweep_ms"], 4),
                              "even_ms": round(sm["even_ms"], 4), "odd_ms": round(sm["odd_ms"], 4),
                              "steps": args.variant_steps,
                              "profile_rel_err_vs_f64": float(np.linalg.norm(r["profile"] - p64) / np.linalg.norm(p64)),
                              "poiseuille_rel_err": r["poiseuille_err"]}
            print(f"[bench] {name}: {sm['mlups']:.0f} MLUPS, {sm['achieved_gbs']:.0f} GB/s", file=sys.stderr,
                  flush=True)
    try:
        copy_gbs = copy_probe(wlb)
    except Exception as e:  # the probe is context only
        print(f"[bench] copy probe failed: {e}", file=sys.stderr)
        copy_gbs = None
    try:
        host_io = host_io_probe(wlb, inputs, args.steps, head["ms_per_step"])
    except Exception as e:  # context only
        print(f"[bench] host I/O probe failed: {e}", file=sys.stderr)
        host_io = None
    cpu = None if args.no_cpu else cpu_baseline(inputs)
    access = (("direct", "lds-staged", "row-vector")[res["lds_staging"]] + "; non-temporal even %d odd %d" % tuple(res["nt"])
              + "; slot rounding %d KiB" % res["slot_round_kib"])
    traffic = load_traffic("f64", access)
    out = {
        "metric": "MLUPS + % HBM roofline: plain FP64 vs FP32/FP16-store vs learned closure",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "D3Q19 TRT (Lambda 3/16) channel 256^3, one block, FP64 deviation storage, "
                               "bounce-back walls in y, periodic x/z, Guo force fx=1e-6, tau=0.8, from rest",
                   "cells": N ** 3, "stencil": "D3Q19", "collision": "TRT", "storage": "f64",
                   "tile": res["tile"], "grid": res["grid"],
                   "odd_sweep": ("direct", "lds-staged", "row-vector")[res["lds_staging"]],
                   "nontemporal": {"even": res["nt"][0], "odd": res["nt"][1]},
                   "slot_round_kib": res["slot_round_kib"]},
        "roofline": {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(head["frac"], 4), "traffic": traffic,
                     "kernel": "sweep_kernel<19,TRT,double> (even AA sweep) and " +
                               (("sweep_odd_lds_kernel<19,TRT,double>", "sweep_odd_vec_kernel<19,TRT,double>")
                                [res["lds_staging"] - 1] if res["lds_staging"] else
                                "sweep_odd_aligned_nt_kernel<19,TRT,double>" if res["nt"][1] == 2 else
                                "sweep_kernel<19,TRT,double>") + " (odd AA sweep)",
                     "algorithmic_bytes_per_launch": head["bytes_per_launch"],
                     "avg_launch_ms": round(head["sweep_ms"], 5), "even_launch_ms": round(head["even_ms"], 5),
                     "odd_launch_ms": round(head["odd_ms"], 5)},
        "cpu_baseline": cpu,
        "timing": {"value": "wall clock of the timed steps, replays of the captured HIP graph",
                   "roofline": "per-kernel HIP events on the library's stream, separate run of as many steps"},
        "variants": variants,
        "exchange_ms_per_step": round(head["exchange_ms"], 5),
        "copy_probe_gbs": None if copy_gbs is None else round(copy_gbs, 1),
        "host_io": host_io,
        "check": {"poiseuille_rel_err": res.get("poiseuille_err"), "mass_rel_drift": res.get("mass_drift")},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
