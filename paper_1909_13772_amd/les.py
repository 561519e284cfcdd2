"""Learned relaxation-time closure: training data, training and evaluation.

Pipeline (every numerical step runs in libwlb's kernels; PyTorch only holds
device buffers and streams):

1. Fine runs: decaying turbulence (band-limited E(k) ~ k^4 exp(-2 (k/4)^2),
   u_rms = 0.05) on an n_f^3 periodic box, D3Q19 SRT, FP32 storage,
   tau_f = 0.51.  Every `snap` fine steps the state is box-filtered by
   `factor` (wlb_box_filter) and turned into training pairs (wlb_les_targets):
   features = (Pi_neq the coarse run would see, rho - 1), target = 3 nu_t of
   the sub-grid stress.
2. Training: minibatches of the pairs, loss on the standardised target,
   gradients by wlb_mlp_grad and Adam by wlb_mlp_adam (FP32 master weights).
3. Evaluation: coarse LES (n_f / factor)^3, tau0 = 1/2 + 3 nu_f / factor
   (acoustic scaling: dx and dt grow by `factor`, velocities unchanged),
   from the filtered fine initial state, with no model, Smagorinsky (C_s 0.1)
   and the MLP, against the filtered fine run of the same seed: kinetic
   energy history and the final shell spectrum.

The paper lets relaxation rates vary per cell, read from a field or set by a
turbulence model (Sec. 5.1.1); the learned closure is this project's
addition and its gain is measured, not assumed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import inputs

# Fine-run relaxation time: nu_f = 1/300.  At 512^3 with u_rms 0.05 this
# fine run is resolved (it stays stable and smooth), while the coarse 128^3
# run at the acoustically scaled tau0 = 0.5025 is not: without a sub-grid
# model it blows up, which is the regime a closure is for.
TAU_F = 0.51
U_RMS = 0.05


def _log(msg):
    print(msg, flush=True)


def coarse_tau(factor, tau_f=TAU_F):
    nu_f = (tau_f - 0.5) / 3.0
    return 0.5 + 3.0 * nu_f / factor


def shell_spectrum(u):
    """E(k) over integer shells of a periodic (3, n, n, n) velocity field."""
    n = u.shape[-1]
    uh = np.fft.rfftn(u, axes=(1, 2, 3)) / n ** 3
    e = 0.5 * (np.abs(uh) ** 2).sum(0)
    e[..., 1:-1 if n % 2 == 0 else None] *= 2.0  # rfft half-spectrum weights
    f = np.fft.fftfreq(n) * n
    fr = np.fft.rfftfreq(n) * n
    k = np.sqrt(f[:, None, None] ** 2 + f[None, :, None] ** 2 + fr[None, None, :] ** 2)
    sh = np.rint(k).astype(np.int64)
    return np.bincount(sh.ravel(), weights=e.ravel())[: n // 2 + 1]


def filtered_energy(filt_dev):
    """Kinetic energy sum rho |u|^2 / 2 of box-filtered fields (host FP64)."""
    F = filt_dev.cpu().numpy().reshape(10, -1)
    return float(0.5 * np.sum(F[0] * (F[1] ** 2 + F[2] ** 2 + F[3] ** 2)))


class FineRun:
    """One fine decaying-turbulence run producing filtered snapshots."""

    def __init__(self, wlb, torch, seed, n, factor, storage=None, tau_f=TAU_F):
        self.wlb, self.torch = wlb, torch
        self.n, self.factor = n, factor
        self.nc = n // factor
        rho, u = inputs.turbulence_bandlimited(n, seed, u_rms=U_RMS)
        st = wlb.F32 if storage is None else storage
        self.B = wlb.Blocks(wlb.single_block((n, n, n)), (n, n, n), (1, 1, 1), stencil=19, storage=st)
        # health check: a fine run that blows up must not feed the training set
        self.B.init(wlb.SRT, wlb.make_params(tau=tau_f, health_every=200, health_umax=0.5), rho, u)
        del rho, u
        self.filt = torch.empty(10 * self.nc ** 3, dtype=torch.float64, device="cuda")

    def filtered(self):
        self.wlb.wlb_box_filter(self.B.h, self.factor, self.filt.data_ptr())
        return self.filt

    def pairs(self, tau0):
        nc3 = self.nc ** 3
        raw = self.torch.empty(nc3 * 7, dtype=self.torch.float32, device="cuda")
        tgt = self.torch.empty(nc3, dtype=self.torch.float32, device="cuda")
        self.wlb.wlb_les_targets(self.filtered().data_ptr(), (self.nc,) * 3, tau0, raw.data_ptr(), tgt.data_ptr(),
                                 self.B.stream.cuda_stream)
        self.B.synchronize()
        return raw.view(nc3, 7), tgt

    def coarse_state(self):
        """Filtered density and velocity (host) of the current state."""
        F = self.filtered().cpu().numpy().reshape(10, self.nc, self.nc, self.nc)
        return F[0].copy(), F[1:4].copy()

    def close(self):
        self.B.close()


def generate(wlb, torch, seeds, n, factor, steps, snap, per_snap, rng_seed=0, tau_f=TAU_F):
    """Training pairs (host float32) from fine runs: raw (M, 7), target (M,),
    and for each seed the filtered kinetic energy / final spectrum."""
    tau0 = coarse_tau(factor, tau_f)
    g = torch.Generator(device="cuda")
    g.manual_seed(rng_seed)
    raws, tgts, sids, refs = [], [], [], {}
    for seed in seeds:
        t0 = time.time()
        fr = FineRun(wlb, torch, seed, n, factor, tau_f=tau_f)
        energy = []
        for s in range(0, steps + 1, snap):
            if s > 0:
                fr.B.step(snap)
            raw, tgt = fr.pairs(tau0)
            energy.append(filtered_energy(fr.filt))
            idx = torch.randint(0, tgt.numel(), (per_snap,), device="cuda", generator=g)
            raws.append(raw[idx].cpu().numpy())
            tgts.append(tgt[idx].cpu().numpy())
            sids.append(np.full(per_snap, seed, np.int32))
        rho_c, u_c = fr.coarse_state()
        refs[seed] = {"energy": energy, "spectrum": shell_spectrum(u_c).tolist()}
        fr.close()
        _log(f"[les] fine seed {seed}: {steps} steps at {n}^3 in {time.time() - t0:.1f} s")
    generate.last_seed_ids = np.concatenate(sids)
    return np.concatenate(raws), np.concatenate(tgts), refs


# The 48 symmetries of the cube act on the stress components (xx, yy, zz, xy,
# xz, yz) by an axis permutation and sign flips; the density and the target
# (a scalar viscosity) are invariant.
_PAIRS = {(0, 1): 3, (0, 2): 4, (1, 2): 5}


def cube_symmetries():
    """(48, 6) source component and (48, 6) sign for each symmetry."""
    import itertools
    out_idx, out_sgn = [], []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            idx, sgn = [perm[0], perm[1], perm[2]], [1, 1, 1]
            for (a, b) in ((0, 1), (0, 2), (1, 2)):
                pa, pb = perm[a], perm[b]
                idx.append(_PAIRS[(min(pa, pb), max(pa, pb))])
                sgn.append(signs[a] * signs[b])
            out_idx.append(idx)
            out_sgn.append(sgn)
    return np.array(out_idx), np.array(out_sgn, np.float32)


def augment(raw, tgt, copies, seed=0):
    """Training pairs plus `copies` images of each under random cube
    symmetries (host numpy; data marshalling before upload)."""
    idx, sgn = cube_symmetries()
    rng = np.random.default_rng(seed)
    raws, tgts = [raw], [tgt]
    for _ in range(copies):
        g = rng.integers(0, 48, raw.shape[0])
        r = raw.copy()
        r[:, :6] = np.take_along_axis(raw[:, :6], idx[g], axis=1) * sgn[g]
        raws.append(r)
        tgts.append(tgt)
    return np.concatenate(raws), np.concatenate(tgts)


def standardisation(raw):
    mean = raw.mean(0).astype(np.float64)
    std = raw.std(0).astype(np.float64)
    return mean, 1.0 / np.maximum(std, 1e-30)


def train(wlb, torch, raw, tgt, vraw, vtgt, epochs=200, batch=16384, lr=2e-3, seed=0):
    """Adam on the library's gradient kernel with a cosine learning-rate
    decay; the output bias starts at softplus^-1(mean target) so that the
    untrained network predicts the mean correction.  Returns the parameters
    with the lowest validation loss, the history and the loss scale."""
    mean, istd = standardisation(raw)
    t_mean = max(float(np.mean(tgt)), 1e-12)
    P = inputs.mlp_params(seed, mean=mean, inv_std=istd, out_bias=math.log(math.expm1(t_mean)))
    inv_scale = 1.0 / max(float(np.std(tgt)), 1e-30)
    dev = torch.device("cuda")
    s = torch.cuda.Stream()
    hist = []
    with torch.cuda.stream(s):  # every buffer op and library call on one stream
        Pd = torch.tensor(P, device=dev)
        m = torch.zeros_like(Pd)
        v = torch.zeros_like(Pd)
        g = torch.empty_like(Pd)
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        R = torch.tensor(raw, device=dev)
        T = torch.tensor(tgt, device=dev)
        VR = torch.tensor(vraw, device=dev)
        VT = torch.tensor(vtgt, device=dev)
        wsb = wlb.wlb_mlp_grad_workspace(max(batch, VT.numel()))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        step = 0
        total_steps = epochs * max(1, T.numel() // batch)
        best, best_P = float("inf"), None
        for ep in range(epochs):
            perm = torch.randperm(T.numel(), device=dev, generator=gen)
            tot, nb = 0.0, 0
            for b0 in range(0, T.numel() - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                rb = R[idx].contiguous()
                tb = T[idx].contiguous()
                wlb.wlb_mlp_grad(Pd.data_ptr(), rb.data_ptr(), tb.data_ptr(), batch, inv_scale, g.data_ptr(),
                                 loss.data_ptr(), ws.data_ptr(), wsb, s.cuda_stream)
                step += 1
                lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * min(step, total_steps) / total_steps))
                wlb.wlb_mlp_adam(Pd.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), step, max(lr_t, 1e-3 * lr),
                                 0.9, 0.999, 1e-8, s.cuda_stream)
                tot += float(loss.item())
                nb += 1
            wlb.wlb_mlp_grad(Pd.data_ptr(), VR.data_ptr(), VT.data_ptr(), VT.numel(), inv_scale, g.data_ptr(),
                             loss.data_ptr(), ws.data_ptr(), wsb, s.cuda_stream)
            vl = float(loss.item())
            hist.append({"epoch": ep, "train_loss": tot / max(nb, 1), "val_loss": vl})
            if vl < best:
                best, best_P = vl, Pd.cpu().numpy()
            if ep % 10 == 0 or ep == epochs - 1:
                _log(f"[les] epoch {ep}: train {tot / max(nb, 1):.4f} val {vl:.4f}")
        s.synchronize()
    return best_P, hist, inv_scale


def les_run(wlb, torch, rho_c, u_c, closure, params, steps, every, tau0, cs=0.1):
    """Coarse LES from (rho_c, u_c); returns kinetic energy every `every`
    steps and the final spectrum (None on divergence)."""
    n = rho_c.shape[-1]
    kw = dict(tau=tau0, closure=closure, cs_smag=cs, health_every=every, health_umax=0.5)
    if closure == wlb.CLOSURE_MLP:
        kw["mlp"] = params
    B = wlb.Blocks(wlb.single_block((n, n, n)), (n, n, n), (1, 1, 1), stencil=19, storage=wlb.F32)
    try:
        B.init(wlb.SRT, wlb.make_params(**kw), rho_c, u_c)
        energy = [float(B.moments(fields=False)[2][4])]
        t0 = time.time()
        for _ in range(0, steps, every):
            try:
                B.step(every)
            except wlb.WlbError as e:
                if e.code == wlb.WLB_ERR_DIVERGED:
                    return {"energy": energy, "spectrum": None, "diverged": True}
                raise
            energy.append(float(B.moments(fields=False)[2][4]))
        B.synchronize()
        dt = time.time() - t0
        _, uu, _ = B.moments()
        return {"energy": energy, "spectrum": shell_spectrum(uu).tolist(), "diverged": False,
                "mlups": n ** 3 * steps / dt / 1e6}
    finally:
        B.close()


def compare(run, ref, kmax):
    """Energy history error, and the final shell spectrum's error per shell
    over all resolved shells (k <= kmax) and over the well-resolved ones
    (k <= kmax / 4, where the box filter of the reference barely acts)."""
    e = np.asarray(run["energy"])
    er = np.asarray(ref["energy"])[: len(e)]
    out = {"energy_rel_err_max": float(np.max(np.abs(e - er) / er)),
           "energy_rel_err_final": float(abs(e[-1] - er[-1]) / er[-1]) if len(e) == len(ref["energy"]) else None}
    if run.get("spectrum") is not None:
        for key, km in (("spectrum_rel_err_max", kmax), ("spectrum_rel_err_max_low_k", max(1, kmax // 4))):
            s = np.asarray(run["spectrum"])[1:km + 1]
            sr = np.asarray(ref["spectrum"])[1:km + 1]
            ok = sr > 1e-30
            out[key] = float(np.max(np.abs(s[ok] - sr[ok]) / sr[ok]))
    return out


# Index of the output bias b3 in the packed parameters (the last value).
B3 = 7 + 7 + 32 * 7 + 32 + 32 * 32 + 32 + 32


def reference(wlb, torch, seed, n, factor, steps, snap, tau_f=TAU_F):
    """Filtered fine run of one seed: the coarse initial state, the filtered
    kinetic energy every `snap` fine steps and the final shell spectrum."""
    fr = FineRun(wlb, torch, seed, n, factor, tau_f=tau_f)
    rho_c, u_c = fr.coarse_state()
    energy = []
    for s in range(0, steps + 1, snap):
        if s > 0:
            fr.B.step(snap)
        energy.append(filtered_energy(fr.filtered()))
    _, u_end = fr.coarse_state()
    fr.close()
    return rho_c, u_c, {"energy": energy, "spectrum": shell_spectrum(u_end).tolist()}


def energy_error(run, ref):
    """Time-averaged relative kinetic-energy error of a coarse run against the
    filtered fine run (infinite when the coarse run blew up)."""
    if run["diverged"]:
        return float("inf")
    e = np.asarray(run["energy"])
    er = np.asarray(ref["energy"])[: len(e)]
    return float(np.mean(np.abs(e - er) / er))


def calibrate(wlb, torch, params, seeds, n, factor, steps, snap, tau_f=TAU_F,
              gains=(0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0), cs_values=(0.06, 0.08, 0.1, 0.13, 0.16, 0.2, 0.25)):
    """A-posteriori calibration against the fine solver: on held-out
    seeds, pick the gain g of the network's correction (applied as
    b3 += ln g, which scales softplus(o) by g wherever the correction is
    small, as it is here) and, for a fair comparison, the Smagorinsky
    constant, each minimising the time-averaged energy error."""
    tau0 = coarse_tau(factor, tau_f)
    csteps, cevery = steps // factor, snap // factor
    refs = [reference(wlb, torch, sd, n, factor, steps, snap, tau_f) for sd in seeds]
    table = {"gain": {}, "cs": {}}
    for g in gains:
        P = params.copy()
        P[B3] += np.float32(math.log(g))
        errs = [energy_error(les_run(wlb, torch, rc, uc, wlb.CLOSURE_MLP, P, csteps, cevery, tau0), ref)
                for rc, uc, ref in refs]
        table["gain"][str(g)] = float(np.mean(errs))
        _log(f"[les] calibration gain {g}: energy error {table['gain'][str(g)]:.4f}")
    for cs in cs_values:
        errs = [energy_error(les_run(wlb, torch, rc, uc, wlb.CLOSURE_SMAG, None, csteps, cevery, tau0, cs=cs), ref)
                for rc, uc, ref in refs]
        table["cs"][str(cs)] = float(np.mean(errs))
        _log(f"[les] calibration C_s {cs}: energy error {table['cs'][str(cs)]:.4f}")
    g_best = float(min(table["gain"], key=lambda k: table["gain"][k]))
    cs_best = float(min(table["cs"], key=lambda k: table["cs"][k]))
    return g_best, cs_best, table


def spsa_minimise(loss, z0, iters, c=0.1, step0=0.1, alpha=0.602, gamma=0.101, seed=0, log=None):
    """Simultaneous-perturbation stochastic approximation (Spall 1992):
    each iteration estimates the gradient of `loss` from two evaluations at
    z +- c_k Delta (Delta random signs), and steps z -= a_k g.  The gain a is
    set from the first gradient estimate so that the first step moves each
    coordinate by about step0.  Returns the best point evaluated and its
    loss, with the history of (iteration, loss+, loss-)."""
    rng = np.random.default_rng(seed)
    z = np.array(z0, np.float64)
    A = 0.1 * iters
    best_z, best_l = z.copy(), loss(z)
    hist = [(0, best_l, best_l)]
    a = None
    for k in range(iters):
        ck = c / (k + 1) ** gamma
        delta = rng.choice((-1.0, 1.0), size=z.size)
        lp, lm = loss(z + ck * delta), loss(z - ck * delta)
        hist.append((k + 1, lp, lm))
        for zz, ll in ((z + ck * delta, lp), (z - ck * delta, lm)):
            if ll < best_l:
                best_z, best_l = zz.copy(), ll
        if not (math.isfinite(lp) and math.isfinite(lm)):
            continue  # a divergent probe carries no slope
        g = (lp - lm) / (2 * ck) * delta
        if a is None:
            gm = float(np.abs(g).mean())
            if gm == 0.0:
                continue
            a = step0 * (A + 1) ** alpha / gm
        z = z - a / (k + 1 + A) ** alpha * g
        if log:
            log(f"[les] spsa {k + 1}/{iters}: loss+ {lp:.5f} loss- {lm:.5f} best {best_l:.5f}")
    return best_z, best_l, hist


def train_a_posteriori(wlb, torch, params, seeds, n, factor, steps, snap, tau_f=TAU_F, iters=40, c=0.1, step0=0.1):
    """Solver-in-the-loop training of the network's output layer (its 32
    weights and the bias): the loss of a parameter vector is the time-averaged
    kinetic-energy error of coarse LES runs with that network against the
    filtered fine runs of the same seeds, minimised by SPSA.  Coordinates are
    scaled by the spread of the output weights, so one unit moves every
    weight by about that much."""
    tau0 = coarse_tau(factor, tau_f)
    csteps, cevery = steps // factor, snap // factor
    refs = []
    for sd in seeds:
        refs.append(reference(wlb, torch, sd, n, factor, steps, snap, tau_f))
        _log(f"[les] reference seed {sd} done")
    lo = B3 - 32
    theta0 = params[lo:B3 + 1].astype(np.float64)
    scale = np.full(33, float(np.std(params[lo:B3])) or 1.0)

    def unpack(z):
        P = params.copy()
        P[lo:B3 + 1] = (theta0 + scale * z).astype(np.float32)
        return P

    def loss(z):
        P = unpack(z)
        errs = [energy_error(les_run(wlb, torch, rc, uc, wlb.CLOSURE_MLP, P, csteps, cevery, tau0), ref)
                for rc, uc, ref in refs]
        m = float(np.mean(errs))
        return m if math.isfinite(m) else float("inf")

    z, best, hist = spsa_minimise(loss, np.zeros(33), iters, c=c, step0=step0, log=_log)
    return unpack(z), best, hist


def evaluate(wlb, torch, seed, params, n, factor, steps, snap, tau_f=TAU_F, keep_series=False, variants=None):
    """A-posteriori comparison on a held-out seed: the coarse LES without a
    model, with Smagorinsky and with the network (and any extra
    (name, closure, params, C_s) variants), each against the filtered fine
    run.  keep_series adds the energy histories and final spectra."""
    tau0 = coarse_tau(factor, tau_f)
    rho_c, u_c, ref = reference(wlb, torch, seed, n, factor, steps, snap, tau_f)
    csteps, cevery = steps // factor, snap // factor
    nc = n // factor
    res = {}
    runs = [("none", wlb.CLOSURE_NONE, None, 0.1), ("smagorinsky", wlb.CLOSURE_SMAG, None, 0.1),
            ("mlp", wlb.CLOSURE_MLP, params, 0.1)] + list(variants or [])
    for name, cl, P, cs in runs:
        r = les_run(wlb, torch, rho_c, u_c, cl, P, csteps, cevery, tau0, cs=cs)
        res[name] = {"diverged": r["diverged"], "mlups": r.get("mlups"), "energy_err_mean": energy_error(r, ref),
                     **compare(r, ref, nc // 2)}
        e, er = np.asarray(r["energy"]), np.asarray(ref["energy"])[: len(r["energy"])]
        res[name]["energy_ratio_final"] = float(e[-1] / er[-1])
        if keep_series:
            res[name]["energy"] = [float(v) for v in r["energy"]]
            res[name]["spectrum"] = r.get("spectrum")
        _log(f"[les] a-posteriori {name}: " + json.dumps({k: v for k, v in res[name].items()
                                                           if k not in ("energy", "spectrum")}))
    if keep_series:
        res["reference"] = {"energy": [float(v) for v in ref["energy"]], "spectrum": ref["spectrum"]}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--factor", type=int, default=4)
    ap.add_argument("--steps", type=int, default=8000)
    ap.add_argument("--snap", type=int, default=400)
    ap.add_argument("--per-snap", type=int, default=2048)
    ap.add_argument("--seeds", type=str, default="0-19", help="phase data: seeds to run")
    ap.add_argument("--train-seeds", type=str, default="0-15")
    ap.add_argument("--val-seeds", type=str, default="16-19")
    ap.add_argument("--test-seed", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--augment", type=int, default=3, help="phase train: symmetry images per training pair")
    ap.add_argument("--calib-seeds", type=str, default="16-17", help="phase train: seeds of the a-posteriori calibration")
    ap.add_argument("--out", type=str, default="les_out")
    ap.add_argument("--phase", choices=["data", "train", "calib", "apost", "eval"], default="data")
    ap.add_argument("--iters", type=int, default=40, help="phase apost: SPSA iterations")
    ap.add_argument("--cs", type=float, default=0.055, help="phase apost: Smagorinsky constant compared against")
    ap.add_argument("--gains", type=str, default="0.15,0.25,0.35,0.5,0.7,1.0,1.5",
                    help="calibration: gains of the network's correction")
    ap.add_argument("--cs-values", type=str, default="0.03,0.045,0.06,0.08,0.1,0.13",
                    help="calibration: Smagorinsky constants")
    ap.add_argument("--tau-f", type=float, default=TAU_F, help="relaxation time of the fine runs")
    ap.add_argument("--params", type=str, default="",
                    help="phase eval / calib: network parameters (.npy); eval defaults to seeded ones")
    ap.add_argument("--data", type=str, default="", help="phase train: comma-separated npz files of pairs")
    args = ap.parse_args(argv)

    def seeds(spec):
        if not spec:
            return []
        if "-" in spec:
            a, b = spec.split("-")
            return list(range(int(a), int(b) + 1))
        return [int(x) for x in spec.split(",") if x]

    import torch

    from . import wlb
    os.makedirs(args.out, exist_ok=True)
    if args.phase == "data":
        sd = seeds(args.seeds)
        raw, tgt, _ = generate(wlb, torch, sd, args.n, args.factor, args.steps, args.snap, args.per_snap, sd[0] + 1,
                               tau_f=args.tau_f)
        name = f"pairs_{sd[0]}-{sd[-1]}.npz"
        np.savez_compressed(os.path.join(args.out, name), raw=raw, tgt=tgt, seed=generate.last_seed_ids)
        _log(f"[les] wrote {name}: {tgt.size} pairs")
        return 0
    if args.phase == "eval":
        P = np.load(args.params) if args.params else inputs.mlp_params(0, inv_std=[300.0] * 6 + [100.0],
                                                                         out_bias=-7.0)
        res = evaluate(wlb, torch, args.test_seed, P, args.n, args.factor, args.steps, args.snap, tau_f=args.tau_f,
                       keep_series=True)
        with open(os.path.join(args.out, f"eval_seed{args.test_seed}_tauf{args.tau_f}.json"), "w") as fh:
            json.dump(res, fh)
        return 0
    if args.phase == "apost":
        # solver-in-the-loop training of the output layer, starting from the
        # given (a-priori trained, gain-calibrated) network
        P0 = np.load(args.params)
        cal = seeds(args.calib_seeds)
        t0 = time.time()
        Pa, best, hist = train_a_posteriori(wlb, torch, P0, cal, args.n, args.factor, args.steps, args.snap,
                                            tau_f=args.tau_f, iters=args.iters)
        np.save(os.path.join(args.out, "mlp_params_aposteriori.npy"), Pa)
        res = evaluate(wlb, torch, args.test_seed, P0, args.n, args.factor, args.steps, args.snap, tau_f=args.tau_f,
                       keep_series=True, variants=[("smagorinsky_calibrated", wlb.CLOSURE_SMAG, None, args.cs),
                                                   ("mlp_aposteriori", wlb.CLOSURE_MLP, Pa, 0.1)])
        out = {"start_params": args.params, "train_seeds": cal, "test_seed": args.test_seed, "iters": args.iters,
               "loss_start": hist[0][1], "loss_best": best, "history": hist, "seconds": time.time() - t0,
               "a_posteriori": res}
        with open(os.path.join(args.out, "apost_summary.json"), "w") as fh:
            json.dump(out, fh, indent=1)
        return 0
    tr, va = seeds(args.train_seeds), seeds(args.val_seeds)
    summary = {"n_fine": args.n, "factor": args.factor, "steps_fine": args.steps, "snap": args.snap,
               "tau_f": args.tau_f, "tau_coarse": coarse_tau(args.factor, args.tau_f), "train_seeds": tr,
               "val_seeds": va, "test_seed": args.test_seed}
    if args.phase == "train":
        parts = [np.load(f) for f in args.data.split(",") if f]
        raw = np.concatenate([p["raw"] for p in parts])
        tgt = np.concatenate([p["tgt"] for p in parts])
        sid = np.concatenate([p["seed"] for p in parts])
        mt, mv = np.isin(sid, tr), np.isin(sid, va)
        ra, ta = augment(raw[mt], tgt[mt], args.augment)
        P, hist, inv_scale = train(wlb, torch, ra, ta, raw[mv], tgt[mv], epochs=args.epochs)
        np.save(os.path.join(args.out, "mlp_params_apriori.npy"), P)
        summary.update({"train_pairs": int(mt.sum()), "val_pairs": int(mv.sum()), "augment_images": args.augment,
                        "history": hist, "inv_scale": inv_scale})
    else:  # calib: the a-priori network from an earlier training run
        P = np.load(args.params)
        summary["params"] = args.params
    cal_seeds = seeds(args.calib_seeds)
    gains = tuple(float(v) for v in args.gains.split(","))
    cs_values = tuple(float(v) for v in args.cs_values.split(","))
    g, cs, table = calibrate(wlb, torch, P, cal_seeds, args.n, args.factor, args.steps, args.snap, tau_f=args.tau_f,
                             gains=gains, cs_values=cs_values)
    Pc = P.copy()
    Pc[B3] += np.float32(math.log(g))
    np.save(os.path.join(args.out, "mlp_params.npy"), Pc)
    res = evaluate(wlb, torch, args.test_seed, P, args.n, args.factor, args.steps, args.snap, tau_f=args.tau_f,
                   keep_series=True, variants=[("smagorinsky_calibrated", wlb.CLOSURE_SMAG, None, cs),
                                               ("mlp_calibrated", wlb.CLOSURE_MLP, Pc, 0.1)])
    summary.update({"calibration_seeds": cal_seeds, "calibration": table, "gain": g, "cs_calibrated": cs,
                    "a_posteriori": res})
    with open(os.path.join(args.out, "summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
