"""GPU parity of the LES training-data kernels (box filter, targets) against
the numpy FP64 oracle in oracle/les.py."""
import numpy as np
import pytest

from gpu_util import inputs, say

pytestmark = pytest.mark.gpu

wlb = pytest.importorskip("paper_1909_13772_amd.wlb", reason="libwlb.so not built")
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("steps", [0, 3])
def test_box_filter_and_targets_match_oracle(steps):
    from oracle import les
    say(f"case les filter steps{steps}")
    n, f = 32, 4
    shape = (n, n, n)
    rho, u = inputs.turbulence_bandlimited(n, seed=2, u_rms=0.03)
    B = wlb.Blocks(wlb.single_block(shape), shape, (1, 1, 1), stencil=19, storage=wlb.F64)
    B.init(wlb.SRT, wlb.make_params(tau=0.6), rho, u)
    B.step(steps)
    r, uu, _ = B.moments()
    nc = n // f
    out = torch.empty(10 * nc ** 3, dtype=torch.float64, device="cuda")
    wlb.wlb_box_filter(B.h, f, out.data_ptr())
    F_gpu = out.cpu().numpy().reshape(10, nc, nc, nc)
    F_orc = les.box_filter(r, uu, f)
    err = np.abs(F_gpu - F_orc).max()
    say(f"filter max abs err {err:.3e}")
    assert err < 1e-14
    raw = torch.empty(nc ** 3 * 7, dtype=torch.float32, device="cuda")
    tgt = torch.empty(nc ** 3, dtype=torch.float32, device="cuda")
    wlb.wlb_les_targets(out.data_ptr(), (nc, nc, nc), 0.5075, raw.data_ptr(), tgt.data_ptr(), B.stream.cuda_stream)
    B.synchronize()
    raw_o, tgt_o = les.les_targets(F_gpu, 0.5075)
    rg = raw.cpu().numpy().reshape(-1, 7).astype(np.float64)
    tg = tgt.cpu().numpy().astype(np.float64)
    assert np.abs(tg - tgt_o).max() <= 1e-6 * max(tgt_o.max(), 1e-12)
    assert np.abs(rg - raw_o).max() <= 1e-6 * np.abs(raw_o).max()
    B.close()


def test_learned_closure_pipeline_small():
    """Fine runs -> filtered pairs -> training with the library's kernels ->
    a-posteriori LES, at toy size (the full-size numbers are a separate run)."""
    from paper_1909_13772_amd import les
    say("case les pipeline small")
    n, f = 32, 4
    raw, tgt, refs = les.generate(wlb, torch, [0, 1], n, f, 40, 20, 256, rng_seed=1)
    vraw, vtgt, _ = les.generate(wlb, torch, [2], n, f, 40, 20, 256, rng_seed=2)
    assert raw.shape == (2 * 3 * 256, 7) and np.all(np.isfinite(raw)) and np.all(tgt >= 0)
    P, hist, _ = les.train(wlb, torch, raw, tgt, vraw, vtgt, epochs=3, batch=256)
    assert np.all(np.isfinite(P)) and len(hist) == 3
    assert hist[-1]["train_loss"] <= hist[0]["train_loss"] * 1.5
    g, cs, table = les.calibrate(wlb, torch, P, [2], n, f, 40, 20, gains=(1.0, 2.0), cs_values=(0.1, 0.2))
    assert g in (1.0, 2.0) and cs in (0.1, 0.2) and len(table["gain"]) == 2
    Pc = P.copy()
    Pc[les.B3] += np.float32(np.log(g))
    res = les.evaluate(wlb, torch, 3, P, n, f, 40, 20, variants=[("mlp_calibrated", wlb.CLOSURE_MLP, Pc, 0.1)])
    for name in ("none", "smagorinsky", "mlp", "mlp_calibrated"):
        assert name in res
    assert not res["smagorinsky"]["diverged"]


def test_trained_closure_keeps_the_coarse_les_stable():
    """What the trained network gains over the method without it, at the
    closure's own working point (128^3, tau0 = 0.5025, decaying turbulence):
    without a model the coarse run blows up within 2000 steps; with the
    committed trained network (and with Smagorinsky) it stays healthy and
    its kinetic energy decays.  The full comparison against the filtered
    512^3 fine run is recorded in paper_1909_13772_amd/mlp_closure_record.json
    (written by `python -m paper_1909_13772_amd.les --phase calib`)."""
    import os

    from paper_1909_13772_amd import les
    say("case trained closure stability 128^3")
    path = os.path.join(os.path.dirname(les.__file__), "mlp_closure.npy")
    P = np.load(path)
    assert P.shape == (wlb.MLP_NPARAM,)
    n = 128
    rho, u = inputs.turbulence_bandlimited(n, 20)
    tau0 = les.coarse_tau(4)
    runs = {}
    for name, cl in (("none", wlb.CLOSURE_NONE), ("smagorinsky", wlb.CLOSURE_SMAG), ("mlp", wlb.CLOSURE_MLP)):
        runs[name] = les.les_run(wlb, torch, rho, u, cl, P if cl == wlb.CLOSURE_MLP else None, 2000, 100, tau0)
        say(f"{name}: diverged {runs[name]['diverged']}, energy {runs[name]['energy'][:1]} -> {runs[name]['energy'][-1:]}")
    assert runs["none"]["diverged"]
    for name in ("smagorinsky", "mlp"):
        r = runs[name]
        assert not r["diverged"] and len(r["energy"]) == 21
        e = np.asarray(r["energy"])
        assert np.all(np.isfinite(e)) and e[-1] < 0.5 * e[0]


def test_solver_in_the_loop_training_small():
    """Solver-in-the-loop training of the output layer at toy size: a 32^3
    fine run per seed filtered to 8^3, two SPSA iterations whose every loss
    is a coarse LES run of the library against the filtered fine run.  The
    losses are finite, the point returned is the best one evaluated (its
    loss is recomputed and matches, runs being deterministic), and only the
    33 output-layer parameters move."""
    from paper_1909_13772_amd import les
    say("case les solver-in-the-loop small")
    n, f = 32, 4
    P0 = inputs.mlp_params(5, mean=np.zeros(7), inv_std=np.array([400.0] * 6 + [150.0]), out_bias=-2.0)
    P, best, hist = les.train_a_posteriori(wlb, torch, P0, [0], n, f, 40, 20, iters=2)
    assert len(hist) == 3
    losses = [hist[0][1]] + [v for h in hist[1:] for v in h[1:]]
    assert all(np.isfinite(losses)), losses
    assert best == min(losses)
    lo, hi = les.B3 - 32, les.B3 + 1
    assert np.array_equal(P[:lo], P0[:lo]) and np.array_equal(P[hi:], P0[hi:])
    # the returned parameters reproduce the best loss
    tau0 = les.coarse_tau(f)
    rc, uc, ref = les.reference(wlb, torch, 0, n, f, 40, 20)
    run = les.les_run(wlb, torch, rc, uc, wlb.CLOSURE_MLP, P, 40 // f, 20 // f, tau0)
    assert abs(les.energy_error(run, ref) - best) <= 1e-12 * max(1.0, best)
