"""Host-side logic of the learned-closure pipeline (no GPU): the cube
symmetries used to augment training pairs, the coarse relaxation time of the
acoustic scaling, and the shell spectrum."""
import itertools
import math

import numpy as np

from paper_1909_13772_amd import les


def _comp(M):
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def test_cube_symmetries_rotate_the_stress_tensor():
    idx, sgn = les.cube_symmetries()
    assert idx.shape == (48, 6)
    rng = np.random.default_rng(0)
    A = rng.normal(size=(3, 3))
    A = A + A.T
    for g, (perm, signs) in enumerate((p, s) for p in itertools.permutations(range(3))
                                      for s in itertools.product((1, -1), repeat=3)):
        P = np.zeros((3, 3))
        for a in range(3):
            P[a, perm[a]] = signs[a]
        assert np.allclose(_comp(A)[idx[g]] * sgn[g], _comp(P @ A @ P.T))
    # the point inversion acts trivially on a rank-2 tensor: 24 distinct maps
    assert len({tuple(i) + tuple(s) for i, s in zip(idx, sgn)}) == 24


def test_augment_keeps_invariants_and_targets():
    rng = np.random.default_rng(1)
    raw = rng.normal(size=(50, 7)).astype(np.float32)
    tgt = rng.random(50).astype(np.float32)
    ra, ta = les.augment(raw, tgt, 3, seed=2)
    assert ra.shape == (200, 7) and ta.shape == (200,)
    assert np.array_equal(ra[:50], raw)
    for k in range(4):
        blk = ra[50 * k:50 * (k + 1)]
        assert np.array_equal(blk[:, 6], raw[:, 6])
        assert np.array_equal(ta[50 * k:50 * (k + 1)], tgt)
        assert np.allclose(blk[:, :3].sum(1), raw[:, :3].sum(1), atol=1e-5)
        fro = lambda x: (x[:, :3] ** 2).sum(1) + 2 * (x[:, 3:6] ** 2).sum(1)
        assert np.allclose(fro(blk), fro(raw), rtol=1e-5)


def test_coarse_tau_keeps_the_physical_viscosity():
    # acoustic scaling: dx and dt grow by the factor, nu_lattice shrinks by it
    for tau_f, f in ((0.53, 4), (0.51, 4), (0.6, 2)):
        nu_f = (tau_f - 0.5) / 3
        assert abs((les.coarse_tau(f, tau_f) - 0.5) / 3 - nu_f / f) < 1e-15


def test_shell_spectrum_single_mode():
    n = 16
    x = np.arange(n)
    u = np.zeros((3, n, n, n))
    u[1] = np.broadcast_to(0.1 * np.cos(2 * np.pi * 3 * x / n)[None, None, :], (n, n, n))
    e = les.shell_spectrum(u)
    # mean of u^2 / 2 over the box, all of it in shell k = 3
    assert abs(e[3] - 0.5 * 0.1 ** 2 / 2) < 1e-15
    assert abs(e.sum() - e[3]) < 1e-15


def test_output_bias_index_is_the_last_parameter():
    # packed layout mean[7], inv_std[7], W1[32][7], b1[32], W2[32][32], b2[32], w3[32], b3
    from paper_1909_13772_amd import inputs
    P = inputs.mlp_params(0, out_bias=-3.25)
    assert les.B3 == P.size - 1 == 1358 and P[les.B3] == np.float32(-3.25)


def test_gain_as_output_bias_shift():
    # g softplus(o) ~ softplus(o + ln g) where softplus(o) is small
    o = np.linspace(-10.0, -5.0, 11)
    sp = np.log1p(np.exp(o))
    for g in (0.5, 2.0, 6.0):
        assert np.all(np.abs(np.log1p(np.exp(o + np.log(g))) / (g * sp) - 1) < 0.02)


def test_spsa_descends_a_quadratic_and_returns_its_best_point():
    """SPSA on a convex quadratic in 33 dimensions (the size of the output
    layer) must cut the loss several-fold, and the point it returns must be
    the best one it evaluated."""
    rng = np.random.default_rng(0)
    H = rng.normal(size=(33, 33))
    H = H @ H.T / 33 + np.eye(33)
    z0 = rng.normal(size=33)
    seen = []

    def f(z):
        v = float(0.5 * z @ H @ z)
        seen.append(v)
        return v

    z, best, hist = les.spsa_minimise(f, z0, 60, c=0.1, step0=0.1)
    assert best < 0.5 * f(z0)
    assert abs(f(z) - best) < 1e-12 and best <= min(seen) + 1e-12
    assert len(hist) == 61


def test_spsa_skips_divergent_probes():
    """A probe whose loss is infinite (a coarse run that blew up) gives no
    slope: the iterate must stay finite and the best point finite."""
    def f(z):
        return float("inf") if z[0] > 0.5 else float((z ** 2).sum())

    z, best, _ = les.spsa_minimise(f, np.full(4, 0.4), 30, c=0.2, step0=0.05, seed=3)
    assert np.all(np.isfinite(z)) and math.isfinite(best) and best <= 4 * 0.16
