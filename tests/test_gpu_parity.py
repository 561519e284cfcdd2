"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  FP64 storage must agree to 1e-12 (relative L2 of the
velocity over fluid cells, and max population error relative to max |f|);
FP32 storage to 1e-5, FP16 storage to 1e-3 (velocity relative L2); BF16
storage is reported against a looser 1e-2 bound (8 significand bits).  The
velocity's max norm (max |u - u_ref| / max |u_ref|) is bounded too, for the
reduced-precision forms by 3 times the L2 bound: the accuracy targets are
stated on the L2 norm, and the largest cell error of a rounding-noise field
sits a few standard deviations above its mean.
Block
decomposition, tile shape, persistent grid, graph replay and sweep/exchange
splitting must not change a single bit."""
import math

import numpy as np
import pytest

from gpu_util import fluid_mask, gpu_run, inputs, oracle_params, oracle_run, pop_err, rel_l2, say

pytestmark = pytest.mark.gpu

wlb = pytest.importorskip("paper_1909_13772_amd.wlb", reason="libwlb.so not built")

TOL = {wlb.F64: 1e-12, wlb.F32: 1e-5, wlb.F16DEV: 1e-3, wlb.BF16DEV: 1e-2}
TOL_MAX = {wlb.F64: 1e-12, wlb.F32: 3e-5, wlb.F16DEV: 3e-3, wlb.BF16DEV: 3e-2}


def _compare(case, storage, q, gpu, orc, solid, n, check_pops=True):
    d, r, u, tot, B = gpu
    do, ro, uo, to = orc
    B.close()
    m = fluid_mask(solid, n)
    uu = u.reshape(3, -1)
    eu = rel_l2(uu, uo, m)
    emax = np.abs(uu[:, m] - uo[:, m]).max() / max(np.abs(uo[:, m]).max(), 1e-300)
    er = np.abs(r.reshape(-1)[m] - ro[m]).max()
    ep = pop_err(d[:, m], do[:, m], q)
    say(f"{case}: u rel L2 {eu:.3e}, u max norm {emax:.3e}, rho max {er:.3e}, pops {ep:.3e}")
    tol = TOL[storage]
    assert eu <= tol, (case, eu)
    assert emax <= TOL_MAX[storage], (case, emax)
    if check_pops and storage == wlb.F64:
        assert ep <= tol, (case, ep)
        assert er <= 1e-12
    return eu


# ---------------------------------------------------------------------------
def test_taylor_green_32_fp64_100_steps():
    """Periodic 32^3 block, D3Q19 SRT, tau 0.8, TGV u0 = 0.01, 100 steps."""
    say("case tgv32 fp64")
    n, steps, tau = 32, 100, 0.8
    shape = (n, n, n)
    rho, u = inputs.taylor_green(n, 0.01)
    p = wlb.make_params(tau=tau)
    gpu = gpu_run(wlb.single_block(shape), shape, (1, 1, 1), 19, wlb.F64, wlb.SRT, p, rho, u, steps=steps)
    orc = oracle_run(oracle_params(19, 0, tau, 0, (1, 1, 1)), shape, rho, u, None, steps)
    _compare("tgv32", wlb.F64, 19, gpu, orc, None, n ** 3)
    tot = gpu[3]
    # exact mass conservation and the analytic energy decay
    assert abs(tot[0] - n ** 3) < 1e-9
    e0 = 0.5 * (u ** 2).sum()
    k = 2 * math.pi / n
    exact = math.exp(-4 * (tau - 0.5) / 3 * k * k * steps)
    assert abs(tot[4] / e0 - exact) < 0.02 * exact


def _plane(q, u, F):
    """D2Q9 has no z velocities: start it without u_z and F_z."""
    if q == 9:
        u = u.copy()
        u[2] = 0.0
        F = (F[0], F[1], 0.0)
    return u, F


@pytest.mark.parametrize("q,coll", [(19, 0), (19, 1), (19, 2), (27, 0), (27, 1), (27, 2), (27, 3), (27, 4),
                                    (9, 0), (9, 1), (15, 0), (15, 1)])
@pytest.mark.parametrize("steps", [6, 7])
def test_random_state_periodic_fp64(q, coll, steps):
    """Ragged 20x18x17 periodic box, random state, body force, every operator
    and velocity set."""
    say(f"case random q{q} coll{coll} steps{steps}")
    shape = (20, 18, 17)
    rho, u = inputs.random_state(shape, seed=q + coll)
    u, F = _plane(q, u, (1e-5, -2e-5, 3e-6))
    kw = dict(tau=0.7, magic=0.11, omega_bulk=1.3, omega_higher=1.1, force=F)
    p = wlb.make_params(**kw)
    gpu = gpu_run(wlb.single_block(shape), shape, (1, 1, 1), q, wlb.F64, coll, p, rho, u, steps=steps)
    op = oracle_params(q, coll, 0.7, 0.11, (1, 1, 1), F, omega_bulk=1.3, omega_higher=1.1)
    orc = oracle_run(op, shape, rho, u, None, steps)
    _compare(f"random q{q} c{coll} s{steps}", wlb.F64, q, gpu, orc, None, np.prod(shape))


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (9, 1), (15, 1)])
def test_channel_walls_force_fp64(q, coll):
    say(f"case channel q{q}")
    shape = (24, 20, 12)
    rho, u = inputs.random_state(shape, seed=5, umag=0.01)
    u, F = _plane(q, u, (2e-5, 0, 0))
    p = wlb.make_params(tau=0.8, magic=3 / 16, force=F, omega_bulk=1.2, omega_higher=0.9)
    gpu = gpu_run(wlb.single_block(shape), shape, (1, 0, 1), q, wlb.F64, coll, p, rho, u, steps=9)
    op = oracle_params(q, coll, 0.8, 3 / 16, (1, 0, 1), F, omega_bulk=1.2, omega_higher=0.9)
    orc = oracle_run(op, shape, rho, u, None, 9)
    _compare(f"channel q{q}", wlb.F64, q, gpu, orc, None, np.prod(shape))


def _porous_case(q, coll, storage, steps, seed=1, **kw):
    blocks, dom = inputs.rectilinear_blocks([8, 12, 6], [10, 6], [7, 9])
    solid, frac, _ = inputs.spheres(dom, seed=seed, rmin=2.0, rmax=4.0, solid_fraction=0.2, clear_x=2)
    rho, u = inputs.random_state(dom, seed=seed + 10, umag=0.01)
    u, _ = _plane(q, u, (0, 0, 0))
    p = wlb.make_params(tau=0.8, magic=3 / 16, omega_bulk=1.2, omega_higher=1.0, pressure_axis=0,
                        rho_in=1.002, rho_out=0.998)
    gpu = gpu_run(blocks, dom, (0, 1, 1), q, storage, coll, p, rho, u, solid, steps=steps, **kw)
    op = oracle_params(q, coll, 0.8, 3 / 16, (0, 1, 1), pressure_axis=0, rho_in=1.002, rho_out=0.998,
                       omega_bulk=1.2, omega_higher=1.0)
    orc = oracle_run(op, dom, rho, u, solid, steps)
    return gpu, orc, solid, dom


@pytest.mark.parametrize("q,coll", [(27, 2), (19, 0), (19, 1), (19, 2), (27, 3), (27, 4), (9, 1), (15, 0), (15, 1)])
@pytest.mark.parametrize("steps", [10, 11])
def test_porous_uneven_blocks_pressure_fp64(q, coll, steps):
    """Uneven rectilinear blocks (3 x 2 x 2), spheres, density faces on x,
    periodic y/z: exercises masks, bounce-back, anti-bounce-back and the
    exchange in both directions."""
    say(f"case porous q{q} coll{coll} steps{steps}")
    gpu, orc, solid, dom = _porous_case(q, coll, wlb.F64, steps)
    _compare(f"porous q{q} c{coll}", wlb.F64, q, gpu, orc, solid, np.prod(dom))


@pytest.mark.parametrize("q,coll,storage", [(27, 2, 0), (19, 1, 0), (27, 2, 1), (19, 1, 1)])
def test_porous_uneven_blocks_long_run(q, coll, storage):
    """The porous case over 400 steps (the density difference drives the flow
    through the spheres until it develops), autotuned as the workload runs:
    FP64 element-wise to 1e-12 on the populations, FP32 to its velocity
    bounds."""
    say(f"case porous long q{q} coll{coll} storage{storage}")
    blocks, dom = inputs.rectilinear_blocks([8, 12, 6], [10, 6], [7, 9])
    solid, frac, _ = inputs.spheres(dom, seed=3, rmin=2.0, rmax=4.0, solid_fraction=0.2, clear_x=2)
    rho, u = inputs.uniform_state(dom)
    p = wlb.make_params(tau=0.8, magic=3 / 16, omega_bulk=1.2, omega_higher=1.0, pressure_axis=0,
                        rho_in=1.002, rho_out=0.998, autotune=1)
    gpu = gpu_run(blocks, dom, (0, 1, 1), q, storage, coll, p, rho, u, solid, steps=400)
    op = oracle_params(q, coll, 0.8, 3 / 16, (0, 1, 1), pressure_axis=0, rho_in=1.002, rho_out=0.998,
                       omega_bulk=1.2, omega_higher=1.0)
    orc = oracle_run(op, dom, rho, u, solid, 400)
    _compare(f"porous long q{q} c{coll}", storage, q, gpu, orc, solid, np.prod(dom))


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (9, 1), (15, 1)])
def test_porous_uneven_blocks_lds_staged_odd_sweep_fp64(q, coll):
    """The porous case with the odd sweep staged in LDS: x-neighbour blocks
    supply the halo elements and take the stores past the row segment."""
    say(f"case porous lds-staged q{q} coll{coll}")
    gpu, orc, solid, dom = _porous_case(q, coll, wlb.F64, 11, lds=True)
    assert gpu[4].info().lds_staging == 1
    _compare(f"porous lds q{q} c{coll}", wlb.F64, q, gpu, orc, solid, np.prod(dom))


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2)])
@pytest.mark.parametrize("nt,lds", [((0, 0), False), ((0, 0), True), ((1, 0), False), ((1, 2), False)])
def test_porous_uneven_blocks_cached_accesses_fp64(q, coll, nt, lds):
    """The porous case with ordinary (cached) instead of non-temporal
    population accesses in one or both sweeps, or the odd sweep's hint on
    its aligned accesses only."""
    say(f"case porous nt{nt} lds{lds} q{q} coll{coll}")
    gpu, orc, solid, dom = _porous_case(q, coll, wlb.F64, 11, nt=nt, lds=lds)
    i = gpu[4].info()
    assert (i.nt_even, i.nt_odd) == nt
    _compare(f"porous nt{nt} q{q} c{coll}", wlb.F64, q, gpu, orc, solid, np.prod(dom))


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (9, 1), (15, 1)])
def test_porous_uneven_blocks_overlapped_exchange_fp64(q, coll):
    """The porous case with each sweep split into interior and frontier and
    the frontier plus the exchange on a second stream."""
    say(f"case porous overlap q{q} coll{coll}")
    gpu, orc, solid, dom = _porous_case(q, coll, wlb.F64, 11, overlap=True)
    assert gpu[4].info().overlap == 1
    _compare(f"porous overlap q{q} c{coll}", wlb.F64, q, gpu, orc, solid, np.prod(dom))


def test_kbc_fp32_storage_vs_fp64_oracle():
    """KBC with FP32 populations (FP32 collision, entropic products in FP32)
    against the FP64 oracle on a random periodic state with a body force."""
    say("case kbc fp32")
    dom = (20, 12, 10)
    rho, u = inputs.random_state(dom, seed=21, umag=0.05)
    F = (1e-5, -2e-6, 0.0)
    p = wlb.make_params(tau=0.52, force=F)
    gpu = gpu_run(wlb.single_block(dom), dom, (1, 1, 1), 27, wlb.F32, wlb.KBC, p, rho, u, steps=9)
    orc = oracle_run(oracle_params(27, wlb.KBC, 0.52, 0, (1, 1, 1), F), dom, rho, u, None, 9)
    _compare("kbc fp32", wlb.F32, 27, gpu, orc, None, np.prod(dom))


def test_cumulant_fp32_storage_vs_fp64_oracle():
    """The cumulant collision with FP32 populations against the FP64 oracle
    on a random periodic state with a body force and a bulk rate."""
    say("case cumulant fp32")
    dom = (20, 12, 10)
    rho, u = inputs.random_state(dom, seed=23, umag=0.05)
    F = (1e-5, -2e-6, 3e-6)
    p = wlb.make_params(tau=0.53, omega_bulk=1.3, force=F)
    gpu = gpu_run(wlb.single_block(dom), dom, (1, 1, 1), 27, wlb.F32, wlb.CUMULANT, p, rho, u, steps=9)
    orc = oracle_run(oracle_params(27, wlb.CUMULANT, 0.53, 0, (1, 1, 1), F, omega_bulk=1.3), dom, rho, u, None, 9)
    _compare("cumulant fp32", wlb.F32, 27, gpu, orc, None, np.prod(dom))


@pytest.mark.parametrize("coll", [3, 4])
def test_kbc_and_cumulant_need_d3q27(coll):
    dom = (8, 6, 4)
    rho, u = inputs.uniform_state(dom)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=19, storage=wlb.F64)
    try:
        with pytest.raises(wlb.WlbError) as e:
            B.init(coll, wlb.make_params(tau=0.8), rho, u)
        assert e.value.code == wlb.WLB_ERR_UNSUPPORTED
    finally:
        B.close()


@pytest.mark.parametrize("q,coll", [(9, 2), (15, 2), (15, 3), (9, 4)])
def test_moment_space_collisions_need_d3q19_or_d3q27(q, coll):
    dom = (8, 6, 4)
    rho, u = inputs.uniform_state(dom)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=q, storage=wlb.F64)
    try:
        with pytest.raises(wlb.WlbError) as e:
            B.init(coll, wlb.make_params(tau=0.8), rho, u)
        assert e.value.code == wlb.WLB_ERR_UNSUPPORTED
    finally:
        B.close()


@pytest.mark.parametrize("q,storage", [(9, 1), (15, 1), (9, 2), (15, 2)])
def test_small_sets_reduced_precision_vs_fp64_oracle(q, storage):
    """D2Q9 / D3Q15 TRT with FP32 and FP16 deviation storage, Smagorinsky
    closure on, against the FP64 oracle."""
    say(f"case small sets q{q} storage{storage}")
    shape = (24, 20, 16)
    rho, u = inputs.random_state(shape, seed=12, umag=0.03)
    u, _ = _plane(q, u, (0, 0, 0))
    p = wlb.make_params(tau=0.6, magic=3 / 16, closure=wlb.CLOSURE_SMAG, cs_smag=0.1)
    gpu = gpu_run(wlb.single_block(shape), shape, (1, 1, 1), q, storage, wlb.TRT, p, rho, u, steps=20)
    orc = oracle_run(oracle_params(q, 1, 0.6, 3 / 16, (1, 1, 1), closure=1, cs_smag=0.1), shape, rho, u, None, 20)
    _compare(f"small q{q} {storage}", storage, q, gpu, orc, None, np.prod(shape), check_pops=False)


@pytest.mark.parametrize("coll", [0, 1])
def test_smagorinsky_fp64(coll):
    say(f"case smagorinsky coll{coll}")
    shape = (16, 12, 10)
    rho, u = inputs.random_state(shape, seed=7, umag=0.05)
    p = wlb.make_params(tau=0.5075, magic=3 / 16, closure=wlb.CLOSURE_SMAG, cs_smag=0.1)
    gpu = gpu_run(wlb.single_block(shape), shape, (1, 1, 1), 19, wlb.F64, coll, p, rho, u, steps=8)
    op = oracle_params(19, coll, 0.5075, 3 / 16, (1, 1, 1), closure=1, cs_smag=0.1)
    orc = oracle_run(op, shape, rho, u, None, 8)
    _compare(f"smag c{coll}", wlb.F64, 19, gpu, orc, None, np.prod(shape))


@pytest.mark.parametrize("q", [19, 27])
def test_smagorinsky_mrt_fp64(q):
    """MRT with the Smagorinsky rate taken from the non-equilibrium moments,
    with a body force on every axis."""
    say(f"case smagorinsky mrt q{q}")
    shape = (12, 10, 9)
    rho, u = inputs.random_state(shape, seed=8, umag=0.05)
    F = (2e-5, -1e-5, 4e-6)
    p = wlb.make_params(tau=0.52, closure=wlb.CLOSURE_SMAG, cs_smag=0.1, omega_bulk=1.1, omega_higher=1.0, force=F)
    gpu = gpu_run(wlb.single_block(shape), shape, (1, 1, 1), q, wlb.F64, 2, p, rho, u, steps=5)
    op = oracle_params(q, 2, 0.52, 0, (1, 1, 1), F, closure=1, cs_smag=0.1, omega_bulk=1.1, omega_higher=1.0)
    orc = oracle_run(op, shape, rho, u, None, 5)
    _compare(f"smag mrt q{q}", wlb.F64, q, gpu, orc, None, np.prod(shape))


@pytest.mark.parametrize("storage", [1, 2, 3])
def test_reduced_precision_storage_vs_fp64_oracle(storage):
    """FP32 / FP16 / BF16 deviation storage with FP32 collision against the
    FP64 oracle (velocity relative L2)."""
    say(f"case precision storage{storage}")
    shape = (24, 20, 16)
    rho, u = inputs.random_state(shape, seed=11, umag=0.03)
    p = wlb.make_params(tau=0.6, magic=3 / 16)
    gpu = gpu_run(wlb.single_block(shape), shape, (1, 1, 1), 19, storage, wlb.TRT, p, rho, u, steps=20)
    orc = oracle_run(oracle_params(19, 1, 0.6, 3 / 16, (1, 1, 1)), shape, rho, u, None, 20)
    _compare(f"precision {storage}", storage, 19, gpu, orc, None, np.prod(shape), check_pops=False)


@pytest.mark.parametrize("storage", [1, 2])
def test_reduced_precision_porous(storage):
    say(f"case precision porous storage{storage}")
    gpu, orc, solid, dom = _porous_case(27, 2, storage, 12)
    _compare(f"porous prec {storage}", storage, 27, gpu, orc, solid, np.prod(dom), check_pops=False)


# ---------------------------------------------------------------------------
# Bitwise invariances of the GPU path
# ---------------------------------------------------------------------------
def _porous_inputs(dom, seed=3):
    solid, _, _ = inputs.spheres(dom, seed=seed, rmin=2.0, rmax=3.5, solid_fraction=0.15, clear_x=2)
    rho, u = inputs.random_state(dom, seed=seed, umag=0.01)
    return solid, rho, u


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_block_decomposition_is_bitwise_invariant(storage):
    say(f"case decomposition storage{storage}")
    dom = (48, 32, 24)
    solid, rho, u = _porous_inputs(dom)
    p = wlb.make_params(tau=0.7, magic=3 / 16, omega_bulk=1.1, omega_higher=1.0, pressure_axis=0, rho_in=1.001,
                        rho_out=0.999)
    layouts = [wlb.single_block(dom), inputs.uniform_blocks(dom, (16, 16, 8))[0],
               inputs.rectilinear_blocks([16, 8, 24], [10, 22], [4, 12, 8])[0]]
    ref = None
    for k, bl in enumerate(layouts):
        for steps in (9,):
            d, r, uu, tot, B = gpu_run(bl, dom, (0, 1, 1), 27, storage, 2, p, rho, u, solid, steps=steps)
            B.close()
            if ref is None:
                ref = d
            else:
                assert np.array_equal(d, ref), f"layout {k} differs"


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (15, 1), (9, 0)])
@pytest.mark.parametrize("variant", ["rows", "segments", "direct", "direct-segments"])
def test_x_wrap_with_solids_across_the_periodic_face_fp64(q, coll, variant):
    """One block periodic in x (x accesses wrap, no x exchange) with spheres
    straddling the periodic x face, a body force and walls in y.  Odd sweep
    staged in LDS over whole rows (the shift wraps inside the row buffer) or
    over row segments (halo elements wrap in memory), or direct (lane to
    lane moves, with several row segments per wavefront)."""
    say(f"case x-wrap solids q{q} coll{coll} {variant}")
    kw = {"rows": dict(tiles=(24, 2, 2, 0), lds=True), "segments": dict(tiles=(8, 4, 2, 0), lds=True),
          "direct": dict(), "direct-segments": dict(tiles=(8, 4, 2, 0))}[variant]
    dom = (24, 14, 12)
    solid, frac, _ = inputs.spheres(dom, seed=5, rmin=2.0, rmax=3.5, solid_fraction=0.15, periodic=(1, 1, 1),
                                    clear_x=0)
    assert solid[:, :, 0].any() and solid[:, :, -1].any(), "spheres must cross the x face"
    rho, u = inputs.random_state(dom, seed=6, umag=0.01)
    u, F = _plane(q, u, (1e-5, 0, 2e-6))
    p = wlb.make_params(tau=0.75, magic=3 / 16, omega_bulk=1.2, omega_higher=1.0, force=F)
    gpu = gpu_run(wlb.single_block(dom), dom, (1, 0, 1), q, wlb.F64, coll, p, rho, u, solid, steps=7, **kw)
    info = gpu[4].info()
    assert info.lds_staging == (not variant.startswith("direct")), variant
    op = oracle_params(q, coll, 0.75, 3 / 16, (1, 0, 1), F, omega_bulk=1.2, omega_higher=1.0)
    orc = oracle_run(op, dom, rho, u, solid, 7)
    _compare(f"x-wrap q{q} c{coll}", wlb.F64, q, gpu, orc, solid, np.prod(dom))


@pytest.mark.parametrize("storage", [0, 1])
def test_wrapping_and_exchanging_decompositions_agree_bitwise(storage):
    """Periodic x: one block (x wraps), blocks split along y/z only (each
    wraps in x, exchanges in y/z) and blocks split along x (x exchange) give
    identical populations."""
    say(f"case wrap decomposition storage{storage}")
    dom = (32, 24, 16)
    solid, _, _ = inputs.spheres(dom, seed=8, rmin=2.0, rmax=3.0, solid_fraction=0.1, periodic=(1, 1, 1), clear_x=0)
    rho, u = inputs.random_state(dom, seed=9, umag=0.01)
    p = wlb.make_params(tau=0.7, magic=3 / 16, force=(1e-5, 1e-6, 0))
    layouts = [wlb.single_block(dom), inputs.rectilinear_blocks([32], [8, 16], [6, 10])[0],
               inputs.rectilinear_blocks([8, 24], [24], [16])[0], inputs.uniform_blocks(dom, (16, 8, 8))[0]]
    ref = {}
    # odd sweep: direct with the default (whole-row) tiles and over row
    # segments, staged in LDS likewise
    variants = [dict(), dict(tiles=(8, 4, 4, 0)), dict(lds=True), dict(lds=True, tiles=(8, 4, 4, 0)), dict(lds=2)]
    for k, bl in enumerate(layouts):
        for kw in variants:
            for steps in (8, 9):  # ends in the natural and in the swapped layout
                d, r, uu, tot, B = gpu_run(bl, dom, (1, 1, 1), 19, storage, 1, p, rho, u, solid, steps=steps, **kw)
                B.close()
                if steps not in ref:
                    ref[steps] = (d, r, uu)
                else:
                    assert np.array_equal(d, ref[steps][0]), f"layout {k} {kw} steps {steps}: populations differ"
                    assert np.array_equal(r, ref[steps][1]) and np.array_equal(uu, ref[steps][2]), f"layout {k} {kw}"


def test_tiles_grid_graph_and_split_are_bitwise_invariant():
    say("case tiles/graph/split")
    dom = (40, 24, 20)
    solid, rho, u = _porous_inputs(dom, seed=4)
    blocks = inputs.rectilinear_blocks([16, 24], [24], [12, 8])[0]
    p = wlb.make_params(tau=0.66, magic=3 / 16, force=(1e-5, 0, 0))
    runs = [dict(), dict(tiles=(16, 4, 4, 0)), dict(tiles=(64, 4, 1, 7)), dict(tiles=(8, 8, 4, 3)),
            dict(graph=False), dict(mode="split"), dict(lds=True), dict(lds=True, tiles=(16, 4, 4, 0)),
            dict(tiles=(0, 0, 0, -1)), dict(tiles=(16, 4, 4, -1), mode="split"), dict(tiles=(-1, 0, 0, 0)),
            dict(tiles=(-1, 0, 0, -1)), dict(tiles=(-1, 0, 0, 5), graph=False),
            # interior/frontier overlap on two streams
            dict(overlap=True), dict(overlap=True, graph=False), dict(overlap=True, mode="split"),
            dict(overlap=True, tiles=(16, 4, 4, -1)), dict(overlap=True, tiles=(64, 4, 1, 7)),
            dict(overlap=True, tiles=(-1, 0, 0, 0)), dict(overlap=True, tiles=(-1, 0, 0, -1), graph=False),
            dict(overlap=True, lds=True),
            # cached instead of non-temporal population accesses, and the odd
            # sweep's hint on its aligned accesses only
            dict(nt=(0, 0)), dict(nt=(1, 0), lds=True), dict(nt=(0, 1), tiles=(-1, 0, 0, 0)),
            dict(nt=(0, 0), overlap=True), dict(nt=(1, 2)), dict(nt=(0, 2), tiles=(-1, 0, 0, 0)),
            dict(nt=(1, 2), overlap=True), dict(nt=(1, 2), lds=True)]
    ref = None
    for kw in runs:
        d, r, uu, tot, B = gpu_run(blocks, dom, (1, 1, 0), 19, wlb.F32, wlb.TRT, p, rho, u, solid, steps=13, **kw)
        assert B.info().overlap == int(kw.get("overlap", False)), kw
        B.close()
        if ref is None:
            ref = d
        else:
            assert np.array_equal(d, ref), kw


def test_tile_shape_per_class_of_runs_is_bitwise_invariant():
    """x-runs of different y extents swept with different tile shapes (the
    autotuner's per-class choice) give the populations of one shape for all."""
    say("case per-class tiles")
    dom = (40, 36, 20)
    solid, rho, u = _porous_inputs(dom, seed=6)
    blocks = inputs.rectilinear_blocks([16, 24], [24, 12], [12, 8])[0]
    p = wlb.make_params(tau=0.66, magic=3 / 16, force=(1e-5, 0, 0))
    ref = None
    for shapes, kw in (({}, {}), ({24: (16, 4, 4), 12: (8, 8, 4)}, {}), ({12: (32, 8, 1)}, dict(overlap=True)),
                       ({24: (64, 4, 1)}, dict(lds=True)), ({24: (8, 8, 4), 12: (16, 4, 4)}, dict(nt=(0, 0)))):
        B = wlb.Blocks(blocks, dom, (1, 1, 0), stencil=19, storage=wlb.F32)
        try:
            B.init(wlb.TRT, p, rho, u, solid)
            B.set_lds_staging(kw.get("lds", False))
            if kw.get("overlap"):
                B.set_overlap(True)
            if "nt" in kw:
                B.set_nontemporal(*kw["nt"])
            for e, s in shapes.items():
                B.set_class_tiles(e, *s)
            assert B.info().n_class_tiles == len(shapes), shapes
            B.step(13)
            d = B.pdfs_get()
        finally:
            B.close()
        if ref is None:
            ref = d
        else:
            assert np.array_equal(d, ref), (shapes, kw)


@pytest.mark.parametrize("storage", [0, 1, 2])
@pytest.mark.parametrize("nt", [(1, 0), (0, 0), (1, 1), (1, 2)])
def test_solid_cells_keep_their_populations(storage, nt):
    """The even sweep stores each solid cell's values back into their own
    slots (in the same instructions as the fluid cells): over many steps the
    solid cells' populations stay bitwise those of the initial state, in
    every storage and with either cache hint, while the fluid cells match a
    run with list tiles, which never touches solid cells."""
    say(f"case solid cells unchanged storage{storage} nt{nt}")
    dom = (40, 24, 20)
    solid, rho, u = _porous_inputs(dom, seed=5)
    blocks = inputs.rectilinear_blocks([16, 24], [24], [12, 8])[0]
    p = wlb.make_params(tau=0.7, magic=3 / 16, omega_bulk=1.1, omega_higher=1.0, pressure_axis=0, rho_in=1.001,
                        rho_out=0.999)
    s = solid.reshape(-1).astype(bool)
    B = wlb.Blocks(blocks, dom, (0, 1, 1), stencil=19, storage=storage)
    try:
        B.init(wlb.TRT, p, rho, u, solid)
        d0 = B.pdfs_get()
        B.set_nontemporal(*nt)
        B.step(14)
        d1 = B.pdfs_get()
    finally:
        B.close()
    assert np.array_equal(d1[:, s], d0[:, s])
    d, r, uu, tot, Bl = gpu_run(blocks, dom, (0, 1, 1), 19, storage, wlb.TRT, p, rho, u, solid, steps=14,
                                tiles=(-1, 0, 0, 0))
    Bl.close()
    assert np.array_equal(d[:, ~s], d1[:, ~s])


def test_slot_stride_is_bitwise_invariant():
    """256^3 FP32 channel (64.5 MiB slots, so the rounding applies): the
    three slot strides give bitwise the same moments, with and without the
    autotuner choosing one."""
    import hashlib
    say("case slot strides")
    n = 256
    dom = (n, n, n)
    rho, u = inputs.uniform_state(dom)
    digests = {}
    for kib, auto in ((16384, 0), (2048, 0), (0, 0), (None, 1)):
        p = wlb.make_params(tau=0.8, magic=3 / 16, force=(1e-6, 0, 0), autotune=auto)
        B = wlb.Blocks(wlb.single_block(dom), dom, (1, 0, 1), stencil=19, storage=wlb.F32)
        try:
            if kib is not None:
                B.set_slot_round(kib)
            B.init(wlb.TRT, p, rho, u)
            if kib is not None:
                assert B.info().slot_round_kib == kib
            B.step(5)
            r, uu, tot = B.moments()
            digests[(kib, auto)] = hashlib.sha1(r.tobytes() + uu.tobytes()).hexdigest()
            del r, uu
        finally:
            B.close()
    assert len(set(digests.values())) == 1, digests


def test_fluid_list_tiles_need_solid_cells():
    say("case list tiles without solids")
    dom = (16, 12, 10)
    rho, u = inputs.random_state(dom, seed=1, umag=0.01)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=19, storage=wlb.F32)
    try:
        B.init(wlb.SRT, wlb.make_params(tau=0.8), rho, u)
        with pytest.raises(wlb.WlbError) as e:
            B.set_tiles(-1, 0, 0, 0)
        assert e.value.code == wlb.WLB_ERR_STATE
    finally:
        B.close()


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2)])
def test_fluid_list_tiles_fp64_vs_oracle(q, coll):
    """Sweeps over lists of fluid cells on uneven blocks with spheres and
    density faces, against the oracle."""
    say(f"case list tiles q{q} coll{coll}")
    blocks, dom = inputs.rectilinear_blocks([8, 12, 6], [10, 6], [7, 9])
    solid, frac, _ = inputs.spheres(dom, seed=3, rmin=2.0, rmax=4.0, solid_fraction=0.2, clear_x=2)
    rho, u = inputs.random_state(dom, seed=13, umag=0.01)
    p = wlb.make_params(tau=0.8, magic=3 / 16, omega_bulk=1.2, omega_higher=1.0, pressure_axis=0, rho_in=1.002,
                        rho_out=0.998)
    gpu = gpu_run(blocks, dom, (0, 1, 1), q, wlb.F64, coll, p, rho, u, solid, steps=9, tiles=(-1, 0, 0, -1))
    assert gpu[4].info().tile[0] == -1
    op = oracle_params(q, coll, 0.8, 3 / 16, (0, 1, 1), pressure_axis=0, rho_in=1.002, rho_out=0.998,
                       omega_bulk=1.2, omega_higher=1.0)
    orc = oracle_run(op, dom, rho, u, solid, 9)
    _compare(f"list tiles q{q} c{coll}", wlb.F64, q, gpu, orc, solid, np.prod(dom))


@pytest.mark.parametrize("storage", [0, 2])
def test_checkpoint_resume_is_bitwise(storage):
    say(f"case resume storage{storage}")
    dom = (20, 16, 12)
    solid, rho, u = _porous_inputs(dom, seed=5)
    p = wlb.make_params(tau=0.7, magic=3 / 16, pressure_axis=0, rho_in=1.001, rho_out=0.999)
    blocks = inputs.rectilinear_blocks([12, 8], [16], [6, 6])[0]
    d_full, *_, B = gpu_run(blocks, dom, (0, 1, 1), 19, storage, wlb.TRT, p, rho, u, solid, steps=15)
    B.close()
    d_mid, *_, B = gpu_run(blocks, dom, (0, 1, 1), 19, storage, wlb.TRT, p, rho, u, solid, steps=7)
    B.close()
    B2 = wlb.Blocks(blocks, dom, (0, 1, 1), stencil=19, storage=storage)
    B2.init(wlb.TRT, p, rho, u, solid)
    B2.pdfs_set(d_mid)
    B2.step(8)
    d_res = B2.pdfs_get()
    B2.close()
    assert np.array_equal(d_res, d_full)


def test_health_check_reports_divergence():
    say("case health")
    dom = (16, 16, 8)
    rho, u = inputs.random_state(dom, seed=6)
    p = wlb.make_params(tau=0.8, health_every=2)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=19, storage=wlb.F32)
    B.init(wlb.SRT, p, rho, u)
    B.step(4)  # healthy
    d = B.pdfs_get()
    d[3, 100] = np.nan
    B.pdfs_set(d)
    with pytest.raises(wlb.WlbError) as e:
        B.step(4)
    assert e.value.code == wlb.WLB_ERR_DIVERGED
    B.close()


def test_totals_match_fsum_of_fields():
    say("case totals")
    dom = (30, 20, 10)
    solid, rho, u = _porous_inputs(dom, seed=9)
    p = wlb.make_params(tau=0.8, force=(1e-5, 0, 0))
    d, r, uu, tot, B = gpu_run(wlb.single_block(dom), dom, (1, 1, 1), 19, wlb.F64, wlb.SRT, p, rho, u, solid,
                               steps=5)
    B.close()
    fl = solid.reshape(-1) == 0
    rr = r.reshape(-1)[fl]
    assert tot[6] == fl.sum()
    assert abs(tot[0] - math.fsum(rr)) <= 4 * np.spacing(tot[0])
    px = math.fsum(rr * uu[0].reshape(-1)[fl])
    assert abs(tot[1] - px) <= 1e-15 * max(1.0, abs(px)) + 1e-18
    assert tot[7] == 5


@pytest.mark.parametrize("nx", [64, 96, 256, 384, 512])
@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (27, 4), (15, 0), (9, 1)])
def test_row_vector_odd_sweep_fp64_vs_oracle_and_direct(nx, q, coll):
    """The row-vector odd sweep (two FP64 cells per lane, x shift by lane
    moves): rows inside one wavefront (64 and 96 cells), rows of two and
    three wavefronts (256, 384) and of a whole workgroup (512), walls in y
    with a body force, then density faces in y; against the oracle and
    bitwise against the direct odd sweep.  Blocks split along y and z
    exchange with each other."""
    say(f"case rows nx{nx} q{q} coll{coll}")
    dom = (nx, 12, 6)
    rho, u = inputs.random_state(dom, seed=nx + q, umag=0.02)
    u, F = _plane(q, u, (1e-5, 0, -2e-6))
    cases = [("walls", wlb.single_block(dom), (1, 0, 1), dict(force=F)),
             ("density", wlb.single_block(dom), (1, 0, 1), dict(pressure_axis=1, rho_in=1.003, rho_out=0.998)),
             ("blocks", inputs.rectilinear_blocks([nx], [5, 7], [2, 4])[0], (1, 1, 1), dict(force=F))]
    for name, blocks, periodic, extra in cases:
        kw = dict(tau=0.7, magic=3 / 16, omega_bulk=1.2, omega_higher=1.1, **extra)
        p = wlb.make_params(**kw)
        runs = []
        for lds in (2, 0):
            d, r, uu, tot, B = gpu_run(blocks, dom, periodic, q, wlb.F64, coll, p, rho, u, steps=7, lds=lds)
            assert B.info().lds_staging == lds, (name, lds)
            B.close()
            runs.append((d, r, uu))
        assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][2], runs[1][2]), name
        op = oracle_params(q, coll, 0.7, 3 / 16, periodic, extra.get("force", (0, 0, 0)),
                           pressure_axis=extra.get("pressure_axis", -1), rho_in=extra.get("rho_in", 1.0),
                           rho_out=extra.get("rho_out", 1.0), omega_bulk=1.2, omega_higher=1.1)
        do, ro, uo, to = oracle_run(op, dom, rho, u, None, 7)
        eu = rel_l2(runs[0][2].reshape(3, -1), uo)
        ep = pop_err(runs[0][0], do, q)
        say(f"rows nx{nx} q{q} c{coll} {name}: u rel L2 {eu:.3e}, pops {ep:.3e}")
        assert eu <= 1e-12 and ep <= 1e-12, (name, eu, ep)
