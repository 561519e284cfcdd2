"""Race freedom of the AA sweeps, checked on the GPU: in one sweep of either
parity, with the exchange after it, every population slot of every fluid
cell is written exactly once and no solid cell is written.  The check runs
the sweep and exchange kernels themselves with stores that count
(wlb_debug_write_coverage), over uneven blocks with spheres and density
faces, a block that wraps onto itself in x, every tile mode (also per class
of x-runs), the LDS-staged odd sweep, the interior/frontier overlap and all
four velocity sets."""
import numpy as np
import pytest

from gpu_util import inputs, say

pytestmark = pytest.mark.gpu

wlb = pytest.importorskip("paper_1909_13772_amd.wlb", reason="libwlb.so not built")

MODES = [dict(), dict(tiles=(16, 4, 4, 0)), dict(tiles=(64, 4, 1, 7)), dict(tiles=(8, 8, 4, 3)),
         dict(lds=True), dict(lds=True, tiles=(16, 4, 4, 0)), dict(tiles=(-1, 0, 0, 0)),
         dict(tiles=(-1, 0, 0, -1)), dict(overlap=True), dict(overlap=True, tiles=(-1, 0, 0, 0)),
         dict(overlap=True, lds=True),
         # per-class tile shapes: x-runs of y extent 10 and 6 (the porous case) tiled differently
         dict(classes={10: (16, 4, 4), 6: (8, 8, 4)}), dict(classes={6: (64, 4, 1)}, overlap=True)]


def _case(name):
    if name == "porous":  # 3 x 2 x 2 uneven blocks, density faces on x
        blocks, dom = inputs.rectilinear_blocks([8, 12, 6], [10, 6], [7, 9])
        solid, _, _ = inputs.spheres(dom, seed=2, rmin=2.0, rmax=4.0, solid_fraction=0.2, clear_x=2)
        return blocks, dom, (0, 1, 1), solid, dict(pressure_axis=0, rho_in=1.002, rho_out=0.998)
    dom = (24, 14, 12)  # one block periodic in x, spheres across the x face, walls in y
    solid, _, _ = inputs.spheres(dom, seed=5, rmin=2.0, rmax=3.5, solid_fraction=0.15, periodic=(1, 1, 1),
                                 clear_x=0)
    return wlb.single_block(dom), dom, (1, 0, 1), solid, dict(force=(1e-5, 0, 0))


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (15, 1), (9, 0)])
@pytest.mark.parametrize("odd", [0, 1])
@pytest.mark.parametrize("case", ["porous", "xwrap"])
def test_every_fluid_slot_is_written_exactly_once(q, coll, odd, case):
    blocks, dom, periodic, solid, extra = _case(case)
    fluid = solid.reshape(-1) == 0
    rho, u = inputs.uniform_state(dom)
    p = wlb.make_params(tau=0.8, magic=3 / 16, omega_bulk=1.2, omega_higher=1.0, **extra)
    for kw in MODES:
        say(f"case coverage {case} q{q} coll{coll} odd{odd} {kw}")
        B = wlb.Blocks(blocks, dom, periodic, stencil=q, storage=wlb.F32)
        try:
            B.init(coll, p, rho, u, solid)
            if "tiles" in kw:
                B.set_tiles(*kw["tiles"])
            B.set_lds_staging(kw.get("lds", False))
            if kw.get("overlap"):
                B.set_overlap(True)
            for e, shape in kw.get("classes", {}).items():
                if case == "porous":
                    B.set_class_tiles(e, *shape)
            c = B.write_coverage(odd)
            info = B.info()
        finally:
            B.close()
        assert info.overlap == int(kw.get("overlap", False)), kw
        fc = c[:, fluid]
        assert fc.min() == 1 and fc.max() == 1, (kw, int(fc.min()), int(fc.max()), int((fc != 1).sum()))
        assert not c[:, ~fluid].any(), kw


def test_coverage_check_needs_fp32_storage_and_a_fresh_init():
    dom = (8, 6, 4)
    rho, u = inputs.uniform_state(dom)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=19, storage=wlb.F64)
    try:
        B.init(wlb.TRT, wlb.make_params(tau=0.8), rho, u)
        with pytest.raises(wlb.WlbError) as e:
            B.write_coverage(0)
        assert e.value.code == wlb.WLB_ERR_UNSUPPORTED
    finally:
        B.close()
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=19, storage=wlb.F32)
    try:
        B.init(wlb.TRT, wlb.make_params(tau=0.8), rho, u)
        c = B.write_coverage(1)
        assert c.min() == 1 and c.max() == 1
        with pytest.raises(wlb.WlbError) as e:  # the state now holds counters
            B.step(1)
        assert e.value.code == wlb.WLB_ERR_STATE
        B.init(wlb.TRT, wlb.make_params(tau=0.8), rho, u)
        B.step(2)
    finally:
        B.close()


# Row-vector odd sweep (wlb_set_lds_staging(2)): blocks that wrap onto
# themselves along x and hold no solid cells.  The counting storage runs it
# with 4 cells per lane, so these rows cover a row held inside one wavefront
# (64 cells: 16 lanes, four rows per wavefront), rows straddling wavefront
# boundaries at odd places (96 cells: 24 lanes), a row of exactly one
# wavefront (256 cells) and rows spanning two and three wavefronts (512 and
# 384 cells: the edge lanes read and write the crossing elements).
@pytest.mark.parametrize("nx", [64, 96, 256, 384, 512])
@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (15, 0), (9, 1)])
@pytest.mark.parametrize("odd", [0, 1])
def test_row_vector_odd_sweep_writes_every_slot_once(nx, q, coll, odd):
    say(f"case coverage rows nx{nx} q{q} coll{coll} odd{odd}")
    dom = (nx, 10, 6)
    rho, u = inputs.uniform_state(dom)
    # walls in y (no ghost rows), periodic z (ghost planes and exchange),
    # then blocks split along z that exchange with each other
    for blocks, periodic in ((wlb.single_block(dom), (1, 0, 1)),
                             (inputs.rectilinear_blocks([nx], [10], [2, 4])[0], (1, 1, 1))):
        B = wlb.Blocks(blocks, dom, periodic, stencil=q, storage=wlb.F32)
        try:
            B.init(coll, wlb.make_params(tau=0.8, magic=3 / 16, omega_bulk=1.2, force=(1e-5, 0, 0)), rho, u)
            B.set_lds_staging(2)
            c = B.write_coverage(odd)
        finally:
            B.close()
        assert c.min() == 1 and c.max() == 1, (periodic, int(c.min()), int(c.max()), int((c != 1).sum()))
