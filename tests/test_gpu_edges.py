"""Edge cases of the GPU path against the FP64 oracle: degenerate and thin
blocks, a one-cell domain, zero steps, a nearly solid domain, ragged rows
and a closed box."""
import numpy as np
import pytest

import oracle as O
from gpu_util import gpu_run, inputs, oracle_params, oracle_run, pop_err, rel_l2, say

pytestmark = pytest.mark.gpu

wlb = pytest.importorskip("paper_1909_13772_amd.wlb", reason="libwlb.so not built")

TOL = 1e-12


def _check(case, q, gpu, orc, solid, n):
    d, r, u, tot, B = gpu
    do, ro, uo, to = orc
    B.close()
    m = np.ones(n, bool) if solid is None else np.asarray(solid).reshape(-1) == 0
    eu = rel_l2(u.reshape(3, -1), uo, m) if np.linalg.norm(uo[:, m]) > 0 else np.abs(u.reshape(3, -1)[:, m]).max()
    ep = pop_err(d[:, m], do[:, m], q)
    er = np.abs(r.reshape(-1)[m] - ro[m]).max()
    say(f"{case}: u {eu:.3e}, pops {ep:.3e}, rho {er:.3e}")
    assert eu <= TOL and ep <= TOL and er <= 1e-12, case
    assert abs(tot[0] - to[0]) <= 1e-9 * max(1.0, abs(to[0])), (case, tot[0], to[0])


@pytest.mark.parametrize("q,coll", [(19, 1), (27, 2), (15, 1), (9, 0)])
@pytest.mark.parametrize("overlap", [False, True])
def test_one_cell_thick_blocks(q, coll, overlap):
    """Blocks one cell thick along every axis: ghost regions are whole blocks
    and every exchange item touches a block's full extent (with the overlap,
    no block has an interior)."""
    say(f"case thin blocks q{q} c{coll} overlap {overlap}")
    blocks, dom = inputs.rectilinear_blocks([1, 6, 1], [1, 4], [2, 1, 3])
    rho, u = inputs.random_state(dom, seed=31, umag=0.02)
    F = (1e-5, -1e-5, 2e-6)
    if q == 9:  # no z velocities in D2Q9
        u[2] = 0.0
        F = (1e-5, -1e-5, 0.0)
    p = wlb.make_params(tau=0.7, magic=3 / 16, omega_bulk=1.1, omega_higher=1.0, force=F)
    for periodic in ((1, 1, 1), (1, 0, 1)):
        gpu = gpu_run(blocks, dom, periodic, q, wlb.F64, coll, p, rho, u, steps=7, overlap=overlap)
        op = oracle_params(q, coll, 0.7, 3 / 16, periodic, F, omega_bulk=1.1, omega_higher=1.0)
        orc = oracle_run(op, dom, rho, u, None, 7)
        _check(f"thin {periodic}", q, gpu, orc, None, np.prod(dom))


@pytest.mark.parametrize("q", [19, 15, 9])
@pytest.mark.parametrize("dom", [(1, 1, 1), (2, 1, 3), (1, 5, 1)])
def test_degenerate_periodic_domains(dom, q):
    """Domains with extent 1 or 2: the block is its own neighbour on every
    periodic face (x wraps onto the same cell)."""
    say(f"case degenerate {dom} q{q}")
    rho, u = inputs.random_state(dom, seed=32, umag=0.02)
    if q == 9:
        u[2] = 0.0
    p = wlb.make_params(tau=0.9, magic=0.2)
    gpu = gpu_run(wlb.single_block(dom), dom, (1, 1, 1), q, wlb.F64, wlb.TRT, p, rho, u, steps=5)
    op = oracle_params(q, wlb.TRT, 0.9, 0.2, (1, 1, 1))
    orc = oracle_run(op, dom, rho, u, None, 5)
    _check(f"degenerate {dom} q{q}", q, gpu, orc, None, np.prod(dom))


def test_zero_steps_reproduce_the_initial_state():
    say("case zero steps")
    dom = (12, 9, 7)
    rho, u = inputs.random_state(dom, seed=33, umag=0.03)
    p = wlb.make_params(tau=0.8)
    d, r, uu, tot, B = gpu_run(wlb.single_block(dom), dom, (1, 1, 1), 27, wlb.F64, wlb.SRT, p, rho, u, steps=0)
    B.close()
    d0 = O.init(27, dom, rho, u, None)
    assert np.abs(d - d0).max() <= 1e-15
    assert np.abs(r - rho).max() <= 1e-14
    assert np.abs(uu - u).max() <= 1e-14


def test_nearly_solid_domain_keeps_mass():
    """Everything solid except a small pocket and a one-cell channel through
    the periodic x face."""
    say("case nearly solid")
    dom = (10, 8, 6)
    solid = np.ones((dom[2], dom[1], dom[0]), np.uint8)
    solid[2:4, 3:5, 3:6] = 0
    solid[3, 4, :] = 0
    rho, u = inputs.random_state(dom, seed=34, umag=0.02)
    p = wlb.make_params(tau=0.75, magic=3 / 16, omega_bulk=1.0, omega_higher=1.0)
    for q, coll in ((19, 1), (27, 2)):
        gpu = gpu_run(inputs.rectilinear_blocks([4, 6], [8], [3, 3])[0], dom, (1, 1, 1), q, wlb.F64, coll, p, rho,
                      u, solid, steps=8)
        op = oracle_params(q, coll, 0.75, 3 / 16, (1, 1, 1), omega_bulk=1.0, omega_higher=1.0)
        orc = oracle_run(op, dom, rho, u, solid, 8)
        _check(f"nearly solid q{q}", q, gpu, orc, solid, np.prod(dom))


def test_ragged_rows_and_closed_box():
    """Rows longer than one tile with a ragged tail (300 cells), and a box
    closed by walls on all six faces split into uneven blocks."""
    say("case ragged rows / closed box")
    dom = (300, 3, 4)
    rho, u = inputs.random_state(dom, seed=35, umag=0.02)
    p = wlb.make_params(tau=0.8, magic=3 / 16, force=(1e-5, 0, 0))
    gpu = gpu_run(wlb.single_block(dom), dom, (1, 0, 1), 19, wlb.F64, wlb.TRT, p, rho, u, steps=6)
    orc = oracle_run(oracle_params(19, wlb.TRT, 0.8, 3 / 16, (1, 0, 1), (1e-5, 0, 0)), dom, rho, u, None, 6)
    _check("ragged 300", 19, gpu, orc, None, np.prod(dom))
    blocks, dom = inputs.rectilinear_blocks([5, 8], [3, 4], [5])
    rho, u = inputs.random_state(dom, seed=36, umag=0.02)
    p = wlb.make_params(tau=0.7, omega_bulk=1.2, omega_higher=1.1)
    gpu = gpu_run(blocks, dom, (0, 0, 0), 27, wlb.F64, wlb.MRT, p, rho, u, steps=9)
    orc = oracle_run(oracle_params(27, wlb.MRT, 0.7, 0, (0, 0, 0), omega_bulk=1.2, omega_higher=1.1), dom, rho, u,
                     None, 9)
    _check("closed box", 27, gpu, orc, None, np.prod(dom))
