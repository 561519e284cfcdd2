"""Parity at the benchmark's full sizes, in the benchmark's launch
configuration (autotuned tiles, graph replay), on sampled regions.

After s steps a cell's state depends only on cells within Chebyshev distance
s (one lattice link per step).  The GPU advances the whole domain; the oracle
recomputes each sampled m^3 region from a crop of the initial data extended
by s cells on every side (wrapped on periodic axes, clipped at real
boundaries, whose boundary conditions the crop then reproduces).  Whatever
the crop does at its artificial faces cannot reach the sampled region.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import crop_compare, inputs, say

pytestmark = pytest.mark.gpu

wlb = pytest.importorskip("paper_1909_13772_amd.wlb", reason="libwlb.so not built")


def test_channel_256_fp64_sampled():
    """The headline configuration (D3Q19 TRT channel 256^3, FP64), random start."""
    say("case full-size channel 256 fp64")
    n, s, m = 256, 4, 8
    dom = (n, n, n)
    rho, u = inputs.random_state(dom, seed=21, umag=0.02)
    p = wlb.make_params(tau=0.8, magic=3 / 16, force=(1e-6, 0, 0), autotune=1)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 0, 1), stencil=19, storage=wlb.F64)
    B.init(wlb.TRT, p, rho, u)
    B.step(s)
    r, uu, tot = B.moments()
    B.close()
    op = O.Params(q=19, collision=O.TRT, tau=0.8, magic=3 / 16, force=(1e-6, 0, 0), periodic=(1, 0, 1))
    regions = [(0, 0, 0), (100, 124, 77), (250, 248, 5), (17, 255 - 7, 200)]
    eu, er = crop_compare(op, dom, (1, 0, 1), rho, u, None, r, uu, regions, m, s)
    say(f"channel 256 sampled: u rel {eu:.3e}, rho abs {er:.3e}")
    assert eu <= 1e-12 and er <= 1e-13


def test_porous_uneven_blocks_fp32_sampled():
    """512 uneven blocks, spheres, D3Q27 MRT, FP32, density faces on x."""
    say("case full-size porous fp32")
    s, m = 4, 8
    blocks, dom = inputs.uneven_blocks(0)
    solid, frac, _ = inputs.spheres(dom, seed=1, rmin=3.0, rmax=8.0, solid_fraction=0.3, clear_x=4)
    rho, u = inputs.random_state(dom, seed=22, umag=0.01)
    p = wlb.make_params(tau=0.8, pressure_axis=0, rho_in=1.0005, rho_out=0.9995, autotune=1)
    B = wlb.Blocks(blocks, dom, (0, 1, 1), stencil=27, storage=wlb.F32)
    B.init(wlb.MRT, p, rho, u, solid)
    B.step(s)
    r, uu, tot = B.moments()
    B.close()
    op = O.Params(q=27, collision=O.MRT, tau=0.8, omega_bulk=1.0, omega_higher=1.0, periodic=(0, 1, 1),
                  pressure_axis=0, rho_in=1.0005, rho_out=0.9995)
    # regions at both density faces, across block boundaries and in the bulk
    regions = [(0, 10, 20), (dom[0] - m, 100, 300), (60, 190, 160), (120, 0, dom[2] - 4)]
    eu, er = crop_compare(op, dom, (0, 1, 1), rho, u, solid, r, uu, regions, m, s)
    say(f"porous sampled: u rel {eu:.3e}, rho abs {er:.3e} (solid fraction {frac:.3f})")
    assert eu <= 1e-5 and er <= 1e-6


def test_turbulence_384_fp64_sampled():
    """The precision study's FP64 reference (D3Q19 TRT, tau 0.5005, 384^3)."""
    say("case full-size turbulence 384 fp64")
    n, s, m = 384, 4, 8
    dom = (n, n, n)
    rho, u = inputs.turbulence_bandlimited(n, 0)
    p = wlb.make_params(tau=0.5005, magic=3 / 16, autotune=1)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=19, storage=wlb.F64)
    B.init(wlb.TRT, p, rho, u)
    B.step(s)
    r, uu, tot = B.moments()
    B.close()
    op = O.Params(q=19, collision=O.TRT, tau=0.5005, magic=3 / 16, periodic=(1, 1, 1))
    regions = [(0, 0, 0), (200, 300, 31), (380, 5, 190)]
    eu, er = crop_compare(op, dom, (1, 1, 1), rho, u, None, r, uu, regions, m, s)
    say(f"turbulence 384 sampled: u rel {eu:.3e}, rho abs {er:.3e}")
    assert eu <= 1e-12 and er <= 1e-13


def test_entropic_kbc_384_fp32_sampled():
    """The entropic-stability configuration (D3Q27 KBC, FP32, tau 0.5005,
    384^3 decaying turbulence), autotuned as the workload runs it."""
    say("case full-size kbc 384 fp32")
    n, s, m = 384, 4, 8
    dom = (n, n, n)
    rho, u = inputs.turbulence_bandlimited(n, 0)
    p = wlb.make_params(tau=0.5005, autotune=1)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=27, storage=wlb.F32)
    B.init(wlb.KBC, p, rho, u)
    B.step(s)
    r, uu, tot = B.moments()
    B.close()
    op = O.Params(q=27, collision=O.KBC, tau=0.5005, periodic=(1, 1, 1))
    regions = [(0, 0, 0), (200, 300, 31), (380, 5, 190)]
    eu, er = crop_compare(op, dom, (1, 1, 1), rho, u, None, r, uu, regions, m, s)
    say(f"kbc 384 sampled: u rel {eu:.3e}, rho abs {er:.3e}")
    assert eu <= 1e-5 and er <= 1e-6


def test_cumulant_384_fp32_sampled():
    """The cumulant collision in the entropic-stability configuration (D3Q27,
    FP32, tau 0.5005, 384^3 decaying turbulence, bulk rate 1), autotuned."""
    say("case full-size cumulant 384 fp32")
    n, s, m = 384, 4, 8
    dom = (n, n, n)
    rho, u = inputs.turbulence_bandlimited(n, 0)
    p = wlb.make_params(tau=0.5005, omega_bulk=1.0, autotune=1)
    B = wlb.Blocks(wlb.single_block(dom), dom, (1, 1, 1), stencil=27, storage=wlb.F32)
    B.init(wlb.CUMULANT, p, rho, u)
    B.step(s)
    r, uu, tot = B.moments()
    B.close()
    op = O.Params(q=27, collision=O.CUMULANT, tau=0.5005, omega_bulk=1.0, periodic=(1, 1, 1))
    regions = [(0, 0, 0), (200, 300, 31), (380, 5, 190)]
    eu, er = crop_compare(op, dom, (1, 1, 1), rho, u, None, r, uu, regions, m, s)
    say(f"cumulant 384 sampled: u rel {eu:.3e}, rho abs {er:.3e}")
    assert eu <= 1e-5 and er <= 1e-6
