"""Helpers for the GPU parity tests: run one configuration through the C ABI
and the same configuration through the CPU oracle."""
import sys

import numpy as np

import oracle as O
from paper_1909_13772_amd import inputs


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(blocks, domain, periodic, q, storage, coll, params, rho, u, solid=None, steps=0, tiles=None,
            graph=True, mode="step"):
    """Returns (d[q][N] natural-layout deviations, rho, u, totals, Blocks)."""
    from paper_1909_13772_amd import wlb
    B = wlb.Blocks(blocks, domain, periodic, stencil=q, storage=storage)
    B.init(coll, params, rho, u, solid)
    if tiles is not None:
        B.set_tiles(*tiles)
    B.set_graph(graph)
    if mode == "step":
        B.step(steps)
    else:
        for _ in range(steps):
            B.sweep()
            B.exchange()
    d = B.pdfs_get()
    r, uu, tot = B.moments()
    return d, r, uu, tot, B


def oracle_params(q, coll, tau, magic, periodic, force=(0, 0, 0), pressure_axis=-1, rho_in=1.0, rho_out=1.0,
                  omega_bulk=1.0, omega_higher=1.0, closure=0, cs_smag=0.0):
    return O.Params(q=q, collision=coll, tau=tau, magic=magic, omega_bulk=omega_bulk, omega_higher=omega_higher,
                    force=tuple(force), closure=closure, cs_smag=cs_smag, periodic=tuple(periodic),
                    pressure_axis=pressure_axis, rho_in=rho_in, rho_out=rho_out)


def oracle_run(p, shape, rho, u, solid, steps):
    d = O.init(p.q, shape, rho, u, solid)
    d = O.run(p, shape, d, steps, solid)
    r, uu, tot = O.moments(p.q, p.force, shape, d, solid)
    return d, r, uu, tot


def rel_l2(a, b, mask=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if mask is not None:
        a = a[..., mask]
        b = b[..., mask]
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def pop_err(d, dref, q):
    """max |f - f_ref| / max |f_ref| with f = w + d."""
    _, w, _ = O.stencil(q)
    fref = dref + w[:, None]
    return np.abs(d - dref).max() / np.abs(fref).max()


def fluid_mask(solid, n):
    if solid is None:
        return np.ones(n, bool)
    return np.asarray(solid).reshape(-1) == 0


__all__ = ["say", "gpu_run", "oracle_params", "oracle_run", "rel_l2", "pop_err", "fluid_mask", "inputs"]
