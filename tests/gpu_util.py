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
            graph=True, mode="step", lds=False, overlap=False, nt=None):
    """Returns (d[q][N] natural-layout deviations, rho, u, totals, Blocks)."""
    from paper_1909_13772_amd import wlb
    B = wlb.Blocks(blocks, domain, periodic, stencil=q, storage=storage)
    B.init(coll, params, rho, u, solid)
    if tiles is not None:
        B.set_tiles(*tiles)
    B.set_graph(graph)
    B.set_lds_staging(lds)
    if overlap:
        B.set_overlap(True)
    if nt is not None:
        B.set_nontemporal(*nt)
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


def crop_compare(p, dom, periodic, rho, u, solid, r_gpu, u_gpu, regions, m, s):
    """Light-cone check: recompute each m^3 region after s steps from a crop of
    the initial data extended by s cells (wrapped on periodic axes, clipped at
    real boundaries) with the oracle, compare with the full-domain fields.
    Returns (max |u diff| / max |u|, max |rho diff|)."""
    worst_u, worst_r, scale = 0.0, 0.0, 0.0
    for lo in regions:
        idx, inner, crop_shape, cper = [], [], [], []
        for a in range(3):
            N = dom[a]
            a0, a1 = lo[a] - s, lo[a] + m + s
            if periodic[a]:
                ix = np.arange(a0, a1) % N
                off = s
            else:
                assert 0 <= lo[a] and lo[a] + m <= N, "sampled region must lie inside on non-periodic axes"
                c0, c1 = max(0, a0), min(N, a1)
                ix = np.arange(c0, c1)
                off = lo[a] - c0
            idx.append(ix)
            inner.append(slice(off, off + m))
            crop_shape.append(len(ix))
            cper.append(periodic[a])
        ixg = np.ix_(idx[2], idx[1], idx[0])
        rc = rho[ixg]
        uc = np.stack([u[k][ixg] for k in range(3)])
        sc = None if solid is None else solid[ixg]
        q = dict(p.__dict__)
        q.pop("_keep", None)
        pc = O.Params(**{**q, "periodic": tuple(int(v) for v in cper)})
        shape = tuple(crop_shape)
        d = O.init(pc.q, shape, np.ascontiguousarray(rc), np.ascontiguousarray(uc), sc)
        d = O.run(pc, shape, d, s, sc)
        ro, uo, _ = O.moments(pc.q, pc.force, shape, d, sc)
        ro = ro.reshape(shape[2], shape[1], shape[0])
        uo = uo.reshape(3, shape[2], shape[1], shape[0])
        sl = (inner[2], inner[1], inner[0])
        gz, gy, gx = (np.arange(lo[2], lo[2] + m) % dom[2], np.arange(lo[1], lo[1] + m) % dom[1],
                      np.arange(lo[0], lo[0] + m) % dom[0])
        gsl = np.ix_(gz, gy, gx)
        worst_r = max(worst_r, float(np.abs(r_gpu[gsl] - ro[sl]).max()))
        du = np.abs(np.stack([u_gpu[k][gsl] for k in range(3)]) - uo[(slice(None),) + sl]).max()
        worst_u = max(worst_u, float(du))
        scale = max(scale, float(np.abs(uo[(slice(None),) + sl]).max()))
    return worst_u / max(scale, 1e-300), worst_r



__all__ = ["say", "gpu_run", "oracle_params", "oracle_run", "rel_l2", "pop_err", "fluid_mask", "inputs", "crop_compare"]
