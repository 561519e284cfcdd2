"""Plain numpy FP64 reference of the LES training-data step -- TEST
INFRASTRUCTURE (tests and the CPU baseline only; shares nothing with the
GPU library).

box_filter: averages over factor^3 fine cells of rho, u, u_a u_b.
les_targets: from filtered fields on a periodic coarse grid with spacing 1:
  S_ab = (d_a u_b + d_b u_a) / 2 (central differences), tau_sgs = avg(uu) - u u,
  nu_t = max(0, -dev(tau_sgs) : S / (2 S:S + 1e-30)), target = 3 nu_t,
  raw features = (-(2/3) rho (tau0 + target) S_{xx,yy,zz,xy,xz,yz}, rho - 1).
The relation Pi_neq = -2 rho c_s^2 tau S (c_s^2 = 1/3) is the first-order
Chapman-Enskog stress that the closure sees in the coarse run (paper Sec.
5.1.1: a relaxation time that varies per cell with the local shear).
"""
from __future__ import annotations

import numpy as np


def box_filter(rho, u, f):
    """rho (nz, ny, nx), u (3, nz, ny, nx) -> (10, ncz, ncy, ncx)."""
    nz, ny, nx = rho.shape
    if nz % f or ny % f or nx % f:
        raise ValueError("factor must divide the grid")

    def avg(a):
        return a.reshape(nz // f, f, ny // f, f, nx // f, f).mean(axis=(1, 3, 5))

    ux, uy, uz = u
    chans = [rho, ux, uy, uz, ux * ux, uy * uy, uz * uz, ux * uy, ux * uz, uy * uz]
    return np.stack([avg(c) for c in chans])


def strain(ubar):
    """Central-difference symmetric gradient of a periodic (3, nz, ny, nx) field:
    (xx, yy, zz, xy, xz, yz)."""
    def d(a, axis):  # axis 0 = x (last array axis)
        ax = {0: 2, 1: 1, 2: 0}[axis]
        return 0.5 * (np.roll(a, -1, axis=ax) - np.roll(a, 1, axis=ax))

    g = [[d(ubar[b], a) for b in range(3)] for a in range(3)]  # g[a][b] = d_a u_b
    return np.stack([g[0][0], g[1][1], g[2][2], 0.5 * (g[0][1] + g[1][0]), 0.5 * (g[0][2] + g[2][0]),
                     0.5 * (g[1][2] + g[2][1])])


def les_targets(filt, tau0):
    """filt (10, ncz, ncy, ncx) -> raw (Nc, 7), target (Nc,)."""
    rho = filt[0]
    ub = filt[1:4]
    S = strain(ub)
    t = np.stack([filt[4] - ub[0] ** 2, filt[5] - ub[1] ** 2, filt[6] - ub[2] ** 2, filt[7] - ub[0] * ub[1],
                  filt[8] - ub[0] * ub[2], filt[9] - ub[1] * ub[2]])
    tr = (t[0] + t[1] + t[2]) / 3.0
    t[0] -= tr
    t[1] -= tr
    t[2] -= tr
    w = np.array([1, 1, 1, 2, 2, 2], np.float64)[:, None, None, None]
    tS = (w * t * S).sum(0)
    SS = (w * S * S).sum(0)
    nu = -tS / (2.0 * SS + 1e-30)
    nu = np.where(nu > 0, nu, 0.0)
    target = 3.0 * nu
    raw = np.empty((7,) + rho.shape)
    raw[:6] = -(2.0 / 3.0) * rho[None] * (tau0 + target)[None] * S
    raw[6] = rho - 1.0
    return raw.reshape(7, -1).T.copy(), target.reshape(-1)
