"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module generates initial conditions, geometries and block layouts only.
It holds none of the lattice Boltzmann arithmetic (no equilibria, no
collision, no streaming): the same arrays are handed both to the GPU library
and to the CPU oracle, which each compute the method on their own.

All arrays are in global lattice order with x fastest: scalar fields have
shape (nz, ny, nx); vector fields (3, nz, ny, nx) with components x, y, z.
"""
from __future__ import annotations

import numpy as np

EDGE_CHOICES = (16, 24, 32, 48, 64)


def uniform_state(shape, rho=1.0, u=(0.0, 0.0, 0.0)):
    """Uniform density and velocity on a (nx, ny, nz) lattice."""
    nx, ny, nz = shape
    r = np.full((nz, ny, nx), float(rho))
    v = np.empty((3, nz, ny, nx))
    for a in range(3):
        v[a] = u[a]
    return r, v


def taylor_green(n=32, u0=0.01, nz=None):
    """z-invariant Taylor-Green vortex on an n x n x nz periodic box:
    u = u0 sin(kx) cos(ky), v = -u0 cos(kx) sin(ky), w = 0, k = 2 pi / n,
    x, y = integer cell indices, rho = 1."""
    nz = n if nz is None else nz
    k = 2.0 * np.pi / n
    x = np.arange(n)
    X, Y = np.meshgrid(x, x, indexing="xy")  # X varies along the last axis
    ux = u0 * np.sin(k * X) * np.cos(k * Y)
    uy = -u0 * np.cos(k * X) * np.sin(k * Y)
    rho = np.ones((nz, n, n))
    u = np.zeros((3, nz, n, n))
    u[0] = ux[None]
    u[1] = uy[None]
    return rho, u


def random_state(shape, seed, drho=1e-3, umag=0.02):
    """Random (smooth-free) density and velocity perturbations; used to
    exercise every population with non-trivial values."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    rho = 1.0 + drho * rng.uniform(-1.0, 1.0, (nz, ny, nx))
    u = umag * rng.uniform(-1.0, 1.0, (3, nz, ny, nx))
    return rho, u


def turbulence(n, seed, u_rms=0.05, k0=4.0, nyz=None):
    """Decaying homogeneous turbulence initial velocity on a periodic n^3 box.

    Energy spectrum E(k) proportional to k^4 exp(-2 (k/k0)^2) over integer
    wavevectors, random phases (white noise from numpy's PCG64 generator
    seeded with ``seed``), solenoidal projection, shell-wise amplitude so the
    shell energy matches E(k), Nyquist planes removed, and a global scale so
    the per-component rms velocity sqrt(<|u|^2>/3) equals ``u_rms``.
    Returns rho (ones) and u.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((3, n, n, n))
    uh = np.fft.fftn(noise, axes=(1, 2, 3))
    del noise
    f = np.fft.fftfreq(n) * n
    kz = f[:, None, None]
    ky = f[None, :, None]
    kx = f[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    kdotu = kx * uh[0] + ky * uh[1] + kz * uh[2]
    with np.errstate(invalid="ignore", divide="ignore"):
        inv = np.where(k2 > 0, 1.0 / k2, 0.0)
    uh[0] -= kx * kdotu * inv
    uh[1] -= ky * kdotu * inv
    uh[2] -= kz * kdotu * inv
    del kdotu
    nyq = (np.abs(kx) == n // 2) | (np.abs(ky) == n // 2) | (np.abs(kz) == n // 2)
    kmag = np.sqrt(k2)
    shell = np.rint(kmag).astype(np.int64)
    e_mode = 0.5 * (np.abs(uh[0]) ** 2 + np.abs(uh[1]) ** 2 + np.abs(uh[2]) ** 2)
    valid = (~nyq) & (k2 > 0)
    nsh = int(shell.max()) + 1
    e_shell = np.bincount(shell[valid], weights=e_mode[valid], minlength=nsh)
    ks = np.arange(nsh, dtype=np.float64)
    e_target = ks ** 4 * np.exp(-2.0 * (ks / k0) ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        gain = np.where(e_shell > 0, np.sqrt(e_target / e_shell), 0.0)
    g = np.where(valid, gain[shell], 0.0)
    uh *= g[None]
    u = np.fft.ifftn(uh, axes=(1, 2, 3)).real
    del uh
    rms = np.sqrt(np.mean(u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / 3.0)
    u *= u_rms / rms
    rho = np.ones((n, n, n))
    return rho, np.ascontiguousarray(u)


def spheres(shape, seed, rmin=3.0, rmax=8.0, solid_fraction=0.3, periodic=(0, 1, 1), clear_x=4):
    """Porous medium of random spheres.

    Radius uniform in [rmin, rmax] (real), centres uniform in the box,
    overlaps allowed, periodic images on periodic axes.  A cell (integer
    coordinates) is solid when its distance to a centre is <= r.  The first
    and last ``clear_x`` x-columns stay fluid.  Spheres are added until the
    solid fraction (over the whole box) reaches ``solid_fraction``.
    Returns (solid mask uint8 (nz, ny, nx), achieved fraction, n_spheres).
    """
    nx, ny, nz = shape
    ext = (nx, ny, nz)
    rng = np.random.default_rng(seed)
    solid = np.zeros((nz, ny, nx), np.uint8)
    total = nx * ny * nz
    count = 0
    nsph = 0
    while count < solid_fraction * total:
        c = rng.uniform(0.0, 1.0, 3) * np.array(ext, np.float64)
        r = rng.uniform(rmin, rmax)
        nsph += 1
        lo = [int(np.ceil(c[a] - r)) for a in range(3)]
        hi = [int(np.floor(c[a] + r)) for a in range(3)]
        ranges = []
        for a in range(3):
            idx = np.arange(lo[a], hi[a] + 1)
            d = idx - c[a]
            if periodic[a]:
                idx = idx % ext[a]
            else:
                keep = (idx >= 0) & (idx < ext[a])
                if a == 0:
                    keep &= (idx >= clear_x) & (idx < ext[a] - clear_x)
                idx, d = idx[keep], d[keep]
            ranges.append((idx, d))
        (ix, dx), (iy, dy), (iz, dz) = ranges
        if ix.size == 0 or iy.size == 0 or iz.size == 0:
            continue
        inside = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2) <= r * r
        sub = solid[np.ix_(iz, iy, ix)]
        newly = inside & (sub == 0)
        count += int(newly.sum())
        sub[inside] = 1
        solid[np.ix_(iz, iy, ix)] = sub
    return solid, count / total, nsph


def rectilinear_blocks(edges_x, edges_y, edges_z):
    """Blocks of a rectilinear grid with per-axis edge lists.  Returns
    (list of (origin, size) tuples, domain (nx, ny, nz))."""
    ox = np.concatenate([[0], np.cumsum(edges_x)[:-1]])
    oy = np.concatenate([[0], np.cumsum(edges_y)[:-1]])
    oz = np.concatenate([[0], np.cumsum(edges_z)[:-1]])
    blocks = []
    for k, ez in enumerate(edges_z):
        for j, ey in enumerate(edges_y):
            for i, ex in enumerate(edges_x):
                blocks.append(((int(ox[i]), int(oy[j]), int(oz[k])), (int(ex), int(ey), int(ez))))
    domain = (int(np.sum(edges_x)), int(np.sum(edges_y)), int(np.sum(edges_z)))
    return blocks, domain


def uneven_blocks(seed, per_axis=8, choices=EDGE_CHOICES):
    """Rectilinear per_axis^3 block grid; each axis has per_axis edges drawn
    uniformly from ``choices`` (numpy PCG64 seeded with ``seed``)."""
    rng = np.random.default_rng(seed)
    ch = np.asarray(choices)
    ex = ch[rng.integers(0, len(ch), per_axis)]
    ey = ch[rng.integers(0, len(ch), per_axis)]
    ez = ch[rng.integers(0, len(ch), per_axis)]
    return rectilinear_blocks(ex, ey, ez)


def uniform_blocks(domain, block):
    """Equal blocks of size ``block`` tiling ``domain`` (must divide)."""
    for a in range(3):
        if domain[a] % block[a]:
            raise ValueError("block size must divide the domain")
    ex = [block[0]] * (domain[0] // block[0])
    ey = [block[1]] * (domain[1] // block[1])
    ez = [block[2]] * (domain[2] // block[2])
    return rectilinear_blocks(ex, ey, ez)


def mlp_params(seed, mean=None, inv_std=None, out_bias=0.0, scale=1.0):
    """Random float32 parameters of the 7-32-32-1 closure network, packed as
    mean[7], inv_std[7], W1[32][7], b1[32], W2[32][32], b2[32], w3[32], b3."""
    rng = np.random.default_rng(seed)
    H, I = 32, 7
    mean = np.zeros(I) if mean is None else np.asarray(mean, np.float64)
    inv_std = np.ones(I) if inv_std is None else np.asarray(inv_std, np.float64)
    W1 = rng.uniform(-1, 1, (H, I)) * np.sqrt(6.0 / (H + I)) * scale
    b1 = rng.uniform(-0.1, 0.1, H) * scale
    W2 = rng.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / (2 * H)) * scale
    b2 = rng.uniform(-0.1, 0.1, H) * scale
    w3 = rng.uniform(-1, 1, H) * np.sqrt(6.0 / (H + 1)) * scale
    P = np.concatenate([mean, inv_std, W1.ravel(), b1, W2.ravel(), b2, w3, [out_bias]])
    return P.astype(np.float32)


def turbulence_bandlimited(n, seed, u_rms=0.05, k0=4.0, kmax=20):
    """Decaying-turbulence initial velocity as a band-limited Fourier series.

    Integer wavevectors with |k_a| <= kmax, random phases (PCG64 seeded with
    ``seed``), solenoidal projection, shell-wise amplitudes so the shell
    energy follows E(k) ~ k^4 exp(-2 (k/k0)^2) (negligible beyond kmax = 20
    for k0 = 4), Hermitian symmetry, evaluated on an n^3 grid by separable
    real DFTs (matrix products).  The same seed gives samples of the same
    continuous field at every resolution, so a fine and a coarse run start
    from one flow.  Scaled so the per-component rms velocity is ``u_rms`` on
    the sampled grid.  Returns rho (ones) and u with shape (3, n, n, n).
    """
    rng = np.random.default_rng(seed)
    K = 2 * kmax + 1
    ks = np.arange(-kmax, kmax + 1)
    kz, ky, kx = np.meshgrid(ks, ks, ks, indexing="ij")
    k2 = kx * kx + ky * ky + kz * kz
    uh = rng.standard_normal((3, K, K, K)) + 1j * rng.standard_normal((3, K, K, K))
    # Hermitian symmetry: u(-k) = conj(u(k))
    uh = 0.5 * (uh + np.conj(uh[:, ::-1, ::-1, ::-1]))
    kdotu = kx * uh[0] + ky * uh[1] + kz * uh[2]
    with np.errstate(invalid="ignore", divide="ignore"):
        inv = np.where(k2 > 0, 1.0 / k2, 0.0)
    uh[0] -= kx * kdotu * inv
    uh[1] -= ky * kdotu * inv
    uh[2] -= kz * kdotu * inv
    kmag = np.sqrt(k2)
    shell = np.rint(kmag).astype(np.int64)
    valid = (k2 > 0) & (kmag <= kmax)
    e_mode = 0.5 * (np.abs(uh[0]) ** 2 + np.abs(uh[1]) ** 2 + np.abs(uh[2]) ** 2)
    nsh = int(shell.max()) + 1
    e_shell = np.bincount(shell[valid], weights=e_mode[valid], minlength=nsh)
    kk = np.arange(nsh, dtype=np.float64)
    e_target = kk ** 4 * np.exp(-2.0 * (kk / k0) ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        gain = np.where(e_shell > 0, np.sqrt(e_target / e_shell), 0.0)
    uh = uh * np.where(valid, gain[shell], 0.0)[None]
    x = np.arange(n)
    E = np.exp(2j * np.pi * np.outer(ks, x) / n)  # (K, n): e^{i k x}
    u = np.empty((3, n, n, n))
    for a in range(3):
        # sum over kx: (kz, ky, kx) x (kx, X) -> (kz, ky, X)
        A = uh[a].reshape(K * K, K) @ E
        A = A.reshape(K, K, n)
        # sum over ky: -> (kz, Y, X)
        Bm = np.einsum("zyx,yY->zYx", A, E, optimize=True)
        # sum over kz: -> (Z, Y, X), real part (Hermitian)
        u[a] = (E.T @ Bm.reshape(K, n * n)).real.reshape(n, n, n)
    rms = np.sqrt(np.mean(u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / 3.0)
    u *= u_rms / rms
    return np.ones((n, n, n)), u
