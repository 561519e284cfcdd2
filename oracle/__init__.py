"""FP64 CPU oracle of the lattice Boltzmann update -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it, and it
shares no code with the GPU library.  The arithmetic lives in ``oracle.c``
(plain C, FP64); this module compiles it with gcc and marshals numpy arrays
through ctypes.

Every function follows the paper's statement of the method (Sec. 5.1.1,
Eqs. 1-3) as documented at the top of ``oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MLP_IN = 7
MLP_H = 32
MLP_OFF_MEAN = 0
MLP_OFF_ISTD = 7
MLP_OFF_W1 = 14
MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN
MLP_OFF_W2 = MLP_OFF_B1 + MLP_H
MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H
MLP_OFF_W3 = MLP_OFF_B2 + MLP_H
MLP_OFF_B3 = MLP_OFF_W3 + MLP_H
MLP_NPARAM = MLP_OFF_B3 + 1

SRT, TRT, MRT, KBC, CUMULANT = 0, 1, 2, 3, 4
CLOSURE_NONE, CLOSURE_SMAG, CLOSURE_MLP = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
               "-D_GNU_SOURCE", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("q", C.c_int),
        ("collision", C.c_int),
        ("tau", C.c_double),
        ("magic", C.c_double),
        ("omega_bulk", C.c_double),
        ("omega_higher", C.c_double),
        ("force", C.c_double * 3),
        ("closure", C.c_int),
        ("cs_smag", C.c_double),
        ("mlp", C.POINTER(C.c_double)),
        ("periodic", C.c_int * 3),
        ("pressure_axis", C.c_int),
        ("rho_in", C.c_double),
        ("rho_out", C.c_double),
    ]


@dataclass
class Params:
    """Physical and numerical parameters of one run (see oracle.c)."""
    q: int = 19
    collision: int = SRT
    tau: float = 0.8
    magic: float = 3.0 / 16.0
    omega_bulk: float = 1.0
    omega_higher: float = 1.0
    force: tuple = (0.0, 0.0, 0.0)
    closure: int = CLOSURE_NONE
    cs_smag: float = 0.0
    mlp: np.ndarray | None = None
    periodic: tuple = (1, 1, 1)
    pressure_axis: int = -1
    rho_in: float = 1.0
    rho_out: float = 1.0
    _keep: list = field(default_factory=list, repr=False)

    def to_c(self) -> _Params:
        p = _Params()
        p.q = self.q
        p.collision = self.collision
        p.tau = self.tau
        p.magic = self.magic
        p.omega_bulk = self.omega_bulk
        p.omega_higher = self.omega_higher
        p.force = (C.c_double * 3)(*self.force)
        p.closure = self.closure
        p.cs_smag = self.cs_smag
        if self.mlp is not None:
            arr = np.ascontiguousarray(self.mlp, dtype=np.float64)
            assert arr.size == MLP_NPARAM
            self._keep = [arr]
            p.mlp = arr.ctypes.data_as(C.POINTER(C.c_double))
        else:
            p.mlp = C.POINTER(C.c_double)()
        p.periodic = (C.c_int * 3)(*self.periodic)
        p.pressure_axis = self.pressure_axis
        p.rho_in = self.rho_in
        p.rho_out = self.rho_out
        return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        P = C.POINTER(_Params)
        L.orc_stencil.argtypes = [C.c_int, ip, dp, ip]
        L.orc_mrt_matrix.argtypes = [C.c_int, dp, dp, ip]
        L.orc_collide_cell.argtypes = [P, dp, dp, dp]
        L.orc_equilibrium.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_guo.argtypes = [C.c_int, dp, dp, dp]
        L.orc_init.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, C.c_void_p, dp]
        L.orc_collide.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_void_p, dp, dp, dp, C.c_int]
        L.orc_stream.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_void_p, dp, C.c_void_p, dp]
        L.orc_run.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_void_p, dp, C.c_int, C.c_int]
        L.orc_moments.argtypes = [C.c_int, dp, C.c_int, C.c_int, C.c_int, C.c_void_p, dp, C.c_void_p,
                                  C.c_void_p, C.c_void_p]
        L.orc_momentum_exchange.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_void_p, dp, dp]
        L.orc_bf16_round.argtypes = [C.c_double]
        L.orc_bf16_round.restype = C.c_double
        L.orc_mlp_forward.argtypes = [dp, C.c_int64, dp, dp, ip]
        L.orc_mlp_backward.argtypes = [dp, C.c_int64, dp, dp, C.c_double, dp, dp]
        L.orc_mlp_undecided.argtypes = [dp, C.c_int64, dp, C.c_double, C.c_double, ip, dp]
        L.orc_mlp_nparam.restype = C.c_int
        L.orc_mlp_set_rounding.argtypes = [C.c_int]
        L.orc_gelu.argtypes = [C.c_double]
        L.orc_gelu.restype = C.c_double
        L.orc_softplus.argtypes = [C.c_double]
        L.orc_softplus.restype = C.c_double
        assert L.orc_mlp_nparam() == MLP_NPARAM
        _lib = L
    return _lib


def _chk(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _solid_ptr(solid):
    if solid is None:
        return None, None
    s = np.ascontiguousarray(solid, dtype=np.uint8).reshape(-1)
    return s, s.ctypes.data_as(C.c_void_p)


def stencil(q: int):
    """Velocity set c[q][3], weights w[q], opposite index opp[q]."""
    c = np.zeros(3 * q, np.int32)
    w = np.zeros(q, np.float64)
    o = np.zeros(q, np.int32)
    _chk(lib().orc_stencil(q, c, w, o), "stencil")
    return c.reshape(q, 3), w, o


def mrt_matrix(q: int):
    """Moment matrix M, its inverse and the rate class of each row
    (0 conserved, 1 shear, 2 bulk, 3 higher)."""
    M = np.zeros(q * q)
    Mi = np.zeros(q * q)
    k = np.zeros(q, np.int32)
    _chk(lib().orc_mrt_matrix(q, M, Mi, k), "mrt_matrix")
    return M.reshape(q, q), Mi.reshape(q, q), k


def equilibrium(q: int, rho: float, u) -> np.ndarray:
    """Deviation f_eq - w of one cell."""
    out = np.zeros(q)
    _chk(lib().orc_equilibrium(q, rho, np.asarray(u, np.float64), out), "equilibrium")
    return out


def guo(q: int, u, F) -> np.ndarray:
    out = np.zeros(q)
    _chk(lib().orc_guo(q, np.asarray(u, np.float64), np.asarray(F, np.float64), out), "guo")
    return out


def collide_cell(p: Params, d):
    """Collide one cell; returns (d_post, rho, u, tau)."""
    d = np.ascontiguousarray(d, np.float64)
    out = np.zeros(p.q)
    rut = np.zeros(5)
    _chk(lib().orc_collide_cell(C.byref(p.to_c()), d, out, rut), "collide_cell")
    return out, rut[0], rut[1:4].copy(), rut[4]


def init(q: int, shape, rho, u, solid=None) -> np.ndarray:
    """d[q][N] = f_eq(rho, u) - w; shape = (nx, ny, nz); arrays x-fastest."""
    nx, ny, nz = shape
    N = nx * ny * nz
    rho = np.ascontiguousarray(rho, np.float64).reshape(-1)
    u = np.ascontiguousarray(u, np.float64).reshape(-1)
    assert rho.size == N and u.size == 3 * N
    s, sp = _solid_ptr(solid)
    d = np.zeros(q * N)
    _chk(lib().orc_init(q, nx, ny, nz, rho, u, sp, d), "init")
    return d.reshape(q, N)


def collide(p: Params, shape, d, solid=None, nthreads=0):
    nx, ny, nz = shape
    N = nx * ny * nz
    d = np.ascontiguousarray(d, np.float64).reshape(-1)
    s, sp = _solid_ptr(solid)
    post = np.zeros(p.q * N)
    uvel = np.zeros(3 * N)
    _chk(lib().orc_collide(C.byref(p.to_c()), nx, ny, nz, sp, d, post, uvel, nthreads), "collide")
    return post.reshape(p.q, N), uvel.reshape(3, N)


def stream(p: Params, shape, post, solid=None, uvel=None):
    nx, ny, nz = shape
    N = nx * ny * nz
    post = np.ascontiguousarray(post, np.float64).reshape(-1)
    s, sp = _solid_ptr(solid)
    up = None
    if uvel is not None:
        uvel = np.ascontiguousarray(uvel, np.float64).reshape(-1)
        up = uvel.ctypes.data_as(C.c_void_p)
    out = np.zeros(p.q * N)
    _chk(lib().orc_stream(C.byref(p.to_c()), nx, ny, nz, sp, post, up, out), "stream")
    return out.reshape(p.q, N)


def run(p: Params, shape, d, nsteps: int, solid=None, nthreads=0) -> np.ndarray:
    """nsteps updates of d (copied); returns the new d[q][N]."""
    nx, ny, nz = shape
    d = np.array(d, np.float64, copy=True).reshape(-1)
    s, sp = _solid_ptr(solid)
    _chk(lib().orc_run(C.byref(p.to_c()), nx, ny, nz, sp, d, int(nsteps), int(nthreads)), "run")
    return d.reshape(p.q, -1)


def moments(q: int, force, shape, d, solid=None):
    """rho[N], u[3][N], totals[8] (mass, momentum xyz, kinetic energy, max|u|, n_fluid, 0)."""
    nx, ny, nz = shape
    N = nx * ny * nz
    d = np.ascontiguousarray(d, np.float64).reshape(-1)
    s, sp = _solid_ptr(solid)
    rho = np.zeros(N)
    u = np.zeros(3 * N)
    tot = np.zeros(8)
    _chk(lib().orc_moments(q, np.asarray(force, np.float64), nx, ny, nz, sp, d,
                           rho.ctypes.data_as(C.c_void_p), u.ctypes.data_as(C.c_void_p),
                           tot.ctypes.data_as(C.c_void_p)), "moments")
    return rho, u.reshape(3, N), tot


def momentum_exchange(p: Params, shape, d, solid=None):
    """Force handed to the obstacles during the step that starts from state d
    (momentum exchange over the half-way bounce-back links): the step's
    collision, then 2 c_j f*_j summed over links whose target is a solid cell
    or beyond a wall.  Returns [F_solid x, y, z, F_wall x, y, z, n_solid_links,
    n_wall_links]."""
    nx, ny, nz = shape
    post, _ = collide(p, shape, d, solid)
    s, sp = _solid_ptr(solid)
    out = np.zeros(8)
    _chk(lib().orc_momentum_exchange(C.byref(p.to_c()), nx, ny, nz, sp,
                                     np.ascontiguousarray(post, np.float64).reshape(-1), out),
         "momentum_exchange")
    return out


def bf16_round(v: float) -> float:
    return lib().orc_bf16_round(float(v))


def gelu(z: float) -> float:
    return lib().orc_gelu(float(z))


def softplus(o: float) -> float:
    return lib().orc_softplus(float(o))


def mlp_set_rounding(on: bool) -> None:
    """Switch the bf16 operand rounding off only for finite-difference checks."""
    lib().orc_mlp_set_rounding(1 if on else 0)


def mlp_forward(params, raw):
    """raw[n][7] -> (o[n], fallback_flag[n])."""
    P = np.ascontiguousarray(params, np.float64)
    raw = np.ascontiguousarray(raw, np.float64).reshape(-1, MLP_IN)
    n = raw.shape[0]
    o = np.zeros(n)
    flag = np.zeros(n, np.int32)
    _chk(lib().orc_mlp_forward(P, n, raw, o, flag), "mlp_forward")
    return o, flag


def mlp_undecided(params, raw, rel0: float, rel2: float):
    """Per sample: the number of bf16 rounding decisions that a
    single-precision evaluation may take differently (operand within its
    error bound of a rounding boundary; GELU(z) evaluated with relative error
    at most rel0 + rel2 z^2), and the summed change of the output when each
    of them alone goes the other way (see orc_mlp_undecided)."""
    P = np.ascontiguousarray(params, np.float64)
    raw = np.ascontiguousarray(raw, np.float64).reshape(-1, MLP_IN)
    n = raw.shape[0]
    cnt = np.zeros(n, np.int32)
    flip = np.zeros(n)
    _chk(lib().orc_mlp_undecided(P, n, raw, float(rel0), float(rel2), cnt, flip), "mlp_undecided")
    return cnt, flip


def mlp_backward(params, raw, target, inv_scale: float):
    """Gradient of L = mean(((softplus(o) - t) * inv_scale)^2); returns (grad, L)."""
    P = np.ascontiguousarray(params, np.float64)
    raw = np.ascontiguousarray(raw, np.float64).reshape(-1, MLP_IN)
    t = np.ascontiguousarray(target, np.float64).reshape(-1)
    g = np.zeros(MLP_NPARAM)
    L = np.zeros(1)
    _chk(lib().orc_mlp_backward(P, raw.shape[0], raw, t, float(inv_scale), g, L), "mlp_backward")
    return g, float(L[0])
