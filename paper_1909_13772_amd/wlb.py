"""ctypes binding of libwlb.so (C ABI in include/wlb.h).

The functions ``wlb_*`` mirror the C entry points one to one (argument
marshalling only).  ``Blocks`` is a thin convenience wrapper that allocates
the device arena and the HIP stream with PyTorch (PyTorch provides device
memory and streams only; every step of the method runs in the library's HIP
kernels).  Importing this module raises if the library has not been built:
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# WLB_LIBRARY may point at another build of the same library (e.g. a debug build).
LIB_PATH = os.environ.get("WLB_LIBRARY") or os.path.join(_HERE, "libwlb.so")

WLB_OK = 0
WLB_ERR_ARG = -1
WLB_ERR_HIP = -2
WLB_ERR_STATE = -3
WLB_ERR_DIVERGED = -4
WLB_ERR_UNSUPPORTED = -5

D2Q9, D3Q15, D3Q19, D3Q27 = 9, 15, 19, 27
SRT, TRT, MRT, KBC, CUMULANT = 0, 1, 2, 3, 4
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
CLOSURE_NONE, CLOSURE_SMAG, CLOSURE_MLP = 0, 1, 2
MLP_NPARAM = 1359
MLP_NOALLOC_MAX_SAMPLES = 262144
ELEM_BYTES = {F64: 8, F32: 4, F16DEV: 2, BF16DEV: 2}
STORAGE_NAMES = {F64: "f64", F32: "f32", F16DEV: "f16dev", BF16DEV: "bf16dev"}


class WlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"wlb error {code}: {msg}")
        self.code = code


class wlb_block_desc(C.Structure):
    _fields_ = [("origin", C.c_int32 * 3), ("size", C.c_int32 * 3)]


class wlb_lbm_params(C.Structure):
    _fields_ = [
        ("tau", C.c_double),
        ("magic", C.c_double),
        ("omega_bulk", C.c_double),
        ("omega_higher", C.c_double),
        ("force", C.c_double * 3),
        ("closure", C.c_int32),
        ("cs_smag", C.c_double),
        ("mlp", C.POINTER(C.c_float)),
        ("pressure_axis", C.c_int32),
        ("rho_in", C.c_double),
        ("rho_out", C.c_double),
        ("health_every", C.c_int32),
        ("health_umax", C.c_double),
        ("autotune", C.c_int32),
    ]


class wlb_info_t(C.Structure):
    _fields_ = [
        ("steps", C.c_int64),
        ("parity", C.c_int32),
        ("n_blocks", C.c_int32),
        ("n_cells", C.c_int64),
        ("n_fluid", C.c_int64),
        ("n_tiles", C.c_int32),
        ("tile", C.c_int32 * 3),
        ("grid", C.c_int32),
        ("lds_staging", C.c_int32),
        ("n_xchg_items", C.c_int32),
        ("xchg_elems", C.c_int64),
        ("arena_bytes", C.c_size_t),
        ("pop_bytes", C.c_size_t),
        ("overlap", C.c_int32),
        ("nt_even", C.c_int32),
        ("nt_odd", C.c_int32),
        ("n_class_tiles", C.c_int32),
        ("slot_round_kib", C.c_int32),
    ]


# PyTorch ships its own HIP runtime with the same soname as the system one;
# importing it first makes libwlb.so bind to that single runtime, so arena
# pointers and streams created by PyTorch are valid in the library.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_1909_13772_amd/build.py "
                      "(the HIP library is the only compute path)")

_lib = C.CDLL(LIB_PATH)
_vp = C.c_void_p
_h = C.c_void_p

_sig = {
    "wlb_blocks_create": (C.c_int, [C.POINTER(wlb_block_desc), C.c_int32, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.c_int32, C.c_int32, C.POINTER(C.c_size_t),
                                    C.POINTER(_h)]),
    "wlb_blocks_bind": (C.c_int, [_h, _vp, C.c_size_t, _vp]),
    "wlb_lbm_init": (C.c_int, [_h, C.c_int32, C.POINTER(wlb_lbm_params), _vp, _vp, _vp]),
    "wlb_lbm_step": (C.c_int, [_h, C.c_int32]),
    "wlb_lbm_sweep": (C.c_int, [_h]),
    "wlb_ghost_exchange": (C.c_int, [_h]),
    "wlb_moments_get": (C.c_int, [_h, _vp, _vp, _vp]),
    "wlb_force_get": (C.c_int, [_h, _vp]),
    "wlb_debug_write_coverage": (C.c_int, [_h, C.c_int32, _vp]),
    "wlb_pdfs_get": (C.c_int, [_h, _vp]),
    "wlb_pdfs_set": (C.c_int, [_h, _vp]),
    "wlb_info": (C.c_int, [_h, C.POINTER(wlb_info_t)]),
    "wlb_set_tiles": (C.c_int, [_h, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "wlb_set_graph": (C.c_int, [_h, C.c_int32]),
    "wlb_set_lds_staging": (C.c_int, [_h, C.c_int32]),
    "wlb_set_nontemporal": (C.c_int, [_h, C.c_int32, C.c_int32]),
    "wlb_set_class_tiles": (C.c_int, [_h, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "wlb_set_slot_round": (C.c_int, [_h, C.c_int32]),
    "wlb_set_overlap": (C.c_int, [_h, C.c_int32]),
    "wlb_set_kernel_timing": (C.c_int, [_h, C.c_int32]),
    "wlb_kernel_times": (C.c_int, [_h, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "wlb_blocks_destroy": (None, [_h]),
    "wlb_last_error": (C.c_char_p, []),
    "wlb_copy_probe": (C.c_int, [_vp, _vp, C.c_size_t, C.c_int32, _vp, C.POINTER(C.c_double)]),
    "wlb_box_filter": (C.c_int, [_h, C.c_int32, _vp]),
    "wlb_les_targets": (C.c_int, [_vp, C.POINTER(C.c_int32), C.c_double, _vp, _vp, _vp]),
    "wlb_mlp_forward": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, _vp, _vp]),
    "wlb_mlp_grad_workspace": (C.c_size_t, [C.c_int64]),
    "wlb_mlp_grad": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_double, _vp, _vp, _vp, C.c_size_t, _vp]),
    "wlb_mlp_grad_noalloc": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.c_double, _vp, _vp, _vp]),
    "wlb_mlp_adam": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double, _vp]),
}
for _n, (_r, _a) in _sig.items():
    _f = getattr(_lib, _n)
    _f.restype = _r
    _f.argtypes = _a

EXPORTED = tuple(_sig.keys())


def wlb_last_error() -> str:
    return _lib.wlb_last_error().decode()


def _check(rc):
    if rc != WLB_OK:
        raise WlbError(rc, wlb_last_error())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_vp)


# --- one-to-one wrappers ---------------------------------------------------
def wlb_blocks_create(blocks, domain, periodic, stencil, storage):
    """blocks: list of ((ox, oy, oz), (nx, ny, nz)).  Returns (handle, arena_bytes)."""
    n = len(blocks)
    arr = (wlb_block_desc * n)()
    for k, (o, s) in enumerate(blocks):
        arr[k].origin = (C.c_int32 * 3)(*o)
        arr[k].size = (C.c_int32 * 3)(*s)
    dom = (C.c_int32 * 3)(*domain)
    per = (C.c_int32 * 3)(*[1 if p else 0 for p in periodic])
    nbytes = C.c_size_t(0)
    h = _h()
    _check(_lib.wlb_blocks_create(arr, n, dom, per, stencil, storage, C.byref(nbytes), C.byref(h)))
    return h, nbytes.value


def wlb_blocks_bind(h, arena_ptr: int, nbytes: int, stream_ptr: int):
    _check(_lib.wlb_blocks_bind(h, _vp(arena_ptr), nbytes, _vp(stream_ptr)))


def wlb_lbm_init(h, collision, params: wlb_lbm_params, rho, u, solid=None):
    _check(_lib.wlb_lbm_init(h, collision, C.byref(params), _ptr(rho), _ptr(u), _ptr(solid)))


def wlb_lbm_step(h, n: int):
    _check(_lib.wlb_lbm_step(h, int(n)))


def wlb_lbm_sweep(h):
    _check(_lib.wlb_lbm_sweep(h))


def wlb_ghost_exchange(h):
    _check(_lib.wlb_ghost_exchange(h))


def wlb_moments_get(h, rho, u, totals):
    _check(_lib.wlb_moments_get(h, _ptr(rho), _ptr(u), _ptr(totals)))


def wlb_force_get(h, out):
    _check(_lib.wlb_force_get(h, _ptr(out)))


def wlb_debug_write_coverage(h, odd, counts):
    _check(_lib.wlb_debug_write_coverage(h, int(odd), _ptr(counts)))


def wlb_pdfs_get(h, d):
    _check(_lib.wlb_pdfs_get(h, _ptr(d)))


def wlb_pdfs_set(h, d):
    _check(_lib.wlb_pdfs_set(h, _ptr(d)))


def wlb_info(h) -> wlb_info_t:
    o = wlb_info_t()
    _check(_lib.wlb_info(h, C.byref(o)))
    return o


def wlb_set_tiles(h, tx, ty, tz, grid):
    _check(_lib.wlb_set_tiles(h, tx, ty, tz, grid))


def wlb_set_slot_round(h, kib):
    _check(_lib.wlb_set_slot_round(h, int(kib)))


def wlb_set_lds_staging(h, on):
    """Odd-sweep kernel: False / 0 direct, True / 1 LDS-staged, 2 row vectors."""
    _check(_lib.wlb_set_lds_staging(h, int(on)))


def wlb_set_overlap(h, on):
    _check(_lib.wlb_set_overlap(h, 1 if on else 0))


def wlb_set_graph(h, on):
    _check(_lib.wlb_set_graph(h, 1 if on else 0))


def wlb_set_kernel_timing(h, on):
    _check(_lib.wlb_set_kernel_timing(h, 1 if on else 0))


def wlb_kernel_times(h):
    ms = (C.c_double * 4)()
    n = (C.c_int64 * 4)()
    _check(_lib.wlb_kernel_times(h, ms, n))
    return list(ms), list(n)


def wlb_blocks_destroy(h):
    _lib.wlb_blocks_destroy(h)


def wlb_copy_probe(dst_ptr, src_ptr, nbytes, reps, stream_ptr):
    ms = C.c_double(0.0)
    _check(_lib.wlb_copy_probe(_vp(dst_ptr), _vp(src_ptr), nbytes, reps, _vp(stream_ptr), C.byref(ms)))
    return ms.value


MLP_WORKSPACE = 4096


def wlb_box_filter(h, factor, out_ptr):
    _check(_lib.wlb_box_filter(h, int(factor), _vp(out_ptr)))


def wlb_les_targets(filt_ptr, nc, tau0, raw_ptr, target_ptr, stream_ptr):
    n = (C.c_int32 * 3)(*nc)
    _check(_lib.wlb_les_targets(_vp(filt_ptr), n, float(tau0), _vp(raw_ptr), _vp(target_ptr), _vp(stream_ptr)))


def wlb_mlp_forward(params, workspace_ptr, raw_ptr, n, out_ptr, fallback_ptr, stream_ptr):
    p = np.ascontiguousarray(params, np.float32)
    assert p.size == MLP_NPARAM
    _check(_lib.wlb_mlp_forward(p.ctypes.data_as(_vp), _vp(workspace_ptr), _vp(raw_ptr), int(n), _vp(out_ptr),
                                _vp(fallback_ptr), _vp(stream_ptr)))


def wlb_mlp_grad_workspace(n):
    return _lib.wlb_mlp_grad_workspace(int(n))


def wlb_mlp_grad(params_ptr, raw_ptr, target_ptr, n, inv_scale, grad_ptr, loss_ptr, ws_ptr, ws_bytes, stream_ptr):
    _check(_lib.wlb_mlp_grad(_vp(params_ptr), _vp(raw_ptr), _vp(target_ptr), int(n), float(inv_scale), _vp(grad_ptr),
                             _vp(loss_ptr), _vp(ws_ptr), int(ws_bytes), _vp(stream_ptr)))


def wlb_mlp_grad_noalloc(params_ptr, raw_ptr, target_ptr, n, inv_scale, grad_ptr, loss_ptr, stream_ptr):
    _check(_lib.wlb_mlp_grad_noalloc(_vp(params_ptr), _vp(raw_ptr), _vp(target_ptr), int(n), float(inv_scale),
                                     _vp(grad_ptr), _vp(loss_ptr), _vp(stream_ptr)))


def wlb_mlp_adam(params_ptr, grad_ptr, m_ptr, v_ptr, step, lr, beta1, beta2, eps, stream_ptr):
    _check(_lib.wlb_mlp_adam(_vp(params_ptr), _vp(grad_ptr), _vp(m_ptr), _vp(v_ptr), int(step), float(lr),
                             float(beta1), float(beta2), float(eps), _vp(stream_ptr)))


# --- convenience wrapper ---------------------------------------------------
def make_params(tau=0.8, magic=3.0 / 16.0, omega_bulk=1.0, omega_higher=1.0, force=(0.0, 0.0, 0.0),
                closure=CLOSURE_NONE, cs_smag=0.0, mlp=None, pressure_axis=-1, rho_in=1.0, rho_out=1.0,
                health_every=0, health_umax=0.0, autotune=0):
    p = wlb_lbm_params()
    p.tau, p.magic, p.omega_bulk, p.omega_higher = tau, magic, omega_bulk, omega_higher
    p.force = (C.c_double * 3)(*force)
    p.closure, p.cs_smag = closure, cs_smag
    keep = None
    if mlp is not None:
        keep = np.ascontiguousarray(mlp, dtype=np.float32)
        assert keep.size == MLP_NPARAM
        p.mlp = keep.ctypes.data_as(C.POINTER(C.c_float))
    p.pressure_axis, p.rho_in, p.rho_out = pressure_axis, rho_in, rho_out
    p.health_every, p.health_umax, p.autotune = health_every, health_umax, autotune
    p._keep = keep  # keep the weight buffer alive with the struct
    return p


class Blocks:
    """A block set on one GPU: arena and stream from PyTorch, compute in libwlb."""

    def __init__(self, blocks, domain, periodic=(1, 1, 1), stencil=D3Q19, storage=F64, device="cuda"):
        import torch

        self.torch = torch
        self.domain = tuple(int(v) for v in domain)
        self.stencil = stencil
        self.storage = storage
        self.h, self.nbytes = wlb_blocks_create(blocks, self.domain, periodic, stencil, storage)
        try:
            self.stream = torch.cuda.Stream(device=device)
            self.arena = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
            base = self.arena.data_ptr()
            self._aligned = (base + 255) // 256 * 256
            wlb_blocks_bind(self.h, self._aligned, self.nbytes, self.stream.cuda_stream)
        except Exception:
            wlb_blocks_destroy(self.h)
            self.h = None
            raise

    @property
    def ncells(self):
        nx, ny, nz = self.domain
        return nx * ny * nz

    def init(self, collision, params, rho, u, solid=None):
        rho = np.ascontiguousarray(rho, np.float64).reshape(-1)
        u = np.ascontiguousarray(u, np.float64).reshape(-1)
        if rho.size != self.ncells or u.size != 3 * self.ncells:
            raise ValueError("rho/u do not match the domain")
        s = None
        if solid is not None:
            s = np.ascontiguousarray(solid, np.uint8).reshape(-1)
            if s.size != self.ncells:
                raise ValueError("solid does not match the domain")
        wlb_lbm_init(self.h, collision, params, rho, u, s)

    def step(self, n=1):
        wlb_lbm_step(self.h, n)

    def sweep(self):
        wlb_lbm_sweep(self.h)

    def exchange(self):
        wlb_ghost_exchange(self.h)

    def force(self):
        """Momentum exchanged with the obstacles during the last step:
        [F_solid x, y, z, F_wall x, y, z, n_solid_links, n_wall_links]."""
        out = np.zeros(8)
        wlb_force_get(self.h, out)
        return out

    def write_coverage(self, odd):
        """Writes per (slot, cell) of one sweep of parity `odd` and its
        exchange, as uint32 [q][N]; the state is gone afterwards (init again)."""
        counts = np.zeros((self.stencil, self.ncells), np.uint32)
        wlb_debug_write_coverage(self.h, odd, counts)
        return counts

    def moments(self, fields=True):
        nx, ny, nz = self.domain
        tot = np.zeros(8)
        if fields:
            rho = np.zeros(self.ncells)
            u = np.zeros(3 * self.ncells)
            wlb_moments_get(self.h, rho, u, tot)
            return rho.reshape(nz, ny, nx), u.reshape(3, nz, ny, nx), tot
        wlb_moments_get(self.h, None, None, tot)
        return None, None, tot

    def pdfs_get(self):
        d = np.zeros(self.stencil * self.ncells)
        wlb_pdfs_get(self.h, d)
        return d.reshape(self.stencil, self.ncells)

    def pdfs_set(self, d):
        d = np.ascontiguousarray(d, np.float64).reshape(-1)
        if d.size != self.stencil * self.ncells:
            raise ValueError("population array does not match")
        wlb_pdfs_set(self.h, d)

    def info(self):
        return wlb_info(self.h)

    def set_tiles(self, tx, ty, tz, grid=0):
        wlb_set_tiles(self.h, tx, ty, tz, grid)

    def set_lds_staging(self, on):
        wlb_set_lds_staging(self.h, on)

    def set_nontemporal(self, even, odd):
        # odd: 0 cached, 1 non-temporal, 2 non-temporal on the aligned accesses only
        _check(_lib.wlb_set_nontemporal(self.h, int(bool(even)), int(odd)))

    def set_class_tiles(self, y_extent, tx, ty, tz):
        _check(_lib.wlb_set_class_tiles(self.h, int(y_extent), int(tx), int(ty), int(tz)))

    def set_slot_round(self, kib):
        _check(_lib.wlb_set_slot_round(self.h, int(kib)))

    def set_overlap(self, on):
        wlb_set_overlap(self.h, on)

    def set_graph(self, on):
        wlb_set_graph(self.h, on)

    def set_kernel_timing(self, on):
        wlb_set_kernel_timing(self.h, on)

    def kernel_times(self):
        return wlb_kernel_times(self.h)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.h is not None:
            wlb_blocks_destroy(self.h)
            self.h = None
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def single_block(domain):
    return [((0, 0, 0), tuple(domain))]
