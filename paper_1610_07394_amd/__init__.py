"""Python binding of libsmx (recursive block-space maps onto discrete
orthogonal simplices, MI355X / gfx950).

Argument marshalling only: every step runs in the HIP kernels of libsmx.so,
called through its C ABI (include/smx.h) with ctypes.  PyTorch provides device
memory and the current HIP stream.  If libsmx.so is missing, or a tensor is not
on the GPU, the calls raise; there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = [
    "MAPS", "PRECS", "SmxError", "Pot", "lib", "volume", "parallel_blocks", "map_tiles_host", "map_blocks_host",
    "workspace_bytes", "simplex_map2", "simplex_map3", "simplex_map4", "simplex_count", "triplet_packed", "triplet_packed_tiled", "triplet_tiled_len", "edm_tiled", "edm_tiled_len", "life_len", "simplex_life", "simplex_decode", "quad_contacts", "edm_packed", "triplet_energy",
    "triplet_energy_grad", "triplet_energy_grad_noalloc", "NOALLOC_MAX_N", "triplet_energy_backward", "TripletEnergy", "profile_enable",
    "profile_reset", "profile_read", "KERNELS", "select_library", "check_flags",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmx.so")
# the same library with device checks compiled in (see smx_check_flags)
LIB_CHECKED_PATH = os.path.join(_HERE, "libsmx_checked.so")

MAPS = {"lambda": 0, "bbox": 1, "linear": 2, "lambda_below": 3, "recursive": 4, "recursive_launch": 5}
PRECS = {"fp32": 0, "bf16": 1, "split_bf16": 2}
KERNELS = {"map2": 0, "map3": 1, "edm_diff": 2, "edm_gram": 3, "gram_prep": 4,
           "triplet_energy": 5, "triplet_grad": 6, "lj": 7, "finalize": 8, "triplet_packed": 9, "map4": 10,
           "quad_words": 11, "quad": 12, "triplet_tiled": 13, "life": 14, "decode": 15}

_i32, _i64, _sz, _vp, _dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double


class _Pot(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("at_on", ctypes.c_int32), ("lj_on", ctypes.c_int32),
                ("lj_eps", ctypes.c_double), ("lj_sigma", ctypes.c_double), ("lj_rc", ctypes.c_double)]


@dataclass(frozen=True)
class Pot:
    """Axilrod-Teller coefficient nu and optional Lennard-Jones pairs."""
    nu: float = 1.0
    at: bool = True
    lj: bool = False
    eps: float = 1.0
    sigma: float = 1.0
    rc: float = 3.0

    def _c(self) -> _Pot:
        return _Pot(self.nu, int(self.at), int(self.lj), self.eps, self.sigma, self.rc)


class SmxError(RuntimeError):
    pass


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_1610_07394_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        L.smx_version.restype = ctypes.c_char_p
        L.smx_last_error.restype = ctypes.c_char_p
        L.smx_volume.argtypes = [_i32, _i64, _i32]
        L.smx_volume.restype = _i64
        L.smx_parallel_blocks.argtypes = [_i32, _i64, _i32, _i32]
        L.smx_parallel_blocks.restype = _i64
        L.smx_map_tiles_host.argtypes = [_i32, _i64, _i32, _i32, _i64, _i64, _vp]
        L.smx_workspace_bytes.argtypes = [_i32, _i64, _i64, _i32, _i32]
        L.smx_workspace_bytes.restype = _sz
        for name in ("smx_simplex_map2", "smx_simplex_map3", "smx_simplex_map4"):
            getattr(L, name).argtypes = [_i64, _i32, _i32, _i32, _vp, _vp, _vp, _sz, _vp]
        L.smx_simplex_count.argtypes = [_i32, _i64, _i32, _i32, _i32, _vp, _vp, _sz, _vp]
        L.smx_triplet_packed.argtypes = [_vp, _i64, _i64, _dbl, _i32, _vp, _vp, _sz, _vp, _vp]
        L.smx_edm_tiled.argtypes = [_vp, _i64, _i64, _i64, _i32, _i32, _vp, _vp, _sz, _vp, _vp]
        L.smx_simplex_life.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp, _sz, _vp]
        L.smx_simplex_decode.argtypes = [_i32, _i64, _i32, _vp, _vp, _sz, _vp]
        L.smx_triplet_packed_tiled.argtypes = [_vp, _i64, _i64, _dbl, _i32, _vp, _vp, _sz, _vp, _vp]
        L.smx_quad_contacts.argtypes = [_vp, _i64, _i64, _dbl, _i32, _vp, _vp, _sz, _vp, _vp]
        L.smx_check_flags.argtypes = [ctypes.POINTER(ctypes.c_uint32), _i32]
        L.smx_map_blocks_host.argtypes = [_i32, _i64, _i32, _i32, _vp, _i64, _vp]
        L.smx_probe_valu.argtypes = [_vp, _i64, _i32, _vp]
        L.smx_edm_packed.argtypes = [_vp, _i64, _i64, _i64, _i32, _i32, _vp, _vp, _sz, _vp, _vp]
        L.smx_triplet_energy.argtypes = [_vp, _i64, _i64, ctypes.POINTER(_Pot), _i32, _vp, _vp, _sz, _vp, _vp]
        L.smx_triplet_energy_grad.argtypes = [_vp, _i64, _i64, ctypes.POINTER(_Pot), _i32, _vp, _vp, _vp,
                                              _sz, _vp]
        L.smx_triplet_energy_grad_noalloc.argtypes = [_vp, _i64, _i64, ctypes.POINTER(_Pot), _i32, _vp, _vp, _vp]
        L.smx_triplet_energy_backward.argtypes = [_vp, _i64, _i64, ctypes.POINTER(_Pot), _i32, _vp, _vp,
                                                  _vp, _sz, _vp]
        L.smx_scale_grad.argtypes = [_vp, _i64, _vp, _vp, _vp]
        L.smx_profile_enable.argtypes = [_i32]
        L.smx_profile_read.argtypes = [_i32, ctypes.POINTER(_dbl), ctypes.POINTER(_i64)]
        _lib = L
    return _lib


def version() -> str:
    return lib().smx_version().decode()


def _check(rc: int) -> None:
    if rc == 0:
        return
    msg = lib().smx_last_error().decode()
    if rc == 1:
        raise ValueError(msg)
    if rc == 2:
        raise OverflowError(msg)
    if rc == 3:
        raise NotImplementedError(msg)
    raise SmxError(msg)


def select_library(checked: bool) -> None:
    """Route every later call through libsmx_checked.so (device checks compiled
    in) or back through libsmx.so.  Both are built in-tree by build.py."""
    global LIB_PATH, _lib
    LIB_PATH = LIB_CHECKED_PATH if checked else os.path.join(_HERE, "libsmx.so")
    _lib = None


def check_flags(clear: bool = True) -> int:
    """Device check flags of the checked library (bit 1: a map left the simplex,
    bit 2: a store left it); synchronises with the device."""
    v = ctypes.c_uint32(0)
    _check(lib().smx_check_flags(ctypes.byref(v), int(clear)))
    return int(v.value)


def _map(m) -> int:
    return MAPS[m] if isinstance(m, str) else int(m)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (got device {t.device})")
    return t.data_ptr()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- host queries
def volume(m: int, n: int, strict: bool = False) -> int:
    return int(lib().smx_volume(m, n, int(strict)))


def parallel_blocks(m: int, n: int, rho: int, map="lambda") -> int:
    v = int(lib().smx_parallel_blocks(m, n, rho, _map(map)))
    if v < 0:
        raise ValueError(f"no parallel space for m={m}, n={n}, rho={rho}, map={map}")
    return v


def map_tiles_host(m: int, n: int, rho: int, map="lambda", first: int = 0, count: int | None = None):
    """Tiles of launched blocks [first, first + count), evaluated on the host (numpy int32 [count, m])."""
    import numpy as np
    if count is None:
        count = parallel_blocks(m, n, rho, map) - first
    out = np.empty((count, m), dtype=np.int32)
    _check(lib().smx_map_tiles_host(m, n, rho, _map(map), first, count, out.ctypes.data))
    return out


def map_blocks_host(m: int, n: int, rho: int, tiles, map="lambda"):
    """Block index of each tile (numpy int32 [count, m]) under `map` (the inverse map), on the host."""
    import numpy as np
    t = np.ascontiguousarray(tiles, dtype=np.int32).reshape(-1, m)
    out = np.empty(t.shape[0], dtype=np.int64)
    _check(lib().smx_map_blocks_host(m, n, rho, _map(map), t.ctypes.data, t.shape[0], out.ctypes.data))
    return out


def workspace_bytes(op: int, n: int, d: int = 3, prec: int = 0, map="lambda") -> int:
    return int(lib().smx_workspace_bytes(op, n, d, prec, _map(map)))


def _ws(nbytes: int, device) -> torch.Tensor | None:
    if nbytes == 0:
        return None
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- map dumps
def _simplex_map(m: int, n: int, rho: int, map, strict: bool, tiles: bool, stats: bool, device):
    device = torch.device(device)
    g = parallel_blocks(m, n, rho, map)
    t = torch.empty((g, m), dtype=torch.int32, device=device) if tiles else None
    s = torch.zeros(4, dtype=torch.int64, device=device) if stats else None
    ws = _ws(workspace_bytes(0, n), device) if stats else None
    fn = {2: lib().smx_simplex_map2, 3: lib().smx_simplex_map3, 4: lib().smx_simplex_map4}[m]
    _check(fn(n, rho, _map(map), int(strict), _ptr(t), _ptr(s), _ptr(ws), 0 if ws is None else ws.numel(),
              _stream()))
    return t, s


def simplex_map2(n: int, rho: int, map="lambda", strict=False, tiles=True, stats=True, device="cuda"):
    """Run the 2-simplex parallel space; returns (tiles int32 [G, 2] | None, stats int64 [4] | None)."""
    return _simplex_map(2, n, rho, map, strict, tiles, stats, device)


def simplex_map3(n: int, rho: int, map="lambda", strict=False, tiles=True, stats=True, device="cuda"):
    """Run the 3-simplex parallel space; returns (tiles int32 [G, 3] | None, stats int64 [4] | None)."""
    return _simplex_map(3, n, rho, map, strict, tiles, stats, device)


def simplex_map4(n: int, rho: int, map="lambda", strict=False, tiles=True, stats=True, device="cuda"):
    """Run the 4-simplex parallel space; returns (tiles int32 [G, 4] | None, stats int64 [4] | None)."""
    return _simplex_map(4, n, rho, map, strict, tiles, stats, device)


def simplex_count(m: int, n: int, rho: int, map="lambda", strict=False, device="cuda"):
    """Parallel space only: int64 [4] = elements (closed form per mapped tile),
    0, mapped blocks, launched blocks."""
    device = torch.device(device)
    s = torch.zeros(4, dtype=torch.int64, device=device)
    ws = _ws(workspace_bytes(0, n), device)
    _check(lib().smx_simplex_count(m, n, rho, _map(map), int(strict), _ptr(s), _ptr(ws), ws.numel(), _stream()))
    return s


# ---------------------------------------------------------------- EDM
def edm_packed(X: torch.Tensor, map="lambda", prec="fp32", stats=False, out=None, ws=None):
    """Packed upper-triangle squared distances of the rows of X (FP32 [n, d])."""
    if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a row-major FP32 matrix")
    n, d = X.shape
    ldx = X.stride(0) if n > 0 else d
    p = PRECS[prec] if isinstance(prec, str) else int(prec)
    D = out if out is not None else torch.empty(n * (n + 1) // 2, dtype=torch.float32, device=X.device)
    s = torch.zeros(4, dtype=torch.int64, device=X.device) if stats else None
    need = workspace_bytes(1, n, d, p, map)
    if ws is None and (p != 0 or stats):
        ws = _ws(need, X.device)
    _check(lib().smx_edm_packed(_dev(X, "X"), n, d, ldx, _map(map), p, _ptr(D), _ptr(ws),
                                0 if ws is None else ws.numel(), _ptr(s), _stream()))
    return (D, s) if stats else D


def edm_tiled_len(n: int) -> int:
    """Floats of the tile-contiguous EDM layout: nb(nb+1)/2 tiles of 128 x 128."""
    nb = -(-n // 128)
    return nb * (nb + 1) // 2 * 16384


def edm_tiled(X: torch.Tensor, map="lambda", prec="fp32", stats=False, out=None, ws=None):
    """Squared distances of the rows of X in the tile-contiguous layout (FP32
    [edm_tiled_len(n)], see smx_edm_tiled)."""
    if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a row-major FP32 matrix")
    n, d = X.shape
    ldx = X.stride(0) if n > 0 else d
    p = PRECS[prec] if isinstance(prec, str) else int(prec)
    D = out if out is not None else torch.empty(edm_tiled_len(n), dtype=torch.float32, device=X.device)
    if D.dtype != torch.float32 or D.numel() < edm_tiled_len(n) or not D.is_contiguous():
        raise ValueError("out must be a contiguous FP32 tensor of edm_tiled_len(n) elements")
    s = torch.zeros(4, dtype=torch.int64, device=X.device) if stats else None
    if ws is None and (p != 0 or stats):
        ws = _ws(workspace_bytes(1, n, d, p, map), X.device)
    _check(lib().smx_edm_tiled(_dev(X, "X"), n, d, ldx, _map(map), p, _ptr(D), _ptr(ws),
                               0 if ws is None else ws.numel(), _ptr(s), _stream()))
    return (D, s) if stats else D


# ---------------------------------------------------------------- triplets
def _xarg(X: torch.Tensor):
    if X.dtype != torch.float32 or X.dim() != 2 or X.shape[1] < 3 or X.stride(1) != 1:
        raise ValueError("X must be a row-major FP32 [n, >=3] matrix")
    return _dev(X, "X"), X.shape[0], (X.stride(0) if X.shape[0] > 0 else 3)


def triplet_energy(X: torch.Tensor, pot: Pot = Pot(), map="lambda", stats=False, ws=None):
    """Energy (FP64 [3]: total, AT, LJ); with stats=True also int64 [8] counters."""
    xp, n, ldx = _xarg(X)
    E = torch.empty(3, dtype=torch.float64, device=X.device)
    s = torch.zeros(8, dtype=torch.int64, device=X.device) if stats else None
    ws = ws if ws is not None else _ws(workspace_bytes(2, n, 3, 0, map), X.device)
    c = pot._c()
    _check(lib().smx_triplet_energy(xp, n, ldx, ctypes.byref(c), _map(map), _ptr(E), _ptr(ws), ws.numel(),
                                    _ptr(s), _stream()))
    return (E, s) if stats else E


def triplet_packed(X: torch.Tensor, nu: float = 1.0, map="lambda", stats=False, out=None, ws=None):
    """Per-triplet Axilrod-Teller energies, FP32 [n(n-1)(n-2)/6] in lexicographic
    i < j < k order; with stats=True also the int64 [4] counters."""
    xp, n, ldx = _xarg(X)
    m = n * (n - 1) * (n - 2) // 6
    E = out if out is not None else torch.empty(m, dtype=torch.float32, device=X.device)
    if E.dtype != torch.float32 or E.numel() < m or not E.is_contiguous() or E.device != X.device:
        raise ValueError("out must be a contiguous FP32 tensor of n(n-1)(n-2)/6 elements on X's device")
    s = torch.zeros(4, dtype=torch.int64, device=X.device) if stats else None
    if stats and ws is None:
        ws = _ws(workspace_bytes(0, n), X.device)
    _check(lib().smx_triplet_packed(xp, n, ldx, float(nu), _map(map), _ptr(E), _ptr(ws),
                                    0 if ws is None else ws.numel(), _ptr(s), _stream()))
    return (E, s) if stats else E


def triplet_tiled_len(n: int) -> int:
    """Floats of the tile-contiguous per-triplet layout: C(nb+2, 3) tiles of 32^3."""
    nb = -(-n // 32)
    return nb * (nb + 1) * (nb + 2) // 6 * 32768


def triplet_packed_tiled(X: torch.Tensor, nu: float = 1.0, map="lambda", stats=False, out=None, ws=None):
    """Per-triplet Axilrod-Teller energies in the tile-contiguous layout (FP32
    [C(nb+2,3) * 32768], see smx_triplet_packed_tiled); with stats=True also the
    int64 [4] counters."""
    xp, n, ldx = _xarg(X)
    m = triplet_tiled_len(n) if n >= 3 else 0
    E = out if out is not None else torch.empty(m, dtype=torch.float32, device=X.device)
    if E.dtype != torch.float32 or E.numel() < m or not E.is_contiguous() or E.device != X.device:
        raise ValueError("out must be a contiguous FP32 tensor of triplet_tiled_len(n) elements on X's device")
    s = torch.zeros(4, dtype=torch.int64, device=X.device) if stats else None
    if stats and ws is None:
        ws = _ws(workspace_bytes(0, n), X.device)
    _check(lib().smx_triplet_packed_tiled(xp, n, ldx, float(nu), _map(map), _ptr(E), _ptr(ws),
                                          0 if ws is None else ws.numel(), _ptr(s), _stream()))
    return (E, s) if stats else E


def simplex_decode(m: int, nb: int, map="lambda", ws=None, out=None):
    """Decode every logical block id of map `map` over the m-simplex of nb tiles
    per dimension, one per lane; int64 [4] stats (see smx_simplex_decode)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    st = out if out is not None else torch.zeros(4, dtype=torch.int64, device=dev)
    if ws is None:
        ws = _ws(workspace_bytes(0, 1), dev)
    _check(lib().smx_simplex_decode(m, nb, _map(map), _ptr(st), _ptr(ws), ws.numel(), _stream()))
    return st


def life_len(n: int) -> int:
    """Bytes of the tile-contiguous cell layout of the 2-simplex: nb(nb+1)/2 tiles of 64 x 64."""
    nb = -(-n // 64)
    return nb * (nb + 1) // 2 * 4096


def simplex_life(S: torch.Tensor, n: int, map="lambda", stats=False, out=None, ws=None):
    """One generation of Life on the 2-simplex of cells; S and the result are
    uint8 [life_len(n)] in the tile-contiguous layout (see smx_simplex_life)."""
    if S.dtype != torch.uint8 or not S.is_contiguous() or S.numel() < life_len(n):
        raise ValueError("S must be a contiguous uint8 tensor of life_len(n) bytes")
    D = out if out is not None else torch.empty(life_len(n), dtype=torch.uint8, device=S.device)
    s = torch.zeros(4, dtype=torch.int64, device=S.device) if stats else None
    if stats and ws is None:
        ws = _ws(workspace_bytes(0, n), S.device)
    _check(lib().smx_simplex_life(_dev(S, "S"), _ptr(D), n, _map(map), _ptr(s), _ptr(ws),
                                  0 if ws is None else ws.numel(), _stream()))
    return (D, s) if stats else D


def quad_contacts(X: torch.Tensor, rc: float, map="lambda", stats=False, out=None, ws=None):
    """Number of quadruplets i < j < k < l with all six pairs in contact (FP32
    squared distance below fl(rc^2)): int64 [1] on X's device; with stats=True
    also the int64 [4] counters."""
    xp, n, ldx = _xarg(X)
    c = out if out is not None else torch.empty(1, dtype=torch.int64, device=X.device)
    if c.dtype != torch.int64 or c.numel() < 1 or c.device != X.device:
        raise ValueError("out must be an int64 tensor on X's device")
    s = torch.zeros(4, dtype=torch.int64, device=X.device) if stats else None
    ws = ws if ws is not None else _ws(workspace_bytes(3, n), X.device)
    _check(lib().smx_quad_contacts(xp, n, ldx, float(rc), _map(map), _ptr(c), _ptr(ws), ws.numel(), _ptr(s),
                                   _stream()))
    return (c, s) if stats else c


def triplet_energy_grad(X: torch.Tensor, pot: Pot = Pot(), map="lambda", ws=None):
    """(E FP64 [3], dE/dX FP32 [n, 3]) in one pass."""
    xp, n, ldx = _xarg(X)
    E = torch.empty(3, dtype=torch.float64, device=X.device)
    G = torch.empty((n, 3), dtype=torch.float32, device=X.device)
    ws = ws if ws is not None else _ws(workspace_bytes(2, n, 3, 0, map), X.device)
    c = pot._c()
    _check(lib().smx_triplet_energy_grad(xp, n, ldx, ctypes.byref(c), _map(map), _ptr(E), _ptr(G), _ptr(ws),
                                         ws.numel(), _stream()))
    return E, G


# largest n of smx_triplet_energy_grad_noalloc (its static device scratch)
NOALLOC_MAX_N = 65536


def triplet_energy_grad_noalloc(X: torch.Tensor, pot: Pot = Pot(), map="lambda", E=None, G=None):
    """As triplet_energy_grad, through the entry point that takes its workspace
    from the library's static device array (n <= NOALLOC_MAX_N).  E (FP64 [3])
    and G (FP32 [n, 3]) may be passed in, preallocated; otherwise they are
    allocated here, on the Python side."""
    xp, n, ldx = _xarg(X)
    E = E if E is not None else torch.empty(3, dtype=torch.float64, device=X.device)
    G = G if G is not None else torch.empty((n, 3), dtype=torch.float32, device=X.device)
    if (E.dtype != torch.float64 or E.numel() < 3 or not E.is_contiguous() or G.dtype != torch.float32
            or G.numel() < 3 * n or not G.is_contiguous()):
        raise ValueError("E must be a contiguous FP64 [3] and G a contiguous FP32 [n, 3]")
    c = pot._c()
    _check(lib().smx_triplet_energy_grad_noalloc(xp, n, ldx, ctypes.byref(c), _map(map), _dev(E, "E"),
                                                 _dev(G, "G"), _stream()))
    return E, G


def triplet_energy_backward(X: torch.Tensor, gradE: torch.Tensor, pot: Pot = Pot(), map="lambda", ws=None):
    """gradE * dE/dX (FP32 [n, 3]); gradE is an FP64 GPU scalar."""
    xp, n, ldx = _xarg(X)
    g = gradE.to(torch.float64).reshape(1).contiguous()
    dX = torch.empty((n, 3), dtype=torch.float32, device=X.device)
    ws = ws if ws is not None else _ws(workspace_bytes(2, n, 3, 0, map), X.device)
    c = pot._c()
    _check(lib().smx_triplet_energy_backward(xp, n, ldx, ctypes.byref(c), _map(map), _dev(g, "gradE"),
                                             _ptr(dX), _ptr(ws), ws.numel(), _stream()))
    return dX


class TripletEnergy(torch.autograd.Function):
    """E(X) = Axilrod-Teller (+ Lennard-Jones) energy, FP64 0-d tensor.

    fused=True: the forward pass computes the energy and its gradient in one
    kernel pass and the backward pass scales the saved gradient;
    fused=False: the forward pass computes only the energy and the backward
    pass recomputes the pair terms (smx_triplet_energy_backward).
    Forces are -dE/dX.
    """

    @staticmethod
    def forward(ctx, X, pot: Pot = Pot(), map="lambda", fused: bool = True):
        ctx.pot, ctx.map, ctx.fused = pot, map, fused
        if fused and X.requires_grad:
            E, G = triplet_energy_grad(X.detach(), pot, map)
            ctx.save_for_backward(G)
        else:
            E = triplet_energy(X.detach(), pot, map)
            ctx.save_for_backward(X.detach())
        return E[0]

    @staticmethod
    def backward(ctx, gE):
        (saved,) = ctx.saved_tensors
        if ctx.fused:
            g = gE.detach().to(torch.float64).reshape(1).contiguous()
            dX = torch.empty_like(saved)
            _check(lib().smx_scale_grad(_dev(saved, "G"), saved.shape[0], _dev(g, "gradE"), _ptr(dX),
                                        _stream()))
        else:
            dX = triplet_energy_backward(saved, gE.detach(), ctx.pot, ctx.map)
        return dX, None, None, None


# ---------------------------------------------------------------- timing
def profile_enable(on: bool = True) -> None:
    _check(lib().smx_profile_enable(int(on)))


def profile_reset() -> None:
    _check(lib().smx_profile_reset())


def profile_read(kernel: str):
    """(total ms, launches) of a kernel since the last reset (synchronises)."""
    ms, cnt = _dbl(0.0), _i64(0)
    _check(lib().smx_profile_read(KERNELS[kernel], ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value
