"""ctypes binding of libgsf (include/gsf.h) for torch tensors on a ROCm device.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  Tensors must be contiguous and on the current HIP device.  Cubes
and filtered cubes are float32, float16 or bfloat16 (the storage type is
taken from the tensor); local mean and std are float32.  torch supplies
device memory and the stream
(``torch.cuda.current_stream().cuda_stream``).  When ``libgsf.so`` is missing
this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsf.so")

GSF_OK, GSF_ERR_INVALID_ARG, GSF_ERR_UNSUPPORTED, GSF_ERR_WORKSPACE, GSF_ERR_DEVICE, GSF_ERR_BUDGET = range(6)
GSF_F32, GSF_F16, GSF_BF16 = 0, 1, 2
GSF_MAX_RADIUS = 64
GSF_MAX_BOX = 4096


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64)]


class Filter(ctypes.Structure):
    _fields_ = [("sigma_xy", ctypes.c_double), ("sigma_z", ctypes.c_double),
                ("truncate", ctypes.c_double)]


class Box(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("bz", ctypes.c_int32)]


class Cube(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int), ("dims", Dims),
                ("halo", ctypes.c_int32 * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("merge_sweeps", ctypes.c_int32), ("merged_shape", ctypes.c_int32),
                ("sweep_blocks", ctypes.c_int32), ("yz_waves", ctypes.c_int32),
                ("pair_spectral", ctypes.c_int32), ("x_exits", ctypes.c_int32)]


class GsfError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"gsf status {status}: {detail}")
        self.status = status


_lib = None
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t
_ST = ctypes.c_int

# (name, restype, argtypes) for every symbol include/gsf.h declares.
SIGNATURES = [
    ("gsf_filter3d_workspace_size", _ST, [Dims, ctypes.POINTER(Filter), ctypes.POINTER(_SZ)]),
    ("gsf_filter3d", _ST, [_P, ctypes.c_int, Dims, ctypes.POINTER(Filter), _P, ctypes.c_int, _P,
                           _SZ, _P]),
    ("gsf_filter3d_weighted_workspace_size", _ST, [Dims, ctypes.POINTER(Filter),
                                                   ctypes.POINTER(_SZ)]),
    ("gsf_filter3d_weighted", _ST, [_P, _P, ctypes.c_int, Dims, ctypes.POINTER(Filter), _P, _P,
                                    _SZ, _P]),
    ("gsf_local_stats_workspace_size", _ST, [Dims, Box, ctypes.POINTER(_SZ)]),
    ("gsf_local_stats", _ST, [_P, ctypes.c_int, Dims, Box, _P, _P, _P, _SZ, _P]),
    ("gsf_threshold", _ST, [_P, ctypes.c_int, _P, _P, Dims, ctypes.c_double, _P, _P]),
    ("gsf_find_workspace_size", _ST, [ctypes.POINTER(Cube), ctypes.c_int32, ctypes.POINTER(Filter),
                                      ctypes.c_int32, Box, ctypes.POINTER(_SZ)]),
    ("gsf_find", _ST, [ctypes.POINTER(Cube), ctypes.c_int32, ctypes.POINTER(Filter), ctypes.c_int32,
                       Box, ctypes.c_double, ctypes.POINTER(_P), ctypes.POINTER(_P),
                       ctypes.POINTER(_P), ctypes.POINTER(_P), _P, _SZ, _P]),
    ("gsf_find_noalloc", _ST, [ctypes.POINTER(Cube), ctypes.c_int32, ctypes.POINTER(Filter),
                               ctypes.c_int32, Box, ctypes.c_double, ctypes.POINTER(_P),
                               ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P), _P]),
    ("gsf_init", _ST, []),
    ("gsf_size_class", ctypes.c_int32, [Dims]),
    ("gsf_tuning_set", _ST, [ctypes.c_int32, ctypes.c_int, ctypes.POINTER(Tuning)]),
    ("gsf_tuning_get", _ST, [ctypes.c_int32, ctypes.c_int, ctypes.POINTER(Tuning)]),
    ("gsf_tuning_reset", _ST, []),
    ("gsf_profile_enable", _ST, [ctypes.c_int]),
    ("gsf_profile_reset", _ST, []),
    ("gsf_profile_collect", ctypes.c_int32, []),
    ("gsf_profile_entry", _ST, [ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p),
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
    ("gsf_mask_words", ctypes.c_int64, [Dims]),
    ("gsf_status_string", ctypes.c_char_p, [_ST]),
    ("gsf_last_error", ctypes.c_char_p, []),
    ("gsf_version", ctypes.c_char_p, []),
]


def lib():
    """Open libgsf.so (built in-tree by ``build.build()``); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(st: int) -> None:
    if st != GSF_OK:
        raise GsfError(st, lib().gsf_last_error().decode())


def _dims(shape) -> Dims:
    nx, ny, nz = (int(s) for s in shape)
    return Dims(nx, ny, nz)


def _filter(f) -> Filter:
    if isinstance(f, Filter):
        return f
    t = float(f[2]) if len(f) > 2 else 3.0
    return Filter(float(f[0]), float(f[1]), t)


def _box(b) -> Box:
    if isinstance(b, Box):
        return b
    if isinstance(b, int):
        return Box(b, b, b)
    bx, by, bz = (int(v) for v in b)
    return Box(bx, by, bz)


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


_DTYPES = {torch.float32: GSF_F32, torch.float16: GSF_F16, torch.bfloat16: GSF_BF16}


def _cube(t: torch.Tensor, name: str, storage: bool = False) -> torch.Tensor:
    """Check a 3-D device tensor; `storage` cubes may also be float16/bfloat16."""
    if not isinstance(t, torch.Tensor) or t.dim() != 3:
        raise ValueError(f"{name} must be a 3-D tensor (nx, ny, nz)")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device")
    if t.dtype not in (_DTYPES if storage else (torch.float32,)):
        raise ValueError(f"{name} must be " + ("float32, float16 or bfloat16" if storage else "float32"))
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def gsf_dtype(t: torch.Tensor) -> int:
    return _DTYPES[t.dtype]


def mask_words(shape) -> int:
    nx, ny, nz = (int(s) for s in shape)
    return nx * ny * ((nz + 63) // 64)


def empty_mask(shape, device) -> torch.Tensor:
    nx, ny, nz = (int(s) for s in shape)
    return torch.empty((nx, ny, (nz + 63) // 64), dtype=torch.int64, device=device)


def unpack_mask(words, shape) -> np.ndarray:
    """Packed mask words (nx, ny, W) -> bool array (nx, ny, nz)."""
    nx, ny, nz = (int(s) for s in shape)
    w = words.detach().cpu().numpy() if isinstance(words, torch.Tensor) else np.asarray(words)
    w = np.ascontiguousarray(w.reshape(nx, ny, -1)).view(np.uint8)
    bits = np.unpackbits(w, axis=2, bitorder="little")
    return bits[:, :, :nz].astype(bool)


def version() -> str:
    return lib().gsf_version().decode()


def filter3d_workspace_size(shape, f) -> int:
    n = _SZ(0)
    _check(lib().gsf_filter3d_workspace_size(_dims(shape), ctypes.byref(_filter(f)), ctypes.byref(n)))
    return int(n.value)


def filter3d(cube: torch.Tensor, f, out: torch.Tensor | None = None,
             ws: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. 2: the cube filtered by one (sigma_xy, sigma_z[, truncate]) Gaussian,
    stored in the cube's dtype."""
    cube = _cube(cube, "cube", storage=True)
    if out is None:
        out = torch.empty_like(cube)
    _cube(out, "out", storage=True)
    need = filter3d_workspace_size(cube.shape, f)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=cube.device)
    _check(lib().gsf_filter3d(cube.data_ptr(), gsf_dtype(cube), _dims(cube.shape),
                              ctypes.byref(_filter(f)), out.data_ptr(), gsf_dtype(out),
                              ws.data_ptr(), ws.numel(), _stream(cube.device)))
    return out


def filter3d_weighted(cube: torch.Tensor, w: torch.Tensor, f, out: torch.Tensor | None = None,
                      ws: torch.Tensor | None = None) -> torch.Tensor:
    """Eq. 1: the weighted convolution sum(d w f) / sum(w f) (float32)."""
    cube, w = _cube(cube, "cube"), _cube(w, "w")
    if w.shape != cube.shape:
        raise ValueError("weights must have the cube's shape")
    if out is None:
        out = torch.empty_like(cube)
    _cube(out, "out")
    n = _SZ(0)
    _check(lib().gsf_filter3d_weighted_workspace_size(_dims(cube.shape), ctypes.byref(_filter(f)),
                                                      ctypes.byref(n)))
    if ws is None:
        ws = torch.empty(int(n.value), dtype=torch.uint8, device=cube.device)
    _check(lib().gsf_filter3d_weighted(cube.data_ptr(), w.data_ptr(), GSF_F32, _dims(cube.shape),
                                       ctypes.byref(_filter(f)), out.data_ptr(), ws.data_ptr(),
                                       ws.numel(), _stream(cube.device)))
    return out


def local_stats_workspace_size(shape, box) -> int:
    n = _SZ(0)
    _check(lib().gsf_local_stats_workspace_size(_dims(shape), _box(box), ctypes.byref(n)))
    return int(n.value)


def local_stats(F: torch.Tensor, box, want_mean: bool = True, want_std: bool = True,
                ws: torch.Tensor | None = None):
    """§3.3: per-voxel local mean and std of F over the clipped box window
    (float32 outputs for any storage type of F)."""
    F = _cube(F, "F", storage=True)
    mean = torch.empty(F.shape, dtype=torch.float32, device=F.device) if want_mean else None
    std = torch.empty(F.shape, dtype=torch.float32, device=F.device) if want_std else None
    need = local_stats_workspace_size(F.shape, box)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=F.device)
    _check(lib().gsf_local_stats(F.data_ptr(), gsf_dtype(F), _dims(F.shape), _box(box),
                                 mean.data_ptr() if mean is not None else None,
                                 std.data_ptr() if std is not None else None,
                                 ws.data_ptr(), ws.numel(), _stream(F.device)))
    return mean, std


def threshold(F: torch.Tensor, mean: torch.Tensor, std: torch.Tensor, k: float,
              mask: torch.Tensor | None = None) -> torch.Tensor:
    """Selection F > mean + k*std, packed along z into int64 words (nx, ny, W)."""
    F, mean, std = _cube(F, "F", storage=True), _cube(mean, "mean"), _cube(std, "std")
    if mask is None:
        mask = empty_mask(F.shape, F.device)
    _check(lib().gsf_threshold(F.data_ptr(), gsf_dtype(F), mean.data_ptr(), std.data_ptr(),
                               _dims(F.shape), float(k), mask.data_ptr(), _stream(F.device)))
    return mask


def _halos(halos, n):
    """None, one (hx, hy, hz) for every cube, or one per cube."""
    if halos is None:
        return [(0, 0, 0)] * n
    if len(halos) == 3 and all(isinstance(v, (int, np.integer)) for v in halos):
        return [tuple(int(v) for v in halos)] * n
    if len(halos) != n:
        raise ValueError("halos: one (hx, hy, hz) per cube")
    return [tuple(int(v) for v in h) for h in halos]


def core_shape(shape, halo) -> tuple:
    return tuple(int(s) - 2 * int(h) for s, h in zip(shape, halo))


def _cube_structs(cubes, halos=None):
    hs = _halos(halos, len(cubes))
    arr = (Cube * len(cubes))()
    for i, c in enumerate(cubes):
        c = _cube(c, f"cubes[{i}]", storage=True)
        arr[i].data = c.data_ptr()
        arr[i].dtype = gsf_dtype(c)
        arr[i].dims = _dims(c.shape)
        arr[i].halo[0], arr[i].halo[1], arr[i].halo[2] = hs[i]
    return arr


def find_workspace_size(cubes, filters, box, halos=None) -> int:
    carr = _cube_structs(cubes, halos)
    farr = (Filter * len(filters))(*[_filter(f) for f in filters])
    n = _SZ(0)
    _check(lib().gsf_find_workspace_size(carr, len(cubes), farr, len(filters), _box(box),
                                         ctypes.byref(n)))
    return int(n.value)


class FindPlan:
    """Pre-marshalled gsf_find call over fixed cubes and output buffers, so a
    timed loop only re-issues the C call.  With ``noalloc`` the plan calls
    gsf_find_noalloc, which works in the library's own scratch (no workspace
    tensor is allocated)."""

    def __init__(self, cubes, filters, box, k: float, want_F: bool = False,
                 want_stats: bool = False, halos=None, noalloc: bool = False):
        self.cubes = [_cube(c, f"cubes[{i}]", storage=True) for i, c in enumerate(cubes)]
        self.filters = [tuple(f) for f in filters]
        self.halos = _halos(halos, len(self.cubes))
        self.cores = [core_shape(c.shape, h) for c, h in zip(self.cubes, self.halos)]
        dev = self.cubes[0].device
        nc, nf = len(self.cubes), len(self.filters)
        self.masks = [[empty_mask(s, dev) for _ in range(nf)] for s in self.cores]
        f32 = dict(dtype=torch.float32, device=dev)
        self.F = ([[torch.empty(s, dtype=c.dtype, device=dev) for _ in range(nf)]
                   for c, s in zip(self.cubes, self.cores)] if want_F else None)
        self.mean = ([[torch.empty(s, **f32) for _ in range(nf)] for s in self.cores]
                     if want_stats else None)
        self.std = ([[torch.empty(s, **f32) for _ in range(nf)] for s in self.cores]
                    if want_stats else None)
        self._carr = _cube_structs(self.cubes, self.halos)
        self._farr = (Filter * nf)(*[_filter(f) for f in self.filters])
        self._box = _box(box)
        self.k = float(k)

        def ptrs(grid):
            if grid is None:
                return None
            return (_P * (nc * nf))(*[grid[c][j].data_ptr() for c in range(nc) for j in range(nf)])

        self._m = ptrs(self.masks)
        self._F = ptrs(self.F)
        self._mu = ptrs(self.mean)
        self._sd = ptrs(self.std)
        self.noalloc = bool(noalloc)
        if self.noalloc:
            self.ws = None
        else:
            need = find_workspace_size(self.cubes, self.filters, box, self.halos)
            self.ws = torch.empty(need, dtype=torch.uint8, device=dev)
        self.device = dev

    def run(self, stream: int | None = None) -> None:
        s = _stream(self.device) if stream is None else stream
        if self.noalloc:
            _check(lib().gsf_find_noalloc(self._carr, len(self.cubes), self._farr,
                                          len(self.filters), self._box, self.k, self._m, self._F,
                                          self._mu, self._sd, s))
            return
        _check(lib().gsf_find(self._carr, len(self.cubes), self._farr, len(self.filters), self._box,
                              self.k, self._m, self._F, self._mu, self._sd, self.ws.data_ptr(),
                              self.ws.numel(), s))


def init() -> None:
    """gsf_init: the library's per-device streams, made outside any graph
    capture."""
    _check(lib().gsf_init())


def size_class(core_shape) -> int:
    """floor(log2(voxels)) of a core: the key of the library's tuning table."""
    return int(lib().gsf_size_class(_dims(core_shape)))


def tuning_set(cfg: dict, size_class: int = -1, dtype=torch.float32) -> None:
    """Install a tuning entry (keys of gsf_tuning) for a size class (-1: all)."""
    t = Tuning(int(cfg.get("merge_sweeps", 1)), int(cfg.get("merged_shape", 0)),
               int(cfg.get("sweep_blocks", 512)), int(cfg.get("yz_waves", 0)),
               int(cfg.get("pair_spectral", 1)), int(cfg.get("x_exits", 1)))
    _check(lib().gsf_tuning_set(int(size_class), _DTYPES[dtype], ctypes.byref(t)))


def tuning_get(size_class: int, dtype=torch.float32) -> dict:
    t = Tuning()
    _check(lib().gsf_tuning_get(int(size_class), _DTYPES[dtype], ctypes.byref(t)))
    return {k: int(getattr(t, k)) for k, _ in Tuning._fields_}


def tuning_reset() -> None:
    _check(lib().gsf_tuning_reset())


def profile_enable(on: bool = True) -> None:
    """Bracket every library kernel with hipEvents on its stream (see gsf.h)."""
    _check(lib().gsf_profile_enable(1 if on else 0))


def profile_reset() -> None:
    _check(lib().gsf_profile_reset())


def profile_collect() -> dict:
    """{kernel name: (launches, total ms)} over the launches recorded so far."""
    L = lib()
    n = L.gsf_profile_collect()
    if n < 0:
        raise GsfError(GSF_ERR_DEVICE, "hipEvent query failed")
    out = {}
    for i in range(n):
        name = ctypes.c_char_p()
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(L.gsf_profile_entry(i, ctypes.byref(name), ctypes.byref(cnt), ctypes.byref(ms)))
        out[name.value.decode()] = (int(cnt.value), float(ms.value))
    return out


NOALLOC_SCRATCH_BYTES = 256 << 20   # GSF_NOALLOC_SCRATCH_BYTES


def find_noalloc(cubes, filters, box, k: float, want_F: bool = False, want_stats: bool = False,
                 halos=None) -> dict:
    """``find`` through gsf_find_noalloc: the library's own scratch instead of
    a workspace (cubes run one after another on the current stream).  Output
    tensors are still allocated here, by torch, for the caller."""
    if isinstance(cubes, torch.Tensor):
        cubes = [cubes]
    plan = FindPlan(cubes, filters, box, k, want_F=want_F, want_stats=want_stats, halos=halos,
                    noalloc=True)
    plan.run()
    return {"mask": plan.masks, "F": plan.F, "mean": plan.mean, "std": plan.std}


def find(cubes, filters, box, k: float, want_F: bool = False, want_stats: bool = False,
         halos=None) -> dict:
    """The whole path over a batch of cubes: for each cube and filter, Eq. 2,
    local mean/std (§3.3) and the mask F > mean + k*std.  With halos, each
    cube's outputs cover its core (see gsf_cube in gsf.h).

    Returns {'mask': [[words]], 'F': [[...]] | None, 'mean': ..., 'std': ...}
    indexed [cube][filter]."""
    if isinstance(cubes, torch.Tensor):
        cubes = [cubes]
    plan = FindPlan(cubes, filters, box, k, want_F=want_F, want_stats=want_stats, halos=halos)
    plan.run()
    return {"mask": plan.masks, "F": plan.F, "mean": plan.mean, "std": plan.std}
