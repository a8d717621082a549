"""ctypes binding of libpmmm.so (the C ABI in include/pmmm.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the far-field pipeline runs in the HIP
kernels of the library.  Importing this module raises if the library has
not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmmm.so")

PMMM_OK, PMMM_EINVAL, PMMM_ENOMEM, PMMM_EHIP, PMMM_EDOMAIN, PMMM_EUNSUPPORTED = range(6)
PMMM_OPEN, PMMM_PERIODIC = 0, 1
PMMM_F32, PMMM_F64, PMMM_BF16X3 = 0, 1, 2
PMMM_MESH_M, PMMM_MESH_L, PMMM_MESH_GREEN = 0, 1, 2
PMMM_PMAX = 10
PMMM_NOALLOC_MAX_N = 1 << 18
PMMM_COEF_EXP_INVALID = -(2 ** 31)
PMMM_COEF_AUTO_EXP = 1

#: every symbol include/pmmm.h declares
EXPORTS = [
    "pmmm_plan_create", "pmmm_plan_destroy", "pmmm_workspace_bytes",
    "pmmm_far_f32", "pmmm_far_f64", "pmmm_far_multi_f32", "pmmm_far_f32_noalloc",
    "pmmm_near_f32", "pmmm_near_f64", "pmmm_total_f32", "pmmm_total_f64",
    "pmmm_plan_sync_status", "pmmm_plan_mesh_bytes", "pmmm_plan_copy_mesh",
    "pmmm_plan_set_profiling", "pmmm_plan_read_profile", "pmmm_plan_set_graphs",
    "pmmm_plan_autotune", "pmmm_plan_get_tuning", "pmmm_plan_set_tuning",
    "pmmm_batch_create", "pmmm_batch_destroy", "pmmm_batch_far_f32", "pmmm_batch_classes",
    "pmmm_batch_set_graphs", "pmmm_batch_sync_status",
    "pmmm_hier_create", "pmmm_hier_destroy", "pmmm_hier_far_f32", "pmmm_hier_total_f32",
    "pmmm_hier_sync_status", "pmmm_hier_set_profiling", "pmmm_hier_read_profile",
    "pmmm_coef_record_words", "pmmm_coef_pack_f32", "pmmm_coef_unpack_f32",
    "pmmm_coef_compose_f32", "pmmm_coef_split_f32",
    "pmmm_error_string", "pmmm_last_error",
]

STAGES = ["bin", "p2m", "fft_fwd", "column", "fft_inv", "l2p", "near"]


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("box", ctypes.c_double * 3),
        ("p", ctypes.c_int), ("cutoff", ctypes.c_int), ("boundary", ctypes.c_int),
        ("precision", ctypes.c_int), ("alpha", ctypes.c_double), ("images", ctypes.c_int),
        ("n_max", ctypes.c_int64),
    ]


COLUMN_KERNELS = {"default": 0, "tile": 1, "stream1": 2, "stream2": 3, "stream4": 4}


class Tuning(ctypes.Structure):
    _fields_ = [("column_kernel", ctypes.c_int), ("column_width", ctypes.c_int),
                ("p2m_lanes", ctypes.c_int)]


class PMMMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load():
    """Load libpmmm.so and declare the prototypes (raises if missing).

    torch is imported first: libpmmm.so needs libamdhip64.so.7, and when
    torch's copy of the HIP runtime (same soname) is already mapped the
    dynamic linker binds the library to it, so torch's streams and device
    pointers and the library's calls share one HIP (and one HSA) runtime.
    Loaded the other way round, the process would map two of each."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                          "(or python paper_1409_5981_amd/build.py) first")
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, ci, cz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
    L.pmmm_plan_create.argtypes = [ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.pmmm_plan_create.restype = ci
    L.pmmm_plan_destroy.argtypes = [vp]
    L.pmmm_plan_destroy.restype = None
    L.pmmm_workspace_bytes.argtypes = [ctypes.POINTER(Params), i64]
    L.pmmm_workspace_bytes.restype = cz
    for name in ("pmmm_far_f32", "pmmm_far_f64", "pmmm_far_f32_noalloc"):
        f = getattr(L, name)
        f.argtypes = [vp, i64] + [vp] * 8 + [vp]
        f.restype = ci
    L.pmmm_far_multi_f32.argtypes = [vp, i64, vp, vp, vp, ci] + [vp] * 5 + [vp]
    L.pmmm_far_multi_f32.restype = ci
    for name in ("pmmm_near_f32", "pmmm_near_f64"):
        f = getattr(L, name)
        f.argtypes = [vp, i64] + [vp] * 8 + [ci, vp]
        f.restype = ci
    for name in ("pmmm_total_f32", "pmmm_total_f64"):
        f = getattr(L, name)
        f.argtypes = [vp, i64] + [vp] * 8 + [vp]
        f.restype = ci
    L.pmmm_plan_sync_status.argtypes = [vp]
    L.pmmm_plan_sync_status.restype = ci
    L.pmmm_plan_mesh_bytes.argtypes = [vp, ci]
    L.pmmm_plan_mesh_bytes.restype = cz
    L.pmmm_plan_copy_mesh.argtypes = [vp, ci, vp, cz]
    L.pmmm_plan_copy_mesh.restype = ci
    L.pmmm_plan_set_graphs.argtypes = [vp, ci]
    L.pmmm_plan_set_graphs.restype = ci
    L.pmmm_plan_set_profiling.argtypes = [vp, ctypes.c_uint]
    L.pmmm_plan_set_profiling.restype = ci
    L.pmmm_plan_read_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ci]
    L.pmmm_plan_read_profile.restype = ci
    L.pmmm_plan_autotune.argtypes = [vp, i64] + [vp] * 8 + [vp]
    L.pmmm_plan_autotune.restype = ci
    L.pmmm_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.pmmm_plan_get_tuning.restype = ci
    L.pmmm_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.pmmm_plan_set_tuning.restype = ci
    L.pmmm_batch_create.argtypes = [ci, ctypes.POINTER(Params), vp, ctypes.POINTER(vp)]
    L.pmmm_batch_create.restype = ci
    L.pmmm_batch_destroy.argtypes = [vp]
    L.pmmm_batch_destroy.restype = None
    L.pmmm_batch_far_f32.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)] + [vp] * 8 + [vp]
    L.pmmm_batch_far_f32.restype = ci
    L.pmmm_batch_classes.argtypes = [vp]
    L.pmmm_batch_classes.restype = ci
    L.pmmm_batch_set_graphs.argtypes = [vp, ci]
    L.pmmm_batch_set_graphs.restype = ci
    L.pmmm_batch_sync_status.argtypes = [vp]
    L.pmmm_batch_sync_status.restype = ci
    L.pmmm_hier_create.argtypes = [ctypes.POINTER(Params), ci, vp, ctypes.POINTER(vp)]
    L.pmmm_hier_create.restype = ci
    L.pmmm_hier_destroy.argtypes = [vp]
    L.pmmm_hier_destroy.restype = None
    for name in ("pmmm_hier_far_f32", "pmmm_hier_total_f32"):
        f = getattr(L, name)
        f.argtypes = [vp, i64] + [vp] * 8 + [vp]
        f.restype = ci
    L.pmmm_hier_sync_status.argtypes = [vp]
    L.pmmm_hier_sync_status.restype = ci
    L.pmmm_hier_set_profiling.argtypes = [vp, ctypes.c_uint]
    L.pmmm_hier_set_profiling.restype = ci
    L.pmmm_hier_read_profile.argtypes = [vp, ci, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ci]
    L.pmmm_hier_read_profile.restype = ci
    L.pmmm_coef_record_words.argtypes = [ci]
    L.pmmm_coef_record_words.restype = ci
    L.pmmm_coef_pack_f32.argtypes = [ci, i64, vp, vp, vp, ctypes.c_uint, vp]
    L.pmmm_coef_pack_f32.restype = ci
    L.pmmm_coef_unpack_f32.argtypes = [ci, i64, vp, vp, vp, vp]
    L.pmmm_coef_unpack_f32.restype = ci
    L.pmmm_coef_compose_f32.argtypes = [ci, i64, vp, vp, vp, vp]
    L.pmmm_coef_compose_f32.restype = ci
    L.pmmm_coef_split_f32.argtypes = [ci, i64, vp, vp, vp, vp]
    L.pmmm_coef_split_f32.restype = ci
    L.pmmm_error_string.argtypes = [ci]
    L.pmmm_error_string.restype = ctypes.c_char_p
    L.pmmm_last_error.argtypes = []
    L.pmmm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check_buffers(ts, dtype, numel, shape=None, what="tensors", device=None):
    """Validate caller buffers before any C call: every tensor must hold
    exactly `numel` elements (and have `shape` when given), be of `dtype`,
    contiguous, on a GPU, and all on one device.  A short output tensor would
    otherwise let the kernels write past its end.  Raises ValueError."""
    ts = tuple(ts)
    if any(t is None for t in ts):
        raise ValueError(f"{what}: None given")
    for t in ts:
        if t.numel() != numel or (shape is not None and tuple(t.shape) != tuple(shape)):
            want = tuple(shape) if shape is not None else f"{numel} elements"
            raise ValueError(f"{what}: expected {want}, got shape {tuple(t.shape)}")
    for t in ts:
        if t.dtype != dtype:
            raise ValueError(f"{what}: expected dtype {dtype}, got {t.dtype}")
    for t in ts:
        if not t.is_contiguous():
            raise ValueError(f"{what}: tensors must be contiguous")
    dev = device
    for t in ts:
        if not t.is_cuda:
            raise ValueError(f"{what}: tensors must be GPU (device) tensors")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{what}: all tensors must be on one device ({dev} and {t.device})")


def _check(rc: int):
    if rc != PMMM_OK:
        L = load()
        raise PMMMError(rc, f"{L.pmmm_error_string(rc).decode()}: {L.pmmm_last_error().decode()}")


def make_params(n: int, p: int, boundary: str, box: float = 1.0, cutoff: int = 2,
                precision: str = "f32", alpha: float = 0.0, images: int = 0,
                n_max: int = 0, shape=None) -> Params:
    """n cells per axis and box edge `box`, or with shape = (nx, ny, nz)
    (open boundary) nx = n cells along the x edge `box` and cubic cells."""
    prm = Params()
    dims = (int(n),) * 3 if shape is None else tuple(int(v) for v in shape)
    if dims[0] != int(n):
        raise ValueError("shape[0] must equal n")
    prm.nx, prm.ny, prm.nz = dims
    for a in range(3):
        prm.box[a] = float(box) * dims[a] / dims[0]
    prm.p = int(p)
    prm.cutoff = int(cutoff)
    prm.boundary = PMMM_OPEN if boundary == "open" else PMMM_PERIODIC
    prm.precision = {"f32": PMMM_F32, "f64": PMMM_F64, "bf16x3": PMMM_BF16X3}[precision]
    prm.alpha = float(alpha)
    prm.images = int(images)
    prm.n_max = int(n_max)
    return prm


def workspace_bytes(prm: Params, n_max: int) -> int:
    return int(load().pmmm_workspace_bytes(ctypes.byref(prm), int(n_max)))


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A PMMM far-field plan (transfer kernel built on creation)."""

    def __init__(self, n: int, p: int, boundary: str, box: float = 1.0, cutoff: int = 2,
                 precision: str = "f32", alpha: float = 0.0, images: int = 0, n_max: int = 0,
                 stream=None, shape=None):
        L = load()
        self.params = make_params(n, p, boundary, box, cutoff, precision, alpha, images, n_max,
                                  shape)
        self.n, self.p, self.boundary, self.box = n, p, boundary, box
        self.shape = (n, n, n) if shape is None else tuple(shape)
        self.cutoff, self.precision = cutoff, precision
        # cells per axis of the computed mesh: open meshes sit in the
        # smallest power-of-two cube (at least 4) that holds them
        nc = n
        if boundary == "open":
            nc = 4
            while nc < max(self.shape):
                nc *= 2
        self.n_mesh = nc
        self.nf = 2 * nc if boundary == "open" else nc
        self._h = ctypes.c_void_p()
        _check(L.pmmm_plan_create(ctypes.byref(self.params), _stream_handle(stream),
                                  ctypes.byref(self._h)))

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == "f64" else torch.float32

    def close(self):
        if self._h:
            load().pmmm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _inputs(self, x, y, z, q):
        """Validate the particle arrays (same length, plan dtype, contiguous,
        one GPU device); returns n."""
        n = x.numel()
        check_buffers((x, y, z, q), self.dtype, n, what="x, y, z, q")
        return n

    def _outputs(self, out, n, device, shape=None, zero=False):
        import torch
        shp = tuple(shape) if shape is not None else (n,)
        if out is None:
            mk = torch.zeros if zero else torch.empty
            return tuple(mk(shp, dtype=self.dtype, device=device) for _ in range(4))
        if len(out) != 4:
            raise ValueError("out must hold four tensors (phi, gx, gy, gz)")
        numel = 1
        for d in shp:
            numel *= d
        check_buffers(out, self.dtype, numel, shape=shape, what="out", device=device)
        return tuple(out)

    def far(self, x, y, z, q, out=None, stream=None):
        """Far-field Phi and grad Phi (input order) as four device tensors."""
        n = self._inputs(x, y, z, q)
        out = self._outputs(out, n, x.device)
        fn = load().pmmm_far_f64 if self.precision == "f64" else load().pmmm_far_f32
        _check(fn(self._h, n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                  *[o.data_ptr() for o in out], _stream_handle(stream)))
        return out

    def far_noalloc(self, x, y, z, q, out, stream=None):
        """pmmm_far_f32_noalloc: the FP32 far field with the library's static
        per-particle scratch (n <= PMMM_NOALLOC_MAX_N; outputs required)."""
        n = self._inputs(x, y, z, q)
        out = self._outputs(out, n, x.device)
        _check(load().pmmm_far_f32_noalloc(self._h, n, x.data_ptr(), y.data_ptr(), z.data_ptr(),
                                           q.data_ptr(), *[o.data_ptr() for o in out],
                                           _stream_handle(stream)))
        return out

    def near(self, x, y, z, q, out=None, accumulate=False, stream=None):
        """Near field (direct sums over the (2c+1)^3 cells around each
        particle's cell); accumulate adds into `out`."""
        n = self._inputs(x, y, z, q)
        if accumulate and out is None:
            raise ValueError("accumulate needs the output tensors")
        out = self._outputs(out, n, x.device)
        fn = load().pmmm_near_f64 if self.precision == "f64" else load().pmmm_near_f32
        _check(fn(self._h, n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                  *[o.data_ptr() for o in out], int(bool(accumulate)), _stream_handle(stream)))
        return out

    def total(self, x, y, z, q, out=None, stream=None):
        """Total Phi and grad Phi = far field + near field, one binning."""
        n = self._inputs(x, y, z, q)
        out = self._outputs(out, n, x.device)
        fn = load().pmmm_total_f64 if self.precision == "f64" else load().pmmm_total_f32
        _check(fn(self._h, n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                  *[o.data_ptr() for o in out], _stream_handle(stream)))
        return out

    def far_multi(self, x, y, z, q, out=None, stream=None):
        """Far field of several charge sets on the same positions.  q is
        [n, nsets] (set index fastest); returns Phi, gx, gy, gz as [n, nsets]
        device tensors in input order."""
        n = x.numel()
        check_buffers((x, y, z), self.dtype, n, what="x, y, z")
        if q.dim() != 2 or q.shape[0] != n:
            raise ValueError("q must have shape [n, nsets]")
        nsets = int(q.shape[1])
        check_buffers((q,), self.dtype, n * nsets, shape=(n, nsets), what="q",
                      device=x.device)
        out = self._outputs(out, n, x.device, shape=(n, nsets))
        _check(load().pmmm_far_multi_f32(self._h, n, x.data_ptr(), y.data_ptr(), z.data_ptr(),
                                         nsets, q.data_ptr(), *[o.data_ptr() for o in out],
                                         _stream_handle(stream)))
        return out

    def autotune(self, x, y, z, q, out=None, stream=None):
        """Time the candidate launch shapes on these particles and keep the
        fastest; returns the kept shapes as a dict (see tuning())."""
        n = self._inputs(x, y, z, q)
        out = self._outputs(out, n, x.device)
        _check(load().pmmm_plan_autotune(self._h, n, x.data_ptr(), y.data_ptr(), z.data_ptr(),
                                         q.data_ptr(), *[o.data_ptr() for o in out],
                                         _stream_handle(stream)))
        return self.tuning()

    def tuning(self):
        """{"column_kernel": name, "column_width": w, "p2m_lanes": g} (0 / "default":
        the library's choice)."""
        t = Tuning()
        _check(load().pmmm_plan_get_tuning(self._h, ctypes.byref(t)))
        names = {v: k for k, v in COLUMN_KERNELS.items()}
        return {"column_kernel": names.get(t.column_kernel, str(t.column_kernel)),
                "column_width": t.column_width, "p2m_lanes": t.p2m_lanes}

    def set_tuning(self, column_kernel="default", column_width=0, p2m_lanes=0):
        t = Tuning(COLUMN_KERNELS[column_kernel], int(column_width), int(p2m_lanes))
        _check(load().pmmm_plan_set_tuning(self._h, ctypes.byref(t)))

    def set_graphs(self, enable: bool):
        """Replay repeated calls as a HIP graph (pmmm_plan_set_graphs)."""
        _check(load().pmmm_plan_set_graphs(self._h, 1 if enable else 0))

    def set_profiling(self, stages):
        """Enable HIP-event timing for the named stages (see STAGES)."""
        mask = 0
        for st in stages:
            mask |= 1 << STAGES.index(st)
        _check(load().pmmm_plan_set_profiling(self._h, mask))

    def read_profile(self, reset=True):
        """{stage: (total ms, launches)} accumulated since the last reset."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(load().pmmm_plan_read_profile(self._h, ms, cnt, int(bool(reset))))
        return {st: (ms[i], cnt[i]) for i, st in enumerate(STAGES)}

    def sync_status(self):
        _check(load().pmmm_plan_sync_status(self._h))

    def mesh(self, which: int) -> np.ndarray:
        """Copy an internal mesh (PMMM_MESH_M / _L / _GREEN) to a numpy array."""
        L = load()
        nbytes = int(L.pmmm_plan_mesh_bytes(self._h, which))
        dt = np.float64 if self.precision == "f64" else np.float32
        buf = np.empty(nbytes // np.dtype(dt).itemsize, dtype=dt)
        _check(L.pmmm_plan_copy_mesh(self._h, which, buf.ctypes.data_as(ctypes.c_void_p), nbytes))
        P, n, nf = (self.p + 1) ** 2, self.n_mesh, self.nf
        if which in (PMMM_MESH_M, PMMM_MESH_L):
            return buf.reshape(P, n, n, n)
        Q = (2 * self.p + 1) ** 2
        nh = nf // 2 + 1
        nhp = (nh + 3) & ~3
        return buf.reshape(nh, nh, Q, nhp)[..., :nh]


class Batch:
    """Independent systems in one call (pmmm_batch_*).  `systems` is a list
    of dicts with the Plan arguments (n, p, boundary, box, cutoff, alpha,
    images, shape); every system runs the FP32 pipeline."""

    def __init__(self, systems, stream=None):
        L = load()
        self.nsys = len(systems)
        arr = (Params * self.nsys)()
        for i, sy in enumerate(systems):
            arr[i] = make_params(sy["n"], sy["p"], sy.get("boundary", "periodic"),
                                 sy.get("box", 1.0), sy.get("cutoff", 2), "f32",
                                 sy.get("alpha", 0.0), sy.get("images", 0),
                                 shape=sy.get("shape"))
        self._params = arr
        self._h = ctypes.c_void_p()
        _check(L.pmmm_batch_create(self.nsys, arr, _stream_handle(stream), ctypes.byref(self._h)))

    @property
    def classes(self) -> int:
        return int(load().pmmm_batch_classes(self._h))

    def set_graphs(self, enable: bool):
        _check(load().pmmm_batch_set_graphs(self._h, int(bool(enable))))

    def close(self):
        if self._h:
            load().pmmm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def far(self, offsets, x, y, z, q, out=None, stream=None):
        """offsets: nsys + 1 particle offsets (host); x, y, z, q: concatenated
        float32 device tensors.  Returns Phi, gx, gy, gz (device, input order)."""
        import torch
        offs = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if offs.shape != (self.nsys + 1,):
            raise ValueError("offsets must have nsys + 1 entries")
        if offs[0] != 0 or np.any(np.diff(offs) < 0):
            raise ValueError("offsets must start at 0 and be non-decreasing")
        n = int(offs[-1])
        check_buffers((x, y, z, q), torch.float32, n, what="x, y, z, q")
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=x.device) for _ in range(4))
        else:
            if len(out) != 4:
                raise ValueError("out must hold four tensors (phi, gx, gy, gz)")
            check_buffers(out, torch.float32, n, what="out", device=x.device)
        self._offs = offs
        _check(load().pmmm_batch_far_f32(self._h, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                         x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                                         *[o.data_ptr() for o in out], _stream_handle(stream)))
        return out

    def sync_status(self):
        _check(load().pmmm_batch_sync_status(self._h))


class Hier:
    """Two-level hierarchical far field (pmmm_hier_*): an open FP32 coarse
    mesh of n^3 cells refined by r per axis."""

    def __init__(self, n: int, p: int, refine: int, box: float = 1.0, cutoff: int = 2,
                 n_max: int = 0, stream=None):
        L = load()
        self.params = make_params(n, p, "open", box, cutoff, "f32", 0.0, 0, n_max)
        self.n, self.p, self.refine, self.box, self.cutoff = n, p, refine, box, cutoff
        self._h = ctypes.c_void_p()
        _check(L.pmmm_hier_create(ctypes.byref(self.params), int(refine), _stream_handle(stream),
                                  ctypes.byref(self._h)))

    def close(self):
        if self._h:
            load().pmmm_hier_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, x, y, z, q, out, stream):
        import torch
        n = x.numel()
        check_buffers((x, y, z, q), torch.float32, n, what="x, y, z, q")
        if out is None:
            out = tuple(torch.empty(n, dtype=torch.float32, device=x.device) for _ in range(4))
        check_buffers(out, torch.float32, n, what="out", device=x.device)
        _check(fn(self._h, n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(),
                  *[o.data_ptr() for o in out], _stream_handle(stream)))
        return out

    def far(self, x, y, z, q, out=None, stream=None):
        return self._call(load().pmmm_hier_far_f32, x, y, z, q, out, stream)

    def total(self, x, y, z, q, out=None, stream=None):
        return self._call(load().pmmm_hier_total_f32, x, y, z, q, out, stream)

    def sync_status(self):
        _check(load().pmmm_hier_sync_status(self._h))

    def set_profiling(self, stages):
        """Enable HIP-event timing of the named stages (see STAGES) on both
        levels; the fine level's eq. M2L sums are its "column" stage."""
        mask = 0
        for st in stages:
            mask |= 1 << STAGES.index(st)
        _check(load().pmmm_hier_set_profiling(self._h, mask))

    def read_profile(self, level, reset=True):
        """{stage: (total ms, timed launches)} of level 0 (coarse) or 1
        (fine) since the last reset."""
        ms = (ctypes.c_double * len(STAGES))()
        cnt = (ctypes.c_int64 * len(STAGES))()
        _check(load().pmmm_hier_read_profile(self._h, int(level), ms, cnt, int(bool(reset))))
        return {st: (ms[i], cnt[i]) for i, st in enumerate(STAGES)}


# ------------------------------------------------- coefficient storage calls
def coef_record_words(p: int) -> int:
    """32-bit words of one per-order fixed-point cell record at order p."""
    w = load().pmmm_coef_record_words(int(p))
    if w < 0:
        raise ValueError(f"order {p} outside 0..{PMMM_PMAX}")
    return int(w)


def _coef_mesh_shape(p, coef):
    if coef.dim() != 2 or coef.shape[0] != (p + 1) ** 2:
        raise ValueError(f"coefficient mesh must have shape [(p+1)^2, ncell], got {tuple(coef.shape)}")
    return int(coef.shape[1])


def coef_pack(p: int, coef, records=None, exps=None, auto_exp: bool = True, stream=None):
    """Per-order fixed-point records of a float32 mesh [(p+1)^2, ncell]
    (pmmm_coef_pack_f32); returns (records [ncell, words] int32 holding the
    uint32 bit patterns, exps [p+1] int32)."""
    import torch
    L = load()
    ncell = _coef_mesh_shape(p, coef)
    w = coef_record_words(p)
    check_buffers((coef,), torch.float32, (p + 1) ** 2 * ncell, what="coef")
    if records is None:
        records = torch.empty((ncell, w), dtype=torch.int32, device=coef.device)
    if exps is None:
        if not auto_exp:
            raise ValueError("caller units need exps")
        exps = torch.empty(p + 1, dtype=torch.int32, device=coef.device)
    check_buffers((records,), torch.int32, ncell * w, what="records", device=coef.device)
    check_buffers((exps,), torch.int32, p + 1, what="exps", device=coef.device)
    _check(L.pmmm_coef_pack_f32(int(p), ncell, coef.data_ptr(), records.data_ptr(), exps.data_ptr(),
                                PMMM_COEF_AUTO_EXP if auto_exp else 0, _stream_handle(stream)))
    return records, exps


def coef_unpack(p: int, records, exps, out=None, stream=None):
    """Float32 mesh [(p+1)^2, ncell] from per-order fixed-point records
    (pmmm_coef_unpack_f32)."""
    import torch
    L = load()
    w = coef_record_words(p)
    if records.dim() != 2 or records.shape[1] != w:
        raise ValueError(f"records must have shape [ncell, {w}], got {tuple(records.shape)}")
    ncell = int(records.shape[0])
    check_buffers((records,), torch.int32, ncell * w, what="records")
    check_buffers((exps,), torch.int32, p + 1, what="exps", device=records.device)
    if out is None:
        out = torch.empty(((p + 1) ** 2, ncell), dtype=torch.float32, device=records.device)
    check_buffers((out,), torch.float32, (p + 1) ** 2 * ncell, shape=((p + 1) ** 2, ncell),
                  what="out", device=records.device)
    _check(L.pmmm_coef_unpack_f32(int(p), ncell, records.data_ptr(), exps.data_ptr(), out.data_ptr(),
                                  _stream_handle(stream)))
    return out


def coef_compose(p: int, a, b, out=None, stream=None):
    """App. D composite [(p+1)^2, ncell, 2] (re, im) of two real float32
    meshes [(p+1)^2, ncell] (pmmm_coef_compose_f32)."""
    import torch
    L = load()
    ncell = _coef_mesh_shape(p, a)
    P = (p + 1) ** 2
    check_buffers((a, b), torch.float32, P * ncell, shape=(P, ncell), what="a, b")
    if out is None:
        out = torch.empty((P, ncell, 2), dtype=torch.float32, device=a.device)
    check_buffers((out,), torch.float32, 2 * P * ncell, shape=(P, ncell, 2), what="out",
                  device=a.device)
    _check(L.pmmm_coef_compose_f32(int(p), ncell, a.data_ptr(), b.data_ptr(), out.data_ptr(),
                                   _stream_handle(stream)))
    return out


def coef_split(p: int, c, a=None, b=None, stream=None):
    """The two real float32 meshes [(p+1)^2, ncell] of an App. D composite
    [(p+1)^2, ncell, 2] (pmmm_coef_split_f32)."""
    import torch
    L = load()
    P = (p + 1) ** 2
    if c.dim() != 3 or c.shape[0] != P or c.shape[2] != 2:
        raise ValueError(f"composite must have shape [(p+1)^2, ncell, 2], got {tuple(c.shape)}")
    ncell = int(c.shape[1])
    check_buffers((c,), torch.float32, 2 * P * ncell, what="c")
    if a is None:
        a = torch.empty((P, ncell), dtype=torch.float32, device=c.device)
    if b is None:
        b = torch.empty((P, ncell), dtype=torch.float32, device=c.device)
    check_buffers((a, b), torch.float32, P * ncell, shape=(P, ncell), what="a, b", device=c.device)
    _check(L.pmmm_coef_split_f32(int(p), ncell, c.data_ptr(), a.data_ptr(), b.data_ptr(),
                                 _stream_handle(stream)))
    return a, b
