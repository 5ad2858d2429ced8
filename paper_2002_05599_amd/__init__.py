"""Batched small-array sorting on AMD MI355X (gfx950).

Thin ctypes binding over ``libsmallsort.so`` (declared in
``include/smallsort.h``).  It only marshals arguments: every step of the sort
runs in the library's HIP kernels.  PyTorch supplies device memory and the
current stream.  If the library has not been built the first call raises
``RuntimeError`` -- there is no fallback implementation.

Method: Bingmann, Marianczuk, Sanders, "Engineering Faster Sorters for Small
Sets of Items": comparator networks for 2..16 keys (Section 2) and Register
Sample Sort for 17..256 keys (Section 3).
"""
import ctypes
import os
import threading

__all__ = [
    "SmallSortError", "lib", "lib_path", "sort_small", "segmented_sort", "device_status",
    "set_tuning", "get_tuning", "load_tuning", "tuning_path", "version", "KEY_CODES",
    "MODE_AUTO", "MODE_PERSISTENT", "MODE_PLAIN", "stream_copy", "segmented_sort_noalloc",
    "NOALLOC_MAX_SEGMENTS", "sort", "sort_workspace_bytes", "tuned",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "libsmallsort.so"

MODE_AUTO, MODE_PERSISTENT, MODE_PLAIN = 0, 1, 2
KEY_CODES = {"uint32": 0, "int32": 1, "uint64": 2, "int64": 3, "float32": 4, "float64": 5}
_SUFFIX = {"uint32": "u32", "int32": "i32", "uint64": "u64", "int64": "i64", "float32": "f32", "float64": "f64"}

# Every symbol include/smallsort.h declares, with its ctypes signature.
_P = ctypes.c_void_p
_SIGS = {
    **{f"sort_small_{s}": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _P])
       for s in _SUFFIX.values()},
    **{f"segmented_sort_{s}": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, _P])
       for s in _SUFFIX.values()},
    "ss_segmented_sort": (ctypes.c_int32, [ctypes.c_int32, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P]),
    "ss_device_status": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "ss_strerror": (ctypes.c_char_p, [ctypes.c_int32]),
    "ss_set_tuning_value": (ctypes.c_int32, [ctypes.c_char_p, ctypes.c_int64]),
    "ss_get_tuning_value": (ctypes.c_int64, [ctypes.c_char_p]),
    "ss_load_tuning": (ctypes.c_int32, [ctypes.c_char_p]),
    "ss_version": (ctypes.c_char_p, []),
    "ss_stream_copy": (ctypes.c_int32, [_P, _P, ctypes.c_int64, _P]),
    "ss_segmented_sort_noalloc": (ctypes.c_int32, [ctypes.c_int32, _P, _P, _P, ctypes.c_int32, _P]),
    "ss_segmented_sort_v": (ctypes.c_int32, [ctypes.c_int32, _P, _P, ctypes.c_int32, _P, ctypes.c_int32,
                                             ctypes.c_int32, _P]),
    "segmented_sort_pairs_u64": (ctypes.c_int32, [_P, _P, _P, ctypes.c_int32, _P]),
    "ss_sort_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]),
    "ss_sort": (ctypes.c_int32, [ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_size_t, _P]),
}

NOALLOC_MAX_SEGMENTS = 1 << 24  # SS_NOALLOC_MAX_SEGMENTS

_lock = threading.Lock()
_lib = None


class SmallSortError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = lib().ss_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")


def lib_path() -> str:
    return os.environ.get("SMALLSORT_LIB", os.path.join(_HERE, LIB_NAME))


def lib() -> ctypes.CDLL:
    """The loaded library; raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            path = lib_path()
            if not os.path.exists(path):
                raise RuntimeError(
                    f"{path} not found: build it with `python -m paper_2002_05599_amd.build` "
                    "(or __graft_entry__.build()); there is no non-GPU fallback")
            # torch first: it maps the HIP runtime it bundles, whose soname
            # the library's dependency then resolves to.  Loaded the other way
            # round, the process would hold two HIP runtimes and torch's
            # streams would be foreign handles to the library's runtime.
            import torch  # noqa: F401
            handle = ctypes.CDLL(path)
            _check_one_hip_runtime()
            for name, (res, args) in _SIGS.items():
                f = getattr(handle, name)
                f.restype = res
                f.argtypes = args
            _lib = handle
            _autoload_tuning(handle)
    return _lib


def _check_one_hip_runtime():
    """Raise if two different HIP runtimes are mapped into the process."""
    try:
        maps = open("/proc/self/maps").read().splitlines()
    except OSError:
        return
    paths = {os.path.realpath(ln.split()[-1]) for ln in maps if "libamdhip64" in ln and "/" in ln}
    if len(paths) > 1:
        raise RuntimeError("two HIP runtimes are loaded (" + ", ".join(sorted(paths)) + "); import torch "
                           "before anything loads libamdhip64 so that one runtime serves both")


def tuning_path() -> str:
    return os.environ.get("SMALLSORT_TUNING", os.path.join(_HERE, "tuning_gfx950.json"))


def _autoload_tuning(handle):
    """Apply the autotuner's saved choices if they were measured on this ROCm.

    SMALLSORT_TUNING=<path> selects another file, SMALLSORT_TUNING=none
    disables loading.  A file recorded under another ROCm version is ignored
    (the defaults apply until the tuner is run again).
    """
    import json
    path = tuning_path()
    if path == "none" or not os.path.exists(path):
        return
    try:
        doc = json.load(open(path))
        import torch
        if doc.get("rocm") not in (None, str(torch.version.hip)):
            return
    except (OSError, ValueError, ImportError):
        return
    handle.ss_load_tuning(os.fsencode(path))


def _check(status, what):
    if status != 0:
        raise SmallSortError(status, what)


def _dtype_name(t):
    name = str(t.dtype).replace("torch.", "")
    if name not in _SUFFIX:
        raise TypeError(f"unsupported key dtype {t.dtype}; use uint32, int32, uint64, int64, float32 or float64")
    return name


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _require_cuda(t, what):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def sort_small(keys, n, count=None, stride=None, stream=None):
    """Sort ``count`` arrays ``keys[i*stride : i*stride+n]`` in place (n <= 256).

    ``keys`` is a contiguous device tensor of uint32/int32/uint64/int64.
    Defaults: stride = n, count = numel // stride.
    """
    _require_cuda(keys, "keys")
    name = _dtype_name(keys)
    stride = n if stride is None else stride
    if count is None:
        count = keys.numel() // stride if stride > 0 else 0
    if count * stride > keys.numel() + (stride - n if count > 0 else 0):
        raise ValueError("keys tensor too small for count*stride")
    f = getattr(lib(), f"sort_small_{_SUFFIX[name]}")
    _check(f(ctypes.c_void_p(keys.data_ptr()), int(n), int(count), int(stride), _stream_ptr(stream)),
           f"sort_small_{_SUFFIX[name]}")
    return keys


def segmented_sort(keys, offsets, vals=None, mode=MODE_AUTO, stream=None):
    """Sort CSR segments ``[offsets[i], offsets[i+1])`` of ``keys`` in place.

    ``offsets``: device int32 tensor of nseg+1 entries.  ``vals``: optional
    device uint32 tensor (or uint64, with 64-bit keys: the key + reference
    items of Section 2.2) permuted with the keys.  ``mode``: MODE_AUTO
    (persistent kernel from a cached graph), MODE_PERSISTENT (no graph) or
    MODE_PLAIN (one launch per size class).
    """
    _require_cuda(keys, "keys")
    _require_cuda(offsets, "offsets")
    name = _dtype_name(keys)
    if str(offsets.dtype) != "torch.int32":
        raise TypeError("offsets must be int32")
    nseg = offsets.numel() - 1
    vptr, vbytes = None, 4
    if vals is not None:
        _require_cuda(vals, "vals")
        if str(vals.dtype) not in ("torch.uint32", "torch.uint64") or vals.numel() != keys.numel():
            raise TypeError("vals must be a uint32 or uint64 tensor shaped like keys")
        vptr = ctypes.c_void_p(vals.data_ptr())
        vbytes = vals.element_size()
    st = lib().ss_segmented_sort_v(KEY_CODES[name], ctypes.c_void_p(keys.data_ptr()), vptr, vbytes,
                                   ctypes.c_void_p(offsets.data_ptr()), max(nseg, 0), int(mode),
                                   _stream_ptr(stream))
    _check(st, "ss_segmented_sort_v")
    return keys, vals


def segmented_sort_noalloc(keys, offsets, vals=None, stream=None):
    """``segmented_sort`` through the entry point that allocates no device
    memory (fixed per-device scratch; at most NOALLOC_MAX_SEGMENTS segments;
    calls that overlap on one device race)."""
    _require_cuda(keys, "keys")
    _require_cuda(offsets, "offsets")
    name = _dtype_name(keys)
    if str(offsets.dtype) != "torch.int32":
        raise TypeError("offsets must be int32")
    nseg = offsets.numel() - 1
    vptr = None
    if vals is not None:
        _require_cuda(vals, "vals")
        if str(vals.dtype) != "torch.uint32" or vals.numel() != keys.numel():
            raise TypeError("vals must be a uint32 tensor shaped like keys")
        vptr = ctypes.c_void_p(vals.data_ptr())
    st = lib().ss_segmented_sort_noalloc(KEY_CODES[name], ctypes.c_void_p(keys.data_ptr()), vptr,
                                         ctypes.c_void_p(offsets.data_ptr()), max(nseg, 0), _stream_ptr(stream))
    _check(st, "ss_segmented_sort_noalloc")
    return keys, vals


def sort_workspace_bytes(dtype_name, n, val_bytes=0) -> int:
    """Device workspace ``sort`` needs for n keys of the named dtype."""
    return int(lib().ss_sort_workspace_bytes(KEY_CODES[dtype_name], int(val_bytes), int(n)))


def sort(keys, vals=None, workspace=None, stream=None):
    """Sort the whole 1-D device tensor ``keys`` (and ``vals``, uint32 or
    uint64) in place: the device-wide sort with the small sorters as base
    case.  ``workspace``: a device tensor of at least sort_workspace_bytes
    bytes; if omitted, one is allocated with torch for this call."""
    import torch
    _require_cuda(keys, "keys")
    name = _dtype_name(keys)
    vptr, vbytes = None, 0
    if vals is not None:
        _require_cuda(vals, "vals")
        if str(vals.dtype) not in ("torch.uint32", "torch.uint64") or vals.numel() != keys.numel():
            raise TypeError("vals must be a uint32 or uint64 tensor shaped like keys")
        vptr, vbytes = ctypes.c_void_p(vals.data_ptr()), vals.element_size()
    need = sort_workspace_bytes(name, keys.numel(), vbytes)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
    st = lib().ss_sort(KEY_CODES[name], ctypes.c_void_p(keys.data_ptr()), vptr, vbytes, keys.numel(),
                       ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                       _stream_ptr(stream))
    _check(st, "ss_sort")
    return keys, vals


def device_status(stream=None) -> int:
    """Synchronise ``stream``, return and clear the device status word."""
    out = ctypes.c_int32(0)
    _check(lib().ss_device_status(_stream_ptr(stream), ctypes.byref(out)), "ss_device_status")
    return out.value


def set_tuning(name: str, value: int):
    _check(lib().ss_set_tuning_value(name.encode(), int(value)), f"ss_set_tuning_value({name})")


def get_tuning(name: str) -> int:
    return int(lib().ss_get_tuning_value(name.encode()))


class tuned:
    """Context manager: set tuning knobs for a block, then restore them (a
    knob kept per key width is restored per width)."""

    def __init__(self, **knobs):
        self.knobs = knobs

    def __enter__(self):
        self.old = {}
        for k in self.knobs:
            names = (f"u32.{k}", f"u64.{k}") if get_tuning(f"u32.{k}") >= 0 else (k,)
            for name in names:
                self.old[name] = get_tuning(name)
        for _ in range(2):  # ordered knobs (the lane-group bounds) may need another pass
            for k, v in self.knobs.items():
                try:
                    set_tuning(k, v)
                except SmallSortError:
                    pass
        try:
            for k, v in self.knobs.items():
                set_tuning(k, v)
        except SmallSortError:
            self.__exit__(None, None, None)  # leave no knob half-set
            raise
        return self

    def __exit__(self, *exc):
        for _ in range(3):  # a bound may only be valid once the others are back
            for k, v in self.old.items():
                try:
                    set_tuning(k, v)
                except SmallSortError:
                    pass
        return False


def load_tuning(path: str):
    _check(lib().ss_load_tuning(os.fsencode(path)), f"ss_load_tuning({path})")


def stream_copy(dst, src, stream=None):
    """Streaming device copy of ``src`` into ``dst`` (same byte size, 16-byte aligned)."""
    _require_cuda(dst, "dst")
    _require_cuda(src, "src")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src must have the same byte size")
    _check(lib().ss_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                int(nbytes), _stream_ptr(stream)), "ss_stream_copy")
    return dst


def version() -> str:
    return lib().ss_version().decode()
