"""CPU oracle for batched small-array sorting -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the bench's CPU-baseline leg may import
this package.  The library (``paper_2002_05599_amd``) never does, and this
package never imports the library.

The result it defines is the one a comparator network must produce (paper,
Section 2.1): every array ends as a permutation of its input in non-decreasing
order.  ``oracle.c`` implements it as insertion sort for n <= 16 and a
separate top-down merge sort above (both stable).

All functions work on copies: inputs are numpy arrays, outputs new arrays.
"""
import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_SUFFIX = {np.dtype(np.uint32): "u32", np.dtype(np.int32): "i32",
           np.dtype(np.uint64): "u64", np.dtype(np.int64): "i64",
           np.dtype(np.float32): "f32", np.dtype(np.float64): "f64"}
# key types that also take a 64-bit payload (names ending in _v64)
_V64 = ("u64", "i64", "f64")

_P = ctypes.c_void_p
_I64 = ctypes.c_int64


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load (building first if absent) an oracle shared object."""
    if not os.path.exists(path):
        _build.build(out=path)
    lib = ctypes.CDLL(path)
    for s in list(_SUFFIX.values()) + [f"{k}_v64" for k in _V64]:
        getattr(lib, f"oracle_insertion_sort_{s}").argtypes = [_P, _P, _I64]
        getattr(lib, f"oracle_insertion_sort_{s}").restype = None
        for name in ("merge_sort", "sort"):
            f = getattr(lib, f"oracle_{name}_{s}")
            f.argtypes = [_P, _P, _I64]
            f.restype = ctypes.c_int
        f = getattr(lib, f"oracle_sort_fixed_{s}")
        f.argtypes = [_P, _I64, _I64, _I64]
        f.restype = ctypes.c_int
        f = getattr(lib, f"oracle_sort_segments_{s}")
        f.argtypes = [_P, _P, _P, _I64]
        f.restype = ctypes.c_int
    return lib


_lib = None


def _get(lib=None):
    global _lib
    if lib is not None:
        return lib
    if _lib is None:
        _lib = load()
    return _lib


def _suffix(keys: np.ndarray, vals=None) -> str:
    try:
        s = _SUFFIX[keys.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {keys.dtype}") from None
    if vals is not None and vals.dtype == np.uint64:
        if s not in _V64:
            raise TypeError("a 64-bit payload needs 64-bit keys")
        s += "_v64"
    return s


def _vals_copy(vals):
    """A copy of the payload as uint64 if it is uint64, else as uint32."""
    if vals is None:
        return None
    v = np.asarray(vals)
    return np.array(v, dtype=np.uint64 if v.dtype == np.uint64 else np.uint32, copy=True)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(rc):
    if rc != 0:
        raise MemoryError("oracle scratch allocation failed")


def insertion_sort(keys, vals=None, lib=None):
    """Insertion sort of one 1-D array (any n); returns (keys, vals) copies."""
    k = np.array(keys, copy=True)
    v = _vals_copy(vals)
    getattr(_get(lib), f"oracle_insertion_sort_{_suffix(k, v)}")(_ptr(k), _ptr(v), k.size)
    return k, v


def merge_sort(keys, vals=None, lib=None):
    """Top-down merge sort of one 1-D array (any n); returns copies."""
    k = np.array(keys, copy=True)
    v = _vals_copy(vals)
    _check(getattr(_get(lib), f"oracle_merge_sort_{_suffix(k, v)}")(_ptr(k), _ptr(v), k.size))
    return k, v


def sort_one(keys, vals=None, lib=None):
    """The dispatching sort: insertion sort if n <= 16, else merge sort."""
    k = np.array(keys, copy=True)
    v = _vals_copy(vals)
    _check(getattr(_get(lib), f"oracle_sort_{_suffix(k, v)}")(_ptr(k), _ptr(v), k.size))
    return k, v


def sort_fixed(keys, n, count, stride, lib=None, threads=1):
    """Sort arrays keys[i*stride : i*stride+n] for i < count; returns a copy.

    ``threads`` > 1 splits the arrays into contiguous ranges sorted by that many
    host threads (ctypes releases the GIL during the call).
    """
    k = np.array(keys, copy=True)
    if count * stride > k.size and count > 0:
        raise ValueError("keys too short for count*stride")
    f = getattr(_get(lib), f"oracle_sort_fixed_{_suffix(k)}")
    item = k.itemsize
    if threads <= 1 or count < 2 * threads:
        _check(f(_ptr(k), n, count, stride))
        return k
    bounds = np.linspace(0, count, threads + 1).astype(np.int64)

    def work(t):
        lo, hi = int(bounds[t]), int(bounds[t + 1])
        return f(k.ctypes.data + lo * stride * item, n, hi - lo, stride)

    with ThreadPoolExecutor(threads) as ex:
        for rc in ex.map(work, range(threads)):
            _check(rc)
    return k


def sort_fixed_inplace(k, n, count, stride, lib=None, threads=1):
    """Like sort_fixed, but sorts the numpy array ``k`` in place (no copy), so a
    timing loop can restore its input outside the timed region."""
    if count * stride > k.size and count > 0:
        raise ValueError("keys too short for count*stride")
    f = getattr(_get(lib), f"oracle_sort_fixed_{_suffix(k)}")
    item = k.itemsize
    if threads <= 1 or count < 2 * threads:
        _check(f(_ptr(k), n, count, stride))
        return k
    bounds = np.linspace(0, count, threads + 1).astype(np.int64)

    def work(t):
        lo, hi = int(bounds[t]), int(bounds[t + 1])
        return f(k.ctypes.data + lo * stride * item, n, hi - lo, stride)

    with ThreadPoolExecutor(threads) as ex:
        for rc in ex.map(work, range(threads)):
            _check(rc)
    return k


def sort_segments(keys, offsets, vals=None, lib=None, threads=1):
    """Sort CSR segments [offsets[i], offsets[i+1]); returns (keys, vals) copies."""
    k = np.array(keys, copy=True)
    v = _vals_copy(vals)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    nseg = off.size - 1
    f = getattr(_get(lib), f"oracle_sort_segments_{_suffix(k, v)}")
    if threads <= 1 or nseg < 2 * threads:
        _check(f(_ptr(k), _ptr(v), _ptr(off), max(nseg, 0)))
        return k, v
    bounds = np.linspace(0, nseg, threads + 1).astype(np.int64)

    def work(t):
        lo, hi = int(bounds[t]), int(bounds[t + 1])
        # offsets are absolute, so each thread gets the same base pointers.
        return f(_ptr(k), _ptr(v), off.ctypes.data + lo * 4, hi - lo)

    with ThreadPoolExecutor(threads) as ex:
        for rc in ex.map(work, range(threads)):
            _check(rc)
    return k, v
