"""The C-ABI library loads and exports what include/smallsort.h declares (no GPU compute)."""
import ctypes
import os
import re

import pytest

import paper_2002_05599_amd as ss

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smallsort.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_0-9]+)\s*\([^;{]*\)\s*;", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ss.lib_path()):
        pytest.fail("libsmallsort.so is not built (run __graft_entry__.build())")
    return ss.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["sort_small_u32", "sort_small_i32", "sort_small_u64", "sort_small_i64",
                 "segmented_sort_u32", "segmented_sort_i32", "segmented_sort_u64", "segmented_sort_i64",
                 "ss_segmented_sort", "ss_device_status", "ss_strerror", "ss_load_tuning",
                 "ss_set_tuning_value", "ss_get_tuning_value", "ss_version", "ss_stream_copy"]:
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(ss.lib_path())
    for name in declared_functions():
        assert hasattr(raw, name), f"{name} declared but not exported"
    assert set(declared_functions()) <= set(ss._SIGS), "binding misses a declared function"


def test_strerror_and_version(lib):
    assert lib.ss_strerror(0) == b"success"
    assert b"aligned" in lib.ss_strerror(-2)
    assert lib.ss_strerror(12345) == b"unknown status"
    assert ss.version().startswith("smallsort")


def test_argument_errors_need_no_device(lib):
    p = ctypes.c_void_p(0x1000)
    # n > 4096, stride < n, negative sizes, misalignment: rejected on the host
    assert lib.sort_small_u32(p, 4097, 1, 4097, None) == -3
    assert lib.sort_small_u32(p, 8, 1, 7, None) == -1
    assert lib.sort_small_u32(p, -1, 1, 8, None) == -1
    assert lib.sort_small_u32(p, 8, -5, 8, None) == -1
    assert lib.sort_small_u64(ctypes.c_void_p(0x1004), 8, 1, 8, None) == -2
    assert lib.sort_small_u32(None, 8, 3, 8, None) == -1
    # no-ops succeed without touching memory
    assert lib.sort_small_u32(None, 8, 0, 8, None) == 0
    assert lib.sort_small_i64(None, 1, 100, 1, None) == 0
    assert lib.sort_small_i32(p, 0, 100, 0, None) == 0
    assert lib.ss_segmented_sort(0, None, None, None, 0, 0, None) == 0
    assert lib.ss_segmented_sort(0, None, None, None, -1, 0, None) == -1
    assert lib.ss_segmented_sort(7, p, None, p, 1, 0, None) == -1
    assert lib.ss_segmented_sort(0, p, None, p, 1, 9, None) == -1
    assert lib.ss_segmented_sort(2, ctypes.c_void_p(0x1004), None, p, 1, 0, None) == -2
    assert lib.ss_device_status(None, None) == -1
    assert lib.ss_stream_copy(p, p, -16, None) == -1
    assert lib.ss_stream_copy(None, None, 0, None) == 0
    assert lib.ss_stream_copy(None, p, 16, None) == -1
    assert lib.ss_stream_copy(p, ctypes.c_void_p(0x1008), 16, None) == -2
    assert lib.ss_stream_copy(p, p, 24, None) == -2


def test_tuning_roundtrip(lib, tmp_path):
    # per-width knobs may differ between the widths: save and restore each width
    old = {w: ss.get_tuning(f"{w}.rss_k_small") for w in ("u32", "u64")}
    old_family = {w: ss.get_tuning(f"{w}.family") for w in ("u32", "u64")}
    ss.set_tuning("rss_k_small", 8)
    assert ss.get_tuning("rss_k_small") == 8
    with pytest.raises(ss.SmallSortError):
        ss.set_tuning("rss_k_small", 5)
    with pytest.raises(ss.SmallSortError):
        ss.set_tuning("rss_k_small", 32)  # a 16-lane group takes at most 16 buckets
    old_mid = {w: ss.get_tuning(f"{w}.rss_k_mid") for w in ("u32", "u64")}
    old_large = {w: ss.get_tuning(f"{w}.rss_k_large") for w in ("u32", "u64")}
    ss.set_tuning("rss_k_mid", 32)
    ss.set_tuning("rss_k_large", 64)
    assert ss.get_tuning("rss_k_mid") == 32 and ss.get_tuning("rss_k_large") == 64
    for name, bad in (("rss_k_mid", 64), ("rss_k_large", 48), ("rss_k_large", 128), ("rss_k_large", 2)):
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning(name, bad)
    for w in ("u32", "u64"):
        ss.set_tuning(f"{w}.rss_k_mid", old_mid[w])
        ss.set_tuning(f"{w}.rss_k_large", old_large[w])
    with pytest.raises(ss.SmallSortError):
        ss.set_tuning("no_such_knob", 1)
    assert ss.get_tuning("no_such_knob") == -1
    f = tmp_path / "t.json"
    f.write_text('{"rss_k_small": 16, "family": 1, "note": "x", "other": 3.5}')
    ss.load_tuning(str(f))
    assert ss.get_tuning("rss_k_small") == 16 and ss.get_tuning("family") == 1
    f.write_text('{"rss_k_small": 4, ')
    with pytest.raises(ss.SmallSortError):
        ss.load_tuning(str(f))
    for name, bad in (("family", 3), ("large_sort", 2)):
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning(name, bad)
    for w in ("u32", "u64"):
        ss.set_tuning(f"{w}.family", old_family[w])
        ss.set_tuning(f"{w}.rss_k_small", old[w])
    old_cap = ss.get_tuning("rss_level_cap")
    for bad in (0, 9):
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning("rss_level_cap", bad)
    ss.set_tuning("rss_level_cap", 1)
    assert ss.get_tuning("rss_level_cap") == 1
    ss.set_tuning("rss_level_cap", old_cap)


def test_binding_maps_one_hip_runtime():
    """Loading the library before torch is imported must still leave one HIP
    runtime in the process: torch's streams are handles of that runtime."""
    import subprocess
    import sys
    code = ("import paper_2002_05599_amd as ss; ss.get_tuning('family'); import torch; import os; "
            "print(len({os.path.realpath(l.split()[-1]) for l in open('/proc/self/maps') "
            "if 'libamdhip64' in l and '/' in l}))")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_library_leaves_no_symbol_of_its_own_undefined():
    """Every kernel set the dispatch refers to was instantiated in some unit."""
    import subprocess
    r = subprocess.run(["nm", "-uC", ss.lib_path()], capture_output=True, text=True, check=True)
    missing = [ln for ln in r.stdout.splitlines() if "ss::" in ln]
    assert not missing, missing


def test_device_sort_workspace_size(lib):
    """ss_sort_workspace_bytes: 0 for invalid arguments, about the data size
    plus a few percent for large n, growing with n."""
    f = lib.ss_sort_workspace_bytes
    assert f(9, 0, 100) == 0 and f(0, 8, 100) == 0 and f(0, 3, 100) == 0 and f(0, 0, -1) == 0
    assert f(0, 0, 2**31) == 0
    for kt, kb in ((0, 4), (2, 8)):
        for vb in (0, 4):
            n = 10_000_000
            w = f(kt, vb, n)
            assert n * (kb + vb) <= w <= 1.2 * n * (kb + vb) + (1 << 20)
            assert f(kt, vb, n // 10) < w
    assert f(2, 8, 1000) > 0


def test_per_width_tuning(lib):
    """Per-width knobs: the plain name sets both widths, a prefixed name one;
    a plain get of differing widths reads -2; global knobs take no prefix;
    the lane-group bounds stay ordered; the tile-form masks take bits 2..16."""
    from helpers import tuned
    with tuned(family=1, rss_bound_small=64, rss_bound_mid=128, fixed_half=0, fixed_wide=0, fixed_wider=0):
        ss.set_tuning("u64.family", 0)
        assert ss.get_tuning("u32.family") == 1 and ss.get_tuning("u64.family") == 0
        assert ss.get_tuning("family") == -2
        ss.set_tuning("family", 2)
        assert ss.get_tuning("family") == 2
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning("u32.rss_rounds", 8)  # one value for every width
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning("rss_bound_small", 65)  # a 16-lane group holds at most 64 keys
        ss.set_tuning("rss_bound_mid", 96)
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning("rss_bound_mid", 32)  # below bound_small (64)
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning("fixed_apt", 3)
        for v in (1, 4):
            ss.set_tuning("rss_oversample", v)
        with pytest.raises(ss.SmallSortError):
            ss.set_tuning("rss_oversample", 5)
        for knob in ("fixed_half", "fixed_wide", "fixed_wider"):
            ss.set_tuning(f"u32.{knob}", 0x1FFFC)
            ss.set_tuning(f"u64.{knob}", 1 << 16)
            assert ss.get_tuning(f"u32.{knob}") == 0x1FFFC and ss.get_tuning(f"u64.{knob}") == 1 << 16
            for bad in (1, 2, 0x20000):  # n = 0, 1 and 17 have no bit
                with pytest.raises(ss.SmallSortError):
                    ss.set_tuning(knob, bad)
