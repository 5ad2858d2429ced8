"""Shared test helpers: device transfer and comparisons against the oracle."""
import numpy as np

_TORCH_DT = None


def torch_dtype(np_dtype):
    import torch
    return {np.dtype(np.uint32): torch.uint32, np.dtype(np.int32): torch.int32,
            np.dtype(np.uint64): torch.uint64, np.dtype(np.int64): torch.int64}[np.dtype(np_dtype)]


def to_dev(a: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def from_dev(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def first_mismatch(got: np.ndarray, want: np.ndarray, row: int = 0):
    """Human-readable description of the first differing row (row length ``row``)."""
    bad = np.nonzero(got != want)[0]
    if bad.size == 0:
        return None
    i = int(bad[0])
    if row:
        r = i // row
        return f"row {r}: got {got[r*row:(r+1)*row]} want {want[r*row:(r+1)*row]}"
    return f"index {i}: got {got[i]} want {want[i]}"


def pairs_multiset_equal(k1, v1, k2, v2, offsets):
    """Per segment, the multisets of (key, val) pairs agree."""
    for i in range(offsets.size - 1):
        lo, hi = offsets[i], offsets[i + 1]
        a = sorted(zip(k1[lo:hi].tolist(), v1[lo:hi].tolist()))
        b = sorted(zip(k2[lo:hi].tolist(), v2[lo:hi].tolist()))
        if a != b:
            return i
    return None


class tuned:
    """Context manager: set tuning knobs, restore them on exit."""

    def __init__(self, **knobs):
        self.knobs = knobs

    def __enter__(self):
        import paper_2002_05599_amd as ss
        self.old = {}
        for k in self.knobs:  # per-width knobs are restored per width
            for name in ((f"u32.{k}", f"u64.{k}") if ss.get_tuning(f"u32.{k}") >= 0 else (k,)):
                self.old[name] = ss.get_tuning(name)
        # ordered knobs (the lane-group bounds) may need another pass
        for _ in range(2):
            for k, v in self.knobs.items():
                try:
                    ss.set_tuning(k, v)
                except ss.SmallSortError:
                    pass
        try:
            for k, v in self.knobs.items():
                ss.set_tuning(k, v)
        except ss.SmallSortError:
            self.__exit__(None, None, None)  # leave no knob half-set
            raise
        return self

    def __exit__(self, *exc):
        import paper_2002_05599_amd as ss
        for _ in range(3):  # a bound may only be valid once the others are back
            for k, v in self.old.items():
                try:
                    ss.set_tuning(k, v)
                except ss.SmallSortError:
                    pass
        return False
