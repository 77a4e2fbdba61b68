"""The C ABI without a GPU: the library loads, exports every function that
include/hm.h declares, and rejects malformed input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2
from tests.conftest import ROOT


def _declared():
    src = open(os.path.join(ROOT, "include", "hm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z_0-9]+)\s*\(", src)) - {"hm_status"})


def test_library_exports_every_declared_function():
    from paper_1812_07152_amd import hm
    names = _declared()
    assert "hm_eval" in names and "hm_load_compressed" in names
    for n in names:
        assert hasattr(hm.lib, n), f"{n} declared in hm.h but not exported"


@pytest.fixture(scope="module")
def good_file(tmp_path_factory):
    w = wl.small("abi", N=600, d=3, m=40)
    H = OracleH2.from_workload(w, wl.gen_points(w))
    path = str(tmp_path_factory.mktemp("abi") / "good.hmc")
    H.write(path)
    return path


def _status(path):
    from paper_1812_07152_amd import hm
    out = ctypes.c_void_p()
    return hm.lib.hm_load_compressed(os.fsencode(path), 0, 1, ctypes.byref(out)), hm.hm_last_error()


def _mutate(src, dst, off, data):
    raw = bytearray(open(src, "rb").read())
    if off is None:
        raw = raw[:data]
    else:
        raw[off:off + len(data)] = data
    open(dst, "wb").write(bytes(raw))


@pytest.mark.parametrize("what,off,data", [
    ("magic", 0, b"XMC1"),
    ("version", 4, np.uint32(7).tobytes()),
    ("truncated", None, 5000),
    ("short_header", None, 100),
    ("n_nodes", 24, np.int32(5).tobytes()),
    ("perm_dup", 128, np.int64(1).tobytes()),   # perm[0] = perm[1] = 1
    ("negative_len", 104, np.int64(-3).tobytes()),
])
def test_malformed_file_is_format_error(good_file, tmp_path, what, off, data):
    from paper_1812_07152_amd import hm
    bad = str(tmp_path / f"{what}.hmc")
    _mutate(good_file, bad, off, data)
    st, msg = _status(bad)
    assert st == hm.HM_ERR_FORMAT, (st, msg)
    assert msg


def test_missing_file_and_null_arguments():
    from paper_1812_07152_amd import hm
    st, msg = _status("/nonexistent/file.hmc")
    assert st == hm.HM_ERR_INVALID and "cannot open" in msg
    assert hm.lib.hm_eval(None, None, 1, None, 1, 1, 0, 0, 0, None) == hm.HM_ERR_INVALID
    assert hm.lib.hm_eval_noalloc(None, None, 1, None, 1, 1, 0, 0, 0, None) == hm.HM_ERR_INVALID
    assert "hm_eval_noalloc" in hm.hm_last_error()
    assert hm.lib.hm_info(None, None) == hm.HM_ERR_INVALID
    assert hm.lib.hm_free(None) == hm.HM_OK
    out = ctypes.c_void_p()
    assert hm.lib.hm_load_compressed_mem(None, 0, 1, ctypes.byref(out)) == hm.HM_ERR_INVALID
    assert hm.lib.hm_load_compressed(b"x", 0, 0, ctypes.byref(out)) == hm.HM_ERR_INVALID
    assert hm.lib.hm_set_points(None, None, 3, 3, 0, 1.0) == hm.HM_ERR_INVALID
    # the near blocks may be left out of the FP64 store only
    no_near_fp32 = hm.HM_LOAD_NO_NEAR_BLOCKS | hm.precbit(hm.HM_PREC_FP64) | hm.precbit(hm.HM_PREC_FP32)
    assert hm.lib.hm_load_compressed(b"x", 0, no_near_fp32, ctypes.byref(out)) == hm.HM_ERR_INVALID
    # so may the far blocks
    no_far_fp32 = hm.HM_LOAD_NO_FAR_BLOCKS | hm.precbit(hm.HM_PREC_FP64) | hm.precbit(hm.HM_PREC_FP32)
    assert hm.lib.hm_load_compressed(b"x", 0, no_far_fp32, ctypes.byref(out)) == hm.HM_ERR_INVALID


def test_inconsistent_host_arrays_are_format_errors():
    """Structural validation of hm_load_compressed_mem, mutating one array at a time."""
    from paper_1812_07152_amd import hm
    w = wl.small("abi2", N=500, d=3, m=40)
    H = OracleH2.from_workload(w, wl.gen_points(w))

    class R:
        pass

    def clone():
        r = R()
        for k in ("N", "d", "n_nodes", "perm", "start", "size", "parent", "left", "right", "level",
                  "rank", "basis_off", "basis", "far_ptr", "far_col", "far_off", "B", "near_ptr",
                  "near_col", "near_off", "D"):
            v = getattr(H, k)
            setattr(r, k, v.copy() if isinstance(v, np.ndarray) else v)
        return r

    mutations = {
        "rank_too_big": lambda r: r.rank.__setitem__(int(np.argmax(r.left < 0)), 10**6),
        "child_range": lambda r: r.start.__setitem__(1, 3),
        "far_col_oob": lambda r: r.far_col.__setitem__(0, r.n_nodes + 5),
        "near_internal": lambda r: r.near_col.__setitem__(0, 0),
        "D_offset": lambda r: r.near_off.__setitem__(len(r.near_off) - 1, len(r.D)),
        "far_self": lambda r: r.far_col.__setitem__(0, int(np.nonzero(np.diff(r.far_ptr))[0][0])),
    }
    for name, mut in mutations.items():
        r = clone()
        mut(r)
        rep, keep = hm.host_repr(r)
        out = ctypes.c_void_p()
        st = hm.lib.hm_load_compressed_mem(ctypes.byref(rep), 0, 1, ctypes.byref(out))
        assert st == hm.HM_ERR_FORMAT, (name, st, hm.hm_last_error())


def test_skeletons_are_validated():
    """Optional skeletons in hm_load_compressed_mem: checked against the ranks
    and N (format errors), and required by HM_LOAD_NO_FAR_BLOCKS."""
    from paper_1812_07152_amd import hm
    w = wl.small("abi3", N=600, d=3, m=40)
    H = OracleH2.from_workload(w, wl.gen_points(w))
    assert len(H.skel) > 0
    fp64 = hm.precbit(hm.HM_PREC_FP64)

    def load(obj, mask, skeletons=True):
        rep, keep = hm.host_repr(obj, skeletons)
        out = ctypes.c_void_p()
        st = hm.lib.hm_load_compressed_mem(ctypes.byref(rep), 0, mask, ctypes.byref(out))
        del keep
        return st

    # without the skeletons the far blocks cannot be left out
    assert load(H, fp64 | hm.HM_LOAD_NO_FAR_BLOCKS, skeletons=False) == hm.HM_ERR_INVALID
    assert "skeletons" in hm.hm_last_error()

    class R:
        pass

    def clone():
        r = R()
        for k in ("N", "d", "n_nodes", "perm", "start", "size", "parent", "left", "right", "level",
                  "rank", "basis_off", "basis", "far_ptr", "far_col", "far_off", "B", "near_ptr",
                  "near_col", "near_off", "D", "skel_ptr", "skel"):
            v = getattr(H, k)
            setattr(r, k, v.copy() if isinstance(v, np.ndarray) else v)
        return r

    a = int(np.argmax(H.rank > 0))
    mutations = {
        "skel_oob": lambda r: r.skel.__setitem__(0, r.N),
        "skel_negative": lambda r: r.skel.__setitem__(len(r.skel) - 1, -1),
        "skel_size": lambda r: r.skel_ptr.__setitem__(a + 1, r.skel_ptr[a + 1] - 1),
    }
    for name, mut in mutations.items():
        r = clone()
        mut(r)
        st = load(r, fp64)
        assert st == hm.HM_ERR_FORMAT, (name, st, hm.hm_last_error())
