"""The C-ABI library loads on a host without a GPU and exports every entry
point the header declares (no compute calls here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "famst.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(famst_[a-z_0-9]+)\s*\(", txt)))


def _lib():
    from paper_2507_14261_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libfamst.so not built")
    return L


def test_header_declares_the_five_phase_calls():
    names = _declared()
    for n in ["famst_knn_graph", "famst_connect", "famst_refine", "famst_mst", "famst_mst_backward"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTS) == _declared()


def test_exports_are_c_symbols():
    L = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _declared():
        assert name in syms, name


def test_host_only_calls():
    L = _lib()
    lib = L.load()
    assert lib.famst_version() >= 100
    assert lib.famst_strerror(-3) == b"edges do not span every cloud"
    assert lib.famst_strerror(-8) == b"a bounded wait inside a kernel ran out"
    assert lib.famst_strerror(0) == b"ok"


def test_constants_match_header():
    L = _lib()
    txt = open(HEADER).read()
    for name in ["FAMST_OK", "FAMST_EINVAL", "FAMST_ECAPACITY", "FAMST_EDISCONNECTED", "FAMST_EHIP",
                 "FAMST_ENOTIMPL", "FAMST_ENONFINITE", "FAMST_EWORKSPACE", "FAMST_ETIMEOUT", "FAMST_WNOTCONVERGED",
                 "FAMST_FP32", "FAMST_BF16", "FAMST_FP8_E4M3", "FAMST_EXACT", "FAMST_BORUVKA",
                 "FAMST_KRUSKAL", "FAMST_DENSE_PRIM", "FAMST_NSTATS", "FAMST_NNDESCENT",
                 "FAMST_REFINE_MAX_ROUNDS"]:
        m = re.search(r"#define\s+" + name + r"\s+\(?(-?\w+)\)?", txt)
        assert m, name
        assert int(m.group(1), 0) == getattr(L, name), name


def test_invalid_arguments_rejected_before_any_launch():
    # argument checks run on the host and never touch the device
    L = _lib()
    lib = L.load()
    sz = ctypes.c_size_t(0)
    assert lib.famst_knn_graph(None, 1, 4, None, 1, 1, 0, 0, None, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL
    assert lib.famst_knn_graph(None, 100, 4, None, 1, 100, 0, 0, None, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL
    assert lib.famst_knn_graph(None, 100, 4, None, 1, 5, 7, 0, None, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL
    assert lib.famst_knn_graph(None, 100, 4, None, 1, 5, 0, 48, None, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL
    assert lib.famst_refine(None, 100, 4, None, None, None, None, None, None, None, None, 0, 0, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL
    # the round cap, and a workspace that grows with the rounds
    mr = L.FAMST_REFINE_MAX_ROUNDS
    assert lib.famst_refine(None, 100, 4, None, None, None, None, None, None, None, None, 0, mr + 1, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL
    sizes = []
    for rounds in (1, 10, mr):
        assert lib.famst_refine(None, 100, 4, None, None, None, None, None, None, None, None, 0, rounds, None, None, None, ctypes.byref(sz), None) == L.FAMST_OK
        sizes.append(sz.value)
    assert sizes[0] < sizes[1] < sizes[2] <= (mr + 1) * 2048
    assert lib.famst_mst(None, 100, 4, None, 1, None, None, 0, None, None, None, 0, 9, None, None, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL
    offs = (ctypes.c_int64 * 3)(0, 1, 100)   # a one-point cloud
    assert lib.famst_mst_backward(None, 100, 4, offs, 2, None, None, None, None, None, ctypes.byref(sz), None) == L.FAMST_EINVAL


PEAKS_HEADER = os.path.join(ROOT, "include", "famst_peaks.h")


def test_peaks_library_exports_its_header():
    from paper_2507_14261_amd import peaks as P
    if not os.path.exists(P.PATH):
        pytest.skip("libfamst_peaks.so not built")
    txt = re.sub(r"/\*.*?\*/", "", open(PEAKS_HEADER).read(), flags=re.S)
    names = sorted(set(re.findall(r"\b(famst_[a-z_0-9]+)\s*\(", txt)))
    assert names == sorted(P.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", P.PATH], capture_output=True, text=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in names:
        assert name in syms, name


def test_knn_limits_and_workspace_queries_on_the_host():
    # k above 64, k above the requested list length, d < 1 and n >= 2^31 are
    # rejected; workspace queries (null workspace) launch nothing and grow
    # with n in every precision
    L = _lib()
    lib = L.load()
    sz = ctypes.c_size_t(0)

    def q(n, d, k, prec, kc=0):
        sz.value = 0
        r = lib.famst_knn_graph(None, ctypes.c_int64(n), d, None, 1, k, prec, kc, None, None, None, None,
                                ctypes.byref(sz), None)
        return r, sz.value

    assert q(1000, 32, 65, L.FAMST_FP32)[0] == L.FAMST_EINVAL
    assert q(1000, 32, 40, L.FAMST_BF16, 32)[0] == L.FAMST_EINVAL
    assert q(1000, 0, 5, L.FAMST_FP32)[0] == L.FAMST_EINVAL
    assert q(1 << 31, 4, 5, L.FAMST_FP32)[0] == L.FAMST_EINVAL
    for prec in (L.FAMST_FP32, L.FAMST_BF16, L.FAMST_FP8_E4M3):
        for d, k in ((32, 10), (128, 64), (960, 20)):
            sizes = []
            for n in (1000, 5000, 40000):
                r, b = q(n, d, k, prec)
                assert r == L.FAMST_OK, (prec, d, k, n, r)
                # at least the candidate lists (k' >= k entries of 8 bytes per row)
                assert b >= n * k * 8
                sizes.append(b)
            assert sizes == sorted(sizes) and sizes[0] < sizes[-1]


def test_noalloc_gradient_limits_on_the_host():
    # the allocation-free gradient validates its arguments and its scratch
    # limit before touching any device: sizes beyond the fixed array return
    # ECAPACITY with the bytes needed, null pointers EINVAL
    L = _lib()
    lib = L.load()
    need = ctypes.c_size_t(0)
    assert lib.famst_mst_backward_noalloc(None, 4_000_000, 8, None, 1, None, None, None, None,
                                          ctypes.byref(need), None) == L.FAMST_ECAPACITY
    assert need.value > L.FAMST_NOALLOC_SCRATCH_BYTES
    need.value = 0
    assert lib.famst_mst_backward_noalloc(None, 1000, 8, None, 1, None, None, None, None,
                                          ctypes.byref(need), None) == L.FAMST_EINVAL
    assert 0 < need.value <= L.FAMST_NOALLOC_SCRATCH_BYTES
    offs = (ctypes.c_int64 * 3)(0, 1, 100)   # a one-point cloud
    assert lib.famst_mst_backward_noalloc(None, 100, 4, offs, 2, None, None, None, None, None,
                                          None) == L.FAMST_EINVAL
    # the largest single cloud the array serves, from the size query
    lo, hi = 1000, 4_000_000
    while hi - lo > 1:
        mid = (lo + hi) // 2
        lib.famst_mst_backward_noalloc(None, mid, 8, None, 1, None, None, None, None, ctypes.byref(need), None)
        lo, hi = (mid, hi) if need.value <= L.FAMST_NOALLOC_SCRATCH_BYTES else (lo, mid)
    assert lo >= 1_000_000


def test_nndescent_flag_checks_on_the_host():
    # NN-Descent runs in float32 only, approximately, for k <= 32 and d <= 256
    L = _lib()
    lib = L.load()
    sz = ctypes.c_size_t(0)

    def q(d, k, prec):
        return lib.famst_knn_graph(None, 5000, d, None, 1, k, prec, 0, None, None, None, None, ctypes.byref(sz),
                                   None)

    assert q(32, 10, L.FAMST_FP32 | L.FAMST_NNDESCENT) == L.FAMST_OK and sz.value > 5000 * 32 * 8
    assert q(32, 10, L.FAMST_BF16 | L.FAMST_NNDESCENT) == L.FAMST_EINVAL
    assert q(32, 10, L.FAMST_FP32 | L.FAMST_NNDESCENT | L.FAMST_EXACT) == L.FAMST_EINVAL
    assert q(32, 33, L.FAMST_FP32 | L.FAMST_NNDESCENT) == L.FAMST_ENOTIMPL
    assert q(300, 10, L.FAMST_FP32 | L.FAMST_NNDESCENT) == L.FAMST_ENOTIMPL
