"""Host-side checks of the C ABI: the library loads, exports every entry point
the header declares, and rejects bad arguments before launching anything.
Runs without a GPU (no call here reaches the HIP runtime)."""

import ctypes

import numpy as np
import os
import re

import pytest

from paper_2203_07329_amd import tik

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "tik.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tik_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = tik.lib()
    names = header_functions()
    assert "tik_sketch" in names and "tik_precond" in names and "tik_lsqr_batch" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(tik.EXPORTS) == set(names)
    assert L.tik_version() >= 100


def _probs(m=100, n=10, lda=None, dtype=tik.F64, reserved=0, A=0x1000, b=0x2000, count=1):
    arr = (tik.CProblem * count)()
    for k in range(count):
        arr[k] = tik.CProblem(m, n, lda if lda is not None else m, dtype, reserved, A, b)
    return arr


def _bytes(arr, count=1, embed=tik.SRHT, sdt=tik.F64, s=(40,)):
    sz = ctypes.c_size_t()
    sarr = (ctypes.c_int64 * count)(*s)
    rc = tik.lib().tik_sketch_bytes(arr, count, embed, sdt, sarr, ctypes.byref(sz))
    return rc, sz.value


@pytest.mark.parametrize("kw,rc", [
    (dict(m=0), tik.EINVAL),
    (dict(n=0), tik.EINVAL),
    (dict(lda=50), tik.EINVAL),
    (dict(dtype=7), tik.EINVAL),
    (dict(reserved=1), tik.EINVAL),
    (dict(A=0), tik.EINVAL),
    (dict(b=0), tik.EINVAL),
])
def test_sketch_rejects_bad_problems(kw, rc):
    got, _ = _bytes(_probs(**kw))
    assert got == rc
    assert tik.lib().tik_last_error().decode()


def test_sketch_size_limits():
    assert _bytes(_probs(), s=(0,))[0] == tik.EINVAL
    assert _bytes(_probs(), s=(101,))[0] == tik.EINVAL          # s above the long dimension
    assert _bytes(_probs(), s=(100,))[0] == tik.OK
    assert _bytes(_probs(), embed=9)[0] == tik.EINVAL
    assert _bytes(_probs(), sdt=tik.BF16)[0] == tik.EINVAL      # BF16 needs the Gaussian sketch
    # SRHT of a wide matrix and beyond 2^18 rows are outside what the library implements
    assert _bytes(_probs(m=10, n=100), s=(5,))[0] == tik.ENOTSUP
    assert _bytes(_probs(m=300000, n=10), s=(40,))[0] == tik.ENOTSUP
    # the first row count rejected: m' = 2^18 is accepted, 2^18 + 1 pads to 2^19
    assert _bytes(_probs(m=1 << 18, n=10), s=(40,))[0] == tik.OK
    assert _bytes(_probs(m=(1 << 18) + 1, n=10), s=(40,))[0] == tik.ENOTSUP
    # s above 16384 is outside the SRHT's row sampler
    assert _bytes(_probs(m=1 << 16, n=10), s=(16384,))[0] == tik.OK
    assert _bytes(_probs(m=1 << 16, n=10), s=(16385,))[0] == tik.ENOTSUP
    assert _bytes(_probs(m=10, n=100), embed=tik.GAUSS, s=(5,))[0] == tik.OK


def test_mixed_orientation_rejected():
    arr = (tik.CProblem * 2)()
    arr[0] = tik.CProblem(100, 10, 100, tik.F64, 0, 0x1000, 0x2000)
    arr[1] = tik.CProblem(10, 100, 10, tik.F64, 0, 0x1000, 0x2000)
    assert _bytes(arr, count=2, embed=tik.GAUSS, s=(20, 5))[0] == tik.EINVAL


def test_workspace_size_grows_with_problem():
    r1, a = _bytes(_probs(m=1000, n=10), s=(40,))
    r2, b = _bytes(_probs(m=1000, n=20), s=(40,))
    assert r1 == r2 == tik.OK and b > a > 40 * 10 * 8


def test_sketch_null_outputs():
    L = tik.lib()
    arr = _probs()
    sarr = (ctypes.c_int64 * 1)(40)
    assert L.tik_sketch(arr, 1, tik.SRHT, tik.F64, sarr, 0, None, 0, None, None) == tik.EINVAL
    h = ctypes.c_void_p()
    # workspace too small / NULL: caught before any launch
    assert L.tik_sketch(arr, 1, tik.SRHT, tik.F64, sarr, 0, None, 0, None,
                        ctypes.byref(h)) == tik.EWORKSPACE
    assert L.tik_sketch(arr, 1, tik.SRHT, tik.F64, sarr, 0, ctypes.c_void_p(0x1108), 1 << 30, None,
                        ctypes.byref(h)) == tik.EWORKSPACE           # misaligned


def test_precond_and_solve_null_handles():
    L = tik.lib()
    sz = ctypes.c_size_t()
    assert L.tik_precond_bytes(None, tik.ROUTE_CHOL, 4, ctypes.byref(sz)) == tik.EINVAL
    assert L.tik_lsqr_batch_bytes(_probs(), 1, None, tik.F64_BATCHED, ctypes.byref(sz)) == tik.EINVAL
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert L.tik_prof_query(b"gemm_n", ctypes.byref(ms), ctypes.byref(n)) == tik.OK
    assert n.value == 0


def test_options_roundtrip_and_rejects():
    old = tik.get_option("graph_chunk")
    try:
        tik.set_option("graph_chunk", 0)
        assert tik.get_option("graph_chunk") == 0
        tik.set_option("graph_chunk", 16)
        assert tik.get_option("graph_chunk") == 16
        for bad in (-1, 65):
            with pytest.raises(tik.TikError):
                tik.set_option("graph_chunk", bad)
        with pytest.raises(tik.TikError):
            tik.set_option("no_such_option", 1)
    finally:
        tik.set_option("graph_chunk", old)


def test_lcurve_corner_host_routine_matches_oracle():
    """tik_lcurve_corner (host C) against the oracle's corner and curvature: an
    ellipse in log space and the L-curve of a Tikhonov problem, in any order."""
    import oracle
    import workloads as W
    rng = np.random.default_rng(0)
    t = np.sort(rng.uniform(-1.2, 1.2, 31))
    cases = [(np.exp(t), np.exp(0.5 * np.sin(t)), np.exp(2.0 * np.cos(t)))]
    p = W.over_svd(m=600, n=50, N=16, lam_lo=1e-12, lam_hi=1.0)
    xn, rn = oracle.lcurve_norms(p.A, p.b, oracle.solve(p.A, p.b, p.lams))
    cases.append((p.lams, xn, rn))
    for lams, xn, rn in cases:
        for perm in (np.arange(lams.size), rng.permutation(lams.size)):
            c, curv = tik.lcurve_corner(lams[perm], xn[perm], rn[perm])
            assert c == oracle.lcurve_corner(lams[perm], xn[perm], rn[perm])
            order = np.argsort(lams[perm])
            want = oracle.lcurve_curvature(np.log(lams[perm][order]), np.log(rn[perm][order]),
                                           np.log(xn[perm][order]))
            got = curv[order]
            assert np.isnan(got[0]) and np.isnan(got[-1])
            assert np.allclose(got[1:-1], want[1:-1], rtol=1e-12, atol=1e-12 * np.nanmax(np.abs(want)))


def test_lcurve_corner_rejects_bad_input():
    lam = np.array([1e-3, 1e-2, 1e-1, 1.0])
    one = np.ones(4)
    for args in [(lam[:2], one[:2], one[:2]),                       # fewer than 3
                 (np.array([1e-3, 1e-2, 1e-2, 1.0]), one, one),    # repeated lambda
                 (-lam, one, one),                                  # non-positive lambda
                 (lam, np.array([1.0, 0.0, 1.0, 1.0]), one)]:       # zero norm
        with pytest.raises(tik.TikError):
            tik.lcurve_corner(*args)


def test_sparse_embedding_limits():
    assert _bytes(_probs(m=1000, n=10), embed=tik.SPARSE, s=(40,))[0] == tik.OK
    assert _bytes(_probs(m=10, n=100), embed=tik.SPARSE, s=(5,))[0] == tik.ENOTSUP   # wide
    assert _bytes(_probs(m=1000, n=10), embed=tik.SPARSE, sdt=tik.BF16, s=(40,))[0] == tik.EINVAL
    old = tik.get_option("sparse_nnz")
    try:
        tik.set_option("sparse_nnz", 8)
        assert _bytes(_probs(m=1000, n=10), embed=tik.SPARSE, s=(7,))[0] == tik.EINVAL   # s < zeta
        assert _bytes(_probs(m=1000, n=10), embed=tik.SPARSE, s=(8,))[0] == tik.OK
        for bad in (0, 17):
            with pytest.raises(tik.TikError):
                tik.set_option("sparse_nnz", bad)
    finally:
        tik.set_option("sparse_nnz", old)


def test_tune_table_roundtrip(tmp_path):
    """tik_tune_load / tik_tune_save: the text table survives a round trip
    (classes at log2 sizes no workload reaches, so no solve picks them up)."""
    f = tmp_path / "in.txt"
    f.write_text("# header comment\n"
                 "0 0 32 40 40 2  256 128 4096\n"
                 "\n"
                 "1 1 16 41 41 1  128 64 1024   # trailing comment\n")
    assert tik.tune_load(str(f)) == 2
    g = tmp_path / "out.txt"
    tik.tune_save(str(g))
    rows = [ln.split() for ln in g.read_text().splitlines() if ln.strip() and not ln.startswith("#")]
    assert "0 0 32 40 40 2 256 128 4096".split() in rows
    assert "1 1 16 41 41 1 128 64 1024".split() in rows
    assert tik.tune_load(str(g)) == len(rows)


@pytest.mark.parametrize("line", [
    "0 0 32 40 40 2  256 128",          # too few fields
    "0 0 3 40 40 2  256 128 4096",      # lambda slots not a power of two up to 32
    "0 0 32 40 40 2  100 128 4096",     # rows per block not 64/128/256
    "0 0 32 40 40 2  256 96 4096",      # columns per block not 64/128
    "2 0 32 40 40 2  256 128 4096",     # orientation not 0/1
    "0 0 32 40 40 3  256 128 4096",     # problem-count class not 0..2
    "0 0 32 40 40 2  256 128 10",       # too few product blocks
    "x 0 32 40 40 2  256 128 4096",     # not a number
])
def test_tune_table_rejects_malformed(tmp_path, line):
    f = tmp_path / "bad.txt"
    f.write_text("0 0 32 42 42 2  256 128 4096\n" + line + "\n")
    with pytest.raises(tik.TikError):
        tik.tune_load(str(f))
    with pytest.raises(tik.TikError):
        tik.tune_load(str(tmp_path / "missing.txt"))


def test_tune_table_rejects_extra_fields(tmp_path):
    f = tmp_path / "bad.txt"
    f.write_text("0 0 32 40 40 2  256 128 4096 7\n")
    with pytest.raises(tik.TikError):
        tik.tune_load(str(f))


def test_record_times_option_and_query_without_call():
    old = tik.get_option("record_times")
    try:
        tik.set_option("record_times", 1)
        assert tik.get_option("record_times") == 1
        with pytest.raises(tik.TikError):
            tik.set_option("record_times", 2)
    finally:
        tik.set_option("record_times", old)
    with pytest.raises(tik.TikError):
        tik.lsqr_times(3, 7)       # no call of that size was recorded on this thread


def test_srht_cols_option_and_workspace():
    """The column-resident SRHT needs no transform scratch: with it switched off
    the same sketch asks for the column-chunk scratch of the two-pass form."""
    old = tik.get_option("srht_cols")
    try:
        probs = _probs(m=20000, n=256)
        tik.set_option("srht_cols", 1)
        rc1, b1 = _bytes(probs, embed=tik.SRHT, s=(300,))
        tik.set_option("srht_cols", 0)
        assert tik.get_option("srht_cols") == 0
        rc0, b0 = _bytes(probs, embed=tik.SRHT, s=(300,))
        assert rc0 == rc1 == tik.OK
        assert b0 > b1
        with pytest.raises(tik.TikError):
            tik.set_option("srht_cols", 2)
    finally:
        tik.set_option("srht_cols", old)


def test_gemm_n_tail_option():
    old = tik.get_option("gemm_n_tail")
    try:
        tik.set_option("gemm_n_tail", 0)
        assert tik.get_option("gemm_n_tail") == 0
        with pytest.raises(tik.TikError):
            tik.set_option("gemm_n_tail", 2)
    finally:
        tik.set_option("gemm_n_tail", old)
    assert tik.get_option("gemm_n_tail") == old


def test_f16_sketch_rejects_wide_and_non_gaussian():
    rc, _ = _bytes(_probs(m=10, n=100), sdt=tik.F16, embed=tik.GAUSS, s=(40,))
    assert rc == tik.ENOTSUP                    # wide: the FP16 sketch is for tall problems
    rc, _ = _bytes(_probs(m=100, n=10), sdt=tik.F16, embed=tik.SRHT, s=(40,))
    assert rc == tik.EINVAL                     # 16-bit sketches are Gaussian
    rc, nb = _bytes(_probs(m=100, n=10), sdt=tik.F16, embed=tik.GAUSS, s=(40,))
    assert rc == tik.OK and nb > 0
