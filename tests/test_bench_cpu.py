"""Host-side checks of bench.py's roofline bookkeeping (no GPU).

`measured_traffic` turns a committed rocprofv3 counter record (profiles/traffic.json) into the
HBM bytes of one launch of a product family, and refuses a record whose kernel sources changed
since the counters were taken.  Exercised here on a synthetic record in a temporary tree."""
import hashlib
import json

import bench


def _tree(tmp_path, bpd, src_text=b"kernel source\n"):
    src = tmp_path / "k.hip"
    src.write_bytes(src_text)
    (tmp_path / "profiles").mkdir()
    rec = {"sources": ["k.hip"], "source_sha256": hashlib.sha256(src_text).hexdigest(),
           "bytes_per_dispatch": bpd}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({"wl": rec}))
    return src


def test_gemm_n_single_launch(tmp_path, monkeypatch):
    """Every row block in one EPI 0 launch: its bytes alone."""
    _tree(tmp_path, {"void tik::k_gemm_n_mfma<double, double, 32, 0, 2>(tik::DevProb const*)": 3.3e9,
                     "tik::k_vec_bot(tik::DevProb const*)": 1.0e6})
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("wl", "gemm_n") == int(3.3e9)


def test_gemm_n_split_tail(tmp_path, monkeypatch):
    """Row blocks and the last round's column pieces in one EPI 3 launch, plus the pieces' sum
    (k_gemm_n_tail_fin of the same compute type): the family's launch is both kernels."""
    _tree(tmp_path, {
        "void tik::k_gemm_n_mfma<double, double, 32, 3, 2>(tik::DevProb const*)": 3.35e9,
        "void tik::(anonymous namespace)::k_gemm_n_tail_fin<double>(tik::DevProb const*)": 3.0e7,
        "void tik::(anonymous namespace)::k_gemm_n_tail_fin<float>(tik::DevProb const*)": 9.9e9,
        "void tik::k_gemm_t_mfma<double, double, double, 32, 64>(tik::DevProb const*)": 3.31e9})
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("wl", "gemm_n") == int(3.35e9 + 3.0e7)
    assert bench.measured_traffic("wl", "gemm_t") == int(3.31e9)


def test_stale_record_is_refused(tmp_path, monkeypatch):
    """A record taken on other kernel sources gives no traffic figure."""
    src = _tree(tmp_path, {"void tik::k_gemm_t_mfma<double, double, double, 32, 64>(x)": 3.31e9})
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("wl", "gemm_t") == int(3.31e9)
    src.write_bytes(b"kernel source, edited\n")
    assert bench.measured_traffic("wl", "gemm_t") is None
    assert bench.measured_traffic("other", "gemm_t") is None
