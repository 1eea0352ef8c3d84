"""Host logic of the benchmark (no GPU): the algorithmic bytes per launch
against the closed form for the 6717-bus, 96-period LP, the validity rule of
the committed counter records, and the one-GPU limit."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2512_06715_amd import ucgen  # noqa: E402


def sizes():
    z = ucgen.size_formulas(6717, 1100, 9000, 96)
    return z["m"], z["n"], z["nnz"]


def test_sizes_of_the_paper_scale_lp():
    assert sizes() == (2034728, 3220992, 7188260)


def test_kernel_bytes_closed_form():
    """Written out term by term for the attempt kernels: structure (16-bit
    form: 2 bytes per row end, 8 per 256-row tile, 2 per index; 32-bit CSR:
    4 (r + 1) + 4 nnz), values, the gathered vector, the streamed vectors and
    the fold of the running sum."""
    m, n, nnz = sizes()
    for vb in (4, 8):
        s_m = 2 * m + 8 * ((m + 255) // 256) + 2 * nnz
        s_n = 2 * n + 8 * ((n + 255) // 256) + 2 * nnz
        dual = s_m + vb * nnz + vb * n + (3 * vb + 1) * m + 2 * vb * m + 2 * vb * m
        primal = s_n + vb * nnz + vb * m + 4 * vb * n + vb * n + 2 * vb * n
        assert bench.kernel_bytes("dual", m, n, nnz, vb) == dual
        assert bench.kernel_bytes("primal", m, n, nnz, vb) == primal
        assert bench.kernel_bytes("primal", m, n, nnz, vb, compact=False) == \
            primal - s_n + 4 * (n + 1) + 4 * nnz
    # the per-launch figures the measurements quote (MB)
    assert round(bench.kernel_bytes("primal", m, n, nnz, 4) / 1e6, 1) == 148.0
    assert round(bench.kernel_bytes("dual", m, n, nnz, 4) / 1e6, 1) == 119.2
    assert round(bench.kernel_bytes("primal", m, n, nnz, 8) / 1e6, 1) == 275.1
    assert round(bench.kernel_bytes("dual", m, n, nnz, 8) / 1e6, 1) == 217.8
    with pytest.raises(ValueError):
        bench.kernel_bytes("control", m, n, nnz, 4)


def test_unit_bytes_match_the_scope_table():
    """The per-unit figures of the scope table on the paper-scale LP: fused
    primal step 270 / 156 MB, fused dual step 202 / 119 MB, full PDLP attempt
    16 nnz + 40 n + 36 m (FP32) and 24 nnz + 76 n + 68 m (FP64)."""
    m, n, nnz = sizes()
    assert round(bench.unit_bytes("primal", m, n, nnz, 8) / 1e6) == 270
    assert round(bench.unit_bytes("primal", m, n, nnz, 4) / 1e6) == 156
    assert round(bench.unit_bytes("dual", m, n, nnz, 8) / 1e6) == 202
    assert round(bench.unit_bytes("dual", m, n, nnz, 4) / 1e6) == 119
    assert bench.unit_bytes("attempt", m, n, nnz, 4) == 16 * nnz + 40 * n + 36 * m
    assert bench.unit_bytes("attempt", m, n, nnz, 8) == 24 * nnz + 76 * n + 68 * m
    # the merge-path SpMV alone, FP32: 8 nnz + 4 (m + 1) + 4 n + 4 m
    assert bench.merge_spmv_bytes(m, n, nnz, 4) == 8 * nnz + 4 * (m + 1) + 4 * n + 4 * m


def test_traffic_records_follow_the_source(tmp_path, monkeypatch):
    """A counter record counts only for the kernel source it was taken on
    (its hash); for any other source the bench reports no traffic."""
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = dict(kernel="k_primal", bytes_per_launch=123, source_hash="0" * 16)
    (prof / "traffic_k_primal_w_mixed.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "f" * 16)
    assert bench.load_traffic("k_primal", "w", "mixed") is None
    rec["valid_for"] = ["f" * 16]   # a note naming another source does not count
    (prof / "traffic_k_primal_w_mixed.json").write_text(json.dumps(rec))
    assert bench.load_traffic("k_primal", "w", "mixed") is None
    rec["source_hash"] = "f" * 16
    (prof / "traffic_k_primal_w_mixed.json").write_text(json.dumps(rec))
    assert bench.load_traffic("k_primal", "w", "mixed") == 123
    assert bench.load_traffic("k_dual", "w", "mixed") is None   # no record


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)


def test_oracle_run_record_lookup(tmp_path, monkeypatch):
    """The bench finds the oracle's own solve by workload and tolerance."""
    (tmp_path / "tests" / "golden").mkdir(parents=True)
    rec = {"uc6717_t96@0.0001": {"info": {"pobj": 1.0, "attempts": 5}, "kkt": {"rel_kkt": 1e-4}}}
    (tmp_path / "tests" / "golden" / "oracle_runs.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.oracle_run("uc6717_t96", 1e-4)["info"]["attempts"] == 5
    assert bench.oracle_run("uc6717_t96", 1e-6) is None
    assert bench.oracle_run("uc1000_t48", 1e-4) is None
