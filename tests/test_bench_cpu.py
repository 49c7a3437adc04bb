"""The benchmark's host-side contract on a machine without a GPU: argument
defaults, the refusal of more than one GPU, the rocprofv3 summaries it
turns into the committed profiles (kernel statistics and HBM counters
scaled by a calibration copy), and the source-hash check that drops a
stored traffic figure once its kernel's source has changed."""
import csv
import io
import os
import subprocess
import sys
from contextlib import redirect_stdout

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_defaults(monkeypatch):
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert a.gpus == 1 and a.steps >= 1 and a.warmup >= 0 and a.workload == "graph"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_stats(tmp_path):
    _write_csv(str(tmp_path / "x" / "prof_kernel_stats.csv"),
               ["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs"],
               [["(anonymous namespace)::k_a(int)", 4, 4000, 1000, 900, 1100],
                ["k_b(int)", 1, 12000, 12000, 12000, 12000]])
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.summarize_stats(str(tmp_path))
    lines = buf.getvalue().splitlines()
    assert lines[1].startswith("k_b(int)") and lines[2].startswith("k_a(int)")
    assert "75.00" in lines[1] and "1.0" in lines[2]


def test_summarize_pmc_scales_by_the_calibration_copy(tmp_path):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy of 1 MiB reads 512 KiB of FETCH_SIZE and writes 1024 KiB:
    # factors 2 and 1
    _write_csv(str(tmp_path / "f" / "p_counter_collection.csv"), hdr,
               [["void at::native::neg_kernel", "FETCH_SIZE", 512.0],
                ["k_tridiag<true, 512>(int)", "FETCH_SIZE", 100.0],
                ["k_tridiag<true, 512>(int)", "FETCH_SIZE", 300.0]])
    _write_csv(str(tmp_path / "w" / "p_counter_collection.csv"), hdr,
               [["void at::native::neg_kernel", "WRITE_SIZE", 1024.0],
                ["k_tridiag<true, 512>(int)", "WRITE_SIZE", 50.0],
                ["k_tridiag<true, 512>(int)", "WRITE_SIZE", 50.0]])
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), "tridiag", 1, "N=8")
    kv = dict(l.split(": ", 1) for l in buf.getvalue().splitlines() if not l.startswith("#"))
    assert float(kv["fetch_factor"]) == pytest.approx(2.0)
    assert float(kv["fetch_bytes_per_launch"]) == pytest.approx(200.0 * 1024 * 2)
    assert float(kv["write_bytes_per_launch"]) == pytest.approx(50.0 * 1024)
    assert kv["sources_sha256"] == bench.sources_sha(bench.PHASE_KERNEL["tridiag"][1])
    assert kv["size"] == "N=8"


def test_stored_traffic_needs_the_current_sources_and_size(tmp_path, monkeypatch):
    files = bench.PHASE_KERNEL["tridiag"][1]
    good = tmp_path / "pmc_k_tridiag_case.txt"
    good.write_text(f"size: N=1064\nsources_sha256: {bench.sources_sha(files)}\n"
                    "traffic_bytes_per_launch: 1234\n")
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.stored_traffic("tridiag", "N=1064") == 1234.0
    # counters taken at another size do not describe this launch
    assert bench.stored_traffic("tridiag", "N=128") is None
    good.write_text("size: N=1064\nsources_sha256: 0\ntraffic_bytes_per_launch: 1234\n")
    assert bench.stored_traffic("tridiag", "N=1064") is None
    assert bench.stored_traffic("no-such-phase", "N=1064") is None


def test_phase_work_and_roofline_candidates():
    # Cholesky of the s x s Gram: s^3 / 3 flops; the append form's M is
    # assembled without a product, the weight form's is a GEMM
    assert bench.phase_work("cholesky", 1064, 1000, 64, 0, 0)[:2] == ("alu", 1000 ** 3 / 3.0)
    assert bench.phase_work("kkt_gemm", 1064, 1000, 64, 0, 0, "append")[0] is None
    assert bench.phase_work("kkt_gemm", 96, 32, 64, 0, 0, "weights")[1] == 2.0 * 96 ** 3
    assert bench.phase_work("subspace_iter", 1064, 1000, 64, 0, 0, "append", None)[0] is None
    assert bench.phase_work("subspace_iter", 1064, 1000, 64, 0, 0, "append", 5e9)[1] == 5e9
    # multi-kernel phases are reported as rates, never as the roofline kernel
    assert "subspace_iter" not in bench.SINGLE_KERNEL_PHASES
    assert "trsm" not in bench.SINGLE_KERNEL_PHASES
    assert set(bench.SINGLE_KERNEL_PHASES) <= set(bench.PHASE_KERNEL)
    assert bench.phase_size("cholesky", 1064, 1000, 64) == "s=1000"
    assert bench.phase_size("tridiag", 1064, 1000, 64) == "N=1064"


def test_head_rows_cuts_every_sparse_matrix():
    from synth.sparse import bernoulli_uniform
    rng = np.random.default_rng(3)
    D, Em = bernoulli_uniform(40, 30, 0.2, rng), bernoulli_uniform(40, 50, 0.2, rng)
    kind, D2, E2 = bench.head_rows(("weights", D, Em), 7)
    assert kind == "weights" and D2.rows == 7 and E2.rows == 7
    np.testing.assert_array_equal(D2.to_dense(), D.to_dense()[:7])
    np.testing.assert_array_equal(E2.to_dense(), Em.to_dense()[:7])
    assert bench.head_rows(("rows", D), 100)[1].rows == 40


def test_summarize_counters_means_and_mfma_flops(tmp_path):
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    _write_csv(str(tmp_path / "c" / "p_counter_collection.csv"), hdr,
               [["(anonymous namespace)::k_gram_lowp<2>(long)", "SQ_INSTS_VALU_MFMA_MOPS_BF16", 1000.0],
                ["(anonymous namespace)::k_gram_lowp<2>(long)", "GRBM_GUI_ACTIVE", 10.0],
                ["(anonymous namespace)::k_gram_lowp<2>(long)", "SQ_INSTS_VALU_MFMA_MOPS_BF16", 3000.0],
                ["(anonymous namespace)::k_gram_lowp<2>(long)", "GRBM_GUI_ACTIVE", 30.0],
                ["k_other(int)", "GRBM_GUI_ACTIVE", 5.0]])
    buf = io.StringIO()
    with redirect_stdout(buf):
        bench.summarize_counters(str(tmp_path))
    lines = buf.getvalue().splitlines()
    assert len(lines) == 2 and lines[0].startswith("k_gram_lowp<2>(long) | dispatches 2")
    assert "GRBM_GUI_ACTIVE=20 " in lines[0] and "SQ_INSTS_VALU_MFMA_MOPS_BF16=2000" in lines[0]
    assert "mfma_flops_bf16=1.024e+06" in lines[0]
    assert "mfma_flops" not in lines[1]


def test_bounded_oracle_samples_time_both_methods():
    from synth import synthetic_factors
    from synth.sparse import bernoulli_uniform
    rng = np.random.default_rng(4)
    U, s, V = synthetic_factors(60, 40, 8, rng)
    up = ("rows", bernoulli_uniform(20, 40, 0.2, rng))
    out = bench.bounded_oracle_samples(dict(U=U, s=s, V=V), up, 6, 4)
    assert [o["cores"] for o in out] == [4, 1]
    assert all(o["value"] > 0 and o["kind"] == "oracle" and "first 6 rows" in o["sample"]
               for o in out)
