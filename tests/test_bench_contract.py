"""The benchmark's command-line contract and roofline bookkeeping, on the
CPU (no GPU is touched): one GPU only, and the traffic figure read from the
committed counter summary only when it belongs to the current kernel
sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + list(args), cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    p = run_bench("--gpus", "2")
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_help_lists_the_contract_flags():
    p = run_bench("--help")
    assert p.returncode == 0
    for flag in ("--gpus", "--steps", "--warmup", "--full-json", "--heff-launch"):
        assert flag in p.stdout


def test_algorithmic_bytes_of_the_pair_gemm():
    # both packed operands once (S bytes per element), one exponent per row
    # of A and per column of B, C written once in FP64
    n, S = 8192, 7
    assert bench.pair_bytes(n, S) == 2 * S * n * n + 8 * n + 8 * n * n
    assert bench.pair_bytes(n, S) / 2 ** 30 == pytest.approx(1.375, abs=1e-3)


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    text = open(bench.COUNTERS_FILE).read()
    rows = [l.split() for l in text.splitlines() if l and l[0].isdigit()]
    assert rows, "the counter summary holds no rows"
    n, S, G, v = (int(x) for x in rows[0][:4])
    fetch, write = float(rows[0][5]), float(rows[0][6])
    meta = dict(l.split(" = ") for l in text.splitlines() if " = " in l and not l.startswith("#"))
    ff, wf = float(meta["fetch_factor"]), float(meta["write_factor"])
    # a summary taken on the current sources gives the scaled counters
    cur = tmp_path / "cur.txt"
    cur.write_text(text.replace("source_sha256 = " + meta["source_sha256"],
                                "source_sha256 = " + bench.pair_source_hash()))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(cur))
    assert bench.pair_traffic(n, S, G, v) == pytest.approx(1024 * (ff * fetch + wf * write), rel=1e-12)
    assert bench.pair_traffic(n, S, G, 99) is None
    # one taken on other sources gives nothing
    old = tmp_path / "old.txt"
    old.write_text(text.replace("source_sha256 = " + meta["source_sha256"], "source_sha256 = " + "0" * 64))
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(old))
    assert bench.pair_traffic(n, S, G, v) is None
