"""Host-side parts of bench.py that need no GPU: the one-GPU refusal, the
algorithmic byte count, and the lookup of committed HBM traffic figures
(only for the kernel source they were measured on)."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_alg_bytes_by_hand():
    # plain: 12 per nonzero, 8 per row, 4 per level pointer, 16 per row and right-hand side
    assert bench.alg_bytes(10, 25, 4, 3) == 12 * 25 + 8 * 10 + 4 * 5 + 16 * 10 * 3
    # rewritten: T's nonzeros with L''s, 12 per row (row pointers of both and the row map)
    assert bench.alg_bytes(10, 25, 4, 3, nnz_t=7, rewritten=True) == 12 * 32 + 12 * 10 + 4 * 5 + 16 * 10 * 3


def test_traffic_lookup_follows_the_source(tmp_path, monkeypatch):
    """A committed figure is returned for the kernel source it was measured on
    and withheld (None) once the source hash differs."""
    kernel = "k_wide_run"
    good = {"bytes_per_launch": 123.0, "source_hash": bench.source_hash(kernel)}
    stale = dict(good, source_hash="0" * 16)
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for entry, want in ((good, 123.0), (stale, None)):
        (prof / "traffic.json").write_text(json.dumps({f"{kernel}:config4_learned": entry}))
        monkeypatch.setattr(bench, "source_hash", lambda k, h=good["source_hash"]: h)
        assert bench.load_traffic(kernel, "config4_learned") == want
    assert bench.load_traffic(kernel, "config9_none") is None
