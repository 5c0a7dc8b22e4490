"""Host-side checks of the benchmark driver: the one-GPU refusal, the algorithmic byte
count of the dominant kernel, and that the committed counter traffic is reported only for
the exact library sources it was measured on."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_sweep_bytes_of_the_2d_workload():
    # 1,010,113 nodes, 9,021,865 stored 1x1 blocks, 16-bit column offsets: FP64 values and
    # 2-byte indices per block, int32 row pointers, x, b, x_out and the diagonal inverse
    n, nnzb = 1010113, 9021865
    expect = nnzb * (8 + 2) + 4 * (n + 1) + 3 * n * 8 + n * 8
    assert bench.sweep_bytes(n, 1, nnzb, 2) == expect == 126582722
    assert bench.sweep_bytes(n, 1, nnzb, 4) == expect + 2 * nnzb
    # block systems: b*b values per block
    assert bench.sweep_bytes(10, 3, 100, 2) == 100 * (72 + 2) + 44 + 3 * 30 * 8 + 10 * 72
    # dictionary form: a 2-byte block index per stored block instead of its values, the
    # distinct blocks once
    assert bench.dict_sweep_bytes(10, 3, 100, 2, 7) == 100 * (2 + 2) + 7 * 72 + 44 + 3 * 30 * 8 + 10 * 72


def test_counter_traffic_tracks_the_sources(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2405_05047_amd", "csrc")
    dst = tmp_path / "paper_2405_05047_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in os.listdir(src):
        if name.endswith((".hip", ".h")):
            shutil.copy(os.path.join(src, name), dst / name)
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(dst)):
        h.update((dst / name).read_bytes())
    (tmp_path / "profiles").mkdir()
    table = {"wl": {"traffic_bytes_per_launch": 12345, "sources_sha256": h.hexdigest()}}
    (tmp_path / "profiles" / "k_sweep_fp64_counters.json").write_text(json.dumps(table))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("wl") == 12345
    assert bench.counter_traffic("other") is None
    any_src = sorted(p for p in os.listdir(dst) if p.endswith(".hip"))[0]
    with open(dst / any_src, "a") as f:
        f.write("\n// changed\n")
    assert bench.counter_traffic("wl") is None
