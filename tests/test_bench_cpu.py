"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the source hash
that decides whether the measured HBM traffic still applies, the coverage of
that table, and a bounded CPU-oracle baseline sample."""
import math
import os
import re
import shutil
import subprocess
import sys

import pytest

import bench
from paper_1208_2643_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1208_2643_amd", "csrc")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _hash_of(tmp_path, edit=None):
    d = tmp_path / "paper_1208_2643_amd" / "csrc"
    d.mkdir(parents=True, exist_ok=True)
    for name in ("kernels.hpp", "tiles.hpp"):
        shutil.copy(os.path.join(CSRC, name), d / name)
    if edit:
        edit(d)
    old = bench.ROOT
    try:
        bench.ROOT = str(tmp_path)
        return bench.kernel_source_hash()
    finally:
        bench.ROOT = old


def test_source_hash_ignores_comments_not_code(tmp_path):
    base = _hash_of(tmp_path / "a")
    assert base == bench.kernel_source_hash()

    def add_comments(d):
        t = (d / "tiles.hpp").read_text()
        (d / "tiles.hpp").write_text("// a new line comment\n/* and a\n block */\n" +
                                     t.replace("\n", "  \n", 3))

    assert _hash_of(tmp_path / "b", add_comments) == base

    def change_code(d):
        t = (d / "kernels.hpp").read_text()
        (d / "kernels.hpp").write_text(t + "\nnamespace mpfc { constexpr int kProbe = 1; }\n")

    assert _hash_of(tmp_path / "c", change_code) != base


def test_measured_traffic_covers_every_tile_shape():
    with open(os.path.join(CSRC, "launch.hpp"), encoding="utf-8") as fh:
        text = fh.read()
    body = re.search(r"kShapes\[\]\s*=\s*\{(.*?)\};", text, re.S).group(1)
    labels = {f"{a}x{b}/{c}" for a, b, c in re.findall(r"\{(\d+),\s*(\d+),\s*(\d+)\}", body)}
    assert len(labels) == 7
    for kind in ("down", "up"):
        assert set(bench.MEASURED_TRAFFIC[kind]) == labels
        # each launch moves at least its compulsory bytes on the 1024^2 finest level
        floor = bench.COMPULSORY_BYTES[kind] * 1024 * 1024
        assert all(v >= floor for v in bench.MEASURED_TRAFFIC[kind].values())


def test_cpu_baseline_is_a_bounded_oracle_sample():
    params = dict(eps=0.025, beta=0.9, M=1.0, h=math.pi / 4, dt=0.05, scheme=2)
    phi0 = I.crystallites(32, 32, params["h"], count=1, radius_cells=6, seed=2)
    r = bench.cpu_baseline(params, phi0, 1e-10, 0.2)
    assert r["kind"] == "oracle" and r["unit"] == "time-steps/s"
    assert r["value"] > 0 and r["cores"] >= 1
    steps = int(re.match(r"first (\d+) step", r["sample"]).group(1))
    assert 1 <= steps <= 20
