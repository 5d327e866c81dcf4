"""The benchmark's command line and its host-side arithmetic (no GPU): the
one-GPU refusal, section names, and the sort's algorithmic byte count."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr and r.stdout == ""


def test_skip_names_are_checked():
    a = bench.parse(["--skip", "serve,cpu", "--no-variants"])
    assert a.skip == {"serve", "cpu", "variants"}
    with pytest.raises(SystemExit):
        bench.parse(["--skip", "serv"])


def test_defaults_are_the_headline_step():
    a = bench.parse([])
    assert (a.gpus, a.key, a.phases, a.skip) == (1, "ot64", "all", set())


@pytest.mark.parametrize("bits,per_key", [(32, 4 + 4 * 2 * 8), (64, 8 + 8 * 2 * 12)])
def test_sort_bytes_per_pair(bits, per_key):
    # one key read for the histogram pass, then a read and a write of the
    # (key, 4-byte index) pair in each of bits/8 passes
    assert bench.sort_algorithmic_bytes(1, bits) == per_key
    assert bench.sort_algorithmic_bytes(2_073_600, bits) == 2_073_600 * per_key
