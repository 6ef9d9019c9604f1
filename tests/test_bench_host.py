"""Host logic of bench.py (no GPU): the one-GPU refusal, the automatic basis
rule the bench reports, and the K4 flop model its roofline object uses."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("nev,block,m", [(50, 2, 450), (16, 2, 144), (2, 2, 40), (1, 2, 40), (5, 3, 45),
                                         (4, 4, 40), (7, 4, 64)])
def test_automatic_basis_is_nine_nev_at_least_forty_rounded_to_the_block(nev, block, m):
    assert bench.auto_basis(nev, block) == m
    assert m % block == 0 and m >= 40 and m >= nev + 4 * block


def test_k4_flop_model():
    # 4 real flops per complex multiply-add over (10/3 + 4/3 + 25) m^3
    assert bench.k4_flops(1) == pytest.approx(4.0 * (29.0 + 2.0 / 3.0))
    assert bench.k4_flops(450) == pytest.approx(bench.k4_flops(1) * 450 ** 3)
    # the figure the roofline object reports for the c2 shape (8 x 450)
    assert 8 * bench.k4_flops(450) == pytest.approx(86508000000.0)
