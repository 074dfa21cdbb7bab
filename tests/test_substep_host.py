"""Host logic of adaptive load stepping (csrc/substep.hpp), compiled with g++ and driven by
scripted outcomes: the fractions it walks, cutting on failure, growing on fast
convergence, the cut budget, and landing exactly on the end of the increment."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("substep") / "substep_driver")
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", os.path.join(HERE, "native", "substep_driver.cpp"),
                    "-o", exe], check=True)
    return exe


def run(exe, *args):
    out = subprocess.run([exe] + [str(a) for a in args], check=True, capture_output=True, text=True).stdout
    return [line.split() for line in out.strip().splitlines()]


def test_whole_increment_when_nothing_fails(driver):
    lines = run(driver, 4, 2, 1.0, 3)
    assert lines[0] == ["start", "0", "1", "0"]
    assert lines[1][0] == "accept" and float(lines[1][1]) == 1.0 and lines[1][4] == "1"


def test_cut_then_finish(driver):
    lines = run(driver, 4, 2, 1.0, "f", 5, 5)
    assert lines[1][0] == "reject" and float(lines[1][3]) == 0.5 and lines[1][4] == "1"
    assert float(lines[2][1]) == 0.5 and float(lines[2][2]) == 0.5
    # slow convergence keeps the length; the second half lands exactly on 1
    assert float(lines[3][1]) == 1.0 and lines[3][4] == "1"


def test_two_cuts_then_growth(driver):
    lines = run(driver, 4, 2, 1.0, "f", "f", 1, 1, 9)
    ends = [float(l[1]) for l in lines if l[0] == "accept"]
    assert ends == [0.25, 0.75, 1.0]  # 0.25, then doubled to 0.5, then the rest (0.25)
    assert lines[-2][4] == "1"


def test_cut_budget(driver):
    lines = run(driver, 2, 2, 1.0, "f", "f", "f")
    rejects = [l for l in lines if l[0] == "reject"]
    assert [l[5] for l in rejects] == ["1", "1", "0"]
    assert rejects[-1][4] == "2"


def test_start_fraction_and_remainder(driver):
    lines = run(driver, 4, 0, 0.3, 9, 9, 9, 9)
    ends = [float(l[1]) for l in lines if l[0] == "accept"]
    assert ends[-1] == 1.0 and len(ends) == 4
    assert abs(ends[0] - 0.3) < 1e-15 and abs(ends[2] - 0.9) < 1e-15


def test_lerp_lands_exactly(driver):
    last = run(driver, 0, 0, 1.0)[-1]
    assert last[0] == "lerp" and last[1] == "1"
    a4, b4 = 0.1 * 4 + 0.3, 1.0 / 7.0
    assert float(last[2]) == a4 + 0.25 * (b4 - a4)
