"""Host logic of the Gram pass: the work plan (chunks of large pairs, groups
of four small pairs, longest first, partial slots) checked for exact
coverage of every match and consistent partial slots, on edge-case and
random pair sizes.  Builds a small C++ checker with g++ (CPU only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_04612_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan") / "gram_plan_check")
    subprocess.run([gxx, "-O2", "-std=c++17", f"-I{CSRC}", os.path.join(ROOT, "tests", "gram_plan_check.cpp"),
                    "-o", exe], check=True, capture_output=True)
    return exe


def _run(exe, sizes):
    inp = f"{len(sizes)} " + " ".join(str(int(s)) for s in sizes)
    r = subprocess.run([exe], input=inp, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


EDGE = [0, 1, 15, 16, 17, 255, 256, 257, 1023, 1024, 1025, 2047, 2048, 2049, 4096, 4097, 20000, 0, 1, 1, 1, 1,
        16, 16, 16, 16, 17, 17, 33, 240, 241]


@pytest.mark.parametrize("sizes", [
    [],
    [0, 0, 0],
    [5],
    [300],
    [1 << 17],
    EDGE,
    EDGE[::-1],
], ids=["none", "all-empty", "one-small", "one-big", "one-huge", "edges", "edges-reversed"])
def test_plan_invariants_edge_cases(checker, sizes):
    out = _run(checker, sizes)
    assert out.count("OK") == 2


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_invariants_power_law_sizes(checker, seed):
    rng = np.random.default_rng(seed)
    # density ~ k^-1.45 on [20, 20000], plus empty and tiny pairs
    u = rng.random(3000)
    a = 1.0 - 1.45
    k = ((20 ** a) + u * ((20000 ** a) - (20 ** a))) ** (1.0 / a)
    k = np.floor(k).astype(int)
    k[rng.random(3000) < 0.05] = 0
    k[rng.random(3000) < 0.05] = 1
    out = _run(checker, k)
    assert out.count("OK") == 2
