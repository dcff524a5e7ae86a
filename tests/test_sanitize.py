"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer: the
library's tree, list, graph and coloring code (csrc/tree.cpp, built with g++
into a driver of its own, no GPU code) and the oracle's combinatorics
(oracle/comb.c), run on the point sets of the host-parity tests (1D
grid and uniform line, star curve, sphere, random 2D/3D points, noisy lines
in 4, 6 and 8 dimensions) and on forests; any sanitizer report fails the
run (-fno-sanitize-recover)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_03406_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]

CASES = [  # points, leaf, geometric?, strong?
    (workloads.grid_1d(64), 8, True, True),
    (workloads.uniform_line(1024, 1), 64, False, False),
    (workloads.star_curve(16384), 64, True, True),
    (workloads.sphere(8192, 3), 128, True, True),
    (workloads.random_points(700, 2, 11), 16, True, True),
    (workloads.random_points(900, 3, 12), 24, True, True),
    (workloads.noisy_line(3000, 4, 0.002), 32, True, True),
    (workloads.noisy_line(3000, 6, 0.002), 32, True, True),
    (workloads.noisy_line(1500, 8, 0.01), 32, True, True),
]


def _have(tool):
    return shutil.which(tool) is not None


@pytest.fixture(scope="module")
def inputs(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    args_lib, args_orc = [], []
    for i, (pts, leaf, geo, strong) in enumerate(CASES):
        f = d / ("pts%d.f64" % i)
        np.ascontiguousarray(pts, np.float64).tofile(f)
        n, dim = pts.shape
        args_lib += [str(f), str(n), str(dim), str(leaf), "0" if geo else "1", "0" if strong else "1"]
        args_orc += [str(f), str(n), str(dim), str(leaf), "0" if geo else "1", "0" if strong else "1"]
    return d, args_lib, args_orc


def _run(exe, args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([exe] + args, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=600)
    assert p.returncode == 0, p.stdout[-4000:]
    return p.stdout


@pytest.mark.skipif(not _have("g++"), reason="g++ not found")
def test_library_tree_code_under_sanitizers(inputs):
    d, args, _ = inputs
    exe = str(d / "tree_main")
    subprocess.check_call(["g++", "-std=c++17", "-pthread", "-ffp-contract=off"] + SAN +
                          ["-I", CSRC, os.path.join(CSRC, "tree.cpp"),
                           os.path.join(HERE, "tree_main.cpp"), "-o", exe])
    out = _run(exe, args)
    assert len([l for l in out.splitlines() if " levels=" in l]) == len(CASES), out


@pytest.mark.skipif(not _have("gcc"), reason="gcc not found")
def test_oracle_combinatorics_under_sanitizers(inputs):
    d, _, args = inputs
    exe = str(d / "comb_main")
    subprocess.check_call(["gcc", "-std=c99"] + SAN +
                          [os.path.join(ROOT, "oracle", "comb.c"),
                           os.path.join(HERE, "comb_main.c"), "-o", exe, "-lm"])
    out = _run(exe, args)
    assert len([l for l in out.splitlines() if " levels=" in l]) == len(CASES), out
