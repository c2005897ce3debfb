"""Host logic: the factorisation plan addresses only memory it allocated.

The planner lays out every operand of the sweep (GEMM products, TSQR
segments, small dense jobs, leaf factorisations, triangular solves, the
low-rank blocks' U and V) as offsets into a few device buffers, with
dimensions that take their run-time values from the ranks.  A kernel's
access past a buffer's end would be a device memory fault, so this CPU test
builds plans for block trees of the workload shapes (uniform points with
leaf 32 and 128, the jittered grid, the line, the clustered mixture, both
admissibility forms of Appendix A and the weak one) at several per-block rank
rooms, and checks every operand's extent at the largest values its
dimensions can take (tests/plan_check.cpp).  A build that under-sizes a
buffer by one element must be caught.
"""
import math
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

import workloads
from oracle import trees

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1709_08625_amd" / "csrc"

SHAPES = [
    # n, kind, leaf, admissibility
    (2000, "uniform", 32, "min"),
    (6000, "uniform", 128, "max"),
    (3000, "uniform", 64, "weak"),
    (12000, "grid", 64, "min"),
    (12000, "line", 64, "min"),
    (16000, "mix", 128, "min"),
]
ROOMS = ["64", "32", "4", "1", "rand"]


def _locs(kind, n):
    if kind == "grid":
        return workloads.jitter_grid(n, int(math.ceil(math.sqrt(n))) + 1, seed=0)[0]
    if kind == "line":
        return workloads.line(n, seed=0)[0]
    if kind == "mix":
        return workloads.mixture(n, seed=0)[0]
    return workloads.uniform(n, seed=0)[0]


def _compile(out, extra=()):
    cmd = ["g++", "-O1", "-std=c++17", f"-I{CSRC}", *extra, str(ROOT / "tests" / "plan_check.cpp"),
           str(CSRC / "plan.cpp"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    return out


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    return _compile(tmp_path_factory.mktemp("plan_check") / "plan_check")


def _block_file(tmp_path, n, kind, leaf, rule):
    tr = trees.cluster_tree(_locs(kind, n), leaf)
    blk = trees.block_tree(tr, 2.0, rule)
    path = tmp_path / f"blocks_{kind}{n}_{leaf}_{rule}.bin"
    with open(path, "wb") as f:
        np.array([n, tr.depth, leaf, len(blk)], dtype=np.int64).tofile(f)
        np.asarray(blk, dtype=np.int64).tofile(f)
    return path


@pytest.mark.parametrize("n,kind,leaf,rule", SHAPES)
def test_plan_operands_inside_buffers(checker, tmp_path, n, kind, leaf, rule):
    path = _block_file(tmp_path, n, kind, leaf, rule)
    layout = set()
    for rooms in ROOMS:
        r = subprocess.run([str(checker), str(path), rooms], capture_output=True, text=True, timeout=300)
        print(r.stdout.strip())
        assert r.returncode == 0, r.stdout + r.stderr
        layout.add(r.stdout.split("dynamic slots ")[1].split(";")[0])
    # a rebuild at grown rooms keeps the slot numbering and the stage sequence
    assert len(layout) == 1, layout


def test_checker_sees_an_undersized_buffer(tmp_path):
    # a planted mistake: the U, V and scratch buffers one element short
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    path = _block_file(tmp_path, 2000, "uniform", 32, "min")
    for buf in (1, 2, 3):   # B_U, B_V, B_SCR
        exe = _compile(tmp_path / f"plan_check_shrink{buf}", (f"-DSHRINK={buf}",))
        r = subprocess.run([str(exe), str(path), "32"], capture_output=True, text=True, timeout=300)
        assert r.returncode == 2, r.stdout
