"""The walk that cuts a gathered streaming update into aligned blocks and
joins (GatherWalk in csrc/hth_kernels.h; the host counts a group's table
with it, the table kernel writes the table with it), compiled for the CPU
and checked against its definition on random cases: every full execution of
the concatenation (carried bytes, then the pieces) is covered once, in
order; a block of 8^L executions starts at a multiple of 8^L, lies inside
one piece and is maximal there (the greedy cut of the tree into aligned
subtrees, Eq. (3)); every other full execution straddles two segments and
is a join, at most one per boundary."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2104_08865_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    assert gxx, "g++ is needed to build the walk's test driver"
    exe = str(tmp_path_factory.mktemp("walk") / "walk")
    subprocess.run([gxx, "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{CSRC}",
                    os.path.join(HERE, "gather_walk_driver.cpp"), "-o", exe], check=True)
    return exe


def _cases(rng, n_cases):
    out = []
    for _ in range(n_cases):
        xb = int(rng.choice([480, 576, 672, 960, 1152, 1344]))
        L = int(rng.integers(0, 7))
        e0 = max(0, int(rng.integers(0, 4)) * 8 ** L - int(rng.integers(0, 9)))  # near an alignment
        carry = int(rng.integers(0, xb))
        lens = []
        for _ in range(int(rng.integers(1, 12))):
            kind = int(rng.integers(0, 5))
            cap = [0, 100, 2 * xb, 80 * xb, 5000 * xb][kind]
            lens.append(int(rng.integers(0, cap + 1)))
        out.append((xb, e0, carry, lens))
    return out


def _check(case, lines):
    xb, e0, carry, lens = case
    starts, at = [], carry  # each piece's offset in the concatenation
    for m in lens:
        starts.append(at)
        at += m
    total = at
    nfull = total // xb
    nxt, nj_seen = 0, 0
    for ln in lines[:-1]:
        f = ln.split()
        if f[0] == "B":
            x, L, k, off = int(f[1]), int(f[2]), int(f[3]) - 1, int(f[4])
            rel = x - e0
            assert rel == nxt, (case, ln)
            size = 8 ** L
            assert x % size == 0, (case, ln)
            lo, hi = rel * xb, (rel + size) * xb
            assert starts[k] <= lo and hi <= starts[k] + lens[k], (case, ln)  # inside piece k
            assert off == lo - starts[k], (case, ln)
            run_end = e0 + (starts[k] + lens[k]) // xb  # the piece's last full execution + 1
            assert L == 19 or x % (8 * size) != 0 or x + 8 * size > run_end, (case, ln)  # maximal
            nxt += size
        else:
            assert f[0] == "J", ln
            j, s = int(f[1]), int(f[2])
            assert j == nj_seen and s == nxt * xb, (case, ln)
            inside = any(starts[k] <= s and s + xb <= starts[k] + lens[k] for k in range(len(lens)))
            assert not inside, (case, ln)  # straddles a boundary
            nj_seen += 1
            nxt += 1
    last = lines[-1].split()
    assert last[0] == "N" and int(last[1]) == nfull == nxt, (case, lines[-1])
    assert int(last[2]) == nj_seen <= sum(1 for m in lens if m), case


def test_gather_walk_matches_definition(driver):
    cases = _cases(np.random.default_rng(61), 400)
    text = "".join(f"{xb} {e0} {c} {len(ls)} {' '.join(map(str, ls))}\n" for xb, e0, c, ls in cases)
    out = subprocess.run([driver], input=text, capture_output=True, text=True, check=True).stdout.splitlines()
    i = 0
    for case in cases:
        j = i
        while not out[j].startswith("N "):
            j += 1
        _check(case, out[i:j + 1])
        i = j + 1
    assert i == len(out)


def test_gather_walk_blocks_of_a_designed_piece(driver):
    """A piece of 2 (8^3 - 1) executions starting one past a multiple of 8^3
    is cut into 7 blocks at each of levels 0, 1, 2 going up and 7 at each
    going down: 42 blocks (the case the GPU test of group splitting uses)."""
    xb = 1344
    text = f"{xb} 0 0 2 {xb} {1022 * xb}\n"
    out = subprocess.run([driver], input=text, capture_output=True, text=True, check=True).stdout.splitlines()
    levels = [int(ln.split()[2]) for ln in out if ln.startswith("B") and ln.split()[3] == "2"]
    assert levels == [0] * 7 + [1] * 7 + [2] * 7 + [2] * 7 + [1] * 7 + [0] * 7
