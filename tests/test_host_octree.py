"""The library's host-side octree code (csrc/host_octree.h, built here with
g++ into a small driver, tests/host/oct_driver.cpp) against the oracle's
adaptation pass (oracle/amr.py), on the CPU.

* One adaptation pass from a 2:1 octree (base 4, two refined spheres) and
  from a uniform base-12 grid (1,728 leaves: the 2:1 check, the balance
  sweeps and the tables run on several host threads) under seeded targets:
  the same new leaves, in the oracle's Morton order, and the same transfer
  plan (kept leaf, split path and source, merged children in child order).
* A leaf at the finest level asking for one more level is refused.
* An exception thrown inside the threaded loop reaches the caller after
  every range has run (the library turns it into an error code).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import amr
from paper_2511_17551_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GXX = shutil.which("g++")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if GXX is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("octdrv") / "oct_driver")
    subprocess.run([GXX, "-O2", "-std=c++17", "-pthread", os.path.join(HERE, "host", "oct_driver.cpp"), "-o", exe],
                   check=True, capture_output=True)
    return exe


def run(exe, text):
    return subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")


def adapt_lib(exe, base, order, target):
    lines = ["adapt", "%d %d" % (base, len(order))]
    lines += ["%d %d %d %d %d" % (c + (target[c],)) for c in order]
    out = run(exe, "\n".join(lines) + "\n")
    if out[0].startswith("error"):
        return out[0], None
    n = int(out[0])
    rows = [list(map(int, l.split())) for l in out[1:1 + n]]
    return [tuple(r[:4]) for r in rows], [r[4:] for r in rows]


def check_pass(exe, base, order, target):
    new_lib, tab = adapt_lib(exe, base, order, target)
    new, plan = amr.adapt(base, order, target)
    new_order = amr.morton_order(base, new)
    assert new_lib == [tuple(c) for c in new_order]
    eid = {c: e for e, c in enumerate(order)}
    kinds = {"keep": 0, "refine": 1, "coarsen": 2}
    for c, row in zip(new_order, tab):
        p = plan[c]
        assert row[0] == kinds[p[0]]
        if p[0] == "keep":
            assert row[3] == eid[p[1]]
        elif p[0] == "refine":
            assert row[1] == len(p[2]) and row[3] == eid[p[1]]
            assert row[2] == sum(ch << (3 * q) for q, ch in enumerate(p[2]))
        else:
            assert row[3:11] == [eid[k] for k in p[1]]
    return plan


def blob_targets(base, order, ctr, r1, r2, rng, noise=0.0):
    t = {}
    for c in order:
        L, i, j, k = c
        h = 1.0 / (base * 2 ** L)
        x = np.array([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h])
        d = np.sqrt((((x - ctr + 0.5) % 1.0 - 0.5) ** 2).sum())
        t[c] = 2 if d < r1 else (1 if d < r2 else 0)
        if noise and rng.random() < noise:
            t[c] = int(rng.integers(0, 3))
    return t


def test_adaptation_matches_the_oracle_on_a_refined_octree(driver):
    base = 4
    x, faces, mortars, level = W.octree_mesh(3, base, (0.4, 0.25), (0.45, 0.5, 0.55))
    h = 1.0 / (base * 2.0 ** level)
    lo = x.min(2)
    leaves = [(int(L), int(round(lo[0, e] / h[e])), int(round(lo[1, e] / h[e])), int(round(lo[2, e] / h[e])))
              for e, L in enumerate(level)]
    order = amr.morton_order(base, leaves)
    rng = np.random.default_rng(3)
    plan = check_pass(driver, base, order, blob_targets(base, order, np.array([0.7, 0.3, 0.5]), 0.2, 0.3, rng))
    kinds = {p[0] for p in plan.values()}
    assert kinds == {"keep", "refine", "coarsen"}


def test_adaptation_matches_the_oracle_on_many_threads(driver):
    base = 12
    order = amr.morton_order(base, [(0, i, j, k) for k in range(base) for j in range(base) for i in range(base)])
    rng = np.random.default_rng(8)
    target = blob_targets(base, order, np.array([0.3, 0.6, 0.5]), 0.12, 0.2, rng, noise=0.01)
    plan = check_pass(driver, base, order, target)
    assert sum(p[0] == "refine" for p in plan.values()) > 500


def test_refusal_beyond_the_finest_level(driver):
    out, _ = adapt_lib(driver, 1, [(12, 0, 0, 0)], {(12, 0, 0, 0): 13})
    assert out.startswith("error")


def test_exception_in_the_threaded_loop_reaches_the_caller(driver):
    assert run(driver, "throw 5000\n")[0] == "caught 1"
