"""Pins of the oracle's random-number layer against things outside it:
the published Philox4x32-10 known-answer vectors, PyTorch's own independent
Philox engine, and the uniformity of the random pairing permutation."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answer_vectors():
    for ctr, key, out in _kat():
        assert list(oracle.philox(ctr, key)) == out


def _torch_ref_binary(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    import torch  # only for its include directory
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("PyTorch Philox header not found")
    exe = str(tmp_path_factory.mktemp("philox") / "ptr")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-I" + inc, "-o", exe,
                           os.path.join(HERE, "philox_torch_ref.cpp")])
    return exe


def test_philox_matches_pytorch_engine(tmp_path_factory):
    exe = _torch_ref_binary(tmp_path_factory)
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(200):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, size=4)]
        cases.append((seed, ctr))
    cases.append((0x2407191510000003, [5, 17, 3, (2 << 8) | 1]))
    inp = "".join("%d %d %d %d %d\n" % (s, *c) for s, c in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    for (seed, ctr), line in zip(cases, out):
        ref = [int(x) for x in line.split()]
        mine = list(oracle.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32]))
        assert mine == ref


def test_shuffle_is_bijection():
    for n in (0, 1, 2, 3, 5, 17, 64, 257, 1000):
        p = oracle.shuffle(n, cell=11, seed=99, step=4, coll=1, slot=0)
        assert sorted(p.tolist()) == list(range(n))


def test_shuffle_positions_uniform():
    """Each particle lands in each position with probability 1/n (chi-square
    over many independent (cell, step) streams)."""
    n = 5
    trials = 6000
    counts = np.zeros((n, n))
    for t in range(trials):
        p = oracle.shuffle(n, cell=t % 97, seed=1234, step=t // 97, coll=0, slot=0)
        counts[p, np.arange(n)] += 1  # particle p[q] at position q
    expected = trials / n
    chi2 = ((counts - expected) ** 2 / expected).sum()
    # 16 degrees of freedom (25 cells, row and column sums fixed);
    # P(chi2 > 45) ~ 1e-4
    assert chi2 < 45.0, chi2


def test_shuffle_streams_differ_by_collision_slot_step():
    a = oracle.shuffle(50, 3, 1, 0, 0, 0)
    assert not np.array_equal(a, oracle.shuffle(50, 3, 1, 0, 1, 0))
    assert not np.array_equal(a, oracle.shuffle(50, 3, 1, 0, 0, 1))
    assert not np.array_equal(a, oracle.shuffle(50, 3, 1, 1, 0, 0))
    assert not np.array_equal(a, oracle.shuffle(50, 4, 1, 0, 0, 0))
    assert np.array_equal(a, oracle.shuffle(50, 3, 1, 0, 0, 0))
