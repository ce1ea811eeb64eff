"""Pins for the oracle's counter-based RNG (reading: Philox4x32-10, Salmon et
al. SC'11, keyed by the run seed, counter = (vehicle id, t, sub-step, 0)).

Two external anchors, neither of which shares code with the oracle:
* numpy's Philox bit generator is the 4x64-10 member of the family; the oracle
  builds its 4x32 and 4x64 generators from one template, so agreement of the
  64-bit instance with numpy pins the round structure and key schedule;
* rocRAND's host-side Philox4x32-10 engine pins the 32-bit instance itself,
  constants included.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox4x64_matches_numpy():
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(50):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2**62, size=4, dtype=np.uint64)
        g = np.random.Philox(key=key, counter=ctr)
        raw = g.random_raw(8).astype(np.uint64)
        # numpy advances its counter by one before producing each block
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        c2 = c1.copy()
        c2[0] += np.uint64(1)
        assert np.array_equal(oracle.philox4x64_10(c1, key), raw[:4])
        assert np.array_equal(oracle.philox4x64_10(c2, key), raw[4:])


@pytest.fixture(scope="module")
def rocrand_ref(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("rr") / "rocrand_philox_ref")
    src = os.path.join(HERE, "helpers", "rocrand_philox_ref.hip")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                           src, "-o", exe], stderr=subprocess.DEVNULL)
    return exe


def test_philox4x32_matches_rocrand(rocrand_ref):
    rng = np.random.Generator(np.random.PCG64(12))
    rows = []
    for _ in range(2000):
        c = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),
             int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        k = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        rows.append((c, k))
    # the counters the simulation actually uses: (id, t, 0|1, 0)
    for vid in (0, 1, 149, 199999):
        for t in (0, 1, 3599, 7199):
            for sub in (0, 1):
                rows.append(([vid, t, sub, 0], [42, 0]))
    inp = "".join("%x %x %x %x %x %x\n" % (*c, *k) for c, k in rows)
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True,
                         text=True, check=True).stdout.split("\n")
    for (c, k), line in zip(rows, out):
        ref = [int(w, 16) for w in line.split()]
        got = oracle.philox4x32_10(np.array(c, np.uint32), np.array(k, np.uint32))
        assert list(map(int, got)) == ref, (c, k)


def test_philox4x32_word0_uniform():
    # sanity, not parity: the slowdown decision u < floor(p 2^32) fires with
    # frequency p (binomial z-test)
    thr = int(0.2 * 2**32)
    n = 40000
    hits = 0
    for i in range(n):
        hits += int(oracle.philox4x32_10(np.array([i, 7, 1, 0], np.uint32),
                                         np.array([42, 0], np.uint32))[0]) < thr
    z = (hits - 0.2 * n) / np.sqrt(n * 0.2 * 0.8)
    assert abs(z) < 5
