"""The library's host tiling code (csrc/tiler.cpp), driven through a small
C++ program: tiles are whole links in order within their lane, cell and
weight caps; the XCD deal is a permutation that keeps each XCD's chunk
contiguous and on that XCD; ORB cuts at weighted medians."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def drv(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("tiler") / "tiler_check")
    csrc = os.path.join(ROOT, "paper_cs_0105004_amd", "csrc")
    subprocess.check_call([hipcc, "-O1", "-std=c++17",
                           "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
                           os.path.join(HERE, "helpers", "tiler_check.cpp"),
                           os.path.join(csrc, "tiler.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    return exe


def run(exe, op, text):
    out = subprocess.run([exe, op], input=text, capture_output=True,
                         text=True, check=True).stdout.split()
    return [int(v) for v in out]


def pack(exe, lanes, lens, w, T, C=-1, W=-1.0):
    n = len(lanes)
    txt = f"{T} {C} {W} {n}\n" + " ".join(map(str, lanes)) + "\n" + \
        " ".join(map(str, lens)) + "\n" + " ".join(repr(float(x)) for x in w) + "\n"
    v = run(exe, "pack", txt)
    return list(zip(v[0::2], v[1::2]))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("caps", ["lanes", "cells", "weight"])
def test_tiles_are_whole_links_within_their_caps(drv, seed, caps):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rng.integers(1, 400))
    lanes = rng.integers(1, 5, size=n)
    lens = rng.integers(6, 3000, size=n)
    w = rng.exponential(1.0, size=n) * (rng.random(n) < 0.9)
    T = int(rng.choice([1, 3, 16, 32, 64]))
    C = int(rng.choice([64, 2048, 8192])) if caps != "lanes" else -1
    W = float(w.sum() / max(1, n // 8)) if caps == "weight" else -1.0
    tiles = pack(drv, lanes, lens, w, T, C, W)
    lane0 = np.concatenate([[0], np.cumsum(lanes)])
    # the tiles partition the lanes in order, on link boundaries
    assert tiles[0][0] == 0
    assert sum(t[1] for t in tiles) == lane0[-1]
    starts = set(int(x) for x in lane0)
    l = 0
    for first, cnt in tiles:
        assert first == lane0[l] and first + cnt in starts
        links = []
        while lane0[l] < first + cnt:
            links.append(l)
            l += 1
        single = len(links) == 1
        assert single or cnt <= T
        if C > 0:
            assert single or sum(int(lanes[k]) * int(lens[k]) for k in links) <= C
        if W > 0:
            assert single or sum(w[k] for k in links) <= W + 1e-9
        # a tile stops only when the next link would break a cap
        if l < n:
            nxt = l
            over = cnt + lanes[nxt] > T
            if C > 0:
                over |= sum(int(lanes[k]) * int(lens[k]) for k in links) + \
                    int(lanes[nxt]) * int(lens[nxt]) > C
            if W > 0:
                over |= sum(w[k] for k in links) + w[nxt] > W
            assert over
    assert l == n


@pytest.mark.parametrize("n", [1, 7, 8, 9, 20, 63, 64, 65, 1000, 2703])
def test_xcd_deal_keeps_each_chunk_on_its_xcd(drv, n):
    pos = run(drv, "deal", f"{n}\n")
    assert sorted(pos) == list(range(n))
    by_xcd = [[i for p, i in enumerate(pos) if p % 8 == x] for x in range(8)]
    # each XCD's tiles are a contiguous chunk of the input, in order, and
    # the chunks follow one another
    flat = []
    for chunk in by_xcd:
        assert chunk == list(range(chunk[0], chunk[0] + len(chunk))) if chunk else True
        flat += chunk
    assert flat == list(range(n))
    sizes = [len(c) for c in by_xcd]
    assert max(sizes) - min(sizes) <= 1


@pytest.mark.parametrize("seed", range(4))
def test_orb_is_a_permutation_cut_at_the_weighted_median(drv, seed):
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    n = int(rng.integers(10, 500))
    x, y = rng.random(n), rng.random(n)
    w = rng.exponential(1.0, size=n)
    txt = f"{n}\n" + "\n".join(" ".join(repr(float(v)) for v in a)
                                for a in (x, y, w)) + "\n"
    order = run(drv, "orb", txt)
    assert sorted(order) == list(range(n))
    # the first cut is along x at the weighted median: in x order (ties by
    # index), the first part runs to the first point at which the running
    # weight reaches half the total; ORB then reorders each part along y,
    # so the final order holds that part, as a set, in front
    xs = np.array(sorted(range(n), key=lambda i: (x[i], i)))
    cum = np.cumsum(w[xs])
    cut = int(np.argmax(cum >= 0.5 * w.sum())) + 1
    cut = min(max(cut, 1), n - 1)
    assert set(order[:cut]) == set(int(i) for i in xs[:cut])
    assert x[order[:cut]].max() <= x[order[cut:]].min()
