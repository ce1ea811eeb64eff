"""The lane-change sub-step's bit formulation, as the GPU pass computes it,
against the per-cell formulation of rule R6, on random links.

The bit formulation keeps one occupancy bit per cell (lanes padded to
32-bit words), reads the gaps ahead and behind from a 32-cell window with a
count of trailing or leading zeros, marks movers in right/left masks,
resolves two movers into one cell word-wise (the one from the lower lane
moves), and places every vehicle in its new lane at the popcount of the
occupied cells ahead of it.  The cell formulation scans cells one by one
and then moves the deciders in cell order.  Both must give the same
decisions, conflicts, move counts and lead-first lane contents, for links
of 2-4 lanes, every vmax up to 7 and every density."""
import random

import pytest

M32 = 0xFFFFFFFF


# ---- per-cell formulation (lat[lane][cell] = vehicle id or -1) -----------

def cell_ahead(lat, length, m, x, vmax):
    n, c = 0, x + 1
    while c < length and n < vmax and lat[m][c] < 0:
        n, c = n + 1, c + 1
    return n


def cell_behind(lat, m, x, vmax):
    n, c = 0, x - 1
    while n < vmax and not (c >= 0 and lat[m][c] >= 0):
        n, c = n + 1, c - 1
    return n


def decide(occupied, ahead, behind, lanes, k, x, v, lo, hi, draw_ok, vmax,
           length, desp):
    """Rule R6 on abstract look-ups: the target lane or -1."""
    if k < lo or k > hi:  # mandatory, toward the turn lanes
        m = k + 1 if k < lo else k - 1
        need = min(vmax, (length - 1 - x) // desp)
        return m if not occupied(m, x) and behind(m, x) >= need else -1
    own = ahead(k, x)
    if own >= min(v + 1, vmax):
        return -1
    best, best_a = -1, -1
    for m in (k - 1, k + 1):
        if m < 0 or m >= lanes or m < lo or m > hi or occupied(m, x):
            continue
        a = ahead(m, x)
        if a <= own or behind(m, x) < vmax:
            continue
        if a > best_a:
            best, best_a = m, a
    return best if best >= 0 and draw_ok else -1


# ---- bit formulation ------------------------------------------------------

def window(words, wpl, c):
    """Bits of cells [c, c+32) of a lane (cell c at bit 0; outside: 0)."""
    q, sh = c >> 5, c & 31
    lo = words[q] if 0 <= q < wpl else 0
    hi = words[q + 1] if 0 <= q + 1 < wpl else 0
    return lo if sh == 0 else ((lo >> sh) | (hi << (32 - sh))) & M32


def ctz(v):
    return (v & -v).bit_length() - 1


def bit_ahead(words, wpl, length, x, vmax):
    lim = min(vmax, length - 1 - x)
    return ctz(window(words, wpl, x + 1) | (1 << lim))


def bit_behind(words, wpl, x, vmax):
    b = window(words, wpl, x - vmax) & ((1 << vmax) - 1)
    return vmax if b == 0 else vmax - 1 - (b.bit_length() - 1)


def popcount(v):
    return bin(v).count("1")


# ---- one random link ------------------------------------------------------

def random_link(rng):
    lanes = rng.randint(2, 4)
    length = rng.choice([rng.randint(6, 40), rng.randint(30, 130),
                         rng.randint(500, 1100)])
    vmax, desp, dens = rng.randint(1, 7), rng.randint(1, 5), rng.random()
    veh, vid = {}, 0
    for k in range(lanes):
        for x in range(length):
            if rng.random() < dens:
                lo = rng.randint(0, lanes - 1)
                hi = rng.randint(lo, lanes - 1)
                veh[(k, x)] = (rng.randint(0, vmax), lo, hi,
                               rng.random() < 0.7, vid)
                vid += 1
    return lanes, length, vmax, desp, veh


def by_cells(lanes, length, vmax, desp, veh):
    lat = [[-1] * length for _ in range(lanes)]
    for (k, x), r in veh.items():
        lat[k][x] = r[4]
    dec = [[-1] * length for _ in range(lanes)]
    for (k, x), (v, lo, hi, ok, _) in veh.items():
        dec[k][x] = decide(lambda m, c: lat[m][c] >= 0,
                           lambda m, c: cell_ahead(lat, length, m, c, vmax),
                           lambda m, c: cell_behind(lat, m, c, vmax),
                           lanes, k, x, v, lo, hi, ok, vmax, length, desp)
    for k in range(lanes):  # a left mover yields to a right mover
        for x in range(length):
            d = dec[k][x]
            if d >= 0 and d == k - 1 and d - 1 >= 0 and dec[d - 1][x] == d:
                dec[k][x] = -2
    moved = 0
    for k in range(lanes):
        for x in range(length):
            d = dec[k][x]
            if d >= 0:
                lat[d][x], lat[k][x] = lat[k][x], -1
                moved += 1
    lanes_out = [[lat[k][x] for x in range(length - 1, -1, -1) if lat[k][x] >= 0]
                 for k in range(lanes)]
    return moved, lanes_out


def by_bits(lanes, length, vmax, desp, veh):
    wpl = (length + 31) // 32
    occ = [[0] * wpl for _ in range(lanes)]
    for (k, x) in veh:
        occ[k][x >> 5] |= 1 << (x & 31)
    rgt = [[0] * wpl for _ in range(lanes)]
    lft = [[0] * wpl for _ in range(lanes)]
    for (k, x), (v, lo, hi, ok, _) in veh.items():
        d = decide(lambda m, c: (occ[m][c >> 5] >> (c & 31)) & 1,
                   lambda m, c: bit_ahead(occ[m], wpl, length, c, vmax),
                   lambda m, c: bit_behind(occ[m], wpl, c, vmax),
                   lanes, k, x, v, lo, hi, ok, vmax, length, desp)
        if d == k + 1:
            rgt[k][x >> 5] |= 1 << (x & 31)
        elif d >= 0:
            lft[k][x >> 5] |= 1 << (x & 31)
    new = [[0] * wpl for _ in range(lanes)]
    moved = 0
    for k in range(lanes):
        for q in range(wpl):
            up = rgt[k][q]
            below = rgt[k - 1][q] if k >= 1 else 0
            down = lft[k][q] & ~(rgt[k - 2][q] if k >= 2 else 0) & M32
            above = lft[k + 1][q] & ~below & M32 if k + 1 < lanes else 0
            new[k][q] = (occ[k][q] & ~up & ~down & M32) | below | above
            moved += popcount(up) + popcount(down)
    counts = [sum(popcount(w) for w in new[k]) for k in range(lanes)]
    lanes_out = [[None] * counts[k] for k in range(lanes)]
    for (k, x), r in veh.items():
        q, b = x >> 5, x & 31
        d = k
        if (rgt[k][q] >> b) & 1:
            d = k + 1
        elif (lft[k][q] >> b) & 1 and not (k >= 2 and (rgt[k - 2][q] >> b) & 1):
            d = k - 1
        j = popcount(new[d][q] >> (b + 1)) + \
            sum(popcount(new[d][qq]) for qq in range(q + 1, wpl))
        assert lanes_out[d][j] is None, "two vehicles in one place"
        lanes_out[d][j] = r[4]
    return moved, lanes_out


@pytest.mark.parametrize("seed", range(4))
def test_bit_lattice_lane_change_equals_cell_scan(seed):
    rng = random.Random(seed)
    total = 0
    for _ in range(600):
        link = random_link(rng)
        a = by_cells(*link)
        assert by_bits(*link) == a
        total += a[0]
    assert total > 0
