"""Seeded synthetic inputs for the TRANSIMS micro-simulation.

This module builds the *inputs* of a simulation run -- road networks, routes
(the "plans" each traveller follows), departure times and initial placements
-- from a seed.  It contains none of the simulation's own arithmetic: it never
moves a vehicle, never draws the per-step random numbers (those are Philox
draws made inside the simulators) and never decides a lane change or an
intersection.  Both the CPU oracle and the GPU library consume what it makes.

The paper's own inputs (the Portland EMME/2 network of 20,024 links, the
200,000-link TIGER network and the Dallas demand) are not available, so the
generators below produce grid-like networks of the same sizes (Section
"Graph partitioning" gives the link counts) with synthetic demand.
"""
from __future__ import annotations

import dataclasses
from fractions import Fraction
from typing import Optional

import numpy as np

FLAG_RING = 1
FLAG_LANE_CHANGE = 2
FLAG_TURN_LANES = 4

WAITING, ACTIVE, ARRIVED = 0, 1, 2


def prob_threshold(p) -> int:
    """floor(p * 2^32) computed exactly from the decimal text of p.

    A vehicle draw u (a uniform 32-bit word) then satisfies u < threshold with
    probability threshold / 2^32, the closest value not above p."""
    f = Fraction(str(p))
    if f < 0 or f > 1:
        raise ValueError("probability must lie in [0, 1]")
    return int(f * (1 << 32))


@dataclasses.dataclass
class Scenario:
    name: str
    # parameters
    flags: int
    vmax: int
    slow_thr: int
    seed: int
    T: int
    lc_thr: int = 1 << 32
    lc_desp: int = 10
    # network (link-indexed unless noted)
    n_nodes: int = 1
    link_from: np.ndarray = None   # int32
    link_to: np.ndarray = None     # int32
    link_len: np.ndarray = None    # int32 cells
    link_lanes: np.ndarray = None  # int8
    link_rank: np.ndarray = None   # int8
    conn_off: Optional[np.ndarray] = None  # int64 [n_links+1]
    conn_out: Optional[np.ndarray] = None  # int32
    conn_lo: Optional[np.ndarray] = None   # int8
    conn_hi: Optional[np.ndarray] = None   # int8
    node_xy: Optional[np.ndarray] = None   # float64 [n_nodes, 2]
    # fixed-time signals at the downstream end of links: plan index per link
    # (-1: none); plan j is red at step t iff (t + offset[j]) % cycle[j] <
    # red[j]
    signal_plan: Optional[np.ndarray] = None  # int8 [n_links]
    plan_cycle: Optional[np.ndarray] = None   # int32 [n_plans]
    plan_red: Optional[np.ndarray] = None     # int32
    plan_offset: Optional[np.ndarray] = None  # int32
    # vehicles
    n_veh: int = 0
    depart: np.ndarray = None      # int32
    route_off: Optional[np.ndarray] = None    # int64 [n+1]
    route_links: Optional[np.ndarray] = None  # int32
    init_status: Optional[np.ndarray] = None  # int8
    init_lane: Optional[np.ndarray] = None    # int8
    init_x: Optional[np.ndarray] = None       # int32
    init_v: Optional[np.ndarray] = None       # int8
    init_rptr: Optional[np.ndarray] = None    # int32
    exit_t0: Optional[np.ndarray] = None      # int32
    t0: int = 0

    @property
    def n_links(self) -> int:
        return int(len(self.link_len))

    @property
    def ring(self) -> bool:
        return bool(self.flags & FLAG_RING)

    @property
    def n_route_entries(self) -> int:
        return 0 if self.route_off is None else int(self.route_off[-1])

    def with_state(self, state: dict, t0: int) -> "Scenario":
        """The same scenario restarted from a saved state at step t0."""
        s = dataclasses.replace(self)
        s.init_status = np.asarray(state["status"], np.int8).copy()
        s.init_lane = np.asarray(state["lane"], np.int8).copy()
        s.init_x = np.asarray(state["x"], np.int32).copy()
        s.init_v = np.asarray(state["v"], np.int8).copy()
        s.init_rptr = np.asarray(state["rptr"], np.int32).copy()
        if not self.ring:
            s.exit_t0 = np.asarray(state["exit_t"], np.int32).copy()
        s.t0 = int(t0)
        return s

    def save(self, path: str) -> None:
        arrays = {}
        scalars = {}
        for f in dataclasses.fields(self):
            val = getattr(self, f.name)
            if isinstance(val, np.ndarray):
                arrays[f.name] = val
            elif val is not None:
                scalars[f.name] = val
        arrays["__scalars__"] = np.frombuffer(repr(scalars).encode(), np.uint8)
        np.savez(path, **arrays)

    @staticmethod
    def load(path: str) -> "Scenario":
        import ast
        with np.load(path, allow_pickle=False) as z:
            scalars = ast.literal_eval(bytes(z["__scalars__"]).decode())
            arrays = {k: z[k] for k in z.files if k != "__scalars__"}
        return Scenario(**scalars, **arrays)


# ---------------------------------------------------------------------------
# ring road


def ring(L: int = 1000, n: int = 150, vmax: int = 5, p="0.2", seed: int = 42,
         T: int = 1000, placement_seed: Optional[int] = None,
         name: str = "ring") -> Scenario:
    """Single-lane periodic road of L cells with n vehicles placed uniformly
    at random without overlap (v = 0); vehicle ids increase with the cell."""
    if not 0 <= n <= L:
        raise ValueError("need 0 <= n <= L")
    rng = np.random.Generator(np.random.PCG64(seed if placement_seed is None
                                              else placement_seed))
    cells = np.sort(rng.choice(L, size=n, replace=False)).astype(np.int32)
    return ring_from_cells(L, cells, np.zeros(n, np.int8), vmax, p, seed, T,
                           name)


def ring_from_cells(L, cells, v0, vmax, p, seed, T, name="ring") -> Scenario:
    n = len(cells)
    return Scenario(
        name=name, flags=FLAG_RING, vmax=int(vmax), slow_thr=prob_threshold(p),
        seed=int(seed), T=int(T), n_nodes=1,
        link_from=np.zeros(1, np.int32), link_to=np.zeros(1, np.int32),
        link_len=np.array([L], np.int32), link_lanes=np.ones(1, np.int8),
        link_rank=np.zeros(1, np.int8), n_veh=n,
        depart=np.zeros(n, np.int32),
        init_status=np.full(n, ACTIVE, np.int8),
        init_lane=np.zeros(n, np.int8),
        init_x=np.asarray(cells, np.int32).copy(),
        init_v=np.asarray(v0, np.int8).copy(),
        init_rptr=np.zeros(n, np.int32))


# ---------------------------------------------------------------------------
# networks


def _ranks_and_conn(n_nodes, frm, to, lanes, xy, turn_lanes: bool):
    """Priority rank of every link at its downstream node, and the lane
    connectivity table (which lanes of a link lead into which out-link).

    rank: links entering one node are ordered by (more lanes first, east-west
    before north-south, link id); rank 0 has priority.
    Lane connectivity: the out-links of the downstream node except the U-turn,
    ordered left to right as seen by the arriving driver; with m movements
    over n lanes (lane 0 leftmost), movement j uses lanes
    [floor(j*n/m), max(floor(j*n/m), ceil((j+1)*n/m) - 1)]."""
    L = len(frm)
    d = xy[to] - xy[frm]
    ew = np.abs(d[:, 0]) >= np.abs(d[:, 1])
    order = np.lexsort((np.arange(L), ~ew, -lanes.astype(np.int64), to))
    rank = np.zeros(L, np.int8)
    pos = 0
    while pos < L:
        node = to[order[pos]]
        j = pos
        while j < L and to[order[j]] == node:
            rank[order[j]] = j - pos
            j += 1
        if j - pos > 127:
            raise ValueError("too many links into one node")
        pos = j
    out_of = [[] for _ in range(n_nodes)]
    for l in range(L):
        out_of[frm[l]].append(l)
    conn_off = np.zeros(L + 1, np.int64)
    conn_out, conn_lo, conn_hi = [], [], []
    for l in range(L):
        din = d[l]
        outs = [o for o in out_of[to[l]] if to[o] != frm[l]]
        # left-to-right: sort by the signed turn angle, left turns first
        ang = []
        for o in outs:
            dout = d[o]
            cross = din[0] * dout[1] - din[1] * dout[0]
            dot = din[0] * dout[0] + din[1] * dout[1]
            ang.append((-np.arctan2(cross, dot), o))
        ang.sort()
        m = len(ang)
        n = int(lanes[l])
        for j, (_, o) in enumerate(ang):
            lo = (j * n) // m
            hi = max(lo, -((-(j + 1) * n) // m) - 1)
            if not turn_lanes:
                lo, hi = 0, n - 1
            conn_out.append(o)
            conn_lo.append(lo)
            conn_hi.append(hi)
        conn_off[l + 1] = len(conn_out)
    return (rank, conn_off, np.array(conn_out, np.int32),
            np.array(conn_lo, np.int8), np.array(conn_hi, np.int8))


def grid_network(rows: int, cols: int, n_links: int, rng: np.random.Generator,
                 lanes_range=(1, 3), len_sampler=None):
    """Grid graph of rows x cols nodes, thinned to n_links/2 undirected edges
    by removing edges outside a random spanning tree (so the directed graph
    stays strongly connected).  Returns (frm, to, length, lanes, xy)."""
    if n_links % 2:
        raise ValueError("n_links must be even")
    n_nodes = rows * cols
    node = lambda r, c: r * cols + c
    edges = []
    for r in range(rows):
        for c in range(cols):
            if c + 1 < cols:
                edges.append((node(r, c), node(r, c + 1)))
            if r + 1 < rows:
                edges.append((node(r, c), node(r + 1, c)))
    edges = np.array(edges, np.int64)
    E = len(edges)
    want = n_links // 2
    if want < n_nodes - 1 or want > E:
        raise ValueError("edge count out of range for the grid")
    # random spanning tree: Kruskal over a random edge order
    perm = rng.permutation(E)
    parent = np.arange(n_nodes)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    in_tree = np.zeros(E, bool)
    for e in perm:
        a, b = find(edges[e, 0]), find(edges[e, 1])
        if a != b:
            parent[a] = b
            in_tree[e] = True
    extra = np.flatnonzero(~in_tree)
    keep_extra = rng.choice(extra, size=want - (n_nodes - 1), replace=False)
    keep = np.sort(np.concatenate([np.flatnonzero(in_tree), keep_extra]))
    und = edges[keep]
    if len_sampler is None:
        elen = rng.integers(20, 201, size=len(und))
    else:
        elen = len_sampler(rng, len(und))
    frm = np.concatenate([und[:, 0], und[:, 1]]).astype(np.int32)
    to = np.concatenate([und[:, 1], und[:, 0]]).astype(np.int32)
    length = np.concatenate([elen, elen]).astype(np.int32)
    lanes = rng.integers(lanes_range[0], lanes_range[1] + 1,
                         size=len(frm)).astype(np.int8)
    rr, cc = np.divmod(np.arange(n_nodes), cols)
    xy = np.stack([cc, -rr], axis=1).astype(np.float64)  # y grows northward
    return frm, to, length, lanes, xy


def shortest_routes(n_nodes, frm, to, length, orig, dest, chunk=512,
                    max_veh_chunk=200_000):
    """Shortest routes by length (scipy Dijkstra) from orig[i] to dest[i].
    Sources are taken `chunk` at a time, fewer when their vehicles exceed
    max_veh_chunk.  Returns (route_off int64, route_links int32)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    L = len(frm)
    w = csr_matrix((length.astype(np.float64), (frm, to)),
                   shape=(n_nodes, n_nodes))
    # link id of a (from, to) pair: the out-links of every node, padded
    outdeg = np.bincount(frm, minlength=n_nodes)
    D = max(1, int(outdeg.max()) if L else 1)
    by_from = np.argsort(frm, kind="stable")
    first = np.zeros(n_nodes + 1, np.int64)
    np.cumsum(outdeg, out=first[1:])
    slot = np.arange(L) - first[frm[by_from]]
    adj_link = np.full((n_nodes, D), -1, np.int64)
    adj_link[frm[by_from], slot] = by_from
    adj_to = np.full((n_nodes, D), -1, np.int64)
    adj_to[frm[by_from], slot] = to[by_from]
    n = len(orig)
    orig = np.asarray(orig, np.int64)
    dest = np.asarray(dest, np.int64)
    uniq = np.unique(orig)
    order = np.argsort(orig, kind="stable")
    sorted_orig = orig[order]
    lens = np.zeros(n, np.int64)
    pieces = []  # (vehicle ids, their links back to front, lengths)
    per_src = np.diff(np.searchsorted(sorted_orig,
                                      np.append(uniq, uniq[-1] + 1)
                                      if len(uniq) else uniq))
    bounds = [0]
    while bounds[-1] < len(uniq):
        b0 = bounds[-1]
        b1 = min(b0 + chunk, len(uniq))
        cum = np.cumsum(per_src[b0:b1])
        fit = int(np.searchsorted(cum, max_veh_chunk, "right"))
        bounds.append(b0 + max(1, min(fit, b1 - b0)))
    for c0, c1 in zip(bounds[:-1], bounds[1:]):
        srcs = uniq[c0:c1]
        _, pred = dijkstra(w, directed=True, indices=srcs,
                           return_predecessors=True)
        lo = np.searchsorted(sorted_orig, srcs[0], "left")
        hi = np.searchsorted(sorted_orig, srcs[-1], "right")
        vids = order[lo:hi]
        rows = np.searchsorted(srcs, orig[vids])
        cur = dest[vids].copy()
        steps = []
        alive = np.flatnonzero(cur != orig[vids])
        while len(alive):
            prev = pred[rows[alive], cur[alive]].astype(np.int64)
            if (prev < 0).any():
                raise ValueError("destination unreachable")
            hit = adj_to[prev] == cur[alive][:, None]
            links = adj_link[prev, hit.argmax(1)]
            step = np.full(len(vids), -1, np.int64)
            step[alive] = links
            steps.append(step)
            cur[alive] = prev
            alive = alive[cur[alive] != orig[vids][alive]]
        if steps:
            mat = np.array(steps[::-1]).T  # vehicle x position, -1 padded
            # the path of each vehicle is the tail of its row
            keep = mat >= 0
            lens[vids] = keep.sum(1)
            pieces.append((vids, mat[keep]))
    route_off = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=route_off[1:])
    route_links = np.zeros(int(route_off[-1]), np.int32)
    for vids, flat in pieces:
        # flat holds the routes of vids back to back, in vids order
        starts = route_off[vids]
        cnt = lens[vids]
        within = np.arange(len(flat)) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        route_links[np.repeat(starts, cnt) + within] = flat
    return route_off, route_links


def grid_scenario(rows: int, cols: int, n_links: int, n_veh: int, T: int,
                  depart_max: int, seed: int, vmax: int = 5, p="0.2",
                  lanes_range=(1, 3), flags: int = 0, len_sampler=None,
                  depart_sampler=None, sim_seed: Optional[int] = None,
                  n_origins: int = 0, signals: Optional[tuple] = None,
                  name: str = "grid") -> Scenario:
    """Grid network with n_veh vehicles routed by shortest path between
    distinct uniformly random nodes, departing uniformly in [0, depart_max].
    n_origins > 0 draws the origins from that many random nodes only (trip
    generation zones), which bounds the routing work of large demands.
    signals = (cycle, red) puts fixed-time signals on every node that at
    least three links enter: its east-west approaches are red in the first
    `red` steps of each cycle, its north-south approaches `cycle // 2` steps
    later (the paper's validation signal is 30 s red, 30 s green)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    frm, to, length, lanes, xy = grid_network(rows, cols, n_links, rng,
                                              lanes_range, len_sampler)
    length = np.maximum(length, vmax + 1).astype(np.int32)
    n_nodes = rows * cols
    rank, conn_off, conn_out, conn_lo, conn_hi = _ranks_and_conn(
        n_nodes, frm, to, lanes, xy, bool(flags & FLAG_TURN_LANES))
    if n_origins > 0 and n_origins < n_nodes:
        zones = rng.choice(n_nodes, size=n_origins, replace=False)
        orig = zones[rng.integers(0, n_origins, size=n_veh)]
    else:
        orig = rng.integers(0, n_nodes, size=n_veh)
    dest = rng.integers(0, n_nodes - 1, size=n_veh)
    dest = dest + (dest >= orig)  # distinct from the origin
    route_off, route_links = shortest_routes(n_nodes, frm, to, length, orig,
                                             dest)
    if depart_sampler is None:
        depart = rng.integers(0, depart_max + 1, size=n_veh).astype(np.int32)
    else:
        depart = depart_sampler(rng, n_veh).astype(np.int32)
    sig = {}
    if signals is not None:
        cycle, red = int(signals[0]), int(signals[1])
        indeg = np.bincount(to, minlength=n_nodes)
        d = xy[to] - xy[frm]
        ew = np.abs(d[:, 0]) >= np.abs(d[:, 1])
        plan = np.where(ew, 0, 1).astype(np.int8)
        plan[indeg[to] < 3] = -1
        sig = dict(signal_plan=plan,
                   plan_cycle=np.array([cycle, cycle], np.int32),
                   plan_red=np.array([red, red], np.int32),
                   plan_offset=np.array([0, cycle // 2], np.int32))
    return Scenario(
        name=name, flags=flags, vmax=vmax, slow_thr=prob_threshold(p),
        seed=int(seed if sim_seed is None else sim_seed), T=T,
        n_nodes=n_nodes, link_from=frm, link_to=to, link_len=length,
        link_lanes=lanes, link_rank=rank, conn_off=conn_off,
        conn_out=conn_out, conn_lo=conn_lo, conn_hi=conn_hi, node_xy=xy,
        n_veh=n_veh, depart=depart, route_off=route_off,
        route_links=route_links, **sig)


def loop_of_links(lengths, n: int, vmax: int = 5, p="0.2", seed: int = 1,
                  T: int = 200, lanes: int = 1, placement_seed: int = 7,
                  flags: int = 0, name: str = "loop") -> Scenario:
    """A cycle of k single-direction links (node j -> node j+1 mod k) with n
    vehicles per lane placed at random; every route runs around the cycle
    far more often than T steps allow, so no trip ends.  Vehicle ids grow
    with the position along the unrolled cycle (lane by lane)."""
    lengths = np.asarray(lengths, np.int32)
    k = len(lengths)
    total = int(lengths.sum())
    rng = np.random.Generator(np.random.PCG64(placement_seed))
    starts = np.concatenate([[0], np.cumsum(lengths)[:-1]])
    laps = (T * vmax) // int(lengths.min()) + 3
    ids_status, ids_lane, ids_x, ids_rptr, routes = [], [], [], [], []
    for lane in range(lanes):
        cells = np.sort(rng.choice(total, size=n, replace=False))
        for c in cells:
            link = int(np.searchsorted(starts, c, "right") - 1)
            ids_lane.append(lane)
            ids_x.append(int(c - starts[link]))
            routes.append([(link + j) % k for j in range(laps + 1)])
    nv = len(routes)
    route_off = np.zeros(nv + 1, np.int64)
    np.cumsum([len(r) for r in routes], out=route_off[1:])
    xy = np.stack([np.cos(2 * np.pi * np.arange(k) / k),
                   np.sin(2 * np.pi * np.arange(k) / k)], 1)
    frm = np.arange(k, dtype=np.int32)
    to = ((np.arange(k) + 1) % k).astype(np.int32)
    lanes_arr = np.full(k, lanes, np.int8)
    conn_off = np.arange(k + 1, dtype=np.int64)
    return Scenario(
        name=name, flags=flags, vmax=vmax, slow_thr=prob_threshold(p),
        seed=seed, T=T, n_nodes=k, link_from=frm, link_to=to,
        link_len=lengths.copy(), link_lanes=lanes_arr,
        link_rank=np.zeros(k, np.int8), conn_off=conn_off,
        conn_out=to.copy(), conn_lo=np.zeros(k, np.int8),
        conn_hi=np.full(k, lanes - 1, np.int8), node_xy=xy, n_veh=nv,
        depart=np.zeros(nv, np.int32), route_off=route_off,
        route_links=np.concatenate(routes).astype(np.int32),
        init_status=np.full(nv, ACTIVE, np.int8),
        init_lane=np.array(ids_lane, np.int8),
        init_x=np.array(ids_x, np.int32), init_v=np.zeros(nv, np.int8),
        init_rptr=np.zeros(nv, np.int32))


def chain(lengths, lanes=None, depart=(0,), vmax: int = 5, p="0", seed=3,
          T: int = 200, name: str = "chain") -> Scenario:
    """A straight chain of links node j -> node j+1; every vehicle travels
    the whole chain from the first link, departing at the given times."""
    lengths = np.asarray(lengths, np.int32)
    k = len(lengths)
    lanes_arr = (np.ones(k, np.int8) if lanes is None
                 else np.asarray(lanes, np.int8))
    n = len(depart)
    frm = np.arange(k, dtype=np.int32)
    to = np.arange(1, k + 1, dtype=np.int32)
    xy = np.stack([np.arange(k + 1), np.zeros(k + 1)], 1).astype(float)
    conn_off = np.zeros(k + 1, np.int64)
    conn_off[1:] = np.minimum(np.arange(1, k + 1), k - 1)
    return Scenario(
        name=name, flags=0, vmax=vmax, slow_thr=prob_threshold(p), seed=seed,
        T=T, n_nodes=k + 1, link_from=frm, link_to=to, link_len=lengths,
        link_lanes=lanes_arr, link_rank=np.zeros(k, np.int8),
        conn_off=conn_off, conn_out=np.arange(1, k, dtype=np.int32),
        conn_lo=np.zeros(k - 1, np.int8),
        conn_hi=(lanes_arr[:-1] - 1).astype(np.int8), node_xy=xy, n_veh=n,
        depart=np.asarray(depart, np.int32),
        route_off=np.arange(n + 1, dtype=np.int64) * k,
        route_links=np.tile(np.arange(k, dtype=np.int32), n))


# ---------------------------------------------------------------------------
# the named workloads


def portland_like(seed: int = 2024, scale: float = 1.0, T: int = 3600,
                  flags: int = 0, depart_max: int = 1799,
                  signals: Optional[tuple] = None) -> Scenario:
    """Portland-sized grid: 77 x 78 = 6,006 nodes thinned to 20,024 directed
    links of 1-3 lanes, edge lengths uniform in 20..200 cells, 200,000
    vehicles with shortest-path routes between random distinct nodes,
    departures uniform over the first 1,800 s.  `scale` < 1 shrinks the grid
    side and the demand for quick parity cases."""
    if scale >= 1.0:
        rows, cols, links, nveh = 77, 78, 20024, 200000
    else:
        rows = max(3, int(round(77 * np.sqrt(scale))))
        cols = max(3, int(round(78 * np.sqrt(scale))))
        nodes = rows * cols
        und_all = rows * (cols - 1) + cols * (rows - 1)
        und = max(nodes - 1, min(und_all, int(round(10012 * scale))))
        links = 2 * und
        nveh = max(1, int(round(200000 * scale)))
    return grid_scenario(rows, cols, links, nveh, T, depart_max, seed,
                         flags=flags, signals=signals,
                         name=f"portland_like(scale={scale})")


def _grid_shape(n_links: int):
    """Near-square grid and an even directed-link count for about n_links
    links at the Portland-like mean out-degree (20,024 links on 6,006
    nodes, 3.33)."""
    nodes = max(4, int(round(n_links / (20024 / 6006))))
    rows = max(2, int(round(np.sqrt(nodes))))
    cols = max(2, int(np.ceil(nodes / rows)))
    nodes = rows * cols
    und_all = rows * (cols - 1) + cols * (rows - 1)
    und = min(und_all, max(nodes - 1, n_links // 2))
    return rows, cols, 2 * und


def batched_scenarios(n: int = 64, seed: int = 77, T: int = 3600,
                      links_lo: int = 1000, links_hi: int = 20000,
                      veh_per_link=(5, 15), depart_max: int = 1799,
                      n_origins: int = 256, scale: float = 1.0):
    """Independent replications of uneven sizes: link counts log-uniform in
    [links_lo, links_hi], each a Portland-style grid with its own network
    seed, links x U{5..15} vehicles departing uniformly in [0, depart_max],
    Philox seed 1000 + k.  `scale` shrinks every size for quick cases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        links = int(round(np.exp(rng.uniform(np.log(links_lo),
                                             np.log(links_hi))) * scale))
        rows, cols, links = _grid_shape(max(links, 8))
        per = int(rng.integers(veh_per_link[0], veh_per_link[1] + 1))
        out.append(grid_scenario(
            rows, cols, links, max(1, links * per), T, depart_max,
            seed=int(rng.integers(0, 2**31)), sim_seed=1000 + k,
            n_origins=n_origins, name=f"batch[{k}]"))
    return out


def serving_pool(n: int = 32, seed: int = 5000, links_lo: int = 1000,
                 links_hi: int = 50000, veh_per_link: int = 10,
                 horizon=(600, 3600), n_origins: int = 256,
                 scale: float = 1.0):
    """Pre-generated (network, demand) sets for the serving loop: link counts
    log-uniform in [links_lo, links_hi], 10 vehicles per link, a horizon
    U{600..3600} steps, departures uniform over its first half, seed
    5000 + k."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        links = int(round(np.exp(rng.uniform(np.log(links_lo),
                                             np.log(links_hi))) * scale))
        rows, cols, links = _grid_shape(max(links, 8))
        T = int(rng.integers(horizon[0], horizon[1] + 1))
        out.append(grid_scenario(
            rows, cols, links, max(1, links * veh_per_link), T, T // 2,
            seed=int(rng.integers(0, 2**31)), sim_seed=seed + k,
            n_origins=n_origins, name=f"pool[{k}]"))
    return out


def large_network(seed: int = 4242, scale: float = 1.0, T: int = 7200,
                  flags: int = FLAG_LANE_CHANGE | FLAG_TURN_LANES,
                  n_origins: int = 1024) -> Scenario:
    """The 200,000-link network: a 245 x 245 grid thinned to 200,000
    directed links of 1-4 lanes, lengths lognormal with median 60 cells and
    sigma 0.5 clamped to [6, 1000], 2,000,000 vehicles departing around the
    morning peak (Gaussian, mean 3,600 s, sigma 1,800 s, redrawn until inside
    [0, 7199]), lane changing with turn lanes.  Origins are drawn from
    n_origins random zone nodes.  `scale` shrinks the grid and the demand."""
    side = 245
    links, nveh = 200000, 2000000
    if scale < 1.0:
        side = max(3, int(round(245 * np.sqrt(scale))))
        und_all = 2 * side * (side - 1)
        links = 2 * max(side * side - 1,
                        min(und_all, int(round(100000 * scale))))
        nveh = max(1, int(round(2000000 * scale)))

    def lengths(rng, m):
        x = np.exp(np.log(60.0) + 0.5 * rng.standard_normal(m))
        return np.clip(np.rint(x), 6, 1000).astype(np.int64)

    def departs(rng, m):
        d = rng.normal(3600.0, 1800.0, size=m)
        bad = (d < 0) | (d > T - 1)
        while bad.any():
            d[bad] = rng.normal(3600.0, 1800.0, size=int(bad.sum()))
            bad = (d < 0) | (d > T - 1)
        return np.floor(d).astype(np.int32)

    return grid_scenario(side, side, links, nveh, T, T - 1, seed,
                         lanes_range=(1, 4), flags=flags, len_sampler=lengths,
                         depart_sampler=departs, n_origins=n_origins,
                         name=f"large_network(scale={scale})")
