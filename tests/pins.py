"""Independent references that pin the CPU oracle to the mathematics.

None of these shares code with the oracle or with the GPU library:
  - brute force over every delta-smooth surface of a tiny volume (the
    definition of the optimal net surface, Section 1.2 and Eq. 1);
  - an exact dynamic program along a single row of columns;
  - the closed form of the max-flow value from the optimal energy;
  - library max-flow routines (scipy, networkx) on the explicit graph, and
    a second oracle built on scipy's: both extreme minimum cuts read off
    its residual graph.
"""
from __future__ import annotations

import itertools

import numpy as np


def neighbours(nx, ny):
    """Unordered 4-neighbour column pairs of an nx x ny grid, flat indices."""
    out = []
    for x in range(nx):
        for y in range(ny):
            if x + 1 < nx:
                out.append((x * ny + y, (x + 1) * ny + y))
            if y + 1 < ny:
                out.append((x * ny + y, x * ny + y + 1))
    return out


def brute_force(cost: np.ndarray, delta: int, alpha: int = 0):
    """E*, the pointwise-lowest and pointwise-highest optimal surfaces.

    Enumerates all K^(nx*ny) height maps, keeps the delta-smooth ones and
    takes the minimum of sum_p c(p, h(p)) + alpha * sum |h(p) - h(q)| over
    neighbour pairs.  The optimal surfaces form a lattice under pointwise
    min/max (the energy is submodular), so the pointwise min (max) over all
    optimal surfaces is itself optimal.
    """
    nx, ny, K = cost.shape
    P = nx * ny
    c = cost.reshape(P, K).astype(np.int64)
    H = np.array(list(itertools.product(range(K), repeat=P)), dtype=np.int64)
    ok = np.ones(len(H), dtype=bool)
    for a, b in neighbours(nx, ny):
        ok &= np.abs(H[:, a] - H[:, b]) <= delta
    H = H[ok]
    E = c[np.arange(P)[None, :], H].sum(axis=1)
    for a, b in neighbours(nx, ny):
        E = E + alpha * np.abs(H[:, a] - H[:, b])
    best = E.min()
    opt = H[E == best]
    return int(best), opt.min(axis=0).reshape(nx, ny), opt.max(axis=0).reshape(nx, ny)


def _window_min(a: np.ndarray, delta: int) -> np.ndarray:
    """out[z] = min(a[z - delta .. z + delta]) clipped to the array."""
    K = a.shape[0]
    out = a.copy()
    for s in range(1, delta + 1):
        if s >= K:
            break
        out[:-s] = np.minimum(out[:-s], a[s:])
        out[s:] = np.minimum(out[s:], a[:-s])
    return out


def _window_min_penalty(a: np.ndarray, delta: int, alpha: int) -> np.ndarray:
    """out[z] = min over |s| <= delta of a[z + s] + alpha * |s| (inside the array)."""
    K = a.shape[0]
    out = a.copy()
    for s in range(1, delta + 1):
        if s >= K:
            break
        out[:-s] = np.minimum(out[:-s], a[s:] + alpha * s)
        out[s:] = np.minimum(out[s:], a[:-s] + alpha * s)
    return out


def row_dp(cost: np.ndarray, delta: int, alpha: int = 0):
    """Exact optimum for a single row of columns (cost shape (n, K)).

    Forward and backward min-plus recurrences over the chain of columns:
    Fw[x][z] = c(x,z) + min_{|z'-z|<=delta} (Fw[x-1][z'] + alpha |z - z'|)
    and the mirror image Bw.  The best surface through (x, z) costs
    Fw + Bw - c; the lowest (highest) z attaining E* at x is h_min(x)
    (h_max(x)).
    """
    c = cost.astype(np.int64)
    n, K = c.shape
    Fw = np.empty_like(c)
    Bw = np.empty_like(c)
    Fw[0] = c[0]
    for x in range(1, n):
        Fw[x] = c[x] + _window_min_penalty(Fw[x - 1], delta, alpha)
    Bw[n - 1] = c[n - 1]
    for x in range(n - 2, -1, -1):
        Bw[x] = c[x] + _window_min_penalty(Bw[x + 1], delta, alpha)
    best = int(Fw[n - 1].min())
    through = Fw + Bw - c
    hit = through == best
    hmin = np.argmax(hit, axis=1)
    hmax = K - 1 - np.argmax(hit[:, ::-1], axis=1)
    return best, hmin.astype(np.int32), hmax.astype(np.int32)


def flow_closed_form(cost: np.ndarray, energy: int) -> int:
    """Max-flow value from the optimal energy.

    With B > max_p c(p,0) the minimum cut is a delta-smooth surface whose
    capacity is W^- + sum_{z <= h(p)} w(p,z) = E(h) - sum_p c(p,0)
    + sum_p sum_{z>=1} max(0, c(p,z-1) - c(p,z)), independent of B.
    """
    c = cost.astype(np.int64)
    drops = np.maximum(0, c[:, :, :-1] - c[:, :, 1:]).sum()
    return int(energy - c[:, :, 0].sum() + drops)


def explicit_arcs(cost: np.ndarray, delta: int, inf: int, alpha: int = 0):
    """(tail, head, capacity) triples of G(c, delta), s = N, t = N + 1; with
    alpha > 0 also the soft arcs (p,z) -> (q,z) of capacity alpha, z >= 1."""
    nx, ny, K = cost.shape
    c = cost.astype(np.int64)
    N = nx * ny * K
    s, t = N, N + 1
    B = int(c[:, :, 0].max()) + 1
    arcs = []
    idx = lambda x, y, z: (x * ny + y) * K + z
    for x in range(nx):
        for y in range(ny):
            for z in range(K):
                v = idx(x, y, z)
                w = int(c[x, y, 0]) - B if z == 0 else int(c[x, y, z] - c[x, y, z - 1])
                if w < 0:
                    arcs.append((s, v, -w))
                elif w > 0:
                    arcs.append((v, t, w))
                if z > 0:
                    arcs.append((v, idx(x, y, z - 1), inf))
                for qx, qy in ((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)):
                    if 0 <= qx < nx and 0 <= qy < ny:
                        arcs.append((v, idx(qx, qy, max(0, z - delta)), inf))
                        if alpha > 0 and z >= 1:
                            arcs.append((v, idx(qx, qy, z), alpha))
    return arcs, s, t, N + 2


def scipy_flow(cost: np.ndarray, delta: int, alpha: int = 0) -> int:
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_flow

    arcs, s, t, n = explicit_arcs(cost, delta, inf=1 << 28, alpha=alpha)
    a = np.array(arcs, dtype=np.int64)
    # parallel arcs (a soft and an infinite arc between the same nodes at
    # delta = 0) add up, as the sparse constructor sums duplicates
    m = sp.csr_array((a[:, 2].astype(np.int32), (a[:, 0], a[:, 1])), shape=(n, n))
    return int(maximum_flow(m, s, t).flow_value)


def scipy_cuts(cost: np.ndarray, delta: int, alpha: int = 0):
    """A second oracle: scipy's max-flow on the explicit graph, and the
    extreme minimum cuts read off its residual graph (Theorem 1.1): S_min is
    what s reaches, S_max what cannot reach t.  Returns (F, h_min, h_max)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import breadth_first_order, maximum_flow

    nx, ny, K = cost.shape
    arcs, s, t, n = explicit_arcs(cost, delta, inf=1 << 28, alpha=alpha)
    a = np.array(arcs, dtype=np.int64)
    cap = sp.csr_array((a[:, 2].astype(np.int32), (a[:, 0], a[:, 1])), shape=(n, n))
    res = maximum_flow(cap, s, t)
    # net flow is antisymmetric, so capacity minus flow is the residual
    # capacity of every ordered pair, reverse arcs included
    r = sp.csr_array(cap.astype(np.int64) - res.flow.astype(np.int64))
    r.data[r.data < 0] = 0
    r.eliminate_zeros()
    from_s = np.zeros(n, bool)
    from_s[breadth_first_order(r, s, directed=True, return_predecessors=False)] = True
    to_t = np.zeros(n, bool)
    to_t[breadth_first_order(sp.csr_array(r.T), t, directed=True, return_predecessors=False)] = True
    smin = from_s[:-2].reshape(nx, ny, K)
    smax = ~to_t[:-2].reshape(nx, ny, K)
    zs = np.arange(K)
    hmin = np.where(smin, zs, -1).max(axis=2).astype(np.int32)
    hmax = np.where(smax, zs, -1).max(axis=2).astype(np.int32)
    return int(res.flow_value), hmin, hmax


def networkx_flow(cost: np.ndarray, delta: int, alpha: int = 0) -> int:
    import networkx as nx_

    arcs, s, t, n = explicit_arcs(cost, delta, inf=-1, alpha=alpha)
    # parallel arcs (a soft and an infinite arc between the same nodes at
    # delta = 0) are merged: infinite if either is, else capacities add
    merged = {}
    for u, v, cap in arcs:
        old = merged.get((u, v))
        merged[(u, v)] = cap if old is None else (-1 if old < 0 or cap < 0 else old + cap)
    g = nx_.DiGraph()
    g.add_nodes_from(range(n))
    for (u, v), cap in merged.items():
        if cap < 0:
            g.add_edge(u, v)          # no capacity attribute = infinite
        else:
            g.add_edge(u, v, capacity=cap)
    return int(nx_.maximum_flow_value(g, s, t))


def reduced_preflow(cost: np.ndarray, delta: int):
    """The hard-bound case of reduced_preflow_soft (no soft arcs); returns
    (excess, sink residual, down flow, lateral flows, flow value)."""
    e, ts, fd, fl, _, flow = reduced_preflow_soft(cost, delta, 0)
    return e, ts, fd, fl, flow


def _fifo_push_relabel(N, t, e, arcs, out, inn):
    """Textbook FIFO push-relabel (Section 2.1) to a maximum preflow, in
    place: arcs are [tail, head, cap (-1 infinite), flow, kind] lists, out/inn
    the arc indices per node, e the excess (source arcs already saturated),
    t = N the sink.  A node whose label reaches N + 2 has no path to t and
    stops."""
    from collections import deque

    n = N + 2
    d = [0] * N
    q = deque(v for v in range(N) if e[v] > 0)
    inq = set(q)
    while q:
        u = q.popleft()
        inq.discard(u)
        while e[u] > 0 and d[u] < n:
            pushed = False
            # residual arcs out of u: forward arcs with room, reverse of arcs into u
            for a in out[u]:
                tail, head, cap, f, _ = arcs[a]
                r = (1 << 62) if cap < 0 else cap - f
                dh = 0 if head == t else d[head]
                if r > 0 and d[u] == dh + 1:
                    amt = min(e[u], r)
                    arcs[a][3] += amt
                    e[u] -= amt
                    if head != t:
                        e[head] += amt
                        if head not in inq:
                            q.append(head); inq.add(head)
                    pushed = True
                    if e[u] == 0:
                        break
            if e[u] > 0:
                for a in inn[u]:
                    tail, head, cap, f, _ = arcs[a]
                    if f > 0 and d[u] == d[tail] + 1:
                        amt = min(e[u], f)
                        arcs[a][3] -= amt
                        e[u] -= amt
                        e[tail] += amt
                        if tail not in inq:
                            q.append(tail); inq.add(tail)
                        pushed = True
                        if e[u] == 0:
                            break
            if e[u] > 0 and not pushed:
                best = n
                for a in out[u]:
                    tail, head, cap, f, _ = arcs[a]
                    if cap < 0 or cap - f > 0:
                        best = min(best, 1 if head == t else d[head] + 1)
                for a in inn[u]:
                    tail, head, cap, f, _ = arcs[a]
                    if f > 0:
                        best = min(best, d[tail] + 1)
                d[u] = best



def reduced_preflow_soft(cost: np.ndarray, delta: int, alpha: int):
    """A maximum preflow of the reduced column graph by textbook FIFO
    push-relabel (Section 2.1), in plain Python loops for tiny volumes.
    With alpha > 0 the graph also has the soft arcs (p,z) -> (q,z), z >= 1,
    of capacity alpha; their flows come back as a fifth array.

    The reduced graph keeps the down arcs and, per 4-neighbour q, the
    lateral arcs (p,z) -> (q, z - delta) for z > delta plus (p,0) -> (q,0);
    source arcs start saturated and excess is never returned to s (a node
    whose label reaches n has no path to t and stops).  Returns the solver
    storage arrays (excess, sink residual, down flow, lateral flows in
    +x,-x,+y,-y order) and the flow value.
    """
    from collections import deque

    nx, ny, K = cost.shape
    c = cost.astype(np.int64)
    N = nx * ny * K
    t = N
    B = int(c[:, :, 0].max()) + 1
    idx = lambda x, y, z: (x * ny + y) * K + z
    # arcs: [tail, head, cap(-1 = inf), flow, kind, slot]
    arcs = []
    out = [[] for _ in range(N)]
    inn = [[] for _ in range(N + 1)]
    e = np.zeros(N, dtype=np.int64)
    dirs = ((1, 0), (-1, 0), (0, 1), (0, -1))

    def add(u, v, cap, kind):
        arcs.append([u, v, cap, 0, kind])
        out[u].append(len(arcs) - 1)
        inn[v].append(len(arcs) - 1)

    for x in range(nx):
        for y in range(ny):
            for z in range(K):
                v = idx(x, y, z)
                w = int(c[x, y, 0]) - B if z == 0 else int(c[x, y, z] - c[x, y, z - 1])
                if w < 0:
                    e[v] = -w
                if w > 0:
                    add(v, t, w, ("t",))
                if z > 0:
                    add(v, v - 1, -1, ("d",))
                for k, (ddx, ddy) in enumerate(dirs):
                    qx, qy = x + ddx, y + ddy
                    if 0 <= qx < nx and 0 <= qy < ny and (z == 0 or z > delta):
                        add(v, idx(qx, qy, 0 if z == 0 else z - delta), -1, ("l", k))
                    if alpha > 0 and 0 <= qx < nx and 0 <= qy < ny and z >= 1:
                        add(v, idx(qx, qy, z), alpha, ("s", k))

    _fifo_push_relabel(N, t, e, arcs, out, inn)

    ts = np.zeros(N, dtype=np.int64)
    fd = np.zeros(N, dtype=np.int64)
    fl = np.zeros((4, N), dtype=np.int64)
    fs = np.zeros((4, N), dtype=np.int64)
    flow = 0
    for tail, head, cap, f, kind in arcs:
        if kind[0] == "t":
            ts[tail] = cap - f
            flow += f
        elif kind[0] == "d":
            fd[tail] = f
        elif kind[0] == "l":
            fl[kind[1], tail] = f
        else:
            fs[kind[1], tail] = f
    sh = (nx, ny, K)
    return (e.reshape(sh).astype(np.int32), ts.reshape(sh).astype(np.int32),
            fd.reshape(sh).astype(np.int32), fl.reshape((4,) + sh).astype(np.int32),
            fs.reshape((4,) + sh).astype(np.int32), flow)


# ---- narrow-band volumes ------------------------------------------------------
#
# Column p holds the heights off[p] .. off[p] + ext[p] - 1; cost[x, y, j] is
# the cost at height off[x, y] + j.  Heights below are heights of the volume.


def band_bounds(off, ext, delta):
    """(lo, hi) per column by propagating the pairwise bounds column by
    column from a queue until they hold everywhere, or None when a column's
    range empties.  (The oracle sweeps all pairs instead.)"""
    from collections import deque

    off = np.asarray(off, dtype=np.int64)
    nx, ny = off.shape
    lo = off.copy()
    hi = off + np.asarray(ext, dtype=np.int64) - 1
    q = deque((x, y) for x in range(nx) for y in range(ny))
    while q:
        x, y = q.popleft()
        for qx, qy in ((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)):
            if not (0 <= qx < nx and 0 <= qy < ny):
                continue
            changed = False
            if lo[x, y] - delta > lo[qx, qy]:
                lo[qx, qy] = lo[x, y] - delta
                changed = True
            if hi[qx, qy] > hi[x, y] + delta:
                hi[qx, qy] = hi[x, y] + delta
                changed = True
            if changed:
                if lo[qx, qy] > hi[qx, qy]:
                    return None
                q.append((qx, qy))
    return lo.astype(np.int32), hi.astype(np.int32)


def brute_force_band(cost, delta, off, ext):
    """Every surface with h(p) in its band and |h(p) - h(q)| <= delta:
    (E*, h_min, h_max, lo, hi) with lo/hi the lowest and highest height any
    such surface takes per column, or None when there is none."""
    nx, ny, K = cost.shape
    P = nx * ny
    o = np.asarray(off).reshape(P)
    e = np.asarray(ext).reshape(P)
    ranges = [range(int(o[p]), int(o[p] + e[p])) for p in range(P)]
    H = np.array(list(itertools.product(*ranges)), dtype=np.int64)
    ok = np.ones(len(H), dtype=bool)
    for a, b in neighbours(nx, ny):
        ok &= np.abs(H[:, a] - H[:, b]) <= delta
    H = H[ok]
    if len(H) == 0:
        return None
    c = cost.reshape(P, K).astype(np.int64)
    E = c[np.arange(P)[None, :], H - o[None, :]].sum(axis=1)
    best = E.min()
    opt = H[E == best]
    sh = (nx, ny)
    return (int(best), opt.min(axis=0).reshape(sh), opt.max(axis=0).reshape(sh),
            H.min(axis=0).reshape(sh), H.max(axis=0).reshape(sh))


def row_dp_band(cost, delta, off, ext):
    """Exact optimum of a single row of band columns (cost (n, K), off and
    ext (n,)): forward and backward min-plus passes over the heights of the
    volume, each step taking the window [z - delta, z + delta] of the
    previous column's band.  Returns (E*, h_min, h_max) or None."""
    n, K = cost.shape
    off = np.asarray(off, dtype=np.int64)
    ext = np.asarray(ext, dtype=np.int64)
    Z = int((off + ext).max())
    INF = 1 << 60
    c = np.full((n, Z), INF, dtype=np.int64)
    for x in range(n):
        c[x, off[x]:off[x] + ext[x]] = cost[x, :ext[x]]

    def window(a):
        out = np.full(Z, INF, dtype=np.int64)
        for z in range(Z):
            out[z] = a[max(0, z - delta):min(Z, z + delta + 1)].min()
        return out

    Fw = np.full((n, Z), INF, dtype=np.int64)
    Fw[0] = c[0]
    for x in range(1, n):
        Fw[x] = np.minimum(c[x] + window(Fw[x - 1]), INF)
    Bw = np.full((n, Z), INF, dtype=np.int64)
    Bw[n - 1] = c[n - 1]
    for x in range(n - 2, -1, -1):
        Bw[x] = np.minimum(c[x] + window(Bw[x + 1]), INF)
    best = int(Fw[n - 1].min())
    if best >= INF:
        return None
    through = np.where((Fw < INF) & (Bw < INF), Fw + Bw - np.where(c < INF, c, 0), INF)
    hit = through == best
    hmin = np.argmax(hit, axis=1)
    hmax = Z - 1 - np.argmax(hit[:, ::-1], axis=1)
    return best, hmin.astype(np.int32), hmax.astype(np.int32)


def band_cost_at(cost, off, h):
    """c(p, h(p)) per column for heights of the volume."""
    nx, ny, K = cost.shape
    j = np.asarray(h, dtype=np.int64) - np.asarray(off, dtype=np.int64)
    return cost.reshape(nx * ny, K)[np.arange(nx * ny), j.reshape(-1)].reshape(nx, ny)


def band_flow_closed_form(cost, off, lo, hi, energy):
    """Max-flow value of the band graph from the optimal energy: the closed
    form of flow_closed_form on each column's feasible heights lo..hi."""
    nx, ny, K = cost.shape
    total = int(energy)
    for x in range(nx):
        for y in range(ny):
            col = cost[x, y, lo[x, y] - off[x, y]:hi[x, y] - off[x, y] + 1].astype(np.int64)
            total -= int(col[0])
            total += int(np.maximum(0, col[:-1] - col[1:]).sum())
    return total


def explicit_band_arcs(cost, delta, off, lo, hi, inf):
    """(tail, head, capacity) triples of the band graph on the feasible
    heights: node (p, z) for lo(p) <= z <= hi(p); B = max c(p, lo(p)) + 1;
    lateral arcs (p, z) -> (q, max(lo(q), z - delta)); s = N, t = N + 1."""
    nx, ny, K = cost.shape
    cnt = (hi - lo + 1).reshape(-1).astype(np.int64)
    base = np.concatenate([[0], np.cumsum(cnt)])
    N = int(base[-1])
    s, t = N, N + 1
    cz = lambda x, y, z: int(cost[x, y, z - off[x, y]])
    node = lambda x, y, z: int(base[x * ny + y] + z - lo[x, y])
    B = max(cz(x, y, lo[x, y]) for x in range(nx) for y in range(ny)) + 1
    arcs = []
    for x in range(nx):
        for y in range(ny):
            for z in range(lo[x, y], hi[x, y] + 1):
                v = node(x, y, z)
                w = cz(x, y, z) - B if z == lo[x, y] else cz(x, y, z) - cz(x, y, z - 1)
                if w < 0:
                    arcs.append((s, v, -w))
                elif w > 0:
                    arcs.append((v, t, w))
                if z > lo[x, y]:
                    arcs.append((v, v - 1, inf))
                for qx, qy in ((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1)):
                    if 0 <= qx < nx and 0 <= qy < ny:
                        arcs.append((v, node(qx, qy, max(lo[qx, qy], z - delta)), inf))
    return arcs, s, t, N + 2


def scipy_band_flow(cost, delta, off, lo, hi) -> int:
    import scipy.sparse as sp
    from scipy.sparse.csgraph import maximum_flow

    arcs, s, t, n = explicit_band_arcs(cost, delta, off, lo, hi, inf=1 << 28)
    a = np.array(arcs, dtype=np.int64)
    m = sp.csr_array((a[:, 2].astype(np.int32), (a[:, 0], a[:, 1])), shape=(n, n))
    return int(maximum_flow(m, s, t).flow_value)


def reduced_preflow_band(cost, delta, off, lo, hi):
    """A maximum preflow of the band graph in the solver's storage: node
    (p, lo(p) + j) at [x, y, j], the lateral arcs (p, j) -> (q, j - sh) for
    j > sh plus (p, 0) -> (q, 0), sh = delta + lo(q) - lo(p); by textbook
    FIFO push-relabel.  Returns (excess, sink residual, down flow, lateral
    flows, flow value), as reduced_preflow does."""
    nx, ny, K = cost.shape
    N = nx * ny * K
    t = N
    idx = lambda x, y, j: (x * ny + y) * K + j
    cz = lambda x, y, j: int(cost[x, y, lo[x, y] - off[x, y] + j])
    B = max(cz(x, y, 0) for x in range(nx) for y in range(ny)) + 1
    arcs, out, inn = [], [[] for _ in range(N)], [[] for _ in range(N + 1)]
    e = np.zeros(N, dtype=np.int64)

    def add(u, v, cap, kind):
        arcs.append([u, v, cap, 0, kind])
        out[u].append(len(arcs) - 1)
        inn[v].append(len(arcs) - 1)

    for x in range(nx):
        for y in range(ny):
            n = int(hi[x, y] - lo[x, y] + 1)
            for j in range(n):
                v = idx(x, y, j)
                w = cz(x, y, 0) - B if j == 0 else cz(x, y, j) - cz(x, y, j - 1)
                if w < 0:
                    e[v] = -w
                if w > 0:
                    add(v, t, w, ("t",))
                if j > 0:
                    add(v, v - 1, -1, ("d",))
                for k, (qx, qy) in enumerate(((x + 1, y), (x - 1, y), (x, y + 1), (x, y - 1))):
                    if not (0 <= qx < nx and 0 <= qy < ny):
                        continue
                    sh = int(delta + lo[qx, qy] - lo[x, y])
                    if j == 0 or j > sh:
                        add(v, idx(qx, qy, 0 if j == 0 else j - sh), -1, ("l", k))
    _fifo_push_relabel(N, t, e, arcs, out, inn)
    ts = np.zeros(N, dtype=np.int64)
    fd = np.zeros(N, dtype=np.int64)
    fl = np.zeros((4, N), dtype=np.int64)
    flow = 0
    for tail, head, cap, f, kind in arcs:
        if kind[0] == "t":
            ts[tail] = cap - f
            flow += f
        elif kind[0] == "d":
            fd[tail] = f
        else:
            fl[kind[1], tail] = f
    sh3 = (nx, ny, K)
    return (e.reshape(sh3).astype(np.int32), ts.reshape(sh3).astype(np.int32),
            fd.reshape(sh3).astype(np.int32), fl.reshape((4,) + sh3).astype(np.int32), flow)
