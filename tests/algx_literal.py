"""Second, independent implementations used to pin the oracle (tests only).

* ``algx_sets`` - Algorithm X written directly on sets (no linked lists): the
  matrix is a dict column -> set of rows and a dict row -> list of columns;
  choosing a row deletes every column the row has a 1 in and every other row
  that has a 1 in one of those columns.  Same deterministic rules as the
  oracle (min-size uncovered primary column, lowest index on ties; rows in
  ascending order; first solution stops; budget tested before counting) and
  the same node trace hash, so status, node count, hash and colors must
  agree with the oracle's dancing-links search exactly.
* ``mark_sets`` - the conflict-marking descent (Algorithm 1's conflict
  candidates) on the same set representation: no backtracking, a column
  with no row left takes the row it lost last.  Must give the oracle's
  colors exactly.
* ``brute_force_colorable`` / ``min_conflicts`` - exhaustive k-colorings
  for tiny graphs.
"""
from __future__ import annotations

import itertools

import numpy as np

FEASIBLE, INFEASIBLE, BUDGET = 0, 1, 2
_FNV_OFFSET = 0xCBF29CE484222325
_FNV_PRIME = 0x100000001B3
_M64 = (1 << 64) - 1
NONE32 = 0xFFFFFFFF


def fnv1a_words(h: int, words) -> int:
    for w in words:
        for b in int(w).to_bytes(4, "little"):
            h ^= b
            h = (h * _FNV_PRIME) & _M64
    return h


def trace_step(h: int, words) -> int:
    """One counted node in the trace fingerprint: h * B + FNV-1a of the
    node's four u32 words (B the FNV prime; a trace starts at h = 0)."""
    return (h * _FNV_PRIME + fnv1a_words(_FNV_OFFSET, words)) & _M64


def trace_concat(h_first: int, h_second: int, n_second: int) -> int:
    """Fingerprint of a trace followed by another of n_second nodes."""
    return (h_first * pow(_FNV_PRIME, n_second, 1 << 64) + h_second) & _M64


def algx_sets(n: int, edges, k: int, budget: int, partner=None):
    """partner (n ints, -1 none): stitch-aware row order - a column whose
    node's partner is colored on the current path tries the row of that
    color first (if present), then the rest ascending."""
    edges = sorted((min(u, w), max(u, w)) for u, w in edges)
    rows = {}
    for v in range(n):
        inc = [e for e, (a, b) in enumerate(edges) if v in (a, b)]
        for c in range(k):
            rows[v * k + c] = [("p", v)] + [("s", e, c) for e in inc]
    cols = {}
    for r, cl in rows.items():
        for col in cl:
            cols.setdefault(col, set()).add(r)
    for v in range(n):
        cols.setdefault(("p", v), set())

    st = {"nodes": 0, "hash": 0, "status": None, "depth": 0}
    solution = []

    def choose_row(r):
        """Delete r's columns and every row clashing with r; return undo log."""
        removed = []
        for col in rows[r]:
            for other in cols[col]:
                for col2 in rows[other]:
                    if col2 != col:
                        cols[col2].discard(other)
            removed.append((col, cols.pop(col)))
        return removed

    def unchoose_row(r, removed):
        for col, members in reversed(removed):
            cols[col] = members
            for other in members:
                for col2 in rows[other]:
                    if col2 != col:
                        cols[col2].add(other)

    def search(depth, row_in):
        if st["nodes"] == budget:
            st["status"] = BUDGET
            st["depth"] = depth
            return
        st["nodes"] += 1
        open_prim = [v for v in range(n) if ("p", v) in cols]
        if not open_prim:
            st["hash"] = trace_step(st["hash"], [depth, row_in, NONE32, 0])
            st["status"] = FEASIBLE
            st["depth"] = depth
            return
        best = min(open_prim, key=lambda v: (len(cols[("p", v)]), v))
        size = len(cols[("p", best)])
        st["hash"] = trace_step(st["hash"], [depth, row_in, best, size])
        if size == 0:
            return
        order = sorted(cols[("p", best)])
        if partner is not None and partner[best] >= 0:
            colored = {row // k: row % k for row in solution}
            pref = colored.get(int(partner[best]))
            if pref is not None and best * k + pref in order:
                order.remove(best * k + pref)
                order.insert(0, best * k + pref)
        for r in order:
            solution.append(r)
            undo = choose_row(r)
            search(depth + 1, r)
            if st["status"] is not None:
                return
            unchoose_row(r, undo)
            solution.pop()

    search(0, NONE32)
    status = INFEASIBLE if st["status"] is None else st["status"]
    colors = np.full(n, -1, dtype=np.int8)
    if status == FEASIBLE:
        for r in solution:
            colors[r // k] = r % k
    depth = 0 if status == INFEASIBLE else st["depth"]
    return status, st["nodes"], st["hash"], depth, colors


def mark_sets(n: int, edges, k: int):
    """Conflict-marking descent on sets.  Columns as in algx_sets; every
    row deleted from a primary column is remembered as that column's last
    lost row.  Repeatedly take the fewest-rows primary column (lowest index
    on ties); include its lowest row, or, when it has none (a conflict
    candidate), the row it lost last.  Including a row deletes its columns
    that are still present, with every row that has a 1 in them."""
    edges = sorted((min(u, w), max(u, w)) for u, w in edges)
    rows = {}
    for v in range(n):
        inc = [e for e, (a, b) in enumerate(edges) if v in (a, b)]
        for c in range(k):
            rows[v * k + c] = [("p", v)] + [("s", e, c) for e in inc]
    cols = {}
    for r, cl in rows.items():
        for col in cl:
            cols.setdefault(col, set()).add(r)
    for v in range(n):
        cols.setdefault(("p", v), set())
    last = {}
    colors = np.full(n, -1, dtype=np.int8)
    while True:
        open_prim = [v for v in range(n) if ("p", v) in cols]
        if not open_prim:
            break
        best = min(open_prim, key=lambda v: (len(cols[("p", v)]), v))
        members = cols[("p", best)]
        r = min(members) if members else last[best]
        for col in rows[r]:
            if col not in cols:
                continue            # already covered: a marked conflict
            for other in cols.pop(col):
                for col2 in rows[other]:
                    if col2 != col and col2 in cols and other in cols[col2]:
                        cols[col2].discard(other)
                        if col2[0] == "p":
                            last[col2[1]] = other
        colors[r // k] = r % k
    return colors


def min_conflicts(n: int, edges, k: int) -> int:
    """Fewest monochromatic edges over all k-colorings (tiny graphs)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if n == 0 or len(e) == 0:
        return 0
    best = len(e)
    for chunk in _colorings(n, k):
        best = min(best, int((chunk[:, e[:, 0]] == chunk[:, e[:, 1]]).sum(axis=1).min()))
    return best


def brute_force_colorable(n: int, edges, k: int) -> bool:
    if n == 0:
        return True
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if len(e) == 0:
        return True
    for chunk in _colorings(n, k):
        ok = np.all(chunk[:, e[:, 0]] != chunk[:, e[:, 1]], axis=1)
        if ok.any():
            return True
    return False


def _colorings(n, k, chunk=1 << 16):
    it = itertools.product(range(k), repeat=n)
    while True:
        block = list(itertools.islice(it, chunk))
        if not block:
            return
        yield np.asarray(block, dtype=np.int8)


def random_graph(rng: np.random.Generator, n: int, p: float):
    return [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]


def complete(n):
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def cycle(n):
    return [(i, (i + 1) % n) for i in range(n)]


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return 10, outer + spokes + inner


def wheel(rim: int):
    """Hub 0 joined to a cycle 1..rim."""
    return rim + 1, [(0, i) for i in range(1, rim + 1)] + [
        (i, i % rim + 1) for i in range(1, rim + 1)]


def grotzsch():
    """Mycielskian of C5: 11 nodes, triangle-free, chromatic number 4."""
    c5 = [(i, (i + 1) % 5) for i in range(5)]
    e = list(c5)
    for u, v in c5:             # shadow u' = u + 5 joined to N(u)
        e.append((u + 5, v))
        e.append((v + 5, u))
    e += [(10, i + 5) for i in range(5)]
    return 11, e


def eq1_cost(n: int, edges, colors, partner=None) -> int:
    """10 per conflict edge colored alike + 1 per stitch pair colored
    differently (Eq. 1 with alpha = 0.1, scaled by 10)."""
    c = sum(10 for u, w in edges if colors[u] == colors[w])
    if partner is not None:
        c += sum(1 for v in range(n) if partner[v] > v and colors[v] != colors[partner[v]])
    return c


def bb_sets(n: int, edges, k: int, colors, budget: int, partner=None):
    """The Eq. 1 branch and bound restated without incremental state: every
    penalty is recounted from the current partial coloring.  Penalty of
    (u, c) = 10 x colored neighbours of color c + 1 when u's partner is
    colored otherwise; bound = cost + sum of the uncolored nodes' least
    penalties; node entry counted after the budget test; leaf replaces the
    incumbent when cheaper; prune at bound >= incumbent; branch on the
    uncolored node with the fewest colors free of colored neighbours of that
    color (lowest index on ties), colors ascending, a color skipped when
    bound - least(v) + penalty(v, c) >= incumbent.  Returns (colors, nodes,
    stopped, cost)."""
    nbrs = [set() for _ in range(n)]
    for u, w in edges:
        nbrs[u].add(w)
        nbrs[w].add(u)
    cur = {}
    best = {"cost": eq1_cost(n, edges, colors, partner), "colors": list(colors)}
    st = {"nodes": 0, "stopped": False, "cost": 0}
    if best["cost"] == 0:
        return np.asarray(colors, np.int8), 0, False, 0

    def pen(u, c):
        p = 10 * sum(1 for w in nbrs[u] if cur.get(w) == c)
        if partner is not None and partner[u] >= 0 and partner[u] in cur and cur[partner[u]] != c:
            p += 1
        return p

    def free(u):
        return sum(1 for c in range(k) if all(cur.get(w) != c for w in nbrs[u]))

    def rec():
        if st["nodes"] == budget:
            st["stopped"] = True
            return
        st["nodes"] += 1
        unc = [u for u in range(n) if u not in cur]
        if not unc:
            if st["cost"] < best["cost"]:
                best["cost"] = st["cost"]
                best["colors"] = [cur[u] for u in range(n)]
            return
        lb = st["cost"] + sum(min(pen(u, c) for c in range(k)) for u in unc)
        if lb >= best["cost"]:
            return
        v = min(unc, key=lambda u: (free(u), u))
        least = min(pen(v, c) for c in range(k))
        for c in range(k):
            p = pen(v, c)
            if lb - least + p >= best["cost"]:
                continue
            cur[v] = c
            st["cost"] += p
            rec()
            st["cost"] -= p
            del cur[v]
            if st["stopped"]:
                return

    rec()
    return np.asarray(best["colors"], np.int8), st["nodes"], st["stopped"], best["cost"]


def min_eq1_cost(n: int, edges, k: int, partner=None) -> int:
    """Least Eq. 1 cost (10 conflicts + stitches) over all k-colorings."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    pairs = ([(v, int(partner[v])) for v in range(n) if partner is not None and partner[v] > v])
    s = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    best = None
    for chunk in _colorings(n, k):
        cost = 10 * (chunk[:, e[:, 0]] == chunk[:, e[:, 1]]).sum(axis=1) if len(e) else 0
        cost = cost + ((chunk[:, s[:, 0]] != chunk[:, s[:, 1]]).sum(axis=1) if len(s) else 0)
        m = int(np.min(cost))
        best = m if best is None else min(best, m)
    return 0 if best is None else best
