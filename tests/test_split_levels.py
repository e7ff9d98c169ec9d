"""The level-synchronous reading of the simplification and sub-graph split
(Sec. 2.2; Algorithm 1's sub-graphs) that the device split is built on,
modelled in plain Python and checked against the oracle's sequential
definitions (FIFO peeling, components by smallest id, BFS numbering):

* FIFO levels are the rounds of synchronous peeling; a node outside levels
  0..L with d conflict neighbours is queued by its (d - k + 1)-th removed
  neighbour (its trigger), which, if it lies in level L, is the one of rank
  d - k + 1 - (neighbours in earlier levels) among its level-L neighbours by
  queue position; level L+1 is ordered by (trigger position, position in
  the trigger's ascending list);
* a BFS node of level d+1 is reached from its numbered neighbour of
  smallest local position; level d+1 is ordered per component by (parent
  position, id);
* components are the union-find classes with the smallest id as root.
"""
import math

import numpy as np

import oracle
import workload
from algx_literal import random_graph


def level_split(n, edges, k, simplify):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    adj = [sorted(x) for x in adj]
    qpos, lvl, trig, queue = [-1] * n, [-1] * n, [-1] * n, []
    if simplify:
        for v in range(n):
            if len(adj[v]) < k:
                qpos[v], lvl[v] = len(queue), 0
                queue.append(v)
    lo, hi, level = 0, len(queue), 0
    while lo < hi:
        cand = sorted({w for u in queue[lo:hi] for w in adj[u] if qpos[w] < 0})
        for w in cand:
            need = len(adj[w]) - k + 1
            before = sum(1 for x in adj[w] if 0 <= lvl[x] < level)
            at = sorted((qpos[x], x) for x in adj[w] if lvl[x] == level)
            trig[w] = at[need - before - 1][1] if before + len(at) >= need else -1
        nxt = hi
        for u in queue[lo:hi]:
            for w in adj[u]:
                if qpos[w] < 0 and trig[w] == u:
                    qpos[w], lvl[w] = nxt, level + 1
                    queue.append(w)
                    nxt += 1
        lo, hi, level = hi, nxt, level + 1
    core = [v for v in range(n) if lvl[v] < 0]
    parent = {v: v for v in core}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x
    for v in core:
        for w in adj[v]:
            if w > v and lvl[w] < 0:
                ra, rb = find(v), find(w)
                if ra != rb:
                    parent[max(ra, rb)] = min(ra, rb)
    roots = sorted(v for v in core if find(v) == v)
    cid = {r: i for i, r in enumerate(roots)}
    comp_of = [-1] * n
    for v in core:
        comp_of[v] = cid[find(v)]
    local = [-1] * n
    comps = [[r] for r in roots]
    for r in roots:
        local[r] = 0
    frontier = list(roots)
    while frontier:
        cand = {w for u in frontier for w in adj[u] if lvl[w] < 0 and local[w] < 0}
        par = {w: min((local[x], x) for x in adj[w] if lvl[x] < 0 and local[x] >= 0)[1]
               for w in cand}
        nf = []
        for u in frontier:   # ordered by (component, position)
            for w in adj[u]:
                if lvl[w] < 0 and local[w] < 0 and par.get(w) == u:
                    local[w] = len(comps[comp_of[u]])
                    comps[comp_of[u]].append(w)
                    nf.append(w)
        frontier = nf
    return queue, comp_of, comps


def same(n, edges, k, simplify):
    ce = np.array(edges, np.int32).reshape(-1, 2)
    rem, comp_of, comps = oracle.simplify(oracle.Graph(n, ce, np.zeros((0, 2), np.int32)), k,
                                          simplify)
    q, co, cs = level_split(n, [tuple(map(int, e)) for e in ce], k, simplify)
    assert list(rem) == q
    assert list(comp_of) == co
    assert [list(c) for c in comps] == cs


def test_random_graphs():
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = int(rng.integers(1, 60))
        k = int(rng.integers(2, 5))
        e = random_graph(rng, n, float(rng.uniform(0.02, 0.3)))
        same(n, e, k, bool(rng.integers(0, 2)))


def test_layouts_and_chains():
    for nr, seed in ((300, 0), (3000, 1)):
        side = round(3000 * math.sqrt(nr / 300))
        r, _ = workload.generate(nr, side, seed)
        for split in (0, 120):
            g = oracle.build_graph(r, 80, split)
            same(g.num_nodes, g.ce, 3, True)
    same(41, [(i, i + 1) for i in range(40)], 2, True)          # a path, peeled pairwise
    same(30, [(i, (i + 1) % 30) for i in range(30)], 2, True)   # a cycle, BFS depth 15
