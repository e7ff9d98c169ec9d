"""Test helper: the components of a layout graph as the oracle's own
front-end splits them (simplification, components, BFS local numbering),
as local edge lists.  Only calls the oracle."""
from __future__ import annotations

import numpy as np

import oracle


def components(g: "oracle.Graph", k: int, simplify: bool = True):
    """(sizes, edge_lists, global ids per component in local order)."""
    _, comp_of, comps = oracle.simplify(g, k, simplify)
    adj = [[] for _ in range(g.num_nodes)]
    for a, b in g.ce.tolist():
        if comp_of[a] >= 0 and comp_of[b] >= 0:
            adj[a].append(b)
            adj[b].append(a)
    sizes, edge_lists = [], []
    for c in comps:
        loc = {int(v): i for i, v in enumerate(c.tolist())}
        e = [(loc[v], loc[u]) for v in c.tolist() for u in adj[v] if loc[v] < loc[u]]
        sizes.append(len(c))
        edge_lists.append(np.asarray(e, dtype=np.int32).reshape(-1, 2))
    return sizes, edge_lists, comps
