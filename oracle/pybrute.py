"""Pure-Python brute force for tiny graphs (a third, independent route).

TEST INFRASTRUCTURE ONLY.  Written with Python sets straight from the
definitions of Section 3.1 (the nine measures) and Section 4.2.1 (an
intermediate b counts only if d_b <= L); used to cross-check the C oracle.
"""
from __future__ import annotations

import math


def neighbour_sets(g):
    off, idx = g.offsets, g.indices
    return [set(int(x) for x in idx[off[v]:off[v + 1]]) for v in range(g.n)]


def measure(name, common, da, dc, degs):
    h = len(common)
    if name == "CN":
        return float(h)
    if name == "JC":
        return h / (da + dc - h)
    if name == "SI":
        return h / (da + dc)
    if name == "SC":
        return h / math.sqrt(da * dc)
    if name == "HP":
        return h / min(da, dc)
    if name == "HD":
        return h / max(da, dc)
    if name == "LHN":
        return h / (da * dc)
    if name == "AA":
        return sum(1.0 / math.log(degs[b]) for b in sorted(common))
    if name == "RA":
        return sum(1.0 / degs[b] for b in sorted(common))
    raise ValueError(name)


def all_candidates(g, L, name):
    """{(a, c): (h, score)} for every candidate pair a < c."""
    nb = neighbour_sets(g)
    degs = [len(s) for s in nb]
    lim = math.inf if L is None else L
    out = {}
    for a in range(g.n):
        for c in range(a + 1, g.n):
            if c in nb[a]:
                continue
            common = {b for b in nb[a] & nb[c] if degs[b] <= lim}
            if not common:
                continue
            out[(a, c)] = (len(common), measure(name, common, degs[a], degs[c], degs))
    return out


def second_order(g, L, a):
    """{c: h} for one vertex: every c != a, c not adjacent to a, h >= 1."""
    nb = neighbour_sets(g)
    degs = [len(s) for s in nb]
    lim = math.inf if L is None else L
    out = {}
    for c in range(g.n):
        if c == a or c in nb[a]:
            continue
        h = sum(1 for b in nb[a] & nb[c] if degs[b] <= lim)
        if h:
            out[c] = h
    return out
