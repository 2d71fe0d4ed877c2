"""Mesh adjacency and greedy vertex colouring (oracle).

Sub-problems sit at vertices (Sec. 8.1), so each needs its incident tets and
its one-ring (vertices sharing a tet).  Gauss-Seidel groups independent
sub-problems by graph colouring (Sec. 8.1): two vertices of one colour never
share a tet.  Reading: greedy colouring of the free vertices in ascending id
order, each taking the smallest colour unused by its already-coloured free
one-ring neighbours.
"""
import numpy as np


def incidence(tets, nV):
    """For every vertex, the ascending list of (tet, corner) pairs touching it."""
    inc = [[] for _ in range(nV)]
    for t in range(tets.shape[0]):
        for c in range(4):
            inc[int(tets[t, c])].append((t, c))
    return inc


def one_ring(tets, nV):
    """For every vertex, the ascending array of other vertices sharing a tet."""
    nb = [set() for _ in range(nV)]
    for t in range(tets.shape[0]):
        vs = [int(v) for v in tets[t]]
        for a in vs:
            for b in vs:
                if a != b:
                    nb[a].add(b)
    return [np.array(sorted(s), dtype=np.int64) for s in nb]


def greedy_coloring(ring, free):
    """colour[v] for free v (-1 for pinned), greedy in index order."""
    nV = len(ring)
    color = np.full(nV, -1, dtype=np.int64)
    for v in range(nV):
        if not free[v]:
            continue
        used = {int(color[a]) for a in ring[v] if free[a] and color[a] >= 0}
        c = 0
        while c in used:
            c += 1
        color[v] = c
    return color
