"""Pins of oracle parts that the sweep and precompute tests do not reach:
the positive-definiteness guard of the local solve, the cubature columns
against their own target, the greedy pick against brute-force NNLS, and the
greedy colouring against its definition."""
import itertools

import numpy as np
import pytest

from oracle import correction as oc, mesh as omesh, sweep as osw


def test_local_solve_without_shift_is_the_plain_solve():
    A = np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]])
    b = np.array([1.0, -2.0, 0.5])
    np.testing.assert_allclose(osw.local_solve(A[None], b[None])[0], -np.linalg.solve(A, b), rtol=1e-14)


def test_local_solve_shifts_an_indefinite_system():
    """A has eigenvalues -1, 3, 4 and LDL^T pivots 1, -3, 4; the guard adds
    (|d_min| + 1e-6 |tr A|) I = 3.000006 I, after which every pivot clears
    1e-6 |tr A| (4.000006, about 3.000012, 7.000006): no doubling."""
    A = np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 4.0]])
    b = np.array([1.0, 1.0, 1.0])
    dx = osw.local_solve(A[None], b[None])[0]
    sigma = 3.0 + 6e-6
    # (A + sigma I) dx = -b in closed form: the 2x2 block has eigenvalues
    # 3 + sigma (along (1,1)) and sigma - 1 (along (1,-1)); b's block is along (1,1)
    expect = -np.array([1.0 / (3.0 + sigma), 1.0 / (3.0 + sigma), 1.0 / (4.0 + sigma)])
    np.testing.assert_allclose(dx, expect, rtol=1e-12)
    # a descent direction of the shifted (positive definite) model
    assert b @ dx < 0


def test_local_solve_shift_doubles_until_positive_definite():
    """Diagonal A = diag(-2, 5, 5): the first shift |d_min| + 1e-6 tr puts
    the smallest pivot exactly on the threshold, which it must exceed, so the
    shift is doubled once: 2 (2 + 8e-6)."""
    A = np.diag([-2.0, 5.0, 5.0])
    b = np.array([1.0, 1.0, 1.0])
    dx = osw.local_solve(A[None], b[None])[0]
    first = 2.0 + 8e-6
    d_first = -2.0 + first
    # whether the first shift passes depends on the rounding of d_first
    # against 8e-6; either way the result is one of the two shifted solves
    sig = first if d_first > 8e-6 else 2.0 * first
    np.testing.assert_allclose(dx, -b / (np.diag(A) + sig), rtol=1e-12)
    assert np.all(np.diag(A) + sig > 0)


def test_cubature_columns_sum_to_the_target(tiny):
    """Each remote vertex's term U-bar_{i,a}^T g_a is split evenly over the
    n_a elements around it, all of them eligible: the columns of all
    eligible elements add up to the right-hand side exactly."""
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl)
    sv = oc.RestSolver(H)
    lam, G, cid = oc.training_poses(mdl, H, sv)
    ring = omesh.one_ring(mdl.tets, mdl.nV)
    for k in (5, 123, 311):
        i = int(tab.verts[k])
        b, column, eligible = oc.cubature_system(mdl, ring, tab.U_full[k], G, cid, i)
        total = sum(column(s) for s in np.nonzero(eligible)[0])
        np.testing.assert_allclose(total, b, atol=1e-12 * np.abs(b).max())
        # and a column never involves vertex i or its one-ring
        assert not np.any(mdl.tets[eligible] == i)


def _nnls_brute(A, b):
    """Non-negative least squares by enumerating supports: the optimum is the
    unconstrained least-squares solution on some support that is itself
    non-negative; the smallest residual over those is the NNLS residual."""
    n = A.shape[1]
    best = np.linalg.norm(b)
    for r in range(1, n + 1):
        for sup in itertools.combinations(range(n), r):
            w, *_ = np.linalg.lstsq(A[:, sup], b, rcond=None)
            if np.all(w >= -1e-12):
                best = min(best, np.linalg.norm(A[:, sup] @ np.clip(w, 0, None) - b))
    return best


def test_greedy_pick_is_the_brute_force_argmin(tiny):
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl)
    sv = oc.RestSolver(H)
    lam, G, cid = oc.training_poses(mdl, H, sv)
    ring = omesh.one_ring(mdl.tets, mdl.nV)
    k = 200
    i = int(tab.verts[k])
    trace = []
    samples, weights, rel = oc.train_vertex(mdl, ring, tab.U_full[k], G, cid, i, S=3, n_cand=12, seed=5,
                                            trace=trace)
    b, column, _ = oc.cubature_system(mdl, ring, tab.U_full[k], G, cid, i)
    chosen = []
    for cands, res, pick in trace:
        brute = np.array([_nnls_brute(np.stack([column(s) for s in chosen + [c]], axis=1), b) for c in cands])
        np.testing.assert_allclose(res, brute, rtol=1e-8, atol=1e-12 * np.linalg.norm(b))
        best = brute.min()
        ties = [c for c, r in zip(cands, brute) if r <= best * (1 + 1e-8) + 1e-14]
        assert pick == min(ties)
        chosen.append(pick)
    assert list(samples[:len(chosen)]) == chosen


def test_greedy_colouring_is_the_smallest_free_colour(tiny):
    """Free vertices in ascending id take the smallest colour not used by a
    free one-ring neighbour of lower id; pinned vertices take none."""
    sc, mdl, tab = tiny
    ring = omesh.one_ring(mdl.tets, mdl.nV)
    col = omesh.greedy_coloring(ring, mdl.free)
    for v in range(mdl.nV):
        if not mdl.free[v]:
            assert col[v] == -1
            continue
        used = {int(col[a]) for a in ring[v] if a < v and mdl.free[a]}
        expect = next(c for c in itertools.count() if c not in used)
        assert col[v] == expect, v
    # and it is a valid colouring: no tet holds two free vertices of one colour
    for t in mdl.tets:
        cs = [col[a] for a in t if mdl.free[a]]
        assert len(cs) == len(set(cs))
