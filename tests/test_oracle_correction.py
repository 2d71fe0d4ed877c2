"""Pins of the oracle's precompute (full-coordinate U-bar, training poses,
greedy NNLS cubature) against the paper's identities and brute force."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import correction as oc, rng as orng


def test_ubar_constraint_and_equilibrium(tiny):
    """S_i U-bar_i = I (constraint of Eq. cms_constraint) and H-bar U-bar_i
    vanishes away from i (the incremental equilibria of Eq. cms)."""
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl)
    for k in [0, 57, 199, 399]:
        i = tab.verts[k]
        U = tab.U_full[k][mdl.free_ids].reshape(-1, 3)
        f = mdl.free_index[i]
        np.testing.assert_allclose(U[3 * f:3 * f + 3], np.eye(3), atol=1e-12)
        HU = H @ U
        HU[3 * f:3 * f + 3] = 0
        assert np.abs(HU).max() < 1e-9 * np.abs(H).max()


def test_ubar_equals_schur_form_by_dense_inverse(tiny):
    """Eq. u (full coordinates) equals Eq. phi's [I; -H_CC^-1 H_Ci] computed
    by brute-force dense inversion of H_CC."""
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl).toarray()
    n = H.shape[0]
    for k in [3, 150]:
        f = mdl.free_index[tab.verts[k]]
        i_d = np.arange(3 * f, 3 * f + 3)
        c_d = np.setdiff1d(np.arange(n), i_d)
        UC = -np.linalg.inv(H[np.ix_(c_d, c_d)]) @ H[np.ix_(c_d, i_d)]
        U = tab.U_full[k][mdl.free_ids].reshape(-1, 3)
        np.testing.assert_allclose(U[c_d], UC, atol=1e-10)


def test_schur_complement_identity(tiny):
    """U-bar^T H-bar U-bar = B^-1 = -G-bar (Eq. block_inv): the exact local
    Hessian is the Schur complement."""
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl).toarray()
    Hinv = np.linalg.inv(H)
    k = 77
    f = mdl.free_index[tab.verts[k]]
    U = tab.U_full[k][mdl.free_ids].reshape(-1, 3)
    B = Hinv[3 * f:3 * f + 3, 3 * f:3 * f + 3]
    np.testing.assert_allclose(U.T @ H @ U, np.linalg.inv(B), rtol=1e-9)


def test_training_poses_are_eigenpairs_and_gap_cut(tiny):
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl).toarray()
    w = sla.eigh(H, eigvals_only=True, subset_by_index=[0, 17])
    nT = tab.lam.size
    assert 8 <= nT <= 16
    np.testing.assert_allclose(tab.lam, w[:nT], rtol=1e-10)
    assert w[nT] / w[nT - 1] > 1 + 1e-3 or nT == 16


def test_training_target_closed_form(tiny):
    """tau_i = B^-1 (H-bar^-1 g)_i - sum_{a in Nbar(i)} U-bar_{i,a}^T g_a for
    any g, since U-bar_{i,a}^T = B^-1 (H-bar^-1)_{i,a} (Eq. u); for an exact
    eigenvector (g = lambda v) the first term is B^-1 v_i."""
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl)
    sv = oc.RestSolver(H)
    lam, G, cid = oc.training_poses(mdl, H, sv)
    k = 123
    i = int(tab.verts[k])
    U = tab.U_full[k]
    nbar = np.zeros(mdl.nV, bool); nbar[tab.ring[i]] = True; nbar[i] = True
    out = mdl.free & ~nbar
    tau_def = np.einsum("vji,tvj->ti", U[out], G[:, out])
    f = mdl.free_index[i]
    Binv = np.linalg.inv(sv.solve(np.eye(H.shape[0])[:, 3 * f:3 * f + 3])[3 * f:3 * f + 3])
    V = G[:, i, :] / lam[:, None]
    inner = np.einsum("vji,tvj->ti", U[nbar & mdl.free], G[:, nbar & mdl.free])
    np.testing.assert_allclose(tau_def, V @ Binv.T - inner, atol=1e-9 * np.abs(tau_def).max())
    # arbitrary gradients (not eigenvectors): only the H-bar^-1 g form holds
    rng = np.random.default_rng(5)
    Gr = np.zeros_like(G)
    Gr[:, mdl.free_ids] = rng.standard_normal((G.shape[0], mdl.free_ids.size, 3))
    tau_r = np.einsum("vji,tvj->ti", U[out], Gr[:, out])
    HiG = np.stack([mdl.from_free(sv.solve(mdl.to_free(Gr[t])))[i] for t in range(G.shape[0])])
    inner_r = np.einsum("vji,tvj->ti", U[nbar & mdl.free], Gr[:, nbar & mdl.free])
    np.testing.assert_allclose(tau_r, HiG @ Binv.T - inner_r, atol=1e-9 * np.abs(tau_r).max())
    assert np.abs(tau_r - (Gr[:, i, :] @ Binv.T - inner_r)).max() > 1e-3 * np.abs(tau_r).max()


def _nnls_brute(A, b):
    """NNLS by enumerating supports: the best strictly-positive unconstrained
    least-squares solution over all column subsets."""
    best = (np.linalg.norm(b), np.zeros(A.shape[1]))
    for r in range(1, A.shape[1] + 1):
        for sub in itertools.combinations(range(A.shape[1]), r):
            w, *_ = np.linalg.lstsq(A[:, sub], b, rcond=None)
            if np.all(w > 0):
                full = np.zeros(A.shape[1]); full[list(sub)] = w
                res = np.linalg.norm(A @ full - b)
                if res < best[0]:
                    best = (res, full)
    return best


def test_nnls_step_matches_support_enumeration():
    rng = np.random.default_rng(5)
    for _ in range(20):
        A = rng.standard_normal((24, 4)); b = rng.standard_normal(24)
        w, r = oc._nnls(A, b)
        rb, wb = _nnls_brute(A, b)
        assert abs(r - rb) < 1e-10
        np.testing.assert_allclose(w, wb, atol=1e-9)


def test_cubature_weights_nonnegative_and_deterministic(tiny):
    sc, mdl, tab = tiny
    assert np.all(tab.weights >= 0)
    assert np.all(tab.samples >= 0)
    # no sample touches its own vertex
    for k, v in enumerate(tab.verts):
        assert not np.any(mdl.tets[tab.samples[k]] == v)
    H = oc.rest_hessian(mdl)
    sv = oc.RestSolver(H)
    lam, G, cid = oc.training_poses(mdl, H, sv)
    for k in [5, 260]:
        U = oc.ubar_rows(mdl, sv, [tab.verts[k]])[0]
        s, w, r = oc.train_vertex(mdl, tab.ring, U, G, cid, int(tab.verts[k]), S=4, n_cand=64, seed=0)
        assert np.array_equal(s, tab.samples[k])
        np.testing.assert_allclose(w, tab.weights[k], rtol=1e-12)


def test_candidate_stream_is_splitmix64():
    # first outputs of SplitMix64 seeded with 0 (published reference values)
    s = 0
    out = []
    for _ in range(3):
        s = (s + orng.GOLDEN) & orng.MASK
        out.append(orng._fin(s))
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert orng.step(0) == 0xE220A8397B1DCDAF


def test_cluster_normalisation_caps_small_clusters(tiny):
    """Reading of Eq. cubature_weight's normalisation: each pose cluster's
    rows of the remote reduced gradient (and of every column) are divided by
    the larger of the cluster's RMS at the vertex and 1e-3 of the largest
    cluster RMS.  Every cluster of the tiny beam's vertex is within that range
    (unit RMS).  A cluster scaled by 1e-2 keeps unit RMS and the system is
    unchanged; one scaled by 1e-7 is not scaled back up: its rows keep their
    direction at an RMS far below one, and the other rows are unchanged."""
    sc, mdl, tab = tiny
    H = oc.rest_hessian(mdl)
    sv = oc.RestSolver(H)
    lam, G, cid = oc.training_poses(mdl, H, sv)
    k = 123
    i = int(tab.verts[k])
    U = tab.U_full[k]
    b0, col0, elig = oc.cubature_system(mdl, tab.ring, U, G, cid, i)
    s = int(np.nonzero(elig)[0][0])
    rows = np.repeat(cid == 0, 3)
    rms = lambda v: np.sqrt(np.mean(v.reshape(-1, 3).__pow__(2).sum(1)))
    ncl = int(cid.max()) + 1
    assert all(rms(b0[np.repeat(cid == c, 3)]) == pytest.approx(1.0) for c in range(ncl))
    for scale in (1e-2, 1e-7):
        Gs = G.copy()
        Gs[cid == 0] *= scale
        b, col, _ = oc.cubature_system(mdl, tab.ring, U, Gs, cid, i)
        np.testing.assert_allclose(b[~rows], b0[~rows], rtol=1e-12)
        np.testing.assert_allclose(col(s)[~rows], col0(s)[~rows], rtol=1e-12, atol=1e-300)
        if scale == 1e-2:
            np.testing.assert_allclose(b, b0, rtol=1e-9, atol=1e-12)
        else:
            ratio = b[rows] / b0[rows]
            assert np.ptp(ratio) <= 1e-9 * np.abs(ratio).max()   # same direction, one factor
            assert 0.0 < rms(b[rows]) < 1e-2
            np.testing.assert_allclose(col(s)[rows], col0(s)[rows] * ratio[0], rtol=1e-9,
                                       atol=1e-12 * np.abs(col0(s)).max())
