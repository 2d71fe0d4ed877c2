"""Precomputed overshoot correction (oracle, float64).

Follows Sec. 4.1 (local perturbation subspace, Eqs. cms and phi), Sec. 4.3
(co-rotated subspace, Eq. tilde_phi), Sec. 5 (cubature, Eqs. cubature and
cubature_weight) and Sec. 6's full-coordinate precompute (Eqs.
cms_multiplier, block_inv and u).

  * Rest Hessian H-bar: the Hessian of the full incremental potential at the
    rest shape, M/h^2 + K(X), over free DOFs, without barriers (the paper
    does not say whether the mass term is included; with it, unpinned
    bodies stay non-singular).
  * U-bar_i = -H-bar^-1 S_i^T G-bar_i with G-bar_i = -(S_i H-bar^-1 S_i^T)^-1
    (Eq. u): one factorisation of H-bar, then 3 solves per vertex.  Row
    blocks U-bar_{i,a} (3x3) act as dx_a = U-bar_{i,a} dx_i; the row at i is
    the identity and rows at pinned vertices are zero.
  * Training poses (Sec. 5, last paragraph): eigenvectors of H-bar with the
    smallest eigenvalues.  Reading: n_T is the smallest n >= 8 with
    lambda_{n+1} / lambda_n > 1 + 1e-3 (capped at 16), so no eigenspace is
    cut; the linearised residual of pose t is g^(t) = H-bar v_t = lambda_t v_t.
  * Training target and columns (Eq. cubature_weight; its normalisation is
    garbled in the text).  Reading, for vertex i with closed one-ring
    Nbar(i) and tet valence n_a:
        tau_i^(t)   = sum_{a not in Nbar(i)} U-bar_{i,a}^T g_a^(t)
        c_{i,s}^(t) = sum_{a in s, a not in Nbar(i)} U-bar_{i,a}^T g_a^(t) / n_a
    (the remote part of the reduced gradient and an element's share of it);
    rows of pose t are divided by the RMS of |tau^(t')| over the poses t' of
    t's eigenvalue cluster, which equals the paper's per-pose norm for
    simple eigenvalues and does not depend on the basis chosen inside a
    degenerate eigenspace.
  * Greedy selection (Sec. 5): |S_i| rounds; each draws up to 64 candidate
    elements (see ``rng``) among eligible ones (not containing i, with a
    free corner outside Nbar(i)), solves NNLS on S_i plus the candidate,
    and keeps the candidate with the smallest residual (ties within
    1e-9 relative go to the lowest element id).  Final weights are the NNLS
    solution on S_i.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.optimize import nnls
from scipy.sparse.csgraph import reverse_cuthill_mckee

from . import mesh as omesh
from . import rng as orng


def rest_hessian(model):
    """H-bar over free DOFs: element Hessians at x = X (elastic + inertia)."""
    return model.assemble(model.element_hessians(model.X))


class RestSolver:
    """Cholesky factor of H-bar: dense for small systems, otherwise banded
    after a reverse Cuthill-McKee ordering (both LAPACK)."""

    def __init__(self, H, dense_max=6000):
        self.n = H.shape[0]
        self.dense = self.n <= dense_max
        if self.dense:
            self.cf = sla.cho_factor(H.toarray(), lower=True)
        else:
            perm = reverse_cuthill_mckee(H.tocsr(), symmetric_mode=True)
            Hp = H.tocsr()[perm][:, perm].tocoo()
            lo = Hp.row >= Hp.col
            r, c, v = Hp.row[lo], Hp.col[lo], Hp.data[lo]
            u = int((r - c).max())
            ab = np.zeros((u + 1, self.n))
            ab[r - c, c] = v
            self.perm = perm
            self.cb = sla.cholesky_banded(ab, lower=True)
            self.bandwidth = u

    def solve(self, B):
        B = np.asarray(B, dtype=np.float64)
        if self.dense:
            return sla.cho_solve(self.cf, B)
        Y = sla.cho_solve_banded((self.cb, True), B[self.perm])
        out = np.empty_like(Y)
        out[self.perm] = Y
        return out


def ubar_rows(model, solver, verts):
    """U-bar_i for each vertex i in ``verts`` as (len(verts), V, 3, 3) row
    blocks, via Eq. u: W = H-bar^-1 S_i^T, B = S_i W = -G-bar_i^-1,
    U-bar_i = W B^-1."""
    verts = np.asarray(verts, dtype=np.int64)
    n = solver.n
    fi = model.free_index[verts]
    if np.any(fi < 0):
        raise ValueError("U-bar is defined for free vertices only")
    RHS = np.zeros((n, 3 * verts.size))
    for k, f in enumerate(fi):
        RHS[3 * f:3 * f + 3, 3 * k:3 * k + 3] = np.eye(3)
    W = solver.solve(RHS)
    out = np.zeros((verts.size, model.nV, 3, 3))
    for k, f in enumerate(fi):
        Wk = W[:, 3 * k:3 * k + 3]
        B = Wk[3 * f:3 * f + 3]
        Uk = Wk @ np.linalg.inv(B)
        out[k, model.free_ids] = Uk.reshape(-1, 3, 3)
    return out


def training_poses(model, H, solver, n_min=8, n_max=16, gap=1e-3):
    """Smallest eigenpairs of H-bar, the gap-cut pose count and clusters.

    Returns (lam (n_T,), G (n_T, V, 3) with G[t] = lambda_t v_t, cluster id
    per pose)."""
    n = H.shape[0]
    k = min(n_max + 1, n - 1)
    if n <= 6000:
        lam, vec = sla.eigh(H.toarray(), subset_by_index=[0, k - 1])
    else:
        op = spla.LinearOperator((n, n), matvec=lambda v: solver.solve(v), dtype=np.float64)
        lam, vec = spla.eigsh(H, k=k, sigma=0.0, which="LM", OPinv=op, tol=1e-13)
        o = np.argsort(lam)
        lam, vec = lam[o], vec[:, o]
    nT = min(n_max, k)
    for m in range(n_min, min(n_max, k - 1) + 1):
        if lam[m] / lam[m - 1] > 1.0 + gap:
            nT = m
            break
    lam, vec = lam[:nT], vec[:, :nT]
    cid = np.zeros(nT, dtype=np.int64)
    for t in range(1, nT):
        cid[t] = cid[t - 1] + (1 if lam[t] / lam[t - 1] > 1.0 + gap else 0)
    G = np.zeros((nT, model.nV, 3))
    for t in range(nT):
        G[t, model.free_ids] = (lam[t] * vec[:, t]).reshape(-1, 3)
    return lam, G, cid


def _nnls(A, b):
    w, r = nnls(A, b, maxiter=50 * max(1, A.shape[1]))
    return w, float(r)


def cubature_system(model, ring, U, G, cid, i):
    """The NNLS system of Eq. cubature_weight for vertex i.

    Returns (b, column, eligible): the normalised remote reduced gradients
    over the poses (the right-hand side, 3 n_T entries), a function giving
    element s's normalised share of them (a column), and the mask of
    eligible elements (not containing i, with a free corner outside the
    closed one-ring).  Every remote vertex a is shared by the n_a elements
    around it, all eligible, so the columns of all eligible elements sum to
    b."""
    tets = model.tets
    nbar = np.zeros(model.nV, dtype=bool)
    nbar[ring[i]] = True
    nbar[i] = True
    outside = model.free & ~nbar
    # remote reduced gradient per pose (the plain definition)
    tau = np.einsum("vji,tvj->ti", U[outside], G[:, outside])          # (n_T, 3)
    # per-cluster RMS normalisation, floored at 1e-3 of the largest cluster
    # RMS at i (a cluster far below the others is near the round-off of the
    # sums above and is not scaled up past 1e3 x)
    nT = tau.shape[0]
    ncl = int(cid.max()) + 1
    rms = np.array([np.sqrt(np.mean(np.sum(tau[cid == c] ** 2, axis=1))) for c in range(ncl)])
    if rms.max() > 0:
        scale = 1.0 / np.maximum(rms[cid], 1e-3 * rms.max())
    else:
        scale = np.zeros(nT)
    b = (tau * scale[:, None]).ravel()
    coef = np.where(outside[tets], 1.0 / model.valence[tets], 0.0)     # (T,4)
    contains_i = np.any(tets == i, axis=1)
    eligible = (~contains_i) & np.any(coef > 0, axis=1)

    def column(s):
        c = np.zeros((nT, 3))
        for k in range(4):
            if coef[s, k] > 0:
                a = tets[s, k]
                c += coef[s, k] * (G[:, a, :] @ U[a])                    # (U^T g)^T = g^T U
        return (c * scale[:, None]).ravel()

    return b, column, eligible


def train_vertex(model, ring, U, G, cid, i, S=4, n_cand=64, seed=0, trace=None):
    """Greedy NNLS cubature for vertex i.

    U: (V,3,3) rows of U-bar_i.  Returns (samples (S,), weights (S,),
    relative residual).  Missing samples (fewer eligible elements than S)
    are -1 with weight 0.  If ``trace`` is a list, each round appends
    (candidates, their NNLS residuals, the pick)."""
    b, column, eligible = cubature_system(model, ring, U, G, cid, i)
    bnorm = float(np.linalg.norm(b))
    chosen, cols = [], []
    for k in range(S):
        cands = orng.draw_candidates(seed, i, k, model.nT, eligible, chosen, n_cand)
        if not cands:
            break
        res = []
        for s in cands:
            A = np.stack(cols + [column(s)], axis=1)
            res.append(_nnls(A, b)[1])
        res = np.array(res)
        best = res.min()
        tie = res <= best + 1e-9 * best + 1e-15 * bnorm
        s_best = min(c for c, t in zip(cands, tie) if t)
        if trace is not None:
            trace.append((list(cands), res.copy(), s_best))
        chosen.append(s_best)
        cols.append(column(s_best))
    samples = np.full(S, -1, dtype=np.int64)
    weights = np.zeros(S)
    rel = 0.0
    if chosen:
        A = np.stack(cols, axis=1)
        w, r = _nnls(A, b)
        samples[:len(chosen)] = chosen
        weights[:len(chosen)] = w
        rel = r / bnorm if bnorm > 0 else 0.0
    return samples, weights, rel


class Tables:
    """Per-vertex correction data for a set of free vertices."""

    def __init__(self, model, verts, ring, U_full, samples, weights, fit_res, lam, cid):
        self.verts = np.asarray(verts, dtype=np.int64)
        self.pos = {int(v): k for k, v in enumerate(self.verts)}
        self.ring = ring
        self.samples = samples
        self.weights = weights
        self.fit_res = fit_res
        self.lam = lam
        self.cid = cid
        n, S = samples.shape
        # one-ring rows (free neighbours only; pinned rows are zero)
        self.nbr = [ring[v][model.free[ring[v]]] for v in self.verts]
        self.U_nbr = [U_full[k][self.nbr[k]] for k in range(n)]
        tets = model.tets
        self.U_samp = np.zeros((n, S, 4, 3, 3))
        self.gcoef = np.zeros((n, S, 4))
        self.U_full = U_full
        for k, v in enumerate(self.verts):
            nbar = set(int(a) for a in ring[v]) | {int(v)}
            for j in range(S):
                s = samples[k, j]
                if s < 0:
                    continue
                for c in range(4):
                    a = int(tets[s, c])
                    self.U_samp[k, j, c] = U_full[k][a]
                    if model.free[a] and a not in nbar:
                        self.gcoef[k, j, c] = weights[k, j] / model.valence[a]


def precompute(model, verts=None, S=4, n_cand=64, seed=0, keep_full=True, solver=None):
    """Full precompute for ``verts`` (default: all free vertices)."""
    ring = omesh.one_ring(model.tets, model.nV)
    H = rest_hessian(model)
    if solver is None:
        solver = RestSolver(H)
    lam, G, cid = training_poses(model, H, solver)
    verts = model.free_ids if verts is None else np.asarray(verts, dtype=np.int64)
    U_full = np.zeros((verts.size, model.nV, 3, 3))
    samples = np.full((verts.size, S), -1, dtype=np.int64)
    weights = np.zeros((verts.size, S))
    fit = np.zeros(verts.size)
    chunk = 64
    for c0 in range(0, verts.size, chunk):
        vs = verts[c0:c0 + chunk]
        U = ubar_rows(model, solver, vs)
        U_full[c0:c0 + vs.size] = U
        for k, v in enumerate(vs):
            samples[c0 + k], weights[c0 + k], fit[c0 + k] = train_vertex(
                model, ring, U[k], G, cid, int(v), S=S, n_cand=n_cand, seed=seed)
    tab = Tables(model, verts, ring, U_full, samples, weights, fit, lam, cid)
    tab.G = G  # training-pose gradients, for rebuilding a vertex's NNLS system
    if not keep_full:
        tab.U_full = None
    return tab
