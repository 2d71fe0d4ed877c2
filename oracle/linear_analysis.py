"""Linear analysis of the vertex sweeps at the rest state (oracle, float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

At the rest state (x = X, every per-vertex rotation the identity, H = H-bar)
each sweep variant is a linear map of the residual: a Jacobi sweep moves
x by  -omega P g  with  P = sum_i S_i^T A_i^-1 C_i,  where A_i is the
variant's 3x3 local matrix and C_i (3 x N) the linear functional that
builds its right-hand side b_i = C_i g from the assembled residual.  The
error of a linear problem then evolves as  e <- (I - omega P H) e, and a
sweep converges on every error iff the spectral radius of that operator is
below one.  Coloured Gauss-Seidel applies the colour blocks of P one after
the other, so its operator is the product over colours of (I - omega P_c H).

This module builds (A_i, C_i) for the readings of the correction (Sec. 4.1
to Sec. 5; Eqs. reduced_local, reduced_h_g, cubature) and for the colour
group sub-problem of Sec. 8.1 (Parallel Implementation), so that every
figure of the convergence study is computed by committed code.  Only dense
linear algebra on small meshes (the 4x4x16 beam: 1,200 DOFs).

Variants (A_i / C_i):
  P0    plain vertex Newton: H_ii / S_i.
  R1    exact co-rotated subspace, all elements: U_i^T H U_i / U_i^T.
        At rest U_i^T H = B_i^-1 S_i (Eq. u), so P = H^-1 (one Newton step).
  R3    one-ring Galerkin terms exact plus the cubature samples of the
        precomputed tables (the library's CUBATURE variant).
  R2    literal Eq. cubature: H_ii plus the sampled (PSD) reduced Hessian /
        g_i plus the sampled remote gradient.
  R2D   damper reading of Sec. 5's closing remark: the sampled reduced
        Hessian damps the plain local solve, the sampled gradient is left
        out: H_ii + sum_s w_s U_s^T H_s U_s / S_i.
  Kk    U-bar_i truncated to the k-ring of i, used consistently
        (Galerkin): U~^T H U~ / U~^T.
  MCs   R3 with the remote part estimated by s elements drawn uniformly
        from the non-incident elements, each with weight (pool size) / s
        (an unbiased Monte Carlo cubature).  With every element drawn it is
        R1.
The colour-group reading (Sec. 8.1): for colour c the basis is constrained
to zero at every other vertex of c, U_c = H^-1 S_c^T (S_c H^-1 S_c^T)^-1,
and each vertex of c solves with the diagonal 3x3 block of the group Schur
complement S_c = U_c^T H U_c against b = U_c^T g.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

from . import correction as ocorr
from . import mesh as omesh
from . import rng as orng


class RestSystem:
    """Dense rest Hessian, its inverse and per-vertex U-bar blocks."""

    def __init__(self, model):
        self.model = model
        self.H = ocorr.rest_hessian(model).toarray()
        self.n = self.H.shape[0]
        self.nf = self.n // 3
        self.Hinv = np.linalg.inv(self.H)
        self.ring = omesh.one_ring(model.tets, model.nV)
        self.inc = omesh.incidence(model.tets, model.nV)
        self.color = omesh.greedy_coloring(self.ring, model.free)[model.free_ids]
        self.He = model.element_hessians(model.X)
        self.U = np.zeros((self.nf, self.n, 3))       # column block of U-bar_i on free DOFs
        for k in range(self.nf):
            s = slice(3 * k, 3 * k + 3)
            self.U[k] = self.Hinv[:, s] @ np.linalg.inv(self.Hinv[s, s])
        self._dist = None

    # ---- helpers -----------------------------------------------------------
    def dofs(self, a):
        """Free-DOF indices of vertex a (empty for a pinned vertex)."""
        f = self.model.free_index[a]
        return np.arange(3 * f, 3 * f + 3) if f >= 0 else np.zeros(0, dtype=np.int64)

    def elem_rows(self, Ucol, t):
        """(12, 3) rows of a basis column block at the corners of element t
        (zero rows at pinned corners)."""
        out = np.zeros((12, 3))
        for c in range(4):
            d = self.dofs(self.model.tets[t, c])
            if d.size:
                out[3 * c:3 * c + 3] = Ucol[d]
        return out

    def graph_distance(self):
        if self._dist is None:
            m = self.model
            r = [v for v in range(m.nV) for _ in self.ring[v]]
            c = [a for v in range(m.nV) for a in self.ring[v]]
            G = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(m.nV, m.nV)).tocsr()
            self._dist = csg.shortest_path(G, unweighted=True)[np.ix_(m.free_ids, m.free_ids)]
        return self._dist

    # ---- local maps ----------------------------------------------------------
    def plain(self):
        A = np.stack([self.H[3 * k:3 * k + 3, 3 * k:3 * k + 3] for k in range(self.nf)])
        C = np.zeros((self.nf, 3, self.n))
        for k in range(self.nf):
            C[k][:, 3 * k:3 * k + 3] = np.eye(3)
        return A, C

    def galerkin(self, Ucols):
        """A_i = U~_i^T H U~_i, C_i = U~_i^T for (nf, n, 3) column blocks."""
        A = np.einsum("kna,nm,kmb->kab", Ucols, self.H, Ucols)
        C = np.transpose(Ucols, (0, 2, 1)).copy()
        return A, C

    def exact(self):
        return self.galerkin(self.U)

    def truncated(self, k):
        d = self.graph_distance()
        mask = np.repeat(d <= k, 3, axis=1)          # [vertex i, dof]
        return self.galerkin(self.U * mask[:, :, None])

    def _one_ring_part(self, k):
        """One-ring Galerkin terms of vertex k: A over incident elements and
        C = S_i^T-part plus U-bar rows at free one-ring neighbours."""
        m = self.model
        v = m.free_ids[k]
        A = np.zeros((3, 3))
        for (t, _c) in self.inc[v]:
            Ue = self.elem_rows(self.U[k], t)
            A += Ue.T @ self.He[t] @ Ue
        C = np.zeros((3, self.n))
        C[:, 3 * k:3 * k + 3] = np.eye(3)
        for a in self.ring[v]:
            d = self.dofs(a)
            if d.size:
                C[:, d] += self.U[k][d].T
        return A, C

    def _remote_share(self, k, s, w):
        """Sampled element s with weight w for vertex k: its reduced Hessian
        term and its share of the remote gradient (corners outside the
        closed one-ring, each divided by its tet valence)."""
        m = self.model
        v = m.free_ids[k]
        Ue = self.elem_rows(self.U[k], s)
        Ah = w * Ue.T @ self.He[s] @ Ue
        C = np.zeros((3, self.n))
        nbar = set(int(a) for a in self.ring[v]) | {int(v)}
        for c in range(4):
            a = int(m.tets[s, c])
            d = self.dofs(a)
            if d.size and a not in nbar:
                C[:, d] += (w / m.valence[a]) * self.U[k][d].T
        return Ah, C

    def cubature(self, samples, weights, form="R3"):
        """(A, C) of R3, R2 or R2D for per-vertex samples/weights (nf, S)."""
        A0, C0 = self.plain()
        A = np.zeros((self.nf, 3, 3))
        C = np.zeros((self.nf, 3, self.n))
        for k in range(self.nf):
            Ah = np.zeros((3, 3))
            Cs = np.zeros((3, self.n))
            for s, w in zip(samples[k], weights[k]):
                if s < 0:
                    continue
                a_s, c_s = self._remote_share(k, int(s), float(w))
                Ah += a_s
                Cs += c_s
            if form == "R3":
                Ar, Cr = self._one_ring_part(k)
                A[k], C[k] = Ar + Ah, Cr + Cs
            elif form == "R2":
                A[k], C[k] = A0[k] + Ah, C0[k] + Cs
            elif form == "R2D":
                A[k], C[k] = A0[k] + Ah, C0[k]
            else:
                raise ValueError(form)
        return A, C

    def remote_pool(self, k):
        """Elements not containing vertex k with at least one free corner.
        Their reduced Hessians and remote-gradient shares, all at weight 1,
        complete the one-ring terms to U_i^T H U_i and U_i^T g exactly (the
        inertia is split into element shares, so H is a sum of element
        terms)."""
        m = self.model
        v = m.free_ids[k]
        return np.nonzero(~np.any(m.tets == v, axis=1) & np.any(m.free[m.tets], axis=1))[0]

    def monte_carlo(self, n_samp, seed=0):
        """Per-vertex uniform draws without replacement (SplitMix64 keyed by
        vertex), weight = pool size / draws.  n_samp=None takes every
        pool element at weight 1."""
        S = []
        W = []
        for k in range(self.nf):
            el = self.remote_pool(k)
            if n_samp is None or n_samp >= el.size:
                S.append(el)
                W.append(np.ones(el.size))
                continue
            key = orng.stream_key(seed, int(self.model.free_ids[k]), 0)
            order = np.argsort([orng.step((key + j * orng.GOLDEN) & orng.MASK) for j in range(el.size)],
                               kind="stable")
            S.append(el[order[:n_samp]])
            W.append(np.full(n_samp, el.size / n_samp))
        width = max(len(s) for s in S)
        samples = np.full((self.nf, width), -1, dtype=np.int64)
        weights = np.zeros((self.nf, width))
        for k in range(self.nf):
            samples[k, :len(S[k])] = S[k]
            weights[k, :len(W[k])] = W[k]
        return self.cubature(samples, weights, "R3")

    # ---- iteration operators ---------------------------------------------------
    def preconditioner(self, A, C):
        P = np.zeros((self.n, self.n))
        for k in range(self.nf):
            P[3 * k:3 * k + 3] = np.linalg.solve(A[k], C[k])
        return P

    def jacobi_operator(self, A, C, omega=1.0):
        return np.eye(self.n) - omega * self.preconditioner(A, C) @ self.H

    def gs_operator(self, A, C, omega=1.0):
        P = self.preconditioner(A, C)
        E = np.eye(self.n)
        for c in range(int(self.color.max()) + 1):
            idx = np.concatenate([np.arange(3 * k, 3 * k + 3) for k in np.nonzero(self.color == c)[0]])
            Pc = np.zeros_like(P)
            Pc[idx] = P[idx]
            E = (np.eye(self.n) - omega * Pc @ self.H) @ E
        return E

    def group_gs_operator(self, k_ring=None):
        """Coloured GS with the colour-group subspace (Sec. 8.1), exact or
        truncated to the k-ring of each vertex (then used in Galerkin form)."""
        E = np.eye(self.n)
        d = self.graph_distance() if k_ring is not None else None
        for c in range(int(self.color.max()) + 1):
            verts = np.nonzero(self.color == c)[0]
            idx = np.concatenate([np.arange(3 * k, 3 * k + 3) for k in verts])
            Sc = np.linalg.inv(self.Hinv[np.ix_(idx, idx)])
            Uc = self.Hinv[:, idx] @ Sc
            if d is not None:
                Uc = Uc * np.repeat(np.repeat(d[:, verts] <= k_ring, 3, axis=0), 3, axis=1)
            Pc = np.zeros((self.n, self.n))
            for j, k in enumerate(verts):
                Ui = Uc[:, 3 * j:3 * j + 3]
                Pc[3 * k:3 * k + 3] = np.linalg.solve(Ui.T @ self.H @ Ui, Ui.T)
            E = (np.eye(self.n) - Pc @ self.H) @ E
        return E


def spectral_radius(M):
    return float(np.max(np.abs(np.linalg.eigvals(M))))


def sweeps_to(rho, tol=1e-5):
    """Asymptotic sweep count to reduce an error by ``tol`` at rate rho."""
    return float(np.log(tol) / np.log(rho)) if rho < 1.0 else float("inf")
