"""Per-vertex local solves and parallel sweeps (oracle, float64).

Sub-problem = one vertex with N_i = 3 DOFs and an analytic 3x3 Newton solve
(Sec. 8.1).  The global-aware local system (Eqs. reduced_local and
reduced_h_g) is the Galerkin projection of the Newton system onto the
perturbation subspace U_i:

    (U_i^T H U_i) dx_i = -U_i^T g,

which, with the exact subspace of Eq. phi, is the i-block of the Newton step
(Sec. 4.2).  Row blocks of the co-rotated subspace (Eq. tilde_phi) are
Phi_{i,a} = R_a U-bar_{i,a} R_i^T with per-vertex rotations R_a from the
polar decomposition of a per-vertex deformation gradient.

Variants (same enum as the HIP library):
  P0  plain vertex Newton (no correction): A_i = H_ii, b_i = g_i.
  R0  exact subspace from the current Hessian, all elements.
  R1  co-rotated precomputed subspace, all elements (exact assembly).
  R3  co-rotated subspace; incident elements and one-ring gradients exact,
      remote elements by cubature (Eq. cubature):
        A_i = sum_{e ni i} Phi_e^T H_e Phi_e + H^B_i
              + sum_{s in S_i} w_s Phi_s^T H_s Phi_s
        b_i = g_i + sum_{a in N(i)} Phi_{i,a}^T g_a
              + sum_{s in S_i} w_s sum_{a in s, a not in Nbar(i)} Phi_{i,a}^T g_a / n_a
      Reading: the paper's sampled "[grad E_C]_e" is taken as the assembled
      residual at e's corners shared by valence, so that b_i = 0 at the
      solution and the solution is a fixed point; with every element not
      containing i sampled at weight 1 this is exactly R1 (the cubature
      candidates are those with a free corner outside Nbar(i); the other
      non-incident elements add Hessian terms only).
  R2, R2G1, R2D  the literal H_ii-plus-sampled forms (see ``r2_systems``);
      R2D is the library's DAMPER variant.
  RX  the exact co-rotated subspace in the literal form of Eq. local_newton
      (the library's EXACT variant): with Eq. relation's derivatives of E_C,
        A_i = H_ii + sum_{a in N(i)} H_{i,a} Phi_{i,a}   (symmetrised)
        b_i = sum_a Phi_{i,a}^T g_a                       (every free vertex)
      The Hessian term needs the one-ring only (H_{i,a} vanishes beyond it);
      the gradient term runs over the whole mesh, exactly.  At rest it is
      the i-block of the Newton step (Sec. 4.2).

Readings of the per-vertex rotation (Sec. 4.3 names a polar decomposition of
a per-vertex deformation gradient without defining the latter): F-bar_a is
the volume-weighted mean of the F_e of the tets around a, and R_a =
U diag(1, 1, det(U V^T)) V^T from the SVD F-bar_a = U Sigma V^T.

The local 3x3 solve is a Cholesky solve; if A_i is not positive definite
(a non-positive LDL^T pivot, or one below 1e-6 tr A_i), A_i is shifted by
(|d_min| + 1e-6 tr A_i) I, doubling the shift until it is.

Jacobi: every free vertex solves from the same iterate.  Gauss-Seidel
("fresh" reading): colours in ascending order; before each colour the
gradients and rotations are recomputed at the current iterate, then all
vertices of that colour solve (from the same iterate) and move.  R2D is the
exception for rotations: they are those of the sweep's starting iterate.
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import correction as ocorr

P0, R0, R1, R2, R2G1, R2D, R3, RX = "P0", "R0", "R1", "R2", "R2G1", "R2D", "R3", "RX"


def polar(F):
    U, _, Vt = np.linalg.svd(F)
    d = np.sign(np.linalg.det(U @ Vt))
    d = np.where(d == 0, 1.0, d)
    D = np.ones(F.shape[:-1])
    D[..., 2] = d
    return np.einsum("...ij,...j,...jk->...ik", U, D, Vt)


def vertex_rotations(model, x):
    F = model.deformation_gradient(x)
    Fbar = np.zeros((model.nV, 3, 3))
    np.add.at(Fbar, model.tets.ravel(), np.repeat(model.vol[:, None, None] * F, 4, axis=0))
    wsum = np.zeros(model.nV)
    np.add.at(wsum, model.tets.ravel(), np.repeat(model.vol, 4))
    Fbar /= wsum[:, None, None]
    return polar(Fbar)


def phase1(model, x, z):
    """Assembled gradient g (pinned rows zero) and per-vertex rotations R."""
    return model.gradient(x, z), vertex_rotations(model, x)


def local_solve(A, b):
    """dx = -A^-1 b for a stack of 3x3 systems with the PD guard above."""
    A = np.array(A, dtype=np.float64)
    out = np.empty(b.shape)
    for k in range(A.shape[0]):
        M = A[k]
        tr = np.trace(M)
        shift = 0.0
        for _ in range(60):
            Ms = M + shift * np.eye(3)
            d = _ldl_pivots(Ms)
            if d.min() > 1e-6 * abs(tr):
                break
            shift = (abs(d.min()) + 1e-6 * abs(tr)) if shift == 0.0 else 2.0 * shift
        out[k] = -np.linalg.solve(Ms, b[k])
    return out


def _ldl_pivots(M):
    d0 = M[0, 0]
    if d0 == 0:
        return np.array([0.0, 0.0, 0.0])
    l10, l20 = M[1, 0] / d0, M[2, 0] / d0
    d1 = M[1, 1] - l10 * l10 * d0
    if d1 == 0:
        return np.array([d0, 0.0, 0.0])
    l21 = (M[2, 1] - l20 * l10 * d0) / d1
    d2 = M[2, 2] - l20 * l20 * d0 - l21 * l21 * d1
    return np.array([d0, d1, d2])


class _Ell:
    """Padded per-vertex index arrays for vectorised R3 assembly."""

    def __init__(self, model, tab, inc):
        n = tab.verts.size
        K = max(1, max(len(a) for a in tab.nbr))
        M = max(len(inc[int(v)]) for v in tab.verts)
        S = tab.samples.shape[1]
        self.K, self.M, self.S = K, M, S
        self.nbr = np.zeros((n, K), dtype=np.int64)
        self.nbr_ok = np.zeros((n, K), dtype=bool)
        self.U_nbr = np.zeros((n, K, 3, 3))
        self.inc_tet = np.zeros((n, M), dtype=np.int64)
        self.inc_ok = np.zeros((n, M), dtype=bool)
        self.inc_slot = np.full((n, M, 4), K + 1, dtype=np.int64)  # K: self, K+1: zero row
        for k, v in enumerate(tab.verts):
            nb = tab.nbr[k]
            self.nbr[k, :nb.size] = nb
            self.nbr_ok[k, :nb.size] = True
            self.U_nbr[k, :nb.size] = tab.U_nbr[k]
            where = {int(a): j for j, a in enumerate(nb)}
            where[int(v)] = K
            for j, (t, _c) in enumerate(inc[int(v)]):
                self.inc_tet[k, j] = t
                self.inc_ok[k, j] = True
                for c in range(4):
                    self.inc_slot[k, j, c] = where.get(int(model.tets[t, c]), K + 1)
        self.samp = np.where(tab.samples >= 0, tab.samples, 0)
        self.samp_ok = tab.samples >= 0


def r3_systems(model, tab, ell, x, g, R, He, Hb, rows=None):
    """A_i, b_i of variant R3 for table rows ``rows`` (default all)."""
    rows = np.arange(tab.verts.size) if rows is None else np.asarray(rows)
    v = tab.verts[rows]
    Ri = R[v]                                                        # (n,3,3)
    K = ell.K
    nb = ell.nbr[rows]
    Phi = np.einsum("nkab,nkbc,ndc->nkad", R[nb], ell.U_nbr[rows], Ri)  # R_a U R_i^T
    Phi *= ell.nbr_ok[rows][:, :, None, None]
    n = rows.size
    ext = np.concatenate([Phi, np.broadcast_to(np.eye(3), (n, 1, 3, 3)),
                          np.zeros((n, 1, 3, 3))], axis=1)           # (n,K+2,3,3)
    # gradient part
    b = g[v] + np.einsum("nkab,nka->nb", Phi, g[nb])
    # incident elements, exact
    slot = ell.inc_slot[rows]                                         # (n,M,4)
    Ue = np.take_along_axis(ext[:, None, :, :, :], slot[:, :, :, None, None], axis=2)  # (n,M,4,3,3)
    Ue = Ue.reshape(n, ell.M, 12, 3) * ell.inc_ok[rows][:, :, None, None]
    Hinc = He[ell.inc_tet[rows]]                                      # (n,M,12,12)
    A = np.einsum("nmpa,nmpq,nmqb->nab", Ue, Hinc, Ue)
    if Hb is not None:
        A += Hb[v]
    # sampled remote elements
    s = ell.samp[rows]                                                # (n,S)
    corners = model.tets[s]                                           # (n,S,4)
    Us = np.einsum("nscab,nscbd,ned->nscae", R[corners], tab.U_samp[rows], Ri)  # (n,S,4,3,3)
    w = tab.weights[rows] * ell.samp_ok[rows]
    Us12 = Us.reshape(n, ell.S, 12, 3)
    A += np.einsum("ns,nspa,nspq,nsqb->nab", w, Us12, He[s], Us12)
    b += np.einsum("nsc,nscab,nsca->nb", tab.gcoef[rows] * ell.samp_ok[rows][:, :, None], Us, g[corners])
    return A, b


def r2_systems(model, tab, ell, x, z, g, R, He, Hb, H, rows, gradient="assembled"):
    """The literal form of Eqs. reduced_local and cubature (variant R2):
    A_i = H_ii + sum_s w_s U_s^T H_s U_s (samples never contain i, so no ii
    block is removed), b_i = g_i + g-tilde_i with g-tilde_i the sampled
    remote gradient, either from the assembled residual (g_a / n_a at sample
    corners outside the closed one-ring, as in R3; gradient="assembled", R2)
    or from the sample's own element gradient over its four corners
    (gradient="own", R2G1); gradient="none" leaves it out (R2D: the sampled
    reduced Hessian only damps the plain local solve, Sec. 5's closing
    remark that the cubature gradient matters less than this damping
    Hessian).  Uses the cubature tables trained for R3."""
    v = tab.verts[rows]
    Ri = R[v]
    n = rows.size
    A = np.zeros((n, 3, 3))
    for k, f in enumerate(rows):
        A[k] = H[3 * f:3 * f + 3, 3 * f:3 * f + 3].toarray()
    if Hb is not None:
        A += Hb[v]
    s = ell.samp[rows]
    corners = model.tets[s]
    Us = np.einsum("nscab,nscbd,ned->nscae", R[corners], tab.U_samp[rows], Ri)
    w = tab.weights[rows] * ell.samp_ok[rows]
    Us12 = Us.reshape(n, ell.S, 12, 3)
    A += np.einsum("ns,nspa,nspq,nsqb->nab", w, Us12, He[s], Us12)
    b = g[v].copy()
    if gradient == "own":
        ge = model.element_gradients(x, z).reshape(model.nT, 12)
        b += np.einsum("ns,nspa,nsp->na", w, Us12, ge[s])
    elif gradient == "assembled":
        b += np.einsum("nsc,nscab,nsca->nb", tab.gcoef[rows] * ell.samp_ok[rows][:, :, None], Us, g[corners])
    elif gradient != "none":
        raise ValueError(gradient)
    return A, b


def full_subspace_systems(model, U_rows, x, g, R, H, verts):
    """A_i = U_i^T H U_i and b_i = U_i^T g from full row blocks U_rows
    (n, V, 3, 3), using the assembled sparse Hessian H (free DOFs)."""
    A = np.zeros((len(verts), 3, 3))
    b = np.zeros((len(verts), 3))
    gf = model.to_free(g)
    for k, v in enumerate(verts):
        Ui = U_rows[k][model.free_ids].reshape(-1, 3)                 # (3 n_free, 3)
        A[k] = Ui.T @ (H @ Ui)
        b[k] = Ui.T @ gf
    return A, b


def literal_exact_systems(model, U_rows, g, H, verts):
    """Variant RX from full co-rotated row blocks U_rows (n, V, 3, 3): the
    i-th 3-row block of H times U_i (H_ii + sum_a H_{i,a} Phi_{i,a}; only
    the one-ring contributes), symmetrised, and b_i = U_i^T g over the free
    DOFs."""
    A = np.zeros((len(verts), 3, 3))
    b = np.zeros((len(verts), 3))
    gf = model.to_free(g)
    Hr = H.tocsr()
    for k, v in enumerate(verts):
        Ui = U_rows[k][model.free_ids].reshape(-1, 3)                 # (3 n_free, 3)
        f = model.free_index[v]
        M = Hr[3 * f:3 * f + 3] @ Ui
        A[k] = 0.5 * (M + M.T)
        b[k] = Ui.T @ gf
    return A, b


def corotated_rows(tab_U_full, R, verts):
    """Phi_{i,a} = R_a U-bar_{i,a} R_i^T for all a (full rows)."""
    return np.einsum("vab,nvbc,ndc->nvad", R, tab_U_full, R[verts])


def exact_rows(model, H, verts):
    """Eq. phi with the current Hessian: rows of [I; -H_CC^-1 H_Ci] computed
    through the full-coordinate identity U = H^-1 S^T (S H^-1 S^T)^-1."""
    lu = spla.splu(H.tocsc())

    class _S:
        n = H.shape[0]

        @staticmethod
        def solve(B):
            return lu.solve(np.asarray(B, dtype=np.float64))
    return ocorr.ubar_rows(model, _S, verts)


def feasibility_clamp(model, x, step):
    """Contact (Sec. 7 with the line-search remark of Sec. 9): each vertex's
    move is scaled by min(1, 0.9 min_p d_p / (-n_p . step)) over the planes it
    approaches, so no vertex reaches a static plane (reading: a per-vertex,
    per-sub-problem step bound)."""
    if model.planes.shape[0] == 0:
        return step
    alpha = np.ones(step.shape[0])
    for p in range(model.planes.shape[0]):
        n, c = model.planes[p, :3], model.planes[p, 3]
        d = x @ n - c
        nd = step @ n
        m = nd < 0
        alpha[m] = np.minimum(alpha[m], np.maximum(0.0, 0.9 * d[m] / (-nd[m])))
    return step * alpha[:, None]


class Sweeper:
    """Oracle sweeps for one model and a table covering all free vertices."""

    def __init__(self, model, tab=None, variant=R3, omega=1.0, line_search=False):
        self.model = model
        self.tab = tab
        self.variant = variant
        self.omega = omega
        self.line_search = line_search
        self.ls_halvings = 0
        from . import mesh as omesh
        self.inc = omesh.incidence(model.tets, model.nV)
        self.ell = _Ell(model, tab, self.inc) if (tab is not None and variant in (R3, R2, R2G1, R2D)) else None
        if tab is not None:
            assert np.array_equal(tab.verts, model.free_ids)

    def systems(self, x, z, verts=None, R=None):
        """A_i, b_i at iterate x for ``verts``; per-vertex rotations from x
        unless given in R."""
        m = self.model
        g, R_x = phase1(m, x, z)
        R = R_x if R is None else R
        Hb = m.barrier_hessian_blocks(x) if m.planes.shape[0] else None
        verts = m.free_ids if verts is None else np.asarray(verts)
        rows = m.free_index[verts]
        if self.variant == R3:
            He = m.element_hessians(x)
            return r3_systems(m, self.tab, self.ell, x, g, R, He, Hb, rows)
        if self.variant in (R2, R2G1, R2D):
            return r2_systems(m, self.tab, self.ell, x, z, g, R, m.element_hessians(x), Hb, m.hessian(x), rows,
                              gradient={R2: "assembled", R2G1: "own", R2D: "none"}[self.variant])
        if self.variant == P0:
            H = m.hessian(x)
            A = np.zeros((verts.size, 3, 3))
            for k, f in enumerate(rows):
                A[k] = H[3 * f:3 * f + 3, 3 * f:3 * f + 3].toarray()
            return A, g[verts].copy()
        H = m.hessian(x)
        if self.variant == RX:
            U = corotated_rows(self.tab.U_full[rows], R, verts)
            return literal_exact_systems(m, U, g, H, verts)  # H carries the barrier blocks
        if self.variant == R1:
            U = corotated_rows(self.tab.U_full[rows], R, verts)
        else:
            U = exact_rows(m, H, verts)
        return full_subspace_systems(m, U, x, g, R, H, verts)

    def jacobi(self, x, z):
        """One Jacobi sweep.  With line_search, the whole move is halved while
        the incremental potential increases (at most 8 times; reading of the
        global backtracking)."""
        m = self.model
        A, b = self.systems(x, z)
        dx = local_solve(A, b)
        step = feasibility_clamp(m, x[m.free_ids], self.omega * dx)
        xn = x.copy()
        xn[m.free_ids] += step
        if self.line_search:
            e0 = m.energy(x, z)
            e1 = m.energy(xn, z)
            k = 0
            while not (e1 <= e0) and k < 8:
                xn[m.free_ids] = x[m.free_ids] + 0.5 * (xn[m.free_ids] - x[m.free_ids])
                e1 = m.energy(xn, z)
                k += 1
                self.ls_halvings += 1
        return xn

    def gauss_seidel(self, x, z, color):
        """One coloured sweep.  Gradients, Hessians and (except for R2D)
        rotations are taken at the current iterate before every colour.  R2D
        keeps the rotations of the sweep's starting iterate x^k for all
        colours (the pose the co-rotated basis is extracted from, Sec. 4.3):
        its local system needs no other vertex's gradient, so nothing else is
        refreshed between colours."""
        xn = x.copy()
        R_sweep = vertex_rotations(self.model, x) if self.variant == R2D else None
        for c in range(int(color.max()) + 1):
            verts = np.nonzero(color == c)[0]
            A, b = self.systems(xn, z, verts, R=R_sweep)
            dx = local_solve(A, b)
            xn[verts] += feasibility_clamp(self.model, xn[verts], self.omega * dx)
        return xn


def run_step(sweeper, xhat, vhat, sweeps=None, tol=1e-5, max_sweeps=1000, mode="jacobi", color=None):
    """One implicit-Euler step from x0 = xhat with a fixed number of sweeps
    (``sweeps``) or until |g|/|g(x0)| <= tol.  Returns (x, v, residuals)."""
    m = sweeper.model
    z = m.inertial_target(xhat, vhat)
    x = xhat.copy()
    r0 = np.linalg.norm(m.to_free(m.gradient(x, z)))
    hist = [1.0]
    k = 0
    while True:
        if sweeps is not None and k >= sweeps:
            break
        if sweeps is None and (hist[-1] <= tol or k >= max_sweeps):
            break
        x = sweeper.jacobi(x, z) if mode == "jacobi" else sweeper.gauss_seidel(x, z, color)
        k += 1
        hist.append(np.linalg.norm(m.to_free(m.gradient(x, z))) / r0 if r0 > 0 else 0.0)
    v = (x - xhat) / m.h
    return x, v, hist
