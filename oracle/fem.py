"""Linear-tetrahedron FEM for the incremental potential (oracle, float64).

Sec. 3 (Eq. variation): every implicit-Euler step minimises
    E(x) = 1/(2h^2) |M^(1/2)(x - z)|^2 + Psi(x),   z = xhat + h vhat + h^2 M^-1 f_ext.

Readings (the paper does not spell these out):
  * M is the lumped mass, m_a = sum over tets e containing a of rho V_e / 4.
  * The inertia term is split into per-element shares: element e carries
    (rho V_e / 4) / (2 h^2) |x_a - z_a|^2 for each of its corners a, so an
    element's energy, gradient and Hessian include inertia.  Summed over
    elements this is exactly the lumped inertia term.
  * f_ext is gravity only; pinned vertices are held at their rest position
    and carry no unknowns (their inertia term, a constant, is dropped by
    taking z = x there).
  * IPC plane contact (Sec. 7, Eq. barrier): for every vertex a and plane
    (n_p, c_p) with signed distance d = n_p . x_a - c_p, the potential gains
    kappa * B(d, d_hat) with B = -(d - d_hat)^2 log(d / d_hat) on
    0 < d < d_hat and 0 beyond.  kappa is not given by the paper (see the
    design notes); it is a scene parameter here.
"""
import numpy as np
import scipy.sparse as sp

from . import snh


class Model:
    """Rest-state quantities of a tet mesh and its material."""

    def __init__(self, X, tets, pinned, E, nu, rho, dt, gravity=(0.0, -9.8, 0.0),
                 planes=None, d_hat=1e-3, kappa=1e4):
        self.X = np.asarray(X, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.nV = self.X.shape[0]
        self.nT = self.tets.shape[0]
        self.pinned = np.asarray(pinned).astype(bool)
        self.free = ~self.pinned
        self.free_ids = np.nonzero(self.free)[0]
        self.free_index = np.full(self.nV, -1, dtype=np.int64)
        self.free_index[self.free_ids] = np.arange(self.free_ids.size)
        self.E = np.broadcast_to(np.asarray(E, dtype=np.float64), (self.nT,)).copy()
        self.nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (self.nT,)).copy()
        self.rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (self.nT,)).copy()
        self.mu, self.lam = snh.lame(self.E, self.nu)
        self.h = float(dt)
        self.gravity = np.asarray(gravity, dtype=np.float64)
        self.planes = np.zeros((0, 4)) if planes is None else np.asarray(planes, dtype=np.float64).reshape(-1, 4)
        self.d_hat = float(d_hat)
        self.kappa = float(kappa)

        Xe = self.X[self.tets]                                   # (T,4,3)
        Dm = np.stack([Xe[:, 1] - Xe[:, 0], Xe[:, 2] - Xe[:, 0], Xe[:, 3] - Xe[:, 0]], axis=-1)
        self.vol = np.linalg.det(Dm) / 6.0
        if np.any(self.vol <= 0):
            raise ValueError("tets must have positive orientation")
        self.Dm_inv = np.linalg.inv(Dm)
        gN = np.empty((self.nT, 4, 3))
        gN[:, 1:, :] = self.Dm_inv                               # rows of Dm^-1
        gN[:, 0, :] = -self.Dm_inv.sum(axis=1)
        self.gradN = gN
        self.mass_share = self.rho * self.vol / 4.0              # per tet corner
        self.mass = np.zeros(self.nV)
        np.add.at(self.mass, self.tets.ravel(), np.repeat(self.mass_share, 4))
        self.valence = np.bincount(self.tets.ravel(), minlength=self.nV)

    # ---- step set-up ---------------------------------------------------
    def inertial_target(self, xhat, vhat):
        """z = xhat + h vhat + h^2 g on free vertices; z = xhat on pinned ones."""
        z = xhat + self.h * vhat + self.h ** 2 * self.gravity[None, :]
        z[self.pinned] = xhat[self.pinned]
        return z

    # ---- kinematics ----------------------------------------------------
    def deformation_gradient(self, x):
        """F_e = sum_a x_a (grad N_a)^T, i.e. D_s D_m^-1."""
        return np.einsum("tai,taj->tij", x[self.tets], self.gradN)

    # ---- energy ----------------------------------------------------------
    def element_energy(self, x, z):
        F = self.deformation_gradient(x)
        el = self.vol * snh.psi(F, self.mu, self.lam)
        d = x[self.tets] - z[self.tets]
        el = el + self.mass_share / (2.0 * self.h ** 2) * np.einsum("tai,tai->t", d, d)
        return el

    def barrier_energy(self, x):
        if self.planes.shape[0] == 0:
            return 0.0
        d = x @ self.planes[:, :3].T - self.planes[:, 3][None, :]
        if np.any(d[self.free] <= 0):
            return np.inf
        act = (d < self.d_hat) & self.free[:, None]
        dd = d[act]
        return self.kappa * float(np.sum(-(dd - self.d_hat) ** 2 * np.log(dd / self.d_hat)))

    def energy(self, x, z):
        return float(np.sum(self.element_energy(x, z))) + self.barrier_energy(x)

    # ---- gradient -------------------------------------------------------
    def element_gradients(self, x, z):
        """(T,4,3): V_e P(F_e) grad N_a + (rho V_e / 4 h^2)(x_a - z_a)."""
        F = self.deformation_gradient(x)
        P = snh.stress(F, self.mu, self.lam)
        ge = self.vol[:, None, None] * np.einsum("tij,taj->tai", P, self.gradN)
        ge += (self.mass_share / self.h ** 2)[:, None, None] * (x[self.tets] - z[self.tets])
        return ge

    def barrier_gradient(self, x):
        g = np.zeros_like(x)
        for p in range(self.planes.shape[0]):
            n, c = self.planes[p, :3], self.planes[p, 3]
            d = x @ n - c
            act = (d < self.d_hat) & (d > 0) & self.free
            dd = d[act]
            db = -2.0 * (dd - self.d_hat) * np.log(dd / self.d_hat) - (dd - self.d_hat) ** 2 / dd
            g[act] += self.kappa * db[:, None] * n[None, :]
        return g

    def gradient(self, x, z):
        """Assembled dE/dx, (V,3); rows of pinned vertices are zero."""
        g = np.zeros_like(x)
        np.add.at(g, self.tets.ravel(), self.element_gradients(x, z).reshape(-1, 3))
        g += self.barrier_gradient(x)
        g[self.pinned] = 0.0
        return g

    # ---- Hessian ----------------------------------------------------------
    def element_hessians(self, x, project=False):
        """(T,12,12) Hessians of the element energies (elastic + inertia share).

        Built column by column from dP applied to unit nodal perturbations.
        With project=True the elastic part is made positive semidefinite by
        clamping its eigenvalues at zero before the inertia share is added
        (projected Newton)."""
        F = self.deformation_gradient(x)
        He = np.zeros((self.nT, 12, 12))
        for b in range(4):
            for d in range(3):
                dF = np.zeros((self.nT, 3, 3))
                dF[:, d, :] = self.gradN[:, b, :]
                dP = snh.dstress(F, dF, self.mu, self.lam)
                col = self.vol[:, None, None] * np.einsum("tij,taj->tai", dP, self.gradN)
                He[:, :, 3 * b + d] = col.reshape(self.nT, 12)
        He = 0.5 * (He + np.transpose(He, (0, 2, 1)))
        if project:
            w, Q = np.linalg.eigh(He)
            He = np.einsum("tij,tj,tkj->tik", Q, np.maximum(w, 0.0), Q)
        He += (self.mass_share / self.h ** 2)[:, None, None] * np.eye(12)[None]
        return He

    def barrier_hessian_blocks(self, x):
        """(V,3,3) per-vertex barrier Hessian kappa B''(d) n n^T (PSD)."""
        Hb = np.zeros((self.nV, 3, 3))
        for p in range(self.planes.shape[0]):
            n, c = self.planes[p, :3], self.planes[p, 3]
            d = x @ n - c
            act = (d < self.d_hat) & (d > 0) & self.free
            dd = d[act]
            r = dd / self.d_hat
            d2 = -2.0 * np.log(r) - 4.0 * (dd - self.d_hat) / dd + (dd - self.d_hat) ** 2 / dd ** 2
            Hb[act] += self.kappa * d2[:, None, None] * np.outer(n, n)[None]
        return Hb

    def assemble(self, He, Hb=None):
        """Sparse symmetric Hessian over the free DOFs (3 per free vertex, in
        free-vertex order)."""
        fi = self.free_index[self.tets]                          # (T,4)
        dof = (3 * fi[:, :, None] + np.arange(3)[None, None, :]).reshape(self.nT, 12)
        ok = np.repeat(fi >= 0, 3, axis=1)
        rows = np.broadcast_to(dof[:, :, None], He.shape)
        cols = np.broadcast_to(dof[:, None, :], He.shape)
        mask = ok[:, :, None] & ok[:, None, :]
        n = 3 * self.free_ids.size
        H = sp.coo_matrix((He[mask], (rows[mask], cols[mask])), shape=(n, n)).tocsr()
        if Hb is not None:
            blocks = Hb[self.free_ids]
            r = (3 * np.arange(self.free_ids.size)[:, None, None] + np.arange(3)[None, :, None])
            c = (3 * np.arange(self.free_ids.size)[:, None, None] + np.arange(3)[None, None, :])
            r = np.broadcast_to(r, blocks.shape)
            c = np.broadcast_to(c, blocks.shape)
            H = H + sp.coo_matrix((blocks.ravel(), (r.ravel(), c.ravel())), shape=(n, n)).tocsr()
        return H

    def hessian(self, x, project=False):
        He = self.element_hessians(x, project=project)
        Hb = self.barrier_hessian_blocks(x) if self.planes.shape[0] else None
        return self.assemble(He, Hb)

    # ---- free-DOF vector helpers -------------------------------------------
    def to_free(self, a):
        return a[self.free_ids].reshape(-1)

    def from_free(self, v):
        out = np.zeros((self.nV, 3))
        out[self.free_ids] = v.reshape(-1, 3)
        return out


def model_from_scene(sc):
    m = sc.mesh
    return Model(m.X, m.tets, m.pinned, sc.E, sc.nu, sc.rho, sc.dt, sc.gravity,
                 sc.planes, sc.d_hat, sc.kappa)
