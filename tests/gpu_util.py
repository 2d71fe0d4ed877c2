"""Helpers shared by GPU tests: drive the C-ABI through the binding and
translate oracle tables into the library's import layout."""
import numpy as np

from paper_2506_06494_amd import jgs2


def make_solver(scene, **params):
    kw = dict(dt=scene.dt, gravity=scene.gravity)
    if scene.planes.shape[0]:
        kw.update(planes=scene.planes, d_hat=scene.d_hat, kappa=scene.kappa)
    kw.update(params)
    s = jgs2.Solver(**kw)
    m = scene.mesh
    s.upload_mesh(m.X, m.tets, m.pinned)
    s.set_material(scene.E, scene.nu, scene.rho)
    return s


def oracle_tables_to_import(tab):
    """Oracle Tables (free vertices in ascending order) -> import arrays."""
    U_ring = np.concatenate([u.reshape(-1, 9) for u in tab.U_nbr], axis=0)
    return dict(S=tab.samples.shape[1], U_ring=U_ring, samples=tab.samples.astype(np.int32),
                weights=tab.weights, U_samp=tab.U_samp)


def bbox_diag(X):
    return float(np.linalg.norm(X.max(0) - X.min(0)))
