"""Global Newton reference (oracle).

Sec. 4 (Eq. newton, Eq. newton_system): the second-order step solves
H dx = -g.  The paper's own baseline is projected Newton with a sparse
direct (Cholesky) solver (Sec. 8.4, comparison with projected Newton).  Here:
per-element PSD projection of the elastic Hessian, a sparse direct solve
(SuperLU through scipy), and backtracking on E.  The projection changes the
path, not the minimiser x*.
"""
import numpy as np
import scipy.sparse.linalg as spla


def sparse_solve(H, b):
    """Direct sparse solve (SuperLU, minimum-degree ordering on H + H^T)."""
    return spla.splu(H.tocsc(), permc_spec="MMD_AT_PLUS_A").solve(b)


def newton_solve(model, xhat, vhat, tol=1e-12, max_iter=60, project=True, x_start=None):
    """Minimise E for one implicit-Euler step from x0 = xhat (or from
    ``x_start`` when given, the residual still being scaled by |g(xhat)|).

    Returns (x*, residual history), the residual being |g(x)| / |g(x0)| over
    free DOFs."""
    z = model.inertial_target(xhat, vhat)
    r0 = np.linalg.norm(model.to_free(model.gradient(xhat, z)))
    x = xhat.copy() if x_start is None else np.array(x_start, dtype=np.float64)
    g = model.gradient(x, z)
    hist = [np.linalg.norm(model.to_free(g)) / r0 if r0 > 0 else 0.0]
    if r0 == 0.0:
        return x, hist
    for _ in range(max_iter):
        if hist[-1] <= tol:
            break
        H = model.hessian(x, project=project)
        dx = model.from_free(sparse_solve(H, -model.to_free(g)))
        e0 = model.energy(x, z)
        slope = float(np.sum(g * dx))
        alpha = 1.0
        if -slope <= 1e-12 * abs(e0):
            # the predicted decrease is below what an FP64 energy sum resolves:
            # backtrack on the gradient norm instead
            gn = np.linalg.norm(model.to_free(g))
            for _ls in range(40):
                if np.linalg.norm(model.to_free(model.gradient(x + alpha * dx, z))) < gn:
                    break
                alpha *= 0.5
        else:
            for _ls in range(40):
                e1 = model.energy(x + alpha * dx, z)
                if e1 <= e0 + 1e-4 * alpha * slope + 1e-14 * abs(e0):
                    break
                alpha *= 0.5
        x = x + alpha * dx
        g = model.gradient(x, z)
        hist.append(np.linalg.norm(model.to_free(g)) / r0)
    return x, hist
