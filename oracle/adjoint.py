"""Implicit-function adjoint of the implicit-Euler step map (oracle, float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper defines the forward step only (Sec. 3, Eq. variation): x_{n+1} is
the minimiser of E(x) = 1/(2h^2)|M^(1/2)(x - z_n)|^2 + Psi(x; theta), with
z_n = x_n + h v_n + h^2 g and v_{n+1} = (x_{n+1} - x_n)/h.  Differentiation
is not in the paper; this module is the plain definition of the derivative
of that map, through the optimality condition

    G(x_{n+1}; x_n, v_n, theta) = grad E = M/h^2 (x_{n+1} - z_n) + grad Psi = 0.

With the symmetric Hessian H = dG/dx_{n+1} at the solution, the cotangent
of the step's outputs (xbar_{n+1}, vbar_{n+1}) is pulled back by

    H y = xbar_{n+1} + vbar_{n+1}/h             (only x_{n+1} enters both)
    thetabar_e -= y_e . grad_{x_e}(V_e Psi_e)    (Psi_e is proportional to E_e = exp(theta_e))
    xbar_n  = M y / h^2 - vbar_{n+1}/h
    vbar_n  = M y / h

over free degrees of freedom (pinned vertices carry no unknowns, so their
rows of y, xbar and vbar are zero).  A single initial velocity u shared by
all free vertices gets ubar = sum over free a of vbar_{0,a}.

Pinned by finite differences of the FP64 forward (converged to 1e-12), by
the dot-product identity against the forward-mode tangent in this module and
by the symmetry of H.
"""
import numpy as np

from . import snh
from .newton import newton_solve, sparse_solve


def elastic_element_forces(model, x):
    """(T,4,3): grad over the element's corners of V_e Psi(F_e), i.e.
    V_e P(F_e) grad N_a; this is also d/dtheta_e of the element's gradient
    because mu and lambda are both proportional to E_e."""
    F = model.deformation_gradient(x)
    P = snh.stress(F, model.mu, model.lam)
    return model.vol[:, None, None] * np.einsum("tij,taj->tai", P, model.gradN)


def set_log_stiffness(model, log_E):
    """Per-tet Young's modulus E_e = exp(theta_e); nu is unchanged."""
    model.E = np.exp(np.asarray(log_E, dtype=np.float64)).copy()
    model.mu, model.lam = snh.lame(model.E, model.nu)


def initial_velocity(model, u):
    """The same velocity u on every free vertex, zero on pinned ones."""
    v = np.zeros((model.nV, 3))
    v[model.free] = np.asarray(u, dtype=np.float64)[None, :]
    return v


def forward(model, x0, v0, n_steps, tol=1e-12):
    """Implicit-Euler steps with the global Newton solve (projected Hessian;
    if that stalls in a linear tail, the exact Hessian from there on, which
    is positive definite near the minimiser); returns the lists of
    positions and velocities x_0..x_N, v_0..v_N."""
    xs, vs = [np.array(x0, dtype=np.float64)], [np.array(v0, dtype=np.float64)]
    for _ in range(n_steps):
        x, hist = newton_solve(model, xs[-1], vs[-1], tol=tol, max_iter=12)
        if hist[-1] > tol:
            x, hist = newton_solve(model, xs[-1], vs[-1], tol=tol, project=False, x_start=x)
        g = np.linalg.norm(model.to_free(model.gradient(x, model.inertial_target(xs[-1], vs[-1]))))
        if hist[-1] > 1e-8 and g > 1e-10:                   # second test: rounding floor near rest [N]
            raise RuntimeError(f"forward Newton stalled at {hist[-1]:.3e} (|g| = {g:.3e} N)")
        v = (x - xs[-1]) / model.h
        v[model.pinned] = 0.0
        xs.append(x)
        vs.append(v)
    return xs, vs


def step_adjoint(model, x_next, xbar, vbar):
    """Pull (xbar_{n+1}, vbar_{n+1}) back through one step that ended at
    x_next.  Returns (dthetabar (T,), xbar_n, vbar_n, y)."""
    H = model.hessian(x_next, project=False)
    rhs = model.to_free(xbar + vbar / model.h)
    y = model.from_free(sparse_solve(H, rhs))
    fe = elastic_element_forces(model, x_next)
    dtheta = -np.einsum("tai,tai->t", y[model.tets], fe)
    My = model.mass[:, None] * y
    xbar_n = My / model.h ** 2 - vbar / model.h
    vbar_n = My / model.h
    xbar_n[model.pinned] = 0.0
    vbar_n[model.pinned] = 0.0
    return dtheta, xbar_n, vbar_n, y


def backward(model, xs, xbar_N, vbar_N=None):
    """Reverse sweep over a trajectory from ``forward``; returns
    (thetabar (T,), xbar_0, vbar_0)."""
    xbar = np.array(xbar_N, dtype=np.float64)
    vbar = np.zeros_like(xbar) if vbar_N is None else np.array(vbar_N, dtype=np.float64)
    xbar[model.pinned] = 0.0
    vbar[model.pinned] = 0.0
    theta = np.zeros(model.nT)
    for n in range(len(xs) - 1, 0, -1):
        d, xbar, vbar, _ = step_adjoint(model, xs[n], xbar, vbar)
        theta += d
    return theta, xbar, vbar


def tangent(model, xs, dtheta, dx0, dv0):
    """Forward-mode derivative of the trajectory along (dtheta, dx0, dv0):
    H dx_{n+1} = M/h^2 (dx_n + h dv_n) - sum_e dtheta_e grad(V_e Psi_e),
    dv_{n+1} = (dx_{n+1} - dx_n)/h.  Returns (dx_N, dv_N)."""
    dx, dv = np.array(dx0, dtype=np.float64), np.array(dv0, dtype=np.float64)
    dx[model.pinned] = 0.0
    dv[model.pinned] = 0.0
    for n in range(1, len(xs)):
        H = model.hessian(xs[n], project=False)
        f = np.zeros((model.nV, 3))
        np.add.at(f, model.tets.ravel(),
                  (np.asarray(dtheta)[:, None, None] * elastic_element_forces(model, xs[n])).reshape(-1, 3))
        rhs = model.mass[:, None] * (dx + model.h * dv) / model.h ** 2 - f
        dxn = model.from_free(sparse_solve(H, model.to_free(rhs)))
        dv = (dxn - dx) / model.h
        dx = dxn
    return dx, dv


def tip_vertices(model):
    """Vertices of the free end face (largest rest x)."""
    xmax = model.X[:, 0].max()
    return np.nonzero(model.X[:, 0] >= xmax - 1e-12)[0]


def tip_loss(model, x, target, tip=None):
    """L = |mean of the tip-face positions - target|^2 and dL/dx (V,3)."""
    tip = tip_vertices(model) if tip is None else tip
    c = x[tip].mean(0)
    r = c - np.asarray(target, dtype=np.float64)
    g = np.zeros_like(x)
    g[tip] = 2.0 * r[None, :] / tip.size
    return float(r @ r), g


def loss_and_grad(model, log_E, u, target, n_steps, tol=1e-12):
    """Differentiable rollout from rest with initial velocity u on free
    vertices: returns (L, dL/dlog_E (T,), dL/du (3,))."""
    set_log_stiffness(model, log_E)
    xs, _ = forward(model, model.X.copy(), initial_velocity(model, u), n_steps, tol=tol)
    L, gx = tip_loss(model, xs[-1], target)
    theta, _, vbar0 = backward(model, xs, gx)
    return L, theta, vbar0[model.free].sum(0)
