"""Pins of the oracle adjoint: central finite differences of the converged
FP64 forward, the dot-product identity with the forward-mode tangent, and
symmetry of the step Hessian."""
import numpy as np
import pytest

from oracle import adjoint as oa, fem
from paper_2506_06494_amd import inputs


@pytest.fixture(scope="module")
def small():
    m = inputs.beam_mesh(6, 2, 2, 0.05)
    mdl = fem.Model(m.X, m.tets, m.pinned, 1e5, 0.45, 1000.0, 1.0 / 120)
    g = inputs.SplitMix64(7)
    logE = np.log(1e5) + g.uniform_array(m.nT, -0.3, 0.3)
    u = np.array([0.05, -0.1, 0.2])
    tip = oa.tip_vertices(mdl)
    target = m.X[tip].mean(0) + np.array([0.01, -0.03, 0.02])
    return mdl, logE, u, target


def test_gradient_matches_central_differences(small):
    mdl, logE, u, target = small
    n = 3
    L, gth, gu = oa.loss_and_grad(mdl, logE, u, target, n)

    def loss(le, uu):
        oa.set_log_stiffness(mdl, le)
        xs, _ = oa.forward(mdl, mdl.X.copy(), oa.initial_velocity(mdl, uu), n)
        return oa.tip_loss(mdl, xs[-1], target)[0]

    # single entries: the loss moves by ~1e-10 of itself, so the forward's
    # rounding floor (~1e-10 relative residual) limits FD to ~1e-4 relative
    h = 1e-3
    rng = np.random.default_rng(0)
    for e in rng.choice(mdl.nT, 6, replace=False):
        d = np.zeros(mdl.nT); d[e] = h
        fd = (loss(logE + d, u) - loss(logE - d, u)) / (2 * h)
        assert abs(fd - gth[e]) <= 1e-3 * abs(gth[e]) + 1e-5 * np.abs(gth).max(), (e, fd, gth[e])
    h = 1e-4
    for k in range(3):
        d = np.zeros(3); d[k] = h
        fd = (loss(logE, u + d) - loss(logE, u - d)) / (2 * h)
        assert abs(fd - gu[k]) <= 1e-6 * np.abs(gu).max() + 1e-12, (k, fd, gu[k])
    # a dense direction through all tets at once
    d = rng.standard_normal(mdl.nT)
    fd = (loss(logE + h * d, u) - loss(logE - h * d, u)) / (2 * h)
    assert abs(fd - gth @ d) <= 1e-5 * abs(fd)


def test_dot_product_identity(small):
    mdl, logE, u, _ = small
    oa.set_log_stiffness(mdl, logE)
    xs, _ = oa.forward(mdl, mdl.X.copy(), oa.initial_velocity(mdl, u), 3)
    rng = np.random.default_rng(1)
    dth = rng.standard_normal(mdl.nT)
    dx0 = rng.standard_normal((mdl.nV, 3)) * 1e-3
    dv0 = rng.standard_normal((mdl.nV, 3))
    dx0[mdl.pinned] = 0; dv0[mdl.pinned] = 0
    xb = rng.standard_normal((mdl.nV, 3)); vb = rng.standard_normal((mdl.nV, 3))
    xb[mdl.pinned] = 0; vb[mdl.pinned] = 0
    dxN, dvN = oa.tangent(mdl, xs, dth, dx0, dv0)
    tb, xb0, vb0 = oa.backward(mdl, xs, xb, vb)
    lhs = np.sum(dxN * xb) + np.sum(dvN * vb)
    rhs = dth @ tb + np.sum(dx0 * xb0) + np.sum(dv0 * vb0)
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1.0)


def test_step_hessian_is_symmetric(small):
    mdl, logE, u, _ = small
    oa.set_log_stiffness(mdl, logE)
    xs, _ = oa.forward(mdl, mdl.X.copy(), oa.initial_velocity(mdl, u), 1)
    H = mdl.hessian(xs[-1], project=False)
    assert abs(H - H.T).max() <= 1e-12 * abs(H).max()


def test_rest_is_stationary_without_gravity(small):
    """Zero gravity and zero velocity: x stays at X, and the adjoint of a
    loss on x_N reduces to the linear response M/h^2 H^-1 chain at rest."""
    mdl, logE, _, _ = small
    m2 = fem.Model(mdl.X, mdl.tets, mdl.pinned, np.exp(logE), 0.45, 1000.0, mdl.h, gravity=(0, 0, 0))
    xs, vs = oa.forward(m2, m2.X.copy(), np.zeros_like(m2.X), 2)
    assert np.abs(xs[-1] - m2.X).max() <= 1e-15
    # at rest no element is stressed, so the stiffness gradient vanishes
    tb, _, _ = oa.backward(m2, xs, np.ones_like(m2.X))
    assert np.abs(tb).max() <= 1e-12
