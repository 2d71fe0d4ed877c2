"""Pins of the oracle's stable Neo-Hookean model and plane barrier against
finite differences and closed forms (CPU, float64)."""
import numpy as np
import pytest

from oracle import fem, snh

rng = np.random.default_rng(1)


def rand_F(n=20, scale=0.3):
    return np.eye(3)[None] + scale * rng.standard_normal((n, 3, 3))


def test_rest_state_is_stress_free():
    mu, lam = snh.lame(1e6, 0.4)
    F = np.eye(3)[None]
    assert abs(snh.psi(F, mu, lam)[0]) < 1e-12
    assert np.abs(snh.stress(F, mu, lam)).max() < 1e-9


def test_stress_is_energy_derivative():
    mu, lam = snh.lame(1e5, 0.45)
    F = rand_F()
    P = snh.stress(F, mu, lam)
    h = 1e-6
    for i in range(3):
        for j in range(3):
            d = np.zeros((3, 3)); d[i, j] = h
            fd = (snh.psi(F + d, mu, lam) - snh.psi(F - d, mu, lam)) / (2 * h)
            np.testing.assert_allclose(fd, P[:, i, j], rtol=1e-7, atol=1e-7 * np.abs(P).max())


def test_stress_differential_is_stress_derivative():
    mu, lam = snh.lame(1e5, 0.45)
    F = rand_F()
    dF = rng.standard_normal((F.shape[0], 3, 3))
    h = 1e-6
    fd = (snh.stress(F + h * dF, mu, lam) - snh.stress(F - h * dF, mu, lam)) / (2 * h)
    an = snh.dstress(F, dF, mu, lam)
    np.testing.assert_allclose(an, fd, rtol=1e-7, atol=1e-7 * np.abs(an).max())


def test_rotation_invariance():
    mu, lam = snh.lame(1e6, 0.3)
    F = rand_F()
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    q *= np.sign(np.linalg.det(q))
    np.testing.assert_allclose(snh.psi(q[None] @ F, mu, lam), snh.psi(F, mu, lam), rtol=1e-12)


def test_cofactor_matches_det_inverse_transpose():
    F = rand_F()
    np.testing.assert_allclose(snh.cof(F), np.linalg.det(F)[:, None, None] * np.linalg.inv(F).transpose(0, 2, 1),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("E,nu", [(1e6, 0.4), (1e5, 0.45), (2e6, 0.3)])
def test_small_strain_limit_is_linear_elasticity(E, nu):
    """Uniaxial strain gives P11/eps -> lam_L + 2 mu_L; simple shear gives
    P12/gamma -> mu_L (textbook linear elasticity)."""
    mu, lam = snh.lame(E, nu)
    mu_l = E / (2 * (1 + nu))
    lam_l = E * nu / ((1 + nu) * (1 - 2 * nu))
    eps = 1e-7
    F = np.eye(3)[None].copy(); F[0, 0, 0] += eps
    assert abs(snh.stress(F, mu, lam)[0, 0, 0] / eps - (lam_l + 2 * mu_l)) < 1e-5 * (lam_l + 2 * mu_l)
    F = np.eye(3)[None].copy(); F[0, 0, 1] += eps
    assert abs(snh.stress(F, mu, lam)[0, 0, 1] / eps - mu_l) < 1e-5 * mu_l


def _plane_model(d_hat=1e-3, kappa=1e4):
    X = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]) + np.array([0, 0, 0.5])
    return fem.Model(X, np.array([[0, 1, 2, 3]]), np.zeros(4, np.uint8), 1e3, 0.3, 1000.0, 0.01,
                     planes=np.array([[0, 0, 1, 0.0]]), d_hat=d_hat, kappa=kappa)


def test_barrier_closed_forms():
    m = _plane_model()
    dh = m.d_hat
    x = m.X.copy()
    # beyond d_hat the barrier, its slope and curvature vanish
    x[0, 2] = dh * (1 + 1e-12)
    assert m.barrier_energy(x) == 0.0
    assert np.abs(m.barrier_gradient(x)).max() == 0.0
    # B''(d_hat/2) = 2 ln 2 + 5 (d_hat-independent)
    x[0, 2] = dh / 2
    Hb = m.barrier_hessian_blocks(x)
    assert abs(Hb[0, 2, 2] / m.kappa * dh ** 2 / dh ** 2 - (2 * np.log(2) + 5)) < 1e-12
    # infinite at contact
    x[0, 2] = 0.0
    assert m.barrier_energy(x) == np.inf


def test_barrier_derivatives_by_fd():
    m = _plane_model()
    x = m.X.copy()
    h = 1e-9
    for d in [1e-4, 3e-4, 7e-4, 9.9e-4]:
        x[0, 2] = d
        xp, xm = x.copy(), x.copy()
        xp[0, 2] += h; xm[0, 2] -= h
        fd = (m.barrier_energy(xp) - m.barrier_energy(xm)) / (2 * h)
        assert abs(fd - m.barrier_gradient(x)[0, 2]) < 1e-6 * max(1.0, abs(fd))
        fd2 = (m.barrier_gradient(xp)[0, 2] - m.barrier_gradient(xm)[0, 2]) / (2 * h)
        assert abs(fd2 - m.barrier_hessian_blocks(x)[0, 2, 2]) < 1e-5 * abs(fd2)


def test_own_diagonal_block_closed_form():
    """For dF = e_d g^T and dF' = e_e g^T (a corner's own 3x3 block) the
    cofactor-derivative term of dP vanishes, (e_e x e_d)^T F (g x g) = 0, so
    the block is mu |g|^2 I + lam (cof F g)(cof F g)^T for any F (inverted
    included): the form the plain sweep kernel evaluates."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        F = rng.standard_normal((3, 3))
        g = rng.standard_normal(3)
        mu, lam = rng.uniform(0.1, 5.0, 2)
        A = np.zeros((3, 3))
        for d in range(3):
            D = np.zeros((3, 3)); D[d] = g
            dP = snh.dstress(F[None], D[None], np.array([mu]), np.array([lam]))[0]
            for e in range(3):
                De = np.zeros((3, 3)); De[e] = g
                A[d, e] = np.sum(dP * De)
        c = snh.cof(F[None])[0] @ g
        np.testing.assert_allclose(A, mu * (g @ g) * np.eye(3) + lam * np.outer(c, c), rtol=1e-12,
                                   atol=1e-12 * np.abs(A).max())
