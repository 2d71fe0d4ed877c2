"""Pins of the oracle's local systems and sweeps (Sec. 4 optimality,
co-rotation, cubature limit, fixed points, equivariance)."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import correction as oc, mesh as omesh, newton, sweep as osw

rng = np.random.default_rng(3)


def test_polar_properties():
    F = np.eye(3)[None] + 0.4 * rng.standard_normal((50, 3, 3))
    R = osw.polar(F)
    np.testing.assert_allclose(np.einsum("nji,njk->nik", R, R), np.broadcast_to(np.eye(3), R.shape), atol=1e-12)
    assert np.allclose(np.linalg.det(R), 1.0)
    S = np.einsum("nji,njk->nik", R, F)
    pos = np.linalg.det(F) > 0
    np.testing.assert_allclose(S[pos], S[pos].transpose(0, 2, 1), atol=1e-12)
    assert np.all(np.linalg.eigvalsh(0.5 * (S[pos] + S[pos].transpose(0, 2, 1))) > 0)


def test_exact_subspace_sweep_is_newton_step(tiny):
    """R0 (Eq. phi with the current Hessian): one Jacobi sweep equals the
    global Newton step -H^-1 g (Sec. 4.2)."""
    sc, mdl, tab = tiny
    z = mdl.inertial_target(sc.x0, sc.v0)
    x = sc.x0 + 1e-3 * rng.standard_normal(sc.x0.shape); x[mdl.pinned] = mdl.X[mdl.pinned]
    sw = osw.Sweeper(mdl, tab, osw.R0)
    x1 = sw.jacobi(x, z)
    H = mdl.hessian(x)
    dx = mdl.from_free(spla.spsolve(H.tocsc(), -mdl.to_free(mdl.gradient(x, z))))
    assert np.abs(x1 - (x + dx)).max() < 1e-10 * np.abs(dx).max()


def test_corotated_subspace_at_rest_is_newton_step(tiny):
    """R1 from x0 = X (R = I, H = H-bar): the first sweep is the Newton step."""
    sc, mdl, tab = tiny
    z = mdl.inertial_target(mdl.X, sc.v0)
    sw = osw.Sweeper(mdl, tab, osw.R1)
    x1 = sw.jacobi(mdl.X.copy(), z)
    H = mdl.hessian(mdl.X)
    dx = mdl.from_free(spla.spsolve(H.tocsc(), -mdl.to_free(mdl.gradient(mdl.X, z))))
    assert np.abs(x1 - (mdl.X + dx)).max() < 1e-10 * np.abs(dx).max()


def _exact_limit_tables(mdl, tab):
    n = tab.verts.size
    T = mdl.nT
    samples = -np.ones((n, T), dtype=np.int64)
    weights = np.zeros((n, T))
    for k, v in enumerate(tab.verts):
        non = np.nonzero(~np.any(mdl.tets == v, axis=1))[0]
        samples[k, :non.size] = non
        weights[k, :non.size] = 1.0
    return oc.Tables(mdl, tab.verts, tab.ring, tab.U_full, samples, weights, tab.fit_res, tab.lam, tab.cid)


def test_cubature_with_every_element_is_exact_galerkin(tiny):
    """R3 with every non-incident element sampled at weight 1 reproduces R1
    (assembled through the sparse global Hessian) at a deformed state."""
    sc, mdl, tab = tiny
    tabx = _exact_limit_tables(mdl, tab)
    z = mdl.inertial_target(sc.x0, sc.v0)
    x = sc.x0 + 2e-3 * rng.standard_normal(sc.x0.shape); x[mdl.pinned] = mdl.X[mdl.pinned]
    verts = mdl.free_ids[::9]
    A3, b3 = osw.Sweeper(mdl, tabx, osw.R3).systems(x, z, verts)
    A1, b1 = osw.Sweeper(mdl, tab, osw.R1).systems(x, z, verts)
    assert np.abs(A3 - A1).max() < 1e-11 * np.abs(A1).max()
    assert np.abs(b3 - b1).max() < 1e-11 * np.abs(b1).max()


def test_solution_is_fixed_point_of_every_variant(tiny):
    sc, mdl, tab = tiny
    xs, hist = newton.newton_solve(mdl, sc.x0, sc.v0, tol=1e-11)
    z = mdl.inertial_target(sc.x0, sc.v0)
    diag = np.linalg.norm(mdl.X.max(0) - mdl.X.min(0))
    for var in [osw.R0, osw.R1, osw.R3, osw.R2, osw.P0]:
        x1 = osw.Sweeper(mdl, tab, var).jacobi(xs, z)
        assert np.abs(x1 - xs).max() < 1e-9 * diag, var
    # the literal form with element-own sample gradients is not stationary at
    # the solution: element forces do not vanish where the assembled residual does
    x1 = osw.Sweeper(mdl, tab, osw.R2G1).jacobi(xs, z)
    assert np.abs(x1 - xs).max() > 1e-6 * diag


def test_literal_form_without_samples_is_plain_jacobi(tiny):
    """With every cubature weight zero, R2 reduces to A_i = H_ii, b_i = g_i."""
    import copy
    sc, mdl, tab = tiny
    t0 = copy.copy(tab)
    t0.weights = np.zeros_like(tab.weights)
    t0.gcoef = np.zeros_like(tab.gcoef)
    z = mdl.inertial_target(sc.x0, sc.v0)
    x = sc.x0 + 1e-4 * np.random.default_rng(5).standard_normal(sc.x0.shape)
    x[mdl.pinned] = mdl.X[mdl.pinned]
    for var in (osw.R2, osw.R2G1):
        A, b = osw.Sweeper(mdl, t0, var).systems(x, z)
        A0, b0 = osw.Sweeper(mdl, None, osw.P0).systems(x, z)
        np.testing.assert_allclose(A, A0, rtol=1e-13, atol=1e-9)
        np.testing.assert_allclose(b, b0, rtol=1e-13, atol=1e-12)


def test_zero_force_at_rest_gives_zero_step(tiny):
    sc, mdl, tab = tiny
    g0 = mdl.gravity.copy()
    mdl.gravity[:] = 0.0
    try:
        z = mdl.inertial_target(mdl.X, 0 * mdl.X)
        for var in [osw.R3, osw.P0]:
            x1 = osw.Sweeper(mdl, tab, var).jacobi(mdl.X.copy(), z)
            assert np.abs(x1 - mdl.X).max() < 1e-14
    finally:
        mdl.gravity[:] = g0


def test_rigid_rotation_equivariance(tiny):
    """Rotating the iterate, velocities and gravity (rest shape unchanged) by
    Q rotates every local system: R_a becomes Q R_a, so the co-rotated rows
    Phi (Eq. tilde_phi) become Q Phi Q^T, A_i -> Q A_i Q^T, b_i -> Q b_i.
    (The solved step inherits this unless the PD guard fires, whose pivot
    test is basis-dependent.)"""
    sc, mdl, tab = tiny
    from oracle import fem
    rng = np.random.default_rng(11)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    q *= np.sign(np.linalg.det(q))
    x = sc.x0 + 1e-3 * rng.standard_normal(sc.x0.shape); x[mdl.pinned] = mdl.X[mdl.pinned]
    v = 0.05 * rng.standard_normal(sc.x0.shape); v[mdl.pinned] = 0
    z = mdl.inertial_target(x, v)
    mdr = fem.Model(mdl.X, mdl.tets, mdl.pinned, mdl.E, mdl.nu, mdl.rho, mdl.h, mdl.gravity @ q.T)
    zr = mdr.inertial_target(x @ q.T, v @ q.T)
    verts = mdl.free_ids
    for var in [osw.R3, osw.R1, osw.RX, osw.P0]:
        A, b = osw.Sweeper(mdl, tab, var).systems(x, z, verts)
        Ar, br = osw.Sweeper(mdr, tab, var).systems(x @ q.T, zr, verts)
        assert np.abs(Ar - q @ A @ q.T).max() < 1e-10 * np.abs(A).max(), var
        assert np.abs(br - b @ q.T).max() < 1e-10 * np.abs(b).max(), var


def test_gauss_seidel_single_colour_equals_jacobi(tiny):
    sc, mdl, tab = tiny
    z = mdl.inertial_target(sc.x0, sc.v0)
    sw = osw.Sweeper(mdl, tab, osw.P0)
    one = np.where(mdl.free, 0, -1)
    np.testing.assert_allclose(sw.gauss_seidel(sc.x0, z, one), sw.jacobi(sc.x0, z), rtol=0, atol=1e-15)


def test_gauss_seidel_plain_converges_monotonically(tiny):
    """Coloured GS with plain vertex Newton decreases the energy every sweep."""
    sc, mdl, tab = tiny
    col = omesh.greedy_coloring(omesh.one_ring(mdl.tets, mdl.nV), mdl.free)
    sw = osw.Sweeper(mdl, tab, osw.P0)
    z = mdl.inertial_target(sc.x0, sc.v0)
    x = sc.x0.copy()
    e = [mdl.energy(x, z)]
    for _ in range(6):
        x = sw.gauss_seidel(x, z, col)
        e.append(mdl.energy(x, z))
    assert np.all(np.diff(e) < 0)
