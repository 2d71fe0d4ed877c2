"""Pins of the linear analysis of the correction readings (Sec. 4.2 to
Sec. 5) and of the finding it supports.

The analysis builds each reading's sweep as a linear operator at the rest
state.  Its operators are checked here against what the oracle's own sweeps
do to a small error about the rest state (a linearisation that shares none
of the analysis code), then the convergence statements are fixed:
  * the exact co-rotated subspace at rest is one Newton step (operator 0);
  * the sampled readings (remote gradient by cubature) have spectral radius
    above one in Jacobi and Gauss-Seidel order, so no sweep count reaches a
    tolerance;
  * the damper reading (sampled reduced Hessian added to H_ii, gradient
    g_i) converges, but more slowly than plain vertex Newton in the same
    order, with or without a step scale;
  * the exact co-rotated subspace in the literal form of Eq. local_newton
    (variant RX) is the Newton step at rest (against a direct solve and a
    dense inverse), is stationary at the solution, and converges within the
    Newton iteration count on the nonlinear steps tried.
"""
import numpy as np
import pytest

from oracle import correction as oc, linear_analysis as la, mesh as omesh, sweep as osw
from paper_2506_06494_amd import inputs
from oracle import fem


@pytest.fixture(scope="module")
def rest(tiny):
    sc, mdl, tab = tiny
    return la.RestSystem(mdl)


def _linear_sweep(sw, mdl, e, mode, color=None, eps=1e-7):
    """One oracle sweep from X + eps e towards the rest state (z = X, so the
    rest state is the solution); returns the new error / eps."""
    g0 = mdl.gravity.copy()
    mdl.gravity[:] = 0.0
    try:
        z = mdl.X.copy()
        x = mdl.X + eps * e
        x1 = sw.jacobi(x, z) if mode == "jacobi" else sw.gauss_seidel(x, z, color)
    finally:
        mdl.gravity[:] = g0
    return (x1 - mdl.X) / eps


def _as_free(mdl, e):
    return e[mdl.free_ids].ravel()


@pytest.mark.parametrize("variant", [osw.P0, osw.R3, osw.R2D])
def test_jacobi_operator_matches_oracle_sweep(tiny, rest, variant):
    """The analysis's Jacobi operator I - P H applied to an error equals one
    oracle Jacobi sweep of the same reading about the rest state, to first
    order in the error."""
    sc, mdl, tab = tiny
    rng = np.random.default_rng(21)
    e = rng.standard_normal(mdl.X.shape)
    e[mdl.pinned] = 0.0
    sw = osw.Sweeper(mdl, tab, variant)
    got = _as_free(mdl, _linear_sweep(sw, mdl, e, "jacobi"))
    A, C = {osw.P0: rest.plain, osw.R3: lambda: rest.cubature(tab.samples, tab.weights, "R3"),
            osw.R2D: lambda: rest.cubature(tab.samples, tab.weights, "R2D")}[variant]()
    want = rest.jacobi_operator(A, C) @ _as_free(mdl, e)
    assert np.abs(got - want).max() <= 1e-4 * np.abs(want).max()


def test_gauss_seidel_operator_matches_oracle_sweep(tiny, rest):
    """The same for coloured Gauss-Seidel with plain vertex Newton: the
    analysis multiplies the colour blocks in the sweep's order."""
    sc, mdl, tab = tiny
    rng = np.random.default_rng(22)
    e = rng.standard_normal(mdl.X.shape)
    e[mdl.pinned] = 0.0
    col = omesh.greedy_coloring(omesh.one_ring(mdl.tets, mdl.nV), mdl.free)
    np.testing.assert_array_equal(col[mdl.free_ids], rest.color)
    got = _as_free(mdl, _linear_sweep(osw.Sweeper(mdl, tab, osw.P0), mdl, e, "gs", col))
    want = rest.gs_operator(*rest.plain()) @ _as_free(mdl, e)
    assert np.abs(got - want).max() <= 1e-4 * np.abs(want).max()


def test_exact_corotated_subspace_operator_vanishes(rest):
    """At rest U-bar_i^T H-bar = B_i^-1 S_i (Eq. u), so the exact reading's
    Jacobi sweep is one Newton step and its error operator is zero."""
    E = rest.jacobi_operator(*rest.exact())
    assert np.abs(E).max() < 1e-8


def test_sampled_readings_diverge_and_the_damper_is_slower_than_plain(tiny, rest):
    sc, mdl, tab = tiny
    r3 = rest.cubature(tab.samples, tab.weights, "R3")
    r2 = rest.cubature(tab.samples, tab.weights, "R2")
    r2d = rest.cubature(tab.samples, tab.weights, "R2D")
    p0 = rest.plain()
    for reading in (r3, r2):
        assert la.spectral_radius(rest.jacobi_operator(*reading)) > 1.0
        assert la.spectral_radius(rest.gs_operator(*reading)) > 1.0
        # eigenvalues of P H with negative real part: no positive step scale helps
        P = rest.preconditioner(*reading)
        assert np.linalg.eigvals(P @ rest.H).real.min() < 0.0
    for omega in (1.0, 1.6):
        rp = la.spectral_radius(rest.gs_operator(*p0, omega=omega))
        rd = la.spectral_radius(rest.gs_operator(*r2d, omega=omega))
        assert rp < rd < 1.0, (omega, rp, rd)


# ---- the exact co-rotated subspace in the literal form of Eq. local_newton ----

def _exact_tables(mdl):
    from types import SimpleNamespace
    solver = oc.RestSolver(oc.rest_hessian(mdl))
    return SimpleNamespace(U_full=oc.ubar_rows(mdl, solver, mdl.free_ids), verts=mdl.free_ids)


@pytest.fixture(scope="module")
def exact_tab(tiny):
    return _exact_tables(tiny[1])


def test_literal_exact_at_rest_is_newton_step(tiny, exact_tab):
    """RX from x = X (R = I, H = H-bar): A_i is the Schur complement S_i and
    b_i = U-bar_i^T g, so the Jacobi sweep is the global Newton step."""
    import scipy.sparse.linalg as spla
    sc, mdl, _ = tiny
    z = mdl.inertial_target(mdl.X, sc.v0)
    x1 = osw.Sweeper(mdl, exact_tab, osw.RX).jacobi(mdl.X.copy(), z)
    H = mdl.hessian(mdl.X)
    dx = mdl.from_free(spla.spsolve(H.tocsc(), -mdl.to_free(mdl.gradient(mdl.X, z))))
    assert np.abs(x1 - (mdl.X + dx)).max() < 1e-10 * np.abs(dx).max()


def test_literal_exact_hessian_term_is_the_schur_complement(tiny, exact_tab, rest):
    """At rest H_ii + sum_a H_{i,a} U-bar_{i,a} = (H-bar^-1)_ii^-1, against a
    dense inverse of H-bar."""
    sc, mdl, _ = tiny
    z = mdl.inertial_target(mdl.X, sc.v0)
    verts = mdl.free_ids[::17]
    A, _ = osw.Sweeper(mdl, exact_tab, osw.RX).systems(mdl.X.copy(), z, verts)
    for k, v in enumerate(verts):
        f = mdl.free_index[v]
        S = np.linalg.inv(rest.Hinv[3 * f:3 * f + 3, 3 * f:3 * f + 3])
        assert np.abs(A[k] - S).max() < 1e-9 * np.abs(S).max()


def test_literal_exact_is_stationary_at_the_solution(tiny, exact_tab):
    from oracle import newton
    sc, mdl, _ = tiny
    xs, _ = newton.newton_solve(mdl, sc.x0, sc.v0, tol=1e-11)
    z = mdl.inertial_target(sc.x0, sc.v0)
    x1 = osw.Sweeper(mdl, exact_tab, osw.RX).jacobi(xs, z)
    diag = np.linalg.norm(mdl.X.max(0) - mdl.X.min(0))
    assert np.abs(x1 - xs).max() < 1e-9 * diag


def test_literal_exact_converges_within_newton_iterations(tiny, exact_tab):
    """The tiny beam's step from rest (Sec. 8.2's near-Newton claim): RX in
    Jacobi order reaches |g| / |g0| <= 1e-5 in at most 1.5 x the global
    Newton iteration count."""
    from oracle import newton
    sc, mdl, _ = tiny
    _, hist_n = newton.newton_solve(mdl, sc.x0, sc.v0, tol=1e-5)
    n_newton = len(hist_n) - 1
    _, _, hist = osw.run_step(osw.Sweeper(mdl, exact_tab, osw.RX), sc.x0, sc.v0, tol=1e-5, max_sweeps=20)
    assert hist[-1] <= 1e-5
    assert len(hist) - 1 <= 1.5 * n_newton, (len(hist) - 1, n_newton)


@pytest.mark.parametrize("E", [1e5, 1e8])
def test_literal_exact_converges_on_a_twisting_beam_at_both_stiffnesses(E):
    """4x4x32 beam (nu 0.45) with the benchmark's initial twist, three steps:
    every step reaches 1e-5 within 6 Jacobi sweeps at E = 1e5 and at E = 1e8
    (plain Gauss-Seidel needs hundreds at 1e5 and stalls at 1e8)."""
    sc = inputs.beam_scene(32, 4, 4, E=E, nu=0.45, steps=3)
    mdl = fem.model_from_scene(sc)
    sw = osw.Sweeper(mdl, _exact_tables(mdl), osw.RX)
    x, v = sc.x0.copy(), sc.v0.copy()
    for _ in range(3):
        x, v, hist = osw.run_step(sw, x, v, tol=1e-5, max_sweeps=12)
        assert hist[-1] <= 1e-5 and len(hist) - 1 <= 6, hist
