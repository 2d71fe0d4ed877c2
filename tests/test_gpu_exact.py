"""GPU parity of the exact co-rotated subspace (variant RX of the oracle,
JGS2_EXACT of the library: the literal form of Eq. local_newton with every
row of U-bar, no cubature).  The library computes its own U-bar rows on the
GPU (FP64 band solves, stored in FP32); the oracle uses a dense FP64
Cholesky factor of the rest Hessian."""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import correction as oc, fem, mesh as omesh, newton, sweep as osw
from paper_2506_06494_amd import inputs, jgs2

from gpu_util import bbox_diag, make_solver

pytestmark = pytest.mark.gpu


def exact_tables(mdl):
    solver = oc.RestSolver(oc.rest_hessian(mdl))
    return SimpleNamespace(U_full=oc.ubar_rows(mdl, solver, mdl.free_ids), verts=mdl.free_ids)


def gpu_exact(sc, **kw):
    s = make_solver(sc, variant=jgs2.EXACT, **kw)
    s.precompute(samples=4, n_cand=64, seed=0)
    return s


@pytest.fixture(scope="module")
def tiny_exact(tiny):
    sc, mdl, _ = tiny
    return exact_tables(mdl)


@pytest.mark.parametrize("order,sweeps", [(jgs2.JACOBI, 1), (jgs2.JACOBI, 3), (jgs2.GS, 2)])
def test_exact_sweeps_match_oracle(tiny, tiny_exact, order, sweeps):
    sc, mdl, _ = tiny
    s = gpu_exact(sc, order=order)
    s.set_state(sc.x0, sc.v0)
    s.begin_step()
    rel = s.iterate(sweeps)
    xg, _ = s.get_state()
    s.close()
    col = omesh.greedy_coloring(omesh.one_ring(mdl.tets, mdl.nV), mdl.free)
    xo, _, hist = osw.run_step(osw.Sweeper(mdl, tiny_exact, osw.RX), sc.x0, sc.v0, sweeps=sweeps,
                               mode="jacobi" if order == jgs2.JACOBI else "gs", color=col)
    moved = np.abs(xo - sc.x0).max()
    err = np.abs(xg - xo).max()
    print(f"order {order} sweeps {sweeps}: max |x_gpu - x_oracle| = {err:.3e} (moved {moved:.3e}); "
          f"rel {rel:.3e} / {hist[-1]:.3e}", flush=True)
    assert err <= 1e-5 * bbox_diag(mdl.X)
    assert err <= 2e-3 * moved
    assert abs(rel - hist[-1]) <= 2e-2 * hist[-1] + 1e-6


@pytest.mark.parametrize("order", [jgs2.JACOBI, jgs2.GS])
def test_exact_step_converges_to_newton_solution(tiny, order):
    sc, mdl, _ = tiny
    s = gpu_exact(sc, order=order, rel_tol=1e-5, max_sweeps=50, check_every=1)
    s.set_state(sc.x0, sc.v0)
    st = s.step()
    xg, vg = s.get_state()
    s.close()
    _, hist_n = newton.newton_solve(mdl, sc.x0, sc.v0, tol=1e-5)
    print(f"order {order}: {st['sweeps']} sweeps (Newton {len(hist_n) - 1} iterations), r {st['r_final']:.2e}",
          flush=True)
    assert st["status"] == jgs2.OK and st["r_final"] <= 1e-5
    assert st["sweeps"] <= 1.5 * (len(hist_n) - 1) + 1
    xs, _ = newton.newton_solve(mdl, sc.x0, sc.v0, tol=1e-11)
    assert np.abs(xg - xs).max() <= 1e-5 * bbox_diag(mdl.X)
    np.testing.assert_allclose(vg, (xg - sc.x0) / sc.dt, atol=1e-4)


@pytest.mark.parametrize("E", [1e5, 1e8])
def test_exact_twisting_beam_steps_match_oracle(E):
    """4x4x32 beam with the benchmark's twist, three converged steps at
    each stiffness: every GPU step reaches 1e-5 within 8 sweeps, and the
    positions match the oracle's converged steps."""
    sc = inputs.beam_scene(32, 4, 4, E=E, nu=0.45, steps=3)
    mdl = fem.model_from_scene(sc)
    s = gpu_exact(sc, order=jgs2.JACOBI, rel_tol=1e-5, max_sweeps=40, check_every=1)
    sw = osw.Sweeper(mdl, exact_tables(mdl), osw.RX)
    s.set_state(sc.x0, sc.v0)
    x, v = sc.x0.copy(), sc.v0.copy()
    diag = bbox_diag(mdl.X)
    for k in range(3):
        st = s.step()
        xg, _ = s.get_state()
        x, v, hist = osw.run_step(sw, x, v, tol=1e-5, max_sweeps=12)
        err = np.abs(xg - x).max()
        print(f"E {E:g} step {k}: GPU {st['sweeps']} sweeps r {st['r_final']:.2e}; oracle {len(hist) - 1} sweeps; "
              f"max |dx| {err:.3e}", flush=True)
        assert st["status"] == jgs2.OK and st["sweeps"] <= 8
        assert err <= 1e-5 * diag
    s.close()


@pytest.mark.parametrize("E", [1e5])
def test_exact_fp16_tiles_steps_match_oracle(E):
    """The same three converged steps with H-bar^-1's tiles stored in FP16
    (each tile scaled by its largest entry), on the soft beam: the tiles only
    form the correction, so the steps converge to the oracle's positions in
    as few sweeps; the conversion halves the streamed bytes, a second call
    changes nothing and a new precompute brings FP32 tiles back.  (At
    E = 1e8 FP16 entries are too coarse for the stiff rest Hessian's
    inverse: the steps stall near r = 1e-2.)"""
    sc = inputs.beam_scene(32, 4, 4, E=E, nu=0.45, steps=3)
    mdl = fem.model_from_scene(sc)
    s = gpu_exact(sc, order=jgs2.JACOBI, rel_tol=1e-5, max_sweeps=40, check_every=1)
    t32 = s.exact_tiles()
    s.exact_tiles_fp16()
    s.exact_tiles_fp16()
    t16 = s.exact_tiles()
    assert t16["n_live"] == t32["n_live"] and t16["live_bytes"] == t32["live_bytes"] / 2
    sw = osw.Sweeper(mdl, exact_tables(mdl), osw.RX)
    s.set_state(sc.x0, sc.v0)
    x, v = sc.x0.copy(), sc.v0.copy()
    diag = bbox_diag(mdl.X)
    for k in range(3):
        st = s.step()
        xg, _ = s.get_state()
        x, v, hist = osw.run_step(sw, x, v, tol=1e-5, max_sweeps=12)
        err = np.abs(xg - x).max()
        print(f"E {E:g} FP16 step {k}: GPU {st['sweeps']} sweeps r {st['r_final']:.2e}; oracle {len(hist) - 1} "
              f"sweeps; max |dx| {err:.3e}", flush=True)
        assert st["status"] == jgs2.OK and st["sweeps"] <= 8
        assert err <= 1e-5 * diag
    s.precompute(samples=4, n_cand=64, seed=0)
    assert s.exact_tiles()["live_bytes"] == t32["live_bytes"]
    s.close()


def test_exact_needs_its_tables(tiny):
    sc, mdl, tab = tiny
    s = make_solver(sc, variant=jgs2.EXACT)
    s.set_state(sc.x0, sc.v0)
    st = s.step(raise_on_error=False)
    assert st["status"] == jgs2.E_NOT_READY
    s.close()


def test_exact_adjoint_matches_oracle_adjoint():
    """The differentiable rollout with the exact subspace in the forward
    steps and in the adjoint's linear sweeps (the same local systems of
    H(x*) y = rhs, residual in place of the gradient): stiffness and initial
    state cotangents against the FP64 oracle adjoint, with few sweeps per
    adjoint solve."""
    from oracle import adjoint as oa
    m = inputs.beam_mesh(8, 3, 3, 0.05)
    g = inputs.SplitMix64(11)
    logE = np.log(1e5) + g.uniform_array(m.nT, -0.3, 0.3)
    u = np.array([0.05, -0.1, 0.2])
    n = 5
    mdl = fem.Model(m.X, m.tets, m.pinned, np.exp(logE), 0.45, 1000.0, 1.0 / 120)
    v0 = np.zeros_like(m.X)
    v0[~m.pinned.astype(bool)] = u
    xs, _ = oa.forward(mdl, mdl.X.copy(), oa.initial_velocity(mdl, u), n)
    rng = np.random.default_rng(3)
    xbar = rng.standard_normal(m.X.shape)
    vbar = 0.01 * rng.standard_normal(m.X.shape)
    th_o, xb_o, vb_o = oa.backward(mdl, xs, xbar, vbar)
    s = jgs2.Solver(variant=jgs2.EXACT, order=jgs2.JACOBI, rel_tol=1e-6, adj_rel_tol=1e-6, check_every=1,
                    max_sweeps=50, adj_max_sweeps=50)
    s.upload_mesh(m.X, m.tets, m.pinned)
    s.set_material(np.exp(logE), 0.45, 1000.0)
    s.precompute(samples=4, n_cand=64, seed=0)
    s.set_state(m.X, v0)
    assert s.rollout(n, ckpt_every=2)["status"] == jgs2.OK
    x, _ = s.get_state()
    assert np.abs(x - xs[-1]).max() <= 1e-5 * bbox_diag(m.X)
    th, xb0, vb0, st = s.rollout_backward(xbar, vbar)
    s.close()
    print(f"exact adjoint: {st['adjoint_sweeps']} adjoint sweeps over {st['steps']} steps, "
          f"max rel res {st['max_rel_res']:.2e}", flush=True)
    assert st["status"] == jgs2.OK and st["steps"] == n and st["max_rel_res"] <= 1e-6
    assert st["adjoint_sweeps"] <= 6 * n
    rel = np.linalg.norm(th - th_o) / np.linalg.norm(th_o)
    cos = th @ th_o / (np.linalg.norm(th) * np.linalg.norm(th_o))
    assert rel <= 1e-2 and cos >= 0.999, (rel, cos)
    pin = m.pinned.astype(bool)
    for a, b in ((xb0, xb_o), (vb0, vb_o)):
        assert np.linalg.norm(a[~pin] - b[~pin]) <= 1e-2 * np.linalg.norm(b[~pin])


def test_exact_sweep_with_indefinite_local_systems_matches_oracle(tiny, tiny_exact):
    """A state where an exact local system is indefinite (one interior
    vertex pushed 0.05 m, a cell length, towards its neighbours; the
    per-vertex mean deformation gradients stay well conditioned, smallest
    singular value 0.68, so the rotations are not in question): the PD guard
    of the local solve shifts it on both sides (the same pivot rule), and one
    Jacobi sweep matches the oracle."""
    sc, mdl, _ = tiny
    x0 = sc.x0.copy()
    x0[156, 1] += 0.05
    z = mdl.inertial_target(x0, sc.v0)          # the GPU step starts from x-hat = x0
    sw = osw.Sweeper(mdl, tiny_exact, osw.RX)
    A, _ = sw.systems(x0, z)
    shifted = [k for k in range(A.shape[0])
               if osw._ldl_pivots(A[k]).min() <= 1e-6 * abs(np.trace(A[k]))]
    assert len(shifted) >= 1
    xo = sw.jacobi(x0, z)
    s = gpu_exact(sc, order=jgs2.JACOBI)
    s.set_state(x0, sc.v0)
    s.begin_step()
    s.iterate(1)
    xg, _ = s.get_state()
    s.close()
    # In one Jacobi sweep every row's step depends on its own system only.
    # Near an inversion some systems are badly conditioned (the guard leaves
    # a shifted system's smallest pivot at 1e-6 tr A, and unshifted ones can
    # sit just above that); the GPU assembles A_i in FP32 (a sum of one-ring
    # terms that largely cancel), good to about 1e-6 of its size, so a row's
    # step is held to (2e-3 + 1e-6 cond(A_i)) of its length, cond taken from
    # the oracle's guarded system.
    def guarded(M):
        tr, shift = np.trace(M), 0.0
        for _ in range(60):
            Ms = M + shift * np.eye(3)
            d = osw._ldl_pivots(Ms)
            if d.min() > 1e-6 * abs(tr):
                return Ms
            shift = (abs(d.min()) + 1e-6 * abs(tr)) if shift == 0.0 else 2.0 * shift
        return Ms
    worst = 0.0
    for k, v in enumerate(mdl.free_ids):
        dg, do = xg[v] - x0[v], xo[v] - x0[v]
        kappa = np.linalg.cond(guarded(A[k]))
        tol = (2e-3 + 1e-6 * kappa) * np.linalg.norm(do) + 1e-12
        worst = max(worst, np.linalg.norm(dg - do) / tol)
        if k in shifted:
            print(f"shifted row {v}: cond {kappa:.2e}, |dx| {np.linalg.norm(do):.3e}, "
                  f"|dx_gpu - dx_oracle| {np.linalg.norm(dg - do):.3e}", flush=True)
        assert np.all(np.isfinite(dg)) and np.linalg.norm(dg - do) <= tol, (v, kappa, dg, do)
    print(f"{len(shifted)} shifted systems; worst error / tolerance {worst:.3f}", flush=True)


def test_exact_batched_bodies_match_the_single_solves():
    """Three beams of different size and stiffness uploaded as one mesh with
    their own bodies, exact Jacobi, two steps: the rest Hessian is block
    diagonal, so every tile coupling two bodies is exactly zero and is not
    streamed even with exact_drop 0; each body's steps match the body solved
    alone to FP32 summation order (the tiles group the sums differently) and
    take the same sweeps within one."""
    specs = [(16, 4, 4, 1e5, 0.45), (12, 3, 5, 1e6, 0.40), (10, 4, 3, 1e8, 0.45)]
    meshes, Es, nus, v0s = [], [], [], []
    for (L, a, b, E, nu) in specs:
        m = inputs.beam_mesh(L, a, b, 0.05)
        meshes.append(m)
        Es.append(np.full(m.nT, E))
        nus.append(np.full(m.nT, nu))
        v0s.append(inputs.twist_velocity(m, 2.0))
    u = inputs.concat_meshes(meshes)
    kw = dict(variant=jgs2.EXACT, order=jgs2.JACOBI, rel_tol=1e-5, check_every=1, max_sweeps=40, exact_drop=0.0)
    s = jgs2.Solver(**kw)
    s.upload_mesh(u.X, u.tets, u.pinned)
    s.set_material(np.concatenate(Es), np.concatenate(nus), 1000.0)
    s.set_bodies(u.body)
    s.precompute(samples=4, n_cand=64, seed=0)
    tiles = s.exact_tiles()
    assert tiles["n_live"] < tiles["n_tiles"], tiles
    s.set_state(u.X, np.concatenate(v0s))
    for _ in range(2):
        s.step()
    xb, _ = s.get_state()
    sweeps_b, _ = s.body_stats()
    off = np.concatenate([[0], np.cumsum([m.nV for m in meshes])])
    for k, m in enumerate(meshes):
        s1 = jgs2.Solver(**kw)
        s1.upload_mesh(m.X, m.tets, m.pinned)
        s1.set_material(Es[k], nus[k], 1000.0)
        s1.precompute(samples=4, n_cand=64, seed=0)
        s1.set_state(m.X, v0s[k])
        for _ in range(2):
            st1 = s1.step()
        x1, _ = s1.get_state()
        err = np.abs(xb[off[k]:off[k + 1]] - x1).max()
        print(f"body {k}: {sweeps_b[k]} / {st1['sweeps']} sweeps (batched / alone), max |dx| {err:.3e}", flush=True)
        assert err <= 1e-6 * bbox_diag(m.X)
        assert abs(int(sweeps_b[k]) - int(st1["sweeps"])) <= 1
        s1.close()
    s.close()
