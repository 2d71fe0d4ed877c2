"""GPU parity of the damper reading of the correction (variant R2D of the
oracle, JGS2_DAMPER of the library) on the tiny cantilever: a fixed number
of sweeps in both parallel orders against the FP64 oracle, and a full step
to the residual tolerance against the global Newton solution."""
import numpy as np
import pytest

from oracle import mesh as omesh, newton, sweep as osw
from paper_2506_06494_amd import jgs2

from gpu_util import bbox_diag, make_solver, oracle_tables_to_import

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order,omega,sweeps", [(jgs2.GS, 1.0, 40), (jgs2.JACOBI, 0.8, 40)])
def test_damper_sweeps_match_oracle(tiny, order, omega, sweeps):
    sc, mdl, tab = tiny
    s = make_solver(sc, variant=jgs2.DAMPER, order=order, omega=omega)
    s.import_correction(**oracle_tables_to_import(tab))
    s.set_state(sc.x0, sc.v0)
    s.begin_step()
    rel = s.iterate(sweeps)
    xg, _ = s.get_state()
    sw = osw.Sweeper(mdl, tab, osw.R2D, omega=omega)
    col = omesh.greedy_coloring(omesh.one_ring(mdl.tets, mdl.nV), mdl.free)
    xo, _, hist = osw.run_step(sw, sc.x0, sc.v0, sweeps=sweeps,
                               mode="jacobi" if order == jgs2.JACOBI else "gs", color=col)
    moved = np.abs(xo - sc.x0).max()
    assert np.abs(xg - xo).max() <= 1e-5 * bbox_diag(mdl.X)
    assert np.abs(xg - xo).max() <= 1e-3 * moved
    assert abs(rel - hist[-1]) <= 1e-3 * hist[-1] + 1e-6


def test_damper_gs_step_converges_to_newton_solution(tiny):
    sc, mdl, tab = tiny
    s = make_solver(sc, variant=jgs2.DAMPER, order=jgs2.GS, rel_tol=1e-5, max_sweeps=20000, check_every=16)
    s.import_correction(**oracle_tables_to_import(tab))
    s.set_state(sc.x0, sc.v0)
    st = s.step()
    assert st["status"] == jgs2.OK and st["r_final"] <= 1e-5
    xg, vg = s.get_state()
    xs, _ = newton.newton_solve(mdl, sc.x0, sc.v0, tol=1e-11)
    assert np.abs(xg - xs).max() <= 1e-5 * bbox_diag(mdl.X)
    np.testing.assert_allclose(vg, (xg - sc.x0) / sc.dt, atol=1e-4)
