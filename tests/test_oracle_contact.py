"""Pins of the oracle's contact handling: the per-vertex feasibility clamp
and the energy backtracking line search."""
import numpy as np

from oracle import fem, sweep as osw
from paper_2506_06494_amd import inputs


def test_feasibility_clamp_keeps_every_vertex_in_front_of_the_planes():
    sc = inputs.sphere_on_floor()
    mdl = fem.model_from_scene(sc)
    rng = np.random.default_rng(0)
    x = sc.x0[mdl.free_ids]
    step = rng.standard_normal(x.shape) * 0.05
    step[:, 2] = -np.abs(step[:, 2])                      # everything approaches the floor
    st = osw.feasibility_clamp(mdl, x, step)
    d0 = x[:, 2]
    d1 = (x + st)[:, 2]
    assert np.all(d1 >= 0.1 * d0 - 1e-15)
    # moves away from the plane, or short enough, are untouched
    short = -step[:, 2] < 0.9 * d0
    np.testing.assert_array_equal(st[short], step[short])
    # no planes: identity
    mdl.planes = np.zeros((0, 4))
    np.testing.assert_array_equal(osw.feasibility_clamp(mdl, x, step), step)


def test_line_search_never_increases_the_potential():
    sc = inputs.sphere_on_floor(speed=3.0)
    mdl = fem.model_from_scene(sc)
    sw = osw.Sweeper(mdl, None, osw.P0, omega=1.0, line_search=True)
    z = mdl.inertial_target(sc.x0, sc.v0)
    x = sc.x0.copy()
    e = [mdl.energy(x, z)]
    for _ in range(8):
        x = sw.jacobi(x, z)
        e.append(mdl.energy(x, z))
        assert np.isfinite(e[-1])
    # each accepted sweep lowers E unless all 8 halvings were spent
    assert e[-1] < e[0]
    assert np.min((x @ mdl.planes[0, :3] - mdl.planes[0, 3])[mdl.free]) > 0
