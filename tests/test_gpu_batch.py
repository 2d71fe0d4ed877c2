"""Batched solve of several disjoint bodies in the same launches (per-body
residuals and stop masks), captured sweep groups, and the launch-shape
tuner.  A batched body must be bitwise the body solved alone."""
import numpy as np
import pytest

from oracle import fem, mesh as omesh, sweep as osw
from paper_2506_06494_amd import inputs, jgs2

from gpu_util import bbox_diag, make_solver

pytestmark = pytest.mark.gpu

BEAMS = [(12, 4, 4, 1e5, 0.45), (16, 3, 5, 3e5, 0.40), (8, 6, 4, 1e4, 0.30), (10, 2, 2, 2e6, 0.48)]


def beam_parts():
    parts = []
    for (L, a, b, E, nu) in BEAMS:
        m = inputs.beam_mesh(L, a, b, 0.05)
        v0 = inputs.twist_velocity(m, 2.0)
        parts.append((m, np.full(m.nT, E), np.full(m.nT, nu), v0))
    return parts


def solver_for(m, E, nu, **kw):
    p = dict(order=jgs2.GS, rel_tol=1e-5, check_every=8, max_sweeps=4000)
    p.update(kw)
    s = jgs2.Solver(**p)
    s.upload_mesh(m.X, m.tets, m.pinned)
    s.set_material(E, nu, 1000.0)
    return s


def batched(parts, **kw):
    u = inputs.concat_meshes([p[0] for p in parts])
    s = solver_for(u, np.concatenate([p[1] for p in parts]), np.concatenate([p[2] for p in parts]), **kw)
    s.set_bodies(u.body)
    s.set_state(u.X, np.concatenate([p[3] for p in parts]))
    return s, u


@pytest.mark.parametrize("order,omega", [(jgs2.GS, 1.0), (jgs2.GS, 1.5), (jgs2.JACOBI, 0.5)])
def test_batched_bodies_are_bitwise_the_single_solves(order, omega):
    parts = beam_parts()
    sb, u = batched(parts, order=order, omega=omega)
    for _ in range(2):
        st = sb.step()
    xb, vb = sb.get_state()
    sweeps_b, rel_b = sb.body_stats()
    off = np.concatenate([[0], np.cumsum([p[0].nV for p in parts])])
    for k, (m, E, nu, v0) in enumerate(parts):
        s1 = solver_for(m, E, nu, order=order, omega=omega)
        s1.set_state(m.X, v0)
        for _ in range(2):
            st1 = s1.step()
        x1, v1 = s1.get_state()
        assert np.array_equal(xb[off[k]:off[k + 1]], x1), k
        assert np.array_equal(vb[off[k]:off[k + 1]], v1), k
        assert sweeps_b[k] == st1["sweeps"], (k, sweeps_b[k], st1["sweeps"])
    assert st["sweeps"] == sweeps_b.max()
    if order == jgs2.GS:
        # the bodies really stopped at different sweep counts
        assert len(set(sweeps_b.tolist())) > 1


def test_batched_body_matches_oracle():
    """One batched body against the oracle with the body's own sweep count."""
    parts = beam_parts()
    sb, u = batched(parts)
    sb.begin_step()
    sb.iterate(24)
    xb, _ = sb.get_state()
    m, E, nu, v0 = parts[1]
    off = parts[0][0].nV
    mdl = fem.Model(m.X, m.tets, m.pinned, E, nu, 1000.0, 1.0 / 120)
    col = omesh.greedy_coloring(omesh.one_ring(mdl.tets, mdl.nV), mdl.free)
    sw_b, _ = sb.body_stats()
    xo, _, _ = osw.run_step(osw.Sweeper(mdl, None, osw.P0), m.X, v0, sweeps=int(sw_b[1]), mode="gs", color=col)
    assert np.abs(xb[off:off + m.nV] - xo).max() <= 1e-5 * bbox_diag(m.X)


@pytest.mark.parametrize("order,check", [(jgs2.GS, 8), (jgs2.JACOBI, 3)])
def test_graph_replay_is_bitwise_eager(order, check):
    parts = beam_parts()
    out = []
    for g in (0, 1):
        s, u = batched(parts, order=order, omega=0.5 if order == jgs2.JACOBI else 1.0, check_every=check, use_graph=g)
        stats = [s.step() for _ in range(3)]
        out.append((s.get_state(), [st["sweeps"] for st in stats], s.body_stats()[0]))
    (x0, v0), sw0, b0 = out[0]
    (x1, v1), sw1, b1 = out[1]
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    assert sw0 == sw1 and np.array_equal(b0, b1)


@pytest.mark.parametrize("lpv,block", [(4, 64), (8, 128), (16, 512), (32, 256), (32, 64)])
def test_launch_shapes_match_oracle(tiny, lpv, block):
    sc, mdl, _ = tiny
    s = make_solver(sc, variant=jgs2.PLAIN, order=jgs2.GS)
    s.set_tuning(lpv, block)
    assert s.tuning() == (lpv, block)
    s.set_state(sc.x0, sc.v0)
    s.begin_step()
    s.iterate(20)
    xg, _ = s.get_state()
    col = omesh.greedy_coloring(omesh.one_ring(mdl.tets, mdl.nV), mdl.free)
    xo, _, _ = osw.run_step(osw.Sweeper(mdl, None, osw.P0), sc.x0, sc.v0, sweeps=20, mode="gs", color=col)
    assert np.abs(xg - xo).max() <= 1e-5 * bbox_diag(mdl.X)


def test_autotune_keeps_state_and_picks_a_valid_shape(tiny):
    sc, mdl, _ = tiny
    s = make_solver(sc, variant=jgs2.PLAIN, order=jgs2.GS)
    s.set_state(sc.x0, sc.v0)
    x0, v0 = s.get_state()
    (lpv, block), ms = s.autotune(8)
    assert lpv in (4, 8, 16, 32) and block in (64, 128, 256, 512)
    assert np.all(ms > 0) and ms.min() == ms[[4, 8, 16, 32].index(lpv), [64, 128, 256, 512].index(block)]
    assert s.tuning() == (lpv, block)
    x, v = s.get_state()
    assert np.array_equal(x, x0) and np.array_equal(v, v0)
    st = s.step()
    assert st["status"] == 0


def test_body_errors():
    m = inputs.beam_mesh(4, 2, 2, 0.05)
    s = solver_for(m, np.full(m.nT, 1e5), np.full(m.nT, 0.45))
    with pytest.raises(jgs2.JGS2Error):
        s.set_bodies(np.arange(m.nV) % 2)          # tets would span two bodies
    with pytest.raises(jgs2.JGS2Error):
        s.set_tuning(3, 256)


@pytest.mark.parametrize("bodies", [False, True])
def test_streamed_records_are_bitwise_cached(bodies):
    """Streaming the incidence records (non-temporal loads) is a cache hint
    only: two steps with it forced on, forced off and on the automatic
    setting agree bit for bit, for one body and for batched bodies."""
    parts = beam_parts()
    out = []
    for mode in (0, 1, -1):
        if bodies:
            s, _ = batched(parts, order=jgs2.GS, omega=1.5, use_graph=1)
        else:
            m, E, nu, v0 = parts[0]
            s = solver_for(m, E, nu, order=jgs2.GS, omega=1.5, use_graph=1)
            s.set_state(m.X, v0)
        s.set_streaming(mode)
        stats = [s.step() for _ in range(2)]
        out.append((s.get_state(), [st["sweeps"] for st in stats]))
    (x0, v0), sw0 = out[0]
    for (x, v), sw in out[1:]:
        assert np.array_equal(x, x0) and np.array_equal(v, v0) and sw == sw0
    with pytest.raises(jgs2.JGS2Error):
        s.set_streaming(2)


@pytest.mark.parametrize("bodies,lpv", [(False, 16), (True, 8), (True, 32)])
def test_persistent_gs_is_bitwise_the_per_colour_launches(bodies, lpv):
    """Coloured GS groups as one cooperative launch (grid barriers between
    colours) give bit for bit the per-colour launches (captured graphs), for
    one body and for batched bodies that stop at different sweep counts, in
    several lane counts per vertex; the sweeps per body agree too."""
    parts = beam_parts()
    out = []
    for persistent in (False, True):
        if bodies:
            s, _ = batched(parts, order=jgs2.GS, omega=1.5, use_graph=1)
        else:
            m, E, nu, v0 = parts[0]
            s = solver_for(m, E, nu, order=jgs2.GS, omega=1.5, use_graph=1)
            s.set_state(m.X, v0)
        s.set_tuning(lpv, 256)
        s.set_persistent(persistent)
        stats = [s.step() for _ in range(2)]
        sweeps = s.body_stats()[0] if bodies else None
        out.append((s.get_state(), [st["sweeps"] for st in stats], sweeps))
    (x0, v0), sw0, b0 = out[0]
    (x1, v1), sw1, b1 = out[1]
    assert np.array_equal(x1, x0) and np.array_equal(v1, v0) and sw1 == sw0
    if bodies:
        assert np.array_equal(b1, b0)
    with pytest.raises(jgs2.JGS2Error):
        s.set_persistent(2)
