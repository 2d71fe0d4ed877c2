"""The allocation-free energy entry point against jgs2_energy on the GPU:
two calls in a row, the second on a smaller mesh, each equal to the energy
of the existing entry point on the same handle and state."""
import numpy as np
import pytest

from paper_2506_06494_amd import inputs, jgs2

from gpu_util import make_solver

pytestmark = pytest.mark.gpu


def _deformed(sc, seed):
    rng = np.random.default_rng(seed)
    x = sc.x0 + 2e-3 * rng.standard_normal(sc.x0.shape)
    x[sc.mesh.pinned] = sc.mesh.X[sc.mesh.pinned]
    return x


def test_energy_noalloc_matches_energy_on_two_calls():
    big = inputs.beam_scene(24, 6, 6, E=1e6, steps=1)        # 1,225 vertices, 5,184 tets
    small = inputs.tiny_beam()                                # 425 vertices, 1,536 tets
    assert small.mesh.nT < big.mesh.nT
    for k, sc in enumerate((big, small)):
        s = make_solver(sc, variant=jgs2.PLAIN, order=jgs2.GS)
        s.set_state(_deformed(sc, k), sc.v0)
        s.begin_step()
        e_ref = s.energy()
        e_new = s.energy_noalloc()
        print(f"call {k}: {sc.mesh.nT} tets, energy {e_ref!r} / noalloc {e_new!r}", flush=True)
        # the same kernels and order of summation: equal up to the last bit
        assert np.isfinite(e_ref) and e_new == e_ref
        s.close()
