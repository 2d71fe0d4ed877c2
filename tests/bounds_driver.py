"""Runs the sweeps of the index-checked library (libjgs2_bounds.so, built
with JGS2_BOUNDS_CHECK) on small generated beams and prints one JSON line:
the first failed index check after each phase (line 0: none), the tile
counts of the exact variant, and the self-test's record.  Phases: exact
Jacobi and GS with dead tiles, exact Jacobi with FP16 tiles, the exact adjoint, plain Jacobi and GS, the
damper sweeps, batched bodies, a plain rollout and its adjoint.  Run by
tests/test_zy_bounds.py in a process of its own (the binding loads one
library per process)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2506_06494_amd import inputs, jgs2  # noqa: E402


def solver(sc, **kw):
    s = jgs2.Solver(dt=sc.dt, gravity=sc.gravity, rel_tol=1e-5, max_sweeps=400, **kw)
    s.upload_mesh(sc.mesh.X, sc.mesh.tets, sc.mesh.pinned)
    s.set_material(sc.E, sc.nu, sc.rho)
    return s


def main():
    jgs2.load(jgs2.BOUNDS_LIB_PATH)
    out = {}

    def record(name, s, sts):
        line, idx, ext = s.bounds_report()
        out[name] = dict(line=line, index=idx, extent=ext, status=[int(r["status"]) for r in sts])
        print(f"[bounds] {name}: line {line} status {out[name]['status']}", file=sys.stderr, flush=True)

    # exact variant, a beam long enough for tiles below the drop threshold
    sc = inputs.beam_scene(64, 4, 4, E=1e5, steps=2)
    s = solver(sc, variant=jgs2.EXACT, order=jgs2.JACOBI, check_every=1, exact_drop=1e-5)
    s.precompute(samples=4, n_cand=64, seed=0)
    out["tiles"] = s.exact_tiles()
    s.set_state(sc.x0, sc.v0)
    record("exact_jacobi", s, [s.step(raise_on_error=False) for _ in range(2)])
    s.set_params(order=jgs2.GS)
    record("exact_gs", s, [s.step(raise_on_error=False) for _ in range(1)])
    s.exact_tiles_fp16()
    s.set_params(order=jgs2.JACOBI)
    record("exact_jacobi_fp16", s, [s.step(raise_on_error=False) for _ in range(2)])
    s.set_params(order=jgs2.JACOBI, exact_drop=0.0)
    s.set_state(sc.x0, sc.v0)
    s.rollout(2, ckpt_every=1)
    xbar = np.zeros_like(sc.x0)
    xbar[-1, 1] = 1.0
    s.rollout_backward(xbar)
    record("exact_rollout_adjoint", s, [])
    s.close()

    # plain Jacobi and GS, damper GS on the tiny beam
    sc = inputs.tiny_beam()
    for name, kw in (("plain_jacobi", dict(variant=jgs2.PLAIN, order=jgs2.JACOBI, omega=0.5)),
                     ("plain_gs", dict(variant=jgs2.PLAIN, order=jgs2.GS)),
                     ("damper_gs", dict(variant=jgs2.DAMPER, order=jgs2.GS))):
        s = solver(sc, **kw)
        if kw["variant"] != jgs2.PLAIN:
            s.precompute(samples=4, n_cand=64, seed=0)
        s.set_state(sc.x0, sc.v0)
        record(name, s, [s.step(raise_on_error=False) for _ in range(2)])
        s.close()

    # two beams as bodies, plain GS; a plain rollout and its adjoint
    parts = [inputs.beam_mesh(8, 2, 2, 0.05), inputs.beam_mesh(12, 3, 2, 0.05)]
    u = inputs.concat_meshes(parts)
    s = jgs2.Solver(dt=1.0 / 120, gravity=(0.0, -9.8, 0.0), rel_tol=1e-5, max_sweeps=400,
                    variant=jgs2.PLAIN, order=jgs2.GS)
    s.upload_mesh(u.X, u.tets, u.pinned)
    s.set_material(np.full(u.nT, 1e5), np.full(u.nT, 0.45), np.full(u.nT, 1000.0))
    s.set_bodies(u.body)
    s.set_state(u.X, np.zeros_like(u.X))
    record("bodies_gs", s, [s.step(raise_on_error=False) for _ in range(2)])
    s.close()

    sc = inputs.tiny_beam()
    s = solver(sc, variant=jgs2.PLAIN, order=jgs2.GS)
    s.set_state(sc.x0, sc.v0)
    s.rollout(3, ckpt_every=2)
    xbar = np.zeros_like(sc.x0)
    xbar[-1, 1] = 1.0
    s.rollout_backward(xbar)
    record("plain_rollout_adjoint", s, [])

    # the reporting path: one recorded failure from a kernel that touches no buffer
    s.bounds_selftest()
    out["selftest"] = list(s.bounds_report(clear=True))
    out["after_clear"] = list(s.bounds_report())
    s.set_state(sc.x0, sc.v0)
    record("after_selftest", s, [s.step(raise_on_error=False)])
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
