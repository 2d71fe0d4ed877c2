"""Writes the stored expected values used by the full-size GPU parity tests.

Calls only the FP64 oracle (``oracle/``) on the seeded single-beam workload
(16x16 cross-section, 128 long, 0.05 m cells; nu 0.45, E 1e5 and 1e8 Pa,
rho 1000, dt 1/120, initial twist 2 rad/s): the precompute on a sample of
free vertices (training-pose eigenvalues, one-ring U-bar rows, cubature
samples, weights, fit residuals, each vertex's NNLS system, and one R3
Jacobi sweep of those vertices from a twisted state), the positions of sampled vertices after
two plain Jacobi sweeps (omega 0.8) of the first step, and (E 1e5) after four
coloured GS sweeps with step scales 1.5 and 1.6, and the positions of
sampled vertices after one Jacobi sweep of the exact co-rotated subspace
from a prescribed twisted configuration.

    python tests/golden/make_goldens.py            # several minutes on one core
    python tests/golden/make_goldens.py gs_w1.6    # one of the files
    python tests/golden/make_goldens.py exact      # the exact-subspace sweep
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import correction as oc, fem, mesh as omesh, sweep as osw  # noqa: E402
from paper_2506_06494_amd import inputs  # noqa: E402

N_SAMPLED = 24
SEED = 0


def sampled_vertices(mdl, n, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(mdl.free_ids, n, replace=False))


def golden_precompute(E):
    sc = inputs.single_beam(E)
    mdl = fem.model_from_scene(sc)
    verts = sampled_vertices(mdl, N_SAMPLED, 1)
    tab = oc.precompute(mdl, verts=verts, S=4, n_cand=64, seed=SEED, keep_full=True)
    out = {"E": E, "lam": tab.lam.tolist(), "cid": tab.cid.tolist(), "verts": verts.tolist(), "rows": []}
    # one R3 Jacobi sweep (omega 1) at the sampled vertices with their own tables,
    # from the beam twisted by 0.3 rad over its length, at rest (x0 = x-hat, v = 0);
    # the local systems and the size of their sampled-element terms go beside it
    angle = 0.3
    x0 = inputs.twisted_positions(sc.mesh, angle)
    z = mdl.inertial_target(x0, np.zeros_like(x0))
    g, R = osw.phase1(mdl, x0, z)
    He = mdl.element_hessians(x0)
    ell = osw._Ell(mdl, tab, omesh.incidence(mdl.tets, mdl.nV))
    A, b = osw.r3_systems(mdl, tab, ell, x0, g, R, He, None)
    dx = osw.local_solve(A, b)
    wabs = np.abs(tab.weights).sum(axis=1) * np.abs(He).max()
    out["r3"] = {"angle": angle, "x": (x0[verts] + dx).tolist(), "dx": dx.tolist(), "A": A.tolist(),
                 "cond": [float(np.linalg.cond(a)) for a in A],
                 "sample_scale": [float(x) for x in wabs]}
    for k, v in enumerate(verts):
        # the vertex's NNLS system of Eq. cubature_weight restricted to its chosen
        # samples (normalised columns and right-hand side), and its conditioning
        b, column, _ = oc.cubature_system(mdl, tab.ring, tab.U_full[k], tab.G, tab.cid, int(v))
        chosen = [int(x) for x in tab.samples[k] if x >= 0]
        A = np.stack([column(x) for x in chosen], axis=1)
        sv = np.linalg.svd(A, compute_uv=False)
        out["rows"].append({"v": int(v), "ring": tab.nbr[k].tolist(),
                            "U_ring": np.asarray(tab.U_nbr[k]).reshape(-1, 9).tolist(),
                            "samples": tab.samples[k].tolist(), "weights": tab.weights[k].tolist(),
                            "U_samp": tab.U_samp[k].reshape(4, 4, 9).tolist(), "fit": float(tab.fit_res[k]),
                            "A": A.tolist(), "b": b.tolist(), "cond": float(sv[0] / sv[-1])})
    return out


def golden_plain_jacobi(E, sweeps=2, omega=0.8):
    sc = inputs.single_beam(E)
    mdl = fem.model_from_scene(sc)
    sw = osw.Sweeper(mdl, None, osw.P0, omega=omega)
    x, v, hist = osw.run_step(sw, sc.x0, sc.v0, sweeps=sweeps)
    verts = sampled_vertices(mdl, 200, 2)
    return {"E": E, "sweeps": sweeps, "omega": omega, "verts": verts.tolist(), "x": x[verts].tolist(),
            "rel_res": hist}


def golden_plain_gs(E, sweeps=4, omega=1.5):
    """Sampled positions after a few over-relaxed coloured GS sweeps (the
    benchmark's headline sweep) of the first step."""
    from oracle import mesh as omesh
    sc = inputs.single_beam(E)
    mdl = fem.model_from_scene(sc)
    col = omesh.greedy_coloring(omesh.one_ring(mdl.tets, mdl.nV), mdl.free)
    sw = osw.Sweeper(mdl, None, osw.P0, omega=omega)
    x, v, hist = osw.run_step(sw, sc.x0, sc.v0, sweeps=sweeps, mode="gs", color=col)
    verts = sampled_vertices(mdl, 200, 3)
    return {"E": E, "sweeps": sweeps, "omega": omega, "verts": verts.tolist(), "x": x[verts].tolist(),
            "rel_res": hist}


def golden_exact_jacobi(E, n=96, angle=0.3):
    """One Jacobi sweep of the exact co-rotated subspace (variant RX) at
    sampled vertices, from the beam twisted by `angle` over its length and at
    rest (x0 = x-hat = twisted, v = 0): each sampled vertex's step needs only
    its own U-bar row (three solves with the rest Hessian), the gradient,
    rotations and Hessian at x0."""
    sc = inputs.single_beam(E)
    mdl = fem.model_from_scene(sc)
    x0 = inputs.twisted_positions(sc.mesh, angle)
    v0 = np.zeros_like(x0)
    z = mdl.inertial_target(x0, v0)
    verts = sampled_vertices(mdl, n, 4)
    solver = oc.RestSolver(oc.rest_hessian(mdl))
    U = oc.ubar_rows(mdl, solver, verts)
    g, R = osw.phase1(mdl, x0, z)
    H = mdl.hessian(x0)
    A, b = osw.literal_exact_systems(mdl, osw.corotated_rows(U, R, verts), g, H, verts)
    dx = osw.local_solve(A, b)
    return {"E": E, "angle": angle, "verts": verts.tolist(), "x": (x0[verts] + dx).tolist(), "dx": dx.tolist(),
            "r0": float(np.linalg.norm(mdl.to_free(g)))}


def main():
    which = sys.argv[1:] or ["precompute", "jacobi", "gs", "exact"]
    for E in (1e5, 1e8):
        if "precompute" in which:
            path = os.path.join(HERE, f"beam16x16x128_E{E:g}_precompute.json")
            json.dump(golden_precompute(E), open(path, "w"))
            print("wrote", path, flush=True)
        if "exact" in which:
            path = os.path.join(HERE, f"beam16x16x128_E{E:g}_exact_jacobi.json")
            json.dump(golden_exact_jacobi(E), open(path, "w"))
            print("wrote", path, flush=True)
        if "jacobi" in which:
            path = os.path.join(HERE, f"beam16x16x128_E{E:g}_plain_jacobi.json")
            json.dump(golden_plain_jacobi(E), open(path, "w"))
            print("wrote", path, flush=True)
        for w in (1.5, 1.6):
            if ("gs" in which or f"gs_w{w:g}" in which) and E == 1e5:
                path = os.path.join(HERE, f"beam16x16x128_E{E:g}_plain_gs_w{w:g}.json")
                json.dump(golden_plain_gs(E, omega=w), open(path, "w"))
                print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
