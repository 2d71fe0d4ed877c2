"""Writes the stored oracle adjoint of the differentiation workload.

Calls only the FP64 oracle (``oracle/``): the 16x16x64 beam (18,785
vertices, 98,304 tets; 0.05 m cells, nu 0.45, rho 1000, dt 1/120, pinned at
x = 0, gravity on), per-tet log E = log 1e6 + U(-0.3, 0.3) and the tip
target from the seeded generator, initial velocity u = 0, 30 implicit-Euler
steps solved by global Newton to |g|/|g0| <= 1e-10, the loss
|tip centroid - target|^2 and its adjoint.  Stores the loss, dL/du, the
norm of dL/dlog E, its entries at 4096 sampled tets, and sampled final
positions.

    python tests/golden/make_adjoint_golden.py      # ~40 min on one core
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import adjoint as oa, fem  # noqa: E402
from paper_2506_06494_amd import inputs  # noqa: E402

N_STEPS = 30


def main():
    sc, logE, target = inputs.diff_beam(0)
    m = sc.mesh
    mdl = fem.Model(m.X, m.tets, m.pinned, np.exp(logE), 0.45, 1000.0, sc.dt)
    t0 = time.time()
    xs, _ = oa.forward(mdl, mdl.X.copy(), oa.initial_velocity(mdl, np.zeros(3)), N_STEPS, tol=1e-10)
    print(f"forward {time.time() - t0:.0f} s", flush=True)
    L, gx = oa.tip_loss(mdl, xs[-1], target)
    th, _, vb0 = oa.backward(mdl, xs, gx)
    print(f"backward done {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(5)
    tets = np.sort(rng.choice(mdl.nT, 4096, replace=False))
    verts = np.sort(rng.choice(mdl.nV, 256, replace=False))
    out = dict(steps=N_STEPS, loss=L, target=np.asarray(target).tolist(), ubar=vb0[mdl.free].sum(0).tolist(),
               thetabar_norm=float(np.linalg.norm(th)), thetabar_sum=float(th.sum()),
               tets=tets.tolist(), thetabar=th[tets].tolist(), verts=verts.tolist(), x=xs[-1][verts].tolist())
    path = os.path.join(HERE, "beam16x16x64_adjoint.json")
    json.dump(out, open(path, "w"))
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
