"""Convergence study of the correction readings (oracle, test infrastructure).

Prints, as a markdown table, the spectral radius of the linearised sweep
at the rest state for every reading built in ``linear_analysis``, on the
4x4x16 beam (nu = 0.4) and on the quarter-scale 4x4x32 beam (nu = 0.45) at
two stiffnesses each.  Run:  python -m oracle.readings_report
"""
import sys
import time

import numpy as np

from paper_2506_06494_amd import inputs

from . import correction as ocorr
from . import fem
from . import linear_analysis as la

CASES = [
    ("4x4x16 nu=0.4", (16, 4, 4, 0.4), (1e5, 1e6)),
    ("4x4x32 nu=0.45", (32, 4, 4, 0.45), (1e5, 1e8)),
]


def model_for(dims, E):
    nl, na, nb, nu = dims
    if (nl, na, nb) == (16, 4, 4):
        sc = inputs.tiny_beam(E=E, nu=nu)
    else:
        sc = inputs.beam_scene(nl, na, nb, E=E, nu=nu)
    return fem.model_from_scene(sc), sc


def row(rs, name, A, C, fit=None):
    P = rs.preconditioner(A, C)
    mu = np.linalg.eigvals(P @ rs.H)
    rj = float(np.max(np.abs(1.0 - mu)))
    om = np.linspace(0.02, 2.0, 199)
    rb = np.array([np.max(np.abs(1.0 - w * mu)) for w in om])
    j = int(np.argmin(rb))
    rg = la.spectral_radius(rs.gs_operator(A, C))
    fit_s = "" if fit is None else f"{fit:.3f}"
    return (f"| {name} | {fit_s} | {rj:.4g} | {mu.real.min():.3g} | {rb[j]:.5f} (w={om[j]:.2f}) "
            f"| {rg:.5g} | {la.sweeps_to(rg):.0f} |")


def main(out=sys.stdout):
    print("| reading | median fit residual | Jacobi rho (w=1) | min Re eig(PH) | best damped Jacobi rho "
          "| GS rho | GS sweeps to 1e-5 |", file=out)
    print("|---|---|---|---|---|---|---|", file=out)
    for label, dims, Es in CASES:
        for E in Es:
            t0 = time.time()
            mdl, sc = model_for(dims, E)
            rs = la.RestSystem(mdl)
            print(f"| **{label}, E={E:g}** (N={rs.n}) | | | | | | |", file=out)
            print(row(rs, "P0 plain vertex Newton", *rs.plain()), file=out)
            print(row(rs, "R1 exact co-rotated subspace", *rs.exact()), file=out)
            for S in (4, 8, 16):
                tab = ocorr.precompute(mdl, S=S, n_cand=64, seed=0, keep_full=False)
                fit = float(np.median(tab.fit_res))
                print(row(rs, f"R3, greedy NNLS, S={S}", *rs.cubature(tab.samples, tab.weights, "R3"), fit), file=out)
                if S == 4:
                    print(row(rs, "R2 literal (H_ii + sampled / g_i + sampled)",
                              *rs.cubature(tab.samples, tab.weights, "R2"), fit), file=out)
                    print(row(rs, "R2D damper (H_ii + sampled / g_i)",
                              *rs.cubature(tab.samples, tab.weights, "R2D"), fit), file=out)
            for s in (4, 16, 64, 256, None):
                print(row(rs, f"R3, uniform Monte Carlo, S={'all' if s is None else s}", *rs.monte_carlo(s)),
                      file=out)
            for k in (1, 2, 4, 8):
                print(row(rs, f"U-bar truncated to {k}-ring (Galerkin)", *rs.truncated(k)), file=out)
            for k in (1, 2, 3, None):
                r = la.spectral_radius(rs.group_gs_operator(k))
                name = "colour-group subspace, exact" if k is None else f"colour-group subspace, {k}-ring"
                print(f"| {name} | | | | | {r:.5g} | {la.sweeps_to(r):.0f} |", file=out)
            # the sampled remote gradient scaled by beta between the damper (beta = 0)
            # and the literal form (beta = 1)
            tab = ocorr.precompute(mdl, S=4, n_cand=64, seed=0, keep_full=False)
            A0, C0 = rs.plain()
            A2, C2 = rs.cubature(tab.samples, tab.weights, "R2")
            for beta in (0.02, 0.05, 0.1, 0.2, 0.5):
                print(row(rs, f"R2 with the sampled gradient scaled by {beta}", A2, C0 + beta * (C2 - C0)),
                      file=out)
            # coloured GS with a step scale (over-relaxation), plain against the damper
            Ad, Cd = rs.cubature(tab.samples, tab.weights, "R2D")
            for om in (1.3, 1.5, 1.6, 1.7, 1.8):
                rp = la.spectral_radius(rs.gs_operator(A0, C0, omega=om))
                rd = la.spectral_radius(rs.gs_operator(Ad, Cd, omega=om))
                print(f"| GS step scale {om}: P0 / R2D | | | | | {rp:.5g} / {rd:.5g} "
                      f"| {la.sweeps_to(rp):.0f} / {la.sweeps_to(rd):.0f} |", file=out)
            out.flush()
            print(f"[{label} E={E:g}: {time.time() - t0:.0f} s]", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
