"""Benchmark: seconds per implicit-Euler step to relative residual 1e-5 on the
single-beam workload (16x16 cross-section, 128 long, 0.05 m cells: 37,281
vertices, 196,608 tets; stable Neo-Hookean, nu 0.45, E 1e5 and 1e8 Pa,
rho 1000, pinned at x = 0, gravity, dt 1/120, 10 steps from an initial twist
of amplitude 2 rad/s), JGS2 against plain Jacobi / Gauss-Seidel on the same
GPU, plus the sweep kernels' bandwidth against the HBM roofline.

Prints one JSON line (see the keys below).  Inputs are synthetic and seeded.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HEADLINE_MODE = "jgs2_exact_jacobi"
METRIC = "s/step to rel. residual 1e-5 (JGS2 vs Jacobi); sweep HBM GB/s; adjoint s/step"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--stiffness", default="1e5,1e8")
    ap.add_argument("--max-sweeps", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="4x4x16 beam instead (quick check)")
    ap.add_argument("--modes", default="jgs2_exact_jacobi,jgs2_exact_jacobi_drop1e-10,jgs2_exact_jacobi_keep_all,jgs2_exact_gs,"
                                       "jgs2_exact_jacobi_fp16,jgs2_damper_gs,"
                                       "jgs2_damper_jacobi_w0.8,"
                                       "jgs2_jacobi,jgs2_gs,plain_jacobi,"
                                       "plain_jacobi_w0.8,plain_jacobi_w0.5,plain_jacobi_w0.3,plain_gs,"
                                       "plain_gs_w1.5,plain_gs_w1.6")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiation leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched many-beam leg")
    ap.add_argument("--shape", default="16x64",
                    help="launch shape (lanes per vertex x block) of the single-beam plain modes; 16x64 is what "
                         "the autotuner picks on the 16x16x128 beam on MI355X")
    ap.add_argument("--tune", action="store_true", help="run the autotuner instead of using --shape")
    ap.add_argument("--jsonl", default=None,
                    help="append one JSON record per timed step of every mode to this file")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every sweep kernel eagerly instead of replaying captured sweep groups (same "
                         "kernels and arguments; used for traced runs)")
    ap.add_argument("--batched-beams", type=int, default=256)
    ap.add_argument("--batched-steps", type=int, default=4, help="steps of the batched leg (30 in its full run)")
    ap.add_argument("--batched-roofline-only", action="store_true",
                    help="batched leg: stop after the sweep kernel's roofline group (for profiling runs)")
    ap.add_argument("--contact-steps", type=int, default=120)
    ap.add_argument("--no-contact", action="store_true", help="skip the 10-sphere contact leg")
    ap.add_argument("--leg", choices=["contact"], help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (5x) to calibrate HBM byte counters")
    return ap.parse_args()


def sync():
    """Device-wide synchronisation in the library's HIP runtime (torch may
    bring a runtime of its own that does not see the library's queues)."""
    from paper_2506_06494_amd import jgs2
    jgs2.device_synchronize()


def calibrate_copy():
    """A plain copy kernel of known size: 1 GiB read + 1 GiB written per copy."""
    import torch
    n = 1 << 28  # float32 elements = 1 GiB
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 5}))


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.leg == "contact":                  # child process of the default run
        print(json.dumps(contact_leg(steps=args.contact_steps)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    # the contact leg runs first, in a child process started before this one
    # touches the GPU, so that a failure there cannot take the whole run down
    con = None if args.no_contact or args.small else contact_leg_child(args.contact_steps)
    from paper_2506_06494_amd import inputs, jgs2

    stiff = [float(e) for e in args.stiffness.split(",")]
    if args.small:
        make = lambda E: inputs.beam_scene(16, 4, 4, E=E, steps=args.steps)
        wl = "beam 4x4x16 (0.05 m cells, 425 vertices, 1,536 tets)"
    else:
        make = lambda E: inputs.single_beam(E)
        wl = "beam 16x16x128 (0.05 m cells, 37,281 vertices, 196,608 tets)"

    modes = [
        # the exact co-rotated subspace (every row of U-bar, no cubature), Jacobi and coloured GS
        # (a residual check after every sweep: a sweep streams the whole of H-bar^-1, so one
        # sweep past convergence costs more than the check)
        # (tiles of H-bar^-1 whose entries are all at most 1e-5 of its largest are skipped: they
        # change only the correction b, whose fixed point g = 0 stays the same, and on these beams
        # not the sweep count; _drop1e-10 is the library default, _keep_all streams every tile)
        ("jgs2_exact_jacobi", dict(variant=jgs2.EXACT, order=jgs2.JACOBI, omega=1.0, check_every=1,
                                   exact_drop=1e-5)),
        ("jgs2_exact_jacobi_drop1e-10", dict(variant=jgs2.EXACT, order=jgs2.JACOBI, omega=1.0, check_every=1,
                                             exact_drop=1e-10)),
        ("jgs2_exact_jacobi_keep_all", dict(variant=jgs2.EXACT, order=jgs2.JACOBI, omega=1.0, check_every=1,
                                            exact_drop=0.0)),
        ("jgs2_exact_gs", dict(variant=jgs2.EXACT, order=jgs2.GS, omega=1.0, check_every=1, exact_drop=1e-5)),
        # the headline mode with the tiles stored in FP16, scaled per tile (half the streamed bytes;
        # the conversion is one-way, so it runs after the other exact modes of the handle)
        ("jgs2_exact_jacobi_fp16", dict(variant=jgs2.EXACT, order=jgs2.JACOBI, omega=1.0, check_every=1,
                                        exact_drop=1e-5, tile_fp16=1)),
        # the damper reading of the correction in coloured GS, no step scale
        ("jgs2_damper_gs", dict(variant=jgs2.DAMPER, order=jgs2.GS, omega=1.0)),
        ("jgs2_damper_jacobi_w0.8", dict(variant=jgs2.DAMPER, order=jgs2.JACOBI, omega=0.8)),
        # reading R3 (one-ring exact, remote sampled): diverges on these beams
        ("jgs2_jacobi", dict(variant=jgs2.CUBATURE, order=jgs2.JACOBI, omega=1.0)),
        ("jgs2_gs", dict(variant=jgs2.CUBATURE, order=jgs2.GS, omega=1.0)),
        ("plain_jacobi", dict(variant=jgs2.PLAIN, order=jgs2.JACOBI, omega=1.0)),
        ("plain_jacobi_w0.8", dict(variant=jgs2.PLAIN, order=jgs2.JACOBI, omega=0.8)),
        ("plain_jacobi_w0.5", dict(variant=jgs2.PLAIN, order=jgs2.JACOBI, omega=0.5)),
        ("plain_jacobi_w0.3", dict(variant=jgs2.PLAIN, order=jgs2.JACOBI, omega=0.3)),
        ("plain_gs", dict(variant=jgs2.PLAIN, order=jgs2.GS, omega=1.0)),
        # the same coloured GS with every vertex step scaled by 1.5 and 1.6 (successive
        # over-relaxation; on the 16x16x128 beam 1.6 needs the fewest sweeps of 1.5..1.9)
        ("plain_gs_w1.5", dict(variant=jgs2.PLAIN, order=jgs2.GS, omega=1.5)),
        ("plain_gs_w1.6", dict(variant=jgs2.PLAIN, order=jgs2.GS, omega=1.6)),
        # the same with each sweep group as one persistent cooperative launch (not a default mode)
        ("plain_gs_w1.6_persistent", dict(variant=jgs2.PLAIN, order=jgs2.GS, omega=1.6, persistent=1)),
    ]
    wanted = args.modes.split(",")
    modes = [m for m in modes if m[0] in wanted]
    results = {}
    kernel_stats = {}
    precompute_s = {}
    corr0 = None
    for E in stiff:
        sc = make(E)
        m = sc.mesh
        corr = None
        exact_keep = {}      # one exact-variant handle, shared by its modes
        for name, cfg in modes:
            kw = dict(check_every=16)
            kw.update(cfg)
            persistent = kw.pop("persistent", 0)
            tile_fp16 = kw.pop("tile_fp16", 0)
            if cfg["variant"] == jgs2.EXACT and exact_keep:
                s = exact_keep["exact"]        # the same H-bar^-1 tiles; only the order and checks change
                s.set_params(**{k: v for k, v in kw.items() if k != "variant"})
            else:
                s = jgs2.Solver(dt=sc.dt, gravity=sc.gravity, rel_tol=1e-5, max_sweeps=args.max_sweeps,
                                use_graph=0 if args.no_graph else 1, **kw)
                s.upload_mesh(m.X, m.tets, m.pinned)
                s.set_material(sc.E, sc.nu, sc.rho)
            if cfg["variant"] == jgs2.EXACT and not exact_keep:
                # its own precompute: H-bar^-1 stays on the device (the same run also
                # trains the cubature tables, which the sampled modes then import)
                key = f"{E:g} exact"
                print(f"[bench] E={E:g} {name}: GPU precompute with H-bar^-1 tiles ...", file=sys.stderr, flush=True)
                t0 = time.perf_counter()
                s.precompute(samples=4, n_cand=64, seed=0)
                precompute_s[key] = time.perf_counter() - t0
                print(f"[bench] E={E:g} precompute (with tiles) {precompute_s[key]:.2f} s", file=sys.stderr, flush=True)
                exact_keep["exact"] = s
                if corr is None:
                    corr = s.export_correction(4)
                    if corr0 is None:
                        corr0 = corr
            elif cfg["variant"] == jgs2.EXACT:
                pass
            elif cfg["variant"] != jgs2.PLAIN:
                if corr is None:
                    print(f"[bench] E={E:g} GPU precompute ...", file=sys.stderr, flush=True)
                    t0 = time.perf_counter()
                    s.precompute(samples=4, n_cand=64, seed=0)
                    precompute_s[E] = time.perf_counter() - t0
                    print(f"[bench] E={E:g} precompute {precompute_s[E]:.2f} s", file=sys.stderr, flush=True)
                    corr = s.export_correction(4)
                    if corr0 is None:
                        corr0 = corr
                else:
                    s.import_correction(4, corr["U_ring"].reshape(-1, 9), corr["samples"], corr["weights"],
                                        corr["U_samp"])
            if persistent:
                s.set_persistent(True)
            if tile_fp16:
                s.exact_tiles_fp16()
            s.set_state(sc.x0, sc.v0)
            tuned = None
            if cfg["variant"] == jgs2.PLAIN:
                if args.tune:
                    tuned, _ = s.autotune(32)    # launch shape of the plain sweep kernel on this mesh
                else:
                    tuned = tuple(int(v) for v in args.shape.split("x"))
                    s.set_tuning(*tuned)
            elif cfg["variant"] == jgs2.DAMPER:
                # the damper sweep (rotation and fused damper kernels) is tuned on this mesh
                tuned, _ = s.autotune(8)
            # warm-up steps (untimed), then the timed steps
            failed = None
            stalled = None
            for _ in range(args.warmup):
                st = s.step(raise_on_error=False)
                if st["status"] < 0:
                    failed = st
                    break
                if st["status"] == jgs2.NOT_CONVERGED:
                    stalled = st           # hit the sweep cap: reported as "> max_sweeps", not timed further
                    break
            recs = []
            kt = {}
            if failed is None and stalled is None:
                # timed region: synchronise, K steps, synchronise
                sync()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    st = s.step(raise_on_error=False)
                    recs.append(st)
                    if st["status"] < 0:
                        failed = st
                        break
                sync()
                wall = time.perf_counter() - t0
                if failed is None:
                    # the same K steps again from the same start with per-kernel HIP events
                    s.set_state(sc.x0, sc.v0)
                    for _ in range(args.warmup):
                        s.step(raise_on_error=False)
                    s.set_profiling(True)
                    for _ in range(args.steps):
                        s.step(raise_on_error=False)
                    kt = s.kernel_times()
                    s.set_profiling(False)
            else:
                wall = 0.0
            if args.jsonl:
                with open(args.jsonl, "a") as fj:
                    for k, r in enumerate(recs):
                        fj.write(json.dumps(dict(mode=name, E=E, step=k, sweeps=int(r["sweeps"]),
                                                 status=jgs2.STATUS_NAMES.get(r["status"], str(r["status"])),
                                                 r0=r["r0"], r_final=r["r_final"], dx_norm=r.get("dx_norm"),
                                                 device_s=r["seconds"])) + "\n")
            ok = failed is None and stalled is None and all(r["status"] == jgs2.OK for r in recs)
            status = (jgs2.STATUS_NAMES[failed["status"]] if failed else
                      "NOT_CONVERGED" if (stalled or not ok) else "OK")
            entry = dict(status=status, converged_all=bool(ok), steps=len(recs))
            if cfg["variant"] == jgs2.EXACT:
                entry["exact_tiles"] = s.exact_tiles()
            if tuned:
                entry["launch_shape"] = list(tuned)
            if failed:
                entry["sweeps_before_failure"] = failed["sweeps"]
            if stalled:
                entry.update(not_converged=f"> {args.max_sweeps} sweeps (>= {stalled['seconds']:.3f} s) "
                                           f"in the warm-up step", r_final=stalled["r_final"])
            if recs and failed is None:
                entry.update(s_per_step=wall / len(recs),
                             device_s_per_step=float(np.mean([r["seconds"] for r in recs])),
                             sweeps_per_step=float(np.mean([r["sweeps"] for r in recs])),
                             r_final_max=float(max(r["r_final"] for r in recs)))
            results.setdefault(name, {})[f"{E:g}"] = entry
            kernel_stats.setdefault(name, {})[f"{E:g}"] = kt
            if cfg["variant"] != jgs2.EXACT:
                s.close()
            print(f"[bench] E={E:g} {name}: {json.dumps(entry)}", file=sys.stderr, flush=True)
        for s in exact_keep.values():
            s.close()
        print(f"[bench] E={E:g} done: " + ", ".join(
            f"{n}={results[n][f'{E:g}'].get('s_per_step', results[n][f'{E:g}']['status'])}" for n, _ in modes),
            file=sys.stderr, flush=True)

    # ---- headline: the JGS2 correction (exact co-rotated subspace, Jacobi) at the first
    # stiffness; a fixed mode, null with its status when it does not reach the tolerance
    E0 = f"{stiff[0]:g}"
    head_mode = HEADLINE_MODE if HEADLINE_MODE in results else None
    head = results[head_mode][E0] if head_mode else {}
    value = head.get("s_per_step") if head.get("converged_all") else None
    compare = compare_table(results, [n for n, _ in modes], stiff, head_mode)

    # ---- roofline of the dominant kernel of the headline mode
    roof = None
    sc0 = make(stiff[0])
    cnt = mesh_counts(sc0)
    probe = jgs2.Solver(dt=sc0.dt)
    probe.upload_mesh(sc0.mesh.X, sc0.mesh.tets, sc0.mesh.pinned)
    n_colors = probe.coloring()[1]
    ring_entries = int(probe.ring_sizes().sum())
    probe.close()
    kt = kernel_stats.get(head_mode, {}).get(E0) or {}
    if kt:
        dom = max(kt, key=lambda k: kt[k][0])
        ms, n = kt[dom]
        # lanes per vertex x block of the tunable sweep kernels; None for the others
        shape = results[head_mode][E0].get("launch_shape") if dom in ("plain", "damper") else None
        tag = ("beam16x16x128" if not args.small else "beam4x4x16") + "_" + head_mode
        if dom == "phase1":       # every launch gathers every free vertex
            per_launch = sweep_bytes("phase1", cnt["T"], cnt["n_inc"], cnt["Vf"], cnt["V"])
            kname = "k_phase1"
        elif dom == "phase2":     # one launch per colour: the sweep's bytes over its launches
            per_launch = sweep_bytes("phase2", cnt["T"], cnt["n_inc"], cnt["Vf"], cnt["V"],
                                     ring_entries=ring_entries) * (1 if "jacobi" in head_mode
                                                                           else 1.0 / n_colors)
            kname = "k_phase2_cubature"
        elif dom == "plain":
            nsweeps = results[head_mode][E0]["sweeps_per_step"] * results[head_mode][E0]["steps"]
            kind = "plain_gs_sweep" if "_gs" in head_mode else "plain_jacobi"
            per_launch = sweep_bytes(kind, **cnt, n_colors=n_colors) * nsweeps / n
            kname = "k_plain"
        elif dom == "damper":     # one launch per colour (GS) or per sweep (Jacobi)
            nsweeps = results[head_mode][E0]["sweeps_per_step"] * results[head_mode][E0]["steps"]
            kind = "damper_gs_sweep" if "_gs" in head_mode else "damper_jacobi"
            per_launch = sweep_bytes(kind, **cnt, n_colors=n_colors) * nsweeps / n
            kname = "k_damper"
        elif dom == "rot":
            per_launch = sweep_bytes("rot", **cnt)
            kname = "k_rot"
        elif dom == "symv":       # one launch per reduced gradient (per sweep, or per colour in GS)
            et = results[head_mode][E0]["exact_tiles"]
            per_launch = sweep_bytes("symv", **cnt, live_bytes=et["live_bytes"], part_bytes=et["part_bytes"])
            kname = "k_symv"
        elif dom == "exact":      # Jacobi: one launch over every row; GS: one per colour
            per_launch = sweep_bytes("exact", **cnt) * (1 if "jacobi" in head_mode else 1.0 / n_colors)
            kname = "k_exact"
        else:
            per_launch, kname = None, dom
        if per_launch is not None:
            achieved = per_launch / (ms * 1e-3 / n) / 1e9
            traffic = measured_traffic(kname, tag)
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else round(traffic), "kernel": kname,
                    "avg_launch_us": round(ms * 1e3 / n, 3), "launches": n,
                    "bytes_per_launch": round(per_launch), "launch_shape": shape}
    jgs2_sweep = measure_cubature_sweep(sc0, corr0) if corr0 is not None else None

    adj = None if args.no_adjoint or args.small else adjoint_leg()
    bat = None if args.no_batched or args.small else batched_leg(args.batched_beams, steps=args.batched_steps,
                                                                 roofline_only=args.batched_roofline_only)

    cpu = None
    if not args.no_cpu_baseline and value is not None:
        cpu = cpu_baseline(sc0, results[head_mode][E0]["sweeps_per_step"])

    line = {
        "metric": METRIC, "value": value, "unit": "s/step", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": None if value is None else round(value * 1e3, 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded procedural beam, random-free initial twist)",
        "config": {"workload": f"{wl}, stable Neo-Hookean nu 0.45, E {E0} Pa, pinned x=0, gravity, "
                               f"dt 1/120, twist 2 rad/s, to rel. residual 1e-5",
                   "mode": head_mode, "status": head.get("status"), "stiffness": stiff},
        "roofline": roof, "cpu_baseline": cpu,
        "headline_kernels": {k: {"avg_launch_us": round(v[0] * 1e3 / v[1], 3), "launches": v[1]}
                             for k, v in (kernel_stats.get(head_mode, {}).get(E0) or {}).items() if v[1]},
        "jgs2_vs_plain": compare,
        "modes": results, "jgs2_sweep": jgs2_sweep, "adjoint": adj, "batched": bat, "contact": con,
        "precompute_s": {(k if isinstance(k, str) else f"{k:g}"): round(v, 3) for k, v in precompute_s.items()},
    }
    print(json.dumps(line))


def compare_table(results, names, stiff, head_mode):
    """Per stiffness: every JGS2 mode's s/step (or its status), the fastest
    converged plain Jacobi and plain Gauss-Seidel modes, and the headline
    mode's time over the fastest plain Jacobi time."""
    out = {}
    for E in stiff:
        k = f"{E:g}"

        def fastest(prefix):
            c = [(n, results[n][k]["s_per_step"]) for n in names
                 if n.startswith(prefix) and results[n][k].get("converged_all")]
            return list(min(c, key=lambda t: t[1])) if c else None
        row = {n: (results[n][k]["s_per_step"] if results[n][k].get("converged_all") else results[n][k]["status"])
               for n in names if n.startswith("jgs2")}
        row["fastest_plain_jacobi"] = fastest("plain_jacobi")
        row["fastest_plain_gs"] = fastest("plain_gs")
        hv = results[head_mode][k].get("s_per_step") if (head_mode and results[head_mode][k].get("converged_all")) \
            else None
        pj = row["fastest_plain_jacobi"]
        row["headline_over_plain_jacobi"] = (hv / pj[1]) if (hv is not None and pj) else None
        out[k] = row
    return out


def batched_leg(n_beams=256, steps=4, loop_steps=2, max_sweeps=20000, check_every=8, omega=1.5, roofline_only=False):
    """Many-beam workload: n_beams beams with cross-section a, b in U{4..24},
    length in U{16..96} cells of 0.05 m, log-uniform E in [1e4, 1e7], nu in
    U[0.3, 0.48] (seed 0), pinned at x = 0, gravity, from rest; coloured GS
    (omega 1.5) with per-beam residuals and stop masks, sweep groups replayed
    from captured graphs, launch shape from the autotuner; `steps` steps, each
    until every beam reaches 1e-5 (or the sweep cap).  Compared with the same
    beams stepped one after another with their own solvers over the first
    `loop_steps` steps (the batched run's first `loop_steps` steps are timed
    separately for that comparison).  roofline_only: return after the
    roofline group (one sweep group of eager, event-timed launches after the
    autotuner; no graph is captured)."""
    from paper_2506_06494_amd import inputs, jgs2
    spec = inputs.batched_beams(n_beams, seed=0)
    meshes, E, nu = [], [], []
    for (L, a, b, Eb, nub) in spec:
        m = inputs.beam_mesh(L, a, b, 0.05)
        meshes.append(m)
        E.append(np.full(m.nT, Eb))
        nu.append(np.full(m.nT, nub))
    u = inputs.concat_meshes(meshes)
    E, nu = np.concatenate(E), np.concatenate(nu)
    kw = dict(order=jgs2.GS, omega=omega, rel_tol=1e-5, max_sweeps=max_sweeps, check_every=check_every)
    s = jgs2.Solver(use_graph=1, **kw)
    s.upload_mesh(u.X, u.tets, u.pinned)
    s.set_material(E, nu, 1000.0)
    s.set_bodies(u.body)
    s.set_state(u.X, np.zeros_like(u.X))
    (lpv, blk), tune_ms = s.autotune(8)
    print(f"[bench] batched: {u.nV} vertices, {u.nT} tets, tuned shape {lpv}x{blk}", file=sys.stderr, flush=True)
    # roofline of the sweep kernel while every beam is still iterating
    s.set_profiling(True)
    s.begin_step()
    s.iterate(check_every)
    kt = s.kernel_times()
    s.set_profiling(False)
    s.set_state(u.X, np.zeros_like(u.X))
    ms, n = kt["plain"]
    cnt = mesh_counts(u)
    probe_colors = s.coloring()[1]
    per_launch = sweep_bytes("plain_gs_sweep", **cnt, n_colors=probe_colors) / probe_colors
    roof = {"bound": "hbm", "kernel": "k_plain", "avg_launch_us": round(ms * 1e3 / n, 3), "launches": n,
            "bytes_per_launch": round(per_launch),
            "achieved": round(per_launch / (ms * 1e-3 / n) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / HBM_PEAK_GBS, 4)
    traffic = measured_traffic("k_plain", f"batch{n_beams}_gs_w{omega:g}")
    roof["traffic"] = None if traffic is None else round(traffic)
    print(f"[bench] batched roofline group: {json.dumps(roof)}", file=sys.stderr, flush=True)
    if roofline_only:
        s.close()
        return {"tuned_shape": [lpv, blk], "roofline": roof}
    stats, t_steps, conv = [], [], []
    for k in range(steps):
        sync()
        t0 = time.perf_counter()
        st = s.step(raise_on_error=False)
        sync()
        t_steps.append(time.perf_counter() - t0)
        stats.append(st)
        sw, rel = s.body_stats()
        conv.append(int(np.sum(rel <= 1e-5)))
        print(f"[bench] batched step {k}: {t_steps[-1]:.3f} s, {st['sweeps']} sweeps, {conv[-1]}/{n_beams} beams "
              f"converged, status {st['status']}", file=sys.stderr, flush=True)
        if k == loop_steps - 1:
            x_graph = s.get_state()[0]
        if st["status"] < 0:
            break
    # the same first steps with each sweep group as one persistent cooperative launch
    s.set_state(u.X, np.zeros_like(u.X))
    s.set_persistent(True)
    t_pers = []
    for k in range(loop_steps):
        sync()
        t0 = time.perf_counter()
        s.step(raise_on_error=False)
        sync()
        t_pers.append(time.perf_counter() - t0)
    pers_bitwise = bool(np.array_equal(s.get_state()[0], x_graph))
    print(f"[bench] batched persistent: {np.mean(t_pers):.3f} s/step over the first {loop_steps} steps, "
          f"bitwise equal to the graph replay: {pers_bitwise}", file=sys.stderr, flush=True)
    s.close()
    tb = float(np.mean(t_steps[:loop_steps]))
    # per-beam launch loop: the same beams, one solver each, same parameters and tuning
    solvers = []
    for m, (L, a, b, Eb, nub) in zip(meshes, spec):
        q = jgs2.Solver(**kw)
        q.upload_mesh(m.X, m.tets, m.pinned)
        q.set_material(np.full(m.nT, Eb), np.full(m.nT, nub), 1000.0)
        q.set_tuning(lpv, blk)
        q.set_state(m.X, np.zeros_like(m.X))
        solvers.append(q)
    sync()
    t0 = time.perf_counter()
    for _ in range(loop_steps):
        for q in solvers:
            q.step(raise_on_error=False)
    sync()
    tl = (time.perf_counter() - t0) / loop_steps
    for q in solvers:
        q.close()
    out = {"workload": f"{n_beams} beams (seed 0): {u.nV:,} vertices, {u.nT:,} tets, cross-section U{{4..24}}^2, "
                       f"length U{{16..96}}, E log-U[1e4,1e7], nu U[0.3,0.48], from rest, gravity",
           "steps": len(stats), "max_sweeps": max_sweeps, "omega": omega, "tuned_shape": [lpv, blk],
           "batched_s_per_step": float(np.mean(t_steps)), "batched_s_per_step_first": tb,
           "per_beam_loop_s_per_step_first": tl, "speedup_first_steps": tl / tb, "loop_steps": loop_steps,
           "persistent_s_per_step_first": float(np.mean(t_pers)), "persistent_bitwise_equal": pers_bitwise,
           "beams_converged_per_step": conv, "all_converged_every_step": all(c == n_beams for c in conv),
           "sweeps_per_step": [st["sweeps"] for st in stats], "status": [st["status"] for st in stats],
           "roofline": roof}
    print(f"[bench] batched: {json.dumps(out)}", file=sys.stderr, flush=True)
    return out


def contact_leg_child(steps=120, timeout_s=900):
    import subprocess
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--leg", "contact", "--contact-steps",
                            str(steps)], capture_output=True,
                           text=True, timeout=timeout_s)
    except subprocess.TimeoutExpired:
        return {"error": f"contact leg exceeded {timeout_s} s"}
    sys.stderr.write(r.stderr)
    sys.stderr.flush()
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"contact leg exited with status {r.returncode}"}
    return json.loads(lines[-1])


def contact_leg(steps=120, max_sweeps=400, check_every=16):
    """Contact workload as configured: the 10 voxelised spheres of radius
    0.3 m (0.01 m grid, 1,217,690 vertices, 6,786,240 tets; five with E 2e6,
    five with E 1e5, nu 0.45) at rest at their seeded centres in the 2 x 2 x 4 m
    box, dropped under gravity (-z) for 120 steps of 1/120 s; floor and four
    walls as IPC plane barriers (d_hat 1e-3 m, kappa 1e4); plain coloured GS
    with the per-vertex feasibility clamp and per-sphere residuals, at most
    `max_sweeps` sweeps per step (a step that stops there is reported as not
    converged).  steps = 0: only the sweep kernel's roofline group (eager,
    event-timed launches after the autotuner; no graph is captured), for
    profiling runs."""
    from paper_2506_06494_amd import inputs, jgs2
    sc = inputs.contact_scene(0)
    m = sc.mesh
    X = m.X.copy()
    v0 = np.zeros_like(X)
    s = jgs2.Solver(dt=sc.dt, gravity=sc.gravity, planes=sc.planes, d_hat=sc.d_hat, kappa=sc.kappa, order=jgs2.GS,
                    omega=1.0, rel_tol=1e-5, max_sweeps=max_sweeps, check_every=check_every, use_graph=1)
    s.upload_mesh(X, m.tets, m.pinned)
    s.set_material(sc.E, sc.nu, sc.rho)
    s.set_bodies(m.body)
    s.set_state(X, v0)
    (lpv, blk), _ = s.autotune(8)
    s.set_profiling(True)
    s.begin_step()
    s.iterate(check_every)
    kt = s.kernel_times()
    s.set_profiling(False)
    ms, n = kt["plain"]
    cnt = mesh_counts(m)
    ncol = s.coloring()[1]
    per_launch = sweep_bytes("plain_gs_sweep", **cnt, n_colors=ncol) / ncol
    roof = {"bound": "hbm", "kernel": "k_plain", "avg_launch_us": round(ms * 1e3 / n, 3), "launches": n,
            "bytes_per_launch": round(per_launch), "achieved": round(per_launch / (ms * 1e-3 / n) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / HBM_PEAK_GBS, 4)
    traffic = measured_traffic("k_plain", "contact10_gs")
    roof["traffic"] = None if traffic is None else round(traffic)
    if steps == 0:
        s.close()
        return {"colours": int(ncol), "tuned_shape": [lpv, blk], "roofline": roof}
    s.set_state(X, v0)
    zmin, stats = [], []
    sync()
    t0 = time.perf_counter()
    for k in range(steps):
        st = s.step(raise_on_error=False)
        stats.append(st)
        if st["status"] < 0:
            break
        if k % 10 == 9 or k == steps - 1:
            x, _ = s.get_state()
            zmin.append(float(x[:, 2].min()))
            print(f"[bench] contact step {k + 1}: {st['sweeps']} sweeps, r {st['r_final']:.2e}, status "
                  f"{st['status']}, lowest vertex z {zmin[-1]:.5f} m", file=sys.stderr, flush=True)
    sync()
    tc = (time.perf_counter() - t0) / len(stats)
    s.close()
    sw = [st["sweeps"] for st in stats]
    status = [st["status"] for st in stats]
    out = {"workload": f"10 spheres r 0.3 m (0.01 m grid): {m.nV:,} vertices, {m.nT:,} tets, at rest at seeded centres "
                       "in the 2 x 2 x 4 m box, dropped; planes z=0, x=0,2, y=0,2, d_hat 1e-3, kappa 1e4",
           "steps": len(stats), "max_sweeps": max_sweeps, "s_per_step": tc,
           "steps_converged": int(sum(1 for v in status if v == jgs2.OK)),
           "steps_at_sweep_cap": int(sum(1 for v in status if v == jgs2.NOT_CONVERGED)),
           "failed": [v for v in status if v < 0], "sweeps_per_step_mean": float(np.mean(sw)),
           "sweeps_per_step": sw, "r_final_max": float(max(st["r_final"] for st in stats)),
           "lowest_vertex_z_every_10_steps": zmin, "colours": int(ncol), "tuned_shape": [lpv, blk],
           "roofline": roof}
    print(f"[bench] contact: {json.dumps({k: v for k, v in out.items() if k != 'sweeps_per_step'})}",
          file=sys.stderr, flush=True)
    return out


def adjoint_leg(n_steps=30, ckpt_every=5):
    """Differentiation workload: 16x16x64 beam (18,785 vertices, 98,304
    tets), per-tet log E = log 1e6 + U(-0.3, 0.3), u = 0, 30 steps to 1e-5,
    loss |tip centroid - target|^2; forward rollout with checkpoints every 5
    steps, then the adjoint (recompute + linear sweeps to 1e-5 + stiffness
    gradient), both timed with a synchronised wall clock.  Run with the exact
    co-rotated subspace in Jacobi order (forward steps and the adjoint's
    linear sweeps; tiles at most 1e-5 of H-bar^-1's largest entry skipped,
    as in the headline mode), and with plain coloured GS at step scale 1.7
    for comparison."""
    from paper_2506_06494_amd import inputs, jgs2
    sc, logE, target = inputs.diff_beam(0)
    m = sc.mesh
    tip = np.nonzero(m.X[:, 0] >= m.X[:, 0].max() - 1e-12)[0]
    legs = {}
    for name, cfg in (("jgs2_exact_jacobi", dict(variant=jgs2.EXACT, order=jgs2.JACOBI, omega=1.0, check_every=1,
                                                 exact_drop=1e-5)),
                      ("plain_gs_w1.7", dict(variant=jgs2.PLAIN, order=jgs2.GS, omega=1.7, check_every=16))):
        s = jgs2.Solver(dt=sc.dt, gravity=sc.gravity, rel_tol=1e-5, adj_rel_tol=1e-5, use_graph=1, **cfg)
        s.upload_mesh(m.X, m.tets, m.pinned)
        s.set_material(np.exp(logE), 0.45, 1000.0)
        if cfg["variant"] == jgs2.EXACT:
            t0 = time.perf_counter()
            s.precompute(samples=4, n_cand=64, seed=0)
            pre = time.perf_counter() - t0
        out = {}
        for rep in range(2):                       # the first pass warms up
            s.set_state(m.X, np.zeros_like(m.X))
            sync()
            t0 = time.perf_counter()
            fst = s.rollout(n_steps, ckpt_every)
            sync()
            tf = time.perf_counter() - t0
            x, _ = s.get_state()
            r = x[tip].mean(0) - target
            xbar = np.zeros_like(x)
            xbar[tip] = 2.0 * r / tip.size
            sync()
            t0 = time.perf_counter()
            th, _, vb0, st = s.rollout_backward(xbar)
            sync()
            tb = time.perf_counter() - t0
            out = {"mode": name, "forward_status": jgs2.STATUS_NAMES.get(fst["status"], fst["status"]),
                   "adjoint_status": jgs2.STATUS_NAMES.get(st["status"], st["status"]),
                   "loss": float(r @ r), "forward_s_per_step": tf / n_steps, "adjoint_s_per_step": tb / n_steps,
                   "ratio": tb / tf, "adjoint_sweeps_per_step": st["adjoint_sweeps"] / n_steps,
                   "recompute_sweeps_per_step": st["forward_sweeps"] / n_steps,
                   "max_adjoint_rel_res": st["max_rel_res"], "thetabar_norm": float(np.linalg.norm(th)),
                   "ubar": st["ubar"].tolist()}
            if cfg["variant"] == jgs2.EXACT:
                out["precompute_s"] = pre
            print(f"[bench] adjoint {name} pass {rep}: {json.dumps(out)}", file=sys.stderr, flush=True)
        s.close()
        legs[name] = out
    return {"workload": "beam 16x16x64 (18,785 vertices, 98,304 tets), log E = log 1e6 + U(-0.3,0.3), 30 steps, "
                        "checkpoints every 5, forward and adjoint to 1e-5", "modes": legs}


def kernel_source_sha1():
    import hashlib
    path = os.path.join(ROOT, "paper_2506_06494_amd", "csrc", "sweep.hip")
    return hashlib.sha1(open(path, "rb").read()).hexdigest()


def measured_traffic(kernel, workload_tag, shape=None):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    counter reads for a 1 GiB copy), or None if that summary is missing, was
    taken on different kernel source or (when both name one) in another
    launch shape."""
    import re
    path = os.path.join(ROOT, "profiles", "pmc_traffic.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if not line.startswith("traffic "):
            continue
        kv = dict(re.findall(r"(\w+)=(\S+)", line))
        if kv.get("kernel") != kernel or kv.get("workload") != workload_tag:
            continue
        if kv.get("sweep_sha1") != kernel_source_sha1():
            return None
        if shape is not None and "shape" in kv and kv["shape"] != "x".join(str(v) for v in shape):
            return None
        return (float(kv["fetch_kib"]) * 1024 * float(kv["fetch_scale"]) +
                float(kv["write_kib"]) * 1024 * float(kv["write_scale"]))
    return None


def sweep_bytes(kind, T, n_inc, Vf, V, ring_entries=0, S=4, n_colors=1, launches=1, live_bytes=None,
                part_bytes=None):
    """Compulsory (algorithmic) bytes moved by one launch of a sweep kernel,
    counting every datum it must touch once: tet records 80 B (64 B without
    the id word), incidence entries 4 B or 16 B with corner ids (plus 4 B
    slot words in phase 2), 64 B incidence records of the plain sweeps,
    one-ring ids + U-bar rows 40 B per entry, 168 B per cubature sample, 32 B
    FP64 displacement and inertial-target records, 16 B gradient and rotation
    records."""
    if kind == "phase1":      # positions; z read, g and R written per free vertex
        return 64.0 * T + 16.0 * n_inc + 64.0 * Vf + 32.0 * V
    if kind == "phase2":      # positions, g, R of every vertex; own record, samples, update
        return 80.0 * T + 8.0 * n_inc + 40.0 * ring_entries + Vf * (40.0 + 168.0 * S) + 64.0 * V
    if kind == "plain_jacobi":  # one 64 B incidence record per (free vertex, incident tet)
        return 64.0 * n_inc + 64.0 * Vf + 32.0 * V
    if kind == "plain_gs_sweep":  # all colour launches of one sweep; positions read once per colour
        return 64.0 * n_inc + 64.0 * Vf + 32.0 * V * n_colors
    if kind == "symv":        # the live tiles of H-bar^-1 (every stored tile unless live_bytes is given;
        q, g = 64, 8          # rows past Vf not read), 1 KB partials written: one per tile row and one
        nt = (Vf + q - 1) // q  # per tile column of each 8 x 8 super-tile (launched ones: part_bytes)
        ns = (nt + g - 1) // g
        rows = sum(min(q, Vf - i * q) * (i + 1) for i in range(nt))
        valid = [min(g, nt - g * k) for k in range(ns)]
        parts = sum(valid[si] + valid[sj] for si in range(ns) for sj in range(si + 1))
        tiles = 36.0 * q * rows if live_bytes is None else live_bytes
        return tiles + (1024.0 * parts if part_bytes is None else part_bytes) + 16.0 * Vf
    if kind == "exact":       # incident tets, positions, y and B^-1 per row, rotations, result
        return 96.0 * n_inc + (16.0 + 36.0 + 16.0) * Vf + 64.0 * V
    if kind == "rot":         # records and positions; row id and count read, rotation written
        return 64.0 * n_inc + 24.0 * Vf + 32.0 * V
    if kind == "damper_gs_sweep":  # plain terms + per sample 168 B record + 80 B tet; rotations per colour
        return 64.0 * n_inc + 64.0 * Vf + 248.0 * S * Vf + (32.0 + 16.0) * V * n_colors
    if kind == "damper_jacobi":
        return 64.0 * n_inc + 64.0 * Vf + 248.0 * S * Vf + (32.0 + 16.0) * V
    raise ValueError(kind)


def mesh_counts(sc):
    m = getattr(sc, "mesh", sc)
    free = ~m.pinned.astype(bool)
    inc = np.bincount(m.tets.ravel(), minlength=m.nV)
    return dict(T=m.nT, n_inc=float(inc[free].sum()), Vf=int(free.sum()), V=m.nV)


def measure_cubature_sweep(sc, corr, sweeps=64):
    """Average device time of the two JGS2 sweep kernels over a fixed number
    of Jacobi sweeps (HIP events), with their algorithmic bytes.  A small step
    scale (1e-3) keeps the iterate finite so the timing is that of ordinary
    arithmetic."""
    from paper_2506_06494_amd import jgs2
    m = sc.mesh
    s = jgs2.Solver(dt=sc.dt, gravity=sc.gravity, variant=jgs2.CUBATURE, order=jgs2.JACOBI, omega=1e-3)
    s.upload_mesh(m.X, m.tets, m.pinned)
    s.set_material(sc.E, sc.nu, sc.rho)
    s.import_correction(4, corr["U_ring"].reshape(-1, 9), corr["samples"], corr["weights"], corr["U_samp"])
    ring_entries = int(s.ring_sizes().sum())
    s.set_state(sc.x0, sc.v0)
    s.begin_step()
    s.iterate(4, raise_on_error=False)
    s.set_profiling(True)
    s.iterate(sweeps, raise_on_error=False)
    kt = s.kernel_times()
    s.close()
    c = mesh_counts(sc)
    out = {}
    for k in ("phase1", "phase2"):
        ms, n = kt[k]
        b = sweep_bytes(k, c["T"], c["n_inc"], c["Vf"], c["V"], ring_entries=ring_entries)
        us = ms * 1e3 / max(n, 1)
        out[k] = dict(avg_launch_us=round(us, 3), launches=n, bytes_per_launch=b,
                      achieved_GBs=round(b / (us * 1e-6) / 1e9, 1))
    t_sweep = sum(out[k]["avg_launch_us"] for k in out)
    out["sweep_us"] = round(t_sweep, 3)
    out["sweep_GBs"] = round((out["phase1"]["bytes_per_launch"] + out["phase2"]["bytes_per_launch"]) /
                             (t_sweep * 1e-6) / 1e9, 1)
    return out


def cpu_baseline(sc, sweeps_per_step, n_rows=192, seed=0):
    """The oracle's exact-subspace Jacobi sweep (variant RX, the headline
    mode), timed on one host core on a bounded sample: the gradient, the
    per-vertex rotations and the sparse Hessian of the whole mesh at the
    iterate (once per sweep), then the local systems (H row block times the
    co-rotated U-bar rows, reduced gradient over every free vertex) and
    solves of `n_rows` rows, scaled to every free row and to the GPU run's
    sweeps per step.  The U-bar rows are seeded stand-ins of the right shape:
    the sweep's cost depends on their shape only, and the oracle's own rows
    for this beam (three band solves per vertex, 2 x 49 GB in FP64) are
    precompute, far beyond a bounded sample."""
    from threadpoolctl import threadpool_limits
    from oracle import fem, sweep as osw
    mdl = fem.model_from_scene(sc)
    rng = np.random.default_rng(seed)
    rows = np.sort(rng.choice(mdl.free_ids, n_rows, replace=False))
    U = 0.01 * rng.standard_normal((n_rows, mdl.nV, 3, 3))
    z = mdl.inertial_target(sc.x0, sc.v0)
    x = sc.x0.copy()
    with threadpool_limits(1):
        t0 = time.perf_counter()
        g, R = osw.phase1(mdl, x, z)
        H = mdl.hessian(x)
        t_mesh = time.perf_counter() - t0
        t0 = time.perf_counter()
        A, b = osw.literal_exact_systems(mdl, osw.corotated_rows(U, R, rows), g, H, rows)
        osw.local_solve(A, b)
        t_rows = time.perf_counter() - t0
    per_sweep = t_mesh + t_rows / n_rows * mdl.free_ids.size
    return {"value": round(per_sweep * sweeps_per_step, 3), "unit": "s/step", "cores": 1, "kind": "oracle",
            "sample": f"oracle RX Jacobi sweep on {sc.mesh.name}: whole-mesh gradient, rotations and Hessian "
                      f"({t_mesh:.2f} s) + {n_rows} sampled rows ({t_rows:.2f} s, stand-in U-bar rows of the same "
                      f"shape), scaled to {mdl.free_ids.size} rows ({per_sweep:.1f} s per sweep) x "
                      f"{sweeps_per_step:.1f} GPU sweeps/step (extrapolated)"}


if __name__ == "__main__":
    main()
