"""Host-side logic without a GPU: the C-ABI structs as the compiler lays them
out against their ctypes mirror, the seeded input generators (counts,
numbering, orientation, reproducibility), parameter marshalling, and the
benchmark's byte accounting and counter-summary parser."""
import ctypes as C
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2506_06494_amd import inputs, jgs2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def c_layout(tmp_path):
    """sizeof and field offsets of the ABI structs, compiled from the header by gcc."""
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "jgs2.h"
#define F(T, f) printf(#T " " #f " %zu\\n", offsetof(T, f))
int main(void) {
    printf("jgs2_params size %zu\\n", sizeof(jgs2_params));
    F(jgs2_params, dt); F(jgs2_params, gravity); F(jgs2_params, variant); F(jgs2_params, order);
    F(jgs2_params, omega); F(jgs2_params, rel_tol); F(jgs2_params, max_sweeps); F(jgs2_params, check_every);
    F(jgs2_params, d_hat); F(jgs2_params, kappa); F(jgs2_params, n_planes); F(jgs2_params, line_search);
    F(jgs2_params, planes); F(jgs2_params, adj_rel_tol); F(jgs2_params, adj_max_sweeps); F(jgs2_params, use_graph);
    F(jgs2_params, exact_drop);
    printf("jgs2_step_stats size %zu\\n", sizeof(jgs2_step_stats));
    F(jgs2_step_stats, sweeps); F(jgs2_step_stats, status); F(jgs2_step_stats, r0); F(jgs2_step_stats, r_final);
    F(jgs2_step_stats, seconds); F(jgs2_step_stats, ls_halvings); F(jgs2_step_stats, dx_norm);
    printf("jgs2_adjoint_stats size %zu\\n", sizeof(jgs2_adjoint_stats));
    F(jgs2_adjoint_stats, steps); F(jgs2_adjoint_stats, status); F(jgs2_adjoint_stats, adjoint_sweeps);
    F(jgs2_adjoint_stats, forward_sweeps); F(jgs2_adjoint_stats, max_rel_res); F(jgs2_adjoint_stats, seconds);
    return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = {}
    for line in subprocess.check_output([str(exe)]).decode().splitlines():
        a, b, v = line.split()
        out[(a, b)] = int(v)
    return out


def test_abi_structs_match_their_ctypes_mirror(tmp_path):
    lay = c_layout(tmp_path)
    for name, cls in (("jgs2_params", jgs2.Params), ("jgs2_step_stats", jgs2.StepStats),
                      ("jgs2_adjoint_stats", jgs2.AdjointStats)):
        assert lay[(name, "size")] == C.sizeof(cls), name
        for fname, _ in cls._fields_:
            if (name, fname) in lay:
                assert lay[(name, fname)] == getattr(cls, fname).offset, (name, fname)


def test_make_params_marshalling():
    p = jgs2.make_params(dt=0.01, gravity=(0, 0, -9.8), omega=1.5, planes=[[0, 0, 1, 0], [1, 0, 0, 0.5]],
                         use_graph=1)
    assert p.dt == 0.01 and p.gravity[2] == -9.8 and p.omega == 1.5 and p.use_graph == 1
    assert p.n_planes == 2 and p.planes[1][0] == 1.0 and p.planes[1][3] == 0.5
    assert p.adj_rel_tol == 1e-5 and p.adj_max_sweeps == 20000 and p.max_sweeps == 20000


def test_splitmix64_published_outputs():
    g = inputs.SplitMix64(0)
    assert [g.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_beam_counts_numbering_and_orientation():
    m = inputs.beam_mesh(16, 4, 4, 0.05)
    assert (m.nV, m.nT, int(m.pinned.sum())) == (425, 1536, 25)
    big = inputs.beam_mesh(128, 16, 16, 0.05)
    assert (big.nV, big.nT, int(big.pinned.sum())) == (37281, 196608, 289)
    # vertex (ix, iy, iz) -> iz + (nb+1)(iy + (na+1) ix): long axis slowest
    ix, iy, iz = 3, 2, 1
    v = iz + 5 * (iy + 5 * ix)
    np.testing.assert_allclose(m.X[v], [0.05 * ix, 0.05 * iy, 0.05 * iz])
    Xe = m.X[m.tets]
    D = np.stack([Xe[:, 1] - Xe[:, 0], Xe[:, 2] - Xe[:, 0], Xe[:, 3] - Xe[:, 0]], axis=-1)
    vol = np.linalg.det(D) / 6
    assert np.all(vol > 0)
    np.testing.assert_allclose(vol.sum(), 0.8 * 0.2 * 0.2, rtol=1e-12)


def test_sphere_counts():
    m = inputs.sphere_mesh(0.3, 0.01)
    assert (m.nV, m.nT) == (121769, 678624)


def test_generators_are_reproducible():
    a = inputs.batched_beams(256, seed=0)
    b = inputs.batched_beams(256, seed=0)
    assert a == b
    for (L, na, nb, E, nu) in a:
        assert 16 <= L <= 96 and 4 <= na <= 24 and 4 <= nb <= 24
        assert 1e4 <= E <= 1e7 and 0.3 <= nu <= 0.48
    V = sum((L + 1) * (na + 1) * (nb + 1) for (L, na, nb, _, _) in a)
    T = sum(6 * L * na * nb for (L, na, nb, _, _) in a)
    assert (V, T) == (3119202, 15948108)
    s1, le1, t1 = inputs.diff_beam(0)
    s2, le2, t2 = inputs.diff_beam(0)
    assert np.array_equal(le1, le2) and np.array_equal(t1, t2)
    assert (s1.mesh.nV, s1.mesh.nT) == (18785, 98304)
    assert np.all(np.abs(le1 - np.log(1e6)) <= 0.3)


def test_bench_byte_accounting_and_traffic_parser(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    m = inputs.beam_mesh(16, 4, 4, 0.05)
    cnt = bench.mesh_counts(m)
    assert cnt["Vf"] == 400 and cnt["T"] == 1536
    # every incidence of a free vertex, summed over the free vertices
    assert cnt["n_inc"] == np.bincount(m.tets.ravel(), minlength=m.nV)[~m.pinned.astype(bool)].sum()
    gs = bench.sweep_bytes("plain_gs_sweep", **cnt, n_colors=8)
    assert gs == 64 * cnt["n_inc"] + 64 * 400 + 32 * 425 * 8
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "pmc_traffic.md").write_text(
        "x\ntraffic kernel=k_plain workload=w fetch_kib=10 write_kib=2 fetch_scale=2.0 write_scale=1.0 "
        f"shape=16x64 sweep_sha1={bench.kernel_source_sha1()}\n"
        "traffic kernel=k_plain workload=old fetch_kib=10 write_kib=2 fetch_scale=2.0 write_scale=1.0 "
        "sweep_sha1=0000\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha1", lambda: open(prof / "pmc_traffic.md").read().split("sweep_sha1=")[1].split()[0])
    assert bench.measured_traffic("k_plain", "w") == (10 * 2.0 + 2 * 1.0) * 1024
    assert bench.measured_traffic("k_plain", "w", [16, 64]) == (10 * 2.0 + 2 * 1.0) * 1024
    assert bench.measured_traffic("k_plain", "w", [32, 256]) is None   # counters taken in another launch shape
    assert bench.measured_traffic("k_plain", "old") is None      # counters taken on other kernel source
    assert bench.measured_traffic("k_phase1", "w") is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
