"""The index-checked build (libjgs2_bounds.so, JGS2_BOUNDS_CHECK): every
index a sweep kernel reads from a table stays inside its buffer over the
exact, plain, damper, batched and adjoint paths (tests/bounds_driver.py, in
a process of its own), the reporting path records and clears a failure, and
the production library refuses the bounds calls."""
import json
import os
import subprocess
import sys

import pytest

from paper_2506_06494_amd import inputs, jgs2

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(300)
def test_sweep_indices_stay_in_bounds():
    if not os.path.exists(jgs2.BOUNDS_LIB_PATH):
        pytest.fail("libjgs2_bounds.so is not built (paper_2506_06494_amd.build --bounds)")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "bounds_driver.py")],
                       capture_output=True, text=True, timeout=280)
    print(r.stderr[-3000:])
    assert r.returncode == 0
    out = json.loads(r.stdout.strip().splitlines()[-1])
    t = out.pop("tiles")
    assert 0 < t["n_live"] < t["n_tiles"]          # the dead-tile paths ran
    line, idx, ext = out.pop("selftest")
    assert line > 0 and idx == 1 and ext == 0
    assert out.pop("after_clear") == [0, 0, 0]
    for name, rec in out.items():
        assert rec["line"] == 0, (name, rec)
        assert all(st in (jgs2.OK, jgs2.NOT_CONVERGED) for st in rec["status"]), (name, rec)


def test_production_build_has_no_bounds_record():
    sc = inputs.tiny_beam()
    s = jgs2.Solver(dt=sc.dt)
    with pytest.raises(jgs2.JGS2Error):
        s.bounds_report()
    with pytest.raises(jgs2.JGS2Error):
        s.bounds_selftest()
    s.close()
