"""Host logic of bench.py (no GPU): the solution-error measures and the
time-to-target-error search against a fake solver, the reading of the stored
oracle samples, and the refusal of more than one GPU."""
import os
import subprocess
import sys
import types

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_solution_errors_scale_and_reference():
    xstar = np.array([1.0, -4.0, 2.0, 0.5])
    samples = {"idx": np.array([0, 2]), "val": xstar[[0, 2]], "meta": {"xstar_max_abs": 4.0}}
    x = torch.tensor(xstar + np.array([1e-3, 0.0, -2e-3, 0.0]))
    e = bench.solution_errors(x, samples, torch.tensor(xstar))
    assert e["err_vs_oracle_sampled"] == pytest.approx(2e-3 / 4.0)
    assert e["err_vs_ref_max"] == pytest.approx(2e-3 / 4.0)
    assert bench.solution_errors(x, None, None) == {}


def test_time_to_error_stops_at_first_rtol_meeting_the_target(monkeypatch):
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    xstar = torch.linspace(-1.0, 1.0, 50, dtype=torch.float64)
    calls = []

    def solve(mh, ph, b, x, o):
        calls.append(o["rtol"])
        x.copy_(xstar + 30.0 * o["rtol"])  # error proportional to the tolerance
        return {"iters": int(-np.log10(o["rtol"])), "relres_true": o["rtol"]}

    fake = types.SimpleNamespace(solve_opts=lambda **kw: kw, sem_pcg_solve=solve)
    m = types.SimpleNamespace(h=1)
    x = torch.empty_like(xstar)
    out = bench.time_to_error(fake, m, None, None, x, None, xstar, (1e-8, 1e-9, 1e-10, 1e-11))
    # errors 3e-7, 3e-8, 3e-9: the third rtol is the first within 1e-8, and the search stops there
    assert calls == [1e-8, 1e-9, 1e-10]
    assert out["to_target"]["rtol"] == 1e-10 and out["to_target"]["error"] == pytest.approx(3e-9)
    assert [r["rtol"] for r in out["runs"]] == calls
    # no tolerance good enough: no target time
    calls.clear()
    out = bench.time_to_error(fake, m, None, None, x, None, xstar, (1e-8, 1e-9))
    assert out["to_target"] is None and len(out["runs"]) == 2


def test_stored_oracle_samples_are_read():
    s = bench.load_xstar_samples(48)
    assert s is not None
    assert len(s["idx"]) == len(s["val"]) == 2000
    assert s["meta"]["xstar_max_abs"] >= np.max(np.abs(s["val"]))
    assert bench.load_xstar_samples(47) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
