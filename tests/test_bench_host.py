"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the ESS block
(a rate only for chains that have mixed), the posterior-agreement distances
in Monte Carlo standard errors, and the host thread count of the CPU
baseline.  None of this touches a GPU or the library."""
import importlib.util
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_normal_quantile(bench):
    assert abs(bench._norm_ppf(0.975) - 1.959963984540054) < 1e-12
    # the family-wise bound the stationary block reports for 12 comparisons
    assert abs(bench._norm_ppf(1.0 - 0.025 / 12) - 2.865) < 1e-3


def test_ess_rate_only_for_mixed_chains(bench):
    rng = np.random.default_rng(11)
    iid = rng.standard_normal((200, 16, 4))
    good = bench.ess_block(iid, wall=10.0)
    assert good["max_rhat"] < 1.05
    assert good["ess_per_sec"] == pytest.approx(good["min_bulk_ess"] / 10.0)
    assert "ess_note" not in good
    # chains stuck around different values: split-R-hat far above 1.05
    stuck = iid + 3.0 * rng.standard_normal((1, 16, 1))
    bad = bench.ess_block(stuck, wall=10.0)
    assert bad["max_rhat"] > 1.05
    assert bad["ess_per_sec"] is None
    assert bad["ess_per_sec_raw"] == pytest.approx(bad["min_bulk_ess"] / 10.0)
    assert "R-hat" in bad["ess_note"]


def test_agreement_separates_equal_and_shifted_posteriors(bench):
    rng = np.random.default_rng(5)
    names = ["a", "b", "ln_gamma", "ln_d"]
    a = rng.standard_normal((400, 32, 4))
    b = rng.standard_normal((400, 32, 4))
    rows, worst = bench.agreement(a, b, names)
    assert set(rows) == set(names)
    # 12 distances of independent exact samplers: each about |N(0, 1)|
    assert worst < bench._norm_ppf(1.0 - 0.025 / 12) + 1.0
    for r in rows.values():
        assert abs(r["mean_a"]) < 0.05 and abs(r["q975_a"] - 1.96) < 0.1
    shifted = b + 0.3
    _, worst_s = bench.agreement(a, shifted, names)
    assert worst_s > 10.0


def test_cpu_threads_follow_the_openmp_share(bench, monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    h = bench.host_cpus()
    assert h["omp_num_threads"] == 3
    assert bench.cpu_threads() == min(3, h["allowed"])
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert 1 <= bench.cpu_threads() <= max(1, h["allowed"])
    assert math.isfinite(bench.MEASURED_TRAFFIC["k_solve_resident<128,16,float>"])
