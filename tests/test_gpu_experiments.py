"""The harness of the paper's dense studies (bench.py --experiment, Sec.
4.1.1-4.1.3) on small configurations: one JSON record per configuration and
mode, each converged to the 1e-10 residual with the solution of the
generator (x_true), iteration counts in quarters."""

import argparse
import json

import pytest

pytestmark = pytest.mark.gpu


def test_experiment_harness_small_configs():
    import bench
    args = argparse.Namespace(experiment="grid", steps=1, warmup=0, maxit=200, seed=0)
    configs = [dict(n=20000, k=20, p=10, d=1.0), dict(n=20000, k=20, p=10, d=0.3),
               dict(n=12000, k=70, p=8, d=1.0)]
    print("CASE experiments", configs, flush=True)
    lines = bench.run_experiment(args, configs)
    assert len(lines) == 2 * len(configs)
    for ln in lines:
        json.dumps(ln)
        assert "error" not in ln, ln
        assert ln["mode"] in ("SaP-C", "SaP-D") and ln["factor_prec"] == "fp32"
        assert ln["converged"] and ln["rel_resid_true"] <= 1e-10
        assert ln["rel_err_vs_xtrue"] <= 1e-8
        assert ln["iters"] * 4 == int(ln["iters"] * 4)
        assert ln["ms"] > 0 and ln["t_factor_ms"] > 0
