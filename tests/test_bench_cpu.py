"""The bench's CPU-baseline leg on a small box (no GPU): the oracle's K-product
rate on all threads and on one, its CG solve and adjoint to the bench
tolerance (run to the end on boxes up to 64^3), and the oracle residual of a
given iterate."""
import types

import numpy as np

import bench
import oracle
from paper_2403_19854_amd import workloads as W


def test_cpu_baseline_fields():
    wl = W.cube(3, 12, 2.5, 1, source="sin", name="c5_small")
    a = types.SimpleNamespace(cpu_seconds=0.2, cpu_cg_cap=10, maxit=100000, tol=1e-12)
    threads = oracle.threads(0)
    res = bench.cpu_baseline(a, wl, gpu_iters=50, d_fixed=np.zeros(wl.shape))
    assert res["kind"] == "oracle" and res["unit"] == "matvec/s"
    assert res["value"] > 0 and res["cores"] == threads
    assert res["one_thread"]["cores"] == 1 and res["one_thread"]["value"] > 0
    assert res["fr_s"] > 0 and res["uh_s"] > 0
    assert oracle.threads(0) == threads          # the thread count is restored
    sol = res["solve"]
    assert sol["rel_res"] <= 1e-12 and "capped_at" not in sol
    assert res["adjoint"]["iterations"] > 0
    # d = 0 leaves the whole load as the residual
    assert abs(res["oracle_rel_res"] - 1.0) < 1e-12


def test_gpu_clocks_parsing(monkeypatch):
    """The bench's clock report keeps rocm-smi's clock entries of the first
    card and gives None when the tool is missing or prints no JSON."""
    import subprocess

    sample = ('{"card0": {"mclk clock speed:": "(2000Mhz)", "mclk clock level:": "0", '
              '"sclk clock speed:": "(2400Mhz)", "sclk clock level:": "1", "PCI Bus": "x"}}')
    monkeypatch.setattr(subprocess, "run",
                        lambda *a, **k: types.SimpleNamespace(stdout=sample, returncode=0))
    got = bench.gpu_clocks()
    assert got == {"mclk clock speed": "(2000Mhz)", "mclk clock level": "0",
                   "sclk clock speed": "(2400Mhz)", "sclk clock level": "1"}
    monkeypatch.setattr(subprocess, "run",
                        lambda *a, **k: types.SimpleNamespace(stdout="not json", returncode=1))
    assert bench.gpu_clocks() is None

    def missing(*a, **k):
        raise FileNotFoundError("rocm-smi")
    monkeypatch.setattr(subprocess, "run", missing)
    assert bench.gpu_clocks() is None
