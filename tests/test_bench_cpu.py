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
