"""fcrkpm_apply_noalloc (the allocation-free apply, scratch in a static
per-GPU array) against fcrkpm_apply through the C ABI: the same kernels on
the same inputs, so the results must agree bit for bit.  Two calls in a row,
the second with a smaller input, so stale scratch contents from the first
call would show."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2403_19854_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def fc():
    from paper_2403_19854_amd import fcrkpm
    return fcrkpm


def _field(p, seed, nrhs, dtype):
    rng = np.random.default_rng(seed)
    x = np.where(p.chi > 0, rng.standard_normal((nrhs,) + p.shape), 0.0)
    return torch.from_numpy(x).to(DEV, dtype)


def _noalloc(g, op, x, out):
    f = fc()
    lib = f.load_library()
    nrhs = x.numel() // g.nn
    return lib.fcrkpm_apply_noalloc(g._h, f._OPS[op], f.F64 if x.dtype == torch.float64 else f.F32,
                                    nrhs, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_apply_two_calls(dtype):
    f = fc()
    big = W.cube(3, 64, 2.5, 1)
    small = W.cube(3, 32, 2.5, 1)
    gb = f.Problem.from_workload(big, device=DEV)
    gs = f.Problem.from_workload(small, device=DEV)
    for g, p, nrhs, ops in ((gb, big, 2, ("K", "FR", "UH")), (gs, small, 1, ("K", "K_FULL", "NT"))):
        for op in ops:
            x = _field(p, 7 + nrhs, nrhs, dtype)
            ref = g.apply(op, x)
            out = torch.full_like(x, float("nan"))
            print(f"\n[noalloc] box {p.dims[0]} nrhs {nrhs} {op} {dtype}", flush=True)
            assert _noalloc(g, op, x, out) == f.OK, f.load_library().fcrkpm_last_error(g._h)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_quadratic_ball_and_mass():
    f = fc()
    p = W.sphere(32, 0.4, 3.0, 2, seed=3)
    g = f.Problem.from_workload(p, device=DEV)
    x = _field(p, 3, 1, torch.float64)
    out = torch.empty_like(x)
    # the mass coefficients are built by the first ordinary M product
    assert _noalloc(g, "M", x, out) == f.ERR_ARG
    ref = g.apply("M", x)
    assert _noalloc(g, "M", x, out) == f.OK
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    ref = g.apply("K", x)
    assert _noalloc(g, "K", x, out) == f.OK
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_rejects_requests_beyond_the_scratch():
    f = fc()
    p = W.cube(3, 128, 2.5, 1)
    g = f.Problem.from_workload(p, device=DEV)
    x = _field(p, 1, 1, torch.float64)
    out = torch.empty_like(x)
    st = _noalloc(g, "K", x, out)
    assert st == f.ERR_ARG
    msg = f.load_library().fcrkpm_last_error(g._h).decode()
    assert "scratch" in msg
    # FP32 at 128^3 with one right-hand side fits exactly
    x32 = x.float()
    out32 = torch.empty_like(x32)
    assert _noalloc(g, "K", x32, out32) == f.OK
    ref = g.apply("K", x32)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out32.cpu().numpy(), ref.cpu().numpy())
