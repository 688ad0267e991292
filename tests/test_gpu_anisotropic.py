"""GPU parity on anisotropic grids: per-axis spacing h_k and normalised
support a~_k (Eq 6, 64, 70), box sizes mixing radix 2, 3, 5 and 7, in 1D, 2D
and 3D with the linear and quadratic basis.  Coefficients, FP64 and FP32 operators
and the FP64 solve against the oracle, at the bars of the isotropic cases."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2403_19854_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _box(dims, h, at, degree, seed):
    """Domain: the box minus its last floor(a~_k) nodes per axis (Eq 67);
    Dirichlet layer on its faces; V = prod h_k; r ~ N(0, 1)."""
    dim = len(dims)
    shape = tuple(reversed(dims))
    chi = np.zeros(shape, np.uint8)
    sl = tuple(slice(0, dims[k] - int(math.floor(at[k]))) for k in reversed(range(dim)))
    chi[sl] = 1
    dirichlet = W.face_dirichlet(chi)
    free = (chi - dirichlet).astype(np.uint8)
    vol = np.where(chi > 0, float(np.prod(h)), 0.0)
    r = np.where(chi > 0, np.random.default_rng(seed).standard_normal(shape), 0.0)
    coords = tuple(h[k] * np.arange(dims[k]) for k in range(dim))
    return W.Problem("aniso", dim, tuple(dims), tuple(h), tuple(float(a) for a in at), degree,
                     chi, dirichlet, free, vol, r, coords)


CASES = {
    "3d_linear_24x20x18": lambda: _box((24, 20, 18), (0.05, 0.0625, 0.08), (2.5, 2.0, 1.5), 1, 81),
    "3d_quadratic_16x12x15": lambda: _box((16, 12, 15), (0.05, 0.07, 0.06), (2.5, 2.5, 2.25), 2, 82),
    "2d_quadratic_30x24": lambda: _box((30, 24), (0.03, 0.05), (2.5, 2.25), 2, 83),
    "2d_linear_40x25": lambda: _box((40, 25), (0.025, 0.04), (1.5, 2.5), 1, 84),
    # radix-7 axes: 28 = 4 7, 21 = 3 7, 14 = 2 7, 49 = 7 7, 35 = 5 7
    "3d_linear_28x21x14_radix7": lambda: _box((28, 21, 14), (0.04, 0.05, 0.07), (2.5, 2.0, 2.5), 1, 85),
    "2d_quadratic_49x35_radix7": lambda: _box((49, 35), (0.02, 0.03), (2.5, 2.75), 2, 86),
    "1d_linear_56_radix7": lambda: _box((56,), (0.018,), (2.5,), 1, 87),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    from paper_2403_19854_amd import fcrkpm
    p = CASES[request.param]()
    print(f"\n[anisotropic {request.param}] h={p.h} support={p.at} degree={p.degree}", flush=True)
    o = oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)
    assert o.singular_node < 0
    return request.param, p, o, fcrkpm.Problem.from_workload(p, device=DEV)


def _rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(b).max()


def test_coefficients(case):
    name, p, o, g = case
    m = p.chi > 0
    b0, ob0 = g.coeffs("b0").cpu().numpy(), o.b0()
    ba, oba = g.coeffs("balpha").cpu().numpy(), o.balpha()
    assert np.abs(b0 - ob0)[:, m].max() <= 1e-10 * np.abs(ob0[:, m]).max()
    for a in range(p.dim):
        assert np.abs(ba[a] - oba[a])[:, m].max() <= 1e-10 * np.abs(oba[a][:, m]).max(), (name, a)


@pytest.mark.parametrize("op", ["K", "FR", "UH"])
def test_operators(case, op):
    name, p, o, g = case
    x = np.where(p.chi > 0, np.random.default_rng(90).standard_normal(p.shape), 0.0)
    ref = {"K": lambda: o.apply_k_free(x, p.free), "FR": lambda: o.apply_fr(x),
           "UH": lambda: o.apply_uh(x)}[op]()
    got = g.apply(op, torch.from_numpy(x).to(DEV)).cpu().numpy()
    got32 = g.apply(op, torch.from_numpy(x).to(DEV).float()).cpu().numpy().astype(np.float64)
    e64, e32 = _rel(got, ref), _rel(got32, ref)
    print(f"  {name} {op}: fp64 {e64:.2e}, fp32 {e32:.2e}")
    assert e64 <= 1e-11
    assert e32 <= 2e-5 * (10 if p.degree == 2 else 1)


def test_solve(case):
    name, p, o, g = case
    ref, its, _ = o.solve(p.free, p.dirichlet, p.r, tol=1e-13)
    d, _, info = g.solve(torch.from_numpy(p.r), mode="f64", tol=1e-13)
    m = p.chi > 0
    err = np.linalg.norm((d.cpu().numpy() - ref)[m]) / np.linalg.norm(ref[m])
    print(f"  {name} solve: rel-L2 {err:.2e} ({info['iters']} / {its} iterations)")
    assert err <= 1e-10
