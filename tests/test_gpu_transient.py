"""GPU parity of the time-dependent part (App. C) against the FP64 CPU oracle:
the consistent mass product (Eq C.8, Alg C.1), the lumped mass (Eq C.13,
Alg C.2), implicit theta-method steps (Alg C.4) in FP64 and refined FP32, and
explicit forward-Euler steps with the lumped mass (Alg C.3).  The cases cover
every basis size and coefficient-row count of the K-type passes (mass: one
row; shifted operator: dim + 1 rows) in 1D, 2D and 3D, cube and ball, and the
register-resident passes at 32^3-128^3.  Bars: FP64 products 1e-11
relative max-norm, FP32 products 2e-5 (2e-4 quadratic), FP64 time stepping
1e-9 relative L2, refined FP32 stepping 1e-8."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2403_19854_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def lib_problem(p):
    from paper_2403_19854_amd import fcrkpm
    return fcrkpm.Problem.from_workload(p, device=DEV)


def orc(p):
    o = oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)
    assert o.singular_node < 0
    return o


def to_np(t):
    return t.detach().cpu().numpy()


def rel_max(a, b):
    den = np.abs(b).max()
    return np.abs(np.asarray(a) - np.asarray(b)).max() / (den if den > 0 else 1.0)


def rel_l2(a, b, mask):
    a = np.asarray(a)[mask]
    b = np.asarray(b)[mask]
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rand_field(p, seed, mask=None):
    m = p.chi if mask is None else mask
    return np.where(m > 0, np.random.default_rng(seed).standard_normal(p.shape), 0.0)


CASES = {
    "1d_linear_64": lambda: W.cube(1, 64, 2.5, 1),
    "1d_quadratic_48": lambda: W.cube(1, 48, 3.0, 2),
    "2d_linear_32": lambda: W.cube(2, 32, 2.5, 1),
    "2d_quadratic_24": lambda: W.cube(2, 24, 2.5, 2),
    "3d_linear_16": lambda: W.cube(3, 16, 2.5, 1),
    "sphere_quadratic_16": lambda: W.sphere(16, 0.4, 3.0, 2, seed=3),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    p = CASES[request.param]()
    print(f"\n[transient case {request.param}] dims={p.dims} degree={p.degree} support={p.at[0]}",
          flush=True)
    return request.param, p, orc(p), lib_problem(p)


def _dirichlet_values(p, seed):
    return np.where(p.dirichlet > 0, 1.0 + 0.5 * np.random.default_rng(seed).standard_normal(p.shape), 0.0)


def test_mass_fp64_matches_oracle(case):
    name, p, o, g = case
    x = rand_field(p, 41)
    got = to_np(g.apply("M", torch.from_numpy(x).to(DEV)))
    err = rel_max(got, o.apply_m(x))
    print(f"  {name} M fp64 rel-max err {err:.2e}")
    assert err <= 1e-11, (name, err)
    assert np.all(got[p.chi == 0] == 0.0)


def test_mass_fp32_matches_oracle(case):
    name, p, o, g = case
    x = rand_field(p, 42)
    got = to_np(g.apply("M", torch.from_numpy(x).to(DEV).float())).astype(np.float64)
    err = rel_max(got, o.apply_m(x))
    print(f"  {name} M fp32 rel-max err {err:.2e}")
    assert err <= 2e-5 * (10 if p.degree == 2 else 1), (name, err)


def test_lumped_mass_matches_oracle(case):
    # Alg C.2 (the load vector of r = 1) against the row sums of Eq C.9
    name, p, o, g = case
    got = to_np(g.coeffs("lumped"))
    err = rel_max(got, o.lumped_mass())
    print(f"  {name} lumped mass rel-max err {err:.2e}")
    assert err <= 1e-11, (name, err)
    assert np.all(got[p.chi == 0] == 0.0)


def test_stiffness_unchanged_after_mass(case):
    # the mass and shifted coefficient sets are swapped in and out around
    # their products: K afterwards equals K before, bit for bit
    name, p, o, g = case
    x = torch.from_numpy(rand_field(p, 43)).to(DEV)
    before = to_np(g.apply("K", x))
    g.apply("M", x)
    g.transient(x, 0.7, 1e-3, 1, mode="f64", tol=1e-10)
    np.testing.assert_array_equal(to_np(g.apply("K", x)), before)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_implicit_fp64_matches_oracle(case, theta):
    # the consistent mass of the smooth RK shape functions is badly conditioned
    # at high frequencies: every step takes hundreds to thousands of CG
    # iterations, so the cases are small and both sides solve to 1e-13
    name, p, o, g = case
    nu, n = 0.7, 2
    dt = 2.0 * min(p.h) ** 2 / nu
    d0 = rand_field(p, 44)
    gv = _dirichlet_values(p, 45)
    print(f"  {name} implicit theta={theta}: oracle steps", flush=True)
    ref, its = o.transient(p.free, p.dirichlet, d0, nu, dt, n, r=p.r, g=gv, theta=theta, tol=1e-13)
    d, _, info = g.transient(torch.from_numpy(d0).to(DEV), nu, dt, n, r=torch.from_numpy(p.r),
                             g=torch.from_numpy(gv), theta=theta, mode="f64", tol=1e-13)
    d = to_np(d)
    err = rel_l2(d, ref, p.chi > 0)
    print(f"  {name} implicit theta={theta} fp64: rel-L2 {err:.2e}, "
          f"{info['iters']} GPU / {its} oracle CG iterations")
    assert err <= 1e-9, (name, err)
    np.testing.assert_array_equal(d[p.dirichlet > 0], gv[p.dirichlet > 0])
    assert np.all(d[p.chi == 0] == 0.0)


@pytest.mark.parametrize("name", ["3d_linear_16", "sphere_quadratic_16", "1d_linear_64"])
def test_implicit_refined_matches_oracle(name):
    p = CASES[name]()
    o = orc(p)
    g = lib_problem(p)
    nu, n = 1.0, 2
    dt = 4.0 * min(p.h) ** 2
    d0 = rand_field(p, 46)
    print(f"\n  {name} implicit refined: oracle steps", flush=True)
    ref, _ = o.transient(p.free, p.dirichlet, d0, nu, dt, n, r=p.r, tol=1e-13)
    d, _, info = g.transient(torch.from_numpy(d0).to(DEV), nu, dt, n, r=torch.from_numpy(p.r),
                             mode="f32_refined", tol=1e-12)
    err = rel_l2(to_np(d), ref, p.chi > 0)
    print(f"\n  {name} implicit refined: rel-L2 {err:.2e}; {info['iters']} FP32 CG iterations, "
          f"{info['outer_iters']} refinement steps")
    assert err <= 1e-8, (name, err)
    # in 3D the FP32 iteration carries every step; on the 61 unknowns of the
    # 1D case it stalls above tol and the solver finishes in FP64 from its
    # best iterate
    if p.dim == 3:
        assert info["fallback_used"] == 0


def test_explicit_matches_oracle(case):
    name, p, o, g = case
    nu, n = 0.7, 5
    dt = 0.02 * min(p.h) ** 2 / nu
    d0 = rand_field(p, 47)
    gv = _dirichlet_values(p, 48)
    ref, _ = o.transient(p.free, p.dirichlet, d0, nu, dt, n, r=p.r, g=gv, scheme="explicit")
    d, _, info = g.transient(torch.from_numpy(d0).to(DEV), nu, dt, n, r=torch.from_numpy(p.r),
                             g=torch.from_numpy(gv), scheme="explicit", mode="f64")
    err = rel_l2(to_np(d), ref, p.chi > 0)
    print(f"  {name} explicit: rel-L2 {err:.2e}")
    assert err <= 1e-10, (name, err)
    assert info["matvecs_f64"] == n


def test_batched_steps_equal_single():
    p = CASES["3d_linear_16"]()
    g = lib_problem(p)
    d0 = np.stack([rand_field(p, 50 + j) for j in range(3)])
    dt = 2.0 * p.h[0] ** 2
    both, _, _ = g.transient(torch.from_numpy(d0).to(DEV), 1.0, dt, 2, r=torch.from_numpy(p.r),
                             mode="f64", tol=1e-12)
    for j in range(3):
        one, _, _ = g.transient(torch.from_numpy(d0[j]).to(DEV), 1.0, dt, 2,
                                r=torch.from_numpy(p.r), mode="f64", tol=1e-12)
        assert rel_l2(to_np(both[j]), to_np(one), p.chi > 0) <= 1e-11


def test_transient_argument_errors():
    from paper_2403_19854_amd import fcrkpm
    p = CASES["3d_linear_16"]()
    g = lib_problem(p)
    d0 = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    for kw in (dict(theta=0.0), dict(theta=1.5), dict(scheme="bogus")):
        with pytest.raises(fcrkpm.FcrkpmError) as e:
            g.transient(d0, 1.0, 1e-3, 1, **kw)
        assert e.value.status == fcrkpm.ERR_ARG
    with pytest.raises(fcrkpm.FcrkpmError) as e:
        g.transient(d0, 1.0, -1e-3, 1)
    assert e.value.status == fcrkpm.ERR_ARG
    with pytest.raises(fcrkpm.FcrkpmError) as e:
        g.transient(d0, 1.0, 1e-3, 1, scheme="explicit", mode="f32_refined")
    assert e.value.status == fcrkpm.ERR_UNSUPPORTED
    # zero steps only imposes the Dirichlet values
    gv = _dirichlet_values(p, 3)
    x = rand_field(p, 4)
    d, _, _ = g.transient(torch.from_numpy(x).to(DEV), 1.0, 1e-3, 0, g=torch.from_numpy(gv))
    np.testing.assert_array_equal(to_np(d), np.where(p.free > 0, x, gv))


@pytest.mark.parametrize("n", [32, 48, 64, 96, 128])
def test_register_path_mass_and_implicit_step(n):
    """The register-resident passes with the mass rows and the shifted rows
    (linear basis; the sets carry their own line-constant records, so the P x Q
    boxes take the register path too, and FP64 runs on the FP64 register path;
    256 points in the test below): M in FP32 and FP64 against the oracle over the
    whole box, and one refined implicit step against the FP64 step, which the
    small cases pin to the oracle."""
    p = W.cube(3, n, 2.5, 1)
    print(f"\n[register path transient {n}^3]", flush=True)
    o = orc(p)
    g = lib_problem(p)
    x = rand_field(p, 60)
    xt = torch.from_numpy(x).to(DEV)
    ref = o.apply_m(x)
    reg = to_np(g.apply("M", xt.float())).astype(np.float64)
    g.set_regpath(False)
    lds = to_np(g.apply("M", xt.float())).astype(np.float64)
    g.set_regpath(True)
    e_reg, e_lds = rel_max(reg, ref), rel_max(lds, ref)
    m64 = to_np(g.apply("M", xt))
    e64 = rel_max(m64, ref)
    print(f"  M fp32: register path {e_reg:.2e}, LDS path {e_lds:.2e}; fp64 {e64:.2e} (rel-max vs oracle)")
    assert e_reg <= 2e-5 and e_lds <= 2e-5 and e64 <= 1e-11
    dt = 4.0 * p.h[0] ** 2
    # two solves that stop at a residual of tol differ by up to cond * tol, and
    # this operator needs thousands of iterations: both go to 1e-13
    d, _, info = g.transient(xt, 1.0, dt, 1, r=torch.from_numpy(p.r), mode="f32_refined", tol=1e-13)
    w64, _, i64 = g.transient(xt, 1.0, dt, 1, r=torch.from_numpy(p.r), mode="f64", tol=1e-13)
    err = rel_l2(to_np(d), to_np(w64), p.chi > 0)
    print(f"  implicit step refined vs FP64: rel-L2 {err:.2e}; {info['iters']} FP32 / "
          f"{i64['iters']} FP64 iterations")
    assert err <= 1e-8
    assert info["fallback_used"] == 0


def test_register_path_mass_256():
    """The consistent mass on a 256^3 box: FP32 on both 256-point layouts (16 x
    16 and 32 lanes x 8) and FP64 on the 32-lane FP64 register path, against
    the oracle over the whole box and against the LDS-tiled passes."""
    from paper_2403_19854_amd import fcrkpm
    p = W.cube(3, 256, 2.5, 1)
    print("\n[register path mass 256^3]", flush=True)
    o = orc(p)
    g = lib_problem(p)
    x = rand_field(p, 61)
    xt = torch.from_numpy(x).to(DEV)
    ref = o.apply_m(x)
    m64 = to_np(g.apply("M", xt))
    g.set_regpath(False)
    lds64 = to_np(g.apply("M", xt))
    g.set_regpath(True)
    e64, e64_lds = rel_max(m64, ref), rel_max(m64, lds64)
    print(f"  M fp64: vs oracle {e64:.2e}, vs LDS-tiled {e64_lds:.2e} (rel-max)", flush=True)
    assert e64 <= 1e-11 and e64_lds <= 1e-12
    chosen = g.get_option(fcrkpm.OPT_REGLAYOUT)
    for lay in (0, 1):
        g.set_option(fcrkpm.OPT_REGLAYOUT, lay)
        m32 = to_np(g.apply("M", xt.float())).astype(np.float64)
        e32 = rel_max(m32, ref)
        print(f"  M fp32, line layout {lay}: vs oracle {e32:.2e}", flush=True)
        assert e32 <= 2e-5
    g.set_option(fcrkpm.OPT_REGLAYOUT, chosen)
