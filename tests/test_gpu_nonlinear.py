"""GPU parity of the nonlinear part (App. B: N(u) = kappa u^3, and the gradient
nonlinearity N(g) = (1 + kappa |g|^2) g of Alg B.1) against the
FP64 CPU oracle: the nonlinear force (Eq B.9, Alg B.2) and Newton solves of
-lap u + kappa u^3 = r (App. B.3) in FP64 and refined FP32, in 1D, 2D and 3D
with the linear and quadratic basis, and a 64^3 solve on the
register-resident passes.  Bars: force 1e-11 relative max-norm, FP64 solves
1e-10 relative L2, refined 1e-8."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2403_19854_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"
KAPPA = 5.0


def lib_problem(p):
    from paper_2403_19854_amd import fcrkpm
    return fcrkpm.Problem.from_workload(p, device=DEV)


def orc(p):
    o = oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)
    assert o.singular_node < 0
    return o


def to_np(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b, mask):
    a = np.asarray(a)[mask]
    b = np.asarray(b)[mask]
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = {
    "1d_linear_64": lambda: W.cube(1, 64, 2.0, 1),
    "2d_linear_32": lambda: W.cube(2, 32, 2.0, 1),
    "2d_quadratic_24": lambda: W.cube(2, 24, 2.5, 2),
    "3d_linear_16": lambda: W.cube(3, 16, 2.5, 1),
    "3d_quadratic_16": lambda: W.cube(3, 16, 2.5, 2),
}


def _source(p):
    # manufactured: r = -lap u + kappa u^3 where u is known, else a scaled random source
    if p.u_exact is not None:
        return p.r + KAPPA * p.u_exact ** 3
    return 20.0 * p.r


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    p = CASES[request.param]()
    print(f"\n[nonlinear case {request.param}] dims={p.dims} degree={p.degree} support={p.at[0]}",
          flush=True)
    return request.param, p, orc(p), lib_problem(p)


def test_force_matches_oracle(case):
    name, p, o, g = case
    d = np.where(p.chi > 0, np.random.default_rng(60).standard_normal(p.shape), 0.0)
    ref = o.apply_fn(d, 2.5)
    got = to_np(g.nonlinear_force(torch.from_numpy(d), 2.5))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  {name} f^N rel-max err {err:.2e}")
    assert err <= 1e-11
    assert np.all(got[p.chi == 0] == 0.0)


def test_newton_fp64_matches_oracle(case):
    name, p, o, g = case
    r = _source(p)
    print(f"  {name} oracle Newton", flush=True)
    ref, steps, its = o.solve_nonlinear(p.free, p.dirichlet, r, KAPPA, newton_tol=1e-11)
    d, uh, info = g.solve_nonlinear(torch.from_numpy(r), KAPPA, mode="f64", tol=1e-13,
                                    newton_tol=1e-11)
    m = p.chi > 0
    err = rel_l2(to_np(d), ref, m)
    print(f"  {name} Newton fp64: rel-L2 {err:.2e}; {info['outer_iters']} / {steps} steps, "
          f"{info['iters']} / {its} CG iterations, |R|/|f| {info['rel_res']:.1e}")
    assert err <= 1e-10, (name, err)
    assert info["rel_res"] <= 1e-11
    if p.u_exact is not None:
        e_gpu = rel_l2(to_np(uh), p.u_exact, m)
        e_orc = rel_l2(o.apply_uh(ref), p.u_exact, m)
        assert abs(e_gpu - e_orc) <= 1e-6 * e_orc


def test_kappa_zero_is_the_linear_solve():
    p = CASES["2d_linear_32"]()
    g = lib_problem(p)
    r = torch.from_numpy(p.r)
    d, _, info = g.solve_nonlinear(r, 0.0, mode="f64", tol=1e-13, newton_tol=1e-11)
    lin, _, _ = g.solve(r, mode="f64", tol=1e-13)
    assert info["outer_iters"] == 1
    assert rel_l2(to_np(d), to_np(lin), p.chi > 0) <= 1e-11


@pytest.mark.parametrize("name", ["3d_linear_16", "2d_linear_32", "3d_quadratic_16"])
def test_newton_refined_matches_oracle(name):
    p = CASES[name]()
    o = orc(p)
    g = lib_problem(p)
    r = _source(p)
    ref, _, _ = o.solve_nonlinear(p.free, p.dirichlet, r, KAPPA, newton_tol=1e-11)
    d, _, info = g.solve_nonlinear(torch.from_numpy(r), KAPPA, mode="f32_refined", tol=1e-12,
                                   newton_tol=1e-11)
    err = rel_l2(to_np(d), ref, p.chi > 0)
    print(f"\n  {name} Newton refined: rel-L2 {err:.2e}; {info['outer_iters']} steps, "
          f"{info['iters']} FP32 iterations")
    assert err <= 1e-8, (name, err)


def test_newton_argument_errors():
    from paper_2403_19854_amd import fcrkpm
    p = CASES["3d_linear_16"]()
    g = lib_problem(p)
    r = torch.from_numpy(_source(p))
    for kw in (dict(kappa=-1.0), dict(kappa=float("nan"))):
        with pytest.raises(fcrkpm.FcrkpmError) as e:
            g.solve_nonlinear(r, **kw)
        assert e.value.status == fcrkpm.ERR_ARG
    with pytest.raises(fcrkpm.FcrkpmError) as e:
        g.solve_nonlinear(r, KAPPA, newton_tol=0.0)
    assert e.value.status == fcrkpm.ERR_ARG
    # one Newton step cannot reach 1e-14: NOCONV with the iterate returned
    d, _, info = g.solve_nonlinear(r, KAPPA, newton_tol=1e-14, maxnewton=1,
                                   raise_on_noconv=False)
    assert info["status"] == fcrkpm.ERR_NOCONV and info["outer_iters"] == 1
    assert torch.isfinite(d).all()


def test_newton_64_register_path():
    """-lap u + 5 u^3 = r on a 64^3 cube (support 2.0h) with the refined
    solver on the register-resident passes (Jacobian records rebuilt every
    step) against the FP64 Newton solve and the manufactured solution."""
    p = W.cube(3, 64, 2.0, 1)
    print("\n[Newton 64^3]", flush=True)
    g = lib_problem(p)
    r = torch.from_numpy(_source(p))
    d32, uh32, i32 = g.solve_nonlinear(r, KAPPA, mode="f32_refined", tol=1e-12, newton_tol=1e-11)
    d64, _, i64 = g.solve_nonlinear(r, KAPPA, mode="f64", tol=1e-12, newton_tol=1e-11)
    m = p.chi > 0
    err = rel_l2(to_np(d32), to_np(d64), m)
    e_exact = rel_l2(to_np(uh32), p.u_exact, m)
    print(f"  refined vs FP64: rel-L2 {err:.2e}; steps {i32['outer_iters']} / {i64['outer_iters']}, "
          f"CG {i32['iters']} / {i64['iters']}; u^h vs exact {e_exact:.2e}")
    assert err <= 1e-8
    assert e_exact <= 1e-3


def test_gradient_force_matches_oracle(case):
    """Alg B.1 with N(g) = (1 + kappa |g|^2) g: the K passes with the
    nonlinearity applied to the implicit gradient; kappa = 0 is K d bit for bit."""
    name, p, o, g = case
    d = np.where(p.chi > 0, np.random.default_rng(61).standard_normal(p.shape), 0.0)
    dt = torch.from_numpy(d).to(DEV)
    k0 = to_np(g.gradient_force(dt, 0.0))
    np.testing.assert_array_equal(k0, to_np(g.apply("K_FULL", dt)))
    kappa = 0.8 * min(p.h) ** 2      # |grad u^h|^2 ~ 1/h^2 for a random d
    ref = o.apply_fn_grad(d, kappa)
    got = to_np(g.gradient_force(dt, kappa))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    lin = np.abs(ref - o.apply_k(d)).max() / np.abs(ref).max()
    print(f"  {name} gradient force rel-max err {err:.2e} (nonlinear share {lin:.2f})")
    assert err <= 1e-11
    assert lin > 0.05
