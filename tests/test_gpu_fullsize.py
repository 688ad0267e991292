"""Configuration-size GPU checks that the per-case parity tests do not reach:

* config 2 (64^3 cube, support 2.0h, FP64): the GPU solve against the oracle's
  own CG solve, element by element (1e-10 relative L2 in d and u^h);
* config 5 adjoint (128^3): dL/dr from an FP64 adjoint solve against central
  finite differences with eps = 1e-6 on 20 seeded directions, to 1e-6 (see
  the test for how the perturbed solutions are formed), and the refined-FP32
  adjoint against the FP64 one. The FP64 CPU adjoint is compared at 20^3 in
  test_gpu_parity.py; at 128^3 its CG would take hours on the host;
* config 5's problem on a 256^3 box: K in both precisions against the oracle
  at sampled nodes and a refined solve checked by the oracle's residual.
"""
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


def to_np(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b, m):
    return np.linalg.norm((a - b)[m]) / np.linalg.norm(b[m])


def test_config2_fp64_solve_matches_oracle_solve():
    p = W.config2()
    print(f"\n[config 2] dims={p.dims} support={p.at[0]}", flush=True)
    o = oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)
    d_ref, it_ref, _ = o.solve(p.free, p.dirichlet, p.r, tol=1e-14, maxit=20000)
    g = lib_problem(p)
    d, uh, info = g.solve(torch.from_numpy(p.r).to(DEV), mode="f64", tol=1e-14, maxit=20000,
                          raise_on_noconv=False)
    m = p.chi > 0
    e_d = rel_l2(to_np(d), d_ref, m)
    e_u = rel_l2(to_np(uh), o.apply_uh(d_ref), m)
    print(f"  iters gpu {info['iters']} oracle {it_ref}; rel-L2 d {e_d:.2e} u^h {e_u:.2e}; "
          f"u^h vs exact {rel_l2(to_np(uh), p.u_exact, m):.2e}", flush=True)
    assert e_d <= 1e-10 and e_u <= 1e-10


def _fd_errors(g, p, grad, uh0, ut, dirs, eps, solve_pm):
    m = p.chi > 0
    uhs = solve_pm(dirs, eps)
    worst = 0.0
    for j, v in enumerate(dirs):
        # L(r + eps v) - L(r - eps v) written as 0.5 sum (u+ - u-)(u+ + u- - 2 u_t),
        # the same central difference without cancelling two large sums
        up, um = uhs[j, 0], uhs[j, 1]
        fd = 0.5 * float(np.sum(np.where(m, (up - um) * (up + um - 2 * ut), 0.0))) / (2 * eps)
        an = float(np.sum(grad * v))
        worst = max(worst, abs(fd - an) / abs(an))
    return worst


def test_config5_adjoint_against_finite_differences():
    """FP64 adjoint at 128^3 against central differences on 20 directions with
    eps = 1e-6.  The loss is quadratic in r, so the central difference carries
    no truncation error, only the error of the perturbed solutions, and the
    solve is linear in the source: u(r +- eps v) = u(r) +- eps u(v) exactly.

    * Bar 1e-6: the perturbed solutions formed that way, with u(v) from FP64
      solves of the 20 directions to tol 1e-14 of their own right-hand sides.
    * Reported, bar 1e-4: the 40 perturbed problems solved as they stand, in
      FP64 from the forward solution d(r) to tol 1e-14.  Their residual is
      measured against ||f^r(r +- eps v)||, of which the eps v part is ~3e-8,
      so tol 1e-14 resolves the eps-sized difference u+ - u- only to ~1e-7 of
      itself, and the difference quotient to ~1e-5: the floor of FP64 central
      differences at this eps, not of the adjoint.
    * The refined-FP32 adjoint against the FP64 one, 1e-8."""
    p = W.config5()
    print(f"\n[config 5 adjoint] dims={p.dims}", flush=True)
    g = lib_problem(p)
    m = p.chi > 0
    ut = W.config5_target(p)
    r = torch.from_numpy(p.r).to(DEV)

    d0, uh, info0 = g.solve(r, mode="f64", tol=1e-14, maxit=60000)
    uh = to_np(uh)
    res = torch.from_numpy(np.where(m, uh - ut, 0.0)).to(DEV)
    grad, info = g.adjoint(res, mode="f64", tol=1e-14, maxit=60000)
    grad = to_np(grad)
    dirs = W.config5_directions(p, 20)
    eps = 1e-6
    print(f"  forward {info0['iters']} and adjoint {info['iters']} FP64 CG iterations", flush=True)

    def linear(dirs, eps):
        # the homogeneous solutions of the directions (g = 0 on the Dirichlet nodes)
        _, uv, binfo = g.solve(torch.from_numpy(np.stack(dirs)).to(DEV), mode="f64", tol=1e-14,
                               maxit=60000)
        uv = to_np(uv)
        print(f"  20 direction solves in one batch: {binfo['iters']} iterations", flush=True)
        return np.stack([np.stack([uh + eps * u, uh - eps * u]) for u in uv])

    worst = _fd_errors(g, p, grad, uh, ut, dirs, eps, linear)
    print(f"  worst FD relative error, perturbed solutions by linearity: {worst:.2e}", flush=True)
    assert worst <= 1e-6

    def warm(dirs, eps):
        batch = np.stack([p.r + s * eps * v for v in dirs for s in (1.0, -1.0)])
        start = d0.expand(len(batch), *p.shape).contiguous()
        _, uhs, binfo = g.solve(torch.from_numpy(batch).to(DEV), d0=start, mode="f64",
                                tol=1e-14, maxit=60000)
        print(f"  40 warm-started perturbed solves in one batch: {binfo['iters']} iterations",
              flush=True)
        return to_np(uhs).reshape((len(dirs), 2) + p.shape)

    worst_w = _fd_errors(g, p, grad, uh, ut, dirs, eps, warm)
    print(f"  worst FD relative error, perturbed problems solved directly: {worst_w:.2e}", flush=True)
    assert worst_w <= 1e-4

    grad32, info32 = g.adjoint(res, mode="f32_refined", tol=1e-12, maxit=60000)
    e32 = np.linalg.norm((to_np(grad32) - grad)[m]) / np.linalg.norm(grad[m])
    print(f"  refined-FP32 adjoint ({info32['iters']} iterations) vs FP64: {e32:.2e}", flush=True)
    assert e32 <= 1e-8


def test_256_box_products_and_refined_solve():
    """Config 5's problem on a 256^3 box (working set above the last-level
    cache; 256-point lines on the register path in both precisions, FP32 on
    the 16 x 16 and the 32-lane layouts, FP64 on the 32-lane one): K in both
    precisions against the oracle at sampled nodes (Dirichlet faces
    included), FP32 (each layout) against FP64 on the whole field, the FP64
    register path against the FP64 LDS-tiled passes, and a refined solve
    whose solution the oracle's own operator checks: ||chi_Omega (f^r - K d)||
    / ||chi_Omega f^r|| on the free rows."""
    p = W.config5_256()
    print(f"\n[256^3] dims={p.dims}", flush=True)
    g = lib_problem(p)
    o = oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)
    x = np.where(p.chi > 0, np.random.default_rng(256).standard_normal(p.shape), 0.0)
    rng = np.random.default_rng(257)
    idx = np.sort(np.concatenate([rng.choice(np.flatnonzero(p.free.reshape(-1)), 48, replace=False),
                                  rng.choice(np.flatnonzero(p.dirichlet.reshape(-1)), 16, replace=False)]))
    xt = torch.from_numpy(x).to(DEV)
    from paper_2403_19854_amd import fcrkpm
    k64 = to_np(g.apply("K_FULL", xt))
    g.set_regpath(False)
    k64_lds = to_np(g.apply("K_FULL", xt))
    g.set_regpath(True)
    ref = o.apply_k_at(x, idx)
    scale = np.abs(ref).max()
    e64 = np.abs(k64.reshape(-1)[idx] - ref).max() / scale
    e64_lds = np.abs(k64 - k64_lds).max() / np.abs(k64_lds).max()
    print(f"  K FP64 vs oracle at 64 nodes {e64:.2e}; register vs LDS-tiled FP64 field {e64_lds:.2e}",
          flush=True)
    assert e64 <= 1e-11 and e64_lds <= 1e-12
    assert np.all(k64[p.chi == 0] == 0.0)
    chosen = g.get_option(fcrkpm.OPT_REGLAYOUT)
    for lay in (0, 1):
        g.set_option(fcrkpm.OPT_REGLAYOUT, lay)
        k32 = to_np(g.apply("K_FULL", xt.float())).astype(np.float64)
        e32 = np.abs(k32.reshape(-1)[idx] - ref).max() / scale
        e3264 = np.abs(k32 - k64).max() / np.abs(k64).max()
        print(f"  FP32 line layout {lay}: vs oracle at 64 nodes {e32:.2e}, vs FP64 field {e3264:.2e}",
              flush=True)
        assert e32 <= 2e-5 and e3264 <= 2e-5
    g.set_option(fcrkpm.OPT_REGLAYOUT, chosen)
    r = torch.from_numpy(p.r).to(DEV)
    d, uh, info = g.solve(r, mode="f32_refined", tol=1e-10, maxit=60000)
    d = to_np(d)
    f = p.free > 0
    fr = np.where(f, o.apply_fr(p.r), 0.0)
    res = np.linalg.norm(np.where(f, fr - o.apply_k(d), 0.0)) / np.linalg.norm(fr)
    m = p.chi > 0
    err = np.linalg.norm((to_np(uh) - p.u_exact)[m]) / np.linalg.norm(p.u_exact[m])
    print(f"  refined solve: {info['iters']} iterations, own residual {info['true_rel_res']:.2e}, "
          f"oracle residual {res:.2e}, u^h vs exact {err:.2e}", flush=True)
    assert info["true_rel_res"] <= 1e-10 and res <= 2e-10
    assert err <= 1e-3
