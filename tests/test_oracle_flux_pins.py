"""Pins of the oracle's boundary flux load (App. A, Eq 28 and A.2-A.3) against
what the mathematics fixes: the exact 1D linear patch with a flux end,
partition of unity (the load integrates the flux exactly), locality of the
load near the flux boundary, and second-order convergence to a manufactured
solution with a flux face (support 2.0h), which a wrong sign or scale of the
flux breaks."""
import math

import numpy as np
import pytest

import oracle
from paper_2403_19854_amd import workloads as W


def make(p):
    return oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)


@pytest.mark.parametrize("at", [1.5, 2.0])
def test_flux_1d_linear_patch_exact(at):
    # u = 1 + 2x on [0, 1]: u(0) = 1 held, flux u'(1) = 2 on the end node
    # (area 1), r = 0; with support in (1, 2] the discrete solution is u
    p = W.cube(1, 40, at, 1, source="zero")
    o = make(p)
    x = p.coords[0]
    n_om = p.meta["n_domain_axis"]
    dirm = np.zeros(p.shape, np.uint8)
    dirm[0] = 1
    free = (p.chi - dirm).astype(np.uint8)
    u = np.where(p.chi > 0, 1 + 2 * x, 0.0)
    area = np.zeros(p.shape)
    area[n_om - 1] = 1.0
    d, _, _ = o.solve_flux(free, dirm, np.zeros(p.shape), np.where(area > 0, 2.0, 0.0), area,
                           g=u, tol=1e-14)
    np.testing.assert_allclose(d[p.chi > 0], u[p.chi > 0], atol=1e-12)


@pytest.mark.parametrize("dim,n,at,deg", [(1, 40, 2.5, 1), (2, 24, 2.5, 1), (3, 14, 2.5, 1),
                                          (3, 14, 3.0, 2)])
def test_flux_load_integrates_the_flux(dim, n, at, deg):
    # sum_I Psi_I = 1 at every domain node, so sum_I f^q_I = sum_S A_S q_S;
    # and f^q vanishes at nodes farther than the support from the flux nodes
    p = W.cube_neumann(dim, n, at, deg)
    o = make(p)
    q = np.where(p.area > 0, np.random.default_rng(9).standard_normal(p.shape), 0.0)
    fq = o.apply_fq(q, p.area)
    assert fq.sum() == pytest.approx(float((p.area * q).sum()), rel=1e-12, abs=1e-14)
    m = int(math.floor(at))
    ix = np.arange(p.dims[0])
    far = ix < p.meta["n_domain_axis"] - 1 - m
    assert np.all(fq[..., far] == 0.0)
    assert np.abs(fq[..., ~far]).max() > 0.0


@pytest.mark.parametrize("dim,ns", [(1, (40, 80)), (2, (24, 48))])
def test_flux_manufactured_second_order(dim, ns):
    errs = []
    for n in ns:
        p = W.cube_neumann(dim, n, 2.0, 1)
        o = make(p)
        m = p.chi > 0
        d, _, _ = o.solve_flux(p.free, p.dirichlet, p.r, p.q, p.area, tol=1e-13)
        errs.append(np.linalg.norm((o.apply_uh(d) - p.u_exact)[m]) / np.linalg.norm(p.u_exact[m]))
        if n == ns[0]:
            # the flux enters with its sign and area: flipping it is an O(1) error
            d2, _, _ = o.solve_flux(p.free, p.dirichlet, p.r, -p.q, p.area, tol=1e-13)
            e2 = np.linalg.norm((o.apply_uh(d2) - p.u_exact)[m]) / np.linalg.norm(p.u_exact[m])
            assert e2 > 0.5
    assert errs[0] < 3e-3
    assert errs[0] / errs[1] > 3.5
