"""Pins of the oracle's time-dependent part (App. C) against what the
mathematics fixes: an independent dense construction of M = N^T V N (Eq C.5),
the exact interior mass row of the 1D linear basis, partition of unity (the
zeroth reproducing condition) behind Eq C.9, symmetry and definiteness of M,
the amplification factors of generalised eigenmodes under the theta method and
under forward Euler with the lumped mass, and the static solution as the fixed
point of every scheme."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2403_19854_amd import workloads as W


def make(p, vol=None):
    return oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol if vol is None else vol)


def _dense_psi_1d(p):
    """Psi[S, J] = Psi_J(x_S) of the 1D linear basis from explicit moment
    matrices with the unscaled basis (Eq 2-3), on the domain nodes."""
    x = p.coords[0]
    a = p.at[0] * p.h[0]
    idx = np.flatnonzero(p.chi)
    Psi = np.zeros((p.nn, p.nn))
    for S in idx:
        M = np.zeros((2, 2))
        for J in idx:
            z = x[S] - x[J]
            M += np.outer([1, z], [1, z]) * oracle.phi1(z / a)
        Mi = np.linalg.inv(M)
        for J in idx:
            z = x[S] - x[J]
            Psi[S, J] = Mi[0] @ np.array([1, z]) * oracle.phi1(z / a)
    return Psi


def test_mass_dense_brute_force_1d():
    p = W.cube(1, 24, 2.5, 1)
    Psi = _dense_psi_1d(p)
    M = Psi.T @ np.diag(p.vol) @ Psi
    o = make(p)
    d = np.random.default_rng(5).standard_normal(p.nn) * p.chi
    np.testing.assert_allclose(o.apply_m(d), M @ d, atol=1e-14 * np.abs(M @ d).max() + 1e-16)
    np.testing.assert_allclose(o.lumped_mass(), M @ p.chi.astype(float), atol=1e-15)


def _phi_frac(o, at):
    z = Fraction(abs(o)) / at
    if z <= Fraction(1, 2):
        return Fraction(2, 3) - 4 * z * z + 4 * z ** 3
    if z < 1:
        return Fraction(4, 3) - 4 * z + 4 * z * z - Fraction(4, 3) * z ** 3
    return Fraction(0)


def test_mass_1d_interior_row_closed_form():
    # With a full symmetric neighbourhood the first moment vanishes, so the
    # linear basis gives Psi_I(x_K) = phi(K - I) / sum_j phi(j) at the nodes and
    # M_IJ = h sum_K S(K - I) S(K - J): the autocorrelation of S, times h.
    at = Fraction(5, 2)
    p = W.cube(1, 48, 2.5, 1, source="zero")
    h = p.h[0]
    o = make(p, np.where(p.chi > 0, h, 0.0))
    ph = {k: _phi_frac(k, at) for k in range(-2, 3)}
    s0 = sum(ph.values())
    S = {k: v / s0 for k, v in ph.items()}
    R = {}
    for a_, va in S.items():
        for b_, vb in S.items():
            R[b_ - a_] = R.get(b_ - a_, 0) + va * vb
    c = 20
    e = np.zeros(p.shape)
    e[c] = 1.0
    col = o.apply_m(e)
    for k in range(-4, 5):
        assert col[c + k] == pytest.approx(float(R[k]) * h, rel=1e-13)
    assert np.all(col[:c - 4] == 0) and np.all(col[c + 5:] == 0)
    # the lumped entry of an interior node is its volume h (rows of M sum to
    # int Psi_I = h sum_K S(K - I) = h)
    assert o.lumped_mass()[c] == pytest.approx(h, rel=1e-13)


@pytest.mark.parametrize("maker", [
    lambda: W.cube(3, 12, 2.5, 1),
    lambda: W.cube(3, 12, 3.0, 2),
    lambda: W.cube(2, 20, 2.0, 1),
    lambda: W.sphere(16, 0.4, 3.0, 2),
])
def test_mass_partition_of_unity_and_total_volume(maker):
    p = maker()
    o = make(p)
    X = W._mesh(p.coords)
    lin = np.ones(p.shape)
    for k in range(p.dim):
        lin = lin + (0.5 + k) * X[k]
    lin = np.where(p.chi > 0, lin, 0.0)
    # sum_I Psi_I = 1 at domain nodes, and N reproduces linear fields exactly:
    # the column sums of M d for d = nodal values of a linear p are sum_K V_K p(x_K)
    fm = o.apply_m(lin)
    assert fm.sum() == pytest.approx(float((p.vol * lin).sum()), rel=1e-12)
    ml = o.lumped_mass()
    assert ml.sum() == pytest.approx(float(p.vol.sum()), rel=1e-12)
    assert np.all(ml[p.chi == 0] == 0.0)
    assert ml[p.chi > 0].min() > 0.0


def _dense(op, idx, nn, shape):
    A = np.zeros((idx.size, idx.size))
    for j, J in enumerate(idx):
        e = np.zeros(nn)
        e[J] = 1.0
        A[:, j] = op(e.reshape(shape)).reshape(-1)[idx]
    return A


def test_mass_symmetric_positive_definite_2d():
    p = W.cube(2, 12, 2.5, 1)
    o = make(p)
    idx = np.flatnonzero(p.chi)
    M = _dense(o.apply_m, idx, p.nn, p.shape)
    np.testing.assert_allclose(M, M.T, atol=1e-15 * np.abs(M).max())
    assert np.linalg.eigvalsh(M).min() > 0.0


def _ops_1d(p, o):
    idx = np.flatnonzero(p.free)
    K = _dense(lambda v: o.apply_k_free(v, p.free), idx, p.nn, p.shape)
    M = _dense(lambda v: np.where(p.free > 0, o.apply_m(np.where(p.free > 0, v, 0.0)), 0.0),
               idx, p.nn, p.shape)
    return idx, K, M


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_implicit_eigenmode_amplification(theta):
    # (K, M) on the free rows: K v = lam M v.  A mode decays by
    # (1 - (1-theta) dt nu lam) / (1 + theta dt nu lam) per step.
    p = W.cube(1, 28, 2.5, 1, source="zero")
    o = make(p)
    idx, K, M = _ops_1d(p, o)
    lam, V = scipy.linalg.eigh(K, M)
    nu, dt, n = 0.7, 2e-3, 5
    for j in (0, 3, idx.size - 1):
        d0 = np.zeros(p.nn)
        d0[idx] = V[:, j]
        d, _ = o.transient(p.free, p.dirichlet, d0.reshape(p.shape), nu, dt, n,
                           scheme="implicit", theta=theta, tol=1e-14)
        amp = (1 - (1 - theta) * dt * nu * lam[j]) / (1 + theta * dt * nu * lam[j])
        np.testing.assert_allclose(d.reshape(-1)[idx], amp ** n * V[:, j],
                                   atol=1e-11 * np.abs(V[:, j]).max())
        assert np.all(d.reshape(-1)[p.free.reshape(-1) == 0] == 0.0)


def test_explicit_eigenmode_amplification():
    # forward Euler with the lumped mass: K v = lam diag(M^l) v decays by
    # (1 - dt nu lam) per step
    p = W.cube(1, 28, 2.5, 1, source="zero")
    o = make(p)
    idx, K, _ = _ops_1d(p, o)
    ml = o.lumped_mass().reshape(-1)[idx]
    lam, V = scipy.linalg.eigh(K, np.diag(ml))
    nu, n = 0.7, 6
    dt = 1.5 / (nu * lam[-1])            # inside the stability limit 2 / (nu lam_max)
    for j in (0, 5, idx.size - 1):
        d0 = np.zeros(p.nn)
        d0[idx] = V[:, j]
        d, _ = o.transient(p.free, p.dirichlet, d0.reshape(p.shape), nu, dt, n, scheme="explicit")
        np.testing.assert_allclose(d.reshape(-1)[idx], (1 - dt * nu * lam[j]) ** n * V[:, j],
                                   atol=1e-12 * np.abs(V[:, j]).max())


@pytest.mark.parametrize("scheme,theta", [("implicit", 1.0), ("implicit", 0.5), ("explicit", 1.0)])
def test_static_solution_is_a_fixed_point(scheme, theta):
    # nu K d* = f^r with d* = g on the Dirichlet nodes is a fixed point of
    # every scheme: a wrong sign, a missing nu or a dropped Dirichlet term moves it
    p = W.cube(2, 14, 2.5, 1, source="linear")
    p.r = np.where(p.chi > 0, 1.0 + W._mesh(p.coords)[0], 0.0)
    o = make(p)
    nu = 0.7
    ds, _, _ = o.solve(p.free, p.dirichlet, p.r / nu, g=p.g, tol=1e-14)
    dt = 1e-3 if scheme == "explicit" else 0.05
    d, _ = o.transient(p.free, p.dirichlet, ds, nu, dt, 3, r=p.r, g=p.g, scheme=scheme,
                       theta=theta, tol=1e-14)
    np.testing.assert_allclose(d, ds, atol=1e-10 * np.abs(ds).max())
    # and a start away from it moves towards it
    d1, _ = o.transient(p.free, p.dirichlet, np.zeros(p.shape), nu, 0.05, 40, r=p.r, g=p.g,
                        scheme="implicit", tol=1e-14)
    d0 = np.where(p.dirichlet > 0, p.g, 0.0)
    assert np.abs(d1 - ds).max() < 0.5 * np.abs(d0 - ds).max()
