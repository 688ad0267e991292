"""FP64 CPU oracle for the FC-RKPM Poisson hot path -- TEST INFRASTRUCTURE ONLY.

A thin ctypes wrapper around ``rkpm_oracle.c``: the traditional neighbour-loop
RKPM (Galerkin, implicit gradients, direct nodal integration, strong Dirichlet
values) written from the paper's definitions, with no FFT and no periodic
wrap-around.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
library never does, and this package never imports the product library.

The boundary flux load (App. A), the nonlinear force and Newton solve
(App. B) and the time-dependent part (App. C:
consistent and lumped mass, implicit and explicit time stepping of the
diffusion equation) are plain numpy on top of the same neighbour-loop
operators.

Every function works on numpy FP64 arrays in C order ``[nz][ny][nx]``
(x fastest), 0/1 masks as uint8.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rkpm_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

_lib = None


# a copy built with AddressSanitizer + UBSan by clang (whose ASan runtime the
# sanitized product library shares), loaded instead when FCRKPM_ORACLE_LIB names it
_SAN_LIB = os.path.join(_HERE, "_build_san", "liborc.so")


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc + OpenMP into ``oracle/liborc.so``, or with
    sanitize=True with clang, ASan and UBSan into ``oracle/_build_san/liborc.so``."""
    out = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(out):
        os.makedirs(os.path.dirname(out), exist_ok=True)
        tmp = out + ".tmp"
        if sanitize:
            cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                   "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                   "-fno-omit-frame-pointer", "-o", tmp, _SRC, "-lm"]
        else:
            cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("FCRKPM_ORACLE_LIB") or _LIB
    if path == _LIB and not os.path.exists(_LIB):
        build(force=True)
    lib = C.CDLL(path)
    P = C.c_void_p
    dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
    up = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
    lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
    ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
    lib.orc_phi1.restype = C.c_double
    lib.orc_phi1.argtypes = [C.c_double]
    lib.orc_threads.restype = C.c_int
    lib.orc_threads.argtypes = [C.c_int]
    lib.orc_basis_size.restype = C.c_int
    lib.orc_basis_size.argtypes = [C.c_int, C.c_int]
    lib.orc_create.restype = P
    lib.orc_create.argtypes = [C.c_int, ip, dp, dp, C.c_int, up, C.c_void_p]
    lib.orc_destroy.argtypes = [P]
    lib.orc_singular_node.restype = C.c_long
    lib.orc_singular_node.argtypes = [P]
    lib.orc_s.restype = C.c_int
    lib.orc_s.argtypes = [P]
    lib.orc_noff.restype = C.c_int
    lib.orc_noff.argtypes = [P]
    lib.orc_get_b0.argtypes = [P, dp]
    lib.orc_get_ba.argtypes = [P, dp]
    for name in ("orc_apply_k", "orc_apply_fr", "orc_apply_nt", "orc_apply_uh",
                 "orc_apply_vn", "orc_apply_b"):
        getattr(lib, name).argtypes = [P, dp, dp]
    lib.orc_apply_k_at.argtypes = [P, dp, lp, C.c_long, dp]
    lib.orc_apply_btv.argtypes = [P, dp, dp]
    lib.orc_cg.restype = C.c_int
    lib.orc_cg.argtypes = [P, up, dp, dp, C.c_double, C.c_int, C.POINTER(C.c_double)]
    lib.orc_solve.restype = C.c_int
    lib.orc_solve.argtypes = [P, up, up, dp, C.c_void_p, dp, C.c_double, C.c_int,
                              C.POINTER(C.c_double)]
    lib.orc_adjoint.restype = C.c_int
    lib.orc_adjoint.argtypes = [P, up, dp, dp, C.c_void_p, C.c_double, C.c_int,
                                C.POINTER(C.c_double)]
    _lib = lib
    return lib


def threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (n > 0); return the count in force."""
    return int(_load().orc_threads(int(n)))


def phi1(z: float) -> float:
    """Cubic B-spline profile of Eq 7 at z = |x|/a."""
    return _load().orc_phi1(float(z))


def basis_size(dim: int, degree: int) -> int:
    """s = (n+d)!/(d! n!) (Eq 5) as produced by the oracle's basis builder."""
    return _load().orc_basis_size(dim, degree)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Traditional RKPM on the domain nodes of a uniform box grid.

    dims: box nodes per active axis, in (x, y, z) order.
    chi: 0/1 domain mask, shape ``dims[::-1]``.
    vol: nodal quadrature weights V (same shape) or None (V = prod h on chi).
    """

    def __init__(self, dims, h, at, degree, chi, vol=None):
        lib = _load()
        self.dim = len(dims)
        self.dims = tuple(int(v) for v in dims)
        self.shape = tuple(reversed(self.dims))
        n = np.ones(3, np.int32)
        n[: self.dim] = self.dims
        hh = np.ones(3)
        hh[: self.dim] = h
        aa = np.zeros(3)
        aa[: self.dim] = at
        self._hh = hh[: self.dim].copy()
        self.chi = np.ascontiguousarray(chi, dtype=np.uint8).reshape(self.shape)
        self._vol = None if vol is None else _f64(vol).reshape(self.shape)
        vptr = None if self._vol is None else self._vol.ctypes.data_as(C.c_void_p)
        self._h = lib.orc_create(self.dim, n, hh, aa, int(degree),
                                 self.chi.reshape(-1), vptr)
        if not self._h:
            raise MemoryError("oracle allocation failed")
        self.s = lib.orc_s(self._h)
        self.noff = lib.orc_noff(self._h)
        self.nn = int(np.prod(self.dims))
        self.singular_node = lib.orc_singular_node(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    # --- coefficient fields -------------------------------------------------
    def b0(self):
        """b^0 (Eq 83) per node: array [s, *shape]."""
        out = np.empty(self.nn * self.s)
        _load().orc_get_b0(self._h, out)
        return out.reshape(self.nn, self.s).T.reshape((self.s,) + self.shape).copy()

    def balpha(self):
        """b^alpha (Eq 84-85, per-axis, scaled basis): array [dim, s, *shape]."""
        out = np.empty(self.nn * self.dim * self.s)
        _load().orc_get_ba(self._h, out)
        a = out.reshape(self.nn, self.dim, self.s).transpose(1, 2, 0)
        return a.reshape((self.dim, self.s) + self.shape).copy()

    # --- operators ----------------------------------------------------------
    def _op(self, name, x):
        x = _f64(x).reshape(-1)
        out = np.empty(self.nn)
        getattr(_load(), name)(self._h, x, out)
        return out.reshape(self.shape)

    def apply_k(self, d):
        """Unmasked K d over the domain nodes (Eq 26 with nodal integration)."""
        return self._op("orc_apply_k", d)

    def apply_k_free(self, d, free):
        """chi_Omega o K (chi_Omega o d): the operator CG works with."""
        f = np.asarray(free).astype(bool)
        return np.where(f, self.apply_k(np.where(f, d, 0.0)), 0.0)

    def apply_fr(self, r):
        """Load vector f^r (Eq 59)."""
        return self._op("orc_apply_fr", r)

    def apply_nt(self, y):
        """N^T y."""
        return self._op("orc_apply_nt", y)

    def apply_uh(self, d):
        """u^h = N d at the nodes (Eq 62)."""
        return self._op("orc_apply_uh", d)

    def apply_vn(self, z):
        """V o N z."""
        return self._op("orc_apply_vn", z)

    def apply_b(self, d):
        """Implicit-gradient field B d: array [dim, *shape]."""
        x = _f64(d).reshape(-1)
        out = np.empty(self.nn * self.dim)
        _load().orc_apply_b(self._h, x, out)
        return out.reshape((self.dim,) + self.shape)

    def apply_k_at(self, d, idx):
        """(K d)_I at flat node indices idx only."""
        idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1)
        out = np.empty(idx.size)
        _load().orc_apply_k_at(self._h, _f64(d).reshape(-1), idx, idx.size, out)
        return out

    # --- solvers ------------------------------------------------------------
    def cg(self, free, rhs, x0=None, tol=1e-12, maxit=100000):
        free = np.ascontiguousarray(free, dtype=np.uint8).reshape(-1)
        x = np.zeros(self.nn) if x0 is None else _f64(x0).reshape(-1).copy()
        rel = C.c_double(0.0)
        it = _load().orc_cg(self._h, free, _f64(rhs).reshape(-1), x, tol, maxit,
                            C.byref(rel))
        return x.reshape(self.shape), it, rel.value

    def solve(self, free, dirichlet, r, g=None, x0=None, tol=1e-12, maxit=100000):
        """Strong-Dirichlet static solve; returns (d, iterations, rel. residual)."""
        free = np.ascontiguousarray(free, dtype=np.uint8).reshape(-1)
        dirm = np.ascontiguousarray(dirichlet, dtype=np.uint8).reshape(-1)
        d = np.zeros(self.nn) if x0 is None else _f64(x0).reshape(-1).copy()
        gg = None if g is None else _f64(g).reshape(-1)
        gptr = None if gg is None else gg.ctypes.data_as(C.c_void_p)
        rel = C.c_double(0.0)
        it = _load().orc_solve(self._h, free, dirm, _f64(r).reshape(-1), gptr, d,
                               tol, maxit, C.byref(rel))
        return d.reshape(self.shape), it, rel.value

    def adjoint(self, free, dl_du, tol=1e-12, maxit=100000):
        """dL/dr = V o N K_ff^-1 chi_Omega o N^T dL/du^h; returns (grad, z, its)."""
        free = np.ascontiguousarray(free, dtype=np.uint8).reshape(-1)
        g = np.empty(self.nn)
        z = np.empty(self.nn)
        rel = C.c_double(0.0)
        it = _load().orc_adjoint(self._h, free, _f64(dl_du).reshape(-1), g,
                                 z.ctypes.data_as(C.c_void_p), tol, maxit, C.byref(rel))
        return g.reshape(self.shape), z.reshape(self.shape), it

    # --- boundary flux (App. A) ---------------------------------------------
    def apply_fq(self, q, area):
        """Boundary load f^q_I = sum_S A_S q_S Psi_I(x_S) over the domain nodes
        (Eq 28 with direct nodal quadrature on the boundary, Eq A.2-A.3):
        N^T (A o q)."""
        return self.apply_nt(_f64(area).reshape(self.shape) * _f64(q).reshape(self.shape))

    def solve_flux(self, free, dirichlet, r, q, area, g=None, tol=1e-12, maxit=100000):
        """Static solve with a flux q on the boundary nodes of area A (Eq 8-9,
        28-29): K_ff x = chi_Omega (f^r + f^q - K d_G), d = x + d_G.  Returns
        (d, iterations, relative residual)."""
        f = np.asarray(free).reshape(self.shape).astype(bool)
        dG = np.zeros(self.shape)
        if g is not None:
            dG = np.where(np.asarray(dirichlet).reshape(self.shape).astype(bool),
                          _f64(g).reshape(self.shape), 0.0)
        rhs = np.where(f, self.apply_fr(r) + self.apply_fq(q, area) - self.apply_k(dG), 0.0)
        x, it, rel = self.cg(f.astype(np.uint8), rhs, tol=tol, maxit=maxit)
        return np.where(f, x, 0.0) + dG, it, rel

    # --- nonlinear problems (App. B) -----------------------------------------
    def apply_fn(self, d, kappa):
        """Nonlinear force f^N = int N^T N(u^h) dOmega with N(u) = kappa u^3
        under nodal integration (Eq B.2, B.4): N^T (V o kappa (N d)^3)."""
        u = self.apply_uh(d)
        return self.apply_fr(kappa * u ** 3)

    def apply_btv(self, g):
        """B^T (V o g) for a field g of shape [dim, *shape] (Eq B.6)."""
        out = np.empty(self.nn)
        _load().orc_apply_btv(self._h, _f64(g).reshape(-1), out)
        return out.reshape(self.shape)

    def apply_fn_grad(self, d, kappa):
        """Force of the gradient nonlinearity N(grad u) = (1 + kappa |grad u|^2)
        grad u under nodal integration (Eq B.5-B.8): B^T (V o N(B d))."""
        g = self.apply_b(d)
        return self.apply_btv((1.0 + kappa * (g ** 2).sum(axis=0)) * g)

    def solve_nonlinear(self, free, dirichlet, r, kappa, g=None, tol=1e-13, newton_tol=1e-11,
                        maxnewton=50, maxit=100000):
        """Static solve of -lap u + kappa u^3 = r (Eq 8 with the term of Eq B.1):
        R(d) = K d + f^N(d) - f^r = 0 on the free rows with d = g on the
        Dirichlet nodes, by Newton's method from d = d_G, each step solving
        (K + N^T diag(3 kappa V u^2) N) delta = -R on the free rows by CG to tol.
        Stops when ||R|| <= newton_tol ||chi_Omega f^r||.  Returns (d, Newton
        steps, CG iterations)."""
        f = np.asarray(free).reshape(self.shape).astype(bool)
        dG = np.zeros(self.shape)
        if g is not None:
            dG = np.where(np.asarray(dirichlet).reshape(self.shape).astype(bool),
                          _f64(g).reshape(self.shape), 0.0)
        fr = self.apply_fr(r)
        fn = float(np.linalg.norm(np.where(f, fr, 0.0)))
        d = dG.copy()
        its = 0
        for step in range(maxnewton + 1):
            u = self.apply_uh(d)
            R = np.where(f, self.apply_k(d) + self.apply_fr(kappa * u ** 3) - fr, 0.0)
            if float(np.linalg.norm(R)) <= newton_tol * fn or step == maxnewton:
                return d, step, its
            w = 3.0 * kappa * u ** 2

            def jac(v, w=w):
                return np.where(f, self.apply_k(v) + self.apply_fr(w * self.apply_uh(v)), 0.0)

            delta, k = _cg(jac, -R, np.zeros(self.shape), tol, maxit)
            its += k
            d = d + np.where(f, delta, 0.0)
        return d, maxnewton, its

    def solve_nonlinear_cg(self, free, dirichlet, r, kappa, kind="cubic", g=None, tol=1e-12,
                           maxit=100000, ls_tol=1e-14, ls_maxit=50):
        """Static nonlinear solve by nonlinear conjugate gradients (App. B.3,
        Alg B.3): from d = d_G, repeated evaluations of the nonlinear force
        update d until ||R(d)|| <= tol ||chi_Omega f^r|| on the free rows.

        kind "cubic":    R(d) = K d + N^T (V kappa (N d)^3) - f^r  (force of
                         Eq B.2/B.4 with N(u) = kappa u^3), the gradient of
                         Pi(d) = d^T K d / 2 + sum_S V_S kappa u_S^4 / 4 - f^r . d;
        kind "gradient": R(d) = B^T (V (1 + kappa |B d|^2) B d) - f^r  (force of
                         Eq B.6/B.8 with N(g) = (1 + kappa |g|^2) g), the gradient of
                         Pi(d) = sum_S V_S (|g_S|^2 / 2 + kappa |g_S|^4 / 4) - f^r . d.

        Both energies are convex for kappa >= 0, so the minimiser is unique.
        Directions are Polak-Ribiere with restarts (beta >= 0); the step along
        p minimises Pi exactly: phi'(alpha) = R(d + alpha p) . p is a sum of
        nodal terms in u + alpha w (w = N p) or g + alpha h (h = B p) plus a
        linear part, and Newton's method on it runs to ls_tol.  Returns (d,
        iterations, final ||R|| / ||chi_Omega f^r||)."""
        shape = self.shape
        f = np.asarray(free).reshape(shape).astype(bool)
        dom = self.chi > 0
        V = self._vol if self._vol is not None else np.where(dom, float(np.prod(self._hh)), 0.0)
        V = np.where(dom, V, 0.0)
        d = np.zeros(shape)
        if g is not None:
            d = np.where(np.asarray(dirichlet).reshape(shape).astype(bool), _f64(g).reshape(shape), 0.0)
        fr = self.apply_fr(r)
        fn = float(np.linalg.norm(np.where(f, fr, 0.0)))
        if fn == 0.0:
            return d, 0, 0.0
        if kind == "cubic":
            u = self.apply_uh(d)
            kd = self.apply_k(d)

            def resid():
                return np.where(f, kd + self.apply_fr(kappa * u ** 3) - fr, 0.0)
        elif kind == "gradient":
            gd = self.apply_b(d)

            def resid():
                return np.where(f, self.apply_btv((1.0 + kappa * (gd ** 2).sum(axis=0)) * gd) - fr, 0.0)
        else:
            raise ValueError("kind must be 'cubic' or 'gradient'")
        R = resid()
        rr = -R
        p = rr.copy()
        rn = float(np.vdot(rr, rr))
        for it in range(maxit + 1):
            if math.sqrt(rn) <= tol * fn or it == maxit:
                return d, it, math.sqrt(rn) / fn
            # exact line search along p: phi'(alpha) = 0
            if kind == "cubic":
                w = self.apply_uh(p)
                kp = self.apply_k(p)
                c0 = float(np.vdot(kd - fr, p))
                c1 = float(np.vdot(kp, p))

                def dphi(a):
                    ua = u + a * w
                    return (c0 + a * c1 + float(np.sum(V * kappa * ua ** 3 * w)),
                            c1 + float(np.sum(3.0 * V * kappa * ua ** 2 * w ** 2)))
            else:
                h = self.apply_b(p)
                c0 = -float(np.vdot(fr, p))

                def dphi(a):
                    ga = gd + a * h
                    s2 = (ga ** 2).sum(axis=0)
                    gh = (ga * h).sum(axis=0)
                    h2 = (h ** 2).sum(axis=0)
                    return (c0 + float(np.sum(V * (1.0 + kappa * s2) * gh)),
                            float(np.sum(V * ((1.0 + kappa * s2) * h2 + 2.0 * kappa * gh ** 2))))
            a = 0.0
            for _ in range(ls_maxit):
                d1, d2 = dphi(a)
                step = d1 / d2
                a -= step
                if abs(step) <= ls_tol * abs(a):
                    break
            d = d + a * p
            if kind == "cubic":
                u = u + a * w
                kd = kd + a * kp
            else:
                gd = gd + a * h
            rr_new = -resid()
            rn_new = float(np.vdot(rr_new, rr_new))
            beta = max(0.0, float(np.vdot(rr_new, rr_new - rr)) / rn)
            p = rr_new + beta * p
            rr, rn = rr_new, rn_new
        return d, maxit, math.sqrt(rn) / fn

    # --- time-dependent problems (App. C) -----------------------------------
    def apply_m(self, d):
        """Consistent mass product f^m = M d with M = int N^T N dOmega under
        direct nodal integration (Eq C.5, C.7): N^T (V o N d), i.e.
        f_I = sum_K V_K Psi_I(x_K) sum_J Psi_J(x_K) d_J over domain nodes."""
        return self.apply_fr(self.apply_uh(d))

    def lumped_mass(self):
        """Lumped mass M^l_II = sum_P M_IP (Eq C.9): M applied to ones on the
        domain nodes."""
        return self.apply_m(self.chi.astype(np.float64))

    def transient(self, free, dirichlet, d0, nu, dt, nsteps, r=None, g=None,
                  scheme="implicit", theta=1.0, tol=1e-13, maxit=100000):
        """Time stepping of M d' + nu K d = f^r (Eq C.1-C.4) with d = g held on
        the Dirichlet nodes and r constant in time.

        scheme "implicit" (Alg C.4): the theta method on the free rows,
            (M + theta dt nu K) x1 = (M - (1-theta) dt nu K) x0 + dt (f^r - nu K d_G),
          each step solved by CG from x0 to a relative residual of tol;
          theta = 1 is backward Euler, theta = 1/2 Crank-Nicolson.
        scheme "explicit" (Alg C.3): forward Euler with the lumped mass,
            x1 = x0 + dt (f^r - nu K (x0 + d_G)) / M^l  on the free rows.
        Returns (d at t = nsteps dt, CG iterations summed over the steps)."""
        shape = self.shape
        f = np.asarray(free).reshape(shape).astype(bool)
        dG = np.zeros(shape)
        if g is not None:
            dG = np.where(np.asarray(dirichlet).reshape(shape).astype(bool),
                          _f64(g).reshape(shape), 0.0)
        fr = self.apply_fr(r) if r is not None else np.zeros(shape)
        c0 = np.where(f, dt * (fr - nu * self.apply_k(dG)), 0.0)
        x = np.where(f, _f64(d0).reshape(shape), 0.0)
        its = 0
        if scheme == "explicit":
            ml = self.lumped_mass()
            for _ in range(nsteps):
                x = np.where(f, x + (c0 - dt * nu * self.apply_k(x)) / np.where(f, ml, 1.0), 0.0)
            return x + dG, 0
        if scheme != "implicit" or not (0.0 < theta <= 1.0):
            raise ValueError("scheme must be 'implicit' (0 < theta <= 1) or 'explicit'")

        def op(v):
            return np.where(f, self.apply_m(v) + theta * dt * nu * self.apply_k(v), 0.0)

        for _ in range(nsteps):
            rhs = self.apply_m(x)
            if theta < 1.0:
                rhs = rhs - (1.0 - theta) * dt * nu * self.apply_k(x)
            b = np.where(f, rhs, 0.0) + c0
            x, k = _cg(op, b, x.copy(), tol, maxit)
            its += k
        return x + dG, its


def _cg(op, b, x, tol, maxit):
    """Plain conjugate gradients on a symmetric positive definite operator,
    stopping when ||b - A x|| (recursive) <= tol ||b||."""
    bn = math.sqrt(float(np.vdot(b, b)))
    if bn == 0.0:
        return np.zeros_like(b), 0
    r = b - op(x)
    p = r.copy()
    rr = float(np.vdot(r, r))
    for it in range(maxit):
        if math.sqrt(rr) <= tol * bn:
            return x, it
        q = op(p)
        alpha = rr / float(np.vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        rr1 = float(np.vdot(r, r))
        p = r + (rr1 / rr) * p
        rr = rr1
    return x, maxit
