"""Python binding of the gfx950 FC-RKPM library (libfcrkpm.so).

Argument marshalling only: every step of the method runs in the HIP library
behind the C ABI of ``include/fcrkpm.h``.  Torch is used for device memory and
the current stream.  If the shared library is missing this module raises; it
has no CPU fallback.

Arrays are torch tensors on a HIP device in C order ``[nz][ny][nx]`` (x
fastest); masks are uint8, fields float64 (or float32 for FP32 applies).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfcrkpm.so")

OK, ERR_ARG, ERR_SINGULAR, ERR_NOCONV, ERR_HIP, ERR_OOM, ERR_UNSUPPORTED = range(7)
OP_K, OP_K_FULL, OP_FR, OP_UH, OP_NT, OP_VN, OP_M, OP_FQ = range(8)
F64, F32 = 0, 1
MODE_F64, MODE_F32_REFINED, MODE_F32_PRODUCTS = 0, 1, 2
COEF_B0, COEF_BALPHA, COEF_FREE, COEF_LUMPED_MASS = 0, 1, 2, 3
TIME_IMPLICIT, TIME_EXPLICIT_LUMPED = 0, 1
NONLIN_CUBIC, NONLIN_GRADIENT = 0, 1
KERNEL_CUBIC_BSPLINE = 0

_OPS = {"K": OP_K, "K_FULL": OP_K_FULL, "FR": OP_FR, "UH": OP_UH, "NT": OP_NT, "VN": OP_VN,
        "M": OP_M, "FQ": OP_FQ}
_MODES = {"f64": MODE_F64, "f32_refined": MODE_F32_REFINED, "f32_products": MODE_F32_PRODUCTS}

EXPORTS = ("fcrkpm_setup", "fcrkpm_apply", "fcrkpm_solve", "fcrkpm_adjoint",
           "fcrkpm_get_coeffs", "fcrkpm_basis_size", "fcrkpm_destroy",
           "fcrkpm_last_error", "fcrkpm_status_str", "fcrkpm_version",
           "fcrkpm_profile", "fcrkpm_profile_read", "fcrkpm_kernel_kinds",
           "fcrkpm_kernel_name", "fcrkpm_solve_batch", "fcrkpm_set_option",
           "fcrkpm_get_option", "fcrkpm_transient", "fcrkpm_set_boundary",
           "fcrkpm_solve_flux", "fcrkpm_nonlinear_force", "fcrkpm_solve_nonlinear",
           "fcrkpm_gradient_force", "fcrkpm_apply_noalloc", "fcrkpm_solve_nonlinear_cg")
OPT_GRAPHS = 1
OPT_REGPATH = 2
OPT_REGLAYOUT = 3
OPT_TUNE_NS0 = 4
OPT_TUNE_NS1 = 5
OPT_TUNE_NS2 = 6
OPT_TUNE_NS3 = 7
OPT_LINECONST = 8
OPT_SEP_LINES32 = 9
OPT_SEP_LINES64 = 10
OPT_TUNE_CACHED = 11
OPT_KN_REGPATH = 12


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3),
                ("dirichlet", C.c_void_p), ("vol", C.c_void_p), ("flags", C.c_int32)]


class Time(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("nsteps", C.c_int32), ("dt", C.c_double),
                ("nu", C.c_double), ("theta", C.c_double)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_iters", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("fallback_used", C.c_int32),
                ("matvecs_f64", C.c_int32), ("matvecs_f32", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _infos_dict(infos, status):
    """Aggregate of per-rhs records (worst case; the rhs iterate in lockstep)
    with the records themselves under "per_rhs"."""
    per = [i.as_dict() for i in infos]
    out = {"iters": max(d["iters"] for d in per),
           "outer_iters": max(d["outer_iters"] for d in per),
           "rel_res": max(d["rel_res"] for d in per),
           "true_rel_res": max(d["true_rel_res"] for d in per),
           "fallback_used": int(any(d["fallback_used"] for d in per)),
           "matvecs_f64": max(d["matvecs_f64"] for d in per),
           "matvecs_f32": max(d["matvecs_f32"] for d in per),
           "status": status, "per_rhs": per}
    return out


class FcrkpmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = None):
    """Load libfcrkpm.so (raises if it has not been built).  FCRKPM_LIB names
    another build of it (the host-sanitized one, for CPU checks)."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = os.environ.get("FCRKPM_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the FC-RKPM path has no CPU fallback)")
    lib = C.CDLL(path)
    V = C.c_void_p
    lib.fcrkpm_setup.restype = C.c_int
    lib.fcrkpm_setup.argtypes = [C.POINTER(Grid), V, C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                 V, C.POINTER(V)]
    lib.fcrkpm_apply.restype = C.c_int
    lib.fcrkpm_apply.argtypes = [V, C.c_int32, C.c_int32, C.c_int32, V, V, V]
    lib.fcrkpm_apply_noalloc.restype = C.c_int
    lib.fcrkpm_apply_noalloc.argtypes = [V, C.c_int32, C.c_int32, C.c_int32, V, V, V]
    lib.fcrkpm_solve.restype = C.c_int
    lib.fcrkpm_solve.argtypes = [V, C.c_int32, C.c_int32, V, V, V, V, C.c_double, C.c_int32,
                                 C.POINTER(Info), V]
    lib.fcrkpm_adjoint.restype = C.c_int
    lib.fcrkpm_adjoint.argtypes = [V, C.c_int32, C.c_int32, V, V, C.c_double, C.c_int32,
                                   C.POINTER(Info), V]
    lib.fcrkpm_get_coeffs.restype = C.c_int
    lib.fcrkpm_get_coeffs.argtypes = [V, C.c_int32, V, V]
    lib.fcrkpm_set_boundary.restype = C.c_int
    lib.fcrkpm_set_boundary.argtypes = [V, V, V]
    lib.fcrkpm_solve_flux.restype = C.c_int
    lib.fcrkpm_solve_flux.argtypes = [V, C.c_int32, C.c_int32, V, V, V, V, V, C.c_double,
                                      C.c_int32, C.POINTER(Info), V]
    lib.fcrkpm_nonlinear_force.restype = C.c_int
    lib.fcrkpm_nonlinear_force.argtypes = [V, C.c_double, C.c_int32, V, V, V]
    lib.fcrkpm_gradient_force.restype = C.c_int
    lib.fcrkpm_gradient_force.argtypes = [V, C.c_double, C.c_int32, V, V, V]
    lib.fcrkpm_solve_nonlinear.restype = C.c_int
    lib.fcrkpm_solve_nonlinear.argtypes = [V, C.c_int32, C.c_double, V, V, V, V, C.c_double,
                                           C.c_double, C.c_int32, C.c_int32, C.POINTER(Info), V]
    lib.fcrkpm_solve_nonlinear_cg.restype = C.c_int
    lib.fcrkpm_solve_nonlinear_cg.argtypes = [V, C.c_int32, C.c_double, V, V, V, V, C.c_double,
                                              C.c_int32, C.POINTER(Info), V]
    lib.fcrkpm_transient.restype = C.c_int
    lib.fcrkpm_transient.argtypes = [V, C.POINTER(Time), C.c_int32, C.c_int32, V, V, V, V,
                                     C.c_double, C.c_int32, C.POINTER(Info), V]
    lib.fcrkpm_basis_size.restype = C.c_int32
    lib.fcrkpm_basis_size.argtypes = [V]
    lib.fcrkpm_destroy.restype = None
    lib.fcrkpm_destroy.argtypes = [V]
    lib.fcrkpm_last_error.restype = C.c_char_p
    lib.fcrkpm_last_error.argtypes = [V]
    lib.fcrkpm_status_str.restype = C.c_char_p
    lib.fcrkpm_status_str.argtypes = [C.c_int]
    lib.fcrkpm_version.restype = C.c_int32
    lib.fcrkpm_version.argtypes = []
    lib.fcrkpm_profile.restype = C.c_int
    lib.fcrkpm_profile.argtypes = [V, C.c_int32]
    lib.fcrkpm_profile_read.restype = C.c_int
    lib.fcrkpm_profile_read.argtypes = [V, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
    lib.fcrkpm_kernel_kinds.restype = C.c_int32
    lib.fcrkpm_kernel_kinds.argtypes = []
    lib.fcrkpm_kernel_name.restype = C.c_char_p
    lib.fcrkpm_kernel_name.argtypes = [C.c_int32]
    lib.fcrkpm_solve_batch.restype = C.c_int
    lib.fcrkpm_solve_batch.argtypes = [C.POINTER(V), C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(V), C.POINTER(V), C.POINTER(V), C.POINTER(V),
                                       C.c_double, C.c_int32, C.POINTER(Info), V]
    lib.fcrkpm_set_option.restype = C.c_int
    lib.fcrkpm_set_option.argtypes = [V, C.c_int32, C.c_int64]
    lib.fcrkpm_get_option.restype = C.c_int
    lib.fcrkpm_get_option.argtypes = [V, C.c_int32, C.POINTER(C.c_int64)]
    _lib = lib
    return lib


def status_name(s: int) -> str:
    try:
        return load_library().fcrkpm_status_str(int(s)).decode()
    except Exception:
        return f"status {s}"


def _stream_ptr(stream=None):
    st = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(st.cuda_stream)


def _dev(x, dtype, device):
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x))
    return x.to(device=device, dtype=dtype).contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_out(out, like):
    """A caller-supplied output goes to the library as a raw pointer, so it must
    match the input exactly: dtype, device, contiguity and element count."""
    if not isinstance(out, torch.Tensor):
        raise TypeError("out must be a torch tensor")
    if out.dtype != like.dtype:
        raise ValueError(f"out has dtype {out.dtype}, expected {like.dtype}")
    if out.device != like.device:
        raise ValueError(f"out is on {out.device}, expected {like.device}")
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    if out.numel() != like.numel():
        raise ValueError(f"out holds {out.numel()} values, expected {like.numel()}")
    return out


class Problem:
    """One FC-RKPM context: a box grid, a domain and its RK coefficients.

    dims: box nodes per active axis (x, y, z order); h, support: per axis;
    degree: 1 or 2; mask/dirichlet: uint8 [nz][ny][nx]; vol: float64 or None.
    """

    def __init__(self, dims, h, support, degree, mask, dirichlet=None, vol=None, device="cuda",
                 stream=None):
        lib = load_library()
        self.device = torch.device(device)
        self.dim = len(dims)
        self.dims = tuple(int(v) for v in dims)
        self.shape = tuple(reversed(self.dims))
        self.nn = int(np.prod(self.dims))
        self._mask = _dev(mask, torch.uint8, self.device).reshape(self.shape)
        self._dir = None if dirichlet is None else _dev(dirichlet, torch.uint8, self.device).reshape(self.shape)
        self._vol = None if vol is None else _dev(vol, torch.float64, self.device).reshape(self.shape)
        g = Grid()
        g.dim = self.dim
        for k in range(3):
            g.n[k] = self.dims[k] if k < self.dim else 1
            g.h[k] = float(h[k]) if k < self.dim else 1.0
        g.dirichlet = _ptr(self._dir)
        g.vol = _ptr(self._vol)
        g.flags = 0
        sup = (C.c_double * 3)(*[float(support[k]) if k < self.dim else 0.0 for k in range(3)])
        h_ = C.c_void_p()
        st = lib.fcrkpm_setup(C.byref(g), _ptr(self._mask), KERNEL_CUBIC_BSPLINE, sup, int(degree),
                              _stream_ptr(stream), C.byref(h_))
        if st != OK:
            raise FcrkpmError(st, lib.fcrkpm_last_error(None).decode())
        self._h = h_
        self.s = lib.fcrkpm_basis_size(self._h)

    @classmethod
    def from_workload(cls, p, device="cuda"):
        """Build from a ``workloads.Problem``."""
        return cls(p.dims, p.h, p.at, p.degree, p.chi, p.dirichlet, p.vol, device=device)

    def close(self):
        if getattr(self, "_h", None):
            load_library().fcrkpm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise FcrkpmError(st, load_library().fcrkpm_last_error(self._h).decode())

    # ------------------------------------------------------------------ ops
    def apply(self, op, x, out=None, stream=None):
        """Apply operator op ('K', 'K_FULL', 'FR', 'UH', 'NT', 'VN', 'M', 'FQ') to x.

        x: float64 or float32 tensor of shape [..., nz, ny, nx]; leading
        dimensions are independent fields.  The precision of x selects the
        arithmetic."""
        opc = _OPS[op] if isinstance(op, str) else int(op)
        if x.dtype not in (torch.float64, torch.float32):
            raise TypeError("x must be float64 or float32")
        x = x.contiguous()
        if x.device != self.device:
            x = x.to(self.device)
        nrhs = x.numel() // self.nn
        if nrhs * self.nn != x.numel() or nrhs < 1:
            raise ValueError("x does not hold whole fields")
        if out is None:
            out = torch.empty_like(x)
        else:
            _check_out(out, x)
        self._check(load_library().fcrkpm_apply(
            self._h, opc, F64 if x.dtype == torch.float64 else F32, nrhs, _ptr(x), _ptr(out),
            _stream_ptr(stream)))
        return out

    def apply_noalloc(self, op, x, out, stream=None):
        """apply() for callers that cannot allocate: the library keeps the
        intermediate fields in its static per-GPU scratch (64 MiB) and
        allocates nothing.  `out` must be given (same dtype, device and size as
        x); calls that overlap in time on one GPU race."""
        opc = _OPS[op] if isinstance(op, str) else int(op)
        if x.dtype not in (torch.float64, torch.float32):
            raise TypeError("x must be float64 or float32")
        if x.device != self.device or not x.is_contiguous():
            raise ValueError("x must be a contiguous tensor on the problem's device")
        nrhs = x.numel() // self.nn
        if nrhs * self.nn != x.numel() or nrhs < 1:
            raise ValueError("x does not hold whole fields")
        _check_out(out, x)
        self._check(load_library().fcrkpm_apply_noalloc(
            self._h, opc, F64 if x.dtype == torch.float64 else F32, nrhs, _ptr(x), _ptr(out),
            _stream_ptr(stream)))
        return out

    def set_boundary(self, area=None, stream=None):
        """Boundary areas A of the flux nodes (None removes them)."""
        a = None if area is None else _dev(area, torch.float64, self.device)
        if a is not None and a.numel() != self.nn:
            raise ValueError("area must hold one value per node")
        self._check(load_library().fcrkpm_set_boundary(self._h, _ptr(a), _stream_ptr(stream)))

    def solve(self, r, g=None, d0=None, mode="f64", tol=1e-12, maxit=20000, want_uh=True,
              stream=None, raise_on_noconv=True, q=None):
        """Strong-Dirichlet static solve of one or more right-hand sides (leading
        dimensions of r), with a boundary flux q on the areas of set_boundary
        when q is given; returns (d, u^h or None, info dict)."""
        r = _dev(r, torch.float64, self.device)
        nrhs = r.numel() // self.nn
        if nrhs < 1 or nrhs * self.nn != r.numel():
            raise ValueError("r does not hold whole fields")
        g = None if g is None else _dev(g, torch.float64, self.device)
        d = torch.zeros_like(r) if d0 is None else _dev(d0, torch.float64, self.device).clone()
        uh = torch.empty_like(r) if want_uh else None
        infos = (Info * nrhs)()
        if q is not None:
            q = _dev(q, torch.float64, self.device).expand_as(r).contiguous()
            st = load_library().fcrkpm_solve_flux(self._h, _MODES[mode], nrhs, _ptr(r), _ptr(q),
                                                  _ptr(g), _ptr(d), _ptr(uh), float(tol),
                                                  int(maxit), infos, _stream_ptr(stream))
        else:
            st = load_library().fcrkpm_solve(self._h, _MODES[mode], nrhs, _ptr(r), _ptr(g),
                                             _ptr(d), _ptr(uh), float(tol), int(maxit), infos,
                                             _stream_ptr(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            self._check(st)
        return d, uh, _infos_dict(infos, st)

    def adjoint(self, dl_duh, mode="f64", tol=1e-12, maxit=20000, stream=None):
        """dL/dr for a loss of u^h; returns (dL/dr, info dict)."""
        y = _dev(dl_duh, torch.float64, self.device)
        nrhs = y.numel() // self.nn
        if nrhs < 1 or nrhs * self.nn != y.numel():
            raise ValueError("dl_duh does not hold whole fields")
        g = torch.empty_like(y)
        infos = (Info * nrhs)()
        self._check(load_library().fcrkpm_adjoint(self._h, _MODES[mode], nrhs, _ptr(y), _ptr(g),
                                                  float(tol), int(maxit), infos,
                                                  _stream_ptr(stream)))
        return g, _infos_dict(infos, OK)

    def transient(self, d0, nu, dt, nsteps, r=None, g=None, scheme="implicit", theta=1.0,
                  mode="f64", tol=1e-12, maxit=20000, want_uh=False, stream=None,
                  raise_on_noconv=True):
        """Time stepping of M d' + nu K d = f^r from d0 (leading dimensions of
        d0 are independent fields); scheme 'implicit' (theta method) or
        'explicit' (forward Euler, lumped mass).  Returns (d, u^h or None,
        info dict)."""
        d = _dev(d0, torch.float64, self.device).clone()
        nrhs = d.numel() // self.nn
        if nrhs < 1 or nrhs * self.nn != d.numel():
            raise ValueError("d0 does not hold whole fields")
        r = None if r is None else _dev(r, torch.float64, self.device).expand_as(d).contiguous()
        g = None if g is None else _dev(g, torch.float64, self.device).expand_as(d).contiguous()
        uh = torch.empty_like(d) if want_uh else None
        tp = Time(TIME_IMPLICIT if scheme == "implicit" else
                  TIME_EXPLICIT_LUMPED if scheme == "explicit" else -1,
                  int(nsteps), float(dt), float(nu), float(theta))
        infos = (Info * nrhs)()
        st = load_library().fcrkpm_transient(self._h, C.byref(tp), _MODES[mode], nrhs, _ptr(r),
                                             _ptr(g), _ptr(d), _ptr(uh), float(tol), int(maxit),
                                             infos, _stream_ptr(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            self._check(st)
        return d, uh, _infos_dict(infos, st)

    def nonlinear_force(self, d, kappa, out=None, stream=None):
        """f^N = N^T (V o kappa (N d)^3) for one or more fields d (FP64)."""
        d = _dev(d, torch.float64, self.device)
        nrhs = d.numel() // self.nn
        if nrhs < 1 or nrhs * self.nn != d.numel():
            raise ValueError("d does not hold whole fields")
        if out is None:
            out = torch.empty_like(d)
        else:
            _check_out(out, d)
        self._check(load_library().fcrkpm_nonlinear_force(self._h, float(kappa), nrhs, _ptr(d),
                                                          _ptr(out), _stream_ptr(stream)))
        return out

    def gradient_force(self, d, kappa, out=None, stream=None):
        """f^N = B^T (V o (1 + kappa |B d|^2) B d) for one or more fields d (FP64)."""
        d = _dev(d, torch.float64, self.device)
        nrhs = d.numel() // self.nn
        if nrhs < 1 or nrhs * self.nn != d.numel():
            raise ValueError("d does not hold whole fields")
        if out is None:
            out = torch.empty_like(d)
        else:
            _check_out(out, d)
        self._check(load_library().fcrkpm_gradient_force(self._h, float(kappa), nrhs, _ptr(d),
                                                         _ptr(out), _stream_ptr(stream)))
        return out

    def solve_nonlinear(self, r, kappa, g=None, d0=None, mode="f64", tol=1e-12,
                        newton_tol=1e-10, maxnewton=30, maxit=20000, want_uh=True, stream=None,
                        raise_on_noconv=True):
        """-lap u + kappa u^3 = r by Newton's method (one field); returns
        (d, u^h or None, info dict with outer_iters = Newton steps)."""
        r = _dev(r, torch.float64, self.device)
        if r.numel() != self.nn:
            raise ValueError("r must hold one field")
        g = None if g is None else _dev(g, torch.float64, self.device)
        d = torch.zeros_like(r) if d0 is None else _dev(d0, torch.float64, self.device).clone()
        uh = torch.empty_like(r) if want_uh else None
        info = (Info * 1)()
        st = load_library().fcrkpm_solve_nonlinear(self._h, _MODES[mode], float(kappa), _ptr(r),
                                                   _ptr(g), _ptr(d), _ptr(uh), float(tol),
                                                   float(newton_tol), int(maxnewton), int(maxit),
                                                   info, _stream_ptr(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            self._check(st)
        return d, uh, _infos_dict(info, st)

    def solve_nonlinear_cg(self, r, kappa, kind="cubic", g=None, d0=None, tol=1e-12, maxit=100000,
                           want_uh=True, stream=None, raise_on_noconv=True):
        """The static nonlinear problem by nonlinear CG (Alg B.3) with the force
        of kind 'cubic' (kappa u^3) or 'gradient' ((1 + kappa |grad u|^2) grad u);
        one field.  Returns (d, u^h or None, info dict: iters = CG iterations,
        outer_iters = line-search steps)."""
        r = _dev(r, torch.float64, self.device)
        if r.numel() != self.nn:
            raise ValueError("r must hold one field")
        g = None if g is None else _dev(g, torch.float64, self.device)
        d = torch.zeros_like(r) if d0 is None else _dev(d0, torch.float64, self.device).clone()
        uh = torch.empty_like(r) if want_uh else None
        code = {"cubic": NONLIN_CUBIC, "gradient": NONLIN_GRADIENT}[kind]
        info = (Info * 1)()
        st = load_library().fcrkpm_solve_nonlinear_cg(self._h, code, float(kappa), _ptr(r), _ptr(g),
                                                      _ptr(d), _ptr(uh), float(tol), int(maxit), info,
                                                      _stream_ptr(stream))
        if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
            self._check(st)
        return d, uh, _infos_dict(info, st)

    def set_regpath(self, on: bool):
        """Use the register-resident FP32 K passes where they apply (default)."""
        self._check(load_library().fcrkpm_set_option(self._h, OPT_REGPATH, 1 if on else 0))

    def set_option(self, option: int, value: int):
        self._check(load_library().fcrkpm_set_option(self._h, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = C.c_int64()
        self._check(load_library().fcrkpm_get_option(self._h, int(option), C.byref(v)))
        return v.value

    def set_graphs(self, on: bool):
        """Replay CG blocks from captured HIP graphs (default) or launch directly."""
        self._check(load_library().fcrkpm_set_option(self._h, OPT_GRAPHS, 1 if on else 0))

    def coeffs(self, which="b0"):
        """Copy of b^0 [s, *shape], b^alpha [dim, s, *shape], chi_Omega [*shape]
        or the lumped mass M^l [*shape] ('lumped')."""
        code = {"b0": COEF_B0, "balpha": COEF_BALPHA, "free": COEF_FREE,
                "lumped": COEF_LUMPED_MASS}[which]
        shape = {"b0": (self.s,) + self.shape, "balpha": (self.dim, self.s) + self.shape,
                 "free": self.shape, "lumped": self.shape}[which]
        out = torch.empty(shape, dtype=torch.float64, device=self.device)
        self._check(load_library().fcrkpm_get_coeffs(self._h, code, _ptr(out), _stream_ptr()))
        return out


    # ------------------------------------------------------------ measurement
    def profile(self, enable: bool):
        """Open (True) or close (False) a kernel-duration sampling window."""
        self._check(load_library().fcrkpm_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{kernel name: (launches, mean ms of sampled launches, bytes per launch)}."""
        lib = load_library()
        out = {}
        for k in range(lib.fcrkpm_kernel_kinds()):
            n = C.c_int64()
            ms = C.c_double()
            by = C.c_double()
            self._check(lib.fcrkpm_profile_read(self._h, k, C.byref(n), C.byref(ms), C.byref(by)))
            if n.value:
                out[lib.fcrkpm_kernel_name(k).decode()] = (n.value, ms.value, by.value)
        return out


def solve_batch(problems, rs, gs=None, mode="f32_refined", tol=1e-12, maxit=20000,
                want_uh=True, stream=None, raise_on_noconv=True):
    """Ragged batch: problem p (its own box) with right-hand sides rs[p]; all
    problems iterate together (fcrkpm_solve_batch).  Returns a list of
    (d, u^h or None, info dict) per problem and the batch status."""
    n = len(problems)
    if n < 1 or len(rs) != n:
        raise ValueError("one r per problem")
    rr, gg, dd, uu, nr = [], [], [], [], []
    for p, r, g in zip(problems, rs, gs if gs is not None else [None] * n):
        r = _dev(r, torch.float64, p.device)
        k = r.numel() // p.nn
        if k < 1 or k * p.nn != r.numel():
            raise ValueError("r does not hold whole fields")
        rr.append(r)
        gg.append(None if g is None else _dev(g, torch.float64, p.device))
        dd.append(torch.zeros_like(r))
        uu.append(torch.empty_like(r) if want_uh else None)
        nr.append(k)
    V = C.c_void_p
    arr = lambda ts: (V * n)(*[t.data_ptr() if t is not None else None for t in ts])
    ctxs = (V * n)(*[p._h for p in problems])
    infos = (Info * sum(nr))()
    st = load_library().fcrkpm_solve_batch(ctxs, n, _MODES[mode], (C.c_int32 * n)(*nr), arr(rr),
                                           arr(gg) if gs is not None else None, arr(dd),
                                           arr(uu) if want_uh else None, float(tol), int(maxit),
                                           infos, _stream_ptr(stream))
    if st != OK and not (st == ERR_NOCONV and not raise_on_noconv):
        problems[0]._check(st)
    out, off = [], 0
    for p in range(n):
        out.append((dd[p], uu[p], _infos_dict(infos[off:off + nr[p]], st)))
        off += nr[p]
    return out, st


class FCRKPMSolve(torch.autograd.Function):
    """u^h(r): forward = strong-Dirichlet solve, backward = adjoint solve."""

    @staticmethod
    def forward(ctx, r, problem: Problem, mode: str = "f64", tol: float = 1e-12,
                maxit: int = 20000):
        _, uh, _ = problem.solve(r.detach(), mode=mode, tol=tol, maxit=maxit, want_uh=True)
        ctx.problem, ctx.mode, ctx.tol, ctx.maxit = problem, mode, tol, maxit
        return uh

    @staticmethod
    def backward(ctx, grad_uh):
        g, _ = ctx.problem.adjoint(grad_uh.contiguous(), mode=ctx.mode, tol=ctx.tol,
                                   maxit=ctx.maxit)
        return g, None, None, None, None


@dataclass
class Version:
    code: int

    def __str__(self):
        return f"{self.code // 10000}.{self.code // 100 % 100}.{self.code % 100}"


def version() -> Version:
    return Version(load_library().fcrkpm_version())
