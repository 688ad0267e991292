"""Seeded synthetic inputs for the FC-RKPM Poisson path.

This module builds the inputs that the paper's static solver reads (Sec 5.4.3,
Alg 5 "Read inputs"): the box grid, the domain mask chi (Eq 40), the Dirichlet
mask chi_Gamma_g (Eq 95), the free-node mask chi_Omega = chi - chi_Gamma_g
(Eq 96), the nodal volumes V (Eq 87) and the source r (Eq 8).  It holds none of
the method's arithmetic (no kernels, moments, shape functions or transforms),
so both the GPU library and the CPU oracle can be fed from it.

Conventions
-----------
* Arrays are numpy, C order ``[nz][ny][nx]`` (x fastest); masks are uint8.
* ``dims`` lists box nodes per active axis in (x, y, z) order.
* A cube domain [lo, hi]^d is embedded in a periodic box of N nodes per axis
  as in Sec 5.1 (Eq 64-67): m = floor(at), h = (hi - lo) / (N - m - 1), the
  domain holds indices 0 .. N-m-1, and the last m box nodes are the extension.
* Cube volumes use the 1D trapezoid weight (1/2 on each face index) per axis;
  the sphere uses h^3 on every domain node.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    name: str
    dim: int
    dims: tuple
    h: tuple
    at: tuple
    degree: int
    chi: np.ndarray
    dirichlet: np.ndarray
    free: np.ndarray
    vol: np.ndarray
    r: np.ndarray
    coords: tuple                      # per-axis 1D node coordinates
    u_exact: Optional[np.ndarray] = None
    g: Optional[np.ndarray] = None     # Dirichlet values (None = homogeneous)
    meta: dict = field(default_factory=dict)
    area: Optional[np.ndarray] = None  # boundary areas A of the flux nodes (Gamma_q)
    q: Optional[np.ndarray] = None     # flux grad u . n on the flux nodes

    @property
    def shape(self):
        return tuple(reversed(self.dims))

    @property
    def nn(self):
        return int(np.prod(self.dims))

    @property
    def n_domain(self):
        return int(self.chi.sum())

    @property
    def n_free(self):
        return int(self.free.sum())


def _mesh(coords):
    """Coordinate arrays X, Y, Z (Eq 71) in [nz][ny][nx] order."""
    rev = [np.asarray(c) for c in reversed(coords)]
    grids = np.meshgrid(*rev, indexing="ij")
    return list(reversed(grids))           # x, y, z


def cube(dim: int, n_box: int, at: float, degree: int, lo: float = 0.0,
         hi: float = 1.0, source: str = "sin", name: str = "cube") -> Problem:
    """Cube domain [lo, hi]^dim embedded in an n_box^dim periodic box.

    source: 'sin'   u = prod sin(pi (x-lo)/(hi-lo)), r = -lap u
            'eq97'  1D, u = 1 - x^2, r = 2               (Eq 97-98)
            'eq101' 2D, u = (1-x^2)(1-y^2)              (Eq 101-102)
            'eq106' 3D, u = (1-x^2)(1-y^2)(1-z^2)       (Eq 106-107)
            'linear' u = 1 + sum_k (k+1) x_k, r = 0 (patch test)
            'zero'  r = 0
    Dirichlet nodes are the domain nodes on a face of the cube.
    """
    m = int(math.floor(at))
    n_om = n_box - m                    # domain nodes per axis
    if n_om < 3:
        raise ValueError("box too small for the support")
    h = (hi - lo) / (n_om - 1)
    dims = (n_box,) * dim
    coords = tuple(lo + h * np.arange(n_box) for _ in range(dim))
    idx = [np.arange(n_box) for _ in range(dim)]
    inside1 = [(i <= n_om - 1).astype(np.uint8) for i in idx]
    face1 = [((i == 0) | (i == n_om - 1)).astype(np.uint8) for i in idx]
    w1 = [np.where(i <= n_om - 1, np.where((i == 0) | (i == n_om - 1), 0.5, 1.0), 0.0)
          for i in idx]

    def outer(vs, op):
        out = vs[0]
        for v in vs[1:]:
            out = op.outer(v, out)       # later axes are slower
        return out

    chi = outer(inside1, np.multiply).astype(np.uint8).reshape(tuple(reversed(dims)))
    onface = outer(face1, np.maximum).astype(np.uint8).reshape(chi.shape)
    dirichlet = (chi & onface).astype(np.uint8)
    free = (chi - dirichlet).astype(np.uint8)
    vol = outer(w1, np.multiply).reshape(chi.shape) * h ** dim

    X = _mesh(coords)
    L = hi - lo
    u = None
    if source == "sin":
        u = np.ones(chi.shape)
        for k in range(dim):
            u = u * np.sin(math.pi * (X[k] - lo) / L)
        r = dim * (math.pi / L) ** 2 * u
    elif source == "eq97":
        assert dim == 1
        u = 1.0 - X[0] ** 2
        r = 2.0 * np.ones(chi.shape)
    elif source == "eq101":
        assert dim == 2
        x, y = X
        u = (1 - x ** 2) * (1 - y ** 2)
        r = 4.0 - 2 * x ** 2 - 2 * y ** 2
    elif source == "eq106":
        assert dim == 3
        x, y, z = X
        u = (1 - x ** 2) * (1 - y ** 2) * (1 - z ** 2)
        r = 2.0 * (3 - 2 * (x ** 2 + y ** 2 + z ** 2) + x ** 2 * y ** 2
                   + x ** 2 * z ** 2 + y ** 2 * z ** 2)
    elif source == "linear":
        u = np.ones(chi.shape)
        for k in range(dim):
            u = u + (k + 1) * X[k]
        r = np.zeros(chi.shape)
    elif source == "zero":
        r = np.zeros(chi.shape)
    else:
        raise ValueError(source)
    r = np.where(chi > 0, r, 0.0)
    if u is not None:
        u = np.where(chi > 0, u, 0.0)
    g = None
    if source == "linear":
        g = np.where(dirichlet > 0, u, 0.0)
    return Problem(name=name, dim=dim, dims=dims, h=(h,) * dim, at=(float(at),) * dim,
                   degree=degree, chi=chi, dirichlet=dirichlet, free=free,
                   vol=np.ascontiguousarray(vol), r=np.ascontiguousarray(r),
                   coords=coords, u_exact=u, g=g,
                   meta=dict(m=m, n_domain_axis=n_om, lo=lo, hi=hi, source=source))


def cube_neumann(dim: int, n_box: int, at: float, degree: int) -> Problem:
    """The 'sin' cube (u = prod sin(pi x_k) on [0, 1]^dim) with a flux boundary
    on the face x = 1: its nodes that lie on no other face form Gamma_q, with
    q = du/dx = -pi prod_{k>0} sin(pi x_k) and areas h^(dim-1) (1 in 1D); the
    other faces keep u = 0 as Dirichlet values."""
    p = cube(dim, n_box, at, degree, source="sin", name="cube_neumann")
    n_om = p.meta["n_domain_axis"]
    idx = [np.arange(n_box) for _ in range(dim)]
    shape = p.chi.shape
    on_x1 = np.zeros(shape, bool)
    on_x1[..., n_om - 1] = True
    other = np.zeros(shape, bool)
    for k in range(1, dim):
        ax = dim - 1 - k                    # axis k is array axis dim-1-k
        face = (idx[k] == 0) | (idx[k] == n_om - 1)
        sl = [None] * dim
        sl[ax] = slice(None)
        other |= np.broadcast_to(face[tuple(sl)], shape)
    neu = (p.chi > 0) & on_x1 & ~other
    X = _mesh(p.coords)
    q = -math.pi * np.ones(shape)
    for k in range(1, dim):
        q = q * np.sin(math.pi * X[k])
    h = p.h[0]
    p.dirichlet = (p.dirichlet.astype(bool) & ~neu).astype(np.uint8)
    p.free = (p.chi - p.dirichlet).astype(np.uint8)
    p.area = np.where(neu, h ** (dim - 1), 0.0)
    p.q = np.where(neu, q, 0.0)
    return p


def face_dirichlet(chi: np.ndarray) -> np.ndarray:
    """Domain nodes with at least one of their 2d face neighbours outside the
    domain (the Dirichlet layer used for embedded shapes)."""
    out = np.zeros_like(chi)
    c = chi.astype(bool)
    for ax in range(chi.ndim):
        for sh in (1, -1):
            nb = np.roll(c, sh, axis=ax)
            out |= (c & ~nb).astype(chi.dtype)
    return out.astype(np.uint8)


def sphere(n_box: int = 128, radius: float = 0.4, at: float = 3.0, degree: int = 2,
           seed: int = 3, name: str = "sphere") -> Problem:
    """Ball of the given radius centred in the unit box, nodes x = i / n_box.

    Membership is decided in integers: |i - n/2|^2 <= floor(radius^2 n^2), which
    is exact because radius^2 n^2 is not an integer for the sizes used.
    r ~ N(0, 1) i.i.d. (numpy PCG64, default_rng(seed)), masked by chi.
    V = h^3 on every domain node; Dirichlet = face-neighbour boundary layer.
    """
    h = 1.0 / n_box
    i = np.arange(n_box) - n_box // 2
    d2 = i[None, None, :] ** 2 + i[None, :, None] ** 2 + i[:, None, None] ** 2
    lim = math.floor(radius * radius * n_box * n_box)
    chi = (d2 <= lim).astype(np.uint8)
    dirichlet = face_dirichlet(chi)
    free = (chi - dirichlet).astype(np.uint8)
    vol = np.where(chi > 0, h ** 3, 0.0)
    rng = np.random.default_rng(seed)
    r = rng.standard_normal((n_box,) * 3)
    r = np.where(chi > 0, r, 0.0)
    coords = tuple(h * np.arange(n_box) for _ in range(3))
    return Problem(name=name, dim=3, dims=(n_box,) * 3, h=(h,) * 3, at=(float(at),) * 3,
                   degree=degree, chi=chi, dirichlet=dirichlet, free=free, vol=vol,
                   r=np.ascontiguousarray(r), coords=coords,
                   meta=dict(radius=radius, seed=seed))


def gaussian_rhs(p: Problem, seed: int) -> np.ndarray:
    """Seeded N(0,1) source field on the domain nodes of p."""
    rng = np.random.default_rng(seed)
    return np.where(p.chi > 0, rng.standard_normal(p.shape), 0.0)


# ---------------------------------------------------------------------------
# The five workloads of the hot path
# ---------------------------------------------------------------------------

def config1() -> Problem:
    """1D Poisson on [0,1], 256-node box, linear basis, support 2.5h, u = sin(pi x)."""
    return cube(1, 256, 2.5, 1, source="sin", name="c1_1d_sin_256")


def config2() -> Problem:
    """3D unit cube, 64^3 box, linear basis, support 2.0h, u = prod sin(pi x_k)."""
    return cube(3, 64, 2.0, 1, source="sin", name="c2_cube_64")


def config3() -> Problem:
    """Sphere r=0.4 in a 128^3 unit box, quadratic basis, support 3.0h, r ~ N(0,1) seed 3."""
    return sphere(128, 0.4, 3.0, 2, seed=3, name="c3_sphere_128_quadratic")


def config4_sizes():
    """Ragged batch: problem k = 0..15 uses an (32 + 16 (k mod 5))^3 box."""
    return [32 + 16 * (k % 5) for k in range(16)]


def config4(k: Optional[int] = None):
    """Batched cube problems (linear basis, support 2.5h, manufactured sine source)."""
    sizes = config4_sizes()
    ks = range(16) if k is None else [k]
    return [cube(3, sizes[j], 2.5, 1, source="sin", name=f"c4_cube_{sizes[j]}_{j}")
            for j in ks]


def config4_rhs_problem() -> Problem:
    """The 96^3 cube that carries the 32 seeded Gaussian right-hand sides."""
    return cube(3, 96, 2.5, 1, source="sin", name="c4_cube_96_multi_rhs")


def config4_rhs(p: Problem, count: int = 32, seed0: int = 4000):
    return [gaussian_rhs(p, seed0 + j) for j in range(count)]


def config5() -> Problem:
    """128^3 unit cube, linear basis, support 2.5h, u = prod sin(pi x_k)."""
    return cube(3, 128, 2.5, 1, source="sin", name="c5_cube_128")


def config5_256() -> Problem:
    """Config 5's problem on a 256^3 box: the FP32 working set (about 0.9 GB)
    is well above the 256 MB last-level cache, so counted bytes are HBM bytes."""
    return cube(3, 256, 2.5, 1, source="sin", name="c5_cube_256")


def config5_target(p: Problem) -> np.ndarray:
    """Smooth seeded target field u_t = sum_{k<8} a_k prod_j sin(l_kj pi x_j)."""
    rng = np.random.default_rng(5)
    ell = rng.integers(1, 4, (8, 3))
    a = rng.standard_normal(8)
    X = _mesh(p.coords)
    ut = np.zeros(p.shape)
    for k in range(8):
        t = a[k] * np.ones(p.shape)
        for j in range(3):
            t = t * np.sin(ell[k, j] * math.pi * X[j])
        ut += t
    return np.where(p.chi > 0, ut, 0.0)


def config5_directions(p: Problem, count: int = 20):
    """Seeded finite-difference directions v_j restricted to the free nodes."""
    return [np.where(p.free > 0, np.random.default_rng(5100 + j).standard_normal(p.shape), 0.0)
            for j in range(count)]


def paper_shape(n_box: int = 128) -> Problem:
    """The paper's 3D verification/timing problem (Eq 106) on [-1,1]^3, support 1.5h."""
    return cube(3, n_box, 1.5, 1, lo=-1.0, hi=1.0, source="eq106", name=f"paper_eq106_{n_box}")


def by_name(name: str) -> Problem:
    table = {"c1": config1, "c2": config2, "c3": config3, "c5": config5,
             "paper": paper_shape}
    return table[name]()
