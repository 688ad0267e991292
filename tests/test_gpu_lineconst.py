"""GPU parity of the register path's line-constant middle pass (FP32 K,
linear basis): along every z line of a cube-like domain the pointwise matrix
V B^T B is constant away from a few nodes near the ends of the z extent, so
the middle pass applies the line's constant in the spectral domain and adds
the end nodes' differences directly (Eq 90-91 regrouped).  Checked against
the same product with a pointwise stage at every node (option off), the
LDS-tiled FP32 passes and the FP64 oracle at sampled nodes, on boxes of 64 and
128 nodes per axis, for supports 1.5h, 2.0h and 2.5h, and on box domains whose
x and y extents end at other positions (pairs of complex lines whose two real
lines have different line constants, lines outside the domain).  A domain
whose z extent leaves too many nodes outside does not take the path (the
option reads 0) and still gives the right product.  Boxes of 32, 48, 80 and
96 nodes run the register path with P x Q line layouts (4 x 8, 6 x 8, 5 x 16
or 10 x 8, 6 x 16 or 12 x 8 points x lanes), which rely on this pass."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2403_19854_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def fc():
    from paper_2403_19854_amd import fcrkpm
    return fcrkpm


def to_np(t):
    return t.detach().cpu().numpy()


def box_domain(n, at, ext):
    """A box domain of ext = (ex, ey, ez) nodes from index 0 in an n^3 box,
    spacing 1/(n - 3), trapezoid volumes, Dirichlet faces, a random source."""
    h = 1.0 / (n - 3)
    dims = (n, n, n)
    idx = np.arange(n)
    ins = [(idx < e).astype(np.uint8) for e in ext]
    face = [((idx == 0) | (idx == e - 1)).astype(np.uint8) for e in ext]
    w = [np.where(idx < e, np.where((idx == 0) | (idx == e - 1), 0.5, 1.0), 0.0) for e in ext]
    chi = (ins[2][:, None, None] * ins[1][None, :, None] * ins[0][None, None, :]).astype(np.uint8)
    onf = np.maximum(np.maximum(face[2][:, None, None], face[1][None, :, None]), face[0][None, None, :])
    dirichlet = (chi & onf).astype(np.uint8)
    free = (chi - dirichlet).astype(np.uint8)
    vol = w[2][:, None, None] * w[1][None, :, None] * w[0][None, None, :] * h ** 3
    r = np.where(chi > 0, np.random.default_rng(5).standard_normal(chi.shape), 0.0)
    return W.Problem("box", 3, dims, (h,) * 3, (at,) * 3, 1, chi, dirichlet, free, vol, r,
                     tuple(h * idx for _ in range(3)))


CASES = {
    "cube64_support2p5": (lambda: W.cube(3, 64, 2.5, 1), 1),
    "cube128_support2p5": (lambda: W.cube(3, 128, 2.5, 1), 1),
    "cube64_support2_config2": (lambda: W.config2(), 1),
    "paper_shape128_support1p5": (lambda: W.paper_shape(128), 1),
    "box128_odd_extents": (lambda: box_domain(128, 2.5, (125, 111, 126)), 1),
    "box64_odd_extents": (lambda: box_domain(64, 2.5, (37, 60, 62)), 1),
    "box64_short_z": (lambda: box_domain(64, 2.5, (62, 62, 40)), 0),
    "cube32_support2p5": (lambda: W.cube(3, 32, 2.5, 1), 1),
    "cube48_support2p5": (lambda: W.cube(3, 48, 2.5, 1), 1),
    "cube80_support2p5": (lambda: W.cube(3, 80, 2.5, 1), 1),
    "cube96_support2p5": (lambda: W.cube(3, 96, 2.5, 1), 1),
    "box96_odd_extents": (lambda: box_domain(96, 2.5, (93, 81, 94)), 1),
    "cube48_paper_support1p5": (lambda: W.paper_shape(48), 1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_line_constant_middle_pass(name):
    f = fc()
    maker, expect = CASES[name]
    p = maker()
    print(f"\n[line-constant {name}] dims={p.dims} support={p.at[0]}", flush=True)
    g = f.Problem.from_workload(p, device=DEV)
    assert g.get_option(f.OPT_LINECONST) == expect
    rng = np.random.default_rng(17)
    x = np.where(p.chi > 0, rng.standard_normal(p.shape), 0.0)
    xt = torch.from_numpy(x).to(DEV).float()
    on = to_np(g.apply("K", xt)).astype(np.float64)
    g.set_option(f.OPT_LINECONST, 0)
    off = to_np(g.apply("K", xt)).astype(np.float64)
    g.set_regpath(False)
    lds = to_np(g.apply("K", xt)).astype(np.float64)
    g.set_regpath(True)
    g.set_option(f.OPT_LINECONST, 1)
    scale = np.abs(off).max()
    d_off = np.abs(on - off).max() / scale
    d_lds = np.abs(on - lds).max() / scale
    o = oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)
    idx = np.sort(np.random.default_rng(3).choice(np.flatnonzero(p.chi.reshape(-1)), 96, replace=False))
    # include nodes at the ends of the z extent and next to the x/y ends
    zend = np.flatnonzero(p.chi.reshape(-1))[-40:]
    idx = np.unique(np.concatenate([idx, zend]))
    ref = o.apply_k_at(np.where(p.free > 0, x, 0.0), idx)
    ref = np.where(p.free.reshape(-1)[idx] > 0, ref, 0.0)
    d_orc = np.abs(on.reshape(-1)[idx] - ref).max() / scale
    print(f"  line-constant vs per-node pointwise {d_off:.2e}, vs LDS-tiled {d_lds:.2e}, "
          f"vs oracle (sampled) {d_orc:.2e}", flush=True)
    assert d_off <= 2e-6 and d_lds <= 2e-5 and d_orc <= 2e-5
    assert np.all(on[p.free == 0] == 0.0)
    if p.dims[0] in (80, 96):
        # both line layouts of these lengths (16 lanes x 5 or 6 points, 8 lanes x 10 or 12)
        chosen = g.get_option(f.OPT_REGLAYOUT)
        for lay in (0, 1):
            g.set_option(f.OPT_REGLAYOUT, lay)
            other = to_np(g.apply("K", xt)).astype(np.float64)
            d_lay = np.abs(other - off).max() / scale
            print(f"  line layout {lay}: vs per-node pointwise {d_lay:.2e}", flush=True)
            assert d_lay <= 2e-5
        g.set_option(f.OPT_REGLAYOUT, chosen)
    # batched products in one launch equal the single ones bit for bit
    two = to_np(g.apply("K", torch.stack([xt, 2 * xt])))
    np.testing.assert_array_equal(two[0], on.astype(np.float32))


@pytest.mark.parametrize("name", ["cube64_support2p5", "cube128_support2p5", "box128_odd_extents",
                                  "paper_shape128_support1p5", "cube64_support2_config2",
                                  "cube32_support2p5", "cube48_support2p5", "cube80_support2p5",
                                  "cube96_support2p5", "box96_odd_extents"])
def test_fp64_register_path(name):
    """The FP64 K product on the register path (FP64 lines, the line-constant
    middle pass) against the FP64 LDS-tiled passes and the oracle, to the FP64
    bar; a batched product equals the single ones bit for bit."""
    f = fc()
    maker, _ = CASES[name]
    p = maker()
    print(f"\n[fp64 register path {name}] dims={p.dims} support={p.at[0]}", flush=True)
    g = f.Problem.from_workload(p, device=DEV)
    x = np.where(p.chi > 0, np.random.default_rng(23).standard_normal(p.shape), 0.0)
    xt = torch.from_numpy(x).to(DEV)
    reg = to_np(g.apply("K_FULL", xt))
    g.set_regpath(False)
    lds = to_np(g.apply("K_FULL", xt))
    g.set_regpath(True)
    scale = np.abs(lds).max()
    o = oracle.Oracle(p.dims, p.h, p.at, p.degree, p.chi, p.vol)
    idx = np.sort(np.random.default_rng(4).choice(np.flatnonzero(p.chi.reshape(-1)), 96, replace=False))
    idx = np.unique(np.concatenate([idx, np.flatnonzero(p.chi.reshape(-1))[-40:]]))
    ref = o.apply_k_at(x, idx)
    d_lds = np.abs(reg - lds).max() / scale
    d_orc = np.abs(reg.reshape(-1)[idx] - ref).max() / np.abs(ref).max()
    print(f"  FP64 register vs LDS-tiled {d_lds:.2e}, vs oracle (sampled) {d_orc:.2e}", flush=True)
    assert d_lds <= 1e-12 and d_orc <= 1e-11
    assert np.all(reg[p.chi == 0] == 0.0)
    two = to_np(g.apply("K_FULL", torch.stack([xt, 2 * xt])))
    np.testing.assert_array_equal(two[0], reg)


def test_line_constant_refined_solve_c5():
    f = fc()
    p = W.config5()
    print(f"\n[line-constant refined solve c5] dims={p.dims}", flush=True)
    g = f.Problem.from_workload(p, device=DEV)
    assert g.get_option(f.OPT_LINECONST) == 1
    r = torch.from_numpy(p.r).to(DEV)
    d32, uh32, i32 = g.solve(r, mode="f32_refined", tol=1e-12, maxit=20000)
    d64, _, i64 = g.solve(r, mode="f64", tol=1e-12, maxit=20000)
    m = p.chi > 0
    e = np.linalg.norm((to_np(d32) - to_np(d64))[m]) / np.linalg.norm(to_np(d64)[m])
    print(f"  refined vs FP64 {e:.2e}; FP32 iterations {i32['iters']}, FP64 {i64['iters']}", flush=True)
    assert e <= 1e-8
