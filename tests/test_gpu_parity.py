"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle, element by
element, on seeded meshes.  FP64 tensor and quadrature kernels: per-cell relative
Frobenius error <= 1e-12.  Split BF16: the 6-product split must reach <= 1e-6; the
3-product split cannot (about 2^-17 per product before cancellation), so it is held to a
per-form bound of 1.5 times its measured maximum on the same seeded inputs -- a loss of
accuracy of the x3 path shows as a failure, not only as a printed number."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import capi, meshgen
from paper_1112_0402_amd.forms import Batch, Form, compute_geometry
from tests.gpu_util import every_cell_errors, rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
SPLIT6_TOL = 1e-6
# measured maximum per-cell error of the 3-product split per (kind, dim, degree) over the
# seeded small meshes of these tests (the largest over the tests that run the form); the
# bound is 1.5 times it
SPLIT3_MEASURED = {
    ("laplace", 2, 1): 1.42e-5, ("laplace", 2, 2): 2.36e-5, ("laplace", 2, 3): 2.33e-5, ("laplace", 2, 4): 1.37e-5,
    ("laplace", 3, 1): 2.27e-5, ("laplace", 3, 2): 3.07e-5, ("laplace", 3, 3): 1.62e-5, ("laplace", 3, 4): 1.42e-5,
    ("mass", 2, 1): 1.71e-5, ("mass", 2, 2): 7.7e-6, ("mass", 2, 3): 1.34e-5, ("mass", 3, 1): 2.02e-5,
    ("mass", 3, 2): 7.7e-6, ("mass", 3, 3): 2.41e-5, ("wlaplace", 2, 4): 7.6e-6, ("wlaplace", 3, 3): 9.3e-6,
    ("elasticity", 2, 3): 1.32e-5, ("elasticity", 3, 2): 1.40e-5, ("ns", 2, 2): 3.34e-5, ("ns", 3, 2): 1.47e-5,
}
SPLIT3_UNMEASURED = 1e-4  # forms without a recorded maximum (the measured value is printed)


def split3_bound(kind, dim, q):
    m = SPLIT3_MEASURED.get((kind, dim, q))
    return 1.5 * m if m is not None else SPLIT3_UNMEASURED


def split_tol(precision, kind, dim, q):
    return SPLIT6_TOL if precision == "bf16x6" else split3_bound(kind, dim, q)


def _small(kind, dim, q, seed=5):
    # 2D: 2 * 11^2 = 242 cells; 3D: 6 * 5^3 = 750 cells -- several 64-cell tiles plus a
    # ragged tail
    n = 11 if dim == 2 else 5
    return meshgen.make_workload(kind, dim, q, n, seed)


ALL_FORMS = [("mass", d, q) for d in (2, 3) for q in (1, 2, 3, 4)] \
    + [("laplace", d, q) for d in (2, 3) for q in (1, 2, 3, 4)] \
    + [("wlaplace", 2, q) for q in (1, 2, 3, 4)] + [("wlaplace", 3, q) for q in (1, 2, 3)] \
    + [("elasticity", d, q) for d in (2, 3) for q in (1, 2, 3)] \
    + [("ns", d, q) for d in (2, 3) for q in (1, 2, 3)]


def _run(form, wl):
    X = to_dev(wl.coords)
    C = to_dev(wl.coeffs)
    out = form.tabulate(X, C)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("kind,dim,q", ALL_FORMS)
@pytest.mark.parametrize("kernel", ["tensor", "quadrature"])
def test_fp64_parity_small(kind, dim, q, kernel):
    require_gpu()
    say(f"[parity] {kernel} fp64 {kind} d={dim} q={q}")
    wl = _small(kind, dim, q)
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    got = _run(Form(kind, dim, q, kernel=kernel), wl)
    emax, emed = rel_fro(got, ref)
    say(f"    max {emax:.2e} median {emed:.2e}")
    assert emax <= FP64_TOL


@pytest.mark.parametrize("kind,dim,q", [("laplace", 2, 1), ("mass", 3, 1), ("laplace", 3, 1), ("laplace", 2, 2),
                                        ("elasticity", 2, 1), ("ns", 2, 1), ("wlaplace", 3, 1), ("piola", 3, 1),
                                        ("nedelec", 3, 1)])
def test_tiny_tensor_tile_shapes(kind, dim, q):
    """Element tensors of at most 36 entries default to one- or two-wave workgroups (32-cell
    tiles of one wave up to 16 entries, 64-cell tiles of two up to 36; forms with
    coefficients from 10 to 36 entries 32-cell tiles of two); every such shape runs the same
    MFMA steps per tile as the 4-wave shape, so all are bitwise equal to it, and match the
    oracle to 1e-12, on a mesh with a ragged last tile."""
    require_gpu()
    wl = meshgen.make_workload(kind, dim, q, 40 if dim == 2 else 9, 83, max_cells=4321)
    f0 = Form(kind, dim, q)
    n_I = f0.info["n_entries"]
    if f0.info["n_coeffs"] > 0 and 9 < n_I <= 36:
        assert (f0.info["tile_cells"], f0.info["waves"]) == (32, 2)
    elif n_I <= 16:
        assert (f0.info["tile_cells"], f0.info["waves"]) == (32, 1)
    elif n_I <= 36:
        assert (f0.info["tile_cells"], f0.info["waves"]) == (64, 2)
    if kind == "piola":
        ref = oracle.piola_mass(dim, wl.coords)
    elif kind == "nedelec":
        ref = oracle.nedelec_mass(dim, wl.coords)
    else:
        ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    base = _run(Form(kind, dim, q, tile_cells=64, waves=4), wl)
    assert rel_fro(base, ref)[0] <= FP64_TOL
    for tc, w in [(0, 0), (32, 1), (64, 1), (64, 2), (16, 1), (32, 2)]:
        got = _run(Form(kind, dim, q, tile_cells=tc, waves=w), wl)
        assert np.array_equal(got, base), (tc, w)


@pytest.mark.parametrize("tile_cells,waves", [(16, 1), (32, 2), (64, 8), (16, 4)])
def test_fp64_launch_shapes(tile_cells, waves):
    require_gpu()
    wl = _small("elasticity", 3, 2)
    ref = oracle.tabulate("elasticity", 3, 2, wl.coords)
    got = _run(Form("elasticity", 3, 2, tile_cells=tile_cells, waves=waves), wl)
    assert rel_fro(got, ref)[0] <= FP64_TOL


@pytest.mark.parametrize("kind,dim,q", [("wlaplace", 3, 3), ("mass", 3, 3), ("laplace", 3, 3), ("laplace", 2, 4),
                                        ("wlaplace", 2, 4), ("ns", 2, 2), ("elasticity", 2, 3), ("mass", 2, 1)])
@pytest.mark.parametrize("precision", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("tile_cells", [16, 32, 64])
def test_persistent_split_bf16_matches_tile_kernel(kind, dim, q, precision, tile_cells):
    """The persistent split-BF16 kernel (B fragments in registers, I/O waves) against the
    per-tile kernel: same pieces and the same K order, so equal bit for bit, over a mesh of
    several tiles per workgroup with a ragged tail, single mesh and as a batch cut at ragged
    sizes; and the oracle on sampled cells."""
    require_gpu()
    n = 70 if dim == 2 else 12
    wl = meshgen.make_workload(kind, dim, q, n, 77, max_cells=9999)
    pers = Form(kind, dim, q, precision=precision, persistent=1, tile_cells=tile_cells)
    tile = Form(kind, dim, q, precision=precision, persistent=-1)
    if not pers.info["persistent_waves"]:
        pytest.skip("form does not fit the persistent split-BF16 kernel")
    assert not tile.info["persistent_waves"]
    a, b = _run(pers, wl), _run(tile, wl)
    assert np.array_equal(a, b)
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    cuts = [0, 65, 3000, wl.cells]
    Xs = [X[:, c0:c1].contiguous() for c0, c1 in zip(cuts, cuts[1:])]
    Cs = [None if C is None else C[:, c0:c1].contiguous() for c0, c1 in zip(cuts, cuts[1:])]
    outs = [pers.empty_out(x.shape[1]).fill_(float("nan")) for x in Xs]
    Batch([pers] * len(Xs), Xs, Cs, outs).run()
    torch.cuda.synchronize()
    assert np.array_equal(np.concatenate([o.cpu().numpy() for o in outs]), a)
    idx = _sample(wl.cells, 64, 5)
    ref = oracle.tabulate(kind, dim, q, np.ascontiguousarray(wl.coords[:, idx]),
                          None if wl.coeffs is None else np.ascontiguousarray(wl.coeffs[:, idx]))
    e = rel_fro(a[idx], ref)[0]
    say(f"[bf16 persistent] {kind} d={dim} q={q} {precision} {tile_cells} cells: steps {pers.info['persistent_kmax']} "
        f"max err {e:.2e}")
    say(f"[x3-max] {kind} {dim} {q} {e:.3e}" if precision == "bf16x3" else "")
    assert e <= split_tol(precision, kind, dim, q)


@pytest.mark.parametrize("kind,dim,q", [("laplace", 2, 1), ("mass", 3, 3), ("laplace", 3, 4), ("wlaplace", 3, 3),
                                        ("elasticity", 3, 1), ("ns", 2, 2), ("wlaplace", 2, 4), ("elasticity", 2, 3),
                                        ("elasticity", 3, 2), ("ns", 3, 2)])
@pytest.mark.parametrize("precision", ["fp64", "bf16x6"])
@pytest.mark.parametrize("tile_cells", [0, 16, 64])
def test_fused_geometry_matches_geometry_pass(kind, dim, q, precision, tile_cells):
    """The one-launch path (affine map computed in the contraction: per tile in LDS, or one
    tile ahead in the persistent kernel) equals the geometry pass plus contraction bit for
    bit, and the oracle to the precision's bound."""
    require_gpu()
    wl = _small(kind, dim, q)
    fused = Form(kind, dim, q, precision=precision, geometry="fused", tile_cells=tile_cells)
    passed = Form(kind, dim, q, precision=precision, geometry="pass", tile_cells=tile_cells)
    a, b = _run(fused, wl), _run(passed, wl)
    if fused.info["persistent_waves"]:
        say(f"[fused] {kind} d={dim} q={q} {precision}: persistent {fused.info['persistent_waves']} waves, "
            f"fused {fused.info['fused_geometry']}; pass form: {passed.info['persistent_waves']} waves")
    assert np.array_equal(a, b)
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    assert rel_fro(a, ref)[0] <= (FP64_TOL if precision == "fp64" else SPLIT6_TOL)


@pytest.mark.parametrize("kind,dim,q", [("elasticity", 3, 2), ("laplace", 3, 3), ("mass", 2, 4), ("wlaplace", 3, 2),
                                        ("elasticity", 2, 1), ("laplace", 2, 2)])
@pytest.mark.parametrize("launch", [dict(), dict(persistent=-1, tile_cells=16), dict(persistent=-1, tile_cells=64),
                                    dict(persistent=-1, tile_cells=32, waves=8, geometry="pass")])
def test_symmetric_tiles(kind, dim, q, launch):
    """Symmetric forms compute the entries i1 <= i2 only and write each at (i2, i1) too: the
    element matrices come out exactly symmetric, agree with every entry computed (symmetry=-1)
    to rounding, and with the oracle to the FP64 bound."""
    require_gpu()
    n = 40 if dim == 2 else 9
    wl = meshgen.make_workload(kind, dim, q, n, 31, max_cells=9999)
    fh, ff = Form(kind, dim, q, **launch), Form(kind, dim, q, symmetry=-1, **launch)
    assert ff.info["symmetric"] == 0
    # every form listed saves MFMA steps with half tiles; direct stores (output rows not
    # staged in LDS) keep every entry
    if not fh.info["symmetric"]:
        assert fh.info["persistent_waves"] == 0
        assert fh.info["tile_cells"] * fh.info["n_entries"] * 8 > 96 * 1024
    half, full = _run(fh, wl), _run(ff, wl)
    half = half.reshape(len(half), -1)
    full = full.reshape(len(full), -1)
    ne = int(round(math.sqrt(half.shape[1])))
    m = half.reshape(-1, ne, ne)
    if fh.info["symmetric"]:
        assert np.array_equal(m, m.transpose(0, 2, 1))
    assert rel_fro(half, full)[0] <= 1e-13
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    assert rel_fro(half, ref)[0] <= FP64_TOL


@pytest.mark.parametrize("kind,dim,q,n_alpha,g_entries", [("laplace", 2, 2, 4, 3), ("laplace", 3, 1, 9, 6),
                                                          ("wlaplace", 3, 3, 36, 24), ("elasticity", 3, 2, 81, 45),
                                                          ("elasticity", 2, 1, 16, 10), ("mass", 3, 2, 1, 1),
                                                          ("ns", 3, 2, 36, 36)])
def test_symmetric_geometry_tensor_fold(kind, dim, q, n_alpha, g_entries):
    """Symmetric G (Laplacian, weighted Laplacian, elasticity): the tensor kernels compute
    each unordered index pair once against summed A^0 columns; |alpha| as the form defines
    it is still reported, and the result matches the quadrature kernel and the oracle."""
    require_gpu()
    f = Form(kind, dim, q)
    assert f.info["n_alpha"] == n_alpha and f.info["g_entries"] == g_entries
    wl = _small(kind, dim, q)
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    assert rel_fro(_run(f, wl), ref)[0] <= FP64_TOL
    assert rel_fro(_run(Form(kind, dim, q, precision="bf16x6"), wl), ref)[0] <= SPLIT6_TOL


def test_nonsymmetric_form_ignores_symmetry():
    require_gpu()
    wl = _small("ns", 3, 2)
    a = _run(Form("ns", 3, 2), wl)
    b = _run(Form("ns", 3, 2, symmetry=-1), wl)
    assert np.array_equal(a, b)
    ne = int(round(math.sqrt(a[0].size)))
    m = a.reshape(-1, ne, ne)
    assert not np.allclose(m, m.transpose(0, 2, 1))


@pytest.mark.parametrize("kind,dim,q", [("laplace", 2, 1), ("mass", 3, 3), ("laplace", 3, 4), ("wlaplace", 3, 3),
                                        ("elasticity", 3, 2), ("ns", 3, 2), ("ns", 2, 2), ("mass", 2, 2)])
@pytest.mark.parametrize("precision", ["bf16x3", "bf16x6"])
def test_split_bf16_parity_small(kind, dim, q, precision):
    require_gpu()
    wl = _small(kind, dim, q)
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    got = _run(Form(kind, dim, q, precision=precision), wl)
    assert got.dtype == np.float32
    emax, emed = rel_fro(got, ref)
    say(f"[split] {precision} {kind} d={dim} q={q}: max {emax:.2e} median {emed:.2e}")
    if precision == "bf16x3":
        say(f"[x3-max] {kind} {dim} {q} {emax:.3e}")
    assert emax <= split_tol(precision, kind, dim, q)


# ---------------------------------------------------------------- full sizes ---

def _sample(cells, k, seed):
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([[0, 1, cells - 2, cells - 1], rng.choice(cells, size=k, replace=False)]))
    return idx


def test_config1_full_mesh():
    """2D Poisson P1, 64 x 64 squares -> 8192 cells: every cell against the oracle."""
    require_gpu()
    wl = meshgen.config1()
    assert wl.cells == 8192
    ref = oracle.tabulate("laplace", 2, 1, wl.coords)
    for kernel in ("tensor", "quadrature"):
        got = _run(Form("laplace", 2, 1, kernel=kernel), wl)
        emax, emed = rel_fro(got, ref)
        say(f"[cfg1] {kernel}: max {emax:.2e} median {emed:.2e}")
        assert emax <= FP64_TOL


def test_config2_every_cell():
    """3D elasticity vector P2, 750,000 cells, default launch shape (the benchmarked one):
    every cell of the tensor and the quadrature kernels against the oracle; two tensor runs
    bitwise identical; tensor and quadrature kernels (independent arithmetic) within 1e-12
    of each other on every cell."""
    require_gpu()
    wl = meshgen.config2()
    assert wl.cells == 750_000
    X = to_dev(wl.coords)
    f = Form("elasticity", 3, 2)
    out1 = f.tabulate(X)
    out2 = f.tabulate(X)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    del out2
    q = Form("elasticity", 3, 2, kernel="quadrature").tabulate(X)
    torch.cuda.synchronize()
    worst = 0.0
    for c0 in range(0, wl.cells, 65536):  # tensor vs quadrature, on the GPU
        a, b = out1[c0:c0 + 65536].reshape(-1, 900), q[c0:c0 + 65536].reshape(-1, 900)
        worst = max(worst, float(((a - b).norm(dim=1) / b.norm(dim=1)).max()))
    say(f"[cfg2] tensor vs quadrature, every cell: max {worst:.2e}")
    assert worst <= FP64_TOL
    errs = every_cell_errors("elasticity", 3, 2, wl.coords, None, {"tensor": out1, "quadrature": q})
    for name, (emax, emed, n) in errs.items():
        say(f"[cfg2] {name} fp64 vs oracle, every cell ({n}): max {emax:.2e} median {emed:.2e}")
        assert n == 750_000 and emax <= FP64_TOL


def test_config3_every_cell():
    """3D weighted Laplacian P3, w in P1 ~ U(0.5, 2), 1,500,282 cells: split BF16 x3 and x6
    (FP32 accumulation) and the FP64 tensor kernel, every cell against the oracle."""
    require_gpu()
    wl = meshgen.config3()
    assert wl.cells == 1_500_282
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    outs = {p: Form("wlaplace", 3, 3, precision=p).tabulate(X, C) for p in ("bf16x3", "bf16x6", "fp64")}
    torch.cuda.synchronize()
    errs = every_cell_errors("wlaplace", 3, 3, wl.coords, wl.coeffs, outs)
    for p, (emax, emed, n) in errs.items():
        say(f"[cfg3] {p} vs oracle, every cell ({n}): max {emax:.2e} median {emed:.2e}")
        if p == "bf16x3":
            say(f"[x3-max] cfg3 wlaplace 3 3 {emax:.3e}")
        assert n == 1_500_282
        assert emax <= (FP64_TOL if p == "fp64" else SPLIT6_TOL if p == "bf16x6" else CFG3_SPLIT3_BOUND)


CFG3_SPLIT3_BOUND = 1.5 * 1.31e-5  # 1.5 times the measured maximum of x3 over every cell of this workload


# measured maximum x3 error per form variant over every cell of the mixed batch's meshes
# (the tails of 10^5-cell meshes reach further than the small meshes above); bound 1.5x
CFG4_SPLIT3_MEASURED = {
    ("laplace", 2, 1): 1.72e-5, ("laplace", 2, 2): 2.86e-5, ("laplace", 2, 3): 2.92e-5, ("laplace", 2, 4): 1.88e-5,
    ("laplace", 3, 1): 3.30e-5, ("laplace", 3, 2): 4.52e-5, ("laplace", 3, 3): 2.48e-5, ("laplace", 3, 4): 2.02e-5,
    ("mass", 2, 1): 1.88e-5, ("mass", 2, 2): 8.5e-6, ("mass", 2, 3): 1.40e-5, ("mass", 3, 1): 2.14e-5,
    ("mass", 3, 2): 8.4e-6, ("mass", 3, 3): 2.43e-5, ("ns", 2, 2): 5.97e-5, ("ns", 3, 2): 2.59e-5,
}


def test_config4_every_mesh_every_cell():
    """The mixed batch at full size (64 meshes, 7,426,598 cells) in the launch sequence the
    bench times, FP64 captured in a graph and replayed, and the split modes x6 and x3 run
    eagerly: every cell of every mesh against the oracle (run once per mesh and shared),
    every output value finite (outputs start as NaN)."""
    require_gpu()
    wls = meshgen.config4()
    assert sum(w.cells for w in wls) == 7_426_598
    X = [to_dev(w.coords) for w in wls]
    C = [to_dev(w.coeffs) for w in wls]
    outs = {}
    for precision in ("fp64", "bf16x6", "bf16x3"):
        forms = {}
        for w in wls:
            key = (w.kind, w.dim, w.degree)
            if key not in forms:
                forms[key] = Form(w.kind, w.dim, w.degree, precision=precision)
        fl = [forms[(w.kind, w.dim, w.degree)] for w in wls]
        o = [f.empty_out(w.cells).fill_(float("nan")) for f, w in zip(fl, wls)]
        s = torch.cuda.Stream()
        b = Batch(fl, X, C, o, stream=s)
        if precision == "fp64":
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                b.run()
            with torch.cuda.stream(s):
                g.replay()
        else:
            b.run()
        torch.cuda.synchronize()
        say(f"[cfg4] {precision}: {b.total_cells} cells, {b.launches} launches")
        outs[precision] = o
    worst = {p: 0.0 for p in outs}
    x3 = {}
    failures = []
    total = 0
    for k, w in enumerate(wls):
        errs = every_cell_errors(w.kind, w.dim, w.degree, w.coords, w.coeffs, {p: outs[p][k] for p in outs})
        total += w.cells
        for p, (emax, _, _) in errs.items():
            worst[p] = max(worst[p], emax)
            if p == "bf16x3":
                key = (w.kind, w.dim, w.degree)
                x3[key] = max(x3.get(key, 0.0), emax)
                tol = 1.5 * CFG4_SPLIT3_MEASURED.get(key, SPLIT3_UNMEASURED / 1.5)
            else:
                tol = FP64_TOL if p == "fp64" else SPLIT6_TOL
            if not emax <= tol:
                failures.append((w.name, p, emax, tol))
    for key, e in sorted(x3.items()):
        say(f"[x3-max] cfg4 {key[0]} {key[1]} {key[2]} {e:.3e}")
    say(f"[cfg4] every cell of every mesh ({total}): max error fp64 {worst['fp64']:.2e}, "
        f"bf16x6 {worst['bf16x6']:.2e}, bf16x3 {worst['bf16x3']:.2e}")
    assert total == 7_426_598
    assert not failures, failures


def test_chunked_geometry_pass_with_coefficients():
    """More cells than the geometry workspace holds (2^21), through the geometry-pass path of a
    form with coefficients, so the chunk loop runs with c0 > 0 and offsets coordinates,
    coefficients and outputs: every cell against the oracle, and bitwise equal to the
    one-launch fused path (which has no chunks)."""
    require_gpu()
    wl = meshgen.make_workload("wlaplace", 3, 1, 71, 8)  # 2,147,286 cells
    assert wl.cells > (1 << 21)
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    fp = Form("wlaplace", 3, 1, geometry="pass")
    ff = Form("wlaplace", 3, 1, geometry="fused")
    assert fp.info["fused_geometry"] == 0 and fp.info["persistent_waves"] == 0 and ff.info["fused_geometry"] == 1
    a = fp.tabulate(X, C)
    b = ff.tabulate(X, C)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    errs = every_cell_errors("wlaplace", 3, 1, wl.coords, wl.coeffs, {"pass": a}, chunk=262144)
    emax, emed, n = errs["pass"]
    say(f"[chunks] wlaplace P1 3D geometry pass, {n} cells in 2 chunks: max {emax:.2e}")
    assert emax <= FP64_TOL


@pytest.mark.parametrize("kind,q", [("elasticity", 2), ("wlaplace", 3)])
def test_chunked_operator_action(kind, q):
    """ffc_apply_tensor on more cells than the geometry workspace holds, on the persistent
    action path (chunks of 2^21 cells, the coefficients offset per chunk): equal to A^K x_K
    from the oracle's element tensors on the cells around the chunk boundary and a sample,
    and to the per-tile action kernel (no chunks) on every cell."""
    require_gpu()
    wl = meshgen.make_workload(kind, 3, q, 71, 9)
    cells = wl.cells
    assert cells > (1 << 21)
    fp = Form(kind, 3, q, persistent=1)
    assert fp.info["persistent_waves"] > 0 and fp.info["persistent_kmax"] <= 16, fp.info
    ft = Form(kind, 3, q, persistent=-1)
    n = fp.n
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    x = torch.from_numpy(np.random.default_rng(2).standard_normal((cells, n))).cuda()
    yp = fp.apply(X, x, C)
    yt = ft.apply(X, x, C)
    torch.cuda.synchronize()
    rel = ((yp - yt).norm(dim=1) / yt.norm(dim=1)).max().item()
    say(f"[chunks] {kind} P{q} action, persistent (chunked) vs per-tile on {cells} cells: max {rel:.2e}")
    assert rel <= 1e-12
    idx = np.unique(np.concatenate([_sample(cells, 400, 6), np.arange((1 << 21) - 40, (1 << 21) + 40)]))
    ref = oracle.tabulate(kind, 3, q, np.ascontiguousarray(wl.coords[:, idx]),
                          None if wl.coeffs is None else np.ascontiguousarray(wl.coeffs[:, idx]))
    xs = x[torch.from_numpy(idx).cuda()].cpu().numpy()
    want = np.einsum("cij,cj->ci", ref, xs)
    got = yp[torch.from_numpy(idx).cuda()].cpu().numpy()
    e = (np.linalg.norm(got - want, axis=1) / np.linalg.norm(want, axis=1)).max()
    say(f"[chunks] {kind} P{q} action vs oracle A^K x on {len(idx)} cells around 2^21: max {e:.2e}")
    assert e <= 1e-12


# ---------------------------------------------------------------- edge cases ---

def test_edge_cases():
    require_gpu()
    f = Form("wlaplace", 3, 2)
    # zero cells: no-op
    X0 = torch.empty((12, 0), dtype=torch.float64, device="cuda")
    C0 = torch.empty((4, 0), dtype=torch.float64, device="cuda")
    assert f.tabulate(X0, C0).shape == (0, 10, 10)
    # one cell
    wl = _small("wlaplace", 3, 2)
    X1 = to_dev(wl.coords[:, :1])
    C1 = to_dev(wl.coeffs[:, :1])
    got = f.tabulate(X1, C1).cpu().numpy()
    ref = oracle.tabulate("wlaplace", 3, 2, wl.coords[:, :1], wl.coeffs[:, :1])
    assert rel_fro(got, ref)[0] <= FP64_TOL
    # missing coefficients are refused before anything is enqueued
    with pytest.raises(ValueError):
        f.tabulate(X1)
    L = capi.lib()
    out = torch.empty((1, 10, 10), dtype=torch.float64, device="cuda")
    assert L.ffc_tabulate_tensor(f.handle, 1, X1.data_ptr(), None, out.data_ptr()) == capi.FFC_E_INVALID
    assert L.ffc_tabulate_tensor(f.handle, -1, X1.data_ptr(), C1.data_ptr(), out.data_ptr()) == capi.FFC_E_INVALID


def test_geometry_pass():
    require_gpu()
    for dim in (2, 3):
        wl = _small("mass", dim, 1)
        am = compute_geometry(to_dev(wl.coords), dim).cpu().numpy()
        cells = wl.cells
        Xv = wl.coords.T.reshape(cells, dim + 1, dim)
        J = np.transpose(Xv[:, 1:, :] - Xv[:, :1, :], (0, 2, 1))
        assert np.allclose(am[0], np.linalg.det(J), rtol=1e-13, atol=0)
        assert np.allclose(am[1:].T.reshape(cells, dim, dim), np.linalg.inv(J), rtol=1e-12, atol=1e-12)


def test_degenerate_orientation_reversed_cells():
    """Negatively oriented cells: |det J| enters, results match the oracle."""
    require_gpu()
    wl = _small("laplace", 3, 2)
    c = wl.coords.reshape(4, 3, -1)[[0, 2, 1, 3]].reshape(12, -1)  # swap vertices 1, 2
    c = np.ascontiguousarray(c)
    ref = oracle.tabulate("laplace", 3, 2, c)
    for kernel in ("tensor", "quadrature"):
        got = _run(Form("laplace", 3, 2, kernel=kernel), meshgen.Workload("laplace", 3, 2, c, None))
        assert rel_fro(got, ref)[0] <= FP64_TOL


# ------------------------------------------------------------------- batches ---

def _batch_inputs(precision, scale):
    wls = meshgen.config4(scale=scale)
    forms = {}
    for wl in wls:
        key = (wl.kind, wl.dim, wl.degree)
        if key not in forms:
            forms[key] = Form(wl.kind, wl.dim, wl.degree, precision=precision)
    return wls, forms


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_persistent_batch_matches_oracle_and_single_calls(precision):
    require_gpu()
    wls, forms = _batch_inputs(precision, scale=0.004)
    fl = [forms[(w.kind, w.dim, w.degree)] for w in wls]
    X = [to_dev(w.coords) for w in wls]
    C = [to_dev(w.coeffs) for w in wls]
    outs = [f.empty_out(w.cells).zero_() for f, w in zip(fl, wls)]
    b = Batch(fl, X, C, outs)
    say(f"[batch] {precision}: {len(wls)} meshes, {b.total_cells} cells, {b.work_units} units, {b.launches} launches")
    b.run()
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    for o in outs:
        o.zero_()
    b.run()  # counters reset themselves: a second run gives the same result
    torch.cuda.synchronize()
    x3, failures = {}, []
    for w, f, x, c, o, o1 in zip(wls, fl, X, C, outs, first):
        tol = FP64_TOL if precision == "fp64" else split_tol(precision, w.kind, w.dim, w.degree)
        assert torch.equal(o, o1)
        single = f.tabulate(x, c)
        torch.cuda.synchronize()
        # same tiles, same geometry arithmetic and same MFMA order as the single launch
        assert torch.equal(o, single), w.name
        ref = oracle.tabulate(w.kind, w.dim, w.degree, w.coords, w.coeffs)
        e_b = rel_fro(o.cpu().numpy(), ref)[0]
        if precision == "bf16x3":
            key = (w.kind, w.dim, w.degree)
            x3[key] = max(x3.get(key, 0.0), e_b)
        if not e_b <= tol:
            failures.append((w.name, e_b, tol))
    for key, e in sorted(x3.items()):
        say(f"[x3-max] small-batch {key[0]} {key[1]} {key[2]} {e:.3e}")
    assert not failures, failures


@pytest.mark.parametrize("precision", ["fp64", "bf16x6"])
def test_batch_launch_classes(precision):
    """Items of every launch class in one batch: two persistent (dim, kind, depth) groups
    sharing the queue counters, several claims per item, tile items staged and direct,
    16- and 64-cell tiles, an empty item, a one-cell item, ragged tails.  The batch equals
    the single-mesh launches bit for bit, and the oracle on sampled cells."""
    require_gpu()
    spec = [("ns", 3, 2, 40000), ("elasticity", 3, 2, 9001), ("laplace", 3, 4, 3001), ("mass", 2, 1, 70001),
            ("wlaplace", 3, 3, 12345), ("laplace", 2, 3, 0), ("ns", 2, 2, 1), ("ns", 3, 2, 17)]
    wls = []
    for k, (kind, dim, q, cells) in enumerate(spec):
        n = max(1, math.ceil(math.sqrt(max(cells, 1) / 2.0)) if dim == 2 else math.ceil((max(cells, 1) / 6.0) ** (1 / 3)))
        wl = meshgen.make_workload(kind, dim, q, n, 900 + k, max_cells=max(cells, 1))
        if cells == 0:
            wl.coords = wl.coords[:, :0].copy()
            wl.coeffs = None if wl.coeffs is None else wl.coeffs[:, :0].copy()
        wls.append(wl)
    forms = {}
    fl = []
    for w in wls:
        key = (w.kind, w.dim, w.degree)
        if key not in forms:
            forms[key] = Form(w.kind, w.dim, w.degree, precision=precision)
        fl.append(forms[key])
    X = [to_dev(w.coords) for w in wls]
    C = [to_dev(w.coeffs) for w in wls]
    outs = [f.empty_out(w.cells).fill_(float("nan")) for f, w in zip(fl, wls)]
    b = Batch(fl, X, C, outs)
    say(f"[batch classes] {precision}: {b.total_cells} cells, {b.work_units} units, {b.launches} launches")
    b.run()
    torch.cuda.synchronize()
    tol = FP64_TOL if precision == "fp64" else SPLIT6_TOL
    for w, f, x, c, o in zip(wls, fl, X, C, outs):
        if w.cells == 0:
            continue
        single = f.tabulate(x, c)
        torch.cuda.synchronize()
        assert torch.equal(o, single), w.name
        idx = np.arange(w.cells) if w.cells <= 80 else _sample(w.cells, 64, 3)
        ref = oracle.tabulate(w.kind, w.dim, w.degree, np.ascontiguousarray(w.coords[:, idx]),
                              None if w.coeffs is None else np.ascontiguousarray(w.coeffs[:, idx]))
        e = rel_fro(o.cpu().numpy()[idx], ref)[0]
        assert e <= tol, (w.kind, w.dim, w.degree, w.cells, e)


def test_batch_graph_replay():
    """The persistent launch captured in a graph and replayed several times, with eager
    work and synchronisations between replays: every replay equals the eager result."""
    require_gpu()
    wls, forms = _batch_inputs("fp64", scale=0.002)
    fl = [forms[(w.kind, w.dim, w.degree)] for w in wls]
    X = [to_dev(w.coords) for w in wls]
    C = [to_dev(w.coeffs) for w in wls]
    outs = [f.empty_out(w.cells) for f, w in zip(fl, wls)]
    s = torch.cuda.Stream()
    b = Batch(fl, X, C, outs, stream=s)
    with torch.cuda.stream(s):
        b.run()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep


def test_contraction_from_shared_geometry():
    """ffc_tabulate_tensor_affine on the output of ffc_compute_geometry equals
    ffc_tabulate_tensor, for two forms sharing one geometry pass."""
    require_gpu()
    wl = _small("wlaplace", 3, 2)
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    am = compute_geometry(X, 3)
    for kind, coeffs in (("wlaplace", C), ("laplace", None)):
        f = Form(kind, 3, 2)
        a = f.tabulate(X, coeffs)
        b = f.tabulate_affine(am, coeffs)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    qf = Form("laplace", 3, 2, kernel="quadrature")
    assert capi.lib().ffc_tabulate_tensor_affine(qf.handle, wl.cells, am.data_ptr(), None,
                                                 qf.empty_out(wl.cells).data_ptr()) == capi.FFC_E_INVALID


@pytest.mark.parametrize("kind,dim,q", [("elasticity", 3, 2), ("ns", 3, 2), ("elasticity", 2, 3), ("wlaplace", 3, 3)])
def test_persistent_kernel_computing_its_affine_maps(kind, dim, q):
    """The 12-wave persistent FP64 kernel that computes each tile's affine map from the
    coordinates (one tile ahead, no geometry pass) equals the 16-wave kernel reading the
    geometry pass's maps bit for bit -- single mesh, and as the persistent launch of a batch
    whose items are cut at ragged sizes -- and the oracle to 1e-12."""
    require_gpu()
    n = 40 if dim == 2 else 9
    wl = meshgen.make_workload(kind, dim, q, n, 61, max_cells=4999)
    f12 = Form(kind, dim, q, waves=12, persistent=1)
    f16 = Form(kind, dim, q, waves=16, persistent=1, geometry="pass")
    assert f12.info["persistent_waves"] == 12 and f12.info["fused_geometry"] == 1
    assert f16.info["persistent_waves"] == 16 and f16.info["fused_geometry"] == 0
    a, b = _run(f12, wl), _run(f16, wl)
    assert np.array_equal(a, b)
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    assert rel_fro(a, ref)[0] <= FP64_TOL
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    cuts = [0, 17, 1300, wl.cells]  # items of 17, 1283 and the rest of the cells
    Xs = [X[:, c0:c1].contiguous() for c0, c1 in zip(cuts, cuts[1:])]
    Cs = [None if C is None else C[:, c0:c1].contiguous() for c0, c1 in zip(cuts, cuts[1:])]
    outs = [f12.empty_out(x.shape[1]).fill_(float("nan")) for x in Xs]
    bt = Batch([f12] * len(Xs), Xs, Cs, outs)
    bt.run()
    torch.cuda.synchronize()
    assert np.array_equal(np.concatenate([o.cpu().numpy() for o in outs]), a)


# mid-size forms (100 to 400 entries) whose 12-wave schedules fit tiles of 32 cells and, up to
# 144 entries, 64 cells (the staged rows of a tile must fit the I/O registers)
MT_FORMS = [("laplace", 3, 2), ("mass", 3, 3), ("laplace", 3, 3), ("laplace", 2, 4), ("elasticity", 2, 2),
            ("wlaplace", 3, 2), ("ns", 2, 2), ("mass", 2, 4)]
MT_EXPECTED = {("laplace", 3, 2): (32, 64), ("mass", 3, 3): (32,), ("laplace", 3, 3): (32,),
               ("laplace", 2, 4): (32,), ("elasticity", 2, 2): (32, 64), ("wlaplace", 3, 2): (32, 64),
               ("ns", 2, 2): (32, 64), ("mass", 2, 4): (32,)}


@pytest.mark.parametrize("kind,dim,q", MT_FORMS)
def test_persistent_kernel_with_32_and_64_cell_tiles(kind, dim, q):
    """Persistent FP64 tiles of 32 and 64 cells (two or four 16-cell blocks per MFMA pass over
    the register-resident operands) run each 16-cell block through the same steps as 16-cell
    tiles: bit for bit equal to them, single mesh and as a batch cut at ragged sizes, and to
    the oracle to 1e-12.  A form whose schedule or staged rows do not fit takes another
    launch, which the form info reports."""
    require_gpu()
    n = 40 if dim == 2 else 9
    wl = meshgen.make_workload(kind, dim, q, n, 71, max_cells=4999)
    base = Form(kind, dim, q, waves=12, persistent=1)
    assert base.info["persistent_waves"] == 12 and base.info["tile_cells"] == 16
    a = _run(base, wl)
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    assert rel_fro(a, ref)[0] <= FP64_TOL
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    taken = []
    for tc in (32, 64):
        f = Form(kind, dim, q, waves=12, persistent=1, tile_cells=tc)
        say(f"[mt] {kind} d={dim} q={q} tile_cells={tc}: n_I {f.info['n_entries']} -> persistent "
            f"{f.info['persistent_waves']} waves, {f.info['tile_cells']}-cell tiles, kmax {f.info['persistent_kmax']}")
        b = _run(f, wl)
        assert rel_fro(b, ref)[0] <= FP64_TOL
        if f.info["persistent_waves"] != 12 or f.info["tile_cells"] != tc:
            continue
        taken.append(tc)
        assert f.info["fused_geometry"] == 1
        assert np.array_equal(a, b)
        cuts = [0, 33, 1000, 1001, wl.cells]  # items of 33, 967, 1 and the rest of the cells
        Xs = [X[:, c0:c1].contiguous() for c0, c1 in zip(cuts, cuts[1:])]
        Cs = [None if C is None else C[:, c0:c1].contiguous() for c0, c1 in zip(cuts, cuts[1:])]
        outs = [f.empty_out(x.shape[1]).fill_(float("nan")) for x in Xs]
        Batch([f] * len(Xs), Xs, Cs, outs).run()
        torch.cuda.synchronize()
        assert np.array_equal(np.concatenate([o.cpu().numpy() for o in outs]), a)
    assert tuple(taken) == MT_EXPECTED.get((kind, dim, q), ()), taken


# the library's default launch per form (ffc_form_create's rules), as the header documents
DEFAULT_LAUNCHES = [
    # kind, dim, q: (persistent waves, tile cells, waves of the tile launch or None, fused geometry)
    ("elasticity", 3, 2, (0, 16, 16, 0)),   # >= 400 entries, no coefficients: 16-cell tiles after a pass
    ("laplace", 3, 3, (0, 16, 16, 0)),
    ("mass", 3, 3, (0, 16, 16, 0)),
    ("ns", 3, 2, (12, 16, None, 1)),        # large, with coefficients: 12-wave persistent, maps in-kernel
    ("wlaplace", 3, 3, (12, 32, None, 1)),  # 400 entries, 16 steps: 32-cell persistent tiles
    ("laplace", 3, 2, (12, 64, None, 1)),   # 100 entries: 64-cell persistent tiles
    ("laplace", 2, 4, (12, 32, None, 1)),   # 225 entries: 32-cell persistent tiles
    ("laplace", 2, 2, (0, 64, 2, 1)),       # 36 entries: 64-cell tiles of two waves
    ("laplace", 2, 1, (0, 32, 1, 1)),       # 9 entries: 32-cell tiles of one wave
    ("wlaplace", 3, 1, (0, 32, 2, 1)),      # 16 entries with a coefficient: 32-cell tiles of two waves
    ("wlaplace", 2, 2, (0, 32, 2, 1)),
    ("ns", 3, 1, (12, 64, None, 1)),        # 144 entries: rows clustered, 9 steps, 64-cell persistent tiles
]


@pytest.mark.parametrize("kind,dim,q,expect", DEFAULT_LAUNCHES)
def test_default_launches(kind, dim, q, expect):
    """The default launch of each form class is the documented one, its element tensors
    equal the same launch requested explicitly bit for bit, and the oracle within 1e-12; for
    the forms that tabulate on 16-cell tiles the operator action matches the oracle's tensors
    applied to x, and for large tensors equals bit for bit the action of a form that asks for
    the 16-wave persistent kernel."""
    require_gpu()
    f = Form(kind, dim, q)
    pw, tc, w, fused = expect
    got = (f.info["persistent_waves"], f.info["tile_cells"], f.info["fused_geometry"])
    assert got == (pw, tc, fused), (kind, dim, q, f.info)
    if w is not None:
        assert f.info["waves"] == w, f.info
    wl = meshgen.make_workload(kind, dim, q, 40 if dim == 2 else 8, 97, max_cells=2999)
    a = _run(f, wl)
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    assert rel_fro(a, ref)[0] <= FP64_TOL
    if pw == 0:
        explicit = Form(kind, dim, q, persistent=-1, tile_cells=tc, waves=w,
                        geometry="fused" if fused else "pass")
    else:
        explicit = Form(kind, dim, q, persistent=1, tile_cells=tc, waves=pw)
    assert np.array_equal(a, _run(explicit, wl))
    if pw == 0 and tc == 16:
        X, C = to_dev(wl.coords), to_dev(wl.coeffs)
        xh = np.random.default_rng(3).standard_normal((wl.cells, f.n))
        y = f.apply(X, torch.from_numpy(xh).cuda(), C)
        torch.cuda.synchronize()
        yref = np.einsum("cij,cj->ci", ref, xh)
        assert np.abs(y.cpu().numpy() - yref).max() <= FP64_TOL * np.abs(yref).max()
        if f.n_I >= 576:
            # large tensors keep the 16-wave schedule for the action
            p = Form(kind, dim, q, persistent=1, waves=16)
            assert p.info["persistent_waves"] == 16
            y2 = p.apply(X, torch.from_numpy(xh).cuda(), C)
            torch.cuda.synchronize()
            assert torch.equal(y, y2)


GRAPH_CASES = [
    ("elasticity", 3, 2, {}), ("ns", 3, 2, {}), ("laplace", 3, 2, {}), ("laplace", 2, 1, {}), ("laplace", 3, 4, {}),
    ("elasticity", 3, 2, {"persistent": 1, "waves": 16}), ("wlaplace", 3, 3, {"precision": "bf16x6"}),
    ("wlaplace", 3, 3, {"precision": "bf16x3"}), ("elasticity", 3, 2, {"kernel": "quadrature"}),
    ("laplace", 3, 3, {"kernel": "auto"}),
]


@pytest.mark.parametrize("kind,dim,q,opts", GRAPH_CASES)
def test_tabulation_graph_replay(kind, dim, q, opts):
    """Each launch class captured in a graph (the geometry pass and the contraction, or one
    fused launch) and replayed three times, with other eager work and synchronisations
    between the replays: every replay equals the eager result bit for bit.  FP64 tensor
    forms also replay their operator action."""
    require_gpu()
    s = torch.cuda.Stream()
    f = Form(kind, dim, q, stream=s, **opts)
    other = Form("mass", 2, 1)
    wl = meshgen.make_workload(kind, dim, q, 40 if dim == 2 else 12, 123, max_cells=9001)
    ow = meshgen.make_workload("mass", 2, 1, 20, 124)
    X, C, OX = to_dev(wl.coords), to_dev(wl.coeffs), to_dev(ow.coords)
    out = f.empty_out(wl.cells)
    act = f.info["out_bytes"] == 8 and opts.get("kernel", "tensor") == "tensor"
    if act:
        x = torch.from_numpy(np.random.default_rng(5).standard_normal((wl.cells, f.n))).cuda()
        y = torch.empty_like(x)
    with torch.cuda.stream(s):
        f.tabulate(X, C, out=out)
        if act:
            f.apply(X, x, C, y=y)
    torch.cuda.synchronize()
    eager = out.clone()
    eager_y = y.clone() if act else None
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        f.tabulate(X, C, out=out)
        if act:
            f.apply(X, x, C, y=y)
    for rep in range(3):
        out.fill_(float("nan"))
        if act:
            y.fill_(float("nan"))
        other.tabulate(OX)  # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), (kind, dim, q, opts, rep)
        if act:
            assert torch.equal(y, eager_y), (kind, dim, q, opts, rep, "action")
    ref = oracle.tabulate(kind, dim, q, wl.coords[:, :64].copy(), None if wl.coeffs is None else wl.coeffs[:, :64].copy())
    tol = FP64_TOL if f.info["out_bytes"] == 8 else split_tol(opts["precision"], kind, dim, q)
    assert rel_fro(out[:64].cpu().numpy(), ref)[0] <= tol


def test_forms_on_concurrent_streams():
    """Forms share no device state: five forms (geometry pass + tile kernel, 12- and 16-wave
    persistent, split-BF16 persistent after a pass, quadrature), each on its own stream,
    tabulate and apply interleaved without synchronisation; every result equals the same
    call run alone."""
    require_gpu()
    specs = [("elasticity", 3, 2, {}), ("ns", 3, 2, {}), ("elasticity", 3, 2, {"persistent": 1, "waves": 16}),
             ("wlaplace", 3, 3, {"precision": "bf16x6"}), ("laplace", 3, 2, {"kernel": "quadrature"})]
    streams = [torch.cuda.Stream() for _ in specs]
    forms = [Form(k, d, q, stream=s, **o) for (k, d, q, o), s in zip(specs, streams)]
    wls = [meshgen.make_workload(k, d, q, 14, 300 + i, max_cells=12000) for i, (k, d, q, _) in enumerate(specs)]
    X = [to_dev(w.coords) for w in wls]
    C = [to_dev(w.coeffs) for w in wls]
    acts = [f.info["out_bytes"] == 8 and o.get("kernel", "tensor") == "tensor" for f, (_, _, _, o) in zip(forms, specs)]
    xs = [torch.from_numpy(np.random.default_rng(i).standard_normal((w.cells, f.n))).cuda()
          for i, (f, w) in enumerate(zip(forms, wls))]
    alone, alone_y = [], []
    for f, s, x, c, xv, a in zip(forms, streams, X, C, xs, acts):
        with torch.cuda.stream(s):
            alone.append(f.tabulate(x, c))
            alone_y.append(f.apply(x, xv, c) if a else None)
        torch.cuda.synchronize()
    outs = [f.empty_out(w.cells).fill_(float("nan")) for f, w in zip(forms, wls)]
    ys = [torch.full_like(xv, float("nan")) for xv in xs]
    torch.cuda.synchronize()
    for rep in range(2):
        for f, s, x, c, o, xv, y, a in zip(forms, streams, X, C, outs, xs, ys, acts):
            with torch.cuda.stream(s):
                f.tabulate(x, c, out=o)
                if a:
                    f.apply(x, xv, c, y=y)
    torch.cuda.synchronize()
    for (k, d, q, o_), o, r, y, ry, a in zip(specs, outs, alone, ys, alone_y, acts):
        assert torch.equal(o, r), (k, d, q, o_)
        if a:
            assert torch.equal(y, ry), (k, d, q, o_, "action")


# split modes, tile launches of small tensors: (tile cells, waves) by default
SPLIT_DEFAULT_TILES = [("laplace", 2, 1, "bf16x6", 64, 1), ("mass", 3, 1, "bf16x6", 64, 2),
                       ("elasticity", 2, 1, "bf16x3", 64, 2), ("laplace", 2, 3, "bf16x6", 64, 4),
                       ("ns", 2, 1, "bf16x3", 64, 4), ("wlaplace", 3, 1, "bf16x6", 64, 4)]


@pytest.mark.parametrize("kind,dim,q,precision,tc,w", SPLIT_DEFAULT_TILES)
def test_split_default_tile_shapes(kind, dim, q, precision, tc, w):
    """The split modes' tile launch of small tensors takes the documented workgroup size; the
    element tensors equal the 8-wave launch of the same tiles bit for bit (each 16-entry tile
    runs the same MFMA chain on whichever wave owns it) and the oracle within the bound."""
    require_gpu()
    f = Form(kind, dim, q, precision=precision)
    assert (f.info["persistent_waves"], f.info["tile_cells"], f.info["waves"]) == (0, tc, w), f.info
    wl = meshgen.make_workload(kind, dim, q, 30 if dim == 2 else 8, 131, max_cells=2999)
    a = _run(f, wl)
    assert np.array_equal(a, _run(Form(kind, dim, q, precision=precision, tile_cells=tc, waves=8), wl))
    ref = oracle.tabulate(kind, dim, q, wl.coords, wl.coeffs)
    assert rel_fro(a, ref)[0] <= split_tol(precision, kind, dim, q)
