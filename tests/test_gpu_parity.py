"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle, element by
element, on seeded meshes.  FP64 tensor and quadrature kernels: per-cell relative
Frobenius error <= 1e-12.  Split-BF16: the measured error is printed per form; the
6-product split must reach <= 1e-6."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1112_0402_amd import capi, meshgen
from paper_1112_0402_amd.forms import Batch, Form, compute_geometry
from tests.gpu_util import rel_fro, require_gpu, say, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
SPLIT6_TOL = 1e-6
SPLIT3_BOUND = 1e-4  # sanity bound; the measured value is reported


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
@pytest.mark.parametrize("tile_cells", [16, 32])
def test_persistent_split_bf16_matches_tile_kernel(kind, dim, q, precision, tile_cells):
    """The persistent split-BF16 kernel (B fragments in registers, I/O waves) against the
    per-tile kernel: same pieces and the same K order, so equal bit for bit, over a mesh of
    several tiles per workgroup with a ragged tail; and the oracle on sampled cells."""
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
    idx = _sample(wl.cells, 64, 5)
    ref = oracle.tabulate(kind, dim, q, np.ascontiguousarray(wl.coords[:, idx]),
                          None if wl.coeffs is None else np.ascontiguousarray(wl.coeffs[:, idx]))
    e = rel_fro(a[idx], ref)[0]
    say(f"[bf16 persistent] {kind} d={dim} q={q} {precision} {tile_cells} cells: steps {pers.info['persistent_kmax']} "
        f"max err {e:.2e}")
    assert e <= (SPLIT6_TOL if precision == "bf16x6" else SPLIT3_BOUND)


@pytest.mark.parametrize("kind,dim,q", [("laplace", 2, 1), ("mass", 3, 3), ("laplace", 3, 4), ("wlaplace", 3, 3),
                                        ("elasticity", 3, 1), ("ns", 2, 2), ("wlaplace", 2, 4), ("elasticity", 2, 3)])
@pytest.mark.parametrize("precision", ["fp64", "bf16x6"])
@pytest.mark.parametrize("tile_cells", [0, 16, 64])
def test_fused_geometry_matches_geometry_pass(kind, dim, q, precision, tile_cells):
    """The one-launch path (affine map computed per tile in LDS) equals the geometry pass
    plus contraction bit for bit, and the oracle to the precision's bound."""
    require_gpu()
    wl = _small(kind, dim, q)
    fused = Form(kind, dim, q, precision=precision, geometry="fused", tile_cells=tile_cells)
    passed = Form(kind, dim, q, precision=precision, geometry="pass", tile_cells=tile_cells)
    a, b = _run(fused, wl), _run(passed, wl)
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
    assert emax <= (SPLIT6_TOL if precision == "bf16x6" else SPLIT3_BOUND)


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


def test_config2_full_size_sampled():
    """3D elasticity vector P2, 750,000 cells, default launch shape (the benchmarked one):
    3000 sampled cells against the oracle, and two runs bitwise identical."""
    require_gpu()
    wl = meshgen.config2()
    assert wl.cells == 750_000
    X = to_dev(wl.coords)
    f = Form("elasticity", 3, 2)
    out1 = f.tabulate(X)
    out2 = f.tabulate(X)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2)
    idx = _sample(wl.cells, 3000, 2)
    ref = oracle.tabulate("elasticity", 3, 2, wl.coords[:, idx])
    emax, emed = rel_fro(out1[torch.from_numpy(idx).cuda()].cpu().numpy(), ref)
    say(f"[cfg2] tensor fp64 sampled: max {emax:.2e} median {emed:.2e}")
    assert emax <= FP64_TOL
    q = Form("elasticity", 3, 2, kernel="quadrature").tabulate(X)
    torch.cuda.synchronize()
    emax, emed = rel_fro(q[torch.from_numpy(idx).cuda()].cpu().numpy(), ref)
    say(f"[cfg2] quadrature fp64 sampled: max {emax:.2e} median {emed:.2e}")
    assert emax <= FP64_TOL


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x6"])
def test_config3_full_size_sampled(precision):
    """3D weighted Laplacian P3, w in P1 ~ U(0.5, 2), 1,500,282 cells, split BF16 with
    FP32 accumulation: 2000 sampled cells against the oracle."""
    require_gpu()
    wl = meshgen.config3()
    assert wl.cells == 1_500_282
    X, C = to_dev(wl.coords), to_dev(wl.coeffs)
    out = Form("wlaplace", 3, 3, precision=precision).tabulate(X, C)
    torch.cuda.synchronize()
    idx = _sample(wl.cells, 2000, 3)
    ref = oracle.tabulate("wlaplace", 3, 3, wl.coords[:, idx], wl.coeffs[:, idx])
    emax, emed = rel_fro(out[torch.from_numpy(idx).cuda()].cpu().numpy(), ref)
    say(f"[cfg3] {precision}: max {emax:.2e} median {emed:.2e}")
    assert emax <= (SPLIT6_TOL if precision == "bf16x6" else SPLIT3_BOUND)


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_config4_full_size_batch_sampled(precision):
    """The mixed batch at full size (64 meshes, 7,426,598 cells) in the launch sequence the
    bench times, captured in a graph and replayed: 24 sampled cells of every mesh against
    the oracle (FP64 to 1e-12; split to its bound)."""
    require_gpu()
    wls, forms = _batch_inputs(precision, scale=1.0)
    assert sum(w.cells for w in wls) == 7_426_598
    fl = [forms[(w.kind, w.dim, w.degree)] for w in wls]
    X = [to_dev(w.coords) for w in wls]
    C = [to_dev(w.coeffs) for w in wls]
    outs = [f.empty_out(w.cells).fill_(float("nan")) for f, w in zip(fl, wls)]
    s = torch.cuda.Stream()
    b = Batch(fl, X, C, outs, stream=s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run()
    with torch.cuda.stream(s):
        g.replay()
    torch.cuda.synchronize()
    worst = 0.0
    for k, (w, o) in enumerate(zip(wls, outs)):
        idx = np.arange(w.cells) if w.cells <= 24 else _sample(w.cells, 20, 100 + k)
        ref = oracle.tabulate(w.kind, w.dim, w.degree, np.ascontiguousarray(w.coords[:, idx]),
                              None if w.coeffs is None else np.ascontiguousarray(w.coeffs[:, idx]))
        got = o[torch.from_numpy(idx).cuda()].cpu().numpy()
        worst = max(worst, rel_fro(got, ref)[0])
    say(f"[cfg4] {precision}: {b.total_cells} cells, {b.launches} launches, max sampled error {worst:.2e}")
    assert worst <= (FP64_TOL if precision == "fp64" else SPLIT3_BOUND)


def test_chunked_tabulation_beyond_workspace():
    """More cells than the geometry workspace holds (2^21): processed in chunks."""
    require_gpu()
    wl = meshgen.make_workload("mass", 2, 1, 1030, 8)  # 2,121,800 cells
    assert wl.cells > (1 << 21)
    out = Form("mass", 2, 1).tabulate(to_dev(wl.coords))
    torch.cuda.synchronize()
    idx = np.unique(np.concatenate([_sample(wl.cells, 1000, 4), np.arange((1 << 21) - 3, (1 << 21) + 3)]))
    ref = oracle.tabulate("mass", 2, 1, wl.coords[:, idx])
    assert rel_fro(out[torch.from_numpy(idx).cuda()].cpu().numpy(), ref)[0] <= FP64_TOL


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
    tol = FP64_TOL if precision == "fp64" else SPLIT3_BOUND
    for w, f, x, c, o, o1 in zip(wls, fl, X, C, outs, first):
        assert torch.equal(o, o1)
        single = f.tabulate(x, c)
        torch.cuda.synchronize()
        # same tiles, same geometry arithmetic and same MFMA order as the single launch
        assert torch.equal(o, single), w.name
        ref = oracle.tabulate(w.kind, w.dim, w.degree, w.coords, w.coeffs)
        e_b = rel_fro(o.cpu().numpy(), ref)[0]
        e_s = rel_fro(single.cpu().numpy(), ref)[0]
        assert e_b <= tol, (w.name, e_b)
        assert e_s <= tol, (w.name, e_s)


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
