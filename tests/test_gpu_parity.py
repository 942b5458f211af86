"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: matvec FP64 exact up to summation order (<= 1e-15 relative),
FP32 <= 1e-6; preconditioner FP64 <= 1e-12 relative, FP32 <= 1e-5 relative;
solves are judged on the oracle's FP64 true residual and, in FP64, on the
iterates of the fixed-iteration protocol.
"""
import numpy as np
import pytest
import torch

import nps_inputs as gi
from oracle import laplacian as lap
from oracle import network as onet
from oracle import npsdo as onpsdo

pytestmark = pytest.mark.gpu

nps = pytest.importorskip("paper_2310_00177_amd")
DEV = "cuda"


def _gpu_available():
    return torch.cuda.is_available()


if not _gpu_available():
    pytest.skip("no GPU", allow_module_level=True)


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elem_err(a, b):
    """max over cells |a - b|, relative to max |b|: catches errors local to a
    tile edge or halo that a global norm would average away."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def random_labels(shape, seed, p=(0.6, 0.2, 0.2)):
    return np.random.default_rng(seed).choice(3, size=shape, p=p).astype(np.uint8)


# ---------------------------------------------------------------------------
# matvec
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(13, 7, 33), (4, 4, 16), (32, 32, 32), (1, 1, 1), (64, 40, 24)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_laplacian_parity(shape, dtype):
    print(f"laplacian {shape} {dtype.__name__}", flush=True)
    lab = random_labels(shape, seed=sum(shape))
    x = np.random.default_rng(1).standard_normal(shape).astype(dtype)
    ref = lap.matvec(lab, x.astype(np.float64))
    y = nps.apply_laplacian(dev(lab), dev(x)).cpu().numpy()
    torch.cuda.synchronize()
    scale = max(np.abs(ref).max(), 1.0)
    tol = 1e-15 if dtype == np.float64 else 1e-6
    assert np.abs(y - ref).max() <= tol * 8 * scale
    assert np.all(y[lab != gi.FLUID] == 0)


def test_laplacian_generated_scene_bitwise_fp64():
    lab = gi.gen_labels(gi.scene_c1(), seed=3)
    x = np.random.default_rng(2).integers(-1000, 1000, size=lab.shape).astype(np.float64)
    # integer data: every partial sum is exact, so the results must agree bit for bit
    y = nps.apply_laplacian(dev(lab), dev(x)).cpu().numpy()
    np.testing.assert_array_equal(y, lap.matvec(lab, x))


# ---------------------------------------------------------------------------
# preconditioner
# ---------------------------------------------------------------------------
def blob(kind, L, seed=0):
    if kind == "xavier":
        return gi.xavier_params(L, seed)
    if kind == "multilevel":
        return gi.multilevel_params(L)
    if kind == "random_bias":
        b = gi.xavier_params(L, seed)
        rng = np.random.default_rng(seed + 100)
        for name, _l, off, size in gi.blob_layout(L):
            if name.endswith("B"):
                b[off:off + size] = rng.uniform(-0.5, 0.5, size)
        return b
    raise ValueError(kind)


PRECOND_CASES = [
    ("c1", (40, 32, 56), 4, "random_bias"),       # 71680 cells: level 1 on MFMA, ragged x tiles
    ("c1", (64, 64, 64), 6, "xavier"),            # level 1 on MFMA, levels >= 2 stored
    ("c1", (32, 32, 32), 6, "xavier"),
    ("c1", (32, 32, 32), 6, "random_bias"),
    ("c1", (32, 32, 32), 6, "multilevel"),
    ("grad", (16, 16, 16), 5, "random_bias"),
    ("c1", (32, 64, 96), 6, "random_bias"),       # non-cubic, several tiles, ragged tiles
    ("rand", (8, 24, 40), 4, "random_bias"),     # random labels: every window class
    ("rand", (34, 38, 70), 2, "random_bias"),    # level 1 on MFMA with partial column footprints in x and y
    ("c1", (34, 38, 70), 2, "xavier"),           # and a 2-plane last z-chunk
]


def make_labels(kind, shape, seed):
    if kind == "rand":
        return random_labels(shape, seed)
    spec = gi.SceneSpec(shape, 6 if kind == "c1" else 3, (2.0, 6.0) if kind == "c1" else (1.0, 3.0), 1,
                        ("flat", shape[0] // 2, shape[0] - 4))
    return gi.gen_labels(spec, seed)


@pytest.mark.parametrize("kind,shape,L,wkind", PRECOND_CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_precond_parity(kind, shape, L, wkind, precision):
    print(f"precond {kind} {shape} L={L} {wkind} {precision}", flush=True)
    lab = make_labels(kind, shape, seed=7)
    params = blob(wkind, L, seed=3)
    r = np.random.default_rng(11).standard_normal(shape)
    ref = onet.Network(params, L, lab).apply(r)
    net = nps.Net(params, L)
    if precision == "fp64":
        d = nps.apply_precond(net, dev(lab), dev(r), nps.FP64).cpu().numpy()
        tol = 1e-12
    else:
        d = nps.apply_precond(net, dev(lab), dev(r, torch.float32), nps.FP32).cpu().numpy().astype(np.float64)
        tol = 1e-5
    print(f"  norm {rel_err(d, ref):.2e}  max-cell {elem_err(d, ref):.2e}", flush=True)
    assert rel_err(d, ref) <= tol, rel_err(d, ref)
    assert elem_err(d, ref) <= tol, elem_err(d, ref)
    assert np.all(d[lab != gi.FLUID] == 0)


# Mixed modes round the generated kernels to one bf16 / fp16 piece per weight
# (counts are exact); the error against the FP64 oracle is measured and
# bounded, globally and per cell.  Bounds: MIXED_BOUNDS[precision] =
# (norm-relative, max-cell relative to max |ref|), about twice the largest
# measured error with random weights and biases (bf16: 2.8e-3 / 3.7e-3 on
# 40 x 32 x 56 at L = 4; fp16: 3.2e-4 / 3.8e-4 there; 128^3: bf16 1.6e-3 /
# 2.6e-3, fp16 2.0e-4 / 3.6e-4; the multilevel blob is exact in both: 1e-7).
MIXED_BOUNDS = {"mixed_bf16": (6e-3, 8e-3), "mixed_fp16": (7e-4, 8e-4)}
MIXED_CASES = [("c1", (64, 64, 96), 6, "random_bias"), ("c1", (40, 32, 56), 4, "random_bias"),
               ("c1", (64, 64, 96), 6, "multilevel"),
               # a one-tile-wide coarse chain with a 128-cell bottom; random labels (every
               # window class) with the bottom at level 3
               ("c1", (32, 32, 64), 4, "random_bias"), ("rand", (16, 32, 64), 3, "random_bias")]


@pytest.mark.parametrize("kind,shape,L,wkind", MIXED_CASES)
@pytest.mark.parametrize("precision", ["mixed_bf16", "mixed_fp16"])
def test_precond_mixed_error_is_bounded(precision, kind, shape, L, wkind):
    """bf16 / fp16 kernel generation: the error against the FP64 oracle is measured and bounded."""
    lab = make_labels(kind, shape, seed=4)
    params = blob(wkind, L, seed=5)
    r = np.random.default_rng(12).standard_normal(lab.shape)
    ref = onet.Network(params, L, lab).apply(r)
    p = nps.MIXED_BF16 if precision == "mixed_bf16" else nps.MIXED_FP16
    d = nps.apply_precond(nps.Net(params, L), dev(lab), dev(r, torch.float32), p).cpu().numpy().astype(np.float64)
    en, ec = rel_err(d, ref), elem_err(d, ref)
    print(f"{precision} {shape} L={L} {wkind}: error vs FP64 oracle norm {en:.3e} max-cell {ec:.3e}", flush=True)
    bn, bc = MIXED_BOUNDS[precision]
    assert en <= bn and ec <= bc
    assert np.all(d[lab != gi.FLUID] == 0)


def _full_size_case():
    lab = gi.gen_labels(gi.scene_c2(), seed=1)
    params = blob("random_bias", 6, seed=6)
    r = np.random.default_rng(13).standard_normal(lab.shape)
    return lab, params, r, onet.Network(params, 6, lab).apply(r)


@pytest.fixture(scope="module")
def full_size_case():
    return _full_size_case()


@pytest.mark.parametrize("precision", ["fp32", "mixed_bf16", "mixed_fp16"])
def test_precond_full_size(full_size_case, precision):
    """128^3 (the benchmark's grid, levels 1-2 on MFMA) against the oracle:
    FP32 bar (1e-5, globally and per cell); mixed modes within their bounds."""
    lab, params, r, ref = full_size_case
    p = {"fp32": nps.FP32, "mixed_bf16": nps.MIXED_BF16, "mixed_fp16": nps.MIXED_FP16}[precision]
    d = nps.apply_precond(nps.Net(params, 6), dev(lab), dev(r, torch.float32), p).cpu().numpy().astype(np.float64)
    en, ec = rel_err(d, ref), elem_err(d, ref)
    print(f"128^3 {precision}: norm {en:.3e} max-cell {ec:.3e}", flush=True)
    bn, bc = (1e-5, 1e-5) if precision == "fp32" else MIXED_BOUNDS[precision]
    assert en <= bn and ec <= bc


def test_precond_ignores_input_off_fluid():
    lab = make_labels("c1", (32, 32, 32), 5)
    params = blob("random_bias", 6, 1)
    r = np.random.default_rng(1).standard_normal(lab.shape)
    r2 = r.copy()
    r2[lab != gi.FLUID] = 1e3
    net = nps.Net(params, 6)
    a = nps.apply_precond(net, dev(lab), dev(r), nps.FP64).cpu().numpy()
    b = nps.apply_precond(net, dev(lab), dev(r2), nps.FP64).cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_precond_is_deterministic():
    lab = make_labels("c1", (32, 64, 96), 9)
    net = nps.Net(blob("random_bias", 6, 2), 6)
    r = dev(np.random.default_rng(3).standard_normal(lab.shape), torch.float32)
    a = nps.apply_precond(net, dev(lab), r, nps.FP32)
    b = nps.apply_precond(net, dev(lab), r, nps.FP32)
    assert torch.equal(a, b)


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------
def c1_problem(seed=1):
    lab = gi.gen_labels(gi.scene_c1(), seed=seed)
    b = gi.gen_rhs(lab, seed=seed + 1)
    return lab, b


@pytest.mark.parametrize("wkind", ["multilevel", "xavier"])
def test_fixed_iterations_fp64_match_oracle_iterates(wkind):
    """FP64, fixed-iteration protocol: the k-th iterate matches the oracle's."""
    lab, b = c1_problem(2)
    params = gi.multilevel_params(6) if wkind == "multilevel" else gi.xavier_params(6, 0)
    net = nps.Net(params, 6)
    P = onet.Network(params, 6, lab)
    for k in (1, 2, 3, 6):
        print(f"fixed-iter fp64 {wkind} k={k}", flush=True)
        ref = onpsdo.solve(lab, b, P.apply, max_iter=k, fixed_iters=True)
        x, info = nps.solve(net, dev(lab), dev(b), max_iter=k, fixed_iters=True, precision=nps.FP64)
        assert info.iterations == k and info.status == 0
        assert rel_err(x.cpu().numpy(), ref.x) <= 1e-9, (k, rel_err(x.cpu().numpy(), ref.x))
        assert info.rel_residual == pytest.approx(ref.rel_residual, rel=1e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed_bf16"])
def test_solve_c1_reaches_tolerance(precision):
    lab, b = c1_problem(1)
    params = gi.multilevel_params(6)
    p = {"fp64": nps.FP64, "fp32": nps.FP32, "mixed_bf16": nps.MIXED_BF16}[precision]
    print(f"solve c1 {precision}", flush=True)
    x, info = nps.solve(nps.Net(params, 6), dev(lab), dev(b), tol=1e-6, max_iter=500, precision=p)
    assert info.status == 0, info
    xs = x.cpu().numpy()
    true_rel = lap.rel_residual(lab, b, xs)
    assert true_rel < 1e-6, true_rel
    assert info.rel_residual == pytest.approx(true_rel, rel=1e-3, abs=1e-12)
    ref = onpsdo.solve_with_network(lab, b, params, 6, tol=1e-6, max_iter=500)
    assert abs(info.iterations - ref.iterations) <= max(2, ref.iterations // 10), (info.iterations, ref.iterations)
    assert np.all(xs[lab != gi.FLUID] == 0)


def test_identity_weights_is_cg_on_gpu():
    """P = fluid mask: NPSDO is CG; the GPU matches the oracle's CG-equivalent iterates."""
    lab, b = c1_problem(3)
    params = gi.identity_params(6)
    net = nps.Net(params, 6)
    ref = onpsdo.solve_with_network(lab, b, params, 6, max_iter=20, fixed_iters=True)
    x, info = nps.solve(net, dev(lab), dev(b), max_iter=20, fixed_iters=True, precision=nps.FP64)
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-8


def test_zero_rhs():
    lab, _ = c1_problem(4)
    x, info = nps.solve(nps.Net(gi.multilevel_params(6), 6), dev(lab), dev(np.zeros(lab.shape)))
    assert info.iterations == 0 and info.status == 0 and torch.count_nonzero(x) == 0


def test_errors_are_reported():
    lab, b = c1_problem(5)
    net = nps.Net(gi.multilevel_params(6), 6)
    bad = lab.copy()
    bad[3, 3, 3] = 7
    with pytest.raises(nps.NpsError) as e:
        nps.solve(net, dev(bad), dev(b))
    assert e.value.code == -3
    with pytest.raises(nps.NpsError) as e:
        nps.solve(net, dev(np.full(lab.shape, gi.SOLID, np.uint8)), dev(b))
    assert e.value.code == -4
    bn = b.copy()
    idx = np.argwhere(lab == gi.FLUID)[0]
    bn[tuple(idx)] = np.inf
    with pytest.raises(nps.NpsError) as e:
        nps.solve(net, dev(lab), dev(bn))
    assert e.value.code == -5
    with pytest.raises(nps.NpsError) as e:
        nps.solve(net, dev(lab[:, :, :16].copy()), dev(b[:, :, :16].copy()))   # 16 % 32 != 0
    assert e.value.code == -2
    # every entry point reports a bad shape as NPS_ESHAPE
    lab16, r16 = dev(lab[:, :, :16].copy()), dev(b[:, :, :16].copy())
    for call in (lambda: nps.apply_precond(net, lab16, r16),
                 lambda: nps.apply_precond_transpose(net, lab16, r16),
                 lambda: nps.net_forward(net, lab16, r16, nps.train_workspace((32, 32, 32), 6, nps.FP64))):
        with pytest.raises(nps.NpsError) as e:
            call()
        assert e.value.code == -2
    x, info = nps.solve(nps.Net(np.zeros(gi.param_count(6)), 6), dev(lab), dev(b), check=False)
    assert info.status == -6 and info.iterations == 0
    assert torch.all(x == 0)   # the last iterate: the step that broke down was not applied
    x, info = nps.solve(net, dev(lab), dev(b), max_iter=3)
    assert info.status == 1 and info.iterations == 3
    assert info.rel_residual == pytest.approx(lap.rel_residual(lab, b, x.cpu().numpy()), rel=1e-6)


def multi_tile_problem():
    """64x64x96: 1536 tiles for at most 1024 blocks, so blocks walk several tiles."""
    spec = gi.SceneSpec((64, 64, 96), 8, (3.0, 10.0), 2, ("flat", 32, 56))
    lab = gi.gen_labels(spec, seed=21)
    return lab, gi.gen_rhs(lab, seed=22)


def test_multi_tile_fixed_iterations_fp64_match_oracle():
    lab, b = multi_tile_problem()
    params = gi.multilevel_params(6)
    P = onet.Network(params, 6, lab)
    ref = onpsdo.solve(lab, b, P.apply, max_iter=4, fixed_iters=True)
    x, info = nps.solve(nps.Net(params, 6), dev(lab), dev(b), max_iter=4, fixed_iters=True, precision=nps.FP64)
    assert info.iterations == 4
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-9


@pytest.mark.parametrize("n_ortho", [0, 1, 3, 4])
@pytest.mark.parametrize("grid", ["single", "multi"])
def test_n_ortho_fixed_iterations_fp64_match_oracle(n_ortho, grid):
    """Every orthogonalisation width the library compiles (Sec. "Algorithm":
    n_ortho = 0 is steepest descent; the appendix on the number of
    orthogonalisations): the k-th FP64 iterate, and the residual, match the
    oracle's, on a single-tile-per-block grid and a multi-tile one.  k runs
    past n_ortho + 1 so the direction ring wraps."""
    lab, b = c1_problem(2) if grid == "single" else multi_tile_problem()
    params = gi.multilevel_params(6)
    P = onet.Network(params, 6, lab)
    net = nps.Net(params, 6)
    ks = (1, 2, n_ortho + 3) if grid == "single" else (n_ortho + 3,)
    for k in ks:
        print(f"n_ortho={n_ortho} {grid} k={k}", flush=True)
        ref = onpsdo.solve(lab, b, P.apply, max_iter=k, fixed_iters=True, n_ortho=n_ortho)
        x, info = nps.solve(net, dev(lab), dev(b), max_iter=k, fixed_iters=True, precision=nps.FP64,
                            n_ortho=n_ortho)
        assert info.iterations == k and info.status == 0
        assert rel_err(x.cpu().numpy(), ref.x) <= 1e-9, (k, rel_err(x.cpu().numpy(), ref.x))
        assert info.rel_residual == pytest.approx(ref.rel_residual, rel=1e-6)


@pytest.mark.parametrize("precision", ["fp32", "mixed_bf16", "mixed_fp16"])
def test_multi_tile_solve_reaches_tolerance(precision):
    lab, b = multi_tile_problem()
    p = {"fp32": nps.FP32, "mixed_bf16": nps.MIXED_BF16, "mixed_fp16": nps.MIXED_FP16}[precision]
    x, info = nps.solve(nps.Net(gi.multilevel_params(6), 6), dev(lab), dev(b), tol=1e-6, max_iter=400, precision=p)
    true_rel = lap.rel_residual(lab, b, x.cpu().numpy())
    print(f"multi-tile {precision}: {info.iterations} its, true rel residual {true_rel:.3e}", flush=True)
    assert info.status == 0 and true_rel < 1e-6


@pytest.mark.parametrize("precision", ["fp32", "mixed_bf16"])
def test_benchmark_workload_solve(precision):
    """The 128^3 benchmark system: the result's FP64 true residual (oracle matvec) meets 1e-6."""
    lab = gi.gen_labels(gi.scene_c2(), seed=1)
    b = gi.gen_rhs(lab, seed=2)
    p = nps.FP32 if precision == "fp32" else nps.MIXED_BF16
    x, info = nps.solve(nps.Net(gi.multilevel_params(6), 6), dev(lab), dev(b), tol=1e-6, max_iter=400, precision=p)
    true_rel = lap.rel_residual(lab, b, x.cpu().numpy())
    print(f"128^3 {precision}: {info.iterations} its, reported {info.rel_residual:.3e}, oracle {true_rel:.3e}", flush=True)
    assert info.status == 0 and true_rel < 1e-6
    assert info.rel_residual == pytest.approx(true_rel, rel=1e-3)
    # the oracle's own solve of this system (tests/golden/oracle_workloads.json,
    # written by make_oracle_reference.py from the oracle alone) takes 66 iterations
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_workloads.json")))["128^3"]
    assert abs(info.iterations - ref["iterations"]) <= max(2, ref["iterations"] // 10), info.iterations
    assert np.all(x.cpu().numpy()[lab != gi.FLUID] == 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "mixed_bf16"])
def test_ragged_mfma_footprints_match_oracle(precision):
    """34 x 38 x 70 with L = 2: level 1 (90,440 cells) runs on the matrix
    cores with partial 64 x 4 column footprints in x and y and a 2-plane last
    z-chunk; FP64 (vector path) and FP32 iterates match the oracle's, the
    mixed path stays within its preconditioner error."""
    shape = (34, 38, 70)
    lab = random_labels(shape, seed=41, p=(0.7, 0.15, 0.15))
    b = gi.gen_rhs(lab, seed=42)
    params = gi.multilevel_params(2)
    P = onet.Network(params, 2, lab)
    p, tol = {"fp64": (nps.FP64, 1e-9), "fp32": (nps.FP32, 1e-4), "mixed_bf16": (nps.MIXED_BF16, 3e-2)}[precision]
    for k in (1, 3):
        print(f"ragged mfma footprints {precision} k={k}", flush=True)
        ref = onpsdo.solve(lab, b, P.apply, max_iter=k, fixed_iters=True)
        x, info = nps.solve(nps.Net(params, 2), dev(lab), dev(b), max_iter=k, fixed_iters=True, precision=p)
        assert info.iterations == k
        assert rel_err(x.cpu().numpy(), ref.x) <= tol, (k, rel_err(x.cpu().numpy(), ref.x))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ragged_column_footprints_match_oracle(precision):
    """10 x 6 x 70 with L = 2: the plane-marching kernels see a partial
    64-column footprint in x, a partial 4-row footprint in y and a 2-plane
    last z-chunk; the k-th iterate matches the oracle's."""
    shape = (10, 6, 70)
    lab = random_labels(shape, seed=31)
    b = gi.gen_rhs(lab, seed=32)
    params = gi.multilevel_params(2)
    P = onet.Network(params, 2, lab)
    p, tol = (nps.FP64, 1e-9) if precision == "fp64" else (nps.FP32, 1e-4)
    for k in (1, 4):
        print(f"ragged footprints {precision} k={k}", flush=True)
        ref = onpsdo.solve(lab, b, P.apply, max_iter=k, fixed_iters=True)
        x, info = nps.solve(nps.Net(params, 2), dev(lab), dev(b), max_iter=k, fixed_iters=True, precision=p)
        assert info.iterations == k
        assert rel_err(x.cpu().numpy(), ref.x) <= tol, (k, rel_err(x.cpu().numpy(), ref.x))
