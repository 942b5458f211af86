"""The no-allocation entry point (nps_apply_precond_noalloc, static device
scratch) against nps_apply_precond (caller workspace), through the C ABI:
identical results on two calls in a row, the second on a smaller grid (the
static scratch keeps the first call's contents), and NPS_ENOMEM beyond the
scratch's size."""
import numpy as np
import pytest
import torch

import nps_inputs as gi

pytestmark = pytest.mark.gpu

nps = pytest.importorskip("paper_2310_00177_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def case(shape, seed, dtype):
    spec = gi.SceneSpec(shape, 6, (2.0, 6.0), 1, ("flat", shape[0] // 2, shape[0] - 4))
    lab = gi.gen_labels(spec, seed)
    r = np.random.default_rng(seed + 1).standard_normal(shape)
    return torch.from_numpy(lab).cuda(), torch.from_numpy(r).to(dtype).cuda()


@pytest.mark.parametrize("precision", ["fp32", "mixed_bf16", "fp64"])
def test_noalloc_matches_workspace_entry_point(precision):
    p = {"fp32": nps.FP32, "mixed_bf16": nps.MIXED_BF16, "fp64": nps.FP64}[precision]
    dtype = torch.float64 if p == nps.FP64 else torch.float32
    params = gi.xavier_params(6, 3)
    rng = np.random.default_rng(4)
    for name, _l, off, size in gi.blob_layout(6):
        if name.endswith("B"):
            params[off:off + size] = rng.uniform(-0.5, 0.5, size)
    net = nps.Net(params, 6)
    # a grid whose level 1 runs on the matrix cores, then a smaller one
    for shape, seed in (((64, 64, 96), 11), ((32, 32, 64), 12)):
        print(f"noalloc {precision} {shape}", flush=True)
        labels, r = case(shape, seed, dtype)
        ref = nps.apply_precond(net, labels, r, p)
        out = nps.apply_precond_noalloc(net, labels, r, p)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)


@pytest.mark.parametrize("shape,precision", [((224, 224, 224), "fp32"), ((160, 160, 160), "fp64")])
def test_noalloc_largest_documented_grids(shape, precision):
    """The largest grids the header promises fit in the static scratch."""
    p = nps.FP32 if precision == "fp32" else nps.FP64
    dtype = torch.float32 if precision == "fp32" else torch.float64
    net = nps.Net(gi.multilevel_params(6), 6)
    labels = torch.from_numpy(gi.gen_labels(gi.scene_serving(shape[0]), seed=5)).cuda()
    r = torch.from_numpy(np.random.default_rng(6).standard_normal(shape)).to(dtype).cuda()
    out = nps.apply_precond_noalloc(net, labels, r, p)
    ref = nps.apply_precond(net, labels, r, p)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_rejects_grids_beyond_its_scratch():
    net = nps.Net(gi.multilevel_params(6), 6)
    # 256^3 in FP32 needs about 10 bytes per cell (x1, dhat, the coarse levels)
    labels = torch.zeros((256, 256, 256), dtype=torch.uint8, device="cuda")
    r = torch.zeros((256, 256, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(nps.NpsError) as e:
        nps.apply_precond_noalloc(net, labels, r, nps.FP32)
    assert e.value.code == -7
