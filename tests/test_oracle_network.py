"""Pins for the oracle's network (Alg. 2, CConv and Aff of Sec. "Architecture").

Checked against: PyTorch CPU avg_pool3d / trilinear interpolate / conv3d,
scipy.ndimage.correlate, closed forms on an all-fluid box, a composition of
library routines for centre-and-bias-only weights, and linearity.
"""
import json
import os

import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy import ndimage

import nps_inputs as gi
from oracle import network as net

torch.set_default_dtype(torch.float64)


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def test_pool_matches_torch():
    v = np.random.default_rng(0).standard_normal((3, 8, 6, 4))
    ref = F.avg_pool3d(t(v)[None], 2)[0].numpy()
    np.testing.assert_allclose(net.pool(v), ref, rtol=1e-15, atol=1e-15)


def test_interpolate_matches_torch_trilinear():
    v = np.random.default_rng(1).standard_normal((4, 3, 5))
    ref = F.interpolate(t(v)[None, None], scale_factor=2, mode="trilinear",
                        align_corners=False)[0, 0].numpy()
    np.testing.assert_allclose(net.interpolate(v), ref, rtol=1e-14, atol=1e-14)


def test_interpolate_constant_and_linear():
    c = np.full((3, 4, 5), 2.5)
    np.testing.assert_allclose(net.interpolate(c), 2.5)
    j = np.arange(6, dtype=float)
    v = np.broadcast_to(j[None, None, :], (2, 2, 6))
    fine = net.interpolate(v)[0, 0]
    # cell centres of fine cell i sit at (i + 0.5)/2 - 0.5 in coarse index units
    i = np.arange(12)
    expect = (i + 0.5) / 2 - 0.5
    np.testing.assert_allclose(fine[1:-1], expect[1:-1], atol=1e-14)


def solid_padded(I):
    pad = np.stack([np.pad(I[0], 1), np.pad(I[1], 1), np.pad(I[2], 1, constant_values=1.0)])
    return pad


@pytest.mark.parametrize("seed", range(3))
def test_cconv_kernels_match_conv3d(seed):
    rng = np.random.default_rng(seed)
    lab = rng.choice(3, size=(6, 5, 7)).astype(np.uint8)
    I = net.image(lab)
    if seed == 2:                     # fractional image (a coarser level)
        I = net.pool(net.image(rng.choice(3, size=(12, 10, 14)).astype(np.uint8)))
    W = rng.standard_normal((27, 3, 3, 3, 3))
    B = rng.standard_normal(27)
    ref = F.conv3d(t(solid_padded(I))[None], t(W), t(B))[0].numpy()
    np.testing.assert_allclose(net.cconv_kernels(I, W, B), ref, rtol=1e-12, atol=1e-12)


def test_cconv_constant_kernel_is_zero_padded_correlation():
    rng = np.random.default_rng(3)
    lab = rng.choice(3, size=(5, 6, 7)).astype(np.uint8)
    r = rng.standard_normal(lab.shape)
    B = rng.standard_normal(27)
    out = net.cconv(net.image(lab), np.zeros((27, 3, 3, 3, 3)), B, r)
    ref = ndimage.correlate(r, B.reshape(3, 3, 3), mode="constant", cval=0.0)
    np.testing.assert_allclose(out, ref, atol=1e-13)


def test_cconv_kernel_taken_at_output_cell():
    """Kernels that depend only on the centre label: out(p) is the correlation
    with the kernel of label(p), so the kernel is indexed at p, not at p + a."""
    rng = np.random.default_rng(4)
    lab = rng.choice(3, size=(6, 6, 6)).astype(np.uint8)
    r = rng.standard_normal(lab.shape)
    V = rng.standard_normal((27, 3))
    W = np.zeros((27, 3, 3, 3, 3))
    W[:, :, 1, 1, 1] = V
    out = net.cconv(net.image(lab), W, np.zeros(27), r)
    ref = np.zeros(lab.shape)
    for c in range(3):
        corr = ndimage.correlate(r, V[:, c].reshape(3, 3, 3), mode="constant", cval=0.0)
        ref[lab == c] = corr[lab == c]
    np.testing.assert_allclose(out, ref, atol=1e-13)


def test_cconv_apply_matches_unfold():
    rng = np.random.default_rng(5)
    r = rng.standard_normal((4, 5, 6))
    K = rng.standard_normal((27, 4, 5, 6))
    win = F.pad(t(r), (1, 1, 1, 1, 1, 1)).unfold(0, 3, 1).unfold(1, 3, 1).unfold(2, 3, 1)
    ref = (win.reshape(4, 5, 6, 27) * t(K).permute(1, 2, 3, 0)).sum(-1).numpy()
    np.testing.assert_allclose(net.cconv_apply(K, r), ref, atol=1e-13)


def test_aff_closed_form_all_fluid_box():
    N = 6
    I = net.image(np.zeros((N, N, N), dtype=np.uint8))
    rng = np.random.default_rng(6)
    Wb = rng.standard_normal((3, 3, 3, 3))
    Bb = 0.3
    total = 0.0
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                s_f = (N - abs(oz)) * (N - abs(oy)) * (N - abs(ox))
                total += Wb[0, oz + 1, oy + 1, ox + 1] * s_f + Wb[2, oz + 1, oy + 1, ox + 1] * (N ** 3 - s_f)
    expect = Bb + total / (27.0 * N ** 3)
    assert net.aff(I, Wb, Bb) == pytest.approx(expect, rel=1e-14)


def test_aff_matches_conv3d_mean():
    rng = np.random.default_rng(7)
    I = net.pool(net.image(rng.choice(3, size=(8, 6, 10)).astype(np.uint8)))
    Wb = rng.standard_normal((3, 3, 3, 3))
    ref = 0.7 + F.conv3d(t(solid_padded(I))[None], t(Wb)[None])[0, 0].numpy().mean() / 27.0
    assert net.aff(I, Wb, 0.7) == pytest.approx(ref, rel=1e-13)


def compose_bias_only(blob, L, lab, r):
    """The network for all-zero W and Wbar, rebuilt from library routines."""
    lay = {(n, l): (o, s) for n, l, o, s in gi.blob_layout(L)}

    def blk(name, l):
        o, s = lay[(name, l)]
        return blob[o:o + s]

    def corr(v, bias):
        return ndimage.correlate(v, bias.reshape(3, 3, 3), mode="constant", cval=0.0)

    fluid = lab == gi.FLUID
    rr = np.where(fluid, r, 0.0)
    x1 = []
    for l in range(1, L):
        x1.append(corr(rr, blk("c1B", l)))
        rr = F.avg_pool3d(t(x1[-1])[None, None], 2)[0, 0].numpy()
    x = corr(rr, blk("c1B", L))
    for l in range(L - 1, 0, -1):
        up = F.interpolate(t(x)[None, None], scale_factor=2, mode="trilinear",
                           align_corners=False)[0, 0].numpy()
        x = blk("a1B", l)[0] * x1[l - 1] + blk("a2B", l)[0] * corr(up, blk("c2B", l))
    return np.where(fluid, x, 0.0)


@pytest.mark.parametrize("L,shape", [(3, (8, 12, 4)), (4, (16, 8, 8))])
def test_network_composition_bias_only(L, shape):
    rng = np.random.default_rng(8)
    blob = np.zeros(gi.param_count(L))
    for name, _l, off, size in gi.blob_layout(L):
        if name.endswith("B"):
            blob[off:off + size] = rng.standard_normal(size)
    lab = rng.choice(3, size=shape, p=(0.6, 0.2, 0.2)).astype(np.uint8)
    r = rng.standard_normal(shape)
    np.testing.assert_allclose(net.forward(blob, L, lab, r), compose_bias_only(blob, L, lab, r),
                               rtol=1e-12, atol=1e-12)


def test_network_identity_blob_is_fluid_mask():
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=1)
    r = np.random.default_rng(9).standard_normal(lab.shape)
    out = net.forward(gi.identity_params(5), 5, lab, r)
    np.testing.assert_array_equal(out, np.where(lab == gi.FLUID, r, 0.0))


def test_network_is_linear_and_masked():
    lab = gi.gen_labels(gi.scene_gradcheck(), seed=2)
    rng = np.random.default_rng(10)
    x, y = rng.standard_normal((2,) + lab.shape)
    P = net.Network(gi.xavier_params(5, seed=3), 5, lab)
    lhs = P.apply(2.0 * x - 0.5 * y)
    rhs = 2.0 * P.apply(x) - 0.5 * P.apply(y)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())
    assert np.all(lhs[lab != gi.FLUID] == 0.0)
    # input values outside fluid are dropped (padding with zeros)
    x2 = x.copy()
    x2[lab != gi.FLUID] = 5.0
    np.testing.assert_array_equal(P.apply(x), P.apply(x2))


def test_param_count_matches_paper(repo_root):
    with open(os.path.join(repo_root, "tests", "golden", "paper_values.json")) as f:
        gold = json.load(f)
    L = gold["levels"]["value"]
    n = net.n_params(L)
    assert n == gi.param_count(L) == 25174
    approx = gold["approx_param_count"]
    assert abs(n - approx["value"]) <= approx["rel_tol"] * approx["value"]
    assert net.unpack(gi.xavier_params(L), L)["c1W"][0].shape == (27, 3, 3, 3, 3)


def test_shape_must_divide():
    with pytest.raises(ValueError):
        net.check_shape((32, 32, 48 + 8), 6)
    net.check_shape((64, 32, 96), 6)


def test_pyramid_channels_sum_to_one():
    lab = gi.gen_labels(gi.scene_c1(), seed=4)
    for I in net.image_pyramid(lab, 6):
        np.testing.assert_allclose(I.sum(0), 1.0, atol=1e-15)
