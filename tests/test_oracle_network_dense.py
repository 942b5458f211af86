"""Brute-force pin of the whole network (Alg. 2) with non-zero weights.

The dense matrix of P(I, .) on a tiny grid, taken column by column from the
oracle, must equal the product of per-level operator matrices built here
independently of the oracle's code:
  * the image pyramid by torch avg_pool3d of the one-hot image;
  * each CConv block as a sparse matrix whose row p holds K_t(p) at column
    p + a_t, with K formed by torch conv3d of *that level's* solid-padded image
    (Sec. "Architecture": kernels from the level's image, correlation);
  * pooling as the 2x2x2 child average, upsampling as torch trilinear
    interpolation (align_corners=False) of unit vectors;
  * the Aff scalars as Bbar + mean over the level of conv3d(image, Wbar) / 27;
  * the input zeroed and the output restricted to fluid.
Planted mistakes in the oracle (an Aff scalar or a kernel from the wrong
level's image, the down-sweep kernel used in the up sweep) must fail it.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import nps_inputs as gi
from oracle import network as onet

OFFS = [(az, ay, ax) for az in (-1, 0, 1) for ay in (-1, 0, 1) for ax in (-1, 0, 1)]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))


def _pyramid(lab, L):
    img = np.stack([(lab == c) for c in range(3)]).astype(np.float64)
    out = [_t(img)[None]]
    for _ in range(L - 1):
        out.append(F.avg_pool3d(out[-1], 2))
    return out                                            # (1, 3, nz, ny, nx) per level


def _solid_pad(I):
    return torch.cat([F.pad(I[:, :2], (1,) * 6), F.pad(I[:, 2:], (1,) * 6, value=1.0)], dim=1)


def _cconv_matrix(I, W, B):
    K = F.conv3d(_solid_pad(I), _t(W), _t(B))[0].numpy()  # (27, nz, ny, nx)
    nz, ny, nx = K.shape[1:]
    n = nz * ny * nx
    M = np.zeros((n, n))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p = ((z * ny + y) * nx + x).ravel()
    for t, (az, ay, ax) in enumerate(OFFS):
        zz, yy, xx = (z + az).ravel(), (y + ay).ravel(), (x + ax).ravel()
        ok = (zz >= 0) & (zz < nz) & (yy >= 0) & (yy < ny) & (xx >= 0) & (xx < nx)
        q = (zz * ny + yy) * nx + xx
        M[p[ok], q[ok]] += K[t].ravel()[ok]
    return M


def _pool_matrix(shape):
    nz, ny, nx = shape
    cz, cy, cx = nz // 2, ny // 2, nx // 2
    M = np.zeros((cz * cy * cx, nz * ny * nx))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                M[((z // 2) * cy + y // 2) * cx + x // 2, (z * ny + y) * nx + x] = 0.125
    return M


def _interp_matrix(coarse_shape):
    n = int(np.prod(coarse_shape))
    eye = torch.eye(n, dtype=torch.float64).reshape((n, 1) + tuple(coarse_shape))
    up = F.interpolate(eye, scale_factor=2, mode="trilinear", align_corners=False)
    return up.reshape(n, -1).numpy().T                    # (fine, coarse)


def _aff(I, Wb, Bb):
    return Bb + F.conv3d(_solid_pad(I), _t(Wb)[None])[0, 0].numpy().mean() / 27.0


def dense_from_operators(blob, L, lab):
    """P as a dense matrix, composed from the per-level operators."""
    lay = {(nm, l): (o, s) for nm, l, o, s in gi.blob_layout(L)}

    def blk(name, l, shape):
        o, s = lay[(name, l)]
        return blob[o:o + s].reshape(shape)

    I = _pyramid(lab, L)
    shapes = [tuple(Il.shape[2:]) for Il in I]
    mask = np.diag((lab == gi.FLUID).ravel().astype(np.float64))
    D = []                                                 # x1^l as a matrix acting on r
    prev = mask
    for l in range(1, L + 1):
        C1 = _cconv_matrix(I[l - 1], blk("c1W", l, (27, 3, 3, 3, 3)), blk("c1B", l, (27,)))
        D.append(C1 @ prev)
        if l < L:
            prev = _pool_matrix(shapes[l - 1]) @ D[-1]
    X = D[L - 1]
    for l in range(L - 1, 0, -1):
        C2 = _cconv_matrix(I[l - 1], blk("c2W", l, (27, 3, 3, 3, 3)), blk("c2B", l, (27,)))
        c1 = _aff(I[l - 1], blk("a1W", l, (3, 3, 3, 3)), blk("a1B", l, (1,))[0])
        c2 = _aff(I[l - 1], blk("a2W", l, (3, 3, 3, 3)), blk("a2B", l, (1,))[0])
        X = c1 * D[l - 1] + c2 * (C2 @ _interp_matrix(shapes[l]) @ X)
    return mask @ X


def dense_from_oracle(P, shape):
    n = int(np.prod(shape))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(P.apply(e.reshape(shape)).ravel())
    return np.stack(cols, axis=1)


def _blob(L, seed):
    """Xavier weights plus non-zero biases: every term of every block is live."""
    b = gi.xavier_params(L, seed)
    rng = np.random.default_rng(seed + 50)
    for name, _l, off, size in gi.blob_layout(L):
        if name.endswith("B"):
            b[off:off + size] = rng.uniform(-0.5, 0.5, size)
    return b


CASES = [(3, (8, 8, 16)), (4, (8, 8, 16))]


def _labels(shape, seed):
    return np.random.default_rng(seed).choice(3, size=shape, p=(0.5, 0.25, 0.25)).astype(np.uint8)


@pytest.mark.parametrize("L,shape", CASES)
def test_dense_network_equals_operator_product(L, shape):
    lab = _labels(shape, 20 + L)
    blob = _blob(L, 3 + L)
    ref = dense_from_operators(blob, L, lab)
    got = dense_from_oracle(onet.Network(blob, L, lab), shape)
    assert np.abs(ref).max() > 1e-3
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _plant(P, kind):
    """Plausible wiring mistakes, planted in a built oracle network."""
    n = P.net
    if kind == "aff_from_coarser_image":          # c1 of level 1 from I^2
        P.c1[0] = onet.aff(P.I[1], n["a1W"][0], n["a1B"][0])
    elif kind == "aff2_from_coarser_image":       # c2 of level 2 from I^3
        P.c2[1] = onet.aff(P.I[2], n["a2W"][1], n["a2B"][1])
    elif kind == "up_kernel_from_upsampled_image":   # K2^1 from Interp(I^2) instead of I^1
        P.K2[0] = onet.cconv_kernels(onet.interpolate(P.I[1]), n["c2W"][0], n["c2B"][0])
    elif kind == "down_kernel_in_up_sweep":       # K1^2 used where K2^2 belongs
        P.K2[1] = P.K1[1]
    elif kind == "aff_normalised_by_fine_cells":   # 1/(27 n_1) instead of 1/(27 n_l) on level 2
        ratio = P.I[1][0].size / P.I[0][0].size
        P.c1[1] = n["a1B"][1] + (P.c1[1] - n["a1B"][1]) * ratio
    return P


@pytest.mark.parametrize("kind", ["aff_from_coarser_image", "aff2_from_coarser_image",
                                  "up_kernel_from_upsampled_image", "down_kernel_in_up_sweep",
                                  "aff_normalised_by_fine_cells"])
def test_planted_wiring_mistakes_fail_the_pin(kind):
    L, shape = 4, (8, 8, 16)
    lab = _labels(shape, 20 + L)
    blob = _blob(L, 3 + L)
    ref = dense_from_operators(blob, L, lab)
    P = _plant(onet.Network(blob, L, lab), kind)
    V = np.random.default_rng(1).standard_normal((8,) + shape)   # a few inputs suffice to see it
    got = np.stack([P.apply(v).ravel() for v in V], axis=1)
    want = ref @ V.reshape(8, -1).T
    assert np.abs(got - want).max() > 1e-6 * np.abs(want).max()


# ---------------------------------------------------------------------------
# the asymmetry measure of the appendix on symmetry, on closed forms
# ---------------------------------------------------------------------------
class _Dense:
    """Stand-in for a network: any linear map given as a matrix."""

    def __init__(self, M):
        self.M = M

    def apply(self, v):
        return (self.M @ v.ravel()).reshape(v.shape)


def test_asymmetry_closed_form_two_cells():
    # M = diag(4, 9) + 3 (e1 e2^T - e2 e1^T): the symmetric part fixes the
    # denominator (x.Mx = 4, y.My = 9 for unit x, y), the skew part the
    # numerator (|x.My - y.Mx| = 2 * 3), so S = 6 / sqrt(36) = 1.
    M = np.array([[4.0, 3.0], [-3.0, 9.0]])
    x, y = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    assert onet.asymmetry(_Dense(M), x, y) == pytest.approx(1.0, rel=1e-15)
    # scale invariance in each argument and symmetry in (x, y)
    assert onet.asymmetry(_Dense(M), -2.5 * x, 0.5 * y) == pytest.approx(1.0, rel=1e-15)
    assert onet.asymmetry(_Dense(M), y, x) == pytest.approx(1.0, rel=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_asymmetry_symmetric_plus_skew(seed):
    # S = 2 |x^T K y| / sqrt(|x^T A x| |y^T A y|) for M = A + K, A symmetric
    # positive definite, K skew: the skew part cancels from x.Mx and y.My and
    # doubles in x.My - y.Mx.  Checked with a skew part of known size.
    rng = np.random.default_rng(seed)
    n = 7
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = rng.uniform(1.0, 5.0, n)
    A = (Q * lam) @ Q.T
    x, y = Q[:, 0], Q[:, 1]                                 # eigenvectors: x.Ax = lam0, y.Ay = lam1
    k = rng.uniform(0.1, 2.0)
    K = k * (np.outer(x, y) - np.outer(y, x))               # x^T K y = k (orthonormal x, y)
    expect = 2.0 * k / np.sqrt(lam[0] * lam[1])
    assert onet.asymmetry(_Dense(A + K), x, y) == pytest.approx(expect, rel=1e-12)
    assert onet.asymmetry(_Dense(A), x, y) == pytest.approx(0.0, abs=1e-14)
