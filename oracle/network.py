"""The spatially-varying-kernel network (oracle, FP64).

Follows Alg. 2 (operations of an L-level network), the CConv and Aff formulas
of Sec. "Architecture" extended to 3D as the paper prescribes (one more index
in every sum), the pad/unpad rule of Sec. "Neural Preconditioner" (input zero
outside fluid, output restricted to fluid), 2x average pooling, and 2x
trilinear interpolation (the 3D analogue of the paper's bilinear upsampling).

Index conventions (readings of the garbled 2D formula, see design notes):
  * image channel c: 0 fluid, 1 air, 2 solid; padding value (0, 0, 1).
  * kernel tap t = 9(az+1) + 3(ay+1) + (ax+1) for offset a = (az, ay, ax).
  * W[t, c, oz+1, oy+1, ox+1]: weight of image channel c at window offset o.
  * both the kernel generation and its application are correlations (+offsets).

TEST INFRASTRUCTURE ONLY: never called by the product path.
"""
from __future__ import annotations

import numpy as np

from .laplacian import shifted, FLUID

OFFSETS = [(az, ay, ax) for az in (-1, 0, 1) for ay in (-1, 0, 1) for ax in (-1, 0, 1)]
SOLID_PAD = (0.0, 0.0, 1.0)


# --------------------------------------------------------------------------
# parameters
# --------------------------------------------------------------------------
def n_params(levels: int) -> int:
    """(2L-1) CConv blocks of 27*81 weights + 27 biases, 2(L-1) Aff blocks of 81 + 1."""
    return (2 * levels - 1) * (27 * 81 + 27) + 2 * (levels - 1) * (81 + 1)


def unpack(params: np.ndarray, levels: int) -> dict:
    """Split a flat float64 blob into per-level blocks.

    Order: CConv_1^l (W, B) for l = 1..L; CConv_2^l (W, B) for l = 1..L-1;
    then for l = 1..L-1: Aff_1^l (Wbar, Bbar), Aff_2^l (Wbar, Bbar).
    Lists are indexed by level - 1.
    """
    p = np.asarray(params, dtype=np.float64)
    if p.size != n_params(levels):
        raise ValueError(f"blob has {p.size} entries, expected {n_params(levels)}")
    pos = 0

    def take(n, shape):
        nonlocal pos
        out = p[pos:pos + n].reshape(shape)
        pos += n
        return out

    net = {"L": levels, "c1W": [], "c1B": [], "c2W": [], "c2B": [],
           "a1W": [], "a1B": [], "a2W": [], "a2B": []}
    for _ in range(levels):
        net["c1W"].append(take(27 * 81, (27, 3, 3, 3, 3)))
        net["c1B"].append(take(27, (27,)))
    for _ in range(levels - 1):
        net["c2W"].append(take(27 * 81, (27, 3, 3, 3, 3)))
        net["c2B"].append(take(27, (27,)))
    for _ in range(levels - 1):
        net["a1W"].append(take(81, (3, 3, 3, 3)))
        net["a1B"].append(float(take(1, (1,))[0]))
        net["a2W"].append(take(81, (3, 3, 3, 3)))
        net["a2B"].append(float(take(1, (1,))[0]))
    assert pos == p.size
    return net


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------
def image(labels: np.ndarray) -> np.ndarray:
    """3-channel indicator image of the fluid / air / solid partition (channels sum to 1)."""
    return np.stack([(labels == c).astype(np.float64) for c in range(3)])


def pool(v: np.ndarray) -> np.ndarray:
    """Average pooling with a 2x2x2 window and stride 2 over the last three axes."""
    *lead, nz, ny, nx = v.shape
    w = v.reshape(*lead, nz // 2, 2, ny // 2, 2, nx // 2, 2)
    return w.mean(axis=(-5, -3, -1))


def _upsample_axis(v: np.ndarray, axis: int) -> np.ndarray:
    """Linear 2x upsampling of cell-centred data along one axis, edges clamped.

    Fine cell 2j sits a quarter cell below coarse cell j, fine cell 2j+1 a
    quarter above: 2j -> 3/4 c[j] + 1/4 c[j-1], 2j+1 -> 3/4 c[j] + 1/4 c[j+1],
    with c[-1] = c[0] and c[n] = c[n-1].
    """
    n = v.shape[axis]
    j = np.arange(n)
    below = np.take(v, np.clip(j - 1, 0, n - 1), axis=axis)
    above = np.take(v, np.clip(j + 1, 0, n - 1), axis=axis)
    even = 0.75 * v + 0.25 * below
    odd = 0.75 * v + 0.25 * above
    out = np.stack([even, odd], axis=axis + 1)
    shape = list(v.shape)
    shape[axis] = 2 * n
    return out.reshape(shape)


def interpolate(v: np.ndarray) -> np.ndarray:
    """Trilinear 2x upsampling (align_corners=False), separable over the last three axes."""
    out = v
    for axis in (-3, -2, -1):
        out = _upsample_axis(out, out.ndim + axis)
    return out


def image_window(I: np.ndarray, off) -> np.ndarray:
    """I(p + off) for all p, with the image padded by solid cells."""
    return np.stack([shifted(I[c], off, SOLID_PAD[c]) for c in range(3)])


def cconv_kernels(I: np.ndarray, W: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Per-cell kernels K[t](p) = B_t + sum_c sum_o W[t, c, o] I_c(p + o).

    The affine map from the 3x3x3 image window to the 27 kernel taps of a
    CConv block.  Returns shape (27, nz, ny, nx).
    """
    shape = I.shape[1:]
    K = np.repeat(B.reshape(27, 1), int(np.prod(shape)), axis=1)
    for o in OFFSETS:
        win = image_window(I, o).reshape(3, -1)                 # (3, n)
        w_o = W[:, :, o[0] + 1, o[1] + 1, o[2] + 1]            # (27, 3)
        K += w_o @ win
    return K.reshape((27,) + shape)


def cconv_apply(K: np.ndarray, r: np.ndarray) -> np.ndarray:
    """out(p) = sum_t K[t](p) r(p + a_t), r padded with zeros."""
    out = np.zeros(r.shape)
    for t, a in enumerate(OFFSETS):
        out += K[t] * shifted(r, a, 0.0)
    return out


def cconv(I, W, B, r):
    """One CConv block: spatially varying 3x3x3 correlation of r with kernels from I."""
    return cconv_apply(cconv_kernels(I, W, B), r)


def aff(I: np.ndarray, Wbar: np.ndarray, Bbar: float) -> float:
    """Aff block: Bbar + (1 / (27 n_l)) sum_p sum_c sum_o Wbar[c, o] I_c(p + o).

    n_l is the number of cells of the level the image lives on; the image is
    padded with solid cells as for CConv.
    """
    n_l = int(np.prod(I.shape[1:]))
    total = 0.0
    for o in OFFSETS:
        win = image_window(I, o)
        for c in range(3):
            total += Wbar[c, o[0] + 1, o[1] + 1, o[2] + 1] * win[c].sum()
    return Bbar + total / (27.0 * n_l)


def image_pyramid(labels: np.ndarray, levels: int) -> list:
    """I^1 = image(labels); I^{l+1} = Pool(I^l)."""
    I = [image(labels)]
    for _ in range(levels - 1):
        I.append(pool(I[-1]))
    return I


def check_shape(shape, levels: int) -> None:
    """Every grid dimension must be divisible by 2^(L-1) (Sec. "Architecture")."""
    m = 2 ** (levels - 1)
    if any(s % m for s in shape):
        raise ValueError(f"grid {shape} not divisible by 2^(L-1) = {m}")


# --------------------------------------------------------------------------
# the network
# --------------------------------------------------------------------------
class Network:
    """P(I, .) for one image.  Kernels and Aff scalars depend only on the image
    and the weights, so they are formed once here and reused by every apply."""

    def __init__(self, params: np.ndarray, levels: int, labels: np.ndarray):
        check_shape(labels.shape, levels)
        self.L = levels
        self.net = unpack(params, levels)
        self.fluid = labels == FLUID
        self.I = image_pyramid(labels, levels)
        n = self.net
        self.K1 = [cconv_kernels(self.I[l], n["c1W"][l], n["c1B"][l]) for l in range(levels)]
        self.K2 = [cconv_kernels(self.I[l], n["c2W"][l], n["c2B"][l]) for l in range(levels - 1)]
        self.c1 = [aff(self.I[l], n["a1W"][l], n["a1B"][l]) for l in range(levels - 1)]
        self.c2 = [aff(self.I[l], n["a2W"][l], n["a2B"][l]) for l in range(levels - 1)]

    def apply(self, r: np.ndarray, acts: dict | None = None) -> np.ndarray:
        """Alg. 2 on input r (zeroed outside fluid first); output restricted to fluid."""
        L = self.L
        rr = np.where(self.fluid, r, 0.0)
        x1 = []
        r1 = [rr]
        for l in range(L - 1):                       # down sweep
            x1.append(cconv_apply(self.K1[l], rr))
            rr = pool(x1[l])
            r1.append(rr)
        x = cconv_apply(self.K1[L - 1], rr)          # coarsest level
        xs = [None] * L
        xs[L - 1] = x
        r2 = [None] * (L - 1)
        x2s = [None] * (L - 1)
        for l in range(L - 2, -1, -1):               # up sweep
            r2[l] = interpolate(x)
            x2s[l] = cconv_apply(self.K2[l], r2[l])
            x = self.c1[l] * x1[l] + self.c2[l] * x2s[l]
            xs[l] = x
        if acts is not None:
            acts.update(r1=r1, x1=x1, r2=r2, x2=x2s, x=xs)
        return np.where(self.fluid, x, 0.0)


def forward(params: np.ndarray, levels: int, labels: np.ndarray, r: np.ndarray) -> np.ndarray:
    """One network evaluation P(I, r)."""
    return Network(params, levels, labels).apply(r)


def asymmetry(net: Network, x: np.ndarray, y: np.ndarray) -> float:
    """S(x, y; I) = |x.P(y) - y.P(x)| / sqrt(|x.P(x)| |y.P(y)|) (appendix on symmetry)."""
    px, py = net.apply(x), net.apply(y)
    return abs(x.ravel() @ py.ravel() - y.ravel() @ px.ravel()) / np.sqrt(
        abs(x.ravel() @ px.ravel()) * abs(y.ravel() @ py.ravel()))
