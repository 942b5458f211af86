"""Seeded synthetic inputs for the neural-preconditioned Poisson solve.

This module only *draws* inputs: voxel label grids, right-hand sides and
network parameter blobs.  It holds none of the solver's or the network's
arithmetic, so the CPU oracle and the HIP path can both consume it without
sharing any of the method.

Label encoding (channel order of the image, Sec. "Spatial Discretization"):
    FLUID = 0, AIR = 1 (Dirichlet, p = 0), SOLID = 2 (Neumann).
Arrays are laid out (nz, ny, nx), x fastest; the free surface is along z.

The paper's scenes are not available; the generator below stands in for its
mixed-boundary water scenes (flat or wavy free surface, solid obstacles,
solid walls), with the paper's grid shapes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import ndimage

FLUID, AIR, SOLID = 0, 1, 2

__all__ = [
    "FLUID", "AIR", "SOLID", "SceneSpec", "gen_labels", "gen_rhs",
    "param_count", "xavier_params", "scene_c1", "scene_c2", "scene_c3",
    "scene_serving", "scene_gradcheck", "blob_layout",
]


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    """Parameters of the label generator.

    shape: (nz, ny, nx).  surface: ("flat", h_lo, h_hi) puts air at cell
    index z >= h with h ~ U{h_lo..h_hi}; ("sine", amplitude) puts air where
    z + 1/2 >= h0 + A sin(.) sin(.) with seeded frequencies and phases.
    Spheres (radius ~ U[r_lo, r_hi]) and 2-cell slabs are solid obstacles.
    """
    shape: tuple
    n_spheres: int
    r_range: tuple
    n_slabs: int
    surface: tuple


def scene_c1() -> SceneSpec:
    """32^3 plain-method scene: 6 spheres r in [2,6], flat surface in [16,28]."""
    return SceneSpec((32, 32, 32), 6, (2.0, 6.0), 0, ("flat", 16, 28))


def scene_c2(n: int = 128) -> SceneSpec:
    """128^3 single-solve scene: 20 spheres r in [4,20], 3 slabs, surface in [64,112]."""
    return scene_serving(n)


def scene_c3() -> SceneSpec:
    """256^3 scene: 60 spheres r in [8,40], 3 slabs, sinusoidal surface (amp 16)."""
    return SceneSpec((256, 256, 256), 60, (8.0, 40.0), 3, ("sine", 16.0))


def scene_serving(n: int) -> SceneSpec:
    """The 128^3 recipe with radii and surface range scaled by n/128."""
    s = n / 128.0
    return SceneSpec((n, n, n), 20, (4.0 * s, 20.0 * s), 3,
                     ("flat", int(round(64 * s)), int(round(112 * s))))


def scene_gradcheck() -> SceneSpec:
    """16^3 copy of the 32^3 recipe, halved: 3 spheres r in [1,3], surface in [8,14]."""
    return SceneSpec((16, 16, 16), 3, (1.0, 3.0), 0, ("flat", 8, 14))


def gen_labels(spec: SceneSpec, seed: int) -> np.ndarray:
    """Draw a uint8 label grid.  Priority SOLID > AIR > FLUID.

    Every fluid component is left touching air (unreached fluid becomes solid),
    so the reduced Laplacian of the scene is positive definite.
    """
    rng = np.random.default_rng(seed)
    nz, ny, nx = spec.shape
    lab = np.full(spec.shape, FLUID, dtype=np.uint8)
    zc = (np.arange(nz) + 0.5)[:, None, None]
    yc = (np.arange(ny) + 0.5)[None, :, None]
    xc = (np.arange(nx) + 0.5)[None, None, :]

    kind = spec.surface[0]
    if kind == "flat":
        h = int(rng.integers(spec.surface[1], spec.surface[2] + 1))
        lab[np.arange(nz) >= h] = AIR
    elif kind == "sine":
        amp = float(spec.surface[1])
        fx, fy = rng.integers(1, 4, size=2)
        px, py = rng.uniform(0.0, 2.0 * math.pi, size=2)
        h0 = rng.uniform(nz / 2 + amp, 7 * nz / 8 - amp)
        h = h0 + amp * np.sin(2 * math.pi * fx * xc / nx + px) * np.sin(2 * math.pi * fy * yc / ny + py)
        lab[np.broadcast_to(zc >= h, spec.shape)] = AIR
    else:
        raise ValueError(f"unknown surface kind {kind!r}")

    solid = np.zeros(spec.shape, dtype=bool)
    for _ in range(spec.n_spheres):
        c = rng.uniform(0.0, 1.0, size=3) * np.array([nz, ny, nx])
        rad = rng.uniform(spec.r_range[0], spec.r_range[1])
        solid |= ((zc - c[0]) ** 2 + (yc - c[1]) ** 2 + (xc - c[2]) ** 2) <= rad * rad

    dims = (nz, ny, nx)
    for _ in range(spec.n_slabs):
        ax = int(rng.integers(0, 3))
        pos = int(rng.integers(2, dims[ax] - 3))
        sl = [slice(None)] * 3
        sl[ax] = slice(pos, pos + 2)
        for other in (a for a in range(3) if a != ax):
            n = dims[other]
            length = int(rng.integers(n // 4, 3 * n // 4 + 1))
            off = int(rng.integers(0, n - length + 1))
            sl[other] = slice(off, off + length)
        solid[tuple(sl)] = True

    solid[0, :, :] = solid[-1, :, :] = True
    solid[:, 0, :] = solid[:, -1, :] = True
    solid[:, :, 0] = solid[:, :, -1] = True
    lab[solid] = SOLID

    # Keep only fluid components that touch air.
    fluid = lab == FLUID
    comp, ncomp = ndimage.label(fluid, structure=ndimage.generate_binary_structure(3, 1))
    if ncomp:
        air = lab == AIR
        near_air = ndimage.binary_dilation(air, structure=ndimage.generate_binary_structure(3, 1))
        keep = np.unique(comp[fluid & near_air])
        keep_mask = np.zeros(ncomp + 1, dtype=bool)
        keep_mask[keep] = True
        keep_mask[0] = False
        lab[fluid & ~keep_mask[comp]] = SOLID
    if not (lab == FLUID).any():
        raise ValueError("scene has no fluid cell")
    return lab


def gen_rhs(labels: np.ndarray, seed: int, normalize: bool = False) -> np.ndarray:
    """N(0,1) on fluid cells, zero elsewhere (float64); optionally unit 2-norm."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(labels.shape)
    b[labels != FLUID] = 0.0
    if normalize:
        b /= np.linalg.norm(b)
    return b


# ---------------------------------------------------------------------------
# Parameter blob.  Order (float64, little-endian):
#   for l = 1..L  : CConv_1^l  W[27,3,3,3,3], B[27]
#   for l = 1..L-1: CConv_2^l  W[27,3,3,3,3], B[27]
#   for l = 1..L-1: Aff_1^l    Wbar[3,3,3,3], Bbar[1];  Aff_2^l  Wbar, Bbar
# W[t, c, oz+1, oy+1, ox+1]: t = 9(az+1) + 3(ay+1) + (ax+1) is the kernel tap,
# c the image channel and o the image-window offset.
# ---------------------------------------------------------------------------
CCONV_W = 27 * 3 * 27
CCONV_B = 27
AFF_W = 3 * 27
AFF_B = 1


def param_count(levels: int) -> int:
    return (2 * levels - 1) * (CCONV_W + CCONV_B) + 2 * (levels - 1) * (AFF_W + AFF_B)


def blob_layout(levels: int) -> list:
    """[(name, level, offset, size)] in blob order; names: c1W c1B c2W c2B a1W a1B a2W a2B."""
    out, off = [], 0

    def put(name, lvl, size):
        nonlocal off
        out.append((name, lvl, off, size))
        off += size

    for lvl in range(1, levels + 1):
        put("c1W", lvl, CCONV_W)
        put("c1B", lvl, CCONV_B)
    for lvl in range(1, levels):
        put("c2W", lvl, CCONV_W)
        put("c2B", lvl, CCONV_B)
    for lvl in range(1, levels):
        put("a1W", lvl, AFF_W)
        put("a1B", lvl, AFF_B)
        put("a2W", lvl, AFF_W)
        put("a2B", lvl, AFF_B)
    assert off == param_count(levels)
    return out


def xavier_params(levels: int, seed: int = 0) -> np.ndarray:
    """Seeded Xavier-uniform weights, zero biases, drawn in blob order.

    Conv fan convention: CConv W as a (27 out, 3 in, 3,3,3) conv has
    fan_in 81, fan_out 729; Aff Wbar as (1, 3, 3,3,3) has fan_in 81, fan_out 27.
    """
    rng = np.random.default_rng(seed)
    blob = np.zeros(param_count(levels), dtype=np.float64)
    bound_c = math.sqrt(6.0 / (81 + 729))
    bound_a = math.sqrt(6.0 / (81 + 27))
    for name, _lvl, off, size in blob_layout(levels):
        if name in ("c1W", "c2W"):
            blob[off:off + size] = rng.uniform(-bound_c, bound_c, size)
        elif name in ("a1W", "a2W"):
            blob[off:off + size] = rng.uniform(-bound_a, bound_a, size)
    return blob


def centre_tap_params(levels: int, scales_1, scales_2, aff1_bias, aff2_bias) -> np.ndarray:
    """Blob whose kernels are spatially constant centre taps (all W = 0).

    CConv_1^l gets bias scales_1[l-1] on the centre tap, CConv_2^l gets
    scales_2[l-1]; Aff_i^l is the constant aff{i}_bias[l-1].  With ones for
    the level-1 scales and Aff_1, and zero for Aff_2, the network is the fluid
    mask (the identity preconditioner on the reduced system).
    """
    blob = np.zeros(param_count(levels), dtype=np.float64)
    centre = 13
    for name, lvl, off, size in blob_layout(levels):
        if name == "c1B":
            blob[off + centre] = scales_1[lvl - 1]
        elif name == "c2B":
            blob[off + centre] = scales_2[lvl - 1]
        elif name == "a1B":
            blob[off] = aff1_bias[lvl - 1]
        elif name == "a2B":
            blob[off] = aff2_bias[lvl - 1]
    return blob


def identity_params(levels: int) -> np.ndarray:
    """Blob for which the network output is r restricted to fluid cells."""
    ones = [1.0] * levels
    return centre_tap_params(levels, ones, ones, [1.0] * (levels - 1), [0.0] * (levels - 1))


def multilevel_params(levels: int, coarse_gain: float = 4.0, fluid_weight: float = 0.5) -> np.ndarray:
    """A hand-set blob that makes the network an additive multilevel preconditioner.

    Seeded Xavier weights are not a preconditioner (the iteration stalls), and
    the paper's trained weights are not available, so this blob stands in for
    them when a convergence-based measurement needs a working P.  All kernels
    are centre taps: CConv_2 and level-1 CConv_1 pass values through, CConv_1
    at coarser levels scales by (1 - w) + w * fluid fraction of the coarse
    cell, Aff_1 = 1 and Aff_2 = coarse_gain (a 4^(l-1) level weighting, the
    h^2 scaling of a multilevel diagonal preconditioner in unit spacing).
    """
    ones = [1.0] * levels
    blob = centre_tap_params(levels, ones, ones, [1.0] * (levels - 1), [coarse_gain] * (levels - 1))
    centre = 13
    for name, lvl, off, size in blob_layout(levels):
        if lvl == 1:
            continue
        if name == "c1W":
            # W[t=centre, c=fluid, o=(0,0,0)]
            blob[off + ((centre * 3 + FLUID) * 27 + 13)] += fluid_weight
        elif name == "c1B":
            blob[off + centre] -= fluid_weight
    return blob
