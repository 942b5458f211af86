"""Training loss of Sec. "Training" and its gradient by a hand-written adjoint (oracle, FP64).

Loss for one system: || b - A P(I, b) ||_2 (b restricted to fluid).  The
gradient with respect to every parameter of the blob is obtained by running
Alg. 2 backwards:
  * CConv out(p) = sum_t K_t(p) r(p + a_t), K_t(p) = B_t + sum_{c,o} W[t,c,o] I_c(p + o):
      dL/dB_t      = sum_p g(p) r(p + a_t)
      dL/dW[t,c,o] = sum_p g(p) r(p + a_t) I_c(p + o)
      dL/dr(q)     = sum_t K_t(q - a_t) g(q - a_t)        (the transposed apply)
  * pooling and upsampling are linear maps; their adjoints are applied exactly
    (the adjoint of the 2x average pool spreads g/8 to the 8 children; the
    adjoint of the separable linear upsampling is built axis by axis);
  * Aff c = Bbar + (1/(27 n)) sum_p sum_c sum_o Wbar[c,o] I_c(p+o):
      dL/dBbar = dL/dc,  dL/dWbar[c,o] = dL/dc * sum_p I_c(p+o) / (27 n).
The matrix A of Sec. "Spatial Discretization" is symmetric, so A^T = A.

TEST INFRASTRUCTURE ONLY: never called by the product path.
"""
from __future__ import annotations

import numpy as np

from . import laplacian
from .laplacian import shifted
from .network import OFFSETS, Network, image_window, unpack


def _pack(net: dict, grads: dict, levels: int) -> np.ndarray:
    """Flatten per-block gradients in the blob order of network.unpack."""
    parts = []
    for l in range(levels):
        parts += [grads["c1W"][l].ravel(), grads["c1B"][l].ravel()]
    for l in range(levels - 1):
        parts += [grads["c2W"][l].ravel(), grads["c2B"][l].ravel()]
    for l in range(levels - 1):
        parts += [grads["a1W"][l].ravel(), np.array([grads["a1B"][l]]),
                  grads["a2W"][l].ravel(), np.array([grads["a2B"][l]])]
    return np.concatenate(parts)


def cconv_apply_transpose(K: np.ndarray, g: np.ndarray) -> np.ndarray:
    """dL/dr(q) = sum_t K_t(q - a_t) g(q - a_t), zero outside the grid."""
    out = np.zeros(g.shape)
    for t, a in enumerate(OFFSETS):
        out += shifted(K[t] * g, (-a[0], -a[1], -a[2]), 0.0)
    return out


def cconv_param_grads(I: np.ndarray, r: np.ndarray, g: np.ndarray):
    """(dL/dW, dL/dB) of one CConv block from its input r, image I and output gradient g."""
    gW = np.zeros((27, 3, 3, 3, 3))
    gB = np.zeros(27)
    u = np.stack([g * shifted(r, a, 0.0) for a in OFFSETS])           # u_t(p) = g(p) r(p + a_t)
    gB[:] = u.reshape(27, -1).sum(axis=1)
    for o in OFFSETS:
        win = image_window(I, o).reshape(3, -1)                        # I_c(p + o)
        gW[:, :, o[0] + 1, o[1] + 1, o[2] + 1] = u.reshape(27, -1) @ win.T
    return gW, gB


def pool_transpose(g: np.ndarray) -> np.ndarray:
    """Adjoint of the 2x2x2 average pool: each child receives g(parent) / 8."""
    return np.repeat(np.repeat(np.repeat(g, 2, axis=-3), 2, axis=-2), 2, axis=-1) / 8.0


def _upsample_axis_transpose(g: np.ndarray, axis: int) -> np.ndarray:
    """Adjoint of network._upsample_axis along one axis."""
    n2 = g.shape[axis]
    n = n2 // 2
    even = np.take(g, np.arange(0, n2, 2), axis=axis)
    odd = np.take(g, np.arange(1, n2, 2), axis=axis)
    out = 0.75 * even + 0.75 * odd
    j = np.arange(n)
    below = np.clip(j - 1, 0, n - 1)     # even fine cell 2j also feeds coarse j-1 (clamped)
    above = np.clip(j + 1, 0, n - 1)     # odd fine cell 2j+1 also feeds coarse j+1 (clamped)
    for src, idx in ((even, below), (odd, above)):
        moved = np.zeros_like(out)
        np.add.at(moved, (slice(None),) * (axis % out.ndim) + (idx,), 0.25 * src)
        out = out + moved
    return out


def interpolate_transpose(g: np.ndarray) -> np.ndarray:
    out = g
    for axis in (-1, -2, -3):
        out = _upsample_axis_transpose(out, out.ndim + axis)
    return out


def transpose_apply(net: Network, g: np.ndarray) -> np.ndarray:
    """P(I, .)^T g: the adjoint of the network in its input vector.

    P is linear in r (kernels and Aff scalars depend on the image only), so
    its adjoint is Alg. 2 run backwards with every linear step replaced by its
    adjoint: the output restriction to fluid, c1 and c2, the transposed CConv
    applies, the adjoints of upsampling and pooling, and the input
    restriction to fluid.  This is the symmetric variant's second half
    (P_sym = P^T o P, appendix on symmetry).
    """
    L = net.L
    gx = np.where(net.fluid, g, 0.0)
    gx1 = [None] * L
    for l in range(L - 1):                       # up sweep, reversed
        gx1[l] = net.c1[l] * gx
        gr2 = cconv_apply_transpose(net.K2[l], net.c2[l] * gx)
        gx = interpolate_transpose(gr2)
    gx1[L - 1] = gx                              # coarsest: x^L = x1^L
    gr = None
    for l in range(L - 1, -1, -1):               # down sweep, reversed
        gl = gx1[l] if gr is None else gx1[l] + pool_transpose(gr)
        gr = cconv_apply_transpose(net.K1[l], gl)
    return np.where(net.fluid, gr, 0.0)


def loss_and_grad(params: np.ndarray, levels: int, labels: np.ndarray, b: np.ndarray):
    """(loss, gradient blob) of || b - A P(I, b) ||_2 for one system."""
    L = levels
    net = unpack(params, L)
    P = Network(params, L, labels)
    fluid = labels == laplacian.FLUID
    bf = np.where(fluid, b, 0.0)
    acts = {}
    y = P.apply(bf, acts)
    res = bf - laplacian.matvec(labels, y)
    loss = float(np.linalg.norm(res))
    g_y = -laplacian.matvec(labels, res) / loss             # A is symmetric
    g_x = [None] * L                                          # gradients of x^l (up-sweep outputs)
    g_x1 = [np.zeros(P.I[l].shape[1:]) for l in range(L)]
    grads = {k: [None] * L for k in ("c1W", "c1B", "c2W", "c2B", "a1W", "a1B", "a2W", "a2B")}
    g_x[0] = np.where(fluid, g_y, 0.0)
    # up sweep, reversed
    for l in range(L - 1):
        I = P.I[l]
        x1, r2, x2 = acts["x1"][l], acts["r2"][l], acts["x2"][l]
        g = g_x[l]
        g_c1, g_c2 = float(np.sum(g * x1)), float(np.sum(g * x2))
        g_x1[l] += P.c1[l] * g
        g_x2 = P.c2[l] * g
        grads["c2W"][l], grads["c2B"][l] = cconv_param_grads(I, r2, g_x2)
        g_r2 = cconv_apply_transpose(P.K2[l], g_x2)
        g_x[l + 1] = interpolate_transpose(g_r2)
        n_l = int(np.prod(I.shape[1:]))
        S = np.zeros((3, 3, 3, 3))
        for o in OFFSETS:
            S[:, o[0] + 1, o[1] + 1, o[2] + 1] = image_window(I, o).reshape(3, -1).sum(axis=1)
        grads["a1W"][l], grads["a1B"][l] = g_c1 * S / (27.0 * n_l), g_c1
        grads["a2W"][l], grads["a2B"][l] = g_c2 * S / (27.0 * n_l), g_c2
    # coarsest level: x^L = x1^L
    g_x1[L - 1] += g_x[L - 1]
    # down sweep, reversed
    for l in range(L - 1, -1, -1):
        r1 = acts["r1"][l]
        grads["c1W"][l], grads["c1B"][l] = cconv_param_grads(P.I[l], r1, g_x1[l])
        if l > 0:
            g_r1 = cconv_apply_transpose(P.K1[l], g_x1[l])
            g_x1[l - 1] += pool_transpose(g_r1)
    return loss, _pack(net, grads, L)


def batch_loss_and_grad(params, levels, labels_list, b_list):
    """Mean loss and mean gradient over a batch of systems."""
    tot, gtot = 0.0, 0.0
    for lab, b in zip(labels_list, b_list):
        loss, g = loss_and_grad(params, levels, lab, b)
        tot, gtot = tot + loss, gtot + g
    n = len(labels_list)
    return tot / n, gtot / n


def loss_only(params, levels, labels, b) -> float:
    fluid = labels == laplacian.FLUID
    bf = np.where(fluid, b, 0.0)
    y = Network(params, levels, labels).apply(bf)
    return float(np.linalg.norm(bf - laplacian.matvec(labels, y)))
