"""Learned warm start: the convolutional encoder-decoder, its loss and its
optimiser, in FP64 on the CPU (TEST INFRASTRUCTURE ONLY).

The paper solves every microstructure from the initial guess u0 = 0 (the
Newton scheme of Alg. 1 starts from a given u_(0); a linear problem is one
PCG solve from it).  The warm start replaces that zero by the output of a
small network evaluated on the phase field; PCG from zero stays the fallback
and the screen.  Nothing of the network is in the paper, so this module is
the definition the GPU path is checked against:

  * features per voxel: chi = [phase == 1], gamma * chi, gamma, with
    gamma = log10(E_inclusion / E_matrix) / 3 given per sample;
  * four levels of 16/32/64/64 channels at n, n/2, n/4, n/8 voxels per axis;
    two 3x3x3 convolutions with periodic wrap and a leaky ReLU (slope 1/8)
    per level; 2x2x2 average pooling down, nearest-neighbour up-sampling
    concatenated with the skip of the same level ([up, skip]) on the way up;
  * a 1x1x1 head with 18 outputs: the fluctuation of the 6 unit Mandel
    strains times 3 components (load-major), in voxel units u * n / l;
  * loss: the squared periodic forward differences of (output - target),
    averaged over samples, channels, voxels and the 3 directions (an H^1
    semi-norm, blind to the per-component constant the fluctuation is only
    defined up to);
  * Adam (Kingma and Ba, 2015) with bias correction.

Convolution: y[o, v] = b[o] + sum_t sum_c W[t, o, c] x[c, v + d_t], where
tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1) has offset d_t = (dz, dy, dx)
and indices wrap periodically.

Storage precision of the GPU path is reproduced when `emulate` is true:
weights, biases, the features, every activation and every activation
gradient are rounded to BF16 (round to nearest even) where the GPU stores
them; all arithmetic here stays FP64.  With `emulate` false the network is
exact FP64 (used for the finite-difference and autograd pins).

Flat parameter vector: for each layer of LAYERS in order, W[27][cout][cin]
then b[cout]; then the head Wh[18][16] and bh[18].
"""
from __future__ import annotations

import numpy as np
import torch

SLOPE = 0.125
NOUT = 18
LAYERS = (
    ("e0a", 3, 16, 0), ("e0b", 16, 16, 0),
    ("e1a", 16, 32, 1), ("e1b", 32, 32, 1),
    ("e2a", 32, 64, 2), ("e2b", 64, 64, 2),
    ("b3a", 64, 64, 3), ("b3b", 64, 64, 3),
    ("d2a", 128, 64, 2), ("d2b", 64, 64, 2),
    ("d1a", 96, 32, 1), ("d1b", 32, 32, 1),
    ("d0a", 48, 16, 0), ("d0b", 16, 16, 0),
)
HEAD_IN = 16
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def param_count() -> int:
    n = sum(27 * ci * co + co for _, ci, co, _ in LAYERS)
    return n + NOUT * HEAD_IN + NOUT


def unflatten(flat):
    """Flat vector -> {name: (W [27][cout][cin], b [cout])}, plus 'head'."""
    if not isinstance(flat, torch.Tensor):
        flat = torch.as_tensor(np.asarray(flat, dtype=np.float64))
    out, k = {}, 0
    for name, ci, co, _ in LAYERS:
        W = flat[k:k + 27 * co * ci].reshape(27, co, ci)
        k += 27 * co * ci
        b = flat[k:k + co]
        k += co
        out[name] = (W, b)
    Wh = flat[k:k + NOUT * HEAD_IN].reshape(NOUT, HEAD_IN)
    k += NOUT * HEAD_IN
    out["head"] = (Wh, flat[k:k + NOUT])
    return out


def flatten(grads) -> np.ndarray:
    parts = []
    for name, _, _, _ in LAYERS:
        W, b = grads[name]
        parts += [W.reshape(-1), b.reshape(-1)]
    Wh, bh = grads["head"]
    parts += [Wh.reshape(-1), bh.reshape(-1)]
    return torch.cat(parts).numpy()


# seeded initial weights are inputs: drawn by the shared input generators
from synth.netinit import init_params  # noqa: E402,F401


def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to the nearest BF16 value (ties to even), returned in FP64."""
    return x.to(torch.bfloat16).to(torch.float64)


def _r(x, emulate):
    return bf16(x) if emulate else x


def features(phase: np.ndarray, gamma) -> torch.Tensor:
    """[B][3][s][s][s]: chi, gamma chi, gamma."""
    ph = torch.as_tensor(np.asarray(phase))
    chi = (ph == 1).to(torch.float64)
    g = torch.as_tensor(np.asarray(gamma, dtype=np.float64)).view(-1, 1, 1, 1)
    return torch.stack([chi, g * chi, g.expand_as(chi)], dim=1)


def conv(x, W, b):
    """Periodic 3x3x3 correlation, the definition in the module docstring."""
    y = b.view(1, -1, 1, 1, 1).expand(x.shape[0], -1, *x.shape[2:]).clone()
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = torch.roll(x, shifts=(-dz, -dy, -dx), dims=(2, 3, 4))   # xs[v] = x[v + d]
        y += torch.einsum("oc,bczyx->bozyx", W[t], xs)
    return y


def conv_input_grad(dy, W):
    """Adjoint of conv in x: dx[c, v] = sum_t sum_o W[t, o, c] dy[o, v - d_t]."""
    dx = None
    for t, (dz, dyy, ddx) in enumerate(TAPS):
        ds = torch.roll(dy, shifts=(dz, dyy, ddx), dims=(2, 3, 4))   # ds[v] = dy[v - d]
        term = torch.einsum("oc,bozyx->bczyx", W[t], ds)
        dx = term if dx is None else dx + term
    return dx


def conv_weight_grad(x, dy):
    """dW[t, o, c] = sum_v dy[o, v] x[c, v + d_t]; db[o] = sum_v dy[o, v]."""
    dW = torch.zeros(27, dy.shape[1], x.shape[1], dtype=torch.float64)
    for t, (dz, dyy, dx) in enumerate(TAPS):
        xs = torch.roll(x, shifts=(-dz, -dyy, -dx), dims=(2, 3, 4))
        dW[t] = torch.einsum("bozyx,bczyx->oc", dy, xs)
    return dW, dy.sum(dim=(0, 2, 3, 4))


def leaky(z):
    return torch.where(z > 0, z, SLOPE * z)


def leaky_grad_from_output(y):
    """Derivative of the leaky ReLU at the pre-activation, read off its
    output (same sign); slope 1/8 is taken at zero."""
    return torch.where(y > 0, torch.ones_like(y), torch.full_like(y, SLOPE))


def pool(x):
    B, C, s = x.shape[0], x.shape[1], x.shape[2]
    h = s // 2
    return x.reshape(B, C, h, 2, h, 2, h, 2).mean(dim=(3, 5, 7))


def up(x):
    return x.repeat_interleave(2, 2).repeat_interleave(2, 3).repeat_interleave(2, 4)


def up_adjoint(y):
    """Sum of the 8 children: the adjoint of nearest up-sampling."""
    B, C, s = y.shape[0], y.shape[1], y.shape[2]
    h = s // 2
    return y.reshape(B, C, h, 2, h, 2, h, 2).sum(dim=(3, 5, 7))


def forward(params, phase, gamma, emulate: bool = False):
    """Network output O [B][18][s][s][s] and the cache for backward."""
    P = unflatten(params)
    R = lambda t: _r(t, emulate)  # noqa: E731
    Wt = {k: (R(W), R(b)) for k, (W, b) in P.items()}
    c = {"I": R(features(phase, gamma))}

    def block(name, x):
        W, b = Wt[name]
        return R(leaky(conv(x, W, b)))

    c["e0a"] = block("e0a", c["I"]);   c["e0"] = block("e0b", c["e0a"])
    c["p0"] = R(pool(c["e0"]))
    c["e1a"] = block("e1a", c["p0"]);  c["e1"] = block("e1b", c["e1a"])
    c["p1"] = R(pool(c["e1"]))
    c["e2a"] = block("e2a", c["p1"]);  c["e2"] = block("e2b", c["e2a"])
    c["p2"] = R(pool(c["e2"]))
    c["b3a"] = block("b3a", c["p2"]);  c["b3"] = block("b3b", c["b3a"])
    c["c2"] = torch.cat([up(c["b3"]), c["e2"]], dim=1)
    c["d2a"] = block("d2a", c["c2"]);  c["d2"] = block("d2b", c["d2a"])
    c["c1"] = torch.cat([up(c["d2"]), c["e1"]], dim=1)
    c["d1a"] = block("d1a", c["c1"]);  c["d1"] = block("d1b", c["d1a"])
    c["c0"] = torch.cat([up(c["d1"]), c["e0"]], dim=1)
    c["d0a"] = block("d0a", c["c0"]);  c["d0"] = block("d0b", c["d0a"])
    Wh, bh = Wt["head"]
    O = torch.einsum("oc,bczyx->bozyx", Wh, c["d0"]) + bh.view(1, -1, 1, 1, 1)
    c["W"] = Wt
    return O, c


def loss(O, T):
    """Mean over samples, channels, voxels and directions of (D_d (O - T))^2,
    D_d e[v] = e[v + e_d] - e[v] with periodic wrap."""
    e = O - T
    tot = 0.0
    for d in (2, 3, 4):
        tot = tot + ((torch.roll(e, -1, d) - e) ** 2).sum()
    return tot / (3.0 * e.numel())


def loss_grad(O, T):
    """dL/dO = (2 / M) sum_d (2 e[v] - e[v - e_d] - e[v + e_d]), M = 3 numel."""
    e = O - T
    g = torch.zeros_like(e)
    for d in (2, 3, 4):
        g += 2.0 * e - torch.roll(e, 1, d) - torch.roll(e, -1, d)
    return g * (2.0 / (3.0 * e.numel()))


def backward(cache, dO, emulate: bool = False):
    """Gradients of the loss w.r.t. every parameter, given dL/dO (the
    reverse of forward, step by step)."""
    R = lambda t: _r(t, emulate)  # noqa: E731
    Wt = cache["W"]
    g = {}
    Wh, _ = Wt["head"]
    g["head"] = (torch.einsum("bozyx,bczyx->oc", dO, cache["d0"]), dO.sum(dim=(0, 2, 3, 4)))
    mask = leaky_grad_from_output
    dz = R(mask(cache["d0"]) * torch.einsum("oc,bozyx->bczyx", Wh, dO))

    def layer(name, x, dzz, input_is_activation=True):
        W, _ = Wt[name]
        g[name] = conv_weight_grad(x, dzz)
        dx = conv_input_grad(dzz, W)
        return R(mask(x) * dx) if input_is_activation else R(dx)

    dz = layer("d0b", cache["d0a"], dz)
    dc0 = layer("d0a", cache["c0"], dz)
    dz = R(up_adjoint(dc0[:, :32]));  ds0 = dc0[:, 32:]
    dz = layer("d1b", cache["d1a"], dz)
    dc1 = layer("d1a", cache["c1"], dz)
    dz = R(up_adjoint(dc1[:, :64]));  ds1 = dc1[:, 64:]
    dz = layer("d2b", cache["d2a"], dz)
    dc2 = layer("d2a", cache["c2"], dz)
    dz = R(up_adjoint(dc2[:, :64]));  ds2 = dc2[:, 64:]
    dz = layer("b3b", cache["b3a"], dz)
    dp2 = layer("b3a", cache["p2"], dz, input_is_activation=False)
    dz = R(ds2 + mask(cache["e2"]) * up(dp2) / 8.0)
    dz = layer("e2b", cache["e2a"], dz)
    dp1 = layer("e2a", cache["p1"], dz, input_is_activation=False)
    dz = R(ds1 + mask(cache["e1"]) * up(dp1) / 8.0)
    dz = layer("e1b", cache["e1a"], dz)
    dp0 = layer("e1a", cache["p0"], dz, input_is_activation=False)
    dz = R(ds0 + mask(cache["e0"]) * up(dp0) / 8.0)
    dz = layer("e0b", cache["e0a"], dz)
    g["e0a"] = conv_weight_grad(cache["I"], dz)
    return flatten(g)


def gradient(params, phase, gamma, target, emulate: bool = False):
    """(loss, flat gradient) for one batch."""
    O, cache = forward(params, phase, gamma, emulate)
    T = torch.as_tensor(np.asarray(target, dtype=np.float64))
    return float(loss(O, T)), backward(cache, loss_grad(O, T), emulate)


def adam(params, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, clip=0.0):
    """One Adam step (t counts from 1); returns new (params, m, v).  With
    clip > 0 the gradient is first scaled to global L2 norm <= clip."""
    if clip > 0.0:
        nrm = float(np.linalg.norm(grad))
        if nrm > clip:
            grad = grad * (clip / nrm)
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def warm_start(O, E, n: int, length: float = 1.0) -> np.ndarray:
    """Initial fluctuation for load E (Mandel 6-vector) from the network
    output of one sample: u[c] = (l / n) sum_j E_j O[3 j + c], shifted to
    zero mean per component.  Returns [3][s][s][s]."""
    O = torch.as_tensor(O, dtype=torch.float64)
    u = torch.zeros((3,) + tuple(O.shape[1:]), dtype=torch.float64)
    for j in range(6):
        u += float(E[j]) * O[3 * j:3 * j + 3]
    u = u * (length / n)
    u -= u.mean(dim=(1, 2, 3), keepdim=True)
    return u.numpy()
