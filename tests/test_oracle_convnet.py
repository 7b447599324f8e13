"""Pins of the warm-start network oracle (CPU, FP64).

Each part is fixed by something other than the oracle itself: brute-force
loops, library routines (torch's conv3d with circular padding, autograd,
torch.optim.Adam, torch's BF16 conversion), finite differences and closed
forms."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import convnet as cn


def rand(*shape, seed=0):
    return torch.as_tensor(np.random.default_rng(seed).standard_normal(shape))


def test_tap_order_and_periodic_conv_brute_force():
    s, ci, co = 3, 2, 3
    x, W, b = rand(1, ci, s, s, s, seed=1), rand(27, co, ci, seed=2), rand(co, seed=3)
    y = cn.conv(x, W, b)
    ref = np.zeros((co, s, s, s))
    for o in range(co):
        for z in range(s):
            for yy in range(s):
                for xx in range(s):
                    acc = float(b[o])
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                                for c in range(ci):
                                    acc += float(W[t, o, c]) * float(
                                        x[0, c, (z + dz) % s, (yy + dy) % s, (xx + dx) % s])
                    ref[o, z, yy, xx] = acc
    assert np.abs(y[0].numpy() - ref).max() < 1e-12


def test_conv_matches_library_circular_conv3d():
    s, ci, co = 6, 4, 5
    x, W, b = rand(2, ci, s, s, s, seed=4), rand(27, co, ci, seed=5), rand(co, seed=6)
    Wt = W.reshape(3, 3, 3, co, ci).permute(3, 4, 0, 1, 2).contiguous()
    ref = F.conv3d(F.pad(x, (1, 1, 1, 1, 1, 1), mode="circular"), Wt, b)
    assert torch.allclose(cn.conv(x, W, b), ref, rtol=0, atol=1e-12)


def test_conv_adjoints():
    s, ci, co = 4, 3, 2
    x, W, dy = rand(2, ci, s, s, s, seed=7), rand(27, co, ci, seed=8), rand(2, co, s, s, s, seed=9)
    zero = torch.zeros(co, dtype=torch.float64)
    lhs = float((cn.conv(x, W, zero) * dy).sum())
    assert abs(lhs - float((x * cn.conv_input_grad(dy, W)).sum())) < 1e-10 * abs(lhs) + 1e-12
    dW, db = cn.conv_weight_grad(x, dy)
    assert abs(lhs - float((W * dW).sum())) < 1e-10 * abs(lhs) + 1e-12
    assert torch.allclose(db, dy.sum(dim=(0, 2, 3, 4)))


def test_pool_and_upsampling():
    x, y = rand(1, 2, 2, 2, 2, seed=10), rand(1, 2, 4, 4, 4, seed=11)
    assert abs(float((cn.up(x) * y).sum()) - float((x * cn.up_adjoint(y)).sum())) < 1e-12
    assert torch.allclose(cn.pool(y), cn.up_adjoint(y) / 8.0)
    # nearest up-sampling: child (z, y, x) copies parent (z//2, y//2, x//2)
    u = cn.up(x)
    assert float(u[0, 1, 3, 2, 1]) == float(x[0, 1, 1, 1, 0])
    assert float(cn.pool(torch.ones(1, 1, 4, 4, 4, dtype=torch.float64)).max()) == 1.0


def test_bf16_rounding_is_nearest_even():
    v = torch.tensor([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -12, -3.0,
                      2.0 ** -130], dtype=torch.float64)
    r = cn.bf16(v).tolist()
    assert r[0] == 1.0                       # tie -> even mantissa
    assert r[1] == 1 + 2.0 ** -6             # tie -> even mantissa
    assert r[2] == 1 + 2.0 ** -7             # above the tie
    assert r[3] == -3.0
    assert r[4] == 2.0 ** -130               # subnormal kept


def test_loss_closed_form_and_gradient():
    B, s, A, k = 2, 8, 0.7, 3
    th = 2 * np.pi * k / s
    O = torch.zeros(B, cn.NOUT, s, s, s, dtype=torch.float64)
    O[1, 5] = A * torch.cos(th * torch.arange(s, dtype=torch.float64)).view(1, 1, s)
    T = torch.zeros_like(O)
    expect = A * A * (1 - np.cos(th)) / (3 * B * cn.NOUT)
    assert abs(float(cn.loss(O, T)) - expect) < 1e-14
    # gradient against central differences at a few entries
    O = rand(1, cn.NOUT, 4, 4, 4, seed=12)
    T = rand(1, cn.NOUT, 4, 4, 4, seed=13)
    g = cn.loss_grad(O, T)
    h = 1e-6
    for idx in [(0, 0, 0, 0, 0), (0, 17, 3, 1, 2), (0, 9, 2, 3, 3)]:
        Op, Om = O.clone(), O.clone()
        Op[idx] += h
        Om[idx] -= h
        fd = (float(cn.loss(Op, T)) - float(cn.loss(Om, T))) / (2 * h)
        assert abs(fd - float(g[idx])) < 1e-8


def _problem(s=8, B=2, seed=0):
    rng = np.random.default_rng(seed)
    phase = (rng.random((B, s, s, s)) < 0.3).astype(np.uint8)
    gamma = rng.uniform(0.3, 1.0, B)
    target = rng.standard_normal((B, cn.NOUT, s, s, s))
    return phase, gamma, target


def test_manual_backward_matches_autograd():
    phase, gamma, target = _problem()
    p = cn.init_params(3)
    loss, g = cn.gradient(p, phase, gamma, target)
    pt = torch.tensor(p, requires_grad=True)
    O, _ = cn.forward(pt, phase, gamma)
    L = cn.loss(O, torch.as_tensor(target))
    L.backward()
    ref = pt.grad.numpy()
    assert abs(float(L.detach()) - loss) < 1e-14 * abs(loss) + 1e-300
    assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max()


def test_gradient_finite_differences():
    phase, gamma, target = _problem(B=1, seed=1)
    p = cn.init_params(4)
    _, g = cn.gradient(p, phase, gamma, target)
    rng = np.random.default_rng(5)
    sizes = [27 * ci * co + co for _, ci, co, _ in cn.LAYERS] + [cn.NOUT * 17]
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    picks = [int(st + rng.integers(sz)) for st, sz in zip(starts, sizes)]
    picks += [int(starts[0] + 27 * 16 * 3 + 5), int(cn.param_count() - 1)]   # a bias, head bias
    h = 1e-6
    for i in picks:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (cn.gradient(pp, phase, gamma, target)[0] -
              cn.gradient(pm, phase, gamma, target)[0]) / (2 * h)
        # central-difference error: O(h^2) truncation + O(eps L / h) cancellation
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]) + 5e-9, (i, fd, g[i])


def test_translation_equivariance():
    phase, gamma, _ = _problem(s=16, B=1, seed=2)
    p = cn.init_params(6)
    O, _ = cn.forward(p, phase, gamma)
    O2, _ = cn.forward(p, np.roll(phase, (8, -8), axis=(1, 3)), gamma)
    assert torch.allclose(torch.roll(O, (8, -8), dims=(2, 4)), O2, atol=1e-12)


def test_emulated_bf16_forward_is_close_to_exact():
    phase, gamma, _ = _problem(s=8, B=1, seed=3)
    p = cn.init_params(7)
    O, _ = cn.forward(p, phase, gamma)
    Oe, _ = cn.forward(p, phase, gamma, emulate=True)
    rel = float((O - Oe).norm() / O.norm())
    assert 1e-5 < rel < 3e-2


def test_adam_matches_library():
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(50)
    grads = [rng.standard_normal(50) for _ in range(3)]
    t = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([t], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k, gk in enumerate(grads, start=1):
        opt.zero_grad()
        t.grad = torch.tensor(gk)
        opt.step()
        p, m, v = cn.adam(p, gk, m, v, k, lr=2e-3)
    assert np.abs(p - t.detach().numpy()).max() < 1e-14


def test_warm_start_is_linear_and_zero_mean():
    O = rand(cn.NOUT, 4, 4, 4, seed=9).numpy()
    E1, E2 = np.eye(6)[2], np.array([0.3, -0.1, 0.2, 0.05, 0.0, 0.4])
    u1 = cn.warm_start(O, E1, n=4, length=2.0)
    u2 = cn.warm_start(O, E2, n=4, length=2.0)
    u12 = cn.warm_start(O, E1 + E2, n=4, length=2.0)
    assert np.abs(u12 - u1 - u2).max() < 1e-14
    assert np.abs(u1.reshape(3, -1).mean(axis=1)).max() < 1e-15
    ref = O[6:9] * 0.5
    ref = ref - ref.reshape(3, -1).mean(axis=1).reshape(3, 1, 1, 1)
    assert np.abs(u1 - ref).max() < 1e-14


def test_shared_generator_describes_the_oracle_architecture():
    from synth.netinit import NET_HEAD_IN, NET_LAYERS, NET_OUT
    assert NET_LAYERS == cn.LAYERS and NET_OUT == cn.NOUT and NET_HEAD_IN == cn.HEAD_IN


def test_param_count():
    p = cn.init_params(0)
    assert p.size == cn.param_count()
    assert sum(v[0].numel() + v[1].numel() for v in cn.unflatten(p).values()) == p.size


def test_clipped_adam_matches_library():
    rng = np.random.default_rng(9)
    p0 = rng.standard_normal(40)
    grads = [rng.standard_normal(40) * s for s in (0.1, 5.0, 20.0)]
    t = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-3)
    p, m, v = p0.copy(), np.zeros(40), np.zeros(40)
    for k, gk in enumerate(grads, start=1):
        opt.zero_grad()
        t.grad = torch.tensor(gk)
        torch.nn.utils.clip_grad_norm_([t], 1.0)
        opt.step()
        p, m, v = cn.adam(p, gk, m, v, k, lr=1e-3, clip=1.0)
    # the library scales by clip / (norm + 1e-6): a relative 1e-6 difference
    # in the clipped gradient, far below the lr-sized updates
    assert np.abs(p - t.detach().numpy()).max() < 1e-9
