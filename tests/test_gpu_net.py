"""GPU parity of the learned warm start, through the C-ABI.

The network's forward pass, its gradients (every layer, batch 1 and 2), the
Adam step and the warm-start assembly are compared with the FP64 oracle of
oracle/convnet.py run in its BF16-storage mode: the oracle rounds weights,
features, activations and activation gradients to BF16 at the points where
the GPU stores them and does all arithmetic in FP64.

BF16 tolerance.  The GPU sums in FP32 in another order, so a stored value
whose exact result lies near a BF16 rounding boundary can land one unit
(2^-8 relative) away from the oracle's.  Each convolution spreads such a flip
to its 27 x channels neighbours, so deep layers differ by one unit in a large
fraction of elements (measured: the first layer agrees to 1e-11, the last
activation differs by one unit in about half of its elements, 4e-3 relative
L2) -- the same size as the error of BF16 storage itself against exact FP64.
Forward: relative L2 error <= 2^-6 = 1.6e-2 (four BF16 units) on the output.
Gradients are sums over all voxels of signed terms and cancel heavily, so
the same one-unit flips move them by a few percent (measured 2e-2 to 5e-2,
equal to the BF16-storage oracle's own distance from exact FP64, with cosine
similarity above 0.998); the stated bound per layer is: relative L2 error
against the BF16-storage oracle <= max(2^-6, 2 x that oracle's distance from
exact FP64) and cosine >= 0.995.  The head bias gradient is zero in exact
arithmetic (the loss ignores constant shifts of the output) and is checked
as such.  A real defect (a wrong tap, mask or channel, a dropped bias) moves
these by O(1): the test weights carry biases of 0.3 so a lost bias is not
hidden.  Adam runs in FP32 on FP32 inputs: within half an FP32 unit of the
parameter per step plus 1e-5 of the update.  The warm-start assembly (a linear
combination, scaling and mean removal of the output) keeps the output's
absolute error: bounded by 2^-6 of the uncentred combination.  The initial-guess path of the solver is compared with the oracle's
warm-started PCG (pcg.py) under the FP64 solve tolerances of
test_gpu_parity.py.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import convnet as cn
from oracle.assembly import assemble_stiffness, rhs
from oracle.pcg import screened_guess, pcg
from oracle.precond import Preconditioner
from synth import batch_workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N64 = 64


def say(*a):
    print("[gpu-net]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fh():
    from paper_2203_02962_amd import fh as fhmod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    fhmod.load_library()
    return fhmod


def _samples(count, seed0):
    wls = batch_workload(count=count, seed0=seed0, fixed_n=N64)
    phase = np.stack([w["phase"] for w in wls]).astype(np.uint8)
    gamma = np.array([np.log10(w["contrast"]) / 3.0 for w in wls], dtype=np.float32)
    return wls, phase, gamma


BF16_TOL = 2.0 ** -6


def _params(seed):
    """Network weights with biases of 0.3 (FP32 values, as the GPU keeps
    them, so the oracle sees the same numbers)."""
    p = cn.init_params(seed)
    rng = np.random.default_rng(seed + 1000)
    k = 0
    for _, ci, co, _ in cn.LAYERS:
        k += 27 * ci * co
        p[k:k + co] = rng.normal(0.0, 0.3, co)
        k += co
    p[-cn.NOUT:] = rng.normal(0.0, 0.3, cn.NOUT)
    return p.astype(np.float32).astype(np.float64)


def _rel(a, b):
    a, b = np.asarray(a, float).ravel(), np.asarray(b, float).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _bf16_bits(x):
    """BF16 bit patterns (as int16) of float64 data, round to nearest even."""
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(
        torch.bfloat16).view(torch.int16)


def test_forward_matches_oracle(fh):
    say("forward n=64 batch 2")
    _, phase, gamma = _samples(2, 500)
    p = _params(11)
    net = fh.Net(N64, 2)
    net.set_params(p.astype(np.float32))
    out = torch.empty((2, cn.NOUT) + (N64,) * 3, dtype=torch.float32, device="cuda")
    net.forward(_dev(phase), gamma, out)
    O, _ = cn.forward(p, phase, gamma.astype(np.float64), emulate=True)
    err = _rel(out.cpu().numpy(), O.numpy())
    Ox, _ = cn.forward(p, phase, gamma.astype(np.float64), emulate=False)
    say("forward rel L2", err, "BF16 storage vs exact", _rel(O.numpy(), Ox.numpy()))
    assert err < BF16_TOL
    go, oo = out.cpu().numpy(), O.numpy()
    for b in range(2):
        for c in (0, 7, 17):
            assert _rel(go[b, c], oo[b, c]) < BF16_TOL


@pytest.mark.parametrize("batch", [1, 2])
def test_gradient_matches_oracle(fh, batch):
    say("gradient n=64 batch", batch)
    _, phase, gamma = _samples(batch, 600 + batch)
    p = _params(12 + batch)
    rng = np.random.default_rng(20 + batch)
    target = rng.standard_normal((batch, cn.NOUT) + (N64,) * 3) * 0.5
    bits = _bf16_bits(target)
    target_q = bits.view(torch.bfloat16).to(torch.float64).numpy()
    net = fh.Net(N64, batch)
    net.set_params(p.astype(np.float32))
    loss, g = net.gradient(_dev(phase), gamma, bits.cuda())
    lo, go = cn.gradient(p, phase, gamma.astype(np.float64), target_q, emulate=True)
    _, gx = cn.gradient(p, phase, gamma.astype(np.float64), target_q, emulate=False)
    say("loss", loss, lo)
    assert abs(loss - lo) < BF16_TOL * abs(lo)

    def check(name, sl):
        err, own = _rel(g[sl], go[sl]), _rel(go[sl], gx[sl])
        cos = float(np.dot(g[sl], go[sl]) / (np.linalg.norm(g[sl]) * np.linalg.norm(go[sl])))
        say(f"{name}: gpu-vs-oracle {err:.3e}  oracle BF16-vs-exact {own:.3e}  cos {cos:.6f}")
        assert err <= max(BF16_TOL, 2.0 * own), (name, err, own)
        assert cos >= 0.995, (name, cos)

    k = 0
    for name, ci, co, _ in cn.LAYERS:
        nw = 27 * ci * co
        check(name + ".W", slice(k, k + nw))
        check(name + ".b", slice(k + nw, k + nw + co))
        k += nw + co
    check("head.W", slice(k, k + cn.NOUT * cn.HEAD_IN))
    gb = g[k + cn.NOUT * cn.HEAD_IN:]
    # sum over voxels of a periodic Laplacian: zero up to FP32 rounding
    assert np.abs(gb).max() < 1e-5 * np.abs(g[k:k + cn.NOUT * cn.HEAD_IN]).max()


@pytest.mark.parametrize("clip", [0.0, 50.0])
def test_adam_matches_oracle(fh, clip):
    say("adam clip", clip)
    net = fh.Net(N64, 1)
    P = net.P
    rng = np.random.default_rng(3)
    p = rng.standard_normal(P).astype(np.float32)
    net.set_params(p)
    pp, m, v = p.astype(np.float64), np.zeros(P), np.zeros(P)
    for t in range(1, 4):
        gk = (rng.standard_normal(P) * 10.0 ** rng.uniform(-3, 1, P)).astype(np.float32)
        net.adam(gk, lr=2e-3, clip=clip)
        pp, m, v = cn.adam(pp, gk.astype(np.float64), m, v, t, lr=2e-3, clip=clip)
    got = net.get_params().astype(np.float64)
    # three steps, each rounding the FP32 parameter once (<= 1/2 unit of the
    # value it passes through, at most |p| plus three updates of <= 3 lr)
    peak = np.maximum(np.abs(p), np.abs(pp)) + 3 * 3 * 2e-3
    assert np.all(np.abs(got - pp) <= 3 * 2.0 ** -24 * peak + 1e-5 * np.abs(pp - p))


def test_warm_guess_matches_oracle(fh):
    say("warm guess assembly")
    _, phase, gamma = _samples(1, 700)
    p = _params(21)
    net = fh.Net(N64, 1)
    net.set_params(p.astype(np.float32))
    E = np.array([[1, 0, 0, 0, 0, 0], [0.2, -0.1, 0.3, 0.05, 0.0, 0.4]], dtype=np.float64)
    x = torch.empty((2, 3) + (N64,) * 3, dtype=torch.float64, device="cuda")
    net.guess(_dev(phase[0]), float(gamma[0]), E, 2.0, x)
    O, _ = cn.forward(p, phase, gamma.astype(np.float64), emulate=True)
    for j in range(2):
        ref = cn.warm_start(O[0].numpy(), E[j], n=N64, length=2.0)
        full = (2.0 / N64) * np.einsum("j,jczyx->czyx", E[j], O[0].numpy().reshape(6, 3, *O.shape[2:]))
        got = x[j].cpu().numpy()
        assert np.linalg.norm(got - ref) <= BF16_TOL * np.linalg.norm(full)
        assert np.abs(got.reshape(3, -1).mean(axis=1)).max() < 1e-12 * np.abs(got).max()


def test_train_steps_reduce_loss(fh):
    say("training steps")
    _, phase, gamma = _samples(4, 800)
    rng = np.random.default_rng(5)
    # a learnable target: a fixed smooth function of the phase field
    chi = (phase == 1).astype(np.float64)
    blur = sum(np.roll(chi, s, axis=a) for a in (1, 2, 3) for s in (-1, 0, 1)) / 9.0
    target = np.stack([np.stack([blur[b] * (c + 1) / 18.0 for c in range(cn.NOUT)])
                       for b in range(4)])
    net = fh.Net(N64, 2)
    net.set_params(cn.init_params(31).astype(np.float32))
    order = np.array([rng.permutation(4)[:2] for _ in range(60)], dtype=np.int32)
    losses = net.train(_dev(phase), gamma, _bf16_bits(target).cuda(), order, 2, lr=3e-4)
    say("loss first/last", losses[:3], losses[-3:])
    assert np.all(np.isfinite(losses))
    assert losses[-5:].mean() < 0.5 * losses[:5].mean()


# ------------------------------------------------------- initial guess path

def _spheres24():
    from tests.test_gpu_parity import _spheres_case
    return _spheres_case(24, (2.5, 4.5), 100.0, 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_initial_guess_solve_matches_oracle(fh, precision):
    from paper_2203_02962_amd.runner import fluctuations, setup_context
    say("initial guess", precision)
    wl, prob = _spheres24()
    K = assemble_stiffness(prob)
    M = Preconditioner(prob, oracle.mean_material(prob))
    AK = lambda v: K @ v  # noqa: E731
    nd = prob.ndof_node
    rng = np.random.default_rng(4)
    # loads 0-2 get a perturbed solution (kept), 3 a constant shift of a
    # good guess (kept), 4 a bad guess (rejected), 5 none (zeros: rejected)
    loads = wl["loads"]
    guesses, ref = [], []
    for j, E in enumerate(loads):
        b = rhs(prob, E)
        xs = pcg(AK, M.apply, b, 1e-12, nd=nd).x
        if j < 3:
            g = xs + 0.02 * np.abs(xs).max() * rng.standard_normal(xs.size)
        elif j == 3:
            g = xs + 0.001 * np.abs(xs).max() * rng.standard_normal(xs.size) + 5.0
        elif j == 4:
            g = 50.0 * np.abs(xs).max() * rng.standard_normal(xs.size)
        else:
            g = np.zeros_like(xs)
        ok, x0, rb, rx = screened_guess(AK, M.apply, b, g, nd)
        res = pcg(AK, M.apply, b, 1e-10, x0=x0, nd=nd, rho_ref=rb)
        guesses.append(g)
        ref.append((ok, np.sqrt(rx / rb), res))
    ctx = setup_context(wl)
    gdev = _dev(np.stack(guesses))
    prec = fh.FH_FP64 if precision == "fp64" else fh.FH_FP32_REFINED
    rc, st = ctx.solve(eta=1e-10, precision=prec, guess_dev=gdev)
    assert rc == 0, st
    us = fluctuations(ctx)
    H = ctx.get_homogenized()
    Ho = oracle.homogenized_energy(prob, loads, [r[2].x for r in ref])
    assert _rel(H, Ho) < 1e-10
    cold_ctx = setup_context(wl)
    _, cold = cold_ctx.solve(eta=1e-10, precision=prec)
    for j, (ok, gres, res) in enumerate(ref):
        assert st["guess_used"][j] == int(ok), (j, st["guess_used"])
        assert abs(st["guess_res"][j] - gres) < 1e-9 * max(gres, 1e-3), (j, st["guess_res"][j], gres)
        assert _rel(us[j], res.x) < 1e-7
        if precision == "fp64":
            tol = max(1, int(0.01 * res.iterations))
            assert abs(st["iterations"][j] - res.iterations) <= tol, (j, st["iterations"][j], res.iterations)
            assert st["rel_res"][j] <= 1e-10 * (1 + 1e-9)
        if ok:
            assert st["iterations"][j] < cold["iterations"][j]
        else:
            assert st["iterations"][j] == cold["iterations"][j]


def test_warm_start_flag_uses_network_guess(fh):
    """FH_FLAG_WARM_START takes the network's guess through the screen: the
    result equals an explicit-guess solve with the same guess."""
    from paper_2203_02962_amd.runner import setup_context
    say("warm start flag")
    wls, phase, gamma = _samples(1, 900)
    wl = dict(wls[0])
    wl["loads"] = np.eye(6)
    net = fh.Net(N64, 1)
    net.set_params(_params(41).astype(np.float32))
    x = torch.empty((6, 3) + (N64,) * 3, dtype=torch.float64, device="cuda")
    net.guess(_dev(phase[0]), float(gamma[0]), np.eye(6), 1.0, x)
    a = setup_context(wl)
    a.set_warm_start(net)
    rc_a, st_a = a.solve(eta=1e-6, warm_start=True)
    b = setup_context(wl)
    rc_b, st_b = b.solve(eta=1e-6, guess_dev=x)
    assert rc_a == 0 and rc_b == 0
    assert st_a["guess_used"] == st_b["guess_used"]
    assert st_a["iterations"] == st_b["iterations"]
    assert np.allclose(st_a["guess_res"], st_b["guess_res"], rtol=1e-12, atol=0)
    assert np.abs(a.get_homogenized() - b.get_homogenized()).max() == 0.0


def test_warm_start_validation_and_recovery(fh):
    """Requests the warm start cannot serve fail with a clear error and leave
    the context usable for a zero start."""
    from paper_2203_02962_amd.runner import setup_context
    from tests.test_gpu_parity import _spheres_case
    say("warm start validation")
    wl, _ = _spheres_case(32, (2.5, 4.5), 50.0, 3)
    c = setup_context(wl)
    with pytest.raises(fh.FHError) as e:
        c.solve(eta=1e-6, warm_start=True)          # no network attached
    assert e.value.code == fh.FH_ESTATE
    net = fh.Net(N64, 1)
    net.set_params(_params(5).astype(np.float32))
    c.set_warm_start(net)
    with pytest.raises(fh.FHError) as e:
        c.solve(eta=1e-6, warm_start=True)          # 32^3 grid, 64^3 network
    assert e.value.code == fh.FH_EINVAL and "grid" in str(e.value)
    rc, st = c.solve(eta=1e-6)                      # zero start still works
    assert rc == 0 and st["guess_used"] == [0] * 6
    c.set_warm_start(None)
