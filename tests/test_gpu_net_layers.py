"""Single-layer parity of the network's MFMA kernels (forward convolution,
input gradient, weight gradient) on identical BF16 inputs, through
fh_net_layer, against the FP64 convolutions of oracle/convnet.py.

Both sides see the same BF16 tensors and BF16-rounded weights, so the only
differences are the GPU's FP32 accumulation (in its own order) and, for the
BF16 outputs, the final rounding.  Bounds:

* forward / input gradient (BF16 outputs): |gpu - y| <= 2^-8 |y| (the
  output's rounding: half a BF16 unit is 2^-9 relative, so a value that
  lands on the other side of a rounding boundary is one unit, at most 2^-8
  relative, away) + g, with g = (terms) 2^-24 sum|terms|, the textbook bound
  on recursive FP32 summation of that many products; and at least 99 % of
  the outputs equal the oracle's BF16 rounding exactly;
* weight gradient (FP32 output): relative L2 error <= 1e-5 against the FP64
  result, and every entry within the recursive-summation bound.
"""
import ctypes
import sys

import numpy as np
import pytest

from oracle import convnet as cn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 64
B = 1


def say(*a):
    print("[gpu-net-layer]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fh():
    from paper_2203_02962_amd import fh as fhmod
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    fhmod.load_library()
    return fhmod


@pytest.fixture(scope="module")
def net(fh):
    nt = fh.Net(N, 2)
    rng = np.random.default_rng(5)
    p = cn.init_params(3)
    p = p + rng.normal(0.0, 0.05, p.shape)      # nonzero biases
    nt.set_params(p.astype(np.float32))
    nt.params = p.astype(np.float32).astype(np.float64)
    yield nt
    nt.close()


def _bf(x):
    """Round to BF16 (ties to even), returned as float64."""
    return torch.from_numpy(np.asarray(x, dtype=np.float64)).to(torch.bfloat16).to(
        torch.float64).numpy()


def _bits(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(
        torch.bfloat16).view(torch.int16).cuda()


def _from_bits(t):
    return t.view(torch.bfloat16).to(torch.float64).cpu().numpy()


def _cf(x_cl, s, c):
    """channels last [B][V][c] (v = x + s (y + s z)) -> [B][c][z][y][x]"""
    return torch.from_numpy(x_cl.reshape(B, s, s, s, c)).permute(0, 4, 1, 2, 3).contiguous()


def _cl(x_cf):
    return x_cf.permute(0, 2, 3, 4, 1).reshape(B, -1, x_cf.shape[1]).numpy()


def _layer_params(netobj, l):
    w = cn.unflatten(netobj.params)
    name = cn.LAYERS[l][0]
    W, b = w[name]
    return torch.from_numpy(_bf(W.numpy())), torch.from_numpy(_bf(b.numpy()))


def _check_bf16(gpu, exact, bound, what):
    diff = np.abs(gpu - exact)
    lim = 2.0 ** -8 * np.abs(exact) + bound + 1e-30
    assert (diff <= lim).all(), (what, float((diff / lim).max()))
    same = np.mean(gpu == _bf(exact))
    say(what, "exact BF16 matches", round(float(same), 5))
    assert same >= 0.99, what


LAYERS_TESTED = [0, 2, 6, 8, 12]


@pytest.mark.parametrize("l", LAYERS_TESTED)
def test_forward_layer(fh, net, l):
    cin, cout, lev = fh.Net.LAYERS[l]
    s = N >> lev
    V = s ** 3
    cinp = (cin + 15) // 16 * 16
    rng = np.random.default_rng(100 + l)
    x = np.zeros((B, V, cinp))
    x[..., :cin] = _bf(rng.normal(size=(B, V, cin)))
    out = torch.empty(B * V * cout, dtype=torch.int16, device="cuda")
    net.layer(l, 0, B, x=_bits(x), out=out)
    W, b = _layer_params(net, l)
    xc = _cf(x[..., :cin].copy(), s, cin)
    y = cn.leaky(cn.conv(xc, W, b))
    mag = cn.conv(xc.abs(), W.abs(), b.abs())
    g = 27 * cinp * 2.0 ** -24 * _cl(mag)
    _check_bf16(_from_bits(out).reshape(B, V, cout), _cl(y), g, f"forward layer {l}")


@pytest.mark.parametrize("l", [2, 6, 8, 12])
@pytest.mark.parametrize("masked", [False, True])
def test_input_gradient_layer(fh, net, l, masked):
    cin, cout, lev = fh.Net.LAYERS[l]
    s = N >> lev
    V = s ** 3
    cinp = (cin + 15) // 16 * 16
    rng = np.random.default_rng(200 + l)
    dz = _bf(rng.normal(size=(B, V, cout)))
    mask = _bf(rng.normal(size=(B, V, cinp))) if masked else None
    out = torch.empty(B * V * cinp, dtype=torch.int16, device="cuda")
    net.layer(l, 1, B, dz=_bits(dz), mask=None if mask is None else _bits(mask), out=out)
    W, _ = _layer_params(net, l)
    dzc = _cf(dz, s, cout)
    dx = cn.conv_input_grad(dzc, W)
    mag = cn.conv_input_grad(dzc.abs(), W.abs())
    dx = _cl(dx)
    mag = _cl(mag)
    if masked:
        f = np.where(mask[..., :cin] > 0, 1.0, cn.SLOPE)
        dx = dx * f
        mag = mag * f
    gpu = _from_bits(out).reshape(B, V, cinp)
    assert not gpu[..., cin:].any()          # padding channels stay zero
    g = 27 * cout * 2.0 ** -24 * mag
    _check_bf16(gpu[..., :cin], dx, g, f"input gradient layer {l} masked={masked}")


@pytest.mark.parametrize("l", LAYERS_TESTED)
def test_weight_gradient_layer(fh, net, l):
    cin, cout, lev = fh.Net.LAYERS[l]
    s = N >> lev
    V = s ** 3
    cinp = (cin + 15) // 16 * 16
    rng = np.random.default_rng(300 + l)
    x = np.zeros((B, V, cinp))
    x[..., :cin] = _bf(rng.normal(size=(B, V, cin)))
    dz = _bf(rng.normal(size=(B, V, cout)))
    out = torch.empty(27 * cin * cout + cout, dtype=torch.float32, device="cuda")
    net.layer(l, 2, B, x=_bits(x), dz=_bits(dz), out=out)
    got = out.cpu().numpy().astype(np.float64)
    xc = _cf(x[..., :cin].copy(), s, cin)
    dzc = _cf(dz, s, cout)
    dW, db = cn.conv_weight_grad(xc, dzc)
    mW, mb = cn.conv_weight_grad(xc.abs(), dzc.abs())
    want = np.concatenate([dW.numpy().ravel(), db.numpy().ravel()])
    mag = np.concatenate([mW.numpy().ravel(), mb.numpy().ravel()])
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    say(f"weight gradient layer {l}: relative L2 {rel:.2e}")
    assert rel <= 1e-5
    assert (np.abs(got - want) <= B * V * 2.0 ** -24 * mag + 1e-30).all()


def test_layer_hook_rejections(fh, net):
    out = torch.empty(16, dtype=torch.float32, device="cuda")
    with pytest.raises(fh.FHError):       # layer index out of range
        net._check(net.lib.fh_net_layer(net.ptr, 14, 0, 1, None, None, None,
                                        ctypes.c_void_p(out.data_ptr())))
    dz = torch.zeros(N ** 3 * 16, dtype=torch.int16, device="cuda")
    o2 = torch.empty(N ** 3 * 16, dtype=torch.int16, device="cuda")
    with pytest.raises(fh.FHError):
        net.layer(0, 1, 1, dz=dz, out=o2)        # the first layer has no input gradient
