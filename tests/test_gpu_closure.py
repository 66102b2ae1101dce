"""GPU tests of the closure network (BF16 MFMA forward / backward / Adam)
against the FP64 oracle network, and of the closure hook in the 2-D step
against the FP64 LB oracle.

Tolerances.  Weights, activations and back-propagated gradients are stored
in BF16 (8 significant bits).  Against the FP64 network the output carries
~1e-2 relative error; the weight gradients grow by ~3x per layer towards
the input (leaky-ReLU kinks flip where z is within BF16 noise of 0), up to
~6e-2 on the first layer.  So each result is checked twice: against the
oracle's BF16 storage model (same rounding points, FP64 arithmetic), which
only FP32 accumulation order separates from the GPU -- 1e-2 -- and against
the FP64 network -- 3e-2 (output), 1.2e-1 (gradients, per layer, relative
L2).  On a network built so that every value is a short dyadic fraction
(exact FP32 sums, nothing for BF16 to round) the outputs, the loss and
every gradient equal the FP64 network's exactly.  The closure hook is plain FP64 / FP32 arithmetic: 1e-12 / 1e-5 as
for the step itself.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import cnn_ref as C
from oracle import ref

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cplb():
    import torch

    from paper_2402_15752_amd import cplb as L
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L.library()
    return L


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def setup_net(cplb, B, H, Wd, seed, cin=5):
    import torch
    rng = np.random.default_rng(seed)
    theta = C.init_params(seed) * np.concatenate(
        [np.full(C.num_params() - (16 * 32 * 9 + 16), 1.0), np.full(16 * 32 * 9 + 16, 5.0)])
    theta += rng.normal(size=theta.size) * 0.02 * (np.arange(theta.size) % 7 == 0)
    theta = theta.astype(np.float32).astype(np.float64)  # the GPU holds FP32 masters
    planes = rng.normal(size=(B, cin, H, Wd))
    scale = rng.uniform(0.5, 1.5, size=cin)
    net = cplb.ClosureNet(B, H, Wd)
    net.set_params(theta)
    net.set_input_scale(scale)
    x = np.zeros((B, 16, H, Wd))
    x[:, :cin] = planes * scale[None, :, None, None]
    # the GPU rounds the scaled inputs to BF16 before the first layer
    x = x.astype(np.float32)
    tp = torch.tensor(planes, dtype=torch.float32, device="cuda").contiguous()
    return net, theta, x, tp


@pytest.mark.parametrize("B,H,Wd", [(2, 16, 48), (1, 12, 40), (3, 8, 64)])
def test_forward_matches_oracle(cplb, B, H, Wd):
    say(f"cnn forward B={B} H={H} W={Wd}")
    net, theta, x, tp = setup_net(cplb, B, H, Wd, seed=B * 100 + H)
    net.set_output_scale(1.5, 0.75)
    out = net.forward(tp).cpu().numpy()
    assert out.shape == (B, 2, H, Wd)
    ref_out = C.output(theta, x, scale=(1.5, 0.75))
    ref16 = C.output(theta, x, scale=(1.5, 0.75), storage="bf16")
    e, e16 = rel(out, ref_out), rel(out, ref16)
    say(f"  rel L2 vs fp64 {e:.2e}, vs bf16 storage model {e16:.2e}")
    assert np.all(np.isfinite(out)) and e <= 3e-2 and e16 <= 1e-2, (e, e16)
    # balanced: the corrections add nothing to a sample's total
    tot = (out[:, 0].astype(np.float64) + out[:, 1]).sum(axis=(1, 2))
    assert np.all(np.abs(tot) <= 1e-5 * np.abs(out).sum(axis=(1, 2, 3))), tot
    net.close()


def dyadic_network(seed, cin=5):
    """Parameters under which every value the network forms is a short
    dyadic fraction: layer 1 sums 0/1 inputs with weights 0 or 1/64, and
    each output channel of layers 2-4 reads one or two (channel, tap) pairs
    of the layer below with weights 1/2 or 1.  Every sum is exact in FP32 and
    every activation has at most 8 significant bits, so BF16 storage rounds
    nothing; the biases are positive, so every pre-activation is (the leaky
    slope never applies, forward or backward), and a correct GPU network
    equals the FP64 one exactly."""
    rng = np.random.default_rng(seed)
    layers = []
    for n, (ci, co) in enumerate(C.LAYERS):
        W = np.zeros((co, ci, 3, 3))
        b = np.zeros(co)
        if n == 0:
            W[:, :cin] = (rng.random((co, cin, 3, 3)) < 0.5) / 64.0
            b[:] = rng.integers(1, 4, size=co) / 64.0
        else:
            for o in range(co):
                for _ in range(1 if n < 3 else 2):
                    W[o, rng.integers(ci), rng.integers(3), rng.integers(3)] = 0.5 if n < 3 else 1.0
            b[:] = rng.integers(1, 4, size=co) / (64.0 * 2 ** n)
        layers.append((W, b))
    return C.pack(layers)


@pytest.mark.parametrize("B,H,Wd", [(2, 8, 64), (1, 16, 32)])
def test_forward_exact_on_dyadic_network(cplb, B, H, Wd):
    """Zero-tolerance pin of the convolution layout (taps, channels, padding
    in y, wrap in x) and of the balance: on the dyadic network the GPU's
    forward and inference outputs equal the FP64 network's bit for bit."""
    import torch
    say(f"cnn exact forward on a dyadic network B={B} H={H} W={Wd}")
    rng = np.random.default_rng(B * 7 + H)
    theta = dyadic_network(B * 13 + Wd)
    planes = (rng.random((B, 5, H, Wd)) < 0.5).astype(np.float64)
    x = np.zeros((B, 16, H, Wd))
    x[:, :5] = planes
    ref64 = C.output(theta, x)
    # the data is what the construction promises: BF16 storage changes nothing
    assert np.array_equal(C.output(theta, x, storage="bf16"), ref64)
    assert np.abs(ref64).max() > 0
    net = cplb.ClosureNet(B, H, Wd)
    net.set_params(theta)
    net.set_input_scale(np.ones(5))
    net.set_output_scale(1.0, 1.0)
    tp = torch.tensor(planes, dtype=torch.float32, device="cuda").contiguous()
    out = net.forward(tp).cpu().numpy().astype(np.float64)
    inf = net.infer(tp).cpu().numpy().astype(np.float64)
    say(f"  max |GPU - FP64| forward {np.abs(out - ref64).max():.1e}, inference {np.abs(inf - ref64).max():.1e}")
    assert np.array_equal(out, ref64) and np.array_equal(inf, ref64)
    net.close()


def test_gradients_exact_on_dyadic_network(cplb):
    """Zero-tolerance pin of the backward pass: on the dyadic network with a
    target that differs from the output by +-1/4 or +-1/2 at four pixels,
    every back-propagated value is again a short dyadic fraction and every
    gradient a sum of a few exact terms, so the GPU's loss and every weight
    and bias gradient equal the FP64 network's bit for bit."""
    import torch
    B, H, Wd = 2, 8, 64
    say(f"cnn exact gradients on a dyadic network B={B} H={H} W={Wd}")
    rng = np.random.default_rng(5)
    theta = dyadic_network(29)
    planes = (rng.random((B, 5, H, Wd)) < 0.5).astype(np.float64)
    x = np.zeros((B, 16, H, Wd))
    x[:, :5] = planes
    out = C.forward(theta, x)[0]
    target = out.copy()
    for _ in range(4):
        target[rng.integers(B), rng.integers(2), rng.integers(H), rng.integers(Wd)] -= \
            rng.choice([-0.5, -0.25, 0.25, 0.5])
    lref, gref = C.loss_and_grad(theta, x, target)
    l16, g16 = C.loss_and_grad(theta, x, target, storage="bf16")
    assert l16 == lref and np.array_equal(g16, gref)  # nothing for BF16 to round
    net = cplb.ClosureNet(B, H, Wd)
    net.set_params(theta)
    net.set_input_scale(np.ones(5))
    net.forward(torch.tensor(planes, dtype=torch.float32, device="cuda").contiguous())
    loss = net.backward(torch.tensor(target, dtype=torch.float32, device="cuda").contiguous())
    g = np.asarray(net.grads(), dtype=np.float64)
    k = 0
    for n, (ci, co) in enumerate(C.LAYERS):
        nw = co * ci * 9
        say(f"  layer {n}: {np.count_nonzero(gref[k:k + nw + co])} nonzero gradients, "
            f"max |GPU - FP64| {np.abs(g[k:k + nw + co] - gref[k:k + nw + co]).max():.1e}")
        assert np.count_nonzero(gref[k:k + nw + co]) > 0
        k += nw + co
    say(f"  loss {loss!r} FP64 {lref!r}")
    assert loss == lref and np.array_equal(g, gref)
    net.close()


@pytest.mark.parametrize("B,H,Wd", [(2, 16, 48), (1, 12, 40)])
def test_gradients_match_oracle(cplb, B, H, Wd):
    import torch
    say(f"cnn gradients B={B} H={H} W={Wd}")
    net, theta, x, tp = setup_net(cplb, B, H, Wd, seed=7 + H)
    rng = np.random.default_rng(11)
    target = rng.normal(size=(B, 2, H, Wd)) * 0.5
    net.forward(tp)
    loss = net.backward(torch.tensor(target, dtype=torch.float32, device="cuda").contiguous())
    g = net.grads()
    lref, gref = C.loss_and_grad(theta, x, target)
    l16, g16 = C.loss_and_grad(theta, x, target, storage="bf16")
    say(f"  loss {loss:.6e} oracle {lref:.6e} bf16 model {l16:.6e}")
    assert abs(loss - lref) <= 3e-2 * lref and abs(loss - l16) <= 1e-3 * l16
    k = 0
    for n, (ci, co) in enumerate(C.LAYERS):
        nw = co * ci * 9
        ew, ew16 = rel(g[k:k + nw], gref[k:k + nw]), rel(g[k:k + nw], g16[k:k + nw])
        eb, eb16 = (rel(g[k + nw:k + nw + co], gref[k + nw:k + nw + co]),
                    rel(g[k + nw:k + nw + co], g16[k + nw:k + nw + co]))
        say(f"  layer {n}: dW {ew:.2e} ({ew16:.2e} vs bf16 model) db {eb:.2e} ({eb16:.2e})")
        assert ew <= 1.2e-1 and eb <= 1.2e-1, (n, ew, eb)
        assert ew16 <= 1e-2 and eb16 <= 1e-2, (n, ew16, eb16)
        k += nw + co
    net.close()


def test_training_fits_a_teacher(cplb):
    """Adam on the GPU fits the output of a different (teacher) parameter set
    on a fixed batch: the FP64 loss falls by more than 10x."""
    import torch
    B, H, Wd = 2, 16, 32
    rng = np.random.default_rng(3)
    planes = rng.normal(size=(B, 5, H, Wd))
    x = np.zeros((B, 16, H, Wd))
    x[:, :5] = planes
    teacher = C.init_params(99)
    teacher[-(16 * 32 * 9 + 16):] *= 5.0
    target = C.forward(teacher, x)[0]
    net = cplb.ClosureNet(B, H, Wd, seed=5)
    tp = torch.tensor(planes, dtype=torch.float32, device="cuda").contiguous()
    tt = torch.tensor(target, dtype=torch.float32, device="cuda").contiguous()
    losses = []
    for it in range(300):
        net.forward(tp)
        losses.append(net.backward(tt))
        net.adam(lr=2e-3)
    say(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.1 * losses[0]
    net.close()


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_closure_hook_matches_oracle(cplb, precision, tol):
    """Random fields, walls, and random per-node corrections of c1 and c2:
    the GPU step with the closure equals the oracle step with the same
    closure."""
    import torch
    p = W.params(nx=67, ny=37, periodic=(1, 0, 1), precision=precision, sigma=2e-3, rho1=3.0,
                 rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07, D2=0.02, Keq=0.6,
                 A=0.4, g=(0.0, -2e-5, 0.0), rho_ref=1.5,
                 ref_f=W.phase_reference(precision))
    f = W.random_fields(p, seed=21)
    s = (np.random.default_rng(4).normal(size=(2,) + W.shape_of(p)) * 1e-3).astype(np.float32)
    g = cplb.Lattice(p)
    g.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    ts = torch.tensor(s, device="cuda").contiguous()
    g.set_closure(ts)
    o = ref.Oracle(p)
    o.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    o.set_closure(s.astype(np.float64))
    g.step(3)
    o.step(3)
    for k in ("phi", "c1", "c2", "ux", "uy", "p"):
        a, b = g.field(k).cpu().numpy(), o.field(k)
        scale = max(np.linalg.norm(b), np.linalg.norm(b - b.mean()))
        e = np.linalg.norm(a - b) / scale
        assert e <= tol, (k, e)
    # the closure really acts: switching it off changes c1 by ~3 s per node
    g2 = cplb.Lattice(p)
    g2.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    g2.step(3)
    d = g.field("c1").cpu().numpy() - g2.field("c1").cpu().numpy()
    assert np.abs(d).max() > 1e-4
    # each step the corrections take sum (s1 + s2) from the total scalar
    r, r2 = g.reduce(), g2.reduce()
    want = -3.0 * float(s.astype(np.float64).sum())
    assert abs((r["sum_c"] - r2["sum_c"]) - want) <= 1e-5 * abs(r2["sum_c"]), (r["sum_c"] - r2["sum_c"], want)


@pytest.mark.parametrize("n,H,Wd,F", [(3, 8, 12, 4), (2, 5, 7, 2), (1, 16, 64, 4)])
def test_restrict_is_the_block_mean(cplb, n, H, Wd, F):
    import torch
    x = np.random.default_rng(n + H).normal(size=(n, H * F, Wd * F)).astype(np.float32)
    out = cplb.restrict(torch.tensor(x, device="cuda"), F).cpu().numpy()
    want = x.astype(np.float64).reshape(n, H, F, Wd, F).mean(axis=(2, 4))
    assert out.shape == (n, H, Wd)
    np.testing.assert_allclose(out, want, rtol=0, atol=2e-6 * np.abs(x).max())


def test_infer_equals_forward_bitwise(cplb):
    """The inference path (no FP32 pre-activations, output written by the
    last convolution) gives the training forward's output bit for bit, on
    another stream too."""
    import torch
    net, theta, x, tp = setup_net(cplb, 3, 16, 48, seed=5)
    net.set_output_scale(2.5, 0.7)
    a = net.forward(tp).cpu().numpy()
    b = net.infer(tp).cpu().numpy()
    assert np.array_equal(a, b)
    s = torch.cuda.Stream()
    net.set_stream(s)
    c = net.infer(tp[:2].contiguous()).cpu().numpy()
    assert np.array_equal(a[:2], c)
    net.close()
