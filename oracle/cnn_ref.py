"""FP64 CPU oracle of the closure network (test infrastructure only).

The closure network maps coarse-grid fields to per-node corrections
(s1, s2) of the two scalars.  Its architecture is fixed:

    x (C0 = 16 input planes; unused planes are zero)
    z1 = conv3x3(x;  W1, b1)   16 -> 32   a1 = lrelu(z1)
    z2 = conv3x3(a1; W2, b2)   32 -> 32   a2 = lrelu(z2)
    z3 = conv3x3(a2; W3, b3)   32 -> 32   a3 = lrelu(z3)
    z4 = conv3x3(a3; W4, b4)   32 -> 16   outputs = z4[channels 0, 1]

with lrelu(z) = z for z > 0 and 0.1 z otherwise, 3x3 cross-correlation
y[co, r, c] = b[co] + sum_{ci, dy, dx} W[co, ci, dy + 1, dx + 1] x[ci, r + dy, c + dx],
periodic in x (columns) and zero outside the sample in y (rows), and the
loss L = mean over both outputs and every node of (output - target)^2.
What is applied to a coarse run (``output``) is the outputs times their
scales, balanced per sample: half the sample's mean of s1 + s2 is taken from
both, so that the corrections add nothing to the sample's total scalar.

The parameter vector stacks, layer by layer, W[co][ci][ky][kx] then b[co].

Everything here is plain numpy in float64: the forward pass as written
above, and its gradient by the chain rule (the adjoint of the padded
correlation is the correlation with the flipped kernel under the same
padding).  An optional storage model rounds the stored operands to BF16
the way a mixed-precision implementation keeps them (see ``forward``).
tests/test_closure_oracle.py pins it against a direct loop convolution,
central finite differences and translation equivariance.
"""
from __future__ import annotations

import numpy as np

LAYERS = ((16, 32), (32, 32), (32, 32), (32, 16))  # (C_in, C_out)
SLOPE = 0.1


def num_params() -> int:
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def unpack(theta):
    """[(W[co][ci][3][3], b[co])] from the flat parameter vector."""
    out, k = [], 0
    for ci, co in LAYERS:
        W = theta[k:k + co * ci * 9].reshape(co, ci, 3, 3)
        k += co * ci * 9
        b = theta[k:k + co]
        k += co
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(seed: int) -> np.ndarray:
    """He-style normal initialisation (std sqrt(2 / (9 C_in))), zero biases;
    the last layer starts at 1/10 of that scale."""
    rng = np.random.default_rng(seed)
    layers = []
    for n, (ci, co) in enumerate(LAYERS):
        std = np.sqrt(2.0 / (9 * ci)) * (0.1 if n == len(LAYERS) - 1 else 1.0)
        layers.append((rng.normal(0.0, std, size=(co, ci, 3, 3)), np.zeros(co)))
    return pack(layers)


def shifted(x, dy, dx):
    """s[..., r, c] = x[..., r + dy, (c + dx) mod W], zero where r + dy is
    outside [0, H)."""
    H = x.shape[-2]
    s = np.roll(x, -dx, axis=-1)
    out = np.zeros_like(s)
    if dy == 0:
        out[...] = s
    elif dy > 0:
        out[..., :H - dy, :] = s[..., dy:, :]
    else:
        out[..., -dy:, :] = s[..., :H + dy, :]
    return out


def conv(x, W, b):
    """x [B, C_in, H, W] -> y [B, C_out, H, W] (the padded 3x3 correlation)."""
    y = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for ky in range(3):
        for kx in range(3):
            xs = shifted(x, ky - 1, kx - 1)
            y += np.einsum("oi,bihw->bohw", W[:, :, ky, kx], xs)
    return y + b[None, :, None, None]


def conv_adjoint(g, W):
    """Adjoint of conv in x: dL/dx from dL/dy = g."""
    dx = np.zeros((g.shape[0], W.shape[1]) + g.shape[2:])
    for ky in range(3):
        for kx in range(3):
            t = np.einsum("oi,bohw->bihw", W[:, :, ky, kx], g)
            dx += shifted(t, -(ky - 1), -(kx - 1))
    return dx


def conv_weight_grad(x, g):
    """dL/dW [co, ci, 3, 3] and dL/db [co] from input x and dL/dy = g."""
    dW = np.zeros((g.shape[1], x.shape[1], 3, 3))
    for ky in range(3):
        for kx in range(3):
            xs = shifted(x, ky - 1, kx - 1)
            dW[:, :, ky, kx] = np.einsum("bohw,bihw->oi", g, xs)
    return dW, g.sum(axis=(0, 2, 3))


def lrelu(z):
    return np.where(z > 0, z, SLOPE * z)


def lrelu_grad(z):
    return np.where(z > 0, 1.0, SLOPE)


def bf16(a):
    """Round to BF16 (8 significant bits, round to nearest, ties to even),
    returned as float64.  Used to model a network that stores its weights,
    activations and back-propagated gradients in BF16 (``storage="bf16"``)."""
    a = np.asarray(a, dtype=np.float32).copy()
    u = a.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return u.view(np.float32).astype(np.float64)


def _identity(a):
    return np.asarray(a, dtype=np.float64)


def forward(theta, x, storage="f64"):
    """Outputs [B, 2, H, W], the pre-activations [z1..z4] and the layer inputs.

    storage="bf16" rounds what a mixed-precision network stores: the input
    and every layer's activations and weights to BF16, the pre-activations
    to FP32; the arithmetic itself stays FP64."""
    rnd = bf16 if storage == "bf16" else _identity
    f32 = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if storage == "bf16" else _identity
    layers = unpack(np.asarray(theta, dtype=np.float64))
    a = rnd(x)
    zs, ins = [], []
    for n, (W, b) in enumerate(layers):
        ins.append(a)
        z = f32(conv(a, rnd(W), b))
        zs.append(z)
        a = rnd(lrelu(z) if n < len(layers) - 1 else z)
    return zs[-1][:, :2], zs, ins


def balance(out):
    """out [B, 2, H, W] minus half of each sample's mean of out[:, 0] + out[:, 1]."""
    out = np.asarray(out, dtype=np.float64)
    m = (out[:, 0] + out[:, 1]).mean(axis=(1, 2)) / 2.0
    return out - m[:, None, None, None]


def output(theta, x, scale=(1.0, 1.0), storage="f64"):
    """The corrections applied to a coarse run: scaled outputs, balanced."""
    out = forward(theta, x, storage)[0]
    return balance(out * np.asarray(scale, dtype=np.float64)[None, :, None, None])


def loss_and_grad(theta, x, target, storage="f64"):
    """Mean squared error and its gradient with respect to theta
    (storage="bf16": the back-propagated gradients dL/dz are stored in BF16
    too, as are the weights they meet)."""
    rnd = bf16 if storage == "bf16" else _identity
    layers = unpack(np.asarray(theta, dtype=np.float64))
    out, zs, ins = forward(theta, x, storage)
    r = out - target
    P = r[:, 0].size  # pixels; the mean runs over both outputs of each
    loss = float(np.sum(r * r) / (2 * P))
    g = np.zeros_like(zs[-1])
    g[:, :2] = rnd(r / P)
    grads = [None] * len(layers)
    for n in range(len(layers) - 1, -1, -1):
        W, _ = layers[n]
        grads[n] = conv_weight_grad(ins[n], g)
        if n > 0:
            g = rnd(conv_adjoint(g, rnd(W)) * lrelu_grad(zs[n - 1]))
    return loss, pack(grads)


def conv_direct(x, W, b):
    """The same correlation by explicit loops (small inputs only)."""
    B, Ci, H, Wd = x.shape
    Co = W.shape[0]
    y = np.zeros((B, Co, H, Wd))
    for bb in range(B):
        for o in range(Co):
            for r in range(H):
                for c in range(Wd):
                    s = b[o]
                    for i in range(Ci):
                        for ky in range(3):
                            rr = r + ky - 1
                            if rr < 0 or rr >= H:
                                continue
                            for kx in range(3):
                                s += W[o, i, ky, kx] * x[bb, i, rr, (c + kx - 1) % Wd]
                    y[bb, o, r, c] = s
    return y
