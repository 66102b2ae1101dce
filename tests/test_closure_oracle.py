"""Pins of the FP64 closure-network oracle (CPU): the vectorised correlation
equals a direct loop, its adjoint satisfies <conv(x), g> = <x, adj(g)>, the
analytic gradient equals central finite differences of the loss, and the
network is equivariant to periodic shifts in x."""
import numpy as np
import pytest

from oracle import cnn_ref as C


def small_case(seed, B=2, H=5, W=6):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(B, 16, H, W))
    t = rng.normal(size=(B, 2, H, W)) * 0.1
    theta = C.init_params(seed) * 3.0  # larger last layer: every layer matters
    theta += rng.normal(size=theta.size) * 0.01  # non-zero biases
    return x, t, theta


def test_conv_matches_direct_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 4, 5))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    np.testing.assert_allclose(C.conv(x, W, b), C.conv_direct(x, W, b), rtol=1e-13, atol=1e-13)


def test_adjoint_identity():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 5, 6, 7))
    g = rng.normal(size=(2, 4, 6, 7))
    W = rng.normal(size=(4, 5, 3, 3))
    lhs = np.sum(C.conv(x, W, np.zeros(4)) * g)
    rhs = np.sum(x * C.conv_adjoint(g, W))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gradient_matches_finite_differences():
    x, t, theta = small_case(2)
    loss, grad = C.loss_and_grad(theta, x, t)
    rng = np.random.default_rng(3)
    # every layer's weights and biases, including the output layer's channels 0 and 1
    idx = list(rng.choice(theta.size, size=60, replace=False))
    k = 0
    for ci, co in C.LAYERS:
        idx += [k, k + co * ci * 9, k + co * ci * 9 + 1]  # first weight, first biases of each layer
        k += co * ci * 9 + co
    h = 1e-5  # the loss is ~90 here: smaller steps drown in its round-off (eps L / h)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (C.loss_and_grad(tp, x, t)[0] - C.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1e-3, abs(grad[i])) + 1e-10, (i, fd, grad[i])


def test_periodic_shift_equivariance_in_x():
    x, t, theta = small_case(4, W=8)
    out = C.forward(theta, x)[0]
    out_s = C.forward(theta, np.roll(x, 3, axis=-1))[0]
    np.testing.assert_allclose(np.roll(out, 3, axis=-1), out_s, rtol=1e-12, atol=1e-14)


def test_zero_padding_in_y_is_per_sample():
    """Stacking samples along the batch axis must not couple them."""
    x, t, theta = small_case(5, B=3)
    out = C.forward(theta, x)[0]
    for b in range(3):
        ob = C.forward(theta, x[b:b + 1])[0]
        np.testing.assert_allclose(ob[0], out[b], rtol=1e-13, atol=1e-15)


def test_param_vector_layout():
    assert C.num_params() == 32 * 16 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 16 * 32 * 9 + 16
    theta = np.arange(C.num_params(), dtype=np.float64)
    assert np.array_equal(C.pack(C.unpack(theta)), theta)


def test_oracle_closure_term_closed_form():
    """Uniform fields at partition equilibrium (no exchange, no gradients)
    and a uniform closure (x, -x), a pure exchange: one step lowers c1 by x
    and raises c2 by x exactly -- the closure's source is the inverse of the
    implicit recovery's response (Sec. III C) applied to the correction."""
    import workloads as W
    from oracle import ref
    p = W.params(nx=6, ny=5, D1=0.07, D2=0.02, Keq=0.6, A=0.4)
    phi, K = 0.3, p["Keq"]
    c2 = 0.5
    c1 = K * phi * c2 / (1.0 - phi)  # e = Keq phi c2 - (1 - phi) c1 = 0
    shp = W.shape_of(p)
    o = ref.Oracle(p)
    o.init_fields(np.full(shp, phi), np.full(shp, c1), np.full(shp, c2))
    x = 1.7e-3
    o.set_closure(np.stack([np.full(shp, x), np.full(shp, -x)]))
    o.step(1)
    np.testing.assert_allclose(o.field("c1"), c1 - x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(o.field("c2"), c2 + x, rtol=0, atol=1e-15)
    np.testing.assert_allclose(o.field("phi"), phi, rtol=0, atol=1e-15)
    # without the closure the state stays put
    o2 = ref.Oracle(p)
    o2.init_fields(np.full(shp, phi), np.full(shp, c1), np.full(shp, c2))
    o2.step(1)
    np.testing.assert_allclose(o2.field("c1"), c1, rtol=0, atol=1e-15)
    # the source it carries: S_k = c_k - s_k with the exact recovery
    # c1' = S1 + a e', c2' = S2 - a e', e' = (Keq phi S2 - (1 - phi) S1) /
    # (1 + a (Keq phi + 1 - phi)), a = A D_m / 2, inverted by hand
    Dm = p["D1"] * p["D2"] / (K * p["D1"] * (1 - phi) + p["D2"] * phi)
    a = 0.5 * p["A"] * Dm
    s1 = (1 + a * (1 - phi)) * x + a * K * phi * x
    s2 = -a * (1 - phi) * x - (1 + a * K * phi) * x
    S1, S2 = c1 - s1, c2 - s2
    e = (K * phi * S2 - (1 - phi) * S1) / (1 + a * (K * phi + 1 - phi))
    assert abs(S1 + a * e - (c1 - x)) <= 1e-15 and abs(S2 - a * e - (c2 + x)) <= 1e-15


def test_bf16_rounding_is_round_to_nearest_even():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins (1)
    vals = np.array([1.0, 1 + 2.0**-8, 1 + 3 * 2.0**-8, 1 + 2.0**-9, -(1 + 2.0**-8), 3.14159, 1e-30])
    want = np.array([1.0, 1.0, 1 + 2.0**-6, 1.0, -1.0, 3.140625, None], dtype=object)
    got = C.bf16(vals)
    for g, w in zip(got[:-1], want[:-1]):
        assert g == w, (g, w)
    assert abs(got[-1] - 1e-30) <= 1e-30 * 2.0**-8


def test_bf16_storage_model_is_close_to_fp64():
    """The BF16 storage model differs from the FP64 network by BF16-sized
    amounts only (and equals it when every stored value is exact)."""
    x, t, theta = small_case(6)
    l64, g64 = C.loss_and_grad(theta, x, t)
    l16, g16 = C.loss_and_grad(theta, x, t, storage="bf16")
    assert abs(l16 - l64) <= 3e-2 * l64
    assert np.linalg.norm(g16 - g64) <= 0.1 * np.linalg.norm(g64)
    # exact case: inputs and weights representable, zero target and biases
    th = C.bf16(theta) * 0
    k = 0
    for ci, co in C.LAYERS:
        th[k:k + co * ci * 9] = C.bf16(theta[k:k + co * ci * 9] * 0 + 0.125)
        k += co * ci * 9 + co
    xx = np.ones_like(x)
    o64 = C.forward(th, xx)[0]
    o16 = C.forward(th, xx, storage="bf16")[0]
    assert np.max(np.abs(o16 - o64)) <= 1e-2 * np.max(np.abs(o64))


def test_balance_removes_the_total_per_sample():
    """The applied corrections add nothing to each sample's total scalar and
    keep the exchange part s1 - s2 of the outputs unchanged."""
    x, t, theta = small_case(8, B=3)
    raw = C.forward(theta, x)[0]
    out = C.output(theta, x, scale=(2.0, 0.5))
    np.testing.assert_allclose((out[:, 0] + out[:, 1]).sum(axis=(1, 2)), 0.0, atol=1e-12)
    np.testing.assert_allclose(out[:, 0] - out[:, 1], 2.0 * raw[:, 0] - 0.5 * raw[:, 1],
                               rtol=1e-12, atol=1e-14)
    # a pure exchange (s2 = -s1) passes through unchanged
    ex = np.stack([raw[:, 0], -raw[:, 0]], axis=1)
    np.testing.assert_allclose(C.balance(ex), ex, rtol=0, atol=1e-15)


def test_oracle_closure_corrections_per_scalar():
    """Uniform fields at partition equilibrium and uniform corrections
    (x1, x2) of either sign: one step lowers c1 by x1 and c2 by x2, so the
    total by x1 + x2 per node."""
    import workloads as W
    from oracle import ref
    p = W.params(nx=6, ny=5, D1=0.07, D2=0.02, Keq=0.6, A=0.4)
    phi, K = 0.3, p["Keq"]
    c2 = 0.5
    c1 = K * phi * c2 / (1.0 - phi)
    shp = W.shape_of(p)
    o = ref.Oracle(p)
    o.init_fields(np.full(shp, phi), np.full(shp, c1), np.full(shp, c2))
    x1, x2 = 1.1e-3, 2.3e-3
    o.set_closure(np.stack([np.full(shp, x1), np.full(shp, x2)]))
    o.step(1)
    np.testing.assert_allclose(o.field("c1"), c1 - x1, rtol=0, atol=1e-15)
    np.testing.assert_allclose(o.field("c2"), c2 - x2, rtol=0, atol=1e-15)
    r = o.reduce()
    n = np.prod(shp)
    assert abs(r["sum_c"] - n * (c1 + c2 - x1 - x2)) <= 1e-13 * n
