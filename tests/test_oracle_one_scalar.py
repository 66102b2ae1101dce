"""Pins of the oracle's one-scalar model (Sec. II D, III D): the total
concentration c = c1 + c2 carried by one population set h3 with
h3^eq built on c / K_eff and a per-node relaxation time from
D_eff = D1 Keq phi + D2 (1 - phi).

Each pin is fixed by the mathematics or by the paper's own 1-D tests
(Sec. IV A), not by the oracle's code:
  - sum_i h3^eq = c and sum_i H3 = 0: total solute conserved to round-off;
  - in a bulk phase (phi = 1 with Keq = 1, or phi = 0 with any Keq) the
    one-scalar model is the two-scalar model's c1 (resp. c2) equation, so
    the two trajectories coincide to round-off, with flow;
  - a Fourier mode in phi = 1 decays at D1 k^2 for any Keq: the 1/K_eff of
    the equilibrium and the Keq of D_eff cancel (Eq. (31) with K_eff = Keq);
  - the steady state is c / K_eff uniform (Eq. (31) has zero flux there),
    at the value fixed by the total solute;
  - pseudo-single-phase case (D1 = D2, Keq = 1): one- and two-scalar
    models agree (Sec. IV A 1);
  - large diffusivity ratio (D1 / D2 = 10^4, Keq = 1): the one-scalar
    model leaks solute into phase 2, the two-scalar model does not
    (Sec. IV A 4).
"""
import numpy as np
import pytest

import workloads as W
from oracle import ref


def one_d(N):
    """Nodes of [-1, 1] (cell centres) and the signed distance of the drop
    |x| < 1/2 in lattice units (phase 1 inside)."""
    x = (np.arange(N) + 0.5) / N * 2.0 - 1.0
    return x, (0.5 - np.abs(x)) * N / 2.0


def total_c(o):
    return o.field("c1") + o.field("c2")


def test_one_scalar_conserves_total_solute():
    p = W.params(nx=23, ny=19, periodic=(1, 0, 1), sigma=3e-3, rho1=3.0, rho2=1.0,
                 visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07, D2=0.02, Keq=0.6,
                 g=(0.0, -2e-5, 0.0), rho_ref=1.5, scalar_model="one")
    f = W.random_fields(p, seed=8)
    o = ref.Oracle(p)
    o.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    r0 = o.reduce()
    o.step(300)
    r = o.reduce()
    assert r["nonfinite"] == 0
    assert abs(r["sum_c"] - r0["sum_c"]) <= 1e-13 * abs(r0["sum_c"])
    assert abs(r["sum_phi"] - r0["sum_phi"]) <= 1e-13 * abs(r0["sum_phi"])
    # c1, c2 read back as the phase parts of c at interfacial equilibrium
    phi, c1, c2 = o.field("phi"), o.field("c1"), o.field("c2")
    keff = p["Keq"] * phi + 1.0 - phi
    np.testing.assert_allclose(c1, p["Keq"] * phi * (c1 + c2) / keff, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("phi0,keq", [(1.0, 1.0), (0.0, 2.5)])
def test_bulk_phase_reduces_to_two_scalar(phi0, keq):
    shp = (17, 24)
    common = dict(nx=24, ny=17, periodic=(1, 1, 1), sigma=0.01, D1=0.07, D2=0.02, Keq=keq,
                  A=0.1, rho1=2.0, rho2=1.0)
    rng = np.random.default_rng(1)
    c = 0.5 + 0.3 * rng.random(shp)
    u = np.zeros((2,) + shp)
    u[0], u[1] = 0.03, -0.02  # uniform flow: advection and the d_t(c u) source
    phi, z = np.full(shp, phi0), np.zeros(shp)
    one = ref.Oracle(W.params(**common, scalar_model="one"))
    two = ref.Oracle(W.params(**common, scalar_model="two"))
    one.init_fields(phi, c, z, u=u)
    if phi0 == 1.0:
        two.init_fields(phi, c, z, u=u)
    else:
        two.init_fields(phi, z, c, u=u)
    one.step(200)
    two.step(200)
    want = two.field("c1" if phi0 == 1.0 else "c2")
    got = total_c(one)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    assert np.abs(got - c).max() > 1e-3  # the field did evolve


@pytest.mark.parametrize("keq", [3.0, 1.0, 0.6])
def test_mode_decays_at_bulk_diffusivity_for_any_keq(keq):
    """(The rest equilibrium c (1 - (1 - w0) / K_eff) and the effective sound
    speed cs^2 / K_eff bound the model's stable range on D2Q9 to
    K_eff >= 1 - w0 = 5/9; Keq = 0.25 in phase 1 diverges.)"""
    N, D1, T = 64, 0.02, 2000
    k = 2 * np.pi / N
    p = W.params(nx=N, ny=1, periodic=(1, 1, 1), sigma=0.0, D1=D1, D2=0.1, Keq=keq,
                 scalar_model="one")
    o = ref.Oracle(p)
    c = 1.0 + 0.1 * np.cos(k * np.arange(N))
    o.init_fields(np.ones((1, N)), c.reshape(1, N), np.zeros((1, N)))
    o.step(T)
    amp = np.abs(np.fft.rfft(total_c(o)[0])[1]) / (N / 2)
    rate = -np.log(amp / 0.1) / T
    # O((k dx)^2) lattice correction: 0.2-0.3 % here; Keq or 1/Keq would be 3x off
    assert abs(rate / (D1 * k * k) - 1.0) <= 1e-2, rate / (D1 * k * k)


@pytest.mark.parametrize("keq", [1.0 / 3.0, 3.0])
def test_steady_state_is_uniform_c_over_keff(keq):
    N = 40
    _, l = one_d(N)
    p = W.params(nx=N, ny=1, periodic=(1, 1, 1), sigma=0.0, D1=0.15, D2=0.1, Keq=keq,
                 scalar_model="one")
    o = ref.Oracle(p)
    o.init_sdf(l.reshape(1, N), c1=(0.0, 2.0))
    o.step(40000)
    phi, c = o.field("phi")[0], total_c(o)[0]
    keff = keq * phi + 1.0 - phi
    plateau = c.sum() / keff.sum()
    assert np.abs(c / keff - plateau).max() <= 1e-9 * plateau
    assert abs(c.sum() - o.reduce()["sum_c"]) <= 1e-12 * c.sum()


def test_pseudo_single_phase_one_and_two_scalar_agree():
    """Sec. IV A 1: D1 = D2, Keq = 1, c1 = 5 exp(-4 x^2) phi,
    c2 = 5 exp(-4 x^2) (1 - phi) on [-1, 1] (N = 200)."""
    N = 200
    x, l = one_d(N)
    phi0 = 0.5 + 0.5 * np.tanh(2.0 * l / 4.0)
    g = 5.0 * np.exp(-4.0 * x ** 2)
    out = {}
    for model in ("one", "two"):
        p = W.params(nx=N, ny=1, periodic=(1, 1, 1), sigma=0.0, D1=0.05, D2=0.05, Keq=1.0,
                     scalar_model=model)
        o = ref.Oracle(p)
        o.init_fields(phi0.reshape(1, N), (g * phi0).reshape(1, N), (g * (1 - phi0)).reshape(1, N))
        o.step(2000)
        out[model] = total_c(o)[0]
    d = np.abs(out["one"] - out["two"]).max() / out["two"].max()
    assert d <= 2e-3, d
    assert np.abs(out["two"] - g).max() > 0.05 * g.max()  # both have diffused visibly


def test_large_diffusivity_ratio_one_scalar_leaks():
    """Sec. IV A 4: D1 = 1, D2 = 1e-4 (here 0.1 and 1e-5 in lattice units),
    Keq = 1, solute initially c1 = phi (two-scalar) or c = phi (one-scalar).
    Leakage: the share of the solute at nodes of phase 2 (phi < 0.01)."""
    N, T = 200, 5000
    _, l = one_d(N)
    leak, peak = {}, {}
    for model in ("two", "one"):
        p = W.params(nx=N, ny=1, periodic=(1, 1, 1), sigma=0.0, D1=0.1, D2=1e-5, Keq=1.0,
                     scalar_model=model)
        o = ref.Oracle(p)
        o.init_sdf(l.reshape(1, N), c1=(0.0, 1.0))
        o.step(T)
        phi, c = o.field("phi")[0], total_c(o)[0]
        out = phi < 0.01
        leak[model] = c[out].sum() / c.sum()
        peak[model] = c[out].max()
    assert leak["two"] <= 1e-3 and peak["two"] <= 0.02, (leak, peak)
    assert leak["one"] >= 0.02 and peak["one"] >= 0.3, (leak, peak)
