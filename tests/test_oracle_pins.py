"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with a re-typing of its own formulas: each
checks a closed form, an invariant, a convergence order or a limit that the
method must satisfy, chosen so that a plausible slip (a dropped source term,
a wrong sign, a wrong weight, cs^2 or relaxation time, a transposed index)
fails at least one of them.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def make(p, phi, c1, c2, u=None, pr=None):
    o = ref.Oracle(p)
    o.init_fields(phi, c1, c2, u=u, p=pr)
    return o


def uniform(p, value):
    return np.full(W.shape_of(p), float(value))


# --------------------------------------------------------------------------
# P1  0-D interfacial exchange (sources H_k and the implicit recovery,
#     Sec. III C).  With uniform fields and no flow only the zeroth moments
#     act: c_k^{n+1} = c_k^n + (M_k^n + M_k^{n+1})/2, so the disequilibrium
#     e = Keq phi c2 - (1-phi) c1 obeys e^{n+1} = r e^n exactly with
#     r = (1 - lam/2)/(1 + lam/2), lam = A D_m (Keq phi + 1 - phi), and
#     c1 + c2 is constant.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,A", [("d2q9", 0.5), ("d2q9", 200.0), ("d3q19_d3q7", 0.5),
                                       ("d3q19_d3q7", 50.0)])
def test_p1_exchange_decays_geometrically(lattice, A):
    kw = dict(nx=4, ny=3, lattice=lattice, A=A, D1=0.1, D2=0.02, Keq=2.0, sigma=0.01,
              rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.2, mu2=0.1)
    if lattice != "d2q9":
        kw.update(nz=3)
    p = W.params(**kw)
    phi0, K = 0.3, 2.0
    o = make(p, uniform(p, phi0), uniform(p, 0.7), uniform(p, 0.2))
    Dm = p["D1"] * p["D2"] / (K * p["D1"] * (1 - phi0) + p["D2"] * phi0)
    lam = A * Dm * (K * phi0 + 1 - phi0)
    r = (1 - lam / 2) / (1 + lam / 2)
    es, sums = [], []
    for _ in range(80):
        phi, c1, c2 = o.field("phi"), o.field("c1"), o.field("c2")
        assert np.ptp(phi) == 0 and np.ptp(c1) < 1e-15 and np.ptp(c2) < 1e-15
        es.append(K * phi.flat[0] * c2.flat[0] - (1 - phi.flat[0]) * c1.flat[0])
        sums.append(c1.flat[0] + c2.flat[0])
        o.step(1)
    es = np.array(es)
    expect = es[0] * r ** np.arange(len(es))
    np.testing.assert_allclose(es, expect, rtol=1e-11, atol=1e-13 * abs(es[0]))
    assert np.ptp(sums) < 1e-14
    if lam > 2:
        assert np.all(np.sign(es[1:10]) != np.sign(es[:9]))  # overdamped: r < 0


def test_p1_equilibrium_is_henry_ratio():
    """Fixed point of the exchange: c~1 / c~2 = Keq with c~1 = c1/phi,
    c~2 = c2/(1-phi) (interfacial equilibrium, Sec. II C)."""
    p = W.params(nx=3, ny=3, A=5.0, D1=0.1, D2=0.05, Keq=0.25, sigma=0.0)
    phi0 = 0.6
    o = make(p, uniform(p, phi0), uniform(p, 1.0), uniform(p, 0.0))
    o.step(400)
    c1, c2 = o.field("c1").flat[0], o.field("c2").flat[0]
    assert abs((c1 / phi0) / (c2 / (1 - phi0)) - 0.25) < 1e-12
    assert abs(c1 + c2 - 1.0) < 1e-14


# --------------------------------------------------------------------------
# P2  conservation of total phase and total solute to round-off: sum_i F_i = 0,
#     H_1 + H_2 and ~H_1 + ~H_2 have zero sum, periodic streaming and half-way
#     bounce-back move populations without loss (the paper states total heat
#     q1 + q2 is conserved, Sec. IV B 1).
# --------------------------------------------------------------------------
def _conservation(o, steps):
    r0 = o.reduce()
    o.step(steps)
    r1 = o.reduce()
    assert r1["nonfinite"] == 0
    return r0, r1


@pytest.mark.parametrize("case", ["static_drop", "bubble_walls", "droplet3d"])
def test_p2_conservation_workloads(case):
    if case == "static_drop":
        w, steps = W.static_drop_64(), 200
    elif case == "bubble_walls":
        w, steps = W.rising_bubble_2d(nx=64, ny=96), 300
        w["params"]["g"] = (0.0, -1e-4, 0.0)  # strong buoyancy so the flow is far from rest
    else:
        w, steps = W.rising_droplet_3d(n=24), 40
    o = ref.Oracle(w["params"])
    o.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    r0, r1 = _conservation(o, steps)
    assert abs(r1["sum_phi"] - r0["sum_phi"]) <= 1e-13 * abs(r0["sum_phi"])
    assert abs(r1["sum_c"] - r0["sum_c"]) <= 1e-13 * abs(r0["sum_c"])
    assert r1["max_u"] > 0


@pytest.mark.parametrize("lattice,periodic", [("d2q9", (0, 0, 1)), ("d2q9", (1, 0, 1)),
                                              ("d3q19_d3q7", (0, 0, 0)), ("d3q19_d3q7", (1, 0, 1))])
def test_p2_conservation_random_fields(lattice, periodic):
    kw = dict(nx=9, ny=7, lattice=lattice, periodic=periodic, sigma=1e-3, rho1=2.0, rho2=1.0,
              visc_law="exp", mu1=0.3, mu2=0.1, D1=0.05, D2=0.02, Keq=0.7, A=0.3,
              g=(0.0, -1e-4, 0.0))
    if lattice != "d2q9":
        kw.update(nz=6)
    p = W.params(**kw)
    f = W.random_fields(p, seed=1, u_amp=0.01)
    o = make(p, f["phi"], f["c1"], f["c2"], u=f["u"], pr=f["p"])
    r0, r1 = _conservation(o, 60)
    assert abs(r1["sum_phi"] - r0["sum_phi"]) <= 1e-13 * abs(r0["sum_phi"])
    assert abs(r1["sum_c"] - r0["sum_c"]) <= 1e-13 * abs(r0["sum_c"])
    # the individual scalars are NOT conserved: the exchange moves solute
    assert abs(r1["sum_c1"] - r0["sum_c1"]) > 1e-6


# --------------------------------------------------------------------------
# P3  flat equilibrium (Sec. IV A 2): with no flow the two-scalar model
#     relaxes to c1 = c~1 phi, c2 = c~2 (1-phi), c~1 = Keq c~2, so that
#     c1 + Keq c2 is flat; mass fixes c~2 = T/(Keq Phi + N - Phi).  On the
#     planar 1-D interface this is reached to round-off.  A sign error in
#     the interface-flux terms, in ~H or in the exchange breaks it.
# --------------------------------------------------------------------------
def _flat_case(D1, D2, K, N=200, steps=120000, n_eps=1e-9):
    dx = 2.0 / N
    # physical D -> lattice: D_lat = D/6 (dt = dx^2/6); A = 1000 in 1/length^2
    # -> A dx^2 = 0.1 in lattice units
    p = W.params(nx=N, ny=1, sigma=0.0, W=4.0, M=0.01, D1=D1 / 6, D2=D2 / 6, Keq=K, A=0.1,
                 n_eps=n_eps)
    x = -1.0 + np.arange(N) * dx
    l = ((0.25 - x ** 2) / dx).reshape(1, N)  # l = -(x-0.5)(x+0.5), lattice units
    o = ref.Oracle(p)
    o.init_sdf(l, c1=(0.0, 2.0), c2=(0.0, 0.0))
    o.step(steps)
    return o


def _golden_flat():
    rows = []
    for line in open(__file__.replace("test_oracle_pins.py", "golden/flat_equilibrium.txt")):
        line = line.split("#")[0].strip()
        if line:
            rows.append([float(v) for v in line.split()])
    return rows


@pytest.mark.parametrize("D1,D2,K", [(1.0, 1.0, 1.0), (1.0, 1.0, 1 / 3), (10.0, 1.0, 1 / 3)])
def test_p3_flat_equilibrium(D1, D2, K):
    # normal regularisation 1e-9: in 1-D the tails carry no flat mixed region,
    # and the equilibrium is reached to round-off within the run
    o = _flat_case(D1, D2, K)
    phi, c1, c2 = o.field("phi")[0], o.field("c1")[0], o.field("c2")[0]
    N = phi.size
    T, Phi = (c1 + c2).sum(), phi.sum()
    c2t = T / (K * Phi + N - Phi)
    c1t = K * c2t
    assert np.abs(c1 - c1t * phi).max() <= 1e-6 * c1t
    assert np.abs(c2 - c2t * (1 - phi)).max() <= 1e-6 * c2t
    psi = c1 + K * c2
    assert np.ptp(psi) <= 1e-6 * psi.mean()
    # printed values of the paper's worked example (golden fixture)
    for gD1, gD2, gK, plateau in _golden_flat():
        if (gD1, gD2) == (D1, D2) and abs(gK - K) < 1e-12:
            assert abs(psi.mean() - plateau) < 1e-3


@pytest.mark.parametrize("n_eps", [1e-3, 1e-4, 1e-5])
def test_p3_flat_equilibrium_regularised_tail(n_eps):
    # With the regularised normal n = grad phi / sqrt(|grad phi|^2 + n_eps^2)
    # the sharpening flux fades where |grad phi| falls below n_eps: the far
    # tails of the tanh profile stop at phi ~ n_eps / 3 instead of relaxing
    # to round-off, and the flat equilibrium's plateau carries an error of
    # the same size.  Both scale linearly with n_eps (measured 0.27 n_eps and
    # 0.31 n_eps at 1e-3, 1e-4 and 1e-5), which pins the regularisation's
    # only effect: the profile's tails.
    K = 1 / 3
    o = _flat_case(1.0, 1.0, K, n_eps=n_eps)
    phi, c1, c2 = o.field("phi")[0], o.field("c1")[0], o.field("c2")[0]
    N = phi.size
    c2t = (c1 + c2).sum() / (K * phi.sum() + N - phi.sum())
    plateau = np.abs(c1 - K * c2t * phi).max() / (K * c2t)
    flat = np.ptp(c1 + K * c2) / (c1 + K * c2).mean()
    tail = min(phi.min(), 1.0 - phi.max())
    assert 0.1 * n_eps <= plateau <= 0.5 * n_eps, plateau
    assert flat <= 0.5 * n_eps, flat
    assert 0.1 * n_eps <= tail <= 0.5 * n_eps, tail


# --------------------------------------------------------------------------
# P4  Laplace law for a static drop: dp = sigma / R in 2-D, 2 sigma / R in
#     3-D (surface tension enters via beta, k and F_s = mu_phi grad phi).
#     The discrete surface tension converges with the interface resolution
#     W/dx; at W = 4 the static drop sits ~7 % under sigma/R and the gap
#     shrinks several-fold from W = 2 to W = 4.
# --------------------------------------------------------------------------
def _laplace(lattice, n, R, Wd, steps):
    kw = dict(nx=n, ny=n, lattice=lattice, sigma=0.01, W=Wd, rho1=1.0, rho2=1.0,
              mu1=0.1, mu2=0.1, D1=0.1, D2=0.01, Keq=0.5, A=0.1)
    if lattice != "d2q9":
        kw["nz"] = n
    p = W.params(**kw)
    c = [n / 2.0] * W.dim_of(p)
    o = ref.Oracle(p)
    o.init_sdf(W.sdf_sphere(p, c, R), c1=(0.0, 1.0), c2=(0.0, 0.0))
    o.step(steps)
    pr = o.field("p")
    r = np.sqrt(sum((x - ci) ** 2 for x, ci in zip(W.coordinates(p), c)))
    dp = pr[r < R - Wd].mean() - pr[r > R + Wd].mean()
    exact = (0.01 if W.dim_of(p) == 2 else 0.02) / R
    return dp / exact


def test_p4_laplace_2d_converges_with_interface_resolution():
    ratio4 = _laplace("d2q9", 64, 16.0, 4.0, 12000)
    ratio2 = _laplace("d2q9", 64, 16.0, 2.0, 12000)
    assert abs(ratio4 - 1) < 0.08
    assert abs(ratio2 - 1) > 2.0 * abs(ratio4 - 1)


def test_p4_laplace_3d():
    ratio = _laplace("d3q19_d3q7", 32, 8.0, 4.0, 800)
    assert abs(ratio - 1) < 0.08


# --------------------------------------------------------------------------
# P5  conservative Allen-Cahn equilibrium: a planar interface relaxes to the
#     hyperbolic-tangent profile of width W (Sec. II A), here from a profile
#     twice too wide.  A wrong sign or scale of the interface term
#     4 phi (1-phi) n / W in F_i, or a wrong tau_f, gives another width.
# --------------------------------------------------------------------------
def test_p5_allen_cahn_profile():
    N, Wd = 128, 4.0
    p = W.params(nx=N, ny=1, sigma=0.0, W=Wd, M=0.02, D1=0.1, D2=0.1)
    l = W.sdf_slab(p, 0, 32.0, 96.0)
    phi_wide = 0.5 + 0.5 * np.tanh(2.0 * l / (2 * Wd))
    o = make(p, phi_wide, phi_wide.copy(), np.zeros_like(phi_wide))
    o.step(20000)
    phi = o.field("phi")[0]
    exact = 0.5 + 0.5 * np.tanh(2.0 * l[0] / Wd)
    assert np.abs(phi - exact).max() < 0.01
    assert np.abs(phi_wide[0] - exact).max() > 0.1  # the start was far from it


# --------------------------------------------------------------------------
# P6  single-phase diffusion: with phi = 1 the scalar set is a linear
#     advection-diffusion LB, a Fourier mode decays at D k^2 with
#     D = (tau_h - 1/2) cs^2 (cs^2 = 1/3 on D2Q9, 1/4 on D3Q7), to O(k^2),
#     isotropically, and is carried at speed u0.
# --------------------------------------------------------------------------
def _mode(lattice, D, n, steps, diag=False, u0=0.0):
    kw = dict(nx=n, ny=n, lattice=lattice, sigma=0.0, D1=D, D2=D, Keq=1.0, A=0.1)
    if lattice != "d2q9":
        kw["nz"] = n
    p = W.params(**kw)
    xs = W.coordinates(p)
    k = 2 * np.pi / n
    arg = k * (xs[0] + (xs[1] if diag else 0.0))
    k2 = k * k * (2 if diag else 1)
    shp, d = W.shape_of(p), W.dim_of(p)
    u = np.zeros((d,) + shp)
    u[0] = u0
    o = make(p, np.ones(shp), 1 + 0.01 * np.cos(arg), np.zeros(shp), u=u)
    o.step(10)
    a0 = ((o.field("c1") - 1) * np.exp(-1j * arg)).sum()
    o.step(steps)
    a1 = ((o.field("c1") - 1) * np.exp(-1j * arg)).sum()
    ratio = a1 / a0
    return ratio, D * k2 * steps, k * u0 * steps


@pytest.mark.parametrize("lattice,D,diag", [("d2q9", 0.02, False), ("d2q9", 0.02, True),
                                            ("d3q19_d3q7", 0.02, False)])
def test_p6_fourier_mode_decay(lattice, D, diag):
    n1, n2 = (32, 64) if lattice == "d2q9" else (12, 24)
    errs = []
    for n in (n1, n2):
        ratio, expo, _ = _mode(lattice, D, n, int(0.4 * n * n), diag)
        rate_err = -np.log(abs(ratio)) / expo - 1
        errs.append(abs(rate_err))
    assert errs[1] < 0.01
    assert errs[1] < errs[0] / 3  # second order in k dx


def test_p6b_advected_mode():
    """A Fourier mode carried by a uniform flow: phase speed u0, decay D k^2,
    no extra u^2 diffusion (the d_t(c u) source removes it)."""
    D, u0 = 0.05, 0.08
    for n in (64, 128):
        ratio, expo, phase = _mode("d2q9", D, n, int(0.2 * n * n), u0=u0)
        rate = -np.log(abs(ratio)) / expo
        # the phase is taken relative to the exact translation
        dphase = np.angle(ratio * np.exp(1j * phase))
        assert abs(rate - 1) < 0.01, (n, rate)
        assert abs(dphase) < 0.01 * phase, (n, dphase)


# --------------------------------------------------------------------------
# P7  shear wave: single-phase flow, u_x = U sin(k y) decays at nu k^2 with
#     mu = rho (tau_g - 1/2) cs^2 (Sec. III B); with the exponential law at
#     c1 = c2 = 1/2 the viscosity is sqrt(mu1 mu2) (Eq. 4.3).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lattice,law,rho", [("d2q9", "linear", 1.0), ("d2q9", "exp", 2.0),
                                             ("d3q19_d3q7", "linear", 1.0)])
def test_p7_shear_wave(lattice, law, rho):
    # single phase (phi = 1) with c1 = c2 = 1/2: no interface exists, so the
    # normal regularisation is set to 1 to keep round-off gradients of phi
    # from steering the interface-flux terms
    n = 64 if lattice == "d2q9" else 32
    kw = dict(nx=4, ny=n, lattice=lattice, sigma=0.0, rho1=rho, rho2=rho, visc_law=law,
              A=0.0, Keq=1.0, D1=0.1, D2=0.1, n_eps=1.0)
    if lattice != "d2q9":
        kw["nz"] = 4
    kw.update(dict(mu1=0.1, mu2=0.1) if law == "linear" else dict(mu1=0.4, mu2=0.025))
    p = W.params(**kw)
    shp, d, xs = W.shape_of(p), W.dim_of(p), W.coordinates(p)
    k = 2 * np.pi / n
    u = np.zeros((d,) + shp)
    u[0] = 1e-3 * np.sin(k * xs[1])
    o = make(p, np.ones(shp), np.full(shp, 0.5), np.full(shp, 0.5), u=u)
    o.step(10)
    a0 = (o.field("ux") * np.sin(k * xs[1])).sum()
    steps = 500 if lattice == "d2q9" else 200
    o.step(steps)
    a1 = (o.field("ux") * np.sin(k * xs[1])).sum()
    nu = 0.1 / rho
    rate = -np.log(a1 / a0) / steps / (nu * k * k)
    assert abs(rate - 1) < 0.005
    assert np.allclose(o.field("mu"), 0.1, rtol=1e-12)


# --------------------------------------------------------------------------
# P8  channel flow with the exponential viscosity law: half-way bounce-back
#     walls, body force G, c1 = c2 = 1/2 so log mu = (log mu1 + log mu2)/2
#     (Sec. IV B 3 states this value); steady u = G (y+1/2)(H-1/2-y)/(2 mu).
# --------------------------------------------------------------------------
def test_p8_poiseuille_exponential_viscosity():
    ny = 32
    p = W.params(nx=4, ny=ny, periodic=(1, 0, 1), sigma=0.0, rho1=10.0, rho2=1.0,
                 visc_law="exp", mu1=1.0, mu2=0.1, A=0.0, Keq=1.0, D1=0.1, D2=0.1,
                 g=(1e-6, 0.0, 0.0), rho_ref=0.0, n_eps=1.0)
    shp = W.shape_of(p)
    o = make(p, np.ones(shp), np.full(shp, 0.5), np.full(shp, 0.5))
    o.step(40000)
    mu = o.field("mu")
    golden = _golden_value("layered_poiseuille_mu")
    assert np.allclose(mu, golden, rtol=1e-12)
    ux = o.field("ux")[:, 0]
    y = np.arange(ny)
    exact = 10 * 1e-6 / (2 * golden) * (y + 0.5) * (ny - 0.5 - y)
    assert np.abs(ux - exact).max() < 0.01 * exact.max()
    assert np.abs(o.field("uy")).max() < 1e-6 * exact.max()


def _golden_value(key):
    path = __file__.replace("test_oracle_pins.py", "golden/values.txt")
    for line in open(path):
        line = line.split("#")[0].strip()
        if line and line.split()[0] == key:
            return float(line.split()[1])
    raise KeyError(key)


# --------------------------------------------------------------------------
# P9  D1Q3 reduction: a y-uniform D2Q9 lattice with ny = 1 must evolve the
#     phase field and both scalars exactly as a 1-D D1Q3 lattice (weights
#     2/3, 1/6, 1/6) when the flow is at rest (sigma = 0, no gravity): the
#     D2Q9 weights summed over c_y are the D1Q3 weights and the stencils
#     coincide.  The D1Q3 lattice below is written independently, in numpy.
# --------------------------------------------------------------------------
def _d1q3_run(phi0, c10, c20, prm, steps):
    w = np.array([2 / 3, 1 / 6, 1 / 6])
    c = np.array([0, 1, -1])
    cs2 = 1 / 3
    Wd, M, D1, D2, K, A = (prm[k] for k in ("W", "M", "D1", "D2", "Keq", "A"))
    tf, t1, t2 = 0.5 + M / cs2, 0.5 + D1 / cs2, 0.5 + D2 / cs2
    f = w[:, None] * phi0[None]
    h1 = w[:, None] * c10[None]
    h2 = w[:, None] * c20[None]
    out = []
    for s in range(steps + 1):
        phi = f.sum(0)
        S1, S2 = h1.sum(0), h2.sum(0)
        Dm = D1 * D2 / (K * D1 * (1 - phi) + D2 * phi)
        a = 0.5 * A * Dm
        det = 1 + a * (1 - phi) + a * K * phi
        x1 = (S1 * (1 + a * K * phi) + a * K * phi * S2) / det
        x2 = (S2 * (1 + a * (1 - phi)) + a * (1 - phi) * S1) / det
        out.append((phi.copy(), x1.copy(), x2.copy()))
        if s == steps:
            break
        psi = x1 + K * x2
        gphi = (np.roll(phi, -1) - np.roll(phi, 1)) * (1 / 6) / cs2
        gpsi = (np.roll(psi, -1) - np.roll(psi, 1)) * (1 / 6) / cs2
        nx_ = gphi / np.sqrt(gphi * gphi + prm["n_eps"] ** 2)
        ex = A * Dm * (K * x2 * phi - x1 * (1 - phi))
        aux = Dm * gphi * gpsi
        fn, h1n, h2n = np.empty_like(f), np.empty_like(h1), np.empty_like(h2)
        for i in range(3):
            Fi = w[i] * c[i] * nx_ * 4 * phi * (1 - phi) / Wd
            H1 = w[i] * (c[i] * nx_ * 4 * (1 - phi) * x1 / Wd + ex)
            H2 = w[i] * (-c[i] * nx_ * 4 * phi * x2 / Wd - ex)
            fs = f[i] - (f[i] - w[i] * phi) / tf + (1 - 0.5 / tf) * Fi
            hs1 = h1[i] - (h1[i] - w[i] * x1) / t1 + (1 - 0.5 / t1) * H1 - w[i] * aux
            hs2 = h2[i] - (h2[i] - w[i] * x2) / t2 + (1 - 0.5 / t2) * H2 + w[i] * aux
            fn[i], h1n[i], h2n[i] = (np.roll(a_, c[i]) for a_ in (fs, hs1, hs2))
        f, h1, h2 = fn, h1n, h2n
    return out


def test_p9_d1q3_reduction():
    N = 64
    p = W.params(nx=N, ny=1, sigma=0.0, W=4.0, M=0.01, D1=0.12, D2=0.03, Keq=1 / 3, A=0.4,
                 rho1=2.0, rho2=1.0)
    l = W.sdf_slab(p, 0, 16.0, 40.0)[0]
    phi0 = 0.5 + 0.5 * np.tanh(2 * l / 4.0)
    c10, c20 = 2.0 * phi0, 0.1 * (1 - phi0)
    ref1d = _d1q3_run(phi0, c10, c20, p, 150)
    o = make(p, phi0[None], c10[None], c20[None])
    for s in (0, 1, 7, 150):
        o2 = make(p, phi0[None], c10[None], c20[None])
        o2.step(s)
        for name, k in (("phi", 0), ("c1", 1), ("c2", 2)):
            np.testing.assert_allclose(o2.field(name)[0], ref1d[s][k], rtol=0, atol=1e-13)
    del o


# --------------------------------------------------------------------------
# P10 symmetry: a centred drop stays mirror- and 90-degree-rotation
#     symmetric (catches a wrong velocity, weight or opposite in one
#     direction only).
# --------------------------------------------------------------------------
def test_p10_symmetry_2d():
    w = W.static_drop_64()
    o = ref.run_workload(w, steps=150)
    phi, c1, ux, uy, pr = (o.field(k) for k in ("phi", "c1", "ux", "uy", "p"))
    ix = (-np.arange(64)) % 64  # x -> 64 - x about the centre 32
    for s in (phi, c1, pr):
        assert np.abs(s - s[:, ix]).max() < 1e-12
        assert np.abs(s - s[ix, :]).max() < 1e-12
        assert np.abs(s - s.T).max() < 1e-12
    assert np.abs(ux + ux[:, ix]).max() < 1e-14
    assert np.abs(ux - uy.T).max() < 1e-14
    assert np.abs(c1 - c1[:, ix]).max() < 1e-12
    assert np.abs(ux).max() > 1e-6


def test_p10_symmetry_3d():
    p = W.params(nx=20, ny=20, nz=20, lattice="d3q19_d3q7", sigma=0.01, rho1=2.0, rho2=1.0,
                 D1=0.05, D2=0.01, Keq=2.0, A=0.2)
    o = ref.Oracle(p)
    o.init_sdf(W.sdf_sphere(p, (10.0, 10.0, 10.0), 5.0), c1=(0.0, 1.0), c2=(0.2, -0.2))
    o.step(30)
    ix = (-np.arange(20)) % 20
    phi, c2, ux, uz = (o.field(k) for k in ("phi", "c2", "ux", "uz"))
    for s in (phi, c2):
        assert np.abs(s - s[:, :, ix]).max() < 1e-12
        assert np.abs(s - np.transpose(s, (0, 2, 1))).max() < 1e-12
        assert np.abs(s - np.transpose(s, (2, 1, 0))).max() < 1e-12
    assert np.abs(ux - np.transpose(uz, (2, 1, 0))).max() < 1e-14


# --------------------------------------------------------------------------
# Galilean advection: with uniform flow, matched densities and no surface
# tension a drop and its solute translate at u0 (f^eq and h^eq first
# moments phi u and c u, Sec. III).
# --------------------------------------------------------------------------
def test_advection_of_drop():
    n, u0, steps = 64, (0.02, 0.01), 1000
    p = W.params(nx=n, ny=n, sigma=0.0, D1=0.05, D2=0.05, Keq=1.0, A=0.1)
    shp, xs = W.shape_of(p), W.coordinates(p)
    phi = 0.5 + 0.5 * np.tanh(2 * W.sdf_sphere(p, (n / 2, n / 2), 10.0) / 4.0)
    u = np.stack([np.full(shp, u0[0]), np.full(shp, u0[1])])
    o = make(p, phi, phi.copy(), np.zeros(shp), u=u)

    def centroid(f):
        return np.array([(np.angle((f * np.exp(2j * np.pi * xs[a] / n)).sum()) % (2 * np.pi))
                         * n / (2 * np.pi) for a in range(2)])

    c0 = centroid(o.field("phi"))
    o.step(steps)
    disp = centroid(o.field("phi")) - c0
    np.testing.assert_allclose(disp, np.array(u0) * steps, rtol=1e-4)
    np.testing.assert_allclose(centroid(o.field("c1")) - c0, np.array(u0) * steps, rtol=1e-3)


# --------------------------------------------------------------------------
# checkpoint / resume and the error contract of the oracle library
# --------------------------------------------------------------------------
def test_checkpoint_resume_bitwise():
    w = W.rising_bubble_2d(nx=32, ny=48)
    a = ref.run_workload(w, steps=20)
    blob = a.save_state()
    a.step(25)
    b = ref.Oracle(w["params"])
    b.load_state(blob)
    b.step(25)
    for k in ("phi", "c1", "c2", "ux", "uy", "p"):
        assert np.array_equal(a.field(k), b.field(k))
    assert a.reduce()["step"] == b.reduce()["step"] == 45


@pytest.mark.parametrize("bad", [dict(D2=0.0), dict(Keq=0.0), dict(M=-1.0), dict(nx=0),
                                 dict(rho1=0.0), dict(lattice="d2q9", g=(0, 0, 1e-5)),
                                 dict(periodic=(1, 0, 1), ny=1)])
def test_oracle_rejects_bad_parameters(bad):
    with pytest.raises(ref.OracleError) as e:
        ref.Oracle(W.params(**bad))
    assert e.value.code == -1


def test_nonfinite_is_reported():
    p = W.params(nx=5, ny=5)
    phi = np.full(W.shape_of(p), 0.5)
    phi[2, 2] = np.nan
    o = make(p, phi, phi.copy(), phi.copy())
    r = o.reduce()
    assert r["nonfinite"] > 0 and r["rc"] == -4


# --------------------------------------------------------------------------
# Conditioning of the trajectory under the normal regularisation: a 1-ulp
# perturbation of the initial phase field stays at round-off size over the
# run (with the paper's bare n = grad phi/|grad phi| the drop interior, where
# phi overshoots 1 on a flat profile, amplifies it to ~1e-5 within 100 steps).
# This is what makes element-wise parity of long runs meaningful.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n_eps", [1e-3, 1e-5])
def test_trajectory_is_well_conditioned(n_eps):
    # A 1-ulp perturbation of the initial drop stays at round-off over 500
    # steps of the 64^2 static drop for every normal regularisation down to
    # n_eps = 1e-5 (measured: 7e-15 at 1e-3 ... 1e-5); at 5e-6 it grows to
    # 3e-11 and at 1e-6 to 4e-5, where the normal at the drop centre is set
    # by round-off.
    w = W.static_drop_64()
    p = dict(w["params"], n_eps=n_eps)
    phi0 = 0.5 + 0.5 * np.tanh(2 * w["sdf"] / p["W"])
    rng = np.random.default_rng(0)
    a = make(p, phi0, phi0.copy(), np.zeros_like(phi0))
    q = phi0 * (1 + 1e-16 * (2 * rng.random(phi0.shape) - 1))
    b = make(p, q, q.copy(), np.zeros_like(q))
    a.step(500)
    b.step(500)
    for k in ("phi", "c1", "c2", "p"):
        fa, fb = a.field(k), b.field(k)
        assert np.linalg.norm(fa - fb) <= 1e-13 * np.linalg.norm(fa), k


def _mirror_asymmetry_3d(n_eps, steps):
    p = W.params(nx=20, ny=20, nz=20, lattice="d3q19_d3q7", sigma=0.01, rho1=2.0, rho2=1.0,
                 D1=0.05, D2=0.01, Keq=2.0, A=0.2, n_eps=n_eps)
    o = ref.Oracle(p)
    o.init_sdf(W.sdf_sphere(p, (10.0, 10.0, 10.0), 5.0), c1=(0.0, 1.0), c2=(0.2, -0.2))
    o.step(steps)
    phi = o.field("phi")
    o.close()
    ix = (-np.arange(20)) % 20
    return float(np.abs(phi - phi[:, :, ix]).max())


@pytest.mark.parametrize("n_eps,bound", [(1e-3, 1e-13), (1e-4, None)])
def test_regularisation_floor_3d(n_eps, bound):
    # Where the tails of periodic images meet (a 20^3 box, drop radius 5),
    # |grad phi| falls to ~1e-5 and the normal turns over within the nodes
    # where |grad phi| < n_eps.  With n_eps = 1e-3 the turn is smooth and the
    # round-off asymmetry of the mirror-symmetric drop stays at 1e-15 over
    # 300 steps; with 1e-4 the sharpening flux turns abruptly and amplifies it
    # to ~3e-3 (measured: 3e-4 -> 1.4e-9, 1e-4 -> 3.0e-3, 1e-5 -> 4.1e-3).
    # This is why the default stays at 1e-3 although the 2-D drop is well
    # conditioned down to 1e-5.
    a = _mirror_asymmetry_3d(n_eps, 300)
    if bound is not None:
        assert a <= bound, a
    else:
        assert a >= 1e-6, a


# --------------------------------------------------------------------------
# P5b  a phase-field Fourier mode carried by a uniform flow (Sec. III A): a
#      small mode phi = 1/2 + 0.01 cos(k x) with a large normal
#      regularisation (n_eps = 100, so the sharpening flux is linear,
#      M 4 phi (1 - phi) / (W n_eps) grad phi) decays at M_eff k^2,
#      M_eff = M (1 - 4 phibar (1 - phibar) / (W n_eps)), and moves at u0.
#      Without the d_t(phi u) part of F_i the decay carries an extra u0^2
#      diffusion (2 % here).
# --------------------------------------------------------------------------
def test_p5b_advected_phase_mode():
    n, u0, M, neps = 128, 0.08, 0.05, 100.0
    p = W.params(nx=n, ny=n, sigma=0.0, rho1=1.0, rho2=1.0, visc_law="linear", mu1=0.1,
                 mu2=0.1, M=M, A=0.0, Keq=1.0, D1=0.05, D2=0.05, n_eps=neps)
    xs, shp = W.coordinates(p), W.shape_of(p)
    k = 2 * np.pi / n
    arg = k * xs[0]
    u = np.zeros((2,) + shp)
    u[0] = u0
    o = make(p, 0.5 + 0.01 * np.cos(arg), np.zeros(shp), np.zeros(shp), u=u)
    o.step(10)
    a0 = ((o.field("phi") - 0.5) * np.exp(-1j * arg)).sum()
    steps = int(0.2 * n * n)
    o.step(steps)
    a1 = ((o.field("phi") - 0.5) * np.exp(-1j * arg)).sum()
    m_eff = M * (1 - 4 * 0.25 / (p["W"] * neps))
    rate = -np.log(abs(a1 / a0)) / (m_eff * k * k * steps)
    phase = k * u0 * steps
    dphase = np.angle(a1 / a0 * np.exp(1j * phase))
    assert abs(rate - 1) < 0.005, rate
    assert abs(dphase) < 1e-3 * phase, dphase


# --------------------------------------------------------------------------
# P7b  the exponential law's end points (Eq. (4.3)): at (c1, c2) = (1, 0)
#      the viscosity is mu1, at (0, 1) it is mu2 -- the shear wave decays at
#      mu / rho k^2 accordingly (P7 and P8 only see the symmetric point).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("c1,c2,which", [(1.0, 0.0, "mu1"), (0.0, 1.0, "mu2")])
def test_p7b_exponential_law_end_points(c1, c2, which):
    n = 64
    p = W.params(nx=4, ny=n, sigma=0.0, rho1=1.0, rho2=1.0, visc_law="exp", mu1=0.4,
                 mu2=0.025, A=0.0, Keq=1.0, D1=0.1, D2=0.1, n_eps=1.0)
    shp, xs = W.shape_of(p), W.coordinates(p)
    k = 2 * np.pi / n
    u = np.zeros((2,) + shp)
    u[0] = 1e-3 * np.sin(k * xs[1])
    o = make(p, np.ones(shp), np.full(shp, c1), np.full(shp, c2), u=u)
    o.step(10)
    a0 = (o.field("ux") * np.sin(k * xs[1])).sum()
    steps = 300
    o.step(steps)
    a1 = (o.field("ux") * np.sin(k * xs[1])).sum()
    rate = -np.log(a1 / a0) / steps / (p[which] * k * k)
    assert abs(rate - 1) < 0.01, rate
    # the decaying shear leaves c1, c2 uniform to ~1e-7 (the d_t(c u) sources)
    assert np.allclose(o.field("mu"), p[which], rtol=1e-6, atol=0.0)


# --------------------------------------------------------------------------
# P11  Galilean invariance with a density contrast (Sec. III B): a drop
#      (rho1 / rho2 = 10, sigma = 0.01) run once at rest and once with the
#      whole box moving at u0 = (0.02, 0) for 200 steps (a shift of 4 nodes):
#      phi, u - u0 and p agree with the resting run shifted by u0 t to the
#      lattice's O(Ma^2) departure from invariance (1.1e-2, 1.8e-3 and
#      1.2e-3 measured).  The pressure's (rho1 - rho2) u.grad phi term or the
#      (rho1 - rho2)(c.u)(c.grad phi) part of G_i, if dropped, break it by
#      5 to 40 times those amounts.
# --------------------------------------------------------------------------
def test_p11_galilean_invariance_with_density_contrast():
    n, steps, u0 = 64, 200, (0.02, 0.0)

    def run(u):
        p = W.params(nx=n, ny=n, sigma=1e-2, rho1=10.0, rho2=1.0, visc_law="linear", mu1=0.1,
                     mu2=0.1, M=0.02, A=0.0, Keq=1.0, D1=0.05, D2=0.05, n_eps=1e-6)
        shp = W.shape_of(p)
        phi = 0.5 + 0.5 * np.tanh(2 * W.sdf_sphere(p, (n / 2, n / 2), 12.0) / p["W"])
        o = make(p, phi, np.zeros(shp), np.zeros(shp),
                 u=np.stack([np.full(shp, u[0]), np.full(shp, u[1])]))
        o.step(steps)
        return {k: o.field(k) for k in ("phi", "ux", "uy", "p")}

    s, m = run((0.0, 0.0)), run(u0)
    shift = int(round(u0[0] * steps))

    def moved(f):  # the resting field carried by u0 t (x is the last axis)
        return np.roll(f, shift, axis=-1)

    assert np.abs(m["phi"] - moved(s["phi"])).max() < 2e-2
    du = max(np.abs(m["ux"] - u0[0] - moved(s["ux"])).max(), np.abs(m["uy"] - moved(s["uy"])).max())
    assert du < 0.2 * u0[0], du
    assert np.abs(m["p"] - moved(s["p"])).max() < 2e-3


# --------------------------------------------------------------------------
# P12  a flat interface at rest carries no pressure jump and drives no flow
#      (Sec. II A): on the tanh profile of width W the chemical potential
#      4 beta phi (phi - 1)(phi - 1/2) - k lap phi vanishes when beta = 12
#      sigma / W and k = 3 sigma W / 2, so the pressure variation and the
#      velocity left are discretisation errors that fall with (dx / W)^2.
#      A wrong beta or k leaves them at O(sigma / W) whatever W.
# --------------------------------------------------------------------------
def test_p12_flat_interface_carries_no_pressure_jump():
    res = {}
    for Wd in (4.0, 8.0):
        n = 128
        p = W.params(nx=n, ny=4, sigma=1e-2, W=Wd, rho1=1.0, rho2=1.0, visc_law="linear",
                     mu1=0.1, mu2=0.1, M=0.02, A=0.0, Keq=1.0, D1=0.05, D2=0.05, n_eps=1e-6)
        shp, x = W.shape_of(p), W.coordinates(p)[0]
        phi = 0.5 + 0.5 * np.tanh(2 * (32.0 - np.abs(x - 64.0)) / Wd)
        o = make(p, phi, np.zeros(shp), np.zeros(shp))
        o.step(400)
        res[Wd] = (np.ptp(o.field("p")), np.abs(o.field("ux")).max())
    assert res[8.0][0] < 1e-4 and res[8.0][1] < 2e-5, res  # sigma / W = 1.25e-3
    assert res[4.0][0] > 4 * res[8.0][0], res  # second order in dx / W
