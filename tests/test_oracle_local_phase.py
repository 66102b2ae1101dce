"""Pins of the oracle's local scheme for grad phi and |grad phi| (Sec. III C,
after Eq. (39)): |grad phi| = (-|C| - B) / D, grad phi = C / (D + B / |grad
phi|), with C = sum c_i f_i - phi u + d_t(phi u) / 2, D = -tau_f cs^2 and
B = 4 M phi (1 - phi) / W, u and d_t(phi u) taken from the previous level
(reading: the force needs grad phi before u is known).

The scheme recovers grad phi from the non-equilibrium part of the phase
populations, so it is pinned by what the phase-field equation fixes
whichever gradient it is fed: the equilibrium tanh profile of width W, the
Laplace pressure of a drop, the transport of an interface by a uniform flow,
and agreement with the central stencil to the order of the discretisation.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ref


def make(p, phi, c1, c2, u=None):
    o = ref.Oracle(p)
    o.init_fields(phi, c1, c2, u=u)
    return o


def _relaxed_profile_error(scheme, widen):
    N, Wd = 128, 4.0
    p = W.params(nx=N, ny=4, sigma=0.0, W=Wd, M=0.02, D1=0.1, D2=0.1, phase_grad=scheme)
    l = W.sdf_slab(p, 0, 32.0, 96.0)
    phi_wide = 0.5 + 0.5 * np.tanh(2.0 * l / (widen * Wd))
    o = make(p, phi_wide, phi_wide.copy(), np.zeros_like(phi_wide))
    o.step(20000)
    exact = 0.5 + 0.5 * np.tanh(2.0 * l / Wd)
    return float(np.abs(o.field("phi") - exact).max())


def test_local_phase_gradient_relaxes_to_the_tanh_profile():
    """A planar interface started 1.25 x too wide relaxes to the profile of
    width W, as with the central stencil (pin P5).  From twice too wide it
    does not: C sees only the populations' non-equilibrium part, and a
    terraced phi (plateaus three nodes long) is a steady state of it --
    measured 0.040 max error against 0.0063 for the central stencil.  This
    limit of the local scheme is pinned so that it stays visible."""
    assert _relaxed_profile_error("local", 1.25) < 0.01
    assert _relaxed_profile_error("central", 2.0) < 0.01
    assert _relaxed_profile_error("local", 2.0) > 0.03


def test_local_phase_gradient_laplace_pressure():
    """A static drop keeps the Laplace pressure sigma / R within the same
    bound as with the central stencil (pin P4; measured ratio 0.976)."""
    n, R, Wd = 64, 16.0, 4.0
    p = W.params(nx=n, ny=n, sigma=0.01, W=Wd, rho1=1.0, rho2=1.0, mu1=0.1, mu2=0.1, D1=0.1,
                 D2=0.01, Keq=0.5, A=0.1, phase_grad="local")
    o = ref.Oracle(p)
    o.init_sdf(W.sdf_sphere(p, (n / 2.0, n / 2.0), R), c1=(0.0, 1.0), c2=(0.0, 0.0))
    o.step(12000)
    pr = o.field("p")
    r = np.sqrt(sum((x - n / 2.0) ** 2 for x in W.coordinates(p)))
    dp = pr[r < R - Wd].mean() - pr[r > R + Wd].mean()
    assert abs(dp / (0.01 / R) - 1) < 0.08, dp / (0.01 / R)


def test_local_phase_gradient_carries_an_interface_with_the_flow():
    """A planar interface in a uniform flow u0 (matched densities, no
    surface tension) moves at u0 and keeps its width: after t steps the
    profile is the initial one shifted by u0 t."""
    N, Wd, u0, t = 128, 4.0, 0.05, 1280
    p = W.params(nx=N, ny=1, sigma=0.0, W=Wd, M=0.02, D1=0.1, D2=0.1, phase_grad="local")
    l = W.sdf_slab(p, 0, 32.0, 96.0)
    phi0 = 0.5 + 0.5 * np.tanh(2.0 * l / Wd)
    u = np.zeros((2,) + W.shape_of(p))
    u[0] = u0
    o = make(p, phi0, np.zeros_like(phi0), np.zeros_like(phi0), u=u)
    o.step(t)
    shifted = np.roll(phi0[0], int(round(u0 * t)))
    assert np.abs(o.field("phi")[0] - shifted).max() < 0.02


def test_local_and_central_phase_gradients_agree():
    """The same static drop with the local and the central gradient: the
    phase fields agree to the discretisation error of either (measured
    difference 2.3e-4 relative L2), far below the drop's own change over the
    run (4.9e-3), and both conserve the phase to round-off."""
    n = 64
    out = {}
    for scheme in ("central", "local"):
        p = W.params(nx=n, ny=n, sigma=0.01, W=4.0, rho1=3.0, rho2=1.0, mu1=0.1, mu2=0.05,
                     D1=0.1, D2=0.02, Keq=0.5, A=0.1, phase_grad=scheme)
        sdf = W.sdf_sphere(p, (n / 2.0, n / 2.0), 12.0)
        o = ref.Oracle(p)
        o.init_sdf(sdf, c1=(0.0, 1.0), c2=(0.0, 0.0))
        s0 = o.reduce()["sum_phi"]
        phi_init = o.field("phi")
        o.step(2000)
        assert abs(o.reduce()["sum_phi"] - s0) <= 1e-12 * s0
        out[scheme] = o.field("phi")
    d = np.linalg.norm(out["local"] - out["central"]) / np.linalg.norm(out["central"])
    moved = np.linalg.norm(out["central"] - phi_init) / np.linalg.norm(out["central"])
    assert d < 1e-3, d
    assert d < 0.2 * moved, (d, moved)
