"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the
benchmark.

This module holds workload *definitions* only: grid sizes, boundary types,
material and transport parameters in lattice units, signed-distance
geometry and seeded random fields.  It contains none of the method's
arithmetic (no equilibria, no phase profile, no collision); each side --
the CPU oracle and the GPU library -- builds its initial state from these
inputs on its own.

Parameter dictionaries use the keys

    nx, ny, nz, lattice ('d2q9' | 'd3q19_d3q7'), visc_law ('linear' | 'exp'),
    periodic (3 flags), rho1, rho2, mu1, mu2, sigma, W, M, D1, D2, Keq, A,
    g (3-vector), rho_ref, n_eps

plus, for the GPU library only, ``precision`` ('f64' | 'f32' | 'f32_s16f' |
'f32_s16b') and the uniform references of its stored scalar populations,
``ref_h1``, ``ref_h2`` (c1_ref, c2_ref: the concentrations that fill most
of the domain), used where h1, h2 have no per-node reference (one-scalar
model, local gradient scheme).  ``ref_f`` and ``ref_g`` are kept for the
parameter layout: the library stores f relative to each node's own phase
and g relative to a pressure bracket, so ``ref_f`` has no effect and
``ref_g`` must be 0.

Every field array is a numpy float64 array of shape (ny, nx) in 2-D or
(nz, ny, nx) in 3-D (x fastest in memory).
"""
from __future__ import annotations

import copy

import numpy as np

DEFAULTS = dict(
    nx=64, ny=64, nz=1, lattice="d2q9", visc_law="linear", periodic=(1, 1, 1),
    rho1=1.0, rho2=1.0, mu1=0.1, mu2=0.1, sigma=0.01, W=4.0, M=0.01,
    D1=0.1, D2=0.1, Keq=1.0, A=0.1, g=(0.0, 0.0, 0.0), rho_ref=0.0, n_eps=1e-3,
    precision="f64", ref_f=0.0, ref_g=0.0, ref_h1=0.0, ref_h2=0.0, scalar_model="two",
    scalar_bc=("noflux",) * 6, c_wall=((0.0, 0.0),) * 6, scalar_grad="central",
    phase_grad="central",
)


def phase_reference(precision: str, bulk_phi: float = 1.0) -> float:
    """A uniform phase reference for a storage precision: 1/2 for FP64 / FP32,
    the bulk phase for 16-bit storage.  The library takes it in ``ref_f``
    and ignores it (see the module docstring); kept so that parameter sets
    written for uniform references still load."""
    return bulk_phi if precision.startswith("f32_s16") else 0.5


def params(**kw) -> dict:
    """Parameter dict with defaults filled in."""
    p = copy.deepcopy(DEFAULTS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    p["periodic"] = tuple(int(x) for x in p["periodic"])
    p["g"] = tuple(float(x) for x in p["g"])
    p["scalar_bc"] = tuple(p["scalar_bc"])
    p["c_wall"] = tuple((float(a), float(b)) for a, b in p["c_wall"])
    return p


def shape_of(p: dict) -> tuple:
    return (p["ny"], p["nx"]) if p["lattice"] == "d2q9" else (p["nz"], p["ny"], p["nx"])


def dim_of(p: dict) -> int:
    return 2 if p["lattice"] == "d2q9" else 3


def n_nodes(p: dict) -> int:
    return int(p["nx"]) * int(p["ny"]) * int(p["nz"])


# ----------------------------------------------------------------- geometry

def coordinates(p: dict):
    """Integer node coordinates (x, y[, z]) as float arrays of the field shape."""
    if dim_of(p) == 2:
        y, x = np.meshgrid(np.arange(p["ny"], dtype=np.float64),
                           np.arange(p["nx"], dtype=np.float64), indexing="ij")
        return x, y
    z, y, x = np.meshgrid(np.arange(p["nz"], dtype=np.float64),
                          np.arange(p["ny"], dtype=np.float64),
                          np.arange(p["nx"], dtype=np.float64), indexing="ij")
    return x, y, z


def sdf_sphere(p: dict, centre, radius: float, inside_positive: bool = True) -> np.ndarray:
    """Signed distance to a circle (2-D) or sphere (3-D) of nodes at integer
    coordinates: positive inside when ``inside_positive`` (the sphere is
    fluid 1), negative inside otherwise (the sphere is fluid 2)."""
    xs = coordinates(p)
    r2 = sum((xi - ci) ** 2 for xi, ci in zip(xs, centre))
    d = radius - np.sqrt(r2)
    return d if inside_positive else -d


def sdf_plane(p: dict, axis: int, offset: float, positive_below: bool = True) -> np.ndarray:
    """Signed distance to the plane coordinate[axis] = offset."""
    x = coordinates(p)[axis]
    d = offset - x
    return d if positive_below else -d


def sdf_slab(p: dict, axis: int, lo: float, hi: float) -> np.ndarray:
    """Signed distance of a slab lo < coordinate[axis] < hi (positive inside)."""
    x = coordinates(p)[axis]
    return np.minimum(x - lo, hi - x)


# ---------------------------------------------------------- named workloads

def static_drop_64():
    """2-D static drop: 64 x 64 periodic, R = 16, W = 4, density ratio 1,
    Keq = 0.5, D1/D2 = 10, solute 1 inside the drop and 0 outside, FP64,
    2000 steps.  The drop is fluid 1."""
    p = params(nx=64, ny=64, nz=1, lattice="d2q9", visc_law="linear", periodic=(1, 1, 1),
               rho1=1.0, rho2=1.0, mu1=0.1, mu2=0.1, sigma=0.01, W=4.0, M=0.01,
               D1=0.1, D2=0.01, Keq=0.5, A=0.1, g=(0, 0, 0), rho_ref=0.0, precision="f64",
               ref_f=0.0, ref_h1=0.0, ref_h2=0.0)
    l = sdf_sphere(p, (32.0, 32.0), 16.0, inside_positive=True)
    return dict(name="static_drop_64x64_f64", params=p, sdf=l,
                init=dict(c1=(0.0, 1.0), c2=(0.0, 0.0)), steps=2000)


def rising_bubble_2d(nx=256, ny=1024, precision="f32", scalar_model="two", Keq=None,
                     scalar_grad="central"):
    """2-D rising bubble with interfacial mass transfer: nx x ny, periodic in x,
    half-way bounce-back walls at the y faces, gravity along -y, bubble
    (fluid 2) of radius nx/16 centred at (nx/2, 3nx/8); density ratio 10,
    exponential viscosity law mu = exp(c1 ln mu1 + c2 ln mu2), Eo = 10,
    Keq = 0.2, D2/D1 = 100; c1 = 0, c2 = 1 - phi0 (all solute starts in the
    bubble).  With mu2 = 0.1 the viscosity is exp(0) = 1 in the solute-free
    liquid and mu2 = 0.1 in the bubble at t = 0, a ratio of 10 (tau_g = 0.8
    in both phases); mu1 = 2 takes over where solute enters the liquid.

    scalar_model="one" runs the one-scalar model; its default Keq is 2
    (the model needs K_eff >= 5/9 in the liquid, see the one-scalar notes
    of the C header)."""
    R = nx / 16.0
    rho1, rho2, sigma, Eo = 10.0, 1.0, 0.01, 10.0
    gmag = Eo * sigma / ((rho1 - rho2) * (2 * R) ** 2)
    p = params(nx=nx, ny=ny, nz=1, lattice="d2q9", visc_law="exp", periodic=(1, 0, 1),
               rho1=rho1, rho2=rho2, mu1=2.0, mu2=0.1, sigma=sigma, W=4.0, M=0.01,
               D1=1e-3, D2=0.1, A=0.1, g=(0.0, -gmag, 0.0), rho_ref=rho1,
               Keq=Keq if Keq is not None else (2.0 if scalar_model == "one" else 0.2),
               precision=precision, ref_f=phase_reference(precision), ref_h1=0.0, ref_h2=0.0,
               scalar_model=scalar_model, scalar_grad=scalar_grad)
    l = sdf_sphere(p, (nx / 2.0, 3.0 * nx / 8.0), R, inside_positive=False)
    tag = ("_one" if scalar_model == "one" else "") + ("_local" if scalar_grad == "local" else "")
    return dict(name=f"rising_bubble{tag}_{nx}x{ny}_{precision}", params=p, sdf=l,
                init=dict(c1=(0.0, 0.0), c2=(1.0, -1.0)), steps=20000)


def rising_droplet_3d(n=256, precision="f32", scalar_grad="central"):
    """3-D rising droplet with heat transfer: n^3, periodic in x and y, walls at
    the z faces, gravity along -z; droplet (fluid 2) of radius 24 n/256 at
    (n/2, n/2, 3R); density ratio 10, exponential viscosity law with the
    bases of the 2-D bubble (viscosity ratio 10 at t = 0), Eo = 10;
    heat: Keq = rho1 Cp1/(rho2 Cp2) = 10 (equal Cp), conductivity ratio 50
    so D1/D2 = 5; q1 = 0, q2 = 1 - phi0 (hot droplet)."""
    R = 24.0 * n / 256.0
    rho1, rho2, sigma, Eo = 10.0, 1.0, 0.01, 10.0
    gmag = Eo * sigma / ((rho1 - rho2) * (2 * R) ** 2)
    p = params(nx=n, ny=n, nz=n, lattice="d3q19_d3q7", visc_law="exp", periodic=(1, 1, 0),
               rho1=rho1, rho2=rho2, mu1=2.0, mu2=0.1, sigma=sigma, W=4.0, M=0.01,
               D1=0.05, D2=0.01, Keq=10.0, A=0.1, g=(0.0, 0.0, -gmag), rho_ref=rho1,
               precision=precision, ref_f=phase_reference(precision), ref_h1=0.0, ref_h2=0.0,
               scalar_grad=scalar_grad)
    l = sdf_sphere(p, (n / 2.0, n / 2.0, 3.0 * R), R, inside_positive=False)
    tag = "_local" if scalar_grad == "local" else ""
    return dict(name=f"rising_droplet{tag}_{n}c_{precision}", params=p, sdf=l,
                init=dict(c1=(0.0, 0.0), c2=(1.0, -1.0)), steps=5000)


# ------------------------------------------------------------ random fields

def batched_sweep(ncases=512, seed=0, precision="f32", side=(64, 256), velocity=0.01):
    """Independent 2-D interfacial-transfer cases for one batched run: each
    side drawn uniformly from ``side`` (inclusive), Keq log-uniform in
    [0.1, 10], diffusivity ratio D_hi/D_lo log-uniform in [1, 1000], Peclet
    number log-uniform in [10, 1000], half static drops (periodic, matched
    density and viscosity), half rising bubbles (walls in y, density ratio 10,
    exponential viscosity law, Eo = 10).  The drop (fluid 2, radius
    min(nx, ny)/8) carries the solute: c1 = 0, c2 = 1 - phi0.

    The Peclet number fixes the fast diffusivity through a velocity scale,
    D_hi = U 2R / Pe with U = ``velocity``, and D_lo = D_hi / ratio.  The
    diffusivity ratio is always kept as drawn: where D_lo would fall below
    the smallest diffusivity the scalar lattice resolves (tau = 1/2 + 1e-3)
    or D_hi above tau = 2, both move together by one factor, which changes
    Pe only; each such case is listed in ``shifted`` (case, Pe asked,
    Pe used).

    Returns dict(name, cases=[dict(params, sdf, init)], shifted, nodes)."""
    rng = np.random.default_rng(seed)
    cs2 = 1.0 / 3.0
    d_lo_lim, d_hi_lim = cs2 * 1e-3, cs2 * 1.5
    cases, shifted = [], []

    def loguni(a, b):
        return float(np.exp(rng.uniform(np.log(a), np.log(b))))

    for k in range(ncases):
        nx = int(rng.integers(side[0], side[1] + 1))
        ny = int(rng.integers(side[0], side[1] + 1))
        keq = loguni(0.1, 10.0)
        ratio = loguni(1.0, 1000.0)
        pe = loguni(10.0, 1000.0)
        rising = bool(rng.integers(0, 2))
        R = min(nx, ny) / 8.0
        d_hi = velocity * 2.0 * R / pe
        d_lo = d_hi / ratio
        shift = max(d_lo_lim / d_lo, 1.0) * min(d_hi_lim / d_hi, 1.0)
        if shift != 1.0:
            d_lo, d_hi = d_lo * shift, d_hi * shift
            shifted.append((k, pe, velocity * 2.0 * R / d_hi))
        common = dict(nx=nx, ny=ny, nz=1, lattice="d2q9", sigma=0.01, W=4.0, M=0.01, A=0.1,
                      Keq=keq, D1=d_lo, D2=d_hi, precision=precision,
                      ref_f=phase_reference(precision), ref_h1=0.0, ref_h2=0.0)
        if rising:
            rho1, rho2, sigma, eo = 10.0, 1.0, 0.01, 10.0
            gmag = eo * sigma / ((rho1 - rho2) * (2 * R) ** 2)
            p = params(**common, visc_law="exp", periodic=(1, 0, 1), rho1=rho1, rho2=rho2,
                       mu1=2.0, mu2=0.1, g=(0.0, -gmag, 0.0), rho_ref=rho1)
            centre = (nx / 2.0, 3.0 * R)
        else:
            p = params(**common, visc_law="linear", periodic=(1, 1, 1), rho1=1.0, rho2=1.0,
                       mu1=0.1, mu2=0.1)
            centre = (nx / 2.0, ny / 2.0)
        l = sdf_sphere(p, centre, R, inside_positive=False)
        cases.append(dict(name=f"case{k}_{nx}x{ny}_{'rising' if rising else 'static'}",
                          params=p, sdf=l, init=dict(c1=(0.0, 0.0), c2=(1.0, -1.0))))
    nodes = sum(c["params"]["nx"] * c["params"]["ny"] for c in cases)
    return dict(name=f"batched_sweep_{ncases}_{precision}", cases=cases, shifted=shifted,
                nodes=nodes, steps=5000)


def random_fields(p: dict, seed: int, u_amp: float = 0.02, p_amp: float = 1e-3):
    """Seeded smooth-ish random macroscopic fields for arithmetic checks:
    phi in (0.05, 0.95), c1, c2 in (0.1, 1.1), |u| <= u_amp, |p| <= p_amp."""
    rng = np.random.default_rng(seed)
    shp = shape_of(p)
    d = dim_of(p)
    phi = 0.05 + 0.9 * rng.random(shp)
    c1 = 0.1 + rng.random(shp)
    c2 = 0.1 + rng.random(shp)
    u = u_amp * (2.0 * rng.random((d,) + shp) - 1.0)
    pr = p_amp * (2.0 * rng.random(shp) - 1.0)
    return dict(phi=phi, c1=c1, c2=c2, u=u, p=pr)
