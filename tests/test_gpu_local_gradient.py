"""GPU parity of the local gradient scheme for grad(c1 + Keq c2) (Eq. (39))
against the oracle, through the C-ABI: FP64 to round-off on random fields
with every wall layout, FP32 over 1000 steps of the rising bubble, and
every tile variant bit for bit."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "c1", "c2", "ux", "uy", "p", "mu", "psi")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cplb():
    import torch

    from paper_2402_15752_amd import cplb as C
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    C.library()
    return C


def rel_err(a, b):
    scale = max(np.linalg.norm(b), np.linalg.norm(b - b.mean()), 1e-300)
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / scale)


def compare(g, o, names, tol, label):
    errs = {k: rel_err(g.field(k).cpu().numpy(), o.field(k)) for k in names}
    say(f"  {label}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (label, bad)


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 1, 1), (1, 0, 1), (0, 0, 1)])
@pytest.mark.parametrize("shape", [(67, 37), (5, 3), (130, 9)])
def test_local_gradient_fp64_random_fields(cplb, shape, periodic):
    nx, ny = shape
    say(f"local gradient fp64 random {shape} periodic={periodic}")
    p = W.params(nx=nx, ny=ny, periodic=periodic, precision="f64", sigma=2e-3, rho1=3.0,
                 rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07, D2=0.02, Keq=0.6, A=0.4,
                 g=(2e-5, -3e-5, 0.0), rho_ref=1.5, scalar_grad="local")
    f = W.random_fields(p, seed=nx * 3 + ny)
    g = cplb.Lattice(p)
    o = ref.Oracle(p)
    for x in (g, o):
        x.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    g.step(3)
    o.step(3)
    compare(g, o, FIELDS, 1e-12, "t=3")


def test_local_gradient_rising_bubble_fp32(cplb):
    w = W.rising_bubble_2d(nx=64, ny=256, scalar_grad="local")
    say("local gradient rising bubble 64x256 fp32, 1000 steps")
    g = cplb.Lattice(w["params"])
    o = ref.Oracle(dict(w["params"], precision="f64"))
    for s in (g, o):
        s.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    r0 = g.reduce()
    g.step(1000)
    o.step(1000)
    compare(g, o, ("phi", "c1", "c2", "ux", "uy", "p"), 1e-5, "t=1000")
    r = g.reduce()
    assert abs(r["sum_c"] - r0["sum_c"]) <= 1e-6 * r0["sum_c"]


def test_local_gradient_variants_bitwise(cplb):
    p = W.params(nx=67, ny=37, periodic=(0, 1, 1), precision="f32", ref_f=0.5, sigma=2e-3,
                 D1=0.07, D2=0.02, Keq=0.6, A=0.4, scalar_grad="local")
    f = W.random_fields(p, seed=23)
    g = cplb.Lattice(p)
    out = []
    for v in range(len(g.variant_names())):
        g.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
        g.variant = v
        g.step(5)
        out.append({k: g.field(k).cpu().numpy() for k in ("phi", "c1", "c2", "ux", "p")})
    for v in range(1, len(out)):
        for k in out[0]:
            assert np.array_equal(out[0][k], out[v][k]), (v, k)


@pytest.mark.parametrize("periodic", [(1, 1, 1), (1, 1, 0), (0, 1, 0), (0, 0, 0)])
def test_local_gradient_fp64_random_fields_3d(cplb, periodic):
    say(f"local gradient fp64 3d random periodic={periodic}")
    p = W.params(nx=35, ny=13, nz=70, lattice="d3q19_d3q7", periodic=periodic, precision="f64",
                 sigma=2e-3, rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07,
                 D2=0.02, Keq=0.6, A=0.4, g=(1e-5, -2e-5, 3e-5), rho_ref=1.5, scalar_grad="local")
    f = W.random_fields(p, seed=5)
    g = cplb.Lattice(p)
    o = ref.Oracle(p)
    for x in (g, o):
        x.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    g.step(3)
    o.step(3)
    compare(g, o, FIELDS + ("uz",), 1e-12, "t=3")


@pytest.mark.parametrize("precision,tol", [("f32", 1e-5), ("f32_s16f", 2e-3)])
def test_local_gradient_droplet3d(cplb, precision, tol):
    w = W.rising_droplet_3d(n=64, precision=precision, scalar_grad="local")
    say(f"local gradient rising droplet 64^3 {precision}, 200 steps")
    g = cplb.Lattice(w["params"])
    o = ref.Oracle(dict(w["params"], precision="f64"))
    for s in (g, o):
        s.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    g.step(200)
    o.step(200)
    names = ("phi", "c1", "c2", "ux", "uy", "uz", "p") if precision == "f32" else ("phi", "c1", "c2")
    compare(g, o, names, tol, f"{precision} t=200")


def test_local_gradient_variants_bitwise_3d(cplb):
    p = W.params(nx=35, ny=13, nz=30, lattice="d3q19_d3q7", periodic=(1, 0, 0), precision="f32",
                 ref_f=0.5, sigma=2e-3, D1=0.07, D2=0.02, Keq=0.6, A=0.4, scalar_grad="local")
    f = W.random_fields(p, seed=29)
    g = cplb.Lattice(p)
    out = []
    for v in range(len(g.variant_names())):
        g.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
        g.variant = v
        g.step(4)
        out.append({k: g.field(k).cpu().numpy() for k in ("phi", "c1", "c2", "uz", "p")})
    for v in range(1, len(out)):
        for k in out[0]:
            assert np.array_equal(out[0][k], out[v][k]), (v, k)
