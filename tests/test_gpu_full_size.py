"""GPU parity at the full sizes the benchmark times, in its launch
configuration (the library's default variant for each lattice), against the
FP64 oracle on the same seeded inputs.

The benchmark's headline lattice (rising bubble 256 x 1024) and the 3-D FP32
droplet at 256^3 are covered in test_gpu_parity.py.  Here: the 3-D droplet
with FP16 storage and with the local gradient scheme (Eq. (39)), the 2-D
lattice at 2048 x 4096 -- beyond the 256 MB Infinity Cache, where the step
takes the variant with non-temporal stores -- and the one-scalar model
(Sec. III D) at 256 x 1024.  A few steps each: the oracle takes ~0.3 s per
step for 8 M nodes and ~0.6 s for 16.7 M nodes on 16 cores.

Tolerances are those of the reduced-size tests: 1e-5 relative L2 for FP32
storage, 2e-3 on phi, c1, c2 for FP16 storage.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def cplb():
    import torch

    from paper_2402_15752_amd import cplb as C
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    C.library()
    return C


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.linalg.norm(b), np.linalg.norm(b - b.mean()), 1e-300)
    return float(np.linalg.norm(a - b) / scale)


def run_pair(cplb, w, steps, names, tol, label):
    g = cplb.Lattice(w["params"])  # the library's default variant, as benchmarked
    o = ref.Oracle(dict(w["params"], precision="f64"))
    for s in (g, o):
        s.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    g.step(steps)
    o.step(steps)
    errs = {}
    for k in names:
        a = g.field(k).cpu().numpy()
        b = o.field(k)
        assert a.shape == b.shape
        assert np.all(np.isfinite(a)), (label, k)
        errs[k] = rel_err(a, b)
    say(f"  {label}: variant {g.variant_names()[g.variant]}: "
        + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (label, bad, tol)


FP32_2D = ("phi", "c1", "c2", "ux", "uy", "p")
FP32_3D = FP32_2D + ("uz",)
S16 = ("phi", "c1", "c2")


def test_droplet3d_fp16_storage_full_size(cplb):
    w = W.rising_droplet_3d(n=256, precision="f32_s16f")
    say("rising droplet 256^3 f32_s16f, 4 steps")
    run_pair(cplb, w, 4, S16, 2e-3, "t=4")


@pytest.mark.parametrize("precision,names,tol", [("f32", FP32_3D, 1e-5), ("f32_s16f", S16, 2e-3)])
def test_droplet3d_local_gradient_full_size(cplb, precision, names, tol):
    w = W.rising_droplet_3d(n=256, precision=precision, scalar_grad="local")
    say(f"rising droplet 256^3 {precision}, local gradient, 4 steps")
    run_pair(cplb, w, 4, names, tol, "t=4")


@pytest.mark.parametrize("grad", ["central", "local"])
def test_hbm_size_2d_random_fields(cplb, grad):
    """The 2048 x 4096 lattice with the rising bubble's parameters and walls,
    from seeded random O(1) fields.  The bubble itself is ill-conditioned for
    a relative norm at the few steps the oracle affords at this size: c1
    starts at zero and u at rest, so after 20 steps both are tiny fields
    (max |u_x| 2e-5) whose absolute FP32 error (4e-8 in c1, 3e-9 in u_x) is
    the same as on the 256 x 1024 lattice but 3e-5 of their norm."""
    w = W.rising_bubble_2d(nx=2048, ny=4096, scalar_grad=grad)
    p = w["params"]
    f = W.random_fields(p, seed=17)
    say(f"2048x4096 f32 random fields, {grad} gradient, 5 steps")
    g = cplb.Lattice(p)  # the library's default variant, as benchmarked
    o = ref.Oracle(dict(p, precision="f64"))
    for s in (g, o):
        s.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    g.step(5)
    o.step(5)
    errs = {}
    for k in FP32_2D + ("psi",):
        a = g.field(k).cpu().numpy()
        assert np.all(np.isfinite(a)), k
        errs[k] = rel_err(a, o.field(k))
    # mu = exp(c1 ln mu1 + c2 ln mu2) (Eq. (4.3)) is held to the field bound
    # against the oracle (1.4e-7 central, 6.2e-7 local, measured) and, node
    # by node, against FP64 exp of the GPU's own c1, c2: the FP32 exponential
    # (v_exp_f32 of x log2 e) is good to a few 1e-7.
    c1, c2, mu = (g.field(k).cpu().numpy().astype(np.float64) for k in ("c1", "c2", "mu"))
    mu_exact = np.exp(c1 * np.log(p["mu1"]) + c2 * np.log(p["mu2"]))
    errs["mu_eval_max"] = float(np.max(np.abs(mu / mu_exact - 1.0)))
    errs["mu_vs_oracle"] = rel_err(mu, o.field("mu"))
    say(f"  t=5: variant {g.variant_names()[g.variant]}: "
        + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bounds = dict({k: 1e-5 for k in FP32_2D + ("psi",)}, mu_eval_max=1e-6, mu_vs_oracle=1e-5)
    bad = {k: v for k, v in errs.items() if not v <= bounds[k]}
    assert not bad, bad


def test_one_scalar_bubble_full_size(cplb):
    w = W.rising_bubble_2d(scalar_model="one")
    say("one-scalar rising bubble 256x1024 f32, 200 steps")
    run_pair(cplb, w, 200, FP32_2D, 1e-5, "t=200")


# ------------------------- lattices beyond 4 GiB (per-set and 64-bit offsets)

def _random_field_pair(cplb, p, steps, names, tol, label):
    f = W.random_fields(p, seed=23)
    g = cplb.Lattice(p)
    o = ref.Oracle(dict(p, precision="f64"))
    for s in (g, o):
        s.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    del f
    g.step(steps)
    o.step(steps)
    errs = {}
    for k in names:
        a = g.field(k).cpu().numpy()
        assert np.all(np.isfinite(a)), k
        errs[k] = rel_err(a, o.field(k))
        del a
    say(f"  {label}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    g.close()
    del g, o
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, (label, bad, tol)


def test_64bit_offsets_3d_fp32(cplb):
    """384^3 FP32: the 19 planes of g span more than 4 GiB, so the step takes
    its 64-bit-offset instantiation (smaller cases take 32-bit offsets).
    Random fields, walls on x and z, 2 steps, every field."""
    n = 384
    assert 19 * n ** 3 * 4 > 1 << 32
    p = W.params(nx=n, ny=n, nz=n, lattice="d3q19_d3q7", periodic=(0, 1, 0), precision="f32",
                 sigma=2e-3, rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07,
                 D2=0.02, Keq=0.6, A=0.4, g=(1e-5, -2e-5, 3e-5), rho_ref=1.5,
                 ref_f=W.phase_reference("f32"))
    say("384^3 f32 random fields (64-bit offsets), 2 steps")
    _random_field_pair(cplb, p, 2, FP32_3D + ("psi",), 1e-5, "t=2")


def test_per_set_offsets_3d_fp64(cplb):
    """256^3 FP64: the 40 population planes span more than 4 GiB but each set
    less, so the 3-D step takes 32-bit offsets from a base per set instead
    of buffer accesses over the whole lattice.  Random fields, walls on y,
    2 steps, every field to FP64 round-off."""
    n = 256
    assert 40 * n ** 3 * 8 > 1 << 32 and 19 * (n ** 3 + 4096) * 8 < 1 << 32
    p = W.params(nx=n, ny=n, nz=n, lattice="d3q19_d3q7", periodic=(1, 0, 1), precision="f64",
                 sigma=2e-3, rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07,
                 D2=0.02, Keq=0.6, A=0.4, g=(1e-5, -2e-5, 3e-5), rho_ref=1.5)
    say("256^3 f64 random fields (32-bit offsets per set), 2 steps")
    _random_field_pair(cplb, p, 2, FP32_3D + ("mu", "psi"), 1e-12, "t=2")


def test_64bit_offsets_2d_fp64(cplb):
    """8000 x 8000 FP64: each 9-plane set spans more than 4 GiB, so the 2-D
    step takes its 64-bit-offset instantiation.  Random fields, walls on y,
    3 steps, every field to FP64 round-off."""
    n = 8000
    assert 9 * n * n * 8 > 1 << 32
    p = W.params(nx=n, ny=n, periodic=(1, 0, 1), precision="f64", sigma=2e-3, rho1=3.0,
                 rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07, D2=0.02, Keq=0.6, A=0.4,
                 g=(2e-5, -3e-5, 0.0), rho_ref=1.5)
    say("8000x8000 f64 random fields (64-bit offsets), 3 steps")
    _random_field_pair(cplb, p, 3, FP32_2D + ("mu", "psi"), 1e-12, "t=3")
