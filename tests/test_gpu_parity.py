"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle,
element by element on the same seeded inputs.

Tolerances (relative L2 per field, p normalised by its variation):
  FP64 GPU vs FP64 oracle : 1e-12 after a few steps on random fields,
                            1e-10 after 2000 steps of the static drop.
                            Both sides round differently (FMA contraction,
                            summation order: ~1e-16 per operation) and the
                            trajectory is well conditioned (a 1-ulp
                            perturbation stays ~1e-15 over 500 steps).
  FP32 compute + storage  : 1e-5 after 1000 steps (stated target).
  16-bit storage          : FP16 2e-3 (stated target) on phi, c1, c2.  BF16
                            keeps 8 significant bits: an O(1) interface
                            population loses ~2e-3 per step, so the run
                            settles near 1e-2; it is held to 2e-2 and does
                            not meet the 2e-3 target.
  phase-mass drift        : 1e-12 over 2000 FP64 steps (round-off accumulates:
                            the oracle itself drifts 2e-13 on that run),
                            1e-6 (FP32).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu


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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.linalg.norm(b), np.linalg.norm(b - b.mean()), 1e-300)
    return float(np.linalg.norm(a - b) / scale)


def max_err(a, b):
    """Largest nodal error over the field's scale (its largest magnitude or
    its largest deviation from the mean, whichever is larger)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = max(np.abs(b).max(), np.abs(b - b.mean()).max(), 1e-300)
    return float(np.abs(a - b).max() / scale)


def compare(g, o, names, tol, label=""):
    """Relative L2 error of each field within tol and, so that an error held
    to a few nodes (a wall row, the interface) cannot hide under the norm,
    its max-abs error within 30 tol (10 tol for the 16-bit bounds, 100 tol
    for the FP64 ones)."""
    errs, maxs = {}, {}
    for k in names:
        a = g.field(k).cpu().numpy()
        b = o.field(k)
        assert a.shape == b.shape
        assert np.all(np.isfinite(a)), (label, k)
        errs[k] = rel_err(a, b)
        maxs[k] = max_err(a, b)
    mtol = (10.0 if tol >= 1e-3 else 30.0 if tol >= 1e-7 else 100.0) * tol
    say(f"  {label}: " + " ".join(f"{k}={v:.2e}/{maxs[k]:.2e}" for k, v in errs.items()))
    bad = {k: (v, maxs[k]) for k, v in errs.items() if not (v <= tol and maxs[k] <= mtol)}
    assert not bad, (label, bad, tol, mtol)
    return errs


def pair_fields(cplb, p, f, steps):
    g = cplb.Lattice(p)
    g.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    o = ref.Oracle(p)
    o.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    g.step(steps)
    o.step(steps)
    return g, o


def pair_workload(cplb, w, steps, precision=None):
    p = dict(w["params"])
    if precision:
        p["precision"] = precision
        p["ref_f"] = W.phase_reference(precision)
    g = cplb.Lattice(p)
    g.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    o = ref.Oracle(p)
    o.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    g.step(steps)
    o.step(steps)
    return g, o


ALL2 = ("phi", "c1", "c2", "ux", "uy", "p", "mu", "psi")
ALL3 = ALL2 + ("uz",)


# ------------------------------------------------------- FP64 arithmetic

@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 1, 1), (1, 0, 1), (0, 0, 1)])
@pytest.mark.parametrize("shape", [(67, 37), (5, 3), (130, 9)])
def test_fp64_random_fields_2d(cplb, periodic, shape):
    """Random non-equilibrium fields, ragged tiles, every wall layout: all
    terms of the step are exercised; FP64 must agree to round-off."""
    nx, ny = shape
    say(f"fp64 2d random {shape} periodic={periodic}")
    p = W.params(nx=nx, ny=ny, periodic=periodic, precision="f64", sigma=2e-3, rho1=3.0,
                 rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07, D2=0.02, Keq=0.6, A=0.4,
                 g=(2e-5, -3e-5, 0.0), rho_ref=1.5)
    f = W.random_fields(p, seed=nx * 7 + ny)
    g, o = pair_fields(cplb, p, f, 0)
    compare(g, o, ALL2, 1e-13, "t=0")
    g.step(3)
    o.step(3)
    compare(g, o, ALL2, 1e-12, "t=3")


@pytest.mark.parametrize("periodic", [(1, 1, 1), (1, 1, 0), (0, 1, 0), (0, 0, 0)])
def test_fp64_random_fields_3d(cplb, periodic):
    say(f"fp64 3d random periodic={periodic}")
    p = W.params(nx=35, ny=13, nz=70, lattice="d3q19_d3q7", periodic=periodic, precision="f64",
                  sigma=2e-3, rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07,
                  D2=0.02, Keq=0.6, A=0.4, g=(1e-5, -2e-5, 3e-5), rho_ref=1.5)
    f = W.random_fields(p, seed=3)
    g, o = pair_fields(cplb, p, f, 0)
    compare(g, o, ALL3, 1e-13, "t=0")
    g.step(3)
    o.step(3)
    compare(g, o, ALL3, 1e-12, "t=3")


@pytest.mark.parametrize("kw", [
    dict(nx=1, ny=24, periodic=(1, 0, 1)),
    dict(nx=19, ny=1, periodic=(0, 1, 1)),
    dict(nx=1, ny=6, nz=20, lattice="d3q19_d3q7", periodic=(1, 1, 0)),
], ids=["2d-nx1", "2d-ny1", "3d-nx1"])
def test_fp64_one_node_wide_periodic_axis(cplb, kw):
    """Degenerate lattices: a periodic axis one node wide, so every stencil
    neighbour and push target along it is the node itself (the gradient
    along it vanishes).  FP64 random fields, 3 steps."""
    say(f"fp64 one node wide {kw}")
    p = W.params(precision="f64", sigma=2e-3, rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.3,
                 mu2=0.08, D1=0.07, D2=0.02, Keq=0.6, A=0.4, rho_ref=1.5,
                 g=(1e-5, -2e-5, 3e-5 if "nz" in kw else 0.0), **kw)
    f = W.random_fields(p, seed=31)
    g, o = pair_fields(cplb, p, f, 3)
    compare(g, o, ALL3 if "nz" in kw else ALL2, 1e-12, "t=3")


def test_static_drop_fp64_full_run(cplb):
    """Static drop, 64 x 64 periodic, FP64, 2000 steps."""
    w = W.static_drop_64()
    say("static drop 64x64 fp64 2000 steps")
    g, o = pair_workload(cplb, w, 0)
    r0 = g.reduce()
    for s in (1, 10, 100, 1000, 889):
        g.step(s)
        o.step(s)
        compare(g, o, ("phi", "c1", "c2", "ux", "uy", "p"), 1e-10, f"t={g.step_count}")
    assert g.step_count == 2000
    r1, ro = g.reduce(), o.reduce()
    assert r1["rc"] == 0 and r1["step"] == 2000
    assert abs(r1["sum_phi"] - r0["sum_phi"]) <= 1e-12 * r0["sum_phi"]
    assert abs(r1["sum_c"] - r0["sum_c"]) <= 1e-12 * r0["sum_c"]
    for k in ("sum_phi", "sum_c1", "sum_c2", "sum_c"):
        assert abs(r1[k] - ro[k]) <= 1e-12 * abs(ro[k]), k
    assert abs(r1["max_u"] - ro["max_u"]) <= 1e-8 * ro["max_u"]
    assert abs(r1["kinetic"] - ro["kinetic"]) <= 1e-8 * ro["kinetic"]


# ------------------------------------------------------------------ FP32

def test_rising_bubble_fp32_reduced(cplb):
    w = W.rising_bubble_2d(nx=64, ny=256)
    say("rising bubble 64x256 fp32 1000 steps")
    g, o = pair_workload(cplb, w, 1000)
    compare(g, o, ("phi", "c1", "c2", "ux", "uy", "p"), 1e-5, "t=1000")
    r = g.reduce()
    g2 = cplb.Lattice(w["params"])
    g2.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    r0 = g2.reduce()
    assert abs(r["sum_phi"] - r0["sum_phi"]) <= 1e-6 * r0["sum_phi"]


def test_rising_bubble_fp32_full_size(cplb):
    """The benchmarked workload at its full size, 256 x 1024, 1000 steps."""
    w = W.rising_bubble_2d()
    say("rising bubble 256x1024 fp32 1000 steps (oracle takes ~1 min)")
    g, o = pair_workload(cplb, w, 1000)
    compare(g, o, ("phi", "c1", "c2", "ux", "uy", "p"), 1e-5, "t=1000")


def test_droplet3d_fp32_reduced(cplb):
    w = W.rising_droplet_3d(n=64)
    say("rising droplet 64^3 fp32 200 steps")
    g, o = pair_workload(cplb, w, 200)
    compare(g, o, ("phi", "c1", "c2", "ux", "uy", "uz", "p"), 1e-5, "t=200")


def test_droplet3d_fp32_1000_steps(cplb):
    """The FP32 target is 1e-5 after 1000 steps: the 3-D droplet on a 64^3
    copy for that long (the oracle takes ~10 s on 16 cores).  Measured on
    MI355X: u 9.6e-6, p 7.6e-6, c2 3.9e-6, c1 1.1e-6, phi 1.5e-7."""
    w = W.rising_droplet_3d(n=64)
    say("rising droplet 64^3 fp32 1000 steps")
    g, o = pair_workload(cplb, w, 1000)
    compare(g, o, ("phi", "c1", "c2", "ux", "uy", "uz", "p"), 1e-5, "t=1000")


def test_droplet3d_fp32_full_size(cplb):
    """256^3 in the benchmarked launch configuration, a few steps (the oracle
    takes seconds per step at this size)."""
    w = W.rising_droplet_3d(n=256)
    say("rising droplet 256^3 fp32 4 steps")
    g, o = pair_workload(cplb, w, 4)
    compare(g, o, ("phi", "c1", "c2", "ux", "uy", "uz", "p"), 1e-5, "t=4")


# ------------------------------------------------------- 16-bit storage

TOL16 = 2e-3
# with BF16 storage p and u miss the target (see the 128^3 1000-step parity);
# both 16-bit formats hold phi, c1 and c2 to it
FIELDS16 = {"f32_s16f": ("phi", "c1", "c2", "ux", "uy", "uz", "p"), "f32_s16b": ("phi", "c1", "c2")}


@pytest.mark.parametrize("precision", ["f32_s16f", "f32_s16b"])
def test_droplet3d_16bit_storage(cplb, precision):
    w = W.rising_droplet_3d(n=64)
    say(f"rising droplet 64^3 {precision} 200 steps")
    g, o = pair_workload(cplb, w, 200, precision=precision)
    compare(g, o, FIELDS16[precision], TOL16, f"{precision} t=200")


@pytest.mark.parametrize("precision", ["f32_s16f", "f32_s16b"])
def test_bubble2d_16bit_storage(cplb, precision):
    w = W.rising_bubble_2d(nx=64, ny=256)
    say(f"rising bubble 64x256 {precision} 1000 steps")
    g, o = pair_workload(cplb, w, 1000, precision=precision)
    compare(g, o, ("phi", "c1", "c2"), TOL16, f"{precision} t=1000")


# ------------------------------------------------ invariants and contract

def test_deterministic_and_resumable(cplb):
    w = W.rising_bubble_2d(nx=64, ny=128)
    say("determinism and checkpoint/resume")
    a = cplb.Lattice(w["params"])
    a.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    a.step(30)
    blob = a.save_state()
    a.step(41)
    b = cplb.Lattice(w["params"])
    b.load_state(blob)
    assert b.step_count == 30
    b.step(41)
    c = cplb.Lattice(w["params"])
    c.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    c.step(71)
    for k in ("phi", "c1", "c2", "ux", "uy", "p"):
        fa = a.field(k).cpu().numpy()
        assert np.array_equal(fa, b.field(k).cpu().numpy()), k
        assert np.array_equal(fa, c.field(k).cpu().numpy()), k


def test_checkpoint_rejects_other_parameters(cplb):
    w = W.rising_bubble_2d(nx=64, ny=128)
    a = cplb.Lattice(w["params"])
    a.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    blob = a.save_state()
    p = dict(w["params"])
    p["Keq"] = 0.3
    b = cplb.Lattice(p)
    with pytest.raises(cplb.CplbError) as e:
        b.load_state(blob)
    assert e.value.code == cplb.CPLB_ESTATE


def test_nonfinite_is_reported(cplb):
    p = W.params(nx=16, ny=16, precision="f32")
    phi = np.full(W.shape_of(p), 0.5)
    phi[3, 4] = np.nan
    g = cplb.Lattice(p)
    g.init_fields(phi, phi.copy(), phi.copy())
    r = g.reduce()
    assert r["rc"] == cplb.CPLB_EUNSTABLE and r["nonfinite"] >= 1


def test_fp32_field_readout_matches_fp64_readout(cplb):
    import torch
    w = W.rising_bubble_2d(nx=64, ny=128)
    g = cplb.Lattice(w["params"])
    g.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    g.step(5)
    a = g.field("phi", dtype=torch.float32).cpu().numpy()
    b = g.field("phi", dtype=torch.float64).cpu().numpy()
    assert np.array_equal(a.astype(np.float64), b)


# ------------------------------------------------------ kernel variants

VARIANT_CASES = [
    ("d2q9 f64", dict(nx=67, ny=37, periodic=(1, 0, 1), precision="f64")),
    ("d2q9 f32", dict(nx=130, ny=9, periodic=(0, 1, 1), precision="f32")),
    ("d2q9 s16f", dict(nx=67, ny=37, periodic=(1, 1, 1), precision="f32_s16f")),
    ("d2q9 one f32", dict(nx=67, ny=37, periodic=(0, 1, 1), precision="f32", scalar_model="one")),
    ("d3 f64", dict(nx=35, ny=13, nz=70, lattice="d3q19_d3q7", periodic=(1, 0, 0),
                    precision="f64")),
    ("d3 f32", dict(nx=35, ny=13, nz=70, lattice="d3q19_d3q7", periodic=(0, 1, 0),
                    precision="f32")),
    ("d3 s16b", dict(nx=35, ny=13, nz=70, lattice="d3q19_d3q7", periodic=(1, 1, 0),
                     precision="f32_s16b")),
]


@pytest.mark.parametrize("label,kw", VARIANT_CASES, ids=[c[0] for c in VARIANT_CASES])
def test_every_variant_is_bitwise_identical(cplb, label, kw):
    """Variants only retile the same per-node arithmetic, so every one of them
    must give the default variant's fields bit for bit (ragged tiles, walls)."""
    p = W.params(sigma=2e-3, rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07,
                 D2=0.02, Keq=0.6, A=0.4, rho_ref=1.5,
                 g=(1e-5, -2e-5, 3e-5 if "nz" in kw else 0.0), **kw)
    f = W.random_fields(p, seed=11)
    names = ALL3 if "nz" in kw else ALL2
    out = {}
    g = cplb.Lattice(p)
    nv = len(g.variant_names())
    assert nv >= 2
    for v in range(nv):
        g.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
        g.variant = v
        g.step(5)
        out[v] = {k: g.field(k).cpu().numpy() for k in names}
    say(f"  {label}: {nv} variants {g.variant_names()}")
    for v in range(1, nv):
        for k in names:
            assert np.array_equal(out[0][k], out[v][k]), (label, g.variant_names()[v], k)


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19_d3q7"])
def test_tune_leaves_the_state_unchanged(cplb, lattice):
    """cplb_tune probes every variant on the idle lattice and restores the
    history: the run it interrupts continues bit for bit."""
    w = W.rising_bubble_2d(nx=64, ny=128) if lattice == "d2q9" else W.rising_droplet_3d(n=48)
    a = cplb.Lattice(w["params"])
    a.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    b = cplb.Lattice(w["params"])
    b.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    a.step(7)
    b.step(7)
    ms = a.tune(3)
    assert ms > 0 and 0 <= a.variant < len(a.variant_names())
    assert a.step_count == 7
    a.step(9)
    b.step(9)
    names = ALL3 if lattice != "d2q9" else ALL2
    for k in names:
        assert np.array_equal(a.field(k).cpu().numpy(), b.field(k).cpu().numpy()), k


def test_set_variant_rejects_unknown_id(cplb):
    g = cplb.Lattice(W.params(nx=16, ny=16, precision="f32"))
    with pytest.raises(cplb.CplbError) as e:
        g.variant = len(g.variant_names())
    assert e.value.code == cplb.CPLB_EINVAL


@pytest.mark.parametrize("lattice", ["d2q9", "d3q19_d3q7"])
def test_graph_replays_match_eager_steps(cplb, lattice):
    """Steps captured in a HIP graph and replayed several times, with field
    reads and reductions between the replays, equal eager steps bit for bit
    (the read-outs recompute from the current populations every time)."""
    import torch
    w = W.rising_bubble_2d(nx=64, ny=128) if lattice == "d2q9" else W.rising_droplet_3d(n=32)
    s = torch.cuda.Stream()
    a = cplb.Lattice(w["params"], stream=s)
    a.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    e = cplb.Lattice(w["params"])
    e.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    a.step(1)
    e.step(1)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.step(4)
    torch.cuda.synchronize()
    names = ALL3 if lattice != "d2q9" else ALL2
    for rep in range(3):
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        e.step(4)
        torch.cuda.synchronize()
        ra, re_ = a.reduce(), e.reduce()
        assert ra["sum_phi"] == re_["sum_phi"] and ra["max_u"] == re_["max_u"], rep
        for k in names:
            assert np.array_equal(a.field(k).cpu().numpy(), e.field(k).cpu().numpy()), (rep, k)


def test_entry_points_reject_bad_arguments(cplb):
    """Every entry point checks its arguments before touching the device and
    returns the documented code with a message (no launch happens)."""
    import ctypes

    import torch
    L = cplb.library()
    lat = cplb.Lattice(W.params(nx=16, ny=8, precision="f32"))
    h = lat.handle
    buf = torch.empty(lat.N, dtype=torch.float32, device="cuda")
    EINVAL, ENOMEM, ESTATE = cplb.CPLB_EINVAL, cplb.CPLB_ENOMEM, cplb.CPLB_ESTATE
    F32 = cplb.DTYPE_F32
    cases = [
        (L.cplb_step(h, -1), EINVAL),
        (L.cplb_read_field(h, 99, buf.data_ptr(), F32), EINVAL),
        (L.cplb_read_field(h, 0, buf.data_ptr(), 7), EINVAL),
        (L.cplb_read_field(h, 0, None, F32), EINVAL),
        (L.cplb_init_fields(h, None, None, None, None, None), EINVAL),
        (L.cplb_init_sdf(h, None, 0.0, 0.0, 0.0, 0.0), EINVAL),
        (L.cplb_set_variant(h, 99), EINVAL),
        (L.cplb_tune(h, 0, None), EINVAL),
    ]
    small = ctypes.create_string_buffer(16)
    cases += [(L.cplb_save_state(h, small, 16), ENOMEM), (L.cplb_load_state(h, small, 16), ESTATE)]
    for rc, want in cases:
        assert rc == want, (rc, want)
        assert L.cplb_last_error(h).decode(), rc
        assert L.cplb_strerror(rc).decode()
    # a null handle is refused without a message to write
    assert L.cplb_step(None, 1) == EINVAL
    assert L.cplb_reduce(None, None) == EINVAL
    # the lattice is unharmed: it still steps and reduces
    lat.init_sdf(np.zeros(lat.shape), c1=(0.5, 0.0), c2=(0.5, 0.0))
    lat.step(2)
    assert lat.reduce()["rc"] == 0
    # a closure applies to D2Q9 lattices only
    lat3 = cplb.Lattice(W.params(nx=8, ny=8, nz=8, lattice="d3q19_d3q7", precision="f32"))
    assert L.cplb_set_closure(lat3.handle, ctypes.c_void_p(buf.data_ptr())) == EINVAL
    lat.close()
    lat3.close()
