"""GPU tests of the batch (many independent D2Q9 lattices in one launch per
size class), through the C-ABI.

The batched kernel runs the single-lattice kernel's tile body on each case,
so every case must equal the same case run alone bit for bit; two small
FP64 cases are also compared with the oracle element by element.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu

FIELDS2 = ("phi", "c1", "c2", "ux", "uy", "p", "mu")


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


def mixed_cases(precision, seed=5):
    """Seven cases across the three size classes: ragged tiles, walls on
    either axis, different physics per case."""
    rng = np.random.default_rng(seed)
    shapes = [(40, 30, (1, 1, 1)), (67, 37, (0, 1, 1)), (130, 9, (1, 0, 1)),
              (100, 150, (1, 0, 1)), (64, 64, (1, 1, 1)), (97, 70, (0, 0, 1)),
              (200, 33, (1, 0, 1))]
    cases = []
    for nx, ny, per in shapes:
        p = W.params(nx=nx, ny=ny, periodic=per, precision=precision,
                     ref_f=W.phase_reference(precision),
                     sigma=float(rng.uniform(1e-3, 1e-2)), rho1=float(rng.uniform(1, 5)),
                     rho2=1.0, visc_law="exp", mu1=float(rng.uniform(0.1, 0.5)),
                     mu2=float(rng.uniform(0.05, 0.1)), D1=float(rng.uniform(0.01, 0.1)),
                     D2=float(rng.uniform(0.01, 0.1)), Keq=float(rng.uniform(0.2, 5)),
                     A=float(rng.uniform(0.05, 0.5)),
                     g=(0.0, float(rng.uniform(-3e-5, 0)), 0.0), rho_ref=1.0)
        R = min(nx, ny) / 4.0
        l = W.sdf_sphere(p, (nx / 2.0 + 0.3, ny / 2.0 - 0.2), R, inside_positive=False)
        cases.append(dict(params=p, sdf=l, init=dict(c1=(0.0, 0.0), c2=(1.0, -1.0))))
    return cases


def make_batch(cplb, cases, stream=None):
    b = cplb.Batch([c["params"] for c in cases], stream=stream)
    for k, c in enumerate(cases):
        b.init_sdf(k, c["sdf"], c1=c["init"]["c1"], c2=c["init"]["c2"])
    return b


def single(cplb, case, steps):
    g = cplb.Lattice(case["params"])
    g.init_sdf(case["sdf"], c1=case["init"]["c1"], c2=case["init"]["c2"])
    g.step(steps)
    return g


@pytest.mark.parametrize("precision", ["f64", "f32", "f32_s16f"])
def test_batch_cases_equal_single_lattices_bitwise(cplb, precision):
    cases = mixed_cases(precision)
    say(f"batch of {len(cases)} mixed cases, {precision}, 25 steps")
    b = make_batch(cplb, cases)
    assert [n for n, _ in b.classes()] == [2, 1, 2, 1, 1]
    b.step(25)
    assert b.step_count == 25
    for k, c in enumerate(cases):
        g = single(cplb, c, 25)
        for f in FIELDS2:
            a = b.field(k, f).cpu().numpy()
            s = g.field(f).cpu().numpy()
            assert np.all(np.isfinite(a)), (k, f)
            assert np.array_equal(a, s), (precision, k, f, float(np.abs(a - s).max()))
        r = b.reduce(k)
        assert r["rc"] == 0 and r["step"] == 25
        g.close()


def test_batch_fp64_matches_oracle(cplb):
    cases = mixed_cases("f64")[:3]
    say("batch fp64 vs oracle, 3 cases, 10 steps")
    b = make_batch(cplb, cases)
    b.step(10)
    for k, c in enumerate(cases):
        o = ref.Oracle(c["params"])
        o.init_sdf(c["sdf"], c1=c["init"]["c1"], c2=c["init"]["c2"])
        o.step(10)
        for f in ("phi", "c1", "c2", "ux", "uy", "p"):
            a = b.field(k, f).cpu().numpy()
            r = o.field(f)
            scale = max(np.linalg.norm(r), np.linalg.norm(r - r.mean()), 1e-300)
            err = np.linalg.norm(a - r) / scale
            assert err <= 1e-12, (k, f, err)


def test_batch_tune_leaves_state_unchanged(cplb):
    cases = mixed_cases("f32")
    a = make_batch(cplb, cases)
    c = make_batch(cplb, cases)
    a.step(6)
    c.step(6)
    ms = a.tune(2)
    assert ms > 0
    lat = cplb.Lattice(cases[0]["params"])
    nv = len(lat.variant_names())  # the 2-D variants, the same table for the batch
    lat.close()
    for cls, (n, v) in enumerate(a.classes()):
        assert 0 <= v < nv
    a.step(7)
    c.step(7)
    for k in range(len(cases)):
        for f in ("phi", "c1", "c2", "ux", "uy", "p"):
            assert np.array_equal(a.field(k, f).cpu().numpy(), c.field(k, f).cpu().numpy()), (k, f)
    with pytest.raises(cplb.CplbError) as e:
        a.set_variant(0, nv)
    assert e.value.code == cplb.CPLB_EINVAL


def test_batch_graph_replays_match_eager_steps(cplb):
    import torch
    cases = mixed_cases("f32")
    s = torch.cuda.Stream()
    a = make_batch(cplb, cases, stream=s)
    e = make_batch(cplb, cases)
    a.step(1)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        a.step(4)
    torch.cuda.synchronize()
    e.step(1)
    for rep in range(3):
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        e.step(4)
        torch.cuda.synchronize()
        for k in range(len(cases)):
            for f in ("phi", "c1", "ux"):
                assert np.array_equal(a.field(k, f).cpu().numpy(),
                                      e.field(k, f).cpu().numpy()), (rep, k, f)


def test_full_sweep_sampled_cases(cplb):
    """The 512-case sweep at full size in the benchmarked launch
    configuration: sampled cases equal their single-lattice runs, every case
    stays finite and conserves its phase."""
    sw = W.batched_sweep()
    cases = sw["cases"]
    say(f"full sweep: {len(cases)} cases, {sw['nodes']} nodes, 20 steps")
    b = make_batch(cplb, cases)
    r0 = [b.reduce(k)["sum_phi"] for k in range(len(cases))]
    b.step(20)
    bad = []
    for k in range(len(cases)):
        r = b.reduce(k)
        if r["rc"] != 0 or abs(r["sum_phi"] - r0[k]) > 1e-5 * abs(r0[k]):
            bad.append((k, r["rc"], r["sum_phi"], r0[k]))
    assert not bad, bad[:5]
    for k in (0, 1, 100, 257, 400, 511):
        g = single(cplb, cases[k], 20)
        for f in ("phi", "c1", "c2", "ux", "uy", "p"):
            assert np.array_equal(b.field(k, f).cpu().numpy(), g.field(f).cpu().numpy()), (k, f)
        g.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_batch_closure_equals_single_lattice_closure(cplb, precision):
    """Per-node closure corrections over the whole batch (case after case,
    its s1 plane then its s2 plane) act on each case exactly as the same
    slice does on the case run alone: bitwise equal fields, and c1 + c2
    moved by exactly what the corrections take (8 sum (s1 + s2))."""
    import torch
    cases = mixed_cases(precision, seed=9)
    say(f"batch closure vs single-lattice closure, {precision}, 8 steps")
    b = make_batch(cplb, cases)
    n = b.num_nodes
    assert n == sum(c["params"]["nx"] * c["params"]["ny"] for c in cases)
    s_host = (np.random.default_rng(2).normal(size=2 * n) * 2e-3).astype(np.float32)
    s = torch.tensor(s_host, device="cuda").contiguous()
    b.set_closure(s)
    c0 = [b.reduce(k)["sum_c"] for k in range(len(cases))]
    b.step(8)
    off = 0
    for k, c in enumerate(cases):
        nx, ny = c["params"]["nx"], c["params"]["ny"]
        g = cplb.Lattice(c["params"])
        g.init_sdf(c["sdf"], c1=c["init"]["c1"], c2=c["init"]["c2"])
        g.set_closure(s[2 * off:2 * (off + nx * ny)].view(2, ny, nx).contiguous())
        g.step(8)
        for f in ("phi", "c1", "c2", "ux", "uy", "p"):
            a, r = b.field(k, f).cpu().numpy(), g.field(f).cpu().numpy()
            assert np.array_equal(a, r), (k, f, float(np.abs(a - r).max()))
        tol = 1e-12 if precision == "f64" else 1e-6
        taken = 8.0 * float(s_host[2 * off:2 * (off + nx * ny)].astype(np.float64).sum())
        assert abs(b.reduce(k)["sum_c"] - (c0[k] - taken)) <= tol * abs(c0[k]), k
        off += nx * ny
        g.close()
    # switching the closure off restores the plain step
    b.set_closure(None)
    p = make_batch(cplb, cases)
    b2 = make_batch(cplb, cases)
    b2.set_closure(s)
    b2.set_closure(None)
    p.step(3)
    b2.step(3)
    assert np.array_equal(p.field(4, "c1").cpu().numpy(), b2.field(4, "c1").cpu().numpy())


def test_batch_gather_layout_and_init_planes(cplb):
    """gather writes field f of case c at [c's offset * nplanes + f * nodes_c]
    (float32 of the same values field() returns) and leaves the extra planes
    alone; init_planes from that buffer equals init_fields from the same
    values (u = p = 0), bitwise, after further steps."""
    import torch
    cases = mixed_cases("f32", seed=13)
    b = make_batch(cplb, cases)
    b.step(7)
    names = ("phi", "c1", "c2", "ux")
    nplanes = 6
    out = torch.full((b.num_nodes * nplanes,), -7.0, dtype=torch.float32, device="cuda")
    g = b.gather(names, out=out, nplanes=nplanes).cpu().numpy()
    off = 0
    for k, c in enumerate(cases):
        nx, ny = c["params"]["nx"], c["params"]["ny"]
        blk = g[off * nplanes:(off + nx * ny) * nplanes].reshape(nplanes, ny, nx)
        for f, name in enumerate(names):
            want = b.field(k, name, dtype=torch.float32).cpu().numpy()
            assert np.array_equal(blk[f], want), (k, name)
        assert np.all(blk[len(names):] == -7.0), k
        off += nx * ny
    # a fresh batch from the gathered phi, c1, c2 (plane order permuted)
    perm = torch.tensor(g).view(-1).clone()
    planes = torch.empty_like(perm)
    off = 0
    for c in cases:
        m = c["params"]["nx"] * c["params"]["ny"]
        src = perm[off * nplanes:(off + m) * nplanes].view(nplanes, m)
        dst = planes[off * nplanes:(off + m) * nplanes].view(nplanes, m)
        dst[:] = src
        dst[0], dst[2], dst[4] = src[2], src[0], src[1]  # c2, phi, c1 at 0, 2, 4
        off += m
    b2 = cplb.Batch([c["params"] for c in cases])
    b2.init_planes(planes.cuda(), nplanes, iphi=2, ic1=4, ic2=0)
    b2.step(5)
    for k, c in enumerate(cases):
        gk = cplb.Lattice(c["params"])
        m = c["params"]["nx"] * c["params"]["ny"]
        shp = (c["params"]["ny"], c["params"]["nx"])
        phi, c1, c2 = (b.field(k, f, dtype=torch.float32).cpu().numpy().astype(np.float64)
                       for f in ("phi", "c1", "c2"))
        gk.init_fields(phi.reshape(shp), c1.reshape(shp), c2.reshape(shp))
        gk.step(5)
        for f in ("phi", "c1", "c2", "ux", "uy", "p"):
            assert np.array_equal(b2.field(k, f).cpu().numpy(), gk.field(f).cpu().numpy()), (k, f)
        assert m > 0
        gk.close()
    with pytest.raises(AssertionError):
        b2.init_planes(planes.cuda()[:-1], nplanes)


@pytest.mark.parametrize("precision", ["f32", "f64", "f32_s16f"])
def test_batch_moment_gather_equals_field_readout(cplb, precision):
    """Fields that need only the node's own moments (phi, c1, c2, psi) are
    gathered straight from the populations; they equal the read-out through
    the macros kernel bit for bit (as float32)."""
    import torch
    cases = mixed_cases(precision, seed=21)
    b = make_batch(cplb, cases)
    b.step(9)
    names = ("c2", "phi", "psi", "c1")
    g = b.gather(names, nplanes=5).cpu().numpy()
    off = 0
    for k, c in enumerate(cases):
        nx, ny = c["params"]["nx"], c["params"]["ny"]
        blk = g[off * 5:(off + nx * ny) * 5].reshape(5, ny, nx)
        for f, name in enumerate(names):
            want = b.field(k, name, dtype=torch.float32).cpu().numpy()
            assert np.array_equal(blk[f], want), (precision, k, name)
        off += nx * ny


def test_full_sweep_5000_steps(cplb):
    """The 512-case sweep for its configured 5000 steps, replayed from one
    captured graph as benchmarked: every case stays finite, keeps its phase
    mass to the 1e-6 target and its scalar mass to a guard at about twice
    the largest drift measured."""
    import torch
    sw = W.batched_sweep()
    cases = sw["cases"]
    say(f"full sweep: {len(cases)} cases, {sw['nodes']} nodes, 5000 steps from a graph")
    stream = torch.cuda.Stream()
    b = cplb.Batch([c["params"] for c in cases], stream=stream)
    for k, c in enumerate(cases):
        b.init_sdf(k, c["sdf"], c1=c["init"]["c1"], c2=c["init"]["c2"])
    r0 = [b.reduce(k) for k in range(len(cases))]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        b.step(1000)
    for _ in range(5):
        with torch.cuda.stream(stream):
            g.replay()
        torch.cuda.synchronize()
    dphi, dc, bad = [], [], []
    for k in range(len(cases)):
        r = b.reduce(k)
        if r["rc"] != 0 or r["nonfinite"] != 0:
            bad.append((k, r["rc"], r["nonfinite"]))
            continue
        dphi.append(abs(r["sum_phi"] - r0[k]["sum_phi"]) / abs(r0[k]["sum_phi"]))
        dc.append(abs(r["sum_c"] - r0[k]["sum_c"]) / abs(r0[k]["sum_c"]))
    # (the host's step counter counts the captured steps, not the replays)
    b.close()
    del g
    assert not bad, bad[:5]
    k1, k2 = int(np.argmax(dphi)), int(np.argmax(dc))
    say(f"  phase-mass drift max {dphi[k1]:.2e} (case {k1}), median {np.median(dphi):.2e}; "
        f"scalar-mass drift max {dc[k2]:.2e} (case {k2}), median {np.median(dc):.2e}")
    assert max(dphi) <= 1e-6, (k1, dphi[k1])
    assert max(dc) <= 5e-7, (k2, dc[k2])  # measured 2.1e-7 (MI355X)
