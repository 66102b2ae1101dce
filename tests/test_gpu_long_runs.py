"""Long runs of the benchmarked configurations on the GPU: the 2-D rising
bubble for 20,000 steps and the 3-D rising droplet for 5,000, checked for
stability (no non-finite value), mass conservation and motion.

The scheme conserves sum phi and sum (c1 + c2) exactly (pin P2 of the
oracle); in finite precision each stored population is rounded.  f, h1 and
h2 are stored relative to the moments of the node they are stored at, so
a rounding is relative to the change of that node's moment over one step,
not to the moment itself.  Measured (MI355X):

  bubble 256 x 1024, FP32, 20,000 steps:  phi 2.1e-9,  c1 + c2 1.3e-7
  droplet 256^3, FP32, 5,000 steps:       phi 1.5e-11, c1 + c2 3.5e-9
  droplet 256^3, FP16 storage, 5,000:     phi 1.8e-8,  c1 + c2 2.4e-4

The phase-mass target, 1e-6, is asserted for every run; the scalar-mass
bounds (no stated target) are regression guards at about twice the
measured drift."""
import numpy as np
import pytest

import workloads as W

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


def drift(r, r0, k):
    return abs(r[k] - r0[k]) / abs(r0[k])


def gas_height(g):
    """Centre of the gas (phi -> 0) along y, in nodes."""
    phi = g.field("phi").cpu().numpy().astype(np.float64)
    gas = 1.0 - phi
    return float((gas * np.arange(phi.shape[0])[:, None]).sum() / gas.sum())


def test_rising_bubble_20000_steps(cplb):
    w = W.rising_bubble_2d()
    say("rising bubble 256x1024 f32, 20000 steps")
    g = cplb.Lattice(w["params"])
    g.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    r0, y0 = g.reduce(), gas_height(g)
    g.step(20000)
    r = g.reduce()
    y1 = gas_height(g)
    say(f"  phi drift {drift(r, r0, 'sum_phi'):.2e}  c drift {drift(r, r0, 'sum_c'):.2e}  "
        f"bubble {y0:.1f} -> {y1:.1f}  max|u| {r['max_u']:.2e}")
    assert r["nonfinite"] == 0 and r["step"] == 20000
    assert drift(r, r0, "sum_phi") <= 1e-6
    assert drift(r, r0, "sum_c") <= 3e-7
    assert y1 - y0 > 50.0  # the bubble rises (85 nodes measured)


@pytest.mark.parametrize("precision,phi_bound,c_bound", [("f32", 1e-6, 1e-8),
                                                         ("f32_s16f", 1e-6, 5e-4)])
def test_rising_droplet_5000_steps(cplb, precision, phi_bound, c_bound):
    w = W.rising_droplet_3d(256, precision)
    say(f"rising droplet 256^3 {precision}, 5000 steps")
    g = cplb.Lattice(w["params"])
    g.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    r0 = g.reduce()
    g.step(5000)
    r = g.reduce()
    say(f"  phi drift {drift(r, r0, 'sum_phi'):.2e}  c drift {drift(r, r0, 'sum_c'):.2e}  "
        f"max|u| {r['max_u']:.2e}")
    assert r["nonfinite"] == 0 and r["step"] == 5000
    assert drift(r, r0, "sum_phi") <= phi_bound
    assert drift(r, r0, "sum_c") <= c_bound
    assert r["max_u"] > 1e-3  # the droplet moves
    g.close()
