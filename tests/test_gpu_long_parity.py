"""Full-length 3-D parity: the HIP path (through the C-ABI) against the FP64
CPU oracle at the lengths the FP32 and 16-bit targets are stated for.

  * 128^3 rising droplet, 1000 steps: FP32 storage, FP16 storage and BF16
    storage (FP32 arithmetic in all three) against one oracle run;
  * 64^3 rising droplet, the workload's full 5000 steps: FP32 and FP16
    storage.

Every field is compared by its relative L2 error and, so that an error
confined to a few nodes -- a wall row, the interface -- cannot hide under
the norm, by its max-abs error: the largest nodal error over the field's
scale (its largest magnitude, p its largest deviation from the mean).
Velocity components are compared as one vector field (the norm of the error
vector over the norm of the velocity), as the target is stated for the
velocity.

The targets are 1e-5 (FP32) and 2e-3 (16-bit storage) after 1000 steps.
Measured on MI355X (rel L2 / max-abs):

  128^3, 1000 steps, FP32:  phi 1.2e-7  c1 1.6e-6  c2 2.5e-6  p 1.22e-5  u 1.16e-5
  128^3, 1000 steps, FP16:  all fields within 2e-3
  128^3, 1000 steps, BF16:  phi 2.5e-5  c1 3.6e-4  c2 4.5e-4  p 1.24e-2  u 2.5e-3
  64^3, 5000 steps, FP32:   phi 1.8e-6  c1 2.5e-6  c2 3.5e-5  p 1.0e-4  u 1.9e-5
  64^3, 5000 steps, FP16:   phi 4.7e-6  c1 1.3e-4  c2 2.7e-4  p 3.8e-3  u 2.2e-4

Where a field meets its target it is asserted at the target.  The misses --
FP32 p and u at 128^3 (1.2x the target), BF16 p and u -- are asserted at
regression guards of about twice the measured value, and each also has an
assertion at the stated target marked xfail(strict): it reports the miss on
every run, and fails the suite the day the miss goes away unnoticed.  The
5000-step runs have no stated field target (it is stated after 1000 steps);
their fields are held to guards, their phase mass to the stated drift
bound, 1e-6."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu

SCALARS = ("phi", "c1", "c2", "p")
FIELDS = SCALARS + ("u",)
TARGET = {"f32": 1e-5, "f32_s16f": 2e-3, "f32_s16b": 2e-3}
MAXABS = {"f32": 3e-4, "f32_s16f": 2e-2, "f32_s16b": 2e-2}
# fields that miss the target after 1000 steps at 128^3: regression guards
GUARD_128 = {"f32": {"p": 2.5e-5, "u": 2.5e-5}, "f32_s16b": {"p": 2.5e-2, "u": 5e-3}}
# 5000 steps on 64^3 (no stated field target at this length): guards
GUARD_5000 = {"f32": {"phi": 1e-5, "c1": 1e-5, "c2": 1e-4, "p": 3e-4, "u": 5e-5},
              "f32_s16f": {"phi": 2e-5, "c1": 5e-4, "c2": 1e-3, "p": 1e-2, "u": 1e-3}}


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


def errors(g, o):
    """Relative L2 and max-abs errors of phi, c1, c2, p and the velocity."""
    out = {}
    for k in SCALARS:
        a = g.field(k).cpu().numpy()
        b = o.field(k)
        assert np.all(np.isfinite(a)), k
        scale_l2 = max(np.linalg.norm(b), np.linalg.norm(b - b.mean()), 1e-300)
        scale_max = max(np.abs(b).max(), np.abs(b - b.mean()).max(), 1e-300)
        if k == "p":  # p is normalised by its variation
            scale_l2 = np.linalg.norm(b - b.mean())
            scale_max = np.abs(b - b.mean()).max()
        out[k] = (float(np.linalg.norm(a - b) / scale_l2), float(np.abs(a - b).max() / scale_max))
    ua = np.stack([g.field(k).cpu().numpy() for k in ("ux", "uy", "uz")])
    ub = np.stack([o.field(k) for k in ("ux", "uy", "uz")])
    du = np.sqrt(((ua - ub) ** 2).sum(axis=0))
    nb = np.sqrt((ub ** 2).sum(axis=0))
    out["u"] = (float(np.linalg.norm(du) / np.linalg.norm(nb)), float(du.max() / nb.max()))
    return out


def report(label, errs):
    say(f"  {label}: " + " ".join(f"{k}={v[0]:.2e}/{v[1]:.2e}" for k, v in errs.items()))


def check(errs, bounds, maxabs, label):
    bad = {k: v for k, v in errs.items() if k in bounds and not (v[0] <= bounds[k] and v[1] <= maxabs)}
    assert not bad, (label, bad, bounds, maxabs)


_runs = {}


def run_128(cplb, oracle_128, precision):
    """Errors of one 128^3 1000-step run, computed once per precision."""
    if precision not in _runs:
        w, o = oracle_128
        p = dict(w["params"], precision=precision, ref_f=W.phase_reference(precision))
        say(f"rising droplet 128^3 {precision} 1000 steps")
        g = cplb.Lattice(p)
        g.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
        g.step(1000)
        errs = errors(g, o)
        g.close()
        report(f"{precision} t=1000", errs)
        _runs[precision] = errs
    return _runs[precision]


@pytest.fixture(scope="module")
def oracle_128():
    w = W.rising_droplet_3d(n=128)
    say("oracle: rising droplet 128^3, 1000 steps (about a minute on 16 cores)")
    o = ref.run_workload(w, steps=1000)
    yield w, o
    o.close()


@pytest.mark.parametrize("precision", ["f32", "f32_s16f", "f32_s16b"])
def test_droplet_128_1000_steps(cplb, oracle_128, precision):
    """Fields that meet the target at the target, the misses at their guards."""
    errs = run_128(cplb, oracle_128, precision)
    guards = GUARD_128.get(precision, {})
    bounds = {k: guards.get(k, TARGET[precision]) for k in FIELDS}
    check(errs, bounds, MAXABS[precision], precision)


@pytest.mark.parametrize("precision", [
    pytest.param("f32", marks=pytest.mark.xfail(strict=True, reason=(
        "FP32 p and u after 1000 steps at 128^3: 1.22e-5 and 1.16e-5 of the 1e-5 target "
        "(FP32 arithmetic of the flow update; 64^3 meets it)"))),
    pytest.param("f32_s16b", marks=pytest.mark.xfail(strict=True, reason=(
        "BF16 storage p and u after 1000 steps: 1.24e-2 and 2.5e-3 of the 2e-3 target "
        "(an 8-bit significand re-rounded every step)"))),
])
def test_droplet_128_missed_fields_at_target(cplb, oracle_128, precision):
    errs = run_128(cplb, oracle_128, precision)
    bounds = {k: TARGET[precision] for k in GUARD_128[precision]}
    check(errs, bounds, MAXABS[precision], precision + " at the stated target")


@pytest.fixture(scope="module")
def oracle_64_5000():
    w = W.rising_droplet_3d(n=64)
    say("oracle: rising droplet 64^3, 5000 steps")
    o = ref.run_workload(w, steps=5000)
    yield w, o
    o.close()


@pytest.mark.parametrize("precision", ["f32", "f32_s16f"])
def test_droplet_64_full_run(cplb, oracle_64_5000, precision):
    w, o = oracle_64_5000
    p = dict(w["params"], precision=precision, ref_f=W.phase_reference(precision))
    say(f"rising droplet 64^3 {precision} 5000 steps")
    g = cplb.Lattice(p)
    g.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    r0 = g.reduce()
    g.step(5000)
    r = g.reduce()
    errs = errors(g, o)
    report(f"{precision} t=5000", errs)
    dphi = abs(r["sum_phi"] - r0["sum_phi"]) / r0["sum_phi"]
    say(f"  phase-mass drift {dphi:.2e}")
    g.close()
    check(errs, GUARD_5000[precision], MAXABS[precision], precision)
    assert dphi <= 1e-6
