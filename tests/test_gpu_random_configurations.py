"""GPU parity over the configuration space: 32 seeded random configurations
mixing lattice (D2Q9 / D3Q19 + D3Q7), grid sizes (one-node-wide axes and
ragged tiles included), walls per axis, scalar model (two-scalar /
one-scalar), gradient scheme (central / local, Eq. (39)), Dirichlet faces,
viscosity law (Eq. (1.8) / Eq. (4.3)) and every physical parameter, from
seeded random fields.  FP64: the GPU step must match the oracle to
round-off (1e-12 relative) on every field after 3 steps.  The draws are
fixed by the seed; the host-side check (`valid`) is the library's own
validation, repeated on the CPU as `make_params` + workspace sizing."""
import numpy as np
import pytest

import workloads as W
from oracle import ref

pytestmark = pytest.mark.gpu

NCONF = 32
ALL2 = ("phi", "c1", "c2", "ux", "uy", "p", "mu", "psi")


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def cplb():
    import torch

    from paper_2402_15752_amd import cplb as C
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    C.library()
    return C


def draw(k):
    rng = np.random.default_rng(9000 + k)
    u = lambda a, b: float(a + (b - a) * rng.random())          # noqa: E731
    lu = lambda a, b: float(np.exp(u(np.log(a), np.log(b))))    # noqa: E731
    three = rng.random() < 0.4
    if three:
        n3 = [int(rng.integers(1, 21)), int(rng.integers(1, 21)), int(rng.integers(2, 25))]
    else:
        n3 = [int(rng.integers(1, 71)), int(rng.integers(1, 41)), 1]
    per = [1, 1, 1]
    for a in range(3 if three else 2):
        per[a] = 1 if n3[a] < 2 else int(rng.random() < 0.5)
    one = (not three) and rng.random() < 0.2
    local = (not one) and rng.random() < 0.3
    bc = ["noflux"] * 6
    cw = [(0.0, 0.0)] * 6
    if not three and not one and not local:
        for f in range(4):
            if not per[f // 2] and rng.random() < 0.4:
                bc[f] = "dirichlet"
                cw[f] = (u(0.0, 1.0), u(0.0, 1.0))
    rho1, rho2 = lu(0.5, 10.0), lu(0.5, 10.0)
    gz = u(-3e-5, 3e-5) if three else 0.0
    return W.params(
        nx=n3[0], ny=n3[1], nz=n3[2], lattice="d3q19_d3q7" if three else "d2q9",
        periodic=tuple(per), precision="f64",
        scalar_model="one" if one else "two", scalar_grad="local" if local else "central",
        scalar_bc=tuple(bc), c_wall=tuple(cw),
        visc_law="exp" if rng.random() < 0.5 else "linear",
        rho1=rho1, rho2=rho2, mu1=lu(0.02, 0.5), mu2=lu(0.02, 0.5), sigma=u(0.0, 1e-2),
        W=u(2.0, 6.0), M=lu(0.005, 0.1), D1=lu(0.005, 0.2), D2=lu(0.005, 0.2),
        Keq=lu(0.6 if one else 0.2, 5.0), A=u(0.0, 0.5),
        g=(u(-3e-5, 3e-5), u(-3e-5, 3e-5), gz), rho_ref=u(min(rho1, rho2), max(rho1, rho2)),
        n_eps=lu(1e-6, 1e-3))


def test_draws_are_valid_and_varied(cplb):
    """Every draw passes the library's validation, and the set covers the
    options it is meant to mix."""
    ps = [draw(k) for k in range(NCONF)]
    for p in ps:
        assert cplb.cplb_workspace_bytes(cplb.make_params(p)) > 0
    assert any(p["lattice"] != "d2q9" for p in ps)
    assert any(p["scalar_model"] == "one" for p in ps)
    assert any(p["scalar_grad"] == "local" for p in ps)
    assert any(p["scalar_grad"] == "local" and p["lattice"] != "d2q9" for p in ps)
    assert any("dirichlet" in p["scalar_bc"] for p in ps)
    assert any(min(p["nx"], p["ny"]) == 1 for p in ps)


@pytest.mark.parametrize("k", range(NCONF))
def test_fp64_random_configuration(cplb, k):
    p = draw(k)
    d3 = p["lattice"] != "d2q9"
    say(f"config {k}: {p['lattice']} {p['nx']}x{p['ny']}x{p['nz']} periodic={p['periodic']} "
        f"{p['scalar_model']} {p['scalar_grad']} bc={[b[0] for b in p['scalar_bc']]} {p['visc_law']}")
    f = W.random_fields(p, seed=100 + k)
    g = cplb.Lattice(p)
    o = ref.Oracle(p)
    for s in (g, o):
        s.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    g.step(3)
    o.step(3)
    names = ALL2 + (("uz",) if d3 else ())
    errs = {}
    for name in names:
        a = g.field(name).cpu().numpy()
        b = o.field(name)
        assert np.all(np.isfinite(a)), name
        scale = max(np.linalg.norm(b), np.linalg.norm(b - b.mean()), 1e-300)
        errs[name] = float(np.linalg.norm(a - b) / scale)
    say("  " + " ".join(f"{n}={e:.1e}" for n, e in errs.items()))
    bad = {n: e for n, e in errs.items() if not e <= 1e-12}
    assert not bad, (k, bad)
    g.close()
