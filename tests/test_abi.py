"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/cplb.h declares, the binding's struct matches the
header byte for byte, and parameter validation rejects what it must."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cplb.h")


@pytest.fixture(scope="module")
def cplb():
    from paper_2402_15752_amd import cplb as C
    if not os.path.exists(C.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return C


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cplb_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(cplb):
    names = declared_functions()
    assert len(names) >= 14
    lib = cplb.library()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(cplb.EXPORTS) == names


def test_params_struct_matches_header(cplb, tmp_path):
    fields = [f for f, _ in cplb.cplb_params._fields_]
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){",
             'printf("%zu\\n", sizeof(cplb_params));']
    for f in fields:
        lines.append(f'printf("%zu\\n", offsetof(cplb_params, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(cplb.cplb_params)
    for f, off in zip(fields, out[1:]):
        assert getattr(cplb.cplb_params, f).offset == off, f


def test_workspace_bytes_cover_two_lattices(cplb):
    for w, qtot, s in ((W.static_drop_64(), 36, 8), (W.rising_bubble_2d(), 36, 4),
                       (W.rising_droplet_3d(n=64), 40, 4)):
        n = W.n_nodes(w["params"])
        b = cplb.cplb_workspace_bytes(cplb.make_params(w["params"]))
        assert b >= 2 * qtot * n * s
        assert b < 2 * qtot * n * s * 1.5


@pytest.mark.parametrize("bad", [dict(D2=0.0), dict(Keq=0.0), dict(M=-1.0), dict(nx=0),
                                 dict(rho1=0.0), dict(g=(0, 0, 1e-5)), dict(n_eps=0.0),
                                 dict(periodic=(1, 0, 1), ny=1), dict(nz=2),
                                 dict(precision="f32", sigma=float("nan")),
                                 dict(scalar_model="one", lattice="d3q19_d3q7", nz=8, nx=8, ny=8),
                                 dict(scalar_bc=("dirichlet",) + ("noflux",) * 5),
                                 dict(periodic=(0, 1, 1), scalar_model="one",
                                      scalar_bc=("dirichlet",) + ("noflux",) * 5),
                                 dict(lattice="d3q19_d3q7", nz=8, nx=8, ny=8, periodic=(1, 1, 0),
                                      scalar_bc=("noflux",) * 4 + ("dirichlet", "noflux")),
                                 dict(scalar_grad="local", scalar_model="one")])
def test_validation_rejects(cplb, bad):
    p = W.params(**bad)
    with pytest.raises(cplb.CplbError) as e:
        cplb.cplb_workspace_bytes(cplb.make_params(p))
    assert e.value.code == cplb.CPLB_EINVAL


def test_scalar_model_field(cplb):
    """The one-scalar model is selected through cplb_params.scalar_model; an
    unknown model id is refused."""
    prm = cplb.make_params(W.params(scalar_model="one"))
    assert prm.scalar_model == cplb.CPLB_ONE_SCALAR
    assert cplb.cplb_workspace_bytes(prm) > 0
    prm.scalar_model = 2
    with pytest.raises(cplb.CplbError) as e:
        cplb.cplb_workspace_bytes(prm)
    assert e.value.code == cplb.CPLB_EINVAL


def test_create_rejects_bad_workspace(cplb):
    prm = cplb.make_params(W.params())
    n = cplb.cplb_workspace_bytes(prm)
    h = ctypes.c_void_p()
    lib = cplb.library()
    # null and misaligned workspaces are refused before any device call
    assert lib.cplb_create(ctypes.byref(prm), None, n, None, ctypes.byref(h)) == cplb.CPLB_EINVAL
    assert lib.cplb_create(ctypes.byref(prm), ctypes.c_void_p(4096 + 8), n, None,
                           ctypes.byref(h)) == cplb.CPLB_EINVAL
    # a workspace smaller than required is refused
    assert lib.cplb_create(ctypes.byref(prm), ctypes.c_void_p(4096), n - 1, None,
                           ctypes.byref(h)) == cplb.CPLB_ENOMEM
    assert lib.cplb_strerror(cplb.CPLB_ENOMEM).decode().startswith("workspace")


# ----------------------------------------------------------------- batches

def test_batch_validation_and_workspace(cplb):
    ps = [W.params(nx=40, ny=30, precision="f32"), W.params(nx=100, ny=64, precision="f32",
                                                             periodic=(1, 0, 1))]
    n = cplb.cplb_batch_workspace_bytes(cplb._params_array(ps), 2)
    single = sum(cplb.cplb_workspace_bytes(cplb.make_params(p)) for p in ps)
    assert n >= single - 2 * 70000  # per-case regions (the single API adds its own partials)
    bad_sets = [
        [W.params(precision="f32"), W.params(precision="f64")],                 # mixed precision
        [W.params(precision="f32"), W.params(nx=8, ny=8, nz=8, lattice="d3q19_d3q7",
                                             precision="f32")],                 # not D2Q9
        [W.params(precision="f32"), W.params(precision="f32", D1=0.0)],         # invalid case
        [W.params(precision="f32"), W.params(precision="f32", scalar_model="one")],  # one-scalar
        [W.params(precision="f32"), W.params(precision="f32", periodic=(0, 1, 1),
                                             scalar_bc=("dirichlet",) + ("noflux",) * 5)],
    ]
    for ps in bad_sets:
        with pytest.raises(cplb.CplbError) as e:
            cplb.cplb_batch_workspace_bytes(cplb._params_array(ps), len(ps))
        assert e.value.code == cplb.CPLB_EINVAL
    lib = cplb.library()
    b = ctypes.c_void_p()
    arr = cplb._params_array([W.params(precision="f32")])
    assert lib.cplb_batch_create(arr, 0, ctypes.c_void_p(4096), 1 << 30, None,
                                 ctypes.byref(b)) == cplb.CPLB_EINVAL
    assert lib.cplb_batch_create(arr, 1, None, 1 << 30, None, ctypes.byref(b)) == cplb.CPLB_EINVAL
    assert lib.cplb_batch_create(arr, 1, ctypes.c_void_p(4096), 1024, None,
                                 ctypes.byref(b)) == cplb.CPLB_ENOMEM


def test_batched_sweep_recipe():
    a, b = W.batched_sweep(64, seed=0), W.batched_sweep(64, seed=0)
    c = W.batched_sweep(64, seed=1)
    assert [x["params"] for x in a["cases"]] == [x["params"] for x in b["cases"]]
    assert [x["params"] for x in a["cases"]] != [x["params"] for x in c["cases"]]
    full = W.batched_sweep()
    assert len(full["cases"]) == 512 and full["nodes"] == sum(
        x["params"]["nx"] * x["params"]["ny"] for x in full["cases"])
    cs2 = 1.0 / 3.0
    ratios = []
    for x in full["cases"]:
        p = x["params"]
        assert 64 <= p["nx"] <= 256 and 64 <= p["ny"] <= 256
        assert 0.1 <= p["Keq"] <= 10.0
        for d in (p["D1"], p["D2"]):
            tau = 0.5 + d / cs2
            assert 0.5 + 1e-3 - 1e-12 <= tau <= 2.0 + 1e-12
        assert p["D2"] >= p["D1"]
        ratios.append(p["D2"] / p["D1"])
        assert x["sdf"].shape == (p["ny"], p["nx"])
    # the diffusivity ratio is never clipped: log-uniform over [1, 1000]
    lr = np.log10(np.array(ratios))
    assert lr.min() >= -1e-12 and lr.max() <= 3.0 + 1e-12
    assert lr.max() > 2.95 and lr.min() < 0.05
    assert abs(np.median(lr) - 1.5) < 0.2
    # a case whose diffusivities were moved keeps its ratio; only Pe changes
    for k, pe_asked, pe_used in full["shifted"]:
        assert pe_asked != pe_used
    kinds = {x["params"]["periodic"][1] for x in full["cases"]}
    assert kinds == {0, 1}  # both static (periodic) and rising (walled) cases
