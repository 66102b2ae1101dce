"""The allocation-free reduction (cplb_reduce_device, partials in a fixed
device array of the library) against cplb_reduce (partials in the handle's
workspace), through the C-ABI: the same FP64 values bit for bit, on two calls
in a row, the second on a smaller lattice, so the shared array holds the
first call's partials when the second starts."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def both(C, lat):
    import torch
    L = C.library()
    host = (ctypes.c_double * 8)()
    assert L.cplb_reduce(lat.handle, host) == 0, L.cplb_last_error(lat.handle)
    dev = torch.full((8,), -7.0, dtype=torch.float64, device="cuda")
    lat.stream.wait_stream(torch.cuda.current_stream())
    rc = L.cplb_reduce_device(lat.handle, ctypes.c_void_p(dev.data_ptr()))
    assert rc == 0, L.cplb_last_error(lat.handle)
    lat.stream.synchronize()
    out = dev.cpu().numpy()
    ref = np.array(host[:7])
    assert np.array_equal(out[:7], ref), (out[:7], ref)
    assert out[7] == -7.0  # the step counter is host state; dev_out[7] is left alone
    return ref


@pytest.fixture(scope="module")
def C():
    import torch

    from paper_2402_15752_amd import cplb
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cplb.library()
    return cplb


def test_reduce_device_matches_reduce_twice(C):
    # first call: a lattice with the full 1024 partials (263,000 nodes)
    say("no-alloc reduce: 2-D 530x500 FP32, then 3-D 24x20x18 FP64")
    p1 = W.params(nx=530, ny=500, periodic=(1, 0, 1), precision="f32", sigma=2e-3, rho1=3.0,
                  rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07, D2=0.02, Keq=0.6, A=0.4,
                  g=(2e-5, -3e-5, 0.0), rho_ref=1.5, ref_f=0.5)
    f1 = W.random_fields(p1, seed=5)
    a = C.Lattice(p1)
    a.init_fields(f1["phi"], f1["c1"], f1["c2"], u=f1["u"], p=f1["p"])
    a.step(3)
    r1 = both(C, a)
    assert r1[6] == 0 and r1[0] > 0
    # second call, smaller input: 8,640 nodes, 34 partials of the 1024 left by the first
    p2 = W.params(nx=24, ny=20, nz=18, lattice="d3q19_d3q7", periodic=(1, 1, 0), precision="f64",
                  sigma=2e-3, rho1=3.0, rho2=1.0, visc_law="exp", mu1=0.3, mu2=0.08, D1=0.07,
                  D2=0.02, Keq=0.6, A=0.4, g=(1e-5, -2e-5, 3e-5), rho_ref=1.5)
    f2 = W.random_fields(p2, seed=6)
    b = C.Lattice(p2)
    b.init_fields(f2["phi"], f2["c1"], f2["c2"], u=f2["u"], p=f2["p"])
    b.step(2)
    r2 = both(C, b)
    assert r2[6] == 0 and abs(r2[0] - r1[0]) > 1.0
    # and the first lattice again, after the smaller one
    r3 = both(C, a)
    assert np.array_equal(r1, r3)
    a.close()
    b.close()


def test_reduce_device_rejects_null_arguments(C):
    L = C.library()
    lat = C.Lattice(W.params(nx=16, ny=8, precision="f32"))
    assert L.cplb_reduce_device(None, None) == C.CPLB_EINVAL
    assert L.cplb_reduce_device(lat.handle, None) == C.CPLB_EINVAL
    assert L.cplb_last_error(lat.handle).decode()
    lat.close()
