"""End-to-end test of the learned closure on the rising bubble: fine-grid
runs of the plain method generate the training data, the closure network is
trained on the GPU by its own kernels, and held-out cases run freely on the
coarse grid with and without it, against the restricted fine run (the
reference for its error).

Walled rising bubbles with interfacial transfer (density ratio 10,
viscosity ratio 10 under the exponential law, Eo = 10), coarse 64 x 256
against fine 256 x 1024 (F = 4 in space, 16 in time), 32 training draws,
100 coarse steps, one training round on targets averaged over spans of 5
coarse steps.  The test shows what the network gains: the median relative
L2 error of (c1, c2) with the closure is well below the plain coarse run's,
most held-out cases improve, the held-out loss falls well below that of the
zero closure (1), and the closure-corrected coarse run is at least 5x
faster than the fine run.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_closure_gains_over_plain_coarse_run():
    import torch

    from paper_2402_15752_amd import closure as CL
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    say("closure pipeline: rising bubble, 32 training draws, 16 held-out, 64x256 vs 256x1024, 100 steps")
    r = CL.experiment(n_train=32, n_test=16, steps=100, nc=64, iters=(1500,), batch=16, seed=3,
                      kind="rising", every=5, skip=0, rounds=1, log=say)
    r.pop("net")
    say(str({k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}))
    assert np.isfinite(r["err_plain_coarse"]) and np.isfinite(r["err_closure"])
    assert r["held_round1"][-1][1] < 0.5, r
    assert r["err_closure"] < 0.85 * r["err_plain_coarse"], r
    assert r["closure_better_cases"] >= 12, r
    assert r["speedup_closure_vs_fine"] >= 5.0, r
