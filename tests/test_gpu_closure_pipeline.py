"""End-to-end test of the learned closure: fine-grid runs of the plain
method generate the training data, the closure network is trained on the
GPU by its own kernels, and held-out cases run freely on the coarse grid
with and without it, against the restricted fine run (the reference for
its error).

Static drops with interfacial transfer, coarse 64 x 64 against fine
256 x 256 (F = 4 in space, 16 in time), 100 coarse steps.  The test
shows what the network gains: the median relative L2 error of (c1, c2)
with the closure is below the plain coarse run's, below 1e-2, and the
closure-corrected coarse run is at least 5x faster than the fine run.
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
    say("closure pipeline: 32 training cases, 16 held-out cases, 64x64 vs 256x256, 100 steps")
    r = CL.experiment(n_train=32, n_test=16, steps=100, nc=64, iters=(1500, 1000), seed=3,
                      log=say)
    r.pop("net")
    say(str({k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}))
    assert np.isfinite(r["err_plain_coarse"]) and np.isfinite(r["err_closure"])
    # the fit beats the zero closure (normalised targets: predicting 0 costs >= 1)
    assert r["loss_round1"] < 1.0 and r["loss_last"] < 1.0, r
    assert r["err_closure"] < 0.95 * r["err_plain_coarse"], r
    assert r["closure_better_cases"] >= 10, r
    assert r["err_closure"] <= 1e-2, r
    assert r["speedup_closure_vs_fine"] >= 5.0, r
