"""Throughput benchmark of the coupled phase-field LB step on one MI355X.

One step = one time step of the whole hot path (moments and implicit
recovery, stencils, flow macros and viscosity law, time-derivative terms,
collision of f, g, h1, h2 with their sources, streaming) over every node.

Default workload: the 3-D rising droplet with heat transfer, 256^3 nodes,
D3Q19 flow set + three D3Q7 sets (phase field, two scalars), FP32 compute
and storage, periodic in x and y, half-way bounce-back walls at the z faces
(6.2 GB of algorithmic traffic per step, far beyond the Infinity Cache, so
the step runs against HBM).  The side measurements cover FP16 / BF16
storage, the local gradient scheme, the 2-D bubble at 256 x 1024 and
2048 x 4096, the one-scalar model, the batched sweep and the learned
closure.  Inputs are synthetic (a signed-distance droplet) and resident in
HBM before the timed region starts.

Prints one JSON line.  `value` is MLUPS (million node updates per second,
all four sets per update) over the timed region; `roofline` relates the
step kernel's algorithmic HBM bytes to its average duration, both measured
with HIP events on the library's stream inside the timed region.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled-LB MLUPS + HBM GB/s vs peak; closure speedup at equal scalar error"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Memory-side bytes per launch of the step kernel, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), each scaled by what
# the same counter reads for a plain 1 GiB copy (FETCH_SIZE x 2, WRITE_SIZE
# x 1).  `src` is the hash of the kernel sources the counters were taken on;
# when the sources differ the figure no longer describes the kernel and the
# bench reports traffic as null.  Commands and raw figures: profiles/.
TRAFFIC = {
    "rising_bubble_256x1024_f32": {"read": 44327722, "write": 43021269,
                                 "src": "56116601f9a4ddd6"},
    "rising_droplet_256c_f32": {"read": 3167235093, "write": 3120879242,
                              "src": "56116601f9a4ddd6"},
    "rising_droplet_256c_f32_s16f": {"read": 1814247360, "write": 1779050981,
                                   "src": "56116601f9a4ddd6"},
    "rising_bubble_2048x4096_f32": {"read": 1396950506, "write": 1380970026,
                                  "src": "56116601f9a4ddd6"},
    "rising_bubble_one_256x1024_f32": {"read": 32821461, "write": 32524096,
                                     "src": "56116601f9a4ddd6"},
    "rising_bubble_local_2048x4096_f32": {"read": 1385056597, "write": 1381315504,
                                        "src": "56116601f9a4ddd6"},
    "rising_droplet_local_256c_f32": {"read": 3133757226, "write": 3122591946,
                                    "src": "56116601f9a4ddd6"},
    "rising_droplet_local_256c_f32_s16f": {"read": 1773479360, "write": 1771738480,
                                         "src": "56116601f9a4ddd6"},
}


# the sources that define the single-lattice step kernels, their launch and
# the default variant
STEP_SOURCES = ("addr.hpp", "api.hip", "common.hpp", "step2d.hip", "step2d_tile.hpp", "step3d.hip")


def kernel_source_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_2402_15752_amd", "csrc")
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        h.update(f.encode())
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    t = TRAFFIC.get(workload)
    if not t or t["src"] != kernel_source_hash():
        return None
    return t["read"] + t["write"]


def alg_bytes_per_node(p):
    """Algorithmic HBM bytes per node and step: every population read once
    and written once, plus the (u, phi, c1, c2) history read and written."""
    d = 2 if p["lattice"] == "d2q9" else 3
    qtot = 36 if d == 2 else 40
    nhist = d + 3
    if p.get("scalar_model", "two") == "one":
        # one-scalar model: f, g, h3 (27 values), history (u, phi, c)
        qtot, nhist = 27, d + 2
    s_pop = {"f64": 8, "f32": 4, "f32_s16f": 2, "f32_s16b": 2}[p["precision"]]
    s_hist = 8 if p["precision"] == "f64" else 4
    return 2 * qtot * s_pop + 2 * nhist * s_hist


def make_workload(name):
    import workloads as W
    if name == "rising_bubble_256x1024":
        return W.rising_bubble_2d(256, 1024, "f32")
    if name == "rising_bubble_one_256x1024":
        # the one-scalar model (h3) on the same bubble, Keq = 2
        return W.rising_bubble_2d(256, 1024, "f32", scalar_model="one")
    if name == "rising_bubble_local_256x1024":
        # grad(c1 + Keq c2) by the local scheme of Eq. (39): no h halo
        return W.rising_bubble_2d(256, 1024, "f32", scalar_grad="local")
    if name == "rising_bubble_local_2048x4096":
        return W.rising_bubble_2d(2048, 4096, "f32", scalar_grad="local")
    if name == "rising_bubble_2048x4096":
        # the same bubble 8x wider: 8.4M nodes, 2.75 GB per step, far beyond the
        # Infinity Cache -- the 2-D step against HBM
        return W.rising_bubble_2d(2048, 4096, "f32")
    if name.startswith("rising_droplet_256c"):
        prec = name[len("rising_droplet_256c_"):] or "f32"
        return W.rising_droplet_3d(256, prec)
    if name.startswith("rising_droplet_local_256c"):
        # grad(c1 + Keq c2) by the local scheme of Eq. (39): no h halo, no psi ring
        prec = name[len("rising_droplet_local_256c_"):] or "f32"
        return W.rising_droplet_3d(256, prec, scalar_grad="local")
    if name == "static_drop_64x64":
        return W.static_drop_64()
    raise SystemExit(f"unknown workload {name}")


def time_gpu(w, steps, warmup, graph=True):
    """Warm up, then time exactly `steps` steps back to back on the lattice's
    own stream, bracketed by a device synchronisation and HIP events on that
    stream.  With graph=True (and an even step count, so that a replay ends
    on the lattice the host expects) the steps are captured once in a HIP
    graph and the timed region is one replay of it: the launches then carry
    no host overhead between them.  Every step is one launch of the fused
    step kernel, so the region time over `steps` is that kernel's average
    launch duration (gaps included)."""
    import torch

    from paper_2402_15752_amd import cplb
    p = w["params"]
    stream = torch.cuda.Stream()
    lat = cplb.Lattice(p, stream=stream)
    lat.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    lat.step(warmup)
    n = int(p["nx"]) * int(p["ny"]) * int(p["nz"])
    use_graph = graph and steps % 2 == 0
    g = None
    if use_graph:
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            lat.step(steps)
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    if use_graph:
        with torch.cuda.stream(stream):
            g.replay()
    else:
        lat.step(steps)
    t_stop.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_stop)
    r = lat.reduce()
    if use_graph:
        r["step"] = warmup + steps  # the capture advanced the host counter once, the replay ran once
    lat.close()
    del g
    return dict(n=n, total_ms=total_ms, avg_kernel_ms=total_ms / steps, graph=use_graph, reduce=r)


def time_gpu_with_reduce(w, steps, warmup, every=100):
    """The same step loop with the FP64 reduction (phase and scalar masses,
    max |u|, kinetic energy, the non-finite check) every `every` steps, as a
    run that monitors its conservation would do.  Each reduction copies its
    eight values to the host and synchronises, so the region is timed on the
    host clock; the steps between reductions are one graph replay."""
    import torch

    from paper_2402_15752_amd import cplb
    assert every % 2 == 0 and steps % every == 0
    stream = torch.cuda.Stream()
    lat = cplb.Lattice(w["params"], stream=stream)
    lat.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    lat.step(warmup)
    n = int(w["params"]["nx"]) * int(w["params"]["ny"]) * int(w["params"]["nz"])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        lat.step(every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // every):
        with torch.cuda.stream(stream):
            g.replay()
        r = lat.reduce()
    dt = time.perf_counter() - t0
    lat.close()
    del g
    return dict(mlups=round(n * steps / dt / 1e6, 2), ms_per_step=round(dt * 1e3 / steps, 5),
                reduce_every=every, nonfinite=r["nonfinite"])


def time_batch(steps, warmup, tune_steps=5, tune=True):
    """The batched sweep: 512 independent 2-D cases (sizes 64..256 a side)
    advanced together, one launch per size class per step, the tile variant
    of each class picked by the autotuner (tune=False: the library's default
    per class, so that separate profiling runs time the same kernels);
    `steps` steps captured in a HIP graph and timed as one replay."""
    import torch

    import workloads as W
    from paper_2402_15752_amd import cplb
    sw = W.batched_sweep()
    stream = torch.cuda.Stream()
    b = cplb.Batch([c["params"] for c in sw["cases"]], stream=stream)
    for k, c in enumerate(sw["cases"]):
        b.init_sdf(k, c["sdf"], c1=c["init"]["c1"], c2=c["init"]["c2"])
    b.step(warmup)
    tuned_ms = b.tune(tune_steps) if tune else None
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        b.step(steps)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    with torch.cuda.stream(stream):
        g.replay()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    nonfinite = sum(b.reduce(k)["nonfinite"] for k in range(0, len(sw["cases"]), 37))
    classes = b.classes()
    b.close()
    del g
    n = sw["nodes"]
    per = ms / steps
    bpn = 328  # D2Q9 x 4 sets, FP32: 2 * 36 * 4 + 2 * 5 * 4
    gbs = bpn * n / (per * 1e-3) / 1e9
    return {"workload": sw["name"], "cases": len(sw["cases"]), "nodes": n, "steps": steps,
            "ms_per_step": round(per, 5), "mlups": round(n * steps / (ms * 1e-3) / 1e6, 1),
            "alg_bytes_per_node": bpn, "achieved_GBs": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "graph": True,
            "tuned_ms_per_step": round(tuned_ms, 4) if tuned_ms is not None else None,
            "classes": [{"cases": c, "variant": v} for c, v in classes],
            "pe_shifted_cases": len(sw["shifted"]), "nonfinite_sampled": nonfinite}


def closure_speedup():
    """The learned closure's side of the metric, on the 2-D rising bubble:
    coarse 128 x 512 against fine 512 x 2048 (F = 4), trained on the GPU from
    fine-grid runs of the plain method for 256 seeded parameter draws (one
    round, targets averaged over spans of 10 coarse steps), evaluated on 16
    held-out draws.  Reports the median (c1, c2) relative L2 error against the
    restricted fine run with and without the closure after 100 coarse steps
    (1600 fine steps), and the wall time of the closure-corrected coarse run
    against the fine run (same cases, same physical time); the errors after
    200 coarse steps are reported beside them."""
    import numpy as np

    from paper_2402_15752_amd import closure as CL
    r = CL.experiment(n_train=256, n_test=16, steps=100, nc=128, iters=(3000,), batch=16, seed=1,
                      kind="rising", every=10, skip=0, rounds=1, chunk=64)
    net = r.pop("net")
    ev = CL.evaluate(CL.draw_cases(16, seed=1001, nc=128, kind="rising"), steps=200, net=net)
    r["err_plain_coarse_200"] = float(np.median([c["plain"] for c in ev["cases"]]))
    r["err_closure_200"] = float(np.median([c["closure"] for c in ev["cases"]]))
    net.close()
    return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}


def cpu_model():
    """Name of the host CPU (first model name line of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(w, seconds=20.0):
    """The FP64 CPU oracle, untuned, on a bounded sample of the same workload:
    a fixed number of steps sized to ~10-30 s of CPU work, timed after two
    untimed steps (first touch of the arrays).  The rate is extrapolated to
    the workload's full run (w["steps"] steps) and stated as such."""
    from oracle import ref
    o = ref.Oracle(w["params"])
    o.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    n = int(w["params"]["nx"]) * int(w["params"]["ny"]) * int(w["params"]["nz"])
    o.step(2)  # first touch of the arrays, not timed
    t0 = time.perf_counter()
    o.step(1)
    per = time.perf_counter() - t0
    steps = max(2, min(20000, int(seconds / max(per, 1e-6))))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    o.close()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    full = int(w.get("steps", steps))
    return {"value": round(n * steps / dt / 1e6, 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{steps} steps of {w['name']} ({n} nodes) on the FP64 C oracle "
                      f"(gcc -O3 -march=x86-64-v3 -ffp-contract=off), OpenMP over {threads} "
                      f"threads, {dt:.1f} s; the full {full}-step run extrapolates to "
                      f"{dt / steps * full / 60:.1f} min"}


def cpu_baseline_one_thread(name, seconds=10.0):
    """The oracle on one thread (OMP_NUM_THREADS=1), in a child process that
    touches no GPU: the bounded sample of cpu_baseline, shorter."""
    import subprocess
    code = ("import json, sys; sys.path.insert(0, %r); import bench; "
            "print(json.dumps(bench.cpu_baseline(bench.make_workload(%r), %r)))"
            % (ROOT, name, seconds))
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def step_entry(name, steps, warmup):
    """Side measurement of one more step workload: graph-timed as the
    headline, algorithmic bytes, fraction of the HBM peak, measured traffic."""
    w = make_workload(name)
    r = time_gpu(w, steps, warmup)
    b = alg_bytes_per_node(w["params"])
    a = b * r["n"] / (r["avg_kernel_ms"] * 1e-3) / 1e9
    e = {"mlups": round(r["n"] * steps / (r["total_ms"] * 1e-3) / 1e6, 1),
         "avg_kernel_ms": round(r["avg_kernel_ms"], 5), "alg_bytes_per_node": b,
         "achieved_GBs": round(a, 1), "frac": round(a / HBM_PEAK_GBS, 4),
         "nonfinite": r["reduce"]["nonfinite"]}
    t = measured_traffic(w["name"])
    if t is not None:
        e["traffic_GBs"] = round(t / (r["avg_kernel_ms"] * 1e-3) / 1e9, 1)
    return w["name"], e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="rising_droplet_256c_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 3-D, batch and closure side measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (5 launches): the reference for "
                         "scaling FETCH_SIZE / WRITE_SIZE counters to bytes")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch part: keep the library's default tile per size class")
    ap.add_argument("--part", choices=("step", "batch", "closure"), default="step",
                    help="batch / closure: run only that side measurement and print its JSON "
                         "(for profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the step is "
              "built and measured on one GPU; across GPUs it would shard as slabs with one "
              "halo exchange per step, which is not built", file=sys.stderr)
        raise SystemExit(2)

    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")

    if args.part == "batch":
        print(json.dumps(time_batch(args.steps, args.warmup, tune=not args.no_tune)), flush=True)
        return
    if args.part == "closure":
        print(json.dumps(closure_speedup()), flush=True)
        return

    if args.copy_calibration:
        # a plain copy of known size: reads and writes exactly 1 GiB per launch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = make_workload(args.workload)
    p = w["params"]
    res = time_gpu(w, args.steps, args.warmup)
    n = res["n"]
    mlups = n * args.steps / (res["total_ms"] * 1e-3) / 1e6
    bpn = alg_bytes_per_node(p)
    achieved = bpn * n / (res["avg_kernel_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(w["name"])
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["total_ms"] / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if p["precision"] != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "lattice": p["lattice"],
                   "grid": [p["nx"], p["ny"], p["nz"]], "precision": p["precision"],
                   "boundaries": "periodic x, bounce-back walls y" if p["lattice"] == "d2q9"
                   else "periodic x y, bounce-back walls z"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else
                     round(traffic / (res["avg_kernel_ms"] * 1e-3) / 1e9, 1)},
        "kernel": {"avg_ms": round(res["avg_kernel_ms"], 5), "alg_bytes_per_node": bpn,
                   "alg_bytes_per_launch": bpn * n, "traffic_bytes_per_launch": traffic,
                   "source_hash": kernel_source_hash(), "graph": res["graph"]},
    }
    r = res["reduce"]
    out["check"] = {"nonfinite": r["nonfinite"], "sum_phi": r["sum_phi"], "step": r["step"]}
    if not args.no_extra:
        # the same workload and window with the FP64 reduction every 100 steps
        # (every K steps when the window is shorter)
        every = 100 if args.steps % 100 == 0 else args.steps
        wr = time_gpu_with_reduce(w, args.steps, args.warmup, every=every)
        wr["overhead"] = round(wr["ms_per_step"] / out["ms_per_step"] - 1.0, 4)
        out["with_reduce"] = wr
        also = {}
        for name, steps in (("rising_droplet_256c_f32_s16f", 100), ("rising_droplet_256c_f32_s16b", 100),
                            ("rising_droplet_local_256c_f32", 100),
                            ("rising_droplet_local_256c_f32_s16f", 100),
                            ("rising_bubble_256x1024", 2000), ("rising_bubble_local_256x1024", 2000),
                            ("rising_bubble_2048x4096", 200), ("rising_bubble_local_2048x4096", 200),
                            ("rising_bubble_one_256x1024", 2000)):
            if name == w["name"]:
                continue
            key, e = step_entry(name, steps, 10 if steps <= 200 else 100)
            also[key] = e
        out["also"] = also
        out["also_batch_512"] = time_batch(40, 5)
        out["closure"] = closure_speedup()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
        one = cpu_baseline_one_thread(args.workload)
        out["cpu_baseline"]["one_thread_value"] = one["value"]
        out["cpu_baseline"]["one_thread_sample"] = one["sample"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
