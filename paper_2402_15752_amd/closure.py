"""Learned closure of the interfacial scalar exchange on a coarse grid.

The plain method resolves the interface with W = 4 lattice spacings.  A
coarse grid F times coarser in space (F^2 in time: diffusive scaling, so
D_k, M and the viscosity keep their lattice values and A scales as 1/dx^2)
resolves the same physical interface with 4 coarse spacings where the fine
grid uses 4 F; its scalar transfer across the interface then carries a
discretisation error.  The closure network (cplb_cnn_*) predicts, from the
coarse fields and the case's transport parameters, a per-node exchange s
that the coarse step applies through cplb_set_closure / the batch closure
(h1 loses w_i s, h2 gains it: c1 + c2 stays exactly conserved).

Training data are fine-grid runs of the plain method next to free coarse
runs of the same cases: the fine fields are restricted (F x F block
averages) to the coarse grid at every coarse time level, and the target is
the exchange part of the growth of the coarse-minus-fine scalar error over
one coarse step (see ``generate``).  Evaluation runs held-out cases freely
on the coarse grid, with and without the network, and compares c1, c2 with
the restricted fine run; the fine run stays the reference and the
fallback.

Every step of this runs in the library's kernels: fine and coarse steps
(batched), field gathers, restriction, initialisation from device planes,
the network's forward / backward / Adam.  torch supplies device memory,
streams, minibatch index gathers and graph capture.
"""
from __future__ import annotations

import time

import numpy as np

import workloads as W
from . import cplb

F = 4                      # coarse / fine spacing ratio
FIELDS = ("phi", "c1", "c2")
N_PARAM_PLANES = 4         # log Keq, D1, D2, A (coarse lattice units)
N_PLANES = len(FIELDS) + N_PARAM_PLANES
INPUT_SCALE = (1.0, 1.0, 1.0, 1.0, 10.0, 10.0, 10.0)


def draw_cases(n, seed, nc=64, precision="f32"):
    """n static-drop transfer cases: coarse nc x nc and fine F nc x F nc
    periodic grids with the same physical drop, interface, diffusivities,
    partition coefficient and exchange rate.  Keq log-uniform in [0.2, 5],
    D1, D2 log-uniform in [0.01, 0.15], coarse A log-uniform in [0.02, 0.2],
    coarse radius uniform in [nc/8, nc/4.5], centre jittered; c1 = 0 and
    c2 = 1 - phi0 (the solute starts in the drop, fluid 2)."""
    rng = np.random.default_rng(seed)

    def loguni(a, b):
        return float(np.exp(rng.uniform(np.log(a), np.log(b))))

    cases = []
    for _ in range(n):
        keq = loguni(0.2, 5.0)
        d1, d2 = loguni(0.01, 0.15), loguni(0.01, 0.15)
        a_c = loguni(0.02, 0.2)
        r_c = float(rng.uniform(nc / 8.0, nc / 4.5))
        cx, cy = nc / 2.0 + rng.uniform(-2, 2), nc / 2.0 + rng.uniform(-2, 2)
        common = dict(lattice="d2q9", visc_law="linear", periodic=(1, 1, 1), rho1=1.0, rho2=1.0,
                      mu1=0.1, mu2=0.1, sigma=1e-3, M=0.01, D1=d1, D2=d2, Keq=keq,
                      precision=precision, ref_f=W.phase_reference(precision))
        pc = W.params(nx=nc, ny=nc, W=4.0, A=a_c, n_eps=1e-3, **common)
        pf = W.params(nx=F * nc, ny=F * nc, W=4.0 * F, A=a_c / F ** 2, n_eps=1e-3 / F, **common)
        # coarse node i is the block of fine nodes F i .. F i + F - 1
        lc = W.sdf_sphere(pc, (cx, cy), r_c, inside_positive=False)
        off = (F - 1) / 2.0
        lf = W.sdf_sphere(pf, (F * cx + off, F * cy + off), F * r_c, inside_positive=False)
        cases.append(dict(coarse=pc, fine=pf, sdf_c=lc, sdf_f=lf, keq=keq, d1=d1, d2=d2, a=a_c))
    return cases


def param_planes(cases, torch, device, nc):
    """[n, N_PARAM_PLANES, nc, nc] constant planes of the transport parameters."""
    v = np.array([[np.log(c["keq"]), c["d1"], c["d2"], c["a"]] for c in cases], dtype=np.float32)
    t = torch.tensor(v, device=device)[:, :, None, None].expand(-1, -1, nc, nc)
    return t.contiguous()


class Runner:
    """Fine and coarse batches of the same cases on one stream."""

    def __init__(self, cases, stream=None):
        import torch
        self.torch = torch
        self.cases = cases
        self.n = len(cases)
        self.nc = cases[0]["coarse"]["nx"]
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.fine = cplb.Batch([c["fine"] for c in cases], stream=self.stream)
        self.coarse = cplb.Batch([c["coarse"] for c in cases], stream=self.stream)
        for k, c in enumerate(cases):
            self.fine.init_sdf(k, c["sdf_f"], c1=(0.0, 0.0), c2=(1.0, -1.0))
        dev = self.fine.device
        nc = self.nc
        self.fine_buf = torch.empty(self.n * 3 * (F * nc) ** 2, dtype=torch.float32, device=dev)
        self.planes = torch.zeros(self.n, N_PLANES, nc, nc, dtype=torch.float32, device=dev)
        self.planes[:, len(FIELDS):] = param_planes(cases, torch, dev, nc)
        self.coarse_buf = torch.empty(self.n * N_PLANES * nc * nc, dtype=torch.float32, device=dev)

    def restricted_fine(self, out):
        """Restricted fine phi, c1, c2 of every case into out [n, 3, nc, nc]."""
        nc, nf = self.nc, F * self.nc
        f = self.fine.gather(FIELDS, out=self.fine_buf)
        with self.torch.cuda.stream(self.stream):
            cplb.restrict(f.view(self.n * 3, nf, nf), F, out=out.view(self.n * 3, nc, nc),
                          stream=self.stream)
        return out

    def coarse_from(self, planes):
        """Coarse cases initialised from planes [n, N_PLANES, nc, nc] (phi, c1, c2 first)."""
        self.coarse.init_planes(planes.view(-1), N_PLANES, 0, 1, 2)


def generate(cases, steps, stream=None, log=None, net=None, skip=5):
    """Training samples of `cases` over `steps` coarse steps:
    inputs [n steps, N_PLANES, nc, nc], targets [n steps, nc, nc].

    The coarse batch runs freely next to the fine batch (one coarse step per
    F^2 fine steps) from the restricted fine initial state; with `net` it
    runs with that closure (a second round on the states the closure itself
    produces).  E_k = coarse(t_k) - restricted fine(t_k) for c1 and c2; the
    target is the exchange part of its growth over one coarse step,
    s_k = (dE_c1 - dE_c2) / 2 with dE = E_k+1 - E_k: the per-node exchange
    that, applied at step k, removes as much of the new error as an
    exchange (h1 -> h2, c1 + c2 kept) can.  With the closure running, the
    exchange it applied at step k is added: the target stays the whole
    exchange, not the residual.  Inputs are the coarse state at
    t_k, as the closure sees it when it runs.  The first `skip` steps are
    dropped."""
    import torch
    R = Runner(cases, stream)
    n, nc = R.n, R.nc
    dev = R.fine.device
    X = torch.empty(steps, n, N_PLANES, nc, nc, dtype=torch.float32, device=dev)
    Y = torch.empty(steps, n, nc, nc, dtype=torch.float32, device=dev)
    fine = torch.empty(n, 3, nc, nc, dtype=torch.float32, device=dev)
    R.restricted_fine(fine)
    with torch.cuda.stream(R.stream):
        R.planes[:, :3] = fine
    R.coarse_from(R.planes)
    s = None
    if net is not None:
        s = torch.zeros(n * nc * nc, dtype=torch.float32, device=dev)
        R.coarse.set_closure(s)
        net.set_stream(R.stream)
    x = R.coarse.gather(FIELDS, out=R.coarse_buf, nplanes=N_PLANES)
    with torch.cuda.stream(R.stream):
        x[:, len(FIELDS):] = R.planes[:, len(FIELDS):]
        err = x[:, 1:3] - fine[:, 1:3]
    t0 = time.perf_counter()
    for k in range(steps):
        with torch.cuda.stream(R.stream):
            X[k] = x
        if net is not None:
            net.infer(x, out=s.view(n, nc, nc))
        R.coarse.step(1)
        R.fine.step(F * F)
        R.restricted_fine(fine)
        x = R.coarse.gather(FIELDS, out=R.coarse_buf, nplanes=N_PLANES)
        with torch.cuda.stream(R.stream):
            e_new = x[:, 1:3] - fine[:, 1:3]
            d = e_new - err
            Y[k] = 0.5 * (d[:, 0] - d[:, 1])
            if s is not None:
                # the exchange already applied is part of the one wanted
                Y[k] += s.view(n, nc, nc)
            err = e_new
        if log and (k + 1) % max(1, steps // 4) == 0:
            torch.cuda.synchronize()
            log(f"  data: {k + 1}/{steps} coarse steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    R.coarse.set_closure(None)
    # the first `skip` steps carry the start-up of the coarse run from the
    # restricted fine state (its populations start at equilibrium), not the
    # per-step transfer error the closure is for
    X, Y = X[skip:], Y[skip:]
    return (X.reshape((steps - skip) * n, N_PLANES, nc, nc),
            Y.reshape((steps - skip) * n, nc, nc))


def train(X, Y, iters=1500, batch=32, lr=2e-3, seed=0, log=None, net=None, capacity=64,
          scale=None):
    """Fit the closure network to (X, Y) on the GPU (minibatch Adam, FP64 loss).
    Returns (net, scale, losses); the network learns Y / scale (scale: the
    standard deviation of Y unless given, as when training continues) and
    its output is scaled back by `scale`.  The network is built for up to
    max(batch, capacity) samples per call (the coarse cases it will drive at
    once)."""
    import torch
    ns, nc = X.shape[0], X.shape[-1]
    if scale is None:
        scale = float(Y.std().item()) or 1.0
    Yn = (Y / scale).contiguous()
    if net is None:
        net = cplb.ClosureNet(max(batch, capacity), nc, nc, seed=seed + 1)
    net.set_input_scale(INPUT_SCALE)
    net.set_output_scale(1.0)
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    losses = []
    for it in range(iters):
        idx = torch.randint(0, ns, (batch,), device=X.device, generator=g)
        xb = X.index_select(0, idx).contiguous()
        yb = Yn.index_select(0, idx).contiguous()
        net.forward(xb)
        losses.append(net.backward(yb))
        net.adam(lr=lr * (0.1 if it > 0.8 * iters else 1.0))
        if log and (it + 1) % max(1, iters // 5) == 0:
            log(f"  train: iter {it + 1}/{iters} loss {np.mean(losses[-50:]):.4e}")
    net.set_output_scale(scale)
    return net, scale, losses


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def evaluate(cases, steps, net=None, stream=None, log=None):
    """Free coarse runs of `cases` for `steps` coarse steps, plain and with
    the closure network, against the restricted fine run of F^2 steps each.
    Returns per-case scalar errors and wall times (the fine run from the
    library's own step loop, the coarse runs replayed from HIP graphs; one
    synchronisation at the end of each run)."""
    import torch
    R = Runner(cases, stream)
    n, nc = R.n, R.nc
    init = torch.empty(n, 3, nc, nc, dtype=torch.float32, device=R.fine.device)
    R.restricted_fine(init)
    with torch.cuda.stream(R.stream):
        R.planes[:, :3] = init
    planes0 = R.planes.clone()
    torch.cuda.synchronize()

    # fine reference
    t0 = time.perf_counter()
    R.fine.step(F * F * steps)
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    ref = torch.empty_like(init)
    R.restricted_fine(ref)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()

    # a captured graph replays its steps from the lattice parity it was
    # captured at: whole graphs of an even number of steps keep it
    assert steps % 2 == 0, "evaluate needs an even number of coarse steps"

    def run(with_net, chunk=10):
        # `chunk` coarse steps (gather, network, step) captured once in a HIP
        # graph on the runner's stream and replayed: the wall time is that
        # of the GPU work, not of the Python launches
        R.coarse_from(planes0)
        s = None
        if with_net:
            s = torch.zeros(n * nc * nc, dtype=torch.float32, device=R.fine.device)
            R.coarse.set_closure(s)
            net.set_stream(R.stream)
        else:
            R.coarse.set_closure(None)
        x = R.coarse.gather(FIELDS, out=R.coarse_buf, nplanes=N_PLANES)
        with torch.cuda.stream(R.stream):
            x[:, len(FIELDS):] = planes0[:, len(FIELDS):]

        def steps_of(k):
            for _ in range(k):
                if with_net:
                    R.coarse.gather(FIELDS, out=R.coarse_buf, nplanes=N_PLANES)
                    net.infer(x, out=s.view(n, nc, nc))
                R.coarse.step(1)

        graphs = {}
        for k in {chunk, steps % chunk} - {0}:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=R.stream):
                steps_of(k)
            graphs[k] = g
        # capturing ran nothing: restart from the initial state
        R.coarse_from(planes0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        with torch.cuda.stream(R.stream):
            for _ in range(steps // chunk):
                graphs[chunk].replay()
            if steps % chunk:
                graphs[steps % chunk].replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out = R.coarse.gather(FIELDS).cpu().numpy()
        R.coarse.set_closure(None)
        del graphs
        return out, dt

    plain, t_plain = run(False)
    closed, t_closed = (run(True) if net is not None else (None, 0.0))
    res = []
    for k in range(n):
        e_plain = rel_l2(plain[k, 1:3], ref[k, 1:3])
        e_closed = rel_l2(closed[k, 1:3], ref[k, 1:3]) if closed is not None else None
        res.append(dict(plain=e_plain, closure=e_closed))
    out = dict(cases=res, t_fine=t_fine, t_coarse=t_plain, t_closure=t_closed,
               fine_nodes=n * (F * nc) ** 2, coarse_nodes=n * nc * nc, steps=steps)
    if log:
        ep = np.median([r["plain"] for r in res])
        msg = f"  eval: median c rel L2 plain {ep:.3e}"
        if closed is not None:
            msg += f", closure {np.median([r['closure'] for r in res]):.3e}"
        log(msg + f"; fine {t_fine * 1e3:.1f} ms, coarse {t_plain * 1e3:.1f} ms, "
                  f"coarse + closure {t_closed * 1e3:.1f} ms")
    return out


def experiment(n_train=64, n_test=16, steps=200, nc=64, iters=(3000, 2000), batch=32, seed=1,
               log=None):
    """Draw cases, train the closure in two rounds (on plain coarse runs,
    then on runs with the closure itself), and evaluate it on held-out cases
    against the fine grid.  Returns a summary: median scalar errors (c1, c2
    relative L2 against the restricted fine run) with and without the
    closure, wall times of the fine, plain coarse and closure-corrected
    coarse runs (`steps` coarse steps, F^2 fine steps each), training time
    and losses."""
    import torch
    t0 = time.perf_counter()
    train_cases = draw_cases(n_train, seed=seed, nc=nc)
    test_cases = draw_cases(n_test, seed=seed + 1000, nc=nc)
    X, Y = generate(train_cases, steps=steps, log=log)
    net, scale, l1 = train(X, Y, iters=iters[0], batch=batch, seed=seed, log=log,
                           capacity=max(n_train, n_test))
    X2, Y2 = generate(train_cases, steps=steps, net=net)
    net, _, l2 = train(torch.cat([X, X2]), torch.cat([Y, Y2]), iters=iters[1], batch=batch,
                       seed=seed + 1, log=log, net=net, scale=scale)
    del X, Y, X2, Y2
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ev = evaluate(test_cases, steps=steps, net=net, log=log)
    ep = float(np.median([r["plain"] for r in ev["cases"]]))
    ec = float(np.median([r["closure"] for r in ev["cases"]]))
    wins = sum(r["closure"] < r["plain"] for r in ev["cases"])
    return dict(
        train_cases=n_train, test_cases=n_test, coarse_grid=[nc, nc], fine_grid=[F * nc, F * nc],
        coarse_steps=steps, fine_steps=F * F * steps,
        err_plain_coarse=ep, err_closure=ec, closure_better_cases=int(wins),
        t_fine_ms=ev["t_fine"] * 1e3, t_coarse_ms=ev["t_coarse"] * 1e3,
        t_closure_ms=ev["t_closure"] * 1e3,
        speedup_closure_vs_fine=ev["t_fine"] / max(ev["t_closure"], 1e-12),
        train_s=t_train, loss_first=float(np.mean(l1[:50])), loss_round1=float(np.mean(l1[-50:])),
        loss_last=float(np.mean(l2[-50:])),
        net=net)
