"""Learned closure of the interfacial scalar transfer on a coarse grid.

The plain method resolves the interface with W = 4 lattice spacings.  A
coarse grid F times coarser in space (F^2 in time: diffusive scaling, so
D_k, M and the viscosity keep their lattice values, A scales as 1/dx^2, the
surface tension as 1/dx and gravity as 1/dx^3) resolves the same physical
interface with 4 coarse spacings where the fine grid uses 4 F; its scalar
transfer across the interface then carries a discretisation error.  The
closure network (cplb_cnn_*) predicts, from the coarse fields and the
case's transport parameters, per-node corrections (x1, x2) of c1 and c2
that the coarse step applies through cplb_set_closure / the batch closure:
each step lowers the node's c_k by x_k (carried by the scalar populations
like the auxiliary source, through the inverse of the implicit recovery's
Jacobian).  x1 - x2 is an exchange between the phases; x1 + x2 moves
solute, and the network's output is balanced per case so that the
corrections add nothing to the case's total: c1 + c2 stays exactly
conserved overall.

Two families of cases:
  "static"  periodic static drops, nc x nc coarse against F nc x F nc fine;
  "rising"  the walled 2-D rising bubble (density ratio 10, viscosity ratio
            10 under the exponential law, Eo = 10), nc x 4 nc coarse against
            F nc x 4 F nc fine, solute starting in the bubble.

Training data are fine-grid runs of the plain method next to free coarse
runs of the same cases: the fine fields are restricted (F x F block
averages) to the coarse grid, and the target is the exchange part of the
growth of the coarse-minus-fine scalar error per coarse step, averaged over
a span of steps (see ``generate``).  Evaluation runs held-out cases freely on the coarse grid,
with and without the network, and compares c1, c2 with the restricted fine
run; the fine run stays the reference and the fallback.

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


def draw_cases(n, seed, nc=64, precision="f32", kind="static"):
    """n transfer cases with the same physics on a coarse grid and on a grid F
    times finer.  Drawn per case: Keq log-uniform in [0.2, 5], D1, D2
    log-uniform in [0.01, 0.15], coarse A log-uniform in [0.02, 0.2]; the
    solute starts in the drop / bubble (fluid 2): c1 = 0, c2 = 1 - phi0.

    kind "static": nc x nc periodic, matched densities, drop radius uniform in
    [nc/8, nc/4.5], centre jittered.
    kind "rising": nc x 4 nc, periodic in x, walls in y, gravity along -y;
    bubble of radius nc/16 at (nc/2, 3 nc/8), centre jittered; density
    ratio 10, exponential viscosity law with mu1 = 2, mu2 = 0.1, Eo = 10 and
    sigma = 0.01 on the coarse grid.

    Fine-grid parameters follow diffusive scaling: W, radius and positions
    times F; A / F^2; n_eps / F; sigma / F and g / F^3 (so the Laplace
    pressure and the buoyancy keep their ratio to the viscous scales); D, M
    and the viscosities unchanged in lattice units."""
    rng = np.random.default_rng(seed)

    def loguni(a, b):
        return float(np.exp(rng.uniform(np.log(a), np.log(b))))

    cases = []
    for _ in range(n):
        keq = loguni(0.2, 5.0)
        d1, d2 = loguni(0.01, 0.15), loguni(0.01, 0.15)
        a_c = loguni(0.02, 0.2)
        common = dict(lattice="d2q9", M=0.01, D1=d1, D2=d2, Keq=keq, precision=precision,
                      ref_f=W.phase_reference(precision))
        if kind == "static":
            ncx = ncy = nc
            r_c = float(rng.uniform(nc / 8.0, nc / 4.5))
            cx, cy = nc / 2.0 + rng.uniform(-2, 2), nc / 2.0 + rng.uniform(-2, 2)
            hyd = dict(visc_law="linear", periodic=(1, 1, 1), rho1=1.0, rho2=1.0, mu1=0.1,
                       mu2=0.1)
            sig_c, g_c = 1e-3, 0.0
        elif kind == "rising":
            ncx, ncy = nc, 4 * nc
            r_c = nc / 16.0
            cx, cy = nc / 2.0 + rng.uniform(-1, 1), 3.0 * nc / 8.0 + rng.uniform(-1, 1)
            rho1, rho2, eo = 10.0, 1.0, 10.0
            sig_c = 0.01
            g_c = eo * sig_c / ((rho1 - rho2) * (2 * r_c) ** 2)
            hyd = dict(visc_law="exp", periodic=(1, 0, 1), rho1=rho1, rho2=rho2, mu1=2.0, mu2=0.1,
                       rho_ref=rho1)
        else:
            raise ValueError(kind)
        pc = W.params(nx=ncx, ny=ncy, W=4.0, A=a_c, n_eps=1e-3, sigma=sig_c,
                      g=(0.0, -g_c, 0.0), **hyd, **common)
        pf = W.params(nx=F * ncx, ny=F * ncy, W=4.0 * F, A=a_c / F ** 2, n_eps=1e-3 / F,
                      sigma=sig_c / F, g=(0.0, -g_c / F ** 3, 0.0), **hyd, **common)
        # coarse node i is the block of fine nodes F i .. F i + F - 1
        lc = W.sdf_sphere(pc, (cx, cy), r_c, inside_positive=False)
        off = (F - 1) / 2.0
        lf = W.sdf_sphere(pf, (F * cx + off, F * cy + off), F * r_c, inside_positive=False)
        cases.append(dict(coarse=pc, fine=pf, sdf_c=lc, sdf_f=lf, keq=keq, d1=d1, d2=d2, a=a_c,
                          kind=kind))
    return cases


def param_planes(cases, torch, device, ny, nx):
    """[n, N_PARAM_PLANES, ny, nx] constant planes of the transport parameters."""
    v = np.array([[np.log(c["keq"]), c["d1"], c["d2"], c["a"]] for c in cases], dtype=np.float32)
    t = torch.tensor(v, device=device)[:, :, None, None].expand(-1, -1, ny, nx)
    return t.contiguous()


class Runner:
    """Fine and coarse batches of the same cases on one stream.  Every tensor
    the runner's work touches is allocated and filled on that stream (so no
    fill on another stream can land after the work that reads it)."""

    def __init__(self, cases, stream=None):
        import torch
        self.torch = torch
        self.cases = cases
        self.n = len(cases)
        self.ny, self.nx = cases[0]["coarse"]["ny"], cases[0]["coarse"]["nx"]
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.fine = cplb.Batch([c["fine"] for c in cases], stream=self.stream)
        self.coarse = cplb.Batch([c["coarse"] for c in cases], stream=self.stream)
        for k, c in enumerate(cases):
            self.fine.init_sdf(k, c["sdf_f"], c1=(0.0, 0.0), c2=(1.0, -1.0))
        dev = self.fine.device
        ny, nx = self.ny, self.nx
        with torch.cuda.stream(self.stream):
            self.fine_buf = torch.empty(self.n * 3 * F * F * ny * nx, dtype=torch.float32,
                                        device=dev)
            self.planes = torch.zeros(self.n, N_PLANES, ny, nx, dtype=torch.float32, device=dev)
            self.planes[:, len(FIELDS):] = param_planes(cases, torch, dev, ny, nx)
            self.coarse_buf = torch.empty(self.n * N_PLANES * ny * nx, dtype=torch.float32,
                                          device=dev)

    def restricted_fine(self, out):
        """Restricted fine phi, c1, c2 of every case into out [n, 3, ny, nx]."""
        ny, nx = self.ny, self.nx
        f = self.fine.gather(FIELDS, out=self.fine_buf)
        with self.torch.cuda.stream(self.stream):
            cplb.restrict(f.view(self.n * 3, F * ny, F * nx), F, out=out.view(self.n * 3, ny, nx),
                          stream=self.stream)
        return out

    def coarse_from(self, planes):
        """Coarse cases initialised from planes [n, N_PLANES, ny, nx] (phi, c1, c2 first)."""
        self.coarse.init_planes(planes.view(-1), N_PLANES, 0, 1, 2)

    def close(self):
        self.fine.close()
        self.coarse.close()


def generate(cases, steps, stream=None, log=None, net=None, skip=5, every=1):
    """Training samples of `cases` over `steps` coarse steps:
    inputs [samples, N_PLANES, ny, nx], targets [samples, 2, ny, nx].

    The coarse batch runs freely next to the fine batch (one coarse step per
    F^2 fine steps) from the restricted fine initial state; with `net` it
    runs with that closure (a second round on the states the closure itself
    produces).  E = coarse - restricted fine for c1 and c2.  Samples start
    at steps k = skip, skip + every, ...; each covers the span of `every`
    coarse steps that follows: the input is the coarse state at k, as the
    closure sees it when it runs, and the target the growth of E over the
    span divided by its length -- the per-step corrections (c_k loses s_k)
    that would have removed it.  Averaging over a span keeps the part of
    the growth that the coarse state predicts and averages out what it does
    not.  With the closure running, the corrections it applied over the
    span (per step, on average) are added: the target stays the whole
    correction, not the residual.  The first `skip` steps carry the
    start-up of the coarse run from the restricted fine state (populations
    at equilibrium), not the transfer error the closure is for."""
    import torch
    R = Runner(cases, stream)
    n, ny, nx = R.n, R.ny, R.nx
    dev = R.fine.device
    ks = list(range(skip, steps - every + 1, every))
    s = acc = None
    with torch.cuda.stream(R.stream):
        X = torch.empty(len(ks), n, N_PLANES, ny, nx, dtype=torch.float32, device=dev)
        Y = torch.empty(len(ks), n, 2, ny, nx, dtype=torch.float32, device=dev)
        fine = torch.empty(n, 3, ny, nx, dtype=torch.float32, device=dev)
        if net is not None:
            s = torch.zeros(n, 2, ny, nx, dtype=torch.float32, device=dev)
            acc = torch.zeros_like(s)
    R.restricted_fine(fine)
    with torch.cuda.stream(R.stream):
        R.planes[:, :3] = fine
    R.coarse_from(R.planes)
    if net is not None:
        R.coarse.set_closure(s)
        net.set_stream(R.stream)
    t0 = time.perf_counter()
    j, err, end = 0, None, -1
    take = set(ks)
    for k in range(steps):
        if k in take or net is not None:
            x = R.coarse.gather(FIELDS, out=R.coarse_buf, nplanes=N_PLANES)
            with torch.cuda.stream(R.stream):
                x[:, len(FIELDS):] = R.planes[:, len(FIELDS):]
        if net is not None:
            net.infer(x, out=s)
        if k in take:
            R.restricted_fine(fine)
            with torch.cuda.stream(R.stream):
                X[j] = x
                err = x[:, 1:3] - fine[:, 1:3]
                if acc is not None:
                    acc.zero_()
            end = k + every
        if acc is not None and err is not None:
            with torch.cuda.stream(R.stream):
                acc += s
        R.coarse.step(1)
        R.fine.step(F * F)
        if err is not None and k + 1 == end:
            R.restricted_fine(fine)
            xn = R.coarse.gather(FIELDS, out=R.coarse_buf, nplanes=N_PLANES)
            with torch.cuda.stream(R.stream):
                d = (xn[:, 1:3] - fine[:, 1:3]) - err
                Y[j] = d / every
                if acc is not None:
                    # the corrections already applied are part of the ones wanted
                    Y[j] += acc / every
            j += 1
            err = None
        if log and (k + 1) % max(1, steps // 4) == 0:
            torch.cuda.synchronize()
            log(f"  data: {k + 1}/{steps} coarse steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    R.coarse.set_closure(None)
    R.close()
    return X.reshape(len(ks) * n, N_PLANES, ny, nx), Y.reshape(len(ks) * n, 2, ny, nx)


def train(X, Y, iters=1500, batch=32, lr=2e-3, seed=0, log=None, net=None, capacity=64,
          scale=None, held=None):
    """Fit the closure network to (X, Y) on the GPU (minibatch Adam, FP64 loss).
    Returns (net, scale, losses, held_losses); the network learns Y / scale
    per output (scale: the standard deviations of Y[:, 0] and Y[:, 1] unless
    given, as when training continues) and its outputs are scaled back by
    `scale`.  `held`, an (X, Y)
    pair of samples of other cases, gives the held-out loss (normalised the
    same way) every iters / 10 iterations.  The network is built for up to
    max(batch, capacity) samples per call (the coarse cases it will drive at
    once)."""
    import torch
    ns, ny, nx = X.shape[0], X.shape[-2], X.shape[-1]
    if scale is None:
        scale = tuple(float(Y[:, c].double().std().item()) or 1.0 for c in range(2))
    if not all(np.isfinite(v) and v > 0 for v in scale):
        raise ValueError(f"closure targets have no finite spread: scales {scale}")
    sc = torch.tensor(scale, dtype=torch.float32, device=Y.device)[None, :, None, None]
    Yn = (Y / sc).contiguous()
    if net is None:
        net = cplb.ClosureNet(max(batch, capacity), ny, nx, seed=seed + 1)
    net.set_input_scale(INPUT_SCALE)
    net.set_output_scale(1.0)
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    losses, held_losses = [], []

    def held_loss():
        hx, hy = held
        tot = 0.0
        for a in range(0, hx.shape[0] - batch + 1, batch):
            net.forward(hx[a:a + batch].contiguous())
            # the loss of the last forward (the gradients it also forms are not applied)
            tot += net.backward((hy[a:a + batch] / sc).contiguous())
        return tot / max(1, hx.shape[0] // batch)

    for it in range(iters):
        idx = torch.randint(0, ns, (batch,), device=X.device, generator=g)
        xb = X.index_select(0, idx).contiguous()
        yb = Yn.index_select(0, idx).contiguous()
        net.forward(xb)
        losses.append(net.backward(yb))
        net.adam(lr=lr * (0.1 if it > 0.8 * iters else 1.0))
        if held is not None and (it + 1) % max(1, iters // 10) == 0:
            held_losses.append((it + 1, held_loss()))
        if log and (it + 1) % max(1, iters // 5) == 0:
            msg = f"  train: iter {it + 1}/{iters} loss {np.mean(losses[-50:]):.4e}"
            if held_losses:
                msg += f" held-out {held_losses[-1][1]:.4e}"
            log(msg)
    net.set_output_scale(*scale)
    return net, scale, losses, held_losses


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def evaluate(cases, steps, net=None, stream=None, log=None):
    """Free coarse runs of `cases` for `steps` coarse steps, plain and with
    the closure network, against the restricted fine run of F^2 steps each.
    Returns per-case scalar errors and wall times (the fine run from the
    library's own step loop, the coarse runs replayed from HIP graphs; one
    synchronisation at the end of each run).  Both batches are tuned first
    (tile variant per size class, state unchanged), so each side of the
    speedup runs its fastest kernels."""
    import torch
    R = Runner(cases, stream)
    R.fine.tune(5)
    R.coarse.tune(5)
    n, ny, nx = R.n, R.ny, R.nx
    with torch.cuda.stream(R.stream):
        init = torch.empty(n, 3, ny, nx, dtype=torch.float32, device=R.fine.device)
    R.restricted_fine(init)
    with torch.cuda.stream(R.stream):
        R.planes[:, :3] = init
        # on the runner's stream, after the copy above
        planes0 = R.planes.clone()
    torch.cuda.synchronize()

    # fine reference
    t0 = time.perf_counter()
    R.fine.step(F * F * steps)
    torch.cuda.synchronize()
    t_fine = time.perf_counter() - t0
    with torch.cuda.stream(R.stream):
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
            with torch.cuda.stream(R.stream):
                s = torch.zeros(n, 2, ny, nx, dtype=torch.float32, device=R.fine.device)
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
                    net.infer(x, out=s)
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
    R.close()
    res = []
    for k in range(n):
        e_plain = rel_l2(plain[k, 1:3], ref[k, 1:3])
        e_closed = rel_l2(closed[k, 1:3], ref[k, 1:3]) if closed is not None else None
        res.append(dict(plain=e_plain, closure=e_closed))
    out = dict(cases=res, t_fine=t_fine, t_coarse=t_plain, t_closure=t_closed,
               fine_nodes=n * F * F * ny * nx, coarse_nodes=n * ny * nx, steps=steps)
    if log:
        ep = np.median([r["plain"] for r in res])
        msg = f"  eval: median c rel L2 plain {ep:.3e}"
        if closed is not None:
            msg += f", closure {np.median([r['closure'] for r in res]):.3e}"
        log(msg + f"; fine {t_fine * 1e3:.1f} ms, coarse {t_plain * 1e3:.1f} ms, "
                  f"coarse + closure {t_closed * 1e3:.1f} ms")
    return out


def generate_chunked(cases, steps, chunk, log=None, net=None, every=1, skip=5):
    """generate() over the cases `chunk` at a time (the fine batch of every
    chunk is resident only while it runs); samples of all chunks, concatenated."""
    import torch
    Xs, Ys = [], []
    for a in range(0, len(cases), chunk):
        X, Y = generate(cases[a:a + chunk], steps=steps, net=net, every=every, skip=skip,
                        log=log if a == 0 else None)
        if not (bool(torch.isfinite(X).all()) and bool(torch.isfinite(Y).all())):
            raise RuntimeError(f"closure data of cases {a}..{a + len(X) - 1}: non-finite values")
        Xs.append(X)
        Ys.append(Y)
        if log and len(cases) > chunk:
            log(f"  data: cases {a + len(cases[a:a + chunk])}/{len(cases)}")
    return (Xs[0], Ys[0]) if len(Xs) == 1 else (torch.cat(Xs), torch.cat(Ys))


def experiment(n_train=64, n_test=16, steps=200, nc=64, iters=(3000, 2000), batch=32, seed=1,
               kind="static", every=1, gen_steps=None, n_held=8, chunk=64, skip=5, rounds=2,
               log=None):
    """Draw cases, train the closure in one or two rounds (on plain coarse
    runs, then on runs with the closure itself), and evaluate it on held-out
    cases against the fine grid.  Data generation runs `gen_steps` coarse steps
    (default `steps`), `chunk` cases at a time, with targets averaged over
    spans of `every` steps; `n_held` further cases give the held-out loss
    during training.  Returns a summary: median scalar errors (c1, c2
    relative L2 against the restricted fine run) with and without the
    closure, wall times of the fine, plain coarse and closure-corrected
    coarse runs (`steps` coarse steps, F^2 fine steps each), the times of data
    generation and of training (a second round's data included), training
    and held-out losses."""
    import torch
    t0 = time.perf_counter()
    gen_steps = gen_steps or steps
    train_cases = draw_cases(n_train, seed=seed, nc=nc, kind=kind)
    test_cases = draw_cases(n_test, seed=seed + 1000, nc=nc, kind=kind)
    held_cases = draw_cases(n_held, seed=seed + 2000, nc=nc, kind=kind)
    X, Y = generate_chunked(train_cases, gen_steps, chunk, log=log, every=every, skip=skip)
    Xh, Yh = generate_chunked(held_cases, gen_steps, chunk, every=every, skip=skip)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, scale, l1, h1 = train(X, Y, iters=iters[0], batch=batch, seed=seed, log=log,
                               capacity=max(n_test, batch, min(chunk, n_train)), held=(Xh, Yh))
    l2, h2 = l1, []
    if rounds > 1:
        X2, Y2 = generate_chunked(train_cases, gen_steps, chunk, net=net, every=every, skip=skip)
        X, Y = torch.cat([X, X2]), torch.cat([Y, Y2])
        del X2, Y2
        net, _, l2, h2 = train(X, Y, iters=iters[1], batch=batch, seed=seed + 1, log=log, net=net,
                               scale=scale, held=(Xh, Yh))
    del X, Y, Xh, Yh
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ev = evaluate(test_cases, steps=steps, net=net, log=log)
    ep = float(np.median([r["plain"] for r in ev["cases"]]))
    ec = float(np.median([r["closure"] for r in ev["cases"]]))
    wins = sum(r["closure"] < r["plain"] for r in ev["cases"])
    ny, nx = test_cases[0]["coarse"]["ny"], test_cases[0]["coarse"]["nx"]
    return dict(
        kind=kind, train_cases=n_train, test_cases=n_test, held_cases=n_held,
        coarse_grid=[nx, ny], fine_grid=[F * nx, F * ny], coarse_steps=steps,
        fine_steps=F * F * steps, data_steps=gen_steps, data_every=every, data_skip=skip,
        rounds=rounds,
        err_plain_coarse=ep, err_closure=ec, closure_better_cases=int(wins),
        t_fine_ms=ev["t_fine"] * 1e3, t_coarse_ms=ev["t_coarse"] * 1e3,
        t_closure_ms=ev["t_closure"] * 1e3,
        speedup_closure_vs_fine=ev["t_fine"] / max(ev["t_closure"], 1e-12),
        gen_s=t_gen, train_s=t_train, loss_first=float(np.mean(l1[:50])),
        loss_round1=float(np.mean(l1[-50:])), loss_last=float(np.mean(l2[-50:])),
        held_round1=[(int(i), float(v)) for i, v in h1], held_round2=[(int(i), float(v)) for i, v in h2],
        net=net)
