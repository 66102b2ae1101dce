"""P13: the FP64 oracle against an independent 50-digit transcription of the
method on tiny grids.

The step below is written afresh from the paper's equations in a different
form from the oracle's C code -- per node, mpmath numbers, a generic linear
solve for the implicit scalar recovery (the oracle uses its closed form),
dictionary lattices -- and shares nothing with it but the inputs.  It takes
the same readings of the paper (backward-difference d_t terms against the
previous level, regularised normal, body force (rho - rho_ref) g, mirror
ghost for the stencils at a wall, half-way bounce-back of every set).  On a
4 x 3 D2Q9 grid with walls in y and a 3 x 3 x 3 D3Q19/D3Q7 grid with walls
in z, from seeded random fields, the oracle must agree to 1e-13 relative
after each of three steps; a dropped term, a wrong sign, index or weight
anywhere in one step of either implementation shows up far above that.

Paper passages: Sec. II (phi profile, chemical potential, mixed
diffusivity, viscosity laws Eq. (1.8) and (4.3)), Sec. III A (f, F_i),
Sec. III B (g, G_i, u, p, tau_g), Sec. III C (h1, h2, H_k, ~H_k, the
implicit recovery, the isotropic central stencils)."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import ref

mpmath = pytest.importorskip("mpmath")
mp = mpmath.mp


def lattice(name):
    """velocities, weights and cs^2 of a DnQm lattice, built from its shells"""
    if name == "D2Q9":
        vel = [(0, 0, 0)] + [(a, b, 0) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
        wt = {0: mpmath.mpf(4) / 9, 1: mpmath.mpf(1) / 9, 2: mpmath.mpf(1) / 36}
        cs2 = mpmath.mpf(1) / 3
    elif name == "D3Q19":
        vel = [(0, 0, 0)] + [c for c in itertools.product((-1, 0, 1), repeat=3)
                             if 0 < sum(abs(v) for v in c) <= 2]
        wt = {0: mpmath.mpf(1) / 3, 1: mpmath.mpf(1) / 18, 2: mpmath.mpf(1) / 36}
        cs2 = mpmath.mpf(1) / 3
    else:  # D3Q7
        vel = [(0, 0, 0)] + [c for c in itertools.product((-1, 0, 1), repeat=3)
                             if sum(abs(v) for v in c) == 1]
        wt = {0: mpmath.mpf(1) / 4, 1: mpmath.mpf(1) / 8}
        cs2 = mpmath.mpf(1) / 4
    w = [wt[sum(abs(v) for v in c)] for c in vel]
    assert abs(sum(w) - 1) < mpmath.mpf(10) ** -45
    return vel, w, cs2


def dot(a, b):
    return sum(x * y for x, y in zip(a, b))


class Brute:
    """One lattice of the coupled method in 50-digit arithmetic."""

    def __init__(self, p, phi, c1, c2, u, pr):
        mp.dps = 50
        self.p = {k: (mpmath.mpf(v) if isinstance(v, float) else v) for k, v in p.items()}
        self.d = 2 if p["lattice"] == "d2q9" else 3
        self.n = (p["nx"], p["ny"], p["nz"])
        self.LF = lattice("D2Q9" if self.d == 2 else "D3Q7")
        self.LG = lattice("D2Q9" if self.d == 2 else "D3Q19")
        self.nodes = list(itertools.product(range(p["nx"]), range(p["ny"]), range(p["nz"])))
        P = self.p
        self.f, self.g, self.h1, self.h2, self.hist = {}, {}, {}, {}, {}
        for x in self.nodes:
            ph, a, b = (mpmath.mpf(float(v[x[2], x[1], x[0]])) for v in (phi, c1, c2))
            ux = [mpmath.mpf(float(u[k][x[2], x[1], x[0]])) if k < self.d else mpmath.mpf(0)
                  for k in range(3)]
            rho = ph * (P["rho1"] - P["rho2"]) + P["rho2"]
            self.f[x] = self.feq(ph, ux)
            self.h1[x] = self.feq(a, ux)
            self.h2[x] = self.feq(b, ux)
            self.g[x] = self.geq(mpmath.mpf(float(pr[x[2], x[1], x[0]])), rho, ux)
            self.hist[x] = (ux, ph, a, b)

    # X^eq = w_i X (1 + c.u/cs^2) for phi, c1, c2 (Sec. III A, III C)
    def feq(self, X, u):
        vel, w, cs2 = self.LF
        return [w[i] * X * (1 + dot(vel[i], u) / cs2) for i in range(len(vel))]

    # g^eq: p/cs^2 (w_i - delta_i0) + rho s_i(u) (Sec. III B)
    def geq(self, p, rho, u):
        vel, w, cs2 = self.LG
        out = []
        for i, c in enumerate(vel):
            cu = dot(c, u)
            s = w[i] * (cu / cs2 + cu * cu / (2 * cs2 * cs2) - dot(u, u) / (2 * cs2))
            out.append(p / cs2 * (w[i] - (1 if i == 0 else 0)) + rho * s)
        return out

    def neighbour(self, x, c):
        """stencil neighbour: periodic wrap, or the mirror ghost (the boundary
        node itself) one step outside a walled axis"""
        y = []
        for a in range(3):
            v = x[a] + c[a]
            if 0 <= v < self.n[a]:
                y.append(v)
            elif self.p["periodic"][a]:
                y.append(v % self.n[a])
            else:
                y.append(x[a])
        return tuple(y)

    def macros(self):
        P = self.p
        vel, w, cs2 = self.LG
        K = P["Keq"]
        m = {}
        for x in self.nodes:
            phi = sum(self.f[x])
            S1, S2 = sum(self.h1[x]), sum(self.h2[x])
            Dm = P["D1"] * P["D2"] / (K * P["D1"] * (1 - phi) + P["D2"] * phi)
            a = P["A"] * Dm / 2
            # c1 = S1 + a (K c2 phi - c1 (1 - phi)),  c2 = S2 - a (K c2 phi - c1 (1 - phi))
            Amat = mpmath.matrix([[1 + a * (1 - phi), -a * K * phi], [-a * (1 - phi), 1 + a * K * phi]])
            sol = mpmath.lu_solve(Amat, mpmath.matrix([S1, S2]))
            m[x] = dict(phi=phi, c1=sol[0], c2=sol[1], Dm=Dm)
        for x in self.nodes:
            q = m[x]
            gphi = [mpmath.mpf(0)] * 3
            gpsi = [mpmath.mpf(0)] * 3
            lap = mpmath.mpf(0)
            for i in range(1, len(vel)):
                y = m[self.neighbour(x, vel[i])]
                psi_y = y["c1"] + K * y["c2"]
                for k in range(3):
                    gphi[k] += w[i] * vel[i][k] * y["phi"] / cs2
                    gpsi[k] += w[i] * vel[i][k] * psi_y / cs2
                lap += 2 * w[i] * (y["phi"] - q["phi"]) / cs2
            q["gphi"], q["gpsi"], q["lap"] = gphi, gpsi, lap
            q["n"] = [v / mpmath.sqrt(dot(gphi, gphi) + P["n_eps"] ** 2) for v in gphi]
            beta, kappa = 12 * P["sigma"] / P["W"], 3 * P["sigma"] * P["W"] / 2
            phi = q["phi"]
            mu_phi = 4 * beta * phi * (phi - 1) * (phi - mpmath.mpf(1) / 2) - kappa * lap
            rho = phi * (P["rho1"] - P["rho2"]) + P["rho2"]
            F = [mu_phi * gphi[k] + (rho - P["rho_ref"]) * mpmath.mpf(P["g"][k]) for k in range(3)]
            mom = [sum(vel[i][k] * self.g[x][i] for i in range(len(vel))) for k in range(3)]
            u = [(mom[k] + F[k] / 2) / rho for k in range(3)]
            s0 = w[0] * (-dot(u, u) / (2 * cs2))
            p = cs2 / (1 - w[0]) * (sum(self.g[x][1:]) + (P["rho1"] - P["rho2"]) * dot(u, gphi) / 2
                                    + rho * s0)
            if P["visc_law"] == "exp":
                mu = mpmath.exp(q["c1"] * mpmath.log(P["mu1"]) + q["c2"] * mpmath.log(P["mu2"]))
            else:
                mu = phi * (P["mu1"] - P["mu2"]) + P["mu2"]
            q.update(F=F, u=u, p=p, rho=rho, mu=mu)
        return m

    def step(self):
        P = self.p
        m = self.macros()
        vF, wF, csF = self.LF
        vG, wG, csG = self.LG
        K = P["Keq"]
        tf = mpmath.mpf(1) / 2 + P["M"] / csF
        t1 = mpmath.mpf(1) / 2 + P["D1"] / csF
        t2 = mpmath.mpf(1) / 2 + P["D2"] / csF
        post = {}
        for x in self.nodes:
            q = m[x]
            uo, pho, c1o, c2o = self.hist[x]
            u, phi, c1, c2 = q["u"], q["phi"], q["c1"], q["c2"]
            dJ = [phi * u[k] - pho * uo[k] for k in range(3)]
            dJ1 = [c1 * u[k] - c1o * uo[k] for k in range(3)]
            dJ2 = [c2 * u[k] - c2o * uo[k] for k in range(3)]
            feq = self.feq(phi, u)
            f = [self.f[x][i] - (self.f[x][i] - feq[i]) / tf + (1 - 1 / (2 * tf)) * wF[i] * (
                dot(vF[i], dJ) / csF + dot(vF[i], q["n"]) * 4 * phi * (1 - phi) / P["W"])
                 for i in range(len(vF))]
            tg = mpmath.mpf(1) / 2 + q["mu"] / (q["rho"] * csG)
            geq = self.geq(q["p"], q["rho"], u)
            g = [self.g[x][i] - (self.g[x][i] - geq[i]) / tg + (1 - 1 / (2 * tg)) * wG[i] * (
                dot(vG[i], q["F"]) / csG + (P["rho1"] - P["rho2"]) * dot(vG[i], u) * dot(vG[i], q["gphi"]) / csG)
                 for i in range(len(vG))]
            ex = P["A"] * q["Dm"] * (K * c2 * phi - c1 * (1 - phi))
            aux = q["Dm"] * dot(q["gphi"], q["gpsi"])
            e1, e2 = self.feq(c1, u), self.feq(c2, u)
            h1, h2 = [], []
            for i in range(len(vF)):
                cn = dot(vF[i], q["n"])
                H1 = wF[i] * (dot(vF[i], dJ1) / csF + cn * 4 * (1 - phi) * c1 / P["W"] + ex)
                H2 = wF[i] * (dot(vF[i], dJ2) / csF - cn * 4 * phi * c2 / P["W"] - ex)
                h1.append(self.h1[x][i] - (self.h1[x][i] - e1[i]) / t1 + (1 - 1 / (2 * t1)) * H1 - wF[i] * aux)
                h2.append(self.h2[x][i] - (self.h2[x][i] - e2[i]) / t2 + (1 - 1 / (2 * t2)) * H2 + wF[i] * aux)
            post[x] = (f, g, h1, h2)
            self.hist[x] = (u, phi, c1, c2)
        # streaming: X_i(x + c_i) <- X_i*(x); a link leaving through a wall
        # returns to x in the opposite direction
        for name, k, L in (("f", 0, self.LF), ("g", 1, self.LG), ("h1", 2, self.LF), ("h2", 3, self.LF)):
            vel = L[0]
            new = {x: [None] * len(vel) for x in self.nodes}
            for x in self.nodes:
                for i, c in enumerate(vel):
                    y, wall = [], False
                    for a in range(3):
                        v = x[a] + c[a]
                        if 0 <= v < self.n[a]:
                            y.append(v)
                        elif self.p["periodic"][a]:
                            y.append(v % self.n[a])
                        else:
                            wall = True
                    if wall:
                        new[x][vel.index(tuple(-v for v in c))] = post[x][k][i]
                    else:
                        new[tuple(y)][i] = post[x][k][i]
            setattr(self, name, new)

    def fields(self):
        m = self.macros()
        out = {}
        for key in ("phi", "c1", "c2", "p"):
            out[key] = {x: m[x][key] for x in self.nodes}
        for k, key in enumerate(("ux", "uy", "uz")):
            out[key] = {x: m[x]["u"][k] for x in self.nodes}
        return out


CASES = [
    dict(nx=4, ny=3, nz=1, lattice="d2q9", periodic=(1, 0, 1), g=(3e-5, -4e-5, 0.0)),
    dict(nx=3, ny=3, nz=3, lattice="d3q19_d3q7", periodic=(1, 1, 0), g=(1e-5, -2e-5, 3e-5)),
]


@pytest.mark.parametrize("case", CASES, ids=["d2q9_4x3_walls_y", "d3q19_3x3x3_walls_z"])
@pytest.mark.parametrize("visc", ["exp", "linear"])
def test_p11_oracle_matches_50_digit_transcription(case, visc):
    p = W.params(precision="f64", sigma=3e-3, rho1=3.0, rho2=1.0, visc_law=visc, mu1=0.3,
                 mu2=0.08, D1=0.07, D2=0.02, Keq=0.6, A=0.4, rho_ref=1.5, M=0.03, W=3.0,
                 n_eps=1e-3, **case)
    f = W.random_fields(p, seed=41, u_amp=0.03, p_amp=2e-3)
    shp3 = (p["nz"], p["ny"], p["nx"])
    d = W.dim_of(p)
    u3 = [f["u"][k].reshape(shp3) if k < d else np.zeros(shp3) for k in range(3)]
    b = Brute(p, f["phi"].reshape(shp3), f["c1"].reshape(shp3), f["c2"].reshape(shp3), u3,
              f["p"].reshape(shp3))
    o = ref.Oracle(p)
    o.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
    names = ("phi", "c1", "c2", "p", "ux", "uy") + (("uz",) if d == 3 else ())
    for step in range(3):
        bf = b.fields()
        for k in names:
            a = o.field(k).reshape(shp3)
            e = np.array([float(bf[k][x]) for x in b.nodes])
            got = np.array([a[x[2], x[1], x[0]] for x in b.nodes])
            scale = max(np.abs(e).max(), np.abs(e - e.mean()).max())
            assert np.abs(got - e).max() <= 1e-13 * scale, (step, k, np.abs(got - e).max() / scale)
        b.step()
        o.step(1)
