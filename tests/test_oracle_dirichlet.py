"""Pins of the oracle's Dirichlet scalar boundary (half-way anti-bounce-back
of h1, h2, Sec. IV) on the paper's linear-equilibrium case (Sec. IV A 3):
a planar interface in the middle of a walled 1-D domain, phase 1 on the
right, c1 = c2 = 0 imposed on the left face and c1 = 2, c2 = 0 on the right.

At steady state each bulk phase carries a constant diffusive flux, so
c2 (left) and c1 (right) are linear; the half-way walls sit half a node
outside the first and last nodes, where the linear profiles must take the
imposed values; and flux continuity with the interfacial equilibrium
c~1 = Keq c~2 fixes the slopes: with L2, L1 the distances wall-interface,
c~2(interface) = 2 D1 L2 / (D2 L1 + Keq D1 L2), slope 2 = c~2i / L2,
slope 1 = (2 - Keq c~2i) / L1.  The interface width (W = 4) changes the
slopes by O((W / L)^2): 0.1-0.3 % here.  The regularised normal keeps its
far tails diffusing (reading R2), so these runs use n_eps = 1e-9."""
import numpy as np
import pytest

import workloads as W
from oracle import ref

N = 64
DIRICHLET_X = ("dirichlet", "dirichlet", "noflux", "noflux", "noflux", "noflux")
C_WALL = ((0.0, 0.0), (2.0, 0.0), (0.0, 0.0), (0.0, 0.0), (0.0, 0.0), (0.0, 0.0))


def steady(D1, D2, K, steps=80000):
    p = W.params(nx=N, ny=1, periodic=(0, 1, 1), sigma=0.0, D1=D1, D2=D2, Keq=K, A=0.1,
                 n_eps=1e-9, scalar_bc=DIRICHLET_X, c_wall=C_WALL)
    x = np.arange(N, dtype=float)
    xi = (N - 1) / 2.0
    o = ref.Oracle(p)
    o.init_sdf((x - xi).reshape(1, N), c1=(0.0, 2.0), c2=(0.0, 0.0))
    o.step(steps)
    return x, xi, o


@pytest.mark.parametrize("D1,D2,K", [(0.15, 0.15, 1.0), (0.15, 0.05, 1.0), (0.15, 0.15, 1.0 / 3.0)])
def test_linear_equilibrium(D1, D2, K):
    x, xi, o = steady(D1, D2, K)
    c1, c2 = o.field("c1")[0], o.field("c2")[0]
    xL, xR = -0.5, N - 0.5  # half-way walls
    left, right = x < xi - 12, x > xi + 12
    a2 = np.polyfit(x[left], c2[left], 1)
    a1 = np.polyfit(x[right], c1[right], 1)
    # bulk profiles are linear
    assert np.abs(np.polyval(a2, x[left]) - c2[left]).max() <= 1e-5
    assert np.abs(np.polyval(a1, x[right]) - c1[right]).max() <= 1e-5
    # the imposed values hold at the half-way walls
    assert abs(np.polyval(a2, xL) - 0.0) <= 1e-5
    assert abs(np.polyval(a1, xR) - 2.0) <= 1e-5
    # flux continuity and the interfacial jump fix the slopes
    L2, L1 = xi - xL, xR - xi
    ct2i = 2.0 * D1 * L2 / (D2 * L1 + K * D1 * L2)
    assert abs(a2[0] / (ct2i / L2) - 1.0) <= 5e-3, (a2[0], ct2i / L2)
    assert abs(a1[0] / ((2.0 - K * ct2i) / L1) - 1.0) <= 5e-3, (a1[0], (2.0 - K * ct2i) / L1)
    # phase 2 holds no c1 and phase 1 no c2 in the bulk
    assert np.abs(c1[left]).max() <= 1e-5 and np.abs(c2[right]).max() <= 1e-5


def test_dirichlet_face_changes_only_the_scalars():
    """f and g keep bounce-back at a Dirichlet face: the phase field and the
    flow of a run with Dirichlet faces equal those of the no-flux run."""
    p0 = W.params(nx=20, ny=9, periodic=(0, 0, 1), sigma=3e-3, rho1=2.0, rho2=1.0, D1=0.07,
                  D2=0.03, Keq=0.5, g=(0.0, -1e-5, 0.0), rho_ref=1.5)
    p1 = dict(p0, scalar_bc=("dirichlet", "noflux", "noflux", "dirichlet", "noflux", "noflux"),
              c_wall=((0.3, 0.1), (0.0, 0.0), (0.0, 0.0), (0.05, 0.7), (0.0, 0.0), (0.0, 0.0)))
    f = W.random_fields(p0, seed=3)
    runs = []
    for p in (p0, p1):
        o = ref.Oracle(p)
        o.init_fields(f["phi"], f["c1"], f["c2"], u=f["u"], p=f["p"])
        o.step(1)
        runs.append(o)
    for k in ("phi",):
        assert np.array_equal(runs[0].field(k), runs[1].field(k)), k
    assert not np.array_equal(runs[0].field("c1"), runs[1].field("c1"))


def test_dirichlet_needs_a_walled_axis():
    p = W.params(nx=8, ny=8, periodic=(1, 1, 1), scalar_bc=DIRICHLET_X, c_wall=C_WALL)
    with pytest.raises(ref.OracleError):
        ref.Oracle(p)
