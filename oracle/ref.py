"""ctypes wrapper of the FP64 CPU oracle (oracle/libcplb_ref.so).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcplb_ref.so")

FIELDS = {"phi": 0, "p": 1, "ux": 2, "uy": 3, "uz": 4, "c1": 5, "c2": 6, "mu": 7, "psi": 8,
          "gpsi_x": 9, "gpsi_y": 10, "gpsi_z": 11}
SETS = {"f": 0, "g": 1, "h1": 2, "h2": 3}
LATTICES = {"d2q9": 0, "d3q19_d3q7": 1}
VISC = {"linear": 0, "exp": 1}
SCALAR_MODELS = {"two": 0, "one": 1}
SCALAR_BC = {"noflux": 0, "dirichlet": 1}
SCALAR_GRAD = {"central": 0, "local": 1}


class RefParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lattice", ctypes.c_int32), ("visc_law", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3),
        ("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
        ("mu1", ctypes.c_double), ("mu2", ctypes.c_double),
        ("sigma", ctypes.c_double), ("W", ctypes.c_double), ("M", ctypes.c_double),
        ("D1", ctypes.c_double), ("D2", ctypes.c_double), ("Keq", ctypes.c_double),
        ("A", ctypes.c_double), ("g", ctypes.c_double * 3), ("rho_ref", ctypes.c_double),
        ("n_eps", ctypes.c_double), ("scalar_model", ctypes.c_int32),
        ("scalar_bc", ctypes.c_int32 * 6), ("c_wall", ctypes.c_double * 12),
        ("scalar_grad", ctypes.c_int32), ("phase_grad", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library not built: {LIB_PATH} (run oracle/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i64 = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int64
        L.cplb_ref_create.argtypes = [ctypes.POINTER(RefParams), ctypes.POINTER(vp)]
        L.cplb_ref_destroy.argtypes = [vp]
        L.cplb_ref_destroy.restype = None
        L.cplb_ref_last_error.argtypes = [vp]
        L.cplb_ref_last_error.restype = ctypes.c_char_p
        L.cplb_ref_init_fields.argtypes = [vp, dp, dp, dp, dp, dp]
        L.cplb_ref_init_sdf.argtypes = [vp, dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double]
        L.cplb_ref_step.argtypes = [vp, i64]
        L.cplb_ref_set_closure.argtypes = [vp, dp]
        L.cplb_ref_field.argtypes = [vp, ctypes.c_int, dp]
        L.cplb_ref_reduce.argtypes = [vp, dp]
        L.cplb_ref_get_populations.argtypes = [vp, ctypes.c_int, dp]
        L.cplb_ref_population_count.argtypes = [vp, ctypes.c_int]
        L.cplb_ref_state_bytes.argtypes = [vp]
        L.cplb_ref_state_bytes.restype = ctypes.c_size_t
        L.cplb_ref_save_state.argtypes = [vp, vp, ctypes.c_size_t]
        L.cplb_ref_load_state.argtypes = [vp, vp, ctypes.c_size_t]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(p: dict) -> RefParams:
    r = RefParams()
    r.nx, r.ny, r.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    r.lattice = LATTICES[p["lattice"]]
    r.visc_law = VISC[p["visc_law"]]
    for a in range(3):
        r.periodic[a] = int(p["periodic"][a])
        r.g[a] = float(p["g"][a])
    for k in ("rho1", "rho2", "mu1", "mu2", "sigma", "W", "M", "D1", "D2", "Keq", "A",
              "rho_ref", "n_eps"):
        setattr(r, k, float(p[k]))
    r.scalar_model = SCALAR_MODELS[p.get("scalar_model", "two")]
    r.scalar_grad = SCALAR_GRAD[p.get("scalar_grad", "central")]
    r.phase_grad = SCALAR_GRAD[p.get("phase_grad", "central")]
    for f in range(6):
        r.scalar_bc[f] = SCALAR_BC[p.get("scalar_bc", ("noflux",) * 6)[f]]
        cw = p.get("c_wall", ((0.0, 0.0),) * 6)[f]
        r.c_wall[2 * f], r.c_wall[2 * f + 1] = float(cw[0]), float(cw[1])
    return r


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


class Oracle:
    """One oracle lattice.  Fields come back as float64 arrays of shape
    (ny, nx) or (nz, ny, nx)."""

    def __init__(self, p: dict):
        self.p = dict(p)
        self.d = 2 if p["lattice"] == "d2q9" else 3
        self.shape = (p["ny"], p["nx"]) if self.d == 2 else (p["nz"], p["ny"], p["nx"])
        self.N = int(p["nx"]) * int(p["ny"]) * int(p["nz"])
        self._prm = make_params(p)
        h = ctypes.c_void_p()
        rc = lib().cplb_ref_create(ctypes.byref(self._prm), ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc, "cplb_ref_create rejected the parameters")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cplb_ref_destroy(self._h)
            self._h = None

    __del__ = close

    def _check(self, rc):
        if rc != 0:
            raise OracleError(rc, lib().cplb_ref_last_error(self._h).decode())

    def init_sdf(self, l, c1=(0.0, 0.0), c2=(0.0, 0.0)):
        l = np.ascontiguousarray(l, dtype=np.float64).reshape(-1)
        assert l.size == self.N
        self._check(lib().cplb_ref_init_sdf(self._h, _dptr(l), c1[0], c1[1], c2[0], c2[1]))

    def init_fields(self, phi, c1, c2, u=None, p=None):
        arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (phi, c1, c2)]
        for a in arrs:
            assert a.size == self.N
        up = None
        if u is not None:
            u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
            assert u.size == self.d * self.N
            up = _dptr(u)
        pp = None
        if p is not None:
            p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
            assert p.size == self.N
            pp = _dptr(p)
        self._check(lib().cplb_ref_init_fields(self._h, _dptr(arrs[0]), _dptr(arrs[1]),
                                               _dptr(arrs[2]), up, pp))

    def set_closure(self, s):
        """Per-node corrections (s1, s2) of c1 and c2 per step, shaped
        (2,) + the lattice shape (None switches them off); the array is kept
        alive by the oracle object."""
        if s is None:
            self._closure = None
            self._check(lib().cplb_ref_set_closure(self._h, None))
            return
        self._closure = np.ascontiguousarray(s, dtype=np.float64).reshape(-1).copy()
        if self._closure.size != 2 * self.N:
            raise ValueError(f"closure needs 2 planes of {self.N} values, got {self._closure.size}")
        self._check(lib().cplb_ref_set_closure(self._h, _dptr(self._closure)))

    def step(self, n=1):
        self._check(lib().cplb_ref_step(self._h, int(n)))

    def field(self, name):
        out = np.empty(self.N, dtype=np.float64)
        self._check(lib().cplb_ref_field(self._h, FIELDS[name], _dptr(out)))
        return out.reshape(self.shape)

    def fields(self, names=("phi", "c1", "c2", "ux", "uy", "p")):
        return {k: self.field(k) for k in names}

    def reduce(self):
        out = np.zeros(8, dtype=np.float64)
        rc = lib().cplb_ref_reduce(self._h, _dptr(out))
        keys = ("sum_phi", "sum_c1", "sum_c2", "sum_c", "max_u", "kinetic", "nonfinite", "step")
        r = dict(zip(keys, out.tolist()))
        r["rc"] = rc
        return r

    def populations(self, name):
        q = lib().cplb_ref_population_count(self._h, SETS[name])
        out = np.empty(q * self.N, dtype=np.float64)
        self._check(lib().cplb_ref_get_populations(self._h, SETS[name], _dptr(out)))
        return out.reshape((q,) + self.shape)

    def save_state(self) -> bytes:
        n = lib().cplb_ref_state_bytes(self._h)
        buf = ctypes.create_string_buffer(n)
        self._check(lib().cplb_ref_save_state(self._h, ctypes.cast(buf, ctypes.c_void_p), n))
        return buf.raw

    def load_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(lib().cplb_ref_load_state(self._h, ctypes.cast(buf, ctypes.c_void_p), len(blob)))


def run_workload(w: dict, steps=None) -> "Oracle":
    """Create an oracle for a workload dict from the workloads module,
    initialise it from the signed distance, and advance ``steps`` steps."""
    o = Oracle(w["params"])
    o.init_sdf(w["sdf"], c1=w["init"]["c1"], c2=w["init"]["c2"])
    o.step(w["steps"] if steps is None else steps)
    return o
