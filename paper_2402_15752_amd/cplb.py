"""ctypes binding of libcplb.so (the C-ABI declared in include/cplb.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch supplies the device workspace and the HIP stream.
There is no fallback: if the library is missing or no GPU is present the
calls raise.

The module-level functions carry the same names as the C entry points; the
``Lattice`` class is a convenience wrapper over them.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcplb.so")

CPLB_OK, CPLB_EINVAL, CPLB_ENOMEM, CPLB_EHIP, CPLB_EUNSTABLE, CPLB_ESTATE = 0, -1, -2, -3, -4, -5
LATTICES = {"d2q9": 0, "d3q19_d3q7": 1}
PRECISIONS = {"f64": 0, "f32": 1, "f32_s16f": 2, "f32_s16b": 3}
VISC = {"linear": 0, "exp": 1}
SCALAR_MODELS = {"two": 0, "one": 1}
CPLB_TWO_SCALAR, CPLB_ONE_SCALAR = 0, 1
SCALAR_BC = {"noflux": 0, "dirichlet": 1}
SCALAR_GRAD = {"central": 0, "local": 1}
FIELDS = {"phi": 0, "p": 1, "ux": 2, "uy": 3, "uz": 4, "c1": 5, "c2": 6, "mu": 7, "psi": 8}
DTYPE_F32, DTYPE_F64 = 0, 1
EXPORTS = ("cplb_workspace_bytes", "cplb_create", "cplb_init_fields", "cplb_init_sdf", "cplb_step",
           "cplb_read_field", "cplb_reduce", "cplb_reduce_device", "cplb_step_count", "cplb_state_bytes",
           "cplb_save_state", "cplb_load_state", "cplb_last_error", "cplb_strerror",
           "cplb_destroy", "cplb_num_variants", "cplb_get_variant", "cplb_set_variant",
           "cplb_variant_name", "cplb_tune",
           "cplb_batch_workspace_bytes", "cplb_batch_create", "cplb_batch_init_sdf",
           "cplb_batch_step", "cplb_batch_num_cases", "cplb_batch_step_count",
           "cplb_batch_read_field", "cplb_batch_reduce", "cplb_batch_num_classes",
           "cplb_batch_case_class", "cplb_batch_class_cases", "cplb_batch_get_variant",
           "cplb_batch_set_variant", "cplb_batch_tune", "cplb_batch_last_error",
           "cplb_batch_destroy", "cplb_set_closure",
           "cplb_cnn_num_params", "cplb_cnn_workspace_bytes", "cplb_cnn_create",
           "cplb_cnn_set_params", "cplb_cnn_init_params", "cplb_cnn_get_params",
           "cplb_cnn_set_input_scale", "cplb_cnn_forward", "cplb_cnn_backward",
           "cplb_cnn_get_grads", "cplb_cnn_adam", "cplb_cnn_last_error", "cplb_cnn_destroy",
           "cplb_batch_num_nodes", "cplb_batch_set_closure", "cplb_batch_gather_fields",
           "cplb_cnn_set_output_scale", "cplb_cnn_restrict", "cplb_batch_init_planes",
           "cplb_cnn_infer", "cplb_cnn_set_stream")


class cplb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lattice", ctypes.c_int32), ("precision", ctypes.c_int32), ("visc_law", ctypes.c_int32),
        ("periodic", ctypes.c_int32 * 3), ("scalar_model", ctypes.c_int32),
        ("rho1", ctypes.c_double), ("rho2", ctypes.c_double),
        ("mu1", ctypes.c_double), ("mu2", ctypes.c_double),
        ("sigma", ctypes.c_double), ("W", ctypes.c_double), ("M", ctypes.c_double),
        ("D1", ctypes.c_double), ("D2", ctypes.c_double), ("Keq", ctypes.c_double),
        ("A", ctypes.c_double), ("g", ctypes.c_double * 3), ("rho_ref", ctypes.c_double),
        ("n_eps", ctypes.c_double), ("ref", ctypes.c_double * 4),
        ("scalar_bc", ctypes.c_int32 * 6), ("c_wall", ctypes.c_double * 12),
        ("scalar_grad", ctypes.c_int32), ("phase_grad", ctypes.c_int32),
    ]


class CplbError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"cplb error {code} ({_strerror(code)}): {msg}")
        self.code = code


_lib = None


def library():
    """Load libcplb.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
        P = ctypes.POINTER(cplb_params)
        L.cplb_workspace_bytes.argtypes = [P, ctypes.POINTER(sz)]
        L.cplb_create.argtypes = [P, vp, sz, vp, ctypes.POINTER(vp)]
        L.cplb_init_fields.argtypes = [vp, dp, dp, dp, dp, dp]
        L.cplb_init_sdf.argtypes = [vp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double]
        L.cplb_step.argtypes = [vp, ctypes.c_int64]
        L.cplb_read_field.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
        L.cplb_reduce.argtypes = [vp, dp]
        L.cplb_reduce_device.argtypes = [vp, vp]
        L.cplb_step_count.argtypes = [vp]
        L.cplb_step_count.restype = ctypes.c_int64
        L.cplb_state_bytes.argtypes = [vp]
        L.cplb_state_bytes.restype = sz
        L.cplb_save_state.argtypes = [vp, vp, sz]
        L.cplb_load_state.argtypes = [vp, vp, sz]
        L.cplb_last_error.argtypes = [vp]
        L.cplb_last_error.restype = ctypes.c_char_p
        L.cplb_strerror.argtypes = [ctypes.c_int]
        L.cplb_strerror.restype = ctypes.c_char_p
        L.cplb_destroy.argtypes = [vp]
        L.cplb_destroy.restype = None
        L.cplb_num_variants.argtypes = [vp]
        L.cplb_get_variant.argtypes = [vp]
        L.cplb_set_variant.argtypes = [vp, ctypes.c_int]
        L.cplb_variant_name.argtypes = [vp, ctypes.c_int]
        L.cplb_variant_name.restype = ctypes.c_char_p
        L.cplb_tune.argtypes = [vp, ctypes.c_int, dp]
        i32 = ctypes.c_int
        L.cplb_batch_workspace_bytes.argtypes = [P, i32, ctypes.POINTER(sz)]
        L.cplb_batch_create.argtypes = [P, i32, vp, sz, vp, ctypes.POINTER(vp)]
        L.cplb_batch_init_sdf.argtypes = [vp, i32, dp, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double]
        L.cplb_batch_step.argtypes = [vp, ctypes.c_int64]
        L.cplb_batch_num_cases.argtypes = [vp]
        L.cplb_batch_step_count.argtypes = [vp]
        L.cplb_batch_step_count.restype = ctypes.c_int64
        L.cplb_batch_read_field.argtypes = [vp, i32, i32, vp, i32]
        L.cplb_batch_reduce.argtypes = [vp, i32, dp]
        for f in ("cplb_batch_num_classes",):
            getattr(L, f).argtypes = [vp]
        for f in ("cplb_batch_case_class", "cplb_batch_class_cases", "cplb_batch_get_variant"):
            getattr(L, f).argtypes = [vp, i32]
        L.cplb_batch_set_variant.argtypes = [vp, i32, i32]
        L.cplb_batch_tune.argtypes = [vp, i32, dp]
        L.cplb_batch_last_error.argtypes = [vp]
        L.cplb_batch_last_error.restype = ctypes.c_char_p
        L.cplb_batch_destroy.argtypes = [vp]
        L.cplb_batch_destroy.restype = None
        L.cplb_set_closure.argtypes = [vp, vp]
        fp = ctypes.POINTER(ctypes.c_float)
        L.cplb_cnn_num_params.argtypes = []
        L.cplb_cnn_workspace_bytes.argtypes = [i32, i32, i32, ctypes.POINTER(sz)]
        L.cplb_cnn_create.argtypes = [i32, i32, i32, vp, sz, vp, ctypes.POINTER(vp)]
        L.cplb_cnn_set_params.argtypes = [vp, fp]
        L.cplb_cnn_init_params.argtypes = [vp, ctypes.c_uint64]
        L.cplb_cnn_get_params.argtypes = [vp, fp]
        L.cplb_cnn_set_input_scale.argtypes = [vp, fp]
        L.cplb_cnn_forward.argtypes = [vp, i32, vp, i32, vp]
        L.cplb_cnn_infer.argtypes = [vp, i32, vp, i32, vp]
        L.cplb_cnn_set_stream.argtypes = [vp, vp]
        L.cplb_cnn_backward.argtypes = [vp, vp, dp]
        L.cplb_cnn_get_grads.argtypes = [vp, fp]
        L.cplb_cnn_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float]
        L.cplb_cnn_last_error.argtypes = [vp]
        L.cplb_cnn_last_error.restype = ctypes.c_char_p
        L.cplb_cnn_destroy.argtypes = [vp]
        L.cplb_cnn_destroy.restype = None
        L.cplb_batch_num_nodes.argtypes = [vp]
        L.cplb_batch_num_nodes.restype = ctypes.c_int64
        L.cplb_batch_set_closure.argtypes = [vp, vp]
        L.cplb_batch_gather_fields.argtypes = [vp, ctypes.POINTER(i32), i32, i32, vp]
        L.cplb_cnn_set_output_scale.argtypes = [vp, ctypes.c_float, ctypes.c_float]
        L.cplb_batch_init_planes.argtypes = [vp, vp, i32, i32, i32, i32]
        L.cplb_cnn_restrict.argtypes = [vp, vp, i32, i32, i32, i32, vp]
        _lib = L
    return _lib


def _strerror(code):
    try:
        return library().cplb_strerror(code).decode()
    except Exception:  # library not loadable while formatting an error
        return "?"


def make_params(p: dict) -> cplb_params:
    """cplb_params from a parameter dict (keys as in the workloads module)."""
    r = cplb_params()
    r.nx, r.ny, r.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    r.lattice = LATTICES[p["lattice"]]
    r.precision = PRECISIONS[p.get("precision", "f64")]
    r.visc_law = VISC[p["visc_law"]]
    for a in range(3):
        r.periodic[a] = int(p["periodic"][a])
        r.g[a] = float(p["g"][a])
    r.scalar_model = SCALAR_MODELS[p.get("scalar_model", "two")]
    r.scalar_grad = SCALAR_GRAD[p.get("scalar_grad", "central")]
    r.phase_grad = SCALAR_GRAD[p.get("phase_grad", "central")]
    for f in range(6):
        r.scalar_bc[f] = SCALAR_BC[p.get("scalar_bc", ("noflux",) * 6)[f]]
        cw = p.get("c_wall", ((0.0, 0.0),) * 6)[f]
        r.c_wall[2 * f], r.c_wall[2 * f + 1] = float(cw[0]), float(cw[1])
    for k in ("rho1", "rho2", "mu1", "mu2", "sigma", "W", "M", "D1", "D2", "Keq", "A", "rho_ref",
              "n_eps"):
        setattr(r, k, float(p[k]))
    for k, name in enumerate(("ref_f", "ref_g", "ref_h1", "ref_h2")):
        r.ref[k] = float(p.get(name, 0.0))
    return r


# ------------------------------------------------- thin C-ABI wrappers

def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def cplb_workspace_bytes(prm: cplb_params) -> int:
    n = ctypes.c_size_t()
    rc = library().cplb_workspace_bytes(ctypes.byref(prm), ctypes.byref(n))
    if rc:
        raise CplbError(rc, "cplb_workspace_bytes rejected the parameters")
    return n.value


def cplb_create(prm: cplb_params, ws_ptr: int, ws_bytes: int, stream_ptr: int):
    h = ctypes.c_void_p()
    rc = library().cplb_create(ctypes.byref(prm), ctypes.c_void_p(ws_ptr), ws_bytes,
                               ctypes.c_void_p(stream_ptr), ctypes.byref(h))
    if rc:
        raise CplbError(rc, "cplb_create failed")
    return h


def _check(h, rc):
    if rc:
        raise CplbError(rc, library().cplb_last_error(h).decode())


def cplb_init_fields(h, phi, c1, c2, u=None, p=None):
    _check(h, library().cplb_init_fields(h, _dp(phi), _dp(c1), _dp(c2), _dp(u), _dp(p)))


def cplb_init_sdf(h, l, c1_a, c1_b, c2_a, c2_b):
    _check(h, library().cplb_init_sdf(h, _dp(l), c1_a, c1_b, c2_a, c2_b))


def cplb_step(h, nsteps: int):
    _check(h, library().cplb_step(h, int(nsteps)))


def cplb_read_field(h, field: int, dev_ptr: int, dtype: int):
    _check(h, library().cplb_read_field(h, int(field), ctypes.c_void_p(dev_ptr), int(dtype)))


def cplb_reduce(h):
    out = np.zeros(8, dtype=np.float64)
    rc = library().cplb_reduce(h, _dp(out))
    if rc not in (CPLB_OK, CPLB_EUNSTABLE):
        _check(h, rc)
    return out, rc


def cplb_step_count(h) -> int:
    return int(library().cplb_step_count(h))


def cplb_state_bytes(h) -> int:
    return int(library().cplb_state_bytes(h))


def cplb_save_state(h) -> bytes:
    n = cplb_state_bytes(h)
    buf = ctypes.create_string_buffer(n)
    _check(h, library().cplb_save_state(h, ctypes.cast(buf, ctypes.c_void_p), n))
    return buf.raw


def cplb_load_state(h, blob: bytes):
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(h, library().cplb_load_state(h, ctypes.cast(buf, ctypes.c_void_p), len(blob)))


def cplb_destroy(h):
    library().cplb_destroy(h)


def cplb_set_closure(h, dev_ptr):
    _check(h, library().cplb_set_closure(h, None if dev_ptr is None else ctypes.c_void_p(dev_ptr)))


def cplb_num_variants(h) -> int:
    return int(library().cplb_num_variants(h))


def cplb_get_variant(h) -> int:
    return int(library().cplb_get_variant(h))


def cplb_set_variant(h, v: int):
    _check(h, library().cplb_set_variant(h, int(v)))


def cplb_variant_name(h, v: int) -> str:
    return library().cplb_variant_name(h, int(v)).decode()


def cplb_tune(h, probe_steps: int) -> float:
    ms = ctypes.c_double()
    _check(h, library().cplb_tune(h, int(probe_steps), ctypes.byref(ms)))
    return ms.value


# ------------------------------------------------------- convenience class

class Lattice:
    """One lattice on one GPU.  Fields are returned as torch tensors on the
    device, shaped (ny, nx) or (nz, ny, nx)."""

    def __init__(self, p: dict, device="cuda:0", stream=None):
        """stream: the torch.cuda.Stream every call of this lattice is ordered
        on (default: the current stream of `device`).  A stream of its own is
        needed to capture steps in a graph."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("cplb needs a GPU: torch.cuda.is_available() is False")
        self.torch = torch
        self.p = dict(p)
        self.device = torch.device(device)
        self.d = 2 if p["lattice"] == "d2q9" else 3
        self.shape = (p["ny"], p["nx"]) if self.d == 2 else (p["nz"], p["ny"], p["nx"])
        self.N = int(p["nx"]) * int(p["ny"]) * int(p["nz"])
        self._prm = make_params(p)
        nbytes = cplb_workspace_bytes(self._prm)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = cplb_create(self._prm, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)

    def close(self):
        """Release the handle once the work queued on its stream has finished
        (the workspace tensor may be reused by torch as soon as it is freed)."""
        if getattr(self, "_h", None):
            self.stream.synchronize()
            cplb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def init_sdf(self, l, c1=(0.0, 0.0), c2=(0.0, 0.0)):
        l = np.ascontiguousarray(l, dtype=np.float64).reshape(-1)
        assert l.size == self.N
        cplb_init_sdf(self._h, l, float(c1[0]), float(c1[1]), float(c2[0]), float(c2[1]))

    def init_fields(self, phi, c1, c2, u=None, p=None):
        a = [np.ascontiguousarray(x, dtype=np.float64).reshape(-1) for x in (phi, c1, c2)]
        assert all(x.size == self.N for x in a)
        if u is not None:
            u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
            assert u.size == self.d * self.N
        if p is not None:
            p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
            assert p.size == self.N
        cplb_init_fields(self._h, a[0], a[1], a[2], u, p)

    def step(self, n=1):
        cplb_step(self._h, n)

    def field(self, name, dtype=None):
        torch = self.torch
        dtype = dtype or torch.float64
        out = torch.empty(self.shape, dtype=dtype, device=self.device)
        cur = torch.cuda.current_stream(self.device)
        other = cur != self.stream
        if other:  # the new tensor is used on the library stream, then by the caller
            self.stream.wait_stream(cur)
        cplb_read_field(self._h, FIELDS[name], out.data_ptr(),
                        DTYPE_F64 if dtype == torch.float64 else DTYPE_F32)
        if other:
            cur.wait_stream(self.stream)
            out.record_stream(self.stream)
        return out

    def fields(self, names=("phi", "c1", "c2", "ux", "uy", "p")):
        return {k: self.field(k) for k in names}

    def reduce(self):
        out, rc = cplb_reduce(self._h)
        keys = ("sum_phi", "sum_c1", "sum_c2", "sum_c", "max_u", "kinetic", "nonfinite", "step")
        r = dict(zip(keys, out.tolist()))
        r["rc"] = rc
        return r

    @property
    def step_count(self):
        return cplb_step_count(self._h)

    @property
    def variant(self):
        return cplb_get_variant(self._h)

    @variant.setter
    def variant(self, v):
        cplb_set_variant(self._h, v)

    def set_closure(self, s):
        """Per-node corrections (s1, s2) of c1 and c2 per step (a float32
        device tensor of 2 N values: the s1 plane then the s2 plane, e.g.
        shaped (2,) + the lattice shape) applied by every following step, or
        None.  The tensor is kept alive while set; the library stream waits
        for the caller's stream."""
        if s is None:
            cplb_set_closure(self._h, None)
            self._closure = None
            return
        t = s
        assert t.dtype == self.torch.float32 and t.is_cuda and t.is_contiguous()
        assert t.numel() == 2 * self.N
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        cplb_set_closure(self._h, t.data_ptr())
        self._closure = t

    def variant_names(self):
        return [cplb_variant_name(self._h, v) for v in range(cplb_num_variants(self._h))]

    def tune(self, probe_steps=20):
        """Pick the fastest compiled step-kernel variant; returns ms/step."""
        return cplb_tune(self._h, probe_steps)

    def save_state(self) -> bytes:
        return cplb_save_state(self._h)

    def load_state(self, blob: bytes):
        cplb_load_state(self._h, blob)


# ------------------------------------------------------------------ batches

def _params_array(ps):
    arr = (cplb_params * len(ps))()
    for k, p in enumerate(ps):
        arr[k] = make_params(p)
    return arr


def _bcheck(b, rc):
    if rc:
        raise CplbError(rc, library().cplb_batch_last_error(b).decode())


def cplb_batch_workspace_bytes(prms, ncases: int) -> int:
    n = ctypes.c_size_t()
    rc = library().cplb_batch_workspace_bytes(prms, ncases, ctypes.byref(n))
    if rc:
        raise CplbError(rc, "cplb_batch_workspace_bytes rejected the parameters")
    return n.value


def cplb_batch_create(prms, ncases: int, ws_ptr: int, ws_bytes: int, stream_ptr: int):
    b = ctypes.c_void_p()
    rc = library().cplb_batch_create(prms, ncases, ctypes.c_void_p(ws_ptr), ws_bytes,
                                     ctypes.c_void_p(stream_ptr), ctypes.byref(b))
    if rc:
        raise CplbError(rc, "cplb_batch_create failed")
    return b


def cplb_batch_init_sdf(b, icase, l, c1_a, c1_b, c2_a, c2_b):
    _bcheck(b, library().cplb_batch_init_sdf(b, icase, _dp(l), c1_a, c1_b, c2_a, c2_b))


def cplb_batch_step(b, nsteps: int):
    _bcheck(b, library().cplb_batch_step(b, nsteps))


def cplb_batch_num_cases(b) -> int:
    return library().cplb_batch_num_cases(b)


def cplb_batch_step_count(b) -> int:
    return library().cplb_batch_step_count(b)


def cplb_batch_read_field(b, icase: int, field: int, dev_ptr: int, dtype: int):
    _bcheck(b, library().cplb_batch_read_field(b, icase, field, ctypes.c_void_p(dev_ptr), dtype))


def cplb_batch_reduce(b, icase: int):
    out = np.zeros(8)
    rc = library().cplb_batch_reduce(b, icase, _dp(out))
    if rc and rc != CPLB_EUNSTABLE:
        _bcheck(b, rc)
    return out, rc


def cplb_batch_num_nodes(b) -> int:
    return library().cplb_batch_num_nodes(b)


def cplb_batch_set_closure(b, dev_ptr):
    _bcheck(b, library().cplb_batch_set_closure(b, None if dev_ptr is None
                                                else ctypes.c_void_p(dev_ptr)))


def cplb_batch_gather_fields(b, field_ids, nplanes, dev_ptr):
    arr = (ctypes.c_int * len(field_ids))(*field_ids)
    _bcheck(b, library().cplb_batch_gather_fields(b, arr, len(field_ids), nplanes,
                                                  ctypes.c_void_p(dev_ptr)))


def cplb_batch_num_classes(b) -> int:
    return library().cplb_batch_num_classes(b)


def cplb_batch_case_class(b, icase: int) -> int:
    return library().cplb_batch_case_class(b, icase)


def cplb_batch_class_cases(b, cls: int) -> int:
    return library().cplb_batch_class_cases(b, cls)


def cplb_batch_get_variant(b, cls: int) -> int:
    return library().cplb_batch_get_variant(b, cls)


def cplb_batch_set_variant(b, cls: int, v: int):
    _bcheck(b, library().cplb_batch_set_variant(b, cls, v))


def cplb_batch_tune(b, probe_steps: int) -> float:
    ms = ctypes.c_double()
    _bcheck(b, library().cplb_batch_tune(b, probe_steps, ctypes.byref(ms)))
    return ms.value


def cplb_batch_last_error(b) -> str:
    return library().cplb_batch_last_error(b).decode()


def cplb_batch_destroy(b):
    library().cplb_batch_destroy(b)


class Batch:
    """Independent D2Q9 lattices (one parameter dict each, same precision)
    advanced together on one GPU.  Fields come back as torch tensors of
    shape (ny, nx) of the case asked for."""

    def __init__(self, params: list, device="cuda:0", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("cplb needs a GPU: torch.cuda.is_available() is False")
        self.torch = torch
        self.params = [dict(p) for p in params]
        self.n = len(self.params)
        self.device = torch.device(device)
        self._prms = _params_array(self.params)
        nbytes = cplb_batch_workspace_bytes(self._prms, self.n)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._b = cplb_batch_create(self._prms, self.n, self.workspace.data_ptr(), nbytes,
                                    self.stream.cuda_stream)

    def close(self):
        """Release the batch once the work queued on its stream has finished."""
        if getattr(self, "_b", None):
            self.stream.synchronize()
            cplb_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._b

    def init_sdf(self, icase, l, c1=(0.0, 0.0), c2=(0.0, 0.0)):
        p = self.params[icase]
        l = np.ascontiguousarray(l, dtype=np.float64).reshape(-1)
        assert l.size == int(p["nx"]) * int(p["ny"])
        cplb_batch_init_sdf(self._b, icase, l, float(c1[0]), float(c1[1]), float(c2[0]),
                            float(c2[1]))

    def init_planes(self, planes, nplanes, iphi=0, ic1=1, ic2=2):
        """Equilibrium initial state of every case from a float32 device
        buffer in the gather layout (u = p = 0)."""
        assert planes.dtype == self.torch.float32 and planes.is_contiguous()
        assert planes.numel() == self.num_nodes * nplanes
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        _bcheck(self._b, library().cplb_batch_init_planes(self._b, ctypes.c_void_p(planes.data_ptr()),
                                                          nplanes, iphi, ic1, ic2))

    def step(self, n=1):
        cplb_batch_step(self._b, n)

    @property
    def step_count(self):
        return cplb_batch_step_count(self._b)

    def field(self, icase, name, dtype=None):
        torch = self.torch
        dtype = dtype or torch.float64
        p = self.params[icase]
        out = torch.empty((p["ny"], p["nx"]), dtype=dtype, device=self.device)
        cur = torch.cuda.current_stream(self.device)
        other = cur != self.stream
        if other:
            self.stream.wait_stream(cur)
        cplb_batch_read_field(self._b, icase, FIELDS[name], out.data_ptr(),
                              DTYPE_F64 if dtype == torch.float64 else DTYPE_F32)
        if other:
            cur.wait_stream(self.stream)
            out.record_stream(self.stream)
        return out

    def reduce(self, icase):
        out, rc = cplb_batch_reduce(self._b, icase)
        keys = ("sum_phi", "sum_c1", "sum_c2", "sum_c", "max_u", "kinetic", "nonfinite", "step")
        r = dict(zip(keys, out.tolist()))
        r["rc"] = rc
        return r

    @property
    def num_nodes(self):
        return cplb_batch_num_nodes(self._b)

    def set_closure(self, s):
        """Per-node corrections of every case (float32 device tensor of
        2 num_nodes values: case after case, its s1 plane then its s2 plane;
        with cases of equal size, shaped [n, 2, ny, nx]), or None; kept alive
        while set."""
        if s is None:
            cplb_batch_set_closure(self._b, None)
            self._closure = None
            return
        assert s.dtype == self.torch.float32 and s.is_contiguous() and s.numel() == 2 * self.num_nodes
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        cplb_batch_set_closure(self._b, s.data_ptr())
        self._closure = s

    def gather(self, names, out=None, nplanes=None):
        """Fields `names` of every case into one float32 device tensor: case c
        owns `nplanes` (default len(names)) planes of its nodes, the first
        len(names) written.  With cases of equal size the result is shaped
        [ncases, nplanes, ny, nx]."""
        torch = self.torch
        nplanes = nplanes or len(names)
        n = self.num_nodes * nplanes
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=self.device)
        assert out.numel() == n and out.dtype == torch.float32 and out.is_contiguous()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        cplb_batch_gather_fields(self._b, [FIELDS[k] for k in names], nplanes, out.data_ptr())
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        shapes = {(p["ny"], p["nx"]) for p in self.params}
        if len(shapes) == 1:
            ny, nx = shapes.pop()
            return out.view(self.n, nplanes, ny, nx)
        return out

    def classes(self):
        """[(cases in class, variant index)] per size class."""
        return [(cplb_batch_class_cases(self._b, c), cplb_batch_get_variant(self._b, c))
                for c in range(cplb_batch_num_classes(self._b))]

    def set_variant(self, cls, v):
        cplb_batch_set_variant(self._b, cls, v)

    def tune(self, probe_steps=10):
        """Pick the fastest tile variant per size class; returns ms per batch step."""
        return cplb_batch_tune(self._b, probe_steps)


# ------------------------------------------------------- closure network

def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _ccheck(c, rc):
    if rc:
        raise CplbError(rc, library().cplb_cnn_last_error(c).decode())


def cplb_cnn_num_params() -> int:
    return library().cplb_cnn_num_params()


def cplb_cnn_workspace_bytes(nsamples, H, W) -> int:
    n = ctypes.c_size_t()
    rc = library().cplb_cnn_workspace_bytes(nsamples, H, W, ctypes.byref(n))
    if rc:
        raise CplbError(rc, "cplb_cnn_workspace_bytes rejected the sizes")
    return n.value


def cplb_cnn_create(nsamples, H, W, ws_ptr, ws_bytes, stream_ptr):
    c = ctypes.c_void_p()
    rc = library().cplb_cnn_create(nsamples, H, W, ctypes.c_void_p(ws_ptr), ws_bytes,
                                   ctypes.c_void_p(stream_ptr), ctypes.byref(c))
    if rc:
        raise CplbError(rc, "cplb_cnn_create failed")
    return c


def cplb_cnn_set_params(c, theta):
    _ccheck(c, library().cplb_cnn_set_params(c, _fp(theta)))


def cplb_cnn_init_params(c, seed):
    _ccheck(c, library().cplb_cnn_init_params(c, seed))


def cplb_cnn_get_params(c, out):
    _ccheck(c, library().cplb_cnn_get_params(c, _fp(out)))


def cplb_cnn_set_input_scale(c, scale):
    _ccheck(c, library().cplb_cnn_set_input_scale(c, _fp(scale)))


def cplb_cnn_forward(c, nsamples, planes_ptr, cin, out_ptr):
    _ccheck(c, library().cplb_cnn_forward(c, nsamples, ctypes.c_void_p(planes_ptr), cin,
                                          None if out_ptr is None else ctypes.c_void_p(out_ptr)))


def cplb_cnn_backward(c, target_ptr) -> float:
    loss = ctypes.c_double()
    _ccheck(c, library().cplb_cnn_backward(c, ctypes.c_void_p(target_ptr), ctypes.byref(loss)))
    return loss.value


def cplb_cnn_get_grads(c, out):
    _ccheck(c, library().cplb_cnn_get_grads(c, _fp(out)))


def cplb_cnn_adam(c, lr, beta1, beta2, eps):
    _ccheck(c, library().cplb_cnn_adam(c, lr, beta1, beta2, eps))


def cplb_cnn_last_error(c) -> str:
    return library().cplb_cnn_last_error(c).decode()


def cplb_cnn_destroy(c):
    library().cplb_cnn_destroy(c)


class ClosureNet:
    """The closure network on one GPU: up to `nsamples` H x W samples per
    call.  Inputs and outputs are float32 device tensors."""

    def __init__(self, nsamples, H, W, device="cuda:0", stream=None, seed=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("cplb needs a GPU: torch.cuda.is_available() is False")
        self.torch = torch
        self.nsamples, self.H, self.W = nsamples, H, W
        self.device = torch.device(device)
        nbytes = cplb_cnn_workspace_bytes(nsamples, H, W)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._c = cplb_cnn_create(nsamples, H, W, self.workspace.data_ptr(), nbytes,
                                  self.stream.cuda_stream)
        self.n_params = cplb_cnn_num_params()
        if seed is not None:
            cplb_cnn_init_params(self._c, seed)

    def close(self):
        """Release the network once the work queued on its stream has finished."""
        if getattr(self, "_c", None):
            self.stream.synchronize()
            cplb_cnn_destroy(self._c)
            self._c = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _order(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def set_params(self, theta):
        cplb_cnn_set_params(self._c, np.ascontiguousarray(theta, dtype=np.float32))

    def params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        cplb_cnn_get_params(self._c, out)
        return out

    def grads(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        cplb_cnn_get_grads(self._c, out)
        return out

    def set_input_scale(self, scale):
        sc = np.zeros(16, dtype=np.float32)
        sc[:len(scale)] = scale
        cplb_cnn_set_input_scale(self._c, sc)

    def forward(self, planes, out=None):
        """planes: [B, cin, H, W] float32 device tensor -> [B, 2, H, W], the
        corrections (s1, s2) of c1 and c2, scaled and balanced per sample."""
        torch = self.torch
        assert planes.dtype == torch.float32 and planes.is_contiguous()
        B, cin = int(planes.shape[0]), int(planes.shape[1])
        if out is None:
            out = torch.empty((B, 2, self.H, self.W), dtype=torch.float32, device=self.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == B * 2 * self.H * self.W
        self._order()
        cplb_cnn_forward(self._c, B, planes.data_ptr(), cin, out.data_ptr())
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def infer(self, planes, out=None):
        """Inference (no training buffers): planes [B, cin, H, W] float32
        device tensor -> [B, 2, H, W], equal to forward()."""
        torch = self.torch
        assert planes.dtype == torch.float32 and planes.is_contiguous()
        B, cin = int(planes.shape[0]), int(planes.shape[1])
        if out is None:
            out = torch.empty((B, 2, self.H, self.W), dtype=torch.float32, device=self.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == B * 2 * self.H * self.W
        self._order()
        _ccheck(self._c, library().cplb_cnn_infer(self._c, B, ctypes.c_void_p(planes.data_ptr()),
                                                  cin, ctypes.c_void_p(out.data_ptr())))
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return out

    def set_stream(self, stream):
        """Run every following call on `stream` (a torch stream), after the
        work already queued on the current one."""
        stream.wait_stream(self.stream)
        _ccheck(self._c, library().cplb_cnn_set_stream(self._c, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def backward(self, target) -> float:
        """Loss of the last forward's two output channels (before output
        scale and balance) against target [B, 2, H, W] (FP64), and every
        gradient."""
        assert target.dtype == self.torch.float32 and target.is_contiguous()
        self._order()
        return cplb_cnn_backward(self._c, target.data_ptr())

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        cplb_cnn_adam(self._c, lr, beta1, beta2, eps)

    def set_output_scale(self, scale1, scale2=None):
        """Scales of the two outputs (the second defaults to the first)."""
        scale2 = scale1 if scale2 is None else scale2
        _ccheck(self._c, library().cplb_cnn_set_output_scale(self._c, float(scale1), float(scale2)))


def restrict(fine, factor, out=None, stream=None):
    """Block average of fine planes [n, H f, W f] (float32 device tensor)
    onto [n, H, W] on the GPU (cplb_cnn_restrict)."""
    import torch
    n, Hf, Wf = (int(v) for v in fine.shape)
    H, W = Hf // factor, Wf // factor
    assert H * factor == Hf and W * factor == Wf and fine.dtype == torch.float32
    fine = fine.contiguous()
    if out is None:
        out = torch.empty((n, H, W), dtype=torch.float32, device=fine.device)
    s = stream if stream is not None else torch.cuda.current_stream(fine.device)
    rc = library().cplb_cnn_restrict(ctypes.c_void_p(s.cuda_stream), ctypes.c_void_p(fine.data_ptr()),
                                     n, H, W, factor, ctypes.c_void_p(out.data_ptr()))
    if rc:
        raise CplbError(rc, "cplb_cnn_restrict failed")
    return out
