"""Thin ctypes binding of libpbsplit (include/pbsplit.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch supplies the device workspace and the HIP stream.  If the
shared library is missing the import fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpbsplit.so")

PBS_OK, PBS_EINVAL, PBS_ESTATE, PBS_ENOMEM, PBS_EDEVICE, PBS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PBS_FP32, PBS_FP64 = 0, 1
PBS_OP_E, PBS_OP_T, PBS_OP_A = 1, 2, 3
PBS_SRC_FP32, PBS_SRC_BF16X3, PBS_SRC_BF16X2, PBS_SRC_BF16X1 = 0, 1, 2, 3
PBS_SCHED_AUTO, PBS_SCHED_ONE_STREAM, PBS_SCHED_TWO_STREAMS = 0, 1, 2
PBS_STOP_BRAGG_KLEEMAN, PBS_STOP_BETHE = 0, 1
PBS_SCAT_HIGHLAND, PBS_SCAT_RUTHERFORD = 0, 1
PBS_MAT_WATER, PBS_MAT_BONE, PBS_MAT_AIR = 0, 1, 2
_NAMES = {0: "PBS_OK", -1: "PBS_EINVAL", -2: "PBS_ESTATE", -3: "PBS_ENOMEM", -4: "PBS_EDEVICE",
          -5: "PBS_EUNSUPPORTED"}

EXPORTS = ["pbs_create", "pbs_workspace_bytes", "pbs_bind", "pbs_set_phantom", "pbs_set_beam", "pbs_step_depth",
           "pbs_run_beam", "pbs_get_dose", "pbs_get_state", "pbs_set_state", "pbs_apply", "pbs_set_source_precision",
           "pbs_profile", "pbs_set_schedule",
           "pbs_profile_read", "pbs_last_error", "pbs_destroy", "pbs_batch_create", "pbs_batch_workspace_bytes",
           "pbs_batch_bind", "pbs_batch_set_phantom", "pbs_batch_prepare", "pbs_batch_run", "pbs_batch_get_dose", "pbs_batch_tuning",
           "pbs_batch_last_error", "pbs_batch_destroy", "pbs_set_surrogate", "pbs_surrogate_sample",
           "pbs_surrogate_records", "pbs_surrogate_report", "pbs_net_param_count", "pbs_net_create",
           "pbs_net_workspace_bytes", "pbs_net_bind", "pbs_net_set_params", "pbs_net_get_params", "pbs_net_forward",
           "pbs_net_gradient", "pbs_net_train_step", "pbs_net_last_error", "pbs_net_destroy", "pbs_bind_static",
           "pbs_set_splitting", "pbs_set_phantom_voxels", "pbs_resample_phantom"]
PBS_STATIC_SCRATCH_BYTES = 64 << 20
_NORET = ("pbs_last_error", "pbs_destroy", "pbs_batch_last_error", "pbs_batch_destroy", "pbs_net_last_error",
          "pbs_net_destroy")
PBS_NET_MAGIC, PBS_NET_VERSION, PBS_NET_CIN, SUR_NFEAT = 0x4E534250, 1, 8, 8
REPORT_KEYS = ["residual", "fallback", "budget", "predicted", "scale", "injected", "own_deposit", "leak",
               "primary_deposit", "primary_escape"]
KINDS = ["epass", "tpass", "apass", "qgemm", "dose"]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nth", C.c_int), ("ng", C.c_int), ("nz", C.c_int),
                ("ngen", C.c_int), ("x_half", C.c_double), ("y_half", C.c_double), ("th_half", C.c_double),
                ("e_lo", C.c_double), ("e_hi", C.c_double), ("dz", C.c_double)]


class Beam(C.Structure):
    _fields_ = [("e0", C.c_double), ("sigma_e", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("sigma_x", C.c_double), ("sigma_y", C.c_double)]


class Physics(C.Structure):
    _fields_ = [("bk_alpha", C.c_double), ("bk_p", C.c_double), ("e_floor", C.c_double),
                ("highland_es", C.c_double), ("x0_water", C.c_double), ("mp", C.c_double),
                ("kappa0", C.c_double), ("e_c", C.c_double), ("lambda_nuc", C.c_double),
                ("gamma_a", C.c_double), ("gamma_b", C.c_double), ("stopping", C.c_int),
                ("straggling", C.c_int), ("scattering", C.c_int), ("material", C.c_int), ("nuc_bands", C.c_int),
                ("nuc_e", C.c_double * 4), ("nuc_lambda", C.c_double * 4), ("nuc_alpha", C.c_double * 4),
                ("nuc_beta", C.c_double * 4)]


class PbsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libpbsplit.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, sz, D = C.c_void_p, C.c_size_t, C.POINTER(C.c_double)
        L.pbs_create.argtypes = [C.POINTER(Grid), C.POINTER(Physics), C.c_int, C.POINTER(vp)]
        L.pbs_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
        L.pbs_bind.argtypes = [vp, vp, sz, vp]
        L.pbs_bind_static.argtypes = [vp, vp]
        L.pbs_set_phantom.argtypes = [vp, D, sz]
        L.pbs_set_phantom_voxels.argtypes = [vp, D, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                             C.c_double, C.c_double]
        L.pbs_resample_phantom.argtypes = [C.POINTER(Grid), D, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                           C.c_double, C.c_double, C.c_double, D]
        L.pbs_set_beam.argtypes = [vp, C.POINTER(Beam)]
        L.pbs_step_depth.argtypes = [vp, C.c_int, C.POINTER(C.c_int)]
        L.pbs_run_beam.argtypes = [vp]
        L.pbs_get_dose.argtypes = [vp, vp, sz, C.c_int]
        L.pbs_get_state.argtypes = [vp, D, sz]
        L.pbs_set_state.argtypes = [vp, D, sz]
        L.pbs_apply.argtypes = [vp, C.c_int, C.c_int, C.c_double]
        L.pbs_set_source_precision.argtypes = [vp, C.c_int]
        L.pbs_profile.argtypes = [vp, C.c_int]
        L.pbs_set_schedule.argtypes = [vp, C.c_int]
        L.pbs_set_splitting.argtypes = [vp, C.c_int]
        L.pbs_profile_read.argtypes = [vp, D, C.POINTER(C.c_long), C.c_int]
        L.pbs_last_error.argtypes = [vp]
        L.pbs_last_error.restype = C.c_char_p
        L.pbs_destroy.argtypes = [vp]
        L.pbs_destroy.restype = None
        L.pbs_batch_create.argtypes = [C.POINTER(Grid), C.POINTER(Beam), C.c_int, C.POINTER(Physics), C.c_int,
                                       C.POINTER(vp)]
        L.pbs_batch_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
        L.pbs_batch_bind.argtypes = [vp, vp, sz, vp]
        L.pbs_batch_set_phantom.argtypes = [vp, C.c_int, D, sz]
        L.pbs_batch_prepare.argtypes = [vp]
        L.pbs_batch_run.argtypes = [vp]
        L.pbs_batch_get_dose.argtypes = [vp, C.c_int, D, sz]
        L.pbs_batch_tuning.argtypes = [vp, C.POINTER(C.c_int)]
        L.pbs_batch_last_error.argtypes = [vp]
        L.pbs_batch_last_error.restype = C.c_char_p
        L.pbs_batch_destroy.argtypes = [vp]
        L.pbs_batch_destroy.restype = None
        F = C.POINTER(C.c_float)
        L.pbs_set_surrogate.argtypes = [vp, vp, sz, C.c_double]
        L.pbs_surrogate_sample.argtypes = [vp, vp, vp, sz]
        L.pbs_surrogate_records.argtypes = [vp, D, sz]
        L.pbs_surrogate_report.argtypes = [vp, D, C.c_int]
        L.pbs_net_param_count.argtypes = [C.POINTER(sz)]
        L.pbs_net_create.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(vp)]
        L.pbs_net_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
        L.pbs_net_bind.argtypes = [vp, vp, sz, vp]
        L.pbs_net_set_params.argtypes = [vp, F, sz]
        L.pbs_net_get_params.argtypes = [vp, F, sz]
        L.pbs_net_forward.argtypes = [vp, vp, vp, C.c_int]
        L.pbs_net_gradient.argtypes = [vp, vp, vp, C.c_int, F, sz, D]
        L.pbs_net_train_step.argtypes = [vp, vp, vp, C.c_int, C.c_double, vp]
        L.pbs_net_last_error.argtypes = [vp]
        L.pbs_net_last_error.restype = C.c_char_p
        L.pbs_net_destroy.argtypes = [vp]
        L.pbs_net_destroy.restype = None
        for n in EXPORTS:
            if n not in _NORET:
                getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


# switches of the physics record that default to 0 (range fit, no straggling, Highland, water, one set of
# nuclear parameters) when a dict does not name them
_OPT_INT = ("stopping", "straggling", "scattering", "material", "nuc_bands")
_OPT_ARR = ("nuc_e", "nuc_lambda", "nuc_alpha", "nuc_beta")


def _mk(cls, d):
    kw = {}
    for k, _ in cls._fields_:
        if k in _OPT_INT:
            kw[k] = int(d.get(k, 0))
        elif k in _OPT_ARR:
            v = (list(d.get(k, [])) + [0.0] * 4)[:4]
            kw[k] = (C.c_double * 4)(*v)
        else:
            kw[k] = d[k]
    return cls(**kw)


def resample_phantom(grid: dict, vox, spacing, corner) -> np.ndarray:
    """pbs_resample_phantom: the nearest-voxel densities of a voxel phantom on a grid (host only)."""
    v = np.ascontiguousarray(vox, dtype=np.float64)
    nz, nx, ny = v.shape
    out = np.zeros((grid["nz"], grid["nx"], grid["ny"]))
    rc = lib().pbs_resample_phantom(C.byref(_mk(Grid, grid)), v.ctypes.data_as(C.POINTER(C.c_double)), nz, nx, ny,
                                    float(spacing[0]), float(spacing[1]), float(spacing[2]), float(corner[0]),
                                    float(corner[1]), out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != PBS_OK:
        raise PbsError(rc, "pbs_resample_phantom rejected the phantom")
    return out


SURROGATE_WEIGHTS = os.path.join(_HERE, "data", "surrogate_c5.pbsn")


def surrogate_weights() -> bytes:
    """Weights of the generation-1 surrogate trained on the config-5 workload (written by
    train_surrogate.py)."""
    with open(SURROGATE_WEIGHTS, "rb") as f:
        return f.read()


def param_count() -> int:
    n = C.c_size_t()
    rc = lib().pbs_net_param_count(C.byref(n))
    if rc != PBS_OK:
        raise PbsError(rc, "pbs_net_param_count")
    return n.value


def pack_weights(params, leak) -> bytes:
    """Weights blob of pbs_set_surrogate: 64-byte header + FP32 parameters.  leak: coefficients
    (l0, l1, l2) of the leak model l(x) = l0 + l1 x + l2 x^2 (a scalar means a constant)."""
    p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
    head = np.zeros(6, dtype=np.float64)   # leak model + 3 reserved: 48 bytes after the 16-byte ids
    lk = np.atleast_1d(np.asarray(leak, dtype=np.float64))
    head[:lk.size] = lk
    u = np.array([PBS_NET_MAGIC, PBS_NET_VERSION, p.size, SUR_NFEAT], dtype=np.uint32)
    return u.tobytes() + head.tobytes() + p.tobytes()


def unpack_weights(blob: bytes):
    """(params float32, leak model coefficients) from a weights blob."""
    u = np.frombuffer(blob[:16], dtype=np.uint32)
    if u[0] != PBS_NET_MAGIC or u[1] != PBS_NET_VERSION:
        raise ValueError("not a pbsplit network blob")
    leak = np.frombuffer(blob[16:40], dtype=np.float64).copy()
    return np.frombuffer(blob[64:], dtype=np.float32).copy(), leak


class Solver:
    """One libpbsplit context bound to a torch-allocated workspace on `device`.

    surrogate: None, "record" (plain march that keeps the per-slice surrogate records) or a weights
    blob (bytes) for the surrogate of generation 1 with fallback at residual_tol.
    static_scratch: bind to the library's own device scratch (pbs_bind_static) instead of a torch
    workspace; nothing is allocated on the device.
    order: splitting in depth, 2 (Strang) or 4 (Richardson-extrapolated Strang steps)."""

    def __init__(self, grid: dict, phys: dict, precision: str = "fp32", device="cuda:0", stream=None,
                 surrogate=None, residual_tol: float = 1e-2, static_scratch: bool = False, order: int = 2):
        import torch

        self.torch = torch
        self.L = lib()
        self.grid = dict(grid)
        self.g = _mk(Grid, grid)
        self.prec = PBS_FP64 if precision == "fp64" else PBS_FP32
        self.ctx = C.c_void_p()
        rc = self.L.pbs_create(C.byref(self.g), C.byref(_mk(Physics, phys)), self.prec, C.byref(self.ctx))
        if rc != PBS_OK:
            raise PbsError(rc, "pbs_create rejected the grid / physics")
        if surrogate is not None:
            if isinstance(surrogate, str):
                if surrogate != "record":
                    raise ValueError("surrogate must be None, 'record' or a weights blob")
                self._check(self.L.pbs_set_surrogate(self.ctx, None, 0, 0.0))
            else:
                self._blob = C.create_string_buffer(bytes(surrogate), len(surrogate))
                self._check(self.L.pbs_set_surrogate(self.ctx, C.cast(self._blob, C.c_void_p), len(surrogate),
                                                     float(residual_tol)))
        if order != 2:
            self._check(self.L.pbs_set_splitting(self.ctx, int(order)))
        nb = C.c_size_t()
        self._check(self.L.pbs_workspace_bytes(self.ctx, C.byref(nb)))
        self.ws_bytes = nb.value
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if static_scratch:
            self._ws = None
            self.ws_ptr = None
            with torch.cuda.device(self.device):
                self._check(self.L.pbs_bind_static(self.ctx, C.c_void_p(self.stream.cuda_stream)))
        else:
            self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            self.ws_ptr = base + ((256 - base % 256) % 256)
            self._check(self.L.pbs_bind(self.ctx, C.c_void_p(self.ws_ptr), self.ws_bytes,
                                        C.c_void_p(self.stream.cuda_stream)))
        m = grid["nth"] - 1
        self.NA = m * m
        self.NP = grid["nx"] * grid["ny"]
        self.state_shape = (grid["ngen"], grid["ng"], 2, self.NA, self.NP)

    def _check(self, rc):
        if rc != PBS_OK:
            raise PbsError(rc, self.L.pbs_last_error(self.ctx).decode())

    def set_phantom(self, rho):
        r = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        self._check(self.L.pbs_set_phantom(self.ctx, r.ctypes.data_as(C.POINTER(C.c_double)), r.size))

    def set_phantom_voxels(self, vox, spacing, corner):
        """A voxel phantom [nz][nx][ny] with spacing (dz, dx, dy) and lateral corner (x_lo, y_lo) in the beam's
        frame, resampled onto the grid by the nearest voxel in the library."""
        v = np.ascontiguousarray(vox, dtype=np.float64)
        nz, nx, ny = v.shape
        self._check(self.L.pbs_set_phantom_voxels(self.ctx, v.ctypes.data_as(C.POINTER(C.c_double)), nz, nx, ny,
                                                  float(spacing[0]), float(spacing[1]), float(spacing[2]),
                                                  float(corner[0]), float(corner[1])))

    def set_beam(self, beam: dict):
        self._check(self.L.pbs_set_beam(self.ctx, C.byref(_mk(Beam, beam))))

    def step(self, n: int) -> int:
        s = C.c_int()
        self._check(self.L.pbs_step_depth(self.ctx, int(n), C.byref(s)))
        return s.value

    def run(self):
        self._check(self.L.pbs_run_beam(self.ctx))

    def dose(self) -> np.ndarray:
        g = self.grid
        out = np.zeros((g["nz"], g["nx"], g["ny"]))
        self._check(self.L.pbs_get_dose(self.ctx, out.ctypes.data_as(C.c_void_p), out.size, 0))
        return out

    def dose_device(self, out):
        """Enqueue the dose into a float64 torch tensor on the device."""
        assert out.dtype == self.torch.float64 and out.is_cuda and out.is_contiguous()
        self._check(self.L.pbs_get_dose(self.ctx, C.c_void_p(out.data_ptr()), out.numel(), 1))

    def state(self) -> np.ndarray:
        out = np.zeros(self.state_shape)
        self._check(self.L.pbs_get_state(self.ctx, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out

    def set_state(self, st):
        s = np.ascontiguousarray(st, dtype=np.float64).reshape(-1)
        self._check(self.L.pbs_set_state(self.ctx, s.ctypes.data_as(C.POINTER(C.c_double)), s.size))

    def apply(self, op: int, layer: int, h: float):
        self._check(self.L.pbs_apply(self.ctx, int(op), int(layer), float(h)))

    def set_source_precision(self, mode: int):
        self._check(self.L.pbs_set_source_precision(self.ctx, int(mode)))

    def set_schedule(self, mode: int):
        """PBS_SCHED_AUTO / ONE_STREAM / TWO_STREAMS: which streams the depth march uses (bitwise the same
        result)."""
        self._check(self.L.pbs_set_schedule(self.ctx, int(mode)))

    def profile(self, enable: bool):
        self._check(self.L.pbs_profile(self.ctx, 1 if enable else 0))

    def profile_read(self) -> dict:
        n = len(KINDS)
        ms = (C.c_double * n)()
        cnt = (C.c_long * n)()
        self._check(self.L.pbs_profile_read(self.ctx, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KINDS)}

    def surrogate_sample(self, x, t):
        """Features (uint8-viewed or bfloat16 tensor of nz*nx*ny*8 values) and FP32 targets into
        device tensors."""
        g = self.grid
        self._check(self.L.pbs_surrogate_sample(self.ctx, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                                g["nz"]))

    def surrogate_records(self) -> np.ndarray:
        g = self.grid
        out = np.zeros((4, g["nz"], g["nx"], g["ny"]))
        self._check(self.L.pbs_surrogate_records(self.ctx, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out

    def surrogate_report(self) -> dict:
        out = (C.c_double * 10)()
        self._check(self.L.pbs_surrogate_report(self.ctx, out, 10))
        return {k: out[i] for i, k in enumerate(REPORT_KEYS)}

    def close(self):
        if getattr(self, "ctx", None):
            self.L.pbs_destroy(self.ctx)
            self.ctx = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many beams of one shape class marched together (pbs_batch_*).  beams: list of dicts with
    keys grid, beam, rho (as produced by inputs.config4)."""

    def __init__(self, beams: list, phys: dict, wave: int = 0, device="cuda:0", stream=None):
        import torch

        self.L = lib()
        self.n = len(beams)
        grids = (Grid * self.n)(*[_mk(Grid, b["grid"]) for b in beams])
        bms = (Beam * self.n)(*[_mk(Beam, b["beam"]) for b in beams])
        self.shapes = [(b["grid"]["nz"], b["grid"]["nx"], b["grid"]["ny"]) for b in beams]
        self.h = C.c_void_p()
        rc = self.L.pbs_batch_create(grids, bms, self.n, C.byref(_mk(Physics, phys)), int(wave), C.byref(self.h))
        if rc != PBS_OK:
            raise PbsError(rc, "pbs_batch_create rejected the beams")
        nb = C.c_size_t()
        self._check(self.L.pbs_batch_workspace_bytes(self.h, C.byref(nb)))
        self.ws_bytes = nb.value
        self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=torch.device(device))
        base = self._ws.data_ptr()
        ptr = base + ((256 - base % 256) % 256)
        # a stream of its own (default priority): the march is captured into a graph
        self.stream = stream if stream is not None else torch.cuda.Stream(device=torch.device(device))
        torch.cuda.current_stream(torch.device(device)).synchronize()
        self._check(self.L.pbs_batch_bind(self.h, C.c_void_p(ptr), self.ws_bytes, C.c_void_p(self.stream.cuda_stream)))
        for i, b in enumerate(beams):
            r = np.ascontiguousarray(b["rho"], dtype=np.float64).reshape(-1)
            self._check(self.L.pbs_batch_set_phantom(self.h, i, r.ctypes.data_as(C.POINTER(C.c_double)), r.size))

    def _check(self, rc):
        if rc != PBS_OK:
            raise PbsError(rc, self.L.pbs_batch_last_error(self.h).decode())

    def prepare(self):
        """Autotune and capture every wave's graph (otherwise done by the first run)."""
        self._check(self.L.pbs_batch_prepare(self.h))

    def run(self):
        self._check(self.L.pbs_batch_run(self.h))

    def dose(self, i: int) -> np.ndarray:
        out = np.zeros(self.shapes[i])
        self._check(self.L.pbs_batch_get_dose(self.h, int(i), out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out

    def tuning(self) -> dict:
        t = (C.c_int * 3)()
        self._check(self.L.pbs_batch_tuning(self.h, t))
        return {"gemm_kernel": ["global", "lds256", "lds128"][t[0]], "tpass_waves_per_block": t[1],
                "apass_cells_per_block": t[2]}

    def close(self):
        if getattr(self, "h", None):
            self.L.pbs_batch_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The surrogate network with its training state (pbs_net_*), bound to a torch workspace."""

    def __init__(self, H: int, W: int, max_batch: int, device="cuda:0", stream=None):
        import torch

        self.torch = torch
        self.L = lib()
        self.H, self.W, self.max_batch = H, W, max_batch
        self.h = C.c_void_p()
        rc = self.L.pbs_net_create(int(H), int(W), int(max_batch), C.byref(self.h))
        if rc != PBS_OK:
            raise PbsError(rc, "pbs_net_create rejected the shape")
        self.npar = param_count()
        nb = C.c_size_t()
        self._check(self.L.pbs_net_workspace_bytes(self.h, C.byref(nb)))
        self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=torch.device(device))
        base = self._ws.data_ptr()
        ptr = base + ((256 - base % 256) % 256)
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self._check(self.L.pbs_net_bind(self.h, C.c_void_p(ptr), nb.value, C.c_void_p(self.stream.cuda_stream)))

    def _check(self, rc):
        if rc != PBS_OK:
            raise PbsError(rc, self.L.pbs_net_last_error(self.h).decode())

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32).reshape(-1)
        self._check(self.L.pbs_net_set_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))

    def params(self) -> np.ndarray:
        a = np.zeros(self.npar, dtype=np.float32)
        self._check(self.L.pbs_net_get_params(self.h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))
        return a

    def forward(self, x, y):
        """x: bfloat16 tensor [n, H, W, 8] on the device; y: float32 tensor [n, H, W] (written)."""
        self._check(self.L.pbs_net_forward(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                           int(x.shape[0])))

    def gradient(self, x, t):
        g = np.zeros(self.npar, dtype=np.float32)
        loss = C.c_double()
        self._check(self.L.pbs_net_gradient(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                            int(x.shape[0]), g.ctypes.data_as(C.POINTER(C.c_float)), g.size,
                                            C.byref(loss)))
        return g, loss.value

    def train_step(self, x, t, lr: float, loss_out=None):
        """One Adam step; loss_out: optional float64 device tensor element receiving the loss."""
        lp = C.c_void_p(loss_out.data_ptr()) if loss_out is not None else None
        self._check(self.L.pbs_net_train_step(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                              int(x.shape[0]), float(lr), lp))

    def close(self):
        if getattr(self, "h", None):
            self.L.pbs_net_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
