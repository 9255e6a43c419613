"""Python access to the FP64 CPU oracle (``pbs_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The product path never
imports this module.  Nothing here is shared with the HIP path: the structs are
declared again below, and inputs come as plain dicts of numbers.

Every function wraps one routine of the C oracle; each C routine cites the
passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pbs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over independent lines)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nth", C.c_int), ("ng", C.c_int), ("nz", C.c_int),
                ("ngen", C.c_int), ("x_half", C.c_double), ("y_half", C.c_double), ("th_half", C.c_double),
                ("e_lo", C.c_double), ("e_hi", C.c_double), ("dz", C.c_double)]


class Beam(C.Structure):
    _fields_ = [("e0", C.c_double), ("sigma_e", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("sigma_x", C.c_double), ("sigma_y", C.c_double)]


class Phys(C.Structure):
    _fields_ = [("bk_alpha", C.c_double), ("bk_p", C.c_double), ("e_floor", C.c_double),
                ("highland_es", C.c_double), ("x0_water", C.c_double), ("mp", C.c_double),
                ("kappa0", C.c_double), ("e_c", C.c_double), ("lambda_nuc", C.c_double),
                ("gamma_a", C.c_double), ("gamma_b", C.c_double), ("stopping", C.c_int),
                ("straggling", C.c_int), ("scattering", C.c_int), ("material", C.c_int), ("nuc_bands", C.c_int),
                ("nuc_e", C.c_double * 4), ("nuc_lambda", C.c_double * 4), ("nuc_alpha", C.c_double * 4),
                ("nuc_beta", C.c_double * 4)]


# switches of the physics record that default to 0 (off / water / single nuclear parameters)
_OPT_INT = ("stopping", "straggling", "scattering", "material", "nuc_bands")
_OPT_ARR = ("nuc_e", "nuc_lambda", "nuc_alpha", "nuc_beta")


def _mk(cls, d):
    kw = {}
    for k, t in cls._fields_:
        if k in _OPT_INT:
            kw[k] = int(d.get(k, 0))
        elif k in _OPT_ARR:
            v = list(d.get(k, [0.0] * 4)) + [0.0] * 4
            kw[k] = (C.c_double * 4)(*v[:4])
        else:
            kw[k] = d[k]
    return cls(**kw)


class Tab(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in ("E_face", "E_mid", "dE", "S_face", "sig_tr", "kappa",
                                                      "T_face", "Tp_face")] + \
               [("band", C.POINTER(C.c_int)), ("P1", C.POINTER(C.c_double)), ("P2", C.POINTER(C.c_double))]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.og_gen_elems.restype = C.c_long
        L.og_stopping.restype = C.c_double
        L.og_bethe_water.restype = C.c_double
        L.og_scatpower.restype = C.c_double
        L.og_superbee.restype = C.c_double
        L.og_defl_angle.restype = C.c_double
        for f in ("og_bethe", "og_williams", "og_williams_deriv", "og_rutherford", "og_straggle",
                  "og_straggle_deriv"):
            getattr(L, f).restype = C.c_double
        L.og_max_threads.restype = C.c_int
        L.og_initial.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _opt(a):
    return None if a is None else _p(a)


class Oracle:
    """One configuration (grid + physics).  Arrays are numpy float64."""

    def __init__(self, grid: dict, phys: dict):
        self.gd, self.ph = dict(grid), dict(phys)
        self.g, self.p = _mk(Grid, grid), _mk(Phys, phys)
        g = self.g
        self.G, self.m = g.ng, g.nth - 1
        self.NA, self.NP = self.m * self.m, g.nx * g.ny
        self.gen_shape = (g.ng, 2, self.NA, self.NP)
        G, NA = self.G, self.NA
        self.E_face = np.zeros(G + 1)
        self.E_mid = np.zeros(G)
        self.dE = np.zeros(G)
        self.S_face = np.zeros(G + 1)
        self.sig_tr = np.zeros(G)
        self.kappa = np.zeros(G)
        self.T_face = np.zeros(G + 1)
        self.Tp_face = np.zeros(G + 1)
        self.band = np.zeros(G, dtype=np.int32)
        self.NB = max(1, int(phys.get("nuc_bands", 0)))
        self.P1 = np.zeros((G, G))
        self.P2 = np.zeros((self.NB, NA, NA)) if self.NB > 1 else np.zeros((NA, NA))
        lib().og_tables(C.byref(g), C.byref(self.p), _p(self.E_face), _p(self.E_mid), _p(self.dE),
                        _p(self.S_face), _p(self.sig_tr), _p(self.kappa), _p(self.T_face), _p(self.Tp_face),
                        self.band.ctypes.data_as(C.POINTER(C.c_int)), _p(self.P1), _p(self.P2))
        self.straggling = bool(phys.get("straggling", 0))
        self._tab = Tab(_p(self.E_face), _p(self.E_mid), _p(self.dE), _p(self.S_face), _p(self.sig_tr),
                        _p(self.kappa), _p(self.T_face) if self.straggling else None,
                        _p(self.Tp_face) if self.straggling else None,
                        self.band.ctypes.data_as(C.POINTER(C.c_int)), _p(self.P1), _p(self.P2))

    # geometry helpers (plain restatements of the grid definition)
    @property
    def dx(self):
        return 2 * self.g.x_half / self.g.nx

    @property
    def dy(self):
        return 2 * self.g.y_half / self.g.ny

    @property
    def dth(self):
        return 2 * self.g.th_half / self.g.nth

    def theta(self):
        return -self.g.th_half + (np.arange(self.m) + 1) * self.dth

    def zeros_state(self):
        return np.zeros((self.g.ngen,) + self.gen_shape)

    def initial(self, beam: dict):
        st = self.zeros_state()
        b = _mk(Beam, beam)
        rc = lib().og_initial(C.byref(self.g), C.byref(b), _p(self.E_face), _p(st[0]))
        if rc != 0:
            raise ValueError("oracle initial state needs an even number of angular nodes")
        return st

    # sub-operators -------------------------------------------------------
    def _strag(self):
        return (_p(self.T_face), _p(self.Tp_face)) if self.straggling else (None, None)

    def energy_rhs_line(self, rho, x1, x2, Q=None):
        o1, o2 = np.zeros(self.G), np.zeros(self.G)
        lib().og_energy_rhs(C.byref(self.g), _p(self.S_face), _p(self.dE), _p(self.kappa), *self._strag(),
                            C.c_double(rho),
                            _p(np.ascontiguousarray(x1, dtype=np.float64)),
                            _p(np.ascontiguousarray(x2, dtype=np.float64)),
                            _opt(None if Q is None else np.ascontiguousarray(Q, dtype=np.float64)), _p(o1), _p(o2))
        return o1, o2

    def energy_cn(self, gen_state, rho, h, Qn=None, Qs=None):
        """In place CN step of one generation ([G,2,NA,NP])."""
        lib().og_energy_cn(C.byref(self.g), _p(self.S_face), _p(self.dE), _p(self.kappa), *self._strag(),
                           _p(rho), C.c_double(h), _p(gen_state), _opt(Qn), _opt(Qs))

    def energy_all(self, state, rho, h):
        dep = np.zeros(self.NP)
        lib().og_energy_all_api(C.byref(self.g), C.byref(self._tab), _p(rho), C.c_double(h), _p(state), _p(dep))
        return dep

    def source(self, prev_gen, rho):
        Q = np.zeros((self.G, self.NA, self.NP))
        lib().og_source(C.byref(self.g), _p(self.dE), _p(self.kappa), _p(self.P1), _p(self.P2),
                        self.band.ctypes.data_as(C.POINTER(C.c_int)), _p(rho), _p(prev_gen), _p(Q))
        return Q

    def transport_cn(self, gen_state, h):
        lib().og_transport_cn(C.byref(self.g), C.c_double(h), _p(gen_state))

    def transport_plane(self, plane, cx, cy, h, dx=None, dy=None):
        pl = np.ascontiguousarray(plane, dtype=np.float64).copy()
        nx, ny = pl.shape
        lib().og_transport_plane_api(nx, ny, C.c_double(dx or self.dx), C.c_double(dy or self.dy),
                                     C.c_double(cx), C.c_double(cy), C.c_double(h), _p(pl))
        return pl

    def angular_cn(self, gen_state, rho, h):
        lib().og_angular_cn(C.byref(self.g), _p(self.sig_tr), _p(rho), C.c_double(h), _p(gen_state))

    def energy_content(self, gen_state):
        out = np.zeros(self.NP)
        lib().og_energy_content(C.byref(self.g), _p(self.E_mid), _p(self.dE), _p(gen_state), _p(out))
        return out

    def number_content(self, gen_state):
        out = np.zeros(self.NP)
        lib().og_number_content(C.byref(self.g), _p(self.dE), _p(gen_state), _p(out))
        return out

    # the march -------------------------------------------------------------
    def run(self, beam: dict, rho, state=None, order=2):
        """Full depth march.  rho: [nz, nx, ny].  Returns (dose [nz,nx,ny], final state).
        order 2: Strang steps; order 4: Richardson-extrapolated Strang steps."""
        g = self.g
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(g.nz, g.nx * g.ny)
        if state is None:
            state = self.initial(beam)
        dose = np.zeros((g.nz, g.nx * g.ny))
        fn = lib().og_run_extrapolated if order == 4 else lib().og_run
        fn(C.byref(g), C.byref(self._tab), _p(rho), _p(state), _p(dose))
        return dose.reshape(g.nz, g.nx, g.ny), state

    def run_records(self, beam: dict, rho, state=None):
        """Full march of a K = 1 grid (ngen = 2) with the per-layer records of the surrogate:
        returns (dose, final state, rec [4, nz, nx, ny]) with rec = injected energy into
        generation 1, energy and number content of generation 0 after the opening half-step,
        deposit of generation 0 alone (MeV)."""
        g = self.g
        if g.ngen != 2:
            raise ValueError("records need ngen = 2")
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(g.nz, g.nx * g.ny)
        if state is None:
            state = self.initial(beam)
        dose = np.zeros((g.nz, g.nx * g.ny))
        rec = np.zeros((4, g.nz, g.nx * g.ny))
        lib().og_run_records(C.byref(g), C.byref(self._tab), _p(rho), _p(state), _p(dose), _p(rec))
        return dose.reshape(g.nz, g.nx, g.ny), state, rec.reshape(4, g.nz, g.nx, g.ny)


def set_threads(n: int) -> None:
    """Number of OpenMP threads of the oracle's parallel loops (results do not depend on it)."""
    lib().og_set_threads(int(n))


def max_threads() -> int:
    return lib().og_max_threads()


def stopping(phys: dict, E: float) -> float:
    return lib().og_stopping(C.byref(_mk(Phys, phys)), C.c_double(E))


def bethe_water(E: float, mp: float = 938.272) -> float:
    """Bethe-Bloch mass stopping power of water (App. A.1), MeV cm^2/g."""
    return lib().og_bethe_water(C.c_double(E), C.c_double(mp))


MEDIA = {"water": 0, "bone": 1, "air": 2}


def bethe(material: int, E: float, mp: float = 938.272) -> float:
    """Bethe-Bloch mass stopping power of a medium (0 water, 1 bone, 2 air), MeV cm^2/g (App. A.1)."""
    return lib().og_bethe(int(material), C.c_double(E), C.c_double(mp))


def williams(material: int, E: float, mp: float = 938.272) -> float:
    """Williams straggling coefficient of a medium, MeV^2 cm^2/g (App. A.2)."""
    return lib().og_williams(int(material), C.c_double(E), C.c_double(mp))


def williams_deriv(material: int, E: float, mp: float = 938.272) -> float:
    return lib().og_williams_deriv(int(material), C.c_double(E), C.c_double(mp))


def rutherford(material: int, E: float, mp: float = 938.272) -> float:
    """Screened-Rutherford momentum-transfer cross section of a medium, cm^2/g (App. A.3)."""
    return lib().og_rutherford(int(material), C.c_double(E), C.c_double(mp))


def scatpower(phys: dict, E: float) -> float:
    return lib().og_scatpower(C.byref(_mk(Phys, phys)), C.c_double(E))


def superbee(th: float) -> float:
    return lib().og_superbee(C.c_double(th))


def defl_angle(u, v, up, vp) -> float:
    return lib().og_defl_angle(C.c_double(u), C.c_double(v), C.c_double(up), C.c_double(vp))
