"""ctypes wrapper of the FP64 CPU oracle (oracle/pic_oracle.c; the 3D one is in oracle/pic3.py).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by the
CPU-baseline leg of bench.py.  The product package never imports it.

Parity unpinned (no closed form or printed value fixes them): the choice of the
energy-conserving gather variant (only exact uniform and linear fields pin the gather),
quantitative PML reflection (only absorption and its growth with depth are pinned), and the
nonlinear laser-wakefield state beyond agreement with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libpic_oracle.so")

FIELDS = ["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "Exo", "Eyo", "Ezo",
          "Exb", "Eyb", "Ezb", "Byx", "Eyx", "Bxo", "Byo", "Bzo"]
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}


_SOURCES = ("pic_oracle.c", "pic_oracle3.c", "pic_oracle.h", "pic_oracle3.h")


def build(force: bool = False) -> str:
    """Compiles the 2-1/2D and the 3D references into one shared library."""
    srcs = [os.path.join(_HERE, f) for f in _SOURCES]
    newest = max(os.path.getmtime(f) for f in srcs)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               *[f for f in srcs if f.endswith(".c")], "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [("nx", C.c_int), ("nz", C.c_int), ("dx_um", C.c_double), ("dz_um", C.c_double),
                ("pml_cells", C.c_int), ("periodic_x", C.c_int), ("periodic_z", C.c_int),
                ("ck_alpha", C.c_double), ("ck_beta", C.c_double), ("ck_gamma", C.c_double),
                ("theta", C.c_double), ("cfl_fraction", C.c_double), ("filter_npass", C.c_int),
                ("filter_compensate", C.c_int), ("gamma_boost", C.c_double),
                ("moving_window", C.c_int), ("seed", C.c_uint64), ("filter_strides", C.c_int),
                ("gather_kind", C.c_int), ("pusher", C.c_int), ("pml_kind", C.c_int)]


class _Plasma(C.Structure):
    _fields_ = [("n0_cm3", C.c_double), ("ramp_um", C.c_double), ("start_um", C.c_double),
                ("ppc", C.c_int), ("ion_mode", C.c_int)]


class _Laser(C.Structure):
    _fields_ = [("lambda_um", C.c_double), ("a0", C.c_double), ("waist_um", C.c_double),
                ("fwhm_fs", C.c_double), ("z_antenna_um", C.c_double), ("t_peak_fs", C.c_double),
                ("pol", C.c_int)]


class _Beam(C.Structure):
    _fields_ = [("beta_b", C.c_double), ("z_inj_um", C.c_double), ("test_only", C.c_int)]


class _Info(C.Structure):
    _fields_ = [("dt", C.c_double), ("dt_crit", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_double), ("v_window", C.c_double), ("n0_norm", C.c_double),
                ("e0_norm", C.c_double), ("omega", C.c_double), ("alpha2", C.c_double),
                ("beta2", C.c_double), ("antenna_weight", C.c_double), ("stored_x", C.c_int),
                ("stored_z", C.c_int), ("pml_x", C.c_int), ("pml_z", C.c_int),
                ("step", C.c_long), ("time", C.c_double), ("shift", C.c_long),
                ("next_row", C.c_long)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        D = C.POINTER(C.c_double)
        U = C.POINTER(C.c_uint32)
        _lib.orc_create.restype = P
        _lib.orc_create.argtypes = [C.POINTER(_Cfg)]
        _lib.orc_destroy.argtypes = [P]
        _lib.orc_init_plasma.argtypes = [P, C.POINTER(_Plasma)]
        _lib.orc_init_laser.argtypes = [P, C.POINTER(_Laser)]
        _lib.orc_add_station.argtypes = [P, C.c_double, C.c_int]
        _lib.orc_step.argtypes = [P, C.c_int]
        for n in ["faraday", "stations", "particles", "filter", "ampere", "advance"]:
            getattr(_lib, "orc_stage_" + n).argtypes = [P]
        _lib.orc_get_info.argtypes = [P, C.POINTER(_Info)]
        _lib.orc_cfl_2d.restype = C.c_double
        _lib.orc_cfl_2d.argtypes = [C.c_double] * 6
        _lib.orc_cfl_3d.restype = C.c_double
        _lib.orc_cfl_3d.argtypes = [C.c_double] * 7
        _lib.orc_get_field.argtypes = [P, C.c_int, D]
        _lib.orc_set_field.argtypes = [P, C.c_int, D]
        _lib.orc_num_particles.restype = C.c_long
        _lib.orc_num_particles.argtypes = [P, C.c_int]
        _lib.orc_get_particles.argtypes = [P, C.c_int, U, D, D, D, D, D, D]
        _lib.orc_set_electrons.argtypes = [P, C.c_long, U, D, D, D, D, D, D]
        _lib.orc_set_ions.argtypes = [P, C.c_long, U, D, D, D]
        _lib.orc_get_antenna.argtypes = [P, D]
        _lib.orc_set_antenna.argtypes = [P, D]
        _lib.orc_set_clock.argtypes = [P, C.c_long, C.c_double, C.c_long, C.c_long]
        _lib.orc_energy.argtypes = [P, D]
        _lib.orc_gauss_residual.argtypes = [P, D]
        _lib.orc_charge_density.argtypes = [P, D]
        _lib.orc_station_samples.restype = C.c_long
        _lib.orc_station_samples.argtypes = [P, C.c_int, D, C.c_long]
        _lib.orc_shape3.restype = C.c_double
        _lib.orc_shape3.argtypes = [C.c_double]
        _lib.orc_boris.argtypes = [C.c_double, C.c_double, D, D, D]
        _lib.orc_vay.argtypes = [C.c_double, C.c_double, D, D, D]
        _lib.orc_gather_at.argtypes = [P, C.c_double, C.c_double, D]
        _lib.orc_deposit_one.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_double]
        _lib.orc_add_beam.argtypes = [P, C.POINTER(_Beam), C.c_long, D, D, D, D, D, D, C.c_long]
        _lib.orc_beam_state.restype = C.c_long
        _lib.orc_beam_state.argtypes = [P, D]
        _lib.orc_beam_history.restype = C.c_long
        _lib.orc_beam_history.argtypes = [P, D, C.c_long]
        _lib.orc_beam_transform.argtypes = [P, C.POINTER(_Beam), C.c_double, C.c_double, C.c_double,
                                            C.c_double, C.c_double, D]
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_threads.restype = C.c_int
        _lib.orc_splitmix64.restype = C.c_uint64
        _lib.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


class Oracle:
    """One FP64 reference simulation."""

    def __init__(self, config: dict):
        L = lib()
        c = _Cfg(**{k: config.get(k, {"filter_strides": 1, "gather_kind": 0, "pusher": 0, "pml_kind": 0}[k]) if k in ("filter_strides", "gather_kind", "pusher", "pml_kind") else config[k] for k, _ in _Cfg._fields_})
        self._h = L.orc_create(C.byref(c))
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self.config = dict(config)

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- set-up -------------------------------------------------------------------
    def init_plasma(self, p: dict):
        if lib().orc_init_plasma(self._h, C.byref(_Plasma(**p))) != 0:
            raise ValueError("bad plasma")

    def init_laser(self, l: dict):
        if lib().orc_init_laser(self._h, C.byref(_Laser(**l))) != 0:
            raise ValueError("bad laser")

    def add_station(self, z_lab_um: float, capacity: int = 100000) -> int:
        return lib().orc_add_station(self._h, z_lab_um, capacity)

    @classmethod
    def from_workload(cls, w: dict, laser=True, plasma=True, stations=()):
        o = cls(w["config"])
        if plasma and w.get("plasma"):
            o.init_plasma(w["plasma"])
        if laser and w.get("laser"):
            o.init_laser(w["laser"])
        for z in stations:
            o.add_station(z)
        return o

    # ---- stepping -----------------------------------------------------------------
    def step(self, n: int = 1):
        lib().orc_step(self._h, n)

    def stage(self, name: str):
        getattr(lib(), "orc_stage_" + name)(self._h)

    # ---- access -------------------------------------------------------------------
    def info(self) -> dict:
        i = _Info()
        lib().orc_get_info(self._h, C.byref(i))
        return {k: getattr(i, k) for k, _ in _Info._fields_}

    @property
    def shape(self):
        i = self.info()
        return (i["stored_z"], i["stored_x"])

    def field(self, name: str) -> np.ndarray:
        out = np.zeros(self.shape, dtype=np.float64)
        lib().orc_get_field(self._h, FIELD_ID[name], _dp(out))
        return out

    def set_field(self, name: str, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.shape)
        lib().orc_set_field(self._h, FIELD_ID[name], _dp(a))

    def num_particles(self, species: int = 0) -> int:
        return lib().orc_num_particles(self._h, species)

    def particles(self, species: int = 0) -> dict:
        n = self.num_particles(species)
        d = {k: np.zeros(n, dtype=np.float64) for k in ["x", "z", "ux", "uy", "uz", "w"]}
        d["id"] = np.zeros(n, dtype=np.uint32)
        lib().orc_get_particles(self._h, species, _up(d["id"]), _dp(d["x"]), _dp(d["z"]),
                                _dp(d["ux"]), _dp(d["uy"]), _dp(d["uz"]), _dp(d["w"]))
        return d

    def set_electrons(self, p: dict):
        n = len(p["x"])
        arr = {k: np.ascontiguousarray(p[k], dtype=np.float64) for k in ["x", "z", "ux", "uy", "uz", "w"]}
        ids = np.ascontiguousarray(p["id"], dtype=np.uint32)
        lib().orc_set_electrons(self._h, n, _up(ids), _dp(arr["x"]), _dp(arr["z"]), _dp(arr["ux"]),
                                _dp(arr["uy"]), _dp(arr["uz"]), _dp(arr["w"]))

    def set_ions(self, ids, x, z0, w):
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        x, z0, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, z0, w))
        lib().orc_set_ions(self._h, len(x), _up(ids), _dp(x), _dp(z0), _dp(w))

    def antenna(self) -> np.ndarray:
        out = np.zeros(self.config["nx"], dtype=np.float64)
        lib().orc_get_antenna(self._h, _dp(out))
        return out

    def set_antenna(self, xm):
        a = np.ascontiguousarray(xm, dtype=np.float64)
        lib().orc_set_antenna(self._h, _dp(a))

    def set_clock(self, step, time, shift, next_row):
        lib().orc_set_clock(self._h, step, time, shift, next_row)

    def energy(self) -> np.ndarray:
        out = np.zeros(3)
        lib().orc_energy(self._h, _dp(out))
        return out

    def gauss_residual(self) -> np.ndarray:
        out = np.zeros(self.shape)
        lib().orc_gauss_residual(self._h, _dp(out))
        return out

    def charge_density(self) -> np.ndarray:
        out = np.zeros(self.shape)
        lib().orc_charge_density(self._h, _dp(out))
        return out

    def station(self, q: int) -> np.ndarray:
        n = lib().orc_station_samples(self._h, q, None, 0)
        out = np.zeros((max(n, 0), 7))
        if n > 0:
            lib().orc_station_samples(self._h, q, _dp(out), n)
        return out

    def gather_at(self, x: float, z: float) -> np.ndarray:
        """E^n and B^n at (x, z) (um) as the particle stage gathers them: Ex, Ey, Ez, Bx, By, Bz."""
        out = np.zeros(6)
        lib().orc_gather_at(self._h, x, z, _dp(out))
        return out

    def add_beam(self, beam: dict, parts: dict, history_cap: int = 100000):
        """Particle beam through a lab-fixed plane (Sec. 3.1.1).  beam: beta_b, z_inj_um,
        test_only; parts: x (um, interior-relative), z (lab um), ux, uy, uz (lab), w."""
        b = _Beam(beta_b=beam["beta_b"], z_inj_um=beam["z_inj_um"], test_only=int(beam.get("test_only", 1)))
        cols = [np.ascontiguousarray(parts[k], dtype=np.float64) for k in ("x", "z", "ux", "uy", "uz", "w")]
        r = lib().orc_add_beam(self._h, C.byref(b), len(cols[0]), *[_dp(c) for c in cols], history_cap)
        if r != 0:
            raise ValueError("orc_add_beam rejected the beam")

    def beam(self) -> dict:
        """x, z (um, window frame), ux, uy, uz (calculation frame), w, t_act, state."""
        n = lib().orc_beam_state(self._h, None)
        out = np.zeros(8 * max(n, 0))
        if n > 0:
            lib().orc_beam_state(self._h, _dp(out))
        cols = out.reshape(8, max(n, 0))
        return {k: cols[q] for q, k in enumerate(("x", "z", "ux", "uy", "uz", "w", "t_act", "state"))}

    def beam_history(self) -> np.ndarray:
        """(records, 8): t', count, sum w, sum w z_lab, sum w t_lab, sum w gamma_lab,
        sum w u_z,lab, sum w u_z,lab^2."""
        n = lib().orc_beam_history(self._h, None, 0)
        out = np.zeros((max(n, 0), 8))
        if n > 0:
            lib().orc_beam_history(self._h, _dp(out), n)
        return out

    def beam_transform(self, beam: dict, x, z, ux, uy, uz) -> np.ndarray:
        """t'*, x*, z'(0), u'x, u'y, u'z of one lab particle."""
        b = _Beam(beta_b=beam["beta_b"], z_inj_um=beam["z_inj_um"], test_only=int(beam.get("test_only", 1)))
        out = np.zeros(6)
        lib().orc_beam_transform(self._h, C.byref(b), x, z, ux, uy, uz, _dp(out))
        return out

    def deposit_one(self, q, w, x0, z0, x1, z1, vy):
        lib().orc_deposit_one(self._h, q, w, x0, z0, x1, z1, vy)


def shape3(r: float) -> float:
    return lib().orc_shape3(r)


def boris(qm, dt, E, B, u):
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    lib().orc_boris(qm, dt, _dp(E), _dp(B), _dp(u))
    return u


def vay(qm, dt, E, B, u):
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    u = np.array(u, dtype=np.float64)
    lib().orc_vay(qm, dt, _dp(E), _dp(B), _dp(u))
    return u


def cfl_2d(a, b, g, dx, dz, theta=0.0):
    return lib().orc_cfl_2d(a, b, g, dx, dz, theta)


def cfl_3d(a, b, g, dx, dy, dz, theta=0.0):
    return lib().orc_cfl_3d(a, b, g, dx, dy, dz, theta)


def splitmix64(seed, k):
    return lib().orc_splitmix64(seed, k)


def set_threads(n: int) -> None:
    """Host threads of the oracle's particle stages (2D and 3D); 1 unless set."""
    lib().orc_set_threads(int(n))


def host_threads(cap: int = 16) -> int:
    """The threads a large oracle run may use: the host's cores, at most cap."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, cap))
