"""ctypes wrapper of the FP64 CPU oracle in 3D (oracle/pic_oracle3.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by the
CPU-baseline leg of bench.py.  The product package never imports it.

Parity unpinned: as for the 2-1/2D oracle (the energy-conserving gather beyond exact uniform
and linear fields, quantitative PML reflection, the nonlinear wake), the 3D PML split
convention (which curl term the stored part holds) and the static field the split layer can
keep inside itself.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _Laser, _Plasma, _dp, _up, lib

FIELDS = ["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "Exo", "Eyo", "Ezo",
          "Exb", "Eyb", "Ezb", "Exs", "Eys", "Ezs", "Bxs", "Bys", "Bzs", "Bxo", "Byo", "Bzo"]
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}


class _Cfg3(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx_um", C.c_double),
                ("dy_um", C.c_double), ("dz_um", C.c_double), ("pml_cells", C.c_int),
                ("periodic_x", C.c_int), ("periodic_y", C.c_int), ("periodic_z", C.c_int),
                ("ck_alpha", C.c_double), ("ck_beta", C.c_double), ("ck_gamma", C.c_double),
                ("theta", C.c_double), ("cfl_fraction", C.c_double), ("filter_npass", C.c_int),
                ("filter_compensate", C.c_int), ("gamma_boost", C.c_double),
                ("moving_window", C.c_int), ("seed", C.c_uint64), ("filter_strides", C.c_int),
                ("gather_kind", C.c_int), ("pusher", C.c_int), ("pml_kind", C.c_int)]


class _Info3(C.Structure):
    _fields_ = [("dt", C.c_double), ("dt_crit", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_double), ("v_window", C.c_double), ("n0_norm", C.c_double),
                ("e0_norm", C.c_double), ("omega", C.c_double), ("antenna_weight", C.c_double),
                ("stored_x", C.c_int), ("stored_y", C.c_int), ("stored_z", C.c_int),
                ("pml_x", C.c_int), ("pml_y", C.c_int), ("pml_z", C.c_int),
                ("step", C.c_long), ("time", C.c_double), ("shift", C.c_long),
                ("next_row", C.c_long)]


_ready = False


def lib3():
    global _ready
    L = lib()
    if not _ready:
        P, D, U = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint32)
        L.orc3_create.restype = P
        L.orc3_create.argtypes = [C.POINTER(_Cfg3)]
        L.orc3_destroy.argtypes = [P]
        L.orc3_init_plasma.argtypes = [P, C.POINTER(_Plasma)]
        L.orc3_init_laser.argtypes = [P, C.POINTER(_Laser)]
        L.orc3_add_station.argtypes = [P, C.c_double, C.c_int]
        L.orc3_step.argtypes = [P, C.c_int]
        for n in ["faraday", "stations", "particles", "filter", "ampere", "advance"]:
            getattr(L, "orc3_stage_" + n).argtypes = [P]
        L.orc3_get_info.argtypes = [P, C.POINTER(_Info3)]
        L.orc3_get_field.argtypes = [P, C.c_int, D]
        L.orc3_set_field.argtypes = [P, C.c_int, D]
        L.orc3_num_particles.restype = C.c_long
        L.orc3_num_particles.argtypes = [P, C.c_int]
        L.orc3_get_particles.argtypes = [P, C.c_int, U, D, D, D, D, D, D, D]
        L.orc3_set_electrons.argtypes = [P, C.c_long, U, D, D, D, D, D, D, D]
        L.orc3_set_ions.argtypes = [P, C.c_long, U, D, D, D, D]
        L.orc3_get_antenna.argtypes = [P, D]
        L.orc3_set_antenna.argtypes = [P, D]
        L.orc3_set_clock.argtypes = [P, C.c_long, C.c_double, C.c_long, C.c_long]
        L.orc3_energy.argtypes = [P, D]
        L.orc3_charge_density.argtypes = [P, D]
        L.orc3_gauss_residual.argtypes = [P, D]
        L.orc3_station_samples.restype = C.c_long
        L.orc3_station_samples.argtypes = [P, C.c_int, D, C.c_long]
        L.orc3_deposit_one.argtypes = [P, C.c_double, C.c_double, D, D]
        L.orc3_gather_at.argtypes = [P, D, D]
        _ready = True
    return L


class Oracle3:
    """One FP64 reference simulation in 3D (fields [z][y][x])."""

    def __init__(self, config: dict):
        c = _Cfg3(**{k: config.get(k, {"filter_strides": 1, "gather_kind": 0, "pusher": 0, "pml_kind": 0}[k]) if k in ("filter_strides", "gather_kind", "pusher", "pml_kind") else config[k] for k, _ in _Cfg3._fields_})
        self._h = lib3().orc3_create(C.byref(c))
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self.config = dict(config)

    def close(self):
        if getattr(self, "_h", None):
            lib3().orc3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_plasma(self, p: dict):
        if lib3().orc3_init_plasma(self._h, C.byref(_Plasma(**p))) != 0:
            raise ValueError("bad plasma")

    def init_laser(self, l: dict):
        if lib3().orc3_init_laser(self._h, C.byref(_Laser(**l))) != 0:
            raise ValueError("bad laser")

    def add_station(self, z_lab_um: float, capacity: int = 100000) -> int:
        return lib3().orc3_add_station(self._h, z_lab_um, capacity)

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

    def step(self, n: int = 1):
        lib3().orc3_step(self._h, n)

    def stage(self, name: str):
        getattr(lib3(), "orc3_stage_" + name)(self._h)

    def info(self) -> dict:
        i = _Info3()
        lib3().orc3_get_info(self._h, C.byref(i))
        return {k: getattr(i, k) for k, _ in _Info3._fields_}

    @property
    def shape(self):
        i = self.info()
        return (i["stored_z"], i["stored_y"], i["stored_x"])

    def field(self, name: str) -> np.ndarray:
        out = np.zeros(self.shape, dtype=np.float64)
        lib3().orc3_get_field(self._h, FIELD_ID[name], _dp(out))
        return out

    def set_field(self, name: str, arr: np.ndarray):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(self.shape)
        lib3().orc3_set_field(self._h, FIELD_ID[name], _dp(a))

    def num_particles(self, species: int = 0) -> int:
        return lib3().orc3_num_particles(self._h, species)

    def particles(self, species: int = 0) -> dict:
        n = self.num_particles(species)
        d = {k: np.zeros(n, dtype=np.float64) for k in ["x", "y", "z", "ux", "uy", "uz", "w"]}
        d["id"] = np.zeros(n, dtype=np.uint32)
        lib3().orc3_get_particles(self._h, species, _up(d["id"]), _dp(d["x"]), _dp(d["y"]),
                                  _dp(d["z"]), _dp(d["ux"]), _dp(d["uy"]), _dp(d["uz"]), _dp(d["w"]))
        return d

    def set_electrons(self, p: dict):
        n = len(p["x"])
        arr = {k: np.ascontiguousarray(p[k], dtype=np.float64)
               for k in ["x", "y", "z", "ux", "uy", "uz", "w"]}
        ids = np.ascontiguousarray(p["id"], dtype=np.uint32)
        lib3().orc3_set_electrons(self._h, n, _up(ids), _dp(arr["x"]), _dp(arr["y"]), _dp(arr["z"]),
                                  _dp(arr["ux"]), _dp(arr["uy"]), _dp(arr["uz"]), _dp(arr["w"]))

    def set_ions(self, ids, x, y, z0, w):
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        x, y, z0, w = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z0, w))
        lib3().orc3_set_ions(self._h, len(x), _up(ids), _dp(x), _dp(y), _dp(z0), _dp(w))

    def antenna(self) -> np.ndarray:
        out = np.zeros(self.config["nx"] * self.config["ny"], dtype=np.float64)
        lib3().orc3_get_antenna(self._h, _dp(out))
        return out

    def set_clock(self, step, time, shift, next_row):
        lib3().orc3_set_clock(self._h, step, time, shift, next_row)

    def energy(self) -> np.ndarray:
        out = np.zeros(3)
        lib3().orc3_energy(self._h, _dp(out))
        return out

    def gauss_residual(self) -> np.ndarray:
        out = np.zeros(self.shape)
        lib3().orc3_gauss_residual(self._h, _dp(out))
        return out

    def charge_density(self) -> np.ndarray:
        out = np.zeros(self.shape)
        lib3().orc3_charge_density(self._h, _dp(out))
        return out

    def station(self, q: int) -> np.ndarray:
        n = lib3().orc3_station_samples(self._h, q, None, 0)
        out = np.zeros((max(n, 0), 7))
        if n > 0:
            lib3().orc3_station_samples(self._h, q, _dp(out), n)
        return out

    def deposit_one(self, q, w, r0, r1):
        a = np.ascontiguousarray(r0, dtype=np.float64)
        b = np.ascontiguousarray(r1, dtype=np.float64)
        lib3().orc3_deposit_one(self._h, q, w, _dp(a), _dp(b))

    def gather_at(self, r) -> np.ndarray:
        """E^n and B^n at r = (x, y, z) (um) as the particle stage gathers them."""
        a = np.ascontiguousarray(r, dtype=np.float64)
        out = np.zeros(6)
        lib3().orc3_gather_at(self._h, _dp(a), _dp(out))
        return out
