"""Python binding of the MI355X boosted-frame laser-wakefield PIC library (libbfpic.so).

Argument marshalling only: every step of the PIC loop runs in the library's HIP kernels.
PyTorch provides the device memory (one torch.uint8 tensor per buffer the library asks for)
and the stream.  The functions bf_* mirror the C ABI of include/bfpic.h; `Sim` is a small
convenience wrapper over them.  Importing this package does not need a GPU; creating a Sim
does, and fails loudly when the compiled library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfpic.so")

ABI_VERSION = 5
FIELDS = ["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "Exo", "Eyo", "Ezo",
          "Exb", "Eyb", "Ezb", "Byx", "Eyx", "Bxo", "Byo", "Bzo", "Jxr", "Jyr", "Jzr",
          "Exs", "Eys", "Ezs", "Bxs", "Bys", "Bzs"]
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}
DIAG_FIELD, DIAG_PARTICLES, DIAG_COUNTS, DIAG_STATION, DIAG_ENERGY, DIAG_GAUSS, DIAG_INFO, \
    DIAG_ANTENNA, DIAG_TIMERS, DIAG_PARTICLE_BLOCK, DIAG_BEAM = range(11)
PARTICLE_BLOCK = 65536
PHASES = ["faraday", "push", "ions", "antenna", "filter", "ampere", "window", "sort", "beam"]
STATUS = {0: "BF_OK", -1: "BF_EINVAL", -2: "BF_ECFL", -3: "BF_ECAPACITY", -4: "BF_ENONFINITE",
          -5: "BF_EDEVICE", -6: "BF_ESTATE", -7: "BF_EUNSUPPORTED"}


class BfError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{STATUS.get(code, code)}: {msg}")


class bf_config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("struct_size", C.c_uint32), ("dim", C.c_int),
                ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx_um", C.c_double),
                ("dy_um", C.c_double), ("dz_um", C.c_double), ("real_bytes", C.c_int),
                ("shape_order", C.c_int), ("ck_alpha", C.c_double), ("ck_beta", C.c_double),
                ("ck_gamma", C.c_double), ("friedman_theta", C.c_double),
                ("cfl_fraction", C.c_double), ("filter_npass", C.c_int),
                ("filter_compensate", C.c_int), ("filter_kind", C.c_int), ("filter_strides", C.c_int),
                ("gather_kind", C.c_int), ("pusher", C.c_int), ("pml_cells", C.c_int),
                ("periodic_mask", C.c_int), ("gamma_boost", C.c_double),
                ("moving_window", C.c_int), ("particle_capacity", C.c_int64),
                ("sort_every", C.c_int), ("tile_x", C.c_int), ("tile_z", C.c_int),
                ("max_stations", C.c_int), ("station_capacity", C.c_int), ("phase_timers", C.c_int),
                ("seed", C.c_uint64), ("beam_capacity", C.c_int64), ("beam_history", C.c_int32),
                ("pml_kind", C.c_int32)]


class bf_plasma(C.Structure):
    _fields_ = [("n0_cm3", C.c_double), ("ramp_um", C.c_double), ("start_um", C.c_double),
                ("ppc", C.c_int), ("ion_mode", C.c_int)]


class bf_laser(C.Structure):
    _fields_ = [("lambda_um", C.c_double), ("a0", C.c_double), ("waist_um", C.c_double),
                ("fwhm_fs", C.c_double), ("z_antenna_um", C.c_double), ("t_peak_fs", C.c_double),
                ("pol", C.c_int)]


class bf_station(C.Structure):
    _fields_ = [("z_lab_um", C.c_double)]


class bf_beam(C.Structure):
    _fields_ = [("beta_b", C.c_double), ("z_inj_um", C.c_double), ("test_only", C.c_int32),
                ("reserved", C.c_int32)]


class bf_buffer_desc(C.Structure):
    _fields_ = [("name", C.c_char_p), ("bytes", C.c_size_t), ("align", C.c_size_t),
                ("dtype", C.c_int)]


class bf_buffer_binding(C.Structure):
    _fields_ = [("name", C.c_char_p), ("ptr", C.c_void_p), ("bytes", C.c_size_t)]


class bf_state(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("struct_size", C.c_uint32), ("step", C.c_int64),
                ("time", C.c_double), ("shift", C.c_int64), ("next_row", C.c_int64),
                ("zoff", C.c_int32), ("e_cur", C.c_int32), ("b_cur", C.c_int32),
                ("p_cur", C.c_int32), ("nseg_e", C.c_int32), ("nseg_i", C.c_int32),
                ("since_sort", C.c_int32), ("have_plasma", C.c_int32), ("have_laser", C.c_int32),
                ("nstations", C.c_int32), ("have_beam", C.c_int32), ("beam_test_only", C.c_int32),
                ("beam_n", C.c_int64), ("beam_records", C.c_int64), ("beam_vbar", C.c_double)]


class bf_info(C.Structure):
    _fields_ = [("dt", C.c_double), ("dt_crit", C.c_double), ("beta", C.c_double),
                ("gamma", C.c_double), ("v_window", C.c_double), ("n0_norm", C.c_double),
                ("e0_norm", C.c_double), ("omega", C.c_double), ("alpha2", C.c_double),
                ("beta2", C.c_double), ("antenna_weight", C.c_double), ("stored_x", C.c_int32),
                ("stored_z", C.c_int32), ("pml_x", C.c_int32), ("pml_z", C.c_int32),
                ("step", C.c_int64), ("time", C.c_double), ("shift", C.c_int64),
                ("next_row", C.c_int64), ("tile_x", C.c_int32), ("tile_z", C.c_int32),
                ("ntiles", C.c_int32), ("sort_every", C.c_int32), ("dim", C.c_int32),
                ("stored_y", C.c_int32), ("pml_y", C.c_int32), ("reserved", C.c_int32)]


EXPORTS = ["bf_query_buffers", "bf_create", "bf_init_plasma", "bf_init_laser", "bf_add_station",
           "bf_load_electrons", "bf_load_electrons3", "bf_add_beam", "bf_step", "bf_diagnose", "bf_set_field", "bf_sync_status",
           "bf_get_state", "bf_set_state", "bf_status_string", "bf_last_error", "bf_destroy",
           "bf_set_learned_filter", "bf_lf_work_bytes", "bf_lf_apply", "bf_lf_train_step",
           "bf_lf_bilinear_params", "bf_lf_apply_noalloc",
           "bf_batch_work_bytes", "bf_batch_create", "bf_batch_step", "bf_batch_destroy"]
FILTER_BILINEAR, FILTER_LEARNED = 0, 1
LF_PARAMS = 7200

_lib = None


def lib(path: str = LIB_PATH):
    """Load libbfpic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built: run __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950) first")
    # torch brings its own copy of the HIP runtime; load it first so that the library's
    # dependency resolves to that same runtime (device pointers and streams come from torch)
    import torch  # noqa: F401
    L = C.CDLL(path)
    P = C.c_void_p
    D = C.POINTER(C.c_double)
    L.bf_query_buffers.argtypes = [C.POINTER(bf_config), C.POINTER(bf_buffer_desc), C.POINTER(C.c_int)]
    L.bf_create.argtypes = [C.POINTER(bf_config), C.POINTER(bf_buffer_binding), C.c_int, P,
                            C.POINTER(P)]
    L.bf_init_plasma.argtypes = [P, C.POINTER(bf_plasma)]
    L.bf_init_laser.argtypes = [P, C.POINTER(bf_laser)]
    L.bf_add_station.argtypes = [P, C.POINTER(bf_station), C.POINTER(C.c_int)]
    L.bf_load_electrons.argtypes = [P, C.c_int64, C.POINTER(C.c_uint32), D, D, D, D, D, D]
    L.bf_load_electrons3.argtypes = [P, C.c_int64, C.POINTER(C.c_uint32), D, D, D, D, D, D, D]
    L.bf_add_beam.argtypes = [P, C.POINTER(bf_beam), C.c_int64, D, D, D, D, D, D]
    L.bf_step.argtypes = [P, C.c_int]
    L.bf_diagnose.argtypes = [P, C.c_int, C.c_int, P, C.c_size_t]
    L.bf_set_field.argtypes = [P, C.c_int, D, C.c_size_t]
    L.bf_sync_status.argtypes = [P]
    L.bf_get_state.argtypes = [P, C.POINTER(bf_state)]
    L.bf_set_state.argtypes = [P, C.POINTER(bf_state)]
    L.bf_status_string.argtypes = [C.c_int]
    L.bf_status_string.restype = C.c_char_p
    L.bf_last_error.argtypes = [P]
    L.bf_last_error.restype = C.c_char_p
    L.bf_destroy.argtypes = [P]
    L.bf_destroy.restype = None
    F = C.POINTER(C.c_float)
    L.bf_set_learned_filter.argtypes = [P, F, C.c_int64]
    L.bf_lf_work_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    L.bf_lf_work_bytes.restype = C.c_int64
    L.bf_lf_apply.argtypes = [P, C.c_int64, P, P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P]
    L.bf_lf_train_step.argtypes = [P, C.c_int64, P, P, P, P, P, C.c_int, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float,
                                   C.c_int64, P, P, P]
    L.bf_lf_bilinear_params.argtypes = [C.c_int, C.c_int, F, C.c_int64]
    L.bf_lf_apply_noalloc.argtypes = [P, P, P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, P]
    L.bf_batch_work_bytes.argtypes = [C.c_int]
    L.bf_batch_work_bytes.restype = C.c_int64
    L.bf_batch_create.argtypes = [C.POINTER(P), C.c_int, P, C.c_int64, P, C.POINTER(P)]
    L.bf_batch_step.argtypes = [P, C.c_int]
    L.bf_batch_destroy.argtypes = [P]
    L.bf_batch_destroy.restype = None
    for n in EXPORTS:
        if n not in ("bf_status_string", "bf_last_error", "bf_destroy", "bf_lf_work_bytes",
                     "bf_batch_work_bytes", "bf_batch_destroy"):
            getattr(L, n).restype = C.c_int
    _lib = L
    return L


# ---- same-name wrappers (marshalling only) ---------------------------------------------------

def bf_query_buffers(cfg: bf_config):
    n = C.c_int(0)
    _check(lib().bf_query_buffers(C.byref(cfg), None, C.byref(n)))
    descs = (bf_buffer_desc * n.value)()
    _check(lib().bf_query_buffers(C.byref(cfg), descs, C.byref(n)))
    return [(d.name.decode(), d.bytes, d.align) for d in descs]


def bf_create(cfg: bf_config, bindings, stream_ptr: int):
    arr = (bf_buffer_binding * len(bindings))()
    for k, (name, ptr, nbytes) in enumerate(bindings):
        arr[k].name = name.encode()
        arr[k].ptr = ptr
        arr[k].bytes = nbytes
    h = C.c_void_p()
    _check(lib().bf_create(C.byref(cfg), arr, len(bindings), C.c_void_p(stream_ptr), C.byref(h)))
    return h


def _check(code, handle=None):
    if code != 0:
        msg = ""
        if handle is not None:
            m = lib().bf_last_error(handle)
            msg = m.decode() if m else ""
        raise BfError(code, msg)
    return code


def make_config(cfg: dict, capacity: int, stations: int = 0, station_capacity: int = 1,
                sort_every: int = 0, tile=(0, 0), timers: bool = False) -> bf_config:
    c = bf_config()
    c.abi_version = ABI_VERSION
    c.struct_size = C.sizeof(bf_config)
    c.dim = int(cfg.get("dim", 2))
    if c.dim == 3:
        c.nx, c.ny, c.nz = cfg["nx"], cfg["ny"], cfg["nz"]
        c.dx_um, c.dy_um, c.dz_um = cfg["dx_um"], cfg["dy_um"], cfg["dz_um"]
    else:
        c.nx, c.ny, c.nz = cfg["nx"], 1, cfg["nz"]
        c.dx_um, c.dy_um, c.dz_um = cfg["dx_um"], cfg["dx_um"], cfg["dz_um"]
    c.real_bytes = 4 if cfg.get("real", "f32") == "f32" else 8
    c.shape_order = 3
    c.ck_alpha, c.ck_beta, c.ck_gamma = cfg["ck_alpha"], cfg["ck_beta"], cfg["ck_gamma"]
    c.friedman_theta = cfg["theta"]
    c.cfl_fraction = cfg["cfl_fraction"]
    c.filter_npass = cfg["filter_npass"]
    c.filter_compensate = cfg["filter_compensate"]
    c.filter_kind = cfg.get("filter_kind", FILTER_BILINEAR)
    c.filter_strides = cfg.get("filter_strides", 1)
    c.gather_kind = cfg.get("gather_kind", 0)
    c.pusher = cfg.get("pusher", 0)
    c.pml_cells = cfg["pml_cells"]
    c.periodic_mask = ((1 if cfg.get("periodic_x") else 0) | (2 if cfg.get("periodic_y") else 0)
                       | (4 if cfg.get("periodic_z") else 0))
    c.gamma_boost = cfg["gamma_boost"]
    c.moving_window = cfg["moving_window"]
    c.particle_capacity = int(capacity)
    c.sort_every = sort_every
    c.tile_x, c.tile_z = tile
    c.max_stations = stations
    c.station_capacity = station_capacity
    c.phase_timers = 1 if timers else 0
    c.seed = cfg["seed"]
    c.beam_capacity = int(cfg.get("beam_capacity", 0))
    c.beam_history = int(cfg.get("beam_history", 0))
    c.pml_kind = int(cfg.get("pml_kind", 0))
    return c


def default_capacity(cfg: dict, ppc: int) -> int:
    ny = cfg["ny"] if cfg.get("dim", 2) == 3 else 1
    return int(cfg["nx"] * ny * (cfg["nz"] + 8) * max(ppc, 1) * 1.15) + 4096


class Sim:
    """One simulation on a HIP device.  Every device byte is a torch tensor owned here."""

    def __init__(self, config: dict, capacity: int | None = None, ppc: int = 1, stations: int = 0,
                 station_capacity: int = 100000, sort_every: int = 0, tile=(0, 0), device=None,
                 stream=None, timers: bool = False):
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the PIC kernels need an MI355X")
        lib()
        self.config = dict(config)
        cap = capacity if capacity is not None else default_capacity(config, ppc)
        self.cfg = make_config(config, cap, stations, station_capacity, sort_every, tile, timers)
        self.device = torch.device(device or "cuda:0")
        self.stream = stream or torch.cuda.current_stream(self.device)
        descs = bf_query_buffers(self.cfg)
        self.buffers = {}
        bindings = []
        for name, nbytes, align in descs:
            t = torch.empty(max(nbytes, align), dtype=torch.uint8, device=self.device)
            assert t.data_ptr() % align == 0
            self.buffers[name] = t
            bindings.append((name, t.data_ptr(), t.numel()))
        self.handle = bf_create(self.cfg, bindings, self.stream.cuda_stream)
        info = self.info()
        self.dim = int(config.get("dim", 2))
        self.shape = ((info["stored_z"], info["stored_y"], info["stored_x"]) if self.dim == 3
                      else (info["stored_z"], info["stored_x"]))

    # ---- lifecycle --------------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            lib().bf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ck(self, code):
        return _check(code, self.handle)

    @classmethod
    def from_workload(cls, w: dict, laser=True, plasma=True, stations=(), **kw):
        ppc = w["plasma"]["ppc"] if (plasma and w.get("plasma")) else 1
        s = cls(w["config"], ppc=ppc, stations=max(len(stations), 0) or 0, **kw)
        if plasma and w.get("plasma"):
            s.init_plasma(w["plasma"])
        if laser and w.get("laser"):
            s.init_laser(w["laser"])
        for z in stations:
            s.add_station(z)
        return s

    # ---- set-up ---------------------------------------------------------------------
    def init_plasma(self, p: dict):
        self._ck(lib().bf_init_plasma(self.handle, C.byref(bf_plasma(**p))))

    def init_laser(self, l: dict):
        self._ck(lib().bf_init_laser(self.handle, C.byref(bf_laser(**l))))

    def add_station(self, z_lab_um: float) -> int:
        i = C.c_int(-1)
        self._ck(lib().bf_add_station(self.handle, C.byref(bf_station(z_lab_um)), C.byref(i)))
        return i.value

    def load_electrons(self, p: dict):
        n = len(p["x"])
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        ids = np.ascontiguousarray(p.get("id", np.arange(n)), dtype=np.uint32)
        if self.dim == 3:
            a3 = {k: np.ascontiguousarray(p[k], dtype=np.float64) for k in ("x", "y", "z", "ux", "uy", "uz", "w")}
            self._ck(lib().bf_load_electrons3(self.handle, n, ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                                              *[dp(a3[k]) for k in ("x", "y", "z", "ux", "uy", "uz", "w")]))
            return
        arr = {k: np.ascontiguousarray(p[k], dtype=np.float64) for k in ("x", "z", "ux", "uy", "uz", "w")}
        self._ck(lib().bf_load_electrons(self.handle, n, ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                                         dp(arr["x"]), dp(arr["z"]), dp(arr["ux"]), dp(arr["uy"]),
                                         dp(arr["uz"]), dp(arr["w"])))

    def add_beam(self, beam: dict, parts: dict):
        """Beam through a lab-fixed plane (bf_add_beam).  beam: beta_b, z_inj_um, test_only;
        parts: lab x (um, interior-relative), z (lab um), ux, uy, uz, w at t = 0.  The run's
        config needs beam_capacity (and beam_history for the per-step records)."""
        n = len(parts["x"])
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        arr = {k: np.ascontiguousarray(parts[k], dtype=np.float64) for k in ("x", "z", "ux", "uy", "uz", "w")}
        b = bf_beam(beta_b=float(beam["beta_b"]), z_inj_um=float(beam["z_inj_um"]),
                    test_only=int(beam.get("test_only", 1)))
        self._ck(lib().bf_add_beam(self.handle, C.byref(b), n, *[dp(arr[k]) for k in ("x", "z", "ux", "uy", "uz", "w")]))

    def beam(self) -> dict:
        """x, z (um, window frame), ux, uy, uz (calculation frame), w, t_act, state."""
        cap = int(self.cfg.beam_capacity)
        out = self._diag(DIAG_BEAM, 0, np.zeros(1 + 8 * max(cap, 1)))
        n = int(out[:1].view(np.int64)[0])
        cols = out[1:1 + 8 * n].reshape(8, n)
        return {k: cols[q].copy() for q, k in enumerate(("x", "z", "ux", "uy", "uz", "w", "t_act", "state"))}

    def beam_history(self) -> np.ndarray:
        """(records, 8): t', count, sum w, sum w z_lab, sum w t_lab, sum w gamma_lab,
        sum w u_z,lab, sum w u_z,lab^2."""
        cap = int(self.cfg.beam_history)
        out = self._diag(DIAG_BEAM, 1, np.zeros(1 + 8 * max(cap, 1)))
        m = int(out[:1].view(np.int64)[0])
        return out[1:1 + 8 * m].reshape(m, 8).copy()

    def set_field(self, name: str, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(self.shape)
        self._ck(lib().bf_set_field(self.handle, FIELD_ID[name], a.ctypes.data_as(C.POINTER(C.c_double)),
                                    a.nbytes))

    # ---- stepping -------------------------------------------------------------------
    def step(self, n: int = 1):
        self._ck(lib().bf_step(self.handle, n))

    def sync_status(self):
        return lib().bf_sync_status(self.handle)

    # ---- diagnostics ----------------------------------------------------------------
    def _diag(self, kind, arg, out: np.ndarray):
        self._ck(lib().bf_diagnose(self.handle, kind, arg, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def info(self) -> dict:
        i = bf_info()
        self._ck(lib().bf_diagnose(self.handle, DIAG_INFO, 0, C.cast(C.byref(i), C.c_void_p), C.sizeof(i)))
        return {k: getattr(i, k) for k, _ in bf_info._fields_}

    def field(self, name: str) -> np.ndarray:
        return self._diag(DIAG_FIELD, FIELD_ID[name], np.zeros(self.shape))

    def counts(self) -> np.ndarray:
        return self._diag(DIAG_COUNTS, 0, np.zeros(4, dtype=np.int64))

    def particles(self, species: int = 0) -> dict:
        n = int(self.counts()[species])
        keys = (["id", "x", "y", "z", "ux", "uy", "uz", "w"] if self.dim == 3
                else ["id", "x", "z", "ux", "uy", "uz", "w"])
        m = len(keys)
        out = self._diag(DIAG_PARTICLES, species, np.zeros((m, max(n, 1))))
        out = out.reshape(m, -1)[:, :n] if n > 0 else np.zeros((m, 0))
        d = {k: out[q].copy() for q, k in enumerate(keys)}
        d["id"] = d["id"].astype(np.uint32)
        return d

    def energy(self) -> np.ndarray:
        return self._diag(DIAG_ENERGY, 0, np.zeros(3))

    def gauss_residual(self) -> np.ndarray:
        return self._diag(DIAG_GAUSS, 0, np.zeros(self.shape))

    def station(self, q: int) -> np.ndarray:
        cap = self.cfg.station_capacity
        raw = self._diag(DIAG_STATION, q, np.zeros(1 + 7 * cap))
        n = int(raw[:1].view(np.int64)[0])
        return raw[1:1 + 7 * n].reshape(n, 7)

    def particle_block(self, species: int, block: int) -> dict:
        """3D: the live particles of slots [block, block + 1) * PARTICLE_BLOCK (a sample)."""
        out = self._diag(DIAG_PARTICLE_BLOCK, species + 2 * block, np.zeros(1 + 8 * PARTICLE_BLOCK))
        n = int(out[:1].view(np.int64)[0])
        cols = out[1:1 + 8 * n].reshape(8, n)
        d = {k: cols[q].copy() for q, k in enumerate(["id", "x", "y", "z", "ux", "uy", "uz", "w"])}
        d["id"] = d["id"].astype(np.uint32)
        return d

    def timers(self, reset: bool = True) -> dict:
        """Accumulated device time (ms) and launch count of each step phase."""
        out = self._diag(DIAG_TIMERS, 1 if reset else 0, np.zeros(2 * len(PHASES)))
        return {p: (out[2 * q], out[2 * q + 1]) for q, p in enumerate(PHASES)}

    def antenna(self) -> np.ndarray:
        n = self.config["nx"] * (self.config["ny"] if self.dim == 3 else 1)
        return self._diag(DIAG_ANTENNA, 0, np.zeros(n))

    def get_state(self) -> bf_state:
        st = bf_state()
        self._ck(lib().bf_get_state(self.handle, C.byref(st)))
        return st

    def set_state(self, st: bf_state):
        self._ck(lib().bf_set_state(self.handle, C.byref(st)))

    def set_learned_filter(self, params):
        """Loads the learned filter's BF_LF_PARAMS FP32 parameters (host array)."""
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        self._ck(lib().bf_set_learned_filter(self.handle, a.ctypes.data_as(C.POINTER(C.c_float)), a.size))


def bilinear_factor_params(npass: int = 4, compensate: bool = True) -> np.ndarray:
    """Learned-filter parameters equal to the n-pass bilinear filter (+ compensation) of
    Sec. 4.1, from the library (bf_lf_bilinear_params)."""
    out = np.zeros(LF_PARAMS, np.float32)
    _ck(lib().bf_lf_bilinear_params(int(npass), 1 if compensate else 0,
                                    out.ctypes.data_as(C.POINTER(C.c_float)), LF_PARAMS))
    return out


def _ck(code):
    if code != 0:
        raise BfError(code, lib().bf_status_string(code).decode())


class Batch:
    """Several Sim handles (FP32, same device) stepped together: each heavy phase of a step is
    one persistent launch over all runs.  The Sims stay usable for diagnostics."""

    def __init__(self, sims, stream=None):
        import torch
        self.torch = torch
        self.sims = list(sims)
        dev = self.sims[0].device
        n = lib().bf_batch_work_bytes(len(self.sims))
        if n < 0:
            raise BfError(-1, "bad batch size")
        self.work = torch.empty(n, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        arr = (C.c_void_p * len(self.sims))(*[s.handle for s in self.sims])
        h = C.c_void_p()
        _ck(lib().bf_batch_create(arr, len(self.sims), C.c_void_p(self.work.data_ptr()), n,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.handle = h

    def step(self, n: int = 1):
        _ck(lib().bf_batch_step(self.handle, n))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            lib().bf_batch_destroy(h)
            self.handle = None


class LearnedFilter:
    """The learned current filter on batches of device images (torch float32 tensors of shape
    (nimg, ny, nx)): inference and training through the library's MFMA kernels.  Holds the
    FP32 parameters and the Adam moments on the device."""

    def __init__(self, params=None, device=None, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        p = np.zeros(LF_PARAMS, np.float32) if params is None else np.asarray(params, np.float32).ravel()
        if p.size != LF_PARAMS:
            raise ValueError(f"expected {LF_PARAMS} parameters")
        self.params = torch.tensor(p, dtype=torch.float32, device=self.device)
        self.m = torch.zeros(LF_PARAMS, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(LF_PARAMS, dtype=torch.float32, device=self.device)
        self.t = 0
        self.stream = stream
        self._work = None

    def _stream_ptr(self):
        s = self.stream if self.stream is not None else self.torch.cuda.current_stream(self.device)
        return C.c_void_p(s.cuda_stream)

    def _work_for(self, nimg, ny, nx):
        n = lib().bf_lf_work_bytes(nimg, ny, nx)
        if n < 0:
            raise BfError(-1, "bad image sizes")
        if self._work is None or self._work.numel() < n:
            self._work = self.torch.empty(n, dtype=self.torch.uint8, device=self.device)
        return self._work

    @staticmethod
    def _check(x):
        if x.dtype != np.float32 and str(x.dtype) != "torch.float32":
            raise TypeError("images must be float32")
        if x.dim() != 3 or not x.is_contiguous():
            raise ValueError("images must be a contiguous (nimg, ny, nx) tensor")

    def apply(self, images, periodic=(False, False)):
        self._check(images)
        nimg, ny, nx = images.shape
        out = self.torch.empty_like(images)
        w = self._work_for(nimg, ny, nx)
        _ck(lib().bf_lf_apply(C.c_void_p(w.data_ptr()), w.numel(), C.c_void_p(self.params.data_ptr()),
                              C.c_void_p(images.data_ptr()), C.c_void_p(out.data_ptr()), nimg, ny, nx,
                              int(periodic[0]), int(periodic[1]), self._stream_ptr()))
        return out

    def apply_noalloc(self, images, out, periodic=(False, False)):
        """The same as apply() through bf_lf_apply_noalloc: no work buffer, out supplied."""
        self._check(images)
        self._check(out)
        nimg, ny, nx = images.shape
        _ck(lib().bf_lf_apply_noalloc(C.c_void_p(self.params.data_ptr()), C.c_void_p(images.data_ptr()),
                                      C.c_void_p(out.data_ptr()), nimg, ny, nx, int(periodic[0]),
                                      int(periodic[1]), self._stream_ptr()))
        return out

    def train_step(self, images, targets, margin, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                   periodic=(False, False), want_grad=False):
        """One step; returns (loss, grad) as device tensors (grad None unless asked)."""
        self._check(images)
        self._check(targets)
        nimg, ny, nx = images.shape
        w = self._work_for(nimg, ny, nx)
        loss = self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        grad = self.torch.empty(LF_PARAMS, dtype=self.torch.float32, device=self.device) if want_grad else None
        if lr != 0:
            self.t += 1
        _ck(lib().bf_lf_train_step(C.c_void_p(w.data_ptr()), w.numel(), C.c_void_p(self.params.data_ptr()),
                                   C.c_void_p(self.m.data_ptr()), C.c_void_p(self.v.data_ptr()),
                                   C.c_void_p(images.data_ptr()), C.c_void_p(targets.data_ptr()),
                                   nimg, ny, nx, margin, int(periodic[0]), int(periodic[1]), lr, beta1,
                                   beta2, eps, max(self.t, 1),
                                   C.c_void_p(grad.data_ptr()) if grad is not None else None,
                                   C.c_void_p(loss.data_ptr()), self._stream_ptr()))
        return loss, grad
