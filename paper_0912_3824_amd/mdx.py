"""Thin Python binding of libmdx (include/md.h): argument marshalling only.

Every step of the MD path runs in the HIP kernels of libmdx.so; this module
converts NumPy arrays and ctypes structures, owns the device workspace as a
torch uint8 tensor and the HIP stream as a torch stream (PyTorch is used for
device memory and streams only), and raises MdError on a non-zero status.
There is no CPU fallback: if libmdx.so is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdx.so")

MD_FP32, MD_DS, MD_MIXED64, MD_FP64 = 0, 1, 2, 3
PRECISIONS = {"fp32": MD_FP32, "ds": MD_DS, "mixed64": MD_MIXED64, "fp64": MD_FP64}
MD_ST_LIST_OVERFLOW, MD_ST_NONFINITE, MD_ST_LOST, MD_ST_AT_FULL_STEP = 1, 2, 4, 256

MD_E_CAPACITY, MD_E_NONFINITE = -4, -5
MD_ST_NO_PAD = 8

STATUS_NAMES = {0: "MD_OK", -1: "MD_E_ARG", -2: "MD_E_BOX", -3: "MD_E_WORKSPACE",
                -4: "MD_E_CAPACITY", -5: "MD_E_NONFINITE", -6: "MD_E_HIP",
                -7: "MD_E_NOSLOT", -8: "MD_E_STATE"}

# Symbols declared in include/md.h (checked by the CPU test-suite).
EXPORTS = [
    "md_workspace_bytes", "md_validate", "md_create", "md_init", "md_destroy",
    "md_attach", "md_detach", "md_rebuild_neighbours", "md_forces", "md_step",
    "md_set_target", "md_advance", "md_poll", "md_observables",
    "md_scale_velocities", "md_profile_steps", "md_sync", "md_get_state", "md_checkpoint_bytes",
    "md_save", "md_restore", "md_debug_neighbours", "md_get_launch",
    "md_set_launch", "md_ds_eval", "md_strerror", "md_last_error",
    "md_abi_version", "md_tcf_workspace_bytes", "md_tcf_create", "md_tcf_sample",
    "md_tcf_read", "md_tcf_destroy", "md_thermostat", "md_cell_order",
    "md_thermostat_noalloc",
]

CELL_ORDERS = {"row": 0, "morton": 1, "hilbert": 2}


class MdConfig(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("eps", ctypes.c_double * 4), ("sigma", ctypes.c_double * 4),
                ("rcut", ctypes.c_double * 4), ("mass", ctypes.c_double),
                ("dt", ctypes.c_double), ("skin", ctypes.c_double),
                ("nbr_capacity", ctypes.c_int32), ("max_slots", ctypes.c_int32),
                ("max_particles", ctypes.c_int64), ("max_cells", ctypes.c_int64),
                ("max_density", ctypes.c_double), ("lanes_per_particle", ctypes.c_int32),
                ("cell_order", ctypes.c_int32), ("smooth", ctypes.c_double),
                ("rebuild_every", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("rebuild_early", ctypes.c_double)]


class MdReplica(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("box", ctypes.c_double)]


class MdObs(ctypes.Structure):
    _fields_ = [("epot", ctypes.c_double), ("ekin", ctypes.c_double), ("etot", ctypes.c_double),
                ("temperature", ctypes.c_double), ("virial", ctypes.c_double),
                ("pressure", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("step", ctypes.c_int64), ("n_rebuilds", ctypes.c_int64),
                ("list_entries", ctypes.c_int64),
                ("status", ctypes.c_int32), ("n", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"epot": self.epot, "ekin": self.ekin, "etot": self.etot,
                "temperature": self.temperature, "virial": self.virial,
                "pressure": self.pressure, "momentum": np.array(list(self.momentum)),
                "step": self.step, "n_rebuilds": self.n_rebuilds,
                "list_entries": self.list_entries,
                "status": self.status, "n": self.n}


class MdLaunch(ctypes.Structure):
    _fields_ = [("step_block", ctypes.c_int32), ("build_width", ctypes.c_int32),
                ("build_block", ctypes.c_int32), ("graph_steps", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("build_lanes", ctypes.c_int32),
                ("build_split", ctypes.c_int32), ("build_bulk", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in
                ("step_block", "build_width", "build_block", "graph_steps", "xcd_remap", "build_lanes",
                 "build_split", "build_bulk")}


class MdError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {text}")
        self.status = status


_lib = None


def load():
    """Load libmdx.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_0912_3824_amd/build.py "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp, fp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float))
    ip = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    cfgp = ctypes.POINTER(MdConfig)
    repp = ctypes.POINTER(MdReplica)
    sig = {
        "md_workspace_bytes": (i64, [cfgp]),
        "md_validate": (i32, [cfgp, repp]),
        "md_create": (i32, [cfgp, vp, i64, vp, ctypes.POINTER(vp)]),
        "md_init": (i32, [cfgp, repp, i32, ip, dp, dp, vp, i64, vp, ctypes.POINTER(vp)]),
        "md_destroy": (None, [vp]),
        "md_attach": (i32, [vp, i32, repp, ip, dp, dp]),
        "md_detach": (i32, [vp, i32]),
        "md_rebuild_neighbours": (i32, [vp]),
        "md_forces": (i32, [vp, i32, dp, dp]),
        "md_step": (i32, [vp, i64]),
        "md_set_target": (i32, [vp, i32, i64]),
        "md_advance": (i32, [vp, i64]),
        "md_poll": (i32, [vp, i64p, ip]),
        "md_observables": (i32, [vp, ctypes.POINTER(MdObs)]),
        "md_scale_velocities": (i32, [vp, i32, ctypes.c_double]),
        "md_sync": (i32, [vp]),
        "md_profile_steps": (i32, [vp, i64, dp]),
        "md_get_state": (i32, [vp, i32, dp, dp, ip]),
        "md_checkpoint_bytes": (i64, [vp, i32]),
        "md_save": (i32, [vp, i32, vp, i64]),
        "md_restore": (i32, [vp, i32, vp, i64]),
        "md_debug_neighbours": (i32, [vp, i32, ip, ip, i32]),
        "md_get_launch": (i32, [vp, ctypes.POINTER(MdLaunch)]),
        "md_set_launch": (i32, [vp, ctypes.POINTER(MdLaunch)]),
        "md_ds_eval": (i32, [i32, i64, vp, vp, vp, vp]),
        "md_strerror": (ctypes.c_char_p, [i32]),
        "md_last_error": (ctypes.c_char_p, [vp]),
        "md_abi_version": (i32, []),
        "md_cell_order": (i32, [i32, i32, ip]),
        "md_tcf_workspace_bytes": (i64, [i32, i32, i32]),
        "md_tcf_create": (i32, [vp, i32, i32, i32, ctypes.c_double, vp, i64, ctypes.POINTER(vp)]),
        "md_tcf_sample": (i32, [vp]),
        "md_tcf_read": (i32, [vp, i64p, dp, i64p]),
        "md_tcf_destroy": (None, [vp]),
        "md_thermostat": (i32, [vp, i32, ctypes.c_double, ctypes.c_uint64, i64, i32]),
        "md_thermostat_noalloc": (i32, [vp, i32, ctypes.c_double, ctypes.c_uint64, i64, i32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def make_config(table, precision, dt: float, skin: float, max_slots: int,
                max_particles: int, mass: float = 1.0, nbr_capacity: int = 0,
                max_cells: int = 0, max_density: float = 0.0,
                lanes_per_particle: int = 0, cell_order="row", rebuild_every: int = 0,
                rebuild_early: float = 0.0) -> MdConfig:
    """md_config from a pair table (md_inputs.PairTable, including its
    smoothing width) and run parameters."""
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    c = MdConfig()
    c.n_species = int(table.n_species)
    c.precision = int(precision)
    for k in range(4):
        a, b = divmod(k, 2)
        c.eps[k] = float(table.eps[a, b])
        c.sigma[k] = float(table.sigma[a, b])
        c.rcut[k] = float(table.rcut[a, b])
    c.mass, c.dt, c.skin = float(mass), float(dt), float(skin)
    c.nbr_capacity = int(nbr_capacity)
    c.max_slots = int(max_slots)
    c.max_particles = int(max_particles)
    c.max_cells = int(max_cells)
    c.max_density = float(max_density)
    c.lanes_per_particle = int(lanes_per_particle)
    c.smooth = float(getattr(table, "smooth", 0.0))
    c.cell_order = CELL_ORDERS[cell_order] if isinstance(cell_order, str) else int(cell_order)
    c.rebuild_every = int(rebuild_every)
    c.rebuild_early = float(rebuild_early)
    return c


def cell_order_ranks(nd: int, order) -> np.ndarray:
    """md_cell_order: rank of every cell c = x + nd (y + nd z) of an nd^3
    grid in the given cell order (host only)."""
    o = CELL_ORDERS[order] if isinstance(order, str) else int(order)
    out = np.zeros(nd ** 3, dtype=np.int32)
    st = int(load().md_cell_order(int(nd), o, _ip(out)))
    if st != 0:
        raise MdError(st, f"md_cell_order(nd={nd}, order={order})")
    return out


def md_workspace_bytes(cfg: MdConfig) -> int:
    return int(load().md_workspace_bytes(ctypes.byref(cfg)))


def md_validate(cfg: MdConfig, n: Optional[int] = None, box: Optional[float] = None) -> int:
    rep = None
    if n is not None:
        r = MdReplica(int(n), 0, float(box))
        rep = ctypes.byref(r)
    return int(load().md_validate(ctypes.byref(cfg), rep))


def md_ds_eval(op: int, a, b, out, stream=None) -> None:
    """Double-single self-test on torch device tensors of shape [n, 2] float32."""
    import torch
    lib = load()
    n = a.shape[0] if op != 3 else a.shape[0]
    st = lib.md_ds_eval(int(op), int(n), ctypes.c_void_p(a.data_ptr()),
                        ctypes.c_void_p(b.data_ptr()) if b is not None else None,
                        ctypes.c_void_p(out.data_ptr()),
                        ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream))
    if st != 0:
        raise MdError(st, "md_ds_eval")


class Tcf:
    """Time-correlation functions of one replica by the blocking scheme
    (md_tcf_*): sample() after each sampling interval; read() returns the
    lags (in samples), term counts and per-species (MSD, VACF, F_s) means."""

    def __init__(self, pool: "MdSystem", slot: int, levels: int, block: int, q: float):
        import torch
        self.pool, self.lib = pool, pool.lib
        self.levels, self.block = int(levels), int(block)
        n = pool.sizes[slot]
        nbytes = int(self.lib.md_tcf_workspace_bytes(n, self.levels, self.block))
        if nbytes < 0:
            raise MdError(nbytes, "md_tcf_workspace_bytes")
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=pool.device)
        h = ctypes.c_void_p()
        pool._check(self.lib.md_tcf_create(pool.h, int(slot), self.levels, self.block, float(q),
                                           ctypes.c_void_p(self.ws.data_ptr()), ctypes.c_int64(nbytes),
                                           ctypes.byref(h)), "md_tcf_create")
        self.h = h

    def sample(self):
        self.pool._check(self.lib.md_tcf_sample(self.h), "md_tcf_sample")

    def read(self):
        k = self.levels * (self.block - 1)
        lags = np.zeros(k, dtype=np.int64)
        terms = np.zeros(k, dtype=np.int64)
        vals = np.zeros(k * 6)
        self.pool._check(self.lib.md_tcf_read(self.h, lags.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                              _dp(vals), terms.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
                         "md_tcf_read")
        return (lags.reshape(self.levels, self.block - 1), vals.reshape(self.levels, self.block - 1, 2, 3),
                terms.reshape(self.levels, self.block - 1))

    def close(self):
        if getattr(self, "h", None):
            self.lib.md_tcf_destroy(self.h)
            self.h = None


class MdSystem:
    """A pool of replica slots on one GPU (md_create / md_init and friends).

    The workspace is a torch uint8 tensor of md_workspace_bytes() bytes and
    the stream a default-priority torch stream; both live as long as this
    object.  Methods carry the C entry points' names without the md_ prefix.
    """

    def __init__(self, cfg: MdConfig, device: str = "cuda:0", stream=None):
        import torch
        self.lib = load()
        self.cfg = cfg
        self.device = torch.device(device)
        nbytes = md_workspace_bytes(cfg)
        if nbytes < 0:
            raise MdError(nbytes, "invalid configuration")
        self.ws_bytes = nbytes
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        st = self.lib.md_create(ctypes.byref(cfg), ctypes.c_void_p(self.ws.data_ptr()),
                                ctypes.c_int64(nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.byref(h))
        if st != 0:
            raise MdError(st, "md_create")
        self.h = h
        self.max_slots = cfg.max_slots
        self.sizes = {}
        self.boxes = {}

    # ---------------------------------------------------------------- helpers
    def _check(self, st: int, what: str):
        if st != 0:
            txt = self.lib.md_last_error(self.h)
            raise MdError(st, f"{what}: {txt.decode() if txt else ''}")

    def close(self):
        for t in list(getattr(self, "_tcfs", [])):
            t.close()
        if getattr(self, "h", None):
            self.lib.md_destroy(self.h)
            self.h = None

    def thermostat(self, slot: int, temperature: float, seed: int, call: int, remove_mean: bool = True):
        """Modified Andersen thermostat call (md_thermostat): Maxwell-Boltzmann
        velocities from the leap-frogged rand48 stream, rescaled to exactly T."""
        self._check(self.lib.md_thermostat(self.h, int(slot), float(temperature), int(seed) & (2 ** 64 - 1),
                                           int(call), 1 if remove_mean else 0), "md_thermostat")

    def thermostat_noalloc(self, slot: int, temperature: float, seed: int, call: int,
                           remove_mean: bool = True):
        """md_thermostat_noalloc: the same call with its scratch in the
        library's static device array (allocates nothing)."""
        self._check(self.lib.md_thermostat_noalloc(self.h, int(slot), float(temperature),
                                                   int(seed) & (2 ** 64 - 1), int(call),
                                                   1 if remove_mean else 0), "md_thermostat_noalloc")

    def andersen(self, slot: int, temperature: float, mu: float, steps: int, seed: int, first_call: int = 0):
        """Advance `steps` steps with the heat bath of collision rate mu: a
        thermostat call every (mu dt)^-1 steps (Sec. 2.3).  Returns the next
        call index."""
        every = max(1, int(round(1.0 / (mu * self.cfg.dt))))
        call, done = first_call, 0
        while done < steps:
            self.thermostat(slot, temperature, seed, call)
            call += 1
            k = min(every, steps - done)
            self.step(k)
            done += k
        return call

    def tcf(self, slot: int, levels: int, block: int, q: float) -> "Tcf":
        """A blocking scheme for time-correlation functions bound to `slot`
        (md_tcf_create); see Tcf."""
        t = Tcf(self, slot, levels, block, q)
        self.__dict__.setdefault("_tcfs", []).append(t)
        return t

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- replicas
    def attach(self, slot: int, n: int, box: float, species, pos, vel):
        sp = np.ascontiguousarray(species, dtype=np.int32)
        p = np.ascontiguousarray(pos, dtype=np.float64)
        v = np.ascontiguousarray(vel, dtype=np.float64)
        if p.shape != (n, 3) or v.shape != (n, 3) or sp.shape != (n,):
            raise ValueError("shape mismatch")
        rep = MdReplica(int(n), 0, float(box))
        self._check(self.lib.md_attach(self.h, int(slot), ctypes.byref(rep), _ip(sp), _dp(p), _dp(v)),
                    "md_attach")
        self.sizes[slot] = int(n)
        self.boxes[slot] = float(box)

    def validate(self, n: int, box: float) -> int:
        """md_validate for a replica of n particles in a box of edge `box`
        against this pool's configuration: 0, or the status it would get in
        an empty pool (MD_E_BOX, MD_E_CAPACITY, MD_E_ARG).  Host only."""
        return md_validate(self.cfg, n, box)

    def attach_system(self, slot: int, s):
        """Attach an md_inputs.System."""
        self.attach(slot, s.n, s.box, s.species, s.pos, s.vel)

    def detach(self, slot: int):
        self._check(self.lib.md_detach(self.h, int(slot)), "md_detach")
        self.sizes.pop(slot, None)
        self.boxes.pop(slot, None)

    # ---------------------------------------------------------------- MD step
    def rebuild_neighbours(self):
        self._check(self.lib.md_rebuild_neighbours(self.h), "md_rebuild_neighbours")

    def forces(self, slot: int = 0, copy: bool = True):
        """Forces and per-particle energies at the current positions (id order)."""
        if not copy:
            self._check(self.lib.md_forces(self.h, int(slot), None, None), "md_forces")
            return None
        n = self.sizes[slot]
        f = np.zeros((n, 3))
        e = np.zeros(n)
        self._check(self.lib.md_forces(self.h, int(slot), _dp(f), _dp(e)), "md_forces")
        return f, e

    def step(self, n_steps: int):
        self._check(self.lib.md_step(self.h, int(n_steps)), "md_step")

    def set_target(self, slot: int, target: int):
        self._check(self.lib.md_set_target(self.h, int(slot), int(target)), "md_set_target")

    def advance(self, n_launch: int):
        self._check(self.lib.md_advance(self.h, int(n_launch)), "md_advance")

    def poll(self):
        """(steps, status) of every slot (md_poll).  A replica that stopped
        with an error bit is reported in `status`, not raised: md_poll's
        MD_E_CAPACITY / MD_E_NONFINITE are how the C ABI flags it."""
        steps = np.zeros(self.max_slots, dtype=np.int64)
        status = np.zeros(self.max_slots, dtype=np.int32)
        st = self.lib.md_poll(self.h, steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ip(status))
        if st not in (0, MD_E_CAPACITY, MD_E_NONFINITE):
            self._check(st, "md_poll")
        return steps, status

    def observables(self, check: bool = True):
        """Observables of every slot (md_observables).  With check=False a
        replica stopped by an error bit is reported in its 'status' instead
        of raising."""
        out = (MdObs * self.max_slots)()
        st = self.lib.md_observables(self.h, out)
        if check or st not in (MD_E_CAPACITY, MD_E_NONFINITE):
            self._check(st, "md_observables")
        return [o.as_dict() for o in out]

    def scale_velocities(self, slot: int, factor: float):
        self._check(self.lib.md_scale_velocities(self.h, int(slot), float(factor)),
                    "md_scale_velocities")

    def profile_steps(self, n_steps: int) -> dict:
        """Eager steps with hipEvent timing of the fused kernel and rebuilds."""
        out = np.zeros(5)
        self._check(self.lib.md_profile_steps(self.h, int(n_steps), _dp(out)), "md_profile_steps")
        return {"step_kernel_ms": out[0], "rebuild_ms_mean": out[1],
                "rebuild_ms_when_rebuilding": out[2], "rebuild_steps": int(out[3]),
                "total_ms": out[4]}

    def sync(self):
        self._check(self.lib.md_sync(self.h), "md_sync")

    # ---------------------------------------------------------------- state
    def get_state(self, slot: int = 0):
        n = self.sizes[slot]
        p = np.zeros((n, 3))
        v = np.zeros((n, 3))
        img = np.zeros((n, 3), dtype=np.int32)
        self._check(self.lib.md_get_state(self.h, int(slot), _dp(p), _dp(v), _ip(img)),
                    "md_get_state")
        return p, v, img

    def save(self, slot: int) -> bytes:
        nb = int(self.lib.md_checkpoint_bytes(self.h, int(slot)))
        if nb < 0:
            self._check(nb, "md_checkpoint_bytes")
        buf = ctypes.create_string_buffer(nb)
        self._check(self.lib.md_save(self.h, int(slot), buf, nb), "md_save")
        return buf.raw

    def restore(self, slot: int, blob: bytes, n: int, box: float):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._check(self.lib.md_restore(self.h, int(slot), buf, len(blob)), "md_restore")
        self.sizes[slot] = int(n)
        self.boxes[slot] = float(box)

    def neighbours(self, slot: int = 0, cap: Optional[int] = None):
        n = self.sizes[slot]
        cap = cap or 256
        cnt = np.zeros(n, dtype=np.int32)
        ids = np.zeros((n, cap), dtype=np.int32)
        self._check(self.lib.md_debug_neighbours(self.h, int(slot), _ip(cnt), _ip(ids), int(cap)),
                    "md_debug_neighbours")
        return cnt, ids

    def get_launch(self) -> dict:
        l = MdLaunch()
        self._check(self.lib.md_get_launch(self.h, ctypes.byref(l)), "md_get_launch")
        return l.as_dict()

    def set_launch(self, **kw):
        l = MdLaunch()
        self._check(self.lib.md_get_launch(self.h, ctypes.byref(l)), "md_get_launch")
        for k, v in kw.items():
            setattr(l, k, int(v))
        self._check(self.lib.md_set_launch(self.h, ctypes.byref(l)), "md_set_launch")


def md_init(systems: Sequence, precision, dt: Optional[float] = None, skin: Optional[float] = None,
            max_slots: Optional[int] = None, extra_particles: int = 0, device: str = "cuda:0",
            **cfg_kw) -> MdSystem:
    """md_init: a pool holding `systems` (md_inputs.System objects, same
    pair table) in slots 0..k-1."""
    systems = list(systems)
    s0 = systems[0]
    total = sum(s.n for s in systems) + extra_particles
    cfg = make_config(s0.table, precision, dt if dt is not None else s0.dt,
                      skin if skin is not None else s0.skin,
                      max_slots or len(systems), total, mass=s0.mass, **cfg_kw)
    pool = MdSystem(cfg, device=device)
    for k, s in enumerate(systems):
        pool.attach_system(k, s)
    return pool
