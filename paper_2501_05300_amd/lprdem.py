"""Python binding of the HIP stepper (include/lprdem.h).

Argument marshalling only: every step of the pipeline runs in the HIP
library paper_2501_05300_amd/liblprdem.so.  PyTorch supplies device memory
(its caching allocator, through the library's allocator callbacks) and the
HIP stream.  There is no CPU fallback: constructing a Bed without the built
library or without a GPU raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblprdem.so")

SLOTS = 16
MAX_WALLS = 16
MAX_BODIES = 4

STATUS = {0: "ok", -1: "invalid argument", -2: "out of memory", -3: "device error", -4: "capacity exceeded",
          -5: "invalid state", -6: "non-finite value", -7: "particle through a wall"}

# Entry points declared in include/lprdem.h
_PER_BED = ("get_state", "set_state", "get_history", "set_history", "read_contacts", "read_forces", "read_reaction",
            "reaction_window", "read_body", "set_clock", "get_clock", "set_body_state", "read_contact_loads",
            "read_wall_pose")
SYMBOLS = ("lpr_bed_create", "lpr_bed_destroy", "lpr_step", "lpr_step_profiled", "lpr_step_phases", "lpr_sync",
           "lpr_get_stats", "lpr_read_contact_loads_noalloc",
           "lpr_status_str", "lpr_last_error", "lpr_batch_create", "lpr_batch_size", "lpr_set_launch",
           "lpr_autotune", "lpr_set_contact_params", "lpr_adjoint_window", "lpr_set_stepper") + tuple("lpr_" + f for f in _PER_BED) + tuple("lpr_batch_" + f for f in _PER_BED)


class LprError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where}: {STATUS.get(status, status)} ({message})")
        self.status = status


class CapacityError(LprError):
    pass


class NumericError(LprError):
    pass


class _Params(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("mu_t", ctypes.c_double), ("mu_r", ctypes.c_double), ("dt", ctypes.c_double),
                ("gamma_factor", ctypes.c_double), ("e_H", ctypes.c_double), ("kappa_t", ctypes.c_double),
                ("s_k", ctypes.c_double), ("g", ctypes.c_double * 3)]


class _Wall(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("body", ctypes.c_int32), ("origin", ctypes.c_double * 3),
                ("axis", ctypes.c_double * 3), ("frame", ctypes.c_double * 9), ("dims", ctypes.c_double * 3),
                ("mu_t", ctypes.c_double), ("mu_r", ctypes.c_double)]


class _Body(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("lin_vel", ctypes.c_double * 3), ("ang_vel", ctypes.c_double),
                ("z_free", ctypes.c_int32), ("mass", ctypes.c_double)]


class _Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("box", ctypes.c_double * 3), ("periodic", ctypes.c_uint32),
                ("pos", ctypes.c_void_p), ("radius", ctypes.c_void_p), ("vel", ctypes.c_void_p),
                ("omega", ctypes.c_void_p), ("n_walls", ctypes.c_int32), ("walls", ctypes.c_void_p),
                ("n_bodies", ctypes.c_int32), ("bodies", ctypes.c_void_p), ("params", _Params),
                ("rebuild_every", ctypes.c_int32), ("skin", ctypes.c_float), ("band_ratio", ctypes.c_float),
                ("cell_factor", ctypes.c_float), ("block", ctypes.c_int32), ("record_forces", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("sort_every", ctypes.c_int32), ("input_order", ctypes.c_int32),
                ("level_cell_factor", ctypes.c_float * 16)]


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
_RELEASE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC), ("release", _RELEASE), ("ctx", ctypes.c_void_p)]


class _Contact(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int64), ("b", ctypes.c_int64)]


class _History(ctypes.Structure):
    _fields_ = [("owner", ctypes.c_int64), ("partner", ctypes.c_int64), ("xi_t", ctypes.c_float * 3),
                ("xi_r", ctypes.c_float * 3)]


# numpy view of lpr_contact_load: 48 bytes, no padding
_LOAD_DT = np.dtype([("a", "<i8"), ("b", "<i8"), ("f", "<f4", (3,)), ("m", "<f4", (3,)), ("fn", "<f4"),
                     ("reserved", "<f4")])

# numpy view of lpr_history (the struct above): 40 bytes, no padding
_HISTORY_DT = np.dtype([("o", "<i8"), ("p", "<i8"), ("v", "<f4", (6,))])
assert _HISTORY_DT.itemsize == ctypes.sizeof(_History)


class _Tuning(ctypes.Structure):
    _fields_ = [("band_ratio", ctypes.c_float), ("cell_factor", ctypes.c_float), ("block", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("ms_per_step", ctypes.c_double),
                ("level_cell_factor", ctypes.c_float * 16)]


class _Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("contacts", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("rebuilds", ctypes.c_int64), ("levels", ctypes.c_int32), ("cells", ctypes.c_int64),
                ("max_owner_slots", ctypes.c_int32), ("skin_trips", ctypes.c_int64),
                ("adjoint_interval", ctypes.c_int32), ("sorts", ctypes.c_int64), ("outside_grid", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads liblprdem.so (importing torch first so that the process shares
    one HIP runtime).  Raises if the library is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
    import torch  # noqa: F401  (brings torch's HIP runtime into the process first)
    L = ctypes.CDLL(path)
    vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sig = {
        "lpr_bed_create": [ctypes.POINTER(_Desc), ctypes.POINTER(_Allocator), vp, ctypes.POINTER(vp)],
        "lpr_bed_destroy": [vp], "lpr_step": [vp, i64], "lpr_sync": [vp],
        "lpr_step_profiled": [vp, i64, vp], "lpr_step_phases": [vp, i64, vp],
        "lpr_get_state": [vp, vp, vp, vp], "lpr_set_state": [vp, vp, vp, vp],
        "lpr_get_history": [vp, vp, i64, ctypes.POINTER(i64)], "lpr_set_history": [vp, vp, i64],
        "lpr_read_contacts": [vp, vp, i64, ctypes.POINTER(i64)], "lpr_read_forces": [vp, vp, vp],
        "lpr_read_reaction": [vp, i32, vp], "lpr_reaction_window": [vp, i32, vp, ctypes.POINTER(i64), i32],
        "lpr_read_body": [vp, i32, vp, vp], "lpr_set_clock": [vp, i64], "lpr_get_clock": [vp, ctypes.POINTER(i64)],
        "lpr_set_body_state": [vp, i32, d, d], "lpr_get_stats": [vp, ctypes.POINTER(_Stats)],
        "lpr_read_contact_loads": [vp, vp, i64, ctypes.POINTER(i64)], "lpr_read_wall_pose": [vp, i32, vp],
        "lpr_read_contact_loads_noalloc": [vp, vp, i64, ctypes.POINTER(i64)],
    }
    for f in _PER_BED:
        args = sig["lpr_" + f]
        sig["lpr_batch_" + f] = [args[0], i32] + args[1:]
    sig["lpr_batch_create"] = [ctypes.POINTER(ctypes.POINTER(_Desc)), i32, ctypes.POINTER(_Allocator), vp,
                               ctypes.POINTER(vp)]
    sig["lpr_batch_size"] = [vp, ctypes.POINTER(i32)]
    sig["lpr_set_launch"] = [vp, i32, i32]
    sig["lpr_set_contact_params"] = [vp, d, d, d]
    sig["lpr_set_stepper"] = [vp, i32, i32]
    sig["lpr_adjoint_window"] = [vp, i64, i32, i32, ctypes.POINTER(d), vp]
    sig["lpr_autotune"] = [ctypes.POINTER(ctypes.POINTER(_Desc)), i32, ctypes.POINTER(_Allocator), vp, i32,
                           ctypes.POINTER(_Tuning), ctypes.POINTER(_Tuning), i32, ctypes.POINTER(i32)]
    for name, args in sig.items():
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = args
    L.lpr_status_str.restype = ctypes.c_char_p
    L.lpr_status_str.argtypes = [ctypes.c_int]
    L.lpr_last_error.restype = ctypes.c_char_p
    L.lpr_last_error.argtypes = []
    _lib = L
    return L


def _check(rc, where):
    if rc == 0:
        return
    msg = _lib.lpr_last_error().decode(errors="replace") if _lib is not None else ""
    if rc == -4:
        raise CapacityError(rc, where, msg)
    if rc == -6:
        raise NumericError(rc, where, msg)
    raise LprError(rc, where, msg)


def params_struct(p) -> _Params:
    q = _Params()
    for f in ("rho", "E", "nu", "mu_t", "mu_r", "dt", "gamma_factor", "e_H", "kappa_t", "s_k"):
        setattr(q, f, p.field(f))
    for a in range(3):
        q.g[a] = float(p.g[a])
    return q


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


class _DescHolder:
    """A filled lpr_bed_desc plus the arrays it points to (kept alive)."""

    def __init__(self, spec, rebuild_every, skin, band_ratio, cell_factor, block, record_forces, persistent=False,
                 sort_every=0, input_order=False, level_cell_factor=None):
        self.pos = np.ascontiguousarray(spec.pos, np.float64)
        self.rad = np.ascontiguousarray(spec.radius, np.float32)
        self.vel = np.ascontiguousarray(spec.vel, np.float32)
        self.omg = np.ascontiguousarray(spec.omega, np.float32)
        nw, nb = len(spec.walls), len(spec.bodies)
        self.walls = (_Wall * max(1, nw))()
        for q, w in enumerate(spec.walls):
            W = self.walls[q]
            W.kind, W.body = int(w.kind), int(w.body)
            for a in range(3):
                W.origin[a], W.axis[a], W.dims[a] = w.origin[a], w.axis[a], w.dims[a]
            for a in range(9):
                W.frame[a] = w.frame[a]
            W.mu_t, W.mu_r = float(w.mu_t), float(w.mu_r)
        self.bodies = (_Body * max(1, nb))()
        for q, b in enumerate(spec.bodies):
            B = self.bodies[q]
            for a in range(3):
                B.origin[a], B.lin_vel[a] = b.origin[a], b.lin_vel[a]
            B.ang_vel, B.z_free, B.mass = float(b.ang_vel), int(b.z_free), float(b.mass)
        D = _Desc()
        D.n = spec.n
        for a in range(3):
            D.box[a] = float(spec.box[a])
        D.periodic = int(spec.periodic)
        D.pos, D.radius = self.pos.ctypes.data, self.rad.ctypes.data
        D.vel, D.omega = self.vel.ctypes.data, self.omg.ctypes.data
        D.n_walls, D.walls = nw, ctypes.addressof(self.walls)
        D.n_bodies, D.bodies = nb, ctypes.addressof(self.bodies)
        D.params = params_struct(spec.params)
        D.rebuild_every = int(rebuild_every)
        D.skin = float(skin)
        D.band_ratio = float(band_ratio)
        D.cell_factor = float(cell_factor)
        D.block = int(block)
        D.record_forces = 1 if record_forces else 0
        D.persistent = 1 if persistent else 0
        D.sort_every = int(sort_every)
        D.input_order = 1 if input_order else 0
        for q, f in enumerate(level_cell_factor or ()):
            D.level_cell_factor[q] = float(f)
        self.desc = D


class _TorchMemory:
    """Allocator callbacks into torch's caching allocator on one stream."""

    def __init__(self, device, stream):
        import torch
        self._live = {}

        def _alloc(ctx, nbytes):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
            except Exception:  # noqa: BLE001  (reported to the library as NULL)
                return None
            self._live[p] = nbytes
            return p

        def _release(ctx, p):
            if p in self._live:
                del self._live[p]
                try:
                    torch.cuda.caching_allocator_delete(p)
                except (AttributeError, TypeError):
                    pass  # torch already torn down at interpreter exit; the process frees its memory

        self._cb = (_ALLOC(_alloc), _RELEASE(_release))
        self.struct = _Allocator(self._cb[0], self._cb[1], None)


def _gpu_or_raise(device):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP stepper needs a GPU (torch.cuda.is_available() is False)")
    return torch.device("cuda", device)


class _Stepper:
    """Common part of Bed and Batch: stepping and the per-bed reads."""

    _batch = False

    def _call(self, name, bed, *args):
        if self._batch:
            return _check(getattr(_lib, "lpr_batch_" + name)(self._h, int(bed), *args), "lpr_batch_" + name)
        if bed != 0:
            raise IndexError("a single bed has index 0")
        return _check(getattr(_lib, "lpr_" + name)(self._h, *args), "lpr_" + name)

    def close(self):
        if getattr(self, "_h", None):
            _lib.lpr_bed_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    # stepping
    def step(self, n=1):
        _check(_lib.lpr_step(self._h, int(n)), "lpr_step")

    def step_profiled(self, n):
        """Steps n times with HIP events around each kernel group; returns
        summed milliseconds {rebuild, step, advance, total}."""
        out = np.zeros(4)
        _check(_lib.lpr_step_profiled(self._h, int(n), _ptr(out)), "lpr_step_profiled")
        return {"rebuild": out[0], "step": out[1], "advance": out[2], "total": out[3]}

    PHASES = ("binning", "resort", "cell_lists", "search", "reverse_lists", "contact_step", "body_reduction")

    def step_phases(self, n):
        """Steps n times with HIP events at every phase boundary; returns
        summed milliseconds per phase (PHASES) and "total"."""
        out = np.zeros(8)
        _check(_lib.lpr_step_phases(self._h, int(n), _ptr(out)), "lpr_step_phases")
        res = {k: float(out[q]) for q, k in enumerate(self.PHASES)}
        res["total"] = float(out[7])
        return res

    def sync(self):
        _check(_lib.lpr_sync(self._h), "lpr_sync")

    def set_launch(self, block, persistent=False):
        _check(_lib.lpr_set_launch(self._h, int(block), 1 if persistent else 0), "lpr_set_launch")

    def set_stepper(self, kind, n_iter=0):
        """kind "explicit" (the compliant step, default) or "spook" (the
        time-implicit step with n_iter projected iterations per step); see
        lpr_set_stepper in include/lprdem.h."""
        k = {"explicit": 0, "spook": 1}[kind]
        _check(_lib.lpr_set_stepper(self._h, k, int(n_iter)), "lpr_set_stepper")

    def set_contact_params(self, s_k, mu_t, mu_r):
        _check(_lib.lpr_set_contact_params(self._h, float(s_k), float(mu_t), float(mu_r)), "lpr_set_contact_params")

    def adjoint_window(self, n_steps, ckpt_every, body):
        """J = mean z reaction on `body` over n_steps and dJ/d(s_k, mu_t, mu_r)."""
        J = ctypes.c_double(0.0)
        g = np.zeros(3)
        _check(_lib.lpr_adjoint_window(self._h, int(n_steps), int(ckpt_every), int(body), ctypes.byref(J), _ptr(g)),
               "lpr_adjoint_window")
        return J.value, g

    def stats(self):
        s = _Stats()
        _check(_lib.lpr_get_stats(self._h, ctypes.byref(s)), "lpr_get_stats")
        return {f: getattr(s, f) for f, _ in _Stats._fields_}

    # state
    def state(self, bed=0):
        n = self._n(bed)
        pos = np.zeros((n, 3), np.float64)
        vel = np.zeros((n, 3), np.float32)
        omg = np.zeros((n, 3), np.float32)
        self._call("get_state", bed, _ptr(pos), _ptr(vel), _ptr(omg))
        return pos, vel, omg

    def set_state(self, pos=None, vel=None, omg=None, bed=0):
        c64 = lambda a: None if a is None else np.ascontiguousarray(a, np.float64).reshape(-1, 3)
        c32 = lambda a: None if a is None else np.ascontiguousarray(a, np.float32).reshape(-1, 3)
        pos, vel, omg = c64(pos), c32(vel), c32(omg)
        self._call("set_state", bed, _ptr(pos), _ptr(vel), _ptr(omg))

    def history(self, bed=0):
        """(keys (k, 2) int64 owner/partner code, values (k, 6) float32)."""
        tot = ctypes.c_int64(0)
        try:
            self._call("get_history", bed, None, 0, ctypes.byref(tot))
        except CapacityError:
            pass
        arr = np.zeros(max(1, tot.value), _HISTORY_DT)
        self._call("get_history", bed, arr.ctypes.data, tot.value, ctypes.byref(tot))
        arr = arr[:tot.value]
        return np.stack([arr["o"], arr["p"]], 1), arr["v"].copy()

    def set_history(self, keys, vals, bed=0):
        keys = np.asarray(keys, np.int64).reshape(-1, 2)
        vals = np.asarray(vals, np.float32).reshape(-1, 6)
        arr = np.zeros(max(1, len(keys)), _HISTORY_DT)
        arr["o"][:len(keys)], arr["p"][:len(keys)] = keys[:, 0], keys[:, 1]
        arr["v"][:len(keys)] = vals
        self._call("set_history", bed, arr.ctypes.data, len(keys))

    # results of the last step
    def contacts(self, bed=0):
        """(k, 2) int64: particle pairs (a < b stable ids) and wall contacts
        (particle, -1 - wall), ascending."""
        tot = ctypes.c_int64(0)
        try:
            self._call("read_contacts", bed, None, 0, ctypes.byref(tot))
        except CapacityError:
            pass
        out = np.zeros((max(1, tot.value), 2), np.int64)
        self._call("read_contacts", bed, _ptr(out), tot.value, ctypes.byref(tot))
        return out[:tot.value]

    def forces(self, bed=0):
        n = self._n(bed)
        F = np.zeros((n, 3), np.float32)
        T = np.zeros((n, 3), np.float32)
        self._call("read_forces", bed, _ptr(F), _ptr(T))
        return F, T

    def contact_loads(self, bed=0):
        """Per contact of the last step, in contacts() order: (pairs (k, 2),
        force on particle a (k, 3), rolling moment on a (k, 3), F_n (k,))."""
        tot = ctypes.c_int64(0)
        try:
            self._call("read_contact_loads", bed, None, 0, ctypes.byref(tot))
        except CapacityError:
            pass
        arr = np.zeros(max(1, tot.value), _LOAD_DT)
        self._call("read_contact_loads", bed, arr.ctypes.data, tot.value, ctypes.byref(tot))
        arr = arr[:tot.value]
        return np.stack([arr["a"], arr["b"]], 1), arr["f"].copy(), arr["m"].copy(), arr["fn"].copy()

    def contact_loads_noalloc(self, capacity):
        """contact_loads() of a single bed through the entry point that
        allocates nothing (its workspace is the library's static device
        array); `capacity` records are offered."""
        tot = ctypes.c_int64(0)
        arr = np.zeros(max(1, int(capacity)), _LOAD_DT)
        _check(_lib.lpr_read_contact_loads_noalloc(self._h, arr.ctypes.data, int(capacity), ctypes.byref(tot)),
               "lpr_read_contact_loads_noalloc")
        arr = arr[:tot.value]
        return np.stack([arr["a"], arr["b"]], 1), arr["f"].copy(), arr["m"].copy(), arr["fn"].copy()

    def wall_pose(self, wall, bed=0):
        """World pose of a wall at the current clock: origin, normal, frame rows (3, 3)."""
        out = np.zeros(15)
        self._call("read_wall_pose", bed, int(wall), _ptr(out))
        return out[0:3], out[3:6], out[6:15].reshape(3, 3)

    def reaction(self, body, bed=0):
        out = np.zeros(6)
        self._call("read_reaction", bed, int(body), _ptr(out))
        return out

    def reaction_window(self, body, reset=False, bed=0):
        s = np.zeros(6)
        k = ctypes.c_int64(0)
        self._call("reaction_window", bed, int(body), _ptr(s), ctypes.byref(k), 1 if reset else 0)
        return s, k.value

    def body(self, body, bed=0):
        o = np.zeros(3)
        v = np.zeros(3)
        self._call("read_body", bed, int(body), _ptr(o), _ptr(v))
        return o, v

    def set_clock(self, step, bed=0):
        self._call("set_clock", bed, int(step))

    def clock(self, bed=0):
        k = ctypes.c_int64(0)
        self._call("get_clock", bed, ctypes.byref(k))
        return k.value

    def set_body_state(self, body, z, vz, bed=0):
        self._call("set_body_state", bed, int(body), float(z), float(vz))


class Bed(_Stepper):
    """A graded bed stepped by the HIP library on one GPU.

    spec: paper_2501_05300_amd.beds.BedSpec.  rebuild_every / skin /
    band_ratio / cell_factor / block / persistent / sort_every / input_order
    choose how contacts are found, how particles are ordered in memory and
    how the step kernel is launched (never which contacts or what results);
    record_forces keeps per-particle contact forces for forces() and
    per-contact loads for contact_loads().
    """

    def __init__(self, spec, rebuild_every=1, skin=0.0, band_ratio=0.0, cell_factor=0.0, block=0,
                 record_forces=False, persistent=False, device=0, torch_memory=True, sort_every=0,
                 input_order=False, level_cell_factor=None):
        import torch
        self.device = _gpu_or_raise(device)
        L = load_library()
        self.spec = spec
        self.n = spec.n
        self.stream = torch.cuda.Stream(self.device)
        self._holder = _DescHolder(spec, rebuild_every, skin, band_ratio, cell_factor, block, record_forces,
                                   persistent, sort_every, input_order, level_cell_factor)
        self._mem = _TorchMemory(self.device, self.stream)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = L.lpr_bed_create(ctypes.byref(self._holder.desc),
                                  ctypes.byref(self._mem.struct) if torch_memory else None,
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(rc, "lpr_bed_create")
        self._h = h

    def _n(self, bed):
        return self.n


class Batch(_Stepper):
    """Many beds stepped together (one launch per kernel covers all beds)."""

    _batch = True

    def __init__(self, specs, rebuild_every=1, skin=0.0, band_ratio=0.0, cell_factor=0.0, block=0,
                 record_forces=False, persistent=False, device=0, layouts=None, sort_every=0, input_order=False,
                 level_cell_factor=None):
        import torch
        self.device = _gpu_or_raise(device)
        L = load_library()
        self.specs = list(specs)
        self.stream = torch.cuda.Stream(self.device)
        self._holders = []
        for q, s in enumerate(self.specs):
            br, cf = (layouts[q] if layouts is not None else (band_ratio, cell_factor))
            self._holders.append(_DescHolder(s, rebuild_every, skin, br, cf, block, record_forces, persistent,
                                             sort_every, input_order, level_cell_factor))
        arr = (ctypes.POINTER(_Desc) * len(self._holders))(*[ctypes.pointer(h.desc) for h in self._holders])
        self._mem = _TorchMemory(self.device, self.stream)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            rc = L.lpr_batch_create(arr, len(self._holders), ctypes.byref(self._mem.struct),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        _check(rc, "lpr_batch_create")
        self._h = h
        self.n = sum(s.n for s in self.specs)

    def _n(self, bed):
        return self.specs[bed].n

    def __len__(self):
        n = ctypes.c_int32(0)
        _check(_lib.lpr_batch_size(self._h, ctypes.byref(n)), "lpr_batch_size")
        return n.value


def autotune(specs, trial_steps=20, rebuild_every=1, skin=0.0, device=0):
    """Runs the library's autotuner on copies of the beds; returns
    (best setting, list of all trials) as dicts."""
    import torch
    dev = _gpu_or_raise(device)
    L = load_library()
    stream = torch.cuda.Stream(dev)
    holders = [_DescHolder(s, rebuild_every, skin, 0.0, 0.0, 0, False) for s in specs]
    arr = (ctypes.POINTER(_Desc) * len(holders))(*[ctypes.pointer(h.desc) for h in holders])
    mem = _TorchMemory(dev, stream)
    best = _Tuning()
    trials = (_Tuning * 32)()
    nt = ctypes.c_int32(0)
    with torch.cuda.device(dev):
        rc = L.lpr_autotune(arr, len(holders), ctypes.byref(mem.struct), ctypes.c_void_p(stream.cuda_stream),
                            int(trial_steps), ctypes.byref(best), trials, 32, ctypes.byref(nt))
    _check(rc, "lpr_autotune")
    def as_dict(t):
        d = {f: getattr(t, f) for f, _ in _Tuning._fields_}
        d["level_cell_factor"] = [float(x) for x in t.level_cell_factor]
        return d
    return as_dict(best), [as_dict(trials[q]) for q in range(nt.value)]


def plate_reaction_window():
    """torch.autograd.Function: J(theta) = mean plate reaction over a window
    of steps from a bed's current state, theta = (s_k, mu_t, mu_r).

    forward(theta, bed, n_steps, ckpt_every, body) sets the bed's contact
    parameters to theta and runs lpr_adjoint_window, which steps the window
    and computes dJ/dtheta by the hand-written adjoint; backward scales that
    gradient by the incoming one.  The bed advances by the window."""
    import torch

    class PlateReactionWindow(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, bed, n_steps, ckpt_every, body):
            th = theta.detach().double().cpu().numpy()
            bed.set_contact_params(th[0], th[1], th[2])
            J, g = bed.adjoint_window(n_steps, ckpt_every, body)
            ctx.save_for_backward(torch.as_tensor(g, dtype=theta.dtype, device=theta.device))
            return torch.as_tensor(J, dtype=theta.dtype, device=theta.device)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None, None, None, None

    return PlateReactionWindow
