"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads oracle/liblproracle.so, built from
oracle/oracle.cpp by build() (plain g++, -ffp-contract=off, OpenMP).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblproracle.so")


def build(verbose=False) -> str:
    """Compiles the oracle with g++ (FP64, no FMA contraction, OpenMP)."""
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", os.path.join(HERE, "oracle.cpp"), "-o", LIB + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


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


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_create.restype = vp
        L.orc_create.argtypes = [i64, vp, vp, vp, vp, vp, ctypes.c_uint32, ctypes.POINTER(_Params), i32, vp, i32, vp]
        L.orc_destroy.argtypes = [vp]
        for name, args in [("orc_set_state", [vp, vp, vp, vp]), ("orc_get_state", [vp, vp, vp, vp]),
                           ("orc_set_clock", [vp, i64]), ("orc_set_body_state", [vp, i32, d, d]),
                           ("orc_get_body_state", [vp, i32, vp, vp]), ("orc_get_history", [vp, vp, vp, i64]),
                           ("orc_set_history", [vp, i64, vp, vp]), ("orc_step", [vp, i64]),
                           ("orc_contact_set", [vp, i32, vp, i64, vp]), ("orc_last_contacts", [vp, vp, i64, vp]),
                           ("orc_last_forces", [vp, vp, vp]), ("orc_last_reaction", [vp, i32, vp]),
                           ("orc_tangent_window", [vp, i64, i32, i32, vp, vp]),
                           ("orc_last_contact_loads", [vp, vp, vp, vp]), ("orc_wall_pose", [vp, i32, vp]),
                           ("orc_last_contact_scales", [vp, vp, vp]),
                           ("orc_set_stepper", [vp, i32, i32])]:
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = args
        L.orc_history_count.restype = i64
        L.orc_history_count.argtypes = [vp]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None else None


def _params(p) -> _Params:
    q = _Params()
    for f in ("rho", "E", "nu", "mu_t", "mu_r", "dt", "gamma_factor", "e_H", "kappa_t", "s_k"):
        setattr(q, f, p.field(f))
    for a in range(3):
        q.g[a] = float(p.g[a])
    return q


def set_threads(n: int) -> int:
    return lib().orc_set_threads(int(n))


class OracleBed:
    """FP64 oracle bed built from a beds.BedSpec."""

    def __init__(self, spec):
        L = lib()
        self.spec = spec
        self.n = spec.n
        self._pos = np.ascontiguousarray(spec.pos, np.float64)
        self._rad = np.ascontiguousarray(spec.radius, np.float32)
        self._vel = np.ascontiguousarray(spec.vel, np.float32)
        self._omg = np.ascontiguousarray(spec.omega, np.float32)
        box = np.array(spec.box, np.float64)
        self._prm = _params(spec.params)
        walls = (_Wall * max(1, len(spec.walls)))()
        for q, w in enumerate(spec.walls):
            walls[q].kind, walls[q].body = int(w.kind), int(w.body)
            for a in range(3):
                walls[q].origin[a], walls[q].axis[a], walls[q].dims[a] = w.origin[a], w.axis[a], w.dims[a]
            for a in range(9):
                walls[q].frame[a] = w.frame[a]
            walls[q].mu_t, walls[q].mu_r = float(w.mu_t), float(w.mu_r)
        bodies = (_Body * max(1, len(spec.bodies)))()
        for q, b in enumerate(spec.bodies):
            for a in range(3):
                bodies[q].origin[a], bodies[q].lin_vel[a] = b.origin[a], b.lin_vel[a]
            bodies[q].ang_vel, bodies[q].z_free, bodies[q].mass = float(b.ang_vel), int(b.z_free), float(b.mass)
        self._h = L.orc_create(self.n, _ptr(self._pos), _ptr(self._rad), _ptr(self._vel), _ptr(self._omg),
                               box.ctypes.data, int(spec.periodic), ctypes.byref(self._prm), len(spec.walls),
                               ctypes.addressof(walls), len(spec.bodies), ctypes.addressof(bodies))
        if not self._h:
            raise ValueError("oracle rejected the bed description")

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def _ok(self, rc, what):
        if rc != 0:
            raise RuntimeError(f"oracle {what} failed ({rc})")

    def step(self, n=1):
        self._ok(lib().orc_step(self._h, int(n)), "step")

    def set_stepper(self, kind, n_iter=0):
        """kind "explicit" (the compliant step) or "spook" (the time-implicit
        step with n_iter projected iterations); see lpr_oracle.h."""
        k = {"explicit": 0, "spook": 1}[kind]
        self._ok(lib().orc_set_stepper(self._h, k, int(n_iter)), "set_stepper")

    def state(self):
        pos = np.zeros((self.n, 3)); vel = np.zeros((self.n, 3)); omg = np.zeros((self.n, 3))
        self._ok(lib().orc_get_state(self._h, _ptr(pos), _ptr(vel), _ptr(omg)), "get_state")
        return pos, vel, omg

    def set_state(self, pos=None, vel=None, omg=None):
        c = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
        pos, vel, omg = c(pos), c(vel), c(omg)
        self._ok(lib().orc_set_state(self._h, _ptr(pos), _ptr(vel), _ptr(omg)), "set_state")

    def set_clock(self, step):
        self._ok(lib().orc_set_clock(self._h, int(step)), "set_clock")

    def set_body_state(self, body, z, vz):
        self._ok(lib().orc_set_body_state(self._h, int(body), float(z), float(vz)), "set_body_state")

    def body_state(self, body):
        o = np.zeros(3); v = np.zeros(3)
        self._ok(lib().orc_get_body_state(self._h, int(body), _ptr(o), _ptr(v)), "body_state")
        return o, v

    def history(self):
        n = lib().orc_history_count(self._h)
        keys = np.zeros((max(n, 1), 2), np.int64); vals = np.zeros((max(n, 1), 6))
        self._ok(lib().orc_get_history(self._h, _ptr(keys), _ptr(vals), n), "get_history")
        return keys[:n], vals[:n]

    def set_history(self, keys, vals):
        keys = np.ascontiguousarray(keys, np.int64).reshape(-1, 2)
        vals = np.ascontiguousarray(vals, np.float64).reshape(-1, 6)
        self._ok(lib().orc_set_history(self._h, len(keys), _ptr(keys), _ptr(vals)), "set_history")

    def contact_set(self, method=0):
        """Contact set at the current state: (k, 2) int64 (owner, partner code)."""
        tot = ctypes.c_int64(0)
        lib().orc_contact_set(self._h, int(method), None, 0, ctypes.byref(tot))
        out = np.zeros((max(tot.value, 1), 2), np.int64)
        self._ok(lib().orc_contact_set(self._h, int(method), _ptr(out), tot.value, ctypes.byref(tot)),
                 "contact_set")
        return out[:tot.value]

    def last_contacts(self):
        tot = ctypes.c_int64(0)
        lib().orc_last_contacts(self._h, None, 0, ctypes.byref(tot))
        out = np.zeros((max(tot.value, 1), 2), np.int64)
        self._ok(lib().orc_last_contacts(self._h, _ptr(out), tot.value, ctypes.byref(tot)), "last_contacts")
        return out[:tot.value]

    def last_forces(self):
        F = np.zeros((self.n, 3)); T = np.zeros((self.n, 3))
        self._ok(lib().orc_last_forces(self._h, _ptr(F), _ptr(T)), "last_forces")
        return F, T

    def last_reaction(self, body):
        out = np.zeros(6)
        self._ok(lib().orc_last_reaction(self._h, int(body), _ptr(out)), "last_reaction")
        return out

    def last_contact_loads(self):
        """Per contact of the last step (last_contacts order): force on the
        owner (k, 3), rolling moment on the owner (k, 3), F_n (k,)."""
        k = len(self.last_contacts())
        F = np.zeros((max(k, 1), 3)); M = np.zeros((max(k, 1), 3)); fn = np.zeros(max(k, 1))
        self._ok(lib().orc_last_contact_loads(self._h, _ptr(F), _ptr(M), _ptr(fn)), "last_contact_loads")
        return F[:k], M[:k], fn[:k]

    def last_contact_scales(self):
        """Per contact of the last explicit step (last_contacts order): the
        summed magnitudes of the law's force terms and of its moment terms."""
        k = len(self.last_contacts())
        sF = np.zeros(max(k, 1)); sM = np.zeros(max(k, 1))
        self._ok(lib().orc_last_contact_scales(self._h, _ptr(sF), _ptr(sM)), "last_contact_scales")
        return sF[:k], sM[:k]

    def wall_pose(self, wall):
        """World pose of a wall at the current clock: origin, normal, frame (3 x 3 rows)."""
        out = np.zeros(15)
        self._ok(lib().orc_wall_pose(self._h, int(wall), _ptr(out)), "wall_pose")
        return out[0:3], out[3:6], out[6:15].reshape(3, 3)

    def tangent_window(self, n_steps, body, component=2):
        """Mean of one reaction component over n_steps and its derivative
        with respect to (s_k, mu_t, mu_r)."""
        J = ctypes.c_double(0.0)
        g = np.zeros(3)
        self._ok(lib().orc_tangent_window(self._h, int(n_steps), int(body), int(component), ctypes.byref(J),
                                          _ptr(g)), "tangent_window")
        return J.value, g
