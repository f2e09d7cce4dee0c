"""Shared helpers of the GPU parity tests (HIP library vs FP64 oracle)."""
import math

import numpy as np

from oracle import oracle as O


def oracle_pairs(cs):
    """Oracle (owner, partner code) -> the library's (a, b) convention, sorted."""
    cs = np.asarray(cs, np.int64).reshape(-1, 2).copy()
    sph = cs[:, 1] >= 0
    a = np.where(sph, np.minimum(cs[:, 0], cs[:, 1]), cs[:, 0])
    b = np.where(sph, np.maximum(cs[:, 0], cs[:, 1]), cs[:, 1])
    out = np.stack([a, b], 1)
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def rel_norm(got, ref):
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(np.asarray(got, np.float64) - ref) / den) if den > 0 else float(np.linalg.norm(got))


def masses(spec):
    r = spec.radius.astype(np.float64)
    m = spec.params.rho * 4.0 / 3.0 * math.pi * r ** 3
    return m, 0.4 * m * r ** 2


def oracle_from_gpu(spec, bed, clock=None):
    """An oracle bed at the GPU bed's current state, history and clock."""
    ob = O.OracleBed(spec)
    x, v, w = bed.state()
    ob.set_state(x, v.astype(np.float64), w.astype(np.float64))
    keys, vals = bed.history()
    ob.set_history(keys, vals.astype(np.float64))
    ob.set_clock(bed.clock() if clock is None else clock)
    for q, b in enumerate(spec.bodies):
        if b.z_free:
            o, v3 = bed.body(q)
            ob.set_body_state(q, o[2], v3[2])
    return ob


def compare_one_step(spec, bed, ftol=1e-5, rtol=1e-5):
    """Steps the GPU bed and an oracle copy of its state once; returns a dict
    of the comparisons (contact sets must be equal)."""
    ob = oracle_from_gpu(spec, bed)
    bed.step(1)
    ob.step(1)
    got = bed.contacts()
    ref = oracle_pairs(ob.last_contacts())
    F, T = bed.forces()
    Fo, To = ob.last_forces()
    res = {"contacts_equal": bool(got.shape == ref.shape and np.array_equal(got, ref)), "n_contacts": len(ref),
           "force_rel": rel_norm(F, Fo), "torque_rel": rel_norm(T, To)}
    for q in range(len(spec.bodies)):
        Rg, Ro = bed.reaction(q), ob.last_reaction(q)
        den = np.linalg.norm(Ro[:3])
        res[f"reaction{q}_rel"] = float(np.linalg.norm(Rg[:3] - Ro[:3]) / den) if den > 0 else float(
            np.linalg.norm(Rg[:3]))
    if not res["contacts_equal"]:
        gs, rs = set(map(tuple, got.tolist())), set(map(tuple, ref.tolist()))
        res["only_gpu"] = sorted(gs - rs)[:10]
        res["only_oracle"] = sorted(rs - gs)[:10]
    return res
