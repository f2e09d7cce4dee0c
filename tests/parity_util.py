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


def oracle_contact_loads(ob):
    """The oracle's per-contact loads of its last step in the library's
    convention: pairs (a, b) ascending, force and rolling moment on particle
    a (the oracle keeps them for the owner, which is b when b < owner id),
    F_n, and the magnitudes of the law's force and moment terms."""
    cs = np.asarray(ob.last_contacts(), np.int64).reshape(-1, 2)
    F, M, fn = ob.last_contact_loads()
    sF, sM = ob.last_contact_scales()
    sph = cs[:, 1] >= 0
    flip = sph & (cs[:, 1] < cs[:, 0])
    a = np.where(flip, cs[:, 1], cs[:, 0])
    b = np.where(flip, cs[:, 0], cs[:, 1])
    sg = np.where(flip, -1.0, 1.0)[:, None]
    order = np.lexsort((b, a))
    return (np.stack([a, b], 1)[order], (sg * F)[order], (sg * M)[order], fn[order], sF[order], sM[order])


def gross_loads(spec, pairs, F, M, sF, sM):
    """Per particle, the scales that FP32 rounding of its summed contact
    force and torque is relative to: over its contacts, the magnitude of the
    contact force plus the magnitudes of the law's terms that made it (an
    elastic and a damping normal term can nearly cancel, as can a spring
    and its damping), and for the torque the same times the lever (at most
    the radius) plus the rolling moment and its terms."""
    n = spec.n
    r = spec.radius.astype(np.float64)
    fm = np.linalg.norm(F, axis=1) + sF
    mm = np.linalg.norm(M, axis=1) + sM
    G = np.zeros(n)
    Gt = np.zeros(n)
    a, b = pairs[:, 0], pairs[:, 1]
    np.add.at(G, a, fm)
    np.add.at(Gt, a, r[a] * fm + mm)
    sph = b >= 0
    np.add.at(G, b[sph], fm[sph])
    np.add.at(Gt, b[sph], r[b[sph]] * fm[sph] + mm[sph])
    return G, Gt


def compare_one_step(spec, bed, ftol=1e-5, rtol=1e-5):
    """Steps the GPU bed and an oracle copy of its state once; returns a dict
    of the comparisons (contact sets must be equal).

    Besides the normwise force and torque errors over all particles:
    - per contact (bed created with record_forces), the largest relative
      error of the contact force and of F_n over the contacts with
      F_n >= 1e-3 max F_n, and the normwise rolling-moment error;
    - per particle, the largest error of its summed force relative to the
      sum over its contacts of the force magnitude and the law's term
      magnitudes (and the same for the torque), so an error confined to the
      light fine spheres shows;
    - the normwise torque error also against 1e-2 of the norm of those
      per-particle torque scales, for beds whose net torques are rounding
      noise (spheres at rest);
    - per body, the reaction force relative to its norm and the reaction
      torque relative to sum |x - o| |F| + |M| over the body's contacts."""
    ob = oracle_from_gpu(spec, bed)
    bed.step(1)
    ob.step(1)
    got = bed.contacts()
    ref = oracle_pairs(ob.last_contacts())
    F, T = bed.forces()
    Fo, To = ob.last_forces()
    res = {"contacts_equal": bool(got.shape == ref.shape and np.array_equal(got, ref)), "n_contacts": len(ref),
           "force_rel": rel_norm(F, Fo), "torque_rel": rel_norm(T, To)}
    if not res["contacts_equal"]:
        gs, rs = set(map(tuple, got.tolist())), set(map(tuple, ref.tolist()))
        res["only_gpu"] = sorted(gs - rs)[:10]
        res["only_oracle"] = sorted(rs - gs)[:10]
        return res
    pairs, Fc, Mc, fn = bed.contact_loads()
    po, Fco, Mco, fno, sFo, sMo = oracle_contact_loads(ob)
    res["loads_pairs_equal"] = bool(np.array_equal(pairs, po) and np.array_equal(pairs, ref))
    if len(fno):
        sel = fno >= 1e-3 * fno.max()
        dF = np.linalg.norm(Fc.astype(np.float64) - Fco, axis=1)
        res["contact_force_max_rel"] = float(np.max(dF[sel] / np.linalg.norm(Fco[sel], axis=1)))
        res["contact_fn_max_rel"] = float(np.max(np.abs(fn[sel] - fno[sel]) / fno[sel]))
        res["contact_moment_rel"] = rel_norm(Mc[sel], Mco[sel])
        res["contacts_checked"] = int(sel.sum())
    G, Gt = gross_loads(spec, po, Fco, Mco, sFo, sMo)
    act = G > 0
    dFp = np.linalg.norm(F.astype(np.float64) - Fo, axis=1)
    dTp = np.linalg.norm(T.astype(np.float64) - To, axis=1)
    res["particle_force_max_rel"] = float(np.max(dFp[act] / G[act])) if act.any() else 0.0
    res["particle_torque_max_rel"] = float(np.max(dTp[act] / Gt[act])) if act.any() else 0.0
    if act.any():   # the worst particle, for diagnosis
        w = int(np.argmax(np.where(act, dFp / np.where(act, G, 1.0), 0.0)))
        res["worst_particle"] = {"id": w, "dF": float(dFp[w]), "F": float(np.linalg.norm(Fo[w])),
                                 "scale": float(G[w]), "contacts": int(np.sum((po[:, 0] == w) | (po[:, 1] == w)))}
    res["torque_rel_scaled"] = float(np.linalg.norm(T.astype(np.float64) - To) /
                                     max(np.linalg.norm(To), 1e-2 * np.linalg.norm(Gt), 1e-300))
    res["free_particles_max_force"] = float(np.max(np.abs(F[~act]))) if (~act).any() else 0.0
    for q in range(len(spec.bodies)):
        Rg, Ro = bed.reaction(q), ob.last_reaction(q)
        den = np.linalg.norm(Ro[:3])
        res[f"reaction{q}_rel"] = float(np.linalg.norm(Rg[:3] - Ro[:3]) / den) if den > 0 else float(
            np.linalg.norm(Rg[:3]))
        walls = [w for w, W in enumerate(spec.walls) if W.body == q]
        on = np.isin(po[:, 1], [-1 - w for w in walls])
        if on.any():
            o, _ = bed.body(q)
            xa = spec_positions_at(bed, po[on, 0])
            lever = np.linalg.norm(xa - o, axis=1) + spec.radius[po[on, 0]].astype(np.float64)
            scale = float(np.sum(lever * (np.linalg.norm(Fco[on], axis=1) + sFo[on]) +
                                 np.linalg.norm(Mco[on], axis=1) + sMo[on]))
            res[f"reaction{q}_torque_rel"] = float(np.linalg.norm(Rg[3:] - Ro[3:]) / scale)
        else:
            res[f"reaction{q}_torque_rel"] = float(np.linalg.norm(Rg[3:] - Ro[3:]))
    return res


def spec_positions_at(bed, ids):
    """Positions of the given particles after the bed's last step (the
    lever of a body contact differs from the one at the start of the step by
    dt |v|, far below the bound's scale)."""
    x, _, _ = bed.state()
    return x[ids]


def assert_parity(res, tol=1e-5, loads=True):
    """The GPU-vs-oracle bars of one compared step."""
    assert res["contacts_equal"], res
    assert res["force_rel"] < tol and res["torque_rel_scaled"] < tol, res
    assert res["particle_force_max_rel"] < tol and res["particle_torque_max_rel"] < tol, res
    assert res["free_particles_max_force"] == 0.0, res
    if loads and res["n_contacts"]:
        assert res["loads_pairs_equal"], res
        assert res["contact_force_max_rel"] < tol and res["contact_fn_max_rel"] < tol, res
        assert res["contact_moment_rel"] < tol, res
    for k, v in res.items():
        if k.startswith("reaction") and k.endswith("_rel"):
            assert v < tol, (k, res)


def relax_on_gpu(spec, steps, chunk=5000):
    """Relaxes a deposited bed on the GPU (the paper's relaxation friction,
    frictionless walls, dt 5e-6 s, gamma_n = 10 dt, candidate lists with a
    skin of a quarter of the smallest radius) and returns a copy of `spec`
    at rest in the relaxed positions."""
    from paper_2501_05300_amd import beds
    from paper_2501_05300_amd.lprdem import Bed
    relax = spec.copy()
    relax.params = beds.settle_params(spec.params).replace(dt=5e-6, gamma_factor=10.0)
    for w in relax.walls:
        w.mu_t, w.mu_r = 0.0, 0.0
    rb = Bed(relax, rebuild_every=5, skin=0.25 * float(spec.radius.min()))
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        rb.step(k)
        rb.sync()
        done += k
    x, _, _ = rb.state()
    rb.close()
    out = spec.copy()
    out.pos = x
    out.vel = np.zeros_like(out.vel)
    out.omega = np.zeros_like(out.omega)
    return out
