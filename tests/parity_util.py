"""Helpers that compare the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (one step, FP32 GPU against FP64 oracle):
  positions    |dx| <= 1e-5 * max(|x|, 0.075 m)
  quaternions  |dq| <= 1e-5
  velocities   |dv| <= 1e-4 * max(|v|, g dt)        angular: 1e-4 * max(|w|, 1 rad/s)
  impulses     |dl| <= 1e-4 * max(|l|, m g dt / 4)  (m g dt / 4 = 1.72e-4 N s for the benchmark block;
                                                    m of the lighter body of the pair in general);
               2e-4 (LAM_TOL_FALLING) for the tilted batches in mid-fall, where the single-precision
               oracle is already 5e-5 to 1e-4 off its FP64 self after one step
               (test_oracle_conditioning.py)
  points       |dp| <= 1e-5 * max(|p|, 0.075 m)
  normals      |dn| <= 1e-5 for face and ground normals; <= 1e-3 for an edge-edge (cross) axis,
               whose direction a_i x b_j / |a_i x b_j| amplifies FP32 rounding by 1 / |a_i x b_j|
  depths       |dd| <= 1e-5 * max(|p|, 0.075 m)  (face and ground; 1e-3 * 0.075 m on cross axes)
Contact-pair sets must agree exactly outside the oracle's precision bands;
colours must agree exactly for towers without a banded pair.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

G_DT = 9.81 / 240.0
LAM_TOL_FALLING = 2e-4
LAM_FLOOR = 0.016875 * 9.81 / 240.0 / 4.0
BAND_MASK = O.BAND_SEPARATION | O.BAND_NORMAL | O.BAND_CROSS | O.BAND_CLIP | O.BAND_GROUND | O.BAND_EMPTY


def gpu_manifolds(contacts, first_body: int) -> dict:
    """Group GPU contact points by (a, b) with tower-local body indices (ground = -1)."""
    out = {}
    for c in contacts:
        a = int(c["body_a"]) - first_body
        b = int(c["body_b"])
        b = -1 if b < 0 else b - first_body
        m = out.setdefault((a, b), dict(colour=int(c["colour"]), order=int(c["order"]), slot=[], point=[], lam=[],
                                       normal=np.array(c["normal"], np.float64), t1=np.array(c["t1"], np.float64),
                                       depth=float(c["depth"])))
        m["slot"].append(int(c["slot"]))
        m["point"].append(np.array(c["point"], np.float64))
        m["lam"].append([float(c["lambda_n"]), float(c["lambda_t1"]), float(c["lambda_t2"])])
    for m in out.values():
        m["point"] = np.array(m["point"]).reshape(-1, 3)
        m["lam"] = np.array(m["lam"]).reshape(-1, 3)
    return out


def oracle_manifolds(ow, t: int) -> dict:
    return {(m["a"], m["b"]): m for m in ow.manifolds(t)}


def compare_contacts(om: dict, gm: dict, masses=None, impulses: bool = True, lam_tol: float = 1e-4,
                     point_tol: float = 1e-5) -> dict:
    """Returns a report; 'ok' is True when every check inside the tolerances passes.
    masses (tower-local, optional): the impulse floor of a pair is then m g dt / 4 of its lighter
    body (the ground counts as infinitely heavy) instead of the benchmark block's.
    impulses=False skips the impulse comparison (statically indeterminate contact sets, where
    only the bodies' net impulses, fixed by the velocities, are unique); lam_tol, point_tol: the
    impulse and point tolerances (1e-4 and 1e-5 by default)."""
    rep = dict(pairs=len(om), banded=0, missing=[], extra=[], colour_mismatch=[], slot_mismatch=[],
               point_err=0.0, lam_err=0.0, normal_err=0.0, normal_err_cross=0.0, depth_err=0.0,
               depth_err_cross=0.0, colours_checked=False)
    banded = {k for k, m in om.items() if m["band"] & BAND_MASK}
    rep["banded"] = len(banded)
    okeys = set(om) - banded
    gkeys = set(gm) - banded
    rep["missing"] = sorted(okeys - gkeys)
    rep["extra"] = sorted(gkeys - okeys)
    # colours are a function of the whole pair set; compare them when the sets agree exactly
    if set(om) == set(gm):
        rep["colours_checked"] = True
        for k in om:
            if om[k]["colour"] != gm[k]["colour"]:
                rep["colour_mismatch"].append(k)
    for k in okeys & gkeys:
        o, g = om[k], gm[k]
        cross = o["axis"] >= 6        # an edge-edge axis (the ground has axis -1)
        en = float(np.abs(o["normal"] - g["normal"]).max())
        pscale = max(float(np.linalg.norm(o["point"], axis=1).max(initial=0.0)), 0.075)
        ed = abs(float(o["depth"]) - float(g["depth"])) / pscale
        if cross:
            rep["normal_err_cross"] = max(rep["normal_err_cross"], en)
            rep["depth_err_cross"] = max(rep["depth_err_cross"], ed)
        else:
            rep["normal_err"] = max(rep["normal_err"], en)
            rep["depth_err"] = max(rep["depth_err"], ed)
        if list(o["slot"]) != list(g["slot"]):
            rep["slot_mismatch"].append((k, list(o["slot"]), list(g["slot"])))
            continue
        scale = np.maximum(np.linalg.norm(o["point"], axis=1), 0.075)
        rep["point_err"] = max(rep["point_err"], float((np.linalg.norm(o["point"] - g["point"], axis=1) / scale).max()))
        floor = LAM_FLOOR
        if masses is not None:
            a, b = k
            mm = masses[a] if b < 0 else min(masses[a], masses[b])
            floor = mm * G_DT / 4.0
        lam_scale = np.maximum(np.abs(o["lam"]), floor)
        if impulses:
            rep["lam_err"] = max(rep["lam_err"], float((np.abs(o["lam"] - g["lam"]) / lam_scale).max()))
    rep["ok"] = (not rep["missing"] and not rep["extra"] and not rep["colour_mismatch"] and not rep["slot_mismatch"]
                 and rep["point_err"] <= point_tol and rep["lam_err"] <= lam_tol
                 and rep["normal_err"] <= 1e-5 and rep["depth_err"] <= 1e-5
                 and rep["normal_err_cross"] <= 1e-3 and rep["depth_err_cross"] <= 1e-3)
    return rep


def compare_state(ow, gpos, gquat, gv, gw, idx=None, vtol: float = 1e-4) -> dict:
    """Positions and orientations at 1e-5, velocities at vtol (1e-4 by default)."""
    idx = slice(None) if idx is None else idx
    x, q, v, w = ow.x[idx], ow.q[idx], ow.v[idx], ow.w[idx]
    gx, gq, gvv, gww = gpos[idx], gquat[idx], gv[idx], gw[idx]
    # quaternions q and -q are the same rotation
    sgn = np.sign(np.sum(q * gq, axis=1, keepdims=True))
    sgn[sgn == 0] = 1
    ex = float((np.linalg.norm(x - gx, axis=1) / np.maximum(np.linalg.norm(x, axis=1), 0.075)).max(initial=0))
    eq = float(np.abs(q - sgn * gq).max(initial=0))
    ev = float((np.linalg.norm(v - gvv, axis=1) / np.maximum(np.linalg.norm(v, axis=1), G_DT)).max(initial=0))
    ew = float((np.linalg.norm(w - gww, axis=1) / np.maximum(np.linalg.norm(w, axis=1), 1.0)).max(initial=0))
    return dict(x=ex, q=eq, v=ev, w=ew, ok=(ex <= 1e-5 and eq <= 1e-5 and ev <= vtol and ew <= vtol))


def fmt(rep: dict) -> str:
    keys = [k for k in rep if k not in ("ok",)]
    return ", ".join(f"{k}={rep[k] if not isinstance(rep[k], list) else rep[k][:4]}" for k in keys)


# ---------------------------------------------------------------------------------------------
# per-point feature records (24 features, k[3], impulses[3])
# ---------------------------------------------------------------------------------------------

def oracle_records(ow, t: int) -> dict:
    """(a, b, slot) -> (record, band) from the oracle's last recorded step of tower t."""
    recs = ow.features[t]
    out, o = {}, 0
    for m in ow.manifolds(t):
        for i in range(m["npts"]):
            out[(m["a"], m["b"], int(m["slot"][i]))] = (recs[o], m["band"])
            o += 1
    assert o == len(recs)
    return out


def gpu_records(contacts, records, first_body: int) -> dict:
    assert len(contacts) == len(records)
    out = {}
    for c, r in zip(contacts, records):
        a = int(c["body_a"]) - first_body
        b = int(c["body_b"])
        b = -1 if b < 0 else b - first_body
        out[(a, b, int(c["slot"]))] = np.asarray(r, np.float64)
    return out


def compare_records(om: dict, gm: dict, lam_tol: float = 1e-4) -> dict:
    """Largest scaled error per record group over the points outside the precision bands.
    Each group's error is already divided by its tolerance: ok means every value <= 1."""
    keys = [k for k, (_, band) in om.items() if not band & BAND_MASK]
    rep = dict(points=len(keys), missing=[k for k in keys if k not in gm])
    groups = dict(pos=0.0, quat=0.0, normal=0.0, depth=0.0, mu=0.0, prev=0.0, lever=0.0, vel=0.0, k=0.0, lam=0.0)
    for key in keys:
        if key not in gm:
            continue
        o, g = om[key][0], gm[key]
        d = np.abs(o - g)
        groups["pos"] = max(groups["pos"], float((d[0:3] / np.maximum(np.abs(o[0:3]), 0.075)).max() / 1e-5))
        groups["quat"] = max(groups["quat"], float(d[3:7].max() / 1e-5))
        groups["normal"] = max(groups["normal"], float(d[7:10].max() / 1e-5))
        groups["depth"] = max(groups["depth"], float(d[10] / (1e-5 * 0.075)))
        groups["mu"] = max(groups["mu"], float(d[11] / 1e-7))
        # previous impulses in the outputs' units lambda k / (|g| dt): the impulse tolerance scaled alike
        prev_floor = LAM_FLOOR * np.abs(o[24:27]) / G_DT
        groups["prev"] = max(groups["prev"], float((d[12:15] / np.maximum(np.abs(o[12:15]), prev_floor)).max() / 1e-4))
        groups["lever"] = max(groups["lever"], float(d[15:21].max() / (1e-5 * 0.075)))
        groups["vel"] = max(groups["vel"], float((d[21:24] / np.maximum(np.abs(o[21:24]), G_DT)).max() / 1e-4))
        groups["k"] = max(groups["k"], float((d[24:27] / np.abs(o[24:27])).max() / 1e-5))
        groups["lam"] = max(groups["lam"], float((d[27:30] / np.maximum(np.abs(o[27:30]), LAM_FLOOR)).max() / lam_tol))
    rep.update(groups)
    rep["ok"] = not rep["missing"] and all(v <= 1.0 for v in groups.values())
    return rep


def impulses_feasible(contacts, mu: float) -> bool:
    """Every GPU impulse satisfies lambda_n >= 0 and |lambda_t| <= mu lambda_n (the clip of
    Eq. (coulomb_pgs), taken after the point's last normal update)."""
    ln = np.asarray(contacts["lambda_n"], np.float64)
    lt = np.abs(np.stack([contacts["lambda_t1"], contacts["lambda_t2"]], 1).astype(np.float64))
    bound = mu * ln[:, None] * (1.0 + 1e-6) + 1e-30
    return bool(np.all(ln >= 0.0) and np.all(lt <= bound))
