"""Element-wise comparison of GPU outputs with the FP64 oracle.

Rule (tolerance `tol`, default 1e-4):
  - the fit-valid bit (UNKNOWN or not) and the near-degenerate bit match exactly
    (both come from exact integer moments);
  - for valid states |dz| <= tol m, |droll|, |dpitch| <= tol rad;
  - |drisk| <= tol, and the curvature / tilt obstacle bits match, except for
    states whose oracle curvature or tilt lies within tol of its threshold
    (risk jumps to 1 there);
  - the traversable bit matches except for those states and for states whose
    oracle risk lies within tol of risk_max;
  - UNKNOWN states have z = roll = pitch = NaN, risk = 1 and status 0.
The number of exempt states is returned so callers can bound it.
"""
import numpy as np

VALID, CURV, TILT, DEGEN, TRAV = 1, 2, 4, 8, 16


def compare(gpu: dict, orc, params, tol: float = 1e-4, angle_tol: float | None = None) -> dict:
    atol = tol if angle_tol is None else angle_tol
    sg = np.asarray(gpu["status"]).astype(np.int64)
    so = np.asarray(orc.status).astype(np.int64)
    assert sg.shape == so.shape
    vo = (so & VALID) > 0
    vg = (sg & VALID) > 0
    n_valid_mismatch = int(np.count_nonzero(vo != vg))
    assert n_valid_mismatch == 0, f"{n_valid_mismatch} states disagree on UNKNOWN"
    n_degen_mismatch = int(np.count_nonzero((so & DEGEN) != (sg & DEGEN)))
    assert n_degen_mismatch == 0, f"{n_degen_mismatch} states disagree on near-degenerate"

    inv = ~vo
    assert np.all(np.isnan(gpu["z"][inv])) and np.all(np.isnan(gpu["roll"][inv]))
    assert np.all(np.isnan(gpu["pitch"][inv]))
    assert np.all(gpu["risk"][inv] == 1.0) and np.all(sg[inv] == 0)

    near_thr = vo & ((np.abs(orc.phi_x - params.phi_x_max) <= atol) |
                     (np.abs(orc.phi_y - params.phi_y_max) <= atol) |
                     (np.abs(orc.kappa / params.kappa_max - 1.0) <= tol))
    near_risk = vo & (np.abs(orc.risk - params.risk_max) <= tol)

    dz = np.abs(gpu["z"][vo].astype(np.float64) - orc.z[vo])
    droll = np.abs(gpu["roll"][vo].astype(np.float64) - orc.roll[vo])
    dpitch = np.abs(gpu["pitch"][vo].astype(np.float64) - orc.pitch[vo])
    m = vo & ~near_thr
    drisk = np.abs(gpu["risk"][m].astype(np.float64) - orc.risk[m])
    stats = dict(
        n=int(so.size), n_valid=int(vo.sum()),
        max_dz=float(dz.max(initial=0.0)), max_droll=float(droll.max(initial=0.0)),
        max_dpitch=float(dpitch.max(initial=0.0)), max_drisk=float(drisk.max(initial=0.0)),
        mean_dz=float(dz.mean()) if dz.size else 0.0,
        mean_drisk=float(drisk.mean()) if drisk.size else 0.0,
        n_exempt_threshold=int(near_thr.sum()), n_exempt_risk=int(near_risk.sum()),
    )
    assert stats["max_dz"] <= tol, stats
    assert stats["max_droll"] <= atol and stats["max_dpitch"] <= atol, stats
    assert stats["max_drisk"] <= tol, stats
    ob = CURV | TILT
    bad_ob = np.count_nonzero(((sg & ob) != (so & ob)) & m)
    assert bad_ob == 0, f"{bad_ob} obstacle-bit mismatches ({stats})"
    bad_tr = np.count_nonzero(((sg & TRAV) != (so & TRAV)) & vo & ~near_thr & ~near_risk)
    assert bad_tr == 0, f"{bad_tr} traversable-bit mismatches ({stats})"
    # How many exempt states actually came out differently.
    stats["n_exempt_differing"] = int(np.count_nonzero(
        (((sg & (ob | TRAV)) != (so & (ob | TRAV))) & (near_thr | near_risk))))
    # Threshold-adjacent states are a property of the data; they must stay rare.
    assert stats["n_exempt_threshold"] + stats["n_exempt_risk"] <= 0.01 * max(1, stats["n_valid"])
    return stats


def to_numpy(out: dict) -> dict:
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def prefill(out: dict, zval: float = 12345.0):
    """Fill outputs with a sentinel so unwritten states are detectable."""
    for k in ("z", "roll", "pitch", "risk"):
        out[k].fill_(zval)
    out["status"].fill_(255)
    return out


def error_table(gpu: dict, orc, params, tol: float = 1e-4) -> dict:
    """Max and mean |GPU - oracle| per output, over all valid states and over
    the near-degenerate ones.  Risk leaves out states whose oracle curvature
    or tilt lies within tol of its threshold (risk jumps to 1 there)."""
    so = np.asarray(orc.status).astype(np.int64)
    vo = (so & VALID) > 0
    near = vo & ((np.abs(orc.phi_x - params.phi_x_max) <= tol) |
                 (np.abs(orc.phi_y - params.phi_y_max) <= tol) |
                 (np.abs(orc.kappa / params.kappa_max - 1.0) <= tol))
    out = {}
    for subset, m in (("valid", vo), ("near-degenerate", vo & ((so & DEGEN) > 0))):
        row = {"states": int(m.sum())}
        for f in ("z", "roll", "pitch", "risk"):
            mm = m & ~near if f == "risk" else m
            d = np.abs(np.asarray(gpu[f])[mm].astype(np.float64) - getattr(orc, f)[mm])
            row[f] = (float(d.max(initial=0.0)), float(d.mean()) if d.size else 0.0)
        out[subset] = row
    return out
