"""C-ABI library checks that need no GPU: it loads, exports every symbol the
public header declares, validates configurations, and plans window moves with
exactly the geometry a brute force over the oracle's footprint reach gives."""
import math
import os
import re

import numpy as np
import pytest

from paper_2503_02412_amd import inputs as I
from paper_2503_02412_amd import seb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "seb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(seb_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    import ctypes
    L = seb.lib()
    syms = header_symbols()
    assert "seb_assess_se2" in syms and "seb_update_window" in syms
    for s in syms:
        assert hasattr(L, s), s
        assert isinstance(getattr(L, s), ctypes._CFuncPtr)
    assert seb.version().startswith("seb-mi355x")


def test_strerror_covers_all_codes():
    L = seb.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.seb_strerror(code).decode() != "unknown status"


@pytest.mark.parametrize("name", list(I.PRESETS))
def test_presets_are_valid(name):
    assert seb.validate(I.PRESETS[name]) == seb.SEB_OK


@pytest.mark.parametrize("change,code", [
    (dict(width=0), seb.SEB_ERR_INVALID),
    (dict(resolution=0.0), seb.SEB_ERR_INVALID),
    (dict(resolution=float("nan")), seb.SEB_ERR_INVALID),
    (dict(n_yaw=0), seb.SEB_ERR_INVALID),
    (dict(fp_nl=0), seb.SEB_ERR_INVALID),
    (dict(fp_length=-1.0), seb.SEB_ERR_INVALID),
    (dict(fp_shape=2), seb.SEB_ERR_INVALID),
    (dict(kappa_max=0.0), seb.SEB_ERR_INVALID),
    (dict(min_valid=2), seb.SEB_ERR_INVALID),
    (dict(precision=3), seb.SEB_ERR_INVALID),
    (dict(fit=2), seb.SEB_ERR_INVALID),
    (dict(fp_length=12.0, fp_width=12.0), seb.SEB_ERR_UNSUPPORTED),   # halo too wide for LDS
])
def test_invalid_configs_are_rejected(change, code):
    assert seb.validate(I.CONFIG1.with_(**change)) == code
    assert seb.lib().seb_last_error().decode() != ""


def brute_band(params, reach, ox, oy, nox, noy):
    """States of the new window whose footprint box meets a changed cell."""
    W, H = params.width, params.height
    dx0, dx1, dy0, dy1 = reach
    dx, dy = nox - ox, noy - oy
    pad = max(-dx0, dx1, -dy0, dy1) + 1
    xs = np.arange(-pad, W + pad)
    ys = np.arange(-pad, H + pad)
    X, Y = np.meshgrid(xs, ys)
    in_new = (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
    in_old = (X >= -dx) & (X < W - dx) & (Y >= -dy) & (Y < H - dy)
    changed = (in_new & ~in_old) | (in_old & ~in_new)
    # 2-D prefix sums to test every state's reach box
    cs = np.zeros((changed.shape[0] + 1, changed.shape[1] + 1), np.int64)
    cs[1:, 1:] = changed.cumsum(0).cumsum(1)
    iy, ix = np.mgrid[0:H, 0:W]
    x0, x1 = ix + dx0 + pad, ix + dx1 + pad + 1
    y0, y1 = iy + dy0 + pad, iy + dy1 + pad + 1
    cnt = cs[y1, x1] - cs[y0, x1] - cs[y1, x0] + cs[y0, x0]
    return cnt > 0, changed & in_new


@pytest.mark.parametrize("pname", ["config1", "config3"])
def test_window_plan_matches_brute_force(pname):
    import oracle
    p = I.PRESETS[pname]
    reach = oracle.reach(p)
    rng = np.random.default_rng(11)
    res = p.resolution
    W, H = p.width, p.height
    for trial in range(60):
        x, y = rng.uniform(-5, 5, 2)
        ox = math.floor(x / res) - W // 2
        oy = math.floor(y / res) - H // 2
        step = rng.choice([0.0, 0.1, 0.5, 1.0, 3.0]) * (W * res / 10)
        ang = rng.uniform(0, 2 * math.pi)
        nx_, ny_ = x + step * math.cos(ang), y + step * math.sin(ang)
        plan = seb.plan_window_move(p, ox, oy, nx_, ny_)
        nox = math.floor(nx_ / res) - W // 2
        noy = math.floor(ny_ / res) - H // 2
        assert (plan.new_origin_x, plan.new_origin_y) == (nox, noy)
        band = np.zeros((H, W), bool)
        area = 0
        for r in range(plan.n_rects):
            x0, y0, w, h = plan.rects[r]
            assert w > 0 and h > 0 and x0 >= 0 and y0 >= 0 and x0 + w <= W and y0 + h <= H
            assert not band[y0:y0 + h, x0:x0 + w].any(), "rectangles overlap"
            band[y0:y0 + h, x0:x0 + w] = True
            area += w * h
        assert plan.n_states == area * p.n_yaw
        if abs(nox - ox) >= W or abs(noy - oy) >= H:
            assert plan.full_reset == 1 and band.all()
            continue
        expect, exposed = brute_band(p, reach, ox, oy, nox, noy)
        assert plan.n_cells_exposed == exposed.sum()
        assert plan.exposed_rows == abs(noy - oy) and plan.exposed_cols == abs(nox - ox)
        # The plan recomputes exactly the affected states.
        assert np.array_equal(band, expect), trial


def test_window_plan_rejects_bad_input():
    with pytest.raises(seb.SebError):
        seb.plan_window_move(I.CONFIG1, 0, 0, float("nan"), 0.0)
    with pytest.raises(seb.SebError):
        seb.plan_window_move(I.CONFIG1.with_(width=0), 0, 0, 0.0, 0.0)
