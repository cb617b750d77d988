"""Audit of the footprint offset geometry for the shipped workloads.

The oracle (gcc) and the HIP library's host code (clang) each build the FP64
grid offsets o = R(theta_k) (u, v) / res on their own.  Both snap components
within 1e-6 of an integer and take floor() of the rest.  They agree on every
snap and floor decision as long as no offset lies within rounding distance of
those decision points; this audit shows a margin of many orders of magnitude
for every workload, so the two independent tables coincide.
"""
import math

import numpy as np
import pytest

from paper_2503_02412_amd import inputs as I

SNAP = 1e-6


def offsets(p, ellipse=False):
    K = p.n_yaw
    i = np.arange(p.fp_nl)[:, None]
    j = np.arange(p.fp_nw)[None, :]
    u = (i + 0.5) * p.fp_length / p.fp_nl - p.fp_length / 2 + 0 * j
    v = (j + 0.5) * p.fp_width / p.fp_nw - p.fp_width / 2 + 0 * i
    out = []
    for k in range(K):
        th = 2.0 * math.pi * k / K
        ox = (u * math.cos(th) - v * math.sin(th)) / p.resolution
        oy = (u * math.sin(th) + v * math.cos(th)) / p.resolution
        out.append(np.stack([ox, oy], -1))
    return np.array(out)          # [K, nl, nw, 2]


@pytest.mark.parametrize("name", ["config1", "config2", "config3", "config5"])
def test_no_knife_edges(name):
    p = I.PRESETS[name]
    o = offsets(p)
    d = np.abs(o - np.round(o))
    snapped = d < SNAP
    # Snapped components are integers up to FP64 rounding ...
    assert np.all(d[snapped] < 1e-12)
    # ... and the rest are far from both the snap threshold and the integers.
    if np.any(~snapped):
        assert d[~snapped].min() > 1e-5
    assert np.all(np.abs(d - SNAP) > 1e-10)


@pytest.mark.parametrize("name", ["config1", "config2", "config3", "config5"])
def test_yaw_zero_offsets_are_quarter_integers(name):
    p = I.PRESETS[name]
    o = offsets(p)[0]
    q = o * 4
    assert np.max(np.abs(q - np.round(q))) < 1e-12


@pytest.mark.parametrize("name", ["config1", "config2", "config3", "config5"])
def test_opposite_yaws_share_sample_positions(name):
    p = I.PRESETS[name]
    o = offsets(p)
    K = p.n_yaw
    for k in range(K // 2):
        a = o[k].reshape(-1, 2)
        b = o[k + K // 2][::-1, ::-1].reshape(-1, 2)     # sample (-p, -q)
        assert np.max(np.abs(a - b)) < 1e-12
