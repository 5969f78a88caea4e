"""Coupled-step pins of the FP64 oracle: rigid-limit capsules in shear flow.

A capsule in plane Couette flow must rotate as Jeffery's solution (Eq. (19),
Sec. 3.1) says: a sphere spins at half the shear rate, an ellipsoid tumbles
with period T = 2 pi / gamma (a/b + b/a).  These runs exercise forces,
spreading, moments, interpolation and the node update together.
"""
import numpy as np
import pytest

import oracle
from paper_1704_04551_amd import workloads as W


def _couette(n, U):
    ulo = np.zeros((3, 3)); uhi = np.zeros((3, 3))
    ulo[2, 0] = -U; uhi[2, 0] = U
    return ulo, uhi


def _spin(X, U):
    """Least-squares rigid rotation rate of the node cloud."""
    c = X.mean(0)
    r = X - c
    V = U.mean(0)
    A = np.zeros((3 * len(r), 3))
    for i, ri in enumerate(r):
        A[3 * i:3 * i + 3] = [[0, ri[2], -ri[1]], [-ri[2], 0, ri[0]], [ri[1], -ri[0], 0]]
    return np.linalg.lstsq(A, (U - V).reshape(-1), rcond=None)[0]


def test_sphere_spins_at_half_shear_rate():
    """A stiff spherical capsule at the channel centre spins about the
    vorticity axis at gamma/2 (Jeffery's a = b limit), and by symmetry its
    centroid stays put.  Measured 0.96 gamma/2 at this resolution (radius 5,
    H = 30): the band below allows for confinement and kernel smearing."""
    n = (32, 32, 32)
    U = 0.01
    gam = 2 * U / (n[2] - 2)
    ulo, uhi = _couette(n, U)
    S, T = W.icosphere(3)
    c = (np.array(n) - 1) / 2.0
    x = S * 5.0 + c
    s = oracle.OracleSim(n, 1.0, wall=(0, 0, 1), u_lo=ulo, u_hi=uhi, delta="peskin4",
                         init_profile=1)
    t = s.add_template(T, x)
    s.add_mesh(t, x, 0.05, 0.001)
    s.step(1000)
    X, Un, F = s.nodes(0)
    om = _spin(X, Un)
    ratio = om[1] / (gam / 2)
    assert 0.94 < ratio < 1.0, ratio
    assert abs(om[0]) < 1e-12 and abs(om[2]) < 1e-12
    assert np.abs(X.mean(0) - c).max() < 1e-10


def _quarter_period(n, a, b, gam, tau, ks, kb, every=25, max_steps=20000):
    """Steps until the major axis has turned by pi/2 from the flow direction."""
    H = n[2] - 2
    ulo, uhi = _couette(n, gam * H / 2)
    S, T = W.icosphere(3)
    x = W.ellipsoid(S, a, b, b) + (np.array(n) - 1) / 2.0
    s = oracle.OracleSim(n, tau, wall=(0, 0, 1), u_lo=ulo, u_hi=uhi, delta="peskin4",
                         init_profile=1)
    t = s.add_template(T, x)
    s.add_mesh(t, x, ks, kb)
    prev = 0.0
    acc = 0.0
    steps = 0
    while steps < max_steps:
        s.step(every)
        steps += every
        X, _, _ = s.nodes(0)
        r = X - X.mean(0)
        w, v = np.linalg.eigh(r.T @ r)
        ax = v[:, -1]
        ang = np.arctan2(ax[2], ax[0])
        acc += (ang - prev + np.pi / 2) % np.pi - np.pi / 2
        prev = ang
        if abs(acc) >= np.pi / 2:
            return steps
    return None


def test_jeffery_quarter_period():
    """Prolate capsule a = 6, b = c = 3 at Re = 0.34: the major axis reaches
    pi/2 at T/4 = (pi / (2 gamma)) (a/b + b/a) by Eq. (19).  At this
    resolution (minor semi-axis 3 lattice units) the oracle is 8-10 % slow;
    the band below states that."""
    gam = 0.00314
    q = _quarter_period((40, 24, 34), 6.0, 3.0, gam, 1.5, 0.5, 0.05)
    T4 = np.pi / (2 * gam) * (6.0 / 3.0 + 3.0 / 6.0)
    assert q is not None and 1.0 <= q / T4 < 1.15, q / T4


def test_jeffery_paper_case():
    """Sec. 3.1 case: a = 6, b = c = 4.5, H = 60, U = 0.01, nu = 1/6
    (tau = 1), 60 x 30 (vorticity) x 60 (+2 wall layers).  The paper reports a
    2.62 % mean relative angle error for its rigid-body variant; the oracle's
    capsule reaches pi/2 within 2 % of T/4 (measured ratio 1.019)."""
    n = (60, 30, 62)
    gam = 2 * 0.01 / 60
    q = _quarter_period(n, 6.0, 4.5, gam, 1.0, 0.5, 0.05, every=100, max_steps=40000)
    T4 = np.pi / (2 * gam) * (6.0 / 4.5 + 4.5 / 6.0)
    print("quarter period ratio", q / T4)
    assert q is not None and abs(q / T4 - 1.0) < 0.05
