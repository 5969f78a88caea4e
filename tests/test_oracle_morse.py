"""Pins of the oracle's inter-object repulsion, the Morse potential of Eq. (13)
(Sec. 2.2; parameters in the table of Sec. 3.5): U(r) = D0 [exp(-2 alpha (r -
r0)) - 2 exp(-alpha (r - r0))] for r < rc, between nodes of different objects.

Checked against what fixes it independently: a two-node closed form, F = -dU/dr
by central differences of the returned energy, Newton's third law (the forces
sum to zero and carry no torque), the equilibrium distance r0, the cutoff, the
exclusion of pairs within one object, and, in the coupled step, the exact
momentum balance of a periodic box (internal forces add nothing)."""
import math

import numpy as np
import pytest

import oracle
from paper_1704_04551_amd import workloads as W

PRM = dict(D0=2.4e-5, alpha=0.8, r0=1.32, rc=1.9)


def test_two_nodes_closed_form():
    """Two nodes of different objects along x at distance r: the force on the
    first is 2 alpha D0 [e^{-2 alpha (r - r0)} - e^{-alpha (r - r0)}] x-hat
    (repulsive inside r0), the second gets its opposite, the energy is U(r)."""
    D0, al, r0, rc = PRM["D0"], PRM["alpha"], PRM["r0"], PRM["rc"]
    for r in (0.7, 1.0, 1.32, 1.6, 1.89):
        X = np.array([[5.0 + r, 6.0, 6.0], [5.0, 6.0, 6.0]])
        F, E = oracle.morse((12, 12, 12), X, [0, 1], **PRM)
        e = math.exp(-al * (r - r0))
        assert abs(F[0, 0] - 2 * al * D0 * (e * e - e)) < 1e-18
        assert np.abs(F[0, 1:]).max() == 0.0 and np.abs(F[0] + F[1]).max() == 0.0
        assert abs(E - D0 * (e * e - 2 * e)) < 1e-18
    # no force at the equilibrium distance; repulsive inside, attractive outside
    X = np.array([[r0, 6.0, 6.0], [0.0, 6.0, 6.0]])  # distance exactly r0
    assert oracle.morse((12, 12, 12), X, [0, 1], **PRM)[0][0, 0] == 0.0
    assert oracle.morse((12, 12, 12), X - [[0.2, 0, 0], [0, 0, 0]], [0, 1], **PRM)[0][0, 0] > 0.0
    assert oracle.morse((12, 12, 12), X + [[0.2, 0, 0], [0, 0, 0]], [0, 1], **PRM)[0][0, 0] < 0.0


def test_cutoff_and_same_object():
    """Pairs at r >= rc, and pairs within one object, exert nothing; with
    rc = r0 (the paper's table) the force vanishes continuously at the cutoff."""
    X = np.array([[5.0 + PRM["rc"], 6.0, 6.0], [5.0, 6.0, 6.0]])
    F, E = oracle.morse((12, 12, 12), X, [0, 1], **PRM)
    assert np.abs(F).max() == 0.0 and E == 0.0
    X = np.array([[5.5, 6.0, 6.0], [5.0, 6.0, 6.0]])
    F, E = oracle.morse((12, 12, 12), X, [3, 3], **PRM)
    assert np.abs(F).max() == 0.0 and E == 0.0
    p = dict(PRM, rc=PRM["r0"])
    X = np.array([[5.0 + p["r0"] - 1e-9, 6.0, 6.0], [5.0, 6.0, 6.0]])
    assert abs(oracle.morse((12, 12, 12), X, [0, 1], **p)[0][0, 0]) < 1e-8 * p["D0"]  # ~2 alpha^2 D0 (r0 - r)


def _cloud(seed, m=60, nobj=4, box=(10, 9, 8)):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.5, np.array(box) - 0.5, size=(m, 3))
    obj = rng.integers(0, nobj, size=m)
    return X, obj


@pytest.mark.parametrize("wall", [(0, 0, 0), (1, 1, 1)])
def test_force_is_minus_gradient(wall):
    """F = -dU/dX for every node, by central differences of the energy (h =
    1e-6), on a random cloud of nodes of four objects; with periodic axes the
    distances are minimum images."""
    box = (10, 9, 8)
    X, obj = _cloud(4, box=box)
    F, E = oracle.morse(box, X, obj, wall=wall, **PRM)
    assert np.abs(F).max() > 0
    h = 1e-6
    G = np.zeros_like(X)
    for i in range(X.shape[0]):
        for a in range(3):
            Xp = X.copy(); Xp[i, a] += h
            Xm = X.copy(); Xm[i, a] -= h
            G[i, a] = -(oracle.morse(box, Xp, obj, wall=wall, **PRM)[1]
                        - oracle.morse(box, Xm, obj, wall=wall, **PRM)[1]) / (2 * h)
    assert np.abs(F - G).max() < 1e-6 * np.abs(F).max()


def test_third_law():
    """Central pair forces: they sum to zero and their torque vanishes (a box
    with walls, so no pair is taken across a periodic boundary)."""
    X, obj = _cloud(5)
    F, _ = oracle.morse((10, 9, 8), X, obj, wall=(1, 1, 1), **PRM)
    assert np.abs(F.sum(0)).max() < 1e-18
    assert np.abs(np.cross(X, F).sum(0)).max() < 1e-16


def test_coupled_momentum_balance_and_effect():
    """Two spherical capsules closer than rc in a fully periodic box with a body
    force: Morse forces are internal, so the fluid momentum still grows by
    exactly N_cells g_body per step; and they push the capsules apart (their
    centroids separate faster than without them)."""
    S, T = W.icosphere(2)
    n = (20, 16, 16)
    gb = np.array([1e-6, 0.0, 0.0])
    sep = {}
    for on in (False, True):
        x1 = S * 3.0 + np.array([6.6, 8.0, 8.0])
        x2 = S * 3.0 + np.array([13.0, 8.0, 8.0])  # node gap about 0.4 lu
        s = oracle.OracleSim(n, 0.9, g_body=tuple(gb), delta="cos")
        t = s.add_template(T, x1)
        s.add_mesh(t, x1, 0.02, 0.004)
        s.add_mesh(t, x2, 0.02, 0.004)
        if on:
            s.set_morse(2.4e-3, 1.0, 1.2, 1.2)  # rc = r0, as in the paper: repulsion only
        _, p0 = s.conservation()
        s.step(40)
        _, p1 = s.conservation()
        assert np.abs(p1 - p0 - 40 * np.prod(n) * gb).max() < 1e-11 * 40 * np.prod(n) * gb[0]
        sep[on] = np.linalg.norm(s.nodes(1)[0].mean(0) - s.nodes(0)[0].mean(0))
    assert sep[True] > sep[False] + 1e-4, sep
