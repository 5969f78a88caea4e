"""Pins of the oracle's full membrane energy, Eq. (6): WLC-POW stretching
(Eq. (7)), global and local area constraints (Eq. (9)) and the volume
constraint (Eq. (10)), each against finite differences of the energy, closed
forms on scaled regular solids, and the invariances of the energy."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1704_04551_amd import workloads as W

TERMS = {"wlc": dict(kbtp=0.02), "area_global": dict(kg=0.3), "area_local": dict(kl=0.4),
         "volume": dict(kv=0.5)}


def _tetra(scale=1.0):
    X = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    T = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int32)
    for k in range(4):  # outward (counter-clockwise seen from outside)
        a, b, c = X[T[k]]
        if np.dot(np.cross(b - a, c - a), a + b + c) < 0:
            T[k] = T[k][[0, 2, 1]]
    return X * scale, T


def _cube(side):
    """A cube of the given side, two outward triangles per face."""
    X = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], float) * side
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    T = []
    for a, b, c, d in quads:
        T += [[a, b, c], [a, c, d]]
    T = np.array(T, np.int32)
    cen = X.mean(0)
    for k in range(T.shape[0]):
        p, q, r = X[T[k]]
        assert np.dot(np.cross(q - p, r - p), (p + q + r) / 3 - cen) > 0
    return X, T


def _mesh(shape):
    S, T = W.icosphere(2)
    X = W.biconcave(S, 6.0) if shape == "rbc" else W.ellipsoid(S, 5.0, 3.0, 2.5)
    return X + np.array([10.2, 9.7, 11.1]), T


def test_rest_area_and_volume_closed_forms():
    """Cube of side s: area 6 s^2, volume s^3; regular tetrahedron of edge a:
    area sqrt(3) a^2, volume a^3 / (6 sqrt 2); the volume does not depend on
    where the mesh sits."""
    for s in (1.0, 2.5):
        X, T = _cube(s)
        a0, A0, V0 = oracle.template_rest(T, X + 100.0)
        assert abs(A0 - 6 * s * s) < 1e-12 and abs(V0 - s ** 3) < 1e-10
        assert np.allclose(a0, s * s / 2, atol=1e-12)
    X, T = _tetra(1.7)
    a = 2 * math.sqrt(2) * 1.7
    _, A0, V0 = oracle.template_rest(T, X)
    assert abs(A0 - math.sqrt(3) * a * a) < 1e-12
    assert abs(V0 - a ** 3 / (6 * math.sqrt(2))) < 1e-12


@pytest.mark.parametrize("term", list(TERMS))
@pytest.mark.parametrize("shape", ["rbc", "ellipsoid"])
def test_full_membrane_force_is_minus_gradient(term, shape):
    """F = -dE/dX by central differences, one term of Eqs. (7), (9), (10) at
    a time, on a randomly deformed mesh."""
    X0, T = _mesh(shape)
    rng = np.random.default_rng(11)
    X = X0 + rng.normal(0, 0.12, X0.shape)
    kw = TERMS[term]
    F, E = oracle.membrane_full(T, X0, X, 0.0, 0.0, **kw)
    assert np.abs(F).max() > 1e-4  # the term is active
    h = 1e-6
    for k in rng.choice(X.shape[0], 10, replace=False):
        for a in range(3):
            Xp = X.copy(); Xp[k, a] += h
            Xm = X.copy(); Xm[k, a] -= h
            fd = -(oracle.membrane_full(T, X0, Xp, 0.0, 0.0, **kw)[1] -
                   oracle.membrane_full(T, X0, Xm, 0.0, 0.0, **kw)[1]) / (2 * h)
            assert abs(F[k, a] - fd) < 2e-7 * max(1.0, np.abs(F).max())


def test_full_membrane_adds_to_springs_and_bending():
    """The terms add: the full force is the spring-and-bending force plus
    each extra term's own force."""
    X0, T = _mesh("rbc")
    X = X0 + np.random.default_rng(12).normal(0, 0.1, X0.shape)
    F_all, E_all = oracle.membrane_full(T, X0, X, 0.3, 0.07, kbtp=0.02, kg=0.3, kl=0.4, kv=0.5)
    F_sb, E_sb = oracle.membrane(T, X0, X, 0.3, 0.07)
    parts = [oracle.membrane_full(T, X0, X, 0.0, 0.0, **kw) for kw in TERMS.values()]
    assert np.abs(F_all - F_sb - sum(p[0] for p in parts)).max() < 1e-12
    assert abs(E_all - E_sb - sum(p[1] for p in parts)) < 1e-10


def test_wlc_pow_tetrahedron_closed_form():
    """A regular tetrahedron scaled by s from its rest shape: every bond has
    x = s / 2 and dU/dl = C (1 / (4 (1 - x)^2) - 1/4 + x) - k_p / l^2 with
    k_p = 5/4 C l0^2.  With rest vertices v of coordinates +-1, the three
    unit bond vectors of a vertex sum to -4 s v / l = -sqrt(2) v, so the vertex
    feels -dU/dl * sqrt(2) * v; zero at s = 1."""
    X0, T = _tetra()
    C = 0.03
    l0 = 2 * math.sqrt(2)
    F1, E1 = oracle.membrane_full(T, X0, X0, 0.0, 0.0, kbtp=C)
    assert np.abs(F1).max() < 1e-15
    for s in (0.7, 1.2, 1.6):
        F, E = oracle.membrane_full(T, X0, X0 * s, 0.0, 0.0, kbtp=C)
        x, l = s / 2, s * l0
        kp = 1.25 * C * l0 * l0
        dUdl = C * (1 / (4 * (1 - x) ** 2) - 0.25 + x) - kp / l ** 2
        assert np.abs(F - (-dUdl * math.sqrt(2) * X0)).max() < 1e-14
        lm = 2 * l0
        Eb = C * lm / 4 * (3 * x * x - 2 * x ** 3) / (1 - x) + kp / l
        assert abs(E - 6 * Eb) < 1e-13


def test_wlc_bond_at_maximum_length_is_an_error():
    X0, T = _tetra()
    with pytest.raises(ValueError):
        oracle.membrane_full(T, X0, X0 * 2.0, 0.0, 0.0, kbtp=0.01)


@pytest.mark.parametrize("s", [0.8, 1.15])
def test_area_volume_tetrahedron_closed_form(s):
    """Scaling a regular tetrahedron (centroid at 0) by s: A = s^2 A0 and
    V = s^3 V0.  A is homogeneous of degree 2 and V of degree 3 in the vertex
    positions, and by symmetry every vertex has the same gradient along v, so
    dA/dv = A v / (2 |v|^2) and dV/dv = 3 V v / (4 |v|^2).  Hence
    F_v = -[(kg + kl)(s^2 - 1) A / 2 + kv (s^3 - 1) 3 V / 4] v / |v|^2, and
    E = (kg + kl) A0 (s^2 - 1)^2 / 2 + kv V0 (s^3 - 1)^2 / 2."""
    X0, T = _tetra()
    _, A0, V0 = oracle.template_rest(T, X0)
    kg, kl, kv = 0.3, 0.2, 0.7
    X = X0 * s
    A, V = s * s * A0, s ** 3 * V0
    F, E = oracle.membrane_full(T, X0, X, 0.0, 0.0, kg=kg, kl=kl, kv=kv)
    r2 = (X * X).sum(1, keepdims=True)
    Fx = -((kg + kl) * (s * s - 1) * A / 2 + kv * (s ** 3 - 1) * 3 * V / 4) * X / r2
    assert np.abs(F - Fx).max() < 1e-13
    Ex = (kg + kl) * A0 * (s * s - 1) ** 2 / 2 + kv * V0 * (s ** 3 - 1) ** 2 / 2
    assert abs(E - Ex) < 1e-13


@pytest.mark.parametrize("shape", ["cube", "rbc"])
def test_euler_homogeneity(shape):
    """A is homogeneous of degree 2 and V of degree 3 in the node positions
    about any point, so sum_v (v - c) . dA/dv = 2 A and sum_v (v - c) . dV/dv
    = 3 V.  With one term on, F = -k (Q - Q0) / Q0 dQ/dX, so
    sum_v (v - c) . F_v = -k (Q - Q0) / Q0 * deg Q, whatever the mesh."""
    if shape == "cube":
        X0, T = _cube(2.0)
        X = X0 + np.random.default_rng(14).normal(0, 0.1, X0.shape)
    else:
        X0, T = _mesh("rbc")
        X = X0 + np.random.default_rng(14).normal(0, 0.1, X0.shape)
    _, A0, V0 = oracle.template_rest(T, X0)
    _, A, V = oracle.template_rest(T, X)
    c = X.mean(0) + 0.3
    for kw, Q, Q0, deg in ((dict(kg=0.4), A, A0, 2), (dict(kv=0.6), V, V0, 3)):
        k = next(iter(kw.values()))
        F, _ = oracle.membrane_full(T, X0, X, 0.0, 0.0, **kw)
        lhs = ((X - c) * F).sum()
        rhs = -k * (Q - Q0) / Q0 * deg * Q
        assert abs(lhs - rhs) < 1e-10 * max(1.0, abs(rhs)), (kw, lhs, rhs)


def test_full_membrane_invariants():
    """Sum F = 0 and sum X x F = 0 (the energy is invariant under translation
    and rotation); F = 0 at the rest shape and at any rigid motion of it; the
    force does not change when the whole mesh is moved far away."""
    X0, T = _mesh("rbc")
    kw = dict(kbtp=0.02, kg=0.3, kl=0.4, kv=0.5)
    rng = np.random.default_rng(13)
    X = X0 + rng.normal(0, 0.1, X0.shape)
    F, _ = oracle.membrane_full(T, X0, X, 0.0, 0.0, **kw)
    assert np.abs(F.sum(0)).max() < 1e-12
    assert np.abs(np.cross(X, F).sum(0)).max() < 1e-10
    F0, E0 = oracle.membrane_full(T, X0, X0, 0.0, 0.0, **kw)
    assert np.abs(F0).max() < 1e-13 and abs(E0 - oracle.membrane_full(T, X0, X0, 0.0, 0.0, kbtp=0.02)[1]) < 1e-9
    R = W.random_rotation(rng)
    Xr = (X0 - 3.0) @ R.T + np.array([1.0, -2.0, 0.5])
    Fr, _ = oracle.membrane_full(T, X0, Xr, 0.0, 0.0, **kw)
    assert np.abs(Fr).max() < 1e-12
    Ff, _ = oracle.membrane_full(T, X0, X + 500.0, 0.0, 0.0, **kw)
    assert np.abs(Ff - F).max() < 1e-10


def test_golden_shear_modulus_of_the_wlc_pow_law():
    """Eq. (11) gives the small-strain shear modulus of the WLC-POW network.
    At the force-free bond ratio x0 = 1/2 (with k_p = 5/4 C l0^2) the bonds
    carry no tension, so a triangular network's modulus is sqrt(3)/4 times
    the bond stiffness d2U/dl2; the oracle's stiffness, by central
    differences of its tetrahedron force, must reproduce Eq. (11).  Sec. 3.2
    lists kBT/p for three meshes with mu0 held at 6 uN/m: Eq. (11) scales as
    C / l0 and l0 as 1 / sqrt(n_tri) on a membrane of fixed area, so
    C sqrt(2 (N - 2)) must be the same for the three.  With a membrane area of
    135 um^2 (the usual red blood cell value; the paper does not state it)
    Eq. (11) lands within 10 % of 6 uN/m."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "rbc_membrane_constants.json")) as fh:
        G = json.load(fh)
    X0, T = _tetra()
    C = 1.0
    l0 = 2 * math.sqrt(2)

    def dUdl(s):  # the vertex force is -dU/dl sqrt(2) v, v = (1, 1, 1) for vertex 0
        F, _ = oracle.membrane_full(T, X0, X0 * s, 0.0, 0.0, kbtp=C)
        return -F[0, 0] / math.sqrt(2)

    h = 1e-5
    k_bond = (dUdl(1 + h) - dUdl(1 - h)) / (2 * h * l0)
    x0, lm, kp = 0.5, 2 * l0, 1.25 * C * l0 * l0
    mu_eq11 = (math.sqrt(3) * C / (4 * lm * x0) * (x0 / (2 * (1 - x0) ** 3) - 1 / (4 * (1 - x0) ** 2) + 0.25)
               + 3 * math.sqrt(3) * kp / (4 * l0 ** 3))
    assert abs(math.sqrt(3) / 4 * k_bond - mu_eq11) < 1e-6 * mu_eq11
    assert abs(dUdl(1.0)) < 1e-15  # force-free at rest
    scaled = [c * math.sqrt(2 * (int(n) - 2)) for n, c in G["kbt_p_by_nodes"].items()]
    assert max(scaled) / min(scaled) - 1 < 0.01
    area = 135e-12
    for n, c in G["kbt_p_by_nodes"].items():
        ntri = 2 * (int(n) - 2)
        l0_n = math.sqrt(4 * area / (math.sqrt(3) * ntri))
        mu = mu_eq11 / C * l0 * c / l0_n  # Eq. (11) scales as C / l0
        assert abs(mu / G["mu0"] - 1) < 0.10, (n, mu)
