"""The bench's full-membrane constants (membrane and Morse) are the paper's red blood cell values
(tests/golden/rbc_membrane_constants.json) in the lattice units the bench
states: dx = 0.5 um (16-cell cells 8 um across), nu = 1e-6 m^2/s at
tau = 0.8, rho = 1000 kg/m^3; kBT/p moved to the 642-node mesh at constant
shear modulus (Eq. (11) scales as kBT/p / l0, l0 as 1 / sqrt(triangles))."""
import json
import math
import os

import bench


def test_full_membrane_constants_are_the_papers_in_lattice_units():
    with open(os.path.join(os.path.dirname(__file__), "golden", "rbc_membrane_constants.json")) as fh:
        G = json.load(fh)
    dx, nu, tau, rho = 0.5e-6, 1e-6, 0.8, 1000.0
    dt = (tau - 0.5) / 3 * dx * dx / nu
    f0 = rho * dx ** 4 / dt ** 2                       # force unit, N
    c1320 = G["kbt_p_by_nodes"]["1320"]
    c642 = c1320 * math.sqrt(2 * (1320 - 2) / (2 * (642 - 2)))
    want = (c642 / f0, G["kg"] / (f0 / dx), G["kl"] / (f0 / dx), G["kv"] / (f0 / dx ** 2))
    for got, w in zip(bench.FULL_MEMBRANE, want):
        assert abs(got / w - 1) < 2e-3, (got, w)
    assert abs(bench.FULL_MEMBRANE_KB / (G["kb"] / (f0 * dx)) - 1) < 2e-3


def test_morse_constants_are_the_papers_in_lattice_units():
    """Eq. (13)'s table values in the same units: D0 over the energy unit
    f0 dx, alpha (per um) times dx, r0 and rc over dx."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "rbc_membrane_constants.json")) as fh:
        G = json.load(fh)["morse"]
    dx, nu, tau, rho = 0.5e-6, 1e-6, 0.8, 1000.0
    dt = (tau - 0.5) / 3 * dx * dx / nu
    f0 = rho * dx ** 4 / dt ** 2
    want = (G["D0"] / (f0 * dx), G["alpha"] * dx * 1e6, G["r0_um"] * 1e-6 / dx, G["rc_um"] * 1e-6 / dx)
    for got, w in zip(bench.PAPER_MORSE, want):
        assert abs(got / w - 1) < 1e-9, (got, w)
