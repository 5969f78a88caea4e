"""GPU parity of the rest of the membrane energy, Eq. (6): WLC-POW stretching
(Eq. (7)), global and local area (Eq. (9)) and volume (Eq. (10)) terms, run
through the C-ABI against the FP64 oracle on the same seeded capsule.

The membrane-term kernel sums node forces in 64-bit fixed point at 2^-46
(order-independent, reproducible): each of a node's shares (at most 6
triangles and 6 bonds on these meshes) is rounded by at most 2^-47, so a node
force differs from the FP64 sum by at most 12 * 2^-47 = 8.5e-14 plus FP64
rounding; the bound below is 1e-12 absolute.  The spring and bending part of
the FP32 / FP16 force kernel keeps its own 2^-40 scale (5.5e-12 per node), so
there the bound is 2e-11."""
import dataclasses

import numpy as np
import pytest

from paper_1704_04551_amd import ibl
from paper_1704_04551_amd import workloads as W
from parity_util import field_err, fluid_mask, node_err, oracle_from_spec

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-5, "f16": 1e-3}
F_ABS = {"f64": 1e-12, "f32": 2e-11, "f16": 2e-11}
TERMS = (1e-3, 0.01, 0.01, 0.01)  # kBT/p, kg, kl, kv


def _spec(terms=TERMS, squeeze=0.97, steps=0):
    """The small Couette capsule, squeezed about its centre (the area and
    volume terms then push back) and stretched along x (the bonds pull)."""
    spec = W.config_small(delta="cos", n=32)
    c = spec.capsules[0]
    cen = c.x_ref.mean(0)
    x = cen + (c.x - cen) * squeeze * np.array([1.04, 1.0, 0.98])
    cap = dataclasses.replace(c, x=x, ks=0.0, membrane=tuple(terms))
    return dataclasses.replace(spec, capsules=[cap])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_membrane_terms_force_matches_oracle(storage):
    """Node forces at the initial positions (observation, no step): every
    term on, springs off (the paper's model), against the oracle."""
    spec = _spec()
    g = ibl.Sim.from_spec(spec, storage=storage)
    o = oracle_from_spec(spec)
    try:
        _, _, Fg = g.nodes(0)
        _, _, Fo = o.nodes(0)
        assert np.abs(Fo).max() > 1e-4
        assert np.abs(Fg - Fo).max() < F_ABS[storage], np.abs(Fg - Fo).max()
        # the terms act: without them the force is the bending force alone
        spec0 = _spec(terms=(0.0, 0.0, 0.0, 0.0))
        g0 = ibl.Sim.from_spec(spec0, storage=storage)
        _, _, F0 = g0.nodes(0)
        g0.close()
        assert np.abs(Fg - F0).max() > 1e-5
    finally:
        g.close()
        o.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_membrane_terms_coupled_steps_match_oracle(storage):
    """300 coupled steps with every term on: velocity, density, node
    positions and forces against the oracle, at the storage's parity bar."""
    spec = _spec()
    g = ibl.Sim.from_spec(spec, storage=storage)
    o = oracle_from_spec(spec)
    try:
        g.step(300)
        g.sync()
        o.step(300)
        mask = fluid_mask(spec)
        rg, ug, _ = g.fields()
        ro, uo, _ = o.observe()
        eu = field_err(ug, uo, mask)
        assert eu[0] < TOL[storage], eu
        assert float(np.abs(rg[mask] - ro[mask]).max()) < TOL[storage]
        Xg, _, Fg = g.nodes(0)
        Xo, _, Fo = o.nodes(0)
        dx, rel = node_err(Xg, Xo, spec.capsules[0].x)
        assert rel < TOL[storage] or dx < 1e-12, (dx, rel)
        if storage == "f64":
            assert np.abs(Fg - Fo).max() < F_ABS[storage]
    finally:
        g.close()
        o.close()


def test_zero_terms_are_bitwise_absent():
    """Setting every constant to zero leaves the run bitwise unchanged."""
    spec0 = _spec(terms=(0.0, 0.0, 0.0, 0.0))
    a = ibl.Sim.from_spec(spec0, storage="f32")
    b = ibl.Sim.from_spec(spec0, storage="f32")
    try:
        b.set_membrane(0, 0.0, 0.0, 0.0, 0.0)
        for s in (a, b):
            s.step(50)
            s.sync()
        assert np.array_equal(a.nodes(0)[0], b.nodes(0)[0])
        assert np.array_equal(a.fields(rho=False, g=False)[1], b.fields(rho=False, g=False)[1])
    finally:
        a.close()
        b.close()


def test_membrane_argument_errors():
    spec = _spec(terms=(0.0, 0.0, 0.0, 0.0))
    s = ibl.Sim.from_spec(spec, storage="f32")
    try:
        with pytest.raises(ibl.IBLError):
            s.set_membrane(0, -1.0, 0.0, 0.0, 0.0)
        with pytest.raises(ibl.IBLError):
            s.set_membrane(0, float("nan"), 0.0, 0.0, 0.0)
        with pytest.raises(ibl.IBLError):
            s.set_membrane(5, 0.0, 0.1, 0.0, 0.0)
    finally:
        s.close()


def test_bond_beyond_maximum_length_is_flagged():
    """A capsule inflated to 2.1 times its rest size has every bond past
    l_m = 2 l0: the WLC-POW energy is not finite there, so the step reports
    the force-range health bit and the run is unstable."""
    spec = _spec(terms=(1e-3, 0.0, 0.0, 0.0), squeeze=2.1)
    s = ibl.Sim.from_spec(spec, storage="f32")
    try:
        s.step(1)
        with pytest.raises(ibl.IBLError) as e:
            s.sync()
        assert e.value.status == -5
        assert s.conservation()[2] & 0x40
    finally:
        s.close()


@pytest.mark.parametrize("skin", [0, 1])
def test_batch_with_membrane_terms_equals_alone(skin):
    """A batch whose members differ in membrane model (one with every term,
    one with springs and bending only, one without capsules), advanced by
    uneven step counts in one launch per phase: bitwise each run alone."""
    specs = [_spec(), W.config_small(delta="cos", n=24),
             W.SimSpec(n=(16, 12, 20), tau=0.6, g_body=(1e-5, 0, 0), wall=(0, 1, 1))]
    steps = [37, 19, 11]
    alone = []
    for sp, k in zip(specs, steps):
        s = ibl.Sim.from_spec(sp, storage="f32")
        s.step(k)
        s.sync()
        alone.append(s)
    members = [ibl.Sim.from_spec(sp, storage="f32", skin=skin) for sp in specs]
    B = ibl.Batch(members)
    try:
        B.step(steps)
        for s in members:
            s.sync()
        for a, b, sp in zip(alone, members, specs):
            assert np.array_equal(a.fields()[1], b.fields()[1])
            for m in range(len(sp.capsules)):
                assert np.array_equal(a.nodes(m)[0], b.nodes(m)[0])
    finally:
        B.close()
        for s in alone + members:
            s.close()


def test_checkpoint_roundtrip_with_membrane_terms():
    """The state (populations, positions, step) restored into a new
    simulation with the same capsules and terms continues bitwise like the
    original."""
    spec = _spec()
    a = ibl.Sim.from_spec(spec, storage="f32")
    b = ibl.Sim.from_spec(spec, storage="f32")
    try:
        a.step(40)
        a.sync()
        b.write_state(a.read_state())
        a.step(60)
        b.step(60)
        a.sync()
        b.sync()
        assert np.array_equal(a.nodes(0)[0], b.nodes(0)[0])
        assert np.array_equal(a.fields(rho=False, g=False)[1], b.fields(rho=False, g=False)[1])
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("variant", ["split", "shares"])
def test_membrane_terms_with_alternative_force_kernels(variant, monkeypatch):
    """The split edge / node kernels and the per-edge-share LDS kernel add
    the membrane terms too: forces at the initial positions and 100 coupled
    steps against the oracle (FP32 storage)."""
    monkeypatch.setenv("IBL_FORCES", variant)
    spec = _spec()
    g = ibl.Sim.from_spec(spec, storage="f32")
    o = oracle_from_spec(spec)
    try:
        _, _, Fg = g.nodes(0)
        _, _, Fo = o.nodes(0)
        assert np.abs(Fg - Fo).max() < F_ABS["f32"] + 1e-7 * np.abs(Fo).max()
        g.step(100)
        g.sync()
        o.step(100)
        mask = fluid_mask(spec)
        _, ug, _ = g.fields()
        _, uo, _ = o.observe()
        assert field_err(ug, uo, mask)[0] < TOL["f32"]
        Xg = g.nodes(0)[0]
        Xo = o.nodes(0)[0]
        dx, rel = node_err(Xg, Xo, spec.capsules[0].x)
        assert rel < TOL["f32"] or dx < 1e-12, (dx, rel)
    finally:
        g.close()
        o.close()


def _big_spec(terms=TERMS):
    """The paper's finer membrane resolution (Sec. 3.2): an icosphere(4)
    capsule of 2562 nodes (radius 7), squeezed and stretched as in _spec, in
    plane Couette flow."""
    S, T = W.icosphere(4)
    n = (36, 28, 28)
    cen = (np.array(n) - 1) / 2.0
    xr = S * 7.0 + cen
    x = cen + (xr - cen) * 0.97 * np.array([1.04, 1.0, 0.98])
    ulo = np.zeros((3, 3)); uhi = np.zeros((3, 3))
    ulo[2, 0] = -0.005; uhi[2, 0] = 0.005
    cap = W.Capsule(x, xr, T, 0.0, 2e-3, "ico4", membrane=tuple(terms))
    return W.SimSpec(n=n, tau=0.9, wall=(0, 0, 1), u_lo=ulo, u_hi=uhi, delta="cos", init_profile=1,
                     capsules=[cap], name="membrane-2562")


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_membrane_terms_2562_node_template(storage):
    """Templates above the LDS kernels' 642 nodes (their sums kept in HBM):
    forces at the initial positions, then 100 coupled steps, against the
    oracle."""
    spec = _big_spec()
    assert spec.capsules[0].x.shape[0] == 2562
    g = ibl.Sim.from_spec(spec, storage=storage)
    o = oracle_from_spec(spec)
    try:
        _, _, Fg = g.nodes(0)
        _, _, Fo = o.nodes(0)
        assert np.abs(Fo).max() > 1e-4
        assert np.abs(Fg - Fo).max() < F_ABS[storage], np.abs(Fg - Fo).max()
        g.step(100)
        g.sync()
        o.step(100)
        _, ug, _ = g.fields(rho=False, g=False)
        _, uo, _ = o.observe()
        eu = field_err(ug, uo, fluid_mask(spec))
        assert eu[0] < TOL[storage], eu
        Xg = g.nodes(0)[0]
        Xo = o.nodes(0)[0]
        dx, rel = node_err(Xg, Xo, spec.capsules[0].x)
        assert rel < TOL[storage] or dx < 1e-12, (dx, rel)
    finally:
        g.close()
        o.close()
