"""Every term of the path in one simulation: deformable capsules with the full
membrane energy, a rigid body, Morse repulsion between the capsules, and
moving walls on two axes, against the FP64 oracle (FP64 storage), and bitwise
the same alone and in a batch beside a plain simulation (FP32 storage)."""
import math

import numpy as np
import pytest

from paper_1704_04551_amd import ibl
from paper_1704_04551_amd import workloads as W

from parity_util import field_err, fluid_mask, node_err, oracle_from_spec, oracle_nodes

pytestmark = pytest.mark.gpu


def _spec():
    n = (34, 26, 28)
    S2, T2 = W.icosphere(2)
    S3, T3 = W.icosphere(3)
    caps = []
    # two capsules 0.5 lu apart (Morse acts), membrane terms on the first
    for xc, terms in ((9.0, (1e-3, 0.01, 0.01, 0.01)), (15.5, (0.0, 0.0, 0.0, 0.0))):
        xr = S2 * 3.0 + np.array([xc, 12.6, 13.4])
        x = xr + 0.03 * np.sin(np.arange(xr.size).reshape(xr.shape))  # off the rest shape
        caps.append(W.Capsule(x, xr, T2, 0.01, 0.002, "sphere3", membrane=terms))
    # a rigid ellipsoid, tilted
    t = 0.3
    R = np.array([[math.cos(t), 0, math.sin(t)], [0, 1, 0], [-math.sin(t), 0, math.cos(t)]])
    xb = W.ellipsoid(S3, 4.5, 3.0, 3.0) @ R.T + np.array([25.0, 12.4, 13.6])
    caps.append(W.Capsule(xb, xb.copy(), T3, 0.0, 0.0, "", rigid=True))
    ulo = np.zeros((3, 3)); uhi = np.zeros((3, 3))
    ulo[2, 0] = -0.008; uhi[2, 0] = 0.008   # shear across z
    ulo[1, 2] = 0.004                       # the y-low wall slides along z
    return W.SimSpec(n=n, tau=0.9, g_body=(2e-6, 0.0, 0.0), wall=(0, 1, 1), u_lo=ulo, u_hi=uhi,
                     delta="cos", init_profile=1, capsules=caps, name="combined",
                     morse=(2.4e-3, 1.0, 1.2, 1.2))


def test_combined_vs_oracle_f64():
    spec = _spec()
    g = ibl.Sim.from_spec(spec, storage="f64")
    o = oracle_from_spec(spec)
    try:
        g.step(120)
        g.sync()
        o.step(120)
        _, ug, _ = g.fields(rho=False, g=False)
        _, uo, _ = o.observe()
        eu = field_err(ug, uo, fluid_mask(spec))[0]
        assert eu < 1e-11, eu
        for i, c in enumerate(spec.capsules):
            dx, rel = node_err(g.nodes(i)[0], oracle_nodes(o, i)[0], c.x)
            assert rel < 1e-11 or dx < 1e-12, (i, dx, rel)
        bo = o.body_state(o.objects[2][1])
        bg = g.body(2)
        assert np.abs(bg["q"] - bo["q"]).max() < 1e-11
        assert np.abs(bo["w"]).max() > 1e-6  # the body turns
    finally:
        g.close()
        o.close()


def test_combined_batch_bitwise():
    spec = _spec()
    ref = ibl.Sim.from_spec(spec, storage="f32")
    ref.step(70)
    ref.sync()
    a = ibl.Sim.from_spec(spec, storage="f32")
    b = ibl.Sim.from_spec(W.SimSpec(n=(16, 12, 20), tau=0.6, g_body=(1e-5, 0, 0), wall=(0, 1, 1)), storage="f32")
    B = ibl.Batch([a, b])
    try:
        B.step([70, 33])
        a.sync()
        assert np.array_equal(ref.fields()[1], a.fields()[1])
        for i in range(len(spec.capsules)):
            assert np.array_equal(ref.nodes(i)[0], a.nodes(i)[0]), i
        for k in ("xc", "q", "v", "w"):
            assert np.array_equal(ref.body(2)[k], a.body(2)[k]), k
    finally:
        B.close()
        for s in (ref, a, b):
            s.close()
