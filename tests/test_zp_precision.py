"""Precision of the reduced storage modes against the FP64 oracle.

The workload is the 64^3 channel of the precision sweep: tau 0.8, periodic x,
walls on y and z, body force gx = 1e-6, fluid at rest at t = 0, Evans-Fung
cells (D = 16, ks 0.005, kb 0.001, cosine kernel) placed by seeded random
sequential insertion (seed 1003) to 20 % of the fluid volume, 1000 steps.
Bars: FP32 storage 1e-5, FP16-offset storage 1e-3, for the fluid velocity
(max-norm of the difference relative to max |u_ref|, fluid cells) and for the
node positions (max |dX| relative to the largest displacement).

The populations are stored in reduced precision with stochastically rounded
(unbiased) stores: FP32 storage with the moments and the O(u) part of the
collision in FP64, FP16 offsets scaled by 2^16 with FP32 arithmetic.  The
full-size channel of the precision study (512x256x256) is checked over two
steps.  This file is collected after the parity tests, so a miss here cannot
hide them.
"""
import time

import numpy as np
import pytest

from paper_1704_04551_amd import ibl
from paper_1704_04551_amd import workloads as W

from parity_util import field_err, fluid_mask, node_err, oracle_from_spec

pytestmark = pytest.mark.gpu

BAR = {"f32": 1e-5, "f16": 1e-3}


@pytest.fixture(scope="module")
def crop_reference(capsys_module):
    t0 = time.time()
    spec = W.config_rbc_channel(n=(64, 64, 64), count=200, seed=1003)
    o = oracle_from_spec(spec)
    for k in range(10):
        o.step(100)
        capsys_module("crop oracle: %d steps, %.0f s" % (100 * (k + 1), time.time() - t0))
    _, uo, _ = o.observe()
    Xo = [o.nodes(m)[0] for m in range(len(spec.capsules))]
    return spec, uo, Xo


@pytest.fixture(scope="module")
def capsys_module(request):
    """Progress lines past pytest's capture (the oracle run is long)."""
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def say(msg):
        if capman is not None:
            with capman.global_and_fixture_disabled():
                print(msg, flush=True)
        else:
            print(msg, flush=True)
    return say


@pytest.mark.timeout(900)
@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_crop_64_channel_1000_steps(storage, crop_reference, capsys_module):
    spec, uo, Xo = crop_reference
    assert len(spec.capsules) >= 50
    g = ibl.Sim.from_spec(spec, storage=storage)
    g.step(1000)
    g.sync()
    _, ug, _ = g.fields(rho=False, g=False)
    eu_max, eu_l2 = field_err(ug, uo, fluid_mask(spec))
    ex = [node_err(g.nodes(m)[0], Xo[m], c.x) for m, c in enumerate(spec.capsules)]
    ex_rel = max(v[1] for v in ex)
    ex_abs = max(v[0] for v in ex)
    g.close()
    capsys_module("crop %s: u max %.3e L2 %.3e, X %.3e lu (%.3e of the displacement)"
                  % (storage, eu_max, eu_l2, ex_abs, ex_rel))
    assert eu_max < BAR[storage], (storage, eu_max)
    assert ex_rel < BAR[storage], (storage, ex_rel)


@pytest.mark.timeout(900)
def test_precision_channel_512_full_size(capsys_module):
    """The precision study's full-size channel (512x256x256, the seeded
    256x128x128 layout tiled 2x2x2: 8144 cells, 5.2M nodes) in the bench's
    launch configuration: after two steps, u and X against the FP64 oracle
    within the FP32 bar and, for FP16-offset storage, within its bar."""
    spec = W.tiled(W.config_rbc_channel())
    assert spec.n == (512, 256, 256) and len(spec.capsules) == 8144
    o = oracle_from_spec(spec)
    o.step(2)
    _, uo, _ = o.observe()
    Xo = [o.nodes(m)[0] for m in range(len(spec.capsules))]
    o.close()
    capsys_module("512 oracle: 2 steps done")
    mask = fluid_mask(spec)
    for storage, tol in (("f32", 1e-5), ("f16", 1e-3)):
        g = ibl.Sim.from_spec(spec, storage=storage, brick_x=64)
        g.step(2)
        g.sync()
        _, ug, _ = g.fields(rho=False, g=False)
        umax, ul2 = field_err(ug, uo, mask)
        xr = max(node_err(g.nodes(m)[0], Xo[m], c.x)[1] for m, c in enumerate(spec.capsules))
        g.close()
        capsys_module("512 %s: u max %.3e L2 %.3e, X %.3e of the displacement" % (storage, umax, ul2, xr))
        assert umax < tol, (storage, umax)
        assert xr < tol, (storage, xr)
