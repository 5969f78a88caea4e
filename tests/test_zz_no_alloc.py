"""The allocation-free batch entry point against the allocating one: two calls
in a row on the static device tables, the second with fewer simulations, each
bitwise equal to ibl_batch_step on the same simulations."""
import numpy as np
import pytest

from paper_1704_04551_amd import ibl
from paper_1704_04551_amd import workloads as W

pytestmark = pytest.mark.gpu


def _specs():
    rng = np.random.default_rng(5)
    S, T = W.icosphere(2)
    x = S * 3.0 + np.array([10.3, 9.1, 8.2])
    ragged = W.SimSpec(n=(23, 19, 17), tau=0.7, g_body=(2e-5, 0.0, 1e-5), wall=(0, 1, 0),
                       capsules=[W.Capsule(x + rng.normal(0, 0.05, x.shape), x, T, 0.02, 0.004, "")],
                       delta="cos")
    ragged.u_lo[1, 2] = 0.004
    return [ragged, W.config_small(delta="cos", n=24),
            W.SimSpec(n=(16, 12, 20), tau=0.6, g_body=(1e-5, 0, 0), wall=(0, 1, 1))]


def _state(sim, spec):
    sim.sync()
    return sim.fields()[1], [sim.nodes(m)[0] for m in range(len(spec.capsules))]


def _same(a, b):
    assert np.array_equal(a[0], b[0])
    for xa, xb in zip(a[1], b[1]):
        assert np.array_equal(xa, xb)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_static_batch_equals_batch(storage):
    specs = _specs()
    first, second = [23, 41, 17], [35, 12]   # the second call: the first two simulations
    ref = [ibl.Sim.from_spec(sp, storage=storage) for sp in specs]
    B = ibl.Batch(ref)
    B.step(first)
    B.close()
    B = ibl.Batch(ref[:2])
    B.step(second)
    B.close()
    sims = [ibl.Sim.from_spec(sp, storage=storage) for sp in specs]
    for s in sims:
        s.sync()
    ibl.batch_step_static(sims, first)
    sims[0].sync()
    for s in sims:
        s.sync()
    ibl.batch_step_static(sims[:2], second)
    for s, sp, r, k in zip(sims, specs, ref, [first[0] + second[0], first[1] + second[1], first[2]]):
        _same(_state(s, sp), _state(r, sp))
        assert s.step_count == r.step_count == k


def test_static_batch_rejects_bad_arguments():
    sp = _specs()[2]
    a = ibl.Sim.from_spec(sp, storage="f32")
    b = ibl.Sim.from_spec(sp, storage="f64")
    with pytest.raises(ibl.IBLError):
        ibl.batch_step_static([a, a], [1, 1])
    with pytest.raises(ibl.IBLError):
        ibl.batch_step_static([a, b], [1, 1])
    with pytest.raises(ibl.IBLError):
        ibl.batch_step_static([a], [-1])
