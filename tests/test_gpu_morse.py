"""Inter-capsule Morse repulsion on the GPU (Eq. (13), Sec. 2.2) against the
FP64 oracle, and its determinism (alone, in a batch, across a checkpoint).

The library bins capsule nodes into a neighbour grid of 2-lattice-unit cells
and sums each node's pair forces exactly (two-word fixed point); the oracle
visits every pair of nodes of different capsules.  Bars as for the capsules:
FP64 storage about 1e-11 relative, FP32 1e-5."""
import numpy as np
import pytest

from paper_1704_04551_amd import ibl
from paper_1704_04551_amd import workloads as W

from parity_util import field_err, fluid_mask, node_err, oracle_from_spec

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-11, "f32": 1e-5}
MORSE = (2.4e-3, 1.0, 1.2, 1.2)  # D0, alpha, r0, rc (rc = r0: repulsion only)


def _ring_spec(n=(20, 16, 16), morse=MORSE, U=0.004):
    """Three spherical capsules (radius 3) in a ring around the periodic x
    axis, node gaps 0.4, 0.6 and 1.0 lu (the last across the periodic
    boundary), in a gentle shear between walls on z."""
    S, T = W.icosphere(2)
    caps = []
    for xc in (6.6, 13.0, 19.6):
        x = S * 3.0 + np.array([xc, 7.7, 7.6])
        caps.append(W.Capsule(x, x.copy(), T, 0.02, 0.004, "sphere3"))
    ulo = np.zeros((3, 3)); uhi = np.zeros((3, 3))
    ulo[2, 0] = -U; uhi[2, 0] = U
    return W.SimSpec(n=n, tau=0.9, wall=(0, 0, 1), u_lo=ulo, u_hi=uhi, delta="cos", init_profile=1,
                     capsules=caps, name="morse-ring", morse=morse)


def test_morse_forces_at_step0_f64():
    """Node forces at time 0 (membrane at rest, so only Eq. (13) acts): the
    GPU's equal the oracle's pair sums to round-off, and they are not zero."""
    spec = _ring_spec()
    g = ibl.Sim.from_spec(spec, storage="f64")
    o = oracle_from_spec(spec)
    o.observe()
    fmax = 0.0
    for i in range(len(spec.capsules)):
        Fg = g.nodes(i)[2]
        Fo = o.nodes(i)[2]
        fmax = max(fmax, np.abs(Fo).max())
        assert np.abs(Fg - Fo).max() < 1e-13 * np.abs(Fo).max(), i
    assert fmax > 1e-4
    # the total is zero: pair forces are exact opposites (across the boundary too)
    tot = sum(g.nodes(i)[2].sum(0) for i in range(len(spec.capsules)))
    assert np.abs(tot).max() < 1e-15


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_morse_ring_vs_oracle(storage):
    """200 coupled steps: fluid velocity and node positions against the
    oracle, at the storage's bar."""
    spec = _ring_spec()
    g = ibl.Sim.from_spec(spec, storage=storage)
    o = oracle_from_spec(spec)
    g.step(200)
    g.sync()
    o.step(200)
    _, ug, _ = g.fields(rho=False, g=False)
    _, uo, _ = o.observe()
    eu = field_err(ug, uo, fluid_mask(spec))[0]
    assert eu < TOL[storage], ("u", eu)
    for i, c in enumerate(spec.capsules):
        dx, rel = node_err(g.nodes(i)[0], o.nodes(i)[0], c.x)
        assert rel < TOL[storage] or dx < 1e-12, ("X", i, dx, rel)


def test_morse_pushes_capsules_apart():
    """With the repulsion on, the two closest capsules separate faster than
    without it (FP32, 200 steps)."""
    sep = {}
    for on in (False, True):
        spec = _ring_spec(morse=MORSE if on else ())
        g = ibl.Sim.from_spec(spec, storage="f32")
        g.step(200)
        g.sync()
        sep[on] = np.linalg.norm(g.nodes(1)[0].mean(0) - g.nodes(0)[0].mean(0))
        g.close()
    assert sep[True] > sep[False] + 1e-4, sep


@pytest.mark.parametrize("skin", [0, 1])
def test_morse_batch_and_checkpoint_bitwise(skin):
    """A simulation with the repulsion runs bitwise the same alone, in a
    batch beside a simulation without it (uneven step counts), and across a
    checkpoint round trip."""
    spec = _ring_spec()
    ref = ibl.Sim.from_spec(spec, storage="f32")
    ref.step(80)
    ref.sync()
    a = ibl.Sim.from_spec(spec, storage="f32", skin=skin)
    b = ibl.Sim.from_spec(W.config_small(delta="cos", n=24), storage="f32")
    B = ibl.Batch([a, b])
    B.step([50, 70])
    B.close()
    blob = a.read_state()
    c = ibl.Sim.from_spec(spec, storage="f32", skin=skin)
    c.write_state(blob)
    c.step(30)
    c.sync()
    assert np.array_equal(ref.fields()[1], c.fields()[1])
    for i in range(len(spec.capsules)):
        for k in range(3):
            assert np.array_equal(ref.nodes(i)[k], c.nodes(i)[k]), (i, k)


def test_morse_setter_rejects_bad_arguments():
    d = ibl.make_desc((16, 16, 16), 0.9, wall=(0, 0, 1))
    s = ibl.Sim(d)  # created without the grid
    with pytest.raises(ibl.IBLError):
        s.set_morse(*MORSE)
    d = ibl.make_desc((16, 16, 16), 0.9, wall=(0, 0, 1), morse=1)
    s = ibl.Sim(d)
    for bad in ((1e-3, 1.0, 1.2, 2.5), (1e-3, 0.0, 1.2, 1.2), (-1.0, 1.0, 1.2, 1.2), (np.nan, 1.0, 1.2, 1.2)):
        with pytest.raises(ibl.IBLError):
            s.set_morse(*bad)
    s.set_morse(*MORSE)
    s.set_morse(0.0, 1.0, 1.2, 1.2)  # off again


def _pair_spec(level, radii, centres, n, D0, name):
    """Capsules of icosphere(level) templates; walls on z, gentle shear."""
    S, T = W.icosphere(level)
    caps = []
    for k, (R, c) in enumerate(zip(radii, centres)):
        x = S * R + np.asarray(c)
        caps.append(W.Capsule(x, x.copy(), T, 0.02, 0.004, "%s%d" % (name, k)))
    ulo = np.zeros((3, 3)); uhi = np.zeros((3, 3))
    ulo[2, 0] = -0.002; uhi[2, 0] = 0.002
    return W.SimSpec(n=n, tau=0.9, wall=(0, 0, 1), u_lo=ulo, u_hi=uhi, delta="cos", init_profile=1,
                     capsules=caps, name=name, morse=(D0, 1.0, 1.2, 1.2))


def _check_forces_and_steps(spec, steps):
    g = ibl.Sim.from_spec(spec, storage="f64")
    o = oracle_from_spec(spec)
    o.observe()
    for i in range(len(spec.capsules)):
        Fg, Fo = g.nodes(i)[2], o.nodes(i)[2]
        assert np.abs(Fo).max() > 0.0
        assert np.abs(Fg - Fo).max() < 1e-13 * np.abs(Fo).max(), i
    g.close()
    g = ibl.Sim.from_spec(spec, storage="f32")
    g.step(steps)
    g.sync()
    o.step(steps)
    _, ug, _ = g.fields(rho=False, g=False)
    _, uo, _ = o.observe()
    assert field_err(ug, uo, fluid_mask(spec))[0] < TOL["f32"]
    for i, c in enumerate(spec.capsules):
        dx, rel = node_err(g.nodes(i)[0], o.nodes(i)[0], c.x)
        assert rel < TOL["f32"] or dx < 1e-12, ("X", i, dx, rel)
    assert g.conservation()[2] == 0


def test_morse_large_templates():
    """Two 2562-node capsules (icosphere(4), radius 8) 0.4 lu apart: more
    nodes than the staged pair kernel takes, so each node reads its
    neighbouring cells from global memory.  Forces at time 0 (FP64) and 30
    coupled steps (FP32) against the oracle."""
    spec = _pair_spec(4, (8.0, 8.0), ((10.5, 12.0, 12.0), (26.9, 12.0, 12.0)), (40, 24, 24), 2.4e-4,
                      "morse-2562")
    _check_forces_and_steps(spec, 30)


def test_morse_stage_overflow():
    """A 642-node capsule (radius 5) inside another (radius 5.6), both
    centred in a 16^3 box: every cell near the inner membrane holds both
    capsules' nodes, more than the staged kernel keeps in LDS for one
    capsule, so both fall back to global reads.  Same checks, 20 steps."""
    spec = _pair_spec(3, (5.0, 5.6), ((8.0, 8.0, 7.9), (8.0, 8.0, 7.9)), (16, 16, 16), 2.4e-5, "morse-nested")
    _check_forces_and_steps(spec, 20)


def test_morse_full_size_sampled():
    """The RBC channel at full size (256x128x128, 1018 cells, 653,556 nodes)
    with the repulsion at the paper's constants (Sec. 3.5 table in lattice
    units: D0 = 2.4e-5, alpha = 0.25, r0 = rc = 1.32), in the bench's launch
    configuration (FP32, 64-wide bricks).  At time 0 each node's Morse force
    is its force with the repulsion minus its force without (the membrane
    part, at the cells' rest shape, is the same bitwise).  Every node in four
    boxes 16 lu wide is checked against the oracle's pair sums over the nodes
    of the box widened by 2 lu (more than rc), within 1e-12 of the largest
    force."""
    import dataclasses
    from oracle import morse as oracle_morse
    D0, al, r0, rc = 2.4e-5, 0.25, 1.32, 1.32
    base = W.config_rbc_channel()
    assert base.nodes == 653556
    Fs = []
    for mo in ((), (D0, al, r0, rc)):
        spec = dataclasses.replace(base, morse=mo)
        g = ibl.Sim.from_spec(spec, storage="f32", brick_x=64, skin=0)
        nodes = [g.nodes(m) for m in range(len(spec.capsules))]
        assert g.conservation()[2] == 0
        g.close()
        Fs.append(np.concatenate([f for _, _, f in nodes]))
    X = np.concatenate([x for x, _, _ in nodes])
    F = Fs[1] - Fs[0]
    obj = np.concatenate([np.full(len(c.x), m) for m, c in enumerate(spec.capsules)])
    n = np.asarray(spec.n, float)
    rng = np.random.default_rng(5)
    checked = hit = 0
    for centre in X[rng.choice(len(X), 4, replace=False)]:
        d = X - centre
        d[:, 0] -= n[0] * np.round(d[:, 0] / n[0])  # periodic x: the nearest image
        crop = np.all(np.abs(d) <= 10.0, axis=1)
        inner = np.all(np.abs(d[crop]) <= 8.0, axis=1)
        Fo, _ = oracle_morse(spec.n, centre + d[crop], obj[crop], D0, al, r0, rc, wall=spec.wall)
        Fg = F[crop][inner]
        scale = max(np.abs(Fo[inner]).max(), 1e-30)
        assert np.abs(Fg - Fo[inner]).max() <= 1e-12 * scale + 1e-300
        checked += int(inner.sum())
        hit += int(np.any(Fo[inner] != 0.0, axis=1).sum())
    assert checked > 1000 and hit > 0, (checked, hit)
