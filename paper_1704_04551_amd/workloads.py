"""Seeded synthetic inputs: membrane meshes, capsule placement, workload specs.

This module holds input generation only -- geometry of the initial meshes and
the parameters of each workload.  It contains none of the method's arithmetic
(no lattice update, no membrane force, no delta kernel); both the GPU library
and the CPU oracle receive the arrays built here as plain inputs.

Meshes are closed triangulated surfaces with outward (counter-clockwise seen
from outside) triangles, node coordinates in lattice units, shape ``(n, 3)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Meshes
# ---------------------------------------------------------------------------


def icosphere(level: int):
    """Unit sphere: an icosahedron refined ``level`` times by edge midpoints.

    Returns ``(verts (10*4**level + 2, 3), tris (20*4**level, 3) int32)``.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    verts = [np.array(p, float) / np.linalg.norm(p) for p in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    X = np.array(verts)
    T = np.array(faces, dtype=np.int32)
    # orient every triangle outward
    for k in range(T.shape[0]):
        a, b, c = X[T[k]]
        if np.dot(np.cross(b - a, c - a), a + b + c) < 0:
            T[k, [1, 2]] = T[k, [2, 1]]
    return X, T


def ellipsoid(unit_sphere_verts, a, b, c):
    """Map unit-sphere nodes to an ellipsoid with semi-axes a (x), b (y), c (z)."""
    return unit_sphere_verts * np.array([a, b, c], float)


# Evans & Fung (1972) biconcave red-cell profile: half-thickness
# z(r) = 0.5 R0 sqrt(1 - p^2) (C0 + C2 p^2 + C4 p^4), p = r / R0.
EVANS_FUNG_C = (0.2072, 2.0026, -1.1228)


def biconcave(unit_sphere_verts, radius):
    """Map unit-sphere nodes onto the Evans-Fung biconcave surface of radius R0.

    Symmetry axis is z.  A sphere point (x, y, z) goes to
    (R0 x, R0 y, z * 0.5 R0 (C0 + C2 p^2 + C4 p^4)), p^2 = x^2 + y^2, which is
    the profile above because |z| = sqrt(1 - p^2) on the unit sphere.
    """
    C0, C2, C4 = EVANS_FUNG_C
    x, y, z = unit_sphere_verts.T
    p2 = x * x + y * y
    out = np.empty_like(unit_sphere_verts)
    out[:, 0] = radius * x
    out[:, 1] = radius * y
    out[:, 2] = z * 0.5 * radius * (C0 + C2 * p2 + C4 * p2 * p2)
    return out


def biconcave_inside(p, radius, margin=0.0):
    """Is the local-frame point p (m,3) inside the biconcave cell grown by margin?"""
    C0, C2, C4 = EVANS_FUNG_C
    R = radius + margin
    r2 = (p[:, 0] ** 2 + p[:, 1] ** 2) / (radius * radius)
    inside = r2 < (R / radius) ** 2
    r2c = np.minimum(r2, 1.0)
    h = 0.5 * radius * np.sqrt(np.maximum(1.0 - r2c, 0.0)) * (C0 + C2 * r2c + C4 * r2c * r2c)
    return inside & (np.abs(p[:, 2]) < h + margin)


def random_rotation(rng):
    """Uniformly random rotation matrix (Shoemake's uniform quaternion)."""
    u1, u2, u3 = rng.random(3)
    q = np.array([math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
                  math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
                  math.sqrt(u1) * math.sin(2 * math.pi * u3),
                  math.sqrt(u1) * math.cos(2 * math.pi * u3)])
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def mesh_volume(X, T):
    """Enclosed volume of a closed outward mesh (divergence theorem)."""
    a, b, c = X[T[:, 0]], X[T[:, 1]], X[T[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


# ---------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------


@dataclass
class Capsule:
    x: np.ndarray          # (n,3) initial node positions
    x_ref: np.ndarray      # (n,3) stress-free reference
    tris: np.ndarray       # (t,3)
    ks: float
    kb: float
    shape_key: str = ""    # capsules with equal keys share one reference state
    membrane: tuple = (0.0, 0.0, 0.0, 0.0)  # kBT/p (WLC-POW), kg, kl (area), kv (volume)
    rigid: bool = False    # a rigid body (the surface at x moves as one body; ks, kb unused)
    density: float = 1.0   # of a rigid body (the fluid's is 1)


@dataclass
class SimSpec:
    n: tuple               # (nx, ny, nz)
    tau: float
    g_body: tuple = (0.0, 0.0, 0.0)
    wall: tuple = (0, 0, 0)
    u_lo: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))
    u_hi: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))
    delta: str = "cos"
    init_profile: int = 0
    capsules: list = field(default_factory=list)
    steps: int = 1
    seed: int = 0
    name: str = ""
    morse: tuple = ()      # (D0, alpha, r0, rc) of the inter-capsule repulsion, or () for none

    @property
    def cells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nodes(self) -> int:
        return int(sum(c.x.shape[0] for c in self.capsules))


def template_groups(spec):
    """Capsule indices grouped by shared reference state (equal non-empty
    ``shape_key``), in first-appearance order.  Every group becomes one
    membrane template, whose rest state is that of its first capsule."""
    groups, key_of = [], {}
    for i, c in enumerate(spec.capsules):
        if c.shape_key and c.shape_key in key_of:
            groups[key_of[c.shape_key]].append(i)
        else:
            if c.shape_key:
                key_of[c.shape_key] = len(groups)
            groups.append([i])
    return groups


def _couette_walls(nz_wall_axis: int, u_top: float, u_bottom: float):
    """Wall velocities for plates on axis 2 moving along x."""
    u_lo = np.zeros((3, 3))
    u_hi = np.zeros((3, 3))
    u_lo[nz_wall_axis, 0] = u_bottom
    u_hi[nz_wall_axis, 0] = u_top
    return u_lo, u_hi


def config_small(delta: str = "peskin4", seed: int = 1001, steps: int = 200, n: int = 32) -> SimSpec:
    """Plain FP64 case: n^3, tau 1, periodic x,y, plates at z=0 and z=n-1
    moving at -/+0.01 along x, one icosphere(3) capsule of radius 5 at the
    centre with N(0, 0.01) jitter, ks 0.005, kb 0.001."""
    rng = np.random.default_rng(seed)
    S, T = icosphere(3)
    c = (n - 1) / 2.0
    x_ref = ellipsoid(S, 5.0, 5.0, 5.0) + c
    x = x_ref + rng.normal(0.0, 0.01, size=x_ref.shape)
    u_lo, u_hi = _couette_walls(2, 0.01, -0.01)
    return SimSpec(n=(n, n, n), tau=1.0, wall=(0, 0, 1), u_lo=u_lo, u_hi=u_hi, delta=delta,
                   init_profile=1, capsules=[Capsule(x, x_ref, T, 0.005, 0.001, "sphere5")],
                   steps=steps, seed=seed, name="capsule-couette-%d" % n)


def _rotations(q):
    """Rotation matrices (m,3,3) from uniform variates q (m,3) (Shoemake)."""
    u1, u2, u3 = q[:, 0], q[:, 1], q[:, 2]
    x = np.sqrt(1 - u1) * np.sin(2 * np.pi * u2)
    y = np.sqrt(1 - u1) * np.cos(2 * np.pi * u2)
    z = np.sqrt(u1) * np.sin(2 * np.pi * u3)
    w = np.sqrt(u1) * np.cos(2 * np.pi * u3)
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
                     np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
                     np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1)],
                    -2)


def _rsa_biconcave(n, wall, count, radius, rng, clearance=0.5, wall_gap=2.5, max_tries=400000,
                   volume_fraction=None):
    """Seeded random sequential addition of non-overlapping biconcave cells
    with uniformly random orientations.  Two cells clash when a node of one
    lies inside the other grown by ``clearance`` (tested both ways, minimum
    image on periodic axes).  Nodes keep ``wall_gap`` from wall layers.
    Stops at ``count`` cells, or earlier once the cells fill
    ``volume_fraction`` of the fluid volume.
    Returns (rotations, centres, (sphere, tris, local_shape))."""
    S, T = icosphere(3)
    local = biconcave(S, radius)
    sub = local[::8]
    n = np.array(n, float)
    if volume_fraction is not None:
        fluid = float(np.prod([n[a] - 2 if wall[a] else n[a] for a in range(3)]))
        count = min(count, int(math.ceil(volume_fraction * fluid / mesh_volume(local, T))))
    per = np.array([0.0 if w else 1.0 for w in wall])
    lo = np.array([wall_gap if w else 0.0 for w in wall])
    hi = np.array([(n[a] - 1 - wall_gap) if wall[a] else n[a] for a in range(3)])
    reach = radius + clearance
    Rs, cs = [], []
    C = np.zeros((0, 3))
    tries = 0
    block = 4096
    while len(cs) < count and tries < max_tries:
        Rb = _rotations(rng.random((block, 3)))
        Ub = rng.random((block, 3))
        for k in range(block):
            if len(cs) >= count or tries >= max_tries:
                break
            tries += 1
            R = Rb[k]
            xn = local @ R.T
            a_lo = lo - xn.min(0)
            a_hi = hi - xn.max(0)
            if np.any(a_hi <= a_lo):
                continue
            c = a_lo + Ub[k] * (a_hi - a_lo)
            if C.shape[0]:
                d = c - C
                d -= per * n * np.round(d / n)
                near = np.nonzero((d * d).sum(1) < (2.0 * reach) ** 2)[0]
                clash = False
                # coarse pass on every 8th node, then the full node sets
                for pts_new, pts_old in ((sub @ R.T, sub), (xn, local)):
                    for j in near:
                        if biconcave_inside((pts_new + d[j]) @ Rs[j], radius, clearance).any() or \
                                biconcave_inside((pts_old @ Rs[j].T - d[j]) @ R, radius, clearance).any():
                            clash = True
                            break
                    if clash:
                        break
                if clash:
                    continue
            Rs.append(R)
            cs.append(c)
            C = np.vstack([C, c[None]])
    return Rs, cs, (S, T, local)


def config_rbc_channel(n=(256, 128, 128), count=1100, diameter=16.0, seed=1002, steps=1000,
                       ks=0.005, kb=0.001, delta="cos", tau=0.8, gx=1e-6,
                       volume_fraction=0.20) -> SimSpec:
    """RBC suspension channel: periodic x, walls on y and z, body force gx,
    biconcave (Evans-Fung) cells of 642 nodes placed by seeded random
    sequential non-overlapping insertion with uniform random orientations."""
    rng = np.random.default_rng(seed)
    wall = (0, 1, 1)
    Rs, cs, (S, T, local) = _rsa_biconcave(n, wall, count, diameter / 2.0, rng,
                                           volume_fraction=volume_fraction)
    caps = []
    for R, c in zip(Rs, cs):
        x = local @ R.T + c
        caps.append(Capsule(x, x.copy(), T, ks, kb, "rbc%g" % diameter))
    return SimSpec(n=tuple(n), tau=tau, g_body=(gx, 0.0, 0.0), wall=wall, delta=delta,
                   init_profile=0, capsules=caps, steps=steps, seed=seed,
                   name="rbc-channel-%dx%dx%d" % tuple(n))


def tiled(spec: SimSpec, reps=(2, 2, 2)) -> SimSpec:
    """The cells of `spec` repeated reps[a] times along each axis (every copy
    keeps its wall clearance, so copies never overlap): the 512x256x256
    channel of the precision study is the seeded 256x128x128 layout tiled
    2x2x2."""
    n = tuple(spec.n[a] * reps[a] for a in range(3))
    caps = []
    for kz in range(reps[2]):
        for ky in range(reps[1]):
            for kx in range(reps[0]):
                sh = np.array([kx * spec.n[0], ky * spec.n[1], kz * spec.n[2]], float)
                for c in spec.capsules:
                    caps.append(Capsule(c.x + sh, c.x_ref + sh, c.tris, c.ks, c.kb, c.shape_key))
    return SimSpec(n=n, tau=spec.tau, g_body=spec.g_body, wall=spec.wall, delta=spec.delta,
                   capsules=caps, steps=spec.steps, seed=spec.seed, name="rbc-channel-%dx%dx%d-tiled" % n)


def config_poiseuille(n=(64, 64, 256), tau=0.8, g=1e-6, axis=2, wall_axis=0, steps=1000) -> SimSpec:
    """Plane Poiseuille channel without cells: flow along `axis` (periodic),
    walls on `wall_axis`, body force g."""
    gb = [0.0, 0.0, 0.0]
    gb[axis] = g
    wall = [0, 0, 0]
    wall[wall_axis] = 1
    return SimSpec(n=tuple(n), tau=tau, g_body=tuple(gb), wall=tuple(wall), delta="cos",
                   steps=steps, name="poiseuille-%dx%dx%d" % tuple(n))


def config_batched(count=64, seed=1004, steps=500, edges=(32, 48, 64, 96)):
    """Uneven batch: per sim, each edge uniform from `edges`; plates on z
    moving at +-U with U uniform in [0.001, 0.01] lattice units per step (the
    configuration's "wall shear rates" carry the unit of a velocity, and read
    as shear rates they would move the 96-cell channels' walls past the
    low-Mach bound of 0.3); tau uniform in
    [0.6, 1.2]; 1-8 sphere/ellipsoid capsules (642 nodes, aspect ratio 1-4,
    equal-volume radius 4) placed with 2 lu clearance."""
    sims = []
    S, T = icosphere(3)
    for i in range(count):
        rng = np.random.default_rng(seed + 7919 * i)
        n = tuple(int(rng.choice(edges)) for _ in range(3))
        U = rng.uniform(0.001, 0.01)
        u_lo, u_hi = _couette_walls(2, U, -U)
        tau = rng.uniform(0.6, 1.2)
        ncap = int(rng.integers(1, 9))
        caps = []
        centres = []
        for _ in range(200):
            if len(caps) >= ncap:
                break
            ar = rng.uniform(1.0, 4.0)
            b = 4.0 * ar ** (-1.0 / 3.0)
            a = ar * b
            R = random_rotation(rng)
            x_ref = ellipsoid(S, a, b, b) @ R.T
            ext = np.abs(x_ref).max(0)
            c = np.empty(3)
            ok = True
            for ax in range(3):
                lo = (3.5 + ext[ax]) if ax == 2 else 0.0
                hi = (n[ax] - 4.5 - ext[ax]) if ax == 2 else float(n[ax])
                if hi <= lo:
                    ok = False
                    break
                c[ax] = rng.uniform(lo, hi)
            if not ok:
                continue
            clash = False
            for (cc, rr) in centres:
                d = c - cc
                for ax in (0, 1):
                    d[ax] -= n[ax] * round(d[ax] / n[ax])
                if np.linalg.norm(d) < a + rr + 2.0:
                    clash = True
                    break
            if clash:
                continue
            centres.append((c, a))
            caps.append(Capsule(x_ref + c, x_ref + c, T, 0.005, 0.001, ""))
        sims.append(SimSpec(n=n, tau=tau, wall=(0, 0, 1), u_lo=u_lo, u_hi=u_hi, delta="cos",
                            init_profile=1, capsules=caps, steps=steps, seed=seed + 7919 * i,
                            name="batch-%d" % i))
    return sims


def job_served(rng, edges=(48, 64, 80, 96, 112, 128), gamma=0.005, steps=(2000, 20000)) -> SimSpec:
    """One served job: a rigid-limit ellipsoid capsule (642 nodes, ks 0.05,
    kb 0.001, aspect ratio uniform in [1.5, 4], equal-volume radius (n-2)/10)
    in plane Couette flow of shear rate gamma on a cubic lattice."""
    S, T = icosphere(3)
    n = int(rng.choice(edges))
    ar = rng.uniform(1.5, 4.0)
    r = (n - 2) / 10.0
    b = r * ar ** (-1.0 / 3.0)
    a = ar * b
    c = (n - 1) / 2.0
    x = ellipsoid(S, a, b, b) + c
    U = gamma * (n - 2) / 2.0
    u_lo, u_hi = _couette_walls(2, U, -U)
    nsteps = int(rng.integers(steps[0], steps[1] + 1))
    return SimSpec(n=(n, n, n), tau=1.0, wall=(0, 0, 1), u_lo=u_lo, u_hi=u_hi, delta="cos",
                   init_profile=1, capsules=[Capsule(x, x.copy(), T, 0.05, 0.001, "")],
                   steps=nsteps, name="job-%d" % n)
