"""Shared helpers of the parity tests: build the same seeded workload on the
GPU library and on the FP64 oracle, and measure their difference."""
import numpy as np

import oracle
from paper_1704_04551_amd.workloads import template_groups


def oracle_from_spec(spec):
    s = oracle.OracleSim(spec.n, spec.tau, g_body=spec.g_body, wall=spec.wall, u_lo=spec.u_lo,
                         u_hi=spec.u_hi, delta=spec.delta, init_profile=spec.init_profile)
    if spec.morse:
        s.set_morse(*spec.morse)
    mesh_of = {}
    for grp in template_groups(spec):
        c0 = spec.capsules[grp[0]]
        t = s.add_template(c0.tris, c0.x_ref)
        for ci in grp:
            mesh_of[ci] = t
    # the library counts rigid bodies as meshes; the oracle keeps them apart:
    # s.objects[i] = ("mesh", oracle mesh index) or ("body", oracle body index)
    s.objects = []
    for ci, c in enumerate(spec.capsules):
        if c.rigid:
            s.objects.append(("body", s.add_body(mesh_of[ci], c.x, c.density)))
            continue
        m = s.add_mesh(mesh_of[ci], c.x, c.ks, c.kb)
        s.objects.append(("mesh", m))
        if any(c.membrane):
            s.set_membrane(m, *c.membrane)
    return s


def oracle_nodes(o, i):
    """(X, U, F) of object i of a spec in the oracle built by oracle_from_spec."""
    kind, k = o.objects[i]
    return o.body_nodes(k) if kind == "body" else o.nodes(k)


def fluid_mask(spec):
    nx, ny, nz = spec.n
    m = np.ones((nz, ny, nx), bool)
    if spec.wall[0]:
        m[:, :, 0] = m[:, :, -1] = False
    if spec.wall[1]:
        m[:, 0, :] = m[:, -1, :] = False
    if spec.wall[2]:
        m[0] = m[-1] = False
    return m


def field_err(a, b, mask):
    """(max-norm, L2) error of vector field a against reference b over fluid
    cells, each relative to the reference's own norm."""
    d = (a - b)[:, mask]
    r = b[:, mask]
    mx = np.abs(d).max() / max(np.abs(r).max(), 1e-300)
    l2 = np.sqrt((d * d).sum()) / max(np.sqrt((r * r).sum()), 1e-300)
    return float(mx), float(l2)


def node_err(Xa, Xb, X0):
    """max |dX| in lattice units, and relative to the largest displacement."""
    d = np.abs(Xa - Xb).max()
    disp = np.abs(Xb - X0).max()
    return float(d), float(d / max(disp, 1e-300))
