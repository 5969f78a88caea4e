"""ctypes binding of the FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle is the plain, slow reference that the GPU
library is checked against.  Only the test-suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The product
package never imports it, and this package imports nothing from the product.

Arrays cross the boundary as contiguous float64 / int32 NumPy arrays:
node coordinates are ``(n, 3)``, fields are ``(nz, ny, nx)`` or
``(3, nz, ny, nx)`` (x fastest), matching the oracle's C layout.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DELTA_COS = 0
DELTA_PESKIN4 = 1
_DELTA = {"cos": DELTA_COS, "peskin4": DELTA_PESKIN4, DELTA_COS: DELTA_COS,
          DELTA_PESKIN4: DELTA_PESKIN4}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.oracle_phi.restype = D
        L.oracle_phi.argtypes = [I, D]
        L.oracle_set_threads.restype = I
        L.oracle_set_threads.argtypes = [I]
        L.oracle_membrane.restype = I
        L.oracle_membrane.argtypes = [I, I, P, P, P, D, D, P, P]
        L.oracle_membrane_full.restype = I
        L.oracle_membrane_full.argtypes = [I, I, P, P, P, D, D, D, D, D, D, P, P]
        L.oracle_template_rest.restype = I
        L.oracle_template_rest.argtypes = [I, I, P, P, P, P, P]
        L.oracle_mesh_membrane.restype = I
        L.oracle_mesh_membrane.argtypes = [P, I, D, D, D, D]
        L.oracle_mesh_edges.restype = I
        L.oracle_mesh_edges.argtypes = [I, I, P, P, P, P, P]
        L.oracle_spread_field.restype = I
        L.oracle_spread_field.argtypes = [P, P, I, I, P, P, P]
        L.oracle_interp_field.restype = I
        L.oracle_interp_field.argtypes = [P, P, P, P, I, I, P, P, P]
        L.oracle_sim_create.restype = P
        L.oracle_sim_create.argtypes = [P, D, P, P, P, P, I, I]
        L.oracle_sim_destroy.restype = None
        L.oracle_sim_destroy.argtypes = [P]
        L.oracle_template_add.restype = I
        L.oracle_template_add.argtypes = [P, I, I, P, P]
        L.oracle_mesh_add.restype = I
        L.oracle_mesh_add.argtypes = [P, I, P, D, D]
        L.oracle_sim_step.restype = I
        L.oracle_sim_step.argtypes = [P, ctypes.c_long]
        L.oracle_sim_observe.restype = I
        L.oracle_sim_observe.argtypes = [P, P, P, P]
        L.oracle_sim_nodes.restype = I
        L.oracle_sim_nodes.argtypes = [P, I, P, P, P]
        L.oracle_sim_conservation.restype = None
        L.oracle_sim_conservation.argtypes = [P, P, P]
        L.oracle_sim_populations.restype = None
        L.oracle_sim_populations.argtypes = [P, P]
        L.oracle_velocity_set.restype = None
        L.oracle_velocity_set.argtypes = [P, P]
        L.oracle_sim_stepcount.restype = ctypes.c_long
        L.oracle_sim_stepcount.argtypes = [P]
        L.oracle_sim_nnodes.restype = I
        L.oracle_sim_nnodes.argtypes = [P]
        L.oracle_mass_properties.restype = I
        L.oracle_mass_properties.argtypes = [I, I, P, P, D, P, P, P]
        L.oracle_body_add.restype = I
        L.oracle_body_add.argtypes = [P, I, P, D, P, P]
        L.oracle_body_state.restype = I
        L.oracle_body_state.argtypes = [P, I, P, P, P, P, P, P]
        L.oracle_body_nodes.restype = I
        L.oracle_body_nodes.argtypes = [P, I, P, P, P]
        L.oracle_morse.restype = D
        L.oracle_morse.argtypes = [P, P, I, P, P, P, P]
        L.oracle_sim_morse.restype = None
        L.oracle_sim_morse.argtypes = [P, D, D, D, D]
        _lib = L
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops from now on; returns the count
    they will use."""
    return int(lib().oracle_set_threads(int(n)))


def phi(kind, r: float) -> float:
    """One-dimensional delta kernel phi(r) (Eq. (16) for "cos")."""
    return lib().oracle_phi(_DELTA[kind], float(r))


def membrane(tris, x_ref, x, ks, kb):
    """Membrane force (n,3) and energy at x, rest state from x_ref."""
    tris = _i32(tris)
    x_ref = _f64(x_ref)
    x = _f64(x)
    F = np.zeros_like(x)
    E = np.zeros(1)
    ne = lib().oracle_membrane(x.shape[0], tris.shape[0], _p(tris), _p(x_ref), _p(x), ks, kb,
                               _p(F), _p(E))
    if ne < 0:
        raise ValueError("mesh is not a closed, consistently oriented manifold")
    return F, float(E[0])


def membrane_full(tris, x_ref, x, ks, kb, kbtp=0.0, kg=0.0, kl=0.0, kv=0.0):
    """Force (n,3) and energy of the paper's membrane energy, Eq. (6): linear
    springs (ks) and dihedral bending (kb) as in `membrane`, plus WLC-POW
    stretching (kbtp = kBT/p, Eq. (7)), global / local area (kg, kl, Eq. (9))
    and volume (kv, Eq. (10)) constraints, rest state from x_ref."""
    tris = _i32(tris)
    x_ref = _f64(x_ref)
    x = _f64(x)
    F = np.zeros_like(x)
    E = np.zeros(1)
    r = lib().oracle_membrane_full(x.shape[0], tris.shape[0], _p(tris), _p(x_ref), _p(x), ks, kb,
                                   kbtp, kg, kl, kv, _p(F), _p(E))
    if r == -1:
        raise ValueError("mesh is not a closed, consistently oriented manifold")
    if r == -2:
        raise ValueError("a bond reached its maximum length")
    return F, float(E[0])


def template_rest(tris, x_ref):
    """(per-triangle rest areas (nt,), total rest area A0, rest volume V0)."""
    tris = _i32(tris)
    x_ref = _f64(x_ref)
    a0 = np.zeros(tris.shape[0])
    A0 = np.zeros(1)
    V0 = np.zeros(1)
    if lib().oracle_template_rest(x_ref.shape[0], tris.shape[0], _p(tris), _p(x_ref), _p(a0),
                                  _p(A0), _p(V0)) != 0:
        raise ValueError("mesh is not a closed, consistently oriented manifold")
    return a0, float(A0[0]), float(V0[0])


def mesh_edges(tris, x_ref):
    """(ev (ne,4) [v0,v1,v2,v3], l0 (ne,), theta0 (ne,))."""
    tris = _i32(tris)
    x_ref = _f64(x_ref)
    cap = 3 * tris.shape[0]
    ev = np.zeros((cap, 4), np.int32)
    l0 = np.zeros(cap)
    th0 = np.zeros(cap)
    ne = lib().oracle_mesh_edges(x_ref.shape[0], tris.shape[0], _p(tris), _p(x_ref), _p(ev),
                                 _p(l0), _p(th0))
    if ne < 0:
        raise ValueError("mesh is not a closed, consistently oriented manifold")
    return ev[:ne], l0[:ne], th0[:ne]


def spread_field(n, X, F, kind="peskin4", wall=(0, 0, 0)):
    """Eq. (15) on a box n=(nx,ny,nz); returns g (3,nz,ny,nx)."""
    n_ = _i32(n)
    w = _i32(wall)
    X = _f64(X)
    F = _f64(F)
    g = np.zeros((3, n[2], n[1], n[0]))
    rc = lib().oracle_spread_field(_p(n_), _p(w), _DELTA[kind], X.shape[0], _p(X), _p(F), _p(g))
    if rc != 0:
        raise ValueError("node outside the admissible range")
    return g


def interp_field(n, X, u, kind="peskin4", wall=(0, 0, 0), u_lo=None, u_hi=None):
    """Eq. (14) from a field u (3,nz,ny,nx); returns U (n,3)."""
    n_ = _i32(n)
    w = _i32(wall)
    ulo = _f64(np.zeros((3, 3)) if u_lo is None else u_lo)
    uhi = _f64(np.zeros((3, 3)) if u_hi is None else u_hi)
    X = _f64(X)
    u = _f64(u)
    U = np.zeros_like(X)
    rc = lib().oracle_interp_field(_p(n_), _p(w), _p(ulo), _p(uhi), _DELTA[kind], X.shape[0],
                                   _p(X), _p(u), _p(U))
    if rc != 0:
        raise ValueError("node outside the admissible range")
    return U


def mass_properties(tris, x, density=1.0):
    """(mass, centre of mass (3,), inertia tensor about it (3,3)) of a uniform
    solid bounded by the closed outward surface (tris, x)."""
    tris = _i32(tris)
    x = _f64(x)
    M = np.zeros(1)
    c = np.zeros(3)
    I = np.zeros((3, 3))
    if lib().oracle_mass_properties(x.shape[0], tris.shape[0], _p(tris), _p(x), float(density), _p(M), _p(c),
                                    _p(I)) != 0:
        raise ValueError("not a closed surface enclosing a positive volume")
    return float(M[0]), c, I


def morse(n, X, obj, D0, alpha, r0, rc, wall=(0, 0, 0)):
    """Eq. (13) between nodes of different objects (obj (m,) int): forces (m, 3)
    and the energy, minimum image on periodic axes of the box n."""
    n_ = _i32(n)
    w = _i32(wall)
    X = _f64(X)
    ob = _i32(obj)
    prm = _f64([D0, alpha, r0, rc])
    F = np.zeros_like(X)
    E = lib().oracle_morse(_p(n_), _p(w), X.shape[0], _p(X), _p(ob), _p(prm), _p(F))
    return F, float(E)


def velocity_set():
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    lib().oracle_velocity_set(_p(c), _p(w))
    return c, w


class OracleSim:
    """The coupled IB-LBM simulation, stepped in FP64 on the CPU.

    n = (nx, ny, nz); wall[a] = 1 puts solid layers at index 0 and n[a]-1 of
    axis a; u_lo[a] / u_hi[a] are those layers' velocities (3-vectors).
    """

    def __init__(self, n, tau, g_body=(0.0, 0.0, 0.0), wall=(0, 0, 0), u_lo=None, u_hi=None,
                 delta="peskin4", init_profile=0):
        self.n = tuple(int(v) for v in n)
        self._n = _i32(self.n)
        gb = _f64(g_body)
        w = _i32(wall)
        ulo = _f64(np.zeros((3, 3)) if u_lo is None else u_lo, (3, 3))
        uhi = _f64(np.zeros((3, 3)) if u_hi is None else u_hi, (3, 3))
        self._h = lib().oracle_sim_create(_p(self._n), float(tau), _p(gb), _p(w), _p(ulo), _p(uhi),
                                          _DELTA[delta], int(init_profile))
        if not self._h:
            raise ValueError("invalid simulation parameters")
        self._mesh_nn = []
        self._tmpl_nn = []
        self._body_nn = []

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def add_template(self, tris, x_ref) -> int:
        tris = _i32(tris)
        x_ref = _f64(x_ref)
        t = lib().oracle_template_add(self._h, x_ref.shape[0], tris.shape[0], _p(tris), _p(x_ref))
        if t < 0:
            raise ValueError("mesh is not a closed, consistently oriented manifold")
        self._tmpl_nn.append(x_ref.shape[0])
        return t

    def add_mesh(self, tmpl, x, ks, kb) -> int:
        x = _f64(x)
        if x.shape[0] != self._tmpl_nn[tmpl]:
            raise ValueError("node count does not match the template")
        m = lib().oracle_mesh_add(self._h, int(tmpl), _p(x), float(ks), float(kb))
        self._mesh_nn.append(x.shape[0])
        return m

    def add_body(self, tmpl, x, density=1.0, v0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0)) -> int:
        """A rigid body (Eq. (17)): the template's surface at node positions x
        (its shape and initial pose), uniform density, initial velocity and
        angular velocity."""
        x = _f64(x)
        if x.shape[0] != self._tmpl_nn[tmpl]:
            raise ValueError("node count does not match the template")
        v = _f64(v0)
        w = _f64(w0)
        b = lib().oracle_body_add(self._h, int(tmpl), _p(x), float(density), _p(v), _p(w))
        if b < 0:
            raise ValueError("bad body (template, density or enclosed volume)")
        self._body_nn.append(x.shape[0])
        return b

    def body_state(self, body):
        """dict: centre of mass xc, orientation q (w, x, y, z), velocity v,
        angular velocity w, hydrodynamic force and torque."""
        out = {k: np.zeros(4 if k == "q" else 3) for k in ("xc", "q", "v", "w", "force", "torque")}
        if lib().oracle_body_state(self._h, int(body), *[_p(out[k]) for k in ("xc", "q", "v", "w", "force",
                                                                              "torque")]) != 0:
            raise RuntimeError("body state failed")
        return out

    def body_nodes(self, body):
        """(X, U rigid-body node velocities, F force on the fluid), each (n, 3)."""
        nn = self._body_nn[body]
        X = np.zeros((nn, 3))
        U = np.zeros((nn, 3))
        F = np.zeros((nn, 3))
        if lib().oracle_body_nodes(self._h, int(body), _p(X), _p(U), _p(F)) < 0:
            raise RuntimeError("body node read failed")
        return X, U, F

    def set_morse(self, D0, alpha, r0, rc):
        """Morse repulsion, Eq. (13), between the nodes of different capsules
        (D0 = 0: off)."""
        lib().oracle_sim_morse(self._h, float(D0), float(alpha), float(r0), float(rc))

    def set_membrane(self, mesh, kbtp=0.0, kg=0.0, kl=0.0, kv=0.0):
        """Adds the rest of the paper's membrane energy to a mesh: WLC-POW
        stretching, area and volume constraints (zero: term absent)."""
        if lib().oracle_mesh_membrane(self._h, int(mesh), float(kbtp), float(kg), float(kl), float(kv)) != 0:
            raise ValueError("unknown mesh")

    def step(self, n=1):
        if lib().oracle_sim_step(self._h, int(n)) != 0:
            raise RuntimeError("oracle step failed: node outside the admissible range")

    @property
    def step_count(self) -> int:
        return lib().oracle_sim_stepcount(self._h)

    def observe(self):
        nx, ny, nz = self.n
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        g = np.zeros((3, nz, ny, nx))
        if lib().oracle_sim_observe(self._h, _p(rho), _p(u), _p(g)) != 0:
            raise RuntimeError("node outside the admissible range")
        return rho, u, g

    def nodes(self, mesh):
        nn = self._mesh_nn[mesh]
        X = np.zeros((nn, 3))
        U = np.zeros((nn, 3))
        F = np.zeros((nn, 3))
        if lib().oracle_sim_nodes(self._h, int(mesh), _p(X), _p(U), _p(F)) < 0:
            raise RuntimeError("node read failed")
        return X, U, F

    def conservation(self):
        m = np.zeros(1)
        p = np.zeros(3)
        lib().oracle_sim_conservation(self._h, _p(m), _p(p))
        return float(m[0]), p

    def populations(self):
        nx, ny, nz = self.n
        f = np.zeros((19, nz, ny, nx))
        lib().oracle_sim_populations(self._h, _p(f))
        return f
