"""Thin ctypes binding of libibl.so (the C-ABI declared in include/ibl.h).

Argument marshalling only: every step of the coupled timestep runs in the HIP
kernels of the library.  PyTorch provides the device arena (a uint8 tensor)
and nothing else.  There is no fallback: if the library is not built, or no
GPU is present, using it raises.

Host arrays: node coordinates (n, 3) float64; fields come back as
(nz, ny, nx) and (3, nz, ny, nx) float64 (x fastest, as on the device).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .workloads import template_groups

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibl.so")

STORAGE = {"f64": 0, "f32": 1, "f16": 2}
DELTA = {"cos": 0, "peskin4": 1}
HEALTH_BITS = {0x1: "nonfinite-f", 0x2: "rho", 0x4: "mach", 0x8: "node-range", 0x10: "overflow",
               0x20: "nonfinite-x", 0x40: "force-range"}


class IBLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ibl status %d: %s" % (status, msg))
        self.status = status


class SimDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("tau", ctypes.c_double),
        ("g_body", ctypes.c_double * 3),
        ("wall", ctypes.c_int32 * 3),
        ("wall_u_lo", (ctypes.c_double * 3) * 3),
        ("wall_u_hi", (ctypes.c_double * 3) * 3),
        ("storage", ctypes.c_int32),
        ("delta", ctypes.c_int32),
        ("init_profile", ctypes.c_int32),
        ("max_nodes", ctypes.c_int32),
        ("max_meshes", ctypes.c_int32),
        ("max_templates", ctypes.c_int32),
        ("max_template_nodes", ctypes.c_int32),
        ("max_template_edges", ctypes.c_int32),
        ("brick_x", ctypes.c_int32),
        ("skin", ctypes.c_int32),
        ("morse", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load libibl.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        if not os.path.exists(LIB_PATH):
            raise ImportError("libibl.so is not built; run `python -m paper_1704_04551_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "ibl_sim_bytes": [ctypes.POINTER(SimDesc), ctypes.POINTER(ctypes.c_size_t)],
            "ibl_sim_create": [ctypes.POINTER(SimDesc), P, ctypes.c_size_t, P, ctypes.POINTER(P)],
            "ibl_sim_destroy": [P],
            "ibl_template_add": [P, I32, I32, P, P, ctypes.POINTER(I32)],
            "ibl_mesh_add": [P, I32, P, D, D, ctypes.POINTER(I32)],
            "ibl_mesh_membrane": [P, I32, D, D, D, D],
            "ibl_body_add": [P, I32, P, D, P, P, ctypes.POINTER(I32)],
            "ibl_read_body": [P, I32, P],
            "ibl_sim_morse": [P, D, D, D, D],
            "ibl_hbm_copy": [P, P, ctypes.c_size_t, P],
            "ibl_step": [P, I64],
            "ibl_sync": [P],
            "ibl_read_fields": [P, P, P, P],
            "ibl_read_nodes": [P, I32, P, P, P],
            "ibl_conservation": [P, P, P, P],
            "ibl_state_bytes": [P, ctypes.POINTER(ctypes.c_size_t)],
            "ibl_read_state": [P, P, ctypes.c_size_t],
            "ibl_write_state": [P, P, ctypes.c_size_t],
            "ibl_step_count": [P, ctypes.POINTER(I64)],
            "ibl_profile_phases": [P, I64, P],
            "ibl_batch_create": [P, I32, ctypes.POINTER(P)],
            "ibl_batch_step": [P, P],
            "ibl_batch_destroy": [P],
            "ibl_batch_step_static": [P, I32, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.ibl_last_error.restype = ctypes.c_char_p
        L.ibl_last_error.argtypes = []
        L.ibl_sim_stream.restype = P
        L.ibl_sim_stream.argtypes = [P]
        _lib = L
    return _lib


def _check(st, allow=()):
    if st != 0 and st not in allow:
        raise IBLError(st, lib().ibl_last_error().decode())
    return st


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_desc(n, tau, g_body=(0, 0, 0), wall=(0, 0, 0), u_lo=None, u_hi=None, storage="f32",
              delta="cos", init_profile=0, max_nodes=0, max_meshes=0, max_templates=0,
              max_template_nodes=0, max_template_edges=0, brick_x=0, skin=0, morse=0) -> SimDesc:
    d = SimDesc()
    for a in range(3):
        d.n[a] = int(n[a])
        d.g_body[a] = float(g_body[a])
        d.wall[a] = int(wall[a])
    ulo = np.zeros((3, 3)) if u_lo is None else np.asarray(u_lo, float).reshape(3, 3)
    uhi = np.zeros((3, 3)) if u_hi is None else np.asarray(u_hi, float).reshape(3, 3)
    for a in range(3):
        for c in range(3):
            d.wall_u_lo[a][c] = float(ulo[a, c])
            d.wall_u_hi[a][c] = float(uhi[a, c])
    d.tau = float(tau)
    d.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    d.delta = DELTA[delta] if isinstance(delta, str) else int(delta)
    d.init_profile = int(init_profile)
    d.max_nodes = int(max_nodes)
    d.max_meshes = int(max_meshes)
    d.max_templates = int(max_templates)
    d.max_template_nodes = int(max_template_nodes)
    d.max_template_edges = int(max_template_edges)
    d.brick_x = int(brick_x)
    d.skin = int(skin)
    d.morse = int(morse)
    return d


def sim_bytes(desc: SimDesc) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().ibl_sim_bytes(ctypes.byref(desc), ctypes.byref(out)))
    return int(out.value)


class Sim:
    """One simulation in a device arena owned by this object (a torch tensor)."""

    def __init__(self, desc: SimDesc, device=None, arena=None):
        import torch
        self.desc = desc
        self.n = tuple(int(v) for v in desc.n)
        self.bytes = sim_bytes(desc)
        if arena is None:
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU: the IB-LBM library runs on the GPU only")
            dev = torch.device("cuda" if device is None else device)
            with torch.cuda.device(dev):
                arena = torch.empty(self.bytes, dtype=torch.uint8, device=dev)
        self.arena = arena
        h = ctypes.c_void_p()
        with torch.cuda.device(arena.device):
            _check(lib().ibl_sim_create(ctypes.byref(desc), ctypes.c_void_p(arena.data_ptr()),
                                        self.bytes, None, ctypes.byref(h)))
        self.h = h
        self._mesh_nn = []
        self._tmpl_nn = []

    # -- construction -------------------------------------------------------
    def add_template(self, tris, x_ref) -> int:
        tris = np.ascontiguousarray(tris, np.int32)
        x_ref = np.ascontiguousarray(x_ref, np.float64)
        out = ctypes.c_int32()
        _check(lib().ibl_template_add(self.h, x_ref.shape[0], tris.shape[0], _p(tris), _p(x_ref),
                                      ctypes.byref(out)))
        self._tmpl_nn.append(x_ref.shape[0])
        return out.value

    def add_mesh(self, template, x, ks, kb) -> int:
        x = np.ascontiguousarray(x, np.float64)
        if x.shape != (self._tmpl_nn[template], 3):
            raise ValueError("node array does not match the template")
        out = ctypes.c_int32()
        _check(lib().ibl_mesh_add(self.h, int(template), _p(x), float(ks), float(kb), ctypes.byref(out)))
        self._mesh_nn.append(x.shape[0])
        return out.value

    def add_body(self, template, x, density=1.0, v0=(0.0, 0.0, 0.0), w0=(0.0, 0.0, 0.0)) -> int:
        """A rigid body: the template's surface at x (shape and initial pose),
        uniform density, initial velocity and angular velocity.  Returns its
        mesh index."""
        x = np.ascontiguousarray(x, np.float64)
        if x.shape != (self._tmpl_nn[template], 3):
            raise ValueError("node array does not match the template")
        v = np.ascontiguousarray(v0, np.float64)
        w = np.ascontiguousarray(w0, np.float64)
        out = ctypes.c_int32()
        _check(lib().ibl_body_add(self.h, int(template), _p(x), float(density), _p(v), _p(w), ctypes.byref(out)))
        self._mesh_nn.append(x.shape[0])
        return out.value

    def body(self, mesh) -> dict:
        """Rigid-body state at the current time: centre of mass xc, orientation
        q (w, x, y, z), velocity v, angular velocity w, force and torque."""
        o = np.zeros(19)
        _check(lib().ibl_read_body(self.h, int(mesh), _p(o)))
        return {"xc": o[0:3], "q": o[3:7], "v": o[7:10], "w": o[10:13], "force": o[13:16], "torque": o[16:19]}

    def set_morse(self, D0, alpha, r0, rc):
        """Morse repulsion between capsules, Eq. (13) (D0 = 0: off); the
        simulation must have been created with morse=1."""
        _check(lib().ibl_sim_morse(self.h, float(D0), float(alpha), float(r0), float(rc)))

    def set_membrane(self, mesh, kbtp=0.0, kg=0.0, kl=0.0, kv=0.0):
        """WLC-POW stretching (kbtp = kBT/p), global / local area (kg, kl) and
        volume (kv) terms of a capsule, in addition to its springs and
        bending (zero: term absent)."""
        _check(lib().ibl_mesh_membrane(self.h, int(mesh), float(kbtp), float(kg), float(kl), float(kv)))

    # -- running ------------------------------------------------------------
    def step(self, n=1):
        _check(lib().ibl_step(self.h, int(n)))

    def sync(self):
        _check(lib().ibl_sync(self.h))

    def sync_status(self) -> int:
        """Like sync(), but returns the status (0, or IBL_ERR_STATE / _UNSTABLE
        from the health word) instead of raising."""
        return int(lib().ibl_sync(self.h))

    @property
    def stream_handle(self) -> int:
        return lib().ibl_sim_stream(self.h)

    @property
    def step_count(self) -> int:
        v = ctypes.c_int64()
        _check(lib().ibl_step_count(self.h, ctypes.byref(v)))
        return v.value

    # -- observation --------------------------------------------------------
    def fields(self, rho=True, u=True, g=True):
        nx, ny, nz = self.n
        R = np.zeros((nz, ny, nx)) if rho else None
        U = np.zeros((3, nz, ny, nx)) if u else None
        G = np.zeros((3, nz, ny, nx)) if g else None
        _check(lib().ibl_read_fields(self.h, None if R is None else _p(R), None if U is None else _p(U),
                                     None if G is None else _p(G)))
        return R, U, G

    def nodes(self, mesh):
        nn = self._mesh_nn[mesh]
        X = np.zeros((nn, 3))
        U = np.zeros((nn, 3))
        F = np.zeros((nn, 3))
        _check(lib().ibl_read_nodes(self.h, int(mesh), _p(X), _p(U), _p(F)))
        return X, U, F

    def conservation(self, raise_on_health=False):
        m = np.zeros(1)
        p = np.zeros(3)
        h = np.zeros(1, np.uint32)
        st = lib().ibl_conservation(self.h, _p(m), _p(p), _p(h))
        if raise_on_health:
            _check(st)
        elif st not in (0, -4, -5):
            _check(st)
        return float(m[0]), p, int(h[0])

    PHASES = ("forces", "lattice", "interp", "advance")

    def profile_phases(self, n):
        """Run n steps phase by phase with HIP events; returns
        ({phase: mean ms per step}, total ms)."""
        ms = np.zeros(len(self.PHASES) + 1)
        _check(lib().ibl_profile_phases(self.h, int(n), _p(ms)))
        return dict(zip(self.PHASES, ms[:-1].tolist())), float(ms[-1])

    def read_state(self) -> bytes:
        nb = ctypes.c_size_t()
        _check(lib().ibl_state_bytes(self.h, ctypes.byref(nb)))
        buf = np.zeros(nb.value, np.uint8)
        _check(lib().ibl_read_state(self.h, _p(buf), nb.value))
        return buf.tobytes()

    def write_state(self, blob: bytes):
        buf = np.frombuffer(blob, np.uint8).copy()
        _check(lib().ibl_write_state(self.h, _p(buf), buf.size))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().ibl_sim_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- from a workload spec ----------------------------------------------
    @classmethod
    def from_spec(cls, spec, storage="f32", device=None, arena=None, brick_x=0, skin=0):
        """Build from a ``workloads.SimSpec``; capsules sharing a non-empty
        shape key share one template (rest state of the first of them)."""
        groups = template_groups(spec)
        nodes = spec.nodes
        tn = sum(spec.capsules[g[0]].x.shape[0] for g in groups)
        te = sum(3 * spec.capsules[g[0]].tris.shape[0] // 2 for g in groups)
        desc = make_desc(spec.n, spec.tau, spec.g_body, spec.wall, spec.u_lo, spec.u_hi, storage,
                         spec.delta, spec.init_profile, max_nodes=nodes,
                         max_meshes=len(spec.capsules), max_templates=len(groups),
                         max_template_nodes=tn, max_template_edges=te, brick_x=brick_x, skin=skin,
                         morse=1 if spec.morse else 0)
        sim = cls(desc, device=device, arena=arena)
        if spec.morse:
            sim.set_morse(*spec.morse)
        mesh_of = {}
        for grp in groups:
            c0 = spec.capsules[grp[0]]
            t = sim.add_template(c0.tris, c0.x_ref)
            for ci in grp:
                mesh_of[ci] = t
        for ci, c in enumerate(spec.capsules):
            if c.rigid:
                sim.add_body(mesh_of[ci], c.x, c.density)
                continue
            m = sim.add_mesh(mesh_of[ci], c.x, c.ks, c.kb)
            if any(c.membrane):
                sim.set_membrane(m, *c.membrane)
        return sim


def hbm_copy(src, dst, stream=None):
    """Plain streaming copy of the device tensor src into dst (same byte
    size, a multiple of 16): the memory-system calibration kernel, launched on
    `stream` (a torch stream; default: torch's current one)."""
    import torch
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("copy: sizes differ")
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(lib().ibl_hbm_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nb,
                              ctypes.c_void_p(st.cuda_stream)))


def batch_step_static(sims, steps):
    """Advance simulation i by steps[i] through the allocation-free batch entry
    point (device tables in the library's static array, plain launches on the
    first simulation's stream)."""
    sims = list(sims)
    st = np.ascontiguousarray(steps, np.int64)
    if st.shape != (len(sims),):
        raise ValueError("one step count per simulation")
    arr = (ctypes.c_void_p * len(sims))(*[s.h.value for s in sims])
    _check(lib().ibl_batch_step_static(arr, len(sims), _p(st)))


class Batch:
    """Several simulations advanced together by one launch per kernel phase."""

    def __init__(self, sims):
        self.sims = list(sims)
        arr = (ctypes.c_void_p * len(self.sims))(*[s.h.value for s in self.sims])
        h = ctypes.c_void_p()
        _check(lib().ibl_batch_create(arr, len(self.sims), ctypes.byref(h)))
        self.h = h

    def step(self, steps):
        st = np.ascontiguousarray(steps, np.int64)
        if st.shape != (len(self.sims),):
            raise ValueError("one step count per simulation")
        _check(lib().ibl_batch_step(self.h, _p(st)))

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().ibl_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
