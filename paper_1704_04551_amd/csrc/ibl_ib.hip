// Immersed-boundary kernels of the coupled step (Sec. 2.2-2.3):
//
//   k_forces_fx   (FP32 / FP16 storage) one workgroup per capsule: every
//                 edge's spring + bending shares on its four vertices (FP64)
//                 are summed per node in LDS as 64-bit fixed-point integers.
//   k_forces_lds  (FP64 storage) one workgroup per capsule: every edge's
//                 shares are kept in LDS and each node gathers its incident
//                 shares in a fixed order.
//   k_edge_forces / k_node_forces  (templates larger than one workgroup
//                 takes) every edge of every capsule in parallel (FP64 shares
//                 to scratch), then every node gathers its incident shares in a
//                 fixed order.
//   k_membrane    (capsules with the rest of the membrane energy of Eq. (6))
//                 one workgroup per capsule, before the force kernel: WLC-POW
//                 stretching, area and volume constraints summed per node in
//                 fixed point; the force kernels add the result.
//   k_morse_bin / k_morse_force  (simulations with the repulsion of Eq. (13))
//                 one workgroup per capsule: the capsule nodes binned into a
//                 neighbour grid, then each node's pair forces from the other
//                 capsules' nodes in its 27 neighbouring cells, staged in LDS;
//                 the force kernels add the result.
//   k_rigid_nodes / k_rigid_body  (rigid bodies, Eq. (17)) the node forces
//                 from the interpolated fluid velocity, then per body the
//                 force and torque and the Newton-Euler update.
//   Each force kernel writes the node's spreading record (stencil base,
//   fractional offset or delta weights, F), adds the step's largest force
//   component to the simulation's maximum, and appends the node to the
//   candidate lists of the lattice bricks its 4x4x4 stencil touches: every
//   step, or with a one-cell skin only when the lists are rebuilt.
//   k_interp      Eq. (14): one workgroup per home cube (16 x 8 x 8 cells),
//                 the cube's velocity and its stencil margin in LDS, one lane
//                 per home node, fixed summation order; X^{n+1} = X^n + U
//                 (FP64).  Clears the cube's node list; with a skin, flags a
//                 rebuild when a node leaves it.
// Force spreading (Eq. (15)) runs per brick inside the collide-stream kernel
// (ibl_kernels.hip), from the candidate lists written here.
#include "ibl_device.h"

namespace ibl {
namespace {

// Store a node's spreading record (see NodeRec).
__device__ __forceinline__ void write_record(const SimDev& S, int gid, const int base[3], int valid,
                                             const double d[3], const double Fv[3]) {
  NodeRec<double> q;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.base[a] = base[a];
    delta_weights(S.delta, d[a], q.w[a]);
    q.F[a] = Fv[a];
  }
  q.valid = valid;
  q.pad = 0.0;
  *(NodeRec<double>*)((GLB NodeRec<double>*)S.rec + gid) = q;
}
__device__ __forceinline__ void write_record(const SimDev& S, int gid, const int base[3], int valid,
                                             const float d[3], const double Fv[3]) {
  NodeRec<float> q;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.base[a] = (int16_t)base[a];
    q.d[a] = d[a];
    q.F[a] = (float)Fv[a];
  }
  q.valid = (int16_t)valid;
  *(NodeRec<float>*)((GLB NodeRec<float>*)S.rec + gid) = q;
}

// Spreading record and validity check of one node (base cell, validity).
// The node arrays F and U are outputs of observation only (mode 1): a step
// (mode 0) passes forces to spreading through the records and velocities to
// the node update in registers.
template <typename R>
__device__ void make_record(const SimDev& S, int gid, const double Xp[3], const double Fv[3], int base[3],
                            int& valid, int mode, int kind = 1) {
  const int64_t ms = (int64_t)S.maxn;
  if (mode == 1) {
    S.F[gid] = Fv[0];
    S.F[ms + gid] = Fv[1];
    S.F[2 * ms + gid] = Fv[2];
  }
  valid = kind;  // 1: a capsule's node, 2: a rigid body's (spread, never interpolated)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (!isfinite(Xp[a])) {
      valid = 0;
      atomicOr((unsigned*)S.health, (uint32_t)kHNonfiniteX);
    } else if (S.wall[a] && !(Xp[a] >= 1.0 && Xp[a] < (double)(S.n[a] - 2))) {
      valid = 0;
      atomicOr((unsigned*)S.health, (uint32_t)kHNodeRange);
    }
  }
  R d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double fb = valid ? floor(Xp[a]) : 0.0;
    // periodic axes: the base cell taken modulo n, so consumers wrap with one compare
    base[a] = S.wall[a] ? (int32_t)fb : wrap((int32_t)(fb - (double)S.n[a] * floor(fb / S.n[a])), S.n[a]);
    d[a] = (R)(valid ? Xp[a] - fb : 0.0);
  }
  write_record(S, gid, base, valid, d, Fv);
  if (!valid && mode == 1) {  // on no candidate list: interpolation never visits it
    S.U[gid] = 0.0;
    S.U[ms + gid] = 0.0;
    S.U[2 * ms + gid] = 0.0;
  }
}

// The bricks along one axis met by cells base-1-w .. base+2+w (the stencil
// widened by a skin of w cells): `cnt` consecutive bricks from `first`, modulo
// the axis's brick count on a periodic axis (the cells wrap; a short axis
// may be covered whole); clipped to the lattice on a wall axis.
__device__ __forceinline__ void skin_bricks(int base, int n, int wall, int shift, int nb, int w, int& first,
                                            int& cnt) {
  const int kW = 4 + 2 * w;
  const int lo = base - 1 - w;
  if (wall) {
    const int c0 = lo < 0 ? 0 : lo, c1 = lo + kW - 1 < n ? lo + kW - 1 : n - 1;
    first = c0 >> shift;
    cnt = (c1 >> shift) - first + 1;
    return;
  }
  const int mask = (1 << shift) - 1;
  int c = ((lo % n) + n) % n;
  first = c >> shift;
  cnt = 1;
  for (int k = 1; k < kW; ++k) {  // a brick starts where the cell index is a multiple
    c = c + 1 == n ? 0 : c + 1;   // of the brick size, or wraps to 0
    cnt += (c & mask) == 0;
  }
  cnt = cnt < nb ? cnt : nb;
}

// Append a node to the candidate list (buffer `buf`) of every brick its
// skin-widened stencil meets.  One device-scope atomic per (node, brick): a
// rebuild happens only when some node has moved a skin's width.
__device__ void append_skin(const SimDev& S, int buf, const int base[3], int gid) {
  int f[3], c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) skin_bricks(base[a], S.n[a], S.wall[a], S.bsh[a], S.nb[a], S.skin, f[a], c[a]);
  const int64_t b0 = (int64_t)buf * S.nbrick;
  for (int jz = 0; jz < c[2]; ++jz) {
    const int bz = f[2] + jz < S.nb[2] ? f[2] + jz : f[2] + jz - S.nb[2];
    for (int jy = 0; jy < c[1]; ++jy) {
      const int by = f[1] + jy < S.nb[1] ? f[1] + jy : f[1] + jy - S.nb[1];
      for (int jx = 0; jx < c[0]; ++jx) {
        const int bx = f[0] + jx < S.nb[0] ? f[0] + jx : f[0] + jx - S.nb[0];
        const int64_t br = b0 + bx + S.nb[0] * (by + (int64_t)S.nb[1] * bz);
        const int pos = atomicAdd((int*)&S.bcount[br], 1);
        if (pos < kCandCap) S.blist[br * kCandCap + pos] = gid;
      }
    }
  }
}

// List state of a simulation's current step, read by the force kernels:
// rebuild flag (always without a skin; an observation always builds its own
// lists, into the free buffer) and the buffer this step's lists are in (the
// first one without a skin, emptied by the spreading once read).
struct ListStep {
  int par, rb, buf;
};
__device__ __forceinline__ ListStep list_step(const SimDev& S, const Items& it, int mode) {
  ListStep L;
  const int4 lc4 = *(const GLB int4*)S.lctl;  // loaded with the step, selected after
  L.par = (int)((*S.step + it.sub) & 1);
  L.rb = mode == 1 || S.skin == 0 ? 1 : (L.par ? lc4.w : lc4.z);
  L.buf = S.skin == 0 ? 0 : (L.par ? lc4.x : lc4.y) ^ L.rb;
  return L;
}

// Skin lists: record of one node; on a rebuild its build-time base cell and
// its list entries.  `fbits` collects the largest force component (float bits).
template <typename R>
__device__ void emit_node(const SimDev& S, const ListStep& L, int gid, const double Xp[3], const double Fv[3],
                          int mode, uint32_t& fbits, int kind = 1) {
  int base[3], valid;
  make_record<R>(S, gid, Xp, Fv, base, valid, mode, kind);
  const float fm = (float)fmax(fabs(Fv[0]), fmax(fabs(Fv[1]), fabs(Fv[2])));
  const uint32_t fb = __float_as_uint(isfinite(fm) ? fm : 0.f);
  fbits = fb > fbits ? fb : fbits;
  if (!L.rb || !valid) return;
  if (mode == 0) {
    GLB int16_t* q = S.bb0 + 4 * (int64_t)gid;
    q[0] = (int16_t)base[0];
    q[1] = (int16_t)base[1];
    q[2] = (int16_t)base[2];
  }
  append_skin(S, L.buf, base, gid);
}


// Without a skin: the bricks a node's stencil touches.  Along an axis the four stencil cells
// are consecutive (modulo n) and bricks are at least four cells long, so they
// meet one or two bricks, a third only on a periodic axis whose last brick is
// one to three cells long.  Combination
// k = ix + 2 iy + 4 iz takes the first (0) or second (1) brick of each axis.
struct NodeBricks {
  int br[8];
  int mask;     // bit k: combination k exists
  int rare;     // an axis meets a third brick: the node is appended directly
  int base[3];  // the stencil base cell (periodic axes wrapped)
};

// brick index along one axis of the four stencil cells from `base`
__device__ __forceinline__ void axis_bricks(int base, int n, int wall, int shift, int b[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int c = base - 1 + k;
    if (!wall) c = c < 0 ? c + n : (c >= n ? c - n : c);
    b[k] = c >> shift;
  }
}


// The bricks of a node's stencil from its base cell (none when the node is
// not valid).
__device__ __forceinline__ void node_bricks(const SimDev& S, const int base[3], int valid, NodeBricks& nb) {
  nb.mask = 0;
  nb.rare = 0;
  nb.base[0] = base[0];
  nb.base[1] = base[1];
  nb.base[2] = base[2];
  if (!valid) return;
  int p0[3], p1[3], h1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int b[4];
    axis_bricks(base[a], S.n[a], S.wall[a], S.bsh[a], b);
    p0[a] = b[0];
    p1[a] = b[1] != b[0] ? b[1] : (b[2] != b[0] ? b[2] : b[3]);
    h1[a] = p1[a] != b[0];
#pragma unroll
    for (int k = 0; k < 4; ++k) nb.rare |= (b[k] != p0[a] && b[k] != p1[a]);
  }
  if (nb.rare) return;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ix = k & 1, iy = (k >> 1) & 1, iz = k >> 2;
    const bool ok = (!ix || h1[0]) && (!iy || h1[1]) && (!iz || h1[2]);
    nb.br[k] = (ix ? p1[0] : p0[0]) + S.nb[0] * ((iy ? p1[1] : p0[1]) + S.nb[1] * (iz ? p1[2] : p0[2]));
    nb.mask |= ok ? (1 << k) : 0;
  }
}

// Candidate-list appends of a workgroup, aggregated per brick in LDS: each
// node takes a rank within its bricks with LDS atomics, then one global add
// per (workgroup, brick) reserves the range.  Device-scope atomics are the
// expensive kind on a multi-XCD GPU; this issues one per brick instead of one
// per (node, brick).  The order of entries in a list is not deterministic;
// the spreading kernels do not depend on it.
constexpr int kBinSlots = 512;
struct BinTable {
  int key[kBinSlots];
  int cnt[kBinSlots];
  int base[kBinSlots];
};

__device__ void bin_clear(BinTable& T) {
  for (int i = threadIdx.x; i < kBinSlots; i += blockDim.x) {
    T.key[i] = -1;
    T.cnt[i] = 0;
  }
}

__device__ int bin_slot(BinTable& T, int key) {
  int h = (int)(((uint32_t)key * 2654435761u) >> 23) & (kBinSlots - 1);
  for (int p = 0; p < 32; ++p) {
    const int cur = atomicCAS(&T.key[h], -1, key);
    if (cur == -1 || cur == key) return h;
    h = (h + 1) & (kBinSlots - 1);
  }
  return -1;  // table crowded: the caller appends directly
}

__device__ __forceinline__ void append_one(const SimDev& S, int buf, int b, int gid) {
  const int64_t br = (int64_t)buf * S.nbrick + b;
  const int pos = atomicAdd((int*)&S.bcount[br], 1);
  if (pos < kCandCap) S.blist[br * kCandCap + pos] = gid;
}

// All threads of the workgroup call this with their node's bricks (mask 0 for
// an inactive thread).  Contains barriers: uniform control flow required.
__device__ void bin_append(const SimDev& S, BinTable& T, int buf, int gid, const NodeBricks& nb) {
  int slot[8], rank[8];
  bin_clear(T);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    slot[k] = -1;
    rank[k] = 0;
    if ((nb.mask >> k) & 1) {
      slot[k] = bin_slot(T, nb.br[k]);
      if (slot[k] >= 0) rank[k] = atomicAdd(&T.cnt[slot[k]], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBinSlots; i += blockDim.x)
    if (T.key[i] >= 0) T.base[i] = atomicAdd((int*)&S.bcount[(int64_t)buf * S.nbrick + T.key[i]], T.cnt[i]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if ((nb.mask >> k) & 1) {
      if (slot[k] < 0) {
        append_one(S, buf, nb.br[k], gid);
      } else {
        const int pos = T.base[slot[k]] + rank[k];
        if (pos < kCandCap) S.blist[((int64_t)buf * S.nbrick + nb.br[k]) * kCandCap + pos] = gid;
      }
    }
  __syncthreads();
}


// A node whose stencil meets a third brick along an axis (short periodic
// axes): appended directly to every distinct brick.
__device__ void append_rare(const SimDev& S, int buf, const NodeBricks& nb, int gid) {
  // every distinct brick: the stencil points first of their brick per axis
  int bx[4], by[4], bz[4];
  axis_bricks(nb.base[0], S.n[0], S.wall[0], S.bsh[0], bx);
  axis_bricks(nb.base[1], S.n[1], S.wall[1], S.bsh[1], by);
  axis_bricks(nb.base[2], S.n[2], S.wall[2], S.bsh[2], bz);
  for (int kz = 0; kz < 4; ++kz) {
    bool fz = true;
    for (int j = 0; j < kz; ++j) fz &= bz[j] != bz[kz];
    for (int ky = 0; ky < 4; ++ky) {
      bool fy = true;
      for (int j = 0; j < ky; ++j) fy &= by[j] != by[ky];
      for (int kx = 0; kx < 4; ++kx) {
        bool fx = true;
        for (int j = 0; j < kx; ++j) fx &= bx[j] != bx[kx];
        if (fx && fy && fz) append_one(S, buf, bx[kx] + S.nb[0] * (by[ky] + S.nb[1] * bz[kz]), gid);
      }
    }
  }
}

// Lists rebuilt every step: record and aggregated appends of one node per
// thread (active = false: no node).  Contains barriers: uniform control flow
// required.
template <typename R>
__device__ void emit_nodes(const SimDev& S, BinTable& T, const ListStep& L, bool active, int gid,
                           const double Xp[3], const double Fv[3], int mode, uint32_t& fbits, int kind = 1) {
  NodeBricks nb;
  nb.mask = 0;
  nb.rare = 0;
  if (active) {
    int base[3], valid;
    make_record<R>(S, gid, Xp, Fv, base, valid, mode, kind);
    const float fm = (float)fmax(fabs(Fv[0]), fmax(fabs(Fv[1]), fabs(Fv[2])));
    const uint32_t fb = __float_as_uint(isfinite(fm) ? fm : 0.f);
    fbits = fb > fbits ? fb : fbits;
    node_bricks(S, base, valid, nb);
    if (nb.rare) append_rare(S, L.buf, nb, gid);
  }
  bin_append(S, T, L.buf, gid, nb);
}

// Workgroup maximum of `fbits` into the step's maximum: one device-scope
// atomic per workgroup, skipped when the recorded value is already larger.
// Contains a barrier: uniform control flow required.
__device__ void flush_fmax(const SimDev& S, int par, uint32_t* wmax, uint32_t fbits) {
  if (fbits) atomicMax(wmax, fbits);
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t v = *wmax;
    *wmax = 0u;
    if (v > __hip_atomic_load(&S.fmax[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax((unsigned*)&S.fmax[par], v);
  }
}

// The first capsule of a simulation clears the next step's rebuild flag,
// which interpolation sets when a node leaves its skin.
__device__ __forceinline__ void clear_next_rebuild(const SimDev& S, const ListStep& L, int m, int mode) {
  if (mode == 0 && m == 0 && threadIdx.x == 0) S.lctl[2 + (L.par ^ 1)] = 0;
}

// ------------------------------------------------------------ forces (LDS) --
// FP64 storage (and, as a tuning alternative, FP32 / FP16 storage): per-edge
// force shares are computed in FP64 and kept in LDS in the precision of the
// spreading record R (double for FP64 storage; float otherwise, where the
// shares carry ~1e-7 relative rounding, far below the FP32 path's own error).
// Vertex positions are read from global memory (one capsule's positions stay
// in L2).  Float shares need 69 KB of LDS, so two 512-thread workgroups share
// a CU; double shares take one 1024-thread workgroup per CU.  Each thread
// gathers up to two nodes.
template <typename R>
constexpr int forces_threads() { return sizeof(R) == 4 ? 512 : 1024; }
static_assert(2 * 512 >= kLdsNodes, "two nodes per thread cover a template of the LDS force kernel");

// Sum of a node's incident shares, in the template's incidence order.  The
// share of a role is a fixed combination of the edge's three stored vectors
// (G0, G3, F1): role 0 -> G0, role 3 -> G3, role 1 -> F1, role 2 (v2) ->
// -(G0 + G3 + F1); it is evaluated branch-free so lanes of different roles
// do not diverge.
template <typename R>
__device__ __forceinline__ void gather_node(const SimDev& S, const R (*pe)[kLdsEdges], int r0, int r1,
                                            int e0, double F[3]) {
  F[0] = F[1] = F[2] = 0.0;
  for (int rb = r0; rb < r1; rb += 8) {
    int ents[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) ents[k] = rb + k < r1 ? S.inc[rb + k] : -1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (ents[k] < 0) continue;
      const int e = (ents[k] >> 2) - e0, role = ents[k] & 3;
      const double c0 = role == 0 ? 1.0 : (role == 2 ? -1.0 : 0.0);
      const double c3 = role == 3 ? 1.0 : (role == 2 ? -1.0 : 0.0);
      const double c1 = role == 1 ? 1.0 : (role == 2 ? -1.0 : 0.0);
#pragma unroll
      for (int a = 0; a < 3; ++a)
        F[a] += c0 * (double)pe[a][e] + c3 * (double)pe[3 + a][e] + c1 * (double)pe[6 + a][e];
    }
  }
}

// Force of a mesh's WLC-POW, area and volume terms (written by k_membrane at
// the same positions), added to a node's spring and bending force.
__device__ __forceinline__ bool mesh_has_terms(const SimDev& S, int m) {
  const GLB double* mm = S.mesh_mem + 4 * (int64_t)m;
  return mm[0] != 0.0 || mm[1] != 0.0 || mm[2] != 0.0 || mm[3] != 0.0;
}

__device__ __forceinline__ void add_membrane_terms(const SimDev& S, const Items& it, int m, bool act, int gid,
                                                   double F[3]) {
  const int64_t ms = (int64_t)S.maxn;
  if (it.membrane && act && mesh_has_terms(S, m)) {
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] += S.Fext[a * ms + gid];
  }
  // the inter-capsule Morse force of the step (k_morse_force), after the
  // membrane's own terms
  if (it.morse && act && S.morse[0] != 0.0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] += S.Fm[a * ms + gid];
  }
}

template <typename R>
__global__ __launch_bounds__(forces_threads<R>()) void k_forces_lds(const SimDev* __restrict__ sims,
                                                                    Items it, int mode) {
  __shared__ R pe[9][kLdsEdges];
  __shared__ BinTable bt;
  __shared__ uint32_t wmax;
  const int tid = threadIdx.x;
  constexpr int NT = forces_threads<R>();
  if (tid == 0) wmax = 0u;
  for (int item = xcd_block(); item < it.mesh_total; item += gridDim.x) {
    const int s = find_sim(it.mesh_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int m = item - it.mesh_off[s];
    const int tm = S.mesh_tmpl[m];
    const int off = S.mesh_off[m];
    const double ks = S.mesh_ks[m], kb = S.mesh_kb[m];
    const int nn = S.t_nn[tm], ne = S.t_ne[tm];
    const int row0 = S.t_node0[tm], e0 = S.t_edge0[tm];
    const int64_t ms = (int64_t)S.maxn;
    const GLB double* X0 = S.X + off;
    const ListStep L = list_step(S, it, mode);
    clear_next_rebuild(S, L, m, mode);
    if (S.mesh_rigid[m]) continue;  // a rigid body (k_rigid_nodes); uniform
    for (int e = tid; e < ne; e += NT) {
      const GLB int* v = S.ev + 4 * (e0 + e);
      D3 p[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int vk = v[k];
        p[k] = {X0[vk], X0[ms + vk], X0[2 * ms + vk]};
      }
      D3 G0, G3, F1;
      edge_forces(p[0], p[1], p[2], p[3], S.el0[e0 + e], S.ec0[e0 + e], S.es0[e0 + e], ks, kb, G0, G3, F1);
      pe[0][e] = (R)G0.x; pe[1][e] = (R)G0.y; pe[2][e] = (R)G0.z;
      pe[3][e] = (R)G3.x; pe[4][e] = (R)G3.y; pe[5][e] = (R)G3.z;
      pe[6][e] = (R)F1.x; pe[7][e] = (R)F1.y; pe[8][e] = (R)F1.z;
    }
    __syncthreads();
    // nodes tid and tid + NT (nn <= kLdsNodes <= 2 NT)
    const int ia = tid, ib = tid + NT;
    const bool acta = ia < nn, actb = ib < nn;
    double Fa[3], Fb[3];
    gather_node<R>(S, pe, acta ? S.inc_ptr[row0 + ia] : 0, acta ? S.inc_ptr[row0 + ia + 1] : 0, e0, Fa);
    gather_node<R>(S, pe, actb ? S.inc_ptr[row0 + ib] : 0, actb ? S.inc_ptr[row0 + ib + 1] : 0, e0, Fb);
    add_membrane_terms(S, it, m, acta, off + ia, Fa);
    add_membrane_terms(S, it, m, actb, off + ib, Fb);
    const double Xa[3] = {acta ? X0[ia] : 0.0, acta ? X0[ms + ia] : 0.0, acta ? X0[2 * ms + ia] : 0.0};
    const double Xb[3] = {actb ? X0[ib] : 0.0, actb ? X0[ms + ib] : 0.0, actb ? X0[2 * ms + ib] : 0.0};
    uint32_t fbits = 0u;
    if (S.skin == 0) {  // uniform
      emit_nodes<R>(S, bt, L, acta, off + ia, Xa, Fa, mode, fbits);
      if (nn > NT) emit_nodes<R>(S, bt, L, actb, off + ib, Xb, Fb, mode, fbits);  // uniform
    } else {
      if (acta) emit_node<R>(S, L, off + ia, Xa, Fa, mode, fbits);
      if (actb) emit_node<R>(S, L, off + ib, Xb, Fb, mode, fbits);
    }
    flush_fmax(S, L.par, &wmax, fbits);  // (its barrier also orders this capsule's
                                         // share reads before the next one's writes)
  }
}

// ------------------------------------------------ forces (fixed point) --
// FP32 / FP16 storage.  Each edge's spring and bending shares (FP64) are added
// to per-node accumulators in LDS as 64-bit fixed-point integers in units of
// 2^-kFxBits.  Integer addition is associative, so a node's sum does not
// depend on the order in which its edges land, and the fourth share of an
// edge is formed in integers as minus the other three, so the membrane's
// internal forces sum to exactly zero.
//
// Resolution 2^-40 (9.1e-13 lattice units, far below the float precision of
// the spreading record).  Single shares are much larger than node sums where
// a triangle is nearly degenerate (the bending share grows as 1 / its area,
// and the shares cancel at the node), so the range is wide: a share component
// is limited to kFxLimit = 2048 lattice units (flagged in the health word
// beyond it); a node meets at most 16 shares on these templates, the fourth of
// an edge at most three times the limit, so a sum stays below 2^17 << 2^23 =
// 2^(63-kFxBits).  With |v 2^40| < 2^51 the rounding to an integer is one FMA:
// v 2^40 + 1.5 2^52 rounds to an integer of the binade [2^52, 2^53), whose bit
// pattern minus that of 1.5 2^52 is round(v 2^40).
// 21.5 KB of LDS per capsule: five 256-thread workgroups share a CU, so the
// capsules of a dense suspension run at once instead of in rounds.
constexpr int kFxThreads = 256;
constexpr int kFxBits = 40;          // resolution 2^-40 (9.1e-13)
constexpr double kFxLimit = 2048.0;  // |share component| limit, lattice units (2^11 = 2^(51-kFxBits))

__device__ __forceinline__ long long fx_quant(const SimDev& S, double v) {
  if (!(fabs(v) < kFxLimit)) {
    atomicOr((unsigned*)S.health, (uint32_t)kHForceRange);
    v = isnan(v) ? 0.0 : copysign(kFxLimit, v);
  }
  return __double_as_longlong(fma(v, 0x1p40, 0x1.8p52)) - __double_as_longlong(0x1.8p52);
}

__device__ __forceinline__ void fx_add(long long* p, long long v) {
  atomicAdd((unsigned long long*)p, (unsigned long long)v);
}

__global__ __launch_bounds__(kFxThreads, 4) void k_forces_fx(const SimDev* __restrict__ sims, Items it, int mode) {
  static_assert(kFxBits == 40, "fx_quant and the readout scale by 2^40");
  __shared__ long long acc[3][kLdsNodes];
  __shared__ double xs[3][kLdsNodes];  // the capsule's positions, read once
  __shared__ BinTable bt;
  __shared__ uint32_t wmax;
  const int tid = threadIdx.x;
  if (tid == 0) wmax = 0u;
  for (int item = xcd_block(); item < it.mesh_total; item += gridDim.x) {
    const int s = find_sim(it.mesh_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int m = item - it.mesh_off[s];
    const int tm = S.mesh_tmpl[m];
    const int off = S.mesh_off[m];
    const double ks = S.mesh_ks[m], kb = S.mesh_kb[m];
    const int nn = S.t_nn[tm], ne = S.t_ne[tm];
    const int e0 = S.t_edge0[tm];
    const int64_t ms = (int64_t)S.maxn;
    const GLB double* X0 = S.X + off;
    const ListStep L = list_step(S, it, mode);
    clear_next_rebuild(S, L, m, mode);
    if (S.mesh_rigid[m]) continue;  // a rigid body (k_rigid_nodes); uniform
    for (int i = tid; i < nn; i += kFxThreads) {
      acc[0][i] = acc[1][i] = acc[2][i] = 0;
      xs[0][i] = X0[i];
      xs[1][i] = X0[ms + i];
      xs[2][i] = X0[2 * ms + i];
    }
    // each edge's four vertices (16 bytes), loaded one edge ahead: the edge
    // loop then waits on LDS only
    const GLB int4* ev4 = (const GLB int4*)(S.ev + 4 * e0);
    int4 nxt;
    nxt.x = nxt.y = nxt.z = nxt.w = 0;
    if (tid < ne) {
      const int4 t = ev4[tid];
      nxt = t;
    }
    __syncthreads();
    for (int e = tid; e < ne; e += kFxThreads) {
      const int4 cur = nxt;
      if (e + kFxThreads < ne) {
        const int4 t = ev4[e + kFxThreads];
        nxt = t;
      }
      const int vk[4] = {cur.x, cur.y, cur.z, cur.w};
      D3 p[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) p[k] = {xs[0][vk[k]], xs[1][vk[k]], xs[2][vk[k]]};
      D3 G0, G3, F1;
      edge_forces(p[0], p[1], p[2], p[3], S.el0[e0 + e], S.ec0[e0 + e], S.es0[e0 + e], ks, kb, G0, G3, F1);
      const double g0[3] = {G0.x, G0.y, G0.z}, g3[3] = {G3.x, G3.y, G3.z}, f1[3] = {F1.x, F1.y, F1.z};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const long long q0 = fx_quant(S, g0[a]), q3 = fx_quant(S, g3[a]), q1 = fx_quant(S, f1[a]);
        fx_add(&acc[a][vk[0]], q0);
        fx_add(&acc[a][vk[1]], q1);
        fx_add(&acc[a][vk[2]], -(q0 + q1 + q3));
        fx_add(&acc[a][vk[3]], q3);
      }
    }
    __syncthreads();
    uint32_t fbits = 0u;
    if (S.skin == 0) {  // uniform
      for (int i0 = 0; i0 < nn; i0 += kFxThreads) {  // uniform: emit_nodes holds barriers
        const int i = i0 + tid;
        const bool act = i < nn;
        double F[3], Xp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          F[a] = act ? (double)acc[a][i] * 0x1p-40 : 0.0;
          Xp[a] = act ? xs[a][i] : 0.0;
        }
        add_membrane_terms(S, it, m, act, off + i, F);
        emit_nodes<float>(S, bt, L, act, off + i, Xp, F, mode, fbits);
      }
    } else {
      for (int i = tid; i < nn; i += kFxThreads) {
        double F[3], Xp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          F[a] = (double)acc[a][i] * 0x1p-40;
          Xp[a] = xs[a][i];
        }
        add_membrane_terms(S, it, m, true, off + i, F);
        emit_node<float>(S, L, off + i, Xp, F, mode, fbits);
      }
    }
    flush_fmax(S, L.par, &wmax, fbits);  // (its barrier: accumulators read before the next
                                         // capsule clears them)
  }
}

// ------------------------------------------- membrane area, volume, WLC-POW --
// The rest of the membrane energy of Eq. (6), per capsule (one workgroup):
//  * WLC-POW stretching, Eq. (7), per edge: x = l / l_m with l_m = 2 l0 (the
//    maximum bond length is twice the rest length), C = kBT / p,
//    dU/dl = C (1 / (4 (1 - x)^2) - 1/4 + x) - k_p / l^2, and k_p = 5/4 C l0^2
//    so that every bond is force-free at its rest length (x = 1/2);
//  * area, Eq. (9): the global term kg (A - A0) / A0 and each triangle's local
//    term kl (A_j - A_j0) / A_j0 multiply dA_j/dp = n x (opposite edge) / 2;
//  * volume, Eq. (10): kv (V - V0) / V0 multiplies dV_j/dp = (q - c) x (r - c)
//    / 6, with V = sum_j (p - c) . ((q - c) x (r - c)) / 6 over the outward
//    triangles about c = the mesh's first node (any fixed point gives the same
//    V on a closed surface; a point on the mesh keeps the terms small).
// A and V are summed per thread in triangle order, then over the workgroup in
// a fixed tree, so they are reproducible.  The node forces are summed in LDS
// as 64-bit fixed-point integers (order-independent; the two shares of a bond
// are exact negatives) and written to Fext, which the force kernels add to the
// spring and bending force.  These shares are bounded by bond lengths and the
// capsule's size (no 1 / area factor as in bending), so the scale is finer
// than k_forces_fx's: units of 2^-46, a share component limited to 32 lattice
// units (health bit beyond), one rounding of at most 2^-47 = 7.1e-15 per
// share, well inside FP64 parity.  A bond at or beyond its maximum length has
// no finite energy: it sets the force-range health bit and contributes nothing.
// Templates beyond the LDS arrays (kBig) read the positions from HBM and sum
// the same fixed-point shares with 64-bit integer atomics in the capsule's
// own Fext range (zeroed first, converted to doubles in place at the end):
// integer sums, so the result is the same as the LDS kernel's.
constexpr int kMemThreads = 256;
constexpr double kMemLimit = 32.0;  // |share component| limit: 2^5 = 2^(51 - 46)

__device__ __forceinline__ long long mem_quant(const SimDev& S, double v) {
  if (!(fabs(v) < kMemLimit)) {
    atomicOr((unsigned*)S.health, (uint32_t)kHForceRange);
    v = isnan(v) ? 0.0 : copysign(kMemLimit, v);
  }
  // |v 2^46| < 2^51: v 2^46 + 1.5 2^52 rounds to an integer of [2^52, 2^53)
  return __double_as_longlong(fma(v, 0x1p46, 0x1.8p52)) - __double_as_longlong(0x1.8p52);
}

template <bool kBig>
__global__ __launch_bounds__(kMemThreads) void k_membrane(const SimDev* __restrict__ sims, Items it, int mode) {
  constexpr int kL = kBig ? 1 : kLdsNodes;
  __shared__ long long acc[3][kL];
  __shared__ double xs[3][kL];  // the capsule's positions, read once
  __shared__ double red[2][kMemThreads];
  const int tid = threadIdx.x;
  for (int item = xcd_block(); item < it.mesh_total; item += gridDim.x) {
    const int s = find_sim(it.mesh_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int m = item - it.mesh_off[s];
    if (!mesh_has_terms(S, m)) continue;  // uniform
    const int tm = S.mesh_tmpl[m];
    const int nn = S.t_nn[tm], ne = S.t_ne[tm], nt = S.t_nt[tm];
    if ((nn > kLdsNodes) != kBig) continue;  // the other variant's capsule
    const GLB double* mm = S.mesh_mem + 4 * (int64_t)m;
    const double kbtp = mm[0], kg = mm[1], kl = mm[2], kv = mm[3];
    const int off = S.mesh_off[m];
    const int e0 = S.t_edge0[tm], tr0 = S.t_tri0[tm];
    const int64_t ms = (int64_t)S.maxn;
    const GLB double* X0 = S.X + off;
    GLB unsigned long long* gacc = (GLB unsigned long long*)(S.Fext + off);  // kBig: [3][ms] from node off
    auto pos = [&](int a, int i) -> double { return kBig ? X0[a * ms + i] : xs[a][i]; };
    auto add = [&](int a, int i, long long v) {
      if constexpr (kBig)
        atomicAdd(gacc + a * ms + i, (unsigned long long)v);
      else
        fx_add(&acc[a][i], v);
    };
    for (int i = tid; i < nn; i += kMemThreads) {
      if constexpr (kBig) {
        gacc[i] = gacc[ms + i] = gacc[2 * ms + i] = 0ull;
      } else {
        acc[0][i] = acc[1][i] = acc[2][i] = 0;
        xs[0][i] = X0[i];
        xs[1][i] = X0[ms + i];
        xs[2][i] = X0[2 * ms + i];
      }
    }
    __syncthreads();  // (kBig: the zeroed sums are in L2 before any atomic)
    const bool surf = kg != 0.0 || kl != 0.0 || kv != 0.0;
    const D3 c = {pos(0, 0), pos(1, 0), pos(2, 0)};
    double cg = 0.0, cv = 0.0;
    if (surf) {  // uniform
      double As = 0.0, Vs = 0.0;
      for (int t = tid; t < nt; t += kMemThreads) {
        const GLB int* q = S.ttri + 3 * (int64_t)(tr0 + t);
        D3 p[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) p[k] = {pos(0, q[k]) - c.x, pos(1, q[k]) - c.y, pos(2, q[k]) - c.z};
        const D3 n = cross(sub(p[1], p[0]), sub(p[2], p[0]));
        As += 0.5 * sqrt(dot(n, n));
        Vs += dot(p[0], cross(p[1], p[2]));  // 6 V_j
      }
      red[0][tid] = As;
      red[1][tid] = Vs;
      __syncthreads();
      for (int w = kMemThreads / 2; w > 0; w >>= 1) {
        if (tid < w) {
          red[0][tid] += red[0][tid + w];
          red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
      }
      const double A0 = S.tav0[2 * tm], V0 = S.tav0[2 * tm + 1];
      cg = kg * (red[0][0] - A0) / A0;
      cv = kv * (red[1][0] / 6.0 - V0) / V0;
    }
    const double ca0 = 0.5 * cg, cv6 = cv / 6.0;  // per 2 dA_j/dp and per 6 dV_j/dp
    __syncthreads();  // sums read
    if (surf) {  // uniform
      for (int t = tid; t < nt; t += kMemThreads) {
        const GLB int* q = S.ttri + 3 * (int64_t)(tr0 + t);
        int v[3];
        D3 p[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          v[k] = q[k];
          p[k] = {pos(0, v[k]) - c.x, pos(1, v[k]) - c.y, pos(2, v[k]) - c.z};
        }
        const D3 n = cross(sub(p[1], p[0]), sub(p[2], p[0]));
        const double nl = sqrt(dot(n, n));
        const double a0 = S.ta0[tr0 + t];
        const double rn = 1.0 / nl;
        // (cg + kl (A_j - A_j0) / A_j0) / 2, with the normal's 1 / |n| folded in
        const double ca = (ca0 + 0.5 * kl * (0.5 * nl - a0) / a0) * rn;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const D3 pn = p[(k + 1) % 3], pp = p[(k + 2) % 3];
          const D3 gA = cross(n, sub(pp, pn));  // 2 |n| dA_j/dp
          const D3 gV = cross(pn, pp);          // 6 dV_j/dp
          const double f[3] = {-(ca * gA.x + cv6 * gV.x), -(ca * gA.y + cv6 * gV.y), -(ca * gA.z + cv6 * gV.z)};
#pragma unroll
          for (int a = 0; a < 3; ++a) add(a, v[k], mem_quant(S, f[a]));
        }
      }
    }
    if (kbtp != 0.0) {  // uniform
      for (int e = tid; e < ne; e += kMemThreads) {
        const GLB int* ev = S.ev + 4 * (e0 + e);
        const int v1 = ev[1], v2 = ev[2];
        const D3 d = {pos(0, v2) - pos(0, v1), pos(1, v2) - pos(1, v1), pos(2, v2) - pos(2, v1)};
        const double l = sqrt(dot(d, d)), l0 = S.el0[e0 + e];
        const double rl = 1.0 / l;
        const double x = 0.5 * l / l0;
        if (!(x < 1.0)) {
          atomicOr((unsigned*)S.health, (uint32_t)kHForceRange);
          continue;
        }
        // dU/dl = C (1 / (4 (1 - x)^2) - 1/4 + x) - k_p / l^2 with k_p = 5/4 C l0^2
        const double r1x = 1.0 / (1.0 - x), l0l = l0 * rl;
        const double dUdl = kbtp * (0.25 * r1x * r1x - 0.25 + x - 1.25 * l0l * l0l);
        const double fl = dUdl * rl;
        const double f[3] = {fl * d.x, fl * d.y, fl * d.z};  // force on v1
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const long long qf = mem_quant(S, f[a]);
          add(a, v1, qf);
          add(a, v2, -qf);
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < nn; i += kMemThreads) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        long long q;
        if constexpr (kBig)  // the atomics' results, from L2
          q = (long long)__hip_atomic_load(gacc + a * ms + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
          q = acc[a][i];
        S.Fext[a * ms + off + i] = (double)q * 0x1p-46;
      }
    }
    __syncthreads();  // accumulators read before the next capsule clears them
  }
}

// ------------------------------------------------ forces (edge / node split) --
// k_edge_forces: every edge of every capsule at once -- its spring and bending
// shares on its four vertices (FP64) go to a scratch slot, 3 * (first node of
// the capsule) + edge (a closed surface of genus <= 1 has at most 3 edges per
// node).  k_node_forces: every node gathers the shares of its incident edges
// in the template's fixed incidence order, then writes its record.
constexpr int kEdgeChunks = 8;   // workgroups per capsule in the edge kernel
constexpr int kNodeChunks = 4;   // workgroups per capsule in the node kernel

__global__ __launch_bounds__(256) void k_edge_forces(const SimDev* __restrict__ sims, Items it, int mode) {
  const int tid = threadIdx.x;
  for (int item = xcd_block(); item < it.mesh_total * kEdgeChunks; item += gridDim.x) {
    const int mi = item / kEdgeChunks, c = item % kEdgeChunks;
    const int s = find_sim(it.mesh_off, it.nsim, mi);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;
    const int m = mi - it.mesh_off[s];
    if (S.mesh_rigid[m]) continue;  // uniform
    const int tm = S.mesh_tmpl[m];
    const int off = S.mesh_off[m];
    const double ks = S.mesh_ks[m], kb = S.mesh_kb[m];
    const int ne = S.t_ne[tm], e0 = S.t_edge0[tm];
    const int64_t ms = (int64_t)S.maxn;
    GLB double* scr = S.escr + 9 * (3 * (int64_t)off);
    for (int e = c * 256 + tid; e < ne; e += 256 * kEdgeChunks) {
      const GLB int* v = S.ev + 4 * (e0 + e);
      D3 p[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int g = off + v[k];
        p[k] = {S.X[g], S.X[ms + g], S.X[2 * ms + g]};
      }
      D3 G0, G3, F1;
      edge_forces(p[0], p[1], p[2], p[3], S.el0[e0 + e], S.ec0[e0 + e], S.es0[e0 + e], ks, kb, G0, G3, F1);
      GLB double* o = scr + 9 * (int64_t)e;
      o[0] = G0.x; o[1] = G0.y; o[2] = G0.z;
      o[3] = G3.x; o[4] = G3.y; o[5] = G3.z;
      o[6] = F1.x; o[7] = F1.y; o[8] = F1.z;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_node_forces(const SimDev* __restrict__ sims, Items it, int mode) {
  __shared__ BinTable bt;
  __shared__ uint32_t wmax;
  const int tid = threadIdx.x;
  if (tid == 0) wmax = 0u;
  for (int item = xcd_block(); item < it.mesh_total * kNodeChunks; item += gridDim.x) {
    const int mi = item / kNodeChunks, c = item % kNodeChunks;
    const int s = find_sim(it.mesh_off, it.nsim, mi);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int m = mi - it.mesh_off[s];
    const int tm = S.mesh_tmpl[m];
    const int off = S.mesh_off[m];
    const int nn = S.t_nn[tm], row0 = S.t_node0[tm], e0 = S.t_edge0[tm];
    const int64_t ms = (int64_t)S.maxn;
    const GLB double* scr = S.escr + 9 * (3 * (int64_t)off);
    const ListStep L = list_step(S, it, mode);
    clear_next_rebuild(S, L, c == 0 ? m : 1, mode);
    if (S.mesh_rigid[m]) continue;  // a rigid body (k_rigid_nodes); uniform
    uint32_t fbits = 0u;
    for (int i0 = c * 256; i0 < nn; i0 += 256 * kNodeChunks) {
      const int i = i0 + tid;
      const bool act = i < nn;
      double F[3] = {0.0, 0.0, 0.0};
      const int r0 = act ? S.inc_ptr[row0 + i] : 0, r1 = act ? S.inc_ptr[row0 + i + 1] : 0;
      for (int rb = r0; rb < r1; rb += 16) {
        int ents[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) ents[k] = rb + k < r1 ? S.inc[rb + k] : -1;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (ents[k] < 0) continue;
          const int role = ents[k] & 3;
          const GLB double* o = scr + 9 * (int64_t)((ents[k] >> 2) - e0);
          for (int a = 0; a < 3; ++a) {
            double v;
            if (role == 0) v = o[a];
            else if (role == 3) v = o[3 + a];
            else if (role == 1) v = o[6 + a];
            else v = -(o[a] + o[3 + a] + o[6 + a]);
            F[a] += v;
          }
        }
      }
      const int gid = off + i;
      add_membrane_terms(S, it, m, act, gid, F);
      const double Xp[3] = {act ? S.X[gid] : 0.0, act ? S.X[ms + gid] : 0.0, act ? S.X[2 * ms + gid] : 0.0};
      if (S.skin == 0) emit_nodes<R>(S, bt, L, act, gid, Xp, F, mode, fbits);  // uniform
      else if (act) emit_node<R>(S, L, gid, Xp, F, mode, fbits);
    }
    flush_fmax(S, L.par, &wmax, fbits);
  }
}

// -------------------------------------------------------- Morse repulsion --
// Eq. (13) between the nodes of different capsules, before the force kernels
// (which add the result to each node's membrane force):
//   k_morse_bin    every capsule node into the neighbour grid of its step
//                  parity (cells at least 2 lattice units wide, so every pair
//                  closer than rc <= 2 lies in neighbouring cells).  One
//                  workgroup per capsule groups its nodes by cell in LDS and
//                  reserves each group's range with one device atomic; each
//                  cell also records its owner: 0 empty, m + 1 when it holds
//                  only capsule m's nodes, -1 when it holds several capsules'
//                  (the final value does not depend on the order of the
//                  appends).  The workgroups also empty the other parity's
//                  grid, used by the previous step.
//   k_morse_force  one workgroup per capsule.  Each node marks its
//                  neighbouring cells that hold other capsules' nodes (inside
//                  a membrane nearly every cell is the capsule's own); the
//                  workgroup stages the nodes of the marked cells (ids, then
//                  positions and capsules, every load of a round in flight
//                  together) in LDS, and each node sums its pair forces from
//                  there: F = 2 alpha D0 (e^{-2 alpha (r - r0)} -
//                  e^{-alpha (r - r0)}) (X_i - X_j) / r for r < rc, each split
//                  into two 64-bit fixed-point words (units 2^-44 and 2^-96)
//                  and summed as integers: the sum is exact to 2^-96 per pair
//                  and does not depend on the order of the cell lists, and the
//                  two nodes of a pair get exact opposites.  A capsule of
//                  more than 1024 nodes, or whose marked cells or their nodes
//                  overflow the LDS tables, reads them from global memory node
//                  by node instead (the same pairs and sums).
//   k_morse_clear  an observation's grid, emptied after it (the next step
//                  bins into the same parity).
constexpr int kMorseThreads = 256;
constexpr int kMorseSlots = 512;         // LDS table of a capsule's cells (power of two)
constexpr int kMorseRound = 4;           // nodes per thread per binning round
constexpr int kMorseStage = 1024;        // other capsules' nodes staged per capsule
constexpr int kMorseNodes = 1024;        // capsule nodes of the staged path
constexpr int kMorseBatch = 4;           // entries per batch of loads (direct path)
constexpr double kMorseHi = 0x1p44;      // unit of the high fixed-point word
constexpr double kMorseLo = 0x1p52;      // unit of the low word, relative to the high one
constexpr double kMorseLimit = 128.0;    // |pair force component| limit (health bit beyond)
static_assert(kMorseWords == 2, "grid cell words: owner, count");

__device__ __forceinline__ int morse_axis(const SimDev& S, int a, double X) {
  const int n = S.n[a], ng = S.ngm[a];
  const double xw = S.wall[a] ? X : X - (double)n * floor(X / (double)n);
  const int c = (int)floor(xw * (double)ng / (double)n);
  return c < 0 ? 0 : (c >= ng ? ng - 1 : c);
}

__device__ __forceinline__ int morse_cell_of(const SimDev& S, const double X[3]) {
  return morse_axis(S, 0, X[0]) + S.ngm[0] * (morse_axis(S, 1, X[1]) + S.ngm[1] * morse_axis(S, 2, X[2]));
}

// LDS hash slot of a cell (inserted on first use); -1 when the table is full
__device__ int morse_slot(int* key, int cell) {
  int h = (int)(((uint32_t)cell * 2654435761u) >> 23) & (kMorseSlots - 1);
  for (int p = 0; p < kMorseSlots; ++p) {
    const int cur = atomicCAS(&key[h], -1, cell);
    if (cur == -1 || cur == cell) return h;
    h = (h + 1) & (kMorseSlots - 1);
  }
  return -1;
}

// slot of a cell already in the table
__device__ __forceinline__ int morse_find(const int* key, int cell) {
  int h = (int)(((uint32_t)cell * 2654435761u) >> 23) & (kMorseSlots - 1);
  for (int p = 0; p < kMorseSlots && key[h] != cell; ++p) h = (h + 1) & (kMorseSlots - 1);
  return h;
}

// a cell's owner after a node of capsule m joined it
__device__ __forceinline__ void morse_own(GLB int32_t* w, int m) {
  const int own = atomicCAS((int*)&w[0], 0, m + 1);
  if (own != 0 && own != m + 1) atomicExch((int*)&w[0], -1);
}

__global__ __launch_bounds__(kMorseThreads) void k_morse_bin(const SimDev* __restrict__ sims, Items it, int mode) {
  __shared__ int key[kMorseSlots], cnt[kMorseSlots], base[kMorseSlots];
  const int tid = threadIdx.x;
  for (int item = xcd_block(); item < it.mesh_total; item += gridDim.x) {
    const int s = find_sim(it.mesh_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    if (S.morse[0] == 0.0) continue;
    const int m = item - it.mesh_off[s];
    const int par = (int)((*S.step + it.sub) & 1);
    if (mode == 0) {
      // empty the previous step's grid: this simulation's workgroups share it out
      const int64_t nwg = it.mesh_off[s + 1] - it.mesh_off[s];
      GLB int32_t* old = S.gcount + (int64_t)(par ^ 1) * kMorseWords * S.ngrid;
      for (int64_t k = m * (int64_t)kMorseThreads + tid; k < kMorseWords * S.ngrid; k += nwg * kMorseThreads)
        old[k] = 0;
    }
    if (S.mesh_rigid[m]) continue;  // uniform: bodies take no part
    const int tm = S.mesh_tmpl[m], off = S.mesh_off[m], nn = S.t_nn[tm];
    const int64_t ms = (int64_t)S.maxn;
    GLB int32_t* gw = S.gcount + (int64_t)par * kMorseWords * S.ngrid;  // (owner, count) per cell
    GLB int32_t* gl = S.glist + (int64_t)par * S.ngrid * kMorseCap;
    for (int i0 = 0; i0 < nn; i0 += kMorseThreads * kMorseRound) {  // uniform
      for (int k = tid; k < kMorseSlots; k += kMorseThreads) {
        key[k] = -1;
        cnt[k] = 0;
      }
      __syncthreads();
      // the round's nodes join their cells' groups
      int cell[kMorseRound], slot[kMorseRound], rank[kMorseRound];
#pragma unroll
      for (int u = 0; u < kMorseRound; ++u) {
        const int i = i0 + u * kMorseThreads + tid;
        cell[u] = -1;
        slot[u] = -1;
        rank[u] = 0;
        if (i < nn) {
          const int gid = off + i;
          const double X[3] = {S.X[gid], S.X[ms + gid], S.X[2 * ms + gid]};
          if (isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2])) {
            cell[u] = morse_cell_of(S, X);
            slot[u] = morse_slot(key, cell[u]);
            if (slot[u] >= 0) rank[u] = atomicAdd(&cnt[slot[u]], 1);
          }
        }
      }
      __syncthreads();
      // one reservation per group, and the owner
      for (int k = tid; k < kMorseSlots; k += kMorseThreads)
        if (key[k] >= 0) {
          GLB int32_t* w = gw + kMorseWords * (int64_t)key[k];
          base[k] = atomicAdd((int*)&w[1], cnt[k]);
          morse_own(w, m);
        }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kMorseRound; ++u) {
        if (cell[u] < 0) continue;
        int pos;
        if (slot[u] >= 0) {
          pos = base[slot[u]] + rank[u];
        } else {  // the table was full: this node appends alone
          GLB int32_t* w = gw + kMorseWords * (int64_t)cell[u];
          pos = atomicAdd((int*)&w[1], 1);
          morse_own(w, m);
        }
        if (pos < kMorseCap) gl[(int64_t)cell[u] * kMorseCap + pos] = off + i0 + u * kMorseThreads + tid;
        else atomicOr((unsigned*)S.health, (uint32_t)kHOverflow);
      }
      __syncthreads();  // the table is cleared for the next round
    }
  }
}

// v added to the two-word accumulator: the whole multiples of 2^-44 (exact,
// |v| 2^44 < 2^51), then the remainder (exact: a double minus its integer
// part) rounded to a multiple of 2^-96.
__device__ __forceinline__ void morse_accumulate(const SimDev& S, double v, long long& hi, long long& lo) {
  if (!(fabs(v) < kMorseLimit)) {
    atomicOr((unsigned*)S.health, (uint32_t)kHForceRange);
    v = isnan(v) ? 0.0 : copysign(kMorseLimit, v);
  }
  const double t = v * kMorseHi;
  const long long h = __double2ll_rz(t);
  hi += h;
  lo += __double2ll_rn((t - (double)h) * kMorseLo);
}

// Constants of the pair force of one simulation
struct MorseParams {
  double D0, al, r0, rc;
  double rc2;    // a bound on r^2 above every r that rounds below rc (the exact test follows)
  double qn[3];  // a quarter of each period
};
__device__ __forceinline__ MorseParams morse_params(const SimDev& S) {
  MorseParams P;
  P.D0 = S.morse[0];
  P.al = S.morse[1];
  P.r0 = S.morse[2];
  P.rc = S.morse[3];
  P.rc2 = P.rc * P.rc * (1.0 + 0x1p-40);
  for (int a = 0; a < 3; ++a) P.qn[a] = 0.25 * S.n[a];
  return P;
}

// the pair force on the node at X from the node at Y, into the sums
__device__ __forceinline__ void morse_pair(const SimDev& S, const MorseParams& P, const double X[3],
                                           double y0, double y1, double y2, long long wh[3], long long wl[3]) {
  const double Y[3] = {y0, y1, y2};
  double d[3], r2 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    d[a] = X[a] - Y[a];
    // minimum image; within a quarter period the image term is exactly zero,
    // so the division is skipped
    if (!S.wall[a] && !(fabs(d[a]) <= P.qn[a])) d[a] -= (double)S.n[a] * floor(d[a] / (double)S.n[a] + 0.5);
    r2 += d[a] * d[a];
  }
  if (!(r2 <= P.rc2)) return;  // beyond the cutoff (taken before the square root)
  const double r = sqrt(r2);
  if (!(r < P.rc) || r == 0.0) return;
  const double e1 = exp(-P.al * (r - P.r0)), f = 2.0 * P.al * P.D0 * (e1 * e1 - e1) / r;
#pragma unroll
  for (int a = 0; a < 3; ++a) morse_accumulate(S, f * d[a], wh[a], wl[a]);
}

// The 27 neighbouring cells of a node's cell (each once; wrapped on periodic
// axes; entries past an axis's count repeat its first cell).
struct MorseCells {
  int cl[3][3], cnt[3];
};
__device__ __forceinline__ void morse_cells(const SimDev& S, const double X[3], MorseCells& C) {
  for (int a = 0; a < 3; ++a) {
    const int ca = morse_axis(S, a, X[a]), ng = S.ngm[a];
    int lo;
    if (ng < 3) {
      lo = 0;  // every cell once
      C.cnt[a] = ng;
    } else if (S.wall[a]) {
      lo = ca > 0 ? ca - 1 : 0;
      C.cnt[a] = (ca + 1 < ng ? ca + 1 : ng - 1) - lo + 1;
    } else {
      lo = ca - 1;
      C.cnt[a] = 3;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int v = lo + k;
      C.cl[a][k] = k >= C.cnt[a] ? lo : (v < 0 ? v + ng : (v >= ng ? v - ng : v));
    }
  }
}
// (selected without indexing the arrays at a run-time position, which would
// put them in scratch memory)
__device__ __forceinline__ int morse_pick(const int v[3], int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }
__device__ __forceinline__ int morse_cell(const SimDev& S, const MorseCells& C, int k) {
  return morse_pick(C.cl[0], k % 3) + S.ngm[0] * (morse_pick(C.cl[1], (k / 3) % 3) + S.ngm[1] * morse_pick(C.cl[2], k / 9));
}

// Bits k = kx + 3 ky + 9 kz of the neighbouring cells that hold other
// capsules' nodes (work), and of those holding several capsules' (mixed).
// The owners are loaded a layer of nine at a time.
__device__ __forceinline__ void morse_marks(const SimDev& S, const GLB int32_t* gw, const MorseCells& C, int m,
                                            uint32_t& work, uint32_t& mixed) {
  work = mixed = 0u;
#pragma unroll 1
  for (int kz = 0; kz < 3; ++kz) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int bit = 9 * kz + k, kx = k % 3, ky = k / 3;
      const int own = gw[kMorseWords * (int64_t)morse_cell(S, C, bit)];
      const bool in = kx < C.cnt[0] && ky < C.cnt[1] && kz < C.cnt[2];
      work |= (in && own != 0 && own != m + 1) ? 1u << bit : 0u;
      mixed |= own < 0 ? 1u << bit : 0u;
    }
  }
}

// the two-word sums as the node's force
__device__ __forceinline__ void morse_store(const SimDev& S, int gid, const long long wh[3], const long long wl[3]) {
  const int64_t ms = (int64_t)S.maxn;
  for (int a = 0; a < 3; ++a) {
    // carry the low word's whole multiples of 2^-44 into the high one; both
    // words then convert exactly while |F| < 2^9
    const long long c = wl[a] >> 52;
    const long long h = wh[a] + c, l = wl[a] - (c << 52);
    S.Fm[a * ms + gid] = (double)h / kMorseHi + (double)l / (kMorseHi * kMorseLo);
  }
}

// One node's pair forces read from global memory (capsules whose marked cells
// do not fit the LDS stage).
__device__ void morse_node_direct(const SimDev& S, const MorseParams& P, const GLB int32_t* gw,
                                  const GLB int32_t* gl, int m, int gid) {
  const int64_t ms = (int64_t)S.maxn;
  const double X[3] = {S.X[gid], S.X[ms + gid], S.X[2 * ms + gid]};
  long long wh[3] = {0, 0, 0}, wl[3] = {0, 0, 0};
  if (isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2])) {
    MorseCells C;
    morse_cells(S, X, C);
    uint32_t work, mixed;
    morse_marks(S, gw, C, m, work, mixed);
    while (work) {
      const int kc = __builtin_ctz(work);
      work &= work - 1u;
      const int64_t cell = morse_cell(S, C, kc);
      const bool mix = (mixed >> kc) & 1u;
      const int c0 = gw[kMorseWords * cell + 1];
      const int nc = c0 < kMorseCap ? c0 : kMorseCap;
      const GLB int32_t* ce = gl + cell * kMorseCap;
      for (int k0 = 0; k0 < nc; k0 += kMorseBatch) {
        int jb[kMorseBatch];
#pragma unroll
        for (int t = 0; t < kMorseBatch; ++t) jb[t] = k0 + t < nc ? ce[k0 + t] : -1;
#pragma unroll
        for (int t = 0; t < kMorseBatch; ++t) {
          if (jb[t] < 0) continue;
          const int j = jb[t];
          if (mix && S.node_mesh[j] == m) continue;  // the same capsule
          morse_pair(S, P, X, S.X[j], S.X[ms + j], S.X[2 * ms + j], wh, wl);
        }
      }
    }
  }
  morse_store(S, gid, wh, wl);
}

struct MorseStageLds {
  int key[kMorseSlots];    // marked cells (-1: free)
  int start[kMorseSlots];  // first staged entry of each (entries: up to the next start)
  double x[3][kMorseStage];
  int mesh[kMorseStage];
  uint32_t work[kMorseNodes];  // each node's marked neighbour cells
  int16_t wlist[kMorseNodes];  // the nodes that have some
  int wsum[kMorseThreads / 64];
  int nwork;               // entries of wlist
  int bucket[28];          // listed nodes by number of marked cells, then their offsets
  int total;               // staged entries
  int flag;                // table full
};

__global__ __launch_bounds__(kMorseThreads, 4) void k_morse_force(const SimDev* __restrict__ sims, Items it, int mode) {
  __shared__ MorseStageLds L;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int item = xcd_block(); item < it.mesh_total; item += gridDim.x) {
    const int s = find_sim(it.mesh_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    if (S.morse[0] == 0.0) continue;
    const int m = item - it.mesh_off[s];
    if (S.mesh_rigid[m]) continue;
    const int tm = S.mesh_tmpl[m], off = S.mesh_off[m], nn = S.t_nn[tm];
    const int64_t ms = (int64_t)S.maxn;
    const int par = (int)((*S.step + it.sub) & 1);
    const GLB int32_t* gw = S.gcount + (int64_t)par * kMorseWords * S.ngrid;  // (owner, count) per cell
    const GLB int32_t* gl = S.glist + (int64_t)par * S.ngrid * kMorseCap;
    const MorseParams P = morse_params(S);
    bool direct = nn > kMorseNodes;  // uniform
    if (!direct) {
      // (1) each node marks its neighbouring cells with other capsules' nodes
      for (int k = tid; k < kMorseSlots; k += kMorseThreads) L.key[k] = -1;
      if (tid < 28) L.bucket[tid] = 0;
      if (tid == 0) L.flag = 0;
      __syncthreads();
      for (int i = tid; i < nn; i += kMorseThreads) {
        const int gid = off + i;
        const double X[3] = {S.X[gid], S.X[ms + gid], S.X[2 * ms + gid]};
        uint32_t work = 0u, mixed;
        if (isfinite(X[0]) && isfinite(X[1]) && isfinite(X[2])) {
          MorseCells C;
          morse_cells(S, X, C);
          morse_marks(S, gw, C, m, work, mixed);
          for (uint32_t w = work; w; w &= w - 1u)
            if (morse_slot(L.key, morse_cell(S, C, __builtin_ctz(w))) < 0) L.flag = 1;
        }
        L.work[i] = work;
        if (!work) {  // no pair force
          const long long z[3] = {0, 0, 0};
          morse_store(S, gid, z, z);
        }
      }
      __syncthreads();
      direct = L.flag != 0;
      // the nodes with marked cells are listed for (4), most marked cells
      // first (a counting sort by their number), so that a wave's lanes
      // have similar loops and its waves hold only such nodes
      if (!direct) {
        constexpr int kPer = kMorseNodes / kMorseThreads;
        int rank[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int i = u * kMorseThreads + tid;
          rank[u] = i < nn && L.work[i] ? atomicAdd(&L.bucket[__popc(L.work[i])], 1) : 0;
        }
        __syncthreads();
        if (tid == 0) {
          int b = 0;
          for (int k = 27; k >= 1; --k) {
            const int c = L.bucket[k];
            L.bucket[k] = b;
            b += c;
          }
          L.nwork = b;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int i = u * kMorseThreads + tid;
          if (i < nn && L.work[i]) L.wlist[L.bucket[__popc(L.work[i])] + rank[u]] = (int16_t)i;
        }
      }
    }
    if (!direct) {
      // (2) entries per marked cell, and their offsets in the stage (a scan
      // over the table, two slots per thread)
      int c2[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int k = 2 * tid + u;
        int c = 0;
        if (L.key[k] >= 0) {
          c = gw[kMorseWords * (int64_t)L.key[k] + 1];
          c = c < kMorseCap ? c : kMorseCap;
        }
        c2[u] = c;
      }
      const int v = c2[0] + c2[1];
      int x = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (lane == 63) L.wsum[wv] = x;
      __syncthreads();
      int pre = 0, total = 0;
#pragma unroll
      for (int k = 0; k < kMorseThreads / 64; ++k) {
        pre += k < wv ? L.wsum[k] : 0;
        total += L.wsum[k];
      }
      L.start[2 * tid] = pre + x - v;
      L.start[2 * tid + 1] = pre + x - v + c2[0];
      if (tid == 0) L.total = total;
      __syncthreads();
      direct = total > kMorseStage;  // uniform
      if (!direct) {
        // (3) stage the entries: ids, then positions and capsules
        constexpr int kPer = kMorseStage / kMorseThreads;
        int jv[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int e = u * kMorseThreads + tid;
          jv[u] = -1;
          if (e < total) {
            int lo = 0, hi = kMorseSlots - 1;  // the last slot starting at or before e
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (L.start[mid] <= e) lo = mid;
              else hi = mid - 1;
            }
            jv[u] = gl[(int64_t)L.key[lo] * kMorseCap + (e - L.start[lo])];
          }
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
          const int e = u * kMorseThreads + tid;
          if (jv[u] < 0) continue;
          const int j = jv[u];
          L.x[0][e] = S.X[j];
          L.x[1][e] = S.X[ms + j];
          L.x[2][e] = S.X[2 * ms + j];
          L.mesh[e] = S.node_mesh[j];
        }
        __syncthreads();
        // (4) the listed nodes' pairs from the stage
        for (int k = tid; k < L.nwork; k += kMorseThreads) {
          const int i = L.wlist[k], gid = off + i;
          long long wh[3] = {0, 0, 0}, wl[3] = {0, 0, 0};
          uint32_t work = L.work[i];
          const double X[3] = {S.X[gid], S.X[ms + gid], S.X[2 * ms + gid]};
          MorseCells C;
          morse_cells(S, X, C);
          while (work) {
            const int kc = __builtin_ctz(work);
            work &= work - 1u;
            const int sl = morse_find(L.key, morse_cell(S, C, kc));
            const int e0 = L.start[sl], e1 = sl + 1 < kMorseSlots ? L.start[sl + 1] : L.total;
            for (int e = e0; e < e1; ++e)
              if (L.mesh[e] != m) morse_pair(S, P, X, L.x[0][e], L.x[1][e], L.x[2][e], wh, wl);
          }
          morse_store(S, gid, wh, wl);
        }
      }
    }
    if (direct)  // uniform
      for (int i = tid; i < nn; i += kMorseThreads) morse_node_direct(S, P, gw, gl, m, off + i);
    __syncthreads();  // the stage is reused by the next capsule
  }
}

// an observation's grid emptied (over the simulation's grid cells)
__global__ void k_morse_clear(const SimDev* __restrict__ sims, Items it) {
  for (int s = 0; s < it.nsim; ++s) {
    const SimDev& S = sims[s];
    if (S.morse[0] == 0.0) continue;
    GLB int32_t* g = S.gcount + (int64_t)(*S.step & 1) * kMorseWords * S.ngrid;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < kMorseWords * S.ngrid;
         k += (int64_t)gridDim.x * blockDim.x)
      g[k] = 0;
  }
}

// ------------------------------------------------------------ rigid bodies --
// A rigid body (Sec. 2.3) is a mesh whose nodes move with one rigid motion:
// X_k = xc + R(q) r_k, with node velocity U_k = v + Omega x (X_k - xc), Omega =
// R Ib^-1 R^T L.  Each step:
//  k_rigid_nodes  per node: the fluid velocity before the immersed-boundary
//                 force, u* = (sum_i f_i c_i + g_body / 2) / rho (Eq. (3)
//                 without the spread force), interpolated at X_k by Eq. (14)
//                 from the populations themselves; the FSI force of Eq. (17),
//                 rho_f (u* - U_k) / dt with rho_f = dt = 1, times the node's
//                 weight dv_k (a third of its triangles' areas times one
//                 lattice spacing).  The body receives it; the fluid receives
//                 its opposite through the node's spreading record.
//  k_rigid_body   per body: the force and torque, summed in a fixed order,
//                 then Newton's second law with dt = 1 (semi-implicit Euler):
//                 v += F / M, L += T, xc += v, the orientation turned by the
//                 angle |Omega| about Omega (from the new L at the old
//                 orientation), and the nodes placed at the new pose.
constexpr int kRigidThreads = 256;
constexpr int kRigidChunks = 4;  // workgroups per body in k_rigid_nodes

__device__ __forceinline__ void quat_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

// Omega = R Ib^-1 R^T L
__device__ __forceinline__ void body_omega(const double R[9], const GLB double* ibinv, const double L[3],
                                           double w[3]) {
  double t[3], t2[3];
  for (int a = 0; a < 3; ++a) t[a] = R[a] * L[0] + R[3 + a] * L[1] + R[6 + a] * L[2];
  for (int a = 0; a < 3; ++a) t2[a] = ibinv[3 * a] * t[0] + ibinv[3 * a + 1] * t[1] + ibinv[3 * a + 2] * t[2];
  for (int a = 0; a < 3; ++a) w[a] = R[3 * a] * t2[0] + R[3 * a + 1] * t2[1] + R[3 * a + 2] * t2[2];
}

// Fluid velocity without the immersed-boundary force, interpolated at X by
// Eq. (14) (stencil base floor(X) - 1 .. + 2, the records' FP64 weights); a
// solid stencil cell contributes its wall's velocity (the first wall axis
// whose layer it is, as in the velocity field).
template <int ST>
__device__ void free_velocity(const SimDev& S, int par, const double X[3], double u[3]) {
  using Rt = RealOf<ST>;
  using T = typename Store<ST>::T;
  double w[3][4];
  int c[3][4];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double fb = floor(X[a]);
    delta_weights(S.delta, X[a] - fb, w[a]);
#pragma unroll
    for (int k = 0; k < 4; ++k) c[a][k] = S.wall[a] ? (int)fb - 1 + k : wrap((int)fb - 1 + k, S.n[a]);
  }
  const GLB T* src = (const GLB T*)S.f[par];
  u[0] = u[1] = u[2] = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j)
      for (int l = 0; l < 4; ++l) {
        const int x = c[0][i], y = c[1][j], z = c[2][l];
        const double ww = w[0][i] * w[1][j] * w[2][l];
        double uc[3];
        if (solid_cell(S, x, y, z)) {
          const int cc[3] = {x, y, z};
          int sa = -1;
          for (int a = 0; a < 3; ++a)
            if (sa < 0 && S.wall[a] && (cc[a] == 0 || cc[a] == S.n[a] - 1)) sa = a;
          const double* uw = cc[sa] == 0 ? S.ulo[sa] : S.uhi[sa];
          uc[0] = uw[0]; uc[1] = uw[1]; uc[2] = uw[2];
        } else {
          const int64_t cell = x + (int64_t)S.n[0] * (y + (int64_t)S.n[1] * z);
          Rt h[kQ];
          pull_cell<ST>(S, src, x, y, z, cell, h);
          double dr = 0.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
          for (int q = 0; q < kQ; ++q) {
            const double hq = (double)h[q];
            dr += hq;
            if (kCx[q]) j[0] += kCx[q] > 0 ? hq : -hq;
            if (kCy[q]) j[1] += kCy[q] > 0 ? hq : -hq;
            if (kCz[q]) j[2] += kCz[q] > 0 ? hq : -hq;
          }
          for (int a = 0; a < 3; ++a) uc[a] = (j[a] + 0.5 * S.gb[a]) / (1.0 + dr);
        }
        for (int a = 0; a < 3; ++a) u[a] += ww * uc[a];
      }
}

template <int ST>
__global__ __launch_bounds__(kRigidThreads) void k_rigid_nodes(const SimDev* __restrict__ sims, Items it, int mode) {
  using R = RealOf<ST>;
  __shared__ BinTable bt;
  __shared__ uint32_t wmax;
  const int tid = threadIdx.x;
  if (tid == 0) wmax = 0u;
  for (int item = xcd_block(); item < it.mesh_total * kRigidChunks; item += gridDim.x) {
    const int mi = item / kRigidChunks, c = item % kRigidChunks;
    const int s = find_sim(it.mesh_off, it.nsim, mi);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int m = mi - it.mesh_off[s];
    if (!S.mesh_rigid[m]) continue;  // uniform
    const int tm = S.mesh_tmpl[m], off = S.mesh_off[m], nn = S.t_nn[tm];
    const int64_t ms = (int64_t)S.maxn;
    const ListStep L = list_step(S, it, mode);
    const int par = (int)((*S.step + it.sub) & 1);
    const GLB double* bs = S.bstate + kBodyState * (int64_t)m;
    const double xc[3] = {bs[0], bs[1], bs[2]}, q[4] = {bs[3], bs[4], bs[5], bs[6]};
    const double v[3] = {bs[7], bs[8], bs[9]}, Lm[3] = {bs[10], bs[11], bs[12]};
    double Rm[9], w[3];
    quat_rot(q, Rm);
    body_omega(Rm, S.bconst + kBodyConst * (int64_t)m + 1, Lm, w);
    uint32_t fbits = 0u;
    for (int i0 = c * kRigidThreads; i0 < nn; i0 += kRigidThreads * kRigidChunks) {  // uniform
      const int i = i0 + tid;
      const bool act = i < nn;
      const int gid = off + i;
      double Xp[3] = {0.0, 0.0, 0.0}, Fv[3] = {0.0, 0.0, 0.0};
      if (act) {
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
          Xp[a] = S.X[a * ms + gid];
          inside &= isfinite(Xp[a]) && (!S.wall[a] || (Xp[a] >= 1.0 && Xp[a] < (double)(S.n[a] - 2)));
        }
        const double r[3] = {Xp[0] - xc[0], Xp[1] - xc[1], Xp[2] - xc[2]};
        const double U[3] = {v[0] + w[1] * r[2] - w[2] * r[1], v[1] + w[2] * r[0] - w[0] * r[2],
                             v[2] + w[0] * r[1] - w[1] * r[0]};
        double us[3] = {U[0], U[1], U[2]};  // a node out of range exerts no force
        if (inside) free_velocity<ST>(S, par, Xp, us);
        const double dv = S.ndv[gid];
        double fb[3];
        for (int a = 0; a < 3; ++a) {
          fb[a] = dv * (us[a] - U[a]);  // on the body, Eq. (17)
          Fv[a] = -fb[a];               // on the fluid
          S.Fext[a * ms + gid] = fb[a];
          if (mode == 1) S.U[a * ms + gid] = U[a];
        }
        GLB double* tq = S.escr + 3 * (int64_t)gid;  // the node's torque about xc
        tq[0] = r[1] * fb[2] - r[2] * fb[1];
        tq[1] = r[2] * fb[0] - r[0] * fb[2];
        tq[2] = r[0] * fb[1] - r[1] * fb[0];
      }
      if (S.skin == 0) emit_nodes<R>(S, bt, L, act, gid, Xp, Fv, mode, fbits, 2);  // uniform: barriers
      else if (act) emit_node<R>(S, L, gid, Xp, Fv, mode, fbits, 2);
    }
    flush_fmax(S, L.par, &wmax, fbits);
  }
}

__global__ __launch_bounds__(kRigidThreads) void k_rigid_body(const SimDev* __restrict__ sims, Items it, int mode) {
  __shared__ double red[6][kRigidThreads];
  __shared__ double pose[12];  // the new xc[3], R[9]
  const int tid = threadIdx.x;
  for (int item = xcd_block(); item < it.mesh_total; item += gridDim.x) {
    const int s = find_sim(it.mesh_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int m = item - it.mesh_off[s];
    if (!S.mesh_rigid[m]) continue;  // uniform
    const int tm = S.mesh_tmpl[m], off = S.mesh_off[m], nn = S.t_nn[tm];
    const int64_t ms = (int64_t)S.maxn;
    // force and torque: per-thread sums in node order, then a fixed tree
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = tid; i < nn; i += kRigidThreads) {
      const int gid = off + i;
      for (int a = 0; a < 3; ++a) {
        acc[a] += S.Fext[a * ms + gid];
        acc[3 + a] += S.escr[3 * (int64_t)gid + a];
      }
    }
    for (int a = 0; a < 6; ++a) red[a][tid] = acc[a];
    __syncthreads();
    for (int o = kRigidThreads / 2; o > 0; o >>= 1) {
      if (tid < o)
        for (int a = 0; a < 6; ++a) red[a][tid] += red[a][tid + o];
      __syncthreads();
    }
    if (tid == 0) {
      GLB double* ft = S.bft + 6 * (int64_t)m;
      for (int a = 0; a < 6; ++a) ft[a] = red[a][0];
      if (mode == 0) {
        GLB double* bs = S.bstate + kBodyState * (int64_t)m;
        const GLB double* bc = S.bconst + kBodyConst * (int64_t)m;
        double xc[3], q[4], v[3], Lm[3], Rm[9], w[3];
        for (int a = 0; a < 3; ++a) {
          v[a] = bs[7 + a] + red[a][0] / bc[0];
          Lm[a] = bs[10 + a] + red[3 + a][0];
          xc[a] = bs[a] + v[a];
        }
        for (int a = 0; a < 4; ++a) q[a] = bs[3 + a];
        quat_rot(q, Rm);
        body_omega(Rm, bc + 1, Lm, w);
        const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (th > 0.0) {
          double sh, ch;
          sincos(0.5 * th, &sh, &ch);
          const double k = sh / th, d[4] = {ch, w[0] * k, w[1] * k, w[2] * k};
          const double n4[4] = {d[0] * q[0] - d[1] * q[1] - d[2] * q[2] - d[3] * q[3],
                                d[0] * q[1] + d[1] * q[0] + d[2] * q[3] - d[3] * q[2],
                                d[0] * q[2] - d[1] * q[3] + d[2] * q[0] + d[3] * q[1],
                                d[0] * q[3] + d[1] * q[2] - d[2] * q[1] + d[3] * q[0]};
          const double nq = sqrt(n4[0] * n4[0] + n4[1] * n4[1] + n4[2] * n4[2] + n4[3] * n4[3]);
          for (int a = 0; a < 4; ++a) q[a] = n4[a] / nq;
          quat_rot(q, Rm);
        }
        for (int a = 0; a < 3; ++a) {
          bs[a] = xc[a];
          bs[7 + a] = v[a];
          bs[10 + a] = Lm[a];
          pose[a] = xc[a];
        }
        for (int a = 0; a < 4; ++a) bs[3 + a] = q[a];
        for (int a = 0; a < 9; ++a) pose[3 + a] = Rm[a];
      }
    }
    __syncthreads();
    if (mode == 0) {
      // the nodes at the new pose; with a skin, a node whose stencil base left
      // its skin raises the next step's rebuild flag
      const int next_par = (int)((*S.step + it.sub + 1) & 1);
      bool out = false;
      for (int i = tid; i < nn; i += kRigidThreads) {
        const int gid = off + i;
        double xn[3];
        for (int a = 0; a < 3; ++a) {
          const double r0 = S.Xr[gid], r1 = S.Xr[ms + gid], r2 = S.Xr[2 * ms + gid];
          xn[a] = pose[a] + pose[3 + 3 * a] * r0 + pose[4 + 3 * a] * r1 + pose[5 + 3 * a] * r2;
          S.X[a * ms + gid] = xn[a];
        }
        if (S.skin) {
          const GLB int16_t* b0 = S.bb0 + 4 * (int64_t)gid;
          for (int a = 0; a < 3; ++a) {
            const double fb = floor(xn[a]);
            if (!(fabs(fb) < 1e9)) {
              out = true;
              continue;
            }
            int dlt = (int)fb - b0[a];
            if (!S.wall[a]) {
              dlt %= S.n[a];
              dlt = dlt > S.n[a] / 2 ? dlt - S.n[a] : (dlt < -S.n[a] / 2 ? dlt + S.n[a] : dlt);
            }
            out |= dlt > S.skin || dlt < -S.skin;
          }
        }
      }
      if (out) atomicOr((unsigned*)&S.lctl[2 + next_par], 1u);
    }
    __syncthreads();  // red and pose are reused by the next body
  }
}

// --------------------------------------------------------------- interp --
// Eq. (14) per home cube (16 x 8 x 8 cells): the workgroup loads the
// velocity of the cube and of the stencil margin around it (cells o-1 ..
// o+size+1 per axis; solid cells hold their wall's velocity) into LDS, and
// each lane sums one home node's 64 stencil points in a fixed order: the
// result does not depend on the list's order.  X^{n+1} = X^n + U in FP64.
// The workgroup also clears the cube's list for the next step's appends.
constexpr int kInterpThreads = 256;
constexpr int kCubeTile = ((1 << kCubeShift[0]) + 3) * ((1 << kCubeShift[1]) + 3) * ((1 << kCubeShift[2]) + 3);

__device__ __forceinline__ int margin_wrap(int c, int n) {
  // the margin spans -1 .. n + 17 at most; an axis shorter than the cube may need
  // several turns
  c = c < 0 ? c + n : c;
  while (c >= n) c -= n;
  return c;
}

template <typename R>
__device__ __forceinline__ void interp_node(const SimDev& S, const R (*ut)[kCubeTile], const NodeRec<R>& q,
                                            int node, const double X0[3], int ox, int oy, int oz, int mode,
                                            int next_par) {
  constexpr int ex = (1 << kCubeShift[0]) + 3, exy = ex * ((1 << kCubeShift[1]) + 3);
  // tile index of stencil point (0, 0, 0): base - 1 relative to o - 1
  const int t0 = (q.base[0] - ox) + ex * (q.base[1] - oy) + exy * (q.base[2] - oz);
  R w3[3][4];
  rec_weights(q, S.delta, w3);
  R sx = (R)0, sy = (R)0, sz = (R)0;
#pragma unroll
  for (int dz = 0; dz < 4; ++dz)
#pragma unroll
    for (int dy = 0; dy < 4; ++dy) {
      const R wyz = w3[1][dy] * w3[2][dz];
      const int trow = t0 + ex * dy + exy * dz;
#pragma unroll
      for (int dx = 0; dx < 4; ++dx) {
        const R w = w3[0][dx] * wyz;
        sx += w * ut[0][trow + dx];
        sy += w * ut[1][trow + dx];
        sz += w * ut[2][trow + dx];
      }
    }
  const int64_t ms = (int64_t)S.maxn;
  const double ux = (double)sx, uy = (double)sy, uz = (double)sz;
  if (mode == 0 && S.skin == 0) {
    S.X[node] = X0[0] + ux;
    S.X[ms + node] = X0[1] + uy;
    S.X[2 * ms + node] = X0[2] + uz;
  } else if (mode == 0) {
    const double xn[3] = {X0[0] + ux, X0[1] + uy, X0[2] + uz};
    S.X[node] = xn[0];
    S.X[ms + node] = xn[1];
    S.X[2 * ms + node] = xn[2];
    // the next step rebuilds the candidate lists when the node's stencil base
    // leaves the skin around its base at the last build
    const GLB int16_t* b0 = S.bb0 + 4 * (int64_t)node;
    bool out = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double fb = floor(xn[a]);
      if (!(fabs(fb) < 1e9)) {
        out = true;
        continue;
      }
      int dlt = (int)fb - b0[a];
      if (!S.wall[a]) {  // periodic: the shortest signed distance modulo n
        dlt %= S.n[a];
        dlt = dlt > S.n[a] / 2 ? dlt - S.n[a] : (dlt < -S.n[a] / 2 ? dlt + S.n[a] : dlt);
      }
      out |= dlt > S.skin || dlt < -S.skin;
    }
    if (out) atomicOr((unsigned*)&S.lctl[2 + next_par], 1u);
  } else {
    S.U[node] = ux;
    S.U[ms + node] = uy;
    S.U[2 * ms + node] = uz;
  }
}


template <typename R>
__global__ __launch_bounds__(kInterpThreads) void k_interp(const SimDev* __restrict__ sims, Items it,
                                                           int mode) {
  __shared__ R ut[3][kCubeTile];
  constexpr int ex = (1 << kCubeShift[0]) + 3, exy = ex * ((1 << kCubeShift[1]) + 3);
  const int tid = threadIdx.x;
  for (int item = xcd_block(); item < it.cube_total; item += gridDim.x) {
    const int s = find_sim(it.cube_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int next_par = S.skin ? (int)((*S.step + it.sub + 1) & 1) : 0;
    const int64_t h = item - it.cube_off[s];
    int cnt = S.hcount[h];
    if (cnt == 0) continue;  // no node has its base here (uniform)
    if (tid == 0 && cnt > kHomeCap) atomicOr((unsigned*)S.health, (uint32_t)kHOverflow);
    cnt = cnt > kHomeCap ? kHomeCap : cnt;
    const int n0 = S.n[0], n1 = S.n[1], n2 = S.n[2];
    const int w0 = S.wall[0], w1 = S.wall[1], w2 = S.wall[2];
    const int64_t r = h / S.nq[0];
    const int ox = (int)(h - r * S.nq[0]) << kCubeShift[0];
    const int oy = (int)(r % S.nq[1]) << kCubeShift[1];
    const int oz = (int)(r / S.nq[1]) << kCubeShift[2];
    const GLB NodeRec<R>* rec = (const GLB NodeRec<R>*)S.rec;
    const GLB int32_t* list = S.hlist + h * kHomeCap;
    // this lane's first list entry, then the tile's loads, then the entry's
    // record: the tile loads do not wait for the list entry
    int node = tid < cnt ? list[tid] : -1;
    NodeRec<R> q;
    double X0[3] = {0.0, 0.0, 0.0};  // the node's position (step mode), loaded with its record
    const int64_t ms = (int64_t)S.maxn;
    const GLB R* uf = (const GLB R*)S.u;  // [3][ncell]
    const uint32_t ncl = (uint32_t)S.ncell;
    // the tile's loads are issued in batches of kBatch per lane before their
    // LDS stores (cell indices fit 32 bits: 2 * cells * element bytes < 4 GiB)
    constexpr int kIter = (kCubeTile + kInterpThreads - 1) / kInterpThreads;
    constexpr int kBatch = 9;
    static_assert(kIter % kBatch == 0, "tile loads in whole batches");
#pragma unroll 1
    for (int k0 = 0; k0 < kIter; k0 += kBatch) {
      R v[kBatch][3];
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int t = tid + (k0 + k) * kInterpThreads;
        const int tz = t / exy, rr = t - tz * exy, ty = rr / ex, tx = rr - ty * ex;
        const int cx = w0 ? ox - 1 + tx : margin_wrap(ox - 1 + tx, n0);
        const int cy = w1 ? oy - 1 + ty : margin_wrap(oy - 1 + ty, n1);
        const int cz = w2 ? oz - 1 + tz : margin_wrap(oz - 1 + tz, n2);
        const bool in = t < kCubeTile && cx >= 0 && cx < n0 && cy >= 0 && cy < n1 && cz >= 0 && cz < n2;
        v[k][0] = v[k][1] = v[k][2] = (R)0;
        if (in) {
          const uint32_t c = (uint32_t)(cx + n0 * (cy + n1 * cz));
          v[k][0] = uf[c];
          v[k][1] = uf[ncl + c];
          v[k][2] = uf[2 * ncl + c];
        }
      }
      if (k0 == 0 && node >= 0) {
        q = *(const NodeRec<R>*)(rec + node);
        if (mode == 0) {
          X0[0] = S.X[node];
          X0[1] = S.X[ms + node];
          X0[2] = S.X[2 * ms + node];
        }
      }
#pragma unroll
      for (int k = 0; k < kBatch; ++k) {
        const int t = tid + (k0 + k) * kInterpThreads;
        if (t < kCubeTile) {
          ut[0][t] = v[k][0];
          ut[1][t] = v[k][1];
          ut[2][t] = v[k][2];
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int i0 = 0; i0 < cnt; i0 += kInterpThreads) {
      if (i0 > 0) {
        node = -1;
        if (i0 + tid < cnt) {
          node = list[i0 + tid];
          q = *(const NodeRec<R>*)(rec + node);
          if (mode == 0) {
            X0[0] = S.X[node];
            X0[1] = S.X[ms + node];
            X0[2] = S.X[2 * ms + node];
          }
        }
      }
      if (node >= 0) interp_node<R>(S, ut, q, node, X0, ox, oy, oz, mode, next_par);
    }
    __syncthreads();
    if (tid == 0) S.hcount[h] = 0;
  }
}

// grid for a grid-stride loop over `items`, a multiple of kXcds (see xcd_block)
int grid_for(int items, int cap) {
  const int g = items < cap ? items : cap;
  return (g + kXcds - 1) / kXcds * kXcds;
}

template <int ST>
void forces_impl(const SimDev* sims, const Items& it, int mode, hipStream_t s) {
  using R = RealOf<ST>;
  if (it.mesh_total <= 0) return;
  if (it.membrane) {
    hipLaunchKernelGGL(k_membrane<false>, dim3(grid_for(it.mesh_total, 1 << 16)), dim3(kMemThreads), 0, s, sims,
                       it, mode);
    if (it.big_templates)
      hipLaunchKernelGGL(k_membrane<true>, dim3(grid_for(it.mesh_total, 1 << 16)), dim3(kMemThreads), 0, s, sims,
                         it, mode);
  }
  if (it.morse) {
    const dim3 grid(grid_for(it.mesh_total, 1 << 20));
    hipLaunchKernelGGL(k_morse_bin, grid, dim3(kMorseThreads), 0, s, sims, it, mode);
    hipLaunchKernelGGL(k_morse_force, grid, dim3(kMorseThreads), 0, s, sims, it, mode);
    if (mode == 1) hipLaunchKernelGGL(k_morse_clear, dim3(256), dim3(256), 0, s, sims, it);
  }
  if (it.rigid) {
    // bodies first: their kernels only read positions and write their own nodes
    hipLaunchKernelGGL(k_rigid_nodes<ST>, dim3(grid_for(it.mesh_total * kRigidChunks, 1 << 20)),
                       dim3(kRigidThreads), 0, s, sims, it, mode);
    hipLaunchKernelGGL(k_rigid_body, dim3(grid_for(it.mesh_total, 1 << 16)), dim3(kRigidThreads), 0, s, sims, it,
                       mode);
  }
  if (it.big_templates || it.forces_variant == 1) {
    hipLaunchKernelGGL(k_edge_forces, dim3(grid_for(it.mesh_total * kEdgeChunks, 1 << 20)), dim3(256), 0, s,
                       sims, it, mode);
    hipLaunchKernelGGL(k_node_forces<R>, dim3(grid_for(it.mesh_total * kNodeChunks, 1 << 20)), dim3(256), 0,
                       s, sims, it, mode);
  } else if (sizeof(R) == 4 && it.forces_variant == 0) {
    hipLaunchKernelGGL(k_forces_fx, dim3(grid_for(it.mesh_total, 1 << 16)), dim3(kFxThreads), 0, s, sims, it,
                       mode);
  } else {
    hipLaunchKernelGGL(k_forces_lds<R>, dim3(grid_for(it.mesh_total, 1 << 16)), dim3(forces_threads<R>()), 0, s,
                       sims, it, mode);
  }
}

}  // namespace

void launch_forces(int storage, const SimDev* sims, const Items& it, int mode, hipStream_t s) {
  if (storage == kF64) forces_impl<kF64>(sims, it, mode, s);
  else if (storage == kF32) forces_impl<kF32>(sims, it, mode, s);
  else forces_impl<kF16>(sims, it, mode, s);
}

void launch_interp(int storage, const SimDev* sims, const Items& it, int mode, hipStream_t s) {
  if (it.mesh_total <= 0 || it.cube_total <= 0) return;
  const dim3 grid(grid_for(it.cube_total, 1 << 20)), block(kInterpThreads);
  if (storage == kF64) hipLaunchKernelGGL(k_interp<double>, grid, block, 0, s, sims, it, mode);
  else hipLaunchKernelGGL(k_interp<float>, grid, block, 0, s, sims, it, mode);
}

}  // namespace ibl
