// gfx950 kernels of the coupled IB-LBM timestep (libibl.so).
//
// Per timestep, on one stream:
//   k_forces   one workgroup per capsule: membrane force F(X^n) in FP64 (linear
//              springs + dihedral bending, Sec. 2.2 / Eq. (8)); per-node
//              spreading record (stencil base, delta weights of Eq. (16) or
//              Peskin's kernel, F); node appended to the candidate lists of
//              the 8^3 bricks its 4x4x4 stencil touches.
//   k_spread   one wave per brick: Eq. (15) as an ordered, atomic-free
//              scatter into LDS -- the brick's candidates are sorted by node
//              id and applied one after another by a single wave (lane =
//              stencil point), so every cell receives its shares in ascending
//              node order; the brick's force field is then written out.
//   k_lattice  one thread per cell: moments with the half-force shift
//              (Eq. (3)), BGK collision with the forcing term (Eq. (1), (2),
//              (4)), push streaming into the other A/B copy with periodic wrap
//              and halfway bounce-back (moving-wall term); u^n is written for
//              the interpolation.
//   k_interp   one wave per node: Eq. (14) over the 4x4x4 stencil with a
//              fixed shuffle-reduction tree; X^{n+1} = X^n + U in FP64.
//   k_advance  per simulation: step counter (A/B parity) and remaining steps.
// Every kernel walks a flattened (simulation, work item) list, so one launch
// serves a single simulation or a batch of uneven ones.
#include <hip/hip_fp16.h>
#include <math.h>

#include "ibl_internal.h"

namespace ibl {
namespace {

// ------------------------------------------------------------------------
// D3Q19 in this file's order: the rest velocity, the z = 0 plane, then the
// z = +-1 links.  Opposite directions are neighbours: (1,2), (3,4), ... (17,18).
// Weights: 1/3 rest, 1/18 axis links, 1/36 diagonal links.
// ------------------------------------------------------------------------
constexpr int kCx[kQ] = {0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0};
constexpr int kCy[kQ] = {0, 0, 0, 1, -1, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1};
constexpr int kCz[kQ] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 1, -1};
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr double wq(int i) {
  return i == 0 ? 1.0 / 3.0 : ((i <= 4 || i == 9 || i == 10) ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---------------------------------------------------------------- storage --
// Every storage mode keeps the offset h_i = f_i - w_i (the equilibrium at rest
// subtracted): at low Mach number f_i differs from w_i only in its low bits,
// and a body-force increment of 1e-6 added to f_i ~ 0.05 would lose most of
// its bits in binary32.  Offsets keep them.  FP16 stores h_i as binary16
// (round to nearest even); FP32 and FP64 store it at full width.
template <int ST>
struct Store;
template <>
struct Store<kF64> {
  using T = double;
  using R = double;
  __device__ static R h(const T* p, int64_t i, int) { return p[i]; }
  __device__ static void put(T* p, int64_t i, int, R hq) { p[i] = hq; }
  __device__ static double hd(const T* p, int64_t i, int) { return p[i]; }
};
template <>
struct Store<kF32> {
  using T = float;
  using R = float;
  __device__ static R h(const T* p, int64_t i, int) { return p[i]; }
  __device__ static void put(T* p, int64_t i, int, R hq) { p[i] = hq; }
  __device__ static double hd(const T* p, int64_t i, int) { return (double)p[i]; }
};
template <>
struct Store<kF16> {
  using T = __half;
  using R = float;
  __device__ static R h(const T* p, int64_t i, int) { return __half2float(p[i]); }
  __device__ static void put(T* p, int64_t i, int, R hq) { p[i] = __float2half_rn(hq); }
  __device__ static double hd(const T* p, int64_t i, int) { return (double)__half2float(p[i]); }
};

template <int ST>
using RealOf = typename Store<ST>::R;

// ------------------------------------------------------------ work items --
__device__ __forceinline__ int find_sim(const int32_t* off, int nsim, int item) {
  int lo = 0, hi = nsim;  // off[lo] <= item < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// ------------------------------------------------------------ geometry ----
struct D3 {
  double x, y, z;
};
__device__ __forceinline__ D3 sub(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 scale(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }

// Bending angle of edge (v1, v2) between the triangles (v1, v2, v0) and
// (v2, v1, v3), both counter-clockwise seen from outside: the signed angle
// between their outward normals nA = e x (v0 - v1), nB = (v3 - v2) x e with
// e = v2 - v1, positive where the surface is convex.  Returns cos and sin.
__device__ __forceinline__ void bend_angle(D3 v0, D3 v1, D3 v2, D3 v3, double& c, double& s) {
  D3 e = sub(v2, v1);
  D3 nA = cross(e, sub(v0, v1));
  D3 nB = cross(sub(v3, v2), e);
  double inv = 1.0 / sqrt(dot(nA, nA) * dot(nB, nB));
  c = dot(nA, nB) * inv;
  s = dot(cross(nA, nB), e) * inv / sqrt(dot(e, e));
}

// Force on the vertex with the given role (0: v0, 1: v1, 2: v2, 3: v3) from the
// bending energy kb (1 - cos(theta - theta0)) of one edge, Eq. (8):
// F = -kb sin(theta - theta0) dtheta/dv.  The angle gradient: the wing
// vertices move their triangle about the edge, dtheta/dv0 = -|e| nA/|nA|^2,
// dtheta/dv3 = -|e| nB/|nB|^2; the edge vertices take the complementary
// shares fixed by translation and rotation invariance, weighted by where the
// wings project onto the edge (t0, t3).
__device__ __forceinline__ D3 bend_force(D3 v0, D3 v1, D3 v2, D3 v3, double c0, double s0,
                                         double kb, int role) {
  D3 e = sub(v2, v1);
  D3 a = sub(v0, v1);
  D3 nA = cross(e, a);
  D3 nB = cross(sub(v3, v2), e);
  double e2 = dot(e, e), le = sqrt(e2);
  double nA2 = dot(nA, nA), nB2 = dot(nB, nB);
  double inv = 1.0 / sqrt(nA2 * nB2);
  double ct = dot(nA, nB) * inv;
  double st = dot(cross(nA, nB), e) * inv / le;
  double dEdth = kb * (st * c0 - ct * s0);  // kb sin(theta - theta0)
  D3 g0 = scale(nA, -le / nA2);
  D3 g3 = scale(nB, -le / nB2);
  double t0 = dot(a, e) / e2;
  double t3 = dot(sub(v3, v1), e) / e2;
  double k0, k3;
  if (role == 0) { k0 = 1.0; k3 = 0.0; }
  else if (role == 3) { k0 = 0.0; k3 = 1.0; }
  else if (role == 1) { k0 = t0 - 1.0; k3 = t3 - 1.0; }
  else { k0 = -t0; k3 = -t3; }
  return {-dEdth * (k0 * g0.x + k3 * g3.x), -dEdth * (k0 * g0.y + k3 * g3.y),
          -dEdth * (k0 * g0.z + k3 * g3.z)};
}

// Four delta weights of one axis for a node at fractional offset d in [0, 1)
// from its base cell, at stencil offsets -1, 0, +1, +2.
__device__ __forceinline__ void delta_weights(int kind, double d, double w[4]) {
  if (kind == kCos) {
    // 1/4 (1 + cos(pi r / 2)) at r = -1-d, -d, 1-d, 2-d, with t = pi d / 2
    double s, c;
    sincos(1.5707963267948966 * d, &s, &c);
    w[0] = 0.25 * (1.0 - s);
    w[1] = 0.25 * (1.0 + c);
    w[2] = 0.25 * (1.0 + s);
    w[3] = 0.25 * (1.0 - c);
  } else {
    // Peskin's 4-point kernel: every offset shares sqrt(1 + 4d - 4d^2)
    double q = sqrt(fmax(1.0 + 4.0 * d - 4.0 * d * d, 0.0));
    w[0] = (3.0 - 2.0 * d - q) * 0.125;
    w[1] = (3.0 - 2.0 * d + q) * 0.125;
    w[2] = (1.0 + 2.0 * d + q) * 0.125;
    w[3] = (1.0 + 2.0 * d - q) * 0.125;
  }
}

__device__ __forceinline__ bool solid_cell(const SimDev& S, int x, int y, int z) {
  return (S.wall[0] && (x == 0 || x == S.n[0] - 1)) || (S.wall[1] && (y == 0 || y == S.n[1] - 1)) ||
         (S.wall[2] && (z == 0 || z == S.n[2] - 1));
}

// ------------------------------------------------------------------ init --
template <int ST>
__global__ __launch_bounds__(kLatticeBlock) void k_init(const SimDev* __restrict__ sims, Items it,
                                                        int profile) {
  using T = typename Store<ST>::T;
  using R = RealOf<ST>;
  for (int item = blockIdx.x; item < it.lat_total; item += gridDim.x) {
    const int s = find_sim(it.lat_off, it.nsim, item);
    const SimDev& S = sims[s];
    const int64_t cell = (int64_t)(item - it.lat_off[s]) * kLatticeBlock + threadIdx.x;
    if (cell < S.nbrick) S.bcount[cell] = 0;
    if (cell == 0) {
      *S.step = 0;
      *S.remaining = 0;
      *S.health = 0u;
    }
    if (cell >= S.ncell) continue;
    const int nx = S.n[0], ny = S.n[1];
    const int x = (int)(cell % nx);
    const int64_t t = cell / nx;
    const int y = (int)(t % ny);
    const int z = (int)(t / ny);
    const int c[3] = {x, y, z};
    R* u = (R*)S.u;
    R* g = (R*)S.g;
    R* rho = (R*)S.rho;
    for (int a = 0; a < 3; ++a) g[a * S.ncell + cell] = (R)0;
    rho[cell] = (R)0;
    T* f0 = (T*)S.f[0];
    T* f1 = (T*)S.f[1];
    // solid layer: hold the velocity of the first wall axis it belongs to
    int sa = -1;
    for (int a = 0; a < 3; ++a)
      if (sa < 0 && S.wall[a] && (c[a] == 0 || c[a] == S.n[a] - 1)) sa = a;
    double u0[3] = {0.0, 0.0, 0.0};
    if (sa >= 0) {
      const double* v = (c[sa] == 0) ? S.ulo[sa] : S.uhi[sa];
      for (int a = 0; a < 3; ++a) u[a * S.ncell + cell] = (R)v[a];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        Store<ST>::put(f0, (int64_t)q * S.ncell + cell, q, (R)0);
        Store<ST>::put(f1, (int64_t)q * S.ncell + cell, q, (R)0);
      }
      continue;
    }
    if (profile) {
      int pa = -1;
      for (int a = 0; a < 3; ++a)
        if (S.wall[a]) pa = a;
      if (pa >= 0) {
        double sfrac = ((double)c[pa] - 0.5) / (double)(S.n[pa] - 2);
        for (int a = 0; a < 3; ++a) u0[a] = S.ulo[pa][a] + (S.uhi[pa][a] - S.ulo[pa][a]) * sfrac;
      }
    }
    for (int a = 0; a < 3; ++a) u[a * S.ncell + cell] = (R)u0[a];
    const double usq = u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const double cu = kCx[q] * u0[0] + kCy[q] * u0[1] + kCz[q] * u0[2];
      // f_eq(rho = 1) - w_q, Eq. (2)
      const double hq = wq(q) * (3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
      Store<ST>::put(f0, (int64_t)q * S.ncell + cell, q, (R)hq);
      Store<ST>::put(f1, (int64_t)q * S.ncell + cell, q, (R)hq);
    }
  }
}

// ----------------------------------------------------------- rest state --
__global__ void k_template_rest(const SimDev* __restrict__ sim, int tmpl, int nedges,
                                const double* __restrict__ xref) {
  const SimDev& S = *sim;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nedges) return;
  const int ge = S.t_edge0[tmpl] + e;
  const int* v = S.ev + 4 * ge;
  D3 p[4];
  for (int k = 0; k < 4; ++k) p[k] = {xref[3 * v[k]], xref[3 * v[k] + 1], xref[3 * v[k] + 2]};
  D3 d = sub(p[2], p[1]);
  S.el0[ge] = sqrt(dot(d, d));
  double c, s;
  bend_angle(p[0], p[1], p[2], p[3], c, s);
  S.ec0[ge] = c;
  S.es0[ge] = s;
}

// --------------------------------------------------------------- forces --
template <typename R>
__global__ __launch_bounds__(256) void k_forces(const SimDev* __restrict__ sims, Items it,
                                                int mode) {
  for (int item = blockIdx.x; item < it.mesh_total; item += gridDim.x) {
    const int s = find_sim(it.mesh_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= 0) continue;
    const int m = item - it.mesh_off[s];
    const int tm = S.mesh_tmpl[m];
    const int off = S.mesh_off[m];
    const double ks = S.mesh_ks[m], kb = S.mesh_kb[m];
    const int nn = S.t_nn[tm];
    const int row0 = S.t_node0[tm];
    const int64_t ms = (int64_t)S.maxn;
    const double* X = S.X;
    NodeRec<R>* rec = (NodeRec<R>*)S.rec;
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
      const int gid = off + i;
      D3 F = {0.0, 0.0, 0.0};
      const int r0 = S.inc_ptr[row0 + i], r1 = S.inc_ptr[row0 + i + 1];
      for (int r = r0; r < r1; ++r) {
        const int ent = S.inc[r];
        const int e = ent >> 2, role = ent & 3;
        const int* v = S.ev + 4 * e;
        D3 p[4];
        for (int k = 0; k < 4; ++k) {
          const int g = off + v[k];
          p[k] = {X[g], X[ms + g], X[2 * ms + g]};
        }
        if (role == 1 || role == 2) {
          // linear spring 1/2 ks (l - l0)^2 on the edge (v1, v2)
          D3 d = sub(p[2], p[1]);
          const double l = sqrt(dot(d, d));
          const double k = ks * (l - S.el0[e]) / l;
          const double sg = (role == 1) ? 1.0 : -1.0;
          F.x += sg * k * d.x;
          F.y += sg * k * d.y;
          F.z += sg * k * d.z;
        }
        if (kb != 0.0) {
          D3 fb = bend_force(p[0], p[1], p[2], p[3], S.ec0[e], S.es0[e], kb, role);
          F.x += fb.x;
          F.y += fb.y;
          F.z += fb.z;
        }
      }
      S.F[gid] = F.x;
      S.F[ms + gid] = F.y;
      S.F[2 * ms + gid] = F.z;
      // spreading record at X^n
      const double Xp[3] = {X[gid], X[ms + gid], X[2 * ms + gid]};
      NodeRec<R> q;
      int valid = 1;
      for (int a = 0; a < 3; ++a) {
        if (!isfinite(Xp[a])) {
          valid = 0;
          atomicOr(S.health, (uint32_t)kHNonfiniteX);
        } else if (S.wall[a] && !(Xp[a] >= 1.0 && Xp[a] < (double)(S.n[a] - 2))) {
          valid = 0;
          atomicOr(S.health, (uint32_t)kHNodeRange);
        }
      }
      q.valid = valid;
      const double Fv[3] = {F.x, F.y, F.z};
      for (int a = 0; a < 3; ++a) {
        const double fb = valid ? floor(Xp[a]) : 0.0;
        q.base[a] = (int32_t)fb;
        double w[4];
        delta_weights(S.delta, valid ? Xp[a] - fb : 0.0, w);
        for (int k = 0; k < 4; ++k) q.w[a][k] = (R)w[k];
        q.F[a] = (R)Fv[a];
      }
      q.pad = (R)0;
      rec[gid] = q;
      if (!valid) continue;
      // candidate lists of the bricks the stencil touches
      int bl[3][4], nbl[3];
      for (int a = 0; a < 3; ++a) {
        nbl[a] = 0;
        for (int k = 0; k < 4; ++k) {
          int c = q.base[a] - 1 + k;
          if (!S.wall[a]) c = wrap(c, S.n[a]);
          const int b = c / kBrick;
          bool dup = false;
          for (int j = 0; j < nbl[a]; ++j) dup |= (bl[a][j] == b);
          if (!dup) bl[a][nbl[a]++] = b;
        }
      }
      for (int iz = 0; iz < nbl[2]; ++iz)
        for (int iy = 0; iy < nbl[1]; ++iy)
          for (int ix = 0; ix < nbl[0]; ++ix) {
            const int64_t b = bl[0][ix] + (int64_t)S.nb[0] * (bl[1][iy] + (int64_t)S.nb[1] * bl[2][iz]);
            const int slot = atomicAdd(&S.bcount[b], 1);
            if (slot < kCandCap) S.blist[b * kCandCap + slot] = gid;
          }
    }
  }
}

// --------------------------------------------------------------- spread --
template <typename R>
__global__ __launch_bounds__(64) void k_spread(const SimDev* __restrict__ sims, Items it, int mode) {
  __shared__ int cand[kCandCap];
  __shared__ R gl[3][kBrickCells];
  const int lane = threadIdx.x;
  const int dx = lane & 3, dy = (lane >> 2) & 3, dz = lane >> 4;
  for (int item = blockIdx.x; item < it.brick_total; item += gridDim.x) {
    const int s = find_sim(it.brick_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= 0) continue;
    const int64_t b = item - it.brick_off[s];
    const int bx = (int)(b % S.nb[0]);
    const int64_t t = b / S.nb[0];
    const int by = (int)(t % S.nb[1]);
    const int bz = (int)(t / S.nb[1]);
    const int ox = bx * kBrick, oy = by * kBrick, oz = bz * kBrick;
    int cnt = S.bcount[b];
    __syncthreads();
    if (lane == 0) {
      S.bcount[b] = 0;
      if (cnt > kCandCap) atomicOr(S.health, (uint32_t)kHOverflow);
    }
    cnt = cnt > kCandCap ? kCandCap : cnt;
    int P = 1;
    while (P < cnt) P <<= 1;
    for (int i = lane; i < P; i += 64) cand[i] = (i < cnt) ? S.blist[b * kCandCap + i] : 0x7fffffff;
    for (int i = lane; i < kBrickCells; i += 64) gl[0][i] = gl[1][i] = gl[2][i] = (R)0;
    __syncthreads();
    // bitonic sort of cand[0..P) ascending
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < P; i += 64) {
          const int l = i ^ j;
          if (l > i) {
            const int ai = cand[i], al = cand[l];
            const bool up = ((i & k) == 0);
            if ((ai > al) == up) {
              cand[i] = al;
              cand[l] = ai;
            }
          }
        }
        __syncthreads();
      }
    }
    // ordered scatter: one node after another, lane = stencil point
    const NodeRec<R>* rec = (const NodeRec<R>*)S.rec;
    for (int k = 0; k < cnt; ++k) {
      const int node = __builtin_amdgcn_readfirstlane(cand[k]);
      const NodeRec<R>& q = rec[node];
      int cx = q.base[0] - 1 + dx, cy = q.base[1] - 1 + dy, cz = q.base[2] - 1 + dz;
      if (!S.wall[0]) cx = wrap(cx, S.n[0]);
      if (!S.wall[1]) cy = wrap(cy, S.n[1]);
      if (!S.wall[2]) cz = wrap(cz, S.n[2]);
      const int lx = cx - ox, ly = cy - oy, lz = cz - oz;
      if (lx >= 0 && lx < kBrick && ly >= 0 && ly < kBrick && lz >= 0 && lz < kBrick &&
          !solid_cell(S, cx, cy, cz)) {
        const R w = q.w[0][dx] * q.w[1][dy] * q.w[2][dz];
        const int li = lx + kBrick * (ly + kBrick * lz);
        gl[0][li] += w * q.F[0];
        gl[1][li] += w * q.F[1];
        gl[2][li] += w * q.F[2];
      }
    }
    __syncthreads();
    R* g = (R*)S.g;
    for (int i = lane; i < kBrickCells; i += 64) {
      const int lx = i % kBrick, ly = (i / kBrick) % kBrick, lz = i / (kBrick * kBrick);
      const int x = ox + lx, y = oy + ly, z = oz + lz;
      if (x < S.n[0] && y < S.n[1] && z < S.n[2]) {
        const int64_t c = x + (int64_t)S.n[0] * (y + (int64_t)S.n[1] * z);
        g[c] = gl[0][i];
        g[S.ncell + c] = gl[1][i];
        g[2 * S.ncell + c] = gl[2][i];
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------------- lattice --
template <int ST>
__global__ __launch_bounds__(kLatticeBlock) void k_lattice(const SimDev* __restrict__ sims,
                                                           Items it, int mode) {
  using T = typename Store<ST>::T;
  using R = RealOf<ST>;
  for (int item = blockIdx.x; item < it.lat_total; item += gridDim.x) {
    const int s = find_sim(it.lat_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= 0) continue;
    const int64_t cell = (int64_t)(item - it.lat_off[s]) * kLatticeBlock + threadIdx.x;
    if (cell >= S.ncell) continue;
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int x = (int)(cell % nx);
    const int64_t t = cell / nx;
    const int y = (int)(t % ny);
    const int z = (int)(t / ny);
    R* uf = (R*)S.u;
    const int64_t nc = S.ncell;
    if (solid_cell(S, x, y, z)) {
      if (mode == 1) {
        R* rf = (R*)S.rho;
        rf[cell] = (R)0;
      }
      continue;
    }
    const int par = (int)(*S.step & 1);
    const T* src = (const T*)S.f[par];
    R h[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) h[q] = Store<ST>::h(src, (int64_t)q * nc + cell, q);
    // moments, Eq. (3): rho = sum f = 1 + sum h ; rho u = sum h c + g/2
    R drho = (R)0, jx = (R)0, jy = (R)0, jz = (R)0;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      drho += h[q];
      if (kCx[q]) jx += kCx[q] > 0 ? h[q] : -h[q];
      if (kCy[q]) jy += kCy[q] > 0 ? h[q] : -h[q];
      if (kCz[q]) jz += kCz[q] > 0 ? h[q] : -h[q];
    }
    R gx = (R)S.gb[0], gy = (R)S.gb[1], gz = (R)S.gb[2];
    if (S.has_ib) {
      const R* gf = (const R*)S.g;
      gx += gf[cell];
      gy += gf[nc + cell];
      gz += gf[2 * nc + cell];
    }
    const R rho = (R)1 + drho;
    const R irho = (R)1 / rho;
    const R ux = (jx + (R)0.5 * gx) * irho;
    const R uy = (jy + (R)0.5 * gy) * irho;
    const R uz = (jz + (R)0.5 * gz) * irho;
    if (mode == 1) {
      R* rf = (R*)S.rho;
      rf[cell] = rho;
      uf[cell] = ux;
      uf[nc + cell] = uy;
      uf[2 * nc + cell] = uz;
      continue;
    }
    if (S.has_ib) {
      uf[cell] = ux;
      uf[nc + cell] = uy;
      uf[2 * nc + cell] = uz;
    }
    // collision, Eq. (1), (2), (4), in offset form h = f - w
    const R om = (R)(1.0 / S.tau);
    const R pre = (R)(1.0 - 0.5 / S.tau);
    const R usq = ux * ux + uy * uy + uz * uz;
    const R ug = ux * gx + uy * gy + uz * gz;
    T* dst = (T*)S.f[par ^ 1];
    const int wx = S.wall[0], wy = S.wall[1], wz = S.wall[2];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const R w = (R)wq(q);
      const R cu = (R)kCx[q] * ux + (R)kCy[q] * uy + (R)kCz[q] * uz;
      const R cg = (R)kCx[q] * gx + (R)kCy[q] * gy + (R)kCz[q] * gz;
      // f_eq - w = w (drho + rho (3 cu + 9/2 cu^2 - 3/2 u^2))
      const R heq = w * (drho + rho * ((R)3 * cu + (R)4.5 * cu * cu - (R)1.5 * usq));
      const R Fq = pre * w * ((R)3 * (cg - ug) + (R)9 * cu * cg);
      const R hs = h[q] - om * (h[q] - heq) + Fq;
      // push to x + c_q
      int xn = x + kCx[q], yn = y + kCy[q], zn = z + kCz[q];
      if (!wx) xn = xn < 0 ? xn + nx : (xn >= nx ? xn - nx : xn);
      if (!wy) yn = yn < 0 ? yn + ny : (yn >= ny ? yn - ny : yn);
      if (!wz) zn = zn < 0 ? zn + nz : (zn >= nz ? zn - nz : zn);
      const bool sx = wx && (xn == 0 || xn == nx - 1);
      const bool sy = wy && (yn == 0 || yn == ny - 1);
      const bool sz = wz && (zn == 0 || zn == nz - 1);
      if (q != 0 && (sx || sy || sz)) {
        // halfway bounce-back off the wall layer of the first wall axis hit
        const int a = sx ? 0 : (sy ? 1 : 2);
        const int cn = a == 0 ? xn : (a == 1 ? yn : zn);
        const double* uw = cn == 0 ? S.ulo[a] : S.uhi[a];
        const R cuw = (R)(kCx[q] * uw[0] + kCy[q] * uw[1] + kCz[q] * uw[2]);
        Store<ST>::put(dst, (int64_t)opp(q) * nc + cell, opp(q), hs - (R)6 * w * cuw);
      } else {
        const int64_t dn = xn + (int64_t)nx * (yn + (int64_t)ny * zn);
        Store<ST>::put(dst, (int64_t)q * nc + dn, q, hs);
      }
    }
  }
}

// --------------------------------------------------------------- interp --
template <typename R>
__global__ __launch_bounds__(256) void k_interp(const SimDev* __restrict__ sims, Items it, int mode) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int dx = lane & 3, dy = (lane >> 2) & 3, dz = lane >> 4;
  for (int item = blockIdx.x; item < it.node_total; item += gridDim.x) {
    const int s = find_sim(it.node_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= 0) continue;
    const int node = (item - it.node_off[s]) * kNodesPerItem + wave;
    if (node >= S.nnodes) continue;
    const NodeRec<R>& q = ((const NodeRec<R>*)S.rec)[node];
    const int64_t ms = (int64_t)S.maxn;
    if (!q.valid) {
      if (lane == 0) S.U[node] = S.U[ms + node] = S.U[2 * ms + node] = 0.0;
      continue;
    }
    int cx = q.base[0] - 1 + dx, cy = q.base[1] - 1 + dy, cz = q.base[2] - 1 + dz;
    if (!S.wall[0]) cx = wrap(cx, S.n[0]);
    if (!S.wall[1]) cy = wrap(cy, S.n[1]);
    if (!S.wall[2]) cz = wrap(cz, S.n[2]);
    const int64_t c = cx + (int64_t)S.n[0] * (cy + (int64_t)S.n[1] * cz);
    const R* u = (const R*)S.u;
    const R w = q.w[0][dx] * q.w[1][dy] * q.w[2][dz];
    R sx = w * u[c], sy = w * u[S.ncell + c], sz = w * u[2 * S.ncell + c];
    // fixed butterfly reduction over the 64 stencil points
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sx += __shfl_xor(sx, o, 64);
      sy += __shfl_xor(sy, o, 64);
      sz += __shfl_xor(sz, o, 64);
    }
    if (lane == 0) {
      const double U[3] = {(double)sx, (double)sy, (double)sz};
      for (int a = 0; a < 3; ++a) S.U[a * ms + node] = U[a];
      if (mode == 0)
        for (int a = 0; a < 3; ++a) S.X[a * ms + node] += U[a];
    }
  }
}

// -------------------------------------------------------------- advance --
__global__ void k_advance(const SimDev* __restrict__ sims, int nsim) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsim) return;
  const SimDev& S = sims[s];
  if (*S.remaining > 0) {
    *S.step += 1;
    *S.remaining -= 1;
  }
}

// -------------------------------------------------------------- reduce --
template <int ST>
__global__ __launch_bounds__(256) void k_reduce(const SimDev* __restrict__ sims, Items it) {
  using T = typename Store<ST>::T;
  __shared__ double sh[4][256];
  for (int item = blockIdx.x; item < it.red_total; item += gridDim.x) {
    const int s = find_sim(it.red_off, it.nsim, item);
    const SimDev& S = sims[s];
    const int64_t c0 = (int64_t)(item - it.red_off[s]) * kReduceItemCells;
    const int par = (int)(*S.step & 1);
    const T* f = (const T*)S.f[par];
    double m = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    uint32_t bad = 0u;
    for (int k = threadIdx.x; k < kReduceItemCells; k += blockDim.x) {
      const int64_t cell = c0 + k;
      if (cell >= S.ncell) break;
      const int x = (int)(cell % S.n[0]);
      const int64_t t = cell / S.n[0];
      const int y = (int)(t % S.n[1]);
      const int z = (int)(t / S.n[1]);
      if (solid_cell(S, x, y, z)) continue;
      double dr = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
      for (int q = 0; q < kQ; ++q) {
        const double hq = Store<ST>::hd(f, (int64_t)q * S.ncell + cell, q);
        dr += hq;
        jx += kCx[q] * hq;
        jy += kCy[q] * hq;
        jz += kCz[q] * hq;
      }
      const double rho = 1.0 + dr;
      if (!isfinite(rho) || !isfinite(jx) || !isfinite(jy) || !isfinite(jz)) bad |= kHNonfiniteF;
      else if (rho <= 0.0) bad |= kHRho;
      else if ((jx * jx + jy * jy + jz * jz) > 0.09 * rho * rho) bad |= kHMach;
      m += rho;
      px += jx;
      py += jy;
      pz += jz;
    }
    if (bad) atomicOr(S.health, bad);
    sh[0][threadIdx.x] = m;
    sh[1][threadIdx.x] = px;
    sh[2][threadIdx.x] = py;
    sh[3][threadIdx.x] = pz;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o)
        for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x < 4) S.red[4 * (int64_t)(item - it.red_off[s]) + threadIdx.x] = sh[threadIdx.x][0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_reduce_final(const SimDev* __restrict__ sims, Items it) {
  __shared__ double sh[4][256];
  const int s = blockIdx.x;
  const SimDev& S = sims[s];
  const int nitem = it.red_off[s + 1] - it.red_off[s];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nitem; i += blockDim.x)
    for (int a = 0; a < 4; ++a) acc[a] += S.red[4 * (int64_t)i + a];
  for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] = acc[a];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 4) S.red_out[threadIdx.x] = sh[threadIdx.x][0];
}

int grid_for(int items, int cap) { return items < cap ? items : cap; }

}  // namespace

// ------------------------------------------------------------ launchers --
hipError_t launch_init(int storage, const SimDev* sims, const Items& it, int profile, hipStream_t s) {
  if (it.lat_total <= 0) return hipSuccess;
  const int grid = grid_for(it.lat_total, 1 << 20);
  if (storage == kF64) hipLaunchKernelGGL(k_init<kF64>, dim3(grid), dim3(kLatticeBlock), 0, s, sims, it, profile);
  else if (storage == kF32) hipLaunchKernelGGL(k_init<kF32>, dim3(grid), dim3(kLatticeBlock), 0, s, sims, it, profile);
  else hipLaunchKernelGGL(k_init<kF16>, dim3(grid), dim3(kLatticeBlock), 0, s, sims, it, profile);
  return hipGetLastError();
}

hipError_t launch_template_rest(const SimDev* sim, int tmpl, int nedges, const double* xref,
                                hipStream_t s) {
  const int grid = (nedges + 255) / 256;
  if (grid > 0) hipLaunchKernelGGL(k_template_rest, dim3(grid), dim3(256), 0, s, sim, tmpl, nedges, xref);
  return hipGetLastError();
}

template <int ST>
static void phase_impl(const SimDev* sims, const Items& it, int phase, int mode, hipStream_t s) {
  using R = RealOf<ST>;
  switch (phase) {
    case kPhaseForces:
      if (it.mesh_total > 0)
        hipLaunchKernelGGL(k_forces<R>, dim3(grid_for(it.mesh_total, 1 << 16)), dim3(256), 0, s, sims, it, mode);
      break;
    case kPhaseSpread:
      if (it.mesh_total > 0 && it.brick_total > 0)
        hipLaunchKernelGGL(k_spread<R>, dim3(grid_for(it.brick_total, 1 << 20)), dim3(64), 0, s, sims, it, mode);
      break;
    case kPhaseLattice:
      hipLaunchKernelGGL(k_lattice<ST>, dim3(grid_for(it.lat_total, 1 << 22)), dim3(kLatticeBlock), 0, s, sims, it, mode);
      break;
    case kPhaseInterp:
      if (it.node_total > 0)
        hipLaunchKernelGGL(k_interp<R>, dim3(grid_for(it.node_total, 1 << 20)), dim3(256), 0, s, sims, it, mode);
      break;
    case kPhaseAdvance:
      if (mode == 0) hipLaunchKernelGGL(k_advance, dim3((it.nsim + 63) / 64), dim3(64), 0, s, sims, it.nsim);
      break;
  }
}

hipError_t launch_phase(int storage, const SimDev* sims, const Items& it, int phase, int mode, hipStream_t s) {
  if (storage == kF64) phase_impl<kF64>(sims, it, phase, mode, s);
  else if (storage == kF32) phase_impl<kF32>(sims, it, phase, mode, s);
  else phase_impl<kF16>(sims, it, phase, mode, s);
  return hipGetLastError();
}

hipError_t launch_step(int storage, const SimDev* sims, const Items& it, int mode, hipStream_t s) {
  for (int ph = 0; ph < kNumPhases; ++ph) {
    hipError_t e = launch_phase(storage, sims, it, ph, mode, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reduce(int storage, const SimDev* sims, const Items& it, hipStream_t s) {
  const int grid = grid_for(it.red_total, 1 << 20);
  if (storage == kF64) hipLaunchKernelGGL(k_reduce<kF64>, dim3(grid), dim3(256), 0, s, sims, it);
  else if (storage == kF32) hipLaunchKernelGGL(k_reduce<kF32>, dim3(grid), dim3(256), 0, s, sims, it);
  else hipLaunchKernelGGL(k_reduce<kF16>, dim3(grid), dim3(256), 0, s, sims, it);
  hipLaunchKernelGGL(k_reduce_final, dim3(it.nsim), dim3(256), 0, s, sims, it);
  return hipGetLastError();
}

}  // namespace ibl
