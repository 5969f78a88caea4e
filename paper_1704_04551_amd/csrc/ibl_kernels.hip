// gfx950 kernels of the coupled IB-LBM timestep (libibl.so).
//
// Per timestep, on one stream:
//   k_forces   membrane forces, spreading records, candidate lists (ibl_ib.hip)
//   k_lattice  one workgroup per lattice brick: force spreading of the
//              brick's candidate nodes into LDS (Eq. (15), fixed-point
//              integer sums), then per cell the moments with the half-force
//              shift (Eq. (3)), BGK collision with the forcing term (Eq. (1),
//              (2), (4)) and pull streaming with periodic wrap and halfway
//              bounce-back (moving-wall term); u^n is written for the
//              interpolation.  The force field never leaves LDS.
//   k_interp   velocity interpolation and node update (ibl_ib.hip)
//   k_advance  per simulation, after a captured sequence of steps: step
//              counter (A/B parity) and remaining steps.
// Every kernel walks a flattened (simulation, work item) list, so one launch
// serves a single simulation or a batch of uneven ones.
#include <type_traits>

// No implicit contraction of a * b + c into an FMA anywhere in this file:
// the compiler may contract differently in different instantiations of a
// kernel (with and without moving walls, say), and results that must be
// bitwise equal across them would then differ in the last bit.  The FMAs of
// the hot paths are written out.
#pragma clang fp contract(off)

#include "ibl_device.h"

namespace ibl {
namespace {

// 1 / r for r near 1: hardware reciprocal, refined by Newton steps to the
// type's precision
__device__ __forceinline__ float rcp_r(float r) {
  const float i = __builtin_amdgcn_rcpf(r);
  return fmaf(i, fmaf(-r, i, 1.0f), i);
}
__device__ __forceinline__ double rcp_r(double r) {
  double i = __builtin_amdgcn_rcp(r);
  i = fma(i, fma(-r, i, 1.0), i);
  return fma(i, fma(-r, i, 1.0), i);
}

// ------------------------------------------------------------------ init --
template <int ST>
__device__ void init_cell(const SimDev& S, int x, int y, int z, int profile) {
  using T = typename Store<ST>::T;
  using R = RealOf<ST>;
  const int64_t cell = x + (int64_t)S.n[0] * (y + (int64_t)S.n[1] * z);
  const int c[3] = {x, y, z};
  GLB R* u = (GLB R*)S.u;  // [3][ncell]
  GLB R* g = (GLB R*)S.g;
  GLB R* rho = (GLB R*)S.rho;
  for (int a = 0; a < 3; ++a) g[a * S.ncell + cell] = (R)0;
  rho[cell] = (R)0;
  GLB T* f0 = (GLB T*)S.f[0];
  GLB T* f1 = (GLB T*)S.f[1];
  // solid layer: hold the velocity of the first wall axis it belongs to
  int sa = -1;
  for (int a = 0; a < 3; ++a)
    if (sa < 0 && S.wall[a] && (c[a] == 0 || c[a] == S.n[a] - 1)) sa = a;
  double u0[3] = {0.0, 0.0, 0.0};
  if (sa >= 0) {
    const double* v = (c[sa] == 0) ? S.ulo[sa] : S.uhi[sa];
    u[cell] = (R)v[0];
    u[S.ncell + cell] = (R)v[1];
    u[2 * S.ncell + cell] = (R)v[2];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      Store<ST>::put(f0, (int64_t)q * S.ncell + cell, q, (R)0);
      Store<ST>::put(f1, (int64_t)q * S.ncell + cell, q, (R)0);
    }
    return;
  }
  // initial velocity u0 at a fluid cell: rest, or the linear profile across
  // the (last) wall axis
  int pa = -1;
  if (profile)
    for (int a = 0; a < 3; ++a)
      if (S.wall[a]) pa = a;
  auto u_init = [&](const int cc[3], double uo[3]) {
    uo[0] = uo[1] = uo[2] = 0.0;
    if (pa >= 0) {
      const double sfrac = ((double)cc[pa] - 0.5) / (double)(S.n[pa] - 2);
      for (int a = 0; a < 3; ++a) uo[a] = S.ulo[pa][a] + (S.uhi[pa][a] - S.ulo[pa][a]) * sfrac;
    }
  };
  // f_eq(rho = 1, v) - w_q, Eq. (2)
  auto h_eq = [](int q, const double v[3]) {
    const double cu = kCx[q] * v[0] + kCy[q] * v[1] + kCz[q] * v[2];
    const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    return wq(q) * (3.0 * cu + 4.5 * cu * cu - 1.5 * vv);
  };
  u_init(c, u0);
  u[cell] = (R)u0[0];
  u[S.ncell + cell] = (R)u0[1];
  u[2 * S.ncell + cell] = (R)u0[2];
  // stored populations are post-collision values that the first step's
  // pull turns into f_eq(1, u0): the one read by the consumer x + c_q, or,
  // where x + c_q is a wall layer, the bounce-back value of direction opp(q)
  // at x itself (the slot carries its wall term, as a step leaves it)
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    int cn[3] = {x + kCx[q], y + kCy[q], z + kCz[q]};
    int wall_axis = -1;
    for (int a = 0; a < 3; ++a) {
      if (!S.wall[a]) cn[a] = cn[a] < 0 ? cn[a] + S.n[a] : (cn[a] >= S.n[a] ? cn[a] - S.n[a] : cn[a]);
      else if (wall_axis < 0 && (cn[a] == 0 || cn[a] == S.n[a] - 1)) wall_axis = a;
    }
    double hq;
    if (q != 0 && wall_axis >= 0) {
      hq = h_eq(opp(q), u0);
    } else {
      double uc[3];
      u_init(cn, uc);
      hq = h_eq(q, uc);
    }
    Store<ST>::put(f0, (int64_t)q * S.ncell + cell, q, (R)hq);
    Store<ST>::put(f1, (int64_t)q * S.ncell + cell, q, (R)hq);
  }
}

template <int ST>
__global__ __launch_bounds__(kBrickThreads) void k_init(const SimDev* __restrict__ sims, Items it,
                                                        int profile) {
  const int tid = threadIdx.x;
  for (int item = xcd_block(); item < it.lat_total; item += gridDim.x) {
    const int s = find_sim(it.lat_off, it.nsim, item);
    const SimDev& S = sims[s];
    const int64_t b = item - it.lat_off[s];
    // the arena may hold a previous user's data: every list is emptied
    for (int64_t j = b * kBrickThreads + tid; j < S.ncube; j += S.nbrick * kBrickThreads) S.hcount[j] = 0;
    for (int64_t j = b * kBrickThreads + tid; j < 2 * kMorseWords * S.ngrid; j += S.nbrick * kBrickThreads) S.gcount[j] = 0;
    if (tid == 0) {
      S.bcount[b] = 0;
      S.bcount[S.nbrick + b] = 0;
      if (b == 0) {
        *S.step = 0;
        *S.remaining = 0;
        *S.health = 0u;
        reset_list_control(S);
      }
    }
    int ox, oy, oz;
    brick_origin(S, b, ox, oy, oz);
    const int x = ox + (tid & (S.bs[0] - 1)), y = oy + (tid >> S.bsh[0]);
    if (x >= S.n[0] || y >= S.n[1]) continue;
    for (int k = 0; k < brick_depth(ST) && oz + k < S.n[2]; ++k) init_cell<ST>(S, x, y, oz + k, profile);
  }
}

// Candidate lists and the Morse neighbour grids emptied, lists marked for a
// rebuild at the next step (after the nodes or the step counter were set
// from the host).
__global__ void k_reset_lists(const SimDev* __restrict__ sim) {
  const SimDev& S = *sim;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < S.nbrick) {
    S.bcount[b] = 0;
    S.bcount[S.nbrick + b] = 0;
  }
  for (int64_t k = b; k < 2 * kMorseWords * S.ngrid; k += (int64_t)gridDim.x * blockDim.x) S.gcount[k] = 0;
  if (b == 0) reset_list_control(S);
}

// ----------------------------------------------------------- rest state --
__global__ void k_template_rest(const SimDev* __restrict__ sim, int tmpl, int nedges,
                                const double* __restrict__ xref) {
  const SimDev& S = *sim;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nedges) return;
  const int ge = S.t_edge0[tmpl] + e;
  const GLB int* v = S.ev + 4 * ge;
  D3 p[4];
  for (int k = 0; k < 4; ++k) p[k] = {xref[3 * v[k]], xref[3 * v[k] + 1], xref[3 * v[k] + 2]};
  D3 d = sub(p[2], p[1]);
  S.el0[ge] = sqrt(dot(d, d));
  double c, s;
  bend_angle(p[0], p[1], p[2], p[3], c, s);
  S.ec0[ge] = c;
  S.es0[ge] = s;
}

// -------------------------------------------------------------- lattice --
// Fixed-point accumulator of the spread force: every share w F is scaled by
// 2^s, s = kBits - e where 2^e bounds the step's largest force component in
// the simulation (collected by the force kernels as an order-independent
// integer max of float bits), rounded to the nearest integer and added with
// an integer LDS atomic.  Integer addition is associative, so the
// per-cell sums are exact and identical whatever order the lanes and waves
// run in: bitwise reproducible without sorting.  Resolution max|F| 2^-kBits
// (below the rounding of one share in the compute precision); headroom 2^4
// (31 - 27, 63 - 58, 20 - 16) times max|F| per cell, while the delta kernel's
// partition of unity bounds a cell's sum by max|F| times the nodes per cell.
//
// Shares are rounded to the nearest integer, halves up (floor(v + 1/2), one
// instruction): the rounding is the same wherever a share is formed.
//
// FP32: three 32-bit sums per cell, one LDS atomic each at a common address
// (x, y and z planes of the field).
//
// FP16 storage: all three sums share one 64-bit word in 21-bit fields,
// z 2^42 + y 2^21 + x, with kBits = 16 (8 B per cell, for bricks twice as
// deep).  The resolution, 2^-16 of the step's largest force, is far below
// the binary16 rounding of the populations that the force feeds.
__device__ __forceinline__ int round_half_up(float v) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(v));
  return r;
}
template <typename R>
struct FixAcc;
template <>
struct FixAcc<float> {
  static constexpr int kBits = 27;
  static constexpr int kCells = kBrickThreads * brick_depth(kF32);
  struct Field {
    int32_t c[3][kCells];
  };
  __device__ static void clear(Field& f, int li) { f.c[0][li] = f.c[1][li] = f.c[2][li] = 0; }
  __device__ static void add(Field& f, int li, float gx, float gy, float gz) {
    atomicAdd(&f.c[0][li], round_half_up(gx));
    atomicAdd(&f.c[1][li], round_half_up(gy));
    atomicAdd(&f.c[2][li], round_half_up(gz));
  }
  __device__ static void get(const Field& f, int li, float inv, float& gx, float& gy, float& gz) {
    gx = (float)f.c[0][li] * inv;
    gy = (float)f.c[1][li] * inv;
    gz = (float)f.c[2][li] * inv;
  }
};
struct FixAcc3 {
  static constexpr int kBits = 16;
  static constexpr int kCells = kBrickThreads * brick_depth(kF16);
  static constexpr long long kF = 1LL << 21;  // field unit
  struct Field {
    long long xyz[kCells];
  };
  __device__ static void clear(Field& f, int li) { f.xyz[li] = 0; }
  __device__ static void add(Field& f, int li, float gx, float gy, float gz) {
    const long long w = (long long)round_half_up(gz) * (kF * kF) + (long long)round_half_up(gy) * kF +
                        (long long)round_half_up(gx);
    atomicAdd((unsigned long long*)&f.xyz[li], (unsigned long long)w);
  }
  // low 21 bits as a signed field
  __device__ static long long field(long long w) { return ((w & (kF - 1)) ^ (kF >> 1)) - (kF >> 1); }
  __device__ static void get(const Field& f, int li, float inv, float& gx, float& gy, float& gz) {
    long long w = f.xyz[li];
    const long long x = field(w);
    w = (w - x) / kF;  // exact: w - x is a multiple of 2^21
    const long long y = field(w);
    const long long z = (w - y) / kF;
    gx = (float)x * inv;
    gy = (float)y * inv;
    gz = (float)z * inv;
  }
};
template <>
struct FixAcc<double> {
  static constexpr int kBits = 58;
  static constexpr int kCells = kBrickThreads * brick_depth(kF64);
  struct Field {
    long long c[3][kCells];
  };
  __device__ static void clear(Field& f, int li) { f.c[0][li] = f.c[1][li] = f.c[2][li] = 0; }
  __device__ static void add(Field& f, int li, double gx, double gy, double gz) {
    atomicAdd((unsigned long long*)&f.c[0][li], (unsigned long long)__double2ll_rn(gx));
    atomicAdd((unsigned long long*)&f.c[1][li], (unsigned long long)__double2ll_rn(gy));
    atomicAdd((unsigned long long*)&f.c[2][li], (unsigned long long)__double2ll_rn(gz));
  }
  __device__ static void get(const Field& f, int li, double inv, double& gx, double& gy, double& gz) {
    gx = (double)f.c[0][li] * inv;
    gy = (double)f.c[1][li] * inv;
    gz = (double)f.c[2][li] * inv;
  }
};

// FP32 / FP16: registers capped for kLatticeWaves waves per SIMD (the
// spreading phase of one brick hides behind the streaming of the others)
#ifndef IBL_LATTICE_WAVES
#define IBL_LATTICE_WAVES 5
#endif
constexpr int kLatticeWaves = IBL_LATTICE_WAVES;
template <int ST>
__global__ __launch_bounds__(kBrickThreads, ST == kF64 ? 1 : kLatticeWaves) void k_lattice(const SimDev* __restrict__ sims,
                                                           Items it, int mode) {
  using T = typename Store<ST>::T;
  using R = RealOf<ST>;
  using D = typename Store<ST>::D;  // type of the collision's O(u) part
  using FA = typename std::conditional<ST == kF16, FixAcc3, FixAcc<R>>::type;
  constexpr int BZ = brick_depth(ST);
  static_assert(FA::kCells == kBrickThreads * BZ, "spread-force field of one brick");
  __shared__ typename FA::Field gq;
  // home-cube lists: the brick's home candidates (base cell inside the brick)
  // counted per cube (a brick meets at most 4 cubes: 64 x 4 -> 4 x 1,
  // 32 x 8 -> 2 x 1, 16 x 16 -> 1 x 2)
  __shared__ int hc[4], hb[4];
  __shared__ uint16_t hr[kCandCap];  // (local cube << 12) | rank, or 0xffff
  const int tid = threadIdx.x;
  for (int item = xcd_block(); item < it.lat_total; item += gridDim.x) {
    const int s = find_sim(it.lat_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= it.sub) continue;  // uniform over the workgroup
    const int64_t b = item - it.lat_off[s];
    int ox, oy, oz;
    brick_origin(S, b, ox, oy, oz);
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int bx = S.bs[0], by = S.bs[1], bz = S.bs[2];
    const int64_t stepn = *S.step + it.sub;
    const int par = (int)(stepn & 1);
    // ---- force spreading, Eq. (15): the brick's candidates, one per lane.
    // List buffer: without a skin always the first, rebuilt every step and
    // emptied once read.  With a skin: the one in use after the previous
    // step, or the other one when this step rebuilt the lists (an observation
    // always builds into the free buffer).
    int rb = 1, buf = 0;
    if (S.skin) {  // uniform
      const int4 lc4 = *(const GLB int4*)S.lctl;
      rb = mode == 1 ? 1 : (par ? lc4.w : lc4.z);
      buf = (par ? lc4.x : lc4.y) ^ rb;
    }
    const int64_t bl = buf * S.nbrick + b;
    int cnt = S.has_ib ? S.bcount[bl] : 0;
    const bool ib = cnt > 0;  // uniform
    R inv = (R)0;
    if (ib) {
      // one fixed-point scale per simulation and step: the sums do not depend
      // on which nodes share a brick
      const uint32_t fmx = S.fmax[par];
      if (tid == 0 && cnt > kCandCap) atomicOr((unsigned*)S.health, (uint32_t)kHOverflow);
      cnt = cnt > kCandCap ? kCandCap : cnt;
      const GLB NodeRec<R>* rec = (const GLB NodeRec<R>*)S.rec;
      const GLB int32_t* list = S.blist + bl * kCandCap;
      // this lane's first candidate, fetched before the field is cleared
      NodeRec<R> q;
      if (tid < cnt) q = *(const NodeRec<R>*)(rec + list[tid]);
#pragma unroll
      for (int k = 0; k < BZ; ++k) FA::clear(gq, tid + kBrickThreads * k);
      if (tid < 4) hc[tid] = 0;
      // cubes the brick meets: nlx along x by (at most 2) along y
      const int nlx = bx >> kCubeShift[0] > 0 ? bx >> kCubeShift[0] : 1;
      __syncthreads();
      int e2;
      frexpf(__uint_as_float(fmx), &e2);
      int sh = FA::kBits - e2;
      sh = sh > 120 ? 120 : sh;  // forces below ~1e-28: their shares round to zero
      const R sc = (R)ldexp(1.0, sh);
      inv = (R)ldexp(1.0, -sh);
      for (int i = tid; i < cnt; i += kBrickThreads) {
        if (i != tid) q = *(const NodeRec<R>*)(rec + list[i]);
        // a capsule's node is interpolated through its home cube's list (one
        // entry per node); a rigid body's node is spread only (its body moves
        // it); a node that is no longer valid is neither spread nor moved
        const bool val = q.valid != 0;
        uint16_t hrank = 0xffffu;
        if (q.valid == 1 && (unsigned)(q.base[0] - ox) < (unsigned)bx && (unsigned)(q.base[1] - oy) < (unsigned)by &&
            (unsigned)(q.base[2] - oz) < (unsigned)bz) {
          const int lc = (q.base[0] >> kCubeShift[0]) - (ox >> kCubeShift[0]) +
                         nlx * ((q.base[1] >> kCubeShift[1]) - (oy >> kCubeShift[1]));
          hrank = (uint16_t)((lc << 12) | atomicAdd(&hc[lc], 1));
        }
        hr[i] = hrank;
        int lx[4], ly[4], lz[4], mx, my, mz;
        axis_cells(q.base[0], ox, nx, S.wall[0], bx, lx, mx);
        axis_cells(q.base[1], oy, ny, S.wall[1], by, ly, my);
        axis_cells(q.base[2], oz, nz, S.wall[2], bz, lz, mz);
        if (!val) mz = 0;
        const R fx = q.F[0] * sc, fy = q.F[1] * sc, fz = q.F[2] * sc;
        R w3[3][4];
        rec_weights(q, S.delta, w3);
#pragma unroll
        for (int dz = 0; dz < 4; ++dz) {
          if (!((mz >> dz) & 1)) continue;
#pragma unroll
          for (int dy = 0; dy < 4; ++dy) {
            if (!((my >> dy) & 1)) continue;
            const R wyz = w3[1][dy] * w3[2][dz];
            const R gx = fx * wyz, gy = fy * wyz, gz = fz * wyz;
            const int row = bx * ly[dy] + kBrickThreads * lz[dz];
#pragma unroll
            for (int dx = 0; dx < 4; ++dx) {
              if (!((mx >> dx) & 1)) continue;
              const R wx = w3[0][dx];
              FA::add(gq, row + lx[dx], gx * wx, gy * wx, gz * wx);
            }
          }
        }
      }
      __syncthreads();
      // home cubes: one global reservation per (brick, cube), then the entries
      const int cube0 = (ox >> kCubeShift[0]) + S.nq[0] * ((oy >> kCubeShift[1]) + S.nq[1] * (oz >> kCubeShift[2]));
      if (tid < 4 && hc[tid] > 0)
        hb[tid] = atomicAdd((int*)&S.hcount[cube0 + tid % nlx + S.nq[0] * (tid / nlx)], hc[tid]);
      __syncthreads();
      for (int i = tid; i < cnt; i += blockDim.x) {
        const uint16_t v = hr[i];
        if (v == 0xffffu) continue;
        const int lc = v >> 12, pos = hb[lc] + (v & 0xfff);
        const int cube = cube0 + lc % nlx + S.nq[0] * (lc / nlx);
        if (pos < kHomeCap) S.hlist[(int64_t)cube * kHomeCap + pos] = list[i];
      }
    }
    if (S.has_ib && tid == 0) {
      // lists rebuilt every step and an observation's lists are dropped once
      // read; after a rebuild the retired buffer becomes the (empty) free one
      if (mode == 1 || S.skin == 0) S.bcount[bl] = 0;
      else if (rb) S.bcount[(buf ^ 1) * S.nbrick + b] = 0;
      if (b == 0) {
        if (mode == 0) S.lctl[par] = buf;
        S.fmax[par ^ 1] = 0u;  // the next step's maximum starts from zero
      }
    }
    // ---- collide-stream, a column of BZ cells per thread
    const int x = ox + (tid & (bx - 1)), y = oy + (tid >> S.bsh[0]);
    uint32_t bad = 0u;  // health bits of this thread's cells
    if (x < nx && y < ny) {
      const int64_t nc = S.ncell;
      const uint32_t salt = (uint32_t)stepn * 0x85EBCA77u + 0x165667B1u;
      const GLB T* src = (const GLB T*)S.f[par];
      GLB T* dst = (GLB T*)S.f[par ^ 1];
      GLB R* uf = (GLB R*)S.u;  // [3][ncell]
#pragma unroll 1
      for (int k = 0; k < BZ; ++k) {
        const int z = oz + k;
        if (z >= nz) break;
        const int64_t cell = x + (int64_t)nx * (y + (int64_t)ny * z);
        const int li = tid + kBrickThreads * k;
        if (solid_cell(S, x, y, z)) {
          if (mode == 1) {
            ((GLB R*)S.rho)[cell] = (R)0;
            GLB R* gf = (GLB R*)S.g;
            gf[cell] = gf[nc + cell] = gf[2 * nc + cell] = (R)0;
          }
          continue;
        }
        // the populations in their stored units, kS h (kS = 2^16 for FP16,
        // else 1): the collision below works in them, with its weights scaled
        // by kS and the moments unscaled once (a power-of-two scale commutes
        // with every rounding, so this is bitwise the unscaled arithmetic)
        constexpr double kS = Store<ST>::kScale;
        auto wqs = [](int q) { return wq(q) * kS; };
        R h[kQ];
        pull_cell<ST, true>(S, src, x, y, z, cell, h);
        // moments, Eq. (3), in type D (FP64 for FP64 / FP32 storage: exact sums
        // of the stored values): rho = sum f = 1 + sum h ; J = rho u = sum h c + g/2
        D drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const D hq = (D)h[q];
          drho += hq;
          if (kCx[q]) jx += kCx[q] > 0 ? hq : -hq;
          if (kCy[q]) jy += kCy[q] > 0 ? hq : -hq;
          if (kCz[q]) jz += kCz[q] > 0 ? hq : -hq;
        }
        if constexpr (kS != 1.0) {
          const D is = (D)(1.0 / kS);
          drho *= is;
          jx *= is;
          jy *= is;
          jz *= is;
        }
        R gix = (R)0, giy = (R)0, giz = (R)0;  // spread force g_IB
        if (ib) FA::get(gq, li, inv, gix, giy, giz);
        const D gx = (D)S.gb[0] + (D)gix, gy = (D)S.gb[1] + (D)giy, gz = (D)S.gb[2] + (D)giz;
        const D Jx = fma((D)0.5, gx, jx), Jy = fma((D)0.5, gy, jy), Jz = fma((D)0.5, gz, jz);
        const D rho = (D)1 + drho;
        // velocity in the compute type R (FP32, or FP64 for FP64 storage)
        const R rr = (R)rho;
        const R ir = rcp_r(rr);
        const R ux = (R)Jx * ir, uy = (R)Jy * ir, uz = (R)Jz * ir;
        const R usq = fma(uz, uz, fma(uy, uy, ux * ux));
        // health, per cell: non-finite populations, rho <= 0, |u| > 0.3
        bad |= !isfinite(drho) ? (uint32_t)kHNonfiniteF
                               : (!(rho > (D)0) ? (uint32_t)kHRho : (!(usq <= (R)0.09) ? (uint32_t)kHMach : 0u));
        if (mode == 1) {
          ((GLB R*)S.rho)[cell] = rr;
          uf[cell] = ux;
          uf[nc + cell] = uy;
          uf[2 * nc + cell] = uz;
          GLB R* gf = (GLB R*)S.g;
          gf[cell] = gix;
          gf[nc + cell] = giy;
          gf[2 * nc + cell] = giz;
          continue;
        }
        if (S.has_ib) {
          uf[cell] = ux;
          uf[nc + cell] = uy;
          uf[2 * nc + cell] = uz;
        }
        // BGK collision toward f_eq of Eq. (2) with the forcing term of Eq. (4),
        // in offset form, h* = (1 - om) h + om (f_eq - w) + F, split by size:
        //   L_q = (1 - om) h_q + om w_q (drho + 3 c_q . J)                 (type D)
        //   N_q = w_q [om rho (9/2 (c_q . u)^2 - 3/2 u^2)
        //              + pre (3 (c_q . g - u . g) + 9 (c_q . u)(c_q . g))]  (type R)
        // For FP32 storage L is FP64: it carries the O(1e-3) part, whose FP32
        // rounding would recur every step in a steady flow and bias it; N is
        // O(u^2, g), where FP32 rounding is far below FP32 storage.  FP16
        // storage computes both in FP32 (its stochastic rounding noise is four
        // orders above that bias), FP64 storage both in FP64.
        // Directions 2k-1 and 2k are opposite (c -> -c): N's even part
        // w_q [(c.u)(9/2 om rho (c.u) + 9 pre (c.g)) + C0] is shared and its odd
        // part 3 pre w_q (c.g) changes sign, as does L's 3 om w_q c.J.
        const R gxr = (R)gx, gyr = (R)gy, gzr = (R)gz;
        const R omr = (R)S.om * rr, prer = (R)S.pre;
        const R k45 = (R)4.5 * omr, k9 = (R)9 * prer, k3 = (R)3 * prer;
        const R C0 = -fma((R)1.5 * omr, usq, k3 * fma(uz, gzr, fma(uy, gyr, ux * gxr)));
        const D omd = (D)S.om * drho, om3 = (D)S.a0, om1 = (D)S.om1;
        // random bits of the stochastic rounding: a hash of (cell, step), then
        // one xorshift step per pair of directions (16 bits each)
        uint32_t rs = (uint32_t)cell * 0x9E3779B1u + salt;
        rs ^= rs >> 16;  // integer finaliser of the "lowbias32" family (Wellons)
        rs *= 0x7feb352du;
        rs ^= rs >> 15;
        rs *= 0x846ca68bu;
        rs ^= rs >> 16;
        rs |= 1u;  // a non-zero xorshift state
        // collision and stores (a moving wall's term is added to the slots
        // next to it afterwards, by k_wall_slots)
        {
          uint32_t r = rs;
          // uniform plane base plus a 32-bit byte offset (as for the loads)
          auto store = [&](int q, D v, uint32_t r16) {
            GLB T* at = (GLB T*)((GLB char*)(dst + (int64_t)q * nc) + (uint32_t)cell * (uint32_t)sizeof(T));
            Store<ST>::put_raw_sr(at, v, r16);
          };
          store(0, fma(om1, (D)h[0], (D)wqs(0) * omd + (D)((R)wqs(0) * C0)), r);
#pragma unroll
          for (int q = 1; q < kQ; q += 2) {
            // c_q . v for c_q with components in {-1, 0, 1}: sums and differences only
            auto cdot = [q](auto vx, auto vy, auto vz) {
              decltype(vx) d = 0;
              if (kCx[q]) d = kCx[q] > 0 ? vx : -vx;
              if (kCy[q]) d = kCy[q] > 0 ? d + vy : d - vy;
              if (kCz[q]) d = kCz[q] > 0 ? d + vz : d - vz;
              return d;
            };
            const R cu = cdot(ux, uy, uz), cg = cdot(gxr, gyr, gzr);
            const D E = (D)wqs(q) * omd, O = ((D)wqs(q) * om3) * cdot(Jx, Jy, Jz);
            const R Ne = (R)wqs(q) * fma(cu, fma(k45, cu, k9 * cg), C0), No = ((R)wqs(q) * k3) * cg;
            r ^= r << 13;
            r ^= r >> 17;
            r ^= r << 5;
            store(q, fma(om1, (D)h[q], (E + O) + (D)(Ne + No)), r);
            store(q + 1, fma(om1, (D)h[q + 1], (E - O) + (D)(Ne - No)), r >> 16);
          }
        }
      }
    }
    // latch this wave's health bits (one atomic per wave, only when some cell is bad)
    if (__any(bad != 0u)) {
      for (int o = 32; o > 0; o >>= 1) bad |= (uint32_t)__shfl_xor((int)bad, o);
      if ((tid & 63) == 0) atomicOr((unsigned*)S.health, bad);
    }
    if (ib) __syncthreads();  // the next brick clears the field
  }
}

// ---------------------------------------------------------- moving walls --
// Halfway bounce-back off a moving wall adds 6 w_i rho_w (c_i . u_wall) to the
// population a fluid cell reflects.  The cell reads that population from its
// own stored slot q (where x + c_q is a wall layer; it returns as opp(q)), so
// the term is added to the slot once collide-stream has stored it: only the
// cells of the layers next to the walls, each slot once (a slot meets exactly
// one wall layer: the first wall axis of x, y, z that x + c_q crosses), in
// the storage's arithmetic with a stochastically rounded store (random bits
// from (cell, step, slot), a hash apart from the collision's).
// Grid: x strides over a simulation's wall planes, y is the simulation.
template <int ST>
__global__ __launch_bounds__(256) void k_wall_slots(const SimDev* __restrict__ sims, Items it) {
  using T = typename Store<ST>::T;
  using D = typename Store<ST>::D;
  constexpr double kS = Store<ST>::kScale;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)gridDim.x * blockDim.x;
  for (int si = blockIdx.y; si < it.nsim; si += gridDim.y) {
    const SimDev& S = sims[si];
    if (*S.remaining <= it.sub) continue;  // uniform
    const int64_t stepn = *S.step + it.sub;
    GLB T* dst = (GLB T*)S.f[(int)(stepn & 1) ^ 1];
    const int64_t nc = S.ncell;
    const int n[3] = {S.n[0], S.n[1], S.n[2]};
    for (int a = 0; a < 3; ++a) {
      if (!S.wall[a]) continue;  // uniform
      const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;  // the plane's axes
      const int64_t plane = (int64_t)n[b] * n[c];
      for (int side = 0; side < 2; ++side) {
        const int layer = 2 * a + side;
        if (!((S.wall_moving >> layer) & 1u)) continue;  // uniform: this wall does not move
        for (int64_t k = t0; k < plane; k += nt) {
          int cc[3];
          cc[a] = side ? n[a] - 2 : 1;
          cc[b] = (int)(k % n[b]);
          cc[c] = (int)(k / n[b]);
          const int x = cc[0], y = cc[1], z = cc[2];
          if (solid_cell(S, x, y, z)) continue;
          const int64_t cell = x + (int64_t)n[0] * (y + (int64_t)n[1] * z);
          const int want = side ? 1 : -1;  // c_q along a pointing into this wall
#pragma unroll
          for (int q = 1; q < kQ; ++q) {
            if ((a == 0 ? kCx[q] : (a == 1 ? kCy[q] : kCz[q])) != want) continue;
            int lq;  // the wall layer this slot meets (the first wall axis)
            (void)pull_source(S, opp(q), x, y, z, (int)cell, lq);
            if (lq != layer) continue;
            GLB T* at = dst + (int64_t)q * nc + cell;
            uint32_t r = (uint32_t)cell * 0x2C1B3C6Du + (uint32_t)stepn * 0x297A2D39u + (uint32_t)q * 0x9E3779B1u;
            r ^= r >> 16;
            r *= 0x7feb352du;
            r ^= r >> 15;
            r *= 0x846ca68bu;
            r ^= r >> 16;
            const D v = (D)Store<ST>::h_raw(at) + (D)(S.bbw[opp(q)][layer] * kS);
            Store<ST>::put_raw_sr(at, v, r);
          }
        }
      }
    }
  }
}

// -------------------------------------------------------------- advance --
// after a sequence of `steps` timesteps: each simulation ran min(remaining, steps)
__global__ void k_advance(const SimDev* __restrict__ sims, int nsim, int steps) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsim) return;
  const SimDev& S = sims[s];
  const int64_t r = *S.remaining, k = r < steps ? r : (int64_t)steps;
  if (k > 0) {
    *S.step += k;
    *S.remaining = r - k;
  }
}

// -------------------------------------------------------------- reduce --
template <int ST>
__global__ __launch_bounds__(256) void k_reduce(const SimDev* __restrict__ sims, Items it) {
  using T = typename Store<ST>::T;
  __shared__ double sh[4][256];
  for (int item = xcd_block(); item < it.red_total; item += gridDim.x) {
    const int s = find_sim(it.red_off, it.nsim, item);
    const SimDev& S = sims[s];
    const int64_t c0 = (int64_t)(item - it.red_off[s]) * kReduceItemCells;
    const int par = (int)(*S.step & 1);
    const GLB T* f = (const GLB T*)S.f[par];
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
      RealOf<ST> hp[kQ];
      pull_cell<ST>(S, f, x, y, z, cell, hp);
      for (int q = 0; q < kQ; ++q) {
        const double hq = (double)hp[q];
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
    if (bad) atomicOr((unsigned*)S.health, bad);
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

// grid for a grid-stride loop over `items`, a multiple of kXcds (see xcd_block)
int grid_for(int items, int cap) {
  const int g = items < cap ? items : cap;
  return (g + kXcds - 1) / kXcds * kXcds;
}

}  // namespace

// ------------------------------------------------------------ launchers --
hipError_t launch_init(int storage, const SimDev* sims, const Items& it, int profile, hipStream_t s) {
  if (it.lat_total <= 0) return hipSuccess;
  const int grid = grid_for(it.lat_total, 1 << 20);
  if (storage == kF64) hipLaunchKernelGGL(k_init<kF64>, dim3(grid), dim3(kBrickThreads), 0, s, sims, it, profile);
  else if (storage == kF32) hipLaunchKernelGGL(k_init<kF32>, dim3(grid), dim3(kBrickThreads), 0, s, sims, it, profile);
  else hipLaunchKernelGGL(k_init<kF16>, dim3(grid), dim3(kBrickThreads), 0, s, sims, it, profile);
  return hipGetLastError();
}

hipError_t launch_reset_lists(const SimDev* sim, int64_t nbrick, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_lists, dim3((unsigned)((nbrick + 255) / 256)), dim3(256), 0, s, sim);
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
  switch (phase) {
    case kPhaseForces:
      launch_forces(ST, sims, it, mode, s);
      break;
    case kPhaseLattice:
      hipLaunchKernelGGL((k_lattice<ST>), dim3(grid_for(it.lat_total, 1 << 22)), dim3(kBrickThreads), 0, s, sims,
                         it, mode);
      if (it.moving_walls && mode == 0)
        hipLaunchKernelGGL((k_wall_slots<ST>), dim3((it.wall_cells + 255) / 256, it.nsim < 65535 ? it.nsim : 65535),
                           dim3(256), 0, s, sims, it);
      break;
    case kPhaseInterp:
      launch_interp(ST, sims, it, mode, s);
      break;
    case kPhaseAdvance:
      if (mode == 0) hipLaunchKernelGGL(k_advance, dim3((it.nsim + 63) / 64), dim3(64), 0, s, sims, it.nsim, 1);
      break;
  }
}

hipError_t launch_phase(int storage, const SimDev* sims, const Items& it, int phase, int mode, hipStream_t s) {
  if (storage == kF64) phase_impl<kF64>(sims, it, phase, mode, s);
  else if (storage == kF32) phase_impl<kF32>(sims, it, phase, mode, s);
  else phase_impl<kF16>(sims, it, phase, mode, s);
  return hipGetLastError();
}

hipError_t launch_steps(int storage, const SimDev* sims, const Items& it, int steps, int mode, hipStream_t s) {
  for (int k = 0; k < steps; ++k) {
    Items ik = it;
    ik.sub = k;
    for (int ph = 0; ph < kPhaseAdvance; ++ph) {
      hipError_t e = launch_phase(storage, sims, ik, ph, mode, s);
      if (e != hipSuccess) return e;
    }
  }
  if (mode == 0) hipLaunchKernelGGL(k_advance, dim3((it.nsim + 63) / 64), dim3(64), 0, s, sims, it.nsim, steps);
  return hipGetLastError();
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
