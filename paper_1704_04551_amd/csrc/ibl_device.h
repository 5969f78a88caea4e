// Device-side helpers shared by the lattice and immersed-boundary kernels.
#pragma once

#include <hip/hip_fp16.h>
#include <math.h>

#include "ibl_internal.h"

#if defined(__HIP_DEVICE_COMPILE__)
#define GLB __attribute__((address_space(1)))
#else
#define GLB
#endif

namespace ibl {
namespace {

// ---------------------------------------------------------------- storage --
// Every storage mode keeps the offset h_i = f_i - w_i (the equilibrium at rest
// subtracted): at low Mach number f_i differs from w_i only in its low bits,
// and a body-force increment of 1e-6 added to f_i ~ 0.05 would lose most of
// its bits in binary32.  Offsets keep them.  FP16 stores 2^16 h_i as binary16
// (see Store<kF16>), FP32 h_i as binary32, FP64 h_i as binary64.
//
// The timestep forms each post-collision value (its O(u) part in FP64 for FP32
// storage, see k_lattice) and stores it with stochastic rounding to the
// storage format.  In a steady or
// slowly varying flow the same populations recur step after step, so a
// deterministic rounding error -- of FP32 arithmetic, or of a round-to-nearest
// store -- is the same every step and acts as a spurious force: about one
// binary32 ulp of h (1e-10) against per-step force increments of about 1e-7.
// Rounding up with probability equal to the discarded fraction makes each
// store unbiased.  The random bits come from a hash of (cell, step), so runs
// stay bitwise reproducible.
//
// The rounding works on the bit pattern of the computed value: random bits are
// added just below the last bit the target format keeps, and the bits below
// it are cleared; the carry rounds the magnitude up with probability equal to
// the discarded fraction (to within 2^-16 of an ulp for FP32 storage, 2^-13
// for FP16), for either sign.  The result has the target's significand width
// and converts exactly.  (Below the target's normal range the conversion then
// rounds to nearest.)
//
// A step reads each stored population once and writes each once, and the
// next read comes a whole step later, after more traffic than the caches
// hold: the timestep's population loads and stores are non-temporal, so the
// caches keep what is re-read within the step (the velocity tiles of the
// interpolation, the spreading records and candidate lists).

// Stochastic rounding of v to `keep` significand bits (52 - drop), given 16
// uniform random bits r16 (the low 16 bits of the argument).
template <int kDrop>
__device__ __forceinline__ double sr_truncate(double v, uint32_t r16) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t t = (b + ((uint64_t)(r16 & 0xffffu) << (kDrop - 16))) & ~((1ull << kDrop) - 1ull);
  return __longlong_as_double((long long)t);
}

template <int ST>
struct Store;
template <>
struct Store<kF64> {
  using T = double;
  using R = double;
  using D = double;
  __device__ static R h(const GLB T* p, int64_t i, int) { return __builtin_nontemporal_load(p + i); }
  __device__ static void put(GLB T* p, int64_t i, int, R hq) { p[i] = hq; }
  __device__ static void put_sr(GLB T* p, double v, uint32_t) { __builtin_nontemporal_store(v, p); }
  __device__ static double hd(const GLB T* p, int64_t i, int) { return p[i]; }
  // the stored value's own units (the same as h's here)
  static constexpr double kScale = 1.0;
  __device__ static R h_raw(const GLB T* p) { return __builtin_nontemporal_load(p); }
  __device__ static void put_raw_sr(GLB T* p, double v, uint32_t r16) { put_sr(p, v, r16); }
};
template <>
struct Store<kF32> {
  using T = float;
  using R = float;
  using D = double;
  __device__ static R h(const GLB T* p, int64_t i, int) { return __builtin_nontemporal_load(p + i); }
  __device__ static void put(GLB T* p, int64_t i, int, R hq) { p[i] = hq; }
  // binary32 keeps 23 of the 52 fraction bits
  __device__ static void put_sr(GLB T* p, double v, uint32_t r16) {
    __builtin_nontemporal_store((float)sr_truncate<29>(v, r16), p);
  }
  __device__ static double hd(const GLB T* p, int64_t i, int) { return (double)p[i]; }
  static constexpr double kScale = 1.0;
  __device__ static R h_raw(const GLB T* p) { return __builtin_nontemporal_load(p); }
  __device__ static void put_raw_sr(GLB T* p, double v, uint32_t r16) { put_sr(p, v, r16); }
};
// binary16 holds 2^16 h_i: a power-of-two scale (exact) that moves the
// binary16 normal range, [2^-14, 65504], to offsets in [2^-30, 0.9995]
// (|h_i| stays below 0.1 at the Mach bound of 0.3), so the small offsets of a
// slow or resting flow keep the full 11-bit significand instead of the
// subnormals' fixed 2^-24 spacing.
constexpr double kF16Scale = 0x1p16;
template <>
struct Store<kF16> {
  using T = __half;
  using R = float;
  using D = float;
  // binary16 moved as its 16 bits
  __device__ static R h(const GLB T* p, int64_t i, int) {
    return __half2float(__ushort_as_half(__builtin_nontemporal_load((const GLB unsigned short*)p + i))) *
           (float)(1.0 / kF16Scale);
  }
  __device__ static void put(GLB T* p, int64_t i, int, R hq) {
    ((GLB unsigned short*)p)[i] = __half_as_ushort(__float2half_rn((float)((double)hq * kF16Scale)));
  }
  // binary16 keeps 10 of binary32's 23 fraction bits: 13 random bits are added
  // below the last kept bit and the 13 bits cleared (on the FP32 bit pattern,
  // as sr_truncate does on FP64)
  __device__ static void put_sr(GLB T* p, float v, uint32_t r16) { put_raw_sr(p, v * (float)kF16Scale, r16); }
  __device__ static double hd(const GLB T* p, int64_t i, int) { return (double)h(p, i, 0); }
  // in the stored units, 2^16 h (the collide-stream kernel works in them:
  // scaling by a power of two commutes with every rounding, so its results
  // are those of scaling each load and store)
  static constexpr double kScale = kF16Scale;
  __device__ static R h_raw(const GLB T* p) {
    return __half2float(__ushort_as_half(__builtin_nontemporal_load((const GLB unsigned short*)p)));
  }
  __device__ static void put_raw_sr(GLB T* p, float v, uint32_t r16) {
    const uint32_t b = __float_as_uint(v);
    const float o = __uint_as_float((b + (r16 & 0x1fffu)) & ~0x1fffu);
    __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(o)), (GLB unsigned short*)p);
  }
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

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Renumber blocks so that the blocks of one XCD take a contiguous range of
// work items (neighbouring bricks / nodes of one capsule share an L2).
// Launches round the grid up to a multiple of kXcds.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block() {
  const int per = (int)gridDim.x / kXcds;
  return (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
}

// Origin (first cell) of brick b.
__device__ __forceinline__ void brick_origin(const SimDev& S, int64_t b, int& ox, int& oy, int& oz) {
  const int64_t r = b / S.nb[0];
  ox = (int)(b - r * S.nb[0]) << S.bsh[0];
  oy = (int)(r % S.nb[1]) << S.bsh[1];
  oz = (int)(r / S.nb[1]) << S.bsh[2];
}

// The four stencil cells from `base` along one axis, relative to the brick
// origin o (periodic images folded in), and the mask of those inside the
// brick (0 <= l < size).
__device__ __forceinline__ void axis_cells(int base, int o, int n, int wall, int size, int l[4], int& mask) {
  mask = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int c = base - 1 + k;
    if (!wall) c = c < 0 ? c + n : (c >= n ? c - n : c);
    l[k] = c - o;
    mask |= ((unsigned)l[k] < (unsigned)size) ? (1 << k) : 0;
  }
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

// Forces of one edge's energy 1/2 ks (l - l0)^2 + kb (1 - cos(theta - theta0))
// on its four vertices: G0 on v0, G3 on v3, F1 on v1; v2 receives
// -(G0 + G3 + F1) since the edge's forces sum to zero.  Same gradient as
// bend_force, evaluated once for all four roles.
__device__ __forceinline__ void edge_forces(D3 v0, D3 v1, D3 v2, D3 v3, double l0, double c0,
                                            double s0, double ks, double kb, D3& G0, D3& G3,
                                            D3& F1) {
  // three reciprocals and two square roots per edge (FP64 division is a long
  // instruction sequence); the rest are products
  const D3 e = sub(v2, v1);
  const double e2 = dot(e, e), le = sqrt(e2), rle = 1.0 / le, re2 = rle * rle;
  F1 = scale(e, ks * (le - l0) * rle);  // spring pulls v1 toward v2 when stretched
  G0 = {0.0, 0.0, 0.0};
  G3 = {0.0, 0.0, 0.0};
  if (kb != 0.0) {
    const D3 a = sub(v0, v1);
    const D3 nA = cross(e, a);
    const D3 nB = cross(sub(v3, v2), e);
    const double rA = 1.0 / dot(nA, nA), rB = 1.0 / dot(nB, nB);
    const double inv = sqrt(rA * rB);  // 1 / (|nA| |nB|)
    const double ct = dot(nA, nB) * inv;
    const double st = dot(cross(nA, nB), e) * inv * rle;
    const double dEdth = kb * (st * c0 - ct * s0);  // kb sin(theta - theta0)
    G0 = scale(nA, dEdth * le * rA);
    G3 = scale(nB, dEdth * le * rB);
    const double t0 = dot(a, e) * re2;
    const double t3 = dot(sub(v3, v1), e) * re2;
    F1.x += (t0 - 1.0) * G0.x + (t3 - 1.0) * G3.x;
    F1.y += (t0 - 1.0) * G0.y + (t3 - 1.0) * G3.y;
    F1.z += (t0 - 1.0) * G0.z + (t3 - 1.0) * G3.z;
  }
}

// delta_weights in the precision of the spreading record
template <typename R>
__device__ __forceinline__ void delta_weights_r(int kind, R d, R w[4]);
template <>
__device__ __forceinline__ void delta_weights_r<double>(int kind, double d, double w[4]) {
  delta_weights(kind, d, w);
}
// sin and cos of t = pi d / 2 for 0 <= d <= 1 from their Taylor series about
// 0, through t^11 and t^12: truncation below 6e-8 and 7e-9 on [0, pi/2];
// evaluated in float, within 2e-7 of the exact values.  A general sincosf
// carries range reduction this argument never needs.
__device__ __forceinline__ void sincos_quarter(float d, float& s, float& c) {
  const float t = 1.5707963267948966f * d, u = t * t;
  s = t * (1.0f + u * (-1.0f / 6 + u * (1.0f / 120 + u * (-1.0f / 5040 + u * (1.0f / 362880 +
                                                                                   u * (-1.0f / 39916800))))));
  c = 1.0f + u * (-0.5f + u * (1.0f / 24 + u * (-1.0f / 720 + u * (1.0f / 40320 + u * (-1.0f / 3628800 +
                                                                                      u * (1.0f / 479001600))))));
}

template <>
__device__ __forceinline__ void delta_weights_r<float>(int kind, float d, float w[4]) {
  if (kind == kCos) {
    float s, c;
    sincos_quarter(d, s, c);
    w[0] = 0.25f * (1.0f - s);
    w[1] = 0.25f * (1.0f + c);
    w[2] = 0.25f * (1.0f + s);
    w[3] = 0.25f * (1.0f - c);
  } else {
    const float q = sqrtf(fmaxf(1.0f + 4.0f * d - 4.0f * d * d, 0.0f));
    w[0] = (3.0f - 2.0f * d - q) * 0.125f;
    w[1] = (3.0f - 2.0f * d + q) * 0.125f;
    w[2] = (1.0f + 2.0f * d + q) * 0.125f;
    w[3] = (1.0f + 2.0f * d - q) * 0.125f;
  }
}

// The 12 delta weights of a spreading record (stored, or evaluated from the
// fractional offsets with the same function that the force kernel used).
__device__ __forceinline__ void rec_weights(const NodeRec<double>& q, int kind, double w[3][4]) {
  (void)kind;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 4; ++k) w[a][k] = q.w[a][k];
}
__device__ __forceinline__ void rec_weights(const NodeRec<float>& q, int kind, float w[3][4]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) delta_weights_r<float>(kind, q.d[a], w[a]);
}


// Both list buffers empty (buffer 0 in use), both step parities marked to
// rebuild, no force maximum recorded.
__device__ __forceinline__ void reset_list_control(const SimDev& S) {
  S.lctl[0] = S.lctl[1] = 0;
  S.lctl[2] = S.lctl[3] = 1;
  S.fmax[0] = S.fmax[1] = 0u;
}

__device__ __forceinline__ bool solid_cell(const SimDev& S, int x, int y, int z) {
  return (S.wall[0] && (x == 0 || x == S.n[0] - 1)) || (S.wall[1] && (y == 0 || y == S.n[1] - 1)) ||
         (S.wall[2] && (z == 0 || z == S.n[2] - 1));
}

// -------------------------------------------------------------- streaming --
// The populations are stored post-collision (f* of the previous step) and
// streamed on read ("pull"): f_q(x) = f*_q(x - c_q).  Where x - c_q is a wall
// layer, halfway bounce-back returns the cell's own opposite population with
// the moving-wall term: f_q(x) = f*_opp(q)(x) + 6 w_q (c_q . u_wall), u_wall
// the velocity of the first wall axis (x, y, z order) whose layer x - c_q is.
// The slot f*_opp(q)(x) of such a link is read by that bounce-back only (its
// streaming neighbour is solid), so the collision stores it with the wall term
// already added, in FP64 before the one rounding to the storage format; the
// pull then reads every population as stored.  Writes are aligned (each cell
// writes its own populations); only the reads are shifted.

// Source of direction q for fluid cell (x, y, z): the element index of the
// value to read, and the bounce-back wall layer (2 * axis + [hi side]) or -1.
// Cell indices fit in 32 bits (the descriptor check bounds the lattice).
__device__ __forceinline__ int pull_source(const SimDev& S, int q, int x, int y, int z, int cell, int& layer) {
  const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
  const int xs = x - kCx[q], ys = y - kCy[q], zs = z - kCz[q];
  const int sy = nx, sz = nx * ny;
  int sc = cell - kCx[q] - sy * kCy[q] - sz * kCz[q];
  // periodic wrap: one axis length in index units (nx, nx ny, nx ny nz)
  if (kCx[q] && !S.wall[0]) sc += xs < 0 ? nx : (xs >= nx ? -nx : 0);
  if (kCy[q] && !S.wall[1]) sc += ys < 0 ? sz : (ys >= ny ? -sz : 0);
  if (kCz[q] && !S.wall[2]) sc += zs < 0 ? (int)S.ncell : (zs >= nz ? -(int)S.ncell : 0);
  const bool bx = kCx[q] && S.wall[0] && (xs == 0 || xs == nx - 1);
  const bool by = kCy[q] && S.wall[1] && (ys == 0 || ys == ny - 1);
  const bool bz = kCz[q] && S.wall[2] && (zs == 0 || zs == nz - 1);
  layer = bx ? (xs != 0) : (by ? 2 + (ys != 0) : (bz ? 4 + (zs != 0) : -1));
  return layer >= 0 ? cell : sc;
}

// The 19 pulled populations of fluid cell (x, y, z) in the storage's compute
// type (bounce-back links include their wall term, see above).
// kRaw: the values in their stored units (Store<ST>::kScale h)
template <int ST, bool kRaw = false>
__device__ __forceinline__ void pull_cell(const SimDev& S, const GLB typename Store<ST>::T* src, int x, int y,
                                          int z, int64_t cell, RealOf<ST> h[kQ]) {
  using T = typename Store<ST>::T;
  const int64_t nc = S.ncell;
  // branch-free addresses, so the 19 loads issue together.  Each load is a
  // uniform base (population min(q, opp q)) plus a 32-bit byte offset: the
  // descriptor check keeps 2 ncell elements below 2^32 bytes.
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    int layer;
    const int sc = pull_source(S, q, x, y, z, (int)cell, layer);
    const int plo = q < opp(q) ? q : opp(q);
    const uint32_t el = (uint32_t)(((layer >= 0 ? opp(q) : q) - plo) * (int)nc + sc);
    const GLB char* base = (const GLB char*)(src + (int64_t)plo * nc);
    const GLB T* at = (const GLB T*)(base + el * (uint32_t)sizeof(T));
    h[q] = kRaw ? Store<ST>::h_raw(at) : Store<ST>::h(at, 0, q);
  }
}

}  // namespace
}  // namespace ibl
