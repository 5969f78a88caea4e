// gfx950 kernels of the coupled IB-LBM timestep (libibl.so).
//
// Per timestep, on one stream:
//   k_forces   membrane forces, spreading records, candidate lists (ibl_ib.hip)
//   k_spread   force spreading into the per-cell force field (ibl_ib.hip)
//   k_lattice  one thread per cell: moments with the half-force shift
//              (Eq. (3)), BGK collision with the forcing term (Eq. (1), (2),
//              (4)), push streaming into the other A/B copy with periodic wrap
//              and halfway bounce-back (moving-wall term); u^n is written for
//              the interpolation.
//   k_interp   velocity interpolation and node update (ibl_ib.hip)
//   k_advance  per simulation: step counter (A/B parity) and remaining steps.
// Every kernel walks a flattened (simulation, work item) list, so one launch
// serves a single simulation or a batch of uneven ones.
#include "ibl_device.h"

namespace ibl {
namespace {

__device__ __forceinline__ bool lat_cell(const SimDev& S, int local_item, int tid, int& x, int& y,
                                         int& z) {
  // a work item is kLatticeBlock consecutive cells in memory order; the item's
  // first cell is split once (uniform), each thread then walks forward
  const int64_t c0 = (int64_t)local_item * kLatticeBlock;
  if (c0 + tid >= S.ncell) return false;
  const int nx = S.n[0], ny = S.n[1];
  int x0 = (int)(c0 % nx);
  const int64_t r0 = c0 / nx;
  y = (int)(r0 % ny);
  z = (int)(r0 / ny);
  x = x0 + tid;
  while (x >= nx) {
    x -= nx;
    if (++y == ny) {
      y = 0;
      ++z;
    }
  }
  return true;
}

// ------------------------------------------------------------------ init --
template <int ST>
__global__ __launch_bounds__(kLatticeBlock) void k_init(const SimDev* __restrict__ sims, Items it,
                                                        int profile) {
  using T = typename Store<ST>::T;
  using R = RealOf<ST>;
  for (int item = xcd_block(); item < it.lat_total; item += gridDim.x) {
    const int s = find_sim(it.lat_off, it.nsim, item);
    const SimDev& S = sims[s];
    int x, y, z;
    if (!lat_cell(S, item - it.lat_off[s], threadIdx.x, x, y, z)) continue;
    const int64_t cell = x + (int64_t)S.n[0] * (y + (int64_t)S.n[1] * z);
    if (cell < S.nbrick) {
      S.bcount[cell] = 0;
      S.bmax[cell] = 0u;
    }
    if (cell == 0) {  // every control word: the arena may hold a previous user's data
      *S.step = 0;
      *S.remaining = 0;
      *S.health = 0u;
    }
    const int c[3] = {x, y, z};
    GLB R4<R>* u = (GLB R4<R>*)S.u;
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
      *(R4<R>*)(u + cell) = R4<R>{(R)v[0], (R)v[1], (R)v[2], (R)0};
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
    *(R4<R>*)(u + cell) = R4<R>{(R)u0[0], (R)u0[1], (R)u0[2], (R)0};
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
template <int ST>
__global__ __launch_bounds__(kLatticeBlock) void k_lattice(const SimDev* __restrict__ sims,
                                                           Items it, int mode) {
  using T = typename Store<ST>::T;
  using R = RealOf<ST>;
  for (int item = xcd_block(); item < it.lat_total; item += gridDim.x) {
    const int s = find_sim(it.lat_off, it.nsim, item);
    const SimDev& S = sims[s];
    if (mode == 0 && *S.remaining <= 0) continue;
    int x, y, z;
    if (!lat_cell(S, item - it.lat_off[s], threadIdx.x, x, y, z)) continue;
    const int nx = S.n[0], ny = S.n[1], nz = S.n[2];
    const int64_t cell = x + (int64_t)nx * (y + (int64_t)ny * z);
    GLB R4<R>* uf = (GLB R4<R>*)S.u;
    const int64_t nc = S.ncell;
    if (solid_cell(S, x, y, z)) {
      if (mode == 1) {
        GLB R* rf = (GLB R*)S.rho;
        rf[cell] = (R)0;
      }
      continue;
    }
    const int par = (int)(*S.step & 1);
    const GLB T* src = (const GLB T*)S.f[par];
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
      const GLB R* gf = (const GLB R*)S.g;
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
      GLB R* rf = (GLB R*)S.rho;
      rf[cell] = rho;
      *(R4<R>*)(uf + cell) = R4<R>{ux, uy, uz, (R)0};
      continue;
    }
    if (S.has_ib) *(R4<R>*)(uf + cell) = R4<R>{ux, uy, uz, (R)0};
    // collision, Eq. (1), (2), (4), in offset form h = f - w
    const R om = (R)(1.0 / S.tau);
    const R pre = (R)(1.0 - 0.5 / S.tau);
    const R usq = ux * ux + uy * uy + uz * uz;
    const R ug = ux * gx + uy * gy + uz * gz;
    GLB T* dst = (GLB T*)S.f[par ^ 1];
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
  switch (phase) {
    case kPhaseForces:
      launch_forces(ST, sims, it, mode, s);
      break;
    case kPhaseSpread:
      launch_spread(ST, sims, it, mode, s);
      break;
    case kPhaseLattice:
      hipLaunchKernelGGL(k_lattice<ST>, dim3(grid_for(it.lat_total, 1 << 22)), dim3(kLatticeBlock), 0, s, sims, it, mode);
      break;
    case kPhaseInterp:
      launch_interp(ST, sims, it, mode, s);
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
