// Host runtime of libibl.so: the C-ABI of include/ibl.h.
//
// A simulation lives in one caller-owned device arena.  The arena holds the
// two A/B population copies, the velocity / force / density fields, the node
// arrays (structure of arrays, FP64 positions), the per-brick candidate lists,
// the membrane templates and meshes, the control words (step counter, steps
// remaining, health) and the simulation's own device descriptor.  Timesteps
// are captured once into HIP graphs and replayed; the A/B parity and the
// remaining-step count live on the device, so a graph is valid at any step.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <map>
#include <string>
#include <vector>

#include "../../include/ibl.h"
#define IBL_HOST_LAYOUT 1
#include "ibl_internal.h"

using namespace ibl;

namespace {

thread_local std::string g_err;

ibl_status fail(ibl_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(IBL_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

constexpr int kGraphSteps = 16;

// Brick shape of a lattice: bs[0] x (kBrickThreads / bs[0]) x brick_depth cells,
// bs[0] the descriptor's brick_x, or by default the widest of 64, 32, 16 that
// the x extent fills (long x rows keep the streaming accesses in whole cache
// lines).
void brick_shape(const ibl_sim_desc* d, int bs[3]) {
  int bx = d->n[0] >= 64 ? 64 : (d->n[0] >= 32 ? 32 : 16);
  if (d->brick_x) bx = d->brick_x;
  bs[0] = bx;
  bs[1] = kBrickThreads / bx;
  bs[2] = brick_depth(d->storage);
}

int log2i(int v) {
  int k = 0;
  while ((1 << k) < v) ++k;
  return k;
}

// Force-kernel variant, a tuning knob read when a launch set is built: the
// default is one LDS workgroup per capsule (fixed-point sums for FP32/FP16
// storage); IBL_FORCES=split selects the edge / node split kernels for every
// template, IBL_FORCES=shares the per-edge-share LDS kernel for FP32/FP16 too.
int forces_variant() {
  const char* v = getenv("IBL_FORCES");
  if (v && strcmp(v, "split") == 0) return 1;
  if (v && strcmp(v, "shares") == 0) return 2;
  return 0;
}

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

int storage_bytes(int st) { return st == kF64 ? 8 : (st == kF32 ? 4 : 2); }
int real_bytes(int st) { return st == kF64 ? 8 : 4; }
size_t rec_bytes(int st) { return st == kF64 ? sizeof(NodeRec<double>) : sizeof(NodeRec<float>); }

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Layout {
  size_t f0, f1, u, g, rho, X, F, U, rec, escr, bcount, blist, bb0, fmax, lctl, hcount, hlist;
  size_t mesh_tmpl, mesh_off, mesh_ks, mesh_kb, mesh_mem, fext;
  size_t t_nn, t_node0, t_edge0, t_ne, inc_ptr, inc, ev, el0, ec0, es0, txref;
  size_t t_nt, t_tri0, ttri, ta0, tav0;
  size_t step, remaining, health, red, red_out, simdev, items;
  size_t total;
  int64_t ncell, nbrick, ncube, nred;
};

ibl_status check_desc(const ibl_sim_desc* d) {
  if (!d) return fail(IBL_ERR_ARG, "null descriptor");
  for (int a = 0; a < 3; ++a) {
    if (d->n[a] < 4) return fail(IBL_ERR_ARG, "every axis needs at least 4 cells");
    if (d->n[a] > 32767) return fail(IBL_ERR_ARG, "at most 32767 cells per axis");
    if (d->wall[a] != 0 && d->wall[a] != 1) return fail(IBL_ERR_ARG, "wall flag must be 0 or 1");
  }
  if (!(d->tau > 0.5)) return fail(IBL_ERR_ARG, "tau must exceed 1/2");
  if (d->storage < 0 || d->storage > 2) return fail(IBL_ERR_ARG, "unknown storage");
  if (d->brick_x != 0 && d->brick_x != 16 && d->brick_x != 32 && d->brick_x != 64)
    return fail(IBL_ERR_ARG, "brick_x must be 0, 16, 32 or 64");
  if (d->skin != 0 && d->skin != 1) return fail(IBL_ERR_ARG, "skin must be 0 or 1");
  if (d->delta < 0 || d->delta > 1) return fail(IBL_ERR_ARG, "unknown delta kernel");
  if (d->init_profile < 0 || d->init_profile > 1) return fail(IBL_ERR_ARG, "unknown init profile");
  if (d->max_nodes < 0 || d->max_meshes < 0 || d->max_templates < 0 || d->max_template_nodes < 0 ||
      d->max_template_edges < 0)
    return fail(IBL_ERR_ARG, "negative capacity");
  // streaming addresses two population planes with 32-bit byte offsets
  if ((d->storage == 0 || d->storage == 1 || d->storage == 2) &&
      2 * (int64_t)d->n[0] * d->n[1] * d->n[2] * storage_bytes(d->storage) >= ((int64_t)1 << 32))
    return fail(IBL_ERR_ARG, "lattice too large for its storage (2 ncell x element bytes must stay below 4 GiB)");
  if (d->max_nodes >= (1 << 26)) return fail(IBL_ERR_ARG, "at most 2^26 - 1 nodes per simulation");
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c)
      if (!isfinite(d->wall_u_lo[a][c]) || !isfinite(d->wall_u_hi[a][c]) || !isfinite(d->g_body[c]))
        return fail(IBL_ERR_ARG, "non-finite wall velocity or body force");
  return IBL_OK;
}

Layout make_layout(const ibl_sim_desc* d) {
  Layout L;
  const int st = d->storage;
  const int64_t ncell = (int64_t)d->n[0] * d->n[1] * d->n[2];
  int bs[3];
  brick_shape(d, bs);
  int64_t nb = 1;
  for (int a = 0; a < 3; ++a) nb *= ceil_div(d->n[a], bs[a]);
  const bool ib = d->max_nodes > 0;
  int64_t nq = 1;
  for (int a = 0; a < 3; ++a) nq *= ceil_div(d->n[a], 1 << kCubeShift[a]);
  L.ncell = ncell;
  L.nbrick = nb;
  L.ncube = nq;
  L.nred = ceil_div(ncell, kReduceItemCells);
  const size_t maxn = (size_t)d->max_nodes;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.f0 = take((size_t)kQ * ncell * storage_bytes(st));
  L.f1 = take((size_t)kQ * ncell * storage_bytes(st));
  L.u = take((size_t)3 * ncell * real_bytes(st));
  L.g = take((size_t)3 * ncell * real_bytes(st));
  L.rho = take((size_t)ncell * real_bytes(st));
  L.X = take(3 * maxn * 8);
  L.F = take(3 * maxn * 8);
  L.U = take(3 * maxn * 8);
  L.rec = take(maxn * rec_bytes(st));
  L.escr = take(maxn * 3 * 9 * 8);
  // the second list buffer and the build-time base cells only with a skin
  const size_t nbuf = d->skin ? 2 : 1;
  L.bcount = take(2 * (size_t)nb * 4);
  L.blist = take(ib ? nbuf * nb * kCandCap * 4 : 4);
  L.bb0 = take(d->skin ? maxn * 8 : 8);
  L.fmax = take(2 * 4);
  L.lctl = take(4 * 4);
  L.hcount = take((size_t)nq * 4);
  L.hlist = take(ib ? (size_t)nq * kHomeCap * 4 : 4);
  L.mesh_tmpl = take((size_t)d->max_meshes * 4);
  L.mesh_off = take((size_t)d->max_meshes * 4);
  L.mesh_ks = take((size_t)d->max_meshes * 8);
  L.mesh_kb = take((size_t)d->max_meshes * 8);
  L.mesh_mem = take((size_t)d->max_meshes * 4 * 8);
  L.fext = take(3 * maxn * 8);
  L.t_nn = take((size_t)d->max_templates * 4);
  L.t_node0 = take((size_t)d->max_templates * 4);
  L.t_edge0 = take((size_t)d->max_templates * 4);
  L.t_ne = take((size_t)d->max_templates * 4);
  L.inc_ptr = take(((size_t)d->max_template_nodes + 1) * 4);
  L.inc = take((size_t)d->max_template_edges * 4 * 4);
  L.ev = take((size_t)d->max_template_edges * 4 * 4);
  L.el0 = take((size_t)d->max_template_edges * 8);
  L.ec0 = take((size_t)d->max_template_edges * 8);
  L.es0 = take((size_t)d->max_template_edges * 8);
  L.txref = take((size_t)d->max_template_nodes * 3 * 8);  // staging of a template's reference shape
  L.t_nt = take((size_t)d->max_templates * 4);
  L.t_tri0 = take((size_t)d->max_templates * 4);
  L.ttri = take((size_t)d->max_template_edges * 3 * 4);  // a closed surface has fewer triangles than edges
  L.ta0 = take((size_t)d->max_template_edges * 8);
  L.tav0 = take((size_t)d->max_templates * 2 * 8);
  L.step = take(8);
  L.remaining = take(8);
  L.health = take(4);
  L.red = take((size_t)L.nred * 4 * 8);
  L.red_out = take(4 * 8);
  L.simdev = take(sizeof(SimDev));
  L.items = take(8 * 4);
  L.total = o;
  return L;
}

}  // namespace

struct ibl_sim_s {
  ibl_sim_desc desc;
  char* arena = nullptr;
  Layout L;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  SimDev hd;                 // host copy of the device descriptor
  SimDev* dd = nullptr;      // device copy (in the arena)
  int32_t* ditems = nullptr; // [10] prefix tables (in the arena)
  Items items;
  // templates
  int ntmpl = 0, tnodes = 0, tedges = 0, ttris = 0;
  std::vector<int> t_nn, t_node0, t_edge0;
  std::vector<char> t_big;  // per template: beyond the LDS force kernel
  std::vector<std::array<double, 3>> t_rest;  // per template: smallest rest triangle area, A0, V0
  int inc_total = 0;
  int big_templates = 0;
  // per template: internal node i holds the caller's node perm[i] (spatial
  // order of the reference shape, so neighbouring nodes share cache lines)
  std::vector<std::vector<int>> t_perm;
  // meshes
  int nmesh = 0, nnodes = 0;
  std::vector<int> mesh_tmpl, mesh_off;
  int membrane = 0;  // some mesh has WLC-POW, area or volume terms
  // graphs (invalidated when the work lists change)
  hipGraphExec_t g1 = nullptr, gN = nullptr;
};

struct ibl_batch_s {
  std::vector<ibl_sim> sims;
  int storage = 0;
  hipStream_t stream = nullptr;
  SimDev* dsims = nullptr;
  int32_t* doffs = nullptr;
  Items items;
  hipGraphExec_t g1 = nullptr, gN = nullptr;
  hipEvent_t ev = nullptr;
};

namespace {

void drop_graphs(hipGraphExec_t& g1, hipGraphExec_t& gN) {
  if (g1) (void)hipGraphExecDestroy(g1);
  if (gN) (void)hipGraphExecDestroy(gN);
  g1 = gN = nullptr;
}

// Capture `steps` timesteps of the given launch set into an executable graph.
ibl_status capture(int storage, const SimDev* sims, const Items& it, hipStream_t s, int steps,
                   hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
  hipError_t le = hipSuccess;
  le = launch_steps(storage, sims, it, steps, 0, s);
  hipError_t ce = hipStreamEndCapture(s, &graph);
  if (le != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(IBL_ERR_DEVICE, std::string("launch during capture: ") + hipGetErrorString(le));
  }
  if (ce != hipSuccess) return fail(IBL_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
  hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(IBL_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
  return IBL_OK;
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

struct StepArgs {
  int64_t* ptr[64];
  int64_t val[64];
  int n;
};
__global__ void k_set_many(StepArgs a) {
  const int i = threadIdx.x;
  if (i < a.n) *a.ptr[i] = a.val[i];
}

// Run `n` steps: remaining <- n on every simulation of the set, then
// replay the N-step graph and the 1-step graph.
ibl_status run_steps(int storage, const SimDev* sims, const Items& it, hipStream_t s,
                     hipGraphExec_t& g1, hipGraphExec_t& gN, int64_t nmax) {
  if (nmax <= 0) return IBL_OK;
  if (!g1) {
    ibl_status st = capture(storage, sims, it, s, 1, &g1);
    if (st) return st;
  }
  if (nmax >= kGraphSteps && !gN) {
    ibl_status st = capture(storage, sims, it, s, kGraphSteps, &gN);
    if (st) return st;
  }
  for (int64_t k = 0; k + kGraphSteps <= nmax; k += kGraphSteps) HIPCHK(hipGraphLaunch(gN, s));
  for (int64_t k = 0; k < nmax % kGraphSteps; ++k) HIPCHK(hipGraphLaunch(g1, s));
  return IBL_OK;
}

ibl_status upload_simdev(ibl_sim S) {
  S->hd.nnodes = S->nnodes;
  S->hd.nmeshes = S->nmesh;
  S->hd.has_ib = S->nmesh > 0 ? 1 : 0;
  int32_t h[8];
  h[0] = 0;
  h[1] = (int32_t)S->L.nbrick;
  h[2] = 0;
  h[3] = (int32_t)S->L.nred;
  h[4] = 0;
  h[5] = S->nmesh;
  h[6] = 0;
  h[7] = S->nmesh > 0 ? (int32_t)S->L.ncube : 0;
  HIPCHK(hipMemcpyAsync(S->dd, &S->hd, sizeof(SimDev), hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(S->ditems, h, sizeof(h), hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  Items& it = S->items;
  it.nsim = 1;
  it.lat_total = h[1];
  it.red_total = h[3];
  it.mesh_total = h[5];
  it.cube_total = h[7];
  it.lat_off = S->ditems + 0;
  it.red_off = S->ditems + 2;
  it.mesh_off = S->ditems + 4;
  it.cube_off = S->ditems + 6;
  it.big_templates = S->big_templates;
  it.forces_variant = forces_variant();
  it.membrane = S->membrane;
  it.sub = 0;
  drop_graphs(S->g1, S->gN);
  return IBL_OK;
}

ibl_status health_status(uint32_t h) {
  if (h & (kHNonfiniteF | kHRho | kHNonfiniteX | kHForceRange))
    return fail(IBL_ERR_UNSTABLE, "simulation became unstable (health word 0x" + std::to_string(h) + ")");
  if (h & (kHNodeRange | kHOverflow))
    return fail(IBL_ERR_STATE, "node outside the admissible range or candidate overflow (health 0x" +
                                   std::to_string(h) + ")");
  if (h & kHMach) return fail(IBL_ERR_UNSTABLE, "velocity above 0.3 lattice units");
  return IBL_OK;
}

template <typename R>
void fields_to_host(const std::vector<char>& raw, int64_t count, double* out) {
  const R* p = (const R*)raw.data();
  for (int64_t i = 0; i < count; ++i) out[i] = (double)p[i];
}

}  // namespace

extern "C" {

const char* ibl_last_error(void) { return g_err.c_str(); }

ibl_status ibl_sim_bytes(const ibl_sim_desc* desc, size_t* out_bytes) {
  if (!out_bytes) return fail(IBL_ERR_ARG, "null output");
  ibl_status st = check_desc(desc);
  if (st) return st;
  *out_bytes = make_layout(desc).total;
  return IBL_OK;
}

ibl_status ibl_sim_create(const ibl_sim_desc* desc, void* dev_arena, size_t arena_bytes,
                          void* hip_stream, ibl_sim* out) {
  if (!out || !dev_arena) return fail(IBL_ERR_ARG, "null argument");
  ibl_status st = check_desc(desc);
  if (st) return st;
  Layout L = make_layout(desc);
  if (arena_bytes < L.total) return fail(IBL_ERR_NOMEM, "arena smaller than ibl_sim_bytes");
  if (((uintptr_t)dev_arena) % 256 != 0) return fail(IBL_ERR_ARG, "arena must be 256-byte aligned");
  int device = 0;
  HIPCHK(hipGetDevice(&device));
  ibl_sim S = new ibl_sim_s();
  S->desc = *desc;
  S->arena = (char*)dev_arena;
  S->L = L;
  S->device = device;
  if (hip_stream) {
    S->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
      delete S;
      return fail(IBL_ERR_DEVICE, "hipStreamCreateWithFlags failed");
    }
    S->own_stream = true;
  }
  char* A = S->arena;
  SimDev& d = S->hd;
  memset(&d, 0, sizeof(d));
  int bs[3];
  brick_shape(desc, bs);
  for (int a = 0; a < 3; ++a) {
    d.n[a] = desc->n[a];
    d.wall[a] = desc->wall[a];
    d.nb[a] = (int32_t)ceil_div(desc->n[a], bs[a]);
    d.bs[a] = bs[a];
    d.bsh[a] = log2i(bs[a]);
    d.gb[a] = desc->g_body[a];
    for (int c = 0; c < 3; ++c) {
      d.ulo[a][c] = desc->wall_u_lo[a][c];
      d.uhi[a][c] = desc->wall_u_hi[a][c];
    }
  }
  for (int q = 0; q < kQ; ++q)
    for (int a = 0; a < 3; ++a)
      for (int hi = 0; hi < 2; ++hi) {
        const double* uw = hi ? d.uhi[a] : d.ulo[a];
        d.bbw[q][2 * a + hi] = 6.0 * wq(q) * (kCx[q] * uw[0] + kCy[q] * uw[1] + kCz[q] * uw[2]);
      }
  d.ncell = L.ncell;
  d.nbrick = L.nbrick;
  d.delta = desc->delta;
  d.tau = desc->tau;
  d.maxn = desc->max_nodes;
  d.skin = desc->skin;
  d.f[0] = A + L.f0;
  d.f[1] = A + L.f1;
  d.u = A + L.u;
  d.g = A + L.g;
  d.rho = A + L.rho;
  d.X = (double*)(A + L.X);
  d.F = (double*)(A + L.F);
  d.U = (double*)(A + L.U);
  d.rec = A + L.rec;
  d.escr = (double*)(A + L.escr);
  d.bcount = (int32_t*)(A + L.bcount);
  d.blist = (int32_t*)(A + L.blist);
  d.bb0 = (int16_t*)(A + L.bb0);
  d.fmax = (uint32_t*)(A + L.fmax);
  d.lctl = (int32_t*)(A + L.lctl);
  d.hcount = (int32_t*)(A + L.hcount);
  d.hlist = (int32_t*)(A + L.hlist);
  d.ncube = L.ncube;
  for (int a = 0; a < 3; ++a) d.nq[a] = (int32_t)ceil_div(desc->n[a], 1 << kCubeShift[a]);
  d.mesh_tmpl = (int32_t*)(A + L.mesh_tmpl);
  d.mesh_off = (int32_t*)(A + L.mesh_off);
  d.mesh_ks = (double*)(A + L.mesh_ks);
  d.mesh_kb = (double*)(A + L.mesh_kb);
  d.mesh_mem = (double*)(A + L.mesh_mem);
  d.Fext = (double*)(A + L.fext);
  d.t_nt = (int32_t*)(A + L.t_nt);
  d.t_tri0 = (int32_t*)(A + L.t_tri0);
  d.ttri = (int32_t*)(A + L.ttri);
  d.ta0 = (double*)(A + L.ta0);
  d.tav0 = (double*)(A + L.tav0);
  d.t_nn = (int32_t*)(A + L.t_nn);
  d.t_node0 = (int32_t*)(A + L.t_node0);
  d.t_edge0 = (int32_t*)(A + L.t_edge0);
  d.t_ne = (int32_t*)(A + L.t_ne);
  d.inc_ptr = (int32_t*)(A + L.inc_ptr);
  d.inc = (int32_t*)(A + L.inc);
  d.ev = (int32_t*)(A + L.ev);
  d.el0 = (double*)(A + L.el0);
  d.ec0 = (double*)(A + L.ec0);
  d.es0 = (double*)(A + L.es0);
  d.step = (int64_t*)(A + L.step);
  d.remaining = (int64_t*)(A + L.remaining);
  d.health = (uint32_t*)(A + L.health);
  d.red = (double*)(A + L.red);
  d.red_out = (double*)(A + L.red_out);
  S->dd = (SimDev*)(A + L.simdev);
  S->ditems = (int32_t*)(A + L.items);
  st = upload_simdev(S);
  if (!st) {
    hipError_t e = launch_init(desc->storage, S->dd, S->items, desc->init_profile, S->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d.inc_ptr, 0, 4, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) st = fail(IBL_ERR_DEVICE, std::string("init: ") + hipGetErrorString(e));
  }
  if (st) {
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    delete S;
    return st;
  }
  *out = S;
  return IBL_OK;
}

ibl_status ibl_sim_destroy(ibl_sim S) {
  if (!S) return IBL_OK;
  (void)hipSetDevice(S->device);  // teardown: nothing to report to
  (void)hipStreamSynchronize(S->stream);
  drop_graphs(S->g1, S->gN);
  if (S->own_stream) (void)hipStreamDestroy(S->stream);
  delete S;
  return IBL_OK;
}

void* ibl_sim_stream(ibl_sim S) { return S ? (void*)S->stream : nullptr; }

ibl_status ibl_template_add(ibl_sim S, int32_t nn, int32_t nt, const int32_t* tris, const double* xref,
                            int32_t* out_template) {
  if (!S || !tris || !xref || !out_template) return fail(IBL_ERR_ARG, "null argument");
  if (nn < 4 || nt < 4) return fail(IBL_ERR_ARG, "a closed surface needs >= 4 nodes and triangles");
  if (nn > kMaxTemplateNodes) return fail(IBL_ERR_UNSUPPORTED, "template has too many nodes");
  for (int64_t k = 0; k < 3 * (int64_t)nn; ++k)
    if (!isfinite(xref[k])) return fail(IBL_ERR_ARG, "non-finite reference coordinate");
  // internal node order: Morton (Z-order) code of the reference position
  std::vector<int> perm(nn), inv(nn);
  {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < nn; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = fmin(lo[a], xref[3 * i + a]);
        hi[a] = fmax(hi[a], xref[3 * i + a]);
      }
    std::vector<std::pair<uint64_t, int>> key(nn);
    for (int i = 0; i < nn; ++i) {
      uint64_t code = 0;
      uint32_t q[3];
      for (int a = 0; a < 3; ++a) {
        const double ext = hi[a] - lo[a];
        q[a] = ext > 0 ? (uint32_t)fmin(1023.0, (xref[3 * i + a] - lo[a]) / ext * 1023.0) : 0u;
      }
      for (int bit = 9; bit >= 0; --bit)
        for (int a = 0; a < 3; ++a) code = (code << 1) | ((q[a] >> bit) & 1u);
      key[i] = std::make_pair(code, i);
    }
    std::sort(key.begin(), key.end());
    for (int i = 0; i < nn; ++i) {
      perm[i] = key[i].second;
      inv[key[i].second] = i;
    }
  }
  // directed edges (internal numbering): (p -> q) -> opposite vertex of its triangle
  std::map<std::pair<int, int>, int> dir;
  for (int t = 0; t < nt; ++t) {
    for (int k = 0; k < 3; ++k) {
      const int p0 = tris[3 * t + k], q0 = tris[3 * t + (k + 1) % 3], r0 = tris[3 * t + (k + 2) % 3];
      if (p0 < 0 || p0 >= nn || q0 < 0 || q0 >= nn || r0 < 0 || r0 >= nn)
        return fail(IBL_ERR_ARG, "triangle with a bad node index");
      const int p = inv[p0], q = inv[q0], r = inv[r0];
      if (p < 0 || p >= nn || q < 0 || q >= nn || r < 0 || r >= nn || p == q || q == r || p == r)
        return fail(IBL_ERR_ARG, "triangle with a bad or repeated node index");
      if (!dir.emplace(std::make_pair(p, q), r).second)
        return fail(IBL_ERR_ARG, "directed edge used twice: mesh not consistently oriented");
    }
  }
  std::vector<int> ev;
  for (const auto& kv : dir) {
    const int p = kv.first.first, q = kv.first.second;
    auto rv = dir.find(std::make_pair(q, p));
    if (rv == dir.end()) return fail(IBL_ERR_ARG, "open edge: mesh is not closed");
    if (p < q) {
      ev.push_back(kv.second);   // v0: opposite in the triangle holding p -> q
      ev.push_back(p);           // v1
      ev.push_back(q);           // v2
      ev.push_back(rv->second);  // v3: opposite in the triangle holding q -> p
    }
  }
  const int ne = (int)(ev.size() / 4);
  // Edge order for the force kernels, whose 256 threads take 256 consecutive
  // edges at a time: the list above is sorted by (v1, v2), so neighbouring
  // edges mostly share v1.  Within each aligned block of 256 edges, the first
  // edge of every v1 comes first (in v1 order), then every second one, and so
  // on: a wave's lanes start from distinct, neighbouring nodes (measured: the
  // fixed-point force kernel runs about 3 % faster).  Sums in fixed point do
  // not depend on the order.
  {
    std::vector<int> ev2(ev.size());
    int o = 0;
    for (int b0 = 0; b0 < ne; b0 += 256) {
      const int b1 = std::min(ne, b0 + 256);
      std::vector<std::pair<int, int>> key;
      int run = 0;
      for (int e = b0; e < b1; ++e) {
        run = (e > b0 && ev[4 * e + 1] == ev[4 * (e - 1) + 1]) ? run + 1 : 0;
        key.push_back(std::make_pair(run, e));
      }
      std::sort(key.begin(), key.end());
      for (const auto& k : key) {
        for (int r = 0; r < 4; ++r) ev2[4 * (size_t)o + r] = ev[4 * (size_t)k.second + r];
        ++o;
      }
    }
    ev.swap(ev2);
  }
  if (ne > 3 * nn) return fail(IBL_ERR_UNSUPPORTED, "more than 3 edges per node (surface of genus > 1)");
  if (S->ntmpl + 1 > S->desc.max_templates || S->tnodes + nn > S->desc.max_template_nodes ||
      S->tedges + ne > S->desc.max_template_edges || S->ttris + nt > S->desc.max_template_edges)
    return fail(IBL_ERR_NOMEM, "template capacity exceeded");
  HIPCHK(hipSetDevice(S->device));
  const int e0 = S->tedges, n0 = S->tnodes;
  // incidence CSR rows of this template's nodes (global edge indices)
  std::vector<std::vector<int>> rows(nn);
  for (int e = 0; e < ne; ++e)
    for (int r = 0; r < 4; ++r) rows[ev[4 * e + r]].push_back(((e0 + e) << 2) | r);
  std::vector<int> ptr(nn + 1), inc;
  ptr[0] = S->inc_total;
  for (int i = 0; i < nn; ++i) {
    inc.insert(inc.end(), rows[i].begin(), rows[i].end());
    ptr[i + 1] = S->inc_total + (int)inc.size();
  }
  SimDev& d = S->hd;
  // the reference shape is staged in the arena (no allocation, so adding a
  // template does not synchronise the device)
  double* dx = (double*)(S->arena + S->L.txref) + 3 * (size_t)n0;
  hipError_t e = hipMemcpyAsync(d.ev + 4 * (size_t)e0, ev.data(), ev.size() * 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.inc + S->inc_total, inc.data(), inc.size() * 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.inc_ptr + n0, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.t_nn + S->ntmpl, &nn, 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.t_node0 + S->ntmpl, &n0, 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.t_edge0 + S->ntmpl, &e0, 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.t_ne + S->ntmpl, &ne, 4, hipMemcpyHostToDevice, S->stream);
  std::vector<double> xr_int(3 * (size_t)nn);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < 3; ++a) xr_int[3 * (size_t)i + a] = xref[3 * (size_t)perm[i] + a];
  if (!e) e = hipMemcpyAsync(dx, xr_int.data(), sizeof(double) * 3 * nn, hipMemcpyHostToDevice, S->stream);
  if (!e) e = launch_template_rest(S->dd, S->ntmpl, ne, dx, S->stream);
  // triangles (internal numbering) with their rest areas, and the rest area and
  // enclosed volume of Eqs. (9) and (10), the volume taken about internal node 0
  // as the membrane kernel does
  const int tr0 = S->ttris;
  std::vector<int> ttri(3 * (size_t)nt);
  std::vector<double> ta0(nt);
  double av0[2] = {0.0, 0.0}, amin = 1e300;
  const double* c0 = xr_int.data();
  for (int t = 0; t < nt; ++t) {
    double p[3][3];
    for (int k = 0; k < 3; ++k) {
      ttri[3 * (size_t)t + k] = inv[tris[3 * t + k]];
      for (int a = 0; a < 3; ++a) p[k][a] = xref[3 * (size_t)tris[3 * t + k] + a] - c0[a];
    }
    const double u[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
    const double w[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
    const double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    ta0[t] = 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double qr[3] = {p[1][1] * p[2][2] - p[1][2] * p[2][1], p[1][2] * p[2][0] - p[1][0] * p[2][2],
                          p[1][0] * p[2][1] - p[1][1] * p[2][0]};
    av0[0] += ta0[t];
    av0[1] += (p[0][0] * qr[0] + p[0][1] * qr[1] + p[0][2] * qr[2]) / 6.0;
    amin = fmin(amin, ta0[t]);
  }
  if (!e) e = hipMemcpyAsync(d.ttri + 3 * (size_t)tr0, ttri.data(), ttri.size() * 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.ta0 + tr0, ta0.data(), ta0.size() * 8, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.tav0 + 2 * (size_t)S->ntmpl, av0, 16, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.t_nt + S->ntmpl, &nt, 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipMemcpyAsync(d.t_tri0 + S->ntmpl, &tr0, 4, hipMemcpyHostToDevice, S->stream);
  if (!e) e = hipStreamSynchronize(S->stream);
  if (e) return fail(IBL_ERR_DEVICE, std::string("template upload: ") + hipGetErrorString(e));
  S->t_nn.push_back(nn);
  S->t_perm.push_back(perm);
  S->t_node0.push_back(n0);
  S->t_edge0.push_back(e0);
  if (nn > kLdsNodes || ne > kLdsEdges) S->big_templates = 1;
  S->t_big.push_back(nn > kLdsNodes || ne > kLdsEdges ? 1 : 0);
  S->t_rest.push_back({amin, av0[0], av0[1]});
  S->tnodes += nn;
  S->tedges += ne;
  S->ttris += nt;
  S->inc_total += (int)inc.size();
  *out_template = S->ntmpl++;
  return IBL_OK;
}

ibl_status ibl_mesh_add(ibl_sim S, int32_t tmpl, const double* x, double ks, double kb, int32_t* out_mesh) {
  if (!S || !x || !out_mesh) return fail(IBL_ERR_ARG, "null argument");
  if (tmpl < 0 || tmpl >= S->ntmpl) return fail(IBL_ERR_ARG, "unknown template");
  if (!isfinite(ks) || !isfinite(kb)) return fail(IBL_ERR_ARG, "non-finite ks or kb");
  const int nn = S->t_nn[tmpl];
  if (S->nmesh + 1 > S->desc.max_meshes || S->nnodes + nn > S->desc.max_nodes)
    return fail(IBL_ERR_NOMEM, "node or mesh capacity exceeded");
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < 3; ++a) {
      const double v = x[3 * i + a];
      if (!isfinite(v)) return fail(IBL_ERR_ARG, "non-finite node coordinate");
      if (S->desc.wall[a] && !(v >= 1.0 && v < (double)(S->desc.n[a] - 2)))
        return fail(IBL_ERR_ARG, "node outside 1 <= X < n-2 on a wall axis");
    }
  HIPCHK(hipSetDevice(S->device));
  const int off = S->nnodes;
  const size_t ms = (size_t)S->desc.max_nodes;
  const std::vector<int>& perm = S->t_perm[tmpl];
  std::vector<double> soa(3 * (size_t)nn);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < 3; ++a) soa[(size_t)a * nn + i] = x[3 * (size_t)perm[i] + a];
  SimDev& d = S->hd;
  for (int a = 0; a < 3; ++a) {
    HIPCHK(hipMemcpyAsync(d.X + a * ms + off, soa.data() + (size_t)a * nn, 8 * (size_t)nn,
                          hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipMemsetAsync(d.U + a * ms + off, 0, 8 * (size_t)nn, S->stream));
    HIPCHK(hipMemsetAsync(d.F + a * ms + off, 0, 8 * (size_t)nn, S->stream));
  }
  HIPCHK(hipMemcpyAsync(d.mesh_tmpl + S->nmesh, &tmpl, 4, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(d.mesh_off + S->nmesh, &off, 4, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(d.mesh_ks + S->nmesh, &ks, 8, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(d.mesh_kb + S->nmesh, &kb, 8, hipMemcpyHostToDevice, S->stream));
  const double no_terms[4] = {0.0, 0.0, 0.0, 0.0};
  HIPCHK(hipMemcpyAsync(d.mesh_mem + 4 * (size_t)S->nmesh, no_terms, 32, hipMemcpyHostToDevice, S->stream));
  HIPCHK(launch_reset_lists(S->dd, S->L.nbrick, S->stream));  // new nodes: rebuild at the next step
  HIPCHK(hipStreamSynchronize(S->stream));
  S->mesh_tmpl.push_back(tmpl);
  S->mesh_off.push_back(off);
  S->nnodes += nn;
  *out_mesh = S->nmesh++;
  return upload_simdev(S);
}

ibl_status ibl_mesh_membrane(ibl_sim S, int32_t mesh, double kbt_p, double kg, double kl, double kv) {
  if (!S) return fail(IBL_ERR_ARG, "null simulation");
  if (mesh < 0 || mesh >= S->nmesh) return fail(IBL_ERR_ARG, "unknown mesh");
  const double k[4] = {kbt_p, kg, kl, kv};
  for (double v : k)
    if (!isfinite(v) || v < 0.0) return fail(IBL_ERR_ARG, "membrane constants must be finite and >= 0");
  const int tm = S->mesh_tmpl[mesh];
  if (S->t_big[tm])
    return fail(IBL_ERR_UNSUPPORTED, "area, volume and WLC-POW terms need a template within the LDS force kernel");
  if ((kl != 0.0 && !(S->t_rest[tm][0] > 0.0)) || (kg != 0.0 && !(S->t_rest[tm][1] > 0.0)) ||
      (kv != 0.0 && !(S->t_rest[tm][2] > 0.0)))
    return fail(IBL_ERR_ARG, "reference shape with a degenerate triangle or no enclosed volume");
  HIPCHK(hipSetDevice(S->device));
  HIPCHK(hipMemcpyAsync(S->hd.mesh_mem + 4 * (size_t)mesh, k, 32, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  if (k[0] != 0.0 || k[1] != 0.0 || k[2] != 0.0 || k[3] != 0.0) S->membrane = 1;
  return upload_simdev(S);
}

ibl_status ibl_step(ibl_sim S, int64_t n) {
  if (!S || n < 0) return fail(IBL_ERR_ARG, "bad argument");
  if (n == 0) return IBL_OK;
  HIPCHK(hipSetDevice(S->device));
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, S->stream, S->hd.remaining, n);
  HIPCHK(hipGetLastError());
  return run_steps(S->desc.storage, S->dd, S->items, S->stream, S->g1, S->gN, n);
}

ibl_status ibl_sync(ibl_sim S) {
  if (!S) return fail(IBL_ERR_ARG, "null simulation");
  HIPCHK(hipSetDevice(S->device));
  HIPCHK(hipStreamSynchronize(S->stream));
  uint32_t h = 0;
  HIPCHK(hipMemcpy(&h, S->hd.health, 4, hipMemcpyDeviceToHost));
  return health_status(h);
}

static ibl_status observe(ibl_sim S) {
  HIPCHK(hipSetDevice(S->device));
  HIPCHK(launch_steps(S->desc.storage, S->dd, S->items, 1, 1, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  return IBL_OK;
}

ibl_status ibl_read_fields(ibl_sim S, double* rho, double* u, double* g) {
  if (!S) return fail(IBL_ERR_ARG, "null simulation");
  ibl_status st = observe(S);
  if (st) return st;
  const int64_t nc = S->L.ncell;
  const int rb = real_bytes(S->desc.storage);
  const bool dbl = S->desc.storage == kF64;
  std::vector<char> raw((size_t)3 * nc * rb);
  const SimDev& d = S->hd;
  auto solid = [&](int64_t c) {
    const int x = (int)(c % d.n[0]);
    const int64_t t = c / d.n[0];
    const int y = (int)(t % d.n[1]), z = (int)(t / d.n[1]);
    return (d.wall[0] && (x == 0 || x == d.n[0] - 1)) || (d.wall[1] && (y == 0 || y == d.n[1] - 1)) ||
           (d.wall[2] && (z == 0 || z == d.n[2] - 1));
  };
  if (rho) {
    HIPCHK(hipMemcpy(raw.data(), d.rho, (size_t)nc * rb, hipMemcpyDeviceToHost));
    if (dbl) fields_to_host<double>(raw, nc, rho); else fields_to_host<float>(raw, nc, rho);
    for (int64_t c = 0; c < nc; ++c)
      if (solid(c)) rho[c] = 0.0;
  }
  if (u) {
    HIPCHK(hipMemcpy(raw.data(), d.u, (size_t)3 * nc * rb, hipMemcpyDeviceToHost));
    if (dbl) fields_to_host<double>(raw, 3 * nc, u); else fields_to_host<float>(raw, 3 * nc, u);
    for (int64_t c = 0; c < nc; ++c)
      if (solid(c)) u[c] = u[nc + c] = u[2 * nc + c] = 0.0;
  }
  if (g) {
    HIPCHK(hipMemcpy(raw.data(), d.g, (size_t)3 * nc * rb, hipMemcpyDeviceToHost));
    if (dbl) fields_to_host<double>(raw, 3 * nc, g); else fields_to_host<float>(raw, 3 * nc, g);
    for (int64_t c = 0; c < nc; ++c)
      for (int a = 0; a < 3; ++a) g[a * nc + c] = solid(c) ? 0.0 : (S->nmesh ? g[a * nc + c] : 0.0) + d.gb[a];
  }
  return IBL_OK;
}

ibl_status ibl_read_nodes(ibl_sim S, int32_t mesh, double* x, double* u, double* f) {
  if (!S) return fail(IBL_ERR_ARG, "null simulation");
  if (mesh < 0 || mesh >= S->nmesh) return fail(IBL_ERR_ARG, "unknown mesh");
  ibl_status st = observe(S);
  if (st) return st;
  const int off = S->mesh_off[mesh];
  const int nn = S->t_nn[S->mesh_tmpl[mesh]];
  const std::vector<int>& perm = S->t_perm[S->mesh_tmpl[mesh]];
  const size_t ms = (size_t)S->desc.max_nodes;
  std::vector<double> tmp((size_t)nn);
  double* src[3] = {S->hd.X, S->hd.U, S->hd.F};
  double* dst[3] = {x, u, f};
  for (int k = 0; k < 3; ++k) {
    if (!dst[k]) continue;
    for (int a = 0; a < 3; ++a) {
      HIPCHK(hipMemcpy(tmp.data(), src[k] + a * ms + off, 8 * (size_t)nn, hipMemcpyDeviceToHost));
      for (int i = 0; i < nn; ++i) dst[k][3 * (size_t)perm[i] + a] = tmp[i];
    }
  }
  return IBL_OK;
}

ibl_status ibl_conservation(ibl_sim S, double* mass, double momentum[3], uint32_t* health) {
  if (!S) return fail(IBL_ERR_ARG, "null simulation");
  HIPCHK(hipSetDevice(S->device));
  HIPCHK(launch_reduce(S->desc.storage, S->dd, S->items, S->stream));
  double out[4];
  uint32_t h = 0;
  HIPCHK(hipStreamSynchronize(S->stream));
  HIPCHK(hipMemcpy(out, S->hd.red_out, sizeof(out), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(&h, S->hd.health, 4, hipMemcpyDeviceToHost));
  if (mass) *mass = out[0];
  if (momentum)
    for (int a = 0; a < 3; ++a) momentum[a] = out[1 + a];
  if (health) *health = h;
  return health_status(h);
}

ibl_status ibl_step_count(ibl_sim S, int64_t* out) {
  if (!S || !out) return fail(IBL_ERR_ARG, "null argument");
  HIPCHK(hipSetDevice(S->device));
  HIPCHK(hipStreamSynchronize(S->stream));
  HIPCHK(hipMemcpy(out, S->hd.step, 8, hipMemcpyDeviceToHost));
  return IBL_OK;
}

// Serialized state: header, populations of the current parity (storage
// format), node positions (SoA, FP64).
struct StateHeader {
  char magic[8];
  int32_t storage, n[3], nnodes, pad;
  int64_t step;
};

ibl_status ibl_state_bytes(ibl_sim S, size_t* out) {
  if (!S || !out) return fail(IBL_ERR_ARG, "null argument");
  *out = sizeof(StateHeader) + (size_t)kQ * S->L.ncell * storage_bytes(S->desc.storage) +
         (size_t)3 * S->nnodes * 8;
  return IBL_OK;
}

ibl_status ibl_read_state(ibl_sim S, void* buf, size_t bytes) {
  size_t need = 0;
  ibl_status st = ibl_state_bytes(S, &need);
  if (st) return st;
  if (!buf || bytes < need) return fail(IBL_ERR_ARG, "state buffer too small");
  int64_t step = 0;
  st = ibl_step_count(S, &step);
  if (st) return st;
  StateHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, "IBLSTAT1", 8);
  h.storage = S->desc.storage;
  for (int a = 0; a < 3; ++a) h.n[a] = S->desc.n[a];
  h.nnodes = S->nnodes;
  h.step = step;
  char* p = (char*)buf;
  memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const size_t fb = (size_t)kQ * S->L.ncell * storage_bytes(S->desc.storage);
  HIPCHK(hipMemcpy(p, S->hd.f[step & 1], fb, hipMemcpyDeviceToHost));
  p += fb;
  for (int a = 0; a < 3; ++a) {
    HIPCHK(hipMemcpy(p, S->hd.X + (size_t)a * S->desc.max_nodes, 8 * (size_t)S->nnodes, hipMemcpyDeviceToHost));
    p += 8 * (size_t)S->nnodes;
  }
  return IBL_OK;
}

ibl_status ibl_write_state(ibl_sim S, const void* buf, size_t bytes) {
  size_t need = 0;
  ibl_status st = ibl_state_bytes(S, &need);
  if (st) return st;
  if (!buf || bytes < need) return fail(IBL_ERR_ARG, "state buffer too small");
  StateHeader h;
  memcpy(&h, buf, sizeof(h));
  if (memcmp(h.magic, "IBLSTAT1", 8) != 0 || h.storage != S->desc.storage || h.nnodes != S->nnodes ||
      h.n[0] != S->desc.n[0] || h.n[1] != S->desc.n[1] || h.n[2] != S->desc.n[2] || h.step < 0)
    return fail(IBL_ERR_ARG, "state does not match this simulation");
  HIPCHK(hipSetDevice(S->device));
  HIPCHK(hipStreamSynchronize(S->stream));
  const char* p = (const char*)buf + sizeof(h);
  const size_t fb = (size_t)kQ * S->L.ncell * storage_bytes(S->desc.storage);
  HIPCHK(hipMemcpy(S->hd.f[h.step & 1], p, fb, hipMemcpyHostToDevice));
  p += fb;
  for (int a = 0; a < 3; ++a) {
    HIPCHK(hipMemcpy(S->hd.X + (size_t)a * S->desc.max_nodes, p, 8 * (size_t)S->nnodes, hipMemcpyHostToDevice));
    p += 8 * (size_t)S->nnodes;
  }
  HIPCHK(hipMemcpy(S->hd.step, &h.step, 8, hipMemcpyHostToDevice));
  HIPCHK(launch_reset_lists(S->dd, S->L.nbrick, S->stream));  // positions replaced: rebuild
  HIPCHK(hipStreamSynchronize(S->stream));
  return IBL_OK;
}

ibl_status ibl_profile_phases(ibl_sim S, int64_t n, double* ms) {
  if (!S || !ms || n <= 0 || n > 100000) return fail(IBL_ERR_ARG, "bad argument");
  HIPCHK(hipSetDevice(S->device));
  const int np = kNumPhases;
  std::vector<hipEvent_t> ev((size_t)n * np + 1, nullptr);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, S->stream, S->hd.remaining, n);
  hipError_t err = hipGetLastError();
  if (!err) err = hipEventRecord(ev[0], S->stream);
  for (int64_t k = 0; k < n && !err; ++k)
    for (int ph = 0; ph < np && !err; ++ph) {
      err = launch_phase(S->desc.storage, S->dd, S->items, ph, 0, S->stream);
      if (!err) err = hipEventRecord(ev[(size_t)k * np + ph + 1], S->stream);
    }
  if (!err) err = hipStreamSynchronize(S->stream);
  for (int ph = 0; ph <= np; ++ph) ms[ph] = 0.0;
  for (int64_t k = 0; k < n && !err; ++k)
    for (int ph = 0; ph < np && !err; ++ph) {
      float t = 0.f;
      err = hipEventElapsedTime(&t, ev[(size_t)k * np + ph], ev[(size_t)k * np + ph + 1]);
      ms[ph] += t / (double)n;
    }
  float tot = 0.f;
  if (!err) err = hipEventElapsedTime(&tot, ev[0], ev[(size_t)n * np]);
  ms[np] = tot;
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (err) return fail(IBL_ERR_DEVICE, std::string("phase profile: ") + hipGetErrorString(err));
  return IBL_OK;
}

ibl_status ibl_batch_create(const ibl_sim* sims, int32_t n, ibl_batch* out) {
  if (!sims || n <= 0 || !out) return fail(IBL_ERR_ARG, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    if (!sims[i]) return fail(IBL_ERR_ARG, "null simulation in batch");
    if (sims[i]->desc.storage != sims[0]->desc.storage) return fail(IBL_ERR_ARG, "mixed storage in batch");
    if (sims[i]->device != sims[0]->device) return fail(IBL_ERR_ARG, "mixed devices in batch");
    for (int j = 0; j < i; ++j)
      if (sims[j] == sims[i]) return fail(IBL_ERR_ARG, "simulation listed twice");
  }
  HIPCHK(hipSetDevice(sims[0]->device));
  ibl_batch B = new ibl_batch_s();
  B->sims.assign(sims, sims + n);
  B->storage = sims[0]->desc.storage;
  B->stream = sims[0]->stream;
  std::vector<SimDev> host(n);
  std::vector<int32_t> offs(4 * (size_t)(n + 1));
  int32_t* lat = offs.data();
  int32_t* red = lat + (n + 1);
  int32_t* msh = red + (n + 1);
  int32_t* brk = msh + (n + 1);
  lat[0] = red[0] = msh[0] = brk[0] = 0;
  for (int i = 0; i < n; ++i) {
    const Items& it = sims[i]->items;
    host[i] = sims[i]->hd;
    lat[i + 1] = lat[i] + it.lat_total;
    red[i + 1] = red[i] + it.red_total;
    msh[i + 1] = msh[i] + it.mesh_total;
    brk[i + 1] = brk[i] + it.cube_total;
  }
  hipError_t e = hipMalloc(&B->dsims, sizeof(SimDev) * n);
  if (!e) e = hipMalloc(&B->doffs, offs.size() * 4);
  if (!e) e = hipMemcpy(B->dsims, host.data(), sizeof(SimDev) * n, hipMemcpyHostToDevice);
  if (!e) e = hipMemcpy(B->doffs, offs.data(), offs.size() * 4, hipMemcpyHostToDevice);
  if (!e) e = hipEventCreateWithFlags(&B->ev, hipEventDisableTiming);
  if (e) {
    (void)hipFree(B->dsims);
    (void)hipFree(B->doffs);
    delete B;
    return fail(IBL_ERR_DEVICE, std::string("batch tables: ") + hipGetErrorString(e));
  }
  Items& it = B->items;
  it.nsim = n;
  it.lat_total = lat[n];
  it.red_total = red[n];
  it.mesh_total = msh[n];
  it.cube_total = brk[n];
  it.lat_off = B->doffs;
  it.red_off = B->doffs + (n + 1);
  it.mesh_off = B->doffs + 2 * (n + 1);
  it.cube_off = B->doffs + 3 * (n + 1);
  it.big_templates = 0;
  it.membrane = 0;
  for (int i = 0; i < n; ++i) {
    it.big_templates |= sims[i]->big_templates;
    it.membrane |= sims[i]->membrane;
  }
  it.forces_variant = forces_variant();
  it.sub = 0;
  *out = B;
  return IBL_OK;
}

ibl_status ibl_batch_step(ibl_batch B, const int64_t* steps) {
  if (!B || !steps) return fail(IBL_ERR_ARG, "null argument");
  const int n = (int)B->sims.size();
  int64_t nmax = 0;
  for (int i = 0; i < n; ++i) {
    if (steps[i] < 0) return fail(IBL_ERR_ARG, "negative step count");
    nmax = steps[i] > nmax ? steps[i] : nmax;
  }
  HIPCHK(hipSetDevice(B->sims[0]->device));
  // order the batch stream after pending work of the members' own streams
  for (int i = 1; i < n; ++i)
    if (B->sims[i]->stream != B->stream) {
      HIPCHK(hipEventRecord(B->ev, B->sims[i]->stream));
      HIPCHK(hipStreamWaitEvent(B->stream, B->ev, 0));
    }
  for (int i0 = 0; i0 < n; i0 += 64) {
    StepArgs a;
    a.n = (n - i0) < 64 ? (n - i0) : 64;
    for (int k = 0; k < a.n; ++k) {
      a.ptr[k] = B->sims[i0 + k]->hd.remaining;
      a.val[k] = steps[i0 + k];
    }
    hipLaunchKernelGGL(k_set_many, dim3(1), dim3(64), 0, B->stream, a);
    HIPCHK(hipGetLastError());
  }
  ibl_status st = run_steps(B->storage, B->dsims, B->items, B->stream, B->g1, B->gN, nmax);
  if (st) return st;
  HIPCHK(hipEventRecord(B->ev, B->stream));
  for (int i = 1; i < n; ++i)
    if (B->sims[i]->stream != B->stream) HIPCHK(hipStreamWaitEvent(B->sims[i]->stream, B->ev, 0));
  return IBL_OK;
}

ibl_status ibl_batch_destroy(ibl_batch B) {
  if (!B) return IBL_OK;
  (void)hipSetDevice(B->sims[0]->device);  // teardown: nothing to report to
  (void)hipStreamSynchronize(B->stream);
  drop_graphs(B->g1, B->gN);
  (void)hipFree(B->dsims);
  (void)hipFree(B->doffs);
  (void)hipEventDestroy(B->ev);
  delete B;
  return IBL_OK;
}

}  // extern "C"
