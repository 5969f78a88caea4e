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
#include <mutex>
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

// Executable graphs of 2^k timesteps, k = 0 .. 4 (the last is kGraphSteps).
struct GraphSet {
  static constexpr int kSizes = 5;
  hipGraphExec_t g[kSizes] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};
static_assert(1 << (GraphSet::kSizes - 1) == kGraphSteps, "graph sizes");

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
  size_t mesh_rigid, bstate, bconst, bft, xr, ndv, node_mesh, gcount, glist, fm;
  size_t t_nn, t_node0, t_edge0, t_ne, inc_ptr, inc, ev, el0, ec0, es0, txref;
  size_t t_nt, t_tri0, ttri, ta0, tav0;
  size_t step, remaining, health, red, red_out, simdev, items;
  size_t total;
  int64_t ncell, nbrick, ncube, nred, ngrid;
  int32_t ngm[3];
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
  if (d->morse != 0 && d->morse != 1) return fail(IBL_ERR_ARG, "morse must be 0 or 1");
  if (d->morse && (int64_t)(d->n[0] / 2 > 0 ? d->n[0] / 2 : 1) * (d->n[1] / 2 > 0 ? d->n[1] / 2 : 1) *
                          (d->n[2] / 2 > 0 ? d->n[2] / 2 : 1) >= ((int64_t)1 << 31))
    return fail(IBL_ERR_ARG, "the Morse neighbour grid is limited to 2^31 cells");
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
  L.mesh_rigid = take((size_t)d->max_meshes * 4);
  L.bstate = take((size_t)d->max_meshes * kBodyState * 8);
  L.bconst = take((size_t)d->max_meshes * kBodyConst * 8);
  L.bft = take((size_t)d->max_meshes * 6 * 8);
  L.xr = take(3 * maxn * 8);
  L.ndv = take(maxn * 8);
  L.node_mesh = take(maxn * 4);
  // Morse neighbour grid: cells at least 2 lattice units wide
  L.ngrid = 0;
  for (int a = 0; a < 3; ++a) L.ngm[a] = d->morse ? (d->n[a] / 2 > 0 ? d->n[a] / 2 : 1) : 0;
  if (d->morse) L.ngrid = (int64_t)L.ngm[0] * L.ngm[1] * L.ngm[2];
  L.gcount = take(2 * (size_t)L.ngrid * kMorseWords * 4);
  L.glist = take(2 * (size_t)L.ngrid * kMorseCap * 4);
  L.fm = take(3 * maxn * 8);
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
  std::vector<std::vector<int>> t_tris;  // per template: triangles, internal node numbering
  // meshes
  int nmesh = 0, nnodes = 0;
  std::vector<int> mesh_tmpl, mesh_off;
  int membrane = 0;  // some mesh has WLC-POW, area or volume terms
  int rigid = 0;     // some mesh is a rigid body
  std::vector<char> mesh_is_rigid;
  // graphs of 1, 2, 4, 8, 16 steps (invalidated when the work lists change)
  GraphSet graphs;
};

struct ibl_batch_s {
  std::vector<ibl_sim> sims;
  int storage = 0;
  hipStream_t stream = nullptr;
  SimDev* dsims = nullptr;
  int32_t* doffs = nullptr;
  Items items;
  GraphSet graphs;
  hipEvent_t ev = nullptr;
};

namespace {

void drop_graphs(GraphSet& G) {
  for (auto& g : G.g) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
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

// The graphs a run of `nmax` steps replays.  The first call that needs one
// not yet captured captures every size, so that later runs of any length
// only replay.
ibl_status ensure_graphs(int storage, const SimDev* sims, const Items& it, hipStream_t s, GraphSet& G,
                         int64_t nmax) {
  if (nmax <= 0) return IBL_OK;
  const int64_t full = nmax / kGraphSteps;
  const int rem = (int)(nmax % kGraphSteps);
  bool missing = false;
  for (int k = GraphSet::kSizes - 1; k >= 0; --k) {
    const int len = 1 << k;
    const bool need = (len == kGraphSteps) ? full > 0 : (rem & len) != 0;
    missing |= need && !G.g[k];
  }
  for (int k = GraphSet::kSizes - 1; missing && k >= 0; --k)
    if (!G.g[k]) {
      ibl_status st = capture(storage, sims, it, s, 1 << k, &G.g[k]);
      if (st) return st;
    }
  return IBL_OK;
}

// Run `n` steps (remaining <- n on every simulation of the set, set by the
// caller): replay the 16-step graph n / 16 times, then
// one graph of each power of two in the binary expansion of n % 16.
ibl_status run_steps(int storage, const SimDev* sims, const Items& it, hipStream_t s, GraphSet& G,
                     int64_t nmax) {
  if (nmax <= 0) return IBL_OK;
  const int64_t full = nmax / kGraphSteps;
  const int rem = (int)(nmax % kGraphSteps);
  for (int k = GraphSet::kSizes - 1; k >= 0; --k) {
    const int len = 1 << k;
    const bool need = (len == kGraphSteps) ? full > 0 : (rem & len) != 0;
    if (need && !G.g[k]) {  // (ensure_graphs captured them)
      ibl_status st = capture(storage, sims, it, s, len, &G.g[k]);
      if (st) return st;
    }
  }
  for (int64_t k = 0; k < full; ++k) HIPCHK(hipGraphLaunch(G.g[GraphSet::kSizes - 1], s));
  for (int k = GraphSet::kSizes - 2; k >= 0; --k)
    if (rem & (1 << k)) HIPCHK(hipGraphLaunch(G.g[k], s));
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
  it.moving_walls = 0;
  it.wall_cells = 0;
  for (int l = 0; l < 6; ++l) {
    if (!((S->hd.wall_moving >> l) & 1u)) continue;
    it.moving_walls = 1;
    const int a = l / 2, b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    const int64_t plane = (int64_t)S->desc.n[b] * S->desc.n[c];
    it.wall_cells = (int32_t)(plane > it.wall_cells ? plane : it.wall_cells);
  }
  it.rigid = S->rigid;
  it.morse = S->hd.morse[0] != 0.0 ? 1 : 0;
  it.sub = 0;
  drop_graphs(S->graphs);
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

// ------------------------------------------------ allocation-free batch --
// ibl_batch_step_static keeps the batch's device tables -- the member
// simulations' descriptors and the work-item prefix tables -- in this
// file-scope device array instead of memory it allocates.  Each GPU holds its
// own copy until the process ends.  In host code the array's name is not a
// device address: the address comes from hipGetSymbolAddress, once per
// device (static_tables), and only that address is passed to kernels.
constexpr int kStaticBatchMax = 64;
struct StaticBatchTables {
  SimDev sims[kStaticBatchMax];
  int32_t offs[4 * (kStaticBatchMax + 1)];  // lattice, reduction, mesh, cube prefixes
};
static __device__ __align__(256) StaticBatchTables scratch;

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
StaticBatchTables* g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`.
ibl_status static_tables(int dev, StaticBatchTables** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(IBL_ERR_UNSUPPORTED, "device index beyond the static table");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_static_ptr[dev] = (StaticBatchTables*)p;
  }
  *out = g_static_ptr[dev];
  return IBL_OK;
}

struct StaticBatchArgs {
  const SimDev* src[kStaticBatchMax];
  int32_t offs[4 * (kStaticBatchMax + 1)];
  int32_t n;
};

// One block per simulation copies its device descriptor into the table;
// block 0 also writes the prefix tables.
__global__ void k_static_tables(StaticBatchArgs a, StaticBatchTables* t) {
  const int i = blockIdx.x;
  const uint32_t* src = (const uint32_t*)a.src[i];
  uint32_t* dst = (uint32_t*)&t->sims[i];
  for (int w = threadIdx.x; w < (int)(sizeof(SimDev) / 4); w += blockDim.x) dst[w] = src[w];
  if (i == 0)
    for (int w = threadIdx.x; w < 4 * (a.n + 1); w += blockDim.x) t->offs[w] = a.offs[w];
}
static_assert(sizeof(SimDev) % 4 == 0, "descriptor copied as 32-bit words");

// plain streaming copy (calibration): 16-byte elements, four per thread in
// flight (loads first, then stores; non-temporal, as the lattice kernel's
// population traffic), grid-stride over blocks of 4 x 256 elements
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_hbm_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                  int64_t n) {
  constexpr int kU = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kU;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x * kU + threadIdx.x; b < n; b += stride) {
    u32x4 v[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int64_t i = b + (int64_t)k * blockDim.x;
      if (i < n) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      const int64_t i = b + (int64_t)k * blockDim.x;
      if (i < n) __builtin_nontemporal_store(v[k], dst + i);
    }
  }
}

}  // namespace

extern "C" {

const char* ibl_last_error(void) { return g_err.c_str(); }

ibl_status ibl_hbm_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16)
    return fail(IBL_ERR_ARG, "copy: null buffer, or a size or address not a multiple of 16");
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return IBL_OK;
  // up to 16 workgroups of 256 threads per compute unit
  int dev = 0, cus = 256;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t need = (n + 1023) / 1024;
  const int grid = (int)(need < 16LL * cus ? need : 16LL * cus);
  hipLaunchKernelGGL(k_hbm_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const u32x4*)src, (u32x4*)dst, n);
  HIPCHK(hipGetLastError());
  return IBL_OK;
}

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
  d.wall_moving = 0u;
  for (int l = 0; l < 6; ++l)
    for (int q = 0; q < kQ; ++q)
      if (desc->wall[l / 2] && d.bbw[q][l] != 0.0) d.wall_moving |= 1u << l;
  d.ncell = L.ncell;
  d.nbrick = L.nbrick;
  d.delta = desc->delta;
  d.tau = desc->tau;
  d.om = 1.0 / desc->tau;
  d.pre = 1.0 - 0.5 / desc->tau;
  d.om1 = 1.0 - d.om;
  d.a0 = 3.0 * d.om;
  d.a1 = 4.5 * d.om;
  d.b0 = 3.0 * d.pre;
  d.b1 = 9.0 * d.pre;
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
  d.mesh_rigid = (int32_t*)(A + L.mesh_rigid);
  d.bstate = (double*)(A + L.bstate);
  d.bconst = (double*)(A + L.bconst);
  d.bft = (double*)(A + L.bft);
  d.Xr = (double*)(A + L.xr);
  d.ndv = (double*)(A + L.ndv);
  d.node_mesh = (int32_t*)(A + L.node_mesh);
  d.gcount = (int32_t*)(A + L.gcount);
  d.glist = (int32_t*)(A + L.glist);
  d.Fm = (double*)(A + L.fm);
  d.ngrid = L.ngrid;
  for (int a = 0; a < 3; ++a) d.ngm[a] = L.ngm[a];
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
  drop_graphs(S->graphs);
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
  S->t_tris.push_back(ttri);
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

}  // extern "C"

namespace {

// Shared by ibl_mesh_add and ibl_body_add: checks, node upload (internal
// order), mesh tables.  `body` (rigid bodies only): state and constants
// records and the per-node body-frame offsets and weights, internal order.
struct BodyInit {
  double state[kBodyState];
  double cons[kBodyConst];
  std::vector<double> xr;  // [3][nn] SoA
  std::vector<double> dv;  // [nn]
};

ibl_status add_mesh(ibl_sim S, int32_t tmpl, const double* x, double ks, double kb, const BodyInit* body,
                    int32_t* out_mesh) {
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
  const int32_t rigid = body ? 1 : 0;
  {
    std::vector<int32_t> nm((size_t)nn, (int32_t)S->nmesh);
    HIPCHK(hipMemcpyAsync(d.node_mesh + off, nm.data(), 4 * (size_t)nn, hipMemcpyHostToDevice, S->stream));
  }
  HIPCHK(hipMemcpyAsync(d.mesh_tmpl + S->nmesh, &tmpl, 4, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(d.mesh_off + S->nmesh, &off, 4, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(d.mesh_ks + S->nmesh, &ks, 8, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(d.mesh_kb + S->nmesh, &kb, 8, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipMemcpyAsync(d.mesh_rigid + S->nmesh, &rigid, 4, hipMemcpyHostToDevice, S->stream));
  const double no_terms[4] = {0.0, 0.0, 0.0, 0.0};
  HIPCHK(hipMemcpyAsync(d.mesh_mem + 4 * (size_t)S->nmesh, no_terms, 32, hipMemcpyHostToDevice, S->stream));
  if (body) {
    HIPCHK(hipMemcpyAsync(d.bstate + kBodyState * (size_t)S->nmesh, body->state, sizeof(body->state),
                          hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipMemcpyAsync(d.bconst + kBodyConst * (size_t)S->nmesh, body->cons, sizeof(body->cons),
                          hipMemcpyHostToDevice, S->stream));
    for (int a = 0; a < 3; ++a)
      HIPCHK(hipMemcpyAsync(d.Xr + a * ms + off, body->xr.data() + (size_t)a * nn, 8 * (size_t)nn,
                            hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipMemcpyAsync(d.ndv + off, body->dv.data(), 8 * (size_t)nn, hipMemcpyHostToDevice, S->stream));
  }
  HIPCHK(launch_reset_lists(S->dd, S->L.nbrick, S->stream));  // new nodes: rebuild at the next step
  HIPCHK(hipStreamSynchronize(S->stream));
  S->mesh_tmpl.push_back(tmpl);
  S->mesh_off.push_back(off);
  S->mesh_is_rigid.push_back((char)rigid);
  S->rigid |= rigid;
  S->nnodes += nn;
  *out_mesh = S->nmesh++;
  return upload_simdev(S);
}

// Mass properties of a uniform solid of density dens bounded by a closed,
// outward triangulated surface (nodes p, triangles tris): the solid is a sum
// of signed tetrahedra (o, a, b, c) over the triangles, o the first node.
// Each contributes its volume a . (b x c) / 6, its first moment (volume times
// its centroid) and its second moment about o, V_t / 20 (aa^T + bb^T + cc^T
// + ss^T) with s = a + b + c (the covariance of a tetrahedron with a vertex at
// the origin).  Returns false for a surface enclosing no positive volume.
bool solid_mass(const std::vector<double>& p, const std::vector<int>& tris, double dens, double& M,
                double cm[3], double I[9]) {
  double V = 0.0, m1[3] = {0.0, 0.0, 0.0}, m2[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double* o = p.data();
  for (size_t t = 0; t + 2 < tris.size(); t += 3) {
    double a[3], b[3], c[3];
    for (int k = 0; k < 3; ++k) {
      a[k] = p[3 * (size_t)tris[t] + k] - o[k];
      b[k] = p[3 * (size_t)tris[t + 1] + k] - o[k];
      c[k] = p[3 * (size_t)tris[t + 2] + k] - o[k];
    }
    const double vt = (a[0] * (b[1] * c[2] - b[2] * c[1]) + a[1] * (b[2] * c[0] - b[0] * c[2]) +
                       a[2] * (b[0] * c[1] - b[1] * c[0])) / 6.0;
    V += vt;
    for (int i = 0; i < 3; ++i) {
      const double si = a[i] + b[i] + c[i];
      m1[i] += vt * si * 0.25;
      for (int j = 0; j < 3; ++j)
        m2[3 * i + j] += vt * 0.05 * (a[i] * a[j] + b[i] * b[j] + c[i] * c[j] + si * (a[j] + b[j] + c[j]));
    }
  }
  if (!(V > 0.0)) return false;
  double r[3];
  for (int i = 0; i < 3; ++i) r[i] = m1[i] / V;
  // second moment about the centre of mass, then I = dens (tr(C) Id - C)
  double C[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = m2[3 * i + j] - V * r[i] * r[j];
  const double tr = C[0] + C[4] + C[8];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) I[3 * i + j] = dens * ((i == j ? tr : 0.0) - C[3 * i + j]);
  M = dens * V;
  for (int i = 0; i < 3; ++i) cm[i] = o[i] + r[i];
  return true;
}

bool invert3(const double A[9], double B[9]) {
  const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
  const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  if (!(fabs(det) > 0.0) || !isfinite(det)) return false;
  const double id = 1.0 / det;
  B[0] = c00 * id; B[1] = (A[2] * A[7] - A[1] * A[8]) * id; B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  B[3] = c01 * id; B[4] = (A[0] * A[8] - A[2] * A[6]) * id; B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  B[6] = c02 * id; B[7] = (A[1] * A[6] - A[0] * A[7]) * id; B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
  return true;
}

}  // namespace

extern "C" {

ibl_status ibl_mesh_add(ibl_sim S, int32_t tmpl, const double* x, double ks, double kb, int32_t* out_mesh) {
  return add_mesh(S, tmpl, x, ks, kb, nullptr, out_mesh);
}

ibl_status ibl_body_add(ibl_sim S, int32_t tmpl, const double* x, double density, const double* v0,
                        const double* w0, int32_t* out_mesh) {
  if (!S || !x || !out_mesh) return fail(IBL_ERR_ARG, "null argument");
  if (tmpl < 0 || tmpl >= S->ntmpl) return fail(IBL_ERR_ARG, "unknown template");
  if (!(density > 0.0) || !isfinite(density)) return fail(IBL_ERR_ARG, "density must be positive and finite");
  for (int a = 0; a < 3; ++a)
    if ((v0 && !isfinite(v0[a])) || (w0 && !isfinite(w0[a]))) return fail(IBL_ERR_ARG, "non-finite velocity");
  const int nn = S->t_nn[tmpl];
  const std::vector<int>& perm = S->t_perm[tmpl];
  // node positions in internal order
  std::vector<double> p(3 * (size_t)nn);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < 3; ++a) {
      p[3 * (size_t)i + a] = x[3 * (size_t)perm[i] + a];
      if (!isfinite(p[3 * (size_t)i + a])) return fail(IBL_ERR_ARG, "non-finite node coordinate");
    }
  BodyInit B;
  double M, cm[3], I[9];
  if (!solid_mass(p, S->t_tris[tmpl], density, M, cm, I) || !invert3(I, B.cons + 1))
    return fail(IBL_ERR_ARG, "the body's surface encloses no volume");
  B.cons[0] = M;
  B.xr.assign(3 * (size_t)nn, 0.0);
  B.dv.assign((size_t)nn, 0.0);
  for (int i = 0; i < nn; ++i)
    for (int a = 0; a < 3; ++a) B.xr[(size_t)a * nn + i] = p[3 * (size_t)i + a] - cm[a];
  const std::vector<int>& tr = S->t_tris[tmpl];
  for (size_t t = 0; t + 2 < tr.size(); t += 3) {
    double e1[3], e2[3];
    for (int a = 0; a < 3; ++a) {
      e1[a] = p[3 * (size_t)tr[t + 1] + a] - p[3 * (size_t)tr[t] + a];
      e2[a] = p[3 * (size_t)tr[t + 2] + a] - p[3 * (size_t)tr[t] + a];
    }
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    const double share = 0.5 * sqrt(cx * cx + cy * cy + cz * cz) / 3.0;  // x one lattice spacing
    for (int k = 0; k < 3; ++k) B.dv[(size_t)tr[t + k]] += share;
  }
  // state: centre of mass, identity orientation (the body frame is the frame
  // of the given positions), velocity, angular momentum L = I w0
  memset(B.state, 0, sizeof(B.state));
  for (int a = 0; a < 3; ++a) {
    B.state[a] = cm[a];
    B.state[7 + a] = v0 ? v0[a] : 0.0;
  }
  B.state[3] = 1.0;
  for (int a = 0; a < 3; ++a)
    B.state[10 + a] = w0 ? I[3 * a] * w0[0] + I[3 * a + 1] * w0[1] + I[3 * a + 2] * w0[2] : 0.0;
  return add_mesh(S, tmpl, x, 0.0, 0.0, &B, out_mesh);
}

ibl_status ibl_sim_morse(ibl_sim S, double D0, double alpha, double r0, double rc) {
  if (!S) return fail(IBL_ERR_ARG, "null simulation");
  if (!isfinite(D0) || D0 < 0.0 || !isfinite(alpha) || !(alpha > 0.0) || !isfinite(r0) || !isfinite(rc) ||
      !(rc > 0.0))
    return fail(IBL_ERR_ARG, "Morse parameters: D0 >= 0, alpha > 0, rc > 0, all finite");
  if (!S->desc.morse) return fail(IBL_ERR_UNSUPPORTED, "the simulation was created without the Morse grid");
  if (rc > 2.0) return fail(IBL_ERR_UNSUPPORTED, "Morse cutoff beyond 2 lattice units (the grid's cell width)");
  HIPCHK(hipSetDevice(S->device));
  S->hd.morse[0] = D0;
  S->hd.morse[1] = alpha;
  S->hd.morse[2] = r0;
  S->hd.morse[3] = rc;
  HIPCHK(hipStreamSynchronize(S->stream));
  HIPCHK(launch_reset_lists(S->dd, S->L.nbrick, S->stream));  // both grids empty
  return upload_simdev(S);
}

ibl_status ibl_mesh_membrane(ibl_sim S, int32_t mesh, double kbt_p, double kg, double kl, double kv) {
  if (!S) return fail(IBL_ERR_ARG, "null simulation");
  if (mesh < 0 || mesh >= S->nmesh) return fail(IBL_ERR_ARG, "unknown mesh");
  const double k[4] = {kbt_p, kg, kl, kv};
  for (double v : k)
    if (!isfinite(v) || v < 0.0) return fail(IBL_ERR_ARG, "membrane constants must be finite and >= 0");
  const int tm = S->mesh_tmpl[mesh];
  if (S->mesh_is_rigid[mesh]) return fail(IBL_ERR_ARG, "a rigid body has no membrane energy");
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
  ibl_status st = ensure_graphs(S->desc.storage, S->dd, S->items, S->stream, S->graphs, n);
  if (st) return st;
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, S->stream, S->hd.remaining, n);
  HIPCHK(hipGetLastError());
  return run_steps(S->desc.storage, S->dd, S->items, S->stream, S->graphs, n);
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

ibl_status ibl_read_body(ibl_sim S, int32_t mesh, double* out) {
  if (!S || !out) return fail(IBL_ERR_ARG, "null argument");
  if (mesh < 0 || mesh >= S->nmesh) return fail(IBL_ERR_ARG, "unknown mesh");
  if (!S->mesh_is_rigid[mesh]) return fail(IBL_ERR_ARG, "not a rigid body");
  ibl_status st = observe(S);  // force and torque at the current state
  if (st) return st;
  double bs[kBodyState], bc[kBodyConst], ft[6];
  HIPCHK(hipMemcpy(bs, S->hd.bstate + kBodyState * (size_t)mesh, sizeof(bs), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(bc, S->hd.bconst + kBodyConst * (size_t)mesh, sizeof(bc), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ft, S->hd.bft + 6 * (size_t)mesh, sizeof(ft), hipMemcpyDeviceToHost));
  // Omega = R Ib^-1 R^T L
  const double w = bs[3], x = bs[4], y = bs[5], z = bs[6];
  const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                       2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                       2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
  double t[3], t2[3], om[3];
  for (int a = 0; a < 3; ++a) t[a] = R[a] * bs[10] + R[3 + a] * bs[11] + R[6 + a] * bs[12];
  for (int a = 0; a < 3; ++a) t2[a] = bc[1 + 3 * a] * t[0] + bc[2 + 3 * a] * t[1] + bc[3 + 3 * a] * t[2];
  for (int a = 0; a < 3; ++a) om[a] = R[3 * a] * t2[0] + R[3 * a + 1] * t2[1] + R[3 * a + 2] * t2[2];
  for (int a = 0; a < 3; ++a) {
    out[a] = bs[a];          // centre of mass
    out[7 + a] = bs[7 + a];  // velocity
    out[10 + a] = om[a];     // angular velocity
    out[13 + a] = ft[a];     // force
    out[16 + a] = ft[3 + a]; // torque
  }
  for (int a = 0; a < 4; ++a) out[3 + a] = bs[3 + a];  // orientation
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
         (size_t)3 * S->nnodes * 8 + (size_t)S->nmesh * kBodyState * 8;
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
  memcpy(h.magic, "IBLSTAT2", 8);
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
  if (S->nmesh)  // rigid-body states (unused records for capsules)
    HIPCHK(hipMemcpy(p, S->hd.bstate, (size_t)S->nmesh * kBodyState * 8, hipMemcpyDeviceToHost));
  return IBL_OK;
}

ibl_status ibl_write_state(ibl_sim S, const void* buf, size_t bytes) {
  size_t need = 0;
  ibl_status st = ibl_state_bytes(S, &need);
  if (st) return st;
  if (!buf || bytes < need) return fail(IBL_ERR_ARG, "state buffer too small");
  StateHeader h;
  memcpy(&h, buf, sizeof(h));
  if (memcmp(h.magic, "IBLSTAT2", 8) != 0 || h.storage != S->desc.storage || h.nnodes != S->nnodes ||
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
  if (S->nmesh) HIPCHK(hipMemcpy(S->hd.bstate, p, (size_t)S->nmesh * kBodyState * 8, hipMemcpyHostToDevice));
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
  it.moving_walls = 0;
  it.wall_cells = 0;
  it.rigid = 0;
  it.morse = 0;
  for (int i = 0; i < n; ++i) {
    it.big_templates |= sims[i]->big_templates;
    it.membrane |= sims[i]->membrane;
    it.moving_walls |= sims[i]->items.moving_walls;
    it.wall_cells = sims[i]->items.wall_cells > it.wall_cells ? sims[i]->items.wall_cells : it.wall_cells;
    it.rigid |= sims[i]->rigid;
    it.morse |= sims[i]->items.morse;
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
  {
    ibl_status st = ensure_graphs(B->storage, B->dsims, B->items, B->stream, B->graphs, nmax);
    if (st) return st;
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
  ibl_status st = run_steps(B->storage, B->dsims, B->items, B->stream, B->graphs, nmax);
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
  drop_graphs(B->graphs);
  (void)hipFree(B->dsims);
  (void)hipFree(B->doffs);
  (void)hipEventDestroy(B->ev);
  delete B;
  return IBL_OK;
}

ibl_status ibl_batch_step_static(const ibl_sim* sims, int32_t n, const int64_t* steps) {
  if (!sims || !steps) return fail(IBL_ERR_ARG, "null argument");
  if (n <= 0) return fail(IBL_ERR_ARG, "at least one simulation");
  if (n > kStaticBatchMax) return fail(IBL_ERR_ARG, "more simulations than the static table holds (64)");
  int64_t nmax = 0;
  for (int i = 0; i < n; ++i) {
    if (!sims[i]) return fail(IBL_ERR_ARG, "null simulation in batch");
    if (sims[i]->desc.storage != sims[0]->desc.storage) return fail(IBL_ERR_ARG, "mixed storage in batch");
    if (sims[i]->device != sims[0]->device) return fail(IBL_ERR_ARG, "mixed devices in batch");
    for (int j = 0; j < i; ++j)
      if (sims[j] == sims[i]) return fail(IBL_ERR_ARG, "simulation listed twice");
    if (steps[i] < 0) return fail(IBL_ERR_ARG, "negative step count");
    nmax = steps[i] > nmax ? steps[i] : nmax;
  }
  HIPCHK(hipSetDevice(sims[0]->device));
  StaticBatchTables* t = nullptr;
  ibl_status st = static_tables(sims[0]->device, &t);
  if (st) return st;
  hipStream_t s = sims[0]->stream;
  StaticBatchArgs a;
  a.n = n;
  int32_t* lat = a.offs;
  int32_t* red = lat + (n + 1);
  int32_t* msh = red + (n + 1);
  int32_t* cub = msh + (n + 1);
  lat[0] = red[0] = msh[0] = cub[0] = 0;
  Items it;
  memset(&it, 0, sizeof(it));
  for (int i = 0; i < n; ++i) {
    const Items& si = sims[i]->items;
    a.src[i] = sims[i]->dd;
    lat[i + 1] = lat[i] + si.lat_total;
    red[i + 1] = red[i] + si.red_total;
    msh[i + 1] = msh[i] + si.mesh_total;
    cub[i + 1] = cub[i] + si.cube_total;
    it.big_templates |= sims[i]->big_templates;
    it.membrane |= sims[i]->membrane;
    it.moving_walls |= si.moving_walls;
    it.wall_cells = si.wall_cells > it.wall_cells ? si.wall_cells : it.wall_cells;
    it.rigid |= sims[i]->rigid;
    it.morse |= si.morse;
  }
  it.nsim = n;
  it.lat_total = lat[n];
  it.red_total = red[n];
  it.mesh_total = msh[n];
  it.cube_total = cub[n];
  it.lat_off = t->offs;  // device addresses inside the table (no dereference here)
  it.red_off = t->offs + (n + 1);
  it.mesh_off = t->offs + 2 * (n + 1);
  it.cube_off = t->offs + 3 * (n + 1);
  it.forces_variant = forces_variant();
  it.sub = 0;
  hipLaunchKernelGGL(k_static_tables, dim3(n), dim3(256), 0, s, a, t);
  HIPCHK(hipGetLastError());
  StepArgs sa;
  sa.n = n;
  for (int i = 0; i < n; ++i) {
    sa.ptr[i] = sims[i]->hd.remaining;
    sa.val[i] = steps[i];
  }
  hipLaunchKernelGGL(k_set_many, dim3(1), dim3(64), 0, s, sa);
  HIPCHK(hipGetLastError());
  // plain launches (instantiating a graph would allocate): sequences of
  // kGraphSteps steps, then the rest
  const SimDev* ds = t->sims;
  for (int64_t k = 0; k < nmax; k += kGraphSteps) {
    const int len = (int)(nmax - k < kGraphSteps ? nmax - k : kGraphSteps);
    HIPCHK(launch_steps(sims[0]->desc.storage, ds, it, len, 0, s));
  }
  return IBL_OK;
}

}  // extern "C"
