// Internal declarations shared by the kernels (ibl_kernels.hip) and the host
// runtime (ibl_runtime.hip) of libibl.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// Pointers inside device descriptors are plain pointers on the host and
// global-address-space pointers in device code, so loads and stores through
// them compile to global (not generic / flat) memory instructions.
// (ibl_runtime.hip, host code only, defines IBL_HOST_LAYOUT to see plain
// pointers in both of its compilation passes; the layout is the same.)
#if defined(__HIP_DEVICE_COMPILE__) && !defined(IBL_HOST_LAYOUT)
#define IBL_G(T) T __attribute__((address_space(1)))*
#else
#define IBL_G(T) T*
#endif

namespace ibl {

constexpr int kQ = 19;
// The lattice is processed in bricks of bs[0] x bs[1] x bs[2] cells with
// bs[0] x bs[1] = kBrickThreads: one workgroup per brick, each thread a column
// of bs[2] cells (brick_depth of the storage mode).  bs[0] (16, 32 or 64) is
// chosen per simulation.
constexpr int kBrickThreads = 256;
constexpr int kCandCap = 4096;       // candidate nodes per brick
// Candidate lists are rebuilt every step (skin 0), or built with a skin of
// `skin` cells around each node's stencil and kept while every node's stencil
// base cell stays within `skin` cells (per axis) of its base when the lists
// were built.
// Interpolation groups nodes by home cube (the cube of their stencil base
// cell), cubes of kCube[0] x kCube[1] x kCube[2] cells.
constexpr int kCubeShift[3] = {4, 3, 3};
constexpr int kHomeCap = 4096;       // nodes per home cube
constexpr int kLatticeBlock = 256;   // threads of the reduction work items
constexpr int kLdsNodes = 642;       // template size handled by the LDS force kernel (icosphere level 3)
constexpr int kLdsEdges = 1920;
constexpr int kReduceItemCells = 4096;
constexpr int kMaxTemplateNodes = 4096;  // nodes per template (one workgroup per mesh)
constexpr int kBodyState = 16;   // doubles per rigid-body state record
constexpr int kBodyConst = 10;   // doubles per rigid-body constants record
constexpr int kMorseCap = 48;    // nodes per cell of the Morse neighbour grid
constexpr int kMorseWords = 2;   // int32 words per cell of that grid (owner, count)

// ------------------------------------------------------------------------
// D3Q19 in the library's order: the rest velocity, the z = 0 plane, then the
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

enum Storage : int { kF64 = 0, kF32 = 1, kF16 = 2 };

// Cells per thread column of a brick.  FP16 storage streams half the bytes,
// so a brick's spreading phase hides less behind the other workgroups'
// streaming: its bricks are twice as deep (and its spread-force field packs
// three sums per word, so the LDS still holds five workgroups per CU).
constexpr int brick_depth(int storage) { return storage == kF16 ? 8 : 4; }
enum Delta : int { kCos = 0, kPeskin4 = 1 };

enum Health : uint32_t {
  kHNonfiniteF = 0x1u,
  kHRho = 0x2u,
  kHMach = 0x4u,
  kHNodeRange = 0x8u,
  kHOverflow = 0x10u,
  kHNonfiniteX = 0x20u,
  kHForceRange = 0x40u,
};

// Spreading record of one node, written by the force kernel at X^n and read by
// the spreading and interpolation kernels of the same step.  FP64 storage
// keeps the 12 delta weights; FP32 / FP16 storage keeps the fractional offset
// of X from its base cell per axis (32 bytes: each record is read by the ~3
// bricks its stencil meets, so its size is HBM traffic) and the readers
// evaluate the same weights from it.
template <typename R>
struct alignas(16) NodeRec {
  int32_t base[3];   // floor(X) per axis (periodic axes: modulo n)
  int32_t valid;     // 0 when the node is outside the admissible range, 1 a capsule's
                     // node (interpolated and moved), 2 a rigid body's node (spread only)
  R w[3][4];         // phi at offsets -1, 0, +1, +2 from base, per axis
  R F[3];            // membrane force
  R pad;
};
template <>
struct alignas(16) NodeRec<float> {
  int16_t base[3];   // floor(X) per axis (periodic axes: modulo n); axes < 2^15 cells
  int16_t valid;     // as above
  float d[3];        // X - base per axis, in [0, 1)
  float F[3];
};
static_assert(sizeof(NodeRec<float>) == 32, "compact spreading record");

// Per-simulation device descriptor.  Lives in device memory; kernels take an
// array of these (one entry for a single simulation, many for a batch).
struct SimDev {
  int32_t n[3];
  int32_t wall[3];
  int64_t ncell;
  int32_t nb[3];          // bricks per axis
  int32_t bs[3];          // brick size per axis (powers of two)
  int32_t bsh[3];         // log2 of bs
  int32_t delta;
  int64_t nbrick;
  int32_t nq[3];          // home cubes per axis
  int64_t ncube;
  double tau;
  // collision coefficients (see k_lattice): om = 1/tau, pre = 1 - 1/(2 tau),
  // then 1 - om, 3 om, 9/2 om, 3 pre, 9 pre
  double om, pre, om1, a0, a1, b0, b1;
  double gb[3];
  double ulo[3][3];
  double uhi[3][3];
  double bbw[kQ][6];      // moving-wall term 6 w_q (c_q . u_wall) of a bounce-back link, per
                          // direction and wall layer (2 * axis + [hi side])
  uint32_t wall_moving;   // bit l: wall layer l has a non-zero term (a moving wall axis)
  uint32_t pad_wm;
  int32_t has_ib;         // 1 when meshes are present
  int32_t nnodes;
  int32_t nmeshes;
  int32_t maxn;           // SoA stride of the node arrays (capacity)
  int32_t skin;           // candidate-list skin in cells (0: lists rebuilt every step)
  // state
  IBL_G(void) f[2];             // populations, [19][ncell] in storage format
  IBL_G(void) u;                // [3][ncell] velocity (compute precision)
  IBL_G(void) g;                // [3][ncell] spread force (compute precision; observation only)
  IBL_G(void) rho;              // [ncell] density (observation only)
  IBL_G(double) X;              // [3][max_nodes] positions
  IBL_G(double) F;              // [3][max_nodes] membrane forces
  IBL_G(double) U;              // [3][max_nodes] interpolated velocities
  IBL_G(void) rec;              // [max_nodes] NodeRec
  IBL_G(double) escr;           // [3 * max_nodes][9] per-edge force shares (G0, G3, F1)
  IBL_G(int32_t) bcount;        // [2][nbrick] candidate counts of the two list buffers
  IBL_G(int32_t) blist;         // [2][nbrick][kCandCap]
  IBL_G(int16_t) bb0;           // [max_nodes][4] stencil base cell when the lists were built
  IBL_G(uint32_t) fmax;         // [2] largest |F component| of the step, by step parity (float bits)
  IBL_G(int32_t) lctl;          // [4] list buffer in use after the step of parity 0, 1;
                                //     lists rebuilt by the step of parity 0, 1 (flags)
  IBL_G(int32_t) hcount;        // [ncube] nodes per home cube
  IBL_G(int32_t) hlist;         // [ncube][kHomeCap]
  // meshes
  IBL_G(int32_t) mesh_tmpl;     // [max_meshes]
  IBL_G(int32_t) mesh_off;      // [max_meshes] first global node
  IBL_G(double) mesh_ks;
  IBL_G(double) mesh_kb;
  IBL_G(double) mesh_mem;       // [max_meshes][4] kBT/p, kg, kl, kv (zero: term absent)
  IBL_G(double) Fext;           // [3][max_nodes] force of those terms (k_membrane); for a
                                //     rigid body's nodes, their FSI force on the body
  // rigid bodies (Sec. 2.3, Eq. (17)): a mesh flagged rigid moves as one body
  IBL_G(int32_t) mesh_rigid;    // [max_meshes] 1: rigid body, 0: deformable capsule
  IBL_G(double) bstate;         // [max_meshes][16] xc[3], q[4] (w, x, y, z), v[3], L[3] (lab frame)
  IBL_G(double) bconst;         // [max_meshes][10] mass, inverse body-frame inertia tensor [9]
  IBL_G(double) bft;            // [max_meshes][6] force and torque on the body, last evaluation
  IBL_G(double) Xr;             // [3][max_nodes] body-frame node offsets from the centre of mass
  IBL_G(double) ndv;            // [max_nodes] node weight: a third of its triangles' areas x 1 lu
  IBL_G(int32_t) node_mesh;     // [max_nodes] mesh of each node
  // inter-capsule Morse repulsion (Eq. (13)): neighbour grid by step parity
  double morse[4];              // D0, alpha, r0, rc (D0 = 0: off)
  int32_t ngm[3];               // grid cells per axis (each at least 2 lattice units wide)
  int64_t ngrid;
  IBL_G(int32_t) gcount;        // [2][ngrid][kMorseWords] per grid cell: owner (0 empty,
                                //   m + 1 only mesh m's nodes, -1 several meshes'), count
  IBL_G(int32_t) glist;         // [2][ngrid][kMorseCap] node ids
  IBL_G(double) Fm;             // [3][max_nodes] Morse force of the step
  // templates
  IBL_G(int32_t) t_nn;          // [max_templates]
  IBL_G(int32_t) t_node0;       // first template-node index
  IBL_G(int32_t) t_edge0;       // first template-edge index
  IBL_G(int32_t) t_ne;          // edges per template
  IBL_G(int32_t) inc_ptr;       // [max_template_nodes + 1] CSR row pointers over all templates
  IBL_G(int32_t) inc;           // incidence entries: (edge << 2) | role, global edge index
  IBL_G(int32_t) ev;            // [max_template_edges][4] template-local node indices
  IBL_G(double) el0;            // [max_template_edges] rest length
  IBL_G(double) ec0;            // cos(theta0)
  IBL_G(double) es0;            // sin(theta0)
  IBL_G(int32_t) t_nt;          // [max_templates] triangles
  IBL_G(int32_t) t_tri0;        // first template-triangle index
  IBL_G(int32_t) ttri;          // [max_template_edges][3] outward triangles, template-local nodes
  IBL_G(double) ta0;            // [max_template_edges] rest triangle area
  IBL_G(double) tav0;           // [max_templates][2] rest area, rest enclosed volume
  // control
  IBL_G(int64_t) step;          // completed steps (A/B parity = step & 1)
  IBL_G(int64_t) remaining;     // steps still to run in the current launch sequence
  IBL_G(uint32_t) health;
  IBL_G(double) red;            // [reduce items][4] partial sums
  IBL_G(double) red_out;        // [4] mass, momentum
};

// Work-item prefix tables of a launch set (one simulation or a batch).
struct Items {
  int32_t nsim;
  int32_t lat_total;         // bricks (every simulation)
  int32_t red_total;         // reduction items
  int32_t mesh_total;        // capsules
  int32_t cube_total;        // home cubes of simulations with capsules (interpolation) (interpolation)
  int32_t big_templates;     // 1 when a template exceeds the LDS force kernel
  int32_t forces_variant;    // 0: one LDS workgroup per capsule, 1: split edge / node kernels,
                             // 2: FP32 / FP16 storage through the edge-share LDS kernel
  int32_t membrane;          // 1 when some mesh has WLC-POW, area or volume terms
  int32_t moving_walls;      // 1 when some simulation has a wall layer with a non-zero velocity
  int32_t wall_cells;        // the largest wall-adjacent layer (cells) of those simulations
  int32_t rigid;             // 1 when some mesh is a rigid body
  int32_t morse;             // 1 when some simulation has the Morse repulsion on
  const int32_t* lat_off;    // [nsim + 1]
  const int32_t* red_off;
  const int32_t* mesh_off;
  const int32_t* cube_off;
  // Index of this timestep within a launch sequence of several: a simulation
  // takes part while its remaining count exceeds it, at parity (step + sub) & 1.
  // The counters advance once, after the sequence.
  int32_t sub;
};

// Phases of one timestep, in launch order.
enum Phase : int {
  kPhaseForces = 0,   // membrane forces, spreading records, candidate lists
  kPhaseLattice = 1,  // per brick: force spreading, moments, collision, streaming (u^n written)
  kPhaseInterp = 2,   // velocity interpolation and node update
  kPhaseAdvance = 3,  // step counter (one step; sequences advance once at their end)
  kNumPhases = 4
};

// Kernel launchers.  mode: 0 = timestep, 1 = observe.
// ibl_ib.hip: immersed-boundary phases.
void launch_forces(int storage, const SimDev* sims, const Items& it, int mode, hipStream_t s);
void launch_interp(int storage, const SimDev* sims, const Items& it, int mode, hipStream_t s);
// ibl_kernels.hip: lattice phases and dispatch.
hipError_t launch_init(int storage, const SimDev* sims, const Items& it, int init_axis_profile,
                       hipStream_t s);
hipError_t launch_template_rest(const SimDev* sim, int tmpl, int nedges, const double* xref,
                                hipStream_t s);
hipError_t launch_reset_lists(const SimDev* sim, int64_t nbrick, hipStream_t s);
hipError_t launch_phase(int storage, const SimDev* sims, const Items& it, int phase, int mode,
                        hipStream_t s);
// `steps` timesteps (mode 0) followed by one counter advance, or one
// observation (mode 1, steps = 1, no advance).
hipError_t launch_steps(int storage, const SimDev* sims, const Items& it, int steps, int mode, hipStream_t s);
hipError_t launch_reduce(int storage, const SimDev* sims, const Items& it, hipStream_t s);

}  // namespace ibl
