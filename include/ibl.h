/*
 * ibl.h -- C-ABI of libibl.so, an MI355X (gfx950) implementation of the
 * coupled immersed-boundary lattice-Boltzmann timestep of Tan, Sinno &
 * Diamond, arXiv:1704.04551.
 *
 * One timestep (Sec. 2.1-2.3 of the paper), in this order:
 *   1. membrane forces F(X^n): linear springs 1/2 ks (l - l0)^2 per edge and the
 *      dihedral bending energy kb (1 - cos(theta - theta0)) of Eq. (8);
 *   2. force spreading g(x) = sum_k F_k delta(x - X_k), Eq. (15), with the
 *      cosine kernel of Eq. (16) or Peskin's 4-point kernel;
 *   3. moments rho = sum f_i, rho u = sum f_i c_i + (g_body + g)/2, Eq. (3);
 *   4. velocity interpolation U_k = sum_x u(x) delta(x - X_k), Eq. (14);
 *   5. node update X^{n+1} = X^n + U_k (unit time step, FP64);
 *   6. D3Q19 BGK collision with the forcing term of Eq. (4), Eq. (1)-(2);
 *   7. streaming, periodic or halfway bounce-back walls (moving-wall term
 *      -6 w_i (c_i . u_wall)).
 *
 * Conventions shared by every call:
 *   - Lattice cell (x, y, z) sits at position (x, y, z); x varies fastest in
 *     every field array.  A wall axis has solid layers at index 0 and n-1;
 *     the fluid occupies 1 .. n-2 and the effective walls lie at 0.5 and n-1.5.
 *   - Node coordinates are FP64, array-of-structures [n_nodes][3], unwrapped
 *     (a capsule may cross a periodic boundary); on a wall axis every node must
 *     satisfy 1 <= X < n - 2.
 *   - Every call returns an ibl_status; 0 is success.  Invalid arguments return
 *     IBL_ERR_ARG and leave all state unchanged.  Asynchronous failures detected
 *     on the device (non-finite values, a node leaving the admissible range, a
 *     candidate-list overflow) are latched in a per-simulation health word and
 *     reported by ibl_sync() / ibl_conservation() as IBL_ERR_UNSTABLE or
 *     IBL_ERR_STATE.  ibl_last_error() gives a message for the calling thread.
 *   - Host buffers are owned by the caller and only read or written during the
 *     call.  The device arena passed to ibl_sim_create is owned by the caller
 *     and must outlive the simulation; the library only sub-allocates it.
 *   - A simulation is not thread-safe; it runs on one HIP stream.
 */
#ifndef IBL_H
#define IBL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  IBL_OK = 0,
  IBL_ERR_ARG = -1,         /* invalid argument; nothing changed */
  IBL_ERR_NOMEM = -2,       /* arena too small or capacity exceeded */
  IBL_ERR_DEVICE = -3,      /* a HIP runtime call failed */
  IBL_ERR_STATE = -4,       /* a node left the admissible range / list overflow */
  IBL_ERR_UNSTABLE = -5,    /* non-finite populations or node positions, rho <= 0 */
  IBL_ERR_UNSUPPORTED = -6  /* valid request that this library does not implement */
} ibl_status;

/* Population storage.  Every mode stores the offset of each population from
 * its rest equilibrium, h_i = f_i - w_i, so that low-Mach populations keep
 * their significant bits.
 *   - Collision arithmetic: FP64 for IBL_F64; for IBL_F32 the moments and the
 *     O(u) part of each post-collision value in FP64, the O(u^2) and forcing
 *     terms in FP32; FP32 for IBL_F16_OFFSET.
 *   - Stores of the timestep round stochastically (up with probability equal
 *     to the discarded fraction, to within 2^-16 of an ulp for binary32 and
 *     2^-13 for binary16) with random bits hashed from (cell, step,
 *     population), so runs are bitwise reproducible.  Values below the
 *     format's normal range, and the initial state, round to nearest.
 *   - Node positions and the conservation sums are FP64 in every mode.
 *     Membrane forces are computed in FP64; with FP32 / FP16 storage each
 *     node's sum is formed in 64-bit fixed point (2^-40 lattice units) and
 *     the spreading carries it as binary32. */
typedef enum {
  IBL_F64 = 0,        /* h_i as binary64 (parity form) */
  IBL_F32 = 1,        /* h_i as binary32 */
  IBL_F16_OFFSET = 2  /* 2^16 h_i as binary16: the exact power-of-two scale puts
                         offsets from 2^-30 to 0.9995 in binary16's normal range */
} ibl_storage;

/* One-dimensional delta kernel phi(r), 4-point support (Sec. 2.3). */
typedef enum {
  IBL_DELTA_COS = 0,     /* Eq. (16): 1/4 (1 + cos(pi r / 2)), |r| <= 2 */
  IBL_DELTA_PESKIN4 = 1  /* Peskin's 4-point kernel (zero first moment) */
} ibl_delta;

/* Health word bits (ibl_sync, ibl_conservation).  The timestep latches the
 * population bits (non-finite, rho, Mach) per fluid cell and the node bits per
 * node as it runs; ibl_conservation re-checks the stored populations. */
#define IBL_HEALTH_NONFINITE_F 0x1u  /* a population is NaN or Inf */
#define IBL_HEALTH_RHO 0x2u          /* rho <= 0 in a fluid cell */
#define IBL_HEALTH_MACH 0x4u         /* |u| > 0.3 in a fluid cell */
#define IBL_HEALTH_NODE_RANGE 0x8u   /* a node left 1 <= X < n-2 on a wall axis */
#define IBL_HEALTH_OVERFLOW 0x10u    /* a brick's candidate list overflowed */
#define IBL_HEALTH_NONFINITE_X 0x20u /* a node position is NaN or Inf */
#define IBL_HEALTH_FORCE_RANGE 0x40u /* a membrane force share was NaN or beyond
                                        its fixed-point range: 2048 lattice
                                        units for spring and bending shares
                                        (FP32 / FP16 storage), 32 for area,
                                        volume and WLC-POW shares; or a bond
                                        reached its WLC maximum length */

typedef struct {
  int32_t n[3];            /* cells per axis, each >= 4 */
  double tau;              /* BGK relaxation time, > 1/2; nu = (tau - 1/2)/3, Eq. (5) */
  double g_body[3];        /* uniform body-force density added to every fluid cell */
  int32_t wall[3];         /* per axis: 0 periodic, 1 solid layers at 0 and n-1 */
  double wall_u_lo[3][3];  /* [axis][component] velocity of the layer at index 0 */
  double wall_u_hi[3][3];  /* [axis][component] velocity of the layer at index n-1 */
  int32_t storage;         /* ibl_storage */
  int32_t delta;           /* ibl_delta */
  int32_t init_profile;    /* 0: fluid at rest; 1: linear profile between the wall
                              layers of the highest-index wall axis (Couette) */
  int32_t max_nodes;       /* capacity: Lagrangian nodes over all meshes */
  int32_t max_meshes;      /* capacity: meshes (capsules) */
  int32_t max_templates;   /* capacity: distinct mesh templates */
  int32_t max_template_nodes; /* capacity: nodes summed over templates */
  int32_t max_template_edges; /* capacity: edges summed over templates */
  int32_t brick_x;         /* lattice brick width along x: 16, 32 or 64 cells (bricks are
                              brick_x x 256/brick_x x 4 cells, 8 deep for FP16 storage,
                              one workgroup each), or 0
                              for the widest that the x extent fills.  A tuning knob:
                              results are bitwise identical across widths. */
  int32_t skin;            /* candidate lists of the spreading (node binning): 0 rebuilds
                              them every step; 1 builds them with a one-cell skin around
                              each node's stencil and rebuilds only after some node's
                              stencil base has moved more than one cell from where it was
                              at the last build.  A tuning knob: results are bitwise
                              identical either way. */
  int32_t morse;           /* 1: reserve the neighbour grid of the inter-capsule Morse
                              repulsion (ibl_sim_morse), (n/2)^3 cells of at least 2
                              lattice units, at most 2^31 of them (IBL_ERR_ARG
                              beyond); 0: none */
} ibl_sim_desc;

typedef struct ibl_sim_s* ibl_sim;
typedef struct ibl_batch_s* ibl_batch;

/* Device-arena bytes a simulation with this description needs (populations,
 * velocity and force fields, node arrays, candidate lists, templates).
 * Errors: IBL_ERR_ARG for an invalid description. */
ibl_status ibl_sim_bytes(const ibl_sim_desc* desc, size_t* out_bytes);

/* Create a simulation inside a caller-owned device arena of arena_bytes (at
 * least ibl_sim_bytes) on the current HIP device, and initialise the
 * populations to equilibrium at rho = 1 and the initial velocity (Sec. 2.1).
 * hip_stream: the hipStream_t to run on, or NULL for a stream the library
 * creates (non-blocking, default priority) and destroys.
 * Errors: IBL_ERR_ARG (tau <= 1/2, n < 4 or > 32767, bad enums, skin not 0 or 1, brick_x not
 * 0/16/32/64, 2 x cells x element bytes >= 4 GiB), IBL_ERR_NOMEM (arena too
 * small), IBL_ERR_DEVICE. */
ibl_status ibl_sim_create(const ibl_sim_desc* desc, void* dev_arena, size_t arena_bytes,
                          void* hip_stream, ibl_sim* out);

ibl_status ibl_sim_destroy(ibl_sim sim);

/* The hipStream_t the simulation runs on. */
void* ibl_sim_stream(ibl_sim sim);

/* Register a membrane template: a closed surface of n_nodes nodes and n_tris
 * outward (counter-clockwise seen from outside) triangles, host int32
 * [n_tris][3], and its stress-free reference coordinates x_ref, host FP64
 * [n_nodes][3].  The rest length l0 of every edge and the rest bending angle
 * theta0 of every edge (Eq. (8)) come from x_ref.  Both arrays are copied.
 * Errors: IBL_ERR_ARG (not a closed, consistently oriented manifold),
 * IBL_ERR_NOMEM (template capacity), IBL_ERR_UNSUPPORTED (more nodes than one
 * workgroup handles). */
ibl_status ibl_template_add(ibl_sim sim, int32_t n_nodes, int32_t n_tris, const int32_t* tris,
                            const double* x_ref, int32_t* out_template);

/* Add a capsule (Sec. 2.2): an instance of a template with current node
 * positions x, host FP64 [n_nodes][3] (copied), spring constant ks and
 * bending constant kb.  Errors: IBL_ERR_ARG (bad template id, node outside the
 * admissible range on a wall axis), IBL_ERR_NOMEM (node/mesh capacity). */
ibl_status ibl_mesh_add(ibl_sim sim, int32_t template_id, const double* x, double ks, double kb,
                        int32_t* out_mesh);

/* Add a rigid body (Sec. 2.3, Eq. (17)): the template's closed surface at node
 * positions x, host FP64 [n_nodes][3] (copied), which fix the body's shape
 * and initial pose, moving as one body of uniform density `density` (the
 * fluid's is 1) with initial velocity v0[3] and angular velocity w0[3]
 * (either may be NULL: zero).  The body counts as a mesh (its index is
 * returned in out_mesh; ibl_read_nodes gives its node positions, rigid-body
 * node velocities and FSI forces on the fluid).  Each step:
 *   - the fluid velocity before the immersed-boundary force, u* = (sum f c +
 *     g_body / 2) / rho, is interpolated at every node X_k (Eq. (14));
 *   - the FSI force of Eq. (17), rho_f (u* - U_k) / dt with rho_f = dt = 1,
 *     U_k = v + Omega x (X_k - x_c), times the node's weight (a third of its
 *     triangles' areas times one lattice spacing) acts on the body, and its
 *     opposite is spread onto the fluid (Eq. (15));
 *   - Newton's second law with the summed force and torque about the centre
 *     of mass, semi-implicit Euler with dt = 1: v += F / M, L += T,
 *     x_c += v, the orientation turned by |Omega| about Omega = R I^-1 R^T L;
 *     mass, centre of mass and inertia tensor are those of the uniform solid
 *     the surface bounds.
 * Errors: IBL_ERR_ARG (bad template, density <= 0, non-finite values, a node
 * outside the admissible range, a surface enclosing no volume),
 * IBL_ERR_NOMEM (node or mesh capacity). */
ibl_status ibl_body_add(ibl_sim sim, int32_t template_id, const double* x, double density, const double* v0,
                        const double* w0, int32_t* out_mesh);

/* State of a rigid body at the current time N, out[19] host FP64: centre of
 * mass [0..2], orientation quaternion (w, x, y, z) relative to the pose given
 * at ibl_body_add [3..6], velocity [7..9], angular velocity [10..12], and the
 * hydrodynamic force [13..15] and torque about the centre of mass [16..18] of
 * Eq. (17) at state N.  Synchronous.  Errors: IBL_ERR_ARG (not a body). */
ibl_status ibl_read_body(ibl_sim sim, int32_t mesh, double* out);

/* Add the rest of the paper's membrane energy, Eq. (6), to a capsule (all
 * zero after ibl_mesh_add; zero: term absent).  They add to the springs and
 * bending of ibl_mesh_add (pass ks = 0 there for the paper's model):
 *   kbt_p  WLC-POW stretching, Eq. (7), C = kBT / p: maximum bond length
 *          l_m = 2 l0, and the repulsive constant k_p = 5/4 C l0^2 that makes
 *          every bond force-free at its rest length l0;
 *   kg, kl global and local area constraints, Eq. (9), rest areas from x_ref;
 *   kv     volume constraint, Eq. (10), rest volume enclosed by x_ref.
 * A bond at or beyond l_m sets IBL_HEALTH_FORCE_RANGE and adds no force; so
 * does a share component beyond 32 lattice units (it is clamped).  Node forces
 * are summed in 64-bit fixed point at 2^-46 lattice units (reproducible, and
 * the same for templates of any size: above 642 nodes the sums are kept in
 * HBM instead of LDS).  Set the terms before ibl_batch_create on a batch
 * holding the simulation.  Errors: IBL_ERR_ARG (unknown mesh or a rigid body,
 * a negative or non-finite constant, a reference shape with a degenerate
 * triangle or no enclosed volume for a term that needs it). */
ibl_status ibl_mesh_membrane(ibl_sim sim, int32_t mesh, double kbt_p, double kg, double kl, double kv);

/* Inter-capsule repulsion (Sec. 2.2, Eq. (13)): the Morse potential
 * U(r) = D0 [exp(-2 alpha (r - r0)) - 2 exp(-alpha (r - r0))] for r < rc between
 * the nodes of different capsules (rigid bodies do not take part), distances
 * by minimum image on periodic axes.  Its force on each node is added to the
 * membrane force before spreading.  D0 = 0 turns it off.  Neighbours are
 * found on a grid of cells at least 2 lattice units wide, at most 48 nodes per
 * cell (IBL_HEALTH_OVERFLOW beyond); pair forces are summed per node in
 * two-word 64-bit fixed point (units 2^-44 and 2^-96 lattice units: exact to
 * 2^-96 per pair), so the sums are reproducible and the pair forces cancel
 * exactly; a pair force component beyond 128 sets IBL_HEALTH_FORCE_RANGE and
 * is clamped.  Set before ibl_batch_create on a batch holding the
 * simulation.  Errors: IBL_ERR_ARG (negative or non-finite
 * D0, alpha <= 0, rc <= 0), IBL_ERR_UNSUPPORTED (rc > 2 lattice units, or a
 * simulation created with morse = 0). */
ibl_status ibl_sim_morse(ibl_sim sim, double D0, double alpha, double r0, double rc);

/* Advance n_steps coupled timesteps, asynchronously on the simulation's
 * stream (replayed HIP graphs).  State afterwards: (f^N, X^N). */
ibl_status ibl_step(ibl_sim sim, int64_t n_steps);

/* Wait for the stream; report latched device failures (the health word:
 * IBL_ERR_UNSTABLE for non-finite values, rho <= 0, |u| > 0.3 or a force out
 * of range; IBL_ERR_STATE for a node out of range or a list overflow). */
ibl_status ibl_sync(ibl_sim sim);

/* Observables at the current time N, computed with the membrane force at X^N
 * (steps 1-3 above) without changing the state.  Host FP64 outputs, caller
 * allocated, any may be NULL: rho [ncell], u [3][ncell], g [3][ncell] (g is
 * g_body + spread force).  Solid cells report rho = 0, u = 0, g = 0.
 * Synchronous. */
ibl_status ibl_read_fields(ibl_sim sim, double* rho, double* u, double* g);

/* Node observables of one mesh at time N: positions X^N, interpolated
 * velocities U^N (step 4 above) and membrane forces F^N, host FP64
 * [n_nodes][3] each, any may be NULL.  Synchronous. */
ibl_status ibl_read_nodes(ibl_sim sim, int32_t mesh, double* x, double* u, double* f);

/* FP64 mass sum_fluid sum_i f_i, momentum sum_fluid sum_i f_i c_i of the
 * stored populations, and the health word (IBL_HEALTH_* bits, latched since
 * creation).  Synchronous.  Returns IBL_ERR_UNSTABLE / IBL_ERR_STATE when the
 * health word is non-zero (outputs are still written). */
ibl_status ibl_conservation(ibl_sim sim, double* mass, double momentum[3], uint32_t* health);

/* Checkpoint: bytes of the serialized state (populations in storage format,
 * node positions, rigid-body states, step counter). */
ibl_status ibl_state_bytes(ibl_sim sim, size_t* out_bytes);
/* Copy the state to a caller-owned host buffer of at least ibl_state_bytes.  */
ibl_status ibl_read_state(ibl_sim sim, void* host_buf, size_t bytes);
/* Restore a state written by ibl_read_state of a simulation with the same
 * description and meshes.  Errors: IBL_ERR_ARG on a size or header mismatch. */
ibl_status ibl_write_state(ibl_sim sim, const void* host_buf, size_t bytes);

/* Number of completed timesteps. */
ibl_status ibl_step_count(ibl_sim sim, int64_t* out_steps);

/* Phase timing, the GPU counterpart of the paper's coupling-cost table
 * (Table 1): run n_steps timesteps (1 .. 100000) on the simulation's stream,
 * launched one phase at a time with a HIP event after each, and return the
 * mean milliseconds per step of every phase in ms_out[0..3] -- 0 membrane
 * forces, spreading records and candidate lists, 1 force spreading
 * (Eq. (15)) fused with collision and streaming, 2 velocity interpolation
 * (Eq. (14)) and node update, 3 step counter -- and the total elapsed
 * milliseconds of the run in ms_out[4].  ms_out holds 5 doubles.  The state
 * advances by n_steps.  Synchronous. */
ibl_status ibl_profile_phases(ibl_sim sim, int64_t n_steps, double* ms_out);

/* Batching: many independent simulations advanced by one launch per kernel
 * phase over a flattened work list, each step captured once in a HIP graph.
 * All simulations must share one storage type and the HIP device; the batch
 * runs on the first simulation's stream.  The batch holds a small device
 * table it allocates itself.  Results of every simulation are bitwise those
 * it gets alone.  The member simulations must outlive the batch: destroy the
 * batch before any of them (ibl_batch_destroy waits on the first member's
 * stream). */
ibl_status ibl_batch_create(const ibl_sim* sims, int32_t n_sims, ibl_batch* out);
/* Advance simulation i by steps_per_sim[i] >= 0 steps (uneven allowed). */
ibl_status ibl_batch_step(ibl_batch batch, const int64_t* steps_per_sim);
ibl_status ibl_batch_destroy(ibl_batch batch);

/* The batch advance of ibl_batch_create + ibl_batch_step + ibl_batch_destroy in
 * one call that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it).  Simulation i advances steps_per_sim[i] >= 0 steps, with results
 * bitwise those of ibl_batch_step (and of each simulation alone).
 *   - The batch's device tables (the members' descriptors, the work-item
 *     prefix tables) live in a static device array of the library, sized for
 *     at most 64 simulations (about 110 KB, held on each GPU the library runs
 *     on until the process ends).  Every call on a GPU reuses that GPU's
 *     array: calls that overlap on one GPU (on different streams) race.
 *   - Kernels are launched directly on the first simulation's stream (no
 *     graph: instantiating one allocates).  Work pending on the other
 *     members' streams must be complete before the call; the call does not
 *     order those streams.
 *   - Asynchronous: ibl_sync on the first simulation waits for it.
 * Errors: IBL_ERR_ARG (null or repeated simulation, mixed storage or device,
 * n_sims outside 1 .. 64, a negative step count), IBL_ERR_DEVICE. */
ibl_status ibl_batch_step_static(const ibl_sim* sims, int32_t n_sims, const int64_t* steps_per_sim);

/* Calibration of the memory system, outside the method: a plain streaming
 * copy of `bytes` bytes from device buffer src to device buffer dst (16-byte
 * vector loads and stores, every workgroup striding over the whole range), on
 * hip_stream (null: the default stream), asynchronous.  Its duration gives
 * the practical HBM ceiling against which the kernels' bandwidth is read, and
 * its profiler byte counters the scale factor of theirs.  Errors:
 * IBL_ERR_ARG (null buffer, a size or an address not a multiple of 16),
 * IBL_ERR_DEVICE. */
ibl_status ibl_hbm_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Message describing the last error on the calling thread ("" if none). */
const char* ibl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IBL_H */
