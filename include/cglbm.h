/*
 * cglbm.h -- C ABI of the MI355X (gfx950) hot path of the two-colour D3Q27
 * colour-gradient lattice Boltzmann model with generalized equilibria
 * (Saito, Takada, Baba, Someya, Ito, arXiv:2309.07801).
 *
 * One time step, per fluid node x (Sec. II, Sec. III.D-E):
 *   1. pull-streaming of the red and blue populations, f^k_i(x,t) =
 *      f^{k*}_i(x - c_i, t-1) (Eq. 5), full-way bounce-back at solid layers;
 *   2. colour densities, momentum, ideal-gas pressure and order parameter
 *      (Eqs. 10-14);
 *   3. isotropic gradient stencil (Eq. 20) of the order parameter, unit
 *      normal (Eq. 17), curvature (Eq. 16), CSF force (Eq. 15) and the
 *      correction term Q (Eq. 65);
 *   4. central-moment MRT collision of the total distribution with the
 *      velocity-independent generalized equilibrium moments (Eqs. 57-63,
 *      Eqs. 25 and 66-67), relaxation from the interpolated viscosity
 *      (Eqs. 21-22);
 *   5. recolouring (Eqs. 18-19).
 *
 * Conventions
 *   - Velocities are ordered as the columns of the matrix of Eq. (1).
 *   - Node index inside a box: x + nx*(y + ny*z); x fastest.  Boxes are
 *     concatenated; box b starts at node offset cglbm_box_offset(h, b).
 *     Offsets are multiples of 64; the arrays' length total_nodes (from
 *     cglbm_query_sizes) is an odd multiple of 64 and may exceed the last
 *     box's end by up to 127 nodes.
 *   - The state at time t is the pre-collision distribution f(x,t).  The
 *     library stores the post-collision distribution of step t-1 at x, so
 *     that a pull reproduces f(x,t).
 *   - All device pointers are caller-owned device memory (for instance torch
 *     tensors).  The library never frees caller memory; it owns only the
 *     handle, small parameter tables, a reduction scratch area, captured
 *     graphs and, for boxes with walls, the wall stashes of the in-place
 *     layout and of the compact schedule (populations of solid nodes only).
 *   - `stream` is a hipStream_t passed as void*.  Every call enqueues its work
 *     on that stream and returns without synchronizing, except where stated.
 *     For boxes with walls, the launch over the tiles near the solid layers
 *     runs on a stream of the handle (default priority) beside the one over
 *     the other tiles; it waits for the work enqueued on `stream` before it
 *     and `stream` waits for it, so the ordering seen by the caller is that
 *     of a single stream (also inside a graph captured from `stream`).
 *   - Return codes: CGLBM_OK (0) or a negative CGLBM_E* code; a message for
 *     the last failure on the calling thread is given by cglbm_last_error().
 *     No exception crosses the ABI.
 */
#ifndef CGLBM_H
#define CGLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGLBM_OK 0
#define CGLBM_EINVAL (-1)      /* bad sizes or parameters                     */
#define CGLBM_EHIP (-2)        /* a HIP runtime call failed                   */
#define CGLBM_EUNSUPPORTED (-3)/* valid by the paper, not built here          */
#define CGLBM_EUNSTABLE (-4)   /* non-finite values found in the state        */
#define CGLBM_ESTATE (-5)      /* call out of order / bad handle              */

/* Per-colour parameters: reference density rho_k^0 (Eq. 14), rest fraction
 * alpha_k with squared sound speed xi (1 - alpha_k), xi = 9/19 (Eq. 13), and
 * kinematic viscosity nu_k (Eq. 21). */
typedef struct {
  double rho0;
  double alpha;
  double nu;
} cglbm_phase;

/* Equilibrium families of Table I: A (Eq. 31, the standard second-order
 * equilibrium), B (Eq. 39), C (Eq. 48), D (Eq. 56, the generalized
 * equilibrium with velocity-independent central moments). */
typedef enum {
  CGLBM_MODEL_A = 0,
  CGLBM_MODEL_B = 1,
  CGLBM_MODEL_C = 2,
  CGLBM_MODEL_D = 3
} cglbm_model;

/* One box.  walls: bit0 = solid node layers at y = 0 and y = ny-1, bit1 =
 * solid layers at z = 0 and z = nz-1 (full-way bounce-back); other axes are
 * periodic.  sigma: interfacial tension of the CSF force (Eq. 15); beta:
 * recolouring parameter (Eq. 19); omega_bulk: omega_2 of Eq. (25);
 * omega_hi: omega_0 and omega_3..omega_10 of Eq. (25), each in (0, 2] (1 is
 * the paper's choice, Sec. III.E; other values relax every central moment
 * of the pulled distribution, a slower path of the three-kernel schedule);
 * body_force: constant force density added to the CSF
 * force; gravity, rho_ref: the buoyancy force -(rho - rho_ref) gravity of the
 * Rayleigh-Taylor case (Sec. IV.E), also added (zero gravity disables it);
 * model: a cglbm_model; q_correction: 1 adds the correction term Q of
 * Eq. (65) to the second-order relaxation, 0 omits it.  Model D with the
 * correction and unit higher-order rates runs the fused schedule; as soon as
 * one box uses another model, omits the correction or sets another rate,
 * every step of the handle runs the three-kernel
 * schedule (same update for the Model D boxes, bit for bit). */
typedef struct {
  int32_t nx, ny, nz;
  uint32_t walls;
  cglbm_phase red, blue;
  double sigma, beta;
  double omega_bulk;
  double omega_hi[9];
  double body_force[3];
  int32_t model;
  int32_t q_correction;
  double gravity[3];
  double rho_ref;
} cglbm_box_params;

/* Population storage formats.  Arithmetic is FP32 in all cases.
 *   CGLBM_FP32        54 float planes (colour c, direction i: plane 27c + i).
 *   CGLBM_FP32_PAIRS  the same values as CGLBM_FP32, bit for bit, stored as
 *                     27 planes of colour pairs (8 bytes: red, then blue):
 *                     faster for batches of small boxes, slower for large
 *                     ones (the same buffer sizes).
 *   CGLBM_FP16_SHIFT  the 26 moving directions of each colour in IEEE half,
 *                     stored as f^k_i - s^k_i with s^k_i = w_i rho_k^0
 *                     (c_s^k)^2 / c_s^2 (the pure-phase rest equilibrium of
 *                     colour k, rounded to half); rest populations in FP64.
 *   CGLBM_BF16_SHIFT  the same with bfloat16.
 *   CGLBM_FP32_EXACT  moving directions in float, rest populations in FP64.
 *   CGLBM_FP16_CSHIFT as CGLBM_FP16_SHIFT, with each moving population stored
 *                     as (f^k_i - c_k s^k_i) 2^-e_k: the shift scaled by the
 *                     colour fraction c_k = rho_k / rho of the node that
 *                     wrote it (red c_r, blue 1 - c_r; s^k_i unrounded), the
 *                     difference scaled exactly by a power of two,
 *                     e_k = floor(log2 rho_k^0) - 10, which keeps a colour's
 *                     small values (a light phase, the other phase's tail at
 *                     an interface) in the normal range of half down to about
 *                     6e-8 rho_k^0; the fraction is
 *                     stored per node as one more 16-bit plane (c_r in half,
 *                     correctly rounded from rho_r / rho: 1 and 0 exactly in
 *                     the pure phases).  A pull decodes each population with
 *                     the fraction of its source node x - c_i.  Pure phases
 *                     store deviations from equilibrium and the opposite
 *                     colour exact zeros, as with the constant shift; at the
 *                     interface each colour stores its deviation from its
 *                     share of the equilibrium instead of a remainder of the
 *                     order of s.  Solid
 *                     wall nodes re-encode the populations they reverse with
 *                     the fraction of their wall-normal fluid neighbour.
 *                     D3Q27 only.
 *   CGLBM_BF16_CSHIFT the same with bfloat16 (the fraction in bfloat16).
 * FP16_SHIFT, BF16_SHIFT, FP32_EXACT and the two CSHIFT formats store colour
 * pairs as well and carry the colour densities in FP64 from the pull to
 * the collision and set each rest population so that the node's colour mass
 * equals the FP64 sum of what the next step reads back: per-colour mass is
 * conserved to FP64 rounding (for the CSHIFT formats in boxes without walls:
 * the re-encoding at solid nodes rounds the reversed populations once more). */
typedef enum {
  CGLBM_FP32 = 0,
  CGLBM_FP16_SHIFT = 1,
  CGLBM_BF16_SHIFT = 2,
  CGLBM_FP32_EXACT = 3,
  CGLBM_FP32_PAIRS = 4,
  CGLBM_FP16_CSHIFT = 5,
  CGLBM_BF16_CSHIFT = 6
} cglbm_storage;

typedef struct cglbm_handle cglbm_handle;

/* Bytes the caller must provide: pop_bytes for EACH of the two population
 * buffers, aux_bytes for the auxiliary field buffer.  Pure host computation;
 * validates the parameters.  Returns CGLBM_EINVAL on bad parameters. */
int cglbm_query_sizes(int32_t n_boxes, const cglbm_box_params *boxes, int32_t storage,
                      size_t *pop_bytes, size_t *aux_bytes, int64_t *total_nodes);

/* Create a handle and write the initial state.
 * pop_a, pop_b: two device buffers of pop_bytes each, or pop_b = NULL for
 *   the in-place layout: one population buffer, which every step reads (in
 *   its pull) and then overwrites with the next state.  This is exact for
 *   the D3Q27 schedules because only the pull reads populations; solid wall
 *   nodes, whose reversed populations other nodes of the same pull still
 *   read, go through a small library-owned stash (allocated here, about
 *   pop_bytes / nodes x wall nodes) and a copy kernel after the pull.  The
 *   results are bit for bit those of the two-buffer layout.
 *   CGLBM_EUNSUPPORTED for a box with a higher-order rate other than 1
 *   (whose collision pulls the populations again).
 * aux: device buffer of aux_bytes.
 * init_rho_r, init_rho_b: device float arrays of total_nodes values (all
 *   boxes concatenated as described above; values in alignment gaps are
 *   ignored); init_u: device float array [3][total_nodes].  Each node gets
 *   f^k = (rho_k/rho) (f^eq(rho, p, u) + eta), with the Model D equilibrium of
 *   Eq. (56) (built from its central moments, Eqs. 57-63) and eta a
 *   SplitMix64 counter noise of amplitude noise_amp (0 disables it).
 *   rho = rho_r + rho_b must be > 0 everywhere (not checked on the device).
 * The handle is returned in *out.  Enqueued on stream; the caller keeps all
 * buffers alive until cglbm_destroy. */
int cglbm_init(cglbm_handle **out, int32_t n_boxes, const cglbm_box_params *boxes,
               int32_t storage, void *pop_a, void *pop_b, void *aux, const float *init_rho_r,
               const float *init_rho_b, const float *init_u, uint64_t noise_seed,
               double noise_amp, void *stream);

/* The two-dimensional lattice D2Q9 of App. A (Eqs. A1-A2, xi = 3/5 so that
 * (c_s^k)^2 = 3 (1 - alpha_k) / 5), with the generalized equilibrium of
 * Eq. (A10) (central moments Eqs. A12-A16), the colour-gradient steps of
 * Sec. II in two dimensions and the correction term Q of Eq. (65) per
 * component.  Same box parameters, buffers, fields, diagnostics and calls as
 * the D3Q27 handle, with these restrictions: nz = 1 and no z walls
 * (CGLBM_EINVAL otherwise); model CGLBM_MODEL_D, omega_hi all 1 and gravity
 * zero (CGLBM_EUNSUPPORTED otherwise); init_u is [3][total_nodes] with its z
 * plane ignored; z components of the fields are zero; the diagnostic R_eff
 * is (V/pi)^(1/2).  Populations: CGLBM_FP32 and CGLBM_FP32_PAIRS both keep 9
 * planes of colour pairs (2 x float, red first), 72 bytes per node, bit for
 * bit the same results; the mass-exact formats keep 8 planes of colour pairs
 * of the moving directions (2 x half or bfloat16 stored minus
 * w_i rho_k^0 (c_s^k)^2 / c_s^2 with the D2Q9 weights of Eq. (A2), or
 * 2 x float), then the two FP64 rest planes, with the mass closure described
 * for D3Q27 (48 or 80 bytes per node).  aux as for D3Q27 (with the FP64
 * colour densities after it for the mass-exact formats).
 * One launch per step (the pull, the interface stencils and the collision
 * of a tile in one kernel, so pop_b must not be NULL: CGLBM_EUNSUPPORTED);
 * cglbm_set_schedule accepts 0 only; variants are
 * its tile shapes (4 of them), chosen by cglbm_autotune, which writes their
 * times to ms_per_variant[0..3]. */
int cglbm_query_sizes_d2q9(int32_t n_boxes, const cglbm_box_params *boxes, int32_t storage,
                           size_t *pop_bytes, size_t *aux_bytes, int64_t *total_nodes);
int cglbm_init_d2q9(cglbm_handle **out, int32_t n_boxes, const cglbm_box_params *boxes,
                    int32_t storage, void *pop_a, void *pop_b, void *aux, const float *init_rho_r,
                    const float *init_rho_b, const float *init_u, uint64_t noise_seed,
                    double noise_amp, void *stream);

/* Lattice of a handle: 0 D3Q27 (cglbm_init), 1 D2Q9 (cglbm_init_d2q9), -1
 * for NULL. */
int cglbm_lattice(const cglbm_handle *h);

/* Tile shape of D2Q9 variant v (0..3): info[0] = x extent, info[1] = y
 * extent of the tile one 256-thread block updates.  CGLBM_EINVAL for other
 * v or a NULL info. */
int cglbm_variant_info_d2q9(int32_t v, int32_t *info);

/* Advance every box by n_steps time steps (steps 1-5 above).  Asynchronous. */
int cglbm_step(cglbm_handle *h, int32_t n_steps, void *stream);

/* Fields of the current state of box `box` into out_dev (device float,
 * [count][nodes_of_box]) in the order of the set bits of field_mask:
 *   bit 0 rho_r, 1 rho_b, 2 phi, 3 p, 4 ux, 5 uy, 6 uz (u includes F/2, Eq. 11),
 *   bit 7 nx, 8 ny, 9 nz (Eq. 17), 10 kappa (Eq. 16), 11 Fx, 12 Fy, 13 Fz
 *   (Eq. 15 plus body force), 14 Qx, 15 Qy, 16 Qz (Eq. 65).
 * Solid nodes report zeros for the interface fields.  Asynchronous. */
int cglbm_moments(cglbm_handle *h, int32_t box, uint32_t field_mask, float *out_dev,
                  void *stream);

/* Per-box diagnostics in FP64, deterministic (a fixed summation order that
 * depends only on the box: never on the launch geometry, the other boxes of
 * the handle or the schedule).  Definitions follow Sec. IV.A (Laplace's law,
 * Eq. 68 in its three-dimensional form 2 sigma / R) and Eqs. 10-14.
 * centre: host array of 3 doubles per box (droplet centre used for the
 * Laplace measurement and the periodic centroid) or NULL (box centre).
 * out: per box CGLBM_NDIAG doubles:
 *   0 M_r, 1 M_b (sums of rho_k over fluid nodes), 2-4 momentum sum rho*u,
 *   5 p_in (mean p where |x-c| < R_eff-3), 6 p_out (mean p where
 *   |x-c| > R_eff+5, periodic distance), 7 R_eff = (3V/4pi)^(1/3) with
 *   V = sum (1+phi)/2, 8-10 red centroid relative to c, 11 kinetic energy
 *   sum rho u^2/2, 12 count of fluid nodes whose pulled local moments
 *   (densities, momentum, second moments) are not all finite.
 * out_is_host != 0: out is host memory; the call synchronizes the stream and
 *   returns CGLBM_EUNSTABLE if any box's count of non-finite values is
 *   nonzero (out is filled either way).
 * out_is_host == 0: out is device memory of n_boxes * CGLBM_NDIAG doubles;
 *   the call only enqueues work on the stream (no host synchronization), so
 *   it cannot inspect the result: the caller reads the non-finite count
 *   from out[13 b + 12].
 * The library's reduction buffers are allocated by cglbm_init. */
#define CGLBM_NDIAG 13
int cglbm_reduce(cglbm_handle *h, const double *centre, double *out, int32_t out_is_host,
                 void *stream);

/* The diagnostics of cglbm_reduce (same kernels, same summation order, the
 * same values bit for bit) for callers that cannot allocate device memory:
 * work captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  The call allocates nothing and never synchronizes: its
 * reduction scratch is a static device array of the library (8.5 MiB per
 * GPU, held until the process ends), used for at most 65536 reduction chunks
 * of 16384 nodes (about 1.07e9 nodes) and 4096 boxes; larger handles get
 * CGLBM_EINVAL (use cglbm_reduce).  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other streams, other threads, other
 * handles) race and must be ordered by the caller.
 * centre: device array of 3 doubles per box, or NULL for the box centres.
 * out: device array of n_boxes * CGLBM_NDIAG doubles (layout of
 * cglbm_reduce); out[13 b + 12] is box b's count of non-finite values.
 * CGLBM_ESTATE for a NULL handle, CGLBM_EINVAL for a NULL out. */
int cglbm_reduce_noalloc(cglbm_handle *h, const double *centre, double *out, void *stream);

/* Node offset of box b in the concatenated arrays, or -1. */
int64_t cglbm_box_offset(const cglbm_handle *h, int32_t box);

/* Checkpoint and resume.  The state of every box is the content of one of
 * the two population buffers (which one alternates with the step parity);
 * aux holds only fields derived from it, and the initial noise enters only
 * through it.  cglbm_state_buffer returns that buffer (pop_a or pop_b, a
 * device pointer to pop_bytes), valid until the next cglbm_step (and, with a
 * resident compact state, only after cglbm_sync_state); NULL for a NULL
 * handle.  A copy of it ordered after the work enqueued so far is a
 * checkpoint.  cglbm_load_state copies pop_bytes from the device buffer src
 * into the state buffer of h, on stream (asynchronous); h must have been
 * created with the same boxes, storage and lattice as the run that wrote the
 * checkpoint (the library cannot check this).  Stepping on from a loaded
 * checkpoint gives bit for bit the results of the uninterrupted run.
 * CGLBM_ESTATE for a NULL handle, CGLBM_EINVAL for a NULL src. */
void *cglbm_state_buffer(const cglbm_handle *h);
int cglbm_load_state(cglbm_handle *h, const void *src, void *stream);

/* Launch schedule of a step (0 and 1 compute the same update, bit for bit):
 *   0 (default) two launches: pull-streaming with local moments, then one
 *     column-marching kernel for the interface stencils and the collision;
 *   1 three launches: pull, LDS-tiled interface stencils, collision;
 *   2 compact: the same update with the state between the steps of one
 *     cglbm_step call held as each node's compact post-collision state
 *     (17 floats: rho_r, rho_b, u, F, the six relaxed second-order central
 *     moments and n; with unit higher-order rates the collided, recoloured
 *     populations of Eqs. 66-67 and 18-19 are a function of them).  Each
 *     step is a column-marching pull that rebuilds the collided populations
 *     of a column and its ring in registers and sums the streamed moments
 *     (Eq. 5), then the fused kernel writing compact states: about 224 bytes
 *     per node and step instead of 520.  The first step of a call pulls the
 *     stored populations and the call ends by storing the populations again
 *     (one extra launch per call), so the stored state, the fields, the
 *     diagnostics and checkpoints are those of schedule 0.  Results equal
 *     schedule 0 bit for bit for one step per call and to FP32 rounding
 *     otherwise (the moment sums run in another order).  Layouts: D3Q27,
 *     two buffers, unit higher rates, and either CGLBM_FP32 or
 *     CGLBM_FP32_PAIRS storage with any equilibrium family and Q switch
 *     (Model D with Q runs the fused kernel; the others the interface and
 *     collide kernels, writing compact states; one step per call then
 *     equals schedule 1 bit for bit), or CGLBM_FP32_EXACT storage with
 *     Model D and Q (the compact state then carries the FP64 colour
 *     densities as well, 84 bytes per node, and per-colour mass stays
 *     exact to FP64 rounding), or one of the 16-bit storages with Model D
 *     and Q: the same compact state, so that within a call the state is
 *     held in FP32 and FP64 and rounded to the 16-bit format only when the
 *     call stores the populations (a call of n steps rounds once, not n
 *     times; one step per call equals schedule 0 bit for bit on boxes
 *     without walls; the solid nodes' populations are re-encoded once per
 *     call); CGLBM_EUNSUPPORTED otherwise.  The compact state
 *     lives in the population buffer that does not hold the state; solid
 *     wall nodes keep their (bounced) populations in two library-owned
 *     wall stashes allocated by cglbm_init.  cglbm_autotune chooses
 *     between 0 and 1 only (select 2 after it); for layouts that admit 2 it
 *     also times the compact fused kernel and pull per geometry and keeps
 *     the fastest for schedule 2.
 * Selecting a schedule loads the fused geometry the autotuner chose for it
 * (or the one cglbm_set_variant set); when that changes the geometry the
 * call synchronizes the device first.
 * Returns CGLBM_EINVAL for other values. */
int cglbm_set_schedule(cglbm_handle *h, int32_t schedule);

/* Schedule the next step runs: 0, 1 or 2 as above (1 whenever a box needs
 * the three-kernel schedule), -1 for a NULL handle. */
int cglbm_get_schedule(const cglbm_handle *h);

/* Resident compact state (schedule 2 only; the moment-representation variant
 * of the update, Sec. II with Eqs. 66-67, kept across calls).  With enable =
 * 1, a schedule-2 call of cglbm_step no longer stores the populations at its
 * end: the compact state of its last step stays in the other population
 * buffer (and the wall stashes), and the next schedule-2 call continues from
 * it without the population pull.  A sequence of calls then gives bit for
 * bit the results of one call of as many steps.  Until the state is stored,
 * the buffer cglbm_state_buffer returns is stale.  It is stored (one launch
 * on the given stream, after which the next call starts from the
 * populations again) by cglbm_sync_state, by cglbm_set_resident with enable
 * = 0, and, before they read the state, by cglbm_moments, cglbm_reduce,
 * cglbm_reduce_noalloc, cglbm_autotune and a cglbm_step in another schedule;
 * cglbm_set_schedule, cglbm_set_variant, cglbm_set_wall_mode and
 * cglbm_set_compact_variant store it on the stream of the last step first.
 * cglbm_load_state discards it.  The caller keeps these calls on the stream
 * of the steps (or orders the streams), as for every other reader.  Has no
 * effect in schedules 0 and 1 and for D2Q9.  Default 0.  CGLBM_ESTATE for a
 * NULL handle, CGLBM_EINVAL for enable other than 0 or 1.
 * cglbm_get_resident returns 1 or 0, -1 for a NULL handle; cglbm_sync_state
 * returns CGLBM_OK when there is nothing to store. */
int cglbm_set_resident(cglbm_handle *h, int32_t enable, void *stream);
int cglbm_get_resident(const cglbm_handle *h);
int cglbm_sync_state(cglbm_handle *h, void *stream);

/* Geometry of the compact schedule's pull: returns its index (-1 for a NULL
 * handle) and, if info is not NULL, writes info[0] = x extent, info[1] =
 * y extent of a block's column, info[2] = its z chunk.  cglbm_autotune
 * chooses it (equal results) whenever the layout admits schedule 2. */
int cglbm_compact_variant(const cglbm_handle *h, int32_t *info);
/* Select the compact pull geometry v (0..4); synchronizes the stream.
 * CGLBM_EINVAL for other v. */
int cglbm_set_compact_variant(cglbm_handle *h, int32_t v, void *stream);

/* Graph execution of cglbm_step: 1 (default) runs pairs of time steps as one
 * captured HIP graph (captured on first use on a private stream of default
 * priority, launched on the caller's stream; captured again after
 * cglbm_set_variant or cglbm_set_schedule; an odd last step is launched
 * directly); 0 launches every kernel directly.  Both give bitwise identical
 * results.  While per-kernel profiling is active steps are launched directly.
 * Returns CGLBM_EINVAL for other values. */
int cglbm_set_graph(cglbm_handle *h, int32_t enable);

/* Launch geometries of the fused kernel (all bitwise equivalent).
 * cglbm_num_variants: how many; cglbm_variant_info: info[0..3] = column
 * extent x, y, z chunk, minimum waves per SIMD; cglbm_set_variant selects one
 * for every schedule (synchronizes the stream); cglbm_get_variant returns
 * the one loaded (the current schedule's: the autotuner keeps one for
 * schedules 0 and 1 and one for schedule 2). */
int cglbm_num_variants(void);
int cglbm_variant_info(int32_t variant, int32_t *info);
int cglbm_set_variant(cglbm_handle *h, int32_t variant, void *stream);
int cglbm_get_variant(const cglbm_handle *h);

/* Wall mode of the tiled launches (fused kernel, compact pull) over boxes
 * with walls, whose tiles within the kernel's reach of a solid layer run a
 * kernel with the wall logic and the others one without it.  Bit 0: the
 * slabs next to z walls form short chunks of their own (else the first and
 * last chunk of every column are near-wall tiles); bit 1: the near-wall
 * launch runs on the handle's side stream beside the other (else after it
 * on the caller's stream).  All four modes give bitwise identical results.
 * cglbm_set_wall_mode selects one for every schedule (synchronizes the
 * device; CGLBM_EINVAL outside 0..3, CGLBM_EUNSUPPORTED for D2Q9 handles);
 * cglbm_autotune chooses one per schedule for layouts with walls and two
 * buffers; cglbm_get_wall_mode returns the one loaded (3 until chosen), -1
 * for a NULL handle. */
int cglbm_set_wall_mode(cglbm_handle *h, int32_t mode, void *stream);
int cglbm_get_wall_mode(const cglbm_handle *h);

/* Autotuner: time every fused variant and the three-kernel schedule `reps`
 * times on the current state (the stored state is not advanced: the kernels
 * after the pull are re-run on the same inputs; in the in-place layout they
 * all write the next state into the one buffer, so the call advances the
 * state by exactly one step) and select the fastest
 * geometry and schedule (the three-kernel schedule wins on boxes too small to
 * fill the GPU with fused columns).  ms_per_variant (optional, length
 * cglbm_num_variants() + 1) receives the mean milliseconds per launch of
 * each fused variant, then of the interface + collide pair.  For layouts
 * with walls and two buffers it then times the four wall modes with the
 * chosen geometries, as replays of a captured graph (the fused kernel; for
 * schedule 2 k_cpull with the compact collision, advancing only the compact
 * state in the other buffer) and keeps the fastest per schedule.
 * Synchronizes the stream. */
int cglbm_autotune(cglbm_handle *h, int32_t reps, double *ms_per_variant, void *stream);

/* Per-kernel timing with HIP events recorded on the caller's stream around
 * every launch of the step.  begin: reserve room for max_launches launches;
 * end: synchronize the events and return, per kernel kind
 * (0 pull/moments: k_pull, or k_cpull in the compact schedule; 1 interface;
 * 2 collide; 3 fused interface+collide, the compact fused kernel in the
 * compact schedule; 4 the population pull that starts a compact call; 5 the
 * emission of populations that ends a compact call), the total milliseconds
 * and the number of launches timed.  Kinds beyond n_kinds are not
 * reported. */
int cglbm_profile_begin(cglbm_handle *h, int32_t max_launches);
int cglbm_profile_end(cglbm_handle *h, double *total_ms, int64_t *launches, int32_t n_kinds);

/* Release the handle and library-owned memory (never caller buffers). */
void cglbm_destroy(cglbm_handle *h);

/* Message of the last failure on the calling thread ("" if none). */
const char *cglbm_last_error(void);

/* Library version string. */
const char *cglbm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CGLBM_H */
