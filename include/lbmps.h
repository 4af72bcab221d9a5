/*
 * lbmps -- lattice Boltzmann particle suspensions on one AMD MI355X (gfx950).
 *
 * C-ABI of the hot path of Rettinger & Ruede, "A comparative study of
 * fluid-particle coupling methods for fully resolved lattice Boltzmann
 * simulations" (arXiv:1702.04910): the D3Q19 stream-collide sweep (Sec. 2.1)
 * coupled to rigid spheres by the momentum exchange method (Sec. 2.2: BB,
 * CLI, refill) or the partially saturated cells method (Sec. 2.3: M1B1, M2B2,
 * M3B2), the per-particle force/torque reduction and the explicit Euler
 * rigid-body update (Sec. 4.1).
 *
 * Conventions
 *  - Lattice units: dx = dt = rho0 = 1, c_s^2 = 1/3 (Sec. 2.1).  The box is
 *    periodic in x, y and z; cell (i, j, k) has its centre at (i+1/2, j+1/2, k+1/2).
 *  - Velocity order q = 0..18 (see lbmps_velocities): rest, then opposite pairs
 *    (q odd, q + 1).  Weights 1/3, 1/18 (axis), 1/36 (diagonal).
 *  - Host PDF arrays hold deviations g_q = f_q - w_q, FP64, index
 *    [q][z][y][x] (x fastest), i.e. g[q*N + (z*ny + y)*nx + x], N = nx*ny*nz.
 *    They are the canonical PDFs f(x, t): after streaming and boundary
 *    handling, before collision.  Solid MEM cells and wall cells read as 0.
 *  - Vectors are (x, y, z).  Host field arrays: rho[N], u[3][N].
 *  - Device memory: the library allocates none.  The caller passes one device
 *    workspace of at least lbmps_workspace_bytes() bytes (e.g. a torch uint8
 *    CUDA tensor) that must outlive the context, and a hipStream_t on which
 *    every kernel and copy is enqueued.  Host buffers are caller-owned and are
 *    copied before the call returns.
 *  - Calls on one context are not thread-safe; distinct contexts are
 *    independent.  No C++ exception crosses this interface.
 *  - Errors: every call returns an lbmps_status; lbmps_last_error() gives the
 *    message of the last failure on that context.  Device-side conditions
 *    (capacity overflow, instability) are detected asynchronously and reported
 *    by the next synchronising call (get_*, lbmps_sync).
 */
#ifndef LBMPS_H
#define LBMPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbmps_status;
#define LBMPS_OK 0
#define LBMPS_EINVAL (-1)       /* invalid argument or configuration */
#define LBMPS_ENOMEM (-2)       /* workspace too small or a list capacity exceeded */
#define LBMPS_EDEVICE (-3)      /* HIP runtime error */
#define LBMPS_EUNSTABLE (-4)    /* non-finite force/velocity or a particle moving >= 1 cell per rigid-body step */
#define LBMPS_ESTATE (-5)       /* call out of order */
#define LBMPS_EUNSUPPORTED (-6) /* feature not available in this build */

/* collision operator of the fluid (Eq. LBM_SRT / Eq. MEM_TRT) */
#define LBMPS_BGK 0
#define LBMPS_TRT 1
/* coupling (Sec. 2.2 / Sec. 2.3) */
#define LBMPS_NONE 0
#define LBMPS_MEM_BB 1  /* momentum exchange, bounce-back, Eq. MEM_BB */
#define LBMPS_MEM_CLI 2 /* momentum exchange, central linear interpolation, Eq. MEM_CLI */
#define LBMPS_PSM 3     /* partially saturated cells, Eq. PSM with psm_m, psm_b */
/* PDF storage precision (compute is FP64 for FP64 storage, FP32 otherwise) */
#define LBMPS_FP64 0
#define LBMPS_FP32 1
#define LBMPS_FP16_DEV 2 /* IEEE half deviations g = f - w, round to nearest even (stochastically in
                            PSM-overlapped cells) */
#define LBMPS_BF16_DEV 3 /* bfloat16 deviations g = f - w; post-collision values rounded stochastically */
/* reconstruction of uncovered MEM cells (Sec. 2.2.3) */
#define LBMPS_REFILL_EXTRAPOLATE 0
#define LBMPS_REFILL_EQUILIBRIUM 1
/* solid-fraction estimator (Sec. 2.3.2) */
#define LBMPS_EPS_FLAT 0      /* eps_n^3 sub-cell sample points, every point tested */
#define LBMPS_EPS_RECURSIVE 1 /* same points, octree blocks classified at once (eps_n power of 2) */
#define LBMPS_EPS_LEARNED 2   /* cells cut by the surface: the network of lbmps_set_eps_model inside its
                                 radius range, flat eps_n^3 supersampling outside it */
#define LBMPS_EPS_EDGE 3      /* covered share of the cell's 12 edges (alternative named in Sec. 2.3.2) */
#define LBMPS_EPS_DISTANCE 4  /* 1/2 - (|x_c - X| - R) clamped to [0, 1]: surface distance of the cell
                                 centre (alternative named in Sec. 2.3.2).  Modes 2-4 store eps_s as the
                                 nearest count out of eps_n^3 (ties to even). */

typedef struct lbmps_config {
  int32_t nx, ny, nz;  /* periodic box (cells) */
  int32_t collision;   /* LBMPS_BGK or LBMPS_TRT */
  int32_t coupling;    /* LBMPS_NONE, LBMPS_MEM_BB, LBMPS_MEM_CLI, LBMPS_PSM */
  int32_t psm_m;       /* 1, 2, 3: solid operator, Eqs. PSM_M1..M3 */
  int32_t psm_b;       /* 1, 2: weighting, Eqs. PSM_B1, PSM_B2 */
  int32_t n_sub;       /* LBM sweeps per rigid-body step, forces averaged over them (Sec. 2.2.4, Sec. 4.1);
                          0 = 2 for MEM, 1 for PSM (Alg. 2) */
  int32_t eps_n;       /* supersampling points per axis (default 8) */
  int32_t eps_mode;    /* LBMPS_EPS_FLAT .. LBMPS_EPS_DISTANCE */
  int32_t precision;   /* LBMPS_FP64 .. LBMPS_BF16_DEV */
  int32_t max_particles;
  int32_t tile_rows;     /* x-rows per sweep workgroup (0 = automatic) */
  int32_t block_threads; /* sweep workgroup size, <= 256 (0 = 256) */
  int32_t grid_blocks;   /* sweep workgroups; 0 = one per tile, > 0 = persistent grid of that size */
  int32_t wall_link_cap; /* capacity of static-wall links (0 = automatic) */
  int32_t sweep_flags;   /* launch tuning only, results unchanged: bit 0 non-temporal loads in the sweep;
                            bit 1 collide PSM cells of a single particle inside the sweep (reads the cell map
                            of every cell; shared cells are collided after the sweep);
                            bit 2 collide them in a pass over the overlap list after the sweep;
                            bit 3 the sweep built for six waves per SIMD (FP32/FP16/BF16 storage);
                            bit 4 collide them in a pass over the overlap list before the sweep, into a
                            staging array that the sweep pushes (reads the cell map of every cell);
                            bits 1, 2, 4 are exclusive; with none of them the library stages when the
                            spheres (diameter D + 2) cover at least 1 % of the PSM cells, else uses bit 2;
                            bits 5-6: at most 3 (value 1) or 2 (value 2) sweep workgroups per CU, by
                            reserving LDS (value 3 is invalid);
                            bit 7 two x-adjacent cells per sweep thread, moved as one word per direction
                            (needs an even nx; ignored with bit 3 and while bit 1 or 4 is in effect);
                            bit 8 four x-adjacent cells per sweep thread, one 8-byte word per direction
                            (FP16/BF16 storage and nx a multiple of 4 only; not with bits 3 or 7; ignored
                            while bit 1 or 4 is in effect) */
  int32_t refill;        /* MEM reconstruction of uncovered cells (Sec. 2.2.3): LBMPS_REFILL_EXTRAPOLATE (0, the
                            paper's: extrapolation along the surface normal, then fallbacks) or
                            LBMPS_REFILL_EQUILIBRIUM (1: every uncovered cell takes the last fallback,
                            f^eq(rho_bar, v)); both then impose the velocity */
  double max_diameter;   /* largest particle diameter that will be set (cells) */
  double nu;             /* kinematic viscosity, nu = (tau - 1/2)/3 (Eq. Viscosity) */
  double magic;          /* TRT parameter Lambda (default 3/16 when 0) */
  double f_ext[3];       /* body force density (Eq. Forcing) */
  double gravity[3];     /* gravitational acceleration acting on (rho_p - 1) V of each particle */
} lbmps_config;

typedef struct lbmps_particle {
  double X[3];     /* centre */
  double U[3];     /* translational velocity */
  double Omega[3]; /* angular velocity */
  double D;        /* diameter (cells) */
  double rho_p;    /* density (fluid density is 1) */
  int32_t fixed;   /* 1: held in place (no rigid-body update) */
  int32_t pad;
} lbmps_particle;

typedef struct lbmps_particle_state {
  double F[3];     /* hydrodynamic force of the last rigid-body step, averaged over its n_sub sweeps */
  double T[3];     /* hydrodynamic torque, same averaging */
  double U[3], Omega[3], X[3];
} lbmps_particle_state;

typedef struct lbmps_ctx lbmps_ctx;

/* Velocity table of the library's q order: c[q][0..2]. */
void lbmps_velocities(int32_t c[19][3]);

/* Bytes of device workspace needed by one instance / a batch of n instances.
 * Pure; returns 0 for an invalid configuration. */
size_t lbmps_workspace_bytes(const lbmps_config* cfg);
size_t lbmps_batch_workspace_bytes(int32_t n, const lbmps_config* cfgs);

/* Create a context for one instance (lbmps_create) or for n independent
 * instances advanced together by every lbmps_step (lbmps_batch_create; all
 * instances share the storage precision; MEM instances share n_sub, and so
 * do PSM instances).
 * dev_workspace: caller-owned device memory of `bytes` >= the size above.
 * hip_stream: a hipStream_t (may be NULL for the default stream).
 * Errors: EINVAL (config), ENOMEM (workspace too small), EDEVICE. */
lbmps_status lbmps_create(const lbmps_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
                          lbmps_ctx** out);
lbmps_status lbmps_batch_create(int32_t n, const lbmps_config* cfgs, void* dev_workspace, size_t bytes,
                                void* hip_stream, lbmps_ctx** out);
void lbmps_destroy(lbmps_ctx* ctx);

/* Set every fluid cell of instance `inst` (0 for lbmps_create contexts) to the
 * equilibrium f^eq(rho, u) of Eq. LBM_EQ.  Asynchronous. */
lbmps_status lbmps_init_equilibrium(lbmps_ctx* ctx, int32_t inst, double rho, const double u[3]);

/* Mark the cells with host_mask[cell] != 0 as one group of static wall cells
 * moving with v_wall, handled by half-way bounce-back (Eq. MEM_BB).  Call
 * before lbmps_set_particles.  Up to 16 groups per instance.
 * Errors: EINVAL, ENOMEM (wall_link_cap exceeded). */
lbmps_status lbmps_set_static_solid(lbmps_ctx* ctx, int32_t inst, const uint8_t* host_mask, const double v_wall[3]);

/* Mark the cells with host_mask[cell] != 0 as one group of outflow cells of
 * instance `inst` (the top of the settling-sphere frame, Sec. 4.1): for every
 * direction q from a fluid cell x into the group, after streaming,
 *   f_qbar(x, t+1) = -f~_q(x, t) + 2 f^eq,+_q(rho_out, u(x, t)),
 * the pressure anti-bounce-back with the even part of Eq. LBM_EQ,
 * f^eq,+_q = w_q (rho_out + 9/2 (c_q.u)^2 - 3/2 u.u), and u(x, t) the velocity of
 * Eq. MacVel from the cell's PDFs before its collision.  Outflow cells are
 * never fluid (fields and PDFs read as for walls) and take one of the 16 wall
 * groups of the instance.  The velocity inflow of the frame is a static wall
 * group moving with the inflow velocity (lbmps_set_static_solid).  Call before
 * lbmps_set_particles.
 * Errors: EINVAL (null mask, rho_out not positive and finite, more than 16
 * groups), ENOMEM (wall_link_cap exceeded), ESTATE (particles already set). */
lbmps_status lbmps_set_outflow(lbmps_ctx* ctx, int32_t inst, const uint8_t* host_mask, double rho_out);

/* Change the kinematic viscosity of instance `inst`: tau (Eq. Viscosity),
 * the TRT/BGK rates and, for PSM, the B2 weights of the current overlaps are
 * recomputed (the Galileo-number calibration of Sec. 4.1 adjusts nu between
 * runs).  Synchronising.  Errors: EINVAL (nu not positive and finite). */
lbmps_status lbmps_set_viscosity(lbmps_ctx* ctx, int32_t inst, double nu);

/* Change the gravitational acceleration of instance `inst` (acting on
 * (rho_p - 1) V of each particle).  Synchronising.  Errors: EINVAL. */
lbmps_status lbmps_set_gravity(lbmps_ctx* ctx, int32_t inst, const double g[3]);

/* Replace the particles of instance `inst` (n <= max_particles) and map them
 * into the lattice (MEM: solid cells and links; PSM: solid fractions).
 * Positions are wrapped into the box.  Particles must not touch each other
 * (there is no contact model).
 * Errors: EINVAL if n > max_particles, D <= 0, D > max_diameter,
 * D + 6 > min(nx, ny, nz), rho_p <= 0 or any value is non-finite. */
lbmps_status lbmps_set_particles(lbmps_ctx* ctx, int32_t inst, int32_t n, const lbmps_particle* host);

/* Advance every instance by n_steps LBM time steps (Alg. 1 / Alg. 2);
 * n_steps must be a multiple of every n_sub in the context.  Asynchronous.
 * A rigid-body step that would move a particle by a cell or more, or give it
 * a non-finite state, is not taken (the particle keeps its position and
 * velocities) and is reported as LBMPS_EUNSTABLE by the next synchronising
 * call; the fluid state after it is not meaningful.
 * Within one call, when its stream is not being captured, the PSM list
 * rebuild and the MEM remap after a rigid-body step run (one after the other)
 * on a second stream of the library beside the next sweep, which then leaves
 * the PSM cells to the overlap kernel after it whatever sweep_flags select;
 * results are bit-identical to running them in order.  That stream waits for
 * the caller's stream, and the caller's stream waits for it before the call
 * returns, so all of the call's work stays ordered on the caller's stream. */
lbmps_status lbmps_step(lbmps_ctx* ctx, int32_t n_steps);

/* For callers that cannot allocate device memory or create HIP objects
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): lbmps_step without any allocation.  Same arguments, results and
 * errors as lbmps_step, bit for bit, except that
 *  - the per-chunk force and torque sums of the reduction (partial results
 *    that lbmps_step keeps in the context's workspace) go to a static device
 *    array of LBMPS_NOALLOC_SCRATCH_BYTES bytes per GPU, which each GPU holds
 *    from the first call until the process ends;
 *  - every kernel runs in order on the context's stream (no second stream and
 *    no event is created);
 *  - it calls no hipMalloc, hipFree, stream or event creation.
 * The context's device must be current.  The array is shared by every call on
 * one GPU and keeps the last call's contents; nothing carries over from one
 * call to the next, so calls in sequence are safe, but calls that overlap in
 * time on one GPU (contexts on different streams, or threads) race and give
 * wrong forces.
 * Errors: as lbmps_step; ENOMEM when the context needs more scratch than
 * LBMPS_NOALLOC_SCRATCH_BYTES (48 bytes per chunk sum: ceil-sized chunk rows
 * of every PSM particle, n_sub sets of link chunk rows of every MEM particle);
 * ESTATE when timing is on or another device is current. */
#define LBMPS_NOALLOC_SCRATCH_BYTES (4u << 20)
lbmps_status lbmps_step_noalloc(lbmps_ctx* ctx, int32_t n_steps);

/* Change the sweep launch shape of an existing context (workgroup size, grid:
 * 0 = one workgroup per tile, > 0 persistent; flags as sweep_flags).  Results
 * do not depend on it.  Drops a captured graph. */
lbmps_status lbmps_set_launch(lbmps_ctx* ctx, int32_t block_threads, int32_t grid_blocks, int32_t sweep_flags);

/* Same as lbmps_step, replayed from a HIP graph: the launch sequence of one
 * period of sweeps (even, and a multiple of every n_sub) is captured on the
 * context's stream at the first call and replayed n_steps/period times.  The
 * capture is redone after lbmps_set_particles / lbmps_set_static_solid.
 * Needs a non-default stream; timing must be off.  Asynchronous.
 * Errors: EINVAL (n_steps not a multiple of the period), ESTATE. */
lbmps_status lbmps_step_graph(lbmps_ctx* ctx, int32_t n_steps);

/* Block until the stream is idle; report device-side errors. */
lbmps_status lbmps_sync(lbmps_ctx* ctx);

/* Particle state of instance `inst` (n must equal the number set).  Synchronising. */
lbmps_status lbmps_get_particles(lbmps_ctx* ctx, int32_t inst, int32_t n, lbmps_particle_state* host);

/* rho[N] and u[3][N] of instance `inst`: Eq. MacVel in fluid cells, Eq. MacVel_PSM
 * in cells overlapped by PSM particles, rho = 1, u = 0 in solid MEM and wall
 * cells.  Synchronising. */
lbmps_status lbmps_get_fields(lbmps_ctx* ctx, int32_t inst, double* rho, double* u);

/* Canonical PDF deviations of instance `inst` (19*N doubles, layout above).
 * get: solid and wall cells read 0.  set: overwrites every cell.  Synchronising. */
lbmps_status lbmps_get_pdfs(lbmps_ctx* ctx, int32_t inst, double* host_g);
lbmps_status lbmps_set_pdfs(lbmps_ctx* ctx, int32_t inst, const double* host_g);

/* Current boundary links (MEM) of all instances: cell index, q (x + c_q is
 * solid), particle (global index) and delta_q; n_out receives the count.
 * Writes at most cap entries.  Synchronising. */
lbmps_status lbmps_get_links(lbmps_ctx* ctx, int64_t cap, int32_t* cell, int32_t* q, int32_t* particle,
                             double* delta, int64_t* n_out);
/* Current PSM overlaps of all instances: cell, particle (global index), eps_s. */
lbmps_status lbmps_get_overlaps(lbmps_ctx* ctx, int64_t cap, int32_t* cell, int32_t* particle, double* eps,
                                int64_t* n_out);

/* Measurement hook: with enable = k > 0, every k-th sweep-kernel launch of
 * lbmps_step from now on (the first included) is bracketed by HIP events
 * recorded on the context's stream; 0 switches timing off, k < 0 is
 * LBMPS_EINVAL.  set_timing resets the totals; get_timing synchronises and
 * returns the summed kernel time (ms) and the number of launches timed. */
lbmps_status lbmps_set_timing(lbmps_ctx* ctx, int32_t enable);
lbmps_status lbmps_get_timing(lbmps_ctx* ctx, double* sweep_ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * Learned solid fraction.  Supersampling (Sec. 2.3.2) costs eps_n^3 point
 * tests per cell cut by a sphere surface and is redone after every
 * rigid-body step of moving particles (the cost Sec. 2.3.4 discusses).  A
 * multilayer perceptron 8 -> 64 -> 64 -> 1 (ReLU hidden layers) replaces it
 * for cut cells; cells entirely inside or outside a sphere stay exact.
 * Inputs of a cell with centre displacement d from a sphere of radius R:
 * |d| - R, then |d_x|/|d|, |d_y|/|d|, |d_z|/|d| sorted descending, then 8/R,
 * then three zeros.
 * Products run in bfloat16 (round to nearest even) on the matrix cores with
 * FP32 accumulation; parameters are FP32.  Parameter blob
 * (LBMPS_MLP_NPARAM floats): W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
 * Prediction y = W3 . relu(W2 relu(W1 x + b1) + b2) + b3; as eps_s it is
 * clamped to [0, 1] and rounded to the nearest multiple of 1/eps_n^3 (so
 * that every estimator yields sample counts). */
#define LBMPS_MLP_NPARAM 4801
#define LBMPS_MLP_MAX_BATCH 65536

/* Install the network used by LBMPS_EPS_LEARNED instances for particles with
 * r_min <= R <= r_max (host_params: LBMPS_MLP_NPARAM floats, copied).  Other
 * radii fall back to flat supersampling.  Required before lbmps_set_particles
 * on such instances; remaps current PSM particles.  Synchronising.
 * Errors: EINVAL (null, non-finite, r_min > r_max), EDEVICE. */
lbmps_status lbmps_set_eps_model(lbmps_ctx* ctx, const float* host_params, double r_min, double r_max);

/* Recompute solid fractions and overlap lists of every PSM particle at the
 * current positions (what each rigid-body step of moving particles does).
 * Asynchronous; for timing the estimator. */
lbmps_status lbmps_rebuild_overlaps(lbmps_ctx* ctx);

/* Judge of the learned estimator: every `stride`-th cut cell that the network
 * evaluated in the last rebuild is recounted by flat eps_n^3 supersampling.
 * out[0] = mean |eps_net - eps_exact|, out[1] = max, out[2] = cells judged.
 * Synchronising.  Errors: EINVAL (stride < 1). */
lbmps_status lbmps_eps_judge(lbmps_ctx* ctx, int32_t stride, double out[3]);

/* Trainer of the network (independent of any lattice context).  Training
 * samples are cells (R, d); targets are exact flat supersampling counts.
 * Device memory: one caller-owned workspace of lbmps_mlp_workspace_bytes()
 * for up to max_samples samples. */
typedef struct lbmps_mlp lbmps_mlp;
size_t lbmps_mlp_workspace_bytes(int64_t max_samples);
lbmps_status lbmps_mlp_create(int64_t max_samples, void* dev_workspace, size_t bytes, void* hip_stream,
                              lbmps_mlp** out);
void lbmps_mlp_destroy(lbmps_mlp* m);
/* Parameters in and out (host, LBMPS_MLP_NPARAM floats); set resets the
 * optimiser state.  Synchronising. */
lbmps_status lbmps_mlp_set_params(lbmps_mlp* m, const float* host);
lbmps_status lbmps_mlp_get_params(lbmps_mlp* m, float* host);
/* Training set: n rows (R, d_x, d_y, d_z), FP64, host.  Features are formed
 * on the device.  Clears the targets.  Errors: EINVAL (n out of range, R <= 0). */
lbmps_status lbmps_mlp_set_samples(lbmps_mlp* m, int64_t n, const double* host_rd);
/* Inputs in use: 5 (default: |d| - R, the three sorted direction cosines,
 * 8/R) or 3 (|d| - R and the two largest direction cosines, without the
 * curvature term: the three-input variant the network's design is compared
 * with).  Unused inputs are set to zero, so their weights get no gradient; a
 * network trained with 3 inputs from zero weights on inputs 3 and 4 evaluates
 * the same with all features present.  Recomputes the current samples'
 * features.  Errors: EINVAL (n_inputs not 3 or 5). */
lbmps_status lbmps_mlp_set_inputs(lbmps_mlp* m, int32_t n_inputs);
/* Targets: eps_s of every sample by flat supersampling with eps_n^3 points
 * (count / eps_n^3, rounded to FP32). */
lbmps_status lbmps_mlp_label(lbmps_mlp* m, int32_t eps_n);
lbmps_status lbmps_mlp_set_targets(lbmps_mlp* m, const float* host);
lbmps_status lbmps_mlp_get_targets(lbmps_mlp* m, float* host);
/* Clamped network output for every sample (host, n floats). */
lbmps_status lbmps_mlp_predict(lbmps_mlp* m, float* host_y);
/* Gradient of the batch loss L = (1/B) sum_k (y(s_k) - t(s_k))^2 (unclamped y)
 * with respect to every parameter, over the samples
 * s_k = (((b0 + k) mod n) * mult + add) mod n, k < B = batch; mult must be
 * coprime to n, 0 <= add < n, 1 <= batch <= LBMPS_MLP_MAX_BATCH. */
lbmps_status lbmps_mlp_gradient(lbmps_mlp* m, int64_t b0, int32_t batch, int64_t mult, int64_t add,
                                float* host_grad);
typedef struct lbmps_mlp_train_cfg {
  int32_t epochs;        /* passes over the training set */
  int32_t batch;         /* samples per Adam step, <= LBMPS_MLP_MAX_BATCH */
  float lr, beta1, beta2, adam_eps;
  const int64_t* mult;   /* per epoch: sample order s -> (s*mult + add) mod n (the caller's random draw) */
  const int64_t* add;
} lbmps_mlp_train_cfg;
/* Adam on the batch loss above, ceil(n / batch) steps per epoch.  Asynchronous. */
lbmps_status lbmps_mlp_train(lbmps_mlp* m, const lbmps_mlp_train_cfg* cfg);
const char* lbmps_mlp_last_error(const lbmps_mlp* m);

/* Global index of particle 0 of instance `inst`. */
int32_t lbmps_particle_base(const lbmps_ctx* ctx, int32_t inst);

const char* lbmps_status_string(lbmps_status s);
const char* lbmps_last_error(const lbmps_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBMPS_H */
