/*
 * mrfv.h -- C ABI of the MI355X (gfx950) hot path of the block-based multiresolution
 * finite-volume solver of Hoppe, Adami & Adams (arXiv 2012.04385) for the 3D
 * compressible Euler equations (eq:Euler with the stiffened-gas EOS eq:StiffenedGas), with
 * optional gravity and viscous terms and Tait's equation of state.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an mrfv_status (0 = success, negative = error), never throws,
 *    never aborts.  On an argument error nothing is written to device memory and the
 *    reason is available from mrfv_last_error().
 *  - "dev" pointers are HIP device pointers owned by the caller (for instance the storage
 *    of torch tensors); the library never frees them.  "host" pointers are ordinary host
 *    memory.  Tables, work lists and scratch inside the context are owned by the library
 *    and released by mrfv_destroy().
 *  - Kernels are launched asynchronously on the stream given to mrfv_create().  Calls
 *    that return host-visible results (mrfv_init_blocks, mrfv_commit_flags, mrfv_step when
 *    it adapts the tree, mrfv_get_blocks) synchronise that stream.
 *  - Block storage (the paper's block concept, Sec. "Modular block-based MR algorithm"):
 *    a block is 16^3 interior cells plus 4 halo layers per side.  The state array U holds
 *    one padded block per slot: U[slot][q][z][y][x], 24^3 per quantity, x fastest,
 *    interior index 4..19, q = (rho, rho u, rho v, rho w, E).  U0 and L hold interiors
 *    only: [slot][q][16][16][16].  The element type is the context dtype (float or
 *    double).
 *  - A context is used by one host thread at a time.
 */
#ifndef MRFV_H
#define MRFV_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MRFV_OK = 0,
    MRFV_EINVAL = -1,    /* bad argument (null pointer, size, index)                  */
    MRFV_EHIP = -2,      /* a HIP runtime call failed                                 */
    MRFV_ENOMEM = -3,    /* slot capacity or device memory exhausted                  */
    MRFV_ESTATE = -4,    /* call out of order (e.g. step before init)                 */
    MRFV_ENONPHYS = -5   /* rho <= 0, p + B <= 0 or a NaN appeared on the device       */
} mrfv_status;

typedef enum { MRFV_F32 = 0, MRFV_F64 = 1 } mrfv_dtype;

/* Flux kernels of Sec. "Numerical Scheme" (the combinations of the weak-scaling runs):
 * Roe with WENO5-JS (the standard configuration: per characteristic field, upwind when the
 * two face cells' eigenvalues agree in sign, else a local Lax-Friedrichs split), Roe with
 * TENO5, local Lax-Friedrichs (Rusanov; every field split, speeds from the two face cells)
 * with WENO5-JS, and HLLC with WENO-AO(5,3) face states (characteristic-wise). */
typedef enum { MRFV_ROE_WENO5 = 0, MRFV_ROE_TENO5 = 1, MRFV_LLF_WENO5 = 2,
               MRFV_HLLC_WAO53 = 3 } mrfv_scheme;

/* Equation of state (Sec. "Governing Equations"; Sec. "Influence of Equation of State").
 * MRFV_TAIT: p = B ((rho/rho0)^gamma - 1) + A depends on the density alone; the energy is
 * a dependent variable, is not evolved and stays zero (the initial pressure is unused).
 * The flux is the standard configuration's characteristic WENO5-JS Roe solver with
 * per-field LLF fallback on the four fields (u-c, u, u, u+c), Roe c~^2 = (p_R - p_L) /
 * (rho_R - rho_L).  Tait runs on the plain kernels: contexts with it must use scheme
 * MRFV_ROE_WENO5, no gravity, no proposer, and not the fused FP32 path (batched with
 * MRFV_F32); mrfv_create returns MRFV_EINVAL otherwise. */
typedef enum { MRFV_STIFFENED_GAS = 0, MRFV_TAIT = 1 } mrfv_eos;
/* External boundaries per axis: periodic; zero gradient (every halo layer a copy of the
 * boundary cell); symmetry (the halo is the mirror image of the interior with the
 * momentum normal to the boundary reversed: a slip wall, the symmetry planes of the
 * paper's Rayleigh-Taylor and implosion cases); fixed values (each halo layer holds a
 * given state, uniform over the boundary plane: mrfv_instance.bc_fixed; the top and
 * bottom of the Rayleigh-Taylor case).  Where halo layers of several boundary axes meet
 * (edges, corners), the axes apply in the order x, y, z, each over the whole padded
 * extent of the others. */
typedef enum { MRFV_BC_PERIODIC = 0, MRFV_BC_ZEROGRAD = 1, MRFV_BC_SYMMETRY = 2,
               MRFV_BC_FIXED = 3 } mrfv_bc;

/* One independent MR problem (one forest of octrees on a box). */
typedef struct {
    double gamma, B;      /* stiffened-gas EOS parameters                               */
    double cfl;           /* CFL number of eq:Cfl                                       */
    double eps;           /* threshold on the finest level; eq:LevelWiseEpsilon scales it
                             by 2^(-3 (lmax - l)) on level l                            */
    double scale_rho;     /* normalisation of rho details                               */
    double scale_E;       /* normalisation of E details                                 */
    double dx0;           /* cell size on level 0                                       */
    int32_t lmax;         /* finest level                                               */
    int32_t n0[3];        /* level-0 blocks per axis                                    */
    int32_t bc[3];        /* mrfv_bc per axis                                           */
    int32_t adapt;        /* 1: refine/coarsen after each step                          */
    double gravity[3];    /* source term of eq:Euler: S(U) = (0, rho g, rho v . g); zero
                             vector: no source                                          */
    int32_t eos;          /* mrfv_eos; the same for every instance of a context          */
    double tait_A, tait_rho0;   /* Tait: p = B ((rho/rho0)^gamma - 1) + A (gamma, B above) */
    double mu;            /* dynamic viscosity (>= 0; 0: Euler equations).  With mu > 0
                             the flux carries the viscous terms of the Navier-Stokes
                             equations: Newtonian stress with Stokes' hypothesis, tau =
                             mu (grad v + grad v^T) - 2/3 mu (div v) I, flux (0, tau_d.,
                             tau_d. . v) subtracted from the convective one, no heat
                             conduction; second-order central differences at the faces
                             (normal: the two cells sharing the face; tangential: the mean
                             of their central differences).  dt is then also bounded by
                             cfl * 3/16 * dx_lmax^2 * min(rho) / mu.  Viscous contexts
                             (any instance with mu > 0) run on the plain kernels and fill
                             all 26 halo regions of the leaves every stage (the
                             tangential derivatives read the edge halos); mrfv_create
                             returns MRFV_EINVAL for one on the fused FP32 path (batched
                             with MRFV_F32), mrfv_step_lts returns MRFV_EINVAL for one. */
    const double *bc_fixed;   /* host, read by mrfv_create only; required when some axis
                             has MRFV_BC_FIXED, else ignored (may be NULL): primitive states
                             (rho, u, v, w, p) of the halo cells beyond the sides of those
                             axes, [6 sides: x-, x+, y-, y+, z-, z+][lmax + 1 levels]
                             [4 layers, the one at the face first][5], converted with the
                             instance's EOS like the initial condition               */
} mrfv_instance;

typedef struct {
    int32_t dtype;          /* mrfv_dtype of U, U0, L                                   */
    int32_t n_instances;    /* >= 1                                                     */
    int32_t slot_capacity;  /* maximum number of blocks over all instances              */
    int32_t batched;        /* 0: plain path (one launch per tree level, unfused update);
                               1: batched path (all leaves of all levels and instances in
                               one fused rhs + update launch; fused for FP32 only);
                               2: batched path with the CFL step and the three RK stages
                               replayed from one hipGraph (captured on first use, valid
                               across tree changes; FP32)                              */
    int32_t scheme;         /* mrfv_scheme: the flux kernel of every leaf               */
} mrfv_config;

typedef struct mrfv_ctx mrfv_ctx;

/* Initial-condition callback: fill prim[5][16][16][16] (rho,u,v,w,p at the interior cell
 * centres, [q][z][y][x]) of block (instance, level, bx, by, bz). Host memory. */
typedef void (*mrfv_ic_fn)(void *user, int32_t instance, int32_t level, int32_t bx,
                           int32_t by, int32_t bz, double *prim);

/* Create a context.  inst: host array of cfg->n_instances problems.  hip_stream: the
 * stream every kernel is launched on (NULL = default stream).  Allocates the library's
 * tables and scratch for cfg->slot_capacity slots. */
int mrfv_create(mrfv_ctx **out, const mrfv_config *cfg, const mrfv_instance *inst,
                void *hip_stream);
int mrfv_destroy(mrfv_ctx *ctx);
const char *mrfv_last_error(const mrfv_ctx *ctx);

/* Size in bytes of U (padded) and of U0 / L (interiors) for the configured capacity. */
int64_t mrfv_state_bytes(const mrfv_ctx *ctx);
int64_t mrfv_interior_bytes(const mrfv_ctx *ctx);

/* init_blocks -- bottom-up initialisation of algo:Init: level-0 forest, then level by
 * level: refine all blocks of the previous level, impose the initial condition (ic,
 * converted to conservative variables on the device), and on levels >= 2 remove sibling
 * groups whose details are all below that level's threshold; finally parents are set to
 * the average of their children (eq:Averaging).  U: dev, capacity-sized padded state. */
int mrfv_init_blocks(mrfv_ctx *ctx, mrfv_ic_fn ic, void *user, void *U);

/* fill_halos -- halo cells of every block, levels coarse to fine: copy from a same-level
 * neighbour (periodic boundaries wrap), else fifth-order prediction from the parent
 * (eq:Prediction), with zero-gradient boundaries clamped to the nearest interior cell.
 * All 26 halo regions (4 layers) are filled. */
int mrfv_fill_halos(mrfv_ctx *ctx, void *U);

/* rhs_stage -- L = -div F for every leaf (eq:Euler, Sec. "Numerical Scheme"): one flux
 * per face from characteristic WENO5-JS inside a Roe solver with local Lax-Friedrichs
 * fallback per characteristic field, with the coarse flux at resolution jumps replaced by
 * the area average of the fine fluxes (coarse cell adjustment of algo:ComputeLoop).
 * Halos must be filled.  L: dev [slot][5][16^3] (written for leaves only). */
int mrfv_rhs_stage(mrfv_ctx *ctx, const void *U, void *L);

/* rk_update -- SSP-RK3 stage (increment form) on every leaf interior:
 * U <- U0 + a_s ((U - U0) + dt L), a = (1, 1/4, 2/3); stage 0 first copies U into U0.
 * dt_dev: dev double[n_instances] (from mrfv_cfl_dt).  Sets the device error word on a
 * non-physical state (see mrfv_check). */
int mrfv_rk_update(mrfv_ctx *ctx, int32_t stage, const double *dt_dev, void *U, void *U0,
                   const void *L);

/* mr_project -- every non-leaf block <- conservative average of its 8 children
 * (eq:Averaging), levels fine to coarse, summed pairwise in double precision. */
int mrfv_mr_project(mrfv_ctx *ctx, void *U);

/* mr_predict -- interiors of the listed blocks <- fifth-order prediction from their
 * parents (eq:Prediction); the parents' halos must be filled.  slots_host: host int32[n]. */
int mrfv_mr_predict(mrfv_ctx *ctx, void *U, const int32_t *slots_host, int32_t n);

/* mr_flag -- details d(B) = max over the 24^3 padded cells and q in {rho, E} of
 * |u_q - P(u_parent)_q| / scale_q (eq:DetailFunction read as u_l - P(u_{l-1})), evaluated
 * in double precision, and refine/keep/coarsen flags (eq:Thresholding with the level
 * thresholds of eq:LevelWiseEpsilon): REFINE (1) if l < lmax and d >= eps_l; COARSEN (-1)
 * if l >= 2, all 8 siblings are leaves with d < eps_l and the parent's d < eps_{l-1};
 * else KEEP (0); non-leaves get 2.  All 26 halo regions must be filled.
 * The prediction is evaluated in its separable form; a slab of a block whose detail lies
 * within a narrow band of its threshold (see mrfv_set_detail_band) is evaluated again with
 * the prediction summed term by term as the appendix writes it (Q_x ... Q_xyz, left to
 * right, no fused multiply-add) and |u - P| divided by the scale, so that every flag is
 * the one that evaluation order gives.
 * flags_dev: dev int8[capacity], det_dev: dev double[capacity] (indexed by slot). */
int mrfv_mr_flag(mrfv_ctx *ctx, const void *U, int8_t *flags_dev, double *det_dev);

/* set_detail_band -- half-width of the band around eps_l inside which mr_flag (and the
 * adaptation of mrfv_step / mrfv_run) re-evaluates a detail in the appendix's term order
 * (default 1e-9, in units of the normalised detail).  0 re-evaluates only exact ties; a
 * large value re-evaluates every block (slow; for checks).  band >= 0, else MRFV_EINVAL.
 * Synchronises the stream. */
int mrfv_set_detail_band(mrfv_ctx *ctx, double band);

/* cfl_dt -- eq:Cfl per instance: dt = cfl dx_lmax / sum_d max(|v_d| + c) over leaf
 * interior cells, reduced in double precision.  dt_dev: dev double[n_instances]. */
int mrfv_cfl_dt(mrfv_ctx *ctx, const void *U, double *dt_dev);

/* totals -- per instance, sum over leaf interior cells of u_q dx_l^3 in double
 * precision with a fixed reduction order.  tot_dev: dev double[n_instances][5]. */
int mrfv_totals(mrfv_ctx *ctx, const void *U, double *tot_dev);

/* totals_noalloc -- mrfv_totals for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result, bitwise, with the per-slot partial sums kept in a
 * static device array of the library (65536 slots x 5 doubles = 2.6 MB per device, held
 * until the process ends) instead of the context's scratch.  Calls no allocating
 * routine.  Every call on one device shares that array and overwrites what it needs
 * before reading it; calls that overlap on one device (several streams or contexts at
 * once) race.  MRFV_EINVAL when the context's slot capacity exceeds 65536, MRFV_ESTATE
 * when the context's device is not current.  tot_dev: dev double[n_instances][5]. */
int mrfv_totals_noalloc(mrfv_ctx *ctx, const void *U, double *tot_dev);

/* commit_flags -- apply flags (host int8[capacity] by slot, as written by mr_flag) to
 * the tree: refine creates 8 children (their interiors are NOT yet predicted), coarsen
 * removes 8 leaf siblings; then rebuilds and uploads the device tables.  The new child
 * slots are written to new_slots_host (capacity-sized host int32 array, may be NULL) and
 * their number to *n_new. */
int mrfv_commit_flags(mrfv_ctx *ctx, const int8_t *flags_host, int32_t *new_slots_host,
                      int32_t *n_new);

/* step -- one global time step of algo:ComputeLoop: cfl_dt; three stages of
 * {mr_project, fill_halos, rhs + jump correction, rk_update}; then, for adaptive
 * instances, mr_project, fill_halos, mr_flag, one device-to-host copy of the flags,
 * commit_flags and mr_predict of the new children.  U0, L: dev scratch of
 * mrfv_interior_bytes.  dt_dev: dev double[n_instances] receives this step's dt.
 * The batched FP32 path runs the stages out of place through two library-owned state
 * buffers (U -> W -> W2 -> U), reading same-level neighbours' interiors directly, and
 * restricts and fills only what the stages read.  Before the details only rho and E are
 * restricted and filled (all components are restricted when the flags change the tree).
 * On return U holds the new state in every leaf interior (call mr_project and fill_halos
 * for restricted parents and complete halos). */
int mrfv_step(mrfv_ctx *ctx, void *U, void *U0, void *L, double *dt_dev);

/* run -- n_steps calls of mrfv_step with the same result, bitwise, for callers that do
 * not touch U in between.  On the batched FP32 graph path of an adaptive context without
 * a proposer, step k+1 is queued before the host has read step k's flags; when those
 * flags change the tree, the CFL reduction of step k+1 finds the change recorded on the
 * device and zeroes that step's work lists (it does nothing), and step k+1 is queued
 * again after the commit.  The device then runs unchanged steps back to back.  A step
 * that follows a step on the same tree inside the call reuses that step's last stage:
 * its restriction into the parents (the first stage then restricts only the other
 * octants) and its per-block CFL maxima (the CFL pass over the leaves is skipped, except
 * for the leaves the jump correction changed; the maxima are bitwise those of the pass).  Returns
 * after the last step with nothing left in flight; dt_dev holds the last step's dt.
 * leaf_cells_host (may be NULL): the leaf cells of each step's tree, summed over the
 * steps run (a step integrates each of them three times). */
int mrfv_run(mrfv_ctx *ctx, void *U, void *U0, void *L, double *dt_dev, int32_t n_steps,
             int64_t *leaf_cells_host);

/* step_lts -- one macro step of local time stepping (eq:LtsTimestep; algo:ComputeLoop with
 * algo:Integration): dt = the eq:Cfl step of level lmax (written to dt_dev, one double per
 * instance), 2^lmax micro steps of dt, level l advancing with dt_l = 2^(lmax - l) dt; the
 * clock advances 2^lmax dt.  Level l completes a step of its own at micro step r when
 * r + 1 is a multiple of 2^(lmax - l) (the active set of algo:ComputeLoop); its first RK
 * stage is evaluated at the micro step its step starts in, all its stages are integrated
 * at the micro step it ends in.  Halo cells of faces without a same-level neighbour are
 * predicted from the state at the macro step's start and then integrated with the flux
 * divergence, which is averaged into parents and predicted into those halos like the
 * state (eq:Averaging, eq:Prediction).  Conservative: leaves sum their boundary face
 * fluxes with the RK weights, and a coarse leaf next to a refined same-level neighbour
 * replaces its own sum by the fine average at the end of its step (coarse cell
 * adjustment).  Adaptive instances run mr_flag, commit_flags and mr_predict once, after
 * the last micro step.  Runs per tree level in the context's dtype (any batched mode):
 * in FP32 the fused stage kernel evaluates the flux divergence (Tait's system: the plain
 * flux kernel), in FP64 the plain flux kernel; separate kernels integrate it.  U0: dev
 * scratch of mrfv_interior_bytes, as for mrfv_step; L is not used
 * (may be NULL); the library allocates its padded flux-divergence field, the jump-halo
 * stage state and the face-flux sums on first use (MRFV_ENOMEM if it cannot).  cell_updates_host (may be
 * NULL): leaf cells times their own steps in this macro step.  Every instance must have
 * the same lmax (else MRFV_EINVAL), and none may be viscous (MRFV_EINVAL). */
int mrfv_step_lts(mrfv_ctx *ctx, void *U, void *U0, void *L, double *dt_dev,
                  int64_t *cell_updates_host);

/* check -- reads and clears the device error word: MRFV_ENONPHYS if a stage produced a
 * non-physical state since the last check, else MRFV_OK.  Synchronises the stream. */
int mrfv_check(mrfv_ctx *ctx);

/* Tree statistics: out_host int64[4] = (blocks, leaves, leaf cells, finest level present).
 * Host data only; no device access. */
int mrfv_stats(mrfv_ctx *ctx, int64_t *out_host);

/* Block table.  info_host: int64[n][8] = (slot, instance, level, bx, by, bz, is_leaf,
 * morton id with headbit).  *n receives the number of blocks (info_host may be NULL). */
int mrfv_get_blocks(mrfv_ctx *ctx, int64_t *info_host, int32_t *n);

/* Explicit tree edits for tests: refine fills all halos of U, then creates the children
 * of a leaf and predicts their interiors; coarsen removes the 8 leaf children of a block
 * (the block's interior must already be their average). */
int mrfv_refine_block(mrfv_ctx *ctx, void *U, int32_t instance, int32_t level, int32_t bx,
                      int32_t by, int32_t bz);
int mrfv_coarsen_block(mrfv_ctx *ctx, int32_t instance, int32_t level, int32_t bx,
                       int32_t by, int32_t bz);

/* Kernel timing: when enabled, every launch of the fused rhs + update kernel (batched
 * path) or of the flux kernel (plain path) is bracketed by HIP events on the context
 * stream; mrfv_kernel_time returns the number of timed launches, their total duration in
 * ms and the leaf cells per launch summed over launches. */
int mrfv_enable_kernel_timing(mrfv_ctx *ctx, int32_t on);
int mrfv_kernel_time(mrfv_ctx *ctx, int64_t *launches, double *total_ms, int64_t *cells);

/* fused_stage -- one SSP-RK3 stage of the batched FP32 path exactly as mrfv_step runs it:
 * mr_project and the stage halo fill on Uin (regions without a same-level neighbour),
 * then the fused rhs + update kernel reading Uin (same-level neighbours' interiors in
 * place) and writing the leaves' new interiors to Uout, with the jump correction.  Uin,
 * Uout: dev, state_bytes each, distinct; U0: dev, interior_bytes (written at stage 0, read
 * at stages 1 and 2); dt_dev: dev double[n_instances].  restrict_parents != 0: leaves on
 * level >= 1 none of whose same-level face neighbours is a non-leaf also write the
 * restriction (eq:Averaging) of their new interior into their parent's octant of Uout,
 * as the step does for a stage whose output is restricted next.  Batched FP32 contexts
 * only. */
int mrfv_fused_stage(mrfv_ctx *ctx, int32_t stage, const double *dt_dev, void *Uin, void *Uout,
                     void *U0, int32_t restrict_parents);

/* Launch shapes of the fused rhs + update kernel (batched FP32 path; 14 for the standard
 * Roe-WENO5 kernel, 3 for the other flux kernels): variant v groups
 * the block's z-planes by shapes_host[4v] and uses |shapes_host[4v+1]| threads per
 * workgroup, one workgroup per leaf, or, when shapes_host[4v+1] < 0, a persistent grid
 * of workgroups looping over the leaves; shapes_host[4v+2] is the number of wavefronts
 * per SIMD the register allocation aims at (1: the compiler's choice); shapes_host[4v+3]
 * is 1 when the stencils are always loaded through per-lane pointers (otherwise through
 * one buffer resource whenever a workgroup's source blocks lie within 4 GiB).  Every
 * variant gives bitwise the same result.  A new context takes the shape GP 2 x 512
 * threads (the first variant of the other kernels).  rhs_variant sets the variant
 * when set >= 0 (captured step graphs are re-captured), writes the number of variants
 * and their shapes (each may be NULL) and returns the current variant (>= 0) or an
 * error.  Host only. */
int mrfv_rhs_variant(mrfv_ctx *ctx, int32_t set, int32_t *n_variants_host, int32_t *shapes_host);

/* autotune -- times every variant on the current tree and state (reps launches each,
 * after one warm-up) and keeps the fastest.  Leaf interiors of U are not modified (its
 * parents are restricted and halos filled, as before a stage); U0, the second state
 * buffer and dt_dev (dev double[n_instances], receives the CFL step) are used as
 * scratch.  ms_host (may be NULL): host float[n_variants] receives the mean launch time
 * of each variant; *choice_host the chosen variant.  Batched FP32 contexts only.
 * Synchronises the stream. */
int mrfv_autotune(mrfv_ctx *ctx, void *U, void *U0, double *dt_dev, int32_t reps, float *ms_host,
                  int32_t *choice_host);

/* step_timing -- host clock of the adaptation phase of mrfv_step, summed over adaptive
 * steps: out_host double[4] = (steps, ms waiting for the judged flags, ms committing the
 * tree and uploading its tables (or adopting staged ones), ms predicting new children). */
int mrfv_step_timing(mrfv_ctx *ctx, double *out_host);

/* Morton ids with a headbit (Sec. "Modular block-based MR algorithm"): 3-bit groups per
 * level, finest group least significant, x = bit 0 of each group; shadow = number of
 * groups above level 0.  Neighbour along axis d in direction dir (+1/-1); *wrapped = 1
 * when the lookup crossed the domain edge (the result is the periodic image). */
uint64_t mrfv_morton_encode(int32_t shadow, int32_t level, int32_t bx, int32_t by, int32_t bz);
uint64_t mrfv_morton_neighbor(uint64_t id, int32_t shadow, int32_t d, int32_t dir,
                              int32_t *wrapped);

/* ---------------------------------------------------------------------------------------
 * Learned refinement proposer.  Not part of the paper's method: a small network predicts,
 * from the state at the start of a step, the refine / keep / coarsen decision that the
 * Harten detail threshold (Sec. "Multiresolution", eq:LevelWiseEpsilon) will take at the
 * end of it, so that the host can build the next tree's tables while the device
 * integrates.  The threshold stays the judge: a proposal is adopted only when it equals
 * the judged flags on every leaf, so the solution never depends on the network.
 *
 * Network: 192 -> 64 -> 64 -> 3 with ReLU; parameters as one FP32 vector
 * (W1[192][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3]; W[in][out] row-major),
 * products on the matrix cores in bfloat16 with FP32 accumulation.  Classes:
 * 0 refine, 1 keep, 2 coarsen.
 * ------------------------------------------------------------------------------------- */
typedef struct mrfv_mlp mrfv_mlp;

/* Network object for up to max_rows samples per call; parameters start at zero.
 * hip_stream: stream every call is queued on (NULL = default stream). */
int mrfv_mlp_create(mrfv_mlp **out, int32_t max_rows, void *hip_stream);
int mrfv_mlp_destroy(mrfv_mlp *mlp);
const char *mrfv_mlp_last_error(const mrfv_mlp *mlp);
int32_t mrfv_mlp_nparams(void);
/* Parameters from / to host float[nparams]; set_params also resets the Adam moments.
 * Both synchronise the stream. */
int mrfv_mlp_set_params(mrfv_mlp *mlp, const float *params_host);
int mrfv_mlp_get_params(mrfv_mlp *mlp, float *params_host);
/* Forward pass: X_dev dev float[N][192] -> logits_dev dev float[N][3].  Asynchronous. */
int mrfv_mlp_forward(mrfv_mlp *mlp, const float *X_dev, int32_t N, float *logits_dev);
/* Class-weighted mean softmax cross-entropy of labels_host int32[N] (0..2) with class
 * weights class_w_host float[3], and its gradient with respect to the parameters, kept on
 * the device for mrfv_mlp_adam_step; loss_host (float, may be NULL) and grad_host
 * (float[nparams], may be NULL) receive copies.  Synchronises the stream. */
int mrfv_mlp_loss_grad(mrfv_mlp *mlp, const float *X_dev, const int32_t *labels_host,
                       const float *class_w_host, int32_t N, float *loss_host, float *grad_host);
/* One Adam update of the parameters with the last gradient (bias-corrected moments). */
int mrfv_mlp_adam_step(mrfv_mlp *mlp, float lr, float beta1, float beta2, float eps);

/* features -- the proposer's input for every leaf, in the order of the all-leaves list:
 * over each of the 4^3 sub-cubes of 4^3 interior cells, the means of rho, |grad rho|
 * (central differences in cell units, one-sided at block faces) and p, written as
 * (mean rho / scale_rho - 1, log(1 + mean |grad rho| / (scale_rho eps_l)),
 * mean p / scale_p - 1) with scale_p = (gamma - 1) scale_E; X_dev[r][3 s + c] with
 * s = (sz 4 + sy) 4 + sx.  X_dev: dev float[capacity][192]; slots_host (may be NULL):
 * host int32[capacity] receives the leaf slots; *n the number of leaves.  Asynchronous. */
int mrfv_features(mrfv_ctx *ctx, const void *U, float *X_dev, int32_t *slots_host, int32_t *n);

/* set_proposer -- mode 0: off (the default); 1: the network mlp (borrowed, must outlive
 * its use) proposes a step's flags when the step before changed the tree (and on the
 * first step after this call), otherwise the proposal is "no change"; 2: persistence,
 * i.e. the proposal is always "no change".
 * With a proposal, mrfv_step commits it on the host tree, builds and uploads its tables to
 * a second device copy while the device integrates, undoes the commit, and adopts the copy
 * when the judged flags equal the proposal; otherwise it commits the judged flags as
 * usual.  Results are identical in every mode. */
int mrfv_set_proposer(mrfv_ctx *ctx, mrfv_mlp *mlp, int32_t mode);

/* last_flags -- the judged flags (host int8[capacity] by slot, as mr_flag writes them) of
 * the last mrfv_step that adapted the tree, with or without a proposer: the training
 * labels of the proposer.  Zero before the first adaptive step.  Synchronises the stream. */
int mrfv_last_flags(mrfv_ctx *ctx, int8_t *flags_host);

/* proposer_stats -- out_host int64[14] = (steps, hits, then for refine, keep, coarsen:
 * true positives, false positives, false negatives, then steps whose proposal changed the
 * tree and was staged, staged proposals adopted, steps on which the network ran);
 * build_ms_host (may be NULL): host milliseconds spent decoding and staging proposals. */
int mrfv_proposer_stats(mrfv_ctx *ctx, int64_t *out_host, double *build_ms_host);

#ifdef __cplusplus
}
#endif
#endif /* MRFV_H */
