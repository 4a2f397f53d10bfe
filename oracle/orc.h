/*
 * orc.h -- FP64 CPU oracle for the block-based multiresolution (MR) finite-volume
 * solver of Hoppe, Adami & Adams, "A modular massively parallel computing environment
 * for three-dimensional multiresolution simulations of compressible flows"
 * (arXiv 2012.04385).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow, obviously-correct
 * reference the GPU path is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code with the HIP
 * library (no headers, helpers, tables or generators) and the GPU library never calls it.
 *
 * Everything is double precision, compiled without floating-point contraction or
 * fast-math, and parallelised only over independent blocks so results do not depend
 * on the thread count.
 *
 * Conventions (the paper's block concept, Sec. "Modular block-based MR algorithm"):
 *   a block holds 16^3 interior cells plus 4 halo layers per side: a padded 24^3 array
 *   per conserved quantity, stored [q][z][y][x] with x fastest; interior index 4..19.
 *   q = (rho, rho*u, rho*v, rho*w, E).
 *
 * Every function here is pinned by a CPU test (tests/test_oracle_*.py) against closed
 * forms, invariants, exact rational arithmetic, published values or brute force: the
 * x-direction flux by consistency, the Roe property, a smooth entropy wave and Sod's
 * exact solution; the y and z directions by bitwise axis permutations (Sod, single level
 * and adaptive; the isentropic vortex) and by fifth-order convergence of the vortex in
 * the x-y plane; the exact Riemann solver by the published star state of Sod's data.
 * What stays unpinned is the solution of the flows without a closed form (shear layer,
 * shock and blobs): there the GPU is compared with this oracle, not with a truth.
 */
#ifndef ORACLE_ORC_API_H
#define ORACLE_ORC_API_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_IC 16   /* interior cells per block edge            */
#define ORC_H 4     /* halo layers per side                     */
#define ORC_P 24    /* padded edge = ORC_IC + 2*ORC_H           */
#define ORC_MAX_LEVELS 16

/* ---------------- pointwise numerics (Sec. "Numerical Scheme", eq:StiffenedGas) ---- */

/* Pressure of a conservative state, stiffened-gas EOS p = (gamma-1) rho e - gamma B. */
double orc_pressure(const double U[5], double gamma, double B);

/* Physical Euler flux along x of a conservative state. */
void orc_flux_x(const double U[5], double gamma, double B, double F[5]);

/* Roe-averaged right (R, columns = eigenvectors) and left (L = R^-1) eigenvector matrices
 * of the x-direction flux Jacobian between states UL and UR, row-major 5x5. */
void orc_roe_matrices(const double UL[5], const double UR[5], double gamma, double B,
                      double R[25], double L[25]);

/* WENO5-JS (Jiang & Shu) value at the right face of the middle point, left-biased. */
double orc_weno5_minus(double a, double b, double c, double d, double e);

/* Numerical flux through the x-face between cells 2 and 3 of a 6-cell stencil
 * st[6][5] (cells i-2..i+3): characteristic WENO5-JS with per-field Roe upwinding and
 * local Lax-Friedrichs fallback.  Returns the number of fields that used LLF. */
int orc_face_flux_x(const double st[30], double gamma, double B, double F[5]);

/* Same along axis d (0,1,2) for a stencil given in the physical component order. */
int orc_face_flux(int d, const double st[30], double gamma, double B, double F[5]);

/* ---------------- the other flux kernels of Sec. "Numerical Scheme" ---------------- */

/* TENO5 (Fu, Hu & Adams) value at the right face of the middle point, left-biased. */
double orc_teno5_minus(double a, double b, double c, double d, double e);
/* WENO-AO(5,3) (Balsara, Garain & Shu) value at the right face of the middle point. */
double orc_wao53_minus(double a, double b, double c, double d, double e);
/* Smoothness indicator of the quartic with cell averages a..e (unit cells -2..2). */
double orc_beta_quartic(double a, double b, double c, double d, double e);
/* HLLC flux along x between two conservative states. */
void orc_hllc_flux_x(const double UL[5], const double UR[5], double gamma, double B, double F[5]);
/* Face flux of the six-cell stencil with one of the paper's flux kernels:
 * 0 Roe + WENO5-JS (orc_face_flux), 1 Roe + TENO5, 2 LLF + WENO5-JS (every field split),
 * 3 HLLC + WENO-AO(5,3) (characteristic-wise face states).  Returns the LLF fields. */
int orc_face_flux_x_scheme(int scheme, const double st[30], double gamma, double B, double F[5]);
int orc_face_flux_scheme(int scheme, int d, const double st[30], double gamma, double B, double F[5]);

/* ---------------- Tait's equation of state (Sec. "Influence of Equation of State") ---- */

/* p = B ((rho/rho0)^gamma - 1) + A and c = sqrt(dp/drho). */
double orc_tait_pressure(double rho, double gamma, double B, double A, double rho0);
double orc_tait_sound_speed(double rho, double gamma, double B, double rho0);
/* Flux along x of the barotropic system (rho, rho v); the energy component is zero. */
void orc_tait_flux_x(const double U[5], double gamma, double B, double A, double rho0, double F[5]);
/* Roe matrices (4x4, row-major; fields u-c, u, u, u+c on rho, m1, m2, m3). */
void orc_tait_roe_matrices(const double UL[5], const double UR[5], double gamma, double B, double A,
                           double rho0, double R[16], double L[16]);
/* Characteristic WENO5-JS Roe flux with per-field LLF fallback, x and axis d. */
int orc_tait_face_flux_x(const double st[30], double gamma, double B, double A, double rho0,
                         double F[5]);
int orc_tait_face_flux(int d, const double st[30], double gamma, double B, double A, double rho0,
                       double F[5]);
/* Exact 1D Riemann solution (rho, u) at x/t = s[i] (out[2 i..]); -1 if vacuum forms. */
int orc_tait_exact_riemann(double rl, double ul, double rr, double ur, double gamma, double B,
                           double A, double rho0, const double *s, int n, double *out);

/* ---------------- MR operators (eq:Averaging, eq:Prediction + appendix Q-terms) ------ */

/* Fifth-order conservative prediction of one fine cell from a padded 24^3 parent array
 * (one component).  (ox,oy,oz) = octant of the child inside the parent, (i,j,k) = the
 * child's padded cell index, each in [0,24).  Implements the appendix Q-term sums. */
double orc_predict_cell(const double *parent, int ox, int oy, int oz, int i, int j, int k);

/* Conservative average of 8 fine values given in (x,y,z) child-offset order c[z][y][x]. */
double orc_average8(const double c[8]);

/* SSP-RK3 (Shu-Osher) stage s = 0,1,2 in increment form:
 * u^(s+1) = u0 + a_s ((u^(s) - u0) + dt L(u^(s))), a = (1, 1/4, 2/3). */
double orc_ssprk3_stage(int stage, double u0, double us, double L, double dt);

/* ---------------- viscous terms (Navier-Stokes form of eq:Euler) ------------------- */

/* Viscous flux through the face between two cells along axis d, from the velocities of
 * the two cells and of their four tangential neighbours: st[s][n][q], s = 0 the cell on
 * the low side, 1 the cell on the high side; n = 0 the cell itself, 1 / 2 its neighbours
 * at -1 / +1 along the lower of the two other axes, 3 / 4 along the higher one; q the
 * conservative state in physical component order.  F = (0, tau_d., tau_d. . v_face) with
 * the Newtonian stress of Stokes' hypothesis, tau = mu (grad v + grad v^T) - 2/3 mu div v I:
 * normal derivatives from the two cells, tangential derivatives as the mean of the two
 * cells' central differences, v_face the mean of the two velocities.  energy = 0 leaves
 * F[4] zero (Tait's barotropic system).  The face's total flux is the convective flux
 * minus this one. */
void orc_visc_face_flux(int d, const double st[50], double mu, int energy, double dx, double F[5]);

/* Explicit time-step bound of the viscous terms: cfl * 3/16 * dx^2 / (mu * max(1/rho)). */
double orc_visc_dt(double cfl, double dx, double mu, double rinv_max);

/* Linear growth rate n > 0 of the Rayleigh-Taylor instability of two viscous fluids with
 * equal dynamic viscosity mu (eq:SinglePhaseGrowth): heavy density rho_h on top of rho_l,
 * gravity g, wavenumber k.  Bisection on n in (0, sqrt(At g k)].  Returns -1 if the
 * relation has no root there. */
double orc_rti_growth_rate(double k, double rho_h, double rho_l, double mu, double g);

/* ---------------- exact Riemann solver (textbook, Toro ch. 4) for the Sod pin ------- */

/* Samples the exact solution of the 1D Riemann problem (ideal gas, B = 0) at x/t = s
 * values; out[3*i..] = (rho, u, p).  Returns 0, or -1 if Newton failed. */
int orc_exact_riemann(double rl, double ul, double pl, double rr, double ur, double pr,
                      double gamma, const double *s, int n, double *out);

/* ---------------- the MR simulation (algo:Init, algo:ComputeLoop with global dt) ---- */

typedef struct {
    double gamma, B;       /* EOS                                              */
    double cfl;            /* CFL number k of eq:Cfl                           */
    double eps;            /* threshold at the finest level (eq:UserEpsilon)   */
    double scale_rho;      /* normalisation of the rho details                 */
    double scale_E;        /* normalisation of the E details                   */
    double dx0;            /* cell size on level 0                             */
    int32_t lmax;          /* finest level                                     */
    int32_t n0[3];         /* level-0 blocks per axis                          */
    int32_t bc[3];         /* per axis: 0 periodic, 1 zero-gradient, 2 symmetry,
                              3 fixed values (bc_fixed)                        */
    int32_t adapt;         /* 1: refine/coarsen after each step                */
    int32_t scheme;        /* flux kernel, see orc_face_flux_scheme            */
    double gravity[3];     /* source term of eq:Euler: S = (0, rho g, rho v.g) */
    int32_t eos;           /* 0 stiffened gas (eq:StiffenedGas), 1 Tait        */
    double tait_A, tait_rho0;   /* Tait: p = B ((rho/rho0)^gamma - 1) + A       */
    double mu;             /* dynamic viscosity (0: Euler equations)           */
    /* fixed-value boundaries: primitive states (rho, u, v, w, p) of the halo cells beyond
     * the sides of the axes with bc 3, [6 sides x-, x+, y-, y+, z-, z+][lmax + 1 levels]
     * [4 layers, the one at the face first][5], uniform over the boundary plane; copied by
     * orc_sim_create; NULL when no axis has bc 3 */
    const double *bc_fixed;
} orc_params;

typedef struct orc_sim orc_sim;

/* IC callback: fill prim[5][16][16][16] = (rho,u,v,w,p) at the cell centres of the
 * interior of block (level, bx, by, bz). */
typedef void (*orc_ic_fn)(void *user, int32_t level, int32_t bx, int32_t by, int32_t bz,
                          double *prim);

orc_sim *orc_sim_create(const orc_params *p);
void orc_sim_free(orc_sim *s);

/* Bottom-up initialisation of algo:Init. 0 on success. */
int orc_sim_init(orc_sim *s, orc_ic_fn ic, void *user);

/* One global time step: CFL dt, three SSP-RK3 stages, then MR adaptation.
 * Returns 0, or -5 when a non-physical state (rho<=0, p+B<=0, NaN) appeared. */
int orc_sim_step(orc_sim *s, double *dt_out);
/* the same step with a given dt (time-step convergence studies) */
int orc_sim_step_dt(orc_sim *s, double dt);
/* One macro step of local time stepping (eq:LtsTimestep, algo:ComputeLoop,
 * algo:Integration): 2^lmax micro steps of dt = the eq:Cfl step of level lmax, level l
 * advancing with 2^(lmax-l) dt; adaptation (if enabled) once, at the end, when every
 * level has reached the same time.  *dt_out = dt; time advances by 2^lmax dt. */
int orc_sim_step_lts(orc_sim *s, double *dt_out);   /* -1: viscous (not supported) */
int orc_sim_step_lts_dt(orc_sim *s, double dt);
/* own steps completed per level since creation (ORC_MAX_LEVELS entries) */
void orc_sim_lts_steps(const orc_sim *s, int64_t *out);
/* lowest level that completes a step of its own at micro step r */
int32_t orc_lts_lowest_ending(int32_t lmax, int32_t r);

/* Block table: n blocks; info[n][8] = (level, bx, by, bz, is_leaf, flag, morton, 0). */
int32_t orc_sim_nblocks(const orc_sim *s);
void orc_sim_blocks(const orc_sim *s, int64_t *info);
/* Padded state of block idx (order of orc_sim_blocks), 5*24^3 values. */
void orc_sim_get_block(const orc_sim *s, int32_t idx, double *out);
void orc_sim_set_block(orc_sim *s, int32_t idx, const double *in);
/* Per-block pieces of the step for sampled checks at full size (same code as the
 * simulation's): the right-hand side -div F of one padded block (no jump correction),
 * L[5][16][16][16], with cell size dx; and the detail of eq:DetailFunction of a padded
 * child block against its padded parent (octant ox, oy, oz). */
void orc_block_rhs(const double *u_padded, double gamma, double B, double dx, double *L);
void orc_block_rhs_scheme(int scheme, const double *u_padded, double gamma, double B, double dx,
                          double *L);
double orc_block_detail(const double *u_padded, const double *parent_padded, int ox, int oy,
                        int oz, double s_rho, double s_E);

/* Last detail value of block idx (-1 for level 0). */
double orc_sim_detail(const orc_sim *s, int32_t idx);

/* Explicit tree edits and single operators, for operator-level parity tests.
 * refine: fills all halos, then leaf -> 8 children whose interiors are P(parent);
 * coarsen: remove the 8
 * (leaf) children of a block.  Return 0 or -1. */
int orc_sim_refine(orc_sim *s, int32_t level, int32_t bx, int32_t by, int32_t bz);
int orc_sim_coarsen(orc_sim *s, int32_t level, int32_t bx, int32_t by, int32_t bz);
void orc_sim_project(orc_sim *s);            /* parents <- A(children), bottom-up      */
void orc_sim_fill_halos(orc_sim *s);         /* all 26 halo regions, coarse to fine    */
/* Right-hand side L (5*16^3 per leaf, leaves in block order) incl. jump flux correction;
 * halos must be filled. Returns number of leaves written. */
int32_t orc_sim_rhs(orc_sim *s, double *L_out);
/* Details of all blocks and resulting flags (block order); flags: 1 refine, 0 keep,
 * -1 coarsen, 2 not a leaf.  Halos must be filled (26 regions). */
void orc_sim_details(orc_sim *s, double *det_out, int8_t *flag_out);
/* CFL time step from the current leaf state. */
double orc_sim_dt(const orc_sim *s);
/* Volume-weighted totals over leaf interior cells: tot[5]. */
void orc_sim_totals(const orc_sim *s, double *tot);
double orc_sim_time(const orc_sim *s);
/* Fraction of face-fields that took the LLF branch during the last rhs evaluation. */
double orc_sim_llf_fraction(const orc_sim *s);
/* Threads the oracle's parallel loops use (OpenMP). */
int orc_num_threads(void);

/* ---------------- learned refinement proposer (not in the paper) -------------------- */

/* Number of parameters of the 192-64-64-3 network (layout W1 b1 W2 b2 W3 b3, weights
 * [in][out] row-major). */
int orc_mlp_nparams(void);
/* Round to the nearest bfloat16, ties to even. */
double orc_bf16_round(double x);
/* logits[N][3] of X[N][192]; bf16_emulation = 1 rounds what the GPU stores in bfloat16. */
void orc_mlp_forward(const double *params, const double *X, int N, int bf16_emulation,
                     double *logits);
/* Class-weighted mean softmax cross-entropy and its gradient (grad may be NULL).
 * labels[N] in {0: refine, 1: keep, 2: coarsen}; class_w[3]. */
double orc_mlp_loss_grad(const double *params, const double *X, const int32_t *labels,
                         const double *class_w, int N, int bf16_emulation, double *grad);
/* Proposer features (192) of one padded block, see orc_mlp.cpp. */
void orc_features(const double *u_padded, double gamma, double B, double s_rho, double s_p,
                  double eps_l, double *out);

/* Morton ids with headbit (Sec. "Modular block-based MR algorithm", eq:NeigboorLookup).
 * shadow = number of 3-bit groups above level 0 (level-0 blocks per edge = 2^shadow). */
uint64_t orc_morton_encode(int32_t shadow, int32_t level, int32_t bx, int32_t by, int32_t bz);
/* neighbour id along axis d (0,1,2) in direction dir (+1/-1) by bit flipping;
 * *wrapped = 1 when the lookup left the domain (and wrapped around). */
uint64_t orc_morton_neighbor(uint64_t id, int32_t d, int32_t dir, int32_t *wrapped);
int32_t orc_morton_level(uint64_t id, int32_t shadow);

#ifdef __cplusplus
}
#endif
#endif
