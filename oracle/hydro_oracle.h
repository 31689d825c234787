/*
 * hydro_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, serial-order, FP64 CPU reference of the Godunov hydrodynamics step
 * described in Wang, "The Kratos Framework for Heterogeneous Astrophysical
 * Simulations" (arXiv 2501.02317), Sec. 3: primitive-variable PLM with the
 * minmod limiter (eq. minmod), HLLC fluxes with the subtraction-safe wave
 * speeds (eqs. hllc-contact-spd, hllc-mixed-dvel), the Heun two-stage
 * integrator (Sec. 3.3) and a global CFL time step (Sec. 3.1).
 *
 * Only the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU product path never links, loads or
 * calls it, and the two share no source, header, table or helper.
 *
 * Conventions (all arrays are caller-owned host memory, FP64):
 *   - ndim in {1,2,3}; n[d] interior cells on axis d (n[d] = 1 for d >= ndim).
 *   - ncomp = 2 + ndim.  Conserved U = (rho, m_1..m_ndim, E); primitive
 *     W = (rho, v_1..v_ndim, p).  Only in-plane momenta are carried.
 *   - Field layout [comp][k][j][i], i (x) fastest, interior cells only,
 *     ncells = n[0]*n[1]*n[2].
 *   - Boundary codes per axis side: 0 periodic, 1 free (zero gradient),
 *     2 outflow, 3 reflecting (Sec. 3.1.1).  Periodic must be set on both
 *     sides of an axis.
 *   - Functions returning int return 0 on success, a positive count of
 *     non-physical cells (rho <= 0, p <= 0 or non-finite) when the state is
 *     not admissible, or -1 on invalid arguments.
 */
#ifndef HYDRO_ORACLE_H
#define HYDRO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_PERIODIC = 0, ORC_BC_FREE = 1, ORC_BC_OUTFLOW = 2, ORC_BC_REFLECT = 3 };

/* Time integrators of Sec. 3.3: Heun (default) and the memory-optimised van Leer. */
enum { ORC_HEUN = 0, ORC_VL2 = 1 };

typedef struct {
    int32_t ndim;
    int32_t n[3];
    double lo[3];
    double hi[3];
    double gamma;
    int32_t bc[3][2];
    int32_t integrator; /* ORC_HEUN or ORC_VL2; used by orc_run */
} orc_mesh;

/* Number of conserved components, 2 + ndim; -1 for an invalid mesh. */
int orc_ncomp(const orc_mesh* m);

/* minmod(a, b), eq. minmod; zero when the signs differ or either is zero. */
double orc_minmod(double a, double b);

/* Pointwise conversions (Sec. 3.1).  W -> U never fails. */
void orc_prim_to_cons(const orc_mesh* m, const double* W, double* U);
int orc_cons_to_prim(const orc_mesh* m, const double* U, double* W);

/*
 * HLLC flux across one face in the face-normal frame.  WL and WR hold
 * (rho, u, t_1..t_ntan, p) with ntan = ndim - 1 tangential velocities; F gets
 * (mass, normal momentum, tangential momenta, energy) fluxes.  When detail is
 * non-NULL it receives, in order: s_L, s_star, s_R, p_star, then U_L, U_R,
 * F_L, F_R, Ustar_L, Ustar_R, Fstar_L, Fstar_R (each ntan+3 values).
 */
void orc_hllc(double gamma, int ntan, const double* WL, const double* WR, double* F,
              double* detail);

/* PLM face states of face j+1/2 from the four cells j-1, j, j+1, j+2 (one
 * scalar component): wl = W_j + delta_j / 2, wr = W_{j+1} - delta_{j+1} / 2. */
void orc_plm_face(const double w4[4], double* wl, double* wr);

/* CFL time step (Sec. 3.1): cfl * min over cells and axes of dx_d/(|v_d|+c).
 * Returns a negative value when the state is not admissible. */
double orc_cfl_dt(const orc_mesh* m, const double* U, double cfl);

/* Ghost fill on a padded primitive array with n_gh = 2 layers on each active
 * axis (inactive axes unpadded); layout [comp][K][J][I] of padded extents. */
int orc_fill_ghosts(const orc_mesh* m, double* Wpad);

/* One stage right-hand side dU = sum_d dt/dx_d (F_{d,i-1/2} - F_{d,i+1/2}). */
int orc_rhs(const orc_mesh* m, const double* U, double dt, double* dU);

/* One Heun step in place (Sec. 3.3). */
int orc_heun_step(const orc_mesh* m, double* U, double dt);

/* Stage right-hand side, as orc_rhs, from an interior primitive state W with
 * piecewise-constant (order 1) or PLM (order 2) face states. */
int orc_rhs_prim(const orc_mesh* m, const double* W, double dt, int order, double* dU);

/* One step of the memory-optimised van Leer integrator (Sec. 3.3):
 * W* = W(U^n + (dt/2) L_1(U^n)) with piecewise-constant states, then
 * U^{n+1} = U^n + dt L_2(W*) with PLM states, in place. */
int orc_vl2_step(const orc_mesh* m, double* U, double dt);

/*
 * Run with the CFL step: at most max_steps steps (max_steps <= 0 means no
 * limit), and when t_end > 0 the last step is shortened to land on t_end.
 * *t is read as the start time and updated; *steps_done receives the count;
 * dts (may be NULL, length max_steps) receives each step's dt.
 */
int orc_run(const orc_mesh* m, double* U, double cfl, int max_steps, double t_end, double* t,
            int* steps_done, double* dts);

/*
 * orc_run on the mesh split into blocks[0] x blocks[1] x blocks[2] blocks of
 * equal extents (blocks[d] divides n[d]; a split axis gives every block at
 * least 2 cells on it; blocks[d] = 1 for d >= ndim).  Each block keeps its
 * own cells and ghost zones: at a face shared by two blocks (a c-boundary,
 * which a periodic axis adds between its end blocks) each block writes its
 * two interior layers next to the face into the other's ghost zone; the
 * faces of the whole mesh follow the p-boundary rules; the time step is the
 * smallest over the blocks.  U is read and written in the mesh layout.
 */
int orc_run_blocks(const orc_mesh* m, const int32_t blocks[3], double* U, double cfl, int max_steps,
                   double t_end, double* t, int* steps_done, double* dts);

/*
 * Static mesh refinement of the block mesh of orc_run_blocks (Sec. 2.3: a
 * refined block is replaced by 2^ndim blocks of half its size with the same
 * cell count, recursively).  refined[] lists nref blocks to refine, each by
 * its code L * 2^26 + (index on the level-L block grid of B_d 2^L blocks per
 * axis, x fastest); a block of level L >= 1 must follow its parent, and L <= 2
 * (leaves reach level 3 at most).  Refinement is added, refining the coarser
 * side, until face-neighbouring leaves differ by at most one level.
 * Refinement needs an even block extent of at least 4 cells on every active
 * axis.  Leaves are ordered by level, and within a level by their index on
 * that level's grid; fields are in the block layout [leaf][comp][k][j][i] of
 * one block's extents.  Cross-level c-boundaries: restriction (pairwise
 * volume averages) onto coarse ghosts, then minmod-limited prolongation onto
 * fine ghosts level by level from the coarsest, fluxes, and the average of
 * the fine fluxes on the coarse side of each level jump; all on primitive
 * variables; one global time step.  Both integrators: Heun, or van Leer
 * with both stages (the piecewise-constant predictor and the PLM corrector)
 * taking the same cross-level ghosts and flux averages.
 *
 * orc_smr_leaves writes (level, c0, c1, c2) per leaf (at most max) and
 * returns the leaf count, or -1 for an invalid refinement.
 * orc_smr_ghosts fills every leaf's padded primitive array (n_gh = 2, the
 * orc_fill_ghosts layout per leaf) from the primitive block-layout field W.
 * orc_smr_totals: the conserved totals, sum over leaves of dV_level U.
 */
int orc_smr_leaves(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined,
                   int32_t* leaves, int max);
int orc_smr_ghosts(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined,
                   const double* W, double* Wpad);
int orc_run_smr(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined, double* U,
                double cfl, int max_steps, double t_end, double* t, int* steps_done, double* dts);
void orc_smr_totals(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined,
                    const double* U, double* totals);

/* dV-weighted conserved totals, compensated (Neumaier) sums in storage order. */
void orc_totals(const orc_mesh* m, const double* U, double* totals);

/*
 * Sampled evaluation for large meshes: for each of the ns flat cell indices
 * in cells[], out[c*ns + s] receives, for orc_rhs_cells, the stage right-hand
 * side at that cell, and for orc_step_cells, the state after one Heun step.
 */
int orc_rhs_cells(const orc_mesh* m, const double* U, double dt, int ns, const int64_t* cells,
                  double* out);
int orc_step_cells(const orc_mesh* m, const double* U, double dt, int ns, const int64_t* cells,
                   double* out);

/* ---- exact Riemann solver (validator for the scheme; exact_riemann.c) ---- */

/*
 * Star-region pressure and velocity of the exact Riemann problem for a
 * gamma-law gas.  method 0 = Newton from the primitive-variable guess,
 * method 1 = bisection.  Returns 0, or -1 when the data generate vacuum or
 * are not positive.
 */
int orc_exact_star(double gamma, double rl, double ul, double pl, double rr, double ur, double pr,
                   int method, double* pstar, double* ustar);

/* Sample the exact solution at similarity coordinate xi = (x - x0)/t. */
int orc_exact_sample(double gamma, double rl, double ul, double pl, double rr, double ur, double pr,
                     double xi, double* rho, double* u, double* p);

#ifdef __cplusplus
}
#endif

#endif
