/*
 * hydro_oracle.c -- TEST INFRASTRUCTURE ONLY (see hydro_oracle.h).
 *
 * Plain FP64 reference of the Godunov step of arXiv 2501.02317, Sec. 3.
 * Every function follows the paper's order of operations:
 *   cons -> prim (Sec. 3.1), ghost zones from the boundary rules (Sec. 3.1.1),
 *   PLM with minmod on primitive variables (eq. minmod, Sec. 3.2.2),
 *   HLLC with the subtraction-safe wave speeds (eqs. hllc-contact-spd and
 *   hllc-mixed-dvel; star states and fluxes from Toro's HLLC, which the paper
 *   cites for the solver), flux-divergence update and the Heun integrator
 *   (Sec. 3.3), CFL time step on the first sub-step (Sec. 3.1).
 *
 * No blocking, fusion or reordering: each face flux is computed once from the
 * padded primitive array, and each cell sums its face differences in axis
 * order x, y, z.  Built without FMA contraction.  The OpenMP pragmas only
 * distribute independent faces and cells over threads; the arithmetic of each
 * value is unchanged, so results do not depend on the thread count.
 */
#include "hydro_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NGH 2   /* ghost layers: PLM is second order (Sec. 3.1, n_gh = spatial order) */
#define MAXC 5  /* largest ncomp (3-D) */

enum { VM_NONE = 0, VM_NEG = 1, VM_CLIP_LO = 2, VM_CLIP_HI = 3 };

/* ------------------------------------------------------------------ mesh */

static int mesh_ok(const orc_mesh* m) {
    if (!m || m->ndim < 1 || m->ndim > 3) return 0;
    if (!(m->gamma > 1.0) || !isfinite(m->gamma)) return 0;
    if (m->integrator != ORC_HEUN && m->integrator != ORC_VL2) return 0;
    for (int d = 0; d < 3; ++d) {
        if (d < m->ndim) {
            if (m->n[d] < 1 || !(m->hi[d] > m->lo[d])) return 0;
            for (int s = 0; s < 2; ++s)
                if (m->bc[d][s] < ORC_BC_PERIODIC || m->bc[d][s] > ORC_BC_REFLECT) return 0;
            int per0 = m->bc[d][0] == ORC_BC_PERIODIC, per1 = m->bc[d][1] == ORC_BC_PERIODIC;
            if (per0 != per1) return 0;
            /* periodic and reflecting ghosts read n_gh distinct interior cells */
            if ((per0 || m->bc[d][0] == ORC_BC_REFLECT || m->bc[d][1] == ORC_BC_REFLECT) &&
                m->n[d] < NGH)
                return 0;
        } else if (m->n[d] != 1) {
            return 0;
        }
    }
    return 1;
}

int orc_ncomp(const orc_mesh* m) { return mesh_ok(m) ? m->ndim + 2 : -1; }

static int64_t ncells(const orc_mesh* m) { return (int64_t)m->n[0] * m->n[1] * m->n[2]; }

static double cell_width(const orc_mesh* m, int d) { return (m->hi[d] - m->lo[d]) / m->n[d]; }

/* ------------------------------------------------------- pointwise physics */

double orc_minmod(double a, double b) {
    /* eq. minmod: the smaller-magnitude argument when both have the same
     * strict sign, zero otherwise (including when either is zero). */
    if ((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0)) return fabs(a) < fabs(b) ? a : b;
    return 0.0;
}

static int admissible(int nc, const double* u, double rho, double p) {
    for (int c = 0; c < nc; ++c)
        if (!isfinite(u[c])) return 0;
    return rho > 0.0 && p > 0.0 && isfinite(p);
}

/* v_d = m_d / rho ; p = (gamma - 1) (E - (1/2) sum_d m_d v_d)   (Sec. 3.1) */
static int cons_to_prim_cell(int ndim, double g, const double* u, double* w) {
    double rho = u[0];
    double ke2 = 0.0; /* twice the kinetic energy density, summed in axis order */
    w[0] = rho;
    for (int d = 0; d < ndim; ++d) {
        double v = u[1 + d] / rho;
        w[1 + d] = v;
        ke2 = ke2 + u[1 + d] * v;
    }
    double p = (g - 1.0) * (u[ndim + 1] - 0.5 * ke2);
    w[ndim + 1] = p;
    return admissible(ndim + 2, u, rho, p);
}

/* m_d = rho v_d ; E = p / (gamma - 1) + (1/2) sum_d m_d v_d   (eq. hydro) */
static void prim_to_cons_cell(int ndim, double g, const double* w, double* u) {
    double rho = w[0];
    double ke2 = 0.0;
    u[0] = rho;
    for (int d = 0; d < ndim; ++d) {
        double mom = rho * w[1 + d];
        u[1 + d] = mom;
        ke2 = ke2 + mom * w[1 + d];
    }
    u[ndim + 1] = w[ndim + 1] / (g - 1.0) + 0.5 * ke2;
}

void orc_prim_to_cons(const orc_mesh* m, const double* W, double* U) {
    if (!mesh_ok(m)) return;
    int nc = m->ndim + 2;
    int64_t N = ncells(m);
    for (int64_t i = 0; i < N; ++i) {
        double w[MAXC] = {0}, u[MAXC] = {0};
        for (int c = 0; c < nc; ++c) w[c] = W[c * N + i];
        prim_to_cons_cell(m->ndim, m->gamma, w, u);
        for (int c = 0; c < nc; ++c) U[c * N + i] = u[c];
    }
}

int orc_cons_to_prim(const orc_mesh* m, const double* U, double* W) {
    if (!mesh_ok(m)) return -1;
    int nc = m->ndim + 2;
    int64_t N = ncells(m);
    int bad = 0;
    for (int64_t i = 0; i < N; ++i) {
        double w[MAXC] = {0}, u[MAXC] = {0};
        for (int c = 0; c < nc; ++c) u[c] = U[c * N + i];
        if (!cons_to_prim_cell(m->ndim, m->gamma, u, w)) ++bad;
        for (int c = 0; c < nc; ++c) W[c * N + i] = w[c];
    }
    return bad;
}

/* ------------------------------------------------------------------ HLLC */

/* Conserved state and physical flux of a normal-frame primitive state
 * (rho, u, t_1..t_nt, p): U = (rho, rho u, rho t, E), F = (rho u, rho u u + p,
 * rho u t, (E + p) u), with E = p/(gamma-1) + (1/2)(rho u u + (sum rho t t)).
 * The tangential terms are summed first (two at most, so their order does
 * not matter): interchanging the two tangential axes leaves E bitwise equal. */
static void state_and_flux(double g, int nt, const double* W, double* U, double* F) {
    int nc = nt + 3;
    double rho = W[0], u = W[1], p = W[nc - 1];
    double mu = rho * u;
    double ket = 0.0;
    U[0] = rho;
    U[1] = mu;
    for (int k = 0; k < nt; ++k) {
        double mt = rho * W[2 + k];
        U[2 + k] = mt;
        ket = ket + mt * W[2 + k];
    }
    double ke2 = mu * u + ket;
    double E = p / (g - 1.0) + 0.5 * ke2;
    U[nc - 1] = E;
    F[0] = mu;
    F[1] = mu * u + p;
    for (int k = 0; k < nt; ++k) F[2 + k] = mu * W[2 + k];
    F[nc - 1] = (E + p) * u;
}

/* HLLC star state of side K (Toro's form): chi = rho_K ds_K / (s_K - s_*),
 * U* = chi (1, s_*, t_K, E_K/rho_K + (s_* - u_K)(s_* + p_K/(rho_K ds_K))). */
static void star_state(int nt, const double* W, const double* U, double sK, double dsK,
                       double ss, double* Us) {
    int nc = nt + 3;
    double rho = W[0], u = W[1], p = W[nc - 1];
    double chi = rho * dsK / (sK - ss);
    Us[0] = chi;
    Us[1] = chi * ss;
    for (int k = 0; k < nt; ++k) Us[2 + k] = chi * W[2 + k];
    Us[nc - 1] = chi * (U[nc - 1] / rho + (ss - u) * (ss + p / (rho * dsK)));
}

void orc_hllc(double g, int nt, const double* WL, const double* WR, double* F, double* detail) {
    int nc = nt + 3;
    double UL[MAXC], UR[MAXC], FL[MAXC], FR[MAXC];
    double UsL[MAXC], UsR[MAXC], FsL[MAXC], FsR[MAXC];
    state_and_flux(g, nt, WL, UL, FL);
    state_and_flux(g, nt, WR, UR, FR);

    double rl = WL[0], ul = WL[1], pl = WL[nc - 1];
    double rr = WR[0], ur = WR[1], pr = WR[nc - 1];
    double cl = sqrt(g * pl / rl);
    double cr = sqrt(g * pr / rr);

    /* pressure estimate for the wave speeds: primitive-variable guess, >= 0 */
    double ppv = 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr);
    double ps = ppv > 0.0 ? ppv : 0.0;

    /* eq. hllc-mixed-dvel: ds_L = -c_L q_L, ds_R = c_R q_R */
    double z = (g + 1.0) / (2.0 * g);
    double ratl = ps / pl, ratr = ps / pr;
    double ql = sqrt(1.0 + z * ((ratl > 1.0 ? ratl : 1.0) - 1.0));
    double qr = sqrt(1.0 + z * ((ratr > 1.0 ? ratr : 1.0) - 1.0));
    double dsl = -cl * ql;
    double dsr = cr * qr;
    double sl = ul + dsl;
    double sr = ur + dsr;

    /* eq. hllc-contact-spd with (s_K - u_K) replaced by ds_K */
    double ss = ((pr - rr * ur * dsr) - (pl - rl * ul * dsl)) / (rl * dsl - rr * dsr);

    star_state(nt, WL, UL, sl, dsl, ss, UsL);
    star_state(nt, WR, UR, sr, dsr, ss, UsR);
    for (int c = 0; c < nc; ++c) {
        FsL[c] = FL[c] + sl * (UsL[c] - UL[c]);
        FsR[c] = FR[c] + sr * (UsR[c] - UR[c]);
    }

    const double* pick;
    if (sl >= 0.0)
        pick = FL;
    else if (ss >= 0.0)
        pick = FsL;
    else if (sr > 0.0)
        pick = FsR;
    else
        pick = FR;
    for (int c = 0; c < nc; ++c) F[c] = pick[c];

    if (detail) {
        double* o = detail;
        *o++ = sl;
        *o++ = ss;
        *o++ = sr;
        *o++ = ps;
        const double* blocks[8] = {UL, UR, FL, FR, UsL, UsR, FsL, FsR};
        for (int b = 0; b < 8; ++b)
            for (int c = 0; c < nc; ++c) *o++ = blocks[b][c];
    }
}

/* ------------------------------------------------------------------- PLM */

void orc_plm_face(const double w[4], double* wl, double* wr) {
    double dj = orc_minmod(w[1] - w[0], w[2] - w[1]);  /* slope of cell j   */
    double dj1 = orc_minmod(w[2] - w[1], w[3] - w[2]); /* slope of cell j+1 */
    *wl = w[1] + 0.5 * dj;
    *wr = w[2] - 0.5 * dj1;
}

/* Flux through the face between w4[1] and w4[2] along axis d, from the
 * global-frame primitive states of the four cells around it: reconstruct each
 * component, rotate so the face normal is the first velocity, solve, rotate back. */
static void face_flux(int ndim, double g, int d, int order, const double (*w4)[MAXC], double* F) {
    int nc = ndim + 2;
    double wl[MAXC], wr[MAXC];
    for (int c = 0; c < nc; ++c) {
        if (order == 1) {
            /* piecewise-constant reconstruction: the face states are the cells' values */
            wl[c] = w4[1][c];
            wr[c] = w4[2][c];
        } else {
            double col[4] = {w4[0][c], w4[1][c], w4[2][c], w4[3][c]};
            orc_plm_face(col, &wl[c], &wr[c]);
        }
    }
    double WLn[MAXC], WRn[MAXC], Fn[MAXC];
    WLn[0] = wl[0];
    WRn[0] = wr[0];
    WLn[1] = wl[1 + d];
    WRn[1] = wr[1 + d];
    int k = 2;
    for (int e = 0; e < ndim; ++e) {
        if (e == d) continue;
        WLn[k] = wl[1 + e];
        WRn[k] = wr[1 + e];
        ++k;
    }
    WLn[nc - 1] = wl[nc - 1];
    WRn[nc - 1] = wr[nc - 1];
    orc_hllc(g, ndim - 1, WLn, WRn, Fn, NULL);
    F[0] = Fn[0];
    F[1 + d] = Fn[1];
    k = 2;
    for (int e = 0; e < ndim; ++e) {
        if (e == d) continue;
        F[1 + e] = Fn[k++];
    }
    F[nc - 1] = Fn[nc - 1];
}

/* ------------------------------------------------------------ boundaries */

/* Interior cell copied into the ghost at position g (g < 0 or g >= N) along an
 * axis, and the treatment of the normal velocity there (Sec. 3.1.1, each side
 * read as the left-x case after rotation). */
static int ghost_src(const orc_mesh* m, int d, int g, int* vmode) {
    int N = m->n[d];
    *vmode = VM_NONE;
    if (g < 0) {
        switch (m->bc[d][0]) {
            case ORC_BC_PERIODIC: return g + N;
            case ORC_BC_FREE: return 0;
            case ORC_BC_OUTFLOW: *vmode = VM_CLIP_LO; return 0;
            default: *vmode = VM_NEG; return -1 - g;
        }
    }
    switch (m->bc[d][1]) {
        case ORC_BC_PERIODIC: return g - N;
        case ORC_BC_FREE: return N - 1;
        case ORC_BC_OUTFLOW: *vmode = VM_CLIP_HI; return N - 1;
        default: *vmode = VM_NEG; return 2 * N - 1 - g;
    }
}

static double apply_vmode(double v, int vmode) {
    switch (vmode) {
        case VM_NEG: return -v;
        case VM_CLIP_LO: return v > 0.0 ? 0.0 : v; /* min{v, 0}: no inflow at the low side  */
        case VM_CLIP_HI: return v < 0.0 ? 0.0 : v; /* max{v, 0}: no inflow at the high side */
        default: return v;
    }
}

/* padded geometry */
typedef struct {
    int pad[3];
    int64_t P[3];
    int64_t total;
} padgeo;

static padgeo pad_geometry(const orc_mesh* m) {
    padgeo p;
    p.total = 1;
    for (int d = 0; d < 3; ++d) {
        p.pad[d] = d < m->ndim ? NGH : 0;
        p.P[d] = m->n[d] + 2 * p.pad[d];
        p.total *= p.P[d];
    }
    return p;
}

static int64_t pidx(const padgeo* p, int i, int j, int k) {
    return ((int64_t)(k + p->pad[2]) * p->P[1] + (j + p->pad[1])) * p->P[0] + (i + p->pad[0]);
}

/* Ghosts of the sides whose cside[d][s] is set were written by a neighbouring
 * block (c-boundaries); the others follow the p-boundary rules. */
static void fill_ghosts_masked(const orc_mesh* m, double* Wpad, const int (*cside)[2]) {
    int nc = m->ndim + 2;
    padgeo pg = pad_geometry(m);
    for (int d = 0; d < m->ndim; ++d) {
        int N = m->n[d];
        int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
        int ghosts[4] = {-2, -1, N, N + 1};
        /* lines along d through interior transverse positions only: the
         * axis-aligned stencil never reads corner ghosts */
        for (int a = 0; a < m->n[e1]; ++a)
            for (int b = 0; b < m->n[e2]; ++b)
                for (int q = 0; q < 4; ++q) {
                    if (cside && cside[d][q < 2 ? 0 : 1]) continue;
                    int vmode;
                    int src = ghost_src(m, d, ghosts[q], &vmode);
                    int gi[3], si[3];
                    gi[d] = ghosts[q];
                    si[d] = src;
                    gi[e1] = si[e1] = a;
                    gi[e2] = si[e2] = b;
                    int64_t go = pidx(&pg, gi[0], gi[1], gi[2]);
                    int64_t so = pidx(&pg, si[0], si[1], si[2]);
                    for (int c = 0; c < nc; ++c) Wpad[c * pg.total + go] = Wpad[c * pg.total + so];
                    Wpad[(1 + d) * pg.total + go] = apply_vmode(Wpad[(1 + d) * pg.total + go], vmode);
                }
    }
}

int orc_fill_ghosts(const orc_mesh* m, double* Wpad) {
    if (!mesh_ok(m)) return -1;
    fill_ghosts_masked(m, Wpad, NULL);
    return 0;
}

/* ------------------------------------------------------------- stage rhs */

static int rhs_core(const orc_mesh* m, const double* dx, const int (*cside)[2], double* Wp, double dt,
                    int order, double* dU);

static int rhs_padded(const orc_mesh* m, double* Wp, double dt, int order, double* dU) {
    return rhs_core(m, NULL, NULL, Wp, dt, order, dU);
}

int orc_rhs(const orc_mesh* m, const double* U, double dt, double* dU) {
    if (!mesh_ok(m)) return -1;
    int ndim = m->ndim, nc = ndim + 2;
    double g = m->gamma;
    int64_t N = ncells(m);
    int n0 = m->n[0], n1 = m->n[1], n2 = m->n[2];
    padgeo pg = pad_geometry(m);

    double* Wp = (double*)calloc((size_t)(nc * pg.total), sizeof(double));
    if (!Wp) return -1;
    int bad = 0;
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                int64_t cell = ((int64_t)k * n1 + j) * n0 + i;
                double u[MAXC], w[MAXC];
                for (int c = 0; c < nc; ++c) u[c] = U[c * N + cell];
                if (!cons_to_prim_cell(ndim, g, u, w)) ++bad;
                int64_t o = pidx(&pg, i, j, k);
                for (int c = 0; c < nc; ++c) Wp[c * pg.total + o] = w[c];
            }
    if (bad) {
        free(Wp);
        return bad;
    }
    int rc = rhs_padded(m, Wp, dt, 2, dU);
    free(Wp);
    return rc;
}

int orc_rhs_prim(const orc_mesh* m, const double* W, double dt, int order, double* dU) {
    if (!mesh_ok(m) || (order != 1 && order != 2)) return -1;
    int nc = m->ndim + 2;
    int64_t N = ncells(m);
    int n0 = m->n[0], n1 = m->n[1], n2 = m->n[2];
    padgeo pg = pad_geometry(m);
    double* Wp = (double*)calloc((size_t)(nc * pg.total), sizeof(double));
    if (!Wp) return -1;
    int bad = 0;
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                int64_t cell = ((int64_t)k * n1 + j) * n0 + i;
                double w[MAXC];
                for (int c = 0; c < nc; ++c) w[c] = W[c * N + cell];
                if (!(w[0] > 0.0) || !(w[nc - 1] > 0.0)) ++bad;
                for (int c = 0; c < nc; ++c)
                    if (!isfinite(w[c])) ++bad;
                int64_t o = pidx(&pg, i, j, k);
                for (int c = 0; c < nc; ++c) Wp[c * pg.total + o] = w[c];
            }
    int rc = bad ? bad : rhs_padded(m, Wp, dt, order, dU);
    free(Wp);
    return rc;
}

/* Face fluxes of one block from its padded primitive array Wp (ghosts
 * filled): axis d has n_d + 1 faces per line, face f separating cells f-1 and
 * f, stored [comp][face] with extents fext[d].  Piecewise-constant (order 1)
 * or PLM (order 2) face states. */
typedef struct {
    double* F[3];
    int64_t fext[3][3];
    int64_t nf[3];
} faceflux;

static void faceflux_free(faceflux* ff) {
    for (int d = 0; d < 3; ++d) {
        free(ff->F[d]);
        ff->F[d] = NULL;
    }
}

static int block_fluxes(const orc_mesh* m, const double* Wp, int order, faceflux* ff) {
    int ndim = m->ndim, nc = ndim + 2;
    double g = m->gamma;
    padgeo pg = pad_geometry(m);
    for (int d = 0; d < 3; ++d) ff->F[d] = NULL;
    for (int d = 0; d < ndim; ++d) {
        for (int e = 0; e < 3; ++e) ff->fext[d][e] = m->n[e] + (e == d ? 1 : 0);
        int64_t nf = ff->fext[d][0] * ff->fext[d][1] * ff->fext[d][2];
        ff->nf[d] = nf;
        ff->F[d] = (double*)malloc((size_t)(nc * nf) * sizeof(double));
        if (!ff->F[d]) {
            faceflux_free(ff);
            return -1;
        }
        double* Fd = ff->F[d];
        const int64_t* fext = ff->fext[d];
#pragma omp parallel for schedule(static)
        for (int fk = 0; fk < (int)fext[2]; ++fk)
            for (int fj = 0; fj < (int)fext[1]; ++fj)
                for (int fi = 0; fi < (int)fext[0]; ++fi) {
                    int f[3] = {fi, fj, fk};
                    double w4[4][MAXC];
                    for (int s = 0; s < 4; ++s) {
                        int c3[3] = {fi, fj, fk};
                        c3[d] = f[d] - 2 + s;
                        int64_t o = pidx(&pg, c3[0], c3[1], c3[2]);
                        for (int c = 0; c < nc; ++c) w4[s][c] = Wp[c * pg.total + o];
                    }
                    double F[MAXC];
                    face_flux(ndim, g, d, order, w4, F);
                    int64_t fo = ((int64_t)fk * fext[1] + fj) * fext[0] + fi;
                    for (int c = 0; c < nc; ++c) Fd[c * nf + fo] = F[c];
                }
    }
    return 0;
}

/* dU_i = sum over d (in order) of dt/dx_d (F_{d,i-1/2} - F_{d,i+1/2}) */
static void flux_update(const orc_mesh* m, const double* dx, const faceflux* ff, double dt, double* dU) {
    int ndim = m->ndim, nc = ndim + 2;
    int64_t N = ncells(m);
    int n0 = m->n[0], n1 = m->n[1], n2 = m->n[2];
    double lam[3];
    for (int d = 0; d < ndim; ++d) lam[d] = dt / (dx ? dx[d] : cell_width(m, d));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                int64_t cell = ((int64_t)k * n1 + j) * n0 + i;
                int c3[3] = {i, j, k};
                for (int c = 0; c < nc; ++c) {
                    double acc = 0.0;
                    for (int d = 0; d < ndim; ++d) {
                        const int64_t* fext = ff->fext[d];
                        int64_t nf = ff->nf[d];
                        int lo3[3] = {c3[0], c3[1], c3[2]};
                        int hi3[3] = {c3[0], c3[1], c3[2]};
                        hi3[d] += 1;
                        int64_t flo = ((int64_t)lo3[2] * fext[1] + lo3[1]) * fext[0] + lo3[0];
                        int64_t fhi = ((int64_t)hi3[2] * fext[1] + hi3[1]) * fext[0] + hi3[0];
                        acc = acc + lam[d] * (ff->F[d][c * nf + flo] - ff->F[d][c * nf + fhi]);
                    }
                    dU[c * N + cell] = acc;
                }
            }
}

/* Stage right-hand side from the padded primitive array Wp (interior filled;
 * the ghosts of sides not marked in cside are filled here by the boundary
 * rules), with piecewise-constant (order 1) or PLM (order 2) face states.
 * dx: cell widths (NULL: those of m). */
static int rhs_core(const orc_mesh* m, const double* dx, const int (*cside)[2], double* Wp, double dt,
                    int order, double* dU) {
    fill_ghosts_masked(m, Wp, cside);
    faceflux ff;
    if (block_fluxes(m, Wp, order, &ff)) return -1;
    flux_update(m, dx, &ff, dt, dU);
    faceflux_free(&ff);
    return 0;
}

/* ------------------------------------------------------------ integrator */

int orc_heun_step(const orc_mesh* m, double* U, double dt) {
    if (!mesh_ok(m) || !(dt > 0.0) || !isfinite(dt)) return -1;
    int nc = m->ndim + 2;
    int64_t N = ncells(m), tot = nc * N;
    double* U1 = (double*)malloc((size_t)tot * sizeof(double));
    double* dU = (double*)malloc((size_t)tot * sizeof(double));
    if (!U1 || !dU) {
        free(U1);
        free(dU);
        return -1;
    }
    int rc = orc_rhs(m, U, dt, dU);
    if (rc == 0) {
        /* predictor U1 = U^n + dU(U^n), kept in full precision (Sec. 3.3) */
        for (int64_t q = 0; q < tot; ++q) U1[q] = U[q] + dU[q];
        rc = orc_rhs(m, U1, dt, dU);
    }
    if (rc == 0) {
        /* corrector U^{n+1} = (1/2) U^n + (1/2) (U1 + dU(U1)) */
        for (int64_t q = 0; q < tot; ++q) U[q] = 0.5 * U[q] + 0.5 * (U1[q] + dU[q]);
    }
    free(U1);
    free(dU);
    return rc;
}

/* The memory-optimised van Leer integrator (Sec. 3.3): a half-step
 * predictor with piecewise-constant states, U* = U^n + (dt/2) L_1(U^n),
 * kept only as primitive variables W* = W(U*); then the full step from the
 * PLM fluxes of W*, U^{n+1} = U^n + dt L_2(W*).  The predictor never enters
 * U^{n+1} directly, so it may be stored at reduced precision. */
int orc_vl2_step(const orc_mesh* m, double* U, double dt) {
    if (!mesh_ok(m) || !(dt > 0.0) || !isfinite(dt)) return -1;
    int ndim = m->ndim, nc = ndim + 2;
    int64_t N = ncells(m), tot = nc * N;
    double* W = (double*)malloc((size_t)tot * sizeof(double));
    double* dU = (double*)malloc((size_t)tot * sizeof(double));
    if (!W || !dU) {
        free(W);
        free(dU);
        return -1;
    }
    int rc = orc_cons_to_prim(m, U, W);
    if (rc == 0) rc = orc_rhs_prim(m, W, 0.5 * dt, 1, dU);
    if (rc == 0) {
        /* W* = W(U^n + dU), cell by cell */
        for (int64_t i = 0; i < N && rc == 0; ++i) {
            double u[MAXC], w[MAXC];
            for (int c = 0; c < nc; ++c) u[c] = U[c * N + i] + dU[c * N + i];
            if (!cons_to_prim_cell(ndim, m->gamma, u, w)) rc = 1;
            for (int c = 0; c < nc; ++c) W[c * N + i] = w[c];
        }
    }
    if (rc == 0) rc = orc_rhs_prim(m, W, dt, 2, dU);
    if (rc == 0)
        for (int64_t q = 0; q < tot; ++q) U[q] = U[q] + dU[q];
    free(W);
    free(dU);
    return rc;
}

double orc_cfl_dt(const orc_mesh* m, const double* U, double cfl) {
    if (!mesh_ok(m) || !(cfl > 0.0)) return -1.0;
    int ndim = m->ndim, nc = ndim + 2;
    double g = m->gamma;
    int64_t N = ncells(m);
    double best = INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        double u[MAXC], w[MAXC];
        for (int c = 0; c < nc; ++c) u[c] = U[c * N + i];
        if (!cons_to_prim_cell(ndim, g, u, w)) return -1.0;
        double cs = sqrt(g * w[nc - 1] / w[0]);
        for (int d = 0; d < ndim; ++d) {
            double cand = cell_width(m, d) / (fabs(w[1 + d]) + cs);
            if (cand < best) best = cand;
        }
    }
    return cfl * best;
}

int orc_run(const orc_mesh* m, double* U, double cfl, int max_steps, double t_end, double* t,
            int* steps_done, double* dts) {
    if (!mesh_ok(m) || !t) return -1;
    if (max_steps <= 0 && !(t_end > 0.0)) return -1;
    int s = 0;
    int rc = 0;
    while (max_steps <= 0 || s < max_steps) {
        if (t_end > 0.0 && !(*t < t_end)) break;
        double dt = orc_cfl_dt(m, U, cfl);
        if (!(dt > 0.0)) {
            rc = 1;
            break;
        }
        int last = 0;
        if (t_end > 0.0 && dt >= t_end - *t) {
            dt = t_end - *t;
            last = 1;
        }
        rc = m->integrator == ORC_VL2 ? orc_vl2_step(m, U, dt) : orc_heun_step(m, U, dt);
        if (rc) break;
        if (dts) dts[s] = dt;
        *t = last ? t_end : *t + dt;
        ++s;
    }
    if (steps_done) *steps_done = s;
    return rc;
}

/* ------------------------------------------------------ multi-block mesh */

/* The mesh split into B[0] x B[1] x B[2] blocks of equal extents (every block
 * holds the same number of cells).  Block b = b0 + B0 (b1 + B1 b2) keeps its
 * cells in its own array, layout [b][comp][k][j][i] of the block's extents,
 * and its own padded primitive array.  At a face shared with another block
 * (a c-boundary) its ghost layers are the neighbour's n_gh interior layers
 * next to that face, which the neighbour writes straight into them; at the
 * faces of the whole mesh the p-boundary rules of Sec. 3.1.1 fill them.  A
 * periodic axis links the blocks at its two ends (one block on that axis is
 * its own neighbour, which is the periodic rule itself). */
typedef struct {
    orc_mesh mb;   /* one block: the block's extents, the mesh's boundary codes */
    int B[3];
    int nblk;
    int64_t nb;    /* cells per block */
    double dx[3];  /* the mesh's cell widths */
} blockgeo;

static int block_geometry(const orc_mesh* m, const int32_t* blocks, blockgeo* bg) {
    if (!mesh_ok(m) || !blocks) return 0;
    bg->mb = *m;
    bg->nblk = 1;
    for (int d = 0; d < 3; ++d) {
        int B = blocks[d];
        if (B < 1 || (d >= m->ndim && B != 1) || m->n[d] % B != 0) return 0;
        /* a neighbour supplies all n_gh ghost layers of a shared face */
        if (B > 1 && m->n[d] / B < NGH) return 0;
        bg->B[d] = B;
        bg->nblk *= B;
        bg->mb.n[d] = m->n[d] / B;
        bg->dx[d] = d < m->ndim ? cell_width(m, d) : 1.0;
    }
    bg->nb = ncells(&bg->mb);
    return mesh_ok(&bg->mb);
}

/* The block across side s (0: low, 1: high) of axis d from block b, or -1 at
 * a face of the whole mesh that is not periodic. */
static int block_nbr(const blockgeo* bg, int b, int d, int s) {
    int c[3] = {b % bg->B[0], (b / bg->B[0]) % bg->B[1], b / (bg->B[0] * bg->B[1])};
    int q = c[d] + (s ? 1 : -1);
    if (q < 0 || q >= bg->B[d]) {
        if (bg->mb.bc[d][s] != ORC_BC_PERIODIC) return -1;
        q = (q + bg->B[d]) % bg->B[d];
    }
    c[d] = q;
    return c[0] + bg->B[0] * (c[1] + bg->B[1] * c[2]);
}

/* Stage right-hand side of every block from X (conserved, or primitive when
 * prim is set), block layout; see orc_rhs and orc_rhs_prim. */
static int blocks_rhs(const blockgeo* bg, const double* X, int prim, double dt, int order, double* dU) {
    const orc_mesh* mb = &bg->mb;
    int ndim = mb->ndim, nc = ndim + 2;
    int n0 = mb->n[0], n1 = mb->n[1], n2 = mb->n[2];
    int64_t nb = bg->nb;
    padgeo pg = pad_geometry(mb);
    double* Wp = (double*)calloc((size_t)bg->nblk * nc * pg.total, sizeof(double));
    if (!Wp) return -1;
    int bad = 0;
    /* each block: its interior primitive state */
    for (int b = 0; b < bg->nblk; ++b) {
        const double* Xb = X + (int64_t)b * nc * nb;
        double* Wb = Wp + (int64_t)b * nc * pg.total;
        for (int k = 0; k < n2; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n0; ++i) {
                    int64_t cell = ((int64_t)k * n1 + j) * n0 + i;
                    double x[MAXC], w[MAXC];
                    for (int c = 0; c < nc; ++c) x[c] = Xb[c * nb + cell];
                    if (prim) {
                        for (int c = 0; c < nc; ++c) {
                            w[c] = x[c];
                            if (!isfinite(w[c])) ++bad;
                        }
                        if (!(w[0] > 0.0) || !(w[nc - 1] > 0.0)) ++bad;
                    } else if (!cons_to_prim_cell(ndim, mb->gamma, x, w)) {
                        ++bad;
                    }
                    int64_t o = pidx(&pg, i, j, k);
                    for (int c = 0; c < nc; ++c) Wb[c * pg.total + o] = w[c];
                }
    }
    if (bad) {
        free(Wp);
        return bad;
    }
    /* c-boundaries: each block writes its n_gh interior layers next to a
     * shared face into the neighbour's ghost layers on the other side of it
     * (its low layers 0, 1 become the low neighbour's ghosts N, N+1; its high
     * layers N-2, N-1 the high neighbour's ghosts -2, -1) */
    for (int b = 0; b < bg->nblk; ++b) {
        const double* Ws = Wp + (int64_t)b * nc * pg.total;
        for (int d = 0; d < ndim; ++d) {
            int N = mb->n[d];
            int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
            for (int s = 0; s < 2; ++s) {
                int nbr = block_nbr(bg, b, d, s);
                if (nbr < 0) continue;
                double* Wd = Wp + (int64_t)nbr * nc * pg.total;
                for (int a = 0; a < mb->n[e1]; ++a)
                    for (int bb = 0; bb < mb->n[e2]; ++bb)
                        for (int L = 0; L < NGH; ++L) {
                            int si[3], di[3];
                            si[d] = s == 0 ? L : N - NGH + L;
                            di[d] = s == 0 ? N + L : -NGH + L;
                            si[e1] = di[e1] = a;
                            si[e2] = di[e2] = bb;
                            int64_t so = pidx(&pg, si[0], si[1], si[2]);
                            int64_t go = pidx(&pg, di[0], di[1], di[2]);
                            for (int c = 0; c < nc; ++c) Wd[c * pg.total + go] = Ws[c * pg.total + so];
                        }
            }
        }
    }
    /* each block: the p-boundary ghosts, the fluxes and the update */
    int rc = 0;
    for (int b = 0; b < bg->nblk && rc == 0; ++b) {
        int cside[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int d = 0; d < ndim; ++d)
            for (int s = 0; s < 2; ++s) cside[d][s] = block_nbr(bg, b, d, s) >= 0;
        rc = rhs_core(mb, bg->dx, (const int(*)[2])cside, Wp + (int64_t)b * nc * pg.total, dt, order,
                      dU + (int64_t)b * nc * nb);
    }
    free(Wp);
    return rc;
}

/* conserved -> primitive over all blocks; returns the count of bad cells */
static int blocks_cons_to_prim(const blockgeo* bg, const double* U, double* W) {
    int nc = bg->mb.ndim + 2, bad = 0;
    for (int b = 0; b < bg->nblk; ++b)
        for (int64_t i = 0; i < bg->nb; ++i) {
            const int64_t o = (int64_t)b * nc * bg->nb + i;
            double u[MAXC], w[MAXC];
            for (int c = 0; c < nc; ++c) u[c] = U[o + c * bg->nb];
            if (!cons_to_prim_cell(bg->mb.ndim, bg->mb.gamma, u, w)) ++bad;
            for (int c = 0; c < nc; ++c) W[o + c * bg->nb] = w[c];
        }
    return bad;
}

static int blocks_heun_step(const blockgeo* bg, double* U, double dt) {
    int64_t tot = (int64_t)bg->nblk * (bg->mb.ndim + 2) * bg->nb;
    double* U1 = (double*)malloc((size_t)tot * sizeof(double));
    double* dU = (double*)malloc((size_t)tot * sizeof(double));
    int rc = (U1 && dU) ? blocks_rhs(bg, U, 0, dt, 2, dU) : -1;
    if (rc == 0) {
        for (int64_t q = 0; q < tot; ++q) U1[q] = U[q] + dU[q];
        rc = blocks_rhs(bg, U1, 0, dt, 2, dU);
    }
    if (rc == 0)
        for (int64_t q = 0; q < tot; ++q) U[q] = 0.5 * U[q] + 0.5 * (U1[q] + dU[q]);
    free(U1);
    free(dU);
    return rc;
}

static int blocks_vl2_step(const blockgeo* bg, double* U, double dt) {
    int64_t tot = (int64_t)bg->nblk * (bg->mb.ndim + 2) * bg->nb;
    double* W = (double*)malloc((size_t)tot * sizeof(double));
    double* dU = (double*)malloc((size_t)tot * sizeof(double));
    int rc = (W && dU) ? blocks_cons_to_prim(bg, U, W) : -1;
    if (rc == 0) rc = blocks_rhs(bg, W, 1, 0.5 * dt, 1, dU);
    if (rc == 0) {
        /* W* = W(U^n + dU), cell by cell */
        for (int64_t q = 0; q < tot; ++q) dU[q] = U[q] + dU[q];
        rc = blocks_cons_to_prim(bg, dU, W) ? 1 : 0;
    }
    if (rc == 0) rc = blocks_rhs(bg, W, 1, dt, 2, dU);
    if (rc == 0)
        for (int64_t q = 0; q < tot; ++q) U[q] = U[q] + dU[q];
    free(W);
    free(dU);
    return rc;
}

/* the global CFL step: the smallest over blocks of each block's own step */
static double blocks_cfl_dt(const blockgeo* bg, const double* U, double cfl) {
    int ndim = bg->mb.ndim, nc = ndim + 2;
    double g = bg->mb.gamma, best = INFINITY;
    for (int b = 0; b < bg->nblk; ++b) {
        double bb = INFINITY;
        for (int64_t i = 0; i < bg->nb; ++i) {
            double u[MAXC], w[MAXC];
            for (int c = 0; c < nc; ++c) u[c] = U[(int64_t)b * nc * bg->nb + c * bg->nb + i];
            if (!cons_to_prim_cell(ndim, g, u, w)) return -1.0;
            double cs = sqrt(g * w[nc - 1] / w[0]);
            for (int d = 0; d < ndim; ++d) {
                double cand = bg->dx[d] / (fabs(w[1 + d]) + cs);
                if (cand < bb) bb = cand;
            }
        }
        if (bb < best) best = bb;
    }
    return cfl * best;
}

/* mesh layout <-> block layout */
static void blocks_relayout(const orc_mesh* m, const blockgeo* bg, double* mesh_f, double* blk_f, int to_blocks) {
    int nc = m->ndim + 2;
    int64_t N = ncells(m);
    const int* nb = bg->mb.n;
    for (int k = 0; k < m->n[2]; ++k)
        for (int j = 0; j < m->n[1]; ++j)
            for (int i = 0; i < m->n[0]; ++i) {
                int b = i / nb[0] + bg->B[0] * (j / nb[1] + bg->B[1] * (k / nb[2]));
                int64_t lc = ((int64_t)(k % nb[2]) * nb[1] + (j % nb[1])) * nb[0] + (i % nb[0]);
                int64_t gc = ((int64_t)k * m->n[1] + j) * m->n[0] + i;
                for (int c = 0; c < nc; ++c) {
                    double* bp = blk_f + (int64_t)b * nc * bg->nb + c * bg->nb + lc;
                    double* mp = mesh_f + c * N + gc;
                    if (to_blocks)
                        *bp = *mp;
                    else
                        *mp = *bp;
                }
            }
}

int orc_run_blocks(const orc_mesh* m, const int32_t blocks[3], double* U, double cfl, int max_steps,
                   double t_end, double* t, int* steps_done, double* dts) {
    blockgeo bg;
    if (!block_geometry(m, blocks, &bg) || !t || !(cfl > 0.0)) return -1;
    if (max_steps <= 0 && !(t_end > 0.0)) return -1;
    int64_t tot = (int64_t)bg.nblk * (m->ndim + 2) * bg.nb;
    double* Ub = (double*)malloc((size_t)tot * sizeof(double));
    if (!Ub) return -1;
    blocks_relayout(m, &bg, U, Ub, 1);
    int s = 0, rc = 0;
    while (max_steps <= 0 || s < max_steps) {
        if (t_end > 0.0 && !(*t < t_end)) break;
        double dt = blocks_cfl_dt(&bg, Ub, cfl);
        if (!(dt > 0.0)) {
            rc = 1;
            break;
        }
        int last = 0;
        if (t_end > 0.0 && dt >= t_end - *t) {
            dt = t_end - *t;
            last = 1;
        }
        rc = m->integrator == ORC_VL2 ? blocks_vl2_step(&bg, Ub, dt) : blocks_heun_step(&bg, Ub, dt);
        if (rc) break;
        if (dts) dts[s] = dt;
        *t = last ? t_end : *t + dt;
        ++s;
    }
    blocks_relayout(m, &bg, U, Ub, 0);
    free(Ub);
    if (steps_done) *steps_done = s;
    return rc;
}

/* ------------------------------------------------- static mesh refinement */

/* Static refinement of the block mesh above (the 2^d-tree of Sec. 2.3):
 * a listed block is replaced by 2^d blocks of half its size, every block
 * keeping the same number of cells, recursively up to level SMR_MAXLEV - 1.
 * A listed block is named by a code, its level L times 2^SMR_LSHIFT plus its
 * index on the level-L block grid (B_d 2^L blocks per axis, x fastest); a
 * block of level L >= 1 can be listed only when its parent is.  As in the
 * paper, refinement is then added until face-neighbouring leaves differ by
 * at most one level: while a leaf of level L touches, across a face, a leaf
 * of level L - 2 or coarser, the coarser leaf is refined.  The leaves are
 * ordered by level, and within a level by their index on that level's grid.
 *
 * A stage follows the cross-level sequence of Sec. 3 (c-boundaries):
 *   (a) ghosts that involve no prolongation: same-level neighbours, the
 *       p-boundary rules at the mesh faces, and on a coarse block facing
 *       finer ones, the volume average (restriction) of the fine cells that
 *       cover each ghost;
 *   (b) prolongation on the coarse side, level by level from the coarsest,
 *       so the coarse block's ghost zone is complete when it is used: each
 *       fine ghost is its coarse cell's value plus, per axis, a quarter of
 *       the minmod-limited (eq. minmod) difference, signed by the side of the
 *       coarse centre the fine centre lies on;
 *   (c) fluxes on every block;
 *   (d) on a coarse face shared with finer blocks the flux is the average of
 *       the fine fluxes through it, so the mass, momentum and energy that
 *       leave one level enter the other.
 * All of this on primitive variables, as the paper's figure of the interface
 * shows; averages are taken pairwise along x, then y, then z. */
enum { NB_PHYS = 0, NB_SAME = 1, NB_COARSE = 2, NB_FINE = 3 };
#define SMR_MAXLEV 4
#define SMR_LSHIFT 26

typedef struct {
    orc_mesh mb;        /* one block: its extents, the mesh's boundary codes */
    int B[3];           /* root blocks per axis */
    int nleaf;
    int nlev;           /* levels present */
    int (*leaf)[4];     /* level, c0, c1, c2 */
    int* look[SMR_MAXLEV];  /* per level: block coordinates -> leaf index, or -1 */
    double dx[SMR_MAXLEV][3];  /* cell widths per level */
    int64_t nb;         /* cells per block */
} smrgeo;

static void smr_free(smrgeo* g) {
    free(g->leaf);
    for (int L = 0; L < SMR_MAXLEV; ++L) free(g->look[L]);
}

/* Extent of the level-L block grid on axis d. */
static int smr_extent(const smrgeo* g, int L, int d) { return d < g->mb.ndim ? g->B[d] << L : 1; }

static int64_t smr_count(const smrgeo* g, int L) {
    return (int64_t)smr_extent(g, L, 0) * smr_extent(g, L, 1) * smr_extent(g, L, 2);
}

static int64_t smr_key(const smrgeo* g, int L, const int* c) {
    int64_t e0 = (int64_t)g->B[0] << L, e1 = (int64_t)g->B[1] << L;
    return ((int64_t)c[2] * e1 + c[1]) * e0 + c[0];
}

static void smr_coords(const smrgeo* g, int L, int64_t f, int* c) {
    int64_t e0 = smr_extent(g, L, 0), e1 = smr_extent(g, L, 1);
    c[0] = (int)(f % e0);
    c[1] = (int)((f / e0) % e1);
    c[2] = (int)(f / (e0 * e1));
}

/* Index on the level L - 1 grid of the parent of level-L block c. */
static int64_t smr_parent(const smrgeo* g, int L, const int* c) {
    int pc[3];
    for (int e = 0; e < 3; ++e) pc[e] = e < g->mb.ndim ? c[e] / 2 : 0;
    return smr_key(g, L - 1, pc);
}

/* Whether level-L block f exists in the tree (a root, or a child of a
 * refined block), given the refined sets ref[0 .. L-1]. */
static int smr_exists(const smrgeo* g, char* const* ref, int L, const int* c) {
    return L == 0 || ref[L - 1][smr_parent(g, L, c)];
}

static int smr_geometry(const orc_mesh* m, const int32_t* blocks, int nref, const int32_t* refined, smrgeo* g) {
    memset(g, 0, sizeof(*g));
    blockgeo bg;
    if (!block_geometry(m, blocks, &bg) || nref < 0 || (nref > 0 && !refined)) return 0;
    g->mb = bg.mb;
    for (int d = 0; d < 3; ++d) {
        g->B[d] = bg.B[d];
        for (int L = 0; L < SMR_MAXLEV; ++L)
            g->dx[L][d] = d < m->ndim ? bg.dx[d] / (double)(1 << L) : 1.0;
        /* a refined block's children align with its cells: restriction of
         * n_gh coarse ghost layers needs 2 n_gh fine layers in one block */
        if (nref > 0 && d < m->ndim && (bg.mb.n[d] % 2 != 0 || bg.mb.n[d] < 2 * NGH)) return 0;
    }
    g->nb = bg.nb;
    char* ref[SMR_MAXLEV] = {0};
    int ok = 1;
    for (int L = 0; L < SMR_MAXLEV && ok; ++L) {
        ref[L] = (char*)calloc((size_t)smr_count(g, L), 1);
        ok = ref[L] != NULL;
    }
    const int64_t mask = ((int64_t)1 << SMR_LSHIFT) - 1;
    for (int r = 0; r < nref && ok; ++r) {
        int L = (int)(refined[r] >> SMR_LSHIFT);
        int64_t f = refined[r] & mask;
        if (refined[r] < 0 || L > SMR_MAXLEV - 2 || f >= smr_count(g, L) || ref[L][f]) {
            ok = 0;
            break;
        }
        ref[L][f] = 1;
    }
    /* every listed block exists: its parent is listed too */
    for (int L = 1; L < SMR_MAXLEV - 1 && ok; ++L)
        for (int64_t f = 0; f < smr_count(g, L) && ok; ++f) {
            int c[3];
            smr_coords(g, L, f, c);
            if (ref[L][f] && !smr_exists(g, ref, L, c)) ok = 0;
        }
    /* 2:1 balance across faces, by refining the coarser side */
    for (int changed = 1; changed && ok;) {
        changed = 0;
        for (int L = 2; L < SMR_MAXLEV; ++L)
            for (int64_t f = 0; f < smr_count(g, L); ++f) {
                int c[3];
                smr_coords(g, L, f, c);
                if (!smr_exists(g, ref, L, c) || (L < SMR_MAXLEV - 1 && ref[L][f])) continue;
                for (int d = 0; d < m->ndim; ++d)
                    for (int sd = 0; sd < 2; ++sd) {
                        int q[3] = {c[0], c[1], c[2]};
                        int E = smr_extent(g, L, d);
                        q[d] += sd ? 1 : -1;
                        if (q[d] < 0 || q[d] >= E) {
                            if (m->bc[d][sd] != ORC_BC_PERIODIC) continue;
                            q[d] = (q[d] + E) % E;
                        }
                        /* the neighbour region at level L: its ancestor at
                         * level L - 2 must not be a leaf */
                        int p1[3], p2[3];
                        for (int e = 0; e < 3; ++e) p1[e] = e < m->ndim ? q[e] / 2 : 0;
                        for (int e = 0; e < 3; ++e) p2[e] = e < m->ndim ? p1[e] / 2 : 0;
                        int64_t k2 = smr_key(g, L - 2, p2);
                        if (!ref[L - 2][k2]) {
                            ref[L - 2][k2] = 1;
                            changed = 1;
                        }
                    }
            }
        /* a block refined for balance may need its own parent refined */
        for (int L = SMR_MAXLEV - 2; L >= 1 && ok; --L)
            for (int64_t f = 0; f < smr_count(g, L); ++f) {
                int c[3];
                smr_coords(g, L, f, c);
                if (ref[L][f] && !smr_exists(g, ref, L, c)) {
                    ref[L - 1][smr_parent(g, L, c)] = 1;
                    changed = 1;
                }
            }
    }
    /* leaves, level by level */
    int64_t nleaf = 0;
    for (int L = 0; L < SMR_MAXLEV && ok; ++L)
        for (int64_t f = 0; f < smr_count(g, L); ++f) {
            int c[3];
            smr_coords(g, L, f, c);
            if (smr_exists(g, ref, L, c) && !ref[L][f]) ++nleaf;
        }
    if (ok && nleaf > 0) {
        g->leaf = (int(*)[4])malloc((size_t)nleaf * sizeof(*g->leaf));
        ok = g->leaf != NULL;
    }
    for (int L = 0; L < SMR_MAXLEV && ok; ++L) {
        g->look[L] = (int*)malloc((size_t)smr_count(g, L) * sizeof(int));
        ok = g->look[L] != NULL;
    }
    int q = 0;
    for (int L = 0; L < SMR_MAXLEV && ok; ++L)
        for (int64_t f = 0; f < smr_count(g, L); ++f) {
            int c[3];
            smr_coords(g, L, f, c);
            g->look[L][f] = -1;
            if (!smr_exists(g, ref, L, c) || ref[L][f]) continue;
            g->leaf[q][0] = L;
            g->leaf[q][1] = c[0];
            g->leaf[q][2] = c[1];
            g->leaf[q][3] = c[2];
            g->look[L][f] = q++;
            if (L + 1 > g->nlev) g->nlev = L + 1;
        }
    for (int L = 0; L < SMR_MAXLEV; ++L) free(ref[L]);
    g->nleaf = q;
    return ok && q == nleaf;
}

/* What lies across side s of axis d of leaf b: NB_PHYS; the leaf index of a
 * same-level (NB_SAME) or one-level coarser (NB_COARSE) neighbour; or
 * NB_FINE with root the level-L coordinates of the refined neighbour block,
 * whose children next to the face are leaves one level finer. */
static int smr_nbr(const smrgeo* g, int b, int d, int s, int* idx, int* root) {
    int L = g->leaf[b][0];
    int c[3] = {g->leaf[b][1], g->leaf[b][2], g->leaf[b][3]};
    int E = smr_extent(g, L, d);
    int q = c[d] + (s ? 1 : -1);
    if (q < 0 || q >= E) {
        if (g->mb.bc[d][s] != ORC_BC_PERIODIC) return NB_PHYS;
        q = (q + E) % E;
    }
    c[d] = q;
    int same = g->look[L][smr_key(g, L, c)];
    if (same >= 0) {
        *idx = same;
        return NB_SAME;
    }
    if (L > 0) {
        int par = g->look[L - 1][smr_parent(g, L, c)];
        if (par >= 0) {
            *idx = par;
            return NB_COARSE;
        }
    }
    for (int e = 0; e < 3; ++e) root[e] = c[e];
    return NB_FINE;
}

/* the level-L leaf holding cell (x, y, z) of the level-L cell grid, and the
 * cell's block-local coordinates */
static int smr_fine_cell(const smrgeo* g, int L, const int* x, int* local) {
    int c[3];
    for (int e = 0; e < 3; ++e) {
        c[e] = x[e] / g->mb.n[e];
        local[e] = x[e] % g->mb.n[e];
    }
    return g->look[L][smr_key(g, L, c)];
}

/* Pairwise means of 2^k values along x, then y, then z (bit 0 of the index
 * is the x offset): equal values give the value back exactly. */
static double tree_mean(double* v, int k) {
    int n = 1 << k;
    for (int a = 0; a < k; ++a) {
        n >>= 1;
        for (int i = 0; i < n; ++i) v[i] = 0.5 * (v[2 * i] + v[2 * i + 1]);
    }
    return v[0];
}

/* Fill every ghost of every leaf's padded primitive array (interiors set). */
static void smr_fill_ghosts(const smrgeo* g, double* Wp) {
    const orc_mesh* mb = &g->mb;
    int ndim = mb->ndim, nc = ndim + 2;
    padgeo pg = pad_geometry(mb);
    const int* n = mb->n;
    /* (a) same-level copies, restriction onto coarse ghosts, p-boundaries */
    for (int b = 0; b < g->nleaf; ++b) {
        double* Wd = Wp + (int64_t)b * nc * pg.total;
        int cside[3][2] = {{0, 0}, {0, 0}, {0, 0}};
        for (int d = 0; d < ndim; ++d) {
            int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
            for (int s = 0; s < 2; ++s) {
                int idx = -1, root[3] = {0, 0, 0};
                int kind = smr_nbr(g, b, d, s, &idx, root);
                cside[d][s] = kind != NB_PHYS;
                if (kind == NB_SAME) {
                    const double* Ws = Wp + (int64_t)idx * nc * pg.total;
                    for (int a = 0; a < n[e1]; ++a)
                        for (int bb = 0; bb < n[e2]; ++bb)
                            for (int l = 0; l < NGH; ++l) {
                                int gi[3], si[3];
                                gi[d] = s ? n[d] + l : -1 - l;
                                si[d] = s ? l : n[d] - 1 - l;
                                gi[e1] = si[e1] = a;
                                gi[e2] = si[e2] = bb;
                                int64_t go = pidx(&pg, gi[0], gi[1], gi[2]), so = pidx(&pg, si[0], si[1], si[2]);
                                for (int c = 0; c < nc; ++c) Wd[c * pg.total + go] = Ws[c * pg.total + so];
                            }
                } else if (kind == NB_FINE) {
                    /* coarse ghost layer l covers fine layers 2l, 2l+1 away
                     * from the face; transverse coarse index t covers fine
                     * 2t, 2t+1 from the refined root's origin */
                    for (int a = 0; a < n[e1]; ++a)
                        for (int bb = 0; bb < n[e2]; ++bb)
                            for (int l = 0; l < NGH; ++l) {
                                int gi[3];
                                gi[d] = s ? n[d] + l : -1 - l;
                                gi[e1] = a;
                                gi[e2] = bb;
                                int64_t go = pidx(&pg, gi[0], gi[1], gi[2]);
                                for (int c = 0; c < nc; ++c) {
                                    double v[8];
                                    for (int o = 0; o < (1 << ndim); ++o) {
                                        int x[3];
                                        for (int e = 0; e < 3; ++e) {
                                            int off = e < ndim ? (o >> e) & 1 : 0;
                                            int fe;
                                            if (e == d) {
                                                /* fine cells 2l, 2l+1 in from the refined
                                                 * root's face (off 0: the lower one) */
                                                fe = s ? 2 * root[d] * n[d] + 2 * l + off
                                                       : 2 * (root[d] + 1) * n[d] - 2 - 2 * l + off;
                                            } else {
                                                fe = e < ndim ? 2 * root[e] * n[e] + 2 * gi[e] + off : 0;
                                            }
                                            x[e] = fe;
                                        }
                                        int loc[3];
                                        int fb = smr_fine_cell(g, g->leaf[b][0] + 1, x, loc);
                                        const double* Wf = Wp + (int64_t)fb * nc * pg.total;
                                        v[o] = Wf[c * pg.total + pidx(&pg, loc[0], loc[1], loc[2])];
                                    }
                                    Wd[c * pg.total + go] = tree_mean(v, ndim);
                                }
                            }
                }
            }
        }
        fill_ghosts_masked(mb, Wd, (const int(*)[2])cside);
    }
    /* (b) prolongation from the coarse side's complete padded array, level
     * by level (a coarse block's own prolonged ghosts come first) */
    for (int lev = 1; lev < g->nlev; ++lev)
    for (int b = 0; b < g->nleaf; ++b) {
        if (g->leaf[b][0] != lev) continue;
        double* Wd = Wp + (int64_t)b * nc * pg.total;
        const int fc[3] = {g->leaf[b][1], g->leaf[b][2], g->leaf[b][3]};
        for (int d = 0; d < ndim; ++d) {
            int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
            for (int s = 0; s < 2; ++s) {
                int idx = -1, root[3];
                if (smr_nbr(g, b, d, s, &idx, root) != NB_COARSE) continue;
                const double* Wc = Wp + (int64_t)idx * nc * pg.total;
                for (int a = 0; a < n[e1]; ++a)
                    for (int bb = 0; bb < n[e2]; ++bb)
                        for (int l = 0; l < NGH; ++l) {
                            int gi[3], ci[3];
                            double sg[3] = {0.0, 0.0, 0.0};
                            gi[d] = s ? n[d] + l : -1 - l;
                            gi[e1] = a;
                            gi[e2] = bb;
                            /* the coarse cell: next to the face along d */
                            ci[d] = s ? 0 : n[d] - 1;
                            sg[d] = s ? (l == 0 ? -1.0 : 1.0) : (l == 0 ? 1.0 : -1.0);
                            for (int e = 0; e < 3; ++e) {
                                if (e == d) continue;
                                if (e >= ndim) {
                                    ci[e] = 0;
                                    continue;
                                }
                                int p = (fc[e] % 2) * n[e] + gi[e]; /* fine index from the parent's origin */
                                ci[e] = p / 2;
                                sg[e] = (p % 2) ? 1.0 : -1.0;
                            }
                            int64_t go = pidx(&pg, gi[0], gi[1], gi[2]);
                            int64_t co = pidx(&pg, ci[0], ci[1], ci[2]);
                            for (int c = 0; c < nc; ++c) {
                                double wc = Wc[c * pg.total + co];
                                double acc = wc;
                                for (int e = 0; e < ndim; ++e) {
                                    int lo[3] = {ci[0], ci[1], ci[2]}, hi[3] = {ci[0], ci[1], ci[2]};
                                    lo[e] -= 1;
                                    hi[e] += 1;
                                    double wl = Wc[c * pg.total + pidx(&pg, lo[0], lo[1], lo[2])];
                                    double wh = Wc[c * pg.total + pidx(&pg, hi[0], hi[1], hi[2])];
                                    acc = acc + (0.25 * sg[e]) * orc_minmod(wc - wl, wh - wc);
                                }
                                Wd[c * pg.total + go] = acc;
                            }
                        }
            }
        }
    }
}

/* Stage right-hand side of every leaf from X (conserved, block layout), with
 * PLM face states (order 2) or piecewise-constant ones (order 1).  The
 * cross-level ghosts are the same for both orders. */
static int smr_rhs(const smrgeo* g, const double* X, double dt, int order, double* dU) {
    const orc_mesh* mb = &g->mb;
    int ndim = mb->ndim, nc = ndim + 2;
    int n0 = mb->n[0], n1 = mb->n[1], n2 = mb->n[2];
    int64_t nb = g->nb;
    padgeo pg = pad_geometry(mb);
    double* Wp = (double*)calloc((size_t)g->nleaf * nc * pg.total, sizeof(double));
    faceflux* ff = (faceflux*)calloc((size_t)g->nleaf, sizeof(faceflux));
    if (!Wp || !ff) {
        free(Wp);
        free(ff);
        return -1;
    }
    int bad = 0;
    for (int b = 0; b < g->nleaf; ++b) {
        const double* Xb = X + (int64_t)b * nc * nb;
        double* Wb = Wp + (int64_t)b * nc * pg.total;
        for (int k = 0; k < n2; ++k)
            for (int j = 0; j < n1; ++j)
                for (int i = 0; i < n0; ++i) {
                    int64_t cell = ((int64_t)k * n1 + j) * n0 + i;
                    double u[MAXC], w[MAXC];
                    for (int c = 0; c < nc; ++c) u[c] = Xb[c * nb + cell];
                    if (!cons_to_prim_cell(ndim, mb->gamma, u, w)) ++bad;
                    int64_t o = pidx(&pg, i, j, k);
                    for (int c = 0; c < nc; ++c) Wb[c * pg.total + o] = w[c];
                }
    }
    int rc = bad;
    if (rc == 0) smr_fill_ghosts(g, Wp);
    for (int b = 0; b < g->nleaf && rc == 0; ++b)
        rc = block_fluxes(mb, Wp + (int64_t)b * nc * pg.total, order, &ff[b]);
    /* (d) coarse faces shared with finer blocks take the fine fluxes' average */
    for (int b = 0; b < g->nleaf && rc == 0; ++b) {
        for (int d = 0; d < ndim; ++d) {
            int e1 = (d + 1) % 3, e2 = (d + 2) % 3;
            for (int s = 0; s < 2; ++s) {
                int idx = -1, root[3] = {0, 0, 0};
                if (smr_nbr(g, b, d, s, &idx, root) != NB_FINE) continue;
                const int64_t* fext = ff[b].fext[d];
                for (int a = 0; a < mb->n[e1]; ++a)
                    for (int bb = 0; bb < mb->n[e2]; ++bb) {
                        int fi[3];
                        fi[d] = s ? mb->n[d] : 0;
                        fi[e1] = a;
                        fi[e2] = bb;
                        int64_t fo = ((int64_t)fi[2] * fext[1] + fi[1]) * fext[0] + fi[0];
                        for (int c = 0; c < nc; ++c) {
                            double v[4];
                            int k = 0;
                            /* transverse offsets in axis order (x, y, z without d) */
                            int tax[2], nt = 0;
                            for (int e = 0; e < ndim; ++e)
                                if (e != d) tax[nt++] = e;
                            for (int o = 0; o < (1 << nt); ++o) {
                                int x[3];
                                x[d] = s ? 2 * root[d] * mb->n[d] : 2 * (root[d] + 1) * mb->n[d] - 1;
                                for (int e = 0; e < 3; ++e) {
                                    if (e == d) continue;
                                    x[e] = e < ndim ? 2 * root[e] * mb->n[e] + 2 * fi[e] : 0;
                                }
                                for (int t = 0; t < nt; ++t) x[tax[t]] += (o >> t) & 1;
                                int loc[3];
                                int fb = smr_fine_cell(g, g->leaf[b][0] + 1, x, loc);
                                /* the fine face on the shared plane: low face of a
                                 * fine cell for s = 1, its high face for s = 0 */
                                int ffi[3] = {loc[0], loc[1], loc[2]};
                                if (!s) ffi[d] += 1;
                                const int64_t* fx = ff[fb].fext[d];
                                int64_t ffo = ((int64_t)ffi[2] * fx[1] + ffi[1]) * fx[0] + ffi[0];
                                v[k++] = ff[fb].F[d][c * ff[fb].nf[d] + ffo];
                            }
                            ff[b].F[d][c * ff[b].nf[d] + fo] = tree_mean(v, nt);
                        }
                    }
            }
        }
    }
    for (int b = 0; b < g->nleaf && rc == 0; ++b)
        flux_update(mb, g->dx[g->leaf[b][0]], &ff[b], dt, dU + (int64_t)b * nc * nb);
    for (int b = 0; b < g->nleaf; ++b) faceflux_free(&ff[b]);
    free(ff);
    free(Wp);
    return rc;
}

static double smr_cfl_dt(const smrgeo* g, const double* U, double cfl) {
    int ndim = g->mb.ndim, nc = ndim + 2;
    double gm = g->mb.gamma, best = INFINITY;
    for (int b = 0; b < g->nleaf; ++b) {
        const double* dx = g->dx[g->leaf[b][0]];
        for (int64_t i = 0; i < g->nb; ++i) {
            double u[MAXC], w[MAXC];
            for (int c = 0; c < nc; ++c) u[c] = U[(int64_t)b * nc * g->nb + c * g->nb + i];
            if (!cons_to_prim_cell(ndim, gm, u, w)) return -1.0;
            double cs = sqrt(gm * w[nc - 1] / w[0]);
            for (int d = 0; d < ndim; ++d) {
                double cand = dx[d] / (fabs(w[1 + d]) + cs);
                if (cand < best) best = cand;
            }
        }
    }
    return cfl * best;
}

int orc_smr_leaves(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined,
                   int32_t* leaves, int max) {
    smrgeo g;
    if (!smr_geometry(m, blocks, nref, refined, &g)) {
        smr_free(&g);
        return -1;
    }
    for (int b = 0; b < g.nleaf && b < max; ++b)
        for (int q = 0; q < 4; ++q) leaves[4 * b + q] = g.leaf[b][q];
    int n = g.nleaf;
    smr_free(&g);
    return n;
}

int orc_smr_ghosts(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined,
                   const double* W, double* Wpad) {
    smrgeo g;
    if (!smr_geometry(m, blocks, nref, refined, &g)) {
        smr_free(&g);
        return -1;
    }
    int nc = m->ndim + 2;
    padgeo pg = pad_geometry(&g.mb);
    memset(Wpad, 0, (size_t)g.nleaf * nc * pg.total * sizeof(double));
    for (int b = 0; b < g.nleaf; ++b)
        for (int k = 0; k < g.mb.n[2]; ++k)
            for (int j = 0; j < g.mb.n[1]; ++j)
                for (int i = 0; i < g.mb.n[0]; ++i) {
                    int64_t cell = ((int64_t)k * g.mb.n[1] + j) * g.mb.n[0] + i;
                    for (int c = 0; c < nc; ++c)
                        Wpad[((int64_t)b * nc + c) * pg.total + pidx(&pg, i, j, k)] =
                            W[((int64_t)b * nc + c) * g.nb + cell];
                }
    smr_fill_ghosts(&g, Wpad);
    smr_free(&g);
    return 0;
}

int orc_run_smr(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined, double* U,
                double cfl, int max_steps, double t_end, double* t, int* steps_done, double* dts) {
    smrgeo g;
    if (!smr_geometry(m, blocks, nref, refined, &g) || !t || !(cfl > 0.0) ||
        (max_steps <= 0 && !(t_end > 0.0)) || (m->integrator != ORC_HEUN && m->integrator != ORC_VL2)) {
        smr_free(&g);
        return -1;
    }
    int64_t tot = (int64_t)g.nleaf * (m->ndim + 2) * g.nb;
    double* U1 = (double*)malloc((size_t)tot * sizeof(double));
    double* dU = (double*)malloc((size_t)tot * sizeof(double));
    int s = 0, rc = (U1 && dU) ? 0 : -1;
    while (rc == 0 && (max_steps <= 0 || s < max_steps)) {
        if (t_end > 0.0 && !(*t < t_end)) break;
        double dt = smr_cfl_dt(&g, U, cfl);
        if (!(dt > 0.0)) {
            rc = 1;
            break;
        }
        int last = 0;
        if (t_end > 0.0 && dt >= t_end - *t) {
            dt = t_end - *t;
            last = 1;
        }
        if (m->integrator == ORC_VL2) {
            /* van Leer (Sec. 3.3): the half-step predictor from
             * piecewise-constant states, U* = U^n + (dt/2) L_1(U^n), then
             * U^{n+1} = U^n + dt L_2(U*) from PLM states of W(U*); both
             * stages with the level-jump ghosts and flux corrections */
            rc = smr_rhs(&g, U, 0.5 * dt, 1, dU);
            if (rc) break;
            for (int64_t q = 0; q < tot; ++q) U1[q] = U[q] + dU[q];
            rc = smr_rhs(&g, U1, dt, 2, dU);
            if (rc) break;
            for (int64_t q = 0; q < tot; ++q) U[q] = U[q] + dU[q];
        } else {
            rc = smr_rhs(&g, U, dt, 2, dU);
            if (rc) break;
            for (int64_t q = 0; q < tot; ++q) U1[q] = U[q] + dU[q];
            rc = smr_rhs(&g, U1, dt, 2, dU);
            if (rc) break;
            for (int64_t q = 0; q < tot; ++q) U[q] = 0.5 * U[q] + 0.5 * (U1[q] + dU[q]);
        }
        if (dts) dts[s] = dt;
        *t = last ? t_end : *t + dt;
        ++s;
    }
    free(U1);
    free(dU);
    smr_free(&g);
    if (steps_done) *steps_done = s;
    return rc;
}

void orc_smr_totals(const orc_mesh* m, const int32_t blocks[3], int nref, const int32_t* refined,
                    const double* U, double* totals) {
    smrgeo g;
    if (!smr_geometry(m, blocks, nref, refined, &g)) {
        smr_free(&g);
        return;
    }
    int nc = m->ndim + 2;
    for (int c = 0; c < nc; ++c) {
        double sum = 0.0, comp = 0.0;
        for (int b = 0; b < g.nleaf; ++b) {
            double dV = 1.0;
            for (int d = 0; d < m->ndim; ++d) dV *= g.dx[g.leaf[b][0]][d];
            for (int64_t i = 0; i < g.nb; ++i) {
                double x = dV * U[((int64_t)b * nc + c) * g.nb + i];
                double tt = sum + x;
                if (fabs(sum) >= fabs(x))
                    comp += (sum - tt) + x;
                else
                    comp += (x - tt) + sum;
                sum = tt;
            }
        }
        totals[c] = sum + comp;
    }
    smr_free(&g);
}

void orc_totals(const orc_mesh* m, const double* U, double* totals) {
    if (!mesh_ok(m)) return;
    int nc = m->ndim + 2;
    int64_t N = ncells(m);
    double dV = 1.0;
    for (int d = 0; d < m->ndim; ++d) dV *= cell_width(m, d);
    for (int c = 0; c < nc; ++c) {
        double sum = 0.0, comp = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double x = U[c * N + i];
            double t = sum + x;
            if (fabs(sum) >= fabs(x))
                comp += (sum - t) + x;
            else
                comp += (x - t) + sum;
            sum = t;
        }
        totals[c] = dV * (sum + comp);
    }
}

/* --------------------------------------------------- sampled evaluation */

/* Field source for the sampled path: the full U^n array, or U^n plus one
 * stage-1 update evaluated on demand (the predictor U1 at any cell). */
typedef struct {
    const orc_mesh* m;
    const double* U;
    double dt;
    int predictor;
} field_src;

static int cell_rhs(const field_src* f, int64_t cell, double* dU);

static int field_get(const field_src* f, int64_t cell, double* u) {
    int nc = f->m->ndim + 2;
    int64_t N = ncells(f->m);
    for (int c = 0; c < nc; ++c) u[c] = f->U[c * N + cell];
    if (!f->predictor) return 0;
    field_src base = {f->m, f->U, f->dt, 0};
    double dU[MAXC];
    int rc = cell_rhs(&base, cell, dU);
    if (rc) return rc;
    for (int c = 0; c < nc; ++c) u[c] = u[c] + dU[c];
    return 0;
}

/* Stage rhs at one interior cell from its axis-aligned 5-cell crosses, with
 * the same face_flux and ghost rules as the full-mesh path. */
static int cell_rhs(const field_src* f, int64_t cell, double* dU) {
    const orc_mesh* m = f->m;
    int ndim = m->ndim, nc = ndim + 2;
    int n0 = m->n[0], n1 = m->n[1];
    int idx[3] = {(int)(cell % n0), (int)((cell / n0) % n1), (int)(cell / ((int64_t)n0 * n1))};
    double acc[MAXC];
    for (int c = 0; c < nc; ++c) acc[c] = 0.0;
    for (int d = 0; d < ndim; ++d) {
        double w5[5][MAXC];
        for (int s = 0; s < 5; ++s) {
            int q = idx[d] - 2 + s;
            int vmode = VM_NONE;
            if (q < 0 || q >= m->n[d]) q = ghost_src(m, d, q, &vmode);
            int c3[3] = {idx[0], idx[1], idx[2]};
            c3[d] = q;
            int64_t src = ((int64_t)c3[2] * n1 + c3[1]) * n0 + c3[0];
            double u[MAXC];
            int rc = field_get(f, src, u);
            if (rc) return rc;
            if (!cons_to_prim_cell(ndim, m->gamma, u, w5[s])) return 1;
            w5[s][1 + d] = apply_vmode(w5[s][1 + d], vmode);
        }
        double Fm[MAXC], Fp[MAXC];
        face_flux(ndim, m->gamma, d, 2, (const double(*)[MAXC])&w5[0], Fm);
        face_flux(ndim, m->gamma, d, 2, (const double(*)[MAXC])&w5[1], Fp);
        double lam = f->dt / cell_width(m, d);
        for (int c = 0; c < nc; ++c) acc[c] = acc[c] + lam * (Fm[c] - Fp[c]);
    }
    for (int c = 0; c < nc; ++c) dU[c] = acc[c];
    return 0;
}

static int check_cells(const orc_mesh* m, int ns, const int64_t* cells) {
    int64_t N = ncells(m);
    for (int s = 0; s < ns; ++s)
        if (cells[s] < 0 || cells[s] >= N) return 0;
    return 1;
}

int orc_rhs_cells(const orc_mesh* m, const double* U, double dt, int ns, const int64_t* cells,
                  double* out) {
    if (!mesh_ok(m) || ns < 0 || !check_cells(m, ns, cells)) return -1;
    int nc = m->ndim + 2;
    field_src f = {m, U, dt, 0};
    for (int s = 0; s < ns; ++s) {
        double dU[MAXC];
        int rc = cell_rhs(&f, cells[s], dU);
        if (rc) return rc;
        for (int c = 0; c < nc; ++c) out[c * ns + s] = dU[c];
    }
    return 0;
}

int orc_step_cells(const orc_mesh* m, const double* U, double dt, int ns, const int64_t* cells,
                   double* out) {
    if (!mesh_ok(m) || ns < 0 || !check_cells(m, ns, cells)) return -1;
    int nc = m->ndim + 2;
    int64_t N = ncells(m);
    field_src base = {m, U, dt, 0};
    field_src pred = {m, U, dt, 1};
    for (int s = 0; s < ns; ++s) {
        double dU1[MAXC], dU2[MAXC];
        int rc = cell_rhs(&base, cells[s], dU1);
        if (!rc) rc = cell_rhs(&pred, cells[s], dU2);
        if (rc) return rc;
        for (int c = 0; c < nc; ++c) {
            double un = U[c * N + cells[s]];
            double u1 = un + dU1[c];
            out[c * ns + s] = 0.5 * un + 0.5 * (u1 + dU2[c]);
        }
    }
    return 0;
}
