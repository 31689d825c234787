// Device kernels of the Godunov hydro step for gfx950 (CDNA4, wave64).
//
// Method (Wang, arXiv 2501.02317, Sec. 3): conserved -> primitive in FP64
// (Sec. 3.1), ghost cells from the boundary rules of Sec. 3.1.1 resolved at
// load time, PLM with minmod on primitive variables (eq. minmod), HLLC with
// the subtraction-safe wave speeds (eqs. hllc-contact-spd, hllc-mixed-dvel),
// flux-divergence update and Heun combine in FP64 (Sec. 3.3), CFL dt
// reduction (Sec. 3.1).
//
// Layout: SoA FP64 U[c][k][j][i], interior only.  The stage kernel is a
// 2.5-D sweep: a work-group owns a TX x TY tile of the (kernel) x-y plane and
// marches along the kernel z axis over a chunk of kz planes.  The z stencil
// (five planes of primitive variables) lives in registers, the in-plane
// stencil in an LDS plane with a two-cell halo.  Every face flux is computed
// once per work-group and is one value shared by both neighbouring cells.
//
// Floating point: the compiler contracts nothing on its own (contraction is
// off), but the code fuses by hand where it pays -- explicit fused
// multiply-adds, FP64 reciprocals and reciprocal square roots from the
// hardware estimates refined by Newton steps (two, about 1 ulp, in the
// conversions and the time step; one, about 2^-45 relative, in the HLLC
// solve), and algebraically equal rearrangements of the written formulas.
// The FP64 path therefore agrees with a plain serial evaluation of the same
// formulas to rounding, not bitwise.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cfloat>
#include <cmath>

#include "hydro_internal.h"

#pragma clang fp contract(off)

namespace hydro {
namespace {

enum { BC_PERIODIC = 0, BC_FREE = 1, BC_OUTFLOW = 2, BC_REFLECT = 3 };
enum { VM_NONE = 0, VM_NEG = 1, VM_CLIP_LO = 2, VM_CLIP_HI = 3 };


__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float dabs(float x) { return __builtin_fabsf(x); }

// Velocity component (index into W/U) along kernel axis ax.
template <int NDIM>
__device__ __forceinline__ constexpr int vcomp(int ax) {
    return ax == 0 ? 1 : (ax == 1 ? 2 : NDIM);
}

// Arithmetic policy.  FP32 (the mixed path's reconstruction and Riemann
// solve): the hardware reciprocal and reciprocal square root (1 ulp), which
// the FP32 tolerance of that path absorbs.  FP64: the hardware estimates
// (relative error up to about 2^-23) refined by Newton steps instead of the
// longer correctly rounded division and square-root sequences -- two steps
// (about 1 ulp) for the conversions and the time step, one step (relative
// error about 2^-45) for the six per HLLC face (rcp1, rsq1), well inside the
// 1e-12 agreement the FP64 path keeps with a plain evaluation.
template <typename R>
struct Ops;

template <>
struct Ops<double> {
    static __device__ __forceinline__ double fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
    static __device__ __forceinline__ double rcp(double x) {
        double r = __builtin_amdgcn_rcp(x);
        double e = __builtin_fma(-x, r, 1.0);
        r = __builtin_fma(r, e, r);
        e = __builtin_fma(-x, r, 1.0);
        return __builtin_fma(r, e, r);
    }
    static __device__ __forceinline__ double rsq(double x) {
        double y = __builtin_amdgcn_rsq(x);
        double e = __builtin_fma(-x * y, y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
        e = __builtin_fma(-x * y, y, 1.0);
        return __builtin_fma(0.5 * y, e, y);
    }
    static __device__ __forceinline__ double rcp1(double x) {
        const double r = __builtin_amdgcn_rcp(x);
        return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    }
    static __device__ __forceinline__ double rsq1(double x) {
        const double y = __builtin_amdgcn_rsq(x);
        return __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
    }
    static __device__ __forceinline__ double max0(double x) { return __builtin_fmax(x, 0.0); }
    // median of (a, b, 0): the minmod of eq. minmod
    static __device__ __forceinline__ double minmod(double a, double b) {
        return __builtin_fmax(__builtin_fmin(a, b), __builtin_fmin(__builtin_fmax(a, b), 0.0));
    }
    // The slopes of the two cells beside a face, minmod(a, m) and
    // minmod(m, b), with m the difference across the face: the median of
    // (x, m, 0) is x clamped to [min(m, 0), max(m, 0)], and the two bounds
    // serve both slopes (FP64 min and max issue at half rate).
    static __device__ __forceinline__ void minmod2(double a, double m, double b, double& sa, double& sb) {
        const double lo = __builtin_fmin(m, 0.0), hi = __builtin_fmax(m, 0.0);
        sa = __builtin_fmin(__builtin_fmax(a, lo), hi);
        sb = __builtin_fmin(__builtin_fmax(b, lo), hi);
    }
};

template <>
struct Ops<float> {
    static __device__ __forceinline__ float fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp1(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float rsq1(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float max0(float x) { return __builtin_fmaxf(x, 0.0f); }
    static __device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
    static __device__ __forceinline__ void minmod2(float a, float m, float b, float& sa, float& sb) {
        sa = __builtin_amdgcn_fmed3f(a, m, 0.0f);
        sb = __builtin_amdgcn_fmed3f(m, b, 0.0f);
    }
};

// Gas constants in the compute precision.
template <typename R>
struct Gas {
    R g;          // gamma
    R z;          // (gamma + 1) / (2 gamma)
    R inv_gm1;    // 1 / (gamma - 1)
    R inv_g_gm1;  // 1 / (gamma (gamma - 1))
};

template <typename R>
__device__ __forceinline__ Gas<R> make_gas(double g) {
    Gas<R> o;
    o.g = (R)g;
    o.z = (R)((g + 1.0) / (2.0 * g));
    o.inv_gm1 = (R)(1.0 / (g - 1.0));
    o.inv_g_gm1 = (R)(1.0 / (g * (g - 1.0)));
    return o;
}

// ----------------------------------------------------------------- physics

// eq. minmod: the slope of smaller magnitude when both have the same strict
// sign, else zero -- which is the median of (a, b, 0).
template <typename R>
__device__ __forceinline__ R minmod(R a, R b) {
    return Ops<R>::minmod(a, b);
}

// Conserved -> primitive in FP64 (Sec. 3.1): r = 1/rho, v_d = m_d r,
// p = (gamma - 1)(E - (1/2) r sum_d m_d^2); returns admissibility.  The
// squares are rounded separately and summed in axis order, so interchanging
// x and y leaves the result bitwise unchanged.  LOWP: the values are rounded
// to FP32 afterwards, so 1/rho takes one Newton step instead of two.
// Admissibility is rho and p positive and finite: a non-finite momentum or
// energy makes p NaN or infinite, so it needs no test of its own.
template <int NDIM, bool LOWP = false>
__device__ __forceinline__ bool cons_to_prim(double gm1, const double (&u)[NDIM + 2],
                                             double (&w)[NDIM + 2]) {
    const double rho = u[0];
    const double r = LOWP ? Ops<double>::rcp1(rho) : Ops<double>::rcp(rho);
    double msq = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        w[1 + d] = u[1 + d] * r;
        msq = msq + u[1 + d] * u[1 + d];
    }
    const double p = gm1 * __builtin_fma(-0.5 * r, msq, u[NDIM + 1]);
    w[0] = rho;
    w[NDIM + 1] = p;
    return rho > 0.0 && rho < __builtin_inf() && p > 0.0 && p < __builtin_inf();
}

// HLLC flux in the face-normal frame, W = (rho, u, t_1..t_NT, p).
//   c_K = sqrt(g p_K / rho_K), evaluated as (g p_K) / sqrt(g p_K rho_K);
//   p* = max(0, primitive-variable guess);
//   ds_L = -c_L q_L, ds_R = c_R q_R with q_K = sqrt(1 + z (max(p*/p_K, 1) - 1))
//   (eq. hllc-mixed-dvel), evaluated as c_K q_K = a_K / sqrt(a_K rho_K) with
//   a_K = g (p_K + z max(p* - p_K, 0)), so ds_K = c_K exactly when p* <= p_K;
//   s_* from the bracketed form of eq. hllc-contact-spd.  Only the selected
//   side's star state and flux are evaluated; E_K/rho_K = c_K^2/(g (g-1)) +
//   |v_K|^2 / 2 and one reciprocal of (s_K - s_*) rho_K ds_K serve the star
//   state, so a face costs six reciprocal(-square-root) evaluations; the
//   tangential fluxes are the mass flux times the upwind side's tangential
//   velocities (the star state carries them unchanged).
template <typename R, int NT>
__device__ __forceinline__ void hllc(const Gas<R>& gas, const R (&WL)[NT + 3], const R (&WR)[NT + 3],
                                     R (&F)[NT + 3]) {
    using O = Ops<R>;
    constexpr int NC = NT + 3;
    const R g = gas.g;
    const R rl = WL[0], ul = WL[1], pl = WL[NC - 1];
    const R rr = WR[0], ur = WR[1], pr = WR[NC - 1];
    const R gpl = g * pl, gpr = g * pr;
    const R cl = gpl * O::rsq1(gpl * rl);
    const R cr = gpr * O::rsq1(gpr * rr);
    const R ppv = R(0.5) * (pl + pr) - R(0.125) * (ur - ul) * (rl + rr) * (cl + cr);
    const R ps = O::max0(ppv);
    const R al = g * O::fma(gas.z, O::max0(ps - pl), pl);
    const R ar = g * O::fma(gas.z, O::max0(ps - pr), pr);
    const R dsl = -(al * O::rsq1(al * rl));
    const R dsr = ar * O::rsq1(ar * rr);
    const R sl = ul + dsl;
    const R sr = ur + dsr;
    const R ml = rl * dsl, mr = rr * dsr;  // rho_K ds_K
    const R ss = (O::fma(-mr, ur, pr) - O::fma(-ml, ul, pl)) * O::rcp1(ml - mr);

    // s_L >= 0: F_L ; s_* >= 0: F*_L ; s_R > 0: F*_R ; else F_R
    const bool left = (sl >= R(0)) || (ss >= R(0));
    const bool star = left ? !(sl >= R(0)) : (sr > R(0));
    const R sK = left ? sl : sr;
    const R mK = left ? ml : mr;
    const R cK = left ? cl : cr;
    R W[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) W[c] = left ? WL[c] : WR[c];

    const R rho = W[0], u = W[1], p = W[NC - 1];
    const R mu = rho * u;
    // tangential |t|^2 as a sum of rounded squares: symmetric in the
    // tangential components, so interchanging two axes is bitwise
    R tsq = R(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) tsq = tsq + W[2 + k] * W[2 + k];
    const R vsq = O::fma(u, u, tsq);
    const R E = O::fma(p, gas.inv_gm1, R(0.5) * rho * vsq);

    // star state chi (1, s_*, t, E/rho + (s_* - u)(s_* + p/(rho ds))),
    // chi = rho ds / (s - s_*), with 1/(s - s_*) and 1/(rho ds) from one
    // reciprocal; F*_K = F_K + s_K (U*_K - U_K) for mass, normal momentum and
    // energy (the upwind flux where no star state applies: there the star
    // quantities may not be finite, so the choice is a select)
    const R t1 = sK - ss;
    const R q = O::rcp1(t1 * mK);
    const R chi = mK * (mK * q);
    const R p_m = p * (t1 * q);
    const R e_rho = O::fma(cK * cK, gas.inv_g_gm1, R(0.5) * vsq);
    const R f0 = O::fma(sK, chi - rho, mu);
    const R f1 = O::fma(sK, chi * ss - mu, O::fma(mu, u, p));
    const R f4 = O::fma(sK, chi * O::fma(ss - u, ss + p_m, e_rho) - E, (E + p) * u);
    F[0] = star ? f0 : mu;
    F[1] = star ? f1 : O::fma(mu, u, p);
    F[NC - 1] = star ? f4 : (E + p) * u;
    // the tangential velocities are carried by the mass flux: in the star
    // regions U*_t = chi t and U_t = rho t give F_t = t (rho u + s_K (chi -
    // rho)) = t F_0, and outside them F_t = rho u t = t F_0 as well
#pragma unroll
    for (int k = 0; k < NT; ++k) F[2 + k] = W[2 + k] * F[0];
}

// Flux through the face between cells w1 and w2 along kernel axis AX from the
// global-frame primitive states of the four cells around it: PLM per
// component, rotate the face normal to the first velocity slot, HLLC, rotate
// back.  Tangential velocities keep increasing component order.
// FIRST: piecewise-constant states (the face states are w1 and w2).
template <int NDIM, int AX, typename R, bool FIRST = false>
__device__ __forceinline__ void face_flux(const Gas<R>& g, const R (&w0)[NDIM + 2], const R (&w1)[NDIM + 2],
                                          const R (&w2)[NDIM + 2], const R (&w3)[NDIM + 2],
                                          R (&F)[NDIM + 2]) {
    constexpr int NC = NDIM + 2;
    constexpr int NT = NDIM - 1;
    constexpr int VN = vcomp<NDIM>(AX);
    R wl[NC], wr[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        if constexpr (FIRST) {
            wl[c] = w1[c];
            wr[c] = w2[c];
        } else {
            R dj, dj1;
            Ops<R>::minmod2(w1[c] - w0[c], w2[c] - w1[c], w3[c] - w2[c], dj, dj1);
            wl[c] = Ops<R>::fma(R(0.5), dj, w1[c]);
            wr[c] = Ops<R>::fma(R(-0.5), dj1, w2[c]);
        }
    }
    R L[NT + 3], Rs[NT + 3], Fn[NT + 3];
    L[0] = wl[0];
    Rs[0] = wr[0];
    L[1] = wl[VN];
    Rs[1] = wr[VN];
    {
        int k = 2;
#pragma unroll
        for (int e = 1; e <= NDIM; ++e) {
            if (e == VN) continue;
            L[k] = wl[e];
            Rs[k] = wr[e];
            ++k;
        }
    }
    L[NT + 2] = wl[NC - 1];
    Rs[NT + 2] = wr[NC - 1];
    hllc<R, NT>(g, L, Rs, Fn);
    F[0] = Fn[0];
    F[VN] = Fn[1];
    {
        int k = 2;
#pragma unroll
        for (int e = 1; e <= NDIM; ++e) {
            if (e == VN) continue;
            F[e] = Fn[k++];
        }
    }
    F[NC - 1] = Fn[NT + 2];
}

// Flux through an in-plane face of a 3-D tile whose axis (0: x, 1: y) is a
// run-time value: the same arithmetic as face_flux<3, 0 or 1>, with the
// rotation done by selects so faces of both axes share one code path.
template <typename R, bool FIRST = false>
__device__ __forceinline__ void face_flux_xy(const Gas<R>& g, bool yaxis, const R (&w0)[5], const R (&w1)[5],
                                             const R (&w2)[5], const R (&w3)[5], R (&F)[5]) {
    R wl[5], wr[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        if constexpr (FIRST) {
            wl[c] = w1[c];
            wr[c] = w2[c];
        } else {
            R dj, dj1;
            Ops<R>::minmod2(w1[c] - w0[c], w2[c] - w1[c], w3[c] - w2[c], dj, dj1);
            wl[c] = Ops<R>::fma(R(0.5), dj, w1[c]);
            wr[c] = Ops<R>::fma(R(-0.5), dj1, w2[c]);
        }
    }
    // normal velocity first, then the other in-plane one, then z
    R L[5] = {wl[0], yaxis ? wl[2] : wl[1], yaxis ? wl[1] : wl[2], wl[3], wl[4]};
    R Rr[5] = {wr[0], yaxis ? wr[2] : wr[1], yaxis ? wr[1] : wr[2], wr[3], wr[4]};
    R Fn[5];
    hllc<R, 2>(g, L, Rr, Fn);
    F[0] = Fn[0];
    F[1] = yaxis ? Fn[2] : Fn[1];
    F[2] = yaxis ? Fn[1] : Fn[2];
    F[3] = Fn[3];
    F[4] = Fn[4];
}

// Flux from already reconstructed face states (global frame) along kernel
// axis AX: the rotation and HLLC of face_flux without the PLM step.
template <int NDIM, int AX, typename R>
__device__ __forceinline__ void face_flux_states(const Gas<R>& g, const R (&wl)[NDIM + 2],
                                                 const R (&wr)[NDIM + 2], R (&F)[NDIM + 2]) {
    constexpr int NC = NDIM + 2;
    constexpr int NT = NDIM - 1;
    constexpr int VN = vcomp<NDIM>(AX);
    R L[NT + 3], Rs[NT + 3], Fn[NT + 3];
    L[0] = wl[0];
    Rs[0] = wr[0];
    L[1] = wl[VN];
    Rs[1] = wr[VN];
    {
        int k = 2;
#pragma unroll
        for (int e = 1; e <= NDIM; ++e) {
            if (e == VN) continue;
            L[k] = wl[e];
            Rs[k] = wr[e];
            ++k;
        }
    }
    L[NT + 2] = wl[NC - 1];
    Rs[NT + 2] = wr[NC - 1];
    hllc<R, NT>(g, L, Rs, Fn);
    F[0] = Fn[0];
    F[VN] = Fn[1];
    {
        int k = 2;
#pragma unroll
        for (int e = 1; e <= NDIM; ++e) {
            if (e == VN) continue;
            F[e] = Fn[k++];
        }
    }
    F[NC - 1] = Fn[NT + 2];
}

// ---------------------------------------------------------------- boundaries

// Interior index for coordinate q on kernel axis ax of the whole mesh
// (extent n * blocks) and the treatment of the normal velocity (Sec. 3.1.1;
// each side read as the left-x case).
__device__ __forceinline__ int resolve_mesh(const Geo& g, int ax, int q, int& vmode) {
    const int N = g.n[ax] * g.blocks[ax];
    vmode = VM_NONE;
    if (q >= 0 && q < N) return q;
    if (q < 0) {
        switch (g.bc[ax][0]) {
            case BC_PERIODIC: return q + N;
            case BC_FREE: return 0;
            case BC_OUTFLOW: vmode = VM_CLIP_LO; return 0;
            default: vmode = VM_NEG; return -1 - q;
        }
    }
    switch (g.bc[ax][1]) {
        case BC_PERIODIC: return q - N;
        case BC_FREE: return N - 1;
        case BC_OUTFLOW: vmode = VM_CLIP_HI; return N - 1;
        default: vmode = VM_NEG; return 2 * N - 1 - q;
    }
}

// The sides of one block: the block-index offset of the neighbour a side
// reads its ghosts from (a c-boundary: inside the mesh, or across a periodic
// axis), or kNoLink at a face of the mesh with a p-boundary rule.
// On a refined mesh a side may instead read a ghost slot (slo/shi: the slot
// index, else -1).
constexpr int kNoLink = 0x7fffffff;
struct Links {
    int lo[3], hi[3];
    int slo[3], shi[3];
};

__device__ __forceinline__ Links block_links(const Geo& g, int blk) {
    Links L;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) L.slo[ax] = L.shi[ax] = -1;
    const int c[3] = {blk % g.blocks[0], (blk / g.blocks[0]) % g.blocks[1], blk / (g.blocks[0] * g.blocks[1])};
    const int stride[3] = {1, g.blocks[0], g.blocks[0] * g.blocks[1]};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int B = g.blocks[ax];
        const int wrap = (B - 1) * stride[ax];
        L.lo[ax] = c[ax] > 0 ? -stride[ax] : (g.bc[ax][0] == BC_PERIODIC ? wrap : kNoLink);
        L.hi[ax] = c[ax] < B - 1 ? stride[ax] : (g.bc[ax][1] == BC_PERIODIC ? -wrap : kNoLink);
    }
    return L;
}

// The sides of a block of a refined mesh, from its side codes.
__device__ __forceinline__ Links table_links(const int* __restrict__ side, int blk) {
    Links L;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int lo = side[6 * blk + 2 * ax], hi = side[6 * blk + 2 * ax + 1];
        L.lo[ax] = lo >= 0 ? lo - blk : kNoLink;
        L.hi[ax] = hi >= 0 ? hi - blk : kNoLink;
        L.slo[ax] = lo <= kSideSlot0 ? kSideSlot0 - lo : -1;
        L.shi[ax] = hi <= kSideSlot0 ? kSideSlot0 - hi : -1;
    }
    return L;
}

// The sides of a launch's block: from the side codes of a refined mesh, else
// from the uniform block grid (selected field by field, so the structure
// stays in registers).
__device__ __forceinline__ Links stage_links(const StageArgs& a, int blk) {
    const Geo& g = a.geo;
    const bool tab = a.side != nullptr;
    const Links G = block_links(g, blk);
    Links L;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int lo = tab ? a.side[6 * blk + 2 * ax] : 0, hi = tab ? a.side[6 * blk + 2 * ax + 1] : 0;
        L.lo[ax] = tab ? (lo >= 0 ? lo - blk : kNoLink) : G.lo[ax];
        L.hi[ax] = tab ? (hi >= 0 ? hi - blk : kNoLink) : G.hi[ax];
        L.slo[ax] = tab && lo <= kSideSlot0 ? kSideSlot0 - lo : -1;
        L.shi[ax] = tab && hi <= kSideSlot0 ? kSideSlot0 - hi : -1;
    }
    return L;
}

// Ghost coordinate q (one block's extent N on kernel axis ax) -> the cell it
// copies: in the linked block dblk (offset in blocks, 0 for the block
// itself) at q -/+ N, or by the p-boundary rule of a mesh face, with the
// treatment of the normal velocity (Sec. 3.1.1); or, at a level jump, the
// ghost slot `slot` (else -1) and the layer returned (0 next to the face).
__device__ __forceinline__ int resolve(const Geo& g, const Links& L, int ax, int q, int& vmode, int& dblk,
                                       int& slot) {
    const int N = g.n[ax];
    vmode = VM_NONE;
    dblk = 0;
    slot = -1;
    if (q >= 0 && q < N) return q;
    if (q < 0) {
        if (L.slo[ax] >= 0) {
            slot = L.slo[ax];
            return -1 - q;
        }
        if (L.lo[ax] != kNoLink) {
            dblk = L.lo[ax];
            return q + N;
        }
        switch (g.bc[ax][0]) {
            case BC_FREE: return 0;
            case BC_OUTFLOW: vmode = VM_CLIP_LO; return 0;
            default: vmode = VM_NEG; return -1 - q;
        }
    }
    if (L.shi[ax] >= 0) {
        slot = L.shi[ax];
        return q - N;
    }
    if (L.hi[ax] != kNoLink) {
        dblk = L.hi[ax];
        return q - N;
    }
    switch (g.bc[ax][1]) {
        case BC_FREE: return N - 1;
        case BC_OUTFLOW: vmode = VM_CLIP_HI; return N - 1;
        default: vmode = VM_NEG; return 2 * N - 1 - q;
    }
}

__device__ __forceinline__ double apply_vmode(double v, int vmode) {
    switch (vmode) {
        case VM_NEG: return -v;
        case VM_CLIP_LO: return v > 0.0 ? 0.0 : v;
        case VM_CLIP_HI: return v < 0.0 ? 0.0 : v;
        default: return v;
    }
}

// Primitive state at kernel coordinates (x, y, z) of the whole mesh, at most
// one of which lies outside it (the axis-aligned stencil never needs corner
// ghosts); U in the block layout.
template <int NDIM, typename R>
__device__ __forceinline__ void load_w(const Geo& g, const double* __restrict__ U, int x, int y, int z,
                                       R (&W)[NDIM + 2], bool& bad) {
    constexpr int NC = NDIM + 2;
    int vm = VM_NONE, ax = -1;
    if (x < 0 || x >= g.n[0] * g.blocks[0]) {
        x = resolve_mesh(g, 0, x, vm);
        ax = 0;
    } else if (y < 0 || y >= g.n[1] * g.blocks[1]) {
        y = resolve_mesh(g, 1, y, vm);
        ax = 1;
    } else if (z < 0 || z >= g.n[2] * g.blocks[2]) {
        z = resolve_mesh(g, 2, z, vm);
        ax = 2;
    }
    const int blk = x / g.n[0] + g.blocks[0] * (y / g.n[1] + g.blocks[1] * (z / g.n[2]));
    const long long cell = ((long long)(z % g.n[2]) * g.n[1] + y % g.n[1]) * g.n[0] + x % g.n[0];
    const double* Ub = U + (long long)blk * NC * g.ncells;
    double u[NC], w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] = Ub[c * g.ncells + cell];
    bad |= !cons_to_prim<NDIM>(g.gamma - 1.0, u, w);
    if (ax >= 0) {
        const int vc = ax == 0 ? 1 : (ax == 1 ? 2 : NDIM);
#pragma unroll
        for (int c = 1; c <= NDIM; ++c)
            if (c == vc) w[c] = apply_vmode(w[c], vm);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) W[c] = (R)w[c];
}

// CFL rate of one cell, max over active kernel axes of (|v| + c)/dx; the
// time step is cfl / (max over cells of the rate), the same quantity as
// cfl * min over cells and axes of dx / (|v| + c) (Sec. 3.1).
template <int NDIM>
__device__ __forceinline__ double cfl_rate(const Geo& g, const double (&w)[NDIM + 2]) {
    const double gp = g.gamma * w[NDIM + 1];
    const double cs = gp * Ops<double>::rsq(gp * w[0]);  // sqrt(gamma p / rho)
    double best = (dabs(w[1]) + cs) * g.inv_dx[0];
    if (NDIM == 3) {
        const double c1 = (dabs(w[2]) + cs) * g.inv_dx[1];
        best = c1 > best ? c1 : best;
    }
    if (NDIM >= 2) {
        const double c2 = (dabs(w[NDIM]) + cs) * g.inv_dx[2];
        best = c2 > best ? c2 : best;
    }
    return best;
}

// dt of the next step from the control block: the CFL step, shortened to
// land on t_end when one is set.
__device__ __forceinline__ double device_dt(const Ctrl* c) {
    double dt = c->dt_raw;
    if (c->t_end > 0.0) {
        const double rem = c->t_end - c->t;
        if (dt >= rem) dt = rem;
    }
    return dt > 0.0 ? dt : 0.0;
}

__device__ __forceinline__ void update_done(Ctrl* c) {
    c->done = (c->t_end > 0.0 && !(c->t < c->t_end)) || (c->max_steps > 0 && c->steps >= c->max_steps);
}

// Advance time by the step just taken and take the next dt from the rate.
__device__ __forceinline__ void finalize_step(Ctrl* c, double cfl) {
    if (c->done) return;
    const double dt = device_dt(c);
    const bool last = c->t_end > 0.0 && c->dt_raw >= c->t_end - c->t;
    if (dt > 0.0) {
        c->t = last ? c->t_end : c->t + dt;
        c->steps += 1;
    }
    c->dt_raw = cfl / __longlong_as_double((long long)c->rate_bits);
    c->dt_valid = 1;
    c->rate_bits = 0ull;
    update_done(c);
}

// Work-groups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous range of tiles so neighbouring tiles share one L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int x = bid % X, i = bid / X;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// ------------------------------------------------------------- stage kernel

// Raw conserved values of one cell; cell = plane offset + column offset.
template <int NC>
__device__ __forceinline__ void load_u(const double* __restrict__ U, long long N, long long cell,
                                       double (&u)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] = U[c * N + cell];
}

// Primitive state of raw values u; the velocity along kernel axis vax (if
// any) takes the boundary treatment vm of the ghost it fills.
template <int NDIM, typename R, bool CHECK = true>
__device__ __forceinline__ void to_prim(double gm1, const double (&u)[NDIM + 2], int vax, int vm,
                                        R (&W)[NDIM + 2], bool& bad) {
    constexpr int NC = NDIM + 2;
    double w[NC];
    const bool ok = cons_to_prim<NDIM, sizeof(R) == 4>(gm1, u, w);
    if (CHECK) bad |= !ok;
    if (vax >= 0) {
        const int vc = vax == 0 ? 1 : (vax == 1 ? 2 : NDIM);
#pragma unroll
        for (int c = 1; c <= NDIM; ++c)
            if (c == vc) w[c] = apply_vmode(w[c], vm);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) W[c] = (R)w[c];
}

// The stencil input of a cell as primitive variables in R: conserved FP64
// values converted (to_prim), or, with PRIM, stored primitive values of type
// R (the van Leer predictor state) held as doubles, with the boundary
// treatment of the normal velocity applied.
template <int NDIM, typename R, bool PRIM, bool CHECK = true>
__device__ __forceinline__ void in_to_w(double gm1, const double (&u)[NDIM + 2], int vax, int vm,
                                        R (&W)[NDIM + 2], bool& bad) {
    constexpr int NC = NDIM + 2;
    if constexpr (PRIM) {
        const int vc = vax == 0 ? 1 : (vax == 1 ? 2 : NDIM);
#pragma unroll
        for (int c = 0; c < NC; ++c) W[c] = (R)((vax >= 0 && c == vc) ? apply_vmode(u[c], vm) : u[c]);
    } else {
        to_prim<NDIM, R, CHECK>(gm1, u, vax, vm, W, bad);
    }
}

// Access to one plane of a [comp][cell] field through a buffer resource:
// the plane base (component base + plane offset, the same for the whole
// work-group) lives in scalar registers and the thread supplies a 32-bit
// byte offset, so no per-thread 64-bit address arithmetic is needed.  The
// resource covers exactly the plane (extent bytes): an offset outside it
// reads 0 and writes nothing.
constexpr int kBufferWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9)
typedef unsigned int u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T* F, long long uniform_off,
                                                             uint32_t extent_bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(F + uniform_off), (short)0, (int)extent_bytes,
                                             kBufferWord3);
}

// Cache policy of the accesses that touch a value for the last time in a
// step (the final update's read of U^n and its write of U^{n+1}): the
// non-temporal hint (slc), so that streaming data does not displace the
// stencil's planes in L2.  Measured 1.5-2.5 % faster for those stages; the
// first stages keep the default policy (their output is read right after,
// and the hint measured neutral to 1.5 % slower there).
constexpr int kNonTemporal = 2;

template <typename T, int CPOL = 0>
__device__ __forceinline__ T plane_load(const T* F, long long uniform_off, uint32_t extent_bytes,
                                        uint32_t thread_bytes) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(F, uniform_off, extent_bytes);
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, thread_bytes, 0, CPOL));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, thread_bytes, 0, CPOL));
}

template <typename T, int CPOL = 0>
__device__ __forceinline__ void plane_store(T* F, long long uniform_off, uint32_t extent_bytes,
                                            uint32_t thread_bytes, T v) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(F, uniform_off, extent_bytes);
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, thread_bytes, 0, CPOL);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, thread_bytes, 0, CPOL);
}

// NC values of one cell from a field of type T (layout [comp][cell]) as doubles.
template <int NC, typename T>
__device__ __forceinline__ void load_as_double(const T* __restrict__ F, long long N, long long cell,
                                               double (&u)[NC]) {
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] = (double)F[c * N + cell];
}

// One stage over a TX x TY tile column and a chunk of kz planes.
//
// Software pipeline per plane k (kernel z): raw U of the interior plane k+3
// and of the halo cells of plane k+1 are loaded one iteration before they are
// converted, and U at plane k for the update is loaded at the top of the
// iteration and used after the flux phase, so global loads stay in flight
// across the two LDS barriers.  Each thread owns at most one halo cell of
// the plane (4 TX + 4 TY <= TX TY).
// Work-groups per CU the compiler is asked to fit: the FP32 path keeps four
// 256-thread groups per CU (16 waves); FP64 needs more registers per thread.
// The input ring and the one-barrier schedule pay in 3-D only: the 2-D
// kernels (one row of 64..256 cells) already run many small work-groups per
// CU, and measured slower with either.
constexpr bool kRing2D = false;
constexpr bool kOne2D = false;

template <int NDIM, typename R, int MODE>
struct StageOccupancy {
    // Input ring: the raw input values of a cell, read for its conversion
    // when its plane enters the z stencil, are kept in a three-plane LDS ring
    // until the update of that plane instead of being read again.  It pays
    // in the mixed stages (measured at 256^3 at the sustained clock: stage 1
    // 392 -> 371 us with 32 x 8 tiles in place of 32 x 16 and one barrier
    // per plane): there the ring's LDS sets the occupancy to three
    // work-groups per CU, which their register use allows without spills.
    // The FP64 stage 1 loses a wave per SIMD to it and does without.
    static constexpr bool kRing =
        sizeof(R) == 4 && (MODE == MODE_STAGE2 || MODE == MODE_STAGE1) && (NDIM == 3 || kRing2D);
    // occupancy range (waves per SIMD) the compiler aims for: at least
    // kWaves (its register budget), at most kWavesMax (8: no bound)
    static constexpr int kWaves =
        sizeof(R) == 4 ? ((kRing || (NDIM == 3 && MODE == MODE_STAGE1)) ? 3 : 4) : 2;
    static constexpr int kWavesMax = 8;
    // One barrier per plane (double-buffered W and flux tiles): measured
    // faster for the FP64 stage 2; the mixed stages would need a fourth ring
    // plane and lose a work-group per CU.
    // The marching loop unrolled by two with two prefetch buffers, so that
    // the prefetched plane is not copied between loop-carried registers
    // (which makes the compiler wait for the load in the iteration that
    // issued it).  It pays where registers allow: the mixed 3-D stage 2; the
    // mixed stage 1 would spill at its four-wave register budget.
    static constexpr bool kUnroll2 = NDIM == 3 && sizeof(R) == 4 && MODE == MODE_STAGE2;
    static constexpr bool kOneBarrier =
        (NDIM == 3 || kOne2D) &&
        sizeof(R) == 8 && MODE == MODE_STAGE2;
    // The raw halo cell of the next plane loaded one iteration ahead, so the
    // barrier after the plane's W does not wait for it: ten more registers.
    // Measured at 256^3: the Heun stage 2 holds them without losing
    // occupancy (mixed 598 -> 556 us; FP64 unchanged); the mixed stage 1
    // gains about 2 %; the FP64 stage 1 loses 6 % and does without.
    static constexpr bool kHaloPrefetch =
        NDIM == 3 && (MODE == MODE_STAGE2 || (MODE == MODE_STAGE1 && sizeof(R) == 4));
    // U^n of the next updated plane loaded during this plane's update,
    // before its stores, instead of at the next update (where the load is
    // consumed at once): ten more registers.  Measured at 256^3: the mixed
    // Heun stage 2 holds them at three waves per SIMD (543 -> 530 us); the
    // FP64 stage 2 loses 2.4 % and does without.
    static constexpr bool kBasePrefetch = NDIM == 3 && sizeof(R) == 4 && MODE == MODE_STAGE2;
    // The waves that convert the halo cells and compute the faces past the
    // tile's last row and column (the first waves of the work-group) run at
    // raised priority through that work, up to the barrier after the faces:
    // they are the ones the other waves wait for there.  Measured at 256^3
    // with two barriers per plane: mixed stage 2 -4.5 %, FP64 stage 1
    // -6.5 %; with one barrier per plane (the other two 3-D kernels) it cost
    // 1.5-4 %, so those keep the default priority.
    static constexpr bool kPrio = NDIM == 3 && !kOneBarrier;
};

template <int NDIM, typename R, int MODE, int TX, int TY>
__device__ __forceinline__ void stage_body(const StageArgs& a, int b, int blk) {
    constexpr int NC = NDIM + 2;
    constexpr bool HY = (NDIM == 3);
    constexpr bool HZ = (NDIM >= 2);
    constexpr int NT = TX * TY;
    // van Leer modes: the predictor (piecewise-constant states, half step,
    // writes the predicted primitive state of type R into a.out; _C: the
    // predicted conserved state in FP64) and the corrector (reads that state
    // as its stencil input, PLM, full step from U^n in a.base, writes
    // U^{n+1} to a.out)
    constexpr bool PRED = MODE == MODE_VL2_PRED || MODE == MODE_VL2_PRED_C;
    constexpr bool CORR = MODE == MODE_VL2_CORR || MODE == MODE_VL2_CORR_C;
    constexpr bool PRIM_OUT = MODE == MODE_VL2_PRED;
    constexpr bool FIRST = PRED;
    constexpr bool PRIM_IN = MODE == MODE_VL2_CORR;
    constexpr bool NEED_UIN = MODE == MODE_STAGE1 || MODE == MODE_STAGE2 || PRED;
    constexpr bool NEED_BASE = MODE == MODE_STAGE2 || CORR;
    constexpr bool EPILOGUE = MODE == MODE_STAGE2 || CORR;
    static_assert(HY || TY == 1, "tile rows need a second in-plane axis");
    static_assert(4 * TX + (HY ? 4 * TY : 0) <= NT || !HY, "one halo cell per thread");
    static_assert(HY || TX >= 4, "one halo cell per thread");

    const Geo& g = a.geo;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const long long N = g.ncells;
    const long long P = (long long)n0 * n1;  // plane stride
    const long long BS = (long long)NC * N;  // elements of one block of a field
    const long long boff = (long long)blk * BS;
    const Links lk = stage_links(a, blk);
    const double gm1 = g.gamma - 1.0;

    const int tix = b % a.tiles_x;
    b /= a.tiles_x;
    const int tiy = b % a.tiles_y;
    b /= a.tiles_y;
    const int x0 = tix * TX, y0 = tiy * TY, z0 = b * a.kz;
    const int z1 = min(z0 + a.kz, n2);
    const int ax = min(TX, n0 - x0);
    const int ay = min(TY, n1 - y0);
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const bool act = lx < ax && ly < ay;
    const long long col = (long long)(y0 + ly) * n0 + (x0 + lx);

    // this thread's halo cell (tile coordinates hx, hy), resolved once to an
    // element offset hcol in the field (its block's offset + the in-plane
    // index) or in the ghost buffer (hslot), with its plane and component
    // strides
    bool hact = false, hslot = false;
    int hx = 0, hy = 0, hvax = -1, hvm = VM_NONE, hk = 0;
    long long hcol = 0, hc = 0;
    {
        const int nhx = 4 * ay;
        const int nhy = HY ? 4 * ax : 0;
        if (tid < nhx) {
            const int q = tid & 3;
            hy = tid >> 2;
            hx = q < 2 ? q - 2 : ax + (q - 2);
            hact = true;
        } else if (tid < nhx + nhy) {
            const int h2 = tid - nhx, q = h2 & 3;
            hx = h2 >> 2;
            hy = q < 2 ? q - 2 : ay + (q - 2);
            hact = true;
        }
        if (hact) {
            int X = x0 + hx, Y = y0 + hy, db = 0, sl = -1;
            if (X < 0 || X >= n0) {
                X = resolve(g, lk, 0, X, hvm, db, sl);
                hvax = 0;
            } else if (Y < 0 || Y >= n1) {
                Y = resolve(g, lk, 1, Y, hvm, db, sl);
                hvax = 1;
            }
            if (sl >= 0) {
                // a ghost slot: [comp][layer][z][y] of an x side, [comp][layer][z][x] of a y side
                hslot = true;
                const long long sb = (long long)sl * NC * a.gcs;
                hcol = hvax == 0 ? sb + ((long long)X * n2) * n1 + Y : sb + ((long long)Y * n2) * n0 + X;
                hk = hvax == 0 ? n1 : n0;
                hc = a.gcs;
            } else {
                hcol = (long long)(blk + db) * BS + (long long)Y * n0 + X;
                hk = (int)P;
                hc = N;
            }
        }
    }

    // whether an in-plane side treats the normal velocity of its ghosts
    // (outflow, reflecting); uniform over the grid
    const bool halo_vm = g.bc[0][0] >= BC_OUTFLOW || g.bc[0][1] >= BC_OUTFLOW ||
                         (HY && (g.bc[1][0] >= BC_OUTFLOW || g.bc[1][1] >= BC_OUTFLOW));
    const double dt_step = a.use_device_dt ? device_dt(a.ctrl) : a.dt_host;
    const double dt = PRED ? 0.5 * dt_step : dt_step;  // the predictor advances half a step
    const double lam0 = dt / g.dx[0];
    const double lam1 = dt / g.dx[1];
    const double lam2 = dt / g.dx[2];
    const Gas<R> gr = make_gas<R>(g.gamma);

    constexpr bool RING = StageOccupancy<NDIM, R, MODE>::kRing && HZ;
    // One barrier per plane: plane k's W and fluxes go to buffer k & 1 and
    // the update of plane k-1 follows the face pass of plane k, so the
    // barrier that publishes plane k's W also publishes plane k-1's fluxes.
    constexpr bool ONE = StageOccupancy<NDIM, R, MODE>::kOneBarrier;
    constexpr int NB = ONE ? 2 : 1;
    constexpr int RS = ONE ? 4 : 3;  // ring slots: planes k-1 .. k+2 live at once
    __shared__ double sRaw[RING ? RS : 1][RING ? NC : 1][RING ? NT : 1];
    // rows of the W tile: in 1-D and 2-D a tile is one row (row offset RO)
    constexpr int RO = HY ? 0 : -2;
    __shared__ R sW[NB][NC][HY ? TY + 4 : 1][TX + 4];
    using FT = R;
    __shared__ FT sFx[NB][NC][TY][TX + 1];
    __shared__ FT sFy[NB][HY ? NC : 1][HY ? TY + 1 : 1][TX];

    bool bad = false;
    double rate = 0.0;
    // z pipeline entering iteration k: W_k, W_{k+1}, d = W_{k+1} - W_k, the
    // left state of face k+1/2 (W_k + delta_k / 2); fza, fzb: the fluxes of
    // faces k-3/2 and k-1/2 (fzb only, without ONE)
    R wk[NC], wk1[NC], dk[NC], lz[NC];
    FT fza[NC], fzb[NC];
    // raw interior plane k+2 in flight (HZ), in two buffers that alternate
    // between iterations so a load lands directly where it is consumed
    double uiA[NC], uiB[NC];
    int vmA = VM_NONE, vmB = VM_NONE;
    // the raw halo cell of this thread (HALO_PF: the next plane's, in flight)
    constexpr bool HALO_PF = StageOccupancy<NDIM, R, MODE>::kHaloPrefetch;
    constexpr bool PRIO = StageOccupancy<NDIM, R, MODE>::kPrio;
    double uhalo[NC];

    // interior plane z (any z: outside the mesh it is a ghost plane)
    // cell (plane offset poff, the same for the work-group) + (in-plane index tc)
    const uint32_t ext8 = (uint32_t)P * 8u, extR = (uint32_t)P * (uint32_t)sizeof(R);
    auto load_in = [&](long long poff, uint32_t tc, double (&u)[NC]) {
        if constexpr (PRIM_IN) {
            const R* F = reinterpret_cast<const R*>(a.in);
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = (double)plane_load(F, c * N + poff, extR, tc * (uint32_t)sizeof(R));
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = plane_load(a.in, c * N + poff, ext8, tc * 8u);
        }
    };
    // the halo cell of plane k: it may lie in another block or in a ghost
    // slot, so it is addressed from the base with a per-thread offset
    auto load_halo = [&](int k, double (&u)[NC]) {
        const long long o = hcol + (long long)k * hk;
        if constexpr (PRIM_IN) {
            // (a refined mesh's ghost slots hold conserved values: its van
            // Leer corrector reads the conserved predictor, not this form)
            const R* F = reinterpret_cast<const R*>(a.in) + o;
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = (double)F[c * hc];
        } else {
            // (the base is selected as an integer: selecting between the two
            // argument fields themselves makes the compiler copy the
            // arguments to private memory)
            const uintptr_t bi = reinterpret_cast<uintptr_t>(a.in), bg = reinterpret_cast<uintptr_t>(a.gbuf);
            const double* F = reinterpret_cast<const double*>(hslot ? bg : bi) + o;
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = F[c * hc];
        }
    };
    const uint32_t col32 = (uint32_t)col;
    auto load_interior = [&](int z, double (&u)[NC], int& vm) {
        vm = VM_NONE;
        int zr = z, db = 0, sl = -1;
        if (z < 0 || z >= n2) zr = resolve(g, lk, 2, z, vm, db, sl);
        if (!PRIM_IN && sl >= 0) {
            // a ghost slot of a z side: [comp][layer][y][x], one plane per layer
#pragma unroll
            for (int c = 0; c < NC; ++c)
                u[c] = plane_load(a.gbuf, ((long long)sl * NC + c) * a.gcs + (long long)zr * P, ext8, col32 * 8u);
        } else {
            load_in((long long)(blk + db) * BS + (long long)zr * P, col32, u);
        }
    };

    if (HZ && act) {
        R w[4][NC];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            int vm;
            double u[NC];
            load_interior(z0 - 2 + s, u, vm);
            in_to_w<NDIM, R, PRIM_IN>(gm1, u, vm == VM_NONE ? -1 : 2, vm, w[s], bad);
            if (RING && s >= 2) {
#pragma unroll
                for (int c = 0; c < NC; ++c) sRaw[RING ? (z0 - 2 + s) % RS : 0][RING ? c : 0][RING ? tid : 0] = u[c];
            }
        }
        // planes z0-2 .. z0+1: face z0-1/2 and the left state of face z0+1/2,
        // in the operations face_flux uses
        R wl[NC], wr[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const R d0 = w[1][c] - w[0][c], d1 = w[2][c] - w[1][c], d2 = w[3][c] - w[2][c];
            R s1, s2;
            Ops<R>::minmod2(d0, d1, d2, s1, s2);
            wl[c] = FIRST ? w[1][c] : Ops<R>::fma(R(0.5), s1, w[1][c]);
            wr[c] = FIRST ? w[2][c] : Ops<R>::fma(R(-0.5), s2, w[2][c]);
            lz[c] = Ops<R>::fma(R(0.5), s2, w[2][c]);
            wk[c] = w[2][c];
            wk1[c] = w[3][c];
            dk[c] = d2;
        }
        {
            R f[NC];
            face_flux_states<NDIM, 2, R>(gr, wl, wr, f);
#pragma unroll
            for (int c = 0; c < NC; ++c) fzb[c] = (FT)f[c];
        }
        load_interior(z0 + 2, uiA, vmA);
    }
    if (HALO_PF && hact && z0 < z1) load_halo(z0, uhalo);
    // (BASE_PF) U^n of the first updated plane, loaded ahead
    constexpr bool BASE_PF = StageOccupancy<NDIM, R, MODE>::kBasePrefetch && NEED_BASE;
    // the buffers alternate with the iterations: every iteration updates a plane
    static_assert(!BASE_PF || !ONE, "base prefetch needs an update in every iteration");
    double ubA[NC], ubB[NC];
    if (BASE_PF && act && z0 < z1) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            ubA[c] = plane_load<double, kNonTemporal>(a.base, c * N + boff + (long long)z0 * P, ext8, col32 * 8u);
    }

    // One iteration: plane k enters the stencil (its raw data ui, the ghost
    // treatment vmi), plane k+3 is loaded into un (vmn), and one plane is
    // updated (BASE_PF: with U^n from ubc, loading the next plane's into ubn).
    auto plane = [&](const int k, double(&ui)[NC], int& vmi, double(&un)[NC], int& vmn, double(&ubc)[NC],
                     double(&ubn)[NC]) __attribute__((always_inline)) {
        const int bw = ONE ? (k & 1) : 0;        // buffer of plane k
        const int ku = ONE ? k - 1 : k;          // plane updated in this iteration
        const int bu = ONE ? (ku & 1) : 0;       // its buffer
        const bool live = !ONE || k < z1;        // plane k exists (the last ONE iteration only updates)
        FT fzc[NC];                              // flux of face k+1/2
        if (live && act) {
            R wc[NC];
            if (HZ) {
                // W_{k+2} arrived: z face k+1/2 from (W_k, W_{k+1}, W_{k+2})
                R w2[NC], wr[NC];
                // the ghost treatment of a plane is the same for the whole
                // work-group: held in a scalar register, it costs no divergence
                const int vz = __builtin_amdgcn_readfirstlane(vmi);
                in_to_w<NDIM, R, PRIM_IN>(gm1, ui, vz == VM_NONE ? -1 : 2, vz, w2, bad);
                // plane k+2 is an interior plane whenever its update comes
                if (RING) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) sRaw[RING ? (k + 2) % RS : 0][RING ? c : 0][RING ? tid : 0] = ui[c];
                }
                // plane k+3 is W_{k'+2} of the next iteration k' = k+1; it lies at
                // most two planes outside the mesh only while that iteration exists
                if (k + 1 < z1) load_interior(k + 3, un, vmn);
                if constexpr (FIRST) {
                    // face k+1/2 from the cells' values W_k and W_{k+1}
                    R f[NC];
                    face_flux_states<NDIM, 2, R>(gr, wk, wk1, f);
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        fzc[c] = (FT)f[c];
                        wc[c] = wk[c];
                        wk[c] = wk1[c];
                        wk1[c] = w2[c];
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const R d2 = w2[c] - wk1[c];
                        const R s1 = minmod(dk[c], d2);
                        wr[c] = Ops<R>::fma(R(-0.5), s1, wk1[c]);
                        const R lnext = Ops<R>::fma(R(0.5), s1, wk1[c]);
                        wc[c] = wk[c];
                        dk[c] = d2;
                        wk[c] = wk1[c];
                        wk1[c] = w2[c];
                        w2[c] = lnext;  // reuse: left state of face k+3/2
                    }
                    {
                        R f[NC];
                        face_flux_states<NDIM, 2, R>(gr, lz, wr, f);
#pragma unroll
                        for (int c = 0; c < NC; ++c) fzc[c] = (FT)f[c];
                    }
#pragma unroll
                    for (int c = 0; c < NC; ++c) lz[c] = w2[c];
                }
            } else {
                double u[NC];
                load_in(boff + (long long)k * P, col32, u);
                in_to_w<NDIM, R, PRIM_IN>(gm1, u, -1, VM_NONE, wc, bad);
            }
#pragma unroll
            for (int c = 0; c < NC; ++c) sW[bw][c][ly + 2 + RO][lx + 2] = wc[c];
        }
        if (live && hact) {
            if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
            R wh[NC];
            // the halo cell of plane k: loaded one iteration ahead (HALO_PF),
            // else now
            if (!HALO_PF) load_halo(k, uhalo);
            // not checked here: every cell is checked by the tile that owns it
            in_to_w<NDIM, R, PRIM_IN, false>(gm1, uhalo, halo_vm ? hvax : -1, hvm, wh, bad);
#pragma unroll
            for (int c = 0; c < NC; ++c) sW[bw][c][hy + 2 + RO][hx + 2] = wh[c];
            if (HALO_PF && k + 1 < z1) load_halo(k + 1, uhalo);
        }
        __syncthreads();

        if (live) {
            // x faces: face i separates tile columns i-1 and i; LDS columns i..i+3
            if (ly < ay && lx <= ax) {
                R w0[NC], w1[NC], w2[NC], w3[NC], F[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    w0[c] = sW[bw][c][ly + 2 + RO][lx];
                    w1[c] = sW[bw][c][ly + 2 + RO][lx + 1];
                    w2[c] = sW[bw][c][ly + 2 + RO][lx + 2];
                    w3[c] = sW[bw][c][ly + 2 + RO][lx + 3];
                }
                face_flux<NDIM, 0, R, FIRST>(gr, w0, w1, w2, w3, F);
#pragma unroll
                for (int c = 0; c < NC; ++c) sFx[bw][c][ly][lx] = (FT)F[c];
            }
            if (HY && lx < ax && ly <= ay) {
                R w0[NC], w1[NC], w2[NC], w3[NC], F[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    w0[c] = sW[bw][c][HY ? ly : 0][lx + 2];
                    w1[c] = sW[bw][c][HY ? ly + 1 : 0][lx + 2];
                    w2[c] = sW[bw][c][ly + 2 + RO][lx + 2];
                    w3[c] = sW[bw][c][HY ? ly + 3 : 0][lx + 2];
                }
                face_flux<NDIM, 1, R, FIRST>(gr, w0, w1, w2, w3, F);
#pragma unroll
                for (int c = 0; c < NC; ++c) sFy[bw][HY ? c : 0][HY ? ly : 0][lx] = (FT)F[c];
            }
            // faces past the last thread column / row of a full tile; in 3-D the
            // x and y ones share one code path (axis chosen per lane)
            const int ex = (ax == TX) ? ay : 0;
            const int ey = (HY && ay == TY) ? ax : 0;
            for (int e = tid; e < ex + ey; e += NT) {
                if constexpr (PRIO) __builtin_amdgcn_s_setprio(2);
                R w0[NC], w1[NC], w2[NC], w3[NC], F[NC];
                if constexpr (HY) {
                    const bool yaxis = e >= ex;
                    // x face (row e, column TX) or y face (row TY, column e - ex)
                    const int r0 = yaxis ? TY : e + 2, c0 = yaxis ? e - ex + 2 : TX;
                    const int dr = yaxis ? 1 : 0, dc = yaxis ? 0 : 1;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        w0[c] = sW[bw][c][HY ? r0 : 0][c0];
                        w1[c] = sW[bw][c][HY ? r0 + dr : 0][c0 + dc];
                        w2[c] = sW[bw][c][HY ? r0 + 2 * dr : 0][c0 + 2 * dc];
                        w3[c] = sW[bw][c][HY ? r0 + 3 * dr : 0][c0 + 3 * dc];
                    }
                    face_flux_xy<R, FIRST>(gr, yaxis, w0, w1, w2, w3, F);
                    if (yaxis) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) sFy[bw][c][TY][e - ex] = (FT)F[c];
                    } else {
#pragma unroll
                        for (int c = 0; c < NC; ++c) sFx[bw][c][e][TX] = (FT)F[c];
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        w0[c] = sW[bw][c][e + 2 + RO][TX];
                        w1[c] = sW[bw][c][e + 2 + RO][TX + 1];
                        w2[c] = sW[bw][c][e + 2 + RO][TX + 2];
                        w3[c] = sW[bw][c][e + 2 + RO][TX + 3];
                    }
                    face_flux<NDIM, 0, R, FIRST>(gr, w0, w1, w2, w3, F);
#pragma unroll
                    for (int c = 0; c < NC; ++c) sFx[bw][c][e][TX] = (FT)F[c];
                }
            }
        }
        if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
        if (!ONE) __syncthreads();

        if (act && ku >= z0) {
            const long long kuP = boff + (long long)ku * P;  // plane offset of the updated cell
            const uint32_t colb = col32 * (uint32_t)sizeof(double);
            // z fluxes of faces ku-1/2 and ku+1/2
            const FT(&zlo)[NC] = ONE ? fza : fzb;
            const FT(&zhi)[NC] = ONE ? fzb : fzc;
            double uin[NC], ubase[NC];
            if (RING) {
#pragma unroll
                for (int c = 0; c < NC; ++c) uin[c] = sRaw[RING ? ku % RS : 0][RING ? c : 0][RING ? tid : 0];
            } else if (NEED_UIN) {
#pragma unroll
                for (int c = 0; c < NC; ++c) uin[c] = plane_load(a.in, c * N + kuP, ext8, colb);
            }
            if (BASE_PF) {
#pragma unroll
                for (int c = 0; c < NC; ++c) ubase[c] = ubc[c];
                if (ku + 1 < z1) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        ubn[c] = plane_load<double, kNonTemporal>(a.base, c * N + kuP + P, ext8, colb);
                }
            } else if (NEED_BASE) {
#pragma unroll
                for (int c = 0; c < NC; ++c) ubase[c] = plane_load<double, kNonTemporal>(a.base, c * N + kuP, ext8, colb);
            }
            double unew[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                // the axis terms summed in x, y, z order from the first one
                // (a sum of two rounded products is the same either way round,
                // so interchanging two axes leaves the update bitwise unchanged)
                double acc = lam0 * ((double)sFx[bu][c][ly][lx] - (double)sFx[bu][c][ly][lx + 1]);
                if (HY)
                    acc = acc + lam1 * ((double)sFy[bu][HY ? c : 0][HY ? ly : 0][lx] -
                                        (double)sFy[bu][HY ? c : 0][HY ? ly + 1 : 0][lx]);
                if (HZ) acc = acc + lam2 * ((double)zlo[c] - (double)zhi[c]);
                double r;
                if (MODE == MODE_RHS)
                    r = acc;
                else if (MODE == MODE_STAGE1 || PRED)
                    r = uin[c] + acc;
                else if (CORR)
                    r = ubase[c] + acc;
                else
                    r = 0.5 * ubase[c] + 0.5 * (uin[c] + acc);
                if (!PRIM_OUT) plane_store<double, EPILOGUE ? kNonTemporal : 0>(a.out, c * N + kuP, ext8, colb, r);
                unew[c] = r;
            }
            if (PRIM_OUT) {
                // the predicted state is kept only as primitive variables of type R
                double w[NC];
                bad |= !cons_to_prim<NDIM>(gm1, unew, w);
                R* wout = reinterpret_cast<R*>(a.out);
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    plane_store(wout, c * N + kuP, extR, col32 * (uint32_t)sizeof(R), (R)w[c]);
            }
            if (EPILOGUE && a.want_dt) {
                double w[NC];
                bad |= !cons_to_prim<NDIM>(gm1, unew, w);
                const double cr = cfl_rate<NDIM>(g, w);
                rate = cr > rate ? cr : rate;
            }
        }
        if (HZ && act) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                if (ONE) fza[c] = fzb[c];
                fzb[c] = fzc[c];
            }
        }
    };

    const int kend = z1 + (ONE ? 1 : 0);
    if constexpr (StageOccupancy<NDIM, R, MODE>::kUnroll2 && HZ) {
        for (int k = z0; k < kend; k += 2) {
            plane(k, uiA, vmA, uiB, vmB, ubA, ubB);
            if (k + 1 < kend) plane(k + 1, uiB, vmB, uiA, vmA, ubB, ubA);
        }
    } else {
        for (int k = z0; k < kend; ++k) plane(k, uiA, vmA, uiA, vmA, ubA, ubA);
    }

    if (bad) atomicOr(&a.ctrl->flags, FLAG_NONPHYSICAL);
    if (EPILOGUE && a.want_dt) {
        __shared__ double red[NT / 64 > 0 ? NT / 64 : 1];
        rate = wave_max(rate);
        if ((tid & 63) == 0) red[tid >> 6] = rate;
        __syncthreads();
        if (tid == 0) {
            double m = red[0];
            for (int i = 1; i < NT / 64; ++i) m = red[i] > m ? red[i] : m;
            atomicMax(&a.ctrl->rate_bits, (unsigned long long)__double_as_longlong(m));
        }
    }
}

template <int NDIM, typename R, int MODE, int TX, int TY>
__global__ __launch_bounds__(TX * TY)
__attribute__((amdgpu_waves_per_eu(StageOccupancy<NDIM, R, MODE>::kWaves, StageOccupancy<NDIM, R, MODE>::kWavesMax)))
void stage_kernel(StageArgs a) {
    if (a.use_device_dt && a.ctrl->done) return;  // uniform over the grid
    // work-group -> (block, work-group within the block), block after block:
    // each XCD's contiguous range of work-groups covers whole blocks (measured
    // faster than taking them in the order of the whole mesh's tile grid)
    int wg = xcd_remap(blockIdx.x, gridDim.x);
    int blk = a.blk0;
    if (a.nblk > 1) {
        const int per = a.tiles_x * a.tiles_y * a.chunks_z;
        const int q = wg / per;
        blk += q;
        wg -= q * per;
    }
    stage_body<NDIM, R, MODE, TX, TY>(a, wg, blk);
}

// Batched stage: work-group -> (member, work-group of the member) from a
// table; members that reached their run limit are skipped.
template <int NDIM, typename R, int MODE, int TX, int TY>
__global__ __launch_bounds__(TX * TY)
__attribute__((amdgpu_waves_per_eu(StageOccupancy<NDIM, R, MODE>::kWaves, StageOccupancy<NDIM, R, MODE>::kWavesMax)))
void stage_kernel_batch(
    const MeshDesc* __restrict__ descs, const int2* __restrict__ blk) {
    const int2 e = blk[xcd_remap(blockIdx.x, gridDim.x)];
    const MeshDesc& d = descs[e.x];
    if (d.ctrl->done) return;  // uniform over the work-group
    StageArgs a{};  // every field set: a batch member is one unrefined block
    a.ctrl = d.ctrl;
    a.geo = d.geo;
    a.dt_host = 0.0;
    a.use_device_dt = 1;
    a.tiles_x = d.tiles_x;
    a.tiles_y = d.tiles_y;
    a.chunks_z = d.chunks_z;
    a.kz = d.kz;
    a.blk0 = 0;
    a.nblk = 1;
    a.conc = 1;
    a.side = nullptr;
    a.gbuf = nullptr;
    a.gcs = 0;
    if (MODE == MODE_STAGE1 || MODE == MODE_VL2_PRED) {
        a.in = d.U;
        a.base = d.U;
        a.out = d.U1;  // van Leer: the predicted primitive state, type R
        a.want_dt = 0;
    } else {
        a.in = d.U1;
        a.base = d.U;
        a.out = d.U;
        a.want_dt = 1;
    }
    stage_body<NDIM, R, MODE, TX, TY>(a, e.y, 0);
}

// ------------------------------------------------------------- small kernels

// blockIdx.y: the block of the mesh (block layout); a refined mesh's blocks
// of level L (from the level starts) take level 0's cell widths times 2^-L
template <int NDIM>
__global__ __launch_bounds__(256) void dt_kernel(Geo g0, LevelStarts starts, const double* __restrict__ U,
                                                 Ctrl* ctrl, int skip_done) {
    constexpr int NC = NDIM + 2;
    if (skip_done && ctrl->done) return;  // uniform over the grid
    Geo g = g0;
    // the block's level: its inverse cell widths are level 0's times 2^L
    // (exact: 1 / (dx 2^-L) rounds to (1 / dx) 2^L)
    int lev = 0;
#pragma unroll
    for (int L = 1; L < kMaxLevels; ++L) lev += (int)blockIdx.y >= starts.s[L - 1] ? 1 : 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) g.inv_dx[k] = __builtin_ldexp(g0.inv_dx[k], lev);
    U += (long long)blockIdx.y * NC * g.ncells;
    double best = 0.0;
    bool bad = false;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < g.ncells;
         cell += (long long)gridDim.x * blockDim.x) {
        double u[NC], w[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) u[c] = U[c * g.ncells + cell];
        bad |= !cons_to_prim<NDIM>(g.gamma - 1.0, u, w);
        const double cr = cfl_rate<NDIM>(g, w);
        best = cr > best ? cr : best;
    }
    if (bad) atomicOr(&ctrl->flags, FLAG_NONPHYSICAL);
    __shared__ double red[4];
    best = wave_max(best);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int i = 1; i < 4; ++i) m = red[i] > m ? red[i] : m;
        atomicMax(&ctrl->rate_bits, (unsigned long long)__double_as_longlong(m));
    }
}

__global__ void ctrl_kernel(Ctrl* c, int op, double a0, double a1, double cfl) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    switch (op) {
        case CTRL_INIT:
            c->t = a0;
            c->steps = 0;
            c->flags = 0;
            c->dt_valid = 0;
            c->dt_raw = 0.0;
            c->rate_bits = 0ull;
            c->t_end = 0.0;
            c->max_steps = 0ull;
            c->done = 0;
            break;
        case CTRL_RESET_MIN:
            c->rate_bits = 0ull;
            break;
        case CTRL_FINALIZE_DT:
            c->dt_raw = cfl / __longlong_as_double((long long)c->rate_bits);
            c->dt_valid = 1;
            c->rate_bits = 0ull;
            break;
        case CTRL_FINALIZE_STEP:
            finalize_step(c, cfl);
            break;
        case CTRL_ADVANCE_T:
            c->t = c->t + a0;
            c->steps += 1;
            c->dt_valid = 0;
            break;
        case CTRL_SET_LIMITS:
            c->t_end = a0;
            c->max_steps = a1 > 0.0 ? c->steps + (unsigned long long)a1 : 0ull;
            update_done(c);
            break;
        default:
            break;
    }
}

// Status of every batch member (done, flags, steps) into one table.
__global__ void status_gather_kernel(const MeshDesc* __restrict__ d, int n, unsigned long long* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const Ctrl* c = d[i].ctrl;
        out[3 * i] = c->done;
        out[3 * i + 1] = c->flags;
        out[3 * i + 2] = c->steps;
    }
}

__global__ void ctrl_batch_kernel(const MeshDesc* __restrict__ d, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) finalize_step(d[i].ctrl, d[i].geo.cfl);
}

// Neumaier-compensated accumulator combined pairwise in a fixed tree.
struct Comp {
    double s, c;
};
__device__ __forceinline__ Comp comp_add(Comp a, double x) {
    const double t = a.s + x;
    if (dabs(a.s) >= dabs(x))
        a.c += (a.s - t) + x;
    else
        a.c += (x - t) + a.s;
    a.s = t;
    return a;
}
__device__ __forceinline__ Comp comp_merge(Comp a, Comp b) {
    Comp r = comp_add(a, b.s);
    r.c += b.c;
    return r;
}

// blockIdx.y: the block of the mesh (block layout); one partial per work-group
template <int NC>
__global__ __launch_bounds__(256) void totals_pass1(long long ncells, const double* __restrict__ U,
                                                    double* __restrict__ parts) {
    __shared__ double ss[NC][256], sc[NC][256];
    U += (long long)blockIdx.y * NC * ncells;
    parts += (long long)blockIdx.y * gridDim.x * NC * 2;
    const long long per = (ncells + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * per;
    const long long hi = lo + per < ncells ? lo + per : ncells;
    Comp acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = Comp{0.0, 0.0};
    for (long long i = lo + threadIdx.x; i < hi; i += 256)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = comp_add(acc[c], U[c * ncells + i]);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        ss[c][threadIdx.x] = acc[c].s;
        sc[c][threadIdx.x] = acc[c].c;
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Comp r = comp_merge(Comp{ss[c][threadIdx.x], sc[c][threadIdx.x]},
                                    Comp{ss[c][threadIdx.x + w], sc[c][threadIdx.x + w]});
                ss[c][threadIdx.x] = r.s;
                sc[c][threadIdx.x] = r.c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            parts[(blockIdx.x * NC + c) * 2] = ss[c][0];
            parts[(blockIdx.x * NC + c) * 2 + 1] = sc[c][0];
        }
}

// The fixed tree over the partials.  out == null: the (sum, compensation)
// pairs go to sums[2 c], sums[2 c + 1]; else out[c] = dV (sum + compensation).
template <int NC>
__global__ __launch_bounds__(256) void totals_pass2(int nparts, const double* __restrict__ parts,
                                                    double* __restrict__ sums, double* __restrict__ out,
                                                    double dV) {
    __shared__ double ss[NC][256], sc[NC][256];
    Comp acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = Comp{0.0, 0.0};
    for (int p = threadIdx.x; p < nparts; p += 256)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            acc[c] = comp_merge(acc[c], Comp{parts[(p * NC + c) * 2], parts[(p * NC + c) * 2 + 1]});
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        ss[c][threadIdx.x] = acc[c].s;
        sc[c][threadIdx.x] = acc[c].c;
    }
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                Comp r = comp_merge(Comp{ss[c][threadIdx.x], sc[c][threadIdx.x]},
                                    Comp{ss[c][threadIdx.x + w], sc[c][threadIdx.x + w]});
                ss[c][threadIdx.x] = r.s;
                sc[c][threadIdx.x] = r.c;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (out) {
                out[c] = dV * (ss[c][0] + sc[c][0]);
            } else {
                sums[2 * c] = ss[c][0];
                sums[2 * c + 1] = sc[c][0];
            }
        }
}

// m_d = rho v_d, E = p/(gamma - 1) + (1/2) sum_d m_d v_d
// W and U may be the same array (each cell is read before it is written);
// blockIdx.y: the block of the mesh (block layout).
template <int NDIM>
__global__ __launch_bounds__(256) void prim_to_cons_kernel(Geo g, const double* W, double* U) {
    constexpr int NC = NDIM + 2;
    W += (long long)blockIdx.y * NC * g.ncells;
    U += (long long)blockIdx.y * NC * g.ncells;
    for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < g.ncells;
         cell += (long long)gridDim.x * blockDim.x) {
        const double rho = W[cell];
        double ke2 = 0.0;
        U[cell] = rho;
#pragma unroll
        for (int d = 0; d < NDIM; ++d) {
            const double v = W[(1 + d) * g.ncells + cell];
            const double mom = rho * v;
            U[(1 + d) * g.ncells + cell] = mom;
            ke2 = ke2 + mom * v;
        }
        U[(NC - 1) * g.ncells + cell] = W[(NC - 1) * g.ncells + cell] / (g.gamma - 1.0) + 0.5 * ke2;
    }
}

// Padded primitive export: physical padded layout [c][K][J][I] with two ghost
// layers on every active physical axis, corners zero.
template <int NDIM, typename R>
__global__ __launch_bounds__(256) void padded_prim_kernel(Geo g, const double* __restrict__ U,
                                                          double* __restrict__ Wp, Ctrl* ctrl) {
    constexpr int NC = NDIM + 2;
    // physical extents of the mesh: axis p of NDIM -> kernel axis (3-D
    // identity; 2-D y is kernel z)
    const int m0 = g.n[0] * g.blocks[0], m1 = g.n[1] * g.blocks[1], m2 = g.n[2] * g.blocks[2];
    int nph[3] = {m0, NDIM == 3 ? m1 : (NDIM == 2 ? m2 : 1), NDIM == 3 ? m2 : 1};
    int P[3];
    for (int d = 0; d < 3; ++d) P[d] = nph[d] + (d < NDIM ? 4 : 0);
    const long long total = (long long)P[0] * P[1] * P[2];
    bool bad = false;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int I = (int)(q % P[0]);
        const int J = (int)((q / P[0]) % P[1]);
        const int K = (int)(q / ((long long)P[0] * P[1]));
        int pc[3] = {I - (NDIM >= 1 ? 2 : 0), J - (NDIM >= 2 ? 2 : 0), K - (NDIM >= 3 ? 2 : 0)};
        int outside = 0;
        for (int d = 0; d < NDIM; ++d) outside += (pc[d] < 0 || pc[d] >= nph[d]);
        double out[NC];
        if (outside > 1) {
            for (int c = 0; c < NC; ++c) out[c] = 0.0;
        } else {
            R w[NC];
            int kx = pc[0], ky = NDIM == 3 ? pc[1] : 0, kzc = NDIM == 3 ? pc[2] : (NDIM == 2 ? pc[1] : 0);
            load_w<NDIM, R>(g, U, kx, ky, kzc, w, bad);
            for (int c = 0; c < NC; ++c) out[c] = (double)w[c];
        }
        for (int c = 0; c < NC; ++c) Wp[c * total + q] = out[c];
    }
    if (bad) atomicOr(&ctrl->flags, FLAG_NONPHYSICAL);
}

// ------------------------------------------------------- static refinement

// The two transverse kernel axes of a side of kernel axis ax (lower first).
__device__ __forceinline__ void transverse(int ax, int& lo, int& hi) {
    lo = ax == 0 ? 1 : 0;
    hi = ax == 2 ? 1 : 2;
}

// Element i (a run-time index) of a three- or four-element array, by
// selects: indexing the array itself would place it in private memory.
__device__ __forceinline__ int at3(const int (&a)[3], int i) { return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]); }
__device__ __forceinline__ void set3(int (&a)[3], int i, int v) {
    a[0] = i == 0 ? v : a[0];
    a[1] = i == 1 ? v : a[1];
    a[2] = i == 2 ? v : a[2];
}
__device__ __forceinline__ int at4(const int (&a)[4], int i) {
    return i == 0 ? a[0] : (i == 1 ? a[1] : (i == 2 ? a[2] : a[3]));
}

// Raw conserved values of cell (x, y, z) of block blk of a refined mesh, at
// most one coordinate outside the block (by up to two cells): through the
// block's side codes, from a neighbouring block, by a mesh face's boundary
// rule (vax, vm: the velocity treatment), or from a ghost slot.
template <int NC>
__device__ __forceinline__ void smr_cell(const Geo& g, const Links& L, const double* __restrict__ U,
                                         const double* __restrict__ gbuf, long long gcs, int blk, int x, int y,
                                         int z, double (&u)[NC], int& vax, int& vm) {
    int c3[3] = {x, y, z};
    int b = blk;
    vax = -1;
    vm = VM_NONE;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (c3[ax] >= 0 && c3[ax] < g.n[ax]) continue;
        int db = 0, sl = -1;
        const int q = resolve(g, L, ax, c3[ax], vm, db, sl);
        if (sl >= 0) {
            int lo, hi;
            transverse(ax, lo, hi);
            const long long o = (long long)sl * NC * gcs + ((long long)q * g.n[hi] + c3[hi]) * g.n[lo] + c3[lo];
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = gbuf[o + c * gcs];
            vm = VM_NONE;
            return;
        }
        c3[ax] = q;
        b = blk + db;
        if (vm != VM_NONE) vax = ax;
        break;
    }
    const long long N = g.ncells;
    const long long o = (long long)b * NC * N + ((long long)c3[2] * g.n[1] + c3[1]) * g.n[0] + c3[0];
#pragma unroll
    for (int c = 0; c < NC; ++c) u[c] = U[o + c * N];
}

// Primitive FP64 state of a refined mesh's cell (see smr_cell).
template <int NDIM>
__device__ __forceinline__ void smr_prim(const Geo& g, const Links& L, const double* __restrict__ U,
                                         const double* __restrict__ gbuf, long long gcs, int blk, int x, int y,
                                         int z, double (&w)[NDIM + 2], bool& bad) {
    double u[NDIM + 2];
    int vax, vm;
    smr_cell<NDIM + 2>(g, L, U, gbuf, gcs, blk, x, y, z, u, vax, vm);
    to_prim<NDIM, double>(g.gamma - 1.0, u, vax, vm, w, bad);
}

// m_d = rho v_d, E = p/(gamma - 1) + (1/2) sum_d m_d v_d
template <int NDIM>
__device__ __forceinline__ void prim_to_cons_cell(double gamma, const double (&w)[NDIM + 2], double (&u)[NDIM + 2]) {
    double ke2 = 0.0;
    u[0] = w[0];
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        const double mom = w[0] * w[1 + d];
        u[1 + d] = mom;
        ke2 = ke2 + mom * w[1 + d];
    }
    u[NDIM + 1] = w[NDIM + 1] / (gamma - 1.0) + 0.5 * ke2;
}

// Kernel axis of the k-th active axis (physical order: x, y, z).
template <int NDIM>
__device__ __forceinline__ constexpr int active_axis(int k) {
    return NDIM == 2 ? (k == 0 ? 0 : 2) : k;
}

// Restriction onto the two ghost layers of a coarse block's side that faces
// finer blocks: each ghost is the volume average of the 2^NDIM fine cells it
// covers (pairwise means along x, then y, then z), on primitive variables;
// stored as conserved values.  blockIdx.x: the slot; one thread per ghost.
template <int NDIM>
__global__ __launch_bounds__(64) void smr_restrict_kernel(Geo g, const double* __restrict__ U,
                                                           const int* __restrict__ side, double* __restrict__ gbuf,
                                                           long long gcs, const GhostTask* __restrict__ tasks,
                                                           Ctrl* ctrl) {
    constexpr int NC = NDIM + 2;
    constexpr int K = 1 << NDIM;
    const GhostTask t = tasks[blockIdx.x];
    int lo, hi;
    transverse(t.ax, lo, hi);
    const int gn[3] = {g.n[0], g.n[1], g.n[2]};
    const int nlo = at3(gn, lo), nhi = at3(gn, hi), face = nlo * nhi;
    bool bad = false;
    const int q = blockIdx.y * blockDim.x + threadIdx.x;
    if (q < 2 * face) {
        const int layer = q / face, r = q - layer * face;
        const int tl = r % nlo, th = r / nlo;
        double v[NC][K];
#pragma unroll
        for (int o = 0; o < K; ++o) {
            int x3[3] = {0, 0, 0};
            int cb[3] = {0, 0, 0};  // child offsets on the transverse axes
#pragma unroll
            for (int k = 0; k < NDIM; ++k) {
                const int ax = active_axis<NDIM>(k);
                const int off = (o >> k) & 1;
                if (ax == t.ax) {
                    // fine cells 2 layer, 2 layer + 1 in from the face (off 0: the lower)
                    x3[ax] = t.s ? 2 * layer + off : g.n[ax] - 2 - 2 * layer + off;
                } else {
                    const int p = 2 * (ax == lo ? tl : th) + off;  // from the refined root's origin
                    cb[ax] = p / g.n[ax];
                    x3[ax] = p - cb[ax] * g.n[ax];
                }
            }
            const int fb = at4(t.src, at3(cb, lo) + 2 * at3(cb, hi));
            const Links L = table_links(side, fb);
            double w[NC];
            smr_prim<NDIM>(g, L, U, gbuf, gcs, fb, x3[0], x3[1], x3[2], w, bad);
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c][o] = w[c];
        }
        double w[NC], u[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            // pairwise means: along x first (bit 0), then y, then z
#pragma unroll
            for (int k = 0; k < NDIM; ++k)
#pragma unroll
                for (int i = 0; i < (K >> (k + 1)); ++i) v[c][i] = 0.5 * (v[c][2 * i] + v[c][2 * i + 1]);
            w[c] = v[c][0];
        }
        prim_to_cons_cell<NDIM>(g.gamma, w, u);
        const long long o = (long long)t.slot * NC * gcs + (long long)layer * face + r;
#pragma unroll
        for (int c = 0; c < NC; ++c) gbuf[o + c * gcs] = u[c];
    }
    if (bad) atomicOr(&ctrl->flags, FLAG_NONPHYSICAL);
}

// Prolongation onto the two ghost layers of a fine block's side that faces a
// coarser block: the coarse cell's value plus, per axis, a quarter of its
// minmod-limited difference (eq. minmod), signed by the side of the coarse
// centre the ghost's centre lies on; the coarse block's own ghosts (same
// level, boundary rule, restricted slots) complete its stencil.  Primitive
// variables; stored as conserved values.  blockIdx.x: the slot; one thread
// per ghost.
template <int NDIM>
__global__ __launch_bounds__(64) void smr_prolong_kernel(Geo g, const double* __restrict__ U,
                                                          const int* __restrict__ side, double* __restrict__ gbuf,
                                                          long long gcs, const GhostTask* __restrict__ tasks,
                                                          Ctrl* ctrl) {
    constexpr int NC = NDIM + 2;
    const GhostTask t = tasks[blockIdx.x];
    int lo, hi;
    transverse(t.ax, lo, hi);
    const int gn[3] = {g.n[0], g.n[1], g.n[2]};
    const int nlo = at3(gn, lo), nhi = at3(gn, hi), face = nlo * nhi;
    const int cblk = t.src[0];
    const Links L = table_links(side, cblk);
    bool bad = false;
    const int q = blockIdx.y * blockDim.x + threadIdx.x;
    if (q < 2 * face) {
        const int layer = q / face, r = q - layer * face;
        int ci[3] = {0, 0, 0};
        double sg[3] = {0.0, 0.0, 0.0};
        const int tl = r % nlo, th = r / nlo;
#pragma unroll
        for (int k = 0; k < NDIM; ++k) {
            const int ax = active_axis<NDIM>(k);
            if (ax == t.ax) {
                // the coarse cell next to the face; the ghost's side of its centre
                ci[ax] = t.s ? 0 : g.n[ax] - 1;
                sg[ax] = t.s ? (layer == 0 ? -1.0 : 1.0) : (layer == 0 ? 1.0 : -1.0);
            } else {
                const int p = t.child[ax] * g.n[ax] + (ax == lo ? tl : th);  // fine index from the parent's origin
                ci[ax] = p >> 1;
                sg[ax] = (p & 1) ? 1.0 : -1.0;
            }
        }
        double wc[NC], acc[NC];
        smr_prim<NDIM>(g, L, U, gbuf, gcs, cblk, ci[0], ci[1], ci[2], wc, bad);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = wc[c];
#pragma unroll
        for (int k = 0; k < NDIM; ++k) {
            const int ax = active_axis<NDIM>(k);
            int a3[3] = {ci[0], ci[1], ci[2]}, b3[3] = {ci[0], ci[1], ci[2]};
            a3[ax] -= 1;
            b3[ax] += 1;
            double wl[NC], wh[NC];
            smr_prim<NDIM>(g, L, U, gbuf, gcs, cblk, a3[0], a3[1], a3[2], wl, bad);
            smr_prim<NDIM>(g, L, U, gbuf, gcs, cblk, b3[0], b3[1], b3[2], wh, bad);
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = acc[c] + (0.25 * sg[ax]) * minmod(wc[c] - wl[c], wh[c] - wc[c]);
        }
        double u[NC];
        prim_to_cons_cell<NDIM>(g.gamma, acc, u);
        const long long o = (long long)t.slot * NC * gcs + (long long)layer * face + r;
#pragma unroll
        for (int c = 0; c < NC; ++c) gbuf[o + c * gcs] = u[c];
    }
    if (bad) atomicOr(&ctrl->flags, FLAG_NONPHYSICAL);
}

// Flux correction at a level jump of kernel axis AX, for coarse face r of
// restriction slot t: the coarse cell next to the face is to get
// factor * lam * (F_coarse - mean of the fine fluxes) (sign by side), so that
// its update uses the fine fluxes' mean in place of its own.  The fluxes are
// recomputed from the same stage input, ghosts and operations as in the
// stage kernel, so F_coarse cancels exactly.  The correction goes to
// dbuf[idx][comp][r]; smr_apply_kernel adds it.
template <int NDIM, typename R, bool FIRST, int AX>
__device__ __forceinline__ void reflux_face(const Geo& g0, const Geo& g1, const double* __restrict__ in,
                                            double* __restrict__ dbuf, double factor, double dt,
                                            const int* __restrict__ side, const double* __restrict__ gbuf,
                                            long long gcs, const GhostTask& t, int idx, int r, bool& bad) {
    constexpr int NC = NDIM + 2;
    constexpr int NT = NDIM - 1;
    // the coarse block's cell width: level 0's times 2^-lev (exact)
    const double lam = dt / __builtin_ldexp(g0.dx[AX], -t.lev);
    const Gas<R> gr = make_gas<R>(g0.gamma);
    const double gm1 = g0.gamma - 1.0;
    int lo, hi;
    transverse(AX, lo, hi);
    const int nlo = g0.n[lo], nhi = g0.n[hi], face = nlo * nhi;
    if (r >= face) return;
    const int n = g0.n[AX];
    const Links Lc = table_links(side, t.leaf);
    const int tl = r % nlo, th = r / nlo;
    int x3[3] = {0, 0, 0};
    x3[lo] = tl;
    x3[hi] = th;
    // the coarse face flux from the four coarse cells across it
    R w[4][NC];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int c3[3] = {x3[0], x3[1], x3[2]};
        c3[AX] = t.s ? n - 2 + j : -2 + j;
        double u[NC];
        int vax, vm;
        smr_cell<NC>(g0, Lc, in, gbuf, gcs, t.leaf, c3[0], c3[1], c3[2], u, vax, vm);
        in_to_w<NDIM, R, false>(gm1, u, vax, vm, w[j], bad);
    }
    R Fc[NC];
    face_flux<NDIM, AX, R, FIRST>(gr, w[0], w[1], w[2], w[3], Fc);
    // the fine fluxes through it, by transverse child offsets
    // pairwise means as the fluxes arrive (offsets 0, 1 -> a; 2, 3 -> b),
    // the same operations as a tree of pairwise means
    double fa[NC], fb2[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) fa[c] = fb2[c] = 0.0;
    // not unrolled: one fine face's stencil and Riemann solve live at a time
#pragma unroll 1
    for (int o = 0; o < (1 << NT); ++o) {
        int f3[3] = {0, 0, 0};
        int cb[3] = {0, 0, 0};
        int bit = 0;
#pragma unroll
        for (int k = 0; k < NDIM; ++k) {
            const int ax = active_axis<NDIM>(k);
            if (ax == AX) continue;
            const int p = 2 * x3[ax] + ((o >> bit) & 1);
            ++bit;
            cb[ax] = p / g1.n[ax];
            f3[ax] = p - cb[ax] * g1.n[ax];
        }
        const int fb = at4(t.src, cb[lo] + 2 * cb[hi]);
        const Links Lf = table_links(side, fb);
        R v[4][NC];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int c3[3] = {f3[0], f3[1], f3[2]};
            c3[AX] = t.s ? -2 + j : g1.n[AX] - 2 + j;
            double u[NC];
            int vax, vm;
            smr_cell<NC>(g1, Lf, in, gbuf, gcs, fb, c3[0], c3[1], c3[2], u, vax, vm);
            in_to_w<NDIM, R, false>(gm1, u, vax, vm, v[j], bad);
        }
        R F[NC];
        face_flux<NDIM, AX, R, FIRST>(gr, v[0], v[1], v[2], v[3], F);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double f = (double)F[c];
            if (o == 0) fa[c] = f;
            else if (o == 1) fa[c] = 0.5 * (fa[c] + f);
            else if (o == 2) fb2[c] = f;
            else fb2[c] = 0.5 * (fb2[c] + f);
        }
    }
    const long long fs = gcs / 2;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double mean = NT == 2 ? 0.5 * (fa[c] + fb2[c]) : fa[c];
        const double d = t.s ? ((double)Fc[c] - mean) : (mean - (double)Fc[c]);
        dbuf[((long long)idx * NC + c) * fs + r] = factor * (lam * d);
    }
}

// The corrections of every restriction slot, one launch for all axes:
// blockIdx.x the slot (in slot order), one thread per coarse face.
// FIRST: the fluxes of piecewise-constant states (the van Leer predictor).
template <int NDIM, typename R, bool FIRST>
__global__ __launch_bounds__(64) void smr_reflux_kernel(Geo g0, Geo g1, const double* __restrict__ in,
                                                         double* __restrict__ dbuf, double factor,
                                                         int use_device_dt, double dt_host,
                                                         const int* __restrict__ side,
                                                         const double* __restrict__ gbuf, long long gcs,
                                                         const GhostTask* __restrict__ tasks, Ctrl* ctrl) {
    if (use_device_dt && ctrl->done) return;  // uniform over the grid
    const double dt = use_device_dt ? device_dt(ctrl) : dt_host;
    const GhostTask t = tasks[blockIdx.x];
    const int r = blockIdx.y * blockDim.x + threadIdx.x;
    bool bad = false;
    if (t.ax == 0) {
        reflux_face<NDIM, R, FIRST, 0>(g0, g1, in, dbuf, factor, dt, side, gbuf, gcs, t, blockIdx.x, r, bad);
    } else if (t.ax == 1) {
        if constexpr (NDIM == 3)
            reflux_face<NDIM, R, FIRST, 1>(g0, g1, in, dbuf, factor, dt, side, gbuf, gcs, t, blockIdx.x, r, bad);
    } else {
        if constexpr (NDIM >= 2)
            reflux_face<NDIM, R, FIRST, 2>(g0, g1, in, dbuf, factor, dt, side, gbuf, gcs, t, blockIdx.x, r, bad);
    }
    if (bad) atomicOr(&ctrl->flags, FLAG_NONPHYSICAL);
}

// Add the corrections of the restriction slots idx0 .. idx0 + gridDim.x - 1
// (one kernel axis) to their coarse cells: out += dbuf.  One launch per axis,
// in axis order, so a coarse cell next to jumps on two axes is corrected in a
// fixed order.
template <int NDIM>
__global__ __launch_bounds__(64) void smr_apply_kernel(Geo g0, double* __restrict__ out,
                                                        const double* __restrict__ dbuf, long long gcs,
                                                        const GhostTask* __restrict__ tasks, int idx0,
                                                        int use_device_dt, Ctrl* ctrl) {
    constexpr int NC = NDIM + 2;
    if (use_device_dt && ctrl->done) return;  // uniform over the grid
    const GhostTask t = tasks[blockIdx.x];
    int lo, hi;
    transverse(t.ax, lo, hi);
    const int nlo = g0.n[lo], face = nlo * g0.n[hi];
    const int r = blockIdx.y * blockDim.x + threadIdx.x;
    if (r >= face) return;
    int c3[3] = {0, 0, 0};
    c3[lo] = r % nlo;
    c3[hi] = r / nlo;
    c3[t.ax] = t.s ? g0.n[t.ax] - 1 : 0;
    const long long N = g0.ncells;
    const long long cell = (long long)t.leaf * NC * N + ((long long)c3[2] * g0.n[1] + c3[1]) * g0.n[0] + c3[0];
    const long long fs = gcs / 2;
#pragma unroll
    for (int c = 0; c < NC; ++c) out[cell + c * N] = out[cell + c * N] + dbuf[((long long)(idx0 + blockIdx.x) * NC + c) * fs + r];
}

// Mesh layout [comp][k][j][i] <-> block layout; q runs over the mesh cells.
__global__ __launch_bounds__(256) void relayout_kernel(Geo g, int nc, double* __restrict__ mesh,
                                                       double* __restrict__ blk, int to_blocks) {
    const long long m0 = (long long)g.n[0] * g.blocks[0], m1 = (long long)g.n[1] * g.blocks[1];
    const long long total = m0 * m1 * ((long long)g.n[2] * g.blocks[2]);
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(q % m0);
        const int y = (int)((q / m0) % m1);
        const int z = (int)(q / (m0 * m1));
        const int b = x / g.n[0] + g.blocks[0] * (y / g.n[1] + g.blocks[1] * (z / g.n[2]));
        const long long cell = ((long long)(z % g.n[2]) * g.n[1] + y % g.n[1]) * g.n[0] + x % g.n[0];
        const long long bo = (long long)b * nc * g.ncells + cell;
        for (int c = 0; c < nc; ++c) {
            if (to_blocks)
                blk[bo + c * g.ncells] = mesh[c * total + q];
            else
                mesh[c * total + q] = blk[bo + c * g.ncells];
        }
    }
}

template <typename R, int NT>
__global__ __launch_bounds__(256) void riemann_kernel(double gamma, long long n,
                                                      const double* __restrict__ WL,
                                                      const double* __restrict__ WR,
                                                      double* __restrict__ F) {
    constexpr int NC = NT + 3;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        R L[NC], Rr[NC], Fo[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            L[c] = (R)WL[c * n + i];
            Rr[c] = (R)WR[c * n + i];
        }
        hllc<R, NT>(make_gas<R>(gamma), L, Rr, Fo);
#pragma unroll
        for (int c = 0; c < NC; ++c) F[c * n + i] = (double)Fo[c];
    }
}

int grid_for(long long work, int block, int cap) {
    long long gb = (work + block - 1) / block;
    if (gb < 1) gb = 1;
    return (int)(gb < cap ? gb : cap);
}

// Launch context: a single mesh (args) or a batch group (descriptor table);
// with rec, a single-mesh launch is described there instead of enqueued.
struct LaunchCtx {
    const StageArgs* a;
    const MeshDesc* d;
    const int2* blk;
    int nblk;
    StageLaunch* rec;
};

// Work-groups of this stage kernel resident on the whole device at once
// (0 if the runtime cannot tell).
template <int NDIM, typename R, int MODE, int TX, int TY>
int stage_slots() {
    static const int slots = [] {
        int dev = 0, cus = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void*>(&stage_kernel<NDIM, R, MODE, TX, TY>), TX * TY, 0) !=
            hipSuccess)
            return 0;
        return cus * nb;
    }();
    return slots;
}

template <int NDIM, typename R, int MODE, int TX, int TY>
hipError_t launch_stage_t(const LaunchCtx& L, hipStream_t s) {
    if (L.a) {
        StageArgs a = *L.a;
        if (a.kz == 0) {
            // automatic chunk length: one round of resident work-groups
            // covers the blocks whose work runs at once (this launch's, or
            // those of the launches on the other streams as well), so no
            // work-group waits for a second round
            const int slots = stage_slots<NDIM, R, MODE, TX, TY>();
            const long long cols = (long long)a.tiles_x * a.tiles_y * (a.conc > a.nblk ? a.conc : a.nblk);
            const int n2 = a.geo.n[2];
            long long kz = slots > 0 ? (n2 * cols + slots - 1) / slots : 32;
            kz = kz < kMinAutoKz ? kMinAutoKz : (kz > kMaxAutoKz ? kMaxAutoKz : kz);
            a.kz = kz > n2 ? n2 : (int)kz;
            a.chunks_z = (n2 + a.kz - 1) / a.kz;
        }
        const long long nb = (long long)a.tiles_x * a.tiles_y * a.chunks_z * a.nblk;
        if (a.nblk < 1 || nb > 0x7fffffffll) return hipErrorInvalidValue;
        if (L.rec) {
            L.rec->func = reinterpret_cast<const void*>(&stage_kernel<NDIM, R, MODE, TX, TY>);
            L.rec->grid = dim3((unsigned)nb);
            L.rec->block = dim3(TX * TY);
            L.rec->args = a;
            return hipSuccess;
        }
        hipLaunchKernelGGL((stage_kernel<NDIM, R, MODE, TX, TY>), dim3((unsigned)nb), dim3(TX * TY), 0, s, a);
    } else if constexpr (MODE == MODE_RHS || MODE == MODE_VL2_PRED_C || MODE == MODE_VL2_CORR_C) {
        return hipErrorInvalidValue;  // not a batch member's stage
    } else {
        if (L.nblk <= 0) return hipSuccess;
        hipLaunchKernelGGL((stage_kernel_batch<NDIM, R, MODE, TX, TY>), dim3(L.nblk), dim3(TX * TY), 0, s,
                           L.d, L.blk);
    }
    return hipGetLastError();
}

// The van Leer stages of a refined mesh (conserved predictor) take one tile
// each: a refined handle is not autotuned.
template <int NDIM, typename R, int MODE>
hipError_t launch_stage_refined(const Tile& t, const LaunchCtx& L, hipStream_t s) {
    if (!L.a) return hipErrorInvalidValue;
    if constexpr (NDIM == 3) {
        if (t.tx == 32 && t.ty == 8) return launch_stage_t<NDIM, R, MODE, 32, 8>(L, s);
    } else {
        if (t.tx == 64 && t.ty == 1) return launch_stage_t<NDIM, R, MODE, 64, 1>(L, s);
    }
    return hipErrorInvalidValue;
}

template <int NDIM, typename R, int MODE>
hipError_t launch_stage_tile(const Tile& t, const LaunchCtx& L, hipStream_t s) {
    if constexpr (NDIM == 3) {
        if (t.tx == 32 && t.ty == 8) return launch_stage_t<NDIM, R, MODE, 32, 8>(L, s);
        if (t.tx == 64 && t.ty == 8) return launch_stage_t<NDIM, R, MODE, 64, 8>(L, s);
        if (t.tx == 16 && t.ty == 16) return launch_stage_t<NDIM, R, MODE, 16, 16>(L, s);
        if (t.tx == 32 && t.ty == 16) return launch_stage_t<NDIM, R, MODE, 32, 16>(L, s);
        return hipErrorInvalidValue;
    } else {
        if (t.ty != 1) return hipErrorInvalidValue;
        if (t.tx == 64) return launch_stage_t<NDIM, R, MODE, 64, 1>(L, s);
        if (t.tx == 128) return launch_stage_t<NDIM, R, MODE, 128, 1>(L, s);
        if (t.tx == 256) return launch_stage_t<NDIM, R, MODE, 256, 1>(L, s);
        return hipErrorInvalidValue;
    }
}

template <int NDIM, typename R>
hipError_t launch_stage_mode(int mode, const Tile& t, const LaunchCtx& L, hipStream_t s) {
    switch (mode) {
        case MODE_RHS:
            if (!L.a) return hipErrorInvalidValue;
            return launch_stage_tile<NDIM, R, MODE_RHS>(t, L, s);
        case MODE_STAGE1: return launch_stage_tile<NDIM, R, MODE_STAGE1>(t, L, s);
        case MODE_STAGE2: return launch_stage_tile<NDIM, R, MODE_STAGE2>(t, L, s);
        case MODE_VL2_PRED: return launch_stage_tile<NDIM, R, MODE_VL2_PRED>(t, L, s);
        case MODE_VL2_CORR: return launch_stage_tile<NDIM, R, MODE_VL2_CORR>(t, L, s);
        case MODE_VL2_PRED_C: return launch_stage_refined<NDIM, R, MODE_VL2_PRED_C>(t, L, s);
        case MODE_VL2_CORR_C: return launch_stage_refined<NDIM, R, MODE_VL2_CORR_C>(t, L, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NDIM>
hipError_t launch_stage_prec(int precision, int mode, const Tile& t, const LaunchCtx& L, hipStream_t s) {
    if (precision == 0) return launch_stage_mode<NDIM, double>(mode, t, L, s);
    return launch_stage_mode<NDIM, float>(mode, t, L, s);
}

hipError_t launch_any(int ndim, int precision, int mode, const Tile& t, const LaunchCtx& L,
                      hipStream_t s) {
    switch (ndim) {
        case 1: return launch_stage_prec<1>(precision, mode, t, L, s);
        case 2: return launch_stage_prec<2>(precision, mode, t, L, s);
        case 3: return launch_stage_prec<3>(precision, mode, t, L, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

Tile default_tile(const Geo& g, int precision, int mode) {
    Tile t;
    if (mode == MODE_VL2_PRED_C || mode == MODE_VL2_CORR_C) {
        // the one tile of the refined mesh's van Leer stages
        t.tx = g.ndim == 3 ? 32 : 64;
        t.ty = g.ndim == 3 ? 8 : 1;
    } else if (g.ndim == 3) {
        // From a sweep at 256^3: 32 x 16 halves the share of halo cells and
        // extra faces where the occupancy allows it; 32 x 8 where a larger
        // work-group would cost occupancy (the mixed Heun stages beside their
        // input rings; the FP64 kernels other than the double-buffered Heun
        // stage 2).
        const bool narrow = precision == 1 ? (mode == MODE_STAGE2 || mode == MODE_STAGE1) : mode != MODE_STAGE2;
        t.tx = 32;
        t.ty = narrow ? 8 : 16;
    } else if (g.ndim == 2) {
        t.tx = g.n[0] >= 256 ? 256 : (g.n[0] >= 128 ? 128 : 64);
        t.ty = 1;
    } else {
        t.tx = 64;
        t.ty = 1;
    }
    // chunk length chosen at launch (one round of resident work-groups)
    t.kz = g.ndim == 1 ? 1 : 0;
    return t;
}

bool tile_supported(int ndim, const Tile& t) {
    if (t.kz < 0 || (t.kz == 0 && ndim == 1)) return false;
    if (ndim == 3)
        return (t.tx == 32 && t.ty == 8) || (t.tx == 64 && t.ty == 8) || (t.tx == 16 && t.ty == 16) ||
               (t.tx == 32 && t.ty == 16);
    return t.ty == 1 && (t.tx == 64 || t.tx == 128 || t.tx == 256);
}

int tile_candidates(const Geo& g, Tile* out, int max) {
    static const int shapes3[4][2] = {{32, 8}, {64, 8}, {16, 16}, {32, 16}};
    static const int shapes12[4][2] = {{64, 1}, {128, 1}, {256, 1}, {0, 0}};
    static const int kzs[5] = {0, 8, 16, 32, 64};  // 0: automatic
    const int(*shapes)[2] = g.ndim == 3 ? shapes3 : shapes12;
    int n = 0;
    for (int s = 0; s < (g.ndim == 3 ? 4 : 3); ++s) {
        // in 1-D and 2-D a row wider than twice the mesh only idles threads
        if (g.ndim < 3 && s > 0 && shapes[s][0] >= 2 * g.n[0]) continue;
        for (int q = 0; q < (g.ndim == 1 ? 1 : 5); ++q) {
            const int kz = g.ndim == 1 ? 1 : kzs[q];
            if (q > 1 && kzs[q - 1] >= g.n[2]) break;  // same chunks as the previous kz
            if (n < max) {
                out[n].tx = shapes[s][0];
                out[n].ty = shapes[s][1];
                out[n].kz = kz;
            }
            ++n;
        }
    }
    return n;
}

// Chunk length for tile t: t.kz, or with t.kz == 0 about 2048 work-groups in
// chunks of 16..64 planes (shorter chunks re-read more ghost planes).
int batch_kz(const Geo& g, const Tile& t) {
    if (t.kz > 0) return t.kz;
    if (g.ndim == 1) return 1;
    const long long cols = (long long)((g.n[0] + t.tx - 1) / t.tx) * ((g.n[1] + t.ty - 1) / t.ty);
    long long kz = (g.n[2] * cols + 2047) / 2048;
    return (int)(kz < 16 ? 16 : (kz > 64 ? 64 : kz));
}

void plan_tiles(const Geo& g, const Tile& t, int& tiles_x, int& tiles_y, int& chunks_z, int& kz) {
    tiles_x = (g.n[0] + t.tx - 1) / t.tx;
    tiles_y = (g.n[1] + t.ty - 1) / t.ty;
    kz = batch_kz(g, t);
    kz = kz > g.n[2] ? g.n[2] : kz;
    chunks_z = (g.n[2] + kz - 1) / kz;
}

hipError_t launch_stage(int precision, int mode, const Tile& t, StageArgs a, hipStream_t s) {
    plan_tiles(a.geo, t, a.tiles_x, a.tiles_y, a.chunks_z, a.kz);
    if (t.kz == 0 && a.geo.ndim > 1) a.kz = 0;  // resolved per kernel at launch
    LaunchCtx L{&a, nullptr, nullptr, 0, nullptr};
    return launch_any(a.geo.ndim, precision, mode, t, L, s);
}

hipError_t plan_stage_launch(int precision, int mode, const Tile& t, StageArgs a, StageLaunch* out) {
    if (!out) return hipErrorInvalidValue;
    plan_tiles(a.geo, t, a.tiles_x, a.tiles_y, a.chunks_z, a.kz);
    if (t.kz == 0 && a.geo.ndim > 1) a.kz = 0;
    LaunchCtx L{&a, nullptr, nullptr, 0, out};
    return launch_any(a.geo.ndim, precision, mode, t, L, nullptr);
}

hipError_t launch_stage_batch(int ndim, int precision, int mode, const Tile& tile, const MeshDesc* d,
                              const int2* blk, int nblk, hipStream_t s) {
    if (mode == MODE_RHS) return hipErrorInvalidValue;
    LaunchCtx L{nullptr, d, blk, nblk, nullptr};
    return launch_any(ndim, precision, mode, tile, L, s);
}

hipError_t launch_status_gather(const MeshDesc* d, int n, unsigned long long* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(status_gather_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, n, out);
    return hipGetLastError();
}

hipError_t launch_ctrl_batch(const MeshDesc* d, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(ctrl_batch_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d, n);
    return hipGetLastError();
}

hipError_t launch_dt_levels(const Geo& g0, const LevelStarts& starts, int nblk, const double* U, Ctrl* ctrl,
                            int skip_done, hipStream_t s) {
    if (nblk < 1) return hipSuccess;
    const dim3 grid(grid_for(g0.ncells, 256, (2048 + nblk - 1) / nblk), nblk);
    switch (g0.ndim) {
        case 1: hipLaunchKernelGGL(dt_kernel<1>, grid, dim3(256), 0, s, g0, starts, U, ctrl, skip_done); break;
        case 2: hipLaunchKernelGGL(dt_kernel<2>, grid, dim3(256), 0, s, g0, starts, U, ctrl, skip_done); break;
        case 3: hipLaunchKernelGGL(dt_kernel<3>, grid, dim3(256), 0, s, g0, starts, U, ctrl, skip_done); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dt(const Geo& g, const double* U, Ctrl* ctrl, hipStream_t s) {
    LevelStarts none;
    for (int L = 0; L < kMaxLevels - 1; ++L) none.s[L] = geo_nblk(g);
    return launch_dt_levels(g, none, geo_nblk(g), U, ctrl, 0, s);
}

hipError_t launch_ctrl(Ctrl* c, int op, double a0, double a1, double cfl, hipStream_t s) {
    hipLaunchKernelGGL(ctrl_kernel, dim3(1), dim3(64), 0, s, c, op, a0, a1, cfl);
    return hipGetLastError();
}

namespace {
// Partials pass then the tree over them; sums or out as in totals_pass2.
hipError_t totals_launch(const Geo& g, const double* U, double* parts, int nparts, double* sums, double* out,
                         double dV, hipStream_t s) {
    // nparts partials shared out over the blocks (at least one each)
    const int nblk = geo_nblk(g);
    if (nblk > nparts) return hipErrorInvalidValue;
    const int nb = grid_for(g.ncells, 256, nparts / nblk);
    const dim3 grid(nb, nblk);
    const int np = nb * nblk;
    const int NC = g.ndim + 2;
    switch (NC) {
        case 3:
            hipLaunchKernelGGL(totals_pass1<3>, grid, dim3(256), 0, s, g.ncells, U, parts);
            hipLaunchKernelGGL(totals_pass2<3>, dim3(1), dim3(256), 0, s, np, parts, sums, out, dV);
            break;
        case 4:
            hipLaunchKernelGGL(totals_pass1<4>, grid, dim3(256), 0, s, g.ncells, U, parts);
            hipLaunchKernelGGL(totals_pass2<4>, dim3(1), dim3(256), 0, s, np, parts, sums, out, dV);
            break;
        case 5:
            hipLaunchKernelGGL(totals_pass1<5>, grid, dim3(256), 0, s, g.ncells, U, parts);
            hipLaunchKernelGGL(totals_pass2<5>, dim3(1), dim3(256), 0, s, np, parts, sums, out, dV);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_totals(const Geo& g, const double* U, double* parts, int nparts, Ctrl* ctrl,
                         hipStream_t s) {
    return totals_launch(g, U, parts, nparts, ctrl->sums, nullptr, 0.0, s);
}

hipError_t launch_totals_out(const Geo& g, const double* U, double* parts, int nparts, double* out, double dV,
                             hipStream_t s) {
    if (!out) return hipErrorInvalidValue;
    return totals_launch(g, U, parts, nparts, nullptr, out, dV, s);
}

hipError_t launch_prim_to_cons(const Geo& g, const double* W, double* U, hipStream_t s) {
    const int nblk = geo_nblk(g);
    const dim3 grid(grid_for(g.ncells, 256, (4096 + nblk - 1) / nblk), nblk);
    switch (g.ndim) {
        case 1: hipLaunchKernelGGL(prim_to_cons_kernel<1>, grid, dim3(256), 0, s, g, W, U); break;
        case 2: hipLaunchKernelGGL(prim_to_cons_kernel<2>, grid, dim3(256), 0, s, g, W, U); break;
        case 3: hipLaunchKernelGGL(prim_to_cons_kernel<3>, grid, dim3(256), 0, s, g, W, U); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_relayout(const Geo& g, double* mesh, double* blk, int to_blocks, hipStream_t s) {
    const int nb = grid_for(g.ncells * geo_nblk(g), 256, 4096);
    hipLaunchKernelGGL(relayout_kernel, dim3(nb), dim3(256), 0, s, g, g.ndim + 2, mesh, blk, to_blocks);
    return hipGetLastError();
}

hipError_t launch_padded_prim(const Geo& g, int precision, const double* U, double* Wp, Ctrl* ctrl,
                              hipStream_t s) {
    const int nb = grid_for(g.ncells * geo_nblk(g) * 2 + 4096, 256, 4096);
#define PP(ND, RT) hipLaunchKernelGGL((padded_prim_kernel<ND, RT>), dim3(nb), dim3(256), 0, s, g, U, Wp, ctrl)
    if (precision == 0) {
        switch (g.ndim) {
            case 1: PP(1, double); break;
            case 2: PP(2, double); break;
            case 3: PP(3, double); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (g.ndim) {
            case 1: PP(1, float); break;
            case 2: PP(2, float); break;
            case 3: PP(3, float); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef PP
    return hipGetLastError();
}

hipError_t launch_smr_restrict(const Geo& g, const double* U, const int* side, double* gbuf, long long gcs,
                               const GhostTask* tasks, int n, Ctrl* ctrl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // one thread per ghost of the largest slot (gcs = its two layers)
    const dim3 grid(n, (unsigned)((gcs + 63) / 64));
    switch (g.ndim) {
        case 1: hipLaunchKernelGGL(smr_restrict_kernel<1>, grid, dim3(64), 0, s, g, U, side, gbuf, gcs, tasks, ctrl); break;
        case 2: hipLaunchKernelGGL(smr_restrict_kernel<2>, grid, dim3(64), 0, s, g, U, side, gbuf, gcs, tasks, ctrl); break;
        case 3: hipLaunchKernelGGL(smr_restrict_kernel<3>, grid, dim3(64), 0, s, g, U, side, gbuf, gcs, tasks, ctrl); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_smr_prolong(const Geo& g, const double* U, const int* side, double* gbuf, long long gcs,
                              const GhostTask* tasks, int n, Ctrl* ctrl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(n, (unsigned)((gcs + 63) / 64));
    switch (g.ndim) {
        case 1: hipLaunchKernelGGL(smr_prolong_kernel<1>, grid, dim3(64), 0, s, g, U, side, gbuf, gcs, tasks, ctrl); break;
        case 2: hipLaunchKernelGGL(smr_prolong_kernel<2>, grid, dim3(64), 0, s, g, U, side, gbuf, gcs, tasks, ctrl); break;
        case 3: hipLaunchKernelGGL(smr_prolong_kernel<3>, grid, dim3(64), 0, s, g, U, side, gbuf, gcs, tasks, ctrl); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_smr_reflux(int precision, int first, const Geo& g0, const Geo& g1, const double* in,
                             double* dbuf, double factor, int use_device_dt, double dt_host, const int* side,
                             const double* gbuf, long long gcs, const GhostTask* tasks, int n, Ctrl* ctrl,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(n, (unsigned)((gcs / 2 + 63) / 64));  // one thread per face of the largest side
#define RF(ND, RT, FO)                                                                                          \
    hipLaunchKernelGGL((smr_reflux_kernel<ND, RT, FO>), grid, dim3(64), 0, s, g0, g1, in, dbuf, factor, \
                       use_device_dt, dt_host, side, gbuf, gcs, tasks, ctrl)
    switch ((g0.ndim * 2 + (precision == 0 ? 0 : 1)) * 2 + (first ? 1 : 0)) {
        case 4: RF(1, double, false); break;
        case 5: RF(1, double, true); break;
        case 6: RF(1, float, false); break;
        case 7: RF(1, float, true); break;
        case 8: RF(2, double, false); break;
        case 9: RF(2, double, true); break;
        case 10: RF(2, float, false); break;
        case 11: RF(2, float, true); break;
        case 12: RF(3, double, false); break;
        case 13: RF(3, double, true); break;
        case 14: RF(3, float, false); break;
        case 15: RF(3, float, true); break;
        default: return hipErrorInvalidValue;
    }
#undef RF
    return hipGetLastError();
}

hipError_t launch_smr_apply(const Geo& g0, double* out, const double* dbuf, long long gcs, const GhostTask* tasks,
                            int idx0, int n, int use_device_dt, Ctrl* ctrl, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid(n, (unsigned)((gcs / 2 + 63) / 64));
#define AP(ND) hipLaunchKernelGGL((smr_apply_kernel<ND>), grid, dim3(64), 0, s, g0, out, dbuf, gcs, tasks, idx0, \
                                  use_device_dt, ctrl)
    switch (g0.ndim) {
        case 1: AP(1); break;
        case 2: AP(2); break;
        case 3: AP(3); break;
        default: return hipErrorInvalidValue;
    }
#undef AP
    return hipGetLastError();
}

hipError_t launch_riemann(int precision, int ntan, double gamma, long long n, const double* WL,
                          const double* WR, double* F, hipStream_t s) {
    const int nb = grid_for(n, 256, 4096);
#define RK(RT, NTAN) \
    hipLaunchKernelGGL((riemann_kernel<RT, NTAN>), dim3(nb), dim3(256), 0, s, gamma, n, WL, WR, F)
    if (precision == 0) {
        switch (ntan) {
            case 0: RK(double, 0); break;
            case 1: RK(double, 1); break;
            case 2: RK(double, 2); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (ntan) {
            case 0: RK(float, 0); break;
            case 1: RK(float, 1); break;
            case 2: RK(float, 2); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef RK
    return hipGetLastError();
}

}  // namespace hydro
