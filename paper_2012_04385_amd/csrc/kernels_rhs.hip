// kernels_rhs.hip -- gfx950 kernels of the per-block right-hand side and stage update.
//
// Flux (Sec. "Numerical Scheme"): one numerical flux per cell face from a Roe-type
// solver with fifth-order WENO-JS reconstruction of the characteristic fluxes.  Per
// characteristic field the eigenvalues of the two cells sharing the face decide: same
// sign -> upwind WENO5 of the characteristic flux; otherwise a local Lax-Friedrichs
// (Rusanov) split whose speed uses only those two cells, each half reconstructed by
// WENO5.  The characteristic projection uses the closed-form left eigenvectors of the
// Roe-averaged Jacobian (eq:StiffenedGas gives c^2 = (gamma-1)(H - |v|^2/2)).
//
// Work decomposition.  Plain path (k_flux): a thread walks one pencil of 16 cells along
// one axis with a six-cell register window, so each cell's primitives are computed once
// per pencil.  Batched path (k_rhs_update): one face per thread inside groups of z-planes,
// fluxes staged in LDS, fused with the stage update.  Each face flux is computed once per
// block on both paths.  Stencils are not contractions, so no MFMA is used here.
//
// Jump correction (algo:ComputeLoop, coarse cell adjustment): the boundary face fluxes of
// every leaf are stored; non-leaf blocks receive the area average of their children's
// (k_ff_restrict), and a coarse leaf next to a non-leaf same-level neighbour replaces its
// own boundary flux by that average.  With one global dt per step the correction is
// applied at every stage.
#include <algorithm>

#include "mrfv_internal.h"

namespace mrfv {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }

template <typename T>
struct Gas {
    T g, B, gm1;
};

// Cell state along the pencil, momentum rotated to (normal, t1, t2).
template <typename T>
struct CellState {
    T r, mn, mt1, mt2, E, p, c, ir, sr;
};

template <int DIR>
struct Axes {   // physical momentum component of the rotated (n, t1, t2) triple
    static constexpr int N1 = DIR == 0 ? 1 : (DIR == 1 ? 2 : 3);
    static constexpr int T1 = DIR == 0 ? 2 : (DIR == 1 ? 3 : 1);
    static constexpr int T2 = DIR == 0 ? 3 : (DIR == 1 ? 1 : 2);
    static constexpr int STRIDE = DIR == 0 ? 1 : (DIR == 1 ? NP : NP * NP);
};

template <typename T, int DIR>
__device__ __forceinline__ void load_state(const T *__restrict__ u, int idx, const Gas<T> &G,
                                           CellState<T> &s) {
    s.r = u[idx];
    s.mn = u[idx + Axes<DIR>::N1 * CELLS_P];
    s.mt1 = u[idx + Axes<DIR>::T1 * CELLS_P];
    s.mt2 = u[idx + Axes<DIR>::T2 * CELLS_P];
    s.E = u[idx + 4 * CELLS_P];
}

// Every multiply-add is an explicit fma: the compiler fuses per basic block, and this
// code is inlined after different load paths (per-lane sources, uniform base), which
// must all give bitwise the same state.
template <typename T>
__device__ __forceinline__ void derive_state(const Gas<T> &G, CellState<T> &s) {
    s.ir = rcp_(s.r);
    const T m2 = fma(s.mt2, s.mt2, fma(s.mt1, s.mt1, s.mn * s.mn));
    const T eint = fma((T)-0.5 * m2, s.ir, s.E);          // E - |m|^2 / (2 rho)
    s.p = fma(G.gm1, eint, -(G.g * G.B));
    s.c = sqrt_(G.g * (s.p + G.B) * s.ir);
    s.sr = sqrt_(s.r);
}

// WENO5-JS value at the right face of c from (a,b,c,d,e); linear weights 0.1/0.6/0.3,
// eps = 1e-6, power 2 (Jiang & Shu), written with the first differences
// w0 = b-a, u = c-b, v = d-c, w3 = e-d:
//   candidate k = c + r_k / 6 with r = (5u - 2 w0, u + 2v, 4v - w3),
//   smoothness beta_k = 13/12 (t_k^2 + 3/13 s_k^2) with t = (u - w0, v - u, w3 - v),
//   s = (t0 + 2u, u + v, t2 - 2v).
// alpha_k = d_k / (eps + beta_k)^2 is normalised with one reciprocal: the common factor
// prod_j (eps + beta_j)^2 (13/12)^-2 cancels, so the value is
//   c + sum_k d_k r_k prod_{j != k} e_j^2 / (6 sum_k d_k prod_{j != k} e_j^2)
// with e_k = 12/13 eps + t_k^2 + 3/13 s_k^2; with 10 d = (1, 6, 3) and the 6 taken into the
// numerator, the terms are (r0 / 6, r1, r2 / 2) over (1, 6, 3).  A constant stencil
// returns c exactly.
template <typename T>
__device__ __forceinline__ T weno5_combine(T e0, T e1, T e2, T h0, T h1, T h2, T c) {
    const T E0 = e0 * e0, E1 = e1 * e1, E2 = e2 * e2;
    const T E12 = E1 * E2, E02 = E0 * E2, E01 = E0 * E1;
    const T num = fma(E12, h0, fma(E02, h1, E01 * h2));
    const T den = fma((T)6, E02, fma((T)3, E01, E12));
    return fma(num, rcp_(den), c);
}

template <typename T>
__device__ __forceinline__ T weno5(T a, T b, T c, T d, T e) {
    const T w0 = b - a, u = c - b, v = d - c, w3 = e - d;
    const T t0 = u - w0, s0 = fma((T)2, u, t0);
    const T t1 = v - u, s1 = u + v;
    const T t2 = w3 - v, s2 = fma((T)-2, v, t2);
    const T eps = (T)(1e-6 * 12.0 / 13.0), k = (T)(3.0 / 13.0);
    const T e0 = fma(t0, t0, fma(s0 * k, s0, eps));
    const T e1 = fma(t1, t1, fma(s1 * k, s1, eps));
    const T e2 = fma(t2, t2, fma(s2 * k, s2, eps));
    const T h0 = fma((T)(5.0 / 6.0), u, (T)(-1.0 / 3.0) * w0);   // r0 / 6
    const T h1 = fma((T)2, v, u);                                  // r1
    const T h2 = fma((T)2, v, (T)-0.5 * w3);                       // r2 / 2
    T r = weno5_combine(e0, e1, e2, h0, h1, h2, c);
    if constexpr (sizeof(T) == 4) {
        // The fourth powers of the indicators leave the FP32 range once they pass ~1e9
        // (steep characteristic fluxes behind strong shocks, LLF splits): the weights are
        // homogeneous of degree zero in (e0, e1, e2), so such lanes evaluate them again
        // with the indicators scaled by their maximum.  Other lanes are unchanged.
        if (!isfinite(r)) {
            const T sc = rcp_(fmax(e0, fmax(e1, e2)));
            r = weno5_combine(e0 * sc, e1 * sc, e2 * sc, h0, h1, h2, c);
        }
    }
    return r;
}

// TENO5 (Fu, Hu & Adams 2016) at the right face of c: the three 3-cell candidates of
// WENO5 with the optimal weights (0.1, 0.6, 0.3), each kept (weight as is) or dropped
// (weight 0) by the cut-off test chi_k >= C_T with chi_k = gamma_k / sum_j gamma_j,
// gamma_k = (1 + tau5 / (beta_k + eps))^6, tau5 = |beta_0 - beta_2|, C_T = 1e-5.  The test
// is evaluated as (R_k / R_m)^6 >= C_T sum_j (R_j / R_m)^6 with R = 1 + tau5 / (beta + eps)
// and m the candidate with the smallest beta (largest R), which cannot overflow; eps is
// 1e-40 in FP64 and 1e-30 in FP32 (above the smallest normal float).
template <typename T>
__device__ __forceinline__ T teno5(T a, T b, T c, T d, T e) {
    const T w0 = b - a, u = c - b, v = d - c, w3 = e - d;
    const T t0 = u - w0, s0 = fma((T)2, u, t0);
    const T t1 = v - u, s1 = u + v;
    const T t2 = w3 - v, s2 = fma((T)-2, v, t2);
    const T k13 = (T)(13.0 / 12.0), eps = sizeof(T) == 8 ? (T)1e-40 : (T)1e-30;
    const T e0 = fma(k13 * t0, t0, fma((T)0.25 * s0, s0, eps));
    const T e1 = fma(k13 * t1, t1, fma((T)0.25 * s1, s1, eps));
    const T e2 = fma(k13 * t2, t2, fma((T)0.25 * s2, s2, eps));
    const T tau = fabs(e0 - e2);
    const T em = fmin(e0, fmin(e1, e2));
    const T fm = em * rcp_(em + tau);                 // 1 / R_m
    auto ratio6 = [&](T ek) {
        const T r = (ek + tau) * rcp_(ek) * fm;       // R_k / R_m in (0, 1]
        const T r2 = r * r;
        return r2 * r2 * r2;
    };
    const T g0 = ratio6(e0), g1 = ratio6(e1), g2 = ratio6(e2);
    const T cut = (T)1e-5 * ((g0 + g1) + g2);
    const T d0 = g0 >= cut ? (T)1 : (T)0, d1 = g1 >= cut ? (T)1 : (T)0, d2 = g2 >= cut ? (T)1 : (T)0;
    // sum_k d_k delta_k (q_k - c) / sum_k d_k delta_k with q_k - c = (r0, r1, r2) / 6
    const T h0 = fma((T)(5.0 / 6.0), u, (T)(-1.0 / 3.0) * w0);   // r0 / 6
    const T h1 = fma((T)2, v, u);                                  // r1
    const T h2 = fma((T)2, v, (T)-0.5 * w3);                       // r2 / 2
    const T num = fma(d0, h0, fma(d1, h1, d2 * h2));
    const T den = fma((T)6, d1, fma((T)3, d2, d0));
    return fma(num, rcp_(den), c);
}

// WENO-AO(5,3) (Balsara, Garain & Shu 2016) at the right face of c: the fifth-order value
// q5 and the three third-order candidates q_l, q_c, q_r combined as
//   (w4 / g4)(q5 - g1 q_l - g2 q_c - g3 q_r) + w1 q_l + w2 q_c + w3 q_r,
// linear weights g = ((1-gH)(1-gL)/2, (1-gH) gL, (1-gH)(1-gL)/2, gH), gH = gL = 0.85,
// normalised weights w_k ~ g_k / (eps + beta_k)^2 (eps = 1e-6), beta_1..3 the Jiang-Shu
// indicators and beta_4 that of the quartic through all five cells, in Legendre form:
//   beta_4 = (U1 + U3/10)^2 + 13/3 (U2 + 123/455 U4)^2 + 781/20 U3^2 + 1421461/2275 U4^2.
// Evaluated relative to c (every candidate minus c), so a constant stencil returns c.
template <typename T>
__device__ __forceinline__ T wao53(T a, T b, T c, T d, T e) {
    const T w0 = b - a, u = c - b, v = d - c, w3 = e - d;
    const T t0 = u - w0, s0 = fma((T)2, u, t0);
    const T t1 = v - u, s1 = u + v;
    const T t2 = w3 - v, s2 = fma((T)-2, v, t2);
    const T k13 = (T)(13.0 / 12.0), eps = (T)1e-6;
    const T b1 = fma(k13 * t0, t0, (T)0.25 * s0 * s0);
    const T b2 = fma(k13 * t1, t1, (T)0.25 * s1 * s1);
    const T b3 = fma(k13 * t2, t2, (T)0.25 * s2 * s2);
    const T U1 = ((T)11 * (a - e) + (T)82 * (d - b)) * (T)(1.0 / 120.0);
    const T U2 = ((T)-3 * (a + e) + (T)40 * (b + d) - (T)74 * c) * (T)(1.0 / 56.0);
    const T U3 = ((e - a) + (T)2 * (b - d)) * (T)(1.0 / 12.0);
    const T U4 = ((a + e) - (T)4 * (b + d) + (T)6 * c) * (T)(1.0 / 24.0);
    const T p1 = fma((T)0.1, U3, U1), p2 = fma((T)(123.0 / 455.0), U4, U2);
    const T b4 = fma(p1, p1, fma((T)(13.0 / 3.0) * p2, p2,
                                 fma((T)(781.0 / 20.0) * U3, U3, (T)(1421461.0 / 2275.0) * U4 * U4)));
    const T g1 = (T)(0.15 * 0.15 / 2.0), g2 = (T)(0.15 * 0.85), g3 = g1, g4 = (T)0.85;
    auto wt = [&](T g, T beta) {
        const T x = eps + beta;
        return g * rcp_(x * x);
    };
    const T wl = wt(g1, b1), wc = wt(g2, b2), wr = wt(g3, b3), wh = wt(g4, b4);
    const T ql = fma((T)(5.0 / 6.0), u, (T)(-1.0 / 3.0) * w0);            // q_l - c
    const T qc = fma((T)(1.0 / 3.0), v, (T)(1.0 / 6.0) * u);              // q_c - c
    const T qr = fma((T)(2.0 / 3.0), v, (T)(-1.0 / 6.0) * w3);            // q_r - c
    const T q5 = fma((T)0.1, ql, fma((T)0.6, qc, (T)0.3 * qr));           // q5 - c
    const T hi = q5 - fma(g1, ql, fma(g2, qc, g3 * qr));
    const T num = fma(wh * (T)(1.0 / 0.85), hi, fma(wl, ql, fma(wc, qc, wr * qr)));
    const T den = (wl + wc) + (wr + wh);
    return fma(num, rcp_(den), c);
}

// Flux kernels of Sec. "Numerical Scheme" (the weak-scaling combinations).
enum { SCH_ROE_WENO5 = 0, SCH_ROE_TENO5 = 1, SCH_LLF_WENO5 = 2, SCH_HLLC_WAO53 = 3 };
// Roe-WENO5 of the barotropic system of Tait's equation (plain path only)
constexpr int SCH_TAIT_ROE_WENO5 = 4;

// Reconstruction of the flux-splitting kernels at the right face of c.
template <int SCH, typename T>
__device__ __forceinline__ T recon(T a, T b, T c, T d, T e) {
    if constexpr (SCH == SCH_ROE_TENO5) return teno5(a, b, c, d, e);
    else return weno5(a, b, c, d, e);
}

// Characteristic flux of one field: upwind by the two face cells' eigenvalues, else LLF
// (always LLF for the LLF kernel).
template <int SCH, typename T>
__device__ __forceinline__ T char_flux(const T W[6], const T G[6], T lL, T lR) {
    if (SCH != SCH_LLF_WENO5) {
        if (lL > (T)0 && lR > (T)0) return recon<SCH>(G[0], G[1], G[2], G[3], G[4]);
        if (lL < (T)0 && lR < (T)0) return recon<SCH>(G[5], G[4], G[3], G[2], G[1]);
    }
    const T al = fmax(fabs(lL), fabs(lR));
    T gp[6], gm[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        gp[j] = (T)0.5 * (G[j] + al * W[j]);
        gm[j] = (T)0.5 * (G[j] - al * W[j]);
    }
    return recon<SCH>(gp[0], gp[1], gp[2], gp[3], gp[4]) + recon<SCH>(gm[5], gm[4], gm[3], gm[2], gm[1]);
}

// Same result with at most two WENO evaluations per wavefront: if any lane of the wave
// needs the LLF split, every lane evaluates W-(g+) + W+(g-) with g+ = g, g- = 0 for
// upwind-right lanes and g+ = 0, g- = g for upwind-left lanes (a WENO of zeros is exactly
// zero); otherwise one WENO with the input order picked per lane.  Equal to char_flux
// on upwind lanes and up to rounding on LLF lanes, but mixed waves no longer execute all
// three branches.
// The split is formed as g+ = cp G + ap W and g- = G - g+ with per-lane coefficients
// (cp, ap) = (1, 0) upwind-right, (0, 0) upwind-left, (1/2, a/2) LLF: g+ = (G + a W)/2
// rounded once (halving is exact), g- = (G - a W)/2 up to rounding, and exactly G, 0 on
// the upwind lanes.
template <int SCH, typename T>
__device__ __forceinline__ T char_flux_uniform(const T W[6], const T G[6], T lL, T lR) {
    const bool up = SCH != SCH_LLF_WENO5 && lL > (T)0 && lR > (T)0;
    const bool dn = SCH != SCH_LLF_WENO5 && lL < (T)0 && lR < (T)0;
    const bool llf = !(up || dn);
    if (SCH != SCH_LLF_WENO5 && !__any(llf)) {
        // the stencil in upwind order, selected per lane from scalar copies (a select
        // between elements of G itself becomes a dynamically indexed array)
        const T g0 = G[0], g1 = G[1], g2 = G[2], g3 = G[3], g4 = G[4], g5 = G[5];
        return recon<SCH>(up ? g0 : g5, up ? g1 : g4, up ? g2 : g3, up ? g3 : g2, up ? g4 : g1);
    }
    const T ha = (T)0.5 * fmax(fabs(lL), fabs(lR));
    const T cp = up ? (T)1 : (dn ? (T)0 : (T)0.5);
    const T ap = llf ? ha : (T)0;
    T gp[6], gm[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        gp[j] = fma(ap, W[j], cp * G[j]);
        gm[j] = G[j] - gp[j];
    }
    return recon<SCH>(gp[0], gp[1], gp[2], gp[3], gp[4]) + recon<SCH>(gm[5], gm[4], gm[3], gm[2], gm[1]);
}

// HLLC flux (Toro, Spruce & Speares 1994) between two rotated conservative states
// (rho, m_n, m_t1, m_t2, E); wave speeds S_L = min(u_L - c_L, u~ - c~), S_R = max(u_R + c_R,
// u~ + c~) from the Roe average of the two states.
template <typename T>
__device__ __forceinline__ void hllc(const T UL[5], const T UR[5], const Gas<T> &G, T F[5]) {
    const T irl = rcp_(UL[0]), irr = rcp_(UR[0]);
    const T ul = UL[1] * irl, ur = UR[1] * irr;
    const T pl = fma(G.gm1, fma((T)-0.5 * fma(UL[3], UL[3], fma(UL[2], UL[2], UL[1] * UL[1])), irl, UL[4]), -(G.g * G.B));
    const T pr = fma(G.gm1, fma((T)-0.5 * fma(UR[3], UR[3], fma(UR[2], UR[2], UR[1] * UR[1])), irr, UR[4]), -(G.g * G.B));
    const T cl = sqrt_(G.g * (pl + G.B) * irl), cr = sqrt_(G.g * (pr + G.B) * irr);
    const T sl = sqrt_(UL[0]), sr = sqrt_(UR[0]);
    const T iw = rcp_(sl + sr);
    const T ut = (sl * ul + sr * ur) * iw;
    const T vt = (sl * (UL[2] * irl) + sr * (UR[2] * irr)) * iw;
    const T wt = (sl * (UL[3] * irl) + sr * (UR[3] * irr)) * iw;
    const T Ht = (sl * ((UL[4] + pl) * irl) + sr * ((UR[4] + pr) * irr)) * iw;
    const T ct = sqrt_(G.gm1 * (Ht - (T)0.5 * (ut * ut + vt * vt + wt * wt)));
    const T SL = fmin(ul - cl, ut - ct), SR = fmax(ur + cr, ut + ct);
    const T ml = UL[0] * (SL - ul), mr = UR[0] * (SR - ur);
    const T Ss = (pr - pl + ul * ml - ur * mr) * rcp_(ml - mr);
    // side K: the physical flux, plus S_K (U*_K - U_K) when the face lies in the star region
    const bool left = SL >= (T)0 || Ss >= (T)0;
    const T *U = left ? UL : UR;
    const T ir = left ? irl : irr, un = left ? ul : ur, p = left ? pl : pr;
    const T S = left ? SL : SR, m = left ? ml : mr;
    const T Fk[5] = {U[1], fma(U[1], un, p), U[2] * un, U[3] * un, (U[4] + p) * un};
    const bool star = left ? SL < (T)0 : SR > (T)0;
    const T f = m * rcp_(S - Ss);
    const T Us[5] = {f, f * Ss, f * (U[2] * ir), f * (U[3] * ir),
                     f * fma(Ss - un, Ss + p * rcp_(m), U[4] * ir)};
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = star ? fma(S, Us[k] - U[k], Fk[k]) : Fk[k];
}

// Numerical flux through the face between window cells 2 and 3 (rotated components).
template <typename T, bool UNIFORM = false, int SCH = SCH_ROE_WENO5>
__device__ __forceinline__ void face_flux(const CellState<T> w[6], const Gas<T> &G, T F[5]) {
    const CellState<T> &L = w[2], &R = w[3];
    const T inv = rcp_(L.sr + R.sr);
    const T wl = L.sr * inv, wr = R.sr * inv;
    const T u = wl * (L.mn * L.ir) + wr * (R.mn * R.ir);
    const T v = wl * (L.mt1 * L.ir) + wr * (R.mt1 * R.ir);
    const T ww = wl * (L.mt2 * L.ir) + wr * (R.mt2 * R.ir);
    const T H = wl * ((L.E + L.p) * L.ir) + wr * ((R.E + R.p) * R.ir);
    const T q2 = u * u + v * v + ww * ww;
    const T c2 = G.gm1 * (H - (T)0.5 * q2);
    const T ic = rsqrt_(c2);
    const T c = c2 * ic;
    const T b1 = G.gm1 * ic * ic;
    const T b2 = (T)0.5 * q2 * b1;
    // halved coefficients (exact): tU, xU, tF, xF below hold t/2 and x/2
    const T hb1 = (T)0.5 * b1, hb2 = (T)0.5 * b2, hic = (T)0.5 * ic;

    // Projection onto the left eigenvectors: with t = b2 a0 + b1 (a4 - u a1 - v a2 - w a3)
    // and x = (a1 - u a0)/c the five components are (t-x)/2, a0-t, a2-v a0, a3-w a0, (t+x)/2.
    T tU[6], xU[6], tF[6], xF[6], a0[6], f0[6], wt1[6], wt2[6], gt1[6], gt2[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const CellState<T> &s = w[j];
        // physical flux f = (mn, mn un + p, mt1 un, mt2 un, (E + p) un); with
        // X = E - u mn - v mt1 - w mt2 its t-combination f4 - u f1 - v f2 - w f3 is
        // un (X + p) - u p, and f1 - u mn = mn (un - u) + p
        const T un = s.mn * s.ir;
        const T X = s.E - u * s.mn - v * s.mt1 - ww * s.mt2;
        tU[j] = hb2 * s.r + hb1 * X;
        xU[j] = (s.mn - u * s.r) * hic;
        tF[j] = hb2 * s.mn + hb1 * (un * (X + s.p) - u * s.p);
        xF[j] = (s.mn * (un - u) + s.p) * hic;
        a0[j] = s.r;
        f0[j] = s.mn;
        wt1[j] = s.mt1 - v * s.r;
        wt2[j] = s.mt2 - ww * s.r;
        gt1[j] = s.mt1 * un - v * s.mn;
        gt2[j] = s.mt2 * un - ww * s.mn;
    }
    if constexpr (SCH == SCH_HLLC_WAO53) {
        // face states: WENO-AO(5,3) of the characteristic variables (left-biased from cells
        // 0..4, right-biased from cells 5..1), back to conservative components; a state
        // that is not physical falls back to the face cell's own state
        T wlf[5], wrf[5];
        {
            T Wm[6];
#pragma unroll
            for (int m = 0; m < 5; ++m) {
#pragma unroll
                for (int j = 0; j < 6; ++j)
                    Wm[j] = m == 0 ? tU[j] - xU[j]
                          : m == 1 ? fma((T)-2, tU[j], a0[j])
                          : m == 2 ? wt1[j]
                          : m == 3 ? wt2[j]
                                   : tU[j] + xU[j];
                wlf[m] = wao53(Wm[0], Wm[1], Wm[2], Wm[3], Wm[4]);
                wrf[m] = wao53(Wm[5], Wm[4], Wm[3], Wm[2], Wm[1]);
            }
        }
        T UL[5], UR[5];
        auto back = [&](const T g_[5], T out[5]) {
            const T s15_ = g_[0] + g_[4];
            out[0] = s15_ + g_[1];
            out[1] = u * out[0] + c * (g_[4] - g_[0]);
            out[2] = v * out[0] + g_[2];
            out[3] = ww * out[0] + g_[3];
            out[4] = H * s15_ + u * c * (g_[4] - g_[0]) + (T)0.5 * q2 * g_[1] + v * g_[2] + ww * g_[3];
        };
        back(wlf, UL);
        back(wrf, UR);
        auto physical = [&](const T U_[5]) {
            const T pk = fma(G.gm1, fma((T)-0.5 * fma(U_[3], U_[3], fma(U_[2], U_[2], U_[1] * U_[1])),
                                        rcp_(U_[0]), U_[4]), -(G.g * G.B));
            return U_[0] > (T)0 && pk + G.B > (T)0;
        };
        if (!physical(UL)) { UL[0] = L.r; UL[1] = L.mn; UL[2] = L.mt1; UL[3] = L.mt2; UL[4] = L.E; }
        if (!physical(UR)) { UR[0] = R.r; UR[1] = R.mn; UR[2] = R.mt1; UR[3] = R.mt2; UR[4] = R.E; }
        hllc(UL, UR, G, F);
        return;
    }
    const T unL = L.mn * L.ir, unR = R.mn * R.ir;
    T W[6], Gc[6], g[5];
    // field 1: u - c
#pragma unroll
    for (int j = 0; j < 6; ++j) { W[j] = tU[j] - xU[j]; Gc[j] = tF[j] - xF[j]; }
#define MRFV_CF(W_, G_, a_, b_) (UNIFORM ? char_flux_uniform<SCH>(W_, G_, a_, b_) : char_flux<SCH>(W_, G_, a_, b_))
    g[0] = MRFV_CF(W, Gc, unL - L.c, unR - R.c);
    // field 2: entropy, u
#pragma unroll
    for (int j = 0; j < 6; ++j) { W[j] = fma((T)-2, tU[j], a0[j]); Gc[j] = fma((T)-2, tF[j], f0[j]); }
    g[1] = MRFV_CF(W, Gc, unL, unR);
    // fields 3, 4: shear, u
    g[2] = MRFV_CF(wt1, gt1, unL, unR);
    g[3] = MRFV_CF(wt2, gt2, unL, unR);
    // field 5: u + c
#pragma unroll
    for (int j = 0; j < 6; ++j) { W[j] = tU[j] + xU[j]; Gc[j] = tF[j] + xF[j]; }
    g[4] = MRFV_CF(W, Gc, unL + L.c, unR + R.c);
#undef MRFV_CF

    // Back to conservative components: F = R g.
    const T s15 = g[0] + g[4];
    F[0] = s15 + g[1];
    F[1] = u * F[0] + c * (g[4] - g[0]);
    F[2] = v * F[0] + g[2];
    F[3] = ww * F[0] + g[3];
    F[4] = H * s15 + u * c * (g[4] - g[0]) + (T)0.5 * q2 * g[1] + v * g[2] + ww * g[3];
}

// Interior cell index (z,y,x) of pencil position p for thread coordinates (r, m).
template <int DIR>
__device__ __forceinline__ int cell_of(int r, int m, int p) {
    if (DIR == 0) return (m * NI + r) * NI + p;
    if (DIR == 1) return (m * NI + p) * NI + r;
    return (p * NI + m) * NI + r;
}

template <int DIR>
__device__ __forceinline__ int pencil_base(int r, int m) {
    if (DIR == 0) return ((m + HW) * NP + (r + HW)) * NP;
    if (DIR == 1) return ((m + HW) * NP) * NP + (r + HW);
    return (m + HW) * NP + (r + HW);
}

// Walks the pencil (r, m) along DIR: 17 faces, flux differences for 16 cells.
// sink.cell(q_phys, cell, dF) and sink.face(side, q_phys, F) receive the results.
template <typename T, int DIR, int SCH, class Sink>
__device__ __forceinline__ void pencil(const T *__restrict__ ub, int r, int m, const Gas<T> &G,
                                       Sink &sink) {
    constexpr int S = Axes<DIR>::STRIDE;
    const int qmap[5] = {0, Axes<DIR>::N1, Axes<DIR>::T1, Axes<DIR>::T2, 4};
    const int base = pencil_base<DIR>(r, m);
    CellState<T> w[6];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        load_state<T, DIR>(ub, base + (j + 1) * S, G, w[j]);
        derive_state(G, w[j]);
    }
    T Fp[5];
#pragma unroll 1
    for (int f = 0; f <= NI; ++f) {
        load_state<T, DIR>(ub, base + (f + 6) * S, G, w[5]);
        derive_state(G, w[5]);
        T F[5];
        face_flux<T, false, SCH>(w, G, F);
        if (f == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sink.face(2 * DIR, qmap[k], F[k]);
        } else {
            const int cell = cell_of<DIR>(r, m, f - 1);
#pragma unroll
            for (int k = 0; k < 5; ++k) sink.cell(qmap[k], cell, F[k] - Fp[k]);
        }
        if (f == NI) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sink.face(2 * DIR + 1, qmap[k], F[k]);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) Fp[k] = F[k];
#pragma unroll
        for (int j = 0; j < 5; ++j) w[j] = w[j + 1];
    }
}

// ------------------------------------------------- Tait's equation of state --------
// Sec. "Influence of Equation of State": p = B (pg - 1) + A with pg = (rho/rho0)^gamma, so
// c^2 = dp/drho = gamma B pg / rho; the energy is not evolved (its flux is zero).  The four
// fields (u - c, u, u, u + c) of the barotropic system are projected with the closed-form
// left eigenvectors at the Roe state (sqrt(rho)-weighted velocity and
// c~^2 = (p_R - p_L)/(rho_R - rho_L)) and reconstructed by char_flux as for the stiffened
// gas.  The secant c~^2 is evaluated without cancellation as
//   B pg_L / rho_L * ((1 + d)^gamma - 1) / d,  d = (rho_R - rho_L) / rho_L,
// with (1 + d)^gamma - 1 = expm1(gamma log1p(d)), and gamma B pg_L / rho_L = c_L^2 at d = 0;
// the plain difference quotient loses all digits when the densities differ by a few
// rounding units, which in FP32 is common in smooth regions.
template <typename T>
struct TaitGas {
    T g, B, A, ir0;   // gamma, B, A, 1 / rho0
};

template <typename T>
struct TaitState {
    T r, mn, mt1, mt2, ir, un, pg, p, c;
};

__device__ __forceinline__ float pow_(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double pow_(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float expm1_(float x) { return expm1f(x); }
__device__ __forceinline__ double expm1_(double x) { return expm1(x); }
__device__ __forceinline__ float log1p_(float x) { return log1pf(x); }
__device__ __forceinline__ double log1p_(double x) { return log1p(x); }

template <typename T, int DIR>
__device__ __forceinline__ void load_tait(const T *__restrict__ u, int idx, const TaitGas<T> &G,
                                          TaitState<T> &s) {
    s.r = u[idx];
    s.mn = u[idx + Axes<DIR>::N1 * CELLS_P];
    s.mt1 = u[idx + Axes<DIR>::T1 * CELLS_P];
    s.mt2 = u[idx + Axes<DIR>::T2 * CELLS_P];
    s.ir = rcp_(s.r);
    s.un = s.mn * s.ir;
    s.pg = pow_(s.r * G.ir0, G.g);
    s.p = fma(G.B, s.pg - (T)1, G.A);
    s.c = sqrt_(G.g * G.B * s.pg * s.ir);
}

template <typename T>
__device__ __forceinline__ void face_flux_tait(const TaitState<T> w[6], const TaitGas<T> &G, T F[5]) {
    const TaitState<T> &L = w[2], &R = w[3];
    const T sl = sqrt_(L.r), sr = sqrt_(R.r);
    const T inv = rcp_(sl + sr);
    const T u = (sl * L.un + sr * R.un) * inv;
    const T v = (sl * (L.mt1 * L.ir) + sr * (R.mt1 * R.ir)) * inv;
    const T ww = (sl * (L.mt2 * L.ir) + sr * (R.mt2 * R.ir)) * inv;
    const T d = (R.r - L.r) * L.ir;
    const T ratio = d == (T)0 ? G.g : expm1_(G.g * log1p_(d)) / d;
    const T c = sqrt_(G.B * L.pg * L.ir * ratio), h = (T)0.5 * rcp_(c);
    const T upc = u + c, umc = u - c;
    T W1[6], W2[6], W3[6], W4[6], G1[6], G2[6], G3[6], G4[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const TaitState<T> &q = w[j];
        const T f1 = fma(q.mn, q.un, q.p);
        W1[j] = (upc * q.r - q.mn) * h;
        W4[j] = (q.mn - umc * q.r) * h;
        W2[j] = q.mt1 - v * q.r;
        W3[j] = q.mt2 - ww * q.r;
        G1[j] = (upc * q.mn - f1) * h;
        G4[j] = (f1 - umc * q.mn) * h;
        G2[j] = q.mt1 * q.un - v * q.mn;
        G3[j] = q.mt2 * q.un - ww * q.mn;
    }
    const T g1 = char_flux<SCH_ROE_WENO5>(W1, G1, L.un - L.c, R.un - R.c);
    const T g2 = char_flux<SCH_ROE_WENO5>(W2, G2, L.un, R.un);
    const T g3 = char_flux<SCH_ROE_WENO5>(W3, G3, L.un, R.un);
    const T g4 = char_flux<SCH_ROE_WENO5>(W4, G4, L.un + L.c, R.un + R.c);
    F[0] = g1 + g4;
    F[1] = umc * g1 + upc * g4;
    F[2] = v * F[0] + g2;
    F[3] = ww * F[0] + g3;
    F[4] = (T)0;
}

// The pencil walk of `pencil` for Tait's system.
template <typename T, int DIR, class Sink>
__device__ __forceinline__ void pencil_tait(const T *__restrict__ ub, int r, int m, const TaitGas<T> &G,
                                            Sink &sink) {
    constexpr int S = Axes<DIR>::STRIDE;
    const int qmap[5] = {0, Axes<DIR>::N1, Axes<DIR>::T1, Axes<DIR>::T2, 4};
    const int base = pencil_base<DIR>(r, m);
    TaitState<T> w[6];
#pragma unroll
    for (int j = 0; j < 5; ++j) load_tait<T, DIR>(ub, base + (j + 1) * S, G, w[j]);
    T Fp[5];
#pragma unroll 1
    for (int f = 0; f <= NI; ++f) {
        load_tait<T, DIR>(ub, base + (f + 6) * S, G, w[5]);
        T F[5];
        face_flux_tait<T>(w, G, F);
        if (f == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sink.face(2 * DIR, qmap[k], F[k]);
        } else {
            const int cell = cell_of<DIR>(r, m, f - 1);
#pragma unroll
            for (int k = 0; k < 5; ++k) sink.cell(qmap[k], cell, F[k] - Fp[k]);
        }
        if (f == NI) {
#pragma unroll
            for (int k = 0; k < 5; ++k) sink.face(2 * DIR + 1, qmap[k], F[k]);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) Fp[k] = F[k];
#pragma unroll
        for (int j = 0; j < 5; ++j) w[j] = w[j + 1];
    }
}

template <typename T>
__device__ __forceinline__ Gas<T> gas_of(const InstDev &P) {
    return Gas<T>{(T)P.gamma, (T)P.B, (T)(P.gamma - 1.0)};
}

// ---------------------------------------------------------------- plain path ---------

template <typename T>
struct GlobalSink {
    T *D;      // this slot's D: [3][5][4096]
    T *FF;     // this slot's FF: [6][5][256]
    int dir, rm;
    __device__ void cell(int q, int c, T v) { D[(dir * 5 + q) * CELLS_I + c] = v; }
    __device__ void face(int side, int q, T v) { FF[(side * 5 + q) * FACE + rm] = v; }
};

template <typename T, int SCH>
__global__ __launch_bounds__(TPB) void k_flux(const T *__restrict__ U, WorkList wl,
                                              const BlockMeta *__restrict__ meta,
                                              const InstDev *__restrict__ inst, T *D, T *FF) {
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int slot = wl.at(b);
    const int r = threadIdx.x & 15, m = threadIdx.x >> 4;
    const T *ub = U + (size_t)slot * 5 * CELLS_P;
    GlobalSink<T> sink{D + (size_t)slot * 3 * 5 * CELLS_I, FF + (size_t)slot * 6 * 5 * FACE,
                       (int)blockIdx.y, m * NI + r};
    if constexpr (SCH == SCH_TAIT_ROE_WENO5) {
        const InstDev &P = inst[meta[slot].inst];
        const TaitGas<T> G{(T)P.gamma, (T)P.B, (T)P.tait_A, (T)(1.0 / P.tait_rho0)};
        if (blockIdx.y == 0) pencil_tait<T, 0>(ub, r, m, G, sink);
        else if (blockIdx.y == 1) pencil_tait<T, 1>(ub, r, m, G, sink);
        else pencil_tait<T, 2>(ub, r, m, G, sink);
    } else {
        const Gas<T> G = gas_of<T>(inst[meta[slot].inst]);
        if (blockIdx.y == 0) pencil<T, 0, SCH>(ub, r, m, G, sink);
        else if (blockIdx.y == 1) pencil<T, 1, SCH>(ub, r, m, G, sink);
        else pencil<T, 2, SCH>(ub, r, m, G, sink);
    }
    }
}

// Non-leaf blocks: face-flux planes <- area average of the children's planes.
template <typename T>
__global__ __launch_bounds__(TPB) void k_ff_restrict(T *FF, WorkList wl,
                                                     const int32_t *__restrict__ child) {
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int slot = wl.at(b);
    const int side = blockIdx.y, d = side >> 1, hi = side & 1;
    const int M = threadIdx.x >> 4, R = threadIdx.x & 15;
    const int cm = M >> 3, cr = R >> 3;
    int o[3];
    o[d] = hi;
    o[d == 0 ? 1 : 0] = cr;
    o[d == 2 ? 1 : 2] = cm;
    const int cs = child[(size_t)slot * 8 + (o[2] << 2) + (o[1] << 1) + o[0]];
    const T *cp = FF + ((size_t)cs * 6 + side) * 5 * FACE;
    T *pp = FF + ((size_t)slot * 6 + side) * 5 * FACE;
    const int m0 = 2 * (M & 7), r0 = 2 * (R & 7);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T *c = cp + q * FACE;
        const T v00 = c[m0 * NI + r0], v10 = c[m0 * NI + r0 + 1];
        const T v01 = c[(m0 + 1) * NI + r0], v11 = c[(m0 + 1) * NI + r0 + 1];
        pp[q * FACE + M * NI + R] = ((v00 + v10) + (v01 + v11)) * (T)0.25;
    }
    }
}

// Region index of the face neighbour on `side` in the 27-entry neighbourhood.
__device__ __forceinline__ int face_region(int side) {
    const int d = side >> 1, s = (side & 1) ? 1 : -1;
    int r[3] = {0, 0, 0};
    r[d] = s;
    return (r[2] + 1) * 9 + (r[1] + 1) * 3 + (r[0] + 1);
}

// Coarse leaves at resolution jumps: replace the own boundary flux by the fine average in
// the flux differences D (plain path).
template <typename T>
__global__ __launch_bounds__(TPB) void k_reflux(T *D, const T *__restrict__ FF, WorkList wl,
                                                const BlockMeta *__restrict__ meta,
                                                const int32_t *__restrict__ nbr) {
    const int nb_ = wl.count();
    for (int b = blockIdx.x; b < nb_; b += gridDim.x) {
    const int slot = wl.at(b);
    const int rm = threadIdx.x, m = rm >> 4, r = rm & 15;
    for (int side = 0; side < 6; ++side) {
        const int nb = nbr[(size_t)slot * 27 + face_region(side)];
        if (nb < 0 || meta[nb].leaf) continue;
        const int d = side >> 1, hi = side & 1;
        const int p = hi ? NI - 1 : 0;
        const int cell = d == 0 ? (m * NI + r) * NI + p : (d == 1 ? (m * NI + p) * NI + r : (p * NI + m) * NI + r);
        T *Dd = D + ((size_t)slot * 3 + d) * 5 * CELLS_I;
        const T *own = FF + ((size_t)slot * 6 + side) * 5 * FACE;
        const T *fine = FF + ((size_t)nb * 6 + (side ^ 1)) * 5 * FACE;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T delta = fine[q * FACE + rm] - own[q * FACE + rm];
            Dd[q * CELLS_I + cell] += hi ? delta : -delta;
        }
        __syncthreads();
    }
    }
}

// Gravity source of eq:Euler at one cell, added to the right-hand side L:
// S(u) = (0, rho g, rho v . g) with the momenta m = rho v of the stage state.
template <typename T>
__device__ __forceinline__ void add_source(const InstDev &P, const T u[5], T L[5]) {
    const T gx = (T)P.gravity[0], gy = (T)P.gravity[1], gz = (T)P.gravity[2];
    L[1] = fma(u[0], gx, L[1]);
    L[2] = fma(u[0], gy, L[2]);
    L[3] = fma(u[0], gz, L[3]);
    L[4] += fma(u[3], gz, fma(u[2], gy, u[1] * gx));
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_combine(const T *__restrict__ D, T *L, WorkList wl,
                                                 const BlockMeta *__restrict__ meta,
                                                 const InstDev *__restrict__ inst,
                                                 const T *__restrict__ U) {
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int slot = wl.at(b);
    const BlockMeta mt = meta[slot];
    const InstDev &P = inst[mt.inst];
    const T inv_dx = (T)(1.0 / ldexp(P.dx0, -mt.level));
    const T *Ds = D + (size_t)slot * 3 * 5 * CELLS_I;
    T *Ls = L + (size_t)slot * 5 * CELLS_I;
    const int c = blockIdx.y * TPB + threadIdx.x;
    T l[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T s = (Ds[q * CELLS_I + c] + Ds[(5 + q) * CELLS_I + c]) + Ds[(10 + q) * CELLS_I + c];
        l[q] = -s * inv_dx;
    }
    if (P.has_source) {   // uniform per workgroup
        const T *ub = U + (size_t)slot * 5 * CELLS_P;
        const int o = ((c / FACE + HW) * NP + (c / NI) % NI + HW) * NP + c % NI + HW;
        T u[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) u[q] = ub[o + q * CELLS_P];
        add_source(P, u, l);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) Ls[q * CELLS_I + c] = l[q];
    }
}

template <typename T>
__device__ __forceinline__ T stage_coef(int stage) {
    return stage == 0 ? (T)1 : (stage == 1 ? (T)0.25 : (T)(2.0 / 3.0));
}

template <typename T>
__device__ __forceinline__ bool physical_state(const T u[5], const Gas<T> &G) {
    const T ke = (T)0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
    const T p = G.gm1 * (u[4] - ke) - G.g * G.B;
    return u[0] > (T)0 && p + G.B > (T)0 && isfinite(u[4]) && isfinite(u[1] + u[2] + u[3]);
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_update(int stage, const double *__restrict__ dt, T *U,
                                                T *U0, const T *__restrict__ L, WorkList wl,
                                                const BlockMeta *__restrict__ meta,
                                                const InstDev *__restrict__ inst, int32_t *err) {
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int slot = wl.at(b);
    const BlockMeta mt = meta[slot];
    const Gas<T> G = gas_of<T>(inst[mt.inst]);
    const T dtt = (T)dt[mt.inst];
    const T a = stage_coef<T>(stage);
    const int c = blockIdx.y * TPB + threadIdx.x;
    const int o = ((c / FACE + HW) * NP + (c / NI) % NI + HW) * NP + c % NI + HW;
    T *ub = U + (size_t)slot * 5 * CELLS_P;
    T *u0b = U0 + (size_t)slot * 5 * CELLS_I;
    const T *lb = L + (size_t)slot * 5 * CELLS_I;
    T un[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T us = ub[o + q * CELLS_P];
        T u0;
        if (stage == 0) {
            u0 = us;
            u0b[q * CELLS_I + c] = us;
        } else {
            u0 = u0b[q * CELLS_I + c];
        }
        un[q] = u0 + a * ((us - u0) + dtt * lb[q * CELLS_I + c]);
        ub[o + q * CELLS_P] = un[q];
    }
    // Tait: any positive density (the energy is not evolved)
    const bool ok = inst[mt.inst].eos == 1 ? un[0] > (T)0 && isfinite(un[1] + un[2] + un[3])
                                           : physical_state(un, G);
    if (!ok) atomicOr(err, 1);
    }
}

// ---------------------------------------------------------------- batched path -------

template <typename T, bool ADD>
struct LdsSink {
    T *acc;    // [5][4096]
    T *FF;     // this slot's FF
    int rm;
    __device__ void cell(int q, int c, T v) {
        if (ADD) acc[q * CELLS_I + c] += v;
        else acc[q * CELLS_I + c] = v;
    }
    __device__ void face(int side, int q, T v) { FF[(side * 5 + q) * FACE + rm] = v; }
};

// One workgroup per leaf.  The block is walked in groups of GP z-planes; for each group
// every x-, y- and z-face flux the group's cells need is computed once, one face per
// thread (coalesced, L1-resident six-cell stencils; all axes share one code path), and
// staged in LDS.  Each thread then owns one (x, y) column: it forms
// D = ((Dx + Dy) + Dz) for the group's cells and writes the SSP-RK3 stage result to the
// other state buffer.  Stencil cells outside the block are read from the same-level
// neighbour's interior where one exists (no halo copy), else from the own halo, which
// the fill has predicted from the parent or clamped at a zero-gradient boundary.
// Template parameters: GP z-planes per group (1, 2, 4) and TPB_F threads (>= 256, the
// column owners); the launch shape is chosen by the autotuner among the instantiated
// variants.  Every variant evaluates each face by the same instruction sequence and sums
// D in the same order, so all give bitwise the same result.
constexpr int NFZ = NI * NI;                  // z-faces per face plane (256)


// Sources of one workgroup's stencils as 32-bit byte offsets from the lowest of them,
// read through one buffer resource (range-checked: out-of-range reads return zero);
// usable (near) when the own block and its six face neighbours lie within 4 GiB.
struct NearSrc {
    __amdgpu_buffer_rsrc_t rsrc;
    unsigned own, lo[3], hi[3];
    bool near;
};
constexpr int BUFFER_RSRC_WORD3 = 0x00020000;   // raw 32-bit loads (gfx9 family)

__device__ __forceinline__ float buffer_f32(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
}

// Face flux along axis D for the stencil starting at padded index base (six cells at
// base + j*stride, padded coordinate pos0 + j along D); cells below / above the interior
// come from lo / hi, which are the neighbour's block shifted by -+16 cells along D (or
// the own block).  The result is returned in physical component order.
template <typename T, int D, int SCH>
__device__ __forceinline__ void face_flux_at(const T *__restrict__ ub, const T *__restrict__ lo,
                                             const T *__restrict__ hi, const NearSrc &ns, int base,
                                             int pos0, const Gas<T> &G, T Fp[5]) {
    constexpr int stride = Axes<D>::STRIDE;
    constexpr int n1 = Axes<D>::N1, t1 = Axes<D>::T1, t2 = Axes<D>::T2;   // rotated components
    CellState<T> w[6];
    static_assert(sizeof(T) == 4, "the fused path is FP32");
    constexpr int CB = CELLS_P * (int)sizeof(T);   // component stride in bytes
    if (ns.near) {
        // 32-bit offsets into one buffer resource: per-lane choice of the source block
        // only where a wavefront's stencils leave the own interior
        auto load = [&](int j, unsigned off) __attribute__((always_inline)) {
            w[j].r = buffer_f32(ns.rsrc, off, 0);
            w[j].mn = buffer_f32(ns.rsrc, off, n1 * CB);
            w[j].mt1 = buffer_f32(ns.rsrc, off, t1 * CB);
            w[j].mt2 = buffer_f32(ns.rsrc, off, t2 * CB);
            w[j].E = buffer_f32(ns.rsrc, off, 4 * CB);
        };
        if (__all(pos0 >= HW && pos0 + 5 < HW + NI)) {
#pragma unroll
            for (int j = 0; j < 6; ++j) load(j, ns.own + (unsigned)(base + j * stride) * (unsigned)sizeof(T));
        } else {
            // selects of values, not of members (a member select keeps ns in scratch)
            const unsigned olo = ns.lo[D], ohi = ns.hi[D], oown = ns.own;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const int pos = pos0 + j;
                const unsigned src = pos < HW ? olo : (pos >= HW + NI ? ohi : oown);
                load(j, src + (unsigned)(base + j * stride) * (unsigned)sizeof(T));
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int pos = pos0 + j;
            const T *src = pos < HW ? lo : (pos >= HW + NI ? hi : ub);
            load_state<T, D>(src, base + j * stride, G, w[j]);
        }
    }
    // the arithmetic follows the loads in one place for both load paths
#pragma unroll
    for (int j = 0; j < 6; ++j) derive_state(G, w[j]);
    T F[5];
    face_flux<T, true, SCH>(w, G, F);
    Fp[0] = F[0];
    Fp[4] = F[4];
    Fp[n1] = F[1];
    Fp[t1] = F[2];
    Fp[t2] = F[3];
}

template <typename T, int GP, int TPB_F, bool PERSIST, int WPE, int SCH>
__global__ __attribute__((amdgpu_flat_work_group_size(TPB_F, TPB_F), amdgpu_waves_per_eu(WPE)))
void k_rhs_update(int stage, const double *__restrict__ dt,
                                                      const T *__restrict__ Uin, T *__restrict__ Uout,
                                                      T *U0, WorkList wl,
                                                      const BlockMeta *__restrict__ meta,
                                                      const int32_t *__restrict__ nbr,
                                                      const InstDev *__restrict__ inst, T *FF,
                                                      int32_t *err, int restrict_parents,
                                                      double *__restrict__ cflmax, int force_ptr) {
    constexpr int NFX = GP * NI * (NI + 1);   // x-faces per group (y-faces alike)
    // x- and y-faces are numbered with the faces 3 .. 13 of each row first: their
    // six-cell stencils lie in the own interior, so whole wavefronts of them take the
    // uniform-base loads of face_flux_at; the faces 0-2 and 14-16 follow
    constexpr int NF_IN = NI - 5, NF_OUT = NI + 1 - NF_IN;
    constexpr int NFX_IN = GP * NI * NF_IN;
    // Groups are pipelined: while the column owners update group g from one buffer, all
    // wavefronts compute the faces of group g + 1 into the other, taking 64-face chunks
    // from an LDS counter (owners join after their update); one barrier per group.
    // z-face planes live in a ring of 2 GP + 1 slots (face plane kf in slot kf mod NZR):
    // the planes of group g (k0 .. k0 + GP) and those group g + 1 adds never share a slot.
    constexpr int NZR = 2 * GP + 1;
    __shared__ T Fx[2][GP][NI][NI + 1][5];   // [buffer][plane][y][face x][q]
    __shared__ T Fy[2][GP][NI + 1][NI][5];   // [buffer][plane][face y][x][q]
    __shared__ T Fz[NZR][NI][NI][5];         // [face plane mod NZR][y][x][q]
    __shared__ int next_chunk[2];            // per buffer: first face not yet handed out
    __shared__ double cfl_acc[3][FACE];      // with cflmax: per owner column, the speed maxima
    // one workgroup per leaf in XCD-aware order (graph launches size the grid by the slot
    // capacity and surplus groups exit), or, persistent, a fixed grid looping over the leaves
    const int nleaf = wl.count();
    auto block = [&](int b) __attribute__((always_inline)) {
    const int slot = wl.at(b);
    const BlockMeta mt = meta[slot];
    const InstDev P = inst[mt.inst];
    const Gas<T> G = gas_of<T>(P);
    const T *ub = Uin + (size_t)slot * 5 * CELLS_P;
    T *ob = Uout + (size_t)slot * 5 * CELLS_P;
    // per face side: the same-level neighbour shifted so that own padded indices address
    // its interior, or the own block (halo filled) at jumps and zero-gradient boundaries
    const T *nlo[3], *nhi[3];
    {
        const int freg[6] = {12, 14, 10, 16, 4, 22};
        const int strd[3] = {1, NP, NP * NP};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int sl = (mt.zg >> (2 * a)) & 1 ? -1 : nbr[(size_t)slot * 27 + freg[2 * a]];
            const int sh = (mt.zg >> (2 * a + 1)) & 1 ? -1 : nbr[(size_t)slot * 27 + freg[2 * a + 1]];
            nlo[a] = sl >= 0 ? Uin + (size_t)sl * 5 * CELLS_P + NI * strd[a] : ub;
            nhi[a] = sh >= 0 ? Uin + (size_t)sh * 5 * CELLS_P - NI * strd[a] : ub;
        }
    }
    NearSrc ns;
    {
        uintptr_t mn = (uintptr_t)ub, mx = (uintptr_t)ub;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            mn = min(mn, min((uintptr_t)nlo[a], (uintptr_t)nhi[a]));
            mx = max(mx, max((uintptr_t)nlo[a], (uintptr_t)nhi[a]));
        }
        // every access lies below the highest source plus one block
        const uintptr_t span = mx - mn + (uintptr_t)(5 * CELLS_P * sizeof(T));
        // force_ptr (a launch argument, so the code is the production code): always the
        // per-lane pointer loads
        ns.near = !force_ptr && span <= (uintptr_t)0xffffffffu;
        ns.rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)(ub - ((uintptr_t)ub - mn) / sizeof(T)),
                                                    (short)0, ns.near ? (int)(unsigned)span : 0,
                                                    BUFFER_RSRC_WORD3);
        ns.own = (unsigned)((uintptr_t)ub - mn);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            ns.lo[a] = (unsigned)((uintptr_t)nlo[a] - mn);
            ns.hi[a] = (unsigned)((uintptr_t)nhi[a] - mn);
        }
    }
    T *ffs = FF + (size_t)slot * 6 * 5 * FACE;
    T *u0b = U0 + (size_t)slot * 5 * CELLS_I;
    const T inv_dx = (T)(1.0 / ldexp(P.dx0, -mt.level));
    const T dtt = (T)dt[mt.inst];
    const T a = stage_coef<T>(stage);
    const int tid = threadIdx.x;
    const bool owner = tid < FACE;              // column owners (x = tid & 15, y = tid >> 4)
    const int cx = tid & 15, cy = tid >> 4;
    bool ok = true;
    // Restriction of the new state into the parent's octant (eq:Averaging): the sum of
    // the 2x2x2 children is formed in FP64 as x pairs, then y pairs (lanes 1 and 16 apart
    // in the wavefront), then z pairs, the order of the restriction kernel, so both give
    // bitwise the same parent values.
    const bool rp = restrict_parents && mt.srestr;   // uniform per workgroup
    // z-plane pair (z0, z0 + 1) of the new state, one column per owner thread
    auto restrict_pair = [&](int z0, const T (&u)[2][5]) {
        T *pb = Uout + (size_t)mt.parent * 5 * CELLS_P +
                (((mt.bz & 1) * 8 + (z0 >> 1) + HW) * NP + (mt.by & 1) * 8 + (cy >> 1) + HW) * NP +
                (mt.bx & 1) * 8 + (cx >> 1) + HW;
        const bool wr = ((cx | cy) & 1) == 0;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            double v0 = (double)u[0][q], v1 = (double)u[1][q];
            v0 += __shfl_xor(v0, 1);
            v1 += __shfl_xor(v1, 1);
            v0 += __shfl_xor(v0, 16);
            v1 += __shfl_xor(v1, 16);
            if (wr) pb[q * CELLS_P] = (T)((v0 + v1) * 0.125);
        }
    };

    T uprev[2][5];   // GP = 1: the even plane of a restriction pair
    auto update_group = [&](int k0, T D[GP][5]) {
        T unew[GP][5];
#pragma unroll
        for (int p = 0; p < GP; ++p) {
            const int z = k0 + p;
            const int c = (z * NI + cy) * NI + cx;
            const int o = ((z + HW) * NP + cy + HW) * NP + cx + HW;
            T un[5], us[5], lq[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                us[q] = ub[o + q * CELLS_P];
                lq[q] = -D[p][q] * inv_dx;
            }
            if (P.has_source) add_source(P, us, lq);   // uniform per workgroup
            if (stage < 0) {   // flux divergence only (local time stepping): L into Uout
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    ob[o + q * CELLS_P] = lq[q];
                    unew[p][q] = lq[q];   // restricted like a new state
                }
                continue;
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                T u0;
                if (stage == 0) {
                    u0 = us[q];
                    u0b[q * CELLS_I + c] = us[q];
                } else {
                    u0 = u0b[q * CELLS_I + c];
                }
                un[q] = u0 + a * ((us[q] - u0) + dtt * lq[q]);
                ob[o + q * CELLS_P] = un[q];
                unew[p][q] = un[q];
            }
            ok = ok && physical_state(un, G);
            if (cflmax) {   // uniform: the last stage of a step, for the next step's CFL
                double sp[3];
                cfl_speeds(un[0], un[1], un[2], un[3], un[4], P.gamma, P.B, sp);
#pragma unroll
                for (int d = 0; d < 3; ++d) cfl_acc[d][tid] = fmax(cfl_acc[d][tid], sp[d]);
            }
        }
        if (rp) {
            if constexpr (GP == 1) {
#pragma unroll
                for (int q = 0; q < 5; ++q) uprev[k0 & 1][q] = unew[0][q];
                if (k0 & 1) restrict_pair(k0 - 1, uprev);
            } else {
#pragma unroll
                for (int p = 0; p < GP; p += 2) {
                    T pr[2][5];
#pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        pr[0][q] = unew[p][q];
                        pr[1][q] = unew[p + 1][q];
                    }
                    restrict_pair(k0 + p, pr);
                }
            }
        }
    };

    // faces of group g: x-faces (plane p, row y, face f), y-faces (plane p, face f,
    // column x), then the z-face planes the group adds (all GP + 1 for the first group)
    auto group_faces = [&](int g) {
        const int k0 = g * GP;
        const int first_z = g == 0 ? 0 : 1;
        const int total = 2 * NFX + (GP + 1 - first_z) * NFZ;
        const int buf = g & 1;
        const int lane = tid & 63;
        for (;;) {
            int c0 = 0;
            if (lane == 0) c0 = atomicAdd(&next_chunk[buf], 64);
            c0 = __shfl(c0, 0);
            if (c0 >= total) break;
            const int t = c0 + lane;
            if (t >= total) continue;
            T F[5];
            if (t < NFX) {
                int f, y, p;
                if (t < NFX_IN) {               // faces 3 .. 13 first: stencils in the interior
                    f = 3 + t % NF_IN;
                    y = (t / NF_IN) % NI;
                    p = t / (NF_IN * NI);
                } else {
                    const int v = t - NFX_IN, fb = v % NF_OUT;
                    f = fb < 3 ? fb : fb + NF_IN;
                    y = (v / NF_OUT) % NI;
                    p = v / (NF_OUT * NI);
                }
                const int base = ((k0 + p + HW) * NP + y + HW) * NP + f + 1;
                face_flux_at<T, 0, SCH>(ub, nlo[0], nhi[0], ns, base, f + 1, G, F);
#pragma unroll
                for (int q = 0; q < 5; ++q) Fx[buf][p][y][f][q] = F[q];
                if (f == 0 || f == NI) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) ffs[((f ? 1 : 0) * 5 + q) * FACE + (k0 + p) * NI + y] = F[q];
                }
            } else if (t < 2 * NFX) {
                const int u = t - NFX;
                int x, f, p;
                if (u < NFX_IN) {
                    x = u % NI;
                    f = 3 + (u / NI) % NF_IN;
                    p = u / (NI * NF_IN);
                } else {
                    const int v = u - NFX_IN, fb = (v / NI) % NF_OUT;
                    x = v % NI;
                    f = fb < 3 ? fb : fb + NF_IN;
                    p = v / (NI * NF_OUT);
                }
                const int base = ((k0 + p + HW) * NP + f + 1) * NP + x + HW;
                face_flux_at<T, 1, SCH>(ub, nlo[1], nhi[1], ns, base, f + 1, G, F);
#pragma unroll
                for (int q = 0; q < 5; ++q) Fy[buf][p][f][x][q] = F[q];
                if (f == 0 || f == NI) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) ffs[((2 + (f ? 1 : 0)) * 5 + q) * FACE + (k0 + p) * NI + x] = F[q];
                }
            } else {
                const int u = t - 2 * NFX;
                const int x = u % NI, y = (u / NI) % NI, j = u / NFZ + first_z;
                const int kf = k0 + j;          // face between interior planes kf-1 and kf
                const int base = ((kf + 1) * NP + y + HW) * NP + x + HW;   // padded z = kf+1 .. kf+6
                face_flux_at<T, 2, SCH>(ub, nlo[2], nhi[2], ns, base, kf + 1, G, F);
#pragma unroll
                for (int q = 0; q < 5; ++q) Fz[kf % NZR][y][x][q] = F[q];
                if (kf == 0 || kf == NI) {
#pragma unroll
                    for (int q = 0; q < 5; ++q) ffs[((4 + (kf ? 1 : 0)) * 5 + q) * FACE + y * NI + x] = F[q];
                }
            }
        }
    };
    auto group_update = [&](int g) {
        const int k0 = g * GP, buf = g & 1;
        T D[GP][5];
#pragma unroll
        for (int p = 0; p < GP; ++p)
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const T dxq = Fx[buf][p][cy][cx + 1][q] - Fx[buf][p][cy][cx][q];
                const T dyq = Fy[buf][p][cy + 1][cx][q] - Fy[buf][p][cy][cx][q];
                const T dzq = Fz[(k0 + p + 1) % NZR][cy][cx][q] - Fz[(k0 + p) % NZR][cy][cx][q];
                D[p][q] = (dxq + dyq) + dzq;
            }
        update_group(k0, D);
    };

    if (tid < 2) next_chunk[tid] = 0;
    if (cflmax && owner)
#pragma unroll
        for (int d = 0; d < 3; ++d) cfl_acc[d][tid] = 0.0;
    __syncthreads();
    // iteration g: update group g (g >= 0) and compute the faces of group g + 1
#pragma unroll 1
    for (int g = -1; g < NI / GP; ++g) {
        if (g >= 0 && owner) group_update(g);
        if (g + 1 < NI / GP) group_faces(g + 1);
        // group g's counter is free again (its faces were done before the last barrier);
        // group g + 2 takes it after the next one
        if (g >= 0 && tid == 0) next_chunk[g & 1] = 0;
        __syncthreads();
    }
    if (!ok) atomicOr(err, 1);
    if (cflmax) {
        // block maxima of the signal speeds (the CFL pass's values, stored as the first slab's
        // maxima, the other slabs zero): over each owner wavefront, then over the four
        double m[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            m[d] = owner ? cfl_acc[d][tid] : 0.0;
            for (int off = 32; off > 0; off >>= 1) m[d] = fmax(m[d], __shfl_xor(m[d], off));
        }
        __syncthreads();
        if (owner && (tid & 63) == 0)
#pragma unroll
            for (int d = 0; d < 3; ++d) cfl_acc[d][tid >> 6] = m[d];
        __syncthreads();
        if (tid < 3) {
            double v = cfl_acc[tid][0];
#pragma unroll
            for (int w = 1; w < FACE / 64; ++w) v = fmax(v, cfl_acc[tid][w]);
            double *bm = cflmax + (size_t)mt.lpos * CFL_SLABS * 3;   // by all-leaves position
            bm[tid] = v;
#pragma unroll
            for (int k = 1; k < CFL_SLABS; ++k) bm[k * 3 + tid] = 0.0;
        }
        __syncthreads();   // cfl_acc is cleared again for a persistent grid's next block
    }
    };
    if constexpr (PERSIST) {
        for (int b = blockIdx.x; b < nleaf; b += gridDim.x) block(b);   // uniform per workgroup
    } else {
        // the grid covers every leaf; the loop-free form keeps the register count down
        const int b = xcd_item(blockIdx.x, gridDim.x, nleaf);
        if (b < nleaf) block(b);
    }
}

// Batched path: the jump correction applied to the already-updated state,
// U += a_s dt (L_corrected - L) on the boundary cells of coarse leaves at jumps.
template <typename T>
__global__ __launch_bounds__(TPB) void k_reflux_update(int stage, const double *__restrict__ dt,
                                                       T *U, const T *__restrict__ FF, WorkList wl,
                                                       const BlockMeta *__restrict__ meta,
                                                       const int32_t *__restrict__ nbr,
                                                       const InstDev *__restrict__ inst) {
    const int nb_ = wl.count();
    for (int b = blockIdx.x; b < nb_; b += gridDim.x) {
    const int slot = wl.at(b);
    const BlockMeta mt = meta[slot];
    const InstDev P = inst[mt.inst];
    const T coef = stage_coef<T>(stage) * (T)dt[mt.inst] * (T)(1.0 / ldexp(P.dx0, -mt.level));
    const int rm = threadIdx.x, m = rm >> 4, r = rm & 15;
    T *ub = U + (size_t)slot * 5 * CELLS_P;
    for (int side = 0; side < 6; ++side) {
        const int nb = nbr[(size_t)slot * 27 + face_region(side)];
        if (nb < 0 || meta[nb].leaf) continue;
        const int d = side >> 1, hi = side & 1;
        const int p = (hi ? NI - 1 : 0) + HW;
        const int o = d == 0 ? ((m + HW) * NP + r + HW) * NP + p
                             : (d == 1 ? ((m + HW) * NP + p) * NP + r + HW
                                       : (p * NP + m + HW) * NP + r + HW);
        const T *own = FF + ((size_t)slot * 6 + side) * 5 * FACE;
        const T *fine = FF + ((size_t)nb * 6 + (side ^ 1)) * 5 * FACE;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T delta = fine[q * FACE + rm] - own[q * FACE + rm];
            // L changes by -(D_new - D)/dx with D_new - D = +delta (high) / -delta (low)
            ub[o + q * CELLS_P] += coef * (hi ? -delta : delta);
        }
        __syncthreads();
    }
    }
}

}  // namespace

template <typename T>
hipError_t launch_flux(int scheme, const T *U, const WorkList &wl, const DevTables &tb,
                       const InstDev *inst, T *D, T *FF, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    const dim3 grid(wl.grid, 3), block(TPB);
    switch (scheme) {
        case SCH_ROE_WENO5: hipLaunchKernelGGL((k_flux<T, SCH_ROE_WENO5>), grid, block, 0, st, U, wl, tb.meta, inst, D, FF); break;
        case SCH_ROE_TENO5: hipLaunchKernelGGL((k_flux<T, SCH_ROE_TENO5>), grid, block, 0, st, U, wl, tb.meta, inst, D, FF); break;
        case SCH_LLF_WENO5: hipLaunchKernelGGL((k_flux<T, SCH_LLF_WENO5>), grid, block, 0, st, U, wl, tb.meta, inst, D, FF); break;
        case SCH_HLLC_WAO53: hipLaunchKernelGGL((k_flux<T, SCH_HLLC_WAO53>), grid, block, 0, st, U, wl, tb.meta, inst, D, FF); break;
        case SCH_TAIT_ROE_WENO5: hipLaunchKernelGGL((k_flux<T, SCH_TAIT_ROE_WENO5>), grid, block, 0, st, U, wl, tb.meta, inst, D, FF); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ff_restrict(T *FF, const WorkList &wl, const DevTables &tb, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ff_restrict<T>, dim3(wl.grid, 6), dim3(TPB), 0, st, FF, wl, tb.child);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reflux(T *D, const T *FF, const WorkList &wl, const DevTables &tb,
                         hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reflux<T>, dim3(wl.grid), dim3(TPB), 0, st, D, FF, wl, tb.meta, tb.nbr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_combine(const T *D, T *L, const WorkList &wl, const DevTables &tb,
                          const InstDev *inst, const T *U, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine<T>, dim3(wl.grid, CELLS_I / TPB), dim3(TPB), 0, st, D, L, wl,
                       tb.meta, inst, U);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_update(int stage, const double *dt, T *U, T *U0, const T *L, const WorkList &wl,
                         const DevTables &tb, const InstDev *inst, int32_t *err, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_update<T>, dim3(wl.grid, CELLS_I / TPB), dim3(TPB), 0, st, stage, dt, U, U0,
                       L, wl, tb.meta, inst, err);
    return hipGetLastError();
}

// Launch shapes of the fused kernel: (z-planes per group, threads per workgroup).
// Variants 9 and 10 are persistent: a grid of as many workgroups as fit on the 256 CUs
// at once (3 waves per SIMD at their register count) loops over the leaves instead of
// one workgroup per leaf.  Variants 11 and 12 ask the register allocator for 5 waves per
// SIMD (at most 96 registers, some spilled to scratch) instead of the default 4.
// Variant 13 is variant 7 (the same code) told at launch to load the stencils through
// per-lane pointers always (the path taken when a workgroup's source blocks span more
// than 4 GiB).
constexpr int N_RHS_VARIANTS = 14;
constexpr int RHS_GP[N_RHS_VARIANTS] = {2, 1, 2, 2, 4, 4, 2, 2, 1, 2, 2, 2, 2, 2};
constexpr int RHS_TPB[N_RHS_VARIANTS] = {320, 256, 256, 384, 320, 512, 448, 512, 320, 512, 384, 320, 640, 512};
constexpr bool RHS_PERSIST[N_RHS_VARIANTS] = {false, false, false, false, false, false, false,
                                              false, false, true, true, false, false, false};
constexpr int RHS_WPE[N_RHS_VARIANTS] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 5, 5, 1};
constexpr bool RHS_PTR[N_RHS_VARIANTS] = {false, false, false, false, false, false, false,
                                          false, false, false, false, false, false, true};
constexpr int persist_grid(int tpb) { return 256 * (12 / (tpb / 64) > 0 ? 12 / (tpb / 64) : 1); }

// The other flux kernels are instantiated in three launch shapes (variants 7, 2, 3 of the
// standard kernel), which the autotuner chooses among.
constexpr int N_ALT_VARIANTS = 3;
constexpr int ALT_VARIANT[N_ALT_VARIANTS] = {7, 2, 3};

template <int V, int SCH>
static void launch_variant(int stage, const double *dt, const float *Uin, float *Uout, float *U0,
                    const WorkList &wl, const DevTables &tb, const InstDev *inst, float *FF,
                    int32_t *err, int restrict_parents, double *cflmax, hipStream_t st) {
    constexpr int G = RHS_GP[V], B = RHS_TPB[V];
    constexpr bool PS = RHS_PERSIST[V];
    constexpr int WP = RHS_WPE[V];
    const int grid = PS ? std::min(wl.grid, persist_grid(B)) : round_xcd(wl.grid);
    hipLaunchKernelGGL((k_rhs_update<float, G, B, PS, WP, SCH>), dim3(grid), dim3(B), 0, st, stage, dt, Uin,
                       Uout, U0, wl, tb.meta, tb.nbr, inst, FF, err, restrict_parents, cflmax,
                       RHS_PTR[V] ? 1 : 0);
}

int rhs_variants(int scheme) { return scheme == SCH_ROE_WENO5 ? N_RHS_VARIANTS : N_ALT_VARIANTS; }

// Until a context is tuned it takes variant 7 (two z-planes per group, 512 threads), the
// shape the autotuner chose on the benchmark trees; the other schemes list it first.
int rhs_default_variant(int scheme) { return scheme == SCH_ROE_WENO5 ? 7 : 0; }

void rhs_variant_shape(int scheme, int v, int *gp, int *tpb, int *wpe, int *ptr) {
    if (scheme != SCH_ROE_WENO5) v = ALT_VARIANT[v];
    *gp = RHS_GP[v];
    *tpb = RHS_PERSIST[v] ? -RHS_TPB[v] : RHS_TPB[v];   // negative: persistent grid
    *wpe = RHS_WPE[v];
    *ptr = RHS_PTR[v] ? 1 : 0;
}

template <int SCH>
static void launch_alt(int variant, int stage, const double *dt, const float *Uin, float *Uout,
                       float *U0, const WorkList &wl, const DevTables &tb, const InstDev *inst,
                       float *FF, int32_t *err, int restrict_parents, double *cflmax, hipStream_t st) {
    switch (ALT_VARIANT[variant]) {
        case 7: launch_variant<7, SCH>(stage, dt, Uin, Uout, U0, wl, tb, inst, FF, err, restrict_parents, cflmax, st); break;
        case 2: launch_variant<2, SCH>(stage, dt, Uin, Uout, U0, wl, tb, inst, FF, err, restrict_parents, cflmax, st); break;
        default: launch_variant<3, SCH>(stage, dt, Uin, Uout, U0, wl, tb, inst, FF, err, restrict_parents, cflmax, st); break;
    }
}

hipError_t launch_rhs_update_f32(int scheme, int variant, int stage, const double *dt, const float *Uin,
                                 float *Uout, float *U0, const WorkList &wl, const DevTables &tb,
                                 const InstDev *inst, float *FF, int32_t *err, int restrict_parents,
                                 double *cflmax, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    if (Uin == Uout) return hipErrorInvalidValue;   // neighbours' interiors are read
    if (variant < 0 || variant >= rhs_variants(scheme)) return hipErrorInvalidValue;
#define MRFV_ARGS stage, dt, Uin, Uout, U0, wl, tb, inst, FF, err, restrict_parents, cflmax, st
    switch (scheme) {
        case SCH_ROE_WENO5:
            switch (variant) {
                case 0: launch_variant<0, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 1: launch_variant<1, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 2: launch_variant<2, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 3: launch_variant<3, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 4: launch_variant<4, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 5: launch_variant<5, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 6: launch_variant<6, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 7: launch_variant<7, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 8: launch_variant<8, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 9: launch_variant<9, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 10: launch_variant<10, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 11: launch_variant<11, SCH_ROE_WENO5>(MRFV_ARGS); break;
                case 12: launch_variant<12, SCH_ROE_WENO5>(MRFV_ARGS); break;
                default: launch_variant<13, SCH_ROE_WENO5>(MRFV_ARGS); break;
            }
            break;
        case SCH_ROE_TENO5: launch_alt<SCH_ROE_TENO5>(variant, MRFV_ARGS); break;
        case SCH_LLF_WENO5: launch_alt<SCH_LLF_WENO5>(variant, MRFV_ARGS); break;
        case SCH_HLLC_WAO53: launch_alt<SCH_HLLC_WAO53>(variant, MRFV_ARGS); break;
        default: return hipErrorInvalidValue;
    }
#undef MRFV_ARGS
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reflux_update(int stage, const double *dt, T *U, const T *FF,
                                const WorkList &wl, const DevTables &tb, const InstDev *inst,
                                hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reflux_update<T>, dim3(wl.grid), dim3(TPB), 0, st, stage, dt, U, FF, wl,
                       tb.meta, tb.nbr, inst);
    return hipGetLastError();
}

#define MRFV_INST_RHS(T)                                                                    \
    template hipError_t launch_flux<T>(int, const T *, const WorkList &, const DevTables &, \
                                       const InstDev *, T *, T *, hipStream_t);             \
    template hipError_t launch_ff_restrict<T>(T *, const WorkList &, const DevTables &,     \
                                              hipStream_t);                                 \
    template hipError_t launch_reflux<T>(T *, const T *, const WorkList &, const DevTables &, \
                                         hipStream_t);                                      \
    template hipError_t launch_combine<T>(const T *, T *, const WorkList &, const DevTables &, \
                                          const InstDev *, const T *, hipStream_t);         \
    template hipError_t launch_update<T>(int, const double *, T *, T *, const T *,          \
                                         const WorkList &, const DevTables &, const InstDev *, \
                                         int32_t *, hipStream_t);                           \
    template hipError_t launch_reflux_update<T>(int, const double *, T *, const T *,        \
                                                const WorkList &, const DevTables &,        \
                                                const InstDev *, hipStream_t);
MRFV_INST_RHS(float)
MRFV_INST_RHS(double)

}  // namespace mrfv
