// kernels_mr.hip -- gfx950 kernels for the MR operators and reductions.
//
//   prim2cons      initial condition (rho,u,v,w,p) -> conservative state (eq:StiffenedGas)
//   fill_halos     same-level copy / prediction from the parent / zero-gradient clamp
//   project        parents <- average of 8 children (eq:Averaging), FP64 pairwise sums
//   predict        interiors of new children <- prediction from the parent (eq:Prediction)
//   details/flags  Harten details and refine/keep/coarsen flags (eq:DetailFunction,
//                  eq:Thresholding, eq:LevelWiseEpsilon), FP64 arithmetic
//   cfl            eq:Cfl, FP64 max-reduction per block then per instance
//   totals         FP64 sums per block then per instance (fixed order)
//
// The prediction is evaluated in its separable form: the appendix Q-terms are the
// tensor products of the 1D operator D u = c0 (u[+1]-u[-1]) + c1 (u[+2]-u[-2]) with
// c0 = -22/128, c1 = 3/128 (Q_x = D_x u, Q_xy = D_x D_y u, Q_xyz = D_x D_y D_z u), so the
// child value is (1 + s_z D_z)(1 + s_y D_y)(1 + s_x D_x) u, s = +1 for the lower child.
// Written in difference form it reproduces a uniform field exactly.
#include <mutex>

#include "mrfv_internal.h"

namespace mrfv {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int pidx(int q, int k, int j, int i) {
    return ((q * NP + k) * NP + j) * NP + i;
}

// One 1D prediction step in difference form.
template <typename C>
__device__ __forceinline__ C pred1(C m2, C m1, C z0, C p1, C p2, C s) {
    const C c0 = (C)(-22.0 / 128.0), c1 = (C)(3.0 / 128.0);
    return z0 + s * (c0 * (p1 - m1) + c1 * (p2 - m2));
}

// Prediction of child padded cell (i,j,k) (octant o) from one component of the parent's
// padded array pu, evaluated in arithmetic type C.
template <typename C, typename T>
__device__ C predict_cell(const T *__restrict__ pu, int ox, int oy, int oz, int i, int j,
                          int k) {
    const int ci = i - HW, cj = j - HW, ck = k - HW;
    const int I = ox * (NI / 2) + (ci >> 1) + HW;   // arithmetic shift = floor division
    const int J = oy * (NI / 2) + (cj >> 1) + HW;
    const int K = oz * (NI / 2) + (ck >> 1) + HW;
    const C sx = (ci & 1) ? (C)-1 : (C)1;
    const C sy = (cj & 1) ? (C)-1 : (C)1;
    const C sz = (ck & 1) ? (C)-1 : (C)1;
    C r[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        C t[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            const T *row = pu + ((K + c - 2) * NP + (J + b - 2)) * NP + I;
            t[b] = pred1<C>((C)row[-2], (C)row[-1], (C)row[0], (C)row[1], (C)row[2], sx);
        }
        r[c] = pred1<C>(t[0], t[1], t[2], t[3], t[4], sy);
    }
    return pred1<C>(r[0], r[1], r[2], r[3], r[4], sz);
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_prim2cons(const double *__restrict__ prim,
                                                   const int32_t *__restrict__ slots, int n,
                                                   T *__restrict__ U,
                                                   const BlockMeta *__restrict__ meta,
                                                   const InstDev *__restrict__ inst) {
    const int b = blockIdx.x;
    if (b >= n) return;
    const int slot = slots[b];
    const InstDev P = inst[meta[slot].inst];
    const int k = blockIdx.y, j = threadIdx.x >> 4, i = threadIdx.x & 15;
    const double *pr = prim + (size_t)b * 5 * CELLS_I;
    const int c = (k * NI + j) * NI + i;
    const double rho = pr[c], u = pr[CELLS_I + c], v = pr[2 * CELLS_I + c],
                 w = pr[3 * CELLS_I + c], p = pr[4 * CELLS_I + c];
    T *ub = U + (size_t)slot * 5 * CELLS_P;
    const int o = pidx(0, k + HW, j + HW, i + HW);
    ub[o] = (T)rho;
    ub[o + CELLS_P] = (T)(rho * u);
    ub[o + 2 * CELLS_P] = (T)(rho * v);
    ub[o + 3 * CELLS_P] = (T)(rho * w);
    // Tait: the pressure follows from the density and the energy is not evolved
    ub[o + 4 * CELLS_P] = P.eos == 1 ? (T)0
                                     : (T)((p + P.gamma * P.B) / (P.gamma - 1.0) +
                                           0.5 * rho * (u * u + v * v + w * w));
}

// Halo regions.  Region (rx, ry, rz) in {-1, 0, 1}^3 \ {0} covers padded indices
// [0, 4) / [4, 20) / [20, 24) along each axis; in the face modes only the 3 layers the
// flux stencils read ([1, 4) and [20, 23)).  One workgroup per (block, region): a region
// is either copied from the same-level neighbour's interior, clamped at an external
// boundary or predicted from the parent, never a mix.  On a clamped axis the region's
// cells take their values from the block's own cells along that axis: all from the
// boundary cell (zero gradient), or each from its mirror image across the boundary face
// (symmetry, padded index mir - i, with the momentum normal to the boundary reversed).
struct Region {
    int r[3];       // region direction after clamping (0 on clamped axes)
    int lo[3], n[3];
    int clamp[3];   // -1, or the padded index every cell of the axis copies/predicts from
    int mirbits;    // bit a: axis a is clamped at a symmetry boundary, where cell i takes
                    // index mir_index(g, a) - i
    int fix;        // -1, or 4 * side + axis of the last axis (x, y, z order) whose
                    // boundary has fixed values: the region then holds those values
};

__device__ __forceinline__ Region make_region(int mode, int ridx, int zg) {
    Region g;
    g.mirbits = 0;
    int r[3];
    const bool faces = (mode & FILL_FACES) != 0;
    if (!faces) {
        const int reg = ridx < 13 ? ridx : ridx + 1;
        r[0] = reg % 3 - 1;
        r[1] = (reg / 3) % 3 - 1;
        r[2] = reg / 9 - 1;
    } else {
        r[0] = r[1] = r[2] = 0;
        r[ridx >> 1] = (ridx & 1) ? 1 : -1;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = r[a] < 0 ? (faces ? 1 : 0) : (r[a] == 0 ? HW : HW + NI);
        g.n[a] = r[a] == 0 ? NI : (faces ? 3 : HW);
        g.clamp[a] = -1;
        g.r[a] = r[a];
        if (r[a] < 0 && (zg & (1 << (2 * a)))) {
            g.clamp[a] = HW;
            g.r[a] = 0;
            if (zg & (64 << (2 * a))) g.mirbits |= 1 << a;
        }
        if (r[a] > 0 && (zg & (1 << (2 * a + 1)))) {
            g.clamp[a] = HW + NI - 1;
            g.r[a] = 0;
            if (zg & (64 << (2 * a + 1))) g.mirbits |= 1 << a;
        }
    }
    g.fix = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r[a] < 0 && (zg & (4096 << (2 * a)))) g.fix = a;
        if (r[a] > 0 && (zg & (4096 << (2 * a + 1)))) g.fix = 4 + a;
    }
    return g;
}

// Mirror constant of a symmetry-clamped axis: halo cell i of the low side takes padded
// index 2 HW - 1 - i, of the high side 2 (HW + NI) - 1 - i.
__device__ __forceinline__ int mir_index(const Region &g, int a) {
    return g.clamp[a] == HW ? 2 * HW - 1 : 2 * (HW + NI) - 1;
}

// Index decomposition without integer division: e / n for 0 <= e < 2^13 and n <= 24 as
// the truncated product with a reciprocal rounded up by 2^-20 relative (the error stays
// below the 1/n gap to the next integer, so the quotient is exact).
struct Div {
    int n;
    float r;
    __device__ __forceinline__ explicit Div(int n_) : n(n_), r(__frcp_rn((float)n_) * 1.000001f) {}
    __device__ __forceinline__ int quot(int e) const { return (int)((float)e * r); }
};

// Parent padded index of child padded index c in octant half o.
__device__ __forceinline__ int parent_of(int c, int o) { return o * (NI / 2) + ((c - HW) >> 1) + HW; }

// LDS of the separable prediction, sized for the worst of the 26 region shapes: parent
// region (a region spans 16 child cells = 12 parent cells on at most two axes and 2 + 4
// on the others: 12 x 12 x 6), x pass (16 x 12 x 6, or 4 x 12 x 12 for x-normal
// regions), y pass (16 x 16 x 6 for z-normal regions, else 16 x 4 x 12).
constexpr int PR_A = 6 * 12 * 12, PR_X = 16 * 12 * 6, PR_Y = 16 * 16 * 6;

// EXT: the context has symmetry or fixed-value sides; without them the mirror and
// fixed-value code is compiled out (the periodic / zero-gradient fill pays nothing for it).
template <typename T, bool EXT>
__global__ __launch_bounds__(TPB) void k_fill_halos(T *__restrict__ U, WorkList wl,
                                                    const BlockMeta *__restrict__ meta,
                                                    const int32_t *__restrict__ nbr, int mode,
                                                    const T *__restrict__ bcfix) {
    __shared__ T A[PR_A];
    __shared__ T X[PR_X];
    __shared__ T Y[PR_Y];
    const int nb = wl.count();
    const int tid = threadIdx.x;
    const int nreg = (mode & FILL_FACES) ? 6 : 26;
    // blocks in XCD-aware order, as in k_details
    for (int base = 0; base < nb; base += gridDim.x) {
        const int m_round = min(nb - base, (int)gridDim.x);
        const int bi = xcd_item(blockIdx.x, gridDim.x, m_round);
        if (bi >= m_round) continue;   // uniform per workgroup
        const int slot = wl.at(base + bi);
        const BlockMeta m = meta[slot];
        // regions blockIdx.y, blockIdx.y + gridDim.y, ... of the block
        for (int ridx = blockIdx.y; ridx < nreg; ridx += gridDim.y) {
            if ((mode & FILL_MASKED) && !((m.pmask >> ridx) & 1)) continue;   // not read
            const Region g = make_region(mode, ridx, EXT ? m.zg : (m.zg & 63));
            // mirrored axes as bits (no run-time indexing into the region's arrays, which would
            // put them in scratch memory)
            const int mirbits = EXT ? g.mirbits : 0;
            if (EXT && g.fix >= 0) {
                // fixed values: the state of the layer (distance from the face) along the last
                // fixed axis, with the normal momentum of later symmetry axes reversed
                if (!bcfix) continue;
                const int fa = g.fix & 3, fhi = g.fix >> 2;
                const T *fv = bcfix + ((size_t)(m.inst * 6 + 2 * fa + fhi) * MAX_LEVELS + m.level) * 4 * 5;
                T *dst = U + (size_t)slot * 5 * CELLS_P;
                const int ncell = g.n[0] * g.n[1] * g.n[2];
                const Div d0(g.n[0]), d1(g.n[1]);
                const bool re = (mode & FILL_RHO_E) != 0;
                const int flipbits = mirbits & ~((2 << fa) - 1);   // mirrored axes after fa
                for (int e = tid; e < ncell; e += TPB) {
                    const int e1 = d0.quot(e), e2 = d1.quot(e1);
                    const int ci = g.lo[0] + e - e1 * g.n[0], cj = g.lo[1] + e1 - e2 * g.n[1], ck = g.lo[2] + e2;
                    const int cf = fa == 0 ? ci : (fa == 1 ? cj : ck);
                    const int layer = fhi ? cf - (HW + NI) : HW - 1 - cf;
    #pragma unroll
                    for (int q = 0; q < 5; ++q) {
                        if (re && q != 0 && q != 4) continue;
                        const bool flip = q >= 1 && q <= 3 && ((flipbits >> (q - 1)) & 1);
                        const T v = fv[layer * 5 + q];
                        dst[pidx(q, ck, cj, ci)] = flip ? -v : v;
                    }
                }
                continue;
            }
            const bool clamped = g.clamp[0] >= 0 || g.clamp[1] >= 0 || g.clamp[2] >= 0;
            const bool own = g.r[0] == 0 && g.r[1] == 0 && g.r[2] == 0;
            const int src = own ? slot : nbr[(size_t)slot * 27 + (g.r[2] + 1) * 9 + (g.r[1] + 1) * 3 + (g.r[0] + 1)];
            if ((mode & FILL_MISSING) && src >= 0 && !clamped) continue;   // read in place
            if ((mode & FILL_PRESENT) && src < 0) continue;                // keeps its values
            T *dst = U + (size_t)slot * 5 * CELLS_P;
            const int ncell = g.n[0] * g.n[1] * g.n[2];
            const Div dc(ncell), d0(g.n[0]), d1(g.n[1]);
            const bool re = (mode & FILL_RHO_E) != 0;
            const int nq = re ? 2 : 5;
            // symmetry: the momentum component normal to a mirrored boundary changes sign
            // (mirrored on two axes: both components)
            auto msign = [&](int q) {
                return (q >= 1 && q <= 3 && ((mirbits >> (q - 1)) & 1)) ? (T)-1 : (T)1;
            };
            if (src >= 0) {
                const T *sb = U + (size_t)src * 5 * CELLS_P;
                if (mirbits == 0) {   // copies and zero-gradient clamps (uniform per workgroup)
    #pragma unroll 4
                    for (int t = tid; t < nq * ncell; t += TPB) {   // unrolled: several loads in flight
                        const int qi = dc.quot(t), e = t - qi * ncell;
                        const int q = re ? 4 * qi : qi;
                        const int e1 = d0.quot(e), e2 = d1.quot(e1);
                        const int i = g.lo[0] + e - e1 * g.n[0], j = g.lo[1] + e1 - e2 * g.n[1], k = g.lo[2] + e2;
                        const int si = g.clamp[0] >= 0 ? g.clamp[0] : i - NI * g.r[0];
                        const int sj = g.clamp[1] >= 0 ? g.clamp[1] : j - NI * g.r[1];
                        const int sk = g.clamp[2] >= 0 ? g.clamp[2] : k - NI * g.r[2];
                        dst[pidx(q, k, j, i)] = sb[pidx(q, sk, sj, si)];
                    }
                } else {              // some axis mirrored
    #pragma unroll 4
                    for (int t = tid; t < nq * ncell; t += TPB) {
                        const int qi = dc.quot(t), e = t - qi * ncell;
                        const int q = re ? 4 * qi : qi;
                        const int e1 = d0.quot(e), e2 = d1.quot(e1);
                        const int i = g.lo[0] + e - e1 * g.n[0], j = g.lo[1] + e1 - e2 * g.n[1], k = g.lo[2] + e2;
                        const int si = (mirbits & 1) ? mir_index(g, 0) - i : (g.clamp[0] >= 0 ? g.clamp[0] : i - NI * g.r[0]);
                        const int sj = (mirbits & 2) ? mir_index(g, 1) - j : (g.clamp[1] >= 0 ? g.clamp[1] : j - NI * g.r[1]);
                        const int sk = (mirbits & 4) ? mir_index(g, 2) - k : (g.clamp[2] >= 0 ? g.clamp[2] : k - NI * g.r[2]);
                        dst[pidx(q, k, j, i)] = msign(q) * sb[pidx(q, sk, sj, si)];
                    }
                }
                continue;
            }
            if (m.parent < 0) continue;   // level 0 is complete: does not happen
            // prediction from the parent, separably through LDS (x, then y, then z: the
            // operation order of predict_cell)
            const int o[3] = {m.bx & 1, m.by & 1, m.bz & 1};
            int me[3], c0[3], p0[3], np[3];
    #pragma unroll
            for (int a = 0; a < 3; ++a) {
                // evaluation points and the first child index: the boundary cell (zero
                // gradient), the mirror images of the region's cells (symmetry), or the region
                const bool ma = (mirbits >> a) & 1;
                me[a] = ma ? g.n[a] : (g.clamp[a] >= 0 ? 1 : g.n[a]);
                c0[a] = ma ? mir_index(g, a) - (g.lo[a] + g.n[a] - 1) : (g.clamp[a] >= 0 ? g.clamp[a] : g.lo[a]);
                p0[a] = parent_of(c0[a], o[a]) - 2;
                np[a] = parent_of(c0[a] + me[a] - 1, o[a]) + 2 - p0[a] + 1;
            }
            const T *pu = U + (size_t)m.parent * 5 * CELLS_P;
            const Div dp0(np[0]), dp1(np[1]), dm0(me[0]), dm1(me[1]);
            // the parent region of component qi is loaded into registers while component
            // qi - 1 runs its passes (at most PR_A / TPB values per thread)
            constexpr int NAT = (PR_A + TPB - 1) / TPB;
            const int na = np[0] * np[1] * np[2];
            int aoff[NAT];
    #pragma unroll
            for (int n = 0; n < NAT; ++n) {
                const int t = tid + n * TPB;
                const int t1 = dp0.quot(t), kk = dp1.quot(t1);
                const int ii = t - t1 * np[0], jj = t1 - kk * np[1];
                aoff[n] = pidx(0, p0[2] + kk, p0[1] + jj, p0[0] + ii);
            }
            T av[NAT];
            auto load_a = [&](int q) {
    #pragma unroll
                for (int n = 0; n < NAT; ++n)
                    if (tid + n * TPB < na) av[n] = pu[q * CELLS_P + aoff[n]];
            };
            load_a(0);
            for (int qi = 0; qi < nq; ++qi) {
                const int q = re ? 4 * qi : qi;
    #pragma unroll
                for (int n = 0; n < NAT; ++n)
                    if (tid + n * TPB < na) A[tid + n * TPB] = av[n];
                if (qi + 1 < nq) load_a(re ? 4 * (qi + 1) : qi + 1);
                __syncthreads();
                const int nx = np[2] * np[1] * me[0];
                for (int t = tid; t < nx; t += TPB) {
                    const int t1 = dm0.quot(t), kk = dp1.quot(t1);
                    const int ex = t - t1 * me[0], jj = t1 - kk * np[1];
                    const int c = c0[0] + ex;
                    const int I = parent_of(c, o[0]) - p0[0];
                    const T *row = A + (kk * np[1] + jj) * np[0] + I;
                    const T sx = ((c - HW) & 1) ? (T)-1 : (T)1;
                    X[t] = pred1<T>(row[-2], row[-1], row[0], row[1], row[2], sx);
                }
                __syncthreads();
                const int ny = np[2] * me[1] * me[0];
                for (int t = tid; t < ny; t += TPB) {
                    const int t1 = dm0.quot(t), kk = dm1.quot(t1);
                    const int ex = t - t1 * me[0], ey = t1 - kk * me[1];
                    const int c = c0[1] + ey;
                    const int J = parent_of(c, o[1]) - p0[1];
                    const T *col = X + (kk * np[1] + J) * me[0] + ex;
                    const int st = me[0];
                    const T sy = ((c - HW) & 1) ? (T)-1 : (T)1;
                    Y[t] = pred1<T>(col[-2 * st], col[-st], col[0], col[st], col[2 * st], sy);
                }
                __syncthreads();
                for (int t = tid; t < ncell; t += TPB) {
                    const int t1 = d0.quot(t), dz = d1.quot(t1);
                    const int dx = t - t1 * g.n[0], dy = t1 - dz * g.n[1];
                    // evaluation point of the cell: its mirror image runs backwards
                    const int ex = (mirbits & 1) ? g.n[0] - 1 - dx : (g.clamp[0] >= 0 ? 0 : dx);
                    const int ey = (mirbits & 2) ? g.n[1] - 1 - dy : (g.clamp[1] >= 0 ? 0 : dy);
                    const int ez = (mirbits & 4) ? g.n[2] - 1 - dz : (g.clamp[2] >= 0 ? 0 : dz);
                    const int c = c0[2] + ez;
                    const int K = parent_of(c, o[2]) - p0[2];
                    const int st = me[0] * me[1];
                    const T *col = Y + (K * me[1] + ey) * me[0] + ex;
                    const T sz = ((c - HW) & 1) ? (T)-1 : (T)1;
                    dst[pidx(q, g.lo[2] + dz, g.lo[1] + dy, g.lo[0] + dx)] =
                        msign(q) * pred1<T>(col[-2 * st], col[-st], col[0], col[st], col[2 * st], sz);
                }
                __syncthreads();
            }
        }
    }
}

// One thread per parent interior cell; components whose bit is set in qmask.  With skip
// set, octants whose child has meta.srestr (the fused stage kernel wrote their
// restriction) are left as they are.
template <typename T>
__global__ __launch_bounds__(TPB) void k_project(T *__restrict__ U, WorkList wl,
                                                 const int32_t *__restrict__ child,
                                                 const BlockMeta *__restrict__ meta, int qmask,
                                                 int skip) {
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int slot = wl.at(b);
    const int K = blockIdx.y, J = threadIdx.x >> 4, I = threadIdx.x & 15;
    const int oct = ((K >> 3) << 2) | ((J >> 3) << 1) | (I >> 3);
    const int cs = child[(size_t)slot * 8 + oct];
    if (skip && meta[cs].srestr) continue;
    const T *cu = U + (size_t)cs * 5 * CELLS_P;
    T *pu = U + (size_t)slot * 5 * CELLS_P;
    const int ci = HW + 2 * (I & 7), cj = HW + 2 * (J & 7), ck = HW + 2 * (K & 7);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (!((qmask >> q) & 1)) continue;
        const T *c0 = cu + pidx(q, ck, cj, ci);
        const T *c1 = c0 + NP * NP;
        const double s = (((double)c0[0] + (double)c0[1]) + ((double)c0[NP] + (double)c0[NP + 1])) +
                         (((double)c1[0] + (double)c1[1]) + ((double)c1[NP] + (double)c1[NP + 1]));
        pu[pidx(q, HW + K, HW + J, HW + I)] = (T)(s * 0.125);
    }
    }
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_predict(T *__restrict__ U,
                                                 const int32_t *__restrict__ list, int n,
                                                 const BlockMeta *__restrict__ meta) {
    const int b = blockIdx.x;
    if (b >= n) return;
    const int slot = list[b];
    const BlockMeta m = meta[slot];
    const T *pu = U + (size_t)m.parent * 5 * CELLS_P;
    T *cu = U + (size_t)slot * 5 * CELLS_P;
    const int k = blockIdx.y + HW, j = (threadIdx.x >> 4) + HW, i = (threadIdx.x & 15) + HW;
#pragma unroll 1
    for (int q = 0; q < 5; ++q)
        cu[pidx(q, k, j, i)] =
            predict_cell<T, T>(pu + q * CELLS_P, m.bx & 1, m.by & 1, m.bz & 1, i, j, k);
}

__device__ __forceinline__ double eps_level(const InstDev &P, int l) {
    return ldexp(P.eps, -3 * (P.lmax - l));
}

// Prediction of child padded cell (i, j, k) in the form the appendix writes it: the
// parent value plus the signed Q-terms in the order Q_x, Q_y, Q_z, Q_xy, Q_xz, Q_yz,
// Q_xyz, each a weighted sum of sign-alternating differences of the parent's 5^3
// neighbourhood in the appendix's term order, every sum taken left to right and no
// multiply fused with an add.  The terms are walked by loops that are not unrolled, so
// the loads stay few at a time.  Slower than the separable form (125 loads per cell), it
// is used only where a detail lies within a narrow band around its threshold: there the flag is
// decided on this value.
template <typename T>
__device__ double predict_qterms(const T *__restrict__ pu, int ox, int oy, int oz, int i, int j,
                                 int k) {
#pragma clang fp contract(off)
    const int ci = i - HW, cj = j - HW, ck = k - HW;
    const int I = ox * (NI / 2) + (ci >> 1) + HW;
    const int J = oy * (NI / 2) + (cj >> 1) + HW;
    const int K = oz * (NI / 2) + (ck >> 1) + HW;
    const T *pc = pu + (K * NP + J) * NP + I;
    auto u = [&](int off) -> double { return (double)pc[off]; };
    const double c0 = -22.0 / 128.0, c1 = 3.0 / 128.0;
    const int st[3] = {1, NP, NP * NP};
    const double sg[3] = {(ci & 1) ? -1.0 : 1.0, (cj & 1) ? -1.0 : 1.0, (ck & 1) ? -1.0 : 1.0};
    // two-axis groups: offsets (a along the first axis, b along the second) and weights
    const int A2[4] = {1, 2, 1, 2}, B2[4] = {1, 2, 2, 1};
    const double W2[4] = {c0 * c0, c1 * c1, c0 * c1, c1 * c0};
    // three-axis groups (x, y, z offsets) and weights
    const int A3[8] = {1, 2, 1, 2, 1, 2, 1, 2}, B3[8] = {1, 2, 1, 2, 2, 1, 2, 1};
    const int C3[8] = {1, 2, 2, 1, 2, 1, 1, 2};
    const double W3[8] = {c0 * c0 * c0, c1 * c1 * c1, c0 * c0 * c1, c1 * c1 * c0,
                          c0 * c1 * c1, c1 * c0 * c0, c0 * c1 * c0, c1 * c0 * c1};
    const int masks[7] = {1, 2, 4, 3, 5, 6, 7};   // x, y, z, xy, xz, yz, xyz
    double pred = u(0);
#pragma unroll 1
    for (int t = 0; t < 7; ++t) {
        const int mk = masks[t];
        double sign = 1.0;
        int ax[3], na = 0;
        for (int a = 0; a < 3; ++a)
            if (mk & (1 << a)) {
                sign = sign * sg[a];
                ax[na++] = a;
            }
        double q = 0.0;
        if (na == 1) {
            const int o = st[ax[0]];
            q = c0 * (u(o) - u(-o));
            q = q + c1 * (u(2 * o) - u(-2 * o));
        } else if (na == 2) {
#pragma unroll 1
            for (int g = 0; g < 4; ++g) {
                const int a = A2[g] * st[ax[0]], b = B2[g] * st[ax[1]];
                const double cr = (u(a + b) + u(-a - b)) - (u(-a + b) + u(a - b));
                q = g == 0 ? W2[0] * cr : q + W2[g] * cr;
            }
        } else {
#pragma unroll 1
            for (int g = 0; g < 8; ++g) {
                const int a = A3[g], b = B3[g] * NP, c = C3[g] * NP * NP;
                const double gr = (u(a + b + c) - u(-a - b - c)) + (u(-a - b + c) - u(a + b - c)) +
                                  (u(a - b - c) - u(-a + b + c)) + (u(-a + b - c) - u(a - b + c));
                q = g == 0 ? W3[0] * gr : q + W3[g] * gr;
            }
        }
        pred = pred + sign * q;
    }
    return pred;
}

// The band around a level's threshold inside which a slab's detail is recomputed with
// predict_qterms (InstDev::detail_band, 1e-9 unless set otherwise).  The separable and the
// Q-term forms of the prediction differ by a few units in the last place of the
// normalised field values (below 1e-12 for values up to 1e3 times their scale), so
// outside the band both forms fall on the same side of the threshold and the flags equal
// those of the Q-term form everywhere.
constexpr int DETAIL_EXACT_GRID = 64;   // workgroups of k_details_exact (loop over the list)

// Details, FP64.  DZ workgroups per block (level >= 1), each for a slab of 24/DZ padded
// z-planes, write their maxima of the rho and E details over the slab to det4[slot][part];
// the detail of the block is the maximum over its slabs (formed by k_flags).  The prediction is applied separably through LDS, in
// the order z, x, y: the parent planes the slab's stencils touch are staged once, the z
// pass makes the slab's child planes on the parent's (x, y) cells, the x pass the child
// x-cells, and the y pass is evaluated at the output.  Both children of a parent cell
// along the pass axis share the five stencil values and the correction (one step gives
// z0 + corr and z0 - corr), so every stencil is read once per sibling pair.
// Cells outside the interior are read from the same-level neighbour's interior where
// one exists (else from the own halo, filled for such regions).
constexpr int DZ = 6;                          // slabs per block
constexpr int DTPB = 384;                      // threads per workgroup (16 rows of 24 cells)
constexpr int SZ = NP / DZ;                    // padded z-planes per slab (4; even)
constexpr int PZ = SZ / 2 + 4;                 // parent planes per slab (6)

// One 1D prediction step for both siblings: lo = z0 + corr, hi = z0 - corr.
__device__ __forceinline__ void pred_pair(double m2, double m1, double z0, double p1, double p2,
                                          double &lo, double &hi) {
    const double corr = (-22.0 / 128.0) * (p1 - m1) + (3.0 / 128.0) * (p2 - m2);
    lo = z0 + corr;
    hi = z0 - corr;
}

template <typename T>
__global__ __launch_bounds__(DTPB) void k_details(const T *__restrict__ U, WorkList wl,
                                                 const BlockMeta *__restrict__ meta,
                                                 const int32_t *__restrict__ nbr,
                                                 const InstDev *__restrict__ inst,
                                                 double *__restrict__ det4, int32_t *recheck) {
    constexpr int R = NI;                       // parent region edge in x and y (16)
    constexpr int NPAIR = NP / 2;               // sibling pairs along a padded axis (12)
    constexpr int NA = (PZ * R * R + DTPB - 1) / DTPB;        // parent loads per thread (4)
    constexpr int YROWS = SZ * NPAIR;                          // y-pass rows (kc, jp): 48
    constexpr int NY = (YROWS + DTPB / NP - 1) / (DTPB / NP);  // y-pass rows per thread (3)
    __shared__ T A[PZ * R * R];                 // parent planes [kk][jj][ii]
    __shared__ double Cz[SZ * R * R];           // z pass [kc][jj][ii]
    __shared__ double Cx[SZ * R * NP];          // x pass [kc][jj][i]
    __shared__ double red[DTPB / 64];
    __shared__ double slab_max;
    const int nb = wl.count();
    const int part = blockIdx.y;
    const int k_lo = part * SZ;                 // first padded output plane
    const int kk0 = ((k_lo - HW) >> 1) + HW - 2;   // first parent plane (region coordinates)
    const int tid = threadIdx.x, lane = tid & 63;
    const int xi = tid % NP, xr = tid / NP;     // y pass: cell i, first row (16 rows apart)
    const int pi = tid % NPAIR, pr = tid / NPAIR;   // x pass: pair, first row (32 rows apart)
    const int rx = xi < HW ? 0 : (xi < HW + NI ? 1 : 2);
    // blocks in XCD-aware order (gridDim.x is a multiple of 8, so the XCD of a workgroup
    // depends on blockIdx.x alone): list neighbours and siblings share an L2
    for (int base = 0; base < nb; base += gridDim.x) {
    const int m_round = min(nb - base, (int)gridDim.x);
    const int bi = xcd_item(blockIdx.x, gridDim.x, m_round);
    if (bi >= m_round) continue;   // uniform per workgroup
    const int b = base + bi;
    const int slot = wl.at(b);
    const BlockMeta m = meta[slot];
    const InstDev P = inst[m.inst];
    const int ox = m.bx & 1, oy = m.by & 1, oz = m.bz & 1;
    const T *pu = U + (size_t)m.parent * 5 * CELLS_P;
    // Global loads are issued ahead of their use (barriers wait for LDS only): the parent
    // planes of rho and E here, the slab's output cells of rho here and those of E after
    // the rho y pass, so that they arrive during E's z and x passes.  Output cell sources:
    // lane r < 27 of each wavefront holds the element offset of region r (the same-level
    // neighbour shifted onto own padded indices, or the own block), read by shuffles.
    T av[2][NA], uv[NY][2];
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            const int t = tid + n * DTPB;
            if (t < PZ * R * R) {
                const int ii = t & 15, jj = (t >> 4) & 15, kk = t >> 8;
                av[v][n] = pu[4 * v * CELLS_P + pidx(0, oz * 8 + kk0 + kk, oy * 8 + jj, ox * 8 + ii)];
            }
        }
    long long src = (long long)slot * 5 * CELLS_P;
    if (lane < 27) {
        const int ex = lane % 3 - 1, ey = (lane / 3) % 3 - 1, ez = lane / 9 - 1;
        const bool zg = (ex < 0 && (m.zg & 1)) || (ex > 0 && (m.zg & 2)) ||
                        (ey < 0 && (m.zg & 4)) || (ey > 0 && (m.zg & 8)) ||
                        (ez < 0 && (m.zg & 16)) || (ez > 0 && (m.zg & 32));
        const int s = (lane == 13 || zg) ? -1 : nbr[(size_t)slot * 27 + lane];
        if (s >= 0) src = (long long)s * 5 * CELLS_P - NI * (ex + NP * (ey + NP * ez));
    }
    auto load_out = [&](int q) {
#pragma unroll
        for (int n = 0; n < NY; ++n) {
            const int row = min(xr + n * (DTPB / NP), YROWS - 1);
            const int kc = row / NPAIR, jp = row - kc * NPAIR, k = k_lo + kc;
            const int rz = k < HW ? 0 : (k < HW + NI ? 1 : 2);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int j = 2 * jp + h;
                const int ry = j < HW ? 0 : (j < HW + NI ? 1 : 2);
                const long long so = __shfl(src, (rz * 3 + ry) * 3 + rx);
                if (xr + n * (DTPB / NP) < YROWS) uv[n][h] = U[so + q * CELLS_P + pidx(0, k, j, xi)];
            }
        }
    };
    load_out(0);
    double d = 0.0;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        const double inv_s = v == 0 ? 1.0 / P.scale_rho : 1.0 / P.scale_E;
        // parent padded cells (oz*8 + kk0 + kk, oy*8 + jj, ox*8 + ii); A was last read by
        // the previous component's z pass, before its second barrier
#pragma unroll
        for (int n = 0; n < NA; ++n)
            if (tid + n * DTPB < PZ * R * R) A[tid + n * DTPB] = av[v][n];
        __syncthreads();
        // z: child planes 2p, 2p+1 of the slab from parent planes p .. p+4
        for (int t = tid; t < (SZ / 2) * R * R; t += DTPB) {
            const int c = t & (R * R - 1), p = t >> 8;
            const T *a = A + p * R * R + c;
            pred_pair((double)a[0], (double)a[R * R], (double)a[2 * R * R], (double)a[3 * R * R],
                      (double)a[4 * R * R], Cz[2 * p * R * R + c], Cz[(2 * p + 1) * R * R + c]);
        }
        __syncthreads();
        // x: child cells 2ip, 2ip+1 of row (kc, jj) from parent cells ip .. ip+4
        for (int row = pr; row < SZ * R; row += DTPB / NPAIR) {
            const double *a = Cz + row * R + pi;
            pred_pair(a[0], a[1], a[2], a[3], a[4], Cx[row * NP + 2 * pi], Cx[row * NP + 2 * pi + 1]);
        }
        __syncthreads();
        // y at the output: child rows 2jp, 2jp+1 of plane kc, cell i, from Cx rows jp .. jp+4
#pragma unroll
        for (int n = 0; n < NY; ++n) {
            const int row = xr + n * (DTPB / NP);
            if (row < YROWS) {
                const int kc = row / NPAIR, jp = row - kc * NPAIR;
                const double *a = Cx + (kc * R + jp) * NP + xi;
                double pv[2];
                pred_pair(a[0], a[NP], a[2 * NP], a[3 * NP], a[4 * NP], pv[0], pv[1]);
#pragma unroll
                for (int h = 0; h < 2; ++h) d = fmax(d, fabs((double)uv[n][h] - pv[h]) * inv_s);
            }
        }
        if (v == 0) load_out(4);
        // Cz and Cx of the next component are written after its first barrier, which
        // every thread reaches only after this y pass
    }
    // wavefront max, then across the workgroup's waves
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off));
    if ((tid & 63) == 0) red[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) {
        double mx = red[0];
        for (int w = 1; w < DTPB / 64; ++w) mx = fmax(mx, red[w]);
        slab_max = mx;
    }
    __syncthreads();
    if (tid == 0) {
        const double mx = slab_max;
        det4[(size_t)slot * DZ + part] = mx;
        // near the threshold: the slab is evaluated again by k_details_exact
        if (fabs(mx - eps_level(P, m.level)) <= P.detail_band) {
            const int at = atomicAdd(recheck, 1);
            recheck[2 + at] = slot * DZ + part;   // the list holds every slab of every slot
        }
    }
    __syncthreads();
    }
}

// Slabs listed by k_details (their maximum lies within the band around the threshold):
// the maximum again with the Q-term prediction and |u - P| / scale divided, not
// multiplied by the reciprocal, which is how the flags are decided there.  A fixed grid
// loops over the list; the last workgroup to finish clears the list for the next launch.
constexpr int XTPB = 256;
template <typename T>
__global__ __launch_bounds__(XTPB) void k_details_exact(const T *__restrict__ U,
                                                       const BlockMeta *__restrict__ meta,
                                                       const int32_t *__restrict__ nbr,
                                                       const InstDev *__restrict__ inst,
                                                       double *__restrict__ det4,
                                                       int32_t *recheck) {
    __shared__ double red[XTPB / 64];
    __shared__ long long srcs[27];
    const int tid = threadIdx.x;
    const int n = __atomic_load_n(recheck, __ATOMIC_RELAXED);
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int item = recheck[2 + it];
        const int slot = item / DZ, part = item % DZ;
        const BlockMeta m = meta[slot];
        const InstDev P = inst[m.inst];
        const int ox = m.bx & 1, oy = m.by & 1, oz = m.bz & 1;
        const T *pu = U + (size_t)m.parent * 5 * CELLS_P;
        if (tid < 27) {
            // the source of each halo region, as k_details reads it
            const int ex = tid % 3 - 1, ey = (tid / 3) % 3 - 1, ez = tid / 9 - 1;
            const bool zg = (ex < 0 && (m.zg & 1)) || (ex > 0 && (m.zg & 2)) ||
                            (ey < 0 && (m.zg & 4)) || (ey > 0 && (m.zg & 8)) ||
                            (ez < 0 && (m.zg & 16)) || (ez > 0 && (m.zg & 32));
            const int s = (tid == 13 || zg) ? -1 : nbr[(size_t)slot * 27 + tid];
            srcs[tid] = s >= 0 ? (long long)s * 5 * CELLS_P - NI * (ex + NP * (ey + NP * ez))
                               : (long long)slot * 5 * CELLS_P;
        }
        __syncthreads();
        double e = 0.0;
        for (int t = tid; t < SZ * NP * NP; t += XTPB) {
            const int i = t % NP, j = (t / NP) % NP, k = part * SZ + t / (NP * NP);
            const int r = ((k < HW ? 0 : (k < HW + NI ? 1 : 2)) * 3 +
                           (j < HW ? 0 : (j < HW + NI ? 1 : 2))) * 3 +
                          (i < HW ? 0 : (i < HW + NI ? 1 : 2));
            const long long so = srcs[r];
            for (int v = 0; v < 2; ++v) {
                const double uq = (double)U[so + 4 * v * CELLS_P + pidx(0, k, j, i)];
                const double pv = predict_qterms(pu + 4 * v * CELLS_P, ox, oy, oz, i, j, k);
                e = fmax(e, fabs(uq - pv) / (v == 0 ? P.scale_rho : P.scale_E));
            }
        }
        for (int off = 32; off > 0; off >>= 1) e = fmax(e, __shfl_xor(e, off));
        if ((tid & 63) == 0) red[tid >> 6] = e;
        __syncthreads();
        if (tid == 0) {
            double mx = red[0];
            for (int w = 1; w < XTPB / 64; ++w) mx = fmax(mx, red[w]);
            det4[(size_t)slot * DZ + part] = mx;
        }
        __syncthreads();
    }
    // the last workgroup out resets the list (every workgroup has read its count)
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(recheck + 1, 1) == (int)gridDim.x - 1) {
            recheck[0] = 0;
            recheck[1] = 0;
        }
    }
}

// Flags of all listed blocks (2 on non-leaves), from the details' slab maxima; also the
// details themselves (det, blocks on level >= 1) and, when given, copies of the flags and
// of the error word in host memory (read by the host after the stream synchronises).
__global__ __launch_bounds__(TPB) void k_flags(WorkList wl,
                                               const BlockMeta *__restrict__ meta,
                                               const int32_t *__restrict__ child,
                                               const InstDev *__restrict__ inst,
                                               const double *__restrict__ det4,
                                               double *__restrict__ det,
                                               int8_t *__restrict__ flags,
                                               int8_t *__restrict__ flags_host,
                                               const int32_t *__restrict__ err,
                                               int32_t *__restrict__ err_host,
                                               int32_t *__restrict__ gate, int cap) {
    auto detail = [&](int s) {
        const double *p = det4 + (size_t)s * DZ;
        double v = p[0];
#pragma unroll
        for (int k = 1; k < DZ; ++k) v = fmax(v, p[k]);
        return v;
    };
    // with a gate word pair (graph launches): the host buffers' half given by the launch
    // parity, and any refine or coarsen recorded in gate[0] for the next launch's gate
    const int half = gate ? gate[1] : 0;
    if (flags_host) flags_host += (size_t)half * cap;
    if (err_host) err_host += half;
    if (err_host && blockIdx.x == 0 && threadIdx.x == 0) *err_host = *err;
    const int nb = wl.count();
    for (int t = blockIdx.x * TPB + threadIdx.x; t < nb; t += gridDim.x * TPB) {
    const int slot = wl.at(t);
    const BlockMeta m = meta[slot];
    const int l = m.level;
    const double d = l >= 1 ? detail(slot) : -1.0;
    if (l >= 1) det[slot] = d;
    if (!m.leaf) {
        flags[slot] = 2;
        if (flags_host) flags_host[slot] = 2;
        continue;
    }
    const InstDev P = inst[m.inst];
    int8_t f = 0;
    if (!P.adapt) {
        f = 0;
    } else if (l < P.lmax && d >= eps_level(P, l)) {
        f = 1;
    } else if (l >= 2) {
        bool small = true;
        const double e = eps_level(P, l);
        for (int o = 0; o < 8; ++o) {
            const int s = child[(size_t)m.parent * 8 + o];
            if (!meta[s].leaf || !(detail(s) < e)) small = false;
        }
        if (small && detail(m.parent) < eps_level(P, l - 1)) f = -1;
    }
    flags[slot] = f;
    if (flags_host) flags_host[slot] = f;
    if (gate && f != 0) gate[0] = 1;
    }
}

// Per-block maxima of |v_d| + c over the interior, FP64, per z-slab of CZ (workgroup y):
// bmax[lpos][slab][d] by the block's position in the all-leaves list (instance ranges are
// contiguous there); wl may be any list of leaves.
constexpr int CZ = CFL_SLABS;
template <typename T>
__global__ __launch_bounds__(TPB) void k_cfl_block(const T *__restrict__ U, WorkList wl,
                                                   const BlockMeta *__restrict__ meta,
                                                   const InstDev *__restrict__ inst,
                                                   double *__restrict__ bmax) {
    constexpr int NC = CELLS_I / CZ / TPB;   // cells per thread (4)
    __shared__ double red[3][TPB / 64];
    const int nb = wl.count();
    const int part = blockIdx.y;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int slot = wl.at(b);
    const InstDev P = inst[meta[slot].inst];
    const T *u = U + (size_t)slot * 5 * CELLS_P;
    double mx[3] = {0.0, 0.0, 0.0};
    T v[NC][5];
#pragma unroll
    for (int n = 0; n < NC; ++n) {
        const int c = part * (CELLS_I / CZ) + n * TPB + threadIdx.x;
        const int o = pidx(0, HW + c / FACE, HW + (c / NI) % NI, HW + c % NI);
#pragma unroll
        for (int q = 0; q < 5; ++q) v[n][q] = u[o + q * CELLS_P];
    }
#pragma unroll
    for (int n = 0; n < NC; ++n) {
        double sp[3];
        if (P.eos == 1)
            cfl_speeds_tait(v[n][0], v[n][1], v[n][2], v[n][3], P.gamma, P.B, P.tait_rho0, sp);
        else
            cfl_speeds(v[n][0], v[n][1], v[n][2], v[n][3], v[n][4], P.gamma, P.B, sp);
#pragma unroll
        for (int a = 0; a < 3; ++a) mx[a] = fmax(mx[a], sp[a]);
    }
    // maxima over the wavefront, then over the workgroup's waves
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int off = 32; off > 0; off >>= 1) mx[a] = fmax(mx[a], __shfl_xor(mx[a], off));
        if ((threadIdx.x & 63) == 0) red[a][threadIdx.x >> 6] = mx[a];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double m = red[threadIdx.x][0];
        for (int w = 1; w < TPB / 64; ++w) m = fmax(m, red[threadIdx.x][w]);
        bmax[((size_t)meta[slot].lpos * CZ + part) * 3 + threadIdx.x] = m;
    }
    __syncthreads();
    }
}

// One workgroup per instance over that instance's contiguous range of the leaf list (and so
// of the block maxima, stored by list position: leaves_off is the list's start in `list`).
// With gate words (step graphs), workgroup 0 also gates the work-list descriptors that
// the step's later kernels read: desc_g = desc, with every count zero when the previous
// step's flags changed the tree (gate[0]), so that a step launched before the host has
// seen those flags does nothing; it clears gate[0] and flips the launch parity gate[1].
// The CFL launches themselves read the ungated leaf list.
constexpr int CTPB = 1024;   // threads of the per-instance reduction
__global__ __launch_bounds__(CTPB) void k_cfl_inst(WorkList leaves,
                                                   const int32_t *__restrict__ off,
                                                   const int32_t *__restrict__ cnt,
                                                   const InstDev *__restrict__ inst,
                                                   const double *__restrict__ bmax,
                                                   double *__restrict__ dt,
                                                   int32_t *__restrict__ gate,
                                                   const int32_t *__restrict__ desc,
                                                   int32_t *__restrict__ desc_g, int n_desc) {
    __shared__ double red[3][CTPB / 64];
    __shared__ int32_t changed;
    const int ins = blockIdx.x;
    if (gate && ins == 0) {
        if (threadIdx.x == 0) changed = gate[0];
        __syncthreads();
        for (int i = threadIdx.x; i < n_desc; i += CTPB) {
            desc_g[2 * i] = desc[2 * i];
            desc_g[2 * i + 1] = changed ? 0 : desc[2 * i + 1];
        }
        if (threadIdx.x == 0) {
            gate[0] = 0;
            gate[1] ^= 1;
        }
    }
    double mx[3] = {0.0, 0.0, 0.0};
    const int n = cnt[ins] * CZ;
    const double *bm = bmax + (size_t)(off[ins] - (leaves.desc ? leaves.desc[0] : leaves.off)) * CZ * 3;
#pragma unroll 4
    for (int t = threadIdx.x; t < n; t += CTPB)
#pragma unroll
        for (int a = 0; a < 3; ++a) mx[a] = fmax(mx[a], bm[(size_t)t * 3 + a]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int o = 32; o > 0; o >>= 1) mx[a] = fmax(mx[a], __shfl_xor(mx[a], o));
        if ((threadIdx.x & 63) == 0) red[a][threadIdx.x >> 6] = mx[a];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m[a] = red[a][0];
            for (int w = 1; w < CTPB / 64; ++w) m[a] = fmax(m[a], red[a][w]);
        }
        // the three directional maxima are added in ascending order: dt does not depend
        // on the labelling of the axes
        const double lo = fmin(fmin(m[0], m[1]), m[2]), hi = fmax(fmax(m[0], m[1]), m[2]);
        const double mid = fmax(fmin(m[0], m[1]), fmin(fmax(m[0], m[1]), m[2]));   // median
        const double s = (lo + mid) + hi;
        const InstDev P = inst[ins];
        const double dx = ldexp(P.dx0, -P.lmax);
        if (n > 0) dt[ins] = P.cfl * dx / s;
    }
}

// Per-block FP64 sums of the 5 conserved quantities over the interior (fixed tree).
template <typename T>
__global__ __launch_bounds__(TPB) void k_sum_block(const T *__restrict__ U, WorkList wl,
                                                   double *__restrict__ bsum) {
    __shared__ double red[TPB];
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
    const int slot = wl.at(b);
    const T *u = U + (size_t)slot * 5 * CELLS_P;
    for (int q = 0; q < 5; ++q) {
        double s = 0.0;
        for (int c = threadIdx.x; c < CELLS_I; c += TPB)
            s += (double)u[pidx(q, HW + c / FACE, HW + (c / NI) % NI, HW + c % NI)];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = TPB / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) bsum[(size_t)slot * 5 + q] = red[0];
        __syncthreads();
    }
    }
}

__global__ __launch_bounds__(TPB) void k_sum_inst(const int32_t *__restrict__ list,
                                                  const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ cnt,
                                                  const BlockMeta *__restrict__ meta,
                                                  const InstDev *__restrict__ inst,
                                                  const double *__restrict__ bsum,
                                                  double *__restrict__ tot) {
    __shared__ double red[TPB];
    const int ins = blockIdx.x;
    const InstDev P = inst[ins];
    for (int q = 0; q < 5; ++q) {
        double s = 0.0;
        for (int t = threadIdx.x; t < cnt[ins]; t += TPB) {
            const int slot = list[off[ins] + t];
            const double dx = ldexp(P.dx0, -meta[slot].level);
            s += bsum[(size_t)slot * 5 + q] * (dx * dx * dx);
        }
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = TPB / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot[ins * 5 + q] = red[0];
        __syncthreads();
    }
}

inline dim3 grid2(int n, int y) { return dim3((unsigned)n, (unsigned)y, 1); }

}  // namespace

template <typename T>
hipError_t launch_prim2cons(const double *prim, const int32_t *slots, int n, T *U,
                            const BlockMeta *meta, const InstDev *inst, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prim2cons<T>, grid2(n, NI), dim3(TPB), 0, st, prim, slots, n, U, meta, inst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_halos(T *U, const WorkList &wl, const DevTables &tb, FillMode mode,
                             hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    // one workgroup per region, except in the mode before the details (all 26 regions of
    // the jump leaves, most of them read in place and skipped): two per block, 13 regions
    // each (0.42 -> 0.38 ms per step of config 5; one workgroup per block in the stages'
    // missing-faces mode measured no faster)
    const int nreg = (mode & FILL_FACES) ? 6 : 26;
    const int gy = ((mode & FILL_MISSING) && !(mode & FILL_FACES)) ? 2 : nreg;
    const dim3 grid = grid2(round_xcd(wl.grid), gy);
    if (tb.ext_bc)
        hipLaunchKernelGGL((k_fill_halos<T, true>), grid, dim3(TPB), 0, st, U, wl, tb.meta, tb.nbr, (int)mode,
                           (const T *)tb.bcfix);
    else
        hipLaunchKernelGGL((k_fill_halos<T, false>), grid, dim3(TPB), 0, st, U, wl, tb.meta, tb.nbr, (int)mode,
                           (const T *)nullptr);
    return hipGetLastError();
}


template <typename T>
hipError_t launch_project(T *U, const WorkList &wl, const DevTables &tb, hipStream_t st,
                          int qmask, bool skip_srestr) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_project<T>, grid2(wl.grid, NI), dim3(TPB), 0, st, U, wl, tb.child, tb.meta,
                       qmask, skip_srestr ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_predict(T *U, const int32_t *list, int n, const DevTables &tb,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_predict<T>, grid2(n, NI), dim3(TPB), 0, st, U, list, n, tb.meta);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_details(const T *U, const WorkList &wl, const DevTables &tb,
                          const InstDev *inst, double *det4, int32_t *recheck, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_details<T>, grid2(round_xcd(wl.grid), DZ), dim3(DTPB), 0, st, U, wl,
                       tb.meta, tb.nbr, inst, det4, recheck);
    hipLaunchKernelGGL(k_details_exact<T>, dim3(DETAIL_EXACT_GRID), dim3(XTPB), 0, st, U, tb.meta,
                       tb.nbr, inst, det4, recheck);
    return hipGetLastError();
}

int details_parts() { return DZ; }

hipError_t launch_flags(const WorkList &wl, const DevTables &tb, const InstDev *inst,
                        const double *det4, double *det, int8_t *flags, int8_t *flags_host,
                        const int32_t *err, int32_t *err_host, int32_t *gate, int cap,
                        hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flags, dim3((wl.grid + TPB - 1) / TPB), dim3(TPB), 0, st, wl, tb.meta,
                       tb.child, inst, det4, det, flags, flags_host, err, err_host, gate, cap);
    return hipGetLastError();
}


template <typename T>
hipError_t launch_cfl(const T *U, const WorkList &leaves, const DevTables &tb,
                      const InstDev *inst, int n_inst, double *blockmax, double *dt,
                      hipStream_t st, int32_t *gate, const int32_t *desc, int32_t *desc_g,
                      int n_desc) {
    if (leaves.grid <= 0 && !gate) return hipSuccess;
    if (leaves.grid > 0)
        hipLaunchKernelGGL(k_cfl_block<T>, grid2(leaves.grid, CZ), dim3(TPB), 0, st, U, leaves,
                           tb.meta, inst, blockmax);
    // per-instance leaf ranges: the lists array starts with [offsets, counts]
    hipLaunchKernelGGL(k_cfl_inst, dim3(n_inst), dim3(CTPB), 0, st, leaves, tb.lists,
                       tb.lists + n_inst, inst, blockmax, dt, gate, desc, desc_g, n_desc);
    return hipGetLastError();
}

int cfl_slabs() { return CZ; }

template <typename T>
hipError_t launch_cfl_blocks(const T *U, const WorkList &wl, const DevTables &tb,
                             const InstDev *inst, double *blockmax, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cfl_block<T>, grid2(wl.grid, CZ), dim3(TPB), 0, st, U, wl, tb.meta, inst,
                       blockmax);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_totals(const T *U, const WorkList &leaves, const DevTables &tb,
                         const InstDev *inst, int n_inst, double *blocksum, double *tot,
                         hipStream_t st) {
    if (leaves.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_block<T>, dim3(leaves.grid), dim3(TPB), 0, st, U, leaves, blocksum);
    hipLaunchKernelGGL(k_sum_inst, dim3(n_inst), dim3(TPB), 0, st, tb.lists, tb.lists,
                       tb.lists + n_inst, tb.meta, inst, blocksum, tot);
    return hipGetLastError();
}

// Per-slot FP64 partial sums of mrfv_totals_noalloc, for callers that cannot allocate:
// a file-scope device array of STATIC_TOTALS_SLOTS * 5 doubles (2.6 MB, held by every
// device the library runs on until the process ends).  Host code never passes the
// array's name to a kernel: it is a host-side stand-in, not a device address.  The
// device address is looked up once per device (static_totals_scratch) and kept.
constexpr int STATIC_TOTALS_SLOTS = 65536;
static __device__ __align__(256) double scratch[(size_t)STATIC_TOTALS_SLOTS * 5];

int static_totals_slots() { return STATIC_TOTALS_SLOTS; }

hipError_t static_totals_scratch(int device, double **ptr) {
    constexpr int MAX_DEV = 64;
    static std::mutex mu;
    static double *addr[MAX_DEV] = {};
    if (device < 0 || device >= MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // resolved with the device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = (double *)p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

#define MRFV_INST(T)                                                                        \
    template hipError_t launch_prim2cons<T>(const double *, const int32_t *, int, T *,     \
                                            const BlockMeta *, const InstDev *, hipStream_t); \
    template hipError_t launch_fill_halos<T>(T *, const WorkList &, const DevTables &,       \
                                             FillMode, hipStream_t);                        \
    template hipError_t launch_project<T>(T *, const WorkList &, const DevTables &,         \
                                          hipStream_t, int, bool);                          \
    template hipError_t launch_predict<T>(T *, const int32_t *, int, const DevTables &,    \
                                          hipStream_t);                                     \
    template hipError_t launch_details<T>(const T *, const WorkList &, const DevTables &,   \
                                          const InstDev *, double *, int32_t *, hipStream_t); \
    template hipError_t launch_cfl<T>(const T *, const WorkList &, const DevTables &,       \
                                      const InstDev *, int, double *, double *, hipStream_t, \
                                      int32_t *, const int32_t *, int32_t *, int);          \
    template hipError_t launch_cfl_blocks<T>(const T *, const WorkList &, const DevTables &, \
                                             const InstDev *, double *, hipStream_t);      \
    template hipError_t launch_totals<T>(const T *, const WorkList &, const DevTables &,    \
                                         const InstDev *, int, double *, double *, hipStream_t);
MRFV_INST(float)
MRFV_INST(double)

}  // namespace mrfv
