// kernels_visc.hip -- gfx950 kernels of the viscous terms (Navier-Stokes form of eq:Euler)
// and of their bound on the time step.
//
// The stress is Newtonian with Stokes' hypothesis, tau = mu (grad v + grad v^T) -
// 2/3 mu (div v) I, with a constant dynamic viscosity per instance and no heat conduction
// (the paper's viscous cases give mu only).  The flux through a face normal to axis d is
// Fv = (0, tau_d., tau_d. . v_face), subtracted from the convective flux.  Derivatives at
// a face are second-order central differences: the normal ones from the two cells sharing
// the face, the tangential ones the mean of the two cells' central differences; v_face is
// the mean of the two velocities.
//
// k_visc runs after the convective flux kernel of the plain path and subtracts the viscous
// flux differences from its per-direction differences D and the boundary face fluxes from
// its face planes FF, so that the jump correction averages total fluxes.  Layout and
// thread mapping are the flux kernel's: one workgroup per (leaf, direction), one thread per
// pencil (r, m) along the direction, walking its 17 faces; each cell's velocity and the
// four tangential differences the faces need are computed once and carried from face to
// face.  The tangential neighbours of the halo cells ahead of and behind the pencil lie in
// the edge halo regions, which the plain path fills for viscous contexts.
//
// k_rinv_block / k_visc_dt: the explicit bound of the viscous terms.  Fourier analysis of
// the central operator gives -(40/3) nu / dx^2 for the most negative eigenvalue of the
// momentum part (checkerboard in every axis, the normal component carrying 4/3), and
// SSP-RK3 is stable on the negative real axis up to about 2.51: dt <= cfl * 3/16 * dx^2 /
// (mu * max(1/rho)) keeps cfl <= 1 inside that with a margin.  Per leaf the largest 1/rho
// (FP64), then per instance dt = min(dt of eq:Cfl, that bound) with dx of level lmax.
#include "mrfv_internal.h"

namespace mrfv {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ int pidx(int q, int k, int j, int i) {
    return ((q * NP + k) * NP + j) * NP + i;
}

// Axis roles of direction DIR: the lower and the higher of the two other axes, and the
// padded-index strides of all three.
template <int DIR>
struct VAxes {
    static constexpr int TLO = DIR == 0 ? 1 : 0;
    static constexpr int THI = DIR == 2 ? 1 : 2;
    static constexpr int S_N = DIR == 0 ? 1 : (DIR == 1 ? NP : NP * NP);
    static constexpr int S_LO = TLO == 0 ? 1 : NP;
    static constexpr int S_HI = THI == 1 ? NP : NP * NP;
};

// Per cell along the pencil: velocity and the undivided central differences of the
// components the stress on a DIR face needs (normal and t_lo components along t_lo,
// normal and t_hi components along t_hi).
template <typename T>
struct VCell {
    T v[3];
    T n_lo, lo_lo, n_hi, hi_hi;
};

template <typename T, int DIR>
__device__ __forceinline__ void load_vcell(const T *__restrict__ u, int o, VCell<T> &c) {
    using A = VAxes<DIR>;
    auto vel = [&](int oo, int comp) { return u[oo + (1 + comp) * CELLS_P] / u[oo]; };
#pragma unroll
    for (int k = 0; k < 3; ++k) c.v[k] = vel(o, k);
    c.n_lo = vel(o + A::S_LO, DIR) - vel(o - A::S_LO, DIR);
    c.lo_lo = vel(o + A::S_LO, A::TLO) - vel(o - A::S_LO, A::TLO);
    c.n_hi = vel(o + A::S_HI, DIR) - vel(o - A::S_HI, DIR);
    c.hi_hi = vel(o + A::S_HI, A::THI) - vel(o - A::S_HI, A::THI);
}

// Viscous flux through the face between cells a (low side) and b (high side).
template <typename T, int DIR>
__device__ __forceinline__ void visc_flux(const VCell<T> &a, const VCell<T> &b, T mu, T inv_dx,
                                          bool energy, T F[5]) {
    using A = VAxes<DIR>;
    const T q = (T)0.25 * inv_dx;
    // G[k][a] = d v_k / d x_a at the face, the entries the stress on this face uses
    const T g_nn = (b.v[DIR] - a.v[DIR]) * inv_dx;
    const T g_lon = (b.v[A::TLO] - a.v[A::TLO]) * inv_dx;    // d v_tlo / d x_n
    const T g_hin = (b.v[A::THI] - a.v[A::THI]) * inv_dx;    // d v_thi / d x_n
    const T g_nlo = (a.n_lo + b.n_lo) * q;                  // d v_n / d x_tlo
    const T g_nhi = (a.n_hi + b.n_hi) * q;                  // d v_n / d x_thi
    const T g_lolo = (a.lo_lo + b.lo_lo) * q;
    const T g_hihi = (a.hi_hi + b.hi_hi) * q;
    T dg[3];   // the diagonal of G, summed in axis order
    dg[DIR] = g_nn;
    dg[A::TLO] = g_lolo;
    dg[A::THI] = g_hihi;
    const T div = (dg[0] + dg[1]) + dg[2];
    T tau[3];
    tau[DIR] = mu * (g_nn + g_nn) - (T)(2.0 / 3.0) * mu * div;
    tau[A::TLO] = mu * (g_nlo + g_lon);
    tau[A::THI] = mu * (g_nhi + g_hin);
    F[0] = (T)0;
    T work = (T)0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[1 + j] = tau[j];
        work += tau[j] * ((T)0.5 * (a.v[j] + b.v[j]));
    }
    F[4] = energy ? work : (T)0;
}

template <typename T, int DIR>
__device__ __forceinline__ void visc_pencil(const T *__restrict__ ub, int r, int m, T mu, T inv_dx,
                                            bool energy, T *__restrict__ D, T *__restrict__ FF) {
    using A = VAxes<DIR>;
    int c[3];
    c[DIR] = HW - 1;
    c[A::TLO] = HW + r;
    c[A::THI] = HW + m;
    const int o0 = pidx(0, c[2], c[1], c[0]);
    const int rm = m * NI + r;
    VCell<T> prev, cur;
    load_vcell<T, DIR>(ub, o0, prev);
    T Fp[5];
#pragma unroll 1
    for (int f = 0; f <= NI; ++f) {
        load_vcell<T, DIR>(ub, o0 + (f + 1) * A::S_N, cur);
        T F[5];
        visc_flux<T, DIR>(prev, cur, mu, inv_dx, energy, F);
        if (f == 0 || f == NI) {
            T *ff = FF + (2 * DIR + (f == NI)) * 5 * FACE + rm;
#pragma unroll
            for (int k = 1; k < 5; ++k) ff[k * FACE] -= F[k];
        }
        if (f > 0) {
            const int p = f - 1;
            const int cell = DIR == 0 ? (m * NI + r) * NI + p : (DIR == 1 ? (m * NI + p) * NI + r : (p * NI + m) * NI + r);
            T *d = D + DIR * 5 * CELLS_I + cell;
#pragma unroll
            for (int k = 1; k < 5; ++k) d[k * CELLS_I] -= F[k] - Fp[k];
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) Fp[k] = F[k];
        prev = cur;
    }
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_visc(const T *__restrict__ U, WorkList wl,
                                              const BlockMeta *__restrict__ meta,
                                              const InstDev *__restrict__ inst, T *D, T *FF) {
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int slot = wl.at(b);
        const BlockMeta mt = meta[slot];
        const InstDev &P = inst[mt.inst];
        if (!(P.mu > 0.0)) continue;   // uniform per workgroup
        const T mu = (T)P.mu, inv_dx = (T)(1.0 / ldexp(P.dx0, -mt.level));
        const bool energy = P.eos == 0;
        const int r = threadIdx.x & 15, m = threadIdx.x >> 4;
        const T *ub = U + (size_t)slot * 5 * CELLS_P;
        T *Ds = D + (size_t)slot * 3 * 5 * CELLS_I;
        T *Fs = FF + (size_t)slot * 6 * 5 * FACE;
        if (blockIdx.y == 0) visc_pencil<T, 0>(ub, r, m, mu, inv_dx, energy, Ds, Fs);
        else if (blockIdx.y == 1) visc_pencil<T, 1>(ub, r, m, mu, inv_dx, energy, Ds, Fs);
        else visc_pencil<T, 2>(ub, r, m, mu, inv_dx, energy, Ds, Fs);
    }
}

// Largest 1/rho over a leaf's interior (FP64), stored by the leaf's all-leaves position.
template <typename T>
__global__ __launch_bounds__(TPB) void k_rinv_block(const T *__restrict__ U, WorkList wl,
                                                    const BlockMeta *__restrict__ meta,
                                                    double *__restrict__ bmax) {
    __shared__ double red[TPB / 64];
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int slot = wl.at(b);
        const T *u = U + (size_t)slot * 5 * CELLS_P;
        double mx = 0.0;
        for (int c = threadIdx.x; c < CELLS_I; c += TPB)
            mx = fmax(mx, 1.0 / (double)u[pidx(0, HW + c / FACE, HW + (c / NI) % NI, HW + c % NI)]);
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = red[0];
            for (int w = 1; w < TPB / 64; ++w) v = fmax(v, red[w]);
            bmax[meta[slot].lpos] = v;
        }
        __syncthreads();
    }
}

// One workgroup per instance over its contiguous range of the all-leaves list.
__global__ __launch_bounds__(TPB) void k_visc_dt(WorkList leaves, const int32_t *__restrict__ off,
                                                 const int32_t *__restrict__ cnt,
                                                 const InstDev *__restrict__ inst,
                                                 const double *__restrict__ bmax,
                                                 double *__restrict__ dt) {
    __shared__ double red[TPB / 64];
    const int ins = blockIdx.x;
    const InstDev P = inst[ins];
    if (!(P.mu > 0.0)) return;   // uniform per workgroup
    const int n = cnt[ins];
    const double *bm = bmax + (off[ins] - (leaves.desc ? leaves.desc[0] : leaves.off));
    double mx = 0.0;
    for (int t = threadIdx.x; t < n; t += TPB) mx = fmax(mx, bm[t]);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0 && n > 0) {
        double m = red[0];
        for (int w = 1; w < TPB / 64; ++w) m = fmax(m, red[w]);
        const double dx = ldexp(P.dx0, -P.lmax);
        dt[ins] = fmin(dt[ins], P.cfl * 0.1875 * dx * dx / (P.mu * m));
    }
}

}  // namespace

template <typename T>
hipError_t launch_visc(const T *U, const WorkList &wl, const DevTables &tb, const InstDev *inst,
                       T *D, T *FF, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_visc<T>, dim3(wl.grid, 3), dim3(TPB), 0, st, U, wl, tb.meta, inst, D, FF);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_visc_dt(const T *U, const WorkList &leaves, const DevTables &tb,
                          const InstDev *inst, int n_inst, double *blockmax, double *dt,
                          hipStream_t st) {
    if (leaves.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rinv_block<T>, dim3(leaves.grid), dim3(TPB), 0, st, U, leaves, tb.meta, blockmax);
    // per-instance leaf ranges: the lists array starts with [offsets, counts]
    hipLaunchKernelGGL(k_visc_dt, dim3(n_inst), dim3(TPB), 0, st, leaves, tb.lists, tb.lists + n_inst,
                       inst, blockmax, dt);
    return hipGetLastError();
}

#define MRFV_INST_VISC(T)                                                                    \
    template hipError_t launch_visc<T>(const T *, const WorkList &, const DevTables &,      \
                                       const InstDev *, T *, T *, hipStream_t);             \
    template hipError_t launch_visc_dt<T>(const T *, const WorkList &, const DevTables &,   \
                                          const InstDev *, int, double *, double *, hipStream_t);
MRFV_INST_VISC(float)
MRFV_INST_VISC(double)

}  // namespace mrfv
