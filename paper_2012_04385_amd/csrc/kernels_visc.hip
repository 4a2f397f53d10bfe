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
// its face planes FF, so that the jump correction averages total fluxes.  It walks the
// z-planes of a leaf with the velocities of three planes in LDS (coalesced row loads, one
// division per cell and plane pass) and evaluates all three face directions there.  The
// tangential neighbours of the halo cells beside the faces lie in the edge halo regions,
// which the plain path fills for viscous contexts.
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

// Axis roles of direction DIR: the lower and the higher of the two other axes.
template <int DIR>
struct VAxes {
    static constexpr int TLO = DIR == 0 ? 1 : 0;
    static constexpr int THI = DIR == 2 ? 1 : 2;
};

// Per cell beside a DIR face: velocity and the undivided central differences of the
// components the stress on the face needs (normal and t_lo components along t_lo, normal
// and t_hi components along t_hi).
template <typename T>
struct VCell {
    T v[3];
    T n_lo, lo_lo, n_hi, hi_hi;
};

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

// One workgroup per (leaf, z-slab of 4 planes), 16 x 16 threads on the (x, y) cells of a
// z-plane, walking the slab's planes.  The velocities of three consecutive planes (z - 1, z, z + 1, each 18 x 18 with
// the one-cell halo ring) sit in LDS, loaded once per plane with coalesced rows; every
// derivative is then two LDS reads.  Per plane a thread evaluates the x-face on the left of
// its cell, the y-face below it and the z-face below the plane (the last column / row /
// plane also the far faces), the x- and y-face fluxes go through LDS to form the
// differences, the z-face flux is carried from plane to plane in registers (the face
// between two slabs is evaluated by both).
constexpr int VR = NI + 2;            // 18: a plane with its halo ring
constexpr int VPL = VR * VR;          // 324 cells
constexpr int VSLABS = 4;             // z-slabs per leaf (workgroups): enough workgroups
constexpr int VSZ = NI / VSLABS;      // to fill the chip on a few hundred leaves

template <typename T>
struct VisLds {
    T v[3][3][VPL];                   // [ring slot][component][(y + 1) * 18 + x + 1]
    T fx[4][NI][NI + 1];              // x-face fluxes (components 1..4) [y][face]
    T fy[4][NI + 1][NI];              // y-face fluxes [face][x]
};

template <typename T>
__device__ __forceinline__ T vat(const VisLds<T> &L, int slot, int comp, int x, int y) {
    return L.v[slot][comp][(y + 1) * VR + x + 1];
}

// The per-cell record of a DIR face: velocity and the undivided central differences along
// the two tangential axes, from the ring (slots of planes z - 1, z, z + 1 for the cell's z).
template <typename T, int DIR>
__device__ __forceinline__ void cell_rec(const VisLds<T> &L, int zm, int z0, int zp, int x, int y,
                                         VCell<T> &c) {
    using A = VAxes<DIR>;
#pragma unroll
    for (int k = 0; k < 3; ++k) c.v[k] = vat(L, z0, k, x, y);
    // difference of component `comp` along axis `ax` (0 x, 1 y, 2 z)
    auto dif = [&](int comp, int ax) {
        if (ax == 0) return vat(L, z0, comp, x + 1, y) - vat(L, z0, comp, x - 1, y);
        if (ax == 1) return vat(L, z0, comp, x, y + 1) - vat(L, z0, comp, x, y - 1);
        return vat(L, zp, comp, x, y) - vat(L, zm, comp, x, y);
    };
    c.n_lo = dif(DIR, A::TLO);
    c.lo_lo = dif(A::TLO, A::TLO);
    c.n_hi = dif(DIR, A::THI);
    c.hi_hi = dif(A::THI, A::THI);
}

template <typename T>
__device__ __forceinline__ void load_plane(const T *__restrict__ ub, VisLds<T> &L, int zz, int tid) {
    const int sl = (zz + 3) % 3;
    for (int c = tid; c < VPL; c += TPB) {
        const int x = c % VR - 1, y = c / VR - 1;
        const int o = pidx(0, HW + zz, HW + y, HW + x);
        const T r = ub[o];
#pragma unroll
        for (int k = 0; k < 3; ++k) L.v[sl][k][c] = ub[o + (1 + k) * CELLS_P] / r;
    }
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_visc(const T *__restrict__ U, WorkList wl,
                                              const BlockMeta *__restrict__ meta,
                                              const InstDev *__restrict__ inst, T *D, T *FF) {
    __shared__ VisLds<T> L;
    const int nb = wl.count();
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int z0s = blockIdx.y * VSZ, z1s = z0s + VSZ;   // this workgroup's planes [z0s, z1s)
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int slot = wl.at(b);
        const BlockMeta mt = meta[slot];
        const InstDev &P = inst[mt.inst];
        if (!(P.mu > 0.0)) continue;   // uniform per workgroup
        const T mu = (T)P.mu, inv_dx = (T)(1.0 / ldexp(P.dx0, -mt.level));
        const bool energy = P.eos == 0;
        const T *ub = U + (size_t)slot * 5 * CELLS_P;
        T *Ds = D + (size_t)slot * 3 * 5 * CELLS_I;
        T *Fs = FF + (size_t)slot * 6 * 5 * FACE;
        load_plane(ub, L, z0s - 1, tid);
        load_plane(ub, L, z0s, tid);
        T Fz[5];   // the z-face below the current plane
#pragma unroll 1
        for (int z = z0s; z < z1s; ++z) {
            load_plane(ub, L, z + 1, tid);
            __syncthreads();
            const int zm = (z + 2) % 3, z0 = z % 3, zp = (z + 1) % 3;   // slots of z - 1, z, z + 1
            VCell<T> a, c;
            T F[5];
            // x-faces: left of the cell, and the far face for the last column
            cell_rec<T, 0>(L, zm, z0, zp, tx - 1, ty, a);
            cell_rec<T, 0>(L, zm, z0, zp, tx, ty, c);
            visc_flux<T, 0>(a, c, mu, inv_dx, energy, F);
#pragma unroll
            for (int k = 0; k < 4; ++k) L.fx[k][ty][tx] = F[k + 1];
            if (tx == NI - 1) {
                cell_rec<T, 0>(L, zm, z0, zp, NI, ty, a);
                visc_flux<T, 0>(c, a, mu, inv_dx, energy, F);
#pragma unroll
                for (int k = 0; k < 4; ++k) L.fx[k][ty][NI] = F[k + 1];
            }
            // y-faces: below the cell, and the far face for the last row
            cell_rec<T, 1>(L, zm, z0, zp, tx, ty - 1, a);
            cell_rec<T, 1>(L, zm, z0, zp, tx, ty, c);
            visc_flux<T, 1>(a, c, mu, inv_dx, energy, F);
#pragma unroll
            for (int k = 0; k < 4; ++k) L.fy[k][ty][tx] = F[k + 1];
            if (ty == NI - 1) {
                cell_rec<T, 1>(L, zm, z0, zp, tx, NI, a);
                visc_flux<T, 1>(c, a, mu, inv_dx, energy, F);
#pragma unroll
                for (int k = 0; k < 4; ++k) L.fy[k][NI][tx] = F[k + 1];
            }
            // z-face below the plane, between cells (x, y, z - 1) and (x, y, z): a z-face
            // needs differences along x and y only
            {
                VCell<T> lo, hi;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    lo.v[k] = vat(L, zm, k, tx, ty);
                    hi.v[k] = vat(L, z0, k, tx, ty);
                }
                // tangential axes of a z-face: x (t_lo) and y (t_hi)
                lo.n_lo = vat(L, zm, 2, tx + 1, ty) - vat(L, zm, 2, tx - 1, ty);
                lo.lo_lo = vat(L, zm, 0, tx + 1, ty) - vat(L, zm, 0, tx - 1, ty);
                lo.n_hi = vat(L, zm, 2, tx, ty + 1) - vat(L, zm, 2, tx, ty - 1);
                lo.hi_hi = vat(L, zm, 1, tx, ty + 1) - vat(L, zm, 1, tx, ty - 1);
                hi.n_lo = vat(L, z0, 2, tx + 1, ty) - vat(L, z0, 2, tx - 1, ty);
                hi.lo_lo = vat(L, z0, 0, tx + 1, ty) - vat(L, z0, 0, tx - 1, ty);
                hi.n_hi = vat(L, z0, 2, tx, ty + 1) - vat(L, z0, 2, tx, ty - 1);
                hi.hi_hi = vat(L, z0, 1, tx, ty + 1) - vat(L, z0, 1, tx, ty - 1);
                T Fn[5];
                visc_flux<T, 2>(lo, hi, mu, inv_dx, energy, Fn);
                const int rm = ty * NI + tx;   // z-face planes: r = x, m = y
                if (z == 0) {
#pragma unroll
                    for (int k = 1; k < 5; ++k) Fs[(4 * 5 + k) * FACE + rm] -= Fn[k];
                } else if (z > z0s) {   // the slab's first face only starts the carry
                    const int cell = ((z - 1) * NI + ty) * NI + tx;
#pragma unroll
                    for (int k = 1; k < 5; ++k) Ds[(2 * 5 + k) * CELLS_I + cell] -= Fn[k] - Fz[k];
                }
#pragma unroll
                for (int k = 0; k < 5; ++k) Fz[k] = Fn[k];
                if (z == z1s - 1) {
                    // the slab's far z-face, between planes z and z + 1 (slot zp)
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        lo.v[k] = hi.v[k];
                        hi.v[k] = vat(L, zp, k, tx, ty);
                    }
                    lo.n_lo = hi.n_lo;
                    lo.lo_lo = hi.lo_lo;
                    lo.n_hi = hi.n_hi;
                    lo.hi_hi = hi.hi_hi;
                    hi.n_lo = vat(L, zp, 2, tx + 1, ty) - vat(L, zp, 2, tx - 1, ty);
                    hi.lo_lo = vat(L, zp, 0, tx + 1, ty) - vat(L, zp, 0, tx - 1, ty);
                    hi.n_hi = vat(L, zp, 2, tx, ty + 1) - vat(L, zp, 2, tx, ty - 1);
                    hi.hi_hi = vat(L, zp, 1, tx, ty + 1) - vat(L, zp, 1, tx, ty - 1);
                    visc_flux<T, 2>(lo, hi, mu, inv_dx, energy, Fn);
                    const int cell = (z * NI + ty) * NI + tx;
#pragma unroll
                    for (int k = 1; k < 5; ++k) {
                        Ds[(2 * 5 + k) * CELLS_I + cell] -= Fn[k] - Fz[k];
                        if (z == NI - 1) Fs[(5 * 5 + k) * FACE + rm] -= Fn[k];
                    }
                }
            }
            __syncthreads();
            // x and y differences of the cell, boundary face planes of the x and y sides
            const int cell = (z * NI + ty) * NI + tx;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                Ds[(0 * 5 + 1 + k) * CELLS_I + cell] -= L.fx[k][ty][tx + 1] - L.fx[k][ty][tx];
                Ds[(1 * 5 + 1 + k) * CELLS_I + cell] -= L.fy[k][ty + 1][tx] - L.fy[k][ty][tx];
            }
            if (tx == 0 || tx == NI - 1) {   // x-face planes: r = y, m = z
                const int side = tx == 0 ? 0 : 1, f = tx == 0 ? 0 : NI;
#pragma unroll
                for (int k = 0; k < 4; ++k) Fs[(side * 5 + 1 + k) * FACE + z * NI + ty] -= L.fx[k][ty][f];
            }
            if (ty == 0 || ty == NI - 1) {   // y-face planes: r = x, m = z
                const int side = ty == 0 ? 2 : 3, f = ty == 0 ? 0 : NI;
#pragma unroll
                for (int k = 0; k < 4; ++k) Fs[(side * 5 + 1 + k) * FACE + z * NI + tx] -= L.fy[k][f][tx];
            }
            __syncthreads();   // the ring slot of z - 1 and the face arrays are reused
        }
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
    hipLaunchKernelGGL(k_visc<T>, dim3(wl.grid, VSLABS), dim3(TPB), 0, st, U, wl, tb.meta, inst, D, FF);
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
