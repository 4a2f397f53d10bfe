// kernels_lts.hip -- gfx950 kernels of local time stepping (eq:LtsTimestep,
// algo:ComputeLoop, algo:Integration).
//
// Level l advances with its own step dt_l = 2^(lmax - l) dt, dt being the eq:Cfl step of
// level lmax.  Per RK stage of a level's step the host runs the plain flux kernels on the
// leaves being evaluated, then
//   lts_combine  the flux divergence of those leaves (from the flux kernel's differences)
//                into the padded field F, whose parents (eq:Averaging) and halos at
//                resolution jumps (eq:Prediction) are built by the state's own kernels
//                (project, fill_halos) applied to F;
//   lts_update   the SSP-RK3 stage of the interior cells and of the halo cells of faces
//                without a same-level neighbour (integrated with the predicted flux
//                divergence, algo:Integration), and the stage's boundary face fluxes added
//                to per-face sums with the stage's weight in the RK scheme (only on the
//                faces a coarse cell adjustment reads);
//   lts_adjust   the coarse cell adjustment at the end of a coarse leaf's step: on faces
//                whose same-level neighbour is refined, the own time-integrated flux is
//                replaced by the area average of the fine sums (built by k_ff_restrict);
//   lts_zero     sums that a coarse leaf has used start again.
// All kernels are memory-bound streams over whole blocks: one workgroup per block part,
// coalesced along x.
#include "mrfv_internal.h"

namespace mrfv {

namespace {

constexpr int TPB = 256;                  // one thread per cell of a z-plane
constexpr int SLAB = 3 * FACE;            // halo cells of one face that the flux reads
// The stage update runs four workgroups per leaf, each over four interior z-planes (its
// loads issued together) and six of the leaf's 24 face pieces (18 halo layers, 6 face-flux
// sums), most of which are skipped: one workgroup per plane and piece took 41 % longer in
// FP32 (27 % in FP64), most of it in starting workgroups that had little or nothing to do.
// The combine keeps one workgroup per z-plane (with four planes each it took 7 % longer,
// at three waves per SIMD instead of eight).
constexpr int PLANES = 4;
constexpr int PARTS = NI / PLANES;
constexpr int PIECES = (6 * 3 + 6) / PARTS;
static_assert(NI % PLANES == 0 && (6 * 3 + 6) % PARTS == 0, "parts must tile the leaf");

__device__ __forceinline__ int pidx(int q, int k, int j, int i) {
    return ((q * NP + k) * NP + j) * NP + i;
}

__device__ __forceinline__ int face_region(int side) {
    const int d = side >> 1, s = (side & 1) ? 1 : -1;
    int r[3] = {0, 0, 0};
    r[d] = s;
    return (r[2] + 1) * 9 + (r[1] + 1) * 3 + (r[0] + 1);
}

// Padded index of cell (m, r) of the plane `p` along axis d: r runs along the lower of the
// two other axes, m along the higher one (the layout of the boundary face fluxes).
__device__ __forceinline__ int plane_cell(int q, int d, int p, int m, int r) {
    int c[3];
    c[d] = p;
    c[d == 0 ? 1 : 0] = HW + r;
    c[d == 2 ? 1 : 2] = HW + m;
    return pidx(q, c[2], c[1], c[0]);
}

template <typename T>
__device__ __forceinline__ T lts_stage_coef(int stage) {
    return stage == 0 ? (T)1 : (stage == 1 ? (T)0.25 : (T)(2.0 / 3.0));
}

template <typename T>
__device__ __forceinline__ bool lts_physical(const T u[5], const InstDev &P) {
    if (P.eos == 1) return u[0] > (T)0 && isfinite(u[1] + u[2] + u[3]);   // Tait
    const T g = (T)P.gamma, B = (T)P.B;
    const T ke = (T)0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
    const T p = (g - (T)1) * (u[4] - ke) - g * B;
    return u[0] > (T)0 && p + B > (T)0 && isfinite(u[4]) && isfinite(u[1] + u[2] + u[3]);
}

// The flux divergence of a leaf, L = -(D_x + D_y + D_z) / dx plus the gravity source of
// eq:Euler (the plain path's combine, in the same operation order), written into the
// padded field F.
template <typename T>
__global__ __launch_bounds__(TPB) void k_lts_combine(const T *__restrict__ D, T *__restrict__ F, WorkList wl,
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
        const int c = blockIdx.y * TPB + threadIdx.x;
        const int o = ((c / FACE + HW) * NP + (c / NI) % NI + HW) * NP + c % NI + HW;
        T l[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T s = (Ds[q * CELLS_I + c] + Ds[(5 + q) * CELLS_I + c]) + Ds[(10 + q) * CELLS_I + c];
            l[q] = -s * inv_dx;
        }
        if (P.has_source) {   // uniform per workgroup
            const T *ub = U + (size_t)slot * 5 * CELLS_P;
            T u[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) u[q] = ub[o + q * CELLS_P];
            const T gx = (T)P.gravity[0], gy = (T)P.gravity[1], gz = (T)P.gravity[2];
            l[1] = fma(u[0], gx, l[1]);
            l[2] = fma(u[0], gy, l[2]);
            l[3] = fma(u[0], gz, l[3]);
            l[4] += fma(u[3], gz, fma(u[2], gy, u[1] * gx));
        }
        T *fs = F + (size_t)slot * 5 * CELLS_P;
#pragma unroll
        for (int q = 0; q < 5; ++q) fs[q * CELLS_P + o] = l[q];
    }
}

// blockIdx.y = part: interior z-planes [PLANES * part, PLANES * (part + 1)) and face pieces
// [PIECES * part, PIECES * (part + 1)) of 24: side * 3 + halo layer for pieces below 18,
// then the face-flux sums of one side.
template <typename T>
__global__ __launch_bounds__(TPB) void k_lts_update(int stage, const double *__restrict__ dt,
                                                    T *U, T *U0, T *H0, const T *__restrict__ F,
                                                    const T *__restrict__ FF, T *ACC, WorkList wl,
                                                    const BlockMeta *__restrict__ meta,
                                                    const int32_t *__restrict__ nbr,
                                                    const InstDev *__restrict__ inst,
                                                    int32_t *err) {
    const int nb_ = wl.count();
    const int part = blockIdx.y, tid = threadIdx.x;
    for (int b = blockIdx.x; b < nb_; b += gridDim.x) {
        const int slot = wl.at(b);
        const BlockMeta mt = meta[slot];
        const InstDev &P = inst[mt.inst];
        const double dtl = ldexp(dt[mt.inst], P.lmax - mt.level);
        const T a = lts_stage_coef<T>(stage);
        T *ub = U + (size_t)slot * 5 * CELLS_P;
        const T *fb = F + (size_t)slot * 5 * CELLS_P;
        {
            // interior: every load of the four planes before the first store (U is read
            // and written through the same pointer, so the compiler keeps program order)
            T *u0b = U0 + (size_t)slot * 5 * CELLS_I;
            int c[PLANES], o[PLANES];
            T us[PLANES][5], u0[PLANES][5], fl[PLANES][5];
#pragma unroll
            for (int k = 0; k < PLANES; ++k) {
                c[k] = (part * PLANES + k) * FACE + tid;
                o[k] = ((c[k] / FACE + HW) * NP + (c[k] / NI) % NI + HW) * NP + c[k] % NI + HW;
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    us[k][q] = ub[o[k] + q * CELLS_P];
                    fl[k][q] = fb[o[k] + q * CELLS_P];
                    u0[k][q] = stage == 0 ? us[k][q] : u0b[q * CELLS_I + c[k]];
                }
            }
            bool ok = true;
#pragma unroll
            for (int k = 0; k < PLANES; ++k) {
                T un[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    if (stage == 0) u0b[q * CELLS_I + c[k]] = us[k][q];
                    un[q] = u0[k][q] + a * ((us[k][q] - u0[k][q]) + (T)dtl * fl[k][q]);
                    ub[o[k] + q * CELLS_P] = un[q];
                }
                ok = ok && lts_physical(un, P);
            }
            if (!ok) atomicOr(err, 1);
        }
        for (int f = part * PIECES; f < (part + 1) * PIECES; ++f) {
            if (f < 18) {
                const int side = f / 3, h = f % 3;
                if (nbr[(size_t)slot * 27 + face_region(side)] != -1) continue;   // not a jump face
                const int d = side >> 1, hi = side & 1;
                const int p = hi ? HW + NI + h : HW - 3 + h;
                T *h0 = H0 + ((size_t)slot * 6 + side) * 5 * SLAB + h * FACE + tid;
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const int n = plane_cell(q, d, p, tid >> 4, tid & 15);
                    const T us = ub[n];
                    T u0;
                    if (stage == 0) {
                        u0 = us;
                        h0[q * SLAB] = us;
                    } else {
                        u0 = h0[q * SLAB];
                    }
                    ub[n] = u0 + a * ((us - u0) + (T)dtl * fb[n]);
                }
            } else {
                // only faces that a coarse cell adjustment reads: jump faces (the fine side)
                // and faces whose same-level neighbour is refined (the coarse side)
                const int side = f - 18;
                const int nbs = nbr[(size_t)slot * 27 + face_region(side)];
                if (!(nbs == -1 || (nbs >= 0 && !meta[nbs].leaf))) continue;
                const double bw = stage == 2 ? 2.0 / 3.0 : 1.0 / 6.0;
                const T w = (T)(bw * dtl);
                const size_t base = ((size_t)slot * 6 + side) * 5 * FACE + tid;
#pragma unroll
                for (int q = 0; q < 5; ++q) ACC[base + q * FACE] += w * FF[base + q * FACE];
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_lts_adjust(T *U, const T *__restrict__ ACC, WorkList wl,
                                                    const BlockMeta *__restrict__ meta,
                                                    const int32_t *__restrict__ nbr,
                                                    const InstDev *__restrict__ inst) {
    const int nb_ = wl.count();
    const int rm = threadIdx.x;
    for (int b = blockIdx.x; b < nb_; b += gridDim.x) {
        const int slot = wl.at(b);
        const BlockMeta mt = meta[slot];
        const T dx = (T)ldexp(inst[mt.inst].dx0, -mt.level);
        T *ub = U + (size_t)slot * 5 * CELLS_P;
        for (int side = 0; side < 6; ++side) {
            const int nb = nbr[(size_t)slot * 27 + face_region(side)];
            if (nb < 0 || meta[nb].leaf) continue;   // uniform per workgroup
            const int d = side >> 1, hi = side & 1;
            const T *own = ACC + ((size_t)slot * 6 + side) * 5 * FACE;
            const T *fine = ACC + ((size_t)nb * 6 + (side ^ 1)) * 5 * FACE;
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const int n = plane_cell(q, d, hi ? HW + NI - 1 : HW, rm >> 4, rm & 15);
                const T o = own[q * FACE + rm], fn = fine[q * FACE + rm];
                ub[n] += hi ? (o - fn) / dx : (fn - o) / dx;
            }
        }
    }
}

// Level of the leaf on the other side of a face of `slot`: its own level unless the face
// is a resolution jump, then the level of the first ancestor whose face neighbour exists
// (that neighbour is the coarser leaf covering the position).
__device__ __forceinline__ int across_level(int slot, int side, const BlockMeta *meta,
                                            const int32_t *nbr) {
    const int fr = face_region(side);
    if (nbr[(size_t)slot * 27 + fr] != -1) return meta[slot].level;   // same level, or outside
    for (int a = meta[slot].parent; a >= 0; a = meta[a].parent)
        if (nbr[(size_t)a * 27 + fr] >= 0) return meta[a].level;
    return 0;
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_lts_zero(T *ACC, WorkList wl, const BlockMeta *__restrict__ meta,
                                                  const int32_t *__restrict__ nbr, int lo_end) {
    const int nb_ = wl.count();
    for (int b = blockIdx.x; b < nb_; b += gridDim.x) {
        const int slot = wl.at(b);
        const int side = blockIdx.y;
        if (across_level(slot, side, meta, nbr) < lo_end) continue;
        T *pl = ACC + ((size_t)slot * 6 + side) * 5 * FACE;
#pragma unroll
        for (int q = 0; q < 5; ++q) pl[q * FACE + threadIdx.x] = (T)0;
    }
}

}  // namespace

template <typename T>
hipError_t launch_lts_combine(const T *D, T *F, const WorkList &wl, const DevTables &tb,
                              const InstDev *inst, const T *U, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lts_combine<T>, dim3(wl.grid, NI), dim3(TPB), 0, st, D, F, wl, tb.meta,
                       inst, U);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lts_update(int stage, const double *dt, T *U, T *U0, T *H0, const T *F,
                             const T *FF, T *ACC, const WorkList &wl, const DevTables &tb,
                             const InstDev *inst, int32_t *err, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lts_update<T>, dim3(wl.grid, PARTS), dim3(TPB), 0, st, stage, dt, U,
                       U0, H0, F, FF, ACC, wl, tb.meta, tb.nbr, inst, err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lts_adjust(T *U, const T *ACC, const WorkList &wl, const DevTables &tb,
                             const InstDev *inst, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lts_adjust<T>, dim3(wl.grid), dim3(TPB), 0, st, U, ACC, wl, tb.meta, tb.nbr,
                       inst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lts_zero(T *ACC, const WorkList &wl, const DevTables &tb, int lo_end,
                           hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lts_zero<T>, dim3(wl.grid, 6), dim3(TPB), 0, st, ACC, wl, tb.meta, tb.nbr,
                       lo_end);
    return hipGetLastError();
}

int lts_halo_slab() { return SLAB; }

#define MRFV_LTS_INST(T)                                                                          \
    template hipError_t launch_lts_combine<T>(const T *, T *, const WorkList &, const DevTables &, \
                                              const InstDev *, const T *, hipStream_t);             \
    template hipError_t launch_lts_update<T>(int, const double *, T *, T *, T *, const T *,      \
                                             const T *, T *, const WorkList &, const DevTables &, \
                                             const InstDev *, int32_t *, hipStream_t);            \
    template hipError_t launch_lts_adjust<T>(T *, const T *, const WorkList &, const DevTables &, \
                                             const InstDev *, hipStream_t);                       \
    template hipError_t launch_lts_zero<T>(T *, const WorkList &, const DevTables &, int,        \
                                           hipStream_t);
MRFV_LTS_INST(float)
MRFV_LTS_INST(double)

}  // namespace mrfv
