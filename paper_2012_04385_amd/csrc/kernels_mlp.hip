// kernels_mlp.hip -- gfx950 kernels of the learned refinement proposer.
//
// The proposer (not part of the paper) is a 192-64-64-3 ReLU network with bfloat16
// weights and activations and FP32 accumulation; its matrix products run on the matrix
// cores (v_mfma_f32_16x16x16_bf16, one wavefront per 16x16 output tile).  Features are
// 4^3 sub-cube means of rho, |grad rho| and p of each leaf block.  The exact Harten
// threshold remains the judge: proposals only let the host prepare tree updates early.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mrfv_internal.h"

namespace mrfv {

namespace {

constexpr int TPB = 256;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Features of every listed leaf, one workgroup per block: 4 threads per sub-cube, each
// summing one 4x4 layer of it; rows of X follow the list order.
template <typename T>
__global__ __launch_bounds__(TPB) void k_features(const T *__restrict__ U, WorkList wl,
                                                  const BlockMeta *__restrict__ meta,
                                                  const InstDev *__restrict__ inst,
                                                  float *__restrict__ X) {
    const int nb = wl.count();
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int slot = wl.at(b);
        const BlockMeta m = meta[slot];
        const InstDev P = inst[m.inst];
        const T *u = U + (size_t)slot * 5 * CELLS_P;
        const int s = threadIdx.x >> 2, part = threadIdx.x & 3;
        const int sx = s & 3, sy = (s >> 2) & 3, sz = s >> 4;
        const int k = 4 * sz + part;
        const float g = (float)P.gamma, Bp = (float)P.B;
        auto rho = [&](int kk, int jj, int ii) {
            return (float)u[((HW + kk) * NP + HW + jj) * NP + HW + ii];
        };
        float sr = 0.f, sg = 0.f, sp = 0.f;
        for (int j = 4 * sy; j < 4 * sy + 4; ++j)
            for (int i = 4 * sx; i < 4 * sx + 4; ++i) {
                const int o = ((HW + k) * NP + HW + j) * NP + HW + i;
                const float r = (float)u[o];
                const float m1 = (float)u[o + CELLS_P], m2 = (float)u[o + 2 * CELLS_P],
                            m3 = (float)u[o + 3 * CELLS_P], E = (float)u[o + 4 * CELLS_P];
                const float p = (g - 1.f) * (E - 0.5f * (m1 * m1 + m2 * m2 + m3 * m3) / r) - g * Bp;
                // central differences inside the block, one-sided at its faces
                const float gx = i == 0 ? rho(k, j, 1) - rho(k, j, 0)
                               : (i == NI - 1 ? rho(k, j, NI - 1) - rho(k, j, NI - 2)
                                              : 0.5f * (rho(k, j, i + 1) - rho(k, j, i - 1)));
                const float gy = j == 0 ? rho(k, 1, i) - rho(k, 0, i)
                               : (j == NI - 1 ? rho(k, NI - 1, i) - rho(k, NI - 2, i)
                                              : 0.5f * (rho(k, j + 1, i) - rho(k, j - 1, i)));
                const float gz = k == 0 ? rho(1, j, i) - rho(0, j, i)
                               : (k == NI - 1 ? rho(NI - 1, j, i) - rho(NI - 2, j, i)
                                              : 0.5f * (rho(k + 1, j, i) - rho(k - 1, j, i)));
                sr += r;
                sg += sqrtf(gx * gx + gy * gy + gz * gz);
                sp += p;
            }
        // the four parts of a sub-cube are consecutive lanes
        sr += __shfl_xor(sr, 1);
        sg += __shfl_xor(sg, 1);
        sp += __shfl_xor(sp, 1);
        sr += __shfl_xor(sr, 2);
        sg += __shfl_xor(sg, 2);
        sp += __shfl_xor(sp, 2);
        if (part == 0) {
            const float eps_l = (float)ldexp(P.eps, -3 * (P.lmax - m.level));
            const float s_rho = (float)P.scale_rho, s_p = (float)(P.scale_E * (P.gamma - 1.0));
            float *x = X + (size_t)b * 192 + 3 * s;
            x[0] = sr * (1.f / 64.f) / s_rho - 1.f;
            x[1] = logf(1.f + sg * (1.f / 64.f) / (s_rho * eps_l));
            x[2] = sp * (1.f / 64.f) / s_p - 1.f;
        }
        __syncthreads();
    }
}

// C[M][Nn] (FP32, ldc) (+)= sum_k A(m,k) B(k,n) with bfloat16 operands addressed by
// strides, A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]; M, Nn, K multiples of
// 16.  One wavefront per 16x16 tile.  Operand layout of v_mfma_f32_16x16x16_bf16: lane
// l holds A[l%16][4(l/16) .. +3], B[4(l/16) .. +3][l%16] and C[4(l/16) .. +3][l%16].
__global__ __launch_bounds__(TPB) void k_gemm_bf16(const uint16_t *__restrict__ A, int sam, int sak,
                                                   const uint16_t *__restrict__ B, int sbk, int sbn,
                                                   float *__restrict__ C, int ldc, int M, int Nn,
                                                   int K, int accumulate) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tile = blockIdx.x * (TPB / 64) + wave;
    const int tiles_n = Nn / 16;
    if (tile >= (M / 16) * tiles_n) return;
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    const int i = lane & 15, kq = lane >> 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const uint16_t *Arow = A + (size_t)(tm * 16 + i) * sam;
    const uint16_t *Bcol = B + (size_t)(tn * 16 + i) * sbn;
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + 4 * kq + e;
            a[e] = (short)Arow[(size_t)k * sak];
            b[e] = (short)Bcol[(size_t)k * sbk];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        float *c = C + (size_t)(tm * 16 + 4 * kq + e) * ldc + tn * 16 + i;
        *c = accumulate ? *c + acc[e] : acc[e];
    }
}

// out[r][c] = bf16(in[r*ldi + c]) for r < rows, c < cols; zero padding up to
// (rows_pad, cols_pad).
__global__ __launch_bounds__(TPB) void k_to_bf16(const float *__restrict__ in, int ldi, int rows,
                                                 int cols, uint16_t *__restrict__ out,
                                                 int rows_pad, int cols_pad) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t >= (size_t)rows_pad * cols_pad) return;
    const int r = (int)(t / cols_pad), c = (int)(t % cols_pad);
    out[t] = (r < rows && c < cols) ? to_bf16(in[(size_t)r * ldi + c]) : (uint16_t)0;
}

// Z[r][c] += b[c]; H[r][c] = bf16(relu? max(Z, 0) : Z), for r < rows_pad, c < cols.
__global__ __launch_bounds__(TPB) void k_bias_act(float *__restrict__ Z, const float *__restrict__ bias,
                                                  uint16_t *__restrict__ H, int rows_pad, int cols,
                                                  int relu) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t >= (size_t)rows_pad * cols) return;
    const int c = (int)(t % cols);
    const float z = Z[t] + bias[c];
    Z[t] = z;
    if (H) H[t] = to_bf16(relu ? fmaxf(z, 0.f) : z);
}

// Per sample: softmax of logits[r][0..2] (ld 16), class-weighted cross-entropy and its
// gradient dL = w_y (p - onehot) / sum_w (FP32 and bfloat16, ld 16, zero padding).
__global__ __launch_bounds__(TPB) void k_softmax_grad(const float *__restrict__ Z, const int32_t *__restrict__ y,
                                                      const float *__restrict__ cw, float inv_wsum, int rows,
                                                      int rows_pad, float *__restrict__ dL,
                                                      uint16_t *__restrict__ dLb, float *__restrict__ loss) {
    const int r = blockIdx.x * TPB + threadIdx.x;
    if (r >= rows_pad) return;
    if (r >= rows) {
        for (int c = 0; c < 16; ++c) { dL[r * 16 + c] = 0.f; dLb[r * 16 + c] = 0; }
        loss[r] = 0.f;
        return;
    }
    const float *z = Z + (size_t)r * 16;
    const float mx = fmaxf(z[0], fmaxf(z[1], z[2]));
    const float e0 = expf(z[0] - mx), e1 = expf(z[1] - mx), e2 = expf(z[2] - mx);
    const float se = e0 + e1 + e2;
    const int t = y[r];
    const float w = cw[t] * inv_wsum;
    loss[r] = w * (logf(se) + mx - z[t]);
    const float p[3] = {e0 / se, e1 / se, e2 / se};
    for (int c = 0; c < 16; ++c) {
        const float g = c < 3 ? w * (p[c] - (c == t ? 1.f : 0.f)) : 0.f;
        dL[r * 16 + c] = g;
        dLb[r * 16 + c] = to_bf16(g);
    }
}

// dZ = dH * [Z > 0] (FP32 and bfloat16).
__global__ __launch_bounds__(TPB) void k_relu_back(const float *__restrict__ dH, const float *__restrict__ Z,
                                                   float *__restrict__ dZ, uint16_t *__restrict__ dZb,
                                                   size_t n) {
    const size_t t = (size_t)blockIdx.x * TPB + threadIdx.x;
    if (t >= n) return;
    const float v = Z[t] > 0.f ? dH[t] : 0.f;
    dZ[t] = v;
    dZb[t] = to_bf16(v);
}

// out[c] = sum over rows < rows of M[r][c] (ld), fixed reduction order; one workgroup per
// column.
__global__ __launch_bounds__(TPB) void k_colsum(const float *__restrict__ M, int ld, int rows,
                                                float *__restrict__ out) {
    __shared__ float red[TPB];
    const int c = blockIdx.x;
    float s = 0.f;
    for (int r = threadIdx.x; r < rows; r += TPB) s += M[(size_t)r * ld + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = TPB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

__global__ __launch_bounds__(TPB) void k_adam(float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int n,
                                              float lr, float b1, float b2, float eps, float bc1,
                                              float bc2) {
    const int t = blockIdx.x * TPB + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.f - b1) * gt;
    const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / bc1) / (sqrtf(vt / bc2) + eps);
}

inline unsigned nblk(size_t n) { return (unsigned)((n + TPB - 1) / TPB); }

}  // namespace

template <typename T>
hipError_t launch_features(const T *U, const WorkList &wl, const DevTables &tb, const InstDev *inst,
                           float *X, hipStream_t st) {
    if (wl.grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features<T>, dim3(wl.grid), dim3(TPB), 0, st, U, wl, tb.meta, inst, X);
    return hipGetLastError();
}
template hipError_t launch_features<float>(const float *, const WorkList &, const DevTables &,
                                           const InstDev *, float *, hipStream_t);
template hipError_t launch_features<double>(const double *, const WorkList &, const DevTables &,
                                            const InstDev *, float *, hipStream_t);

hipError_t launch_gemm_bf16(const uint16_t *A, int sam, int sak, const uint16_t *B, int sbk, int sbn,
                            float *C, int ldc, int M, int Nn, int K, int accumulate, hipStream_t st) {
    const int tiles = (M / 16) * (Nn / 16);
    if (tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm_bf16, dim3((tiles + 3) / 4), dim3(TPB), 0, st, A, sam, sak, B, sbk, sbn, C,
                       ldc, M, Nn, K, accumulate);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float *in, int ldi, int rows, int cols, uint16_t *out, int rows_pad,
                          int cols_pad, hipStream_t st) {
    const size_t n = (size_t)rows_pad * cols_pad;
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(TPB), 0, st, in, ldi, rows, cols, out, rows_pad,
                       cols_pad);
    return hipGetLastError();
}

hipError_t launch_bias_act(float *Z, const float *bias, uint16_t *H, int rows_pad, int cols, int relu,
                           hipStream_t st) {
    const size_t n = (size_t)rows_pad * cols;
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(n)), dim3(TPB), 0, st, Z, bias, H, rows_pad, cols, relu);
    return hipGetLastError();
}

hipError_t launch_softmax_grad(const float *Z, const int32_t *y, const float *cw, float inv_wsum,
                               int rows, int rows_pad, float *dL, uint16_t *dLb, float *loss,
                               hipStream_t st) {
    if (rows_pad <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_softmax_grad, dim3(nblk(rows_pad)), dim3(TPB), 0, st, Z, y, cw, inv_wsum, rows,
                       rows_pad, dL, dLb, loss);
    return hipGetLastError();
}

hipError_t launch_relu_back(const float *dH, const float *Z, float *dZ, uint16_t *dZb, size_t n,
                            hipStream_t st) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_relu_back, dim3(nblk(n)), dim3(TPB), 0, st, dH, Z, dZ, dZb, n);
    return hipGetLastError();
}

hipError_t launch_colsum(const float *M, int ld, int rows, int cols, float *out, hipStream_t st) {
    if (cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(TPB), 0, st, M, ld, rows, out);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(TPB), 0, st, p, g, m, v, n, lr, b1, b2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace mrfv
