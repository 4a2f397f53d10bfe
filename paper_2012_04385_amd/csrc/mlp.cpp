// mlp.cpp -- the learned refinement proposer's network object and its C ABI.
//
// 192-64-64-3 ReLU network, master parameters and Adam moments in FP32, bfloat16 copies
// of weights and activations for the matrix-core products, FP32 accumulation.  The
// forward pass, the class-weighted cross-entropy gradient and the Adam step all run on the
// device; the host only chooses sizes and reads back the loss.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mrfv_internal.h"

using namespace mrfv;

namespace mrfv {
hipError_t launch_gemm_bf16(const uint16_t *A, int sam, int sak, const uint16_t *B, int sbk, int sbn,
                            float *C, int ldc, int M, int Nn, int K, int accumulate, hipStream_t st);
hipError_t launch_to_bf16(const float *in, int ldi, int rows, int cols, uint16_t *out, int rows_pad,
                          int cols_pad, hipStream_t st);
hipError_t launch_bias_act(float *Z, const float *bias, uint16_t *H, int rows_pad, int cols, int relu,
                           hipStream_t st);
hipError_t launch_softmax_grad(const float *Z, const int32_t *y, const float *cw, float inv_wsum,
                               int rows, int rows_pad, float *dL, uint16_t *dLb, float *loss,
                               hipStream_t st);
hipError_t launch_relu_back(const float *dH, const float *Z, float *dZ, uint16_t *dZb, size_t n,
                            hipStream_t st);
hipError_t launch_colsum(const float *M, int ld, int rows, int cols, float *out, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t st);
}  // namespace mrfv

namespace {
constexpr int NIN = 192, NH = 64, NOUT = 3, NOP = 16;
constexpr int OW1 = 0, OB1 = OW1 + NIN * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NOUT, NPAR = OB3 + NOUT;
}  // namespace

struct mrfv_mlp {
    hipStream_t st = nullptr;
    int max_rows = 0, rows_pad_max = 0, t = 0;
    std::string err;
    float *par = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr, *b3pad = nullptr, *cw = nullptr;
    uint16_t *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;
    uint16_t *Xb = nullptr, *H1b = nullptr, *H2b = nullptr, *dLb = nullptr, *dZ2b = nullptr, *dZ1b = nullptr;
    float *Z1 = nullptr, *Z2 = nullptr, *Z3 = nullptr, *dL = nullptr, *dH2 = nullptr, *dZ2 = nullptr,
          *dH1 = nullptr, *dZ1 = nullptr, *dW3 = nullptr, *loss = nullptr, *loss1 = nullptr;
    int32_t *y = nullptr;
    std::vector<void *> allocs;
};

namespace {

int mfail(mrfv_mlp *m, int code, const std::string &msg) {
    if (m) m->err = msg;
    return code;
}

#define MHIP(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return mfail(mm, MRFV_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

int pad16(int n) { return (n + 15) & ~15; }

// Weights -> bfloat16 copies, b3 -> zero-padded bias, X -> bfloat16, forward to Z3.
int forward_core(mrfv_mlp *mm, const float *X, int N) {
    const int Np = pad16(N);
    hipStream_t st = mm->st;
    MHIP(launch_to_bf16(mm->par + OW1, NH, NIN, NH, mm->W1b, NIN, NH, st));
    MHIP(launch_to_bf16(mm->par + OW2, NH, NH, NH, mm->W2b, NH, NH, st));
    MHIP(launch_to_bf16(mm->par + OW3, NOUT, NH, NOUT, mm->W3b, NH, NOP, st));
    MHIP(hipMemsetAsync(mm->b3pad, 0, NOP * sizeof(float), st));
    MHIP(hipMemcpyAsync(mm->b3pad, mm->par + OB3, NOUT * sizeof(float), hipMemcpyDeviceToDevice, st));
    MHIP(launch_to_bf16(X, NIN, N, NIN, mm->Xb, Np, NIN, st));
    MHIP(launch_gemm_bf16(mm->Xb, NIN, 1, mm->W1b, NH, 1, mm->Z1, NH, Np, NH, NIN, 0, st));
    MHIP(launch_bias_act(mm->Z1, mm->par + OB1, mm->H1b, Np, NH, 1, st));
    MHIP(launch_gemm_bf16(mm->H1b, NH, 1, mm->W2b, NH, 1, mm->Z2, NH, Np, NH, NH, 0, st));
    MHIP(launch_bias_act(mm->Z2, mm->par + OB2, mm->H2b, Np, NH, 1, st));
    MHIP(launch_gemm_bf16(mm->H2b, NH, 1, mm->W3b, NOP, 1, mm->Z3, NOP, Np, NOP, NH, 0, st));
    MHIP(launch_bias_act(mm->Z3, mm->b3pad, nullptr, Np, NOP, 0, st));
    return MRFV_OK;
}

}  // namespace

extern "C" {

int mrfv_mlp_create(mrfv_mlp **out, int32_t max_rows, void *hip_stream) {
    if (!out || max_rows < 1 || max_rows > (1 << 24)) return MRFV_EINVAL;
    mrfv_mlp *mm = new mrfv_mlp();
    mm->st = (hipStream_t)hip_stream;
    mm->max_rows = max_rows;
    mm->rows_pad_max = pad16(max_rows);
    const size_t R = mm->rows_pad_max;
    auto al = [&](void **p, size_t bytes) {
        if (hipMalloc(p, bytes) != hipSuccess) return false;
        mm->allocs.push_back(*p);
        return true;
    };
    bool ok = al((void **)&mm->par, NPAR * 4) && al((void **)&mm->grad, NPAR * 4) &&
              al((void **)&mm->m, NPAR * 4) && al((void **)&mm->v, NPAR * 4) &&
              al((void **)&mm->b3pad, NOP * 4) && al((void **)&mm->cw, 4 * 4) &&
              al((void **)&mm->W1b, NIN * NH * 2) && al((void **)&mm->W2b, NH * NH * 2) &&
              al((void **)&mm->W3b, NH * NOP * 2) && al((void **)&mm->Xb, R * NIN * 2) &&
              al((void **)&mm->H1b, R * NH * 2) && al((void **)&mm->H2b, R * NH * 2) &&
              al((void **)&mm->dLb, R * NOP * 2) && al((void **)&mm->dZ2b, R * NH * 2) &&
              al((void **)&mm->dZ1b, R * NH * 2) && al((void **)&mm->Z1, R * NH * 4) &&
              al((void **)&mm->Z2, R * NH * 4) && al((void **)&mm->Z3, R * NOP * 4) &&
              al((void **)&mm->dL, R * NOP * 4) && al((void **)&mm->dH2, R * NH * 4) &&
              al((void **)&mm->dZ2, R * NH * 4) && al((void **)&mm->dH1, R * NH * 4) &&
              al((void **)&mm->dZ1, R * NH * 4) && al((void **)&mm->dW3, NH * NOP * 4) &&
              al((void **)&mm->loss, R * 4) && al((void **)&mm->loss1, 4) &&
              al((void **)&mm->y, R * 4);
    if (!ok) {
        mrfv_mlp_destroy(mm);
        return MRFV_ENOMEM;
    }
    if (hipMemset(mm->m, 0, NPAR * 4) != hipSuccess || hipMemset(mm->v, 0, NPAR * 4) != hipSuccess ||
        hipMemset(mm->par, 0, NPAR * 4) != hipSuccess) {
        mrfv_mlp_destroy(mm);
        return MRFV_EHIP;
    }
    *out = mm;
    return MRFV_OK;
}

int mrfv_mlp_destroy(mrfv_mlp *mm) {
    if (!mm) return MRFV_EINVAL;
    if (mm->st) hipStreamSynchronize(mm->st);
    else hipDeviceSynchronize();
    for (void *p : mm->allocs) hipFree(p);
    delete mm;
    return MRFV_OK;
}

const char *mrfv_mlp_last_error(const mrfv_mlp *mm) { return mm ? mm->err.c_str() : "null"; }

int32_t mrfv_mlp_nparams(void) { return NPAR; }

int mrfv_mlp_set_params(mrfv_mlp *mm, const float *params_host) {
    if (!mm || !params_host) return MRFV_EINVAL;
    MHIP(hipMemcpyAsync(mm->par, params_host, NPAR * 4, hipMemcpyHostToDevice, mm->st));
    MHIP(hipMemsetAsync(mm->m, 0, NPAR * 4, mm->st));
    MHIP(hipMemsetAsync(mm->v, 0, NPAR * 4, mm->st));
    MHIP(hipStreamSynchronize(mm->st));
    mm->t = 0;
    return MRFV_OK;
}

int mrfv_mlp_get_params(mrfv_mlp *mm, float *params_host) {
    if (!mm || !params_host) return MRFV_EINVAL;
    MHIP(hipMemcpyAsync(params_host, mm->par, NPAR * 4, hipMemcpyDeviceToHost, mm->st));
    MHIP(hipStreamSynchronize(mm->st));
    return MRFV_OK;
}

int mrfv_mlp_forward(mrfv_mlp *mm, const float *X_dev, int32_t N, float *logits_dev) {
    if (!mm || !X_dev || !logits_dev) return MRFV_EINVAL;
    if (N < 1 || N > mm->max_rows) return mfail(mm, MRFV_EINVAL, "mlp_forward: bad row count");
    int rc = forward_core(mm, X_dev, N);
    if (rc != MRFV_OK) return rc;
    MHIP(hipMemcpy2DAsync(logits_dev, NOUT * sizeof(float), mm->Z3, NOP * sizeof(float),
                          NOUT * sizeof(float), N, hipMemcpyDeviceToDevice, mm->st));
    return MRFV_OK;
}

int mrfv_mlp_loss_grad(mrfv_mlp *mm, const float *X_dev, const int32_t *labels_host,
                       const float *class_w_host, int32_t N, float *loss_host, float *grad_host) {
    if (!mm || !X_dev || !labels_host || !class_w_host) return MRFV_EINVAL;
    if (N < 1 || N > mm->max_rows) return mfail(mm, MRFV_EINVAL, "mlp_loss_grad: bad row count");
    double wsum = 0.0;
    for (int i = 0; i < N; ++i) {
        if (labels_host[i] < 0 || labels_host[i] > 2) return mfail(mm, MRFV_EINVAL, "label out of range");
        wsum += class_w_host[labels_host[i]];
    }
    if (!(wsum > 0.0)) return mfail(mm, MRFV_EINVAL, "class weights sum to zero");
    hipStream_t st = mm->st;
    const int Np = pad16(N);
    MHIP(hipMemcpyAsync(mm->y, labels_host, N * 4, hipMemcpyHostToDevice, st));
    MHIP(hipMemcpyAsync(mm->cw, class_w_host, 3 * 4, hipMemcpyHostToDevice, st));
    int rc = forward_core(mm, X_dev, N);
    if (rc != MRFV_OK) return rc;
    MHIP(launch_softmax_grad(mm->Z3, mm->y, mm->cw, (float)(1.0 / wsum), N, Np, mm->dL, mm->dLb,
                             mm->loss, st));
    MHIP(launch_colsum(mm->loss, 1, N, 1, mm->loss1, st));
    // output layer
    MHIP(launch_gemm_bf16(mm->H2b, 1, NH, mm->dLb, NOP, 1, mm->dW3, NOP, NH, NOP, Np, 0, st));
    MHIP(hipMemcpy2DAsync(mm->grad + OW3, NOUT * 4, mm->dW3, NOP * 4, NOUT * 4, NH,
                          hipMemcpyDeviceToDevice, st));
    MHIP(launch_colsum(mm->dL, NOP, N, NOUT, mm->grad + OB3, st));
    // second hidden layer
    MHIP(launch_gemm_bf16(mm->dLb, NOP, 1, mm->W3b, 1, NOP, mm->dH2, NH, Np, NH, NOP, 0, st));
    MHIP(launch_relu_back(mm->dH2, mm->Z2, mm->dZ2, mm->dZ2b, (size_t)Np * NH, st));
    MHIP(launch_gemm_bf16(mm->H1b, 1, NH, mm->dZ2b, NH, 1, mm->grad + OW2, NH, NH, NH, Np, 0, st));
    MHIP(launch_colsum(mm->dZ2, NH, N, NH, mm->grad + OB2, st));
    // first hidden layer
    MHIP(launch_gemm_bf16(mm->dZ2b, NH, 1, mm->W2b, 1, NH, mm->dH1, NH, Np, NH, NH, 0, st));
    MHIP(launch_relu_back(mm->dH1, mm->Z1, mm->dZ1, mm->dZ1b, (size_t)Np * NH, st));
    MHIP(launch_gemm_bf16(mm->Xb, 1, NIN, mm->dZ1b, NH, 1, mm->grad + OW1, NH, NIN, NH, Np, 0, st));
    MHIP(launch_colsum(mm->dZ1, NH, N, NH, mm->grad + OB1, st));
    if (loss_host) MHIP(hipMemcpyAsync(loss_host, mm->loss1, 4, hipMemcpyDeviceToHost, st));
    if (grad_host) MHIP(hipMemcpyAsync(grad_host, mm->grad, NPAR * 4, hipMemcpyDeviceToHost, st));
    MHIP(hipStreamSynchronize(st));
    return MRFV_OK;
}

int mrfv_mlp_adam_step(mrfv_mlp *mm, float lr, float beta1, float beta2, float eps) {
    if (!mm || !(lr > 0.f)) return MRFV_EINVAL;
    mm->t += 1;
    const float bc1 = 1.f - std::pow(beta1, (float)mm->t), bc2 = 1.f - std::pow(beta2, (float)mm->t);
    MHIP(launch_adam(mm->par, mm->grad, mm->m, mm->v, NPAR, lr, beta1, beta2, eps, bc1, bc2, mm->st));
    return MRFV_OK;
}

}  // extern "C"

// Forward pass on a given stream (used by the step when the proposer is active).
int mrfv::mlp_forward_on(mrfv_mlp *mm, hipStream_t st, const float *X, int N, float *logits) {
    if (!mm || N < 1 || N > mm->max_rows) return MRFV_EINVAL;
    hipStream_t keep = mm->st;
    mm->st = st;
    int rc = mrfv_mlp_forward(mm, X, N, logits);
    mm->st = keep;
    return rc;
}
