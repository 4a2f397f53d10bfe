// orc_mlp.cpp -- oracle of the learned refinement proposer (test infrastructure only).
//
// The proposer is not part of the paper: it predicts next-step refine/keep/coarsen flags
// so that tree bookkeeping can start early; the exact Harten threshold stays the judge.
// This file is the plain FP64 reference of its features, forward pass, loss and
// gradients.  With bf16 = 1 it rounds, with round-to-nearest-even, exactly the tensors
// the GPU stores in bfloat16 (inputs, weights, hidden activations, and the gradients fed
// to the backward matrix products); with bf16 = 0 it is the FP64 function itself, whose
// gradients are pinned by finite differences.
//
// Network: 192 -> 64 -> 64 -> 3, ReLU, weights stored [in][out] row-major; parameter
// vector layout W1, b1, W2, b2, W3, b3.  Loss: class-weighted mean softmax cross-entropy.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "orc.h"

namespace {

constexpr int NIN = 192, NH = 64, NOUT = 3;
constexpr int OW1 = 0, OB1 = OW1 + NIN * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH,
              OW3 = OB2 + NH, OB3 = OW3 + NH * NOUT, NPAR = OB3 + NOUT;

// Round to the nearest bfloat16 (8 significant bits), ties to even.
double bf16(double x) {
    if (!std::isfinite(x) || x == 0.0) return x;
    int e;
    const double m = std::frexp(x, &e);       // x = m 2^e, 0.5 <= |m| < 1
    const double s = std::ldexp(m, 8);        // 8 significant bits
    double r = std::nearbyint(s);             // default rounding mode: to nearest even
    return std::ldexp(r, e - 8);
}

struct Fwd {
    std::vector<double> x, z1, h1, z2, h2, lg;
};

void forward(const double *P, const double *X, int N, int rb, Fwd &f) {
    auto R = [&](double v) { return rb ? bf16(v) : v; };
    f.x.resize((size_t)N * NIN);
    f.z1.assign((size_t)N * NH, 0.0);
    f.h1.resize((size_t)N * NH);
    f.z2.assign((size_t)N * NH, 0.0);
    f.h2.resize((size_t)N * NH);
    f.lg.assign((size_t)N * NOUT, 0.0);
    for (size_t i = 0; i < (size_t)N * NIN; ++i) f.x[i] = R(X[i]);
    for (int n = 0; n < N; ++n) {
        for (int o = 0; o < NH; ++o) {
            double s = 0.0;
            for (int i = 0; i < NIN; ++i) s += f.x[(size_t)n * NIN + i] * R(P[OW1 + i * NH + o]);
            f.z1[(size_t)n * NH + o] = s + P[OB1 + o];
            f.h1[(size_t)n * NH + o] = R(std::fmax(f.z1[(size_t)n * NH + o], 0.0));
        }
        for (int o = 0; o < NH; ++o) {
            double s = 0.0;
            for (int i = 0; i < NH; ++i) s += f.h1[(size_t)n * NH + i] * R(P[OW2 + i * NH + o]);
            f.z2[(size_t)n * NH + o] = s + P[OB2 + o];
            f.h2[(size_t)n * NH + o] = R(std::fmax(f.z2[(size_t)n * NH + o], 0.0));
        }
        for (int o = 0; o < NOUT; ++o) {
            double s = 0.0;
            for (int i = 0; i < NH; ++i) s += f.h2[(size_t)n * NH + i] * R(P[OW3 + i * NOUT + o]);
            f.lg[(size_t)n * NOUT + o] = s + P[OB3 + o];
        }
    }
}

}  // namespace

extern "C" {

int orc_mlp_nparams(void) { return NPAR; }

double orc_bf16_round(double x) { return bf16(x); }

void orc_mlp_forward(const double *params, const double *X, int N, int bf16_emulation,
                     double *logits) {
    Fwd f;
    forward(params, X, N, bf16_emulation, f);
    std::memcpy(logits, f.lg.data(), sizeof(double) * (size_t)N * NOUT);
}

double orc_mlp_loss_grad(const double *P, const double *X, const int32_t *labels,
                         const double *class_w, int N, int rb, double *grad) {
    auto R = [&](double v) { return rb ? bf16(v) : v; };
    Fwd f;
    forward(P, X, N, rb, f);
    double wsum = 0.0;
    for (int n = 0; n < N; ++n) wsum += class_w[labels[n]];
    double loss = 0.0;
    std::vector<double> dl((size_t)N * NOUT);
    for (int n = 0; n < N; ++n) {
        const double *z = &f.lg[(size_t)n * NOUT];
        double mx = z[0];
        for (int o = 1; o < NOUT; ++o) mx = std::fmax(mx, z[o]);
        double se = 0.0;
        for (int o = 0; o < NOUT; ++o) se += std::exp(z[o] - mx);
        const double w = class_w[labels[n]] / wsum;
        loss += w * (std::log(se) + mx - z[labels[n]]);
        for (int o = 0; o < NOUT; ++o) {
            const double p = std::exp(z[o] - mx) / se;
            dl[(size_t)n * NOUT + o] = w * (p - (o == labels[n] ? 1.0 : 0.0));
        }
    }
    if (!grad) return loss;
    std::memset(grad, 0, sizeof(double) * NPAR);
    std::vector<double> dz2((size_t)N * NH), dz1((size_t)N * NH);
    for (int n = 0; n < N; ++n) {
        // output layer
        for (int o = 0; o < NOUT; ++o) {
            const double g = dl[(size_t)n * NOUT + o];
            grad[OB3 + o] += g;
            for (int i = 0; i < NH; ++i) grad[OW3 + i * NOUT + o] += f.h2[(size_t)n * NH + i] * R(g);
        }
        // second hidden layer
        for (int i = 0; i < NH; ++i) {
            double s = 0.0;
            for (int o = 0; o < NOUT; ++o) s += R(dl[(size_t)n * NOUT + o]) * R(P[OW3 + i * NOUT + o]);
            dz2[(size_t)n * NH + i] = f.z2[(size_t)n * NH + i] > 0.0 ? s : 0.0;
        }
        for (int o = 0; o < NH; ++o) {
            const double g = dz2[(size_t)n * NH + o];
            grad[OB2 + o] += g;
            for (int i = 0; i < NH; ++i) grad[OW2 + i * NH + o] += f.h1[(size_t)n * NH + i] * R(g);
        }
        // first hidden layer
        for (int i = 0; i < NH; ++i) {
            double s = 0.0;
            for (int o = 0; o < NH; ++o) s += R(dz2[(size_t)n * NH + o]) * R(P[OW2 + i * NH + o]);
            dz1[(size_t)n * NH + i] = f.z1[(size_t)n * NH + i] > 0.0 ? s : 0.0;
        }
        for (int o = 0; o < NH; ++o) {
            const double g = dz1[(size_t)n * NH + o];
            grad[OB1 + o] += g;
            for (int i = 0; i < NIN; ++i) grad[OW1 + i * NH + o] += f.x[(size_t)n * NIN + i] * R(g);
        }
    }
    return loss;
}

// Features of one leaf block: over each of the 4^3 sub-cubes of 4^3 interior cells, the
// means of rho, |grad rho| (central differences inside the block, one-sided at its
// faces, in units of one cell) and p; transformed to (mean rho / s_rho - 1,
// log(1 + mean |grad rho| / (s_rho eps_l)), mean p / s_p - 1); out[3 s + c] with the
// sub-cube index s = (sz*4 + sy)*4 + sx.
void orc_features(const double *u, double gamma, double B, double s_rho, double s_p,
                  double eps_l, double *out) {
    const int P = ORC_P, H = ORC_H, N = ORC_IC;
    auto rho = [&](int k, int j, int i) { return u[((0 * P + H + k) * P + H + j) * P + H + i]; };
    auto comp = [&](int q, int k, int j, int i) { return u[((q * P + H + k) * P + H + j) * P + H + i]; };
    auto d1 = [&](int a, int k, int j, int i) {
        int c[3] = {i, j, k};
        int lo[3] = {i, j, k}, hi[3] = {i, j, k};
        double den = 2.0;
        if (c[a] == 0) { hi[a] = 1; den = 1.0; }
        else if (c[a] == N - 1) { lo[a] = N - 2; den = 1.0; }
        else { lo[a] = c[a] - 1; hi[a] = c[a] + 1; }
        return (rho(hi[2], hi[1], hi[0]) - rho(lo[2], lo[1], lo[0])) / den;
    };
    for (int sz = 0; sz < 4; ++sz)
        for (int sy = 0; sy < 4; ++sy)
            for (int sx = 0; sx < 4; ++sx) {
                double sr = 0.0, sg = 0.0, sp = 0.0;
                for (int k = 4 * sz; k < 4 * sz + 4; ++k)
                    for (int j = 4 * sy; j < 4 * sy + 4; ++j)
                        for (int i = 4 * sx; i < 4 * sx + 4; ++i) {
                            const double r = rho(k, j, i);
                            const double gx = d1(0, k, j, i), gy = d1(1, k, j, i), gz = d1(2, k, j, i);
                            const double m1 = comp(1, k, j, i), m2 = comp(2, k, j, i), m3 = comp(3, k, j, i);
                            const double p = (gamma - 1.0) * (comp(4, k, j, i) - 0.5 * (m1 * m1 + m2 * m2 + m3 * m3) / r) - gamma * B;
                            sr += r;
                            sg += std::sqrt(gx * gx + gy * gy + gz * gz);
                            sp += p;
                        }
                const int s = (sz * 4 + sy) * 4 + sx;
                out[3 * s + 0] = sr / 64.0 / s_rho - 1.0;
                out[3 * s + 1] = std::log(1.0 + sg / 64.0 / (s_rho * eps_l));
                out[3 * s + 2] = sp / 64.0 / s_p - 1.0;
            }
}

}  // extern "C"
