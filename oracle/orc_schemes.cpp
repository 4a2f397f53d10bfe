// orc_schemes.cpp -- the paper's other flux kernels, for the oracle (test infrastructure
// only).  Sec. "Numerical Scheme" names three approximate Riemann solvers (Roe, Rusanov /
// local Lax-Friedrichs with the eigenvalues of the two cells sharing a face, HLLC) and
// three fifth-order reconstructions used inside them (WENO5-JS, TENO5, WENO-AO(5,3)); the
// weak-scaling section runs four combinations: Roe-WENO5 (the standard configuration),
// Roe-TENO5, LLF-WENO5 and HLLC-WENO-AO(5,3).  The constants of the published methods:
//   TENO5 (Fu, Hu & Adams 2016): C = 1, q = 6, eps = 1e-40, cut-off C_T = 1e-5;
//   WENO-AO(5,3) (Balsara, Garain & Shu 2016): gamma_Hi = gamma_Lo = 0.85, weights
//     gamma_k / (eps + beta_k)^2 with eps = 1e-6 (as the WENO5-JS weights here);
//   HLLC (Toro, Spruce & Speares 1994): wave speeds S_L = min(u_L - c_L, u~ - c~),
//     S_R = max(u_R + c_R, u~ + c~) with the Roe average of the two face states.
// Roe and LLF use the characteristic flux splitting of orc_euler.cpp; HLLC reconstructs the
// two face states characteristic-wise (Roe eigenvectors of the two face cells), falling
// back to the face cells' own states where a reconstructed state is not physical.
#include "orc.h"
#include <algorithm>
#include <cmath>

namespace {

double weno5_js(double a, double b, double c, double d, double e) {
    return orc_weno5_minus(a, b, c, d, e);
}

// Jiang-Shu smoothness indicators of the three 3-cell candidates (a,b,c), (b,c,d), (c,d,e).
void js_betas(double a, double b, double c, double d, double e, double beta[3]) {
    beta[0] = 13.0 / 12.0 * (a - 2.0 * b + c) * (a - 2.0 * b + c) + 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
    beta[1] = 13.0 / 12.0 * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
    beta[2] = 13.0 / 12.0 * (c - 2.0 * d + e) * (c - 2.0 * d + e) + 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
}

// Third-order candidate values at the right face of c.
void candidates(double a, double b, double c, double d, double e, double q[3]) {
    q[0] = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    q[1] = (-b + 5.0 * c + 2.0 * d) / 6.0;
    q[2] = (2.0 * c + 5.0 * d - e) / 6.0;
}

}  // namespace

extern "C" {

double orc_teno5_minus(double a, double b, double c, double d, double e) {
    double beta[3], q[3];
    js_betas(a, b, c, d, e, beta);
    candidates(a, b, c, d, e, q);
    const double dk[3] = {0.1, 0.6, 0.3};         // optimal weights of the 5th-order combination
    const double tau5 = std::fabs(beta[0] - beta[2]);
    double gam[3], sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double r = 1.0 + tau5 / (beta[k] + 1e-40);
        gam[k] = (r * r) * (r * r) * (r * r);      // (C + tau5 / (beta + eps))^q, C = 1, q = 6
        sum += gam[k];
    }
    double num = 0.0, den = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double chi = gam[k] / sum;
        const double delta = chi < 1e-5 ? 0.0 : 1.0;   // stencils below the cut-off are dropped
        num += dk[k] * delta * q[k];
        den += dk[k] * delta;
    }
    return num / den;
}

double orc_beta_quartic(double a, double b, double c, double d, double e) {
    // Smoothness of the quartic whose cell averages over cells -2..2 (unit width) are
    // a..e: the sum over derivative orders l = 1..4 of the integral of (d^l P / dx^l)^2 over
    // the centre cell.  The quartic's monomial coefficients are Minv u, where M maps them
    // to the five cell averages (inverted once by Gauss-Jordan); the integrals are exact.
    // Tables built once: Minv (monomial coefficients from the five averages) and G, with
    // G[m][n] = sum over l of m!/(m-l)! n!/(n-l)! times the integral of x^(m-l+n-l) over the
    // centre cell, so that beta = c^T G c for the coefficients c = Minv u.
    struct Tables {
        double Minv[5][5], G[5][5];
    };
    static const Tables T = [] {
        Tables t{};
        double M[5][10];
        for (int j = 0; j < 5; ++j) {
            const double lo = (j - 2) - 0.5, hi = (j - 2) + 0.5;
            for (int m = 0; m < 5; ++m) M[j][m] = (std::pow(hi, m + 1) - std::pow(lo, m + 1)) / (m + 1);
            for (int m = 0; m < 5; ++m) M[j][5 + m] = j == m ? 1.0 : 0.0;
        }
        for (int col = 0; col < 5; ++col) {          // Gauss-Jordan with partial pivoting
            int piv = col;
            for (int r = col + 1; r < 5; ++r)
                if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
            for (int k = 0; k < 10; ++k) std::swap(M[col][k], M[piv][k]);
            const double inv = 1.0 / M[col][col];
            for (int k = 0; k < 10; ++k) M[col][k] *= inv;
            for (int r = 0; r < 5; ++r) {
                if (r == col) continue;
                const double f = M[r][col];
                for (int k = 0; k < 10; ++k) M[r][k] -= f * M[col][k];
            }
        }
        for (int m = 0; m < 5; ++m)
            for (int j = 0; j < 5; ++j) t.Minv[m][j] = M[m][5 + j];
        auto falling = [](int m, int l) {        // m! / (m - l)!
            double r = 1.0;
            for (int i = 0; i < l; ++i) r *= (m - i);
            return r;
        };
        for (int l = 1; l <= 4; ++l)
            for (int m = l; m < 5; ++m)
                for (int n = l; n < 5; ++n) {
                    const int k = (m - l) + (n - l);
                    if (k & 1) continue;             // odd powers integrate to zero
                    t.G[m][n] += falling(m, l) * falling(n, l) * 2.0 * std::pow(0.5, k + 1) / (k + 1);
                }
        return t;
    }();
    const double u[5] = {a, b, c, d, e};
    double coef[5];
    for (int m = 0; m < 5; ++m) {
        double s = 0.0;
        for (int j = 0; j < 5; ++j) s += T.Minv[m][j] * u[j];
        coef[m] = s;
    }
    double beta = 0.0;
    for (int m = 1; m < 5; ++m)
        for (int n = 1; n < 5; ++n) beta += coef[m] * T.G[m][n] * coef[n];
    return beta;
}

double orc_wao53_minus(double a, double b, double c, double d, double e) {
    double beta[4], q[3];
    js_betas(a, b, c, d, e, beta);
    beta[3] = orc_beta_quartic(a, b, c, d, e);
    candidates(a, b, c, d, e, q);
    const double q5 = (2.0 * a - 13.0 * b + 47.0 * c + 27.0 * d - 3.0 * e) / 60.0;
    const double ghi = 0.85, glo = 0.85;
    const double g[4] = {(1.0 - ghi) * (1.0 - glo) / 2.0, (1.0 - ghi) * glo,
                         (1.0 - ghi) * (1.0 - glo) / 2.0, ghi};
    double w[4], sum = 0.0;
    for (int k = 0; k < 4; ++k) {
        w[k] = g[k] / ((1e-6 + beta[k]) * (1e-6 + beta[k]));
        sum += w[k];
    }
    for (int k = 0; k < 4; ++k) w[k] /= sum;
    return w[3] / g[3] * (q5 - g[0] * q[0] - g[1] * q[1] - g[2] * q[2]) + w[0] * q[0] + w[1] * q[1] +
           w[2] * q[2];
}

void orc_hllc_flux_x(const double UL[5], const double UR[5], double gamma, double B, double F[5]) {
    const double pl = orc_pressure(UL, gamma, B), pr = orc_pressure(UR, gamma, B);
    const double ul = UL[1] / UL[0], ur = UR[1] / UR[0];
    const double cl = std::sqrt(gamma * (pl + B) / UL[0]), cr = std::sqrt(gamma * (pr + B) / UR[0]);
    // Roe average of the two states (velocity and total enthalpy, sqrt(rho) weights)
    const double sl_ = std::sqrt(UL[0]), sr_ = std::sqrt(UR[0]);
    const double ut = (sl_ * ul + sr_ * ur) / (sl_ + sr_);
    const double vt = (sl_ * UL[2] / UL[0] + sr_ * UR[2] / UR[0]) / (sl_ + sr_);
    const double wt = (sl_ * UL[3] / UL[0] + sr_ * UR[3] / UR[0]) / (sl_ + sr_);
    const double Ht = (sl_ * (UL[4] + pl) / UL[0] + sr_ * (UR[4] + pr) / UR[0]) / (sl_ + sr_);
    const double ct = std::sqrt((gamma - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt + wt * wt)));
    const double SL = std::min(ul - cl, ut - ct), SR = std::max(ur + cr, ut + ct);
    const double Ss = (pr - pl + UL[0] * ul * (SL - ul) - UR[0] * ur * (SR - ur)) /
                      (UL[0] * (SL - ul) - UR[0] * (SR - ur));
    double FL[5], FR[5];
    orc_flux_x(UL, gamma, B, FL);
    orc_flux_x(UR, gamma, B, FR);
    auto star = [&](const double U[5], double p, double u, double S, const double Fk[5], double out[5]) {
        const double f = U[0] * (S - u) / (S - Ss);
        const double Us[5] = {f, f * Ss, f * U[2] / U[0], f * U[3] / U[0],
                              f * (U[4] / U[0] + (Ss - u) * (Ss + p / (U[0] * (S - u))))};
        for (int k = 0; k < 5; ++k) out[k] = Fk[k] + S * (Us[k] - U[k]);
    };
    if (SL >= 0.0) {
        for (int k = 0; k < 5; ++k) F[k] = FL[k];
    } else if (Ss >= 0.0) {
        star(UL, pl, ul, SL, FL, F);
    } else if (SR > 0.0) {
        star(UR, pr, ur, SR, FR, F);
    } else {
        for (int k = 0; k < 5; ++k) F[k] = FR[k];
    }
}

static bool physical_state(const double U[5], double gamma, double B) {
    return U[0] > 0.0 && orc_pressure(U, gamma, B) + B > 0.0;
}

int orc_face_flux_x_scheme(int scheme, const double st[30], double gamma, double B, double F[5]) {
    if (scheme == 0) return orc_face_flux_x(st, gamma, B, F);
    const double *U[6];
    for (int j = 0; j < 6; ++j) U[j] = st + 5 * j;
    double R[25], L[25];
    orc_roe_matrices(U[2], U[3], gamma, B, R, L);
    double w[6][5];
    for (int j = 0; j < 6; ++j)
        for (int r = 0; r < 5; ++r) {
            double s = 0.0;
            for (int c = 0; c < 5; ++c) s += L[r * 5 + c] * U[j][c];
            w[j][r] = s;
        }
    if (scheme == 3) {
        // HLLC with WENO-AO(5,3) face states
        double wl[5], wr[5], UL[5], UR[5];
        for (int m = 0; m < 5; ++m) {
            wl[m] = orc_wao53_minus(w[0][m], w[1][m], w[2][m], w[3][m], w[4][m]);
            wr[m] = orc_wao53_minus(w[5][m], w[4][m], w[3][m], w[2][m], w[1][m]);
        }
        for (int r = 0; r < 5; ++r) {
            double sl = 0.0, sr = 0.0;
            for (int c = 0; c < 5; ++c) {
                sl += R[r * 5 + c] * wl[c];
                sr += R[r * 5 + c] * wr[c];
            }
            UL[r] = sl;
            UR[r] = sr;
        }
        if (!physical_state(UL, gamma, B))
            for (int k = 0; k < 5; ++k) UL[k] = U[2][k];
        if (!physical_state(UR, gamma, B))
            for (int k = 0; k < 5; ++k) UR[k] = U[3][k];
        orc_hllc_flux_x(UL, UR, gamma, B, F);
        return 0;
    }
    // characteristic flux splitting: Roe upwinding with LLF fallback and TENO5 (scheme 1),
    // or LLF in every field with WENO5-JS (scheme 2)
    double g[6][5];
    for (int j = 0; j < 6; ++j) {
        double f[5];
        orc_flux_x(U[j], gamma, B, f);
        for (int r = 0; r < 5; ++r) {
            double s = 0.0;
            for (int c = 0; c < 5; ++c) s += L[r * 5 + c] * f[c];
            g[j][r] = s;
        }
    }
    auto rec = [&](double a, double b, double c, double d, double e) {
        return scheme == 1 ? orc_teno5_minus(a, b, c, d, e) : weno5_js(a, b, c, d, e);
    };
    double lam[2][5];
    for (int s = 0; s < 2; ++s) {
        const double *Uc = U[2 + s];
        const double u = Uc[1] / Uc[0];
        const double c = std::sqrt(gamma * (orc_pressure(Uc, gamma, B) + B) / Uc[0]);
        lam[s][0] = u - c;
        lam[s][1] = lam[s][2] = lam[s][3] = u;
        lam[s][4] = u + c;
    }
    double gh[5];
    int n_llf = 0;
    for (int m = 0; m < 5; ++m) {
        const bool llf_only = scheme == 2;
        if (!llf_only && lam[0][m] > 0.0 && lam[1][m] > 0.0) {
            gh[m] = rec(g[0][m], g[1][m], g[2][m], g[3][m], g[4][m]);
        } else if (!llf_only && lam[0][m] < 0.0 && lam[1][m] < 0.0) {
            gh[m] = rec(g[5][m], g[4][m], g[3][m], g[2][m], g[1][m]);
        } else {
            ++n_llf;
            const double alpha = std::fmax(std::fabs(lam[0][m]), std::fabs(lam[1][m]));
            double gp[6], gm[6];
            for (int j = 0; j < 6; ++j) {
                gp[j] = 0.5 * (g[j][m] + alpha * w[j][m]);
                gm[j] = 0.5 * (g[j][m] - alpha * w[j][m]);
            }
            gh[m] = rec(gp[0], gp[1], gp[2], gp[3], gp[4]) + rec(gm[5], gm[4], gm[3], gm[2], gm[1]);
        }
    }
    for (int r = 0; r < 5; ++r) {
        double s = 0.0;
        for (int c = 0; c < 5; ++c) s += R[r * 5 + c] * gh[c];
        F[r] = s;
    }
    return n_llf;
}

int orc_face_flux_scheme(int scheme, int d, const double st[30], double gamma, double B, double F[5]) {
    const int perm[3][3] = {{1, 2, 3}, {2, 3, 1}, {3, 1, 2}};
    double r[30];
    for (int j = 0; j < 6; ++j) {
        r[5 * j + 0] = st[5 * j + 0];
        r[5 * j + 1] = st[5 * j + perm[d][0]];
        r[5 * j + 2] = st[5 * j + perm[d][1]];
        r[5 * j + 3] = st[5 * j + perm[d][2]];
        r[5 * j + 4] = st[5 * j + 4];
    }
    double Fr[5];
    const int n = orc_face_flux_x_scheme(scheme, r, gamma, B, Fr);
    F[0] = Fr[0];
    F[perm[d][0]] = Fr[1];
    F[perm[d][1]] = Fr[2];
    F[perm[d][2]] = Fr[3];
    F[4] = Fr[4];
    return n;
}

}  // extern "C"
