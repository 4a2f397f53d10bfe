// orc_tait.cpp -- Tait's equation of state in the oracle (test infrastructure only).
//
// Sec. "Influence of Equation of State" replaces the stiffened gas by Tait's equation
// (after Fedkiw et al. 1999), p = B ((rho/rho0)^gamma - 1) + A.  The pressure then depends
// on the density alone and the energy equation of eq:Euler drops out: the energy becomes
// a dependent variable and is not evolved (it stays zero here).  The remaining system
// (rho, rho v) is solved with the standard configuration's flux kernel: characteristic
// WENO5-JS inside a Roe solver with a per-field local Lax-Friedrichs fallback, the fields
// now being (u - c, u, u, u + c) with c^2 = dp/drho.  The Roe average uses sqrt(rho)
// weights for the velocity and c~^2 = (p_R - p_L)/(rho_R - rho_L) (dp/drho at the mean
// density when the densities agree), which makes F(U_R) - F(U_L) = A~ (U_R - U_L) exact.
#include "orc.h"
#include <cmath>

namespace {

double tait_p(double rho, const double t[4]) {
    // t = (gamma, B, A, rho0)
    return t[1] * (std::pow(rho / t[3], t[0]) - 1.0) + t[2];
}

double tait_c2(double rho, const double t[4]) {
    return t[0] * t[1] / t[3] * std::pow(rho / t[3], t[0] - 1.0);
}

double weno5_plus(double a, double b, double c, double d, double e) {
    return orc_weno5_minus(e, d, c, b, a);
}

}  // namespace

extern "C" {

double orc_tait_pressure(double rho, double gamma, double B, double A, double rho0) {
    const double t[4] = {gamma, B, A, rho0};
    return tait_p(rho, t);
}

double orc_tait_sound_speed(double rho, double gamma, double B, double rho0) {
    const double t[4] = {gamma, B, 0.0, rho0};
    return std::sqrt(tait_c2(rho, t));
}

void orc_tait_flux_x(const double U[5], double gamma, double B, double A, double rho0, double F[5]) {
    const double t[4] = {gamma, B, A, rho0};
    const double u = U[1] / U[0];
    F[0] = U[1];
    F[1] = U[1] * u + tait_p(U[0], t);
    F[2] = U[2] * u;
    F[3] = U[3] * u;
    F[4] = 0.0;
}

void orc_tait_roe_matrices(const double UL[5], const double UR[5], double gamma, double B, double A,
                           double rho0, double R[16], double L[16]) {
    const double t[4] = {gamma, B, A, rho0};
    const double sl = std::sqrt(UL[0]), sr = std::sqrt(UR[0]);
    const double u = (UL[1] / sl + UR[1] / sr) / (sl + sr);
    const double v = (UL[2] / sl + UR[2] / sr) / (sl + sr);
    const double w = (UL[3] / sl + UR[3] / sr) / (sl + sr);
    const double drho = UR[0] - UL[0];
    double c2;
    if (std::fabs(drho) > 1e-9 * (UL[0] + UR[0]))
        c2 = (tait_p(UR[0], t) - tait_p(UL[0], t)) / drho;
    else
        c2 = tait_c2(0.5 * (UL[0] + UR[0]), t);
    const double c = std::sqrt(c2);
    // right eigenvectors as columns, fields (u - c, u, u, u + c) on (rho, m1, m2, m3)
    const double r[4][4] = {{1.0, u - c, v, w}, {0.0, 0.0, 1.0, 0.0}, {0.0, 0.0, 0.0, 1.0}, {1.0, u + c, v, w}};
    for (int col = 0; col < 4; ++col)
        for (int row = 0; row < 4; ++row) R[row * 4 + col] = r[col][row];
    const double l[4][4] = {{(u + c) / (2.0 * c), -1.0 / (2.0 * c), 0.0, 0.0},
                            {-v, 0.0, 1.0, 0.0},
                            {-w, 0.0, 0.0, 1.0},
                            {-(u - c) / (2.0 * c), 1.0 / (2.0 * c), 0.0, 0.0}};
    for (int row = 0; row < 4; ++row)
        for (int col = 0; col < 4; ++col) L[row * 4 + col] = l[row][col];
}

int orc_tait_face_flux_x(const double st[30], double gamma, double B, double A, double rho0,
                         double F[5]) {
    const double t[4] = {gamma, B, A, rho0};
    const double *U[6];
    for (int j = 0; j < 6; ++j) U[j] = st + 5 * j;
    double R[16], L[16];
    orc_tait_roe_matrices(U[2], U[3], gamma, B, A, rho0, R, L);
    double w[6][4], g[6][4];
    for (int j = 0; j < 6; ++j) {
        double f[5];
        orc_tait_flux_x(U[j], gamma, B, A, rho0, f);
        for (int m = 0; m < 4; ++m) {
            double sw = 0.0, sg = 0.0;
            for (int k = 0; k < 4; ++k) {
                sw += L[m * 4 + k] * U[j][k];
                sg += L[m * 4 + k] * f[k];
            }
            w[j][m] = sw;
            g[j][m] = sg;
        }
    }
    double lam[2][4];
    for (int s = 0; s < 2; ++s) {
        const double *Uc = U[2 + s];
        const double u = Uc[1] / Uc[0], c = std::sqrt(tait_c2(Uc[0], t));
        lam[s][0] = u - c;
        lam[s][1] = u;
        lam[s][2] = u;
        lam[s][3] = u + c;
    }
    double gh[4];
    int n_llf = 0;
    for (int m = 0; m < 4; ++m) {
        if (lam[0][m] > 0.0 && lam[1][m] > 0.0) {
            gh[m] = orc_weno5_minus(g[0][m], g[1][m], g[2][m], g[3][m], g[4][m]);
        } else if (lam[0][m] < 0.0 && lam[1][m] < 0.0) {
            gh[m] = weno5_plus(g[1][m], g[2][m], g[3][m], g[4][m], g[5][m]);
        } else {
            ++n_llf;
            const double alpha = std::fmax(std::fabs(lam[0][m]), std::fabs(lam[1][m]));
            double gp[6], gm[6];
            for (int j = 0; j < 6; ++j) {
                gp[j] = 0.5 * (g[j][m] + alpha * w[j][m]);
                gm[j] = 0.5 * (g[j][m] - alpha * w[j][m]);
            }
            gh[m] = orc_weno5_minus(gp[0], gp[1], gp[2], gp[3], gp[4]) +
                    weno5_plus(gm[1], gm[2], gm[3], gm[4], gm[5]);
        }
    }
    for (int row = 0; row < 4; ++row) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += R[row * 4 + k] * gh[k];
        F[row] = s;
    }
    F[4] = 0.0;
    return n_llf;
}

int orc_tait_face_flux(int d, const double st[30], double gamma, double B, double A, double rho0,
                       double F[5]) {
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
    const int n = orc_tait_face_flux_x(r, gamma, B, A, rho0, Fr);
    F[0] = Fr[0];
    F[perm[d][0]] = Fr[1];
    F[perm[d][1]] = Fr[2];
    F[perm[d][2]] = Fr[3];
    F[4] = 0.0;
    return n;
}

// Exact solution of the 1D Riemann problem of the barotropic system: the 1- and 4-waves
// are shocks (Rankine-Hugoniot: mass flux j with j^2 = (p* - p_K)/(1/rho_K - 1/rho*)) or
// rarefactions (Riemann invariant u +- 2c/(gamma - 1), which for Tait's c(rho) integrates
// int c/rho drho in closed form); the middle state (rho*, u*) joins them, found by
// bisection on rho*.  out[2 i..] = (rho, u) at x/t = s[i].
int orc_tait_exact_riemann(double rl, double ul, double rr, double ur, double gamma, double B,
                           double A, double rho0, const double *s, int n, double *out) {
    const double t[4] = {gamma, B, A, rho0};
    const double k = 2.0 / (gamma - 1.0);
    // velocity change across the K-wave as a function of the middle density
    auto f = [&](double r, double rk) {
        if (r > rk) {
            const double dp = tait_p(r, t) - tait_p(rk, t);
            return std::sqrt(dp * (r - rk) / (r * rk));
        }
        return k * (std::sqrt(tait_c2(r, t)) - std::sqrt(tait_c2(rk, t)));
    };
    auto g = [&](double r) { return f(r, rl) + f(r, rr) + (ur - ul); };
    double lo = 1e-12 * std::fmin(rl, rr), hi = 10.0 * std::fmax(rl, rr);
    if (g(lo) > 0.0) return -1;   // vacuum forms
    while (g(hi) < 0.0) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        (g(mid) < 0.0 ? lo : hi) = mid;
    }
    const double rs = 0.5 * (lo + hi);
    const double us = 0.5 * (ul + ur) + 0.5 * (f(rs, rr) - f(rs, rl));
    const double cl = std::sqrt(tait_c2(rl, t)), cr = std::sqrt(tait_c2(rr, t));
    const double cs = std::sqrt(tait_c2(rs, t));
    for (int i = 0; i < n; ++i) {
        const double x = s[i];
        double rho, u;
        if (x <= us) {   // left of the contact
            if (rs > rl) {   // left shock
                const double sh = (rs * us - rl * ul) / (rs - rl);
                rho = x < sh ? rl : rs;
                u = x < sh ? ul : us;
            } else if (x <= ul - cl) {
                rho = rl;
                u = ul;
            } else if (x >= us - cs) {
                rho = rs;
                u = us;
            } else {   // inside the left fan: u - c = x, u + k c = ul + k cl
                const double c = (ul + k * cl - x) / (k + 1.0);
                rho = rho0 * std::pow(c * c * rho0 / (gamma * B), 1.0 / (gamma - 1.0));
                u = x + c;
            }
        } else {
            if (rs > rr) {   // right shock
                const double sh = (rs * us - rr * ur) / (rs - rr);
                rho = x > sh ? rr : rs;
                u = x > sh ? ur : us;
            } else if (x >= ur + cr) {
                rho = rr;
                u = ur;
            } else if (x <= us + cs) {
                rho = rs;
                u = us;
            } else {   // inside the right fan: u + c = x, u - k c = ur - k cr
                const double c = (x - ur + k * cr) / (k + 1.0);
                rho = rho0 * std::pow(c * c * rho0 / (gamma * B), 1.0 / (gamma - 1.0));
                u = x - c;
            }
        }
        out[2 * i] = rho;
        out[2 * i + 1] = u;
    }
    return 0;
}

}  // extern "C"
