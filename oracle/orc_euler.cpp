// orc_euler.cpp -- pointwise Euler numerics of the oracle (test infrastructure only).
//
// Follows the paper's "Governing Equations" (eq:Euler, eq:StiffenedGas) and "Numerical
// Scheme" (one flux per cell face from an approximate Riemann solver, Roe type, with
// fifth-order WENO reconstruction inside the solver).  The reading used for "Roe with
// local Lax-Friedrichs fallback" is the characteristic-wise flux-split scheme: per
// characteristic field, upwind WENO when the eigenvalues of the two cells sharing the face
// agree in sign, otherwise a Rusanov (LLF) split whose speed uses only those two cells.
#include "orc.h"
#include <cmath>

extern "C" {

double orc_pressure(const double U[5], double gamma, double B) {
    const double rho = U[0];
    const double kinetic = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;
    const double rho_e = U[4] - kinetic;  // E = rho e + 1/2 rho |v|^2
    return (gamma - 1.0) * rho_e - gamma * B;
}

void orc_flux_x(const double U[5], double gamma, double B, double F[5]) {
    const double p = orc_pressure(U, gamma, B);
    const double u = U[1] / U[0];
    F[0] = U[1];
    F[1] = U[1] * u + p;
    F[2] = U[2] * u;
    F[3] = U[3] * u;
    F[4] = (U[4] + p) * u;
}

void orc_roe_matrices(const double UL[5], const double UR[5], double gamma, double B,
                      double R[25], double L[25]) {
    // Roe average with sqrt(rho) weights of velocity and total enthalpy H = (E+p)/rho.
    const double sl = std::sqrt(UL[0]);
    const double sr = std::sqrt(UR[0]);
    const double pl = orc_pressure(UL, gamma, B);
    const double pr = orc_pressure(UR, gamma, B);
    const double ul = UL[1] / UL[0], vl = UL[2] / UL[0], wl = UL[3] / UL[0];
    const double ur = UR[1] / UR[0], vr = UR[2] / UR[0], wr = UR[3] / UR[0];
    const double hl = (UL[4] + pl) / UL[0];
    const double hr = (UR[4] + pr) / UR[0];
    const double den = sl + sr;
    const double u = (sl * ul + sr * ur) / den;
    const double v = (sl * vl + sr * vr) / den;
    const double w = (sl * wl + sr * wr) / den;
    const double H = (sl * hl + sr * hr) / den;
    const double q2 = u * u + v * v + w * w;
    // For the stiffened gas c^2 = gamma (p+B)/rho = (gamma-1)(H - |v|^2/2) as well.
    const double c2 = (gamma - 1.0) * (H - 0.5 * q2);
    const double c = std::sqrt(c2);

    // Right eigenvectors as columns: (u-c, u, u, u, u+c).
    const double r[5][5] = {
        {1.0, u - c, v, w, H - u * c},
        {1.0, u, v, w, 0.5 * q2},
        {0.0, 0.0, 1.0, 0.0, v},
        {0.0, 0.0, 0.0, 1.0, w},
        {1.0, u + c, v, w, H + u * c},
    };
    for (int col = 0; col < 5; ++col)
        for (int row = 0; row < 5; ++row) R[row * 5 + col] = r[col][row];

    // Left eigenvectors (rows of R^-1), closed form with b1 = (gamma-1)/c^2, b2 = b1 |v|^2/2.
    const double b1 = (gamma - 1.0) / c2;
    const double b2 = 0.5 * q2 * b1;
    const double l[5][5] = {
        {0.5 * (b2 + u / c), 0.5 * (-b1 * u - 1.0 / c), 0.5 * (-b1 * v), 0.5 * (-b1 * w), 0.5 * b1},
        {1.0 - b2, b1 * u, b1 * v, b1 * w, -b1},
        {-v, 0.0, 1.0, 0.0, 0.0},
        {-w, 0.0, 0.0, 1.0, 0.0},
        {0.5 * (b2 - u / c), 0.5 * (-b1 * u + 1.0 / c), 0.5 * (-b1 * v), 0.5 * (-b1 * w), 0.5 * b1},
    };
    for (int row = 0; row < 5; ++row)
        for (int col = 0; col < 5; ++col) L[row * 5 + col] = l[row][col];
}

double orc_weno5_minus(double a, double b, double c, double d, double e) {
    // Three third-order candidate values at the right face of c.
    const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    const double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    const double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    // Jiang-Shu smoothness indicators.
    const double t0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, s1 = b - d;
    const double t2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
    const double beta0 = 13.0 / 12.0 * t0 * t0 + 0.25 * s0 * s0;
    const double beta1 = 13.0 / 12.0 * t1 * t1 + 0.25 * s1 * s1;
    const double beta2 = 13.0 / 12.0 * t2 * t2 + 0.25 * s2 * s2;
    const double epsw = 1e-6;
    const double a0 = 0.1 / ((epsw + beta0) * (epsw + beta0));
    const double a1 = 0.6 / ((epsw + beta1) * (epsw + beta1));
    const double a2 = 0.3 / ((epsw + beta2) * (epsw + beta2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

static double weno5_plus(double a, double b, double c, double d, double e) {
    // Right-biased reconstruction at the left face of c: the mirror image of W-.
    return orc_weno5_minus(e, d, c, b, a);
}

static void matvec5(const double M[25], const double x[5], double y[5]) {
    for (int r = 0; r < 5; ++r) {
        double s = 0.0;
        for (int c = 0; c < 5; ++c) s += M[r * 5 + c] * x[c];
        y[r] = s;
    }
}

int orc_face_flux_x(const double st[30], double gamma, double B, double F[5]) {
    const double *U[6];
    for (int j = 0; j < 6; ++j) U[j] = st + 5 * j;
    double R[25], L[25];
    orc_roe_matrices(U[2], U[3], gamma, B, R, L);

    // Characteristic variables and characteristic fluxes of the six stencil cells.
    double w[6][5], g[6][5];
    for (int j = 0; j < 6; ++j) {
        double f[5];
        orc_flux_x(U[j], gamma, B, f);
        matvec5(L, U[j], w[j]);
        matvec5(L, f, g[j]);
    }
    // Eigenvalues (u-c, u, u, u, u+c) of each of the two cells sharing the face.
    double lam[2][5];
    for (int s = 0; s < 2; ++s) {
        const double *Uc = U[2 + s];
        const double u = Uc[1] / Uc[0];
        const double c = std::sqrt(gamma * (orc_pressure(Uc, gamma, B) + B) / Uc[0]);
        lam[s][0] = u - c;
        lam[s][1] = u;
        lam[s][2] = u;
        lam[s][3] = u;
        lam[s][4] = u + c;
    }
    double gh[5];
    int n_llf = 0;
    for (int m = 0; m < 5; ++m) {
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
    matvec5(R, gh, F);
    return n_llf;
}

int orc_face_flux(int d, const double st[30], double gamma, double B, double F[5]) {
    // Rotate the momentum so that the face normal comes first: cyclic (n, t1, t2).
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
    const int n = orc_face_flux_x(r, gamma, B, Fr);
    F[0] = Fr[0];
    F[perm[d][0]] = Fr[1];
    F[perm[d][1]] = Fr[2];
    F[perm[d][2]] = Fr[3];
    F[4] = Fr[4];
    return n;
}

}  // extern "C"
