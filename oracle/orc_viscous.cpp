// orc_viscous.cpp -- viscous terms of the Navier-Stokes form of eq:Euler in the oracle
// (test infrastructure only).
//
// The paper solves the compressible Euler or Navier-Stokes equations; its viscous cases
// (the Rayleigh-Taylor growth-rate study, the 3D implosion of the strong-scaling runs) give
// a dynamic viscosity mu and no heat conductivity.  The stress is the Newtonian one with
// Stokes' hypothesis, tau = mu (grad v + grad v^T) - 2/3 mu (div v) I; the viscous flux
// through a face normal to axis d is (0, tau_d., tau_d. . v), subtracted from the
// convective flux.  Derivatives at a face are second-order central differences: normal
// ones from the two cells sharing the face, tangential ones the mean of the two cells'
// central differences.  The paper states no discretisation of these terms; this is the
// plain choice.
#include "orc.h"
#include <cmath>

extern "C" {

void orc_visc_face_flux(int d, const double st[50], double mu, int energy, double dx, double F[5]) {
    // v[s][n][k]: velocity component k of cell n (see orc.h) on side s
    double v[2][5][3];
    for (int s = 0; s < 2; ++s)
        for (int n = 0; n < 5; ++n) {
            const double *u = st + (s * 5 + n) * 5;
            for (int k = 0; k < 3; ++k) v[s][n][k] = u[1 + k] / u[0];
        }
    const int t_lo = d == 0 ? 1 : 0, t_hi = d == 2 ? 1 : 2;
    // G[k][a] = d v_k / d x_a at the face
    double G[3][3];
    for (int k = 0; k < 3; ++k) {
        G[k][d] = (v[1][0][k] - v[0][0][k]) / dx;
        G[k][t_lo] = 0.5 * ((v[0][2][k] - v[0][1][k]) + (v[1][2][k] - v[1][1][k])) / (2.0 * dx);
        G[k][t_hi] = 0.5 * ((v[0][4][k] - v[0][3][k]) + (v[1][4][k] - v[1][3][k])) / (2.0 * dx);
    }
    const double div = G[0][0] + G[1][1] + G[2][2];
    double tau[3];
    for (int j = 0; j < 3; ++j) tau[j] = mu * (G[d][j] + G[j][d]) - (j == d ? 2.0 / 3.0 * mu * div : 0.0);
    F[0] = 0.0;
    double work = 0.0;
    for (int j = 0; j < 3; ++j) {
        F[1 + j] = tau[j];
        work += tau[j] * 0.5 * (v[0][0][j] + v[1][0][j]);
    }
    F[4] = energy ? work : 0.0;
}

// Fourier analysis of the central operator above: the most negative eigenvalue of the
// momentum part is -(40/3) nu / dx^2 (checkerboard in all three axes, the normal component
// carrying 4/3), and SSP-RK3 is stable on the negative real axis up to about 2.51; 3/16
// keeps cfl <= 1 inside that with a margin.
double orc_visc_dt(double cfl, double dx, double mu, double rinv_max) {
    return cfl * 0.1875 * dx * dx / (mu * rinv_max);
}

double orc_rti_growth_rate(double k, double rho_h, double rho_l, double mu, double g) {
    const double ah = rho_h / (rho_l + rho_h), al = rho_l / (rho_l + rho_h);
    const double nu_h = mu / rho_h, nu_l = mu / rho_l;
    auto f = [&](double n) {
        const double ql = std::sqrt(k * k + n / nu_l), qh = std::sqrt(k * k + n / nu_h);
        return -((g * k / (n * n)) * (al - ah) + 1.0) * (ah * ql + al * qh - k) - 4.0 * k * al * ah;
    };
    // f > 0 for small n (the gravity term dominates) and f = -4 k al ah < 0 at the inviscid
    // rate sqrt(At g k), where the first bracket vanishes
    double lo = 0.0, hi = std::sqrt((ah - al) * g * k);
    if (!(hi > 0.0) || !(f(hi) < 0.0)) return -1.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        (f(mid) > 0.0 ? lo : hi) = mid;
    }
    return 0.5 * (lo + hi);
}

}  // extern "C"
