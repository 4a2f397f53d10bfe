// orc_riemann.cpp -- exact solution of the 1D Riemann problem for an ideal gas
// (test infrastructure only).  Textbook construction (Toro, "Riemann Solvers and
// Numerical Methods for Fluid Dynamics", ch. 4): Newton iteration on the pressure
// function f(p) = f_L(p) + f_R(p) + (u_R - u_L) for the star pressure, then sampling of
// the self-similar wave pattern at speed s = x/t.  It serves as the closed-form pin of the
// Sod shock tube used in the paper's verification section.
#include "orc.h"
#include <cmath>

namespace {
struct Side { double rho, u, p, c; };

// f_K(p) and its derivative for one side (shock if p > p_K, rarefaction otherwise).
void pressure_fn(double p, const Side &K, double g, double *f, double *df) {
    if (p > K.p) {
        const double A = 2.0 / ((g + 1.0) * K.rho);
        const double Bc = (g - 1.0) / (g + 1.0) * K.p;
        const double q = std::sqrt(A / (p + Bc));
        *f = (p - K.p) * q;
        *df = q * (1.0 - 0.5 * (p - K.p) / (p + Bc));
    } else {
        const double pr = p / K.p;
        *f = 2.0 * K.c / (g - 1.0) * (std::pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
        *df = 1.0 / (K.rho * K.c) * std::pow(pr, -(g + 1.0) / (2.0 * g));
    }
}
}  // namespace

extern "C" int orc_exact_riemann(double rl, double ul, double pl, double rr, double ur,
                                 double pr, double g, const double *s, int n, double *out) {
    const Side L{rl, ul, pl, std::sqrt(g * pl / rl)};
    const Side R{rr, ur, pr, std::sqrt(g * pr / rr)};
    // Newton iteration from the two-rarefaction guess.
    const double z = (g - 1.0) / (2.0 * g);
    double p = std::pow((L.c + R.c - 0.5 * (g - 1.0) * (R.u - L.u)) /
                            (L.c / std::pow(L.p, z) + R.c / std::pow(R.p, z)),
                        1.0 / z);
    if (!(p > 0.0)) p = 1e-8;
    bool ok = false;
    for (int it = 0; it < 100; ++it) {
        double fl, dfl, fr, dfr;
        pressure_fn(p, L, g, &fl, &dfl);
        pressure_fn(p, R, g, &fr, &dfr);
        double pn = p - (fl + fr + R.u - L.u) / (dfl + dfr);
        if (pn < 1e-12) pn = 1e-12;
        const double change = 2.0 * std::fabs(pn - p) / (pn + p);
        p = pn;
        if (change < 1e-14) { ok = true; break; }
    }
    if (!ok) return -1;
    double fl, dfl, fr, dfr;
    pressure_fn(p, L, g, &fl, &dfl);
    pressure_fn(p, R, g, &fr, &dfr);
    const double us = 0.5 * (L.u + R.u) + 0.5 * (fr - fl);
    const double gm = (g - 1.0) / (g + 1.0);

    for (int i = 0; i < n; ++i) {
        const double S = s[i];
        double rho, u, pp;
        if (S <= us) {  // left of the contact
            if (p > L.p) {  // left shock
                const double SL = L.u - L.c * std::sqrt((g + 1.0) / (2.0 * g) * p / L.p + z);
                if (S <= SL) { rho = L.rho; u = L.u; pp = L.p; }
                else { rho = L.rho * (p / L.p + gm) / (gm * p / L.p + 1.0); u = us; pp = p; }
            } else {  // left rarefaction
                const double SHL = L.u - L.c;
                const double cs = L.c * std::pow(p / L.p, z);
                const double STL = us - cs;
                if (S <= SHL) { rho = L.rho; u = L.u; pp = L.p; }
                else if (S >= STL) { rho = L.rho * std::pow(p / L.p, 1.0 / g); u = us; pp = p; }
                else {
                    u = 2.0 / (g + 1.0) * (L.c + 0.5 * (g - 1.0) * L.u + S);
                    const double c = 2.0 / (g + 1.0) * (L.c + 0.5 * (g - 1.0) * (L.u - S));
                    rho = L.rho * std::pow(c / L.c, 2.0 / (g - 1.0));
                    pp = L.p * std::pow(c / L.c, 2.0 * g / (g - 1.0));
                }
            }
        } else {  // right of the contact
            if (p > R.p) {  // right shock
                const double SR = R.u + R.c * std::sqrt((g + 1.0) / (2.0 * g) * p / R.p + z);
                if (S >= SR) { rho = R.rho; u = R.u; pp = R.p; }
                else { rho = R.rho * (p / R.p + gm) / (gm * p / R.p + 1.0); u = us; pp = p; }
            } else {  // right rarefaction
                const double SHR = R.u + R.c;
                const double cs = R.c * std::pow(p / R.p, z);
                const double STR = us + cs;
                if (S >= SHR) { rho = R.rho; u = R.u; pp = R.p; }
                else if (S <= STR) { rho = R.rho * std::pow(p / R.p, 1.0 / g); u = us; pp = p; }
                else {
                    u = 2.0 / (g + 1.0) * (-R.c + 0.5 * (g - 1.0) * R.u + S);
                    const double c = 2.0 / (g + 1.0) * (R.c - 0.5 * (g - 1.0) * (R.u - S));
                    rho = R.rho * std::pow(c / R.c, 2.0 / (g - 1.0));
                    pp = R.p * std::pow(c / R.c, 2.0 * g / (g - 1.0));
                }
            }
        }
        out[3 * i + 0] = rho;
        out[3 * i + 1] = u;
        out[3 * i + 2] = pp;
    }
    return 0;
}
