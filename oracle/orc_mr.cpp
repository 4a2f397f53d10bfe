// orc_mr.cpp -- MR operators of the oracle (test infrastructure only).
//
// Prediction: eq:Prediction with the Q-terms of the appendix ("Definitions of Q-terms"),
// written out term by term in the paper's notation.  Two printed terms are read as typos
// and corrected to the tensor-product structure every other term follows:
//   * Q_z: the c1 term uses u_{i,j,k+2} - u_{i,j,k-2} (printed u_{i+2,j,k+2}).
//   * Q_xyz, c111 group: the last pair is u_{i-2,j+2,k-2} - u_{i+2,j-2,k+2}
//     (printed u_{i+2,j-2,k-2}, which repeats the previous pair's first entry).
// Child index convention in (-1)^i: i = 0 is the lower child and receives +Q.
//
// Averaging: eq:Averaging, the mean of the 8 children, summed pairwise
// ((x-pairs, then y-pairs, then z-pair)) so that a uniform field is reproduced exactly.
#include "orc.h"

extern "C" {

static inline int floordiv2(int a) { return (a >= 0) ? a / 2 : -((-a + 1) / 2); }

double orc_predict_cell(const double *parent, int ox, int oy, int oz, int i, int j, int k) {
    // Child padded index -> parent cell (padded index) and child parity per axis.
    const int ci = i - ORC_H, cj = j - ORC_H, ck = k - ORC_H;
    const int I = ox * (ORC_IC / 2) + floordiv2(ci) + ORC_H;
    const int J = oy * (ORC_IC / 2) + floordiv2(cj) + ORC_H;
    const int K = oz * (ORC_IC / 2) + floordiv2(ck) + ORC_H;
    const int pi = ci - 2 * floordiv2(ci);
    const int pj = cj - 2 * floordiv2(cj);
    const int pk = ck - 2 * floordiv2(ck);
    auto u = [&](int a, int b, int c) -> double {
        return parent[(K + c) * ORC_P * ORC_P + (J + b) * ORC_P + (I + a)];
    };

    const double c0 = -22.0 / 128.0, c1 = 3.0 / 128.0;
    const double c00 = c0 * c0, c01 = c0 * c1, c10 = c1 * c0, c11 = c1 * c1;
    const double c000 = c0 * c0 * c0, c111 = c1 * c1 * c1;
    const double c001 = c0 * c0 * c1, c110 = c1 * c1 * c0;
    const double c011 = c0 * c1 * c1, c100 = c1 * c0 * c0;
    const double c010 = c0 * c1 * c0, c101 = c1 * c0 * c1;

    const double Qx = c0 * (u(1, 0, 0) - u(-1, 0, 0)) + c1 * (u(2, 0, 0) - u(-2, 0, 0));
    const double Qy = c0 * (u(0, 1, 0) - u(0, -1, 0)) + c1 * (u(0, 2, 0) - u(0, -2, 0));
    const double Qz = c0 * (u(0, 0, 1) - u(0, 0, -1)) + c1 * (u(0, 0, 2) - u(0, 0, -2));

    const double Qxy = c00 * ((u(1, 1, 0) + u(-1, -1, 0)) - (u(-1, 1, 0) + u(1, -1, 0))) +
                       c11 * ((u(2, 2, 0) + u(-2, -2, 0)) - (u(-2, 2, 0) + u(2, -2, 0))) +
                       c01 * ((u(1, 2, 0) + u(-1, -2, 0)) - (u(-1, 2, 0) + u(1, -2, 0))) +
                       c10 * ((u(2, 1, 0) + u(-2, -1, 0)) - (u(-2, 1, 0) + u(2, -1, 0)));
    const double Qxz = c00 * ((u(1, 0, 1) + u(-1, 0, -1)) - (u(-1, 0, 1) + u(1, 0, -1))) +
                       c11 * ((u(2, 0, 2) + u(-2, 0, -2)) - (u(-2, 0, 2) + u(2, 0, -2))) +
                       c01 * ((u(1, 0, 2) + u(-1, 0, -2)) - (u(-1, 0, 2) + u(1, 0, -2))) +
                       c10 * ((u(2, 0, 1) + u(-2, 0, -1)) - (u(-2, 0, 1) + u(2, 0, -1)));
    const double Qyz = c00 * ((u(0, 1, 1) + u(0, -1, -1)) - (u(0, -1, 1) + u(0, 1, -1))) +
                       c11 * ((u(0, 2, 2) + u(0, -2, -2)) - (u(0, -2, 2) + u(0, 2, -2))) +
                       c01 * ((u(0, 1, 2) + u(0, -1, -2)) - (u(0, -1, 2) + u(0, 1, -2))) +
                       c10 * ((u(0, 2, 1) + u(0, -2, -1)) - (u(0, -2, 1) + u(0, 2, -1)));

    // Q_xyz: for each offset triple (a,b,c), the eight sign-weighted corner values
    // grouped in four differences exactly as the appendix lists them.
    auto group = [&](int a, int b, int c) -> double {
        return (u(a, b, c) - u(-a, -b, -c)) + (u(-a, -b, c) - u(a, b, -c)) +
               (u(a, -b, -c) - u(-a, b, c)) + (u(-a, b, -c) - u(a, -b, c));
    };
    const double Qxyz = c000 * group(1, 1, 1) + c111 * group(2, 2, 2) + c001 * group(1, 1, 2) +
                        c110 * group(2, 2, 1) + c011 * group(1, 2, 2) + c100 * group(2, 1, 1) +
                        c010 * group(1, 2, 1) + c101 * group(2, 1, 2);

    const double si = pi == 0 ? 1.0 : -1.0;
    const double sj = pj == 0 ? 1.0 : -1.0;
    const double sk = pk == 0 ? 1.0 : -1.0;
    return u(0, 0, 0) + si * Qx + sj * Qy + sk * Qz + si * sj * Qxy + si * sk * Qxz +
           sj * sk * Qyz + si * sj * sk * Qxyz;
}

double orc_average8(const double c[8]) {
    // c[z*4 + y*2 + x]
    const double s = ((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7]));
    return s / 8.0;
}

}  // extern "C"
