// Corrector and end-of-step interpolation constants of the modified Hermite
// integrators (Dittmann 2020, arXiv:2006.02501), order 2(p+1), p = 1, 2, 3.
//
// Endpoint form used by the kernels: with s_k = +1 for even k, -1 for odd k,
//   v1 - v0 = sum_{k=0..p}   CV[p][k] (a1^(k) + s_k a0^(k)) dt^(k+1)
//   x1 - x0 = sum_{k=0..p+1} CX[c][p][k] (q1^(k) + s_k q0^(k)) dt^(k+1),
//   q^(0) = v (the new v1 at the end), q^(k) = a^(k-1).
//
// Velocity: Eq. 6 (even-term quadrature up to F_2p) with the even terms
// expressed through the known half sums / differences by solving the Eq. 8
// system; never printed in the paper.  At 4th order this is the standard
// 1/2, -1/12 Hermite velocity corrector.
// Position, modified (c = 0): Eq. 22 (p = 1), Eq. 23 (p = 2), Eq. 24 (p = 3),
// i.e. Eq. 7 with beta of Eq. 21 (11/3, -11/5, 163/35).
// Position, beta = 1 (c = 1): Eq. 7 with beta = 1.
// Position, shifted (c = 2): Eq. 7 with beta = 2 - beta_opt, whose last
// coefficient vanishes (the same-order velocity formula applied to x).
#pragma once

namespace hermite {

constexpr int kMaxP = 3;

// CV[p][k], k = 0..p
constexpr double CV[kMaxP + 1][kMaxP + 1] = {
    {0.0, 0.0, 0.0, 0.0},
    {1.0 / 2.0, -1.0 / 12.0, 0.0, 0.0},
    {1.0 / 2.0, -1.0 / 10.0, 1.0 / 120.0, 0.0},
    {1.0 / 2.0, -3.0 / 28.0, 1.0 / 84.0, -1.0 / 1680.0},
};

// CX[corrector][p][k], k = 0..p+1
constexpr double CX[3][kMaxP + 1][kMaxP + 2] = {
    {   // modified (Eq. 22-24)
        {0.0, 0.0, 0.0, 0.0, 0.0},
        {1.0 / 2.0, -7.0 / 60.0, 1.0 / 60.0, 0.0, 0.0},
        {1.0 / 2.0, -4.0 / 35.0, 13.0 / 840.0, -1.0 / 840.0, 0.0},
        {1.0 / 2.0, -29.0 / 252.0, 1.0 / 63.0, -1.0 / 720.0, 1.0 / 15120.0},
    },
    {   // beta = 1
        {0.0, 0.0, 0.0, 0.0, 0.0},
        {1.0 / 2.0, -1.0 / 10.0, 1.0 / 120.0, 0.0, 0.0},
        {1.0 / 2.0, -3.0 / 28.0, 1.0 / 84.0, -1.0 / 1680.0, 0.0},
        {1.0 / 2.0, -1.0 / 9.0, 1.0 / 72.0, -1.0 / 1008.0, 1.0 / 30240.0},
    },
    {   // beta = 2 - beta_opt
        {0.0, 0.0, 0.0, 0.0, 0.0},
        {1.0 / 2.0, -1.0 / 12.0, 0.0, 0.0, 0.0},
        {1.0 / 2.0, -1.0 / 10.0, 1.0 / 120.0, 0.0, 0.0},
        {1.0 / 2.0, -3.0 / 28.0, 1.0 / 84.0, -1.0 / 1680.0, 0.0},
    },
};

// End-of-step higher derivatives a^(k)(t1), k = p+1..2p-1, from the
// degree-(2p+1) Hermite interpolant through a^(0..p) at both ends of the step
// (the paper stores a^(0..2p-1) for its Taylor predictor, Sec. 3, but only
// evaluates a^(0..p); the remaining ones are carried this way):
//   a^(k)_1 dt^k = sum_m (IA0[..][m] a0^(m) + IA1[..][m] a1^(m)) dt^m.
// 6th order (p = 2): a^(3).
constexpr double I6_A0[3] = {-60.0, -24.0, -3.0};
constexpr double I6_A1[3] = {60.0, -36.0, 9.0};
// 8th order (p = 3): a^(4) then a^(5).
constexpr double I8_4_A0[4] = {840.0, 360.0, 60.0, 4.0};
constexpr double I8_4_A1[4] = {-840.0, 480.0, -120.0, 16.0};
constexpr double I8_5_A0[4] = {10080.0, 4680.0, 840.0, 60.0};
constexpr double I8_5_A1[4] = {-10080.0, 5400.0, -1200.0, 120.0};

}  // namespace hermite
