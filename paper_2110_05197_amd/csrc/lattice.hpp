// lattice.hpp -- D2Q9 and D3Q19 velocity sets and the colour-gradient
// constants, as compile-time tables for the device code.
//
// D3Q19 (arXiv:2110.05197, section 2): velocities Eq. speeds, weights
// Eq. weights, perturbation constants B_i (after Eq. perturbationOp),
// enhanced-equilibrium constants psi_i and xi_i (after Eq. phi) and the rest
// fractions phi_i(alpha) of Eq. phi: alpha, (1-alpha)/12, (1-alpha)/24.
// D2Q9 is not in the paper; its constants satisfy the same moment
// conditions: phi alpha, (1-alpha)/5, (1-alpha)/20; B -4/27, 2/27, 5/108;
// psi -8/3, -1/6, 1/12; xi 0, 1/2, 1/8.
//
// Ordering: 0 = rest, then opposite pairs (i, i+1) for odd i, axis
// directions before diagonals.  The "group" of a direction is |c|^2 (0, 1, 2).
#pragma once

namespace mclbm {

struct D2Q9 {
    static constexpr int D = 2;
    static constexpr int Q = 9;
    static constexpr int cx[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int cy[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int grp[9] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
    // per group: rest, axis, diagonal
    static constexpr double w[3] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0};
    static constexpr double B[3] = {-4.0 / 27.0, 2.0 / 27.0, 5.0 / 108.0};
    static constexpr double psi[3] = {-8.0 / 3.0, -1.0 / 6.0, 1.0 / 12.0};
    static constexpr double xi[3] = {0.0, 0.5, 0.125};
    // phi(alpha) = phi_a * alpha + phi_b
    static constexpr double phi_a[3] = {1.0, -0.2, -0.05};
    static constexpr double phi_b[3] = {0.0, 0.2, 0.05};
    static constexpr double inv_len[3] = {0.0, 1.0, 0.70710678118654752440};
};

struct D3Q19 {
    static constexpr int D = 3;
    static constexpr int Q = 19;
    static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int grp[19] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};
    static constexpr double w[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    static constexpr double B[3] = {-2.0 / 9.0, 1.0 / 54.0, 1.0 / 27.0};
    static constexpr double psi[3] = {-2.5, -1.0 / 6.0, 1.0 / 24.0};
    static constexpr double xi[3] = {0.0, 0.25, 0.125};
    static constexpr double phi_a[3] = {1.0, -1.0 / 12.0, -1.0 / 24.0};
    static constexpr double phi_b[3] = {0.0, 1.0 / 12.0, 1.0 / 24.0};
    static constexpr double inv_len[3] = {0.0, 1.0, 0.70710678118654752440};
};

// D2Q9 seen as a 3-D lattice of a single y plane: velocities (cx, 0, cy),
// same order and constants.  A 2-D box nx x ny is then the 3-D box
// nx x 1 x ny with the same node numbering, and the one-pass kernel marches
// along the 2-D y axis.
struct D2Q9Z : D2Q9 {
    static constexpr int cy[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int cz[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
};

// Multirange neighbourhood of the two-component Shan-Chen forces (Eq.
// pweights): the vectors of {-2..2}^3 with |c|^2 in {1, 2, 3, 4, 5, 6, 8}
// (92 of them; belt 1 is |c|^2 <= 2, the D3Q19 set).  Both weights are even
// in c, so the table keeps one vector of each pair (c, -c) -- the one whose
// last non-zero component is positive -- and a force sum over the
// neighbourhood is taken pairwise, sum_b weight_b (X(x + c_b) - X(x - c_b)) c_b.
// p_b by shell: 4/135, 1/63, 2/315, 5/1512, 1/945, 1/1890, 1/15120;
// w_b: the D3Q19 weight on belt 1 (1/18, 1/36), zero on belt 2.
struct BeltTable {
    int c[46][3];
    double p[46];
    double w[46];
};

constexpr double belt_weight_p(int r2)
{
    return r2 == 1 ? 4.0 / 135.0 : r2 == 2 ? 1.0 / 63.0 : r2 == 3 ? 2.0 / 315.0 : r2 == 4 ? 5.0 / 1512.0
         : r2 == 5 ? 1.0 / 945.0 : r2 == 6 ? 1.0 / 1890.0 : r2 == 8 ? 1.0 / 15120.0 : 0.0;
}

constexpr BeltTable make_belt_table()
{
    BeltTable T{};
    int k = 0;
    const int shells[7] = {1, 2, 3, 4, 5, 6, 8};
    for (int s = 0; s < 7; ++s)
        for (int a = -2; a <= 2; ++a)
            for (int b = -2; b <= 2; ++b)
                for (int c = -2; c <= 2; ++c) {
                    if (a * a + b * b + c * c != shells[s]) continue;
                    const int last = c != 0 ? c : (b != 0 ? b : a);
                    if (last < 0) continue;
                    T.c[k][0] = a;
                    T.c[k][1] = b;
                    T.c[k][2] = c;
                    T.p[k] = belt_weight_p(shells[s]);
                    T.w[k] = shells[s] == 1 ? 1.0 / 18.0 : (shells[s] == 2 ? 1.0 / 36.0 : 0.0);
                    ++k;
                }
    return T;
}

struct Belts {
    static constexpr int n = 46;
    static constexpr BeltTable tab = make_belt_table();
};

}  // namespace mclbm
