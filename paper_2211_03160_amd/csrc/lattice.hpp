// lattice.hpp -- compile-time lattice tables of the fused thermal LBM step.
//
// Velocity sets of Section 2.2 (Fig. 1): D2Q9 and D3Q19 for the flow
// populations f, D2Q5 and D3Q7 for the temperature populations g.
// 2D order: rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1); the
// thermal D2Q5 set is its first five.  3D order: rest, then opposite pairs
// (+x,-x), (+y,-y), (+z,-z), then the twelve edge velocities in opposite
// pairs.  Moment bases (rows = moments) have integer entries; they are the
// bases whose Guo forcing moments are the vectors of Eqs. (6a)/(6b).  All
// rows are mutually orthogonal, so M^-1 = M^T diag(1/|row|^2).
#pragma once

#include <cstdint>

namespace lbm {

enum RowKind : int {
    kRho = 0,  // conserved density (flow) or temperature (thermal)
    kJx, kJy, kJz,   // conserved momentum (flow) / relaxed heat flux (thermal)
    kE,        // energy
    kEps,      // energy square
    kQ,        // energy flux
    kNu,       // stress (shear rate)
    kPi,       // fourth-order stress companions (3D)
    kM         // third-order odd moments (3D)
};

template <int DIM> struct Flow;
template <int DIM> struct Heat;

template <> struct Flow<2> {
    static constexpr int Q = 9;
    static constexpr int ex[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int ey[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int ez[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr int opp[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
    // weights of the second-order equilibrium: 4/9, 1/9 (axes), 1/36 (diagonals)
    static constexpr double w[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr int kind[Q] = {kRho, kE, kEps, kJx, kQ, kJy, kQ, kNu, kNu};
    static constexpr int M(int k, int i) {
        const int x = ex[i], y = ey[i], s = x * x + y * y;
        switch (k) {
        case 0: return 1;
        case 1: return 3 * s - 4;
        case 2: return (9 * s * s - 21 * s + 8) / 2;
        case 3: return x;
        case 4: return (3 * s - 5) * x;
        case 5: return y;
        case 6: return (3 * s - 5) * y;
        case 7: return x * x - y * y;
        default: return x * y;
        }
    }
};

template <> struct Flow<3> {
    static constexpr int Q = 19;
    static constexpr int ex[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
    static constexpr double w[Q] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                    1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr int kind[Q] = {kRho, kE,  kEps, kJx, kQ,  kJy, kQ,  kJz, kQ, kNu,
                                    kPi,  kNu, kPi,  kNu, kNu, kNu, kM,  kM,  kM};
    static constexpr int M(int k, int i) {
        const int x = ex[i], y = ey[i], z = ez[i], s = x * x + y * y + z * z;
        switch (k) {
        case 0: return 1;
        case 1: return 19 * s - 30;
        case 2: return (21 * s * s - 53 * s + 24) / 2;
        case 3: return x;
        case 4: return (5 * s - 9) * x;
        case 5: return y;
        case 6: return (5 * s - 9) * y;
        case 7: return z;
        case 8: return (5 * s - 9) * z;
        case 9: return 3 * x * x - s;
        case 10: return (3 * s - 5) * (3 * x * x - s);
        case 11: return y * y - z * z;
        case 12: return (3 * s - 5) * (y * y - z * z);
        case 13: return x * y;
        case 14: return y * z;
        case 15: return x * z;
        case 16: return (y * y - z * z) * x;
        case 17: return (z * z - x * x) * y;
        default: return (x * x - y * y) * z;
        }
    }
};

template <> struct Heat<2> {
    static constexpr int Q = 5;
    static constexpr int ex[Q] = {0, 1, 0, -1, 0};
    static constexpr int ey[Q] = {0, 0, 1, 0, -1};
    static constexpr int ez[Q] = {0, 0, 0, 0, 0};
    static constexpr int opp[Q] = {0, 3, 4, 1, 2};
    static constexpr int kind[Q] = {kRho, kJx, kJy, kE, kNu};
    static constexpr int M(int k, int i) {
        const int x = ex[i], y = ey[i], s = x * x + y * y;
        switch (k) {
        case 0: return 1;
        case 1: return x;
        case 2: return y;
        case 3: return 5 * s - 4;
        default: return x * x - y * y;
        }
    }
    // rest-state equilibrium weights g_eq(T=1, u=0): rest (1 - a_T)/5,
    // moving (4 + a_T)/20; c_sT^2 = 2 w_moving
    static double w_rest(double a_t) { return (1.0 - a_t) / 5.0; }
    static double w_move(double a_t) { return (4.0 + a_t) / 20.0; }
    static constexpr double a_t_default = -1.5;
};

template <> struct Heat<3> {
    static constexpr int Q = 7;
    static constexpr int ex[Q] = {0, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[Q] = {0, 0, 0, 1, -1, 0, 0};
    static constexpr int ez[Q] = {0, 0, 0, 0, 0, 1, -1};
    static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5};
    static constexpr int kind[Q] = {kRho, kJx, kJy, kJz, kE, kNu, kNu};
    static constexpr int M(int k, int i) {
        const int x = ex[i], y = ey[i], z = ez[i], s = x * x + y * y + z * z;
        switch (k) {
        case 0: return 1;
        case 1: return x;
        case 2: return y;
        case 3: return z;
        case 4: return 7 * s - 6;
        case 5: return 3 * x * x - s;
        default: return y * y - z * z;
        }
    }
    static double w_rest(double a_t) { return (1.0 - a_t) / 7.0; }
    static double w_move(double a_t) { return (6.0 + a_t) / 42.0; }
    static constexpr double a_t_default = -0.75;
};

// |row k|^2 of a basis, evaluated at compile time
template <class L> constexpr int row_norm(int k) {
    int acc = 0;
    for (int i = 0; i < L::Q; ++i) acc += L::M(k, i) * L::M(k, i);
    return acc;
}

// |M_k|^2 shared by every row of one kind, or 0 if they differ
template <class L> constexpr int kind_norm(int kind) {
    int n = 0;
    for (int k = 0; k < L::Q; ++k) {
        if (L::kind[k] != kind) continue;
        const int r = row_norm<L>(k);
        if (n == 0) n = r;
        else if (n != r) return 0;
    }
    return n;
}

// true when every kind's rows share |M_k|^2, so that a relaxation rate per
// kind can carry the 1/|M_k|^2 of the inverse transform (D2Q9 and D2Q5: yes;
// D3Q19, whose rows 3p_xx and p_ww relax together: no)
template <class L> constexpr bool kinds_share_norm() {
    for (int k = 0; k < L::Q; ++k)
        if (kind_norm<L>(L::kind[k]) == 0) return false;
    return true;
}

}  // namespace lbm
