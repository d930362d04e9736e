// mrtfd_consts.h -- host construction of the factored transformation matrix.
//
// With S, X, Y, D the per-group angular sums (mrtfd_device.h), the rows of M
// (Appendix, m_1..m_16) reduce to, per group g with moving-component size
// a_g (1, 6, sqrt 2, 3/sqrt 2), speed^2 c2_g (1, 36, 4, 9) and eta_g^2
// (eta0^2 on the |v| = 1 group, 0 elsewhere):
//   m_1 = sum S          m_4 = sum (c2+eta2) S     m_5 = sum c2 S
//   m_14 = sum c2 (c2+eta2) S
//   m_2 = sum a X        m_8 = sum a (c2+eta2) X   m_10 = sum a c2 X
//   m_12 = sum_axis a^3 X                 (v_x (v_x^2 - v_y^2) vanishes on diagonals)
//   m_3, m_9, m_11 likewise with Y;  m_13 = - sum_axis a^3 Y
//   m_6 = sum_axis c2 D    m_16 = sum_axis c2 (c2+eta2) D
//   m_7 = sum_diag a^2 D   m_15 = sum_diag a^2 c2 D
// The blocks are inverted in long double; the inverse angular sums contribute
// 1/4 (S, D, diagonal X and Y) and 1/2 (axis X and Y).
#pragma once
#include <cmath>
#include <cstring>

#include "mrtfd_device.h"

namespace mrtfd {

template <int N>
static bool invert_small(const long double (&A)[N][N], long double (&X)[N][N])
{
    long double a[N][2 * N];
    for (int r = 0; r < N; ++r)
        for (int c = 0; c < 2 * N; ++c) a[r][c] = (c < N) ? A[r][c] : (long double)((c - N) == r);
    for (int col = 0; col < N; ++col) {
        int piv = col;
        for (int r = col + 1; r < N; ++r)
            if (fabsl(a[r][col]) > fabsl(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0L) return false;
        for (int c = 0; c < 2 * N; ++c) {
            long double t = a[col][c];
            a[col][c] = a[piv][c];
            a[piv][c] = t;
        }
        long double iv = 1.0L / a[col][col];
        for (int c = 0; c < 2 * N; ++c) a[col][c] *= iv;
        for (int r = 0; r < N; ++r) {
            if (r == col) continue;
            long double m = a[r][col];
            for (int c = 0; c < 2 * N; ++c) a[r][c] -= m * a[col][c];
        }
    }
    for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) X[r][c] = a[r][N + c];
    return true;
}

static bool build_blocks(double eta0, Blocks* out)
{
    const long double r2 = sqrtl(2.0L);
    const long double a[4] = {1.0L, 6.0L, r2, 3.0L / r2};
    long double c2[4], e2[4];
    for (int g = 0; g < 4; ++g) {
        c2[g] = (g < 2) ? a[g] * a[g] : 2.0L * a[g] * a[g];
        e2[g] = (g == 0) ? (long double)eta0 * eta0 : 0.0L;
    }
    long double F0[4][4], FX[4][4], FY[4][4], FDa[2][2], FDd[2][2];
    for (int g = 0; g < 4; ++g) {
        long double ax = (g < 2) ? 1.0L : 0.0L;
        F0[0][g] = 1.0L;
        F0[1][g] = c2[g] + e2[g];
        F0[2][g] = c2[g];
        F0[3][g] = c2[g] * (c2[g] + e2[g]);
        FX[0][g] = a[g];
        FX[1][g] = a[g] * (c2[g] + e2[g]);
        FX[2][g] = a[g] * c2[g];
        FX[3][g] = ax * a[g] * a[g] * a[g];
        FY[0][g] = a[g];
        FY[1][g] = a[g] * (c2[g] + e2[g]);
        FY[2][g] = a[g] * c2[g];
        FY[3][g] = -ax * a[g] * a[g] * a[g];
    }
    for (int g = 0; g < 2; ++g) {
        FDa[0][g] = c2[g];
        FDa[1][g] = c2[g] * (c2[g] + e2[g]);
        FDd[0][g] = a[2 + g] * a[2 + g];
        FDd[1][g] = a[2 + g] * a[2 + g] * c2[2 + g];
    }
    long double I0[4][4], IX[4][4], IY[4][4], IDa[2][2], IDd[2][2];
    if (!invert_small<4>(F0, I0) || !invert_small<4>(FX, IX) || !invert_small<4>(FY, IY) ||
        !invert_small<2>(FDa, IDa) || !invert_small<2>(FDd, IDd))
        return false;
    // the Y block is the X block with its last row negated, so its inverse is
    // the X inverse with its last column negated
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 4; ++k)
            if (fabsl(IY[r][k] - (k == 3 ? -IX[r][k] : IX[r][k])) > 1e-15L * (1.0L + fabsl(IX[r][k]))) return false;
    Blocks& B = *out;
    std::memset(&B, 0, sizeof(B));
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            B.F0[r][c] = (double)F0[r][c];
            B.FX[r][c] = (double)FX[r][c];
            long double sx = (r < 2) ? 0.5L : 0.25L;   // row r of an inverse is group r
            B.I0[r][c] = (double)(0.25L * I0[r][c]);
            B.IX[r][c] = (double)(sx * IX[r][c]);
        }
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            B.FDa[r][c] = (double)FDa[r][c];
            B.FDd[r][c] = (double)FDd[r][c];
            B.IDa[r][c] = (double)(0.25L * IDa[r][c]);
            B.IDd[r][c] = (double)(0.25L * IDd[r][c]);
        }
    for (int g = 0; g < 4; ++g) B.vmag[g] = (double)a[g];
#if MARCH2_MFMA
    for (int k = 0; k < NQ; ++k) {
        double e[NQ] = {0.0}, m[NQ];
        e[k] = 1.0;
        moments(B, all_sums(e), m);
        for (int i = 0; i < NQ; ++i) B.Md[i][k] = m[i];
    }
#endif
    return true;
}

}  // namespace mrtfd
