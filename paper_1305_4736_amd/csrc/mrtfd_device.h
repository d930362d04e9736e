// mrtfd_device.h -- device-side arithmetic of the D2V16 MRT-FD step for gfx950.
//
// Velocity i = 4 g + k (group g, k counter-clockwise).  Per group the four
// populations are reduced to the angular sums
//     S = sum f,  X = sum sgn(v_x) f,  Y = sum sgn(v_y) f,
//     D = f_0 - f_1 + f_2 - f_3
// and every row of M (Appendix, m_1..m_16) is a short combination of one kind
// of sum over the four groups, so fhat = M f costs 4 x 8 adds plus five small
// blocks (4x4, 4x4, 4x4, 2x2, 2x2) instead of a dense 16x16 product.  M^-1 is
// the inverse blocks followed by the inverse angular sums.  The blocks are
// built on the host (mrtfd_consts.h) and reach the kernels as arguments.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace mrtfd {

constexpr int NQ = 16;
constexpr int HALO = 2;     // ghost layers on every side

// Component signs of the 16 velocities (Sec. II, Fig. 1).
__host__ __device__ constexpr int sgx(int i)
{
    return (i < 8) ? ((i & 3) == 0 ? 1 : ((i & 3) == 2 ? -1 : 0))
                   : (((i & 3) == 0 || (i & 3) == 3) ? 1 : -1);
}
__host__ __device__ constexpr int sgy(int i)
{
    return (i < 8) ? ((i & 3) == 1 ? 1 : ((i & 3) == 3 ? -1 : 0))
                   : (((i & 3) == 0 || (i & 3) == 1) ? 1 : -1);
}

// Forward blocks: rows of M acting on the per-group sums.
//   F0: (m_1, m_4, m_5, m_14) from S_g        FX: (m_2, m_8, m_10, m_12) from X_g
//   (m_3, m_9, m_11, m_13) from Y_g are FX with the last row negated
//   FDa: (m_6, m_16) from D_0, D_1            FDd: (m_7, m_15) from D_2, D_3
// Inverse blocks (already carrying the inverse angular-sum factors 1/4, 1/2):
//   I0[g][c]  : S'_g from column c of (m_1, m_4, m_5, m_14)
//   IX[g][c], IDa[g][c], IDd[g][c] likewise; the Y block is IX with its last
//   column negated.
// MARCH2_MFMA = 1 builds the matrix-core trial of the two-step kernel: its
// second step takes the moments M f of a row as FP64 16 x 16 x 4 matrix
// products from the ring (not bitwise equal to the other kernels; for
// measurement only), reading the dense M kept in Md.
#ifndef MARCH2_MFMA
#define MARCH2_MFMA 0
#endif
struct Blocks {
    double F0[4][4], FX[4][4], FDa[2][2], FDd[2][2];
    double I0[4][4], IX[4][4], IDa[2][2], IDd[2][2];
    double vmag[4];     // |v_x| (= |v_y|) of a moving component, per group
#if MARCH2_MFMA
    double Md[NQ][NQ];  // dense M (row: moment, column: velocity)
#endif
};

// Everything a step needs that is uniform over the grid.
struct StepArgs {
    const Blocks* __restrict__ Bp;   // device copy of the blocks (read with scalar loads)
    double rdt[NQ];             // -dt * s_k: relaxation rates scaled for the update
    double b, inv_b, dt;
    double nux[4], nuy[4];      // Courant numbers |v_ia| dt / d_a per group
    double cx[4], cy[4];        // (1 - nu) / 2 per group and axis
    float nux32[4], nuy32[4];   // the same rounded to FP32 (FP32-storage convection)
    float cx32[4], cy32[4];
    // coefficients of the MC jump as limited() returns it (scaled by 4 in
    // FP64, by 2 in FP32): (1 - nu) / 8 in FP64, (1 - nu) / 4 in FP32
    double cxq[4], cyq[4];
    float cx32h[4], cy32h[4];
    double c8dt, c9dt;          // -dt (s_8 / s_5 - 1), -dt (s_9 / s_5 - 1); 0 when the correction is off
    double inv2dx, inv2dy;
    double side[4][4];          // (rho, ux, uy, T) of each side: equilibrium ghosts, walls
    int nx, ny;
    long pitch;                 // element stride between rows of a plane
    long plane;                 // element stride between planes
    long elems;                 // elements of a state buffer
    long org;                   // element offset of node (0, 0) inside a plane
    // FP32 storage only: the conserved moments (rho, j_x, j_y, e) of every
    // node in FP64, in four planes beside the populations (offsets in
    // doubles from the start of the buffer; 0 in FP64 storage)
    long corg;                  // node (0, 0) of conserved plane 0
    long cpitch;                // stride between rows
    long cplane;                // stride between the four planes
    int x0, x1, y0, y1;         // evolved node range [x0, x1) x [y0, y1)
    int ntx, nty;               // step-kernel tiles along x and y
    int per_xcd;                // tiles per XCD slot (grid = 8 * per_xcd blocks)
    int band;                   // tile columns per band of the XCD-aware order
    int m_nsx, m_nby, m_rows;   // row-marching form: strips, bands, rows per band
    int m_per_xcd;              // row-marching blocks per XCD slot
    int p_nsx, p_nby, p_rows;   // two steps per pass: strips, bands and rows per band
    int p_per_xcd;              // two steps per pass: blocks (pairs) per XCD slot
    int bc[4];                  // kinds of x-lo, x-hi, y-lo, y-hi
    int correction;
    int* flag;                  // set to 1 when a node is unphysical
};

// ---------------------------------------------------------------------------
// Angular sums of one group (axis groups 0, 1 and diagonal groups 2, 3).
template <int G>
__host__ __device__ __forceinline__ void group_sums(double f0, double f1, double f2, double f3, double& S,
                                           double& X, double& Y, double& D)
{
    double p02 = f0 + f2, p13 = f1 + f3;
    double m02 = f0 - f2, m13 = f1 - f3;
    S = p02 + p13;
    D = p02 - p13;
    if (G < 2) {
        X = m02;
        Y = m13;
    } else {
        X = m02 - m13;
        Y = m02 + m13;
    }
}

// Inverse angular sums of one group from pre-scaled S', X', Y', D'.
template <int G>
__host__ __device__ __forceinline__ void group_unsums(double S, double X, double Y, double D, double* f)
{
    if (G < 2) {
        double a = S + D, c = S - D;
        f[0] = a + X;
        f[2] = a - X;
        f[1] = c + Y;
        f[3] = c - Y;
    } else {
        double sp = S + D, sm = S - D;
        double xp = X + Y, xm = X - Y;
        f[0] = sp + xp;
        f[1] = sm - xm;
        f[2] = sp - xp;
        f[3] = sm + xm;
    }
}

struct Sums {
    double S[4], X[4], Y[4], D[4];
};

__host__ __device__ __forceinline__ Sums all_sums(const double* f)
{
    Sums a;
    group_sums<0>(f[0], f[1], f[2], f[3], a.S[0], a.X[0], a.Y[0], a.D[0]);
    group_sums<1>(f[4], f[5], f[6], f[7], a.S[1], a.X[1], a.Y[1], a.D[1]);
    group_sums<2>(f[8], f[9], f[10], f[11], a.S[2], a.X[2], a.Y[2], a.D[2]);
    group_sums<3>(f[12], f[13], f[14], f[15], a.S[3], a.X[3], a.Y[3], a.D[3]);
    return a;
}

// (r may point into any address space: generic, or the constant space the
// row-marching kernel reads its blocks from)
template <class P>
__host__ __device__ __forceinline__ double dot4(P r, const double* v)
{
    return fma(r[0], v[0], fma(r[1], v[1], fma(r[2], v[2], r[3] * v[3])));
}

// The conserved moments (m_1..m_4: rho, j_x, j_y, e) from the angular sums,
// formed exactly as moments() forms them.
template <class BT>
__host__ __device__ __forceinline__ void cons_of(const BT& B, const Sums& a, double* c)
{
    c[0] = (a.S[0] + a.S[1]) + (a.S[2] + a.S[3]);
    c[1] = dot4(B.FX[0], a.X);
    c[2] = dot4(B.FX[0], a.Y);
    c[3] = dot4(B.F0[1], a.S);
}

// fhat = M f from the angular sums (all 16 moments).
template <class BT>
__host__ __device__ __forceinline__ void moments(const BT& B, const Sums& a, double* m)
{
    m[0] = (a.S[0] + a.S[1]) + (a.S[2] + a.S[3]);
    m[3] = dot4(B.F0[1], a.S);
    m[4] = dot4(B.F0[2], a.S);
    m[13] = dot4(B.F0[3], a.S);
    m[1] = dot4(B.FX[0], a.X);
    m[7] = dot4(B.FX[1], a.X);
    m[9] = dot4(B.FX[2], a.X);
    m[11] = dot4(B.FX[3], a.X);
    m[2] = dot4(B.FX[0], a.Y);
    m[8] = dot4(B.FX[1], a.Y);
    m[10] = dot4(B.FX[2], a.Y);
    m[12] = -dot4(B.FX[3], a.Y);
    m[5] = fma(B.FDa[0][0], a.D[0], B.FDa[0][1] * a.D[1]);
    m[15] = fma(B.FDa[1][0], a.D[0], B.FDa[1][1] * a.D[1]);
    m[6] = fma(B.FDd[0][0], a.D[2], B.FDd[0][1] * a.D[3]);
    m[14] = fma(B.FDd[1][0], a.D[2], B.FDd[1][1] * a.D[3]);
}

// 1 / x from the hardware reciprocal estimate refined by two steps of
// Newton's iteration r <- r + r (1 - x r), each of which squares the
// relative error: about a third of the instructions of a correctly rounded
// division, within an ulp of it.  Every kernel forms u = j / rho and
// T = P / rho with it.
__host__ __device__ __forceinline__ double recip(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
#else
    return 1.0 / x;
#endif
}

// Equilibria of all 16 moments (Appendix, closing equations) from the
// conserved ones, R = 1, written with u = j / rho.  Returns P; eq[0..3] are
// the conserved moments themselves.
__device__ __forceinline__ void equilibria(double rho, double ux, double uy, double P, double e,
                                           double b, double* eq)
{
    double ux2 = ux * ux, uy2 = uy * uy, u2 = ux2 + uy2;
    double ru2 = rho * u2;
    double rdu = rho * (ux2 - uy2);
    double T = P * recip(rho);
    eq[0] = rho;
    eq[1] = rho * ux;
    eq[2] = rho * uy;
    eq[3] = e;
    eq[4] = 2.0 * P + ru2;
    eq[5] = rdu;
    eq[6] = rho * ux * uy;
    double e2p = e + 2.0 * P;
    eq[7] = e2p * ux;
    eq[8] = e2p * uy;
    double q4 = 4.0 * P + ru2;
    eq[9] = q4 * ux;
    eq[10] = q4 * uy;
    eq[11] = (2.0 * P + rdu) * ux;
    eq[12] = (rdu - 2.0 * P) * uy;
    eq[13] = 2.0 * (b + 2.0) * P * T + (6.0 + b) * P * u2 + ru2 * u2;
    double hb = (b + 4.0) * P + ru2;
    eq[14] = hb * ux * uy;
    eq[15] = hb * (ux2 - uy2);
}

// v = M^-1 w for a moment vector w with w_1..w_4 = 0 (the collision residual
// and the non-equilibrium part), using the pre-scaled inverse blocks.
template <class BT>
__host__ __device__ __forceinline__ void inverse_nc(const BT& B, const double* w, double* v)
{
    double S[4], X[4], Y[4], D[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        S[g] = fma(B.I0[g][2], w[4], B.I0[g][3] * w[13]);
        X[g] = fma(B.IX[g][1], w[7], fma(B.IX[g][2], w[9], B.IX[g][3] * w[11]));
        Y[g] = fma(B.IX[g][1], w[8], fma(B.IX[g][2], w[10], -B.IX[g][3] * w[12]));
    }
    D[0] = fma(B.IDa[0][0], w[5], B.IDa[0][1] * w[15]);
    D[1] = fma(B.IDa[1][0], w[5], B.IDa[1][1] * w[15]);
    D[2] = fma(B.IDd[0][0], w[6], B.IDd[0][1] * w[14]);
    D[3] = fma(B.IDd[1][0], w[6], B.IDd[1][1] * w[14]);
    group_unsums<0>(S[0], X[0], Y[0], D[0], v + 0);
    group_unsums<1>(S[1], X[1], Y[1], D[1], v + 4);
    group_unsums<2>(S[2], X[2], Y[2], D[2], v + 8);
    group_unsums<3>(S[3], X[3], Y[3], D[3], v + 12);
}

// v = M^-1 w for a full moment vector.
template <class BT>
__host__ __device__ __forceinline__ void inverse_full(const BT& B, const double* w, double* v)
{
    double S[4], X[4], Y[4], D[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        S[g] = fma(B.I0[g][0], w[0], fma(B.I0[g][1], w[3], fma(B.I0[g][2], w[4], B.I0[g][3] * w[13])));
        X[g] = fma(B.IX[g][0], w[1], fma(B.IX[g][1], w[7], fma(B.IX[g][2], w[9], B.IX[g][3] * w[11])));
        Y[g] = fma(B.IX[g][0], w[2], fma(B.IX[g][1], w[8], fma(B.IX[g][2], w[10], -B.IX[g][3] * w[12])));
    }
    D[0] = fma(B.IDa[0][0], w[5], B.IDa[0][1] * w[15]);
    D[1] = fma(B.IDa[1][0], w[5], B.IDa[1][1] * w[15]);
    D[2] = fma(B.IDd[0][0], w[6], B.IDd[0][1] * w[14]);
    D[3] = fma(B.IDd[1][0], w[6], B.IDd[1][1] * w[14]);
    group_unsums<0>(S[0], X[0], Y[0], D[0], v + 0);
    group_unsums<1>(S[1], X[1], Y[1], D[1], v + 4);
    group_unsums<2>(S[2], X[2], Y[2], D[2], v + 8);
    group_unsums<3>(S[3], X[3], Y[3], D[3], v + 12);
}

// v = M^-1 w for a moment vector whose only non-zero entries are the
// conserved ones w_1..w_4 (d[0..3]).
template <class BT>
__host__ __device__ __forceinline__ void inverse_cons(const BT& B, const double* d, double* v)
{
    double S[4], X[4], Y[4], D[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        S[g] = fma(B.I0[g][0], d[0], B.I0[g][1] * d[3]);
        X[g] = B.IX[g][0] * d[1];
        Y[g] = B.IX[g][0] * d[2];
    }
    group_unsums<0>(S[0], X[0], Y[0], D[0], v + 0);
    group_unsums<1>(S[1], X[1], Y[1], D[1], v + 4);
    group_unsums<2>(S[2], X[2], Y[2], D[2], v + 8);
    group_unsums<3>(S[3], X[3], Y[3], D[3], v + 12);
}

// FP32 storage keeps, beside the populations f~ rounded to FP32, the
// conserved moments c of the FP64 populations they were rounded from.  The
// node stands for f = f~ + M^-1 (c - M f~)_{1..4}: the rounded populations
// with their conserved moments put back to c (their other moments unchanged).
template <class BT>
__host__ __device__ __forceinline__ void resync(const BT& B, const double* ft, const double* c, double* f)
{
    double m[4], d[4], v[NQ];
    cons_of(B, all_sums(ft), m);
#pragma unroll
    for (int k = 0; k < 4; ++k) d[k] = c[k] - m[k];
    inverse_cons(B, d, v);
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i] = ft[i] + v[i];
}

// f^eq in velocity space from primitive variables (rho, u, T).
template <class BT>
__device__ __forceinline__ void feq_velocity(const BT& B, double b, double rho, double ux,
                                             double uy, double T, double* out)
{
    double P = rho * T;
    double e = b * P + rho * (ux * ux + uy * uy);
    double eq[NQ];
    equilibria(rho, ux, uy, P, e, b, eq);
    inverse_full(B, eq, out);
}

// rho, u, T of a node from its 16 populations.
template <class BT>
__device__ __forceinline__ void macro_of(const BT& B, double inv_b, const double* f,
                                         double& rho, double& ux, double& uy, double& T)
{
    Sums a = all_sums(f);
    rho = (a.S[0] + a.S[1]) + (a.S[2] + a.S[3]);
    double jx = dot4(B.FX[0], a.X);
    double jy = dot4(B.FX[0], a.Y);
    double e = dot4(B.F0[1], a.S);
    double ir = recip(rho);
    ux = jx * ir;
    uy = jy * ir;
    double P = (e - rho * (ux * ux + uy * uy)) * inv_b;
    T = P * ir;
}

// rho, u, T from the conserved moments c = (rho, j_x, j_y, e).
__device__ __forceinline__ void macro_of_cons(double inv_b, const double* c, double& rho, double& ux, double& uy,
                                              double& T)
{
    rho = c[0];
    double ir = recip(rho);
    ux = c[1] * ir;
    uy = c[2] * ir;
    double P = (c[3] - rho * (ux * ux + uy * uy)) * inv_b;
    T = P * ir;
}

// Velocity from rho and j (neighbour ring of the correction).
__device__ __forceinline__ void velocity_of_cons(double rho, double jx, double jy, double& ux, double& uy)
{
    double ir = recip(rho);
    ux = jx * ir;
    uy = jy * ir;
}

// Density and velocity only (neighbour ring of the correction).
template <class BT>
__device__ __forceinline__ void velocity_of(const BT& B, const double* f, double& ux, double& uy)
{
    Sums a = all_sums(f);
    double rho = (a.S[0] + a.S[1]) + (a.S[2] + a.S[3]);
    velocity_of_cons(rho, dot4(B.FX[0], a.X), dot4(B.FX[0], a.Y), ux, uy);
}

// ---------------------------------------------------------------------------
// Limited jump psi(theta) * dn with theta = up / dn, in division-free and
// branch-free form, equal to the printed piecewise limiter wherever theta is
// defined and zero when the downstream jump vanishes:
//   minmod: the one of up, dn nearer zero when they have the same sign, else
//           zero -- the median of (0, up, dn);
//   MC:     minmod(2 up, 2 dn, (up + dn) / 2)
//           = 2 median(0, minmod(up, dn), (up + dn) / 4)
//           = (sgn up + sgn dn) min(|up|, |dn|, |up + dn| / 4).
// Every form picks one of the candidates and scales it by a power of two,
// so all of them give the same value up to that power.  MC is returned
// scaled (lim_exp below: by 4 in FP64, by 2 in FP32) and the flux
// coefficient is scaled down to match, so the product is the same to the
// bit; the scaling is the output modifier of an instruction the limiter
// issues anyway, which saves the quarter of (up + dn) per face:
//   FP64: 4 t = min(4 min(|up|, |dn|), |up + dn|), returned as
//         copysign(4 t, up) + copysign(4 t, dn) (8 t with the common
//         sign, or 0);
//   FP32: med3(0, 4 med3(0, up, dn), up + dn) = 2 MC.
// FP64 minmod is max(min(up, dn), min(max(up, dn), 0)).  The FP64 minima
// are written as instructions: the IEEE-mode minimum of operands the
// compiler cannot prove quiet (values moved across lanes or carried round
// the loop) would otherwise first be quieted, one more instruction each,
// for NaNs that a valid state never holds.  The output modifier applies
// only with denormals flushed, which the library is built with (its
// populations, moments and their differences never come near the
// denormal range), and with the IEEE mode bit clear (convect_mode).
// Output modifiers apply only while the wave's IEEE mode bit is clear, so
// every kernel that convects clears it on entry (the bit belongs to the
// wave and is set again for the next launch).  With it clear, minimum and
// maximum treat NaN operands differently (no quieting first); arithmetic,
// comparisons and therefore the unphysical-node check are unchanged.
__device__ __forceinline__ void convect_mode()
{
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 9, 1), 0\n\ts_nop 3" ::: "memory");
}

template <int LIM, typename R>
constexpr int lim_exp() { return (LIM == 0) ? (sizeof(R) == 8 ? 2 : 1) : 0; }

__device__ __forceinline__ double min_abs3_x4(double a, double b, double c)
{
    double t;   // min(4 min(|a|, |b|), |c|)
    asm("v_min_f64 %0, |%1|, |%2| mul:4\n\tv_min_f64 %0, %0, |%3|" : "=&v"(t) : "v"(a), "v"(b), "v"(c));
    return t;
}
__device__ __forceinline__ float med3_0_x4(float a, float b)
{
    float m;    // 4 med3(0, a, b)
    asm("v_med3_f32 %0, 0, %1, %2 mul:4" : "=v"(m) : "v"(a), "v"(b));
    return m;
}
__device__ __forceinline__ double median0(double a, double b)
{
    double lo, hi;   // max(min(a, b), min(max(a, b), 0))
    asm("v_min_f64 %0, %2, %3\n\tv_max_f64 %1, %2, %3\n\tv_min_f64 %1, %1, 0\n\tv_max_f64 %0, %0, %1"
        : "=&v"(lo), "=&v"(hi) : "v"(a), "v"(b));
    return lo;
}

template <int LIM, typename R>
__device__ __forceinline__ R limited(R up, R dn)
{
    if constexpr (LIM == 2) {           // Lax-Wendroff
        return dn;
    } else if constexpr (LIM == 3) {    // first-order upwind
        return R(0);
    } else if constexpr (sizeof(R) == 4) {
        if constexpr (LIM == 0)
            return __builtin_amdgcn_fmed3f(0.0f, med3_0_x4(up, dn), up + dn);   // twice the MC jump
        else
            return __builtin_amdgcn_fmed3f(0.0f, up, dn);
    } else if constexpr (LIM == 0) {
        const R t = min_abs3_x4(up, dn, up + dn);                               // 4 times the MC jump
        return copysign(t, up) + copysign(t, dn);
    } else {
        return median0(up, dn);
    }
}

// Convective increment of one population along one axis, added to acc:
//   acc - nu [ (f_J - f_{J-s}) + c (L(f_J - f_{J-s}, f_{J+s} - f_J) - L(f_{J-s} - f_{J-2s}, f_J - f_{J-s})) ]
// with c = (1 - nu) / 2, s the sign of the velocity component.
// (conv_add is the last step, shared by every kernel so that all of them
// round it alike; the library is built with contraction of a * b + c only
// within one source expression.)
template <typename R>
__device__ __forceinline__ R conv_add(R acc, R l1, R l0, R d1, R nu, R c)
{
    return fma(-nu, fma(c, l1 - l0, d1), acc);
}

// Precision of the convective part of the step for a storage type: FP64
// storage convects in FP64; FP32 storage convects in FP32 (MRTFD_CONV64 = 1
// makes it FP64, with FP32 values widened before any difference is taken).
#ifndef MRTFD_CONV64
#define MRTFD_CONV64 0
#endif
template <typename T>
using conv_t = typename std::conditional<(MRTFD_CONV64 != 0), double, T>::type;

// A node's new population f + c + a_x + a_y (c the collision increment, a
// the two convective increments), shared by every step kernel so that all
// of them round it alike.  FP64 storage seeds the accumulator with c and
// adds f last; FP32 storage sums its FP32 convection apart and adds f, the
// sum and c in FP64.
template <typename T, typename R>
__device__ __forceinline__ R acc_start(double c)
{
    if constexpr (sizeof(T) == 8) return c;
    else return R(0);
}
// (returned in FP64 before the store rounds it to T: FP32 storage also
// keeps the conserved moments of these FP64 values)
template <typename T, typename R>
__device__ __forceinline__ double new_value(R f0, R acc, double c)
{
    if constexpr (sizeof(T) == 8) return f0 + acc;
    else return (double)f0 + (double)acc + c;
}

// Whether a storage type keeps the conserved moments in FP64 planes beside
// its populations (FP32 storage).
template <typename T>
constexpr bool keeps_cons() { return sizeof(T) == 4; }

// Courant number and (1 - nu) / 2 of group g along x (AX = 0) or y (AX = 1)
// in the convection precision R.
template <typename R, int AX, class AT>
__device__ __forceinline__ R nu_of(const AT& a, int g)
{
    if constexpr (sizeof(R) == 8) return AX ? a.nuy[g] : a.nux[g];
    else return AX ? a.nuy32[g] : a.nux32[g];
}
// (over 2^lim_exp: the coefficient of the limited jump as limited() returns it)
template <typename R, int AX, int LIM, class AT>
__device__ __forceinline__ R c_of(const AT& a, int g)
{
    static_assert(lim_exp<LIM, R>() == 0 || lim_exp<LIM, R>() == (sizeof(R) == 8 ? 2 : 1), "coefficient table");
    if constexpr (sizeof(R) == 8) {
        if constexpr (lim_exp<LIM, R>() == 2) return AX ? a.cyq[g] : a.cxq[g];
        else return AX ? a.cy[g] : a.cx[g];
    } else {
        if constexpr (lim_exp<LIM, R>() == 1) return AX ? a.cy32h[g] : a.cx32h[g];
        else return AX ? a.cy32[g] : a.cx32[g];
    }
}

template <int LIM, typename R>
__device__ __forceinline__ R conv1(R acc, R fm2, R fm1, R f0, R fp1, R nu, R c)
{
    R d0 = fm1 - fm2, d1 = f0 - fm1, d2 = fp1 - f0;
    R l1 = limited<LIM>(d1, d2);
    R l0 = limited<LIM>(d0, d1);
    return conv_add(acc, l1, l0, d1, nu, c);
}

}  // namespace mrtfd
