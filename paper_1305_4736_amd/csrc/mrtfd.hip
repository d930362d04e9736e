// mrtfd.hip -- gfx950 kernels and the C ABI (include/mrtfd.h) of the D2V16
// MRT finite-difference lattice-Boltzmann step (arXiv:1305.4736).
//
// State layout in HBM: 16 planes (structure of arrays, one per velocity),
// each (ny + 4) rows of `pitch` elements; node (x, y) of plane i sits at
// i * plane + org + y * pitch + x, with two ghost layers on every side and
// the first interior node of a row on a 128-byte line.  Two such buffers
// ping-pong between steps.
//
// One time step is ONE kernel launch (k_step): every thread owns one evolved
// node and computes, from level n only,
//   moments and macroscopic state (Sec. II), the velocity of its four axis
//   neighbours (energy-flux correction, Sec. II), equilibria (Appendix),
//   the relaxed residual and its image in velocity space (Sec. III update
//   eq.), the limited x and y flux differences of its 16 populations
//   (Sec. III flux / limiter eqs.), the new populations, and the boundary
//   images it is responsible for (periodic and outflow ghosts, the wall node
//   and ghosts next to it).  Equilibrium ghosts are constant and written once.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mrtfd.h"
#include "mrtfd_consts.h"
#include "mrtfd_device.h"

using namespace mrtfd;

namespace {

enum { BC_PERIODIC = MRTFD_BC_PERIODIC, BC_EQUIL = MRTFD_BC_EQUILIBRIUM, BC_OUTFLOW = MRTFD_BC_OUTFLOW,
       BC_WALL = MRTFD_BC_WALL_NEE };

constexpr int BX = 64;   // threads along x per block (one wavefront)
constexpr int BY = 4;    // rows per block
// Step-kernel tile (nodes per block = threads per block): TXW x BYR.
#ifndef STEP_TXW64
#define STEP_TXW64 32
#endif
#ifndef STEP_BYR64
#define STEP_BYR64 4
#endif
#ifndef STEP_TXW32
#define STEP_TXW32 32
#endif
#ifndef STEP_BYR32
#define STEP_BYR32 8
#endif
template <typename T> struct TileOf;
template <> struct TileOf<double> { static constexpr int TXW = STEP_TXW64, BYR = STEP_BYR64; };
template <> struct TileOf<float> { static constexpr int TXW = STEP_TXW32, BYR = STEP_BYR32; };
#ifndef STEP_WAVES_PER_SIMD
#define STEP_WAVES_PER_SIMD 4
#endif
#ifndef STEP_PREFETCH
#define STEP_PREFETCH 4   // planes staged ahead in registers
#endif
#ifndef STEP_BAND
#define STEP_BAND (1 << 20)   // tile columns per band of the XCD-aware tile order (default: whole rows)
#endif
#ifndef STEP_PLANE_FENCE
#define STEP_PLANE_FENCE() __builtin_amdgcn_sched_barrier(0)
#endif

__device__ __forceinline__ long node(const StepArgs& a, int x, int y)
{
    return a.org + (long)y * a.pitch + x;
}

template <typename T>
__device__ __forceinline__ void load16(const T* __restrict__ f, const StepArgs& a, long n, double* out)
{
#pragma unroll
    for (int i = 0; i < NQ; ++i) out[i] = (double)f[i * a.plane + n];
}

template <typename T>
__device__ __forceinline__ void store16(T* __restrict__ f, const StepArgs& a, long n, const T* v)
{
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i * a.plane + n] = v[i];
}

// Non-equilibrium extrapolation wall from the fluid node next to it (f1):
// wall node n_w and its two ghosts n_w + step, n_w + 2 step.
template <typename T>
__device__ void wall_fill(const StepArgs& a, T* __restrict__ f, const double* f1, int side, long nw, long step)
{
    double r1, u1x, u1y, T1;
    macro_of(*a.Bp, a.inv_b, f1, r1, u1x, u1y, T1);
    const double* st = a.side[side];
    double rw = r1 * T1 / st[3];           // carry the pressure over: rho_w T_w = rho_1 T_1
    double ew[NQ], e1[NQ];
    feq_velocity(*a.Bp, a.b, rw, st[1], st[2], st[3], ew);
    feq_velocity(*a.Bp, a.b, r1, u1x, u1y, T1, e1);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        double fw = ew[i] + (f1[i] - e1[i]);
        f[i * a.plane + nw] = (T)fw;
        f[i * a.plane + nw + step] = (T)(2.0 * fw - f1[i]);
        f[i * a.plane + nw + 2 * step] = (T)(3.0 * fw - 2.0 * f1[i]);
    }
}

// ---------------------------------------------------------------------------
// The fused step, per node.

// Relaxed residual of the non-conserved moments, mapped back to velocity
// space and scaled by -dt (the collision term of the update).
__device__ __forceinline__ void collision(const StepArgs& a, const double* m, double rho, double ux, double uy,
                                          double P, bool corr, double dxux, double dxuy, double dyux,
                                          double dyuy, double* coll)
{
    double eq[NQ];
    equilibria(rho, ux, uy, P, m[3], a.b, eq);
    double w[NQ];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = 0.0;
#pragma unroll
    for (int k = 4; k < NQ; ++k) w[k] = a.s[k] * (m[k] - eq[k]);
    if (corr) {
        // energy-flux correction of moments 8 and 9 (central differences of u)
        const double div4b = 4.0 * a.inv_b * (dxux + dyuy);
        const double shear2 = 2.0 * (dxuy + dyux);
        w[7] += a.k8 * P * (ux * (4.0 * dxux - div4b) + uy * shear2);
        w[8] += a.k9 * P * (ux * shear2 + uy * (4.0 * dyuy - div4b));
    }
#pragma unroll
    for (int k = 4; k < NQ; ++k) w[k] *= -a.dt;
    inverse_nc(*a.Bp, w, coll);
}

// Limited x and y flux differences of the 16 populations and the update,
// stored plane by plane (the centre value is re-read with its stencil, so
// only the 16 collision terms stay live across the loop).
template <int LIM, typename T>
__device__ __forceinline__ void convect_update(const T* __restrict__ fin, T* __restrict__ fout, const StepArgs& a,
                                               long n0, const double* coll)
{
    using R = T;   // convection precision (FP64, or FP32 in FP32-storage mode)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const long pi = i * a.plane + n0;
        const int g = i >> 2;
        const R f0 = fin[pi];
        R acc = R(0);
        if (sgx(i) != 0) {
            const long s = sgx(i);
            acc += conv1<LIM, R>(fin[pi - 2 * s], fin[pi - s], f0, fin[pi + s], (R)a.nux[g], (R)a.cx[g]);
        }
        if (sgy(i) != 0) {
            const long s = sgy(i) * a.pitch;
            acc += conv1<LIM, R>(fin[pi - 2 * s], fin[pi - s], f0, fin[pi + s], (R)a.nuy[g], (R)a.cy[g]);
        }
        fout[pi] = (T)((double)f0 + (double)acc + coll[i]);
        STEP_PLANE_FENCE();
    }
}

// Periodic and outflow ghost images owned by node (x, y): up to 4 along x
// and 4 along y (a single-node axis wraps onto all four ghosts).  Returns the
// count; offs[] are element offsets relative to the node.  Wall nodes and
// their ghosts are filled afterwards by k_fill (walls only).
__device__ __forceinline__ int image_offsets(const StepArgs& a, int x, int y, int* offs)
{
    int n = 0;
    if (a.bc[0] == BC_PERIODIC) {
        if (x < 2 || x >= a.nx - 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int xg = (q < 2) ? (q - 2) : (a.nx + q - 2);
                if ((((xg % a.nx) + a.nx) % a.nx) == x) offs[n++] = xg - x;
            }
        }
    } else {
        if (a.bc[0] == BC_OUTFLOW && x == 0) {
            offs[n++] = -1;
            offs[n++] = -2;
        }
        if (a.bc[1] == BC_OUTFLOW && x == a.nx - 1) {
            offs[n++] = 1;
            offs[n++] = 2;
        }
    }
    const int pitch = (int)a.pitch;
    if (a.bc[2] == BC_PERIODIC) {
        if (y < 2 || y >= a.ny - 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int yg = (q < 2) ? (q - 2) : (a.ny + q - 2);
                if ((((yg % a.ny) + a.ny) % a.ny) == y) offs[n++] = (yg - y) * pitch;
            }
        }
    } else {
        if (a.bc[2] == BC_OUTFLOW && y == 0) {
            offs[n++] = -pitch;
            offs[n++] = -2 * pitch;
        }
        if (a.bc[3] == BC_OUTFLOW && y == a.ny - 1) {
            offs[n++] = pitch;
            offs[n++] = 2 * pitch;
        }
    }
    return n;
}

// The fused step kernel.  A block owns a TXW x BYR tile of nodes, one node
// per thread.  It first copies the tile with a two-node halo, all 16 planes,
// into LDS with every load in flight at once (f is read from HBM once per
// step; the halo rows come from L2).  After one barrier everything is read
// from LDS: each node's moments and velocity, the velocity of the one-node
// ring around the tile, then (second barrier) the central differences of u,
// the equilibria and the collision term, and the limited x / y flux
// differences of each plane; the new value of each plane is stored as soon
// as it is known.  Two blocks per CU alternate between loading and
// computing.
//
// Blocks are assigned round-robin to the 8 XCDs (each with its own L2):
// block b takes tile t = (b mod 8) * per_xcd + b / 8 of an order that
// sweeps bands of `band` tile columns row by row, so that the tiles resident
// on one XCD are neighbours and share their halo rows in its L2.
template <int LIM, typename T, int TXW, int BYR>
__global__ void __launch_bounds__(TXW * BYR, 1) k_step(const T* __restrict__ fin, T* __restrict__ fout,
                                                      StepArgs a)
{
    constexpr int TW = TXW + 4, TH = BYR + 4, TN = TW * TH;   // staged tile (with halo)
    constexpr int NT = TXW * BYR;                              // threads = nodes
    constexpr int PER = (TN + NT - 1) / NT;                    // staged elements per thread per plane
    constexpr int UW = TXW + 2;                                // velocity tile width (one-node ring)
    __shared__ T tile[NQ * TN];
    __shared__ double sux[(BYR + 2) * UW], suy[(BYR + 2) * UW];

    const int tid = threadIdx.x;
    const int bid = blockIdx.x;
    const int t = (bid & 7) * a.per_xcd + (bid >> 3);
    if (t >= a.ntx * a.nty) return;
    const int band_tiles = a.band * a.nty;
    const int bnd = t / band_tiles, rr = t - bnd * band_tiles;
    const int bw = min(a.band, a.ntx - bnd * a.band);
    const int tyy = rr / bw, txx = bnd * a.band + (rr - tyy * bw);
    const int xb = a.x0 + txx * TXW, yb = a.y0 + tyy * BYR;
    const int ty = tid / TXW, tx = tid - ty * TXW;
    const int x = xb + tx, y = yb + ty;
    const bool active = (x < a.x1) && (y < a.y1);
    const int pitch = (int)a.pitch;
    const int n0 = (int)a.org + y * pitch + x;     // offset inside a plane
    const bool corr = a.correction != 0;

    // ---- copy the tile (all planes, two-node halo) into LDS
    {
        int soff[PER];
        bool sok[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = tid + k * NT;
            const int r = e / TW, c = e - r * TW;
            const int gx = xb - 2 + c, gy = yb - 2 + r;
            sok[k] = (e < TN) && gx >= -2 && gx <= a.nx + 1 && gy >= -2 && gy <= a.ny + 1;
            soff[k] = (int)a.org + gy * pitch + gx;
        }
        T v[NQ][PER];
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const T* pl = fin + (long)i * a.plane;
#pragma unroll
            for (int k = 0; k < PER; ++k) v[i][k] = sok[k] ? pl[soff[k]] : T(0);
        }
#pragma unroll
        for (int i = 0; i < NQ; ++i)
#pragma unroll
            for (int k = 0; k < PER; ++k)
                if (tid + k * NT < TN) tile[i * TN + tid + k * NT] = v[i][k];
    }
    __syncthreads();

    // ---- moments of the own node, velocity of the own node and of the ring
    const int c0 = (ty + 2) * TW + tx + 2;           // own position in a staged plane
    double m[NQ], rho = 1.0, ux = 0.0, uy = 0.0, P = 1.0;
    {
        double f[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) f[i] = (double)tile[i * TN + c0];
        Sums sm = all_sums(f);
        moments(*a.Bp, sm, m);
        rho = m[0];
        const double ir = 1.0 / rho;
        ux = m[1] * ir;
        uy = m[2] * ir;
        P = (m[3] - rho * (ux * ux + uy * uy)) * a.inv_b;
    }
    double dxux = 0.0, dxuy = 0.0, dyux = 0.0, dyuy = 0.0;
    if (corr) {
        sux[(ty + 1) * UW + tx + 1] = ux;
        suy[(ty + 1) * UW + tx + 1] = uy;
        if (tid < 2 * TXW + 2 * BYR) {
            int lx, ly;                                  // ring node in tile coordinates (-1 .. TXW, -1 .. BYR)
            if (tid < TXW) {
                lx = tid; ly = -1;
            } else if (tid < 2 * TXW) {
                lx = tid - TXW; ly = BYR;
            } else if (tid < 2 * TXW + BYR) {
                lx = -1; ly = tid - 2 * TXW;
            } else {
                lx = TXW; ly = tid - 2 * TXW - BYR;
            }
            double g[NQ], vx = 0.0, vy = 0.0;
            const int cr = (ly + 2) * TW + lx + 2;
#pragma unroll
            for (int i = 0; i < NQ; ++i) g[i] = (double)tile[i * TN + cr];
            const int rx = xb + lx, ry = yb + ly;
            if (rx >= a.x0 - 1 && rx <= a.x1 && ry >= a.y0 - 1 && ry <= a.y1) velocity_of(*a.Bp, g, vx, vy);
            sux[(ly + 1) * UW + lx + 1] = vx;
            suy[(ly + 1) * UW + lx + 1] = vy;
        }
        __syncthreads();
        const int cu = (ty + 1) * UW + tx + 1;
        dxux = (sux[cu + 1] - sux[cu - 1]) * a.inv2dx;
        dxuy = (suy[cu + 1] - suy[cu - 1]) * a.inv2dx;
        dyux = (sux[cu + UW] - sux[cu - UW]) * a.inv2dy;
        dyuy = (suy[cu + UW] - suy[cu - UW]) * a.inv2dy;
    }
    if (!active) return;
    if (!(rho > 0.0 && P > 0.0)) atomicOr(a.flag, 1);
    double coll[NQ];
    collision(a, m, rho, ux, uy, P, corr, dxux, dxuy, dyux, dyuy, coll);

    // ---- limited fluxes and the update, plane by plane
    using R = T;   // convection precision (FP64, or FP32 in FP32-storage mode)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const T* tb = tile + i * TN;
        const int g = i >> 2;
        const R f0 = tb[c0];
        R acc = R(0);
        if (sgx(i) != 0) {
            const int sx = sgx(i);
            acc += conv1<LIM, R>(tb[c0 - 2 * sx], tb[c0 - sx], f0, tb[c0 + sx], (R)a.nux[g], (R)a.cx[g]);
        }
        if (sgy(i) != 0) {
            const int sy = sgy(i) * TW;
            acc += conv1<LIM, R>(tb[c0 - 2 * sy], tb[c0 - sy], f0, tb[c0 + sy], (R)a.nuy[g], (R)a.cy[g]);
        }
        fout[(long)i * a.plane + n0] = (T)((double)f0 + (double)acc + coll[i]);
    }

    int offs[8];
    const int nimg = image_offsets(a, x, y, offs);
    if (nimg > 0) {
        // copy this thread's own new values (same thread, same addresses)
        for (int i = 0; i < NQ; ++i) {
            T* pl = fout + (long)i * a.plane;
            const T v = pl[n0];
            for (int q = 0; q < nimg; ++q) pl[n0 + offs[q]] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation, standalone boundary fill, outputs and checkpoint copies.
template <typename T>
__global__ void k_init(T* __restrict__ f, const double* __restrict__ rho, const double* __restrict__ ux,
                       const double* __restrict__ uy, const double* __restrict__ Tf, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const long d = (long)y * a.nx + x;
    double fe[NQ];
    feq_velocity(*a.Bp, a.b, rho[d], ux[d], uy[d], Tf[d], fe);
    const long n = node(a, x, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i * a.plane + n] = (T)fe[i];
}

// Ghost fill of one axis from the interior (x-sides over rows, then y-sides
// over columns, two launches); used after init and set_f.
template <typename T>
__global__ void k_fill(T* __restrict__ f, StepArgs a, int axis, int walls_only)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_line = (axis == 0) ? a.ny : a.nx;
    if (t >= 2 * n_line) return;
    const int side_lo = (t & 1) == 0;
    const int line = t >> 1;
    const int side = 2 * axis + (side_lo ? 0 : 1);
    const int n = (axis == 0) ? a.nx : a.ny;
    const long stride = (axis == 0) ? 1 : a.pitch;
    const long base = (axis == 0) ? node(a, 0, line) : node(a, line, 0);   // node at coordinate 0
    const int kind = a.bc[side];
    if (walls_only && kind != BC_WALL) return;
    double v[NQ];
    if (kind == BC_WALL) {
        const int c1 = side_lo ? 1 : n - 2, cw = side_lo ? 0 : n - 1;
        load16(f, a, base + c1 * stride, v);
        wall_fill(a, f, v, side, base + cw * stride, side_lo ? -stride : stride);
        return;
    }
    if (kind == BC_EQUIL) {
        const double* st = a.side[side];
        feq_velocity(*a.Bp, a.b, st[0], st[1], st[2], st[3], v);
    }
    for (int k = 1; k <= 2; ++k) {
        const int cg = side_lo ? -k : n - 1 + k;
        if (kind == BC_PERIODIC) load16(f, a, base + (long)(((cg % n) + n) % n) * stride, v);
        else if (kind == BC_OUTFLOW) load16(f, a, base + (long)(side_lo ? 0 : n - 1) * stride, v);
#pragma unroll
        for (int i = 0; i < NQ; ++i) f[i * a.plane + base + (long)cg * stride] = (T)v[i];
    }
}

template <typename T>
__global__ void k_macros(const T* __restrict__ f, double* rho, double* ux, double* uy, double* Tf, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    double v[NQ], r, vx, vy, t;
    load16(f, a, node(a, x, y), v);
    macro_of(*a.Bp, a.inv_b, v, r, vx, vy, t);
    const long d = (long)y * a.nx + x;
    if (rho) rho[d] = r;
    if (ux) ux[d] = vx;
    if (uy) uy[d] = vy;
    if (Tf) Tf[d] = t;
}

// Delta = M (f - f^eq) = fhat - fhat^eq; Delta* = M*(u) (f - f^eq) with
// f - f^eq = M^-1 Delta and M* the rows of M at v - u (Sec. V, Appendix).
template <typename T>
__global__ void k_noneq(const T* __restrict__ f, int star, double* __restrict__ out, StepArgs a, double eta0)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    double v[NQ], m[NQ], eq[NQ], dl[NQ];
    load16(f, a, node(a, x, y), v);
    Sums sm = all_sums(v);
    moments(*a.Bp, sm, m);
    const double rho = m[0], ir = 1.0 / rho, ux = m[1] * ir, uy = m[2] * ir;
    const double P = (m[3] - rho * (ux * ux + uy * uy)) * a.inv_b;
    equilibria(rho, ux, uy, P, m[3], a.b, eq);
#pragma unroll
    for (int k = 0; k < 4; ++k) dl[k] = 0.0;
#pragma unroll
    for (int k = 4; k < NQ; ++k) dl[k] = m[k] - eq[k];
    const long plane = (long)a.nx * a.ny, d = (long)y * a.nx + x;
    if (!star) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) out[k * plane + d] = dl[k];
        return;
    }
    double gq[NQ], ds[NQ];
    inverse_nc(*a.Bp, dl, gq);
#pragma unroll
    for (int k = 0; k < NQ; ++k) ds[k] = 0.0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int g = i >> 2;
        const double cx = sgx(i) * a.Bp->vmag[g] - ux, cy = sgy(i) * a.Bp->vmag[g] - uy;
        const double c2 = cx * cx + cy * cy, ce = c2 + ((g == 0) ? eta0 * eta0 : 0.0);
        const double dxy = cx * cx - cy * cy, q = gq[i];
        ds[0] += q;
        ds[1] += cx * q;
        ds[2] += cy * q;
        ds[3] += ce * q;
        ds[4] += c2 * q;
        ds[5] += dxy * q;
        ds[6] += cx * cy * q;
        ds[7] += cx * ce * q;
        ds[8] += cy * ce * q;
        ds[9] += cx * c2 * q;
        ds[10] += cy * c2 * q;
        ds[11] += cx * dxy * q;
        ds[12] += cy * dxy * q;
        ds[13] += c2 * ce * q;
        ds[14] += cx * cy * ce * q;
        ds[15] += dxy * ce * q;
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) out[k * plane + d] = ds[k];
}

template <typename T>
__global__ void k_gather(const T* __restrict__ f, double* __restrict__ out, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const long plane = (long)a.nx * a.ny, d = (long)y * a.nx + x, n = node(a, x, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) out[i * plane + d] = (double)f[i * a.plane + n];
}

template <typename T>
__global__ void k_scatter(T* __restrict__ f, const double* __restrict__ in, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const long plane = (long)a.nx * a.ny, d = (long)y * a.nx + x, n = node(a, x, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i * a.plane + n] = (T)in[i * plane + d];
}

// ---------------------------------------------------------------------------
// Host side.
thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(MRTFD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

struct Layout {
    size_t esize;
    long pitch, plane, org;
    size_t buf_bytes;
};

Layout layout_of(const mrtfd_params& p)
{
    Layout L;
    L.esize = (p.precision == MRTFD_FP32_STORAGE) ? 4 : 8;
    const long line = 128 / (long)L.esize;   // elements per 128-byte line
    const long xoff = line;                  // x = 0 starts a line; ghosts sit before it
    L.pitch = ((xoff + p.nx + HALO + line - 1) / line) * line;
    L.org = (long)HALO * L.pitch + xoff;
    L.plane = (long)(p.ny + 2 * HALO) * L.pitch;
    L.buf_bytes = (size_t)NQ * L.plane * L.esize;
    return L;
}

int validate(const mrtfd_params* p)
{
    if (!p) return fail(MRTFD_EINVAL, "params is NULL");
    if (p->nx < 1 || p->ny < 1) return fail(MRTFD_EINVAL, "grid %d x %d must be at least 1 x 1", p->nx, p->ny);
    if (!(p->dx > 0 && p->dy > 0 && p->dt > 0)) return fail(MRTFD_EINVAL, "dx, dy, dt must be > 0");
    if (!(p->b > 0)) return fail(MRTFD_EINVAL, "b must be > 0");
    if (p->limiter < 0 || p->limiter > 3) return fail(MRTFD_EINVAL, "unknown limiter %d", p->limiter);
    if (p->precision != MRTFD_FP64 && p->precision != MRTFD_FP32_STORAGE)
        return fail(MRTFD_EINVAL, "unknown precision %d", p->precision);
    for (int s = 0; s < 4; ++s)
        if (p->bc[s].kind < 0 || p->bc[s].kind > 3) return fail(MRTFD_EINVAL, "unknown boundary kind on side %d", s);
    for (int ax = 0; ax < 2; ++ax)
        if ((p->bc[2 * ax].kind == BC_PERIODIC) != (p->bc[2 * ax + 1].kind == BC_PERIODIC))
            return fail(MRTFD_EINVAL, "periodic boundaries must be paired on axis %d", ax);
    const int wx = (p->bc[0].kind == BC_WALL) + (p->bc[1].kind == BC_WALL);
    const int wy = (p->bc[2].kind == BC_WALL) + (p->bc[3].kind == BC_WALL);
    if (wx && wy) return fail(MRTFD_EINVAL, "walls on both axes are not supported");
    if (wx && p->nx < wx + 1) return fail(MRTFD_EINVAL, "nx = %d too small for %d wall(s)", p->nx, wx);
    if (wy && p->ny < wy + 1) return fail(MRTFD_EINVAL, "ny = %d too small for %d wall(s)", p->ny, wy);
    for (int s = 0; s < 4; ++s) {
        const int k = p->bc[s].kind;
        if ((k == BC_EQUIL && !(p->bc[s].rho > 0 && p->bc[s].T > 0)) || (k == BC_WALL && !(p->bc[s].T > 0)))
            return fail(MRTFD_EINVAL, "side %d state needs rho > 0 and T > 0", s);
    }
    // unsplit Courant bound: |v_x| dt/dx + |v_y| dt/dy <= 1 for every velocity
    const double r2 = std::sqrt(2.0), mag[4] = {1.0, 6.0, r2, 3.0 / r2};
    for (int g = 0; g < 4; ++g) {
        const double c = (g < 2) ? mag[g] * p->dt * std::fmax(1.0 / p->dx, 1.0 / p->dy)
                                 : mag[g] * p->dt * (1.0 / p->dx + 1.0 / p->dy);
        if (c > 1.0 + 1e-12) return fail(MRTFD_EINVAL, "Courant number %.4g > 1 on velocity group %d", c, g + 1);
    }
    double smax = 0.0;
    for (int k = 4; k < NQ; ++k) {
        if (!(p->s[k] >= 0)) return fail(MRTFD_EINVAL, "s_%d must be >= 0", k + 1);
        smax = std::fmax(smax, p->s[k]);
    }
    if (p->dt * smax >= 2.0) return fail(MRTFD_EINVAL, "dt * max(s) = %.4g must be < 2", p->dt * smax);
    if (p->energy_flux_correction && !(p->s[4] > 0)) return fail(MRTFD_EINVAL, "the correction needs s_5 > 0");
    if (!(p->eta0 >= 0)) return fail(MRTFD_EINVAL, "eta0 must be >= 0");
    const Layout L = layout_of(*p);
    if (L.plane >= (1L << 31))
        return fail(MRTFD_EINVAL, "grid %d x %d too large: a padded plane must stay below 2^31 elements", p->nx, p->ny);
    return MRTFD_OK;
}

}  // namespace

struct mrtfd_s {
    mrtfd_params p;
    hipStream_t stream;
    Layout L;
    void* buf[2];
    int cur;
    int* flag;
    double* staging;
    size_t staging_bytes;
    StepArgs args;
    Blocks blocks;          // host copy
    Blocks* blocks_dev;     // device copy read by the kernels
    bool ready;
    long steps;
    hipEvent_t ev0, ev1;
};

namespace {

void fill_args(mrtfd_s* h)
{
    const mrtfd_params& p = h->p;
    StepArgs& a = h->args;
    std::memset(&a, 0, sizeof(a));
    a.Bp = h->blocks_dev;
    for (int k = 0; k < NQ; ++k) a.s[k] = p.s[k];
    a.b = p.b;
    a.inv_b = 1.0 / p.b;
    a.dt = p.dt;
    for (int g = 0; g < 4; ++g) {
        a.nux[g] = h->blocks.vmag[g] * p.dt / p.dx;
        a.nuy[g] = h->blocks.vmag[g] * p.dt / p.dy;
        a.cx[g] = 0.5 * (1.0 - a.nux[g]);
        a.cy[g] = 0.5 * (1.0 - a.nuy[g]);
    }
    a.correction = p.energy_flux_correction ? 1 : 0;
    a.k8 = a.correction ? p.s[7] / p.s[4] - 1.0 : 0.0;
    a.k9 = a.correction ? p.s[8] / p.s[4] - 1.0 : 0.0;
    a.inv2dx = 0.5 / p.dx;
    a.inv2dy = 0.5 / p.dy;
    for (int s = 0; s < 4; ++s) {
        a.bc[s] = p.bc[s].kind;
        a.side[s][0] = p.bc[s].rho;
        a.side[s][1] = p.bc[s].ux;
        a.side[s][2] = p.bc[s].uy;
        a.side[s][3] = p.bc[s].T;
    }
    a.nx = p.nx;
    a.ny = p.ny;
    a.pitch = h->L.pitch;
    a.plane = h->L.plane;
    a.org = h->L.org;
    a.x0 = (p.bc[0].kind == BC_WALL);
    a.x1 = p.nx - (p.bc[1].kind == BC_WALL);
    a.y0 = (p.bc[2].kind == BC_WALL);
    a.y1 = p.ny - (p.bc[3].kind == BC_WALL);
    const int txw = (p.precision == MRTFD_FP32_STORAGE) ? STEP_TXW32 : STEP_TXW64;
    const int byr = (p.precision == MRTFD_FP32_STORAGE) ? STEP_BYR32 : STEP_BYR64;
    a.ntx = (a.x1 - a.x0 + txw - 1) / txw;
    a.nty = (a.y1 - a.y0 + byr - 1) / byr;
    a.per_xcd = (a.ntx * a.nty + 7) / 8;
    a.band = STEP_BAND;
    a.flag = h->flag;
}

dim3 node_grid(int nx, int ny) { return dim3((nx + BX - 1) / BX, (ny + BY - 1) / BY); }

int ensure_staging(mrtfd_s* h, size_t bytes)
{
    if (h->staging_bytes >= bytes) return MRTFD_OK;
    if (h->staging) {
        HIPCHK(hipStreamSynchronize(h->stream));
        HIPCHK(hipFree(h->staging));
        h->staging = nullptr;
        h->staging_bytes = 0;
    }
    if (hipMalloc(&h->staging, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MRTFD_ENOMEM, "cannot allocate %zu bytes of staging", bytes);
    }
    h->staging_bytes = bytes;
    return MRTFD_OK;
}

template <typename T>
int launch_step_t(mrtfd_s* h)
{
    StepArgs& a = h->args;
    const T* fin = (const T*)h->buf[h->cur];
    T* fout = (T*)h->buf[1 - h->cur];
    const int ex = a.x1 - a.x0, ey = a.y1 - a.y0;
    if (ex > 0 && ey > 0) {
        constexpr int TXW = TileOf<T>::TXW, BYR = TileOf<T>::BYR;
        dim3 grid(8 * a.per_xcd), block(TXW * BYR);
        switch (h->p.limiter) {
        case 0: hipLaunchKernelGGL((k_step<0, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
        case 1: hipLaunchKernelGGL((k_step<1, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
        case 2: hipLaunchKernelGGL((k_step<2, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
        default: hipLaunchKernelGGL((k_step<3, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
        }
        HIPCHK(hipGetLastError());
        for (int axis = 0; axis < 2; ++axis) {
            if (a.bc[2 * axis] != BC_WALL && a.bc[2 * axis + 1] != BC_WALL) continue;
            const int n = 2 * ((axis == 0) ? a.ny : a.nx);
            hipLaunchKernelGGL((k_fill<T>), dim3((n + 127) / 128), dim3(128), 0, h->stream, fout, a, axis, 1);
            HIPCHK(hipGetLastError());
        }
    }
    h->cur = 1 - h->cur;
    return MRTFD_OK;
}

int launch_step(mrtfd_s* h)
{
    return (h->p.precision == MRTFD_FP32_STORAGE) ? launch_step_t<float>(h) : launch_step_t<double>(h);
}

template <typename T>
int refill_t(mrtfd_s* h)
{
    T* f = (T*)h->buf[h->cur];
    for (int axis = 0; axis < 2; ++axis) {
        const int n = 2 * ((axis == 0) ? h->p.ny : h->p.nx);
        hipLaunchKernelGGL((k_fill<T>), dim3((n + 127) / 128), dim3(128), 0, h->stream, f, h->args, axis, 0);
        HIPCHK(hipGetLastError());
    }
    // both buffers carry the (constant) equilibrium ghosts
    HIPCHK(hipMemcpyAsync(h->buf[1 - h->cur], h->buf[h->cur], h->L.buf_bytes, hipMemcpyDeviceToDevice, h->stream));
    return MRTFD_OK;
}

int refill(mrtfd_s* h)
{
    return (h->p.precision == MRTFD_FP32_STORAGE) ? refill_t<float>(h) : refill_t<double>(h);
}

}  // namespace

// ===========================================================================
extern "C" {

const char* mrtfd_last_error(void) { return g_err.c_str(); }

int mrtfd_footprint(const mrtfd_params* p, size_t* bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes) return fail(MRTFD_EINVAL, "bytes is NULL");
    Layout L = layout_of(*p);
    *bytes = 2 * L.buf_bytes + 256;
    return MRTFD_OK;
}

int mrtfd_create(const mrtfd_params* p, void* hip_stream, mrtfd_t* out)
{
    if (!out) return fail(MRTFD_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    mrtfd_s* h = new (std::nothrow) mrtfd_s();
    if (!h) return fail(MRTFD_ENOMEM, "host allocation failed");
    h->p = *p;
    h->stream = (hipStream_t)hip_stream;
    h->L = layout_of(*p);
    for (int k = 0; k < 2; ++k) {
        if (hipMalloc(&h->buf[k], h->L.buf_bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (k == 1) (void)hipFree(h->buf[0]);
            delete h;
            return fail(MRTFD_ENOMEM, "cannot allocate 2 x %zu bytes of state", h->L.buf_bytes);
        }
    }
    if (!build_blocks(p->eta0, &h->blocks)) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
        delete h;
        return fail(MRTFD_EINVAL, "singular moment blocks for eta0 = %g", p->eta0);
    }
    if (hipMalloc(&h->flag, sizeof(int)) != hipSuccess || hipMalloc(&h->blocks_dev, sizeof(Blocks)) != hipSuccess ||
        hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
        delete h;
        return fail(MRTFD_EDEVICE, "device set-up failed");
    }
    fill_args(h);
    if (hipMemcpyAsync(h->blocks_dev, &h->blocks, sizeof(Blocks), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
        mrtfd_destroy(h);
        return fail(MRTFD_EDEVICE, "device set-up failed");
    }
    if (hipMemsetAsync(h->flag, 0, sizeof(int), h->stream) != hipSuccess ||
        hipMemsetAsync(h->buf[0], 0, h->L.buf_bytes, h->stream) != hipSuccess ||
        hipMemsetAsync(h->buf[1], 0, h->L.buf_bytes, h->stream) != hipSuccess) {
        mrtfd_destroy(h);
        return fail(MRTFD_EDEVICE, "device set-up failed");
    }
    *out = h;
    return MRTFD_OK;
}

int mrtfd_destroy(mrtfd_t h)
{
    if (!h) return MRTFD_OK;
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->buf[0]);
    (void)hipFree(h->buf[1]);
    (void)hipFree(h->flag);
    (void)hipFree(h->blocks_dev);
    if (h->staging) (void)hipFree(h->staging);
    (void)hipEventDestroy(h->ev0);
    (void)hipEventDestroy(h->ev1);
    delete h;
    return MRTFD_OK;
}

int mrtfd_init(mrtfd_t h, const double* rho, const double* ux, const double* uy, const double* T, int on_device)
{
    if (!h || !rho || !ux || !uy || !T) return fail(MRTFD_EINVAL, "NULL argument");
    const size_t n = (size_t)h->p.nx * h->p.ny;
    const double* src[4] = {rho, ux, uy, T};
    if (!on_device) {
        int rc = ensure_staging(h, 4 * n * sizeof(double));
        if (rc) return rc;
        for (int q = 0; q < 4; ++q) {
            HIPCHK(hipMemcpyAsync(h->staging + q * n, src[q], n * sizeof(double), hipMemcpyHostToDevice, h->stream));
            src[q] = h->staging + q * n;
        }
    }
    h->cur = 0;
    dim3 grid = node_grid(h->p.nx, h->p.ny), block(BX, BY);
    if (h->p.precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_init<float>), grid, block, 0, h->stream, (float*)h->buf[0], src[0], src[1], src[2], src[3], h->args);
    else
        hipLaunchKernelGGL((k_init<double>), grid, block, 0, h->stream, (double*)h->buf[0], src[0], src[1], src[2], src[3], h->args);
    HIPCHK(hipGetLastError());
    int rc = refill(h);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(h->stream));
    h->ready = true;
    h->steps = 0;
    return MRTFD_OK;
}

int mrtfd_step(mrtfd_t h, long nsteps)
{
    if (!h) return fail(MRTFD_EINVAL, "NULL handle");
    if (!h->ready) return fail(MRTFD_ESTATE, "mrtfd_step before mrtfd_init / mrtfd_set_f");
    if (nsteps < 0) return fail(MRTFD_EINVAL, "nsteps < 0");
    for (long k = 0; k < nsteps; ++k) {
        int rc = launch_step(h);
        if (rc) return rc;
    }
    h->steps += nsteps;
    return MRTFD_OK;
}

int mrtfd_step_timed(mrtfd_t h, long nsteps, double* elapsed_ms)
{
    if (!h || !elapsed_ms) return fail(MRTFD_EINVAL, "NULL argument");
    HIPCHK(hipEventRecord(h->ev0, h->stream));
    int rc = mrtfd_step(h, nsteps);
    if (rc) return rc;
    HIPCHK(hipEventRecord(h->ev1, h->stream));
    HIPCHK(hipEventSynchronize(h->ev1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    *elapsed_ms = ms;
    return MRTFD_OK;
}

int mrtfd_macros(mrtfd_t h, double* rho, double* ux, double* uy, double* T, int on_device)
{
    if (!h) return fail(MRTFD_EINVAL, "NULL handle");
    if (!h->ready) return fail(MRTFD_ESTATE, "mrtfd_macros before mrtfd_init / mrtfd_set_f");
    const size_t n = (size_t)h->p.nx * h->p.ny;
    double* dst[4] = {rho, ux, uy, T};
    if (!on_device) {
        int rc = ensure_staging(h, 4 * n * sizeof(double));
        if (rc) return rc;
        for (int q = 0; q < 4; ++q) dst[q] = dst[q] ? h->staging + q * n : nullptr;
    }
    dim3 grid = node_grid(h->p.nx, h->p.ny), block(BX, BY);
    if (h->p.precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_macros<float>), grid, block, 0, h->stream, (const float*)h->buf[h->cur], dst[0], dst[1], dst[2], dst[3], h->args);
    else
        hipLaunchKernelGGL((k_macros<double>), grid, block, 0, h->stream, (const double*)h->buf[h->cur], dst[0], dst[1], dst[2], dst[3], h->args);
    HIPCHK(hipGetLastError());
    if (!on_device) {
        double* host[4] = {rho, ux, uy, T};
        for (int q = 0; q < 4; ++q)
            if (host[q]) HIPCHK(hipMemcpyAsync(host[q], h->staging + q * n, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return MRTFD_OK;
}

int mrtfd_noneq(mrtfd_t h, int star, double* delta, int on_device)
{
    if (!h || !delta) return fail(MRTFD_EINVAL, "NULL argument");
    if (!h->ready) return fail(MRTFD_ESTATE, "mrtfd_noneq before mrtfd_init / mrtfd_set_f");
    const size_t n = (size_t)h->p.nx * h->p.ny;
    double* dst = delta;
    if (!on_device) {
        int rc = ensure_staging(h, NQ * n * sizeof(double));
        if (rc) return rc;
        dst = h->staging;
    }
    dim3 grid = node_grid(h->p.nx, h->p.ny), block(BX, BY);
    if (h->p.precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_noneq<float>), grid, block, 0, h->stream, (const float*)h->buf[h->cur], star, dst, h->args, h->p.eta0);
    else
        hipLaunchKernelGGL((k_noneq<double>), grid, block, 0, h->stream, (const double*)h->buf[h->cur], star, dst, h->args, h->p.eta0);
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(delta, h->staging, NQ * n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return MRTFD_OK;
}

int mrtfd_get_f(mrtfd_t h, double* f, int on_device)
{
    if (!h || !f) return fail(MRTFD_EINVAL, "NULL argument");
    if (!h->ready) return fail(MRTFD_ESTATE, "mrtfd_get_f before mrtfd_init / mrtfd_set_f");
    const size_t n = (size_t)h->p.nx * h->p.ny;
    double* dst = f;
    if (!on_device) {
        int rc = ensure_staging(h, NQ * n * sizeof(double));
        if (rc) return rc;
        dst = h->staging;
    }
    dim3 grid = node_grid(h->p.nx, h->p.ny), block(BX, BY);
    if (h->p.precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_gather<float>), grid, block, 0, h->stream, (const float*)h->buf[h->cur], dst, h->args);
    else
        hipLaunchKernelGGL((k_gather<double>), grid, block, 0, h->stream, (const double*)h->buf[h->cur], dst, h->args);
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(f, h->staging, NQ * n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return MRTFD_OK;
}

int mrtfd_set_f(mrtfd_t h, const double* f, int on_device)
{
    if (!h || !f) return fail(MRTFD_EINVAL, "NULL argument");
    const size_t n = (size_t)h->p.nx * h->p.ny;
    const double* src = f;
    if (!on_device) {
        int rc = ensure_staging(h, NQ * n * sizeof(double));
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(h->staging, f, NQ * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
        src = h->staging;
    }
    h->cur = 0;
    dim3 grid = node_grid(h->p.nx, h->p.ny), block(BX, BY);
    if (h->p.precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_scatter<float>), grid, block, 0, h->stream, (float*)h->buf[0], src, h->args);
    else
        hipLaunchKernelGGL((k_scatter<double>), grid, block, 0, h->stream, (double*)h->buf[0], src, h->args);
    HIPCHK(hipGetLastError());
    int rc = refill(h);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(h->flag, 0, sizeof(int), h->stream));
    if (!on_device) HIPCHK(hipStreamSynchronize(h->stream));
    h->ready = true;
    h->steps = 0;
    return MRTFD_OK;
}

int mrtfd_sync(mrtfd_t h)
{
    if (!h) return fail(MRTFD_EINVAL, "NULL handle");
    HIPCHK(hipStreamSynchronize(h->stream));
    int flag = 0;
    HIPCHK(hipMemcpy(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
        HIPCHK(hipMemset(h->flag, 0, sizeof(int)));
        return fail(MRTFD_ENONFINITE, "a node reached rho <= 0, T <= 0 or NaN");
    }
    return MRTFD_OK;
}

long mrtfd_steps_done(mrtfd_t h) { return h ? h->steps : -1; }

int mrtfd_constants(double eta0, double* M, double* Minv)
{
    Blocks B;
    if (!build_blocks(eta0, &B)) return fail(MRTFD_EINVAL, "singular blocks for eta0 = %g", eta0);
    for (int i = 0; i < NQ; ++i) {
        double e[NQ] = {0}, m[NQ], col[NQ];
        e[i] = 1.0;
        Sums s = all_sums(e);
        moments(B, s, m);
        inverse_full(B, e, col);
        for (int k = 0; k < NQ; ++k) {
            if (M) M[k * NQ + i] = m[k];
            if (Minv) Minv[k * NQ + i] = col[k];
        }
    }
    return MRTFD_OK;
}

}  // extern "C"
