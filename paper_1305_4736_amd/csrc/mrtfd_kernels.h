// mrtfd_kernels.h -- gfx950 kernels of the D2V16 MRT finite-difference LB
// step (arXiv:1305.4736), shared by the single-instance and batched entry
// points.
//
// State layout in HBM: 16 planes (structure of arrays, one per velocity),
// each (ny + 4) rows of `pitch` elements; node (x, y) of plane i sits at
// i * plane + org + y * pitch + x, with two ghost layers on every side and
// the first interior node of a row on a 128-byte line.  Two such buffers
// ping-pong between steps.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "../../include/mrtfd.h"
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
#ifndef STEP_BAND
#define STEP_BAND (1 << 20)   // tile columns per band of the XCD-aware tile order (default: whole rows)
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

// Offset (in doubles) of node (x, y) in conserved plane 0 (FP32 storage).
__device__ __forceinline__ long cnode(const StepArgs& a, int x, int y)
{
    return a.corg + (long)y * a.cpitch + x;
}

// Conserved moments (rho, j_x, j_y, e) of node (x, y): the stored FP64
// planes in FP32 storage, the sums of the populations in FP64 storage.
template <typename T>
__device__ __forceinline__ void cons_node(const T* __restrict__ f, const StepArgs& a, int x, int y, double* c)
{
    if constexpr (keeps_cons<T>()) {
        const double* cp = (const double*)f + cnode(a, x, y);
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = cp[k * a.cplane];
    } else {
        double v[NQ];
        load16(f, a, node(a, x, y), v);
        cons_of(*a.Bp, all_sums(v), c);
    }
}

// The FP64 populations node (x, y) stands for (FP32 storage: the rounded
// populations put back onto their conserved moments).
template <typename T>
__device__ __forceinline__ void load_node(const T* __restrict__ f, const StepArgs& a, int x, int y, double* out)
{
    if constexpr (keeps_cons<T>()) {
        double ft[NQ], c[4];
        load16(f, a, node(a, x, y), ft);
        cons_node(f, a, x, y, c);
        resync(*a.Bp, ft, c, out);
    } else {
        load16(f, a, node(a, x, y), out);
    }
}

// Store FP64 populations v at node (x, y): rounded to T, and in FP32
// storage their conserved moments beside them.
template <typename T>
__device__ __forceinline__ void store_node(T* __restrict__ f, const StepArgs& a, int x, int y, const double* v)
{
    const long n = node(a, x, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i * a.plane + n] = (T)v[i];
    if constexpr (keeps_cons<T>()) {
        double c[4];
        cons_of(*a.Bp, all_sums(v), c);
        double* cp = (double*)f + cnode(a, x, y);
#pragma unroll
        for (int k = 0; k < 4; ++k) cp[k * a.cplane] = c[k];
    }
}

// Copy node (xs, ys) to (xd, yd) bit for bit (populations and, in FP32
// storage, conserved moments).
template <typename T>
__device__ __forceinline__ void copy_node(T* __restrict__ f, const StepArgs& a, int xs, int ys, int xd, int yd)
{
    const long ns = node(a, xs, ys), nd = node(a, xd, yd);
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i * a.plane + nd] = f[i * a.plane + ns];
    if constexpr (keeps_cons<T>()) {
        double* cp = (double*)f;
        const long cs = cnode(a, xs, ys), cd = cnode(a, xd, yd);
#pragma unroll
        for (int k = 0; k < 4; ++k) cp[k * a.cplane + cd] = cp[k * a.cplane + cs];
    }
}


// Non-equilibrium extrapolation wall from the fluid node next to it (f1):
// fw[i] is the wall node's population i; its ghosts k = 1, 2 beyond the
// wall hold (k + 1) fw - k f1.
template <class AT, class BT>
__device__ __forceinline__ void wall_values(const AT& a, const BT& B, const double* f1, int side, double* fw)
{
    double r1, u1x, u1y, T1;
    macro_of(B, a.inv_b, f1, r1, u1x, u1y, T1);
    const double st3 = a.side[side][3];
    double rw = r1 * T1 / st3;             // carry the pressure over: rho_w T_w = rho_1 T_1
    double ew[NQ], e1[NQ];
    feq_velocity(B, a.b, rw, a.side[side][1], a.side[side][2], st3, ew);
    feq_velocity(B, a.b, r1, u1x, u1y, T1, e1);
#pragma unroll
    for (int i = 0; i < NQ; ++i) fw[i] = ew[i] + (f1[i] - e1[i]);
}

// Ghost k (1 or 2) beyond a wall: the line through f_1 and the wall node
// continued, (k + 1) f_w - k f_1 (one expression per k, shared by every
// kernel so that all of them round it alike).
__device__ __forceinline__ double wall_ghost(double fw, double f1, int k)
{
    return (k == 1) ? 2.0 * fw - f1 : 3.0 * fw - 2.0 * f1;
}

// The wall node (xw, yw) and its two ghosts one and two nodes further out
// along (sx, sy), from the populations f1 of the fluid node next to it.
template <typename T>
__device__ void wall_fill(const StepArgs& a, T* __restrict__ f, const double* f1, int side, int xw, int yw, int sx,
                          int sy)
{
    double fw[NQ], g[NQ];
    wall_values(a, *a.Bp, f1, side, fw);
    store_node(f, a, xw, yw, fw);
#pragma unroll
    for (int k = 1; k <= 2; ++k) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) g[i] = wall_ghost(fw[i], f1[i], k);
        store_node(f, a, xw + k * sx, yw + k * sy, g);
    }
}

// ---------------------------------------------------------------------------
// The fused step, per node.

// Relaxed residual of the non-conserved moments, mapped back to velocity
// space and scaled by -dt (the collision term of the update).
//
// CONS (FP32 storage): dc holds the node's stored conserved moments minus
// those of its rounded populations; they enter the increment unscaled, so
// that the new populations carry the stored conserved moments (the rounded
// ones are put back onto them before the update).
template <bool CONS, class AT, class BT>
__device__ __forceinline__ void collision(const AT& a, const BT& B, const double* m, double rho, double ux, double uy,
                                          double P, bool corr, double dxux, double dxuy, double dyux,
                                          double dyuy, const double* dc, double* coll)
{
    double eq[NQ];
    equilibria(rho, ux, uy, P, m[3], a.b, eq);
    double w[NQ];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = CONS ? dc[k] : 0.0;
#pragma unroll
    for (int k = 4; k < NQ; ++k) w[k] = a.rdt[k] * (m[k] - eq[k]);
    if (corr) {
        // energy-flux correction of moments 8 and 9 (central differences of u)
        const double div4b = 4.0 * a.inv_b * (dxux + dyuy);
        const double shear2 = 2.0 * (dxuy + dyux);
        w[7] += a.c8dt * P * (ux * (4.0 * dxux - div4b) + uy * shear2);
        w[8] += a.c9dt * P * (ux * shear2 + uy * (4.0 * dyuy - div4b));
    }
    if constexpr (CONS) inverse_full(B, w, coll);
    else inverse_nc(B, w, coll);
}

// Moments of a node from its stored populations ft: all 16 from the
// populations, then in FP32 storage the conserved ones replaced by the
// stored c, with dc = c - (those of ft).
template <typename T, class BT>
__device__ __forceinline__ void node_moments(const BT& B, const double* ft, const double* c, double* m, double* dc)
{
    moments(B, all_sums(ft), m);
    if constexpr (keeps_cons<T>()) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            dc[k] = c[k] - m[k];
            m[k] = c[k];
        }
    }
}

// Periodic and outflow ghost images owned by node (x, y): up to 4 along x
// and 4 along y (a single-node axis wraps onto all four ghosts).  Returns the
// count; (ox[q], oy[q]) are the images' offsets from the node.  Wall nodes
// and their ghosts are filled afterwards by k_fill (walls only).
template <class AT>
__device__ __forceinline__ int image_offsets(const AT& a, int x, int y, int* ox, int* oy)
{
    int n = 0;
    if (a.bc[0] == BC_PERIODIC) {
        if (x < 2 || x >= a.nx - 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int xg = (q < 2) ? (q - 2) : (a.nx + q - 2);
                if ((((xg % a.nx) + a.nx) % a.nx) == x) {
                    ox[n] = xg - x;
                    oy[n++] = 0;
                }
            }
        }
    } else {
        if (a.bc[0] == BC_OUTFLOW && x == 0) {
            ox[n] = -1; oy[n++] = 0;
            ox[n] = -2; oy[n++] = 0;
        }
        if (a.bc[1] == BC_OUTFLOW && x == a.nx - 1) {
            ox[n] = 1; oy[n++] = 0;
            ox[n] = 2; oy[n++] = 0;
        }
    }
    if (a.bc[2] == BC_PERIODIC) {
        if (y < 2 || y >= a.ny - 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int yg = (q < 2) ? (q - 2) : (a.ny + q - 2);
                if ((((yg % a.ny) + a.ny) % a.ny) == y) {
                    ox[n] = 0;
                    oy[n++] = yg - y;
                }
            }
        }
    } else {
        if (a.bc[2] == BC_OUTFLOW && y == 0) {
            ox[n] = 0; oy[n++] = -1;
            ox[n] = 0; oy[n++] = -2;
        }
        if (a.bc[3] == BC_OUTFLOW && y == a.ny - 1) {
            ox[n] = 0; oy[n++] = 1;
            ox[n] = 0; oy[n++] = 2;
        }
    }
    return n;
}

// The fused step.  A block owns a TXW x BYR tile of nodes, one node per
// thread.  It first copies the tile with a two-node halo, all 16 planes,
// into LDS with every load in flight at once (f is read from HBM once per
// step; the halo rows come from L2).  After one barrier everything is read
// from LDS: each node's moments and velocity, the velocity of the one-node
// ring around the tile, then (second barrier) the central differences of u,
// the equilibria and the collision term, and the limited x / y flux
// differences of each plane; the new value of each plane is stored as soon
// as it is known.  Two blocks per CU alternate between loading and
// computing.  Tiles are numbered in bands of `band` tile columns swept row by
// row.
// LDS of one tile.  FLAT tiles are single rows of an instance with one row
// whose y ghosts are copies of that row (periodic or outflow in y): every y
// difference is then exactly zero, so no y halo is staged.
template <typename T, int TXW, int BYR, bool FLAT = false>
struct TileSmem {
    static constexpr int HY = FLAT ? 0 : 2;                           // y halo
    static constexpr int TW = TXW + 4, TH = BYR + 2 * HY, TN = TW * TH;
    static constexpr int UW = TXW + 2;                                // velocity tile width (one-node ring)
    T tile[NQ * TN];
    double sux[(BYR + 2) * UW], suy[(BYR + 2) * UW];
};

// One tile t (in the band order of a.ntx x a.nty tiles) of one instance.
// All threads of the block call it with the same arguments.
template <int LIM, typename T, int TXW, int BYR, bool FLAT = false>
__device__ __forceinline__ void step_tile(const T* __restrict__ fin, T* __restrict__ fout, const StepArgs& a, int t,
                                          TileSmem<T, TXW, BYR, FLAT>& sm_)
{
    static_assert(!FLAT || BYR == 1, "flat tiles are one row");
    constexpr int HY = FLAT ? 0 : 2;
    constexpr int TW = TXW + 4, TH = BYR + 2 * HY, TN = TW * TH;   // staged tile (with halo)
    constexpr int NT = TXW * BYR;                                  // threads = nodes
    constexpr int PER = (TN + NT - 1) / NT;                        // staged elements per thread per plane
    constexpr int UW = TXW + 2;                                    // velocity tile width (one-node ring)
    T* tile = sm_.tile;
    double* sux = sm_.sux;
    double* suy = sm_.suy;

    const int tid = threadIdx.x;
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
            const int gx = xb - 2 + c, gy = yb - HY + r;
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
    const int c0 = (ty + HY) * TW + tx + 2;          // own position in a staged plane
    double m[NQ], dc[4], rho = 1.0, ux = 0.0, uy = 0.0, P = 1.0;
    {
        double f[NQ], c[4] = {1.0, 0.0, 0.0, 1.0};
#pragma unroll
        for (int i = 0; i < NQ; ++i) f[i] = (double)tile[i * TN + c0];
        // (FP32 storage: the stored conserved moments, on the grid and its
        // ghosts; threads beyond them keep a placeholder nobody reads)
        if (keeps_cons<T>() && x >= -2 && x <= a.nx + 1 && y >= -2 && y <= a.ny + 1) cons_node(fin, a, x, y, c);
        node_moments<T>(*a.Bp, f, c, m, dc);
        rho = m[0];
        velocity_of_cons(rho, m[1], m[2], ux, uy);
        P = (m[3] - rho * (ux * ux + uy * uy)) * a.inv_b;
    }
    double dxux = 0.0, dxuy = 0.0, dyux = 0.0, dyuy = 0.0;
    if (corr) {
        sux[(ty + 1) * UW + tx + 1] = ux;
        suy[(ty + 1) * UW + tx + 1] = uy;
        // ring nodes: rows above / below (none for flat tiles), columns left /
        // right; a wide tile has more ring nodes than threads
        constexpr int RY = FLAT ? 0 : TXW;
        for (int q = tid; q < 2 * RY + 2 * BYR; q += NT) {
            int lx, ly;                                  // ring node in tile coordinates (-1 .. TXW, -1 .. BYR)
            if (q < RY) {
                lx = q; ly = -1;
            } else if (q < 2 * RY) {
                lx = q - RY; ly = BYR;
            } else if (q < 2 * RY + BYR) {
                lx = -1; ly = q - 2 * RY;
            } else {
                lx = TXW; ly = q - 2 * RY - BYR;
            }
            double vx = 0.0, vy = 0.0;
            const int cr = (ly + HY) * TW + lx + 2;
            const int rx = xb + lx, ry = yb + ly;
            if (rx >= a.x0 - 1 && rx <= a.x1 && ry >= a.y0 - 1 && ry <= a.y1) {
                if constexpr (keeps_cons<T>()) {
                    double c[4];
                    cons_node(fin, a, rx, ry, c);
                    velocity_of_cons(c[0], c[1], c[2], vx, vy);
                } else {
                    double g[NQ];
#pragma unroll
                    for (int i = 0; i < NQ; ++i) g[i] = (double)tile[i * TN + cr];
                    velocity_of(*a.Bp, g, vx, vy);
                }
            }
            sux[(ly + 1) * UW + lx + 1] = vx;
            suy[(ly + 1) * UW + lx + 1] = vy;
        }
        __syncthreads();
        const int cu = (ty + 1) * UW + tx + 1;
        dxux = (sux[cu + 1] - sux[cu - 1]) * a.inv2dx;
        dxuy = (suy[cu + 1] - suy[cu - 1]) * a.inv2dx;
        if (!FLAT) {
            dyux = (sux[cu + UW] - sux[cu - UW]) * a.inv2dy;
            dyuy = (suy[cu + UW] - suy[cu - UW]) * a.inv2dy;
        }
    }
    if (!active) return;
    if (!(rho > 0.0 && P > 0.0)) atomicOr(a.flag, 1);
    double coll[NQ];
    collision<keeps_cons<T>()>(a, *a.Bp, m, rho, ux, uy, P, corr, dxux, dxuy, dyux, dyuy, dc, coll);

    // ---- limited fluxes and the update, plane by plane
    using R = conv_t<T>;   // convection precision
    double vd[NQ];         // new populations in FP64 (FP32 storage keeps their conserved moments)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const T* tb = tile + i * TN;
        const int g = i >> 2;
        const R f0 = tb[c0];
        R acc = acc_start<T, R>(coll[i]);
        if (sgx(i) != 0) {
            const int sx = sgx(i);
            acc = conv1<LIM, R>(acc, tb[c0 - 2 * sx], tb[c0 - sx], f0, tb[c0 + sx], nu_of<R, 0>(a, g), c_of<R, 0, LIM>(a, g));
        }
        if (!FLAT && sgy(i) != 0) {
            const int sy = sgy(i) * TW;
            acc = conv1<LIM, R>(acc, tb[c0 - 2 * sy], tb[c0 - sy], f0, tb[c0 + sy], nu_of<R, 1>(a, g), c_of<R, 1, LIM>(a, g));
        }
        vd[i] = new_value<T, R>(f0, acc, coll[i]);
        fout[(long)i * a.plane + n0] = (T)vd[i];
    }
    if constexpr (keeps_cons<T>()) {
        double c[4];
        cons_of(*a.Bp, all_sums(vd), c);
        double* cp = (double*)fout + cnode(a, x, y);
#pragma unroll
        for (int k = 0; k < 4; ++k) cp[k * a.cplane] = c[k];
    }

    int ox[8], oy[8];
    const int nimg = image_offsets(a, x, y, ox, oy);
    // copy this thread's own new values (same thread, same addresses)
    for (int q = 0; q < nimg; ++q) copy_node(fout, a, x, y, x + ox[q], y + oy[q]);
}

// Single instance: one block per tile.  Blocks are assigned round-robin to
// the 8 XCDs (each with its own L2); block b takes tile
// t = (b mod 8) * per_xcd + b / 8, so each XCD sweeps its own contiguous
// range of the tile order.
template <int LIM, typename T, int TXW, int BYR>
__global__ void __launch_bounds__(TXW * BYR, 1) k_step(const T* __restrict__ fin, T* __restrict__ fout,
                                                      StepArgs a)
{
    __shared__ TileSmem<T, TXW, BYR> sm_;
    convect_mode();
    const int bid = blockIdx.x;
    const int t = (bid & 7) * a.per_xcd + (bid >> 3);
    if (t >= a.ntx * a.nty) return;
    step_tile<LIM, T, TXW, BYR>(fin, fout, a, t, sm_);
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
    store_node(f, a, x, y, fe);
}

// Ghost fill of one side line: thread index t covers line t / 2 of axis
// `axis` (rows for x, columns for y), low side for even t.  With walls_only
// only wall sides are refilled (after a step; the other kinds are written by
// the step itself).
template <typename T>
__device__ void fill_line(T* __restrict__ f, const StepArgs& a, int axis, int t, int walls_only)
{
    const int side_lo = (t & 1) == 0;
    const int line = t >> 1;
    const int side = 2 * axis + (side_lo ? 0 : 1);
    const int n = (axis == 0) ? a.nx : a.ny;
    const int kind = a.bc[side];
    if (walls_only && kind != BC_WALL) return;
    // coordinate c along the axis -> node of this line
    auto px = [&](int c) { return (axis == 0) ? c : line; };
    auto py = [&](int c) { return (axis == 0) ? line : c; };
    const int out = side_lo ? -1 : 1;
    if (kind == BC_WALL) {
        const int c1 = side_lo ? 1 : n - 2, cw = side_lo ? 0 : n - 1;
        double v[NQ];
        load_node(f, a, px(c1), py(c1), v);
        wall_fill(a, f, v, side, px(cw), py(cw), (axis == 0) ? out : 0, (axis == 0) ? 0 : out);
        return;
    }
    double v[NQ];
    if (kind == BC_EQUIL) {
        const double* st = a.side[side];
        feq_velocity(*a.Bp, a.b, st[0], st[1], st[2], st[3], v);
    }
    for (int k = 1; k <= 2; ++k) {
        const int cg = side_lo ? -k : n - 1 + k;
        if (kind == BC_EQUIL) {
            store_node(f, a, px(cg), py(cg), v);
        } else {
            const int cs = (kind == BC_PERIODIC) ? ((cg % n) + n) % n : (side_lo ? 0 : n - 1);
            copy_node(f, a, px(cs), py(cs), px(cg), py(cg));
        }
    }
}

// Ghost fill of one axis (x-sides over rows, then y-sides over columns: two
// launches); used after init and set_f, and after each step for the walls
// the step kernel leaves (walls along x, and the LDS-tile form's).
template <typename T>
__global__ void k_fill(T* __restrict__ f, StepArgs a, int axis, int walls_only)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int n_line = (axis == 0) ? a.ny : a.nx;
    if (t >= 2 * n_line) return;
    fill_line(f, a, axis, t, walls_only);
}

template <typename T>
__global__ void k_macros(const T* __restrict__ f, double* rho, double* ux, double* uy, double* Tf, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    double r, vx, vy, t;
    if constexpr (keeps_cons<T>()) {
        double c[4];
        cons_node(f, a, x, y, c);
        macro_of_cons(a.inv_b, c, r, vx, vy, t);
    } else {
        double v[NQ];
        load16(f, a, node(a, x, y), v);
        macro_of(*a.Bp, a.inv_b, v, r, vx, vy, t);
    }
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
    double v[NQ], m[NQ], eq[NQ], dl[NQ], c[4], dc[4];
    load16(f, a, node(a, x, y), v);
    if constexpr (keeps_cons<T>()) cons_node(f, a, x, y, c);
    node_moments<T>(*a.Bp, v, c, m, dc);
    const double rho = m[0], ir = recip(rho), ux = m[1] * ir, uy = m[2] * ir;
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
    const long plane = (long)a.nx * a.ny, d = (long)y * a.nx + x;
    double v[NQ];
    load_node(f, a, x, y, v);
#pragma unroll
    for (int i = 0; i < NQ; ++i) out[i * plane + d] = v[i];
}

template <typename T>
__global__ void k_scatter(T* __restrict__ f, const double* __restrict__ in, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const long plane = (long)a.nx * a.ny, d = (long)y * a.nx + x;
    double v[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) v[i] = in[i * plane + d];
    store_node(f, a, x, y, v);
}


// The stored state of every grid node as doubles, exactly: the 16 stored
// populations, then (FP32 storage) the 4 conserved moments; (nplanes, ny, nx).
template <typename T>
__device__ __forceinline__ int state_planes() { return keeps_cons<T>() ? NQ + 4 : NQ; }

template <typename T>
__global__ void k_gather_state(const T* __restrict__ f, double* __restrict__ out, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const long plane = (long)a.nx * a.ny, d = (long)y * a.nx + x, n = node(a, x, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) out[i * plane + d] = (double)f[i * a.plane + n];
    if constexpr (keeps_cons<T>()) {
        const double* cp = (const double*)f + cnode(a, x, y);
#pragma unroll
        for (int k = 0; k < 4; ++k) out[(NQ + k) * plane + d] = cp[k * a.cplane];
    }
}

template <typename T>
__global__ void k_scatter_state(T* __restrict__ f, const double* __restrict__ in, StepArgs a)
{
    const int x = blockIdx.x * BX + threadIdx.x, y = blockIdx.y * BY + threadIdx.y;
    if (x >= a.nx || y >= a.ny) return;
    const long plane = (long)a.nx * a.ny, d = (long)y * a.nx + x, n = node(a, x, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i * a.plane + n] = (T)in[i * plane + d];
    if constexpr (keeps_cons<T>()) {
        double* cp = (double*)f + cnode(a, x, y);
#pragma unroll
        for (int k = 0; k < 4; ++k) cp[k * a.cplane] = in[(NQ + k) * plane + d];
    }
}

// ---------------------------------------------------------------------------
// Batched form: many independent instances advance in one persistent launch
// per tile-shape class.  Each slot carries its own arguments and ping-pong
// buffers.  The batch counts steps (L) and rounds (R): a round is one step,
// or two steps for the slots that take two per launch ("pair" slots) while
// the others take two one-step launches.  A slot's current buffer is the
// parity of its clock (R for pair slots, L for the others) against pstart,
// and it steps while L < stop, so slots join, finish and leave without
// per-launch uploads.
struct BatchSlot {
    StepArgs a;
    void* buf[2];
    long start;   // step counter at which the slot's step count starts
    long stop;    // first step counter at which the slot no longer steps
    long pstart;  // clock value at which buffer 0 held the slot's state
    int pair;     // 1: the slot's clock is R (it takes two steps per launch in two-step rounds)
};

// Work items are the tiles of the listed slots, numbered slot after slot
// (prefix[k] = first item of list[k]); block b takes items b, b + grid, ...
template <int LIM, typename T, int TXW, int BYR, bool FLAT>
__global__ void __launch_bounds__(TXW * BYR, 1) k_step_batch(const BatchSlot* __restrict__ slots,
                                                            const int* __restrict__ prefix,
                                                            const int* __restrict__ list, int nlist, long L)
{
    __shared__ TileSmem<T, TXW, BYR, FLAT> sm_;
    convect_mode();
    const int nitems = prefix[nlist];
    for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        int lo = 0, hi = nlist;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= item) lo = mid;
            else hi = mid;
        }
        const BatchSlot& sl = slots[list[lo]];
        if (L < sl.stop) {
            const int par = (int)((L - sl.pstart) & 1);   // never a pair slot
            step_tile<LIM, T, TXW, BYR, FLAT>((const T*)sl.buf[par], (T*)sl.buf[par ^ 1], sl.a, item - prefix[lo], sm_);
        }
        __syncthreads();   // LDS is reused by the next item
    }
}

// Wall refill after a batched launch at step counter L and round R: one
// block per listed slot with walls, refilling the buffer the launch wrote.
template <typename T>
__global__ void k_wall_batch(const BatchSlot* __restrict__ slots, const int* __restrict__ wlist, long L, long R)
{
    const BatchSlot& sl = slots[wlist[blockIdx.x]];
    if (L >= sl.stop) return;
    const int par = (int)(((sl.pair ? R : L) - sl.pstart) & 1);
    T* f = (T*)sl.buf[par ^ 1];
    for (int axis = 0; axis < 2; ++axis) {
        if (sl.a.bc[2 * axis] != BC_WALL && sl.a.bc[2 * axis + 1] != BC_WALL) continue;
        const int n = 2 * ((axis == 0) ? sl.a.ny : sl.a.nx);
        for (int t = threadIdx.x; t < n; t += blockDim.x) fill_line(f, sl.a, axis, t, 1);
    }
}

}  // namespace
