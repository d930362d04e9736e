// mrtfd_march.h -- row-marching form of the fused D2V16 MRT-FD step
// (arXiv:1305.4736, Sec. III update eq.) for one large instance.
//
// A wavefront owns a strip of 64 columns and a band of rows.  Its lanes are
// the strip's columns: the two lanes at each side are halo, the 60 inner
// lanes produce output.  The wavefront walks the band one row at a time and
// holds four rows of all 16 planes in registers (the rows behind, at and
// ahead of the output row, and the next row, whose loads are in flight while
// the current row is computed); HBM is read once per row plus four halo rows
// per band and written once.  Neighbours along x come from the adjacent lanes
// (DPP whole-wavefront shifts), neighbours along y from the register window.
// The limited jump of each y face is evaluated once and carried to the next
// row.  Every value is formed from the same operands in the same order as in
// the LDS-tile kernel (k_step), so both give bitwise identical results.
//
// Periodic and outflow sides are read at their source nodes (a column is
// remapped once per lane, a row once per row), so this kernel writes no
// ghost images; equilibrium ghosts are constant.  NEE walls along y are
// refilled by the wavefronts whose bands end at a wall, after their walk
// (and between the two steps of a pair, in its ring); walls along x by a
// separate launch after the step.
//
// Two steps per pass (k_march2): a block holds two wavefronts on the same
// strip and band.  The first takes step n -> n+1 from HBM and leaves each
// new row in a ring of rows in LDS; the second takes step n+1 -> n+2 from
// that ring and writes HBM.  A barrier per row keeps the two in step.  HBM
// sees one read and one write of the state per two steps.
#pragma once
#include <algorithm>

#include "mrtfd_kernels.h"

namespace {

constexpr int MW = 64;           // lanes of a wavefront = columns of a strip
constexpr int MOUT = MW - 4;     // output columns of a strip
#ifndef MARCH_WPB
#define MARCH_WPB 4
#endif
constexpr int MWPB = MARCH_WPB;  // wavefronts (independent strips) per block
// Fewest rows per band.  Small grids are bound by the latency of walking
// the band row after row, so they get as many one-row bands as the device
// holds (4 x 200: 10 us per step, against 25 us with 8-row bands); large
// grids are limited by the resident wavefronts instead.
#ifndef MARCH_RMIN
#define MARCH_RMIN 1
#endif
constexpr int MRMIN = MARCH_RMIN;
#ifndef MARCH_LOAD_AUX
#define MARCH_LOAD_AUX 0         // cache policy bits of the state loads
#endif
#ifndef MARCH_STORE_AUX
#define MARCH_STORE_AUX 0        // cache policy bits of the state stores
#endif
#ifndef MARCH_ALTERNATE
#define MARCH_ALTERNATE 1        // adjacent bands march in opposite directions
#endif
// Wave priority (s_setprio) of the first wavefront of a fused pair: with the
// first step ahead in the SIMDs' issue order the pair kernel runs 6.5 %
// faster (FP64; FP32 7 %); priority 3 measured the same, raising the second
// wavefront's or raising it only while a row's loads are issued gained
// nothing, nor did the latter for the one-step kernel.
#ifndef MARCH2_PRIO_FIRST
#define MARCH2_PRIO_FIRST 1
#endif
// Bands are sized so that the launch has this fraction of the wavefronts
// the device holds at once.  FP64 does best with about one wavefront per
// SIMD (longer bands: fewer halo rows and fewer concurrent streams); FP32,
// whose step is bound by its FP64 collision arithmetic, with two.
#ifndef MARCH_FRAC64
#define MARCH_FRAC64 0.5
#endif
#ifndef MARCH_FRAC32
#define MARCH_FRAC32 1.0
#endif

// Whole-wavefront lane moves (DPP wave_shr:1 / wave_shl:1): lane l receives
// the value of lane l - 1 (FROM_LEFT) or l + 1 (FROM_RIGHT); the lane at the
// end receives 0 (bound control).  All 64 lanes must be active.
constexpr int FROM_LEFT = 0x138;
constexpr int FROM_RIGHT = 0x130;

template <int CTRL>
__device__ __forceinline__ double lane_move(double v)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, true);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float lane_move(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Kernel arguments and moment blocks are read through the constant address
// space: loads from it stay scalar (s_load) even in a loop that stores.
#define MRTFD_CONSTANT __attribute__((address_space(4)))
using CArgs = const MRTFD_CONSTANT StepArgs;
using CBlocks = const MRTFD_CONSTANT Blocks;

__device__ __forceinline__ CBlocks& blocks_of(CArgs& a) { return *(CBlocks*)a.Bp; }

// Buffer resources: loads and stores address plane i, row y of a state
// buffer as a scalar offset (i * plane + org - 2 + y * pitch elements) plus a
// per-lane offset (column + 2) that stays fixed for the whole walk, so no
// per-lane address arithmetic is spent per row.  The march is only used for
// buffers below 2 GiB, where both offsets fit 31 bits.  Lanes that must not
// store use the per-lane offset NO_STORE: at least 2 GiB, beyond the buffer's
// size, so the hardware range check discards the store.
constexpr int BUF_WORD3 = 0x00020000;   // raw 32-bit data format (gfx9 family)
constexpr unsigned NO_STORE = 0x80000000u;
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
// s_waitcnt immediate (gfx9 family) that waits for every vector memory
// operation of the wavefront: vmcnt 0, expcnt and lgkmcnt at their maxima.
constexpr int MRTFD_WAIT_VM0 = 0x0F70;

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double*)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, MARCH_LOAD_AUX));
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float*)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, MARCH_LOAD_AUX));
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)voff, (int)soff, MARCH_STORE_AUX);
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, MARCH_STORE_AUX);
}

// Per-lane byte offset of a conserved-moment plane (FP64) from that of a
// population plane (FP32 storage, 4-byte elements): twice as far; NO_STORE
// stays NO_STORE.
__device__ __forceinline__ unsigned cons_off(unsigned voff) { return (voff == NO_STORE) ? NO_STORE : 2u * voff; }

// Coordinate c in [-2, n + 1] of an axis with n nodes, mapped to the node
// that holds its value: periodic sides wrap, outflow sides repeat the last
// node, equilibrium and wall sides keep their stored ghosts.
__device__ __forceinline__ int source_of(int c, int n, int lo_kind, int hi_kind)
{
    if (c < 0) {
        if (lo_kind == BC_PERIODIC) return (n == 1) ? 0 : c + n;
        if (lo_kind == BC_OUTFLOW) return 0;
    } else if (c >= n) {
        if (hi_kind == BC_PERIODIC) return (n == 1) ? 0 : c - n;
        if (hi_kind == BC_OUTFLOW) return n - 1;
    }
    return c;
}

// Coordinate c in [-4, n + 3] mapped to the node whose value the first step
// of a fused pair reads there: periodic sides wrap (any distance), outflow
// sides repeat the last node, equilibrium sides keep their stored ghosts
// (coordinates beyond the two ghost layers read the outer one; no output
// the pair keeps depends on them).
__device__ __forceinline__ int source_ext(int c, int n, int lo_kind, int hi_kind)
{
    if (c < 0) {
        if (lo_kind == BC_PERIODIC) {   // c >= -4: at most four turns (n = 1)
            while (c < 0) c += n;
            return c;
        }
        if (lo_kind == BC_OUTFLOW) return 0;
        return max(c, -2);
    }
    if (c >= n) {
        if (hi_kind == BC_PERIODIC) {   // c <= n + 3
            while (c >= n) c -= n;
            return c;
        }
        if (hi_kind == BC_OUTFLOW) return n - 1;
        return min(c, n + 1);
    }
    return c;
}

// Coordinate c in [-2, n + 1] mapped to the node whose step result the
// second step of a pair reads there: outflow ghosts repeat the last node
// (its new value); periodic ghosts were computed by the first step at their
// own lane or row, equilibrium ghosts passed through unchanged.
__device__ __forceinline__ int source_out(int c, int n, int lo_kind, int hi_kind)
{
    if (c < 0 && lo_kind == BC_OUTFLOW) return 0;
    if (c >= n && hi_kind == BC_OUTFLOW) return n - 1;
    return c;
}

// Roles of a marching wavefront: one whole step (HBM to HBM), or the first
// (HBM to LDS ring) or second (LDS ring to HBM) step of a fused pair.
enum { ROLE_SINGLE = 0, ROLE_FIRST = 1, ROLE_SECOND = 2 };
constexpr int PRING = 4;          // rows held by the ring of a pair
constexpr int POUT = MW - 8;      // output columns of a pair's strip

// The ring: row y of the first step's result lives in slot (y + 4) mod 4
// (y >= -2), lane l of the strip at [slot][plane][l]; FP32 storage also
// passes each row's FP64 conserved moments, at [slot][k][l].
template <typename T>
struct PairRing {
    T v[PRING][NQ][MW];
#if MARCH2_MFMA
    double mt[NQ][MW];   // matrix-core trial: a row's moments, moment-major
#endif
};
template <>
struct PairRing<float> {
    float v[PRING][NQ][MW];
    double c[PRING][4][MW];
};

// Wall rows of step n + 1 in a pair's ring, lane `lane`: the first step's
// row c1 next to the wall gives, by the same arithmetic as the refill after
// a one-step launch, the wall node's row w (kmin = 0) and its first ghost
// row w + out (kmax = 1; out = -1 on the low side, +1 on the high side).
// A row of FP64 populations v written to ring slot `sl` at lane `lane`
// (rounded to T; FP32 storage also writes their conserved moments).
template <typename T>
__device__ __forceinline__ void ring_put(CArgs& a, PairRing<T>* ring, int sl, int lane, const double* v)
{
#pragma unroll
    for (int i = 0; i < NQ; ++i) ring->v[sl][i][lane] = (T)v[i];
    if constexpr (keeps_cons<T>()) {
        double c[4];
        cons_of(blocks_of(a), all_sums(v), c);
#pragma unroll
        for (int k = 0; k < 4; ++k) ring->c[sl][k][lane] = c[k];
    }
}

template <typename T>
__device__ __forceinline__ void ring_wall(CArgs& a, PairRing<T>* ring, int lane, int side, int c1, int w, int out,
                                          int kmin, int kmax)
{
    const int s1 = (c1 + 4) & (PRING - 1);
    double f1[NQ], fw[NQ];
    if constexpr (keeps_cons<T>()) {
        double ft[NQ], c[4];
#pragma unroll
        for (int i = 0; i < NQ; ++i) ft[i] = (double)ring->v[s1][i][lane];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = ring->c[s1][k][lane];
        resync(blocks_of(a), ft, c, f1);
    } else {
#pragma unroll
        for (int i = 0; i < NQ; ++i) f1[i] = (double)ring->v[s1][i][lane];
    }
    wall_values(a, blocks_of(a), f1, side, fw);
    if (kmin == 0) ring_put(a, ring, (w + 4) & (PRING - 1), lane, fw);
    if (kmax == 1) {
        double g[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) g[i] = wall_ghost(fw[i], f1[i], 1);
        ring_put(a, ring, (w + out + 4) & (PRING - 1), lane, g);
    }
}

// One wavefront's walk through its band in direction DIR (+1: increasing y).
// Output row j reads rows j, j + DIR and, for the planes whose y-upstream
// side is ahead, j + 2 DIR.  The planes whose upstream side is behind need
// the jump f_j - f_{j - DIR}, which is the jump the previous row took on its
// downstream side (the same operands): it is carried, like each y face's
// limited jump, so row j - DIR itself is not kept.  The window W holds three
// rows of all 16 planes: for output row j walked in phase PH, slot PH % 3
// holds row j, (PH + 1) % 3 row j + DIR, and (PH + 2) % 3 receives row
// j + 2 DIR, whose loads are issued at the start of row j.  The next row is
// walked in phase PH + 1, so three rows in phases 0..2 move the window by
// renaming alone; advance() moves it by copies and keeps phase 0.  The
// velocities U, V use the same slots, except that slot (PH + 2) % 3 holds
// that of row j - DIR (for the central differences of the correction) until
// row j + 2 DIR's replaces it at the end of row j.
//
// In a fused pair (ROLE_FIRST / ROLE_SECOND) the lanes of both wavefronts
// are columns x0 + 56 s - 4 .. x0 + 56 s + 59 of strip s.  The first step
// is valid on lanes 2..61, the second on lanes 4..59 (its output).  The
// second copies its rows from the ring where the first left them.
template <int LIM, typename T, int DIR, int ROLE = ROLE_SINGLE>
struct Marcher {
    using R = conv_t<T>;   // convection precision
    using value_type = T;
    static constexpr int dir = DIR;
    static constexpr int role = ROLE;
    // ROLE_SECOND copies each row from the ring into its window, as the
    // first step loads them from HBM, and takes the neighbouring columns by
    // lane moves.  Measured alternatives, same boxes: reading the rows in
    // the ring where they are used (DIRECT; no window copies) 7-8 % slower
    // in FP64 (0.140-0.142 against 0.131-0.133 ms per step; the reads sit
    // on each row's critical path) and more instructions in FP32; reading
    // the FP64 neighbouring columns in the ring instead of two lane moves
    // per double (LDS_X) 2.5 % fewer VALU instructions per wavefront but
    // 3 % slower (0.136-0.139 ms).
#ifndef MARCH2_DIRECT
#define MARCH2_DIRECT 0
#endif
#ifndef MARCH2_LDS_X64
#define MARCH2_LDS_X64 0
#endif
    static constexpr bool DIRECT = (ROLE == ROLE_SECOND) && MARCH2_DIRECT;
    static constexpr bool LDS_X = (ROLE == ROLE_SECOND) && sizeof(R) == 8 && MARCH2_LDS_X64;

    CArgs* argp;                      // kernel arguments
    __amdgpu_buffer_rsrc_t rin, rout;
    unsigned vin;                     // per-lane load offset (bytes)
    unsigned vout;                    // per-lane store offset, NO_STORE off the output columns
    PairRing<T>* ring;                // fused pair: the LDS ring
    int lane;                         // ROLE_FIRST: own lane; ROLE_SECOND: lane read from the ring
    int laneL, laneR;                 // ROLE_SECOND: lanes read for the columns x - 1 and x + 1
    bool pass;                        // ROLE_FIRST: an equilibrium ghost column (value passes through)
    bool chk;                         // ROLE_FIRST: an interior column this wavefront checks
    T W[3][NQ];                       // the window (see above)
    double CW[3][4];                  // FP32 storage: conserved moments of each window row
    double U[3], V[3];                // velocity (u_x, u_y) of each window row, and of row j - DIR
    R carry[NQ];                      // limited jump of the y face carried from the previous row
    R dcarry[NQ];                     // planes with sgy == DIR: the jump f_j - f_{j - DIR}
#if MARCH2_MFMA
    double Ma[4];                     // matrix-core trial: M[i][4 s + k] at lane i + 16 k, s = 0..3
#endif

    __device__ __forceinline__ Marcher(CArgs* ap, const T* fin, T* fout, unsigned bytes, int x, bool out)
        : argp(ap),
          rin(__builtin_amdgcn_make_buffer_rsrc((void*)fin, (short)0, (int)bytes, BUF_WORD3)),
          rout(__builtin_amdgcn_make_buffer_rsrc((void*)fout, (short)0, (int)bytes, BUF_WORD3)),
          vin((unsigned)(source_of(min(x, ap->nx + 1), ap->nx, ap->bc[0], ap->bc[1]) + 2) * (unsigned)sizeof(T)),
          vout(out ? (unsigned)(x + 2) * (unsigned)sizeof(T) : NO_STORE), ring(nullptr), lane(0), laneL(0),
          laneR(0), pass(false), chk(false)
    {
    }

    // A wavefront of a fused pair; l is its lane, x the lane's column.
    __device__ __forceinline__ Marcher(CArgs* ap, const T* fin, T* fout, unsigned bytes, int x, int l,
                                       PairRing<T>* rg)
        : argp(ap),
          rin(__builtin_amdgcn_make_buffer_rsrc((void*)fin, (short)0, (int)bytes, BUF_WORD3)),
          rout(__builtin_amdgcn_make_buffer_rsrc((void*)fout, (short)0, (int)bytes, BUF_WORD3)), ring(rg)
    {
        const int nx = ap->nx, lo = ap->bc[0], hi = ap->bc[1];
        if (ROLE == ROLE_FIRST) {
            vin = (unsigned)(source_ext(x, nx, lo, hi) + 2) * (unsigned)sizeof(T);
            vout = NO_STORE;
            lane = l;
            laneL = laneR = 0;
            pass = (x < 0 && lo == BC_EQUIL) || (x >= nx && hi == BC_EQUIL);
            chk = l >= 2 && l < MW - 2 && x >= ap->x0 && x < ap->x1;
        } else {
            vin = 0;
            const bool out = l >= 4 && l < MW - 4 && x < ap->x1;
            vout = out ? (unsigned)(x + 2) * (unsigned)sizeof(T) : NO_STORE;
            // the lane holding column x + q's value (outflow ghost columns:
            // the column they repeat), kept inside the strip
            auto lane_of = [&](int q) {
                return min(max(l + q + (source_out(x + q, nx, lo, hi) - (x + q)), 0), MW - 1);
            };
            lane = lane_of(0);
            laneL = lane_of(-1);
            laneR = lane_of(1);
            pass = false;
            chk = false;
        }
    }

    // The kernel arguments, re-read at every row: hiding the pointer from the
    // optimiser keeps it from hoisting ~150 constant dwords out of the loop
    // into scalar registers (they are scalar-cache hits).
    __device__ __forceinline__ CArgs& args() const
    {
        CArgs* p = argp;
        asm volatile("" : "+s"(p));
        return *p;
    }
    // The same, not before the value dep is computed (the collision reads
    // its constants through it; measured against reading them through
    // args(): the same instructions and scalar spills).
    __device__ __forceinline__ CArgs& args_after(double dep) const
    {
        CArgs* p = argp;
        asm volatile("" : "+s"(p) : "v"(dep));
        return *p;
    }

    // ROLE_SECOND: the ring slot of row y of the first step's result
    // (outflow ghost rows: the row they repeat).
    __device__ __forceinline__ int rslot(int y, CArgs& a) const
    {
        const int ys = source_out(max(-2, min(y, a.ny + 1)), a.ny, a.bc[2], a.bc[3]);
        return (ys + 4) & (PRING - 1);
    }

    // Population i and (FP32 storage) conserved moment k of the row in slot
    // s: a window slot, or for ROLE_SECOND a ring slot.
    __device__ __forceinline__ T pop(int s, int i) const
    {
        if (DIRECT) return ring->v[s][i][lane];
        return W[s][i];
    }
    __device__ __forceinline__ double cons(int s, int k) const
    {
        if (DIRECT) return ring->c[s][k][lane];
        return CW[s][k];
    }

    __device__ __forceinline__ void load(T (&dst)[NQ], int y, CArgs& a) const
    {
        if (ROLE == ROLE_SECOND) {
            const int sl = rslot(y, a);
#pragma unroll
            for (int i = 0; i < NQ; ++i) dst[i] = ring->v[sl][i][lane];
            return;
        }
        // rows beyond the ghost layers are only ever prefetched past a band's
        // end and never used: read the last ghost row instead
        const int ys = (ROLE == ROLE_FIRST) ? source_ext(y, a.ny, a.bc[2], a.bc[3])
                                            : source_of(max(-2, min(y, a.ny + 1)), a.ny, a.bc[2], a.bc[3]);
        const unsigned base = (unsigned)((a.org - 2 + (long)ys * a.pitch) * (long)sizeof(T));
        const unsigned pb = (unsigned)(a.plane * (long)sizeof(T));
#pragma unroll
        for (int i = 0; i < NQ; ++i) dst[i] = buf_load(rin, vin, base + (unsigned)i * pb, (T*)nullptr);
    }

    // FP32 storage: the conserved moments of row y, from the same source as load().
    __device__ __forceinline__ void load_cons(double (&dst)[4], int y, CArgs& a) const
    {
        if constexpr (keeps_cons<T>()) {
            if (ROLE == ROLE_SECOND) {
                const int sl = rslot(y, a);
#pragma unroll
                for (int k = 0; k < 4; ++k) dst[k] = ring->c[sl][k][lane];
                return;
            }
            const int ys = (ROLE == ROLE_FIRST) ? source_ext(y, a.ny, a.bc[2], a.bc[3])
                                                : source_of(max(-2, min(y, a.ny + 1)), a.ny, a.bc[2], a.bc[3]);
            const unsigned base = (unsigned)((a.corg - 2 + (long)ys * a.cpitch) * 8L);
            const unsigned pb = (unsigned)(a.cplane * 8L);
#pragma unroll
            for (int k = 0; k < 4; ++k) dst[k] = buf_load(rin, 2u * vin, base + (unsigned)k * pb, (double*)nullptr);
        }
    }

    // A whole window row: populations and (FP32 storage) conserved moments.
    __device__ __forceinline__ void load_row(int s, int y, CArgs& a)
    {
        load(W[s], y, a);
        load_cons(CW[s], y, a);
    }

    // Velocity slot vs from the row in slot s (see pop()): from its
    // populations, or in FP32 storage from its stored conserved moments.
    __device__ __forceinline__ void velocity(int s, int vs, CArgs& a)
    {
        if constexpr (keeps_cons<T>()) {
            velocity_of_cons(cons(s, 0), cons(s, 1), cons(s, 2), U[vs], V[vs]);
        } else {
            double g[NQ];
#pragma unroll
            for (int i = 0; i < NQ; ++i) g[i] = (double)pop(s, i);
            velocity_of(blocks_of(a), g, U[vs], V[vs]);
        }
    }

    // The jumps carried into output row j from rows j - 2 DIR (e), j - DIR
    // (b), j (c) and j + DIR (d): what the row before j would have left.
    __device__ __forceinline__ void start_carry(const T* e, const T* b, const T* c, const T* d)
    {
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
            const int sy = sgy(i);
            if (sy == DIR) {
                carry[i] = limited<LIM, R>((R)b[i] - (R)e[i], (R)c[i] - (R)b[i]);
                dcarry[i] = (R)c[i] - (R)b[i];
            } else if (sy == -DIR) {
                carry[i] = limited<LIM, R>((R)c[i] - (R)d[i], (R)b[i] - (R)c[i]);
            }
        }
    }

#if MARCH2_MFMA
    // Matrix-core trial (FP64 storage, second step of a pair): the moments
    // of the row in ring slot sC as D = M F, F the 16 x 64 block of the row
    // (velocity x column), in four 16-column blocks of four K = 4 products;
    // F is read from the ring in operand layout (lane k' * 16 + c holds
    // plane 4 s + k' of column 16 b + c), D leaves register r of lane
    // 16 q + c with moment q + 4 r of column 16 b + c (the layout measured
    // on gfx950) and goes back to one column per lane through LDS.
    typedef double double4_t __attribute__((ext_vector_type(4)));
    __device__ __forceinline__ void mfma_load_a()
    {
        CArgs& a = args();
        const double* Md = &((const Blocks*)a.Bp)->Md[0][0];
        const int i = lane_id() & 15, k = lane_id() >> 4;
#pragma unroll
        for (int st = 0; st < 4; ++st) Ma[st] = Md[i * NQ + 4 * st + k];
    }
    __device__ __forceinline__ static int lane_id() { return (int)__lane_id(); }
    __device__ __forceinline__ void mfma_moments(int sC, double* m)
    {
        const int l = lane_id(), c = l & 15, q = l >> 4;
        double4_t d[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) d[b] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                d[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ma[st], (double)ring->v[sC][4 * st + q][16 * b + c], d[b],
                                                           0, 0, 0);
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) ring->mt[q + 4 * r][16 * b + c] = d[b][r];
        // this wavefront's own LDS writes, read back by other lanes: LDS
        // keeps a wavefront's operations in order; the compiler must too
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
        for (int i = 0; i < NQ; ++i) m[i] = ring->mt[i][lane];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    }
#endif

    // New value of plane i at output row j; rows j, j + DIR, j + 2 DIR in
    // slots sC, sD, sE (see pop()), row j in ring slot rC (ROLE_SECOND).
    __device__ __forceinline__ double plane_value(int i, const double* coll, CArgs& a, int sC, int sD, int sE,
                                                  int rC)
    {
        const int g = i >> 2;
        const R f0 = (R)pop(sC, i);
        R acc = acc_start<T, R>(coll[i]);
        const int sx = sgx(i), sy = sgy(i);
        if (sx != 0) {
            R d1, d2;
            if (LDS_X) {
                // the neighbouring columns from the ring (same operands as
                // the lane moves below)
                const R fl = (R)ring->v[rC][i][laneL], fr = (R)ring->v[rC][i][laneR];
                d1 = f0 - ((sx > 0) ? fl : fr);
                d2 = ((sx > 0) ? fr : fl) - f0;
            } else {
                const R fm1 = (sx > 0) ? lane_move<FROM_LEFT>(f0) : lane_move<FROM_RIGHT>(f0);
                d1 = f0 - fm1;
                // the downstream jump is the next lane's upstream one (same operands)
                d2 = (sx > 0) ? lane_move<FROM_RIGHT>(d1) : lane_move<FROM_LEFT>(d1);
            }
            const R l1 = limited<LIM, R>(d1, d2);
            const R l0 = (sx > 0) ? lane_move<FROM_LEFT>(l1) : lane_move<FROM_RIGHT>(l1);
            acc = conv_add(acc, l1, l0, d1, nu_of<R, 0>(a, g), c_of<R, 0, LIM>(a, g));
        }
        if (sy != 0) {
            R d1, l1, l0;
            if (sy == DIR) {        // upstream row is behind: its jump and face value are carried
                d1 = dcarry[i];
                const R d2 = (R)pop(sD, i) - f0;
                l1 = limited<LIM, R>(d1, d2);
                l0 = carry[i];
                carry[i] = l1;
                dcarry[i] = d2;
            } else {                // upstream row is ahead: needs row j + 2 DIR
                const R fd = (R)pop(sD, i);
                d1 = f0 - fd;
                l1 = carry[i];
                l0 = limited<LIM, R>(fd - (R)pop(sE, i), d1);
                carry[i] = l0;
            }
            acc = conv_add(acc, l1, l0, d1, nu_of<R, 1>(a, g), c_of<R, 1, LIM>(a, g));
        }
        return new_value<T, R>(f0, acc, coll[i]);
    }

    // Output row j in phase PH.
    template <int PH>
    __device__ __forceinline__ void row(int j)
    {
        constexpr int C = PH % 3, D = (PH + 1) % 3, E = (PH + 2) % 3;
        CArgs& a = args();
        int sC = C, sD = D, sE = E;
        const int rC = (ROLE == ROLE_SECOND) ? rslot(j, a) : 0;
        if (DIRECT) {
            sC = rC;
            sD = rslot(j + DIR, a);
            sE = rslot(j + 2 * DIR, a);
        } else {
            load_row(E, j + 2 * DIR, a);
        }

        // moments, equilibria, correction and collision of row j
        double m[NQ], dc[4];
#if MARCH2_MFMA
        if constexpr (ROLE == ROLE_SECOND && sizeof(T) == 8) {
            mfma_moments(rC, m);
        } else
#endif
        {
            double g[NQ], c[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < NQ; ++i) g[i] = (double)pop(sC, i);
            if constexpr (keeps_cons<T>()) {
#pragma unroll
                for (int k = 0; k < 4; ++k) c[k] = cons(sC, k);
            }
            node_moments<T>(blocks_of(a), g, c, m, dc);
        }
        const double rho = m[0];
        const double vx = U[C], vy = V[C];
        const double P = (m[3] - rho * (vx * vx + vy * vy)) * a.inv_b;
        const bool corr = a.correction != 0;
        double dxux = 0.0, dxuy = 0.0, dyux = 0.0, dyuy = 0.0;
        if (corr) {
            dxux = (lane_move<FROM_RIGHT>(vx) - lane_move<FROM_LEFT>(vx)) * a.inv2dx;
            dxuy = (lane_move<FROM_RIGHT>(vy) - lane_move<FROM_LEFT>(vy)) * a.inv2dx;
            // velocity slot E still holds row j - DIR
            const double uxp = (DIR > 0) ? U[D] : U[E], uxm = (DIR > 0) ? U[E] : U[D];
            const double uyp = (DIR > 0) ? V[D] : V[E], uym = (DIR > 0) ? V[E] : V[D];
            dyux = (uxp - uxm) * a.inv2dy;
            dyuy = (uyp - uym) * a.inv2dy;
        }
        const bool checked = (ROLE == ROLE_FIRST) ? (chk && j >= a.y0 && j < a.y1) : (vout != NO_STORE);
        if (checked && !(rho > 0.0 && P > 0.0)) atomicOr(a.flag, 1);
        double coll[NQ];
        {
            CArgs& ac = args_after(P);
            collision<keeps_cons<T>()>(ac, blocks_of(ac), m, rho, vx, vy, P, corr, dxux, dxuy, dyux, dyuy, dc, coll);
        }

        const unsigned base = (unsigned)((a.org - 2 + (long)j * a.pitch) * (long)sizeof(T));
        const unsigned pb = (unsigned)(a.plane * (long)sizeof(T));
        // equilibrium ghost rows (uniform) and columns keep their (constant) values
        constexpr bool KEEP_SELECT = sizeof(T) == 4;
        const bool keep_row = (ROLE == ROLE_FIRST) &&
                              ((j < 0 && a.bc[2] == BC_EQUIL) || (j >= a.ny && a.bc[3] == BC_EQUIL));
        const bool keep = (ROLE == ROLE_FIRST) &&
                          (pass || (j < 0 && a.bc[2] == BC_EQUIL) || (j >= a.ny && a.bc[3] == BC_EQUIL));
        const int rs = (j + 4) & (PRING - 1);
        T(*dst)[MW] = (ROLE == ROLE_FIRST) ? ring->v[rs] : nullptr;
        double vd[NQ];   // new populations in FP64 (FP32 storage keeps their conserved moments)
        // planes that do not need row j + 2 DIR first, so its loads have time
#pragma unroll
        for (int ps = 0; ps < 2; ++ps) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                if ((ps == 1) != (sgy(i) == -DIR)) continue;
                vd[i] = plane_value(i, coll, a, sC, sD, sE, rC);
                const T v = (T)vd[i];
                if (ROLE == ROLE_FIRST)
                    dst[i][lane] = KEEP_SELECT ? (keep ? W[C][i] : v) : v;
                else
                    buf_store(v, rout, vout, base + (unsigned)i * pb);
            }
        }
        if constexpr (keeps_cons<T>()) {
            double cn[4];
            cons_of(blocks_of(a), all_sums(vd), cn);
            if (ROLE == ROLE_FIRST) {
#pragma unroll
                for (int k = 0; k < 4; ++k) ring->c[rs][k][lane] = keep ? CW[C][k] : cn[k];
            } else {
                const unsigned cb = (unsigned)((a.corg - 2 + (long)j * a.cpitch) * 8L);
                const unsigned cpb = (unsigned)(a.cplane * 8L);
#pragma unroll
                for (int k = 0; k < 4; ++k) buf_store(cn[k], rout, cons_off(vout), cb + (unsigned)k * cpb);
            }
        }
        // FP64: the kept values overwrite the new ones afterwards, on the few
        // wavefronts that hold such a column or row, instead of a select per
        // plane (two per double) on every wavefront: 0.5-1 % faster; FP32
        // (one select per plane, a larger kernel, the conserved moments
        // selected too) keeps the select, which measured 12 % faster there
        // (0.135 against 0.154 ms per step at 4096 x 1024)
        if (ROLE == ROLE_FIRST && !KEEP_SELECT && (__builtin_amdgcn_ballot_w64(pass) != 0 || keep_row)) {
            if (pass || keep_row) {
#pragma unroll
                for (int i = 0; i < NQ; ++i) dst[i][lane] = W[C][i];
            }
        }
        velocity(sE, E, a);
    }

    // ROLE_FIRST: row j of step n + 1 on a high wall side (k = 0: the wall
    // node's row, 1: its first ghost row), refilled from the row below the
    // wall instead of stepped; equilibrium ghost columns keep their value.
    __device__ __forceinline__ void wall_row(int j, int k)
    {
        CArgs& a = args();
        if (pass) {
            T v[NQ];
            load(v, j, a);
            const int sl = (j + 4) & (PRING - 1);
            T(*dst)[MW] = ring->v[sl];
#pragma unroll
            for (int i = 0; i < NQ; ++i) dst[i][lane] = v[i];
            if constexpr (keeps_cons<T>()) {
                double c[4];
                load_cons(c, j, a);
#pragma unroll
                for (int k = 0; k < 4; ++k) ring->c[sl][k][lane] = c[k];
            }
        } else {
            ring_wall(a, ring, lane, 3, a.ny - 2, a.ny - 1, 1, k, k);
        }
    }

    // NEE walls along y of the new state, refilled by the wavefront whose
    // band ends at a wall, after its walk: the row next to the wall is read
    // back from the output (this lane wrote it) and the wall node's row and
    // its two ghost rows are written by the same arithmetic as the refill
    // launch, on the output lanes.  Walls along x are refilled by a launch.
    __device__ __forceinline__ void refill_walls(int yb, int ye)
    {
        CArgs& a = args();
        if (a.bc[0] == BC_WALL || a.bc[1] == BC_WALL) return;
        const bool lo = a.bc[2] == BC_WALL && yb == a.y0;
        const bool hi = a.bc[3] == BC_WALL && ye == a.y1;
        if ((!lo && !hi) || vout == NO_STORE) return;
        // this lane's stores of the walk are complete before the row is read
        __builtin_amdgcn_s_waitcnt(MRTFD_WAIT_VM0);
        if (lo) wall_rows(a, 2, a.y0, a.y0 - 1, -1);
        if (hi) wall_rows(a, 3, a.y1 - 1, a.y1, 1);
    }

    // Wall node row cw and its ghost rows cw + out, cw + 2 out from output
    // row c1, on this lane's column.
    __device__ __forceinline__ void wall_rows(CArgs& a, int side, int c1, int cw, int out)
    {
        const unsigned pb = (unsigned)(a.plane * (long)sizeof(T));
        const unsigned b1 = (unsigned)((a.org - 2 + (long)c1 * a.pitch) * (long)sizeof(T));
        const unsigned b0 = (unsigned)((a.org - 2 + (long)cw * a.pitch) * (long)sizeof(T));
        const unsigned step = (unsigned)((long)out * a.pitch * (long)sizeof(T));
        double f1[NQ], fw[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) f1[i] = (double)buf_load(rout, vout, b1 + (unsigned)i * pb, (T*)nullptr);
        if constexpr (keeps_cons<T>()) {
            double c[4], ft[NQ];
            const unsigned cb1 = (unsigned)((a.corg - 2 + (long)c1 * a.cpitch) * 8L), cpb = (unsigned)(a.cplane * 8L);
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = buf_load(rout, cons_off(vout), cb1 + (unsigned)k * cpb, (double*)nullptr);
#pragma unroll
            for (int i = 0; i < NQ; ++i) ft[i] = f1[i];
            resync(blocks_of(a), ft, c, f1);
        }
        wall_values(a, blocks_of(a), f1, side, fw);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            double g[NQ];
#pragma unroll
            for (int i = 0; i < NQ; ++i) g[i] = (r == 0) ? fw[i] : wall_ghost(fw[i], f1[i], r);
#pragma unroll
            for (int i = 0; i < NQ; ++i) buf_store((T)g[i], rout, vout, b0 + (unsigned)r * step + (unsigned)i * pb);
            if constexpr (keeps_cons<T>()) {
                double c[4];
                cons_of(blocks_of(a), all_sums(g), c);
                const unsigned cb = (unsigned)((a.corg - 2 + (long)(cw + r * out) * a.cpitch) * 8L);
                const unsigned cpb = (unsigned)(a.cplane * 8L);
#pragma unroll
                for (int k = 0; k < 4; ++k) buf_store(c[k], rout, cons_off(vout), cb + (unsigned)k * cpb);
            }
        }
    }

    // The window, velocities and carried jumps of output row j in phase 0:
    // rows j (slot 0) and j + DIR (slot 1); rows j - 2 DIR and j - DIR only
    // for the carries and the velocity of j - DIR (velocity slot 2).
    __device__ __forceinline__ void prime(int j)
    {
        CArgs& a = args();
        T e[NQ], b[NQ];
#if MARCH2_MFMA
        if constexpr (ROLE == ROLE_SECOND && sizeof(T) == 8) mfma_load_a();
#endif
        if (DIRECT) {
            const int s1 = rslot(j - DIR, a), s0 = rslot(j, a), sd = rslot(j + DIR, a);
            load(e, j - 2 * DIR, a);
            load(b, j - DIR, a);
            velocity(s1, 2, a);
            velocity(s0, 0, a);
            velocity(sd, 1, a);
            T c[NQ], d[NQ];
            load(c, j, a);
            load(d, j + DIR, a);
            start_carry(e, b, c, d);
        } else {
            load(e, j - 2 * DIR, a);
            load_row(2, j - DIR, a);
            load_row(0, j, a);
            load_row(1, j + DIR, a);
            velocity(2, 2, a);
            velocity(0, 0, a);
            velocity(1, 1, a);
#pragma unroll
            for (int i = 0; i < NQ; ++i) b[i] = W[2][i];
            start_carry(e, b, W[0], W[1]);
        }
    }

    // Move the window one row on by copies (phase 0 before and after); the
    // velocity of row j becomes that of the new row's j - DIR.
    __device__ __forceinline__ void advance()
    {
        if (!DIRECT) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                W[0][i] = W[1][i];
                W[1][i] = W[2][i];
            }
            if constexpr (keeps_cons<T>()) {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    CW[0][k] = CW[1][k];
                    CW[1][k] = CW[2][k];
                }
            }
        }
        const double u0 = U[0], v0 = V[0];
        U[0] = U[1]; V[0] = V[1];
        U[1] = U[2]; V[1] = V[2];
        U[2] = u0; V[2] = v0;
    }

    // Output rows [yb, ye), walked from yb up (DIR > 0) or from ye - 1 down.
    __device__ __forceinline__ void walk(int yb, int ye)
    {
        if (ye <= yb) return;
        int j = (DIR > 0) ? yb : ye - 1;
        prime(j);
        for (int left = ye - yb;;) {
            row<0>(j);
            if (--left == 0) break;
            j += DIR;
            advance();
        }
    }
};

// The step of one instance (arguments in device memory): wavefront w of
// block b takes work item ((b mod 8) * per_xcd + b / 8) * MWPB + w (blocks go
// round-robin to the 8 XCDs, so each XCD sweeps a contiguous range of
// items); items are numbered band after band, strip by strip within a band.
// Adjacent bands march in opposite directions, so the halo rows two bands
// share are read by both at about the same time.
#ifndef MARCH_MINW32
#define MARCH_MINW32 2           // wavefronts per SIMD the FP32 kernel must fit (register budget)
#endif
template <typename T>
constexpr int march_min_waves() { return sizeof(T) == 4 ? MARCH_MINW32 : 1; }

template <int LIM, typename T>
__global__ void __launch_bounds__(MW * MWPB, march_min_waves<T>()) k_march(const T* __restrict__ fin, T* __restrict__ fout,
                                                    const StepArgs* __restrict__ ap)
{
    convect_mode();
    CArgs& a = *(CArgs*)ap;
    // the wavefront index is uniform across the wavefront: say so, so that
    // band, strip and row offsets live in scalar registers
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / MW)), lane = threadIdx.x % MW;
    const int bid = blockIdx.x;
    const int item = ((bid & 7) * a.m_per_xcd + (bid >> 3)) * MWPB + w;
    if (item >= a.m_nsx * a.m_nby) return;     // whole wavefront
    const int band = item / a.m_nsx, strip = item - band * a.m_nsx;
    const int x = a.x0 + strip * MOUT - 2 + lane;
    const bool out = lane >= 2 && lane < MW - 2 && x < a.x1;
    const int yb = a.y0 + band * a.m_rows, ye = min(yb + a.m_rows, a.y1);
    const unsigned bytes = (unsigned)(a.elems * (long)sizeof(T));
    if (MARCH_ALTERNATE && (band & 1)) {
        Marcher<LIM, T, -1> mr(&a, fin, fout, bytes, x, out);
        mr.walk(yb, ye);
        mr.refill_walls(yb, ye);
    } else {
        Marcher<LIM, T, 1> mr(&a, fin, fout, bytes, x, out);
        mr.walk(yb, ye);
        mr.refill_walls(yb, ye);
    }
}

// Steady rows of a pair three at a time with the window moved by renaming
// (phases 0..2), or one at a time with copies.  (With the former four-row
// window, renaming made FP32 storage 7 % faster -- 110.4 against 118.9 us
// per step at 4096 x 1024 -- and FP64 6 % slower: its registers ran out,
// 256 with spills, and the kernel's code outgrew the instruction cache.)
#ifndef MARCH2_RENAME64
#define MARCH2_RENAME64 1
#endif
#ifndef MARCH2_RENAME32
#define MARCH2_RENAME32 1
#endif

// Barrier between the two wavefronts of a pair that orders their LDS
// accesses only: outstanding HBM loads and stores are not waited for.
__device__ __forceinline__ void pair_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// n rows of a pair's steady part from row j on, one barrier after each:
// three rows per trip in phases 0..2 (the window moves by renaming) where
// that is faster, the rest in phase 0 with copies.
template <class M>
__device__ __forceinline__ void pair_rows(M& m, int j, int n)
{
    constexpr int DIR = M::dir;
    constexpr bool rename = (sizeof(typename M::value_type) == 8) ? MARCH2_RENAME64 : MARCH2_RENAME32;
    int k = 0;
    if (rename) {
        for (; k + 3 <= n; k += 3) {
            m.template row<0>(j);
            pair_sync();
            m.template row<1>(j + DIR);
            pair_sync();
            m.template row<2>(j + 2 * DIR);
            pair_sync();
            j += 3 * DIR;
        }
    }
    for (; k < n; ++k) {
        m.template row<0>(j);
        j += DIR;
        m.advance();
        pair_sync();
    }
}

// The walk of a pair through output rows [yb, ye) (H rows) in direction
// DIR, in H + 6 barrier-separated iterations; r(k) = row of march position
// k.  The first wavefront makes rows r(-2) .. r(H + 1) of step n + 1 at
// iterations 0..3 and 5..H+4; the second reads r(-2) .. r(1) at
// iteration 4 (its carried jumps and velocities) and makes row r(k) of
// step n + 2 at iteration k + 6 from rows r(k) .. r(k + 2) in the ring, the
// last of which the first finished one iteration before.  A ring slot is
// rewritten at the iteration after it was last read at the earliest
// (outflow ghost rows read the last interior row).
//
// Walls along y (DIR > 0 only): the second step needs the wall rows of step
// n + 1 as the refill after a step leaves them.  On the high side the first
// wavefront refills its last rows that reach the wall (at most two: the
// wall node's row and its ghost, from row ny - 2) at their own iterations,
// after its window is dead.  On the low side rows 0 and -1 are made before
// row 1, so the second wavefront, idle until iteration 4, refills them at
// iteration 3 from row 1 (made by iteration 2) while the first writes
// r(1), which is row 2 or 3 and lands in another slot.
template <int LIM, typename T, int DIR>
__device__ __forceinline__ void pair_walk(int role, CArgs& a, const T* fin, T* fout, unsigned bytes, int x, int lane,
                                          int yb, int ye, PairRing<T>* ring)
{
    const int H = ye - yb;
    const int j0 = (DIR > 0) ? yb : ye - 1;
    // both wavefronts pass H + 6 barriers: 6 in the start-up, one per row
    // of the steady part
    if (role == 0) {
#if MARCH2_PRIO_FIRST
        __builtin_amdgcn_s_setprio(MARCH2_PRIO_FIRST);
#endif
        Marcher<LIM, T, DIR, ROLE_FIRST> m(&a, fin, fout, bytes, x, lane, ring);
        // rows r(k) >= ny - 1 on a high wall side are refilled, not stepped
        const int lead = (DIR > 0 && a.bc[3] == BC_WALL) ? max(0, ye + 3 - a.ny) : 0;
        const int nn = H + 4 - lead;             // rows stepped: r(-2) .. r(nn - 3)
        const int ns = min(nn, 4);
        int j = j0 - 2 * DIR;
        m.prime(j);
        for (int t = 0; t < ns; ++t) {           // rows r(-2) .. r(ns - 3), iterations 0 .. ns - 1
            m.template row<0>(j);
            j += DIR;
            m.advance();
            pair_sync();
        }
        int it = ns;
        if (nn >= 4) {
            pair_sync();                         // iteration 4: the second loads its window
            pair_rows(m, j, nn - 4);             // iterations 5 .. nn: rows r(2) .. r(nn - 3)
            it = nn + 1;
        }
        // refilled rows (only with lead > 0, so DIR > 0 and r(k) = yb + k),
        // each at its own iteration
        for (int k = nn - 2; k <= H + 1; ++k) {
            const int at = (k <= 1) ? k + 2 : k + 3;
            for (; it < at; ++it) pair_sync();
            m.wall_row(yb + k, yb + k - (a.ny - 1));
            pair_sync();
            ++it;
        }
        for (; it < H + 6; ++it) pair_sync();    // through iteration H + 5
    } else {
        Marcher<LIM, T, DIR, ROLE_SECOND> m(&a, fin, fout, bytes, x, lane, ring);
        int j = j0;
        for (int t = 0; t < 3; ++t) pair_sync(); // iterations 0 .. 2
        if (DIR > 0 && a.bc[2] == BC_WALL && yb <= 2) {
            const bool pass = (x < 0 && a.bc[0] == BC_EQUIL) || (x >= a.nx && a.bc[1] == BC_EQUIL);
            if (!pass) ring_wall(a, ring, lane, 2, 1, 0, -1, 0, (yb == 1) ? 1 : 0);
        }
        pair_sync();                             // iteration 3
        m.prime(j);                              // iteration 4
        pair_sync();
        pair_sync();                             // iteration 5
        pair_rows(m, j, H);                      // iterations 6 .. H + 5: rows r(0) .. r(H - 1)
        m.refill_walls(yb, ye);
    }
}

// Two steps per pass: block b holds one pair, item (b mod 8) * per_xcd +
// b / 8 (XCD-aware, as in k_march), numbered band after band, strip by
// strip within a band; wavefront 0 takes the first step, wavefront 1 the
// second.  Walls along y are refilled inside the pair (every band walks up);
// walls along x are not supported.
#ifndef MARCH2_MINW
#define MARCH2_MINW 2            // wavefronts per SIMD the pair kernel must fit (register budget)
#endif
// Pairs walk every band in the same direction: 1 % faster than alternating
// (measured twice), and the CUs run half the code.
#ifndef MARCH2_ALTERNATE
#define MARCH2_ALTERNATE 0
#endif
template <int LIM, typename T>
__global__ void __launch_bounds__(2 * MW, MARCH2_MINW) k_march2(const T* __restrict__ fin, T* __restrict__ fout,
                                                          const StepArgs* __restrict__ ap)
{
    __shared__ PairRing<T> ring;
    convect_mode();
    CArgs& a = *(CArgs*)ap;
    const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / MW)), lane = threadIdx.x % MW;
    const int bid = blockIdx.x;
    const int item = (bid & 7) * a.p_per_xcd + (bid >> 3);
    if (item >= a.p_nsx * a.p_nby) return;     // both wavefronts
    const int band = item / a.p_nsx, strip = item - band * a.p_nsx;
    const int x = a.x0 + strip * POUT - 4 + lane;
    const int yb = a.y0 + band * a.p_rows, ye = min(yb + a.p_rows, a.y1);
    const unsigned bytes = (unsigned)(a.elems * (long)sizeof(T));
    if (MARCH2_ALTERNATE && (band & 1))
        pair_walk<LIM, T, -1>(role, a, fin, fout, bytes, x, lane, yb, ye, &ring);
    else
        pair_walk<LIM, T, 1>(role, a, fin, fout, bytes, x, lane, yb, ye, &ring);
}

// Strips, bands and rows per band of the pair kernel: the launch holds the
// fraction `frac` of the pairs the device holds at once.
#ifndef MARCH2_FRAC
#define MARCH2_FRAC 1.0
#endif
// Fewest rows per pair band for which a handle takes two steps per launch
// by default.  Measured: FP64 2-row bands are 10 % slower fused, 5-row
// bands 9 % faster, 80-row bands 28 %; FP32 5-row bands 2 % slower,
// 10-row bands 1 % faster, 19-row bands 4 %, 80-row bands 12 %.
#ifndef MARCH2_MIN_ROWS64
#define MARCH2_MIN_ROWS64 4
#endif
#ifndef MARCH2_MIN_ROWS32
#define MARCH2_MIN_ROWS32 8
#endif
inline void set_pair(StepArgs& a, long capacity_pairs, double frac)
{
    const int ex = a.x1 - a.x0, ey = a.y1 - a.y0;
    a.p_nsx = (ex + POUT - 1) / POUT;
    long nby = (long)(frac * (double)capacity_pairs) / (a.p_nsx > 0 ? a.p_nsx : 1);
    nby = std::max(1L, std::min(nby, (long)ey));
    a.p_rows = (int)((ey + nby - 1) / nby);
    if (a.p_rows < 1) a.p_rows = 1;
    a.p_nby = (ey + a.p_rows - 1) / a.p_rows;
    a.p_per_xcd = (a.p_nsx * a.p_nby + 7) / 8;
}

// The march addresses a state buffer with 31-bit byte offsets.
template <typename T>
inline bool march_fits(const StepArgs& a)
{
    return (double)a.elems * (double)sizeof(T) < 2147483648.0;
}

// Strips, bands and rows per band: as many bands as give the launch the
// fraction `frac` of the wavefronts the device holds at once
// (capacity_waves), but at least MRMIN rows per band unless the grid has
// fewer rows.
inline void set_march(StepArgs& a, long capacity_waves, double frac)
{
    const int ex = a.x1 - a.x0, ey = a.y1 - a.y0;
    a.m_nsx = (ex + MOUT - 1) / MOUT;
    long nby = (long)(frac * (double)capacity_waves) / (a.m_nsx > 0 ? a.m_nsx : 1);
    nby = std::max(1L, std::min(nby, (long)((ey + MRMIN - 1) / MRMIN)));
    a.m_rows = (int)((ey + nby - 1) / nby);
    if (a.m_rows < 1) a.m_rows = 1;
    a.m_nby = (ey + a.m_rows - 1) / a.m_rows;
    const int nblk = (a.m_nsx * a.m_nby + MWPB - 1) / MWPB;
    a.m_per_xcd = (nblk + 7) / 8;
}

}  // namespace
