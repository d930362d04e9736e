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
    macro_of(a.B, a.inv_b, f1, r1, u1x, u1y, T1);
    const double* st = a.side[side];
    double rw = r1 * T1 / st[3];           // carry the pressure over: rho_w T_w = rho_1 T_1
    double ew[NQ], e1[NQ];
    feq_velocity(a.B, a.b, rw, st[1], st[2], st[3], ew);
    feq_velocity(a.B, a.b, r1, u1x, u1y, T1, e1);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        double fw = ew[i] + (f1[i] - e1[i]);
        f[i * a.plane + nw] = (T)fw;
        f[i * a.plane + nw + step] = (T)(2.0 * fw - f1[i]);
        f[i * a.plane + nw + 2 * step] = (T)(3.0 * fw - 2.0 * f1[i]);
    }
}

// ---------------------------------------------------------------------------
// The fused step.
template <int LIM, typename T>
__global__ void __launch_bounds__(BX * BY) k_step(const T* __restrict__ fin, T* __restrict__ fout, StepArgs a)
{
    using R = T;   // convection precision (FP64, or FP32 in FP32-storage mode)
    const int x = a.x0 + blockIdx.x * BX + threadIdx.x;
    const int y = a.y0 + blockIdx.y * BY + threadIdx.y;
    if (x >= a.x1 || y >= a.y1) return;
    const long n0 = node(a, x, y);

    T fT[NQ];
    double f[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        fT[i] = fin[i * a.plane + n0];
        f[i] = (double)fT[i];
    }

    // moments and macroscopic state
    double m[NQ];
    Sums sm = all_sums(f);
    moments(a.B, sm, m);
    const double rho = m[0];
    const double ir = 1.0 / rho;
    const double ux = m[1] * ir, uy = m[2] * ir;
    const double P = (m[3] - rho * (ux * ux + uy * uy)) * a.inv_b;
    if (!(rho > 0.0 && P > 0.0)) atomicOr(a.flag, 1);

    // relaxed residual of the non-conserved moments
    double eq[NQ];
    equilibria(rho, ux, uy, P, m[3], a.b, eq);
    double w[NQ];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = 0.0;
#pragma unroll
    for (int k = 4; k < NQ; ++k) w[k] = a.s[k] * (m[k] - eq[k]);

    if (a.correction) {
        // energy-flux correction: central differences of u at level n
        double g[NQ], uxw, uyw, uxe, uye, uxs, uys, uxn, uyn;
        load16(fin, a, n0 - 1, g);
        velocity_of(a.B, g, uxw, uyw);
        load16(fin, a, n0 + 1, g);
        velocity_of(a.B, g, uxe, uye);
        load16(fin, a, n0 - a.pitch, g);
        velocity_of(a.B, g, uxs, uys);
        load16(fin, a, n0 + a.pitch, g);
        velocity_of(a.B, g, uxn, uyn);
        const double dxux = (uxe - uxw) * a.inv2dx, dxuy = (uye - uyw) * a.inv2dx;
        const double dyux = (uxn - uxs) * a.inv2dy, dyuy = (uyn - uys) * a.inv2dy;
        const double div4b = 4.0 * a.inv_b * (dxux + dyuy);
        const double shear2 = 2.0 * (dxuy + dyux);
        w[7] += a.k8 * P * (ux * (4.0 * dxux - div4b) + uy * shear2);
        w[8] += a.k9 * P * (ux * shear2 + uy * (4.0 * dyuy - div4b));
    }
#pragma unroll
    for (int k = 4; k < NQ; ++k) w[k] *= -a.dt;
    double coll[NQ];
    inverse_nc(a.B, w, coll);

    // limited fluxes, x then y, and the update
    T fnew[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const long pi = i * a.plane + n0;
        const int g = i >> 2;
        R acc = R(0);
        if (sgx(i) != 0) {
            const long s = sgx(i);
            acc += conv1<LIM, R>(fin[pi - 2 * s], fin[pi - s], fT[i], fin[pi + s], (R)a.nux[g], (R)a.cx[g]);
        }
        if (sgy(i) != 0) {
            const long s = sgy(i) * a.pitch;
            acc += conv1<LIM, R>(fin[pi - 2 * s], fin[pi - s], fT[i], fin[pi + s], (R)a.nuy[g], (R)a.cy[g]);
        }
        fnew[i] = (T)(f[i] + (double)acc + coll[i]);
    }
    store16(fout, a, n0, fnew);

    // boundary images owned by this node
    if (a.bc[0] == BC_PERIODIC) {
        if (x < 2 || x >= a.nx - 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int xg = (q < 2) ? (q - 2) : (a.nx + q - 2);
                if ((((xg % a.nx) + a.nx) % a.nx) == x) store16(fout, a, n0 + (xg - x), fnew);
            }
        }
    } else {
        if (a.bc[0] == BC_OUTFLOW && x == 0) {
            store16(fout, a, n0 - 1, fnew);
            store16(fout, a, n0 - 2, fnew);
        }
        if (a.bc[1] == BC_OUTFLOW && x == a.nx - 1) {
            store16(fout, a, n0 + 1, fnew);
            store16(fout, a, n0 + 2, fnew);
        }
    }
    if (a.bc[2] == BC_PERIODIC) {
        if (y < 2 || y >= a.ny - 2) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int yg = (q < 2) ? (q - 2) : (a.ny + q - 2);
                if ((((yg % a.ny) + a.ny) % a.ny) == y) store16(fout, a, n0 + (long)(yg - y) * a.pitch, fnew);
            }
        }
    } else {
        if (a.bc[2] == BC_OUTFLOW && y == 0) {
            store16(fout, a, n0 - a.pitch, fnew);
            store16(fout, a, n0 - 2 * a.pitch, fnew);
        }
        if (a.bc[3] == BC_OUTFLOW && y == a.ny - 1) {
            store16(fout, a, n0 + a.pitch, fnew);
            store16(fout, a, n0 + 2 * a.pitch, fnew);
        }
    }
    const bool wy_lo = (a.bc[2] == BC_WALL && y == 1), wy_hi = (a.bc[3] == BC_WALL && y == a.ny - 2);
    const bool wx_lo = (a.bc[0] == BC_WALL && x == 1), wx_hi = (a.bc[1] == BC_WALL && x == a.nx - 2);
    if (wy_lo || wy_hi || wx_lo || wx_hi) {
        double fn[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) fn[i] = (double)fnew[i];
        if (wy_lo) wall_fill(a, fout, fn, 2, n0 - a.pitch, -a.pitch);
        if (wy_hi) wall_fill(a, fout, fn, 3, n0 + a.pitch, a.pitch);
        if (wx_lo) wall_fill(a, fout, fn, 0, n0 - 1, -1);
        if (wx_hi) wall_fill(a, fout, fn, 1, n0 + 1, 1);
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
    feq_velocity(a.B, a.b, rho[d], ux[d], uy[d], Tf[d], fe);
    const long n = node(a, x, y);
#pragma unroll
    for (int i = 0; i < NQ; ++i) f[i * a.plane + n] = (T)fe[i];
}

// Ghost fill of one axis from the interior (x-sides over rows, then y-sides
// over columns, two launches); used after init and set_f.
template <typename T>
__global__ void k_fill(T* __restrict__ f, StepArgs a, int axis)
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
    double v[NQ];
    if (kind == BC_WALL) {
        const int c1 = side_lo ? 1 : n - 2, cw = side_lo ? 0 : n - 1;
        load16(f, a, base + c1 * stride, v);
        wall_fill(a, f, v, side, base + cw * stride, side_lo ? -stride : stride);
        return;
    }
    if (kind == BC_EQUIL) {
        const double* st = a.side[side];
        feq_velocity(a.B, a.b, st[0], st[1], st[2], st[3], v);
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
    macro_of(a.B, a.inv_b, v, r, vx, vy, t);
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
    moments(a.B, sm, m);
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
    inverse_nc(a.B, dl, gq);
#pragma unroll
    for (int k = 0; k < NQ; ++k) ds[k] = 0.0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int g = i >> 2;
        const double cx = sgx(i) * a.B.vmag[g] - ux, cy = sgy(i) * a.B.vmag[g] - uy;
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
    build_blocks(p.eta0, &a.B);
    for (int k = 0; k < NQ; ++k) a.s[k] = p.s[k];
    a.b = p.b;
    a.inv_b = 1.0 / p.b;
    a.dt = p.dt;
    for (int g = 0; g < 4; ++g) {
        a.nux[g] = a.B.vmag[g] * p.dt / p.dx;
        a.nuy[g] = a.B.vmag[g] * p.dt / p.dy;
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
        dim3 grid = node_grid(ex, ey), block(BX, BY);
        switch (h->p.limiter) {
        case 0: hipLaunchKernelGGL((k_step<0, T>), grid, block, 0, h->stream, fin, fout, a); break;
        case 1: hipLaunchKernelGGL((k_step<1, T>), grid, block, 0, h->stream, fin, fout, a); break;
        case 2: hipLaunchKernelGGL((k_step<2, T>), grid, block, 0, h->stream, fin, fout, a); break;
        default: hipLaunchKernelGGL((k_step<3, T>), grid, block, 0, h->stream, fin, fout, a); break;
        }
        HIPCHK(hipGetLastError());
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
        hipLaunchKernelGGL((k_fill<T>), dim3((n + 127) / 128), dim3(128), 0, h->stream, f, h->args, axis);
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
    if (hipMalloc(&h->flag, sizeof(int)) != hipSuccess || hipEventCreate(&h->ev0) != hipSuccess ||
        hipEventCreate(&h->ev1) != hipSuccess) {
        (void)hipFree(h->buf[0]);
        (void)hipFree(h->buf[1]);
        delete h;
        return fail(MRTFD_EDEVICE, "device set-up failed");
    }
    fill_args(h);
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
