// mrtfd_host.h -- host-side helpers shared by the entry points: error
// reporting, the padded state layout, parameter validation and the
// per-instance kernel arguments.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/mrtfd.h"
#include "mrtfd_consts.h"
#include "mrtfd_kernels.h"

namespace mrtfd {
// Message of the last failure on this thread (defined once, in mrtfd.hip).
std::string& error_buffer();

inline int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    error_buffer() = buf;
    return code;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(MRTFD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

// State layout: 16 planes of (ny + 4) padded rows, interleaved by row: the
// 16 rows (one per plane) of grid row y are adjacent (row stride 16 pitch,
// plane stride pitch).  FP32 storage follows each row with four FP64 planes
// of the conserved moments (rho, j_x, j_y, e) of its nodes, pitch doubles
// each, so a row holds 16 pitch floats and then 4 pitch doubles.  Kernels
// only use the strides and the origins.
struct Layout {
    size_t esize;
    long pitch;     // elements of one padded row of one plane
    long row;       // element stride between consecutive rows of a plane
    long plane;     // element stride between planes
    long org;       // element offset of node (0, 0) in plane 0
    long elems;     // elements of a buffer
    size_t buf_bytes;
    long corg, cpitch, cplane;   // FP32 storage: conserved planes, in doubles (0 otherwise)
};

inline Layout layout_of(const mrtfd_params& p)
{
    Layout L;
    const bool cons = p.precision == MRTFD_FP32_STORAGE;
    L.esize = cons ? 4 : 8;
    const long line = 128 / (long)L.esize;   // elements per 128-byte line
    const long xoff = line;                  // x = 0 starts a line; ghosts sit before it
    L.pitch = ((xoff + p.nx + HALO + line - 1) / line) * line;
    const long rows = (long)(p.ny + 2 * HALO);
    // a conserved plane's row (pitch doubles) is 2 pitch floats
    L.row = NQ * L.pitch + (cons ? 4 * 2 * L.pitch : 0);
    L.plane = L.pitch;
    L.org = (long)HALO * L.row + xoff;
    L.elems = rows * L.row;
    L.buf_bytes = (size_t)L.elems * L.esize;
    if (cons) {
        L.cpitch = L.row / 2;
        L.cplane = L.pitch;
        L.corg = (long)HALO * L.cpitch + NQ * L.pitch / 2 + 32;   // x = 0 at a 256-byte offset of its row
    } else {
        L.corg = L.cpitch = L.cplane = 0;
    }
    return L;
}

// Largest element offset inside one plane's addressing (kernels form the
// offset of a node within its plane in 32-bit integers).
inline long plane_span(const Layout& L) { return L.elems; }

inline int validate(const mrtfd_params* p)
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
    if (plane_span(L) >= (1L << 31))
        return fail(MRTFD_EINVAL, "grid %d x %d too large: node offsets must stay below 2^31 elements", p->nx, p->ny);
    return MRTFD_OK;
}

// Kernel arguments of one instance (blocks and flag are device pointers).
inline StepArgs make_args(const mrtfd_params& p, const Layout& L, const Blocks& hb, const Blocks* blocks_dev,
                          int* flag, int txw, int byr, int band)
{
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.Bp = blocks_dev;
    for (int k = 0; k < NQ; ++k) a.rdt[k] = -p.dt * p.s[k];
    a.b = p.b;
    a.inv_b = 1.0 / p.b;
    a.dt = p.dt;
    for (int g = 0; g < 4; ++g) {
        a.nux[g] = hb.vmag[g] * p.dt / p.dx;
        a.nuy[g] = hb.vmag[g] * p.dt / p.dy;
        a.cx[g] = 0.5 * (1.0 - a.nux[g]);
        a.cy[g] = 0.5 * (1.0 - a.nuy[g]);
        a.nux32[g] = (float)a.nux[g];
        a.nuy32[g] = (float)a.nuy[g];
        a.cx32[g] = (float)a.cx[g];
        a.cy32[g] = (float)a.cy[g];
        a.cxq[g] = 0.25 * a.cx[g];
        a.cyq[g] = 0.25 * a.cy[g];
        a.cx32h[g] = 0.5f * a.cx32[g];
        a.cy32h[g] = 0.5f * a.cy32[g];
    }
    a.correction = p.energy_flux_correction ? 1 : 0;
    a.c8dt = a.correction ? -p.dt * (p.s[7] / p.s[4] - 1.0) : 0.0;
    a.c9dt = a.correction ? -p.dt * (p.s[8] / p.s[4] - 1.0) : 0.0;
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
    a.pitch = L.row;
    a.plane = L.plane;
    a.org = L.org;
    a.elems = L.elems;
    a.corg = L.corg;
    a.cpitch = L.cpitch;
    a.cplane = L.cplane;
    a.x0 = (p.bc[0].kind == BC_WALL);
    a.x1 = p.nx - (p.bc[1].kind == BC_WALL);
    a.y0 = (p.bc[2].kind == BC_WALL);
    a.y1 = p.ny - (p.bc[3].kind == BC_WALL);
    a.ntx = (a.x1 - a.x0 + txw - 1) / txw;
    a.nty = (a.y1 - a.y0 + byr - 1) / byr;
    a.per_xcd = (a.ntx * a.nty + 7) / 8;
    a.band = band;
    a.flag = flag;
    return a;
}

}  // namespace mrtfd
