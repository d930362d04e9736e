// mrtfd.hip -- C ABI (include/mrtfd.h) of the D2V16 MRT finite-difference
// lattice-Boltzmann step (arXiv:1305.4736): single-instance entry points.
//
// A time step is one pass of a fused step kernel (mrtfd_march.h: the
// row-marching form, one step per launch or, on large grids without walls
// along x, two steps per launch through an LDS ring of rows): each node's new
// populations come, from level n only, from its moments
// and macroscopic state (Sec. II), the velocity of its four axis neighbours
// (energy-flux correction, Sec. II), the equilibria (Appendix), the relaxed
// residual mapped back to velocity space (Sec. III update eq.), the limited x
// and y flux differences of its 16 populations (Sec. III flux and limiter
// eqs.) and the new populations.  The march reads periodic and outflow
// sides at their source nodes (the LDS-tile form for states of 2 GiB and
// more writes those ghost images instead); NEE walls along y are refilled
// by the march kernels themselves (by the wavefronts whose bands end at a
// wall, and between the two steps of a two-step launch in its ring of
// rows), other walls by a small kernel after the step; equilibrium ghosts
// are constant and written once.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mrtfd_host.h"
#include "mrtfd_march.h"

using namespace mrtfd;

std::string& mrtfd::error_buffer()
{
    thread_local std::string buf;
    return buf;
}


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
    StepArgs* args_dev;     // device copy of args (read by the row-marching step)
    bool ready;
    long steps;
    long march_capacity;    // wavefronts of the step kernel resident at once
    long pair_capacity;     // pairs of the two-step kernel resident at once
    int per_launch;         // steps per launch requested: 1, or 2 (fused pairs) where supported
    hipEvent_t ev0, ev1;
};

namespace {

void fill_args(mrtfd_s* h)
{
    const bool f32 = h->p.precision == MRTFD_FP32_STORAGE;
    h->args = make_args(h->p, h->L, h->blocks, h->blocks_dev, h->flag, f32 ? STEP_TXW32 : STEP_TXW64,
                        f32 ? STEP_BYR32 : STEP_BYR64, STEP_BAND);
    set_march(h->args, h->march_capacity, f32 ? MARCH_FRAC32 : MARCH_FRAC64);
    set_pair(h->args, h->pair_capacity, MARCH2_FRAC);
}

// Whether this instance can take two steps per launch: the march form
// (state below 2 GiB) and no walls along x (walls along y are refilled
// inside the pair, whose bands all walk up).
bool pair_supported(const mrtfd_s* h)
{
    const StepArgs& a = h->args;
    if (a.bc[0] == BC_WALL || a.bc[1] == BC_WALL) return false;
    if (MARCH2_ALTERNATE && (a.bc[2] == BC_WALL || a.bc[3] == BC_WALL)) return false;
    const bool fits = (h->p.precision == MRTFD_FP32_STORAGE) ? march_fits<float>(a) : march_fits<double>(a);
    return fits && a.x1 > a.x0 && a.y1 > a.y0;
}

template <typename T>
const void* pair_kernel(int limiter)
{
    switch (limiter) {
    case 0: return (const void*)k_march2<0, T>;
    case 1: return (const void*)k_march2<1, T>;
    case 2: return (const void*)k_march2<2, T>;
    default: return (const void*)k_march2<3, T>;
    }
}

template <typename T>
const void* march_kernel(int limiter)
{
    switch (limiter) {
    case 0: return (const void*)k_march<0, T>;
    case 1: return (const void*)k_march<1, T>;
    case 2: return (const void*)k_march<2, T>;
    default: return (const void*)k_march<3, T>;
    }
}

// Wavefronts of the step kernel that the device holds at once.
int query_march_capacity(mrtfd_s* h)
{
    const void* k = (h->p.precision == MRTFD_FP32_STORAGE) ? march_kernel<float>(h->p.limiter)
                                                            : march_kernel<double>(h->p.limiter);
    int dev = 0, cus = 0, nb = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, MW * MWPB, 0));
    h->march_capacity = (long)std::max(nb, 1) * MWPB * std::max(cus, 1);
    const void* k2 = (h->p.precision == MRTFD_FP32_STORAGE) ? pair_kernel<float>(h->p.limiter)
                                                             : pair_kernel<double>(h->p.limiter);
    nb = 0;
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k2, 2 * MW, 0));
    h->pair_capacity = (long)std::max(nb, 1) * std::max(cus, 1);
    return MRTFD_OK;
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

// Wall columns or rows and their ghosts of the new state fout, from the
// nodes next to the walls, after a launch that did not refill them: the
// LDS-tile form, and walls along x (the march kernels refill walls along y
// themselves).
template <typename T>
int refill_walls(mrtfd_s* h, T* fout, bool march)
{
    const StepArgs& a = h->args;
    for (int axis = 0; axis < 2; ++axis) {
        if (a.bc[2 * axis] != BC_WALL && a.bc[2 * axis + 1] != BC_WALL) continue;
        if (march && axis == 1) continue;
        const int n = 2 * ((axis == 0) ? a.ny : a.nx);
        hipLaunchKernelGGL((k_fill<T>), dim3((n + 127) / 128), dim3(128), 0, h->stream, fout, a, axis, 1);
        HIPCHK(hipGetLastError());
    }
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
        if (march_fits<T>(a)) {
            dim3 grid(8 * a.m_per_xcd), block(MW * MWPB);
            switch (h->p.limiter) {
            case 0: hipLaunchKernelGGL((k_march<0, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
            case 1: hipLaunchKernelGGL((k_march<1, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
            case 2: hipLaunchKernelGGL((k_march<2, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
            default: hipLaunchKernelGGL((k_march<3, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
            }
        } else {
            // state buffers of 2 GiB and more: the LDS-tile form
            constexpr int TXW = TileOf<T>::TXW, BYR = TileOf<T>::BYR;
            dim3 grid(8 * a.per_xcd), block(TXW * BYR);
            switch (h->p.limiter) {
            case 0: hipLaunchKernelGGL((k_step<0, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
            case 1: hipLaunchKernelGGL((k_step<1, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
            case 2: hipLaunchKernelGGL((k_step<2, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
            default: hipLaunchKernelGGL((k_step<3, T, TXW, BYR>), grid, block, 0, h->stream, fin, fout, a); break;
            }
        }
        HIPCHK(hipGetLastError());
        int rc = refill_walls<T>(h, fout, march_fits<T>(a));
        if (rc) return rc;
    }
    h->cur = 1 - h->cur;
    return MRTFD_OK;
}

int launch_step(mrtfd_s* h)
{
    return (h->p.precision == MRTFD_FP32_STORAGE) ? launch_step_t<float>(h) : launch_step_t<double>(h);
}

// Two steps in one launch (pair_supported(h) holds).
template <typename T>
int launch_pair_t(mrtfd_s* h)
{
    const StepArgs& a = h->args;
    const T* fin = (const T*)h->buf[h->cur];
    T* fout = (T*)h->buf[1 - h->cur];
    dim3 grid(8 * a.p_per_xcd), block(2 * MW);
    switch (h->p.limiter) {
    case 0: hipLaunchKernelGGL((k_march2<0, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
    case 1: hipLaunchKernelGGL((k_march2<1, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
    case 2: hipLaunchKernelGGL((k_march2<2, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
    default: hipLaunchKernelGGL((k_march2<3, T>), grid, block, 0, h->stream, fin, fout, h->args_dev); break;
    }
    HIPCHK(hipGetLastError());
    // (no walls along x; walls along y are refilled by the kernel)
    h->cur = 1 - h->cur;
    return MRTFD_OK;
}

int launch_pair(mrtfd_s* h)
{
    return (h->p.precision == MRTFD_FP32_STORAGE) ? launch_pair_t<float>(h) : launch_pair_t<double>(h);
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

// Diagnostics: the core clock a stretch of launches ran at.  Each block's
// first lane records its XCD's shader-clock counter and the device-wide
// constant 100 MHz counter in that XCD's pair of out[16] (the shader-clock
// counters of different XCDs are not aligned, so a clock is only measured
// between two stamps of the same XCD).  Launched with one block per XCD.
__global__ void k_clock_stamp(unsigned long long* out)
{
    if (threadIdx.x == 0) {
        const unsigned xcc = __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7;   // HW_REG_XCC_ID
        const unsigned long long t = __builtin_amdgcn_s_memtime();
        const unsigned long long r = __builtin_amdgcn_s_memrealtime();
        out[2 * xcc] = t;
        out[2 * xcc + 1] = r;
    }
}

// ---------------------------------------------------------------------------
// The no-allocation solve: the state of one solve lives in a file-scope
// device array instead of library allocations, for callers that cannot
// allocate.

constexpr size_t NOALLOC_BYTES = size_t(64) << 20;   // the array's size on every device
constexpr size_t NOALLOC_HEAD = 4096;                // blocks, arguments and flag before the state buffers
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

// Device address of `scratch` on each device, taken once per device with
// that device current (host code never uses the array's name as an address).
std::mutex g_scratch_mu;
std::vector<void*> g_scratch;

int scratch_address(void** out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(MRTFD_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return MRTFD_OK;
}

// Blocks, arguments and a cleared flag written into the array by a kernel
// (the values travel as kernel arguments; no copy from host memory).
__global__ void k_put_setup(Blocks b, StepArgs a, Blocks* bdst, StepArgs* adst, int* flag)
{
    if (threadIdx.x == 0) {
        *bdst = b;
        *adst = a;
        *flag = 0;
    }
}

// Zero `n` 8-byte words (the state buffers' padding is never read, but a
// solve then starts from the same bytes as one on fresh buffers).
__global__ void k_zero(unsigned long long* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}


}  // namespace

// ===========================================================================
extern "C" {

int mrtfd_clock_stamp(void* hip_stream, unsigned long long* out)
{
    if (!out) return fail(MRTFD_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_clock_stamp, dim3(8), dim3(64), 0, (hipStream_t)hip_stream, out);
    HIPCHK(hipGetLastError());
    return MRTFD_OK;
}

const char* mrtfd_last_error(void) { return error_buffer().c_str(); }

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
    // every failure below releases what was set up so far through
    // mrtfd_destroy (members start null; freeing null is a no-op)
    for (int k = 0; k < 2; ++k) {
        const hipError_t e = hipMalloc(&h->buf[k], h->L.buf_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->buf[k] = nullptr;
            mrtfd_destroy(h);
            return fail(MRTFD_ENOMEM, "cannot allocate 2 x %zu bytes of state (%s)", layout_of(*p).buf_bytes,
                        hipGetErrorString(e));
        }
    }
    if (!build_blocks(p->eta0, &h->blocks)) {
        mrtfd_destroy(h);
        return fail(MRTFD_EINVAL, "singular moment blocks for eta0 = %g", p->eta0);
    }
    if (hipMalloc(&h->flag, sizeof(int)) != hipSuccess || hipMalloc(&h->blocks_dev, sizeof(Blocks)) != hipSuccess ||
        hipMalloc(&h->args_dev, sizeof(StepArgs)) != hipSuccess ||
        hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
        (void)hipGetLastError();
        mrtfd_destroy(h);
        return fail(MRTFD_EDEVICE, "device set-up failed");
    }
    if (query_march_capacity(h) != MRTFD_OK) {
        mrtfd_destroy(h);
        return MRTFD_EDEVICE;
    }
    fill_args(h);
    // Default: fused pairs on grids whose pair bands are tall enough.  A
    // pair's band costs six more barrier iterations than rows, so short
    // bands (small grids, bound by the latency of the walk) are faster one
    // step per launch.
    const int min_rows = (h->p.precision == MRTFD_FP32_STORAGE) ? MARCH2_MIN_ROWS32 : MARCH2_MIN_ROWS64;
    h->per_launch = (pair_supported(h) && h->args.p_rows >= min_rows) ? 2 : 1;
    if (hipMemcpyAsync(h->blocks_dev, &h->blocks, sizeof(Blocks), hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(h->args_dev, &h->args, sizeof(StepArgs), hipMemcpyHostToDevice, h->stream) != hipSuccess) {
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
    (void)hipFree(h->args_dev);
    if (h->staging) (void)hipFree(h->staging);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
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
    long k = 0;
    if (h->per_launch == 2)
        for (; k + 2 <= nsteps; k += 2) {
            int rc = launch_pair(h);
            if (rc) return rc;
        }
    for (; k < nsteps; ++k) {
        int rc = launch_step(h);
        if (rc) return rc;
    }
    h->steps += nsteps;
    return MRTFD_OK;
}

int mrtfd_set_steps_per_launch(mrtfd_t h, int k)
{
    if (!h) return fail(MRTFD_EINVAL, "NULL handle");
    if (k != 1 && k != 2) return fail(MRTFD_EINVAL, "steps per launch must be 1 or 2, got %d", k);
    if (k == 2 && !pair_supported(h))
        return fail(MRTFD_EINVAL, "two steps per launch need no walls along x and a state below 2 GiB");
    h->per_launch = k;
    return MRTFD_OK;
}

int mrtfd_get_steps_per_launch(mrtfd_t h, int* k)
{
    if (!h || !k) return fail(MRTFD_EINVAL, "NULL argument");
    *k = h->per_launch;
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

int mrtfd_state_planes(mrtfd_t h, int* nplanes)
{
    if (!h || !nplanes) return fail(MRTFD_EINVAL, "NULL argument");
    *nplanes = (h->p.precision == MRTFD_FP32_STORAGE) ? NQ + 4 : NQ;
    return MRTFD_OK;
}

int mrtfd_get_state(mrtfd_t h, double* state, int on_device)
{
    if (!h || !state) return fail(MRTFD_EINVAL, "NULL argument");
    if (!h->ready) return fail(MRTFD_ESTATE, "mrtfd_get_state before mrtfd_init / mrtfd_set_f");
    const int np = (h->p.precision == MRTFD_FP32_STORAGE) ? NQ + 4 : NQ;
    const size_t n = (size_t)h->p.nx * h->p.ny;
    double* dst = state;
    if (!on_device) {
        int rc = ensure_staging(h, np * n * sizeof(double));
        if (rc) return rc;
        dst = h->staging;
    }
    dim3 grid = node_grid(h->p.nx, h->p.ny), block(BX, BY);
    if (h->p.precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_gather_state<float>), grid, block, 0, h->stream, (const float*)h->buf[h->cur], dst, h->args);
    else
        hipLaunchKernelGGL((k_gather_state<double>), grid, block, 0, h->stream, (const double*)h->buf[h->cur], dst, h->args);
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(state, h->staging, np * n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    return MRTFD_OK;
}

int mrtfd_set_state(mrtfd_t h, const double* state, int on_device)
{
    if (!h || !state) return fail(MRTFD_EINVAL, "NULL argument");
    const int np = (h->p.precision == MRTFD_FP32_STORAGE) ? NQ + 4 : NQ;
    const size_t n = (size_t)h->p.nx * h->p.ny;
    const double* src = state;
    if (!on_device) {
        int rc = ensure_staging(h, np * n * sizeof(double));
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(h->staging, state, np * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
        src = h->staging;
    }
    h->cur = 0;
    dim3 grid = node_grid(h->p.nx, h->p.ny), block(BX, BY);
    if (h->p.precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_scatter_state<float>), grid, block, 0, h->stream, (float*)h->buf[0], src, h->args);
    else
        hipLaunchKernelGGL((k_scatter_state<double>), grid, block, 0, h->stream, (double*)h->buf[0], src, h->args);
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

int mrtfd_device_memory(size_t* free_bytes, size_t* total_bytes)
{
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    if (free_bytes) *free_bytes = fr;
    if (total_bytes) *total_bytes = tot;
    return MRTFD_OK;
}

int mrtfd_solve_noalloc(const mrtfd_params* p, void* hip_stream, const double* rho, const double* ux,
                        const double* uy, const double* T, long nsteps, double* rho_out, double* ux_out,
                        double* uy_out, double* T_out)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!rho || !ux || !uy || !T) return fail(MRTFD_EINVAL, "NULL input field");
    if (nsteps < 0) return fail(MRTFD_EINVAL, "nsteps < 0");
#if MARCH2_MFMA
    return fail(MRTFD_EINVAL, "the no-allocation solve is not part of the matrix-core trial build");
#endif
    static_assert(MARCH2_MFMA || (sizeof(Blocks) <= 1024 && sizeof(StepArgs) <= 2048),
                  "set-up area of the array too small");
    const Layout L = layout_of(*p);
    const size_t buf = (L.buf_bytes + 255) / 256 * 256;
    if (NOALLOC_HEAD + 2 * buf > NOALLOC_BYTES)
        return fail(MRTFD_EINVAL, "grid %d x %d needs %zu bytes of state; the no-allocation solve holds %zu",
                    p->nx, p->ny, NOALLOC_HEAD + 2 * buf, NOALLOC_BYTES);
    void* base = nullptr;
    rc = scratch_address(&base);
    if (rc) return rc;
    // a handle on the host stack whose device state is the array
    mrtfd_s h{};
    h.p = *p;
    h.stream = (hipStream_t)hip_stream;
    h.L = L;
    char* b = (char*)base;
    h.blocks_dev = (Blocks*)b;
    h.args_dev = (StepArgs*)(b + 1024);
    h.flag = (int*)(b + 3072);
    h.buf[0] = b + NOALLOC_HEAD;
    h.buf[1] = b + NOALLOC_HEAD + buf;
    if (!build_blocks(p->eta0, &h.blocks)) return fail(MRTFD_EINVAL, "singular moment blocks for eta0 = %g", p->eta0);
    rc = query_march_capacity(&h);
    if (rc) return rc;
    fill_args(&h);
    const int min_rows = (p->precision == MRTFD_FP32_STORAGE) ? MARCH2_MIN_ROWS32 : MARCH2_MIN_ROWS64;
    h.per_launch = (pair_supported(&h) && h.args.p_rows >= min_rows) ? 2 : 1;
    // fresh state buffers, constants, arguments and flag, all by kernels
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, h.stream, (unsigned long long*)h.buf[0], 2 * buf / 8);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_put_setup, dim3(1), dim3(64), 0, h.stream, h.blocks, h.args, h.blocks_dev, h.args_dev, h.flag);
    HIPCHK(hipGetLastError());
    // f = f^eq of the fields, ghosts and walls, the steps, the outputs
    h.cur = 0;
    dim3 grid = node_grid(p->nx, p->ny), block(BX, BY);
    if (p->precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_init<float>), grid, block, 0, h.stream, (float*)h.buf[0], rho, ux, uy, T, h.args);
    else
        hipLaunchKernelGGL((k_init<double>), grid, block, 0, h.stream, (double*)h.buf[0], rho, ux, uy, T, h.args);
    HIPCHK(hipGetLastError());
    rc = refill(&h);
    if (rc) return rc;
    h.ready = true;
    rc = mrtfd_step(&h, nsteps);
    if (rc) return rc;
    if (rho_out || ux_out || uy_out || T_out) return mrtfd_macros(&h, rho_out, ux_out, uy_out, T_out, 1);
    return MRTFD_OK;
}

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
