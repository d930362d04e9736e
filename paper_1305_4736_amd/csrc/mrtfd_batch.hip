// mrtfd_batch.hip -- batched entry points of the C ABI (include/mrtfd.h):
// many independent MRT-FD instances of different sizes, states and
// parameters advance together, one persistent launch per tile-shape class
// and step.
//
// Each occupied slot owns its parameters, its device state (two ping-pong
// buffers from the stream-ordered pool allocator) and a step budget.  The
// kernels find a slot's current buffer from the batch launch counter, so
// adding, finishing or removing a slot only rewrites that slot's descriptor
// and the work lists (stream-ordered copies), never the state of the others:
// a slot's result does not depend on which other slots share its launches.
//
// Shape classes: the row-marching strips of mrtfd_march.h (60 output
// columns x bands of up to 12 rows per wavefront), and LDS tiles of 256
// threads: 32 x 8, 64 x 4, 128 x 2, and 256 x 1 rows for one-row instances.
// Strip slots without walls along x and with at least 4 rows take two
// steps per launch (k_march2_batch, bands of 32 to 160 rows fitted to the
// load, items in a balanced order) in two-step
// rounds, which the batch runs while their work fills the device; the
// other slots, and such slots with one step left, then take one-step
// launches.
// Each slot gets the class with the smallest estimated cost (work units x
// cost per unit; a unit is a tile, or one row of a strip including the halo
// rows of its bands); mrtfd_batch_autotune measures the cost per unit of
// every class on calibration grids and reassigns.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <new>
#include <vector>

#include "mrtfd_host.h"
#include "mrtfd_march.h"

using namespace mrtfd;

// The batched strip kernels (they use the single-instance march's row
// walk and pair schedule).
namespace {

// Rows per band of a batched instance: short bands balance the static
// assignment of items to wavefronts over instances of mixed sizes (8-12
// rows measured best on a 512-instance mix; 32 rows cost 19 % more).
#ifndef MARCH_BROWS
#define MARCH_BROWS 12
#endif
constexpr int MBROWS = MARCH_BROWS;

// Band layout of a batched instance: bands of at most MBROWS rows.
inline void set_march_rows(StepArgs& a, int rows)
{
    const int ex = a.x1 - a.x0, ey = a.y1 - a.y0;
    a.m_nsx = (ex + MOUT - 1) / MOUT;
    a.m_rows = std::max(1, std::min(rows, ey));
    a.m_nby = (ey + a.m_rows - 1) / a.m_rows;
    a.m_per_xcd = 0;
}

// Batched form: persistent wavefronts stride over the (band, strip) items
// of the listed slots, numbered slot after slot (prefix[k] = first item of
// list[k]); wavefront g of the launch takes items g, g + G, ... where the
// wavefronts of each XCD are numbered contiguously (the grid is a multiple
// of 8 blocks).  The step and round counters L and R decide each slot's
// current buffer and whether it still steps, as in the tile form.
template <int LIM, typename T>
__global__ void __launch_bounds__(MW * MWPB) k_march_batch(const BatchSlot* __restrict__ slots,
                                                          const int* __restrict__ prefix,
                                                          const int* __restrict__ list, int nlist, long L, long R)
{
    convect_mode();
    const MRTFD_CONSTANT BatchSlot* cs = (const MRTFD_CONSTANT BatchSlot*)slots;
    const MRTFD_CONSTANT int* cpre = (const MRTFD_CONSTANT int*)prefix;
    const MRTFD_CONSTANT int* clist = (const MRTFD_CONSTANT int*)list;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / MW)), lane = threadIdx.x % MW;
    const int nb = gridDim.x, bid = blockIdx.x;
    const int g = ((bid & 7) * (nb >> 3) + (bid >> 3)) * MWPB + w;
    const int G = nb * MWPB;
    const int nitems = cpre[nlist];
    for (int item = g; item < nitems; item += G) {
        int lo = 0, hi = nlist;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cpre[mid] <= item) lo = mid;
            else hi = mid;
        }
        const MRTFD_CONSTANT BatchSlot& sl = cs[clist[lo]];
        if (L >= sl.stop) continue;
        CArgs& a = sl.a;
        const int par = (int)(((sl.pair ? R : L) - sl.pstart) & 1);
        const T* fin = (const T*)sl.buf[par];
        T* fout = (T*)sl.buf[par ^ 1];
        const int r = item - cpre[lo];
        const int band = r / a.m_nsx, strip = r - band * a.m_nsx;
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
}

}  // namespace

namespace {

// Rows per pair band of a batched instance (the shortest of the heights
// fit_pair_rows chooses from), and the fewest rows an instance needs to take
// two steps per launch in the batch.  With items dealt out in slot order, by
// a stride, 32 / 8 beat bands of 16, 24, 48 and 64 rows and minimums of 1,
// 4, 16 and 32 by 1-7 % on the 512-instance Riemann mix; with the balanced
// order and fitted heights a minimum of 4 rows is 3 % faster than 8 on the
// same mix (0.784 against 0.808 ms per step, same box, three runs each; 2
// rows 0.788).
#ifndef MARCH2_BROWS
#define MARCH2_BROWS 32
#endif
#ifndef MARCH2_BATCH_MIN_ROWS
#define MARCH2_BATCH_MIN_ROWS 4
#endif
constexpr int MBROWS2 = MARCH2_BROWS;

// Pair-band layout of a batched instance: bands of at most MBROWS2 rows.
inline void set_pair_rows(StepArgs& a, int rows)
{
    const int ex = a.x1 - a.x0, ey = a.y1 - a.y0;
    a.p_nsx = (ex + POUT - 1) / POUT;
    a.p_rows = std::max(1, std::min(rows, ey));
    a.p_nby = (ey + a.p_rows - 1) / a.p_rows;
    a.p_per_xcd = 0;
}

// Batched two-step form: persistent blocks (one pair each) take the
// (band, strip) items of the listed pair slots.  The list holds runs of
// bands of one slot (list[e] the slot, band[e] its first band, prefix[e]
// the run's first item), ordered by band height, tallest first (the host's
// order, rebuild_lists); item i of a run is band band[e] + i / strips,
// strip i % strips.  Block g (numbered XCD-aware as in k_march_batch) takes
// item g of each pass of nb items on even passes and item nb - 1 - g on
// odd ones, so that the shorter items at the end even out the blocks'
// totals.  Every listed slot has two steps left (the caller's rule), and
// its current buffer is the parity of R.  Both wavefronts of a block take
// the same items, so they pass the same number of barriers.
template <int LIM, typename T>
__global__ void __launch_bounds__(2 * MW, MARCH2_MINW) k_march2_batch(const BatchSlot* __restrict__ slots,
                                                                  const int* __restrict__ prefix,
                                                                  const int* __restrict__ list,
                                                                  const int* __restrict__ band0, int nlist, long L,
                                                                  long R)
{
    __shared__ PairRing<T> ring;
    convect_mode();
    const MRTFD_CONSTANT BatchSlot* cs = (const MRTFD_CONSTANT BatchSlot*)slots;
    const MRTFD_CONSTANT int* cpre = (const MRTFD_CONSTANT int*)prefix;
    const MRTFD_CONSTANT int* clist = (const MRTFD_CONSTANT int*)list;
    const MRTFD_CONSTANT int* cband = (const MRTFD_CONSTANT int*)band0;
    const int role = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / MW)), lane = threadIdx.x % MW;
    const int nb = gridDim.x, bid = blockIdx.x;
    const int g = (bid & 7) * (nb >> 3) + (bid >> 3);
    const int nitems = cpre[nlist];
    int odd = 0;
    for (int base = 0; base < nitems; base += nb, odd ^= 1) {
        const int item = base + (odd ? nb - 1 - g : g);
        if (item >= nitems) continue;
        int lo = 0, hi = nlist;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (cpre[mid] <= item) lo = mid;
            else hi = mid;
        }
        const MRTFD_CONSTANT BatchSlot& sl = cs[clist[lo]];
        if (L + 1 >= sl.stop) continue;      // (not listed by the caller) both wavefronts skip
        CArgs& a = sl.a;
        const int par = (int)((R - sl.pstart) & 1);
        const T* fin = (const T*)sl.buf[par];
        T* fout = (T*)sl.buf[par ^ 1];
        const int r = item - cpre[lo];
        const int rb = r / a.p_nsx, strip = r - rb * a.p_nsx;
        const int band = cband[lo] + rb;
        const int x = a.x0 + strip * POUT - 4 + lane;
        const int yb = a.y0 + band * a.p_rows, ye = min(yb + a.p_rows, a.y1);
        const unsigned bytes = (unsigned)(a.elems * (long)sizeof(T));
        pair_walk<LIM, T, 1>(role, a, fin, fout, bytes, x, lane, yb, ye, &ring);
    }
}

}  // namespace

namespace {

constexpr int NSHAPE = 5;
constexpr int MARCH = 4;   // index of the row-marching class
// work lists: one per class, then the strip slots split into those that
// take two steps per launch in two-step rounds and the others
constexpr int LIST_PAIR = NSHAPE, LIST_SINGLE = NSHAPE + 1, NLIST = NSHAPE + 2;
struct ShapeDef {
    int txw, byr;
    bool flat;
};
constexpr ShapeDef SHAPES[NSHAPE] = {{32, 8, false}, {64, 4, false}, {128, 2, false}, {256, 1, true}, {MOUT, MBROWS, false}};
// Cost per work unit before autotuning (microseconds, measured on the
// 4096 x 1024 shock-interface grid in FP32 storage; only the ratios matter).
constexpr double DEFAULT_COST[NSHAPE] = {0.028, 0.028, 0.029, 0.045, 0.0019};

bool shape_fits(const mrtfd_params& p, int s)
{
    if (s == MARCH) {
        const Layout L = layout_of(p);
        return (double)L.buf_bytes < 2147483648.0;
    }
    if (!SHAPES[s].flat) return true;
    // one row whose y ghosts copy the row
    return p.ny == 1 && (p.bc[2].kind == BC_PERIODIC || p.bc[2].kind == BC_OUTFLOW) &&
           (p.bc[3].kind == BC_PERIODIC || p.bc[3].kind == BC_OUTFLOW);
}

// Work units of an instance in class s (tiles; for strips, strip rows
// including the four halo rows each band loads).
long tiles_of(const mrtfd_params& p, int s)
{
    const int ex = p.nx - (p.bc[0].kind == BC_WALL) - (p.bc[1].kind == BC_WALL);
    const int ey = p.ny - (p.bc[2].kind == BC_WALL) - (p.bc[3].kind == BC_WALL);
    if (s == MARCH) {
        const long nby = (ey + MBROWS - 1) / MBROWS;
        return (long)((ex + MOUT - 1) / MOUT) * (ey + 4 * nby);
    }
    return (long)((ex + SHAPES[s].txw - 1) / SHAPES[s].txw) * ((ey + SHAPES[s].byr - 1) / SHAPES[s].byr);
}

// Work items of one launch for a slot in work list s.
long items_of(const StepArgs& a, int s)
{
    if (s == LIST_PAIR) return (long)a.p_nsx * a.p_nby;
    return (s == MARCH || s == LIST_SINGLE) ? (long)a.m_nsx * a.m_nby : (long)a.ntx * a.nty;
}

}  // namespace

struct mrtfd_batch_s {
    int capacity, precision, limiter;
    hipStream_t stream;
    std::vector<BatchSlot> slot;        // host mirror of the device descriptors
    std::vector<mrtfd_params> prm;
    std::vector<Layout> lay;
    std::vector<Blocks> blk;
    std::vector<int> used, shape;
    BatchSlot* d_slot;
    Blocks* d_blocks;
    int* d_flags;
    int* d_lists;                       // NLIST x (capacity + 1) prefixes, then NLIST x capacity slot lists, then
                                        // capacity walls, then the two-step list: 2 capacity + 1 prefixes,
                                        // 2 capacity slots, 2 capacity first bands
    int nlist[NLIST], nwall;
    bool dirty;
    long L;                             // steps taken by the batch
    long R;                             // rounds (one or two steps each)
    long rounds1, rounds2;              // one-step and two-step rounds run (diagnostics)
    int mrows;                          // band height of the strip slots' one-step launches
    int prows;                          // band height of the strip slots' two-step launches
    bool fit_rows;                      // fit mrows to the load (off for calibration batches)
    std::vector<long> rstop;            // R at which a pair slot stopped stepping (LONG_MAX while it steps)
    int per_launch;                     // 2: two-step rounds where possible; 1: one step per round
    double cost[NSHAPE];                // device microseconds per work unit of each class
    double launch_us[NSHAPE];           // device microseconds of one launch of a class, beside its work
    double* staging;
    size_t staging_bytes;
    hipEvent_t ev0, ev1;
    // a second stream (default priority) for the one-step launches of a
    // two-step round, which overlap the pair launch (they step other slots)
    hipStream_t side;
    hipEvent_t fork, join;
    int max_blocks;
    int march_blocks;                   // resident blocks of the strip kernel on the device
    int pair_blocks;                    // resident blocks (pairs) of the two-step strip kernel
    long pair_items;                    // work items (pair bands x strips) of the two-step list
};

namespace {

int* prefix_dev(mrtfd_batch_s* B, int s) { return B->d_lists + s * (B->capacity + 1); }
int* list_dev(mrtfd_batch_s* B, int s) { return B->d_lists + NLIST * (B->capacity + 1) + s * B->capacity; }
int* wall_dev(mrtfd_batch_s* B) { return B->d_lists + NLIST * (B->capacity + 1) + NLIST * B->capacity; }
// the two-step list: up to two runs per slot (its full bands, its shorter last band)
size_t pair_region_ints(int capacity) { return 3 * (size_t)(2 * capacity) + 1; }
int* pair_prefix_dev(mrtfd_batch_s* B) { return wall_dev(B) + B->capacity; }
int* pair_list_dev(mrtfd_batch_s* B) { return pair_prefix_dev(B) + 2 * B->capacity + 1; }
int* pair_band_dev(mrtfd_batch_s* B) { return pair_list_dev(B) + 2 * B->capacity; }

int check_slot(mrtfd_batch_s* B, int k)
{
    if (!B) return fail(MRTFD_EINVAL, "NULL batch");
    if (k < 0 || k >= B->capacity || !B->used[k]) return fail(MRTFD_EINVAL, "slot %d is not occupied", k);
    return MRTFD_OK;
}

// Occupied slots in class s.
int members(const mrtfd_batch_s* B, int s)
{
    int n = 0;
    for (int k = 0; k < B->capacity; ++k) n += (B->used[k] && B->shape[k] == s);
    return n;
}

// Class of a new slot: the smallest estimated device time per step, where a
// class with no slot yet also pays for its launch.
int pick_shape(const mrtfd_batch_s* B, const mrtfd_params& p)
{
    int best = 0;
    double best_cost = 1e300;
    for (int s = 0; s < NSHAPE; ++s) {
        if (!shape_fits(p, s)) continue;
        const double c = (double)tiles_of(p, s) * B->cost[s] + (members(B, s) ? 0.0 : B->launch_us[s]);
        if (c < best_cost) {
            best_cost = c;
            best = s;
        }
    }
    return best;
}

// Whether slot k takes two steps per launch in two-step rounds: a strip
// slot without walls along x and with at least MARCH2_BATCH_MIN_ROWS rows
// (the batched pairs walk up, so walls along y are refilled inside them).
bool pair_capable(const mrtfd_batch_s* B, int k)
{
    if (B->per_launch != 2 || B->shape[k] != MARCH) return false;
    const mrtfd_params& p = B->prm[k];
    if (p.bc[0].kind == BC_WALL || p.bc[1].kind == BC_WALL) return false;
    return p.ny >= MARCH2_BATCH_MIN_ROWS;
}

// Buffer holding the slot's current state: the parity of its clock (R for
// pair slots, frozen where they stopped; L for the others, frozen at stop).
int current_buffer(const mrtfd_batch_s* B, int k)
{
    const BatchSlot& sl = B->slot[k];
    const long c = sl.pair ? std::min(B->R, B->rstop[k]) : std::min(B->L, sl.stop);
    return (int)(((c - sl.pstart) % 2 + 2) % 2);
}

// Restart slot k's clock so that buffer `cur` is current under its rule.
void rebase(mrtfd_batch_s* B, int k, int cur)
{
    BatchSlot& sl = B->slot[k];
    B->rstop[k] = (B->L >= sl.stop) ? B->R : LONG_MAX;
    const long c = sl.pair ? B->R : std::min(B->L, sl.stop);
    sl.pstart = c - cur;
}

// Arguments and pair flag of slot k for its class (the caller rebases).
void set_args(mrtfd_batch_s* B, int k)
{
    const int s = B->shape[k];
    const ShapeDef& sd = SHAPES[s == MARCH ? 0 : s];
    B->slot[k].a = make_args(B->prm[k], B->lay[k], B->blk[k], B->d_blocks + k, B->d_flags + k, sd.txw, sd.byr, 1 << 20);
    set_march_rows(B->slot[k].a, B->mrows);
    set_pair_rows(B->slot[k].a, B->prows);
    B->slot[k].pair = pair_capable(B, k) ? 1 : 0;
}

int upload_slot(mrtfd_batch_s* B, int k)
{
    HIPCHK(hipMemcpyAsync(B->d_slot + k, &B->slot[k], sizeof(BatchSlot), hipMemcpyHostToDevice, B->stream));
    return MRTFD_OK;
}

// Whether slot k takes two steps per launch in the next two-step round: a
// pair slot with two steps left.  A pair slot with one step left takes a
// one-step launch in that round instead (its clock, R, still advances by one).
bool takes_pair(const mrtfd_batch_s* B, int k)
{
    return B->slot[k].pair && B->slot[k].stop - B->L >= 2;
}

// Whether slot k is in work list s (slots that still step).
bool in_list(const mrtfd_batch_s* B, int k, int s)
{
    if (!B->used[k] || B->L >= B->slot[k].stop) return false;
    const int cls = (s == LIST_PAIR || s == LIST_SINGLE) ? MARCH : s;
    if (B->shape[k] != cls) return false;
    if (s == LIST_PAIR) return takes_pair(B, k);
    if (s == LIST_SINGLE) return !takes_pair(B, k);
    return true;
}

// Band height of the strip slots' one-step launches: the tallest of 12, 6,
// 3, 2 and 1 rows whose work items fill the resident wavefronts.  A batch
// too light to fill the device is bound by the rows each wavefront walks
// (its four window rows plus the band), so it gets shorter bands; heavy
// batches keep 12.  Bands grow back only once the taller level fills the
// device 1.5 times over, so a load near a threshold does not flip levels;
// a change re-uploads the descriptors of the occupied slots in one copy.
int fit_march_rows(mrtfd_batch_s* B)
{
    if (!B->fit_rows) return MRTFD_OK;
    const long cap = (long)B->march_blocks * MWPB;
    const int levels[] = {MBROWS, MBROWS / 2, MBROWS / 4, 2, 1};
    int r = 1;
    for (int lv : levels) {
        if (lv < 1) continue;
        long items = 0;
        for (int k = 0; k < B->capacity; ++k) {
            if (!B->used[k] || B->L >= B->slot[k].stop || B->shape[k] != MARCH) continue;
            const StepArgs& a = B->slot[k].a;
            items += (long)a.m_nsx * ((a.y1 - a.y0 + lv - 1) / lv);
        }
        const long need = (lv > B->mrows) ? cap + cap / 2 : cap;
        if (items >= need) {
            r = lv;
            break;
        }
    }
    if (r == B->mrows) return MRTFD_OK;
    B->mrows = r;
    int k0 = B->capacity, k1 = -1;
    for (int k = 0; k < B->capacity; ++k) {
        if (!B->used[k]) continue;
        k0 = std::min(k0, k);
        k1 = k;
        if (B->shape[k] == MARCH) set_march_rows(B->slot[k].a, r);
    }
    if (k1 >= k0)
        HIPCHK(hipMemcpyAsync(B->d_slot + k0, &B->slot[k0], (size_t)(k1 - k0 + 1) * sizeof(BatchSlot),
                              hipMemcpyHostToDevice, B->stream));
    return MRTFD_OK;
}

// Band height of the two-step launches: the tallest of 160, 128, 96, 80,
// 64, 48 and 32 rows that still gives the resident pairs PAIR_ITEMS_PER_PAIR
// items each, so that the balanced order (rebuild_lists) evens them out.
// Taller bands walk fewer halo rows per output row, and a light batch keeps
// 32-row bands, whose launches are shortest.  Growing takes 1.25 times the
// items, so a load near a threshold does not flip heights; a change
// re-uploads the descriptors of the occupied slots in one copy.  Measured
// on the 512-instance Riemann mix (FP32 storage, ms per step, fixed
// heights): 24 rows 0.917, 32 0.890, 40 0.856, 48 0.838, 56 0.840, 64
// 0.827, 80 0.805, 112 0.815, 160 0.796, 256 0.828 (10, 7.7 and 6.7 items
// per pair at 80, 160 and 256 rows); on 20 s of the served stream, fixed
// 80-row bands against 32 raised the overloaded stream's achieved rate
// from 3.00e10 to 3.27e10 node-updates/s but the median latency at 25 and
// 15 requests/s from 0.63 to 0.95 s and from 0.14 to 0.26 s.
#ifndef PAIR_ITEMS_PER_PAIR
#define PAIR_ITEMS_PER_PAIR 8
#endif
int fit_pair_rows(mrtfd_batch_s* B)
{
    if (!B->fit_rows) return MRTFD_OK;
    const long need = (long)PAIR_ITEMS_PER_PAIR * B->pair_blocks;
    const int levels[] = {5 * MBROWS2, 4 * MBROWS2, 3 * MBROWS2, 5 * MBROWS2 / 2, 2 * MBROWS2, 3 * MBROWS2 / 2};
    int r = MBROWS2;
    for (int lv : levels) {
        long items = 0;
        for (int k = 0; k < B->capacity; ++k) {
            if (!in_list(B, k, LIST_PAIR)) continue;
            const StepArgs& a = B->slot[k].a;
            items += (long)a.p_nsx * ((a.y1 - a.y0 + lv - 1) / lv);
        }
        if (items >= ((lv > B->prows) ? need + need / 4 : need)) {
            r = lv;
            break;
        }
    }
    if (r == B->prows) return MRTFD_OK;
    B->prows = r;
    int k0 = B->capacity, k1 = -1;
    for (int k = 0; k < B->capacity; ++k) {
        if (!B->used[k]) continue;
        k0 = std::min(k0, k);
        k1 = k;
        if (B->shape[k] == MARCH) set_pair_rows(B->slot[k].a, r);
    }
    if (k1 >= k0)
        HIPCHK(hipMemcpyAsync(B->d_slot + k0, &B->slot[k0], (size_t)(k1 - k0 + 1) * sizeof(BatchSlot),
                              hipMemcpyHostToDevice, B->stream));
    return MRTFD_OK;
}

// Rebuild the work lists over slots that still step.
int rebuild_lists(mrtfd_batch_s* B)
{
    int rc = fit_march_rows(B);
    if (rc) return rc;
    rc = fit_pair_rows(B);
    if (rc) return rc;
    const size_t base = NLIST * (B->capacity + 1) + NLIST * B->capacity + B->capacity;
    std::vector<int> host(base + pair_region_ints(B->capacity), 0);
    B->nwall = 0;
    for (int s = 0; s < NLIST; ++s) {
        if (s == LIST_PAIR) continue;
        int n = 0, acc = 0;
        int* pre = host.data() + s * (B->capacity + 1);
        int* lst = host.data() + NLIST * (B->capacity + 1) + s * B->capacity;
        for (int k = 0; k < B->capacity; ++k) {
            if (!in_list(B, k, s)) continue;
            pre[n] = acc;
            lst[n] = k;
            acc += (int)items_of(B->slot[k].a, s);
            ++n;
        }
        pre[n] = acc;
        B->nlist[s] = n;
    }
    // The two-step list, ordered so that the persistent pairs' totals even
    // out: each slot's bands of the full height as one run and its shorter
    // last band as another, the runs sorted by band height, tallest first
    // (stable, so a slot's runs keep slot order among equals).  With the
    // snake order in which k_march2_batch deals the items out, the pairs'
    // totals differ by little more than the shortest items.  (Items dealt
    // out in slot order, by a stride, left the most loaded pair about 16 %
    // above the mean on the 512-instance Riemann mix, by a count of barrier
    // iterations per item.)
    {
        struct Run {
            int k, band0, nbands, height;
        };
        std::vector<Run> runs;
        for (int k = 0; k < B->capacity; ++k) {
            if (!in_list(B, k, LIST_PAIR)) continue;
            const StepArgs& a = B->slot[k].a;
            const int ey = a.y1 - a.y0, nfull = ey / a.p_rows, rest = ey - nfull * a.p_rows;
            if (nfull > 0) runs.push_back({k, 0, nfull, a.p_rows});
            if (rest > 0) runs.push_back({k, nfull, 1, rest});
        }
        std::stable_sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) { return x.height > y.height; });
        int* pre = host.data() + base;
        int* lst = pre + 2 * B->capacity + 1;
        int* bnd = lst + 2 * B->capacity;
        long acc = 0;
        int n = 0;
        for (const Run& r : runs) {
            pre[n] = (int)acc;
            lst[n] = r.k;
            bnd[n] = r.band0;
            acc += (long)B->slot[r.k].a.p_nsx * r.nbands;
            ++n;
        }
        pre[n] = (int)acc;
        B->nlist[LIST_PAIR] = n;
        B->pair_items = acc;
    }
    // slots whose walls a refill launch rewrites after each step: walls in
    // the tile classes, and walls along x (the strip kernels refill walls
    // along y themselves; strip slots with walls along x never take pairs)
    int* wl = host.data() + NLIST * (B->capacity + 1) + NLIST * B->capacity;
    for (int k = 0; k < B->capacity; ++k) {
        if (!B->used[k] || B->L >= B->slot[k].stop) continue;
        const mrtfd_params& p = B->prm[k];
        const bool wx = p.bc[0].kind == BC_WALL || p.bc[1].kind == BC_WALL;
        const bool wy = p.bc[2].kind == BC_WALL || p.bc[3].kind == BC_WALL;
        if (wx || (wy && B->shape[k] != MARCH)) wl[B->nwall++] = k;
    }
    HIPCHK(hipMemcpyAsync(B->d_lists, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice, B->stream));
    B->dirty = false;
    return MRTFD_OK;
}

// One launch over work list s at step counter L on stream st.
template <int LIM, typename T>
int launch_list(mrtfd_batch_s* B, int s, long items, long L, hipStream_t st)
{
    const int* pre = prefix_dev(B, s);
    const int* lst = list_dev(B, s);
    const int n = B->nlist[s];
    if (s == LIST_PAIR) {
        // persistent pairs, a multiple of 8 blocks for the XCD-aware numbering
        long blocks = std::min<long>(items, B->pair_blocks);
        blocks = (blocks + 7) / 8 * 8;
        hipLaunchKernelGGL((k_march2_batch<LIM, T>), dim3((int)blocks), dim3(2 * MW), 0, st, B->d_slot,
                           pair_prefix_dev(B), pair_list_dev(B), pair_band_dev(B), n, L, B->R);
        HIPCHK(hipGetLastError());
        return MRTFD_OK;
    }
    if (s == MARCH || s == LIST_SINGLE) {
        // persistent wavefronts; the XCD-aware numbering needs a multiple of 8 blocks
        long blocks = std::min<long>((items + MWPB - 1) / MWPB, B->march_blocks);
        blocks = (blocks + 7) / 8 * 8;
        hipLaunchKernelGGL((k_march_batch<LIM, T>), dim3((int)blocks), dim3(MW * MWPB), 0, st, B->d_slot, pre,
                           lst, n, L, B->R);
        HIPCHK(hipGetLastError());
        return MRTFD_OK;
    }
    const int grid = (int)std::min<long>(items, B->max_blocks);
    switch (s) {
    case 0: hipLaunchKernelGGL((k_step_batch<LIM, T, 32, 8, false>), dim3(grid), dim3(256), 0, st, B->d_slot, pre, lst, n, L); break;
    case 1: hipLaunchKernelGGL((k_step_batch<LIM, T, 64, 4, false>), dim3(grid), dim3(256), 0, st, B->d_slot, pre, lst, n, L); break;
    case 2: hipLaunchKernelGGL((k_step_batch<LIM, T, 128, 2, false>), dim3(grid), dim3(256), 0, st, B->d_slot, pre, lst, n, L); break;
    default: hipLaunchKernelGGL((k_step_batch<LIM, T, 256, 1, true>), dim3(grid), dim3(256), 0, st, B->d_slot, pre, lst, n, L); break;
    }
    HIPCHK(hipGetLastError());
    return MRTFD_OK;
}

// Launches over work lists `lists` at step counter L on stream st, then the
// refill launch for the walls the kernels leave (refill = true).
template <typename T>
int launch_lists(mrtfd_batch_s* B, const int* lists, int nl, long L, bool refill, hipStream_t st)
{
    for (int q = 0; q < nl; ++q) {
        const int s = lists[q];
        if (!B->nlist[s]) continue;
        long items = 0;
        for (int k = 0; k < B->capacity; ++k)
            if (in_list(B, k, s)) items += items_of(B->slot[k].a, s);
        int rc = 0;
        switch (B->limiter) {
        case 0: rc = launch_list<0, T>(B, s, items, L, st); break;
        case 1: rc = launch_list<1, T>(B, s, items, L, st); break;
        case 2: rc = launch_list<2, T>(B, s, items, L, st); break;
        default: rc = launch_list<3, T>(B, s, items, L, st); break;
        }
        if (rc) return rc;
    }
    if (refill && B->nwall) {
        hipLaunchKernelGGL((k_wall_batch<T>), dim3(B->nwall), dim3(256), 0, st, B->d_slot, wall_dev(B), L, B->R);
        HIPCHK(hipGetLastError());
    }
    return MRTFD_OK;
}

// Whether the next round can take two steps: some slot takes two steps per
// launch (a pair slot with two steps left; the lists are current) and the
// two-step launch fills the device.  (A pair band's 32 rows take 38
// barrier-bound iterations for two steps, against about 26 rows walked by
// two one-step launches of 12-row bands, so a batch far too small to fill
// the device is faster one step at a time.)
// Two-step work items a two-step round needs, in multiples of the resident
// pairs.  Measured on the served stream at 15 requests/s, median / 99th
// percentile latency (two runs each): 0.264 / 0.86 s with 1, 0.28-0.31 /
// 0.93-0.96 s with 2, 0.28-0.29 / 0.96-0.98 s with 4, 0.336 / 0.76 s with
// 0 (two-step rounds whenever a slot takes pairs), 0.29 / 0.98 s without
// two-step rounds; the overloaded stream achieves 2.7-2.8e10 node-updates/s
// with any of them and 1.76e10 without.
#ifndef MARCH2_BATCH_FILL
#define MARCH2_BATCH_FILL 1
#endif
bool two_step_round_ok(const mrtfd_batch_s* B)
{
    return B->per_launch == 2 && B->nlist[LIST_PAIR] > 0 &&
           B->pair_items >= (long)MARCH2_BATCH_FILL * B->pair_blocks;
}

// One round: one step of every stepping slot, or (two = true) two steps,
// the pair slots in one launch and the others in two one-step launches.
template <typename T>
int launch_round_t(mrtfd_batch_s* B, bool two)
{
    if (B->dirty) {
        int rc = rebuild_lists(B);
        if (rc) return rc;
    }
    const long L0 = B->L;
    if (two) {
        // the other slots' two one-step launches run on the side stream,
        // beside the pair launch (forked after the list upload, joined back
        // before anything else on the batch's stream)
        const int others[] = {0, 1, 2, 3, LIST_SINGLE};
        bool any = B->nwall > 0;
        for (int s : others) any = any || B->nlist[s] > 0;
        if (any) {
            HIPCHK(hipEventRecord(B->fork, B->stream));
            HIPCHK(hipStreamWaitEvent(B->side, B->fork, 0));
            for (int h = 0; h < 2; ++h) {
                int rc = launch_lists<T>(B, others, 5, L0 + h, true, B->side);
                if (rc) return rc;
            }
            HIPCHK(hipEventRecord(B->join, B->side));
        }
        const int pairs[] = {LIST_PAIR};
        int rc = launch_lists<T>(B, pairs, 1, L0, false, B->stream);
        if (rc) return rc;
        if (any) HIPCHK(hipStreamWaitEvent(B->stream, B->join, 0));
        B->L += 2;
        ++B->rounds2;
    } else {
        const int all[] = {0, 1, 2, 3, MARCH};
        int rc = launch_lists<T>(B, all, 5, L0, true, B->stream);
        if (rc) return rc;
        B->L += 1;
        ++B->rounds1;
    }
    B->R += 1;
    // slots whose budget just ran out leave the work lists (pair slots keep
    // the round at which they stopped); pair slots left with one step move
    // to the one-step list
    for (int k = 0; k < B->capacity; ++k) {
        if (!B->used[k]) continue;
        const long stop = B->slot[k].stop;
        if (stop > L0 && stop <= B->L) {
            B->dirty = true;
            if (B->slot[k].pair) B->rstop[k] = B->R;
        }
        if (B->slot[k].pair && stop - B->L == 1) B->dirty = true;
    }
    return MRTFD_OK;
}

int launch_round(mrtfd_batch_s* B, bool two)
{
    return (B->precision == MRTFD_FP32_STORAGE) ? launch_round_t<float>(B, two) : launch_round_t<double>(B, two);
}

int ensure_staging(mrtfd_batch_s* B, size_t bytes)
{
    if (B->staging_bytes >= bytes) return MRTFD_OK;
    if (B->staging) {
        HIPCHK(hipStreamSynchronize(B->stream));
        HIPCHK(hipFree(B->staging));
        B->staging = nullptr;
        B->staging_bytes = 0;
    }
    if (hipMalloc(&B->staging, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MRTFD_ENOMEM, "cannot allocate %zu bytes of staging", bytes);
    }
    B->staging_bytes = bytes;
    return MRTFD_OK;
}

template <typename T>
const void* march_batch_kernel(int limiter)
{
    switch (limiter) {
    case 0: return (const void*)k_march_batch<0, T>;
    case 1: return (const void*)k_march_batch<1, T>;
    case 2: return (const void*)k_march_batch<2, T>;
    default: return (const void*)k_march_batch<3, T>;
    }
}

template <typename T>
const void* pair_batch_kernel(int limiter)
{
    switch (limiter) {
    case 0: return (const void*)k_march2_batch<0, T>;
    case 1: return (const void*)k_march2_batch<1, T>;
    case 2: return (const void*)k_march2_batch<2, T>;
    default: return (const void*)k_march2_batch<3, T>;
    }
}

// Rewrite every ghost layer of a slot's current buffer from its interior.
template <typename T>
int refill_current_t(mrtfd_batch_s* B, int k)
{
    const mrtfd_params& p = B->prm[k];
    T* f = (T*)B->slot[k].buf[current_buffer(B, k)];
    for (int axis = 0; axis < 2; ++axis) {
        const int n = 2 * ((axis == 0) ? p.ny : p.nx);
        hipLaunchKernelGGL((k_fill<T>), dim3((n + 127) / 128), dim3(128), 0, B->stream, f, B->slot[k].a, axis, 0);
        HIPCHK(hipGetLastError());
    }
    return MRTFD_OK;
}

// Move slot k to shape class s.  The strip kernel reads periodic and
// outflow sides at their source nodes and leaves those ghosts stale, while
// the tile kernels read the ghosts: leaving the strip class refills them.
int assign_shape(mrtfd_batch_s* B, int k, int s)
{
    const int old = B->shape[k];
    if (old == s) return MRTFD_OK;
    const int cur = current_buffer(B, k);
    B->shape[k] = s;
    set_args(B, k);
    rebase(B, k, cur);
    int rc = upload_slot(B, k);
    if (rc) return rc;
    if (old == MARCH) {
        rc = (B->precision == MRTFD_FP32_STORAGE) ? refill_current_t<float>(B, k) : refill_current_t<double>(B, k);
        if (rc) return rc;
    }
    B->dirty = true;
    return MRTFD_OK;
}

template <typename T>
int init_slot_t(mrtfd_batch_s* B, int k, const double* const* src, const double* fsrc)
{
    const StepArgs& a = B->slot[k].a;
    const mrtfd_params& p = B->prm[k];
    T* f = (T*)B->slot[k].buf[0];
    dim3 grid((p.nx + 63) / 64, (p.ny + 3) / 4), block(64, 4);
    if (fsrc) hipLaunchKernelGGL((k_scatter<T>), grid, block, 0, B->stream, f, fsrc, a);
    else hipLaunchKernelGGL((k_init<T>), grid, block, 0, B->stream, f, src[0], src[1], src[2], src[3], a);
    HIPCHK(hipGetLastError());
    for (int axis = 0; axis < 2; ++axis) {
        const int n = 2 * ((axis == 0) ? p.ny : p.nx);
        hipLaunchKernelGGL((k_fill<T>), dim3((n + 127) / 128), dim3(128), 0, B->stream, f, a, axis, 0);
        HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(B->slot[k].buf[1], f, B->lay[k].buf_bytes, hipMemcpyDeviceToDevice, B->stream));
    HIPCHK(hipMemsetAsync(B->d_flags + k, 0, sizeof(int), B->stream));
    return MRTFD_OK;
}

int init_slot(mrtfd_batch_s* B, int k, const double* const* src, const double* fsrc)
{
    return (B->precision == MRTFD_FP32_STORAGE) ? init_slot_t<float>(B, k, src, fsrc) : init_slot_t<double>(B, k, src, fsrc);
}

}  // namespace

extern "C" {

int mrtfd_batch_create(int capacity, int precision, int limiter, void* hip_stream, mrtfd_batch_t* out)
{
    if (!out) return fail(MRTFD_EINVAL, "out is NULL");
    *out = nullptr;
    if (capacity < 1 || capacity > 65536) return fail(MRTFD_EINVAL, "capacity %d out of range [1, 65536]", capacity);
    if (precision != MRTFD_FP64 && precision != MRTFD_FP32_STORAGE) return fail(MRTFD_EINVAL, "unknown precision");
    if (limiter < 0 || limiter > 3) return fail(MRTFD_EINVAL, "unknown limiter");
    mrtfd_batch_s* B = new (std::nothrow) mrtfd_batch_s();
    if (!B) return fail(MRTFD_ENOMEM, "host allocation failed");
    B->capacity = capacity;
    B->precision = precision;
    B->limiter = limiter;
    B->stream = (hipStream_t)hip_stream;
    B->slot.resize(capacity);
    B->prm.resize(capacity);
    B->lay.resize(capacity);
    B->blk.resize(capacity);
    B->used.assign(capacity, 0);
    B->shape.assign(capacity, 0);
    B->rstop.assign(capacity, LONG_MAX);
    B->per_launch = 2;
    B->mrows = MBROWS;
    B->prows = MBROWS2;
    B->fit_rows = true;
    for (int s = 0; s < NSHAPE; ++s) {
        B->cost[s] = DEFAULT_COST[s];
        B->launch_us[s] = 10.0;
    }
    const size_t lists = ((size_t)(NLIST * (capacity + 1) + NLIST * capacity + capacity) + pair_region_ints(capacity)) *
                         sizeof(int);
    if (hipMalloc(&B->d_slot, capacity * sizeof(BatchSlot)) != hipSuccess ||
        hipMalloc(&B->d_blocks, capacity * sizeof(Blocks)) != hipSuccess ||
        hipMalloc(&B->d_flags, capacity * sizeof(int)) != hipSuccess || hipMalloc(&B->d_lists, lists) != hipSuccess ||
        hipEventCreate(&B->ev0) != hipSuccess || hipEventCreate(&B->ev1) != hipSuccess ||
        hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&B->join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        mrtfd_batch_destroy(B);
        return fail(MRTFD_ENOMEM, "batch set-up failed");
    }
    if (hipMemsetAsync(B->d_flags, 0, capacity * sizeof(int), B->stream) != hipSuccess ||
        hipMemsetAsync(B->d_lists, 0, lists, B->stream) != hipSuccess) {
        mrtfd_batch_destroy(B);
        return fail(MRTFD_EDEVICE, "batch set-up failed");
    }
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    B->max_blocks = 4 * ncu;   // persistent grid: a few resident blocks per CU
    int nb = 0;
    const void* km = (precision == MRTFD_FP32_STORAGE) ? march_batch_kernel<float>(limiter) : march_batch_kernel<double>(limiter);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, km, MW * MWPB, 0) != hipSuccess) (void)hipGetLastError();
    B->march_blocks = std::max(nb, 1) * ncu;
    nb = 0;
    const void* kp = (precision == MRTFD_FP32_STORAGE) ? pair_batch_kernel<float>(limiter) : pair_batch_kernel<double>(limiter);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kp, 2 * MW, 0) != hipSuccess) (void)hipGetLastError();
    B->pair_blocks = std::max(nb, 1) * ncu;
    B->dirty = true;
    *out = B;
    return MRTFD_OK;
}

int mrtfd_batch_destroy(mrtfd_batch_t B)
{
    if (!B) return MRTFD_OK;
    // slot buffers come from the stream-ordered pool: return them on the
    // batch's stream, then wait for it
    for (int k = 0; k < B->capacity; ++k)
        if (B->used[k]) {
            (void)hipFreeAsync(B->slot[k].buf[0], B->stream);
            (void)hipFreeAsync(B->slot[k].buf[1], B->stream);
        }
    (void)hipStreamSynchronize(B->stream);
    (void)hipFree(B->d_slot);
    (void)hipFree(B->d_blocks);
    (void)hipFree(B->d_flags);
    (void)hipFree(B->d_lists);
    if (B->staging) (void)hipFree(B->staging);
    if (B->ev0) (void)hipEventDestroy(B->ev0);
    if (B->ev1) (void)hipEventDestroy(B->ev1);
    if (B->side) {
        (void)hipStreamSynchronize(B->side);
        (void)hipStreamDestroy(B->side);
    }
    if (B->fork) (void)hipEventDestroy(B->fork);
    if (B->join) (void)hipEventDestroy(B->join);
    delete B;
    return MRTFD_OK;
}

int mrtfd_batch_add(mrtfd_batch_t B, const mrtfd_params* p, const double* rho, const double* ux, const double* uy,
                    const double* T, int on_device, long nsteps, int* slot_out)
{
    if (!B || !p || !slot_out || !rho || !ux || !uy || !T) return fail(MRTFD_EINVAL, "NULL argument");
    *slot_out = -1;
    int rc = validate(p);
    if (rc) return rc;
    if (p->precision != B->precision || p->limiter != B->limiter)
        return fail(MRTFD_EINVAL, "instance precision / limiter differ from the batch's");
    int k = 0;
    while (k < B->capacity && B->used[k]) ++k;
    if (k == B->capacity) return fail(MRTFD_ENOMEM, "all %d slots are occupied", B->capacity);
    B->prm[k] = *p;
    B->lay[k] = layout_of(*p);
    if (!build_blocks(p->eta0, &B->blk[k])) return fail(MRTFD_EINVAL, "singular moment blocks for eta0 = %g", p->eta0);
    void* b0 = nullptr;
    void* b1 = nullptr;
    if (hipMallocAsync(&b0, B->lay[k].buf_bytes, B->stream) != hipSuccess ||
        hipMallocAsync(&b1, B->lay[k].buf_bytes, B->stream) != hipSuccess) {
        (void)hipGetLastError();
        if (b0) (void)hipFreeAsync(b0, B->stream);
        return fail(MRTFD_ENOMEM, "cannot allocate 2 x %zu bytes for slot %d", B->lay[k].buf_bytes, k);
    }
    B->slot[k].buf[0] = b0;
    B->slot[k].buf[1] = b1;
    B->shape[k] = pick_shape(B, *p);
    set_args(B, k);
    B->slot[k].start = B->L;
    B->slot[k].stop = (nsteps < 0) ? LONG_MAX : B->L + nsteps;
    rebase(B, k, 0);   // the state starts in buffer 0
    B->used[k] = 1;
    rc = [&]() -> int {
        HIPCHK(hipMemcpyAsync(B->d_blocks + k, &B->blk[k], sizeof(Blocks), hipMemcpyHostToDevice, B->stream));
        int r = upload_slot(B, k);
        if (r) return r;
        const size_t n = (size_t)p->nx * p->ny;
        const double* src[4] = {rho, ux, uy, T};
        if (!on_device) {
            r = ensure_staging(B, 4 * n * sizeof(double));
            if (r) return r;
            for (int q = 0; q < 4; ++q) {
                HIPCHK(hipMemcpyAsync(B->staging + q * n, src[q], n * sizeof(double), hipMemcpyHostToDevice, B->stream));
                src[q] = B->staging + q * n;
            }
        }
        r = init_slot(B, k, src, nullptr);
        if (r) return r;
        if (!on_device) HIPCHK(hipStreamSynchronize(B->stream));
        return MRTFD_OK;
    }();
    if (rc) {
        (void)hipFreeAsync(b0, B->stream);
        (void)hipFreeAsync(b1, B->stream);
        B->used[k] = 0;
        return rc;
    }
    B->dirty = true;
    *slot_out = k;
    return MRTFD_OK;
}

int mrtfd_batch_remove(mrtfd_batch_t B, int k)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    HIPCHK(hipFreeAsync(B->slot[k].buf[0], B->stream));
    HIPCHK(hipFreeAsync(B->slot[k].buf[1], B->stream));
    B->slot[k].buf[0] = B->slot[k].buf[1] = nullptr;
    B->slot[k].stop = B->L;
    B->used[k] = 0;
    B->dirty = true;
    return MRTFD_OK;
}

int mrtfd_batch_set_steps(mrtfd_batch_t B, int k, long nsteps)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    // keep the current buffer: restart the count at this launch
    const int cur = current_buffer(B, k);
    if (cur) {
        std::swap(B->slot[k].buf[0], B->slot[k].buf[1]);
    }
    B->slot[k].start = B->L;
    B->slot[k].stop = (nsteps < 0) ? LONG_MAX : B->L + nsteps;
    rebase(B, k, 0);
    rc = upload_slot(B, k);
    if (rc) return rc;
    B->dirty = true;
    return MRTFD_OK;
}

int mrtfd_batch_step(mrtfd_batch_t B, long nsteps)
{
    if (!B) return fail(MRTFD_EINVAL, "NULL batch");
    if (nsteps < 0) return fail(MRTFD_EINVAL, "nsteps < 0");
    for (long s = 0; s < nsteps;) {
        if (B->dirty) {
            int rc = rebuild_lists(B);
            if (rc) return rc;
        }
        const bool two = nsteps - s >= 2 && two_step_round_ok(B);
        int rc = launch_round(B, two);
        if (rc) return rc;
        s += two ? 2 : 1;
    }
    return MRTFD_OK;
}

int mrtfd_batch_get_steps_per_launch(mrtfd_batch_t B, int* k)
{
    if (!B || !k) return fail(MRTFD_EINVAL, "NULL argument");
    *k = B->per_launch;
    return MRTFD_OK;
}

int mrtfd_batch_set_steps_per_launch(mrtfd_batch_t B, int k)
{
    if (!B) return fail(MRTFD_EINVAL, "NULL batch");
    if (k != 1 && k != 2) return fail(MRTFD_EINVAL, "steps per launch must be 1 or 2, got %d", k);
    if (k == B->per_launch) return MRTFD_OK;
    B->per_launch = k;
    for (int q = 0; q < B->capacity; ++q) {
        if (!B->used[q]) continue;
        const int cur = current_buffer(B, q);
        B->slot[q].pair = pair_capable(B, q) ? 1 : 0;
        rebase(B, q, cur);
        int rc = upload_slot(B, q);
        if (rc) return rc;
    }
    B->dirty = true;
    return MRTFD_OK;
}

int mrtfd_batch_step_timed(mrtfd_batch_t B, long nsteps, double* elapsed_ms)
{
    if (!B || !elapsed_ms) return fail(MRTFD_EINVAL, "NULL argument");
    if (B->dirty) {
        int rc = rebuild_lists(B);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(B->ev0, B->stream));
    int rc = mrtfd_batch_step(B, nsteps);
    if (rc) return rc;
    HIPCHK(hipEventRecord(B->ev1, B->stream));
    HIPCHK(hipEventSynchronize(B->ev1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, B->ev0, B->ev1));
    *elapsed_ms = ms;
    return MRTFD_OK;
}

long mrtfd_batch_steps_done(mrtfd_batch_t B, int k)
{
    if (check_slot(B, k)) return -1;
    return std::min(B->L, B->slot[k].stop) - B->slot[k].start;
}

int mrtfd_batch_rounds(mrtfd_batch_t B, long* one_step, long* two_step)
{
    if (!B || !one_step || !two_step) return fail(MRTFD_EINVAL, "NULL argument");
    *one_step = B->rounds1;
    *two_step = B->rounds2;
    return MRTFD_OK;
}

int mrtfd_batch_pair_rows(mrtfd_batch_t B, int* rows)
{
    if (!B || !rows) return fail(MRTFD_EINVAL, "NULL argument");
    *rows = B->prows;
    return MRTFD_OK;
}

int mrtfd_batch_remaining(mrtfd_batch_t B, int k, long* remaining)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    if (!remaining) return fail(MRTFD_EINVAL, "NULL argument");
    *remaining = (B->slot[k].stop == LONG_MAX) ? -1 : std::max(0L, B->slot[k].stop - B->L);
    return MRTFD_OK;
}

int mrtfd_batch_macros(mrtfd_batch_t B, int k, double* rho, double* ux, double* uy, double* T, int on_device)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    const mrtfd_params& p = B->prm[k];
    const size_t n = (size_t)p.nx * p.ny;
    double* dst[4] = {rho, ux, uy, T};
    if (!on_device) {
        rc = ensure_staging(B, 4 * n * sizeof(double));
        if (rc) return rc;
        for (int q = 0; q < 4; ++q) dst[q] = dst[q] ? B->staging + q * n : nullptr;
    }
    const void* f = B->slot[k].buf[current_buffer(B, k)];
    dim3 grid((p.nx + 63) / 64, (p.ny + 3) / 4), block(64, 4);
    if (B->precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_macros<float>), grid, block, 0, B->stream, (const float*)f, dst[0], dst[1], dst[2], dst[3], B->slot[k].a);
    else
        hipLaunchKernelGGL((k_macros<double>), grid, block, 0, B->stream, (const double*)f, dst[0], dst[1], dst[2], dst[3], B->slot[k].a);
    HIPCHK(hipGetLastError());
    if (!on_device) {
        double* host[4] = {rho, ux, uy, T};
        for (int q = 0; q < 4; ++q)
            if (host[q]) HIPCHK(hipMemcpyAsync(host[q], B->staging + q * n, n * sizeof(double), hipMemcpyDeviceToHost, B->stream));
        HIPCHK(hipStreamSynchronize(B->stream));
    }
    return MRTFD_OK;
}

int mrtfd_batch_get_f(mrtfd_batch_t B, int k, double* f, int on_device)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    if (!f) return fail(MRTFD_EINVAL, "NULL argument");
    const mrtfd_params& p = B->prm[k];
    const size_t n = (size_t)p.nx * p.ny;
    double* dst = f;
    if (!on_device) {
        rc = ensure_staging(B, NQ * n * sizeof(double));
        if (rc) return rc;
        dst = B->staging;
    }
    const void* src = B->slot[k].buf[current_buffer(B, k)];
    dim3 grid((p.nx + 63) / 64, (p.ny + 3) / 4), block(64, 4);
    if (B->precision == MRTFD_FP32_STORAGE)
        hipLaunchKernelGGL((k_gather<float>), grid, block, 0, B->stream, (const float*)src, dst, B->slot[k].a);
    else
        hipLaunchKernelGGL((k_gather<double>), grid, block, 0, B->stream, (const double*)src, dst, B->slot[k].a);
    HIPCHK(hipGetLastError());
    if (!on_device) {
        HIPCHK(hipMemcpyAsync(f, B->staging, NQ * n * sizeof(double), hipMemcpyDeviceToHost, B->stream));
        HIPCHK(hipStreamSynchronize(B->stream));
    }
    return MRTFD_OK;
}

int mrtfd_batch_set_f(mrtfd_batch_t B, int k, const double* f, int on_device)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    if (!f) return fail(MRTFD_EINVAL, "NULL argument");
    const mrtfd_params& p = B->prm[k];
    const size_t n = (size_t)p.nx * p.ny;
    const double* src = f;
    if (!on_device) {
        rc = ensure_staging(B, NQ * n * sizeof(double));
        if (rc) return rc;
        HIPCHK(hipMemcpyAsync(B->staging, f, NQ * n * sizeof(double), hipMemcpyHostToDevice, B->stream));
        src = B->staging;
    }
    // the state restarts in buffer 0 with the remaining budget
    const long remaining = (B->slot[k].stop == LONG_MAX) ? -1 : std::max(0L, B->slot[k].stop - B->L);
    B->slot[k].start = B->L;
    B->slot[k].stop = (remaining < 0) ? LONG_MAX : B->L + remaining;
    rebase(B, k, 0);
    rc = upload_slot(B, k);
    if (rc) return rc;
    rc = init_slot(B, k, nullptr, src);
    if (rc) return rc;
    if (!on_device) HIPCHK(hipStreamSynchronize(B->stream));
    B->dirty = true;
    return MRTFD_OK;
}

int mrtfd_batch_status(mrtfd_batch_t B, int* flags)
{
    if (!B) return fail(MRTFD_EINVAL, "NULL batch");
    HIPCHK(hipStreamSynchronize(B->stream));
    std::vector<int> h(B->capacity, 0);
    HIPCHK(hipMemcpy(h.data(), B->d_flags, B->capacity * sizeof(int), hipMemcpyDeviceToHost));
    int bad = 0;
    for (int k = 0; k < B->capacity; ++k) {
        if (flags) flags[k] = h[k];
        bad += (h[k] != 0);
    }
    if (bad) {
        HIPCHK(hipMemset(B->d_flags, 0, B->capacity * sizeof(int)));
        return fail(MRTFD_ENONFINITE, "%d slot(s) reached rho <= 0, T <= 0 or NaN", bad);
    }
    return MRTFD_OK;
}

int mrtfd_batch_shape(mrtfd_batch_t B, int k, int* txw, int* byr)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    const bool m = B->shape[k] == MARCH;
    if (txw) *txw = m ? MOUT : SHAPES[B->shape[k]].txw;
    if (byr) *byr = m ? B->slot[k].a.m_rows : SHAPES[B->shape[k]].byr;
    return MRTFD_OK;
}

int mrtfd_batch_set_shape(mrtfd_batch_t B, int k, int shape)
{
    int rc = check_slot(B, k);
    if (rc) return rc;
    if (shape < 0 || shape >= NSHAPE) return fail(MRTFD_EINVAL, "unknown shape class %d", shape);
    if (!shape_fits(B->prm[k], shape)) return fail(MRTFD_EINVAL, "shape class %d does not fit slot %d", shape, k);
    return assign_shape(B, k, shape);
}

// Measure the cost per work unit of every shape class on calibration
// instances (a 2-D grid for the strips and the three 2-D tiles, a one-row
// grid for the row tile), then give every occupied slot the cheapest class.
// Slot states are untouched.
int mrtfd_batch_autotune(mrtfd_batch_t B, double* cost_per_unit_us)
{
    if (!B) return fail(MRTFD_EINVAL, "NULL batch");
    HIPCHK(hipStreamSynchronize(B->stream));
    // time `steps` launches of one calibration instance forced into class s
    auto time_class = [&](int s, int nx, int ny, int steps, double* ms) -> int {
        mrtfd_params p;
        std::memset(&p, 0, sizeof(p));
        p.nx = nx;
        p.ny = ny;
        p.dx = p.dy = 1.0 / 512;
        p.dt = 0.05 * p.dx / 6.0;
        p.eta0 = 2.5;
        for (int q = 0; q < NQ; ++q) p.s[q] = 0.5 / p.dt;
        p.b = 5.0;
        p.limiter = B->limiter;
        p.precision = B->precision;
        p.energy_flux_correction = 1;
        for (int q = 0; q < 4; ++q) p.bc[q] = mrtfd_bc{MRTFD_BC_PERIODIC, 1.0, 0.0, 0.0, 1.0};
        mrtfd_batch_t C = nullptr;
        int rc = mrtfd_batch_create(1, B->precision, B->limiter, B->stream, &C);
        if (rc) return rc;
        C->fit_rows = false;     // per-unit costs at the standard band height
        const size_t n = (size_t)p.nx * p.ny;
        std::vector<double> one(n, 1.0), zero(n, 0.0);
        int k = -1;
        rc = mrtfd_batch_add(C, &p, one.data(), zero.data(), zero.data(), one.data(), 0, -1, &k);
        if (!rc) rc = assign_shape(C, k, s);
        if (!rc) rc = mrtfd_batch_step(C, 3);
        if (!rc) rc = mrtfd_batch_step_timed(C, steps, ms);
        mrtfd_batch_destroy(C);
        return rc;
    };
    for (int s = 0; s < NSHAPE; ++s) {
        const bool flat = SHAPES[s].flat;
        const int nx = flat ? 262144 : 2048, ny = flat ? 1 : 512;
        double ms = 0.0, ms0 = 0.0;
        int rc = time_class(s, nx, ny, 20, &ms);
        if (!rc) rc = time_class(s, flat ? 256 : 16, flat ? 1 : 16, 20, &ms0);   // one small launch
        if (rc) return rc;
        mrtfd_params p;
        std::memset(&p, 0, sizeof(p));
        p.nx = nx;
        p.ny = ny;
        for (int q = 0; q < 4; ++q) p.bc[q].kind = MRTFD_BC_PERIODIC;
        B->launch_us[s] = 1e3 * ms0 / 20.0;
        B->cost[s] = std::max(1e3 * (ms - ms0) / 20.0, 1e-3) / (double)tiles_of(p, s);   // per work unit
        if (cost_per_unit_us) cost_per_unit_us[s] = B->cost[s];
    }
    // every slot to its cheapest class by work; then a class whose slots
    // together would save less than its launch costs returns them to the
    // strips
    std::vector<int> pick(B->capacity, -1);
    for (int k = 0; k < B->capacity; ++k) {
        if (!B->used[k]) continue;
        double best = 1e300;
        for (int s = 0; s < NSHAPE; ++s) {
            if (!shape_fits(B->prm[k], s)) continue;
            const double c = (double)tiles_of(B->prm[k], s) * B->cost[s];
            if (c < best) {
                best = c;
                pick[k] = s;
            }
        }
    }
    for (int s = 0; s < NSHAPE; ++s) {
        if (s == MARCH) continue;
        double saving = 0.0;
        for (int k = 0; k < B->capacity; ++k) {
            if (pick[k] != s) continue;
            if (!shape_fits(B->prm[k], MARCH)) saving = 1e300;   // no alternative
            else saving += (double)tiles_of(B->prm[k], MARCH) * B->cost[MARCH] - (double)tiles_of(B->prm[k], s) * B->cost[s];
        }
        if (saving < B->launch_us[s])
            for (int k = 0; k < B->capacity; ++k)
                if (pick[k] == s) pick[k] = MARCH;
    }
    for (int k = 0; k < B->capacity; ++k) {
        if (!B->used[k]) continue;
        int rc = assign_shape(B, k, pick[k]);
        if (rc) return rc;
    }
    B->dirty = true;
    return MRTFD_OK;
}

int mrtfd_batch_sync(mrtfd_batch_t B)
{
    if (!B) return fail(MRTFD_EINVAL, "NULL batch");
    HIPCHK(hipStreamSynchronize(B->stream));
    return MRTFD_OK;
}

}  // extern "C"
