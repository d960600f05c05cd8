// Internal declarations shared by the kernels and the host entry points of libfof.so.
// Target: gfx950 (CDNA4), wave64.  Everything here is device-side plumbing; the public
// interface is include/fof.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fof.h"

// The link predicate must round exactly like its definition (no fused multiply-add).
#pragma clang fp contract(off)

namespace fof {

constexpr int kWave = 64;
constexpr int kDefaultBlock = 256;
constexpr int kScanItems = 8;                  // elements per thread in the scan kernels
constexpr int kMaxFine = 10;                   // fine cells per coarse cell per axis (max)
constexpr int kMaxFineKeys = kMaxFine * kMaxFine * kMaxFine;
constexpr int kMaxTableWords = (kMaxFineKeys + 31) / 32;
// Dense-pass work cursors: per pass (4 modes x small/big cells) kCursorGroups counters, each
// on its own 64-byte line so that groups do not contend.
constexpr int kCursorGroups = 64;
constexpr int kCursorStride = 16;
constexpr int kCursorInts = 8 * kCursorGroups * kCursorStride;
constexpr int kTableHeader = 4;  // dense-cell table: cell, ncomp, units, reserved
// Link tiles: kTileX x kTileY x kTileZ coarse cells per block (z fastest, like the cells).
constexpr int kTileX = 4, kTileY = 4, kTileZ = 16;

// Per-box constants, computed once on the host in double precision and copied into the
// workspace by the caller.  Layout is private to this library.
struct alignas(16) BoxDesc {
    int64_t off;        // first particle of the box in the concatenated arrays
    int64_t cell_base;  // first coarse cell of the box in the concatenated cell table
    int64_t tile_base;  // first link tile of the box (tiled boxes only)
    int32_t n;          // particles in the box
    int32_t m;          // fine (clique) cells per coarse cell per axis
    int32_t nc[3];      // coarse cells per axis
    int32_t nf[3];      // fine cells per axis (nc * m)
    int32_t R;          // fine-cell reach: a friend lies at most R fine cells away per axis
    int32_t dense_ok;   // 1 if this box may use the clique-cell path (>= 3 cells per axis)
    int32_t tiled;      // 1 if the LDS-tiled link kernel handles this box
    int32_t ntile[3];   // link tiles per axis
    double L[3];        // box lengths
    double halfL[3];    // 0.5 * L (exact)
    double b2;          // b * b, rounded once in double
    float inv_fine[3];  // float(nf / L): fine index = trunc(x * inv_fine)
    float side[3];      // float(L / nc): coarse cell side
    float reach;        // pruning distance: b plus the bound on index rounding error
    float fine_side;    // smallest fine cell side less the index error (float, rounded down)
    float fine[3];      // fine cell side per axis, L / nf (float)
    float slack;        // margin added to fine-cell boxes before a distance skip
    float Lup[3];       // smallest float >= L: a float x is below L exactly when x < Lup
    uint32_t mdiv;      // ceil(2^32 / m) for m > 1: fine / m as one multiply-high
};

// Status bits (public values in fof.h) and the counters block.
struct Counters {
    int32_t status;
    int32_t n_dense;     // dense cells found
    int32_t n_big;       // dense cells linked by a whole block
    int32_t n_spill;       // link tiles queued in tile_list for the windowed kernel
    int32_t n_link_edges;  // hooks the tiled kernel deferred to the edge list
    int32_t n_flagged;     // particles with a friend (length of Work::flist)
    int32_t n_dense_edges; // hooks the sparse-dense pass deferred (pairs in Work::temp)
    int32_t dense_edge_over;  // set when they did not all fit
    int32_t pad[8];
    unsigned long long stats[24];  // event counts of diagnostic builds (-DFOF_STATS)
};

// Event counters for diagnostic builds; compiled out otherwise.
enum Stat {
    ST_TILES, ST_TILES_OVERFLOW, ST_OWN_STAGED, ST_OWN_GLOBAL, ST_PAIRS_TILED, ST_PAIRS_GLOBAL,
    ST_DN_CALLS, ST_DN_UNITS, ST_CELL_CYCLES, ST_CC_UNIT_PAIRS, ST_CELL_MAX_CYCLES,
    ST_CROSS_UNIT_PAIRS, ST_CELLS_TIMED, ST_UNIONS, ST_CROSS_CELLPAIRS, ST_SPARE,
    ST_CC_SMALL_CYCLES, ST_CC_SMALL_CELLS, ST_CC_BIG_CYCLES, ST_CC_BIG_CELLS, ST_CC_UNITS,
    ST_CC_MEMBER_TESTS, ST_CC_SKIPS, ST_CC_FAR_CELLS
};
#if defined(FOF_STATS) && !defined(FOF_TIMING)
#define FOF_STAT(ctr, k, v) atomicAdd(&(ctr)->stats[k], (unsigned long long)(v))
#define FOF_STAT_MAX(ctr, k, v) atomicMax(&(ctr)->stats[k], (unsigned long long)(v))
#else
#define FOF_STAT(ctr, k, v) ((void)0)
#define FOF_STAT_MAX(ctr, k, v) ((void)0)
#endif

constexpr int kSmallCell = 256;  // dense cells up to this size are linked by one wave

// ---------------------------------------------------------------------------------------
// Box lookup: box k owns global indices [off_k, off_k + n_k); boxes are in order.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int find_box(const BoxDesc *__restrict__ d, int nbox, int64_t i)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].off <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Box owning coarse cell c (cells are numbered box after box from each box's cell_base).
__device__ __forceinline__ int find_box_cell(const BoxDesc *d, int nbox, int64_t c)
{
    int lo = 0, hi = nbox - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (d[mid].cell_base <= c)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Fine (clique) cell index along one axis: trunc(x * inv_fine) clamped to nf - 1.  The
// coarse index is fine / m, so fine cells nest exactly inside coarse cells.  The computed
// fine cell is the exact cell of some x' with |x' - x| <= L 2^-23 (1 + 2^-10).
__device__ __forceinline__ int fine_index(float x, float inv, int nf)
{
    int f = (int)(x * inv);
    return f < nf - 1 ? f : nf - 1;
}

// Coarse index of a fine index f: f / m, as the high word of f * ceil(2^32 / m).  With
// ceil(2^32 / m) m = 2^32 + e, e < m <= 10, the quotient is exact for f < 2^32 / e, far above
// any fine index (at most 10 * 2^20).
__device__ __forceinline__ int coarse_of(int f, const BoxDesc &B)
{
    return B.m == 1 ? f : (int)__umulhi((uint32_t)f, B.mdiv);
}

// Coarse cell coordinate of a float coordinate along axis a.
__device__ __forceinline__ int coarse_index(float x, const BoxDesc &B, int a)
{
    return coarse_of(fine_index(x, B.inv_fine[a], B.nf[a]), B);
}

// Linear coarse cell id with z fastest (C order over (ix, iy, iz)).  The paper's grid uses
// x fastest; z fastest makes the counting sort nearly sequential for particles stored in
// C order of a Lagrangian lattice, the usual N-body layout.  No result depends on it.
// Offsets to visit along one axis, deduplicated when the grid has fewer than 3 cells:
// a neighbour is needed only if the particle lies within `reach` of the shared face.
struct AxisSpan {
    int lo, hi;  // visit o in [lo, hi] (o = -1, 0, +1), skipping none in between
};

__device__ __forceinline__ AxisSpan axis_span(float x, int ix, float side, int nc, float reach)
{
    if (nc == 1)
        return {0, 0};
    float g_lo = x - (float)ix * side;          // distance to the lower face
    float g_hi = (float)(ix + 1) * side - x;    // distance to the upper face
    bool need_lo = g_lo < reach;
    bool need_hi = g_hi < reach;
    if (nc == 2)  // the single other cell is both the lower and the upper neighbour
        return {0, (need_lo || need_hi) ? 1 : 0};
    return {need_lo ? -1 : 0, need_hi ? 1 : 0};
}

// The k-th offset of a span, own offset first: 0, then lo if it is -1, then hi if it is +1.
// Walking offsets in this order lets lanes whose positions need different neighbours share
// loop steps (a wave runs max-over-lanes steps, not the union of the offsets).
__device__ __forceinline__ int span_offset(const AxisSpan &s, int k)
{
    return k == 0 ? 0 : (k == 1 && s.lo < 0 ? -1 : 1);
}

__device__ __forceinline__ int wrap_cell(int c, int nc)
{
    return c < 0 ? c + nc : (c >= nc ? c - nc : c);
}

// Fine-key range of a neighbour dense cell that a particle at fine coordinate f (relative
// to that cell's origin, in the particle's periodic frame) can reach.
__device__ __forceinline__ void key_range(float f, float rf, int m, int &lo, int &hi)
{
    lo = (int)floorf(f - rf);
    hi = (int)floorf(f + rf);
    lo = lo < 0 ? 0 : lo;
    hi = hi > m - 1 ? m - 1 : hi;
}

__device__ __forceinline__ int64_t coarse_cell(const BoxDesc &B, int ix, int iy, int iz)
{
    return B.cell_base + ((int64_t)ix * B.nc[1] + iy) * B.nc[2] + iz;
}

// Block index remapped so that the blocks the hardware hands to one XCD (blockIdx mod 8)
// process one contiguous stretch of the cell-sorted particles, keeping neighbour cells in
// that XCD's L2.
__device__ __forceinline__ int64_t xcd_block()
{
    const int64_t g = gridDim.x, b = blockIdx.x;
    const int64_t per = g / 8, rem = g % 8, x = b % 8, k = b / 8;
    // XCD x owns per + (x < rem) consecutive logical blocks
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + k;
}

// Exact link predicate: per axis d = (double)xi - (double)xj, wrapped once by +-L when
// |d| > L/2; s = ((dx*dx + dy*dy) + dz*dz) in double; friends iff s < b*b.
__device__ __forceinline__ double min_image(double d, double L, double h)
{
    if (d > h)
        d -= L;
    else if (d < -h)
        d += L;
    return d;
}

// The predicate's box constants.  Kernels copy them out of the descriptor once (pred_of),
// so they stay in registers across stores the compiler cannot prove disjoint from the
// descriptor; dist2 and linked take either.
struct Pred {
    double L[3], halfL[3], b2;
    float nowrap[3];   // |dx| below this (float) implies |dx| < L/2 exactly: no image shift
    float b2lo, b2hi;  // float sums below b2lo are links, above b2hi are not (see linked)
};

__device__ __forceinline__ Pred pred_of(const BoxDesc &B)
{
    Pred P;
    for (int a = 0; a < 3; ++a) {
        P.L[a] = B.L[a];
        P.halfL[a] = B.halfL[a];
        P.nowrap[a] = (float)(B.halfL[a] * (1.0 - 0x1.0p-20));
    }
    P.b2 = B.b2;
    P.b2lo = (float)(B.b2 * (1.0 - 0x1.0p-18));
    P.b2hi = (float)(B.b2 * (1.0 + 0x1.0p-18));
    return P;
}

// Descriptor of the box a whole wave works on: the index is made wave-uniform, so its
// fields are read with scalar loads.
__device__ __forceinline__ const BoxDesc &uniform_box(const BoxDesc *desc, int k)
{
    return desc[__builtin_amdgcn_readfirstlane(k)];
}

template <class Box>
__device__ __forceinline__ double dist2(const Box &B, float xi, float yi, float zi, float xj,
                                        float yj, float zj)
{
    double dx = min_image((double)xi - (double)xj, B.L[0], B.halfL[0]);
    double dy = min_image((double)yi - (double)yj, B.L[1], B.halfL[1]);
    double dz = min_image((double)zi - (double)zj, B.L[2], B.halfL[2]);
    double sx = __dmul_rn(dx, dx);
    double sy = __dmul_rn(dy, dy);
    double sz = __dmul_rn(dz, dz);
    return __dadd_rn(__dadd_rn(sx, sy), sz);
}

__device__ __forceinline__ bool linked(const BoxDesc &B, float xi, float yi, float zi, float xj,
                                       float yj, float zj)
{
    return dist2(B, xi, yi, zi, xj, yj, zj) < B.b2;
}

// The same decision with a float prefilter.  Each float difference is within 2^-24 of the
// exact one (relative), so the float sum of squares s is within 5 * 2^-24 of d^2; the double
// path rounds d^2 by at most 3 * 2^-53.  With b2lo/b2hi 2^-18 below/above b^2 (rounded to
// float: 2^-24 more), s < b2lo implies the double sum is below b^2 and s > b2hi that it is
// not, so the result always equals the double predicate; sums in between, and pairs whose
// float differences are near L/2 on some axis (where the image shift matters), take it.
__device__ __forceinline__ bool linked(const Pred &P, float xi, float yi, float zi, float xj,
                                       float yj, float zj)
{
    const float dx = xi - xj, dy = yi - yj, dz = zi - zj;
    if (fabsf(dx) < P.nowrap[0] && fabsf(dy) < P.nowrap[1] && fabsf(dz) < P.nowrap[2]) {
        const float s = (dx * dx + dy * dy) + dz * dz;
        if (s < P.b2lo)
            return true;
        if (s > P.b2hi)
            return false;
    }
    return dist2(P, xi, yi, zi, xj, yj, zj) < P.b2;
}

// ---------------------------------------------------------------------------------------
// Lock-free union-find over sorted positions.  parent[i] packs (key << 32) | index, where
// key is the particle's original index; a root holds its own packed value.  Hooks always
// put the root with the larger key under the one with the smaller key, so every tree's
// root is its member with the smallest original index.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t uf_idx(uint64_t v) { return (uint32_t)v; }
__device__ __forceinline__ uint32_t uf_key(uint64_t v) { return (uint32_t)(v >> 32); }

// Returns the packed value of the root of x, halving the path on the way (only non-root
// entries are rewritten, so this never races with a hook, which only targets roots).
__device__ __forceinline__ uint64_t uf_find(uint64_t *P, uint32_t x)
{
    uint64_t px = ld_relaxed(P + x);
    while (uf_idx(px) != x) {
        uint32_t y = uf_idx(px);
        uint64_t py = ld_relaxed(P + y);
        if (uf_idx(py) != y)
            st_relaxed(P + x, py);
        x = y;
        px = py;
    }
    return px;
}

// Root lookup without writes.  Used once no hook can happen any more (the compress pass),
// so that every thread is the only writer of its own entry there.
__device__ __forceinline__ uint64_t uf_find_ro(const uint64_t *P, uint32_t x)
{
    uint64_t px = ld_relaxed(P + x);
    while (uf_idx(px) != x) {
        x = uf_idx(px);
        px = ld_relaxed(P + x);
    }
    return px;
}

__device__ __forceinline__ void uf_union(uint64_t *P, uint32_t a, uint32_t b)
{
    uint64_t ra = uf_find(P, a);
    uint64_t rb = uf_find(P, b);
    while (ra != rb) {
        if (ra > rb) {  // keys are unique, so packed order is key order
            uint64_t t = ra;
            ra = rb;
            rb = t;
        }
        uint32_t hi = uf_idx(rb);
        uint64_t old = atomicCAS((unsigned long long *)(P + hi), (unsigned long long)rb,
                                 (unsigned long long)ra);
        if (old == rb)
            return;
        rb = uf_find(P, hi);
        ra = uf_find(P, uf_idx(ra));
    }
}

// ---------------------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gtid_xcd() { return xcd_block() * blockDim.x + threadIdx.x; }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Orders the LDS accesses of a wave's lanes around it (LDS operations of one wave complete
// in issue order, so no wait is needed beyond keeping the compiler from moving them).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Inclusive sum over the lanes of a wave (lane l gets lanes 0..l): shifts by 1, 2, 4, 8 lanes
// inside each row of 16, then the totals of rows 0 and 0-1 broadcast into the rows above
// (data-parallel primitives of the wave64 VALU, no LDS traffic).  Every lane must be active.
__device__ __forceinline__ int wave_incl_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

}  // namespace fof

// ---------------------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files, called by the entry points).
// ---------------------------------------------------------------------------------------
namespace fof {
// Shape of the bucketed cell binning (fof_build.hip).  Cells are sorted in buckets of
// 2^sshift consecutive cell ids (sshift <= kBinSortShift, so a sorting block's per-cell
// table fits in LDS).  Particles are first placed by bucket of 2^shift cells (at most
// kBinMaxBuckets buckets, so a placing block's histogram fits in LDS); G blocks each stream
// one contiguous chunk of particles.  When a grid has more cells than kBinMaxBuckets
// sorting buckets hold, shift > sshift: each placed bucket is split once more, into
// 2^(shift - sshift) sorting buckets (two-level).  ok = false: too many cells even so,
// the per-particle counting sort is used instead.
constexpr int kBinMaxBuckets = 16384;
constexpr int kBinSortShift = 13;
constexpr int kBinMaxSplit = 6;   // at most 64 sorting buckets per placed bucket
constexpr int kBinMaxBlocks = 512;

struct BinShape {
    int shift;    // cells per placed bucket: 2^shift
    int sshift;   // cells per sorting bucket: 2^sshift
    int G;
    int64_t nbk;  // placed buckets
    int64_t nsb;  // sorting buckets
    int64_t chunk;
    bool ok;
};

__host__ __device__ inline BinShape bin_shape(int64_t n, int64_t ncell)
{
    BinShape b;
    // buckets of about 8192 particles (what one sorting block holds in registers), then
    // larger ones if there would be too many buckets
    b.sshift = 6;
    while (b.sshift < kBinSortShift && (ncell >> b.sshift) * 8192 > n)
        ++b.sshift;
    while (b.sshift < kBinSortShift &&
           ((ncell + (1ll << b.sshift) - 1) >> b.sshift) > kBinMaxBuckets)
        ++b.sshift;
    b.shift = b.sshift;
    while (b.shift < b.sshift + kBinMaxSplit &&
           ((ncell + (1ll << b.shift) - 1) >> b.shift) > kBinMaxBuckets)
        ++b.shift;
    b.nbk = (ncell + (1ll << b.shift) - 1) >> b.shift;
    b.nsb = (ncell + (1ll << b.sshift) - 1) >> b.sshift;
    int64_t g = (n + 32767) / 32768;
    b.G = (int)(g < 1 ? 1 : (g > kBinMaxBlocks ? kBinMaxBlocks : g));
    b.chunk = (n + b.G - 1) / b.G;
    // a split keeps the sorting buckets' bounds in the (bucket, block) table: nsb + 1 <=
    // nbk * G entries
    b.ok = n > 0 && ncell > 0 && b.nbk <= kBinMaxBuckets &&
           (b.shift == b.sshift || (1ll << (b.shift - b.sshift)) < b.G);
    return b;
}

struct Work {  // device pointers resolved from a fof_grid and a workspace base
    const BoxDesc *desc;
    Counters *ctr;
    int32_t *cell_count;
    int32_t *cell_start;
    int32_t *scan;
    int32_t *rank;
    float4 *sorted;
    uint64_t *parent;
    uint64_t *flags;
    uint32_t *keep;
    int32_t *keep_prefix;
    int32_t *cnt;
    int32_t *groot;
    int32_t *flist;       // sorted indices of the particles with a friend, ascending
    int32_t *dense_list;  // dense cell ids in discovery order
    int32_t *big_list;    // dense ids of cells too large for one wave
    int32_t *table;       // per dense cell: header, key bitmask, popcount prefix
    float4 *temp;         // staging for dense cells too large for LDS
    int32_t *tile_list;   // link tiles left to the windowed kernel
    int2 *edges;          // hooks deferred by the tiled kernel
    int32_t edge_cap;
    int32_t *cursors;     // work cursors of the dense passes, kCursorStride ints apart
    int64_t dense_edge_cap;  // deferred sparse-dense hooks Work::temp takes (pairs)
    int32_t *classify;    // per-chunk dense / big counts and their scans (binning)
    int32_t *bin_hist;    // bucketed binning: per (bucket, block) counts, then their scan
    int32_t nbox;
    int32_t block;
    int64_t n;
    int64_t ncell;
    int64_t ntiles;           // link tiles over all tiled boxes
    int64_t n_plain;          // particles of boxes without link tiles
    int32_t dense_threshold;  // cells with more particles take the clique path (< 0: never)
    int32_t dense_cap;        // dense cells with tables
    int32_t table_words;      // words of one key bitmask
    int32_t table_stride;     // int32 entries per dense-cell table
};

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                           hipStream_t s);
// exclusive scan of max(in[i], 0)
hipError_t launch_scan_nonneg(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                              hipStream_t s);
// exclusive scan of (in[i] != 0)
hipError_t launch_scan_nonzero(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                               hipStream_t s);
// exclusive scan over [K][vcap] of "(k, v) is the root of a component of at least min_size
// members" in per-sample forests, v < *nv (a device count)
hipError_t launch_scan_sample_keep(const int32_t *forest, const int32_t *cnt, const int32_t *nv,
                                   int64_t vcap, int32_t K, int32_t min_size, int32_t *out,
                                   int32_t *scratch, hipStream_t s);
hipError_t launch_scan_popc(const uint32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                            hipStream_t s);
int64_t scan_scratch_elems(int64_t n);

hipError_t launch_build(const Work &w, const float *pos, hipStream_t s);
// A helper stream and three events of one device: fof_link runs its dense-cell passes on
// the helper stream, concurrently with the sparse passes on the caller's stream.
struct SideStream {
    hipStream_t stream;
    hipEvent_t fork, cc, join;  // flags cleared; sparse-dense hooks listed; dense pairs done
};

hipError_t launch_link(const Work &w, int32_t *root, hipStream_t s, const SideStream *side);
hipError_t launch_dense_build(const Work &w, hipStream_t s, bool classified);
hipError_t launch_dense(const Work &w, hipStream_t s, hipEvent_t hooks_listed);
hipError_t launch_dense_hooks(const Work &w, hipStream_t s);
hipError_t launch_flag_list(const Work &w, hipStream_t s);
hipError_t launch_group_dispersion(const Work &w, int32_t cap, const int32_t *n_groups,
                                   const int32_t *sizes, const double *com, double *sigx,
                                   hipStream_t s);
size_t subhalo_scratch_bytes(int64_t n, int32_t G);
hipError_t launch_subhalo(const Work &w, const float *pos, const float *vel,
                          const int32_t *group_id, int32_t G, const int32_t *sizes,
                          const double *norm_x, const double *norm_v, double b6, void *scratch,
                          int32_t *sub, hipStream_t s);
hipError_t launch_backward_dispersion(const Work &w, const float *pos, const int32_t *group_id,
                                      int32_t G, const int32_t *sizes, const double *com,
                                      const double *sigx, const double *g_sigx, float *grad_pos,
                                      hipStream_t s);
hipError_t launch_groups(const Work &w, int32_t min_size, const float *vel, int32_t cap,
                         int32_t *group_id, int32_t *n_groups, int32_t *sizes, double *com,
                         double *vmean, double *sigv, hipStream_t s);
int sample_layout_ok(const fof_sample &S, int64_t n);
hipError_t launch_sample(const Work &w, const fof_sample &S, int32_t *root, hipStream_t s);
hipError_t launch_score(const Work &w, const fof_sample &S, const double *loss, int32_t baseline,
                        float *grad_pos, hipStream_t s);
hipError_t launch_groups_sampled(const Work &w, const fof_sample &S, int32_t min_size,
                                 int32_t cap, int32_t *n_groups, int32_t *sizes, double *com,
                                 hipStream_t s);
// Streaming labelling in z-slabs (fof_stream.hip).
struct SlabGeom {
    double Lz;     // box length along z
    double width;  // slab thickness, Lz / nslab
    double ghost;  // ghost layer on each side, >= b
    int32_t nslab;
};
int64_t slab_chunks(int64_t n);
int slab_max();
hipError_t launch_slab_count(const float *pos, int64_t n, const SlabGeom &G, int64_t *counts,
                             hipStream_t s);
hipError_t launch_slab_gather(const float *pos, int64_t n, const SlabGeom &G, int k,
                              int32_t *ccount, int32_t *coff, int32_t *scan_scratch, int64_t cap,
                              float *spos, int32_t *map, int32_t *status, hipStream_t s);
hipError_t launch_fuse_init(int32_t *root, int64_t n, hipStream_t s);
hipError_t launch_slab_fuse(const int32_t *map, const int32_t *sroot, int64_t m, int32_t *root,
                            hipStream_t s);
hipError_t launch_or_status(const Counters *from, int32_t *to, hipStream_t s);
hipError_t launch_fuse_final(int32_t *root, int64_t n, hipStream_t s);
hipError_t launch_backward(int64_t n, int32_t block, const int32_t *group_id, int32_t G,
                           const int32_t *sizes, const double *vmean, const double *sigv,
                           const float *vel, const double *g_com, const double *g_sigv,
                           float *grad_pos, float *grad_vel, hipStream_t s);
}  // namespace fof
