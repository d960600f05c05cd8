// Friends-of-Friends linking (paper Sec. 2 steps (iii)-(v), Alg. 2): candidate search over
// the 27-cell stencil of the coarse grid, the exact minimum-image predicate, and connected
// components by a lock-free union-find instead of a fixed number of label sweeps.
//
// Each particle tests every candidate in the neighbour cells that its own position can
// reach (a neighbour cell is skipped when the particle is farther than `reach` from the
// shared face), so every pair is tested from both ends (the tiled kernel tests a pair of
// its own particles once and marks both).  That lets a particle that finds no friend write
// its final label (itself) at once; only particles with at least one friend are marked in
// the flag bitmap and resolved by the compress pass.  Each friend pair is hooked once.
//
// Cells with clique tables (fof_dense.hip) are skipped here: the dense kernels link their
// own particles, and list the hooks of the ordinary particles around them (applied after
// these kernels), marking those that find a friend there; the compress pass then replaces
// any label written here for them.
#include "fof_internal.h"
#include "fof_tile.h"

namespace fof {

namespace {

// Where a hook goes.  DirectHook unions straight into the global forest.  DeferHook (the
// tiled kernel, which publishes its local forests with plain stores and so must not touch
// the global forest itself) appends the pair to a small LDS buffer, spilling to the global
// edge list, which k_link_edges unions after the kernel.  A pair that finds the global list
// full raises the block's overflow flag: the tile is then redone with direct hooks.
struct DirectHook {
    uint64_t *parent;
    __device__ void operator()(uint32_t a, uint32_t b) const { uf_union(parent, a, b); }
};

constexpr int kLocalEdges = 96;  // LDS edge buffer of the tiled kernel

struct DeferHook {
    int2 *lbuf;
    int *lcnt, *lover;
    int2 *gbuf;
    int *gcnt;
    int gcap;
    __device__ void operator()(uint32_t a, uint32_t b) const
    {
        const int k = atomicAdd(lcnt, 1);
        if (k < kLocalEdges) {
            lbuf[k] = make_int2((int)a, (int)b);
            return;
        }
        const int gk = atomicAdd(gcnt, 1);
        if (gk < gcap)
            gbuf[gk] = make_int2((int)a, (int)b);
        else
            *lover = 1;
    }
};

// Whether particle p (sorted index i) sits in a cell linked by the dense kernels.
__device__ __forceinline__ bool in_dense_cell(const Work &w, const BoxDesc &B, int ix, int iy,
                                              int iz)
{
    if (!(w.dense_cap > 0 && w.dense_threshold >= 0 && B.dense_ok))
        return false;
    const int64_t c0 = coarse_cell(B, ix, iy, iz);
    return w.cell_start[c0 + 1] - w.cell_start[c0] > w.dense_threshold && w.cell_count[c0] >= 0;
}

// Candidates of particle p (sorted index i, coarse cell (ix, iy, iz)) straight from global
// memory, one neighbour row (ox, oy) at a time: with cells z fastest, the row's cells
// iz + sz.lo .. iz + sz.hi are one contiguous run of particles unless the run wraps around
// the box along z (then two runs).  Cells with clique tables are cut out of a run (the
// dense passes make their pairs); a run whose total count is at most the dense threshold
// holds none, so the dense test costs a load only next to crowded cells.  Returns true if
// p has a friend; each pair is hooked from the end with the smaller original index, the
// rule every link path shares (the other end may be staged elsewhere).
__device__ bool link_particle_global(const Work &w, const BoxDesc &B, const Pred &P, int64_t i,
                                     float4 p, int ix, int iy, int iz)
{
    const bool box_dense = w.dense_cap > 0 && w.dense_threshold >= 0 && B.dense_ok;
    const int32_t oi = __float_as_int(p.w);
    bool has_friend = false;
    const AxisSpan sx = axis_span(p.x, ix, B.side[0], B.nc[0], B.reach);
    const AxisSpan sy = axis_span(p.y, iy, B.side[1], B.nc[1], B.reach);
    const AxisSpan sz = axis_span(p.z, iz, B.side[2], B.nc[2], B.reach);
    const int nz = B.nc[2];
    const int nx = sx.hi - sx.lo + 1, ny = sy.hi - sy.lo + 1;
    for (int kx = 0; kx < nx; ++kx) {
        const int cx = wrap_cell(ix + span_offset(sx, kx), B.nc[0]);
        for (int ky = 0; ky < ny; ++ky) {
            const int cy = wrap_cell(iy + span_offset(sy, ky), B.nc[1]);
            const int64_t row = coarse_cell(B, cx, cy, 0);
            int oz = sz.lo;
            while (oz <= sz.hi) {
                // the longest run of consecutive cells from iz + oz that does not wrap
                const int za = wrap_cell(iz + oz, nz);
                int zb = za;
                while (oz < sz.hi && zb + 1 < nz && wrap_cell(iz + oz + 1, nz) == zb + 1) {
                    ++oz;
                    ++zb;
                }
                ++oz;
                const int32_t a = w.cell_start[row + za], e = w.cell_start[row + zb + 1];
                const bool split = box_dense && e - a > w.dense_threshold;
                FOF_STAT(w.ctr, ST_PAIRS_GLOBAL, e - a);
                for (int z = za; z <= (split ? zb : za); ++z) {
                    int32_t j0 = a, j1 = e;
                    if (split) {  // one cell at a time, skipping those with clique tables
                        j0 = w.cell_start[row + z];
                        j1 = w.cell_start[row + z + 1];
                        if (j1 - j0 > w.dense_threshold && w.cell_count[row + z] >= 0)
                            continue;
                    }
                    for (int32_t j = j0; j < j1; ++j) {
                        if (j == i)
                            continue;
                        const float4 q = w.sorted[j];
                        if (linked(P, p.x, p.y, p.z, q.x, q.y, q.z)) {
                            has_friend = true;
                            if (oi < __float_as_int(q.w))
                                uf_union(w.parent, (uint32_t)i, (uint32_t)j);
                        }
                    }
                }
            }
        }
    }
    return has_friend;
}

__device__ __forceinline__ void finish_particle(const Work &w, int32_t *root, int64_t i,
                                                int32_t orig, bool has_friend)
{
    if (has_friend)
        atomicOr((unsigned long long *)(w.flags + (i >> 6)), 1ull << (i & 63));
    else
        root[orig] = orig;
}

// Per-particle kernel for boxes the tiled kernel does not take (fewer than 3 cells on an
// axis).  Dense-cell particles were marked by the dense kernels.
__global__ void k_link(Work w, int32_t *__restrict__ root)
{
    const int64_t i = gtid_xcd();
    if (i >= w.n)
        return;
    const BoxDesc &B = w.desc[find_box(w.desc, w.nbox, i)];
    if (B.tiled)
        return;
    const float4 p = w.sorted[i];
    const int ix = coarse_index(p.x, B, 0);
    const int iy = coarse_index(p.y, B, 1);
    const int iz = coarse_index(p.z, B, 2);
    if (in_dense_cell(w, B, ix, iy, iz))
        return;
    finish_particle(w, root, i, __float_as_int(p.w),
                    link_particle_global(w, B, pred_of(B), i, p, ix, iy, iz));
}

// ---------------------------------------------------------------------------------------
// LDS-tiled linking.  A block owns kTileX x kTileY x kTileZ coarse cells.  With cells z
// fastest, every (x, y) row of the tile's one-cell halo is one contiguous run of particles
// in cell order, so a particle's candidates in one neighbour row (up to three consecutive
// cells) form one contiguous LDS range once the halo is staged.  Staging is flat: staged
// slot s belongs to the halo cell whose offset range holds s, found by a fixed-length
// binary search, so each thread issues its few global loads back to back.  Cells with
// clique tables are not staged: particles reach them through their unit tables.
//
// k_link_tiled stages whole tiles.  A tile whose halo holds more than kTileCap particles is
// queued for k_link_windows, which stages it in z-windows (the longest runs of z-layers
// that fit) and searches a single z-layer too full to stage from global memory.  The
// windowed kernel needs many more registers, so it is kept out of the common path.
// ---------------------------------------------------------------------------------------
constexpr int kWindowBlocks = 1024;  // grid of the windowed kernel (it loops over the queue)

// Union-find over staged slots in LDS, keyed like the global one by original index (the w
// field of the staged particle): a hook puts the root with the larger key under the other,
// so a local root is its component's member with the smallest original index.
__device__ __forceinline__ int lds_find(int *lpar, int x)
{
    int px = lpar[x];
    while (px != x) {
        const int gx = lpar[px];
        if (gx != px)
            lpar[x] = gx;  // halving: only non-root entries are rewritten
        x = px;
        px = gx;
    }
    return x;
}

__device__ __forceinline__ void lds_union(int *lpar, const float4 *part, int a, int b)
{
    a = lds_find(lpar, a);
    b = lds_find(lpar, b);
    while (a != b) {
        if (__float_as_int(part[a].w) > __float_as_int(part[b].w)) {
            const int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(lpar + b, b, a) == b)  // b, the larger key, goes under a
            return;
        a = lds_find(lpar, a);
        b = lds_find(lpar, b);
    }
}

__device__ __forceinline__ int lds_find_ro(const int *lpar, int x)
{
    int px = lpar[x];
    while (px != x) {
        x = px;
        px = lpar[x];
    }
    return x;
}

// Sets the friend bit of sorted index i for every active lane with has_friend.  The lanes
// of a wave hold increasing sorted indices, so lanes sharing a 64-bit word are adjacent:
// their bits are OR-ed across the wave and the first lane of each word does one atomic.
__device__ __forceinline__ void flag_friends_wave(uint64_t *flags, bool active, int64_t i,
                                                  bool has_friend)
{
    const int lane = lane_id();
    const int64_t word = active ? (i >> 6) : -1;
    uint64_t v = (active && has_friend) ? (1ull << (i & 63)) : 0ull;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t w2 = __shfl_down(word, o, kWave);
        const uint64_t v2 = __shfl_down(v, o, kWave);
        if (lane + o < kWave && w2 == word)
            v |= v2;
    }
    const int64_t wprev = __shfl_up(word, 1, kWave);
    if (active && v && (lane == 0 || wprev != word))
        atomicOr((unsigned long long *)(flags + word), (unsigned long long)v);
}

// Candidates of particle p (sorted index i, own halo cell (hx, hy, hz)) in the staged
// window of the windowed kernel: neighbour row r's halo cells [z_first, ...] sit at LDS
// wb[r] + slot - hoff[...].  Returns whether p has a friend; pairs are hooked from the
// smaller original index.
template <class Hook>
__device__ __forceinline__ bool link_staged(const Work &w, const BoxDesc &B, const Pred &P,
                                            const float4 *part, const int *hoff, const int *gst,
                                            int64_t i, float4 p, int ls, int hx, int hy, int hz,
                                            int ix, int iy, int iz, const int *wb, int z_first,
                                            const Hook &hook)
{
    const int32_t oi = __float_as_int(p.w);
    bool has_friend = false;
    const AxisSpan sx = axis_span(p.x, ix, B.side[0], B.nc[0], B.reach);
    const AxisSpan sy = axis_span(p.y, iy, B.side[1], B.nc[1], B.reach);
    const AxisSpan sz = axis_span(p.z, iz, B.side[2], B.nc[2], B.reach);
    for (int ox = sx.lo; ox <= sx.hi; ++ox)
        for (int oy = sy.lo; oy <= sy.hi; ++oy) {
            const int row2 = (hx + ox) * kHY + hy + oy;
            const int rb2 = row2 * kHZ;
            const int shift = wb[row2] - hoff[rb2 + z_first];  // slot -> LDS
            const int a = hoff[rb2 + hz + sz.lo] + shift;
            const int e = hoff[rb2 + hz + sz.hi + 1] + shift;
            FOF_STAT(w.ctr, ST_PAIRS_TILED, e - a);
            for (int j = a; j < e; ++j) {
                if (j == ls)
                    continue;
                const float4 q4 = part[j];
                if (linked(P, p.x, p.y, p.z, q4.x, q4.y, q4.z)) {
                    has_friend = true;
                    if (oi < __float_as_int(q4.w)) {  // each pair hooked from one end
                        const int sj = j - shift;
                        const int hj = rb2 + last_le<kHZ>(hoff + rb2, sj);
                        FOF_STAT(w.ctr, ST_UNIONS, 1);
                        hook((uint32_t)i, (uint32_t)(gst[hj] + (sj - hoff[hj])));
                    }
                }
            }
        }
    return has_friend;
}

// Own particle k of wave `wid`'s own rows (the 4 rows with hx = 1 + wid): its staged slot and
// own halo cell.  c1, c2, c3 are the wave's cumulative own counts after its rows 0, 1, 2, so
// the row is found with three compares.
struct OwnSlot {
    int slot, hs;
};

__device__ __forceinline__ OwnSlot own_slot(const int *hoff, int wid, int k, int c1, int c2,
                                            int c3)
{
    const int r = (k >= c1) + (k >= c2) + (k >= c3);
    const int before = r == 0 ? 0 : (r == 1 ? c1 : (r == 2 ? c2 : c3));
    const int rb = ((1 + wid) * kHY + 1 + r) * kHZ;
    OwnSlot o;
    o.slot = hoff[rb + 1] + (k - before);
    o.hs = rb + 1 + last_le<kTileZ>(hoff + rb + 1, o.slot);
    return o;
}

// ---------------------------------------------------------------------------------------
// Pair queue of one wave.  A particle's candidates in one neighbour row are one contiguous
// range of staged slots, an item (particle slot, first slot, length).  Lanes test pairs,
// not particles: items are appended to a ring in LDS in the order the wave produces them,
// their pairs numbered consecutively, and each round lane l tests pair base + l.  A lane
// finds its item from markers: the items after `head` write a byte at their first pair's
// position in the round, and the lane counts the marks at or below its own position.  So
// every lane tests one pair per round however unequal the candidate counts are, where a
// loop per particle would keep the wave as long as its busiest lane.
// ---------------------------------------------------------------------------------------
constexpr int kRing = 128;  // live items never exceed 64 (pending) + 64 (one new row step)
constexpr int kSlotBits = 10;
static_assert(kTileCap <= (1 << kSlotBits), "staged slots are packed in 10 bits");

struct PairQueue {
    int head;   // ring index of the item holding pair `base` (or ending right at it)
    int tail;   // ring index past the last item
    int base;   // first pair not tested yet
    int total;  // pairs queued so far
};

struct TileLds {
    const float4 *part;
    int *lpar;
    const int *hoff, *gst;    // the halo table (a slot's sorted index, on the rare deferred hook)
    const uint64_t *ownw;     // bit per staged slot: an own particle of this tile
    unsigned char *fbyte;     // staged slots that have a friend
};

// Sorted index of staged slot sl: the halo cell whose offset range holds it, then its start.
__device__ __forceinline__ uint32_t slot_index(const int *hoff, const int *gst, int sl)
{
    const int h = last_le<kHalo>(hoff, sl);
    return (uint32_t)(gst[h] + (sl - hoff[h]));
}

// Appends each lane's item (candidate slots [a, a + len) of the particle in `slot`; len 0:
// none) to the wave's ring, numbering its pairs after those queued so far.
__device__ __forceinline__ void queue_push(int2 *ring, PairQueue &q, int a, int len, int slot,
                                           Counters *ctr)
{
    const int lane = lane_id();
    const int x = wave_incl_sum(len);
    const int ts = __builtin_amdgcn_readlane(x, kWave - 1);
    const uint64_t ne = __ballot(len > 0);
    if (len > 0) {
        const int idx = q.tail + __popcll(ne & ((1ull << lane) - 1ull));
        ring[idx & (kRing - 1)] = make_int2(q.total + x - len, a | (slot << kSlotBits));
    }
    q.tail += __popcll(ne);
    q.total += ts;
    if (lane == 0)
        FOF_STAT(ctr, ST_PAIRS_TILED, ts);
    wave_sync();  // ring stores before the rounds' loads
}

// Tests pairs [q.base, q.base + cnt) of the wave's queue, one per lane (cnt <= kWave).
template <class Hook>
__device__ __forceinline__ void queue_round(const Pred &P, const TileLds &T, const int2 *ring,
                                            unsigned char *mark, PairQueue &q,
                                            int cnt, const Hook &hook)
{
    const int lane = lane_id();
    const int it = q.head + 1 + lane;
    const int rel = it < q.tail ? ring[it & (kRing - 1)].x - q.base : kWave;
    if (rel < kWave)  // items after head start at pair base or later: rel >= 0
        mark[rel] = 1;
    wave_sync();  // the marks of every lane before any lane reads its own
    const uint64_t m = __ballot(mark[lane] != 0);
    mark[lane] = 0;
    const int mine = q.head + __popcll(m & ((2ull << lane) - 1ull));
    q.head += __popcll(m);
    if (lane < cnt) {
        const int2 iv = ring[mine & (kRing - 1)];
        const int ps = iv.y >> kSlotBits;
        const int j = (iv.y & ((1 << kSlotBits) - 1)) + (q.base + lane - iv.x);
        if (j != ps) {
            const float4 p = T.part[ps], c = T.part[j];
            if (linked(P, p.x, p.y, p.z, c.x, c.y, c.z)) {
                T.fbyte[ps] = 1;
                if ((T.ownw[j >> 6] >> (j & 63)) & 1ull) {  // tested only from here
                    T.fbyte[j] = 1;
                    if (T.lpar[ps] != T.lpar[j])  // one parent: already one set
                        lds_union(T.lpar, T.part, ps, j);
                } else if (__float_as_int(p.w) < __float_as_int(c.w)) {
                    // a halo particle's own tile tests the pair too: hooked from one end
                    hook(slot_index(T.hoff, T.gst, ps), slot_index(T.hoff, T.gst, j));
                }
            }
        }
    }
    q.base += cnt;
}

__global__ __launch_bounds__(kTileBlock, 5) void k_link_tiled(Work w, int32_t *__restrict__ root)
{
    constexpr int kWaves = kTileBlock / kWave;
    __shared__ float4 part[kTileCap];
    __shared__ int hoff[kHalo + 1];  // staged offset of each halo cell
    __shared__ int gst[kHalo];       // global (sorted) start, or -1 - dense id
    __shared__ int scr[kWaves];
    __shared__ int lpar[kTileCap];   // LDS union-find over staged slots
    __shared__ int2 lbuf[kLocalEdges];  // deferred hooks of this tile
    __shared__ int2 ring[kWaves][kRing];
    __shared__ uint64_t ownw[kTileCap / kWave];
    __shared__ uint64_t rowbad;      // bit r: halo row r is not one contiguous global run
    __shared__ int rstart[kRowsH];   // staged offset of each halo row
    __shared__ unsigned char fbyte[kTileCap];
    __shared__ unsigned char mark[kWaves][kWave];
    __shared__ int lcnt, lover, gbase;

    const int64_t tile = xcd_block();
    if (tile >= w.ntiles)
        return;
    const BoxDesc &B = uniform_box(w.desc, find_box_tile(w.desc, w.nbox, tile));
    const Pred P = pred_of(B);
    const TileGeom g = tile_geom(B, tile);
    const bool box_dense = w.dense_cap > 0 && w.dense_threshold >= 0 && B.dense_ok;
    const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;

    if (t == 0) {
        rowbad = 0;
        lcnt = 0;
        lover = 0;
    }
    mark[wid][lane] = 0;
#pragma unroll
    for (int k = 0; k < kStagePerT; ++k)
        fbyte[t + k * kTileBlock] = 0;
    const int total = build_halo(w, B, g, box_dense, hoff, gst, scr);
    if (t == 0)
        FOF_STAT(w.ctr, ST_TILES, 1);
    if (total > kTileCap) {  // block-uniform: the windowed kernel takes this tile
        if (t == 0) {
            FOF_STAT(w.ctr, ST_TILES_OVERFLOW, 1);
            w.tile_list[atomicAdd(&w.ctr->n_spill, 1)] = (int32_t)tile;
        }
        return;
    }
    // A halo row is staged by plain copying when its cells are one contiguous run of the
    // sorted particles: every cell starts where the run says (no clique cell cut out, no
    // wrap of the z index inside the row).
#pragma unroll
    for (int k = 0; k < kPerT; ++k) {
        const int h = t * kPerT + k;
        if (h < kHalo) {
            const int r0 = h - h % kHZ;
            if (gst[h] != gst[r0] + (hoff[h] - hoff[r0]) || gst[r0] < 0)
                atomicOr((unsigned long long *)&rowbad, 1ull << (h / kHZ));
        }
    }
    if (t < kRowsH)
        rstart[t] = hoff[t * kHZ];
    __syncthreads();
    // staging, slot by slot: the row by a search over the 36 row starts, then a plain offset
    // into the row's run (or, in a row that is not one run, a search over its cells).  The
    // own-slot bitmap comes out of the same pass: a wave's lanes hold 64 consecutive slots.
    const uint64_t bad = rowbad;
#pragma unroll
    for (int k = 0; k < kStagePerT; ++k) {  // LDS stores cannot alias the global loads
        const int sl = t + k * kTileBlock;
        bool own = false;
        if (sl < total) {
            const int row = last_le<kRowsH>(rstart, sl);
            const int rb = row * kHZ;
            int src;
            if (!((bad >> row) & 1ull)) {
                src = gst[rb] + (sl - rstart[row]);
            } else {
                const int h = rb + last_le<kHZ>(hoff + rb, sl);
                src = gst[h] + (sl - hoff[h]);
            }
            const int hx = row / kHY, hy = row - hx * kHY;
            own = hx >= 1 && hx < g.hxe && hy >= 1 && hy < g.hye && sl >= hoff[rb + 1] &&
                  sl < hoff[rb + g.hze];
            part[sl] = w.sorted[src];
            lpar[sl] = sl;
        }
        const uint64_t ob = __ballot(own);
        if (lane == 0)
            ownw[sl >> 6] = ob;
    }
    __syncthreads();

    // own particles: wave wid takes the own rows with hx = 1 + wid
    const bool own_plane = 1 + wid < g.hxe;
    int c1 = 0, c2 = 0, c3 = 0, nown = 0;
    if (own_plane) {
        int acc = 0;
#pragma unroll
        for (int r = 0; r < kTileY; ++r) {
            const int rb = ((1 + wid) * kHY + 1 + r) * kHZ;
            if (1 + r < g.hye)
                acc += hoff[rb + g.hze] - hoff[rb + 1];
            if (r == 0)
                c1 = acc;
            else if (r == 1)
                c2 = acc;
            else if (r == 2)
                c3 = acc;
        }
        nown = acc;
    }
    if (lane == 0)
        FOF_STAT(w.ctr, ST_OWN_STAGED, nown);
    // phase A: candidate search through the wave's pair queue; pairs of own particles are
    // joined in LDS, every other hook (halo particles of other tiles) is deferred to the
    // edge list
    const DeferHook hook{lbuf, &lcnt, &lover, w.edges, &w.ctr->n_link_edges, w.edge_cap};
    const TileLds T{part, lpar, hoff, gst, ownw, fbyte};
    int2 *wring = ring[wid];
    unsigned char *wmark = mark[wid];
    PairQueue q{0, 0, 0, 0};
    for (int k0 = 0; k0 < nown; k0 += kWave) {  // wave-uniform
        const int k = k0 + lane;
        const bool act = k < nown;
        int slot = 0, hx = 0, hy = 0, hz = 0, nrow = 0, ny = 1;
        AxisSpan sx{0, 0}, sy{0, 0}, sz{0, 0};
        if (act) {
            const OwnSlot o = own_slot(hoff, wid, k, c1, c2, c3);
            slot = o.slot;
            const float4 p = part[slot];
            hz = o.hs % kHZ;
            hy = (o.hs / kHZ) % kHY;
            hx = o.hs / (kHZ * kHY);
            sx = axis_span(p.x, g.x0 - 1 + hx, B.side[0], B.nc[0], B.reach);
            sy = axis_span(p.y, g.y0 - 1 + hy, B.side[1], B.nc[1], B.reach);
            sz = axis_span(p.z, g.z0 - 1 + hz, B.side[2], B.nc[2], B.reach);
            ny = sy.hi - sy.lo + 1;
            nrow = (sx.hi - sx.lo + 1) * ny;
        }
        for (int s = 0; __ballot(s < nrow) != 0; ++s) {
            // the row's candidates, cut to the pairs this particle tests: each pair of own
            // particles is tested once, from the lower halo row or, in one row, from the
            // lower slot, so an own row below this particle's row contributes its halo cells
            // only and its own row the slots above its own
            int a1 = 0, l1 = 0, a2 = 0, l2 = 0;
            if (s < nrow) {
                const int kx = s / ny, ky = s - kx * ny;
                const int qx = hx + span_offset(sx, kx), qy = hy + span_offset(sy, ky);
                const int rq = qx * kHY + qy, rb2 = rq * kHZ;
                const int a = hoff[rb2 + hz + sz.lo], e = hoff[rb2 + hz + sz.hi + 1];
                a1 = a;
                if (rq > hx * kHY + hy || qx < 1 || qx >= g.hxe || qy < 1 || qy >= g.hye) {
                    l1 = e - a;
                } else {
                    l1 = max(0, min(e, hoff[rb2 + 1]) - a);
                    a2 = max(a, rq == hx * kHY + hy ? slot + 1 : hoff[rb2 + g.hze]);
                    l2 = max(0, e - a2);
                }
            }
            queue_push(wring, q, a1, l1, slot, w.ctr);
            while (q.total - q.base >= kWave)
                queue_round(P, T, wring, wmark, q, kWave, hook);
            if (__ballot(l2 > 0) != 0) {
                queue_push(wring, q, a2, l2, slot, w.ctr);
                while (q.total - q.base >= kWave)
                    queue_round(P, T, wring, wmark, q, kWave, hook);
            }
        }
    }
    if (q.total > q.base)
        queue_round(P, T, wring, wmark, q, q.total - q.base, hook);
    __syncthreads();
    {  // move the LDS edge buffer to the global list
        const int nl = min(lcnt, kLocalEdges);
        if (t == 0)
            gbase = nl ? atomicAdd(&w.ctr->n_link_edges, nl) : 0;
        __syncthreads();
        if (t < nl) {
            if (gbase + t < w.edge_cap)
                w.edges[gbase + t] = lbuf[t];
            else
                lover = 1;
        }
    }
    __syncthreads();
    // phase B: publish the local forest.  No thread of this kernel hooks in the global
    // forest, so every own entry still holds itself and a plain store points it at its local
    // root.  Particles with no friend write their final label; the others set their bit of
    // the flag bitmap, one atomic per word and wave.  The rings are free now: they hold the
    // sorted index of every own slot, which local roots (own slots) are looked up in.
    int *gown = reinterpret_cast<int *>(&ring[0][0]);
    static_assert(sizeof(ring) >= kTileCap * sizeof(int), "own indices fit the rings");
    for (int k = lane; k < nown; k += kWave) {
        const OwnSlot o = own_slot(hoff, wid, k, c1, c2, c3);
        gown[o.slot] = gst[o.hs] + (o.slot - hoff[o.hs]);
    }
    __syncthreads();
    for (int k0 = 0; k0 < nown; k0 += kWave) {  // wave-uniform
        const int k = k0 + lane;
        const bool act = k < nown;
        int64_t i = 0;
        bool f = false;
        if (act) {
            const int slot = own_slot(hoff, wid, k, c1, c2, c3).slot;
            i = gown[slot];
            f = fbyte[slot] != 0;
            if (!f) {
                const int32_t oi = __float_as_int(part[slot].w);
                root[oi] = oi;
            } else {
                const int lr = lds_find_ro(lpar, slot);
                if (lr != slot)
                    w.parent[i] = ((uint64_t)(uint32_t)__float_as_int(part[lr].w) << 32) |
                                  (uint32_t)gown[lr];
            }
        }
        flag_friends_wave(w.flags, act, i, f);
    }
    __syncthreads();
    if (t == 0 && lover)  // some hooks were lost: the windowed kernel redoes the tile
        w.tile_list[atomicAdd(&w.ctr->n_spill, 1)] = (int32_t)tile;
}

// The hooks the tiled kernel deferred, now that every local forest is published.
__global__ void k_link_edges(Work w)
{
    const int64_t m = min(w.ctr->n_link_edges, w.edge_cap);
    for (int64_t e = gtid(); e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int2 ab = w.edges[e];
        uf_union(w.parent, (uint32_t)ab.x, (uint32_t)ab.y);
    }
}

// Tiles queued by k_link_tiled, each staged in z-windows: own layers [za, zb) with halo
// layers [za - 1, zb].  Window bounds come from LDS values every thread reads alike, so
// all threads of a block take the same windows.
__global__ __launch_bounds__(kTileBlock) void k_link_windows(Work w, int32_t *__restrict__ root)
{
    __shared__ float4 part[kTileCap];
    __shared__ int hoff[kHalo + 1];
    __shared__ int gst[kHalo];
    __shared__ int colsum[kHZ];        // particles per halo z-layer
    __shared__ int wbase[kRowsH + 1];  // LDS start of each halo row's part of the window
    __shared__ int ownoff[kOwnRows + 1];
    __shared__ int scr[kTileBlock / kWave];

    const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
    const int nq = w.ctr->n_spill;
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {
        const int64_t tile = w.tile_list[q];
        const BoxDesc &B = uniform_box(w.desc, find_box_tile(w.desc, w.nbox, tile));
        const Pred P = pred_of(B);
        const TileGeom g = tile_geom(B, tile);
        const bool box_dense = w.dense_cap > 0 && w.dense_threshold >= 0 && B.dense_ok;
        build_halo(w, B, g, box_dense, hoff, gst, scr);
        if (t < kHZ) {
            int c = 0;
            for (int row = 0; row < kRowsH; ++row)
                c += hoff[row * kHZ + t + 1] - hoff[row * kHZ + t];
            colsum[t] = c;
        }
        __syncthreads();
        int za = 1;
        while (za < g.hze) {
            int tot = colsum[za - 1] + colsum[za] + colsum[za + 1];
            int zb = za + 1;
            const bool fits = tot <= kTileCap;
            if (fits)
                while (zb < g.hze && tot + colsum[zb + 1] <= kTileCap)
                    tot += colsum[++zb];
            if (wid == 0) {  // row r's halo cells [za-1, zb] go to LDS [wbase[r], wbase[r+1])
                const int n =
                    lane < kRowsH ? hoff[lane * kHZ + zb + 1] - hoff[lane * kHZ + za - 1] : 0;
                int x = n;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    int y = __shfl_up(x, o, kWave);
                    if (lane >= o)
                        x += y;
                }
                if (lane < kRowsH)
                    wbase[lane] = x - n;
                if (lane == kRowsH - 1)
                    wbase[kRowsH] = x;
            }
            if (t <= kOwnRows) {  // own particles of the window before each own row
                int acc = 0;
                for (int r = 0; r < t; ++r) {
                    const int hx = 1 + r / kTileY, hy = 1 + r % kTileY;
                    const int rb = (hx * kHY + hy) * kHZ;
                    if (hx < g.hxe && hy < g.hye)
                        acc += hoff[rb + zb] - hoff[rb + za];
                }
                ownoff[t] = acc;
            }
            __syncthreads();
            if (fits) {
                for (int l = t; l < wbase[kRowsH]; l += kTileBlock) {
                    const int row = last_le<kRowsH>(wbase, l);
                    const int slot = hoff[row * kHZ + za - 1] + (l - wbase[row]);
                    // search the row's own kHZ cells only (reads stay inside hoff)
                    const int h = row * kHZ + last_le<kHZ>(hoff + row * kHZ, slot);
                    part[l] = w.sorted[gst[h] + (slot - hoff[h])];
                }
            }
            __syncthreads();
            const int nown = ownoff[kOwnRows];
            if (t == 0)
                FOF_STAT(w.ctr, fits ? ST_OWN_STAGED : ST_OWN_GLOBAL, nown);
            for (int k = t; k < nown; k += kTileBlock) {
                int r = 0;
                while (ownoff[r + 1] <= k)
                    ++r;
                const int row = (1 + r / kTileY) * kHY + 1 + r % kTileY;
                const int rb = row * kHZ;
                const int slot = hoff[rb + za] + (k - ownoff[r]);
                const int hz = last_le<kHZ>(hoff + rb, slot);  // own cell, inside the row
                const int64_t i = gst[rb + hz] + (slot - hoff[rb + hz]);
                const int hx = row / kHY, hy = row % kHY;
                const int ix = g.x0 - 1 + hx, iy = g.y0 - 1 + hy, iz = g.z0 - 1 + hz;
                bool f;
                float4 p;
                if (fits) {
                    const int ls = wbase[row] + slot - hoff[rb + za - 1];
                    p = part[ls];
                    f = link_staged(w, B, P, part, hoff, gst, i, p, ls, hx, hy, hz, ix, iy, iz,
                                    wbase, za - 1, DirectHook{w.parent});
                } else {
                    p = w.sorted[i];
                    f = link_particle_global(w, B, P, i, p, ix, iy, iz);
                }
                finish_particle(w, root, i, __float_as_int(p.w), f);
            }
            za = zb;
            __syncthreads();  // the next window reuses part, wbase and ownoff
        }
    }
}

// Particles with a friend (the flagged list): follow the union-find to the root and write
// the root's key (its original index, the smallest in the component) as the label.  Also
// leaves every flagged entry pointing straight at its root for the group passes.  The lookup must not
// halve paths: a halving write by one thread could replace the root another thread has
// just stored in its own entry with a stale grandparent.
__global__ void k_compress(const float4 *__restrict__ sorted, const int32_t *__restrict__ list,
                           const Counters *__restrict__ ctr, uint64_t *__restrict__ parent,
                           int32_t *__restrict__ root)
{
    const int64_t nf = ctr->n_flagged;
    for (int64_t k = gtid(); k < nf; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)list[k];
        const uint64_t r = uf_find_ro(parent, i);
        st_relaxed(parent + i, r);
        root[__float_as_int(sorted[i].w)] = (int32_t)uf_key(r);
    }
}

}  // namespace

// The components and dense-pair passes touch only dense-cell particles (their parent
// entries, and flag words through atomic ORs); the sparse-dense pass only lists its hooks
// (and ORs flag words); the tiled pass touches only ordinary particles, with plain stores to
// their own entries and no global hooks; the deferred, windowed and global sparse kernels
// hook ordinary particles only.  So with a helper stream all dense passes run concurrently
// with those kernels: fork after the flag fill.  The listed sparse-dense hooks are applied
// once the tiled kernel's plain stores are done (and the list is complete), beside the
// dense pairs (both hook through the lock-free forest).  Join before compress.
hipError_t launch_link(const Work &w, int32_t *root, hipStream_t s, const SideStream *side)
{
    if (w.n <= 0)
        return hipSuccess;
    hipError_t e = launch_fill_u64(w.flags, (w.n + 63) / 64, 0ull, s);
    if (e != hipSuccess)
        return e;
    const bool fork = side && w.ntiles > 0 && w.dense_cap > 0 && w.dense_threshold >= 0;
    if (fork) {
        if ((e = hipEventRecord(side->fork, s)) != hipSuccess ||
            (e = hipStreamWaitEvent(side->stream, side->fork, 0)) != hipSuccess)
            return e;
    }
    e = launch_dense(w, fork ? side->stream : s, fork ? side->cc : nullptr);
    if (e != hipSuccess)
        return e;
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    if (w.ntiles > 0) {
        e = launch_fill_i32(&w.ctr->n_spill, 2, 0, s);  // n_spill, n_link_edges
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_link_tiled, dim3((unsigned)w.ntiles), dim3(kTileBlock), 0, s, w,
                           root);
        hipLaunchKernelGGL(k_link_edges, dim3(1024), dim3(256), 0, s, w);
        const unsigned wb = (unsigned)(w.ntiles < kWindowBlocks ? w.ntiles : kWindowBlocks);
        hipLaunchKernelGGL(k_link_windows, dim3(wb), dim3(kTileBlock), 0, s, w, root);
    }
    if (w.n_plain > 0)  // boxes too small for tiles
        hipLaunchKernelGGL(k_link, dim3(nb), dim3(w.block), 0, s, w, root);
    if (fork && (e = hipStreamWaitEvent(s, side->cc, 0)) != hipSuccess)
        return e;
    e = launch_dense_hooks(w, s);  // after every plain store of the tiled kernel
    if (e != hipSuccess)
        return e;
    if (fork) {
        if ((e = hipEventRecord(side->join, side->stream)) != hipSuccess ||
            (e = hipStreamWaitEvent(s, side->join, 0)) != hipSuccess)
            return e;
    }
    // the flagged particles, listed once for compress and the group passes
    e = launch_flag_list(w, s);
    if (e != hipSuccess)
        return e;
    const unsigned lb = nb < 4096u ? nb : 4096u;
    hipLaunchKernelGGL(k_compress, dim3(lb), dim3(w.block), 0, s, w.sorted, w.flist, w.ctr,
                       w.parent, root);
    return hipGetLastError();
}

}  // namespace fof
