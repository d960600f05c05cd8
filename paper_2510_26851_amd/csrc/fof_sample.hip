// Stochastic linking and the score-function gradient (paper Sec. 3.2).
//
// Candidate edges are the pairs closer than the plan's linking length (the cut radius);
// edge e = {i, j} is kept in sample s when u(seed, s, i, j) < p_e, p_e = 1/(1 + exp(-z_e)),
// z_e = (b - d_e)/tau, or the paper's z_e = alpha (b^2 - d_e^2)/b^2.  The neighbour structure is built once and reused by all K samples,
// as the paper does ("we do not rebuild the neighbor list").
//
//   k_edges(_tiled) candidate search (the hard link's grid, LDS tiles and predicate, with
//                  the cut radius), edges as original indices i < j, their squared distance
//                  and sorted positions
//   k_touch, scan  compact the particles that touch an edge: one union-find per sample over
//                  those only, in original-index order
//   k_sample_union one thread per (edge, sample): Philox uniform, keep, hook
//   k_sample_label labels of every particle in every sample (smallest member index): a
//                  stream of identity labels, then the particles that touch an edge (only
//                  when the caller asks for the K x n label arrays)
//   k_sg_*, scan   per-sample groups over the touched particles: flatten each forest and
//                  count members, number the kept roots in ascending order (one scan over
//                  all samples), FP64 minimum-image sums about the root, centre and size
//   k_score        per edge: w_e = (1/K) sum_s adv_s (y_es - p_e), and -+ w_e (x_i - x_j)
//                  c_e, c_e = 1/(tau d_e) or 2 alpha / b^2, added in 64-bit fixed point to
//                  the sums of both ends (so the result does not depend on the order)
//   k_score_out    those sums scaled back into the float position gradient
#include "fof_internal.h"
#include "fof_tile.h"

namespace fof {

namespace {

constexpr int kBlock = 256;

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64x64->128-bit
// products; the key advances by the Weyl increments between rounds.
__device__ __forceinline__ uint64_t philox_first_word(uint64_t c0, uint64_t c1, uint64_t c2,
                                                      uint64_t c3, uint64_t k0, uint64_t k1)
{
    const uint64_t mA = 0xD2E7470EE14C6C93ull, mB = 0xCA5A826395121157ull;
    const uint64_t wA = 0x9E3779B97F4A7C15ull, wB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k0 += wA;
            k1 += wB;
        }
        const uint64_t h0 = __umul64hi(mA, c0), l0 = mA * c0;
        const uint64_t h1 = __umul64hi(mB, c2), l1 = mB * c2;
        const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
    }
    return c0;
}

__device__ __forceinline__ double edge_uniform(uint64_t seed, uint32_t s, uint32_t i, uint32_t j)
{
    const uint64_t w = philox_first_word((uint64_t)i | ((uint64_t)j << 32), (uint64_t)s, 0ull, 0ull,
                                         seed, 0ull);
    return (double)(w >> 11) * 0x1.0p-53;
}

struct SampleArgs {
    double b, tau, alpha;
    int32_t form;  // FOF_PROB_DISTANCE or FOF_PROB_QUADRATIC
    uint64_t seed;
    uint32_t s_first;  // global index of local sample 0
    int32_t K, edge_cap;
    int32_t *ei, *ej;
    double *d2;
    int32_t *n_edges;
    // scratch
    int32_t *vflag;    // [n] 1 + sorted index if the particle touches an edge, else 0
    int32_t *vmap;     // [n + 1] exclusive scan of (vflag != 0): local index
    int32_t *scan;     // scan tile sums
    int32_t *vlist;    // [vcap] local index -> original index (ascending)
    int32_t *vsorted;  // [vcap] local index -> sorted index
    int32_t *si, *sj;  // [edge_cap] sorted indices of the edge ends
    int32_t *forest;   // [K][vcap]
    int32_t *cnt;      // [K][vcap] members per root (per-sample groups)
    int32_t *gpre;     // [K * vcap + 1] exclusive scan of the kept roots
    int32_t *gscan;    // scan tile sums of gpre
    double *adv;       // [K] loss minus baseline
    uint8_t *keep;             // [edge_cap][8] keep bits of each edge, sample s at bit s of
                               // the 8 bytes (written when K <= 64)
    unsigned long long *acc;   // [3 vcap] score gradient of each touched particle, fixed point
    unsigned long long *amax;  // [1] bits of max_s |adv[s]| (non-negative doubles order as
                               // their bit patterns)
    int64_t vcap;
};

// Keep probability of an edge with squared distance d2 (Sec. 3.2).
__device__ __forceinline__ double edge_prob(double d2, const SampleArgs &a)
{
    const double z = a.form == FOF_PROB_QUADRATIC ? (a.alpha * (a.b * a.b - d2)) / (a.b * a.b)
                                                  : (a.b - sqrt(d2)) / a.tau;
    return 1.0 / (1.0 + exp(-z));
}

__device__ __forceinline__ int32_t edge_count(const SampleArgs &a)
{
    const int32_t m = *a.n_edges;
    return m < a.edge_cap ? m : a.edge_cap;
}

constexpr int kBlockEdges = 128;  // edges a tile block collects before writing them out

__device__ __forceinline__ void emit_edge(const Work &w, const SampleArgs &a, int32_t oi,
                                          int32_t oj, double s2, int32_t si, int32_t sj)
{
    const int32_t k = atomicAdd(a.n_edges, 1);
    if (k < a.edge_cap) {
        a.ei[k] = oi;
        a.ej[k] = oj;
        a.d2[k] = s2;
        a.si[k] = si;
        a.sj[k] = sj;
    } else {
        atomicOr(&w.ctr->status, (int32_t)FOF_STATUS_EDGE_CAP);
    }
}

__device__ void edges_of(const Work &w, const SampleArgs &a, int64_t i)
{
    const BoxDesc &B = w.desc[0];
    const float4 p = w.sorted[i];
    const int32_t oi = __float_as_int(p.w);
    const int ix = coarse_index(p.x, B, 0);
    const int iy = coarse_index(p.y, B, 1);
    const int iz = coarse_index(p.z, B, 2);
    // neighbour cells within reach of the particle (the cut radius plus the index error)
    const AxisSpan sx = axis_span(p.x, ix, B.side[0], B.nc[0], B.reach);
    const AxisSpan sy = axis_span(p.y, iy, B.side[1], B.nc[1], B.reach);
    const AxisSpan sz = axis_span(p.z, iz, B.side[2], B.nc[2], B.reach);
    for (int ox = sx.lo; ox <= sx.hi; ++ox) {
        const int cx = wrap_cell(ix + ox, B.nc[0]);
        for (int oy = sy.lo; oy <= sy.hi; ++oy) {
            const int cy = wrap_cell(iy + oy, B.nc[1]);
            for (int oz = sz.lo; oz <= sz.hi; ++oz) {
                const int cz = wrap_cell(iz + oz, B.nc[2]);
                const int64_t c = coarse_cell(B, cx, cy, cz);
                for (int32_t j = w.cell_start[c]; j < w.cell_start[c + 1]; ++j) {
                    const float4 q = w.sorted[j];
                    const int32_t oj = __float_as_int(q.w);
                    if (oj <= oi)
                        continue;  // each unordered pair once, from its lower index
                    const double s2 = dist2(B, p.x, p.y, p.z, q.x, q.y, q.z);
                    if (!(s2 < B.b2))
                        continue;
                    emit_edge(w, a, oi, oj, s2, (int32_t)i, j);
                }
            }
        }
    }
}

// Candidate edges of one tile (box with LDS tiles): the tile and its halo are staged
// (every cell, clique tables are not used here) and each own particle tests the LDS ranges
// of the neighbour rows its position can reach.  The exact double squared distance is
// computed for the pairs the (exact) predicate accepts.  A tile whose halo does not fit
// searches its own particles from global memory.
__global__ __launch_bounds__(kTileBlock) void k_edges_tiled(Work w, SampleArgs a)
{
    __shared__ float4 part[kTileCap];
    __shared__ int hoff[kHalo + 1];
    __shared__ int gst[kHalo];
    __shared__ int ownoff[kOwnRows + 1];
    __shared__ int scr[kTileBlock / kWave];
    // edges of this block, written out with one counter update (one global counter bumped
    // by every edge would serialize)
    __shared__ int lei[kBlockEdges], lej[kBlockEdges], lsi[kBlockEdges], lsj[kBlockEdges];
    __shared__ double ld2[kBlockEdges];
    __shared__ int lcnt, lbase;

    const int64_t tile = xcd_block();
    if (tile >= w.ntiles)
        return;
    const BoxDesc &B = uniform_box(w.desc, 0);  // sampling plans hold one box
    const Pred P = pred_of(B);
    const TileGeom g = tile_geom(B, tile);
    const int t = threadIdx.x;
    const int total = build_halo(w, B, g, false, hoff, gst, scr);
    if (t <= kOwnRows) {  // own particles before each own row
        int acc = 0;
        for (int r = 0; r < t; ++r) {
            const int hx = 1 + r / kTileY, hy = 1 + r % kTileY;
            const int rb = (hx * kHY + hy) * kHZ;
            if (hx < g.hxe && hy < g.hye)
                acc += hoff[rb + g.hze] - hoff[rb + 1];
        }
        ownoff[t] = acc;
    }
    const bool staged = total <= kTileCap;  // block-uniform
    if (t == 0)
        lcnt = 0;
    if (staged) {
#pragma unroll
        for (int k = 0; k < kStagePerT; ++k) {
            const int sl = t + k * kTileBlock;
            if (sl < total) {
                const int h = last_le<kHalo>(hoff, sl);
                part[sl] = w.sorted[gst[h] + (sl - hoff[h])];
            }
        }
    }
    __syncthreads();
    const int nown = ownoff[kOwnRows];
    for (int k = t; k < nown; k += kTileBlock) {
        int r = 0;
        while (ownoff[r + 1] <= k)
            ++r;
        const int rb = ((1 + r / kTileY) * kHY + 1 + r % kTileY) * kHZ;
        const int slot = hoff[rb + 1] + (k - ownoff[r]);
        const int hs = rb + 1 + last_le<kTileZ>(hoff + rb + 1, slot);
        const int64_t i = gst[hs] + (slot - hoff[hs]);
        if (!staged) {
            edges_of(w, a, i);
            continue;
        }
        const float4 p = part[slot];
        const int32_t oi = __float_as_int(p.w);
        const int hz = hs % kHZ, hy = (hs / kHZ) % kHY, hx = hs / (kHZ * kHY);
        const AxisSpan sx = axis_span(p.x, g.x0 - 1 + hx, B.side[0], B.nc[0], B.reach);
        const AxisSpan sy = axis_span(p.y, g.y0 - 1 + hy, B.side[1], B.nc[1], B.reach);
        const AxisSpan sz = axis_span(p.z, g.z0 - 1 + hz, B.side[2], B.nc[2], B.reach);
        for (int ox = sx.lo; ox <= sx.hi; ++ox)
            for (int oy = sy.lo; oy <= sy.hi; ++oy) {
                const int rb2 = ((hx + ox) * kHY + hy + oy) * kHZ;
                const int j0 = hoff[rb2 + hz + sz.lo], j1 = hoff[rb2 + hz + sz.hi + 1];
                for (int j = j0; j < j1; ++j) {
                    const float4 q = part[j];
                    const int32_t oj = __float_as_int(q.w);
                    if (oj <= oi || !linked(P, p.x, p.y, p.z, q.x, q.y, q.z))
                        continue;  // each unordered pair once, from its lower index
                    const double s2 = dist2(B, p.x, p.y, p.z, q.x, q.y, q.z);
                    const int hj = rb2 + last_le<kHZ>(hoff + rb2, j);
                    const int32_t sj = gst[hj] + (j - hoff[hj]);
                    const int l = atomicAdd(&lcnt, 1);
                    if (l < kBlockEdges) {
                        lei[l] = oi;
                        lej[l] = oj;
                        ld2[l] = s2;
                        lsi[l] = (int32_t)i;
                        lsj[l] = sj;
                    } else {
                        emit_edge(w, a, oi, oj, s2, (int32_t)i, sj);
                    }
                }
            }
    }
    __syncthreads();
    const int nl = min(lcnt, kBlockEdges);
    if (t == 0)
        lbase = nl ? atomicAdd(a.n_edges, nl) : 0;
    __syncthreads();
    for (int l = t; l < nl; l += kTileBlock) {
        const int k2 = lbase + l;
        if (k2 < a.edge_cap) {
            a.ei[k2] = lei[l];
            a.ej[k2] = lej[l];
            a.d2[k2] = ld2[l];
            a.si[k2] = lsi[l];
            a.sj[k2] = lsj[l];
        } else {
            atomicOr(&w.ctr->status, (int32_t)FOF_STATUS_EDGE_CAP);
        }
    }
}

__global__ void k_edges(Work w, SampleArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gtid(); i < w.n; i += stride)
        edges_of(w, a, i);
}

// Marks the particles that touch an edge with 1 + their sorted index (every writer of one
// entry stores the same value).
__global__ void k_touch(SampleArgs a)
{
    const int64_t m = edge_count(a), stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = gtid(); e < m; e += stride) {
        a.vflag[a.ei[e]] = a.si[e] + 1;
        a.vflag[a.ej[e]] = a.sj[e] + 1;
    }
}

__global__ void k_vlist(int64_t n, SampleArgs a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gtid(); i < n; i += stride) {
        const int32_t f = a.vflag[i];
        if (f) {
            const int32_t v = a.vmap[i];
            a.vlist[v] = (int32_t)i;
            a.vsorted[v] = f - 1;
        }
    }
}

__global__ void k_forest_init(int64_t n, SampleArgs a)
{
    const int64_t nv = a.vmap[n];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = gtid(); v < nv; v += stride)
        for (int32_t s = 0; s < a.K; ++s)
            a.forest[(int64_t)s * a.vcap + v] = (int32_t)v;
}

__device__ __forceinline__ int32_t ffind(const int32_t *f, int32_t x)
{
    for (;;) {
        const int32_t p = __hip_atomic_load(f + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (p == x)
            return x;
        x = p;
    }
}

// Hook the larger root under the smaller: local order is original-index order, so each
// tree's root is its member with the smallest original index.
__device__ __forceinline__ void funion(int32_t *f, int32_t a, int32_t b)
{
    for (;;) {
        a = ffind(f, a);
        b = ffind(f, b);
        if (a == b)
            return;
        if (a < b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(f + a, a, b) == a)
            return;
    }
}

// Samples [kSampleChunk * blockIdx.y, + kSampleChunk) of one item per thread: the item's
// data is read once per chunk, and chunks keep enough threads for the union latencies.
constexpr int kSampleChunk = 8;

__global__ void k_sample_union(SampleArgs a)
{
    const int64_t m = edge_count(a), stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t s0 = (int32_t)blockIdx.y * kSampleChunk, s1 = min(s0 + kSampleChunk, a.K);
    for (int64_t e = gtid(); e < m; e += stride) {
        const int32_t i = a.ei[e], j = a.ej[e];
        const int32_t vi = a.vmap[i], vj = a.vmap[j];
        const double p = edge_prob(a.d2[e], a);
        uint32_t bits = 0;
        for (int32_t s = s0; s < s1; ++s)
            if (edge_uniform(a.seed, a.s_first + (uint32_t)s, (uint32_t)i, (uint32_t)j) < p) {
                funion(a.forest + (int64_t)s * a.vcap, vi, vj);
                bits |= 1u << (s - s0);
            }
        if (a.K <= 64)  // the score pass reads the draws back instead of repeating them
            a.keep[8 * e + blockIdx.y] = (uint8_t)bits;
    }
}

// Labels of the K samples in two passes: every particle first gets itself (a coalesced
// stream; sample blockIdx.y), then the particles that touch a candidate edge, one thread
// per (particle, sample), get their tree's smallest original index.
__global__ void k_sample_label_self(int64_t n, int32_t *__restrict__ root)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int32_t *row = root + (int64_t)blockIdx.y * n;
    for (int64_t i = gtid(); i < n; i += stride)
        row[i] = (int32_t)i;
}

__global__ void k_sample_label(int64_t n, SampleArgs a, int32_t *__restrict__ root)
{
    const int64_t nv = a.vmap[n], stride = (int64_t)gridDim.x * blockDim.x;
    const int32_t s = (int32_t)blockIdx.y;
    const int32_t *f = a.forest + (int64_t)s * a.vcap;
    for (int64_t v = gtid(); v < nv; v += stride)
        root[(int64_t)s * n + a.vlist[v]] = a.vlist[ffind(f, (int32_t)v)];
}

// ---- per-sample groups (the halos of each sampled graph) ----------------------------
// Sample blockIdx.y, touched particles v < nv.  The forests are final (every union is done),
// so pointing each entry at its root cannot mislead a concurrent find: it only ever sees a
// parent or the root.
__global__ void k_sg_zero(int64_t n, SampleArgs a)
{
    const int64_t nv = a.vmap[n], stride = (int64_t)gridDim.x * blockDim.x;
    int32_t *c = a.cnt + (int64_t)blockIdx.y * a.vcap;
    for (int64_t v = gtid(); v < nv; v += stride)
        c[v] = 0;
}

__global__ void k_sg_flatten(int64_t n, SampleArgs a)
{
    const int64_t nv = a.vmap[n], stride = (int64_t)gridDim.x * blockDim.x;
    int32_t *f = a.forest + (int64_t)blockIdx.y * a.vcap;
    int32_t *c = a.cnt + (int64_t)blockIdx.y * a.vcap;
    for (int64_t v = gtid(); v < nv; v += stride) {
        const int32_t r = ffind(f, (int32_t)v);
        if (r != (int32_t)v)
            __hip_atomic_store(f + v, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        atomicAdd(c + r, 1);
    }
}

// Group number of the kept root r of sample k (its rank among that sample's kept roots).
__device__ __forceinline__ int32_t sg_group(const SampleArgs &a, int64_t k, int32_t r)
{
    const int64_t base = k * a.vcap;
    return a.gpre[base + r] - a.gpre[base];
}

// n_groups[k], the overflow flag, and the sums: each member adds its minimum-image offset
// from the root particle to its group's row of com (FP64); each kept root leaves its local
// index in its group's sizes slot for k_sg_final.
__global__ void k_sg_sum(int64_t n, Work w, SampleArgs a, int32_t min_size, int32_t cap,
                         int32_t *__restrict__ n_groups, int32_t *__restrict__ sizes,
                         double *__restrict__ com)
{
    const int64_t k = blockIdx.y, nv = a.vmap[n], stride = (int64_t)gridDim.x * blockDim.x;
    if (gtid() == 0) {
        const int32_t G = a.gpre[(k + 1) * a.vcap] - a.gpre[k * a.vcap];
        n_groups[k] = G;
        if (G > cap)
            atomicOr(&w.ctr->status, (int32_t)FOF_STATUS_OVERFLOW);
    }
    const int32_t *f = a.forest + k * a.vcap;
    const int32_t *c = a.cnt + k * a.vcap;
    const BoxDesc &B = w.desc[0];
    for (int64_t v = gtid(); v < nv; v += stride) {
        const int32_t r = f[v];
        if (c[r] < min_size)
            continue;
        const int32_t g = sg_group(a, k, r);
        if (g >= cap)
            continue;
        double *acc = com + 3 * (k * cap + g);
        if (r == (int32_t)v) {
            sizes[k * cap + g] = r;
            continue;  // the root's own offset is 0
        }
        const float4 p = w.sorted[a.vsorted[v]], q = w.sorted[a.vsorted[r]];
        atomicAdd(acc + 0, min_image((double)p.x - (double)q.x, B.L[0], B.halfL[0]));
        atomicAdd(acc + 1, min_image((double)p.y - (double)q.y, B.L[1], B.halfL[1]));
        atomicAdd(acc + 2, min_image((double)p.z - (double)q.z, B.L[2], B.halfL[2]));
    }
}

__global__ void k_sg_clear(SampleArgs a, int32_t cap, double *__restrict__ com)
{
    const int64_t k = blockIdx.y, stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t G = a.gpre[(k + 1) * a.vcap] - a.gpre[k * a.vcap];
    const int64_t m = 3 * (G < cap ? G : cap);
    double *row = com + 3 * k * cap;
    for (int64_t t = gtid(); t < m; t += stride)
        row[t] = 0.0;
}

// centre = wrap(x_root + sum / n), as the hard catalogue; sizes from the member counts.
__global__ void k_sg_final(Work w, SampleArgs a, int32_t cap, const int32_t *__restrict__ n_groups,
                           int32_t *__restrict__ sizes, double *__restrict__ com)
{
    const int64_t k = blockIdx.y, stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t G = n_groups[k] < cap ? n_groups[k] : cap;
    const BoxDesc &B = w.desc[0];
    for (int64_t g = gtid(); g < G; g += stride) {
        const int32_t r = sizes[k * cap + g];
        const int32_t m = a.cnt[k * a.vcap + r];
        const float4 q = w.sorted[a.vsorted[r]];
        const double x[3] = {(double)q.x, (double)q.y, (double)q.z};
        double *c = com + 3 * (k * cap + g);
        for (int d = 0; d < 3; ++d) {
            double v = x[d] + c[d] / (double)m;
            if (v >= B.L[d])
                v -= B.L[d];
            if (v < 0.0)
                v += B.L[d];
            c[d] = v;
        }
        sizes[k * cap + g] = m;
    }
}

// Advantage of each sample: loss minus baseline.
__global__ void k_advantage(const double *__restrict__ loss, int32_t K, int32_t baseline,
                            double *__restrict__ adv, unsigned long long *__restrict__ amax)
{
    const int s = threadIdx.x + blockIdx.x * blockDim.x;
    if (s >= K)
        return;
    double sum = 0.0;
    for (int k = 0; k < K; ++k)
        sum += loss[k];
    double beta = 0.0;
    if (baseline == FOF_BASELINE_MEAN)
        beta = sum / (double)K;
    else if (baseline == FOF_BASELINE_LOO && K > 1)
        beta = (sum - loss[s]) / (double)(K - 1);
    adv[s] = loss[s] - beta;
    atomicMax(amax, (unsigned long long)__double_as_longlong(fabs(adv[s])));
}

// Fixed-point unit of the score sums: every term f (x_i - x_j) of an edge is at most
// max_s |adv_s| times 1/tau (distance form: |x_i - x_j| <= d) or 2 alpha r / b^2 (quadratic
// form, r the plan's linking length, which bounds d); the unit makes that bound < 2^40, so
// a particle's 64-bit sum holds 2^23 such terms.  Integer sums are exact and commutative:
// the gradient does not depend on the order of the edges or of the atomics.
struct FixedUnit {
    int ex;     // bound < 2^ex; a term t is stored as llrint(t * 2^(40 - ex))
    bool zero;  // every advantage is 0: no term
    bool bad;   // a non-finite advantage
};

__device__ __forceinline__ FixedUnit fixed_unit(const Work &w, const SampleArgs &a)
{
    const double amax = __longlong_as_double((long long)*a.amax);
    const double r = sqrt(w.desc[0].b2);
    const double bound = amax * (a.form == FOF_PROB_QUADRATIC ? 2.0 * a.alpha * r / (a.b * a.b)
                                                              : 1.0 / a.tau);
    FixedUnit u;
    u.bad = !isfinite(bound);
    u.zero = !u.bad && !(bound > 0.0);
    int ex = 0;
    if (!u.bad && !u.zero)
        frexp(bound, &ex);
    u.ex = ex;
    return u;
}

__device__ void score_edge(const Work &w, const SampleArgs &a, int64_t e, const FixedUnit &fu)
{
    const int32_t i = a.ei[e], j = a.ej[e];
    const double p = edge_prob(a.d2[e], a);
    double wsum = 0.0;
    if (a.K <= 64) {  // the keep bits the union pass recorded
        const uint64_t y = *reinterpret_cast<const uint64_t *>(a.keep + 8 * e);
        for (int32_t s = 0; s < a.K; ++s)
            wsum += a.adv[s] * ((double)((y >> s) & 1ull) - p);
    } else {
        for (int32_t s = 0; s < a.K; ++s) {
            const double u =
                edge_uniform(a.seed, a.s_first + (uint32_t)s, (uint32_t)i, (uint32_t)j);
            wsum += a.adv[s] * ((u < p ? 1.0 : 0.0) - p);
        }
    }
    const double wgt = wsum / (double)a.K;
    const BoxDesc &B = w.desc[0];
    const float4 pi = w.sorted[a.si[e]], pj = w.sorted[a.sj[e]];
    const double dx = min_image((double)pi.x - (double)pj.x, B.L[0], B.halfL[0]);
    const double dy = min_image((double)pi.y - (double)pj.y, B.L[1], B.halfL[1]);
    const double dz = min_image((double)pi.z - (double)pj.z, B.L[2], B.halfL[2]);
    // distance form: (x_i - x_j)/d has no direction where the two particles coincide; such
    // an edge contributes no gradient (the symmetric subgradient of d at 0)
    const double d2e = a.d2[e];
    const double f = a.form == FOF_PROB_QUADRATIC ? wgt * (2.0 * a.alpha / (a.b * a.b))
                     : (d2e > 0.0 ? wgt / (a.tau * sqrt(d2e)) : 0.0);
    const double d[3] = {dx, dy, dz};
    unsigned long long *gi = a.acc + 3 * (int64_t)a.vmap[i];
    unsigned long long *gj = a.acc + 3 * (int64_t)a.vmap[j];
    for (int c = 0; c < 3; ++c) {
        const long long q = llrint(ldexp(f * d[c], 40 - fu.ex));
        atomicAdd(gi + c, (unsigned long long)(-q));
        atomicAdd(gj + c, (unsigned long long)q);
    }
}

__global__ void k_score(Work w, SampleArgs a)
{
    const FixedUnit fu = fixed_unit(w, a);
    if (fu.zero || fu.bad)
        return;  // no term, or NaN written by k_score_out
    const int64_t m = edge_count(a), stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = gtid(); e < m; e += stride)
        score_edge(w, a, e, fu);
}

// The fixed-point sums of the touched particles, scaled back (exactly, by a power of two)
// and rounded to float; the other particles keep the zeros filled before.
__global__ void k_score_out(int64_t n, Work w, SampleArgs a, float *__restrict__ grad)
{
    const FixedUnit fu = fixed_unit(w, a);
    if (fu.zero)
        return;
    const int64_t nv = a.vmap[n], stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = gtid(); v < nv; v += stride) {
        const int64_t o = a.vlist[v];
        for (int c = 0; c < 3; ++c)
            grad[3 * o + c] = fu.bad ? __builtin_nanf("")
                                     : (float)ldexp((double)(long long)a.acc[3 * v + c],
                                                    fu.ex - 40);
    }
}
unsigned blocks_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > (1 << 20))
        b = 1 << 20;  // grid-stride kernels cover the rest
    return (unsigned)(b > 0 ? b : 1);
}

// Grid of a grid-stride pass over the candidate edges, whose count (at most the capacity)
// is only known on the device: enough blocks to fill the chip, not one per possible edge.
unsigned edge_blocks(int64_t cap)
{
    const unsigned b = blocks_for(cap);
    return b < 2048u ? b : 2048u;
}

}  // namespace

// Scratch layout (256-byte aligned): vflag [n], vmap [n + 1], scan [tiles], vlist [vcap],
// si [cap], sj [cap], forest [K][vcap].  Fails when the scratch is too small.
static bool carve(const fof_sample &S, int64_t n, SampleArgs &a)
{
    char *base = (char *)S.scratch;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = base + o;
        o = (o + bytes + 255) / 256 * 256;
        return p;
    };
    a.vcap = 2 * (int64_t)S.edge_cap < n ? 2 * (int64_t)S.edge_cap : n;
    a.vflag = (int32_t *)take(4 * (size_t)n);
    a.vmap = (int32_t *)take(4 * ((size_t)n + 1));
    a.scan = (int32_t *)take(4 * (size_t)scan_scratch_elems(n));
    const size_t vc = (size_t)(a.vcap > 0 ? a.vcap : 1);
    a.vlist = (int32_t *)take(4 * vc);
    a.vsorted = (int32_t *)take(4 * vc);
    a.si = (int32_t *)take(4 * (size_t)(S.edge_cap > 0 ? S.edge_cap : 1));
    a.sj = (int32_t *)take(4 * (size_t)(S.edge_cap > 0 ? S.edge_cap : 1));
    a.forest = (int32_t *)take(4 * (size_t)S.K * vc);
    a.cnt = (int32_t *)take(4 * (size_t)S.K * vc);
    a.gpre = (int32_t *)take(4 * ((size_t)S.K * vc + 1));
    a.gscan = (int32_t *)take(4 * (size_t)scan_scratch_elems((int64_t)S.K * (int64_t)vc));
    a.adv = (double *)take(8 * (size_t)S.K);
    a.keep = (uint8_t *)take(8 * (size_t)(S.edge_cap > 0 ? S.edge_cap : 1));
    a.acc = (unsigned long long *)take(24 * vc);
    a.amax = (unsigned long long *)take(8);
    return o <= S.scratch_bytes;
}

static void fill_args(const fof_sample &S, SampleArgs &a)
{
    a.b = S.b;
    a.tau = S.tau;
    a.alpha = S.alpha;
    a.form = S.form;
    a.seed = S.seed;
    a.s_first = (uint32_t)S.s_first;
    a.K = S.K;
    a.edge_cap = S.edge_cap;
    a.ei = S.ei;
    a.ej = S.ej;
    a.d2 = S.d2;
    a.n_edges = S.n_edges;
}

int sample_layout_ok(const fof_sample &S, int64_t n)
{
    SampleArgs a;
    return carve(S, n, a) ? 1 : 0;
}

hipError_t launch_sample(const Work &w, const fof_sample &S, int32_t *root, hipStream_t s)
{
    SampleArgs a;
    fill_args(S, a);
    carve(S, w.n, a);
    hipError_t e = launch_fill_i32(a.n_edges, 1, 0, s);
    if (e != hipSuccess)
        return e;
    e = launch_fill_i32(a.vflag, w.n, 0, s);
    if (e != hipSuccess)
        return e;
    if (w.n > 0) {
        if (w.ntiles > 0)
            hipLaunchKernelGGL(k_edges_tiled, dim3((unsigned)w.ntiles), dim3(kTileBlock), 0, s,
                               w, a);
        else
            hipLaunchKernelGGL(k_edges, dim3(blocks_for(w.n)), dim3(kBlock), 0, s, w, a);
    }
    // edges at most edge_cap: the grid of the following kernels is sized for the cap
    hipLaunchKernelGGL(k_touch, dim3(edge_blocks(S.edge_cap)), dim3(kBlock), 0, s, a);
    e = launch_scan_nonzero(a.vflag, a.vmap, w.n, a.scan, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_vlist, dim3(blocks_for(w.n)), dim3(kBlock), 0, s, w.n, a);
    hipLaunchKernelGGL(k_forest_init, dim3(blocks_for(a.vcap)), dim3(kBlock), 0, s,
                       w.n, a);
    const unsigned chunks = (unsigned)((S.K + kSampleChunk - 1) / kSampleChunk);
    hipLaunchKernelGGL(k_sample_union, dim3(edge_blocks(S.edge_cap), chunks), dim3(kBlock), 0,
                       s, a);
    if (root) {
        const unsigned rows = (unsigned)S.K, nb = blocks_for(w.n);
        hipLaunchKernelGGL(k_sample_label_self, dim3(nb < 4096u ? nb : 4096u, rows), dim3(kBlock),
                           0, s, w.n, root);
        hipLaunchKernelGGL(k_sample_label, dim3(blocks_for(a.vcap), rows), dim3(kBlock), 0, s,
                           w.n, a, root);
    }
    return hipGetLastError();
}

hipError_t launch_groups_sampled(const Work &w, const fof_sample &S, int32_t min_size,
                                 int32_t cap, int32_t *n_groups, int32_t *sizes, double *com,
                                 hipStream_t s)
{
    SampleArgs a;
    fill_args(S, a);
    carve(S, w.n, a);
    const unsigned K = (unsigned)S.K, vb = edge_blocks(a.vcap);
    const unsigned cb = edge_blocks(cap);
    hipLaunchKernelGGL(k_sg_zero, dim3(vb, K), dim3(kBlock), 0, s, w.n, a);
    hipLaunchKernelGGL(k_sg_flatten, dim3(vb, K), dim3(kBlock), 0, s, w.n, a);
    hipError_t e = launch_scan_sample_keep(a.forest, a.cnt, a.vmap + w.n, a.vcap > 0 ? a.vcap : 1,
                                           S.K, min_size, a.gpre, a.gscan, s);
    if (e != hipSuccess)
        return e;
    if (cap > 0)
        hipLaunchKernelGGL(k_sg_clear, dim3(cb, K), dim3(kBlock), 0, s, a, cap, com);
    hipLaunchKernelGGL(k_sg_sum, dim3(vb, K), dim3(kBlock), 0, s, w.n, w, a, min_size, cap,
                       n_groups, sizes, com);
    if (cap > 0)
        hipLaunchKernelGGL(k_sg_final, dim3(cb, K), dim3(kBlock), 0, s, w, a, cap, n_groups,
                           sizes, com);
    return hipGetLastError();
}

hipError_t launch_score(const Work &w, const fof_sample &S, const double *loss, int32_t baseline,
                        float *grad_pos, hipStream_t s)
{
    SampleArgs a;
    fill_args(S, a);
    carve(S, w.n, a);
    hipError_t e = hipSuccess;
    if ((e = launch_fill_u64(reinterpret_cast<uint64_t *>(a.amax), 1, 0ull, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_advantage, dim3((S.K + 255) / 256), dim3(256), 0, s, loss, S.K, baseline,
                       a.adv, a.amax);
    if (grad_pos) {
        if ((e = launch_fill_u32((uint32_t *)grad_pos, 3 * w.n, 0u, s)) != hipSuccess ||
            (e = launch_fill_u64(reinterpret_cast<uint64_t *>(a.acc), 3 * (a.vcap > 0 ? a.vcap : 1), 0ull,
                                 s)) != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_score, dim3(edge_blocks(S.edge_cap)), dim3(kBlock), 0, s, w, a);
        hipLaunchKernelGGL(k_score_out, dim3(blocks_for(a.vcap)), dim3(kBlock), 0, s, w.n, w, a,
                           grad_pos);
    }
    return hipGetLastError();
}

}  // namespace fof
