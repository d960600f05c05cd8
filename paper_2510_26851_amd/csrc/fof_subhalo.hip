// Six-dimensional sub-halo pass (paper Sec. 2, sub-halo finding): a second Friends-of-Friends
// pass inside each host halo in phase space, two members linking when
//   d^2 = |mi(x_i - x_j)|^2 / norm_x[g] + |v_i - v_j|^2 / norm_v[g] < b6^2.
// Hosts are small next to the box (tens to thousands of members), so every pair of a host is
// tested, one block per host.  A host of up to kSubLds members is held whole in LDS with its
// union-find, its pair triangle cut into 64 x 64 tiles spread over the block's waves; a larger
// one streams its members a block at a time through LDS (positions and velocities) against
// each thread's own member held in registers, with hooks into the packed lock-free union-find
// over the host's member slots in HBM.  Every pair is first put to a float prefilter that
// settles all but near-ties and pairs near a wrap, which the FP64 test decides.  The label is
// the smallest original index of the phase-space component (the union-find's root key).
#include <algorithm>

#include "fof_internal.h"

namespace fof {

namespace {

constexpr int kSubBlock = 1024;
constexpr int kSubLds = 2048;  // hosts up to this size keep members and union-find in LDS
constexpr int kSubJ = 4;       // partners tested per step of the LDS path

// Every slot starts as a root of its own holding a valid particle index, so that a slot no
// particle fills (sizes inconsistent with group_id) is still safe to read.
__global__ void k_sub_init(int64_t n, uint64_t *__restrict__ par, int32_t *__restrict__ member)
{
    for (int64_t s = gtid(); s < n; s += (int64_t)gridDim.x * blockDim.x) {
        par[s] = (uint64_t)(uint32_t)s;
        member[s] = 0;
    }
}

// Members of each host, host by host: slot = off[g] + arrival order (any order within a host;
// the label does not depend on it).  Slots beyond the host's size or the buffer are dropped
// and flagged, so inconsistent sizes can never write out of bounds.  A union-find entry holds
// its parent's packed value, so the member's own index is kept beside it in member[].
__global__ void k_sub_scatter(int64_t n, const int32_t *__restrict__ group_id, int32_t G,
                              const int32_t *__restrict__ sizes, const int32_t *__restrict__ off,
                              int32_t *__restrict__ cur, uint64_t *__restrict__ par,
                              int32_t *__restrict__ member, Counters *__restrict__ ctr)
{
    const int64_t i = gtid();
    if (i >= n)
        return;
    const int32_t g = group_id[i];
    if (g < 0 || g >= G)
        return;
    const int32_t k = atomicAdd(cur + g, 1);
    const int64_t slot = (int64_t)off[g] + k;
    if (k >= sizes[g] || off[g] < 0 || slot >= n) {
        atomicOr(&ctr->status, (int32_t)FOF_STATUS_RANGE);
        return;
    }
    par[slot] = ((uint64_t)(uint32_t)i << 32) | (uint32_t)slot;
    member[slot] = (int32_t)i;
}

// d^2 of the six-dimensional metric, each squared norm summed ((c0*c0 + c1*c1) + c2*c2) in
// FP64 without contraction, so that the decision is the same as a plain evaluation.
__device__ __forceinline__ bool phase_friends(const BoxDesc &B, const float (&xi)[6],
                                              const float (&xj)[6], double inx, double inv,
                                              double bb)
{
#pragma clang fp contract(off)
    double d[6];
    for (int a = 0; a < 3; ++a)
        d[a] = min_image((double)xi[a] - (double)xj[a], B.L[a], B.halfL[a]);
    for (int a = 3; a < 6; ++a)
        d[a] = (double)xi[a] - (double)xj[a];
    const double sx = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    const double sv = (d[3] * d[3] + d[4] * d[4]) + d[5] * d[5];
    return sx / inx + sv / inv < bb;
}

// The same decision without the divisions for all but near-ties: with rx = 1/norm_x and
// rv = 1/norm_v rounded, sx*rx + sv*rv is within a few units in the last place of the exact
// expression's rounded value (every term is non-negative), far inside the 1e-12 margin; a
// NaN (0 * inf) fails both tests and falls through to the exact form.
__device__ __forceinline__ bool phase_friends_fast(const BoxDesc &B, const float (&xi)[6],
                                                   const float (&xj)[6], double inx,
                                                   double inv, double rx, double rv, double bb,
                                                   double lo, double hi)
{
#pragma clang fp contract(off)
    double d[6];
    for (int a = 0; a < 3; ++a)
        d[a] = min_image((double)xi[a] - (double)xj[a], B.L[a], B.halfL[a]);
    for (int a = 3; a < 6; ++a)
        d[a] = (double)xi[a] - (double)xj[a];
    const double sx = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    const double sv = (d[3] * d[3] + d[4] * d[4]) + d[5] * d[5];
    const double approx = sx * rx + sv * rv;
    if (approx > hi)
        return false;
    if (approx < lo)
        return true;
    return sx / inx + sv / inv < bb;
}

// Float prefilter of the same decision, for the pairs it can settle.  With u = 2^-24: each
// float difference is within u of the exact one (relative), its square within 3u, each sum
// of three squares within 5u (all terms non-negative), the factors rx, rv (1/norm rounded
// to double, then to float) within u + 2^-53, so sx*rx + sv*rv is within about 9u of the
// exact value E of the metric; FP64 evaluates E within a few 2^-53.  The thresholds
// b6^2 (1 -+ 2^-16), rounded to float, are 256u away from b6^2: a value below the lower one
// means E < b6^2, above the upper one E > b6^2.  A pair closer than nowrap (just under half
// the box) to a wrap on some axis, a NaN, or a host whose factors 1/norm or b6^2 lie
// outside [1e-15, 1e15] (q.on false; a factor may also be 0) is left to the FP64 test.  In
// that range a term near the thresholds is a normal float, and a square that underflows
// adds far less than the margin.
struct SubPre {
    float rx, rv, lo, hi, nowrap[3];
    bool on;
};

__device__ __forceinline__ SubPre sub_prefilter(const BoxDesc &B, double inx, double inv,
                                                double bb)
{
    SubPre q;
    q.rx = (float)(1.0 / inx);
    q.rv = (float)(1.0 / inv);
    q.lo = (float)(bb * (1.0 - 0x1p-16));
    q.hi = (float)(bb * (1.0 + 0x1p-16));
    for (int a = 0; a < 3; ++a)
        q.nowrap[a] = (float)(B.halfL[a] * (1.0 - 0x1p-20));
    const auto in_range = [](float f) { return f == 0.0f || (f >= 1e-15f && f <= 1e15f); };
    q.on = bb >= 1e-15 && bb <= 1e15 && in_range(q.rx) && in_range(q.rv);
    return q;
}

// +1: friends, 0: not friends, -1: left to the FP64 test.
__device__ __forceinline__ int phase_prefilter(const SubPre &q, const float (&xi)[6],
                                               const float (&xj)[6])
{
#pragma clang fp contract(off)
    float d[6];
    bool near_wrap = false;
    for (int a = 0; a < 3; ++a) {
        d[a] = xi[a] - xj[a];
        near_wrap |= !(fabsf(d[a]) < q.nowrap[a]);
    }
    for (int a = 3; a < 6; ++a)
        d[a] = xi[a] - xj[a];
    const float sx = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    const float sv = (d[3] * d[3] + d[4] * d[4]) + d[5] * d[5];
    const float e = sx * q.rx + sv * q.rv;
    if (near_wrap)
        return -1;
    return e < q.lo ? 1 : (e > q.hi ? 0 : -1);
}

// Union-find over local member slots in LDS: larger root hooked under the smaller, path
// halving rewrites only non-root entries.
__device__ __forceinline__ int lds_ld(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int lds_find(int *p, int x)
{
    int px = lds_ld(p + x);
    while (px != x) {
        const int py = lds_ld(p + px);
        if (py != px)
            __hip_atomic_store(p + x, py, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        x = px;
        px = py;
    }
    return x;
}

__device__ __forceinline__ void lds_union(int *p, int a, int b)
{
    a = lds_find(p, a);
    b = lds_find(p, b);
    while (a != b) {
        if (a > b) {
            const int t = a;
            a = b;
            b = t;
        }
        const int old = atomicCAS(p + b, b, a);
        if (old == b)
            return;
        b = lds_find(p, b);
        a = lds_find(p, a);
    }
}

__device__ __forceinline__ void load_member(const float *__restrict__ pos,
                                            const float *__restrict__ vel, int64_t o, float (&p)[6])
{
    for (int a = 0; a < 3; ++a) {
        p[a] = pos[3 * o + a];
        p[3 + a] = vel[3 * o + a];
    }
}

__global__ __launch_bounds__(kSubBlock) void k_sub_link(
    int64_t n, const BoxDesc *__restrict__ desc, int nbox, const float *__restrict__ pos,
    const float *__restrict__ vel, int32_t G, const int32_t *__restrict__ sizes,
    const int32_t *__restrict__ off, const int32_t *__restrict__ cur,
    const double *__restrict__ norm_x, const double *__restrict__ norm_v, double bb,
    uint64_t *__restrict__ par, const int32_t *__restrict__ member, int32_t *__restrict__ sub)
{
    __shared__ float hx[6][kSubLds];  // the whole host, or one tile per block on the HBM path
    __shared__ int lpar[kSubLds];
    __shared__ int lmin[kSubLds];
    const int32_t g = blockIdx.x;
    const int64_t base = off[g];
    int64_t m = min(cur[g], sizes[g]);
    if (base < 0 || base >= n)
        m = 0;
    else if (m > n - base)
        m = n - base;
    if (m <= 0)
        return;  // block-uniform
    uint64_t *P = par;
    const BoxDesc &B = desc[find_box(desc, nbox, member[base])];
    const double inx = norm_x[g], inv = norm_v[g];
    const bool metric_ok = inx > 0.0 && inv > 0.0;  // otherwise the host stays singletons
    if (m <= kSubLds) {  // block-uniform
        for (int k = threadIdx.x; k < m; k += kSubBlock) {
            float q[6];
            load_member(pos, vel, member[base + k], q);
            for (int a = 0; a < 6; ++a)
                hx[a][k] = q[a];
            lpar[k] = k;
            lmin[k] = INT32_MAX;
        }
        __syncthreads();
        if (metric_ok) {
            const double rx = 1.0 / inx, rv = 1.0 / inv;
            const double lo = bb * (1.0 - 1e-12), hi = bb * (1.0 + 1e-12);
            const SubPre pre = sub_prefilter(B, inx, inv, bb);
            const int mi = (int)m;
            // The pair triangle in 64 x 64 tiles (I <= J), dealt round-robin to the waves, so
            // that every wave tests about as many pairs (a wave per row of members would leave
            // the first rows' waves with all the work).  Lane = member i of tile row I.
            const int nt = (mi + kWave - 1) / kWave;
            const int ntp = nt * (nt + 1) / 2;
            const int lane = lane_id();
            for (int tp = (int)threadIdx.x / kWave; tp < ntp; tp += kSubBlock / kWave) {
                int I = 0, rem = tp;  // row-major over I: row I holds tiles J = I .. nt - 1
                while (rem >= nt - I) {
                    rem -= nt - I;
                    ++I;
                }
                const int J = I + rem;
                const int i = I * kWave + lane;
                const int jhi = min(J * kWave + kWave, mi);
                float mine[6];
                for (int a = 0; a < 6; ++a)
                    mine[a] = i < mi ? hx[a][i] : 0.f;
                int ri = i < mi ? i : 0;  // a root i had (it may have been hooked since)
                // all lanes of a wave read the same j (an LDS broadcast); j > i is masked.
                // Most friend pairs of a clump are already joined: j's root is looked up once
                // per wave, and a lane hooks only when its own root differs from it.
                // kSubJ values of j per step: their reads and tests are issued before any
                // hook, so the LDS latency of one overlaps the arithmetic of the others.
                for (int j0 = J * kWave; j0 < jhi; j0 += kSubJ) {
                    bool f[kSubJ];
#pragma unroll
                    for (int u = 0; u < kSubJ; ++u) {
                        const int j = min(j0 + u, jhi - 1);
                        const float other[6] = {hx[0][j], hx[1][j], hx[2][j],
                                                hx[3][j], hx[4][j], hx[5][j]};
                        const int pf = pre.on ? phase_prefilter(pre, mine, other) : -1;
                        f[u] = j0 + u < jhi && j0 + u > i && i < mi &&
                               (pf == 1 ||
                                (pf < 0 && phase_friends_fast(B, mine, other, inx, inv, rx, rv,
                                                              bb, lo, hi)));
                    }
#pragma unroll
                    for (int u = 0; u < kSubJ; ++u) {
                        if (!ballot(f[u]))
                            continue;
                        const int j = j0 + u;
                        const int rj = lds_find(lpar, j);
                        if (f[u] && ri != rj) {
                            ri = lds_find(lpar, i);
                            if (ri != rj) {
                                lds_union(lpar, i, j);
                                ri = lds_find(lpar, i);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < m; k += kSubBlock)
            atomicMin(lmin + lds_find(lpar, k), member[base + k]);
        __syncthreads();
        for (int k = threadIdx.x; k < m; k += kSubBlock)
            sub[member[base + k]] = lmin[lds_find(lpar, k)];
        return;
    }
    float (*tile)[kSubLds] = hx;
    const SubPre pre = sub_prefilter(B, inx, inv, bb);
    for (int64_t i0 = 0; i0 < m; i0 += kSubBlock) {
        const int64_t i = i0 + threadIdx.x;
        float mine[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (i < m)
            load_member(pos, vel, member[base + i], mine);
        for (int64_t j0 = i0; j0 < m; j0 += kSubBlock) {
            __syncthreads();  // the previous tile is no longer read
            const int64_t jl = j0 + threadIdx.x;
            if (jl < m) {
                float q[6];
                load_member(pos, vel, member[base + jl], q);
                for (int a = 0; a < 6; ++a)
                    tile[a][threadIdx.x] = q[a];
            }
            __syncthreads();
            if (i < m && metric_ok) {
                const int cnt = (int)min((int64_t)kSubBlock, m - j0);
                for (int t = 0; t < cnt; ++t) {
                    if (j0 + t <= i)
                        continue;
                    const float other[6] = {tile[0][t], tile[1][t], tile[2][t],
                                            tile[3][t], tile[4][t], tile[5][t]};
                    const int pf = pre.on ? phase_prefilter(pre, mine, other) : -1;
                    if (pf == 1 || (pf < 0 && phase_friends(B, mine, other, inx, inv, bb)))
                        uf_union(P, (uint32_t)(base + i), (uint32_t)(base + j0 + t));
                }
            }
        }
    }
    __syncthreads();
    for (int64_t k = threadIdx.x; k < m; k += kSubBlock)
        sub[member[base + k]] = (int32_t)uf_key(uf_find_ro(P, (uint32_t)(base + k)));
}

}  // namespace

size_t subhalo_scratch_bytes(int64_t n, int32_t G)
{
    return 256 + 12 * (size_t)n + 4 * (2 * (size_t)G + (size_t)scan_scratch_elems(G) + 2);
}

hipError_t launch_subhalo(const Work &w, const float *pos, const float *vel,
                          const int32_t *group_id, int32_t G, const int32_t *sizes,
                          const double *norm_x, const double *norm_v, double b6, void *scratch,
                          int32_t *sub, hipStream_t s)
{
    if (w.n <= 0)
        return hipSuccess;
    hipError_t e = launch_fill_i32(sub, w.n, -1, s);
    if (e != hipSuccess || G <= 0)
        return e;
    char *p = (char *)scratch;
    uint64_t *par = (uint64_t *)p;
    int32_t *member = (int32_t *)(p + 8 * (size_t)w.n);
    int32_t *off = member + w.n;
    int32_t *cur = off + G;
    int32_t *scan = cur + G;
    // a negative size counts as 0, so host ranges never overlap; its members are dropped
    // and flagged by the scatter (k >= sizes[g])
    if ((e = launch_scan_nonneg(sizes, off, G, scan, s)) != hipSuccess)
        return e;
    if ((e = launch_fill_i32(cur, G, 0, s)) != hipSuccess)
        return e;
    const unsigned ib = (unsigned)std::min<int64_t>((w.n + 1023) / 1024, 65536);
    hipLaunchKernelGGL(k_sub_init, dim3(ib), dim3(1024), 0, s, w.n, par, member);
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    hipLaunchKernelGGL(k_sub_scatter, dim3(nb), dim3(w.block), 0, s, w.n, group_id, G, sizes, off,
                       cur, par, member, w.ctr);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sub_link, dim3((unsigned)G), dim3(kSubBlock), 0, s, w.n, w.desc, w.nbox,
                       pos, vel, G, sizes, off, cur, norm_x, norm_v, b6 * b6, par, member, sub);
    return hipGetLastError();
}

}  // namespace fof
