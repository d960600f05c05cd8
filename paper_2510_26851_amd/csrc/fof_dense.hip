// Clique-cell path for dense cells.
//
// Inside a coarse cell that holds many particles, pair testing is quadratic.  The cell is
// cut into m^3 fine cells whose side is small enough (<= 0.999 b / sqrt(3), allowing for the
// float32 index error) that any two particles of one fine cell are friends: every
// non-empty fine cell is a clique ("unit"), the idea of cell-based FoF with cells of side
// b/sqrt(3) that the paper's linked-cell section cites as its inspiration.  Units then only
// need one friend pair to be joined, so tests stop at the first hit.
//
// Build stage (index construction):
//   k_classify   cells with more than `dense_threshold` particles get a dense id and a table
//   k_dense_sort sort each dense cell by fine key (in LDS when it fits, else through a
//                staging buffer) and write the key bitmask, its popcount prefix and the
//                start of every unit
// Link stage:
//   k_dense_cc   union-find over the units of one cell in LDS (first hit joins two units),
//                then every member's entry points at the component member with the
//                smallest original index; units record their component number
//   k_dense_cross units of neighbouring dense cells, each cell pair handled once (by the
//                lower cell index), stopping as soon as two single-component cells meet
// Particles of sparse cells reach dense neighbours through the unit tables (fof_link.hip).
#include "fof_internal.h"

namespace fof {

namespace {

constexpr int kDenseBlock = 256;
constexpr int kLdsCap = 2048;  // particles a dense cell may hold to be handled in LDS

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

struct CellXYZ {
    int x, y, z;
};

__device__ __forceinline__ CellXYZ cell_xyz(const BoxDesc &B, int64_t c)
{
    int64_t l = c - B.cell_base;
    CellXYZ r;
    r.x = (int)(l % B.nc[0]);
    l /= B.nc[0];
    r.y = (int)(l % B.nc[1]);
    r.z = (int)(l / B.nc[1]);
    return r;
}

// Fine key of a particle inside its coarse cell (cx, cy, cz).
__device__ __forceinline__ int fine_key(const BoxDesc &B, const CellXYZ &cc, float4 p)
{
    const int m = B.m;
    int fx = fine_index(p.x, B.inv_fine[0], B.nf[0]) - cc.x * m;
    int fy = fine_index(p.y, B.inv_fine[1], B.nf[1]) - cc.y * m;
    int fz = fine_index(p.z, B.inv_fine[2], B.nf[2]) - cc.z * m;
    return (fz * m + fy) * m + fx;
}

__device__ __forceinline__ int table_rank(const int32_t *T, int words, int k)
{
    uint32_t w = (uint32_t)T[kTableHeader + (k >> 5)];
    return T[kTableHeader + words + (k >> 5)] + __popc(w & ((1u << (k & 31)) - 1u));
}

__device__ __forceinline__ bool table_has(const int32_t *T, int k)
{
    return ((uint32_t)T[kTableHeader + (k >> 5)] >> (k & 31)) & 1u;
}

// LDS union-find over fine keys: hook the larger root under the smaller.
__device__ __forceinline__ int lfind(int *uf, int x)
{
    for (;;) {
        int p = __hip_atomic_load(uf + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (p == x)
            return x;
        x = p;
    }
}

__device__ __forceinline__ void lunion(int *uf, int a, int b)
{
    for (;;) {
        a = lfind(uf, a);
        b = lfind(uf, b);
        if (a == b)
            return;
        if (a < b) {
            int t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(uf + a, a, b) == a)
            return;
    }
}

// Block-wide exclusive scan of one int per thread (kDenseBlock threads).
__device__ int block_scan(int v, int *total, int *scratch /* kDenseBlock / kWave ints */)
{
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o, kWave);
        if (lane >= o)
            x += y;
    }
    if (lane == kWave - 1)
        scratch[wid] = x;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int k = 0; k < kDenseBlock / kWave; ++k) {
        int s = scratch[k];
        if (k < wid)
            pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__device__ __forceinline__ int dense_count(const Counters *ctr, int cap)
{
    int nd = __hip_atomic_load(&ctr->n_dense, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return nd < cap ? nd : cap;
}

// ---------------------------------------------------------------------------------------
__global__ void k_dense_reset(Counters *ctr)
{
    if (threadIdx.x == 0)
        ctr->n_dense = 0;
}

__global__ void k_classify(Work w)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = gtid(); c < w.ncell; c += stride) {
        const int32_t cnt = w.cell_start[c + 1] - w.cell_start[c];
        if (cnt <= w.dense_threshold)
            continue;
        const BoxDesc &B = w.desc[find_box_cell(w.desc, w.nbox, c)];
        int32_t tag = -1;
        if (B.dense_ok) {
            int32_t d = atomicAdd(&w.ctr->n_dense, 1);
            if (d < w.dense_cap) {
                w.dense_list[d] = (int32_t)c;
                tag = d;
            } else {
                atomicOr(&w.ctr->status, (int32_t)FOF_STATUS_DENSE_CAP);
            }
        }
        w.cell_count[c] = tag;  // the counters are dead after the scan: reused as tags
    }
}

// ---------------------------------------------------------------------------------------
// Sort one dense cell by fine key and write its tables.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kDenseBlock) void k_dense_sort(Work w)
{
    __shared__ int kcnt[kMaxFineKeys];
    __shared__ int koff[kMaxFineKeys + 1];
    __shared__ uint32_t kbits[kMaxTableWords];
    __shared__ int kpre[kMaxTableWords];
    __shared__ int scr[kDenseBlock / kWave];
    constexpr int kPer = kLdsCap / kDenseBlock;

    const int nd = dense_count(w.ctr, w.dense_cap);
    for (int d = blockIdx.x; d < nd; d += gridDim.x) {
        const int64_t c = w.dense_list[d];
        const int32_t s = w.cell_start[c];
        const int32_t n = w.cell_start[c + 1] - s;
        const BoxDesc &B = w.desc[find_box(w.desc, w.nbox, s)];
        const CellXYZ cc = cell_xyz(B, c);
        const int K = B.m * B.m * B.m;
        const int W = w.table_words;
        int32_t *T = w.table + (int64_t)d * w.table_stride;
        const bool lds = n <= kLdsCap;

        for (int k = threadIdx.x; k < K; k += kDenseBlock)
            kcnt[k] = 0;
        for (int k = threadIdx.x; k < kMaxTableWords; k += kDenseBlock)
            kbits[k] = 0u;
        __syncthreads();

        // keys and per-key ranks
        float4 preg[kPer];
        int kreg[kPer], rreg[kPer];
        if (lds) {
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int t = threadIdx.x + j * kDenseBlock;
                if (t < n) {
                    preg[j] = w.sorted[s + t];
                    kreg[j] = fine_key(B, cc, preg[j]);
                    rreg[j] = atomicAdd(kcnt + kreg[j], 1);
                }
            }
        } else {
            for (int t = threadIdx.x; t < n; t += kDenseBlock)
                atomicAdd(kcnt + fine_key(B, cc, w.sorted[s + t]), 1);
        }
        __syncthreads();

        // exclusive scan over keys (each thread owns 4 consecutive keys: K <= 1024)
        int loc[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = threadIdx.x * 4 + q;
            loc[q] = k < K ? kcnt[k] : 0;
            sum += loc[q];
        }
        int tot;
        int run = block_scan(sum, &tot, scr);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = threadIdx.x * 4 + q;
            if (k < K) {
                koff[k] = run;
                if (loc[q] > 0)
                    atomicOr(kbits + (k >> 5), 1u << (k & 31));
            }
            run += loc[q];
        }
        if (threadIdx.x == 0)
            koff[K] = n;
        __syncthreads();
        if (threadIdx.x < W) {
            int pre = 0;
            for (int q = 0; q < (int)threadIdx.x; ++q)
                pre += __popc(kbits[q]);
            kpre[threadIdx.x] = pre;
        }
        __syncthreads();

        // place the particles in key order
        if (lds) {
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
                const int t = threadIdx.x + j * kDenseBlock;
                if (t < n)
                    w.sorted[s + koff[kreg[j]] + rreg[j]] = preg[j];
            }
        } else {
            for (int k = threadIdx.x; k < K; k += kDenseBlock)
                kcnt[k] = 0;  // reused as per-key cursors
            __syncthreads();
            for (int t = threadIdx.x; t < n; t += kDenseBlock) {
                const float4 p = w.sorted[s + t];
                const int k = fine_key(B, cc, p);
                w.temp[s + koff[k] + atomicAdd(kcnt + k, 1)] = p;
            }
            __threadfence();
            __syncthreads();
            for (int t = threadIdx.x; t < n; t += kDenseBlock)
                w.sorted[s + t] = w.temp[s + t];
        }

        // tables: header, bitmask, popcount prefix, unit starts (absolute sorted index)
        if (threadIdx.x == 0) {
            T[0] = (int32_t)c;
            T[1] = 0;
            T[2] = kpre[W - 1] + __popc(kbits[W - 1]);
            T[3] = 0;
        }
        for (int q = threadIdx.x; q < W; q += kDenseBlock) {
            T[kTableHeader + q] = (int32_t)kbits[q];
            T[kTableHeader + W + q] = kpre[q];
        }
        for (int k = threadIdx.x; k < K; k += kDenseBlock) {
            if ((kbits[k >> 5] >> (k & 31)) & 1u) {
                const int r = kpre[k >> 5] + __popc(kbits[k >> 5] & ((1u << (k & 31)) - 1u));
                w.rank[s + r] = s + koff[k];
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// Union-find over the units of one dense cell, in LDS.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kDenseBlock) void k_dense_cc(Work w)
{
    __shared__ float4 pbuf[kLdsCap];
    __shared__ int kuf[kMaxFineKeys];
    __shared__ int ucomp[kMaxFineKeys];      // component number by root key
    __shared__ unsigned long long kmin[kMaxFineKeys];
    __shared__ short ulist[kMaxFineKeys];    // key of each unit, by unit rank
    __shared__ int ustart[kMaxFineKeys + 1]; // unit start relative to the cell, by rank
    __shared__ int sh_ncomp;

    const int nd = dense_count(w.ctr, w.dense_cap);
    for (int d = blockIdx.x; d < nd; d += gridDim.x) {
        const int64_t c = w.dense_list[d];
        const int32_t s = w.cell_start[c];
        const int32_t n = w.cell_start[c + 1] - s;
        const BoxDesc &B = w.desc[find_box(w.desc, w.nbox, s)];
        const int m = B.m, K = m * m * m, R = B.R;
        const int W = w.table_words;
        int32_t *T = w.table + (int64_t)d * w.table_stride;
        const int u = T[2];
        const bool lds = n <= kLdsCap;
        const float4 *mem = lds ? pbuf : (w.sorted + s);

        if (threadIdx.x == 0)
            sh_ncomp = 0;
        for (int k = threadIdx.x; k < K; k += kDenseBlock) {
            kuf[k] = k;
            kmin[k] = ~0ull;
        }
        if (lds)
            for (int t = threadIdx.x; t < n; t += kDenseBlock)
                pbuf[t] = w.sorted[s + t];
        for (int r = threadIdx.x; r < u; r += kDenseBlock)
            ustart[r] = w.rank[s + r] - s;
        if (threadIdx.x == 0)
            ustart[u] = n;
        for (int q = threadIdx.x; q < W; q += kDenseBlock) {
            uint32_t bits = (uint32_t)T[kTableHeader + q];
            int r = T[kTableHeader + W + q];
            while (bits) {
                int bpos = __ffs(bits) - 1;
                bits &= bits - 1u;
                ulist[r++] = (short)(q * 32 + bpos);
            }
        }
        __syncthreads();

        // member with the smallest original index in each unit
        for (int r = threadIdx.x; r < u; r += kDenseBlock) {
            unsigned long long best = ~0ull;
            for (int t = ustart[r]; t < ustart[r + 1]; ++t) {
                unsigned long long v =
                    ((unsigned long long)(uint32_t)__float_as_int(mem[t].w) << 32) | (uint32_t)t;
                best = v < best ? v : best;
            }
            kmin[ulist[r]] = best;
        }

        // join units of this cell: forward offsets within [-R, R]^3, first friend pair wins
        const int side = 2 * R + 1, half = (side * side * side - 1) / 2;
        const double fs = (double)B.fine_side;
        for (int task = threadIdx.x; task < u * half; task += kDenseBlock) {
            const int r = task / half;
            const int q = half + 1 + task % half;  // forward offsets follow the centre
            const int dx = q % side - R, dy = (q / side) % side - R, dz = q / (side * side) - R;
            const int ka = ulist[r];
            const int ax = ka % m + dx, ay = (ka / m) % m + dy, az = ka / (m * m) + dz;
            if (ax < 0 || ay < 0 || az < 0 || ax >= m || ay >= m || az >= m)
                continue;
            const double gx = fmax(0.0, (double)(abs(dx) - 1)) * fs;
            const double gy = fmax(0.0, (double)(abs(dy) - 1)) * fs;
            const double gz = fmax(0.0, (double)(abs(dz) - 1)) * fs;
            if (gx * gx + gy * gy + gz * gz >= B.b2)
                continue;
            const int kb = (az * m + ay) * m + ax;
            if (!table_has(T, kb))
                continue;
            if (lfind(kuf, ka) == lfind(kuf, kb))
                continue;
            const int rb = table_rank(T, W, kb);
            bool hit = false;
            for (int i = ustart[r]; i < ustart[r + 1] && !hit; ++i) {
                const float4 p = mem[i];
                for (int j = ustart[rb]; j < ustart[rb + 1]; ++j) {
                    const float4 q4 = mem[j];
                    if (linked(B, p.x, p.y, p.z, q4.x, q4.y, q4.z)) {
                        hit = true;
                        break;
                    }
                }
            }
            if (hit)
                lunion(kuf, ka, kb);
        }
        __syncthreads();

        // flatten, component minimum, component numbers
        int rootreg[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = threadIdx.x + j * kDenseBlock;
            rootreg[j] = r < u ? lfind(kuf, ulist[r]) : 0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = threadIdx.x + j * kDenseBlock;
            if (r < u)
                kuf[ulist[r]] = rootreg[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = threadIdx.x + j * kDenseBlock;
            if (r < u) {
                const int k = ulist[r];
                if (rootreg[j] != k)
                    atomicMin(kmin + rootreg[j], kmin[k]);
                else
                    ucomp[k] = atomicAdd(&sh_ncomp, 1);
            }
        }
        __syncthreads();

        // every member points at its component's smallest original index
        for (int r = threadIdx.x; r < u; r += kDenseBlock) {
            const int root = kuf[ulist[r]];
            const unsigned long long lead = kmin[root];
            const uint64_t packed = (lead & 0xffffffff00000000ull) | (uint32_t)(s + (uint32_t)lead);
            for (int t = ustart[r]; t < ustart[r + 1]; ++t)
                w.parent[s + t] = packed;
            w.cnt[s + r] = ucomp[root];
        }
        if (threadIdx.x == 0)
            T[1] = sh_ncomp;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// Units of neighbouring dense cells.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kDenseBlock) void k_dense_cross(Work w)
{
    __shared__ short ukey[kMaxFineKeys];
    __shared__ int ubeg[kMaxFineKeys + 1];
    __shared__ int ucmp[kMaxFineKeys];
    __shared__ uint32_t pairbits[32];
    __shared__ int done;

    const int nd = dense_count(w.ctr, w.dense_cap);
    for (int d = blockIdx.x; d < nd; d += gridDim.x) {
        const int64_t c = w.dense_list[d];
        const int32_t s = w.cell_start[c];
        const int32_t n = w.cell_start[c + 1] - s;
        const BoxDesc &B = w.desc[find_box(w.desc, w.nbox, s)];
        const CellXYZ cc = cell_xyz(B, c);
        const int m = B.m, R = B.R;
        const int W = w.table_words;
        const int32_t *T = w.table + (int64_t)d * w.table_stride;
        const int u = T[2], ncomp = T[1];

        for (int r = threadIdx.x; r < u; r += kDenseBlock) {
            ubeg[r] = w.rank[s + r];
            ucmp[r] = w.cnt[s + r];
        }
        if (threadIdx.x == 0)
            ubeg[u] = s + n;
        for (int q = threadIdx.x; q < W; q += kDenseBlock) {
            uint32_t bits = (uint32_t)T[kTableHeader + q];
            int r = T[kTableHeader + W + q];
            while (bits) {
                int bpos = __ffs(bits) - 1;
                bits &= bits - 1u;
                ukey[r++] = (short)(q * 32 + bpos);
            }
        }
        __syncthreads();

        for (int o = 0; o < 27; ++o) {
            if (o == 13)
                continue;
            const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
            int nx = cc.x + ox, ny = cc.y + oy, nz = cc.z + oz;
            nx += nx < 0 ? B.nc[0] : (nx >= B.nc[0] ? -B.nc[0] : 0);
            ny += ny < 0 ? B.nc[1] : (ny >= B.nc[1] ? -B.nc[1] : 0);
            nz += nz < 0 ? B.nc[2] : (nz >= B.nc[2] ? -B.nc[2] : 0);
            const int64_t c2 = coarse_cell(B, nx, ny, nz);
            if (c2 <= c)
                continue;  // each pair of cells once, by the lower index
            const int32_t s2 = w.cell_start[c2];
            const int32_t n2 = w.cell_start[c2 + 1] - s2;
            if (n2 <= w.dense_threshold)
                continue;
            const int32_t d2 = w.cell_count[c2];
            if (d2 < 0)
                continue;  // cell without tables: its particles search themselves
            const int32_t *T2 = w.table + (int64_t)d2 * w.table_stride;
            const int u2 = T2[2], ncomp2 = T2[1];
            const bool dedupe = ncomp * ncomp2 <= 1024;
            const bool single = ncomp == 1 && ncomp2 == 1;
            if (threadIdx.x < 32)
                pairbits[threadIdx.x] = 0u;
            if (threadIdx.x == 0)
                done = 0;
            __syncthreads();
            for (int r = threadIdx.x; r < u; r += kDenseBlock) {
                if (__hip_atomic_load(&done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                    break;
                const int ka = ukey[r];
                // unit A in the frame of the neighbour cell
                const int rx = ka % m - ox * m, ry = (ka / m) % m - oy * m, rz = ka / (m * m) - oz * m;
                const int x0 = max(0, rx - R), x1 = min(m - 1, rx + R);
                const int y0 = max(0, ry - R), y1 = min(m - 1, ry + R);
                const int z0 = max(0, rz - R), z1 = min(m - 1, rz + R);
                bool stop = false;
                for (int bz = z0; bz <= z1 && !stop; ++bz)
                    for (int by = y0; by <= y1 && !stop; ++by)
                        for (int bx = x0; bx <= x1 && !stop; ++bx) {
                            const double gx = fmax(0.0, (double)(abs(bx - rx) - 1)) * B.fine_side;
                            const double gy = fmax(0.0, (double)(abs(by - ry) - 1)) * B.fine_side;
                            const double gz = fmax(0.0, (double)(abs(bz - rz) - 1)) * B.fine_side;
                            if (gx * gx + gy * gy + gz * gz >= B.b2)
                                continue;
                            const int kb = (bz * m + by) * m + bx;
                            if (!table_has(T2, kb))
                                continue;
                            const int rb = table_rank(T2, W, kb);
                            const int cb = w.cnt[s2 + rb];
                            const int bit = ucmp[r] * ncomp2 + cb;
                            if (dedupe && ((pairbits[bit >> 5] >> (bit & 31)) & 1u))
                                continue;
                            const int32_t b0 = w.rank[s2 + rb];
                            const int32_t b1 = rb + 1 < u2 ? w.rank[s2 + rb + 1] : s2 + n2;
                            bool hit = false;
                            for (int32_t i = ubeg[r]; i < ubeg[r + 1] && !hit; ++i) {
                                const float4 p = w.sorted[i];
                                for (int32_t j = b0; j < b1; ++j) {
                                    const float4 q4 = w.sorted[j];
                                    if (linked(B, p.x, p.y, p.z, q4.x, q4.y, q4.z)) {
                                        uf_union(w.parent, (uint32_t)i, (uint32_t)j);
                                        hit = true;
                                        break;
                                    }
                                }
                            }
                            if (hit) {
                                if (dedupe)
                                    atomicOr(pairbits + (bit >> 5), 1u << (bit & 31));
                                if (single) {
                                    __hip_atomic_store(&done, 1, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                                    stop = true;
                                }
                            }
                        }
            }
            __syncthreads();
        }
    }
}

unsigned persistent_blocks(int cap)
{
    int b = cap < 4096 ? cap : 4096;
    return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

hipError_t launch_dense_build(const Work &w, hipStream_t s)
{
    if (w.dense_cap <= 0 || w.dense_threshold < 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_dense_reset, dim3(1), dim3(64), 0, s, w.ctr);
    int64_t nb = (w.ncell + 255) / 256;
    if (nb > 65536)
        nb = 65536;
    hipLaunchKernelGGL(k_classify, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s, w);
    hipLaunchKernelGGL(k_dense_sort, dim3(persistent_blocks(w.dense_cap)), dim3(kDenseBlock), 0, s,
                       w);
    return hipGetLastError();
}

hipError_t launch_dense(const Work &w, hipStream_t s)
{
    if (w.dense_cap <= 0 || w.dense_threshold < 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_dense_cc, dim3(persistent_blocks(w.dense_cap)), dim3(kDenseBlock), 0, s,
                       w);
    hipLaunchKernelGGL(k_dense_cross, dim3(persistent_blocks(w.dense_cap)), dim3(kDenseBlock), 0,
                       s, w);
    return hipGetLastError();
}

}  // namespace fof
