// Group catalogue (paper Sec. 2 step (vi), Alg. 2 compaction; Sec. 3.1 halo position).
//
// Works in cell-sorted order on the state fof_link leaves behind: particles without a
// friend are singleton components; every flagged particle's union-find entry points
// straight at its root, whose key is the component label (smallest original index).
//
//   g_compact  flist = sorted indices of the flagged particles, ascending (popcount scan
//              of the flag bitmap); built at the end of fof_link (launch_flag_list), which
//              also walks it; the passes marked (list) below walk only flist
//   g_zero     cnt[i] = 0 for flagged i (every non-singleton root is flagged)   (list)
//   g_count    cnt[root] += 1 for flagged i                                     (list)
//   g_keep     set keep bit [label] for kept components (size >= min_size); with
//              min_size > 1 only non-singleton roots qualify                  (list)
//   scan       popcount prefix over the keep bitmap -> group id = rank of the label
//   g_assign   group_id[orig]; with min_size > 1 group_id is filled with -1 first and only
//              flagged particles are visited (list); per kept group: size, root slot, and
//              the moment accumulators cleared (singleton groups are finished here)
//   g_sum      FP64 sums of minimum-image offsets from the root and of velocities (list);
//              with min_size > 1 and centres wanted it also does g_assign's work for the
//              flagged particles, after g_clear has cleared the kept groups' moments
//   g_mean     com = wrap(x_root + sum / n), vmean = vsum / n
//   g_dev      sum of squared velocity deviations (list); g_sig: sigv = sqrt(sum / (3 n))
#include "fof_internal.h"

namespace fof {

namespace {

// Runs of equal keys inside a wave (consecutive lanes): each lane learns the first lane of
// its run; the last lane of a run performs the run's single atomic.  Members of one group
// sit next to each other in cell-sorted order, so a large group costs one atomic per run
// instead of one per member.
struct Run {
    int head;   // first lane of this lane's run
    bool tail;  // last lane of its run
};

__device__ __forceinline__ Run wave_run(int64_t key)
{
    const int lane = lane_id();
    const int64_t prev = __shfl_up(key, 1, kWave);
    const int64_t next = __shfl_down(key, 1, kWave);
    const bool head = lane == 0 || prev != key;
    const uint64_t heads = ballot(head);
    const uint64_t below = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    Run r;
    r.head = 63 - __clzll((long long)below);
    r.tail = lane == kWave - 1 || next != key;
    return r;
}

// Inclusive sum over the lane's run (segmented scan); exact: no cancellation.
template <typename T>
__device__ __forceinline__ T run_sum(T v, int head)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const T u = __shfl_up(v, o, kWave);
        if (lane - o >= head)
            v += u;
    }
    return v;
}

__device__ __forceinline__ bool flagged(const uint64_t *flags, int64_t i)
{
    return (flags[i >> 6] >> (i & 63)) & 1ull;
}

__device__ __forceinline__ int32_t group_of(const uint32_t *keep, const int32_t *keep_prefix,
                                            uint32_t label)
{
    uint32_t w = keep[label >> 5];
    uint32_t bit = 1u << (label & 31);
    if (!(w & bit))
        return -1;
    return keep_prefix[label >> 5] + __popc(w & (bit - 1u));
}

// Flagged-list compaction: one wave per 64-bit flag word, lane l owning particle 64 q + l;
// `prefix` is the exclusive popcount scan of the flag bitmap read as 32-bit words, so the
// word's first slot is prefix[2 q].  The list comes out in ascending order.
__global__ void g_compact(const uint64_t *__restrict__ flags, int64_t n,
                          const int32_t *__restrict__ prefix, int64_t nwords32,
                          int32_t *__restrict__ list, Counters *__restrict__ ctr)
{
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    const int64_t nq = (n + 63) / 64;
    for (int64_t q = wave; q < nq; q += nwaves) {
        const uint64_t word = flags[q];
        if ((word >> lane) & 1ull)
            list[prefix[2 * q] + __popcll(word & ((1ull << lane) - 1ull))] =
                (int32_t)(64 * q + lane);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        ctr->n_flagged = prefix[nwords32];
}

// The list-driven passes below walk flist in grid-sized rounds: lanes of a wave take
// consecutive entries, so members of one group (adjacent in cell-sorted order) stay in
// consecutive lanes for the run reductions.

__global__ void g_zero(const int32_t *__restrict__ list, const Counters *__restrict__ ctr,
                       int32_t *__restrict__ cnt)
{
    const int64_t nf = ctr->n_flagged;
    for (int64_t k = gtid(); k < nf; k += (int64_t)gridDim.x * blockDim.x)
        cnt[list[k]] = 0;
}

__global__ void g_count(const int32_t *__restrict__ list, const Counters *__restrict__ ctr,
                        const uint64_t *__restrict__ parent, int32_t *__restrict__ cnt)
{
    const int64_t nf = ctr->n_flagged;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nf; base += stride) {
        const int64_t k = base + threadIdx.x;
        const bool in = k < nf;
        const int64_t key = in ? (int64_t)uf_idx(parent[list[k]]) : -1 - (int64_t)lane_id();
        const Run r = wave_run(key);
        const int c = run_sum(in ? 1 : 0, r.head);
        if (in && r.tail)
            atomicAdd(cnt + key, c);
    }
}

// min_size > 1: only roots of non-singleton components can be kept; a root's key is its
// own label.
__global__ void g_keep_roots(const int32_t *__restrict__ list, const Counters *__restrict__ ctr,
                             const uint64_t *__restrict__ parent, const int32_t *__restrict__ cnt,
                             int32_t min_size, uint32_t *__restrict__ keep)
{
    const int64_t nf = ctr->n_flagged;
    for (int64_t k = gtid(); k < nf; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = list[k];
        const uint64_t e = parent[i];
        if (uf_idx(e) == (uint32_t)i && cnt[i] >= min_size) {
            const uint32_t label = uf_key(e);
            atomicOr(keep + (label >> 5), 1u << (label & 31));
        }
    }
}

__global__ void g_keep(const float4 *__restrict__ sorted, int64_t n,
                       const uint64_t *__restrict__ parent, const uint64_t *__restrict__ flags,
                       const int32_t *__restrict__ cnt, int32_t min_size,
                       uint32_t *__restrict__ keep)
{
    int64_t i = gtid();
    if (i >= n)
        return;
    const bool fl = flagged(flags, i);
    if (!fl && min_size > 1)
        return;  // a particle without a friend is a group of one
    int32_t size;
    if (fl) {
        if (uf_idx(parent[i]) != (uint32_t)i)
            return;  // not a root
        size = cnt[i];
    } else {
        size = 1;
    }
    if (size >= min_size) {
        uint32_t label = (uint32_t)__float_as_int(sorted[i].w);
        atomicOr(keep + (label >> 5), 1u << (label & 31));
    }
}

struct GroupOut {
    int32_t *group_id, *groot, *sizes;
    double *com, *vmean, *sigv;
    const float *vel;
    int32_t cap;
};

// group_id of one particle; the root of a kept group also writes the group's size and root
// slot and clears its moment accumulators (a singleton group is finished here).
__device__ __forceinline__ void assign_one(const float4 *__restrict__ sorted,
                                           const uint64_t *__restrict__ parent, bool fl,
                                           uint32_t i, const int32_t *__restrict__ cnt,
                                           const uint32_t *__restrict__ keep,
                                           const int32_t *__restrict__ keep_prefix,
                                           const GroupOut &o)
{
    const float4 p = sorted[i];
    const int32_t orig = __float_as_int(p.w);
    const uint64_t e = fl ? parent[i] : 0;
    const uint32_t rs = fl ? uf_idx(e) : i;
    const uint32_t label = fl ? uf_key(e) : (uint32_t)orig;
    const int32_t g = group_of(keep, keep_prefix, label);
    o.group_id[orig] = g;
    if (g < 0 || g >= o.cap || rs != i)
        return;
    o.groot[g] = (int32_t)i;
    const double c[3] = {(double)p.x, (double)p.y, (double)p.z};
    if (fl) {
        o.sizes[g] = cnt[i];
        if (o.com)
            for (int a = 0; a < 3; ++a)
                o.com[3 * g + a] = 0.0;
        if (o.vel) {
            if (o.vmean)
                for (int a = 0; a < 3; ++a)
                    o.vmean[3 * g + a] = 0.0;
            if (o.sigv)
                o.sigv[g] = 0.0;
        }
    } else {
        o.sizes[g] = 1;
        if (o.com)
            for (int a = 0; a < 3; ++a)
                o.com[3 * g + a] = c[a];
        if (o.vel) {
            if (o.vmean)
                for (int a = 0; a < 3; ++a)
                    o.vmean[3 * g + a] = (double)o.vel[3 * (int64_t)orig + a];
            if (o.sigv)
                o.sigv[g] = 0.0;
        }
    }
}

// Every particle (min_size <= 1: groups of one are kept).
__global__ void g_assign(const float4 *__restrict__ sorted, int64_t n,
                         const uint64_t *__restrict__ parent, const uint64_t *__restrict__ flags,
                         const int32_t *__restrict__ cnt, const uint32_t *__restrict__ keep,
                         const int32_t *__restrict__ keep_prefix, GroupOut o)
{
    const int64_t i = gtid();
    if (i < n)
        assign_one(sorted, parent, flagged(flags, i), (uint32_t)i, cnt, keep, keep_prefix, o);
}

// Particles with a friend only (min_size > 1: group_id was filled with -1 beforehand).
__global__ void g_assign_list(const float4 *__restrict__ sorted, const int32_t *__restrict__ list,
                              const Counters *__restrict__ ctr,
                              const uint64_t *__restrict__ parent, const int32_t *__restrict__ cnt,
                              const uint32_t *__restrict__ keep,
                              const int32_t *__restrict__ keep_prefix, GroupOut o)
{
    const int64_t nf = ctr->n_flagged;
    for (int64_t k = gtid(); k < nf; k += (int64_t)gridDim.x * blockDim.x)
        assign_one(sorted, parent, true, (uint32_t)list[k], cnt, keep, keep_prefix, o);
}

// Members of non-singleton groups only: singleton groups were finished by the assign pass.
// With `a.group_id` set (min_size > 1: group_id filled with -1 and the moments cleared
// beforehand), the same pass also writes each member's group id and each kept root's size
// and root slot, which saves the separate assign pass over the list.
struct Assign {
    int32_t *group_id, *groot, *sizes;
    const int32_t *cnt;
};

__global__ void g_sum(const float4 *__restrict__ sorted, const int32_t *__restrict__ list,
                      const Counters *__restrict__ ctr, const BoxDesc *__restrict__ desc,
                      int nbox, const uint64_t *__restrict__ parent,
                      const uint32_t *__restrict__ keep, const int32_t *__restrict__ keep_prefix,
                      const float *__restrict__ vel, int32_t cap, double *__restrict__ com,
                      double *__restrict__ vmean, Assign a)
{
    const int64_t nf = ctr->n_flagged;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nf; base += stride) {
        const int64_t k = base + threadIdx.x;
        int32_t g = -1, i = 0;
        uint64_t r = 0;
        float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (k < nf) {
            i = list[k];
            r = parent[i];
            g = group_of(keep, keep_prefix, uf_key(r));
            if (a.group_id && g >= 0) {
                p = sorted[i];
                a.group_id[__float_as_int(p.w)] = g;
                if (g < cap && uf_idx(r) == (uint32_t)i) {
                    a.groot[g] = i;
                    a.sizes[g] = a.cnt[i];
                }
            }
            if (g >= cap)
                g = -1;
        }
        const bool in = g >= 0;
        const Run run = wave_run(in ? (int64_t)g : -1 - (int64_t)lane_id());
        double d[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
        if (in) {
            if (!a.group_id)
                p = sorted[i];
            if (com) {
                const BoxDesc &B = desc[find_box(desc, nbox, i)];
                const float4 q = sorted[uf_idx(r)];
                d[0] = min_image((double)p.x - (double)q.x, B.L[0], B.halfL[0]);
                d[1] = min_image((double)p.y - (double)q.y, B.L[1], B.halfL[1]);
                d[2] = min_image((double)p.z - (double)q.z, B.L[2], B.halfL[2]);
            }
            if (vel && vmean) {
                const int64_t o = __float_as_int(p.w);
                v[0] = (double)vel[3 * o + 0];
                v[1] = (double)vel[3 * o + 1];
                v[2] = (double)vel[3 * o + 2];
            }
        }
        if (com) {
            for (int a = 0; a < 3; ++a) {
                const double sa = run_sum(d[a], run.head);
                if (in && run.tail)
                    atomicAdd(com + 3 * g + a, sa);
            }
        }
        if (vel && vmean) {
            for (int a = 0; a < 3; ++a) {
                const double sa = run_sum(v[a], run.head);
                if (in && run.tail)
                    atomicAdd(vmean + 3 * g + a, sa);
            }
        }
    }
}

// The moment accumulators of the kept groups, cleared before the fused sum pass.
__global__ void g_clear(const int32_t *__restrict__ n_groups, int32_t cap,
                        double *__restrict__ com, double *__restrict__ vmean,
                        double *__restrict__ sigv)
{
    const int64_t G = *n_groups < cap ? *n_groups : cap;
    for (int64_t g = gtid(); g < G; g += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < 3; ++c) {
            if (com)
                com[3 * g + c] = 0.0;
            if (vmean)
                vmean[3 * g + c] = 0.0;
        }
        if (sigv)
            sigv[g] = 0.0;
    }
}

__global__ void g_mean(const float4 *__restrict__ sorted, const BoxDesc *__restrict__ desc,
                       int nbox, const int32_t *__restrict__ n_groups, int32_t cap,
                       const int32_t *__restrict__ groot, const int32_t *__restrict__ sizes,
                       const float *__restrict__ vel, double *__restrict__ com,
                       double *__restrict__ vmean)
{
    int64_t g = gtid();
    int32_t G = *n_groups < cap ? *n_groups : cap;
    if (g >= G)
        return;
    const int32_t r = groot[g];
    const int32_t nn = sizes[g];
    if (nn <= 1)
        return;  // singleton groups were written by g_assign
    const double dn = (double)nn;
    if (com) {
        const BoxDesc &B = desc[find_box(desc, nbox, r)];
        const float4 q = sorted[r];
        const float qc[3] = {q.x, q.y, q.z};
        for (int a = 0; a < 3; ++a) {
            double v = (double)qc[a] + com[3 * g + a] / dn;
            if (v >= B.L[a])
                v -= B.L[a];
            if (v < 0.0)
                v += B.L[a];
            com[3 * g + a] = v;
        }
    }
    if (vel && vmean)
        for (int a = 0; a < 3; ++a)
            vmean[3 * g + a] = vmean[3 * g + a] / dn;
}

__global__ void g_dev(const float4 *__restrict__ sorted, const int32_t *__restrict__ list,
                      const Counters *__restrict__ ctr, const uint64_t *__restrict__ parent,
                      const uint32_t *__restrict__ keep, const int32_t *__restrict__ keep_prefix,
                      const float *__restrict__ vel, int32_t cap,
                      const double *__restrict__ vmean, double *__restrict__ sigv)
{
    const int64_t nf = ctr->n_flagged;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nf; base += stride) {
        const int64_t k = base + threadIdx.x;
        int32_t g = -1, i = 0;
        if (k < nf) {
            i = list[k];
            g = group_of(keep, keep_prefix, uf_key(parent[i]));
            if (g >= cap)
                g = -1;
        }
        const bool in = g >= 0;
        const Run run = wave_run(in ? (int64_t)g : -1 - (int64_t)lane_id());
        double s2 = 0.0;
        if (in) {
            const int64_t o = __float_as_int(sorted[i].w);
            for (int a = 0; a < 3; ++a) {
                const double dv = (double)vel[3 * o + a] - vmean[3 * g + a];
                s2 += dv * dv;
            }
        }
        s2 = run_sum(s2, run.head);
        if (in && run.tail)
            atomicAdd(sigv + g, s2);
    }
}

// Position dispersion (the decoration of Sec. 3.1's decorated frozen assignment): sum over
// the members of group g of |mi(x_i - com_g)|^2, mi the per-axis minimum image, FP64.
__global__ void g_sigx(const float4 *__restrict__ sorted, const int32_t *__restrict__ list,
                       const Counters *__restrict__ ctr, const BoxDesc *__restrict__ desc,
                       int nbox, const uint64_t *__restrict__ parent,
                       const uint32_t *__restrict__ keep, const int32_t *__restrict__ keep_prefix,
                       int32_t cap, const double *__restrict__ com, double *__restrict__ sigx)
{
    const int64_t nf = ctr->n_flagged;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nf; base += stride) {
        const int64_t k = base + threadIdx.x;
        int32_t g = -1, i = 0;
        if (k < nf) {
            i = list[k];
            g = group_of(keep, keep_prefix, uf_key(parent[i]));
            if (g >= cap)
                g = -1;
        }
        const bool in = g >= 0;
        const Run run = wave_run(in ? (int64_t)g : -1 - (int64_t)lane_id());
        double s2 = 0.0;
        if (in) {
            const float4 p = sorted[i];
            const BoxDesc &B = desc[find_box(desc, nbox, i)];
            const double c[3] = {(double)p.x, (double)p.y, (double)p.z};
            for (int a = 0; a < 3; ++a) {
                const double d = min_image(c[a] - com[3 * g + a], B.L[a], B.halfL[a]);
                s2 += d * d;
            }
        }
        s2 = run_sum(s2, run.head);
        if (in && run.tail)
            atomicAdd(sigx + g, s2);
    }
}

__global__ void g_sig(const int32_t *__restrict__ n_groups, int32_t cap,
                      const int32_t *__restrict__ sizes, double *__restrict__ sigv)
{
    int64_t g = gtid();
    int32_t G = *n_groups < cap ? *n_groups : cap;
    if (g >= G)
        return;
    const int32_t nn = sizes[g];
    if (nn > 1)
        sigv[g] = sqrt(sigv[g] / (3.0 * (double)nn));
}

__global__ void g_total(const int32_t *__restrict__ keep_prefix, int64_t nwords,
                        int32_t *__restrict__ n_groups, int32_t cap, Counters *__restrict__ ctr)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int32_t G = keep_prefix[nwords];
        *n_groups = G;
        if (G > cap)
            atomicOr(&ctr->status, (int32_t)FOF_STATUS_OVERFLOW);
    }
}

}  // namespace

// sigx[g] = sqrt(sum_i |mi(x_i - com_g)|^2 / (3 n_g)) for g < min(n_groups, cap); groups of
// one get 0.  Uses the flagged list and the keep tables of the last fof_groups call.
hipError_t launch_group_dispersion(const Work &w, int32_t cap, const int32_t *n_groups,
                                   const int32_t *sizes, const double *com, double *sigx,
                                   hipStream_t s)
{
    if (cap <= 0)
        return hipSuccess;
    hipError_t e = launch_fill_f64(sigx, cap, 0.0, s);
    if (e != hipSuccess)
        return e;
    if (w.n > 0) {
        const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
        const unsigned lb = nb < 4096u ? nb : 4096u;
        hipLaunchKernelGGL(g_sigx, dim3(lb), dim3(w.block), 0, s, w.sorted, w.flist, w.ctr,
                           w.desc, w.nbox, w.parent, w.keep, w.keep_prefix, cap, com, sigx);
    }
    const unsigned gb = (unsigned)((cap + 255) / 256);
    hipLaunchKernelGGL(g_sig, dim3(gb), dim3(256), 0, s, n_groups, cap, sizes, sigx);
    return hipGetLastError();
}

hipError_t launch_flag_list(const Work &w, hipStream_t s)
{
    if (w.n <= 0)
        return hipSuccess;
    const int64_t nwords = (w.n + 31) / 32;
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    const unsigned lb = nb < 4096u ? nb : 4096u;
    hipError_t e = launch_scan_popc((const uint32_t *)w.flags, w.keep_prefix, nwords, w.scan, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(g_compact, dim3(lb), dim3(w.block), 0, s, w.flags, w.n, w.keep_prefix,
                       nwords, w.flist, w.ctr);
    return hipGetLastError();
}

hipError_t launch_groups(const Work &w, int32_t min_size, const float *vel, int32_t cap,
                         int32_t *group_id, int32_t *n_groups, int32_t *sizes, double *com,
                         double *vmean, double *sigv, hipStream_t s)
{
    const int64_t nwords = (w.n + 31) / 32;
    const unsigned nb = (unsigned)((w.n + w.block - 1) / w.block);
    // grid of the list-driven passes: a few rounds of a full chip
    const unsigned lb = nb < 4096u ? (nb > 0 ? nb : 1u) : 4096u;
    // flist and n_flagged were left by fof_link (launch_flag_list)
    hipError_t e = launch_fill_u32(w.keep, nwords, 0u, s);
    if (e != hipSuccess)
        return e;
    const bool lonely_cut = min_size > 1;
    if (w.n > 0) {
        hipLaunchKernelGGL(g_zero, dim3(lb), dim3(w.block), 0, s, w.flist, w.ctr, w.cnt);
        hipLaunchKernelGGL(g_count, dim3(lb), dim3(w.block), 0, s, w.flist, w.ctr, w.parent,
                           w.cnt);
        if (lonely_cut)
            hipLaunchKernelGGL(g_keep_roots, dim3(lb), dim3(w.block), 0, s, w.flist, w.ctr,
                               w.parent, w.cnt, min_size, w.keep);
        else
            hipLaunchKernelGGL(g_keep, dim3(nb), dim3(w.block), 0, s, w.sorted, w.n, w.parent,
                               w.flags, w.cnt, min_size, w.keep);
    }
    e = launch_scan_popc(w.keep, w.keep_prefix, nwords, w.scan, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(g_total, dim3(1), dim3(64), 0, s, w.keep_prefix, nwords, n_groups, cap,
                       w.ctr);
    if (w.n == 0)
        return hipGetLastError();
    GroupOut o;
    o.group_id = group_id;
    o.groot = w.groot;
    o.sizes = sizes;
    o.com = com;
    o.vmean = vmean;
    o.sigv = sigv;
    o.vel = vel;
    o.cap = cap;
    // min_size > 1 with moments wanted: the assignment rides along the sum pass
    const bool fused = lonely_cut && cap > 0 && com;
    Assign as{nullptr, nullptr, nullptr, nullptr};
    if (fused) {
        e = launch_fill_i32(group_id, w.n, -1, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(g_clear, dim3(256), dim3(256), 0, s, n_groups, cap, com,
                           (vel && vmean) ? vmean : nullptr, (vel && sigv) ? sigv : nullptr);
        as = Assign{group_id, w.groot, sizes, w.cnt};
    } else if (lonely_cut) {
        e = launch_fill_i32(group_id, w.n, -1, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(g_assign_list, dim3(lb), dim3(w.block), 0, s, w.sorted, w.flist,
                           w.ctr, w.parent, w.cnt, w.keep, w.keep_prefix, o);
    } else {
        hipLaunchKernelGGL(g_assign, dim3(nb), dim3(w.block), 0, s, w.sorted, w.n, w.parent,
                           w.flags, w.cnt, w.keep, w.keep_prefix, o);
    }
    if (cap <= 0)
        return hipGetLastError();
    const unsigned gb = (unsigned)((cap + 255) / 256);
    const float *v = (vmean || sigv) ? vel : nullptr;
    hipLaunchKernelGGL(g_sum, dim3(lb), dim3(w.block), 0, s, w.sorted, w.flist, w.ctr, w.desc,
                       w.nbox, w.parent, w.keep, w.keep_prefix, v, cap, com, vmean, as);
    hipLaunchKernelGGL(g_mean, dim3(gb), dim3(256), 0, s, w.sorted, w.desc, w.nbox, n_groups, cap,
                       w.groot, sizes, v, com, vmean);
    if (v && vmean && sigv) {
        hipLaunchKernelGGL(g_dev, dim3(lb), dim3(w.block), 0, s, w.sorted, w.flist, w.ctr,
                           w.parent, w.keep, w.keep_prefix, v, cap, vmean, sigv);
        hipLaunchKernelGGL(g_sig, dim3(gb), dim3(256), 0, s, n_groups, cap, sizes, sigv);
    }
    return hipGetLastError();
}

}  // namespace fof
