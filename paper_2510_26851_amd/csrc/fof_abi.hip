// Host entry points of libfof.so (declared in include/fof.h): planning, argument
// validation and kernel launches.  Nothing here allocates, frees, synchronises or prints.
#include <math.h>
#include <string.h>

#include <mutex>

#include "fof_internal.h"

namespace fof {
namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kDefaultDense = 32;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Bound on how far a float32 cell index can move a coordinate: the computed fine cell of
// x is the exact cell of some x' with |x' - x| <= L 2^-23 (1 + 2^-10) (one rounding of the
// scale factor to float32 and one of the product).  `reach` adds the rounding of the
// float32 face distance (< 1.5 L 2^-23) on top, with room to spare.
double index_eps(double Lmax) { return ldexp(Lmax, -23) * (1.0 + ldexp(1.0, -10)); }
double reach_of(double b, double Lmax) { return b + 4.0 * ldexp(Lmax, -23); }

float round_up_f(double v)
{
    float f = (float)v;
    if ((double)f < v)
        f = nextafterf(f, INFINITY);
    return f;
}

bool box_ok(const fof_box &bx)
{
    if (!(bx.b > 0.0) || !isfinite(bx.b))
        return false;
    for (int a = 0; a < 3; ++a)
        if (!(bx.L[a] > 0.0) || !isfinite(bx.L[a]) || !(2.0 * bx.b < bx.L[a]))
            return false;
    return true;
}

// Per-box plan: coarse cells per axis and fine cells per coarse cell.
int plan_box(const fof_box &bx, int64_t n, const fof_tune *tune, int64_t cell_base, int64_t off,
             BoxDesc *d)
{
    const double Lmax = fmax(bx.L[0], fmax(bx.L[1], bx.L[2]));
    const double V = bx.L[0] * bx.L[1] * bx.L[2];
    const double reach = reach_of(bx.b, Lmax);
    const double eps = index_eps(Lmax);
    // Largest clique cell side: any two points of one fine cell (each placed within eps of
    // its exact cell) are closer than 0.999 b.
    const double a_max = 0.999 * bx.b / sqrt(3.0) - 2.0 * eps;
    if (!(a_max > 0.0))
        return FOF_EINVAL;
    const double factor = (tune && tune->cell_factor > 0.0) ? tune->cell_factor : 1.0;
    double s = (tune && tune->cell_side > 0.0) ? tune->cell_side
                                               : (n > 0 ? factor * cbrt(V / (double)n) : Lmax);
    // never more than about 8 coarse cells per particle
    s = fmax(s, cbrt(V / (8.0 * (double)n + 64.0)));
    double side_max = 0.0;
    for (int a = 0; a < 3; ++a) {
        // cells per axis: from the requested side, then at least enough that a cell holds
        // at most kMaxFine clique cells, and at most as many as keep the side >= reach
        double q = floor(bx.L[a] / s);
        double q_min = ceil(bx.L[a] / ((double)kMaxFine * a_max));
        double q_max = floor(bx.L[a] / reach);
        q = fmax(q, q_min);
        q = fmin(q, q_max);
        int64_t nc = q < 1.0 ? 1 : (int64_t)q;
        if (nc > (1 << 20) || (nc > 1 && bx.L[a] / (double)nc < reach))
            return FOF_EINVAL;
        d->nc[a] = (int32_t)nc;
        side_max = fmax(side_max, bx.L[a] / (double)nc);
    }
    int m = (int)ceil(side_max / a_max);
    if (m < 1)
        m = 1;
    if (m > kMaxFine)
        return FOF_EINVAL;
    d->m = m;
    d->mdiv = m > 1 ? (uint32_t)(((1ull << 32) + (uint64_t)m - 1) / (uint64_t)m) : 0u;
    d->off = off;
    d->n = (int32_t)n;
    d->cell_base = cell_base;
    for (int a = 0; a < 3; ++a) {
        d->nf[a] = d->nc[a] * m;
        d->L[a] = bx.L[a];
        d->halfL[a] = 0.5 * bx.L[a];
        d->Lup[a] = round_up_f(bx.L[a]);
        d->inv_fine[a] = (float)((double)d->nf[a] / bx.L[a]);
        d->side[a] = (float)(bx.L[a] / (double)d->nc[a]);
    }
    d->b2 = bx.b * bx.b;
    d->reach = round_up_f(reach);
    // Fine cells: a friend lies at most R fine cells away per axis (its exact cell is within
    // b + 2 eps); the fine side stored for gap pruning is a lower bound, less 2 eps.
    double a_min = fmin(bx.L[0] / d->nf[0], fmin(bx.L[1] / d->nf[1], bx.L[2] / d->nf[2]));
    d->R = (int32_t)floor((bx.b + 2.0 * eps) / a_min) + 1;
    float fs = (float)(a_min - 2.0 * eps);
    if ((double)fs > a_min - 2.0 * eps)
        fs = nextafterf(fs, 0.0f);
    d->fine_side = fs > 0.0f ? fs : 0.0f;
    for (int a = 0; a < 3; ++a)
        d->fine[a] = (float)(bx.L[a] / (double)d->nf[a]);
    // a member lies within eps of its exact fine cell; float box bounds and differences add
    // a few ulps of L: 8 L 2^-23 covers both with room to spare
    d->slack = round_up_f(8.0 * ldexp(Lmax, -23));
    d->dense_ok = (d->nc[0] >= 3 && d->nc[1] >= 3 && d->nc[2] >= 3 && d->R <= 3) ? 1 : 0;
    // the tiled link kernel needs every halo cell of a tile to be a distinct cell
    d->tiled = (d->nc[0] >= kTileX + 2 && d->nc[1] >= kTileY + 2 && d->nc[2] >= kTileZ + 2 &&
                !(tune && (tune->flags & FOF_TUNE_NO_TILES)))
                   ? 1
                   : 0;
    d->ntile[0] = (d->nc[0] + kTileX - 1) / kTileX;
    d->ntile[1] = (d->nc[1] + kTileY - 1) / kTileY;
    d->ntile[2] = (d->nc[2] + kTileZ - 1) / kTileZ;
    return FOF_OK;
}

struct Layout {
    size_t off_desc, off_status, off_cell_count, off_cell_start, off_scan, off_rank, off_sorted,
        off_parent, off_flags, off_keep, off_keep_prefix, off_cnt, off_groot, off_flist, off_dense,
        off_big, off_table, off_temp, off_tiles, off_edges, off_cursors, off_classify, off_bin, total;
    int64_t edge_cap;
};

int32_t table_stride(int32_t words) { return kTableHeader + 2 * words; }

// Deferred hooks of the tiled link kernel (pairs crossing a tile face, links into dense
// cells): a fraction of a hook per particle in clustered boxes.  Tiles that overflow it are
// redone with direct hooks, so the capacity only affects speed.
int64_t link_edge_cap(int64_t n)
{
    int64_t c = n / 4 + 65536;
    return c < INT32_MAX ? c : INT32_MAX;
}

Layout layout(int32_t nbox, int64_t n, int64_t ncell, int64_t dense_cap, int32_t words,
              int64_t ntiles, int64_t link_edges)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    const int64_t nwords = (n + 31) / 32;
    int64_t scan_n = ncell > nwords ? ncell : nwords;
    const BinShape bs = bin_shape(n, ncell);
    const int64_t bin_n = bs.ok ? bs.nbk * bs.G : 0;  // bucketed binning table
    if (bin_n > scan_n)
        scan_n = bin_n;
    L.off_desc = take(sizeof(BoxDesc) * (size_t)nbox);
    L.off_status = take(sizeof(Counters));
    L.off_cell_count = take(sizeof(int32_t) * (size_t)ncell);
    L.off_cell_start = take(sizeof(int32_t) * (size_t)(ncell + 1));
    L.off_scan = take(sizeof(int32_t) * (size_t)scan_scratch_elems(scan_n));
    L.off_rank = take(sizeof(int32_t) * (size_t)n);
    L.off_sorted = take(sizeof(float4) * (size_t)n);
    L.off_parent = take(sizeof(uint64_t) * (size_t)n);
    L.off_flags = take(sizeof(uint64_t) * (size_t)((n + 63) / 64));
    L.off_keep = take(sizeof(uint32_t) * (size_t)nwords);
    L.off_keep_prefix = take(sizeof(int32_t) * (size_t)(nwords + 1));
    L.off_cnt = take(sizeof(int32_t) * (size_t)n);
    L.off_groot = take(sizeof(int32_t) * (size_t)n);
    L.off_flist = take(sizeof(int32_t) * (size_t)n);
    L.off_dense = take(sizeof(int32_t) * (size_t)dense_cap);
    L.off_big = take(sizeof(int32_t) * (size_t)dense_cap);
    L.off_table = take(sizeof(int32_t) * (size_t)dense_cap * (size_t)table_stride(words));
    // staging: the bucketed binning, then dense cells too large to sort in LDS
    L.off_temp = take(dense_cap > 0 || bin_n > 0 ? sizeof(float4) * (size_t)n : 0);
    L.off_tiles = take(sizeof(int32_t) * (size_t)ntiles);
    L.edge_cap = ntiles > 0 ? link_edges : 0;
    L.off_edges = take(sizeof(int2) * (size_t)L.edge_cap);
    L.off_cursors = take(dense_cap > 0 ? sizeof(int32_t) * (size_t)kCursorInts : 0);
    // dense-cell classification: counts and scans per chunk of 4096 cells (fof_dense.hip)
    L.off_classify = take(dense_cap > 0 ? sizeof(int32_t) * 4 * (size_t)(ncell / 4096 + 2) : 0);
    // counts per (bucket, block), then their exclusive scan (+ total) in place of a copy
    L.off_bin = take(bin_n > 0 ? sizeof(int32_t) * (size_t)(2 * bin_n + 1) : 0);
    L.total = o;
    return L;
}

// FOF_OK, FOF_EINVAL (no plan, no or misaligned workspace, a plan no fof_workspace_bytes
// could have made) or FOF_ENOMEM (a workspace smaller than the plan needs).
int ws_check(const fof_grid *g, const void *ws, size_t ws_bytes)
{
    if (!(g && ws && ((uintptr_t)ws % kAlign) == 0 && g->nbox >= 1 && g->n >= 0 &&
          g->link_edges >= 0 && g->link_edges <= INT32_MAX && g->block >= kWave &&
          g->block % kWave == 0 && g->block <= 1024))
        return FOF_EINVAL;
    return ws_bytes < g->ws_bytes ? FOF_ENOMEM : FOF_OK;
}

Work resolve(const fof_grid *g, void *ws)
{
    char *base = (char *)ws;
    Layout L = layout(g->nbox, g->n, g->ncell, g->dense_cap, g->table_words, g->ntiles,
                      g->link_edges);
    Work w;
    w.desc = (const BoxDesc *)(base + L.off_desc);
    w.ctr = (Counters *)(base + L.off_status);
    w.cell_count = (int32_t *)(base + L.off_cell_count);
    w.cell_start = (int32_t *)(base + L.off_cell_start);
    w.scan = (int32_t *)(base + L.off_scan);
    w.rank = (int32_t *)(base + L.off_rank);
    w.sorted = (float4 *)(base + L.off_sorted);
    w.parent = (uint64_t *)(base + L.off_parent);
    w.flags = (uint64_t *)(base + L.off_flags);
    w.keep = (uint32_t *)(base + L.off_keep);
    w.keep_prefix = (int32_t *)(base + L.off_keep_prefix);
    w.cnt = (int32_t *)(base + L.off_cnt);
    w.groot = (int32_t *)(base + L.off_groot);
    w.flist = (int32_t *)(base + L.off_flist);
    w.dense_list = (int32_t *)(base + L.off_dense);
    w.big_list = (int32_t *)(base + L.off_big);
    w.table = (int32_t *)(base + L.off_table);
    w.temp = (float4 *)(base + L.off_temp);
    w.tile_list = (int32_t *)(base + L.off_tiles);
    w.edges = (int2 *)(base + L.off_edges);
    w.cursors = (int32_t *)(base + L.off_cursors);
    w.classify = (int32_t *)(base + L.off_classify);
    w.bin_hist = (int32_t *)(base + L.off_bin);
    w.edge_cap = (int32_t)L.edge_cap;
    // the staging buffer holds 2n int2 pairs; the plan's hook capacity bounds both lists
    w.dense_edge_cap = g->dense_cap > 0 ? std::min<int64_t>(2 * g->n, g->link_edges) : 0;
    w.dense_threshold = g->dense_threshold;
    w.dense_cap = (int32_t)g->dense_cap;
    w.table_words = g->table_words;
    w.table_stride = table_stride(g->table_words);
    w.nbox = g->nbox;
    w.block = g->block;
    w.n = g->n;
    w.ncell = g->ncell;
    w.ntiles = g->ntiles;
    w.n_plain = g->n_plain;
    return w;
}

// HIP error behind the calling thread's last FOF_EDEVICE.
thread_local hipError_t g_last_device_error = hipSuccess;

int dev_err(hipError_t e)
{
    if (e == hipSuccess)
        return FOF_OK;
    g_last_device_error = e;
    return FOF_EDEVICE;
}

// Helper streams made by fof_init, one per device; calls that use one hold the lock, so
// that concurrent callers do not interleave their fork and join events.
constexpr int kMaxDevices = 64;
SideStream g_side[kMaxDevices];
bool g_side_ok[kMaxDevices];
std::mutex g_side_lock;

// The runtime's last-error slot may hold an error of another caller's earlier API call;
// clear it so that only this call's launches are reported.
void clear_stale_error() { (void)hipGetLastError(); }

// Device addresses of the static workspace (`scratch` below), one per device: the array's
// host-side name is only a stand-in, so kernels get the address the runtime reports for
// the current device.  Looked up once per device, under the lock.
void *g_scratch[kMaxDevices];
std::mutex g_scratch_lock;

// Descriptor block of a one-box plan, written into the static workspace by a kernel whose
// argument carries it (no host copy, nothing allocated).
__global__ void k_put_desc(BoxDesc d, BoxDesc *dst)
{
    if (threadIdx.x == 0)
        *dst = d;
}

__global__ void k_copy_status(const Counters *ctr, int32_t *status)
{
    if (threadIdx.x == 0)
        *status = ctr->status;
}

__global__ void k_copy_word(const int32_t *from, int32_t *to)
{
    if (threadIdx.x == 0)
        *to = *from;
}

}  // namespace
}  // namespace fof

// Workspace of fof_find_groups_static: one copy per device, held until the process ends.
static __device__ __align__(256) unsigned char scratch[FOF_STATIC_SCRATCH_BYTES];

namespace fof {
namespace {

// The current device's address of `scratch`, found with hipGetSymbolAddress on first use.
int static_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return FOF_EDEVICE;
    if (dev >= kMaxDevices)
        return FOF_ENOTSUP;
    std::lock_guard<std::mutex> hold(g_scratch_lock);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return dev_err(e);
        if (!p || ((uintptr_t)p % kAlign) != 0)
            return FOF_EDEVICE;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return FOF_OK;
}

}  // namespace
}  // namespace fof

using namespace fof;

extern "C" {

int fof_workspace_bytes(int32_t nbox, const int64_t *count, const fof_box *box,
                        const fof_tune *tune, fof_grid *grid, void *desc, size_t desc_cap)
{
    if (nbox < 1 || !count || !box || !grid)
        return FOF_EINVAL;
    if (tune && ((tune->flags & ~FOF_TUNE_NO_TILES) != 0 || tune->link_edges < 0 ||
                 tune->block < 0 || (tune->block % kWave) != 0 ||
                 tune->block > 1024 || !(tune->cell_side >= 0.0) ||
                 !(tune->cell_factor >= 0.0) || !isfinite(tune->cell_factor) ||
                 tune->dense_cells < 0))
        return FOF_EINVAL;
    int64_t n = 0, ncell = 0, ntiles = 0, n_plain = 0;
    int32_t mmax = 1, any_dense = 0;
    BoxDesc *out = (BoxDesc *)desc;
    const size_t need = sizeof(BoxDesc) * (size_t)nbox;
    if (desc && desc_cap < need)
        return FOF_EINVAL;
    for (int32_t k = 0; k < nbox; ++k) {
        if (count[k] < 0 || !box_ok(box[k]))
            return FOF_EINVAL;
        BoxDesc d;
        memset(&d, 0, sizeof(d));
        int rc = plan_box(box[k], count[k], tune, ncell, n, &d);
        if (rc)
            return rc;
        d.tile_base = ntiles;
        if (d.tiled)
            ntiles += (int64_t)d.ntile[0] * d.ntile[1] * d.ntile[2];
        else
            n_plain += count[k];
        n += count[k];
        ncell += (int64_t)d.nc[0] * d.nc[1] * d.nc[2];
        if (n > INT32_MAX || ncell > INT32_MAX - 1)
            return FOF_EINVAL;
        if (d.m > mmax)
            mmax = d.m;
        any_dense |= d.dense_ok;
        if (out)
            out[k] = d;
    }
    // Dense (clique-cell) path: cells holding more than `thr` particles.  The table count is
    // the exact bound n / (thr + 1), limited to 2 GiB of tables and to tune->dense_cells;
    // cells beyond the cap take the plain path and set FOF_STATUS_DENSE_CAP.
    int32_t thr = (tune && tune->dense_threshold) ? tune->dense_threshold : kDefaultDense;
    int32_t words = (mmax * mmax * mmax + 31) / 32;
    int64_t dense_cap = 0;
    if (thr > 0 && any_dense && n > thr) {
        dense_cap = n / ((int64_t)thr + 1) + 1;
        if (dense_cap > ncell)
            dense_cap = ncell;
        int64_t lim = ((int64_t)2 << 30) / (4 * (int64_t)table_stride(words));
        if (dense_cap > lim)
            dense_cap = lim;
        if (tune && tune->dense_cells > 0 && dense_cap > tune->dense_cells)
            dense_cap = tune->dense_cells;
    }
    if (thr <= 0)
        thr = -1;
    const int64_t link_edges =
        (tune && tune->link_edges > 0) ? (int64_t)tune->link_edges : link_edge_cap(n);
    Layout L = layout(nbox, n, ncell, dense_cap, words, ntiles, link_edges);
    memset(grid, 0, sizeof(*grid));
    grid->nbox = nbox;
    grid->block = (tune && tune->block) ? tune->block : kDefaultBlock;
    grid->n = n;
    grid->ncell = ncell;
    grid->dense_threshold = thr;
    grid->ntiles = ntiles;
    grid->n_plain = n_plain;
    grid->link_edges = link_edges;
    grid->dense_cap = dense_cap;
    grid->table_words = words;
    grid->ws_bytes = L.total;
    grid->desc_bytes = need;
    grid->off_desc = L.off_desc;
    grid->off_status = L.off_status;
    grid->off_counters = L.off_status;
    grid->off_cell_count = L.off_cell_count;
    grid->off_cell_start = L.off_cell_start;
    grid->off_rank = L.off_rank;
    grid->off_sorted = L.off_sorted;
    grid->off_parent = L.off_parent;
    grid->off_flags = L.off_flags;
    grid->off_keep = L.off_keep;
    grid->off_scan = L.off_scan;
    grid->off_dense = L.off_dense;
    grid->off_table = L.off_table;
    grid->off_aux = L.off_rank;
    grid->off_units = L.off_cnt;
    return FOF_OK;
}

int fof_build_grid(const fof_grid *grid, const float *pos, void *ws, size_t ws_bytes,
                   void *stream)
{
    if (int rc = ws_check(grid, ws, ws_bytes))
        return rc;
    if (grid->n > 0 && !pos)
        return FOF_EINVAL;
    Work w = resolve(grid, ws);
    clear_stale_error();
    return dev_err(launch_build(w, pos, (hipStream_t)stream));
}

static bool sample_ok(const fof_grid *grid, const fof_sample *S)
{
    const bool prob_ok =
        S->form == FOF_PROB_DISTANCE
            ? S->tau > 0.0 && isfinite(S->tau) && isfinite(S->b)
            : S->form == FOF_PROB_QUADRATIC && S->alpha > 0.0 && isfinite(S->alpha) &&
                  S->b > 0.0 && isfinite(S->b);
    return grid->nbox == 1 && S->K >= 1 && S->K <= 65535 && S->edge_cap >= 0 && prob_ok &&
           S->s_first >= 0 && S->s_first <= INT32_MAX - S->K &&
           S->n_edges && S->scratch && ((uintptr_t)S->scratch % 256) == 0 &&
           (S->edge_cap == 0 || (S->ei && S->ej && S->d2)) &&
           S->scratch_bytes >= FOF_SAMPLE_SCRATCH_BYTES(grid->n, S->K, S->edge_cap) &&
           sample_layout_ok(*S, grid->n);
}

int fof_link(const fof_grid *grid, void *ws, size_t ws_bytes, const fof_sample *sample,
             int32_t *root, void *stream)
{
    if (int rc = ws_check(grid, ws, ws_bytes))
        return rc;
    Work w = resolve(grid, ws);
    clear_stale_error();
    if (sample) {
        if (!sample_ok(grid, sample))
            return FOF_EINVAL;
        return dev_err(launch_sample(w, *sample, root, (hipStream_t)stream));
    }
    if (grid->n > 0 && !root)
        return FOF_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices && g_side_ok[dev]) {
        std::lock_guard<std::mutex> hold(g_side_lock);
        return dev_err(launch_link(w, root, (hipStream_t)stream, &g_side[dev]));
    }
    return dev_err(launch_link(w, root, (hipStream_t)stream, nullptr));
}

int fof_groups(const fof_grid *grid, void *ws, size_t ws_bytes, const fof_sample *sample,
               int32_t min_size, const float *vel, int32_t cap, int32_t *group_id,
               int32_t *n_groups, int32_t *sizes, double *com, double *vmean, double *sigv,
               void *stream)
{
    if (int rc = ws_check(grid, ws, ws_bytes))
        return rc;
    if (sample) {  // per-sample catalogues of the K sampled graphs
        if (!sample_ok(grid, sample) || min_size < 2 || !n_groups || cap < 0 ||
            (cap > 0 && (!sizes || !com)) || vel || vmean || sigv || group_id)
            return FOF_EINVAL;
        Work w = resolve(grid, ws);
        clear_stale_error();
        return dev_err(launch_groups_sampled(w, *sample, min_size, cap, n_groups, sizes, com,
                                             (hipStream_t)stream));
    }
    if (!n_groups || cap < 0 || (grid->n > 0 && !group_id) || (cap > 0 && !sizes))
        return FOF_EINVAL;
    if ((vmean == nullptr) != (sigv == nullptr) || (vel == nullptr && vmean != nullptr))
        return FOF_EINVAL;
    Work w = resolve(grid, ws);
    clear_stale_error();
    return dev_err(launch_groups(w, min_size, vel, cap, group_id, n_groups, sizes, com, vmean,
                                 sigv, (hipStream_t)stream));
}

int fof_backward(const fof_grid *grid, void *ws, size_t ws_bytes, int32_t mode,
                 const int32_t *group_id, int32_t G,
                 const int32_t *sizes, const double *vmean, const double *sigv, const float *vel,
                 const double *g_mass, const double *g_com, const double *g_sigv,
                 const fof_sample *sample, const double *loss, int32_t baseline, float *grad_pos,
                 float *grad_vel, void *stream)
{
    (void)g_mass;  // the member count has zero gradient with memberships frozen
    if (!grid || grid->n < 0)
        return FOF_EINVAL;
    if (mode == FOF_SCORE) {
        if (int rc = ws_check(grid, ws, ws_bytes))
            return rc;
        if (!sample || !sample_ok(grid, sample) || !loss ||
            baseline < FOF_BASELINE_NONE || baseline > FOF_BASELINE_LOO)
            return FOF_EINVAL;
        Work w = resolve(grid, ws);
        clear_stale_error();
        return dev_err(launch_score(w, *sample, loss, baseline, grad_pos, (hipStream_t)stream));
    }
    if (mode != FOF_FROZEN)
        return FOF_EINVAL;
    if (G < 0 || (grid->n > 0 && !group_id) || (G > 0 && !sizes))
        return FOF_EINVAL;
    if (grad_vel && g_sigv && (!vel || !vmean || !sigv))
        return FOF_EINVAL;
    const int32_t block = grid->block > 0 ? grid->block : kDefaultBlock;
    clear_stale_error();
    return dev_err(launch_backward(grid->n, block, group_id, G, sizes, vmean, sigv, vel, g_com,
                                   g_sigv, grad_pos, grad_vel, (hipStream_t)stream));
}

int fof_group_dispersion(const fof_grid *grid, void *ws, size_t ws_bytes, int32_t cap,
                         const int32_t *n_groups, const int32_t *sizes, const double *com,
                         double *sigx, void *stream)
{
    if (int rc = ws_check(grid, ws, ws_bytes))
        return rc;
    if (cap < 0 || !n_groups || (cap > 0 && (!sizes || !com || !sigx)))
        return FOF_EINVAL;
    Work w = resolve(grid, ws);
    clear_stale_error();
    return dev_err(launch_group_dispersion(w, cap, n_groups, sizes, com, sigx,
                                           (hipStream_t)stream));
}

int fof_backward_dispersion(const fof_grid *grid, void *ws, size_t ws_bytes, const float *pos,
                            const int32_t *group_id, int32_t G, const int32_t *sizes,
                            const double *com, const double *sigx, const double *g_sigx,
                            float *grad_pos, void *stream)
{
    if (int rc = ws_check(grid, ws, ws_bytes))
        return rc;
    if (G < 0)
        return FOF_EINVAL;
    if (grid->n > 0 && G > 0 && (!pos || !group_id || !sizes || !com || !sigx || !g_sigx ||
                                 !grad_pos))
        return FOF_EINVAL;
    Work w = resolve(grid, ws);
    clear_stale_error();
    return dev_err(launch_backward_dispersion(w, pos, group_id, G, sizes, com, sigx, g_sigx,
                                              grad_pos, (hipStream_t)stream));
}

size_t fof_subhalo_scratch_bytes(int64_t n, int32_t G)
{
    return n < 0 || G < 0 ? 0 : subhalo_scratch_bytes(n, G);
}

int fof_subhalo(const fof_grid *grid, void *ws, size_t ws_bytes, const float *pos,
                const float *vel, const int32_t *group_id, int32_t G, const int32_t *sizes,
                const double *norm_x, const double *norm_v, double b6, void *scratch,
                size_t scratch_bytes, int32_t *sub, void *stream)
{
    if (int rc = ws_check(grid, ws, ws_bytes))
        return rc;
    if (G < 0 || G > grid->n || !(b6 > 0.0) || !isfinite(b6))
        return FOF_EINVAL;
    if (grid->n > 0 && !sub)
        return FOF_EINVAL;
    if (grid->n > 0 && G > 0 &&
        (!pos || !vel || !group_id || !sizes || !norm_x || !norm_v || !scratch ||
         ((uintptr_t)scratch % 256) != 0 || scratch_bytes < subhalo_scratch_bytes(grid->n, G)))
        return FOF_EINVAL;
    Work w = resolve(grid, ws);
    clear_stale_error();
    return dev_err(launch_subhalo(w, pos, vel, group_id, G, sizes, norm_x, norm_v, b6, scratch,
                                  sub, (hipStream_t)stream));
}

int fof_status(const fof_grid *grid, void *ws, size_t ws_bytes, int32_t **status)
{
    if (int rc = ws_check(grid, ws, ws_bytes))
        return rc;
    if (!status)
        return FOF_EINVAL;
    *status = (int32_t *)((char *)ws + grid->off_status);
    return FOF_OK;
}

int fof_init(void)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return FOF_EDEVICE;
    if (dev >= kMaxDevices)
        return FOF_ENOTSUP;
    void *sp = nullptr;
    if (int rc = static_scratch(&sp))
        return rc;
    std::lock_guard<std::mutex> hold(g_side_lock);
    if (g_side_ok[dev])
        return FOF_OK;
    SideStream &sd = g_side[dev];
    hipError_t e = hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&sd.cc, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipEventCreateWithFlags(&sd.join, hipEventDisableTiming);
    if (e != hipSuccess)
        return dev_err(e);
    g_side_ok[dev] = true;
    return FOF_OK;
}

int fof_find_groups_static(const fof_box *box, int64_t n, const fof_tune *tune,
                           const float *pos, int32_t min_size, const float *vel, int32_t cap,
                           int32_t *root, int32_t *group_id, int32_t *n_groups, int32_t *sizes,
                           double *com, double *vmean, double *sigv, int32_t *status,
                           void *stream)
{
    if (!box || n < 0 || !n_groups || !status || cap < 0 || (cap > 0 && (!sizes || !com)) ||
        (n > 0 && (!pos || !root || !group_id)))
        return FOF_EINVAL;
    if ((vmean == nullptr) != (sigv == nullptr) || (vel == nullptr && vmean != nullptr))
        return FOF_EINVAL;
    fof_grid grid;
    BoxDesc desc;
    if (int rc = fof_workspace_bytes(1, &n, box, tune, &grid, &desc, sizeof(desc)))
        return rc;
    if (grid.ws_bytes > (size_t)FOF_STATIC_SCRATCH_BYTES)
        return FOF_ENOMEM;
    void *ws = nullptr;
    if (int rc = static_scratch(&ws))
        return rc;
    const hipStream_t s = (hipStream_t)stream;
    Work w = resolve(&grid, ws);
    clear_stale_error();
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, desc,
                       (BoxDesc *)((char *)ws + grid.off_desc));
    hipError_t e = launch_build(w, pos, s);
    if (e == hipSuccess)
        e = launch_link(w, root, s, nullptr);
    if (e == hipSuccess)
        e = launch_groups(w, min_size, vel, cap, group_id, n_groups, sizes, com, vmean, sigv, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, s, w.ctr, status);
        e = hipGetLastError();
    }
    return dev_err(e);
}

// Streaming labelling: slab geometry and the tuning every slab run uses (the whole box's
// cell grid, no link tiles, which would cover the whole grid for each slab).
static int stream_setup(const fof_box *box, int64_t n, int32_t nslab, const fof_tune *tune,
                        SlabGeom *G, fof_tune *st)
{
    if (!box || !box_ok(*box) || n < 0 || n > INT32_MAX || nslab < 1 || nslab > slab_max())
        return FOF_EINVAL;
    G->Lz = box->L[2];
    G->nslab = nslab;
    G->width = box->L[2] / (double)nslab;
    G->ghost = 1.5 * box->b;
    if (nslab > 1 && !(G->width >= 2.0 * G->ghost))
        return FOF_EINVAL;
    memset(st, 0, sizeof(*st));
    if (tune)
        *st = *tune;
    if (!(st->cell_side > 0.0) && n > 0) {
        const double V = box->L[0] * box->L[1] * box->L[2];
        const double f = st->cell_factor > 0.0 ? st->cell_factor : 1.0;
        st->cell_side = f * cbrt(V / (double)n);
        st->cell_factor = 0.0;
    }
    st->flags |= FOF_TUNE_NO_TILES;
    return FOF_OK;
}

// Byte offsets of the streaming workspace: the slab plan's workspace (sized for the largest
// slab), the slab's positions, map to original indices and labels, the gather's chunk
// counts, offsets and scan scratch, and the stream's status word.
struct StreamLayout {
    size_t plan, spos, map, sroot, ccount, coff, scan, status, total;
    int64_t cap;
};

static int stream_layout(const fof_box *box, int64_t n, int32_t nslab, const int64_t *counts,
                         const fof_tune *st, StreamLayout *out)
{
    size_t plan = 0;
    int64_t cap = 0;
    for (int32_t k = 0; k < nslab; ++k) {
        if (counts[k] < 0 || counts[k] > INT32_MAX)
            return FOF_EINVAL;
        fof_grid g;
        if (int rc = fof_workspace_bytes(1, &counts[k], box, st, &g, nullptr, 0))
            return rc;
        plan = plan > g.ws_bytes ? plan : g.ws_bytes;
        cap = cap > counts[k] ? cap : counts[k];
    }
    const int64_t nch = slab_chunks(n);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    out->plan = take(plan);
    out->spos = take(12 * (size_t)cap);
    out->map = take(4 * (size_t)cap);
    out->sroot = take(4 * (size_t)cap);
    out->ccount = take(4 * (size_t)nch);
    out->coff = take(4 * (size_t)(nch + 1));
    out->scan = take(4 * (size_t)scan_scratch_elems(nch));
    out->status = take(sizeof(int32_t));
    out->total = o;
    out->cap = cap;
    return FOF_OK;
}

int fof_stream_counts(const fof_box *box, int64_t n, const float *pos, int32_t nslab,
                      int64_t *counts, void *stream)
{
    SlabGeom G;
    fof_tune st;
    if (int rc = stream_setup(box, n, nslab, nullptr, &G, &st))
        return rc;
    if (!counts || (n > 0 && !pos))
        return FOF_EINVAL;
    clear_stale_error();
    return dev_err(launch_slab_count(pos, n, G, counts, (hipStream_t)stream));
}

int fof_stream_workspace_bytes(const fof_box *box, int64_t n, int32_t nslab,
                               const int64_t *counts, const fof_tune *tune, size_t *bytes)
{
    SlabGeom G;
    fof_tune st;
    if (int rc = stream_setup(box, n, nslab, tune, &G, &st))
        return rc;
    if (!counts || !bytes)
        return FOF_EINVAL;
    StreamLayout SL;
    if (int rc = stream_layout(box, n, nslab, counts, &st, &SL))
        return rc;
    *bytes = SL.total;
    return FOF_OK;
}

int fof_link_stream(const fof_box *box, int64_t n, const float *pos, int32_t nslab,
                    const int64_t *counts, const fof_tune *tune, void *ws, size_t ws_bytes,
                    int32_t *root, int32_t *status, void *stream)
{
    SlabGeom G;
    fof_tune st;
    if (int rc = stream_setup(box, n, nslab, tune, &G, &st))
        return rc;
    if (!counts || !ws || ((uintptr_t)ws % kAlign) != 0 || !status || (n > 0 && (!pos || !root)))
        return FOF_EINVAL;
    StreamLayout SL;
    if (int rc = stream_layout(box, n, nslab, counts, &st, &SL))
        return rc;
    if (ws_bytes < SL.total)
        return FOF_ENOMEM;
    const hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    float *spos = (float *)(base + SL.spos);
    int32_t *map = (int32_t *)(base + SL.map), *sroot = (int32_t *)(base + SL.sroot);
    int32_t *ccount = (int32_t *)(base + SL.ccount), *coff = (int32_t *)(base + SL.coff);
    int32_t *scan = (int32_t *)(base + SL.scan), *sstat = (int32_t *)(base + SL.status);
    clear_stale_error();
    hipError_t e = launch_fill_i32(sstat, 1, 0, s);
    if (e == hipSuccess)
        e = launch_fuse_init(root, n, s);
    for (int32_t k = 0; k < nslab && e == hipSuccess; ++k) {
        const int64_t m = counts[k];
        if (m == 0)
            continue;
        e = launch_slab_gather(pos, n, G, k, ccount, coff, scan, m, spos, map, sstat, s);
        if (e != hipSuccess)
            break;
        fof_grid grid;
        BoxDesc desc;
        if (int rc = fof_workspace_bytes(1, &m, box, &st, &grid, &desc, sizeof(desc)))
            return rc;
        void *pws = base + SL.plan;
        Work w = resolve(&grid, pws);
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, desc,
                           (BoxDesc *)((char *)pws + grid.off_desc));
        e = launch_build(w, spos, s);
        if (e == hipSuccess)
            e = launch_link(w, sroot, s, nullptr);
        if (e == hipSuccess)
            e = launch_or_status(w.ctr, sstat, s);
        if (e == hipSuccess)
            e = launch_slab_fuse(map, sroot, m, root, s);
    }
    if (e == hipSuccess)
        e = launch_fuse_final(root, n, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_copy_word, dim3(1), dim3(64), 0, s, sstat, status);
        e = hipGetLastError();
    }
    return dev_err(e);
}

int fof_last_device_error(const char **name)
{
    if (name)
        *name = hipGetErrorName(g_last_device_error);
    return (int)g_last_device_error;
}

const char *fof_strerror(int code)
{
    switch (code) {
    case FOF_OK:
        return "ok";
    case FOF_EINVAL:
        return "invalid argument";
    case FOF_ENOMEM:
        return "workspace too small";
    case FOF_EOVERFLOW:
        return "more groups than the output capacity";
    case FOF_EDEVICE:
        return "HIP launch failed";
    case FOF_ENOTSUP:
        return "option not supported";
    default:
        return "unknown error";
    }
}

}  // extern "C"
