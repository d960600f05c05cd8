/*
 * fof.h -- C ABI of the MI355X Friends-of-Friends library (libfof.so).
 *
 * The library finds Friends-of-Friends groups in periodic boxes of float32 particles: two
 * particles are friends when their minimum-image separation is below the linking length b,
 * and groups are the connected components of the friend relation (paper: Sec. 2, steps
 * (i)-(vi); Sec. 2.2 linked-cell grid; Alg. 2).  The forward pass is exact; gradients
 * (Sec. 3) are separate calls.
 *
 * Conventions for every entry point:
 *  - Pointers marked (dev) are device pointers on the device that owns `stream`; pointers
 *    marked (host) are host memory.  The caller owns every buffer.  No call allocates,
 *    frees, synchronises or prints: all device work is enqueued on `stream` (a hipStream_t
 *    passed as void*; NULL = the default stream), or, after fof_init, partly on a helper
 *    stream that fof_link forks from and joins back to `stream`.
 *  - Return value: FOF_OK (0) or a negative FOF_E* code.  Argument errors are detected on the
 *    host before anything is enqueued.  Data errors that only the device can see
 *    (coordinates outside [0, L) or NaN, more groups than the caller's table holds) set bits
 *    of the device status word (fof_status).
 *  - Every call that takes the workspace `ws` also takes its size `ws_bytes`: FOF_ENOMEM when
 *    it is below grid->ws_bytes (nothing is enqueued).
 *  - Particle indices are int32: n <= 2^31 - 1 in total.
 *  - Several boxes can be processed in one call ("batch"): box k owns the particles
 *    [offset_k, offset_k + count_k) of the concatenated arrays, with offset_0 = 0 and
 *    offset_{k+1} = offset_k + count_k.  A single box is the batch of one.  Components never
 *    span boxes; labels are global indices into the concatenated arrays.
 */
#ifndef FOF_H
#define FOF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FOF_OK 0
#define FOF_EINVAL (-1)     /* bad argument (null pointer, n out of range, b or L invalid)   */
#define FOF_ENOMEM (-2)     /* workspace smaller than fof_workspace_bytes asked for          */
#define FOF_EOVERFLOW (-3)  /* more groups than `cap`; counts still hold the true totals    */
#define FOF_EDEVICE (-4)    /* a HIP launch failed                                            */
#define FOF_ENOTSUP (-5)    /* option not supported by this library                           */

/* Bits of the device status word (see fof_status). */
#define FOF_STATUS_RANGE 1u     /* some coordinate was NaN or outside [0, L)                  */
#define FOF_STATUS_DENSE_CAP 2u /* dense-cell tables overflowed; those cells took the plain path */
#define FOF_STATUS_EDGE_CAP 4u  /* more candidate edges than fof_sample.edge_cap              */
#define FOF_STATUS_OVERFLOW 8u  /* fof_groups found more groups than `cap` (in some sample); the
                                   group counts hold the true totals, the tables the first cap */
#define FOF_STATUS_SLAB_CAP 16u /* fof_link_stream: a slab's member count differed from the
                                   count it was planned with (the labels are not valid)        */

/* fof_backward modes */
#define FOF_FROZEN 0 /* frozen assignment (paper Sec. 3.1)                                     */
#define FOF_SCORE 1  /* score-function (REINFORCE) estimator over sampled edges (Sec. 3.2)    */

/* Baselines of the score-function estimator */
#define FOF_BASELINE_NONE 0
#define FOF_BASELINE_MEAN 1 /* mean loss of the K samples                                       */
#define FOF_BASELINE_LOO 2  /* mean loss of the other K-1 samples (exactly unbiased)            */

/* One periodic box: side lengths L (physical) and the physical linking length b.
 * Requirements: L[c] finite and > 0, b finite and > 0, 2 b < L[c] for every axis (so that
 * within b the minimum image of a pair is unique).  The dimensionless form
 * b_phys = b_dimless * (V/N)^(1/3) (paper Sec. 2 step (ii)) is the caller's business. */
typedef struct fof_box {
    double L[3];
    double b;
} fof_box;

/* Tuning knobs.  Zero fields take defaults.  None of them changes any result. */
#define FOF_TUNE_NO_TILES 1u /* link every particle from global memory, without LDS tiles    */
typedef struct fof_tune {
    double cell_side;        /* requested coarse cell side; raised to b plus a rounding margin */
    int32_t dense_threshold; /* cells holding more particles take the clique-cell path;
                                0 = default, < 0 = never                                      */
    int32_t block;           /* threads per block for per-particle kernels (multiple of 64)    */
    uint32_t flags;          /* FOF_TUNE_* bits; other bits must be 0                          */
    int32_t link_edges;      /* capacity of the link pass's deferred cross-tile hooks (pairs);
                                0 = n/4 + 65536.  Tiles that overflow it are relinked with
                                direct hooks, so it trades memory for time only             */
    double cell_factor;      /* when cell_side is 0: the coarse side of every box is this many
                                of its own mean particle spacings (0 = 1), so one value suits
                                a batch of boxes of different densities                       */
    int64_t dense_cells;     /* at most this many dense cells get clique tables (0 = as many
                                as the threshold allows, up to 2 GiB of tables); cells beyond
                                it take the plain path and set FOF_STATUS_DENSE_CAP, so it
                                trades memory for time only                                   */
} fof_tune;

/* Stochastic linking (paper Sec. 3.2: every potential edge between nearby particles is a
 * Bernoulli variable).  The candidate edges are the pairs closer than the plan's linking
 * length (the cut radius r_c: plan the batch with fof_box.b = r_c); edge e = {i, j} is kept
 * in sample s with probability p_e = 1 / (1 + exp(-z_e)), d_e its minimum-image distance,
 *   form FOF_PROB_DISTANCE:  z_e = (b - d_e) / tau,
 *   form FOF_PROB_QUADRATIC: z_e = (alpha * (b*b - d_e^2)) / (b*b)  (the paper's Bernoulli
 *                            form, evaluated in this order in FP64),
 * when u(seed, s, i, j) < p_e, where u is the first word of
 * Philox4x64-10 (Salmon et al. 2011) at counter (i | j << 32, s, 0, 0) and key (seed, 0),
 * shifted right by 11 and scaled by 2^-53, on original indices i < j.  A call covers the
 * samples s = s_first .. s_first + K - 1 (local sample k = s - s_first), so a batch of K
 * equals K calls of one sample each.  All pointers are device pointers owned by the caller. */
typedef struct fof_sample {
    double b;           /* linking length of the probability                                   */
    double tau;         /* temperature, > 0                                                    */
    uint64_t seed;
    int32_t K;          /* sampled graphs, 1 <= K <= 65535                                     */
    int32_t edge_cap;   /* capacity of ei, ej, d2                                              */
    int32_t *ei, *ej;   /* [edge_cap] candidate edges (original indices, ei < ej), any order   */
    double *d2;         /* [edge_cap] squared minimum-image distances                          */
    int32_t *n_edges;   /* [1] number of candidate edges (may exceed edge_cap: status bit)     */
    void *scratch;      /* >= FOF_SAMPLE_SCRATCH_BYTES(n, K, edge_cap) bytes, 256-aligned      */
    size_t scratch_bytes;
    int32_t form;       /* FOF_PROB_DISTANCE (0) or FOF_PROB_QUADRATIC (1)                     */
    double alpha;       /* relaxation of FOF_PROB_QUADRATIC, > 0 (tau is then unused)          */
    int32_t s_first;    /* index of the first sample, >= 0, s_first + K <= 2^31 - 1            */
} fof_sample;

#define FOF_PROB_DISTANCE 0
#define FOF_PROB_QUADRATIC 1

/* Scratch of the sampled labelling: a vertex map over all particles, the sorted ends of
 * every edge, per sample a union-find, member counts and group numbering over the
 * particles that touch a candidate edge (at most vcap = min(n, 2 edge_cap) of them, so the
 * scratch and the per-sample passes scale with the edge capacity the caller chooses), the
 * keep bits of every edge (K <= 64) and the score gradient's fixed-point sums over those
 * particles. */
#define FOF_SAMPLE_VCAP(n, edge_cap)                                                          \
    (2 * (size_t)(edge_cap) < (size_t)(n) ? 2 * (size_t)(edge_cap) : (size_t)(n))
#define FOF_SAMPLE_SCRATCH_BYTES(n, K, edge_cap)                                              \
    (8192 + 8 * ((size_t)(n) + 1) + 4 * ((size_t)(n) / 2048 + 2) + 8 * (size_t)(edge_cap) +   \
     8 * (size_t)(K) + 8 * FOF_SAMPLE_VCAP(n, edge_cap) +                                     \
     12 * (size_t)(K) * FOF_SAMPLE_VCAP(n, edge_cap) +                                        \
     4 * ((size_t)(K) * FOF_SAMPLE_VCAP(n, edge_cap) / 2048 + 3) +                            \
     24 * FOF_SAMPLE_VCAP(n, edge_cap) + 8 + 8 * (size_t)(edge_cap))

/* Host-side plan of one batch: filled by fof_workspace_bytes, then passed unchanged to the
 * other calls.  Plain data; the byte offsets locate the regions of the caller's workspace. */
typedef struct fof_grid {
    int32_t nbox;
    int32_t block;
    int64_t n;            /* total particles                                                  */
    int64_t ncell;        /* total coarse cells over all boxes                                */
    int64_t dense_cap;    /* dense cells that can get clique tables                           */
    int64_t ntiles;       /* link tiles (blocks of the LDS-tiled link kernel)                 */
    int64_t n_plain;      /* particles of the boxes too small for link tiles                  */
    int32_t dense_threshold;
    int32_t table_words;  /* 32-bit words of one clique bitmask                               */
    int64_t link_edges;   /* capacity of the deferred link hooks (pairs)                      */
    size_t ws_bytes;      /* size of the workspace the caller must provide                    */
    size_t desc_bytes;    /* size of the box descriptor block                                 */
    size_t off_desc;      /* where the caller copies the descriptor block (see below)         */
    size_t off_status, off_counters, off_cell_count, off_cell_start, off_rank, off_sorted,
        off_parent, off_flags, off_keep, off_scan, off_dense, off_units, off_table, off_aux;
} fof_grid;

/* Plans a batch of `nbox` boxes with count[k] particles each (host arrays).  Fills *grid.
 * If `desc` (host) is not NULL it must hold grid->desc_bytes bytes (call once with NULL to
 * learn the size): it receives the packed box descriptors, which the caller must copy into
 * the workspace at byte offset grid->off_desc before fof_build_grid runs (the library never
 * copies host memory itself).  Errors: FOF_EINVAL for a bad box, count < 0, a total above
 * 2^31 - 1, or a `desc` buffer smaller than desc_bytes. */
int fof_workspace_bytes(int32_t nbox, const int64_t *count /*host*/, const fof_box *box /*host*/,
                        const fof_tune *tune /*host, may be NULL*/, fof_grid *grid /*host*/,
                        void *desc /*host or NULL*/, size_t desc_cap);

/* Cell binning (paper Alg. 2: cell indexing with x fastest, sort by cell).  pos (dev) is
 * float32 [n][3] (x, y, z per particle, AoS), every coordinate in [0, L) of its box.
 * Builds, inside ws (dev, grid->ws_bytes bytes, 256-byte aligned), the per-cell offsets and
 * the cell-sorted particle copy used by fof_link and fof_groups.  Clears the status word. */
int fof_build_grid(const fof_grid *grid, const float *pos /*dev*/, void *ws /*dev*/,
                   size_t ws_bytes, void *stream);

/* Friends-of-Friends labels (paper Sec. 2 steps (iii)-(v); Alg. 2 candidate search, minimum
 * image filter and label propagation, run here to convergence as a union-find).
 * root (dev, int32 [n]) receives, for every particle i, the smallest index j in the
 * connected component of i (so root[root[i]] == root[i]).  The link predicate is exact:
 * per axis d = (double)x_i - (double)x_j wrapped once by +-L when |d| > L/2, then
 * ((dx*dx + dy*dy) + dz*dz) < b*b in IEEE double without fused multiply-add.
 * With sample != NULL (single-box plans only; Sec. 3.2 stochastic linking): writes the
 * candidate edges into the sample buffers, links the K sampled graphs in the sample's
 * scratch (which fof_groups and fof_backward(FOF_SCORE) then read), and, only when root is
 * not NULL, writes root (dev, int32 [K][n]) the smallest-index labels of every sampled graph
 * (K * n words: leave it NULL when the per-sample group tables suffice). */
int fof_link(const fof_grid *grid, void *ws /*dev*/, size_t ws_bytes,
             const fof_sample *sample /*host or NULL*/, int32_t *root /*dev*/, void *stream);

/* Group catalogue (paper Sec. 2 step (vi); Alg. 2 compaction; Sec. 3.1 halo position).
 * Must follow fof_link without a sample (the labelling pass) on the same workspace: it reads
 * the union-find state and the list of linked particles that call leaves.  Components with at
 * least min_size members
 * are kept and numbered 0..G-1 in ascending order of their label (the smallest member
 * index); group_id (dev, int32 [n]) gets that number, or -1 for particles of cut
 * components.  *n_groups (dev, one int32) receives G.  For g < min(G, cap):
 *   sizes[g] (dev int32)       member count
 *   com[g][3] (dev double)     centre of mass: members unwrapped about the label particle
 *                              by minimum image, averaged, wrapped into [0, L)
 *   vmean[g][3], sigv[g]       (dev double, only when vel != NULL) mean velocity and the
 *                              1-D dispersion sqrt(sum_i sum_c (v_ic - vmean_c)^2 / (3 n))
 * vel (dev) is float32 [n][3] or NULL; vmean and sigv may be NULL when vel is NULL.
 * When G > cap the call sets FOF_STATUS_OVERFLOW in the status word (the device alone knows
 * G, and no call synchronises); *n_groups still holds G and group ids >= cap have no table
 * entries.
 *
 * Sampled form, sample != NULL (Sec. 3.2: the loss of each sampled graph is a function of its
 * halos): must follow fof_link with the same sample.  For each local sample k < K, the
 * components of that sampled graph with at least min_size >= 2 members, numbered in
 * ascending order of their label as above: n_groups (dev int32 [K]) gets G_k, and for
 * g < min(G_k, cap), sizes[k * cap + g] and com[(k * cap + g) * 3 + c] as above (FP64,
 * members unwrapped about the label particle).  Particles that touch no candidate edge are
 * singletons in every sample, so groups are built over the touched particles only; no K * n
 * array is written.  vel, vmean, sigv and group_id must be NULL.  G_k > cap sets
 * FOF_STATUS_OVERFLOW. */
int fof_groups(const fof_grid *grid, void *ws /*dev*/, size_t ws_bytes,
               const fof_sample *sample /*host or NULL*/, int32_t min_size, const float *vel,
               int32_t cap, int32_t *group_id, int32_t *n_groups, int32_t *sizes, double *com,
               double *vmean, double *sigv, void *stream);

/* Backward passes (paper Sec. 3: the forward is exact; gradients never differentiate the
 * neighbour structure).  mode = FOF_FROZEN (Sec. 3.1 and its table of differentiation
 * modes): memberships from the forward are held fixed.  With upstream gradients g_mass[G],
 * g_com[G][3], g_sigv[G] (dev double; any may be NULL = zero) of mass_g = n_g, com, sigv:
 *   grad_pos[i][c] = g_com[g][c] / n_g                        (mass has zero gradient)
 *   grad_vel[i][c] = g_sigv[g] (v_ic - vmean[g][c]) / (3 n_g sigv[g])   (0 if sigv[g] = 0)
 * where g = group_id[i]; particles with g < 0 or g >= G get zeros.  sizes, vmean, sigv are
 * the forward's outputs; G is the number of groups the tables hold (<= cap).
 * mode = FOF_SCORE (Sec. 3.2, REINFORCE): with the edges of the last fof_link(sample) and the
 * sampled graphs' losses loss[K] (dev double),
 *   grad_pos = (1/K) sum_k (loss_k - beta_k) sum_e (y_e,s_first+k - p_e) dz_e/dx,
 *   z_e as in fof_sample, dz_e/dx_i = -dz_e/dx_j = -(x_i - x_j)/(tau d_e) (FOF_PROB_DISTANCE;
 *   0 for an edge with d_e = 0, where the direction is undefined) or -2 alpha (x_i - x_j)/b^2
 *   (FOF_PROB_QUADRATIC), x_i - x_j the minimum image,
 * beta_s per `baseline` (FOF_BASELINE_*); the frozen-mode arguments are ignored and grad_vel
 * is not written.  The sums over edges are taken in 64-bit fixed point (a unit of about
 * 2^-40 of the largest possible term, max_s |loss_s - beta_s| / tau, or times 2 alpha r / b^2
 * with r the plan's linking length), so grad_pos is the same bit for bit from run to run
 * whatever the order of the edges; non-finite losses give NaN for every particle on an edge.
 * grad_pos and grad_vel (dev float32 [n][3]) may be NULL to skip them. */
int fof_backward(const fof_grid *grid, void *ws /*dev*/, size_t ws_bytes, int32_t mode,
                 const int32_t *group_id /*dev*/, int32_t G, const int32_t *sizes /*dev*/,
                 const double *vmean /*dev*/, const double *sigv /*dev*/, const float *vel /*dev*/,
                 const double *g_mass, const double *g_com, const double *g_sigv,
                 const fof_sample *sample /*host*/, const double *loss /*dev [K]*/,
                 int32_t baseline, float *grad_pos, float *grad_vel, void *stream);

/* Position dispersion of each group, the halo "decoration" of the decorated frozen
 * assignment (paper Sec. 3.1, its inverse mass proxy: the particle standard deviation):
 *   sigx[g] = sqrt(sum_{i in g} |mi(x_i - com[g])|^2 / (3 n_g)),  mi the per-axis minimum
 * image, FP64, the same 1-D reading as sigv; groups of one get 0.  Must follow fof_groups on
 * the same workspace with the same cap, and reads that call's n_groups, sizes and com (dev);
 * sigx (dev double [cap]) receives min(G, cap) values and zeros beyond. */
int fof_group_dispersion(const fof_grid *grid, void *ws /*dev*/, size_t ws_bytes, int32_t cap,
                         const int32_t *n_groups, const int32_t *sizes, const double *com,
                         double *sigx, void *stream);

/* Gradient of the decoration with memberships frozen (paper Sec. 3.1, decorated frozen
 * assignment): for every particle i with 0 <= g = group_id[i] < G and sigx[g] > 0,
 *   grad_pos[i][c] += g_sigx[g] * mi(pos[i][c] - com[g][c]) / (3 n_g sigx[g])
 * (the terms through com cancel).  ADDS to grad_pos (dev float32 [n][3]), so it composes with
 * fof_backward(FOF_FROZEN).  pos (dev float32 [n][3]) is the forward's input; group_id,
 * sizes, com and sigx are the forward's outputs (dev); g_sigx (dev double [G]). */
int fof_backward_dispersion(const fof_grid *grid, void *ws /*dev*/, size_t ws_bytes,
                            const float *pos,
                            const int32_t *group_id, int32_t G, const int32_t *sizes,
                            const double *com, const double *sigx, const double *g_sigx,
                            float *grad_pos, void *stream);

/* Six-dimensional sub-halo pass (paper Sec. 2, sub-halo finding): inside each host halo g
 * (the particles with group_id[i] == g, 0 <= g < G, as fof_groups labels them) a second
 * Friends-of-Friends pass in phase space, two members linking when
 *   |mi(x_i - x_j)|^2 / norm_x[g] + |v_i - v_j|^2 / norm_v[g] < b6^2,
 * the paper's metric with its normalisation factors dividing the squared separations as
 * printed (pass variances, e.g. sigx^2 and sigv^2, for a dispersion-scaled metric); mi is the
 * per-axis minimum image of the particle's box; each squared norm is summed
 * ((c0*c0 + c1*c1) + c2*c2) in FP64 from the float32 inputs.  Particles of different hosts
 * never link.  sub (dev int32 [n]) receives the smallest original index of each member's
 * phase-space component and -1 outside every host.  pos, vel (dev float32 [n][3]), group_id
 * (dev int32 [n]), sizes (dev int32 [G], the member count of each host), norm_x, norm_v
 * (dev double [G]; a host whose factors are not both positive splits into singletons).  scratch: dev, 256-byte aligned, >= fof_subhalo_scratch_bytes(n, G) bytes,
 * owned by the caller, contents not preserved.  Every pair of a host is tested (cost grows
 * with the square of the host's size).  Sizes that disagree with group_id drop the extra
 * members and set FOF_STATUS_RANGE (cleared by fof_build_grid); a negative size counts as 0
 * (all of that host's members are dropped), so the other hosts are unaffected.  FOF_EINVAL for b6 not
 * positive and finite, G < 0 or G > n, or missing buffers. */
size_t fof_subhalo_scratch_bytes(int64_t n, int32_t G);
int fof_subhalo(const fof_grid *grid, void *ws /*dev*/, size_t ws_bytes, const float *pos,
                const float *vel,
                const int32_t *group_id, int32_t G, const int32_t *sizes, const double *norm_x,
                const double *norm_v, double b6, void *scratch, size_t scratch_bytes,
                int32_t *sub, void *stream);

/* Device address of the int32 status word inside ws (FOF_STATUS_* bits; 0 = clean).  It is
 * cleared by fof_build_grid; read it after synchronising the stream. */
int fof_status(const fof_grid *grid, void *ws /*dev*/, size_t ws_bytes,
               int32_t **status /*host out: dev ptr*/);

/* Optional, once per device (the current one), before fof_link is called from a captured
 * or performance-critical context: creates a helper stream (default priority) and three
 * events, so that fof_link runs its dense-cell passes concurrently with the sparse passes
 * (fork, components-done and join through the events; the call still orders everything
 * after the caller's earlier work and before its later work).  Without it, every call runs on the caller's
 * stream alone.  Allocates no device memory.  Errors: FOF_EDEVICE, FOF_ENOTSUP (device
 * index 64 or above). */
int fof_init(void);

/* For callers that cannot allocate device memory: code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  One box, the whole labelling pipeline of
 * fof_build_grid + fof_link + fof_groups (same kernels, same results) with the workspace in a
 * static device array of FOF_STATIC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends, so the call needs no `ws` and allocates nothing.
 * box, tune: host, as for fof_workspace_bytes (one box of n particles).  pos, vel, root,
 * group_id, n_groups, sizes, com, vmean, sigv: as for fof_build_grid, fof_link and fof_groups
 * (dev, caller-owned).  status (dev, one int32) receives the device status word
 * (FOF_STATUS_* bits) at the end of the call; read it after synchronising.
 * Errors: FOF_ENOMEM when the plan's workspace exceeds FOF_STATIC_SCRATCH_BYTES (about
 * 73 bytes per particle: up to roughly 2.2 million particles), FOF_EINVAL as for the calls it
 * combines, FOF_EDEVICE, FOF_ENOTSUP (device index 64 or above).
 * Every call on one device shares that device's array, which keeps the last call's
 * contents: calls that overlap on one device (different streams or threads) race and must
 * be ordered by the caller.  Runs on `stream` only (no helper stream). */
#define FOF_STATIC_SCRATCH_BYTES ((size_t)160 << 20)
int fof_find_groups_static(const fof_box *box /*host*/, int64_t n,
                           const fof_tune *tune /*host, may be NULL*/, const float *pos /*dev*/,
                           int32_t min_size, const float *vel /*dev or NULL*/, int32_t cap,
                           int32_t *root, int32_t *group_id, int32_t *n_groups, int32_t *sizes,
                           double *com, double *vmean, double *sigv, int32_t *status /*dev*/,
                           void *stream);

/* Streaming labelling of one box in z-slabs, with a workspace bounded by the largest slab
 * (paper Sec. 2.3: the box is cut into slabs, each slab is processed with a ghost layer of
 * its neighbours' particles, and groups that meet in the overlap are fused).  Slab k of
 * nslab owns the particles with k L_z/nslab <= z < (k+1) L_z/nslab; its ghosts are the
 * particles of the two neighbouring slabs (periodically) within 1.5 b of the shared face, so
 * every friend pair lies in one slab's set.  Each slab is linked as a periodic box of the
 * full lengths holding only those particles (same kernels and predicate as fof_link, on the
 * cell grid the whole box would get), and the slab labels are fused in one union-find over
 * `root`: root (dev int32 [n]) receives exactly what fof_link gives for the whole box.
 * Three calls, so that no call synchronises:
 *   fof_stream_counts           writes the member count (own + ghosts) of every slab into
 *                               counts (dev int64 [nslab]);
 *   fof_stream_workspace_bytes  (host) the workspace for those counts (copied to the host
 *                               by the caller), in *bytes;
 *   fof_link_stream             the labels, with the same counts (host) and a workspace of
 *                               at least that size (dev, 256-byte aligned, caller-owned);
 *                               status (dev, one int32) receives the OR of the slab runs'
 *                               status bits, FOF_STATUS_SLAB_CAP if a slab's member
 *                               count differed from counts[k] (then root is not valid).
 * box: host; pos: dev float32 [n][3] in [0, L); tune: as for fof_workspace_bytes (host, may
 * be NULL; the slabs always run without link tiles).  Requirements: 1 <= nslab <= 4096 and,
 * for nslab > 1, L_z / nslab >= 3 b.  Errors: FOF_EINVAL, FOF_ENOMEM (workspace smaller
 * than fof_stream_workspace_bytes), FOF_EDEVICE. */
int fof_stream_counts(const fof_box *box /*host*/, int64_t n, const float *pos /*dev*/,
                      int32_t nslab, int64_t *counts /*dev*/, void *stream);
int fof_stream_workspace_bytes(const fof_box *box /*host*/, int64_t n, int32_t nslab,
                               const int64_t *counts /*host*/, const fof_tune *tune /*host*/,
                               size_t *bytes /*host*/);
int fof_link_stream(const fof_box *box /*host*/, int64_t n, const float *pos /*dev*/,
                    int32_t nslab, const int64_t *counts /*host*/, const fof_tune *tune /*host*/,
                    void *ws /*dev*/, size_t ws_bytes, int32_t *root /*dev*/,
                    int32_t *status /*dev*/, void *stream);

/* Static text for a FOF_E* code. */
const char *fof_strerror(int code);

/* The HIP error code (hipError_t) behind the calling thread's most recent FOF_EDEVICE, or 0.
 * If `name` is not NULL it receives the runtime's static name of that code. */
int fof_last_device_error(const char **name /*host out, may be NULL*/);

#ifdef __cplusplus
}
#endif
#endif /* FOF_H */
