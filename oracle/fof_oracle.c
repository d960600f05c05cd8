/*
 * CPU oracle for the Friends-of-Friends hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the slow, plain reference that the GPU library is checked against.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the product path never calls it.  It shares no code, header, table or helper with the
 * GPU library.
 *
 * What it computes (paper: Sec. 2 "Halo finding via Friends of Friends", steps (i)-(vi);
 * Alg. 2 "Periodic FoF with precomputed neighbour lists"; Sec. 3.1 "Frozen assignment"):
 *
 *   link predicate   two particles are friends when their periodic minimum-image
 *                    separation is below the linking length (Sec. 2 step (iv)).  Fixed
 *                    reading: per axis in x, y, z order d = (double)x_i - (double)x_j,
 *                    wrapped once by +-L when |d| > L/2; s = ((dx*dx + dy*dy) + dz*dz) in
 *                    double with no fused multiply-add; linked iff s < b*b (strict).
 *   components       groups are the connected components of the friend graph (Sec. 2
 *                    step (v)); the label of a particle is the smallest index in its
 *                    component, which is what min-label propagation from l_i = i (step (i),
 *                    Alg. 2 label propagation) converges to.  Computed here with a
 *                    union-find that always attaches the larger root under the smaller.
 *   candidates       a sparse cell list (Sec. 2.2 linked-cell grid, Alg. 2 cell indexing)
 *                    whose cell side is strictly larger than b, so the 27-cell stencil
 *                    is complete; neighbour cells are found by binary search over the
 *                    sorted cell keys (as Alg. 2 does with lower/upper bound).
 *   groups           sizes, a minimum-size cut, compaction of the kept labels in ascending
 *                    label order (Sec. 2 step (vi), Alg. 2 compaction).
 *   centre of mass   mean member position (Sec. 3.1 halo position), made periodic by
 *                    unwrapping each member about the label particle with the minimum
 *                    image and wrapping the mean back into [0, L).
 *   velocity moments mean velocity and the 1-D population dispersion
 *                    sigma_v = sqrt(sum_i sum_c (v_ic - vbar_c)^2 / (3 n)).
 *   frozen backward  gradients of (mass, centre of mass, sigma_v) with memberships held
 *                    fixed (Sec. 3.1): d com / d x_i = 1/n, mass has zero gradient,
 *                    d sigma_v / d v_ic = (v_ic - vbar_c) / (3 n sigma_v).
 *   stochastic links candidate edges closer than a cut radius, their logistic linking
 *                    probability, and K sampled graphs (Sec. 3.2 Bernoulli edges), with the
 *                    uniforms drawn from Philox4x64-10 keyed by a seed and counted by
 *                    (edge, sample) so that any implementation can reproduce them.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no -ffast-math: IEEE round-to-nearest,
 * no contraction, denormals kept).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-3)

/* ------------------------------------------------------------------------------------ */
/* Link predicate                                                                       */
/* ------------------------------------------------------------------------------------ */

/* Minimum-image separation along one axis, as defined above. */
static double minimg(double d, double L)
{
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

double oracle_dist2(const float *xi, const float *xj, const double *L)
{
    double dx = minimg((double)xi[0] - (double)xj[0], L[0]);
    double dy = minimg((double)xi[1] - (double)xj[1], L[1]);
    double dz = minimg((double)xi[2] - (double)xj[2], L[2]);
    double sx = dx * dx;
    double sy = dy * dy;
    double sz = dz * dz;
    double s = sx + sy;
    s = s + sz;
    return s;
}

int oracle_linked(const float *xi, const float *xj, const double *L, double b)
{
    double b2 = b * b;
    return oracle_dist2(xi, xj, L) < b2;
}

/* ------------------------------------------------------------------------------------ */
/* Union-find: attach the larger root under the smaller; find with path halving.         */
/* ------------------------------------------------------------------------------------ */

static int32_t uf_find(int32_t *parent, int32_t i)
{
    while (parent[i] != i) {
        parent[i] = parent[parent[i]];
        i = parent[i];
    }
    return i;
}

static void uf_union(int32_t *parent, int32_t i, int32_t j)
{
    int32_t ri = uf_find(parent, i);
    int32_t rj = uf_find(parent, j);
    if (ri == rj)
        return;
    if (ri < rj)
        parent[rj] = ri;
    else
        parent[ri] = rj;
}

/* ------------------------------------------------------------------------------------ */
/* Sparse cell list                                                                      */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    uint64_t key;
    int64_t idx;
} keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

typedef struct {
    int64_t n;
    int64_t nc[3];     /* cells per axis */
    keyed *rec;        /* n records sorted by (key, idx) */
    uint64_t *ukey;    /* unique keys */
    int64_t *ustart;   /* start of each unique key in rec, plus n at the end */
    int64_t nu;        /* number of non-empty cells */
} cell_list;

static void cells_free(cell_list *c)
{
    free(c->rec);
    free(c->ukey);
    free(c->ustart);
    memset(c, 0, sizeof(*c));
}

/* Cell side strictly larger than the search radius r: nc = max(1, floor((L/r)(1 - 2^-20))). */
static int cells_build(cell_list *c, int64_t n, const float *pos, const double *L, double r)
{
    memset(c, 0, sizeof(*c));
    c->n = n;
    for (int a = 0; a < 3; ++a) {
        double q = floor((L[a] / r) * (1.0 - ldexp(1.0, -20)));
        c->nc[a] = q < 1.0 ? 1 : (int64_t)q;
    }
    c->rec = (keyed *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed));
    c->ukey = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    c->ustart = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!c->rec || !c->ukey || !c->ustart) {
        cells_free(c);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t ix[3];
        for (int a = 0; a < 3; ++a) {
            double t = floor(((double)pos[3 * i + a] * (double)c->nc[a]) / L[a]);
            int64_t k = (int64_t)t;
            if (k > c->nc[a] - 1)
                k = c->nc[a] - 1;
            if (k < 0)
                k = 0;
            ix[a] = k;
        }
        c->rec[i].key = (uint64_t)((ix[2] * c->nc[1] + ix[1]) * c->nc[0] + ix[0]);
        c->rec[i].idx = i;
    }
    qsort(c->rec, (size_t)n, sizeof(keyed), cmp_keyed);
    int64_t nu = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || c->rec[i].key != c->rec[i - 1].key) {
            c->ukey[nu] = c->rec[i].key;
            c->ustart[nu] = i;
            ++nu;
        }
    }
    c->ustart[nu] = n;
    c->nu = nu;
    return ORC_OK;
}

/* Index of key k among the unique keys, or -1 (binary search). */
static int64_t cells_find(const cell_list *c, uint64_t k)
{
    int64_t lo = 0, hi = c->nu;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (c->ukey[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < c->nu && c->ukey[lo] == k) ? lo : -1;
}

/* The distinct neighbour keys (own cell included) of the cell with key k; returns count. */
static int cells_neighbours(const cell_list *c, uint64_t k, uint64_t out[27])
{
    int64_t ix = (int64_t)(k % (uint64_t)c->nc[0]);
    int64_t iy = (int64_t)((k / (uint64_t)c->nc[0]) % (uint64_t)c->nc[1]);
    int64_t iz = (int64_t)(k / ((uint64_t)c->nc[0] * (uint64_t)c->nc[1]));
    int m = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int64_t jx = ((ix + dx) % c->nc[0] + c->nc[0]) % c->nc[0];
                int64_t jy = ((iy + dy) % c->nc[1] + c->nc[1]) % c->nc[1];
                int64_t jz = ((iz + dz) % c->nc[2] + c->nc[2]) % c->nc[2];
                uint64_t kk = (uint64_t)((jz * c->nc[1] + jy) * c->nc[0] + jx);
                int dup = 0;
                for (int q = 0; q < m; ++q)
                    if (out[q] == kk)
                        dup = 1;
                if (!dup)
                    out[m++] = kk;
            }
    return m;
}

/* Visit every unordered pair {i, j} whose cells are neighbours, exactly once. */
typedef void (*pair_fn)(void *ctx, int64_t i, int64_t j);

static void cells_pairs(const cell_list *c, pair_fn fn, void *ctx)
{
    uint64_t nb[27];
    for (int64_t u = 0; u < c->nu; ++u) {
        int m = cells_neighbours(c, c->ukey[u], nb);
        for (int q = 0; q < m; ++q) {
            if (nb[q] < c->ukey[u])
                continue;
            int64_t v = cells_find(c, nb[q]);
            if (v < 0)
                continue;
            for (int64_t a = c->ustart[u]; a < c->ustart[u + 1]; ++a) {
                int64_t b0 = (v == u) ? a + 1 : c->ustart[v];
                for (int64_t bb = b0; bb < c->ustart[v + 1]; ++bb)
                    fn(ctx, c->rec[a].idx, c->rec[bb].idx);
            }
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Friends-of-Friends labels                                                              */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    const float *pos;
    const double *L;
    double b2;
    int32_t *parent;
    int64_t nlinks;
} link_ctx;

static void link_pair(void *vctx, int64_t i, int64_t j)
{
    link_ctx *x = (link_ctx *)vctx;
    if (oracle_dist2(x->pos + 3 * i, x->pos + 3 * j, x->L) < x->b2) {
        uf_union(x->parent, (int32_t)i, (int32_t)j);
        x->nlinks++;
    }
}

static int check_args(int64_t n, const float *pos, const double *L, double b)
{
    if (n < 0 || n > INT32_MAX || (n > 0 && !pos) || !L)
        return ORC_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!(L[a] > 0.0) || !isfinite(L[a]) || !(2.0 * b < L[a]))
            return ORC_EINVAL;
    if (!(b > 0.0) || !isfinite(b))
        return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double v = (double)pos[3 * i + a];
            if (!(v >= 0.0 && v < L[a]))
                return ORC_EINVAL;
        }
    return ORC_OK;
}

/* root[i] = smallest index in the component of i.  Returns the number of links found
 * (>= 0) or a negative error code. */
int64_t oracle_fof(int64_t n, const float *pos, const double *L, double b, int32_t *root)
{
    int rc = check_args(n, pos, L, b);
    if (rc)
        return rc;
    cell_list c;
    rc = cells_build(&c, n, pos, L, b);
    if (rc)
        return rc;
    for (int64_t i = 0; i < n; ++i)
        root[i] = (int32_t)i;
    link_ctx ctx = {pos, L, b * b, root, 0};
    cells_pairs(&c, link_pair, &ctx);
    for (int64_t i = 0; i < n; ++i)
        root[i] = uf_find(root, (int32_t)i);
    cells_free(&c);
    return ctx.nlinks;
}

/* ------------------------------------------------------------------------------------ */
/* Multi-threaded labels (OpenMP): the same definition, for full-size checks and the CPU   */
/* baseline.  Three steps, each a parallel form of the serial one above:                 */
/*   1. the cell list: records are dealt into one bucket per z-layer of cells (the key's  */
/*      slowest axis, so bucket order is key order) and each bucket is sorted on its own; */
/*      the result is the serial (key, index) order exactly;                              */
/*   2. the pair enumeration of the serial oracle, over cells in parallel;                */
/*   3. each friend pair is merged into one shared union-find whose roots only ever move  */
/*      to a smaller index (a root is re-pointed by compare-and-swap, and only while it is */
/*      still a root), so every tree's root is its smallest member whatever the order of  */
/*      the merges, and root[i] equals the serial result.                                  */
/* ------------------------------------------------------------------------------------ */

static int32_t ufa_find(int32_t *parent, int32_t i)
{
    for (;;) {
        int32_t p = __atomic_load_n(parent + i, __ATOMIC_RELAXED);
        if (p == i)
            return i;
        int32_t g = __atomic_load_n(parent + p, __ATOMIC_RELAXED);
        if (g == p)
            return p;
        /* i is not a root and never becomes one again: pointing it at an ancestor is safe */
        __atomic_store_n(parent + i, g, __ATOMIC_RELAXED);
        i = g;
    }
}

/* Root lookup without writes, for the final pass: there every thread stores the root into
   its own entry, and a halving store by another thread could replace that root with a stale
   grandparent, leaving a label that is not the component's smallest index. */
static int32_t ufa_find_ro(const int32_t *parent, int32_t i)
{
    for (;;) {
        int32_t p = __atomic_load_n(parent + i, __ATOMIC_RELAXED);
        if (p == i)
            return i;
        i = p;
    }
}

static void ufa_union(int32_t *parent, int32_t i, int32_t j)
{
    for (;;) {
        int32_t ri = ufa_find(parent, i);
        int32_t rj = ufa_find(parent, j);
        if (ri == rj)
            return;
        if (ri > rj) {
            int32_t t = ri;
            ri = rj;
            rj = t;
        }
        int32_t expect = rj;  /* the larger root goes under the smaller, if still a root */
        if (__atomic_compare_exchange_n(parent + rj, &expect, ri, 0, __ATOMIC_RELAXED,
                                        __ATOMIC_RELAXED))
            return;
        i = ri;
        j = rj;
    }
}

static int cells_build_par(cell_list *c, int64_t n, const float *pos, const double *L, double r)
{
    memset(c, 0, sizeof(*c));
    c->n = n;
    for (int a = 0; a < 3; ++a) {
        double q = floor((L[a] / r) * (1.0 - ldexp(1.0, -20)));
        c->nc[a] = q < 1.0 ? 1 : (int64_t)q;
    }
    const int64_t nb = c->nc[2];
    keyed *tmp = (keyed *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed));
    int64_t *bstart = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
    c->rec = (keyed *)malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed));
    c->ukey = (uint64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint64_t));
    c->ustart = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!tmp || !bstart || !c->rec || !c->ukey || !c->ustart) {
        free(tmp);
        free(bstart);
        cells_free(c);
        return ORC_ENOMEM;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t ix[3];
        for (int a = 0; a < 3; ++a) {
            double t = floor(((double)pos[3 * i + a] * (double)c->nc[a]) / L[a]);
            int64_t k = (int64_t)t;
            if (k > c->nc[a] - 1)
                k = c->nc[a] - 1;
            if (k < 0)
                k = 0;
            ix[a] = k;
        }
        tmp[i].key = (uint64_t)((ix[2] * c->nc[1] + ix[1]) * c->nc[0] + ix[0]);
        tmp[i].idx = i;
    }
    /* one bucket per z-layer; records keep index order inside a bucket */
    const uint64_t layer = (uint64_t)(c->nc[0] * c->nc[1]);
    for (int64_t i = 0; i < n; ++i)
        bstart[tmp[i].key / layer + 1]++;
    for (int64_t z = 0; z < nb; ++z)
        bstart[z + 1] += bstart[z];
    int64_t *cur = (int64_t *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(int64_t));
    if (!cur) {
        free(tmp);
        free(bstart);
        cells_free(c);
        return ORC_ENOMEM;
    }
    memcpy(cur, bstart, (size_t)nb * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        c->rec[cur[tmp[i].key / layer]++] = tmp[i];
    free(cur);
    free(tmp);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t z = 0; z < nb; ++z)
        qsort(c->rec + bstart[z], (size_t)(bstart[z + 1] - bstart[z]), sizeof(keyed), cmp_keyed);
    free(bstart);
    int64_t nu = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || c->rec[i].key != c->rec[i - 1].key) {
            c->ukey[nu] = c->rec[i].key;
            c->ustart[nu] = i;
            ++nu;
        }
    }
    c->ustart[nu] = n;
    c->nu = nu;
    return ORC_OK;
}

/* root[i] = smallest index in the component of i, with `threads` OpenMP threads (0: the
 * runtime's default).  Same result as oracle_fof; returns the number of links or a negative
 * error code. */
int64_t oracle_fof_par(int64_t n, const float *pos, const double *L, double b, int32_t *root,
                       int threads)
{
    int rc = check_args(n, pos, L, b);
    if (rc)
        return rc;
    if (threads > 0)
        omp_set_num_threads(threads);
    cell_list c;
    rc = cells_build_par(&c, n, pos, L, b);
    if (rc)
        return rc;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        root[i] = (int32_t)i;
    const double b2 = b * b;
    int64_t nlinks = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nlinks)
    for (int64_t u = 0; u < c.nu; ++u) {
        uint64_t nb[27];
        int m = cells_neighbours(&c, c.ukey[u], nb);
        for (int q = 0; q < m; ++q) {
            if (nb[q] < c.ukey[u])
                continue;
            int64_t v = cells_find(&c, nb[q]);
            if (v < 0)
                continue;
            for (int64_t a = c.ustart[u]; a < c.ustart[u + 1]; ++a) {
                const int64_t i = c.rec[a].idx;
                int64_t b0 = (v == u) ? a + 1 : c.ustart[v];
                for (int64_t bb = b0; bb < c.ustart[v + 1]; ++bb) {
                    const int64_t j = c.rec[bb].idx;
                    if (oracle_dist2(pos + 3 * i, pos + 3 * j, L) < b2) {
                        ufa_union(root, (int32_t)i, (int32_t)j);
                        nlinks++;
                    }
                }
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        __atomic_store_n(root + i, ufa_find_ro(root, (int32_t)i), __ATOMIC_RELAXED);
    cells_free(&c);
    return nlinks;
}

/* Threads the OpenMP runtime uses by default (what oracle_fof_par(..., 0) runs with). */
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------------------ */
/* Component of one particle (breadth-first search through the cell list), for sampled   */
/* checks at sizes where the full oracle is too slow to run inside a test.               */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    cell_list c;
    const float *pos;
    double L[3];
    double b;
    /* reverse map: position of particle i in rec */
    int64_t *where;
    int64_t *cellof;  /* unique-cell index of particle i */
} oracle_index;

void *oracle_index_build(int64_t n, const float *pos, const double *L, double b)
{
    if (check_args(n, pos, L, b))
        return NULL;
    oracle_index *ix = (oracle_index *)calloc(1, sizeof(oracle_index));
    if (!ix)
        return NULL;
    if (cells_build(&ix->c, n, pos, L, b)) {
        free(ix);
        return NULL;
    }
    ix->pos = pos;
    memcpy(ix->L, L, sizeof(ix->L));
    ix->b = b;
    ix->cellof = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!ix->cellof) {
        cells_free(&ix->c);
        free(ix);
        return NULL;
    }
    for (int64_t u = 0; u < ix->c.nu; ++u)
        for (int64_t a = ix->c.ustart[u]; a < ix->c.ustart[u + 1]; ++a)
            ix->cellof[ix->c.rec[a].idx] = u;
    return ix;
}

void oracle_index_free(void *p)
{
    oracle_index *ix = (oracle_index *)p;
    if (!ix)
        return;
    cells_free(&ix->c);
    free(ix->cellof);
    free(ix);
}

/* Writes the members of the component of particle `seed` (unsorted) into out[cap] and
 * returns their number; if the component is larger than cap, returns -(size).  `mark` is a
 * caller-owned byte array of n zeros; it is restored to zeros before returning. */
int64_t oracle_component(void *p, int64_t seed, int64_t *out, int64_t cap, uint8_t *mark)
{
    oracle_index *ix = (oracle_index *)p;
    const cell_list *c = &ix->c;
    double b2 = ix->b * ix->b;
    int64_t qcap = 1024, qn = 0, head = 0;
    int64_t *queue = (int64_t *)malloc((size_t)qcap * sizeof(int64_t));
    if (!queue)
        return 0;
    queue[qn++] = seed;
    mark[seed] = 1;
    uint64_t nb[27];
    while (head < qn) {
        int64_t i = queue[head++];
        int64_t u = ix->cellof[i];
        int m = cells_neighbours(c, c->ukey[u], nb);
        for (int q = 0; q < m; ++q) {
            int64_t v = cells_find(c, nb[q]);
            if (v < 0)
                continue;
            for (int64_t a = c->ustart[v]; a < c->ustart[v + 1]; ++a) {
                int64_t j = c->rec[a].idx;
                if (mark[j])
                    continue;
                if (oracle_dist2(ix->pos + 3 * i, ix->pos + 3 * j, ix->L) < b2) {
                    if (qn == qcap) {
                        qcap *= 2;
                        int64_t *nq = (int64_t *)realloc(queue, (size_t)qcap * sizeof(int64_t));
                        if (!nq) {
                            free(queue);
                            return 0;
                        }
                        queue = nq;
                    }
                    mark[j] = 1;
                    queue[qn++] = j;
                }
            }
        }
    }
    int64_t ret = qn <= cap ? qn : -qn;
    for (int64_t k = 0; k < qn; ++k) {
        if (k < cap)
            out[k] = queue[k];
        mark[queue[k]] = 0;
    }
    free(queue);
    return ret;
}

/* ------------------------------------------------------------------------------------ */
/* Groups: sizes, cut, compaction in ascending label order, centre of mass, velocities.  */
/* ------------------------------------------------------------------------------------ */

/* root[i] must be a canonical labelling (root[root[i]] == root[i]).  Outputs:
 *   group_id[i] = rank of root[i] among kept labels, or -1 when the component is cut;
 *   sizes/com/vmean/sigv for the first min(G, cap) groups; *n_groups = G.
 * vel, vmean and sigv may be NULL.  Returns ORC_EOVERFLOW when G > cap. */
int oracle_groups(int64_t n, const float *pos, const float *vel, const double *L,
                  const int32_t *root, int32_t min_size, int32_t cap, int32_t *group_id,
                  int32_t *n_groups, int32_t *sizes, double *com, double *vmean,
                  double *sigv)
{
    if (n < 0 || !L || (n > 0 && (!pos || !root || !group_id)) || !n_groups || cap < 0)
        return ORC_EINVAL;
    int64_t *count = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int32_t *rank = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!count || !rank) {
        free(count);
        free(rank);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i)
        count[root[i]]++;
    int32_t G = 0;
    for (int64_t r = 0; r < n; ++r) {
        rank[r] = -1;
        if (count[r] > 0 && count[r] >= min_size)
            rank[r] = G++;
    }
    for (int64_t i = 0; i < n; ++i)
        group_id[i] = rank[root[i]];
    *n_groups = G;
    /* per-group sums in ascending member index */
    double *acc = (double *)calloc((size_t)(G > 0 ? G : 1) * 3, sizeof(double));
    double *vacc = (double *)calloc((size_t)(G > 0 ? G : 1) * 3, sizeof(double));
    double *sacc = (double *)calloc((size_t)(G > 0 ? G : 1), sizeof(double));
    int32_t *groot = (int32_t *)malloc((size_t)(G > 0 ? G : 1) * sizeof(int32_t));
    if (!acc || !vacc || !sacc || !groot) {
        free(count);
        free(rank);
        free(acc);
        free(vacc);
        free(sacc);
        free(groot);
        return ORC_ENOMEM;
    }
    for (int64_t r = 0; r < n; ++r)
        if (rank[r] >= 0)
            groot[rank[r]] = (int32_t)r;
    for (int64_t i = 0; i < n; ++i) {
        int32_t g = group_id[i];
        if (g < 0)
            continue;
        int32_t r = groot[g];
        for (int a = 0; a < 3; ++a) {
            acc[3 * g + a] += minimg((double)pos[3 * i + a] - (double)pos[3 * r + a], L[a]);
            if (vel)
                vacc[3 * g + a] += (double)vel[3 * i + a];
        }
    }
    if (vel) {
        for (int64_t i = 0; i < n; ++i) {
            int32_t g = group_id[i];
            if (g < 0)
                continue;
            double nn = (double)count[groot[g]];
            for (int a = 0; a < 3; ++a) {
                double dv = (double)vel[3 * i + a] - vacc[3 * g + a] / nn;
                sacc[g] += dv * dv;
            }
        }
    }
    for (int32_t g = 0; g < G && g < cap; ++g) {
        int32_t r = groot[g];
        double nn = (double)count[r];
        if (sizes)
            sizes[g] = (int32_t)count[r];
        if (com)
            for (int a = 0; a < 3; ++a) {
                double v = (double)pos[3 * r + a] + acc[3 * g + a] / nn;
                if (v >= L[a])
                    v -= L[a];
                if (v < 0.0)
                    v += L[a];
                com[3 * g + a] = v;
            }
        if (vel && vmean)
            for (int a = 0; a < 3; ++a)
                vmean[3 * g + a] = vacc[3 * g + a] / nn;
        if (vel && sigv)
            sigv[g] = sqrt(sacc[g] / (3.0 * nn));
    }
    free(count);
    free(rank);
    free(acc);
    free(vacc);
    free(sacc);
    free(groot);
    return G > cap ? ORC_EOVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Frozen-assignment backward (Sec. 3.1)                                                  */
/* ------------------------------------------------------------------------------------ */

/* Given memberships group_id[n] (-1 = cut), the forward outputs sizes[G], vmean[G][3],
 * sigv[G], and upstream gradients g_mass[G], g_com[G][3], g_sigv[G] (any may be NULL =
 * zero), writes grad_pos[n][3] and grad_vel[n][3] (either may be NULL). */
int oracle_frozen_backward(int64_t n, const float *vel, const int32_t *group_id, int32_t G,
                           const int32_t *sizes, const double *vmean, const double *sigv,
                           const double *g_mass, const double *g_com, const double *g_sigv,
                           double *grad_pos, double *grad_vel)
{
    (void)g_mass; /* group mass n_g * m_p has no gradient with memberships frozen */
    if (n < 0 || (n > 0 && !group_id))
        return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        int32_t g = group_id[i];
        for (int a = 0; a < 3; ++a) {
            double gp = 0.0, gv = 0.0;
            if (g >= 0 && g < G) {
                double nn = (double)sizes[g];
                if (g_com)
                    gp = g_com[3 * g + a] / nn;
                if (g_sigv && vel && sigv[g] > 0.0)
                    gv = g_sigv[g] * ((double)vel[3 * i + a] - vmean[3 * g + a]) /
                         (3.0 * nn * sigv[g]);
            }
            if (grad_pos)
                grad_pos[3 * i + a] = gp;
            if (grad_vel)
                grad_vel[3 * i + a] = gv;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Topological mode (Sec. 3.2): stochastic linking sampled with a counter-based RNG       */
/* ------------------------------------------------------------------------------------ */

/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
 *   (hi0, lo0) = M0 * x0,  (hi1, lo1) = M1 * x2   (full 128-bit products)
 *   x = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
 * with the key advanced by the Weyl constants (W0, W1) between rounds. */
void oracle_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Uniform in [0, 1) for edge {i, j} (original indices, i < j) in sample s:
 * counter = (i | j << 32, s, 0, 0), key = (seed, 0); u = (first word >> 11) * 2^-53. */
double oracle_uniform(uint64_t seed, uint32_t s, uint32_t i, uint32_t j)
{
    uint64_t ctr[4] = {(uint64_t)i | ((uint64_t)j << 32), (uint64_t)s, 0, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    oracle_philox4x64(ctr, key, out);
    return (double)(out[0] >> 11) * ldexp(1.0, -53);
}

typedef struct {
    const float *pos;
    const double *L;
    double r2;
    int64_t cap, count;
    int32_t *ei, *ej;
    double *d2;
} edge_ctx;

static void edge_pair(void *vctx, int64_t i, int64_t j)
{
    edge_ctx *x = (edge_ctx *)vctx;
    double s = oracle_dist2(x->pos + 3 * i, x->pos + 3 * j, x->L);
    if (s < x->r2) {
        if (x->count < x->cap) {
            x->ei[x->count] = (int32_t)(i < j ? i : j);
            x->ej[x->count] = (int32_t)(i < j ? j : i);
            x->d2[x->count] = s;
        }
        x->count++;
    }
}

typedef struct {
    int32_t i, j;
    double d2;
} edge_rec;

static int cmp_edge(const void *a, const void *b)
{
    const edge_rec *x = (const edge_rec *)a, *y = (const edge_rec *)b;
    if (x->i != y->i)
        return x->i < y->i ? -1 : 1;
    return x->j < y->j ? -1 : (x->j > y->j);
}

/* Candidate edges: every unordered pair closer than r (same minimum-image squared distance
 * as the link predicate, compared s < r*r), listed as (i < j) in ascending (i, j) order with
 * the squared distance.  Returns the total count (which may exceed cap: then only the
 * first cap edges of the enumeration are stored and the order is not sorted). */
int64_t oracle_candidate_edges(int64_t n, const float *pos, const double *L, double r,
                               int64_t cap, int32_t *ei, int32_t *ej, double *d2)
{
    int rc = check_args(n, pos, L, r);
    if (rc)
        return rc;
    cell_list c;
    rc = cells_build(&c, n, pos, L, r);
    if (rc)
        return rc;
    edge_ctx ctx = {pos, L, r * r, cap, 0, ei, ej, d2};
    cells_pairs(&c, edge_pair, &ctx);
    cells_free(&c);
    if (ctx.count <= cap && ctx.count > 1) {
        edge_rec *e = (edge_rec *)malloc((size_t)ctx.count * sizeof(edge_rec));
        if (!e)
            return ORC_ENOMEM;
        for (int64_t k = 0; k < ctx.count; ++k) {
            e[k].i = ei[k];
            e[k].j = ej[k];
            e[k].d2 = d2[k];
        }
        qsort(e, (size_t)ctx.count, sizeof(edge_rec), cmp_edge);
        for (int64_t k = 0; k < ctx.count; ++k) {
            ei[k] = e[k].i;
            ej[k] = e[k].j;
            d2[k] = e[k].d2;
        }
        free(e);
    }
    return ctx.count;
}

/* Linking probability of an edge (Sec. 3.2 Bernoulli edges), logistic in
 * z = (b - d) / tau with d = sqrt(d2): p = 1 / (1 + exp(-z)). */
double oracle_edge_prob(double d2, double b, double tau)
{
    double z = (b - sqrt(d2)) / tau;
    return 1.0 / (1.0 + exp(-z));
}

/* K sampled graphs: y_{e,s} = [u(seed, s, i_e, j_e) < p_e]; root[s][i] = smallest index in
 * the component of i among the kept edges of sample s.  keep (optional, [K][ne] bytes)
 * receives the sampled edge indicators. */
int oracle_sample_labels(int64_t n, int64_t ne, const int32_t *ei, const int32_t *ej,
                         const double *p, uint64_t seed, int32_t K, int32_t *root,
                         uint8_t *keep)
{
    if (n < 0 || ne < 0 || K < 0)
        return ORC_EINVAL;
    for (int32_t s = 0; s < K; ++s) {
        int32_t *par = root + (int64_t)s * n;
        for (int64_t i = 0; i < n; ++i)
            par[i] = (int32_t)i;
        for (int64_t e = 0; e < ne; ++e) {
            double u = oracle_uniform(seed, (uint32_t)s, (uint32_t)ei[e], (uint32_t)ej[e]);
            int y = u < p[e];
            if (keep)
                keep[(int64_t)s * ne + e] = (uint8_t)y;
            if (y)
                uf_union(par, ei[e], ej[e]);
        }
        for (int64_t i = 0; i < n; ++i)
            par[i] = uf_find(par, (int32_t)i);
    }
    return ORC_OK;
}
