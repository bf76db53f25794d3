/*
 * rtree_oracle.c -- plain, slow, scalar CPU oracle for R-tree range select and
 * R-tree spatial join.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  The GPU library
 * never links, includes or calls it, and this file shares no source, header,
 * table or helper with the GPU library.
 *
 * What it computes (all comparisons are IEEE fp32, which are exact):
 *
 *   overlap(r, s) = r.lx <= s.hx && s.lx <= r.hx && r.ly <= s.hy && s.ly <= r.hy
 *
 *   The range-select predicate compares the query's high x, high y, low x and
 *   low y with an entry's low x, low y, high x and high y (section 3, scalar
 *   select).  The join predicate uses the same four comparisons between an
 *   outer and an inner entry (section 4.1, step 3); the paper prints those
 *   four inequalities with reversed signs, and the qualifying (intersecting)
 *   form above is the only reading under which its outer-slicing and
 *   inner-shrinking pruning rules are sound.  Boundaries are closed:
 *   rectangles that touch intersect (the paper does not say; closed is the
 *   reading adopted).
 *
 *   select(q) = ascending { i : overlap(rect[i], q) }
 *   join(A,B) = lexicographic { (a,b) : overlap(A[a], B[b]) }
 *
 * How (so a reader can check each step against the paper):
 *   - Tree: an in-memory 2D R-tree whose node holds up to F entries
 *     (MBR, ptr) plus its depth and entry count (section 2.3).  Construction
 *     is not given by the paper; this oracle bulk-loads with Sort-Tile-
 *     Recursive (Leutenegger, Lopez, Edgington 1997): sort by x-center, cut
 *     into ceil(sqrt(P)) vertical slices of S*F entries, sort each slice by
 *     y-center, pack runs of F, repeat on the node MBRs until one node is left.
 *     Center keys are summed in double; ties are broken by entry id.
 *   - Select: the paper's best scalar variant, a recursive depth-first
 *     traversal from the root using the logical-and predicate (section 3 and
 *     the scalar results of section 5.1), then each query's ids are sorted.
 *   - Join: the R-tree join of Brinkhoff, Kriegel and Seeger that the paper
 *     uses as its scalar join (section 4): traverse both trees from the roots
 *     and follow every intersecting child pair.  When one side reaches its
 *     leaves first, that leaf entry stays fixed and only the other side
 *     descends.  Pairs are sorted at the end.
 *   - Join with sorted nodes (section 4.1 pruning rules and the many-to-many
 *     approach of section 4.2): every node's entries in ascending low-x
 *     order; O3 stops the outer scan at the first outer child whose low x
 *     exceeds every inner high x; O4 stops the inner scan of one outer child
 *     at the first inner child whose low x exceeds the outer high x; O5 finds
 *     the same stop for a batch of 16 outer children by the gather / compare /
 *     update rounds of the many-to-many approach.  Same pairs as the join.
 *   - Brute force: nested loops over the plain definitions above.
 *   - Threaded drivers (ora_select_mt, ora_join_mt): the same search and
 *     join run on several host threads over a static partition of the
 *     queries (or of the intersecting root-entry pairs), for the all-cores
 *     timing baseline; the results are those of the single-thread calls.
 *   - Tree invariants: every parent entry MBR equals the exact union of its
 *     child's entries, every object appears in exactly one leaf entry with its
 *     own rectangle, levels decrease by one per edge down to 0 at every leaf,
 *     and 1 <= count <= F (the root may be empty only for an empty tree).
 *
 * Mutants: building with -DORA_MUTANT=k plants one deliberate mistake (used
 * only by the test that shows the pins catch such mistakes).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef ORA_MUTANT
#define ORA_MUTANT 0
#endif

typedef struct {
    uint32_t fanout;
    uint32_t height;      /* levels including the leaf level; 0 for no tree */
    uint32_t n_nodes;
    uint32_t root;
    uint64_t n_objects;
    uint64_t n_entries;
    uint32_t *level;      /* per node, 0 = leaf */
    uint32_t *count;      /* per node, number of entries */
    uint64_t *first;      /* per node, index of its first entry */
    float *lx, *ly, *hx, *hy;   /* per entry */
    uint32_t *ptr;        /* per entry: object id (leaf) or child node index */
} ora_tree;

/* ------------------------------------------------------------------------ */
/* predicate                                                                 */
/* ------------------------------------------------------------------------ */

static int overlap4(float alx, float aly, float ahx, float ahy,
                    float blx, float bly, float bhx, float bhy)
{
#if ORA_MUTANT == 1          /* open boundaries */
    return alx < bhx && blx < ahx && aly < bhy && bly < ahy;
#elif ORA_MUTANT == 2        /* x and y transposed in one term */
    return alx <= bhy && blx <= ahx && aly <= bhy && bly <= ahy;
#elif ORA_MUTANT == 3        /* one term dropped */
    return alx <= bhx && blx <= ahx && bly <= ahy;
#else
    return alx <= bhx && blx <= ahx && aly <= bhy && bly <= ahy;
#endif
}

/* ------------------------------------------------------------------------ */
/* small growable buffers                                                   */
/* ------------------------------------------------------------------------ */

typedef struct { uint32_t *v; size_t n, cap; } vec32;
typedef struct { uint64_t *v; size_t n, cap; } vec64;

static int v32_push(vec32 *b, uint32_t x)
{
    if (b->n == b->cap) {
        size_t nc = b->cap ? b->cap * 2 : 1024;
        uint32_t *p = (uint32_t *)realloc(b->v, nc * sizeof(uint32_t));
        if (!p) return -1;
        b->v = p; b->cap = nc;
    }
    b->v[b->n++] = x;
    return 0;
}

static int v64_push(vec64 *b, uint64_t x)
{
    if (b->n == b->cap) {
        size_t nc = b->cap ? b->cap * 2 : 1024;
        uint64_t *p = (uint64_t *)realloc(b->v, nc * sizeof(uint64_t));
        if (!p) return -1;
        b->v = p; b->cap = nc;
    }
    b->v[b->n++] = x;
    return 0;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

void ora_free_buf(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* STR bulk load                                                             */
/* ------------------------------------------------------------------------ */

typedef struct { double key; uint32_t id; uint32_t pos; } keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* smallest s with s*s >= p */
static uint64_t ceil_sqrt(uint64_t p)
{
    uint64_t s = (uint64_t)sqrt((double)p);
    while (s * s < p) s++;
    while (s > 0 && (s - 1) * (s - 1) >= p) s--;
    return s;
}

void ora_free_tree(ora_tree *t)
{
    if (!t) return;
    free(t->level); free(t->count); free(t->first);
    free(t->lx); free(t->ly); free(t->hx); free(t->hy); free(t->ptr);
    memset(t, 0, sizeof(*t));
}

/* Items of the level being packed: rectangles plus the id that the parent
 * entry will point to (object id at the leaf level, node index above). */
typedef struct { float lx, ly, hx, hy; uint32_t id; } item;

int ora_build_str(const float *rects, uint64_t n, uint32_t fanout, ora_tree *t)
{
    memset(t, 0, sizeof(*t));
    if (fanout < 2 || n > 0xFFFFFFFFull) return -1;
    for (uint64_t i = 0; i < n; i++) {
        const float *r = rects + 4 * i;
        if (isnan(r[0]) || isnan(r[1]) || isnan(r[2]) || isnan(r[3])) return -1;
        if (!(r[0] <= r[2]) || !(r[1] <= r[3])) return -1;
    }
    t->fanout = fanout;
    t->n_objects = n;

    /* Upper bounds on nodes and entries: every level has at most
     * ceil(count / F) nodes. */
    uint64_t max_nodes = 1, max_entries = n, c = n;
    while (c > fanout) { c = (c + fanout - 1) / fanout; max_nodes += c; max_entries += c; }
    t->level = (uint32_t *)malloc(max_nodes * sizeof(uint32_t));
    t->count = (uint32_t *)malloc(max_nodes * sizeof(uint32_t));
    t->first = (uint64_t *)malloc(max_nodes * sizeof(uint64_t));
    size_t ne = (size_t)(max_entries ? max_entries : 1);
    t->lx = (float *)malloc(ne * sizeof(float));
    t->ly = (float *)malloc(ne * sizeof(float));
    t->hx = (float *)malloc(ne * sizeof(float));
    t->hy = (float *)malloc(ne * sizeof(float));
    t->ptr = (uint32_t *)malloc(ne * sizeof(uint32_t));
    item *cur = (item *)malloc((size_t)(n ? n : 1) * sizeof(item));
    keyed *ord = (keyed *)malloc((size_t)(n ? n : 1) * sizeof(keyed));
    if (!t->level || !t->count || !t->first || !t->lx || !t->ly || !t->hx ||
        !t->hy || !t->ptr || !cur || !ord) {
        free(cur); free(ord); ora_free_tree(t); return -2;
    }
    for (uint64_t i = 0; i < n; i++) {
        cur[i].lx = rects[4 * i + 0]; cur[i].ly = rects[4 * i + 1];
        cur[i].hx = rects[4 * i + 2]; cur[i].hy = rects[4 * i + 3];
        cur[i].id = (uint32_t)i;
    }
    uint64_t cnt = n;
    uint32_t lvl = 0;
    uint32_t nn = 0;
    uint64_t e = 0;

    while (cnt > fanout) {
        uint64_t P = (cnt + fanout - 1) / fanout;
        uint64_t S = ceil_sqrt(P);
        uint64_t slice = S * fanout;
        /* sort by x-center */
        for (uint64_t i = 0; i < cnt; i++) {
            ord[i].key = (double)cur[i].lx + (double)cur[i].hx;
            ord[i].id = cur[i].id;
            ord[i].pos = (uint32_t)i;
        }
        qsort(ord, (size_t)cnt, sizeof(keyed), cmp_keyed);
        /* within each vertical slice sort by y-center */
        for (uint64_t s0 = 0; s0 < cnt; s0 += slice) {
            uint64_t s1 = s0 + slice < cnt ? s0 + slice : cnt;
            for (uint64_t i = s0; i < s1; i++)
                ord[i].key = (double)cur[ord[i].pos].ly + (double)cur[ord[i].pos].hy;
            qsort(ord + s0, (size_t)(s1 - s0), sizeof(keyed), cmp_keyed);
        }
        /* pack runs of F inside each slice into nodes of this level */
        item *next = (item *)malloc((size_t)P * sizeof(item) + sizeof(item) * 2);
        if (!next) { free(cur); free(ord); ora_free_tree(t); return -2; }
        uint64_t np = 0;
        for (uint64_t s0 = 0; s0 < cnt; s0 += slice) {
            uint64_t s1 = s0 + slice < cnt ? s0 + slice : cnt;
#if ORA_MUTANT == 5          /* last item of every slice dropped */
            if (s1 - s0 > 1) s1--;
#endif
            for (uint64_t r0 = s0; r0 < s1; r0 += fanout) {
                uint64_t r1 = r0 + fanout < s1 ? r0 + fanout : s1;
                uint32_t node = nn++;
                t->level[node] = lvl;
                t->count[node] = (uint32_t)(r1 - r0);
                t->first[node] = e;
                float mlx = INFINITY, mly = INFINITY, mhx = -INFINITY, mhy = -INFINITY;
                for (uint64_t i = r0; i < r1; i++) {
                    const item *it = &cur[ord[i].pos];
                    t->lx[e] = it->lx; t->ly[e] = it->ly;
                    t->hx[e] = it->hx; t->hy[e] = it->hy;
                    t->ptr[e] = it->id;
                    e++;
                    if (it->lx < mlx) mlx = it->lx;
                    if (it->ly < mly) mly = it->ly;
#if ORA_MUTANT == 4          /* parent MBR loses the high-x union */
                    mhx = it->hx;
#else
                    if (it->hx > mhx) mhx = it->hx;
#endif
                    if (it->hy > mhy) mhy = it->hy;
                }
                next[np].lx = mlx; next[np].ly = mly;
                next[np].hx = mhx; next[np].hy = mhy;
                next[np].id = node;
                np++;
            }
        }
        free(cur);
        cur = next;
        cnt = np;
        lvl++;
    }
    /* root: the remaining <= F items (a single leaf when n <= F) */
    uint32_t root = nn++;
    t->level[root] = lvl;
    t->count[root] = (uint32_t)cnt;
    t->first[root] = e;
    for (uint64_t i = 0; i < cnt; i++) {
        t->lx[e] = cur[i].lx; t->ly[e] = cur[i].ly;
        t->hx[e] = cur[i].hx; t->hy[e] = cur[i].hy;
        t->ptr[e] = cur[i].id;
        e++;
    }
    free(cur);
    free(ord);
    t->root = root;
    t->n_nodes = nn;
    t->n_entries = e;
    t->height = lvl + 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* range select: recursive depth-first search, logical-and predicate         */
/* ------------------------------------------------------------------------ */

static int search(const ora_tree *t, uint32_t node, const float *q, vec32 *out)
{
    uint64_t e0 = t->first[node], e1 = e0 + t->count[node];
    for (uint64_t e = e0; e < e1; e++) {
        /* entry low x/low y/high x/high y against query high x/high y/low x/low y */
        if (overlap4(t->lx[e], t->ly[e], t->hx[e], t->hy[e], q[0], q[1], q[2], q[3])) {
            if (t->level[node] == 0) {
                if (v32_push(out, t->ptr[e])) return -2;
            } else {
                if (search(t, t->ptr[e], q, out)) return -2;
            }
        }
    }
    return 0;
}

/* offsets: caller array of nq+1; *ids_out: malloc'ed, free with ora_free_buf */
int ora_select(const ora_tree *t, const float *queries, uint64_t nq,
               uint64_t *offsets, uint32_t **ids_out, uint64_t *total)
{
    vec32 all = {0, 0, 0};
    offsets[0] = 0;
    for (uint64_t k = 0; k < nq; k++) {
        size_t start = all.n;
        if (t->n_nodes > 0 && search(t, t->root, queries + 4 * k, &all)) {
            free(all.v); return -2;
        }
#if ORA_MUTANT != 6          /* mutant 6: ids left in traversal order */
        qsort(all.v + start, all.n - start, sizeof(uint32_t), cmp_u32);
#endif
        offsets[k + 1] = all.n;
    }
    *ids_out = all.v;
    *total = all.n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* spatial join: synchronized traversal of both trees                        */
/* ------------------------------------------------------------------------ */

static int emit(vec64 *out, uint32_t a, uint32_t b)
{
    return v64_push(out, ((uint64_t)a << 32) | b);
}

/* A's leaf entry ea stays fixed; descend B from node v */
static int join_fixed_a(const ora_tree *A, uint64_t ea, const ora_tree *B, uint32_t v, vec64 *out)
{
    uint64_t f0 = B->first[v], f1 = f0 + B->count[v];
    for (uint64_t f = f0; f < f1; f++) {
        if (overlap4(A->lx[ea], A->ly[ea], A->hx[ea], A->hy[ea],
                     B->lx[f], B->ly[f], B->hx[f], B->hy[f])) {
            if (B->level[v] == 0) { if (emit(out, A->ptr[ea], B->ptr[f])) return -2; }
            else if (join_fixed_a(A, ea, B, B->ptr[f], out)) return -2;
        }
    }
    return 0;
}

/* B's leaf entry fb stays fixed; descend A from node u */
static int join_fixed_b(const ora_tree *A, uint32_t u, const ora_tree *B, uint64_t fb, vec64 *out)
{
    uint64_t e0 = A->first[u], e1 = e0 + A->count[u];
    for (uint64_t e = e0; e < e1; e++) {
        if (overlap4(A->lx[e], A->ly[e], A->hx[e], A->hy[e],
                     B->lx[fb], B->ly[fb], B->hx[fb], B->hy[fb])) {
#if ORA_MUTANT == 7          /* pair emitted with its sides swapped */
            if (A->level[u] == 0) { if (emit(out, B->ptr[fb], A->ptr[e])) return -2; }
#else
            if (A->level[u] == 0) { if (emit(out, A->ptr[e], B->ptr[fb])) return -2; }
#endif
            else if (join_fixed_b(A, A->ptr[e], B, fb, out)) return -2;
        }
    }
    return 0;
}

static int join_nodes(const ora_tree *A, uint32_t u, const ora_tree *B, uint32_t v, vec64 *out);

/* entry e of A's node u and entry f of B's node v intersect: emit the pair
 * (both leaves), descend both (both internal), or descend the internal side
 * with the leaf entry fixed */
static int join_entries(const ora_tree *A, uint32_t u, uint64_t e, const ora_tree *B, uint32_t v, uint64_t f,
                        vec64 *out)
{
    int la = A->level[u] == 0, lb = B->level[v] == 0;
    if (la && lb) return emit(out, A->ptr[e], B->ptr[f]);
    if (!la && !lb) return join_nodes(A, A->ptr[e], B, B->ptr[f], out);
    if (la) return join_fixed_a(A, e, B, B->ptr[f], out);
    return join_fixed_b(A, A->ptr[e], B, f, out);
}

static int join_nodes(const ora_tree *A, uint32_t u, const ora_tree *B, uint32_t v, vec64 *out)
{
    uint64_t e0 = A->first[u], e1 = e0 + A->count[u];
    uint64_t f0 = B->first[v], f1 = f0 + B->count[v];
    for (uint64_t e = e0; e < e1; e++) {
        for (uint64_t f = f0; f < f1; f++) {
            if (!overlap4(A->lx[e], A->ly[e], A->hx[e], A->hy[e],
                          B->lx[f], B->ly[f], B->hx[f], B->hy[f]))
                continue;
            int rc = join_entries(A, u, e, B, v, f, out);
            if (rc) return rc;
        }
    }
    return 0;
}

/* *pairs_out: malloc'ed u32 array of 2*n (a0,b0,a1,b1,...), free with ora_free_buf */
int ora_join(const ora_tree *A, const ora_tree *B, uint32_t **pairs_out, uint64_t *n_out)
{
    vec64 acc = {0, 0, 0};
    if (A->n_nodes > 0 && B->n_nodes > 0 && A->n_objects > 0 && B->n_objects > 0) {
        if (join_nodes(A, A->root, B, B->root, &acc)) { free(acc.v); return -2; }
    }
    qsort(acc.v, acc.n, sizeof(uint64_t), cmp_u64);
    uint32_t *p = (uint32_t *)malloc((acc.n ? acc.n : 1) * 2 * sizeof(uint32_t));
    if (!p) { free(acc.v); return -2; }
    for (size_t i = 0; i < acc.n; i++) {
        p[2 * i] = (uint32_t)(acc.v[i] >> 32);
        p[2 * i + 1] = (uint32_t)(acc.v[i] & 0xFFFFFFFFu);
    }
    free(acc.v);
    *pairs_out = p;
    *n_out = acc.n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the same select and join spread over host threads (a timing baseline for  */
/* all host cores; results are those of ora_select and ora_join)             */
/* ------------------------------------------------------------------------ */

typedef struct {
    const ora_tree *t;
    const float *q;
    uint64_t q0, q1;          /* this thread's queries [q0, q1) */
    uint64_t *counts;         /* ids per query, indexed like the queries */
    vec32 ids;
    int rc;
} sel_part;

static void *sel_worker(void *arg)
{
    sel_part *p = (sel_part *)arg;
    for (uint64_t k = p->q0; k < p->q1; k++) {
        size_t start = p->ids.n;
        if (p->t->n_nodes > 0 && search(p->t, p->t->root, p->q + 4 * k, &p->ids)) { p->rc = -2; return NULL; }
#if ORA_MUTANT != 6
        qsort(p->ids.v + start, p->ids.n - start, sizeof(uint32_t), cmp_u32);
#endif
        p->counts[k] = p->ids.n - start;
    }
    return NULL;
}

/* ora_select with the queries cut into nthreads contiguous parts, one thread
 * each (static partition) */
int ora_select_mt(const ora_tree *t, const float *queries, uint64_t nq, int nthreads,
                  uint64_t *offsets, uint32_t **ids_out, uint64_t *total)
{
    if (nthreads < 1) nthreads = 1;
    sel_part *parts = (sel_part *)calloc((size_t)nthreads, sizeof(sel_part));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!parts || !th) { free(parts); free(th); return -2; }
    for (int i = 0; i < nthreads; i++) {
        parts[i].t = t;
        parts[i].q = queries;
        parts[i].q0 = nq * (uint64_t)i / (uint64_t)nthreads;
        parts[i].q1 = nq * (uint64_t)(i + 1) / (uint64_t)nthreads;
        parts[i].counts = offsets + 1;
    }
    int started = 0, rc = 0;
    for (; started < nthreads; started++)
        if (pthread_create(&th[started], NULL, sel_worker, &parts[started])) { rc = -2; break; }
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    uint64_t n = 0;
    for (int i = 0; i < nthreads && !rc; i++) {
        if (parts[i].rc) rc = parts[i].rc;
        n += parts[i].ids.n;
    }
    uint32_t *all = rc ? NULL : (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    if (!rc && !all) rc = -2;
    if (!rc) {
        uint64_t at = 0;
        for (int i = 0; i < nthreads; i++) {
            if (parts[i].ids.n) memcpy(all + at, parts[i].ids.v, parts[i].ids.n * sizeof(uint32_t));
            at += parts[i].ids.n;
        }
        offsets[0] = 0;
        for (uint64_t k = 0; k < nq; k++) offsets[k + 1] += offsets[k];
        *ids_out = all;
        *total = n;
    }
    for (int i = 0; i < nthreads; i++) free(parts[i].ids.v);
    free(parts); free(th);
    return rc;
}

/* intersecting entry pairs (entry e of A's node u, entry f of B's node v) */
typedef struct { uint64_t *u, *e, *v, *f; size_t n, cap; } pairvec;

static int pv_push(pairvec *p, uint64_t u, uint64_t e, uint64_t v, uint64_t f)
{
    if (p->n == p->cap) {
        size_t nc = p->cap ? p->cap * 2 : 256;
        uint64_t *a = (uint64_t *)realloc(p->u, nc * sizeof(uint64_t));
        if (a) p->u = a;
        uint64_t *b = (uint64_t *)realloc(p->e, nc * sizeof(uint64_t));
        if (b) p->e = b;
        uint64_t *c = (uint64_t *)realloc(p->v, nc * sizeof(uint64_t));
        if (c) p->v = c;
        uint64_t *d = (uint64_t *)realloc(p->f, nc * sizeof(uint64_t));
        if (d) p->f = d;
        if (!a || !b || !c || !d) return -1;
        p->cap = nc;
    }
    p->u[p->n] = u; p->e[p->n] = e; p->v[p->n] = v; p->f[p->n] = f;
    p->n++;
    return 0;
}

static void pv_free(pairvec *p) { free(p->u); free(p->e); free(p->v); free(p->f); }

/* every intersecting entry pair of A's node u and B's node v */
static int pv_node_pairs(const ora_tree *A, uint32_t u, const ora_tree *B, uint32_t v, pairvec *out)
{
    uint64_t e0 = A->first[u], e1 = e0 + A->count[u];
    uint64_t f0 = B->first[v], f1 = f0 + B->count[v];
    for (uint64_t e = e0; e < e1; e++)
        for (uint64_t f = f0; f < f1; f++)
            if (overlap4(A->lx[e], A->ly[e], A->hx[e], A->hy[e], B->lx[f], B->ly[f], B->hx[f], B->hy[f]))
                if (pv_push(out, u, e, v, f)) return -2;
    return 0;
}

typedef struct {
    const ora_tree *A, *B;
    const pairvec *work;
    int tid, nthreads;        /* this thread takes pairs tid, tid + nthreads, ... */
    vec64 out;
    int rc;
} join_part;

static void *join_worker(void *arg)
{
    join_part *p = (join_part *)arg;
    const pairvec *w = p->work;
    for (size_t k = (size_t)p->tid; k < w->n; k += (size_t)p->nthreads)
        if (join_entries(p->A, (uint32_t)w->u[k], w->e[k], p->B, (uint32_t)w->v[k], w->f[k], &p->out)) {
            p->rc = -2;
            break;
        }
    return NULL;
}

/* ora_join on nthreads threads.  The intersecting entry pairs of the two
 * roots are expanded level by level -- a pair of internal entries is
 * replaced by the intersecting entry pairs of their two children, which is
 * what the join does next with it -- until there are at least 64 pairs per
 * thread (or only pairs with a leaf side are left); the pairs are then dealt
 * round-robin to the threads, each finishing its pairs as the join would. */
int ora_join_mt(const ora_tree *A, const ora_tree *B, int nthreads, uint32_t **pairs_out, uint64_t *n_out)
{
    if (nthreads < 1) nthreads = 1;
    vec64 acc = {0, 0, 0};
    int rc = 0;
    if (A->n_nodes > 0 && B->n_nodes > 0 && A->n_objects > 0 && B->n_objects > 0) {
        pairvec cur = {0}, nxt = {0};
        rc = pv_node_pairs(A, A->root, B, B->root, &cur);
        while (!rc && cur.n < (size_t)64 * (size_t)nthreads) {
            int grew = 0;
            nxt.n = 0;
            for (size_t k = 0; k < cur.n && !rc; k++) {
                uint32_t u = (uint32_t)cur.u[k], v = (uint32_t)cur.v[k];
                if (A->level[u] > 0 && B->level[v] > 0) {
                    rc = pv_node_pairs(A, A->ptr[cur.e[k]], B, B->ptr[cur.f[k]], &nxt);
                    grew = 1;
                } else {
                    rc = pv_push(&nxt, u, cur.e[k], v, cur.f[k]) ? -2 : 0;
                }
            }
            pairvec t = cur; cur = nxt; nxt = t;
            if (!grew) break;
        }
        pv_free(&nxt);
        join_part *parts = (join_part *)calloc((size_t)nthreads, sizeof(join_part));
        pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
        if (!parts || !th) rc = -2;
        int started = 0;
        for (; !rc && started < nthreads; started++) {
            parts[started] = (join_part){A, B, &cur, started, nthreads, {0, 0, 0}, 0};
            if (pthread_create(&th[started], NULL, join_worker, &parts[started])) { rc = -2; break; }
        }
        for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
        for (int i = 0; i < started && !rc; i++) {
            if (parts[i].rc) { rc = parts[i].rc; break; }
            for (size_t k = 0; k < parts[i].out.n; k++)
                if (v64_push(&acc, parts[i].out.v[k])) { rc = -2; break; }
        }
        for (int i = 0; i < started; i++) free(parts[i].out.v);
        free(parts); free(th);
        pv_free(&cur);
    }
    if (rc) { free(acc.v); return rc; }
    qsort(acc.v, acc.n, sizeof(uint64_t), cmp_u64);
    uint32_t *p = (uint32_t *)malloc((acc.n ? acc.n : 1) * 2 * sizeof(uint32_t));
    if (!p) { free(acc.v); return -2; }
    for (size_t i = 0; i < acc.n; i++) {
        p[2 * i] = (uint32_t)(acc.v[i] >> 32);
        p[2 * i + 1] = (uint32_t)(acc.v[i] & 0xFFFFFFFFu);
    }
    free(acc.v);
    *pairs_out = p;
    *n_out = acc.n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* join over nodes sorted by low x: outer slicing (O3) and inner shrinking   */
/* (O4 one outer child at a time, O5 a batch of outer children at once)      */
/* ------------------------------------------------------------------------ */

/* Entries of every node in ascending low-x order, ties kept in their order
 * (section 4.1 assumes nodes sorted on one MBR key; low x is the paper's
 * example).  Children are moved with their entries. */
typedef struct { float lx, ly, hx, hy; uint32_t ptr; uint32_t pos; } sent;

static int cmp_sent(const void *a, const void *b)
{
    const sent *x = (const sent *)a, *y = (const sent *)b;
    if (x->lx < y->lx) return -1;
    if (x->lx > y->lx) return 1;
    return (x->pos > y->pos) - (x->pos < y->pos);
}

int ora_sort_entries_lx(ora_tree *t)
{
    sent *buf = (sent *)malloc((size_t)(t->fanout ? t->fanout : 1) * sizeof(sent));
    if (!buf) return -2;
    for (uint32_t u = 0; u < t->n_nodes; u++) {
        uint64_t e0 = t->first[u];
        uint32_t c = t->count[u];
        if (c > t->fanout) { free(buf); return -1; }
        for (uint32_t k = 0; k < c; k++) {
            buf[k].lx = t->lx[e0 + k]; buf[k].ly = t->ly[e0 + k];
            buf[k].hx = t->hx[e0 + k]; buf[k].hy = t->hy[e0 + k];
            buf[k].ptr = t->ptr[e0 + k]; buf[k].pos = k;
        }
        qsort(buf, c, sizeof(sent), cmp_sent);
        for (uint32_t k = 0; k < c; k++) {
            t->lx[e0 + k] = buf[k].lx; t->ly[e0 + k] = buf[k].ly;
            t->hx[e0 + k] = buf[k].hx; t->hy[e0 + k] = buf[k].hy;
            t->ptr[e0 + k] = buf[k].ptr;
        }
    }
    free(buf);
    return 0;
}

static int node_sorted_lx(const ora_tree *t, uint32_t u)
{
    for (uint64_t e = t->first[u] + 1; e < t->first[u] + t->count[u]; e++)
        if (t->lx[e] < t->lx[e - 1]) return 0;
    return 1;
}

/* Many-to-many inner shrinking (section 4.2, steps 2-4; figure 6 works one
 * update through).  Each outer lane k holds a gather index gidx[k] into the
 * low-x-sorted inner children and a flip index flip[k]: the inner position
 * from which on no child can qualify for that outer child.  One update takes
 * the compare mask of out.hx >= in.lx[gidx] (bit k for lane k):
 *   bit set   -> that inner child (and all before it) may qualify: move up,
 *                gidx += step
 *   bit clear -> it and all after it cannot: flip = gidx, move down,
 *                gidx -= step
 * Lanes whose index has left the search range [0, n_pow) are not updated. */
void ora_m2m_update(uint32_t w, uint64_t mask, uint32_t step, uint32_t n_pow, uint32_t *gidx, uint32_t *flip)
{
    for (uint32_t k = 0; k < w; k++) {
        if (gidx[k] >= n_pow) continue;
        if ((mask >> k) & 1u) {
            gidx[k] += step;
        } else {
            flip[k] = gidx[k];
#if ORA_MUTANT == 8          /* clear bit moves the wrong way */
            gidx[k] += step;
#else
            gidx[k] -= step;
#endif
        }
    }
}

/* Flip indices of w outer children against n_in inner children sorted by low
 * x: flip[k] = the first j with in_lx[j] > out_hx[k], or n_in if none.  The
 * search runs over n_pow = the smallest power of two >= n_in positions
 * (positions >= n_in never qualify); it starts every lane at n_pow/2 with
 * flip = n_pow ("all qualify") and takes log2(n_pow) + 1 gather/compare/update
 * rounds, the step halving from n_pow/4 down to 1 and staying at 1 for the
 * last round.  With n_in = n_pow = F this is the paper's schedule. */
void ora_m2m_flip(uint32_t w, const float *out_hx, const float *in_lx, uint32_t n_in, uint32_t *flip)
{
    if (w > 64) w = 64;   /* at most 64 lanes */
    uint32_t n_pow = 1, lg = 0;
    while (n_pow < n_in) { n_pow <<= 1; lg++; }
    uint32_t gidx[64];
    for (uint32_t k = 0; k < w; k++) { gidx[k] = n_pow / 2; flip[k] = n_pow; }
    for (uint32_t it = 0; it <= lg; it++) {
        uint64_t mask = 0;
        for (uint32_t k = 0; k < w; k++) {
            uint32_t g = gidx[k];
            if (g < n_in && out_hx[k] >= in_lx[g]) mask |= 1ull << k;
        }
        uint32_t step = (it + 2 <= lg) ? (n_pow >> (it + 2)) : 1;
        ora_m2m_update(w, mask, step, n_pow, gidx, flip);
    }
}

#define ORA_O3 1
#define ORA_O4 2
#define ORA_O5 4
#define ORA_W 16   /* outer children per many-to-many batch: one 512-bit vector of fp32 */

static int join_nodes_opt(const ora_tree *A, uint32_t u, const ora_tree *B, uint32_t v, int flags, vec64 *out,
                          uint64_t *tests)
{
    uint64_t e0 = A->first[u], f0 = B->first[v];
    uint32_t na = A->count[u], nb = B->count[v];
    /* O3: the first outer child whose low x exceeds every inner high x ends
     * the outer scan; later outer children have a larger low x still */
    uint32_t cut = na;
    if (flags & ORA_O3) {
        for (uint32_t i = 0; i < na; i++) {
            int any = 0;
            for (uint32_t j = 0; j < nb && !any; j++)
#if ORA_MUTANT == 9          /* touching children treated as disjoint */
                any = A->lx[e0 + i] < B->hx[f0 + j];
#else
                any = A->lx[e0 + i] <= B->hx[f0 + j];
#endif
            if (!any) { cut = i; break; }
        }
    }
    /* inner limit per outer child */
    uint32_t lim[64];
    for (uint32_t i = 0; i < cut; i++) lim[i] = nb;
    if (flags & ORA_O5) {
        float ohx[ORA_W], ilx[64];
        for (uint32_t j = 0; j < nb; j++) ilx[j] = B->lx[f0 + j];
        for (uint32_t i0 = 0; i0 < cut; i0 += ORA_W) {
            uint32_t w = cut - i0 < ORA_W ? cut - i0 : ORA_W;
            for (uint32_t k = 0; k < w; k++) ohx[k] = A->hx[e0 + i0 + k];
            ora_m2m_flip(w, ohx, ilx, nb, lim + i0);
        }
    } else if (flags & ORA_O4) {
        /* O4: scan the inner children of one outer child in low-x order and
         * stop at the first one that starts right of the outer child's high x */
        for (uint32_t i = 0; i < cut; i++) {
            uint32_t j = 0;
            while (j < nb && B->lx[f0 + j] <= A->hx[e0 + i]) j++;
            lim[i] = j;
        }
    }
    for (uint32_t i = 0; i < cut; i++) {
        uint64_t e = e0 + i;
        for (uint32_t j = 0; j < lim[i]; j++) {
            uint64_t f = f0 + j;
            (*tests)++;
            if (!overlap4(A->lx[e], A->ly[e], A->hx[e], A->hy[e], B->lx[f], B->ly[f], B->hx[f], B->hy[f]))
                continue;
            int la = A->level[u] == 0, lb = B->level[v] == 0;
            int rc;
            if (la && lb) rc = emit(out, A->ptr[e], B->ptr[f]);
            else if (!la && !lb) rc = join_nodes_opt(A, A->ptr[e], B, B->ptr[f], flags, out, tests);
            else if (la) rc = join_fixed_a(A, e, B, B->ptr[f], out);
            else rc = join_fixed_b(A, A->ptr[e], B, f, out);
            if (rc) return rc;
        }
    }
    return 0;
}

/* Join with the pruning options of section 4 (flags: 1 = O3, 2 = O4, 4 = O5;
 * O5 takes precedence over O4).  Pruning needs every node sorted by low x
 * (returns -1 otherwise).  *tests_out: pair predicates evaluated in node-pair
 * expansions (the leaf-entry-fixed descent of trees of unequal height is not
 * pruned and not counted).  Same output format as ora_join. */
int ora_join_opt(const ora_tree *A, const ora_tree *B, int flags, uint32_t **pairs_out, uint64_t *n_out,
                 uint64_t *tests_out)
{
    if (A->fanout > 64 || B->fanout > 64) return -1;
    if (flags & (ORA_O3 | ORA_O4 | ORA_O5)) {
        for (uint32_t u = 0; u < A->n_nodes; u++) if (!node_sorted_lx(A, u)) return -1;
        for (uint32_t v = 0; v < B->n_nodes; v++) if (!node_sorted_lx(B, v)) return -1;
    }
    vec64 acc = {0, 0, 0};
    uint64_t tests = 0;
    if (A->n_nodes > 0 && B->n_nodes > 0 && A->n_objects > 0 && B->n_objects > 0) {
        if (join_nodes_opt(A, A->root, B, B->root, flags, &acc, &tests)) { free(acc.v); return -2; }
    }
    qsort(acc.v, acc.n, sizeof(uint64_t), cmp_u64);
    uint32_t *p = (uint32_t *)malloc((acc.n ? acc.n : 1) * 2 * sizeof(uint32_t));
    if (!p) { free(acc.v); return -2; }
    for (size_t i = 0; i < acc.n; i++) {
        p[2 * i] = (uint32_t)(acc.v[i] >> 32);
        p[2 * i + 1] = (uint32_t)(acc.v[i] & 0xFFFFFFFFu);
    }
    free(acc.v);
    *pairs_out = p;
    *n_out = acc.n;
    *tests_out = tests;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* brute force                                                               */
/* ------------------------------------------------------------------------ */

int ora_brute_select(const float *rects, uint64_t n, const float *queries, uint64_t nq,
                     uint64_t *offsets, uint32_t **ids_out, uint64_t *total)
{
    vec32 all = {0, 0, 0};
    offsets[0] = 0;
    for (uint64_t k = 0; k < nq; k++) {
        const float *q = queries + 4 * k;
        for (uint64_t i = 0; i < n; i++) {
            const float *r = rects + 4 * i;
            if (overlap4(r[0], r[1], r[2], r[3], q[0], q[1], q[2], q[3]))
                if (v32_push(&all, (uint32_t)i)) { free(all.v); return -2; }
        }
        offsets[k + 1] = all.n;
    }
    *ids_out = all.v;
    *total = all.n;
    return 0;
}

int ora_brute_join(const float *A, uint64_t na, const float *B, uint64_t nb,
                   uint32_t **pairs_out, uint64_t *n_out)
{
    vec32 all = {0, 0, 0};
    for (uint64_t a = 0; a < na; a++) {
        const float *r = A + 4 * a;
        for (uint64_t b = 0; b < nb; b++) {
            const float *s = B + 4 * b;
            if (overlap4(r[0], r[1], r[2], r[3], s[0], s[1], s[2], s[3])) {
                if (v32_push(&all, (uint32_t)a) || v32_push(&all, (uint32_t)b)) {
                    free(all.v); return -2;
                }
            }
        }
    }
    *pairs_out = all.v;
    *n_out = all.n / 2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* tree invariants                                                           */
/* ------------------------------------------------------------------------ */

static int fail(char *msg, int len, int code, const char *text, uint64_t a, uint64_t b)
{
    if (msg && len > 0) snprintf(msg, (size_t)len, "%s (%llu, %llu)", text,
                                 (unsigned long long)a, (unsigned long long)b);
    return code;
}

/* rects may be NULL (then leaf rectangles are not compared to the input). */
int ora_check_tree(const ora_tree *t, const float *rects, char *msg, int msglen)
{
    if (msg && msglen > 0) msg[0] = 0;
    if (t->n_nodes == 0) return t->n_objects == 0 ? 0 : fail(msg, msglen, 1, "no nodes", 0, 0);
    if (t->root >= t->n_nodes) return fail(msg, msglen, 2, "root out of range", t->root, t->n_nodes);
    if (t->level[t->root] + 1 != t->height)
        return fail(msg, msglen, 3, "root level != height-1", t->level[t->root], t->height);
    uint8_t *seen_node = (uint8_t *)calloc(t->n_nodes, 1);
    uint8_t *seen_obj = (uint8_t *)calloc((size_t)(t->n_objects ? t->n_objects : 1), 1);
    uint32_t *stack = (uint32_t *)malloc((size_t)t->n_nodes * sizeof(uint32_t));
    if (!seen_node || !seen_obj || !stack) {
        free(seen_node); free(seen_obj); free(stack);
        return fail(msg, msglen, 99, "out of memory", 0, 0);
    }
    int rc = 0;
    uint64_t objs = 0;
    size_t sp = 0;
    stack[sp++] = t->root;
    seen_node[t->root] = 1;
    while (sp && !rc) {
        uint32_t u = stack[--sp];
        uint32_t c = t->count[u];
        if (c > t->fanout) { rc = fail(msg, msglen, 4, "count > fanout", u, c); break; }
        if (c == 0 && !(u == t->root && t->n_objects == 0)) { rc = fail(msg, msglen, 5, "empty node", u, 0); break; }
        if (t->first[u] + c > t->n_entries) { rc = fail(msg, msglen, 6, "entries out of range", u, c); break; }
        for (uint64_t e = t->first[u]; e < t->first[u] + c && !rc; e++) {
            float lx = t->lx[e], ly = t->ly[e], hx = t->hx[e], hy = t->hy[e];
            if (isnan(lx) || isnan(ly) || isnan(hx) || isnan(hy) || !(lx <= hx) || !(ly <= hy)) {
                rc = fail(msg, msglen, 7, "bad entry rectangle", u, e); break;
            }
            uint32_t p = t->ptr[e];
            if (t->level[u] == 0) {
                if (p >= t->n_objects) { rc = fail(msg, msglen, 8, "object id out of range", u, p); break; }
                if (seen_obj[p]) { rc = fail(msg, msglen, 9, "object twice", p, 0); break; }
                seen_obj[p] = 1;
                objs++;
                if (rects) {
                    const float *r = rects + 4 * (uint64_t)p;
                    if (r[0] != lx || r[1] != ly || r[2] != hx || r[3] != hy) {
                        rc = fail(msg, msglen, 10, "leaf rectangle differs from input", p, e); break;
                    }
                }
            } else {
                if (p >= t->n_nodes) { rc = fail(msg, msglen, 11, "child out of range", u, p); break; }
                if (seen_node[p]) { rc = fail(msg, msglen, 12, "node reached twice", p, 0); break; }
                seen_node[p] = 1;
#if ORA_MUTANT != 11          /* mutant 11: levels are not compared */
                if (t->level[p] + 1 != t->level[u]) { rc = fail(msg, msglen, 13, "child level", u, p); break; }
#endif
                uint32_t cc = t->count[p];
                if (cc == 0 || t->first[p] + cc > t->n_entries) { rc = fail(msg, msglen, 14, "child entries", p, cc); break; }
                float ulx = INFINITY, uly = INFINITY, uhx = -INFINITY, uhy = -INFINITY;
                for (uint64_t f = t->first[p]; f < t->first[p] + cc; f++) {
                    if (t->lx[f] < ulx) ulx = t->lx[f];
                    if (t->ly[f] < uly) uly = t->ly[f];
                    if (t->hx[f] > uhx) uhx = t->hx[f];
                    if (t->hy[f] > uhy) uhy = t->hy[f];
                }
#if ORA_MUTANT != 10          /* mutant 10: the union comparison is skipped */
                if (ulx != lx || uly != ly || uhx != hx || uhy != hy) {
                    rc = fail(msg, msglen, 15, "parent MBR != union of child entries", u, p); break;
                }
#endif
                stack[sp++] = p;
            }
        }
    }
    if (!rc && objs != t->n_objects) rc = fail(msg, msglen, 16, "object count", objs, t->n_objects);
    if (!rc) {
        for (uint32_t u = 0; u < t->n_nodes; u++)
            if (!seen_node[u]) { rc = fail(msg, msglen, 17, "unreachable node", u, 0); break; }
    }
    free(seen_node); free(seen_obj); free(stack);
    return rc;
}
