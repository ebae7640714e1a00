/*
 * CPU oracle for the MBR filter step of the spatial intersection join
 * (Tsitsigkos, Bouros, Mamoulis, Terrovitis, "Parallel In-Memory Evaluation
 * of Spatial Joins", SIGSPATIAL 2019 / arXiv 1908.11740).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Three modes, each computing the same set
 *     J = { (i,j) : r_i and s_j share at least one point }          (Sec. 1)
 * over float32 rectangles given as (x_l, y_l, x_u, y_u):
 *
 *   oracle_bruteforce  the definition itself, a double loop (Sec. 1).
 *   oracle_sweep       Algorithm 1 (forward-scan plane sweep, Sec. 2.1)
 *                      over the whole input: no partitioning.
 *   oracle_pbsm        the paper's partition-based join: uniform K x K grid
 *                      (Sec. 2.2, PBSM), the parallel partitioning phase of
 *                      Sec. 3.4 (count per thread, sum, allocate, scatter into
 *                      per-thread sub-segments), per-tile sort by x_l and
 *                      Algorithm 1, and the reference-point duplicate test of
 *                      Eq. (1), with OpenMP threads as the paper's m threads.
 *
 * Readings taken where the paper is silent (all intersection tests closed,
 * i.e. touching edges/corners count; the y-test of Algorithm 1 is the closed
 * interval test; tiles are half-open [i/K,(i+1)/K) in the domain with cell
 * indices clamped to [0,K-1]; Eq. (1) evaluated on cell indices of the one
 * cell function used for assignment).
 *
 * All output pairs are 0-based positions (i in R, j in S).  Every function
 * returns the pair count and hands back a malloc'ed array of 2*count int32
 * (r,s) values in *out (NULL when the count is 0), released with
 * oracle_free().  A negative return means an allocation failed.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

/* ------------------------------------------------------------------ */
/* growable pair list                                                  */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t *v;   /* 2*n int32 */
    int64_t n, cap;
} plist;

static int plist_push(plist *p, int32_t r, int32_t s) {
    if (p->n == p->cap) {
        int64_t nc = p->cap ? 2 * p->cap : 1024;
        int32_t *nv = (int32_t *)realloc(p->v, (size_t)nc * 2 * sizeof(int32_t));
        if (!nv) return -1;
        p->v = nv;
        p->cap = nc;
    }
    p->v[2 * p->n] = r;
    p->v[2 * p->n + 1] = s;
    p->n++;
    return 0;
}

void oracle_free(void *p) { free(p); }

static double now_s(void) {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------ */
/* The definition (Sec. 1): r and s intersect iff their x-projections    */
/* and their y-projections both intersect as closed intervals.           */
/* ------------------------------------------------------------------ */
static int intersects(const float *r, const float *s) {
    return r[0] <= s[2] && s[0] <= r[2] && r[1] <= s[3] && s[1] <= r[3];
}

int64_t oracle_bruteforce(const float *R, int64_t nR, const float *S, int64_t nS,
                          int32_t **out) {
    plist p = {0, 0, 0};
    for (int64_t i = 0; i < nR; i++)
        for (int64_t j = 0; j < nS; j++)
            if (intersects(R + 4 * i, S + 4 * j))
                if (plist_push(&p, (int32_t)i, (int32_t)j)) { free(p.v); return -1; }
    *out = p.v;
    return p.n;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1: forward-scan plane sweep over two lists of entries.      */
/* ------------------------------------------------------------------ */
typedef struct {
    float xl, yl, xu, yu;
    int32_t id;
} entry;

static int by_xl(const void *a, const void *b) {
    float x = ((const entry *)a)->xl, y = ((const entry *)b)->xl;
    return (x > y) - (x < y);
}

/* Duplicate-test context: the tile (tx,ty) the sweep runs in and the cell
 * function of the grid; ctx == NULL means no partitioning (single tile). */
typedef struct {
    double x0, y0, sx, sy; /* cell(v) = floor((v - x0) * sx), sx = K / width */
    int K;
    int tx, ty;
} tile_ctx;

/* Cell index of a coordinate: floor of its offset from the domain's lower
 * edge in units of the tile extent, clamped into the grid.  Monotone in v. */
static int cell_of(double v, double lo, double scale, int K) {
    double c = floor((v - lo) * scale);
    if (c < 0) return 0;
    if (c > K - 1) return K - 1;
    return (int)c;
}

/* Eq. (1): report the pair found in tile T only if the reference point
 * p = (max{r.x_l,s.x_l}, max{r.y_l,s.y_l}) lies at or beyond T's lower
 * boundaries, where "at or beyond the lower boundary of tile t" is read as
 * "cell(p) >= t" for the same cell function that assigned the rectangles. */
static int reference_point_in_tile(const entry *r, const entry *s, const tile_ctx *c) {
    if (!c) return 1;
    double px = r->xl > s->xl ? r->xl : s->xl;
    double py = r->yl > s->yl ? r->yl : s->yl;
    return cell_of(px, c->x0, c->sx, c->K) >= c->tx && cell_of(py, c->y0, c->sy, c->K) >= c->ty;
}

/* y-test of Algorithm 1, read as closed-interval intersection. */
static int y_intersects(const entry *r, const entry *s) {
    return r->yl <= s->yu && s->yl <= r->yu;
}

/* First index in A[lo..hi) whose x_l is > v (strict = 1) or >= v (strict =
 * 0); hi if none.  A is sorted by x_l. */
static int64_t first_beyond(const entry *A, int64_t lo, int64_t hi, float v, int strict) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int before = strict ? (A[mid].xl <= v) : (A[mid].xl < v);
        if (before) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

/* Algorithm 1 (Sec. 2.1) over two lists sorted by x_l.  The sweep visits
 * the elements of both lists in x_l order (on equal x_l an element of S
 * before one of R) and, at each element, scans the elements of the other
 * list that come later in that order, as long as their x_l does not exceed
 * its x_u.  So the candidates of an r are the s with r.x_l < s.x_l <= r.x_u,
 * those of an s the r with s.x_l <= r.x_l <= s.x_u, and every pair whose
 * x-intervals meet is a candidate exactly once.  Each candidate gets the
 * closed y-test and, in a tile, the reference-point test of Eq. (1). */
static int sweep_sorted(const entry *Rl, int64_t nr, const entry *Sl, int64_t ns,
                        const tile_ctx *ctx, plist *out) {
    for (int64_t i = 0; i < nr; i++) {
        const entry *r = &Rl[i];
        int64_t from = first_beyond(Sl, 0, ns, r->xl, 1);
        int64_t to = first_beyond(Sl, from, ns, r->xu, 1);
        for (int64_t k = from; k < to; k++)
            if (y_intersects(r, &Sl[k]) && reference_point_in_tile(r, &Sl[k], ctx))
                if (plist_push(out, r->id, Sl[k].id)) return -1;
    }
    for (int64_t j = 0; j < ns; j++) {
        const entry *s = &Sl[j];
        int64_t from = first_beyond(Rl, 0, nr, s->xl, 0);
        int64_t to = first_beyond(Rl, from, nr, s->xu, 1);
        for (int64_t k = from; k < to; k++)
            if (y_intersects(&Rl[k], s) && reference_point_in_tile(&Rl[k], s, ctx))
                if (plist_push(out, Rl[k].id, s->id)) return -1;
    }
    return 0;
}

static entry *to_entries(const float *A, int64_t n) {
    entry *e = (entry *)malloc((size_t)(n ? n : 1) * sizeof(entry));
    if (!e) return NULL;
    for (int64_t i = 0; i < n; i++) {
        e[i].xl = A[4 * i];
        e[i].yl = A[4 * i + 1];
        e[i].xu = A[4 * i + 2];
        e[i].yu = A[4 * i + 3];
        e[i].id = (int32_t)i;
    }
    return e;
}

int64_t oracle_sweep(const float *R, int64_t nR, const float *S, int64_t nS, int32_t **out) {
    entry *Re = to_entries(R, nR), *Se = to_entries(S, nS);
    plist p = {0, 0, 0};
    int64_t ret = -1;
    if (!Re || !Se) goto done;
    qsort(Re, (size_t)nR, sizeof(entry), by_xl);
    qsort(Se, (size_t)nS, sizeof(entry), by_xl);
    if (sweep_sorted(Re, nR, Se, nS, NULL, &p)) goto done;
    ret = p.n;
    *out = p.v;
    p.v = NULL;
done:
    free(Re);
    free(Se);
    free(p.v);
    return ret;
}

/* ------------------------------------------------------------------ */
/* PBSM with the parallel partitioning and joining phases of Sec. 3.4.  */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t *off;    /* K*K + 1 segment offsets                          */
    entry *seg;      /* contiguous per-tile segments                     */
    int64_t total;   /* number of (replicated) entries                   */
} partitioned;

/* Cell ranges covered by rectangle a: every tile it intersects (Sec. 2.2). */
static void cell_range(const float *a, const tile_ctx *g, int *cx0, int *cx1, int *cy0,
                       int *cy1) {
    *cx0 = cell_of(a[0], g->x0, g->sx, g->K);
    *cx1 = cell_of(a[2], g->x0, g->sx, g->K);
    *cy0 = cell_of(a[1], g->y0, g->sy, g->K);
    *cy1 = cell_of(a[3], g->y0, g->sy, g->K);
}

/* Steps 1-4 of Sec. 3.4 for one input with m threads. */
static int partition_input(const float *A, int64_t n, const tile_ctx *g, int m,
                           partitioned *P) {
    const int64_t C = (int64_t)g->K * g->K;
    /* step 1: m equi-sized parts */
    int64_t part = (n + m - 1) / m;
    /* step 2: per-thread per-tile counts |A_T^i| */
    uint32_t *cnt = (uint32_t *)calloc((size_t)m * (size_t)C, sizeof(uint32_t));
    P->off = (int64_t *)malloc((size_t)(C + 1) * sizeof(int64_t));
    P->seg = NULL;
    if (!cnt || !P->off) { free(cnt); return -1; }
#pragma omp parallel num_threads(m)
    {
        int t = omp_get_thread_num();
        int64_t lo = t * part, hi = lo + part < n ? lo + part : n;
        uint32_t *c = cnt + (size_t)t * (size_t)C;
        for (int64_t i = lo; i < hi; i++) {
            int cx0, cx1, cy0, cy1;
            cell_range(A + 4 * i, g, &cx0, &cx1, &cy0, &cy1);
            for (int y = cy0; y <= cy1; y++)
                for (int x = cx0; x <= cx1; x++) c[(int64_t)y * g->K + x]++;
        }
    }
    /* step 3: |A_T| = sum_i |A_T^i|; allocate one contiguous segment per tile,
     * logically divided into per-thread sub-segments */
    int64_t run = 0;
    for (int64_t T = 0; T < C; T++) {
        P->off[T] = run;
        for (int t = 0; t < m; t++) {
            uint32_t v = cnt[(size_t)t * (size_t)C + T];
            cnt[(size_t)t * (size_t)C + T] = (uint32_t)(run - P->off[T]); /* sub-segment start */
            run += v;
        }
    }
    P->off[C] = run;
    P->total = run;
    P->seg = (entry *)malloc((size_t)(run ? run : 1) * sizeof(entry));
    if (!P->seg) { free(cnt); return -1; }
    /* step 4: thread i writes its part into its sub-segments */
#pragma omp parallel num_threads(m)
    {
        int t = omp_get_thread_num();
        int64_t lo = t * part, hi = lo + part < n ? lo + part : n;
        uint32_t *c = cnt + (size_t)t * (size_t)C;
        for (int64_t i = lo; i < hi; i++) {
            int cx0, cx1, cy0, cy1;
            const float *a = A + 4 * i;
            cell_range(a, g, &cx0, &cx1, &cy0, &cy1);
            for (int y = cy0; y <= cy1; y++)
                for (int x = cx0; x <= cx1; x++) {
                    int64_t T = (int64_t)y * g->K + x;
                    entry *e = &P->seg[P->off[T] + c[T]++];
                    e->xl = a[0];
                    e->yl = a[1];
                    e->xu = a[2];
                    e->yu = a[3];
                    e->id = (int32_t)i;
                }
        }
    }
    free(cnt);
    return 0;
}

/* domain: x0,y0,x1,y1 of the grid (NULL or all zero = unit square).
 * threads <= 0: all available.  t_part / t_join (may be NULL) receive the
 * wall seconds of the two phases. */
int64_t oracle_pbsm(const float *R, int64_t nR, const float *S, int64_t nS, int K,
                    const float *domain, int threads, int32_t **out, double *t_part,
                    double *t_join) {
    if (K < 1) return -2;
    int m = threads > 0 ? threads : omp_get_max_threads();
    tile_ctx g;
    double d[4] = {0.0, 0.0, 1.0, 1.0};
    if (domain && !(domain[0] == 0 && domain[1] == 0 && domain[2] == 0 && domain[3] == 0))
        for (int k = 0; k < 4; k++) d[k] = domain[k];
    g.x0 = d[0];
    g.y0 = d[1];
    g.sx = K / (d[2] - d[0]);
    g.sy = K / (d[3] - d[1]);
    g.K = K;
    g.tx = g.ty = 0;
    const int64_t C = (int64_t)K * K;

    double t0 = now_s();
    partitioned PR = {0, 0, 0}, PS = {0, 0, 0};
    int64_t ret = -1;
    plist *outs = NULL;
    if (partition_input(R, nR, &g, m, &PR) || partition_input(S, nS, &g, m, &PS)) goto done;
    double t1 = now_s();

    /* step 5: one sort task per tile and input */
#pragma omp parallel for schedule(dynamic, 64) num_threads(m)
    for (int64_t T = 0; T < C; T++) {
        qsort(PR.seg + PR.off[T], (size_t)(PR.off[T + 1] - PR.off[T]), sizeof(entry), by_xl);
        qsort(PS.seg + PS.off[T], (size_t)(PS.off[T + 1] - PS.off[T]), sizeof(entry), by_xl);
    }
    /* step 6: one join task per tile (Algorithm 1 + Eq. (1)) */
    outs = (plist *)calloc((size_t)m, sizeof(plist));
    if (!outs) goto done;
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(m) reduction(| : failed)
    for (int64_t T = 0; T < C; T++) {
        tile_ctx c = g;
        c.tx = (int)(T % K);
        c.ty = (int)(T / K);
        if (sweep_sorted(PR.seg + PR.off[T], PR.off[T + 1] - PR.off[T], PS.seg + PS.off[T],
                         PS.off[T + 1] - PS.off[T], &c, &outs[omp_get_thread_num()]))
            failed = 1;
    }
    if (failed) goto done;
    double t2 = now_s();
    int64_t total = 0;
    for (int t = 0; t < m; t++) total += outs[t].n;
    int32_t *v = (int32_t *)malloc((size_t)(total ? total : 1) * 2 * sizeof(int32_t));
    if (!v) goto done;
    int64_t at = 0;
    for (int t = 0; t < m; t++) {
        if (outs[t].n) memcpy(v + 2 * at, outs[t].v, (size_t)outs[t].n * 2 * sizeof(int32_t));
        at += outs[t].n;
    }
    *out = v;
    ret = total;
    if (t_part) *t_part = t1 - t0;
    if (t_join) *t_join = t2 - t1;
done:
    if (outs)
        for (int t = 0; t < m; t++) free(outs[t].v);
    free(outs);
    free(PR.off);
    free(PR.seg);
    free(PS.off);
    free(PS.seg);
    return ret;
}

/* Per-tile membership of one input under the oracle's own grid: writes the
 * K*K+1 offsets and the ids of each tile's segment, ids ascending within a
 * tile.  Used by tests that check partition invariants.  Returns the number
 * of entries, or -1.  *ids is malloc'ed (release with oracle_free). */
int64_t oracle_partition_ids(const float *A, int64_t n, int K, const float *domain,
                             int64_t *off, int32_t **ids) {
    tile_ctx g;
    double d[4] = {0.0, 0.0, 1.0, 1.0};
    if (domain && !(domain[0] == 0 && domain[1] == 0 && domain[2] == 0 && domain[3] == 0))
        for (int k = 0; k < 4; k++) d[k] = domain[k];
    g.x0 = d[0];
    g.y0 = d[1];
    g.sx = K / (d[2] - d[0]);
    g.sy = K / (d[3] - d[1]);
    g.K = K;
    partitioned P = {0, 0, 0};
    if (partition_input(A, n, &g, 1, &P)) { free(P.off); free(P.seg); return -1; }
    const int64_t C = (int64_t)K * K;
    memcpy(off, P.off, (size_t)(C + 1) * sizeof(int64_t));
    int32_t *v = (int32_t *)malloc((size_t)(P.total ? P.total : 1) * sizeof(int32_t));
    if (!v) { free(P.off); free(P.seg); return -1; }
    for (int64_t k = 0; k < P.total; k++) v[k] = P.seg[k].id;
    *ids = v;
    int64_t tot = P.total;
    free(P.off);
    free(P.seg);
    return tot;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Epsilon-distance join of point sets (Sec. 1), the definition:        */
/* every (i, j) with dx*dx + dy*dy <= eps*eps, evaluated in double from */
/* the float coordinates, each operation rounded once (the build turns  */
/* off contraction into fused multiply-adds).  Points are (x, y) pairs.  */
/* ------------------------------------------------------------------ */
static int within(const float *p, const float *q, double e2) {
    double dx = (double)p[0] - (double)q[0];
    double dy = (double)p[1] - (double)q[1];
    return dx * dx + dy * dy <= e2;
}

int64_t oracle_distance_brute(const float *P, int64_t nP, const float *Q, int64_t nQ, float eps,
                              int32_t **out) {
    plist p = {0, 0, 0};
    double e2 = (double)eps * (double)eps;
    for (int64_t i = 0; i < nP; i++)
        for (int64_t j = 0; j < nQ; j++)
            if (within(P + 2 * i, Q + 2 * j, e2))
                if (plist_push(&p, (int32_t)i, (int32_t)j)) { free(p.v); return -1; }
    *out = p.v;
    return p.n;
}

/* The refinement step alone: keep the candidate pairs (2*n int32) that
 * satisfy the distance test, in place; returns how many were kept. */
int64_t oracle_distance_refine(const float *P, const float *Q, float eps, int32_t *pairs,
                               int64_t n) {
    double e2 = (double)eps * (double)eps;
    int64_t k = 0;
    for (int64_t c = 0; c < n; c++) {
        int32_t i = pairs[2 * c], j = pairs[2 * c + 1];
        if (within(P + 2 * (int64_t)i, Q + 2 * (int64_t)j, e2)) {
            pairs[2 * k] = i;
            pairs[2 * k + 1] = j;
            k++;
        }
    }
    return k;
}

/* ------------------------------------------------------------------ */
/* GBDA (grouping-based duplicate avoidance, the mini-joins the paper  */
/* sketches before Sec. 3.3): in tile T a rectangle is of class A if   */
/* its x- and y-projections both begin inside T, B if only x does, C   */
/* if only y does, D if neither ("begins inside T" = its lower corner's */
/* cell index equals the tile's, the integer form of the tile bounds). */
/* Of the 16 class-class joins only the 9 in which some rectangle      */
/* begins inside T along x and some along y can produce a pair whose   */
/* reference point lies in T; they are joined with Algorithm 1 and no  */
/* duplicate test.                                                     */
/* ------------------------------------------------------------------ */
static int gbda_class(const entry *e, const tile_ctx *c) {
    int bx = cell_of(e->xl, c->x0, c->sx, c->K) == c->tx;
    int by = cell_of(e->yl, c->y0, c->sy, c->K) == c->ty;
    return (bx ? 0 : 2) + (by ? 0 : 1); /* A 0, B 1, C 2, D 3 */
}

static int gbda_valid(int a, int b) {
    int bxa = a < 2, bya = (a & 1) == 0, bxb = b < 2, byb = (b & 1) == 0;
    return (bxa || bxb) && (bya || byb);
}

int64_t oracle_gbda(const float *R, int64_t nR, const float *S, int64_t nS, int K,
                    const float *domain, int32_t **out) {
    if (K < 1) return -2;
    tile_ctx g;
    double d[4] = {0.0, 0.0, 1.0, 1.0};
    if (domain && !(domain[0] == 0 && domain[1] == 0 && domain[2] == 0 && domain[3] == 0))
        for (int k = 0; k < 4; k++) d[k] = domain[k];
    g.x0 = d[0];
    g.y0 = d[1];
    g.sx = K / (d[2] - d[0]);
    g.sy = K / (d[3] - d[1]);
    g.K = K;
    g.tx = g.ty = 0;
    partitioned PR = {0, 0, 0}, PS = {0, 0, 0};
    plist p = {0, 0, 0};
    int64_t ret = -1;
    entry *grp = NULL;
    if (partition_input(R, nR, &g, 1, &PR) || partition_input(S, nS, &g, 1, &PS)) goto done;
    const int64_t C = (int64_t)K * K;
    for (int64_t T = 0; T < C; T++) {
        tile_ctx c = g;
        c.tx = (int)(T % K);
        c.ty = (int)(T / K);
        const entry *Rt = PR.seg + PR.off[T], *St = PS.seg + PS.off[T];
        int64_t nr = PR.off[T + 1] - PR.off[T], ns = PS.off[T + 1] - PS.off[T];
        if (!nr || !ns) continue;
        /* the four class groups of each list, each sorted by x_l */
        entry *gr = (entry *)malloc((size_t)(nr + ns) * sizeof(entry));
        if (!gr) goto done;
        free(grp);
        grp = gr;
        int64_t rs[5] = {0}, ss[5] = {0};
        for (int cl = 0, at = 0; cl < 4; cl++) {
            rs[cl] = at;
            for (int64_t i = 0; i < nr; i++)
                if (gbda_class(&Rt[i], &c) == cl) grp[at++] = Rt[i];
            rs[cl + 1] = at;
        }
        for (int cl = 0, at = 0; cl < 4; cl++) {
            ss[cl] = at;
            for (int64_t i = 0; i < ns; i++)
                if (gbda_class(&St[i], &c) == cl) grp[nr + at++] = St[i];
            ss[cl + 1] = at;
        }
        for (int cl = 0; cl < 4; cl++) {
            qsort(grp + rs[cl], (size_t)(rs[cl + 1] - rs[cl]), sizeof(entry), by_xl);
            qsort(grp + nr + ss[cl], (size_t)(ss[cl + 1] - ss[cl]), sizeof(entry), by_xl);
        }
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++)
                if (gbda_valid(a, b) &&
                    sweep_sorted(grp + rs[a], rs[a + 1] - rs[a], grp + nr + ss[b], ss[b + 1] - ss[b],
                                 NULL, &p))
                    goto done;
    }
    ret = p.n;
    *out = p.v;
    p.v = NULL;
done:
    free(grp);
    free(p.v);
    free(PR.off);
    free(PR.seg);
    free(PS.off);
    free(PS.seg);
    return ret;
}
