/*
 * ORACLE -- test infrastructure only.  Plain, slow, single-threaded CPU
 * McSplit for the maximum common induced subgraph (MCS).  Only tests/, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never links it and shares no code with it.
 *
 * What it computes (paper Sec. II.A): the largest k such that k vertices of G
 * and k vertices of H induce isomorphic subgraphs, i.e. the largest injective
 * partial map f: V_G -> V_H with A_G(u,u') = A_H(f(u),f(u')) for every ordered
 * pair of distinct mapped vertices (and equal vertex labels when labelled).
 * The common subgraph need not be connected.
 *
 * How (paper Sec. II.B and Algorithm 1, the Solve procedure, run
 * sequentially):
 *   - vertices of each graph are ordered by descending degree (total degree
 *     when directed), ties kept in input order (Sec. IV.A names this as the
 *     ordering McSplit uses);
 *   - a label class ("bidomain") is a pair (L, R) of unmatched vertex lists,
 *     of G and of H, whose vertices carry the same label -- the bit string of
 *     their adjacency to the already-mapped vertices, in mapping order
 *     (Table 1);
 *   - bound = |M| + sum over classes of min(|L|, |R|)   (Eq. 1);
 *   - a node updates the incumbent when |M| > |M_best|, then returns if
 *     bound <= |M_best|;
 *   - otherwise it picks a class (smallest max(|L|,|R|), ties to the class
 *     holding the smallest G vertex index), the smallest v of its L, and for
 *     each w of its R in ascending order recurses on M + (v,w) with every
 *     class split by adjacency to v (G side) and to w (H side)
 *     (filterDomain); sub-classes empty on either side are dropped since they
 *     add 0 to Eq. 1 and can never be matched;
 *   - finally it recurses with v removed from G ("v unmatched").
 * Directed graphs split each class four ways by the pair of arcs (v->x, x->v)
 * against (w->y, y->w); labelled graphs start from one class per vertex label
 * present in both graphs (the paper leaves both variants to "small
 * algorithmic variations").
 *
 * Node count: one per entry into the recursive procedure, including entries
 * that prune at once and the root.
 *
 * Representation: dense uint8 adjacency matrices and sorted int vertex
 * lists -- deliberately unlike the bitset GPU search.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Test-only: a nonzero ORACLE_PLANT builds a deliberately wrong variant so a
 * test can show that the pins catch it (1: Eq. 1 drops a class, 2: H side
 * split by the arc in the wrong direction, 3: H side split around v instead
 * of w, 4: no "v unmatched" branch).  The shipped oracle is built with 0. */
#ifndef ORACLE_PLANT
#define ORACLE_PLANT 0
#endif

typedef struct {
    int32_t n;
    int32_t directed;
    const uint8_t *adj;   /* n*n row-major, adj[i*n+j] = 1 iff arc i -> j */
    const int32_t *label; /* n vertex labels, or NULL when unlabelled */
} oracle_graph;

typedef struct {
    int *l;
    int nl;
    int *r;
    int nr;
} bidomain;

/* Per recursion level scratch: classes of the child being built and the
 * vertex storage they point into. */
typedef struct {
    bidomain *cls;
    int *verts;
} level_buf;

typedef struct {
    int nG, nH, directed;
    uint8_t *aG, *aH; /* degree-ordered adjacency */
    int *ordG, *ordH; /* ordered index -> original vertex */
    level_buf *lev;
    int nlev;
    int *mg, *mh;     /* current mapping (ordered ids) */
    int *bg, *bh;     /* best mapping */
    int best;
    int64_t nodes, node_limit;
    int aborted;
    int target; /* > 0: stop as soon as a mapping of this size is found */
} search_ctx;

/* ---- degree ordering (Sec. IV.A) ------------------------------------- */

static void degree_order(const oracle_graph *g, int *ord)
{
    int n = g->n;
    int *deg = (int *)calloc((size_t)(n ? n : 1), sizeof(int));
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            deg[i] += g->adj[i * n + j];
            if (g->directed)
                deg[i] += g->adj[j * n + i];
        }
    for (int i = 0; i < n; i++)
        ord[i] = i;
    /* insertion sort: descending degree, stable on original index */
    for (int i = 1; i < n; i++) {
        int x = ord[i], k = i - 1;
        while (k >= 0 && deg[ord[k]] < deg[x]) {
            ord[k + 1] = ord[k];
            k--;
        }
        ord[k + 1] = x;
    }
    free(deg);
}

static uint8_t *reorder(const oracle_graph *g, const int *ord)
{
    int n = g->n;
    uint8_t *a = (uint8_t *)malloc((size_t)(n > 0 ? n * n : 1));
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            a[i * n + j] = g->adj[ord[i] * n + ord[j]];
    return a;
}

/* Adjacency "letter" of x relative to v: undirected 0/1, directed
 * [v->x] + 2[x->v]. */
static int letter(const uint8_t *a, int n, int directed, int v, int x)
{
    int c = a[v * n + x];
    if (directed)
        c += 2 * a[x * n + v];
    return c;
}

/* ---- Eq. 1 ----------------------------------------------------------- */

static int eq1_bound(int m, const bidomain *C, int K)
{
    int b = m;
    for (int k = (ORACLE_PLANT == 1 ? 1 : 0); k < K; k++)
        b += C[k].nl < C[k].nr ? C[k].nl : C[k].nr;
    return b;
}

/* ---- selectLabelClass / selectVertex ---------------------------------- */

static int select_class(const bidomain *C, int K)
{
    int best = -1, best_size = 0, best_v = 0;
    for (int k = 0; k < K; k++) {
        int size = C[k].nl > C[k].nr ? C[k].nl : C[k].nr;
        int v = C[k].l[0]; /* lists are sorted ascending */
        if (best < 0 || size < best_size || (size == best_size && v < best_v)) {
            best = k;
            best_size = size;
            best_v = v;
        }
    }
    return best;
}

/* ---- filterDomain: split every class by adjacency to v and to w ------ */

static int filter_domains(const search_ctx *s, const bidomain *C, int K, int v, int w,
                          bidomain *out, int *verts)
{
    int nletters = s->directed ? 4 : 2;
    int Kout = 0, used = 0;
    for (int k = 0; k < K; k++) {
        for (int a = 0; a < nletters; a++) {
            int *l = verts + used, nl = 0;
            for (int i = 0; i < C[k].nl; i++) {
                int x = C[k].l[i];
                if (x != v && letter(s->aG, s->nG, s->directed, v, x) == a)
                    l[nl++] = x;
            }
            int *r = l + nl, nr = 0;
            for (int i = 0; i < C[k].nr; i++) {
                int y = C[k].r[i];
#if ORACLE_PLANT == 2
                if (y != w && letter(s->aH, s->nH, s->directed, y, w) == a)
#elif ORACLE_PLANT == 3
                if (y != w && letter(s->aH, s->nH, s->directed, v < s->nH ? v : w, y) == a)
#else
                if (y != w && letter(s->aH, s->nH, s->directed, w, y) == a)
#endif
                    r[nr++] = y;
            }
            if (nl > 0 && nr > 0) {
                out[Kout].l = l;
                out[Kout].nl = nl;
                out[Kout].r = r;
                out[Kout].nr = nr;
                Kout++;
                used += nl + nr;
            }
        }
    }
    return Kout;
}

/* ---- Solve (Algorithm 1, sequential) ---------------------------------- */

static void solve(search_ctx *s, int level, int m, const bidomain *C, int K)
{
    if (s->aborted)
        return;
    s->nodes++;
    if (s->node_limit > 0 && s->nodes > s->node_limit) {
        s->aborted = 1;
        return;
    }
    if (m > s->best) {
        s->best = m;
        memcpy(s->bg, s->mg, sizeof(int) * (size_t)m);
        memcpy(s->bh, s->mh, sizeof(int) * (size_t)m);
        if (s->target > 0 && m >= s->target) {
            s->aborted = 1; /* found what was asked for */
            return;
        }
    }
    if (eq1_bound(m, C, K) <= s->best)
        return;

    int sel = select_class(C, K);
    int v = C[sel].l[0];
    level_buf *nb = &s->lev[level + 1];

    for (int i = 0; i < C[sel].nr; i++) {
        int w = C[sel].r[i];
        int K2 = filter_domains(s, C, K, v, w, nb->cls, nb->verts);
        s->mg[m] = v;
        s->mh[m] = w;
        solve(s, level + 1, m + 1, nb->cls, K2);
        if (s->aborted)
            return;
    }

    if (ORACLE_PLANT == 4)
        return;
    /* v unmatched: G = G \ v, M unchanged */
    int K2 = 0, used = 0;
    for (int k = 0; k < K; k++) {
        int *l = nb->verts + used, nl = 0;
        for (int i = 0; i < C[k].nl; i++)
            if (C[k].l[i] != v)
                l[nl++] = C[k].l[i];
        if (nl == 0)
            continue;
        int *r = l + nl;
        memcpy(r, C[k].r, sizeof(int) * (size_t)C[k].nr);
        nb->cls[K2].l = l;
        nb->cls[K2].nl = nl;
        nb->cls[K2].r = r;
        nb->cls[K2].nr = C[k].nr;
        K2++;
        used += nl + C[k].nr;
    }
    solve(s, level + 1, m, nb->cls, K2);
}

/* ---- set-up shared by the entry points -------------------------------- */

static int ctx_init_orders(search_ctx *s, const oracle_graph *G, const oracle_graph *H,
                           const int32_t *ordG, const int32_t *ordH);

static int ctx_init(search_ctx *s, const oracle_graph *G, const oracle_graph *H, int ordered)
{
    memset(s, 0, sizeof(*s));
    s->nG = G->n;
    s->nH = H->n;
    s->directed = G->directed;
    int nG1 = G->n ? G->n : 1, nH1 = H->n ? H->n : 1;
    s->ordG = (int *)malloc(sizeof(int) * (size_t)nG1);
    s->ordH = (int *)malloc(sizeof(int) * (size_t)nH1);
    if (ordered) {
        degree_order(G, s->ordG);
        degree_order(H, s->ordH);
    } else {
        for (int i = 0; i < G->n; i++)
            s->ordG[i] = i;
        for (int i = 0; i < H->n; i++)
            s->ordH[i] = i;
    }
    s->aG = reorder(G, s->ordG);
    s->aH = reorder(H, s->ordH);
    s->nlev = G->n + 2;
    s->lev = (level_buf *)calloc((size_t)s->nlev, sizeof(level_buf));
    int ncls = (nG1 < nH1 ? nG1 : nH1) + 1;
    for (int t = 0; t < s->nlev; t++) {
        s->lev[t].cls = (bidomain *)malloc(sizeof(bidomain) * (size_t)ncls);
        s->lev[t].verts = (int *)malloc(sizeof(int) * (size_t)(nG1 + nH1));
    }
    s->mg = (int *)malloc(sizeof(int) * (size_t)nG1);
    s->mh = (int *)malloc(sizeof(int) * (size_t)nG1);
    s->bg = (int *)malloc(sizeof(int) * (size_t)nG1);
    s->bh = (int *)malloc(sizeof(int) * (size_t)nG1);
    return 0;
}

/* As ctx_init, with the vertex orders given (ordG[k] = the vertex of G placed
 * at position k); used for the alternative ordering of Sec. IV.A. */
static int ctx_init_orders(search_ctx *s, const oracle_graph *G, const oracle_graph *H,
                           const int32_t *ordG, const int32_t *ordH)
{
    ctx_init(s, G, H, 0);
    for (int i = 0; i < G->n; i++)
        s->ordG[i] = ordG[i];
    for (int i = 0; i < H->n; i++)
        s->ordH[i] = ordH[i];
    free(s->aG);
    free(s->aH);
    s->aG = reorder(G, s->ordG);
    s->aH = reorder(H, s->ordH);
    return 0;
}

static void ctx_free(search_ctx *s)
{
    for (int t = 0; t < s->nlev; t++) {
        free(s->lev[t].cls);
        free(s->lev[t].verts);
    }
    free(s->lev);
    free(s->aG);
    free(s->aH);
    free(s->ordG);
    free(s->ordH);
    free(s->mg);
    free(s->mh);
    free(s->bg);
    free(s->bh);
}

/* Root classes into level 0: one class of all vertices when unlabelled, else
 * one class per label value present in both graphs. */
static int root_classes(search_ctx *s, const oracle_graph *G, const oracle_graph *H)
{
    level_buf *b = &s->lev[0];
    if (G->n == 0 || H->n == 0)
        return 0;
    if (!G->label) {
        int *l = b->verts, *r = b->verts + G->n;
        for (int i = 0; i < G->n; i++)
            l[i] = i;
        for (int i = 0; i < H->n; i++)
            r[i] = i;
        b->cls[0].l = l;
        b->cls[0].nl = G->n;
        b->cls[0].r = r;
        b->cls[0].nr = H->n;
        return 1;
    }
    int K = 0, used = 0;
    for (int i = 0; i < G->n; i++) {
        int lab = G->label[s->ordG[i]];
        int seen = 0;
        for (int j = 0; j < i; j++)
            if (G->label[s->ordG[j]] == lab)
                seen = 1;
        if (seen)
            continue;
        int *l = b->verts + used, nl = 0;
        for (int j = 0; j < G->n; j++)
            if (G->label[s->ordG[j]] == lab)
                l[nl++] = j;
        int *r = l + nl, nr = 0;
        for (int j = 0; j < H->n; j++)
            if (H->label[s->ordH[j]] == lab)
                r[nr++] = j;
        if (nr == 0)
            continue;
        b->cls[K].l = l;
        b->cls[K].nl = nl;
        b->cls[K].r = r;
        b->cls[K].nr = nr;
        K++;
        used += nl + nr;
    }
    return K;
}

/* ---- public entry points ---------------------------------------------- */

/*
 * Solve MCS(G, H).  Returns the size found; writes that many pairs (original
 * vertex ids) to map_g/map_h (capacity min(nG, nH)), the node count, whether
 * the search completed (0 when node_limit > 0 stopped it; the size is then a
 * lower bound) and the root bound.  G and H must agree on directed and on
 * label presence.
 */
static int32_t run_mcs(search_ctx *sp, const oracle_graph *G, const oracle_graph *H,
                       int64_t node_limit, int32_t *map_g, int32_t *map_h, int64_t *nodes,
                       int32_t *complete, int32_t *root_bound);

int32_t oracle_mcs(const oracle_graph *G, const oracle_graph *H, int64_t node_limit,
                   int32_t *map_g, int32_t *map_h, int64_t *nodes, int32_t *complete,
                   int32_t *root_bound)
{
    search_ctx s;
    ctx_init(&s, G, H, 1);
    return run_mcs(&s, G, H, node_limit, map_g, map_h, nodes, complete, root_bound);
}

/* As oracle_mcs, with the vertex orders given instead of descending degree
 * (ordG[k] = the vertex of G placed at position k, likewise ordH). */
int32_t oracle_mcs_ordered(const oracle_graph *G, const oracle_graph *H, const int32_t *ordG,
                           const int32_t *ordH, int64_t node_limit, int32_t *map_g,
                           int32_t *map_h, int64_t *nodes, int32_t *complete,
                           int32_t *root_bound)
{
    search_ctx s;
    ctx_init_orders(&s, G, H, ordG, ordH);
    return run_mcs(&s, G, H, node_limit, map_g, map_h, nodes, complete, root_bound);
}

static int32_t run_mcs(search_ctx *sp, const oracle_graph *G, const oracle_graph *H,
                       int64_t node_limit, int32_t *map_g, int32_t *map_h, int64_t *nodes,
                       int32_t *complete, int32_t *root_bound)
{
    search_ctx s = *sp;
    s.node_limit = node_limit;
    int K = root_classes(&s, G, H);
    if (root_bound)
        *root_bound = eq1_bound(0, s.lev[0].cls, K);
    solve(&s, 0, 0, s.lev[0].cls, K);
    for (int i = 0; i < s.best; i++) {
        if (map_g)
            map_g[i] = s.ordG[s.bg[i]];
        if (map_h)
            map_h[i] = s.ordH[s.bh[i]];
    }
    if (nodes)
        *nodes = s.nodes;
    if (complete)
        *complete = !s.aborted;
    int best = s.best;
    ctx_free(&s);
    return best;
}

/*
 * Replay the splits along a given path of k steps, in original vertex ids and
 * without reordering: step t maps path_g[t] -> path_h[t], or, when
 * path_h[t] < 0, removes path_g[t] from G ("v unmatched").  After the last
 * step writes, for every vertex, the index of the class holding it (-1 when
 * matched, removed or in no class), and returns the number of classes.
 * bounds[t] (t = 0..k) is the Eq. 1 bound before step t and after the last.
 * Returns -1 if a step pairs vertices that are not in the same class.
 */
int32_t oracle_path(const oracle_graph *G, const oracle_graph *H, int32_t k,
                    const int32_t *path_g, const int32_t *path_h, int32_t *bounds,
                    int32_t *cls_g, int32_t *cls_h)
{
    if (k < 0 || k > G->n)
        return -1;
    search_ctx s;
    ctx_init(&s, G, H, 0);
    int K = root_classes(&s, G, H);
    bidomain *C = s.lev[0].cls;
    int m = 0;
    int ok = 1;
    for (int t = 0; t < k && ok; t++) {
        bounds[t] = eq1_bound(m, C, K);
        int v = path_g[t], w = path_h[t];
        level_buf *nb = &s.lev[t + 1];
        int found = -1;
        for (int c = 0; c < K; c++)
            for (int i = 0; i < C[c].nl; i++)
                if (C[c].l[i] == v)
                    found = c;
        if (found < 0) {
            ok = 0;
            break;
        }
        if (w >= 0) {
            int inR = 0;
            for (int i = 0; i < C[found].nr; i++)
                if (C[found].r[i] == w)
                    inR = 1;
            if (!inR) {
                ok = 0;
                break;
            }
            K = filter_domains(&s, C, K, v, w, nb->cls, nb->verts);
            m++;
        } else {
            int K2 = 0, used = 0;
            for (int c = 0; c < K; c++) {
                int *l = nb->verts + used, nl = 0;
                for (int i = 0; i < C[c].nl; i++)
                    if (C[c].l[i] != v)
                        l[nl++] = C[c].l[i];
                if (nl == 0)
                    continue;
                int *r = l + nl;
                memcpy(r, C[c].r, sizeof(int) * (size_t)C[c].nr);
                nb->cls[K2].l = l;
                nb->cls[K2].nl = nl;
                nb->cls[K2].r = r;
                nb->cls[K2].nr = C[c].nr;
                K2++;
                used += nl + C[c].nr;
            }
            K = K2;
        }
        C = nb->cls;
    }
    int ret = -1;
    if (ok) {
        bounds[k] = eq1_bound(m, C, K);
        for (int i = 0; i < G->n; i++)
            cls_g[i] = -1;
        for (int i = 0; i < H->n; i++)
            cls_h[i] = -1;
        for (int c = 0; c < K; c++) {
            for (int i = 0; i < C[c].nl; i++)
                cls_g[C[c].l[i]] = c;
            for (int i = 0; i < C[c].nr; i++)
                cls_h[C[c].r[i]] = c;
        }
        ret = K;
    }
    ctx_free(&s);
    return ret;
}

/*
 * Does some common induced subgraph of size >= target contain the pairs of a
 * given path?  Replays the class split along the path (original ids; every
 * step must map v and w of one class), then searches on from there exactly
 * as Solve does, with the incumbent set to target - 1 so that only larger
 * mappings count, stopping at the first one found.  Returns 1 (yes), 0 (no),
 * -1 (the path is not a legal sequence of steps) or -2 (node_limit > 0 was
 * reached first).
 */
int32_t oracle_extend(const oracle_graph *G, const oracle_graph *H, int32_t k,
                      const int32_t *path_g, const int32_t *path_h, int32_t target,
                      int64_t node_limit, int64_t *nodes)
{
    if (k < 0 || k > G->n || k > H->n)
        return -1;
    search_ctx s;
    ctx_init(&s, G, H, 0);
    int K = root_classes(&s, G, H);
    bidomain *C = s.lev[0].cls;
    for (int t = 0; t < k; t++) {
        int v = path_g[t], w = path_h[t];
        int found = -1;
        for (int c = 0; c < K; c++)
            for (int i = 0; i < C[c].nl; i++)
                if (C[c].l[i] == v)
                    for (int j = 0; j < C[c].nr; j++)
                        if (C[c].r[j] == w)
                            found = c;
        if (found < 0) {
            ctx_free(&s);
            return -1;
        }
        level_buf *nb = &s.lev[t + 1];
        K = filter_domains(&s, C, K, v, w, nb->cls, nb->verts);
        s.mg[t] = v;
        s.mh[t] = w;
        C = nb->cls;
    }
    s.best = target - 1;
    s.target = target;
    s.node_limit = node_limit;
    solve(&s, k, k, C, K);
    int ret;
    if (s.best >= target)
        ret = 1;
    else if (s.aborted)
        ret = -2;
    else
        ret = 0;
    if (nodes)
        *nodes = s.nodes;
    ctx_free(&s);
    return ret;
}

/*
 * Proof cost of branching on a chosen vertex: replay the path (original
 * ids, in the descending-degree numbering the search uses), then expand that
 * node as Solve does but with v_first as the branching vertex (it must lie in
 * the class the node would select), the incumbent fixed at `incumbent` (so
 * nothing improves and only refutation work is counted), and count every
 * entry into Solve.  Returns the node count, -1 for an illegal path or
 * v_first, or -2 if node_limit > 0 was reached.
 */
int64_t oracle_branch_cost(const oracle_graph *G, const oracle_graph *H, int32_t k,
                           const int32_t *path_g, const int32_t *path_h, int32_t v_first,
                           int32_t incumbent, int64_t node_limit)
{
    if (k < 0 || k > G->n || k > H->n)
        return -1;
    search_ctx s;
    ctx_init(&s, G, H, 1);
    int nG = G->n, nH = H->n;
    int *invG = (int *)malloc(sizeof(int) * (size_t)(nG ? nG : 1));
    int *invH = (int *)malloc(sizeof(int) * (size_t)(nH ? nH : 1));
    for (int i = 0; i < nG; i++)
        invG[s.ordG[i]] = i;
    for (int i = 0; i < nH; i++)
        invH[s.ordH[i]] = i;
    int K = root_classes(&s, G, H);
    bidomain *C = s.lev[0].cls;
    int64_t ret = 0;
    for (int t = 0; t < k && ret == 0; t++) {
        int v = invG[path_g[t]], w = invH[path_h[t]];
        int found = -1;
        for (int c = 0; c < K; c++)
            for (int i = 0; i < C[c].nl; i++)
                if (C[c].l[i] == v)
                    for (int j = 0; j < C[c].nr; j++)
                        if (C[c].r[j] == w)
                            found = c;
        if (found < 0) {
            ret = -1;
            break;
        }
        level_buf *nb = &s.lev[t + 1];
        K = filter_domains(&s, C, K, v, w, nb->cls, nb->verts);
        s.mg[t] = v;
        s.mh[t] = w;
        C = nb->cls;
    }
    int vf = (v_first >= 0 && v_first < nG) ? invG[v_first] : -1;
    int sel = K > 0 ? select_class(C, K) : -1;
    int ok = 0;
    if (ret == 0 && sel >= 0)
        for (int i = 0; i < C[sel].nl; i++)
            if (C[sel].l[i] == vf)
                ok = 1;
    if (ret == 0 && !ok)
        ret = -1;
    if (ret == 0) {
        s.best = incumbent;
        s.node_limit = node_limit;
        s.nodes = 1; /* the node itself */
        int m = k;
        if (eq1_bound(m, C, K) > s.best) {
            level_buf *nb = &s.lev[k + 1];
            for (int i = 0; i < C[sel].nr && !s.aborted; i++) {
                int w = C[sel].r[i];
                int K2 = filter_domains(&s, C, K, vf, w, nb->cls, nb->verts);
                s.mg[m] = vf;
                s.mh[m] = w;
                solve(&s, k + 1, m + 1, nb->cls, K2);
            }
            if (!s.aborted) {
                int K2 = 0, used = 0;
                for (int c = 0; c < K; c++) {
                    int *l = nb->verts + used, nl = 0;
                    for (int i = 0; i < C[c].nl; i++)
                        if (C[c].l[i] != vf)
                            l[nl++] = C[c].l[i];
                    if (nl == 0)
                        continue;
                    int *r = l + nl;
                    memcpy(r, C[c].r, sizeof(int) * (size_t)C[c].nr);
                    nb->cls[K2].l = l;
                    nb->cls[K2].nl = nl;
                    nb->cls[K2].r = r;
                    nb->cls[K2].nr = C[c].nr;
                    K2++;
                    used += nl + C[c].nr;
                }
                solve(&s, k + 1, m, nb->cls, K2);
            }
        }
        ret = s.aborted ? -2 : s.nodes;
    }
    free(invG);
    free(invH);
    ctx_free(&s);
    return ret;
}
