/*
 * ged_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of what the K-Best
 * graph-edit-distance search computes.  It exists to check the GPU library
 * against; nothing in the product path may link or call it.  Only tests,
 * the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * It shares no code with the GPU library: graphs are held as dense n x n
 * edge matrices, the implied edge costs are found by a scalar scan over the
 * previously edited vertices, and the K best children are chosen by a full
 * sort.
 *
 * Source of each function (the paper: "Efficient Accelerated Graph Edit
 * Distance Computation on GPU"):
 *   oracle_induced_cost  -- the edit cost of a complete vertex mapping, from
 *                           the GED definition (Sec. 2.2), the implied edge
 *                           operations (Sec. 2.3) and the cost function
 *                           (Sec. 2.4).
 *   oracle_exact         -- exact GED, the limit K -> infinity of the search
 *                           (Sec. 4.5): the minimum of oracle_induced_cost over
 *                           every injective mapping V1 -> V2 u {deleted}.
 *   oracle_kbest         -- the K-Best search (Alg. 1), with branching
 *                           (Sec. 4.2.1), partial edit distance by implied edges
 *                           (Sec. 2.3, Alg. 2), selection of the best K
 *                           (Sec. 4.3) and final insertion of the unmatched
 *                           target vertices (Sec. 4.4.1).
 *   oracle_kbest_ex      -- the same with a choice of last level: the literal
 *                           reading above, or "complete then take the minimum":
 *                           every child of the last level is completed by the
 *                           insertions of Sec. 4.4.1 and the least total wins
 *                           (Alg. 1's final minimum taken over all of them
 *                           instead of over the K kept by partial distance).
 *
 * Directed graphs (each function's `directed` argument): the edges are arcs
 * (a, b), a != b, at most one per ordered pair, so a and b may be joined by
 * two arcs.  Every place that looks at the unordered pair {a, b} of an
 * undirected graph looks at the ordered pairs (a, b) and (b, a) instead: the
 * implied operations of Sec. 2.3 between the edited vertex and an earlier
 * one are taken for each direction (the "source or destination" scan of
 * Sec. 4.4.1, read as both arc directions), and each arc is one edit
 * operation.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes): g1 vertices are processed in index order; the children of a node
 * are the substitutions by ascending g2 index followed by the deletion;
 * among children of equal partial edit distance the earlier one in that
 * generation order wins the last places of the K; the search selects the
 * best K at every level including the last and then adds the insertions;
 * among leaves of equal total cost the first in beam order is returned.
 *
 * Parity pins live in tests/: networkx exact GED, an independent
 * matrix-form brute force, a from-scratch beam, closed forms and
 * hand-derived values.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENOMEM = 2, OR_ETOOBIG = 3 };

typedef struct {
    int n;
    const int32_t *vl;   /* vertex labels [n] */
    uint8_t *has;        /* has[a*n+b] = 1 iff {a,b} is an edge */
    int32_t *lab;        /* lab[a*n+b] = label of edge {a,b} (0 when unlabelled) */
    int m;
    int directed;        /* 1: has[a*n+b] is the arc a -> b only */
} dgraph;

static void dg_free(dgraph *g) {
    free(g->has);
    free(g->lab);
    g->has = NULL;
    g->lab = NULL;
}

/* Build the dense form; rejects out-of-range vertices, self-loops and
 * repeated edges (the paper's graphs are simple, Sec. 2.1).  Directed: edge k
 * is the arc eu[k] -> ev[k]; the reverse arc is another edge. */
static int dg_build(dgraph *g, int n, const int32_t *vl, int m, const int32_t *eu,
                    const int32_t *ev, const int32_t *el, int directed) {
    g->n = n;
    g->vl = vl;
    g->m = m;
    g->directed = directed ? 1 : 0;
    g->has = NULL;
    g->lab = NULL;
    if (n < 0 || m < 0) return OR_EINVAL;
    size_t nn = (size_t)n * (size_t)n;
    g->has = (uint8_t *)calloc(nn ? nn : 1, 1);
    g->lab = (int32_t *)calloc(nn ? nn : 1, sizeof(int32_t));
    if (!g->has || !g->lab) { dg_free(g); return OR_ENOMEM; }
    for (int k = 0; k < m; k++) {
        int a = eu[k], b = ev[k];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b) { dg_free(g); return OR_EINVAL; }
        if (g->has[(size_t)a * n + b]) { dg_free(g); return OR_EINVAL; }
        int32_t l = el ? el[k] : 0;
        g->has[(size_t)a * n + b] = 1;
        g->lab[(size_t)a * n + b] = l;
        if (!g->directed) {
            g->has[(size_t)b * n + a] = 1;
            g->lab[(size_t)b * n + a] = l;
        }
    }
    return OR_OK;
}

static int edge(const dgraph *g, int a, int b) { return g->has[(size_t)a * g->n + b]; }
static int32_t elab(const dgraph *g, int a, int b) { return g->lab[(size_t)a * g->n + b]; }

/* costs[6] = vsub, vdel, vins, esub, edel, eins */
static int costs_ok(const int32_t *c) {
    for (int k = 0; k < 6; k++)
        if (c[k] < 0) return 0;
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Edit cost of a complete mapping (Sec. 2.2-2.4).  map[v] in {-1 (deleted),
 * 0..n2-1}; g2 vertices not in the image are inserted.                    */
static int64_t induced_cost(const dgraph *g1, const dgraph *g2, const int32_t *c,
                            const int32_t *map, int *pre /* [n2] scratch */) {
    int64_t cost = 0;
    for (int u = 0; u < g2->n; u++) pre[u] = -1;
    for (int v = 0; v < g1->n; v++) {
        if (map[v] < 0) {
            cost += c[1];                                 /* vertex deletion */
        } else {
            pre[map[v]] = v;
            if (g1->vl[v] != g2->vl[map[v]]) cost += c[0]; /* vertex substitution */
        }
    }
    for (int u = 0; u < g2->n; u++)
        if (pre[u] < 0) cost += c[2];                     /* vertex insertion */
    /* every g1 edge: deleted unless both ends map onto a g2 edge; substituted
     * when it does and the labels differ.  Undirected: each pair a < b once;
     * directed: every ordered pair (a, b), the arc a -> b onto phi(a) -> phi(b) */
    for (int a = 0; a < g1->n; a++)
        for (int b = g1->directed ? 0 : a + 1; b < g1->n; b++) {
            if (b == a || !edge(g1, a, b)) continue;
            int x = map[a], y = map[b];
            if (x < 0 || y < 0 || !edge(g2, x, y)) cost += c[4];
            else if (elab(g1, a, b) != elab(g2, x, y)) cost += c[3];
        }
    /* every g2 edge not the image of a g1 edge is inserted */
    for (int x = 0; x < g2->n; x++)
        for (int y = g2->directed ? 0 : x + 1; y < g2->n; y++) {
            if (y == x || !edge(g2, x, y)) continue;
            int a = pre[x], b = pre[y];
            if (a < 0 || b < 0 || !edge(g1, a, b)) cost += c[5];
        }
    return cost;
}

static int check_map(const int32_t *map, int n1, int n2, int *seen) {
    for (int u = 0; u < n2; u++) seen[u] = 0;
    for (int v = 0; v < n1; v++) {
        if (map[v] == -1) continue;
        if (map[v] < 0 || map[v] >= n2 || seen[map[v]]) return 0;
        seen[map[v]] = 1;
    }
    return 1;
}

int oracle_induced_cost(int n1, const int32_t *vl1, int m1, const int32_t *eu1,
                        const int32_t *ev1, const int32_t *el1, int n2, const int32_t *vl2,
                        int m2, const int32_t *eu2, const int32_t *ev2, const int32_t *el2,
                        const int32_t *costs, int directed, const int32_t *map, int64_t *cost_out) {
    if (!costs_ok(costs)) return OR_EINVAL;
    dgraph g1, g2;
    int st = dg_build(&g1, n1, vl1, m1, eu1, ev1, el1, directed);
    if (st) return st;
    st = dg_build(&g2, n2, vl2, m2, eu2, ev2, el2, directed);
    if (st) { dg_free(&g1); return st; }
    int *pre = (int *)malloc(sizeof(int) * (size_t)(n2 + 1));
    if (!pre) { dg_free(&g1); dg_free(&g2); return OR_ENOMEM; }
    if (!check_map(map, n1, n2, pre)) st = OR_EINVAL;
    else *cost_out = induced_cost(&g1, &g2, costs, map, pre);
    free(pre);
    dg_free(&g1);
    dg_free(&g2);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Exact GED: every injective partial mapping, cost from scratch, keep the
 * first minimum in enumeration order (substitutions by ascending g2 index,
 * then deletion, for g1 vertices in index order).                          */
typedef struct {
    const dgraph *g1, *g2;
    const int32_t *c;
    int32_t *map, *best_map;
    int *used, *pre;
    int64_t best;
} exact_ctx;

static void exact_rec(exact_ctx *x, int v) {
    if (v == x->g1->n) {
        int64_t cost = induced_cost(x->g1, x->g2, x->c, x->map, x->pre);
        if (cost < x->best) {
            x->best = cost;
            memcpy(x->best_map, x->map, sizeof(int32_t) * (size_t)x->g1->n);
        }
        return;
    }
    for (int u = 0; u < x->g2->n; u++) {
        if (x->used[u]) continue;
        x->used[u] = 1;
        x->map[v] = u;
        exact_rec(x, v + 1);
        x->used[u] = 0;
    }
    x->map[v] = -1;
    exact_rec(x, v + 1);
}

/* number of complete mappings: sum_s C(n1,s) * n2!/(n2-s)! */
double oracle_count_mappings(int n1, int n2) {
    double total = 0.0;
    for (int s = 0; s <= n1 && s <= n2; s++) {
        double comb = 1.0, perm = 1.0;
        for (int k = 0; k < s; k++) {
            comb = comb * (double)(n1 - k) / (double)(k + 1);
            perm *= (double)(n2 - k);
        }
        total += comb * perm;
    }
    return total;
}

int oracle_exact(int n1, const int32_t *vl1, int m1, const int32_t *eu1, const int32_t *ev1,
                 const int32_t *el1, int n2, const int32_t *vl2, int m2, const int32_t *eu2,
                 const int32_t *ev2, const int32_t *el2, const int32_t *costs, int directed,
                 double max_mappings, int64_t *dist, int32_t *map_out) {
    if (!costs_ok(costs)) return OR_EINVAL;
    if (oracle_count_mappings(n1, n2) > max_mappings) return OR_ETOOBIG;
    dgraph g1, g2;
    int st = dg_build(&g1, n1, vl1, m1, eu1, ev1, el1, directed);
    if (st) return st;
    st = dg_build(&g2, n2, vl2, m2, eu2, ev2, el2, directed);
    if (st) { dg_free(&g1); return st; }
    exact_ctx x;
    x.g1 = &g1;
    x.g2 = &g2;
    x.c = costs;
    x.map = (int32_t *)calloc((size_t)n1 + 1, sizeof(int32_t));
    x.best_map = (int32_t *)calloc((size_t)n1 + 1, sizeof(int32_t));
    x.used = (int *)calloc((size_t)n2 + 1, sizeof(int));
    x.pre = (int *)calloc((size_t)n2 + 1, sizeof(int));
    x.best = INT64_MAX;
    if (!x.map || !x.best_map || !x.used || !x.pre) {
        st = OR_ENOMEM;
    } else {
        exact_rec(&x, 0);
        *dist = x.best;
        memcpy(map_out, x.best_map, sizeof(int32_t) * (size_t)n1);
    }
    free(x.map);
    free(x.best_map);
    free(x.used);
    free(x.pre);
    dg_free(&g1);
    dg_free(&g2);
    return st;
}

/* ---------------------------------------------------------------------- */
/* K-Best search (Alg. 1).                                                 */
#define DELETED (-1)

typedef struct {
    int64_t ped;   /* partial edit distance of the child */
    int64_t order; /* position in generation order */
} rank_key;

static int cmp_rank(const void *a, const void *b) {
    const rank_key *x = (const rank_key *)a, *y = (const rank_key *)b;
    if (x->ped != y->ped) return x->ped < y->ped ? -1 : 1;
    if (x->order != y->order) return x->order < y->order ? -1 : 1;
    return 0;
}

static int cmp_order(const void *a, const void *b) {
    const rank_key *x = (const rank_key *)a, *y = (const rank_key *)b;
    return x->order < y->order ? -1 : (x->order > y->order ? 1 : 0);
}

/* Partial edit distance added by substituting g1 vertex i by g2 vertex u,
 * given the parent's mapping of vertices 0..i-1 (Alg. 2 and Sec. 2.3):
 * the vertex substitution cost plus, for every previously edited vertex j,
 * the implied operation on the pair (i, j) versus (u, phi[j]).            */
static int64_t pair_op(const dgraph *g1, const dgraph *g2, const int32_t *c, int a, int b, int x,
                       int y) {
    int e1 = edge(g1, a, b);
    int e2 = (x != DELETED && y != DELETED) && edge(g2, x, y);
    if (e1 && !e2) return c[4];                                       /* edge deletion */
    if (!e1 && e2) return c[5];                                       /* edge insertion */
    if (e1 && e2 && elab(g1, a, b) != elab(g2, x, y)) return c[3];    /* substitution */
    return 0;
}

/* Directed graphs: the pair (i, j) is the arc i -> j and the arc j -> i, each
 * against its image. */
static int64_t sub_step(const dgraph *g1, const dgraph *g2, const int32_t *c, int i, int u,
                        const int32_t *phi) {
    int64_t d = (g1->vl[i] != g2->vl[u]) ? c[0] : 0;
    for (int j = 0; j < i; j++) {
        d += pair_op(g1, g2, c, i, j, u, phi[j]);
        if (g1->directed) d += pair_op(g1, g2, c, j, i, phi[j], u);
    }
    return d;
}

/* Deleting g1 vertex i deletes it and its edges to earlier vertices. */
static int64_t del_step(const dgraph *g1, const int32_t *c, int i) {
    int64_t d = c[1];
    for (int j = 0; j < i; j++) {
        if (edge(g1, i, j)) d += c[4];
        if (g1->directed && edge(g1, j, i)) d += c[4];
    }
    return d;
}

/* Insertions that complete a mapping whose used g2 vertices are marked in
 * `used` (Sec. 4.4.1): every unused g2 vertex and every g2 edge with an
 * unused end. */
static int64_t completion(const dgraph *g2, const int32_t *c, const int *used) {
    int64_t t = 0;
    for (int u = 0; u < g2->n; u++)
        if (!used[u]) t += c[2];
    for (int x = 0; x < g2->n; x++)
        for (int y = g2->directed ? 0 : x + 1; y < g2->n; y++)
            if (y != x && edge(g2, x, y) && (!used[x] || !used[y])) t += c[5];
    return t;
}

int oracle_kbest_cand(int n1, const int32_t *vl1, int m1, const int32_t *eu1, const int32_t *ev1,
                      const int32_t *el1, int n2, const int32_t *vl2, int m2, const int32_t *eu2,
                      const int32_t *ev2, const int32_t *el2, const int32_t *costs, int64_t K,
                      int last_complete, int directed, int64_t *dist, int32_t *map_out, int64_t *cand_out);

int oracle_kbest_ex(int n1, const int32_t *vl1, int m1, const int32_t *eu1, const int32_t *ev1,
                    const int32_t *el1, int n2, const int32_t *vl2, int m2, const int32_t *eu2,
                    const int32_t *ev2, const int32_t *el2, const int32_t *costs, int64_t K,
                    int last_complete, int directed, int64_t *dist, int32_t *map_out) {
    return oracle_kbest_cand(n1, vl1, m1, eu1, ev1, el1, n2, vl2, m2, eu2, ev2, el2, costs, K, last_complete,
                             directed, dist, map_out, NULL);
}

int oracle_kbest(int n1, const int32_t *vl1, int m1, const int32_t *eu1, const int32_t *ev1,
                 const int32_t *el1, int n2, const int32_t *vl2, int m2, const int32_t *eu2,
                 const int32_t *ev2, const int32_t *el2, const int32_t *costs, int64_t K,
                 int64_t *dist, int32_t *map_out) {
    return oracle_kbest_cand(n1, vl1, m1, eu1, ev1, el1, n2, vl2, m2, eu2, ev2, el2, costs, K, 0, 0, dist,
                             map_out, NULL);
}

/* The search; *cand_out (may be NULL) gets the number of children generated
 * over all levels (Alg. 1's branching, Sec. 4.2.1: per level, one child per
 * unused g2 vertex of every retained node plus its deletion child), each of
 * which has its partial edit distance evaluated once. */
int oracle_kbest_cand(int n1, const int32_t *vl1, int m1, const int32_t *eu1, const int32_t *ev1,
                      const int32_t *el1, int n2, const int32_t *vl2, int m2, const int32_t *eu2,
                      const int32_t *ev2, const int32_t *el2, const int32_t *costs, int64_t K,
                      int last_complete, int directed, int64_t *dist, int32_t *map_out, int64_t *cand_out) {
    if (!costs_ok(costs) || K < 1) return OR_EINVAL;
    int64_t generated = 0;
    dgraph g1, g2;
    int st = dg_build(&g1, n1, vl1, m1, eu1, ev1, el1, directed);
    if (st) return st;
    st = dg_build(&g2, n2, vl2, m2, eu2, ev2, el2, directed);
    if (st) { dg_free(&g1); return st; }

    const size_t width = (size_t)(n1 > 0 ? n1 : 1);
    /* beam: B nodes, each a mapping phi[0..level) and its partial edit distance */
    int64_t B = 1;
    int32_t *phi = (int32_t *)calloc(width, sizeof(int32_t));
    int64_t *ped = (int64_t *)calloc(1, sizeof(int64_t));
    int *used = (int *)calloc((size_t)n2 + 1, sizeof(int));
    if (!phi || !ped || !used) { st = OR_ENOMEM; goto done; }

    for (int i = 0; i < n1; i++) {
        /* branching: every node yields one child per unused g2 vertex, then a
         * deletion child (Sec. 4.2.1); children are listed node by node */
        int64_t cap = B * (int64_t)(n2 + 1);
        int32_t *c_par = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
        int32_t *c_u = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
        rank_key *keys = (rank_key *)malloc(sizeof(rank_key) * (size_t)cap);
        if (!c_par || !c_u || !keys) {
            free(c_par); free(c_u); free(keys);
            st = OR_ENOMEM;
            goto done;
        }
        int64_t C = 0;
        for (int64_t p = 0; p < B; p++) {
            const int32_t *ph = phi + p * width;
            for (int u = 0; u < n2; u++) used[u] = 0;
            for (int j = 0; j < i; j++)
                if (ph[j] != DELETED) used[ph[j]] = 1;
            for (int u = 0; u < n2; u++) {
                if (used[u]) continue;
                c_par[C] = (int32_t)p;
                c_u[C] = u;
                keys[C].ped = ped[p] + sub_step(&g1, &g2, costs, i, u, ph);
                keys[C].order = C;
                C++;
            }
            c_par[C] = (int32_t)p;
            c_u[C] = DELETED;
            keys[C].ped = ped[p] + del_step(&g1, costs, i);
            keys[C].order = C;
            C++;
        }
        generated += C;
        int64_t keep;
        if (last_complete && i == n1 - 1) {
            /* last level, complete-then-minimum: each child's partial edit
             * distance plus its completion; the least total, the first in
             * generation order on ties, is the only child kept */
            int64_t best = INT64_MAX, best_t = 0;
            for (int64_t t = 0; t < C; t++) {
                const int32_t *ph = phi + (int64_t)c_par[t] * width;
                for (int u = 0; u < n2; u++) used[u] = 0;
                for (int j = 0; j < i; j++)
                    if (ph[j] != DELETED) used[ph[j]] = 1;
                if (c_u[t] != DELETED) used[c_u[t]] = 1;
                const int64_t total = keys[t].ped + completion(&g2, costs, used);
                if (total < best) {
                    best = total;
                    best_t = t;
                }
            }
            keys[0] = keys[best_t];
            keep = 1;
        } else {
            /* selection: the K children of least partial edit distance (Sec. 4.3) */
            qsort(keys, (size_t)C, sizeof(rank_key), cmp_rank);
            keep = C < K ? C : K;
        }
        /* the next beam keeps the survivors in generation order */
        qsort(keys, (size_t)keep, sizeof(rank_key), cmp_order);
        int32_t *nphi = (int32_t *)malloc(sizeof(int32_t) * width * (size_t)keep);
        int64_t *nped = (int64_t *)malloc(sizeof(int64_t) * (size_t)keep);
        if (!nphi || !nped) {
            free(nphi); free(nped); free(c_par); free(c_u); free(keys);
            st = OR_ENOMEM;
            goto done;
        }
        for (int64_t s = 0; s < keep; s++) {
            int64_t t = keys[s].order;
            memcpy(nphi + s * width, phi + (int64_t)c_par[t] * width, sizeof(int32_t) * (size_t)i);
            nphi[s * width + i] = c_u[t];
            nped[s] = keys[s].ped;
        }
        free(phi);
        free(ped);
        free(c_par);
        free(c_u);
        free(keys);
        phi = nphi;
        ped = nped;
        B = keep;
    }

    /* completion: insert the unmatched g2 vertices and every g2 edge with an
     * unmatched end (Sec. 4.4.1); return the cheapest leaf, the first one in
     * beam order on ties (Alg. 1) */
    {
        int64_t best = INT64_MAX, best_p = 0;
        for (int64_t p = 0; p < B; p++) {
            const int32_t *ph = phi + p * width;
            for (int u = 0; u < n2; u++) used[u] = 0;
            for (int j = 0; j < n1; j++)
                if (ph[j] != DELETED) used[ph[j]] = 1;
            int64_t total = ped[p] + completion(&g2, costs, used);
            if (total < best) {
                best = total;
                best_p = p;
            }
        }
        *dist = best;
        for (int j = 0; j < n1; j++) map_out[j] = phi[best_p * width + j];
        if (cand_out) *cand_out = generated;
    }
done:
    free(phi);
    free(ped);
    free(used);
    dg_free(&g1);
    dg_free(&g2);
    return st;
}

/* Loop of oracle_kbest over many pairs drawn from concatenated graph arrays
 * (the layout of the workload generator); map_out[map_off[p] ..] gets pair p's
 * mapping, cand_out[p] (cand_out may be NULL) its generated children.
 * Returns the first non-zero status, with *failed_pair set. */
int oracle_kbest_pairs(const int32_t *n, const int32_t *m, const int64_t *voff,
                       const int64_t *eoff, const int32_t *vlabel, const int32_t *eu,
                       const int32_t *ev, const int32_t *elabel, const int64_t *pairs,
                       int64_t npairs, const int32_t *costs, int64_t K, int last_complete, int directed,
                       int64_t *dist, int32_t *map_out, const int64_t *map_off, int64_t *cand_out,
                       int64_t *failed_pair) {
    for (int64_t p = 0; p < npairs; p++) {
        int64_t a = pairs[2 * p], b = pairs[2 * p + 1];
        const int32_t *el_a = elabel ? elabel + eoff[a] : NULL;
        const int32_t *el_b = elabel ? elabel + eoff[b] : NULL;
        int st = oracle_kbest_cand(n[a], vlabel + voff[a], m[a], eu + eoff[a], ev + eoff[a], el_a,
                                   n[b], vlabel + voff[b], m[b], eu + eoff[b], ev + eoff[b], el_b,
                                   costs, K, last_complete, directed, dist + p, map_out + map_off[p],
                                   cand_out ? cand_out + p : NULL);
        if (st) {
            *failed_pair = p;
            return st;
        }
    }
    return OR_OK;
}
