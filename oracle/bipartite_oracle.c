/*
 * bipartite_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded CPU implementation of the bipartite K-best
 * approximation of graph edit distance: a node-assignment cost matrix,
 * the K assignments of least cost enumerated by partitioning the solution
 * space, and the exact induced edit cost of each, the least of which is the
 * distance bound.  It exists to check the GPU library against; nothing in
 * the product path may link or call it.  It shares no code with the GPU
 * library.
 *
 * The paper's own method is the tree search of ged_oracle.c; this variant
 * is not in the paper.  What it uses from the paper: the edit operations
 * and their costs (Sec. 2.2-2.4) and the induced cost of a mapping.  The
 * rest is textbook, restated here:
 *
 *   Cost matrix (Riesen and Bunke's bipartite edit cost): substituting
 *   g1 vertex i by g2 vertex j costs the vertex substitution plus the least
 *   cost of an assignment between the edges incident to i and those
 *   incident to j; deleting i costs the vertex deletion plus the deletion
 *   of its edges; inserting j costs the vertex insertion plus the
 *   insertion of its edges.  The least edge assignment has a closed form
 *   for these costs: with degrees d1, d2, mm = min(d1, d2) and `common` the
 *   number of equal-label pairs (sum over labels of the smaller count),
 *       edel (d1 - mm) + eins (d2 - mm) + min(esub, edel + eins) (mm - common).
 *   The matrix has M = n1 + n2 columns: g2's vertices, then one deletion
 *   column per g1 vertex (vertex i may use only deletion column n2 + i).
 *   Insertion is folded in: a substitution entry is sub(i, j) - ins(j), and
 *   the cost of a mapping is sum_j ins(j) plus its rows' entries.  A
 *   constant D = max_j ins(j) is added to the entries of g1's rows so that
 *   all are non-negative (each such row takes exactly one entry, so the
 *   order of mappings is unchanged).  n2 filler rows of zero cost make the
 *   matrix square: a filler row on a g2 column leaves that vertex to be
 *   inserted, on a deletion column leaves it unused.  Every column is then
 *   always taken, so the potentials of the solver stay valid when an
 *   assignment is removed.  Each vertex mapping is one assignment of g1's
 *   rows; the filler rows' placement never changes the cost.
 *
 *   Assignment solver: the Hungarian method in its shortest-augmenting-path
 *   form with row and column potentials (Kuhn; Munkres; Jonker and
 *   Volgenant).  A row is inserted by a Dijkstra search over reduced costs
 *   from that row; among columns of equal tentative distance the lowest
 *   index is taken.  The first solution inserts rows 0 .. M-1 (g1's rows,
 *   then the filler rows) from zero potentials.
 *
 *   K best assignments (Murty's partitioning over g1's rows, so that no
 *   mapping is found twice): a popped subproblem with solution s and free
 *   (not fixed) g1 rows r_0 < r_1 < ... yields one child
 *   per free row r_t: rows r_0 .. r_{t-1} fixed to their columns in s and
 *   the pair (r_t, s(r_t)) forbidden.  A child is solved from its parent's
 *   potentials and solution with the pair removed and row r_t re-inserted
 *   (one augmenting path; Miller, Stone and Cox).  Subproblems are popped
 *   in order of (assignment cost, creation number); the search stops after
 *   K pops or when none is left.  Each popped mapping is evaluated by its
 *   induced edit cost; the least, first popped among equals, is returned.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { BO_OK = 0, BO_EINVAL = 1, BO_ENOMEM = 2 };

#define BINF ((int64_t)1 << 60)

typedef struct {
    int n;
    const int32_t *vl;
    uint8_t *has;
    int32_t *lab;
    int m;
    int *deg;
} bgraph;

static void bg_free(bgraph *g) {
    free(g->has);
    free(g->lab);
    free(g->deg);
}

static int bg_build(bgraph *g, int n, const int32_t *vl, int m, const int32_t *eu, const int32_t *ev,
                    const int32_t *el) {
    g->n = n;
    g->vl = vl;
    g->m = m;
    size_t nn = (size_t)n * n;
    g->has = (uint8_t *)calloc(nn ? nn : 1, 1);
    g->lab = (int32_t *)calloc(nn ? nn : 1, sizeof(int32_t));
    g->deg = (int *)calloc(n ? n : 1, sizeof(int));
    if (!g->has || !g->lab || !g->deg) return BO_ENOMEM;
    for (int e = 0; e < m; e++) {
        int a = eu[e], b = ev[e];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b || g->has[(size_t)a * n + b]) return BO_EINVAL;
        int32_t l = el ? el[e] : 0;
        g->has[(size_t)a * n + b] = g->has[(size_t)b * n + a] = 1;
        g->lab[(size_t)a * n + b] = g->lab[(size_t)b * n + a] = l;
        g->deg[a]++;
        g->deg[b]++;
    }
    return BO_OK;
}

/* number of pairs (edge at a in g1, edge at b in g2) of equal label that can
 * be matched one to one: sum over labels of the smaller count */
static int common_labels(const bgraph *g1, int a, const bgraph *g2, int b) {
    int total = 0;
    /* labels of a's edges, each matched to an unused equal-label edge of b */
    uint8_t *taken = (uint8_t *)calloc(g2->n ? g2->n : 1, 1);
    if (!taken) return -1;
    for (int x = 0; x < g1->n; x++) {
        if (!g1->has[(size_t)a * g1->n + x]) continue;
        int32_t l = g1->lab[(size_t)a * g1->n + x];
        for (int y = 0; y < g2->n; y++) {
            if (g2->has[(size_t)b * g2->n + y] && !taken[y] && g2->lab[(size_t)b * g2->n + y] == l) {
                taken[y] = 1;
                total++;
                break;
            }
        }
    }
    free(taken);
    return total;
}

typedef struct {
    int n1, n2, M;      /* g1 rows, g2 columns, order of the square matrix (n1 + n2) */
    int64_t *C;         /* g1's rows, n1 x M, BINF where a row may never go; filler rows are 0 */
    int64_t ins_sum;    /* sum_j ins(j) */
    int64_t shift;      /* D */
} bmatrix;

static int build_matrix(const bgraph *g1, const bgraph *g2, const int32_t *c, bmatrix *B) {
    const int n1 = g1->n, n2 = g2->n, M = n1 + n2;
    B->n1 = n1;
    B->n2 = n2;
    B->M = M;
    const size_t cells = (size_t)n1 * (size_t)M;
    B->C = (int64_t *)malloc(sizeof(int64_t) * (cells > 0 ? cells : 1));
    if (!B->C) return BO_ENOMEM;
    int64_t D = 0, sum = 0;
    for (int j = 0; j < n2; j++) {
        int64_t ins = (int64_t)c[2] + (int64_t)c[5] * g2->deg[j];
        sum += ins;
        if (ins > D) D = ins;
    }
    B->ins_sum = sum;
    B->shift = D;
    const int64_t cross = c[3] < (int64_t)c[4] + c[5] ? c[3] : (int64_t)c[4] + c[5];
    for (int i = 0; i < n1; i++) {
        for (int j = 0; j < M; j++) B->C[(size_t)i * M + j] = BINF;
        const int d1 = g1->deg[i];
        for (int j = 0; j < n2; j++) {
            const int d2 = g2->deg[j];
            const int mm = d1 < d2 ? d1 : d2;
            const int com = common_labels(g1, i, g2, j);
            if (com < 0) return BO_ENOMEM;
            int64_t sub = (g1->vl[i] != g2->vl[j]) ? c[0] : 0;
            sub += (int64_t)c[4] * (d1 - mm) + (int64_t)c[5] * (d2 - mm) + cross * (mm - com);
            const int64_t ins = (int64_t)c[2] + (int64_t)c[5] * d2;
            B->C[(size_t)i * M + j] = sub - ins + D;
        }
        B->C[(size_t)i * M + n2 + i] = (int64_t)c[1] + (int64_t)c[4] * d1 + D;
    }
    return BO_OK;
}

/* a subproblem of the partitioning */
typedef struct {
    int64_t cost;       /* rectangular assignment cost (with the shift) */
    int64_t seq;        /* creation number */
    int *fixed;         /* [n1]: fixed column or -1 */
    int nforb;
    int *forb;          /* [2 * nforb]: forbidden (row, column) pairs */
    int64_t *u, *v;     /* potentials [M] (rows), [M] (columns) */
    int *p;             /* [M]: row on each column or -1 */
    int popped;
} bnode;

static void node_free(bnode *x) {
    free(x->fixed);
    free(x->forb);
    free(x->u);
    free(x->v);
    free(x->p);
}

static int64_t entry(const bmatrix *B, int i, int j) { return i < B->n1 ? B->C[(size_t)i * B->M + j] : 0; }

static int allowed(const bmatrix *B, const bnode *x, const int *colfix, int i, int j) {
    if (colfix[j] >= 0 && colfix[j] != i) return 0;
    if (i >= B->n1) return 1;   /* filler rows: any column not fixed to a g1 row */
    if (B->C[(size_t)i * B->M + j] >= BINF) return 0;
    if (x->fixed[i] >= 0 && x->fixed[i] != j) return 0;
    for (int k = 0; k < x->nforb; k++)
        if (x->forb[2 * k] == i && x->forb[2 * k + 1] == j) return 0;
    return 1;
}

/* insert unassigned row r into the assignment x->p with a shortest
 * augmenting path over reduced costs; 0 when no column can take it */
static int augment(const bmatrix *B, bnode *x, int r, int64_t *minv, int *way, uint8_t *used, int *colfix,
                   int64_t *steps) {
    const int M = B->M;
    for (int j = 0; j < M; j++) colfix[j] = -1;
    for (int i = 0; i < B->n1; i++)
        if (x->fixed[i] >= 0) colfix[x->fixed[i]] = i;
    for (int j = 0; j < M; j++) {
        minv[j] = BINF;
        way[j] = -1;
        used[j] = 0;
    }
    int i0 = r, j0 = -1;
    for (;;) {
        ++*steps;
        /* relax the columns from row i0 */
        for (int j = 0; j < M; j++) {
            if (used[j] || !allowed(B, x, colfix, i0, j)) continue;
            int64_t cur = entry(B, i0, j) - x->u[i0] - x->v[j];
            if (cur < minv[j]) {
                minv[j] = cur;
                way[j] = j0;
            }
        }
        /* the unused column of least distance, lowest index first */
        int64_t delta = BINF;
        int j1 = -1;
        for (int j = 0; j < M; j++)
            if (!used[j] && minv[j] < delta) {
                delta = minv[j];
                j1 = j;
            }
        if (j1 < 0) return 0;
        /* potentials: rows and columns of the tree, and the distances */
        x->u[r] += delta;
        for (int j = 0; j < M; j++) {
            if (used[j]) {
                x->u[x->p[j]] += delta;
                x->v[j] -= delta;
            } else if (minv[j] < BINF) {
                minv[j] -= delta;
            }
        }
        used[j1] = 1;
        j0 = j1;
        if (x->p[j1] < 0) break;
        i0 = x->p[j1];
    }
    /* flip the path back to r */
    while (j0 >= 0) {
        int jp = way[j0];
        x->p[j0] = jp < 0 ? r : x->p[jp];
        j0 = jp;
    }
    return 1;
}

static int64_t assignment_cost(const bmatrix *B, const bnode *x) {
    int64_t s = 0;
    for (int j = 0; j < B->M; j++)
        if (x->p[j] >= 0) s += entry(B, x->p[j], j);
    return s;
}

static int node_alloc(bnode *x, int n1, int M, int nforb) {
    memset(x, 0, sizeof *x);
    x->fixed = (int *)malloc(sizeof(int) * (n1 ? n1 : 1));
    x->forb = (int *)malloc(sizeof(int) * (2 * nforb + 2));
    x->u = (int64_t *)malloc(sizeof(int64_t) * (M ? M : 1));
    x->v = (int64_t *)malloc(sizeof(int64_t) * (M ? M : 1));
    x->p = (int *)malloc(sizeof(int) * (M ? M : 1));
    return (x->fixed && x->forb && x->u && x->v && x->p) ? BO_OK : BO_ENOMEM;
}

/* induced edit cost of a mapping (Sec. 2.2-2.4), written out over the
 * dense edge matrices */
static int64_t induced(const bgraph *g1, const bgraph *g2, const int32_t *c, const int32_t *map, int *pre) {
    int64_t cost = 0;
    for (int y = 0; y < g2->n; y++) pre[y] = -1;
    for (int a = 0; a < g1->n; a++) {
        if (map[a] < 0) cost += c[1];
        else {
            pre[map[a]] = a;
            if (g1->vl[a] != g2->vl[map[a]]) cost += c[0];
        }
    }
    for (int y = 0; y < g2->n; y++)
        if (pre[y] < 0) cost += c[2];
    for (int a = 0; a < g1->n; a++)
        for (int b = a + 1; b < g1->n; b++) {
            if (!g1->has[(size_t)a * g1->n + b]) continue;
            int x = map[a], y = map[b];
            if (x < 0 || y < 0 || !g2->has[(size_t)x * g2->n + y]) cost += c[4];
            else if (g1->lab[(size_t)a * g1->n + b] != g2->lab[(size_t)x * g2->n + y]) cost += c[3];
        }
    for (int x = 0; x < g2->n; x++)
        for (int y = x + 1; y < g2->n; y++) {
            if (!g2->has[(size_t)x * g2->n + y]) continue;
            int a = pre[x], b = pre[y];
            if (a < 0 || b < 0 || !g1->has[(size_t)a * g1->n + b]) cost += c[5];
        }
    return cost;
}

/* The bipartite K-best bound of one pair.  dist, map[n1] (-1 = deleted),
 * *solves = assignment problems solved (the first solution counts one).
 * Optional traces of the popped subproblems in pop order: pop_cost[K]
 * (assignment cost in the square form: sum of the chosen substitution and
 * deletion entries plus the insertions of the unused g2 vertices), pop_map
 * [K * n1] and *npop, and *dijkstra_steps: the solver's search steps (each
 * relaxes the n1 + n2 columns from one row), a count of the work done. */
int oracle_bipartite(int n1, const int32_t *vl1, int m1, const int32_t *eu1, const int32_t *ev1,
                     const int32_t *el1, int n2, const int32_t *vl2, int m2, const int32_t *eu2,
                     const int32_t *ev2, const int32_t *el2, const int32_t *costs, int64_t K, int64_t *dist,
                     int32_t *map, int64_t *solves, int64_t *pop_cost, int32_t *pop_map, int64_t *npop,
                     int64_t *dijkstra_steps) {
    if (K < 1 || n1 < 0 || n2 < 0) return BO_EINVAL;
    for (int k = 0; k < 6; k++)
        if (costs[k] < 0) return BO_EINVAL;
    bgraph g1 = {0}, g2 = {0};
    bmatrix B = {0};
    bnode *q = NULL;
    int64_t nq = 0, capq = 0;
    int64_t *minv = NULL;
    int *way = NULL, *colfix = NULL, *pre = NULL, *rows = NULL;
    uint8_t *used = NULL;
    int32_t *cur = NULL;
    int st = bg_build(&g1, n1, vl1, m1, eu1, ev1, el1);
    if (st == BO_OK) st = bg_build(&g2, n2, vl2, m2, eu2, ev2, el2);
    if (st == BO_OK) st = build_matrix(&g1, &g2, costs, &B);
    const int M = n1 + n2;
    if (st == BO_OK) {
        minv = (int64_t *)malloc(sizeof(int64_t) * (M + 1));
        way = (int *)malloc(sizeof(int) * (M + 1));
        colfix = (int *)malloc(sizeof(int) * (M + 1));
        used = (uint8_t *)malloc(M + 1);
        pre = (int *)malloc(sizeof(int) * (n2 + 1));
        rows = (int *)malloc(sizeof(int) * (n1 + 1));
        cur = (int32_t *)malloc(sizeof(int32_t) * (n1 + 1));
        capq = 64;
        q = (bnode *)calloc((size_t)capq, sizeof(bnode));
        if (!minv || !way || !colfix || !used || !pre || !rows || !cur || !q) st = BO_ENOMEM;
    }
    int64_t nsolve = 0, popped = 0, seq = 0, best = BINF, nsteps = 0;
    if (st == BO_OK) {
        /* first solution: rows 0 .. n1-1 from zero potentials (each row's
         * deletion column keeps it feasible) */
        st = node_alloc(&q[0], n1, M, 0);
        if (st == BO_OK) {
            bnode *r = &q[0];
            for (int i = 0; i < n1; i++) r->fixed[i] = -1;
            for (int j = 0; j < M; j++) {
                r->u[j] = 0;
                r->v[j] = 0;
                r->p[j] = -1;
            }
            for (int i = 0; i < M && st == BO_OK; i++)
                if (!augment(&B, r, i, minv, way, used, colfix, &nsteps)) st = BO_EINVAL;   /* cannot happen */
            r->cost = assignment_cost(&B, r);
            r->seq = seq++;
            nq = 1;
            nsolve = 1;
        }
    }
    while (st == BO_OK && popped < K) {
        /* pop the least (cost, creation number) */
        int64_t at = -1;
        for (int64_t k = 0; k < nq; k++) {
            if (q[k].popped) continue;
            if (at < 0 || q[k].cost < q[at].cost || (q[k].cost == q[at].cost && q[k].seq < q[at].seq)) at = k;
        }
        if (at < 0) break;
        q[at].popped = 1;
        /* its mapping and edit cost */
        for (int i = 0; i < n1; i++) cur[i] = -1;
        for (int j = 0; j < n2; j++)
            if (q[at].p[j] >= 0 && q[at].p[j] < n1) cur[q[at].p[j]] = j;
        const int64_t d = induced(&g1, &g2, costs, cur, pre);
        if (pop_cost) pop_cost[popped] = q[at].cost - (int64_t)n1 * B.shift + B.ins_sum;
        if (pop_map) memcpy(pop_map + (size_t)popped * n1, cur, sizeof(int32_t) * n1);
        popped++;
        if (d < best) {
            best = d;
            memcpy(map, cur, sizeof(int32_t) * n1);
        }
        if (popped == K) break;
        /* partition: one child per free row, in ascending row order */
        int nfree = 0;
        int *colof = (int *)malloc(sizeof(int) * (n1 + 1));
        if (!colof) {
            st = BO_ENOMEM;
            break;
        }
        for (int j = 0; j < M; j++)
            if (q[at].p[j] >= 0 && q[at].p[j] < n1) colof[q[at].p[j]] = j;
        for (int i = 0; i < n1; i++)
            if (q[at].fixed[i] < 0) rows[nfree++] = i;
        for (int t = 0; t < nfree && st == BO_OK; t++) {
            if (nq == capq) {
                bnode *g = (bnode *)realloc(q, sizeof(bnode) * (size_t)(capq * 2));
                if (!g) {
                    st = BO_ENOMEM;
                    break;
                }
                q = g;
                capq *= 2;
            }
            bnode *par = &q[at];
            bnode *ch = &q[nq];
            st = node_alloc(ch, n1, M, par->nforb + 1);
            if (st != BO_OK) break;
            memcpy(ch->fixed, par->fixed, sizeof(int) * n1);
            for (int s = 0; s < t; s++) ch->fixed[rows[s]] = colof[rows[s]];
            ch->nforb = par->nforb + 1;
            memcpy(ch->forb, par->forb, sizeof(int) * 2 * par->nforb);
            const int r = rows[t], cr = colof[r];
            ch->forb[2 * par->nforb] = r;
            ch->forb[2 * par->nforb + 1] = cr;
            memcpy(ch->u, par->u, sizeof(int64_t) * M);
            memcpy(ch->v, par->v, sizeof(int64_t) * M);
            memcpy(ch->p, par->p, sizeof(int) * M);
            ch->p[cr] = -1;
            nsolve++;
            if (augment(&B, ch, r, minv, way, used, colfix, &nsteps)) {
                ch->cost = assignment_cost(&B, ch);
                ch->seq = seq++;
                ch->popped = 0;
                nq++;
            } else {
                node_free(ch);
            }
        }
        free(colof);
    }
    if (st == BO_OK) {
        *dist = best;
        *solves = nsolve;
        if (npop) *npop = popped;
        if (dijkstra_steps) *dijkstra_steps = nsteps;
    }
    for (int64_t k = 0; k < nq; k++) node_free(&q[k]);
    free(q);
    free(minv);
    free(way);
    free(colfix);
    free(used);
    free(pre);
    free(rows);
    free(cur);
    free(B.C);
    bg_free(&g1);
    bg_free(&g2);
    return st;
}

/* oracle_bipartite over many pairs of concatenated graph arrays */
int oracle_bipartite_pairs(const int32_t *n, const int32_t *m, const int64_t *voff, const int64_t *eoff,
                           const int32_t *vlabel, const int32_t *eu, const int32_t *ev, const int32_t *elabel,
                           const int64_t *pairs, int64_t npairs, const int32_t *costs, int64_t K, int64_t *dist,
                           int32_t *map_out, const int64_t *map_off, int64_t *solves, int64_t *steps,
                           int64_t *failed_pair) {
    for (int64_t p = 0; p < npairs; p++) {
        int64_t a = pairs[2 * p], b = pairs[2 * p + 1];
        const int32_t *el_a = elabel ? elabel + eoff[a] : NULL;
        const int32_t *el_b = elabel ? elabel + eoff[b] : NULL;
        int st = oracle_bipartite(n[a], vlabel + voff[a], m[a], eu + eoff[a], ev + eoff[a], el_a, n[b],
                                  vlabel + voff[b], m[b], eu + eoff[b], ev + eoff[b], el_b, costs, K, dist + p,
                                  map_out + map_off[p], solves + p, NULL, NULL, NULL, steps ? steps + p : NULL);
        if (st) {
            *failed_pair = p;
            return st;
        }
    }
    return BO_OK;
}
