/*
 * CPU oracle for the refactorization + FGMRES-IR solver of sparse KKT sequences
 * (Swirydowicz et al., "Iterative Methods in GPU-Resident Linear Solvers for Nonlinear
 * Constrained Optimization").
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct reference code: only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * source with the GPU library.  Build: gcc -O2 -ffp-contract=off -fno-fast-math (IEEE
 * binary64 / binary32, round-to-nearest-even, every product and difference rounded
 * separately).
 *
 * Contents (each function cites the passage it follows):
 *   or_order       fill-reducing ordering Q (deterministic BFS nested dissection; the paper
 *                  leaves the ordering to KLU, Section 1.3 / Section 4.1.1)
 *   or_factor      left-looking sparse LU with threshold partial pivoting of K(:,Q): the
 *                  "full symbolic analysis and numerical factorization with pivoting for
 *                  the first system" of Section 1.3
 *   or_refactor    numeric refactorization with the pivot sequence and patterns fixed
 *                  (static pivoting, Section 1.3 and Section 2.1), FP64 or FP32
 *   or_solve       x = Q U^-1 L^-1 P b (the direct solve, Section 1.3 step 3)
 *   or_residual, or_metrics   rho = b - K x, NRBE (eq. (nbre), Section 2.2), NSR (Section 1.3)
 *   or_condest     Hager/Higham 1-norm condition estimate (published method, Higham 1988)
 *   or_fgmres_ir   FGMRES-IR with the LU factors as right preconditioner, CGS2 (or delayed CGS2) Arnoldi,
 *                  estimated residual, solution formed only at restart/convergence
 *                  (Section 2.1, stopping tests of Section 2.2, refine decision of 2.3)
 *   or_richardson  Richardson iterative refinement with MA57's ratio stop (Section 1.3)
 *
 * Where the paper is silent: a refinement that does not converge returns the iterate with the
 * lowest true residual seen (x0 included), and no iterate whose true residual exceeds that of
 * x0 is accepted (NRBE alone is lenient when ||x|| grows).
 *
 * Parity pins (tests under tests/): dense brute force on tiny matrices (same pivot rule),
 * LAPACK getrf agreement with tau = 1 and Q = I, closed-form 2x2 KKT blocks, the
 * backward-error invariant, scipy GMRES with M = I, and the condition number bound.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2
#define OR_ESINGULAR 3

/* ------------------------------------------------------------------------------------ */
/* small helpers                                                                          */
/* ------------------------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

typedef struct {
    int64_t len, cap;
    int32_t *idx;
    double *val;
} vec_t;

static int vec_push(vec_t *v, int32_t i, double x) {
    if (v->len == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        int32_t *ni = (int32_t *)realloc(v->idx, (size_t)nc * sizeof(int32_t));
        if (!ni) return OR_ENOMEM;
        v->idx = ni;
        double *nv = (double *)realloc(v->val, (size_t)nc * sizeof(double));
        if (!nv) return OR_ENOMEM;
        v->val = nv;
        v->cap = nc;
    }
    v->idx[v->len] = i;
    v->val[v->len] = x;
    v->len++;
    return OR_OK;
}

/* Validate a CSR matrix: 0-based, rowptr monotone, columns in range, strictly ascending. */
int or_check_csr(int64_t n, const int64_t *rp, const int32_t *ci) {
    if (n < 1 || rp[0] != 0) return OR_EINVAL;
    for (int64_t i = 0; i < n; i++) {
        if (rp[i + 1] < rp[i]) return OR_EINVAL;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            if (ci[p] < 0 || ci[p] >= n) return OR_EINVAL;
            if (p > rp[i] && ci[p] <= ci[p - 1]) return OR_EINVAL;
        }
    }
    return OR_OK;
}

/* Transpose a CSR matrix into CSC form (column c lists its rows ascending). */
static int csr_to_csc(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                      int64_t **cp_out, int32_t **ri_out, double **cv_out) {
    int64_t nnz = rp[n];
    int64_t *cp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *ri = (int32_t *)malloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
    double *cv = (double *)malloc((size_t)(nnz ? nnz : 1) * sizeof(double));
    int64_t *next = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!cp || !ri || !cv || !next) {
        free(cp); free(ri); free(cv); free(next);
        return OR_ENOMEM;
    }
    for (int64_t p = 0; p < nnz; p++) cp[ci[p] + 1]++;
    for (int64_t c = 0; c < n; c++) cp[c + 1] += cp[c];
    for (int64_t c = 0; c < n; c++) next[c] = cp[c];
    for (int64_t i = 0; i < n; i++)
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            int64_t q = next[ci[p]]++;
            ri[q] = (int32_t)i;
            cv[q] = v ? v[p] : 0.0;
        }
    free(next);
    *cp_out = cp;
    *ri_out = ri;
    *cv_out = cv;
    return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Ordering: nested dissection by BFS level structures.                                   */
/*                                                                                        */
/* Graph: pattern of A + A^T with the diagonal removed.  ND(S):                           */
/*  - |S| <= 64 (the leaf size): S in ascending vertex order.                                             */
/*  - S disconnected in G[S]: ND of each component, components taken in order of their    */
/*    smallest vertex.                                                                    */
/*  - S connected: pseudo-peripheral root (start at the minimum-degree vertex of G[S];    */
/*    BFS; move to the minimum-degree vertex of the deepest level while the eccentricity  */
/*    grows; ties always to the smaller vertex).  Levels L_0..L_e from the root; if e < 2 */
/*    order S ascending.  Separator L_s, s = first level with cumulative size >= |S|/2,   */
/*    clamped to 1..e-1.  Output ND(levels < s), ND(levels > s), separator ascending.     */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int64_t *gp;
    int32_t *gi;
    int32_t *label;  /* id of the set a vertex currently belongs to */
    int32_t next_label;
    int64_t *stamp;  /* BFS visit marks */
    int64_t cur_stamp;
    int32_t *level;
    int32_t *queue;
    int32_t *out;
    int64_t pos;
    int64_t leaf;   /* sets of at most this many vertices are leaves (64 by default) */
} nd_t;

static int build_sym_graph(int64_t n, const int64_t *rp, const int32_t *ci, int64_t **gp_out,
                           int32_t **gi_out) {
    int64_t nnz = rp[n];
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return OR_ENOMEM;
    for (int64_t i = 0; i < n; i++)
        for (int64_t p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] != i) {
                cnt[i + 1]++;
                cnt[ci[p] + 1]++;
            }
    for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    int32_t *tmp = (int32_t *)malloc((size_t)(cnt[n] ? cnt[n] : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!tmp || !fill) {
        free(cnt); free(tmp); free(fill);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < n; i++) fill[i] = cnt[i];
    for (int64_t i = 0; i < n; i++)
        for (int64_t p = rp[i]; p < rp[i + 1]; p++)
            if (ci[p] != i) {
                tmp[fill[i]++] = ci[p];
                tmp[fill[ci[p]]++] = (int32_t)i;
            }
    /* sort and deduplicate each adjacency list */
    int64_t *gp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!gp) {
        free(cnt); free(tmp); free(fill);
        return OR_ENOMEM;
    }
    int64_t w = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t *a = tmp + cnt[i];
        int64_t len = cnt[i + 1] - cnt[i];
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
        gp[i] = w;
        for (int64_t t = 0; t < len; t++)
            if (t == 0 || a[t] != a[t - 1]) tmp[w++] = a[t];
    }
    gp[n] = w;
    free(cnt);
    free(fill);
    *gp_out = gp;
    *gi_out = tmp; /* compacted in place; tail unused */
    (void)nnz;
    return OR_OK;
}

static int64_t deg_in_set(nd_t *c, int32_t v, int32_t id) {
    int64_t d = 0;
    for (int64_t p = c->gp[v]; p < c->gp[v + 1]; p++)
        if (c->label[c->gi[p]] == id) d++;
    return d;
}

/* BFS from root inside set `id`; fills c->queue[0..cnt) in level order and c->level.
   Returns the eccentricity; *cnt_out = number of vertices reached. */
static int32_t bfs_levels(nd_t *c, int32_t root, int32_t id, int64_t *cnt_out) {
    c->cur_stamp++;
    int64_t head = 0, tail = 0;
    c->queue[tail++] = root;
    c->stamp[root] = c->cur_stamp;
    c->level[root] = 0;
    int32_t ecc = 0;
    while (head < tail) {
        int32_t v = c->queue[head++];
        for (int64_t p = c->gp[v]; p < c->gp[v + 1]; p++) {
            int32_t u = c->gi[p];
            if (c->label[u] != id || c->stamp[u] == c->cur_stamp) continue;
            c->stamp[u] = c->cur_stamp;
            c->level[u] = c->level[v] + 1;
            if (c->level[u] > ecc) ecc = c->level[u];
            c->queue[tail++] = u;
        }
    }
    *cnt_out = tail;
    return ecc;
}

static void emit_sorted(nd_t *c, int32_t *S, int64_t s) {
    qsort(S, (size_t)s, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < s; t++) c->out[c->pos++] = S[t];
}

static int nd_rec(nd_t *c, int32_t *S, int64_t s, int32_t id) {
    if (s <= c->leaf) {
        emit_sorted(c, S, s);
        return OR_OK;
    }
    qsort(S, (size_t)s, sizeof(int32_t), cmp_i32);
    /* connected components of G[S], in order of their smallest vertex */
    int64_t cnt;
    bfs_levels(c, S[0], id, &cnt);
    if (cnt < s) {
        int32_t *comp = (int32_t *)malloc((size_t)s * sizeof(int32_t));
        int64_t *cstart = (int64_t *)malloc((size_t)(s + 1) * sizeof(int64_t));
        if (!comp || !cstart) {
            free(comp); free(cstart);
            return OR_ENOMEM;
        }
        /* mark with one stamp, collecting components in ascending-smallest-vertex order */
        c->cur_stamp++;
        int64_t seen_stamp = c->cur_stamp;
        int64_t w = 0, ncomp = 0;
        for (int64_t t = 0; t < s; t++) {
            int32_t r = S[t];
            if (c->stamp[r] == seen_stamp) continue;
            cstart[ncomp++] = w;
            int64_t head = w;
            comp[w++] = r;
            c->stamp[r] = seen_stamp;
            while (head < w) {
                int32_t v = comp[head++];
                for (int64_t p = c->gp[v]; p < c->gp[v + 1]; p++) {
                    int32_t u = c->gi[p];
                    if (c->label[u] != id || c->stamp[u] == seen_stamp) continue;
                    c->stamp[u] = seen_stamp;
                    comp[w++] = u;
                }
            }
        }
        cstart[ncomp] = w;
        int rc = OR_OK;
        for (int64_t k = 0; k < ncomp && rc == OR_OK; k++) {
            int32_t nid = c->next_label++;
            for (int64_t t = cstart[k]; t < cstart[k + 1]; t++) c->label[comp[t]] = nid;
            rc = nd_rec(c, comp + cstart[k], cstart[k + 1] - cstart[k], nid);
        }
        free(comp);
        free(cstart);
        return rc;
    }
    /* pseudo-peripheral root */
    int32_t root = -1;
    int64_t best = INT64_MAX;
    for (int64_t t = 0; t < s; t++) { /* S ascending: strict < keeps the smallest index */
        int64_t d = deg_in_set(c, S[t], id);
        if (d < best) {
            best = d;
            root = S[t];
        }
    }
    int32_t ecc = bfs_levels(c, root, id, &cnt);
    for (;;) {
        int32_t cand = -1;
        int64_t bd = INT64_MAX;
        for (int64_t t = 0; t < cnt; t++) {
            int32_t v = c->queue[t];
            if (c->level[v] != ecc) continue;
            int64_t d = deg_in_set(c, v, id);
            if (d < bd || (d == bd && v < cand)) {
                bd = d;
                cand = v;
            }
        }
        int64_t cnt2;
        int32_t ecc2 = bfs_levels(c, cand, id, &cnt2);
        if (ecc2 > ecc) {
            root = cand;
            ecc = ecc2;
            cnt = cnt2;
        } else {
            break;
        }
    }
    ecc = bfs_levels(c, root, id, &cnt);
    if (ecc < 2) {
        emit_sorted(c, S, s);
        return OR_OK;
    }
    int64_t *lsize = (int64_t *)calloc((size_t)ecc + 1, sizeof(int64_t));
    if (!lsize) return OR_ENOMEM;
    for (int64_t t = 0; t < s; t++) lsize[c->level[S[t]]]++;
    int64_t cum = 0;
    int32_t sl = 0;
    for (int32_t t = 0; t <= ecc; t++) {
        cum += lsize[t];
        if (2 * cum >= s) {
            sl = t;
            break;
        }
    }
    if (sl < 1) sl = 1;
    if (sl > ecc - 1) sl = ecc - 1;
    free(lsize);
    int32_t *part = (int32_t *)malloc((size_t)s * sizeof(int32_t));
    if (!part) return OR_ENOMEM;
    int64_t na = 0, nb = 0, ns = 0;
    for (int64_t t = 0; t < s; t++)
        if (c->level[S[t]] < sl) na++;
        else if (c->level[S[t]] > sl) nb++;
    int64_t ia = 0, ib = na, is = na + nb;
    for (int64_t t = 0; t < s; t++) {
        int32_t v = S[t];
        int32_t l = c->level[v];
        if (l < sl) part[ia++] = v;
        else if (l > sl) part[ib++] = v;
        else part[is++] = v;
    }
    ns = s - na - nb;
    int32_t ida = c->next_label++;
    for (int64_t t = 0; t < na; t++) c->label[part[t]] = ida;
    int32_t idb = c->next_label++;
    for (int64_t t = na; t < na + nb; t++) c->label[part[t]] = idb;
    int32_t ids = c->next_label++;
    for (int64_t t = na + nb; t < s; t++) c->label[part[t]] = ids;
    int rc = nd_rec(c, part, na, ida);
    if (rc == OR_OK) rc = nd_rec(c, part + na, nb, idb);
    if (rc == OR_OK) emit_sorted(c, part + na + nb, ns);
    free(part);
    return rc;
}

/* Q[j] = original column eliminated at step j.  leaf >= 1 (the spec uses 64). */
int or_order_leaf(int64_t n, const int64_t *rp, const int32_t *ci, int64_t leaf, int32_t *Q) {
    if (or_check_csr(n, rp, ci) != OR_OK || leaf < 1) return OR_EINVAL;
    nd_t c;
    memset(&c, 0, sizeof(c));
    c.n = n;
    c.leaf = leaf;
    int rc = build_sym_graph(n, rp, ci, &c.gp, &c.gi);
    if (rc != OR_OK) return rc;
    c.label = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    c.stamp = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    c.level = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    c.queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *S = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    c.out = Q;
    c.next_label = 1;
    if (!c.label || !c.stamp || !c.level || !c.queue || !S) {
        rc = OR_ENOMEM;
    } else {
        for (int64_t v = 0; v < n; v++) S[v] = (int32_t)v;
        rc = nd_rec(&c, S, n, 0);
        if (rc == OR_OK && c.pos != n) rc = OR_EINVAL;
    }
    free(c.gp); free(c.gi); free(c.label); free(c.stamp); free(c.level); free(c.queue); free(S);
    return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Ordering: exact minimum degree on the elimination graph.                               */
/*                                                                                        */
/* Graph: pattern of A + A^T without the diagonal.  Repeat n times: eliminate the vertex  */
/* of least current degree (ties: smallest original index); its neighbours become a      */
/* clique (the fill of symmetric elimination) and lose it as a neighbour.  Written on    */
/* the explicit elimination graph with sorted adjacency arrays.                          */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int64_t deg;
    int32_t v;
} md_item;

static int md_less(md_item a, md_item b) { return a.deg < b.deg || (a.deg == b.deg && a.v < b.v); }

static void md_push(md_item *h, int64_t *hn, md_item x) {
    int64_t i = (*hn)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!md_less(h[i], h[p])) break;
        md_item t = h[i];
        h[i] = h[p];
        h[p] = t;
        i = p;
    }
}

static md_item md_pop(md_item *h, int64_t *hn) {
    md_item top = h[0];
    h[0] = h[--(*hn)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *hn && md_less(h[l], h[m])) m = l;
        if (r < *hn && md_less(h[r], h[m])) m = r;
        if (m == i) break;
        md_item t = h[i];
        h[i] = h[m];
        h[m] = t;
        i = m;
    }
    return top;
}

int or_order_md(int64_t n, const int64_t *rp, const int32_t *ci, int32_t *Q) {
    if (or_check_csr(n, rp, ci) != OR_OK) return OR_EINVAL;
    int64_t *gp;
    int32_t *gi;
    int rc = build_sym_graph(n, rp, ci, &gp, &gi);
    if (rc != OR_OK) return rc;
    int32_t **adj = (int32_t **)calloc((size_t)n, sizeof(int32_t *));
    int64_t *len = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *cap = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    char *gone = (char *)calloc((size_t)n, 1);
    int64_t hcap = 4 * n + 16, hn = 0;
    md_item *heap = (md_item *)malloc((size_t)hcap * sizeof(md_item));
    int32_t *merged = NULL;
    int64_t mcap = 0;
    if (!adj || !len || !cap || !gone || !heap) {
        rc = OR_ENOMEM;
        goto done;
    }
    for (int64_t v = 0; v < n; v++) {
        len[v] = gp[v + 1] - gp[v];
        cap[v] = len[v] + 4;
        adj[v] = (int32_t *)malloc((size_t)cap[v] * sizeof(int32_t));
        if (!adj[v]) {
            rc = OR_ENOMEM;
            goto done;
        }
        memcpy(adj[v], gi + gp[v], (size_t)len[v] * sizeof(int32_t));
        md_item it = {len[v], (int32_t)v};
        md_push(heap, &hn, it);
    }
    for (int64_t step = 0; step < n; step++) {
        md_item it;
        do {
            it = md_pop(heap, &hn);
        } while (gone[it.v] || it.deg != len[it.v]);
        int32_t p = it.v;
        Q[step] = p;
        gone[p] = 1;
        /* neighbours of p (all alive, sorted) become a clique */
        int32_t *nb = adj[p];
        int64_t nn = len[p];
        for (int64_t a = 0; a < nn; a++) {
            int32_t u = nb[a];
            /* new adjacency of u: (adj[u] \ {p}) U (nb \ {u}), sorted merge */
            int64_t need = len[u] + nn;
            if (need > mcap) {
                mcap = 2 * need;
                int32_t *t = (int32_t *)realloc(merged, (size_t)mcap * sizeof(int32_t));
                if (!t) {
                    rc = OR_ENOMEM;
                    goto done;
                }
                merged = t;
            }
            int64_t x = 0, y = 0, w = 0;
            int32_t *au = adj[u];
            while (x < len[u] || y < nn) {
                int32_t c;
                if (y >= nn || (x < len[u] && au[x] < nb[y])) c = au[x++];
                else if (x >= len[u] || nb[y] < au[x]) c = nb[y++];
                else {
                    c = au[x];
                    x++;
                    y++;
                }
                if (c == p || c == u) continue;
                merged[w++] = c;
            }
            if (w > cap[u]) {
                int32_t *t = (int32_t *)realloc(adj[u], (size_t)(2 * w) * sizeof(int32_t));
                if (!t) {
                    rc = OR_ENOMEM;
                    goto done;
                }
                adj[u] = t;
                cap[u] = 2 * w;
            }
            memcpy(adj[u], merged, (size_t)w * sizeof(int32_t));
            len[u] = w;
            if (hn == hcap) {
                hcap *= 2;
                md_item *t = (md_item *)realloc(heap, (size_t)hcap * sizeof(md_item));
                if (!t) {
                    rc = OR_ENOMEM;
                    goto done;
                }
                heap = t;
            }
            md_item ni = {w, u};
            md_push(heap, &hn, ni);
        }
        free(adj[p]);
        adj[p] = NULL;
        len[p] = 0;
    }
done:
    if (adj)
        for (int64_t v = 0; v < n; v++) free(adj[v]);
    free(adj); free(len); free(cap); free(gone); free(heap); free(merged); free(gp); free(gi);
    return rc;
}

/* Default ordering (minimum degree); or_order_leaf gives the nested dissection. */
int or_order(int64_t n, const int64_t *rp, const int32_t *ci, int32_t *Q) {
    return or_order_md(n, rp, ci, Q);
}

/* ------------------------------------------------------------------------------------ */
/* Pivoted sparse LU (left-looking, one column at a time) of A(:,Q).                      */
/*                                                                                        */
/* Column j (c = Q[j]):                                                                   */
/*  1. x = A(:,c), indexed by original row.                                               */
/*  2. Structural closure: starting from the rows of A(:,c), a pivoted row r (pivot step   */
/*     k) brings in every row of L(:,k).  Reached steps = pattern of U(:,j) above the      */
/*     diagonal; reached unpivoted rows = candidates.                                      */
/*  3. For the reached steps k in ascending order: u_kj = x[prow(k)]; then                */
/*     x[i] = x[i] - L(i,k) * u_kj for i in L(:,k)  (product and difference rounded        */
/*     separately).                                                                        */
/*  4. Pivot among the candidates: amax = max |x_i|; take the diagonal row c when it is a  */
/*     candidate and |x_c| >= tau * amax, else the largest |x_i| (ties: smallest row).     */
/*     amax == 0 or no candidate: structurally/numerically singular column j.             */
/*  5. U(j,j) = x[piv]; L(i,j) = x[i] / U(j,j) for the other candidates (kept even when    */
/*     zero: the patterns are structural).                                                 */
/* L(:,j) lists original rows ascending; U(:,j) lists steps ascending, diagonal last.      */
/* ------------------------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int64_t *Lp;
    int32_t *Li; /* original row indices */
    double *Lx;
    int64_t *Up;
    int32_t *Ui; /* pivot steps */
    double *Ux;
    int32_t *prow; /* prow[k] = original row pivoted at step k */
    int32_t *pinv; /* pinv[row] = step */
    int32_t *Q;    /* Q[k] = original column of step k */
} or_lu_t;

void or_free(or_lu_t *f) {
    if (!f) return;
    free(f->Lp); free(f->Li); free(f->Lx);
    free(f->Up); free(f->Ui); free(f->Ux);
    free(f->prow); free(f->pinv); free(f->Q);
    free(f);
}

or_lu_t *or_factor(int64_t n, const int64_t *rp, const int32_t *ci, const double *vals,
                   const int32_t *Q, double tau, int *status, int64_t *bad_col) {
    *status = OR_OK;
    *bad_col = -1;
    if (or_check_csr(n, rp, ci) != OR_OK) {
        *status = OR_EINVAL;
        return NULL;
    }
    int64_t *cp;
    int32_t *ri;
    double *cv;
    if (csr_to_csc(n, rp, ci, vals, &cp, &ri, &cv) != OR_OK) {
        *status = OR_ENOMEM;
        return NULL;
    }
    or_lu_t *f = (or_lu_t *)calloc(1, sizeof(or_lu_t));
    double *x = (double *)calloc((size_t)n, sizeof(double));
    int64_t *mark = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t *stack = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *reach = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *cand = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    vec_t L = {0, 0, NULL, NULL}, U = {0, 0, NULL, NULL};
    int rc = OR_OK;
    if (!f || !x || !mark || !stack || !reach || !cand) {
        rc = OR_ENOMEM;
        goto done;
    }
    f->n = n;
    f->Lp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    f->Up = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    f->prow = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    f->pinv = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    f->Q = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!f->Lp || !f->Up || !f->prow || !f->pinv || !f->Q) {
        rc = OR_ENOMEM;
        goto done;
    }
    memcpy(f->Q, Q, (size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) {
        f->pinv[i] = -1;
        mark[i] = -1;
    }
    for (int64_t j = 0; j < n; j++) {
        int32_t c = Q[j];
        if (c < 0 || c >= n) {
            rc = OR_EINVAL;
            goto done;
        }
        int64_t nreach = 0, ncand = 0, top = 0;
        /* each row enters the stack at most once (marked when pushed) */
        for (int64_t p = cp[c]; p < cp[c + 1]; p++) {
            x[ri[p]] = cv[p];
            mark[ri[p]] = j;
            stack[top++] = ri[p];
        }
        while (top > 0) {
            int32_t r = stack[--top];
            int32_t k = f->pinv[r];
            if (k >= 0) {
                reach[nreach++] = k;
                for (int64_t q = f->Lp[k]; q < f->Lp[k + 1]; q++)
                    if (mark[L.idx[q]] != j) {
                        mark[L.idx[q]] = j;
                        stack[top++] = L.idx[q];
                    }
            } else {
                cand[ncand++] = r;
            }
        }
        qsort(reach, (size_t)nreach, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < nreach; t++) {
            int32_t k = reach[t];
            double u = x[f->prow[k]];
            if ((rc = vec_push(&U, k, u)) != OR_OK) goto done;
            for (int64_t q = f->Lp[k]; q < f->Lp[k + 1]; q++) {
                double prod = L.val[q] * u;
                x[L.idx[q]] = x[L.idx[q]] - prod;
            }
        }
        qsort(cand, (size_t)ncand, sizeof(int32_t), cmp_i32);
        double amax = 0.0;
        int32_t piv = -1;
        for (int64_t t = 0; t < ncand; t++) {
            double a = fabs(x[cand[t]]);
            if (a > amax) { /* strict: ties keep the smaller row */
                amax = a;
                piv = cand[t];
            }
        }
        if (ncand == 0 || !(amax > 0.0)) {
            rc = OR_ESINGULAR;
            *bad_col = j;
            goto done;
        }
        if (mark[c] == j && f->pinv[c] < 0 && fabs(x[c]) >= tau * amax) piv = c;
        double ujj = x[piv];
        if ((rc = vec_push(&U, (int32_t)j, ujj)) != OR_OK) goto done;
        f->Up[j + 1] = U.len;
        f->prow[j] = piv;
        f->pinv[piv] = (int32_t)j;
        for (int64_t t = 0; t < ncand; t++) {
            int32_t r = cand[t];
            if (r == piv) continue;
            if ((rc = vec_push(&L, r, x[r] / ujj)) != OR_OK) goto done;
        }
        f->Lp[j + 1] = L.len;
        for (int64_t t = 0; t < ncand; t++) x[cand[t]] = 0.0;
        for (int64_t t = 0; t < nreach; t++) x[f->prow[reach[t]]] = 0.0;
    }
done:
    free(cp); free(ri); free(cv);
    free(x); free(mark); free(stack); free(reach); free(cand);
    if (rc != OR_OK) {
        free(L.idx); free(L.val); free(U.idx); free(U.val);
        or_free(f);
        *status = rc;
        return NULL;
    }
    f->Li = L.idx; f->Lx = L.val;
    f->Ui = U.idx; f->Ux = U.val;
    if (!f->Li) { f->Li = (int32_t *)malloc(sizeof(int32_t)); f->Lx = (double *)malloc(sizeof(double)); }
    return f;
}

void or_lu_sizes(const or_lu_t *f, int64_t *lnz, int64_t *unz) {
    *lnz = f->Lp[f->n];
    *unz = f->Up[f->n];
}

void or_lu_export(const or_lu_t *f, int64_t *Lp, int32_t *Li, double *Lx, int64_t *Up, int32_t *Ui,
                  double *Ux, int32_t *prow, int32_t *Q) {
    int64_t n = f->n;
    if (Lp) memcpy(Lp, f->Lp, (size_t)(n + 1) * sizeof(int64_t));
    if (Li) memcpy(Li, f->Li, (size_t)f->Lp[n] * sizeof(int32_t));
    if (Lx) memcpy(Lx, f->Lx, (size_t)f->Lp[n] * sizeof(double));
    if (Up) memcpy(Up, f->Up, (size_t)(n + 1) * sizeof(int64_t));
    if (Ui) memcpy(Ui, f->Ui, (size_t)f->Up[n] * sizeof(int32_t));
    if (Ux) memcpy(Ux, f->Ux, (size_t)f->Up[n] * sizeof(double));
    if (prow) memcpy(prow, f->prow, (size_t)n * sizeof(int32_t));
    if (Q) memcpy(Q, f->Q, (size_t)n * sizeof(int32_t));
}

/* ------------------------------------------------------------------------------------ */
/* Static-pivot refactorization (pivot sequence and patterns fixed by or_factor).         */
/* Same left-looking column loop and operation order as or_factor, with no search and no  */
/* pivot choice.  Tiny-pivot guard (the paper is silent on it): when |u_jj| <=            */
/* u * max_i |A(i,Q[j])| (u = unit roundoff of the working precision) or u_jj is not      */
/* finite, u_jj is replaced by sign(u_jj) * u * colmax (sign +1 for zero/NaN; colmax      */
/* taken as 1 for an all-zero column) and counted; guard_policy 1 reports ESINGULAR.      */
/* ------------------------------------------------------------------------------------ */

int or_refactor64(const or_lu_t *f, const int64_t *rp, const int32_t *ci, const double *vals,
                  int guard_policy, double *Lx, double *Ux, int64_t *nguard, int64_t *bad_col) {
    int64_t n = f->n;
    int64_t *cp;
    int32_t *ri;
    double *cv;
    *nguard = 0;
    *bad_col = -1;
    if (csr_to_csc(n, rp, ci, vals, &cp, &ri, &cv) != OR_OK) return OR_ENOMEM;
    double *x = (double *)calloc((size_t)n, sizeof(double));
    if (!x) {
        free(cp); free(ri); free(cv);
        return OR_ENOMEM;
    }
    const double ur = ldexp(1.0, -53);
    int rc = OR_OK;
    for (int64_t j = 0; j < n && rc == OR_OK; j++) {
        int32_t c = f->Q[j];
        double colmax = 0.0;
        for (int64_t p = cp[c]; p < cp[c + 1]; p++) {
            x[ri[p]] = cv[p];
            if (fabs(cv[p]) > colmax) colmax = fabs(cv[p]);
        }
        int64_t ud = f->Up[j + 1] - 1; /* diagonal position */
        for (int64_t p = f->Up[j]; p < ud; p++) {
            int32_t k = f->Ui[p];
            double u = x[f->prow[k]];
            Ux[p] = u;
            for (int64_t q = f->Lp[k]; q < f->Lp[k + 1]; q++) {
                double prod = Lx[q] * u;
                x[f->Li[q]] = x[f->Li[q]] - prod;
            }
        }
        double ujj = x[f->prow[j]];
        double cm = colmax > 0.0 ? colmax : 1.0;
        if (!(fabs(ujj) > ur * cm) || !isfinite(ujj)) {
            if (guard_policy == 1) {
                rc = OR_ESINGULAR;
                *bad_col = j;
                break;
            }
            ujj = (ujj < 0.0 ? -1.0 : 1.0) * ur * cm;
            (*nguard)++;
        }
        Ux[ud] = ujj;
        for (int64_t q = f->Lp[j]; q < f->Lp[j + 1]; q++) Lx[q] = x[f->Li[q]] / ujj;
        for (int64_t q = f->Lp[j]; q < f->Lp[j + 1]; q++) x[f->Li[q]] = 0.0;
        for (int64_t p = f->Up[j]; p <= ud; p++) x[f->prow[f->Ui[p]]] = 0.0;
    }
    free(x); free(cp); free(ri); free(cv);
    return rc;
}

int or_refactor32(const or_lu_t *f, const int64_t *rp, const int32_t *ci, const double *vals,
                  int guard_policy, float *Lx, float *Ux, int64_t *nguard, int64_t *bad_col) {
    int64_t n = f->n;
    int64_t *cp;
    int32_t *ri;
    double *cv;
    *nguard = 0;
    *bad_col = -1;
    if (csr_to_csc(n, rp, ci, vals, &cp, &ri, &cv) != OR_OK) return OR_ENOMEM;
    float *x = (float *)calloc((size_t)n, sizeof(float));
    if (!x) {
        free(cp); free(ri); free(cv);
        return OR_ENOMEM;
    }
    const float ur = ldexpf(1.0f, -24);
    int rc = OR_OK;
    for (int64_t j = 0; j < n && rc == OR_OK; j++) {
        int32_t c = f->Q[j];
        float colmax = 0.0f;
        for (int64_t p = cp[c]; p < cp[c + 1]; p++) {
            float a = (float)cv[p];
            x[ri[p]] = a;
            if (fabsf(a) > colmax) colmax = fabsf(a);
        }
        int64_t ud = f->Up[j + 1] - 1;
        for (int64_t p = f->Up[j]; p < ud; p++) {
            int32_t k = f->Ui[p];
            float u = x[f->prow[k]];
            Ux[p] = u;
            for (int64_t q = f->Lp[k]; q < f->Lp[k + 1]; q++) {
                float prod = Lx[q] * u;
                x[f->Li[q]] = x[f->Li[q]] - prod;
            }
        }
        float ujj = x[f->prow[j]];
        float cm = colmax > 0.0f ? colmax : 1.0f;
        if (!(fabsf(ujj) > ur * cm) || !isfinite(ujj)) {
            if (guard_policy == 1) {
                rc = OR_ESINGULAR;
                *bad_col = j;
                break;
            }
            ujj = (ujj < 0.0f ? -1.0f : 1.0f) * ur * cm;
            (*nguard)++;
        }
        Ux[ud] = ujj;
        for (int64_t q = f->Lp[j]; q < f->Lp[j + 1]; q++) Lx[q] = x[f->Li[q]] / ujj;
        for (int64_t q = f->Lp[j]; q < f->Lp[j + 1]; q++) x[f->Li[q]] = 0.0f;
        for (int64_t p = f->Up[j]; p <= ud; p++) x[f->prow[f->Ui[p]]] = 0.0f;
    }
    free(x); free(cp); free(ri); free(cv);
    return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Direct solve with given factor values: x = Q U^-1 L^-1 P b (column sweeps).            */
/* ------------------------------------------------------------------------------------ */

int or_solve_with(const or_lu_t *f, const double *Lx, const double *Ux, const double *b, double *x) {
    int64_t n = f->n;
    double *w = (double *)malloc((size_t)n * sizeof(double)); /* by original row */
    double *z = (double *)malloc((size_t)n * sizeof(double)); /* by step */
    if (!w || !z) {
        free(w); free(z);
        return OR_ENOMEM;
    }
    memcpy(w, b, (size_t)n * sizeof(double));
    for (int64_t k = 0; k < n; k++) {
        double yk = w[f->prow[k]];
        z[k] = yk;
        for (int64_t q = f->Lp[k]; q < f->Lp[k + 1]; q++) {
            double prod = Lx[q] * yk;
            w[f->Li[q]] = w[f->Li[q]] - prod;
        }
    }
    for (int64_t j = n - 1; j >= 0; j--) {
        int64_t ud = f->Up[j + 1] - 1;
        double zj = z[j] / Ux[ud];
        z[j] = zj;
        for (int64_t p = f->Up[j]; p < ud; p++) {
            double prod = Ux[p] * zj;
            z[f->Ui[p]] = z[f->Ui[p]] - prod;
        }
    }
    for (int64_t j = 0; j < n; j++) x[f->Q[j]] = z[j];
    free(w); free(z);
    return OR_OK;
}

/* The same solve carried out in binary32 on FP32 factors (input and output FP64). */
int or_solve_with32(const or_lu_t *f, const float *Lx, const float *Ux, const double *b, double *x) {
    int64_t n = f->n;
    float *w = (float *)malloc((size_t)n * sizeof(float));
    float *z = (float *)malloc((size_t)n * sizeof(float));
    if (!w || !z) {
        free(w); free(z);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < n; i++) w[i] = (float)b[i];
    for (int64_t k = 0; k < n; k++) {
        float yk = w[f->prow[k]];
        z[k] = yk;
        for (int64_t q = f->Lp[k]; q < f->Lp[k + 1]; q++) {
            float prod = Lx[q] * yk;
            w[f->Li[q]] = w[f->Li[q]] - prod;
        }
    }
    for (int64_t j = n - 1; j >= 0; j--) {
        int64_t ud = f->Up[j + 1] - 1;
        float zj = z[j] / Ux[ud];
        z[j] = zj;
        for (int64_t p = f->Up[j]; p < ud; p++) {
            float prod = Ux[p] * zj;
            z[f->Ui[p]] = z[f->Ui[p]] - prod;
        }
    }
    for (int64_t j = 0; j < n; j++) x[f->Q[j]] = (double)z[j];
    free(w); free(z);
    return OR_OK;
}

int or_solve(const or_lu_t *f, const double *b, double *x) { return or_solve_with(f, f->Lx, f->Ux, b, x); }

/* ------------------------------------------------------------------------------------ */
/* Residual and error measures.                                                           */
/* ------------------------------------------------------------------------------------ */

/* rho = b - K x; each row's products summed in ascending column order, then subtracted. */
void or_residual(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                 const double *b, double *r) {
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            double prod = v[p] * x[ci[p]];
            s = s + prod;
        }
        r[i] = b[i] - s;
    }
}

/* Extended-precision residual (the higher-precision residual of iterative refinement,     */
/* Section 2): each row's sum b_i - sum_p v_p x_c is carried as an unevaluated pair of     */
/* doubles (hi + lo) and rounded to double once at the end.                                */
/*   two_sum:  Knuth's error-free sum, s + e = a + b exactly.                               */
/*   fast_two_sum: Dekker's version, valid when |a| >= |b| or a = 0.                         */
/*   two_prod: p + e = a * b exactly, e from one fused multiply-add.                         */
/*   dw_add: double-word + double-word, the accurate algorithm of Joldes, Muller and        */
/*           Popescu (ACM TOMS 2017, Algorithm 6), relative error <= 3 u^2.                 */
/* Row order: start from (b_i, 0), then add (-p_hi, -p_lo) of each product in CSR order.    */
static void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

static void fast_two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    *e = b - (x - a);
    *s = x;
}

static void two_prod(double a, double b, double *p, double *e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

static void dw_add(double xh, double xl, double yh, double yl, double *zh, double *zl) {
    double sh, sl, th, tl, vh, vl;
    two_sum(xh, yh, &sh, &sl);
    two_sum(xl, yl, &th, &tl);
    double c = sl + th;
    fast_two_sum(sh, c, &vh, &vl);
    double w = tl + vl;
    fast_two_sum(vh, w, zh, zl);
}

void or_residual_dd(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                    const double *b, double *r) {
    for (int64_t i = 0; i < n; i++) {
        double hi = b[i], lo = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            double ph, pl;
            two_prod(v[p], x[ci[p]], &ph, &pl);
            dw_add(hi, lo, -ph, -pl, &hi, &lo);
        }
        r[i] = hi;
    }
}

double or_norm_inf_mat(int64_t n, const int64_t *rp, const double *v) {
    double m = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) s = s + fabs(v[p]);
        if (s > m) m = s;
    }
    return m;
}

static double nrm2(int64_t n, const double *a) {
    /* scaled sum of squares: no overflow/underflow for any finite input */
    double scale = 0.0, ssq = 1.0;
    for (int64_t i = 0; i < n; i++) {
        if (a[i] != 0.0) {
            double t = fabs(a[i]);
            if (scale < t) {
                ssq = 1.0 + ssq * (scale / t) * (scale / t);
                scale = t;
            } else {
                ssq = ssq + (t / scale) * (t / scale);
            }
        }
    }
    return scale * sqrt(ssq);
}

static double nrminf(int64_t n, const double *a) {
    double m = 0.0;
    for (int64_t i = 0; i < n; i++)
        if (fabs(a[i]) > m) m = fabs(a[i]);
    return m;
}

/* out[0] = NRBE = ||rho||_2 / (||K||_inf ||x||_2 + ||b||_2)      (eq. (nbre))
   out[1] = NSR  = ||rho||_inf / (||K||_inf ||x||_inf)             (MA57's measure, Section 1.3)
   out[2] = ||rho||_2, out[3] = ||K||_inf, out[4] = ||x||_2, out[5] = ||b||_2,
   out[6] = ||rho||_2 / ||b||_2  (the refine test of Section 2.3)                          */
int or_metrics(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
               const double *b, double *out) {
    double *r = (double *)malloc((size_t)n * sizeof(double));
    if (!r) return OR_ENOMEM;
    or_residual(n, rp, ci, v, x, b, r);
    double rn = nrm2(n, r), kn = or_norm_inf_mat(n, rp, v), xn = nrm2(n, x), bn = nrm2(n, b);
    out[0] = rn / (kn * xn + bn);
    out[1] = nrminf(n, r) / (kn * nrminf(n, x));
    out[2] = rn;
    out[3] = kn;
    out[4] = xn;
    out[5] = bn;
    out[6] = rn / bn;
    free(r);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* 1-norm condition estimate kappa_1 ~ ||K||_1 * est ||K^-1||_1.                          */
/* Hager's method as refined by Higham (ACM TOMS 14, 1988, "FORTRAN codes for estimating  */
/* the one-norm of a real or complex matrix"): power-like iteration on sign vectors, at   */
/* most 5 solves with K^-1 and K^-T, plus Higham's alternating-sign extra vector.  K is   */
/* symmetric here, so K^-T = K^-1 and ||K||_1 = ||K||_inf; the estimate is a lower bound. */
/* ------------------------------------------------------------------------------------ */

double or_condest(const or_lu_t *f, const int64_t *rp, const double *v) {
    int64_t n = f->n;
    double *x = (double *)malloc((size_t)n * sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    double *sg = (double *)malloc((size_t)n * sizeof(double));
    if (!x || !y || !sg) {
        free(x); free(y); free(sg);
        return -1.0;
    }
    for (int64_t i = 0; i < n; i++) x[i] = 1.0 / (double)n;
    double est = 0.0;
    int64_t jprev = -1;
    for (int it = 0; it < 5; it++) {
        or_solve(f, x, y); /* y = K^-1 x */
        double e = 0.0;
        for (int64_t i = 0; i < n; i++) e += fabs(y[i]);
        if (it > 0 && e <= est) break;
        est = e;
        for (int64_t i = 0; i < n; i++) sg[i] = y[i] >= 0.0 ? 1.0 : -1.0;
        or_solve(f, sg, y); /* z = K^-T sign(y) = K^-1 sign(y) */
        int64_t jmax = 0;
        for (int64_t i = 1; i < n; i++)
            if (fabs(y[i]) > fabs(y[jmax])) jmax = i;
        if (it > 0 && jmax == jprev) break;
        double ztx = 0.0;
        for (int64_t i = 0; i < n; i++) ztx += y[i] * x[i];
        if (it > 0 && fabs(y[jmax]) <= ztx) break;
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
        x[jmax] = 1.0;
        jprev = jmax;
    }
    /* extra vector x_i = (-1)^i (1 + i/(n-1)) */
    for (int64_t i = 0; i < n; i++) {
        double t = n > 1 ? 1.0 + (double)i / (double)(n - 1) : 1.0;
        x[i] = (i % 2 == 0) ? t : -t;
    }
    or_solve(f, x, y);
    double e2 = 0.0;
    for (int64_t i = 0; i < n; i++) e2 += fabs(y[i]);
    e2 = 2.0 * e2 / (3.0 * (double)n);
    if (e2 > est) est = e2;
    free(x); free(y); free(sg);
    return est * or_norm_inf_mat(n, rp, v);
}

/* ------------------------------------------------------------------------------------ */
/* FGMRES-IR (Section 2.1).                                                               */
/*  x0 = M^-1 b with M = the LU factors; rho0 = b - K x0.                                 */
/*  Skip refinement when the initial solution already passes (Section 2.3).               */
/*  Each cycle: v_1 = rho/||rho||; for j: z_j = M^-1 v_j (right preconditioning, kept:    */
/*  flexible basis), w = K z_j, CGS2 (two classical Gram-Schmidt passes), h_{j+1,j} =     */
/*  ||w||, Givens rotations on the Hessenberg column, estimated residual |g_{j+1}|.  The  */
/*  solution x += Z y is formed only at the end of a cycle (restart or convergence), then */
/*  the true residual decides.                                                            */
/*  mode 0: inner test |g_{j+1}| <= eta (||K||_inf ||x_cycle||_2 + ||b||_2), accept iff    */
/*          true NRBE <= eta; refine iff NRBE(x0) > eta.                                   */
/*  mode 1 (paper's test): inner test |g_{j+1}| < eta ||rho0||_2 (RR on the estimated      */
/*          residual), refine iff ||rho0||/||b|| >= eta, accept when the estimate passes. */
/*  mode | 2: residuals rho = b - K x in extended precision (or_residual_dd).             */
/*  mode | 4: delayed CGS2 (DCGS2), one of the low-synchronization variants the paper     */
/*          cites for FGMRES (Section 2.1; Bielich et al., Parallel Computing 2022): one    */
/*          reduction per step, the second Gram-Schmidt pass of u_j and its normalization   */
/*          deferred to step j + 1, where they share the reduction with K M^-1 u_j; the     */
/*          Hessenberg column, the preconditioned vector and the next vector are corrected  */
/*          for the deferred pass (see fgmres_cycle_dcgs2).                                  */
/* precision 0: FP64 factors; 1: FP32 factors (Lx32/Ux32), preconditioner in binary32.    */
/* info: [0] iterations, [1] cycles, [2] final NRBE, [3] RR (true), [4] converged flag,   */
/*       [5] NRBE of x0, [6] final estimated residual, [7] final true residual norm,      */
/*       [8] preconditioner applications (x0 included)                                    */
/* ------------------------------------------------------------------------------------ */

static void apply_m(const or_lu_t *f, const double *Lx, const double *Ux, const float *Lx32,
                    const float *Ux32, int precision, const double *in, double *out) {
    if (precision == 1) or_solve_with32(f, Lx32, Ux32, in, out);
    else or_solve_with(f, Lx, Ux, in, out);
}

static void matvec(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                   double *y) {
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            double prod = v[p] * x[ci[p]];
            s = s + prod;
        }
        y[i] = s;
    }
}

/* Work arrays of one FGMRES(R) run. */
typedef struct {
    int64_t n;
    int R;
    double *V;   /* R + 1 basis vectors (slot j + 1 holds the next, not yet final, vector) */
    double *Z;   /* R preconditioned vectors z_j = M^-1 v_j */
    double *H;   /* rotated Hessenberg, column-major (R + 1) x R: upper triangular */
    double *Hu;  /* the final Hessenberg columns before rotation, (R + 1) x R */
    double *cs, *sn, *g, *h, *h2, *c, *sv, *e, *hs, *w;
} fg_ws_t;

/* Column j of the Hessenberg matrix, col[0..j+1], is complete: apply rotations 0..j-1,
   choose rotation j to annihilate col[j+1], rotate g, store the column.  Returns the
   estimated residual |g[j+1]|. */
static double givens_close(fg_ws_t *ws, int j, double *col) {
    double *cs = ws->cs, *sn = ws->sn, *g = ws->g;
    for (int t = 0; t < j; t++) {
        double a = col[t], bb = col[t + 1];
        col[t] = cs[t] * a + sn[t] * bb;
        col[t + 1] = -sn[t] * a + cs[t] * bb;
    }
    double a = col[j], bb = col[j + 1];
    double rr = hypot(a, bb);
    if (rr == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
    } else {
        cs[j] = a / rr;
        sn[j] = bb / rr;
    }
    col[j] = rr;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    for (int t = 0; t <= j; t++) ws->H[(size_t)j * (ws->R + 1) + t] = col[t];
    return fabs(g[j + 1]);
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* One FGMRES cycle with CGS2 (V[0] and g already set): for j = 0, 1, ...: z_j = M^-1 v_j,
   w = K z_j, two classical Gram-Schmidt passes against v_0..v_j, h_{j+1,j} = ||w||, rotation,
   estimate; stop on the inner tolerance, a breakdown (h_{j+1,j} <= 1e-14 ||K z_j||) or after
   R steps.  Returns the number of Hessenberg columns (steps) completed. */
static int fgmres_cycle_cgs2(fg_ws_t *ws, const or_lu_t *f, const double *Lx, const double *Ux,
                             const float *Lx32, const float *Ux32, int precision, const int64_t *rp,
                             const int32_t *ci, const double *v, double inner_tol, double *est,
                             long *applications, double *hist, int64_t *nh, int64_t hist_cap) {
    const int64_t n = ws->n;
    const int R = ws->R;
    double *V = ws->V, *Z = ws->Z, *h = ws->h, *h2 = ws->h2, *w = ws->w;
    int jdone = 0;
    for (int j = 0; j < R; j++) {
        double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
        apply_m(f, Lx, Ux, Lx32, Ux32, precision, vj, zj);
        (*applications)++;
        matvec(n, rp, ci, v, zj, w);
        double win = nrm2(n, w);
        for (int t = 0; t <= j; t++) h[t] = 0.0;
        for (int pass = 0; pass < 2; pass++) {
            for (int t = 0; t <= j; t++) h2[t] = dot(n, V + (size_t)t * n, w);
            for (int t = 0; t <= j; t++) {
                const double *vt = V + (size_t)t * n;
                for (int64_t i = 0; i < n; i++) w[i] -= h2[t] * vt[i];
                h[t] += h2[t];
            }
        }
        double hn = nrm2(n, w);
        h[j + 1] = hn;
        for (int t = 0; t <= j + 1; t++) ws->Hu[(size_t)j * (ws->R + 1) + t] = h[t];
        *est = givens_close(ws, j, h);
        jdone = j + 1;
        if (hist && *nh < hist_cap) hist[(*nh)++] = *est;
        int breakdown = !(hn > 1e-14 * win);
        if (!breakdown)
            for (int64_t i = 0; i < n; i++) V[(size_t)(j + 1) * n + i] = w[i] / hn;
        if (*est <= inner_tol || breakdown) break;
    }
    return jdone;
}

/* One FGMRES cycle with delayed CGS2 (V[0] and g already set).  Step j works on u_j, the
   vector after one Gram-Schmidt pass (u_0 = v_0, already final):
     z~ = M^-1 u_j, w = K z~                               (none at j = R)
     one reduction: s_t = v_t.u_j, c_t = v_t.w (t < j), alpha = u_j.u_j, d = u_j.w
     j > 0: second pass of u_j: beta = sqrt(alpha - |s|^2), v_j = (u_j - V s) / beta, so
            column j-1 becomes final: (p + s, beta) with p its one-pass part; rotation,
            estimate, stop test (inner tolerance, breakdown beta <= 1e-14 |column|, j = R)
     z_j = (z~ - Z s) / beta = M^-1 v_j  (M^-1 is linear)
     K z_j = (w - K Z s) / beta = (w - V Hu s) / beta  (Arnoldi relation K Z = V Hu), so with
     e = V_{0..j}^T w (e_t = c_t for t < j, e_j = (d - s.c) / beta) the one-pass column j is
     p = (e - Hu s) / beta and u_{j+1} = K z_j - V p = (w - V e) / beta.
   beta = 1 and s = () at j = 0.  In absolute size s_t beta and s.c / beta are of the order
   of rounding (u ||K z||), like the second-pass coefficients of CGS2; the terms divided by
   the small beta (V s, Z s, Hu s) are what keep V orthonormal and K Z = V Hu.
   Returns the number of final columns. */
static int fgmres_cycle_dcgs2(fg_ws_t *ws, const or_lu_t *f, const double *Lx, const double *Ux,
                              const float *Lx32, const float *Ux32, int precision, const int64_t *rp,
                              const int32_t *ci, const double *v, double inner_tol, double *est,
                              long *applications, double *hist, int64_t *nh, int64_t hist_cap) {
    const int64_t n = ws->n;
    const int R = ws->R;
    double *V = ws->V, *Z = ws->Z, *Hu = ws->Hu, *w = ws->w;
    double *p = ws->h, *col = ws->h2, *c = ws->c, *sv = ws->sv, *e = ws->e, *hs = ws->hs;
    int jdone = 0;
    for (int j = 0; j <= R; j++) {
        double *uj = V + (size_t)j * n;
        double *zj = Z + (size_t)j * n;
        const int have_w = j < R;
        if (have_w) {
            apply_m(f, Lx, Ux, Lx32, Ux32, precision, uj, zj);
            (*applications)++;
            matvec(n, rp, ci, v, zj, w);
        }
        for (int t = 0; t < j; t++) {
            sv[t] = dot(n, V + (size_t)t * n, uj);
            if (have_w) c[t] = dot(n, V + (size_t)t * n, w);
        }
        double alpha = dot(n, uj, uj);
        double d = have_w ? dot(n, uj, w) : 0.0;
        double beta = 1.0;
        if (j > 0) {
            double ss = 0.0;
            for (int t = 0; t < j; t++) ss += sv[t] * sv[t];
            beta = alpha - ss > 0.0 ? sqrt(alpha - ss) : 0.0;
            for (int t = 0; t < j; t++) col[t] = p[t] + sv[t];
            col[j] = beta;
            double cn = 0.0;
            for (int t = 0; t <= j; t++) cn += col[t] * col[t];
            cn = sqrt(cn);
            for (int t = 0; t <= j; t++) Hu[(size_t)(j - 1) * (R + 1) + t] = col[t];
            *est = givens_close(ws, j - 1, col);
            jdone = j;
            if (hist && *nh < hist_cap) hist[(*nh)++] = *est;
            int breakdown = !(beta > 1e-14 * cn);
            if (*est <= inner_tol || breakdown || j == R) break;
            for (int64_t i = 0; i < n; i++) {
                double a = uj[i], b2 = zj[i];
                for (int t = 0; t < j; t++) {
                    a -= V[(size_t)t * n + i] * sv[t];
                    b2 -= Z[(size_t)t * n + i] * sv[t];
                }
                uj[i] = a / beta;
                zj[i] = b2 / beta;
            }
        }
        double sc = 0.0;
        for (int t = 0; t < j; t++) {
            e[t] = c[t];
            sc += sv[t] * c[t];
        }
        e[j] = (d - sc) / beta;
        for (int t = 0; t <= j; t++) {
            hs[t] = 0.0;
            for (int k = 0; k < j; k++) hs[t] += Hu[(size_t)k * (R + 1) + t] * sv[k];
            p[t] = (e[t] - hs[t]) / beta;
        }
        double *un = V + (size_t)(j + 1) * n;
        for (int64_t i = 0; i < n; i++) {
            double a = w[i];
            for (int t = 0; t <= j; t++) a -= V[(size_t)t * n + i] * e[t];
            un[i] = a / beta;
        }
    }
    return jdone;
}

int or_fgmres_ir(const or_lu_t *f, const double *Lx, const double *Ux, const float *Lx32,
                 const float *Ux32, int precision, const int64_t *rp, const int32_t *ci,
                 const double *v, const double *b, double *x, int restart, int max_restarts,
                 double eta, int mode, double *info, double *hist, int64_t hist_cap) {
    int64_t n = f->n;
    int R = restart;
    if (R < 1) return OR_EINVAL;
    fg_ws_t ws;
    ws.n = n;
    ws.R = R;
    ws.V = (double *)malloc((size_t)n * (R + 1) * sizeof(double));
    ws.Z = (double *)malloc((size_t)n * R * sizeof(double));
    ws.H = (double *)calloc((size_t)(R + 1) * R, sizeof(double));
    ws.Hu = (double *)calloc((size_t)(R + 1) * R, sizeof(double));
    ws.cs = (double *)malloc((size_t)R * sizeof(double));
    ws.sn = (double *)malloc((size_t)R * sizeof(double));
    ws.g = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.h = (double *)malloc((size_t)(R + 2) * sizeof(double));
    ws.h2 = (double *)malloc((size_t)(R + 2) * sizeof(double));
    ws.c = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.sv = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.e = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.hs = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.w = (double *)malloc((size_t)n * sizeof(double));
    double *yv = (double *)malloc((size_t)R * sizeof(double));
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *xbest = (double *)malloc((size_t)n * sizeof(double));
    int ok = ws.V && ws.Z && ws.H && ws.Hu && ws.cs && ws.sn && ws.g && ws.h && ws.h2 && ws.c &&
             ws.sv && ws.e && ws.hs && ws.w && yv && r && xbest;
    int status = OR_ENOMEM;
    if (ok) {
        double *V = ws.V, *Z = ws.Z, *H = ws.H, *g = ws.g;
        int64_t nh = 0;
        long applications = 0;
        void (*resid)(int64_t, const int64_t *, const int32_t *, const double *, const double *,
                      const double *, double *) = (mode & 2) ? or_residual_dd : or_residual;
        const int dcgs2 = (mode & 4) != 0;
        const int inner_solver = (mode & 8) != 0; /* a correction solve: no best-iterate restore */
        mode &= 1;
        double kn = or_norm_inf_mat(n, rp, v);
        double bn = nrm2(n, b);
        apply_m(f, Lx, Ux, Lx32, Ux32, precision, b, x);
        applications++;
        resid(n, rp, ci, v, x, b, r);
        double rho0 = nrm2(n, r);
        double rn = rho0;
        double nrbe = rn / (kn * nrm2(n, x) + bn);
        info[5] = nrbe;
        int iters = 0, cycles = 0, converged = 0;
        double est = rn;
        /* the iterate with the lowest true residual so far (x0 included) is returned when the
           refinement does not converge; best_nrbe is its NRBE */
        double best_rn = rn, best_nrbe = nrbe;
        memcpy(xbest, x, (size_t)n * sizeof(double));
        if (mode == 0 ? (nrbe <= eta) : (rn / bn < eta)) converged = 1;
        while (!converged && cycles <= max_restarts) {
            cycles++;
            double beta = rn;
            if (!(beta > 0.0)) {
                converged = 1;
                break;
            }
            double xn = nrm2(n, x);
            double inner_tol = mode == 0 ? eta * (kn * xn + bn) : eta * rho0;
            for (int64_t i = 0; i < n; i++) V[i] = r[i] / beta;
            for (int t = 0; t <= R; t++) g[t] = 0.0;
            g[0] = beta;
            int jdone;
            if (dcgs2)
                jdone = fgmres_cycle_dcgs2(&ws, f, Lx, Ux, Lx32, Ux32, precision, rp, ci, v, inner_tol,
                                           &est, &applications, hist, &nh, hist_cap);
            else
                jdone = fgmres_cycle_cgs2(&ws, f, Lx, Ux, Lx32, Ux32, precision, rp, ci, v, inner_tol,
                                          &est, &applications, hist, &nh, hist_cap);
            iters += jdone;
            /* y = H^-1 g (upper triangular, jdone x jdone), then x += Z y */
            for (int t = jdone - 1; t >= 0; t--) {
                double s = g[t];
                for (int u = t + 1; u < jdone; u++) s -= H[(size_t)u * (R + 1) + t] * yv[u];
                yv[t] = s / H[(size_t)t * (R + 1) + t];
            }
            for (int t = 0; t < jdone; t++) {
                const double *zt = Z + (size_t)t * n;
                for (int64_t i = 0; i < n; i++) x[i] += yv[t] * zt[i];
            }
            resid(n, rp, ci, v, x, b, r);
            rn = nrm2(n, r);
            nrbe = rn / (kn * nrm2(n, x) + bn);
            /* an iterate whose true residual exceeds that of x0 is never accepted: the NRBE
               test alone passes when rounding makes ||x|| grow without bound */
            if ((mode == 0 ? (nrbe <= eta) : (est < eta * rho0)) && rn <= rho0) converged = 1;
            if (rn < best_rn) {
                best_rn = rn;
                best_nrbe = nrbe;
                memcpy(xbest, x, (size_t)n * sizeof(double));
            }
        }
        if (!converged && !inner_solver && rn > best_rn) {
            memcpy(x, xbest, (size_t)n * sizeof(double));
            rn = best_rn;
            nrbe = best_nrbe;
        }
        info[0] = iters;
        info[1] = cycles;
        info[2] = nrbe;
        info[3] = rho0 > 0.0 ? rn / rho0 : 0.0;
        info[4] = converged;
        info[6] = est;
        info[7] = rn;
        info[8] = (double)applications;
        status = converged ? OR_OK : 4;
    }
    free(ws.V); free(ws.Z); free(ws.H); free(ws.Hu); free(ws.cs); free(ws.sn); free(ws.g);
    free(ws.h); free(ws.h2); free(ws.c); free(ws.sv); free(ws.e); free(ws.hs); free(ws.w);
    free(yv); free(r); free(xbest);
    return status;
}

/* One Arnoldi cycle of FGMRES(R) from r0 with the preconditioner M = (Lx, Ux), run to R
   steps (or a breakdown), returning the basis V (n x (R+1)), Z = M^-1 V (n x R) and the
   Hessenberg matrix before rotation (column-major (R+1) x R) so that tests can check the
   Arnoldi relation K Z_k = V_{k+1} Hbar_k and the orthonormality of V.  gs: 0 CGS2, 1 DCGS2
   (whose last vector, v_k, is left after its first pass: the relation holds for k - 1
   columns).  precision 1 applies the FP32 factors (Lx32, Ux32) in binary32, as
   or_fgmres_ir does.  Returns k, the number of Hessenberg columns, or -1 on error. */
int or_arnoldi(const or_lu_t *f, const double *Lx, const double *Ux, const float *Lx32, const float *Ux32,
               int precision, const int64_t *rp, const int32_t *ci, const double *v, const double *r0, int R,
               int gs, double *Vout, double *Zout, double *Hout) {
    const int64_t n = f->n;
    if (R < 1) return -1;
    fg_ws_t ws;
    ws.n = n;
    ws.R = R;
    ws.V = Vout;
    ws.Z = Zout;
    ws.Hu = Hout;
    ws.H = (double *)calloc((size_t)(R + 1) * R, sizeof(double));
    ws.cs = (double *)malloc((size_t)R * sizeof(double));
    ws.sn = (double *)malloc((size_t)R * sizeof(double));
    ws.g = (double *)calloc((size_t)(R + 1), sizeof(double));
    ws.h = (double *)malloc((size_t)(R + 2) * sizeof(double));
    ws.h2 = (double *)malloc((size_t)(R + 2) * sizeof(double));
    ws.c = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.sv = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.e = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.hs = (double *)malloc((size_t)(R + 1) * sizeof(double));
    ws.w = (double *)malloc((size_t)n * sizeof(double));
    int k = -1;
    if (ws.H && ws.cs && ws.sn && ws.g && ws.h && ws.h2 && ws.c && ws.sv && ws.e && ws.hs && ws.w) {
        memset(Vout, 0, (size_t)n * (R + 1) * sizeof(double));
        memset(Zout, 0, (size_t)n * R * sizeof(double));
        memset(Hout, 0, (size_t)(R + 1) * R * sizeof(double));
        double beta = nrm2(n, r0);
        for (int64_t i = 0; i < n; i++) Vout[i] = r0[i] / beta;
        ws.g[0] = beta;
        double est = beta;
        long applications = 0;
        int64_t nh = 0;
        if (gs == 1)
            k = fgmres_cycle_dcgs2(&ws, f, Lx, Ux, Lx32, Ux32, precision, rp, ci, v, 0.0, &est, &applications,
                                   NULL, &nh, 0);
        else
            k = fgmres_cycle_cgs2(&ws, f, Lx, Ux, Lx32, Ux32, precision, rp, ci, v, 0.0, &est, &applications,
                                  NULL, &nh, 0);
    }
    free(ws.H); free(ws.cs); free(ws.sn); free(ws.g); free(ws.h); free(ws.h2); free(ws.c);
    free(ws.sv); free(ws.e); free(ws.hs); free(ws.w);
    return k;
}

/* ------------------------------------------------------------------------------------ */
/* Richardson iterative refinement (Section 1.3): x0 = M^-1 b; then repeatedly           */
/* rho = b - K x, d = M^-1 rho, x = x + d.  Stopping (MA57's ratio test on the norm of    */
/* scaled residuals, NSR = ||rho||_inf / (||K||_inf ||x||_inf)): stop when               */
/* ||rho||_2 < tol ||rho0||_2, or when NSR_new > ratio * NSR_old (the step no longer     */
/* reduces it enough), or after max_it corrections.                                      */
/* With inner_restart > 0 the correction d solves K d = rho by FGMRES(inner_restart)     */
/* preconditioned by the same factors, to the relative tolerance inner_tol (the          */
/* "iterative solver on the error system" variant, Section 2.1).                        */
/* info: [0] corrections, [1] preconditioner applications, [2] final NSR, [3] final      */
/*       NRBE, [4] converged (relative residual test passed), [5] final ||rho||_2 /     */
/*       ||rho0||_2.  hist: NSR after each correction.                                   */
/* ------------------------------------------------------------------------------------ */

int or_richardson(const or_lu_t *f, const double *Lx, const double *Ux, const int64_t *rp, const int32_t *ci,
                  const double *v, const double *b, double *x, int max_it, double tol, double ratio,
                  int inner_restart, double inner_tol, double *info, double *hist, int64_t hist_cap) {
    int64_t n = f->n;
    double *r = (double *)malloc((size_t)n * sizeof(double));
    double *d = (double *)malloc((size_t)n * sizeof(double));
    double *xbest = (double *)malloc((size_t)n * sizeof(double));
    if (!r || !d || !xbest) {
        free(r); free(d); free(xbest);
        return OR_ENOMEM;
    }
    double kn = or_norm_inf_mat(n, rp, v);
    double bn = nrm2(n, b);
    long applications = 1;
    or_solve_with(f, Lx, Ux, b, x);
    or_residual(n, rp, ci, v, x, b, r);
    double rho0 = nrm2(n, r);
    double rn = rho0;
    double nsr = nrminf(n, r) / (kn * nrminf(n, x));
    /* the iterate with the lowest true residual (x0 included) is returned if not converged */
    double best_rn = rn, best_nsr = nsr;
    memcpy(xbest, x, (size_t)n * sizeof(double));
    int it = 0, converged = rn < tol * rho0;
    while (!converged && it < max_it) {
        if (inner_restart > 0) {
            double inner[9];
            or_fgmres_ir(f, Lx, Ux, NULL, NULL, 0, rp, ci, v, r, d, inner_restart, 0, inner_tol, 1 | 8, inner,
                         NULL, 0);
            applications += (long)inner[8];
        } else {
            or_solve_with(f, Lx, Ux, r, d);
            applications += 1;
        }
        for (int64_t i = 0; i < n; i++) x[i] = x[i] + d[i];
        it++;
        or_residual(n, rp, ci, v, x, b, r);
        rn = nrm2(n, r);
        double nsr_new = nrminf(n, r) / (kn * nrminf(n, x));
        if (hist && it <= hist_cap) hist[it - 1] = nsr_new;
        converged = rn < tol * rho0;
        int stalled = nsr_new > ratio * nsr;
        nsr = nsr_new;
        if (rn < best_rn) {
            best_rn = rn;
            best_nsr = nsr;
            memcpy(xbest, x, (size_t)n * sizeof(double));
        }
        if (stalled) break;
    }
    if (!converged && rn > best_rn) {
        memcpy(x, xbest, (size_t)n * sizeof(double));
        rn = best_rn;
        nsr = best_nsr;
    }
    info[0] = it;
    info[1] = (double)applications;
    info[2] = nsr;
    info[3] = rn / (kn * nrm2(n, x) + bn);
    info[4] = converged;
    info[5] = rho0 > 0.0 ? rn / rho0 : 0.0;
    free(r); free(d); free(xbest);
    return converged ? OR_OK : 4;
}

/* Export the step-indexed pivot inverse (row -> step) for convenience. */
void or_lu_pinv(const or_lu_t *f, int32_t *pinv) { memcpy(pinv, f->pinv, (size_t)f->n * sizeof(int32_t)); }
