/*
 * mst_oracle.c -- CPU oracle for the minimum spanning tree.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load this library.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * What is computed (Durbhakula, "Parallel Minimum Spanning Tree Algorithms
 * and Evaluation", arXiv 2005.06913):
 *
 *   Input: an undirected graph given as an edge list src[e] -- dst[e] with
 *   weight w[e] (Section 2.1, data structures; src and dest are
 *   interchangeable).  The paper assumes a connected graph with distinct
 *   weights (Section 2.1, inputs).  This oracle accepts any graph and orders
 *   edges by the strict total order
 *
 *       e < f   iff   (w[e], e) < (w[f], f)      (lexicographic),
 *
 *   i.e. by weight, then by input position.  With distinct weights this is
 *   the order by weight alone, so the result is the paper's unique MST.  With
 *   ties it picks one particular MST deterministically.  A disconnected graph
 *   yields the minimum spanning forest and status ORACLE_DISCONNECTED.
 *
 *   Output: in_mst[e] in {0,1} in input order and the exact uint64 total.
 *
 * Independent routines:
 *   oracle_kruskal   -- Kruskal's algorithm (named in Section 1): edges in
 *                       increasing order, keep an edge iff it joins two
 *                       different trees of the forest built so far.
 *   oracle_boruvka   -- the sequential Boruvka algorithm of Section 2.1 with
 *                       the "covered" optimisation described after it, in the
 *                       paper's step order, plus per-round statistics.
 *   oracle_check_mst -- a certificate checker: spanning-forest structure, the
 *                       cycle property under the total order, and the total.
 *   oracle_min_edge_keys -- the first round's edge loop alone: the lightest
 *                       edge at every vertex.
 *
 * Plain and slow on purpose: qsort, a union-find with union by size and
 * path halving, arrays indexed directly.
 */

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_DISCONNECTED 1
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_RANGE (-2)
#define ORACLE_ERR_NOMEM (-4)

/* Position of edge e in the strict total order: weight first, then index. */
static uint64_t order_key(const uint32_t* w, int64_t e) {
    return ((uint64_t)w[e] << 32) | (uint64_t)e;
}

static int check_args(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      const uint32_t* w) {
    if (n < 0 || m < 0) return ORACLE_ERR_ARG;
    if (m > 0 && (!src || !dst || !w)) return ORACLE_ERR_ARG;
    if (m > (int64_t)0xFFFFFFFFLL) return ORACLE_ERR_ARG;
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return ORACLE_ERR_RANGE;
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------- union-find */

typedef struct {
    int32_t* parent;
    int32_t* size;
} uf_t;

static int uf_init(uf_t* u, int32_t n) {
    size_t k = n > 0 ? (size_t)n : 1;
    u->parent = (int32_t*)malloc(k * sizeof(int32_t));
    u->size = (int32_t*)malloc(k * sizeof(int32_t));
    if (!u->parent || !u->size) {
        free(u->parent);
        free(u->size);
        return ORACLE_ERR_NOMEM;
    }
    for (int32_t v = 0; v < n; ++v) {
        u->parent[v] = v;
        u->size[v] = 1;
    }
    return ORACLE_OK;
}

static void uf_free(uf_t* u) {
    free(u->parent);
    free(u->size);
}

/* Root of v's tree; path halving on the way. */
static int32_t uf_find(uf_t* u, int32_t v) {
    while (u->parent[v] != v) {
        u->parent[v] = u->parent[u->parent[v]];
        v = u->parent[v];
    }
    return v;
}

/* Join the trees rooted at ra != rb; the larger tree's root stays root. */
static void uf_union_roots(uf_t* u, int32_t ra, int32_t rb) {
    if (u->size[ra] < u->size[rb]) {
        int32_t t = ra;
        ra = rb;
        rb = t;
    }
    u->parent[rb] = ra;
    u->size[ra] += u->size[rb];
}

/* ------------------------------------------------------------------ Kruskal */

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return (x > y) - (x < y);
}

/*
 * Kruskal: visit edges in increasing (w, e) order; an edge is a tree edge iff
 * its endpoints are in different trees of the forest built so far.  Returns
 * ORACLE_OK (spanning tree), ORACLE_DISCONNECTED (spanning forest) or an error.
 */
int oracle_kruskal(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   const uint32_t* w, uint8_t* in_mst, uint64_t* total) {
    int rc = check_args(n, m, src, dst, w);
    if (rc != ORACLE_OK) return rc;
    if (!total || (m > 0 && !in_mst)) return ORACLE_ERR_ARG;
    if (m > 0) memset(in_mst, 0, (size_t)m);
    *total = 0;

    uint64_t* keys = (uint64_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
    uf_t uf;
    if (!keys) return ORACLE_ERR_NOMEM;
    if (uf_init(&uf, n) != ORACLE_OK) {
        free(keys);
        return ORACLE_ERR_NOMEM;
    }
    for (int64_t e = 0; e < m; ++e) keys[e] = order_key(w, e);
    qsort(keys, (size_t)m, sizeof(uint64_t), cmp_u64);

    int64_t taken = 0;
    for (int64_t i = 0; i < m && taken + 1 < (int64_t)n; ++i) {
        int64_t e = (int64_t)(keys[i] & 0xFFFFFFFFull);
        int32_t ra = uf_find(&uf, src[e]);
        int32_t rb = uf_find(&uf, dst[e]);
        if (ra == rb) continue; /* would close a cycle (or is a self-loop) */
        uf_union_roots(&uf, ra, rb);
        in_mst[e] = 1;
        *total += w[e];
        ++taken;
    }
    free(keys);
    uf_free(&uf);
    return (n <= 1 || taken == (int64_t)n - 1) ? ORACLE_OK : ORACLE_DISCONNECTED;
}

/* ------------------------------------------------------ sequential Boruvka */

/*
 * Sequential Boruvka of Section 2.1 with the "covered" optimisation.
 *
 * Every vertex starts as its own component.  Each round:
 *   1. minimum[] <- -1 for every vertex;
 *   2. for every edge not yet covered: find the components of both ends; if
 *      they are the same the edge is internal and becomes covered; otherwise
 *      the edge replaces minimum[] of each end's component when it precedes
 *      the current minimum in the (w, e) order;
 *   3. for every vertex v with minimum[v] != -1: find the components of the
 *      minimum edge's ends again; if they differ, add the edge to the tree,
 *      cover it, and unite the two components (the larger one's root
 *      becomes the root).
 * Rounds repeat while more than one component remains.  A round that adds no
 * edge while several components remain means the graph is disconnected; the
 * loop stops there and the result is the minimum spanning forest.
 *
 * Statistics per round r (stats[3r + k]):
 *   k=0: components at the start of the round,
 *   k=1: live edges -- edges whose ends lie in different components at the
 *        start of the round (self-loops are never live),
 *   k=2: edges added to the tree in the round.
 * *rounds receives the number of rounds that ran (at most max_rounds are
 * recorded; the algorithm itself always runs to completion).
 *
 * If labels != NULL it receives, for every vertex, the smallest vertex id in
 * its final component (a labelling independent of the union rule).
 */
int oracle_boruvka(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   const uint32_t* w, uint8_t* in_mst, uint64_t* total, int64_t* stats,
                   int32_t max_rounds, int32_t* rounds, int32_t* labels) {
    int rc = check_args(n, m, src, dst, w);
    if (rc != ORACLE_OK) return rc;
    if (!total || (m > 0 && !in_mst)) return ORACLE_ERR_ARG;
    if (m > 0) memset(in_mst, 0, (size_t)m);
    *total = 0;
    if (rounds) *rounds = 0;

    uf_t comp;
    if (uf_init(&comp, n) != ORACLE_OK) return ORACLE_ERR_NOMEM;
    int64_t* minimum = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    uint8_t* covered = (uint8_t*)calloc((size_t)(m > 0 ? m : 1), 1);
    if (!minimum || !covered) {
        free(minimum);
        free(covered);
        uf_free(&comp);
        return ORACLE_ERR_NOMEM;
    }

    int64_t components = n;
    int32_t r = 0;
    int status = ORACLE_OK;
    while (components > 1) {
        /* 1. reset the per-component minimum */
        for (int32_t v = 0; v < n; ++v) minimum[v] = -1;

        /* 2. edge loop */
        int64_t live = 0;
        for (int64_t e = 0; e < m; ++e) {
            if (covered[e]) continue;
            int32_t c1 = uf_find(&comp, src[e]);
            int32_t c2 = uf_find(&comp, dst[e]);
            if (c1 == c2) {
                covered[e] = 1;
                continue;
            }
            ++live;
            uint64_t k = order_key(w, e);
            if (minimum[c1] == -1 || order_key(w, minimum[c1]) > k) minimum[c1] = e;
            if (minimum[c2] == -1 || order_key(w, minimum[c2]) > k) minimum[c2] = e;
        }

        /* 3. component loop */
        int64_t added = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (minimum[v] == -1) continue;
            int64_t e = minimum[v];
            int32_t c1 = uf_find(&comp, src[e]);
            int32_t c2 = uf_find(&comp, dst[e]);
            if (c1 == c2) continue;
            in_mst[e] = 1;
            covered[e] = 1;
            *total += w[e];
            ++added;
            uf_union_roots(&comp, c1, c2);
        }

        if (stats && r < max_rounds) {
            stats[3 * (int64_t)r + 0] = components;
            stats[3 * (int64_t)r + 1] = live;
            stats[3 * (int64_t)r + 2] = added;
        }
        ++r;
        if (added == 0) {
            status = ORACLE_DISCONNECTED;
            break;
        }
        components -= added;
    }
    if (rounds) *rounds = r;

    if (labels) {
        /* smallest vertex id of each final component */
        for (int32_t v = 0; v < n; ++v) labels[v] = -1;
        for (int32_t v = 0; v < n; ++v) {
            int32_t root = uf_find(&comp, v);
            if (labels[root] == -1) labels[root] = v; /* first visit is the smallest id */
        }
        for (int32_t v = 0; v < n; ++v) labels[v] = labels[uf_find(&comp, v)];
    }

    free(minimum);
    free(covered);
    uf_free(&comp);
    return status;
}

/* ----------------------------------------------------- certificate checker */

#define CHECK_OK 0
#define CHECK_BAD_FLAG (-10)      /* in_mst holds a value other than 0 or 1 */
#define CHECK_LOOP_IN_TREE (-11)  /* a self-loop is marked */
#define CHECK_CYCLE (-12)         /* the marked edges contain a cycle */
#define CHECK_NOT_SPANNING (-13)  /* marked edge count != n - #components */
#define CHECK_NOT_MINIMUM (-14)   /* a non-tree edge precedes its tree-path maximum */
#define CHECK_TOTAL (-15)         /* total != sum of marked weights */

/*
 * Certifies that in_mst marks the unique minimum spanning forest under the
 * (w, e) order, and that total is its weight:
 *   (a) the marked edges form a forest (no cycle, no self-loop);
 *   (b) it has n - c edges where c is the number of connected components of
 *       the input, so it spans every component;
 *   (c) cycle property: every unmarked non-loop edge comes after every edge
 *       on the forest path between its endpoints;
 *   (d) total equals the sum of the marked weights.
 * (a)-(c) hold exactly for the minimum spanning forest under a strict total
 * order.  Path maxima use binary lifting over a BFS-rooted forest.
 */
int oracle_check_mst(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                     const uint32_t* w, const uint8_t* in_mst, uint64_t total) {
    int rc = check_args(n, m, src, dst, w);
    if (rc != ORACLE_OK) return rc;
    if (m > 0 && !in_mst) return ORACLE_ERR_ARG;

    int64_t marked = 0;
    uint64_t sum = 0;
    for (int64_t e = 0; e < m; ++e) {
        if (in_mst[e] > 1) return CHECK_BAD_FLAG;
        if (in_mst[e]) {
            if (src[e] == dst[e]) return CHECK_LOOP_IN_TREE;
            ++marked;
            sum += w[e];
        }
    }

    /* (a) forest check and (b) edge count */
    uf_t all, tree;
    if (uf_init(&all, n) != ORACLE_OK) return ORACLE_ERR_NOMEM;
    if (uf_init(&tree, n) != ORACLE_OK) {
        uf_free(&all);
        return ORACLE_ERR_NOMEM;
    }
    int64_t comps = n;
    int bad = CHECK_OK;
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = uf_find(&all, src[e]), b = uf_find(&all, dst[e]);
        if (a != b) {
            uf_union_roots(&all, a, b);
            --comps;
        }
        if (in_mst[e]) {
            int32_t x = uf_find(&tree, src[e]), y = uf_find(&tree, dst[e]);
            if (x == y) {
                bad = CHECK_CYCLE;
                break;
            }
            uf_union_roots(&tree, x, y);
        }
    }
    uf_free(&all);
    uf_free(&tree);
    if (bad != CHECK_OK) return bad;
    if (marked != (int64_t)n - comps) return CHECK_NOT_SPANNING;

    /* (c) cycle property via binary lifting */
    if (n > 1 && m > 0) {
        int levels = 1;
        while ((1LL << levels) < (long long)n) ++levels;
        size_t N = (size_t)n;
        int64_t* head = (int64_t*)malloc((N + 1) * sizeof(int64_t));
        int32_t* adj_v = (int32_t*)malloc((size_t)(2 * marked + 1) * sizeof(int32_t));
        uint64_t* adj_k = (uint64_t*)malloc((size_t)(2 * marked + 1) * sizeof(uint64_t));
        int32_t* depth = (int32_t*)malloc(N * sizeof(int32_t));
        int32_t* queue = (int32_t*)malloc(N * sizeof(int32_t));
        int32_t* up = (int32_t*)malloc(N * (size_t)levels * sizeof(int32_t));
        uint64_t* upmax = (uint64_t*)malloc(N * (size_t)levels * sizeof(uint64_t));
        if (!head || !adj_v || !adj_k || !depth || !queue || !up || !upmax) {
            free(head); free(adj_v); free(adj_k); free(depth); free(queue); free(up); free(upmax);
            return ORACLE_ERR_NOMEM;
        }
        /* CSR of the forest */
        memset(head, 0, (N + 1) * sizeof(int64_t));
        for (int64_t e = 0; e < m; ++e)
            if (in_mst[e]) {
                head[src[e] + 1]++;
                head[dst[e] + 1]++;
            }
        for (size_t v = 0; v < N; ++v) head[v + 1] += head[v];
        int64_t* fill = (int64_t*)malloc(N * sizeof(int64_t));
        if (!fill) {
            free(head); free(adj_v); free(adj_k); free(depth); free(queue); free(up); free(upmax);
            return ORACLE_ERR_NOMEM;
        }
        memcpy(fill, head, N * sizeof(int64_t));
        for (int64_t e = 0; e < m; ++e)
            if (in_mst[e]) {
                uint64_t k = order_key(w, e);
                adj_v[fill[src[e]]] = dst[e];
                adj_k[fill[src[e]]++] = k;
                adj_v[fill[dst[e]]] = src[e];
                adj_k[fill[dst[e]]++] = k;
            }
        free(fill);
        /* BFS from each unvisited vertex: parent (level 0) and depth */
        for (size_t v = 0; v < N; ++v) depth[v] = -1;
        for (int32_t s = 0; s < n; ++s) {
            if (depth[s] != -1) continue;
            depth[s] = 0;
            up[s] = s;
            upmax[s] = 0;
            int64_t qh = 0, qt = 0;
            queue[qt++] = s;
            while (qh < qt) {
                int32_t v = queue[qh++];
                for (int64_t i = head[v]; i < head[v + 1]; ++i) {
                    int32_t u = adj_v[i];
                    if (depth[u] != -1) continue;
                    depth[u] = depth[v] + 1;
                    up[u] = v;
                    upmax[u] = adj_k[i];
                    queue[qt++] = u;
                }
            }
        }
        /* up[j][v] = 2^j-th ancestor, upmax[j][v] = max key on that stretch */
        for (int j = 1; j < levels; ++j) {
            int32_t* U0 = up + (size_t)(j - 1) * N;
            uint64_t* M0 = upmax + (size_t)(j - 1) * N;
            int32_t* U1 = up + (size_t)j * N;
            uint64_t* M1 = upmax + (size_t)j * N;
            for (size_t v = 0; v < N; ++v) {
                int32_t mid = U0[v];
                U1[v] = U0[mid];
                M1[v] = M0[v] > M0[mid] ? M0[v] : M0[mid];
            }
        }
        for (int64_t e = 0; e < m && bad == CHECK_OK; ++e) {
            if (in_mst[e] || src[e] == dst[e]) continue;
            int32_t a = src[e], b = dst[e];
            uint64_t pmax = 0;
            if (depth[a] < depth[b]) {
                int32_t t = a;
                a = b;
                b = t;
            }
            int32_t diff = depth[a] - depth[b];
            for (int j = 0; diff; ++j, diff >>= 1)
                if (diff & 1) {
                    uint64_t x = upmax[(size_t)j * N + a];
                    if (x > pmax) pmax = x;
                    a = up[(size_t)j * N + a];
                }
            if (a != b) {
                for (int j = levels - 1; j >= 0; --j) {
                    int32_t ua = up[(size_t)j * N + a], ub = up[(size_t)j * N + b];
                    if (ua != ub) {
                        uint64_t x = upmax[(size_t)j * N + a], y = upmax[(size_t)j * N + b];
                        if (x > pmax) pmax = x;
                        if (y > pmax) pmax = y;
                        a = ua;
                        b = ub;
                    }
                }
                uint64_t x = upmax[a], y = upmax[b];
                if (x > pmax) pmax = x;
                if (y > pmax) pmax = y;
                a = up[a];
                b = up[b];
            }
            /* a == b is the lowest common ancestor (same tree by (b) above) */
            if (order_key(w, e) < pmax) bad = CHECK_NOT_MINIMUM;
        }
        free(head); free(adj_v); free(adj_k); free(depth); free(queue); free(up); free(upmax);
        if (bad != CHECK_OK) return bad;
    }

    /* (d) total */
    if (sum != total) return CHECK_TOTAL;
    return CHECK_OK;
}

/*
 * The first Boruvka step on its own (Section 2.1, the edge loop with every
 * vertex its own component): keys[v] = smallest (w[e] << 32) | e over the
 * non-loop edges e incident to v, or UINT64_MAX when there is none.
 */
int oracle_min_edge_keys(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         const uint32_t* w, uint64_t* keys) {
    int rc = check_args(n, m, src, dst, w);
    if (rc != ORACLE_OK) return rc;
    if (n > 0 && !keys) return ORACLE_ERR_ARG;
    for (int32_t v = 0; v < n; ++v) keys[v] = UINT64_MAX;
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] == dst[e]) continue;
        uint64_t k = order_key(w, e);
        if (k < keys[src[e]]) keys[src[e]] = k;
        if (k < keys[dst[e]]) keys[dst[e]] = k;
    }
    return ORACLE_OK;
}
