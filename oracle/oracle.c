/*
 * Betweenness-centrality oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU code used to check the GPU library.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code, header or table with the library under
 * paper_1209_6007_amd/.
 *
 * Precision: IEEE binary64 throughout (the paper does not fix a precision).
 * Scores are over ORDERED source/target pairs with no normalisation, as in the
 * definition of Section 2.1, Eq. (1).
 *
 * Functions:
 *   oracle_bc_plain     -- Algorithm 1 (Bc-Org, Brandes) on an undirected
 *                          unweighted graph in CRS form, Section 2.1.
 *   oracle_bc_weighted  -- Algorithm 2 (Bc-Reach, Section 3.2.1) extended by
 *                          the identical-vertex rules of Section 3.3.3 (sigma
 *                          update, dependency update and accumulation weighted
 *                          by ident).  Returns bc' of the attributed graph.
 *   oracle_bc_classes   -- oracle_bc_weighted for piece vertices that stand for
 *                          ident[v] identical vertices of possibly different
 *                          reaches summing to reach[v]: the members' paths are
 *                          those of Section 3.3.3, each member's hung vertices
 *                          are sources (weight: the sum) and targets (the
 *                          dependency starts at the members' mean reach minus
 *                          one).  Equal reaches r give reach[v] = ident[v] * r
 *                          and oracle_bc_weighted's result.
 *   oracle_single_source-- one source of the weighted algorithm, returning the
 *                          BFS levels, path counts and dependencies.
 *   oracle_bc_pieces    -- oracle_bc_weighted on every piece of a packed set of
 *                          pieces (all sources of each piece), for checking a
 *                          whole shattered graph piece by piece.
 *   oracle_bc_side      -- Algorithm 3 (Bfs-Side, Section 3.3.2) for a list of
 *                          side vertices removed one after another.
 *   oracle_farness_pieces -- weighted farness: for every vertex x of every
 *                          piece, the sum over the vertices y of x's piece
 *                          that x reaches of weight[y] * dist(x, y) (exact
 *                          int64).  With one piece and unit weights this is
 *                          the farness whose reciprocal is closeness
 *                          centrality, the measure the paper names as the
 *                          next one to shatter and compress (Sections 1 and
 *                          5); the paper gives no formulas for it, so the
 *                          oracle is the plain definition, one breadth-first
 *                          search per vertex.
 *
 * Threads split the source list into contiguous static blocks; each thread
 * keeps private arrays and the per-thread scores are added in thread order,
 * so a given (input, thread count) always produces the same bits.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *reach;   /* NULL => all ones */
    const int32_t *ident;   /* NULL => all ones */
    const int32_t *sources; /* NULL => 0..n-1 */
    int64_t src_begin, src_end;
    int weighted;
    int classes;            /* reach holds the members' reach sum (oracle_bc_classes) */
    double *bc;             /* private accumulator, length n */
    int status;
} oracle_job;

/* Workspace of one source: the vertices in order of distance from the source
 * (and where each distance starts), and per vertex its distance d, path
 * count sigma and dependency delta. */
typedef struct {
    int32_t *order, *start, *d;
    double *sigma, *delta;
} oracle_ws;

static int ws_alloc(oracle_ws *w, int32_t n, int64_t arcs) {
    (void)arcs;
    size_t nn = n > 0 ? (size_t)n : 1;
    w->order = malloc(nn * sizeof(int32_t));
    w->start = malloc((nn + 2) * sizeof(int32_t));
    w->d = malloc(nn * sizeof(int32_t));
    w->sigma = malloc(nn * sizeof(double));
    w->delta = malloc(nn * sizeof(double));
    return w->order && w->start && w->d && w->sigma && w->delta;
}

static void ws_free(oracle_ws *w) {
    free(w->order); free(w->start); free(w->d); free(w->sigma); free(w->delta);
}

/*
 * One source s, distance by distance.
 *
 * Distances: a breadth-first search lists the vertices reachable from s in
 * non-decreasing distance (order[], with distance k occupying
 * order[start[k] .. start[k+1])).
 *
 * Path counts (Section 2.1), nearest first: sigma[s] = 1 and for every other
 * reached w, sigma[w] is the sum over its neighbours v one step closer to s
 * of the paths that reach v and can be continued through it: sigma[v], times
 * ident[v] when v != s stands for identical vertices (Section 3.3.3).
 *
 * Dependencies, farthest first, Eq. (3): delta[v] starts at the targets v
 * stands for besides itself -- reach[v]-1 in Algorithm 2 (Section 3.2.1), 0
 * in Algorithm 1 -- and adds, for every neighbour w one step farther from s,
 * sigma[v]/sigma[w] * ident[w] * (1 + delta[w]) (ident[w] = 1 without
 * identical vertices).  Every reached v != s then adds delta[v] to bc[v],
 * times the weight of the source: reach[s]*ident[s] (Algorithm 2 with
 * Section 3.3.3), or for oracle_bc_classes the members' reach sum reach[s],
 * the dependency then starting at the members' mean reach minus one.
 *
 * The arrays d/sigma/delta are left holding this source's values (d = -1 and
 * sigma = delta = 0 where s does not reach).
 */
static void one_source(const oracle_job *J, oracle_ws *w, int32_t s, double *bc) {
    const int32_t n = J->n;
    const int32_t *rp = J->row_ptr, *col = J->col;
    const int weighted = J->weighted;
    for (int32_t v = 0; v < n; ++v) {
        w->d[v] = -1;
        w->sigma[v] = 0.0;
        w->delta[v] = 0.0;
    }
    /* distances */
    int32_t cnt = 0, levels = 0;
    w->order[cnt++] = s;
    w->d[s] = 0;
    w->start[0] = 0;
    for (int32_t lo = 0; lo < cnt; ++levels) {
        const int32_t hi = cnt;
        w->start[levels + 1] = hi;
        for (int32_t k = lo; k < hi; ++k) {
            const int32_t v = w->order[k];
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
                if (w->d[col[e]] < 0) {
                    w->d[col[e]] = w->d[v] + 1;
                    w->order[cnt++] = col[e];
                }
        }
        lo = hi;
    }
    /* path counts, nearest first */
    w->sigma[s] = 1.0;
    for (int32_t k = 1; k < cnt; ++k) {
        const int32_t x = w->order[k];
        double paths = 0.0;
        for (int32_t e = rp[x]; e < rp[x + 1]; ++e) {
            const int32_t v = col[e];
            if (w->d[v] != w->d[x] - 1) continue;
            double through = w->sigma[v];
            if (weighted && J->ident && v != s) through *= (double)J->ident[v];
            paths += through;
        }
        w->sigma[x] = paths;
    }
    /* dependencies, farthest first, and the source's weight */
    double weight = 1.0;
    if (J->classes) weight = (double)J->reach[s];
    else if (weighted) weight = (J->reach ? (double)J->reach[s] : 1.0) * (J->ident ? (double)J->ident[s] : 1.0);
    for (int32_t k = cnt - 1; k >= 0; --k) {
        const int32_t v = w->order[k];
        double dv = 0.0;
        if (J->classes) dv = (double)J->reach[v] / (double)J->ident[v] - 1.0;
        else if (weighted && J->reach) dv = (double)(J->reach[v] - 1);
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            const int32_t x = col[e];
            if (w->d[x] != w->d[v] + 1) continue;
            const double kx = (weighted && J->ident) ? (double)J->ident[x] : 1.0;
            dv += w->sigma[v] / w->sigma[x] * kx * (1.0 + w->delta[x]);
        }
        w->delta[v] = dv;
        if (v != s && bc) bc[v] += weight * dv;
    }
}

static void *worker(void *arg) {
    oracle_job *J = (oracle_job *)arg;
    oracle_ws w;
    if (!ws_alloc(&w, J->n, J->n > 0 ? J->row_ptr[J->n] : 0)) {
        ws_free(&w);
        J->status = -7;
        return NULL;
    }
    for (int64_t i = J->src_begin; i < J->src_end; ++i) {
        int32_t s = J->sources ? J->sources[i] : (int32_t)i;
        one_source(J, &w, s, J->bc);
    }
    ws_free(&w);
    J->status = 0;
    return NULL;
}

static int run_threads_k(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *reach,
                         const int32_t *ident, int weighted, int classes, int64_t nsrc, const int32_t *sources,
                         int nthreads, double *bc_out);

static int run_threads(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *reach,
                       const int32_t *ident, int weighted, int64_t nsrc, const int32_t *sources,
                       int nthreads, double *bc_out) {
    return run_threads_k(n, row_ptr, col, reach, ident, weighted, 0, nsrc, sources, nthreads, bc_out);
}

static int run_threads_k(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *reach,
                         const int32_t *ident, int weighted, int classes, int64_t nsrc, const int32_t *sources,
                         int nthreads, double *bc_out) {
    if (n < 0 || !row_ptr || (n > 0 && !col) || !bc_out) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nsrc < nthreads) nthreads = nsrc > 0 ? (int)nsrc : 1;
    for (int32_t v = 0; v < n; ++v) bc_out[v] = 0.0;
    if (nsrc == 0 || n == 0) return 0;
    oracle_job *jobs = calloc((size_t)nthreads, sizeof(oracle_job));
    pthread_t *tid = calloc((size_t)nthreads, sizeof(pthread_t));
    double *acc = calloc((size_t)nthreads * (size_t)n, sizeof(double));
    if (!jobs || !tid || !acc) {
        free(jobs); free(tid); free(acc);
        return -7;
    }
    for (int t = 0; t < nthreads; ++t) {
        oracle_job *J = &jobs[t];
        J->n = n; J->row_ptr = row_ptr; J->col = col;
        J->reach = reach; J->ident = ident; J->sources = sources;
        J->weighted = weighted;
        J->classes = classes;
        J->src_begin = nsrc * t / nthreads;
        J->src_end = nsrc * (t + 1) / nthreads;
        J->bc = acc + (size_t)t * (size_t)n;
        J->status = -1;
    }
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&tid[t], NULL, worker, &jobs[t]) != 0) jobs[t].status = -99;
    worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t)
        if (jobs[t].status != -99) pthread_join(tid[t], NULL);
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].status == -99) worker(&jobs[t]); /* thread creation failed: run inline */
        if (jobs[t].status != 0) rc = jobs[t].status;
    }
    for (int t = 0; t < nthreads; ++t)
        for (int32_t v = 0; v < n; ++v) bc_out[v] += acc[(size_t)t * (size_t)n + v];
    free(jobs); free(tid); free(acc);
    return rc;
}

/* Algorithm 1 over all sources (sources == NULL) or the listed ones. */
int oracle_bc_plain(int32_t n, const int32_t *row_ptr, const int32_t *col, int64_t nsrc,
                    const int32_t *sources, int nthreads, double *bc_out) {
    if (!sources) nsrc = n;
    return run_threads(n, row_ptr, col, NULL, NULL, 0, nsrc, sources, nthreads, bc_out);
}

/* Algorithm 2 with identical-vertex weights; reach/ident may be NULL (= 1). */
int oracle_bc_weighted(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *reach,
                       const int32_t *ident, int64_t nsrc, const int32_t *sources, int nthreads,
                       double *bc_out) {
    if (!sources) nsrc = n;
    return run_threads(n, row_ptr, col, reach, ident, 1, nsrc, sources, nthreads, bc_out);
}

/* oracle_bc_weighted for class vertices: ident[v] members whose reaches sum
 * to reach[v] (both required, every reach[v] >= ident[v] >= 1). */
int oracle_bc_classes(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *reach,
                      const int32_t *ident, int nthreads, double *bc_out) {
    if (n > 0 && (!reach || !ident)) return -1;
    for (int32_t v = 0; v < n; ++v)
        if (ident[v] < 1 || reach[v] < ident[v]) return -1;
    return run_threads_k(n, row_ptr, col, reach, ident, 1, 1, n, NULL, nthreads, bc_out);
}

/* Levels (d, -1 when unreachable), path counts and dependencies of source s. */
int oracle_single_source(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *reach,
                         const int32_t *ident, int32_t s, int32_t *dist, double *sigma, double *delta) {
    if (n <= 0 || s < 0 || s >= n || !row_ptr || !col) return -1;
    oracle_job J;
    memset(&J, 0, sizeof J);
    J.n = n; J.row_ptr = row_ptr; J.col = col; J.reach = reach; J.ident = ident; J.weighted = 1;
    oracle_ws w;
    if (!ws_alloc(&w, n, row_ptr[n])) {
        ws_free(&w);
        return -7;
    }
    one_source(&J, &w, s, NULL);
    for (int32_t v = 0; v < n; ++v) {
        if (dist) dist[v] = w.d[v];
        if (sigma) sigma[v] = w.sigma[v];
        if (delta) delta[v] = w.delta[v];
    }
    ws_free(&w);
    return 0;
}

/*
 * Algorithm 2 with identical-vertex weights on every piece of a packed set of
 * pieces.  Piece p owns packed vertices [vtx_off[p], vtx_off[p+1]); row[] holds
 * arc offsets into col[] (absolute), col[] piece-local ids; reach/ident are per
 * packed vertex.  bc_out[V] receives, for each packed vertex, the sum over the
 * sources of its own piece -- the same quantity oracle_bc_weighted gives for
 * the piece on its own.
 *
 * Threads take contiguous ranges of packed source ids with about equal work
 * (arcs + vertices of the source's piece); each keeps a private accumulator
 * over the vertices of the pieces its range touches, and the accumulators are
 * added in thread order.
 */
typedef struct {
    const int32_t *vtx_off, *row, *col, *reach, *ident;
    int32_t P;
    int64_t g0, g1;      /* packed source ids [g0, g1) */
    int64_t span0;       /* first packed vertex of the accumulator */
    double *acc;         /* accumulator over [span0, span0 + span) */
    int32_t maxnp;
    int64_t maxarcs;
    int status;
} pieces_job;

static int32_t piece_of(const int32_t *vtx_off, int32_t P, int64_t g) {
    int32_t lo = 0, hi = P - 1;
    while (lo < hi) {               /* last p with vtx_off[p] <= g */
        int32_t mid = (lo + hi + 1) / 2;
        if (vtx_off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

static void *pieces_worker(void *arg) {
    pieces_job *J = (pieces_job *)arg;
    oracle_ws w;
    int32_t *rel = malloc(((size_t)J->maxnp + 1) * sizeof(int32_t));
    if (!rel || !ws_alloc(&w, J->maxnp, J->maxarcs)) {
        free(rel);
        J->status = -7;
        return NULL;
    }
    int64_t g = J->g0;
    while (g < J->g1) {
        int32_t p = piece_of(J->vtx_off, J->P, g);
        int32_t vb = J->vtx_off[p], np = J->vtx_off[p + 1] - vb;
        int64_t a0 = J->row[vb];
        for (int32_t v = 0; v <= np; ++v) rel[v] = (int32_t)(J->row[vb + v] - a0);
        oracle_job pj;
        memset(&pj, 0, sizeof pj);
        pj.n = np;
        pj.row_ptr = rel;
        pj.col = J->col + a0;
        pj.reach = J->reach ? J->reach + vb : NULL;
        pj.ident = J->ident ? J->ident + vb : NULL;
        pj.weighted = 1;
        int64_t gend = (int64_t)vb + np < J->g1 ? (int64_t)vb + np : J->g1;
        double *acc = J->acc + ((int64_t)vb - J->span0);
        for (; g < gend; ++g) one_source(&pj, &w, (int32_t)(g - vb), acc);
    }
    ws_free(&w);
    free(rel);
    J->status = 0;
    return NULL;
}

int oracle_bc_pieces(int32_t P, const int32_t *vtx_off, const int32_t *row, const int32_t *col,
                     const int32_t *reach, const int32_t *ident, int nthreads, double *bc_out) {
    if (P < 0 || !vtx_off || !row || !bc_out) return -1;
    int64_t V = P > 0 ? vtx_off[P] : 0;
    for (int64_t v = 0; v < V; ++v) bc_out[v] = 0.0;
    if (V == 0) return 0;
    int32_t maxnp = 1;
    int64_t maxarcs = 1;
    double total = 0.0;
    for (int32_t p = 0; p < P; ++p) {
        int32_t np = vtx_off[p + 1] - vtx_off[p];
        int64_t arcs = (int64_t)row[vtx_off[p + 1]] - row[vtx_off[p]];
        if (np > maxnp) maxnp = np;
        if (arcs > maxarcs) maxarcs = arcs;
        total += (double)np * (double)(arcs + np);
    }
    if (nthreads < 1) nthreads = 1;
    if ((int64_t)nthreads > V) nthreads = (int)V;
    pieces_job *jobs = calloc((size_t)nthreads, sizeof(pieces_job));
    pthread_t *tid = calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs); free(tid);
        return -7;
    }
    /* equal-work ranges of packed source ids */
    int64_t g = 0;
    double done = 0.0;
    int32_t p = 0;
    for (int t = 0; t < nthreads; ++t) {
        pieces_job *J = &jobs[t];
        J->vtx_off = vtx_off; J->row = row; J->col = col; J->reach = reach; J->ident = ident;
        J->P = P; J->maxnp = maxnp; J->maxarcs = maxarcs; J->status = -1;
        J->g0 = g;
        double target = total * (double)(t + 1) / (double)nthreads;
        while (g < V && (t == nthreads - 1 || done < target)) {
            while (vtx_off[p + 1] <= g) ++p;
            int32_t np = vtx_off[p + 1] - vtx_off[p];
            int64_t arcs = (int64_t)row[vtx_off[p + 1]] - row[vtx_off[p]];
            done += (double)(arcs + np);
            ++g;
        }
        J->g1 = g;
    }
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        pieces_job *J = &jobs[t];
        if (J->g1 > J->g0) {
            int32_t pa = piece_of(vtx_off, P, J->g0), pb = piece_of(vtx_off, P, J->g1 - 1);
            J->span0 = vtx_off[pa];
            J->acc = calloc((size_t)(vtx_off[pb + 1] - vtx_off[pa]), sizeof(double));
            if (!J->acc) rc = -7;
        }
    }
    if (rc == 0) {
        for (int t = 1; t < nthreads; ++t)
            if (jobs[t].g1 > jobs[t].g0 && pthread_create(&tid[t], NULL, pieces_worker, &jobs[t]) != 0)
                jobs[t].status = -99;
        if (jobs[0].g1 > jobs[0].g0) pieces_worker(&jobs[0]);
        for (int t = 1; t < nthreads; ++t)
            if (jobs[t].g1 > jobs[t].g0 && jobs[t].status != -99) pthread_join(tid[t], NULL);
        for (int t = 0; t < nthreads; ++t) {
            pieces_job *J = &jobs[t];
            if (J->g1 <= J->g0) continue;
            if (J->status == -99) pieces_worker(J); /* thread creation failed: run inline */
            if (J->status != 0) rc = J->status;
        }
        for (int t = 0; t < nthreads && rc == 0; ++t) {
            pieces_job *J = &jobs[t];
            if (J->g1 <= J->g0) continue;
            int32_t pb = piece_of(vtx_off, P, J->g1 - 1);
            for (int64_t v = J->span0; v < vtx_off[pb + 1]; ++v) bc_out[v] += J->acc[v - J->span0];
        }
    }
    for (int t = 0; t < nthreads; ++t) free(jobs[t].acc);
    free(jobs); free(tid);
    return rc;
}

/*
 * Algorithm 3 (Bfs-Side, Section 3.3.2) for the side vertices sides[0..nside)
 * of an attributed graph (reach, no ident), removed one after another in that
 * order.  Side vertex sides[i] is removed from the graph left after removing
 * sides[0..i-1], so its breadth-first search runs on that graph: the earlier
 * ones are skipped as if deleted.  With delta from the search (initialised
 * to reach-1 as in Algorithm 2), every vertex w != sides[i] of that graph gets
 *   reach[s]*delta[w] + reach[s]*(delta[w] - (reach[w]-1))
 * -- the dependencies of the sources s stands for, and those of the pairs
 * whose target s stands for, which the smaller graph can no longer see.
 * The searches of different i are independent given i, so threads take
 * contiguous ranges of i.
 */
typedef struct {
    const int32_t *row_ptr, *col, *reach, *sides, *rank;
    int32_t n;
    int64_t i0, i1;
    double *acc;
    int status;
} side_job;

static void *side_worker(void *arg) {
    side_job *J = (side_job *)arg;
    const int32_t n = J->n;
    int32_t *Q = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *d = malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    double *sigma = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *delta = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!Q || !d || !sigma || !delta) {
        free(Q); free(d); free(sigma); free(delta);
        J->status = -7;
        return NULL;
    }
    for (int64_t i = J->i0; i < J->i1; ++i) {
        const int32_t s = J->sides[i];
        /* vertex v is still present iff it is not a side vertex removed before s */
        for (int32_t v = 0; v < n; ++v) {
            d[v] = -1;
            sigma[v] = 0.0;
        }
        int32_t qh = 0, qt = 0;
        Q[qt++] = s;
        d[s] = 0;
        sigma[s] = 1.0;
        while (qh < qt) {
            const int32_t v = Q[qh++];
            for (int32_t e = J->row_ptr[v]; e < J->row_ptr[v + 1]; ++e) {
                const int32_t x = J->col[e];
                if (J->rank[x] < i) continue;                /* removed earlier */
                if (d[x] < 0) {
                    d[x] = d[v] + 1;
                    Q[qt++] = x;
                }
                if (d[x] == d[v] + 1) sigma[x] += sigma[v];
            }
        }
        /* back propagation in reverse BFS order: each vertex takes its
           dependency from its successors */
        for (int32_t k = qt - 1; k >= 0; --k) {
            const int32_t v = Q[k];
            double dv = (double)(J->reach[v] - 1);
            for (int32_t e = J->row_ptr[v]; e < J->row_ptr[v + 1]; ++e) {
                const int32_t x = J->col[e];
                if (J->rank[x] < i) continue;
                if (d[x] == d[v] + 1) dv += sigma[v] / sigma[x] * (1.0 + delta[x]);
            }
            delta[v] = dv;
            if (v != s) {
                const double rs = (double)J->reach[s];
                J->acc[v] += rs * dv + rs * (dv - (double)(J->reach[v] - 1));
            }
        }
    }
    free(Q); free(d); free(sigma); free(delta);
    J->status = 0;
    return NULL;
}

int oracle_bc_side(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *reach, int64_t nside,
                   const int32_t *sides, int nthreads, double *bc_out) {
    if (n < 0 || !row_ptr || (n > 0 && !col) || !reach || !bc_out || nside < 0 || (nside > 0 && !sides)) return -1;
    for (int32_t v = 0; v < n; ++v) bc_out[v] = 0.0;
    if (nside == 0 || n == 0) return 0;
    int32_t *rank = malloc((size_t)n * sizeof(int32_t));
    if (!rank) return -7;
    for (int32_t v = 0; v < n; ++v) rank[v] = INT32_MAX;
    for (int64_t i = 0; i < nside; ++i) {
        if (sides[i] < 0 || sides[i] >= n || rank[sides[i]] != INT32_MAX) {
            free(rank);
            return -1;
        }
        rank[sides[i]] = (int32_t)i;
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > nside) nthreads = (int)nside;
    side_job *jobs = calloc((size_t)nthreads, sizeof(side_job));
    pthread_t *tid = calloc((size_t)nthreads, sizeof(pthread_t));
    double *acc = calloc((size_t)nthreads * (size_t)n, sizeof(double));
    if (!jobs || !tid || !acc) {
        free(rank); free(jobs); free(tid); free(acc);
        return -7;
    }
    for (int t = 0; t < nthreads; ++t) {
        side_job *J = &jobs[t];
        J->row_ptr = row_ptr; J->col = col; J->reach = reach; J->sides = sides; J->rank = rank; J->n = n;
        J->i0 = nside * t / nthreads;
        J->i1 = nside * (t + 1) / nthreads;
        J->acc = acc + (size_t)t * (size_t)n;
        J->status = -1;
    }
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&tid[t], NULL, side_worker, &jobs[t]) != 0) jobs[t].status = -99;
    side_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t)
        if (jobs[t].status != -99) pthread_join(tid[t], NULL);
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].status == -99) side_worker(&jobs[t]);
        if (jobs[t].status != 0) rc = jobs[t].status;
    }
    for (int t = 0; t < nthreads; ++t)
        for (int32_t v = 0; v < n; ++v) bc_out[v] += acc[(size_t)t * (size_t)n + v];
    free(rank); free(jobs); free(tid); free(acc);
    return rc;
}


/* ---------------------------------------------------------------------------
 * Weighted farness per piece: one breadth-first search per vertex, summing
 * weight[y] * level(y) over the vertices it reaches.  int64 throughout, so the
 * result is exact (the caller keeps weight * distance sums below 2^63).
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t P;
    const int32_t *vtx_off, *row, *col, *weight;
    int64_t g0, g1; /* packed vertices of this thread (indexes into `sources` when it is set) */
    const int32_t *sources; /* one piece only: the vertices to search from, or NULL for all */
    int64_t *out;
    int status;
} far_job;

static void *far_worker(void *arg) {
    far_job *J = (far_job *)arg;
    int32_t maxn = 0;
    for (int32_t p = 0; p < J->P; ++p)
        if (J->vtx_off[p + 1] - J->vtx_off[p] > maxn) maxn = J->vtx_off[p + 1] - J->vtx_off[p];
    size_t nn = maxn > 0 ? (size_t)maxn : 1;
    int32_t *Q = malloc(nn * sizeof(int32_t));
    int32_t *d = malloc(nn * sizeof(int32_t));
    if (!Q || !d) {
        free(Q); free(d);
        J->status = -7;
        return NULL;
    }
    int32_t p = (J->g0 < J->g1 && !J->sources) ? piece_of(J->vtx_off, J->P, J->g0) : 0;
    for (int64_t k = J->g0; k < J->g1; ++k) {
        const int64_t g = J->sources ? J->sources[k] : k;
        while (g >= J->vtx_off[p + 1]) ++p;
        const int32_t vb = J->vtx_off[p], np = J->vtx_off[p + 1] - vb;
        const int32_t *rp = J->row + vb;
        for (int32_t v = 0; v < np; ++v) d[v] = -1;
        const int32_t s = (int32_t)(g - vb);
        int64_t sum = 0;
        int32_t qh = 0, qt = 0;
        Q[qt++] = s;
        d[s] = 0;
        while (qh < qt) {
            const int32_t v = Q[qh++];
            sum += (int64_t)d[v] * (J->weight ? (int64_t)J->weight[vb + v] : 1);
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int32_t w = J->col[e];
                if (w < 0 || w >= np) {
                    free(Q); free(d);
                    J->status = -5;
                    return NULL;
                }
                if (d[w] < 0) {
                    d[w] = d[v] + 1;
                    Q[qt++] = w;
                }
            }
        }
        J->out[k] = sum;
    }
    free(Q); free(d);
    J->status = 0;
    return NULL;
}

static int far_run(int32_t P, const int32_t *vtx_off, const int32_t *row, const int32_t *col, const int32_t *weight,
                   int64_t nsrc, const int32_t *sources, int nthreads, int64_t *out) {
    if (P < 0 || (P > 0 && (!vtx_off || !row || !out))) return -1;
    if (P == 0) return 0;
    for (int32_t p = 0; p < P; ++p)
        if (vtx_off[p + 1] < vtx_off[p]) return -1;
    if (vtx_off[P] == 0) return 0;
    if (!col && row[vtx_off[P]] > row[0]) return -1;
    if (sources)
        for (int64_t k = 0; k < nsrc; ++k)
            if (sources[k] < 0 || sources[k] >= vtx_off[P]) return -1;
    const int64_t V = sources ? nsrc : vtx_off[P];
    if (V == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > V) nthreads = (int)V;
    far_job *jobs = calloc((size_t)nthreads, sizeof(far_job));
    pthread_t *tid = calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs); free(tid);
        return -7;
    }
    for (int t = 0; t < nthreads; ++t) {
        far_job *J = &jobs[t];
        J->P = P; J->vtx_off = vtx_off; J->row = row; J->col = col; J->weight = weight; J->out = out;
        J->sources = sources;
        J->g0 = V * t / nthreads;
        J->g1 = V * (t + 1) / nthreads;
        J->status = -1;
    }
    for (int t = 1; t < nthreads; ++t)
        if (pthread_create(&tid[t], NULL, far_worker, &jobs[t]) != 0) jobs[t].status = -99;
    far_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t)
        if (jobs[t].status != -99) pthread_join(tid[t], NULL);
    int rc = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].status == -99) far_worker(&jobs[t]);
        if (jobs[t].status != 0) rc = jobs[t].status;
    }
    free(jobs); free(tid);
    return rc;
}

int oracle_farness_pieces(int32_t P, const int32_t *vtx_off, const int32_t *row, const int32_t *col,
                          const int32_t *weight, int nthreads, int64_t *out) {
    return far_run(P, vtx_off, row, col, weight, 0, NULL, nthreads, out);
}

/* One graph (row_ptr[n+1], col), the farness of the listed sources only:
 * out[k] belongs to sources[k]. */
int oracle_farness_sources(int32_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *weight,
                           int64_t nsrc, const int32_t *sources, int nthreads, int64_t *out) {
    if (n < 0 || nsrc < 0 || (nsrc > 0 && !sources)) return -1;
    if (n == 0 || nsrc == 0) return 0;
    const int32_t vtx_off[2] = {0, n};
    return far_run(1, vtx_off, row_ptr, col, weight, nsrc, sources, nthreads, out);
}
