/*
 * FP64 CPU oracle for the QAOA MaxCut energy expectation of
 * "Performance Evaluation and Acceleration of the QTensor Quantum Circuit
 * Simulator on GPUs" (arXiv 2204.06045).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or helper with the HIP library it checks.
 *
 * Everything is plain C99 in double and double complex, written for a reader
 * to check against the paper by eye:
 *
 *   qtno_statevector_zz   <Z_j Z_k> from the full 2^N state (Sec. II-A,
 *                         Eq. 1 and Eq. 2), the plain definition.
 *   qtno_p1_closed_form   the depth-1 closed form of Wang, Hadfield, Jiang
 *                         and Rieffel (PRA 97, 022304, 2018), a published
 *                         result used as an independent pin.
 *   qtno_edge_zz          one light-cone tensor network (Sec. II-B) contracted
 *                         by bucket elimination (Sec. II-B), one bucket index
 *                         at a time, in the plain loop order.
 *   qtno_edge_zz_bruteforce  the same network summed over every assignment.
 *   qtno_energy           Sec. II-B energy identity over all edges,
 *                         E = |E|/2 - 1/2 sum_jk e_jk.
 *   qtno_contract_bucket  one bucket (or a merged group, Sec. II-C) from
 *                         caller-given tensors, for per-kernel checks.
 *
 * Readings where the paper is silent (all listed with the design notes):
 *   - mixer exp(-i beta X) per qubit, cost phase exp(-i gamma [z_a != z_b])
 *     per edge (Eq. 1, Eq. 2);
 *   - the light cone of edge (j,k) at layer l keeps mixers on vertices within
 *     distance p-l of {j,k} and cost gates on edges with an endpoint there
 *     (the reverse light cone behind the cancellation argument of Sec. II-B);
 *   - greedy min-fill elimination order, ties by current degree, then by
 *     variable id (variables numbered in creation order).
 *
 * Parity pins live in the tests: statevector against the closed form and the
 * closed-form optimum 0.6924 printed in Sec. II-A, statevector against a
 * dense-matrix exponential, bucket elimination against the statevector and the
 * brute-force network sum, order independence, light-cone forms against each
 * other, and the energy invariants.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define QTNO_OK 0
#define QTNO_EINVAL (-1)
#define QTNO_ERANGE (-2)
#define QTNO_ENOMEM (-3)

static __thread char g_err[256];

static int fail(int code, const char *msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

const char *qtno_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ graph */

static int check_graph(int n, int m, const int *edges)
{
    if (n < 2 || m < 1 || !edges)
        return fail(QTNO_EINVAL, "graph needs n >= 2 and m >= 1");
    for (int e = 0; e < m; e++) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b)
            return fail(QTNO_EINVAL, "edge endpoint out of range or self-loop");
        for (int f = 0; f < e; f++) {
            int c = edges[2 * f], d = edges[2 * f + 1];
            if ((a == c && b == d) || (a == d && b == c))
                return fail(QTNO_EINVAL, "repeated edge");
        }
    }
    return QTNO_OK;
}

/* Breadth-first distance of every vertex from the set {j, k}; -1 if
 * unreachable. */
static void distances(int n, int m, const int *edges, int j, int k, int *dist)
{
    int *queue = malloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; v++)
        dist[v] = -1;
    int head = 0, tail = 0;
    dist[j] = 0;
    queue[tail++] = j;
    if (dist[k] < 0) {
        dist[k] = 0;
        queue[tail++] = k;
    }
    while (head < tail) {
        int u = queue[head++];
        for (int e = 0; e < m; e++) {
            int a = edges[2 * e], b = edges[2 * e + 1], w = -1;
            if (a == u)
                w = b;
            else if (b == u)
                w = a;
            if (w >= 0 && dist[w] < 0) {
                dist[w] = dist[u] + 1;
                queue[tail++] = w;
            }
        }
    }
    free(queue);
}

/* ---------------------------------------------------------------- network */

typedef struct {
    int rank;
    int *idx;   /* variable ids; idx[0] is the most significant axis */
    cplx *data; /* 2^rank entries, row-major */
} otensor;

typedef struct {
    int n_vars;
    int n_tensors, cap;
    otensor *t;
} onet;

static void net_free(onet *net)
{
    for (int i = 0; i < net->n_tensors; i++) {
        free(net->t[i].idx);
        free(net->t[i].data);
    }
    free(net->t);
    memset(net, 0, sizeof *net);
}

static void net_add(onet *net, int rank, const int *idx, const cplx *data)
{
    if (net->n_tensors == net->cap) {
        net->cap = net->cap ? 2 * net->cap : 64;
        net->t = realloc(net->t, sizeof(otensor) * (size_t)net->cap);
    }
    otensor *t = &net->t[net->n_tensors++];
    t->rank = rank;
    t->idx = malloc(sizeof(int) * (size_t)(rank > 0 ? rank : 1));
    t->data = malloc(sizeof(cplx) * ((size_t)1 << rank));
    for (int i = 0; i < rank; i++)
        t->idx[i] = idx[i];
    for (size_t i = 0; i < ((size_t)1 << rank); i++)
        t->data[i] = data[i];
}

/*
 * The tensor network of <+| U^dagger Z_j Z_k U |+> restricted to the light
 * cone of edge (j,k).  Qubit values are binary variables; a variable lives
 * from one mixer to the next.
 *
 *   ket:  h(x) = 1/sqrt2 on each starting variable;
 *         layer l = 1..p: cost phase P_l(x_a, x_b) = exp(-i gamma_l [x_a != x_b])
 *         for each kept edge, then for each kept mixer qubit a new variable x'
 *         and R_l(x', x) = <x'| exp(-i beta_l X) |x> = cos beta_l (x' == x),
 *         -i sin beta_l (x' != x);
 *   observable: Z(x_j) Z(x_k), Z(x) = 1 - 2x, on the final variables;
 *   bra:  the same gates conjugated, walked from layer p down to 1, sharing
 *         the final variables with the ket.
 *
 * mode 0: reverse light cone, mixers of layer l on {dist <= p-l}, cost gates
 *         of layer l on edges with an endpoint at dist <= p-l;
 * mode 1: the subgraph S of edges with an endpoint at dist <= p-1 on every
 *         layer and mixers on every vertex of S (literal reading of Sec. II-B);
 * mode 2: the whole graph on every layer (no light cone).
 */
static int build_network(int n, int m, const int *edges, int edge_id, int p,
                         const double *gamma, const double *beta, int mode,
                         onet *net)
{
    memset(net, 0, sizeof *net);
    if (edge_id < 0 || edge_id >= m)
        return fail(QTNO_EINVAL, "edge id out of range");
    if (p < 1)
        return fail(QTNO_EINVAL, "p must be >= 1");
    if (mode < 0 || mode > 2)
        return fail(QTNO_EINVAL, "mode must be 0, 1 or 2");
    int j = edges[2 * edge_id], k = edges[2 * edge_id + 1];
    int *dist = malloc(sizeof(int) * (size_t)n);
    distances(n, m, edges, j, k, dist);

    int *qubit = calloc((size_t)n, sizeof(int));
    for (int q = 0; q < n; q++)
        qubit[q] = (mode == 2) ? 1 : (dist[q] >= 0 && dist[q] <= p);

    int *cur = malloc(sizeof(int) * (size_t)n);
    const double r2 = 1.0 / sqrt(2.0);
    const cplx hdat[2] = {r2, r2};
    for (int q = 0; q < n; q++) {
        cur[q] = -1;
        if (qubit[q]) {
            cur[q] = net->n_vars++;
            net_add(net, 1, &cur[q], hdat);
        }
    }

    /* which mixers / cost gates belong to layer l (1-based) */
#define MIXER_IN(q, l)                                                        \
    (mode == 2 ? 1                                                            \
               : (mode == 1 ? qubit[q]                                        \
                            : (dist[q] >= 0 && dist[q] <= p - (l))))
#define EDGE_IN(a, b, l)                                                      \
    (mode == 2 ? 1                                                            \
               : ((dist[a] >= 0 && dist[a] <= p - (mode == 1 ? 1 : (l))) ||   \
                  (dist[b] >= 0 && dist[b] <= p - (mode == 1 ? 1 : (l)))))

    for (int l = 1; l <= p; l++) {
        cplx ph = cexp(-I * gamma[l - 1]);
        cplx pdat[4] = {1.0, ph, ph, 1.0};
        for (int e = 0; e < m; e++) {
            int a = edges[2 * e], b = edges[2 * e + 1];
            if (EDGE_IN(a, b, l)) {
                int ix[2] = {cur[a], cur[b]};
                net_add(net, 2, ix, pdat);
            }
        }
        double c = cos(beta[l - 1]), s = sin(beta[l - 1]);
        cplx rdat[4] = {c, -I * s, -I * s, c};
        for (int q = 0; q < n; q++) {
            if (qubit[q] && MIXER_IN(q, l)) {
                int nv = net->n_vars++;
                int ix[2] = {nv, cur[q]};
                net_add(net, 2, ix, rdat);
                cur[q] = nv;
            }
        }
    }

    const cplx zdat[2] = {1.0, -1.0};
    net_add(net, 1, &cur[j], zdat);
    net_add(net, 1, &cur[k], zdat);

    for (int l = p; l >= 1; l--) {
        double c = cos(beta[l - 1]), s = sin(beta[l - 1]);
        cplx rdat[4] = {c, I * s, I * s, c}; /* conj(R_l) */
        for (int q = 0; q < n; q++) {
            if (qubit[q] && MIXER_IN(q, l)) {
                int nv = net->n_vars++;
                int ix[2] = {cur[q], nv}; /* (later, earlier) in time */
                net_add(net, 2, ix, rdat);
                cur[q] = nv;
            }
        }
        cplx ph = cexp(I * gamma[l - 1]); /* conj(P_l) */
        cplx pdat[4] = {1.0, ph, ph, 1.0};
        for (int e = 0; e < m; e++) {
            int a = edges[2 * e], b = edges[2 * e + 1];
            if (EDGE_IN(a, b, l)) {
                int ix[2] = {cur[a], cur[b]};
                net_add(net, 2, ix, pdat);
            }
        }
    }
#undef MIXER_IN
#undef EDGE_IN

    for (int q = 0; q < n; q++)
        if (qubit[q])
            net_add(net, 1, &cur[q], hdat);

    free(cur);
    free(qubit);
    free(dist);
    return QTNO_OK;
}

/* -------------------------------------------------------------- min-fill */

/* Greedy min-fill on the interaction graph of the network (one vertex per
 * variable, a clique per tensor).  Ties: fewest remaining neighbours, then
 * smallest variable id. */
static void minfill_order(const onet *net, int *order)
{
    int n = net->n_vars;
    unsigned char *adj = calloc((size_t)n * (size_t)n, 1);
    unsigned char *gone = calloc((size_t)n, 1);
    int *nb = malloc(sizeof(int) * (size_t)n);
    for (int t = 0; t < net->n_tensors; t++)
        for (int a = 0; a < net->t[t].rank; a++)
            for (int b = 0; b < net->t[t].rank; b++) {
                int u = net->t[t].idx[a], v = net->t[t].idx[b];
                if (u != v)
                    adj[(size_t)u * n + v] = 1;
            }
    for (int step = 0; step < n; step++) {
        int best = -1;
        long best_fill = 0;
        int best_deg = 0;
        for (int v = 0; v < n; v++) {
            if (gone[v])
                continue;
            int deg = 0;
            for (int u = 0; u < n; u++)
                if (!gone[u] && adj[(size_t)v * n + u])
                    nb[deg++] = u;
            long fill = 0;
            for (int a = 0; a < deg; a++)
                for (int b = a + 1; b < deg; b++)
                    if (!adj[(size_t)nb[a] * n + nb[b]])
                        fill++;
            if (best < 0 || fill < best_fill ||
                (fill == best_fill && deg < best_deg)) {
                best = v;
                best_fill = fill;
                best_deg = deg;
            }
        }
        int deg = 0;
        for (int u = 0; u < n; u++)
            if (!gone[u] && adj[(size_t)best * n + u])
                nb[deg++] = u;
        for (int a = 0; a < deg; a++)
            for (int b = 0; b < deg; b++)
                if (a != b)
                    adj[(size_t)nb[a] * n + nb[b]] = 1;
        gone[best] = 1;
        order[step] = best;
    }
    free(nb);
    free(gone);
    free(adj);
}

/* ------------------------------------------------------ bucket elimination */

typedef struct {
    int *ids;
    int n, cap;
} ilist;

static void ilist_push(ilist *l, int x)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 8;
        l->ids = realloc(l->ids, sizeof(int) * (size_t)l->cap);
    }
    l->ids[l->n++] = x;
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* The element of tensor t at union assignment ux (union U of width w,
 * U[0] the most significant bit of ux). upos[q] is the position in U of
 * t->idx[q]. */
static cplx tensor_at(const otensor *t, const int *upos, int w, uint64_t ux)
{
    uint64_t off = 0;
    for (int q = 0; q < t->rank; q++)
        off |= ((ux >> (w - 1 - upos[q])) & 1u) << (t->rank - 1 - q);
    return t->data[off];
}

/*
 * Bucket elimination (Sec. II-B).  Every tensor goes to the bucket of its
 * earliest-eliminated index.  Buckets are taken in order; a non-empty bucket
 * with bucket index v and index union U is replaced by
 *     out[U \ {v}] = sum_{v in {0,1}} prod_{t in bucket} t[U_t]
 * (v = 0 first, tensors in the order they entered the bucket), and out goes
 * to the bucket of its earliest remaining index, or, with no index left, is
 * multiplied into the network's scalar.
 * widths_out[i] receives the width |U| of bucket i (0 when empty).
 */
static int eliminate(onet *net, const int *order, cplx *value, int *widths_out,
                     int max_width)
{
    int n = net->n_vars;
    int *pos = malloc(sizeof(int) * (size_t)n);
    for (int v = 0; v < n; v++)
        pos[v] = -1;
    for (int i = 0; i < n; i++) {
        if (order[i] < 0 || order[i] >= n || pos[order[i]] >= 0) {
            free(pos);
            return fail(QTNO_EINVAL, "order is not a permutation of the variables");
        }
        pos[order[i]] = i;
    }
    ilist *bucket = calloc((size_t)n, sizeof(ilist));
    /* tensors owned here: the network's gates, then intermediates */
    int n_all = net->n_tensors, cap_all = net->n_tensors + n + 1;
    otensor *all = malloc(sizeof(otensor) * (size_t)cap_all);
    for (int t = 0; t < net->n_tensors; t++) {
        all[t] = net->t[t];
        net->t[t].idx = NULL;
        net->t[t].data = NULL;
    }
    cplx scalar = 1.0;
    int rc = QTNO_OK;

    for (int t = 0; t < n_all; t++) {
        if (all[t].rank == 0) {
            scalar *= all[t].data[0];
            continue;
        }
        int b = pos[all[t].idx[0]];
        for (int q = 1; q < all[t].rank; q++)
            if (pos[all[t].idx[q]] < b)
                b = pos[all[t].idx[q]];
        ilist_push(&bucket[b], t);
    }

    int *uni = malloc(sizeof(int) * (size_t)n);
    /* 64 slots per operand: an operand's rank never exceeds the width cap */
    int *upos = malloc(sizeof(int) * (size_t)cap_all * 64);
    for (int i = 0; i < n; i++) {
        if (widths_out)
            widths_out[i] = 0;
        ilist *bk = &bucket[i];
        if (bk->n == 0)
            continue;
        int v = order[i];
        /* union of the bucket's indices, ascending by variable id */
        int w = 0;
        for (int a = 0; a < bk->n; a++) {
            otensor *t = &all[bk->ids[a]];
            for (int q = 0; q < t->rank; q++) {
                int seen = 0;
                for (int u = 0; u < w; u++)
                    if (uni[u] == t->idx[q])
                        seen = 1;
                if (!seen)
                    uni[w++] = t->idx[q];
            }
        }
        qsort(uni, (size_t)w, sizeof(int), cmp_int);
        if (widths_out)
            widths_out[i] = w;
        if (w > max_width) {
            rc = fail(QTNO_ERANGE, "bucket width over the cap");
            break;
        }
        int pv = 0;
        while (uni[pv] != v)
            pv++;
        /* positions in U of every operand index */
        for (int a = 0; a < bk->n; a++) {
            otensor *t = &all[bk->ids[a]];
            for (int q = 0; q < t->rank; q++)
                for (int u = 0; u < w; u++)
                    if (uni[u] == t->idx[q])
                        upos[a * 64 + q] = u;
        }
        int ro = w - 1;
        uint64_t nout = (uint64_t)1 << ro;
        cplx *out = malloc(sizeof(cplx) * nout);
        int *oidx = malloc(sizeof(int) * (size_t)(ro > 0 ? ro : 1));
        if (!out || !oidx) {
            free(out);
            free(oidx);
            rc = fail(QTNO_ENOMEM, "host allocation failed");
            break;
        }
        for (int u = 0, q = 0; u < w; u++)
            if (u != pv)
                oidx[q++] = uni[u];
        int bv = w - 1 - pv; /* bit of v in the union index */
        for (uint64_t o = 0; o < nout; o++) {
            uint64_t hi = (o >> bv) << (bv + 1), lo = o & (((uint64_t)1 << bv) - 1);
            cplx acc = 0.0;
            for (uint64_t xv = 0; xv < 2; xv++) {
                uint64_t ux = hi | (xv << bv) | lo;
                cplx prod = 1.0;
                for (int a = 0; a < bk->n; a++)
                    prod *= tensor_at(&all[bk->ids[a]], &upos[a * 64], w, ux);
                acc += prod;
            }
            out[o] = acc;
        }
        for (int a = 0; a < bk->n; a++) {
            otensor *t = &all[bk->ids[a]];
            free(t->idx);
            free(t->data);
            t->idx = NULL;
            t->data = NULL;
        }
        if (ro == 0) {
            scalar *= out[0];
            free(out);
            free(oidx);
            continue;
        }
        int nt = n_all++;
        all[nt].rank = ro;
        all[nt].idx = oidx;
        all[nt].data = out;
        int b = pos[oidx[0]];
        for (int q = 1; q < ro; q++)
            if (pos[oidx[q]] < b)
                b = pos[oidx[q]];
        ilist_push(&bucket[b], nt);
    }
    *value = scalar;
    for (int t = 0; t < n_all; t++) {
        free(all[t].idx);
        free(all[t].data);
    }
    free(all);
    for (int i = 0; i < n; i++)
        free(bucket[i].ids);
    free(bucket);
    free(uni);
    free(upos);
    free(pos);
    return rc;
}

/* ------------------------------------------------------------- public ABI */

int qtno_lightcone_size(int n, int m, const int *edges, int edge_id, int p,
                        int mode, int *n_vars, int *n_tensors)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    double *zero = calloc((size_t)(p > 0 ? p : 1), sizeof(double));
    onet net;
    rc = build_network(n, m, edges, edge_id, p, zero, zero, mode, &net);
    free(zero);
    if (rc)
        return rc;
    if (n_vars)
        *n_vars = net.n_vars;
    if (n_tensors)
        *n_tensors = net.n_tensors;
    net_free(&net);
    return QTNO_OK;
}

/*
 * e_jk of edge `edge_id` by bucket elimination.
 * order_kind 0: greedy min-fill; 1: min-fill reversed; 2: `order` as given
 * (a permutation of the network's variables, numbered in creation order).
 * widths_out (optional, n_vars entries) gets each bucket's width.
 */
int qtno_edge_zz(int n, int m, const int *edges, int edge_id, int p,
                 const double *gamma, const double *beta, int mode,
                 int order_kind, const int *order, int max_width, double *re,
                 double *im, int *widths_out)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    if (!gamma || !beta)
        return fail(QTNO_EINVAL, "angles are NULL");
    onet net;
    rc = build_network(n, m, edges, edge_id, p, gamma, beta, mode, &net);
    if (rc)
        return rc;
    int *ord = malloc(sizeof(int) * (size_t)net.n_vars);
    if (order_kind == 2) {
        if (!order) {
            net_free(&net);
            free(ord);
            return fail(QTNO_EINVAL, "order_kind 2 needs an order");
        }
        memcpy(ord, order, sizeof(int) * (size_t)net.n_vars);
    } else {
        minfill_order(&net, ord);
        if (order_kind == 1)
            for (int a = 0, b = net.n_vars - 1; a < b; a++, b--) {
                int t = ord[a];
                ord[a] = ord[b];
                ord[b] = t;
            }
    }
    cplx val = 0.0;
    rc = eliminate(&net, ord, &val, widths_out, max_width > 0 ? max_width : 34);
    free(ord);
    net_free(&net);
    if (rc)
        return rc;
    *re = creal(val);
    *im = cimag(val);
    return QTNO_OK;
}

/* The oracle's min-fill order for one light cone (n_vars entries). */
int qtno_edge_order(int n, int m, const int *edges, int edge_id, int p,
                    int mode, int *order_out)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    double *zero = calloc((size_t)(p > 0 ? p : 1), sizeof(double));
    onet net;
    rc = build_network(n, m, edges, edge_id, p, zero, zero, mode, &net);
    free(zero);
    if (rc)
        return rc;
    minfill_order(&net, order_out);
    net_free(&net);
    return QTNO_OK;
}

/* Bucket widths of one light cone under the oracle's min-fill order, from the
 * index sets alone (no arithmetic): widths_out[i] is the width of the bucket
 * at elimination position i, 0 when empty.  Used to scale timed samples. */
int qtno_edge_widths(int n, int m, const int *edges, int edge_id, int p,
                     int mode, int *widths_out)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    double *zero = calloc((size_t)(p > 0 ? p : 1), sizeof(double));
    onet net;
    rc = build_network(n, m, edges, edge_id, p, zero, zero, mode, &net);
    free(zero);
    if (rc)
        return rc;
    int nv = net.n_vars;
    int *ord = malloc(sizeof(int) * (size_t)nv);
    int *pos = malloc(sizeof(int) * (size_t)nv);
    minfill_order(&net, ord);
    for (int i = 0; i < nv; i++)
        pos[ord[i]] = i;
    /* index sets as bitmaps over variables, one per live tensor */
    int words = (nv + 63) / 64, cap = net.n_tensors + nv + 1, cnt = net.n_tensors;
    uint64_t *sets = calloc((size_t)cap * (size_t)words, sizeof(uint64_t));
    int *bucket_of = malloc(sizeof(int) * (size_t)cap);
    for (int t = 0; t < net.n_tensors; t++) {
        int b = nv;
        for (int q = 0; q < net.t[t].rank; q++) {
            int v = net.t[t].idx[q];
            sets[(size_t)t * words + v / 64] |= (uint64_t)1 << (v % 64);
            if (pos[v] < b)
                b = pos[v];
        }
        bucket_of[t] = b;
    }
    uint64_t *u = malloc(sizeof(uint64_t) * (size_t)words);
    for (int i = 0; i < nv; i++) {
        memset(u, 0, sizeof(uint64_t) * (size_t)words);
        int any = 0;
        for (int t = 0; t < cnt; t++)
            if (bucket_of[t] == i) {
                any = 1;
                bucket_of[t] = -1;
                for (int k = 0; k < words; k++)
                    u[k] |= sets[(size_t)t * words + k];
            }
        widths_out[i] = 0;
        if (!any)
            continue;
        int w = 0, b = nv;
        for (int k = 0; k < words; k++)
            w += __builtin_popcountll(u[k]);
        widths_out[i] = w;
        int v = ord[i];
        u[v / 64] &= ~((uint64_t)1 << (v % 64));
        for (int x = 0; x < nv; x++)
            if ((u[x / 64] >> (x % 64)) & 1u)
                if (pos[x] < b)
                    b = pos[x];
        if (b < nv) {
            memcpy(&sets[(size_t)cnt * words], u, sizeof(uint64_t) * (size_t)words);
            bucket_of[cnt++] = b;
        }
    }
    free(u);
    free(bucket_of);
    free(sets);
    free(pos);
    free(ord);
    net_free(&net);
    return QTNO_OK;
}

/* The same network summed over every assignment of its variables. */
int qtno_edge_zz_bruteforce(int n, int m, const int *edges, int edge_id, int p,
                            const double *gamma, const double *beta, int mode,
                            double *re, double *im)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    onet net;
    rc = build_network(n, m, edges, edge_id, p, gamma, beta, mode, &net);
    if (rc)
        return rc;
    if (net.n_vars > 28) {
        net_free(&net);
        return fail(QTNO_ERANGE, "too many variables for the brute-force sum");
    }
    cplx total = 0.0;
    uint64_t count = (uint64_t)1 << net.n_vars;
    for (uint64_t x = 0; x < count; x++) {
        cplx prod = 1.0;
        for (int t = 0; t < net.n_tensors; t++) {
            const otensor *tt = &net.t[t];
            uint64_t off = 0;
            for (int q = 0; q < tt->rank; q++)
                off = (off << 1) | ((x >> tt->idx[q]) & 1u);
            prod *= tt->data[off];
        }
        total += prod;
    }
    net_free(&net);
    *re = creal(total);
    *im = cimag(total);
    return QTNO_OK;
}

/* -------------------------------------------------------------- statevector */

/* Amplitudes of |gamma, beta>_p (Eq. 2) on n <= 26 qubits, z bit q = qubit q,
 * then e_jk = sum_z |psi(z)|^2 (-1)^(z_j xor z_k) for every edge. */
int qtno_statevector_zz(int n, int m, const int *edges, int p,
                        const double *gamma, const double *beta, double *zz)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    if (n > 26)
        return fail(QTNO_ERANGE, "statevector limited to 26 qubits");
    uint64_t dim = (uint64_t)1 << n;
    cplx *psi = malloc(sizeof(cplx) * dim);
    if (!psi)
        return fail(QTNO_ENOMEM, "host allocation failed");
    double amp = 1.0 / sqrt((double)dim);
    for (uint64_t z = 0; z < dim; z++)
        psi[z] = amp;
    for (int l = 0; l < p; l++) {
        for (uint64_t z = 0; z < dim; z++) {
            int cut = 0;
            for (int e = 0; e < m; e++)
                cut += (int)(((z >> edges[2 * e]) ^ (z >> edges[2 * e + 1])) & 1u);
            psi[z] *= cexp(-I * gamma[l] * cut);
        }
        double c = cos(beta[l]), s = sin(beta[l]);
        for (int q = 0; q < n; q++) {
            uint64_t bit = (uint64_t)1 << q;
            for (uint64_t z = 0; z < dim; z++) {
                if (z & bit)
                    continue;
                cplx a0 = psi[z], a1 = psi[z | bit];
                psi[z] = c * a0 - I * s * a1;
                psi[z | bit] = -I * s * a0 + c * a1;
            }
        }
    }
    for (int e = 0; e < m; e++) {
        double acc = 0.0;
        int a = edges[2 * e], b = edges[2 * e + 1];
        for (uint64_t z = 0; z < dim; z++) {
            double pr = creal(psi[z]) * creal(psi[z]) + cimag(psi[z]) * cimag(psi[z]);
            acc += (((z >> a) ^ (z >> b)) & 1u) ? -pr : pr;
        }
        zz[e] = acc;
    }
    free(psi);
    return QTNO_OK;
}

/* ------------------------------------------------------------ closed form */

/* Depth-1 closed form (Wang, Hadfield, Jiang, Rieffel 2018, Theorem 1):
 *   <C_uv> = 1/2 + 1/4 sin(4b) sin(g) (cos^du g + cos^dv g)
 *          - 1/4 sin^2(2b) cos^(du+dv-2f) g (1 - cos^f (2g)),
 * du = deg(u)-1, dv = deg(v)-1, f = triangles through (u,v);
 * returned as e_uv = 1 - 2 <C_uv>. */
int qtno_p1_closed_form(int n, int m, const int *edges, double g, double b,
                        double *zz)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    int *deg = calloc((size_t)n, sizeof(int));
    unsigned char *adj = calloc((size_t)n * (size_t)n, 1);
    for (int e = 0; e < m; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        deg[u]++;
        deg[v]++;
        adj[(size_t)u * n + v] = adj[(size_t)v * n + u] = 1;
    }
    for (int e = 0; e < m; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        int f = 0;
        for (int w = 0; w < n; w++)
            if (adj[(size_t)u * n + w] && adj[(size_t)v * n + w])
                f++;
        int du = deg[u] - 1, dv = deg[v] - 1;
        double c = cos(g);
        double cuv = 0.5 + 0.25 * sin(4 * b) * sin(g) * (pow(c, du) + pow(c, dv)) -
                     0.25 * sin(2 * b) * sin(2 * b) * pow(c, du + dv - 2 * f) *
                         (1.0 - pow(cos(2 * g), f));
        zz[e] = 1.0 - 2.0 * cuv;
    }
    free(adj);
    free(deg);
    return QTNO_OK;
}

/* ----------------------------------------------------------------- energy */

typedef struct {
    int n, m, p, mode;
    const int *edges;
    const double *gamma, *beta;
    const int *edge_list;
    int n_list;
    double *re, *im;
    int next;
    int rc;
    pthread_mutex_t lock;
} energy_job;

static void *energy_worker(void *arg)
{
    energy_job *job = arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int i = job->next++;
        int stop = job->rc != QTNO_OK;
        pthread_mutex_unlock(&job->lock);
        if (i >= job->n_list || stop)
            break;
        int e = job->edge_list ? job->edge_list[i] : i;
        double re = 0, im = 0;
        int rc = qtno_edge_zz(job->n, job->m, job->edges, e, job->p, job->gamma,
                              job->beta, job->mode, 0, NULL, 0, &re, &im, NULL);
        pthread_mutex_lock(&job->lock);
        if (rc)
            job->rc = rc;
        job->re[i] = re;
        job->im[i] = im;
        pthread_mutex_unlock(&job->lock);
    }
    return NULL;
}

/*
 * e_jk for the edges in edge_list (NULL = all m edges, in edge order), by
 * bucket elimination with min-fill orders, n_threads host threads over light
 * cones.  When every edge is evaluated, *energy = |E|/2 - 1/2 sum Re e_jk
 * (Sec. II-B), summed in edge order with Neumaier compensation.
 */
int qtno_energy(int n, int m, const int *edges, int p, const double *gamma,
                const double *beta, int mode, int n_threads,
                const int *edge_list, int n_list, double *zz_re, double *zz_im,
                double *energy)
{
    int rc = check_graph(n, m, edges);
    if (rc)
        return rc;
    if (!edge_list)
        n_list = m;
    energy_job job = {n, m, p, mode, edges, gamma, beta, edge_list, n_list,
                      zz_re, zz_im, 0, QTNO_OK, PTHREAD_MUTEX_INITIALIZER};
    if (n_threads < 1)
        n_threads = 1;
    pthread_t *th = malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int t = 0; t < n_threads; t++)
        pthread_create(&th[t], NULL, energy_worker, &job);
    for (int t = 0; t < n_threads; t++)
        pthread_join(th[t], NULL);
    free(th);
    if (job.rc)
        return job.rc;
    if (energy && !edge_list) {
        double sum = 0.0, comp = 0.0;
        for (int e = 0; e < m; e++) {
            double x = zz_re[e], t = sum + x;
            if (fabs(sum) >= fabs(x))
                comp += (sum - t) + x;
            else
                comp += (x - t) + sum;
            sum = t;
        }
        *energy = 0.5 * m - 0.5 * (sum + comp);
    }
    return QTNO_OK;
}

/* ---------------------------------------------------------- single bucket */

/*
 * out[out_idx] = sum over the n_sum variables in sum_vars of
 *                prod_t tensor_t[idx_t]
 * for caller-given tensors (ranks[t], their variable ids in idx_flat,
 * row-major data as interleaved (re, im) doubles in data_flat with idx[0] the
 * most significant axis).  out_idx lists the kept variables in the layout
 * wanted for out_data (row-major, interleaved).  Every tensor index must be in
 * out_idx or sum_vars.  The summed assignments are visited in increasing
 * binary order, tensors in the order given.
 */
int qtno_contract_bucket(int n_tensors, const int *ranks, const int *idx_flat,
                         const double *data_flat, int n_sum,
                         const int *sum_vars, int out_rank, const int *out_idx,
                         double *out_data)
{
    int w = n_sum + out_rank;
    if (n_tensors < 1 || w > 30 || n_sum < 0 || out_rank < 0)
        return fail(QTNO_EINVAL, "bad bucket shape");
    int *uni = malloc(sizeof(int) * (size_t)(w > 0 ? w : 1));
    for (int q = 0; q < out_rank; q++)
        uni[q] = out_idx[q];
    for (int q = 0; q < n_sum; q++)
        uni[out_rank + q] = sum_vars[q];
    int total_rank = 0;
    for (int t = 0; t < n_tensors; t++)
        total_rank += ranks[t];
    int *upos = malloc(sizeof(int) * (size_t)(total_rank > 0 ? total_rank : 1));
    size_t *doff = malloc(sizeof(size_t) * (size_t)n_tensors);
    size_t off = 0;
    for (int t = 0, r0 = 0; t < n_tensors; t++) {
        doff[t] = off;
        off += (size_t)1 << ranks[t];
        for (int q = 0; q < ranks[t]; q++) {
            int found = -1;
            for (int u = 0; u < w; u++)
                if (uni[u] == idx_flat[r0 + q])
                    found = u;
            if (found < 0) {
                free(uni);
                free(upos);
                free(doff);
                return fail(QTNO_EINVAL, "tensor index not in the union");
            }
            upos[r0 + q] = found;
        }
        r0 += ranks[t];
    }
    uint64_t nout = (uint64_t)1 << out_rank, nsum = (uint64_t)1 << n_sum;
    for (uint64_t o = 0; o < nout; o++) {
        cplx acc = 0.0;
        for (uint64_t s = 0; s < nsum; s++) {
            uint64_t ux = (o << n_sum) | s; /* union = out_idx then sum_vars */
            cplx prod = 1.0;
            for (int t = 0, r0 = 0; t < n_tensors; t++) {
                uint64_t e = 0;
                for (int q = 0; q < ranks[t]; q++)
                    e |= ((ux >> (w - 1 - upos[r0 + q])) & 1u) << (ranks[t] - 1 - q);
                const double *d = &data_flat[2 * (doff[t] + e)];
                prod *= d[0] + I * d[1];
                r0 += ranks[t];
            }
            acc += prod;
        }
        out_data[2 * o] = creal(acc);
        out_data[2 * o + 1] = cimag(acc);
    }
    free(uni);
    free(upos);
    free(doff);
    return QTNO_OK;
}

/* ------------------------------------------------------------- cost model */

/*
 * FP64 reference of the cost-model network: 16 inputs, two hidden layers of
 * 64 rectified-linear units, 4 linear outputs (predicted log launch time of
 * each kernel variant).  Parameters are packed as
 *   W1[16][64], b1[64], W2[64][64], b2[64], W3[64][4], b3[4]
 * (row-major, input index first).  The loss is the mean of the squared
 * errors over the measured entries:
 *   loss = sum_{i,k} m_ik (y_ik - t_ik)^2 / sum_{i,k} m_ik.
 * qtno_mlp_loss_grad returns the loss and d loss / d params; qtno_mlp_adam
 * takes one Adam step (Kingma & Ba 2015) with bias correction at step t.
 */
#define MLP_IN 16
#define MLP_H 64
#define MLP_OUT 4
#define MLP_NPARAM (MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H * MLP_OUT + MLP_OUT)

int qtno_mlp_nparams(void) { return MLP_NPARAM; }

static void mlp_views(const double *p, const double **w1, const double **b1,
                      const double **w2, const double **b2, const double **w3,
                      const double **b3)
{
    *w1 = p;
    *b1 = *w1 + MLP_IN * MLP_H;
    *w2 = *b1 + MLP_H;
    *b2 = *w2 + MLP_H * MLP_H;
    *w3 = *b2 + MLP_H;
    *b3 = *w3 + MLP_H * MLP_OUT;
}

int qtno_mlp_forward(const double *params, const double *x, int n, double *y)
{
    const double *w1, *b1, *w2, *b2, *w3, *b3;
    mlp_views(params, &w1, &b1, &w2, &b2, &w3, &b3);
    double h1[MLP_H], h2[MLP_H];
    for (int i = 0; i < n; i++) {
        const double *xi = &x[i * MLP_IN];
        for (int j = 0; j < MLP_H; j++) {
            double a = b1[j];
            for (int k = 0; k < MLP_IN; k++)
                a += xi[k] * w1[k * MLP_H + j];
            h1[j] = a > 0 ? a : 0;
        }
        for (int j = 0; j < MLP_H; j++) {
            double a = b2[j];
            for (int k = 0; k < MLP_H; k++)
                a += h1[k] * w2[k * MLP_H + j];
            h2[j] = a > 0 ? a : 0;
        }
        for (int j = 0; j < MLP_OUT; j++) {
            double a = b3[j];
            for (int k = 0; k < MLP_H; k++)
                a += h2[k] * w3[k * MLP_OUT + j];
            y[i * MLP_OUT + j] = a;
        }
    }
    return QTNO_OK;
}

int qtno_mlp_loss_grad(const double *params, const double *x, const double *t,
                       const double *m, int n, double *loss, double *grad)
{
    const double *w1, *b1, *w2, *b2, *w3, *b3;
    mlp_views(params, &w1, &b1, &w2, &b2, &w3, &b3);
    double *gw1 = grad, *gb1 = gw1 + MLP_IN * MLP_H, *gw2 = gb1 + MLP_H;
    double *gb2 = gw2 + MLP_H * MLP_H, *gw3 = gb2 + MLP_H, *gb3 = gw3 + MLP_H * MLP_OUT;
    for (int q = 0; q < MLP_NPARAM; q++)
        grad[q] = 0;
    double msum = 0;
    for (int q = 0; q < n * MLP_OUT; q++)
        msum += m[q];
    if (msum <= 0)
        return fail(QTNO_EINVAL, "no measured entries");
    double l = 0;
    double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H], y[MLP_OUT];
    double dy[MLP_OUT], dh2[MLP_H], dh1[MLP_H];
    for (int i = 0; i < n; i++) {
        const double *xi = &x[i * MLP_IN];
        for (int j = 0; j < MLP_H; j++) {
            double a = b1[j];
            for (int k = 0; k < MLP_IN; k++)
                a += xi[k] * w1[k * MLP_H + j];
            z1[j] = a;
            h1[j] = a > 0 ? a : 0;
        }
        for (int j = 0; j < MLP_H; j++) {
            double a = b2[j];
            for (int k = 0; k < MLP_H; k++)
                a += h1[k] * w2[k * MLP_H + j];
            z2[j] = a;
            h2[j] = a > 0 ? a : 0;
        }
        for (int j = 0; j < MLP_OUT; j++) {
            double a = b3[j];
            for (int k = 0; k < MLP_H; k++)
                a += h2[k] * w3[k * MLP_OUT + j];
            y[j] = a;
            const double e = y[j] - t[i * MLP_OUT + j], mm = m[i * MLP_OUT + j];
            l += mm * e * e;
            dy[j] = 2.0 * mm * e / msum;
        }
        for (int j = 0; j < MLP_OUT; j++) {
            gb3[j] += dy[j];
            for (int k = 0; k < MLP_H; k++)
                gw3[k * MLP_OUT + j] += h2[k] * dy[j];
        }
        for (int k = 0; k < MLP_H; k++) {
            double a = 0;
            for (int j = 0; j < MLP_OUT; j++)
                a += w3[k * MLP_OUT + j] * dy[j];
            dh2[k] = z2[k] > 0 ? a : 0;
        }
        for (int j = 0; j < MLP_H; j++) {
            gb2[j] += dh2[j];
            for (int k = 0; k < MLP_H; k++)
                gw2[k * MLP_H + j] += h1[k] * dh2[j];
        }
        for (int k = 0; k < MLP_H; k++) {
            double a = 0;
            for (int j = 0; j < MLP_H; j++)
                a += w2[k * MLP_H + j] * dh2[j];
            dh1[k] = z1[k] > 0 ? a : 0;
        }
        for (int j = 0; j < MLP_H; j++) {
            gb1[j] += dh1[j];
            for (int k = 0; k < MLP_IN; k++)
                gw1[k * MLP_H + j] += xi[k] * dh1[j];
        }
    }
    *loss = l / msum;
    return QTNO_OK;
}

/* One Adam step on params (moments mom1, mom2 updated in place), step t >= 1. */
int qtno_mlp_adam(double *params, double *mom1, double *mom2, const double *grad,
                  int t, double lr, double beta1, double beta2, double eps)
{
    const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int q = 0; q < MLP_NPARAM; q++) {
        mom1[q] = beta1 * mom1[q] + (1 - beta1) * grad[q];
        mom2[q] = beta2 * mom2[q] + (1 - beta2) * grad[q] * grad[q];
        params[q] -= lr * (mom1[q] / c1) / (sqrt(mom2[q] / c2) + eps);
    }
    return QTNO_OK;
}
