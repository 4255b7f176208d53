/*
 * CPU oracle for exact s-t max-flow / min-cut in the excess form of the paper
 * (Sec. 2: network G=(V,E,s,t,c,e), preflow constraints eq. (2), residual
 * network, flow value |f| = sum_u f(u,t), optimality test "no excess vertex
 * reaches t in G_f", cut (T-bar, T)).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the tests, the smoke check and the bench's CPU-baseline leg load.  It
 * shares no code, header, table or helper with the GPU solver.
 *
 * Contents
 *   orc_pushrelabel  textbook highest-label push-relabel (Sec. 2, generic
 *                    Push / Relabel of Goldberg-Tarjan) with gap and global
 *                    relabel; int64 arithmetic; phase 1 (maximum preflow).
 *   orc_dinic        Dinic blocking flows on the explicit s-t network (a second,
 *                    independent solver that produces a true flow).
 *   orc_cuts         residual reachability: S_max = V \ {v : v -> t} (Sec. 2,
 *                    max-preflow test) and S_min = {v : some excess vertex
 *                    reaches v}.
 *   orc_boundary_relabel  the heuristic of Sec. 6.1 alone on a residual state.
 *   orc_ard          reference region discharge: Init, Alg. 1 (S-ARD) or Alg. 2
 *                    (P-ARD, label and flow fusion), Proc. ARD with Augment
 *                    (Sec. 4.2), region relabel (Alg. 3, ARD variant) and the
 *                    global gap heuristic (Sec. 5.1) over boundary labels, with
 *                    optional per-sweep checks of the statements of Sec. 4;
 *                    optionally with partial discharges (Sec. 6.2) and the
 *                    boundary relabel heuristic (Sec. 6.1) after every sweep.
 *
 * Input network format (all entry points): n non-terminal vertices 0..n-1 and
 * np vertex pairs {pu[i], pv[i]} with capacities c(pu,pv)=cuv[i] and
 * c(pv,pu)=cvu[i] (the symmetric arc set of Sec. 2: a missing direction is a
 * zero).  cs[v] = c(s,v) is folded into the excess by Init; ct[v] = c(v,t).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ENOMEM 1
#define ORC_EINVAL 2
#define ORC_ECHECK 3   /* an invariant check of orc_ard failed */
#define ORC_ESWEEPS 4  /* orc_ard exceeded max_sweeps */

/* ------------------------------------------------------------------------ */
/* Residual network in CSR form.                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    int64_t m;        /* directed arcs = 2 * np */
    int64_t *first;   /* [n+1] */
    int32_t *head;    /* [m] */
    int32_t *tail;    /* [m] */
    int64_t *rev;     /* [m] index of the reverse arc */
    int64_t *res;     /* [m] residual capacity c_f */
    int64_t *pair_fw; /* [np] arc index of pu->pv */
    int64_t *pair_bw; /* [np] arc index of pv->pu */
} net_t;

static void net_free(net_t *g) {
    free(g->first); free(g->head); free(g->tail); free(g->rev); free(g->res);
    free(g->pair_fw); free(g->pair_bw);
    memset(g, 0, sizeof(*g));
}

static int net_build(net_t *g, int32_t n, int64_t np, const int32_t *pu, const int32_t *pv,
                     const int32_t *cuv, const int32_t *cvu) {
    memset(g, 0, sizeof(*g));
    g->n = n;
    g->m = 2 * np;
    g->first = calloc((size_t)n + 1, sizeof(int64_t));
    g->head = malloc(sizeof(int32_t) * (size_t)(g->m ? g->m : 1));
    g->tail = malloc(sizeof(int32_t) * (size_t)(g->m ? g->m : 1));
    g->rev = malloc(sizeof(int64_t) * (size_t)(g->m ? g->m : 1));
    g->res = malloc(sizeof(int64_t) * (size_t)(g->m ? g->m : 1));
    g->pair_fw = malloc(sizeof(int64_t) * (size_t)(np ? np : 1));
    g->pair_bw = malloc(sizeof(int64_t) * (size_t)(np ? np : 1));
    if (!g->first || !g->head || !g->tail || !g->rev || !g->res || !g->pair_fw || !g->pair_bw) {
        net_free(g);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < np; i++) {
        if (pu[i] < 0 || pu[i] >= n || pv[i] < 0 || pv[i] >= n || cuv[i] < 0 || cvu[i] < 0) {
            net_free(g);
            return ORC_EINVAL;
        }
        g->first[pu[i] + 1]++;
        g->first[pv[i] + 1]++;
    }
    for (int32_t v = 0; v < n; v++) g->first[v + 1] += g->first[v];
    int64_t *fill = malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!fill) { net_free(g); return ORC_ENOMEM; }
    memcpy(fill, g->first, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < np; i++) {
        int64_t a = fill[pu[i]]++;
        int64_t b = fill[pv[i]]++;
        g->head[a] = pv[i]; g->tail[a] = pu[i]; g->res[a] = cuv[i]; g->rev[a] = b;
        g->head[b] = pu[i]; g->tail[b] = pv[i]; g->res[b] = cvu[i]; g->rev[b] = a;
        g->pair_fw[i] = a;
        g->pair_bw[i] = b;
    }
    free(fill);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Residual reachability (the cuts).                                        */
/* ------------------------------------------------------------------------ */
/* smax[v] = 1 iff v does NOT reach t in G_f (source side of the paper's cut
 * (T-bar, T)); smin[v] = 1 iff some vertex with positive excess reaches v.
 * Both are the extremal minimum cuts once the preflow is maximum. */
static int cuts_from_residual(const net_t *g, const int64_t *rt, const int64_t *ex,
                              uint8_t *smin, uint8_t *smax) {
    int32_t n = g->n;
    int32_t *queue = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    uint8_t *mark = calloc((size_t)(n ? n : 1), 1);
    if (!queue || !mark) { free(queue); free(mark); return ORC_ENOMEM; }
    /* backward search from t: v reaches t if c_f(v,t) > 0 or c_f(v,w) > 0 for a w reaching t */
    int64_t qh = 0, qt = 0;
    for (int32_t v = 0; v < n; v++)
        if (rt[v] > 0) { mark[v] = 1; queue[qt++] = v; }
    while (qh < qt) {
        int32_t w = queue[qh++];
        for (int64_t a = g->first[w]; a < g->first[w + 1]; a++) {
            int32_t u = g->head[a];
            if (!mark[u] && g->res[g->rev[a]] > 0) { mark[u] = 1; queue[qt++] = u; }
        }
    }
    if (smax) for (int32_t v = 0; v < n; v++) smax[v] = mark[v] ? 0 : 1;
    /* forward search from the excess vertices */
    memset(mark, 0, (size_t)(n ? n : 1));
    qh = qt = 0;
    for (int32_t v = 0; v < n; v++)
        if (ex[v] > 0) { mark[v] = 1; queue[qt++] = v; }
    while (qh < qt) {
        int32_t u = queue[qh++];
        for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
            int32_t w = g->head[a];
            if (!mark[w] && g->res[a] > 0) { mark[w] = 1; queue[qt++] = w; }
        }
    }
    if (smin) for (int32_t v = 0; v < n; v++) smin[v] = mark[v];
    free(queue); free(mark);
    return ORC_OK;
}

static void write_outputs(const net_t *g, int64_t np, const int64_t *rt, const int64_t *ex,
                          const int32_t *ct, int64_t *r_uv, int64_t *r_vu, int64_t *rt_out,
                          int64_t *ex_out, int64_t *flow_out) {
    int64_t flow = 0;
    for (int32_t v = 0; v < g->n; v++) flow += (int64_t)ct[v] - rt[v];
    if (flow_out) *flow_out = flow;
    for (int64_t i = 0; i < np; i++) {
        if (r_uv) r_uv[i] = g->res[g->pair_fw[i]];
        if (r_vu) r_vu[i] = g->res[g->pair_bw[i]];
    }
    if (rt_out) memcpy(rt_out, rt, sizeof(int64_t) * (size_t)g->n);
    if (ex_out) memcpy(ex_out, ex, sizeof(int64_t) * (size_t)g->n);
}

/* ------------------------------------------------------------------------ */
/* Highest-label push-relabel (Sec. 2, generic Push/Relabel).               */
/* ------------------------------------------------------------------------ */
typedef struct {
    net_t *g;
    int64_t *ex, *rt;
    int32_t *d;        /* labels: d(t)=0, DINF = n + 1 means "cannot reach t" */
    int32_t dinf;
    int64_t *cur;      /* current arc */
    /* active vertices: one stack per label */
    int32_t *act_next, *act_top;
    /* all vertices with finite label: doubly linked list per label (gap detection) */
    int32_t *all_next, *all_prev, *all_head;
    int32_t amax;      /* upper bound on the highest active label */
    int32_t dmax;      /* upper bound on the highest finite label in use */
    int64_t relabels_since_global;
    int32_t *queue;
} pr_t;

static void pr_all_insert(pr_t *P, int32_t v) {
    int32_t l = P->d[v];
    P->all_prev[v] = -1;
    P->all_next[v] = P->all_head[l];
    if (P->all_head[l] >= 0) P->all_prev[P->all_head[l]] = v;
    P->all_head[l] = v;
    if (l > P->dmax) P->dmax = l;
}

static void pr_all_remove(pr_t *P, int32_t v) {
    int32_t l = P->d[v];
    if (P->all_prev[v] >= 0) P->all_next[P->all_prev[v]] = P->all_next[v];
    else P->all_head[l] = P->all_next[v];
    if (P->all_next[v] >= 0) P->all_prev[P->all_next[v]] = P->all_prev[v];
}

static void pr_act_push(pr_t *P, int32_t v) {
    int32_t l = P->d[v];
    P->act_next[v] = P->act_top[l];
    P->act_top[l] = v;
    if (l > P->amax) P->amax = l;
}

/* Exact labels by breadth-first search from t over residual arcs (the
 * "global relabel" of push-relabel codes); rebuilds both bucket structures. */
static void pr_global_relabel(pr_t *P) {
    net_t *g = P->g;
    int32_t n = g->n;
    for (int32_t l = 0; l <= P->dinf; l++) { P->act_top[l] = -1; P->all_head[l] = -1; }
    for (int32_t v = 0; v < n; v++) P->d[v] = P->dinf;
    int64_t qh = 0, qt = 0;
    for (int32_t v = 0; v < n; v++)
        if (P->rt[v] > 0) { P->d[v] = 1; P->queue[qt++] = v; }
    while (qh < qt) {
        int32_t w = P->queue[qh++];
        for (int64_t a = g->first[w]; a < g->first[w + 1]; a++) {
            int32_t u = g->head[a];
            if (P->d[u] == P->dinf && g->res[g->rev[a]] > 0) {
                P->d[u] = P->d[w] + 1;
                P->queue[qt++] = u;
            }
        }
    }
    P->amax = 0;
    P->dmax = 0;
    for (int32_t v = 0; v < n; v++) {
        P->cur[v] = g->first[v];
        if (P->d[v] < P->dinf) {
            pr_all_insert(P, v);
            if (P->ex[v] > 0) pr_act_push(P, v);
        }
    }
    P->relabels_since_global = 0;
}

/* Gap: no vertex has label g, so every vertex above g cannot reach t. */
static void pr_gap(pr_t *P, int32_t gap) {
    for (int32_t l = gap + 1; l <= P->dmax; l++) {
        int32_t v = P->all_head[l];
        while (v >= 0) {
            int32_t nx = P->all_next[v];
            P->d[v] = P->dinf;
            v = nx;
        }
        P->all_head[l] = -1;
        P->act_top[l] = -1;
    }
    if (gap < P->dmax) P->dmax = gap;
    if (P->amax > gap) P->amax = gap;
}

static void pr_discharge(pr_t *P, int32_t v) {
    net_t *g = P->g;
    while (P->ex[v] > 0 && P->d[v] < P->dinf) {
        /* Push to t: admissible when d(v) = d(t) + 1 = 1. */
        if (P->d[v] == 1 && P->rt[v] > 0) {
            int64_t delta = P->ex[v] < P->rt[v] ? P->ex[v] : P->rt[v];
            P->rt[v] -= delta;
            P->ex[v] -= delta;
            continue;
        }
        int64_t end = g->first[v + 1];
        int64_t a = P->cur[v];
        for (; a < end && P->ex[v] > 0; a++) {
            int32_t w = g->head[a];
            if (g->res[a] > 0 && P->d[v] == P->d[w] + 1) {
                int64_t delta = P->ex[v] < g->res[a] ? P->ex[v] : g->res[a];
                g->res[a] -= delta;
                g->res[g->rev[a]] += delta;
                P->ex[v] -= delta;
                if (P->ex[w] == 0 && P->d[w] < P->dinf) { P->ex[w] += delta; pr_act_push(P, w); }
                else P->ex[w] += delta;
                if (P->ex[v] == 0) break;
            }
        }
        if (P->ex[v] == 0) { P->cur[v] = a; break; }
        /* Relabel: d(v) := min(DINF, min{d(w)+1 : c_f(v,w) > 0}), with t at label 0. */
        int32_t nd = P->dinf;
        if (P->rt[v] > 0) nd = 1;
        for (int64_t b = g->first[v]; b < end; b++)
            if (g->res[b] > 0 && P->d[g->head[b]] + 1 < nd) nd = P->d[g->head[b]] + 1;
        int32_t old = P->d[v];
        pr_all_remove(P, v);
        P->cur[v] = g->first[v];
        P->relabels_since_global++;
        if (P->all_head[old] < 0) {
            /* v was the last vertex with label old: gap at old */
            P->d[v] = P->dinf;
            pr_gap(P, old);
            break;
        }
        P->d[v] = nd;
        if (nd >= P->dinf) break;
        pr_all_insert(P, v);
    }
}

int orc_pushrelabel(int32_t n, int64_t np, const int32_t *pu, const int32_t *pv,
                    const int32_t *cuv, const int32_t *cvu, const int32_t *cs, const int32_t *ct,
                    int64_t *r_uv, int64_t *r_vu, int64_t *rt_out, int64_t *ex_out,
                    int64_t *flow_out, uint8_t *smin, uint8_t *smax) {
    net_t g;
    int rc = net_build(&g, n, np, pu, pv, cuv, cvu);
    if (rc) return rc;
    pr_t P;
    memset(&P, 0, sizeof(P));
    P.g = &g;
    P.dinf = n + 1;
    size_t nn = (size_t)(n ? n : 1), nl = (size_t)n + 2;
    P.ex = malloc(sizeof(int64_t) * nn);
    P.rt = malloc(sizeof(int64_t) * nn);
    P.d = malloc(sizeof(int32_t) * nn);
    P.cur = malloc(sizeof(int64_t) * nn);
    P.act_next = malloc(sizeof(int32_t) * nn);
    P.all_next = malloc(sizeof(int32_t) * nn);
    P.all_prev = malloc(sizeof(int32_t) * nn);
    P.queue = malloc(sizeof(int32_t) * nn);
    P.act_top = malloc(sizeof(int32_t) * nl);
    P.all_head = malloc(sizeof(int32_t) * nl);
    if (!P.ex || !P.rt || !P.d || !P.cur || !P.act_next || !P.all_next || !P.all_prev ||
        !P.queue || !P.act_top || !P.all_head) {
        rc = ORC_ENOMEM;
        goto done;
    }
    /* Init (Sec. 2): saturate the s-links into the excess, f := 0, d := 0. */
    for (int32_t v = 0; v < n; v++) {
        if (cs[v] < 0 || ct[v] < 0) { rc = ORC_EINVAL; goto done; }
        P.ex[v] = cs[v];
        P.rt[v] = ct[v];
    }
    pr_global_relabel(&P);
    const int64_t global_every = (int64_t)n + 16;
    for (;;) {
        while (P.amax >= 0 && P.act_top[P.amax] < 0) P.amax--;
        if (P.amax < 0) break;
        int32_t v = P.act_top[P.amax];
        P.act_top[P.amax] = P.act_next[v];
        if (P.ex[v] == 0 || P.d[v] != P.amax) continue; /* stale entry */
        pr_discharge(&P, v);
        if (P.relabels_since_global > global_every) pr_global_relabel(&P);
    }
    write_outputs(&g, np, P.rt, P.ex, ct, r_uv, r_vu, rt_out, ex_out, flow_out);
    rc = cuts_from_residual(&g, P.rt, P.ex, smin, smax);
done:
    free(P.ex); free(P.rt); free(P.d); free(P.cur); free(P.act_next); free(P.all_next);
    free(P.all_prev); free(P.queue); free(P.act_top); free(P.all_head);
    net_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Dinic on the explicit s-t network.                                       */
/* ------------------------------------------------------------------------ */
/* The s-links and t-links become ordinary arcs of vertices S=n and T=n+1.
 * The result is a true flow; its residual s-arc capacities equal the excess
 * that the excess form of Sec. 2 would leave at each vertex. */
int orc_dinic(int32_t n, int64_t np, const int32_t *pu, const int32_t *pv, const int32_t *cuv,
              const int32_t *cvu, const int32_t *cs, const int32_t *ct, int64_t *r_uv,
              int64_t *r_vu, int64_t *rt_out, int64_t *ex_out, int64_t *flow_out,
              uint8_t *smin, uint8_t *smax) {
    int32_t N = n + 2, S = n, T = n + 1;
    int64_t NP = np + 2 * (int64_t)n;
    int32_t *PU = malloc(sizeof(int32_t) * (size_t)(NP ? NP : 1));
    int32_t *PV = malloc(sizeof(int32_t) * (size_t)(NP ? NP : 1));
    int32_t *CU = malloc(sizeof(int32_t) * (size_t)(NP ? NP : 1));
    int32_t *CV = malloc(sizeof(int32_t) * (size_t)(NP ? NP : 1));
    int rc = ORC_OK;
    net_t g;
    memset(&g, 0, sizeof(g));
    int32_t *level = NULL, *queue = NULL;
    int64_t *it = NULL, *stack_arc = NULL;
    if (!PU || !PV || !CU || !CV) { rc = ORC_ENOMEM; goto out; }
    for (int64_t i = 0; i < np; i++) { PU[i] = pu[i]; PV[i] = pv[i]; CU[i] = cuv[i]; CV[i] = cvu[i]; }
    for (int32_t v = 0; v < n; v++) {
        if (cs[v] < 0 || ct[v] < 0) { rc = ORC_EINVAL; goto out; }
        PU[np + v] = S; PV[np + v] = v; CU[np + v] = cs[v]; CV[np + v] = 0;
        PU[np + n + v] = v; PV[np + n + v] = T; CU[np + n + v] = ct[v]; CV[np + n + v] = 0;
    }
    rc = net_build(&g, N, NP, PU, PV, CU, CV);
    if (rc) goto out;
    level = malloc(sizeof(int32_t) * (size_t)N);
    queue = malloc(sizeof(int32_t) * (size_t)N);
    it = malloc(sizeof(int64_t) * (size_t)N);
    stack_arc = malloc(sizeof(int64_t) * (size_t)N);
    if (!level || !queue || !it || !stack_arc) { rc = ORC_ENOMEM; goto out; }
    for (;;) {
        for (int32_t v = 0; v < N; v++) level[v] = -1;
        int64_t qh = 0, qt = 0;
        level[S] = 0;
        queue[qt++] = S;
        while (qh < qt) {
            int32_t u = queue[qh++];
            for (int64_t a = g.first[u]; a < g.first[u + 1]; a++)
                if (g.res[a] > 0 && level[g.head[a]] < 0) {
                    level[g.head[a]] = level[u] + 1;
                    queue[qt++] = g.head[a];
                }
        }
        if (level[T] < 0) break;
        for (int32_t v = 0; v < N; v++) it[v] = g.first[v];
        /* blocking flow by repeated depth-first search with current arcs */
        for (;;) {
            int32_t depth = 0, u = S;
            int found = 0;
            while (1) {
                if (u == T) { found = 1; break; }
                int64_t a = it[u];
                for (; a < g.first[u + 1]; a++)
                    if (g.res[a] > 0 && level[g.head[a]] == level[u] + 1) break;
                it[u] = a;
                if (a == g.first[u + 1]) {
                    /* dead end: retreat */
                    level[u] = -1;
                    if (depth == 0) break;
                    depth--;
                    u = g.tail[stack_arc[depth]];
                    it[u]++;
                    continue;
                }
                stack_arc[depth++] = a;
                u = g.head[a];
            }
            if (!found) break;
            int64_t delta = INT64_MAX;
            for (int32_t i = 0; i < depth; i++)
                if (g.res[stack_arc[i]] < delta) delta = g.res[stack_arc[i]];
            for (int32_t i = 0; i < depth; i++) {
                g.res[stack_arc[i]] -= delta;
                g.res[g.rev[stack_arc[i]]] += delta;
            }
        }
    }
    {
        /* Translate back to the excess form over the n non-terminal vertices. */
        int64_t *rt = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
        int64_t *ex = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
        if (!rt || !ex) { free(rt); free(ex); rc = ORC_ENOMEM; goto out; }
        for (int32_t v = 0; v < n; v++) {
            ex[v] = g.res[g.pair_fw[np + v]];     /* residual of s -> v */
            rt[v] = g.res[g.pair_fw[np + n + v]]; /* residual of v -> t */
        }
        int64_t flow = 0;
        for (int32_t v = 0; v < n; v++) flow += (int64_t)ct[v] - rt[v];
        if (flow_out) *flow_out = flow;
        for (int64_t i = 0; i < np; i++) {
            if (r_uv) r_uv[i] = g.res[g.pair_fw[i]];
            if (r_vu) r_vu[i] = g.res[g.pair_bw[i]];
        }
        if (rt_out) memcpy(rt_out, rt, sizeof(int64_t) * (size_t)n);
        if (ex_out) memcpy(ex_out, ex, sizeof(int64_t) * (size_t)n);
        /* cuts: restrict the n+2 network to the n vertices by the same searches */
        uint8_t *mark = calloc((size_t)N, 1);
        if (!mark) { free(rt); free(ex); rc = ORC_ENOMEM; goto out; }
        int64_t qh = 0, qt = 0;
        mark[S] = 1;
        queue[qt++] = S;
        while (qh < qt) {
            int32_t u = queue[qh++];
            for (int64_t a = g.first[u]; a < g.first[u + 1]; a++)
                if (!mark[g.head[a]] && g.res[a] > 0) { mark[g.head[a]] = 1; queue[qt++] = g.head[a]; }
        }
        if (smin) for (int32_t v = 0; v < n; v++) smin[v] = mark[v];
        memset(mark, 0, (size_t)N);
        qh = qt = 0;
        mark[T] = 1;
        queue[qt++] = T;
        while (qh < qt) {
            int32_t w = queue[qh++];
            for (int64_t a = g.first[w]; a < g.first[w + 1]; a++) {
                int32_t u = g.head[a];
                if (!mark[u] && g.res[g.rev[a]] > 0) { mark[u] = 1; queue[qt++] = u; }
            }
        }
        if (smax) for (int32_t v = 0; v < n; v++) smax[v] = mark[v] ? 0 : 1;
        free(mark); free(rt); free(ex);
    }
out:
    free(PU); free(PV); free(CU); free(CV); free(level); free(queue); free(it); free(stack_arc);
    net_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Cuts of a given residual state (used to certify states made elsewhere).  */
/* ------------------------------------------------------------------------ */
int orc_cuts(int32_t n, int64_t np, const int32_t *pu, const int32_t *pv, const int64_t *r_uv,
             const int64_t *r_vu, const int64_t *rt, const int64_t *ex, uint8_t *smin,
             uint8_t *smax) {
    /* build with zero caps, then load the residuals */
    int32_t *z = calloc((size_t)(np ? np : 1), sizeof(int32_t));
    if (!z) return ORC_ENOMEM;
    net_t g;
    int rc = net_build(&g, n, np, pu, pv, z, z);
    free(z);
    if (rc) return rc;
    for (int64_t i = 0; i < np; i++) {
        g.res[g.pair_fw[i]] = r_uv[i];
        g.res[g.pair_bw[i]] = r_vu[i];
    }
    rc = cuts_from_residual(&g, rt, ex, smin, smax);
    net_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Reference region discharge (Sec. 3 Alg. 1/2, Sec. 4.2 ARD, Sec. 5.1).    */
/* ------------------------------------------------------------------------ */
typedef struct {
    net_t *g;
    const int32_t *region;  /* region id of every vertex */
    int32_t nreg;
    int64_t *ex, *rt;
    int32_t *d;             /* labels in {0..dinf} */
    int32_t dinf;           /* |B|, at least 1 */
    uint8_t *inB;           /* boundary membership (Sec. 4.1) */
    int64_t *first_r;       /* vertices grouped by region: members[first_r[k]..first_r[k+1]) */
    int32_t *members;
    /* scratch */
    int64_t *parent;
    int32_t *queue;
    uint8_t *seen;
    int32_t *newd;
    int64_t *push;          /* per arc: flow sent over an outgoing boundary arc in this discharge */
} ard_t;

static int ard_is_boundary_arc(const ard_t *A, int64_t a) {
    return A->region[A->g->tail[a]] != A->region[A->g->head[a]];
}

/* Augment(R, T_k) of Sec. 4.2: while a residual path of G^R leads from a vertex
 * of R with positive excess to t or to a boundary vertex w with d(w) < k, push
 * min(excess of its first vertex, bottleneck) along it.  Paths are found by
 * breadth-first search from all excess vertices at once.  Arcs from B^R into R
 * have capacity 0 in G^R and are never used; the search never leaves R except
 * by the last arc of a path. */
static int64_t ard_augment(ard_t *A, int32_t rk, int32_t k, const int32_t *dold) {
    net_t *g = A->g;
    int64_t lo = A->first_r[rk], hi = A->first_r[rk + 1];
    int64_t to_t = 0;
    for (;;) {
        int64_t qh = 0, qt = 0;
        for (int64_t i = lo; i < hi; i++) A->seen[A->members[i]] = 0;
        for (int64_t i = lo; i < hi; i++) {
            int32_t v = A->members[i];
            if (A->ex[v] > 0) { A->seen[v] = 1; A->parent[v] = -1; A->queue[qt++] = v; }
        }
        int32_t end_vertex = -1;
        int64_t end_arc = -1; /* -1: path ends in t; else the boundary arc used */
        while (qh < qt && end_vertex < 0) {
            int32_t u = A->queue[qh++];
            if (A->rt[u] > 0) { end_vertex = u; end_arc = -1; break; }
            for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
                if (g->res[a] <= 0) continue;
                int32_t w = g->head[a];
                if (ard_is_boundary_arc(A, a)) {
                    if (dold[w] < k) { end_vertex = u; end_arc = a; break; }
                    continue;
                }
                if (!A->seen[w]) { A->seen[w] = 1; A->parent[w] = a; A->queue[qt++] = w; }
            }
        }
        if (end_vertex < 0) break;
        /* bottleneck along the path, ending with the t-link or the boundary arc */
        int64_t delta = end_arc < 0 ? A->rt[end_vertex] : g->res[end_arc];
        int32_t v = end_vertex;
        while (A->parent[v] >= 0) {
            int64_t a = A->parent[v];
            if (g->res[a] < delta) delta = g->res[a];
            v = g->tail[a];
        }
        if (A->ex[v] < delta) delta = A->ex[v];
        /* augment */
        A->ex[v] -= delta;
        int32_t x = end_vertex;
        while (A->parent[x] >= 0) {
            int64_t a = A->parent[x];
            g->res[a] -= delta;
            g->res[g->rev[a]] += delta;
            x = g->tail[a];
        }
        if (end_arc < 0) {
            A->rt[end_vertex] -= delta;
            to_t += delta;
        } else {
            g->res[end_arc] -= delta;   /* the reverse arc stays untouched until fusion */
            A->push[end_arc] += delta;
        }
    }
    return to_t;
}

/* Region relabel (Alg. 3, ARD variant): labels of R become
 * min{k : u reaches T_k} with T_k = {t} u {w in B^R : d(w) < k}, or dinf. */
static void ard_region_relabel(ard_t *A, int32_t rk, const int32_t *dold) {
    net_t *g = A->g;
    int64_t lo = A->first_r[rk], hi = A->first_r[rk + 1];
    for (int64_t i = lo; i < hi; i++) A->newd[A->members[i]] = A->dinf;
    int32_t cur = 0;
    int64_t qh = 0, qt = 0;
    /* seeds at level 0: vertices of R with a residual t-link */
    for (int64_t i = lo; i < hi; i++) {
        int32_t u = A->members[i];
        if (A->rt[u] > 0) { A->newd[u] = 0; A->queue[qt++] = u; }
    }
    for (;;) {
        /* flood backward inside R: an unlabeled u with c_f(u,v) > 0 to an open v gets cur */
        while (qh < qt) {
            int32_t v = A->queue[qh++];
            for (int64_t a = g->first[v]; a < g->first[v + 1]; a++) {
                int32_t u = g->head[a];
                if (A->region[u] != rk) continue;
                if (A->newd[u] == A->dinf && g->res[g->rev[a]] > 0) {
                    A->newd[u] = cur;
                    A->queue[qt++] = u;
                }
            }
        }
        /* next seed level: smallest d(w)+1 > cur over residual boundary arcs from unlabeled u */
        int32_t next = -1;
        for (int64_t i = lo; i < hi; i++) {
            int32_t u = A->members[i];
            if (A->newd[u] != A->dinf) continue;
            for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
                if (!ard_is_boundary_arc(A, a) || g->res[a] <= 0) continue;
                int32_t w = g->head[a];
                if (dold[w] >= A->dinf) continue;
                int32_t lvl = dold[w] + 1;
                if (lvl > cur && (next < 0 || lvl < next)) next = lvl;
            }
        }
        if (next < 0) break;
        cur = next;
        for (int64_t i = lo; i < hi; i++) {
            int32_t u = A->members[i];
            if (A->newd[u] != A->dinf) continue;
            for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
                if (!ard_is_boundary_arc(A, a) || g->res[a] <= 0) continue;
                int32_t w = g->head[a];
                if (dold[w] < A->dinf && dold[w] + 1 == cur) {
                    A->newd[u] = cur;
                    A->queue[qt++] = u;
                    break;
                }
            }
        }
    }
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Proc. ARD: stages k in {0} u {d(w)+1 : w in B^R, d(w) < dinf}, ascending (the
 * targets T_k only change at these values), then region relabel.  dold holds
 * the labels the discharge reads (boundary labels stay fixed).  Pushes over
 * outgoing boundary arcs are accumulated in A->push.  Stages above cap are not
 * run (partial discharge, Sec. 6.2: cap = the sweep index); the region relabel
 * is always complete. */
static int64_t ard_discharge(ard_t *A, int32_t rk, const int32_t *dold, int32_t cap) {
    net_t *g = A->g;
    int64_t lo = A->first_r[rk], hi = A->first_r[rk + 1];
    int64_t cnt = 0;
    int32_t *lv = NULL;
    for (int64_t i = lo; i < hi; i++) {
        int32_t u = A->members[i];
        for (int64_t a = g->first[u]; a < g->first[u + 1]; a++)
            if (ard_is_boundary_arc(A, a)) cnt++;
    }
    lv = malloc(sizeof(int32_t) * (size_t)(cnt + 1));
    int64_t nl = 0;
    lv[nl++] = 0;
    for (int64_t i = lo; i < hi; i++) {
        int32_t u = A->members[i];
        for (int64_t a = g->first[u]; a < g->first[u + 1]; a++)
            if (ard_is_boundary_arc(A, a) && dold[g->head[a]] < A->dinf)
                lv[nl++] = dold[g->head[a]] + 1;
    }
    qsort(lv, (size_t)nl, sizeof(int32_t), cmp_i32);
    int64_t to_t = 0;
    for (int64_t i = 0; i < nl; i++) {
        if (i > 0 && lv[i] == lv[i - 1]) continue;
        if (lv[i] > cap) break;
        to_t += ard_augment(A, rk, lv[i], dold);
    }
    free(lv);
    ard_region_relabel(A, rk, dold);
    return to_t;
}

/* Global gap over boundary labels (Sec. 5.1 with the |B|-bin histogram of
 * Sec. 5.3): if no vertex of B has label g >= 1 below the highest finite
 * boundary label, every vertex with g < d < dinf cannot reach t. */
static void ard_gap(ard_t *A) {
    int32_t n = A->g->n;
    int32_t top = -1;
    for (int32_t v = 0; v < n; v++)
        if (A->inB[v] && A->d[v] < A->dinf && A->d[v] > top) top = A->d[v];
    if (top < 2) return;
    uint8_t *present = calloc((size_t)top + 1, 1);
    for (int32_t v = 0; v < n; v++)
        if (A->inB[v] && A->d[v] < A->dinf) present[A->d[v]] = 1;
    int32_t gap = -1;
    for (int32_t l = 1; l < top; l++)
        if (!present[l]) { gap = l; break; }
    free(present);
    if (gap < 0) return;
    for (int32_t v = 0; v < n; v++)
        if (A->d[v] > gap && A->d[v] < A->dinf) A->d[v] = A->dinf;
}

/* 0-1 breadth-first search from t: exact region distance d*B (Sec. 4.1),
 * arcs between regions have length 1, arcs inside a region length 0.
 * Processed level by level: a level's list grows while it is scanned
 * (length-0 arcs), length-1 arcs feed the next level's list. */
static void ard_region_distance(ard_t *A, int32_t *dist) {
    net_t *g = A->g;
    int32_t n = g->n;
    int32_t *cur = malloc(sizeof(int32_t) * (size_t)(2 * (int64_t)n + 1));
    int32_t *nxt = malloc(sizeof(int32_t) * (size_t)(2 * (int64_t)n + 1));
    int64_t ncur = 0, nnxt = 0;
    for (int32_t v = 0; v < n; v++) dist[v] = A->dinf;
    for (int32_t v = 0; v < n; v++)
        if (A->rt[v] > 0) { dist[v] = 0; cur[ncur++] = v; }
    int32_t level = 0;
    while (ncur > 0) {
        for (int64_t i = 0; i < ncur; i++) {
            int32_t w = cur[i];
            if (dist[w] != level) continue; /* settled at a smaller level already */
            for (int64_t a = g->first[w]; a < g->first[w + 1]; a++) {
                int32_t u = g->head[a];
                if (g->res[g->rev[a]] <= 0) continue;
                if (A->region[u] == A->region[w]) {
                    if (dist[u] > level) { dist[u] = level; cur[ncur++] = u; }
                } else if (dist[u] > level + 1) {
                    dist[u] = level + 1;
                    nxt[nnxt++] = u;
                }
            }
        }
        int32_t *t = cur; cur = nxt; nxt = t;
        ncur = nnxt; nnxt = 0;
        level++;
    }
    for (int32_t v = 0; v < n; v++) if (dist[v] > A->dinf) dist[v] = A->dinf;
    free(cur); free(nxt);
}

/* Boundary relabel heuristic (Sec. 6.1), with the auxiliary graph built as
 * the section describes:
 *   - nodes: the vertices of every region grouped by label, labels below dinf
 *     only (vertices labelled dinf take no part);
 *   - an arc of length 0 from each group to the group of the next larger label
 *     of the same region (a vertex may reach a higher-labelled one inside its
 *     region, never a lower-labelled one: validity);
 *   - an arc of length 1 from the group of u to the group of w for every
 *     residual arc (u, w) between regions.
 * d'(u) is the length of a shortest path from the group of u to a group of
 * label 0, by Dijkstra's algorithm (run from the label-0 groups over the
 * reversed arcs), and the labels become max(d, d'), with dinf where no label-0
 * group is reached.  The section groups the boundary vertices; interior
 * vertices are grouped too, so the whole labeling stays valid (an interior
 * group has no arc of length 1, so it only passes on the distance of the next
 * larger label of its region, and the boundary groups' distances are the same
 * either way).  Returns 0 or ORC_ENOMEM. */
typedef struct { int64_t key; int32_t v; } brl_item_t;

static int brl_cmp(const void *a, const void *b) {
    int64_t x = ((const brl_item_t *)a)->key, y = ((const brl_item_t *)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int ard_boundary_relabel(ard_t *A) {
    net_t *g = A->g;
    const int32_t n = g->n;
    const int64_t INF = INT64_MAX;
    int rc = ORC_OK;
    brl_item_t *it = malloc(sizeof(brl_item_t) * (size_t)(n ? n : 1));
    int32_t *grp = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *glab = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *greg = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *first = NULL, *dist = NULL, *heap = NULL;
    int32_t *to = NULL, *len = NULL, *afrom = NULL, *ato = NULL, *alen = NULL;
    if (!it || !grp || !glab || !greg) { rc = ORC_ENOMEM; goto out; }
    /* groups: vertices with d < dinf sorted by (region, label) */
    int32_t cnt = 0;
    for (int32_t v = 0; v < n; v++) {
        grp[v] = -1;
        if (A->d[v] >= A->dinf) continue;
        it[cnt].key = (int64_t)A->region[v] * ((int64_t)A->dinf + 1) + A->d[v];
        it[cnt].v = v;
        cnt++;
    }
    qsort(it, (size_t)cnt, sizeof(brl_item_t), brl_cmp);
    int32_t ng = 0;
    for (int32_t i = 0; i < cnt; i++) {
        if (i == 0 || it[i].key != it[i - 1].key) {
            glab[ng] = A->d[it[i].v];
            greg[ng] = A->region[it[i].v];
            ng++;
        }
        grp[it[i].v] = ng - 1;
    }
    /* arcs of the auxiliary graph, (from, to, length) */
    int64_t cap = (int64_t)ng + g->m + 1, na = 0;
    afrom = malloc(sizeof(int32_t) * (size_t)cap);
    ato = malloc(sizeof(int32_t) * (size_t)cap);
    alen = malloc(sizeof(int32_t) * (size_t)cap);
    if (!afrom || !ato || !alen) { rc = ORC_ENOMEM; goto out; }
    for (int32_t q = 0; q + 1 < ng; q++)
        if (greg[q] == greg[q + 1]) { afrom[na] = q; ato[na] = q + 1; alen[na] = 0; na++; }
    for (int64_t a = 0; a < g->m; a++) {
        if (g->res[a] <= 0) continue;
        int32_t u = g->tail[a], w = g->head[a];
        if (A->region[u] == A->region[w] || grp[u] < 0 || grp[w] < 0) continue;
        afrom[na] = grp[u]; ato[na] = grp[w]; alen[na] = 1; na++;
    }
    /* reversed adjacency (CSR over the arc heads) */
    first = calloc((size_t)ng + 1, sizeof(int64_t));
    to = malloc(sizeof(int32_t) * (size_t)(na ? na : 1));
    len = malloc(sizeof(int32_t) * (size_t)(na ? na : 1));
    dist = malloc(sizeof(int64_t) * (size_t)(ng ? ng : 1));
    heap = malloc(sizeof(int64_t) * (size_t)(na + ng + 1));
    if (!first || !to || !len || !dist || !heap) { rc = ORC_ENOMEM; goto out; }
    for (int64_t e = 0; e < na; e++) first[ato[e] + 1]++;
    for (int32_t q = 0; q < ng; q++) first[q + 1] += first[q];
    {
        int64_t *fill = malloc(sizeof(int64_t) * ((size_t)ng + 1));
        if (!fill) { rc = ORC_ENOMEM; goto out; }
        memcpy(fill, first, sizeof(int64_t) * ((size_t)ng + 1));
        for (int64_t e = 0; e < na; e++) {
            int64_t k = fill[ato[e]]++;
            to[k] = afrom[e];
            len[k] = alen[e];
        }
        free(fill);
    }
    /* Dijkstra from every label-0 group; heap entries are dist * 2^31 + group */
    int64_t hn = 0;
    for (int32_t q = 0; q < ng; q++) {
        dist[q] = INF;
        if (glab[q] == 0) {
            dist[q] = 0;
            heap[hn++] = q; /* distance 0: key = group */
        }
    }
    /* heapify (keys are distinct: the group is part of the key) */
    for (int64_t i = hn / 2 - 1; i >= 0; i--) {
        int64_t j = i;
        for (;;) {
            int64_t l = 2 * j + 1, r = l + 1, m = j;
            if (l < hn && heap[l] < heap[m]) m = l;
            if (r < hn && heap[r] < heap[m]) m = r;
            if (m == j) break;
            int64_t t = heap[j]; heap[j] = heap[m]; heap[m] = t; j = m;
        }
    }
    while (hn > 0) {
        int64_t top = heap[0];
        heap[0] = heap[--hn];
        for (int64_t j = 0;;) {
            int64_t l = 2 * j + 1, r = l + 1, m = j;
            if (l < hn && heap[l] < heap[m]) m = l;
            if (r < hn && heap[r] < heap[m]) m = r;
            if (m == j) break;
            int64_t t = heap[j]; heap[j] = heap[m]; heap[m] = t; j = m;
        }
        int64_t du = top >> 31;
        int32_t q = (int32_t)(top & 0x7fffffff);
        if (du != dist[q]) continue; /* stale entry */
        for (int64_t k = first[q]; k < first[q + 1]; k++) {
            int32_t p = to[k];
            int64_t nd = du + len[k];
            if (nd < dist[p]) {
                dist[p] = nd;
                int64_t j = hn++;
                heap[j] = (nd << 31) | p;
                while (j > 0 && heap[(j - 1) / 2] > heap[j]) {
                    int64_t t = heap[j]; heap[j] = heap[(j - 1) / 2]; heap[(j - 1) / 2] = t;
                    j = (j - 1) / 2;
                }
            }
        }
    }
    /* d := max(d, d') */
    for (int32_t v = 0; v < n; v++) {
        if (grp[v] < 0) continue;
        int64_t dp = dist[grp[v]];
        if (dp > A->dinf) dp = A->dinf;
        if (dp > A->d[v]) A->d[v] = (int32_t)dp;
    }
out:
    free(it); free(grp); free(glab); free(greg); free(first); free(dist); free(heap);
    free(to); free(len); free(afrom); free(ato); free(alen);
    return rc;
}

/* The heuristic alone on a given residual state: c(pu, pv) = r_uv[i] and
 * c(pv, pu) = r_vu[i] are the residuals, labels (n entries, values in
 * 0..dinf) are raised in place. */
int orc_boundary_relabel(int32_t n, int64_t np, const int32_t *pu, const int32_t *pv,
                         const int32_t *r_uv, const int32_t *r_vu, const int32_t *region,
                         int32_t dinf, int32_t *labels) {
    net_t g;
    int rc = net_build(&g, n, np, pu, pv, r_uv, r_vu);
    if (rc) return rc;
    ard_t A;
    memset(&A, 0, sizeof(A));
    A.g = &g;
    A.region = region;
    A.d = labels;
    A.dinf = dinf;
    rc = ard_boundary_relabel(&A);
    net_free(&g);
    return rc;
}

/* Validity of a labeling w.r.t. the region distance (Sec. 4.1). */
static int ard_valid(const ard_t *A, const int32_t *d) {
    net_t *g = A->g;
    for (int32_t u = 0; u < g->n; u++) {
        if (A->rt[u] > 0 && d[u] > 0) return 0;
        for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
            if (g->res[a] <= 0) continue;
            int32_t v = g->head[a];
            int32_t len = A->region[u] != A->region[v] ? 1 : 0;
            if (d[u] > d[v] + len) return 0;
        }
    }
    return 1;
}

/* check bits */
#define ORC_CHK_VALID 1     /* labeling valid after every sweep */
#define ORC_CHK_MONO 2      /* labels never decrease */
#define ORC_CHK_ACTIVE_B 4  /* after the first sweep only boundary vertices are active */
#define ORC_CHK_LOWER 8     /* labels never exceed the exact region distance */
#define ORC_CHK_DISCHARGE 16 /* no active vertex left in a region right after its discharge */

/* heuristics of Sec. 6 (bits of orc_ard's heur) */
#define ORC_HEUR_PARTIAL 1  /* partial discharges (Sec. 6.2) */
#define ORC_HEUR_BRL 2      /* boundary relabel after every sweep (Sec. 6.1) */

int orc_ard(int32_t n, int64_t np, const int32_t *pu, const int32_t *pv, const int32_t *cuv,
            const int32_t *cvu, const int32_t *cs, const int32_t *ct, const int32_t *region,
            int32_t parallel, int32_t heur, int64_t max_sweeps, int32_t checks, int64_t *r_uv,
            int64_t *r_vu,
            int64_t *rt_out, int64_t *ex_out, int64_t *flow_out, uint8_t *smin, uint8_t *smax,
            int32_t *labels_out, int64_t *sweeps_out, int64_t *bsize_out, int32_t *failed_check) {
    net_t g;
    int rc = net_build(&g, n, np, pu, pv, cuv, cvu);
    if (rc) return rc;
    ard_t A;
    memset(&A, 0, sizeof(A));
    A.g = &g;
    A.region = region;
    int32_t nreg = 0;
    for (int32_t v = 0; v < n; v++) {
        if (region[v] < 0) { net_free(&g); return ORC_EINVAL; }
        if (region[v] + 1 > nreg) nreg = region[v] + 1;
    }
    A.nreg = nreg;
    size_t nn = (size_t)(n ? n : 1);
    A.ex = malloc(sizeof(int64_t) * nn);
    A.rt = malloc(sizeof(int64_t) * nn);
    A.d = malloc(sizeof(int32_t) * nn);
    A.inB = calloc(nn, 1);
    A.first_r = calloc((size_t)nreg + 1, sizeof(int64_t));
    A.members = malloc(sizeof(int32_t) * nn);
    A.parent = malloc(sizeof(int64_t) * nn);
    A.queue = malloc(sizeof(int32_t) * nn);
    A.seen = malloc(nn);
    A.newd = malloc(sizeof(int32_t) * nn);
    A.push = calloc((size_t)(g.m ? g.m : 1), sizeof(int64_t));
    int32_t *dsnap = malloc(sizeof(int32_t) * nn);
    int32_t *dprev = malloc(sizeof(int32_t) * nn);
    int32_t *dstar = malloc(sizeof(int32_t) * nn);
    if (!A.ex || !A.rt || !A.d || !A.inB || !A.first_r || !A.members || !A.parent || !A.queue ||
        !A.seen || !A.newd || !A.push || !dsnap || !dprev || !dstar) {
        rc = ORC_ENOMEM;
        goto done;
    }
    if (failed_check) *failed_check = 0;
    /* boundary B: vertices incident to a pair whose ends lie in different regions */
    int64_t bsize = 0;
    for (int64_t i = 0; i < np; i++)
        if (region[pu[i]] != region[pv[i]]) { A.inB[pu[i]] = 1; A.inB[pv[i]] = 1; }
    for (int32_t v = 0; v < n; v++) bsize += A.inB[v];
    A.dinf = bsize > 0 ? (int32_t)bsize : 1;
    if (bsize_out) *bsize_out = bsize;
    for (int32_t v = 0; v < n; v++) A.first_r[region[v] + 1]++;
    for (int32_t k = 0; k < nreg; k++) A.first_r[k + 1] += A.first_r[k];
    {
        int64_t *fill = malloc(sizeof(int64_t) * ((size_t)nreg + 1));
        memcpy(fill, A.first_r, sizeof(int64_t) * ((size_t)nreg + 1));
        for (int32_t v = 0; v < n; v++) A.members[fill[region[v]]++] = v;
        free(fill);
    }
    /* Init */
    for (int32_t v = 0; v < n; v++) {
        if (cs[v] < 0 || ct[v] < 0) { rc = ORC_EINVAL; goto done; }
        A.ex[v] = cs[v];
        A.rt[v] = ct[v];
        A.d[v] = 0;
    }
    int64_t sweeps = 0;
    for (;;) {
        int any_active = 0;
        for (int32_t v = 0; v < n && !any_active; v++)
            if (A.ex[v] > 0 && A.d[v] < A.dinf) any_active = 1;
        if (!any_active) break;
        if (sweeps >= max_sweeps) {
            /* stopped early: the state after max_sweeps sweeps (no cuts) */
            if (sweeps_out) *sweeps_out = sweeps;
            if (labels_out) memcpy(labels_out, A.d, sizeof(int32_t) * (size_t)n);
            write_outputs(&g, np, A.rt, A.ex, ct, r_uv, r_vu, rt_out, ex_out, flow_out);
            rc = ORC_ESWEEPS;
            goto done;
        }
        if (sweeps > 0 && (checks & ORC_CHK_ACTIVE_B)) {
            for (int32_t v = 0; v < n; v++)
                if (A.ex[v] > 0 && A.d[v] < A.dinf && !A.inB[v]) {
                    rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_ACTIVE_B; goto done;
                }
        }
        memcpy(dprev, A.d, sizeof(int32_t) * nn);
        /* partial discharges: sweep s runs stages up to s only */
        const int32_t cap = (heur & ORC_HEUR_PARTIAL) ? (int32_t)(sweeps < INT32_MAX ? sweeps : INT32_MAX)
                                                      : INT32_MAX;
        sweeps++;
        if (parallel) {
            /* Alg. 2: all regions discharge against the labels of the sweep start */
            memcpy(dsnap, A.d, sizeof(int32_t) * nn);
            memset(A.push, 0, sizeof(int64_t) * (size_t)(g.m ? g.m : 1));
            for (int32_t rk = 0; rk < nreg; rk++) {
                int has_active = 0;
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t v = A.members[i];
                    if (A.ex[v] > 0 && dsnap[v] < A.dinf) { has_active = 1; break; }
                }
                if (!has_active) continue; /* a region with no active vertex is skipped */
                ard_discharge(&A, rk, dsnap, cap);
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t v = A.members[i];
                    A.d[v] = A.newd[v]; /* fuse labels */
                    if ((checks & ORC_CHK_DISCHARGE) && A.ex[v] > 0 && A.newd[v] < A.dinf) {
                        rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_DISCHARGE; goto done;
                    }
                }
            }
            /* fuse flow: a push over (u,v) between regions stays iff alpha(v,u) = [d'(v) <= d'(u)+1];
             * otherwise it returns to u (Alg. 2 valid pairs). */
            for (int64_t a = 0; a < g.m; a++) {
                if (A.push[a] == 0) continue;
                int32_t u = g.tail[a], v = g.head[a];
                int64_t p = A.push[a];
                if (A.d[v] <= A.d[u] + 1) {
                    g.res[g.rev[a]] += p;
                    A.ex[v] += p;
                } else {
                    g.res[a] += p;
                    A.ex[u] += p;
                }
            }
            /* boundary relabel on the fused state, then the gap over its labels */
            if ((heur & ORC_HEUR_BRL) && (rc = ard_boundary_relabel(&A)) != ORC_OK) goto done;
            ard_gap(&A);
        } else {
            /* Alg. 1: regions one by one, each sees the current state */
            for (int32_t rk = 0; rk < nreg; rk++) {
                int has_active = 0;
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t v = A.members[i];
                    if (A.ex[v] > 0 && A.d[v] < A.dinf) { has_active = 1; break; }
                }
                if (!has_active) continue;
                memset(A.push, 0, sizeof(int64_t) * (size_t)(g.m ? g.m : 1));
                ard_discharge(&A, rk, A.d, cap);
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t v = A.members[i];
                    A.d[v] = A.newd[v];
                    if ((checks & ORC_CHK_DISCHARGE) && A.ex[v] > 0 && A.newd[v] < A.dinf) {
                        rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_DISCHARGE; goto done;
                    }
                }
                /* apply the discharge's flow on the boundary arcs: G := G_f' */
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t u = A.members[i];
                    for (int64_t a = g.first[u]; a < g.first[u + 1]; a++) {
                        if (A.push[a] == 0) continue;
                        g.res[g.rev[a]] += A.push[a];
                        A.ex[g.head[a]] += A.push[a];
                    }
                }
                ard_gap(&A);
            }
            if ((heur & ORC_HEUR_BRL) && (rc = ard_boundary_relabel(&A)) != ORC_OK) goto done;
        }
        if (checks & ORC_CHK_MONO)
            for (int32_t v = 0; v < n; v++)
                if (A.d[v] < dprev[v]) {
                    rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_MONO; goto done;
                }
        if ((checks & ORC_CHK_VALID) && !ard_valid(&A, A.d)) {
            rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_VALID; goto done;
        }
        if (checks & ORC_CHK_LOWER) {
            ard_region_distance(&A, dstar);
            for (int32_t v = 0; v < n; v++)
                if (A.d[v] > dstar[v]) {
                    rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_LOWER; goto done;
                }
        }
    }
    if (sweeps_out) *sweeps_out = sweeps;
    if (labels_out) memcpy(labels_out, A.d, sizeof(int32_t) * (size_t)n);
    write_outputs(&g, np, A.rt, A.ex, ct, r_uv, r_vu, rt_out, ex_out, flow_out);
    rc = cuts_from_residual(&g, A.rt, A.ex, smin, smax);
done:
    free(A.ex); free(A.rt); free(A.d); free(A.inB); free(A.first_r); free(A.members);
    free(A.parent); free(A.queue); free(A.seen); free(A.newd); free(A.push);
    free(dsnap); free(dprev); free(dstar);
    net_free(&g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Push-relabel region discharge (Sec. 3, Proc. PRD) with the generic       */
/* drivers: Alg. 1 (S-PRD) and Alg. 2 (P-PRD, label and flow fusion).       */
/* Labels are the distance labels of Sec. 2: d(t) = 0, every arc has length */
/* 1, valid iff d(u) <= d(v) + 1 on every residual arc; dinf = n.           */
/* ------------------------------------------------------------------------ */

/* Proc. PRD on the region network of region rk: Push and Relabel, first in
 * first out over the active vertices of the region, until none is left.  The
 * labels of the boundary vertices outside the region (dold) stay fixed; a
 * push over an arc (u, w) leaving the region is recorded in push[] and
 * removed from c_f(u, w) (the arcs (w, u) belong to the neighbour's network).
 * New labels of the region's vertices go to newd. */
static void prd_discharge(ard_t *A, int32_t rk, const int32_t *dold) {
    net_t *g = A->g;
    const int64_t lo = A->first_r[rk], hi = A->first_r[rk + 1];
    int32_t *d = A->newd;
    for (int64_t i = lo; i < hi; i++) d[A->members[i]] = dold[A->members[i]];
    /* FIFO of active vertices; a vertex is queued at most once at a time */
    const int64_t cap = hi - lo + 1;
    int64_t qh = 0, qt = 0;
    for (int64_t i = lo; i < hi; i++) {
        int32_t v = A->members[i];
        A->seen[v] = 0;
        if (A->ex[v] > 0 && d[v] < A->dinf) { A->queue[qt++ % cap] = v; A->seen[v] = 1; }
    }
    while (qh != qt) {
        int32_t u = A->queue[qh++ % cap];
        A->seen[u] = 0;
        while (A->ex[u] > 0 && d[u] < A->dinf) {
            int pushed = 0;
            /* Push: to t if d(u) = 1, else along (u, v) with d(u) = d(v) + 1 */
            if (A->rt[u] > 0 && d[u] == 1) {
                int64_t delta = A->ex[u] < A->rt[u] ? A->ex[u] : A->rt[u];
                A->rt[u] -= delta;
                A->ex[u] -= delta;
                pushed = 1;
            }
            for (int64_t a = g->first[u]; a < g->first[u + 1] && A->ex[u] > 0; a++) {
                if (g->res[a] <= 0) continue;
                int32_t v = g->head[a];
                const int inside = A->region[v] == rk;
                const int32_t dv = inside ? d[v] : dold[v];
                if (d[u] != dv + 1) continue;
                int64_t delta = A->ex[u] < g->res[a] ? A->ex[u] : g->res[a];
                g->res[a] -= delta;
                A->ex[u] -= delta;
                if (inside) {
                    g->res[g->rev[a]] += delta;
                    A->ex[v] += delta;
                    if (!A->seen[v] && d[v] < A->dinf) { A->queue[qt++ % cap] = v; A->seen[v] = 1; }
                } else {
                    A->push[a] += delta;
                }
                pushed = 1;
            }
            if (A->ex[u] <= 0) break;
            if (!pushed || A->ex[u] > 0) {
                /* Relabel: 1 + the smallest label over residual arcs (t counts 0) */
                int64_t best = A->rt[u] > 0 ? 1 : (int64_t)A->dinf;
                for (int64_t a = g->first[u]; a < g->first[u + 1]; a++) {
                    if (g->res[a] <= 0) continue;
                    int32_t v = g->head[a];
                    const int32_t dv = A->region[v] == rk ? d[v] : dold[v];
                    if ((int64_t)dv + 1 < best) best = (int64_t)dv + 1;
                }
                if (best > A->dinf) best = A->dinf;
                if (best <= d[u]) best = d[u] + 1; /* no admissible arc left: strictly up */
                if (best > A->dinf) best = A->dinf;
                d[u] = (int32_t)best;
            }
        }
    }
}

/* Global gap over all labels (Sec. 5.1): the smallest g >= 1 below the largest
 * finite label with no vertex labelled g; labels above it go to dinf. */
static void prd_gap(ard_t *A) {
    int32_t n = A->g->n, top = -1;
    for (int32_t v = 0; v < n; v++)
        if (A->d[v] < A->dinf && A->d[v] > top) top = A->d[v];
    if (top < 2) return;
    uint8_t *present = calloc((size_t)top + 1, 1);
    if (!present) return;
    for (int32_t v = 0; v < n; v++)
        if (A->d[v] < A->dinf) present[A->d[v]] = 1;
    int32_t gap = -1;
    for (int32_t l = 1; l < top; l++)
        if (!present[l]) { gap = l; break; }
    free(present);
    if (gap < 0) return;
    for (int32_t v = 0; v < n; v++)
        if (A->d[v] > gap && A->d[v] < A->dinf) A->d[v] = A->dinf;
}

/* Validity of distance labels (Sec. 2): d(u) <= d(v) + 1 on residual arcs,
 * d(u) <= 1 where c_f(u, t) > 0. */
static int prd_valid(const ard_t *A) {
    net_t *g = A->g;
    for (int32_t u = 0; u < g->n; u++) {
        if (A->rt[u] > 0 && A->d[u] > 1) return 0;
        for (int64_t a = g->first[u]; a < g->first[u + 1]; a++)
            if (g->res[a] > 0 && A->d[u] > A->d[g->head[a]] + 1) return 0;
    }
    return 1;
}

int orc_prd(int32_t n, int64_t np, const int32_t *pu, const int32_t *pv, const int32_t *cuv,
            const int32_t *cvu, const int32_t *cs, const int32_t *ct, const int32_t *region,
            int32_t parallel, int32_t gap_on, int64_t max_sweeps, int32_t checks, int64_t *r_uv,
            int64_t *r_vu, int64_t *rt_out, int64_t *ex_out, int64_t *flow_out, uint8_t *smin,
            uint8_t *smax, int32_t *labels_out, int64_t *sweeps_out, int32_t *failed_check) {
    net_t g;
    int rc = net_build(&g, n, np, pu, pv, cuv, cvu);
    if (rc) return rc;
    ard_t A;
    memset(&A, 0, sizeof(A));
    A.g = &g;
    A.region = region;
    int32_t nreg = 0;
    for (int32_t v = 0; v < n; v++) {
        if (region[v] < 0) { net_free(&g); return ORC_EINVAL; }
        if (region[v] + 1 > nreg) nreg = region[v] + 1;
    }
    A.nreg = nreg;
    A.dinf = n > 0 ? n : 1;
    size_t nn = (size_t)(n ? n : 1);
    A.ex = malloc(sizeof(int64_t) * nn);
    A.rt = malloc(sizeof(int64_t) * nn);
    A.d = malloc(sizeof(int32_t) * nn);
    A.first_r = calloc((size_t)nreg + 1, sizeof(int64_t));
    A.members = malloc(sizeof(int32_t) * nn);
    A.queue = malloc(sizeof(int32_t) * (nn + 1));
    A.seen = malloc(nn);
    A.newd = malloc(sizeof(int32_t) * nn);
    A.push = calloc((size_t)(g.m ? g.m : 1), sizeof(int64_t));
    int32_t *dsnap = malloc(sizeof(int32_t) * nn);
    int32_t *dprev = malloc(sizeof(int32_t) * nn);
    if (!A.ex || !A.rt || !A.d || !A.first_r || !A.members || !A.queue || !A.seen || !A.newd ||
        !A.push || !dsnap || !dprev) {
        rc = ORC_ENOMEM;
        goto done;
    }
    if (failed_check) *failed_check = 0;
    for (int32_t v = 0; v < n; v++) A.first_r[region[v] + 1]++;
    for (int32_t k = 0; k < nreg; k++) A.first_r[k + 1] += A.first_r[k];
    {
        int64_t *fill = malloc(sizeof(int64_t) * ((size_t)nreg + 1));
        if (!fill) { rc = ORC_ENOMEM; goto done; }
        memcpy(fill, A.first_r, sizeof(int64_t) * ((size_t)nreg + 1));
        for (int32_t v = 0; v < n; v++) A.members[fill[region[v]]++] = v;
        free(fill);
    }
    for (int32_t v = 0; v < n; v++) {
        if (cs[v] < 0 || ct[v] < 0) { rc = ORC_EINVAL; goto done; }
        A.ex[v] = cs[v];
        A.rt[v] = ct[v];
        A.d[v] = 0;
    }
    int64_t sweeps = 0;
    for (;;) {
        int any_active = 0;
        for (int32_t v = 0; v < n && !any_active; v++)
            if (A.ex[v] > 0 && A.d[v] < A.dinf) any_active = 1;
        if (!any_active) break;
        if (sweeps >= max_sweeps) { rc = ORC_ESWEEPS; goto done; }
        memcpy(dprev, A.d, sizeof(int32_t) * nn);
        sweeps++;
        if (parallel) {
            memcpy(dsnap, A.d, sizeof(int32_t) * nn);
            memset(A.push, 0, sizeof(int64_t) * (size_t)(g.m ? g.m : 1));
            for (int32_t rk = 0; rk < nreg; rk++) {
                int has_active = 0;
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1] && !has_active; i++) {
                    int32_t v = A.members[i];
                    if (A.ex[v] > 0 && dsnap[v] < A.dinf) has_active = 1;
                }
                if (!has_active) continue;
                prd_discharge(&A, rk, dsnap);
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t v = A.members[i];
                    A.d[v] = A.newd[v];
                }
            }
            /* flow fusion of Alg. 2: a push over (u,v) between regions stays iff
             * d'(v) <= d'(u) + 1, otherwise it returns to u */
            for (int64_t a = 0; a < g.m; a++) {
                if (A.push[a] == 0) continue;
                int32_t u = g.tail[a], v = g.head[a];
                int64_t p = A.push[a];
                if (A.d[v] <= A.d[u] + 1) {
                    g.res[g.rev[a]] += p;
                    A.ex[v] += p;
                } else {
                    g.res[a] += p;
                    A.ex[u] += p;
                }
            }
            if (gap_on) prd_gap(&A);
        } else {
            for (int32_t rk = 0; rk < nreg; rk++) {
                int has_active = 0;
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1] && !has_active; i++) {
                    int32_t v = A.members[i];
                    if (A.ex[v] > 0 && A.d[v] < A.dinf) has_active = 1;
                }
                if (!has_active) continue;
                memset(A.push, 0, sizeof(int64_t) * (size_t)(g.m ? g.m : 1));
                prd_discharge(&A, rk, A.d);
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t v = A.members[i];
                    A.d[v] = A.newd[v];
                }
                for (int64_t i = A.first_r[rk]; i < A.first_r[rk + 1]; i++) {
                    int32_t u = A.members[i];
                    for (int64_t a = g.first[u]; a < g.first[u + 1]; a++) {
                        if (A.push[a] == 0) continue;
                        g.res[g.rev[a]] += A.push[a];
                        A.ex[g.head[a]] += A.push[a];
                    }
                }
                if (gap_on) prd_gap(&A);
            }
        }
        if (checks & ORC_CHK_MONO)
            for (int32_t v = 0; v < n; v++)
                if (A.d[v] < dprev[v]) {
                    rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_MONO; goto done;
                }
        if ((checks & ORC_CHK_VALID) && !prd_valid(&A)) {
            rc = ORC_ECHECK; if (failed_check) *failed_check = ORC_CHK_VALID; goto done;
        }
    }
    if (sweeps_out) *sweeps_out = sweeps;
    if (labels_out) memcpy(labels_out, A.d, sizeof(int32_t) * (size_t)n);
    write_outputs(&g, np, A.rt, A.ex, ct, r_uv, r_vu, rt_out, ex_out, flow_out);
    rc = cuts_from_residual(&g, A.rt, A.ex, smin, smax);
done:
    free(A.ex); free(A.rt); free(A.d); free(A.first_r); free(A.members); free(A.queue);
    free(A.seen); free(A.newd); free(A.push); free(dsnap); free(dprev);
    net_free(&g);
    return rc;
}
