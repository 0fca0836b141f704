/*
 * CPU FP64 oracle for the geodesic-interaction hot path of arXiv 2404.19751.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product path. Shares no code
 * with the HIP library. Plain, slow, obviously correct; built with
 * -O2 -ffp-contract=off and no fast-math.
 *
 * Sections:
 *   1. mesh: half-edges, corner angles, pseudo-source vertices (Sec. 2.2)
 *   2. geodesics by brute-force unfolding enumeration + Dijkstra over the
 *      bend vertices (Sec. 2.2 MMP paragraph; Sec. 3.1)
 *   2b. geodesics by window propagation with trimming (Sec. 2.2, the MMP
 *      continuous Dijkstra): a second exact route and the method's work count
 *   3. the shift walk (Sec. 3.2, steps (a)-(d), straightest rule at vertices)
 *   4. Philox4x32-10 (noise for the Brownian update of Sec. 2.1)
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559
#define PSEUDO_TOL 1e-9   /* angle sum >= 2 pi - tol counts as saddle (safe superset) */
#define TIE_REL 1e-9      /* default: candidates within this relative gap form the tie set */
#define DIR_DUP 1e-11     /* tangents closer than this angle are one direction: the same straight
                             link reached by two enumeration routes, which agree to rounding */
#define SEG_MIN_REL 1e-12 /* cone slices shorter than this (x edge length) are dropped */
#define CONE_EPS 1e-12    /* closed-cone slack for membership tests */
#define MAX_DEPTH 200000

/* ======================================================================
 * 1. Mesh
 * ====================================================================== */
struct orc_mesh {
    int nv, nf;
    double *V;             /* [nv][3] */
    int *T;                /* [nf][3]; half-edge h = 3f+k runs T[h] -> T[3f+(k+1)%3] */
    int *twin;             /* [3nf], -1 on the boundary */
    double *len;           /* [3nf] half-edge length */
    double *corner;        /* [3nf] angle of face h/3 at the tail of h */
    double *theta;         /* [nv] corner-angle sum */
    unsigned char *bnd;    /* [nv] boundary vertex */
    unsigned char *pseudo; /* [nv] saddle (theta >= 2pi - tol) or boundary */
    int *fan_off, *fan;    /* outgoing half-edges of each vertex in CCW order;
                              boundary fans start at the clockwise-most one */
    double *ex, *ey, *nrm; /* [nf][3] face frame: ex along edge 0, nrm outward */
    double mean_edge, max_edge;
};

static inline int he_next(int h) { return h - h % 3 + (h % 3 + 1) % 3; }
static inline int he_prev(int h) { return h - h % 3 + (h % 3 + 2) % 3; }

static inline void sub3(const double *a, const double *b, double *o) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double norm3(const double *a) { return sqrt(dot3(a, a)); }
static inline void unit3(double *a) {
    double l = norm3(a);
    a[0] /= l; a[1] /= l; a[2] /= l;
}

typedef struct { int a, b, h; } ekey;
static int ekey_cmp(const void *x, const void *y) {
    const ekey *p = (const ekey *)x, *q = (const ekey *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return p->h < q->h ? -1 : (p->h > q->h);
}

void orc_mesh_free(orc_mesh *m) {
    if (!m) return;
    free(m->V); free(m->T); free(m->twin); free(m->len); free(m->corner); free(m->theta);
    free(m->bnd); free(m->pseudo); free(m->fan_off); free(m->fan); free(m->ex); free(m->ey); free(m->nrm);
    free(m);
}

int orc_mesh_build(int nv, const double *V, int nf, const int *T, orc_mesh **out) {
    *out = NULL;
    if (nv <= 0 || nf <= 0 || !V || !T) return 1;
    for (int i = 0; i < 3 * nf; i++)
        if (T[i] < 0 || T[i] >= nv) return 1;
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    int ne = 3 * nf, rc = 0;
    m->nv = nv; m->nf = nf;
    m->V = (double *)malloc(sizeof(double) * 3 * nv);
    m->T = (int *)malloc(sizeof(int) * ne);
    memcpy(m->V, V, sizeof(double) * 3 * nv);
    memcpy(m->T, T, sizeof(int) * ne);
    m->twin = (int *)malloc(sizeof(int) * ne);
    m->len = (double *)malloc(sizeof(double) * ne);
    m->corner = (double *)malloc(sizeof(double) * ne);
    m->theta = (double *)calloc(nv, sizeof(double));
    m->bnd = (unsigned char *)calloc(nv, 1);
    m->pseudo = (unsigned char *)calloc(nv, 1);
    m->ex = (double *)malloc(sizeof(double) * 3 * nf);
    m->ey = (double *)malloc(sizeof(double) * 3 * nf);
    m->nrm = (double *)malloc(sizeof(double) * 3 * nf);

    /* twins: pair up the two half-edges of every undirected edge */
    ekey *keys = (ekey *)malloc(sizeof(ekey) * ne);
    for (int h = 0; h < ne; h++) {
        int a = m->T[h], b = m->T[he_next(h)];
        keys[h].a = a < b ? a : b; keys[h].b = a < b ? b : a; keys[h].h = h;
        m->twin[h] = -1;
    }
    qsort(keys, ne, sizeof(ekey), ekey_cmp);
    for (int i = 0; i < ne;) {
        int j = i;
        while (j < ne && keys[j].a == keys[i].a && keys[j].b == keys[i].b) j++;
        if (j - i > 2) { rc = 2; break; }
        if (j - i == 2) {
            int h1 = keys[i].h, h2 = keys[i + 1].h;
            if (m->T[h1] != m->T[he_next(h2)] || m->T[he_next(h1)] != m->T[h2]) { rc = 3; break; }
            m->twin[h1] = h2; m->twin[h2] = h1;
        }
        i = j;
    }
    free(keys);
    if (rc) { orc_mesh_free(m); return rc; }

    /* lengths, corner angles, face frames */
    double esum = 0.0; int ecount = 0;
    m->max_edge = 0.0;
    for (int f = 0; f < nf; f++) {
        for (int k = 0; k < 3; k++) {
            int h = 3 * f + k;
            const double *P = m->V + 3 * m->T[h], *Q = m->V + 3 * m->T[he_next(h)], *R = m->V + 3 * m->T[he_prev(h)];
            double e1[3], e2[3], c[3];
            sub3(Q, P, e1); sub3(R, P, e2);
            m->len[h] = norm3(e1);
            cross3(e1, e2, c);
            m->corner[h] = atan2(norm3(c), dot3(e1, e2));
            if (!(m->corner[h] > 1e-6)) rc = 5;
            m->theta[m->T[h]] += m->corner[h];
            if (m->twin[h] < 0 || h < m->twin[h]) { esum += m->len[h]; ecount++; }
            if (m->len[h] > m->max_edge) m->max_edge = m->len[h];
        }
        const double *P0 = m->V + 3 * m->T[3 * f], *P1 = m->V + 3 * m->T[3 * f + 1], *P2 = m->V + 3 * m->T[3 * f + 2];
        double a[3], b[3], n[3], y[3];
        sub3(P1, P0, a); sub3(P2, P0, b);
        cross3(a, b, n); unit3(n); unit3(a);
        cross3(n, a, y);
        memcpy(m->ex + 3 * f, a, sizeof a); memcpy(m->ey + 3 * f, y, sizeof y); memcpy(m->nrm + 3 * f, n, sizeof n);
    }
    m->mean_edge = esum / ecount;
    if (rc) { orc_mesh_free(m); return rc; }

    /* vertex fans */
    m->fan_off = (int *)calloc(nv + 1, sizeof(int));
    m->fan = (int *)malloc(sizeof(int) * ne);
    for (int h = 0; h < ne; h++) m->fan_off[m->T[h] + 1]++;
    for (int v = 0; v < nv; v++) m->fan_off[v + 1] += m->fan_off[v];
    int *cursor = (int *)malloc(sizeof(int) * nv);
    int *first = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; v++) { cursor[v] = m->fan_off[v]; first[v] = -1; }
    for (int h = 0; h < ne; h++) {
        int v = m->T[h];
        if (first[v] < 0 || m->twin[h] < 0) first[v] = h; /* boundary start wins */
    }
    for (int v = 0; v < nv && !rc; v++) {
        int deg = m->fan_off[v + 1] - m->fan_off[v];
        if (deg == 0) continue; /* isolated vertex: unused */
        int h = first[v], cnt = 0;
        if (m->twin[h] < 0) m->bnd[v] = 1;
        while (h >= 0 && cnt <= deg) {
            m->fan[cursor[v]++] = h;
            cnt++;
            int p = m->twin[he_prev(h)];
            if (p < 0) { m->bnd[v] = 1; break; }
            if (p == first[v]) break;
            h = p;
        }
        if (cnt != deg) rc = 4;
        m->pseudo[v] = m->bnd[v] || m->theta[v] >= TWO_PI - PSEUDO_TOL;
    }
    free(cursor); free(first);
    if (rc) { orc_mesh_free(m); return rc; }
    *out = m;
    return 0;
}

void orc_mesh_export(const orc_mesh *m, int *twin, double *theta, unsigned char *pseudo, unsigned char *boundary) {
    if (twin) memcpy(twin, m->twin, sizeof(int) * 3 * m->nf);
    if (theta) memcpy(theta, m->theta, sizeof(double) * m->nv);
    if (pseudo) memcpy(pseudo, m->pseudo, m->nv);
    if (boundary) memcpy(boundary, m->bnd, m->nv);
}

/* ======================================================================
 * 2. Geodesics by brute-force unfolding
 *
 * Every root (the source point, or a pseudo-source vertex at distance D) is
 * placed at the origin of a plane. Faces are unfolded one by one into that
 * plane across the edge crossed; a "window" is the slice [A, B] of the entry
 * edge that rays from the origin can reach without leaving the faces crossed
 * so far. Each window spawns at most two children (the two far edges),
 * clipped to the cone. No trimming, no dominance: every straight link from
 * the root shorter than the bound is enumerated. A Dijkstra over the roots
 * strings links into chains; the minimum over chains is the geodesic
 * distance (the MMP characterisation: shortest paths are straight in an
 * unfolding and bend only at saddle or boundary vertices).
 * ====================================================================== */
typedef struct { double d, t[2]; } tang_t;
/* best distance and the tie set: every direction within the band of it
 * (a growable array, so no direction is ever dropped) */
typedef struct { double best; int nt, cap; tang_t *e; } cand_t;

typedef struct {
    int h;             /* entry half-edge (X -> Y) of face h/3 */
    double X[2], Y[2]; /* unfolded tail / head, root at the origin, root right of X->Y */
    double A[2], B[2]; /* reachable slice of XY: A towards X, B towards Y */
    int depth;
} owin;

struct orc_pairs {
    int nsrc;
    int64_t *off;
    int32_t *nbr;
    double *dist, *tan;
    uint8_t *flags;
    int64_t *tie_off;
    double *tie_tan, *tie_dist;
    int64_t count, tcount;
    int64_t counters[5];
    int64_t wcounters[7]; /* window propagation (section 2b) */
};

typedef struct {
    /* per target particle */
    cand_t *tc;
    int *t_touched; int nt_touched; unsigned char *t_mark;
    /* per vertex (bend candidates) */
    cand_t *rc;
    int *r_touched; int nr_touched; unsigned char *r_mark, *r_done;
    /* Dijkstra heap over roots */
    double *hk; int *hv; int hn, hcap;
    owin *stk; int scap;
    int64_t cnt[5];
    double band;       /* tie band: directions within band * d of the best are kept */
    cand_t root;       /* copy of the tie set of the vertex being expanded */
} work_t;

static void cand_reset(cand_t *c) { c->best = INFINITY; c->nt = 0; }

/* Add candidate distance d with tangent t (2D, source-face frame); the set
 * keeps every direction whose distance is within rel * d of the best. */
static void cand_add(cand_t *c, double d, const double *t, double rel) {
    double tol = rel * (d < c->best ? d : c->best);
    if (d > c->best + tol) return;
    if (d < c->best) {
        c->best = d;
        int k = 0;
        for (int i = 0; i < c->nt; i++)
            if (c->e[i].d <= d + rel * d) c->e[k++] = c->e[i];
        c->nt = k;
    }
    for (int i = 0; i < c->nt; i++) {
        double cr = c->e[i].t[0] * t[1] - c->e[i].t[1] * t[0];
        double dt = c->e[i].t[0] * t[0] + c->e[i].t[1] * t[1];
        if (fabs(atan2(cr, dt)) < DIR_DUP) {
            /* one direction: it keeps the shorter path's length and tangent */
            if (d < c->e[i].d) { c->e[i].d = d; c->e[i].t[0] = t[0]; c->e[i].t[1] = t[1]; }
            return;
        }
    }
    if (c->nt == c->cap) {
        c->cap = c->cap ? 2 * c->cap : 4;
        c->e = (tang_t *)realloc(c->e, sizeof(tang_t) * c->cap);
    }
    c->e[c->nt].d = d; c->e[c->nt].t[0] = t[0]; c->e[c->nt].t[1] = t[1];
    c->nt++;
}

static void heap_push(work_t *w, double k, int v) {
    if (w->hn == w->hcap) {
        w->hcap = w->hcap ? 2 * w->hcap : 256;
        w->hk = (double *)realloc(w->hk, sizeof(double) * w->hcap);
        w->hv = (int *)realloc(w->hv, sizeof(int) * w->hcap);
    }
    int i = w->hn++;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (w->hk[p] <= k) break;
        w->hk[i] = w->hk[p]; w->hv[i] = w->hv[p]; i = p;
    }
    w->hk[i] = k; w->hv[i] = v;
}
static int heap_pop(work_t *w, double *k, int *v) {
    if (w->hn == 0) return 0;
    *k = w->hk[0]; *v = w->hv[0];
    double lk = w->hk[--w->hn]; int lv = w->hv[w->hn];
    int i = 0;
    for (;;) {
        int c = 2 * i + 1;
        if (c >= w->hn) break;
        if (c + 1 < w->hn && w->hk[c + 1] < w->hk[c]) c++;
        if (w->hk[c] >= lk) break;
        w->hk[i] = w->hk[c]; w->hv[i] = w->hv[c]; i = c;
    }
    if (w->hn > 0) { w->hk[i] = lk; w->hv[i] = lv; }
    return 1;
}

static void push_win(work_t *w, int *sn, const owin *x) {
    if (*sn == w->scap) {
        w->scap = w->scap ? 2 * w->scap : 1024;
        w->stk = (owin *)realloc(w->stk, sizeof(owin) * w->scap);
    }
    w->stk[(*sn)++] = *x;
}

static inline double cross2(const double *a, const double *b) { return a[0] * b[1] - a[1] * b[0]; }
static inline double len2(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1]); }

/* third vertex of the face left of X->Y, from the side lengths */
static void unfold_third(const double *X, const double *Y, double L, double lzx, double lyz, double *Z) {
    double e[2] = {(Y[0] - X[0]) / L, (Y[1] - X[1]) / L};
    double a = (L * L + lzx * lzx - lyz * lyz) / (2.0 * L);
    double b2 = lzx * lzx - a * a;
    double b = b2 > 0.0 ? sqrt(b2) : 0.0;
    Z[0] = X[0] + a * e[0] - b * e[1];
    Z[1] = X[1] + a * e[1] + b * e[0];
}

/* point where the ray from the origin along dir meets the line through P, Q */
static void ray_line(const double *dir, const double *P, const double *Q, double *out) {
    double d[2] = {Q[0] - P[0], Q[1] - P[1]};
    double lam = cross2(P, d) / cross2(dir, d);
    out[0] = lam * dir[0]; out[1] = lam * dir[1];
}

static double point_seg_dist0(const double *A, const double *B) {
    double d[2] = {B[0] - A[0], B[1] - A[1]};
    double dd = d[0] * d[0] + d[1] * d[1];
    double t = dd > 0.0 ? -(A[0] * d[0] + A[1] * d[1]) / dd : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double p[2] = {A[0] + t * d[0], A[1] + t * d[1]};
    return len2(p);
}

/* q inside the closed cone spanned CCW from direction r to direction l,
 * widened on both sides by the angle whose sine is eps */
static int in_cone(const double *r, const double *l, const double *q, double eps) {
    double nq = len2(q);
    return cross2(r, q) >= -eps * len2(r) * nq && cross2(q, l) >= -eps * len2(l) * nq;
}

typedef struct {
    const orc_mesh *m;
    const int *face; const double *bary;
    const int *fp_off, *fp;  /* particles per face */
    int src;
    double U;                /* prune bound */
    double cone;             /* angular slack (sine) of the target membership test */
} ctx_t;

/* record candidate for target j (via root with distance D, tangent set ts or,
 * for the source root, the direction of q itself) */
static void add_target(ctx_t *c, work_t *w, int j, double d, const double *q, const cand_t *root) {
    if (j == c->src || !(d < c->U)) return;
    if (!w->t_mark[j]) { w->t_mark[j] = 1; w->t_touched[w->nt_touched++] = j; cand_reset(&w->tc[j]); }
    if (!root) {
        double l = len2(q), t[2] = {0.0, 0.0};
        if (l > 0.0) { t[0] = q[0] / l; t[1] = q[1] / l; }
        cand_add(&w->tc[j], d, t, w->band);
    } else {
        for (int i = 0; i < root->nt; i++) cand_add(&w->tc[j], d, root->e[i].t, w->band);
    }
}

static void add_root(ctx_t *c, work_t *w, int v, double d, const double *q, const cand_t *root) {
    if (!c->m->pseudo[v] || !(d < c->U)) return;
    if (!w->r_mark[v]) { w->r_mark[v] = 1; w->r_touched[w->nr_touched++] = v; cand_reset(&w->rc[v]); w->r_done[v] = 0; }
    double before = w->rc[v].best;
    if (!root) {
        double l = len2(q), t[2] = {0.0, 0.0};
        if (l > 0.0) { t[0] = q[0] / l; t[1] = q[1] / l; }
        cand_add(&w->rc[v], d, t, w->band);
    } else {
        for (int i = 0; i < root->nt; i++) cand_add(&w->rc[v], d, root->e[i].t, w->band);
    }
    if (w->rc[v].best < before) {
        w->cnt[3]++;
        heap_push(w, w->rc[v].best, v);
    }
}

static void targets_in_face(ctx_t *c, work_t *w, int g, int slot_x, const double *X, const double *Y,
                            const double *Z, double D, const cand_t *root, const double *cr, const double *cl) {
    for (int a = c->fp_off[g]; a < c->fp_off[g + 1]; a++) {
        int j = c->fp[a];
        if (j == c->src) continue;
        const double *b = c->bary + 3 * j;
        double bx = b[slot_x], by = b[(slot_x + 1) % 3], bz = b[(slot_x + 2) % 3];
        double q[2] = {bx * X[0] + by * Y[0] + bz * Z[0], bx * X[1] + by * Y[1] + bz * Z[1]};
        if (cr && !in_cone(cr, cl, q, c->cone)) continue;
        add_target(c, w, j, D + len2(q), q, root);
    }
}

/* Process every window reachable from the windows already on the stack. */
static void drain(ctx_t *c, work_t *w, int *sn, double D, const cand_t *root) {
    const orc_mesh *m = c->m;
    while (*sn > 0) {
        owin x = w->stk[--(*sn)];
        w->cnt[0]++;
        if (x.depth > MAX_DEPTH) continue;
        if (D + point_seg_dist0(x.A, x.B) >= c->U) { w->cnt[1]++; continue; }
        int h = x.h, g = h / 3, k = h % 3;
        double Z[2];
        unfold_third(x.X, x.Y, m->len[h], m->len[he_prev(h)], m->len[he_next(h)], Z);
        /* cone: CCW from r = B (head side) to l = A (tail side) */
        const double *r = x.B, *l = x.A;
        targets_in_face(c, w, g, k, x.X, x.Y, Z, D, root, r, l);
        int vz = m->T[he_prev(h)];
        if (in_cone(r, l, Z, CONE_EPS)) add_root(c, w, vz, D + len2(Z), Z, root);
        /* child across Y->Z: entry tail Z, head Y */
        int t1 = m->twin[he_next(h)];
        if (t1 >= 0) {
            const double *rc = cross2(r, x.Y) > 0.0 ? x.Y : r; /* more counter-clockwise */
            const double *lc = cross2(l, Z) > 0.0 ? l : Z;     /* more clockwise */
            if (cross2(rc, lc) >= 0.0) {
                owin y; y.h = t1; y.depth = x.depth + 1;
                y.X[0] = Z[0]; y.X[1] = Z[1]; y.Y[0] = x.Y[0]; y.Y[1] = x.Y[1];
                if (rc == x.Y) { y.B[0] = x.Y[0]; y.B[1] = x.Y[1]; } else ray_line(rc, Z, x.Y, y.B);
                if (lc == Z) { y.A[0] = Z[0]; y.A[1] = Z[1]; } else ray_line(lc, Z, x.Y, y.A);
                double sl[2] = {y.B[0] - y.A[0], y.B[1] - y.A[1]};
                if (len2(sl) > SEG_MIN_REL * m->len[t1]) push_win(w, sn, &y);
            }
        }
        /* child across Z->X: entry tail X, head Z */
        int t2 = m->twin[he_prev(h)];
        if (t2 >= 0) {
            const double *rc = cross2(r, Z) > 0.0 ? Z : r;
            const double *lc = cross2(l, x.X) > 0.0 ? l : x.X;
            if (cross2(rc, lc) >= 0.0) {
                owin y; y.h = t2; y.depth = x.depth + 1;
                y.X[0] = x.X[0]; y.X[1] = x.X[1]; y.Y[0] = Z[0]; y.Y[1] = Z[1];
                if (rc == Z) { y.B[0] = Z[0]; y.B[1] = Z[1]; } else ray_line(rc, x.X, Z, y.B);
                if (lc == x.X) { y.A[0] = x.X[0]; y.A[1] = x.X[1]; } else ray_line(lc, x.X, Z, y.A);
                double sl[2] = {y.B[0] - y.A[0], y.B[1] - y.A[1]};
                if (len2(sl) > SEG_MIN_REL * m->len[t2]) push_win(w, sn, &y);
            }
        }
    }
}

static void seed_edge(work_t *w, int *sn, int twin_h, const double *X, const double *Y) {
    if (twin_h < 0) return;
    owin y; y.h = twin_h; y.depth = 0;
    y.X[0] = X[0]; y.X[1] = X[1]; y.Y[0] = Y[0]; y.Y[1] = Y[1];
    y.A[0] = X[0]; y.A[1] = X[1]; y.B[0] = Y[0]; y.B[1] = Y[1];
    push_win(w, sn, &y);
}

/* Root = the source particle, in its face's frame (ex, ey), at the origin. */
static int expand_source(ctx_t *c, work_t *w) {
    const orc_mesh *m = c->m;
    int f = c->face[c->src];
    const double *b = c->bary + 3 * c->src;
    int nzero = (b[0] <= 0.0) + (b[1] <= 0.0) + (b[2] <= 0.0);
    if (nzero >= 2) return -1; /* on a vertex: tangent plane undefined */
    double P[3][2];
    P[0][0] = 0.0; P[0][1] = 0.0;
    P[1][0] = m->len[3 * f]; P[1][1] = 0.0;
    unfold_third(P[0], P[1], m->len[3 * f], m->len[3 * f + 2], m->len[3 * f + 1], P[2]);
    double s[2] = {b[0] * P[0][0] + b[1] * P[1][0] + b[2] * P[2][0], b[0] * P[0][1] + b[1] * P[1][1] + b[2] * P[2][1]};
    for (int k = 0; k < 3; k++) { P[k][0] -= s[0]; P[k][1] -= s[1]; }
    targets_in_face(c, w, f, 0, P[0], P[1], P[2], 0.0, NULL, NULL, NULL);
    for (int k = 0; k < 3; k++) add_root(c, w, m->T[3 * f + k], len2(P[k]), P[k], NULL);
    int sn = 0;
    for (int k = 0; k < 3; k++) {
        int h = 3 * f + k, t = m->twin[h];
        const double *X = P[k], *Y = P[(k + 1) % 3];
        if (b[(k + 2) % 3] > 0.0) {
            seed_edge(w, &sn, t, Y, X); /* twin runs Y -> X */
        } else if (t >= 0) {
            /* source on this edge: the face across it contains the source too */
            int g = t / 3, mm = t % 3;
            double Z[2];
            unfold_third(Y, X, m->len[t], m->len[he_prev(t)], m->len[he_next(t)], Z);
            targets_in_face(c, w, g, mm, Y, X, Z, 0.0, NULL, NULL, NULL);
            add_root(c, w, m->T[he_prev(t)], len2(Z), Z, NULL);
            seed_edge(w, &sn, m->twin[he_next(t)], Z, X);  /* next(t) runs X -> Z */
            seed_edge(w, &sn, m->twin[he_prev(t)], Y, Z);  /* prev(t) runs Z -> Y */
        }
    }
    drain(c, w, &sn, 0.0, NULL);
    return 0;
}

/* Root = pseudo-source vertex v at distance D with tangent set root. */
static void expand_vertex(ctx_t *c, work_t *w, int v, double D, const cand_t *root) {
    const orc_mesh *m = c->m;
    int sn = 0;
    for (int a = m->fan_off[v]; a < m->fan_off[v + 1]; a++) {
        int h = m->fan[a], g = h / 3, k = h % 3;
        double O[2] = {0.0, 0.0}, U1[2] = {m->len[h], 0.0}, U2[2];
        unfold_third(O, U1, m->len[h], m->len[he_prev(h)], m->len[he_next(h)], U2);
        targets_in_face(c, w, g, k, O, U1, U2, D, root, NULL, NULL);
        add_root(c, w, m->T[he_next(h)], D + len2(U1), U1, root);
        add_root(c, w, m->T[he_prev(h)], D + len2(U2), U2, root);
        seed_edge(w, &sn, m->twin[he_next(h)], U2, U1); /* twin of (u1 -> u2) */
    }
    drain(c, w, &sn, D, root);
}

/* all-pairs bound: graph distance over edges + one max edge */
static double graph_bound(const orc_mesh *m, int f, const double *b, double *dist, work_t *w) {
    for (int v = 0; v < m->nv; v++) dist[v] = INFINITY;
    w->hn = 0;
    for (int k = 0; k < 3; k++) {
        int v = m->T[3 * f + k];
        const double *P = m->V + 3 * v;
        double x[3] = {0, 0, 0};
        for (int q = 0; q < 3; q++)
            for (int d = 0; d < 3; d++) x[d] += b[q] * m->V[3 * m->T[3 * f + q] + d];
        double e[3]; sub3(P, x, e);
        dist[v] = norm3(e);
        heap_push(w, dist[v], v);
    }
    double kk; int v;
    while (heap_pop(w, &kk, &v)) {
        if (kk > dist[v]) continue;
        for (int a = m->fan_off[v]; a < m->fan_off[v + 1]; a++) {
            int h = m->fan[a];
            int u1 = m->T[he_next(h)], u2 = m->T[he_prev(h)];
            if (dist[v] + m->len[h] < dist[u1]) { dist[u1] = dist[v] + m->len[h]; heap_push(w, dist[u1], u1); }
            if (dist[v] + m->len[he_prev(h)] < dist[u2]) { dist[u2] = dist[v] + m->len[he_prev(h)]; heap_push(w, dist[u2], u2); }
        }
    }
    double mx = 0.0;
    for (int u = 0; u < m->nv; u++)
        if (isfinite(dist[u]) && dist[u] > mx) mx = dist[u];
    return mx + 2.0 * m->max_edge;
}

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

typedef struct { int n; int32_t *nbr; double *dist, *tan; uint8_t *flags; int *nt; double *tt, *td; } row_t;

orc_pairs *orc_geodesic_pairs(const orc_mesh *m, int n, const int *face, const double *bary, double cutoff,
                              int nsrc, const int *src, int nthreads, double tie_rel, double cone_slack) {
    if (!m || n < 0 || (n > 0 && (!face || !bary))) return NULL;
    if (!(tie_rel > 0.0)) tie_rel = TIE_REL;
    if (!(cone_slack > CONE_EPS)) cone_slack = CONE_EPS;
    for (int j = 0; j < n; j++)
        if (face[j] < 0 || face[j] >= m->nf) return NULL;
    int all = !(cutoff > 0.0) || !isfinite(cutoff);
    if (!src) nsrc = n;
    int *fp_off = (int *)calloc(m->nf + 1, sizeof(int));
    int *fp = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int j = 0; j < n; j++) fp_off[face[j] + 1]++;
    for (int f = 0; f < m->nf; f++) fp_off[f + 1] += fp_off[f];
    {
        int *cur = (int *)malloc(sizeof(int) * (m->nf + 1));
        memcpy(cur, fp_off, sizeof(int) * (m->nf + 1));
        for (int j = 0; j < n; j++) fp[cur[face[j]]++] = j;
        free(cur);
    }
    row_t *rows = (row_t *)calloc(nsrc > 0 ? nsrc : 1, sizeof(row_t));
    orc_pairs *res = (orc_pairs *)calloc(1, sizeof(orc_pairs));
    res->nsrc = nsrc;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        work_t w;
        memset(&w, 0, sizeof w);
        w.band = tie_rel;
        w.tc = (cand_t *)calloc(n > 0 ? n : 1, sizeof(cand_t));
        w.t_touched = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
        w.t_mark = (unsigned char *)calloc(n > 0 ? n : 1, 1);
        w.rc = (cand_t *)calloc(m->nv, sizeof(cand_t));
        w.r_touched = (int *)malloc(sizeof(int) * m->nv);
        w.r_mark = (unsigned char *)calloc(m->nv, 1);
        w.r_done = (unsigned char *)calloc(m->nv, 1);
        double *gdist = all ? (double *)malloc(sizeof(double) * m->nv) : NULL;
#pragma omp for schedule(dynamic, 1)
        for (int si = 0; si < nsrc; si++) {
            int i = src ? src[si] : si;
            ctx_t c;
            c.m = m; c.face = face; c.bary = bary; c.fp_off = fp_off; c.fp = fp; c.src = i;
            c.U = all ? graph_bound(m, face[i], bary + 3 * i, gdist, &w) : cutoff;
            c.cone = cone_slack;
            w.hn = 0; w.nt_touched = 0; w.nr_touched = 0;
            if (expand_source(&c, &w) != 0) {
                w.cnt[4]++;
            } else {
                double k; int v;
                while (heap_pop(&w, &k, &v)) {
                    if (k > w.rc[v].best || w.r_done[v]) continue;
                    if (!(k < c.U)) break;
                    w.r_done[v] = 1;
                    w.cnt[2]++;
                    /* the vertex's own set may grow while it is expanded: expand a copy */
                    const cand_t *rv = &w.rc[v];
                    if (w.root.cap < rv->nt) {
                        w.root.cap = rv->nt;
                        w.root.e = (tang_t *)realloc(w.root.e, sizeof(tang_t) * w.root.cap);
                    }
                    w.root.best = rv->best;
                    w.root.nt = rv->nt;
                    memcpy(w.root.e, rv->e, sizeof(tang_t) * rv->nt);
                    expand_vertex(&c, &w, v, w.root.best, &w.root);
                }
            }
            /* collect */
            qsort(w.t_touched, w.nt_touched, sizeof(int), cmp_int);
            row_t *rw = &rows[si];
            int cnt = 0, tcnt = 0;
            for (int a = 0; a < w.nt_touched; a++) {
                int j = w.t_touched[a];
                if (all || w.tc[j].best < cutoff) { cnt++; tcnt += w.tc[j].nt; }
            }
            rw->n = cnt;
            rw->nbr = (int32_t *)malloc(sizeof(int32_t) * (cnt + 1));
            rw->dist = (double *)malloc(sizeof(double) * (cnt + 1));
            rw->tan = (double *)malloc(sizeof(double) * 3 * (cnt + 1));
            rw->flags = (uint8_t *)malloc(cnt + 1);
            rw->nt = (int *)malloc(sizeof(int) * (cnt + 1));
            rw->tt = (double *)malloc(sizeof(double) * 3 * (tcnt + 1));
            rw->td = (double *)malloc(sizeof(double) * (tcnt + 1));
            const double *ex = m->ex + 3 * face[i], *ey = m->ey + 3 * face[i];
            int q = 0, tq = 0;
            for (int a = 0; a < w.nt_touched; a++) {
                int j = w.t_touched[a];
                cand_t *cj = &w.tc[j];
                if (!(all || cj->best < cutoff)) continue;
                rw->nbr[q] = j; rw->dist[q] = cj->best;
                /* representative tangent: the entry with the smallest distance */
                int bi = 0;
                for (int e = 1; e < cj->nt; e++)
                    if (cj->e[e].d < cj->e[bi].d) bi = e;
                for (int d = 0; d < 3; d++) rw->tan[3 * q + d] = cj->e[bi].t[0] * ex[d] + cj->e[bi].t[1] * ey[d];
                uint8_t fl = 0;
                if (cj->nt > 1) fl |= 1;
                if (cj->best == 0.0) fl |= 2;
                rw->flags[q] = fl;
                rw->nt[q] = cj->nt;
                for (int e = 0; e < cj->nt; e++, tq++) {
                    for (int d = 0; d < 3; d++) rw->tt[3 * tq + d] = cj->e[e].t[0] * ex[d] + cj->e[e].t[1] * ey[d];
                    rw->td[tq] = cj->e[e].d;
                }
                q++;
            }
            for (int a = 0; a < w.nt_touched; a++) w.t_mark[w.t_touched[a]] = 0;
            for (int a = 0; a < w.nr_touched; a++) { w.r_mark[w.r_touched[a]] = 0; w.r_done[w.r_touched[a]] = 0; }
        }
#pragma omp critical
        {
            for (int z = 0; z < 5; z++) res->counters[z] += w.cnt[z];
        }
        for (int j = 0; j < n; j++) free(w.tc[j].e);
        for (int v = 0; v < m->nv; v++) free(w.rc[v].e);
        free(w.root.e);
        free(w.tc); free(w.t_touched); free(w.t_mark); free(w.rc); free(w.r_touched); free(w.r_mark);
        free(w.r_done); free(w.hk); free(w.hv); free(w.stk); free(gdist);
    }
    /* flatten */
    res->off = (int64_t *)malloc(sizeof(int64_t) * (nsrc + 1));
    res->off[0] = 0;
    int64_t tot = 0, ttot = 0;
    for (int s = 0; s < nsrc; s++) {
        tot += rows[s].n;
        res->off[s + 1] = tot;
        for (int q = 0; q < rows[s].n; q++) ttot += rows[s].nt[q];
    }
    res->count = tot; res->tcount = ttot;
    res->nbr = (int32_t *)malloc(sizeof(int32_t) * (tot + 1));
    res->dist = (double *)malloc(sizeof(double) * (tot + 1));
    res->tan = (double *)malloc(sizeof(double) * 3 * (tot + 1));
    res->flags = (uint8_t *)malloc(tot + 1);
    res->tie_off = (int64_t *)malloc(sizeof(int64_t) * (tot + 1));
    res->tie_tan = (double *)malloc(sizeof(double) * 3 * (ttot + 1));
    res->tie_dist = (double *)malloc(sizeof(double) * (ttot + 1));
    int64_t p = 0, tp = 0;
    res->tie_off[0] = 0;
    for (int s = 0; s < nsrc; s++) {
        row_t *rw = &rows[s];
        int tq = 0;
        for (int q = 0; q < rw->n; q++, p++) {
            res->nbr[p] = rw->nbr[q]; res->dist[p] = rw->dist[q];
            memcpy(res->tan + 3 * p, rw->tan + 3 * q, sizeof(double) * 3);
            res->flags[p] = rw->flags[q];
            for (int e = 0; e < rw->nt[q]; e++, tq++, tp++) {
                memcpy(res->tie_tan + 3 * tp, rw->tt + 3 * tq, sizeof(double) * 3);
                res->tie_dist[tp] = rw->td[tq];
            }
            res->tie_off[p + 1] = tp;
        }
        free(rw->nbr); free(rw->dist); free(rw->tan); free(rw->flags); free(rw->nt); free(rw->tt); free(rw->td);
    }
    free(rows); free(fp_off); free(fp);
    return res;
}

int64_t orc_pairs_count(const orc_pairs *p) { return p->count; }
int64_t orc_pairs_tie_count(const orc_pairs *p) { return p->tcount; }
void orc_pairs_export(const orc_pairs *p, int64_t *off, int32_t *nbr, double *dist, double *tan, uint8_t *flags,
                      int64_t *tie_off, double *tie_tan, double *tie_dist) {
    if (off) memcpy(off, p->off, sizeof(int64_t) * (p->nsrc + 1));
    if (nbr) memcpy(nbr, p->nbr, sizeof(int32_t) * p->count);
    if (dist) memcpy(dist, p->dist, sizeof(double) * p->count);
    if (tan) memcpy(tan, p->tan, sizeof(double) * 3 * p->count);
    if (flags) memcpy(flags, p->flags, p->count);
    if (tie_off) memcpy(tie_off, p->tie_off, sizeof(int64_t) * (p->count + 1));
    if (tie_tan) memcpy(tie_tan, p->tie_tan, sizeof(double) * 3 * p->tcount);
    if (tie_dist) memcpy(tie_dist, p->tie_dist, sizeof(double) * p->tcount);
}
void orc_pairs_counters(const orc_pairs *p, int64_t *c5) { memcpy(c5, p->counters, sizeof(int64_t) * 5); }
void orc_pairs_free(orc_pairs *p) {
    if (!p) return;
    free(p->off); free(p->nbr); free(p->dist); free(p->tan); free(p->flags); free(p->tie_off); free(p->tie_tan);
    free(p->tie_dist);
    free(p);
}

/* ======================================================================
 * 2b. Geodesics by window propagation with trimming (the exact method of
 *     Sec. 2.2: Mitchell, Mount & Papadimitriou's continuous Dijkstra, in
 *     the interval form of Surazhsky et al.)
 *
 * A second, independent route to the exact distances of section 2, and the
 * method's own measure of work. A window lives on a half-edge h and stands
 * for the straight rays that enter face(h) across the slice [b0, b1] of h
 * from one image p of their root: the source, or a pseudo-source vertex at
 * distance sg. Coordinates are h's edge frame: origin at h's tail A, x
 * along A->B, y into face(h); the image lies on the other side (py < 0).
 * Windows are processed in the order of their distance to their slice.
 * Processing unfolds face(h)'s third vertex C, lowers the distances D(v) of
 * the vertices the closed cone reaches, and continues the rays into at most
 * two child windows on the far edges (Sec. 2.2: propagation across a face).
 * A child is inserted on the twin of its edge after trimming against the
 * windows already there: on the overlap of two slices each keeps the part
 * where its distance is the smaller (the pointwise minimum), so a window
 * may shrink, split or vanish. Every window is a family of real paths, so
 * trimming never makes a distance too short, and it never cuts a shortest
 * path: past a point reached by two shortest paths no path is shortest.
 * A pseudo-source vertex is launched once, at its final distance: windows
 * from it on the edge opposite it in each face around it, and its
 * neighbours relaxed along the edges. A target's distance is the minimum
 * over the source term (same face), the pseudo-source vertices of its face
 * (D(v) + |v - x|) and the windows on its face's half-edges whose cone
 * holds it.
 * ====================================================================== */
#define WMAXP 256 /* pieces one insertion may hold; beyond it a comparison is skipped (no trim: safe) */

typedef struct {
    int h, root, alive, done, gen, next;
    double b0, b1;     /* slice of h, measured from h's tail */
    double px, py, sg; /* image of the root in h's frame (py < 0), distance of the root */
    double c, s;       /* source-frame direction of the frame's x axis (source-rooted windows) */
} wwin;

typedef struct {
    const orc_mesh *m;
    double U;                                /* prune bound */
    wwin *w; int nw, cap;
    int *hhead; int *htouch; int nht;        /* windows on each half-edge (linked), half-edges used */
    double *hk; int *hid, *hgen; int hn, hcap; /* heap: key, window id or -1 - vertex, generation */
    double *D, *Dt;                          /* vertex distance and its tangent (source frame) */
    unsigned char *launched;
    int *vtouch; int nvt;
    unsigned char *fmark; int *ftouch; int nft;
    int64_t cnt[7];
} wctx;

static void wheap_push(wctx *c, double k, int id, int gen) {
    if (c->hn == c->hcap) {
        c->hcap = c->hcap ? 2 * c->hcap : 1024;
        c->hk = (double *)realloc(c->hk, sizeof(double) * c->hcap);
        c->hid = (int *)realloc(c->hid, sizeof(int) * c->hcap);
        c->hgen = (int *)realloc(c->hgen, sizeof(int) * c->hcap);
    }
    int i = c->hn++;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (c->hk[p] <= k) break;
        c->hk[i] = c->hk[p]; c->hid[i] = c->hid[p]; c->hgen[i] = c->hgen[p];
        i = p;
    }
    c->hk[i] = k; c->hid[i] = id; c->hgen[i] = gen;
}

static int wheap_pop(wctx *c, double *k, int *id, int *gen) {
    if (c->hn == 0) return 0;
    *k = c->hk[0]; *id = c->hid[0]; *gen = c->hgen[0];
    c->hn--;
    double lk = c->hk[c->hn]; int lid = c->hid[c->hn], lg = c->hgen[c->hn];
    int i = 0;
    for (;;) {
        int ch = 2 * i + 1;
        if (ch >= c->hn) break;
        if (ch + 1 < c->hn && c->hk[ch + 1] < c->hk[ch]) ch++;
        if (c->hk[ch] >= lk) break;
        c->hk[i] = c->hk[ch]; c->hid[i] = c->hid[ch]; c->hgen[i] = c->hgen[ch];
        i = ch;
    }
    if (c->hn > 0) { c->hk[i] = lk; c->hid[i] = lid; c->hgen[i] = lg; }
    return 1;
}

/* length of the path through the point (x, 0) of the window's edge */
static inline double wdist(const wwin *w, double x) { return w->sg + hypot(x - w->px, w->py); }

/* the window's key: its distance to the nearest point of its slice */
static double wkey(const wwin *w) {
    double x = w->px < w->b0 ? w->b0 : (w->px > w->b1 ? w->b1 : w->px);
    return wdist(w, x);
}

/* store a window, link it on its half-edge and queue it unless processed */
static void wlink(wctx *c, const wwin *x) {
    if (c->nw == c->cap) {
        c->cap = c->cap ? 2 * c->cap : 4096;
        c->w = (wwin *)realloc(c->w, sizeof(wwin) * c->cap);
    }
    int id = c->nw++;
    c->w[id] = *x;
    if (c->hhead[x->h] < 0) c->htouch[c->nht++] = x->h;
    c->w[id].next = c->hhead[x->h];
    c->hhead[x->h] = id;
    if (!x->done) wheap_push(c, wkey(x), id, x->gen);
}

/* the points of (lo, hi) where two windows' distances can be equal. With
 * equal root distances that is where the images' bisector meets the edge;
 * otherwise the real roots of the quadratic left after squaring the
 * equation twice. A cut that is no crossing (a root of the other sign
 * branch, or the vertex of the quadratic taken when rounding makes a double
 * root's discriminant negative) only splits a piece: each piece between
 * cuts goes to the window shorter at its midpoint. */
static int wcross(const wwin *a, const wwin *b, double lo, double hi, double *x) {
    double dl = b->sg - a->sg;
    double al = 2.0 * (b->px - a->px);
    double be = a->px * a->px + a->py * a->py - b->px * b->px - b->py * b->py - dl * dl;
    double r[2]; int nr = 0;
    if (dl == 0.0) {
        if (al != 0.0) r[nr++] = -be / al;
    } else {
        double A2 = al * al - 4.0 * dl * dl;
        double B2 = 2.0 * al * be + 8.0 * dl * dl * b->px;
        double C2 = be * be - 4.0 * dl * dl * (b->px * b->px + b->py * b->py);
        double scale = fabs(A2) * (hi * hi + 1.0) + fabs(B2) * (fabs(hi) + 1.0) + fabs(C2);
        if (!(scale > 0.0)) return 0;
        if (fabs(A2) * (hi * hi + 1.0) <= 1e-13 * scale) {
            if (B2 != 0.0) r[nr++] = -C2 / B2;
        } else {
            double disc = B2 * B2 - 4.0 * A2 * C2;
            double sq = disc > 0.0 ? sqrt(disc) : 0.0;
            double q = -0.5 * (B2 + (B2 >= 0.0 ? sq : -sq));
            if (q != 0.0) {
                r[nr++] = q / A2;
                r[nr++] = C2 / q;
            } else {
                r[nr++] = 0.0;
            }
        }
    }
    int k = 0;
    for (int i = 0; i < nr; i++)
        if (r[i] > lo && r[i] < hi) x[k++] = r[i];
    if (k == 2 && x[0] > x[1]) { double t = x[0]; x[0] = x[1]; x[1] = t; }
    return k;
}

/* window o loses the ordered runs [r0, r1]: what is left stays as o (the
 * first piece) and new windows (the others); an unprocessed window is
 * queued again under its new key */
static void wtrim(wctx *c, int o, const double *r0, const double *r1, int nr) {
    wwin ow = c->w[o];
    const double eps = SEG_MIN_REL * c->m->len[ow.h];
    double k0[WMAXP + 2], k1[WMAXP + 2]; int nk = 0;
    double cur = ow.b0;
    for (int i = 0; i < nr; i++) {
        if (r0[i] - cur > eps) { k0[nk] = cur; k1[nk++] = r0[i]; }
        if (r1[i] > cur) cur = r1[i];
    }
    if (ow.b1 - cur > eps) { k0[nk] = cur; k1[nk++] = ow.b1; }
    c->cnt[2]++;
    if (nk == 0) { c->w[o].alive = 0; return; }
    c->w[o].b0 = k0[0]; c->w[o].b1 = k1[0];
    if (!ow.done) { c->w[o].gen++; wheap_push(c, wkey(&c->w[o]), o, c->w[o].gen); }
    for (int i = 1; i < nk; i++) {
        wwin y = ow;
        y.b0 = k0[i]; y.b1 = k1[i]; y.gen = 0;
        wlink(c, &y);
    }
}

/* insert window x on its half-edge as the pointwise minimum with the
 * windows already there */
static void winsert(wctx *c, const wwin *x) {
    const int h = x->h;
    const double eps = SEG_MIN_REL * c->m->len[h];
    double p0[WMAXP], p1[WMAXP]; int np = 1;
    p0[0] = x->b0; p1[0] = x->b1;
    for (int o = c->hhead[h]; o >= 0 && np > 0; o = c->w[o].next) {
        if (!c->w[o].alive || 5 * np > WMAXP) continue;
        const wwin ow = c->w[o];
        double q0[WMAXP], q1[WMAXP]; int nq = 0;  /* what the new window keeps */
        double r0[WMAXP], r1[WMAXP]; int nr = 0;  /* what the old window loses */
        for (int q = 0; q < np; q++) {
            double lo = p0[q] > ow.b0 ? p0[q] : ow.b0, hi = p1[q] < ow.b1 ? p1[q] : ow.b1;
            if (hi - lo <= eps) { q0[nq] = p0[q]; q1[nq++] = p1[q]; continue; }
            double cut[4]; int nc = 0;
            cut[nc++] = lo;
            nc += wcross(x, &ow, lo, hi, cut + nc);
            cut[nc++] = hi;
            if (lo > p0[q]) { q0[nq] = p0[q]; q1[nq++] = lo; }
            for (int i = 0; i + 1 < nc; i++) {
                double a = cut[i], b = cut[i + 1], mid = 0.5 * (a + b);
                if (wdist(x, mid) < wdist(&ow, mid)) {
                    if (nq > 0 && q1[nq - 1] >= a) q1[nq - 1] = b;
                    else { q0[nq] = a; q1[nq++] = b; }
                    if (nr > 0 && r1[nr - 1] >= a) r1[nr - 1] = b;
                    else { r0[nr] = a; r1[nr++] = b; }
                }
            }
            if (hi < p1[q]) {
                if (nq > 0 && q1[nq - 1] >= hi) q1[nq - 1] = p1[q];
                else { q0[nq] = hi; q1[nq++] = p1[q]; }
            }
        }
        if (nr > 0) wtrim(c, o, r0, r1, nr);
        np = 0;
        for (int q = 0; q < nq; q++)
            if (q1[q] - q0[q] > eps) { p0[np] = q0[q]; p1[np++] = q1[q]; }
    }
    if (np == 0) { c->cnt[5]++; return; }
    for (int q = 0; q < np; q++) {
        wwin y = *x;
        y.b0 = p0[q]; y.b1 = p1[q]; y.alive = 1; y.done = 0; y.gen = 0;
        if (!(wkey(&y) < c->U)) { c->cnt[5]++; continue; }
        c->cnt[0]++;
        wlink(c, &y);
    }
}

/* the third vertex C of face(h) in h's frame, from the edge lengths */
static void third_in_frame(const orc_mesh *m, int h, double *cx, double *cy) {
    double L = m->len[h], lp = m->len[he_prev(h)], ln = m->len[he_next(h)];
    *cx = (L * L + lp * lp - ln * ln) / (2.0 * L);
    double y2 = lp * lp - *cx * *cx;
    *cy = y2 > 0.0 ? sqrt(y2) : 0.0;
}

/* the source-frame unit direction of a window's ray (dx, dy) in its frame,
 * or the tangent of its root vertex */
static void wtangent(const wctx *c, const wwin *w, double dx, double dy, double *t) {
    if (w->root >= 0) { t[0] = c->Dt[2 * w->root]; t[1] = c->Dt[2 * w->root + 1]; return; }
    double l = hypot(dx, dy);
    t[0] = t[1] = 0.0;
    if (!(l > 0.0)) return;
    dx /= l; dy /= l;
    t[0] = w->c * dx - w->s * dy;
    t[1] = w->s * dx + w->c * dy;
}

static void wvertex(wctx *c, int v, double d, const double *t) {
    if (!(d < c->U) || !(d < c->D[v])) return;
    if (!isfinite(c->D[v])) c->vtouch[c->nvt++] = v;
    c->D[v] = d;
    c->Dt[2 * v] = t[0]; c->Dt[2 * v + 1] = t[1];
    if (c->m->pseudo[v] && !c->launched[v]) wheap_push(c, d, -1 - v, 0);
}

/* a child window on half-edge th from the rays of w through the part of its
 * slice that reaches th's edge; (ox, oy) = th's tail and (ux, uy) = its unit
 * direction, in w's frame; s0, s1 = the slice on th */
static void wchild(wctx *c, const wwin *w, int th, double ox, double oy, double ux, double uy, double s0, double s1) {
    const double Lt = c->m->len[th];
    if (s0 < 0.0) s0 = 0.0;
    if (s1 > Lt) s1 = Lt;
    if (!(s1 - s0 > SEG_MIN_REL * Lt)) return;
    double qx = w->px - ox, qy = w->py - oy;
    wwin y = *w;
    y.h = th; y.b0 = s0; y.b1 = s1;
    y.px = ux * qx + uy * qy;
    y.py = ux * qy - uy * qx;
    if (!(y.py < 0.0)) return; /* rays grazing the edge's line enter no face */
    y.c = w->c * ux - w->s * uy;
    y.s = w->s * ux + w->c * uy;
    y.alive = 1; y.done = 0; y.gen = 0;
    winsert(c, &y);
}

/* parameter along the line O + s u where the ray from w's image through
 * (x, 0) meets it */
static double wray_hit(const wwin *w, double x, double ox, double oy, double ux, double uy) {
    double dx = x - w->px, dy = -w->py;
    double rx = w->px - ox, ry = w->py - oy;
    return (rx * dy - ry * dx) / (ux * dy - uy * dx);
}

static void wprocess(wctx *c, int id) {
    const orc_mesh *m = c->m;
    wwin w = c->w[id];
    c->w[id].done = 1;
    c->cnt[1]++;
    int h = w.h, f = h / 3;
    if (!c->fmark[f]) { c->fmark[f] = 1; c->ftouch[c->nft++] = f; c->cnt[4]++; }
    double L = m->len[h], cx, cy, t[2];
    third_in_frame(m, h, &cx, &cy);
    const double tol = CONE_EPS * L;
    /* where the ray from the image through C crosses the edge */
    double txc = w.px + (cx - w.px) * (-w.py) / (cy - w.py);
    if (txc >= w.b0 - tol && txc <= w.b1 + tol) {
        wtangent(c, &w, cx - w.px, cy - w.py, t);
        wvertex(c, m->T[he_prev(h)], w.sg + hypot(cx - w.px, cy - w.py), t);
    }
    if (w.b0 <= tol) {
        wtangent(c, &w, -w.px, -w.py, t);
        wvertex(c, m->T[h], w.sg + hypot(w.px, w.py), t);
    }
    if (w.b1 >= L - tol) {
        wtangent(c, &w, L - w.px, -w.py, t);
        wvertex(c, m->T[he_next(h)], w.sg + hypot(L - w.px, w.py), t);
    }
    /* rays through [b0, min(b1, txc)] cross A->C: child on twin(prev(h)),
     * whose frame has origin A and x towards C */
    int tp = m->twin[he_prev(h)];
    if (tp >= 0 && w.b0 < txc) {
        double lp = m->len[he_prev(h)], ux = cx / lp, uy = cy / lp;
        double s0 = wray_hit(&w, w.b0, 0.0, 0.0, ux, uy);
        double s1 = w.b1 >= txc ? lp : wray_hit(&w, w.b1, 0.0, 0.0, ux, uy);
        wchild(c, &w, tp, 0.0, 0.0, ux, uy, s0, s1);
    }
    /* rays through [max(b0, txc), b1] cross C->B: child on twin(next(h)),
     * whose frame has origin C and x towards B */
    int tn = m->twin[he_next(h)];
    if (tn >= 0 && w.b1 > txc) {
        double ln = m->len[he_next(h)], ux = (L - cx) / ln, uy = -cy / ln;
        double s0 = w.b0 <= txc ? 0.0 : wray_hit(&w, w.b0, cx, cy, ux, uy);
        double s1 = wray_hit(&w, w.b1, cx, cy, ux, uy);
        wchild(c, &w, tn, cx, cy, ux, uy, s0, s1);
    }
}

/* pseudo-source vertex v at its final distance: a window from v on the
 * edge opposite it in every face around it, neighbours relaxed */
static void wlaunch(wctx *c, int v) {
    const orc_mesh *m = c->m;
    c->launched[v] = 1;
    c->cnt[3]++;
    const double Dv = c->D[v], tv[2] = {c->Dt[2 * v], c->Dt[2 * v + 1]};
    for (int a = m->fan_off[v]; a < m->fan_off[v + 1]; a++) {
        int hv = m->fan[a], hn = he_next(hv), hp = he_prev(hv); /* v -> u1, u1 -> u2, u2 -> v */
        wvertex(c, m->T[hn], Dv + m->len[hv], tv);
        wvertex(c, m->T[hp], Dv + m->len[hp], tv);
        int t = m->twin[hn];
        if (t < 0) continue;
        /* t runs u2 -> u1; v lies at distance len[hp] from u2 and len[hv] from u1 */
        double L = m->len[t], a2 = m->len[hp], a1 = m->len[hv];
        double px = (L * L + a2 * a2 - a1 * a1) / (2.0 * L), y2 = a2 * a2 - px * px;
        wwin y;
        memset(&y, 0, sizeof y);
        y.h = t; y.root = v; y.alive = 1;
        y.b0 = 0.0; y.b1 = L;
        y.px = px; y.py = -(y2 > 0.0 ? sqrt(y2) : 0.0); y.sg = Dv;
        y.c = 1.0; y.s = 0.0;
        if (y.py < 0.0) winsert(c, &y);
    }
}

/* a window from the source (the origin of the source frame) on half-edge th
 * whose tail is O and head Q in that frame; 0 when the source lies on the
 * edge's line (no window: the face across holds the source too) */
static int wseed(wctx *c, int th, const double *O, const double *Q) {
    if (th < 0) return 1;
    double L = c->m->len[th], ux = (Q[0] - O[0]) / L, uy = (Q[1] - O[1]) / L;
    wwin y;
    memset(&y, 0, sizeof y);
    y.h = th; y.root = -1; y.alive = 1;
    y.b0 = 0.0; y.b1 = L;
    y.px = -O[0] * ux - O[1] * uy;
    y.py = -O[1] * ux + O[0] * uy;
    y.c = ux; y.s = uy;
    if (!(y.py < 0.0)) return 0;
    winsert(c, &y);
    return 1;
}

static void wsource_vertex(wctx *c, int v, const double *P) {
    double l = len2(P), t[2] = {0.0, 0.0};
    if (l > 0.0) { t[0] = P[0] / l; t[1] = P[1] / l; }
    wvertex(c, v, l, t);
}

/* one source: seed, propagate, then the distance and tangent to every
 * target (best[j] = INFINITY where none is found below the bound) */
static int wsource(wctx *c, int src, const int *face, const double *bary, int n, double *best, double *tang) {
    const orc_mesh *m = c->m;
    int f = face[src];
    const double *b = bary + 3 * src;
    for (int j = 0; j < n; j++) best[j] = INFINITY;
    if ((b[0] <= 0.0) + (b[1] <= 0.0) + (b[2] <= 0.0) >= 2) return -1; /* on a vertex */
    double P[3][2];
    P[0][0] = 0.0; P[0][1] = 0.0;
    P[1][0] = m->len[3 * f]; P[1][1] = 0.0;
    unfold_third(P[0], P[1], m->len[3 * f], m->len[3 * f + 2], m->len[3 * f + 1], P[2]);
    double s[2] = {b[0] * P[0][0] + b[1] * P[1][0] + b[2] * P[2][0], b[0] * P[0][1] + b[1] * P[1][1] + b[2] * P[2][1]};
    for (int k = 0; k < 3; k++) { P[k][0] -= s[0]; P[k][1] -= s[1]; }
    /* faces holding the source, with their corners in the source frame */
    int sf[4] = {f, -1, -1, -1}, nsf = 1;
    double SP[4][3][2];
    memcpy(SP[0], P, sizeof P);
    for (int k = 0; k < 3; k++) wsource_vertex(c, m->T[3 * f + k], P[k]);
    for (int k = 0; k < 3; k++) {
        int h = 3 * f + k, t = m->twin[h];
        const double *X = P[k], *Y = P[(k + 1) % 3];
        if (b[(k + 2) % 3] > 0.0 && wseed(c, t, Y, X)) continue; /* the twin runs Y -> X */
        if (t < 0) continue;
        /* the source is on this edge (exactly, or up to rounding): the face
         * across holds it too */
        double Z[2];
        unfold_third(Y, X, m->len[t], m->len[he_prev(t)], m->len[he_next(t)], Z);
        sf[nsf] = t / 3;
        int kk = t % 3; /* corner order of face t/3: T[t] = Y, next = X, prev = Z */
        memcpy(SP[nsf][kk], Y, sizeof(double) * 2);
        memcpy(SP[nsf][(kk + 1) % 3], X, sizeof(double) * 2);
        memcpy(SP[nsf][(kk + 2) % 3], Z, sizeof(double) * 2);
        nsf++;
        wsource_vertex(c, m->T[he_prev(t)], Z);
        wseed(c, m->twin[he_next(t)], Z, X); /* next(t) runs X -> Z */
        wseed(c, m->twin[he_prev(t)], Y, Z); /* prev(t) runs Z -> Y */
    }
    /* continuous Dijkstra */
    double k; int id, gen;
    while (wheap_pop(c, &k, &id, &gen)) {
        if (!(k < c->U)) break;
        if (id < 0) {
            int v = -1 - id;
            if (c->launched[v] || k > c->D[v]) continue;
            wlaunch(c, v);
        } else {
            const wwin *w = &c->w[id];
            if (!w->alive || w->done || w->gen != gen) continue;
            wprocess(c, id);
        }
    }
    /* targets */
    for (int j = 0; j < n; j++) {
        if (j == src) continue;
        int g = face[j];
        const double *bj = bary + 3 * j;
        double bd = INFINITY, bt[2] = {0.0, 0.0};
        for (int z = 0; z < nsf; z++) {
            if (sf[z] != g) continue;
            double q[2] = {0.0, 0.0};
            for (int a = 0; a < 3; a++) { q[0] += bj[a] * SP[z][a][0]; q[1] += bj[a] * SP[z][a][1]; }
            double d = len2(q);
            if (d < bd) { bd = d; bt[0] = d > 0.0 ? q[0] / d : 0.0; bt[1] = d > 0.0 ? q[1] / d : 0.0; }
        }
        double x3[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; a++)
            for (int d = 0; d < 3; d++) x3[d] += bj[a] * m->V[3 * m->T[3 * g + a] + d];
        for (int a = 0; a < 3; a++) {
            int v = m->T[3 * g + a];
            if (!m->pseudo[v] || !isfinite(c->D[v])) continue;
            double e[3];
            sub3(x3, m->V + 3 * v, e);
            double d = c->D[v] + norm3(e);
            if (d < bd) { bd = d; bt[0] = c->Dt[2 * v]; bt[1] = c->Dt[2 * v + 1]; }
        }
        for (int a = 0; a < 3; a++) {
            int h = 3 * g + a;
            if (c->hhead[h] < 0) continue;
            double L = m->len[h], cx, cy;
            third_in_frame(m, h, &cx, &cy);
            /* the target in h's frame: corners A = (0, 0), B = (L, 0), C */
            double xx = bj[(a + 1) % 3] * L + bj[(a + 2) % 3] * cx, xy = bj[(a + 2) % 3] * cy;
            const double tol = CONE_EPS * L;
            for (int o = c->hhead[h]; o >= 0; o = c->w[o].next) {
                const wwin *w = &c->w[o];
                if (!w->alive) continue;
                double tx = w->px + (xx - w->px) * (-w->py) / (xy - w->py);
                if (tx < w->b0 - tol || tx > w->b1 + tol) continue;
                double d = w->sg + hypot(xx - w->px, xy - w->py);
                if (d < bd) { bd = d; wtangent(c, w, xx - w->px, xy - w->py, bt); }
            }
        }
        if (bd < c->U) { best[j] = bd; tang[2 * j] = bt[0]; tang[2 * j + 1] = bt[1]; }
    }
    return 0;
}

static void wreset(wctx *c) {
    for (int i = 0; i < c->nht; i++) c->hhead[c->htouch[i]] = -1;
    for (int i = 0; i < c->nvt; i++) { c->D[c->vtouch[i]] = INFINITY; c->launched[c->vtouch[i]] = 0; }
    for (int i = 0; i < c->nft; i++) c->fmark[c->ftouch[i]] = 0;
    c->nht = c->nvt = c->nft = 0;
    c->nw = 0; c->hn = 0;
}

orc_pairs *orc_geodesic_pairs_windows(const orc_mesh *m, int n, const int *face, const double *bary, double cutoff,
                                      int nsrc, const int *src, int nthreads) {
    if (!m || n < 0 || (n > 0 && (!face || !bary))) return NULL;
    for (int j = 0; j < n; j++)
        if (face[j] < 0 || face[j] >= m->nf) return NULL;
    int all = !(cutoff > 0.0) || !isfinite(cutoff);
    if (!src) nsrc = n;
    row_t *rows = (row_t *)calloc(nsrc > 0 ? nsrc : 1, sizeof(row_t));
    orc_pairs *res = (orc_pairs *)calloc(1, sizeof(orc_pairs));
    res->nsrc = nsrc;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        wctx c;
        memset(&c, 0, sizeof c);
        c.m = m;
        c.hhead = (int *)malloc(sizeof(int) * 3 * m->nf);
        c.htouch = (int *)malloc(sizeof(int) * 3 * m->nf);
        for (int h = 0; h < 3 * m->nf; h++) c.hhead[h] = -1;
        c.D = (double *)malloc(sizeof(double) * m->nv);
        c.Dt = (double *)malloc(sizeof(double) * 2 * m->nv);
        for (int v = 0; v < m->nv; v++) c.D[v] = INFINITY;
        c.launched = (unsigned char *)calloc(m->nv, 1);
        c.vtouch = (int *)malloc(sizeof(int) * m->nv);
        c.fmark = (unsigned char *)calloc(m->nf, 1);
        c.ftouch = (int *)malloc(sizeof(int) * m->nf);
        double *best = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
        double *tang = (double *)malloc(sizeof(double) * 2 * (n > 0 ? n : 1));
        work_t gw;
        memset(&gw, 0, sizeof gw);
        double *gdist = all ? (double *)malloc(sizeof(double) * m->nv) : NULL;
#pragma omp for schedule(dynamic, 1)
        for (int si = 0; si < nsrc; si++) {
            int i = src ? src[si] : si;
            c.U = all ? graph_bound(m, face[i], bary + 3 * i, gdist, &gw) : cutoff;
            row_t *rw = &rows[si];
            if (wsource(&c, i, face, bary, n, best, tang) != 0) c.cnt[6]++;
            int cnt = 0;
            for (int j = 0; j < n; j++)
                if (best[j] < c.U) cnt++;
            rw->n = cnt;
            rw->nbr = (int32_t *)malloc(sizeof(int32_t) * (cnt + 1));
            rw->dist = (double *)malloc(sizeof(double) * (cnt + 1));
            rw->tan = (double *)malloc(sizeof(double) * 3 * (cnt + 1));
            rw->flags = (uint8_t *)malloc(cnt + 1);
            const double *ex = m->ex + 3 * face[i], *ey = m->ey + 3 * face[i];
            int q = 0;
            for (int j = 0; j < n; j++) {
                if (!(best[j] < c.U)) continue;
                rw->nbr[q] = j; rw->dist[q] = best[j];
                for (int d = 0; d < 3; d++) rw->tan[3 * q + d] = tang[2 * j] * ex[d] + tang[2 * j + 1] * ey[d];
                rw->flags[q] = best[j] == 0.0 ? 2 : 0;
                q++;
            }
            wreset(&c);
        }
#pragma omp critical
        {
            for (int z = 0; z < 7; z++) res->wcounters[z] += c.cnt[z];
        }
        free(c.w); free(c.hhead); free(c.htouch); free(c.hk); free(c.hid); free(c.hgen); free(c.D); free(c.Dt);
        free(c.launched); free(c.vtouch); free(c.fmark); free(c.ftouch); free(best); free(tang);
        free(gw.hk); free(gw.hv); free(gdist);
    }
    /* flatten: one direction per pair, no tie sets */
    res->off = (int64_t *)malloc(sizeof(int64_t) * (nsrc + 1));
    res->off[0] = 0;
    int64_t tot = 0;
    for (int s = 0; s < nsrc; s++) { tot += rows[s].n; res->off[s + 1] = tot; }
    res->count = res->tcount = tot;
    res->nbr = (int32_t *)malloc(sizeof(int32_t) * (tot + 1));
    res->dist = (double *)malloc(sizeof(double) * (tot + 1));
    res->tan = (double *)malloc(sizeof(double) * 3 * (tot + 1));
    res->flags = (uint8_t *)malloc(tot + 1);
    res->tie_off = (int64_t *)malloc(sizeof(int64_t) * (tot + 1));
    res->tie_tan = (double *)malloc(sizeof(double) * 3 * (tot + 1));
    res->tie_dist = (double *)malloc(sizeof(double) * (tot + 1));
    res->tie_off[0] = 0;
    int64_t p = 0;
    for (int s = 0; s < nsrc; s++) {
        row_t *rw = &rows[s];
        for (int q = 0; q < rw->n; q++, p++) {
            res->nbr[p] = rw->nbr[q]; res->dist[p] = rw->dist[q];
            memcpy(res->tan + 3 * p, rw->tan + 3 * q, sizeof(double) * 3);
            memcpy(res->tie_tan + 3 * p, rw->tan + 3 * q, sizeof(double) * 3);
            res->tie_dist[p] = rw->dist[q];
            res->flags[p] = rw->flags[q];
            res->tie_off[p + 1] = p + 1;
        }
        free(rw->nbr); free(rw->dist); free(rw->tan); free(rw->flags);
    }
    free(rows);
    return res;
}

void orc_pairs_window_counters(const orc_pairs *p, int64_t *c7) { memcpy(c7, p->wcounters, sizeof(int64_t) * 7); }

/* ======================================================================
 * 3. The shift walk (Sec. 3.2): straight across faces; at an edge, move to
 *    the face across it and rotate the direction (and the velocity) about
 *    the edge; at a vertex, leave along the straightest direction (equal
 *    angle sums on both sides); at a boundary edge, reflect.
 * ====================================================================== */
#define WALK_CAP 10000
#define VTX_TOL 1e-12
#define NEAR_TOL 1e-9

static void rotate_about_edge(const double *e, const double *m_out, const double *m_in, double *vec) {
    double ue = dot3(vec, e), um = dot3(vec, m_out);
    for (int d = 0; d < 3; d++) vec[d] = ue * e[d] + um * m_in[d];
}

int orc_walk(const orc_mesh *m, int n, int *face, double *bary, const double *disp, double *vel, int64_t *stats,
             uint8_t *flags) {
    int64_t st[5] = {0, 0, 0, 0, 0};
    double lbar = m->mean_edge;
    for (int p = 0; p < n; p++) {
        int f = face[p];
        double b[3] = {bary[3 * p], bary[3 * p + 1], bary[3 * p + 2]};
        double u[3] = {disp[3 * p], disp[3 * p + 1], disp[3 * p + 2]};
        double v[3] = {0, 0, 0};
        uint8_t fl = 0;
        if (vel) { v[0] = vel[3 * p]; v[1] = vel[3 * p + 1]; v[2] = vel[3 * p + 2]; }
        const double *nf = m->nrm + 3 * f;
        double un = dot3(u, nf);
        for (int d = 0; d < 3; d++) u[d] -= un * nf[d];
        double vn = dot3(v, nf);
        for (int d = 0; d < 3; d++) v[d] -= vn * nf[d];
        double L = norm3(u);
        if (L > 0.0) {
            for (int d = 0; d < 3; d++) u[d] /= L;
            int ignore = -1, only = -1, it = 0;
            for (;;) {
                if (++it > WALK_CAP) { st[3]++; fl |= 4; break; }
                nf = m->nrm + 3 * f;
                const double *P[3] = {m->V + 3 * m->T[3 * f], m->V + 3 * m->T[3 * f + 1], m->V + 3 * m->T[3 * f + 2]};
                double e01[3], e02[3], cr[3];
                sub3(P[1], P[0], e01); sub3(P[2], P[0], e02); cross3(e01, e02, cr);
                double A2 = norm3(cr);
                double beta[3], s[3];
                for (int k = 0; k < 3; k++) {
                    double ek[3], g[3];
                    sub3(P[(k + 2) % 3], P[(k + 1) % 3], ek);
                    cross3(nf, ek, g);
                    beta[k] = dot3(u, g) / A2;
                    s[k] = INFINITY;
                    if (k == ignore) continue;
                    if (only >= 0 && k != only) continue;
                    if (beta[k] < 0.0) { s[k] = -b[k] / beta[k]; if (s[k] < 0.0) s[k] = 0.0; }
                }
                int k1 = 0;
                for (int k = 1; k < 3; k++) if (s[k] < s[k1]) k1 = k;
                double s2 = INFINITY; int k2 = -1;
                for (int k = 0; k < 3; k++) if (k != k1 && s[k] < s2) { s2 = s[k]; k2 = k; }
                double s1 = s[k1];
                if (!(L > s1)) { /* ends inside (or on the boundary of) this face */
                    for (int k = 0; k < 3; k++) b[k] += L * beta[k];
                    break;
                }
                if (k2 >= 0 && s2 - s1 <= NEAR_TOL * lbar && !(s2 - s1 <= VTX_TOL * lbar)) { st[4]++; fl |= 2; }
                if (k2 >= 0 && s2 - s1 <= VTX_TOL * lbar) {
                    /* passes through the vertex where b[k1] = b[k2] = 0 */
                    int ws = 3 - k1 - k2, wv = m->T[3 * f + ws];
                    L -= s1;
                    st[1]++; fl |= 1;
                    if (m->bnd[wv]) {
                        for (int d = 0; d < 3; d++) { u[d] = -u[d]; v[d] = -v[d]; }
                        b[0] = b[1] = b[2] = 0.0; b[ws] = 1.0;
                        only = ws; ignore = -1;
                        continue;
                    }
                    /* polar angle of the reversed incoming direction */
                    int hin = 3 * f + ws, jin = -1;
                    double off = 0.0, phi_back = 0.0, theta = m->theta[wv];
                    for (int a = m->fan_off[wv]; a < m->fan_off[wv + 1]; a++) {
                        if (m->fan[a] == hin) { jin = a; break; }
                        off += m->corner[m->fan[a]];
                    }
                    {
                        double e1[3], back[3] = {-u[0], -u[1], -u[2]}, c[3];
                        sub3(m->V + 3 * m->T[he_next(hin)], m->V + 3 * wv, e1); unit3(e1);
                        cross3(e1, back, c);
                        double beta_ang = atan2(dot3(c, nf), dot3(e1, back));
                        if (beta_ang < 0.0) beta_ang = 0.0;
                        if (beta_ang > m->corner[hin]) beta_ang = m->corner[hin];
                        phi_back = off + beta_ang;
                    }
                    (void)jin;
                    /* velocity angle relative to the direction of travel */
                    double vm = norm3(v), psi = 0.0;
                    if (vm > 0.0) {
                        double c[3]; cross3(u, v, c);
                        psi = atan2(dot3(c, nf), dot3(u, v));
                    }
                    double phi_out = fmod(phi_back + 0.5 * theta, theta);
                    double acc = 0.0; int hout = m->fan[m->fan_off[wv + 1] - 1];
                    for (int a = m->fan_off[wv]; a < m->fan_off[wv + 1]; a++) {
                        double c = m->corner[m->fan[a]];
                        if (phi_out < acc + c) { hout = m->fan[a]; break; }
                        acc += c;
                    }
                    double gam = phi_out - acc;
                    if (gam < 0.0) gam = 0.0;
                    if (gam > m->corner[hout]) gam = m->corner[hout];
                    int g = hout / 3;
                    const double *ng = m->nrm + 3 * g;
                    double e1[3], e1p[3];
                    sub3(m->V + 3 * m->T[he_next(hout)], m->V + 3 * wv, e1); unit3(e1);
                    cross3(ng, e1, e1p);
                    for (int d = 0; d < 3; d++) u[d] = cos(gam) * e1[d] + sin(gam) * e1p[d];
                    if (vm > 0.0) {
                        double up[3]; cross3(ng, u, up);
                        for (int d = 0; d < 3; d++) v[d] = vm * (cos(psi) * u[d] + sin(psi) * up[d]);
                    }
                    f = g;
                    b[0] = b[1] = b[2] = 0.0; b[hout % 3] = 1.0;
                    only = hout % 3; ignore = -1;
                    continue;
                }
                /* edge crossing through the edge opposite slot k1 */
                for (int k = 0; k < 3; k++) b[k] += s1 * beta[k];
                b[k1] = 0.0;
                L -= s1;
                int h = 3 * f + (k1 + 1) % 3, t = m->twin[h];
                double e[3], mo[3];
                sub3(P[(k1 + 2) % 3], P[(k1 + 1) % 3], e); unit3(e);
                cross3(e, nf, mo);
                if (t < 0) {
                    st[2]++; fl |= 8;
                    double um = dot3(u, mo), vmo = dot3(v, mo);
                    for (int d = 0; d < 3; d++) { u[d] -= 2.0 * um * mo[d]; v[d] -= 2.0 * vmo * mo[d]; }
                    ignore = k1; only = -1;
                    continue;
                }
                st[0]++;
                int g = t / 3, mm = t % 3;
                double nb[3];
                nb[mm] = b[(k1 + 2) % 3];
                nb[(mm + 1) % 3] = b[(k1 + 1) % 3];
                nb[(mm + 2) % 3] = 0.0;
                double mi[3];
                cross3(e, m->nrm + 3 * g, mi);
                rotate_about_edge(e, mo, mi, u);
                rotate_about_edge(e, mo, mi, v);
                f = g; b[0] = nb[0]; b[1] = nb[1]; b[2] = nb[2];
                ignore = (mm + 2) % 3; only = -1;
            }
        }
        face[p] = f;
        bary[3 * p] = b[0]; bary[3 * p + 1] = b[1]; bary[3 * p + 2] = b[2];
        if (vel) { vel[3 * p] = v[0]; vel[3 * p + 1] = v[1]; vel[3 * p + 2] = v[2]; }
        if (flags) flags[p] = fl;
    }
    if (stats) memcpy(stats, st, sizeof st);
    return 0;
}

/* ======================================================================
 * 4. Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of
 *    the multiply-xor bijection with a Weyl-sequence key schedule.
 * ====================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------
 * Restricted Voronoi neighbours (Sec. 5: the in-surface Voronoi diagram,
 * generated there as a restricted Euclidean Voronoi diagram, whose cells
 * give each particle's number of neighbours). The plain definition: the cell
 * of particle i is the set of surface points no farther (3D distance) from
 * x_i than from any other particle; i and j are neighbours when the surface
 * points equidistant from x_i and x_j and no farther from them than from any
 * other particle form a set of positive length. In one triangle that set is
 * the triangle cut by the bisector plane of x_i and x_j, clipped by the
 * half-spaces {|x - x_i| <= |x - x_k|} of every other particle k.
 * ---------------------------------------------------------------------- */

/* squared distance from p to the triangle (a, b, c): the closest point is a
 * vertex, a point of an edge, or the projection into the interior, chosen by
 * the Voronoi regions of the triangle's features (the closest-point method
 * of C. Ericson, Real-Time Collision Detection, 2005, Sec. 5.1.5) */
static double point_tri_dist2(const double *p, const double *a, const double *b, const double *c) {
    double ab[3], ac[3], ap[3], q[3];
    sub3(b, a, ab);
    sub3(c, a, ac);
    sub3(p, a, ap);
    const double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) return dot3(ap, ap);
    double bp[3];
    sub3(p, b, bp);
    const double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) return dot3(bp, bp);
    const double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        const double v = d1 / (d1 - d3);
        for (int k = 0; k < 3; ++k) q[k] = a[k] + v * ab[k];
    } else {
        double cp[3];
        sub3(p, c, cp);
        const double d5 = dot3(ab, cp), d6 = dot3(ac, cp);
        if (d6 >= 0.0 && d5 <= d6) return dot3(cp, cp);
        const double vb = d5 * d2 - d1 * d6;
        if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
            const double w = d2 / (d2 - d6);
            for (int k = 0; k < 3; ++k) q[k] = a[k] + w * ac[k];
        } else {
            const double va = d3 * d6 - d5 * d4;
            if (va <= 0.0 && (d4 - d3) >= 0.0 && (d5 - d6) >= 0.0) {
                const double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
                for (int k = 0; k < 3; ++k) q[k] = b[k] + w * (c[k] - b[k]);
            } else {
                const double den = 1.0 / (va + vb + vc);
                const double v = vb * den, w = vc * den;
                for (int k = 0; k < 3; ++k) q[k] = a[k] + ab[k] * v + ac[k] * w;
            }
        }
    }
    double d[3];
    sub3(p, q, d);
    return dot3(d, d);
}

static double dist2(const double *a, const double *b) {
    double d[3];
    sub3(a, b, d);
    return dot3(d, d);
}

int orc_voronoi_pairs(const orc_mesh *m, int n, const double *xyz, double tol, unsigned char *adj) {
    if (!m || n < 2 || !xyz || !adj) return 1;
    memset(adj, 0, (size_t)n * (size_t)n);
    int *cand = (int *)malloc(sizeof(int) * (size_t)n);
    if (!cand) return 1;
    for (int f = 0; f < m->nf; ++f) {
        const double *A = m->V + 3 * (size_t)m->T[3 * f], *B = m->V + 3 * (size_t)m->T[3 * f + 1],
                     *Cv = m->V + 3 * (size_t)m->T[3 * f + 2];
        const double *P[3] = {A, B, Cv};
        /* a particle can be nearest somewhere in the triangle only if its
         * distance to the triangle is at most the smallest, over particles,
         * of the farthest vertex distance (distance is convex, so the
         * farthest point of the triangle is a vertex) */
        double mT2 = INFINITY;
        for (int j = 0; j < n; ++j) {
            double far2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                const double d2 = dist2(P[k], xyz + 3 * (size_t)j);
                if (d2 > far2) far2 = d2;
            }
            if (far2 < mT2) mT2 = far2;
        }
        int nc = 0;
        for (int i = 0; i < n; ++i)
            if (point_tri_dist2(xyz + 3 * (size_t)i, A, B, Cv) <= mT2 * (1.0 + 1e-9)) cand[nc++] = i;
        for (int a = 0; a < nc; ++a)
            for (int b = a + 1; b < nc; ++b) {
                const int i = cand[a], j = cand[b];
                const double *xi = xyz + 3 * (size_t)i, *xj = xyz + 3 * (size_t)j;
                if (adj[(size_t)i * n + j]) continue;
                /* bisector plane: g(x) = 2 (xj - xi).x - (|xj|^2 - |xi|^2) */
                double nrmv[3];
                sub3(xj, xi, nrmv);
                const double rhs = dot3(xj, xj) - dot3(xi, xi);
                double g[3];
                for (int k = 0; k < 3; ++k) g[k] = 2.0 * dot3(nrmv, P[k]) - rhs;
                if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue; /* triangle in the plane */
                double pts[6][3];
                int np = 0;
                for (int k = 0; k < 3; ++k) {
                    const int k2 = (k + 1) % 3;
                    if (g[k] == 0.0) {
                        memcpy(pts[np++], P[k], sizeof(double) * 3);
                    } else if ((g[k] < 0.0 && g[k2] > 0.0) || (g[k] > 0.0 && g[k2] < 0.0)) {
                        const double t = g[k] / (g[k] - g[k2]);
                        for (int d = 0; d < 3; ++d) pts[np][d] = P[k][d] + t * (P[k2][d] - P[k][d]);
                        ++np;
                    }
                }
                if (np < 2) continue;
                /* the segment between the two points farthest apart */
                int s0 = 0, s1 = 1;
                double best = -1.0;
                for (int u = 0; u < np; ++u)
                    for (int v = u + 1; v < np; ++v) {
                        const double d2 = dist2(pts[u], pts[v]);
                        if (d2 > best) {
                            best = d2;
                            s0 = u;
                            s1 = v;
                        }
                    }
                const double *S = pts[s0], *E = pts[s1];
                double dir[3];
                sub3(E, S, dir);
                const double len = norm3(dir);
                if (!(len > tol)) continue;
                /* clip t in [0, 1] by |x - xi|^2 <= |x - xk|^2 for every other k:
                 * 2 (xk - xi).x <= |xk|^2 - |xi|^2, linear in t */
                double t0 = 0.0, t1 = 1.0;
                for (int k = 0; k < n && t0 < t1; ++k) {
                    if (k == i || k == j) continue;
                    const double *xk = xyz + 3 * (size_t)k;
                    double w[3];
                    sub3(xk, xi, w);
                    const double c = dot3(xk, xk) - dot3(xi, xi);
                    const double h0 = 2.0 * dot3(w, S) - c;    /* at t = 0; allowed where <= 0 */
                    const double h1 = 2.0 * dot3(w, dir);      /* slope */
                    if (h1 == 0.0) {
                        if (h0 > 0.0) t1 = t0 - 1.0;
                    } else {
                        const double tz = -h0 / h1;
                        if (h1 > 0.0) {
                            if (tz < t1) t1 = tz;
                        } else {
                            if (tz > t0) t0 = tz;
                        }
                    }
                }
                if ((t1 - t0) * len > tol) {
                    adj[(size_t)i * n + j] = 1;
                    adj[(size_t)j * n + i] = 1;
                }
            }
    }
    free(cand);
    return 0;
}

