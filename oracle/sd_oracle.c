/*
 * FP64 reference ("oracle") for the smooth distance of Madan & Levin,
 * "Fast Evaluation of Smooth Distance Constraints on Co-Dimensional Geometry".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or constant with the HIP
 * path.  Everything is plain, unblocked FP64 arithmetic so that each step can
 * be checked against the paper by eye:
 *
 *   distances and closest points ........ App. B (Eq. 10, Eq. 11)
 *   blending weights w = (A w~)^S ........ Sec. 3.3, App. C (polynomial
 *                                          coefficients are solved in oracle.py
 *                                          and passed in here per class)
 *   weight gradient (chain rule) ......... Sec. 3.3 Eq. 5
 *   log-sum-exp value and gradient ....... Sec. 3 Eq. 3 and Eq. 4, evaluated
 *                                          two-pass with the maximum factored out
 *   Barnes-Hut far field ................. Sec. 3.5, App. D, Alg. 1 and Alg. 2
 *   rigid-query adjoint .................. d/dR, d/dt, d/dx of d(R x + t)
 *
 * Scene inputs are the FP32 arrays the GPU receives, promoted to double;
 * queries are passed as double so that finite differences can be taken.
 * Build: gcc -O2 -fopenmp -shared -fPIC sd_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 ld(const float *p) { return mk((double)p[0], (double)p[1], (double)p[2]); }
static v3 ldd(const double *p) { return mk(p[0], p[1], p[2]); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static double norm(v3 a) { return sqrt(dot(a, a)); }

/* ------------------------------------------------------------------------ */
/* Scene and parameters                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t nP; const float *P;                     /* nP x 3 point coordinates          */
    int64_t nE; const float *E;                     /* nE x 6: v0, v1                    */
    const int32_t *Ecls; const double *Ecoef;       /* per-edge class; class x 5 monomial coeffs */
    int64_t nT; const float *T;                     /* nT x 9: v0, v1, v2                */
    const int32_t *Tcls; const double *Tcoef;       /* per-tri class; class x 64 slots, c_ab at a*8+b (a+b<=7) */
    double logA_E, logA_T;                          /* log of the global weight scale A per class */
} or_scene;

typedef struct {
    double alpha, alpha_u, beta;
    int32_t metric_r2;   /* 1: barycentric gradients measured in the alpha-scaled metric (Sec. 3.3) */
    int32_t cut_f32;     /* 1: take the open/accept decision of Sec. 3.5 in FP32 (see accept_far) */
} or_params;

/* One exported hierarchy (one per primitive class). */
typedef struct {
    int64_t n_nodes;
    const float *box;        /* n x 6: min xyz, max xyz                      */
    const int32_t *left;     /* child ids, -1 for leaves                     */
    const int32_t *right;
    const int32_t *prim;     /* original primitive id for leaves, -1 else    */
} or_tree;

/* ------------------------------------------------------------------------ */
/* App. B: exact distances with closest point, barycentrics and d(phi)/dq    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double d;          /* distance                                          */
    v3 c;              /* closest point on the primitive                    */
    double phi[2];     /* barycentric coordinates of the closest point      */
    v3 dphi[2];        /* gradient of each barycentric coordinate wrt q     */
    int region;        /* 0 interior (face / segment), 1 edge, 2 vertex      */
} closest;

/* closest point of segment a + t (b - a), t in [0,1] */
static double seg_t(v3 q, v3 a, v3 b, int *interior) {
    v3 e = sub(b, a);
    double ee = dot(e, e);
    *interior = 0;
    if (ee == 0.0) return 0.0;
    double t = dot(sub(q, a), e) / ee;
    if (t <= 0.0) return 0.0;
    if (t >= 1.0) return 1.0;
    *interior = 1;
    return t;
}

static void point_closest(v3 q, v3 p, closest *o) {
    o->c = p;
    o->d = norm(sub(q, p));
    o->phi[0] = o->phi[1] = 0.0;
    o->dphi[0] = o->dphi[1] = mk(0, 0, 0);
    o->region = 2;
}

/* segment v0 -> v1, barycentric phi: point = (1 - phi) v0 + phi v1 */
static void segment_closest(v3 q, v3 a, v3 b, closest *o) {
    int interior;
    double t = seg_t(q, a, b, &interior);
    v3 e = sub(b, a);
    o->c = add(a, scl(e, t));
    o->d = norm(sub(q, o->c));
    o->phi[0] = t; o->phi[1] = 0.0;
    o->dphi[0] = interior ? scl(e, 1.0 / dot(e, e)) : mk(0, 0, 0);
    o->dphi[1] = mk(0, 0, 0);
    o->region = interior ? 0 : 2;
}

/* triangle f(phi) = (1 - phi1 - phi2) v0 + phi1 v1 + phi2 v2 (App. B).
 * The minimiser of the convex quadratic |q - f(phi)|^2 over the simplex is the
 * unconstrained plane projection when that lies inside the triangle, else it
 * lies on the boundary, i.e. on the closest of the three edges. */
static void triangle_closest(v3 q, v3 v0, v3 v1, v3 v2, closest *o) {
    v3 e1 = sub(v1, v0), e2 = sub(v2, v0), r = sub(q, v0);
    double g11 = dot(e1, e1), g12 = dot(e1, e2), g22 = dot(e2, e2);
    double det = g11 * g22 - g12 * g12;
    v3 n = cross(e1, e2);
    if (dot(n, n) > 0.0 && det > 0.0) {
        double r1 = dot(e1, r), r2 = dot(e2, r);
        double p1 = (g22 * r1 - g12 * r2) / det;
        double p2 = (g11 * r2 - g12 * r1) / det;
        if (p1 >= 0.0 && p2 >= 0.0 && p1 + p2 <= 1.0) {
            o->phi[0] = p1; o->phi[1] = p2;
            o->c = add(v0, add(scl(e1, p1), scl(e2, p2)));
            o->d = norm(sub(q, o->c));
            /* d(phi)/dq = G^-1 [e1^T; e2^T] */
            o->dphi[0] = scl(sub(scl(e1, g22), scl(e2, g12)), 1.0 / det);
            o->dphi[1] = scl(sub(scl(e2, g11), scl(e1, g12)), 1.0 / det);
            o->region = 0;
            return;
        }
    }
    /* boundary: edges (v0,v1) -> phi=(t,0); (v1,v2) -> phi=(1-t,t); (v2,v0) -> phi=(0,1-t) */
    v3 A[3] = {v0, v1, v2}, B[3] = {v1, v2, v0};
    double best = INFINITY; int bi = 0; double bt = 0; int bint = 0;
    int degenerate = !(dot(n, n) > 0.0 && det > 0.0);
    if (degenerate) {
        /* zero area (the paper is silent): the triangle is its longest edge,
         * which covers the other two, so the closest point and barycentrics
         * do not depend on how ties between the three edges are broken */
        double lmax = -1.0;
        for (int k = 0; k < 3; ++k) {
            double l = dot(sub(B[k], A[k]), sub(B[k], A[k]));
            if (l > lmax) { lmax = l; bi = k; }
        }
        bt = seg_t(q, A[bi], B[bi], &bint);
        best = norm(sub(q, add(A[bi], scl(sub(B[bi], A[bi]), bt))));
    }
    for (int k = 0; k < 3 && !degenerate; ++k) {
        int interior;
        double t = seg_t(q, A[k], B[k], &interior);
        double d = norm(sub(q, add(A[k], scl(sub(B[k], A[k]), t))));
        if (d < best) { best = d; bi = k; bt = t; bint = interior; }
    }
    v3 e = sub(B[bi], A[bi]);
    v3 dt = bint ? scl(e, 1.0 / dot(e, e)) : mk(0, 0, 0);
    o->c = add(A[bi], scl(e, bt));
    o->d = best;
    o->region = bint ? 1 : 2;
    if (bi == 0) { o->phi[0] = bt; o->phi[1] = 0; o->dphi[0] = dt; o->dphi[1] = mk(0, 0, 0); }
    else if (bi == 1) { o->phi[0] = 1 - bt; o->phi[1] = bt; o->dphi[0] = scl(dt, -1); o->dphi[1] = dt; }
    else { o->phi[0] = 0; o->phi[1] = 1 - bt; o->dphi[0] = mk(0, 0, 0); o->dphi[1] = scl(dt, -1); }
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.3 / App. C: weights.  Returns log w and grad(log w) wrt q.        */
/* ------------------------------------------------------------------------ */
static double poly1(const double *c, double x, double *dx) {
    double v = 0, d = 0, p = 1;
    for (int a = 0; a <= 4; ++a) {
        v += c[a] * p;
        if (a < 4) d += (a + 1) * c[a + 1] * p;
        p *= x;
    }
    *dx = d;
    return v;
}

static double poly2(const double *c, double x, double y, double *dx, double *dy) {
    double v = 0, gx = 0, gy = 0;
    for (int a = 0; a <= 7; ++a)
        for (int b = 0; a + b <= 7; ++b) {
            double k = c[a * 8 + b];
            if (k == 0.0) continue;
            double xa = pow(x, a), yb = pow(y, b);
            v += k * xa * yb;
            if (a > 0) gx += k * a * pow(x, a - 1) * yb;
            if (b > 0) gy += k * b * xa * pow(y, b - 1);
        }
    *dx = gx; *dy = gy;
    return v;
}

/* S = alpha / max(alpha, alpha_U)   (Sec. 3.3, attenuation) */
static double atten(const or_params *p) {
    return p->alpha / (p->alpha > p->alpha_u ? p->alpha : p->alpha_u);
}

/* ------------------------------------------------------------------------ */
/* Term list and the log-sum-exp of Eq. 3 / Eq. 4                            */
/* ------------------------------------------------------------------------ */
typedef struct { double L; v3 g; } term;   /* L = log w - alpha d,  g = grad d - grad(log w)/alpha */

typedef struct {
    term *t; int64_t n, cap;
} termlist;

static void push(termlist *tl, double L, v3 g) {
    if (tl->n == tl->cap) {
        tl->cap = tl->cap ? 2 * tl->cap : 256;
        tl->t = (term *)realloc(tl->t, (size_t)tl->cap * sizeof(term));
    }
    tl->t[tl->n].L = L; tl->t[tl->n].g = g; tl->n++;
}

/* d = -(1/alpha) log sum_i exp(L_i), grad = sum_i p_i g_i with p the softmax of L.
 * Empty sum: d = +inf, grad = 0. */
static void lse_finish(const termlist *tl, double alpha, double *d, double *g) {
    if (tl->n == 0) { *d = INFINITY; g[0] = g[1] = g[2] = 0; return; }
    double M = -INFINITY;
    for (int64_t i = 0; i < tl->n; ++i) if (tl->t[i].L > M) M = tl->t[i].L;
    double s = 0; v3 G = mk(0, 0, 0);
    for (int64_t i = 0; i < tl->n; ++i) {
        double e = exp(tl->t[i].L - M);
        s += e;
        G = add(G, scl(tl->t[i].g, e));
    }
    *d = -(M + log(s)) / alpha;
    g[0] = G.x / s; g[1] = G.y / s; g[2] = G.z / s;
}

/* exact contribution of one primitive (class 0 point, 1 edge, 2 triangle) */
static void exact_term(const or_scene *sc, const or_params *p, int cls, int64_t i, v3 q,
                       termlist *tl, double *dmin) {
    closest cp;
    double logw = 0.0, S = atten(p);
    v3 glogw = mk(0, 0, 0);
    if (cls == 0) {
        point_closest(q, ld(sc->P + 3 * i), &cp);
    } else if (cls == 1) {
        segment_closest(q, ld(sc->E + 6 * i), ld(sc->E + 6 * i + 3), &cp);
        double dw, w = poly1(sc->Ecoef + 5 * sc->Ecls[i], cp.phi[0], &dw);
        logw = S * (sc->logA_E + log(w));
        glogw = scl(cp.dphi[0], S * dw / w);
    } else {
        const float *t = sc->T + 9 * i;
        triangle_closest(q, ld(t), ld(t + 3), ld(t + 6), &cp);
        double dw1, dw2;
        double w = poly2(sc->Tcoef + 64 * (int64_t)sc->Tcls[i], cp.phi[0], cp.phi[1], &dw1, &dw2);
        logw = S * (sc->logA_T + log(w));
        glogw = scl(add(scl(cp.dphi[0], dw1), scl(cp.dphi[1], dw2)), S / w);
    }
    if (p->metric_r2) glogw = scl(glogw, 1.0 / p->alpha);
    /* Eq. 11: grad d = (q - c)/|q - c|, zero when d = 0 */
    v3 gd = cp.d > 0 ? scl(sub(q, cp.c), 1.0 / cp.d) : mk(0, 0, 0);
    push(tl, logw - p->alpha * cp.d, sub(gd, scl(glogw, 1.0 / p->alpha)));
    if (cp.d < *dmin) *dmin = cp.d;
}

/* ------------------------------------------------------------------------ */
/* Public: brute force over every primitive (beta = 0 semantics)             */
/* ------------------------------------------------------------------------ */
int or_brute(const or_scene *sc, const or_params *p, int64_t nq, const double *Q,
             double *d_out, double *g_out, double *dmin_out) {
    if (!(p->alpha > 0)) return -1;
#pragma omp parallel
    {
        termlist tl = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nq; ++k) {
            v3 q = ldd(Q + 3 * k);
            double dmin = INFINITY;
            tl.n = 0;
            for (int64_t i = 0; i < sc->nP; ++i) exact_term(sc, p, 0, i, q, &tl, &dmin);
            for (int64_t i = 0; i < sc->nE; ++i) exact_term(sc, p, 1, i, q, &tl, &dmin);
            for (int64_t i = 0; i < sc->nT; ++i) exact_term(sc, p, 2, i, q, &tl, &dmin);
            lse_finish(&tl, p->alpha, d_out + k, g_out + 3 * k);
            if (dmin_out) dmin_out[k] = dmin;
        }
        free(tl.t);
    }
    return 0;
}

/* Exact minimum distance only (Eq. 2). */
int or_dmin(const or_scene *sc, int64_t nq, const double *Q, double *dmin_out) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < nq; ++k) {
        v3 q = ldd(Q + 3 * k);
        double m = INFINITY;
        closest cp;
        for (int64_t i = 0; i < sc->nP; ++i) { point_closest(q, ld(sc->P + 3 * i), &cp); if (cp.d < m) m = cp.d; }
        for (int64_t i = 0; i < sc->nE; ++i) { segment_closest(q, ld(sc->E + 6 * i), ld(sc->E + 6 * i + 3), &cp); if (cp.d < m) m = cp.d; }
        for (int64_t i = 0; i < sc->nT; ++i) {
            const float *t = sc->T + 9 * i;
            triangle_closest(q, ld(t), ld(t + 3), ld(t + 6), &cp);
            if (cp.d < m) m = cp.d;
        }
        dmin_out[k] = m;
    }
    return 0;
}

/* Eq. 2 by branch and bound over given hierarchies (every box contains its
 * primitives): a node is skipped only when the distance from q to its box,
 * which no primitive inside can undercut, is at least the best distance found
 * so far, so the result equals the brute-force minimum.  For the
 * conservativeness checks on large query sets. */
typedef struct { const or_scene *sc; const or_tree *tr; int cls; v3 q; double best; } nn_ctx;

static double prim_distance(const or_scene *sc, int cls, int64_t i, v3 q) {
    closest cp;
    if (cls == 0) point_closest(q, ld(sc->P + 3 * i), &cp);
    else if (cls == 1) segment_closest(q, ld(sc->E + 6 * i), ld(sc->E + 6 * i + 3), &cp);
    else triangle_closest(q, ld(sc->T + 9 * i), ld(sc->T + 9 * i + 3), ld(sc->T + 9 * i + 6), &cp);
    return cp.d;
}

static double box_distance(const float *b, v3 q) {
    v3 y = mk(fmin(fmax(q.x, b[0]), b[3]), fmin(fmax(q.y, b[1]), b[4]), fmin(fmax(q.z, b[2]), b[5]));
    return norm(sub(q, y));
}

static void nearest(nn_ctx *cx, int32_t node) {
    if (box_distance(cx->tr->box + 6 * (int64_t)node, cx->q) >= cx->best) return;
    if (cx->tr->left[node] < 0) {
        double d = prim_distance(cx->sc, cx->cls, cx->tr->prim[node], cx->q);
        if (d < cx->best) cx->best = d;
        return;
    }
    int32_t a = cx->tr->left[node], b = cx->tr->right[node];
    /* nearer child first, so the bound tightens early */
    if (box_distance(cx->tr->box + 6 * (int64_t)b, cx->q) < box_distance(cx->tr->box + 6 * (int64_t)a, cx->q)) {
        int32_t t = a; a = b; b = t;
    }
    nearest(cx, a);
    nearest(cx, b);
}

int or_dmin_tree(const or_scene *sc, const or_tree *trees, int64_t nq, const double *Q, double *dmin_out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < nq; ++k) {
        nn_ctx cx;
        cx.sc = sc; cx.q = ldd(Q + 3 * k); cx.best = INFINITY;
        for (int c = 0; c < 3; ++c) {
            if (trees[c].n_nodes <= 0) continue;
            cx.cls = c; cx.tr = &trees[c];
            nearest(&cx, 0);
        }
        dmin_out[k] = cx.best;
    }
    return 0;
}

/* Single primitive closest-point query, exposed for the pin tests. */
int or_closest(int cls, const float *prim, const double *q, double *out /* d, c[3], phi[2], dphi[6], region */) {
    closest cp;
    v3 qq = ldd(q);
    if (cls == 0) point_closest(qq, ld(prim), &cp);
    else if (cls == 1) segment_closest(qq, ld(prim), ld(prim + 3), &cp);
    else triangle_closest(qq, ld(prim), ld(prim + 3), ld(prim + 6), &cp);
    out[0] = cp.d; out[1] = cp.c.x; out[2] = cp.c.y; out[3] = cp.c.z;
    out[4] = cp.phi[0]; out[5] = cp.phi[1];
    out[6] = cp.dphi[0].x; out[7] = cp.dphi[0].y; out[8] = cp.dphi[0].z;
    out[9] = cp.dphi[1].x; out[10] = cp.dphi[1].y; out[11] = cp.dphi[1].z;
    out[12] = cp.region;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 / Alg. 2 with the conservative far field of Sec. 3.5 and App. D    */
/* ------------------------------------------------------------------------ */
typedef struct {
    const or_scene *sc; const or_params *p; v3 q; int cls;
    const or_tree *tr; const int64_t *nleaf; double logA;
    termlist *tl; double dmin_near; double margin;
    int64_t visited, far, leaves;
} bh_ctx;

/* number of primitives under each node (n_B of App. D), by recursion */
static int64_t count_leaves(const or_tree *tr, int32_t node, int64_t *out) {
    int64_t c;
    if (tr->left[node] < 0) c = 1;
    else c = count_leaves(tr, tr->left[node], out) + count_leaves(tr, tr->right[node], out);
    out[node] = c;
    return c;
}

/* The Barnes-Hut opening test of Sec. 3.5: a node is taken as one far-field
 * term iff its box diagonal |B| is below beta times the distance D from the
 * query to the box.  It decides which terms enter the sum, so a comparison
 * with a single-precision evaluator must take it in the same precision: with
 * cut_f32 the test is made on squared lengths in FP32 (query and box corners
 * rounded to FP32, each coordinate difference rounded, the sums of three
 * squares formed as fma(x, x, fma(y, y, z * z)), beta^2 rounded to FP32,
 * accept iff |B|^2 < beta^2 D^2).  Otherwise it is the FP64 test as written.
 * Only the decision changes; every term is still evaluated in FP64. */
static int accept_far(const or_params *p, const float *b, v3 q, double D, double diam) {
    if (!p->cut_f32) return diam < p->beta * D;
    float qx = (float)q.x, qy = (float)q.y, qz = (float)q.z;
    float dx = qx - fminf(fmaxf(qx, b[0]), b[3]);
    float dy = qy - fminf(fmaxf(qy, b[1]), b[4]);
    float dz = qz - fminf(fmaxf(qz, b[2]), b[5]);
    float ex = b[3] - b[0], ey = b[4] - b[1], ez = b[5] - b[2];
    float D2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float B2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
    float bf = (float)p->beta;
    float beta2 = bf * bf;
    return B2 < beta2 * D2;
}

static void collect(bh_ctx *cx, int32_t node) {
    const float *b = cx->tr->box + 6 * (int64_t)node;
    v3 lo = ld(b), hi = ld(b + 3), q = cx->q;
    /* y_B: the point of the box closest to q */
    v3 y = mk(fmin(fmax(q.x, lo.x), hi.x), fmin(fmax(q.y, lo.y), hi.y), fmin(fmax(q.z, lo.z), hi.z));
    double D = norm(sub(q, y));
    double diam = norm(sub(hi, lo));       /* |B| = box diagonal */
    cx->visited++;
    if (D > 0) {
        double m = fabs(cx->p->beta * D - diam) / D;
        if (m < cx->margin) cx->margin = m;
    }
    if (accept_far(cx->p, b, q, D, diam)) {
        /* far field: W_B exp(-alpha D) with W_B = n_B A^S, direction (q - y_B)/D */
        double logW = log((double)cx->nleaf[node]) + atten(cx->p) * cx->logA;
        push(cx->tl, logW - cx->p->alpha * D, scl(sub(q, y), 1.0 / D));
        cx->far++;
        return;
    }
    if (cx->tr->left[node] < 0) {
        double dm = INFINITY;
        exact_term(cx->sc, cx->p, cx->cls, cx->tr->prim[node], q, cx->tl, &dm);
        cx->leaves++;
        return;
    }
    collect(cx, cx->tr->left[node]);
    collect(cx, cx->tr->right[node]);
}

/* trees[3]: point, edge, triangle hierarchies (n_nodes == 0 if the class is empty).
 * stats (optional): per query [margin, visited, far, leaves]. */
int or_barnes_hut(const or_scene *sc, const or_params *p, const or_tree *trees,
                  int64_t nq, const double *Q, double *d_out, double *g_out, double *stats) {
    if (!(p->alpha > 0) || !(p->beta >= 0)) return -1;
    int64_t *nleaf[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        if (trees[c].n_nodes <= 0) continue;
        nleaf[c] = (int64_t *)calloc((size_t)trees[c].n_nodes, sizeof(int64_t));
        count_leaves(&trees[c], 0, nleaf[c]);
    }
    double logA[3] = {0.0, sc->logA_E, sc->logA_T};
#pragma omp parallel
    {
        termlist tl = {0, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nq; ++k) {
            tl.n = 0;
            bh_ctx cx;
            memset(&cx, 0, sizeof cx);
            cx.sc = sc; cx.p = p; cx.q = ldd(Q + 3 * k); cx.tl = &tl; cx.margin = INFINITY;
            for (int c = 0; c < 3; ++c) {
                if (trees[c].n_nodes <= 0) continue;
                cx.cls = c; cx.tr = &trees[c]; cx.nleaf = nleaf[c]; cx.logA = logA[c];
                collect(&cx, 0);
            }
            lse_finish(&tl, p->alpha, d_out + k, g_out + 3 * k);
            if (stats) {
                stats[4 * k + 0] = cx.margin; stats[4 * k + 1] = (double)cx.visited;
                stats[4 * k + 2] = (double)cx.far; stats[4 * k + 3] = (double)cx.leaves;
            }
        }
        free(tl.t);
    }
    for (int c = 0; c < 3; ++c) free(nleaf[c]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sec. 3.4: edges and triangles as query primitives                        */
/* ------------------------------------------------------------------------ */
/* A query primitive g has nv = 1, 2 or 3 vertices.  d(f_i, g) is the convex
 * QP of App. B over both simplices (Eq. 10); its minimiser gives the closest
 * point g(lambda) on g.  Sec. 3.4 then evaluates every formula of the point
 * query with q replaced by g(lambda): the distance from g(lambda) to f_i is
 * d(f_i, g), the weight uses the closest point on f_i, and the gradient is
 * the point-query gradient at g(lambda) (a rigid translation of g).
 *
 * The QP minimum of two convex simplices is found by enumeration: either the
 * two intersect (distance 0) or a closest pair has a point on a boundary
 * feature of one of them, so the candidates are the vertex-simplex and
 * edge-edge pairs (plus the interior edge-edge solution), each solved in
 * closed form below. */

/* closest points of segments p0 p1 and q0 q1: returns |x - y| and the point y
 * on the second segment */
static double segseg(v3 p0, v3 p1, v3 q0, v3 q1, v3 *y_out) {
    v3 u = sub(p1, p0), v = sub(q1, q0), w = sub(p0, q0);
    double a = dot(u, u), b = dot(u, v), c = dot(v, v), d = dot(u, w), e = dot(v, w);
    double best = INFINITY;
    v3 by = q0;
    double den = a * c - b * b;
    if (a > 0 && c > 0 && den > 1e-300 * a * c) {          /* interior stationary point */
        double s = (b * e - c * d) / den, t = (a * e - b * d) / den;
        if (s >= 0 && s <= 1 && t >= 0 && t <= 1) {
            v3 x = add(p0, scl(u, s)), y = add(q0, scl(v, t));
            best = norm(sub(x, y)); by = y;
        }
    }
    /* boundary: an endpoint of one segment against the other segment */
    closest cp;
    segment_closest(p0, q0, q1, &cp); if (cp.d < best) { best = cp.d; by = cp.c; }
    segment_closest(p1, q0, q1, &cp); if (cp.d < best) { best = cp.d; by = cp.c; }
    segment_closest(q0, p0, p1, &cp); if (cp.d < best) { best = cp.d; by = q0; }
    segment_closest(q1, p0, p1, &cp); if (cp.d < best) { best = cp.d; by = q1; }
    *y_out = by;
    return best;
}

/* does segment p0 p1 cross triangle t0 t1 t2?  returns 1 and the crossing point */
static int seg_tri_cross(v3 p0, v3 p1, v3 t0, v3 t1, v3 t2, v3 *x) {
    v3 n = cross(sub(t1, t0), sub(t2, t0));
    double nn = dot(n, n);
    if (!(nn > 0)) return 0;
    double s0 = dot(n, sub(p0, t0)), s1 = dot(n, sub(p1, t0));
    if ((s0 > 0 && s1 > 0) || (s0 < 0 && s1 < 0) || s0 == s1) return 0;
    double a = s0 / (s0 - s1);
    v3 y = add(p0, scl(sub(p1, p0), a));
    closest cp;
    triangle_closest(y, t0, t1, t2, &cp);
    if (cp.d > 1e-12 * (1 + norm(y))) return 0;
    *x = y;
    return 1;
}

/* segment p0 p1 against triangle t0 t1 t2: distance, the closest point on the
 * segment (*xs) and on the triangle (*xt) */
static double segtri(v3 p0, v3 p1, v3 t0, v3 t1, v3 t2, v3 *xs, v3 *xt) {
    v3 x;
    if (seg_tri_cross(p0, p1, t0, t1, t2, &x)) { *xs = x; *xt = x; return 0.0; }
    double best = INFINITY;
    closest cp;
    triangle_closest(p0, t0, t1, t2, &cp); if (cp.d < best) { best = cp.d; *xs = p0; *xt = cp.c; }
    triangle_closest(p1, t0, t1, t2, &cp); if (cp.d < best) { best = cp.d; *xs = p1; *xt = cp.c; }
    v3 T[3] = {t0, t1, t2};
    for (int k = 0; k < 3; ++k) {
        v3 y, xx;
        double d = segseg(T[k], T[(k + 1) % 3], p0, p1, &xx);   /* xx on p0 p1 */
        if (d < best) {
            best = d; *xs = xx;
            segment_closest(xx, T[k], T[(k + 1) % 3], &cp); *xt = cp.c;
        }
        (void)y;
    }
    return best;
}

/* closest point on the query primitive g (nv vertices) to data primitive
 * (class cls, index i) */
static v3 closest_on_query(const or_scene *sc, int cls, int64_t i, const v3 *g, int nv) {
    closest cp;
    if (nv == 1) return g[0];
    if (cls == 0) {
        v3 p = ld(sc->P + 3 * i);
        if (nv == 2) segment_closest(p, g[0], g[1], &cp);
        else triangle_closest(p, g[0], g[1], g[2], &cp);
        return cp.c;
    }
    if (cls == 1) {
        v3 a = ld(sc->E + 6 * i), b = ld(sc->E + 6 * i + 3), y, xs, xt;
        if (nv == 2) { segseg(a, b, g[0], g[1], &y); return y; }
        segtri(a, b, g[0], g[1], g[2], &xs, &xt);
        return xt;                                   /* point on the query triangle */
    }
    const float *t = sc->T + 9 * i;
    v3 t0 = ld(t), t1 = ld(t + 3), t2 = ld(t + 6), xs, xt;
    if (nv == 2) { segtri(g[0], g[1], t0, t1, t2, &xs, &xt); return xs; }
    /* triangle against triangle: a crossing edge gives distance 0; otherwise
     * the closest pair involves an edge of one of them */
    double best = INFINITY;
    v3 out = g[0];
    v3 G3[3] = {g[0], g[1], g[2]}, F3[3] = {t0, t1, t2};
    for (int k = 0; k < 3; ++k) {
        double d = segtri(G3[k], G3[(k + 1) % 3], t0, t1, t2, &xs, &xt);   /* xs on g */
        if (d < best) { best = d; out = xs; }
    }
    for (int k = 0; k < 3; ++k) {
        double d = segtri(F3[k], F3[(k + 1) % 3], g[0], g[1], g[2], &xs, &xt);   /* xt on g */
        if (d < best) { best = d; out = xt; }
    }
    return out;
}

static int load_query(const double *G, int nv, int64_t k, v3 *g) {
    for (int a = 0; a < nv; ++a) g[a] = ldd(G + 3 * (nv * k + a));
    return nv;
}

/* exact smooth distance for general query primitives (beta = 0 semantics) */
int or_brute_prims(const or_scene *sc, const or_params *p, int64_t nq, const double *G, int nv,
                   double *d_out, double *g_out, double *dmin_out) {
    if (!(p->alpha > 0) || nv < 1 || nv > 3) return -1;
#pragma omp parallel
    {
        termlist tl = {0, 0, 0};
#pragma omp for schedule(dynamic, 4)
        for (int64_t k = 0; k < nq; ++k) {
            v3 g[3];
            load_query(G, nv, k, g);
            double dmin = INFINITY;
            tl.n = 0;
            for (int64_t i = 0; i < sc->nP; ++i) exact_term(sc, p, 0, i, closest_on_query(sc, 0, i, g, nv), &tl, &dmin);
            for (int64_t i = 0; i < sc->nE; ++i) exact_term(sc, p, 1, i, closest_on_query(sc, 1, i, g, nv), &tl, &dmin);
            for (int64_t i = 0; i < sc->nT; ++i) exact_term(sc, p, 2, i, closest_on_query(sc, 2, i, g, nv), &tl, &dmin);
            lse_finish(&tl, p->alpha, d_out + k, g_out + 3 * k);
            if (dmin_out) dmin_out[k] = dmin;
        }
        free(tl.t);
    }
    return 0;
}

/* App. D for a general query primitive: the box is the intersection of six
 * halfspaces; along each axis g lies entirely above the box (min over its
 * vertices beyond max), entirely below, or neither.  The per-axis gaps
 * delta_a (signed, 0 for "neither") give D = |delta|, a lower bound of the
 * distance between the box and g (exact for a point, where delta = q - y_B),
 * and the far-field direction delta / D.  No outside halfspace: D = 0 and the
 * node is opened.  With cut_f32 the gaps, D^2 and the test are formed in FP32
 * as for points. */
static v3 query_gap(const float *b, const v3 *g, int nv) {
    double gp[3];
    for (int a = 0; a < 3; ++a) {
        double mn = INFINITY, mx = -INFINITY;
        for (int v = 0; v < nv; ++v) {
            double c = a == 0 ? g[v].x : (a == 1 ? g[v].y : g[v].z);
            if (c < mn) mn = c;
            if (c > mx) mx = c;
        }
        gp[a] = mn > b[3 + a] ? mn - b[3 + a] : (mx < b[a] ? mx - b[a] : 0.0);
    }
    return mk(gp[0], gp[1], gp[2]);
}

static int accept_far_query(const or_params *p, const float *b, const v3 *g, int nv, double D, double diam) {
    if (!p->cut_f32) return diam < p->beta * D;
    float gp[3];
    for (int a = 0; a < 3; ++a) {
        float mn = INFINITY, mx = -INFINITY;
        for (int v = 0; v < nv; ++v) {
            float c = (float)(a == 0 ? g[v].x : (a == 1 ? g[v].y : g[v].z));
            mn = fminf(mn, c);
            mx = fmaxf(mx, c);
        }
        gp[a] = mn > b[3 + a] ? mn - b[3 + a] : (mx < b[a] ? mx - b[a] : 0.0f);
    }
    float D2 = fmaf(gp[0], gp[0], fmaf(gp[1], gp[1], gp[2] * gp[2]));
    float ex = b[3] - b[0], ey = b[4] - b[1], ez = b[5] - b[2];
    float B2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
    float bf = (float)p->beta;
    return B2 < (bf * bf) * D2;
}

typedef struct {
    const or_scene *sc; const or_params *p; const v3 *g; int nv; int cls;
    const or_tree *tr; const int64_t *nleaf; double logA;
    termlist *tl; double margin; int64_t visited, far, leaves;
} bhq_ctx;

static void collect_q(bhq_ctx *cx, int32_t node) {
    const float *b = cx->tr->box + 6 * (int64_t)node;
    v3 lo = ld(b), hi = ld(b + 3);
    v3 gap = query_gap(b, cx->g, cx->nv);
    double D = norm(gap);
    double diam = norm(sub(hi, lo));
    cx->visited++;
    if (D > 0) {
        double m = fabs(cx->p->beta * D - diam) / D;
        if (m < cx->margin) cx->margin = m;
    }
    if (accept_far_query(cx->p, b, cx->g, cx->nv, D, diam)) {
        double logW = log((double)cx->nleaf[node]) + atten(cx->p) * cx->logA;
        push(cx->tl, logW - cx->p->alpha * D, scl(gap, 1.0 / D));
        cx->far++;
        return;
    }
    if (cx->tr->left[node] < 0) {
        double dm = INFINITY;
        int64_t i = cx->tr->prim[node];
        exact_term(cx->sc, cx->p, cx->cls, i, closest_on_query(cx->sc, cx->cls, i, cx->g, cx->nv), cx->tl, &dm);
        cx->leaves++;
        return;
    }
    collect_q(cx, cx->tr->left[node]);
    collect_q(cx, cx->tr->right[node]);
}

int or_barnes_hut_prims(const or_scene *sc, const or_params *p, const or_tree *trees, int64_t nq,
                        const double *G, int nv, double *d_out, double *g_out, double *stats) {
    if (!(p->alpha > 0) || !(p->beta >= 0) || nv < 1 || nv > 3) return -1;
    int64_t *nleaf[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        if (trees[c].n_nodes <= 0) continue;
        nleaf[c] = (int64_t *)calloc((size_t)trees[c].n_nodes, sizeof(int64_t));
        count_leaves(&trees[c], 0, nleaf[c]);
    }
    double logA[3] = {0.0, sc->logA_E, sc->logA_T};
#pragma omp parallel
    {
        termlist tl = {0, 0, 0};
#pragma omp for schedule(dynamic, 8)
        for (int64_t k = 0; k < nq; ++k) {
            v3 g[3];
            load_query(G, nv, k, g);
            tl.n = 0;
            bhq_ctx cx;
            memset(&cx, 0, sizeof cx);
            cx.sc = sc; cx.p = p; cx.g = g; cx.nv = nv; cx.tl = &tl; cx.margin = INFINITY;
            for (int c = 0; c < 3; ++c) {
                if (trees[c].n_nodes <= 0) continue;
                cx.cls = c; cx.tr = &trees[c]; cx.nleaf = nleaf[c]; cx.logA = logA[c];
                collect_q(&cx, 0);
            }
            lse_finish(&tl, p->alpha, d_out + k, g_out + 3 * k);
            if (stats) {
                stats[4 * k + 0] = cx.margin; stats[4 * k + 1] = (double)cx.visited;
                stats[4 * k + 2] = (double)cx.far; stats[4 * k + 3] = (double)cx.leaves;
            }
        }
        free(tl.t);
    }
    for (int c = 0; c < 3; ++c) free(nleaf[c]);
    return 0;
}

/* the closest pair of two simplices (for the pins): distance and the point
 * on the second; nva, nvb in 1..3 vertices, A and B as xyz rows */
int or_simplex_distance(const double *A, int nva, const double *B, int nvb, double *out) {
    v3 a[3], b[3];
    for (int k = 0; k < nva; ++k) a[k] = ldd(A + 3 * k);
    for (int k = 0; k < nvb; ++k) b[k] = ldd(B + 3 * k);
    v3 y = b[0], xs, xt;
    double d;
    closest cp;
    if (nva == 1) {
        if (nvb == 1) { d = norm(sub(a[0], b[0])); y = b[0]; }
        else if (nvb == 2) { segment_closest(a[0], b[0], b[1], &cp); d = cp.d; y = cp.c; }
        else { triangle_closest(a[0], b[0], b[1], b[2], &cp); d = cp.d; y = cp.c; }
    } else if (nva == 2) {
        if (nvb == 1) { segment_closest(b[0], a[0], a[1], &cp); d = cp.d; y = b[0]; }
        else if (nvb == 2) d = segseg(a[0], a[1], b[0], b[1], &y);
        else { d = segtri(a[0], a[1], b[0], b[1], b[2], &xs, &xt); y = xt; }
    } else {
        if (nvb == 1) { triangle_closest(b[0], a[0], a[1], a[2], &cp); d = cp.d; y = b[0]; }
        else if (nvb == 2) { d = segtri(b[0], b[1], a[0], a[1], a[2], &xs, &xt); y = xs; }
        else {
            d = INFINITY;
            for (int k = 0; k < 3; ++k) {
                double e = segtri(b[k], b[(k + 1) % 3], a[0], a[1], a[2], &xs, &xt);
                if (e < d) { d = e; y = xs; }
            }
            for (int k = 0; k < 3; ++k) {
                double e = segtri(a[k], a[(k + 1) % 3], b[0], b[1], b[2], &xs, &xt);
                if (e < d) { d = e; y = xt; }
            }
        }
    }
    out[0] = d; out[1] = y.x; out[2] = y.y; out[3] = y.z;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Rigidly moved queries x' = R_k x_j + t_k and the adjoint of d(x')          */
/* ------------------------------------------------------------------------ */
/* X: m x 3, R: K x 9 row-major, t: K x 3  ->  Qout: (K*m) x 3 (double) */
int or_rigid_apply(const float *X, int64_t m, const float *R, const float *t, int64_t K, double *Qout) {
    for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < m; ++j) {
            const float *r = R + 9 * k;
            double x = X[3 * j], y = X[3 * j + 1], z = X[3 * j + 2];
            double *o = Qout + 3 * (k * m + j);
            o[0] = r[0] * x + r[1] * y + r[2] * z + t[3 * k];
            o[1] = r[3] * x + r[4] * y + r[5] * z + t[3 * k + 1];
            o[2] = r[6] * x + r[7] * y + r[8] * z + t[3 * k + 2];
        }
    return 0;
}

/* With u_kj = gbar_kj * grad d(x'_kj):  tbar_k = sum_j u_kj,
 * Rbar_k = sum_j u_kj x_j^T,  xbar_j = sum_k R_k^T u_kj. */
int or_rigid_adjoint(const float *X, int64_t m, const float *R, int64_t K,
                     const double *gbar, const double *grad,
                     double *Rbar, double *tbar, double *Xbar) {
    memset(Rbar, 0, sizeof(double) * 9 * K);
    memset(tbar, 0, sizeof(double) * 3 * K);
    memset(Xbar, 0, sizeof(double) * 3 * m);
    for (int64_t k = 0; k < K; ++k)
        for (int64_t j = 0; j < m; ++j) {
            const double *g = grad + 3 * (k * m + j);
            double u[3] = {gbar[k * m + j] * g[0], gbar[k * m + j] * g[1], gbar[k * m + j] * g[2]};
            for (int a = 0; a < 3; ++a) {
                tbar[3 * k + a] += u[a];
                for (int b = 0; b < 3; ++b) Rbar[9 * k + 3 * a + b] += u[a] * X[3 * j + b];
            }
            for (int b = 0; b < 3; ++b)
                for (int a = 0; a < 3; ++a) Xbar[3 * j + b] += R[9 * k + 3 * a + b] * u[a];
        }
    return 0;
}
