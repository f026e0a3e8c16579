/*
 * sd.h — smooth distance to co-dimensional geometry on MI355X (gfx950).
 *
 * C ABI of libsd.so.  It evaluates, for many query points q, the weighted
 * LogSumExp smooth minimum distance of Madan & Levin, "Fast Evaluation of
 * Smooth Distance Constraints on Co-Dimensional Geometry":
 *
 *     d(q) = -(1/alpha) log sum_i w_i(q) exp(-alpha d_i(q))        (Sec. 3, Eq. 3)
 *
 * and its gradient (Eq. 4), over a data mesh of points, edges and triangles,
 * with the paper's blending weights w_i = (A w~_i)^S (Sec. 3.3, App. C) and its
 * conservative Barnes-Hut far field (Sec. 3.5, App. D, Alg. 1, Alg. 2).
 *
 * Precision: distances, closest points and barycentric coordinates are formed
 * in FP64 from the FP32 inputs, the weight polynomials evaluated in FP64, the
 * sums accumulated in FP64 and the result rounded once to FP32; directions,
 * weight gradients and exponentials are FP32.  Results are conservative,
 * d <= d_min, unless SD_NO_CONSERVATIVE_ROUNDING is given.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless the name ends in _host.
 *     Float arrays are FP32, row-major; index arrays are int32.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Evaluation calls are asynchronous on that stream; outputs are written
 *     into caller-allocated device memory.  sd_build_bvh synchronises the
 *     stream once before it returns.
 *   - Return value: SD_OK (0) or a negative error code; no C++ exception
 *     crosses the ABI.  sd_last_error() gives a message for the last failing
 *     call made on the calling thread.
 *   - A scene is read-only after sd_build_bvh; it may be evaluated from several
 *     host threads / streams at once.  Freeing it while evaluations are in
 *     flight is the caller's error.
 */
#ifndef SD_H
#define SD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SD_OK = 0,
    SD_EINVAL = -1,         /* bad argument (null pointer, size, index out of range, parameter) */
    SD_ENOMEM = -2,         /* device allocation failed                                          */
    SD_EHIP = -3,           /* a HIP runtime call failed                                         */
    SD_EUNSUPPORTED = -4    /* valid input the library does not handle (see the message)         */
};

/* sd_build_bvh flags */
#define SD_BUILD_A_PAPER_LITERAL 0x1u  /* triangle scale A_T = max_i v_i exactly as printed in
                                          App. C.3; the default raises it to the smallest value
                                          with A_T w~_i >= 1 everywhere (Sec. 3.3)              */

/* sd_params.flags */
#define SD_GRAD_PAPER_METRIC 0x1u   /* barycentric gradients in the alpha-scaled metric of Sec. 3.3
                                       (weight-gradient term divided by alpha once more); the
                                       default is the exact derivative of Eq. 3                 */
#define SD_ROOTLOG_F64       0x2u   /* accepted and without effect: the final logarithm of the
                                       accumulated sum (Alg. 2) is always taken in FP64        */
#define SD_NO_QUERY_SORT     0x4u   /* evaluate queries in input order (no Morton reordering)    */
#define SD_NO_CONSERVATIVE_ROUNDING 0x8u /* skip the final clamp that keeps d <= d_min in FP32:
                                       by default d is lowered to the smallest rigorous lower
                                       bound of a summed term's distance where it exceeds it
                                       (App. A, Sec. 3.5: d <= every term distance <= d_min);
                                       only results within rounding of that bound change     */
#define SD_NO_PRUNE          0x10u  /* visit every node Alg. 1 visits, even subtrees whose terms
                                       are all below exp(-64) of the running maximum (by default
                                       those are skipped when alpha x scene diagonal > 1000:
                                       they cannot change an FP32 result)                      */
#define SD_COUNTERS_BY_CLASS 0x20u  /* sd_eval_counters: exact leaf terms per primitive class   */
#define SD_LSE_COMPENSATED_F32 0x40u /* value + gradient of point queries (sd_eval_grad,
                                        sd_eval_grad_ordered, _noalloc): the running sums of Eq. 3-4
                                        in compensated FP32 (Neumaier; product errors by FMA)
                                        instead of FP64; log-terms stay FP64.  A compiled variant
                                        kept for comparison: on this GPU the FP64 sums are as fast
                                        and exact to FP64 rounding.  SD_EUNSUPPORTED elsewhere. */

typedef struct sd_params {
    float alpha;     /* accuracy / smoothness, > 0 (Eq. 3)                                   */
    float alpha_u;   /* attenuation threshold alpha_U >= 0; S = alpha / max(alpha, alpha_U)   */
    float beta;      /* Barnes-Hut opening parameter >= 0; 0 evaluates every primitive exactly */
    uint32_t flags;  /* SD_GRAD_PAPER_METRIC | SD_ROOTLOG_F64 | SD_NO_QUERY_SORT | ...        */
} sd_params;

typedef struct sd_scene sd_scene;

typedef struct sd_scene_info {
    int64_t n_prims[3];     /* points, edges, triangles                                     */
    int64_t n_nodes[3];     /* hierarchy nodes per class (2 n - 1, or 0)                    */
    double A[3];            /* global weight scale per class (points: 1)                    */
    double A_T_literal;     /* max_i v_i over the triangles (App. C.3 as printed)           */
    double diam_max;        /* largest primitive bounding-box diagonal (rounding margin)    */
    int64_t device_bytes;   /* device memory owned by the scene                             */
    int32_t n_tri_classes;  /* distinct (v, e) triangle valence pairs                       */
    int32_t pad;
} sd_scene_info;

/*
 * Build the evaluation structure for the data mesh M_d = (V, F) (Sec. 3).
 *
 *   V   nV x 3 vertex coordinates.
 *   P   nP vertex ids used as point primitives (Sec. 3.1).  P == NULL with nP < 0
 *       makes every vertex a point (F omitted for point clouds, Sec. 3).
 *   E   nE x 2 vertex ids per edge;  T  nT x 3 vertex ids per triangle.  The
 *       given vertex order is kept: barycentrics are measured from E[i][0] and
 *       T[i][0] (App. B).  Any count may be 0 (its pointer may then be NULL).
 *
 * Valences for the weights (App. C) are counted within each class: edges per
 * vertex among E; triangles per vertex and per edge among T.  One linear BVH
 * (Morton order, one primitive per leaf) is built per non-empty class.
 * Inputs are copied; the caller may free them once the call returns.
 * Errors: SD_EINVAL for negative sizes, null pointers with a positive count or
 * indices outside [0, nV); SD_EUNSUPPORTED for a triangle valence above 1023
 * or more than 2^26 primitives in one class.
 */
int sd_build_bvh(const float *V, int64_t nV,
                 const int32_t *P, int64_t nP,
                 const int32_t *E, int64_t nE,
                 const int32_t *T, int64_t nT,
                 uint32_t flags, void *stream, sd_scene **out);

/* Release a scene and its device memory.  NULL is ignored. */
int sd_free_scene(sd_scene *scene);

/* Sizes and weight scales of a built scene (host struct, filled
 * synchronously without device work).  SD_EINVAL for NULL arguments. */
int sd_scene_info_get(const sd_scene *scene, sd_scene_info *out_host);

/*
 * Smooth distance value (Eq. 3) with the Barnes-Hut traversal of Alg. 1 and the
 * finalisation of Alg. 2, for nQ queries Q (nQ x 3).  d_out: nQ values.
 * An empty scene gives +inf.  Errors: SD_EINVAL for alpha <= 0, beta < 0,
 * alpha_u < 0, nQ < 0 or null pointers with nQ > 0.
 */
int sd_eval(const sd_scene *scene, const float *Q, int64_t nQ, const sd_params *params,
            float *d_out, void *stream);

/* As sd_eval, plus the gradient (Eq. 4) with respect to each query, grad_out
 * nQ x 3.  Alg. 2's epsilon is not needed: the running sum is at least 1. */
int sd_eval_grad(const sd_scene *scene, const float *Q, int64_t nQ, const sd_params *params,
                 float *d_out, float *grad_out, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sd_eval_grad
 * with the same arguments and the same results, bit for bit, that allocates
 * nothing.  The query ordering's scratch (Morton keys and radix-sort buffers,
 * about 24 bytes per query) lives in a static device array inside the library:
 * every GPU the library runs on holds one copy (28 MiB) from the first call on
 * that GPU until the process ends.  Limit: nQ <= SD_NOALLOC_MAX_QUERIES per
 * call (SD_EINVAL above it; split larger batches).  All calls on one GPU share
 * that GPU's array: calls that overlap in time on one GPU (different streams
 * or host threads without ordering between them) race and must not be made.
 * Inputs, outputs and errors as sd_eval_grad.
 */
#define SD_NOALLOC_MAX_QUERIES (1 << 20)
int sd_eval_grad_noalloc(const sd_scene *scene, const float *Q, int64_t nQ, const sd_params *params,
                         float *d_out, float *grad_out, void *stream);

/*
 * Query ordering for coherent traversal: perm_out (nQ uint32) receives the
 * query indices sorted by 30-bit Morton code in the scene box enlarged by half
 * its extent on each side (a stable radix sort; ties keep input order).
 * sd_eval / sd_eval_grad do this internally for nQ >= 4096 unless
 * SD_NO_QUERY_SORT is set; it is exposed so that a caller can order once and
 * evaluate many times, or time the two stages separately.
 */
int sd_query_order(const sd_scene *scene, const float *Q, int64_t nQ, uint32_t *perm_out,
                   void *stream);

/* sd_eval_grad evaluating the queries in the order perm (a permutation of
 * 0..nQ-1 from sd_query_order, or NULL for input order); results are still
 * written at each query's own index.  Entries of perm >= nQ are skipped (their
 * slot is evaluated by no lane); a perm that is not a permutation leaves the
 * outputs of the missing indices unwritten. */
int sd_eval_grad_ordered(const sd_scene *scene, const float *Q, const uint32_t *perm, int64_t nQ,
                         const sd_params *params, float *d_out, float *grad_out, void *stream);

/* Exact evaluation (beta = 0 semantics) by a tiled all-pairs sweep over every
 * primitive instead of the hierarchy; grad_out may be NULL. */
int sd_eval_brute(const sd_scene *scene, const float *Q, int64_t nQ, const sd_params *params,
                  float *d_out, float *grad_out, void *stream);

/* Per-query work counters of the Barnes-Hut traversal: counts_out nQ x 3 int32
 * = (nodes visited, far-field terms, exact leaf terms); with
 * SD_COUNTERS_BY_CLASS in params->flags, nQ x 5 = (nodes visited, far-field
 * terms, exact point, edge and triangle leaf terms). */
int sd_eval_counters(const sd_scene *scene, const float *Q, int64_t nQ, const sd_params *params,
                     int32_t *counts_out, void *stream);

/*
 * Copy one class's hierarchy to host memory (for reference checks).
 * cls: 0 points, 1 edges, 2 triangles.  Arrays sized by n_nodes[cls]:
 *   box_host   n x 6 (min xyz, max xyz)
 *   left_host, right_host   child node ids, -1 at leaves
 *   prim_host  original primitive id at leaves, -1 at internal nodes
 * Node 0 is the root.  Synchronises the stream.
 */
int sd_export_bvh(const sd_scene *scene, int cls, float *box_host, int32_t *left_host,
                  int32_t *right_host, int32_t *prim_host, void *stream);

/* Weight data of one class in original primitive order, to host:
 *   edges:     wt_host nE x 2 = (1/|N_i0|, 1/|N_i1|)                      (App. C.2)
 *   triangles: wt_host nT x 3 = (1/v_i, 1/e_i, (v_i - 1)/v_i), or (1,1,1)
 *              for an isolated triangle (v_i = 1)                          (App. C.3) */
int sd_export_weights(const sd_scene *scene, int cls, float *wt_host, void *stream);

/* The universal triangle weight bases (App. C.3): w~ = (1/v) B_V + (1/e) B_E +
 * ((v-1)/v) B_C with each basis a degree-7 polynomial in (phi1, phi2);
 * coef_host receives 3 x 64 doubles, entry [k][a*8+b] multiplying phi1^a phi2^b. */
int sd_triangle_weight_basis(double *coef_host);

/*
 * Rigidly moved queries (the paper's rigid-body degrees of freedom, Sec. 4.5):
 *   Q_out[k*m + j] = R_k X_j + t_k,   X m x 3, R K x 9 (row-major 3x3), t K x 3,
 *   Q_out (K*m) x 3.
 */
int sd_rigid_transform(const float *X, int64_t m, const float *R, const float *t, int64_t K,
                       float *Q_out, void *stream);

/*
 * Adjoint of L(R, t, X) given upstream gbar = dL/dd (K x m) and the smooth
 * distance gradients grad (K*m x 3, from sd_eval_grad on sd_rigid_transform's
 * output): with u_kj = gbar_kj grad_kj,
 *   tbar_k = sum_j u_kj,   Rbar_k = sum_j u_kj X_j^T  (K x 9),
 *   Xbar_j = sum_k R_k^T u_kj (m x 3; Xbar may be NULL).
 * Deterministic (no atomics).
 */
int sd_rigid_adjoint(const float *X, int64_t m, const float *R, int64_t K,
                     const float *gbar, const float *grad,
                     float *Rbar, float *tbar, float *Xbar, void *stream);

/*
 * The same adjoint for the query-mesh distances D_k of the K rigidly moved
 * copies of the m points (Sec. 3.6, Eq. 6-8, with the rigid degrees of freedom
 * of Sec. 4.5): gbar_kj = w_kj * Dbar_k is formed inside the kernels from
 * w = dD_k/dd_kj (K x m, the weights of sd_query_mesh_lse) and the upstream
 * Dbar = dL/dD_k (K), all device memory.  Same outputs, layout and
 * determinism as sd_rigid_adjoint; SD_EINVAL for a null Dbar when K > 0.
 */
int sd_rigid_qmesh_adjoint(const float *X, int64_t m, const float *R, int64_t K, const float *w,
                           const float *Dbar, const float *grad, float *Rbar, float *tbar, float *Xbar,
                           void *stream);

/*
 * Value and gradient for query primitives that are edges or triangles
 * (Sec. 3.4): G is n x nv x 3 (nv = 2: edges, 3: triangles; 1: points, the
 * same as sd_eval_grad), device memory.  d(f_i, g) is the simplex-simplex
 * distance of App. B (Eq. 10); each data primitive's term is the point-query
 * term at the point g(lambda) of g closest to it (weights at the closest
 * point on f_i), so grad_out is the derivative for a rigid translation of g
 * in that reading.  Far-field boxes use the per-axis gaps of the box
 * halfspaces that g lies outside of (App. D): a lower bound of the box
 * distance (the far field stays conservative), equal to the point formula
 * for a point; no such halfspace opens the node.  Intersecting primitives
 * give distance 0 with the weight at one point of the intersection.
 * Errors: SD_EINVAL for a null scene or pointers, n < 0, nv outside 1..3,
 * bad p (as sd_eval).
 */
int sd_eval_grad_prims(const sd_scene *scene, const float *G, int32_t nv, int64_t n, const sd_params *p,
                       float *d_out, float *grad_out, void *stream);

/*
 * Sphere tracing of the level set d = level of the smooth distance (Sec. 4.2
 * renders the zero isosurface this way; Hart 1996): for each ray i with
 * origin O_i and unit direction U_i (n x 3 each), x = O_i + t U_i starts at
 * t = 0 and advances by r = d(x) - level (Eq. 3 through Alg. 1 / Alg. 2 with
 * the parameters p, value only) until r <= eps: t_out[i] = t (a hit);
 * t > t_max, max_steps evaluations or a NaN distance: t_out[i] = +inf.
 * steps_out (may be NULL) receives the number of evaluations per ray.  A step
 * of r is safe where d is 1-Lipschitz (point clouds; the blended weights of
 * edges and triangles can raise |grad d| slightly above 1).  All arrays are
 * device memory; the march runs inside one kernel.
 * Errors: SD_EINVAL for a null scene or pointers, n < 0, bad p (as sd_eval),
 * eps <= 0, t_max < 0, a non-finite level or max_steps < 1.
 */
int sd_sphere_trace(const sd_scene *scene, const float *O, const float *U, int64_t n,
                    const sd_params *p, float level, float eps, float t_max, int32_t max_steps,
                    float *t_out, int32_t *steps_out, void *stream);

/*
 * Smooth distance between the data mesh and a query mesh (Sec. 3.6), for K
 * instances of one query mesh (e.g. K rigid placements of a body): from the
 * per-primitive smooth distances d (K x m, row k = instance k, as computed by
 * sd_eval_grad for the instance's query primitives) and their gradients grad
 * (K x m x 3),
 *   D_k = -(1/alpha_q) log sum_j exp(-alpha_q d_kj)                  (Eq. 6),
 *   w_kj = dD_k/dd_kj = exp(-alpha_q d_kj) / sum_j exp(-alpha_q d_kj),
 *   vgrad_kv = sum over primitives g_j containing vertex v of
 *              w_kj / (n(g_j) + 1) grad_kj                         (Eq. 7, Eq. 8):
 * each exponential is split equally between the n(g_j) + 1 vertices of its
 * primitive, whose gradient moves it rigidly.
 * prim: m x 3 int32 vertex ids per query primitive (-1 for unused corners: a
 * point has one vertex, an edge two, a triangle three), ids in [0, nV); or
 * NULL when primitive j is vertex j (a point query mesh; nV is then m).
 * All arrays are device memory.  Outputs: D (K), w (K x m, may be NULL),
 * vgrad (K x nV x 3, may be NULL; grad may be NULL when vgrad is).
 * The largest term is factored out and the sum is formed in FP64 in a fixed
 * order (D and w bitwise reproducible); vertex gradients of a general query
 * mesh are added with atomics (summation order not fixed).  An instance with
 * m = 0 or every d = +inf gives D = +inf, w = 0, vgrad = 0; a NaN distance
 * makes its instance NaN.
 * Errors: SD_EINVAL for alpha_q <= 0 or not finite, negative sizes, null
 * pointers, primitive ids outside [0, nV) or a primitive without vertices
 * (checked on the device; the call then synchronises the stream);
 * SD_EUNSUPPORTED for K > 65535 or m > 2^28.
 */
int sd_query_mesh_lse(const float *d, const float *grad, int64_t K, int64_t m,
                      const int32_t *prim, int64_t nV, float alpha_q,
                      float *D, float *w, float *vgrad, void *stream);

/*
 * Learned surrogate of the smooth distance.  The paper has no learned part:
 * this network approximates d of Eq. 3 for one scene and one (alpha, alpha_u,
 * beta, flags) setting, is trained on values the exact evaluation produces,
 * and hands queries near the zero isosurface back to the exact Barnes-Hut
 * evaluation (Alg. 1, Alg. 2).
 *
 * Architecture (fixed):
 *   gamma(x) = [sin(2 pi B x), cos(2 pi B x)]     B: 64 x 3 (row-major)
 *   z_l = W_l a_{l-1} + b_l,  a_l = z_l / (1 + exp(-z_l)),  l = 1..4, width 256
 *   y = w5 . a_4 + b5
 * Parameters: SD_SURR_N_PARAMS FP32 values, in this order (matrices out x in,
 * row-major): W1 (256 x 128), b1, W2 (256 x 256), b2, W3, b3, W4, b4, w5 (256),
 * b5.  The FP32 values are the master copy trained by Adam; evaluation and
 * training products use W1..W4 and w5 rounded to BF16 (nearest even) on the
 * matrix cores with FP32 accumulation; biases stay FP32.
 *
 * A handle owns its device buffers (master weights, Adam moments, packed BF16
 * weights, a training workspace for max_batch rows).  Calls on one handle
 * must not overlap (training mutates it); sd_surrogate_forward and
 * sd_eval_surrogate only read it.
 */
#define SD_SURR_N_FREQ 64
#define SD_SURR_WIDTH 256
#define SD_SURR_DEPTH 4
#define SD_SURR_N_PARAMS 230657

typedef struct sd_surrogate sd_surrogate;

/* B_host: 64 x 3 frequencies; theta_host: initial parameters (both host, FP32,
 * copied).  max_batch: largest training batch, a multiple of 64 (0 = inference
 * only).  Adam moments start at zero, step 0, certified margin +inf.
 * Synchronises `stream` once.  SD_ENOMEM when the workspace does not fit. */
int sd_surrogate_create(const float *B_host, const float *theta_host, int64_t max_batch,
                        void *stream, sd_surrogate **out);
/* Release a surrogate handle and its device memory.  NULL is ignored. */
int sd_surrogate_free(sd_surrogate *sur);

/* Surrogate value d_out (nQ) and, when grad_out is not NULL, its gradient in x
 * (nQ x 3), for the queries Q (nQ x 3).  Asynchronous. */
int sd_surrogate_forward(const sd_surrogate *sur, const float *Q, int64_t nQ, float *d_out,
                         float *grad_out, void *stream);

/* Mean squared error L = mean_b (y(x_b) - label_b)^2 over one batch and its
 * gradient dL/dtheta (SD_SURR_N_PARAMS FP32, device) with the batch rows
 * x_b = X[idx[b]], label_b = labels[idx[b]] (idx NULL: rows 0..n-1).  X holds
 * n_rows x 3 values and labels n_rows; an index outside [0, n_rows) makes the
 * loss and gradient NaN.  n is a positive multiple of 64, at most max_batch.
 * grad_out / loss_out (device, may be NULL) receive copies.  Asynchronous. */
int sd_surrogate_loss_grad(sd_surrogate *sur, const float *X, const float *labels, int64_t n_rows,
                           const int32_t *idx, int64_t n, float *grad_out, float *loss_out,
                           void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments) on
 * the master weights with the gradient grad (device; NULL = the handle's last
 * sd_surrogate_loss_grad result) and learning rate lr >= 0; then refreshes
 * the BF16 copies.  Asynchronous. */
int sd_surrogate_adam(sd_surrogate *sur, const float *grad, float lr, void *stream);

/* sd_surrogate_loss_grad followed by sd_surrogate_adam.  Asynchronous. */
int sd_surrogate_train_step(sd_surrogate *sur, const float *X, const float *labels, int64_t n_rows,
                            const int32_t *idx, int64_t n, float lr, float *loss_out,
                            void *stream);

/* Certified margin: eps = safety * max_i |y(X_i) - labels_i| over a held-out
 * set (n rows, device), stored in the handle and returned in *eps_host.
 * safety >= 1.  Synchronises `stream`. */
int sd_surrogate_certify(sd_surrogate *sur, const float *X, const float *labels, int64_t n,
                         float safety, void *stream, float *eps_host);

/* Local certificate: as sd_surrogate_certify (which it runs first, setting the
 * global margin), plus a grid of grid^3 cells over the box [lo_host, hi_host]
 * (host, 3 floats each): the margin of a cell is safety x the largest error of
 * the held-out samples in the cell and its 26 neighbours (the global margin
 * when there is none).  sd_eval_surrogate then routes a query inside the box
 * when |y| < band + margin of its cell, outside the box with the global
 * margin.  A cell whose margin exceeds max_margin (> 0; +inf for no limit)
 * sends every query in it to the exact evaluation, so that the error of the
 * answers left to the network stays within max_margin (empirically).
 * sd_surrogate_certify and sd_surrogate_load drop the grid.  grid in
 * [1, 256].  Synchronises `stream`. */
int sd_surrogate_certify_cells(sd_surrogate *sur, const float *X, const float *labels, int64_t n,
                               float safety, int grid, const float *lo_host, const float *hi_host,
                               float max_margin, void *stream, float *eps_host);

/* Host copies of the state (every output may be NULL): master parameters,
 * Adam moments (SD_SURR_N_PARAMS each), frequencies (64 x 3), step count,
 * certified margin.  Synchronous (device-wide). */
int sd_surrogate_save(const sd_surrogate *sur, float *theta_host, float *m_host, float *v_host,
                      float *B_host, int64_t *step_host, float *eps_host);

/* Replace the master parameters (and the Adam moments, zero when NULL), step
 * count and certified margin from host arrays. */
int sd_surrogate_load(sd_surrogate *sur, const float *theta_host, const float *m_host,
                      const float *v_host, int64_t step, float eps_cert, void *stream);

/* Smooth distance and gradient with the surrogate where it is certified:
 * every query gets the surrogate value y and gradient; the queries with
 * |y| < band + eps_cert (the certified margin of sd_surrogate_certify; after
 * sd_surrogate_certify_cells, band + the margin of the query's cell) are then
 * evaluated exactly (sd_eval_grad semantics with `params`, in Morton order
 * unless SD_NO_QUERY_SORT) and overwritten.  routed (nQ bytes, may be
 * NULL) receives 1 for those queries.  *n_fallback (device, one uint32; may
 * be NULL) receives their number.  The surrogate must have been trained for
 * this scene and params.  Asynchronous: the number of routed queries stays on
 * the device, where the compaction, the Morton order and the exact pass read
 * it (their launches are sized for nQ; waves beyond the count exit at once),
 * so the call never waits for the GPU. */
int sd_eval_surrogate(const sd_scene *scene, const sd_surrogate *sur, const float *Q, int64_t nQ,
                      const sd_params *params, float band, float *d_out, float *grad_out,
                      uint8_t *routed, uint32_t *n_fallback, void *stream);

/* Device memory budget of the library (all devices together; default: none).
 * Every device allocation of the library (scene hierarchies, surrogate state,
 * the stream-ordered scratch of a call) that would take the bytes it holds
 * above `bytes` fails with SD_ENOMEM, as a failed device allocation does; the
 * call that made it releases everything it had taken and returns SD_ENOMEM.
 * bytes < 0 removes the budget.  The static array of sd_eval_grad_noalloc is
 * not counted.  Callers: services that share a GPU and must bound the
 * library's footprint, and tests of the out-of-memory paths. */
int sd_set_memory_budget(int64_t bytes);

/* Device bytes the library holds now: scenes, surrogates, and the scratch of
 * calls whose release has not been enqueued yet (scratch is returned to the
 * stream's pool in stream order when its call returns). */
int sd_memory_in_use(int64_t *bytes_out);

/* Message of the last failed call on this thread (thread-local storage owned
 * by the library; valid until the next failing call on the thread). */
const char *sd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SD_H */
