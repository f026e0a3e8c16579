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
#define SD_ROOTLOG_F64       0x2u   /* final logarithm of the accumulated sum in FP64 (Alg. 2)   */
#define SD_NO_QUERY_SORT     0x4u   /* evaluate queries in input order (no Morton reordering)    */
#define SD_NO_CONSERVATIVE_ROUNDING 0x8u /* skip the downward rounding of terms and result     */
#define SD_NO_PRUNE          0x10u  /* visit every node Alg. 1 visits, even subtrees whose terms
                                       are all below exp(-64) of the running maximum (by default
                                       those are skipped: they cannot change an FP32 result)   */

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
 * indices outside [0, nV); SD_EUNSUPPORTED for a triangle valence above 1023.
 */
int sd_build_bvh(const float *V, int64_t nV,
                 const int32_t *P, int64_t nP,
                 const int32_t *E, int64_t nE,
                 const int32_t *T, int64_t nT,
                 uint32_t flags, void *stream, sd_scene **out);

/* Release a scene and its device memory.  NULL is ignored. */
int sd_free_scene(sd_scene *scene);

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
 * = (nodes visited, far-field terms, exact leaf terms). */
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

const char *sd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SD_H */
