// Internal declarations shared by the HIP translation units of libsd.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/sd.h"

namespace sd {
// fractional bits of the fixed-point log n_B in a node's payload
constexpr int kLogFracBits = 26;
}  // namespace sd

namespace sd {

// ---------------------------------------------------------------------------
// Error plumbing: every ABI entry point returns a code and records a message.
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

#define SD_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t _e = (call);                                                       \
        if (_e != hipSuccess)                                                         \
            return ::sd::fail(_e == hipErrorOutOfMemory ? SD_ENOMEM : SD_EHIP,        \
                              std::string(#call) + ": " + hipGetErrorString(_e));     \
    } while (0)

// ---------------------------------------------------------------------------
// Device memory: every allocation of the library goes through these, which
// keep the bytes it holds and enforce the optional budget
// (sd_set_memory_budget).  A refused or failed allocation returns SD_ENOMEM
// and leaves *p null.
// ---------------------------------------------------------------------------
int dev_malloc(void **p, size_t bytes, const char *what);
int dev_malloc_async(void **p, size_t bytes, hipStream_t s, const char *what);
void dev_free(void *p);
void dev_free_async(void *p, hipStream_t s);

#define SD_TRY(expr)                        \
    do {                                    \
        int _rc = (expr);                   \
        if (_rc != SD_OK) return _rc;       \
    } while (0)

// Stream-ordered scratch of one call: every allocation made through it is
// released with hipFreeAsync on the same stream when it goes out of scope,
// after the work enqueued before that point, on the normal path and on every
// early error return alike.
class AsyncScratch {
  public:
    explicit AsyncScratch(hipStream_t s) : s_(s) {}
    AsyncScratch(const AsyncScratch &) = delete;
    AsyncScratch &operator=(const AsyncScratch &) = delete;
    ~AsyncScratch() {
        for (size_t k = n_; k-- > 0;) dev_free_async(ptr_[k], s_);
    }
    // count elements of T (at least one); SD_ENOMEM / SD_EHIP on failure
    template <class T>
    int alloc(T **p, int64_t count) {
        *p = nullptr;
        if (n_ == kMax) return fail(SD_EHIP, "AsyncScratch: too many buffers");
        size_t bytes = (size_t)(count > 1 ? count : 1) * sizeof(T);
        int rc = dev_malloc_async((void **)p, bytes, s_, "scratch");
        if (rc != SD_OK) return rc;
        ptr_[n_++] = (void *)*p;
        return SD_OK;
    }

  private:
    static constexpr size_t kMax = 24;
    hipStream_t s_;
    void *ptr_[kMax] = {};
    size_t n_ = 0;
};

// ---------------------------------------------------------------------------
// Device layout of one class hierarchy (depth-first order, escape indices).
//
//   node_lo[i] = (min.x, min.y, min.z, bits: escape index, -1 = end)
//   node_hi[i] = (max.x, max.y, max.z, payload)
//   payload: internal node -> int log(n_B) * 2^kLogFracBits, rounded to nearest
//            (n_B = leaves below; non-negative);
//            leaf           -> int bits 0x80000000 | leaf slot.
//   The left child of internal node i is i + 1; its right child is the left
//   child's escape index.
//
// Leaf records (leaf slot k = k-th leaf in depth-first order):
//   points:    1 x float4 (p.xyz, 1) for the all-pairs kernel; the traversal
//              takes the point from its leaf's box
//   edges:     2 x float4 (v0.xyz, 1/N0), (v1.xyz, 1/N1)
//   triangles: 3 x float4 (v0.xyz, iv), (v1.xyz, ie), (v2.xyz, ic)
// ---------------------------------------------------------------------------
struct TreeView {
    const float4 *lo;
    const float4 *hi;
    const float4 *leaf;   // edges / triangles only
    int32_t n_nodes;
    float lwmax;          // bound on the log-weight of any term of the class
    double slogA;         // S log A of the class, filled per evaluation
};

struct EvalArgs {
    TreeView tree[3];
    // Triangle weights (App. C.3) as the 36 FP64 monomial coefficients of
    // each valence class in Horner order (see triangle_monomial_horner).
    const double *tri_table;  // n_classes x 36 (class id in the leaf record)
    int32_t tri_uniform;      // 1: a single class (row 0), read with scalar loads
    float alpha, inv_alpha, beta2, S;
    double alpha64, inv_alpha64;
    int32_t clamp;        // 1: result clamped to a lower bound of the smallest term distance (default)
    int32_t defer;        // 1: wave-cooperative leaf stage, 0: leaves evaluated inline
    float prune;          // skip subtrees whose terms are below exp(-prune) of the reference
    uint32_t flags;
    int32_t nq;            // number of queries (bound of the entries of perm)
    int32_t nthr;          // number of threads: perm entries (nq without perm)
    const uint32_t *nthr_dev = nullptr;  // optional device count: min(nthr, *nthr_dev) threads work
    const float *Q;
    const uint32_t *perm;  // optional query order (nullptr = identity)
    float *d_out;
    float *g_out;          // nullptr for value only
    int32_t *counts;       // nullptr unless counting
};

// Host-side weight constants (weights.cpp)
int triangle_basis_f64(double out[3][64]);
double triangle_weight_min_f64(int v, int e);   // min over the barycentric triangle
void triangle_bernstein(int v, int e, float out[36]);
// monomial coefficients c_ab of w~ for (v, e) in Horner order: a = 7 .. 0,
// and for each a, b = 7 - a .. 0 (w~ = 1 for v <= 1)
void triangle_monomial_horner(int v, int e, double out[36]);

// Sorting and scans (sort.hip)
size_t radix_sort_temp_bytes(int64_t n);
// Stable ascending sort of (key, val) pairs by the low `bits` bits of key.
// With n_dev, the first min(n, *n_dev) pairs are sorted (the count read on the
// device; n sizes the launches and the scratch).
int radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_tmp, uint32_t *vals_tmp,
                     int64_t n, int bits, void *temp, hipStream_t s, const uint32_t *n_dev = nullptr);
int exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, void *temp,
                       hipStream_t s);

}  // namespace sd

// Opaque scene handle
struct sd_scene {
    int64_t n[3] = {0, 0, 0};
    int64_t n_nodes[3] = {0, 0, 0};
    float4 *lo[3] = {nullptr, nullptr, nullptr};
    float4 *hi[3] = {nullptr, nullptr, nullptr};
    float4 *leaf[3] = {nullptr, nullptr, nullptr};
    int32_t *prim_id[3] = {nullptr, nullptr, nullptr};   // leaf slot -> original id
    float *wt[3] = {nullptr, nullptr, nullptr};          // original order weight data
    double A[3] = {1.0, 1.0, 1.0};
    double A_T_literal = 1.0;
    double diam_max = 0.0;
    float box[6] = {0, 0, 0, 0, 0, 0};                    // union of class boxes
    int32_t n_tri_classes = 0;
    double *tri_table = nullptr;                          // n_tri_classes x 36 monomial coefs (Horner order)
    double tri_mono0[36];                                 // host copy of class 0
    double tri_wmax = 1.0;                                // largest Bernstein coefficient
    int64_t device_bytes = 0;
    int device = 0;
};

namespace sd {
// Query Morton ordering used by the evaluation (eval.hip)
// With idx, only the queries idx[0..nq) are ordered (perm gets those indices);
// with n_dev as well, only idx[0..min(nq, *n_dev)) (a count on the device).
int query_order(const sd_scene *sc, const float *Q, int64_t nq, uint32_t *perm, hipStream_t s,
                const uint32_t *idx = nullptr, const uint32_t *n_dev = nullptr);
// value + gradient with the query order's scratch in a static device array
// (no allocation; at most SD_NOALLOC_MAX_QUERIES queries) (eval.hip)
int eval_grad_noalloc(const sd_scene *sc, const float *Q, int64_t nq, const sd_params *p, float *d_out,
                      float *g_out, hipStream_t s);
// nthr >= 0 with perm_in: nthr threads evaluate the queries perm_in[0..nthr)
// out of nq; results land at the original query indices.  With nthr_dev as
// well, the launch is sized for nthr and min(nthr, *nthr_dev) threads work.
// value + gradient for edge (nv = 2) or triangle (nv = 3) query primitives (eval.hip)
int evalq_dispatch(const sd_scene *sc, const float *G, int nv, int64_t n, const sd_params *p, float *d_out,
                   float *g_out, hipStream_t s);
// sphere tracing of the level set d = level along rays (O, U) (eval.hip)
int trace_dispatch(const sd_scene *sc, const float *O, const float *U, int64_t n, const sd_params *p,
                   float level, float eps, float t_max, int32_t max_steps, float *t_out, int32_t *steps_out,
                   hipStream_t s);
int eval_dispatch(const sd_scene *sc, const float *Q, const uint32_t *perm_in, int64_t nq,
                  const sd_params *p, float *d_out, float *g_out, int32_t *counts, bool brute,
                  hipStream_t s, int64_t nthr = -1, const uint32_t *nthr_dev = nullptr);
}  // namespace sd
