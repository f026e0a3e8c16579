// C ABI entry points: argument checks, scene lifetime, error reporting.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "sd_internal.h"

namespace sd {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

// ---------------------------------------------------------------------------
// Device memory accounting: the bytes of every live allocation, their sum and
// the budget, under one lock (allocations are few per call).
// ---------------------------------------------------------------------------
namespace {
std::mutex g_mem_mu;
std::unordered_map<void *, size_t> g_mem_live;
int64_t g_mem_in_use = 0;
int64_t g_mem_budget = -1;   // < 0: none

int mem_admit(size_t bytes, const char *what) {
    if (g_mem_budget >= 0 && g_mem_in_use + (int64_t)bytes > g_mem_budget)
        return fail(SD_ENOMEM, std::string(what) + ": " + std::to_string(bytes) +
                                   " bytes would exceed the device memory budget of " +
                                   std::to_string(g_mem_budget) + " bytes (" + std::to_string(g_mem_in_use) +
                                   " in use)");
    return SD_OK;
}

int mem_failed(hipError_t e, size_t bytes, const char *what) {
    return fail(e == hipErrorOutOfMemory ? SD_ENOMEM : SD_EHIP,
                std::string(what) + ": device allocation of " + std::to_string(bytes) + " bytes: " +
                    hipGetErrorString(e));
}

void mem_record(void *p, size_t bytes) {
    g_mem_live[p] = bytes;
    g_mem_in_use += (int64_t)bytes;
}

void mem_forget(void *p) {
    auto it = g_mem_live.find(p);
    if (it == g_mem_live.end()) return;
    g_mem_in_use -= (int64_t)it->second;
    g_mem_live.erase(it);
}
}  // namespace

int dev_malloc(void **p, size_t bytes, const char *what) {
    *p = nullptr;
    std::lock_guard<std::mutex> lock(g_mem_mu);
    SD_TRY(mem_admit(bytes, what));
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return mem_failed(e, bytes, what);
    }
    mem_record(*p, bytes);
    return SD_OK;
}

int dev_malloc_async(void **p, size_t bytes, hipStream_t s, const char *what) {
    *p = nullptr;
    std::lock_guard<std::mutex> lock(g_mem_mu);
    SD_TRY(mem_admit(bytes, what));
    hipError_t e = hipMallocAsync(p, bytes, s);
    if (e != hipSuccess) {
        *p = nullptr;
        return mem_failed(e, bytes, what);
    }
    mem_record(*p, bytes);
    return SD_OK;
}

void dev_free(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_mem_mu);
    mem_forget(p);
    (void)hipFree(p);
}

void dev_free_async(void *p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> lock(g_mem_mu);
    mem_forget(p);
    (void)hipFreeAsync(p, s);
}

int build_scene(sd_scene *sc, const float *V, int64_t nV, const int32_t *P, int64_t nP,
                const int32_t *E, int64_t nE, const int32_t *T, int64_t nT, uint32_t flags,
                hipStream_t s);

static int check_params(const sd_params *p, const char *who) {
    if (!p) return fail(SD_EINVAL, std::string(who) + ": null params");
    if (!(p->alpha > 0.f) || !isfinite(p->alpha))
        return fail(SD_EINVAL, std::string(who) + ": alpha must be finite and > 0");
    if (!(p->beta >= 0.f) || !isfinite(p->beta))
        return fail(SD_EINVAL, std::string(who) + ": beta must be finite and >= 0");
    if (!(p->alpha_u >= 0.f) || !isfinite(p->alpha_u))
        return fail(SD_EINVAL, std::string(who) + ": alpha_u must be finite and >= 0");
    return SD_OK;
}

static int check_eval(const sd_scene *sc, const float *Q, int64_t nq, const sd_params *p,
                      const void *out, const char *who) {
    if (!sc) return fail(SD_EINVAL, std::string(who) + ": null scene");
    if (nq < 0) return fail(SD_EINVAL, std::string(who) + ": nQ < 0");
    if (nq > 0 && (!Q || !out)) return fail(SD_EINVAL, std::string(who) + ": null array");
    return check_params(p, who);
}

}  // namespace sd

extern "C" {

const char *sd_last_error(void) { return sd::g_err.c_str(); }

int sd_set_memory_budget(int64_t bytes) {
    std::lock_guard<std::mutex> lock(sd::g_mem_mu);
    sd::g_mem_budget = bytes < 0 ? -1 : bytes;
    return SD_OK;
}

int sd_memory_in_use(int64_t *bytes_out) {
    if (!bytes_out) return sd::fail(SD_EINVAL, "sd_memory_in_use: null output");
    std::lock_guard<std::mutex> lock(sd::g_mem_mu);
    *bytes_out = sd::g_mem_in_use;
    return SD_OK;
}

int sd_build_bvh(const float *V, int64_t nV, const int32_t *P, int64_t nP, const int32_t *E,
                 int64_t nE, const int32_t *T, int64_t nT, uint32_t flags, void *stream,
                 sd_scene **out) {
    using sd::fail;
    if (!out) return fail(SD_EINVAL, "sd_build_bvh: null output handle");
    *out = nullptr;
    if (nV < 0 || nE < 0 || nT < 0) return fail(SD_EINVAL, "sd_build_bvh: negative size");
    if (nP < 0) {
        if (P) return fail(SD_EINVAL, "sd_build_bvh: nP < 0 requires P == NULL (all vertices)");
        nP = nV;
    } else if (nP > 0 && !P) {
        return fail(SD_EINVAL, "sd_build_bvh: P is NULL with nP > 0");
    }
    if ((nV > 0 && !V) || (nE > 0 && !E) || (nT > 0 && !T))
        return fail(SD_EINVAL, "sd_build_bvh: null array with a positive count");
    if (nV == 0 && (nP > 0 || nE > 0 || nT > 0))
        return fail(SD_EINVAL, "sd_build_bvh: primitives reference an empty vertex array");
    if (nV > 0x7fffffff) return fail(SD_EUNSUPPORTED, "sd_build_bvh: more than 2^31 vertices");
    sd_scene *sc = new (std::nothrow) sd_scene();
    if (!sc) return fail(SD_ENOMEM, "sd_build_bvh: host allocation");
    SD_HIP(hipGetDevice(&sc->device));
    int rc = sd::build_scene(sc, V, nV, P, nP, E, nE, T, nT, flags, (hipStream_t)stream);
    if (rc != SD_OK) {
        std::string keep = sd::g_err;
        sd_free_scene(sc);
        sd::g_err = keep;
        return rc;
    }
    *out = sc;
    return SD_OK;
}

int sd_free_scene(sd_scene *sc) {
    if (!sc) return SD_OK;
    for (int c = 0; c < 3; ++c) {
        // hi[c] points into the interleaved lo[c] allocation
        for (void *p : {(void *)sc->lo[c], (void *)sc->leaf[c], (void *)sc->prim_id[c],
                        (void *)sc->wt[c]})
            sd::dev_free(p);
    }
    sd::dev_free(sc->tri_table);
    delete sc;
    return SD_OK;
}

int sd_scene_info_get(const sd_scene *sc, sd_scene_info *out) {
    if (!sc || !out) return sd::fail(SD_EINVAL, "sd_scene_info_get: null argument");
    for (int c = 0; c < 3; ++c) {
        out->n_prims[c] = sc->n[c];
        out->n_nodes[c] = sc->n_nodes[c];
        out->A[c] = sc->A[c];
    }
    out->A_T_literal = sc->A_T_literal;
    out->diam_max = sc->diam_max;
    out->device_bytes = sc->device_bytes;
    out->n_tri_classes = sc->n_tri_classes;
    out->pad = 0;
    return SD_OK;
}

int sd_eval(const sd_scene *sc, const float *Q, int64_t nQ, const sd_params *p, float *d_out,
            void *stream) {
    SD_TRY(sd::check_eval(sc, Q, nQ, p, d_out, "sd_eval"));
    return sd::eval_dispatch(sc, Q, nullptr, nQ, p, d_out, nullptr, nullptr, false, (hipStream_t)stream);
}

int sd_eval_grad_prims(const sd_scene *sc, const float *G, int32_t nv, int64_t n, const sd_params *p,
                       float *d_out, float *grad_out, void *stream) {
    if (!sc) return sd::fail(SD_EINVAL, "sd_eval_grad_prims: null scene");
    if (n < 0) return sd::fail(SD_EINVAL, "sd_eval_grad_prims: negative count");
    if (nv < 1 || nv > 3) return sd::fail(SD_EINVAL, "sd_eval_grad_prims: nv must be 1, 2 or 3");
    SD_TRY(sd::check_params(p, "sd_eval_grad_prims"));
    if (n > 0 && (!G || !d_out || !grad_out)) return sd::fail(SD_EINVAL, "sd_eval_grad_prims: null pointer");
    if (nv == 1)   // a point: the point query
        return sd::eval_dispatch(sc, G, nullptr, n, p, d_out, grad_out, nullptr, false, (hipStream_t)stream);
    return sd::evalq_dispatch(sc, G, nv, n, p, d_out, grad_out, (hipStream_t)stream);
}

int sd_sphere_trace(const sd_scene *sc, const float *O, const float *U, int64_t n, const sd_params *p,
                    float level, float eps, float t_max, int32_t max_steps, float *t_out, int32_t *steps_out,
                    void *stream) {
    if (!sc) return sd::fail(SD_EINVAL, "sd_sphere_trace: null scene");
    if (n < 0) return sd::fail(SD_EINVAL, "sd_sphere_trace: negative ray count");
    SD_TRY(sd::check_params(p, "sd_sphere_trace"));
    if (!(eps > 0.f) || !isfinite(eps) || !(t_max >= 0.f) || !isfinite(level) || max_steps < 1)
        return sd::fail(SD_EINVAL, "sd_sphere_trace: need eps > 0, t_max >= 0, finite level, max_steps >= 1");
    if (n > 0 && (!O || !U || !t_out)) return sd::fail(SD_EINVAL, "sd_sphere_trace: null pointer");
    return sd::trace_dispatch(sc, O, U, n, p, level, eps, t_max, max_steps, t_out, steps_out,
                              (hipStream_t)stream);
}

int sd_eval_grad(const sd_scene *sc, const float *Q, int64_t nQ, const sd_params *p, float *d_out,
                 float *grad_out, void *stream) {
    SD_TRY(sd::check_eval(sc, Q, nQ, p, d_out, "sd_eval_grad"));
    if (nQ > 0 && !grad_out) return sd::fail(SD_EINVAL, "sd_eval_grad: null grad_out");
    return sd::eval_dispatch(sc, Q, nullptr, nQ, p, d_out, grad_out, nullptr, false, (hipStream_t)stream);
}

int sd_eval_grad_noalloc(const sd_scene *sc, const float *Q, int64_t nQ, const sd_params *p, float *d_out,
                         float *grad_out, void *stream) {
    SD_TRY(sd::check_eval(sc, Q, nQ, p, d_out, "sd_eval_grad_noalloc"));
    if (nQ > 0 && !grad_out) return sd::fail(SD_EINVAL, "sd_eval_grad_noalloc: null grad_out");
    return sd::eval_grad_noalloc(sc, Q, nQ, p, d_out, grad_out, (hipStream_t)stream);
}

int sd_query_order(const sd_scene *sc, const float *Q, int64_t nQ, uint32_t *perm_out,
                   void *stream) {
    if (!sc) return sd::fail(SD_EINVAL, "sd_query_order: null scene");
    if (nQ < 0) return sd::fail(SD_EINVAL, "sd_query_order: nQ < 0");
    if (nQ > 0 && (!Q || !perm_out)) return sd::fail(SD_EINVAL, "sd_query_order: null array");
    if (nQ > 0xffffffffll) return sd::fail(SD_EUNSUPPORTED, "sd_query_order: too many queries");
    return sd::query_order(sc, Q, nQ, perm_out, (hipStream_t)stream);
}

int sd_eval_grad_ordered(const sd_scene *sc, const float *Q, const uint32_t *perm, int64_t nQ,
                         const sd_params *p, float *d_out, float *grad_out, void *stream) {
    SD_TRY(sd::check_eval(sc, Q, nQ, p, d_out, "sd_eval_grad_ordered"));
    sd_params q = *p;
    if (!perm) q.flags |= SD_NO_QUERY_SORT;
    return sd::eval_dispatch(sc, Q, perm, nQ, &q, d_out, grad_out, nullptr, false, (hipStream_t)stream);
}

int sd_eval_brute(const sd_scene *sc, const float *Q, int64_t nQ, const sd_params *p, float *d_out,
                  float *grad_out, void *stream) {
    SD_TRY(sd::check_eval(sc, Q, nQ, p, d_out, "sd_eval_brute"));
    return sd::eval_dispatch(sc, Q, nullptr, nQ, p, d_out, grad_out, nullptr, true, (hipStream_t)stream);
}

int sd_eval_counters(const sd_scene *sc, const float *Q, int64_t nQ, const sd_params *p,
                     int32_t *counts_out, void *stream) {
    SD_TRY(sd::check_eval(sc, Q, nQ, p, counts_out, "sd_eval_counters"));
    return sd::eval_dispatch(sc, Q, nullptr, nQ, p, nullptr, nullptr, counts_out, false, (hipStream_t)stream);
}

int sd_export_bvh(const sd_scene *sc, int cls, float *box_host, int32_t *left_host,
                  int32_t *right_host, int32_t *prim_host, void *stream) {
    using sd::fail;
    if (!sc || cls < 0 || cls > 2) return fail(SD_EINVAL, "sd_export_bvh: bad scene or class");
    int64_t nn = sc->n_nodes[cls];
    if (nn == 0) return SD_OK;
    if (!box_host || !left_host || !right_host || !prim_host)
        return fail(SD_EINVAL, "sd_export_bvh: null output");
    hipStream_t s = (hipStream_t)stream;
    std::vector<float4> rec(2 * nn), lo(nn), hi(nn);
    std::vector<int32_t> pid(sc->n[cls]);
    SD_HIP(hipMemcpyAsync(rec.data(), sc->lo[cls], 2 * nn * sizeof(float4), hipMemcpyDeviceToHost, s));
    SD_HIP(hipMemcpyAsync(pid.data(), sc->prim_id[cls], sc->n[cls] * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < nn; ++i) {
        lo[i] = rec[2 * i];
        hi[i] = rec[2 * i + 1];
    }
    for (int64_t i = 0; i < nn; ++i) {
        box_host[6 * i] = lo[i].x; box_host[6 * i + 1] = lo[i].y; box_host[6 * i + 2] = lo[i].z;
        box_host[6 * i + 3] = hi[i].x; box_host[6 * i + 4] = hi[i].y; box_host[6 * i + 5] = hi[i].z;
        int32_t pay;
        __builtin_memcpy(&pay, &hi[i].w, 4);
        if (pay < 0) {
            left_host[i] = right_host[i] = -1;
            prim_host[i] = pid[pay & 0x7fffffff];
        } else {
            int32_t l = (int32_t)(i + 1), r;
            __builtin_memcpy(&r, &lo[l].w, 4);   // right child = escape of the left child
            left_host[i] = l;
            right_host[i] = r;
            prim_host[i] = -1;
        }
    }
    return SD_OK;
}

int sd_export_weights(const sd_scene *sc, int cls, float *wt_host, void *stream) {
    using sd::fail;
    if (!sc || cls < 1 || cls > 2) return fail(SD_EINVAL, "sd_export_weights: bad scene or class");
    if (sc->n[cls] == 0) return SD_OK;
    if (!wt_host) return fail(SD_EINVAL, "sd_export_weights: null output");
    int k = cls == 1 ? 2 : 3;
    SD_HIP(hipMemcpyAsync(wt_host, sc->wt[cls], sc->n[cls] * k * sizeof(float), hipMemcpyDeviceToHost,
                          (hipStream_t)stream));
    SD_HIP(hipStreamSynchronize((hipStream_t)stream));
    return SD_OK;
}

}  // extern "C"
