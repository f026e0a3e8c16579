// Smooth distance between the data mesh and a query mesh (Sec. 3.6).
//
// For each of K instances of one query mesh (e.g. K rigid placements of a
// body) the per-primitive smooth distances d_kj (row k) are combined with an
// outer log-sum-exp of sharpness alpha_q (Eq. 6):
//   D_k = M_k - log(S_k) / alpha_q,   S_k = sum_j exp(-alpha_q (d_kj - M_k)),
// M_k = min_j d_kj factored out so that nothing overflows.  dD_k/dd_kj =
// w_kj = exp(-alpha_q (d_kj - M_k)) / S_k, and the vertex gradients of Eq. 8
// give each vertex of primitive g_j the share w_kj / (n(g_j) + 1) of the
// primitive's (rigid-translation) gradient.
//
// The work is HBM-bound (one pass for the minima, one for the sums, one for
// the outputs over K x m distances); partials are combined in a fixed order,
// so D and w are bitwise reproducible.  Vertex gradients of a general query
// mesh are scattered with float atomics (summation order not fixed); for a
// point query mesh (each primitive its own vertex) they are written directly.
#include <math.h>

#include <algorithm>

#include "sd_internal.h"

namespace sd {
namespace {

constexpr int kB = 256;
constexpr int64_t kChunk = 4096;   // distances per (instance, chunk) workgroup

// minimum that propagates NaN (an instance with a NaN distance gives NaN)
__device__ __forceinline__ float nanmin(float a, float b) {
    return (a != a || b != b) ? __builtin_nanf("") : fminf(a, b);
}

__device__ __forceinline__ float block_min(float v, float *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = nanmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    return red[0];
}

// pass 1: minimum over each (instance k, chunk c)
__global__ void __launch_bounds__(kB)
k_qm_min(const float *__restrict__ d, int64_t m, float *__restrict__ pmin) {
    __shared__ float red[kB];
    const int64_t k = blockIdx.x, c = blockIdx.y, C = gridDim.y;
    const int64_t j0 = c * kChunk, j1 = min(m, j0 + kChunk);
    float v = INFINITY;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kB) v = nanmin(v, d[k * m + j]);
    v = block_min(v, red);
    if (threadIdx.x == 0) pmin[k * C + c] = v;
}

// pass 2: sum over each (instance, chunk) of exp(-alpha_q (d - M_k)) in FP64
__global__ void __launch_bounds__(kB)
k_qm_sum(const float *__restrict__ d, int64_t m, const float *__restrict__ pmin, float alpha_q,
         double *__restrict__ psum) {
    __shared__ double red[kB];
    const int64_t k = blockIdx.x, c = blockIdx.y, C = gridDim.y;
    float M = INFINITY;
    for (int64_t i = 0; i < C; ++i) M = nanmin(M, pmin[k * C + i]);
    const int64_t j0 = c * kChunk, j1 = min(m, j0 + kChunk);
    double s = 0.0;
    if (M != INFINITY) {   // a NaN M makes the sum NaN
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kB)
            s += (double)expf(-alpha_q * (d[k * m + j] - M));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) psum[k * C + c] = red[0];
}

// pass 3: per instance, M_k, S_k (chunk partials in order) and D_k
__global__ void __launch_bounds__(kB)
k_qm_final(const float *__restrict__ pmin, const double *__restrict__ psum, int64_t K, int64_t C,
           float alpha_q, float *__restrict__ D, double *__restrict__ ms) {
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k >= K) return;
    float M = INFINITY;
    double S = 0.0;
    for (int64_t i = 0; i < C; ++i) {
        M = nanmin(M, pmin[k * C + i]);
        S += psum[k * C + i];
    }
    // empty instance or every distance +inf: the empty sum, D = +inf
    D[k] = M != INFINITY ? (float)((double)M - log(S) / (double)alpha_q) : INFINITY;
    ms[2 * k] = (double)M;
    ms[2 * k + 1] = S;
}

__global__ void __launch_bounds__(kB) k_qm_fill(float *__restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = v;
}

// pass 4: weights w_kj and vertex gradients
__global__ void __launch_bounds__(kB)
k_qm_out(const float *__restrict__ d, const float *__restrict__ grad, int64_t K, int64_t m,
         float alpha_q, const double *__restrict__ ms, const int32_t *__restrict__ prim, int64_t nV,
         float *__restrict__ w, float *__restrict__ vgrad) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= K * m) return;
    const int64_t k = i / m, j = i - k * m;
    const float M = (float)ms[2 * k];
    const double S = ms[2 * k + 1];
    const float wk = M != INFINITY ? (float)((double)expf(-alpha_q * (d[i] - M)) / S) : 0.f;
    if (w) w[i] = wk;
    if (!vgrad) return;
    const float gx = grad[3 * i], gy = grad[3 * i + 1], gz = grad[3 * i + 2];
    if (!prim) {   // point query mesh: primitive j is vertex j
        vgrad[3 * i] = wk * gx;
        vgrad[3 * i + 1] = wk * gy;
        vgrad[3 * i + 2] = wk * gz;
        return;
    }
    const int32_t vs[3] = {prim[3 * j], prim[3 * j + 1], prim[3 * j + 2]};
    const int n = (vs[0] >= 0) + (vs[1] >= 0) + (vs[2] >= 0);   // n(g_j) + 1
    if (n == 0) return;
    const float share = wk / (float)n;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int32_t v = vs[a];
        if (v < 0) continue;
        float *o = vgrad + 3 * (k * nV + v);
        atomicAdd(o, share * gx);
        atomicAdd(o + 1, share * gy);
        atomicAdd(o + 2, share * gz);
    }
}

// index check of the primitive table: bad[0] = 1 if any id is >= nV or < -1,
// or a primitive has no vertex
__global__ void __launch_bounds__(kB)
k_qm_check(const int32_t *__restrict__ prim, int64_t m, int64_t nV, int32_t *__restrict__ bad) {
    const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (j >= m) return;
    int n = 0;
    for (int a = 0; a < 3; ++a) {
        int32_t v = prim[3 * j + a];
        if (v < -1 || v >= nV) bad[0] = 1;
        n += v >= 0;
    }
    if (n == 0) bad[0] = 1;
}

unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kB - 1) / kB); }

}  // namespace
}  // namespace sd

extern "C" int sd_query_mesh_lse(const float *d, const float *grad, int64_t K, int64_t m,
                                 const int32_t *prim, int64_t nV, float alpha_q, float *D, float *w,
                                 float *vgrad, void *stream) {
    if (K < 0 || m < 0) return sd::fail(SD_EINVAL, "sd_query_mesh_lse: negative size");
    if (!(alpha_q > 0.f) || !(alpha_q < INFINITY))
        return sd::fail(SD_EINVAL, "sd_query_mesh_lse: alpha_q must be positive and finite");
    if (!prim) nV = m;
    if (prim && nV <= 0) return sd::fail(SD_EINVAL, "sd_query_mesh_lse: nV must be positive with prim");
    if (K == 0) return SD_OK;
    if (!D || (m > 0 && !d) || (m > 0 && vgrad && !grad))
        return sd::fail(SD_EINVAL, "sd_query_mesh_lse: null pointer");
    if (K > 0xffff || m > ((int64_t)1 << 28) || (prim && nV > ((int64_t)1 << 28)))
        return sd::fail(SD_EUNSUPPORTED, "sd_query_mesh_lse: more than 65535 instances or 2^28 primitives");
    hipStream_t s = (hipStream_t)stream;
    if (prim && m > 0) {
        int32_t *bad_dev = nullptr, bad = 0;
        sd::AsyncScratch tmp(s);
        SD_TRY(tmp.alloc(&bad_dev, 1));
        SD_HIP(hipMemcpyAsync(bad_dev, &bad, sizeof(int32_t), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(sd::k_qm_check, dim3(sd::grid1(m)), dim3(sd::kB), 0, s, prim, m, nV, bad_dev);
        SD_HIP(hipMemcpyAsync(&bad, bad_dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SD_HIP(hipStreamSynchronize(s));
        if (bad) return sd::fail(SD_EINVAL, "sd_query_mesh_lse: primitive vertex id outside [0, nV) or empty primitive");
    }
    if (vgrad && (prim || m == 0))   // scattered (or empty): start from zero
        hipLaunchKernelGGL(sd::k_qm_fill, dim3(sd::grid1(K * nV * 3)), dim3(sd::kB), 0, s, vgrad, K * nV * 3, 0.f);
    if (m == 0) {
        hipLaunchKernelGGL(sd::k_qm_fill, dim3(sd::grid1(K)), dim3(sd::kB), 0, s, D, K, INFINITY);
        SD_HIP(hipGetLastError());
        return SD_OK;
    }
    const int64_t C = (m + sd::kChunk - 1) / sd::kChunk;
    char *scratch = nullptr;
    const size_t bytes = (size_t)K * C * (sizeof(float) + sizeof(double)) + (size_t)K * 2 * sizeof(double);
    sd::AsyncScratch tmp(s);
    SD_TRY(tmp.alloc(&scratch, (int64_t)bytes));
    double *psum = (double *)scratch;
    double *ms = psum + K * C;
    float *pmin = (float *)(ms + 2 * K);
    hipLaunchKernelGGL(sd::k_qm_min, dim3((unsigned)K, (unsigned)C), dim3(sd::kB), 0, s, d, m, pmin);
    hipLaunchKernelGGL(sd::k_qm_sum, dim3((unsigned)K, (unsigned)C), dim3(sd::kB), 0, s, d, m, pmin, alpha_q, psum);
    hipLaunchKernelGGL(sd::k_qm_final, dim3(sd::grid1(K)), dim3(sd::kB), 0, s, pmin, psum, K, C, alpha_q, D, ms);
    if (w || vgrad)
        hipLaunchKernelGGL(sd::k_qm_out, dim3(sd::grid1(K * m)), dim3(sd::kB), 0, s, d, grad, K, m, alpha_q, ms,
                           prim, nV, w, vgrad);
    SD_HIP(hipGetLastError());
    return SD_OK;
}
