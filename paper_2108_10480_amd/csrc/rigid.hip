// Rigidly moved query points and the adjoint of the smooth distance with
// respect to the rigid transform and the body points.
//
// Forward:  x'_kj = R_k x_j + t_k for K transforms of m body points.
// Adjoint:  with u_kj = gbar_kj * grad d(x'_kj)  (gbar = dL/dd upstream),
//   tbar_k = sum_j u_kj,  Rbar_k = sum_j u_kj x_j^T,  xbar_j = sum_k R_k^T u_kj.
// For the query-mesh distance D_k of the moved points (Eq. 6-8), gbar_kj =
// w_kj * Dbar_k with w_kj = dD_k/dd_kj and Dbar_k = dL/dD_k; the product is
// formed in the kernels (kscale = Dbar).
// The reductions use a fixed order (per-thread strided sums over a chunk, an
// LDS tree, then the chunk partials in order), so results are bitwise
// reproducible.
#include <algorithm>
#include <string>

#include "sd_internal.h"

namespace sd {
namespace {

constexpr int kB = 256;

__global__ void __launch_bounds__(kB)
k_rigid_apply(const float *__restrict__ X, int64_t m, const float *__restrict__ R,
              const float *__restrict__ t, int64_t K, float *__restrict__ Q) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= K * m) return;
    int64_t k = i / m, j = i - k * m;
    const float *r = R + 9 * k;
    float x = X[3 * j], y = X[3 * j + 1], z = X[3 * j + 2];
    Q[3 * i] = fmaf(r[0], x, fmaf(r[1], y, fmaf(r[2], z, t[3 * k])));
    Q[3 * i + 1] = fmaf(r[3], x, fmaf(r[4], y, fmaf(r[5], z, t[3 * k + 1])));
    Q[3 * i + 2] = fmaf(r[6], x, fmaf(r[7], y, fmaf(r[8], z, t[3 * k + 2])));
}

// Partial sums of one (transform, chunk of body points): 12 sums (tbar 3,
// Rbar 9) per workgroup, written to part[k][chunk][12].
__global__ void __launch_bounds__(kB)
k_rigid_rt_part(const float *__restrict__ X, int64_t m, int64_t chunk, const float *__restrict__ gbar,
                const float *__restrict__ kscale, const float *__restrict__ grad, float *__restrict__ part) {
    __shared__ float red[12][kB];
    const int64_t k = blockIdx.x;
    const float ks = kscale ? kscale[k] : 1.f;
    const int64_t j0 = (int64_t)blockIdx.y * chunk, j1 = min(m, j0 + chunk);
    float acc[12];
#pragma unroll
    for (int a = 0; a < 12; ++a) acc[a] = 0.f;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += kB) {
        int64_t i = k * m + j;
        float g = kscale ? gbar[i] * ks : gbar[i];
        float u0 = g * grad[3 * i], u1 = g * grad[3 * i + 1], u2 = g * grad[3 * i + 2];
        float x0 = X[3 * j], x1 = X[3 * j + 1], x2 = X[3 * j + 2];
        acc[0] += u0; acc[1] += u1; acc[2] += u2;
        acc[3] = fmaf(u0, x0, acc[3]); acc[4] = fmaf(u0, x1, acc[4]); acc[5] = fmaf(u0, x2, acc[5]);
        acc[6] = fmaf(u1, x0, acc[6]); acc[7] = fmaf(u1, x1, acc[7]); acc[8] = fmaf(u1, x2, acc[8]);
        acc[9] = fmaf(u2, x0, acc[9]); acc[10] = fmaf(u2, x1, acc[10]); acc[11] = fmaf(u2, x2, acc[11]);
    }
#pragma unroll
    for (int a = 0; a < 12; ++a) red[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int w = kB / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int a = 0; a < 12; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 12) part[(k * gridDim.y + blockIdx.y) * 12 + threadIdx.x] = red[threadIdx.x][0];
}

// tbar, Rbar of transform k: the chunk partials added in chunk order
__global__ void k_rigid_rt_final(const float *__restrict__ part, int64_t K, int chunks,
                                 float *__restrict__ Rbar, float *__restrict__ tbar) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= K * 12) return;
    int64_t k = i / 12;
    int a = (int)(i % 12);
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(k * chunks + c) * 12 + a];
    if (a < 3) tbar[3 * k + a] = s;
    else Rbar[9 * k + a - 3] = s;
}

// xbar partials: thread per body point, transforms [k0, k1) of this chunk;
// part[chunk][j][3]
__global__ void __launch_bounds__(kB)
k_rigid_x_part(const float *__restrict__ R, int64_t K, int64_t kchunk, int64_t m,
               const float *__restrict__ gbar, const float *__restrict__ kscale, const float *__restrict__ grad,
               float *__restrict__ part) {
    int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (j >= m) return;
    const int64_t k0 = (int64_t)blockIdx.y * kchunk, k1 = min(K, k0 + kchunk);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    for (int64_t k = k0; k < k1; ++k) {
        int64_t i = k * m + j;
        float g = kscale ? gbar[i] * kscale[k] : gbar[i];
        float u0 = g * grad[3 * i], u1 = g * grad[3 * i + 1], u2 = g * grad[3 * i + 2];
        const float *r = R + 9 * k;
        a0 = fmaf(r[0], u0, fmaf(r[3], u1, fmaf(r[6], u2, a0)));
        a1 = fmaf(r[1], u0, fmaf(r[4], u1, fmaf(r[7], u2, a1)));
        a2 = fmaf(r[2], u0, fmaf(r[5], u1, fmaf(r[8], u2, a2)));
    }
    float *o = part + ((int64_t)blockIdx.y * m + j) * 3;
    o[0] = a0;
    o[1] = a1;
    o[2] = a2;
}

__global__ void k_rigid_x_final(const float *__restrict__ part, int64_t m, int chunks,
                                float *__restrict__ Xbar) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= 3 * m) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * 3 * m + i];
    Xbar[i] = s;
}

}  // namespace
}  // namespace sd

extern "C" int sd_rigid_transform(const float *X, int64_t m, const float *R, const float *t,
                                  int64_t K, float *Q_out, void *stream) {
    if (m < 0 || K < 0) return sd::fail(SD_EINVAL, "sd_rigid_transform: negative size");
    if (m == 0 || K == 0) return SD_OK;
    if (!X || !R || !t || !Q_out) return sd::fail(SD_EINVAL, "sd_rigid_transform: null pointer");
    hipStream_t s = (hipStream_t)stream;
    int64_t n = K * m;
    hipLaunchKernelGGL(sd::k_rigid_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, m, R,
                       t, K, Q_out);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

namespace {
int rigid_adjoint(const char *name, const float *X, int64_t m, const float *R, int64_t K, const float *gbar,
                  const float *kscale, const float *grad, float *Rbar, float *tbar, float *Xbar, void *stream) {
    if (m < 0 || K < 0) return sd::fail(SD_EINVAL, std::string(name) + ": negative size");
    if (K == 0) return SD_OK;
    if (!R || !Rbar || !tbar || (m > 0 && (!X || !gbar || !grad)))
        return sd::fail(SD_EINVAL, std::string(name) + ": null pointer");
    if (K > 0x7fffffff) return sd::fail(SD_EUNSUPPORTED, std::string(name) + ": too many transforms");
    hipStream_t s = (hipStream_t)stream;
    // split each reduction so that the grid fills the chip; partials are added
    // in a fixed order (bitwise reproducible)
    const int64_t chunk = std::max<int64_t>(1024, (m + 15) / 16);
    const int chunks = m > 0 ? (int)((m + chunk - 1) / chunk) : 1;
    const int64_t kchunk = 16;
    const int kchunks = (int)((K + kchunk - 1) / kchunk);
    const bool want_x = Xbar && m > 0;
    size_t bytes = (size_t)K * chunks * 12 * sizeof(float);
    if (want_x) bytes = std::max(bytes, (size_t)kchunks * m * 3 * sizeof(float));
    float *part = nullptr;
    sd::AsyncScratch tmp(s);
    SD_TRY(tmp.alloc(&part, (int64_t)(bytes / sizeof(float))));
    if (m > 0) {
        hipLaunchKernelGGL(sd::k_rigid_rt_part, dim3((unsigned)K, (unsigned)chunks), dim3(256), 0, s, X, m, chunk,
                           gbar, kscale, grad, part);
        hipLaunchKernelGGL(sd::k_rigid_rt_final, dim3((unsigned)((K * 12 + 255) / 256)), dim3(256), 0, s, part, K,
                           chunks, Rbar, tbar);
    } else {
        SD_HIP(hipMemsetAsync(Rbar, 0, K * 9 * sizeof(float), s));
        SD_HIP(hipMemsetAsync(tbar, 0, K * 3 * sizeof(float), s));
    }
    if (want_x) {
        hipLaunchKernelGGL(sd::k_rigid_x_part, dim3((unsigned)((m + 255) / 256), (unsigned)kchunks), dim3(256), 0,
                           s, R, K, kchunk, m, gbar, kscale, grad, part);
        hipLaunchKernelGGL(sd::k_rigid_x_final, dim3((unsigned)((3 * m + 255) / 256)), dim3(256), 0, s, part, m,
                           kchunks, Xbar);
    }
    SD_HIP(hipGetLastError());
    return SD_OK;
}
}  // namespace

extern "C" int sd_rigid_adjoint(const float *X, int64_t m, const float *R, int64_t K,
                                const float *gbar, const float *grad, float *Rbar, float *tbar,
                                float *Xbar, void *stream) {
    return rigid_adjoint("sd_rigid_adjoint", X, m, R, K, gbar, nullptr, grad, Rbar, tbar, Xbar, stream);
}

extern "C" int sd_rigid_qmesh_adjoint(const float *X, int64_t m, const float *R, int64_t K, const float *w,
                                      const float *Dbar, const float *grad, float *Rbar, float *tbar,
                                      float *Xbar, void *stream) {
    if (K > 0 && !Dbar) return sd::fail(SD_EINVAL, "sd_rigid_qmesh_adjoint: null pointer");
    return rigid_adjoint("sd_rigid_qmesh_adjoint", X, m, R, K, w, Dbar, grad, Rbar, tbar, Xbar, stream);
}
