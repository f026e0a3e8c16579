// Stable LSD radix sort of (uint64 key, uint32 value) pairs and an exclusive
// prefix sum, for the hierarchy build (Morton keys, edge keys) and the query
// ordering.  Wave64 design: each 256-thread block owns a tile of 2048 keys;
// ranks inside a tile come from 64-lane ballots (match-any on the 8-bit digit)
// and per-wave digit counters in LDS, so no atomics touch global memory and
// the result is deterministic.  The sort can take its key count from device
// memory (n_dev, at most the host bound n that sizes the launches), so that a
// count produced on the GPU never has to reach the host.
#include "sd_internal.h"

namespace sd {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;   // 2048
constexpr int kRadix = 256;

__device__ inline uint64_t lanemask_lt() {
    int lane = __lane_id();
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__global__ void __launch_bounds__(kThreads)
k_digit_hist(const uint64_t *__restrict__ keys, int64_t n, const uint32_t *__restrict__ n_dev, int shift,
             uint32_t *__restrict__ hist, int nblocks) {
    __shared__ uint32_t h[kRadix];
    if (n_dev) n = min(n, (int64_t)*n_dev);
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = 0; i < kItems; ++i) {
        int64_t idx = base + (int64_t)i * kThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xff], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kThreads)
k_digit_scatter(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                uint64_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out, int64_t n,
                const uint32_t *__restrict__ n_dev, int shift, const uint32_t *__restrict__ offs, int nblocks) {
    __shared__ uint32_t wcnt[kWaves][kRadix];
    if (n_dev) n = min(n, (int64_t)*n_dev);
    __shared__ uint32_t goff[kRadix];
    const int lane = __lane_id();
    const int w = threadIdx.x >> 6;
    for (int k = 0; k < kWaves; ++k) wcnt[k][threadIdx.x] = 0;
    goff[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();

    uint64_t kk[kItems];
    uint32_t vv[kItems], rank[kItems];
    int dg[kItems];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)w * (64 * kItems);
    const uint64_t lt = lanemask_lt();
    for (int r = 0; r < kItems; ++r) {
        int64_t idx = base + r * 64 + lane;
        bool valid = idx < n;
        uint64_t key = valid ? keys[idx] : 0;
        int d = (int)((key >> shift) & 0xff);
        uint64_t m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        uint32_t before = valid ? wcnt[w][d] : 0;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        bool leader = valid && ((m & lt) == 0);
        if (leader) wcnt[w][d] = before + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        kk[r] = key;
        vv[r] = valid ? vals[idx] : 0;
        dg[r] = valid ? d : -1;
        rank[r] = before + (uint32_t)__popcll(m & lt);
    }
    __syncthreads();
    {
        uint32_t run = 0;
        for (int k = 0; k < kWaves; ++k) {
            uint32_t t = wcnt[k][threadIdx.x];
            wcnt[k][threadIdx.x] = run;
            run += t;
        }
    }
    __syncthreads();
    for (int r = 0; r < kItems; ++r) {
        if (dg[r] < 0) continue;
        uint32_t pos = goff[dg[r]] + wcnt[w][dg[r]] + rank[r];
        keys_out[pos] = kk[r];
        vals_out[pos] = vv[r];
    }
}

// ---------------------------------------------------------------------------
// exclusive scan (uint32), three phases over tiles of 2048
// ---------------------------------------------------------------------------
__device__ inline uint32_t wave_incl_scan(uint32_t x) {
    const int lane = __lane_id();
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// block-wide exclusive scan of one value per thread; returns total in *tot
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t *tot) {
    __shared__ uint32_t ws[kWaves];
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(x);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
    for (int k = 0; k < kWaves; ++k) {
        if (k < w) off += ws[k];
        all += ws[k];
    }
    __syncthreads();
    *tot = all;
    return off + inc - x;
}

__global__ void __launch_bounds__(kThreads)
k_scan_reduce(const uint32_t *__restrict__ in, int64_t n, uint32_t *__restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t s = 0;
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) s += in[base + i];
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kThreads)
k_scan_partials(uint32_t *part, int64_t np) {
    uint32_t carry = 0;
    for (int64_t b = 0; b < np; b += kThreads) {
        int64_t i = b + threadIdx.x;
        uint32_t x = i < np ? part[i] : 0;
        uint32_t tot;
        uint32_t ex = block_excl_scan(x, &tot);
        if (i < np) part[i] = ex + carry;
        carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads)
k_scan_down(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, int64_t n,
            const uint32_t *__restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems], s = 0;
    for (int i = 0; i < kItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + part[blockIdx.x];
    for (int i = 0; i < kItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t scan_temp_bytes(int64_t n) { return (size_t)(ceil_div(n, kTile) + 64) * sizeof(uint32_t); }

}  // namespace

int exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, void *temp, hipStream_t s) {
    if (n <= 0) return SD_OK;
    int64_t nb = ceil_div(n, kTile);
    uint32_t *part = (uint32_t *)temp;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, s, part, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kThreads), 0, s, in, out, n, part);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

size_t radix_sort_temp_bytes(int64_t n) {
    int64_t nb = ceil_div(std::max<int64_t>(n, 1), kTile);
    size_t hist = (size_t)nb * kRadix * sizeof(uint32_t);
    return 2 * hist + scan_temp_bytes(nb * kRadix) + 256;
}

int radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_tmp, uint32_t *vals_tmp,
                     int64_t n, int bits, void *temp, hipStream_t s, const uint32_t *n_dev) {
    if (n <= 1) return SD_OK;
    if (n > (int64_t)0xffffffffll) return fail(SD_EUNSUPPORTED, "radix sort: more than 2^32 keys");
    int nb = (int)ceil_div(n, kTile);
    size_t hbytes = (size_t)nb * kRadix * sizeof(uint32_t);
    uint32_t *hist = (uint32_t *)temp;
    uint32_t *offs = (uint32_t *)((char *)temp + hbytes);
    void *stemp = (char *)temp + 2 * hbytes;
    uint64_t *ka = keys, *kb = keys_tmp;
    uint32_t *va = vals, *vb = vals_tmp;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_digit_hist, dim3(nb), dim3(kThreads), 0, s, ka, n, n_dev, shift, hist, nb);
        SD_TRY(exclusive_scan_u32(hist, offs, (int64_t)nb * kRadix, stemp, s));
        hipLaunchKernelGGL(k_digit_scatter, dim3(nb), dim3(kThreads), 0, s, ka, va, kb, vb, n,
                           n_dev, shift, offs, nb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    SD_HIP(hipGetLastError());
    if (ka != keys) {
        SD_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        SD_HIP(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    return SD_OK;
}

}  // namespace sd
