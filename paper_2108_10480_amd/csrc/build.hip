// Scene ingest, valences / weight data and the linear BVH build.
//
// Per non-empty primitive class (points, edges, triangles) one binary
// hierarchy is built (the paper leaves the hierarchy open: "a BVH", Sec. 3.5):
//   1. primitive boxes and centroid bounds
//   2. 63-bit Morton keys of the centroids, stable radix sort
//   3. Karras' radix-tree topology over the sorted keys (index tie-break)
//   4. bottom-up box refit (agent-scope acquire/release counters)
//   5. depth-first renumbering: node with first leaf l reached through t
//      left-child edges sits at 2 l + t; escape = position + subtree size
//   6. leaf records in depth-first leaf order, with the weight data of App. C.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sd_internal.h"

namespace sd {
namespace {

constexpr int kB = 256;

inline unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kB - 1) / kB); }

__device__ inline uint32_t f2o(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float o2f(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    float f;
    __builtin_memcpy(&f, &b, 4);
    return f;
}

// scratch reduction record written by the box kernels
struct Reduce {
    uint32_t cmin[3], cmax[3];   // centroid bounds (ordered bits)
    uint32_t bmin[3], bmax[3];   // primitive box bounds (ordered bits)
    uint32_t diam;               // max primitive box diagonal (ordered bits)
    uint32_t bad;                // index error flag
    uint32_t maxv;               // max valence
    uint32_t pad;
};

template <int K>
__device__ inline int load_ids(const int32_t *ids, int64_t i, int64_t nV, int out[3], uint32_t *bad) {
    int ok = 1;
    for (int k = 0; k < K; ++k) {
        int v = ids ? ids[i * K + k] : (int)i;
        if (v < 0 || v >= nV) { ok = 0; v = 0; }
        out[k] = v;
    }
    if (!ok) atomicOr(bad, 1u);
    return ok;
}

// min / max over the 64 lanes of a wave (every lane takes part)
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, o, 64));
    return x;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, 64));
    return x;
}

// Primitive boxes, plus the scene-wide bounds: each thread reduces the
// primitives of its grid-stride loop, then each workgroup (lane shuffles, then
// the four wave results through LDS), so that one thread per workgroup
// updates the shared record.  Its 13 words share one cache line, whose atomics
// the L2 serialises, so the grid is capped (kBoxBlocks workgroups) rather than
// one workgroup per 256 primitives.
constexpr unsigned kBoxBlocks = 1024;
template <int K>
__global__ void __launch_bounds__(kB)
k_prim_boxes(const float *__restrict__ V, int64_t nV, const int32_t *__restrict__ ids, int64_t n,
             float4 *__restrict__ blo, float4 *__restrict__ bhi, Reduce *red) {
    uint32_t cmn[3], cmx[3], bmn[3], bmx[3], dmx = 0u;
    for (int a = 0; a < 3; ++a) { cmn[a] = bmn[a] = 0xffffffffu; cmx[a] = bmx[a] = 0u; }
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        int id[3];
        load_ids<K>(ids, i, nV, id, &red->bad);
        float lo[3], hi[3];
        for (int a = 0; a < 3; ++a) lo[a] = hi[a] = V[3 * (int64_t)id[0] + a];
        for (int k = 1; k < K; ++k)
            for (int a = 0; a < 3; ++a) {
                float x = V[3 * (int64_t)id[k] + a];
                lo[a] = fminf(lo[a], x);
                hi[a] = fmaxf(hi[a], x);
            }
        blo[i] = make_float4(lo[0], lo[1], lo[2], 0.f);
        bhi[i] = make_float4(hi[0], hi[1], hi[2], 0.f);
        float dd = 0.f;
        for (int a = 0; a < 3; ++a) {
            const uint32_t c = f2o(0.5f * (lo[a] + hi[a]));
            cmn[a] = min(cmn[a], c);
            cmx[a] = max(cmx[a], c);
            bmn[a] = min(bmn[a], f2o(lo[a]));
            bmx[a] = max(bmx[a], f2o(hi[a]));
            float e = hi[a] - lo[a];
            dd = fmaf(e, e, dd);
        }
        dmx = max(dmx, f2o(sqrtf(dd)));
    }
    for (int a = 0; a < 3; ++a) {
        cmn[a] = wave_min_u32(cmn[a]);
        cmx[a] = wave_max_u32(cmx[a]);
        bmn[a] = wave_min_u32(bmn[a]);
        bmx[a] = wave_max_u32(bmx[a]);
    }
    dmx = wave_max_u32(dmx);
    constexpr int kW = kB / 64;
    __shared__ uint32_t part[13][kW];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int a = 0; a < 3; ++a) {
            part[a][w] = cmn[a];
            part[3 + a][w] = cmx[a];
            part[6 + a][w] = bmn[a];
            part[9 + a][w] = bmx[a];
        }
        part[12][w] = dmx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kW; ++k)
            for (int a = 0; a < 3; ++a) {
                cmn[a] = min(cmn[a], part[a][k]);
                cmx[a] = max(cmx[a], part[3 + a][k]);
                bmn[a] = min(bmn[a], part[6 + a][k]);
                bmx[a] = max(bmx[a], part[9 + a][k]);
            }
        for (int k = 1; k < kW; ++k) dmx = max(dmx, part[12][k]);
        for (int a = 0; a < 3; ++a) {
            atomicMin(&red->cmin[a], cmn[a]);
            atomicMax(&red->cmax[a], cmx[a]);
            atomicMin(&red->bmin[a], bmn[a]);
            atomicMax(&red->bmax[a], bmx[a]);
        }
        atomicMax(&red->diam, dmx);
    }
}

__global__ void __launch_bounds__(kB)
k_check_ids(const int32_t *__restrict__ ids, int64_t m, int64_t nV, uint32_t bit, Reduce *red) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= m) return;
    int v = ids[i];
    if (v < 0 || v >= nV) atomicOr(&red->bad, bit);
}

__device__ inline uint64_t spread21(uint64_t x) {
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

__global__ void __launch_bounds__(kB)
k_morton(const float4 *__restrict__ blo, const float4 *__restrict__ bhi, int64_t n,
         const Reduce *red, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    float4 l = blo[i], h = bhi[i];
    float c[3] = {0.5f * (l.x + h.x), 0.5f * (l.y + h.y), 0.5f * (l.z + h.z)};
    uint64_t code = 0;
    for (int a = 0; a < 3; ++a) {
        float mn = o2f(red->cmin[a]), mx = o2f(red->cmax[a]);
        float ext = mx - mn;
        float u = ext > 0.f ? (c[a] - mn) / ext : 0.f;
        u = fminf(fmaxf(u, 0.f), 1.f);
        uint64_t q = (uint64_t)fminf(u * 2097152.f, 2097151.f);
        code |= spread21(q) << (2 - a);
    }
    keys[i] = code;
    vals[i] = (uint32_t)i;
}

// Karras (2012) radix tree: internal nodes 0..n-2, leaf k has id n-1+k.
__device__ inline int delta(const uint64_t *keys, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = keys[i], b = keys[j];
    if (a == b) return 64 + __clz((uint32_t)(i ^ j));
    return __clzll(a ^ b);
}

__global__ void __launch_bounds__(kB)
k_karras(const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ left,
         int32_t *__restrict__ right, int32_t *__restrict__ first, int32_t *__restrict__ last,
         int32_t *__restrict__ parent) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(keys, n, i, i - d);
    int64_t lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = delta(keys, n, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t lc = (lo == gamma) ? (int32_t)(n - 1 + gamma) : (int32_t)gamma;
    int32_t rc = (hi == gamma + 1) ? (int32_t)(n - 1 + gamma + 1) : (int32_t)(gamma + 1);
    left[i] = lc;
    right[i] = rc;
    first[i] = (int32_t)lo;
    last[i] = (int32_t)hi;
    parent[lc] = (int32_t)i;
    parent[rc] = (int32_t)i;
    if (i == 0) parent[0] = -1;
}

// Bottom-up refit in two launches.  A node's box is formed by the second of
// its two children to finish (a counter per node orders the two), from the
// children's boxes.  The release/acquire that orders one thread's box write
// before another's read is cheap inside a workgroup, but between workgroups,
// which may run on different XCDs with separate L2 caches, it writes back and
// invalidates the whole L2 on every node.  So the first launch refits only the
// nodes whose leaves all belong to one workgroup's unit of kRU consecutive
// leaves (each thread takes kRU / kRB of them in turn); a finished child whose
// parent spans several units is appended to a list instead.  The second
// launch, a single workgroup, refits the nodes above from that list (the
// first launch's boxes are visible after the launch boundary, and its own
// threads synchronise at workgroup scope).  Large units keep that list short:
// it holds the finished children of the nodes that span units, which are
// few per unit.
constexpr int kRB = 1024;
constexpr int64_t kRU = 16 * kRB;

__device__ __forceinline__ void refit_node(int32_t cur, const int32_t *__restrict__ left,
                                           const int32_t *__restrict__ right, float4 *nlo, float4 *nhi) {
    const float4 al = nlo[left[cur]], ah = nhi[left[cur]];
    const float4 bl = nlo[right[cur]], bh = nhi[right[cur]];
    nlo[cur] = make_float4(fminf(al.x, bl.x), fminf(al.y, bl.y), fminf(al.z, bl.z), 0.f);
    nhi[cur] = make_float4(fmaxf(ah.x, bh.x), fmaxf(ah.y, bh.y), fmaxf(ah.z, bh.z), 0.f);
}

__global__ void __launch_bounds__(kRB)
k_refit_local(const float4 *__restrict__ plo, const float4 *__restrict__ phi,
              const uint32_t *__restrict__ order, int64_t n, const int32_t *__restrict__ left,
              const int32_t *__restrict__ right, const int32_t *__restrict__ parent,
              const int32_t *__restrict__ first, const int32_t *__restrict__ last,
              uint32_t *__restrict__ flag, float4 *nlo, float4 *nhi, int32_t *__restrict__ ready,
              uint32_t *__restrict__ n_ready) {
    // leaves [wlo, whi] belong to this workgroup
    const int64_t wlo = (int64_t)blockIdx.x * kRU, whi = wlo + kRU - 1;
    for (int64_t k = wlo + threadIdx.x; k <= whi && k < n; k += kRB) {
        int32_t node = (int32_t)(n - 1 + k);
        const uint32_t p = order[k];
        nlo[node] = plo[p];
        nhi[node] = phi[p];
        if (n == 1) return;   // the leaf is the root (no parent links are built)
        int32_t cur = parent[node];
        while (cur >= 0) {
            if (first[cur] < wlo || last[cur] > whi) {
                // the parent spans several units: left to the second launch
                const uint32_t slot = __hip_atomic_fetch_add(n_ready, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ready[slot] = node;
                break;
            }
            const uint32_t old = __hip_atomic_fetch_add(&flag[cur], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;   // the sibling subtree is not finished yet
            refit_node(cur, left, right, nlo, nhi);
            node = cur;
            cur = parent[cur];   // the next counter update releases this box
        }
    }
}

__global__ void __launch_bounds__(kRB)
k_refit_upper(const int32_t *__restrict__ left, const int32_t *__restrict__ right,
              const int32_t *__restrict__ parent, uint32_t *__restrict__ flag, float4 *nlo, float4 *nhi,
              const int32_t *__restrict__ ready, const uint32_t *__restrict__ n_ready) {
    const uint32_t m = *n_ready;
    for (uint32_t e = threadIdx.x; e < m; e += kRB) {
        int32_t cur = parent[ready[e]];
        while (cur >= 0) {
            const uint32_t old = __hip_atomic_fetch_add(&flag[cur], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == 0) break;
            refit_node(cur, left, right, nlo, nhi);
            cur = parent[cur];
        }
    }
}

// log(count) from FP64, rounded to the nearest float
// log n_B in fixed point with kLogFracBits fractional bits: exact to 2^-27
// (an FP32 log n_B would be off by up to 2^-21 for n_B near 2^26, i.e. a
// relative error of 5e-7 in a far-field weight); n_B <= 2^26 keeps the value
// below 18.03 * 2^26 < 2^31, a non-negative int32 (leaves store a negative one)
__device__ inline int32_t log_count_fx(int64_t c) {
    return __double2int_rn(log((double)c) * (double)(1 << kLogFracBits));
}

__global__ void __launch_bounds__(kB)
k_dfs_layout(int64_t n, const int32_t *__restrict__ left, const int32_t *__restrict__ first,
             const int32_t *__restrict__ last, const int32_t *__restrict__ parent,
             const float4 *__restrict__ blo, const float4 *__restrict__ bhi,
             float4 *__restrict__ out_lo, float4 *__restrict__ out_hi) {
    int64_t x = (int64_t)blockIdx.x * kB + threadIdx.x;
    int64_t total = 2 * n - 1;
    if (x >= total) return;
    bool leaf = x >= n - 1;
    int64_t l = leaf ? x - (n - 1) : first[x];
    int64_t cnt = leaf ? 1 : (int64_t)last[x] - first[x] + 1;
    int64_t turns = 0;
    int64_t cur = x;
    while (true) {
        int32_t p = (cur == 0 && n > 1) ? -1 : (n == 1 ? -1 : parent[cur]);
        if (p < 0) break;
        if (left[p] == cur) ++turns;
        cur = p;
    }
    int64_t pos = 2 * l + turns;
    int64_t esc = pos + 2 * cnt - 1;
    int32_t esc32 = esc >= total ? -1 : (int32_t)esc;
    float4 a = blo[x], b = bhi[x];
    a.w = __int_as_float(esc32);
    b.w = __int_as_float(leaf ? (int32_t)(0x80000000u | (uint32_t)l) : log_count_fx(cnt));
    out_lo[2 * pos] = a;   // records interleaved: lo, hi of a node share a cache line
    out_hi[2 * pos] = b;
}

// ---------------------------------------------------------------------------
// valences and weight data (App. C), counted within each class
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kB)
k_count(const int32_t *__restrict__ ids, int64_t m, int64_t nV, uint32_t *__restrict__ cnt) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= m) return;
    int v = ids[i];
    if (v >= 0 && v < nV) atomicAdd(&cnt[v], 1u);
}

__global__ void __launch_bounds__(kB)
k_edge_weights(const int32_t *__restrict__ E, int64_t nE, int64_t nV,
               const uint32_t *__restrict__ cnt, float *__restrict__ wt, Reduce *red) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    uint32_t vmax = 0;
    if (i < nE) {
        int a = E[2 * i], b = E[2 * i + 1];
        if (a >= 0 && a < nV && b >= 0 && b < nV) {
            uint32_t na = cnt[a], nb = cnt[b];
            wt[2 * i] = 1.0f / (float)na;
            wt[2 * i + 1] = 1.0f / (float)nb;
            vmax = na > nb ? na : nb;
        }
    }
    vmax = wave_max_u32(vmax);   // one atomic per wave
    if ((threadIdx.x & 63) == 0) atomicMax(&red->maxv, vmax);
}

__global__ void __launch_bounds__(kB)
k_tri_edge_keys(const int32_t *__restrict__ T, int64_t nT, int64_t nV, uint64_t *__restrict__ keys,
                uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= 3 * nT) return;
    int64_t t = i / 3;
    int s = (int)(i - 3 * t);
    int64_t a = T[3 * t + s], b = T[3 * t + (s + 1) % 3];
    a = a < 0 ? 0 : (a >= nV ? 0 : a);
    b = b < 0 ? 0 : (b >= nV ? 0 : b);
    int64_t lo = a < b ? a : b, hi = a < b ? b : a;
    keys[i] = (uint64_t)lo * (uint64_t)nV + (uint64_t)hi;
    vals[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(kB)
k_edge_runs(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t m,
            uint32_t *__restrict__ ecount) {
    int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (j >= m) return;
    if (j > 0 && keys[j - 1] == keys[j]) return;   // not the head of a run
    int64_t L = 1;
    while (j + L < m && keys[j + L] == keys[j]) ++L;
    for (int64_t t = 0; t < L; ++t) ecount[vals[j + t]] = (uint32_t)L;
}

__global__ void __launch_bounds__(kB)
k_tri_weights(const int32_t *__restrict__ T, int64_t nT, int64_t nV,
              const uint32_t *__restrict__ vcnt, const uint32_t *__restrict__ ecount,
              float *__restrict__ wt, uint32_t *__restrict__ present, Reduce *red) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    const bool live = i < nT;
    uint32_t v = 0, e = 0;
    if (live) {
        for (int s = 0; s < 3; ++s) {
            int a = T[3 * i + s];
            if (a >= 0 && a < nV) v = max(v, vcnt[a]);
            e = max(e, ecount[3 * i + s]);
        }
        if (v <= 1) {
            wt[3 * i] = 1.f; wt[3 * i + 1] = 1.f; wt[3 * i + 2] = 1.f;
        } else {
            wt[3 * i] = 1.0f / (float)v;
            wt[3 * i + 1] = 1.0f / (float)e;
            wt[3 * i + 2] = (float)((double)(v - 1) / (double)v);
        }
    }
    // one atomic per wave for the largest valence; the (v, e) class bits are
    // set by one lane per distinct class in the wave (usually one)
    uint32_t vmax = wave_max_u32(v);
    const int lane = threadIdx.x & 63;
    if (lane == 0) atomicMax(&red->maxv, vmax);
    const bool fits = v < 1024 && e < 1024;
    if (live && !fits) atomicOr(&red->bad, 2u);
    const uint32_t bit = v * 1024 + e;
    bool pending = live && fits;
    while (true) {
        uint64_t m = __ballot(pending);
        if (m == 0) break;
        int leader = __ffsll((unsigned long long)m) - 1;
        uint32_t lb = (uint32_t)__shfl((int)bit, leader, 64);
        if (pending && bit == lb) {
            if (lane == leader) atomicOr(&present[lb >> 5], 1u << (lb & 31));
            pending = false;
        }
    }
}

template <int K>
__global__ void __launch_bounds__(kB)
k_leaf_records(const float *__restrict__ V, const int32_t *__restrict__ ids,
               const uint32_t *__restrict__ order, const float *__restrict__ wt,
               const int32_t *__restrict__ cls, int64_t n, float4 *__restrict__ leaf,
               int32_t *__restrict__ prim_id) {
    int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k >= n) return;
    uint32_t p = order[k];
    prim_id[k] = (int32_t)p;
    if (K == 1) {
        int64_t v = ids ? ids[p] : (int64_t)p;
        leaf[k] = make_float4(V[3 * v], V[3 * v + 1], V[3 * v + 2], 1.f);
        return;
    }
    for (int s = 0; s < K; ++s) {
        int v = ids[(int64_t)p * K + s];
        // edges: (1/N0, 1/N1); triangles: (class id bits, 1/v, 1/e)
        float w = (K == 3) ? (s == 0 ? __int_as_float(cls[p]) : wt[(int64_t)p * K + s - 1])
                           : wt[(int64_t)p * K + s];
        leaf[k * K + s] = make_float4(V[3 * (int64_t)v], V[3 * (int64_t)v + 1],
                                      V[3 * (int64_t)v + 2], w);
    }
}

// valence class id of each triangle from its stored (1/v, 1/e)
__global__ void __launch_bounds__(kB)
k_tri_class(const float *__restrict__ wt, int64_t nT, const int32_t *__restrict__ lut,
            int32_t *__restrict__ cls) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= nT) return;
    int v = (int)rintf(1.f / wt[3 * i]), e = (int)rintf(1.f / wt[3 * i + 1]);
    v = min(max(v, 0), 1023);
    e = min(max(e, 0), 1023);
    cls[i] = lut[v * 1024 + e];
}

template <typename T>
int dalloc(T **p, int64_t count, hipStream_t s, int64_t *acc = nullptr) {
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    SD_TRY(dev_malloc_async((void **)p, bytes, s, "sd_build_bvh"));
    if (acc) *acc += (int64_t)bytes;
    return SD_OK;
}

int bits_for(uint64_t maxval) {
    int b = 1;
    while (b < 64 && (maxval >> b)) ++b;
    return b;
}

}  // namespace

// Builds one class hierarchy into sc.  ids: n x K vertex ids (device), or
// nullptr for "vertex i" (points only).
template <int K>
static int build_class(sd_scene *sc, int cls, const float *V, int64_t nV, const int32_t *ids,
                       int64_t n, const float *wt, hipStream_t s, Reduce *red_dev,
                       Reduce *red_host, const int32_t *tri_cls = nullptr) {
    if (n <= 0) return SD_OK;
    // node records are addressed with 32-bit byte offsets: 2n - 1 nodes x 32 B < 2^32
    if (n > ((int64_t)1 << 26)) return fail(SD_EUNSUPPORTED, "more than 2^26 primitives in a class");
    int64_t nn = 2 * n - 1;
    float4 *plo, *phi, *blo, *bhi;
    uint64_t *keys, *keys2;
    uint32_t *vals, *vals2, *flag;
    int32_t *left, *right, *first, *last, *parent;
    char *temp;
    size_t tb = radix_sort_temp_bytes(n);
    AsyncScratch tmp(s);
    SD_TRY(tmp.alloc(&plo, n)); SD_TRY(tmp.alloc(&phi, n));
    SD_TRY(tmp.alloc(&blo, nn)); SD_TRY(tmp.alloc(&bhi, nn));
    SD_TRY(tmp.alloc(&keys, n)); SD_TRY(tmp.alloc(&keys2, n));
    SD_TRY(tmp.alloc(&vals, n)); SD_TRY(tmp.alloc(&vals2, n));
    SD_TRY(tmp.alloc(&flag, nn + 1));
    uint32_t *n_ready = flag + nn;   // the count of the refit's list, cleared with the counters
    int32_t *ready;                  // a node has two children: at most 2 (n - 1) entries
    SD_TRY(tmp.alloc(&ready, std::max<int64_t>(1, 2 * (n - 1))));
    SD_TRY(tmp.alloc(&left, nn)); SD_TRY(tmp.alloc(&right, nn));
    SD_TRY(tmp.alloc(&first, nn)); SD_TRY(tmp.alloc(&last, nn)); SD_TRY(tmp.alloc(&parent, nn));
    SD_TRY(tmp.alloc(&temp, (int64_t)tb));

    // reset the reduction record: mins to +max, maxes to 0 (ordered encoding)
    Reduce init;
    for (int a = 0; a < 3; ++a) {
        init.cmin[a] = init.bmin[a] = 0xffffffffu;
        init.cmax[a] = init.bmax[a] = 0u;
    }
    init.diam = 0; init.bad = red_host->bad; init.maxv = red_host->maxv; init.pad = 0;
    SD_HIP(hipMemcpyAsync(red_dev, &init, sizeof(Reduce), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_prim_boxes<K>, dim3(std::min(grid_for(n), kBoxBlocks)), dim3(kB), 0, s, V, nV, ids, n, plo, phi,
                       red_dev);
    hipLaunchKernelGGL(k_morton, dim3(grid_for(n)), dim3(kB), 0, s, plo, phi, n, red_dev, keys, vals);
    SD_TRY(radix_sort_pairs(keys, vals, keys2, vals2, n, 63, temp, s));
    SD_HIP(hipMemsetAsync(flag, 0, (nn + 1) * sizeof(uint32_t), s));
    if (n > 1)
        hipLaunchKernelGGL(k_karras, dim3(grid_for(n - 1)), dim3(kB), 0, s, keys, n, left, right,
                           first, last, parent);
    hipLaunchKernelGGL(k_refit_local, dim3((unsigned)((n + kRU - 1) / kRU)), dim3(kRB), 0, s, plo, phi, vals,
                       n, left, right, parent, first, last, flag, blo, bhi, ready, n_ready);
    hipLaunchKernelGGL(k_refit_upper, dim3(1), dim3(kRB), 0, s, left, right, parent, flag, blo, bhi, ready,
                       n_ready);
    int64_t acc = 0;
    SD_TRY(dalloc(&sc->lo[cls], 2 * nn, s, &acc));
    sc->hi[cls] = sc->lo[cls] + 1;
    SD_TRY(dalloc(&sc->prim_id[cls], n, s, &acc));
    hipLaunchKernelGGL(k_dfs_layout, dim3(grid_for(nn)), dim3(kB), 0, s, n, left, first, last,
                       parent, blo, bhi, sc->lo[cls], sc->hi[cls]);
    SD_TRY(dalloc(&sc->leaf[cls], n * K, s, &acc));
    hipLaunchKernelGGL(k_leaf_records<K>, dim3(grid_for(n)), dim3(kB), 0, s, V, ids, vals, wt,
                       tri_cls, n, sc->leaf[cls], sc->prim_id[cls]);
    SD_HIP(hipGetLastError());
    SD_HIP(hipMemcpyAsync(red_host, red_dev, sizeof(Reduce), hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    sc->n[cls] = n;
    sc->n_nodes[cls] = nn;
    sc->device_bytes += acc;
    float dm = o2f(red_host->diam);
    sc->diam_max = std::max(sc->diam_max, (double)dm);
    float bx[6];
    for (int a = 0; a < 3; ++a) { bx[a] = o2f(red_host->bmin[a]); bx[3 + a] = o2f(red_host->bmax[a]); }
    bool first_class = sc->n[0] + sc->n[1] + sc->n[2] == n;
    for (int a = 0; a < 3; ++a) {
        sc->box[a] = first_class ? bx[a] : std::min(sc->box[a], bx[a]);
        sc->box[3 + a] = first_class ? bx[3 + a] : std::max(sc->box[3 + a], bx[3 + a]);
    }
    return SD_OK;
}

int build_scene(sd_scene *sc, const float *V, int64_t nV, const int32_t *P, int64_t nP,
                const int32_t *E, int64_t nE, const int32_t *T, int64_t nT, uint32_t flags,
                hipStream_t s) {
    AsyncScratch tmp(s);
    Reduce *red_dev;
    SD_TRY(tmp.alloc(&red_dev, 1));
    Reduce red_host;
    memset(&red_host, 0, sizeof(red_host));

    // every index is checked before any kernel dereferences it
    SD_HIP(hipMemcpyAsync(red_dev, &red_host, sizeof(Reduce), hipMemcpyHostToDevice, s));
    if (P && nP > 0)
        hipLaunchKernelGGL(k_check_ids, dim3(grid_for(nP)), dim3(kB), 0, s, P, nP, nV, 1u, red_dev);
    if (nE > 0)
        hipLaunchKernelGGL(k_check_ids, dim3(grid_for(2 * nE)), dim3(kB), 0, s, E, 2 * nE, nV, 2u, red_dev);
    if (nT > 0)
        hipLaunchKernelGGL(k_check_ids, dim3(grid_for(3 * nT)), dim3(kB), 0, s, T, 3 * nT, nV, 4u, red_dev);
    SD_HIP(hipGetLastError());
    SD_HIP(hipMemcpyAsync(&red_host, red_dev, sizeof(Reduce), hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    if (red_host.bad) {
        const char *what = (red_host.bad & 1u) ? "point" : (red_host.bad & 2u) ? "edge" : "triangle";
        return fail(SD_EINVAL, std::string("sd_build_bvh: ") + what + " index outside [0, nV)");
    }

    // points: w = 1
    SD_TRY(build_class<1>(sc, 0, V, nV, P, nP, nullptr, s, red_dev, &red_host));

    // edges: 1/|N_k| at both ends (App. C.2); A_E = max_k |N_k|
    if (nE > 0) {
        uint32_t *cnt;
        float *wt;
        SD_TRY(tmp.alloc(&cnt, nV));
        SD_TRY(dalloc(&wt, 2 * nE, s));
        sc->wt[1] = wt;   // owned by the scene from here (freed with it on failure)
        sc->device_bytes += 2 * nE * sizeof(float);
        SD_HIP(hipMemsetAsync(cnt, 0, nV * sizeof(uint32_t), s));
        red_host.maxv = 0;
        SD_HIP(hipMemcpyAsync(red_dev, &red_host, sizeof(Reduce), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_count, dim3(grid_for(2 * nE)), dim3(kB), 0, s, E, 2 * nE, nV, cnt);
        hipLaunchKernelGGL(k_edge_weights, dim3(grid_for(nE)), dim3(kB), 0, s, E, nE, nV, cnt, wt,
                           red_dev);
        SD_HIP(hipMemcpyAsync(&red_host, red_dev, sizeof(Reduce), hipMemcpyDeviceToHost, s));
        SD_HIP(hipStreamSynchronize(s));
        sc->A[1] = (double)std::max<uint32_t>(red_host.maxv, 1u);
        SD_TRY(build_class<2>(sc, 1, V, nV, E, nE, wt, s, red_dev, &red_host));
    }

    // triangles: 1/v, 1/e, (v-1)/v (App. C.3); A_T strict or literal
    if (nT > 0) {
        uint32_t *vcnt, *ecnt, *present, *vals, *vals2;
        uint64_t *keys, *keys2;
        float *wt;
        char *temp;
        int64_t m = 3 * nT;
        const int64_t nbits = 1024 * 1024 / 32;
        SD_TRY(tmp.alloc(&vcnt, nV));
        SD_TRY(tmp.alloc(&ecnt, m));
        SD_TRY(tmp.alloc(&present, nbits));
        SD_TRY(tmp.alloc(&keys, m)); SD_TRY(tmp.alloc(&keys2, m));
        SD_TRY(tmp.alloc(&vals, m)); SD_TRY(tmp.alloc(&vals2, m));
        SD_TRY(dalloc(&wt, 3 * nT, s));
        sc->wt[2] = wt;   // owned by the scene from here (freed with it on failure)
        sc->device_bytes += 3 * nT * sizeof(float);
        size_t tb = radix_sort_temp_bytes(m);
        SD_TRY(tmp.alloc(&temp, (int64_t)tb));
        SD_HIP(hipMemsetAsync(vcnt, 0, nV * sizeof(uint32_t), s));
        SD_HIP(hipMemsetAsync(present, 0, nbits * sizeof(uint32_t), s));
        red_host.maxv = 0;
        SD_HIP(hipMemcpyAsync(red_dev, &red_host, sizeof(Reduce), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_count, dim3(grid_for(m)), dim3(kB), 0, s, T, m, nV, vcnt);
        hipLaunchKernelGGL(k_tri_edge_keys, dim3(grid_for(m)), dim3(kB), 0, s, T, nT, nV, keys, vals);
        SD_TRY(radix_sort_pairs(keys, vals, keys2, vals2, m, bits_for((uint64_t)nV * (uint64_t)nV),
                                temp, s));
        hipLaunchKernelGGL(k_edge_runs, dim3(grid_for(m)), dim3(kB), 0, s, keys, vals, m, ecnt);
        hipLaunchKernelGGL(k_tri_weights, dim3(grid_for(nT)), dim3(kB), 0, s, T, nT, nV, vcnt, ecnt,
                           wt, present, red_dev);
        std::vector<uint32_t> pres(nbits);
        SD_HIP(hipMemcpyAsync(pres.data(), present, nbits * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        SD_HIP(hipMemcpyAsync(&red_host, red_dev, sizeof(Reduce), hipMemcpyDeviceToHost, s));
        SD_HIP(hipStreamSynchronize(s));
        if (red_host.bad & 2u)
            return fail(SD_EUNSUPPORTED, "sd_build_bvh: triangle valence above 1023");
        double A = std::max<uint32_t>(red_host.maxv, 1u);
        sc->A_T_literal = A;
        int ncls = 0;
        std::vector<int32_t> lut(1024 * 1024, 0);
        std::vector<double> table;
        for (int64_t b = 0; b < nbits * 32; ++b) {
            if (!((pres[b >> 5] >> (b & 31)) & 1u)) continue;
            int v = (int)(b / 1024), e = (int)(b % 1024);
            lut[b] = ncls++;
            double mono[36];
            triangle_monomial_horner(v, e, mono);
            table.insert(table.end(), mono, mono + 36);
            // the largest Bernstein coefficient bounds w~ from above (convex hull)
            float bern[36];
            triangle_bernstein(v, e, bern);
            for (float c : bern) sc->tri_wmax = std::max(sc->tri_wmax, (double)c);
            if (v <= 1) continue;
            double wmin = triangle_weight_min_f64(v, e);
            if (!(wmin > 0))
                return fail(SD_EUNSUPPORTED, "sd_build_bvh: triangle weight polynomial not positive"
                                             " for valences (" + std::to_string(v) + "," +
                                             std::to_string(e) + ")");
            A = std::max(A, 1.0 / wmin);
        }
        sc->n_tri_classes = ncls;
        sc->A[2] = (flags & SD_BUILD_A_PAPER_LITERAL) ? sc->A_T_literal : A;
        memcpy(sc->tri_mono0, table.data(), sizeof(sc->tri_mono0));
        int32_t *lut_dev, *tri_cls;
        SD_TRY(tmp.alloc(&lut_dev, 1024 * 1024));
        SD_TRY(tmp.alloc(&tri_cls, nT));
        int64_t acc = 0;
        SD_TRY(dalloc(&sc->tri_table, (int64_t)table.size(), s, &acc));
        sc->device_bytes += acc;
        SD_HIP(hipMemcpyAsync(lut_dev, lut.data(), lut.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        SD_HIP(hipMemcpyAsync(sc->tri_table, table.data(), table.size() * sizeof(double),
                              hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_tri_class, dim3(grid_for(nT)), dim3(kB), 0, s, wt, nT, lut_dev, tri_cls);
        SD_TRY(build_class<3>(sc, 2, V, nV, T, nT, wt, s, red_dev, &red_host, tri_cls));
    }
    SD_HIP(hipStreamSynchronize(s));
    return SD_OK;
}

}  // namespace sd
