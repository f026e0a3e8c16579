// Learned surrogate of the smooth distance (Eq. 3): a Fourier-feature SiLU
// network, trained on values the exact method produces and evaluated on the
// BF16 matrix cores with FP32 accumulation.  Queries whose surrogate value
// lies in a band around the zero isosurface go back to the exact Barnes-Hut
// evaluation (Alg. 1, Alg. 2).  The paper has no learned part; this file is
// the library's extension of it.
//
// Network:  gamma(x) = [sin 2 pi B x, cos 2 pi B x]  (B: 64 x 3)
//           z_l = W_l a_{l-1} + b_l,  a_l = silu(z_l)  (l = 1..4, width 256)
//           y = w5 . a_4 + b5
// Matrices W_l and w5 are used in BF16 (rounded to nearest even from the FP32
// masters); biases stay FP32.
//
// Inference kernel (value and input gradient, reverse mode):
//   One wave owns 32 queries (two 16-query blocks) and computes each layer as
//   (out features x queries) += W (out x in) * A (in x queries) with
//   v_mfma_f32_16x16x32_bf16: weight fragments are the A operand, activations
//   the B operand.  A 16x16 accumulator tile holds, in lane l and register r,
//   feature 4 (l / 16) + r of the tile for query l % 16.  The K index of the
//   next layer is permuted so that tiles 2k and 2k+1 of one layer's output are,
//   lane for lane, the B operand of K-block k of the next layer: the
//   activations never leave the registers.  The weight fragments are packed
//   in that permuted order once per weight update and streamed through LDS in
//   16 KB chunks shared by the workgroup's four waves.  The derivative of
//   silu at every hidden unit is kept in registers (BF16) for the backward
//   sweep; the last layer's never needs storing.
//   The network runs in a base-2 scaled domain: a'_l = log2(e) a_l, so that
//   the logistic function is 1 / (1 + 2^-z') with z' the scaled
//   pre-activation (one exp2 and one rcp per unit); scaling the first layer's
//   input and the biases by log2(e) and w5 by 1/log2(e) leaves every weight
//   matrix unchanged.
//
// Training kernels: plain tiled BF16 MFMA GEMMs over a batch (forward with a
// fused bias + silu epilogue, backward input products with the fused silu'
// product, weight gradients as split-K products reduced in a fixed order),
// a loss kernel, column sums, and Adam on FP32 master weights.
#include <math.h>

#include <type_traits>
#include <utility>
#include <vector>

#include "sd_internal.h"

namespace sd {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int NF = 64;          // Fourier frequencies
constexpr int NIN = 2 * NF;     // first-layer inputs
constexpr int WD = 256;         // hidden width
constexpr int64_t NPAR = 230657;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kInvLog2e = 0.6931471805599453f;

__host__ __device__ constexpr int64_t off_W(int l) {   // l = 1..4
    return l == 1 ? 0 : (int64_t)WD * NIN + WD + (int64_t)(l - 2) * (WD * WD + WD);
}
__host__ __device__ constexpr int fan_in(int l) { return l == 1 ? NIN : WD; }
__host__ __device__ constexpr int64_t off_b(int l) { return off_W(l) + (int64_t)WD * fan_in(l); }
constexpr int64_t OFF_W5 = off_b(4) + WD;
constexpr int64_t OFF_B5 = OFF_W5 + WD;
static_assert(OFF_B5 + 1 == NPAR, "parameter layout");

// inference weight stream: 28 chunks of 32 fragments x 64 lanes x 16 bytes
// (32 KB): four output tiles of 8 K-blocks, or eight of 4 for the first layer
constexpr int kChunkU4 = 32 * 64;
constexpr int kChunksFwd = 2 + 3 * 4;        // W1, W2..W4
constexpr int kChunks = kChunksFwd + 3 * 4 + 2;  // then W4..W2 transposed, W1 transposed

__device__ __forceinline__ uint32_t pk2(float lo, float hi) {
    f32x2 v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ __bf16 to_bf(float f) { return (__bf16)f; }

__device__ __forceinline__ f32x4 mma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// sin and cos of 2 pi t with the hardware sine (argument in revolutions)
__device__ __forceinline__ void sincos_rev(float t, float &s, float &c) {
    float r = t - rintf(t);
    s = __builtin_amdgcn_sinf(r);
    c = __builtin_amdgcn_cosf(r);
}

// K index of the permuted order: K-block kb, lane group g = lane / 16, j = 0..7
__host__ __device__ __forceinline__ int perm_k(int kb, int g, int j) {
    return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

// ---------------------------------------------------------------------------
// weight packing (after every update)
// ---------------------------------------------------------------------------
__global__ void k_pack_infer(const float *__restrict__ th, uint16_t *__restrict__ frag,
                             float *__restrict__ bias_s, float *__restrict__ w5s) {
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n_el = (int64_t)kChunks * kChunkU4 * 8;
    if (e < n_el) {
        int c = (int)(e / (kChunkU4 * 8));
        int rem = (int)(e % (kChunkU4 * 8));
        int f = rem / 512, lane = (rem / 8) % 64, j = rem % 8;
        int g = lane >> 4, li = lane & 15;
        int64_t src;
        if (c < 2) {                           // W1 forward: 8 tiles x 4 K-blocks per chunk
            int t = 8 * c + f / 4, kb = f % 4;
            src = off_W(1) + (int64_t)(16 * t + li) * NIN + perm_k(kb, g, j);
        } else if (c < kChunksFwd) {           // W2..W4 forward: 4 tiles x 8 K-blocks
            int l = 2 + (c - 2) / 4, t = 4 * ((c - 2) % 4) + f / 8, kb = f % 8;
            src = off_W(l) + (int64_t)(16 * t + li) * WD + perm_k(kb, g, j);
        } else if (c < kChunksFwd + 12) {      // W4..W2 transposed: tiles of inputs, K = outputs
            int l = 4 - (c - kChunksFwd) / 4, t = 4 * ((c - kChunksFwd) % 4) + f / 8, kb = f % 8;
            src = off_W(l) + (int64_t)perm_k(kb, g, j) * WD + 16 * t + li;
        } else {                               // W1 transposed: 8 tiles of gamma features
            int t = 4 * (c - kChunksFwd - 12) + f / 8, kb = f % 8;
            src = off_W(1) + (int64_t)perm_k(kb, g, j) * NIN + 16 * t + li;
        }
        frag[e] = __builtin_bit_cast(uint16_t, to_bf(th[src]));
    }
    if (e < 4 * WD) bias_s[e] = kLog2e * th[off_b(1 + (int)(e / WD)) + e % WD];
    if (e < WD) w5s[e] = (float)to_bf(th[OFF_W5 + e]) * kInvLog2e;
}

// BF16 copies for training: rows (out x in) and transposes (in x out)
__global__ void k_pack_train(const float *__restrict__ th, __bf16 *__restrict__ wr,
                             __bf16 *__restrict__ wc) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= NPAR) return;
    __bf16 b = to_bf(th[i]);
    wr[i] = b;
    for (int l = 1; l <= 4; ++l) {
        int64_t o = off_W(l), n = (int64_t)WD * fan_in(l);
        if (i >= o && i < o + n) {
            int64_t r = (i - o) / fan_in(l), k = (i - o) % fan_in(l);
            wc[o + k * WD + r] = b;
        }
    }
}

// ---------------------------------------------------------------------------
// inference: value (and input gradient), optional routing flag
// ---------------------------------------------------------------------------
struct MlpArgs {
    const u32x4 *frag;
    const float *bias_s;
    const float *w5s;
    const float *b5;       // device scalar
    const float *Bf;       // 64 x 3
    const float *Q;
    int64_t nq;
    float *d_out;
    float *g_out;          // nullptr: value only
    uint8_t *routed;       // nullptr: no routing flag
    float band;            // routed[i] = |d_i| < band
    const float *label;    // certification: |d_i - label_i| -> err_out
    float *err_out;
    // local certificate: routed[i] = |d_i| < band0 + eps of the query's cell
    // (queries outside the grid box use band); cell_eps == nullptr: band only
    const float *cell_eps;
    float band0;
    int grid;
    float glo[3], ginv[3];
};

// cell of a point in the certificate grid, or -1 outside the (closed) grid box
__device__ __forceinline__ int cert_cell(const MlpArgs &A, float x, float y, float z) {
    float p[3] = {x, y, z};
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float t = (p[a] - A.glo[a]) * A.ginv[a];
        if (!(t >= 0.f && t <= (float)A.grid)) return -1;
        c[a] = min((int)t, A.grid - 1);
    }
    return (c[0] * A.grid + c[1]) * A.grid + c[2];
}

// Weight stream through LDS: three 32 KB slots.  Chunk k is loaded straight
// into slot k % 3 (global_load_lds, lane i -> slot base + 16 i) at the start
// of chunk k - 2; the barrier that ends chunk k - 1 waits for those loads.  So
// while chunk k is being computed, chunk k + 1 is readable as well (the next
// tile's fragments can be read ahead across a chunk boundary) and slot
// (k + 2) % 3, last read during chunk k - 1, is being refilled.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(3))) char lds_char_t;
constexpr int kSlots = 3;

template <int NW>
struct Pipe {
    u32x4 *lds;
    const u32x4 *src;
    int wave, lane;
    template <int C> __device__ __forceinline__ void load() {
        constexpr int per_wave = kChunkU4 / NW;
        const u32x4 *g = src + (int64_t)C * kChunkU4 + wave * per_wave + lane;
        lds_char_t *l = (lds_char_t *)(lds + (C % kSlots) * kChunkU4 + wave * per_wave);
#pragma unroll
        for (int k = 0; k < per_wave / 64; ++k)
            __builtin_amdgcn_global_load_lds((const void *)(g + 64 * k), (lds_void_t *)(l + 1024 * k), 16, 0, 0);
    }
    template <int C, int LAST> __device__ __forceinline__ void pre() {
        if constexpr (C + 2 <= LAST) load<C + 2>();
    }
    template <int C> __device__ __forceinline__ const u32x4 *slot() const {
        return lds + (C % kSlots) * kChunkU4;
    }
};

// compile-time loop: f(std::integral_constant<int, i>) for i = 0..N-1
template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F> __device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// One layer in out-tile-major order: tile t's K loop (NKB K-blocks of 32,
// both query blocks), then the epilogue of tile t-1, so that one tile's
// elementwise work overlaps the next tile's matrix products.  Chunks hold TPC
// tiles; chunk C0 + t / TPC.  init(t, acc) sets the accumulator, epi(t, acc)
// consumes it.
template <int C0, int LAST, int NT, int NKB, int TPC, int QBN, int NW, class Init, class Epi>
__device__ __forceinline__ void run_layer(Pipe<NW> &P, const u32x4 (&bin)[8][QBN], int lane,
                                          Init &&init, Epi &&epi) {
    // with one wave per SIMD the next tile's fragments are read a tile ahead;
    // with two, the other wave hides the LDS latency and registers are short
    constexpr bool AHEAD = QBN > 1;
    f32x4 acc[2][QBN];
    u32x4 fr[AHEAD ? 2 : 1][NKB];
    if constexpr (AHEAD) {
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb) fr[0][kb] = P.template slot<C0>()[kb * 64 + lane];
    }
    sfor<NT>([&](auto T) {
        constexpr int t = decltype(T)::value;
        constexpr int c = C0 + t / TPC;
        constexpr int tl = t % TPC;
        constexpr int cur = AHEAD ? (t & 1) : 0;
        if constexpr (tl == 0) P.template pre<c, LAST>();
        if constexpr (AHEAD && t + 1 < NT) {
            constexpr int c1 = C0 + (t + 1) / TPC, tl1 = (t + 1) % TPC;
            const u32x4 *w = P.template slot<c1>() + tl1 * NKB * 64 + lane;
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) fr[(t + 1) & 1][kb] = w[kb * 64];
            __builtin_amdgcn_sched_barrier(0);   // keep the reads a full tile ahead
        }
        if constexpr (!AHEAD) {
            const u32x4 *w = P.template slot<c>() + tl * NKB * 64 + lane;
#pragma unroll
            for (int kb = 0; kb < NKB; ++kb) fr[0][kb] = w[kb * 64];
        }
        init(T, acc[t & 1]);
#pragma unroll
        for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
            for (int qb = 0; qb < QBN; ++qb) acc[t & 1][qb] = mma(fr[cur][kb], bin[kb][qb], acc[t & 1][qb]);
        if constexpr (t > 0) epi(std::integral_constant<int, t - 1>{}, acc[(t - 1) & 1]);
        if constexpr (tl == TPC - 1) __syncthreads();
    });
    epi(std::integral_constant<int, NT - 1>{}, acc[(NT - 1) & 1]);
}

// scaled silu: s = 1 / (1 + 2^-z'), a' = z' s, silu'(z) = s + a' (1 - s) / log2(e)
__device__ __forceinline__ void silu_s(float z, float &a, float &d) {
    float s = __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-z));
    a = z * s;
    d = fmaf(a, fmaf(-s, kInvLog2e, kInvLog2e), s);
}

// tile t of a layer output -> half (t & 1) of K-block t / 2 of the next B operand
template <int t, int QBN>
__device__ __forceinline__ void put_b(u32x4 (&b)[8][QBN], int qb, float v0, float v1, float v2, float v3) {
    b[t >> 1][qb][(t & 1) * 2] = pk2(v0, v1);
    b[t >> 1][qb][(t & 1) * 2 + 1] = pk2(v2, v3);
}

// QBN 16-query blocks per wave, NW waves per workgroup
template <bool GRAD, int QBN, int NW>
__device__ __forceinline__ void mlp_body(const MlpArgs &A, u32x4 *lds) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, li = lane & 15;
    constexpr int LAST = GRAD ? kChunks - 1 : kChunksFwd - 1;

    Pipe<NW> P;
    P.lds = lds;
    P.src = A.frag;
    P.wave = wave;
    P.lane = lane;
    P.template load<0>();
    P.template load<1>();

    const int64_t q0 = (int64_t)blockIdx.x * (NW * 16 * QBN) + wave * (16 * QBN) + li;
    float x[QBN][3];
#pragma unroll
    for (int qb = 0; qb < QBN; ++qb) {
        int64_t q = q0 + 16 * qb;
        bool live = q < A.nq;
#pragma unroll
        for (int a = 0; a < 3; ++a) x[qb][a] = live ? A.Q[3 * q + a] : 0.f;
    }

    // first-layer input: lane holds gamma features 16 t + 4 g + r, t = 0..7
    // (sines for t < 4, cosines of the same frequencies for t >= 4)
    u32x4 bA[8][QBN], bB[8][QBN];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float sn[QBN][4], cs[QBN][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float *b = A.Bf + 3 * (16 * t + 4 * g + r);
            float b0 = b[0], b1 = b[1], b2 = b[2];
#pragma unroll
            for (int qb = 0; qb < QBN; ++qb) {
                float th = fmaf(b0, x[qb][0], fmaf(b1, x[qb][1], b2 * x[qb][2]));
                sincos_rev(th, sn[qb][r], cs[qb][r]);
            }
        }
#pragma unroll
        for (int qb = 0; qb < QBN; ++qb) {
            bA[t >> 1][qb][(t & 1) * 2] = pk2(kLog2e * sn[qb][0], kLog2e * sn[qb][1]);
            bA[t >> 1][qb][(t & 1) * 2 + 1] = pk2(kLog2e * sn[qb][2], kLog2e * sn[qb][3]);
            bA[2 + (t >> 1)][qb][(t & 1) * 2] = pk2(kLog2e * cs[qb][0], kLog2e * cs[qb][1]);
            bA[2 + (t >> 1)][qb][(t & 1) * 2 + 1] = pk2(kLog2e * cs[qb][2], kLog2e * cs[qb][3]);
        }
    }
    __syncthreads();

    uint32_t S1[16][QBN][2], S2[16][QBN][2], S3[16][QBN][2];
    auto bias_init = [&](const float *bias) {
        return [=](auto T, f32x4(&acc)[QBN]) {
            constexpr int t = decltype(T)::value;
            f32x4 v = *(const f32x4 *)(bias + 16 * t + 4 * g);
#pragma unroll
            for (int qb = 0; qb < QBN; ++qb) acc[qb] = v;
        };
    };
    auto zero_init = [](auto, f32x4(&acc)[QBN]) {
#pragma unroll
        for (int qb = 0; qb < QBN; ++qb) acc[qb] = (f32x4){0.f, 0.f, 0.f, 0.f};
    };
    // hidden layer epilogue: next B operand from a', silu' kept for the backward sweep
    auto hidden = [&](u32x4(&bo)[8][QBN], uint32_t(&S)[16][QBN][2]) {
        return [&](auto T, const f32x4(&acc)[QBN]) {
            constexpr int t = decltype(T)::value;
#pragma unroll
            for (int qb = 0; qb < QBN; ++qb) {
                float a[4], d[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) silu_s(acc[qb][r], a[r], d[r]);
                put_b<t, QBN>(bo, qb, a[0], a[1], a[2], a[3]);
                if (GRAD) {
                    S[t][qb][0] = pk2(d[0], d[1]);
                    S[t][qb][1] = pk2(d[2], d[3]);
                }
            }
        };
    };

    run_layer<0, LAST, 16, 4, 8, QBN>(P, bA, lane, bias_init(A.bias_s), hidden(bB, S1));
    run_layer<2, LAST, 16, 8, 4, QBN>(P, bB, lane, bias_init(A.bias_s + WD), hidden(bA, S2));
    run_layer<6, LAST, 16, 8, 4, QBN>(P, bA, lane, bias_init(A.bias_s + 2 * WD), hidden(bB, S3));

    // last hidden layer: output y = (w5 / log2 e) . a'_4 + b5 and the seed of
    // the backward sweep u4 = (w5 / log2 e) silu'(z4)
    float y[QBN];
#pragma unroll
    for (int qb = 0; qb < QBN; ++qb) y[qb] = 0.f;
    run_layer<10, LAST, 16, 8, 4, QBN>(P, bB, lane, bias_init(A.bias_s + 3 * WD), [&](auto T, const f32x4(&acc)[QBN]) {
        constexpr int t = decltype(T)::value;
        f32x4 w = *(const f32x4 *)(A.w5s + 16 * t + 4 * g);
#pragma unroll
        for (int qb = 0; qb < QBN; ++qb) {
            float a[4], d[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                silu_s(acc[qb][r], a[r], d[r]);
                y[qb] = fmaf(a[r], w[r], y[qb]);
            }
            if (GRAD) put_b<t, QBN>(bA, qb, w[0] * d[0], w[1] * d[1], w[2] * d[2], w[3] * d[3]);
        }
    });
#pragma unroll
    for (int qb = 0; qb < QBN; ++qb) {
        y[qb] += __shfl_xor(y[qb], 16);
        y[qb] += __shfl_xor(y[qb], 32);
        y[qb] += *A.b5;
    }

    float gx[QBN][3];
#pragma unroll
    for (int qb = 0; qb < QBN; ++qb) gx[qb][0] = gx[qb][1] = gx[qb][2] = 0.f;
    if constexpr (GRAD) {
        // backward: u_{l-1} = (W_l^T u_l) silu'(z_{l-1})
        auto back = [&](u32x4(&bo)[8][QBN], const uint32_t(&S)[16][QBN][2]) {
            return [&](auto T, const f32x4(&acc)[QBN]) {
                constexpr int t = decltype(T)::value;
#pragma unroll
                for (int qb = 0; qb < QBN; ++qb)
                    put_b<t, QBN>(bo, qb, acc[qb][0] * bf_lo(S[t][qb][0]), acc[qb][1] * bf_hi(S[t][qb][0]),
                             acc[qb][2] * bf_lo(S[t][qb][1]), acc[qb][3] * bf_hi(S[t][qb][1]));
            };
        };
        run_layer<14, LAST, 16, 8, 4, QBN>(P, bA, lane, zero_init, back(bB, S3));   // through W4
        run_layer<18, LAST, 16, 8, 4, QBN>(P, bB, lane, zero_init, back(bA, S2));   // through W3
        run_layer<22, LAST, 16, 8, 4, QBN>(P, bA, lane, zero_init, back(bB, S1));   // through W2
        // through W1: dy/d(a'_0) for the 128 gamma features, all tiles kept
        f32x4 g0[8][QBN];
        run_layer<26, LAST, 8, 8, 4, QBN>(P, bB, lane, zero_init, [&](auto T, const f32x4(&acc)[QBN]) {
            constexpr int t = decltype(T)::value;
#pragma unroll
            for (int qb = 0; qb < QBN; ++qb) g0[t][qb] = acc[qb];
        });
        // dy/dgamma = log2(e) g0; chain through sin and cos of 2 pi b.x
        const float cg = kLog2e * 6.283185307179586f;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float *b = A.Bf + 3 * (16 * t + 4 * g + r);
                float b0 = b[0], b1 = b[1], b2 = b[2];
#pragma unroll
                for (int qb = 0; qb < QBN; ++qb) {
                    float sn, cs;
                    float th = fmaf(b0, x[qb][0], fmaf(b1, x[qb][1], b2 * x[qb][2]));
                    sincos_rev(th, sn, cs);
                    float k = cg * (g0[t][qb][r] * cs - g0[t + 4][qb][r] * sn);
                    gx[qb][0] = fmaf(k, b0, gx[qb][0]);
                    gx[qb][1] = fmaf(k, b1, gx[qb][1]);
                    gx[qb][2] = fmaf(k, b2, gx[qb][2]);
                }
            }
#pragma unroll
        for (int qb = 0; qb < QBN; ++qb)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                gx[qb][a] += __shfl_xor(gx[qb][a], 16);
                gx[qb][a] += __shfl_xor(gx[qb][a], 32);
            }
    }

    if (g == 0) {
#pragma unroll
        for (int qb = 0; qb < QBN; ++qb) {
            int64_t q = q0 + 16 * qb;
            if (q >= A.nq) continue;
            if (A.d_out) A.d_out[q] = y[qb];
            if (GRAD && A.g_out) {
                A.g_out[3 * q] = gx[qb][0];
                A.g_out[3 * q + 1] = gx[qb][1];
                A.g_out[3 * q + 2] = gx[qb][2];
            }
            if (A.routed) {
                float thr = A.band;
                if (A.cell_eps) {
                    int cell = cert_cell(A, x[qb][0], x[qb][1], x[qb][2]);
                    if (cell >= 0) thr = A.band0 + A.cell_eps[cell];
                }
                A.routed[q] = fabsf(y[qb]) < thr ? 1 : 0;
            }
            if (A.err_out) A.err_out[q] = fabsf(y[qb] - A.label[q]);
        }
    }
}

// Launch shapes: queries per wave = 16 x QB, waves per workgroup, waves per
// SIMD the register budget allows.
#ifndef SD_MLP_GRAD_QB
#define SD_MLP_GRAD_QB 1
#endif
#ifndef SD_MLP_GRAD_NW
#define SD_MLP_GRAD_NW 8
#endif
#ifndef SD_MLP_GRAD_WPE
#define SD_MLP_GRAD_WPE 2
#endif
#ifndef SD_MLP_VAL_QB
#define SD_MLP_VAL_QB 1
#endif
#ifndef SD_MLP_VAL_NW
#define SD_MLP_VAL_NW 8
#endif
#ifndef SD_MLP_VAL_WPE
#define SD_MLP_VAL_WPE 2
#endif
constexpr int kGradQ = 16 * SD_MLP_GRAD_QB * SD_MLP_GRAD_NW;   // queries per workgroup
constexpr int kValQ = 16 * SD_MLP_VAL_QB * SD_MLP_VAL_NW;

__global__ void __launch_bounds__(64 * SD_MLP_GRAD_NW)
__attribute__((amdgpu_waves_per_eu(SD_MLP_GRAD_WPE, SD_MLP_GRAD_WPE)))
k_mlp_grad(MlpArgs A) {
    __shared__ u32x4 lds[kSlots * kChunkU4];
    mlp_body<true, SD_MLP_GRAD_QB, SD_MLP_GRAD_NW>(A, lds);
}

__global__ void __launch_bounds__(64 * SD_MLP_VAL_NW)
__attribute__((amdgpu_waves_per_eu(SD_MLP_VAL_WPE, SD_MLP_VAL_WPE)))
k_mlp_value(MlpArgs A) {
    __shared__ u32x4 lds[kSlots * kChunkU4];
    mlp_body<false, SD_MLP_VAL_QB, SD_MLP_VAL_NW>(A, lds);
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
// gamma(x) of the batch rows (x = X[idx[b]]), rows and transposed copies; a
// row index outside [0, n_rows) reads as NaN (the loss becomes NaN)
__global__ void k_fourier_rows(const float *__restrict__ X, int64_t n_rows,
                               const int32_t *__restrict__ idx, int64_t n, const float *__restrict__ Bf,
                               __bf16 *__restrict__ A0, __bf16 *__restrict__ A0T) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n * NF) return;
    int64_t b = i / NF;
    int m = (int)(i % NF);
    int64_t src = idx ? (int64_t)idx[b] : b;
    float th = NAN;
    if (src >= 0 && src < n_rows)
        th = fmaf(Bf[3 * m], X[3 * src], fmaf(Bf[3 * m + 1], X[3 * src + 1], Bf[3 * m + 2] * X[3 * src + 2]));
    float s, c;
    sincos_rev(th, s, c);
    A0[b * NIN + m] = to_bf(s);
    A0[b * NIN + NF + m] = to_bf(c);
    A0T[(int64_t)m * n + b] = to_bf(s);
    A0T[(int64_t)(NF + m) * n + b] = to_bf(c);
}

enum { EPI_FWD = 0, EPI_BWD = 1, EPI_PART = 2 };

struct GemmArgs {
    const __bf16 *A;     // M x K, row-major
    int64_t lda;
    const __bf16 *Bt;    // N x K, row-major (the right operand transposed)
    int64_t ldb;
    int M, N, K, kchunk;
    const float *bias;   // EPI_FWD: N
    const float *S_in;   // EPI_BWD: M x N multiplier
    float *S_out;        // EPI_FWD: silu'(z), M x N
    float *F_out;        // EPI_FWD: silu(z) in FP32, M x N (optional)
    __bf16 *O_row;       // M x N
    __bf16 *O_col;       // N x M (ld = M)
    float *P_out;        // EPI_PART: gridDim.z x M x N
};

// C (M x N) = A (M x K) B (K x N): 64 x 64 tile per workgroup, 32 x 32 per wave
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs G) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, li = lane & 15;
    const int m0 = blockIdx.y * 64 + (wave & 1) * 32, n0 = blockIdx.x * 64 + (wave >> 1) * 32;
    const int kbeg = blockIdx.z * G.kchunk, kend = min(G.K, kbeg + G.kchunk);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i) acc[i][0] = acc[i][1] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const __bf16 *pa0 = G.A + (int64_t)(m0 + li) * G.lda + 8 * g;
    const __bf16 *pa1 = pa0 + 16 * G.lda;
    const __bf16 *pb0 = G.Bt + (int64_t)(n0 + li) * G.ldb + 8 * g;
    const __bf16 *pb1 = pb0 + 16 * G.ldb;
#pragma unroll 2
    for (int k = kbeg; k < kend; k += 32) {
        u32x4 a0 = *(const u32x4 *)(pa0 + k), a1 = *(const u32x4 *)(pa1 + k);
        u32x4 b0 = *(const u32x4 *)(pb0 + k), b1 = *(const u32x4 *)(pb1 + k);
        acc[0][0] = mma(a0, b0, acc[0][0]);
        acc[0][1] = mma(a0, b1, acc[0][1]);
        acc[1][0] = mma(a1, b0, acc[1][0]);
        acc[1][1] = mma(a1, b1, acc[1][1]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + 16 * j + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + 16 * i + 4 * g + r;
                const int64_t o = (int64_t)m * G.N + n;
                float v = acc[i][j][r];
                if (EPI == EPI_FWD) {
                    float z = v + G.bias[n];
                    float s = __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-z * kLog2e));
                    float a = z * s;
                    G.S_out[o] = s * fmaf(z, 1.f - s, 1.f);
                    if (G.F_out) G.F_out[o] = a;
                    G.O_row[o] = to_bf(a);
                    G.O_col[(int64_t)n * G.M + m] = to_bf(a);
                } else if (EPI == EPI_BWD) {
                    float u = v * G.S_in[o];
                    G.O_row[o] = to_bf(u);
                    G.O_col[(int64_t)n * G.M + m] = to_bf(u);
                } else {
                    G.P_out[(int64_t)blockIdx.z * G.M * G.N + o] = v;
                }
            }
        }
}

// output layer and loss: y_b = w5 . a4_b + b5, r_b = y_b - t_b, dy_b = 2 r_b / n,
// G4 = dy_b w5 silu'(z4_b) (rows and transposed), dyr_b = (dy_b, r_b^2).
// One wave per sample.
__global__ void __launch_bounds__(256)
k_out_loss(const float *__restrict__ A4, const float *__restrict__ S4, const __bf16 *__restrict__ w5,
           const float *__restrict__ b5, const float *__restrict__ t, int64_t n_rows,
           const int32_t *__restrict__ idx, int64_t n, float inv_n, __bf16 *__restrict__ G4, __bf16 *__restrict__ G4T, float *__restrict__ dyr) {
    const int lane = threadIdx.x & 63;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n) return;
    float w[4], s = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w[k] = (float)w5[4 * lane + k];
        s = fmaf(A4[b * WD + 4 * lane + k], w[k], s);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    float y = s + *b5;
    const int64_t src = idx ? (int64_t)idx[b] : b;
    float r = y - (src >= 0 && src < n_rows ? t[src] : NAN);
    float dy = 2.f * r * inv_n;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int f = 4 * lane + k;
        __bf16 u = to_bf(dy * w[k] * S4[b * WD + f]);
        G4[b * WD + f] = u;
        G4T[(int64_t)f * n + b] = u;
    }
    if (lane == 0) {
        dyr[2 * b] = dy;
        dyr[2 * b + 1] = r * r;
    }
}

// partial column sums: part[chunk][c] = sum over rows of the chunk of
// scale[row] * src[row][c] (fixed order)
template <class T>
__global__ void __launch_bounds__(256)
k_colsum(const T *__restrict__ src, int cols, int64_t rows, int64_t rows_per_chunk,
         const float *__restrict__ scale, int scale_ld, float *__restrict__ part) {
    const int c = threadIdx.x;
    if (c >= cols) return;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_chunk;
    const int64_t r1 = min(rows, r0 + rows_per_chunk);
    float s = 0.f;
#pragma unroll 8
    for (int64_t r = r0; r < r1; ++r) {
        float v = (float)src[r * cols + c];
        s = scale ? fmaf(scale[r * scale_ld], v, s) : s + v;
    }
    part[(int64_t)blockIdx.x * cols + c] = s;
}

// out[i] = scale * sum over chunks of part[chunk * ld + i], in chunk order
__global__ void k_reduce_chunks(const float *__restrict__ part, int chunks, int64_t len, int64_t ld,
                                float *__restrict__ out, float scale) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    float s = 0.f;
#pragma unroll 8
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * ld + i];
    out[i] = s * scale;
}

// b1, b2 and their complements c1 = 1 - b1, c2 = 1 - b2 are each the FP32
// rounding of the exact constant (1 - b formed in FP32 would be off by the
// rounding of b, 1.3e-5 relative for 0.999)
__global__ void k_adam(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ gr, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps, float inv_bc1, float inv_bc2) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float g = gr[i];
    float mi = fmaf(b1, m[i], c1 * g);
    float vi = fmaf(b2, v[i], c2 * g * g);
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi * inv_bc1) / (sqrtf(vi * inv_bc2) + eps);
}

// largest value of a non-negative array (NaN counts as +inf)
__global__ void __launch_bounds__(256) k_max_part(const float *__restrict__ x, int64_t n,
                                                  float *__restrict__ part) {
    __shared__ float red[256];
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float v = x[i];
        m = (v != v) ? INFINITY : fmaxf(m, v);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_flags_u32(const uint8_t *__restrict__ f, int64_t n, uint32_t *__restrict__ o) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) o[i] = f[i];
}

__global__ void k_compact(const uint8_t *__restrict__ f, const uint32_t *__restrict__ pos, int64_t n,
                          uint32_t *__restrict__ idx) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n && f[i]) idx[pos[i]] = (uint32_t)i;
}

// number of flagged entries: the exclusive prefix sum at the last entry plus
// its flag (one thread)
__global__ void k_flag_count(const uint8_t *__restrict__ f, const uint32_t *__restrict__ pos, int64_t n,
                             uint32_t *__restrict__ count) {
    if (threadIdx.x == 0 && blockIdx.x == 0) count[0] = n > 0 ? pos[n - 1] + (f[n - 1] ? 1u : 0u) : 0u;
}

// per-cell maximum of the sample errors (non-negative floats order like their
// bit patterns; -1 marks an empty cell)
__global__ void k_cell_max(const float *__restrict__ X, const float *__restrict__ err, int64_t n,
                           MlpArgs A, int *__restrict__ cell_bits) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int c = cert_cell(A, X[3 * i], X[3 * i + 1], X[3 * i + 2]);
    float e = err[i];
    if (c >= 0) atomicMax(cell_bits + c, e == e ? __float_as_int(e) : 0x7f800000);
}

// certificate of a cell: safety x the largest error over the cell and its 26
// neighbours; cells with no sample in that neighbourhood take eps_global
__global__ void k_cell_final(const int *__restrict__ cell_bits, int G, float safety, float eps_global,
                             float max_margin, float *__restrict__ cell_eps) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)G * G * G) return;
    int cx = (int)(i / (G * G)), cy = (int)(i / G % G), cz = (int)(i % G);
    int best = -1;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                int x = cx + dx, y = cy + dy, z = cz + dz;
                if (x < 0 || y < 0 || z < 0 || x >= G || y >= G || z >= G) continue;
                best = max(best, cell_bits[((int64_t)x * G + y) * G + z]);
            }
    float e = best < 0 ? eps_global : safety * __int_as_float(best);
    cell_eps[i] = e > max_margin ? INFINITY : e;   // cells above the target route every query
}

__global__ void k_fill_i32(int *__restrict__ p, int64_t n, int v) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace
}  // namespace sd

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct sd_surrogate {
    int device = 0;
    int64_t max_batch = 0;
    int64_t step = 0;
    float eps_cert = INFINITY;
    // local certificate (grid^3 cells over [glo, ghi]); cell_eps null when absent
    float *cell_eps = nullptr;
    int64_t cell_cap = 0;
    int grid = 0;
    float glo[3] = {0.f, 0.f, 0.f}, ginv[3] = {0.f, 0.f, 0.f};
    float *Bf = nullptr;           // 64 x 3
    float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *frag = nullptr;      // inference stream
    float *bias_s = nullptr, *w5s = nullptr;
    __bf16 *wr = nullptr, *wc = nullptr;   // training copies
    // training workspace (max_batch rows)
    __bf16 *A0 = nullptr, *A0T = nullptr, *Ar[4] = {}, *AT[4] = {}, *Gr[4] = {}, *GT[4] = {};
    float *S[4] = {}, *A4f = nullptr, *dyr = nullptr, *part = nullptr, *loss = nullptr;
    int64_t part_len = 0;
    std::vector<void *> owned;
};

namespace sd {
namespace {

constexpr int kSplitRows = 2048;   // split-K length of the weight-gradient products
constexpr int kSumRows = 256;      // rows per partial of the column sums (bias gradients)

int sur_alloc(sd_surrogate *h, void **p, size_t bytes) {
    SD_TRY(dev_malloc(p, bytes, "surrogate"));
    h->owned.push_back(*p);
    return SD_OK;
}

int pack(sd_surrogate *h, hipStream_t s) {
    const int64_t n_el = (int64_t)kChunks * kChunkU4 * 8;
    hipLaunchKernelGGL(k_pack_infer, dim3(blocks(n_el)), dim3(256), 0, s, h->theta, h->frag,
                       h->bias_s, h->w5s);
    hipLaunchKernelGGL(k_pack_train, dim3(blocks(NPAR)), dim3(256), 0, s, h->theta, h->wr, h->wc);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

int launch_mlp(const sd_surrogate *h, const float *Q, int64_t nq, float *d, float *gr,
               uint8_t *routed, float band, const float *label, float *err, hipStream_t s,
               float band0 = 0.f) {
    if (nq <= 0) return SD_OK;
    MlpArgs A;
    A.frag = (const u32x4 *)h->frag;
    A.bias_s = h->bias_s;
    A.w5s = h->w5s;
    A.b5 = h->theta + OFF_B5;
    A.Bf = h->Bf;
    A.Q = Q;
    A.nq = nq;
    A.d_out = d;
    A.g_out = gr;
    A.routed = routed;
    A.band = band;
    A.label = label;
    A.err_out = err;
    A.cell_eps = nullptr;
    A.band0 = 0.f;
    A.grid = h->grid;
    for (int a = 0; a < 3; ++a) {
        A.glo[a] = h->glo[a];
        A.ginv[a] = h->ginv[a];
    }
    if (routed && h->grid > 0 && h->cell_eps) {
        A.cell_eps = h->cell_eps;
        A.band0 = band0;
    }
    if (gr)
        hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((nq + kGradQ - 1) / kGradQ)), dim3(64 * SD_MLP_GRAD_NW),
                           0, s, A);
    else
        hipLaunchKernelGGL(k_mlp_value, dim3((unsigned)((nq + kValQ - 1) / kValQ)), dim3(64 * SD_MLP_VAL_NW),
                           0, s, A);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

int gemm(int epi, const GemmArgs &G, int splits, hipStream_t s) {
    dim3 grid(G.N / 64, G.M / 64, splits);
    if (epi == EPI_FWD) hipLaunchKernelGGL(k_gemm<EPI_FWD>, grid, dim3(256), 0, s, G);
    else if (epi == EPI_BWD) hipLaunchKernelGGL(k_gemm<EPI_BWD>, grid, dim3(256), 0, s, G);
    else hipLaunchKernelGGL(k_gemm<EPI_PART>, grid, dim3(256), 0, s, G);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

// loss gradient of one batch into h->grad and the loss into h->loss
int loss_grad(sd_surrogate *h, const float *X, const float *y, int64_t n_rows, const int32_t *idx,
              int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fourier_rows, dim3(blocks(n * NF)), dim3(256), 0, s, X, n_rows, idx, n, h->Bf,
                       h->A0, h->A0T);
    // forward
    for (int l = 1; l <= 4; ++l) {
        GemmArgs G = {};
        G.A = l == 1 ? h->A0 : h->Ar[l - 2];
        G.lda = fan_in(l);
        G.Bt = h->wr + off_W(l);
        G.ldb = fan_in(l);
        G.M = (int)n; G.N = WD; G.K = fan_in(l); G.kchunk = fan_in(l);
        G.bias = h->theta + off_b(l);
        G.S_out = h->S[l - 1];
        G.F_out = l == 4 ? h->A4f : nullptr;
        G.O_row = h->Ar[l - 1];
        G.O_col = h->AT[l - 1];
        SD_TRY(gemm(EPI_FWD, G, 1, s));
    }
    hipLaunchKernelGGL(k_out_loss, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, h->A4f, h->S[3],
                       h->wr + OFF_W5, h->theta + OFF_B5, y, n_rows, idx, n, 1.f / (float)n, h->Gr[3], h->GT[3], h->dyr);
    // backward through W4..W2 (dL/dz of the layer below)
    for (int l = 4; l >= 2; --l) {
        GemmArgs G = {};
        G.A = h->Gr[l - 1];
        G.lda = WD;
        G.Bt = h->wc + off_W(l);
        G.ldb = WD;
        G.M = (int)n; G.N = WD; G.K = WD; G.kchunk = WD;
        G.S_in = h->S[l - 2];
        G.O_row = h->Gr[l - 2];
        G.O_col = h->GT[l - 2];
        SD_TRY(gemm(EPI_BWD, G, 1, s));
    }
    // weight gradients dW_l = G_l^T A_{l-1}, split over the batch
    const int splits = (int)((n + kSplitRows - 1) / kSplitRows);
    for (int l = 1; l <= 4; ++l) {
        GemmArgs G = {};
        G.A = h->GT[l - 1];
        G.lda = n;
        G.Bt = l == 1 ? h->A0T : h->AT[l - 2];
        G.ldb = n;
        G.M = WD; G.N = fan_in(l); G.K = (int)n; G.kchunk = kSplitRows;
        G.P_out = h->part;
        SD_TRY(gemm(EPI_PART, G, splits, s));
        int64_t len = (int64_t)WD * fan_in(l);
        hipLaunchKernelGGL(k_reduce_chunks, dim3(blocks(len)), dim3(256), 0, s, h->part, splits, len,
                           len, h->grad + off_W(l), 1.f);
        // bias: column sums of G_l
        int64_t chunks = (n + kSumRows - 1) / kSumRows;
        hipLaunchKernelGGL(k_colsum<__bf16>, dim3((unsigned)chunks), dim3(256), 0, s, h->Gr[l - 1], WD, n,
                           (int64_t)kSumRows, (const float *)nullptr, 0, h->part);
        hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, s, h->part, (int)chunks, (int64_t)WD,
                           (int64_t)WD, h->grad + off_b(l), 1.f);
    }
    // output layer: dw5 = sum dy a4, db5 = sum dy; loss = mean r^2
    int64_t chunks = (n + kSumRows - 1) / kSumRows;
    hipLaunchKernelGGL(k_colsum<float>, dim3((unsigned)chunks), dim3(256), 0, s, h->A4f, WD, n,
                       (int64_t)kSumRows, h->dyr, 2, h->part);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, s, h->part, (int)chunks, (int64_t)WD,
                       (int64_t)WD, h->grad + OFF_W5, 1.f);
    hipLaunchKernelGGL(k_colsum<float>, dim3((unsigned)chunks), dim3(256), 0, s, h->dyr, 2, n,
                       (int64_t)kSumRows, (const float *)nullptr, 0, h->part);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, s, h->part, (int)chunks, (int64_t)1,
                       (int64_t)2, h->grad + OFF_B5, 1.f);
    hipLaunchKernelGGL(k_reduce_chunks, dim3(1), dim3(256), 0, s, h->part + 1, (int)chunks, (int64_t)1,
                       (int64_t)2, h->loss, 1.f / (float)n);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

}  // namespace
}  // namespace sd

using namespace sd;

extern "C" int sd_surrogate_create(const float *B_host, const float *theta_host, int64_t max_batch,
                                   void *stream, sd_surrogate **out) {
    if (!out) return fail(SD_EINVAL, "sd_surrogate_create: null output");
    *out = nullptr;
    if (!B_host || !theta_host) return fail(SD_EINVAL, "sd_surrogate_create: null input");
    if (max_batch < 0 || max_batch % 64 != 0 || max_batch > (1 << 24))
        return fail(SD_EINVAL, "sd_surrogate_create: max_batch must be a multiple of 64 in [0, 2^24]");
    hipStream_t s = (hipStream_t)stream;
    auto *h = new (std::nothrow) sd_surrogate();
    if (!h) return fail(SD_ENOMEM, "sd_surrogate_create: host allocation");
    hipError_t de = hipGetDevice(&h->device);
    if (de != hipSuccess) {
        delete h;
        return fail(SD_EHIP, std::string("sd_surrogate_create: hipGetDevice: ") + hipGetErrorString(de));
    }
    h->max_batch = max_batch;
    auto fl = [&](float **p, size_t n) { return sur_alloc(h, (void **)p, n * sizeof(float)); };
    auto bf = [&](__bf16 **p, size_t n) { return sur_alloc(h, (void **)p, n * sizeof(__bf16)); };
    int rc = SD_OK;
    const int64_t n_el = (int64_t)kChunks * kChunkU4 * 8;
    if (!rc) rc = fl(&h->Bf, 3 * NF);
    if (!rc) rc = fl(&h->theta, NPAR);
    if (!rc) rc = fl(&h->m, NPAR);
    if (!rc) rc = fl(&h->v, NPAR);
    if (!rc) rc = fl(&h->grad, NPAR);
    if (!rc) rc = sur_alloc(h, (void **)&h->frag, n_el * sizeof(uint16_t));
    if (!rc) rc = fl(&h->bias_s, 4 * WD);
    if (!rc) rc = fl(&h->w5s, WD);
    if (!rc) rc = bf(&h->wr, NPAR);
    if (!rc) rc = bf(&h->wc, NPAR);
    if (!rc) rc = fl(&h->loss, 1);
    if (max_batch > 0) {
        const size_t nb = (size_t)max_batch;
        if (!rc) rc = bf(&h->A0, nb * NIN);
        if (!rc) rc = bf(&h->A0T, nb * NIN);
        for (int l = 0; l < 4 && !rc; ++l) {
            rc = bf(&h->Ar[l], nb * WD);
            if (!rc) rc = bf(&h->AT[l], nb * WD);
            if (!rc) rc = bf(&h->Gr[l], nb * WD);
            if (!rc) rc = bf(&h->GT[l], nb * WD);
            if (!rc) rc = fl(&h->S[l], nb * WD);
        }
        if (!rc) rc = fl(&h->A4f, nb * WD);
        if (!rc) rc = fl(&h->dyr, 2 * nb);
        const int64_t splits = (max_batch + kSplitRows - 1) / kSplitRows;
        h->part_len = std::max(splits * (int64_t)WD * WD, (max_batch + kSumRows - 1) / kSumRows * (int64_t)WD);
        if (!rc) rc = fl(&h->part, (size_t)h->part_len);
    }
    if (!rc) {
        hipError_t e = hipMemcpyAsync(h->Bf, B_host, 3 * NF * sizeof(float), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(h->theta, theta_host, NPAR * sizeof(float), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(h->m, 0, NPAR * sizeof(float), s);
        if (e == hipSuccess) e = hipMemsetAsync(h->v, 0, NPAR * sizeof(float), s);
        if (e != hipSuccess) rc = fail(SD_EHIP, std::string("sd_surrogate_create: ") + hipGetErrorString(e));
    }
    if (!rc) rc = pack(h, s);
    if (rc) {
        for (void *p : h->owned) dev_free(p);
        delete h;
        return rc;
    }
    *out = h;
    return SD_OK;
}

extern "C" int sd_surrogate_free(sd_surrogate *h) {
    if (!h) return SD_OK;
    dev_free(h->cell_eps);
    for (void *p : h->owned) dev_free(p);
    delete h;
    return SD_OK;
}

extern "C" int sd_surrogate_forward(const sd_surrogate *h, const float *Q, int64_t nQ, float *d_out,
                                    float *grad_out, void *stream) {
    if (!h) return fail(SD_EINVAL, "sd_surrogate_forward: null handle");
    if (nQ < 0) return fail(SD_EINVAL, "sd_surrogate_forward: nQ < 0");
    if (nQ > 0 && (!Q || !d_out)) return fail(SD_EINVAL, "sd_surrogate_forward: null array");
    return launch_mlp(h, Q, nQ, d_out, grad_out, nullptr, 0.f, nullptr, nullptr, (hipStream_t)stream);
}

extern "C" int sd_surrogate_loss_grad(sd_surrogate *h, const float *X, const float *y,
                                      int64_t n_rows, const int32_t *idx, int64_t n, float *grad_out,
                                      float *loss_out, void *stream) {
    if (!h) return fail(SD_EINVAL, "sd_surrogate_loss_grad: null handle");
    if (n <= 0 || n % 64 != 0 || n > h->max_batch)
        return fail(SD_EINVAL, "sd_surrogate_loss_grad: batch must be a positive multiple of 64 "
                               "no larger than max_batch");
    if (!X || !y) return fail(SD_EINVAL, "sd_surrogate_loss_grad: null array");
    if (!idx && n_rows < n) return fail(SD_EINVAL, "sd_surrogate_loss_grad: fewer rows than the batch");
    hipStream_t s = (hipStream_t)stream;
    SD_TRY(loss_grad(h, X, y, n_rows, idx, n, s));
    if (grad_out) SD_HIP(hipMemcpyAsync(grad_out, h->grad, NPAR * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (loss_out) SD_HIP(hipMemcpyAsync(loss_out, h->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
    return SD_OK;
}

extern "C" int sd_surrogate_adam(sd_surrogate *h, const float *grad, float lr, void *stream) {
    if (!h) return fail(SD_EINVAL, "sd_surrogate_adam: null handle");
    if (!(lr >= 0.f)) return fail(SD_EINVAL, "sd_surrogate_adam: lr must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const double b1 = 0.9, b2 = 0.999;
    h->step += 1;
    float ib1 = (float)(1.0 / (1.0 - pow(b1, (double)h->step)));
    float ib2 = (float)(1.0 / (1.0 - pow(b2, (double)h->step)));
    hipLaunchKernelGGL(k_adam, dim3(blocks(NPAR)), dim3(256), 0, s, h->theta, h->m, h->v,
                       grad ? grad : h->grad, NPAR, lr, (float)b1, (float)b2, (float)(1.0 - b1),
                       (float)(1.0 - b2), 1e-8f, ib1, ib2);
    SD_HIP(hipGetLastError());
    return pack(h, s);
}

extern "C" int sd_surrogate_train_step(sd_surrogate *h, const float *X, const float *y,
                                       int64_t n_rows, const int32_t *idx, int64_t n, float lr,
                                       float *loss_out, void *stream) {
    SD_TRY(sd_surrogate_loss_grad(h, X, y, n_rows, idx, n, nullptr, loss_out, stream));
    return sd_surrogate_adam(h, nullptr, lr, stream);
}

extern "C" int sd_surrogate_certify(sd_surrogate *h, const float *X, const float *y, int64_t n,
                                    float safety, void *stream, float *eps_host) {
    if (!h) return fail(SD_EINVAL, "sd_surrogate_certify: null handle");
    if (n <= 0 || !X || !y) return fail(SD_EINVAL, "sd_surrogate_certify: empty validation set");
    if (!(safety >= 1.f)) return fail(SD_EINVAL, "sd_surrogate_certify: safety factor must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    float *err = nullptr, *part = nullptr;
    const int nblk = 1024;
    AsyncScratch tmp(s);
    SD_TRY(tmp.alloc(&err, n));
    SD_TRY(tmp.alloc(&part, nblk));
    SD_TRY(launch_mlp(h, X, n, nullptr, nullptr, nullptr, 0.f, y, err, s));
    hipLaunchKernelGGL(k_max_part, dim3(nblk), dim3(256), 0, s, err, n, part);
    hipLaunchKernelGGL(k_max_part, dim3(1), dim3(256), 0, s, part, (int64_t)nblk, part);
    SD_HIP(hipGetLastError());
    float mx = 0.f;
    SD_HIP(hipMemcpyAsync(&mx, part, sizeof(float), hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
    h->eps_cert = safety * mx;
    h->grid = 0;   // a global certificate replaces any local one
    if (eps_host) *eps_host = h->eps_cert;
    return SD_OK;
}

extern "C" int sd_surrogate_certify_cells(sd_surrogate *h, const float *X, const float *y, int64_t n,
                                          float safety, int grid, const float *lo_host,
                                          const float *hi_host, float max_margin, void *stream,
                                          float *eps_host) {
    if (!(max_margin > 0.f)) return fail(SD_EINVAL, "sd_surrogate_certify_cells: max_margin must be > 0");
    if (!h || !lo_host || !hi_host) return fail(SD_EINVAL, "sd_surrogate_certify_cells: null argument");
    if (grid < 1 || grid > 256) return fail(SD_EINVAL, "sd_surrogate_certify_cells: grid must be in [1, 256]");
    for (int a = 0; a < 3; ++a)
        if (!(hi_host[a] > lo_host[a])) return fail(SD_EINVAL, "sd_surrogate_certify_cells: empty box");
    SD_TRY(sd_surrogate_certify(h, X, y, n, safety, stream, eps_host));
    hipStream_t s = (hipStream_t)stream;
    const int64_t nc = (int64_t)grid * grid * grid;
    if (h->cell_eps && h->cell_cap < nc) {
        dev_free(h->cell_eps);
        h->cell_eps = nullptr;
        h->cell_cap = 0;
    }
    if (!h->cell_eps) {
        SD_TRY(dev_malloc((void **)&h->cell_eps, nc * sizeof(float), "sd_surrogate_certify_cells"));
        h->cell_cap = nc;
    }
    MlpArgs A = {};
    A.grid = grid;
    for (int a = 0; a < 3; ++a) {
        h->glo[a] = lo_host[a];
        h->ginv[a] = (float)grid / (hi_host[a] - lo_host[a]);
        A.glo[a] = h->glo[a];
        A.ginv[a] = h->ginv[a];
    }
    float *err = nullptr;
    int *bits = nullptr;
    AsyncScratch tmp(s);
    SD_TRY(tmp.alloc(&err, n));
    SD_TRY(tmp.alloc(&bits, nc));
    SD_TRY(launch_mlp(h, X, n, nullptr, nullptr, nullptr, 0.f, y, err, s));
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks(nc)), dim3(256), 0, s, bits, nc, -1);
    hipLaunchKernelGGL(k_cell_max, dim3(blocks(n)), dim3(256), 0, s, X, err, n, A, bits);
    hipLaunchKernelGGL(k_cell_final, dim3(blocks(nc)), dim3(256), 0, s, bits, grid, safety, h->eps_cert,
                       max_margin, h->cell_eps);
    SD_HIP(hipGetLastError());
    SD_HIP(hipStreamSynchronize(s));
    h->grid = grid;
    return SD_OK;
}

extern "C" int sd_surrogate_save(const sd_surrogate *h, float *theta_host, float *m_host, float *v_host,
                                 float *B_host, int64_t *step_host, float *eps_host) {
    if (!h) return fail(SD_EINVAL, "sd_surrogate_save: null handle");
    if (theta_host) SD_HIP(hipMemcpy(theta_host, h->theta, NPAR * sizeof(float), hipMemcpyDeviceToHost));
    if (m_host) SD_HIP(hipMemcpy(m_host, h->m, NPAR * sizeof(float), hipMemcpyDeviceToHost));
    if (v_host) SD_HIP(hipMemcpy(v_host, h->v, NPAR * sizeof(float), hipMemcpyDeviceToHost));
    if (B_host) SD_HIP(hipMemcpy(B_host, h->Bf, 3 * NF * sizeof(float), hipMemcpyDeviceToHost));
    if (step_host) *step_host = h->step;
    if (eps_host) *eps_host = h->eps_cert;
    return SD_OK;
}

extern "C" int sd_surrogate_load(sd_surrogate *h, const float *theta_host, const float *m_host,
                                 const float *v_host, int64_t step, float eps_cert, void *stream) {
    if (!h || !theta_host) return fail(SD_EINVAL, "sd_surrogate_load: null argument");
    if (step < 0) return fail(SD_EINVAL, "sd_surrogate_load: step < 0");
    hipStream_t s = (hipStream_t)stream;
    SD_HIP(hipMemcpyAsync(h->theta, theta_host, NPAR * sizeof(float), hipMemcpyHostToDevice, s));
    if (m_host) SD_HIP(hipMemcpyAsync(h->m, m_host, NPAR * sizeof(float), hipMemcpyHostToDevice, s));
    else SD_HIP(hipMemsetAsync(h->m, 0, NPAR * sizeof(float), s));
    if (v_host) SD_HIP(hipMemcpyAsync(h->v, v_host, NPAR * sizeof(float), hipMemcpyHostToDevice, s));
    else SD_HIP(hipMemsetAsync(h->v, 0, NPAR * sizeof(float), s));
    h->step = step;
    h->eps_cert = eps_cert;
    h->grid = 0;
    return pack(h, s);
}

extern "C" int sd_eval_surrogate(const sd_scene *sc, const sd_surrogate *h, const float *Q, int64_t nQ,
                                 const sd_params *p, float band, float *d_out, float *grad_out,
                                 uint8_t *routed, uint32_t *n_fallback, void *stream) {
    if (!sc || !h || !p) return fail(SD_EINVAL, "sd_eval_surrogate: null argument");
    if (nQ < 0) return fail(SD_EINVAL, "sd_eval_surrogate: nQ < 0");
    if (!(band >= 0.f)) return fail(SD_EINVAL, "sd_eval_surrogate: band must be >= 0");
    if (!(p->alpha > 0.f) || !(p->beta >= 0.f) || !(p->alpha_u >= 0.f))
        return fail(SD_EINVAL, "sd_eval_surrogate: bad parameters");
    if (sc->n[0] + sc->n[1] + sc->n[2] == 0) return fail(SD_EINVAL, "sd_eval_surrogate: empty scene");
    if (nQ > 0x7fffffffll - 256) return fail(SD_EUNSUPPORTED, "sd_eval_surrogate: more than 2^31 queries");
    hipStream_t s = (hipStream_t)stream;
    if (nQ == 0) {
        if (n_fallback) {
            hipLaunchKernelGGL(k_flag_count, dim3(1), dim3(64), 0, s, nullptr, nullptr, (int64_t)0, n_fallback);
            SD_HIP(hipGetLastError());
        }
        return SD_OK;
    }
    if (!Q || !d_out || !grad_out) return fail(SD_EINVAL, "sd_eval_surrogate: null array");
    uint8_t *flag = routed;
    uint32_t *f32 = nullptr, *pos = nullptr, *idx = nullptr, *ord = nullptr, *nfb = n_fallback;
    char *temp = nullptr;
    AsyncScratch tmp(s);
    if (!flag) SD_TRY(tmp.alloc(&flag, nQ));
    if (!nfb) SD_TRY(tmp.alloc(&nfb, 1));
    SD_TRY(launch_mlp(h, Q, nQ, d_out, grad_out, flag, band + h->eps_cert, nullptr, nullptr, s, band));
    // compaction of the routed queries (in index order), then Morton order
    SD_TRY(tmp.alloc(&f32, nQ));
    SD_TRY(tmp.alloc(&pos, nQ));
    SD_TRY(tmp.alloc(&temp, (int64_t)radix_sort_temp_bytes(nQ)));
    hipLaunchKernelGGL(k_flags_u32, dim3(blocks(nQ)), dim3(256), 0, s, flag, nQ, f32);
    SD_TRY(exclusive_scan_u32(f32, pos, nQ, temp, s));
    // the count of routed queries stays on the device: the compaction, the
    // Morton order and the exact pass are launched for all nQ and read it
    hipLaunchKernelGGL(k_flag_count, dim3(1), dim3(64), 0, s, flag, pos, nQ, nfb);
    SD_TRY(tmp.alloc(&idx, nQ));
    hipLaunchKernelGGL(k_compact, dim3(blocks(nQ)), dim3(256), 0, s, flag, pos, nQ, idx);
    SD_HIP(hipGetLastError());
    const uint32_t *perm = idx;
    int rc = SD_OK;
    if (!(p->flags & SD_NO_QUERY_SORT) && nQ >= 4096) {
        SD_TRY(tmp.alloc(&ord, nQ));
        rc = query_order(sc, Q, nQ, ord, s, idx, nfb);
        perm = ord;
    }
    if (!rc) rc = eval_dispatch(sc, Q, perm, nQ, p, d_out, grad_out, nullptr, false, s, nQ, nfb);
    return rc;
}
