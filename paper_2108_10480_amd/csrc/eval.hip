// Smooth-distance evaluation kernels.
//
//   k_eval     one lane per query: stackless depth-first traversal of each class
//              hierarchy (Alg. 1), conservative far field (Sec. 3.5, App. D),
//              exact leaf terms (App. B distances, App. C weights, Eq. 5
//              weight gradients), online log-sum-exp (Eq. 3, Eq. 4), Alg. 2
//              finalisation.
//   k_brute    the same leaf terms over every primitive, primitives staged
//              through LDS in tiles (beta = 0 semantics).
//
// Precision.  Every term enters the log-sum-exp through its log-term
// L_i = log w_i - alpha d_i, and an error e in d_i changes the term's weight by
// the factor exp(alpha e): with FP32 distances (e ~ 2^-23 d) that is 3e-5 at
// alpha = 500, d = 1, which shows in the gradient.  So distances, closest
// points and barycentric coordinates are formed in FP64 from the FP32 inputs
// (differences of FP32 values are exact in FP64), and the triangle weight
// polynomial is evaluated in FP64 (monomial Horner form): an FP64 FMA issues
// at the rate of an FP32 one on this GPU, so this costs registers rather than
// issue slots.  Directions, weight gradients and exponentials stay FP32.
//
// Online log-sum-exp state per lane: the largest log-term L* so far (FP64), the
// sum s of exp(L_i - L*) and the gradient numerator G (FP64 sums of FP32
// terms).  d = -(L* + log s) / alpha, formed in FP64 and rounded once.
//
// Conservativeness (App. A, Sec. 3.5).  With every weight >= 1 the exact
// log-sum-exp is at most the smallest term distance, which is at most the
// exact minimum distance d_min (each far-field box distance D_B is below the
// distances of its primitives).  Each term also carries a rigorous lower bound
// of its exact distance; by default the result is clamped to the smallest of
// these, so d <= d_min holds for the FP32 output whatever the rounding, and
// the clamp changes the result only where it is within rounding of that
// smallest term distance.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "sd_internal.h"

namespace sd {
namespace {

constexpr int kB = 256;

// Kahan's difference of products a*b - c*d with one FMA correction.
__device__ __forceinline__ float dop(float a, float b, float c, float d) {
    float w = c * d;
    float e = fmaf(-c, d, w);
    float f = fmaf(a, b, -w);
    return f + e;
}

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz) {
    return fmaf(ax, bx, fmaf(ay, by, az * bz));
}
__device__ __forceinline__ double ddot3(double ax, double ay, double az, double bx, double by, double bz) {
    return fma(ax, bx, fma(ay, by, az * bz));
}

// Hardware square root and reciprocal (1 ulp) instead of the correctly rounded
// multi-instruction sequences; the error bounds below allow for them.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fdiv(float a, float b) { return a * frcp(b); }

// The distance sqrt(s) in FP64 from its FP64 square s and an FP32 estimate r
// within a few ulps of it (inv_r = 1/r): one Newton step r + (s - r^2) / (2 r)
// leaves a relative error near 2^-44 (the FP32 rounding of 1/(2r) only
// scales the correction, itself about 2^-22 r).  Two FP64 FMAs.  r = 0 gives 0.
__device__ __forceinline__ double sqrt_newton_pos(double s, float r, float inv_r) {   // r > 0
    const double rr = (double)r;
    return fma(fma(-rr, rr, s), (double)(0.5f * inv_r), rr);
}
__device__ __forceinline__ double sqrt_newton(double s, float r, float inv_r) {
    return r > 0.f ? sqrt_newton_pos(s, r, inv_r) : 0.0;
}

// Lower-bound factor of an FP32 distance formed from rounded FP32 differences,
// a sum of squares by FMA and the hardware square root (at most about 2^-21.8
// relative error): d (1 - 2^-21) is below the exact distance.
constexpr float kLo = 1.f - 0x1p-21f;
// Lower bound of an edge or triangle distance r (FP32 square root of the FP64
// square s): the closest point q - c is formed in FP64 from exact differences
// with its parameters clamped to the primitive, so sqrt(s) falls short of the
// exact distance by at most a few FP64 roundings of the vectors involved
// (o1 bounds their 1-norms); 2^-40 o1 covers that with a wide margin.
__device__ __forceinline__ float dist_lo(float r, float o1) { return fmaf(-0x1p-40f, o1, r * kLo); }

struct LSE64 {
    double L;                // largest log-term so far (-inf: none yet)
    double s, gx, gy, gz;    // sum of exp(L_i - L*) and the gradient numerator
    float Lf;                // L* rounded to FP32 (pruning bound)
    float mlo;               // lower bound of the smallest term distance
};
using LSE = LSE64;

// The same state with the four sums in FP32, each compensated (Neumaier's
// variant of Kahan summation, with the rounding error of every product taken
// by an FMA): a sum is the unevaluated pair hi + lo.  The compiled variant
// selected by SD_LSE_COMPENSATED_F32.
struct LSEc32 {
    double L;
    float s, cs, gx, cx, gy, cy, gz, cz;
    float Lf;
    float mlo;
};

__device__ __forceinline__ void lse_init(LSE64 &st) {
    st.L = -INFINITY;
    st.s = st.gx = st.gy = st.gz = 0.0;
    st.Lf = -INFINITY;
    st.mlo = INFINITY;
}

__device__ __forceinline__ void lse_init(LSEc32 &st) {
    st.L = -INFINITY;
    st.s = st.cs = st.gx = st.cx = st.gy = st.cy = st.gz = st.cz = 0.f;
    st.Lf = -INFINITY;
    st.mlo = INFINITY;
}

__device__ __forceinline__ bool lse_empty(const LSE64 &st) { return st.s == 0.0 && st.L == -INFINITY; }
__device__ __forceinline__ bool lse_empty(const LSEc32 &st) { return st.s == 0.f && st.L == -INFINITY; }
__device__ __forceinline__ double lse_sum(const LSE64 &st) { return st.s; }
__device__ __forceinline__ double lse_sum(const LSEc32 &st) { return (double)st.s + (double)st.cs; }
__device__ __forceinline__ void lse_num(const LSE64 &st, double &x, double &y, double &z) {
    x = st.gx;
    y = st.gy;
    z = st.gz;
}
__device__ __forceinline__ void lse_num(const LSEc32 &st, double &x, double &y, double &z) {
    x = (double)st.gx + (double)st.cx;
    y = (double)st.gy + (double)st.cy;
    z = (double)st.gz + (double)st.cz;
}

// s + x into (s, c): the sum rounded and its rounding error added to c
__device__ __forceinline__ void neumaier_add(float &s, float &c, float x) {
    const float t = s + x;
    c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// (s + c) * e + x into (s, c)
__device__ __forceinline__ void neumaier_scale_add(float &s, float &c, float e, float x) {
    const float p = s * e;
    c = fmaf(c, e, fmaf(s, e, -p));   // error of the product, and the old compensation scaled
    s = p;
    neumaier_add(s, c, x);
}

// (s + c) + e * g into (s, c)
__device__ __forceinline__ void neumaier_fma(float &s, float &c, float e, float g) {
    const float p = e * g;
    c += fmaf(e, g, -p);
    neumaier_add(s, c, p);
}

template <bool GRAD>
__device__ __forceinline__ void lse_fold(LSEc32 &st, float t, double Lnew, float gx, float gy, float gz) {
    if (t <= 0.f) {
        const float e = __expf(t);
        neumaier_add(st.s, st.cs, e);
        if (GRAD) {
            neumaier_fma(st.gx, st.cx, e, gx);
            neumaier_fma(st.gy, st.cy, e, gy);
            neumaier_fma(st.gz, st.cz, e, gz);
        }
    } else {
        const float e = __expf(-t);
        neumaier_scale_add(st.s, st.cs, e, 1.f);
        if (GRAD) {
            neumaier_scale_add(st.gx, st.cx, e, gx);
            neumaier_scale_add(st.gy, st.cy, e, gy);
            neumaier_scale_add(st.gz, st.cz, e, gz);
        }
        st.L = Lnew;
        st.Lf = (float)Lnew;
    }
}

// Fold one term with exponent t = L_i - L* (FP32); Lnew is the term's log-term
// in FP64, which becomes the reference when t > 0.
template <bool GRAD>
__device__ __forceinline__ void lse_fold(LSE64 &st, float t, double Lnew, float gx, float gy, float gz) {
    if (t <= 0.f) {
        double e = (double)__expf(t);
        st.s += e;
        if (GRAD) {
            st.gx = fma(e, (double)gx, st.gx);
            st.gy = fma(e, (double)gy, st.gy);
            st.gz = fma(e, (double)gz, st.gz);
        }
    } else {
        double e = (double)__expf(-t);
        st.s = fma(st.s, e, 1.0);
        if (GRAD) {
            st.gx = fma(st.gx, e, (double)gx);
            st.gy = fma(st.gy, e, (double)gy);
            st.gz = fma(st.gz, e, (double)gz);
        }
        st.L = Lnew;
        st.Lf = (float)Lnew;
    }
}

// The running lower bound of the smallest term distance, updated in one
// integer min on the bit patterns (fminf costs a second instruction that
// quiets signalling NaNs).  Non-negative floats order as their bit patterns,
// so the result is exact for non-negative bounds; a negative bound (a query
// on a primitive) orders below every non-negative one, and of two negative
// bounds this keeps the one nearer zero, which is still <= 0 <= every
// distance: the result stays a lower bound of the smallest term distance.
__device__ __forceinline__ float min_bound(float a, float b) {
    return __int_as_float(min(__float_as_int(a), __float_as_int(b)));
}

// One term: log-term L (FP64), lower bound dlo of its distance, and g = grad d -
// grad(log w)/alpha (the Eq. 4 numerator direction).
template <bool GRAD, class St>
__device__ __forceinline__ void lse_add(St &st, double L, float dlo, float gx, float gy, float gz) {
    st.mlo = min_bound(st.mlo, dlo);
    lse_fold<GRAD>(st, (float)(L - st.L), L, gx, gy, gz);
}

// A far-field term: log-term L, distance lower bound dlo, and the direction
// given as the exact FP64 difference u = q - y_B with 1/D: the gradient
// numerator takes (e / D) u, one FP32 product and three FP64 FMAs, instead of
// forming and converting an FP32 direction.
template <bool GRAD>
__device__ __forceinline__ void lse_add_far(LSE64 &st, double L, float dlo, double ux, double uy, double uz,
                                            float inv) {
    st.mlo = min_bound(st.mlo, dlo);
    const float t = (float)(L - st.L);
    if (t <= 0.f) {
        const float e = __expf(t);
        st.s += (double)e;
        if (GRAD) {
            const double ei = (double)(e * inv);
            st.gx = fma(ei, ux, st.gx);
            st.gy = fma(ei, uy, st.gy);
            st.gz = fma(ei, uz, st.gz);
        }
    } else {
        const double e = (double)__expf(-t);
        st.s = fma(st.s, e, 1.0);
        if (GRAD) {
            const double i64 = (double)inv;
            st.gx = fma(st.gx, e, ux * i64);
            st.gy = fma(st.gy, e, uy * i64);
            st.gz = fma(st.gz, e, uz * i64);
        }
        st.L = L;
        st.Lf = (float)L;
    }
}
template <bool GRAD>
__device__ __forceinline__ void lse_add_far(LSEc32 &st, double L, float dlo, double ux, double uy, double uz,
                                            float inv) {
    lse_add<GRAD>(st, L, dlo, (float)ux * inv, (float)uy * inv, (float)uz * inv);
}

// clamp(q, lo, hi) in one v_med3_f32 (lo <= hi for every box)
__device__ __forceinline__ float clampf(float q, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(q, lo, hi);
}

// ---------------------------------------------------------------------------
// Triangle weight polynomial (App. C.3): w~ = sum_{a+b<=7} c_ab phi1^a phi2^b
// in FP64, Horner in phi1 outside and in phi2 inside, with both partial
// derivatives carried along.  The monomial form cancels by up to ~500x, which
// FP64 absorbs (~1e-13 relative).  Coefficient k runs over a = 7 .. 0 and,
// for each a, b = 7 - a .. 0.
// ---------------------------------------------------------------------------
struct Poly2 {
    double w, wx, wy;
};

template <class Coef>
__device__ __forceinline__ Poly2 tri_weight(Coef coef, double x, double y) {
    double w = 0.0, wx = 0.0, wy = 0.0;
    int k = 0;
#pragma unroll
    for (int a = 7; a >= 0; --a) {
        coef.next_row();
        double p = coef(k++), dp = 0.0;   // P_a(y) = sum_b c_ab y^b and P_a'(y)
#pragma unroll
        for (int b = 7 - a - 1; b >= 0; --b) {
            dp = fma(dp, y, p);
            p = fma(p, y, coef(k++));
        }
        wx = fma(wx, x, w);
        w = fma(w, x, p);
        wy = fma(wy, x, dp);
    }
    return Poly2{w, wx, wy};
}

// Single valence class: the class's one row, read with scalar loads where
// the polynomial is evaluated, one Horner row (at most 8 coefficients) at a
// time.  The row address passes through an empty asm statement before each
// Horner row, so that the compiler can neither hoist the 36 loads to the
// kernel's entry (keeping 72 scalar registers occupied through the whole
// traversal, which spilled other scalars into vector lanes read back on every
// node step) nor issue them all at once.  The table is read-only while a
// kernel runs, so the row is read through the constant address space, which
// makes the loads scalar.
typedef __attribute__((address_space(4))) const double ConstF64;
struct CoefUniform {
    const double *row;
    __device__ __forceinline__ void next_row() { asm volatile("" : "+s"(row)); }
    __device__ __forceinline__ double operator()(int k) const { return ((ConstF64 *)row)[k]; }
};
__device__ __forceinline__ CoefUniform coef_uniform(const double *row) { return CoefUniform{row}; }
// Several valence classes: the lane's row of the class table, read as the
// Horner loop consumes it (a rolled loop keeps the row out of the registers).
__device__ __forceinline__ Poly2 tri_weight_table(const double *__restrict__ row, double x, double y) {
    double w = 0.0, wx = 0.0, wy = 0.0;
    int k = 0;
#pragma unroll 1
    for (int a = 7; a >= 0; --a) {
        double p = row[k++], dp = 0.0;
#pragma unroll 1
        for (int b = 7 - a - 1; b >= 0; --b) {
            dp = fma(dp, y, p);
            p = fma(p, y, row[k++]);
        }
        wx = fma(wx, x, w);
        w = fma(w, x, p);
        wy = fma(wy, x, dp);
    }
    return Poly2{w, wx, wy};
}

// ---------------------------------------------------------------------------
// Exact leaf terms.  Each returns the distance d (FP64), the log-weight lw,
// a lower bound dlo of the exact distance and, when GRAD, g = grad d -
// grad(log w)/alpha.
// ---------------------------------------------------------------------------
struct Term {
    double d;
    float lw, dlo, gx, gy, gz;
};

template <bool GRAD, class QT>
__device__ __forceinline__ Term point_term(float4 p, QT qx, QT qy, QT qz) {
    const double ex = (double)qx - (double)p.x, ey = (double)qy - (double)p.y, ez = (double)qz - (double)p.z;
    const double s = ddot3(ex, ey, ez, ex, ey, ez);
    const float r = fsqrt((float)s);
    const float inv = r > 0.f ? frcp(r) : 0.f;
    Term t;
    t.d = sqrt_newton(s, r, inv);
    t.lw = 0.f;
    t.dlo = r * kLo;
    t.gx = t.gy = t.gz = 0.f;
    if (GRAD) {
        t.gx = (float)ex * inv; t.gy = (float)ey * inv; t.gz = (float)ez * inv;
    }
    return t;
}

// segment v0 -> v1 with end weights a = 1/|N_0|, b = 1/|N_1| (App. C.2 quartic)
template <bool GRAD, class QT>
__device__ __forceinline__ Term edge_term(float4 r0, float4 r1, QT qx, QT qy, QT qz,
                                          float S, float slogA, float inv_alpha, bool metric) {
    const double ex = (double)r1.x - (double)r0.x, ey = (double)r1.y - (double)r0.y,
                 ez = (double)r1.z - (double)r0.z;
    const double px = (double)qx - (double)r0.x, py = (double)qy - (double)r0.y,
                 pz = (double)qz - (double)r0.z;
    const double ee = ddot3(ex, ey, ez, ex, ey, ez);
    double t = ee > 0.0 ? ddot3(px, py, pz, ex, ey, ez) / ee : 0.0;
    const bool interior = t > 0.0 && t < 1.0;
    t = fmin(fmax(t, 0.0), 1.0);
    const double cx = fma(-t, ex, px), cy = fma(-t, ey, py), cz = fma(-t, ez, pz);
    const double s = ddot3(cx, cy, cz, cx, cy, cz);
    const float r = fsqrt((float)s);
    const float inv = r > 0.f ? frcp(r) : 0.f;
    // w~ = a + (b - a)(3t^2 - 2t^3) + 16 (1 - (a+b)/2) t^2 (1-t)^2
    const double a = r0.w, b = r1.w;
    const double u = t * (1.0 - t);
    const double bump = 16.0 * (1.0 - 0.5 * (a + b));
    const double w = fma(b - a, t * t * (3.0 - 2.0 * t), fma(bump, u * u, a));
    Term o;
    o.d = sqrt_newton(s, r, inv);
    o.lw = fmaf(S, __logf((float)w), slogA);
    o.dlo = dist_lo(r, (float)(fabs(px) + fabs(py) + fabs(pz) + fabs(ex) + fabs(ey) + fabs(ez)));
    o.gx = o.gy = o.gz = 0.f;
    if (GRAD) {
        float gx = (float)cx * inv, gy = (float)cy * inv, gz = (float)cz * inv;
        if (interior) {
            // dw~/dt = 6 (b - a) t (1 - t) + 2 bump t (1 - t)(1 - 2t)
            const float dw = (float)(u * fma(6.0, b - a, 2.0 * bump * (1.0 - 2.0 * t)));
            float k = S * dw * frcp((float)w * (float)ee) * inv_alpha;
            if (metric) k *= inv_alpha;
            gx = fmaf(-k, (float)ex, gx); gy = fmaf(-k, (float)ey, gy); gz = fmaf(-k, (float)ez, gz);
        }
        o.gx = gx; o.gy = gy; o.gz = gz;
    }
    return o;
}

// triangle (v0, v1, v2), barycentric phi1 <-> v1, phi2 <-> v2 (App. B).
// Region classification after Ericson (Real-Time Collision Detection, 5.1.5)
// in FP64 on the exact edge and offset vectors; the region's barycentric
// coordinates give the closest point, q - f(phi) = ap - phi1 ab - phi2 ac.
template <bool GRAD, class QT>
__device__ __forceinline__ Term tri_term(float4 r0, float4 r1, float4 r2, QT qx, QT qy,
                                         QT qz, const EvalArgs &A, float slogA, bool metric) {
    const float S = A.S, inv_alpha = A.inv_alpha;
    const double abx = (double)r1.x - (double)r0.x, aby = (double)r1.y - (double)r0.y,
                 abz = (double)r1.z - (double)r0.z;
    const double acx = (double)r2.x - (double)r0.x, acy = (double)r2.y - (double)r0.y,
                 acz = (double)r2.z - (double)r0.z;
    const double apx = (double)qx - (double)r0.x, apy = (double)qy - (double)r0.y,
                 apz = (double)qz - (double)r0.z;
    const double g11 = ddot3(abx, aby, abz, abx, aby, abz), g12 = ddot3(abx, aby, abz, acx, acy, acz),
                 g22 = ddot3(acx, acy, acz, acx, acy, acz);
    const double d1 = ddot3(abx, aby, abz, apx, apy, apz), d2 = ddot3(acx, acy, acz, apx, apy, apz);
    // the same products against bp = ap - ab and cp = ap - ac
    const double d3 = d1 - g11, d4 = d2 - g12, d5 = d1 - g12, d6 = d2 - g22;
    const double nx = aby * acz - abz * acy, ny = abz * acx - abx * acz, nz = abx * acy - aby * acx;
    const double nn = ddot3(nx, ny, nz, nx, ny, nz);
    const double det = g11 * g22 - g12 * g12;

    // region: 0 face, 1 edge ab, 2 edge ac, 3 edge bc, 4 vertex; the edge and
    // face coordinates are num / den.  Every test is formed and the first that
    // holds, in Ericson's order (vertex a, vertex b, edge ab, vertex c, edge
    // ac, edge bc, else the face), is selected without branches: the 64
    // (query, triangle) pairs a wave evaluates together fall in different
    // regions, and branches would run most of the paths anyway.
    const double vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
    const double e43 = d4 - d3, e56 = d5 - d6;
    const bool in_a = d1 <= 0.0 && d2 <= 0.0;
    const bool in_b = d3 >= 0.0 && d4 <= d3;
    const bool in_ab = vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0;
    const bool in_c = d6 >= 0.0 && d5 <= d6;
    const bool in_ac = vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0;
    const bool in_bc = va <= 0.0 && e43 >= 0.0 && e56 >= 0.0;
    int region = 0;
    double num = vb, num2 = vc, den = va + vb + vc;
    if (in_bc) { region = 3; num = e43; den = e43 + e56; }
    if (in_ac) { region = 2; num = d2; den = d2 - d6; }
    if (in_c) region = 4;
    if (in_ab) { region = 1; num = d1; den = d1 - d3; }
    if (in_b || in_a) region = 4;
    double p1 = (in_b && !in_a) ? 1.0 : 0.0;
    double p2 = (in_c && !(in_a || in_b || in_ab)) ? 1.0 : 0.0;
    if (!(nn > 0.0 && det > 0.0)) {
        // zero-area triangle: it is its longest edge (which covers the other
        // two), first of ab, bc, ca on ties, so the barycentrics are unique
        const double bcx = acx - abx, bcy = acy - aby, bcz = acz - abz;   // exact: v2 - v1
        const double lbc = ddot3(bcx, bcy, bcz, bcx, bcy, bcz);
        p1 = p2 = 0.0;
        if (g11 >= lbc && g11 >= g22) {
            region = 1; num = d1; den = g11;                       // t along ab
        } else if (lbc >= g22) {
            region = 3; num = e43; den = lbc;                      // t along bc
        } else {
            region = 2; num = d2; den = g22;                       // t along ac
        }
    }
    double inv_den = 0.0;
    if (region != 4) {
        inv_den = den > 0.0 ? 1.0 / den : 0.0;
        const double t = fmin(fmax(num * inv_den, 0.0), 1.0);   // degenerate edges clamp here
        p1 = region == 0 ? num * inv_den : (region == 1 ? t : (region == 3 ? 1.0 - t : 0.0));
        p2 = region == 0 ? num2 * inv_den : ((region == 2 || region == 3) ? t : 0.0);
        if (!(nn > 0.0 && det > 0.0) && !(t > 0.0 && t < 1.0)) region = 4;
    }
    const double cx = fma(-p2, acx, fma(-p1, abx, apx)), cy = fma(-p2, acy, fma(-p1, aby, apy)),
                 cz = fma(-p2, acz, fma(-p1, abz, apz));
    const double s = ddot3(cx, cy, cz, cx, cy, cz);
    const float r = fsqrt((float)s);
    const float inv = r > 0.f ? frcp(r) : 0.f;
    const Poly2 w = A.tri_uniform ? tri_weight(coef_uniform(A.tri_table), p1, p2)
                                  : tri_weight_table(A.tri_table + 36 * __float_as_int(r0.w), p1, p2);
    const float o1 = (float)(fabs(apx) + fabs(apy) + fabs(apz) + fabs(abx) + fabs(aby) + fabs(abz) +
                             fabs(acx) + fabs(acy) + fabs(acz));
    Term o;
    o.d = sqrt_newton(s, r, inv);
    o.lw = fmaf(S, __logf((float)w.w), slogA);
    o.dlo = dist_lo(r, o1);
    o.gx = o.gy = o.gz = 0.f;
    if (GRAD) {
        float gx = (float)cx * inv, gy = (float)cy * inv, gz = (float)cz * inv;
        float k = S * frcp((float)w.w) * inv_alpha;
        if (metric) k *= inv_alpha;
        // grad w~ (Eq. 5) in FP64: the barycentric gradients are large (1 / the
        // triangle's altitude) and their combination cancels.  grad w~ =
        // c1 ab + c2 ac in every region.  Face: grad phi1 = (g22 ab - g12 ac) /
        // det, grad phi2 = (g11 ac - g12 ab) / det (va + vb + vc = det is the
        // face region's denominator).  Edge e with parameter t: d t / dq = e /
        // |e|^2 (the edge regions' denominator den is |e|^2), and bc = ac - ab.
        // Vertex: 0 (inv_den = 0 there as well).
        const double cf1 = (w.wx * g22 - w.wy * g12) * inv_den, cf2 = (w.wy * g11 - w.wx * g12) * inv_den;
        const double cbc = (w.wy - w.wx) * inv_den;
        const double c1 = region == 0 ? cf1 : (region == 1 ? w.wx * inv_den : (region == 3 ? -cbc : 0.0));
        const double c2 = region == 0 ? cf2 : (region == 2 ? w.wy * inv_den : (region == 3 ? cbc : 0.0));
        const double wgx = fma(c1, abx, c2 * acx), wgy = fma(c1, aby, c2 * acy), wgz = fma(c1, abz, c2 * acz);
        o.gx = fmaf(-k, (float)wgx, gx);
        o.gy = fmaf(-k, (float)wgy, gy);
        o.gz = fmaf(-k, (float)wgz, gz);
    }
    return o;
}

// ---------------------------------------------------------------------------
// Alg. 1 over one class hierarchy
// ---------------------------------------------------------------------------
template <int CLS, bool GRAD>
__device__ __forceinline__ Term leaf_term(const TreeView &T, const EvalArgs &A, int slot, float4 lo,
                                          float qx, float qy, float qz, bool metric) {
    // a point's leaf record holds the point (its leaf box's corner): reading it
    // here leaves the traversal's node record free to be overwritten by the
    // next node's load
    if (CLS == 0) return point_term<GRAD>(T.leaf[slot], qx, qy, qz);
    if (CLS == 1)
        return edge_term<GRAD>(T.leaf[2 * slot], T.leaf[2 * slot + 1], qx, qy, qz, A.S, (float)T.slogA,
                               A.inv_alpha, metric);
    return tri_term<GRAD>(T.leaf[3 * slot], T.leaf[3 * slot + 1], T.leaf[3 * slot + 2], qx, qy, qz, A,
                          (float)T.slogA, metric);
}

// log-term of a leaf term: L = log w - alpha d
__device__ __forceinline__ double log_term(const EvalArgs &A, const Term &t) {
    return fma(-A.alpha64, t.d, (double)t.lw);
}

// a node record is 32 B (lo, hi); a 32-bit byte offset from the array base
// gives the loads' scalar-base + vector-offset form (node counts stay far
// below 2^27, which the build checks)
__device__ __forceinline__ void load_node(const TreeView &T, int node, float4 &lo, float4 &hi) {
    const char *base = reinterpret_cast<const char *>(T.lo);
    uint32_t off = static_cast<uint32_t>(node) << 5;
    lo = *reinterpret_cast<const float4 *>(base + off);
    hi = *reinterpret_cast<const float4 *>(base + off + 16);
}

// The query in FP64 for the far-field terms' exact differences q - y_B.  The
// traversal loops form it once and pin it in registers (an empty asm that
// takes and returns it), since the compiler would otherwise convert the query
// again for every far-field term.
struct Q64 {
    double x, y, z;
};
__device__ __forceinline__ Q64 q64_pinned(float qx, float qy, float qz) {
    Q64 q{(double)qx, (double)qy, (double)qz};
    asm volatile("" : "+v"(q.x), "+v"(q.y), "+v"(q.z));
    return q;
}

// One step of Alg. 1 on `node`, whose record (lo, hi) is in registers: the
// opening test, then the next node (escape after a far-field term or a leaf,
// else the left child node + 1), whose record is loaded into (lo, hi) before
// the far-field term is added, so that the load overlaps that arithmetic.
// Returns the leaf slot to evaluate, or -1.
template <bool GRAD, bool COUNT, bool PRUNE, class St>
__device__ __forceinline__ int node_visit(const TreeView &T, const EvalArgs &A, float qx, float qy,
                                          float qz, const Q64 &qd, St &st, float4 &lo, float4 &hi,
                                          int &node, float4 &leaf_lo, int &n_vis, int &n_far) {
    const float yx = clampf(qx, lo.x, hi.x);
    const float yy = clampf(qy, lo.y, hi.y);
    const float yz = clampf(qz, lo.z, hi.z);
    const float dx = qx - yx, dy = qy - yy, dz = qz - yz;
    const float D2 = dot3(dx, dy, dz, dx, dy, dz);
    const float ex = hi.x - lo.x, ey = hi.y - lo.y, ez = hi.z - lo.z;
    const float diag2 = dot3(ex, ey, ez, ex, ey, ez);
    const int esc = __float_as_int(lo.w);
    const int pay = __float_as_int(hi.w);
    if (COUNT) ++n_vis;
    // Negligible subtree: every term below this node is at most
    // n_B W_max exp(-alpha D) (D <= each d_i), i.e. its exponent relative to
    // the running maximum is below -A.prune (64: < 1e-27 of the sum), so it
    // cannot change the FP32 result; skip it.
    // D > (log n_B + log W_max - L* + prune) / alpha, tested on squares.
    bool skip = false;
    if (PRUNE) {
        const float logn = (float)max(pay, 0) * (1.f / (1 << kLogFracBits));
        const float thr = (logn + T.lwmax - st.Lf + A.prune) * A.inv_alpha;
        skip = thr < 0.f || D2 > thr * thr;
    }
    const bool far = !skip && diag2 < A.beta2 * D2;
    const bool leaf = !skip && !far && pay < 0;
    int slot = -1;
    if (leaf) {
        slot = pay & 0x7fffffff;
        leaf_lo = lo;
    }
    node = (skip || far || leaf) ? esc : node + 1;
    // every lane loads (a finished lane reads the root's record and ignores it),
    // so the load needs no branch and writes the record registers in place
    load_node(T, node < 0 ? 0 : node, lo, hi);
    if (far) {
        // far field at the closest box point y_B: weight n_B A^S (App. D).
        // D > 0 here: the test passed, so D^2 > |B|^2 / beta^2 >= 0.  The
        // distance in FP64 from the exact differences q - y_B.
        const float D = fsqrt(D2);
        const float inv = frcp(D);
        const double ux = qd.x - (double)yx, uy = qd.y - (double)yy, uz = qd.z - (double)yz;
        const double D64 = sqrt_newton_pos(ddot3(ux, uy, uz, ux, uy, uz), D, inv);
        // log n_B from the payload's fixed point (a leaf's negative payload
        // gives log 1 = 0)
        const double L = fma(-A.alpha64, D64,
                             fma((double)max(pay, 0), 1.0 / (1 << kLogFracBits), T.slogA));
        lse_add_far<GRAD>(st, L, D * kLo, ux, uy, uz, inv);
        if (COUNT) ++n_far;
    }
    return slot;
}

// Alg. 1 over one class hierarchy, stackless (escape indices).  Exact leaf
// terms are expensive and rare (a few percent of the nodes a query visits),
// so a lane that reaches a leaf queues it and the wave evaluates queued leaves
// together once some lane's queue is full (or none can continue); far-field
// terms are added inline.  The set of terms, and so the value up to summation
// order, is that of the recursive Alg. 1.
// Reference for the running maximum before any term is seen: descend to the
// leaf whose box is nearest at every level and take the lower bound
// -alpha (D_leaf + |leaf box| + 1/alpha) of that leaf's term (its weight is
// >= 1 up to rounding).  The traversal's largest term is at least this large
// (the leaf, or a far-field ancestor of it, enters the sum), so s cannot
// underflow, and most terms then fall below the reference, which keeps the
// rescaling branch of lse_fold rare across a wave.
__device__ __forceinline__ float seed_distance(const TreeView &T, float qx, float qy, float qz,
                                               float inv_alpha) {
    int node = 0;
    float4 lo = T.lo[0], hi = T.hi[0];
    while (__float_as_int(hi.w) >= 0) {
        int l = node + 1;
        float4 llo = T.lo[2 * l], lhi = T.hi[2 * l];
        int r = __float_as_int(llo.w);
        float4 rlo = T.lo[2 * r], rhi = T.hi[2 * r];
        float ax = qx - clampf(qx, llo.x, lhi.x), ay = qy - clampf(qy, llo.y, lhi.y),
              az = qz - clampf(qz, llo.z, lhi.z);
        float bx = qx - clampf(qx, rlo.x, rhi.x), by = qy - clampf(qy, rlo.y, rhi.y),
              bz = qz - clampf(qz, rlo.z, rhi.z);
        bool left = dot3(ax, ay, az, ax, ay, az) <= dot3(bx, by, bz, bx, by, bz);
        node = left ? l : r;
        lo = left ? llo : rlo;
        hi = left ? lhi : rhi;
    }
    float dx = qx - clampf(qx, lo.x, hi.x), dy = qy - clampf(qy, lo.y, hi.y),
          dz = qz - clampf(qz, lo.z, hi.z);
    float ex = hi.x - lo.x, ey = hi.y - lo.y, ez = hi.z - lo.z;
    return fsqrt(dot3(dx, dy, dz, dx, dy, dz)) + fsqrt(dot3(ex, ey, ez, ex, ey, ez)) + inv_alpha;
}

template <class St>
__device__ __forceinline__ void lse_seed(St &st, const TreeView &T, const EvalArgs &A, float qx, float qy,
                                         float qz) {
    if (lse_empty(st)) {
        const float sd = seed_distance(T, qx, qy, qz, A.inv_alpha);
        if (sd == sd) {   // NaN queries keep the empty reference
            st.L = -A.alpha64 * (double)sd;
            st.Lf = (float)st.L;
        }
    }
}

// Per-wave LDS queue of the cooperative leaf stage: queued leaf slots and their
// results, lane-minor so that the 64 lanes touch consecutive banks.  A result
// is the term's exponent relative to the owner's reference at the time of the
// flush as an unevaluated sum of two floats (so that a term that becomes the
// new reference enters with its exact log-term) and its gradient direction;
// the worker that evaluated entry (k, owner) overwrites the slot it read with
// the term's distance lower bound.
#ifndef SD_LEAF_QUEUE
#define SD_LEAF_QUEUE 5
#endif
constexpr int kQ = SD_LEAF_QUEUE;   // queued leaves per lane
static_assert(kQ >= 1 && kQ <= 7, "leaf queue depth (three bits in an entry and in the count)");
struct LeafQueue {
    int slot[kQ][64];
    int ent[kQ * 64];
    float res[kQ][5][64];
};

// LDS written by some lanes of a wave and read by others: order within the wave
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fold the owner's queued results: entry k has exponent t_k relative to the
// reference `base` the owner held at the flush (rescalings by earlier entries
// move the reference, so each exponent is re-based in FP64).
template <bool GRAD, class St>
__device__ __forceinline__ void fold_queue(St &st, const LeafQueue &lq, int cnt, int lane) {
    const double base = st.L;
    for (int k = 0; k < cnt; ++k) {
        float gx = 0.f, gy = 0.f, gz = 0.f;
        if (GRAD) { gx = lq.res[k][2][lane]; gy = lq.res[k][3][lane]; gz = lq.res[k][4][lane]; }
        const double Lk = (base + (double)lq.res[k][0][lane]) + (double)lq.res[k][1][lane];
        st.mlo = min_bound(st.mlo, __int_as_float(lq.slot[k][lane]));
        lse_fold<GRAD>(st, (float)(Lk - st.L), Lk, gx, gy, gz);
    }
}

template <int CLS, bool GRAD, bool COUNT, bool PRUNE, class St>
__device__ __forceinline__ void traverse(const TreeView &T, const EvalArgs &A, float qx, float qy,
                                         float qz, St &st, int &n_vis, int &n_far, int &n_leaf,
                                         LeafQueue &lq, bool active = true) {
    const bool metric = (A.flags & SD_GRAD_PAPER_METRIC) != 0;
    int node = (active && T.n_nodes > 0) ? 0 : -1;
    float4 leaf_lo = make_float4(0.f, 0.f, 0.f, 0.f);
    if (node >= 0) lse_seed(st, T, A, qx, qy, qz);
    // (lo, hi): the record of `node` while node >= 0, loaded one step ahead
    float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
    if (node >= 0) load_node(T, node, lo, hi);
    if (CLS == 0 || A.defer == 0) {
        // leaves inline; the loop condition is a wave-uniform mask (see below)
        if (__builtin_amdgcn_sicmp(node, 0, 39 /* >= */) != 0) {
            const Q64 qd = q64_pinned(qx, qy, qz);
            do {
                if (node >= 0) {
                    int slot = node_visit<GRAD, COUNT, PRUNE>(T, A, qx, qy, qz, qd, st, lo, hi, node,
                                                              leaf_lo, n_vis, n_far);
                    if (slot >= 0) {
                        if (COUNT) ++n_leaf;
                        Term t = leaf_term<CLS, GRAD>(T, A, slot, leaf_lo, qx, qy, qz, metric);
                        lse_add<GRAD>(st, log_term(A, t), t.dlo, t.gx, t.gy, t.gz);
                    }
                }
            } while (__builtin_amdgcn_sicmp(node, 0, 39) != 0);
        }
        return;
    }
    // Wave-cooperative leaves: a lane that reaches a leaf queues its slot (up to
    // kQ per lane) in the wave's LDS queue and keeps traversing.  When a lane's
    // queue is full, or no lane can continue, the wave evaluates every queued
    // (query, leaf) pair with all lanes busy (the owner's query and reference
    // are read with lane shuffles), then each owner folds its results into its
    // own sum.
    const int lane = __lane_id();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int cnt = 0;
    while (true) {
        // Node steps until no lane can continue or some lane's queue is full
        // (flush before a lane stalls).  The condition is formed from two
        // compare masks (lanes with a node left, lanes with queue room; no
        // ballot materialisation) and tested at the bottom, so the loop exits
        // uniformly: the compiler then keeps the sum state in place instead of
        // copying it out, on every iteration, for lanes that might leave early.
        uint64_t live = __builtin_amdgcn_sicmp(node, 0, 39 /* >= */);
        uint64_t room = __builtin_amdgcn_sicmp(cnt, kQ, 40 /* < */);
        bool go = ((live & room) != 0) & ((live & ~room) == 0);
        if (go) {
            const Q64 qd = q64_pinned(qx, qy, qz);
            do {
                if (node >= 0 && cnt < kQ) {
                    int slot = node_visit<GRAD, COUNT, PRUNE>(T, A, qx, qy, qz, qd, st, lo, hi, node,
                                                              leaf_lo, n_vis, n_far);
                    if (slot >= 0) {
                        lq.slot[cnt][lane] = slot;
                        ++cnt;
                        if (COUNT) ++n_leaf;
                    }
                }
                live = __builtin_amdgcn_sicmp(node, 0, 39);
                room = __builtin_amdgcn_sicmp(cnt, kQ, 40);
                go = ((live & room) != 0) & ((live & ~room) == 0);
            } while (go);
        }
        if (__ballot(cnt > 0) == 0) break;
        // exclusive prefix of the per-lane counts (kQ <= 7: three bit planes)
        int off = 0, total = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uint64_t m = __ballot((cnt >> b) & 1);
            total += __popcll(m) << b;
            off += __popcll(m & lt) << b;
        }
        for (int k = 0; k < cnt; ++k) lq.ent[off + k] = (lane << 3) | k;
        wave_sync();
        // spread the entries over the lanes still present in the wave (lanes
        // past the end of the query array have already exited)
        const uint64_t present = __ballot(true);
        const int rank = __popcll(present & lt), npresent = __popcll(present);
        const int Lhi = __double2hiint(st.L), Llo = __double2loint(st.L);
        for (int base = 0; base < total; base += npresent) {
            int e = base + rank;
            bool act = e < total;
            int code = act ? lq.ent[e] : 0;
            int owner = code >> 3, k = code & 7;
            float ox = __shfl(qx, owner, 64), oy = __shfl(qy, owner, 64), oz = __shfl(qz, owner, 64);
            const double oL = __hiloint2double(__shfl(Lhi, owner, 64), __shfl(Llo, owner, 64));
            if (act) {
                Term t = leaf_term<CLS, GRAD>(T, A, lq.slot[k][owner], leaf_lo, ox, oy, oz, metric);
                const double tk = log_term(A, t) - oL;
                const float thi = (float)tk;
                lq.res[k][0][owner] = thi;
                lq.res[k][1][owner] = (float)(tk - (double)thi);
                lq.slot[k][owner] = __float_as_int(t.dlo);
                if (GRAD) {
                    lq.res[k][2][owner] = t.gx;
                    lq.res[k][3][owner] = t.gy;
                    lq.res[k][4][owner] = t.gz;
                }
            }
        }
        wave_sync();
        fold_queue<GRAD>(st, lq, cnt, lane);
        cnt = 0;
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// Edges and triangles as query primitives (Sec. 3.4).  A query primitive g
// has NV = 2 or 3 vertices.  Each data primitive's term is the point-query
// term at g(lambda), the point of g closest to it (the simplex-simplex QP of
// App. B, Eq. 10, solved by enumerating its boundary candidates); far-field
// boxes use the per-axis gaps of the halfspaces g lies outside of (App. D),
// a lower bound of the box distance that equals the point formula for a
// point, and direction gap / |gap|.
// ---------------------------------------------------------------------------
// The closest-pair routines are written once for the scalar type R: the
// query vertices travel in FP32 (V3), and the closest point g(lambda) is
// formed in FP64 (V3D) from the exact FP64 vertices, so that it lies on g to
// FP64 rounding and the term at it is exact to the FP64 arithmetic (an FP32
// g(lambda) moves the distance by its rounding at first order where a vertex
// or an edge of g is closest).  The degeneracy thresholds scale with R.
template <class R>
struct V3T {
    R x, y, z;
};
using V3 = V3T<float>;
using V3D = V3T<double>;
template <class R> struct GeomTol;
template <> struct GeomTol<float> {
    static constexpr float tri = 1e-12f, par = 1e-6f, cross = 1e-12f;
};
template <> struct GeomTol<double> {
    static constexpr double tri = 1e-20, par = 1e-14, cross = 1e-24;
};
// a b - c d in FP64: one rounded product and one FMA (the FP32 form above
// keeps the product's rounding error; FP64 has the margin without it)
__device__ __forceinline__ double dop(double a, double b, double c, double d) { return fma(a, b, -(c * d)); }
__device__ __forceinline__ float fmaR(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float rcpR(float x) { return frcp(x); }
// FP64 reciprocal: the hardware estimate and two Newton steps (each squares
// the relative error), instead of the correctly rounded division sequence;
// the closest-pair parameters need no correct rounding.
__device__ __forceinline__ double rcpR(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float med01(float x) { return __builtin_amdgcn_fmed3f(x, 0.f, 1.f); }
__device__ __forceinline__ double med01(double x) { return fmin(fmax(x, 0.0), 1.0); }

__device__ __forceinline__ V3 v3m(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3D v3m(double x, double y, double z) { return V3D{x, y, z}; }
__device__ __forceinline__ V3D v3d(V3 a) { return V3D{(double)a.x, (double)a.y, (double)a.z}; }
template <class R>
__device__ __forceinline__ V3T<R> vsub(V3T<R> a, V3T<R> b) { return v3m(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class R>
__device__ __forceinline__ V3T<R> vaxpy(V3T<R> a, R s, V3T<R> e) {   // a + s e
    return v3m(fmaR(s, e.x, a.x), fmaR(s, e.y, a.y), fmaR(s, e.z, a.z));
}
template <class R>
__device__ __forceinline__ R vdot(V3T<R> a, V3T<R> b) { return fmaR(a.x, b.x, fmaR(a.y, b.y, a.z * b.z)); }
template <class R>
__device__ __forceinline__ V3T<R> vcross(V3T<R> a, V3T<R> b) {
    return v3m(dop(a.y, b.z, a.z, b.y), dop(a.z, b.x, a.x, b.z), dop(a.x, b.y, a.y, b.x));
}
template <class R>
__device__ __forceinline__ R vdist2(V3T<R> a, V3T<R> b) {
    V3T<R> d = vsub(a, b);
    return vdot(d, d);
}

// closest point of segment a b to p
template <class R>
__device__ __forceinline__ V3T<R> seg_point(V3T<R> p, V3T<R> a, V3T<R> b) {
    V3T<R> e = vsub(b, a);
    R ee = vdot(e, e);
    R t = ee > R(0) ? med01(vdot(vsub(p, a), e) * rcpR(ee)) : R(0);
    return vaxpy(a, t, e);
}

// closest point of triangle a b c to p: the plane projection when its
// barycentrics are inside, else the closest of the three edges
template <class R>
__device__ __forceinline__ V3T<R> tri_point(V3T<R> p, V3T<R> a, V3T<R> b, V3T<R> c) {
    V3T<R> e1 = vsub(b, a), e2 = vsub(c, a), r = vsub(p, a);
    R g11 = vdot(e1, e1), g12 = vdot(e1, e2), g22 = vdot(e2, e2);
    R det = dop(g11, g22, g12, g12);
    if (det > GeomTol<R>::tri * g11 * g22) {
        R r1 = vdot(e1, r), r2 = vdot(e2, r);
        R inv = rcpR(det);
        R u = dop(g22, r1, g12, r2) * inv, v = dop(g11, r2, g12, r1) * inv;
        if (u >= R(0) && v >= R(0) && u + v <= R(1)) return vaxpy(vaxpy(a, u, e1), v, e2);
    }
    V3T<R> best = seg_point(p, a, b);
    R bd = vdist2(p, best);
    V3T<R> y = seg_point(p, b, c);
    R d = vdist2(p, y);
    if (d < bd) { bd = d; best = y; }
    y = seg_point(p, c, a);
    d = vdist2(p, y);
    if (d < bd) best = y;
    return best;
}

// the interior stationary point of |x(s) - y(t)|^2 over the two segments, when
// the segments are not (nearly) parallel and it lies inside both: squared
// distance (else +inf), the point on q
template <class R>
__device__ __forceinline__ R seg_seg_interior(V3T<R> p0, V3T<R> p1, V3T<R> q0, V3T<R> q1, V3T<R> &on_q) {
    V3T<R> u = vsub(p1, p0), v = vsub(q1, q0), w = vsub(p0, q0);
    R a = vdot(u, u), b = vdot(u, v), c = vdot(v, v), d = vdot(u, w), e = vdot(v, w);
    R best = R(INFINITY);
    R den = dop(a, c, b, b);
    if (den > GeomTol<R>::par * a * c) {
        R inv = rcpR(den);
        R s = dop(b, e, c, d) * inv, t = dop(a, e, b, d) * inv;
        if (s >= R(0) && s <= R(1) && t >= R(0) && t <= R(1)) {
            V3T<R> x = vaxpy(p0, s, u), y = vaxpy(q0, t, v);
            best = vdist2(x, y);
            on_q = y;
        }
    }
    return best;
}

// closest points of segments p0 p1 and q0 q1: the interior stationary point or
// an endpoint of one against the other; squared distance, point on q
template <class R>
__device__ __forceinline__ R seg_seg(V3T<R> p0, V3T<R> p1, V3T<R> q0, V3T<R> q1, V3T<R> &on_q) {
    R best = seg_seg_interior(p0, p1, q0, q1, on_q);
    V3T<R> y = seg_point(p0, q0, q1);
    R dd = vdist2(p0, y);
    if (dd < best) { best = dd; on_q = y; }
    y = seg_point(p1, q0, q1);
    dd = vdist2(p1, y);
    if (dd < best) { best = dd; on_q = y; }
    dd = vdist2(q0, seg_point(q0, p0, p1));
    if (dd < best) { best = dd; on_q = q0; }
    dd = vdist2(q1, seg_point(q1, p0, p1));
    if (dd < best) { best = dd; on_q = q1; }
    return best;
}

// Quantities of a triangle a b c shared by every test against it: edge
// vectors e1 = b - a, e2 = c - a, their Gram entries, the reciprocal of the
// Gram determinant (0 for a degenerate triangle) and the normal e1 x e2.
template <class R>
struct TriFrame {
    V3T<R> a, e1, e2, n;
    R g11, g12, g22, inv;
    bool ok;
};
template <class R>
__device__ __forceinline__ TriFrame<R> tri_frame(V3T<R> a, V3T<R> b, V3T<R> c) {
    TriFrame<R> f;
    f.a = a;
    f.e1 = vsub(b, a);
    f.e2 = vsub(c, a);
    f.n = vcross(f.e1, f.e2);
    f.g11 = vdot(f.e1, f.e1);
    f.g12 = vdot(f.e1, f.e2);
    f.g22 = vdot(f.e2, f.e2);
    R det = dop(f.g11, f.g22, f.g12, f.g12);
    f.ok = det > GeomTol<R>::tri * f.g11 * f.g22;
    f.inv = f.ok ? rcpR(det) : R(0);
    return f;
}

// Projection y of p onto the plane of the triangle; true when it falls inside
// the triangle (the face region; tri_point's inside test)
template <class R>
__device__ __forceinline__ bool face_proj(const TriFrame<R> &f, V3T<R> p, V3T<R> &y) {
    V3T<R> r = vsub(p, f.a);
    R r1 = vdot(f.e1, r), r2 = vdot(f.e2, r);
    R u = dop(f.g22, r1, f.g12, r2) * f.inv, v = dop(f.g11, r2, f.g12, r1) * f.inv;
    y = vaxpy(vaxpy(f.a, u, f.e1), v, f.e2);
    return f.ok && u >= R(0) && v >= R(0) && u + v <= R(1);
}

// Segment p0 p1 crossing the triangle t0 t1 t2 (frame f): the crossing point,
// accepted when it lies on the triangle up to rounding
template <class R>
__device__ __forceinline__ bool seg_crosses(V3T<R> p0, V3T<R> p1, const TriFrame<R> &f, V3T<R> t0, V3T<R> t1,
                                            V3T<R> t2, V3T<R> &y) {
    R s0 = vdot(f.n, vsub(p0, f.a)), s1 = vdot(f.n, vsub(p1, f.a));
    if (!((s0 <= R(0) && s1 >= R(0)) || (s0 >= R(0) && s1 <= R(0))) || s0 == s1) return false;
    y = vaxpy(p0, s0 * rcpR(s0 - s1), vsub(p1, p0));
    V3T<R> z = tri_point(y, t0, t1, t2);
    return vdist2(y, z) <= GeomTol<R>::cross * (R(1) + vdot(y, y));
}

// Segment p0 p1 against triangle t0 t1 t2: squared distance, the closest point
// on the segment (xs) and on the triangle (xt); a crossing gives 0.  Apart
// from a crossing, the closest pair is an endpoint against the face interior
// or the segment against one of the triangle's edges (App. B's QP optimum lies
// on those boundary faces).
template <class R>
__device__ __forceinline__ R seg_tri(V3T<R> p0, V3T<R> p1, V3T<R> t0, V3T<R> t1, V3T<R> t2, V3T<R> &xs,
                                     V3T<R> &xt) {
    const TriFrame<R> f = tri_frame(t0, t1, t2);
    V3T<R> y;
    if (seg_crosses(p0, p1, f, t0, t1, t2, y)) {
        xs = y;
        xt = y;
        return R(0);
    }
    R best = R(INFINITY);
    xs = p0;
    xt = t0;
    if (face_proj(f, p0, y)) { best = vdist2(p0, y); xt = y; }
    if (face_proj(f, p1, y)) {
        R d = vdist2(p1, y);
        if (d < best) { best = d; xs = p1; xt = y; }
    }
    V3T<R> T3[3] = {t0, t1, t2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R d = seg_seg(T3[k], T3[(k + 1) % 3], p0, p1, y);   // y on p0 p1
        if (d < best) {
            best = d;
            xs = y;
            xt = seg_point(y, T3[k], T3[(k + 1) % 3]);
        }
    }
    return best;
}

// Triangle g against triangle t: the point of g closest to t.  The triangles
// meet when an edge of one crosses the other; otherwise the closest pair is a
// vertex of one against the other's face interior, or a pair of edges.
template <class R>
__device__ __forceinline__ V3T<R> tri_tri_on_g(const V3T<R> (&t)[3], const V3T<R> (&g)[3]) {
    const TriFrame<R> ft = tri_frame(t[0], t[1], t[2]), fg = tri_frame(g[0], g[1], g[2]);
    V3T<R> y;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (seg_crosses(g[k], g[(k + 1) % 3], ft, t[0], t[1], t[2], y)) return y;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (seg_crosses(t[k], t[(k + 1) % 3], fg, g[0], g[1], g[2], y)) return y;
    R best = R(INFINITY);
    V3T<R> out = g[0];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (face_proj(ft, g[k], y)) {
            R d = vdist2(g[k], y);
            if (d < best) { best = d; out = g[k]; }
        }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (face_proj(fg, t[k], y)) {
            R d = vdist2(t[k], y);
            if (d < best) { best = d; out = y; }
        }
    // edge pairs: the interior stationary points, then each vertex of one
    // triangle against each edge of the other (every endpoint candidate of the
    // nine segment pairs, each formed once)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            R d = seg_seg_interior(t[i], t[(i + 1) % 3], g[j], g[(j + 1) % 3], y);   // y on g's edge
            if (d < best) { best = d; out = y; }
        }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            y = seg_point(t[i], g[j], g[(j + 1) % 3]);
            R d = vdist2(t[i], y);
            if (d < best) { best = d; out = y; }
            d = vdist2(g[j], seg_point(g[j], t[i], t[(i + 1) % 3]));
            if (d < best) { best = d; out = g[j]; }
        }
    return out;
}

template <int NV>
struct QPrim {
    V3 v[NV];
    float mn[3], mx[3];   // per-axis extent of the vertices
};

// The point of the query primitive (vertices gv) closest to the data primitive
// (vertices dv: 1 point, 2 edge, 3 triangle), all in one frame, in FP64.
template <int CLS, int NV>
__device__ __forceinline__ V3D closest_on_query(const V3D (&dv)[3], const V3D (&gv)[NV]) {
    V3D y, xs, xt;
    if (CLS == 0) return NV == 2 ? seg_point(dv[0], gv[0], gv[1]) : tri_point(dv[0], gv[0], gv[1], gv[NV - 1]);
    if (CLS == 1) {
        if (NV == 2) {
            seg_seg(dv[0], dv[1], gv[0], gv[1], y);
            return y;
        }
        seg_tri(dv[0], dv[1], gv[0], gv[1], gv[NV - 1], xs, y);
        return y;
    }
    if (NV == 2) {
        seg_tri(gv[0], gv[1], dv[0], dv[1], dv[2], xs, xt);
        return xs;
    }
    const V3D g3[3] = {gv[0], gv[1], gv[NV - 1]};
    return tri_tri_on_g(dv, g3);
}

// Leaf term for a query primitive: the point-query term at g(lambda), the
// point of g closest to the data primitive.  The closest pair is solved in
// FP64 in the frame of the data primitive's first vertex o (the vertex
// differences are exact in FP64), and the term is formed from the data
// primitive's own records and o + g(lambda); a rounding of g(lambda) of
// 2^-50 of the local offsets, and the skipped interior stationary points of
// nearly parallel edges, lower the distance bound by 2^-24 |g(lambda) - o|_1.
template <int CLS, bool GRAD, int NV>
__device__ __forceinline__ Term leaf_term_q(const TreeView &T, const EvalArgs &A, int slot, float4 leaf_lo,
                                            const QPrim<NV> &g, bool metric) {
    float4 r[3];
    if (CLS == 0) {
        r[0] = leaf_lo;
    } else if (CLS == 1) {
        r[0] = T.leaf[2 * slot];
        r[1] = T.leaf[2 * slot + 1];
    } else {
        r[0] = T.leaf[3 * slot];
        r[1] = T.leaf[3 * slot + 1];
        r[2] = T.leaf[3 * slot + 2];
    }
    constexpr int ND = CLS + 1;
    const V3D o = v3m((double)r[0].x, (double)r[0].y, (double)r[0].z);
    V3D dv[3], gv[NV];
    dv[0] = v3m(0.0, 0.0, 0.0);
#pragma unroll
    for (int k = 1; k < 3; ++k)
        dv[k] = k < ND ? vsub(v3m((double)r[k].x, (double)r[k].y, (double)r[k].z), o) : dv[0];
#pragma unroll
    for (int k = 0; k < NV; ++k) gv[k] = vsub(v3d(g.v[k]), o);
    const V3D ql = closest_on_query<CLS, NV>(dv, gv);
    const double qx = o.x + ql.x, qy = o.y + ql.y, qz = o.z + ql.z;
    Term t;
    if (CLS == 0) {
        t = point_term<GRAD>(r[0], qx, qy, qz);
    } else if (CLS == 1) {
        t = edge_term<GRAD>(r[0], r[1], qx, qy, qz, A.S, (float)T.slogA, A.inv_alpha, metric);
    } else {
        t = tri_term<GRAD>(r[0], r[1], r[2], qx, qy, qz, A, (float)T.slogA, metric);
    }
    t.dlo = fmaf(-0x1p-24f, (float)(fabs(ql.x) + fabs(ql.y) + fabs(ql.z)), t.dlo);
    return t;
}

// Alg. 1 step for a query primitive (compare node_visit): the box distance from
// the per-axis gaps, max(mn - hi, 0) + min(mx - lo, 0), in FP32
template <bool GRAD, int NV>
__device__ __forceinline__ int node_visit_q(const TreeView &T, const EvalArgs &A, const QPrim<NV> &g, LSE &st,
                                            float4 &lo, float4 &hi, int &node, float4 &leaf_lo) {
    float dx = fmaxf(g.mn[0] - hi.x, 0.f) + fminf(g.mx[0] - lo.x, 0.f);
    float dy = fmaxf(g.mn[1] - hi.y, 0.f) + fminf(g.mx[1] - lo.y, 0.f);
    float dz = fmaxf(g.mn[2] - hi.z, 0.f) + fminf(g.mx[2] - lo.z, 0.f);
    float D2 = dot3(dx, dy, dz, dx, dy, dz);
    float ex = hi.x - lo.x, ey = hi.y - lo.y, ez = hi.z - lo.z;
    float diag2 = dot3(ex, ey, ez, ex, ey, ez);
    int esc = __float_as_int(lo.w);
    int pay = __float_as_int(hi.w);
    bool far = diag2 < A.beta2 * D2;
    bool leaf = !far && pay < 0;
    int slot = -1;
    if (leaf) {
        slot = pay & 0x7fffffff;
        leaf_lo = lo;
    }
    node = (far || leaf) ? esc : node + 1;
    if (node >= 0) load_node(T, node, lo, hi);
    if (far) {
        // the gaps are rounded FP32 differences: the FP32 distance is as
        // accurate as the far-field box distance can be here
        float D = fsqrt(D2);
        float inv = frcp(D);
        const double L = fma(-A.alpha64, (double)D, fma((double)max(pay, 0), 1.0 / (1 << kLogFracBits), T.slogA));
        lse_add<GRAD>(st, L, D * kLo, dx * inv, dy * inv, dz * inv);
    }
    return slot;
}

// Alg. 1 over one class hierarchy for query primitives, with the same
// wave-cooperative leaf stage as the point traversal (the owner's vertices
// travel by lane shuffles)
template <int CLS, bool GRAD, int NV>
__device__ __forceinline__ void traverse_q(const TreeView &T, const EvalArgs &A, const QPrim<NV> &g, LSE &st,
                                           LeafQueue &lq) {
    const bool metric = (A.flags & SD_GRAD_PAPER_METRIC) != 0;
    int node = T.n_nodes > 0 ? 0 : -1;
    float4 leaf_lo = make_float4(0.f, 0.f, 0.f, 0.f);
    // any vertex of g bounds the distance to the seed leaf from above
    if (node >= 0) lse_seed(st, T, A, g.v[0].x, g.v[0].y, g.v[0].z);
    float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
    if (node >= 0) load_node(T, node, lo, hi);
    if (CLS == 0 || A.defer == 0) {
        if (__builtin_amdgcn_sicmp(node, 0, 39) != 0) {
            do {
                if (node >= 0) {
                    int slot = node_visit_q<GRAD, NV>(T, A, g, st, lo, hi, node, leaf_lo);
                    if (slot >= 0) {
                        Term t = leaf_term_q<CLS, GRAD, NV>(T, A, slot, leaf_lo, g, metric);
                        lse_add<GRAD>(st, log_term(A, t), t.dlo, t.gx, t.gy, t.gz);
                    }
                }
            } while (__builtin_amdgcn_sicmp(node, 0, 39) != 0);
        }
        return;
    }
    const int lane = __lane_id();
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int cnt = 0;
    while (true) {
        uint64_t live = __builtin_amdgcn_sicmp(node, 0, 39);
        uint64_t room = __builtin_amdgcn_sicmp(cnt, kQ, 40);
        bool go = ((live & room) != 0) & ((live & ~room) == 0);
        if (go) {
            do {
                if (node >= 0 && cnt < kQ) {
                    int slot = node_visit_q<GRAD, NV>(T, A, g, st, lo, hi, node, leaf_lo);
                    if (slot >= 0) {
                        lq.slot[cnt][lane] = slot;
                        ++cnt;
                    }
                }
                live = __builtin_amdgcn_sicmp(node, 0, 39);
                room = __builtin_amdgcn_sicmp(cnt, kQ, 40);
                go = ((live & room) != 0) & ((live & ~room) == 0);
            } while (go);
        }
        if (__ballot(cnt > 0) == 0) break;
        int off = 0, total = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            uint64_t m = __ballot((cnt >> b) & 1);
            total += __popcll(m) << b;
            off += __popcll(m & lt) << b;
        }
        for (int k = 0; k < cnt; ++k) lq.ent[off + k] = (lane << 3) | k;
        wave_sync();
        const uint64_t present = __ballot(true);
        const int rank = __popcll(present & lt), npresent = __popcll(present);
        const int Lhi = __double2hiint(st.L), Llo = __double2loint(st.L);
        for (int base = 0; base < total; base += npresent) {
            int e = base + rank;
            bool act = e < total;
            int code = act ? lq.ent[e] : 0;
            int owner = code >> 3, k = code & 7;
            const double oL = __hiloint2double(__shfl(Lhi, owner, 64), __shfl(Llo, owner, 64));
            QPrim<NV> og;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                og.v[v] = v3m(__shfl(g.v[v].x, owner, 64), __shfl(g.v[v].y, owner, 64), __shfl(g.v[v].z, owner, 64));
            if (act) {
                Term t = leaf_term_q<CLS, GRAD, NV>(T, A, lq.slot[k][owner], leaf_lo, og, metric);
                const double tk = log_term(A, t) - oL;
                const float thi = (float)tk;
                lq.res[k][0][owner] = thi;
                lq.res[k][1][owner] = (float)(tk - (double)thi);
                lq.slot[k][owner] = __float_as_int(t.dlo);
                if (GRAD) {
                    lq.res[k][2][owner] = t.gx;
                    lq.res[k][3][owner] = t.gy;
                    lq.res[k][4][owner] = t.gz;
                }
            }
        }
        wave_sync();
        fold_queue<GRAD>(st, lq, cnt, lane);
        cnt = 0;
        wave_sync();
    }
}

// Spread consecutive logical blocks over one XCD: hardware dispatches workgroup
// i to XCD i % 8, so logical block = start(XCD) + i / 8 keeps each XCD's L2 on
// a contiguous range of (Morton-ordered) queries.
__device__ __forceinline__ int xcd_block(int i, int G) {
    const int nx = 8;
    int q = G / nx, r = G % nx;
    int x = i % nx, k = i / nx;
    return x * q + min(x, r) + k;
}

// Alg. 2: d = -(L* + log s) / alpha in FP64, rounded once to FP32; grad = G / s.
// By default d is then clamped to the smallest lower bound of a term distance
// (see the head of this file), which keeps d <= d_min in FP32.
template <bool GRAD, class St>
__device__ __forceinline__ void final_value(const EvalArgs &A, const St &st, float &d, float &gx,
                                            float &gy, float &gz) {
    gx = gy = gz = 0.f;
    const double s = lse_sum(st);
    if (!(s > 0.0) && !(s != s)) {
        d = INFINITY;   // empty scene: the empty sum
        return;
    }
    d = (float)(-(st.L + log(s)) * A.inv_alpha64);
    if (A.clamp && d > st.mlo) d = st.mlo;   // NaN stays NaN
    if (GRAD) {
        const double inv = 1.0 / s;
        double nx, ny, nz;
        lse_num(st, nx, ny, nz);
        gx = (float)(nx * inv);
        gy = (float)(ny * inv);
        gz = (float)(nz * inv);
    }
}

template <bool GRAD, class St>
__device__ __forceinline__ void finalize(const EvalArgs &A, const St &st, int qi) {
    float d, gx, gy, gz;
    final_value<GRAD>(A, st, d, gx, gy, gz);
    A.d_out[qi] = d;
    if (GRAD) {
        A.g_out[3 * (int64_t)qi] = gx;
        A.g_out[3 * (int64_t)qi + 1] = gy;
        A.g_out[3 * (int64_t)qi + 2] = gz;
    }
}


// Waves per SIMD the traversal is compiled for (register budget): four, i.e.
// at most 128 registers.  Single-class variants fit without it (triangles:
// 124); the mixed-class ones would take 133-140 registers and run three
// waves, and the fourth wave is worth about 6 % on the three-class street
// scene at the cost of 12-20 bytes of spills.
#ifndef SD_EVAL_WPE
#define SD_EVAL_WPE 4
#endif
#define SD_EVAL_ATTR __attribute__((amdgpu_waves_per_eu(SD_EVAL_WPE, SD_EVAL_WPE)))
// (Point-only variants would fit eight waves per SIMD; measured on the
// 20M-point terrain they run 20 % slower than with four: the extra queries in
// flight evict each other's hierarchy nodes from the caches.)
// One wave per workgroup: a workgroup's resources are released when its
// slowest wave ends, and the traversal's trip counts spread widely, so the
// smallest workgroup wastes the least.  Measured against 256, 512 and 1024
// threads on the terrain and icosphere workloads: 2-5 % faster than 256,
// while 1024 threads are 14-22 % slower.
#ifndef SD_EVAL_BLOCK
#define SD_EVAL_BLOCK 64
#endif
constexpr int kEB = SD_EVAL_BLOCK;
template <bool GRAD, bool COUNT, int MASK, bool C32 = false>
__global__ void __launch_bounds__(kEB) SD_EVAL_ATTR
k_eval(EvalArgs A) {
    // With a thread count on the device the launch is sized for its upper
    // bound: the blocks with work are the first ceil(count / kB), spread over
    // the XCDs by the same mapping sized for them, and the rest exit.
    int nthr = A.nthr, G = gridDim.x;
    if (A.nthr_dev) {
        nthr = min(nthr, (int)min(*A.nthr_dev, 0x7fffffffu));
        G = (nthr + kEB - 1) / kEB;
        if ((int)blockIdx.x >= G) return;
    }
    int i = xcd_block(blockIdx.x, G) * kEB + threadIdx.x;
    if (i >= nthr) return;
    int qi = A.perm ? (int)A.perm[i] : i;
    if ((unsigned)qi >= (unsigned)A.nq) return;
    float qx = A.Q[3 * (int64_t)qi], qy = A.Q[3 * (int64_t)qi + 1], qz = A.Q[3 * (int64_t)qi + 2];
    __shared__ LeafQueue lqs[(MASK & 6) ? kEB / 64 : 1];
    LeafQueue &lq = lqs[(MASK & 6) ? threadIdx.x / 64 : 0];
    typename std::conditional<C32, LSEc32, LSE64>::type st;
    lse_init(st);
    int nv = 0, nf = 0, nl = 0, nl0 = 0, nl1 = 0;
    constexpr bool PRUNE = (MASK & 8) != 0;
    if (MASK & 1) traverse<0, GRAD, COUNT, PRUNE>(A.tree[0], A, qx, qy, qz, st, nv, nf, nl, lq);
    if (COUNT) nl0 = nl;
    if (MASK & 2) traverse<1, GRAD, COUNT, PRUNE>(A.tree[1], A, qx, qy, qz, st, nv, nf, nl, lq);
    if (COUNT) nl1 = nl - nl0;
    if (MASK & 4) traverse<2, GRAD, COUNT, PRUNE>(A.tree[2], A, qx, qy, qz, st, nv, nf, nl, lq);
    if (COUNT) {
        if (A.flags & SD_COUNTERS_BY_CLASS) {
            int32_t *c = A.counts + 5 * (int64_t)qi;
            c[0] = nv; c[1] = nf; c[2] = nl0; c[3] = nl1; c[4] = nl - nl0 - nl1;
        } else {
            A.counts[3 * (int64_t)qi] = nv;
            A.counts[3 * (int64_t)qi + 1] = nf;
            A.counts[3 * (int64_t)qi + 2] = nl;
        }
        return;
    }
    finalize<GRAD>(A, st, qi);
}

// all-pairs: tiles of leaf records in LDS, every primitive evaluated exactly
template <int CLS, int K, bool GRAD>
__device__ __forceinline__ void brute_class(const TreeView &T, int64_t n, const EvalArgs &A,
                                            float4 *tile, float qx, float qy, float qz, LSE &st) {
    const bool metric = (A.flags & SD_GRAD_PAPER_METRIC) != 0;
    for (int64_t base = 0; base < n; base += kB) {
        int cnt = (int)min<int64_t>(kB, n - base);
        __syncthreads();
        for (int j = threadIdx.x; j < cnt * K; j += kB) tile[j] = T.leaf[base * K + j];
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            Term t;
            if (CLS == 0) t = point_term<GRAD>(tile[j], qx, qy, qz);
            else if (CLS == 1)
                t = edge_term<GRAD>(tile[2 * j], tile[2 * j + 1], qx, qy, qz, A.S, (float)T.slogA,
                                    A.inv_alpha, metric);
            else
                t = tri_term<GRAD>(tile[3 * j], tile[3 * j + 1], tile[3 * j + 2], qx, qy, qz,
                                   A, (float)T.slogA, metric);
            lse_add<GRAD>(st, log_term(A, t), t.dlo, t.gx, t.gy, t.gz);
        }
    }
}

template <bool GRAD>
__global__ void __launch_bounds__(kB) k_brute(EvalArgs A, int64_t n0, int64_t n1, int64_t n2) {
    __shared__ float4 tile[3 * kB];
    int i = blockIdx.x * kB + threadIdx.x;
    bool live = i < A.nq;
    int qi = live ? i : 0;
    float qx = A.Q[3 * (int64_t)qi], qy = A.Q[3 * (int64_t)qi + 1], qz = A.Q[3 * (int64_t)qi + 2];
    LSE st;
    lse_init(st);
    brute_class<0, 1, GRAD>(A.tree[0], n0, A, tile, qx, qy, qz, st);
    brute_class<1, 2, GRAD>(A.tree[1], n1, A, tile, qx, qy, qz, st);
    brute_class<2, 3, GRAD>(A.tree[2], n2, A, tile, qx, qy, qz, st);
    if (live) finalize<GRAD>(A, st, qi);
}

// ---------------------------------------------------------------------------
// query ordering: 30-bit Morton keys in the (enlarged) scene box
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ff;
    x = (x | x << 16) & 0x030000ff;
    x = (x | x << 8) & 0x0300f00f;
    x = (x | x << 4) & 0x030c30c3;
    x = (x | x << 2) & 0x09249249;
    return x;
}

__global__ void __launch_bounds__(kB)
k_query_keys(const float *__restrict__ Q, const uint32_t *__restrict__ idx, int64_t n,
             const uint32_t *__restrict__ n_dev, float lx, float ly, float lz, float sx, float sy,
             float sz, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (n_dev) n = min(n, (int64_t)*n_dev);
    if (i >= n) return;
    int64_t j = idx ? (int64_t)idx[i] : i;
    float u[3] = {(Q[3 * j] - lx) * sx, (Q[3 * j + 1] - ly) * sy, (Q[3 * j + 2] - lz) * sz};
    uint32_t c = 0;
    for (int a = 0; a < 3; ++a) {
        float v = fminf(fmaxf(u[a], 0.f), 1.f);   // NaN -> 0
        uint32_t q = (uint32_t)fminf(v * 1024.f, 1023.f);
        c |= spread10(q) << (2 - a);
    }
    keys[i] = c;
    vals[i] = (uint32_t)j;
}

// Sphere tracing of the level set d = level (Hart 1996; Sec. 4.2 renders the
// zero isosurface this way): per ray, x = o + t u starts at t = 0 and moves by
// r = d(x) - level until r <= eps (hit at t), t > t_max or max_steps steps
// (miss: +inf).  Each step is one full Alg. 1 / Alg. 2 evaluation (value only)
// inside this kernel; a lane whose ray has ended leaves the loop, and the
// traversal's wave-cooperative leaf stage works with the lanes still present.
// value + gradient for query primitives with NV vertices (G: n x NV x 3)
// Compiled for three waves per SIMD (at most 168 registers): the FP64
// closest-pair geometry spills heavily within 128 registers (up to 290 for
// triangles on triangles), and the third wave's budget is about 10 % faster
// for edges and triangles as queries than the fourth wave's.
template <int NV, int MASK>
__global__ void __launch_bounds__(kEB) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_evalq(EvalArgs A, const float *__restrict__ G) {
    int i = xcd_block(blockIdx.x, gridDim.x) * kEB + threadIdx.x;
    if (i >= A.nthr) return;
    int qi = A.perm ? (int)A.perm[i] : i;
    if ((unsigned)qi >= (unsigned)A.nq) return;
    QPrim<NV> g;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const float *p = G + 3 * ((int64_t)qi * NV + v);
        g.v[v] = v3m(p[0], p[1], p[2]);
    }
    g.mn[0] = g.mx[0] = g.v[0].x;
    g.mn[1] = g.mx[1] = g.v[0].y;
    g.mn[2] = g.mx[2] = g.v[0].z;
#pragma unroll
    for (int v = 1; v < NV; ++v) {
        g.mn[0] = fminf(g.mn[0], g.v[v].x); g.mx[0] = fmaxf(g.mx[0], g.v[v].x);
        g.mn[1] = fminf(g.mn[1], g.v[v].y); g.mx[1] = fmaxf(g.mx[1], g.v[v].y);
        g.mn[2] = fminf(g.mn[2], g.v[v].z); g.mx[2] = fmaxf(g.mx[2], g.v[v].z);
    }
    __shared__ LeafQueue lqs[(MASK & 6) ? kEB / 64 : 1];
    LeafQueue &lq = lqs[(MASK & 6) ? threadIdx.x / 64 : 0];
    LSE st;
    lse_init(st);
    if (MASK & 1) traverse_q<0, true, NV>(A.tree[0], A, g, st, lq);
    if (MASK & 2) traverse_q<1, true, NV>(A.tree[1], A, g, st, lq);
    if (MASK & 4) traverse_q<2, true, NV>(A.tree[2], A, g, st, lq);
    finalize<true>(A, st, qi);
}

__global__ void __launch_bounds__(kB)
k_centroids(const float *__restrict__ G, int nv, int64_t n, float *__restrict__ C) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i >= n) return;
    float c[3] = {0.f, 0.f, 0.f};
    for (int v = 0; v < nv; ++v)
        for (int a = 0; a < 3; ++a) c[a] += G[3 * (i * nv + v) + a];
    for (int a = 0; a < 3; ++a) C[3 * i + a] = c[a] / (float)nv;
}

template <int NV>
void launch_evalq(const EvalArgs &A, const float *G, int mask, hipStream_t s) {
    const unsigned grid = (unsigned)(((int64_t)A.nthr + kEB - 1) / kEB);
    switch (mask & 7) {
#define SD_CASE(m) \
    case m: hipLaunchKernelGGL((k_evalq<NV, m>), dim3(grid), dim3(kEB), 0, s, A, G); break;
        SD_CASE(1) SD_CASE(2) SD_CASE(3) SD_CASE(4) SD_CASE(5) SD_CASE(6) SD_CASE(7)
#undef SD_CASE
        default: break;
    }
}

struct TraceArgs {
    const float *O, *U;
    float level, eps, t_max;
    int32_t max_steps;
    float *t_out;
    int32_t *steps_out;
};

template <int MASK>
__global__ void __launch_bounds__(kEB) k_trace(EvalArgs A, TraceArgs R) {
    const int i = blockIdx.x * kEB + threadIdx.x;
    if (i >= A.nq) return;
    const float ox = R.O[3 * (int64_t)i], oy = R.O[3 * (int64_t)i + 1], oz = R.O[3 * (int64_t)i + 2];
    const float ux = R.U[3 * (int64_t)i], uy = R.U[3 * (int64_t)i + 1], uz = R.U[3 * (int64_t)i + 2];
    __shared__ LeafQueue lqs[(MASK & 6) ? kEB / 64 : 1];
    LeafQueue &lq = lqs[(MASK & 6) ? threadIdx.x / 64 : 0];
    float t = 0.f, t_hit = INFINITY;
    int steps = 0;
    while (true) {
        const float qx = fmaf(t, ux, ox), qy = fmaf(t, uy, oy), qz = fmaf(t, uz, oz);
        LSE st;
        lse_init(st);
        int nv = 0, nf = 0, nl = 0;
        if (MASK & 1) traverse<0, false, false, false>(A.tree[0], A, qx, qy, qz, st, nv, nf, nl, lq);
        if (MASK & 2) traverse<1, false, false, false>(A.tree[1], A, qx, qy, qz, st, nv, nf, nl, lq);
        if (MASK & 4) traverse<2, false, false, false>(A.tree[2], A, qx, qy, qz, st, nv, nf, nl, lq);
        float d, gx, gy, gz;
        final_value<false>(A, st, d, gx, gy, gz);
        ++steps;
        const float r = d - R.level;
        if (r <= R.eps) {
            t_hit = t;
            break;
        }
        t += r;
        if (!(t <= R.t_max) || steps >= R.max_steps) break;   // also ends NaN rays
    }
    R.t_out[i] = t_hit;
    if (R.steps_out) R.steps_out[i] = steps;
}

void launch_trace(const EvalArgs &A, const TraceArgs &R, int mask, hipStream_t s) {
    const unsigned grid = (unsigned)(((int64_t)A.nq + kEB - 1) / kEB);
    switch (mask & 7) {
#define SD_CASE(m) \
    case m: hipLaunchKernelGGL((k_trace<m>), dim3(grid), dim3(kEB), 0, s, A, R); break;
        SD_CASE(1) SD_CASE(2) SD_CASE(3) SD_CASE(4) SD_CASE(5) SD_CASE(6) SD_CASE(7)
#undef SD_CASE
        default: break;
    }
}

__global__ void __launch_bounds__(kB) k_fill_f32(float *__restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (i < n) p[i] = v;
}

template <bool GRAD, bool COUNT, bool C32 = false>
void launch_eval(const EvalArgs &A, int mask, hipStream_t s) {
    const unsigned grid = (unsigned)(((int64_t)A.nthr + kEB - 1) / kEB);
    switch (mask) {
#define SD_CASE(m) \
    case m: hipLaunchKernelGGL((k_eval<GRAD, COUNT, m, C32>), dim3(grid), dim3(kEB), 0, s, A); break;
        SD_CASE(1) SD_CASE(2) SD_CASE(3) SD_CASE(4) SD_CASE(5) SD_CASE(6) SD_CASE(7)
        SD_CASE(9) SD_CASE(10) SD_CASE(11) SD_CASE(12) SD_CASE(13) SD_CASE(14) SD_CASE(15)
#undef SD_CASE
        default: break;
    }
}

}  // namespace

// Scratch of query_order_into for nq queries: the Morton keys, the sort's
// second key and value buffers and its histogram / scan space, each aligned to
// 256 bytes.
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t query_order_scratch_bytes(int64_t nq) {
    const size_t n = (size_t)std::max<int64_t>(nq, 1);
    return 2 * align256(n * sizeof(uint64_t)) + align256(n * sizeof(uint32_t)) +
           align256(radix_sort_temp_bytes(nq));
}

// Morton order of the queries in the scene box enlarged by half its extent on
// every side (queries outside clamp to the boundary cells), with the scratch
// given by the caller (query_order_scratch_bytes(nq) bytes, 256-aligned).
// With idx, only the n queries idx[0..n) are ordered and perm receives those
// indices sorted; with n_dev as well, only idx[0..min(n, *n_dev)).
int query_order_into(const sd_scene *sc, const float *Q, int64_t nq, uint32_t *perm, void *scratch,
                     hipStream_t s, const uint32_t *idx, const uint32_t *n_dev = nullptr) {
    if (nq <= 0) return SD_OK;
    char *p = static_cast<char *>(scratch);
    const size_t n = (size_t)nq;
    uint64_t *keys = reinterpret_cast<uint64_t *>(p);
    p += align256(n * sizeof(uint64_t));
    uint64_t *keys2 = reinterpret_cast<uint64_t *>(p);
    p += align256(n * sizeof(uint64_t));
    uint32_t *vals2 = reinterpret_cast<uint32_t *>(p);
    p += align256(n * sizeof(uint32_t));
    float ext[3], lo[3];
    for (int a = 0; a < 3; ++a) {
        float e = std::max(sc->box[3 + a] - sc->box[a], 1e-6f);
        lo[a] = sc->box[a] - 0.5f * e;
        ext[a] = 2.f * e;
    }
    unsigned grid = (unsigned)((nq + kB - 1) / kB);
    hipLaunchKernelGGL(k_query_keys, dim3(grid), dim3(kB), 0, s, Q, idx, nq, n_dev, lo[0], lo[1], lo[2],
                       1.f / ext[0], 1.f / ext[1], 1.f / ext[2], keys, perm);
    SD_TRY(radix_sort_pairs(keys, perm, keys2, vals2, nq, 30, p, s, n_dev));
    return SD_OK;
}

// query_order_into with stream-ordered scratch of its own
int query_order(const sd_scene *sc, const float *Q, int64_t nq, uint32_t *perm, hipStream_t s,
                const uint32_t *idx, const uint32_t *n_dev) {
    if (nq <= 0) return SD_OK;
    char *scratch;
    AsyncScratch tmp(s);
    SD_TRY(tmp.alloc(&scratch, (int64_t)query_order_scratch_bytes(nq)));
    return query_order_into(sc, Q, nq, perm, scratch, s, idx, n_dev);
}

// ---------------------------------------------------------------------------
// Allocation-free evaluation: the query order's scratch lives in this
// file-scope device array (one copy per GPU the library runs on, held until
// the process ends).  Host code must not use the array's name as a device
// address: its address on each device comes from hipGetSymbolAddress, taken
// once per device with that device current.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxQ = SD_NOALLOC_MAX_QUERIES;
constexpr size_t kNoAllocBytes =
    4 * kNoAllocMaxQ + 2 * 8 * kNoAllocMaxQ + 4 * kNoAllocMaxQ + (size_t)(4 << 20);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static int noalloc_scratch(void **out) {
    static std::mutex mu;
    static void *ptr[64] = {};
    int dev = 0;
    SD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(SD_EUNSUPPORTED, "sd_eval_grad_noalloc: device index above 63");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SD_EHIP, std::string("sd_eval_grad_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return SD_OK;
}

int eval_grad_noalloc(const sd_scene *sc, const float *Q, int64_t nq, const sd_params *p, float *d_out,
                      float *g_out, hipStream_t s) {
    if (nq > kNoAllocMaxQ)
        return fail(SD_EINVAL, "sd_eval_grad_noalloc: nQ = " + std::to_string(nq) + " exceeds the limit of " +
                                   std::to_string(kNoAllocMaxQ) + " queries per call");
    if (nq == 0) return SD_OK;
    sd_params q = *p;
    const uint32_t *perm = nullptr;
    // the same ordering rule as sd_eval_grad: Morton order from 4096 queries on
    if (!(p->flags & SD_NO_QUERY_SORT) && nq >= 4096 && sc->n_nodes[0] + sc->n_nodes[1] + sc->n_nodes[2] > 0) {
        void *base;
        SD_TRY(noalloc_scratch(&base));
        uint32_t *pm = static_cast<uint32_t *>(base);
        void *rest = static_cast<char *>(base) + align256((size_t)nq * sizeof(uint32_t));
        if (align256((size_t)nq * 4) + query_order_scratch_bytes(nq) > kNoAllocBytes)
            return fail(SD_EHIP, "sd_eval_grad_noalloc: scratch layout exceeds the static array");
        SD_TRY(query_order_into(sc, Q, nq, pm, rest, s, nullptr));
        perm = pm;
    }
    q.flags |= SD_NO_QUERY_SORT;
    return eval_dispatch(sc, Q, perm, nq, &q, d_out, g_out, nullptr, false, s);
}

// Leaf evaluation mode: 1 = wave-cooperative leaf stage (default), 0 = each
// lane evaluates its leaves inline; SD_LEAF_MODE overrides it for comparisons.
static int defer_threshold() {
    static int v = [] {
        const char *e = getenv("SD_LEAF_MODE");
        return e ? (atoi(e) != 0 ? 1 : 0) : 1;
    }();
    return v;
}

// alpha x scene diagonal above which the evaluation skips negligible
// subtrees (SD_PRUNE_ALPHA_DIAG overrides it for comparisons)
static double prune_alpha_diag() {
    static double v = [] {
        const char *e = getenv("SD_PRUNE_ALPHA_DIAG");
        return e ? atof(e) : 1000.0;
    }();
    return v;
}

// Arguments common to every evaluation (per-class hierarchies, weight data,
// alpha, beta, flags); returns the kernel variant: class mask (bits 1, 2, 4)
// plus 8 when negligible subtrees are skipped.
static int make_args(const sd_scene *sc, const sd_params *p, EvalArgs &A) {
    memset(&A, 0, sizeof(A));
    double alpha = p->alpha;
    double S = alpha / std::max<double>(alpha, p->alpha_u);
    for (int c = 0; c < 3; ++c) {
        A.tree[c].lo = sc->lo[c];
        A.tree[c].hi = sc->hi[c];
        A.tree[c].leaf = sc->leaf[c];
        A.tree[c].n_nodes = (int32_t)sc->n_nodes[c];
        A.tree[c].slogA = S * log(sc->A[c]);
        // largest possible log-weight of any term of the class (pruning bound):
        // w~ <= 1 + |a - b|/2 <= 1.5 for edges, <= the largest Bernstein
        // coefficient for triangles (convex hull), w = 1 for points
        double wmax = c == 0 ? 1.0 : (c == 1 ? 1.5 : std::max(1.0, sc->tri_wmax));
        A.tree[c].lwmax = (float)(S * (log(sc->A[c]) + log(wmax))) + 1e-3f;
    }
    A.tri_uniform = sc->n_tri_classes <= 1 ? 1 : 0;
    A.tri_table = sc->tri_table;
    A.alpha = p->alpha;
    A.inv_alpha = (float)(1.0 / alpha);
    A.beta2 = p->beta * p->beta;
    A.S = (float)S;
    A.alpha64 = alpha;
    A.inv_alpha64 = 1.0 / alpha;
    A.clamp = (p->flags & SD_NO_CONSERVATIVE_ROUNDING) ? 0 : 1;
    A.defer = defer_threshold();
    A.prune = 64.f;
    A.flags = p->flags;
    int mask = (sc->n[0] > 0 ? 1 : 0) | (sc->n[1] > 0 ? 2 : 0) | (sc->n[2] > 0 ? 4 : 0);
    // Negligible-subtree skipping (bit 8 of the kernel variant) only where it
    // can pay for its per-node test: a subtree is skipped when it lies at
    // least 64/alpha beyond the running reference, which inside a scene of
    // diagonal L happens only for alpha L well above 64.
    {
        double ex = sc->box[3] - sc->box[0], ey = sc->box[4] - sc->box[1], ez = sc->box[5] - sc->box[2];
        double diag = sqrt(ex * ex + ey * ey + ez * ez);
        if (mask != 0 && !(p->flags & SD_NO_PRUNE) && alpha * diag > prune_alpha_diag()) mask |= 8;
    }
    return mask;
}

int eval_dispatch(const sd_scene *sc, const float *Q, const uint32_t *perm_in, int64_t nq,
                  const sd_params *p, float *d_out, float *g_out, int32_t *counts, bool brute,
                  hipStream_t s, int64_t nthr, const uint32_t *nthr_dev) {
    if (nthr < 0) nthr = nq;
    if (nq == 0 || nthr == 0) return SD_OK;
    if (nq > (int64_t)0x7fffffff - kB) return fail(SD_EUNSUPPORTED, "more than 2^31 queries per call");
    if (nthr != nq && (!perm_in || brute || counts || nthr > nq))
        return fail(SD_EINVAL, "a thread count below the query count needs an index list");
    if (nthr_dev && (!perm_in || brute || counts))
        return fail(SD_EINVAL, "a thread count on the device needs an index list");
    const bool c32 = (p->flags & SD_LSE_COMPENSATED_F32) != 0;
    if (c32 && (brute || counts || !g_out))
        return fail(SD_EUNSUPPORTED,
                    "SD_LSE_COMPENSATED_F32 is compiled for the value + gradient traversal only");
    EvalArgs A;
    int mask = make_args(sc, p, A);
    A.nq = (int32_t)nq;
    A.nthr = (int32_t)nthr;
    A.nthr_dev = nthr_dev;
    A.Q = Q;
    A.d_out = d_out;
    A.g_out = g_out;
    A.counts = counts;
    unsigned grid = (unsigned)((nthr + kB - 1) / kB);

    if (mask == 0) {
        // empty scene: the empty sum gives +inf and a zero gradient
        if (counts) {
            const int64_t k = (p->flags & SD_COUNTERS_BY_CLASS) ? 5 : 3;
            SD_HIP(hipMemsetAsync(counts, 0, k * nq * sizeof(int32_t), s));
            return SD_OK;
        }
        brute = true;
    }
    if (brute) {
        if (g_out)
            hipLaunchKernelGGL(k_brute<true>, dim3(grid), dim3(kB), 0, s, A, sc->n[0], sc->n[1], sc->n[2]);
        else
            hipLaunchKernelGGL(k_brute<false>, dim3(grid), dim3(kB), 0, s, A, sc->n[0], sc->n[1], sc->n[2]);
        SD_HIP(hipGetLastError());
        return SD_OK;
    }
    uint32_t *perm = nullptr;
    AsyncScratch tmp(s);
    if (perm_in) {
        A.perm = perm_in;
    } else if (!(p->flags & SD_NO_QUERY_SORT) && nq >= 4096) {
        SD_TRY(tmp.alloc(&perm, nq));
        SD_TRY(query_order(sc, Q, nq, perm, s));
        A.perm = perm;
    }
    if (counts) {
        if (g_out) launch_eval<true, true>(A, mask, s);
        else launch_eval<false, true>(A, mask, s);
    } else if (g_out && c32) {
        launch_eval<true, false, true>(A, mask, s);
    } else if (g_out) {
        launch_eval<true, false>(A, mask, s);
    } else {
        launch_eval<false, false>(A, mask, s);
    }
    SD_HIP(hipGetLastError());
    return SD_OK;
}

int evalq_dispatch(const sd_scene *sc, const float *G, int nv, int64_t n, const sd_params *p, float *d_out,
                   float *g_out, hipStream_t s) {
    if (n == 0) return SD_OK;
    if (n > (int64_t)0x7fffffff - kB) return fail(SD_EUNSUPPORTED, "more than 2^31 query primitives per call");
    if (p->flags & SD_LSE_COMPENSATED_F32)
        return fail(SD_EUNSUPPORTED, "SD_LSE_COMPENSATED_F32 is compiled for the point-query traversal only");
    EvalArgs A;
    const int mask = make_args(sc, p, A) & 7;
    A.nq = (int32_t)n;
    A.nthr = (int32_t)n;
    A.d_out = d_out;
    A.g_out = g_out;
    const unsigned grid = (unsigned)((n + kB - 1) / kB);
    if (mask == 0) {   // empty scene: the empty sum
        A.Q = G;   // unused by the brute kernel when every class is empty
        hipLaunchKernelGGL(k_brute<true>, dim3(grid), dim3(kB), 0, s, A, (int64_t)0, (int64_t)0, (int64_t)0);
        SD_HIP(hipGetLastError());
        return SD_OK;
    }
    uint32_t *perm = nullptr;
    float *cen = nullptr;
    AsyncScratch tmp(s);
    if (!(p->flags & SD_NO_QUERY_SORT) && n >= 4096) {
        SD_TRY(tmp.alloc(&cen, n * 3));
        SD_TRY(tmp.alloc(&perm, n));
        hipLaunchKernelGGL(k_centroids, dim3(grid), dim3(kB), 0, s, G, nv, n, cen);
        SD_TRY(query_order(sc, cen, n, perm, s));
        A.perm = perm;
    }
    if (nv == 2) launch_evalq<2>(A, G, mask, s);
    else launch_evalq<3>(A, G, mask, s);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

int trace_dispatch(const sd_scene *sc, const float *O, const float *U, int64_t n, const sd_params *p,
                   float level, float eps, float t_max, int32_t max_steps, float *t_out, int32_t *steps_out,
                   hipStream_t s) {
    if (n == 0) return SD_OK;
    if (n > (int64_t)0x7fffffff - kB) return fail(SD_EUNSUPPORTED, "more than 2^31 rays per call");
    if (p->flags & SD_LSE_COMPENSATED_F32)
        return fail(SD_EUNSUPPORTED, "SD_LSE_COMPENSATED_F32 is compiled for the point-query traversal only");
    EvalArgs A;
    const int mask = make_args(sc, p, A) & 7;   // value only, no subtree skipping
    A.nq = (int32_t)n;
    A.nthr = (int32_t)n;
    const unsigned grid = (unsigned)((n + kB - 1) / kB);
    if (mask == 0) {   // empty scene: d = +inf everywhere, every ray misses
        hipLaunchKernelGGL(k_fill_f32, dim3(grid), dim3(kB), 0, s, t_out, n, INFINITY);
        if (steps_out) SD_HIP(hipMemsetAsync(steps_out, 0, n * sizeof(int32_t), s));
        SD_HIP(hipGetLastError());
        return SD_OK;
    }
    TraceArgs R{O, U, level, eps, t_max, max_steps, t_out, steps_out};
    launch_trace(A, R, mask, s);
    SD_HIP(hipGetLastError());
    return SD_OK;
}

}  // namespace sd
