// Host FP64 construction of the triangle weight polynomials (App. C.3).
//
// The weight w~(phi1, phi2) is a degree-7 polynomial (36 monomial
// coefficients) fixed by 10 point values and by zero normal derivatives on the
// three sides of the barycentric triangle.  The system is consistent but rank
// deficient, and the paper takes the pseudoinverse (minimum-norm) solution.
// Because the right-hand side is linear in the three constraint values
// (1/v at the vertices, 1/e at the edge points, (v-1)/v at the centre), so is
// the minimum-norm solution:
//     w~ = (1/v) B_V + (1/e) B_E + ((v-1)/v) B_C,
// with three universal bases computed once here by a one-sided Jacobi SVD.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "sd_internal.h"

namespace sd {
namespace {

constexpr int kRows = 10 + 4 * 7;
constexpr int kCols = 36;

struct Mono {
    int a, b;
};

std::vector<Mono> monomials() {
    std::vector<Mono> m;
    for (int a = 0; a <= 7; ++a)
        for (int b = 0; a + b <= 7; ++b) m.push_back({a, b});
    return m;
}

double binom(int n, int k) {
    double r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// coefficient of t^k in t^p (1 - t)^q
double tp_1mt_q(int p, int q, int k) {
    int j = k - p;
    if (j < 0 || j > q) return 0.0;
    return binom(q, j) * ((j & 1) ? -1.0 : 1.0);
}

void build_system(double M[kRows][kCols]) {
    auto mono = monomials();
    memset(M, 0, sizeof(double) * kRows * kCols);
    const double pts[10][2] = {{0, 0}, {1, 0}, {0, 1},
                               {1.0 / 3, 0}, {2.0 / 3, 0}, {1.0 / 3, 2.0 / 3},
                               {2.0 / 3, 1.0 / 3}, {0, 1.0 / 3}, {0, 2.0 / 3},
                               {1.0 / 3, 1.0 / 3}};
    for (int r = 0; r < 10; ++r)
        for (int j = 0; j < kCols; ++j)
            M[r][j] = pow(pts[r][0], mono[j].a) * pow(pts[r][1], mono[j].b);
    for (int j = 0; j < kCols; ++j) {
        int a = mono[j].a, b = mono[j].b;
        for (int k = 0; k < 7; ++k) {
            // d/dphi1 on phi1 = 0 (phi2 = t): only a == 1 survives, giving t^b
            M[10 + k][j] = (a == 1 && b == k) ? 1.0 : 0.0;
            // d/dphi2 on phi2 = 0 (phi1 = t): only b == 1 survives, giving t^a
            M[17 + k][j] = (b == 1 && a == k) ? 1.0 : 0.0;
            // (d/dphi1 + d/dphi2) on (t, 1 - t) and on (1 - t, t)
            double s1 = 0, s2 = 0;
            if (a > 0) {
                s1 += a * tp_1mt_q(a - 1, b, k);   // x^(a-1) y^b, x = t, y = 1 - t
                s2 += a * tp_1mt_q(b, a - 1, k);   // x = 1 - t, y = t
            }
            if (b > 0) {
                s1 += b * tp_1mt_q(a, b - 1, k);
                s2 += b * tp_1mt_q(b - 1, a, k);
            }
            M[24 + k][j] = s1;
            M[31 + k][j] = s2;
        }
    }
}

// Minimum-norm solutions x_i of M x = r_i via one-sided Jacobi SVD of M.
void pinv_solve(double M[kRows][kCols], const double R[3][kRows], double X[3][kCols]) {
    static double A[kRows][kCols], V[kCols][kCols];
    memcpy(A, M, sizeof(A));
    for (int i = 0; i < kCols; ++i)
        for (int j = 0; j < kCols; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int p = 0; p < kCols; ++p)
            for (int q = p + 1; q < kCols; ++q) {
                double app = 0, aqq = 0, apq = 0;
                for (int i = 0; i < kRows; ++i) {
                    app += A[i][p] * A[i][p];
                    aqq += A[i][q] * A[i][q];
                    apq += A[i][p] * A[i][q];
                }
                if (apq == 0.0) continue;
                double rel = fabs(apq) / sqrt(app * aqq + 1e-300);
                off = std::max(off, rel);
                if (rel < 1e-15) continue;
                double zeta = (aqq - app) / (2 * apq);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1 + zeta * zeta));
                double c = 1 / sqrt(1 + t * t), s = c * t;
                for (int i = 0; i < kRows; ++i) {
                    double x = A[i][p], y = A[i][q];
                    A[i][p] = c * x - s * y;
                    A[i][q] = s * x + c * y;
                }
                for (int i = 0; i < kCols; ++i) {
                    double x = V[i][p], y = V[i][q];
                    V[i][p] = c * x - s * y;
                    V[i][q] = s * x + c * y;
                }
            }
        if (off < 1e-15) break;
    }
    double sig[kCols], smax = 0;
    for (int j = 0; j < kCols; ++j) {
        double s = 0;
        for (int i = 0; i < kRows; ++i) s += A[i][j] * A[i][j];
        sig[j] = sqrt(s);
        smax = std::max(smax, sig[j]);
    }
    for (int k = 0; k < 3; ++k) {
        for (int j = 0; j < kCols; ++j) X[k][j] = 0;
        for (int j = 0; j < kCols; ++j) {
            if (sig[j] <= 1e-10 * smax) continue;
            double ur = 0;   // u_j . r with u_j = A_j / sigma_j
            for (int i = 0; i < kRows; ++i) ur += A[i][j] * R[k][i];
            ur /= sig[j] * sig[j];
            for (int i = 0; i < kCols; ++i) X[k][i] += ur * V[i][j];
        }
    }
}

double g_basis[3][64];
bool g_ready = false;

void ensure_basis() {
    if (g_ready) return;
    static double M[kRows][kCols];
    build_system(M);
    double R[3][kRows];
    memset(R, 0, sizeof(R));
    for (int i = 0; i < 3; ++i) R[0][i] = 1.0;        // vertex points
    for (int i = 3; i < 9; ++i) R[1][i] = 1.0;        // edge points
    R[2][9] = 1.0;                                     // centre
    double X[3][kCols];
    pinv_solve(M, R, X);
    auto mono = monomials();
    memset(g_basis, 0, sizeof(g_basis));
    for (int k = 0; k < 3; ++k)
        for (int j = 0; j < kCols; ++j) g_basis[k][mono[j].a * 8 + mono[j].b] = X[k][j];
    g_ready = true;
}

double eval_w(int v, int e, double x, double y) {
    double cv = 1.0 / v, ce = 1.0 / e, cc = (v - 1.0) / v;
    double px[8], py[8];
    px[0] = py[0] = 1;
    for (int i = 1; i < 8; ++i) { px[i] = px[i - 1] * x; py[i] = py[i - 1] * y; }
    double w = 0;
    for (int a = 0; a <= 7; ++a)
        for (int b = 0; a + b <= 7; ++b) {
            int k = a * 8 + b;
            double c = cv * g_basis[0][k] + ce * g_basis[1][k] + cc * g_basis[2][k];
            w += c * px[a] * py[b];
        }
    return w;
}

}  // namespace

int triangle_basis_f64(double out[3][64]) {
    ensure_basis();
    memcpy(out, g_basis, sizeof(g_basis));
    return SD_OK;
}

// Bernstein-Bezier coefficients b_ijk (i + j + k = 7, i on lambda0 = 1 - phi1
// - phi2, j on phi1, k on phi2) of w~ for valences (v, e), in the compact
// order idx(j, k) = 8 j - j (j - 1) / 2 + k.  On the triangle the Bernstein
// basis is non-negative and sums to one, so evaluating in this form keeps FP32
// rounding near a few ulps (the monomial form cancels by up to ~500x).
// From lambda1^a lambda2^b (lambda0 + lambda1 + lambda2)^(7-a-b):
//   b_ijk = sum_{a<=j, b<=k} c_ab (7-a-b)! j! k! / (7! (j-a)! (k-b)!).
void triangle_bernstein(int v, int e, float out[36]) {
    ensure_basis();
    if (v <= 1) {
        for (int t = 0; t < 36; ++t) out[t] = 1.f;   // w~ = 1
        return;
    }
    double fact[8] = {1, 1, 2, 6, 24, 120, 720, 5040};
    double cv = 1.0 / v, ce = 1.0 / e, cc = (v - 1.0) / v;
    int t = 0;
    for (int j = 0; j <= 7; ++j)
        for (int k = 0; j + k <= 7; ++k) {
            double s = 0;
            for (int a = 0; a <= j; ++a)
                for (int b = 0; b <= k; ++b) {
                    int m = a * 8 + b;
                    double c = cv * g_basis[0][m] + ce * g_basis[1][m] + cc * g_basis[2][m];
                    s += c * fact[7 - a - b] * fact[j] * fact[k] /
                         (fact[7] * fact[j - a] * fact[k - b]);
                }
            out[t++] = (float)s;
        }
}

// Monomial coefficients c_ab of w~ for valences (v, e) in the order the
// device evaluates them (Horner in phi1 outside, in phi2 inside): a = 7 down to
// 0, and for each a, b = 7 - a down to 0.  FP64 throughout; w~ = 1 for v <= 1.
void triangle_monomial_horner(int v, int e, double out[36]) {
    ensure_basis();
    int t = 0;
    for (int a = 7; a >= 0; --a)
        for (int b = 7 - a; b >= 0; --b) {
            const int k = a * 8 + b;
            out[t++] = v <= 1 ? (k == 0 ? 1.0 : 0.0)
                              : (1.0 / v) * g_basis[0][k] + (1.0 / e) * g_basis[1][k] +
                                    ((v - 1.0) / v) * g_basis[2][k];
        }
}

// Minimum of w~ over {phi1, phi2 >= 0, phi1 + phi2 <= 1}: grid, then a compass
// search kept inside the simplex from the best grid points.
double triangle_weight_min_f64(int v, int e) {
    ensure_basis();
    if (v <= 1) return 1.0;
    // coefficients of w~ for (v, e), formed once; Horner in y inside Horner in x
    double c[8][8] = {};
    {
        const double cv = 1.0 / v, ce = 1.0 / e, cc = (v - 1.0) / v;
        for (int a = 0; a <= 7; ++a)
            for (int b = 0; a + b <= 7; ++b) {
                const int k = a * 8 + b;
                c[a][b] = cv * g_basis[0][k] + ce * g_basis[1][k] + cc * g_basis[2][k];
            }
    }
    auto eval_w = [&c](int, int, double x, double y) {
        double w = 0;
        for (int a = 7; a >= 0; --a) {
            double r = 0;
            for (int b = 7 - a; b >= 0; --b) r = r * y + c[a][b];
            w = w * x + r;
        }
        return w;
    };
    const int n = 256;
    struct Cand { double w, x, y; };
    std::vector<Cand> best;
    best.reserve((n + 1) * (n + 2) / 2);
    for (int i = 0; i <= n; ++i)
        for (int j = 0; i + j <= n; ++j) {
            double x = double(i) / n, y = double(j) / n;
            best.push_back({eval_w(v, e, x, y), x, y});
        }
    std::partial_sort(best.begin(), best.begin() + 12, best.end(),
                      [](const Cand &a, const Cand &b) { return a.w < b.w; });
    double m = best[0].w;
    auto feasible = [](double x, double y) { return x >= 0 && y >= 0 && x + y <= 1; };
    const double dirs[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, -1}, {-1, 1}, {1, 1}, {-1, -1}};
    for (int c = 0; c < 12; ++c) {
        double x = best[c].x, y = best[c].y, w = best[c].w, h = 1.0 / n;
        while (h > 1e-13) {
            bool moved = false;
            for (auto &d : dirs) {
                double nx = x + h * d[0], ny = y + h * d[1];
                if (!feasible(nx, ny)) {
                    // slide onto the boundary along this direction
                    nx = std::max(nx, 0.0); ny = std::max(ny, 0.0);
                    double s = nx + ny;
                    if (s > 1) { nx /= s; ny /= s; }
                }
                double nw = eval_w(v, e, nx, ny);
                if (nw < w) { x = nx; y = ny; w = nw; moved = true; }
            }
            if (!moved) h *= 0.5;
        }
        m = std::min(m, w);
    }
    return m;
}

}  // namespace sd

extern "C" int sd_triangle_weight_basis(double *coef_host) {
    if (!coef_host) return sd::fail(SD_EINVAL, "sd_triangle_weight_basis: null output");
    double b[3][64];
    sd::triangle_basis_f64(b);
    memcpy(coef_host, b, sizeof(b));
    return SD_OK;
}
