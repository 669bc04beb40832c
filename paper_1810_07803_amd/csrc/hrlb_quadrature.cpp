// hrlb_quadrature.cpp -- velocity sets of the mixed quadrature (Sec. III) in extended precision.
//
// Half-range Gauss-Hermite rule for omega(z) = exp(-z^2/2)/sqrt(2 pi) on [0, inf): the three-term
// recurrence of its orthogonal polynomials is obtained by the discretized Stieltjes procedure
// (Gautschi, "Orthogonal Polynomials: Computation and Approximation", 2004, Sec. 2.2.3) on a
// composite Gauss-Legendre discretisation of omega, in long double; nodes are the eigenvalues of
// the Jacobi matrix (Sturm-sequence bisection), weights the Christoffel numbers.  The full-range
// rule uses the known recurrence of the probabilists' Hermite polynomials (alpha = 0, beta_k = k).
#include "hrlb_quadrature.h"

#include <cfloat>
#include <cmath>
#include <vector>

namespace hrlb {

static const long double kPiL = 3.141592653589793238462643383279502884L;

// n-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n
static void gauss_legendre(int n, std::vector<long double>& x, std::vector<long double>& w)
{
    x.assign(n, 0.0L);
    w.assign(n, 0.0L);
    for (int i = 0; i < n; ++i) {
        long double z = cosl(kPiL * (i + 0.75L) / (n + 0.5L));
        long double dp = 1.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-21L) break;
        }
        long double p0 = 1.0L, p1 = z;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0L);
        x[i] = z;
        w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

Recurrence half_range_recurrence(int n)
{
    // discretise int_0^40 f(z) omega(z) dz with 160 panels x 32 Gauss-Legendre points
    const int panels = 160, per = 32;
    const long double zmax = 40.0L, h = zmax / panels;
    std::vector<long double> gx, gw;
    gauss_legendre(per, gx, gw);
    std::vector<long double> Z, W;
    Z.reserve(panels * per);
    W.reserve(panels * per);
    const long double norm = 1.0L / sqrtl(2.0L * kPiL);
    for (int p = 0; p < panels; ++p) {
        const long double a = p * h;
        for (int k = 0; k < per; ++k) {
            const long double z = a + 0.5L * h * (gx[k] + 1.0L);
            Z.push_back(z);
            W.push_back(0.5L * h * gw[k] * norm * expl(-0.5L * z * z));
        }
    }
    const size_t M = Z.size();
    Recurrence r;
    r.alpha.assign(n, 0.0L);
    r.beta.assign(n, 0.0L);
    std::vector<long double> qprev(M, 0.0L), q(M), nxt(M);
    long double mass = 0.0L;
    for (size_t m = 0; m < M; ++m) mass += W[m];
    r.beta[0] = mass;
    const long double q0 = 1.0L / sqrtl(mass);
    for (size_t m = 0; m < M; ++m) q[m] = q0;
    long double sb_prev = 0.0L;  // sqrt(beta_k)
    for (int k = 0; k < n; ++k) {
        long double a = 0.0L;
        for (size_t m = 0; m < M; ++m) a += W[m] * Z[m] * q[m] * q[m];
        r.alpha[k] = a;
        if (k + 1 == n) break;
        long double b = 0.0L;
        for (size_t m = 0; m < M; ++m) {
            nxt[m] = (Z[m] - a) * q[m] - sb_prev * qprev[m];
            b += W[m] * nxt[m] * nxt[m];
        }
        r.beta[k + 1] = b;
        const long double sb = sqrtl(b);
        for (size_t m = 0; m < M; ++m) {
            qprev[m] = q[m];
            q[m] = nxt[m] / sb;
        }
        sb_prev = sb;
    }
    return r;
}

Recurrence hermite_recurrence(int n)
{
    Recurrence r;
    r.alpha.assign(n, 0.0L);
    r.beta.assign(n, 0.0L);
    r.beta[0] = 1.0L;
    for (int k = 1; k < n; ++k) r.beta[k] = (long double)k;
    return r;
}

// orthonormal polynomial values q_0..q_L at z (orthonormal w.r.t. the measure of mass beta_0)
void orthonormal_values(const Recurrence& r, int L, long double z, long double* out)
{
    long double prev = 0.0L, cur = 1.0L / sqrtl(r.beta[0]);
    out[0] = cur;
    for (int k = 0; k < L; ++k) {
        const long double sb_next = sqrtl(r.beta[k + 1]);
        const long double sb = k > 0 ? sqrtl(r.beta[k]) : 0.0L;
        const long double nx = ((z - r.alpha[k]) * cur - sb * prev) / sb_next;
        prev = cur;
        cur = nx;
        out[k + 1] = cur;
    }
}

// number of eigenvalues of the n x n Jacobi matrix below x (Sturm count of LDL^T pivots)
static int sturm_count(const Recurrence& r, int n, long double x)
{
    int cnt = 0;
    long double d = r.alpha[0] - x;
    if (d < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
        if (d == 0.0L) d = LDBL_MIN;
        d = (r.alpha[k] - x) - r.beta[k] / d;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// Gauss rule with n nodes (ascending) and Christoffel weights (summing to beta_0)
void gauss_from_recurrence(const Recurrence& r, int n, std::vector<long double>& nodes,
                           std::vector<long double>& weights)
{
    long double lo = 1e300L, hi = -1e300L;
    for (int k = 0; k < n; ++k) {
        const long double off = (k > 0 ? sqrtl(r.beta[k]) : 0.0L) + (k + 1 < n ? sqrtl(r.beta[k + 1]) : 0.0L);
        lo = fminl(lo, r.alpha[k] - off);
        hi = fmaxl(hi, r.alpha[k] + off);
    }
    nodes.assign(n, 0.0L);
    weights.assign(n, 0.0L);
    std::vector<long double> qv(n);
    for (int i = 0; i < n; ++i) {
        long double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const long double m = 0.5L * (a + b);
            if (m == a || m == b) break;
            if (sturm_count(r, n, m) > i)
                b = m;
            else
                a = m;
        }
        const long double z = 0.5L * (a + b);
        nodes[i] = z;
        orthonormal_values(r, n - 1, z, qv.data());
        long double s = 0.0L;
        for (int l = 0; l < n; ++l) s += qv[l] * qv[l];
        weights[i] = 1.0L / s;
    }
}

}  // namespace hrlb
