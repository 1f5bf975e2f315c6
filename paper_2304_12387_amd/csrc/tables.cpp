// 1D tables of the interpolation-histopolation basis (Section 2.1) and of the
// Gauss-Legendre change of basis used by the local CG (Section 2.5).
//
// Built on the host once per degree.  Construction here is independent of any
// other implementation: Gauss points by Newton iteration on Legendre
// polynomials (three-term recurrence), histopolation functions through the
// identity h_j = sum_{i>j} l_i' (whose sub-interval integrals telescope to
// delta_jk), and the inverse of the p x p change-of-basis matrix by
// Gauss-Jordan elimination with partial pivoting.
#include "hd_internal.hpp"

#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

namespace hd {

namespace {

// Legendre P_n(x) and P_n'(x) on [-1, 1] by the three-term recurrence.
void legendre(int n, double x, double& P, double& dP) {
    double p0 = 1.0, p1 = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    P = p1;
    // (x^2 - 1) P_n' = n (x P_n - P_{n-1})
    dP = n * (x * p1 - p0) / (x * x - 1.0);
}

}  // namespace

void gauss_legendre01(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, t, P, dP);
            double dt = P / dP;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double P, dP;
        legendre(n, t, P, dP);
        // descending t -> ascending x
        x[n - 1 - i] = 0.5 * (t + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dP * dP);  // (2 / (...)) / 2
    }
}

void gauss_lobatto01(int p, double* xi) {
    xi[0] = 0.0;
    xi[p] = 1.0;
    // interior points: roots of P_p' ; Newton with P_p'' from Legendre's ODE
    for (int i = 1; i < p; ++i) {
        double t = -std::cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(p, t, P, dP);
            double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
            double dt = dP / d2P;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        xi[i] = 0.5 * (t + 1.0);
    }
}

static double lagrange_val(const double* nodes, int n, int i, double x) {
    double v = 1.0;
    for (int m = 0; m < n; ++m)
        if (m != i) v *= (x - nodes[m]) / (nodes[i] - nodes[m]);
    return v;
}

static double lagrange_der(const double* nodes, int n, int i, double x) {
    double s = 0.0;
    for (int m = 0; m < n; ++m) {
        if (m == i) continue;
        double t = 1.0 / (nodes[i] - nodes[m]);
        for (int k = 0; k < n; ++k)
            if (k != i && k != m) t *= (x - nodes[k]) / (nodes[i] - nodes[k]);
        s += t;
    }
    return s;
}

// h_j(x) = sum_{i=j+1}^{p} l_i'(x) on the Gauss-Lobatto nodes
static double histo_val(const double* gll, int p, int j, double x) {
    double s = 0.0;
    for (int i = j + 1; i <= p; ++i) s += lagrange_der(gll, p + 1, i, x);
    return s;
}

static void invert(int n, const double* A, double* Ainv) {
    std::vector<double> a(A, A + n * n), b(n * n, 0.0);
    for (int i = 0; i < n; ++i) b[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[r * n + c]) > std::fabs(a[piv * n + c])) piv = r;
        if (a[piv * n + c] == 0.0) throw std::runtime_error("singular change-of-basis matrix");
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[c * n + k], a[piv * n + k]);
                std::swap(b[c * n + k], b[piv * n + k]);
            }
        double d = 1.0 / a[c * n + c];
        for (int k = 0; k < n; ++k) { a[c * n + k] *= d; b[c * n + k] *= d; }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            double f = a[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) { a[r * n + k] -= f * a[c * n + k]; b[r * n + k] -= f * b[c * n + k]; }
        }
    }
    std::memcpy(Ainv, b.data(), sizeof(double) * n * n);
}

template <typename T>
static void fill(int p, Tables<T>& t) {
    std::memset(&t, 0, sizeof(t));
    const int q = p + 1;
    double gll[HD_MAXP + 1], xq[HD_MAXQ], wq[HD_MAXQ], g[HD_MAXP], gw[HD_MAXP];
    gauss_lobatto01(p, gll);
    gauss_legendre01(q, xq, wq);
    gauss_legendre01(p, g, gw);
    for (int i = 0; i <= p; ++i) t.gll[i] = (T)gll[i];
    for (int a = 0; a < q; ++a) {
        t.wq[a] = (T)wq[a];
        t.xq[a] = (T)xq[a];
        for (int i = 0; i <= p; ++i) t.L[a][i] = (T)lagrange_val(gll, p + 1, i, xq[a]);
        for (int j = 0; j < p; ++j) {
            double h = histo_val(gll, p, j, xq[a]);
            t.H[a][j] = (T)h;
            t.H2[a][j] = (T)(h * h);
        }
        for (int i = 0; i <= p; ++i) {
            double l = lagrange_val(gll, p + 1, i, xq[a]);
            t.L2[a][i] = (T)(l * l);
        }
        for (int m = 0; m < p; ++m) {
            double b = lagrange_val(g, p, m, xq[a]);
            t.Bg[a][m] = (T)b;
            t.Bg2[a][m] = (T)(b * b);
        }
    }
    // change of basis: IH coefficients c -> values at the p Gauss-Legendre
    // nodes v = Tm c with Tm[m][j] = h_j(g_m); store Tm^{-1}
    double Tm[HD_MAXP * HD_MAXP], Ti[HD_MAXP * HD_MAXP];
    for (int m = 0; m < p; ++m)
        for (int j = 0; j < p; ++j) Tm[m * p + j] = histo_val(gll, p, j, g[m]);
    invert(p, Tm, Ti);
    for (int r = 0; r < p; ++r)
        for (int c = 0; c < p; ++c) t.Tinv[r][c] = (T)Ti[r * p + c];
}

void build_tables(int p, Tables<double>& t64, Tables<float>& t32) {
    fill<double>(p, t64);
    fill<float>(p, t32);
}

}  // namespace hd

extern "C" int hd_host_tables(int p, double* gll, double* gl_x, double* gl_w) {
    if (p < 1 || p > HD_MAXP) return HD_ERR_ARG;
    if (gll) hd::gauss_lobatto01(p, gll);
    if (gl_x && gl_w) hd::gauss_legendre01(p + 1, gl_x, gl_w);
    return HD_OK;
}
