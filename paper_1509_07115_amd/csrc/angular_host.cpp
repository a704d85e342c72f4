// Host FP64 tables of the angular transform (Sec. 4.1): Gauss-Legendre
// quadrature and the associated Legendre blocks orthonormalised on it.
#include <cmath>
#include <vector>

#include "angular.h"

namespace dsbt {

void gauss_legendre(int n, std::vector<double>& eta, std::vector<double>& w) {
    const double pi = 3.14159265358979323846;
    eta.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        // i-th largest root of P_n: Newton from the asymptotic guess
        double x = std::cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;   // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double pn = n == 0 ? 1.0 : (n == 1 ? x : p1);
            const double pm = n == 1 ? 1.0 : p0;   // P_{n-1}
            dp = n * (x * pn - pm) / (x * x - 1.0);
            const double dx = pn / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        eta[n - 1 - i] = x;   // ascending
        w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

// Pbar_l^m(x) for l = m .. m + count - 1 (m >= 0), unit L2 norm on [-1, 1],
// Condon-Shortley phase, by the recurrences in l for fixed m.
static void assoc_legendre(int m, int count, double x, double* out) {
    const double s = std::sqrt(std::fmax(0.0, 1.0 - x * x));
    double pmm = std::sqrt(0.5);   // Pbar_0^0
    for (int k = 1; k <= m; ++k) pmm *= -std::sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
    out[0] = pmm;
    if (count == 1) return;
    double pm1 = std::sqrt(2.0 * m + 3.0) * x * pmm;   // Pbar_{m+1}^m
    out[1] = pm1;
    double a2 = pmm, a1 = pm1;
    for (int l = m + 2; l < m + count; ++l) {
        const double al = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        const double bl = std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
        const double v = al * (x * a1 - bl * a2);
        out[l - m] = v;
        a2 = a1;
        a1 = v;
    }
}

void sht_p_tables(int n_theta, int n_phi, std::vector<double>& P) {
    std::vector<double> eta, w;
    gauss_legendre(n_theta, eta, w);
    const int M = (n_phi - 1) / 2;
    P.assign((size_t)n_phi * n_theta * n_theta, 0.0);
    std::vector<double> col(n_theta);
    for (int q = 0; q < n_phi; ++q) {
        const int m = q - M, am = m < 0 ? -m : m;
        const double sgn = (m < 0 && (am & 1)) ? -1.0 : 1.0;   // Pbar_l^{-m} = (-1)^m Pbar_l^m
        double* B = P.data() + (size_t)q * n_theta * n_theta;   // B[t][j]
        for (int j = 0; j < n_theta; ++j) {
            assoc_legendre(am, n_theta, eta[j], col.data());
            const double sw = std::sqrt(w[j]);
            for (int t = 0; t < n_theta; ++t) B[(size_t)t * n_theta + j] = sgn * col[t] * sw;
        }
        // modified Gram-Schmidt over the rows t, in order
        for (int t = 0; t < n_theta; ++t) {
            double* rt = B + (size_t)t * n_theta;
            for (int u = 0; u < t; ++u) {
                const double* ru = B + (size_t)u * n_theta;
                double d = 0.0;
                for (int j = 0; j < n_theta; ++j) d += ru[j] * rt[j];
                for (int j = 0; j < n_theta; ++j) rt[j] -= d * ru[j];
            }
            double nn = 0.0;
            for (int j = 0; j < n_theta; ++j) nn += rt[j] * rt[j];
            const double inv = 1.0 / std::sqrt(nn);
            for (int j = 0; j < n_theta; ++j) rt[j] *= inv;
        }
    }
}

}  // namespace dsbt
