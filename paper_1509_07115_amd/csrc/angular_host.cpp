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

// P[q] = the associated Legendre functions Pbar_{|m|+t}^m(eta_j) sqrt(w_j),
// t < n_theta, orthonormalised in t on the quadrature.  Pbar_l^m is
// (1 - eta^2)^{|m|/2} times a polynomial of degree l - |m| (leading coefficient
// of sign (-1)^m for m > 0, + for m <= 0: Condon-Shortley phase), so the rows
// are sqrt(W_j) times the orthonormal polynomials of the discrete weights
// W_j = w_j (1 - eta_j^2)^|m|.  They are built by the Lanczos recurrence on the
// weighted nodes (multiply by eta, remove the projections on the earlier rows
// twice, normalise): for large |m| the sampled functions themselves are nearly
// dependent and Gram-Schmidt on them loses digits, this form does not.
void sht_p_tables(int n_theta, int n_phi, std::vector<double>& P) {
    std::vector<double> eta, w;
    gauss_legendre(n_theta, eta, w);
    const int M = (n_phi - 1) / 2;
    P.assign((size_t)n_phi * n_theta * n_theta, 0.0);
    std::vector<double> v(n_theta);
    for (int q = 0; q < n_phi; ++q) {
        const int m = q - M, am = m < 0 ? -m : m;
        double* U = P.data() + (size_t)q * n_theta * n_theta;   // U[t][j]
        double nn = 0.0;
        for (int j = 0; j < n_theta; ++j) {
            U[j] = std::sqrt(w[j]) * std::pow(std::sqrt(std::fmax(0.0, 1.0 - eta[j] * eta[j])), am);
            nn += U[j] * U[j];
        }
        for (int j = 0; j < n_theta; ++j) U[j] /= std::sqrt(nn);
        for (int t = 1; t < n_theta; ++t) {
            for (int j = 0; j < n_theta; ++j) v[j] = eta[j] * U[(size_t)(t - 1) * n_theta + j];
            for (int pass = 0; pass < 2; ++pass)
                for (int u = 0; u < t; ++u) {
                    const double* ru = U + (size_t)u * n_theta;
                    double d = 0.0;
                    for (int j = 0; j < n_theta; ++j) d += ru[j] * v[j];
                    for (int j = 0; j < n_theta; ++j) v[j] -= d * ru[j];
                }
            double s2 = 0.0;
            for (int j = 0; j < n_theta; ++j) s2 += v[j] * v[j];
            const double inv = 1.0 / std::sqrt(s2);
            for (int j = 0; j < n_theta; ++j) U[(size_t)t * n_theta + j] = v[j] * inv;
        }
        if (m > 0 && (m & 1))
            for (size_t e = 0; e < (size_t)n_theta * n_theta; ++e) U[e] = -U[e];
    }
}

}  // namespace dsbt
