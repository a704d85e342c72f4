// Host tables of the monomial-moment variant (Sec. 2.6).
//
// xi_nu(n) is minus the coefficient of m^nu in the DDLOP of a regular row,
//   P'_l(n - m, 2n) = c_n sum_{j=1}^{l} l(l, j) j (n - 1 - m)^(j-1 falling) / (2n - 1)^(j falling),
//   c_n = 2 / (1 + P_l(-1, 2n - 1)),
// the backward difference of the falling-factorial DLOP of Sec. 2.3 with
// l(l, j) = (-1)^j C(l, j) C(l + j, j).  The alternating terms cancel by many
// orders of magnitude, so the expansion runs in binary128 and is rounded to
// FP64 once.  alpha_n = 1 / |(I - L)_n| (Sec. 2.4) comes from FP64 DLOP values:
// (I - L)_n = c_n (w_m nabla P_l(n - m, 2n - 1) for m < n; 1 at m = n).
#include <cmath>
#include <vector>

#include "monomial.h"
#include "plan_host.h"

namespace dsbt {

namespace {

typedef __float128 quad;

// 1 + P_l(-1, M): the terms C(l, j) C(l + j, j) j! / M^(j falling) are positive
quad one_plus_dlop_at_minus_one(int ell, int M) {
    quad t = 1, sum = 2;   // j = 0 term of P plus the 1
    for (int j = 1; j <= ell; ++j) {
        t = t * (quad)(ell - j + 1) * (quad)(ell + j) / ((quad)j * (quad)(M - j + 1));
        sum += t;
    }
    return sum;
}

}  // namespace

void monomial_tables(int N, int ell, std::vector<double>& xi, std::vector<double>& alpha,
                     std::vector<double>& comp) {
    const int p = parity_p(ell), n0 = n0_of(ell), k = n_extra(ell);
    const int Nl = N + p - 1;
    const int nu0 = (ell + 1) % 2;
    const int rows = Nl - n0 + 1;
    xi.assign((size_t)rows * k, 0.0);
    alpha.assign(rows, 0.0);
    comp.assign((size_t)k * N, 0.0);
    std::vector<quad> prod(ell + 1), acc(ell + 1);
    std::vector<double> P(N + 2);
    for (int n = n0; n <= Nl; ++n) {
        const int M = 2 * n - 1;
        const quad c = (quad)2 / one_plus_dlop_at_minus_one(ell, M);
        // acc = sum_j u_j j (n - 1 - m)^(j-1 falling), u_j = l(l, j) / M^(j falling)
        for (int t = 0; t <= ell; ++t) acc[t] = prod[t] = 0;
        prod[0] = 1;
        int deg = 0;
        quad u = 1;
        for (int j = 1; j <= ell; ++j) {
            u = u * (quad)(-(ell - j + 1)) * (quad)(ell + j) / ((quad)j * (quad)j * (quad)(M - j + 1));
            if (j >= 2) {   // times (a - m), a = n - j + 1
                const quad a = (quad)(n - j + 1);
                for (int t = deg + 1; t >= 1; --t) prod[t] = a * prod[t] - prod[t - 1];
                prod[0] = a * prod[0];
                ++deg;
            }
            const quad w = u * (quad)j;
            for (int t = 0; t <= deg; ++t) acc[t] += w * prod[t];
        }
        for (int q = 0; q < k; ++q) xi[(size_t)(n - n0) * k + q] = (double)(-c * acc[nu0 + 2 * q]);
        // alpha_n from P_l(x, 2n - 1), x = 0..n
        dlop_values(ell, M, n, P.data());
        double ss = 1.0;
        for (int m = p; m < n; ++m) {
            const double d = P[n - m] - P[n - m - 1];
            ss += (m == 0 ? 0.5 : 1.0) * d * d;
        }
        alpha[n - n0] = 1.0 / ((double)c * std::sqrt(ss));
    }
    // completion rows n = p + q: w_m P_{2n-p}(Nl - m, 2 Nl), normalised (eq. Tadd)
    for (int q = 0; q < k; ++q) {
        const int n = p + q;
        dlop_values(2 * n - p, 2 * Nl, Nl - p, P.data());
        double ss = 0.0;
        for (int j = 0; j < N; ++j) {
            const int m = j + p;
            const double v = (m == 0 ? std::sqrt(0.5) : 1.0) * P[Nl - m];
            comp[(size_t)q * N + j] = v;
            ss += v * v;
        }
        const double inv = 1.0 / std::sqrt(ss);
        for (int j = 0; j < N; ++j) comp[(size_t)q * N + j] *= inv;
    }
}

}  // namespace dsbt
