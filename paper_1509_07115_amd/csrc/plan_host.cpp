// Host FP64 plan generation for the orthogonal DSBT.  See plan_host.h for the
// tiled moment form; the formulas cited here are those of Sec. 2.3-2.5.
#include "plan_host.h"
#include <cstring>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace dsbt {

int parity_p(int ell) { return (ell % 2 == 0) ? 1 : 0; }
int n0_of(int ell) { return (ell + 2) / 2; }            // ceil((l+1)/2), Sec. 2.4
int n_extra(int ell) { return n0_of(ell) - parity_p(ell); }  // ceil(l/2), Sec. 2.5

// Degree recurrence of the DLOP at fixed x (an identity of the
// falling-factorial definition in Sec. 2.3):
//   (j+1)(M-j) P_{j+1} = (2j+1)(M-2x) P_j - j(M+j+1) P_{j-1},  P_0 = 1, P_1 = 1 - 2x/M.
// Fills out[j][x] for j = 0..dmax, x = 0..xmax.
static void dlop_degree_table(int dmax, int M, int xmax, double* out) {
    const int X = xmax + 1;
    for (int x = 0; x <= xmax; ++x) out[x] = 1.0;
    if (dmax == 0) return;
    for (int x = 0; x <= xmax; ++x) out[X + x] = 1.0 - 2.0 * x / M;
    for (int j = 1; j < dmax; ++j) {
        const double a = 2.0 * j + 1.0, c = j * (M + j + 1.0), den = (j + 1.0) * (M - j);
        const double* pm = out + (size_t)(j - 1) * X;
        const double* pc = out + (size_t)j * X;
        double* pn = out + (size_t)(j + 1) * X;
        for (int x = 0; x <= xmax; ++x) pn[x] = (a * (M - 2.0 * x) * pc[x] - c * pm[x]) / den;
    }
}

// Difference equation of the DLOP in x (Hahn form, alpha = beta = 0):
//   B(x) y(x+1) = [d(d+1) + B(x) + D(x)] y(x) - D(x) y(x-1),
//   B(x) = (x+1)(x-M), D(x) = x(x-M-1), y(0) = 1.
static void dlop_march(int d, int M, int xmax, double* y) {
    y[0] = 1.0;
    if (xmax >= 1) y[1] = 1.0 - d * (d + 1.0) / M;
    const double lam = d * (d + 1.0);
    for (int x = 1; x < xmax; ++x) {
        const double B = (x + 1.0) * (x - M), D = x * (x - M - 1.0);
        y[x + 1] = ((lam + B + D) * y[x] - D * y[x - 1]) / B;
    }
}

void dlop_values(int d, int M, int xmax, double* out) {
    if (d < 0 || d > M || xmax > M) throw std::invalid_argument("dlop_values: bad degree or range");
    if (M == 0) {
        for (int x = 0; x <= xmax; ++x) out[x] = 1.0;
        return;
    }
    if ((long long)d * d <= 2LL * M) {
        // degree recurrence, keeping only the last two degrees
        std::vector<double> a(xmax + 1, 1.0), b(xmax + 1), c(xmax + 1);
        if (d == 0) {
            std::copy(a.begin(), a.end(), out);
            return;
        }
        for (int x = 0; x <= xmax; ++x) b[x] = 1.0 - 2.0 * x / M;
        for (int j = 1; j < d; ++j) {
            const double aa = 2.0 * j + 1.0, cc = j * (M + j + 1.0), den = (j + 1.0) * (M - j);
            for (int x = 0; x <= xmax; ++x) c[x] = (aa * (M - 2.0 * x) * b[x] - cc * a[x]) / den;
            std::swap(a, b);
            std::swap(b, c);
        }
        std::copy(b.begin(), b.end(), out);
        return;
    }
    dlop_march(d, M, xmax, out);
}

void tile_basis(int ell, int t, double* out) {
    const int p = parity_p(ell), k = n_extra(ell);
    if (k == 0) return;
    const int M = 2 * t - 2, xmax = t - 1;   // DLOP grid 0..2t-2 centred at t-1
    const int dmax = 2 * (k - 1) + p;          // highest degree, <= l - 1
    if (dmax > M) throw std::invalid_argument("tile_basis: tile too small for the degree");
    // degrees handled by the recurrence: d^2 <= 2M
    int drec = 0;
    while ((long long)(drec + 1) * (drec + 1) <= 2LL * M && drec + 1 <= dmax) ++drec;
    std::vector<double> rec;
    if (M > 0) {
        rec.resize((size_t)(drec + 1) * (xmax + 1));
        dlop_degree_table(drec, M, xmax, rec.data());
    }
    std::vector<double> tmp(xmax + 1);
    for (int kk = 0; kk < k; ++kk) {
        const int d = 2 * kk + p;
        const double* P;
        if (M == 0) {
            tmp[0] = 1.0;
            P = tmp.data();
        } else if (d <= drec) {
            P = rec.data() + (size_t)d * (xmax + 1);
        } else {
            dlop_march(d, M, xmax, tmp.data());
            P = tmp.data();
        }
        // q(m) = (-1)^d P_d(t-1-m, M): the polynomial in m has parity (-1)^d
        const double sg = (d & 1) ? -1.0 : 1.0;
        double* q = out + (size_t)kk * t;
        double nrm = 0.0;
        for (int m = 0; m < t; ++m) {
            q[m] = sg * P[t - 1 - m];
            nrm += (m == 0 ? 0.5 : 1.0) * q[m] * q[m];
        }
        const double inv = 1.0 / std::sqrt(nrm);
        for (int m = 0; m < t; ++m) q[m] *= inv;
    }
}

int auto_tile(int ell, int N) {
    // B >= 32: the tile steps form a serial chain per channel, so fewer, wider
    // tiles (N/B steps) beat the smaller (B + k)^2 / B block cost of B = 16
    int B = 32;
    while (B < n0_of(ell)) B *= 2;
    return std::min(B, N);
}

// Regular row n of T divided by w_m (Sec. 2.4 eq. Tdef/Ldef): kappa(m) for
// m = 0..n, with kappa(n) the diagonal.  Up to a positive factor the row of
// I - L is v_nn = 1, v_nm = w_m [P_l(n-m, 2n-1) - P_l(n-m-1, 2n-1)]; alpha_n is
// the numerical norm of the weighted row over m = p..n.  kappa(0) is the kernel
// polynomial's value at m = 0 also for even l, where m = 0 is not a grid slot.
static void regular_row(int ell, int n, std::vector<double>& P, std::vector<double>& kap) {
    const int p = parity_p(ell);
    P.resize(n + 1);
    dlop_values(ell, 2 * n - 1, n, P.data());
    kap.resize(n + 1);
    for (int m = 0; m < n; ++m) kap[m] = P[n - m] - P[n - m - 1];
    kap[n] = 1.0;
    double nrm = 0.0;
    for (int m = p; m <= n; ++m) nrm += ((m == 0) ? 0.5 : 1.0) * kap[m] * kap[m];
    const double beta = 1.0 / std::sqrt(nrm);
    for (int m = 0; m <= n; ++m) kap[m] *= beta;
}

void build_ftb_blocks(int ell, int B, int NT, std::vector<double>& blocks, int nthreads) {
    const int p = parity_p(ell), k = n_extra(ell), n0 = n0_of(ell);
    const int R = B + k;
    if (B < n0) throw std::invalid_argument("tile smaller than the first regular row");
    blocks.assign((size_t)NT * R * R, 0.0);
    std::atomic<int> next(0);
    auto work = [&]() {
        std::vector<double> qA, qB, P, kap;
        for (;;) {
            const int J = next.fetch_add(1);
            if (J >= NT) break;
            double* Mj = blocks.data() + (size_t)J * R * R;
            const int t0 = p + J * B, t1 = t0 + B;
            if (k > 0) {
                qA.resize((size_t)k * t1);
                tile_basis(ell, t1, qA.data());
                if (J >= 1) {
                    qB.resize((size_t)k * t0);
                    tile_basis(ell, t0, qB.data());
                }
            }
            for (int s = 0; s < B; ++s) {
                const int n = t0 + s;
                if (n < n0) continue;   // completion rows come from the final moments
                regular_row(ell, n, P, kap);
                double* row = Mj + (size_t)s * R;
                for (int sp = 0; sp <= s; ++sp) row[sp] = kap[t0 + sp];
                if (J >= 1) {
                    for (int kk = 0; kk < k; ++kk) {
                        const double* q = qB.data() + (size_t)kk * t0;
                        double acc = 0.5 * kap[0] * q[0];
                        for (int m = 1; m < t0; ++m) acc += kap[m] * q[m];
                        row[B + kk] = acc;
                    }
                }
            }
            for (int a = 0; a < k; ++a) {
                double* row = Mj + (size_t)(B + a) * R;
                const double* qa = qA.data() + (size_t)a * t1;
                for (int s = 0; s < B; ++s) row[s] = qa[t0 + s];
                if (J >= 1) {
                    for (int c = 0; c < k; ++c) {
                        const double* qc = qB.data() + (size_t)c * t0;
                        double acc = 0.5 * qa[0] * qc[0];
                        for (int m = 1; m < t0; ++m) acc += qa[m] * qc[m];
                        row[B + c] = acc;
                    }
                }
            }
        }
    };
    int nt = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::min(nt, NT);
    std::vector<std::thread> pool;
    for (int i = 1; i < nt; ++i) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
}

void arrange_mfma_blocks(const std::vector<double>& blocks, int B, int k, int p, int NT, int NB, bool inverse,
                         std::vector<double>& out) {
    const int R = B + k, R16 = 16 * NB, NK = 4 * NB;
    if (R > R16) throw std::invalid_argument("arrange_mfma_blocks: block larger than the padded size");
    out.assign((size_t)NT * R16 * R16, 0.0);
    const double w0 = std::sqrt(0.5);
    for (int J = 0; J < NT; ++J) {
        const double* M = blocks.data() + (size_t)J * R * R;
        for (int rb = 0; rb < NB; ++rb) {
            for (int l = 0; l < 64; ++l) {
                const int row = 16 * rb + (l % 16);
                // float group g = kc / 4 of lane l: 64 lanes x 4 floats contiguous
                double* o = out.data() + ((size_t)J * NB + rb) * NK * 64 + 4 * l;
                for (int kc = 0; kc < NK; ++kc) {
                    const int q = 4 * kc + l / 16;
                    if (row >= R || q >= R) continue;
                    double v = inverse ? M[(size_t)q * R + row] : M[(size_t)row * R + q];
                    // slot 0 of tile 0 is m = 0 for odd l, weighted by w_0
                    if (J == 0 && p == 0 && (inverse ? row == 0 : q == 0)) v *= w0;
                    o[(kc / 4) * 256 + kc % 4] = v;
                }
            }
        }
    }
}

// j_l(x) and j_{l+1}(x), x > 0, FP64: upward recurrence from j_0, j_1 where it
// is stable (x well above l), else Miller's downward recurrence normalised by
// j_0 (or j_1 near a zero of j_0).
static void sph_bessel_pair(int l, double x, double& jl, double& jl1) {
    const double s = std::sin(x), c = std::cos(x);
    const double j0 = s / x, j1 = s / (x * x) - c / x;
    if (x > l + 25.0) {
        double a = j0, b = j1;
        for (int n = 1; n <= l; ++n) {
            const double nb = (2.0 * n + 1.0) / x * b - a;
            a = b;
            b = nb;
        }
        jl = a;
        jl1 = b;
        return;
    }
    const int L = l + 30 + (int)(x + 10.0 * std::sqrt(l + x + 10.0));
    double fp = 0.0, f = 1e-300, f0 = 0.0, f1 = 0.0, fl = 0.0, fl1 = 0.0;
    for (int n = L; n >= 1; --n) {   // f is f_n, fp is f_{n+1}; produce f_{n-1}
        if (n == l + 1) fl1 = f;
        if (n == l) fl = f;
        if (n == 1) f1 = f;
        const double fm = (2.0 * n + 1.0) / x * f - fp;
        fp = f;
        f = fm;
        if (std::fabs(f) > 1e250) {   // rescale everything kept so far
            f *= 1e-250;
            fp *= 1e-250;
            fl *= 1e-250;
            fl1 *= 1e-250;
            f1 *= 1e-250;
        }
    }
    f0 = f;
    if (l == 0) fl = f0;
    const double scale = std::fabs(j0) > std::fabs(j1) ? j0 / f0 : j1 / f1;
    jl = fl * scale;
    jl1 = fl1 * scale;
}

void corrected_momenta(int N, int ell, double rmax, double* k) {
    const int p = parity_p(ell), kx = n_extra(ell), n0 = n0_of(ell);
    const int need = N + p - 1 - n0 + 1;   // regular rows n0 .. N_l
    const double pi = 3.14159265358979323846;
    for (int j = 0; j < kx; ++j) k[j] = N * pi / rmax;   // completion rows keep the top momentum
    // even l: roots of chi_l(x) = x j_l(x); odd l: roots of chi_l'(x) = (l+1) j_l(x) - x j_{l+1}(x)
    auto f = [&](double x) {
        double a, b;
        sph_bessel_pair(ell, x, a, b);
        return p ? x * a : (ell + 1.0) * a - x * b;
    };
    const double h = 0.05;
    double x0 = 1e-3, f0 = f(x0);
    int found = 0;
    while (found < need) {
        const double x1 = x0 + h, f1 = f(x1);
        if ((f0 < 0.0 && f1 > 0.0) || (f0 > 0.0 && f1 < 0.0)) {
            double a = x0, b = x1, fa = f0;
            for (int it = 0; it < 80 && b - a > 1e-14 * b; ++it) {
                const double m = 0.5 * (a + b), fm = f(m);
                if ((fa < 0.0) == (fm < 0.0)) {
                    a = m;
                    fa = fm;
                } else {
                    b = m;
                }
            }
            k[kx + found] = 0.5 * (a + b) / rmax;
            ++found;
        }
        x0 = x1;
        f0 = f1;
        if (x0 > (N + ell + 8.0) * pi) throw std::runtime_error("corrected momenta: root scan ran past its range");
    }
}

void fft_quarter_roots(int N, std::vector<double>& cs) {
    const double pi = 3.14159265358979323846;
    cs.resize(2 * (size_t)(N / 4));
    for (int e = 0; e < N / 4; ++e) {
        const double a = 2.0 * pi * e / (double)N;
        cs[2 * e] = std::cos(a);
        cs[2 * e + 1] = std::sin(a);
    }
}

void fft_post_twiddles(int N, std::vector<double>& post) {
    const double pi = 3.14159265358979323846;
    post.resize(2 * (size_t)N);
    for (int t = 0; t < N; ++t) {
        const double b = -pi * t / (2.0 * N);
        post[2 * t] = std::cos(b);
        post[2 * t + 1] = std::sin(b);
    }
}

}  // namespace dsbt
