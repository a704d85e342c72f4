// C ABI of the angular transform Y = P Phi (Sec. 4.1): dsbt_sht_* in include/dsbt.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/dsbt.h"
#include "angular.h"

struct dsbt_sht_s {
    int Nr = 0, nt = 0, nphi = 0, precision = DSBT_C64;
    void* d_phi = nullptr;   // Phi[q][k] complex (interleaved), precision of the data
    void* d_work = nullptr;  // a[j][q][i], complex
    void* d_pm = nullptr;    // [2][q][16 NR][16 NR] zero-padded P[q] (forward) and P[q]^T (inverse), data precision
    void* d_fm = nullptr;    // 2 N_phi <= 128 (complex64) or 64: [2][F16][F16] real forms of Phi and Phi^H, zero-padded
    void release() {
        if (d_phi) (void)hipFree(d_phi);
        if (d_work) (void)hipFree(d_work);
        if (d_pm) (void)hipFree(d_pm);
        if (d_fm) (void)hipFree(d_fm);
        d_phi = d_work = nullptr;
        d_pm = d_fm = nullptr;
    }
};

namespace {

template <typename S>
hipError_t upload(const std::vector<double>& h, void** d) {
    std::vector<S> v(h.begin(), h.end());
    hipError_t e = hipMalloc(d, sizeof(S) * (v.empty() ? 1 : v.size()));
    if (e != hipSuccess) return e;
    return hipMemcpy(*d, v.data(), sizeof(S) * v.size(), hipMemcpyHostToDevice);
}

template <typename S>
hipError_t run(dsbt_sht_s* p, const void* src, void* dst, bool inverse, hipStream_t s) {
    const int nt = p->nt, nf = p->nphi, Nr = p->Nr;
    const int64_t lf = (int64_t)nf * Nr, lt = (int64_t)nt * Nr;
    const S* F = static_cast<const S*>(p->d_phi);
    const int64_t q16 = (nt + 15) / 16 * 16;
    const int64_t f16 = (2 * nf + 15) / 16 * 16;
    // matrix cores (the complex128 DFT while 2 N_phi <= 64), the vector kernel otherwise
    auto legendre = [&](bool tr, const void* x, int64_t so, int64_t sq, void* y, int64_t dout, int64_t dq) {
        const S* pm = static_cast<const S*>(p->d_pm) + (tr ? nf * q16 * q16 : 0);
        if constexpr (std::is_same<S, float>::value)
            return dsbt::launch_axis_mfma(false, pm, q16 * q16, x, so, sq, y, dout, dq, nt, nf, Nr, s);
        else
            return dsbt::launch_axis_mfma64(false, pm, q16 * q16, x, so, sq, y, dout, dq, nt, nf, Nr, s);
    };
    auto azimuth = [&](bool inv, const void* x, void* y) {
        if (p->d_fm) {
            const S* fm = static_cast<const S*>(p->d_fm) + (inv ? f16 * f16 : 0);
            if constexpr (std::is_same<S, float>::value)
                return dsbt::launch_axis_mfma(true, fm, 0, x, lf, Nr, y, lf, Nr, nf, nt, Nr, s);
            else
                return dsbt::launch_axis_mfma64(true, fm, 0, x, lf, Nr, y, lf, Nr, nf, nt, Nr, s);
        }
        return dsbt::launch_axis_apply<S, true>(F, 0, inv, inv, x, lf, Nr, y, lf, Nr, nf, nt, Nr, s);
    };
    hipError_t e;
    if (!inverse) {
        // a[j][q][i] = sum_k Phi[q][k] psi[j][k][i]; c[q][t][i] = sum_j P[q][t][j] a[j][q][i]
        e = azimuth(false, src, p->d_work);
        if (e == hipSuccess) e = legendre(false, p->d_work, Nr, lf, dst, lt, Nr);
    } else {
        // a[j][q][i] = sum_t P[q][t][j] c[q][t][i]; psi[j][k][i] = sum_q conj(Phi[q][k]) a[j][q][i]
        e = legendre(true, src, lt, Nr, p->d_work, Nr, lf);
        if (e == hipSuccess) e = azimuth(true, p->d_work, dst);
    }
    return e;
}

}  // namespace

extern "C" {

dsbt_status dsbt_sht_grid(int32_t n_theta, int32_t n_phi, double* eta, double* w, double* phi) {
    if (n_theta < 1 || n_theta > dsbt::kShtMaxQ || n_phi < 1 || n_phi > dsbt::kShtMaxPhi || n_phi % 2 == 0)
        return dsbt::set_error(DSBT_ERR_UNSUPPORTED, "need 1 <= N_theta <= 64 and odd 1 <= N_phi <= 63");
    std::vector<double> e, ww;
    dsbt::gauss_legendre(n_theta, e, ww);
    for (int j = 0; j < n_theta; ++j) {
        if (eta) eta[j] = e[j];
        if (w) w[j] = ww[j];
    }
    const double pi = 3.14159265358979323846;
    for (int k = 0; phi && k < n_phi; ++k) phi[k] = 2.0 * pi * k / n_phi;
    return DSBT_OK;
}

dsbt_status dsbt_sht_host_tables(int32_t n_theta, int32_t n_phi, double* P) {
    if (!P) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "P is NULL");
    dsbt_status st = dsbt_sht_grid(n_theta, n_phi, nullptr, nullptr, nullptr);
    if (st != DSBT_OK) return st;
    std::vector<double> h;
    dsbt::sht_p_tables(n_theta, n_phi, h);
    for (size_t i = 0; i < h.size(); ++i) P[i] = h[i];
    return DSBT_OK;
}

dsbt_status dsbt_sht_create(dsbt_sht* out, int32_t Nr, int32_t n_theta, int32_t n_phi, int32_t precision) {
    if (!out) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (Nr < 1) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "Nr must be positive");
    if (precision != DSBT_C64 && precision != DSBT_C128)
        return dsbt::set_error(DSBT_ERR_UNSUPPORTED, "precision must be DSBT_C64 or DSBT_C128");
    dsbt_status st = dsbt_sht_grid(n_theta, n_phi, nullptr, nullptr, nullptr);
    if (st != DSBT_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return dsbt::set_error(DSBT_ERR_NO_DEVICE, "no HIP device");
    dsbt_sht_s* p = new (std::nothrow) dsbt_sht_s();
    if (!p) return dsbt::set_error(DSBT_ERR_OOM, "host allocation failed");
    p->Nr = Nr;
    p->nt = n_theta;
    p->nphi = n_phi;
    p->precision = precision;
    std::vector<double> P, F((size_t)2 * n_phi * n_phi);
    dsbt::sht_p_tables(n_theta, n_phi, P);
    const int M = (n_phi - 1) / 2;
    const double pi = 3.14159265358979323846, sc = 1.0 / std::sqrt((double)n_phi);
    for (int q = 0; q < n_phi; ++q)
        for (int k = 0; k < n_phi; ++k) {
            const int mk = (((q - M) * k) % n_phi + n_phi) % n_phi;   // m k mod N_phi, exact
            const double a = 2.0 * pi * mk / n_phi;
            F[2 * ((size_t)q * n_phi + k)] = std::cos(a) * sc;
            F[2 * ((size_t)q * n_phi + k) + 1] = -std::sin(a) * sc;
        }
    const size_t work = (size_t)n_theta * n_phi * Nr * (precision == DSBT_C128 ? 16 : 8);
    hipError_t e = dsbt::set_lds_limits_axis();
    if (e == hipSuccess) e = precision == DSBT_C128 ? upload<double>(F, &p->d_phi) : upload<float>(F, &p->d_phi);
    if (e == hipSuccess) e = hipMalloc(&p->d_work, work);
    if (e == hipSuccess) {
        const size_t q16 = (size_t)(n_theta + 15) / 16 * 16, blk = q16 * q16;
        std::vector<double> pm(2 * n_phi * blk, 0.0);
        for (int q = 0; q < n_phi; ++q)
            for (int t = 0; t < n_theta; ++t)
                for (int j = 0; j < n_theta; ++j) {
                    const double v = P[((size_t)q * n_theta + t) * n_theta + j];
                    pm[q * blk + t * q16 + j] = v;                     // forward: rows t, columns j
                    pm[(n_phi + q) * blk + j * q16 + t] = v;           // inverse: rows j, columns t
                }
        e = precision == DSBT_C128 ? upload<double>(pm, &p->d_pm) : upload<float>(pm, &p->d_pm);
    }
    if (e == hipSuccess && 2 * n_phi <= (precision == DSBT_C64 ? 128 : 64)) {
        // [[Re, -Im], [Im, Re]] per element: forward A(q, k) = Phi[q][k], inverse A(k, q) = conj(Phi[q][k])
        const size_t f16 = (size_t)(2 * n_phi + 15) / 16 * 16, blk = f16 * f16;
        std::vector<double> fm(2 * blk, 0.0);
        for (int q = 0; q < n_phi; ++q)
            for (int k = 0; k < n_phi; ++k) {
                const double re = F[2 * ((size_t)q * n_phi + k)], im = F[2 * ((size_t)q * n_phi + k) + 1];
                double* f = fm.data() + 2 * q * f16 + 2 * k;       // forward: rows 2q + a, columns 2k + b
                f[0] = re;
                f[1] = -im;
                f[f16] = im;
                f[f16 + 1] = re;
                double* g = fm.data() + blk + 2 * k * f16 + 2 * q;   // inverse: rows 2k + a, columns 2q + b
                g[0] = re;
                g[1] = im;
                g[f16] = -im;
                g[f16 + 1] = re;
            }
        e = precision == DSBT_C128 ? upload<double>(fm, &p->d_fm) : upload<float>(fm, &p->d_fm);
    }
    if (e != hipSuccess) {
        p->release();
        delete p;
        return dsbt::set_error(e == hipErrorOutOfMemory ? DSBT_ERR_OOM : DSBT_ERR_HIP, hipGetErrorString(e));
    }
    *out = p;
    return DSBT_OK;
}

dsbt_status dsbt_sht_destroy(dsbt_sht p) {
    if (!p) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL transform");
    p->release();
    delete p;
    return DSBT_OK;
}

static dsbt_status sht_apply(dsbt_sht p, const void* src, void* dst, bool inverse, void* stream) {
    if (!p || !src || !dst) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL argument");
    const hipError_t e = p->precision == DSBT_C128 ? run<double>(p, src, dst, inverse, (hipStream_t)stream)
                                                   : run<float>(p, src, dst, inverse, (hipStream_t)stream);
    if (e != hipSuccess) return dsbt::set_error(DSBT_ERR_HIP, hipGetErrorString(e));
    return DSBT_OK;
}

dsbt_status dsbt_sht_forward(dsbt_sht p, const void* grid, void* coef, void* stream) {
    return sht_apply(p, grid, coef, false, stream);
}

dsbt_status dsbt_sht_inverse(dsbt_sht p, const void* coef, void* grid, void* stream) {
    return sht_apply(p, coef, grid, true, stream);
}

dsbt_status dsbt_sht_potential_phase(dsbt_sht p, void* grid, const double* V0, const double* V1, double F, double dt,
                                     void* stream) {
    if (!p || !grid) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (!std::isfinite(F) || !std::isfinite(dt)) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "non-finite F or dt");
    const int64_t n = (int64_t)p->Nr * p->nt * p->nphi;
    const hipError_t e = p->precision == DSBT_C128
                             ? dsbt::launch_grid_phase<double>(grid, V0, V1, F, dt, n, (hipStream_t)stream)
                             : dsbt::launch_grid_phase<float>(grid, V0, V1, F, dt, n, (hipStream_t)stream);
    if (e != hipSuccess) return dsbt::set_error(DSBT_ERR_HIP, hipGetErrorString(e));
    return DSBT_OK;
}

dsbt_status dsbt_sht_momentum_order(dsbt_sht p, const void* src, void* dst, int32_t inverse, void* stream) {
    if (!p || !src || !dst) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL argument");
    const size_t bytes = (size_t)p->Nr * p->nt * p->nphi * (p->precision == DSBT_C128 ? 16 : 8);
    const char* a = static_cast<const char*>(src);
    const char* b = static_cast<const char*>(dst);
    if (a < b + bytes && b < a + bytes) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "src and dst overlap");
    const hipError_t e =
        p->precision == DSBT_C128
            ? dsbt::launch_momentum_order<double>(src, dst, p->nt, p->nphi, p->Nr, inverse != 0, (hipStream_t)stream)
            : dsbt::launch_momentum_order<float>(src, dst, p->nt, p->nphi, p->Nr, inverse != 0, (hipStream_t)stream);
    if (e != hipSuccess) return dsbt::set_error(DSBT_ERR_HIP, hipGetErrorString(e));
    return DSBT_OK;
}

dsbt_status dsbt_step3d(dsbt_sht y, dsbt_plan p, void* grid, void* work, const double* V0, const double* V1, double F,
                        double dt, void* stream) {
    if (!y || !p || !grid || !work) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL argument");
    dsbt_status st = dsbt_sht_potential_phase(y, grid, V0, V1, F, dt, stream);
    if (st == DSBT_OK) st = dsbt_sht_forward(y, grid, work, stream);
    if (st == DSBT_OK) st = dsbt_kinetic_step(p, work, 1, nullptr, 0, stream);
    if (st == DSBT_OK) st = dsbt_sht_inverse(y, work, grid, stream);
    if (st == DSBT_OK) st = dsbt_sht_potential_phase(y, grid, V0, V1, F, dt, stream);
    return st;
}

dsbt_status dsbt_sht_kinetic(dsbt_sht y, double rmax, int32_t kinetic, double* K, void* stream) {
    if (!y || !K) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (!(rmax > 0.0) || !std::isfinite(rmax)) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "rmax must be positive");
    if (kinetic != DSBT_K_PLAIN && kinetic != DSBT_K_CORRECTED)
        return dsbt::set_error(DSBT_ERR_INVALID_ARG, "unknown kinetic option");
    const int nt = y->nt, nphi = y->nphi, Nr = y->Nr, M = (nphi - 1) / 2;
    std::vector<double> h((size_t)nt * nphi * Nr), k(Nr);
    for (int q = 0; q < nphi; ++q) {
        for (int t = 0; t < nt; ++t) {
            const int ell = std::abs(q - M) + t;
            const dsbt_status st = dsbt_kinetic_momenta(Nr, ell, rmax, kinetic, k.data());
            if (st != DSBT_OK) return st;
            double* row = h.data() + ((size_t)q * nt + t) * Nr;
            for (int i = 0; i < Nr; ++i) row[i] = 0.5 * k[i] * k[i];   // eq. KinMat
        }
    }
    const hipError_t e = hipMemcpyAsync(K, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize((hipStream_t)stream) : e;
    if (e2 != hipSuccess) return dsbt::set_error(DSBT_ERR_HIP, (std::string("dsbt_sht_kinetic: ") + hipGetErrorString(e2)).c_str());
    return DSBT_OK;
}

dsbt_status dsbt_sht_momentum_pz(dsbt_sht y, double rmax, double* Pz, void* stream) {
    if (!y || !Pz) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (!(rmax > 0.0) || !std::isfinite(rmax)) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "rmax must be positive");
    const int nt = y->nt, nphi = y->nphi, Nr = y->Nr;
    std::vector<double> eta(nt);
    dsbt_status st = dsbt_sht_grid(nt, nphi, eta.data(), nullptr, nullptr);
    if (st != DSBT_OK) return st;
    const double dk = 3.14159265358979323846 / rmax;
    std::vector<double> h((size_t)nt * nphi * Nr);
    for (int j = 0; j < nt; ++j)
        for (int q = 0; q < nphi; ++q) {
            double* row = h.data() + ((size_t)j * nphi + q) * Nr;
            for (int i = 0; i < Nr; ++i) row[i] = -2.0 * eta[j] * (double)(i + 1) * dk;   // k~_n = n dk, n = i + 1
        }
    const hipError_t e = hipMemcpyAsync(Pz, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize((hipStream_t)stream) : e;
    if (e2 != hipSuccess)
        return dsbt::set_error(DSBT_ERR_HIP, (std::string("dsbt_sht_momentum_pz: ") + hipGetErrorString(e2)).c_str());
    return DSBT_OK;
}

dsbt_status dsbt_step3d_velocity(dsbt_sht y, dsbt_plan p, void* grid, void* work1, void* work2, const double* V0,
                                 const double* K, const double* Pz, double A, double dt, void* stream) {
    if (!y || !p || !grid || !work1 || !work2 || !K || !Pz) return dsbt::set_error(DSBT_ERR_INVALID_ARG, "NULL argument");
    dsbt_status st = dsbt_sht_potential_phase(y, grid, V0, nullptr, 0.0, dt, stream);
    if (st == DSBT_OK) st = dsbt_sht_forward(y, grid, work1, stream);
    if (st == DSBT_OK) st = dsbt_forward(p, work1, work1, stream);                       // c = B Y psi
    if (st == DSBT_OK) st = dsbt_sht_potential_phase(y, work1, K, nullptr, 0.0, dt, stream);   // exp(-i K dt/2)
    if (st == DSBT_OK) st = dsbt_sht_momentum_order(y, work1, work2, 0, stream);
    if (st == DSBT_OK) st = dsbt_sht_inverse(y, work2, work1, stream);                   // Ytilde^H: plane waves
    if (st == DSBT_OK) st = dsbt_sht_potential_phase(y, work1, nullptr, Pz, A, dt, stream);   // exp(i A k eta dt)
    if (st == DSBT_OK) st = dsbt_sht_forward(y, work1, work2, stream);
    if (st == DSBT_OK) st = dsbt_sht_momentum_order(y, work2, work1, 1, stream);
    if (st == DSBT_OK) st = dsbt_sht_potential_phase(y, work1, K, nullptr, 0.0, dt, stream);
    if (st == DSBT_OK) st = dsbt_inverse(p, work1, work1, stream);
    if (st == DSBT_OK) st = dsbt_sht_inverse(y, work1, grid, stream);
    if (st == DSBT_OK) st = dsbt_sht_potential_phase(y, grid, V0, nullptr, 0.0, dt, stream);
    return st;
}

}  // extern "C"
