// Angular transform Y = P Phi of the DSBT-DVR solver (Sec. 4.1), internal header.
//
// Grid values psi[j][k][i] on Gauss-Legendre nodes eta_j (ascending), azimuths
// phi_k = 2 pi k / N_phi and radial points i (fastest) map to coefficients
// c[q][t][i] of the spherical harmonics (l, m), m = q - M (N_phi = 2M + 1),
// l = |m| + t.  Forward: a[j][q][i] = sum_k Phi[q][k] psi[j][k][i], then
// c[q][t][i] = sum_j P[q][t][j] a[j][q][i]; inverse: the conjugate transpose.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "../../include/dsbt.h"

namespace dsbt {

constexpr int kShtMaxQ = 64;   // largest N_theta and N_phi of the axis kernel
constexpr int kShtMaxPhi = 63; // largest N_phi accepted (|m| <= 31)

// Records msg as the thread's last error (dsbt_last_error) and returns s.
dsbt_status set_error(dsbt_status s, const char* msg);

// FP64 host tables: Gauss-Legendre nodes (ascending) and weights, and
// P[q][t][j] = Pbar_{|m|+t}^m(eta_j) sqrt(w_j) orthonormalised in t on the
// quadrature (Pbar with unit L2 norm on [-1, 1], Condon-Shortley phase), built
// by the Lanczos recurrence on the weighted nodes.
void gauss_legendre(int n, std::vector<double>& eta, std::vector<double>& w);
void sht_p_tables(int n_theta, int n_phi, std::vector<double>& P);

// dst[o*dout + q'*dq + i] = sum_q A_o(q', q) src[o*so + q*sq + i] for o < nouter,
// q, q' < Q, i < Nr; A_o(q', q) = mat[o*mso + (tr ? q*Q + q' : q'*Q + q)], conjugated
// with cj.  S: float or double; CA: complex (interleaved) or real matrix.
// Raise the dynamic-LDS limit of the axis kernel (up to 128 KiB for FP64
// complex matrices); call before launching or capturing.
hipError_t set_lds_limits_axis();
template <typename S, bool CA>
hipError_t launch_axis_apply(const S* mat, int64_t mso, bool tr, bool cj, const void* src, int64_t so, int64_t sq,
                             void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr, hipStream_t s);

// launch_axis_apply for complex64 data on the matrix cores, the matrix given
// as a real FP32 table mat16 + o*mso, row-major Q16 x Q16, zero outside the
// used block, 16-byte aligned.  Real matrix (complex_matrix false):
// A_o(q', q) = mat16[o*mso + q'*Q16 + q], Q16 = Q rounded up to 16.  Complex
// matrix: row 2 q' + a, column 2 q + b hold [[Re, -Im], [Im, Re]][a][b] of
// A_o(q', q), Q16 = 2 Q rounded up to 16.  Q16 <= 64 (real) or 128 (complex;
// above 64 only with mso = 0), else hipErrorInvalidValue.
hipError_t launch_axis_mfma(bool complex_matrix, const float* mat16, int64_t mso, const void* src, int64_t so,
                            int64_t sq, void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr,
                            hipStream_t s);

// launch_axis_mfma for complex128 data on the FP64 matrix cores, the matrix as
// an FP64 table of the same layout (Q16 <= 64).
hipError_t launch_axis_mfma64(bool complex_matrix, const double* mat16, int64_t mso, const void* src, int64_t so,
                              int64_t sq, void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr,
                              hipStream_t s);

// x[i] *= exp(-i (V0[i] + F V1[i]) dt/2) for i < n (complex of S; V0, V1 FP64
// device arrays or null), angles reduced mod 2 pi in FP64.
template <typename S>
hipError_t launch_grid_phase(void* x, const double* V0, const double* V1, double F, double dt, int64_t n,
                             hipStream_t s);

// Coefficient channels (layout c[q][t][i]) to the unified momentum order and
// back, with the factor i^-l (forward) or i^l (inverse) of the modified
// spherical harmonics; src and dst must not overlap.
template <typename S>
hipError_t launch_momentum_order(const void* src, void* dst, int nt, int nphi, int Nr, bool inverse, hipStream_t s);

}  // namespace dsbt
