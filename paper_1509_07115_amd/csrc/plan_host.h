// Host-side FP64 plan generation for the orthogonal DSBT (internal header).
//
// The Fourier-to-Bessel matrix T of Sec. 2.4-2.5 is applied in a tiled moment
// form.  Slots j = n - p are cut into tiles of B.  For tile J (slots [JB, JB+B),
// momentum indices m in [t_J, t_J + B) with t_J = p + J B) the product is
//
//     [ b_J     ]   [ W_J  E_J ] [ g_J  ]
//     [ mu_J+1  ] = [ Q_J  D_J ] [ mu_J ]            g_m = w_m f_m,
//
// where mu_J are the moments sum_{m < t_J} q^(J)_k(m) g_m of the data against an
// orthonormal polynomial basis q^(J) of the regular-row kernel space on
// [0, t_J) (DLOPs on the symmetric grid of 2 t_J - 1 points, Sec. 2.3), W_J is
// the in-tile band of T, E_J the expansion of each row's kernel in q^(J), Q_J
// the tile's contribution to the next moments and D_J the change of basis
// q^(J+1) -> q^(J) restricted to [0, t_J).  The completion rows of eq. Tadd are
// (-1)^p mu_NT: on the full grid the tile basis is exactly those DLOP rows.
// The inverse applies the transposed blocks in reverse tile order.
#pragma once
#include <cstdint>
#include <vector>

namespace dsbt {

int parity_p(int ell);
int n0_of(int ell);
int n_extra(int ell);

// P_d(x, M) for integer x = 0..xmax (xmax <= M), FP64: the degree recurrence
// when d^2 <= 2M, else the difference equation in x marched from x = 0.
void dlop_values(int d, int M, int xmax, double* out);

// Orthonormal basis q_kk(m), m in [0, t), kk < ceil(l/2), degree 2 kk + p, with
// the half-grid inner product (weight 1/2 at m = 0); out is [k][t].
void tile_basis(int ell, int t, double* out);

// Smallest admissible power-of-two tile (>= n0, >= 32) for l, capped at N.
int auto_tile(int ell, int N);

// Moment-tile blocks for (ell, B) over NT tiles, row-major M_J[r][q], R = B + k.
// Rows of T are the same for every N, so one table serves every N = NT' B <= NT B.
// `nthreads` host threads are used (0 = hardware concurrency).
void build_ftb_blocks(int ell, int B, int NT, std::vector<double>& blocks, int nthreads);

// Rearrange row-major blocks into the matrix-core operand layout (see
// MItem::mf_f in kernels.h): A' = M_J (forward) or M_J^T (inverse), padded to
// R16 = 16 NB, with the weight w_0 = 1/sqrt(2) of odd l folded into the slot-0
// column (forward) or row (inverse) of tile 0.
void arrange_mfma_blocks(const std::vector<double>& blocks, int B, int k, int p, int NT, int NB, bool inverse,
                         std::vector<double>& out);

// Momenta k of the kinetic diagonal in slot order (N values): the completion
// rows take N dk; regular row n takes x_j / rmax with x_j the j-th positive
// root (j = n - n0 + 1) of chi_l(x) = x j_l(x) for even l or of chi_l'(x) for
// odd l (Sec. 3, eq. kcorr), FP64, bracketed on a scan from x = 0 and bisected.
void corrected_momenta(int N, int ell, double rmax, double* k);

// FP64 tables of the size-N sine/cosine stage as interleaved pairs:
// fft_quarter_roots, (cos, sin) of 2 pi e/N for e < N/4, from which the FFT
// kernels form every pass twiddle exp(-2 pi i m/N) (m = e + q N/4: the
// product by exp(-2 pi i e/N), then by (-i)^q); fft_post_twiddles,
// exp(-i pi k/(2N)) for k < N.
void fft_quarter_roots(int N, std::vector<double>& cs);
void fft_post_twiddles(int N, std::vector<double>& post);

}  // namespace dsbt
