// Kernels on whole channel states used by the imaginary-time method (Sec. 4.3):
// Gram-Schmidt orthonormalisation within sets of channels and the energy
// terms of eq. H_DVR (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dsbt {

// One channel for the energy terms: data at [off, off + N), the FP64 potential
// term V tau/2 per point and the FP64 kinetic energy K_n = k_n^2/2 per slot.
struct EChan {
    int64_t off;
    int N;
    int pad_;
    const double* vangle;
    const double* kin;
};

// out[3 c + 0..2] = sum_i |psi_i|^2, sum_i V_i |psi_i|^2, sum_j K_j |b_j|^2 for
// channel c (FP64 sums), with V_i = vangle_i * vscale and b = T F psi given.
// S: float (complex64 data) or double (complex128 data).
template <typename S>
hipError_t launch_energy_terms(const EChan* d_chans, int nch, const void* psi, const void* b, double vscale,
                               double* out, hipStream_t s);

// Modified Gram-Schmidt, in channel order, within each set k of channels
// [first[k], first[k + 1]) (all of one N): channel j loses its components along
// the already orthonormalised channels of its set, then is scaled to unit norm
// (left zero if its norm is zero).  Channel c has offset off[c] and size N[c].
// One workgroup per set; in place on psi.
template <typename S>
hipError_t launch_orthonormalize(const int64_t* d_off, const int* d_N, const int* d_first, int nsets, void* psi,
                                 hipStream_t s);

}  // namespace dsbt
