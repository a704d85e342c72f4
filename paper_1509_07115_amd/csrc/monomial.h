// The paper's own fast Fourier-to-Bessel multiplication with monomial moments
// (Sec. 2.6), an FP64 variant of the moment stage for complex128 plans
// (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>

#include "kernels.h"

namespace dsbt {

// One channel of the monomial stage.  Regular rows n = n0..Nl (Nl = N + p - 1)
// use xi[(n - n0) k + q] = xi_nu(n) for nu = nu0 + 2 q (q < k = ceil(l/2), the
// coefficients of eq. DP_expan of the parity of l + 1) and alpha[n - n0]; the
// completion rows are comp[q N + j], q < k, over slots j (eq. Tadd).
struct LChan {
    int64_t off;
    int N, ell, p, n0, k, nu0;
    const double* xi;
    const double* alpha;
    const double* comp;
    const void* kphase;   // exp(-i K_n tau) per slot (double2), or nullptr
};

// Host FP64 tables of one (N, l): xi (from a binary128 expansion of the DLOP
// backward difference, rounded once), alpha (row norms of I - L from FP64 DLOP
// values) and the completion rows.  Sizes: xi (Nl - n0 + 1) k, alpha
// Nl - n0 + 1, comp k N.
void monomial_tables(int N, int ell, std::vector<double>& xi, std::vector<double>& alpha,
                     std::vector<double>& comp);

// One wave per channel, complex128 data, in place allowed.  Forward: b = T f by
// the prefix sums of eq. rec_sum_b_f, the kinetic phase (ph.use) fused into
// the stores.  Inverse: f = T^T b by the suffix sums of eq. rec_sum_f_b.
hipError_t launch_monomial(const LChan* d_chans, int nch, const void* src, void* dst, bool inverse, PhaseArgs ph,
                           hipStream_t s);

}  // namespace dsbt
