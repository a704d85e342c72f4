// Device-side descriptors and launchers of the DSBT kernels (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dsbt {

constexpr int kBlock = 256;          // threads per workgroup of every transform kernel
constexpr int kMaxChanPerItem = 16;  // channels sharing one moment-table pass

// One channel of the sine/cosine stage (Sec. 2.2, eq. csFourierBasis).
struct FChan {
    int64_t off;          // element offset of the channel in every data buffer
    int N, log2N;
    int p;                // 1: even l (DST-II), 0: odd l (DCT-II)
    float sign;           // (-1)^ceil(l/2), or +1 for the printed F
    const void* tw;       // exp(-2 pi i t/N), t < N, complex of the data precision
    const void* post;     // exp(-i pi t/(2N)), t < N
    const float2* vphase; // unit-modulus exp(-i V tau/2) per point, or nullptr
    const double* vangle; // V tau/2 per point (FP64), or nullptr
};

// One work item of the moment stage: up to kMaxChanPerItem channels with the
// same (l, N) sharing one pass over the tiles.
struct MItem {
    const void* tab_f;     // NT blocks, A[q][r] = M_J[r][q]
    const void* tab_i;     // NT blocks, A[q][r] = M_J[q][r]
    const float2* kphase;  // unit-modulus exp(-i K_n tau) per slot, or nullptr
    int B, k, R, NT, p, nch;
    int64_t off[kMaxChanPerItem];
};

// How a stage multiplies by the diagonal phases of the split step.
struct PhaseArgs {
    int use;             // 0: no phase
    int conj;            // 1: conjugated (adjoint step)
    const float* scale;  // per-step FP32 potential strengths, or nullptr (all ones)
    int step;            // index into scale
};

// Raise the dynamic-LDS limit of the transform kernels (call before launching
// or capturing; not a stream operation).
template <typename T>
hipError_t set_lds_limits(size_t fstage_bytes, size_t mstage_bytes);

// Launchers.  T = float (complex64 data) or double (complex128 data).
template <typename T>
hipError_t launch_fstage(const FChan* d_chans, int nch, int maxN, const void* src, void* dst,
                         bool inverse, PhaseArgs ph, hipStream_t s);

template <typename T>
hipError_t launch_mstage(const MItem* d_items, int nitems, int maxR, const void* src, void* dst,
                         bool inverse, PhaseArgs ph, hipStream_t s);

// Partial sums of sum_i vangle_i Im(conj(l1) p1 + conj(l0) p0) per channel into
// scratch[nch], then out[0] = their sum (FP64).
template <typename T>
hipError_t launch_grad_s(const FChan* d_chans, int nch, const void* p0, const void* p1,
                         const void* l0, const void* l1, double* scratch, double* out,
                         hipStream_t s);

}  // namespace dsbt
