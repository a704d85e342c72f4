// Whole-state kernels of the imaginary-time method (Sec. 4.3): energy terms of
// eq. H_DVR per channel and Gram-Schmidt orthonormalisation within sets of
// channels.  Both are small memory-bound passes (one workgroup per channel or
// set) with FP64 accumulation.
#include "state.h"

namespace dsbt {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename S> struct Cplx;
template <> struct Cplx<float> { typedef float2 t; };
template <> struct Cplx<double> { typedef double2 t; };

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sums NV values over the workgroup; every thread receives the totals.  red
// holds NV * kWaves doubles; the trailing barrier lets red be reused at once.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q * kWaves + wave] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) t += red[q * kWaves + w];
        v[q] = t;
    }
    __syncthreads();
}

template <typename S>
__global__ void __launch_bounds__(kThreads) energy_terms(const EChan* __restrict__ chans,
                                                         const typename Cplx<S>::t* __restrict__ psi,
                                                         const typename Cplx<S>::t* __restrict__ b, double vscale,
                                                         double* __restrict__ out) {
    const EChan c = chans[blockIdx.x];
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < c.N; i += kThreads) {
        const auto z = psi[c.off + i];
        const auto w = b[c.off + i];
        const double a2 = (double)z.x * z.x + (double)z.y * z.y;
        v[0] += a2;
        v[1] += c.vangle[i] * vscale * a2;
        v[2] += c.kin[i] * ((double)w.x * w.x + (double)w.y * w.y);
    }
    __shared__ double red[3 * kWaves];
    block_sum<3>(v, red);
    if (threadIdx.x < 3) out[3 * blockIdx.x + threadIdx.x] = v[threadIdx.x];
}

template <typename S>
__global__ void __launch_bounds__(kThreads) orthonormalize(const int64_t* __restrict__ off,
                                                           const int* __restrict__ Nc,
                                                           const int* __restrict__ first,
                                                           typename Cplx<S>::t* __restrict__ psi) {
    using V = typename Cplx<S>::t;
    const int c0 = first[blockIdx.x], c1 = first[blockIdx.x + 1];
    __shared__ double red[2 * kWaves];
    constexpr int kRegs = 16;   // values per thread of the one-channel path
    if (c1 - c0 == 1 && Nc[c0] >= 1 && Nc[c0] <= kThreads * kRegs) {
        // A set of one channel is only normalised: the channel is held in
        // registers (one read and one write; the loads come from clamped
        // addresses with no branch, so they are all in flight at once).  Each
        // thread sums its values in the order of the loop below, so the result
        // is the same.
        V* pj = psi + off[c0];
        const int N = Nc[c0];
        V z[kRegs];
#pragma unroll
        for (int u = 0; u < kRegs; ++u) z[u] = pj[min((int)threadIdx.x + kThreads * u, N - 1)];
        double n2[1] = {0.0};
#pragma unroll
        for (int u = 0; u < kRegs; ++u)
            n2[0] += (int)threadIdx.x + kThreads * u < N ? (double)z[u].x * z[u].x + (double)z[u].y * z[u].y : 0.0;
        block_sum<1>(n2, red);
        const double sc = n2[0] > 0.0 ? 1.0 / sqrt(n2[0]) : 0.0;
#pragma unroll
        for (int u = 0; u < kRegs; ++u) {
            const int k = threadIdx.x + kThreads * u;
            if (k < N) {
                V z1 = z[u];
                z1.x = (S)(z1.x * sc);
                z1.y = (S)(z1.y * sc);
                pj[k] = z1;
            }
        }
        return;
    }
    for (int j = c0; j < c1; ++j) {
        V* pj = psi + off[j];
        const int N = Nc[j];
        for (int i = c0; i < j; ++i) {
            const V* pi = psi + off[i];
            // <psi_i | psi_j> = sum conj(psi_i) psi_j
            double d[2] = {0.0, 0.0};
            for (int k = threadIdx.x; k < N; k += kThreads) {
                const V a = pi[k], z = pj[k];
                d[0] += (double)a.x * z.x + (double)a.y * z.y;
                d[1] += (double)a.x * z.y - (double)a.y * z.x;
            }
            block_sum<2>(d, red);
            // each thread rewrites only the elements it read, so no barrier is needed
            for (int k = threadIdx.x; k < N; k += kThreads) {
                const V a = pi[k];
                V z = pj[k];
                z.x = (S)((double)z.x - (d[0] * a.x - d[1] * a.y));
                z.y = (S)((double)z.y - (d[0] * a.y + d[1] * a.x));
                pj[k] = z;
            }
        }
        double n2[1] = {0.0};
        for (int k = threadIdx.x; k < N; k += kThreads) {
            const V z = pj[k];
            n2[0] += (double)z.x * z.x + (double)z.y * z.y;
        }
        block_sum<1>(n2, red);
        const double sc = n2[0] > 0.0 ? 1.0 / sqrt(n2[0]) : 0.0;
        for (int k = threadIdx.x; k < N; k += kThreads) {
            V z = pj[k];
            z.x = (S)(z.x * sc);
            z.y = (S)(z.y * sc);
            pj[k] = z;
        }
        // channel j is read by later channels of the set through other threads
        __syncthreads();
    }
}

}  // namespace

template <typename S>
hipError_t launch_energy_terms(const EChan* d_chans, int nch, const void* psi, const void* b, double vscale,
                               double* out, hipStream_t s) {
    using V = typename Cplx<S>::t;
    if (nch <= 0) return hipSuccess;
    hipLaunchKernelGGL(energy_terms<S>, dim3(nch), dim3(kThreads), 0, s, d_chans, (const V*)psi, (const V*)b, vscale,
                       out);
    return hipGetLastError();
}

template <typename S>
hipError_t launch_orthonormalize(const int64_t* d_off, const int* d_N, const int* d_first, int nsets, void* psi,
                                 hipStream_t s) {
    if (nsets <= 0) return hipSuccess;
    hipLaunchKernelGGL(orthonormalize<S>, dim3(nsets), dim3(kThreads), 0, s, d_off, d_N, d_first,
                       (typename Cplx<S>::t*)psi);
    return hipGetLastError();
}

template hipError_t launch_energy_terms<float>(const EChan*, int, const void*, const void*, double, double*,
                                               hipStream_t);
template hipError_t launch_energy_terms<double>(const EChan*, int, const void*, const void*, double, double*,
                                                hipStream_t);
template hipError_t launch_orthonormalize<float>(const int64_t*, const int*, const int*, int, void*, hipStream_t);
template hipError_t launch_orthonormalize<double>(const int64_t*, const int*, const int*, int, void*, hipStream_t);

}  // namespace dsbt
