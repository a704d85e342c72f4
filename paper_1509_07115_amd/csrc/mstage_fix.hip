// Correction of a split moment pass (matrix-core path, B = 32).
//
// The tile chain of the moment stage (Sec. 2.4-2.5, tiled moment form) is a
// linear recursion in the moments, so a pass over tiles can be cut in two
// ranges that run at the same time: the second starts from zero moments and
// misses the term G_J mu_H that the first range's final moments mu_H carry
// into each of its tiles (FixItem in kernels.h).  This kernel adds that rank-k
// term, G_J mu_H as v_mfma_f32_16x16x4_f32 products (16 rows x 16 real
// columns = 8 channels per product; lane l: A[l%16][l/16], B[l/16][l%16],
// result register v: row 4 (l/16) + v), to the pass output in place, and on
// the forward pass writes the completion rows (-1)^p (mu_NT^0 + Phi mu_H).
#include "kernels.h"

namespace dsbt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

// (a + ib)(wr + i wi) on the lane pair (re, im) of one complex value
__device__ __forceinline__ float lane_cmul(float x, f2 w, bool im, bool cj) {
    const float y = __shfl_xor(x, 1, 64);
    const float s = cj ? -w.y : w.y;
    return im ? x * w.x + y * s : x * w.x - y * s;
}

// acc = A (one row block: 8 operand floats of this lane) * B (8 chunks)
__device__ __forceinline__ f4 prod8(const float DSBT_GLOBAL* a, const float* b) {
    const f4 a0 = *reinterpret_cast<const f4 DSBT_GLOBAL*>(a);
    const f4 a1 = *reinterpret_cast<const f4 DSBT_GLOBAL*>(a + 4);
    f4 c0 = f4{0.0f, 0.0f, 0.0f, 0.0f}, c1 = c0;
#pragma unroll
    for (int kc = 0; kc < 4; kc += 2) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[kc], b[kc], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[kc + 1], b[kc + 1], c1, 0, 0, 0);
    }
#pragma unroll
    for (int kc = 0; kc < 4; kc += 2) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[kc], b[4 + kc], c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[kc + 1], b[4 + kc + 1], c1, 0, 0, 0);
    }
    return c0 + c1;
}

template <bool INV, bool KPH>
__global__ void __launch_bounds__(256) mstage_fix(const FixItem* __restrict__ items, float2* data, PhaseArgs ph) {
    const FixItem& it = items[blockIdx.x];
    if (it.nch == 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, q = lane >> 4, col = lane & 15;
    float DSBT_GLOBAL* d = as_global_rw(reinterpret_cast<float*>(data));
    const float DSBT_GLOBAL* g = as_global(it.g);
    const f2 DSBT_GLOBAL* kph = as_global(reinterpret_cast<const f2*>(it.kphase));
    const bool cj = ph.conj != 0;
    const int NCB = it.NCB;
    // mu_H in the B-operand layout, per column block (at most 2)
    float mb[2][8];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int kc = 0; kc < 8; ++kc)
            mb[cb][kc] = cb < NCB ? it.mu_h[(cb * 32 + 4 * kc + q) * 16 + col] : 0.0f;
    for (int t = wave; t < it.NTF; t += 4) {
        const int J = it.J0 + t;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const float DSBT_GLOBAL* a = g + (((size_t)t * 2 + rb) * 64 + lane) * 8;
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                if (cb >= NCB) continue;
                const f4 c = prod8(a, mb[cb]);
                const int ch = cb * 8 + (col >> 1);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int slot = 16 * rb + 4 * q + v;
                    float x = c[v];
                    if constexpr (KPH) x = lane_cmul(x, kph[J * 32 + slot], col & 1, cj);
                    if (ch < it.nch) {
                        const int64_t e = 2 * (it.off[ch] + (int64_t)J * 32 + slot) + (col & 1);
                        d[e] += x;
                    }
                }
            }
        }
    }
    if (!INV && wave == 0) {
        // completion rows (-1)^p (mu_NT^0 + Phi mu_H) into slots 0..k-1 of tile 0
        const float sgn = it.p ? -1.0f : 1.0f;
        const float DSBT_GLOBAL* phi = as_global(it.phi);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                if (cb >= NCB) continue;
                const f4 c = prod8(phi + ((size_t)rb * 64 + lane) * 8, mb[cb]);
                const int ch = cb * 8 + (col >> 1);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rb + 4 * q + v;
                    float x = sgn * (c[v] + it.mu_end[(cb * 32 + row) * 16 + col]);
                    if constexpr (KPH) x = lane_cmul(x, kph[row], col & 1, cj);
                    if (ch < it.nch && row < it.k) d[2 * it.off[ch] + 2 * row + (col & 1)] = x;
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_mstage_fix(const FixItem* d_items, int nitems, void* data, bool inverse, PhaseArgs ph,
                             hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (inverse && ph.use) return hipErrorInvalidValue;
    float2* x = (float2*)data;
    if (inverse)
        hipLaunchKernelGGL((mstage_fix<true, false>), dim3(nitems), dim3(256), 0, s, d_items, x, ph);
    else if (ph.use)
        hipLaunchKernelGGL((mstage_fix<false, true>), dim3(nitems), dim3(256), 0, s, d_items, x, ph);
    else
        hipLaunchKernelGGL((mstage_fix<false, false>), dim3(nitems), dim3(256), 0, s, d_items, x, ph);
    return hipGetLastError();
}

}  // namespace dsbt
