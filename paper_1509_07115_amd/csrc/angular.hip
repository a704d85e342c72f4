// Axis contractions of the angular transform (Sec. 4.1): one small dense matrix
// (the azimuthal DFT, or the per-m associated Legendre block) applied along one
// grid axis for every radial point; radius is the fastest axis of both layouts,
// so every load and store is coalesced along it.
//  * axis_mfma (complex64) and axis_mfma64 (complex128): the contraction as a
//    real product on the matrix cores, for matrices up to 64 x 64 in real form
//    (every Legendre block; the DFT while 2 N_phi <= 64).
//  * axis_mfma_big: the complex64 DFT for 64 < 2 N_phi <= 128, matrix in LDS.
//  * axis_apply: the vector kernel for the larger complex128 DFT.  A workgroup
//    takes one outer index and 64 consecutive radial points: their Q input
//    vectors and the Q x Q matrix are staged in LDS, and each of the four waves
//    accumulates every fourth output row for its 64 points, reading the matrix
//    as LDS broadcasts (one element per row and input, the same for the whole
//    wave).
// grid_phase and momentum_order are the diagonal factors and the reordering
// of the 3D split steps.
#include <algorithm>
#include <atomic>

#include "angular.h"

namespace dsbt {

namespace {

template <typename S> struct Cx;
template <> struct Cx<float> { typedef float2 t; };
template <> struct Cx<double> { typedef double2 t; };

constexpr int kRows = kShtMaxQ / 4;   // output rows per thread

// LDS bytes of one workgroup: 64 points x Q4 inputs and the Q x Q4 matrix, Q4 =
// Q rounded up to 4 (zero-padded), so that a wave reads four matrix columns as
// one 16-byte (real) or two (complex) broadcasts
__host__ __device__ constexpr int round4(int q) { return (q + 3) & ~3; }
template <typename S, bool CA>
constexpr size_t axis_lds_bytes(int Q) {
    return sizeof(typename Cx<S>::t) * 64 * (size_t)round4(Q) + sizeof(S) * (CA ? 2 : 1) * (size_t)Q * round4(Q);
}

template <typename S, bool CA>
__global__ void __launch_bounds__(256) axis_apply(const S* __restrict__ mat, int64_t mso, int tr, int cj,
                                                  const typename Cx<S>::t* __restrict__ src, int64_t so, int64_t sq,
                                                  typename Cx<S>::t* __restrict__ dst, int64_t dout, int64_t dq,
                                                  int Q, int Nr) {
    using V = typename Cx<S>::t;
    constexpr int AW = CA ? 2 : 1;   // scalars per matrix element
    const int Q4 = round4(Q);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    V* X = reinterpret_cast<V*>(lds_raw);                       // X[q * 64 + point], q < Q4
    S* A = reinterpret_cast<S*>(lds_raw + sizeof(V) * 64 * Q4);  // A[(q' Q4 + q) AW], untransposed, q < Q4
    const int o = blockIdx.y;
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave index (uniform)
    const bool live = i < Nr;
    // Staging: every lane issues its loads from addresses clamped into the rows,
    // points and matrix elements that exist, with no branch, and zeroes the rest
    // when it writes LDS; a load under a branch would be waited for inside it,
    // one round trip after another.
    {
        const int ic = min(i, Nr - 1);
        V xin[kShtMaxQ / 4];
#pragma unroll
        for (int u = 0; u < kShtMaxQ / 4; ++u) xin[u] = src[o * so + min(r + 4 * u, Q - 1) * sq + ic];
        constexpr int kMatPerThread = kShtMaxQ * kShtMaxQ / 256;
        const S* Ag = mat + o * mso;
        S av[kMatPerThread][AW];
#pragma unroll
        for (int u = 0; u < kMatPerThread; ++u) {
            const int e = min((int)threadIdx.x + 256 * u, Q * Q4 - 1);
            const int qo = e / Q4, q = min(e - qo * Q4, Q - 1);
            const int64_t g = tr ? (int64_t)q * Q + qo : (int64_t)qo * Q + q;
#pragma unroll
            for (int c = 0; c < AW; ++c) av[u][c] = Ag[AW * g + c];
        }
#pragma unroll
        for (int u = 0; u < kShtMaxQ / 4; ++u) {
            const int q = r + 4 * u;
            if (q < Q4) X[q * 64 + (threadIdx.x & 63)] = (live && q < Q) ? xin[u] : V{0, 0};
        }
#pragma unroll
        for (int u = 0; u < kMatPerThread; ++u) {
            const int e = threadIdx.x + 256 * u;
            if (e < Q * Q4) {
                const int qo = e / Q4, q = e - qo * Q4;
                if constexpr (CA) {
                    A[2 * e] = q < Q ? av[u][0] : S(0);
                    A[2 * e + 1] = q < Q ? (cj ? -av[u][1] : av[u][1]) : S(0);
                } else {
                    A[e] = q < Q ? av[u][0] : S(0);
                }
            }
        }
    }
    __syncthreads();
    V acc[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) acc[u] = V{0, 0};
    for (int q = 0; q < Q4; q += 4) {
        V x[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = X[(q + c) * 64 + (threadIdx.x & 63)];
#pragma unroll
        for (int u = 0; u < kRows; ++u) {
            const int qo = r + 4 * u;
            if (qo < Q) {
                const S* a = A + ((size_t)qo * Q4 + q) * AW;
                if constexpr (CA) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const S ar = a[2 * c], ai = a[2 * c + 1];
                        acc[u].x += ar * x[c].x - ai * x[c].y;
                        acc[u].y += ar * x[c].y + ai * x[c].x;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        acc[u].x += a[c] * x[c].x;
                        acc[u].y += a[c] * x[c].y;
                    }
                }
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
        const int qo = r + 4 * u;
        if (qo < Q) dst[o * dout + qo * dq + i] = acc[u];
    }
}

// Axis step on the matrix cores, complex64 data, as one real FP32 product
// D = A X of (Q16 x Q16) x (Q16 x NCOL) per block of 64 radial points,
// Q16 = 16 NR:
//  * real matrix (the per-m Legendre blocks): it acts on real and imaginary
//    parts alike, so the 64 points are NCOL = 128 real columns (2 i + part)
//    and the contraction index is q;
//  * complex matrix (the azimuthal DFT): the contraction index is k = 2 q + part
//    and the output row 2 q' + part', with A = [[Re, -Im], [Im, Re]] per element,
//    so the 64 points are NCOL = 64 columns.
// Workgroup (x, o) takes the point blocks x, x + gridDim.x, ... of outer index
// o: its matrix is loaded once (into registers, or for the real form into LDS),
// and the inputs of the next block are loaded into registers while the current
// one is multiplied and stored, so that memory and matrix work overlap inside
// the workgroup.  The
// inputs are staged transposed in LDS (Xt[column][k], row pitch Q16 + 4 floats,
// so that the 16-byte reads of 16 lanes cover all 64 banks once); wave w takes
// NCOL / 4 columns and every row block.  v_mfma_f32_16x16x4_f32: lane l
// supplies A[l%16][l/16] and B[l/16][l%16], result register v of lane l is
// D[4 (l/16) + v][l%16].  The contraction index is split as
// k = 16 G + 4 (l/16) + s for instruction s of group G, so that each lane holds
// the four k of its four instructions as one 16-byte word, of the zero-padded
// matrix (row-major [Q16][Q16] at mat16 + o mso in global memory; As, pitch XS,
// for the real form) and of Xt.
// Results pass through LDS (over Xt, row pitch NCOL + 4 floats: conflict-free)
// and are written back coalesced.
typedef float f4v __attribute__((ext_vector_type(4)));

template <int NR, bool CPX>
__global__ void __launch_bounds__(256) axis_mfma(const float* __restrict__ mat16, int64_t mso,
                                                 const float2* __restrict__ src, int64_t so, int64_t sq,
                                                 float2* __restrict__ dst, int64_t dout, int64_t dq, int Q, int Nr) {
    constexpr int Q16 = 16 * NR, XS = Q16 + 4;
    constexpr int NCOL = CPX ? 64 : 128, NCB = NCOL / 64, YP = NCOL + 4;
    constexpr int NPF = CPX ? 2 : 4;   // input rows per staging item
    static_assert(Q16 * YP <= NCOL * XS, "result staging must fit in the input buffer");
    __shared__ __align__(16) float Xt[NCOL * XS];
    const int o = blockIdx.y;
    const int nblk = (Nr + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float2* sp = src + o * so;
    float2* dp = dst + o * dout;
    // the matrix fragments: the complex form (at most 64 x 64, shared by every
    // outer index) in registers for the whole workgroup; the real per-m block
    // staged once in LDS (As[row][k], pitch XS), which leaves registers for a
    // third workgroup per compute unit
    f4v a[CPX ? NR : 1][NR];   // [G][rb]
    __shared__ __align__(16) float As[CPX ? 4 : Q16 * XS];
    if constexpr (CPX) {
        const float* Am = mat16 + o * mso + (lane & 15) * Q16 + 4 * (lane >> 4);
#pragma unroll
        for (int G = 0; G < NR; ++G)
#pragma unroll
            for (int rb = 0; rb < NR; ++rb) a[G][rb] = *reinterpret_cast<const f4v*>(Am + 16 * rb * Q16 + 16 * G);
        // have them in registers here: a first use inside the block loop would
        // put a wait on every memory operation in flight into each iteration
#pragma unroll
        for (int G = 0; G < NR; ++G)
#pragma unroll
            for (int rb = 0; rb < NR; ++rb) asm volatile("" ::"v"(a[G][rb]));
    } else {
        for (int e = threadIdx.x; e < Q16 * Q16 / 4; e += 256) {
            const int r = e / (Q16 / 4), k4 = e - r * (Q16 / 4);
            *reinterpret_cast<f4v*>(As + r * XS + 4 * k4) =
                *reinterpret_cast<const f4v*>(mat16 + o * mso + r * Q16 + 4 * k4);
        }
    }
    // staging item (g, il) = threadIdx.x + 256 u holds the contraction indices
    // 4 g .. 4 g + 3 of point il: input rows 2 g, 2 g + 1 (complex matrix) or
    // 4 g .. 4 g + 3 (real matrix)
    float2 pf[NR][NPF];
    // Every lane loads from an address clamped into the rows and points that
    // exist, with no branch, and the values outside are zeroed only when they
    // are staged: a load under a branch, or a value selected right after its
    // load, would be waited for at once, and the loads of the next block are
    // meant to stay in flight while the current one is multiplied.  Past the
    // last block every lane reads the same clamped element.
    auto fetch = [&](int bx) {
        const int ic = min(bx * 64 + (threadIdx.x & 63), Nr - 1);
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int g = (threadIdx.x + 256 * u) >> 6;
#pragma unroll
            for (int c = 0; c < NPF; ++c) pf[u][c] = sp[min(NPF * g + c, Q - 1) * sq + ic];
        }
    };
    int bx = blockIdx.x;
    fetch(bx);
    for (; bx < nblk; bx += gridDim.x) {
        const bool live = bx * 64 + (threadIdx.x & 63) < Nr;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int e = threadIdx.x + 256 * u, il = e & 63, g = e >> 6;
            float2 v[NPF];
#pragma unroll
            for (int c = 0; c < NPF; ++c) v[c] = (live && NPF * g + c < Q) ? pf[u][c] : float2{0.f, 0.f};
            if constexpr (CPX) {
                *reinterpret_cast<f4v*>(Xt + il * XS + 4 * g) = f4v{v[0].x, v[0].y, v[1].x, v[1].y};
            } else {
                *reinterpret_cast<f4v*>(Xt + (2 * il) * XS + 4 * g) = f4v{v[0].x, v[1].x, v[2].x, v[3].x};
                *reinterpret_cast<f4v*>(Xt + (2 * il + 1) * XS + 4 * g) = f4v{v[0].y, v[1].y, v[2].y, v[3].y};
            }
        }
        __syncthreads();
        fetch(bx + gridDim.x);
        f4v acc[NR][NCB];
#pragma unroll
        for (int rb = 0; rb < NR; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int G = 0; G < NR; ++G) {
            f4v ag[NR];
#pragma unroll
            for (int rb = 0; rb < NR; ++rb) {
                if constexpr (CPX)
                    ag[rb] = a[G][rb];
                else
                    ag[rb] = *reinterpret_cast<const f4v*>(As + (16 * rb + (lane & 15)) * XS + 16 * G + 4 * (lane >> 4));
            }
            f4v b[NCB];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                b[cb] = *reinterpret_cast<const f4v*>(Xt + (16 * (NCB * w + cb) + (lane & 15)) * XS + 16 * G +
                                                      4 * (lane >> 4));
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int rb = 0; rb < NR; ++rb)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        acc[rb][cb] =
                            __builtin_amdgcn_mfma_f32_16x16x4f32(ag[rb][s], b[cb][s], acc[rb][cb], 0, 0, 0);
        }
        __syncthreads();
        float* Ys = Xt;   // Ys[row][column], pitch YP
#pragma unroll
        for (int rb = 0; rb < NR; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    Ys[(16 * rb + 4 * (lane >> 4) + v) * YP + 16 * (NCB * w + cb) + (lane & 15)] = acc[rb][cb][v];
        __syncthreads();
        const int i0 = bx * 64;
        for (int e = threadIdx.x; e < Q * 64; e += 256) {
            const int t = e >> 6, il = e & 63;
            if (i0 + il >= Nr) continue;
            if constexpr (CPX)
                dp[t * dq + i0 + il] = float2{Ys[(2 * t) * YP + il], Ys[(2 * t + 1) * YP + il]};
            else
                dp[t * dq + i0 + il] = *reinterpret_cast<const float2*>(Ys + t * YP + 2 * il);
        }
        __syncthreads();
    }
}

// The complex64 azimuthal DFT for 64 < 2 N_phi <= 128 on the matrix cores: the
// real form of axis_mfma<NR, true> with NR = 5..8 row blocks, whose matrix does
// not fit in registers: it is staged once per workgroup in LDS (As[row][k],
// pitch Q16 + 4 like Xt, so the 16-byte fragment reads of 16 lanes cover all
// banks once), with the results in a third LDS buffer (Ys, pitch 68).  Dynamic
// LDS: (64 + Q16) (Q16 + 4) + 68 Q16 floats.
__host__ __device__ constexpr size_t axis_big_lds_bytes(int NR) {
    return sizeof(float) * ((size_t)(64 + 16 * NR) * (16 * NR + 4) + (size_t)68 * 16 * NR);
}

template <int NR>
__global__ void __launch_bounds__(256) axis_mfma_big(const float* __restrict__ mat16,
                                                     const float2* __restrict__ src, int64_t so, int64_t sq,
                                                     float2* __restrict__ dst, int64_t dout, int64_t dq, int Q,
                                                     int Nr) {
    constexpr int Q16 = 16 * NR, XS = Q16 + 4, YP = 68;
    extern __shared__ __align__(16) unsigned char lds_big[];
    float* Xt = reinterpret_cast<float*>(lds_big);   // Xt[point][k], 64 x XS
    float* As = Xt + 64 * XS;                         // As[row][k], Q16 x XS
    float* Ys = As + Q16 * XS;                        // Ys[row][point], Q16 x YP
    const int o = blockIdx.y;
    const int nblk = (Nr + 63) / 64;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float2* sp = src + o * so;
    float2* dp = dst + o * dout;
    for (int e = threadIdx.x; e < Q16 * Q16 / 4; e += 256) {
        const int r = e / (Q16 / 4), k4 = e - r * (Q16 / 4);
        *reinterpret_cast<f4v*>(As + r * XS + 4 * k4) = *reinterpret_cast<const f4v*>(mat16 + r * Q16 + 4 * k4);
    }
    // staging item (g, il) = threadIdx.x + 256 u: input rows 2 g, 2 g + 1 of point
    // il; loads from clamped addresses with no branch, zeroed when staged
    float2 pf[NR][2];
    auto fetch = [&](int bx) {
        const int ic = min(bx * 64 + (threadIdx.x & 63), Nr - 1);
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int g = (threadIdx.x + 256 * u) >> 6;
#pragma unroll
            for (int c = 0; c < 2; ++c) pf[u][c] = sp[min(2 * g + c, Q - 1) * sq + ic];
        }
    };
    int bx = blockIdx.x;
    fetch(bx);
    for (; bx < nblk; bx += gridDim.x) {
        const bool live = bx * 64 + (threadIdx.x & 63) < Nr;
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int e = threadIdx.x + 256 * u, il = e & 63, g = e >> 6;
            const float2 v0 = (live && 2 * g < Q) ? pf[u][0] : float2{0.f, 0.f};
            const float2 v1 = (live && 2 * g + 1 < Q) ? pf[u][1] : float2{0.f, 0.f};
            *reinterpret_cast<f4v*>(Xt + il * XS + 4 * g) = f4v{v0.x, v0.y, v1.x, v1.y};
        }
        __syncthreads();
        fetch(bx + gridDim.x);
        f4v acc[NR];
#pragma unroll
        for (int rb = 0; rb < NR; ++rb) acc[rb] = f4v{0.f, 0.f, 0.f, 0.f};
        const int kl = 4 * (lane >> 4);
#pragma unroll
        for (int G = 0; G < NR; ++G) {
            const f4v b = *reinterpret_cast<const f4v*>(Xt + (16 * w + (lane & 15)) * XS + 16 * G + kl);
            f4v a[NR];
#pragma unroll
            for (int rb = 0; rb < NR; ++rb)
                a[rb] = *reinterpret_cast<const f4v*>(As + (16 * rb + (lane & 15)) * XS + 16 * G + kl);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int rb = 0; rb < NR; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[rb][s], b[s], acc[rb], 0, 0, 0);
        }
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < NR; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Ys[(16 * rb + 4 * (lane >> 4) + v) * YP + 16 * w + (lane & 15)] = acc[rb][v];
        __syncthreads();
        const int i0 = bx * 64;
        for (int e = threadIdx.x; e < Q * 64; e += 256) {
            const int t = e >> 6, il = e & 63;
            if (i0 + il < Nr) dp[t * dq + i0 + il] = float2{Ys[(2 * t) * YP + il], Ys[(2 * t + 1) * YP + il]};
        }
        __syncthreads();
    }
}

// The axis steps for complex128 data on the FP64 matrix cores, in the forms of
// axis_mfma: the real per-m Legendre block on 32 radial points per block (64
// real columns 2 i + part), or the azimuthal DFT in its real form
// [[Re, -Im], [Im, Re]] (contraction index 2 q + part) on 64 points per block;
// either way 64 columns, wave w taking columns 16 w .. 16 w + 15.
// v_mfma_f64_16x16x4_f64 takes the operands of the FP32 form (lane l:
// A[l%16][l/16], B[l/16][l%16]) and returns row 4 v + l/16, column l%16 in
// result register v.  The contraction index is split as k = 16 G + 4 (l/16) + s,
// so that each lane holds the four k of its four instructions in 32 contiguous
// bytes of the matrix (registers, loaded once) and of the transposed LDS copy
// Xt[column][k] (pitch Q16 + 2).  Workgroups loop over point blocks of one
// outer index with the next block's loads issued, from clamped addresses with
// no branch, before the current one is multiplied.
typedef double d4v __attribute__((ext_vector_type(4)));

template <int NR, bool CPX>
__global__ void __launch_bounds__(256) axis_mfma64(const double* __restrict__ mat16, int64_t mso,
                                                   const double2* __restrict__ src, int64_t so, int64_t sq,
                                                   double2* __restrict__ dst, int64_t dout, int64_t dq, int Q,
                                                   int Nr) {
    constexpr int Q16 = 16 * NR, XS = Q16 + 2, NCOL = 64, YP = NCOL + 2, PB = CPX ? 64 : 32;
    constexpr int NIT = 2 * NR;   // staging items per thread: (input row, point)
    static_assert(Q16 * YP <= NCOL * XS, "result staging must fit in the input buffer");
    __shared__ __align__(16) double Xt[NCOL * XS];
    const int o = blockIdx.y;
    const int nblk = (Nr + PB - 1) / PB;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double2* sp = src + o * so;
    double2* dp = dst + o * dout;
    d4v a[NR][NR];   // [G][rb]: A[16 rb + l%16][16 G + 4 (l/16) + s]
    {
        const double* Am = mat16 + o * mso + (lane & 15) * Q16 + 4 * (lane >> 4);
#pragma unroll
        for (int G = 0; G < NR; ++G)
#pragma unroll
            for (int rb = 0; rb < NR; ++rb) {
                const double2 lo = *reinterpret_cast<const double2*>(Am + 16 * rb * Q16 + 16 * G);
                const double2 hi = *reinterpret_cast<const double2*>(Am + 16 * rb * Q16 + 16 * G + 2);
                a[G][rb] = d4v{lo.x, lo.y, hi.x, hi.y};
            }
        // have them in registers here: a first use inside the block loop would
        // put a wait on every memory operation in flight into each iteration
#pragma unroll
        for (int G = 0; G < NR; ++G)
#pragma unroll
            for (int rb = 0; rb < NR; ++rb) {
                // two 16-byte halves: a 32-byte operand here drops the kernel's host stub
                const d4v t = a[G][rb];
                asm volatile("" ::"v"(t.lo), "v"(t.hi));
            }
    }
    double2 pf[NIT];   // item e = threadIdx.x + 256 u: input row e / PB, point e % PB
    auto fetch = [&](int bx) {
#pragma unroll
        for (int u = 0; u < NIT; ++u) {
            const int e = threadIdx.x + 256 * u;
            pf[u] = sp[min(e / PB, Q - 1) * sq + min(bx * PB + e % PB, Nr - 1)];
        }
    };
    int bx = blockIdx.x;
    fetch(bx);
    for (; bx < nblk; bx += gridDim.x) {
        const int i0 = bx * PB;
#pragma unroll
        for (int u = 0; u < NIT; ++u) {
            const int e = threadIdx.x + 256 * u, q = e / PB, il = e % PB;
            const double2 v = (q < Q && i0 + il < Nr) ? pf[u] : double2{0.0, 0.0};
            if constexpr (CPX) {
                *reinterpret_cast<double2*>(Xt + il * XS + 2 * q) = v;
            } else {
                Xt[(2 * il) * XS + q] = v.x;
                Xt[(2 * il + 1) * XS + q] = v.y;
            }
        }
        __syncthreads();
        fetch(bx + gridDim.x);
        d4v acc[NR];
#pragma unroll
        for (int rb = 0; rb < NR; ++rb) acc[rb] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int G = 0; G < NR; ++G) {
            const double* xb = Xt + (16 * w + (lane & 15)) * XS + 16 * G + 4 * (lane >> 4);
            const double2 lo = *reinterpret_cast<const double2*>(xb);
            const double2 hi = *reinterpret_cast<const double2*>(xb + 2);
            const double b[4] = {lo.x, lo.y, hi.x, hi.y};
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int rb = 0; rb < NR; ++rb)
                    acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[G][rb][s], b[s], acc[rb], 0, 0, 0);
        }
        __syncthreads();
        double* Ys = Xt;   // Ys[row][column], pitch YP
#pragma unroll
        for (int rb = 0; rb < NR; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) Ys[(16 * rb + 4 * v + (lane >> 4)) * YP + 16 * w + (lane & 15)] = acc[rb][v];
        __syncthreads();
        for (int e = threadIdx.x; e < Q * PB; e += 256) {
            const int t = e / PB, il = e % PB;
            if (i0 + il >= Nr) continue;
            if constexpr (CPX)
                dp[t * dq + i0 + il] = double2{Ys[(2 * t) * YP + il], Ys[(2 * t + 1) * YP + il]};
            else
                dp[t * dq + i0 + il] = double2{Ys[t * YP + 2 * il], Ys[t * YP + 2 * il + 1]};
        }
        __syncthreads();
    }
}

// x[i] *= exp(-i (V0[i] + F V1[i]) dt/2), the angle formed and reduced mod 2 pi
// in FP64 (V0 or V1 may be null: zero)
template <typename S>
__global__ void __launch_bounds__(256) grid_phase(typename Cx<S>::t* __restrict__ x, const double* __restrict__ V0,
                                                  const double* __restrict__ V1, double F, double half_dt,
                                                  int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double a = ((V0 ? V0[i] : 0.0) + (V1 ? F * V1[i] : 0.0)) * half_dt;
    const double twopi = 6.283185307179586476925286766559;
    a -= twopi * rint(a / twopi);
    S sn, cs;
    if constexpr (sizeof(S) == sizeof(float)) {
        sincosf((float)a, &sn, &cs);
    } else {
        sincos(a, &sn, &cs);
    }
    const typename Cx<S>::t z = x[i];
    x[i] = {z.x * cs + z.y * sn, z.y * cs - z.x * sn};
}

// Channel (q, t), l = |q - M| + t, of Nr slots: forward, out[u] = i^-l in[j(u)]
// with j(u) = (u + 1) mod Nr for odd l (the n = 0 slot moves to the top of the
// unified grid n = 1..Nr) and j(u) = u for even l; inverse, out[j] = i^l in[u(j)].
template <typename S>
__global__ void __launch_bounds__(256) momentum_order(const typename Cx<S>::t* __restrict__ src,
                                                      typename Cx<S>::t* __restrict__ dst, int nt, int M, int Nr,
                                                      int inverse) {
    const int c = blockIdx.y;
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= Nr) return;
    const int q = c / nt, t = c - q * nt;
    const int l = (q > M ? q - M : M - q) + t;
    int from = x;
    if (l & 1) from = inverse ? (x + Nr - 1) % Nr : (x + 1) % Nr;
    const typename Cx<S>::t z = src[(int64_t)c * Nr + from];
    // multiply by i^e, e = -l (forward) or l (inverse), e mod 4
    const int e = ((inverse ? l : -l) % 4 + 4) % 4;
    typename Cx<S>::t w;
    if (e == 0) w = z;
    else if (e == 1) w = {-z.y, z.x};
    else if (e == 2) w = {-z.x, -z.y};
    else w = {z.y, -z.x};
    dst[(int64_t)c * Nr + x] = w;
}

}  // namespace

template <typename S>
hipError_t launch_momentum_order(const void* src, void* dst, int nt, int nphi, int Nr, bool inverse, hipStream_t s) {
    hipLaunchKernelGGL(momentum_order<S>, dim3((unsigned)((Nr + 255) / 256), (unsigned)(nt * nphi)), dim3(256), 0, s,
                       (const typename Cx<S>::t*)src, (typename Cx<S>::t*)dst, nt, (nphi - 1) / 2, Nr,
                       inverse ? 1 : 0);
    return hipGetLastError();
}
template hipError_t launch_momentum_order<float>(const void*, void*, int, int, int, bool, hipStream_t);
template hipError_t launch_momentum_order<double>(const void*, void*, int, int, int, bool, hipStream_t);

template <typename S>
hipError_t launch_grid_phase(void* x, const double* V0, const double* V1, double F, double dt, int64_t n,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(grid_phase<S>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (typename Cx<S>::t*)x, V0, V1, F, 0.5 * dt, n);
    return hipGetLastError();
}
template hipError_t launch_grid_phase<float>(void*, const double*, const double*, double, double, int64_t,
                                             hipStream_t);
template hipError_t launch_grid_phase<double>(void*, const double*, const double*, double, double, int64_t,
                                              hipStream_t);

template <typename S, bool CA>
hipError_t launch_axis_apply(const S* mat, int64_t mso, bool tr, bool cj, const void* src, int64_t so, int64_t sq,
                             void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr, hipStream_t s) {
    using V = typename Cx<S>::t;
    if (Q < 1 || Q > kShtMaxQ || nouter < 1 || Nr < 1) return hipErrorInvalidValue;
    const size_t lds = axis_lds_bytes<S, CA>(Q);
    hipLaunchKernelGGL((axis_apply<S, CA>), dim3((Nr + 63) / 64, nouter), dim3(256), lds, s, mat, mso, tr ? 1 : 0,
                       cj ? 1 : 0, (const V*)src, so, sq, (V*)dst, dout, dq, Q, Nr);
    return hipGetLastError();
}

// Workgroups of axis_mfma<nr, CPX> resident on the device at once, queried on
// the first call (set_lds_limits_axis makes that call before any launch, so
// that no query falls inside a stream capture); -1 if the query fails.
template <bool CPX>
static int axis_mfma_fit(int nr) {
    static std::atomic<int> fit[4] = {{0}, {0}, {0}, {0}};
    if (nr < 1 || nr > 4) return -1;
    int f = fit[nr - 1].load(std::memory_order_relaxed);
    if (f > 0) return f;
    const void* k = nr == 1   ? (const void*)axis_mfma<1, CPX>
                    : nr == 2 ? (const void*)axis_mfma<2, CPX>
                    : nr == 3 ? (const void*)axis_mfma<3, CPX>
                              : (const void*)axis_mfma<4, CPX>;
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, 256, 0) != hipSuccess)
        return -1;
    f = std::max(1, occ) * std::max(1, ncu);
    fit[nr - 1].store(f, std::memory_order_relaxed);
    return f;
}

// Workgroups of axis_mfma_big<nr> (nr = 5..8) resident on the device at once,
// with its dynamic LDS (queried once, first from set_lds_limits_axis); -1 if
// the query fails.
static int axis_big_fit(int nr) {
    static std::atomic<int> fit[4] = {{0}, {0}, {0}, {0}};
    if (nr < 5 || nr > 8) return -1;
    int f = fit[nr - 5].load(std::memory_order_relaxed);
    if (f > 0) return f;
    const void* k = nr == 5   ? (const void*)axis_mfma_big<5>
                    : nr == 6 ? (const void*)axis_mfma_big<6>
                    : nr == 7 ? (const void*)axis_mfma_big<7>
                              : (const void*)axis_mfma_big<8>;
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, 256, axis_big_lds_bytes(nr)) != hipSuccess)
        return -1;
    f = std::max(1, occ) * std::max(1, ncu);
    fit[nr - 5].store(f, std::memory_order_relaxed);
    return f;
}

template <bool CPX>
static hipError_t launch_axis_mfma_t(const float* mat16, int64_t mso, const void* src, int64_t so, int64_t sq,
                                     void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr, hipStream_t s) {
    const int nr = ((CPX ? 2 * Q : Q) + 15) / 16;
    if (Q < 1 || nr > (CPX ? 8 : 4) || nouter < 1 || Nr < 1) return hipErrorInvalidValue;
    if (CPX && nr > 4 && mso != 0) return hipErrorInvalidValue;   // the large form takes one shared matrix
    const int fit0 = nr > 4 ? axis_big_fit(nr) : axis_mfma_fit<CPX>(nr);
    if (fit0 < 0) return hipErrorInvalidValue;
    const int nblk = (Nr + 63) / 64;
    // as many workgroups as fit on the device at once (at least one per outer
    // index), each taking an equal share of the point blocks of its outer index
    const int fit = std::max(1, std::min(nblk, fit0 / nouter));
    const int per = (nblk + fit - 1) / fit;
    const dim3 grid((unsigned)((nblk + per - 1) / per), (unsigned)nouter);
    const float2* x = static_cast<const float2*>(src);
    float2* y = static_cast<float2*>(dst);
    if (nr > 4) {
        const size_t lds = axis_big_lds_bytes(nr);
        switch (nr) {
            case 5: hipLaunchKernelGGL(axis_mfma_big<5>, grid, dim3(256), lds, s, mat16, x, so, sq, y, dout, dq, Q, Nr); break;
            case 6: hipLaunchKernelGGL(axis_mfma_big<6>, grid, dim3(256), lds, s, mat16, x, so, sq, y, dout, dq, Q, Nr); break;
            case 7: hipLaunchKernelGGL(axis_mfma_big<7>, grid, dim3(256), lds, s, mat16, x, so, sq, y, dout, dq, Q, Nr); break;
            default: hipLaunchKernelGGL(axis_mfma_big<8>, grid, dim3(256), lds, s, mat16, x, so, sq, y, dout, dq, Q, Nr); break;
        }
        return hipGetLastError();
    }
    switch (nr) {
        case 1: hipLaunchKernelGGL((axis_mfma<1, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
        case 2: hipLaunchKernelGGL((axis_mfma<2, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
        case 3: hipLaunchKernelGGL((axis_mfma<3, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
        default: hipLaunchKernelGGL((axis_mfma<4, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
    }
    return hipGetLastError();
}

// Workgroups of axis_mfma64<nr, CPX> resident on the device at once (queried
// once, first from set_lds_limits_axis); -1 if the query fails.
template <bool CPX>
static int axis_mfma64_fit(int nr) {
    static std::atomic<int> fit[4] = {{0}, {0}, {0}, {0}};
    if (nr < 1 || nr > 4) return -1;
    int f = fit[nr - 1].load(std::memory_order_relaxed);
    if (f > 0) return f;
    const void* k = nr == 1   ? (const void*)axis_mfma64<1, CPX>
                    : nr == 2 ? (const void*)axis_mfma64<2, CPX>
                    : nr == 3 ? (const void*)axis_mfma64<3, CPX>
                              : (const void*)axis_mfma64<4, CPX>;
    int dev = 0, ncu = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, 256, 0) != hipSuccess)
        return -1;
    f = std::max(1, occ) * std::max(1, ncu);
    fit[nr - 1].store(f, std::memory_order_relaxed);
    return f;
}

template <bool CPX>
static hipError_t launch_axis_mfma64_t(const double* mat16, int64_t mso, const void* src, int64_t so, int64_t sq,
                                       void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr,
                                       hipStream_t s) {
    const int nr = ((CPX ? 2 * Q : Q) + 15) / 16;
    if (Q < 1 || nr > 4 || nouter < 1 || Nr < 1) return hipErrorInvalidValue;
    const int fit0 = axis_mfma64_fit<CPX>(nr);
    if (fit0 < 0) return hipErrorInvalidValue;
    const int pb = CPX ? 64 : 32;
    const int nblk = (Nr + pb - 1) / pb;
    const int fit = std::max(1, std::min(nblk, fit0 / nouter));
    const int per = (nblk + fit - 1) / fit;
    const dim3 grid((unsigned)((nblk + per - 1) / per), (unsigned)nouter);
    const double2* x = static_cast<const double2*>(src);
    double2* y = static_cast<double2*>(dst);
    switch (nr) {
        case 1: hipLaunchKernelGGL((axis_mfma64<1, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
        case 2: hipLaunchKernelGGL((axis_mfma64<2, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
        case 3: hipLaunchKernelGGL((axis_mfma64<3, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
        default: hipLaunchKernelGGL((axis_mfma64<4, CPX>), grid, dim3(256), 0, s, mat16, mso, x, so, sq, y, dout, dq, Q, Nr); break;
    }
    return hipGetLastError();
}

hipError_t launch_axis_mfma64(bool complex_matrix, const double* mat16, int64_t mso, const void* src, int64_t so,
                              int64_t sq, void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr,
                              hipStream_t s) {
    return complex_matrix ? launch_axis_mfma64_t<true>(mat16, mso, src, so, sq, dst, dout, dq, Q, nouter, Nr, s)
                          : launch_axis_mfma64_t<false>(mat16, mso, src, so, sq, dst, dout, dq, Q, nouter, Nr, s);
}

hipError_t launch_axis_mfma(bool complex_matrix, const float* mat16, int64_t mso, const void* src, int64_t so,
                            int64_t sq, void* dst, int64_t dout, int64_t dq, int Q, int nouter, int Nr,
                            hipStream_t s) {
    return complex_matrix ? launch_axis_mfma_t<true>(mat16, mso, src, so, sq, dst, dout, dq, Q, nouter, Nr, s)
                          : launch_axis_mfma_t<false>(mat16, mso, src, so, sq, dst, dout, dq, Q, nouter, Nr, s);
}

hipError_t set_lds_limits_axis() {
    {
        const void* big[4] = {(const void*)axis_mfma_big<5>, (const void*)axis_mfma_big<6>,
                              (const void*)axis_mfma_big<7>, (const void*)axis_mfma_big<8>};
        for (int i = 0; i < 4; ++i) {
            const hipError_t e = hipFuncSetAttribute(big[i], hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)axis_big_lds_bytes(5 + i));
            if (e != hipSuccess) return e;
            if (axis_big_fit(5 + i) < 0) return hipErrorInvalidDeviceFunction;
        }
    }
    for (int nr = 1; nr <= 4; ++nr)
        if (axis_mfma_fit<true>(nr) < 0 || axis_mfma_fit<false>(nr) < 0 ||
            axis_mfma64_fit<true>(nr) < 0 || axis_mfma64_fit<false>(nr) < 0)
            return hipErrorInvalidDeviceFunction;
    hipError_t e = hipFuncSetAttribute((const void*)axis_apply<float, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)axis_lds_bytes<float, true>(kShtMaxQ));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)axis_apply<float, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)axis_lds_bytes<float, false>(kShtMaxQ));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)axis_apply<double, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)axis_lds_bytes<double, true>(kShtMaxQ));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)axis_apply<double, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)axis_lds_bytes<double, false>(kShtMaxQ));
    return e;
}

template hipError_t launch_axis_apply<float, true>(const float*, int64_t, bool, bool, const void*, int64_t, int64_t,
                                                   void*, int64_t, int64_t, int, int, int, hipStream_t);
template hipError_t launch_axis_apply<float, false>(const float*, int64_t, bool, bool, const void*, int64_t, int64_t,
                                                    void*, int64_t, int64_t, int, int, int, hipStream_t);
template hipError_t launch_axis_apply<double, true>(const double*, int64_t, bool, bool, const void*, int64_t, int64_t,
                                                    void*, int64_t, int64_t, int, int, int, hipStream_t);
template hipError_t launch_axis_apply<double, false>(const double*, int64_t, bool, bool, const void*, int64_t,
                                                     int64_t, void*, int64_t, int64_t, int, int, int, hipStream_t);

}  // namespace dsbt
