// Device-side descriptors and launchers of the DSBT kernels (internal header).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dsbt {

constexpr int kBlock = 256;          // threads per workgroup of every transform kernel
constexpr int kMaxChanPerItem = 16;  // channels sharing one moment-table pass

// One channel of the sine/cosine stage (Sec. 2.2, eq. csFourierBasis).
//
// An FP32 unit number has a modulus 1 + O(eps) with a fixed sign per entry,
// and repeated transforms of the same data would turn products by it into a
// norm drift.  So FP32 plans carry every unit factor (FFT roots, post-twiddles,
// phase factors) as hi = the nearest FP32 value and lo = the FP32 rounding of
// the rest, multiplied as z hi + z lo (mul_unit).  FP64 plans have no lo
// parts (the lo pointers are nullptr).
struct FChan {
    int64_t off;          // element offset of the channel in every data buffer
    int N, log2N;
    int p;                // 1: even l (DST-II), 0: odd l (DCT-II)
    float sign;           // (-1)^ceil(l/2), or +1 for the printed F
    const void* roots;    // (cos, sin) of 2 pi e/N, e < N/4, 16 bytes per entry: FP64 (c, s) or
                          // FP32 (c hi, s hi, c lo, s lo); the FFT passes form their twiddles from it
    const void* post;     // exp(-i pi t/(2N)), t < N
    const void* post_lo;  // FP32 plans: the lo parts of post
    const void* vphase;   // exp(-i V tau/2) per point (complex of the arithmetic precision), or nullptr
    const void* vphase_lo;// FP32 plans: the lo parts of vphase
    const double* vangle; // V tau/2 per point (FP64), or nullptr
};

// One work item of the moment stage: up to kMaxChanPerItem channels with the
// same (l, N) sharing one pass over the tiles.
struct MItem {
    const void* tab_f;     // NT blocks, A[q][r] = M_J[r][q]
    const void* tab_i;     // NT blocks, A[q][r] = M_J[q][r]
    const void* mf_f;      // MFMA operand layout of the forward blocks (FP32, or FP64 for FP64
                           // arithmetic on complex64 data), or nullptr
    const void* mf_i;      // MFMA operand layout of the inverse blocks
    const void* kphase;    // exp(-i K_n tau) per slot (complex of the arithmetic precision), or nullptr
    const void* kphase_lo; // FP32 plans: the lo parts of kphase (see FChan)
    int B, k, R, NT, p, nch;
    int NB;                // 16-row blocks of the padded block size R16 = 16 NB (1, 2, 4 or 8)
    int NCB;               // 8-channel column blocks of the item (mfma_ncb on the matrix-core path)
    int64_t off[kMaxChanPerItem];
};

// MFMA operand layout of one direction's blocks: for tile J, row block rb,
// float group g < NB (chunks kc = 4 g .. 4 g + 3) and lane l, the 4 consecutive
// floats A'[16 rb + l%16][4 kc + l/16] at ((J NB + rb) NB + g) 256 + 4 l, where
// A' is the zero-padded R16 x R16 block mapping the input vector (tile data,
// then moments) to the output vector (tile result, then next moments).  A
// 16-byte load of group g by the 64 lanes reads 1 KiB contiguous.  size:
// NT * R16 * R16 floats.
inline size_t mfma_table_floats(int NT, int NB) { return (size_t)NT * 256 * NB * NB; }

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
hipError_t set_lds_limits(size_t mstage_bytes);

// Pointers read from descriptor structs are generic (flat) to the compiler;
// flat loads also count against the LDS counter, so an LDS wait would drain
// them.  Kernels cast such pointers to the global address space.
#define DSBT_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const T DSBT_GLOBAL* as_global(const T* p) {
    return (const T DSBT_GLOBAL*)p;
}
template <typename T>
__device__ __forceinline__ T DSBT_GLOBAL* as_global_rw(T* p) {
    return (T DSBT_GLOBAL*)p;
}

// Workgroup barrier that orders LDS only.  __syncthreads() is a workgroup
// release fence on all memory, which makes every thread wait for its
// outstanding global loads (prefetches included) before the barrier; the
// kernels here only exchange data through LDS, so the fence is limited to it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// x c for a constant c = hi + lo (hi its FP32 rounding).  The product with hi
// alone scales every value by the same relative error hi/c - 1, which repeated
// transforms turn into a norm drift; so the rounding error of p = x hi is
// recovered exactly (e = fma(x, hi, -p)) and added back with x lo, leaving a
// result within about one rounding of x c.
__device__ __forceinline__ float mul_const(float x, float hi, float lo) {
#pragma clang fp contract(off)   // p must be the rounded product, and p + (...) a plain sum
    const float p = x * hi;
    const float e = __builtin_fmaf(x, hi, -p);
    return p + __builtin_fmaf(x, lo, e);
}

// z w for a unit number w = h + l carried as FP32 hi and lo parts (FChan):
// the small product z l first, then the two main products, each fused.
__device__ __forceinline__ float2 mul_unit(float2 z, float2 h, float2 l) {
    const float cx = __builtin_fmaf(z.x, l.x, -(z.y * l.y));
    const float cy = __builtin_fmaf(z.x, l.y, z.y * l.x);
    return make_float2(__builtin_fmaf(z.x, h.x, __builtin_fmaf(-z.y, h.y, cx)),
                       __builtin_fmaf(z.x, h.y, __builtin_fmaf(z.y, h.x, cy)));
}

// Launchers.  T = float (complex64 data) or double (complex128 data).

// Sine/cosine stage for channels that all have N points (compile-time FFT
// size); T arithmetic and table precision, S data precision.
template <typename T, typename S>
hipError_t launch_fstage_n(int N, const FChan* d_chans, int nch, const void* src, void* dst, bool inverse,
                           PhaseArgs ph, hipStream_t s);
// The sine/cosine stage over channels of every N in one launch: task b is
// `count` channels of size N starting at entry `first` of the channel list
// (count <= kMultiThreads / (N/8): one block of kMultiThreads threads, N/8
// per channel).  mode: 0 forward, 1 inverse, 2 inverse then forward (as
// launch_fstage_inv_fwd, data in place, mid as there).  lds:
// fstage_multi_lds maximised over the tasks' N.
constexpr int kMultiThreads = 1024;
struct FTask {
    int N, first, count;
};
template <typename T>
size_t fstage_multi_lds(int N);
template <typename T, typename S>
hipError_t launch_fstage_multi(const FTask* d_tasks, int ntasks, const FChan* d_chans, const void* src, void* dst,
                               void* mid, int mode, PhaseArgs ph, PhaseArgs ph2, size_t lds, hipStream_t s);

// One step's inverse stage followed by the next step's forward stage, in place
// on the channels' data (one launch, one pass over the data): F^T with the
// phases ph_inv on its output, then F with ph_fwd on its input.  mid: nullptr,
// or a data buffer that also receives the state between the two stages (what
// the inverse stage alone would store).
template <typename T, typename S>
hipError_t launch_fstage_inv_fwd(int N, const FChan* d_chans, int nch, void* data, void* mid, PhaseArgs ph_inv,
                                 PhaseArgs ph_fwd, hipStream_t s);
template <typename T>
hipError_t set_lds_limits_fstage_n();

// Generic moment stage: T arithmetic and table precision, S data precision
// (float/float, double/double, or double arithmetic on complex64 data).
template <typename T, typename S>
hipError_t launch_mstage(const MItem* d_items, int nitems, int maxR, const void* src, void* dst,
                         bool inverse, PhaseArgs ph, hipStream_t s);

// Moment stage on the matrix cores (FP32 data).  waves = 4 when every item
// has NB <= 4, else 8.  Every item has 8 NCB channel slots (off[]): slots past
// nch repeat a real channel, whose results they then write again unchanged.
// Phases (ph.use) are supported on the forward direction only.
// lds: bytes of dynamic LDS, mfma_lds_bytes_for() maximised over the items.
hipError_t launch_mstage_mfma(const MItem* d_items, int nitems, int waves, size_t lds, const void* src,
                              void* dst, bool inverse, PhaseArgs ph, hipStream_t s);
// Tile B that the matrix-core kernel is built for, given the padded block size
// 16 NB (NB = 4 or 8: B = 32 or 64; the rows past B + k are zero padding).
__host__ __device__ constexpr int mfma_tile_for(int NB) { return 8 * NB; }
// 8-channel column blocks per item: enough row x column blocks for the waves.
__host__ __device__ constexpr int mfma_ncb(int waves, int NB) { return NB * 2 <= waves ? 2 : 1; }
inline size_t mfma_lds_bytes_for(int NB, int NCB, int B) {
    return sizeof(float) * (size_t)(2 * NCB * 16 * NB * 16 + 2 * NCB * B * 16);
}
hipError_t set_lds_limits_mfma();
// Moment stage for items with NB = 4 (B = 32, k <= 32) as a four-wave pipeline
// per item (Q x, moment chain, two result row blocks); 256 threads.  T = float
// (FP32 tables and arithmetic, complex64 data) or double (FP64 tables and
// arithmetic, items of one column block, complex64 or complex128 data).  An item has NCB = 1 or 2 blocks of
// 8 channels (off[]: slots past nch repeat a real channel); ncb is the largest
// NCB of the launched items and sizes the LDS.  Runs in place.  Phases
// (ph.use, complex of T per slot) are supported on the inverse direction only,
// where they multiply the input (the other moment kernels apply them to the
// forward's output: the kinetic factor of a split step sits between the two).
// D: data scalar in memory, float (complex64) or, with T = double, double
// (complex128).
template <typename T, typename D>
hipError_t launch_mstage_chain(const MItem* d_items, int nitems, int ncb, const void* src, void* dst, bool inverse,
                               PhaseArgs ph, hipStream_t s);
template <typename T>
hipError_t set_lds_limits_chain();
template <typename T>
size_t chain_lds_bytes(int ncb);

// *flag = 1 if any value of the channels' data is a NaN or an infinity
// (checked plans); the flag is cleared first by the same launcher.  One
// workgroup per channel; plain stores of 1, no atomics.  S: data scalar.
template <typename S>
hipError_t launch_scan_nonfinite(const FChan* d_chans, int nch, const void* data, int* flag, hipStream_t s);

// Partial sums of sum_i vangle_i Im(conj(l1) p1 + conj(l0) p0) per channel into
// scratch[nch], then out[0] = their sum (FP64).
template <typename T>
hipError_t launch_grad_s(const FChan* d_chans, int nch, const void* p0, const void* p1,
                         const void* l0, const void* l1, double* scratch, double* out,
                         hipStream_t s);
// The same for steps t = 0 .. nsteps - 1 in two launches: step t reads
// p_t = states + t stride, p_t+1, l_t = lams + t stride, l_t+1 (stride in
// complex elements) and writes out[t]; scratch holds nsteps nch partials.
// Each out[t] is bitwise what launch_grad_s gives for the same vectors.
template <typename T>
hipError_t launch_grad_s_steps(const FChan* d_chans, int nch, int nsteps, const void* states, const void* lams,
                               int64_t stride, double* scratch, double* out, hipStream_t s);

}  // namespace dsbt
