// Moment stage for tiles of B = 32 on the CDNA4 matrix cores, as a pipeline
// of four waves per item: 8 NCB complex channels with the same l and N, in
// NCB = 1 or 2 blocks of 16 matrix columns.  Every table operand a lane loads
// feeds NCB matrix instructions.  The arithmetic type T is float (FP32 tables)
// or double (FP64 tables, NCB = 1); data in memory are complex64, or
// complex128 with FP64 arithmetic (D, the data scalar).
//
// Per tile J the tiled moment form (Sec. 2.4-2.5) maps [x_J; mu_J] to
// [o_J; mu_J+1] with the zero-padded 64 x 64 block A' (M_J forward, M_J^T
// inverse): rows/columns 0..31 are the tile slots, 32..63 the moments.  The
// only serial dependence is mu_J+1 = Q x_J + D mu_J, so the work of a tile is
// split by role:
//   pre wave     q_J = Q x_J = A'[32:64, 0:32] x_J -> LDS, with x_J read
//                from LDS in the operand layout at the start of its phase;
//   chain wave   mu_J+1 = q_J + A'[32:64, 32:64] mu_J, with mu kept in
//                registers: the FP32 result layout is turned into the operand
//                layout by two lane-swap stages (the FP64 one already is);
//                mu_J+1 -> LDS; it also stages the tile data, x_J+4 -> LDS
//                (contiguous 16-byte loads, natural layout), which keeps
//                that work off the pre wave, the role with the most matrix
//                instructions;
//   result waves o_J = A'[16 r : 16 r + 16, :] [x_J; mu_J], r = 0, 1, from
//                LDS, the two waves trading r from tile to tile so that both
//                carry the same matrix work; each 16 x 16 result block is
//                rearranged (FP32: between lane pairs; FP64: through LDS) so
//                that a lane stores two consecutive complex slots of one
//                channel (16 bytes); tile J - 1 is read out and stored while
//                tile J's matrix instructions run.
// The kinetic factors of a split step (Sec. 4.1) multiply the inverse's input
// where the chain wave stages it (and the completion slots it starts from),
// which keeps them off the result waves of the forward direction.
// The waves run one phase of kPhase tiles apart (pre, chain, results) and
// meet at one LDS barrier per phase.  All global reads of a tile happen two
// phases before any write of it, so the stage may run in place.  Global
// operands are prefetched kPD tiles ahead into kSets register sets, and each
// role's loop (kSets / kPhase phases per iteration) has no branch: tiles past
// NT exist only when NT < kSets, a separate instantiation.  So the compiler's
// memory-counter waits cover just the prefetch distance.
//
// v_mfma_f32_16x16x4_f32 layouts: lane l holds A[l%16][l/16] and
// B[l/16][l%16]; result register v of lane l is D[4 (l/16) + v][l%16]
// (v_mfma_f64_16x16x4_f64: the same operands, result row 4 v + l/16).  The 16
// columns of block cb are channels 8 cb .. 8 cb + 7 times (re, im).  Operands
// use the table layout of MItem::mf_f / mf_i with NB = 4 (per tile, row block
// rb and group g of 4 chunks, 64 lanes x the 4 values A'[16 rb + l%16][4 kc +
// l/16]).  Zero blocks are skipped: the in-tile band of T and the
// moment-to-moment block are triangular (lower forward, upper inverse), and
// moment columns past k = ceil(l/2) are padding (KB = ceil(k/16) chunks of 16).
#include "kernels.h"

namespace dsbt {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
// 16-byte global access of two complex64 values, which are 8-byte aligned
typedef float f4u __attribute__((ext_vector_type(4), aligned(8)));

// Data in memory: four scalars (two consecutive complex slots of a channel) per
// lane access, 8-byte aligned for complex64, 16-byte aligned for complex128.
template <typename D>
struct Data;
template <>
struct Data<float> {
    typedef float v4 __attribute__((ext_vector_type(4), aligned(8)));
};
template <>
struct Data<double> {
    typedef double v4 __attribute__((ext_vector_type(4), aligned(16)));
};

// Arithmetic precision of the pipeline: float (complex64 plans) or double
// (FP64 arithmetic and tables, complex64 or complex128 data).
template <typename T>
struct Arith;
template <>
struct Arith<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef float v2 __attribute__((ext_vector_type(2)));
    static __device__ v4 mfma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <>
struct Arith<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    typedef double v2 __attribute__((ext_vector_type(2)));
    static __device__ v4 mfma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};

constexpr int kPhase = 2;               // tiles per phase
constexpr int kPD = 3;                  // prefetch distance of the global operands, in tiles
constexpr int kSets = kPD + 1;          // register sets; set = tile mod kSets
constexpr int kRep = kSets / kPhase;    // phases per loop iteration
static_assert(kSets % kPhase == 0, "a loop iteration must cycle through the register sets exactly once");
// tile data: the pre wave writes tile t + 1 during step t, the result waves
// read a tile two phases after its phase; 3 kPhase + 1 slots live
constexpr int kXRing = 4 * kPhase;
constexpr int kQRing = 2 * kPhase;      // Q x: read one phase after it is written
constexpr int kMRing = 3 * kPhase;      // moments: 2 kPhase + 1 slots live
static_assert(kMRing >= 2 * kPhase + 1, "moment ring too small");
constexpr int kXCh = 68;                // values per channel of a data slot (32 complex + padding)
constexpr int kYCol = 20;               // result staging: values per column (16 rows + padding)

// LDS values (of the arithmetic type) of an item of ncb column blocks: data
// ring (natural layout), Q x and moment rings (8 values per lane and block),
// result staging of the two result waves
__host__ __device__ constexpr int chain_lds_values(int ncb) {
    return kXRing * 8 * ncb * kXCh + (kQRing + kMRing) * 64 * 8 * ncb + 2 * ncb * 16 * kYCol;
}

// Orders this wave's LDS accesses across a point (the hardware keeps one
// wave's LDS operations in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// (row 4 (l/16) + v, column l%16) in register v  ->  (row 4 j + l/16) in out[j]:
// a transpose of the 4 x 4 grid (lane quarter, register) of 32-bit words.  The
// 32-lane swap exchanges the high bits of the two indices, the 16-lane swap
// the low bits.
__device__ __forceinline__ void transpose_words(const unsigned* m, unsigned* out) {
    const auto a = __builtin_amdgcn_permlane32_swap(m[0], m[2], false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(m[1], m[3], false, false);
    const auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
    const auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
    out[0] = c[0];
    out[1] = c[1];
    out[2] = d[0];
    out[3] = d[1];
}
__device__ __forceinline__ void result_to_operand(Arith<float>::v4 m, float* out) {
    const unsigned w[4] = {__float_as_uint(m[0]), __float_as_uint(m[1]), __float_as_uint(m[2]), __float_as_uint(m[3])};
    unsigned o[4];
    transpose_words(w, o);
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = __uint_as_float(o[j]);
}
// v_mfma_f64_16x16x4_f64 returns row 4 v + l/16 in register v (measured on
// gfx950): its result is already in the operand layout
__device__ __forceinline__ void result_to_operand(Arith<double>::v4 m, double* out) {
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = m[j];
}

template <typename T, typename D, bool INV, bool KPH, int KB, bool TAIL, int NCB>
struct Pipe {
    using DV4 = typename Data<D>::v4;
    using V4 = typename Arith<T>::v4;
    using V2 = typename Arith<T>::v2;
    // chunk kc = A' columns 4 kc .. 4 kc + 3 (0..7 tile data, 8.. moments)
    static constexpr int MHI = 8 + 4 * KB;
    static constexpr int R0LO = 0, R0HI = INV ? 8 : 4;      // result rows 0..15, data chunks
    static constexpr int R1LO = INV ? 4 : 0, R1HI = 8;      // result rows 16..31
    static constexpr int C2LO = 8, C2HI = INV ? MHI : 12;   // moment rows 0..15, moment chunks
    static constexpr int C3LO = INV ? 12 : 8, C3HI = MHI;   // moment rows 16..31 (KB = 2)
    static constexpr int NC2 = (C2HI - C2LO) / 4, NC3 = KB == 2 ? (C3HI - C3LO) / 4 : 0;
    // values per Q x / moment slot: 4 values of moment rows 16 h + 4 (l/16) .. of
    // block cb for lane l at 256 (2 cb + h) + 4 l (lane-contiguous 16-byte accesses)
    static constexpr int SLOT = 64 * 8 * NCB;
    static constexpr int XSLOT = 8 * NCB * kXCh;            // values per data slot
    static constexpr int YWAVE = NCB * 16 * kYCol;          // result staging per result wave
    static constexpr int LPC = 8 / NCB, FPL = 8 * NCB;      // pre-wave loads: lanes per channel, floats per lane

    const D DSBT_GLOBAL* src;
    D DSBT_GLOBAL* dst;
    const T DSBT_GLOBAL* tab;
    const V2 DSBT_GLOBAL* kphase;   // complex of the arithmetic precision
    const V2 DSBT_GLOBAL* kphase_lo;   // FP32: lo parts of the kinetic factors (kernels.h)
    T* xring;
    T* qring;
    T* mring;
    T* yring;
    int NT, k, p, lane, q, col, nact;
    int64_t e0[NCB];   // scalar index of (channel 8 cb + col/2, slot 0, re/im col%2)
    // natural layout: the pre wave's lane l loads channel l/LPC, FPL floats
    // from slot 4 (l%LPC) NCB of a tile; a result wave's lane l stores slots
    // 2 (l%8), 2 (l%8) + 1 of channel 8 cb + l/8 in a 16-row block
    int64_t gpre;      // scalar index of the pre wave's first scalar in tile 0
    int64_t g0[NCB];   // scalar index of (channel 8 cb + l/8, slot 0)
    int xnat;          // offset of the pre wave's loaded values in a data slot
    int xop[NCB];      // offset of operand (slot l/16, column l%16 of block cb) in a data slot
    bool conj;

    __device__ Pipe(const MItem& it, const void* s_, void* d_, const PhaseArgs& ph, T* lds)
        : src(as_global(static_cast<const D*>(s_))), dst(as_global_rw(static_cast<D*>(d_))) {
        NT = it.NT;
        k = it.k;
        p = it.p;
        lane = threadIdx.x & 63;
        q = lane >> 4;
        col = lane & 15;
        conj = ph.conj != 0;
        tab = as_global(static_cast<const T*>(INV ? it.mf_i : it.mf_f));
        kphase = as_global(reinterpret_cast<const V2*>(it.kphase));
        kphase_lo = as_global(reinterpret_cast<const V2*>(it.kphase_lo));
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            e0[cb] = 2 * it.off[8 * cb + (col >> 1)] + (col & 1);
            g0[cb] = 2 * it.off[8 * cb + (lane >> 3)];
            xop[cb] = (8 * cb + (col >> 1)) * kXCh + 2 * q + (col & 1);
        }
        gpre = 2 * it.off[lane / LPC] + FPL * (lane % LPC);
        xnat = (lane / LPC) * kXCh + FPL * (lane % LPC);
        xring = lds;
        qring = lds + kXRing * XSLOT;
        mring = qring + kQRing * SLOT;
        yring = mring + kMRing * SLOT;
        nact = (NT + kPhase - 1) / kPhase;   // phases in which a role has tiles
    }

    __device__ int tile(int t) const {
        const int c = t < NT ? t : NT - 1;
        return INV ? NT - 1 - c : c;
    }
    // this lane's operand floats of chunks 4 g .. 4 g + 3, g = G .. G + N - 1, of
    // row block rb of tile J (each group: 64 lanes x 4 floats contiguous)
    template <int N>
    __device__ void seg(V4* o, int J, int rb, int G) const {
        const V4 DSBT_GLOBAL* s = reinterpret_cast<const V4 DSBT_GLOBAL*>(tab + (size_t)(J * 4 + rb) * 1024) + lane;
#pragma unroll
        for (int i = 0; i < N; ++i) o[i] = s[64 * (G + i)];
    }
    // for every block cb: acc[cb] += A[:, chunks LO..HI) B_cb, alternating two
    // accumulators; A chunk kc is value kc - LO of av, B_cb chunk kc is
    // bv[BS cb + kc - LO]
    template <int LO, int HI, int BS>
    static __device__ void mac(V4* c0, V4* c1, const V4* av, const T* bv) {
#pragma unroll
        for (int kc = LO; kc < HI; ++kc) {
            const int j = kc - LO;
            const T x = av[j >> 2][j & 3];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                if (j & 1) c1[cb] = Arith<T>::mfma(x, bv[BS * cb + j], c1[cb]);
                else c0[cb] = Arith<T>::mfma(x, bv[BS * cb + j], c0[cb]);
            }
        }
    }
    // x (w.x + i w.y) on the lane pair (re, im) of one complex value; FP32
    // factors carry hi (w) and lo (wl) parts (kernels.h)
    static __device__ T phase(T x, V2 w, V2 wl, bool im, bool cj) {
        const T y = __shfl_xor(x, 1, 64);
        if constexpr (sizeof(T) == sizeof(float)) {
            const float2 z = im ? make_float2(y, x) : make_float2(x, y);
            const float2 r = mul_unit(z, make_float2(w.x, cj ? -w.y : w.y), make_float2(wl.x, cj ? -wl.y : wl.y));
            return im ? r.y : r.x;
        } else {
            const T s = cj ? -w.y : w.y;
            return im ? x * w.x + y * s : x * w.x - y * s;
        }
    }
    // the value of lane l ^ 1 (DPP quad permutation 1, 0, 3, 2)
    static __device__ float swap_pair(float x) {
        return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, false));
    }
    static __device__ V4 ld4(const T* p) { return *reinterpret_cast<const V4*>(p); }
    static __device__ void st4(T* p, V4 v) { *reinterpret_cast<V4*>(p) = v; }
    static __device__ V4 zero4() { return V4{0, 0, 0, 0}; }

    // Tile data in the natural layout: lane l loads channel l/LPC, FPL floats
    // from slot 4 (l%LPC) NCB of tile t, and writes them to the tile's LDS slot.
    __device__ void load_dat(DV4* x, int t) const {
        const DV4 DSBT_GLOBAL* g = reinterpret_cast<const DV4 DSBT_GLOBAL*>(src + gpre + 64 * (int64_t)tile(t));
#pragma unroll
        for (int i = 0; i < 2 * NCB; ++i) x[i] = g[i];
    }
    // With KPH (inverse only) the staged values are the input times the
    // kinetic factors of their slots (conjugated for the adjoint step), which
    // load_kph fetches ahead into registers.
    struct Kph {
        V4 w[2 * NCB], wl[2 * NCB];   // factors of the lane's slot pairs (wl: FP32 lo parts)
    };
    __device__ int slot0(int t) const { return 32 * tile(t) + (FPL / 2) * (lane % LPC); }   // slot of x[0].xy
    __device__ void load_kph(Kph& k, int t) const {
        const int n0 = slot0(t);
#pragma unroll
        for (int i = 0; i < 2 * NCB; ++i) {
            k.w[i] = *reinterpret_cast<const V4 DSBT_GLOBAL*>(kphase + n0 + 2 * i);
            if constexpr (sizeof(T) == sizeof(float))
                k.wl[i] = *reinterpret_cast<const V4 DSBT_GLOBAL*>(kphase_lo + n0 + 2 * i);
        }
    }
    __device__ void write_dat(const DV4* x, int t, const Kph& k) const {
        T* xs = xring + (t % kXRing) * XSLOT;
#pragma unroll
        for (int i = 0; i < 2 * NCB; ++i) {
            V4 v = __builtin_convertvector(x[i], V4);
            if constexpr (KPH) v = times_kphase(v, k.w[i], k.wl[i]);
            st4(xs + xnat + 4 * i, v);
        }
    }
    // (v.x + i v.y, v.z + i v.w) times the factors (w.x + i w.y, w.z + i w.w)
    __device__ V4 times_kphase(V4 v, V4 w, V4 l) const {
        const T s1 = conj ? -w.y : w.y, s2 = conj ? -w.w : w.w;
        if constexpr (sizeof(T) == sizeof(float)) {
            const T l1 = conj ? -l.y : l.y, l2 = conj ? -l.w : l.w;
            const float2 a = mul_unit(make_float2(v.x, v.y), make_float2(w.x, s1), make_float2(l.x, l1));
            const float2 b = mul_unit(make_float2(v.z, v.w), make_float2(w.z, s2), make_float2(l.z, l2));
            return V4{a.x, a.y, b.x, b.y};
        } else {
            return V4{v.x * w.x - v.y * s1, v.x * s1 + v.y * w.x, v.z * w.z - v.w * s2, v.z * s2 + v.w * w.z};
        }
    }

    // ---- pre wave: q_t = Q x_t ----
    // A phase starts with the LDS reads of its tiles in the operand layout
    // (the chain wave staged them in the phase before); step t issues the
    // read-out of tile t - 1 (in the same phase), the matrix instructions of
    // tile t and the table loads of tile t + kPD.
    struct Pre {
        V4 a[kSets][2 * KB];                // tables, tile t in set t % kSets
        T xv[kPhase][NCB * 8];              // operand layout of the phase's tiles
        V4 c0[kPhase][KB][NCB], c1[kPhase][KB][NCB];   // accumulators per step of a phase
    };
    template <int S>
    __device__ void pre_load_tab(Pre& r, int t) const {
        const int J = tile(t);
        seg<2>(r.a[S], J, 2, 0);
        if constexpr (KB == 2) seg<2>(r.a[S] + 2, J, 3, 0);
    }
    // tile t from its LDS data slot in the operand layout -> xv[I]
    template <int I>
    __device__ void pre_read(Pre& r, int t) const {
        const T* xs = xring + (t % kXRing) * XSLOT;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int kc = 0; kc < 8; ++kc) r.xv[I][8 * cb + kc] = xs[xop[cb] + 8 * kc];
    }
    template <int S>
    __device__ void pre_mfma(Pre& r) const {
        constexpr int I = S % kPhase;
#pragma unroll
        for (int h = 0; h < KB; ++h) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) r.c0[I][h][cb] = r.c1[I][h][cb] = zero4();
            mac<0, 8, 8>(r.c0[I][h], r.c1[I][h], r.a[S] + 2 * h, r.xv[I]);
        }
    }
    template <int I>
    __device__ void pre_readout(const Pre& r, int t) const {
        T* qs = qring + (t % kQRing) * SLOT + 4 * lane;
#pragma unroll
        for (int h = 0; h < KB; ++h)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) st4(qs + (2 * cb + h) * 256, r.c0[I][h][cb] + r.c1[I][h][cb]);
    }
    template <int S>
    __device__ void pre_step(Pre& r, int t) const {
        __builtin_amdgcn_sched_barrier(0);   // keep the steps (and their prefetches) in order
        if constexpr (S % kPhase > 0) pre_readout<S % kPhase - 1>(r, t - 1);
        pre_mfma<S>(r);
        // the table set refilled here was read by the matrix instructions of
        // tile t - 1; loading it only after tile t's instructions are issued
        // keeps the loads from waiting for those reads
        __builtin_amdgcn_sched_barrier(0);
        pre_load_tab<(S + kPD) % kSets>(r, t + kPD);
    }
    // steps of one phase (tiles t0 .. t0 + kPhase - 1, register sets I0 ..)
    template <int I0, int I = 0>
    __device__ void pre_phase(Pre& r, int t0) const {
        if constexpr (I < kPhase) {
            pre_step<I0 + I>(r, t0 + I);
            pre_phase<I0, I + 1>(r, t0);
        } else {
            pre_readout<kPhase - 1>(r, t0 + kPhase - 1);
        }
    }
    template <int I = 0>
    __device__ void pre_read_phase(Pre& r, int t0) const {
        if constexpr (I < kPhase) {
            pre_read<I>(r, t0 + I);
            pre_read_phase<I + 1>(r, t0);
        }
    }
    template <int I0>
    __device__ void pre_phase_body(Pre& r, int t0) const {
        pre_read_phase(r, t0);
        pre_phase<I0>(r, t0);
        lds_barrier();
    }
    // phases ph .. ph + kRep - 1
    template <int P = 0>
    __device__ void pre_iter(Pre& r, int ph) const {
        if constexpr (P < kRep) {
            pre_phase_body<P * kPhase>(r, (ph + P) * kPhase);
            pre_iter<P + 1>(r, ph);
        }
    }
    __device__ void run_pre() const {
        Pre r;
        __builtin_amdgcn_sched_barrier(0);   // prologue loads in the order of the steps
        pre_load_tab<0>(r, 0);
        pre_load_tab<1>(r, 1);
        pre_load_tab<2>(r, 2);
        // tiles 0 .. kPhase - 1 -> LDS (the chain wave stages the later ones)
#pragma unroll
        for (int u = 0; u < kPhase; ++u) {
            DV4 x[2 * NCB];
            load_dat(x, u);
            Kph k;
            if constexpr (KPH) load_kph(k, u);
            write_dat(x, u, k);
        }
        wave_lds_fence();
        int ph = 0;
        for (; ph + kRep <= nact; ph += kRep) pre_iter(r, ph);
        if constexpr (TAIL) {
            if (ph < nact) pre_phase_body<0>(r, ph * kPhase);   // nact < kRep
        }
        lds_barrier();
        lds_barrier();
    }

    // ---- chain wave: mu_t+1 = q_t + D mu_t ----
    // The chain wave also stages the tile data for the other roles: step t
    // writes tile t + kStage to its LDS slot (the pre wave reads it a phase
    // later) and loads tile t + 2 kStage in its place, kStage = 2 kPhase.
    static constexpr int kStage = 2 * kPhase;
    static_assert(kStage == kSets, "staging set t % kSets holds tile t + kStage");
    // kinetic factors are fetched kKS steps before their tile is staged (two
    // sets of registers for items of one column block, one for two)
    static constexpr int kKS = NCB == 1 ? 2 : 1;
    static_assert(kSets % kKS == 0, "a loop iteration must cycle through the factor sets");
    struct Chain {
        V4 a[kSets][NC2 + NC3];
        V4 qg[kPhase][NCB][KB];
        T bm[NCB * 4 * KB];   // block cb: moment row 4 j + l/16 in bm[4 KB cb + j]
        DV4 x[kSets][2 * NCB];   // natural-layout data, tile t + kStage in set t % kSets
        Kph k[kKS];              // KPH: kinetic factors of tile t + kStage in k[t % kKS]
    };
    template <int S>
    __device__ void chain_load(Chain& r, int t) const {
        __builtin_amdgcn_sched_barrier(0);
        const int J = tile(t);
        seg<NC2>(r.a[S], J, 2, C2LO / 4);
        if constexpr (KB == 2) seg<NC3>(r.a[S] + NC2, J, 3, C3LO / 4);
    }
    __device__ void store_mu(const Chain& r, int t) const {
        T* ms = mring + (t % kMRing) * SLOT + 4 * lane;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const T* b = r.bm + 4 * KB * cb;
            st4(ms + 2 * cb * 256, V4{b[0], b[1], b[2], b[3]});
            if constexpr (KB == 2) st4(ms + (2 * cb + 1) * 256, V4{b[4], b[5], b[6], b[7]});
        }
    }
    template <int S>
    __device__ void chain_step(Chain& r, int t) const {
        if constexpr (TAIL) {
            if (t >= NT) return;   // bm must keep mu_NT
        }
        __builtin_amdgcn_sched_barrier(0);
        V4 c0[NCB], c1[NCB], m2[NCB], m3[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            c0[cb] = r.qg[S % kPhase][cb][0];
            c1[cb] = zero4();
        }
        mac<C2LO, C2HI, 4 * KB>(c0, c1, r.a[S], r.bm + (C2LO - 8));
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) m2[cb] = c0[cb] + c1[cb];
        if constexpr (KB == 2) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                c0[cb] = r.qg[S % kPhase][cb][1];
                c1[cb] = zero4();
            }
            mac<C3LO, C3HI, 4 * KB>(c0, c1, r.a[S] + NC2, r.bm + (C3LO - 8));
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) m3[cb] = c0[cb] + c1[cb];
        }
        __builtin_amdgcn_sched_barrier(0);
        chain_load<(S + kPD) % kSets>(r, t + kPD);   // after tile t's matrix instructions (see pre_step)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            result_to_operand(m2[cb], r.bm + 4 * KB * cb);
            if constexpr (KB == 2) result_to_operand(m3[cb], r.bm + 4 * KB * cb + 4);
        }
        store_mu(r, t + 1);
        write_dat(r.x[S], t + kStage, r.k[S % kKS]);
        load_dat(r.x[S], t + 2 * kStage);
        if constexpr (KPH) load_kph(r.k[S % kKS], t + kStage + kKS);   // staged kKS steps on
    }
    template <int I0, int I = 0>
    __device__ void chain_phase(Chain& r, int t0) const {
        if constexpr (I < kPhase) {
            chain_step<I0 + I>(r, t0 + I);
            chain_phase<I0, I + 1>(r, t0);
        }
    }
    template <int I0>
    __device__ void chain_phase_body(Chain& r, int t0) const {
#pragma unroll
        for (int i = 0; i < kPhase; ++i) {
            const T* qs = qring + ((t0 + i) % kQRing) * SLOT + 4 * lane;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                r.qg[i][cb][0] = ld4(qs + 2 * cb * 256);
                if constexpr (KB == 2) r.qg[i][cb][1] = ld4(qs + (2 * cb + 1) * 256);
            }
        }
        chain_phase<I0>(r, t0);
        lds_barrier();
    }
    template <int P = 0>
    __device__ void chain_iter(Chain& r, int ph) const {
        if constexpr (P < kRep) {
            chain_phase_body<P * kPhase>(r, (ph + P) * kPhase);
            chain_iter<P + 1>(r, ph);
        }
    }
    __device__ void run_chain(T* bm_out) const {
        Chain r;
        chain_load<0>(r, 0);
        chain_load<1>(r, 1);
        chain_load<2>(r, 2);
        // staging: tiles kPhase .. kStage - 1 (read by the pre wave in its
        // second phase) now, tiles kStage .. 2 kStage - 1 into the sets
#pragma unroll
        for (int u = kPhase; u < kStage; ++u) load_dat(r.x[u], u);
#pragma unroll
        for (int u = 0; u < kPhase; ++u) load_dat(r.x[u], u + kStage);
#pragma unroll
        for (int u = kPhase; u < kStage; ++u) {
            if constexpr (KPH) load_kph(r.k[0], u);
            write_dat(r.x[u], u, r.k[0]);
            load_dat(r.x[u], u + kStage);
        }
        if constexpr (KPH) {
#pragma unroll
            for (int i = 0; i < kKS; ++i) load_kph(r.k[(kStage + i) % kKS], kStage + i);
        }
        // mu_0: zero forward; inverse (-1)^p times the completion slots 0..k-1 of tile 0
        const T sgn = p ? -1 : 1;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int j = 0; j < 4 * KB; ++j) {
                const int row = 4 * j + q;
                T x = (INV && row < k) ? sgn * (T)src[e0[cb] + 2 * row] : T(0);
                if constexpr (KPH) {
                    // lanes col and col ^ 1 hold the (re, im) pair of one slot
                    const V2 wl = sizeof(T) == sizeof(float) ? kphase_lo[row] : V2{0, 0};
                    x = phase(x, kphase[row], wl, col & 1, conj);
                }
                r.bm[4 * KB * cb + j] = x;
            }
        store_mu(r, 0);
        lds_barrier();
        int ph = 0;
        for (; ph + kRep <= nact; ph += kRep) chain_iter(r, ph);
        if constexpr (TAIL) {
            if (ph < nact) chain_phase_body<0>(r, ph * kPhase);
        }
        lds_barrier();
#pragma unroll
        for (int j = 0; j < NCB * 4 * KB; ++j) bm_out[j] = r.bm[j];
    }

    // forward completion rows (-1)^p mu_NT into slots 0..k-1 of tile 0
    // (operand layout: moment row 4 j + l/16 of block cb is bm[4 KB cb + j])
    __device__ void completion(const T* bm) const {
        const T sgn = p ? -1 : 1;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int j = 0; j < 4 * KB; ++j) {
                const int row = 4 * j + q;
                const T x = sgn * bm[4 * KB * cb + j];
                if (row < k) dst[e0[cb] + 2 * row] = (D)x;
            }
    }

    // ---- result waves: rows 16 RB .. 16 RB + 15 of o_t ----
    // The two result waves W = 0, 1 take row block rb(W, t) of tile t: the
    // heavier block (rows 16..31 forward, 0..15 inverse) on every other tile,
    // so that both carry the same matrix work.
    // Step t issues the loads of tile t + kPD, the read-out and stores of tile
    // t - 1 and the matrix instructions of tile t, so that the read-out runs
    // while the matrix core works.  The first loop iteration is peeled (no tile
    // -1), which keeps every loop body free of branches around memory operations.
    static constexpr int rb(int W, int t) { return ((INV ? 0 : 1) + W + t) & 1; }
    static constexpr int lo_of(int RB) { return RB == 0 ? R0LO : R1LO; }
    static constexpr int hi_of(int RB) { return RB == 0 ? R0HI : R1HI; }
    static constexpr int nd_of(int RB) { return (hi_of(RB) - lo_of(RB)) / 4; }
    static constexpr int NDMAX = nd_of(0) > nd_of(1) ? nd_of(0) : nd_of(1);
    struct Out {
        V4 a[kSets][NDMAX + KB];      // tile t: data chunks of its row block, then the moment chunks
        T x[kPhase][NCB * 8];         // block cb: data chunk kc in x[.][8 cb + kc]
        T mu[kPhase][NCB * 4 * KB];
        V4 c0[2][NCB], c1[2][NCB];    // accumulators of tile t in [t % 2]
    };
    template <int W, int S>
    __device__ void out_load(Out& r, int t) const {
        __builtin_amdgcn_sched_barrier(0);
        constexpr int RB = rb(W, S);
        const int J = tile(t);
        seg<nd_of(RB)>(r.a[S], J, RB, lo_of(RB) / 4);
        seg<KB>(r.a[S] + nd_of(RB), J, RB, 2);
    }
    // read-out of tile t (row block RB) from accumulators [P]: result layout ->
    // (channel 8 cb + l/8, slots 2 (l%8), 2 (l%8) + 1) through this wave's LDS
    // staging area, 16-byte store
    template <int W, int RB, int P>
    __device__ void out_epilogue(Out& r, int t) const {
        const int J = tile(t);
        if constexpr (sizeof(T) == sizeof(float)) {
            // lane l holds rows 4 (l/16) + v of column l%16, the re (even
            // column) or im (odd) part of channel 8 cb + (l%16)/2: the lane
            // pair (col, col ^ 1) trades two values (one DPP move each) so that
            // the even lane holds rows 4 (l/16) + 0, 1 and the odd one rows
            // 4 (l/16) + 2, 3 as (re, im, re, im), two consecutive slots
            const bool odd = col & 1;
            const int s0 = 16 * RB + 4 * q + 2 * (col & 1);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const V4 o = r.c0[P][cb] + r.c1[P][cb];
                const float g0 = swap_pair(odd ? o[0] : o[2]);
                const float g1 = swap_pair(odd ? o[1] : o[3]);
                const V4 v = odd ? V4{g0, o[2], g1, o[3]} : V4{o[0], g0, o[1], g1};
                // forward: slots 0..k-1 of tile 0 are rewritten with the completion rows at the end
                *reinterpret_cast<DV4 DSBT_GLOBAL*>(dst + (e0[cb] - (col & 1)) + 64 * (int64_t)J + 2 * s0) =
                    __builtin_convertvector(v, DV4);
            }
            return;
        }
        const int c = lane >> 3, s0 = 2 * (lane & 7);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            T* y = yring + (W * NCB + cb) * 16 * kYCol;
            const V4 o = r.c0[P][cb] + r.c1[P][cb];
#pragma unroll
            for (int v = 0; v < 4; ++v) y[col * kYCol + 4 * v + q] = o[v];   // rows 4 v + l/16
            wave_lds_fence();
            const V2 re = *reinterpret_cast<const V2*>(y + 2 * c * kYCol + s0);
            const V2 im = *reinterpret_cast<const V2*>(y + (2 * c + 1) * kYCol + s0);
            wave_lds_fence();
            const V4 v = V4{re.x, im.x, re.y, im.y};
            // forward: slots 0..k-1 of tile 0 are rewritten with the completion rows at the end
            *reinterpret_cast<DV4 DSBT_GLOBAL*>(dst + g0[cb] + 64 * (int64_t)J + 2 * (16 * RB + s0)) =
                __builtin_convertvector(v, DV4);
        }
    }
    template <int W, int S, bool FIRST>
    __device__ void out_step(Out& r, int t) const {
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!FIRST) {
            if constexpr (TAIL) {
                if (t - 1 < NT) out_epilogue<W, rb(W, S + 1), (S + 1) & 1>(r, t - 1);
            } else {
                out_epilogue<W, rb(W, S + 1), (S + 1) & 1>(r, t - 1);
            }
        }
        constexpr int RB = rb(W, S), LO = lo_of(RB), HI = hi_of(RB), P = S & 1;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) r.c0[P][cb] = r.c1[P][cb] = zero4();
        mac<LO, HI, 8>(r.c0[P], r.c1[P], r.a[S], r.x[S % kPhase] + LO);
        mac<8, MHI, 4 * KB>(r.c0[P], r.c1[P], r.a[S] + nd_of(RB), r.mu[S % kPhase]);
        __builtin_amdgcn_sched_barrier(0);
        out_load<W, (S + kPD) % kSets>(r, t + kPD);   // after tile t's matrix instructions (see pre_step)
    }
    template <int W, int I0, bool FIRST, int I = 0>
    __device__ void out_phase(Out& r, int t0) const {
        if constexpr (I < kPhase) {
            out_step<W, I0 + I, FIRST && I0 + I == 0>(r, t0 + I);
            out_phase<W, I0, FIRST, I + 1>(r, t0);
        }
    }
    // operands of the phase's tiles (t0 even: tile t0 + i has row block rb(W, i))
    template <int W, int I = 0>
    __device__ void out_read(Out& r, int t0) const {
        if constexpr (I < kPhase) {
            constexpr int RB = rb(W, I);
            const T* xs = xring + ((t0 + I) % kXRing) * XSLOT;
            const T* ms = mring + ((t0 + I) % kMRing) * SLOT + 4 * lane;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
                for (int kc = lo_of(RB); kc < hi_of(RB); ++kc) r.x[I][8 * cb + kc] = xs[xop[cb] + 8 * kc];
                const V4 m0 = ld4(ms + 2 * cb * 256);
#pragma unroll
                for (int j = 0; j < 4; ++j) r.mu[I][4 * KB * cb + j] = m0[j];
                if constexpr (KB == 2) {
                    const V4 m1 = ld4(ms + (2 * cb + 1) * 256);
#pragma unroll
                    for (int j = 0; j < 4; ++j) r.mu[I][4 * KB * cb + 4 + j] = m1[j];
                }
            }
            out_read<W, I + 1>(r, t0);
        }
    }
    template <int W, int I0, bool FIRST>
    __device__ void out_phase_body(Out& r, int t0) const {
        out_read<W>(r, t0);
        out_phase<W, I0, FIRST>(r, t0);
        lds_barrier();
    }
    template <int W, bool FIRST, int P = 0>
    __device__ void out_iter(Out& r, int ph) const {
        if constexpr (P < kRep) {
            out_phase_body<W, P * kPhase, FIRST>(r, (ph + P) * kPhase);
            out_iter<W, FIRST, P + 1>(r, ph);
        }
    }
    template <int W>
    __device__ void run_out() const {
        Out r;
        out_load<W, 0>(r, 0);
        out_load<W, 1>(r, 1);
        out_load<W, 2>(r, 2);
        lds_barrier();
        lds_barrier();
        const int tl = nact * kPhase - 1;   // last step (odd)
        if constexpr (TAIL) {
            // nact == 1 < kRep: one phase
            out_phase_body<W, 0, true>(r, 0);
            if (tl < NT) out_epilogue<W, rb(W, 1), 1>(r, tl);
        } else {
            out_iter<W, true>(r, 0);
            for (int ph = kRep; ph + kRep <= nact; ph += kRep) out_iter<W, false>(r, ph);
            out_epilogue<W, rb(W, 1), 1>(r, tl);   // nact is a multiple of kRep
        }
    }

    __device__ void run() const {
        // roles by wave: pre, result, chain, result.  Two workgroups on a
        // compute unit place their waves on the SIMDs in the order 0, 2, 1, 3,
        // the second starting one SIMD further along, so that each SIMD holds
        // wave w of one and wave w - 1 of the other: this order pairs every
        // result wave with a pre or chain wave.
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        T bm[NCB * 4 * KB];
        switch (wave) {
            case 0: run_pre(); break;
            case 1: run_out<0>(); break;
            case 2: run_chain(bm); break;
            default: run_out<1>(); break;
        }
        if constexpr (!INV) {
            // the result waves' stores of tile 0 are ordered before the
            // completion rows that replace slots 0..k-1
            __syncthreads();
            if (wave == 2) completion(bm);
        }
    }
};

template <typename T, typename D, bool INV, bool KPH, int NCB>
__device__ void run_item(const MItem& it, const void* src, void* dst, const PhaseArgs& ph, T* lds) {
    const bool tail = it.NT % kSets != 0;
    if (it.k > 16) {
        if (tail) Pipe<T, D, INV, KPH, 2, true, NCB>(it, src, dst, ph, lds).run();
        else Pipe<T, D, INV, KPH, 2, false, NCB>(it, src, dst, ph, lds).run();
    } else {
        if (tail) Pipe<T, D, INV, KPH, 1, true, NCB>(it, src, dst, ph, lds).run();
        else Pipe<T, D, INV, KPH, 1, false, NCB>(it, src, dst, ph, lds).run();
    }
}

template <typename T, typename D, bool INV, bool KPH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == sizeof(float) ? 2 : 1))) mstage_chain(const MItem* __restrict__ items, const void* src, void* dst,
                                                    PhaseArgs ph) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T* lds = reinterpret_cast<T*>(lds_raw);
    const MItem& it = items[blockIdx.x];
    if (it.nch == 0) return;   // idle slot of the per-XCD schedule
    if constexpr (sizeof(T) == sizeof(float)) {
        if (it.NCB == 2) {
            run_item<T, D, INV, KPH, 2>(it, src, dst, ph, lds);
            return;
        }
    }
    run_item<T, D, INV, KPH, 1>(it, src, dst, ph, lds);   // FP64 items have one column block
}

}  // namespace

template <typename T>
size_t chain_lds_bytes(int ncb) {
    return sizeof(T) * (size_t)chain_lds_values(ncb > 1 ? 2 : 1);
}

template <typename T>
hipError_t set_lds_limits_chain() {
    hipError_t e = hipSuccess;
    const int bytes = (int)chain_lds_bytes<T>(sizeof(T) == sizeof(float) ? 2 : 1);
    auto set = [&](const void* f) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    };
    set((const void*)mstage_chain<T, float, true, false>);
    set((const void*)mstage_chain<T, float, true, true>);
    set((const void*)mstage_chain<T, float, false, false>);
    if constexpr (sizeof(T) == sizeof(double)) {
        set((const void*)mstage_chain<T, double, true, false>);
        set((const void*)mstage_chain<T, double, true, true>);
        set((const void*)mstage_chain<T, double, false, false>);
    }
    return e;
}

template <typename T, typename D>
hipError_t launch_mstage_chain(const MItem* d_items, int nitems, int ncb, const void* src, void* dst, bool inverse,
                               PhaseArgs ph, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (!inverse && ph.use) return hipErrorInvalidValue;   // phases are applied to the inverse's input only
    if (sizeof(T) != sizeof(float) && ncb != 1) return hipErrorInvalidValue;
    if (sizeof(D) > sizeof(T)) return hipErrorInvalidValue;
    const size_t lds = chain_lds_bytes<T>(ncb);
    if (inverse && ph.use)
        hipLaunchKernelGGL((mstage_chain<T, D, true, true>), dim3(nitems), dim3(256), lds, s, d_items, src, dst, ph);
    else if (inverse)
        hipLaunchKernelGGL((mstage_chain<T, D, true, false>), dim3(nitems), dim3(256), lds, s, d_items, src, dst, ph);
    else
        hipLaunchKernelGGL((mstage_chain<T, D, false, false>), dim3(nitems), dim3(256), lds, s, d_items, src, dst, ph);
    return hipGetLastError();
}

template size_t chain_lds_bytes<float>(int);
template size_t chain_lds_bytes<double>(int);
template hipError_t set_lds_limits_chain<float>();
template hipError_t set_lds_limits_chain<double>();
template hipError_t launch_mstage_chain<float, float>(const MItem*, int, int, const void*, void*, bool, PhaseArgs,
                                                      hipStream_t);
template hipError_t launch_mstage_chain<double, float>(const MItem*, int, int, const void*, void*, bool, PhaseArgs,
                                                       hipStream_t);
template hipError_t launch_mstage_chain<double, double>(const MItem*, int, int, const void*, void*, bool, PhaseArgs,
                                                        hipStream_t);

}  // namespace dsbt
