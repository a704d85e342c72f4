// Moment stage of the Fourier-to-Bessel transform on the CDNA4 matrix cores.
//
// One work item = 8 NCB channel slots with the same (l, N) (NCB = column
// blocks, chosen so that the row x column blocks cover the waves); when fewer
// channels share (l, N) the remaining slots repeat a real channel and write
// its results again unchanged.  Per tile J the item
// computes out = A' x with A' the zero-padded R16 x R16 tile block of the
// tiled moment form (Sec. 2.4-2.5) and x = [tile data; moments] for every
// channel: a (R16 x R16) x (R16 x 16 NCB) product done with
// v_mfma_f32_16x16x4_f32, 16 output rows x 16 real columns (8 complex
// channels) per unit.  Lane layout of that instruction: lane l holds
// A[l%16][l/16] and B[l/16][l%16]; result register v of lane l is
// D[4 (l/16) + v][l%16].
//
// Wave w owns row block rb = w % NB for the column blocks it takes; its
// NK = 4 NB operand floats per tile come straight from global memory (16-byte
// loads, each reading 1 KiB contiguous over the wave).  Operands and tile data are loaded two tiles ahead
// into three register sets; the tile loop is unrolled by three so that no set
// is renamed while its loads are in flight, and the loop body has no branch
// around a global access (every thread issues the same loads and stores each
// tile), so the compiler's memory-counter waits stay exact.  The input vector
// sits transposed in LDS (Xt[q][16 columns]) in two parity buffers; a tile
// costs one LDS-only barrier.  Results pass through LDS (Yt) and are written
// to global memory coalesced.
#include "kernels.h"

namespace dsbt {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));   // complex64 value in global memory

// prefetch distance in tiles: operands and data of tile t + PD are requested
// while tile t is multiplied
constexpr int kMfmaPrefetch = 3;

template <int WAVES, int NB, int NCB, bool INV, bool KPH>
struct MfmaTile {
    static constexpr int PD = kMfmaPrefetch, SETS = PD + 1;
    static constexpr int R16 = 16 * NB, NK = 4 * NB, NTH = WAVES * 64, NCH = 8 * NCB;
    static constexpr int B = mfma_tile_for(NB);
    static constexpr int NE = NCH * B;                       // tile elements of the item
    static constexpr int GM = NE >= NTH ? NE / NTH : 1;       // elements per thread
    static constexpr int UMAX = (NB * NCB + WAVES - 1) / WAVES;
    static_assert(NE % NTH == 0 || NE < NTH, "tile elements must spread evenly");
    static_assert((NB * NCB) % WAVES == 0 || NB * NCB < WAVES, "units must spread evenly");

    const MItem& it;
    const f2 DSBT_GLOBAL* src;
    f2 DSBT_GLOBAL* dst;
    float* Xt;   // [2][NCB][R16][16]: input vector (tile data, then moments), two parities
    float* Yt;   // [2][NCB][B][16]: tile results
    const float DSBT_GLOBAL* tab;
    const f2 DSBT_GLOBAL* kphase;
    const f2 DSBT_GLOBAL* kphase_lo;
    int k, NT, tid, lane, rb;
    int cbs[UMAX];
    bool conj;
    f4 a[SETS][NK / 4];    // operand sets of SETS consecutive tiles
    f2 g[SETS][GM];        // data of SETS consecutive tiles
    // this thread's tile elements (channel, slot): global element index of
    // slot s at tile 0, LDS float offsets in Xt and Yt, slot s
    int64_t gofs[GM];
    int lofs[GM], yofs[GM], sidx[GM];

    __device__ MfmaTile(const MItem& it_, const float2* s_, float2* d_, const PhaseArgs& ph, float* lds)
        : it(it_), src(as_global(reinterpret_cast<const f2*>(s_))), dst(as_global_rw(reinterpret_cast<f2*>(d_))) {
        k = it.k;
        NT = it.NT;
        tid = threadIdx.x;
        lane = tid & 63;
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave
        rb = wave % NB;
        // units u = wave + WAVES i; when there are fewer units than waves a wave
        // repeats unit u mod (NB NCB) and writes the same values again
#pragma unroll
        for (int i = 0; i < UMAX; ++i) cbs[i] = ((wave + WAVES * i) % (NB * NCB)) / NB;
        Xt = lds;
        Yt = lds + 2 * NCB * R16 * 16;
        tab = as_global(static_cast<const float*>(INV ? it.mf_i : it.mf_f));
        kphase = as_global(reinterpret_cast<const f2*>(it.kphase));
        kphase_lo = as_global(reinterpret_cast<const f2*>(it.kphase_lo));
        conj = ph.conj != 0;
        // element e = (channel, slot): 4 consecutive slots of one channel per
        // 4 lanes (32-byte global segments), channels across lanes, so the LDS
        // row [slot][16 columns] is written with 8-byte stores without conflicts
#pragma unroll
        for (int i = 0; i < GM; ++i) {
            const int e = (tid + i * NTH) % NE;   // threads past NE duplicate an element
            const int grp = e >> 2;                // 4-slot group
            const int ch = grp % NCH, s = 4 * (grp / NCH) + (e & 3);
            gofs[i] = it.off[ch] + s;
            lofs[i] = ((ch >> 3) * R16 + s) * 16 + 2 * (ch & 7);
            yofs[i] = ((ch >> 3) * B + s) * 16 + 2 * (ch & 7);
            sidx[i] = s;
        }
    }
    __device__ int tile_of(int step) const { return INV ? NT - 1 - step : step; }
    __device__ float* xt(int par, int cb, int row) const { return Xt + ((par * NCB + cb) * R16 + row) * 16; }
    __device__ float* yt(int par, int cb, int row) const { return Yt + ((par * NCB + cb) * B + row) * 16; }
    // x times the kinetic factor of slot i (hi + lo parts, kernels.h)
    __device__ f2 kph(f2 x, int i) const {
        f2 h = kphase[i], l = kphase_lo[i];
        if (conj) {
            h.y = -h.y;
            l.y = -l.y;
        }
        const float2 r = mul_unit(make_float2(x.x, x.y), make_float2(h.x, h.y), make_float2(l.x, l.y));
        return f2{r.x, r.y};
    }

    template <int S>
    __device__ void load(int step) {   // issue the loads of one tile (clamped to the last) into set S
        const int J = tile_of(step < NT ? step : NT - 1);
        const f4 DSBT_GLOBAL* ap = reinterpret_cast<const f4 DSBT_GLOBAL*>(tab + ((size_t)J * NB + rb) * NK * 64) + lane;
#pragma unroll
        for (int i = 0; i < NK / 4; ++i) a[S][i] = ap[64 * i];
#pragma unroll
        for (int i = 0; i < GM; ++i) g[S][i] = src[gofs[i] + J * B];
    }
    template <int S>
    __device__ void stage_data(int par) {   // set S -> Xt[par] rows [0, B)
        float* X = Xt + par * NCB * R16 * 16;
#pragma unroll
        for (int i = 0; i < GM; ++i) *reinterpret_cast<f2*>(X + lofs[i]) = g[S][i];
    }
    template <int S>
    __device__ void step(int st) {
        constexpr int S1 = (S + 1) % SETS, SP = (S + PD) % SETS;
        const int par = st & 1;
        load<SP>(st + PD);
        // UMAX accumulators per wave; with one unit the K range is split over two
        // chains (even / odd kc) so consecutive matrix instructions are independent
        constexpr int NCHAIN = UMAX == 1 ? 2 : 1;
        f4 acc[UMAX][NCHAIN];
        float bv[UMAX][NK];
#pragma unroll
        for (int i = 0; i < UMAX; ++i) {
#pragma unroll
            for (int c = 0; c < NCHAIN; ++c) acc[i][c] = f4{0.0f, 0.0f, 0.0f, 0.0f};
            const float* xb = xt(par, cbs[i], 0) + (lane >> 4) * 16 + (lane & 15);
#pragma unroll
            for (int kc = 0; kc < NK; ++kc) bv[i][kc] = xb[kc * 64];
        }
#pragma unroll
        for (int kc = 0; kc < NK; ++kc) {
            const float av = a[S][kc >> 2][kc & 3];
#pragma unroll
            for (int i = 0; i < UMAX; ++i)
                acc[i][kc % NCHAIN] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[i][kc], acc[i][kc % NCHAIN], 0, 0, 0);
        }
        if constexpr (NCHAIN == 2) {
#pragma unroll
            for (int i = 0; i < UMAX; ++i) acc[i][0] += acc[i][1];
        }
        // row block rb holds tile results (rows < B) or next moments (rows >= B);
        // B is a multiple of 16, so the choice is uniform per wave
#pragma unroll
        for (int i = 0; i < UMAX; ++i) {
            const int row0 = 16 * rb + 4 * (lane >> 4);
            if (16 * rb < B) {
                float* y = yt(par, cbs[i], row0) + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v) y[16 * v] = acc[i][0][v];
            } else {
                float* x = xt(par ^ 1, cbs[i], row0) + (lane & 15);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (row0 + v < B + k) x[16 * v] = acc[i][0][v];
            }
        }
        stage_data<S1>(par ^ 1);   // next tile's data (a harmless copy after the last tile)
        lds_barrier();
        const int J = tile_of(st);
        const float* Y = Yt + par * NCB * B * 16;
#pragma unroll
        for (int i = 0; i < GM; ++i) {
            f2 v = *reinterpret_cast<const f2*>(Y + yofs[i]);
            if constexpr (KPH) v = kph(v, J * B + sidx[i]);
            dst[gofs[i] + J * B] = v;   // forward: tile-0 completion slots are rewritten at the end
        }
    }

    template <int I>
    __device__ void prologue() {   // loads of tiles 0 .. PD-1
        if constexpr (I < PD) {
            load<I>(I);
            prologue<I + 1>();
        }
    }
    template <int I>
    __device__ void steps(int st) {   // one full round of SETS tiles
        if constexpr (I < SETS) {
            step<I>(st + I);
            steps<I + 1>(st);
        }
    }
    template <int I>
    __device__ void tail(int st) {   // the last NT mod SETS tiles
        if constexpr (I < SETS - 1) {
            if (st + I < NT) step<I>(st + I);
            tail<I + 1>(st);
        }
    }

    __device__ void run() {
        const float sgn = it.p ? -1.0f : 1.0f;  // completion rows = (-1)^p mu_NT
        for (int e = tid; e < 2 * NCB * R16 * 16; e += NTH) Xt[e] = 0.0f;
        prologue<0>();
        lds_barrier();
        if constexpr (INV) {
            for (int e = tid; e < NCH * k; e += NTH) {
                const int ch = e / k, kk = e % k;
                const f2 v = src[it.off[ch] + kk];
                float* x = xt(0, ch >> 3, B + kk) + 2 * (ch & 7);
                x[0] = sgn * v.x;
                x[1] = sgn * v.y;
            }
        }
        stage_data<0>(0);
        lds_barrier();
        int st = 0;
        for (; st + SETS <= NT; st += SETS) steps<0>(st);
        tail<0>(st);
        if constexpr (!INV) {
            // completion rows, written by the thread that wrote the same slot of tile 0
            const float* X = Xt + (NT & 1) * NCB * R16 * 16;
#pragma unroll
            for (int i = 0; i < GM; ++i) {
                if (sidx[i] >= k) continue;
                const int o = lofs[i] + B * 16;   // moment row B + s of the same column
                f2 v = *reinterpret_cast<const f2*>(X + o);
                v = f2{sgn * v.x, sgn * v.y};
                if constexpr (KPH) v = kph(v, sidx[i]);
                dst[gofs[i]] = v;
            }
        }
    }
};

template <int WAVES, bool INV, bool KPH>
__global__ void __launch_bounds__(WAVES * 64) mstage_mfma(const MItem* __restrict__ items, const float2* src,
                                                          float2* dst, PhaseArgs ph) {
    extern __shared__ __align__(16) float lds_f[];
    const MItem& it = items[blockIdx.x];
    if (it.nch == 0) return;   // idle slot of the per-XCD schedule
    switch (it.NB) {
        case 4: { MfmaTile<WAVES, 4, mfma_ncb(WAVES, 4), INV, KPH> t(it, src, dst, ph, lds_f); t.run(); } break;
        case 8:
            if constexpr (WAVES == 8) {
                MfmaTile<WAVES, 8, mfma_ncb(WAVES, 8), INV, KPH> t(it, src, dst, ph, lds_f);
                t.run();
            }
            break;
        default: break;
    }
}

static size_t mfma_lds_bytes() { return mfma_lds_bytes_for(8, 2, 64); }

hipError_t set_lds_limits_mfma() {
    const int b = (int)mfma_lds_bytes();
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    };
    set((const void*)mstage_mfma<4, false, false>);
    set((const void*)mstage_mfma<4, false, true>);
    set((const void*)mstage_mfma<4, true, false>);
    set((const void*)mstage_mfma<8, false, false>);
    set((const void*)mstage_mfma<8, false, true>);
    set((const void*)mstage_mfma<8, true, false>);
    return e;
}

hipError_t launch_mstage_mfma(const MItem* d_items, int nitems, int waves, size_t lds, const void* src,
                              void* dst, bool inverse, PhaseArgs ph, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (inverse && ph.use) return hipErrorInvalidValue;   // phases are applied on the forward output only
    const float2* a = (const float2*)src;
    float2* b = (float2*)dst;
    const bool kph = ph.use != 0;
    if (waves == 8) {
        if (inverse)
            hipLaunchKernelGGL((mstage_mfma<8, true, false>), dim3(nitems), dim3(512), lds, s, d_items, a, b, ph);
        else if (kph)
            hipLaunchKernelGGL((mstage_mfma<8, false, true>), dim3(nitems), dim3(512), lds, s, d_items, a, b, ph);
        else
            hipLaunchKernelGGL((mstage_mfma<8, false, false>), dim3(nitems), dim3(512), lds, s, d_items, a, b, ph);
    } else {
        if (inverse)
            hipLaunchKernelGGL((mstage_mfma<4, true, false>), dim3(nitems), dim3(256), lds, s, d_items, a, b, ph);
        else if (kph)
            hipLaunchKernelGGL((mstage_mfma<4, false, true>), dim3(nitems), dim3(256), lds, s, d_items, a, b, ph);
        else
            hipLaunchKernelGGL((mstage_mfma<4, false, false>), dim3(nitems), dim3(256), lds, s, d_items, a, b, ph);
    }
    return hipGetLastError();
}

}  // namespace dsbt
