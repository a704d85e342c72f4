// Sine / cosine stage of the DSBT (Sec. 2.2, eq. csFourierBasis) with the FFT
// size known at compile time.
//
// Forward, for one complex channel x of N points: even l flips x_i -> (-1)^i x_i
// (the DST-II is the DCT-II of that sequence read backwards); the DCT-II
// reorders v_j = x_2j, v_{N-1-j} = x_{2j+1}, takes V = FFT_N(v) and combines
// X_k = (w^k V_k + w^-k V_{N-k})/2, w = exp(-i pi/(2N)); the orthonormal scale
// sqrt((2 - delta_k0)/N) and the sign (-1)^ceil(l/2) follow.  The inverse
// applies the exact transpose of every step; since the DFT matrix is
// symmetric it uses the same forward FFT.
//
// Layout: a block handles CPB channels of N points with N/8 threads each; each
// thread owns 8 points per Stockham pass (radix 8, then one radix-2 or radix-4
// pass for the remaining factor), data stay in LDS with one pad slot per 32
// complex values.  Twiddles: the block copies the plan's quarter-circle roots
// exp(2 pi i e/N), e < N/4 (16 bytes each) into LDS once, and a pass twiddle
// exp(-2 pi i m/N) is the product by the conjugate root of e = m mod N/4
// followed by the exact quarter turn (-i)^(m div N/4); so the passes read no
// table from global memory.  In FP32 no product by a fixed unit number or
// constant may change the modulus of the data systematically (kernels.h,
// FChan): roots, post-twiddles and phase factors are hi + lo pairs, the
// radix-8 rotations by -pi/4 are shears, and products by constants are
// compensated.
#include "kernels.h"

#include <algorithm>

namespace dsbt {

template <typename T> struct CV;
template <> struct CV<float> { using t = float2; };
template <> struct CV<double> { using t = double2; };

template <typename V> __device__ __forceinline__ V f_add(V a, V b) { return {a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V f_sub(V a, V b) { return {a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V f_mul(V a, V b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V, typename S> __device__ __forceinline__ V f_scale(V a, S s) { return {a.x * s, a.y * s}; }

// Multiplication by a constant c = hi + lo that is not representable in FP32
// (sqrt(1/2), sqrt(2/N) for even log2 N): mul_const (kernels.h), so that the
// rounding of the constant does not scale every value by the same factor.
// FP64 arithmetic uses hi alone (lo = 0).
template <typename T> struct Split {
    T hi, lo;
};
template <typename T>
__device__ __forceinline__ Split<T> split_const(double c) {
    const T hi = (T)c;
    return {hi, (T)(c - (double)hi)};
}
template <typename T>
__device__ __forceinline__ T s_mul(T x, Split<T> c) {
    if constexpr (sizeof(T) == sizeof(float)) return mul_const(x, c.hi, c.lo);
    else return x * c.hi;
}

// One complex table value through the global address space (the HIP vector
// types have no constructors from address-space qualified values).
typedef float nf2 __attribute__((ext_vector_type(2)));
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
template <typename V>
__device__ __forceinline__ V ld_c(const V DSBT_GLOBAL* p, int i) {
    if constexpr (sizeof(V) == sizeof(float2)) {
        const nf2 v = reinterpret_cast<const nf2 DSBT_GLOBAL*>(p)[i];
        return V{v.x, v.y};
    } else {
        const nd2 v = reinterpret_cast<const nd2 DSBT_GLOBAL*>(p)[i];
        return V{v.x, v.y};
    }
}

// A unit number w = h + l (l = 0 for FP64 arithmetic) and a product by it.
template <typename V> struct Unit {
    V h, l;
};
template <typename V>
__device__ __forceinline__ V u_mul(V a, const Unit<V>& w) {
    if constexpr (sizeof(V) == sizeof(float2)) return mul_unit(a, w.h, w.l);
    else return f_mul(a, w.h);
}
template <typename V>
__device__ __forceinline__ Unit<V> unit_at(const V DSBT_GLOBAL* hi, const V DSBT_GLOBAL* lo, int i) {
    if constexpr (sizeof(V) == sizeof(float2)) return {ld_c(hi, i), ld_c(lo, i)};
    else return {ld_c(hi, i), V{0, 0}};
}
template <typename V, typename T>
__device__ __forceinline__ V f_scale(V a, Split<T> c) { return {s_mul(a.x, c), s_mul(a.y, c)}; }
template <typename V> __device__ __forceinline__ V f_negi(V a) { return {a.y, -a.x}; }   // -i a
template <typename V> __device__ __forceinline__ V f_posi(V a) { return {-a.y, a.x}; }   // +i a

__device__ __forceinline__ int pidx(int i) { return i + (i >> 5); }   // one LDS pad per 32 values

// in-register DFTs with the forward sign exp(-2 pi i jk/R)
template <typename T, typename V>
__device__ __forceinline__ void dft2(V& a, V& b) {
    const V t = a;
    a = f_add(t, b);
    b = f_sub(t, b);
}
template <typename T, typename V>
__device__ __forceinline__ void dft4(V* v) {
    const V a0 = f_add(v[0], v[2]), a1 = f_sub(v[0], v[2]);
    const V a2 = f_add(v[1], v[3]), a3 = f_negi(f_sub(v[1], v[3]));
    v[0] = f_add(a0, a2);
    v[2] = f_sub(a0, a2);
    v[1] = f_add(a1, a3);
    v[3] = f_sub(a1, a3);
}
template <typename T, typename V>
__device__ __forceinline__ void dft8(V* v) {
    // two radix-4 on even/odd, then combine with exp(-2 pi i k/8)
    V e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft4<T>(e);
    dft4<T>(o);
    V o1, o3;
    if constexpr (sizeof(T) == sizeof(float)) {
        // rotations by -pi/4 as three shears (t = tan(pi/8), s = -sin(pi/4)):
        // determinant one whatever the rounding of t and s, so no systematic
        // change of the modulus (the rounded constant sqrt(1/2) alone would
        // scale every value by the same factor)
        constexpr float tq = 0.41421356237309504880f, sq = -0.70710678118654752440f;
        auto rot = [](V a) {
            a.x = __builtin_fmaf(tq, a.y, a.x);
            a.y = __builtin_fmaf(sq, a.x, a.y);
            a.x = __builtin_fmaf(tq, a.y, a.x);
            return a;
        };
        o1 = rot(o[1]);                // o1 exp(-i pi/4)
        o3 = f_negi(rot(o[3]));        // o3 exp(-3 i pi/4)
    } else {
        constexpr T h = (T)0.70710678118654752440;
        o1 = {(o[1].x + o[1].y) * h, (o[1].y - o[1].x) * h};
        o3 = {(o[3].y - o[3].x) * h, -(o[3].x + o[3].y) * h};
    }
    const V o2 = f_negi(o[2]);         // o2 exp(-i pi/2)
    v[0] = f_add(e[0], o[0]);
    v[4] = f_sub(e[0], o[0]);
    v[1] = f_add(e[1], o1);
    v[5] = f_sub(e[1], o1);
    v[2] = f_add(e[2], o2);
    v[6] = f_sub(e[2], o2);
    v[3] = f_add(e[3], o3);
    v[7] = f_sub(e[3], o3);
}

// Table pointers are cast to the global address space (as_global): generic
// (flat) loads would also count against the LDS counter, so each LDS wait of
// the passes would wait for them too.
template <typename T> using TabPtr = const typename CV<T>::t DSBT_GLOBAL*;

// One quarter-circle root in LDS: FP64 (c, s), FP32 (c hi, s hi, c lo, s lo).
template <typename T> struct Root;
template <> struct Root<float> { typedef float t __attribute__((ext_vector_type(4))); };
template <> struct Root<double> { typedef double t __attribute__((ext_vector_type(2))); };

// Roots in LDS: e < N/4, or e <= N/8 (octant) where the quarter does not fit
// beside the data (FP64 arithmetic at N = 8192).
constexpr size_t kLdsMax = 160 * 1024;
// channels per block: N/8 threads each, at least 256 threads per block
constexpr int fstage_cpb(int N) { return N / 8 >= 256 ? 1 : 256 / (N / 8); }
template <typename T>
constexpr size_t fstage_root_offset(int N, int cpb) {
    return (sizeof(typename CV<T>::t) * (size_t)cpb * (N + N / 32) + 15) / 16 * 16;
}
template <typename T>
constexpr bool root_octant(int N) { return fstage_root_offset<T>(N, fstage_cpb(N)) + 16 * (size_t)(N / 4) > kLdsMax; }
template <typename T>
constexpr int root_count(int N) { return root_octant<T>(N) ? N / 8 + 1 : N / 4; }
// LDS slots of the roots: root e sits at slot root_slot(e), a permutation
// within each aligned group of 16 (so the table takes root_count rounded up to
// 16 slots) that spreads the power-of-two strides of the passes' reads over
// the LDS banks.
__device__ __forceinline__ int root_slot(int e) {
    return __builtin_amdgcn_ubfe(e ^ (e >> 4) ^ (e >> 8), 0, 4) | (e & ~15);
}
template <typename T>
constexpr size_t fstage_lds_bytes(int N, int cpb) {
    return fstage_root_offset<T>(N, cpb) + 16 * (size_t)((root_count<T>(N) + 15) / 16 * 16);
}

// z exp(-2 pi i m/N) for 0 <= m < Q N/4: z (c - i s) with the root of
// e = m mod N/4 (octant tables: the root of N/4 - e with c and s exchanged
// when e > N/8), then (-i)^q, q = m div N/4 < Q (exact swaps and sign changes).
template <typename T, int N, int Q>
__device__ __forceinline__ typename CV<T>::t root_mul(typename CV<T>::t z, const typename Root<T>::t* qt, int m) {
    using V = typename CV<T>::t;
    const int e = m & (N / 4 - 1);
    typename Root<T>::t w;
    if constexpr (root_octant<T>(N)) {
        const bool sw = e > N / 8;
        w = qt[root_slot(sw ? N / 4 - e : e)];
        if (sw) {
            if constexpr (sizeof(T) == sizeof(float)) w = w.yxwz;
            else w = w.yx;
        }
    } else {
        w = qt[root_slot(e)];
    }
    V y;
    if constexpr (sizeof(T) == sizeof(float)) y = mul_unit(z, V{w.x, -w.y}, V{w.z, -w.w});
    else y = f_mul(z, V{w.x, -w.y});
    if constexpr (Q > 1) {
        const int q = m / (N / 4);
        if (q & 1) y = f_negi(y);
        if constexpr (Q > 2) {
            if (q & 2) y = V{-y.x, -y.y};
        }
    }
    return y;
}

// v[r] *= w^r for r = R0 .. R - 1, w = exp(-2 pi i m1/N), m1 < N/R: r m1 spans
// ceil(4 r/R) quarter turns.
template <typename T, int N, int R, int R0 = 1>
__device__ __forceinline__ void twiddle_row(typename CV<T>::t* v, const typename Root<T>::t* qt, int m1) {
    if constexpr (R0 < R) {
        v[R0] = root_mul<T, N, (4 * R0 + R - 1) / R>(v[R0], qt, R0 * m1);
        twiddle_row<T, N, R, R0 + 1>(v, qt, m1);
    }
}

// One Stockham pass of radix R on the channel at buf (padded indexing);
// thread t of the channel owns butterflies j = t + u N/8, u < 8/R.
template <typename T, int N, int R>
__device__ __forceinline__ void fft_pass(typename CV<T>::t* buf, int Ns, const typename Root<T>::t* qt, int t) {
    using V = typename CV<T>::t;
    constexpr int NR = N / R, U = 8 / R;
    V v[U][R];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = t + u * (N / 8);
#pragma unroll
        for (int r = 0; r < R; ++r) v[u][r] = buf[pidx(j + r * NR)];
        const int jm = j & (Ns - 1);
        // w^r, w = exp(-2 pi i jm/(Ns R)) = exp(-2 pi i m1/N)
        if (Ns > 1) twiddle_row<T, N, R>(v[u], qt, jm * (N / (Ns * R)));
        if constexpr (R == 8) dft8<T>(v[u]);
        else if constexpr (R == 4) dft4<T>(v[u]);
        else dft2<T>(v[u][0], v[u][1]);
    }
    lds_barrier();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = t + u * (N / 8);
        const int jm = j & (Ns - 1);
        const int base = (j - jm) * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pidx(base + r * Ns)] = v[u][r];
    }
    lds_barrier();
}

template <typename T, int N>
__device__ __forceinline__ void fft_n(typename CV<T>::t* buf, const typename Root<T>::t* qt, int t) {
    constexpr int L = __builtin_ctz(N);
    int Ns = 1;
#pragma unroll
    for (int s = 0; s < L / 3; ++s) {
        fft_pass<T, N, 8>(buf, Ns, qt, t);
        Ns *= 8;
    }
    if constexpr (L % 3 == 1) fft_pass<T, N, 2>(buf, Ns, qt, t);
    if constexpr (L % 3 == 2) fft_pass<T, N, 4>(buf, Ns, qt, t);
}

// The potential factor exp(-i s V tau/2) of point i: from the plan's table
// when every strength is one, else from the FP64 angle s V tau/2 reduced mod
// 2 pi, then sine and cosine in the arithmetic precision (lo = 0: the factors
// change from step to step, so their rounding does not add up to a drift).
template <typename V>
__device__ __forceinline__ Unit<V> phase_factor(const FChan& c, int i, const PhaseArgs& ph) {
    Unit<V> z;
    if (ph.scale == nullptr) {
        z = unit_at(as_global(static_cast<const V*>(c.vphase)), as_global(static_cast<const V*>(c.vphase_lo)), i);
    } else {
        double a = (double)ph.scale[ph.step] * as_global(c.vangle)[i];
        const double twopi = 6.283185307179586476925286766559;
        a -= twopi * rint(a / twopi);
        if constexpr (sizeof(V) == sizeof(float2)) {
            float sn, cs;
            sincosf((float)a, &sn, &cs);
            z.h = V{cs, -sn};
        } else {
            double sn, cs;
            sincos(a, &sn, &cs);
            z.h = V{cs, -sn};
        }
        z.l = V{0, 0};
    }
    if (ph.conj) {
        z.h.y = -z.h.y;
        z.l.y = -z.l.y;
    }
    return z;
}

constexpr int fstage_threads(int N) { return N / 8 >= 256 ? N / 8 : 256; }

// Two consecutive complex values of the data precision as one vector access
// (8-byte aligned for complex64: channel offsets may be odd).
template <typename S> struct Pair;
template <> struct Pair<float> { typedef float t __attribute__((ext_vector_type(4), aligned(8))); };
template <> struct Pair<double> { typedef double t __attribute__((ext_vector_type(4), aligned(16))); };

// Complex value conversion between the storage and the arithmetic precision.
template <typename V, typename W> __device__ __forceinline__ V to_prec(W w) {
    return {(decltype(V{}.x))w.x, (decltype(V{}.x))w.y};
}

// T: arithmetic and table precision; S: data precision in memory.  MODE 0:
// forward F (phases ph on the input); 1: inverse F^T (phases ph on the
// output); 2: F^T then F on the same channels (one step's inverse, then the
// next step's forward), the two steps' phases ph and ph2 applied in LDS
// between them -- exactly the products the two separate launches make, with
// one pass over the data instead of two.
// The work of one block: channel group `group` (cpb channels of N/8 threads
// each) of the nch channels at chans.
template <typename T, typename S, int N, int MODE>
__device__ __forceinline__ void fstage_body(const FChan* __restrict__ chans, int nch, int cpb, int group,
                                            const typename CV<S>::t* src, typename CV<S>::t* dst, PhaseArgs ph,
                                            PhaseArgs ph2, typename CV<S>::t* mid) {
    using V = typename CV<T>::t;
    using SV = typename CV<S>::t;
    using P2 = typename Pair<S>::t;
    constexpr int TPC = N / 8;              // threads per channel
    constexpr int PADN = N + N / 32;        // padded LDS slots per channel
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int cl = threadIdx.x / TPC, t = threadIdx.x % TPC;
    const int cidx = group * cpb + cl;
    V* buf = reinterpret_cast<V*>(smem_raw) + cl * PADN;
    // a block's last slots may be past the channel list: they take part in the
    // barriers on a copy of the last descriptor (valid tables) and store nothing
    const bool live = cidx < nch;
    const FChan c = chans[live ? cidx : nch - 1];
    // the quarter-circle roots (all channels of a block have the same N) after the data
    using RT = typename Root<T>::t;
    RT* qt = reinterpret_cast<RT*>(smem_raw + fstage_root_offset<T>(N, cpb));
    {
        const RT DSBT_GLOBAL* g = as_global(static_cast<const RT*>(c.roots));
        for (int i = threadIdx.x; i < root_count<T>(N); i += blockDim.x) qt[root_slot(i)] = g[i];
    }
    const TabPtr<T> post = as_global(reinterpret_cast<const V*>(c.post));
    const TabPtr<T> postl = as_global(reinterpret_cast<const V*>(c.post_lo));
    // the sign (-1)^ceil(l/2) (an exact product); the orthonormal scales are in the post table
    const T sg = (T)c.sign;

    // forward: X_k for k = 2m, 2m + 1 from the FFT in buf, stored as one
    // 16-byte pair (reversed for the sine form)
    auto forward_out = [&]() {
        if (!live) return;
        SV* y = dst + c.off;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int m = t + u * TPC;
            SV o[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int k = 2 * m + e;
                // c w^k with the orthonormal scale c folded into the table
                const Unit<V> w = unit_at(post, postl, k);
                const V a = buf[pidx(k)], b = buf[pidx((N - k) & (N - 1))];
                // w a + conj(w) b = (w.x (a.x + b.x) + w.y (b.y - a.y), w.x (a.y + b.y) + w.y (a.x - b.x))
                const T sx = a.x + b.x, dy = b.y - a.y, sy = a.y + b.y, dx = a.x - b.x;
                V X;
                if constexpr (sizeof(T) == sizeof(float)) {
                    X = {__builtin_fmaf(w.h.x, sx, __builtin_fmaf(w.h.y, dy, w.l.x * sx + w.l.y * dy)),
                         __builtin_fmaf(w.h.x, sy, __builtin_fmaf(w.h.y, dx, w.l.x * sy + w.l.y * dx))};
                } else {
                    X = {w.h.x * sx + w.h.y * dy, w.h.x * sy + w.h.y * dx};
                }
                o[e] = to_prec<SV>(f_scale(X, sg));
            }
            if (c.p)
                *reinterpret_cast<P2*>(y + (N - 2 - 2 * m)) = P2{o[1].x, o[1].y, o[0].x, o[0].y};
            else
                *reinterpret_cast<P2*>(y + 2 * m) = P2{o[0].x, o[0].y, o[1].x, o[1].y};
        }
    };

    if constexpr (MODE == 0) {
        if (live) {
            // pairs x_{2j}, x_{2j+1} (one 16-byte load) go to v_j and v_{N-1-j}
            const SV* x = src + c.off;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = t + u * TPC;
                const P2 w = *reinterpret_cast<const P2*>(x + 2 * j);
                V a = to_prec<V>(SV{w[0], w[1]}), b = to_prec<V>(SV{w[2], w[3]});
                if (ph.use) {
                    a = u_mul(a, phase_factor<V>(c, 2 * j, ph));
                    b = u_mul(b, phase_factor<V>(c, 2 * j + 1, ph));
                }
                if (c.p) b = {-b.x, -b.y};
                buf[pidx(j)] = a;
                buf[pidx(N - 1 - j)] = b;
            }
        }
        lds_barrier();
        fft_n<T, N>(buf, qt, t);
        forward_out();
    } else {
        if (live) {
            // slots j = 2m, 2m + 1 loaded as one 16-byte pair
            const SV* f = src + c.off;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int m = t + u * TPC;
                const P2 v = *reinterpret_cast<const P2*>(f + 2 * m);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int j = 2 * m + e;
                    const int k = c.p ? (N - 1 - j) : j;
                    buf[pidx(k)] = f_scale(to_prec<V>(SV{v[2 * e], v[2 * e + 1]}), sg);
                }
            }
        }
        lds_barrier();
        // U = A^T S X (S the orthonormal scales): U_0 = sqrt(1/N) X_0 = 2 c_0 X_0,
        // U_j = (w^j/2) sqrt(2/N) (X_j + i X_{N-j}) = c w^j (X_j + i X_{N-j})
        V u8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = t + u * TPC;
            if (j == 0) {
                Unit<V> w0 = unit_at(post, postl, 0);
                w0.h = f_scale(w0.h, (T)2);
                w0.l = f_scale(w0.l, (T)2);
                u8[u] = u_mul(buf[0], w0);
            } else {
                const V s = f_add(buf[pidx(j)], f_posi(buf[pidx(N - j)]));
                u8[u] = u_mul(s, unit_at(post, postl, j));
            }
        }
        lds_barrier();
#pragma unroll
        for (int u = 0; u < 8; ++u) buf[pidx(t + u * TPC)] = u8[u];
        lds_barrier();
        fft_n<T, N>(buf, qt, t);
        if constexpr (MODE == 1) {
            if (live) {
                // v_j and v_{N-1-j} go out as the pair x_{2j}, x_{2j+1} (one 16-byte store)
                SV* x = dst + c.off;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = t + u * TPC;
                    V a = buf[pidx(j)], b = buf[pidx(N - 1 - j)];
                    if (c.p) b = {-b.x, -b.y};
                    if (ph.use) {
                        a = u_mul(a, phase_factor<V>(c, 2 * j, ph));
                        b = u_mul(b, phase_factor<V>(c, 2 * j + 1, ph));
                    }
                    const SV sa = to_prec<SV>(a), sb = to_prec<SV>(b);
                    *reinterpret_cast<P2*>(x + 2 * j) = P2{sa.x, sa.y, sb.x, sb.y};
                }
            }
        } else {
            // x_{2j} = v_j and x_{2j+1} = (-1)^p v_{N-1-j} take both steps' phases
            // and go back to slots j and N-1-j, where the forward transform reads
            // them (the two sign changes cancel); the data precision is kept
            // between the steps, as the separate launches do
            if (live) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = t + u * TPC;
                    V a = buf[pidx(j)], b = buf[pidx(N - 1 - j)];
                    if (ph.use) {
                        a = u_mul(a, phase_factor<V>(c, 2 * j, ph));
                        b = u_mul(b, phase_factor<V>(c, 2 * j + 1, ph));
                    }
                    const SV sa = to_prec<SV>(a), sb = to_prec<SV>(b);
                    if (mid) {
                        // the state between the two steps, as mode 1 stores it
                        const SV sbs = c.p ? SV{-sb.x, -sb.y} : sb;
                        *reinterpret_cast<P2*>(mid + c.off + 2 * j) = P2{sa.x, sa.y, sbs.x, sbs.y};
                    }
                    a = to_prec<V>(sa);
                    b = to_prec<V>(sb);
                    if (ph2.use) {
                        a = u_mul(a, phase_factor<V>(c, 2 * j, ph2));
                        b = u_mul(b, phase_factor<V>(c, 2 * j + 1, ph2));
                    }
                    buf[pidx(j)] = a;
                    buf[pidx(N - 1 - j)] = b;
                }
            }
            lds_barrier();
            fft_n<T, N>(buf, qt, t);
            forward_out();
        }
    }
}

template <typename T, typename S, int N, int MODE>
__global__ void __launch_bounds__(fstage_threads(N)) fstage_n(const FChan* __restrict__ chans, int nch, int cpb,
                                                const typename CV<S>::t* src, typename CV<S>::t* dst, PhaseArgs ph,
                                                PhaseArgs ph2, typename CV<S>::t* mid) {
    fstage_body<T, S, N, MODE>(chans, nch, cpb, blockIdx.x, src, dst, ph, ph2, mid);
}

// Every N of a plan in one launch: block b takes task b, a group of channels
// of one N with kMultiThreads / (N/8) channels (8192 points for N >= 16),
// and runs that N's body.  The plan lists the tasks largest N first, so the
// hardware dispatcher, which hands out blocks in index order as compute
// units free up, schedules the heaviest tasks first.
template <typename T, typename S, int MODE>
__global__ void __launch_bounds__(kMultiThreads) fstage_multi(const FTask* __restrict__ tasks,
                                                           const FChan* __restrict__ chans,
                                                           const typename CV<S>::t* src, typename CV<S>::t* dst,
                                                           PhaseArgs ph, PhaseArgs ph2, typename CV<S>::t* mid) {
    const FTask task = tasks[blockIdx.x];
    const FChan* c = chans + task.first;
#define DSBT_MB(NN)                                                                                      \
    case NN:                                                                                             \
        fstage_body<T, S, NN, MODE>(c, task.count, kMultiThreads / (NN / 8), 0, src, dst, ph, ph2, mid); \
        break;
    switch (task.N) {
        DSBT_MB(16) DSBT_MB(32) DSBT_MB(64) DSBT_MB(128) DSBT_MB(256) DSBT_MB(512) DSBT_MB(1024)
        DSBT_MB(2048) DSBT_MB(4096) DSBT_MB(8192)
        default: break;
    }
#undef DSBT_MB
}

// Threads per block for size N and channels per block.
static inline void fstage_shape(int N, int& cpb, int& threads) {
    const int tpc = N / 8;
    cpb = fstage_cpb(N);
    threads = tpc * cpb;
}

template <typename T, typename S, int MODE>
static hipError_t launch_n(int N, const FChan* d, int nch, const void* src, void* dst, PhaseArgs ph, PhaseArgs ph2,
                           void* mid, hipStream_t s) {
    using SV = typename CV<S>::t;
    int cpb, threads;
    fstage_shape(N, cpb, threads);
    const int blocks = (nch + cpb - 1) / cpb;
    const size_t lds = fstage_lds_bytes<T>(N, cpb);
#define DSBT_FN(NN)                                                                                      \
    case NN:                                                                                             \
        hipLaunchKernelGGL((fstage_n<T, S, NN, MODE>), dim3(blocks), dim3(threads), lds, s, d, nch, cpb, \
                           (const SV*)src, (SV*)dst, ph, ph2, (SV*)mid);                                 \
        break;
    switch (N) {
        DSBT_FN(16) DSBT_FN(32) DSBT_FN(64) DSBT_FN(128) DSBT_FN(256) DSBT_FN(512) DSBT_FN(1024)
        DSBT_FN(2048) DSBT_FN(4096) DSBT_FN(8192)
        default: return hipErrorInvalidValue;
    }
#undef DSBT_FN
    return hipGetLastError();
}

template <typename T, typename S>
hipError_t launch_fstage_n(int N, const FChan* d_chans, int nch, const void* src, void* dst, bool inverse,
                           PhaseArgs ph, hipStream_t s) {
    if (nch <= 0) return hipSuccess;
    return inverse ? launch_n<T, S, 1>(N, d_chans, nch, src, dst, ph, PhaseArgs{}, nullptr, s)
                   : launch_n<T, S, 0>(N, d_chans, nch, src, dst, ph, PhaseArgs{}, nullptr, s);
}

template <typename T, typename S>
hipError_t launch_fstage_inv_fwd(int N, const FChan* d_chans, int nch, void* data, void* mid, PhaseArgs ph_inv,
                                 PhaseArgs ph_fwd, hipStream_t s) {
    if (nch <= 0) return hipSuccess;
    return launch_n<T, S, 2>(N, d_chans, nch, data, data, ph_inv, ph_fwd, mid, s);
}

template <typename T>
size_t fstage_multi_lds(int N) {
    return fstage_lds_bytes<T>(N, kMultiThreads / (N / 8));
}

template <typename T, typename S>
hipError_t launch_fstage_multi(const FTask* d_tasks, int ntasks, const FChan* d_chans, const void* src, void* dst,
                               void* mid, int mode, PhaseArgs ph, PhaseArgs ph2, size_t lds, hipStream_t s) {
    using SV = typename CV<S>::t;
    if (ntasks <= 0) return hipSuccess;
    const dim3 grid(ntasks), block(kMultiThreads);
    const SV* in = (const SV*)src;
    SV* out = (SV*)dst;
    SV* mi = (SV*)mid;
    if (mode == 0)
        hipLaunchKernelGGL((fstage_multi<T, S, 0>), grid, block, lds, s, d_tasks, d_chans, in, out, ph, ph2, mi);
    else if (mode == 1)
        hipLaunchKernelGGL((fstage_multi<T, S, 1>), grid, block, lds, s, d_tasks, d_chans, in, out, ph, ph2, mi);
    else
        hipLaunchKernelGGL((fstage_multi<T, S, 2>), grid, block, lds, s, d_tasks, d_chans, in, out, ph, ph2, mi);
    return hipGetLastError();
}

template <typename T, typename S, int MODE>
static hipError_t lds_attr_all() {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f, int N) {
        int cpb, threads;
        fstage_shape(N, cpb, threads);
        const size_t lds = fstage_lds_bytes<T>(N, cpb);
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    };
    set((const void*)fstage_n<T, S, 16, MODE>, 16);
    set((const void*)fstage_n<T, S, 32, MODE>, 32);
    set((const void*)fstage_n<T, S, 64, MODE>, 64);
    set((const void*)fstage_n<T, S, 128, MODE>, 128);
    set((const void*)fstage_n<T, S, 256, MODE>, 256);
    set((const void*)fstage_n<T, S, 512, MODE>, 512);
    set((const void*)fstage_n<T, S, 1024, MODE>, 1024);
    set((const void*)fstage_n<T, S, 2048, MODE>, 2048);
    set((const void*)fstage_n<T, S, 4096, MODE>, 4096);
    set((const void*)fstage_n<T, S, 8192, MODE>, 8192);
    return e;
}

template <typename T>
hipError_t set_lds_limits_fstage_n() {
    hipError_t e = hipSuccess;
    auto multi = [&](const void* f) {
        size_t most = 0;
        for (int N = 16; N <= 8192; N *= 2) most = std::max(most, fstage_multi_lds<T>(N));
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)most);
    };
    multi((const void*)fstage_multi<T, T, 0>);
    multi((const void*)fstage_multi<T, T, 1>);
    multi((const void*)fstage_multi<T, T, 2>);
    if constexpr (sizeof(T) == sizeof(double)) {
        multi((const void*)fstage_multi<double, float, 0>);
        multi((const void*)fstage_multi<double, float, 1>);
        multi((const void*)fstage_multi<double, float, 2>);
    }
    if (e == hipSuccess) e = lds_attr_all<T, T, 0>();
    if (e == hipSuccess) e = lds_attr_all<T, T, 1>();
    if (e == hipSuccess) e = lds_attr_all<T, T, 2>();
    if constexpr (sizeof(T) == sizeof(double)) {
        if (e == hipSuccess) e = lds_attr_all<double, float, 0>();
        if (e == hipSuccess) e = lds_attr_all<double, float, 1>();
        if (e == hipSuccess) e = lds_attr_all<double, float, 2>();
    }
    return e;
}

template hipError_t launch_fstage_n<float, float>(int, const FChan*, int, const void*, void*, bool, PhaseArgs,
                                                  hipStream_t);
template hipError_t launch_fstage_n<double, double>(int, const FChan*, int, const void*, void*, bool, PhaseArgs,
                                                    hipStream_t);
template hipError_t launch_fstage_n<double, float>(int, const FChan*, int, const void*, void*, bool, PhaseArgs,
                                                   hipStream_t);
template hipError_t launch_fstage_inv_fwd<float, float>(int, const FChan*, int, void*, void*, PhaseArgs, PhaseArgs,
                                                         hipStream_t);
template hipError_t launch_fstage_inv_fwd<double, double>(int, const FChan*, int, void*, void*, PhaseArgs, PhaseArgs,
                                                           hipStream_t);
template hipError_t launch_fstage_inv_fwd<double, float>(int, const FChan*, int, void*, void*, PhaseArgs, PhaseArgs,
                                                          hipStream_t);
template size_t fstage_multi_lds<float>(int);
template size_t fstage_multi_lds<double>(int);
template hipError_t launch_fstage_multi<float, float>(const FTask*, int, const FChan*, const void*, void*, void*, int,
                                                      PhaseArgs, PhaseArgs, size_t, hipStream_t);
template hipError_t launch_fstage_multi<double, double>(const FTask*, int, const FChan*, const void*, void*, void*,
                                                        int, PhaseArgs, PhaseArgs, size_t, hipStream_t);
template hipError_t launch_fstage_multi<double, float>(const FTask*, int, const FChan*, const void*, void*, void*,
                                                       int, PhaseArgs, PhaseArgs, size_t, hipStream_t);
template hipError_t set_lds_limits_fstage_n<float>();
template hipError_t set_lds_limits_fstage_n<double>();

}  // namespace dsbt
