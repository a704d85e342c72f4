// HIP kernels of the orthogonal DSBT for CDNA4 (gfx950).
//
// Stage F (Sec. 2.2, eq. csFourierBasis): the orthonormal DCT-II (odd l) or
// DST-II (even l) of a complex channel through one N-point complex FFT held in
// LDS: the DST is the DCT of (-1)^i x read backwards; the DCT reorders
// v_j = x_2j, v_{N-1-j} = x_{2j+1}, transforms, and combines
// X_k = (w^k V_k + w^-k V_{N-k}) / 2 with w = exp(-i pi/(2N)) (the
// complex-linear form of the real-input identity).  The inverse is the exact
// transpose of that chain (it also uses the forward FFT, which is symmetric).
//
// Stage M (Sec. 2.4-2.5): the Fourier-to-Bessel matrix T applied as a sequence
// of tile steps [b_J; mu_J+1] = M_J [g_J; mu_J] (forward) or
// [h_J; lam_J] = M_J^T [y_J; lam_J+1] (inverse, tiles in reverse).  Several
// channels with the same (l, N) share each load of a table entry.
#include "kernels.h"

namespace dsbt {

template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return {a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return {a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cconjmul(V a, V b) {  // conj(a) * b
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) { return {a.x * s, a.y * s}; }
template <typename V> __device__ __forceinline__ V cmul_negi(V a) { return {a.y, -a.x}; }  // -i a
template <typename V> __device__ __forceinline__ V cmul_posi(V a) { return {-a.y, a.x}; }  // +i a

template <typename V> __device__ __forceinline__ V from_f2(float2 z);
template <> __device__ __forceinline__ float2 from_f2<float2>(float2 z) { return z; }
template <> __device__ __forceinline__ double2 from_f2<double2>(float2 z) { return {(double)z.x, (double)z.y}; }

// Phase factor of point i of a channel: the unit-modulus table when every
// step has strength one, otherwise exp(-i s angle) from the FP64 angle reduced
// mod 2 pi before the FP32 sine/cosine.
template <typename V>
__device__ __forceinline__ V vphase_at(const FChan& c, int i, const PhaseArgs& ph) {
    float2 z;
    if (ph.scale == nullptr) {
        z = c.vphase[i];
    } else {
        const double s = (double)ph.scale[ph.step];
        double a = s * c.vangle[i];
        const double twopi = 6.283185307179586476925286766559;
        a -= twopi * rint(a / twopi);
        float sn, cs;
        sincosf((float)a, &sn, &cs);
        z = make_float2(cs, -sn);
    }
    if (ph.conj) z.y = -z.y;
    return from_f2<V>(z);
}

// ---------------------------------------------------------------------------
// LDS FFT: Stockham autosort, radix 4 (and one radix-2 stage for odd log2 N).
// buf holds N complex values; every thread of the block takes part.
// ---------------------------------------------------------------------------

template <int R, typename V>
__device__ __forceinline__ void dft_small(V* v) {
    if constexpr (R == 2) {
        const V a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else {
        const V a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        const V a2 = cadd(v[1], v[3]), a3 = cmul_negi(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    }
}

template <int R, int MAXU, typename V>
__device__ __forceinline__ void stockham_stage(V* buf, int N, int Ns, const V* tw, int tid) {
    const int NR = N / R;
    const int stride = N / (Ns * R);  // twiddle exp(-2 pi i r jm/(Ns R)) = tw[r jm stride]
    V v[MAXU][R];
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
        const int j = tid + u * kBlock;
        if (j < NR) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = buf[j + r * NR];
            const int jm = j & (Ns - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], tw[r * jm * stride]);
            dft_small<R>(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXU; ++u) {
        const int j = tid + u * kBlock;
        if (j < NR) {
            const int jm = j & (Ns - 1);
            const int base = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[u][r];
        }
    }
    __syncthreads();
}

// N = 2^log2N in [16, 8192]; kBlock threads.
template <typename V>
__device__ void lds_fft(V* buf, int N, int log2N, const V* tw, int tid) {
    int Ns = 1;
    if (log2N & 1) {
        stockham_stage<2, 16>(buf, N, Ns, tw, tid);
        Ns = 2;
    }
    while (Ns < N) {
        stockham_stage<4, 8>(buf, N, Ns, tw, tid);
        Ns *= 4;
    }
}

// ---------------------------------------------------------------------------
// Stage F kernels: one workgroup per channel.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock) fstage_fwd(const FChan* __restrict__ chans,
                                                     const typename C2<T>::t* src,
                                                     typename C2<T>::t* dst,
                                                     PhaseArgs ph) {
    using V = typename C2<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* buf = reinterpret_cast<V*>(smem_raw);
    const FChan c = chans[blockIdx.x];
    const int N = c.N, tid = threadIdx.x;
    const V* x = src + c.off;
    // pre-permutation: v_j = x_2j, v_{N-1-j} = x_{2j+1}; even l first flips (-1)^i
    for (int i = tid; i < N; i += kBlock) {
        V a = x[i];
        if (ph.use) a = cmul(a, vphase_at<V>(c, i, ph));
        if (c.p && (i & 1)) a = {-a.x, -a.y};
        const int pos = (i & 1) ? (N - 1 - (i >> 1)) : (i >> 1);
        buf[pos] = a;
    }
    __syncthreads();
    lds_fft(buf, N, c.log2N, reinterpret_cast<const V*>(c.tw), tid);
    const V* post = reinterpret_cast<const V*>(c.post);
    const T s0 = (T)c.sign * sqrt((T)1 / (T)N), s1 = (T)c.sign * sqrt((T)2 / (T)N);
    V* y = dst + c.off;
    for (int k = tid; k < N; k += kBlock) {
        const V w = post[k];
        const V a = buf[k], b = buf[(N - k) & (N - 1)];
        V X = cadd(cmul(w, a), cconjmul(w, b));   // w a + conj(w) b
        X = cscale(X, (T)0.5 * (k == 0 ? s0 : s1));
        y[c.p ? (N - 1 - k) : k] = X;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) fstage_inv(const FChan* __restrict__ chans,
                                                     const typename C2<T>::t* src,
                                                     typename C2<T>::t* dst,
                                                     PhaseArgs ph) {
    using V = typename C2<T>::t;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* buf = reinterpret_cast<V*>(smem_raw);
    const FChan c = chans[blockIdx.x];
    const int N = c.N, tid = threadIdx.x;
    const T s0 = (T)c.sign * sqrt((T)1 / (T)N), s1 = (T)c.sign * sqrt((T)2 / (T)N);
    const V* f = src + c.off;
    // X_k = scale_k sigma f_slot(k), slot(k) = k (odd l) or N-1-k (even l)
    for (int j = tid; j < N; j += kBlock) {
        const int k = c.p ? (N - 1 - j) : j;
        buf[k] = cscale(f[j], k == 0 ? s0 : s1);
    }
    __syncthreads();
    // U = A^T X: U_0 = X_0, U_j = (w^j / 2)(X_j + i X_{N-j})
    const V* post = reinterpret_cast<const V*>(c.post);
    constexpr int MAXU = 8192 / kBlock;
    V u[MAXU];
#pragma unroll
    for (int t = 0; t < MAXU; ++t) {
        const int j = tid + t * kBlock;
        if (j < N) {
            if (j == 0) {
                u[t] = buf[0];
            } else {
                const V s = cadd(buf[j], cmul_posi(buf[N - j]));
                u[t] = cscale(cmul(post[j], s), (T)0.5);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXU; ++t) {
        const int j = tid + t * kBlock;
        if (j < N) buf[j] = u[t];
    }
    __syncthreads();
    lds_fft(buf, N, c.log2N, reinterpret_cast<const V*>(c.tw), tid);
    V* x = dst + c.off;
    for (int i = tid; i < N; i += kBlock) {
        V a = (i & 1) ? buf[N - 1 - (i >> 1)] : buf[i >> 1];
        if (c.p && (i & 1)) a = {-a.x, -a.y};
        if (ph.use) a = cmul(a, vphase_at<V>(c, i, ph));
        x[i] = a;
    }
}

// ---------------------------------------------------------------------------
// Stage M: tiled moment form of T.  Thread (r, cs): row r of the block
// product for the channels cs, cs + NS, ... of the item, NS = kBlock / RP.
// LDS holds X[c][0..R): the tile data (B) followed by the moments (k).
// ---------------------------------------------------------------------------

template <typename T, int RP>
__global__ void __launch_bounds__(kBlock) mstage(const MItem* __restrict__ items,
                                                 const typename C2<T>::t* src,
                                                 typename C2<T>::t* dst,
                                                 int inverse, PhaseArgs ph) {
    using V = typename C2<T>::t;
    constexpr int NS = kBlock / RP;
    constexpr int CPT = (kMaxChanPerItem + NS - 1) / NS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    V* X = reinterpret_cast<V*>(smem_raw);
    const MItem& it = items[blockIdx.x];
    const int B = it.B, k = it.k, R = it.R, NT = it.NT, p = it.p, nch = it.nch;
    const int tid = threadIdx.x;
    const int r = tid % RP, cs = tid / RP;
    const T* tab = reinterpret_cast<const T*>(inverse ? it.tab_i : it.tab_f);
    const T sgn = p ? (T)-1 : (T)1;      // completion rows = (-1)^p mu_NT
    const T w0 = p ? (T)1 : (T)0.70710678118654752440;  // w_m at m = 0 (odd l)

    // initial moments: forward mu_0 = 0; inverse lam_NT = (-1)^p b[0..k)
    for (int e = tid; e < nch * k; e += kBlock) {
        const int ch = e / k, kk = e % k;
        V v = {(T)0, (T)0};
        if (inverse) {
            v = src[it.off[ch] + kk];
            if (ph.use && it.kphase) {
                float2 z = it.kphase[kk];
                if (ph.conj) z.y = -z.y;
                v = cmul(v, from_f2<V>(z));
            }
            v = cscale(v, sgn);
        }
        X[ch * R + B + kk] = v;
    }
    for (int step = 0; step < NT; ++step) {
        const int J = inverse ? (NT - 1 - step) : step;
        // load the tile data: forward g = w f, inverse y = b (kinetic phase if asked)
        for (int e = tid; e < nch * B; e += kBlock) {
            const int ch = e / B, s = e % B;
            const int slot = J * B + s;
            V v = src[it.off[ch] + slot];
            if (!inverse) {
                if (slot == 0) v = cscale(v, w0);
            } else if (ph.use && it.kphase) {
                float2 z = it.kphase[slot];
                if (ph.conj) z.y = -z.y;
                v = cmul(v, from_f2<V>(z));
            }
            X[ch * R + s] = v;
        }
        __syncthreads();
        V acc[CPT];
#pragma unroll
        for (int u = 0; u < CPT; ++u) acc[u] = {(T)0, (T)0};
        if (r < R) {
            const T* A = tab + (size_t)J * R * R + r;
            for (int q = 0; q < R; ++q) {
                const T a = A[(size_t)q * R];
#pragma unroll
                for (int u = 0; u < CPT; ++u) {
                    const int ch = cs + u * NS;
                    if (ch < nch) {
                        const V x = X[ch * R + q];
                        acc[u].x += a * x.x;
                        acc[u].y += a * x.y;
                    }
                }
            }
        }
        __syncthreads();
        if (r < R) {
#pragma unroll
            for (int u = 0; u < CPT; ++u) {
                const int ch = cs + u * NS;
                if (ch >= nch) continue;
                if (r >= B) {
                    X[ch * R + r] = acc[u];          // next moments
                } else {
                    const int slot = J * B + r;
                    V v = acc[u];
                    if (!inverse) {
                        if (J == 0 && r < k) continue;   // completion rows written last
                        if (ph.use && it.kphase) {
                            float2 z = it.kphase[slot];
                            if (ph.conj) z.y = -z.y;
                            v = cmul(v, from_f2<V>(z));
                        }
                    } else if (slot == 0) {
                        v = cscale(v, w0);
                    }
                    dst[it.off[ch] + slot] = v;
                }
            }
        }
    }
    if (!inverse) {
        __syncthreads();
        for (int e = tid; e < nch * k; e += kBlock) {
            const int ch = e / k, kk = e % k;
            V v = cscale(X[ch * R + B + kk], sgn);
            if (ph.use && it.kphase) {
                float2 z = it.kphase[kk];
                if (ph.conj) z.y = -z.y;
                v = cmul(v, from_f2<V>(z));
            }
            dst[it.off[ch] + kk] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Reduction for the strength gradient of a step.
// ---------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock) grad_s_partial(const FChan* __restrict__ chans,
                                                         const typename C2<T>::t* p0,
                                                         const typename C2<T>::t* p1,
                                                         const typename C2<T>::t* l0,
                                                         const typename C2<T>::t* l1,
                                                         double* __restrict__ part) {
    const FChan c = chans[blockIdx.x];
    double acc = 0.0;
    for (int i = threadIdx.x; i < c.N; i += kBlock) {
        const int64_t g = c.off + i;
        const double a = (double)l1[g].x * p1[g].y - (double)l1[g].y * p1[g].x
                       + (double)l0[g].x * p0[g].y - (double)l0[g].y * p0[g].x;
        acc += c.vangle[i] * a;
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kBlock) sum_partials(const double* __restrict__ part, int n,
                                                       double* __restrict__ out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) acc += part[i];
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
hipError_t launch_fstage(const FChan* d_chans, int nch, int maxN, const void* src, void* dst,
                         bool inverse, PhaseArgs ph, hipStream_t s) {
    using V = typename C2<T>::t;
    if (nch <= 0) return hipSuccess;
    const size_t lds = sizeof(V) * (size_t)maxN;
    if (inverse) {
        hipLaunchKernelGGL(fstage_inv<T>, dim3(nch), dim3(kBlock), lds, s, d_chans, (const V*)src, (V*)dst, ph);
    } else {
        hipLaunchKernelGGL(fstage_fwd<T>, dim3(nch), dim3(kBlock), lds, s, d_chans, (const V*)src, (V*)dst, ph);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mstage(const MItem* d_items, int nitems, int maxR, const void* src, void* dst,
                         bool inverse, PhaseArgs ph, hipStream_t s) {
    using V = typename C2<T>::t;
    if (nitems <= 0) return hipSuccess;
    const size_t lds = sizeof(V) * (size_t)kMaxChanPerItem * maxR;
    if (maxR <= 64) {
        hipLaunchKernelGGL((mstage<T, 64>), dim3(nitems), dim3(kBlock), lds, s, d_items, (const V*)src,
                           (V*)dst, inverse ? 1 : 0, ph);
    } else if (maxR <= 128) {
        hipLaunchKernelGGL((mstage<T, 128>), dim3(nitems), dim3(kBlock), lds, s, d_items, (const V*)src,
                           (V*)dst, inverse ? 1 : 0, ph);
    } else {
        hipLaunchKernelGGL((mstage<T, 256>), dim3(nitems), dim3(kBlock), lds, s, d_items, (const V*)src,
                           (V*)dst, inverse ? 1 : 0, ph);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_s(const FChan* d_chans, int nch, const void* p0, const void* p1, const void* l0,
                         const void* l1, double* scratch, double* out, hipStream_t s) {
    using V = typename C2<T>::t;
    hipLaunchKernelGGL(grad_s_partial<T>, dim3(nch), dim3(kBlock), 0, s, d_chans, (const V*)p0, (const V*)p1,
                       (const V*)l0, (const V*)l1, scratch);
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(kBlock), 0, s, scratch, nch, out);
    return hipGetLastError();
}

template <typename T>
hipError_t set_lds_limits(size_t fstage_bytes, size_t mstage_bytes) {
    hipError_t e;
    e = hipFuncSetAttribute((const void*)fstage_fwd<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fstage_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)fstage_inv<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fstage_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)mstage<T, 64>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mstage_bytes);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)mstage<T, 128>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mstage_bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)mstage<T, 256>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mstage_bytes);
}

template hipError_t set_lds_limits<float>(size_t, size_t);
template hipError_t set_lds_limits<double>(size_t, size_t);
template hipError_t launch_fstage<float>(const FChan*, int, int, const void*, void*, bool, PhaseArgs, hipStream_t);
template hipError_t launch_fstage<double>(const FChan*, int, int, const void*, void*, bool, PhaseArgs, hipStream_t);
template hipError_t launch_mstage<float>(const MItem*, int, int, const void*, void*, bool, PhaseArgs, hipStream_t);
template hipError_t launch_mstage<double>(const MItem*, int, int, const void*, void*, bool, PhaseArgs, hipStream_t);
template hipError_t launch_grad_s<float>(const FChan*, int, const void*, const void*, const void*, const void*,
                                         double*, double*, hipStream_t);
template hipError_t launch_grad_s<double>(const FChan*, int, const void*, const void*, const void*, const void*,
                                          double*, double*, hipStream_t);

}  // namespace dsbt
