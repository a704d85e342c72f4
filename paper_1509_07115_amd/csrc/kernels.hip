// HIP kernels of the orthogonal DSBT for CDNA4 (gfx950): the generic moment
// stage (complex128 plans and items the matrix-core kernel does not take) and
// the reduction of the strength gradient.  The sine/cosine stage lives in
// fstage.hip, the matrix-core moment stage in mstage_mfma.hip.
//
// Stage M (Sec. 2.4-2.5): the Fourier-to-Bessel matrix T applied as a sequence
// of tile steps [b_J; mu_J+1] = M_J [g_J; mu_J] (forward) or
// [h_J; lam_J] = M_J^T [y_J; lam_J+1] (inverse, tiles in reverse).  Several
// channels with the same (l, N) share each load of a table entry.
#include "kernels.h"

#include <type_traits>

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

// ---------------------------------------------------------------------------
// Stage M: tiled moment form of T.  Thread (r, cs): row r of the block
// product for the channels cs, cs + NS, ... of the item, NS = kBlock / RP.
// LDS holds X[c][0..R): the tile data (B) followed by the moments (k).
// ---------------------------------------------------------------------------

// Complex value conversion between the storage and the arithmetic precision.
template <typename V, typename W> __device__ __forceinline__ V cvt(W w) {
    return {(decltype(V{}.x))w.x, (decltype(V{}.x))w.y};
}

// v times the kinetic factor of slot i of an item (conjugated for the adjoint
// step); FP32 factors carry hi + lo parts (kernels.h).
template <typename V>
__device__ __forceinline__ V kin_factor(const MItem& it, V v, int i, bool cj) {
    V z = static_cast<const V*>(it.kphase)[i];
    if (cj) z.y = -z.y;
    if constexpr (sizeof(V) == sizeof(float2)) {
        V l = static_cast<const V*>(it.kphase_lo)[i];
        if (cj) l.y = -l.y;
        return mul_unit(v, z, l);
    } else {
        return cmul(v, z);
    }
}

// T: arithmetic (and table) precision; S: data precision in memory.
template <typename T, typename S, int RP>
__global__ void __launch_bounds__(kBlock) mstage(const MItem* __restrict__ items,
                                                 const typename C2<S>::t* src,
                                                 typename C2<S>::t* dst,
                                                 int inverse, PhaseArgs ph) {
    using V = typename C2<T>::t;
    using SV = typename C2<S>::t;
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
    // w_m at m = 0 (odd l): sqrt(1/2), as a compensated FP32 product (kernels.h)
    auto w0_scale = [&](V v) -> V {
        if (p) return v;
        constexpr double h = 0.70710678118654752440;
        if constexpr (sizeof(T) == sizeof(float)) {
            constexpr float hi = (float)h, lo = (float)(h - (double)(float)h);
            return {mul_const(v.x, hi, lo), mul_const(v.y, hi, lo)};
        } else {
            return cscale(v, (T)h);
        }
    };

    // initial moments: forward mu_0 = 0; inverse lam_NT = (-1)^p b[0..k)
    for (int e = tid; e < nch * k; e += kBlock) {
        const int ch = e / k, kk = e % k;
        V v = {(T)0, (T)0};
        if (inverse) {
            v = cvt<V>(src[it.off[ch] + kk]);
            if (ph.use && it.kphase) v = kin_factor(it, v, kk, ph.conj != 0);
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
            V v = cvt<V>(src[it.off[ch] + slot]);
            if (!inverse) {
                if (slot == 0) v = w0_scale(v);
            } else if (ph.use && it.kphase) {
                v = kin_factor(it, v, slot, ph.conj != 0);
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
                        if (ph.use && it.kphase) v = kin_factor(it, v, slot, ph.conj != 0);
                    } else if (slot == 0) {
                        v = w0_scale(v);
                    }
                    dst[it.off[ch] + slot] = cvt<SV>(v);
                }
            }
        }
    }
    if (!inverse) {
        __syncthreads();
        for (int e = tid; e < nch * k; e += kBlock) {
            const int ch = e / k, kk = e % k;
            V v = cscale(X[ch * R + B + kk], sgn);
            if (ph.use && it.kphase) v = kin_factor(it, v, kk, ph.conj != 0);
            dst[it.off[ch] + kk] = cvt<SV>(v);
        }
    }
}

// ---------------------------------------------------------------------------
// Scan for non-finite values (checked plans).
// ---------------------------------------------------------------------------

__global__ void clear_flag(int* flag) { flag[threadIdx.x] = 0; }

template <typename S>
__global__ void __launch_bounds__(kBlock) scan_nonfinite(const FChan* __restrict__ chans, const S* data, int* flag) {
    const FChan c = chans[blockIdx.x];
    const S* x = data + 2 * c.off;
    bool bad = false;
    for (int i = threadIdx.x; i < 2 * c.N; i += kBlock) bad |= !isfinite(x[i]);
    if (bad) flag[0] = 1;
}

template <typename S>
hipError_t launch_scan_nonfinite(const FChan* d_chans, int nch, const void* data, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(clear_flag, dim3(1), dim3(1), 0, s, flag);
    if (nch > 0)
        hipLaunchKernelGGL(scan_nonfinite<S>, dim3(nch), dim3(kBlock), 0, s, d_chans, static_cast<const S*>(data), flag);
    return hipGetLastError();
}

template hipError_t launch_scan_nonfinite<float>(const FChan*, int, const void*, int*, hipStream_t);
template hipError_t launch_scan_nonfinite<double>(const FChan*, int, const void*, int*, hipStream_t);

// ---------------------------------------------------------------------------
// Reduction for the strength gradient of a step.
// ---------------------------------------------------------------------------

// Block (c, t): channel c of step t, whose vectors sit t stride elements
// after p0, p1, l0, l1; the partial goes to part[t nch + c].
template <typename T>
__global__ void __launch_bounds__(kBlock) grad_s_partial(const FChan* __restrict__ chans,
                                                         const typename C2<T>::t* p0,
                                                         const typename C2<T>::t* p1,
                                                         const typename C2<T>::t* l0,
                                                         const typename C2<T>::t* l1,
                                                         int64_t stride, double* __restrict__ part) {
    const FChan c = chans[blockIdx.x];
    const int64_t ts = stride * blockIdx.y;
    p0 += ts;
    p1 += ts;
    l0 += ts;
    l1 += ts;
    part += (size_t)blockIdx.y * gridDim.x;
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

// block t: out[t] = the sum of part[t n .. t n + n)
__global__ void __launch_bounds__(kBlock) sum_partials(const double* __restrict__ part, int n,
                                                       double* __restrict__ out) {
    part += (size_t)blockIdx.x * n;
    out += blockIdx.x;
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

template <typename T, typename S>
hipError_t launch_mstage(const MItem* d_items, int nitems, int maxR, const void* src, void* dst,
                         bool inverse, PhaseArgs ph, hipStream_t s) {
    using SV = typename C2<S>::t;
    using V = typename C2<T>::t;
    if (nitems <= 0) return hipSuccess;
    const size_t lds = sizeof(V) * (size_t)kMaxChanPerItem * maxR;
    if (maxR <= 64) {
        hipLaunchKernelGGL((mstage<T, S, 64>), dim3(nitems), dim3(kBlock), lds, s, d_items, (const SV*)src,
                           (SV*)dst, inverse ? 1 : 0, ph);
    } else if (maxR <= 128) {
        hipLaunchKernelGGL((mstage<T, S, 128>), dim3(nitems), dim3(kBlock), lds, s, d_items, (const SV*)src,
                           (SV*)dst, inverse ? 1 : 0, ph);
    } else {
        hipLaunchKernelGGL((mstage<T, S, 256>), dim3(nitems), dim3(kBlock), lds, s, d_items, (const SV*)src,
                           (SV*)dst, inverse ? 1 : 0, ph);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_s(const FChan* d_chans, int nch, const void* p0, const void* p1, const void* l0,
                         const void* l1, double* scratch, double* out, hipStream_t s) {
    using V = typename C2<T>::t;
    hipLaunchKernelGGL(grad_s_partial<T>, dim3(nch), dim3(kBlock), 0, s, d_chans, (const V*)p0, (const V*)p1,
                       (const V*)l0, (const V*)l1, (int64_t)0, scratch);
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(kBlock), 0, s, scratch, nch, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_s_steps(const FChan* d_chans, int nch, int nsteps, const void* states, const void* lams,
                               int64_t stride, double* scratch, double* out, hipStream_t s) {
    using V = typename C2<T>::t;
    if (nch <= 0 || nsteps <= 0) return hipSuccess;
    const V* p = static_cast<const V*>(states);
    const V* l = static_cast<const V*>(lams);
    hipLaunchKernelGGL(grad_s_partial<T>, dim3(nch, nsteps), dim3(kBlock), 0, s, d_chans, p, p + stride, l,
                       l + stride, stride, scratch);
    hipLaunchKernelGGL(sum_partials, dim3(nsteps), dim3(kBlock), 0, s, scratch, nch, out);
    return hipGetLastError();
}

template <typename T>
hipError_t set_lds_limits(size_t mstage_bytes) {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mstage_bytes);
    };
    set((const void*)mstage<T, T, 64>);
    set((const void*)mstage<T, T, 128>);
    set((const void*)mstage<T, T, 256>);
    if constexpr (std::is_same<T, double>::value) {
        set((const void*)mstage<double, float, 64>);
        set((const void*)mstage<double, float, 128>);
        set((const void*)mstage<double, float, 256>);
    }
    return e;
}

template hipError_t set_lds_limits<float>(size_t);
template hipError_t set_lds_limits<double>(size_t);
template hipError_t launch_mstage<float, float>(const MItem*, int, int, const void*, void*, bool, PhaseArgs,
                                                hipStream_t);
template hipError_t launch_mstage<double, double>(const MItem*, int, int, const void*, void*, bool, PhaseArgs,
                                                  hipStream_t);
template hipError_t launch_mstage<double, float>(const MItem*, int, int, const void*, void*, bool, PhaseArgs,
                                                 hipStream_t);
template hipError_t launch_grad_s<float>(const FChan*, int, const void*, const void*, const void*, const void*,
                                         double*, double*, hipStream_t);
template hipError_t launch_grad_s<double>(const FChan*, int, const void*, const void*, const void*, const void*,
                                          double*, double*, hipStream_t);
template hipError_t launch_grad_s_steps<float>(const FChan*, int, int, const void*, const void*, int64_t, double*,
                                               double*, hipStream_t);
template hipError_t launch_grad_s_steps<double>(const FChan*, int, int, const void*, const void*, int64_t, double*,
                                                double*, hipStream_t);

}  // namespace dsbt
