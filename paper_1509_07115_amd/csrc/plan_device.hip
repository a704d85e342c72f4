// FP64 plan generation on the GPU: the tile blocks M_J of the tiled moment
// form of T for one l, the same quantities as the host generator
// (plan_host.cpp), computed by three kernels:
//
//   plan_rows   one workgroup per regular row n >= n_0: the DLOP P_l(x, 2n-1),
//               x = 0..n (Sec. 2.3; degree recurrence when l^2 <= 2(2n-1),
//               else the Hahn difference equation marched in x), then the row
//               kappa_n(m) = P(n-m) - P(n-m-1), kappa_n(n) = 1, divided by its
//               weighted norm (Sec. 2.4 eq. Tdef/Ldef, rows normalised
//               numerically).
//   plan_basis  one workgroup per tile boundary t = p + J B: the k orthonormal
//               polynomials q_kk(m) = (-1)^d P_d(t-1-m, 2t-2), d = 2kk + p, on
//               m = 0..t-1 with the weight 1/2 at m = 0.
//   plan_blocks one workgroup per (tile, row of M_J): band entries and weighted
//               inner products over m < t_J.
//
// Scratch layout (doubles): row n at n(n+1)/2 - n_0(n_0+1)/2, n + 1 values;
// the basis of boundary J (J = 1..NT) at k ((J-1) p + B (J-1) J/2), k rows of
// t_J values.
#include "plan_device.h"

#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

namespace dsbt {

namespace {

constexpr int kPlanThreads = 256;

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the workgroup (kPlanThreads); red holds kPlanThreads/64 doubles.
__device__ double block_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    v = warp_sum(v);
    __syncthreads();
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kPlanThreads / 64; ++i) s += red[i];
    return s;
}

__host__ __device__ inline int64_t row_off(int n, int n0) {
    return (int64_t)n * (n + 1) / 2 - (int64_t)n0 * (n0 + 1) / 2;
}
__host__ __device__ inline int64_t basis_off(int J, int p, int B, int k) {
    return (int64_t)k * ((int64_t)(J - 1) * p + (int64_t)B * (J - 1) * J / 2);
}

// P_d(x, M), x = 0..xmax, by the degree recurrence
//   (j+1)(M-j) P_{j+1} = (2j+1)(M-2x) P_j - j(M+j+1) P_{j-1}
// for the x of this thread; coefA/coefC hold (2j+1)/((j+1)(M-j)) and
// j(M+j+1)/((j+1)(M-j)).
__device__ __forceinline__ double dlop_rec(int d, int M, int x, const double* coefA, const double* coefC) {
    if (d == 0) return 1.0;
    double a = 1.0, b = 1.0 - 2.0 * x / M;
    const double mx = (double)M - 2.0 * x;
    for (int j = 1; j < d; ++j) {
        const double c = coefA[j] * mx * b - coefC[j] * a;
        a = b;
        b = c;
    }
    return b;
}

__device__ void fill_coefs(int d, int M, double* coefA, double* coefC) {
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        const double den = (j + 1.0) * ((double)M - j);
        coefA[j] = (2.0 * j + 1.0) / den;
        coefC[j] = j * ((double)M + j + 1.0) / den;
    }
}

// Hahn difference equation in x (alpha = beta = 0), one thread:
//   B(x) y(x+1) = [d(d+1) + B(x) + D(x)] y(x) - D(x) y(x-1),
//   B(x) = (x+1)(x-M), D(x) = x(x-M-1), y(0) = 1.
template <typename Store>
__device__ void dlop_march(int d, int M, int xmax, Store store) {
    double ym = 1.0;
    store(0, ym);
    if (xmax < 1) return;
    double y = 1.0 - d * (d + 1.0) / M;
    store(1, y);
    const double lam = d * (d + 1.0);
    for (int x = 1; x < xmax; ++x) {
        const double Bx = (x + 1.0) * ((double)x - M), Dx = x * ((double)x - M - 1.0);
        const double yn = ((lam + Bx + Dx) * y - Dx * ym) / Bx;
        ym = y;
        y = yn;
        store(x + 1, y);
    }
}

__global__ void __launch_bounds__(kPlanThreads) plan_rows(int ell, int n0, int p, double* rows) {
    extern __shared__ double lds[];
    __shared__ double red[kPlanThreads / 64];
    __shared__ double coefA[256], coefC[256];
    const int n = n0 + blockIdx.x;
    const int M = 2 * n - 1;
    double* P = lds;   // n + 1 values
    if ((long long)ell * ell <= 2LL * M) {
        fill_coefs(ell, M, coefA, coefC);
        __syncthreads();
        for (int x = threadIdx.x; x <= n; x += blockDim.x) P[x] = dlop_rec(ell, M, x, coefA, coefC);
    } else if (threadIdx.x == 0) {
        dlop_march(ell, M, n, [&](int x, double v) { P[x] = v; });
    }
    __syncthreads();
    // kappa(m) = P(n-m) - P(n-m-1), m < n; kappa(n) = 1; norm over m = p..n
    double s = 0.0;
    for (int m = threadIdx.x; m <= n; m += blockDim.x) {
        const double kv = (m < n) ? P[n - m] - P[n - m - 1] : 1.0;
        if (m >= p) s += (m == 0 ? 0.5 : 1.0) * kv * kv;
    }
    const double beta = 1.0 / sqrt(block_sum(s, red));
    double* out = rows + row_off(n, n0);
    for (int m = threadIdx.x; m <= n; m += blockDim.x) {
        const double kv = (m < n) ? P[n - m] - P[n - m - 1] : 1.0;
        out[m] = kv * beta;
    }
}

__global__ void __launch_bounds__(kPlanThreads) plan_basis(int ell, int p, int k, int B, double* basis) {
    __shared__ double red[kPlanThreads / 64];
    __shared__ double coefA[256], coefC[256];
    const int J = blockIdx.x + 1;
    const int t = p + J * B;
    const int M = 2 * t - 2, xmax = t - 1;
    const int dmax = 2 * (k - 1) + p;
    int drec = 0;
    while ((long long)(drec + 1) * (drec + 1) <= 2LL * M && drec + 1 <= dmax) ++drec;
    double* q0 = basis + basis_off(J, p, B, k);
    // degrees d <= drec: the recurrence at each x, storing the degrees 2kk + p
    fill_coefs(drec, M, coefA, coefC);
    __syncthreads();
    for (int x = threadIdx.x; x <= xmax; x += blockDim.x) {
        const int m = t - 1 - x;
        double a = 1.0, b = 1.0 - 2.0 * x / M;
        const double mx = (double)M - 2.0 * x;
        // degree 0 and 1
        if (p == 0 && k > 0) q0[m] = 1.0;                       // kk = 0, d = 0
        if (p == 1 && k > 0 && drec >= 1) q0[m] = -b;           // kk = 0, d = 1 (sign (-1)^d)
        for (int j = 1; j < drec; ++j) {
            const double c = coefA[j] * mx * b - coefC[j] * a;
            a = b;
            b = c;
            const int d = j + 1;
            if (((d - p) & 1) == 0) {
                const int kk = (d - p) >> 1;
                q0[(size_t)kk * t + m] = (d & 1) ? -c : c;
            }
        }
    }
    // degrees above drec: marched in x, one thread per function
    for (int kk = threadIdx.x; kk < k; kk += blockDim.x) {
        const int d = 2 * kk + p;
        if (d <= drec) continue;
        double* q = q0 + (size_t)kk * t;
        const double sg = (d & 1) ? -1.0 : 1.0;
        dlop_march(d, M, xmax, [&](int x, double v) { q[t - 1 - x] = sg * v; });
    }
    __syncthreads();
    // normalise with the weight 1/2 at m = 0
    for (int kk = 0; kk < k; ++kk) {
        double* q = q0 + (size_t)kk * t;
        double s = 0.0;
        for (int m = threadIdx.x; m < t; m += blockDim.x) s += (m == 0 ? 0.5 : 1.0) * q[m] * q[m];
        const double inv = 1.0 / sqrt(block_sum(s, red));
        for (int m = threadIdx.x; m < t; m += blockDim.x) q[m] *= inv;
        __syncthreads();
    }
}

// sum_{m < len} w_m a[m] b_c[m] for c = c0..c0+15 (w_0 = 1/2), into out[c].
__device__ void weighted_dots16(const double* a, const double* b, int ldb, int len, int c0, int cn, double* out,
                                double* red) {
    double acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0;
    for (int m = threadIdx.x; m < len; m += blockDim.x) {
        const double av = (m == 0 ? 0.5 : 1.0) * a[m];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (c0 + i < cn) acc[i] += av * b[(size_t)(c0 + i) * ldb + m];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const double s = block_sum(acc[i], red);
        if (threadIdx.x == 0 && c0 + i < cn) out[c0 + i] = s;
    }
}

__global__ void __launch_bounds__(kPlanThreads) plan_blocks(int ell, int p, int k, int n0, int B, const double* rows,
                                                            const double* basis, double* blocks) {
    __shared__ double red[kPlanThreads / 64];
    __shared__ double dots[256];
    const int J = blockIdx.x, r = blockIdx.y;
    const int R = B + k;
    const int t0 = p + J * B;
    double* row = blocks + ((size_t)J * R + r) * R;
    for (int c = threadIdx.x; c < R; c += blockDim.x) row[c] = 0.0;
    __syncthreads();
    if (r < B) {
        const int n = t0 + r;
        if (n < n0) return;   // completion rows come from the final moments
        const double* kap = rows + row_off(n, n0);
        for (int sp = threadIdx.x; sp <= r; sp += blockDim.x) row[sp] = kap[t0 + sp];
        if (J >= 1 && k > 0) {
            const double* qB = basis + basis_off(J, p, B, k);
            for (int c0 = 0; c0 < k; c0 += 16) weighted_dots16(kap, qB, t0, t0, c0, k, dots, red);
            __syncthreads();
            for (int c = threadIdx.x; c < k; c += blockDim.x) row[B + c] = dots[c];
        }
    } else {
        const int a = r - B;
        const int t1 = t0 + B;
        const double* qa = basis + basis_off(J + 1, p, B, k) + (size_t)a * t1;
        for (int s = threadIdx.x; s < B; s += blockDim.x) row[s] = qa[t0 + s];
        if (J >= 1) {
            const double* qB = basis + basis_off(J, p, B, k);
            for (int c0 = 0; c0 < k; c0 += 16) weighted_dots16(qa, qB, t0, t0, c0, k, dots, red);
            __syncthreads();
            for (int c = threadIdx.x; c < k; c += blockDim.x) row[B + c] = dots[c];
        }
    }
}

void check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw std::runtime_error(std::string("plan generation: ") + what + ": " + hipGetErrorString(e));
}

}  // namespace

size_t device_plan_scratch_doubles(int ell, int B, int NT) {
    const int p = parity_p(ell), k = n_extra(ell), n0 = n0_of(ell);
    const int ntop = p + NT * B - 1;
    const size_t rows = (size_t)row_off(ntop + 1, n0);
    const size_t basis = (size_t)basis_off(NT + 1, p, B, k);
    const size_t blocks = (size_t)NT * (B + k) * (B + k);
    return rows + basis + blocks;
}

void build_ftb_blocks_device(int ell, int B, int NT, double* scratch, std::vector<double>& blocks,
                             hipStream_t stream) {
    const int p = parity_p(ell), k = n_extra(ell), n0 = n0_of(ell);
    const int R = B + k;
    if (B < n0) throw std::invalid_argument("tile smaller than the first regular row");
    if (ell > 255) throw std::invalid_argument("l above 255");
    const int ntop = p + NT * B - 1;
    double* rows = scratch;
    double* basis = rows + row_off(ntop + 1, n0);
    double* blk = basis + basis_off(NT + 1, p, B, k);
    const int nrows = ntop - n0 + 1;
    const size_t lds = sizeof(double) * (size_t)(ntop + 1);
    check(hipFuncSetAttribute((const void*)plan_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
          "LDS limit");
    if (nrows > 0) hipLaunchKernelGGL(plan_rows, dim3(nrows), dim3(kPlanThreads), lds, stream, ell, n0, p, rows);
    check(hipGetLastError(), "plan_rows");
    if (k > 0) hipLaunchKernelGGL(plan_basis, dim3(NT), dim3(kPlanThreads), 0, stream, ell, p, k, B, basis);
    check(hipGetLastError(), "plan_basis");
    hipLaunchKernelGGL(plan_blocks, dim3(NT, R), dim3(kPlanThreads), 0, stream, ell, p, k, n0, B, rows, basis, blk);
    check(hipGetLastError(), "plan_blocks");
    blocks.resize((size_t)NT * R * R);
    check(hipMemcpyAsync(blocks.data(), blk, sizeof(double) * blocks.size(), hipMemcpyDeviceToHost, stream),
          "copy blocks");
    check(hipStreamSynchronize(stream), "sync");
}

}  // namespace dsbt
