// Moment stage by the paper's monomial prefix sums (Sec. 2.6), FP64, one wave
// per channel.  Lane q carries the sum of the monomial nu = nu0 + 2 q (the
// ceil(l/2) nonzero coefficients of eq. DP_expan) through the serial
// recurrence of eq. rec_sum_b_f (forward, n ascending) or eq. rec_sum_f_b
// (inverse, m descending); the sum over nu of each row is a wave reduction.
// Rows are processed in chunks (64 forward, 32 inverse): the chunk's data, alpha and xi rows are
// staged in LDS with coalesced loads, and its results are written back after
// the chunk, which keeps the stage safe in place (a chunk's slots are read
// before they are written; the completion slots are read first and written
// last).
#include "monomial.h"

namespace dsbt {

namespace {

constexpr int kLanes = 64;
constexpr int kMaxK = 64;
constexpr int kRowsI = 32;   // rows per chunk of the inverse (its LDS holds xi and completion rows)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, kLanes);
    return v;
}
__device__ __forceinline__ double2 wave_sum2(double2 v) { return make_double2(wave_sum(v.x), wave_sum(v.y)); }
__device__ __forceinline__ double2 scale(double a, double2 z) { return make_double2(a * z.x, a * z.y); }
__device__ __forceinline__ double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void __launch_bounds__(kLanes) mono_forward(const LChan* __restrict__ chans, const double2* src,
                                                       double2* dst, PhaseArgs ph) {
    const LChan c = chans[blockIdx.x];
    const int lane = threadIdx.x;
    const int Nl = c.N + c.p - 1;
    const bool act = lane < c.k;
    const int inu = c.nu0 + 2 * lane;
    const double nu = (double)inu;
    const double2* f = src + c.off;
    double2* b = dst + c.off;
    const double2* kph = (ph.use && c.kphase) ? static_cast<const double2*>(c.kphase) : nullptr;

    __shared__ double2 fch[kLanes];
    __shared__ double2 bout[kLanes];
    __shared__ double ach[kLanes];
    __shared__ double xch[kLanes * kMaxK];

    // completion rows (eq. lown_b_vs_f), read before any store
    double2 bq = make_double2(0.0, 0.0);
    for (int q = 0; q < c.k; ++q) {
        double2 acc = make_double2(0.0, 0.0);
        for (int j = lane; j < c.N; j += kLanes) acc = add(acc, scale(c.comp[(size_t)q * c.N + j], f[j]));
        acc = wave_sum2(acc);
        if (lane == q) bq = acc;
    }
    const double2 f0 = c.p == 0 ? f[0] : make_double2(0.0, 0.0);

    double2 s = make_double2(0.0, 0.0), aprev = make_double2(0.0, 0.0);
    for (int base = 1; base <= Nl; base += kLanes) {
        const int cnt = min(kLanes, Nl - base + 1);
        const int nl = base + lane;
        fch[lane] = lane < cnt ? f[nl - c.p] : make_double2(0.0, 0.0);
        ach[lane] = (lane < cnt && nl >= c.n0) ? c.alpha[nl - c.n0] : 0.0;
        const int r0 = max(base, c.n0);               // first regular row of the chunk
        const int nrow = base + cnt - r0;
        for (int i = lane; i < nrow * c.k; i += kLanes) xch[i] = c.xi[(size_t)(r0 - c.n0) * c.k + i];
        __syncthreads();
        for (int t = 0; t < cnt; ++t) {
            const int n = base + t;
            const double2 fn = fch[t];
            const double2 a = act ? scale(pow((double)n, nu), fn) : make_double2(0.0, 0.0);
            if (n == 1)   // eq. sum_in_b_f at n = 1: f_0 enters with weight 1/sqrt(2)
                s = add((act && inu == 0) ? scale(sqrt(0.5), f0) : make_double2(0.0, 0.0), scale(0.5, a));
            else
                s = add(s, scale(0.5, add(a, aprev)));
            aprev = a;
            if (n >= c.n0) {
                const double x = act ? xch[(n - r0) * c.k + lane] : 0.0;
                const double2 tot = wave_sum2(scale(x, s));
                const double al = ach[t];
                double2 bn = sub(scale(al, fn), scale(al, tot));
                if (kph) {
                    double2 z = kph[n - c.p];
                    if (ph.conj) z.y = -z.y;
                    bn = cmul(bn, z);
                }
                if (lane == 0) bout[t] = bn;
            }
        }
        __syncthreads();
        if (lane < cnt && nl >= c.n0) b[nl - c.p] = bout[lane];
        __syncthreads();
    }
    if (act) {
        if (kph) {
            double2 z = kph[lane];
            if (ph.conj) z.y = -z.y;
            bq = cmul(bq, z);
        }
        b[lane] = bq;
    }
}

__global__ void __launch_bounds__(kLanes) mono_inverse(const LChan* __restrict__ chans, const double2* src,
                                                       double2* dst) {
    const LChan c = chans[blockIdx.x];
    const int lane = threadIdx.x;
    const int Nl = c.N + c.p - 1;
    const bool act = lane < c.k;
    const double nu = (double)(c.nu0 + 2 * lane);
    const double2* b = src + c.off;
    double2* f = dst + c.off;

    __shared__ double2 bch[kRowsI];
    __shared__ double2 fout[kRowsI];
    __shared__ double ach[kRowsI];
    __shared__ double xch[kRowsI * kMaxK];
    __shared__ double cch[kRowsI * kMaxK];

    const double2 bq = act ? b[lane] : make_double2(0.0, 0.0);   // completion coefficients, read first
    double2 st = make_double2(0.0, 0.0), tprev = make_double2(0.0, 0.0);
    for (int top = Nl; top >= c.n0; top -= kRowsI) {
        const int lo = max(c.n0, top - kRowsI + 1);
        const int cnt = top - lo + 1;
        const int ml = lo + lane;
        if (lane < kRowsI) {
            bch[lane] = lane < cnt ? b[ml - c.p] : make_double2(0.0, 0.0);
            ach[lane] = lane < cnt ? c.alpha[ml - c.n0] : 0.0;
        }
        for (int i = lane; i < cnt * c.k; i += kLanes) xch[i] = c.xi[(size_t)(lo - c.n0) * c.k + i];
        for (int i = lane; i < cnt * c.k; i += kLanes) {
            const int q = i / cnt, t = i - q * cnt;
            cch[t * c.k + q] = c.comp[(size_t)q * c.N + (lo + t - c.p)];
        }
        __syncthreads();
        for (int t = cnt - 1; t >= 0; --t) {
            const int m = lo + t;
            const double2 bm = bch[t];
            const double al = ach[t];
            const double2 term = act ? scale(al * xch[t * c.k + lane], bm) : make_double2(0.0, 0.0);
            if (m == Nl)
                st = scale(0.5, term);
            else
                st = add(st, scale(0.5, add(term, tprev)));
            tprev = term;
            // completion part g_m (lane q) minus m^nu s~_nu,m (lane nu), eq. fast_f_b
            double2 part = make_double2(0.0, 0.0);
            if (act) part = sub(scale(cch[t * c.k + lane], bq), scale(pow((double)m, nu), st));
            const double2 tot = wave_sum2(part);
            if (lane == 0) fout[t] = add(scale(al, bm), tot);
        }
        __syncthreads();
        if (lane < cnt) f[ml - c.p] = fout[lane];
        __syncthreads();
    }
    // rows m < n_0 (eq. fast_f_b_lowm) with s~_nu,n0+1/2 = s~_nu,n0 + alpha_n0 xi_nu(n0) b_n0 / 2
    const double2 half = add(st, scale(0.5, tprev));
    for (int m = c.p; m < c.n0; ++m) {
        const int j = m - c.p;
        double2 part = make_double2(0.0, 0.0);
        if (act) {
            const double w = m == 0 ? sqrt(0.5) : 1.0;
            part = sub(scale(c.comp[(size_t)lane * c.N + j], bq), scale(w * pow((double)m, nu), half));
        }
        const double2 tot = wave_sum2(part);
        if (lane == 0) f[j] = tot;
    }
}

}  // namespace

hipError_t launch_monomial(const LChan* d_chans, int nch, const void* src, void* dst, bool inverse, PhaseArgs ph,
                           hipStream_t s) {
    if (nch <= 0) return hipSuccess;
    if (inverse)
        hipLaunchKernelGGL(mono_inverse, dim3(nch), dim3(kLanes), 0, s, d_chans, (const double2*)src, (double2*)dst);
    else
        hipLaunchKernelGGL(mono_forward, dim3(nch), dim3(kLanes), 0, s, d_chans, (const double2*)src, (double2*)dst,
                           ph);
    return hipGetLastError();
}

}  // namespace dsbt
