// C ABI of the MI355X DSBT library: plan management, table upload and the
// launch sequences of forward / inverse / split step (declared in include/dsbt.h).
#include "../../include/dsbt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "kernels.h"
#include "plan_device.h"
#include "plan_host.h"
#include "angular.h"
#include "monomial.h"
#include "state.h"

namespace {

thread_local std::string g_last_error;

dsbt_status fail(dsbt_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

struct HipError : std::runtime_error {
    hipError_t code;
    HipError(hipError_t c, const char* what) : std::runtime_error(what), code(c) {}
};

void hip_check(hipError_t e, const char* where) {
    if (e != hipSuccess) {
        std::string m = std::string(where) + ": " + hipGetErrorString(e);
        throw HipError(e, m.c_str());
    }
}

struct StatusError : std::runtime_error {
    dsbt_status st;
    StatusError(dsbt_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Complex factors z_i (FP64) as a device table: FP64 pairs for plans with FP64
// arithmetic; for FP32 arithmetic the hi parts (nearest FP32 values) of all n
// factors followed by their lo parts (FP32 roundings of z - hi), which the
// kernels multiply as z hi + z lo (kernels.h, FChan).
std::vector<unsigned char> factor_table(const std::vector<double2>& z, bool fp64) {
    const size_t n = z.size();
    std::vector<unsigned char> out(n * (fp64 ? sizeof(double2) : 2 * sizeof(float2)));
    for (size_t i = 0; i < n; ++i) {
        if (fp64) {
            std::memcpy(out.data() + i * sizeof(double2), &z[i], sizeof(double2));
        } else {
            const float2 h = make_float2((float)z[i].x, (float)z[i].y);
            const float2 l = make_float2((float)(z[i].x - (double)h.x), (float)(z[i].y - (double)h.y));
            std::memcpy(out.data() + i * sizeof(float2), &h, sizeof(h));
            std::memcpy(out.data() + (n + i) * sizeof(float2), &l, sizeof(l));
        }
    }
    return out;
}

// exp(-i a) for every angle a, reduced mod 2 pi in FP64.
std::vector<unsigned char> phase_table(const std::vector<double>& ang, bool fp64) {
    const double twopi = 6.283185307179586476925286766559;
    std::vector<double2> z(ang.size());
    for (size_t i = 0; i < ang.size(); ++i) {
        const double a = ang[i] - twopi * std::nearbyint(ang[i] / twopi);
        z[i] = make_double2(std::cos(a), -std::sin(a));
    }
    return factor_table(z, fp64);
}

// exp(-a) for every exponent a (imaginary time, t -> -i t): real factors stored
// as complex values with zero imaginary part, in the layout of phase_table.
std::vector<unsigned char> decay_table(const std::vector<double>& ex, bool fp64) {
    std::vector<double2> z(ex.size());
    for (size_t i = 0; i < ex.size(); ++i) z[i] = make_double2(std::exp(-ex[i]), 0.0);
    return factor_table(z, fp64);
}

}  // namespace

namespace dsbt {
dsbt_status set_error(dsbt_status s, const char* msg) { return fail(s, msg); }
}  // namespace dsbt

// Scratch of dsbt_step_grad_s_noalloc: one FP64 partial sum per channel, in a
// fixed device array (each GPU the library runs on holds its own copy until
// the process ends).  Host code never passes the array's name to a kernel: it
// uses the device address that hipGetSymbolAddress returns for the current
// device, looked up once per device on the entry point's first call there.
static __device__ __align__(256) double noalloc_scratch[DSBT_NOALLOC_MAX_CHANNELS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};

// Device address of noalloc_scratch on the current device.
double* noalloc_scratch_ptr() {
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) throw StatusError(DSBT_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)), "hipGetSymbolAddress");
        if (!ptr) throw HipError(hipErrorInvalidSymbol, "hipGetSymbolAddress returned NULL");
        g_noalloc_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_noalloc_ptr[dev];
}

}  // namespace

struct dsbt_plan_s {
    int device = 0;
    int precision = DSBT_C64;
    dsbt_plan_opts opts{};
    std::vector<dsbt_channel> ch;
    int64_t elems = 0;
    size_t elem_bytes = 8;   // data element in memory
    size_t cmp_bytes = 8;    // complex value in the arithmetic precision (tables, LDS, phases)
    int maxN = 0, maxR = 0;

    // groups of channels with equal (N, l, rmax)
    struct Group {
        int N, ell, p, k, B, R, NT;
        double rmax;
        std::vector<int> chans;
        void* d_kphase = nullptr;    // per slot (complex of the data precision), after set_potential
        double* d_kin = nullptr;     // K_n = k_n^2/2 per slot (FP64), after set_potential
    };
    std::vector<Group> groups;

    std::vector<void*> allocs;
    int64_t table_bytes = 0;

    dsbt::FChan* d_fchans = nullptr;     // one per channel, channel order
    std::vector<dsbt::FChan> h_fchans;
    dsbt::FChan* d_fchans_n = nullptr;   // sorted by N, for one launch per N
    std::vector<int> order_n;            // channel index of each entry of d_fchans_n
    std::vector<std::tuple<int, int, int>> n_ranges;  // (N, first, count) in d_fchans_n
    // plans with several N: the sine/cosine stage as one launch over tasks of
    // one N each (largest N first), and the dynamic LDS it needs
    dsbt::FTask* d_ftasks = nullptr;
    int n_ftasks = 0;
    size_t ftask_lds = 0;
    // moment-stage work items: matrix-core kernel (FP32, R16 <= 128) and the
    // generic kernel (FP64 plans, larger blocks); per-channel items for the
    // plain form
    std::vector<dsbt::MItem> h_items_mf, h_items_v1, h_items1;
    std::vector<char> items1_mf;          // per channel: item uses the matrix-core kernel
    dsbt::MItem* d_items_mf = nullptr;
    dsbt::MItem* d_items_v1 = nullptr;
    dsbt::MItem* d_items1 = nullptr;
    int mf_waves = 4;
    int chain_ncb = 1;   // largest column-block count of the batched four-wave items
    size_t mf_lds = 0;

    // potential
    bool has_potential = false;
    double dt = 0.0;
    void* d_vphase = nullptr;     // complex of the data precision
    double* d_vangle = nullptr;
    bool imaginary = false;       // tables hold exp(-V tau/2), exp(-K tau) (DSBT_TIME_IMAGINARY)
    dsbt::EChan* d_echans = nullptr;   // per channel, for dsbt_energy

    // monomial-moment variant (DSBT_ALG_MONOMIAL): per channel, in channel order
    std::vector<dsbt::LChan> h_lchans;
    dsbt::LChan* d_lchans = nullptr;

    // dsbt_orthonormalize: channel offsets and sizes, and the last set table
    int64_t* d_off = nullptr;
    int* d_nch = nullptr;
    int* d_sets = nullptr;
    int sets_cap = 0;
    std::vector<int> h_sets;
    double* d_scratch = nullptr;

    // stage timing (dsbt_profile_enable)
    bool profiling = false;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> prof_events;   // (stage, start, stop)
    std::vector<hipEvent_t> event_pool;
    hipEvent_t take_event() {
        hipEvent_t e = nullptr;
        if (!event_pool.empty()) {
            e = event_pool.back();
            event_pool.pop_back();
        } else {
            hip_check(hipEventCreate(&e), "hipEventCreate");
        }
        return e;
    }

    // graph cache for dsbt_kinetic_step
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    std::tuple<void*, int, const float*, int> graph_key{nullptr, 0, nullptr, 0};
    float* d_sgraph = nullptr;    // strengths staged for graph replays
    int sgraph_cap = 0;

    // dsbt_adjoint_segment: states psi_a .. psi_a+n, two adjoint states, the
    // segment's strengths and gradients (plan buffers, grown to the largest n),
    // and the graph of one segment's launches on them
    void* seg_states = nullptr;
    void* seg_lam = nullptr;
    float* seg_s = nullptr;
    double* seg_gs = nullptr;
    double* seg_part = nullptr;   // per-channel partials of the segment's gradients
    int seg_cap = 0;
    // a second stream (default priority) and two events: a batched segment
    // runs its recompute and its adjoint chain side by side
    hipStream_t seg_side = nullptr;
    hipEvent_t seg_fork = nullptr, seg_join = nullptr;
    hipGraphExec_t seg_exec = nullptr;
    hipGraph_t seg_graph = nullptr;
    int seg_graph_n = 0;

    // checked plans (opts.check_finite): device flag and its pinned host copy
    int* d_flag = nullptr;
    int* h_flag = nullptr;

    // device memory through the caller's allocator (opts.dev_alloc) or hipMalloc
    void* dalloc_raw(size_t bytes) {
        void* p = nullptr;
        if (bytes == 0) bytes = 16;
        if (opts.dev_alloc) {
            p = opts.dev_alloc(bytes, opts.alloc_ctx);
            if (!p) throw StatusError(DSBT_ERR_OOM, "dev_alloc returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess)
                throw StatusError(DSBT_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
        return p;
    }
    void dfree(void* p) {
        if (!p) return;
        if (opts.dev_free) opts.dev_free(p, opts.alloc_ctx);
        else (void)hipFree(p);
    }
    // a device buffer owned by the plan (freed by release)
    void* dalloc(size_t bytes) {
        void* p = dalloc_raw(bytes);
        allocs.push_back(p);
        table_bytes += (int64_t)(bytes == 0 ? 16 : bytes);
        return p;
    }
    void drop_graphs() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        if (seg_exec) (void)hipGraphExecDestroy(seg_exec);
        if (seg_graph) (void)hipGraphDestroy(seg_graph);
        seg_exec = nullptr;
        seg_graph = nullptr;
        seg_graph_n = 0;
    }
    void free_segment() {
        dfree(seg_states);
        dfree(seg_lam);
        dfree(seg_s);
        dfree(seg_gs);
        dfree(seg_part);
        seg_states = seg_lam = nullptr;
        seg_s = nullptr;
        seg_gs = nullptr;
        seg_part = nullptr;
        seg_cap = 0;
    }
    void release() {
        drop_graphs();
        free_segment();
        if (seg_fork) (void)hipEventDestroy(seg_fork);
        if (seg_join) (void)hipEventDestroy(seg_join);
        if (seg_side) (void)hipStreamDestroy(seg_side);
        seg_fork = seg_join = nullptr;
        seg_side = nullptr;
        for (void* p : allocs) dfree(p);
        allocs.clear();
        if (h_flag) (void)hipHostFree(h_flag);
        h_flag = nullptr;
        for (auto& t : prof_events) {
            (void)hipEventDestroy(std::get<1>(t));
            (void)hipEventDestroy(std::get<2>(t));
        }
        prof_events.clear();
        for (auto e : event_pool) (void)hipEventDestroy(e);
        event_pool.clear();
    }
};

namespace {

// Complex table (re, im pairs, FP64 values v) of factors in the arithmetic
// precision: FP64 as is; FP32 as the hi table followed by the lo table
// (factor_table).  Returns the hi table; *lo receives the lo table (FP32) or
// nullptr.
template <typename T>
void* upload_unit_table(dsbt_plan_s* P, const std::vector<double>& v, hipStream_t s, const void** lo) {
    std::vector<double2> z(v.size() / 2);
    for (size_t i = 0; i < z.size(); ++i) z[i] = make_double2(v[2 * i], v[2 * i + 1]);
    const std::vector<unsigned char> h = factor_table(z, sizeof(T) == sizeof(double));
    void* d = P->dalloc(h.size());
    hip_check(hipMemcpyAsync(d, h.data(), h.size(), hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
    *lo = sizeof(T) == sizeof(float) ? static_cast<const unsigned char*>(d) + z.size() * sizeof(float2) : nullptr;
    return d;
}

// The quarter-circle roots (cos, sin) pairs of fft_quarter_roots, 16 bytes per
// entry: FP64 (c, s), or FP32 (c hi, s hi, c lo, s lo) with hi the nearest
// FP32 value and lo the FP32 rounding of the rest (kernels.h, FChan).
template <typename T>
void* upload_roots(dsbt_plan_s* P, const std::vector<double>& cs, hipStream_t s) {
    const size_t n = cs.size() / 2;
    std::vector<unsigned char> h(16 * n);
    for (size_t e = 0; e < n; ++e) {
        if (sizeof(T) == sizeof(double)) {
            std::memcpy(h.data() + 16 * e, &cs[2 * e], 16);
        } else {
            float v[4];
            for (int j = 0; j < 2; ++j) {
                v[j] = (float)cs[2 * e + j];
                v[2 + j] = (float)(cs[2 * e + j] - (double)v[j]);
            }
            std::memcpy(h.data() + 16 * e, v, 16);
        }
    }
    void* d = P->dalloc(h.size());
    hip_check(hipMemcpyAsync(d, h.data(), h.size(), hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
    return d;
}

// Temporary device buffer for the plan generator, freed on scope exit (through
// the plan's allocator when P is given; the generator synchronises before it
// returns, so nothing reads the buffer when it is handed back).
struct DeviceScratch {
    dsbt_plan_s* P = nullptr;
    double* ptr = nullptr;
    void alloc(size_t doubles) {
        if (doubles == 0) return;
        if (P) {
            ptr = static_cast<double*>(P->dalloc_raw(sizeof(double) * doubles));
            return;
        }
        hipError_t e = hipMalloc(&ptr, sizeof(double) * doubles);
        if (e != hipSuccess) {
            ptr = nullptr;
            throw StatusError(DSBT_ERR_OOM, std::string("plan scratch: ") + hipGetErrorString(e));
        }
    }
    ~DeviceScratch() {
        if (!ptr) return;
        if (P) P->dfree(ptr);
        else (void)hipFree(ptr);
    }
};

// A named range for rocprofv3 --marker-trace around an entry point.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
};

void device_blocks(int ell, int B, int NT, double* scratch, std::vector<double>& blk, hipStream_t s) {
    try {
        dsbt::build_ftb_blocks_device(ell, B, NT, scratch, blk, s);
    } catch (const std::runtime_error& e) {
        throw HipError(hipErrorLaunchFailure, e.what());
    }
}

template <typename T>
void* upload_converted(dsbt_plan_s* P, const std::vector<double>& v, hipStream_t s) {
    std::vector<T> h(v.size());
    for (size_t i = 0; i < v.size(); ++i) h[i] = (T)v[i];
    void* d = P->dalloc(h.size() * sizeof(T));
    hip_check(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
    return d;
}

dsbt_status validate_channels(const dsbt_channel* ch, int nch, int precision, size_t max_lds) {
    if (!ch || nch <= 0) return fail(DSBT_ERR_INVALID_ARG, "no channels");
    std::vector<std::pair<int64_t, int64_t>> iv;
    for (int c = 0; c < nch; ++c) {
        const dsbt_channel& x = ch[c];
        if (!is_pow2(x.N) || x.N < 16 || x.N > 8192)
            return fail(DSBT_ERR_UNSUPPORTED, "channel " + std::to_string(c) + ": N must be a power of two in [16, 8192]");
        const size_t lds = (size_t)x.N * (precision == DSBT_C64 ? 8 : 16);
        if (lds > max_lds)
            return fail(DSBT_ERR_UNSUPPORTED, "channel " + std::to_string(c) + ": N too large for LDS at this precision");
        if (x.ell < 0 || x.ell > 2 * x.N - 2 || x.ell > 255)
            return fail(DSBT_ERR_UNSUPPORTED, "channel " + std::to_string(c) + ": need 0 <= l <= min(2N-2, 255)");
        if (!(x.rmax > 0.0) || !std::isfinite(x.rmax))
            return fail(DSBT_ERR_INVALID_ARG, "channel " + std::to_string(c) + ": rmax must be positive");
        if (x.offset < 0) return fail(DSBT_ERR_INVALID_ARG, "channel " + std::to_string(c) + ": negative offset");
        iv.emplace_back(x.offset, x.offset + x.N);
    }
    std::sort(iv.begin(), iv.end());
    for (size_t i = 1; i < iv.size(); ++i)
        if (iv[i].first < iv[i - 1].second) return fail(DSBT_ERR_INVALID_ARG, "channels overlap");
    return DSBT_OK;
}

void upload_fchans_n(dsbt_plan_s* P) {
    std::vector<dsbt::FChan> v(P->ch.size());
    for (size_t i = 0; i < v.size(); ++i) v[i] = P->h_fchans[P->order_n[i]];
    hip_check(hipMemcpy(P->d_fchans_n, v.data(), sizeof(dsbt::FChan) * v.size(), hipMemcpyHostToDevice), "fchans");
}

// Tables and channel descriptors of the monomial-moment variant, per (N, l) group.
void build_monomial(dsbt_plan_s* P) {
    P->h_lchans.assign(P->ch.size(), dsbt::LChan{});
    for (auto& g : P->groups) {
        std::vector<double> xi, alpha, comp;
        dsbt::monomial_tables(g.N, g.ell, xi, alpha, comp);
        auto up = [&](const std::vector<double>& v) -> const double* {
            auto* d = (double*)P->dalloc(sizeof(double) * v.size());
            if (!v.empty())
                hip_check(hipMemcpy(d, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice), "monomial tables");
            return d;
        };
        const double* dx = up(xi);
        const double* da = up(alpha);
        const double* dc = up(comp);
        for (int c : g.chans)
            P->h_lchans[c] = dsbt::LChan{P->ch[c].offset, g.N, g.ell, g.p, dsbt::n0_of(g.ell), g.k, (g.ell + 1) % 2,
                                         dx, da, dc, nullptr};
    }
    P->d_lchans = (dsbt::LChan*)P->dalloc(sizeof(dsbt::LChan) * P->h_lchans.size());
    hip_check(hipMemcpy(P->d_lchans, P->h_lchans.data(), sizeof(dsbt::LChan) * P->h_lchans.size(),
                        hipMemcpyHostToDevice), "monomial channels");
}

template <typename T>
void build_plan(dsbt_plan_s* P, hipStream_t s) {
    const int nch = (int)P->ch.size();
    // groups
    std::map<std::tuple<int, int, double>, int> gid;
    for (int c = 0; c < nch; ++c) {
        const auto& x = P->ch[c];
        auto key = std::make_tuple(x.N, x.ell, x.rmax);
        auto itg = gid.find(key);
        if (itg == gid.end()) {
            dsbt_plan_s::Group g;
            g.N = x.N;
            g.ell = x.ell;
            g.rmax = x.rmax;
            g.p = dsbt::parity_p(x.ell);
            g.k = dsbt::n_extra(x.ell);
            gid[key] = (int)P->groups.size();
            P->groups.push_back(g);
            itg = gid.find(key);
        }
        P->groups[itg->second].chans.push_back(c);
    }
    // tile per l: shared by every N with that l
    std::map<int, int> minN, maxN;
    for (auto& g : P->groups) {
        minN[g.ell] = minN.count(g.ell) ? std::min(minN[g.ell], g.N) : g.N;
        maxN[g.ell] = std::max(maxN[g.ell], g.N);
    }
    std::map<int, int> tileB;
    for (auto& kv : minN) {
        const int ell = kv.first;
        int B = dsbt::auto_tile(ell, kv.second);
        const int req = P->opts.tile;
        if (req > 0) {
            if (!is_pow2(req) || req < dsbt::n0_of(ell) || req > kv.second)
                throw StatusError(DSBT_ERR_UNSUPPORTED, "requested tile does not fit l = " + std::to_string(ell));
            B = req;
        }
        tileB[ell] = B;
    }
    // moment tables per l
    struct Tab { const void* f; const void* i; const void* mf; const void* mi; int NB; };
    std::map<int, Tab> tabs;
    const bool fp32 = std::is_same<T, float>::value;
    const bool fp64mf = P->precision == DSBT_C64_FP64 || P->precision == DSBT_C128;   // FP64 arithmetic
    // FP64 blocks generated on the device (default) or by host threads
    DeviceScratch scratch;
    scratch.P = P;
    if (P->opts.plan_where == DSBT_PLAN_ON_DEVICE) {
        size_t most = 0;
        for (auto& kv : tileB)
            most = std::max(most, dsbt::device_plan_scratch_doubles(kv.first, kv.second, maxN[kv.first] / kv.second));
        scratch.alloc(most);
    }
    for (auto& kv : tileB) {
        const int ell = kv.first, B = kv.second, NT = maxN[ell] / B;
        const int k = dsbt::n_extra(ell), R = B + k;
        std::vector<double> blk;
        if (P->opts.plan_where == DSBT_PLAN_ON_DEVICE)
            device_blocks(ell, B, NT, scratch.ptr, blk, s);
        else
            dsbt::build_ftb_blocks(ell, B, NT, blk, 0);
        Tab t{nullptr, nullptr, nullptr, nullptr, 0};
        // matrix-core path: B = 32 with R <= 64, or B = 64 with R <= 128
        const int R16 = 2 * B;
        if (fp32 && (B == 32 || B == 64) && R <= R16) {
            t.NB = R16 / 16;
            std::vector<double> arr;
            dsbt::arrange_mfma_blocks(blk, B, k, dsbt::parity_p(ell), NT, t.NB, false, arr);
            t.mf = upload_converted<float>(P, arr, s);
            dsbt::arrange_mfma_blocks(blk, B, k, dsbt::parity_p(ell), NT, t.NB, true, arr);
            t.mi = upload_converted<float>(P, arr, s);
        } else if (fp64mf && B == 32 && R <= R16) {
            // FP64 tables in the same operand layout for the FP64 four-wave pipeline
            t.NB = 4;
            std::vector<double> arr;
            dsbt::arrange_mfma_blocks(blk, B, k, dsbt::parity_p(ell), NT, t.NB, false, arr);
            t.mf = upload_converted<double>(P, arr, s);
            dsbt::arrange_mfma_blocks(blk, B, k, dsbt::parity_p(ell), NT, t.NB, true, arr);
            t.mi = upload_converted<double>(P, arr, s);
        } else {
            std::vector<double> tr(blk.size());
            for (int J = 0; J < NT; ++J) {
                const double* a = blk.data() + (size_t)J * R * R;
                double* b = tr.data() + (size_t)J * R * R;
                for (int q = 0; q < R; ++q)
                    for (int r = 0; r < R; ++r) b[(size_t)q * R + r] = a[(size_t)r * R + q];
            }
            t.f = upload_converted<T>(P, tr, s);
            t.i = upload_converted<T>(P, blk, s);
        }
        tabs[ell] = t;
    }
    // per N: the quarter-circle roots the FFT passes form their twiddles from,
    // and the post-twiddles times the orthonormal scale, 0.5 sqrt(2/N) w^k
    // (k >= 1) and 0.5 sqrt(1/N) (k = 0), with their lo parts
    std::map<int, std::array<const void*, 3>> twd;
    for (auto& g : P->groups) {
        if (twd.count(g.N)) continue;
        std::vector<double> cs, post;
        dsbt::fft_quarter_roots(g.N, cs);
        dsbt::fft_post_twiddles(g.N, post);
        std::array<const void*, 3> a{};
        a[0] = upload_roots<T>(P, cs, s);
        const double sc1 = 0.5 * std::sqrt(2.0 / g.N), sc0 = 0.5 * std::sqrt(1.0 / g.N);
        for (int k = 0; k < g.N; ++k) {
            const double f = k == 0 ? sc0 : sc1;
            post[2 * k] *= f;
            post[2 * k + 1] *= f;
        }
        a[1] = upload_unit_table<T>(P, post, s, &a[2]);
        twd[g.N] = a;
    }
    // channel descriptors
    P->h_fchans.resize(nch);
    P->maxN = 0;
    for (int c = 0; c < nch; ++c) {
        const auto& x = P->ch[c];
        dsbt::FChan f{};
        f.off = x.offset;
        f.N = x.N;
        f.log2N = ilog2(x.N);
        f.p = dsbt::parity_p(x.ell);
        const int sg = (((x.ell + 1) / 2) % 2) ? -1 : 1;
        f.sign = (P->opts.sign == DSBT_SIGN_PRINTED_F) ? 1.0f : (float)sg;
        f.roots = twd[x.N][0];
        f.post = twd[x.N][1];
        f.post_lo = twd[x.N][2];
        P->h_fchans[c] = f;
        P->maxN = std::max(P->maxN, x.N);
    }
    P->d_fchans = (dsbt::FChan*)P->dalloc(sizeof(dsbt::FChan) * nch);
    hip_check(hipMemcpy(P->d_fchans, P->h_fchans.data(), sizeof(dsbt::FChan) * nch, hipMemcpyHostToDevice), "fchans");
    P->order_n.resize(nch);
    for (int c = 0; c < nch; ++c) P->order_n[c] = c;
    std::stable_sort(P->order_n.begin(), P->order_n.end(), [&](int a, int b) { return P->ch[a].N > P->ch[b].N; });
    P->n_ranges.clear();
    for (int i = 0; i < nch; ++i) {
        const int N = P->ch[P->order_n[i]].N;
        if (P->n_ranges.empty() || std::get<0>(P->n_ranges.back()) != N) P->n_ranges.emplace_back(N, i, 0);
        std::get<2>(P->n_ranges.back())++;
    }
    P->d_fchans_n = (dsbt::FChan*)P->dalloc(sizeof(dsbt::FChan) * nch);
    upload_fchans_n(P);
    if (P->n_ranges.size() > 1 && P->opts.mode == DSBT_MODE_BATCHED) {
        std::vector<dsbt::FTask> tasks;
        for (auto& r : P->n_ranges) {
            const int N = std::get<0>(r), per = dsbt::kMultiThreads / (N / 8);
            for (int i = 0; i < std::get<2>(r); i += per)
                tasks.push_back({N, std::get<1>(r) + i, std::min(per, std::get<2>(r) - i)});
            P->ftask_lds = std::max(P->ftask_lds, dsbt::fstage_multi_lds<T>(N));
        }
        P->d_ftasks = (dsbt::FTask*)P->dalloc(sizeof(dsbt::FTask) * tasks.size());
        hip_check(hipMemcpy(P->d_ftasks, tasks.data(), sizeof(dsbt::FTask) * tasks.size(), hipMemcpyHostToDevice),
                  "tasks");
        P->n_ftasks = (int)tasks.size();
    }
    // moment items
    const int cpb = P->opts.chans_per_block;
    bool any_nb8 = false;
    for (auto& g : P->groups)
        if (tabs[g.ell].NB == 8) any_nb8 = true;
    P->mf_waves = any_nb8 ? 8 : 4;
    int ncu = 256;
    {
        int dev = 0;
        hipDeviceProp_t pr;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&pr, dev) == hipSuccess &&
            pr.multiProcessorCount >= 8)
            ncu = pr.multiProcessorCount;
    }
    // four-wave pipeline: 16 channels (two column blocks) per item halve the
    // table reads per channel, but only while that still gives every compute
    // unit an item (each item is a serial chain of tile steps)
    int wide = 1;
    if (fp32 && P->mf_waves == 4 && (cpb <= 0 || cpb > 8)) {
        size_t n16 = 0;
        for (auto& g : P->groups)
            if (tabs[g.ell].mf) n16 += (g.chans.size() + 15) / 16;
        wide = n16 >= (size_t)ncu ? 2 : 1;
    }
    std::vector<dsbt::MItem> items_mf, items_v1;
    std::vector<int> items_mf_ell;
    P->h_items1.assign(nch, dsbt::MItem{});
    P->items1_mf.assign(nch, 0);
    P->maxR = 0;
    P->mf_lds = 0;
    for (auto& g : P->groups) {
        const Tab& t = tabs[g.ell];
        g.B = tileB[g.ell];
        g.R = g.B + g.k;
        g.NT = g.N / g.B;
        P->maxR = std::max(P->maxR, g.R);
        dsbt::MItem base{};
        base.tab_f = t.f;
        base.tab_i = t.i;
        base.mf_f = t.mf;
        base.mf_i = t.mi;
        base.B = g.B;
        base.k = g.k;
        base.R = g.R;
        base.NT = g.NT;
        base.p = g.p;
        base.NB = t.NB;
        const bool mf = t.mf != nullptr;
        int per = dsbt::kMaxChanPerItem;
        if (mf) {
            base.NCB = P->mf_waves == 4 ? wide : dsbt::mfma_ncb(P->mf_waves, base.NB);
            per = 8 * base.NCB;
        }
        if (cpb > 0) per = std::min(per, cpb);
        for (size_t i0 = 0; i0 < g.chans.size(); i0 += per) {
            dsbt::MItem it = base;
            it.nch = (int)std::min<size_t>(per, g.chans.size() - i0);
            if (mf && P->mf_waves == 4 && it.NCB == 2) {
                // the rest of an l group in items of one column block (half the
                // matrix work of two): a last item of at most 8 channels, and
                // for k <= 16 every last item, which leaves the scheduler light
                // items to pair on the compute units that must hold two
                const size_t rest = g.chans.size() - i0;
                if (rest <= 8 || (rest < 16 && g.k <= 16)) {
                    it.NCB = 1;
                    it.nch = (int)std::min<size_t>(8, rest);
                    per = 8;
                }
            }
            for (int j = 0; j < dsbt::kMaxChanPerItem; ++j)
                it.off[j] = P->ch[g.chans[i0 + (j < it.nch ? j : 0)]].offset;   // repeat a real channel
            if (mf) {
                items_mf.push_back(it);
                items_mf_ell.push_back(g.ell);
                P->chain_ncb = std::max(P->chain_ncb, it.NCB);
                P->mf_lds = std::max(P->mf_lds, dsbt::mfma_lds_bytes_for(it.NB, it.NCB, it.B));
            } else {
                items_v1.push_back(it);
            }
        }
        for (int c : g.chans) {
            dsbt::MItem it = base;
            it.nch = 1;
            if (mf && P->mf_waves == 4) it.NCB = 1;
            for (int j = 0; j < dsbt::kMaxChanPerItem; ++j) it.off[j] = P->ch[c].offset;
            P->h_items1[c] = it;
            P->items1_mf[c] = mf ? 1 : 0;
            if (mf) P->mf_lds = std::max(P->mf_lds, dsbt::mfma_lds_bytes_for(it.NB, it.NCB, it.B));
        }
    }
    // generic kernel: heaviest items first
    std::stable_sort(items_v1.begin(), items_v1.end(), [](const dsbt::MItem& a, const dsbt::MItem& b) {
        return (double)a.NT * a.R * a.R * a.nch > (double)b.NT * b.R * b.R * b.nch;
    });
    // matrix-core kernel: workgroup b runs on XCD b % 8, and the XCD hands its
    // workgroups to its compute units in turn, so blocks b, b + 8 C, b + 16 C
    // (C compute units per XCD) share a compute unit while all are resident.
    // Items of one l are cut into chunks of up to 4 (they read the same table
    // at the same time, so a chunk shares that XCD's L2), chunks are dealt to
    // the XCDs heaviest first by least accumulated cost; within an XCD the items
    // are dealt to compute units the same way, and round r of the XCD's list
    // holds the r-th heaviest item of every compute unit.
    {
        const int nx = 8, chunk = 4;
        const int cpx = ncu / nx;
        // matrix instructions per tile: the four-wave pipeline skips zero blocks
        auto cost_of = [&](const dsbt::MItem& it) {
            if (P->mf_waves == 4) return (double)it.NT * it.NCB * (it.k > 16 ? 56.0 : 32.0);
            return (double)it.NT * it.NB * it.NB;
        };
        std::vector<std::pair<double, std::vector<int>>> chunks;
        std::map<int, std::vector<int>> by_ell;
        for (size_t i = 0; i < items_mf.size(); ++i) by_ell[items_mf_ell[i]].push_back((int)i);
        for (auto& kv : by_ell) {
            for (size_t j = 0; j < kv.second.size(); j += chunk) {
                std::vector<int> ids(kv.second.begin() + j, kv.second.begin() + std::min(kv.second.size(), j + chunk));
                double cost = 0.0;
                for (int i : ids) cost += cost_of(items_mf[i]);
                chunks.emplace_back(cost, ids);
            }
        }
        std::stable_sort(chunks.begin(), chunks.end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        // least loaded XCD, among those where the chunk's items that should
        // not share a compute unit with anything but the lightest items (all
        // but the lightest class) still find a compute unit of their own
        double lightest = 0.0;
        for (auto& it : items_mf) {
            const double c = cost_of(it);
            if (lightest == 0.0 || c < lightest) lightest = c;
        }
        std::vector<std::vector<int>> bins(nx);
        std::vector<double> load(nx, 0.0);
        std::vector<int> nbig(nx, 0);
        for (auto& ch : chunks) {
            int big = 0;
            for (int i : ch.second) big += cost_of(items_mf[i]) > lightest ? 1 : 0;
            int x = -1;
            for (int y = 0; y < nx; ++y)
                if (nbig[y] + big <= cpx && (x < 0 || load[y] < load[x])) x = y;
            if (x < 0) x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (int i : ch.second) bins[x].push_back(i);
            load[x] += ch.first;
            nbig[x] += big;
        }
        std::vector<std::vector<int>> order(nx);   // per XCD, in block order; -1: idle slot
        for (int x = 0; x < nx; ++x) {
            std::vector<int> ids = bins[x];
            std::stable_sort(ids.begin(), ids.end(),
                             [&](int a, int b) { return cost_of(items_mf[a]) > cost_of(items_mf[b]); });
            std::vector<std::vector<int>> cu(cpx);
            std::vector<double> cl(cpx, 0.0);
            for (int i : ids) {
                const int c = (int)(std::min_element(cl.begin(), cl.end()) - cl.begin());
                cu[c].push_back(i);
                cl[c] += cost_of(items_mf[i]);
            }
            size_t rounds = 0;
            for (auto& v : cu) rounds = std::max(rounds, v.size());
            for (size_t r = 0; r < rounds; ++r)
                for (int c = 0; c < cpx; ++c) order[x].push_back(r < cu[c].size() ? cu[c][r] : -1);
            while (!order[x].empty() && order[x].back() < 0) order[x].pop_back();
        }
        size_t depth = 0;
        for (auto& o : order) depth = std::max(depth, o.size());
        std::vector<dsbt::MItem> placed(depth * nx, dsbt::MItem{});   // nch = 0: idle slot
        for (int x = 0; x < nx; ++x)
            for (size_t j = 0; j < order[x].size(); ++j)
                if (order[x][j] >= 0) placed[j * nx + x] = items_mf[order[x][j]];
        if (items_mf.empty()) placed.clear();
        P->h_items_mf = placed;
    }
    P->h_items_v1 = items_v1;
    auto upload_items = [&](const std::vector<dsbt::MItem>& v) -> dsbt::MItem* {
        if (v.empty()) return nullptr;
        auto* d = (dsbt::MItem*)P->dalloc(sizeof(dsbt::MItem) * v.size());
        hip_check(hipMemcpy(d, v.data(), sizeof(dsbt::MItem) * v.size(), hipMemcpyHostToDevice), "items");
        return d;
    };
    P->d_items_mf = upload_items(P->h_items_mf);
    P->d_items_v1 = upload_items(P->h_items_v1);
    P->d_items1 = upload_items(P->h_items1);
    P->d_scratch = (double*)P->dalloc(sizeof(double) * (nch + 1));
    const size_t m_lds = P->cmp_bytes * (size_t)dsbt::kMaxChanPerItem * P->maxR;
    hip_check(dsbt::set_lds_limits<T>(m_lds), "set LDS limits");
    hip_check(dsbt::set_lds_limits_mfma(), "set LDS limits");
    hip_check(dsbt::set_lds_limits_chain<float>(), "set LDS limits");
    hip_check(dsbt::set_lds_limits_chain<double>(), "set LDS limits");
    hip_check(dsbt::set_lds_limits_fstage_n<T>(), "set LDS limits");
    if (P->opts.algorithm == DSBT_ALG_MONOMIAL) build_monomial(P);
}

// Runs `launch` between two recorded events when profiling is on.
template <typename F>
void timed(dsbt_plan_s* P, int stage, hipStream_t s, F&& launch) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!P->profiling || hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
        launch();
        return;
    }
    hipEvent_t a = P->take_event(), b = P->take_event();
    hip_check(hipEventRecord(a, s), "hipEventRecord");
    launch();
    hip_check(hipEventRecord(b, s), "hipEventRecord");
    P->prof_events.emplace_back(stage, a, b);
}

// Matrix-core moment stage: the four-wave pipeline when every item has B = 32,
// else the row-block kernel (B = 64 items need 8 waves).  ncb: the largest
// column-block count of the launched items.
// T: arithmetic precision, S: data scalar (T = double: FP64 arithmetic on
// complex64 or complex128 data, whose matrix-core tables are all B = 32).
template <typename T, typename S>
hipError_t launch_mf(dsbt_plan_s* P, const dsbt::MItem* items, int n, int ncb, const void* src, void* dst,
                     bool inverse, dsbt::PhaseArgs ph, hipStream_t s) {
    if (P->mf_waves == 4) return dsbt::launch_mstage_chain<T, S>(items, n, ncb, src, dst, inverse, ph, s);
    return dsbt::launch_mstage_mfma(items, n, P->mf_waves, P->mf_lds, src, dst, inverse, ph, s);
}

// kin: the kinetic factors of a split step, which sit between the forward and
// the inverse moment stage: callers pass the same kin to both directions, and
// each kernel applies it on its side (the four-wave pipeline to the inverse's
// input, the other moment kernels to the forward's output).
inline dsbt::PhaseArgs kin_for(bool chain_kernel, bool inverse, dsbt::PhaseArgs kin) {
    return (chain_kernel ? inverse : !inverse) ? kin : dsbt::PhaseArgs{};
}

template <typename T, typename S>
void enqueue_mstage(dsbt_plan_s* P, const void* src, void* dst, bool inverse, hipStream_t s, dsbt::PhaseArgs kin) {
    if (P->d_lchans) {
        timed(P, DSBT_STAGE_MOMENT, s, [&] {
            hip_check(dsbt::launch_monomial(P->d_lchans, (int)P->h_lchans.size(), src, dst, inverse,
                                            kin_for(false, inverse, kin), s), "monomial");
        });
        return;
    }
    if (P->d_items_mf)
        timed(P, DSBT_STAGE_MOMENT, s, [&] {
            hip_check(launch_mf<T, S>(P, P->d_items_mf, (int)P->h_items_mf.size(), P->chain_ncb, src, dst, inverse,
                                      kin_for(P->mf_waves == 4, inverse, kin), s), "mstage_mfma");
        });
    if (P->d_items_v1)
        timed(P, DSBT_STAGE_MOMENT, s, [&] {
            hip_check(dsbt::launch_mstage<T, S>(P->d_items_v1, (int)P->h_items_v1.size(), P->maxR, src, dst, inverse,
                                                kin_for(false, inverse, kin), s), "mstage");
        });
}

template <typename T, typename S>
void enqueue_mstage_one(dsbt_plan_s* P, int c, const void* src, void* dst, bool inverse, hipStream_t s,
                        dsbt::PhaseArgs kin) {
    timed(P, DSBT_STAGE_MOMENT, s, [&] {
        if (P->items1_mf[c])
            hip_check(launch_mf<T, S>(P, P->d_items1 + c, 1, 1, src, dst, inverse,
                                      kin_for(P->mf_waves == 4, inverse, kin), s), "mstage_mfma");
        else
            hip_check(dsbt::launch_mstage<T, S>(P->d_items1 + c, 1, P->maxR, src, dst, inverse,
                                                kin_for(false, inverse, kin), s), "mstage");
    });
}

// The batched sine/cosine stage: mode 0 forward, 1 inverse, 2 inverse then
// forward (in place; ph on the inverse, ph2 on the forward; mid, if not null,
// also receives the state between the two).  One launch per distinct N, or
// one launch over all N (plans with several N).
template <typename T, typename S>
void enqueue_fstage(dsbt_plan_s* P, const void* src, void* dst, int mode, dsbt::PhaseArgs ph, dsbt::PhaseArgs ph2,
                    hipStream_t s, void* mid = nullptr) {
    if (P->d_ftasks) {
        timed(P, DSBT_STAGE_SINCOS, s, [&] {
            hip_check(dsbt::launch_fstage_multi<T, S>(P->d_ftasks, P->n_ftasks, P->d_fchans_n, src, dst, mid, mode, ph,
                                                      ph2, P->ftask_lds, s), "fstage");
        });
        return;
    }
    for (auto& r : P->n_ranges)
        timed(P, DSBT_STAGE_SINCOS, s, [&] {
            const int N = std::get<0>(r), first = std::get<1>(r), count = std::get<2>(r);
            if (mode == 2)
                hip_check(dsbt::launch_fstage_inv_fwd<T, S>(N, P->d_fchans_n + first, count, dst, mid, ph, ph2, s),
                          "fstage");
            else
                hip_check(dsbt::launch_fstage_n<T, S>(N, P->d_fchans_n + first, count, src, dst, mode == 1, ph, s),
                          "fstage");
        });
}

template <typename T, typename S>
void enqueue_forward(dsbt_plan_s* P, const void* src, void* dst, hipStream_t s, dsbt::PhaseArgs pv,
                     dsbt::PhaseArgs pk) {
    const int nch = (int)P->ch.size();
    if (P->opts.mode == DSBT_MODE_PLAIN) {
        for (int c = 0; c < nch; ++c) {
            timed(P, DSBT_STAGE_SINCOS, s, [&] {
                hip_check(dsbt::launch_fstage_n<T, S>(P->ch[c].N, P->d_fchans + c, 1, src, dst, false, pv, s), "fstage");
            });
            enqueue_mstage_one<T, S>(P, c, dst, dst, false, s, pk);
        }
        return;
    }
    enqueue_fstage<T, S>(P, src, dst, 0, pv, dsbt::PhaseArgs{}, s);
    enqueue_mstage<T, S>(P, dst, dst, false, s, pk);
}

// pk: the kinetic factors given to the preceding enqueue_forward (see
// enqueue_mstage), or none
template <typename T, typename S>
void enqueue_inverse(dsbt_plan_s* P, const void* src, void* dst, hipStream_t s, dsbt::PhaseArgs pv,
                     dsbt::PhaseArgs pk = dsbt::PhaseArgs{}) {
    const int nch = (int)P->ch.size();
    if (P->opts.mode == DSBT_MODE_PLAIN) {
        for (int c = 0; c < nch; ++c) {
            enqueue_mstage_one<T, S>(P, c, src, dst, true, s, pk);
            timed(P, DSBT_STAGE_SINCOS, s, [&] {
                hip_check(dsbt::launch_fstage_n<T, S>(P->ch[c].N, P->d_fchans + c, 1, dst, dst, true, pv, s), "fstage");
            });
        }
        return;
    }
    enqueue_mstage<T, S>(P, src, dst, true, s, pk);
    enqueue_fstage<T, S>(P, dst, dst, 1, pv, dsbt::PhaseArgs{}, s);
}

// nsteps split steps in place.  Batched plans run one step's inverse sine /
// cosine stage and the next step's forward one as a single launch
// (launch_fstage_inv_fwd), so a step costs three launches and three passes
// over the data instead of four.
template <typename T, typename S>
void enqueue_steps(dsbt_plan_s* P, void* psi, int nsteps, const float* sc, bool adjoint, hipStream_t s) {
    auto pv_of = [&](int u) {
        const int t = adjoint ? (nsteps - 1 - u) : u;
        return dsbt::PhaseArgs{1, adjoint ? 1 : 0, sc, t};
    };
    const dsbt::PhaseArgs pk{1, adjoint ? 1 : 0, nullptr, 0}, none{};
    if (P->opts.mode == DSBT_MODE_PLAIN) {
        for (int u = 0; u < nsteps; ++u) {
            enqueue_forward<T, S>(P, psi, psi, s, pv_of(u), pk);
            enqueue_inverse<T, S>(P, psi, psi, s, pv_of(u), pk);
        }
        return;
    }
    enqueue_fstage<T, S>(P, psi, psi, 0, pv_of(0), none, s);
    for (int u = 0; u < nsteps; ++u) {
        enqueue_mstage<T, S>(P, psi, psi, false, s, pk);
        enqueue_mstage<T, S>(P, psi, psi, true, s, pk);
        if (u + 1 < nsteps)
            enqueue_fstage<T, S>(P, psi, psi, 2, pv_of(u), pv_of(u + 1), s);
        else
            enqueue_fstage<T, S>(P, psi, psi, 1, pv_of(u), none, s);
    }
}

// Captures what `enqueue` launches (on a capture stream) as a graph and instantiates it.
template <typename F>
void capture_graph(F&& enqueue, hipGraph_t* graph, hipGraphExec_t* exec) {
    hipStream_t cap;
    hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        try {
            enqueue(cap);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cap, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipStreamDestroy(cap);
            throw;
        }
        e = hipStreamEndCapture(cap, graph);
    }
    (void)hipStreamDestroy(cap);
    hip_check(e, "graph capture");
    hip_check(hipGraphInstantiate(exec, *graph, nullptr, nullptr, 0), "graph instantiate");
}

// Adjoint buffer holding the segment's result lam_a: the batched form keeps
// lam_t in buffer t; the plain form alternates two buffers.
inline int segment_result_buffer(const dsbt_plan_s* P, int n) {
    return P->opts.mode == DSBT_MODE_PLAIN ? (n & 1) : 0;
}

// One checkpoint segment of the adjoint method on the plan's segment buffers
// (dsbt_adjoint_segment): states 1..n from state 0, then the n adjoint steps
// lam_{t+1} -> lam_t and the strength gradients.  Batched plans carry each
// pass in a work buffer (adjoint buffers n + 1 and n + 2) through the fused
// inverse + forward stage, which also stores the state between two steps:
// psi_t into state t, lam_t into adjoint buffer t (lam_n is given there).
// The adjoint chain needs no psi, so it runs on the plan's second stream
// beside the recompute (its launches are small); all n gradients then take
// two launches once both are done.  The plain form alternates lam between
// adjoint buffers 0 and 1 and reduces each step's gradient in turn.  Both
// give the results of separate step and gradient calls bitwise.
template <typename T, typename S>
void enqueue_segment(dsbt_plan_s* P, int n, hipStream_t q) {
    const size_t sb = (size_t)P->elems * P->elem_bytes;
    auto state = [&](int t) { return static_cast<unsigned char*>(P->seg_states) + sb * (size_t)t; };
    auto lam = [&](int t) { return static_cast<unsigned char*>(P->seg_lam) + sb * (size_t)t; };
    const int nch = (int)P->ch.size();
    if (P->opts.mode == DSBT_MODE_PLAIN) {
        for (int t = 0; t < n; ++t) {
            const dsbt::PhaseArgs pv{1, 0, P->seg_s, t}, pk{1, 0, nullptr, 0};
            enqueue_forward<T, S>(P, state(t), state(t + 1), q, pv, pk);
            enqueue_inverse<T, S>(P, state(t + 1), state(t + 1), q, pv, pk);
        }
        int cur = 0;   // buffer cur holds lam_{t+1}
        for (int t = n - 1; t >= 0; --t) {
            const dsbt::PhaseArgs pv{1, 1, P->seg_s, t}, pk{1, 1, nullptr, 0};
            enqueue_forward<T, S>(P, lam(cur), lam(cur ^ 1), q, pv, pk);
            enqueue_inverse<T, S>(P, lam(cur ^ 1), lam(cur ^ 1), q, pv, pk);
            hip_check(dsbt::launch_grad_s<S>(P->d_fchans, nch, state(t), state(t + 1), lam(cur ^ 1), lam(cur),
                                             P->d_scratch, P->seg_gs + t, q), "grad_s");
            cur ^= 1;
        }
        return;
    }
    const dsbt::PhaseArgs none{};
    hipStream_t a = P->seg_side;
    hip_check(hipEventRecord(P->seg_fork, q), "segment fork");
    hip_check(hipStreamWaitEvent(a, P->seg_fork, 0), "segment fork");
    {
        void* w = lam(n + 1);
        const dsbt::PhaseArgs pk{1, 0, nullptr, 0};
        auto pv = [&](int t) { return dsbt::PhaseArgs{1, 0, P->seg_s, t}; };
        enqueue_fstage<T, S>(P, state(0), w, 0, pv(0), none, q);
        for (int t = 0; t < n; ++t) {
            enqueue_mstage<T, S>(P, w, w, false, q, pk);
            enqueue_mstage<T, S>(P, w, w, true, q, pk);
            if (t + 1 < n)
                enqueue_fstage<T, S>(P, w, w, 2, pv(t), pv(t + 1), q, state(t + 1));
            else
                enqueue_fstage<T, S>(P, w, state(n), 1, pv(t), none, q);
        }
    }
    {
        void* w = lam(n + 2);
        const dsbt::PhaseArgs pk{1, 1, nullptr, 0};
        auto pv = [&](int t) { return dsbt::PhaseArgs{1, 1, P->seg_s, t}; };
        enqueue_fstage<T, S>(P, lam(n), w, 0, pv(n - 1), none, a);
        for (int t = n - 1; t >= 0; --t) {
            enqueue_mstage<T, S>(P, w, w, false, a, pk);
            enqueue_mstage<T, S>(P, w, w, true, a, pk);
            if (t > 0)
                enqueue_fstage<T, S>(P, w, w, 2, pv(t), pv(t - 1), a, lam(t));
            else
                enqueue_fstage<T, S>(P, w, lam(0), 1, pv(t), none, a);
        }
    }
    hip_check(hipEventRecord(P->seg_join, a), "segment join");
    hip_check(hipStreamWaitEvent(q, P->seg_join, 0), "segment join");
    hip_check(dsbt::launch_grad_s_steps<S>(P->d_fchans, nch, n, state(0), lam(0), (int64_t)P->elems, P->seg_part,
                                           P->seg_gs, q), "grad_s");
}

// Checked plans: scan the channels of `data` for NaN and infinities on s and
// wait for the answer.
void check_finite_data(dsbt_plan_s* P, const void* data, hipStream_t s, const char* what) {
    const int nch = (int)P->ch.size();
    if (P->precision == DSBT_C128)
        hip_check(dsbt::launch_scan_nonfinite<double>(P->d_fchans, nch, data, P->d_flag, s), "scan");
    else
        hip_check(dsbt::launch_scan_nonfinite<float>(P->d_fchans, nch, data, P->d_flag, s), "scan");
    hip_check(hipMemcpyAsync(P->h_flag, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, s), "scan flag");
    hip_check(hipStreamSynchronize(s), "scan sync");
    if (*P->h_flag) throw StatusError(DSBT_ERR_NONFINITE, std::string(what) + ": NaN or infinity in the data");
}

template <typename F>
dsbt_status guarded(F&& f) {
    try {
        return f();
    } catch (const StatusError& e) {
        return fail(e.st, e.what());
    } catch (const HipError& e) {
        return fail(DSBT_ERR_HIP, e.what());
    } catch (const std::bad_alloc&) {
        return fail(DSBT_ERR_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(DSBT_ERR_INVALID_ARG, e.what());
    }
}

}  // namespace

extern "C" {

void dsbt_plan_opts_default(dsbt_plan_opts* o) {
    if (o) std::memset(o, 0, sizeof(*o));
}

dsbt_status dsbt_plan_create(dsbt_plan* out, const dsbt_channel* ch, int32_t nch, const dsbt_plan_opts* o,
                             void* stream) {
    Range range("dsbt_plan_create");
    if (!out) return fail(DSBT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    return guarded([&]() -> dsbt_status {
        dsbt_plan_opts opts{};
        if (o) opts = *o;
        if (opts.precision != DSBT_C64 && opts.precision != DSBT_C128 && opts.precision != DSBT_C64_FP64)
            return fail(DSBT_ERR_INVALID_ARG, "unknown precision");
        if (opts.kinetic != DSBT_K_PLAIN && opts.kinetic != DSBT_K_CORRECTED)
            return fail(DSBT_ERR_INVALID_ARG, "unknown kinetic option");
        if (opts.mode != DSBT_MODE_BATCHED && opts.mode != DSBT_MODE_PLAIN)
            return fail(DSBT_ERR_INVALID_ARG, "unknown mode");
        if (opts.plan_where != DSBT_PLAN_ON_DEVICE && opts.plan_where != DSBT_PLAN_ON_HOST)
            return fail(DSBT_ERR_INVALID_ARG, "unknown plan_where");
        if (opts.algorithm != DSBT_ALG_TILED && opts.algorithm != DSBT_ALG_MONOMIAL)
            return fail(DSBT_ERR_INVALID_ARG, "unknown algorithm");
        if (opts.check_finite != 0 && opts.check_finite != 1) return fail(DSBT_ERR_INVALID_ARG, "check_finite must be 0 or 1");
        if ((opts.dev_alloc == nullptr) != (opts.dev_free == nullptr))
            return fail(DSBT_ERR_INVALID_ARG, "dev_alloc and dev_free must be given together");
        if (opts.algorithm == DSBT_ALG_MONOMIAL) {
            if (opts.precision != DSBT_C128 || opts.mode != DSBT_MODE_BATCHED)
                return fail(DSBT_ERR_UNSUPPORTED, "the monomial variant needs DSBT_C128 and DSBT_MODE_BATCHED");
            for (int c = 0; ch && c < nch; ++c) {
                const int k = (ch[c].ell + 1) / 2;
                if (k > 64 || (ch[c].ell > 1 && (ch[c].ell - 1) * std::log10((double)ch[c].N) > 300.0))
                    return fail(DSBT_ERR_UNSUPPORTED, "monomial variant: N^(l-1) exceeds the FP64 range or l > 128");
            }
        }
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(DSBT_ERR_NO_DEVICE, "no HIP device");
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        hipDeviceProp_t prop;
        hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
        size_t max_lds = prop.sharedMemPerBlock;
        if (prop.maxSharedMemoryPerMultiProcessor > max_lds) max_lds = prop.maxSharedMemoryPerMultiProcessor;
        dsbt_status st = validate_channels(ch, nch, opts.precision, max_lds);
        if (st != DSBT_OK) return st;
        dsbt_plan_s* P = new dsbt_plan_s();
        P->device = dev;
        P->opts = opts;
        P->precision = opts.precision;
        P->elem_bytes = opts.precision == DSBT_C128 ? 16 : 8;
        P->cmp_bytes = opts.precision == DSBT_C64 ? 8 : 16;
        P->ch.assign(ch, ch + nch);
        for (auto& x : P->ch) P->elems = std::max<int64_t>(P->elems, x.offset + x.N);
        try {
            hipStream_t s = (hipStream_t)stream;
            if (P->precision == DSBT_C64)
                build_plan<float>(P, s);
            else
                build_plan<double>(P, s);   // complex128, or complex64 data with FP64 arithmetic
            if (P->opts.check_finite) {
                P->d_flag = static_cast<int*>(P->dalloc(sizeof(int)));
                hip_check(hipHostMalloc((void**)&P->h_flag, sizeof(int), hipHostMallocDefault), "hipHostMalloc");
            }
            hip_check(hipStreamSynchronize(s), "plan sync");
        } catch (...) {
            P->release();
            delete P;
            throw;
        }
        *out = P;
        return DSBT_OK;
    });
}

dsbt_status dsbt_plan_create_uniform(dsbt_plan* out, int32_t N, double rmax, const int32_t* ells, int32_t nell,
                                     int32_t all_m, const dsbt_plan_opts* o, void* stream) {
    if (!out) return fail(DSBT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!ells || nell <= 0) return fail(DSBT_ERR_INVALID_ARG, "no l values");
    std::vector<dsbt_channel> ch;
    int64_t off = 0;
    for (int i = 0; i < nell; ++i) {
        if (ells[i] < 0) return fail(DSBT_ERR_UNSUPPORTED, "negative l");
        const int reps = all_m ? 2 * ells[i] + 1 : 1;
        for (int m = 0; m < reps; ++m) {
            ch.push_back(dsbt_channel{N, ells[i], rmax, off});
            off += N;
        }
    }
    return dsbt_plan_create(out, ch.data(), (int32_t)ch.size(), o, stream);
}

dsbt_status dsbt_plan_destroy(dsbt_plan p) {
    if (!p) return DSBT_OK;
    p->release();
    delete p;
    return DSBT_OK;
}

dsbt_status dsbt_plan_info(dsbt_plan p, int32_t* nch, int64_t* elems, int32_t* precision, int64_t* table_bytes) {
    if (!p) return fail(DSBT_ERR_INVALID_ARG, "plan is NULL");
    if (nch) *nch = (int32_t)p->ch.size();
    if (elems) *elems = p->elems;
    if (precision) *precision = p->precision;
    if (table_bytes) *table_bytes = p->table_bytes;
    return DSBT_OK;
}

dsbt_status dsbt_forward(dsbt_plan p, const void* psi, void* b, void* stream) {
    Range range("dsbt_forward");
    if (!p || !psi || !b) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    return guarded([&]() -> dsbt_status {
        if (p->opts.check_finite) check_finite_data(p, psi, (hipStream_t)stream, "dsbt_forward input");
        dsbt::PhaseArgs none{};
        if (p->precision == DSBT_C128)
            enqueue_forward<double, double>(p, psi, b, (hipStream_t)stream, none, none);
        else if (p->precision == DSBT_C64_FP64)
            enqueue_forward<double, float>(p, psi, b, (hipStream_t)stream, none, none);
        else
            enqueue_forward<float, float>(p, psi, b, (hipStream_t)stream, none, none);
        return DSBT_OK;
    });
}

dsbt_status dsbt_inverse(dsbt_plan p, const void* b, void* psi, void* stream) {
    Range range("dsbt_inverse");
    if (!p || !psi || !b) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    return guarded([&]() -> dsbt_status {
        if (p->opts.check_finite) check_finite_data(p, b, (hipStream_t)stream, "dsbt_inverse input");
        dsbt::PhaseArgs none{};
        if (p->precision == DSBT_C128)
            enqueue_inverse<double, double>(p, b, psi, (hipStream_t)stream, none);
        else if (p->precision == DSBT_C64_FP64)
            enqueue_inverse<double, float>(p, b, psi, (hipStream_t)stream, none);
        else
            enqueue_inverse<float, float>(p, b, psi, (hipStream_t)stream, none);
        return DSBT_OK;
    });
}

dsbt_status dsbt_set_potential(dsbt_plan p, const double* V, double dt) {
    return dsbt_set_potential_ex(p, V, dt, 0);
}

dsbt_status dsbt_set_potential_ex(dsbt_plan p, const double* V, double dt, int32_t flags) {
    Range range("dsbt_set_potential");
    if (!p || !V) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DSBT_ERR_INVALID_ARG, "dt must be positive");
    if (flags & ~DSBT_TIME_IMAGINARY) return fail(DSBT_ERR_INVALID_ARG, "unknown potential flag");
    const bool imag = (flags & DSBT_TIME_IMAGINARY) != 0;
    return guarded([&]() -> dsbt_status {
        const int64_t n = p->elems;
        const bool fp64 = p->precision != DSBT_C64;   // phases in the arithmetic precision
        std::vector<double> ang(n, 0.0);
        for (auto& x : p->ch) {
            for (int i = 0; i < x.N; ++i) {
                const double v = V[x.offset + i];
                if (!std::isfinite(v)) throw StatusError(DSBT_ERR_INVALID_ARG, "non-finite potential");
                ang[x.offset + i] = v * dt / 2.0;
            }
        }
        const std::vector<unsigned char> ph = imag ? decay_table(ang, fp64) : phase_table(ang, fp64);
        if (!p->d_vphase) {
            p->d_vphase = p->dalloc(ph.size());
            p->d_vangle = (double*)p->dalloc(sizeof(double) * n);
        }
        hip_check(hipMemcpy(p->d_vphase, ph.data(), ph.size(), hipMemcpyHostToDevice), "vphase");
        hip_check(hipMemcpy(p->d_vangle, ang.data(), sizeof(double) * n, hipMemcpyHostToDevice), "vangle");
        // kinetic phases per group: K = (n dk)^2/2 for regular rows, (N dk)^2/2 for completion rows
        const double pi = 3.14159265358979323846;
        for (auto& g : p->groups) {
            const double dk = pi / g.rmax;
            std::vector<double> ka(g.N), kin(g.N), kc;
            if (p->opts.kinetic == DSBT_K_CORRECTED) {
                kc.resize(g.N);
                dsbt::corrected_momenta(g.N, g.ell, g.rmax, kc.data());
            }
            for (int j = 0; j < g.N; ++j) {
                const int nidx = j + g.p;
                const double kn = !kc.empty() ? kc[j] : ((j < g.k) ? g.N * dk : nidx * dk);
                kin[j] = 0.5 * kn * kn;
                ka[j] = kin[j] * dt;
            }
            const std::vector<unsigned char> kp = imag ? decay_table(ka, fp64) : phase_table(ka, fp64);
            if (!g.d_kphase) g.d_kphase = p->dalloc(kp.size());
            hip_check(hipMemcpy(g.d_kphase, kp.data(), kp.size(), hipMemcpyHostToDevice), "kphase");
            if (!g.d_kin) g.d_kin = (double*)p->dalloc(sizeof(double) * g.N);
            hip_check(hipMemcpy(g.d_kin, kin.data(), sizeof(double) * g.N, hipMemcpyHostToDevice), "kin");
        }
        // energy descriptors
        {
            std::vector<dsbt::EChan> ec(p->ch.size());
            for (auto& g : p->groups)
                for (int c : g.chans)
                    ec[c] = dsbt::EChan{p->ch[c].offset, p->ch[c].N, 0, p->d_vangle + p->ch[c].offset, g.d_kin};
            if (!p->d_echans) p->d_echans = (dsbt::EChan*)p->dalloc(sizeof(dsbt::EChan) * ec.size());
            hip_check(hipMemcpy(p->d_echans, ec.data(), sizeof(dsbt::EChan) * ec.size(), hipMemcpyHostToDevice),
                      "echans");
        }
        // refresh descriptors with the phase pointers (FP32 plans: the lo parts
        // follow the hi parts of all n points)
        for (size_t c = 0; c < p->ch.size(); ++c) {
            const auto* base = static_cast<const unsigned char*>(p->d_vphase);
            p->h_fchans[c].vphase = base + p->cmp_bytes * p->ch[c].offset;
            p->h_fchans[c].vphase_lo = fp64 ? nullptr : base + p->cmp_bytes * (n + p->ch[c].offset);
            p->h_fchans[c].vangle = p->d_vangle + p->ch[c].offset;
        }
        hip_check(hipMemcpy(p->d_fchans, p->h_fchans.data(), sizeof(dsbt::FChan) * p->ch.size(),
                            hipMemcpyHostToDevice), "fchans");
        upload_fchans_n(p);
        std::map<int64_t, const dsbt_plan_s::Group*> by_off;
        for (auto& g : p->groups)
            for (int c : g.chans) by_off[p->ch[c].offset] = &g;
        auto refresh = [&](std::vector<dsbt::MItem>& v, dsbt::MItem* d) {
            for (auto& it : v) {
                if (it.nch <= 0) continue;
                const auto* g = by_off[it.off[0]];
                it.kphase = g->d_kphase;
                it.kphase_lo = fp64 ? nullptr : static_cast<const unsigned char*>(g->d_kphase) + sizeof(float2) * g->N;
            }
            if (d) hip_check(hipMemcpy(d, v.data(), sizeof(dsbt::MItem) * v.size(), hipMemcpyHostToDevice), "items");
        };
        if (p->d_lchans) {
            for (auto& x : p->h_lchans) x.kphase = by_off[x.off]->d_kphase;
            hip_check(hipMemcpy(p->d_lchans, p->h_lchans.data(), sizeof(dsbt::LChan) * p->h_lchans.size(),
                                hipMemcpyHostToDevice), "monomial channels");
        }
        refresh(p->h_items_mf, p->d_items_mf);
        refresh(p->h_items_v1, p->d_items_v1);
        refresh(p->h_items1, p->d_items1);
        p->has_potential = true;
        p->imaginary = imag;
        p->dt = dt;
        p->drop_graphs();
        return DSBT_OK;
    });
}

dsbt_status dsbt_kinetic_step(dsbt_plan p, void* psi, int32_t nsteps, const float* s, int32_t flags, void* stream) {
    Range range("dsbt_kinetic_step");
    if (!p || !psi) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (nsteps < 0) return fail(DSBT_ERR_INVALID_ARG, "negative step count");
    if (!p->has_potential) return fail(DSBT_ERR_PLAN_MISMATCH, "dsbt_set_potential has not been called");
    if (flags & ~(DSBT_STEP_ADJOINT | DSBT_STEP_GRAPH | DSBT_STEP_RESIDENT))
        return fail(DSBT_ERR_INVALID_ARG, "unknown step flag");
    if (flags & DSBT_STEP_RESIDENT) return fail(DSBT_ERR_UNSUPPORTED, "resident step kernel not built in");
    if (p->imaginary && s) return fail(DSBT_ERR_INVALID_ARG, "strengths are not supported in imaginary time");
    if (nsteps == 0) return DSBT_OK;
    return guarded([&]() -> dsbt_status {
        hipStream_t st = (hipStream_t)stream;
        const bool adj = (flags & DSBT_STEP_ADJOINT) != 0;
        if (p->opts.check_finite) {
            check_finite_data(p, psi, st, "dsbt_kinetic_step input");
            flags &= ~DSBT_STEP_GRAPH;   // a checked call synchronises; it is not worth a graph
        }
        auto enqueue = [&](hipStream_t q) {
            if (p->precision == DSBT_C128)
                enqueue_steps<double, double>(p, psi, nsteps, s, adj, q);
            else if (p->precision == DSBT_C64_FP64)
                enqueue_steps<double, float>(p, psi, nsteps, s, adj, q);
            else
                enqueue_steps<float, float>(p, psi, nsteps, s, adj, q);
        };
        if (!(flags & DSBT_STEP_GRAPH)) {
            enqueue(st);
            if (p->opts.check_finite) check_finite_data(p, psi, st, "dsbt_kinetic_step result");
            return DSBT_OK;
        }
        // The strengths are staged into a plan buffer that the graph reads, so a
        // replay with other strengths (same psi, nsteps, flags) reuses the graph.
        if (s) {
            if (p->sgraph_cap < nsteps) {
                p->d_sgraph = static_cast<float*>(p->dalloc(sizeof(float) * (size_t)nsteps));
                p->sgraph_cap = nsteps;
            }
            hip_check(hipMemcpyAsync(p->d_sgraph, s, sizeof(float) * (size_t)nsteps, hipMemcpyDeviceToDevice, st),
                      "stage strengths");
            s = p->d_sgraph;
        }
        auto key = std::make_tuple(psi, (int)nsteps, s, (int)flags);
        if (!p->graph_exec || p->graph_key != key) {
            if (p->graph_exec) {
                (void)hipGraphExecDestroy(p->graph_exec);
                (void)hipGraphDestroy(p->graph);
                p->graph_exec = nullptr;
                p->graph = nullptr;
            }
            capture_graph(enqueue, &p->graph, &p->graph_exec);
            p->graph_key = key;
        }
        hip_check(hipGraphLaunch(p->graph_exec, st), "graph launch");
        return DSBT_OK;
    });
}

dsbt_status dsbt_step_grad_s(dsbt_plan p, const void* psi_t, const void* psi_t1, const void* lam_t,
                             const void* lam_t1, double* out, void* stream) {
    Range range("dsbt_step_grad_s");
    if (!p || !psi_t || !psi_t1 || !lam_t || !lam_t1 || !out) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_potential) return fail(DSBT_ERR_PLAN_MISMATCH, "dsbt_set_potential has not been called");
    if (p->imaginary) return fail(DSBT_ERR_PLAN_MISMATCH, "the potential was set for imaginary time");
    return guarded([&]() -> dsbt_status {
        const int nch = (int)p->ch.size();
        hipStream_t st = (hipStream_t)stream;
        if (p->precision == DSBT_C128)
            hip_check(dsbt::launch_grad_s<double>(p->d_fchans, nch, psi_t, psi_t1, lam_t, lam_t1, p->d_scratch, out,
                                                  st), "grad_s");
        else
            hip_check(dsbt::launch_grad_s<float>(p->d_fchans, nch, psi_t, psi_t1, lam_t, lam_t1, p->d_scratch, out,
                                                 st), "grad_s");
        return DSBT_OK;
    });
}

dsbt_status dsbt_adjoint_segment(dsbt_plan p, const void* psi_a, int32_t nsteps, const float* s, void* lam,
                                 double* gs, int32_t flags, void* stream) {
    Range range("dsbt_adjoint_segment");
    if (!p || !psi_a || !s || !lam || !gs) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (nsteps < 1) return fail(DSBT_ERR_INVALID_ARG, "a segment has at least one step");
    if (flags & ~DSBT_STEP_GRAPH) return fail(DSBT_ERR_INVALID_ARG, "unknown segment flag");
    if (!p->has_potential) return fail(DSBT_ERR_PLAN_MISMATCH, "dsbt_set_potential has not been called");
    if (p->imaginary) return fail(DSBT_ERR_PLAN_MISMATCH, "the potential was set for imaginary time");
    return guarded([&]() -> dsbt_status {
        hipStream_t st = (hipStream_t)stream;
        const size_t sb = (size_t)p->elems * p->elem_bytes;
        if (p->opts.check_finite) {
            check_finite_data(p, psi_a, st, "dsbt_adjoint_segment psi_a");
            check_finite_data(p, lam, st, "dsbt_adjoint_segment lam");
            flags &= ~DSBT_STEP_GRAPH;
        }
        if (p->seg_cap < nsteps) {
            hip_check(hipStreamSynchronize(st), "segment buffers");   // the old buffers may still be read
            p->drop_graphs();
            p->free_segment();
            p->seg_states = p->dalloc_raw(sb * (size_t)(nsteps + 1));
            p->seg_lam = p->dalloc_raw(sb * (size_t)(nsteps + 3));
            p->seg_s = static_cast<float*>(p->dalloc_raw(sizeof(float) * (size_t)nsteps));
            p->seg_gs = static_cast<double*>(p->dalloc_raw(sizeof(double) * (size_t)nsteps));
            p->seg_part = static_cast<double*>(p->dalloc_raw(sizeof(double) * (size_t)nsteps * p->ch.size()));
            p->seg_cap = nsteps;
        }
        if (p->opts.mode != DSBT_MODE_PLAIN && !p->seg_side) {
            hip_check(hipStreamCreateWithFlags(&p->seg_side, hipStreamNonBlocking), "segment stream");
            hip_check(hipEventCreateWithFlags(&p->seg_fork, hipEventDisableTiming), "segment event");
            hip_check(hipEventCreateWithFlags(&p->seg_join, hipEventDisableTiming), "segment event");
        }
        auto lam_buf = [&](int t) { return static_cast<unsigned char*>(p->seg_lam) + sb * (size_t)t; };
        hip_check(hipMemcpyAsync(p->seg_states, psi_a, sb, hipMemcpyDeviceToDevice, st), "segment psi_a");
        // lam_{a+n} where the steps start from it (buffer n batched, 0 plain);
        // the buffer lam_a ends in also gets lam, as its gaps between
        // channels (never written by the steps) must hold lam's
        const int first = p->opts.mode == DSBT_MODE_PLAIN ? 0 : nsteps, last = segment_result_buffer(p, nsteps);
        hip_check(hipMemcpyAsync(lam_buf(first), lam, sb, hipMemcpyDeviceToDevice, st), "segment lam");
        if (last != first)
            hip_check(hipMemcpyAsync(lam_buf(last), lam, sb, hipMemcpyDeviceToDevice, st), "segment lam");
        hip_check(hipMemcpyAsync(p->seg_s, s, sizeof(float) * (size_t)nsteps, hipMemcpyDeviceToDevice, st),
                  "segment strengths");
        auto enqueue = [&](hipStream_t q) {
            if (p->precision == DSBT_C128)
                enqueue_segment<double, double>(p, nsteps, q);
            else if (p->precision == DSBT_C64_FP64)
                enqueue_segment<double, float>(p, nsteps, q);
            else
                enqueue_segment<float, float>(p, nsteps, q);
        };
        if (flags & DSBT_STEP_GRAPH) {
            if (!p->seg_exec || p->seg_graph_n != nsteps) {
                if (p->seg_exec) (void)hipGraphExecDestroy(p->seg_exec);
                if (p->seg_graph) (void)hipGraphDestroy(p->seg_graph);
                p->seg_exec = nullptr;
                p->seg_graph = nullptr;
                capture_graph(enqueue, &p->seg_graph, &p->seg_exec);
                p->seg_graph_n = nsteps;
            }
            hip_check(hipGraphLaunch(p->seg_exec, st), "graph launch");
        } else {
            enqueue(st);
        }
        hip_check(hipMemcpyAsync(lam, lam_buf(last), sb, hipMemcpyDeviceToDevice, st), "segment lam_a");
        hip_check(hipMemcpyAsync(gs, p->seg_gs, sizeof(double) * (size_t)nsteps, hipMemcpyDeviceToDevice, st),
                  "segment gradients");
        if (p->opts.check_finite) check_finite_data(p, lam, st, "dsbt_adjoint_segment result");
        return DSBT_OK;
    });
}

dsbt_status dsbt_step_grad_s_noalloc(dsbt_plan p, const void* psi_t, const void* psi_t1, const void* lam_t,
                                     const void* lam_t1, double* out, void* stream) {
    if (!p || !psi_t || !psi_t1 || !lam_t || !lam_t1 || !out) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (!p->has_potential) return fail(DSBT_ERR_PLAN_MISMATCH, "dsbt_set_potential has not been called");
    if (p->imaginary) return fail(DSBT_ERR_PLAN_MISMATCH, "the potential was set for imaginary time");
    const int nch = (int)p->ch.size();
    if (nch > DSBT_NOALLOC_MAX_CHANNELS)
        return fail(DSBT_ERR_UNSUPPORTED, "dsbt_step_grad_s_noalloc: the plan has " + std::to_string(nch) +
                                              " channels, more than DSBT_NOALLOC_MAX_CHANNELS = " +
                                              std::to_string(DSBT_NOALLOC_MAX_CHANNELS));
    return guarded([&]() -> dsbt_status {
        double* part = noalloc_scratch_ptr();
        hipStream_t st = (hipStream_t)stream;
        // the partial sums are written (not accumulated) for every channel before they are read
        if (p->precision == DSBT_C128)
            hip_check(dsbt::launch_grad_s<double>(p->d_fchans, nch, psi_t, psi_t1, lam_t, lam_t1, part, out, st),
                      "grad_s");
        else
            hip_check(dsbt::launch_grad_s<float>(p->d_fchans, nch, psi_t, psi_t1, lam_t, lam_t1, part, out, st),
                      "grad_s");
        return DSBT_OK;
    });
}

dsbt_status dsbt_energy(dsbt_plan p, const void* psi, void* work, double* out, void* stream) {
    Range range("dsbt_energy");
    if (!p || !psi || !work || !out) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (psi == work) return fail(DSBT_ERR_INVALID_ARG, "work must not alias psi");
    if (!p->has_potential) return fail(DSBT_ERR_PLAN_MISMATCH, "dsbt_set_potential has not been called");
    return guarded([&]() -> dsbt_status {
        hipStream_t st = (hipStream_t)stream;
        dsbt::PhaseArgs none{};
        const int nch = (int)p->ch.size();
        const double vscale = 2.0 / p->dt;   // d_vangle holds V tau/2
        if (p->precision == DSBT_C128) {
            enqueue_forward<double, double>(p, psi, work, st, none, none);
            hip_check(dsbt::launch_energy_terms<double>(p->d_echans, nch, psi, work, vscale, out, st), "energy");
        } else {
            if (p->precision == DSBT_C64_FP64)
                enqueue_forward<double, float>(p, psi, work, st, none, none);
            else
                enqueue_forward<float, float>(p, psi, work, st, none, none);
            hip_check(dsbt::launch_energy_terms<float>(p->d_echans, nch, psi, work, vscale, out, st), "energy");
        }
        return DSBT_OK;
    });
}

dsbt_status dsbt_orthonormalize(dsbt_plan p, void* psi, const int32_t* sets, int32_t nsets, void* stream) {
    if (!p || !psi || (!sets && nsets > 0)) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (nsets < 0) return fail(DSBT_ERR_INVALID_ARG, "negative set count");
    if (nsets == 0) return DSBT_OK;
    const int nch = (int)p->ch.size();
    for (int k = 0; k < nsets; ++k) {
        if (sets[k] < 0 || sets[k + 1] <= sets[k] || sets[k + 1] > nch)
            return fail(DSBT_ERR_INVALID_ARG, "set boundaries must increase strictly within [0, nch]");
        for (int c = sets[k] + 1; c < sets[k + 1]; ++c)
            if (p->ch[c].N != p->ch[sets[k]].N) return fail(DSBT_ERR_INVALID_ARG, "channels of a set differ in N");
    }
    return guarded([&]() -> dsbt_status {
        hipStream_t st = (hipStream_t)stream;
        if (!p->d_off) {
            std::vector<int64_t> off(nch);
            std::vector<int> n(nch);
            for (int c = 0; c < nch; ++c) {
                off[c] = p->ch[c].offset;
                n[c] = p->ch[c].N;
            }
            p->d_off = (int64_t*)p->dalloc(sizeof(int64_t) * nch);
            p->d_nch = (int*)p->dalloc(sizeof(int) * nch);
            hip_check(hipMemcpy(p->d_off, off.data(), sizeof(int64_t) * nch, hipMemcpyHostToDevice), "offsets");
            hip_check(hipMemcpy(p->d_nch, n.data(), sizeof(int) * nch, hipMemcpyHostToDevice), "sizes");
        }
        const std::vector<int> want(sets, sets + nsets + 1);
        if (want != p->h_sets) {
            // a new set table: wait until no queued launch can still read the old one
            hip_check(hipStreamSynchronize(st), "stream synchronize");
            if (p->sets_cap < nsets + 1) {
                p->d_sets = (int*)p->dalloc(sizeof(int) * (nsets + 1));
                p->sets_cap = nsets + 1;
            }
            hip_check(hipMemcpy(p->d_sets, want.data(), sizeof(int) * (nsets + 1), hipMemcpyHostToDevice), "sets");
            p->h_sets = want;
        }
        if (p->precision == DSBT_C128)
            hip_check(dsbt::launch_orthonormalize<double>(p->d_off, p->d_nch, p->d_sets, nsets, psi, st), "orthonormalize");
        else
            hip_check(dsbt::launch_orthonormalize<float>(p->d_off, p->d_nch, p->d_sets, nsets, psi, st), "orthonormalize");
        return DSBT_OK;
    });
}

dsbt_status dsbt_profile_enable(dsbt_plan p, int32_t enable) {
    if (!p) return fail(DSBT_ERR_INVALID_ARG, "plan is NULL");
    return guarded([&]() -> dsbt_status {
        if (enable == 1) {
            for (auto& t : p->prof_events) {
                p->event_pool.push_back(std::get<1>(t));
                p->event_pool.push_back(std::get<2>(t));
            }
            p->prof_events.clear();
        }
        p->profiling = enable != 0;
        return DSBT_OK;
    });
}

dsbt_status dsbt_profile_read(dsbt_plan p, double* ms, int64_t* launches, int32_t nstages) {
    if (!p || !ms || !launches || nstages < 0 || nstages > DSBT_NUM_STAGES)
        return fail(DSBT_ERR_INVALID_ARG, "bad profile arguments");
    return guarded([&]() -> dsbt_status {
        for (int i = 0; i < nstages; ++i) {
            ms[i] = 0.0;
            launches[i] = 0;
        }
        for (auto& t : p->prof_events) {
            const int st = std::get<0>(t);
            hip_check(hipEventSynchronize(std::get<2>(t)), "hipEventSynchronize");
            float e = 0.0f;
            hip_check(hipEventElapsedTime(&e, std::get<1>(t), std::get<2>(t)), "hipEventElapsedTime");
            if (st < nstages) {
                ms[st] += e;
                launches[st] += 1;
            }
        }
        return DSBT_OK;
    });
}

dsbt_status dsbt_host_ftb_tables(int32_t N, int32_t ell, int32_t B, double* out, int64_t out_len, int64_t* needed) {
    if (!is_pow2(N) || N < 2) return fail(DSBT_ERR_UNSUPPORTED, "N must be a power of two");
    if (ell < 0 || ell > 2 * N - 2) return fail(DSBT_ERR_UNSUPPORTED, "need 0 <= l <= 2N-2");
    if (!is_pow2(B) || B > N || B < dsbt::n0_of(ell)) return fail(DSBT_ERR_UNSUPPORTED, "bad tile");
    const int R = B + dsbt::n_extra(ell), NT = N / B;
    const int64_t need = (int64_t)R * R * NT;
    if (needed) *needed = need;
    if (!out || out_len < need) return DSBT_OK;
    return guarded([&]() -> dsbt_status {
        std::vector<double> blk;
        dsbt::build_ftb_blocks(ell, B, NT, blk, 0);
        std::memcpy(out, blk.data(), sizeof(double) * blk.size());
        return DSBT_OK;
    });
}

dsbt_status dsbt_host_monomial_tables(int32_t N, int32_t ell, double* xi, double* alpha, double* comp,
                                      int64_t* sizes) {
    if (N < 2 || ell < 0 || ell > 2 * N - 2 || (ell + 1) / 2 > 64) return fail(DSBT_ERR_UNSUPPORTED, "bad N or l");
    return guarded([&]() -> dsbt_status {
        std::vector<double> x, a, c;
        dsbt::monomial_tables(N, ell, x, a, c);
        if (sizes) {
            sizes[0] = (int64_t)x.size();
            sizes[1] = (int64_t)a.size();
            sizes[2] = (int64_t)c.size();
        }
        if (xi) std::copy(x.begin(), x.end(), xi);
        if (alpha) std::copy(a.begin(), a.end(), alpha);
        if (comp) std::copy(c.begin(), c.end(), comp);
        return DSBT_OK;
    });
}

dsbt_status dsbt_device_ftb_tables(int32_t N, int32_t ell, int32_t B, double* out, int64_t out_len,
                                   int64_t* needed, void* stream) {
    if (!is_pow2(N) || N < 2) return fail(DSBT_ERR_UNSUPPORTED, "N must be a power of two");
    if (ell < 0 || ell > 2 * N - 2 || ell > 255) return fail(DSBT_ERR_UNSUPPORTED, "need 0 <= l <= min(2N-2, 255)");
    if (!is_pow2(B) || B > N || B < dsbt::n0_of(ell)) return fail(DSBT_ERR_UNSUPPORTED, "bad tile");
    const int R = B + dsbt::n_extra(ell), NT = N / B;
    const int64_t need = (int64_t)R * R * NT;
    if (needed) *needed = need;
    if (!out || out_len < need) return DSBT_OK;
    return guarded([&]() -> dsbt_status {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(DSBT_ERR_NO_DEVICE, "no HIP device");
        DeviceScratch scratch;
        scratch.alloc(dsbt::device_plan_scratch_doubles(ell, B, NT));
        std::vector<double> blk;
        device_blocks(ell, B, NT, scratch.ptr, blk, (hipStream_t)stream);
        std::memcpy(out, blk.data(), sizeof(double) * blk.size());
        return DSBT_OK;
    });
}

dsbt_status dsbt_kinetic_momenta(int32_t N, int32_t ell, double rmax, int32_t kinetic, double* k) {
    if (!k) return fail(DSBT_ERR_INVALID_ARG, "NULL argument");
    if (!is_pow2(N) || N < 2) return fail(DSBT_ERR_UNSUPPORTED, "N must be a power of two");
    if (ell < 0 || ell > 2 * N - 2 || ell > 255) return fail(DSBT_ERR_UNSUPPORTED, "need 0 <= l <= min(2N-2, 255)");
    if (!(rmax > 0.0)) return fail(DSBT_ERR_INVALID_ARG, "rmax must be positive");
    if (kinetic != DSBT_K_PLAIN && kinetic != DSBT_K_CORRECTED) return fail(DSBT_ERR_INVALID_ARG, "unknown kinetic option");
    return guarded([&]() -> dsbt_status {
        const double dk = 3.14159265358979323846 / rmax;
        const int p = dsbt::parity_p(ell), kx = dsbt::n_extra(ell);
        if (kinetic == DSBT_K_CORRECTED) {
            dsbt::corrected_momenta(N, ell, rmax, k);
        } else {
            for (int j = 0; j < N; ++j) k[j] = (j < kx) ? N * dk : (j + p) * dk;
        }
        return DSBT_OK;
    });
}

const char* dsbt_status_string(dsbt_status s) {
    switch (s) {
        case DSBT_OK: return "ok";
        case DSBT_ERR_INVALID_ARG: return "invalid argument";
        case DSBT_ERR_UNSUPPORTED: return "unsupported size or option";
        case DSBT_ERR_OOM: return "out of memory";
        case DSBT_ERR_HIP: return "HIP error";
        case DSBT_ERR_PLAN_MISMATCH: return "call does not fit the plan";
        case DSBT_ERR_NONFINITE: return "NaN or infinity in the data";
        case DSBT_ERR_NO_DEVICE: return "no HIP device";
        default: return "unknown status";
    }
}

const char* dsbt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
