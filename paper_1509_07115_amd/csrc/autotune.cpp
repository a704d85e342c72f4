// Tile and batch-shape search for a channel set (dsbt_autotune).
//
// Candidates are the moment tile B (0 = the plan's own choice per l, 32, 64)
// crossed with the channels per moment work item (0 = the plan's own choice,
// 8, 4).  Each candidate is a full plan; those the channel set does not admit
// (a tile below ceil((l+1)/2) or above N) are skipped.  A candidate is timed
// with HIP events over `nrep` forward + inverse pairs on device scratch
// buffers, after one untimed pair.  The buffers hold hashed pseudo-random
// values in [-1, 1): the transforms have no data-dependent control flow, but
// constant data draws less power and can run at higher clocks than real data.
//
// Results are cached as JSON lines, one object per tuned channel set:
//   {"key": "<16 hex>", "tile": B, "chans_per_block": C, "ms": t}
// The key hashes (FNV-1a, 64 bit) the device's architecture name, the
// precision, the mode and the sorted (N, l, count) multiset of the channels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dsbt.h"

namespace {

// x[i] = a value in [-1, 1) hashed from i (one 32-bit mix per scalar)
template <typename S>
__global__ void fill_hashed(S* x, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 16;
    h *= 2246822519u;
    h ^= h >> 13;
    x[i] = (S)((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
}

uint64_t fnv1a(const std::string& s) {
    uint64_t h = 1469598103934665603ull;
    for (unsigned char c : s) {
        h ^= c;
        h *= 1099511628211ull;
    }
    return h;
}

std::string cache_key(const dsbt_channel* ch, int nch, const dsbt_plan_opts& o) {
    std::map<std::tuple<int, int, long long>, int> ms;
    for (int c = 0; c < nch; ++c) ms[std::make_tuple(ch[c].N, ch[c].ell, (long long)std::llround(ch[c].rmax * 1e6))]++;
    std::string s;
    int dev = 0;
    hipDeviceProp_t pr;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&pr, dev) == hipSuccess) s += pr.gcnArchName;
    s += "|p" + std::to_string(o.precision) + "|m" + std::to_string(o.mode) + "|a" + std::to_string(o.algorithm);
    for (auto& kv : ms)
        s += "|" + std::to_string(std::get<0>(kv.first)) + "," + std::to_string(std::get<1>(kv.first)) + "x" +
             std::to_string(kv.second);
    char buf[17];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)fnv1a(s));
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, int& tile, int& cpb, double& ms) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    const std::string want = "\"key\": \"" + key + "\"";
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strstr(line, want.c_str())) continue;
        int t = 0, c = 0;
        double m = 0;
        const char* pt = std::strstr(line, "\"tile\":");
        const char* pc = std::strstr(line, "\"chans_per_block\":");
        const char* pm = std::strstr(line, "\"ms\":");
        if (pt && pc && pm && std::sscanf(pt + 7, "%d", &t) == 1 && std::sscanf(pc + 18, "%d", &c) == 1 &&
            std::sscanf(pm + 5, "%lf", &m) == 1) {
            tile = t;
            cpb = c;
            ms = m;
            found = true;   // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, int tile, int cpb, double ms) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%s\", \"tile\": %d, \"chans_per_block\": %d, \"ms\": %.6f}\n", key.c_str(), tile, cpb,
                 ms);
    std::fclose(f);
}

}  // namespace

extern "C" dsbt_status dsbt_autotune(const dsbt_channel* ch, int32_t nch, const dsbt_plan_opts* base, int32_t nrep,
                                     const char* cache_path, dsbt_plan_opts* best, double* ms_out, void* stream) {
    if (!ch || nch <= 0 || !best || nrep <= 0) return DSBT_ERR_INVALID_ARG;
    dsbt_plan_opts o{};
    if (base) o = *base;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return DSBT_ERR_NO_DEVICE;
    const std::string key = cache_key(ch, nch, o);
    int tile = 0, cpb = 0;
    double ms = 0;
    if (cache_path && cache_lookup(cache_path, key, tile, cpb, ms)) {
        *best = o;
        best->tile = tile;
        best->chans_per_block = cpb;
        if (ms_out) *ms_out = ms;
        return DSBT_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    int64_t elems = 0;
    for (int c = 0; c < nch; ++c) elems = std::max<int64_t>(elems, ch[c].offset + ch[c].N);
    const size_t bytes = (size_t)elems * (o.precision == DSBT_C128 ? 16 : 8);
    void *x = nullptr, *y = nullptr;
    if (hipMalloc(&x, bytes) != hipSuccess) return DSBT_ERR_OOM;
    if (hipMalloc(&y, bytes) != hipSuccess) {
        (void)hipFree(x);
        return DSBT_ERR_OOM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    dsbt_status result = DSBT_ERR_UNSUPPORTED;
    double best_ms = 0;
    const size_t nscal = (size_t)elems * 2;
    const unsigned grid = (unsigned)((nscal + 255) / 256);
    if (o.precision == DSBT_C128)
        hipLaunchKernelGGL(fill_hashed<double>, dim3(grid), dim3(256), 0, s, (double*)x, nscal);
    else
        hipLaunchKernelGGL(fill_hashed<float>, dim3(grid), dim3(256), 0, s, (float*)x, nscal);
    if (hipGetLastError() != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        result = DSBT_ERR_HIP;
    } else {
        for (int t : {0, 32, 64}) {
            for (int c : {0, 8, 4}) {
                dsbt_plan_opts cand = o;
                cand.tile = t;
                cand.chans_per_block = c;
                dsbt_plan p = nullptr;
                if (dsbt_plan_create(&p, ch, nch, &cand, stream) != DSBT_OK) continue;   // not admitted
                bool ok = dsbt_forward(p, x, y, stream) == DSBT_OK && dsbt_inverse(p, y, x, stream) == DSBT_OK &&
                          hipEventRecord(e0, s) == hipSuccess;
                for (int r = 0; ok && r < nrep; ++r)
                    ok = dsbt_forward(p, x, y, stream) == DSBT_OK && dsbt_inverse(p, y, x, stream) == DSBT_OK;
                float t_ms = 0;
                ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&t_ms, e0, e1) == hipSuccess;
                dsbt_plan_destroy(p);
                if (!ok) {
                    result = DSBT_ERR_HIP;
                    break;
                }
                const double per = t_ms / nrep;
                if (result != DSBT_OK || per < best_ms) {
                    best_ms = per;
                    *best = cand;
                    result = DSBT_OK;
                }
            }
            if (result == DSBT_ERR_HIP) break;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(y);
    if (result == DSBT_OK) {
        if (ms_out) *ms_out = best_ms;
        if (cache_path) cache_store(cache_path, key, best->tile, best->chans_per_block, best_ms);
    }
    return result;
}
