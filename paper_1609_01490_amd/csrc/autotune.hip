// Autotuner: picks the tile size and the map (with or without the XCD
// swizzle) for a workload and a problem size by timing every candidate on
// this GPU with HIP events, on scratch buffers the tuner allocates itself.
// Results are kept in a process-wide cache keyed by GPU architecture, CU
// count, workload, size bucket (floor(log2 n)) and dimension, which can be
// saved to and loaded from a small JSON file.  Tiles never change integer or
// Life results (the bodies are the same), so the choice is purely a speed
// decision; for the distance map the tile changes only FP32 summation order.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace trimap {

struct TuneKey {
    std::string arch;
    int cus;
    int workload;
    int bucket;
    int64_t d;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(arch, cus, workload, bucket, d) <
               std::tie(o.arch, o.cus, o.workload, o.bucket, o.d);
    }
};

static std::mutex g_tune_mu;
static std::map<TuneKey, tri_tune_choice> g_tune;

static int size_bucket(int64_t n)
{
    int b = 0;
    while ((int64_t)1 << (b + 1) <= n) ++b;
    return b;
}

static tri_status device_key(int workload, int64_t n, int64_t d, TuneKey &k)
{
    int dev = 0;
    TRI_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    TRI_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    // d is the dimension of the distance maps and the generations per timed
    // call of Life; it does not enter the elementwise keys
    k = TuneKey{arch, prop.multiProcessorCount, workload, size_bucket(n),
                workload == TRI_TUNE_ELEMENTWISE_F32 || workload == TRI_TUNE_ELEMENTWISE_I32 ? 0
                                                                                           : d};
    return TRI_OK;
}

// scratch buffers owned by one tuning call
struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
    void *get(size_t bytes, hipError_t &e)
    {
        void *p = nullptr;
        e = hipMalloc(&p, bytes ? bytes : 1);
        if (e == hipSuccess) ptrs.push_back(p);
        return p;
    }
};

struct Candidate {
    int tile, map;
    uint32_t flags;
};

// Distance-map candidates are timed on coordinates uniform in [0, 1) (an
// integer hash of the index, top 24 bits), not on zeros: with every point
// equal, every pair falls below the near-duplicate threshold and the
// timing would be that of the FP32 recompute.
__global__ void __launch_bounds__(256) k_tune_fill(float *x, int64_t count)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    uint32_t h = (uint32_t)q * 0x9E3779B9u + (uint32_t)(q >> 32);
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    x[q] = (float)(h >> 8) * (1.0f / 16777216.0f);
}

static std::vector<Candidate> candidates(int workload, int64_t n)
{
    std::vector<int> tiles;
    std::vector<int> maps = {TRI_MAP_BB, TRI_MAP_RB, TRI_MAP_REC, TRI_MAP_LAMBDA};
    bool utm = false;
    switch (workload) {
    case TRI_TUNE_ELEMENTWISE_F32: tiles = {8, 16, 32, 64, 128}; utm = true; break;
    case TRI_TUNE_ELEMENTWISE_I32: tiles = {8, 16, 32, 64}; utm = true; break;
    case TRI_TUNE_LIFE: tiles = {8, 16, 32, 64}; utm = true; break;
    case TRI_TUNE_EDM_FP32: tiles = {16, 32, 64, 128}; break;
    case TRI_TUNE_EDM_BF16X3: tiles = {128}; break;
    }
    std::vector<Candidate> c;
    for (int t : tiles)
        for (int m : maps) {
            c.push_back({t, m, 0u});
            if (m == TRI_MAP_LAMBDA) {
                c.push_back({t, m, (uint32_t)TRI_FLAG_XCD_SWIZZLE});
                c.push_back({t, m, (uint32_t)TRI_FLAG_ORDER_REVERSE});
                c.push_back({t, m, (uint32_t)TRI_FLAG_ORDER_PAIRS});
                c.push_back({t, m, (uint32_t)(TRI_FLAG_XCD_SWIZZLE | TRI_FLAG_ORDER_PAIRS)});
            }
        }
    if (utm) c.push_back({32, TRI_MAP_UTM, 0u});
    if (workload == TRI_TUNE_ELEMENTWISE_F32)  // strips of 4, 8 and 16 tiles at tiles 16, 32
        for (int t : {16, 32})
            for (uint32_t st : {(uint32_t)TRI_FLAG_STRIP(2), (uint32_t)TRI_FLAG_STRIP(3),
                                (uint32_t)TRI_FLAG_STRIP(4)}) {
                for (int m : maps) c.push_back({t, m, st});
                c.push_back({t, TRI_MAP_LAMBDA, st | (uint32_t)TRI_FLAG_ORDER_PAIRS});
                c.push_back({t, TRI_MAP_LAMBDA, st | (uint32_t)TRI_FLAG_XCD_SWIZZLE});
                c.push_back({t, TRI_MAP_LAMBDA, st | (uint32_t)TRI_FLAG_STRIP_ALIGN});
                c.push_back({t, TRI_MAP_LAMBDA, st | (uint32_t)(TRI_FLAG_STRIP_ALIGN | TRI_FLAG_ORDER_PAIRS)});
                // two-row bands (2 x 2 tile blocks at tile 16)
                c.push_back({t, TRI_MAP_BB, st | (uint32_t)TRI_FLAG_STRIP_BAND});
                c.push_back({t, TRI_MAP_LAMBDA, st | (uint32_t)TRI_FLAG_STRIP_BAND});
                c.push_back({t, TRI_MAP_LAMBDA, st | (uint32_t)(TRI_FLAG_STRIP_BAND | TRI_FLAG_ORDER_PAIRS)});
            }
    if (workload == TRI_TUNE_EDM_BF16X3)  // column-major strips of 8, 16 and 32 tiles, both schedules
        for (uint32_t st : {(uint32_t)TRI_FLAG_STRIP(3), (uint32_t)TRI_FLAG_STRIP(4),
                            (uint32_t)TRI_FLAG_STRIP(5)}) {
            c.push_back({128, TRI_MAP_LAMBDA, (uint32_t)TRI_FLAG_STRIP_COLS | st});
            c.push_back({128, TRI_MAP_LAMBDA, (uint32_t)TRI_FLAG_STRIP_COLS | TRI_FLAG_XCD_SWIZZLE | st});
            c.push_back({128, TRI_MAP_LAMBDA, (uint32_t)TRI_FLAG_STRIP_COLS | TRI_FLAG_EDM_PIPE | st});
        }
    if (workload == TRI_TUNE_LIFE)  // tile 64 in strips of 4 and 8 tiles, both forms
        for (uint32_t st : {(uint32_t)TRI_FLAG_STRIP(2), (uint32_t)TRI_FLAG_STRIP(3)}) {
            for (uint32_t tf : {0u, (uint32_t)TRI_FLAG_LIFE_TEMPORAL}) {
                c.push_back({64, TRI_MAP_BB, st | tf});
                c.push_back({64, TRI_MAP_LAMBDA, st | tf});
                c.push_back({64, TRI_MAP_LAMBDA, st | tf | (uint32_t)TRI_FLAG_STRIP_ALIGN});
                c.push_back({64, TRI_MAP_LAMBDA, st | tf | (uint32_t)TRI_FLAG_XCD_SWIZZLE});
            }
            // neighbouring tiles moved in pairs, both forms
            const uint32_t w = (uint32_t)TRI_FLAG_LIFE_WIDE;
            for (uint32_t tf : {0u, (uint32_t)TRI_FLAG_LIFE_TEMPORAL}) {
                c.push_back({64, TRI_MAP_BB, st | w | tf});
                c.push_back({64, TRI_MAP_LAMBDA, st | w | tf | (uint32_t)(TRI_FLAG_STRIP_ALIGN | TRI_FLAG_XCD_SWIZZLE)});
                c.push_back({64, TRI_MAP_LAMBDA, st | w | tf | (uint32_t)(TRI_FLAG_STRIP_ALIGN | TRI_FLAG_XCD_SWIZZLE |
                                                                       TRI_FLAG_ORDER_PAIRS)});
            }
        }
    if (workload == TRI_TUNE_LIFE)  // temporal blocking (tiles 16..64)
        for (int t : {16, 32, 64}) {
            c.push_back({t, TRI_MAP_BB, (uint32_t)TRI_FLAG_LIFE_TEMPORAL});
            c.push_back({t, TRI_MAP_LAMBDA, (uint32_t)TRI_FLAG_LIFE_TEMPORAL});
            c.push_back({t, TRI_MAP_LAMBDA, (uint32_t)(TRI_FLAG_LIFE_TEMPORAL | TRI_FLAG_XCD_SWIZZLE)});
            c.push_back({t, TRI_MAP_LAMBDA, (uint32_t)(TRI_FLAG_LIFE_TEMPORAL | TRI_FLAG_XCD_SWIZZLE |
                                                       TRI_FLAG_ORDER_PAIRS)});
        }
    (void)n;
    return c;
}

}  // namespace trimap

using namespace trimap;

extern "C" {

// Generations per Life timing when the caller gives none: two launches of
// the deepest temporal kernel (the step count's parity fixes the number of
// launches), so that the dispatch orders are ranked as long runs use them
constexpr int kTuneLifeGens = 32;

// Timed calls per candidate are ranked by their median: one slow call (a
// clock change, another process) does not decide the choice.
static float median_of(std::vector<float> v)
{
    std::sort(v.begin(), v.end());
    const size_t k = v.size();
    return k % 2 ? v[k / 2] : 0.5f * (v[k / 2 - 1] + v[k / 2]);
}

tri_status tri_autotune(int workload, int64_t n, int64_t d, int reps, int use_cache, void *stream,
                        tri_tune_choice *best, tri_tune_choice *all, int32_t all_cap,
                        int32_t *all_count)
{
    clear_error();
    if (!best) return fail(TRI_E_INVAL, "tri_autotune: best is NULL");
    if (workload < TRI_TUNE_ELEMENTWISE_F32 || workload > TRI_TUNE_EDM_BF16X3)
        return fail(TRI_E_INVAL, "tri_autotune: workload = %d", workload);
    if (n < 2 || n >= (1ll << 31)) return fail(TRI_E_RANGE, "tri_autotune: n = %lld", (long long)n);
    const bool edm = workload == TRI_TUNE_EDM_FP32 || workload == TRI_TUNE_EDM_BF16X3;
    if (edm && (d < 1 || d > 4096)) return fail(TRI_E_RANGE, "tri_autotune: d = %lld", (long long)d);
    if (workload == TRI_TUNE_LIFE && (d < 0 || d > 100000))
        return fail(TRI_E_RANGE, "tri_autotune: %lld Life generations", (long long)d);
    const int life_gens = workload == TRI_TUNE_LIFE && d > 0 ? (int)d : kTuneLifeGens;
    if (reps < 1) reps = 1;
    if (all_count) *all_count = 0;

    TuneKey key;
    tri_status st = device_key(workload, n, d, key);
    if (st != TRI_OK) return st;
    if (use_cache) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            *best = it->second;
            return TRI_OK;
        }
    }

    hipStream_t s = (hipStream_t)stream;
    Scratch sc;
    hipError_t e = hipSuccess;
    // buffers sized for the workload; contents zeroed (timing only), the
    // distance maps' coordinates filled as above; Life rows padded to 16
    // bytes (the layout the bit-sliced kernel moves as vectors)
    const int64_t ld = workload == TRI_TUNE_LIFE ? (n + 15) / 16 * 16 : (n + 3) / 4 * 4;
    void *x = nullptr, *y = nullptr, *c = nullptr, *ws = nullptr;
    size_t ws_bytes = 0;
    switch (workload) {
    case TRI_TUNE_ELEMENTWISE_F32:
        x = sc.get(sizeof(float) * n * ld, e);
        if (e == hipSuccess) y = sc.get(sizeof(float) * n * ld, e);
        if (e == hipSuccess) c = sc.get(sizeof(float) * n * ld, e);
        if (e == hipSuccess) e = hipMemsetAsync(x, 0, sizeof(float) * n * ld, s);
        if (e == hipSuccess) e = hipMemsetAsync(y, 0, sizeof(float) * n * ld, s);
        break;
    case TRI_TUNE_ELEMENTWISE_I32:
        x = sc.get(sizeof(uint32_t) * n, e);
        if (e == hipSuccess) y = sc.get(sizeof(uint32_t) * n, e);
        if (e == hipSuccess) c = sc.get(sizeof(int32_t) * n * ld, e);
        if (e == hipSuccess) e = hipMemsetAsync(x, 0, sizeof(uint32_t) * n, s);
        if (e == hipSuccess) e = hipMemsetAsync(y, 0, sizeof(uint32_t) * n, s);
        break;
    case TRI_TUNE_LIFE:
        x = sc.get((size_t)n * ld, e);
        if (e == hipSuccess) y = sc.get((size_t)n * ld, e);
        if (e == hipSuccess) e = hipMemsetAsync(x, 0, (size_t)n * ld, s);
        if (e == hipSuccess) e = hipMemsetAsync(y, 0, (size_t)n * ld, s);
        break;
    default: {
        x = sc.get(sizeof(float) * n * d, e);
        if (e == hipSuccess) c = sc.get(sizeof(float) * (size_t)(n * (n - 1) / 2), e);
        if (e == hipSuccess) {
            const int64_t cnt = n * d;
            k_tune_fill<<<dim3((uint32_t)((cnt + 255) / 256)), 256, 0, s>>>((float *)x, cnt);
            e = hipGetLastError();
        }
        if (e == hipSuccess && workload == TRI_TUNE_EDM_BF16X3) {
            tri_plan *p = nullptr;
            if (tri_map_plan(&p, n, 128, TRI_MAP_LAMBDA, 0, 0) == TRI_OK) {
                tri_edm_workspace_size(p, d, TRI_EDM_BF16X3, &ws_bytes);
                tri_plan_destroy(p);
            }
            ws = sc.get(ws_bytes, e);
        }
        break;
    }
    }
    if (e != hipSuccess) return hip_fail(e, "tri_autotune: scratch");

    // one event per timed call boundary: call r is timed from ev[r] to ev[r + 1]
    std::vector<hipEvent_t> ev(reps + 1, nullptr);
    for (auto &x_ev : ev)
        if ((e = hipEventCreate(&x_ev)) != hipSuccess) break;
    auto destroy_events = [&]() {
        for (auto &x_ev : ev)
            if (x_ev) (void)hipEventDestroy(x_ev);
    };
    if (e != hipSuccess) {
        destroy_events();
        return hip_fail(e, "tri_autotune: event");
    }
    tri_tune_choice bestc{0, -1, 0u, 0.f};
    int32_t nall = 0;
    st = TRI_OK;
    for (const Candidate &cd : candidates(workload, n)) {
        tri_plan *p = nullptr;
        if (tri_map_plan(&p, n, cd.tile, cd.map, edm ? 0 : 1, cd.flags) != TRI_OK) continue;
        auto run = [&]() -> tri_status {
            switch (workload) {
            case TRI_TUNE_ELEMENTWISE_F32:
                return tri_launch_elementwise(p, TRI_OP_AXPYT_F32, x, y, c, ld, 1.25f, s);
            case TRI_TUNE_ELEMENTWISE_I32:
                return tri_launch_elementwise(p, TRI_OP_XORMUL_I32, x, y, c, ld, 0.f, s);
            case TRI_TUNE_LIFE:
                return tri_launch_stencil(p, (uint8_t *)x, (uint8_t *)y, ld, life_gens, 0, s);
            case TRI_TUNE_EDM_FP32:
                return tri_edm(p, (const float *)x, d, d, (float *)c, TRI_EDM_FP32, 1e-2f, nullptr, 0, s);
            default:
                return tri_edm(p, (const float *)x, d, d, (float *)c, TRI_EDM_BF16X3, 1e-2f, ws,
                               ws_bytes, s);
            }
        };
        tri_status rs = run();  // warm-up; also rejects unsupported combinations
        if (rs != TRI_OK) {
            tri_plan_destroy(p);
            if (rs == TRI_E_HIP) { st = rs; break; }
            continue;
        }
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < reps && rs == TRI_OK; ++r) {
            rs = run();
            (void)hipEventRecord(ev[r + 1], s);
        }
        e = hipEventSynchronize(ev[reps]);
        tri_plan_destroy(p);
        if (rs != TRI_OK || e != hipSuccess) {
            st = rs != TRI_OK ? rs : hip_fail(e, "tri_autotune: timing");
            break;
        }
        std::vector<float> t(reps, 0.f);
        for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[r], ev[r], ev[r + 1]);
        float ms = median_of(t);
        if (workload == TRI_TUNE_LIFE) ms /= (float)life_gens;  // per generation
        const tri_tune_choice ch{cd.tile, cd.map, cd.flags, ms};
        if (all && nall < all_cap) all[nall] = ch;
        ++nall;
        if (bestc.map < 0 || ms < bestc.ms) bestc = ch;
    }
    destroy_events();
    if (st != TRI_OK) return st;
    if (bestc.map < 0) return fail(TRI_E_UNSUPPORTED, "tri_autotune: no candidate ran");
    if (all_count) *all_count = std::min(nall, all_cap);
    *best = bestc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = bestc;
    return TRI_OK;
}

tri_status tri_tune_cache_save(const char *path)
{
    clear_error();
    if (!path) return fail(TRI_E_INVAL, "tri_tune_cache_save: path is NULL");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = fopen(path, "w");
    if (!f) return fail(TRI_E_INVAL, "tri_tune_cache_save: cannot open %s", path);
    fprintf(f, "{\n  \"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : g_tune) {
        const TuneKey &k = kv.first;
        const tri_tune_choice &c = kv.second;
        fprintf(f,
                "    {\"arch\": \"%s\", \"cus\": %d, \"workload\": %d, \"bucket\": %d, \"d\": %lld, "
                "\"tile\": %d, \"map\": %d, \"flags\": %u, \"ms\": %.6g}%s\n",
                k.arch.c_str(), k.cus, k.workload, k.bucket, (long long)k.d, c.tile, c.map, c.flags,
                (double)c.ms, ++i < g_tune.size() ? "," : "");
    }
    fprintf(f, "  ]\n}\n");
    fclose(f);
    return TRI_OK;
}

// Reads the format written by tri_tune_cache_save: one entry object per line.
tri_status tri_tune_cache_load(const char *path)
{
    clear_error();
    if (!path) return fail(TRI_E_INVAL, "tri_tune_cache_load: path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(TRI_E_INVAL, "tri_tune_cache_load: cannot open %s", path);
    char line[1024], arch[128];
    int loaded = 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    while (fgets(line, sizeof line, f)) {
        int cus, workload, bucket, tile, map;
        long long d;
        unsigned flags;
        double ms;
        if (sscanf(line,
                   " {\"arch\": \"%127[^\"]\", \"cus\": %d, \"workload\": %d, \"bucket\": %d, "
                   "\"d\": %lld, \"tile\": %d, \"map\": %d, \"flags\": %u, \"ms\": %lf",
                   arch, &cus, &workload, &bucket, &d, &tile, &map, &flags, &ms) == 9) {
            g_tune[TuneKey{arch, cus, workload, bucket, (int64_t)d}] =
                tri_tune_choice{tile, map, flags, (float)ms};
            ++loaded;
        }
    }
    fclose(f);
    return TRI_OK;
}

tri_status tri_tune_cache_clear(void)
{
    clear_error();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return TRI_OK;
}

}  // extern "C"
