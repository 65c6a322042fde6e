// Plans (tile space and launch grid of a map), error reporting, and the map
// test hooks.  Tile space and block count: Section 3.1 (m = ceil(n / rho),
// m (m + 1) / 2 blocks for lambda, m x m for the bounding box); other grids:
// Section 4.2.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "common.hpp"
#include "maps.hpp"

namespace trimap {

static thread_local char g_err[512];

void clear_error() { g_err[0] = 0; }

tri_status fail(tri_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

tri_status hip_fail(hipError_t e, const char *what)
{
    return fail(TRI_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Largest grid x extent in blocks: keeps blocks x threads (<= 256) under the
// 2^32 work-item limit of one grid dimension.
static constexpr uint64_t kMaxGridX = 1ull << 24;

static bool grid_1d(uint64_t blocks, uint32_t &gx, uint32_t &gy)
{
    if (blocks <= kMaxGridX) {
        gx = (uint32_t)(blocks ? blocks : 1);
        gy = 1;
        return true;
    }
    const uint64_t x = 1ull << 16;
    const uint64_t y = (blocks + x - 1) / x;
    if (y > kMaxGridY) return false;
    gx = (uint32_t)x;
    gy = (uint32_t)y;
    return true;
}

static TileGrid tile_grid(const tri_plan *p)
{
    uint32_t f = p->flags;
    if (p->map == TRI_MAP_LAMBDA && p->gy == 1 && (uint64_t)p->gx == (uint64_t)p->T &&
        p->T <= (1ll << 24) &&
        (f & ~(uint32_t)(TRI_FLAG_XCD_SWIZZLE | TRI_FLAG_STRIP_MASK | TRI_FLAG_STRIP_COLS | TRI_FLAG_STRIP_ALIGN |
                        TRI_FLAG_STRIP_BAND | TRI_FLAG_EDM_PIPE)) == 0)
        f |= kLambda24;
    else if (p->map == TRI_MAP_LAMBDA && p->gy > 1 && p->gx == (1u << 16) &&
             (f & ~(uint32_t)(TRI_FLAG_STRIP_MASK | TRI_FLAG_STRIP_COLS | TRI_FLAG_STRIP_ALIGN |
                             TRI_FLAG_STRIP_BAND | TRI_FLAG_EDM_PIPE)) == 0 && p->T < (1ll << 32))
        f |= kLambda32;
    return TileGrid{(int32_t)p->m, f, (uint64_t)p->T};
}

// ---------------------------------------------------------------------------
// map dump / lambda evaluation kernels
// ---------------------------------------------------------------------------
template <int MAP>
__global__ void __launch_bounds__(64) k_map_dump(TileGrid g, int64_t *out)
{
    if (threadIdx.x != 0) return;
    const uint64_t b = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
    int32_t bi, bj;
    if (tile_of_block_raw<MAP>(g, bi, bj)) {
        out[2 * b] = bi;
        out[2 * b + 1] = bj;
    } else {
        out[2 * b] = -1;
        out[2 * b + 1] = -1;
    }
}

__global__ void __launch_bounds__(kUtmThreads) k_utm_dump(int64_t side, int64_t elements,
                                                          int32_t row_off, int64_t *out)
{
    const uint64_t k = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * kUtmThreads + threadIdx.x;
    if (k >= (uint64_t)elements) return;
    int32_t i, j;
    utm_cell(k, side, i, j);
    out[2 * k] = i + row_off;
    out[2 * k + 1] = j;
}

__global__ void __launch_bounds__(256) k_lambda_eval(const uint64_t *omega, int64_t count,
                                                     int32_t row_off, uint32_t flags,
                                                     int64_t *out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= count) return;
    const uint64_t w = omega[t];
    const uint32_t i = lambda_row(w, flags);
    out[2 * t] = (int64_t)i + row_off;
    out[2 * t + 1] = (int64_t)(w - (uint64_t)i * (i + 1) / 2);
}

}  // namespace trimap

using namespace trimap;

extern "C" {

const char *tri_status_str(tri_status st)
{
    switch (st) {
    case TRI_OK: return "TRI_OK";
    case TRI_E_INVAL: return "TRI_E_INVAL";
    case TRI_E_RANGE: return "TRI_E_RANGE";
    case TRI_E_NOMEM: return "TRI_E_NOMEM";
    case TRI_E_HIP: return "TRI_E_HIP";
    case TRI_E_UNSUPPORTED: return "TRI_E_UNSUPPORTED";
    }
    return "TRI_E_?";
}

const char *tri_last_error(void) { return g_err; }

tri_status tri_map_plan(tri_plan **out, int64_t n, int tile, int map, int include_diag,
                        uint32_t flags)
{
    clear_error();
    if (!out) return fail(TRI_E_INVAL, "tri_map_plan: out is NULL");
    *out = nullptr;
    if (n < 0) return fail(TRI_E_INVAL, "tri_map_plan: n = %lld < 0", (long long)n);
    if (n >= (1ll << 31)) return fail(TRI_E_RANGE, "tri_map_plan: n = %lld >= 2^31", (long long)n);
    if (tile != 8 && tile != 16 && tile != 32 && tile != 64 && tile != 128)
        return fail(TRI_E_INVAL, "tri_map_plan: tile = %d not in {8,16,32,64,128}", tile);
    if (map < TRI_MAP_BB || map > TRI_MAP_LAMBDA)
        return fail(TRI_E_INVAL, "tri_map_plan: map = %d", map);
    if (include_diag != 0 && include_diag != 1)
        return fail(TRI_E_INVAL, "tri_map_plan: include_diag = %d", include_diag);
    if (flags & ~(uint32_t)(TRI_FLAG_XCD_SWIZZLE | TRI_FLAG_SQRT_RSQ | TRI_FLAG_SQRT_F64 |
                            TRI_FLAG_ORDER_REVERSE | TRI_FLAG_ORDER_PAIRS |
                            TRI_FLAG_LIFE_TEMPORAL | TRI_FLAG_SQRT_NEWTON |
                            TRI_FLAG_SQRT_EPS | TRI_FLAG_STRIP_MASK | TRI_FLAG_STRIP_COLS |
                            TRI_FLAG_STRIP_ALIGN | TRI_FLAG_EDM_PIPE | TRI_FLAG_STRIP_BAND |
                            TRI_FLAG_LIFE_WIDE))
        return fail(TRI_E_INVAL, "tri_map_plan: unknown flags 0x%x", flags);
    if (((flags & TRI_FLAG_STRIP_MASK) >> 8) > 6)
        return fail(TRI_E_INVAL, "tri_map_plan: strip length beyond 32 tiles (flags 0x%x)", flags);

    tri_plan p{};
    p.n = n;
    p.diag = include_diag;
    p.row_off = include_diag ? 0 : 1;
    p.ne = include_diag ? n : (n > 0 ? n - 1 : 0);
    p.tile = tile;
    p.map = map;
    p.flags = flags;
    p.m = (p.ne + tile - 1) / tile;
    p.T = p.m * (p.m + 1) / 2;
    p.elements = include_diag ? n * (n + 1) / 2 : n * (n - 1) / 2;

    const int64_t m = p.m;
    uint64_t gx = 0, gy = 0;
    switch (map) {
    case TRI_MAP_BB:
        gx = m;
        gy = m;
        break;
    case TRI_MAP_RB:
        if (m % 2) { gx = m; gy = (m + 1) / 2; }
        else { gx = m + 1; gy = m / 2; }
        break;
    case TRI_MAP_REC:
        if (m & (m - 1))
            return fail(TRI_E_UNSUPPORTED,
                        "tri_map_plan: REC needs a power-of-two tile count, m = %lld",
                        (long long)m);
        if (m == 1) { gx = 1; gy = 1; }
        else if (m > 1) { gx = m / 2; gy = m + 1; }
        break;
    case TRI_MAP_LAMBDA: {
        uint32_t x, y;
        if (!grid_1d((uint64_t)p.T, x, y))
            return fail(TRI_E_RANGE, "tri_map_plan: %lld tiles exceed the grid", (long long)p.T);
        gx = p.T ? x : 0;
        gy = p.T ? y : 0;
        break;
    }
    case TRI_MAP_UTM: {
        const uint64_t blocks = ((uint64_t)p.elements + kUtmThreads - 1) / kUtmThreads;
        uint32_t x, y;
        if (!grid_1d(blocks, x, y))
            return fail(TRI_E_RANGE, "tri_map_plan: %lld cells exceed the grid",
                        (long long)p.elements);
        gx = blocks ? x : 0;
        gy = blocks ? y : 0;
        break;
    }
    }
    if (gx > kMaxGridX || gy > kMaxGridY)
        return fail(TRI_E_RANGE, "tri_map_plan: grid %llu x %llu too large",
                    (unsigned long long)gx, (unsigned long long)gy);
    p.gx = (uint32_t)gx;
    p.gy = (uint32_t)gy;
    p.blocks = (int64_t)(gx * gy);

    p.graphs = new (std::nothrow) PlanGraphs();
    if (!p.graphs) return fail(TRI_E_NOMEM, "tri_map_plan: out of host memory");
    tri_plan *h = new (std::nothrow) tri_plan(p);
    if (!h) {
        delete p.graphs;
        return fail(TRI_E_NOMEM, "tri_map_plan: out of host memory");
    }
    *out = h;
    return TRI_OK;
}

tri_status tri_plan_destroy(tri_plan *plan)
{
    clear_error();
    if (!plan) return TRI_OK;
    if (plan->graphs) {
        for (auto &kv : plan->graphs->execs) (void)hipGraphExecDestroy(kv.second);
        delete plan->graphs;
    }
    delete plan;
    return TRI_OK;
}

tri_status tri_plan_query(const tri_plan *p, tri_plan_info *info)
{
    clear_error();
    if (!p || !info) return fail(TRI_E_INVAL, "tri_plan_query: NULL argument");
    std::memset(info, 0, sizeof *info);
    info->n = p->n;
    info->tile = p->tile;
    info->m = p->m;
    info->tiles = p->T;
    info->grid_x = p->gx;
    info->grid_y = p->gy;
    info->grid_blocks = p->blocks;
    info->elements = p->elements;
    info->map = p->map;
    info->include_diag = p->diag;
    info->flags = p->flags;
    if (p->map == TRI_MAP_UTM) {
        info->wasted_blocks = 0;
        info->dump_entries = p->elements;
    } else {
        info->wasted_blocks = p->blocks - p->T;
        info->dump_entries = p->blocks;
    }
    return TRI_OK;
}

tri_status tri_map_dump(const tri_plan *p, int64_t *dev_out, void *stream)
{
    clear_error();
    if (!p || !dev_out) return fail(TRI_E_INVAL, "tri_map_dump: NULL argument");
    if (p->blocks == 0) return TRI_OK;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid(p->gx, p->gy);
    const TileGrid g = tile_grid(p);
    switch (p->map) {
    case TRI_MAP_BB: k_map_dump<MAP_BB><<<grid, 64, 0, s>>>(g, dev_out); break;
    case TRI_MAP_RB: k_map_dump<MAP_RB><<<grid, 64, 0, s>>>(g, dev_out); break;
    case TRI_MAP_REC: k_map_dump<MAP_REC><<<grid, 64, 0, s>>>(g, dev_out); break;
    case TRI_MAP_LAMBDA: k_map_dump<MAP_LAMBDA><<<grid, 64, 0, s>>>(g, dev_out); break;
    case TRI_MAP_UTM:
        k_utm_dump<<<grid, kUtmThreads, 0, s>>>(p->ne, p->elements, p->row_off, dev_out);
        break;
    }
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

tri_status tri_lambda_eval(const uint64_t *dev_omega, int64_t count, int include_diag,
                           uint32_t flags, int64_t *dev_out, void *stream)
{
    clear_error();
    if (count < 0 || (count > 0 && (!dev_omega || !dev_out)))
        return fail(TRI_E_INVAL, "tri_lambda_eval: bad arguments");
    if (flags & ~(uint32_t)(TRI_FLAG_SQRT_RSQ | TRI_FLAG_SQRT_F64 | TRI_FLAG_SQRT_NEWTON |
                            TRI_FLAG_SQRT_EPS))
        return fail(TRI_E_INVAL, "tri_lambda_eval: unknown flags 0x%x", flags);
    if (count == 0) return TRI_OK;
    const int64_t blocks = (count + 255) / 256;
    if ((uint64_t)blocks > kMaxGridX) return fail(TRI_E_RANGE, "tri_lambda_eval: count too large");
    k_lambda_eval<<<dim3((uint32_t)blocks), 256, 0, (hipStream_t)stream>>>(
        dev_omega, count, include_diag ? 0 : 1, flags, dev_out);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

}  // extern "C"

namespace trimap {
TileGrid plan_tile_grid(const tri_plan *p) { return tile_grid(p); }
}  // namespace trimap
