// The dummy kernel of the square-root study (Section 5.1): every cell (i, j)
// of the plan's domain forms its coordinates through the map and computes
// i + j; only cells whose sum equals a target store it.  With a target no
// cell reaches, nothing is written and the kernel costs the dispatch, the
// map and the per-cell test alone, which is what the paper's improvement
// factors compare (its version stores every sum to one fixed address; on
// this hardware those stores would serialise on one L2 channel and hide the
// map's cost).
#include "common.hpp"
#include "maps.hpp"

namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

struct DummyArgs {
    TileGrid g;
    int32_t n;
    int32_t row_off;  // 1 for the strict triangle
    int32_t target;
    int32_t *sink;
};

template <int TILE>
struct DummyShape {
    static constexpr int NT = TILE * TILE < 256 ? TILE * TILE : 256;
    static constexpr int PASSES = TILE * TILE / NT;
};

template <int MAP, int TILE>
__global__ void __launch_bounds__((DummyShape<TILE>::NT)) k_dummy(DummyArgs p)
{
    using S = DummyShape<TILE>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
#pragma unroll
    for (int ps = 0; ps < S::PASSES; ++ps) {
        const int t = threadIdx.x + ps * S::NT;
        const int32_t i = p.row_off + bi * TILE + t / TILE;
        const int32_t j = bj * TILE + t % TILE;
        if (i < p.n && j < i + 1 - p.row_off && (int64_t)i + j == p.target) p.sink[0] = i + j;
    }
}

__global__ void __launch_bounds__(kUtmThreads) k_dummy_utm(DummyArgs p, int64_t side,
                                                           int64_t cells)
{
    const uint64_t k = ((uint64_t)blockIdx.y * gridDim.x + blockIdx.x) * kUtmThreads + threadIdx.x;
    if (k >= (uint64_t)cells) return;
    int32_t i, j;
    utm_cell(k, side, i, j);
    i += p.row_off;
    if (i < p.n && j < i + 1 - p.row_off && (int64_t)i + j == p.target) p.sink[0] = i + j;
}

template <int MAP>
static bool dummy_tile(const tri_plan *p, const DummyArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 8: k_dummy<MAP, 8><<<grid, DummyShape<8>::NT, 0, s>>>(a); return true;
    case 16: k_dummy<MAP, 16><<<grid, DummyShape<16>::NT, 0, s>>>(a); return true;
    case 32: k_dummy<MAP, 32><<<grid, DummyShape<32>::NT, 0, s>>>(a); return true;
    case 64: k_dummy<MAP, 64><<<grid, DummyShape<64>::NT, 0, s>>>(a); return true;
    }
    return false;
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_launch_dummy(const tri_plan *p, int32_t target, int32_t *sink,
                                       void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_launch_dummy: plan is NULL");
    if (p->tile > 64) return fail(TRI_E_UNSUPPORTED, "tri_launch_dummy: tile %d > 64", p->tile);
    if (!sink || ((uintptr_t)sink & 3)) return fail(TRI_E_INVAL, "tri_launch_dummy: sink");
    if (p->elements == 0) return TRI_OK;
    DummyArgs a{plan_tile_grid(p), (int32_t)p->n, p->row_off, target, sink};
    hipStream_t s = (hipStream_t)stream;
    bool ok = true;
    switch (p->map) {
    case TRI_MAP_BB: ok = dummy_tile<MAP_BB>(p, a, s); break;
    case TRI_MAP_RB: ok = dummy_tile<MAP_RB>(p, a, s); break;
    case TRI_MAP_REC: ok = dummy_tile<MAP_REC>(p, a, s); break;
    case TRI_MAP_LAMBDA: ok = dummy_tile<MAP_LAMBDA>(p, a, s); break;
    case TRI_MAP_UTM:
        k_dummy_utm<<<dim3(p->gx, p->gy), kUtmThreads, 0, s>>>(a, p->ne, p->elements);
        break;
    }
    if (!ok) return fail(TRI_E_UNSUPPORTED, "tri_launch_dummy: tile %d", p->tile);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
