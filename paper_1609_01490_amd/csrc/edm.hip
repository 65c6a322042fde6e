// Euclidean distance map over the strict lower triangle (the EDM test of
// Section 5; distance d(i, j) = sqrt(sum_k (x_ik - x_jk)^2)), written to the
// condensed array out[i (i - 1) / 2 + j], which is the numbering of the map
// without diagonal (Eq. eq_theorem_nodiag).
//
// Tile (bi, bj) of the plan covers rows 1 + bi rho .. and columns bj rho ..
// (the strict triangle of side n is the diagonal-including triangle of side
// n - 1 shifted down one row).
//
// TRI_EDM_FP32: direct sum of squared differences, FP32 FMA, both point
// blocks staged in LDS dimension-major so that a lane's 4x4 register block
// reads broadcast / consecutive words.  Bound by the vector ALU (2 VALU ops
// per pair and dimension).
#include "common.hpp"
#include "maps.hpp"

namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

struct EdmArgs {
    TileGrid g;
    int32_t n;
    int32_t d;
    int64_t ldx;
    const float *x;
    float *out;
};

template <int TILE>
struct EdmF32Shape {
    static constexpr int NT = 256;
    static constexpr int TX = 16;                 // lanes along columns
    static constexpr int TY = NT / TX;            // lanes along rows
    static constexpr int RB = TILE / TY;          // register rows per lane
    static constexpr int CB = TILE / TX;          // register columns per lane
    static constexpr int K = TILE >= 64 ? 32 : 64; // dimensions staged per step
    static_assert(RB >= 1 && CB >= 1 && RB * TY == TILE && CB * TX == TILE, "edm tile");
};

template <int MAP, int TILE>
__global__ void __launch_bounds__(256) k_edm_f32(EdmArgs p)
{
    using S = EdmF32Shape<TILE>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;

    __shared__ float XI[S::K][TILE + 1];
    __shared__ float XJ[S::K][TILE + 1];
    const int32_t n = p.n, d = p.d;
    const int64_t ldx = p.ldx;
    const int32_t ri0 = 1 + bi * TILE;  // first row of the tile
    const int32_t cj0 = bj * TILE;      // first column of the tile
    const int tx = threadIdx.x % S::TX, ty = threadIdx.x / S::TX;

    float acc[S::RB][S::CB];
#pragma unroll
    for (int a = 0; a < S::RB; ++a)
#pragma unroll
        for (int c = 0; c < S::CB; ++c) acc[a][c] = 0.f;

    for (int32_t k0 = 0; k0 < d; k0 += S::K) {
        for (int idx = threadIdx.x; idx < TILE * S::K; idx += S::NT) {
            const int row = idx / S::K, kk = idx % S::K;
            const int32_t k = k0 + kk;
            const int32_t gi = ri0 + row, gj = cj0 + row;
            XI[kk][row] = (gi < n && k < d) ? p.x[(int64_t)gi * ldx + k] : 0.f;
            XJ[kk][row] = (gj < n && k < d) ? p.x[(int64_t)gj * ldx + k] : 0.f;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < S::K; ++kk) {
            float xa[S::RB], xb[S::CB];
#pragma unroll
            for (int a = 0; a < S::RB; ++a) xa[a] = XI[kk][ty + S::TY * a];
#pragma unroll
            for (int c = 0; c < S::CB; ++c) xb[c] = XJ[kk][tx + S::TX * c];
#pragma unroll
            for (int a = 0; a < S::RB; ++a)
#pragma unroll
                for (int c = 0; c < S::CB; ++c) {
                    const float df = xa[a] - xb[c];
                    acc[a][c] = __builtin_fmaf(df, df, acc[a][c]);
                }
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < S::RB; ++a) {
        const int32_t i = ri0 + ty + S::TY * a;
        if (i >= n) continue;
        float *orow = p.out + (int64_t)i * (i - 1) / 2;
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            const int32_t j = cj0 + tx + S::TX * c;
            if (j < i) __builtin_nontemporal_store(__builtin_sqrtf(acc[a][c]), orow + j);
        }
    }
}

template <int MAP>
static bool edm_f32_tile(const tri_plan *p, const EdmArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 16: k_edm_f32<MAP, 16><<<grid, 256, 0, s>>>(a); return true;
    case 32: k_edm_f32<MAP, 32><<<grid, 256, 0, s>>>(a); return true;
    case 64: k_edm_f32<MAP, 64><<<grid, 256, 0, s>>>(a); return true;
    }
    return false;
}

static bool edm_f32(const tri_plan *p, const EdmArgs &a, hipStream_t s)
{
    switch (p->map) {
    case TRI_MAP_BB: return edm_f32_tile<MAP_BB>(p, a, s);
    case TRI_MAP_RB: return edm_f32_tile<MAP_RB>(p, a, s);
    case TRI_MAP_REC: return edm_f32_tile<MAP_REC>(p, a, s);
    case TRI_MAP_LAMBDA: return edm_f32_tile<MAP_LAMBDA>(p, a, s);
    }
    return false;
}

static tri_status edm_check(const tri_plan *p, int64_t d, int mode)
{
    if (!p) return fail(TRI_E_INVAL, "tri_edm: plan is NULL");
    if (p->diag) return fail(TRI_E_INVAL, "tri_edm: the plan must exclude the diagonal");
    if (p->map == TRI_MAP_UTM) return fail(TRI_E_UNSUPPORTED, "tri_edm: UTM is not supported");
    if (d < 1 || d > 4096) return fail(TRI_E_RANGE, "tri_edm: d = %lld not in [1, 4096]", (long long)d);
    if (mode == TRI_EDM_FP32) {
        if (p->tile != 16 && p->tile != 32 && p->tile != 64)
            return fail(TRI_E_UNSUPPORTED, "tri_edm: FP32 mode needs tile 16, 32 or 64");
        return TRI_OK;
    }
    if (mode == TRI_EDM_BF16X3 || mode == TRI_EDM_BF16)
        return fail(TRI_E_UNSUPPORTED, "tri_edm: MFMA modes not built yet");
    return fail(TRI_E_INVAL, "tri_edm: mode = %d", mode);
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_edm_workspace_size(const tri_plan *p, int64_t d, int mode, size_t *bytes)
{
    clear_error();
    if (!bytes) return fail(TRI_E_INVAL, "tri_edm_workspace_size: bytes is NULL");
    *bytes = 0;
    tri_status st = edm_check(p, d, mode);
    if (st != TRI_OK) return st;
    return TRI_OK;
}

extern "C" tri_status tri_edm(const tri_plan *p, const float *x, int64_t d, int64_t ldx,
                              float *out, int mode, float fixup_thr, void *ws, size_t ws_bytes,
                              void *stream)
{
    clear_error();
    tri_status st = edm_check(p, d, mode);
    if (st != TRI_OK) return st;
    (void)fixup_thr;
    (void)ws;
    (void)ws_bytes;
    if (p->n < 2) return TRI_OK;
    if (!x || !out) return fail(TRI_E_INVAL, "tri_edm: NULL buffer");
    if (ldx < d) return fail(TRI_E_INVAL, "tri_edm: ldx < d");
    if (((uintptr_t)x | (uintptr_t)out) & 3) return fail(TRI_E_INVAL, "tri_edm: unaligned buffer");
    EdmArgs a{plan_tile_grid(p), (int32_t)p->n, (int32_t)d, ldx, x, out};
    hipStream_t s = (hipStream_t)stream;
    if (!edm_f32(p, a, s)) return fail(TRI_E_UNSUPPORTED, "tri_edm: tile");
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
