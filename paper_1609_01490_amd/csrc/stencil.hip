// Game of Life (B3/S23) on the lower-triangular domain: the shared-memory
// neighbourhood case of the paper (Section 5, where lambda keeps the 2-D
// thread block and therefore the tile with its halo).
//
// One workgroup per rho x rho tile.  The tile plus a one-cell halo is staged
// in LDS as 32-bit words of four cells ((rho + 2) rows x (rho/4 + 2) words:
// the halo columns come in as whole words).  Each thread then updates a
// vertical strip of words with byte-sliced (SWAR) arithmetic: four cells per
// 32-bit operation, neighbour sums never exceed 9 so no byte carries.
// Cells outside the domain (j > i, outside the n x n square) are zeroed as
// they are loaded and never stored, so the upper triangle is never touched.
#include "common.hpp"
#include "maps.hpp"

namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

struct LifeArgs {
    TileGrid g;
    int32_t n;
    int64_t ld;
    const uint8_t *cur;
    uint8_t *nxt;
};

template <int TILE>
struct LifeShape {
    static constexpr int WPR = TILE / 4;                                  // words per row
    static constexpr int NT = TILE == 8 ? 16 : (TILE == 64 ? 256 : 64);   // threads
    static constexpr int STRIPS = NT / WPR;                               // strips per column
    static constexpr int SH = TILE / STRIPS;                              // rows per strip
    static constexpr int LW = WPR + 2;                                    // LDS words per row
    static constexpr int LR = TILE + 2;                                   // LDS rows
    static_assert(SH * STRIPS == TILE && SH >= 1, "life tile shape");
};

// bytes of the word at column j (4-aligned) of row i that lie in the domain
// (j + b <= i); 0 when none does
__device__ __forceinline__ uint32_t domain_mask(int32_t i, int32_t j)
{
    const int32_t k = i - j;  // number of in-domain bytes minus one
    if (k >= 3) return 0xFFFFFFFFu;
    if (k < 0) return 0u;
    return 0xFFFFFFFFu >> (8 * (3 - k));
}

// one byte (0x01) per zero byte of t, for bytes below 0x80
__device__ __forceinline__ uint32_t zero_bytes(uint32_t t)
{
    const uint32_t nz = (t + 0x7F7F7F7Fu) | t;
    return (~nz & 0x80808080u) >> 7;
}

// horizontal 3-sums of a word given its west and east neighbour words
__device__ __forceinline__ uint32_t hsum3(uint32_t west, uint32_t w, uint32_t east)
{
    const uint32_t wl = __builtin_amdgcn_alignbit(w, west, 24);  // (w << 8) | (west >> 24)
    const uint32_t wr = __builtin_amdgcn_alignbit(east, w, 8);   // (w >> 8) | (east << 24)
    return w + wl + wr;
}

template <int MAP, int TILE>
__global__ void __launch_bounds__(LifeShape<TILE>::NT) k_life(LifeArgs p)
{
    using S = LifeShape<TILE>;
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;

    __shared__ uint32_t L[S::LR][S::LW];
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t i0 = bi * TILE, j0 = bj * TILE;
    const bool interior = (bi != bj) && bj > 0 && (i0 + TILE < n) && (j0 + TILE + 3 < i0);

    // stage rows i0-1 .. i0+TILE, words at columns j0-4 .. j0+TILE
    for (int idx = threadIdx.x; idx < S::LR * S::LW; idx += S::NT) {
        const int lr = idx / S::LW, lw = idx % S::LW;
        const int32_t gi = i0 - 1 + lr;
        const int32_t gj = j0 - 4 + 4 * lw;
        uint32_t v = 0;
        if (interior) {
            v = *(const uint32_t *)(p.cur + (int64_t)gi * ld + gj);
        } else if (gi >= 0 && gi < n && gj >= 0 && gj <= gi) {
            v = *(const uint32_t *)(p.cur + (int64_t)gi * ld + gj) & domain_mask(gi, gj);
        }
        L[lr][lw] = v;
    }
    __syncthreads();

    const int wc = threadIdx.x % S::WPR;  // word column inside the tile
    const int st = threadIdx.x / S::WPR;  // strip
    const int lw = wc + 1;
    const int r0 = st * S::SH + 1;        // first LDS row of the strip

    uint32_t hprev = hsum3(L[r0 - 1][lw - 1], L[r0 - 1][lw], L[r0 - 1][lw + 1]);
    uint32_t hcur = hsum3(L[r0][lw - 1], L[r0][lw], L[r0][lw + 1]);
#pragma unroll
    for (int k = 0; k < S::SH; ++k) {
        const int lr = r0 + k;
        const uint32_t hnext = hsum3(L[lr + 1][lw - 1], L[lr + 1][lw], L[lr + 1][lw + 1]);
        const uint32_t self = L[lr][lw];
        const uint32_t s9 = hprev + hcur + hnext;  // 3x3 sum including the cell
        // alive next: s9 == 3, or s9 == 4 and alive now
        const uint32_t nv = zero_bytes(s9 ^ 0x03030303u) | (zero_bytes(s9 ^ 0x04040404u) & self);
        hprev = hcur;
        hcur = hnext;

        const int32_t gi = i0 + lr - 1;
        const int32_t gj = j0 + 4 * wc;
        if (interior || (gi < n && gj + 3 <= gi)) {
            *(uint32_t *)(p.nxt + (int64_t)gi * ld + gj) = nv;
        } else if (gi < n && gj <= gi) {  // the word holding the diagonal cell
            uint8_t *q = p.nxt + (int64_t)gi * ld + gj;
            for (int b = 0; b <= gi - gj; ++b) q[b] = (uint8_t)(nv >> (8 * b));
        }
    }
}

template <int MAP>
static bool life_tile(const tri_plan *p, const LifeArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 8: k_life<MAP, 8><<<grid, LifeShape<8>::NT, 0, s>>>(a); return true;
    case 16: k_life<MAP, 16><<<grid, LifeShape<16>::NT, 0, s>>>(a); return true;
    case 32: k_life<MAP, 32><<<grid, LifeShape<32>::NT, 0, s>>>(a); return true;
    case 64: k_life<MAP, 64><<<grid, LifeShape<64>::NT, 0, s>>>(a); return true;
    }
    return false;
}

static bool life_step(const tri_plan *p, const LifeArgs &a, hipStream_t s)
{
    switch (p->map) {
    case TRI_MAP_BB: return life_tile<MAP_BB>(p, a, s);
    case TRI_MAP_RB: return life_tile<MAP_RB>(p, a, s);
    case TRI_MAP_REC: return life_tile<MAP_REC>(p, a, s);
    case TRI_MAP_LAMBDA: return life_tile<MAP_LAMBDA>(p, a, s);
    }
    return false;
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_launch_stencil(const tri_plan *p, uint8_t *cur, uint8_t *nxt,
                                         int64_t ld, int steps, int use_graph, void *stream)
{
    clear_error();
    if (!p) return fail(TRI_E_INVAL, "tri_launch_stencil: plan is NULL");
    if (!p->diag) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: needs include_diag = 1");
    if (p->map == TRI_MAP_UTM)
        return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: UTM has no tile to stage a halo in");
    if (p->tile > 64) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: tile %d > 64", p->tile);
    if (steps < 0) return fail(TRI_E_INVAL, "tri_launch_stencil: steps < 0");
    if (p->n == 0 || steps == 0) return TRI_OK;
    if (!cur || !nxt || cur == nxt) return fail(TRI_E_INVAL, "tri_launch_stencil: bad buffers");
    if (ld < p->n || ld % 4) return fail(TRI_E_INVAL, "tri_launch_stencil: ld must be >= n and a multiple of 4");
    if (((uintptr_t)cur | (uintptr_t)nxt) & 3)
        return fail(TRI_E_INVAL, "tri_launch_stencil: buffers must be 4-byte aligned");
    if (use_graph) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: graph replay not built yet");

    hipStream_t s = (hipStream_t)stream;
    LifeArgs a{plan_tile_grid(p), (int32_t)p->n, ld, cur, nxt};
    for (int k = 0; k < steps; ++k) {
        a.cur = (k & 1) ? nxt : cur;
        a.nxt = (k & 1) ? cur : nxt;
        if (!life_step(p, a, s)) return fail(TRI_E_UNSUPPORTED, "tri_launch_stencil: tile");
        TRI_HIP(hipGetLastError());
    }
    return TRI_OK;
}
