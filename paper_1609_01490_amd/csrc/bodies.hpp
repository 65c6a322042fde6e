// Tile bodies shared by the one-launch-per-domain kernels and the batched
// persistent kernel: a body computes one rho x rho tile (bi, bj) of one
// triangular domain with NT threads, using the LDS buffer it is given.
// Every body contains barriers, so all NT threads of the workgroup call it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace trimap {

// ---------------------------------------------------------------------------
// Game of Life B3/S23 on the lower triangle (cells j > i and outside the
// n x n square are dead and never written).  The tile plus a one-cell halo is
// staged in LDS as 32-bit words of four cells; each thread updates a vertical
// strip of words with byte-sliced arithmetic (neighbour sums never exceed 9,
// so bytes never carry).
// ---------------------------------------------------------------------------
struct LifeTile {
    int32_t n;
    int64_t ld;
    const uint8_t *cur;
    uint8_t *nxt;
};

template <int TILE, int NT>
struct LifeShape {
    static constexpr int WPR = TILE / 4;                          // words per row
    static constexpr int STRIPS_RAW = NT / WPR;
    static constexpr int STRIPS = STRIPS_RAW < TILE ? STRIPS_RAW : TILE;  // strips
    static constexpr int SH = TILE / STRIPS;                      // rows per strip
    static constexpr int ACTIVE = STRIPS * WPR;                   // computing threads
    static constexpr int LW = WPR + 2;                            // LDS words per row
    static constexpr int LR = TILE + 2;                           // LDS rows
    static constexpr int LDS_WORDS = LR * LW;
    static_assert(SH * STRIPS == TILE && SH >= 1 && ACTIVE <= NT, "life tile shape");
};

// bytes of the word at column j (4-aligned) of row i that lie in the domain
// (j + b <= i); 0 when none does
__device__ __forceinline__ uint32_t life_domain_mask(int32_t i, int32_t j)
{
    const int32_t k = i - j;  // number of in-domain bytes minus one
    if (k >= 3) return 0xFFFFFFFFu;
    if (k < 0) return 0u;
    return 0xFFFFFFFFu >> (8 * (3 - k));
}

// one byte (0x01) per zero byte of t, for bytes below 0x80
__device__ __forceinline__ uint32_t life_zero_bytes(uint32_t t)
{
    const uint32_t nz = (t + 0x7F7F7F7Fu) | t;
    return (~nz & 0x80808080u) >> 7;
}

// horizontal 3-sums of a word given its west and east neighbour words
__device__ __forceinline__ uint32_t life_hsum3(uint32_t west, uint32_t w, uint32_t east)
{
    const uint32_t wl = __builtin_amdgcn_alignbit(w, west, 24);  // (w << 8) | (west >> 24)
    const uint32_t wr = __builtin_amdgcn_alignbit(east, w, 8);   // (w >> 8) | (east << 24)
    return w + wl + wr;
}

// HOIST: issue every staging load before the first is used (more registers;
// the standalone kernels and the batched kernel's multi-generation path,
// where it measured 10.1 -> 8.9 ms for the Life half of the 512-instance
// batch), else load and store word by word (the batched kernel's
// one-generation path).
template <int TILE, int NT, bool HOIST = true>
__device__ __forceinline__ void life_tile_body(const LifeTile &p, int32_t bi, int32_t bj,
                                               uint32_t *lds)
{
    using S = LifeShape<TILE, NT>;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t i0 = bi * TILE, j0 = bj * TILE;
    // the halo and the tile lie wholly inside the domain and the square
    const bool interior = (bi != bj) && bj > 0 && (i0 + TILE < n) && (j0 + TILE + 3 < i0);

    // stage rows i0-1 .. i0+TILE, words at columns j0-4 .. j0+TILE.  Every
    // load is unconditional, from an address clamped into the grid, and
    // masked afterwards, so that all of a thread's loads are in flight at
    // once (a load under a condition is waited for where the branches join).
    auto mask_of = [&](int32_t gi, int32_t gj) -> uint32_t {
        if (interior) return 0xFFFFFFFFu;
        return (gi >= 0 && gi < n && gj >= 0 && gj <= gi) ? life_domain_mask(gi, gj) : 0u;
    };
    auto clamped = [&](int32_t gi, int32_t gj) -> const uint32_t * {
        gi = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
        gj = gj < 0 ? 0 : (gj > (int32_t)ld - 4 ? (int32_t)ld - 4 : gj);
        return (const uint32_t *)(p.cur + (int64_t)gi * ld + gj);
    };
    if constexpr (HOIST) {
        constexpr int IT = (S::LDS_WORDS + NT - 1) / NT;
        uint32_t raw[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int idx = threadIdx.x + u * NT;
            raw[u] = *clamped(i0 - 1 + idx / S::LW, j0 - 4 + 4 * (idx % S::LW));
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int idx = threadIdx.x + u * NT;
            if (idx >= S::LDS_WORDS) break;
            lds[idx] = raw[u] & mask_of(i0 - 1 + idx / S::LW, j0 - 4 + 4 * (idx % S::LW));
        }
    } else {
        for (int idx = threadIdx.x; idx < S::LDS_WORDS; idx += NT) {
            const int32_t gi = i0 - 1 + idx / S::LW, gj = j0 - 4 + 4 * (idx % S::LW);
            const uint32_t m = mask_of(gi, gj);
            lds[idx] = m ? *clamped(gi, gj) & m : 0u;
        }
    }
    __syncthreads();
    if (threadIdx.x >= S::ACTIVE) return;

    const int wc = threadIdx.x % S::WPR;  // word column inside the tile
    const int st = threadIdx.x / S::WPR;  // strip
    const int lw = wc + 1;
    const int r0 = st * S::SH + 1;        // first LDS row of the strip
    auto L = [lds](int r, int c) { return lds[r * S::LW + c]; };

    uint32_t hprev = life_hsum3(L(r0 - 1, lw - 1), L(r0 - 1, lw), L(r0 - 1, lw + 1));
    uint32_t hcur = life_hsum3(L(r0, lw - 1), L(r0, lw), L(r0, lw + 1));
#pragma unroll
    for (int k = 0; k < S::SH; ++k) {
        const int lr = r0 + k;
        const uint32_t hnext = life_hsum3(L(lr + 1, lw - 1), L(lr + 1, lw), L(lr + 1, lw + 1));
        const uint32_t self = L(lr, lw);
        const uint32_t s9 = hprev + hcur + hnext;  // 3x3 sum including the cell
        // alive next: s9 == 3, or s9 == 4 and alive now
        const uint32_t nv =
            life_zero_bytes(s9 ^ 0x03030303u) | (life_zero_bytes(s9 ^ 0x04040404u) & self);
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

// ---------------------------------------------------------------------------
// Temporal blocking of the Game of Life: one call advances a tile by up to
// kLifeMaxGen generations.  The tile is staged with a halo of kLifeMaxGen
// rows and one word (4 cells) on each side; the generations run in LDS; only
// the tile is written.  After g generations every cell at least g cells
// inside the staged window is exact (the light cone of a cell grows by one
// cell per generation), so the tile is exact after up to four.  Cells
// outside the domain are forced dead after every generation, as the rule
// requires.  HBM traffic per generation falls from one read and one write of
// the tile to about (1 + halo) / g reads and 1 / g writes.
// ---------------------------------------------------------------------------
constexpr int kLifeMaxGen = 4;

template <int TILE>
struct LifeMultiShape {
    static constexpr int NT = 256;
    static constexpr int W = TILE / 4 + 2;            // words per staged row
    static constexpr int R = TILE + 2 * kLifeMaxGen;  // staged rows
    static constexpr int PW = W + 2;                  // padded LDS row (zero border)
    static constexpr int PR = R + 2;
    static constexpr int STRIPS = NT / W;             // strips of rows per word column
    static constexpr int SH = (R + STRIPS - 1) / STRIPS;
    static constexpr int WORDS = PR * PW;             // one buffer; the body uses two
};

// domain mask of the staged word at row gi, column gj (4-aligned): bytes of
// cells 0 <= gj + b <= gi < n
__device__ __forceinline__ uint32_t life_window_mask(int32_t gi, int32_t gj, int32_t n)
{
    if (gi < 0 || gi >= n || gj < 0) return 0u;
    return life_domain_mask(gi, gj);
}

// ---------------------------------------------------------------------------
// Bit-sliced variant for 64 x 64 tiles: one bit per cell, 32 cells per word.
// The staged window (rows i0-K .. i0+63+K, cells j0-H .. j0+63+H for a halo
// of K rows and H = 4, 8 or 16 cells) is kept as four words per row covering
// cells j0-32 .. j0+95: word 0 holds the left halo in its top H bits, words
// 1 and 2 the tile's 64 cells, word 3 the right halo in its low H bits.
// Rows moved byte by byte are packed with one wave ballot per 64 cells and
// unpacked one cell per lane; rows moved as 16-byte vectors are packed and
// unpacked four cells at a time by multiplies.  Per generation a word's eight neighbour
// planes are summed with bitwise adders: the row above and the row below as
// 2-bit horizontal sums (west, self, east), the own row without the cell;
// with s = their total, a cell lives next iff (s >> 1) == 1 and (s & 1 or it
// lives now), i.e. s = 3, or s = 2 and alive (B3/S23).  Cells outside the
// staged window are not loaded; like cells beyond the byte-sliced window
// they only reach the tile after more generations than the halo is deep.
// ---------------------------------------------------------------------------
// Generations per launch of the bit-sliced body with 16-byte rows in the
// batched kernel (an 8-row, 8-cell halo: its 80 staged rows take the same
// five 16-row rounds of loads as the 72 of a 4-row halo; a deeper halo does
// not fit that kernel's 128 registers)
constexpr int kLifeBitsMaxGen = 8;
// The same in the stencil kernel: a 16-row, 16-cell halo (96 staged rows)
// halves the launches, and so the round trips of the grid through HBM, for
// a fifth more arithmetic per useful generation than the 8-row halo
constexpr int kLifeBitsStencilGen = 16;

template <int KH = kLifeMaxGen>
struct LifeBitsShape {
    static constexpr int TILE = 64;
    static constexpr int K = KH;             // halo rows (generations per launch at most)
    static constexpr int R = TILE + 2 * K;   // staged rows
    static constexpr int PR = R + 2;         // plus a zero row above and below
    static constexpr int WPR = 4;            // words per row
    // one buffer and a guard word (the body uses two buffers between three
    // zero guard words)
    static constexpr int WORDS = PR * WPR + 2;
};

// bits b of word c (cells jb + b, jb = j0 - 32 + 32 c) of staged row gi that
// lie in the domain 0 <= j <= gi < n
__device__ __forceinline__ uint32_t life_bits_mask(int32_t gi, int32_t jb, int32_t n)
{
    if (gi < 0 || gi >= n) return 0u;
    const int32_t lo = jb < 0 ? -jb : 0;        // first bit with j >= 0
    const int32_t hi = gi - jb;                 // last bit with j <= gi
    if (hi < lo || lo > 31) return 0u;
    const uint32_t upto = hi >= 31 ? 0xFFFFFFFFu : ((2u << hi) - 1u);
    return upto & (0xFFFFFFFFu << lo);
}

// Four cells (bytes) to four bits, cell k to bit k: domain cells hold 0 or
// 1, so bit 0 of each byte is the cell; one multiply gathers bit 0 of byte
// k at bit 24 + k with no carries (the other partial products land below
// bit 24 or beyond bit 31).  Bytes outside the domain may hold anything:
// their bits are cleared by the domain masks after staging.
__device__ __forceinline__ uint32_t life_cells4_to_bits(uint32_t x)
{
    x &= 0x01010101u;
    return (x * 0x01020408u) >> 24;
}

// The inverse for four bits: bit k to byte k (0 or 1); the four shifted
// copies of the nibble overlap only away from bits 0, 8, 16 and 24.
__device__ __forceinline__ uint32_t life_bits4_to_cells(uint32_t b)
{
    return (b * 0x00204081u) & 0x01010101u;
}

// The update run by one wave per tile (64 threads): no workgroup barriers,
// and four times as many tiles in flight per CU as with 256 threads, which
// is what the load-then-compute pattern needs to keep HBM busy on large
// grids (on small grids the byte-sliced body, whose tile finishes sooner,
// is faster).  lds: at least 2 * LifeBitsShape<KH>::WORDS words.
// VEC (ld a multiple of 16, 16-byte aligned grids): rows are staged with
// 16-byte loads, four lanes per row, and written back with 16-byte stores:
// 5 loads and 4 stores per lane and tile instead of 72 single-byte loads and
// 64 single-byte stores, whose instruction count bounds the byte path.
// KH: halo rows above and below the tile (and at most that many
// generations); other than 4 only with VEC, which stages 4 halo cells left
// and right of each row for KH <= 4, 8 for KH <= 8 and 16 for KH <= 16.
template <bool VEC = false, int KH = kLifeMaxGen>
__device__ __forceinline__ void life_bits_wave_body(const LifeTile &p, int32_t bi, int32_t bj,
                                                    int gens, uint32_t *lds)
{
    static_assert(VEC || KH == kLifeMaxGen, "byte row moves stage a 4-row halo");
    static_assert(KH >= 1 && KH <= 16, "halo");
    using S = LifeBitsShape<KH>;
    constexpr int T = S::TILE, K = S::K;
    constexpr int RB = (S::R + 15) / 16;       // staged rows per lane in the update
    constexpr int CH = 18;                     // rows per load batch
    constexpr int HG = S::R / 8;               // halo groups of eight rows
    static_assert(VEC || (S::R % CH == 0 && S::R % 8 == 0), "row batches");
    constexpr int BUF = S::PR * S::WPR;
    uint32_t *A = lds + 1, *B = lds + 2 + BUF;  // lds[0], A[BUF] = B[-1], B[BUF]: zero
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t i0 = bi * T, j0 = bj * T;
    const int lane = threadIdx.x & 63;  // any wave of the workgroup runs its own tile

    if (lane < S::WPR) {
        A[lane] = A[(S::PR - 1) * S::WPR + lane] = 0u;
        B[lane] = B[(S::PR - 1) * S::WPR + lane] = 0u;
        if (lane < 3) lds[lane * (BUF + 1)] = 0u;
    }
    const int32_t gj = j0 + lane;
    // the update's word layout: lane = 4 * band + column, and band b owns
    // staged rows b * RB .. b * RB + RB - 1 of one word column
    const int wc = lane & 3, rb0 = (lane >> 2) * RB;
    // a tile whose staged window (rows i0 - K .. i0 + 63 + K, the four
    // words' cells j0 - 32 .. j0 + 95) lies inside the domain needs no
    // masks: every word then has 0 <= j <= i for all its cells
    static_assert(2 * T >= 96 + K, "inner tiles are two tile columns off the diagonal");
    const bool inner = bj >= 1 && bi - bj >= 2 && i0 + T + K <= n;
    uint32_t msk[RB];
    if (inner) {
#pragma unroll
        for (int k = 0; k < RB; ++k) msk[k] = rb0 + k < S::R ? ~0u : 0u;
    } else {
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const int r = rb0 + k;
            msk[k] = r < S::R ? life_bits_mask(i0 - K + r, j0 - 32 + 32 * wc, n) : 0u;
        }
    }
    if constexpr (VEC) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        constexpr int RND = (S::R + 15) / 16;   // rounds of 16 rows
        constexpr int HR = (2 * S::R + 63) / 64;  // rounds of 64 halo words
        const int q = lane & 3, rr = lane >> 2;  // chunk q (16 cells) of row rr
        const int32_t ldi = (int32_t)ld;
        const int32_t col = j0 + 16 * q < ldi - 16 ? j0 + 16 * q : ldi - 16;
        // every load from a clamped address first, masked afterwards
        constexpr int HW = K > 8 ? 16 : (K > 4 ? 8 : 4);  // halo cells left and right
        typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
        u32x4 cv[RND];
        u32x4 hv[HR];
#pragma unroll
        for (int r = 0; r < RND; ++r) {
            const int32_t gi = i0 - K + 16 * r + rr;
            const int32_t gic = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
            // rows past the staged window (last round) are not loaded
            if (S::R % 16 == 0 || r + 1 < RND || 16 * r + rr < S::R)
                cv[r] = *(const u32x4 *)(p.cur + (int64_t)gic * ld + col);
            else
                cv[r] = u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < HR; ++k) {
            const int t = lane + 64 * k;  // halo word t: row t / 2, west or east
            const int row = (t >> 1) < S::R ? (t >> 1) : S::R - 1;
            const int32_t gi = i0 - K + row;
            const int32_t gic = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
            int32_t hc = (t & 1) ? j0 + T : j0 - HW;
            hc = hc < 0 ? 0 : (hc > ldi - HW ? ldi - HW : hc);
            if constexpr (HW == 16) {
                hv[k] = *(const u32x4 *)(p.cur + (int64_t)gic * ld + hc);
            } else if constexpr (HW == 8) {
                const u32x2 v = *(const u32x2 *)(p.cur + (int64_t)gic * ld + hc);
                hv[k] = u32x4{v.x, v.y, 0u, 0u};
            } else {
                hv[k] = u32x4{*(const uint32_t *)(p.cur + (int64_t)gic * ld + hc), 0u, 0u, 0u};
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        uint16_t *A16 = (uint16_t *)A;
#pragma unroll
        for (int r = 0; r < RND; ++r) {
            const int row = 16 * r + rr;
            if (row < S::R) {
                const uint32_t b16 = life_cells4_to_bits(cv[r].x) |
                                     (life_cells4_to_bits(cv[r].y) << 4) |
                                     (life_cells4_to_bits(cv[r].z) << 8) |
                                     (life_cells4_to_bits(cv[r].w) << 12);
                A16[((row + 1) * S::WPR + 1 + (q >> 1)) * 2 + (q & 1)] = (uint16_t)b16;
            }
        }
#pragma unroll
        for (int k = 0; k < HR; ++k) {
            const int t = lane + 64 * k;
            if (t < 2 * S::R) {
                // west cells end at bit 31 of word 0, east cells start at
                // bit 0 of word 3
                const uint32_t hb = life_cells4_to_bits(hv[k].x) |
                                    (HW >= 8 ? life_cells4_to_bits(hv[k].y) << 4 : 0u) |
                                    (HW == 16 ? life_cells4_to_bits(hv[k].z) << 8 |
                                                    life_cells4_to_bits(hv[k].w) << 12
                                              : 0u);
                A[((t >> 1) + 1) * S::WPR + ((t & 1) ? 3 : 0)] = (t & 1) ? hb : hb << (32 - HW);
            }
        }
        // then clear every staged bit outside the domain (rows beyond the
        // grid, cells above the diagonal or left of column 0, clamped loads)
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        if (!inner) {
#pragma unroll
            for (int k = 0; k < RB; ++k)
                if (rb0 + k < S::R) A[(rb0 + k + 1) * S::WPR + wc] &= msk[k];
        }
    } else {
    // halo cells of all rows: lane covers row 8 q + lane / 8, cell lane % 8
    uint64_t hb[HG];
    {
        const int hh = lane & 7;
        const int32_t hj = hh < 4 ? j0 - 4 + hh : j0 + T + (hh - 4);
        // raw values and their conditions kept apart until every load is
        // issued (a value masked at once makes its load wait at once)
        uint32_t hv[HG];
        bool hok[HG];
#pragma unroll
        for (int q = 0; q < HG; ++q) {
            const int32_t gi = i0 - K + 8 * q + (lane >> 3);
            const int32_t gic = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
            const int32_t hjc = hj < 0 ? 0 : (hj < gic ? hj : gic);
            hv[q] = p.cur[(int64_t)gic * ld + hjc];
            hok[q] = gi >= 0 && gi < n && hj >= 0 && hj <= gi;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < HG; ++q) hb[q] = __ballot(hok[q] && hv[q] != 0u);
    }
    // the 64 cells of each row, CH rows per batch of loads
#pragma unroll
    for (int b0 = 0; b0 < S::R; b0 += CH) {
        uint32_t cv[CH];
        bool cok[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int32_t gi = i0 - K + b0 + k;
            const int32_t gic = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
            cv[k] = p.cur[(int64_t)gic * ld + (gj < gic ? gj : gic)];
            cok[k] = gi >= 0 && gi < n && gj <= gi;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int r = b0 + k;
            const uint64_t c64 = __ballot(cok[k] && cv[k] != 0u);
            const uint32_t h8 = (uint32_t)(hb[r >> 3] >> (8 * (r & 7))) & 0xFFu;
            if (lane == 0) {
                uint32_t *row = A + (r + 1) * S::WPR;
                row[0] = (h8 & 0xFu) << 28;
                row[1] = (uint32_t)c64;
                row[2] = (uint32_t)(c64 >> 32);
                row[3] = h8 >> 4;
            }
        }
    }
    }
    // LDS operations of one wave complete in order; the wait and the
    // barrier keep the compiler from moving reads of other lanes' words
    // above the writes they depend on
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();

    // Neighbour sums of staged row r (A's row r + 1; rows -1 and R are the
    // zero rows): the west and east neighbours of each cell as a 2-bit sum
    // (h0, h1) and with the cell itself (s0, s1).  A lane walks its band
    // downwards and computes each row's sums once for the three rows that
    // use them.  The shifts take only bit 31 of the west word and bit 0 of
    // the east word, so the edge columns read across the row boundary (or
    // into a guard word) without a test: generation g reads bit 31 of
    // word 3 and bit 0 of word 0 clear, since the staged halo cells fill at
    // most the low and the high 16 bits and the g - 1 <= 15 generations
    // before it spread life by at most one bit each.
    const auto row_sums = [&](const uint32_t *src, int r, uint32_t &s0, uint32_t &s1,
                              uint32_t &h0, uint32_t &h1, uint32_t &x) {
        const uint32_t *row = src + (r + 1) * S::WPR;
        const uint32_t w = row[wc - 1], e = row[wc + 1];
        x = row[wc];
        const uint32_t W = __builtin_amdgcn_alignbit(x, w, 31), E = __builtin_amdgcn_alignbit(e, x, 1);
        h0 = W ^ E;
        h1 = W & E;
        s0 = h0 ^ x;
        s1 = h1 | (x & h0);
    };
    constexpr bool FULL = S::R % 16 == 0;  // every band holds RB rows
    if constexpr (KH == 1) {
        // one generation: only the tile's own words (1 and 2 of staged rows
        // 1 .. 64) are needed, two rows of one word per lane; no output
        // mask, since only cells of the domain are written back
        const int c1 = 1 + (lane & 1), r1 = 1 + 2 * (lane >> 1);
        const auto sums_at = [&](int r, uint32_t &s0, uint32_t &s1, uint32_t &h0, uint32_t &h1,
                                 uint32_t &x) {
            const uint32_t *row = A + (r + 1) * S::WPR;
            const uint32_t w = row[c1 - 1], e = row[c1 + 1];
            x = row[c1];
            const uint32_t W = __builtin_amdgcn_alignbit(x, w, 31),
                           E = __builtin_amdgcn_alignbit(e, x, 1);
            h0 = W ^ E;
            h1 = W & E;
            s0 = h0 ^ x;
            s1 = h1 | (x & h0);
        };
        uint32_t u0, u1, m0, m1, mc, q0, q1, z0, z1, z2;
        sums_at(r1 - 1, u0, u1, z0, z1, z2);
        sums_at(r1, q0, q1, m0, m1, mc);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int r = r1 + k;
            uint32_t d0, d1, n0, n1, nc;
            sums_at(r + 1, d0, d1, n0, n1, nc);
            const uint32_t t0 = u0 ^ d0 ^ m0;
            const uint32_t c0 = (u0 & d0) | (m0 & (u0 ^ d0));
            const uint32_t x1 = u1 ^ d1 ^ m1 ^ c0;
            const uint32_t h2 = ((u1 & d1) | (m1 & (u1 ^ d1))) | (c0 & (u1 | d1 | m1));
            B[(r + 1) * S::WPR + c1] = x1 & ~h2 & (t0 | mc);
            u0 = q0; u1 = q1;
            q0 = d0; q1 = d1;
            m0 = n0; m1 = n1; mc = nc;
        }
        (void)gens;
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        uint32_t *t = A;
        A = B;
        B = t;
    } else
    for (int g = 0; g < gens; ++g) {
        if (FULL || rb0 < S::R) {
            uint32_t u0, u1, m0, m1, mc, q0, q1, z0, z1, z2;
            row_sums(A, rb0 - 1, u0, u1, z0, z1, z2);
            row_sums(A, rb0, q0, q1, m0, m1, mc);
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const int r = rb0 + k;
                if (FULL || r < S::R) {
                    uint32_t d0, d1, n0, n1, nc;
                    row_sums(A, r + 1, d0, d1, n0, n1, nc);
                    // 0..8 live neighbours: bit 0 t0, bit 1 x1, 4 or more h2
                    const uint32_t t0 = u0 ^ d0 ^ m0;
                    const uint32_t c0 = (u0 & d0) | (m0 & (u0 ^ d0));
                    const uint32_t x1 = u1 ^ d1 ^ m1 ^ c0;
                    const uint32_t h2 = ((u1 & d1) | (m1 & (u1 ^ d1))) | (c0 & (u1 | d1 | m1));
                    B[(r + 1) * S::WPR + wc] = x1 & ~h2 & (t0 | mc) & msk[k];
                    u0 = q0; u1 = q1;
                    q0 = d0; q1 = d1;
                    m0 = n0; m1 = n1; mc = nc;
                }
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        uint32_t *t = A;
        A = B;
        B = t;
    }

    if constexpr (VEC) {
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
        const int q = lane & 3, rr = lane >> 2;
        const int32_t jc = j0 + 16 * q;
#pragma unroll
        for (int r0 = 0; r0 < T; r0 += 16) {
            const int tr = r0 + rr;
            const int32_t gi = i0 + tr;
            if (gi >= n) continue;
            const uint32_t b16 =
                (A[(K + tr + 1) * S::WPR + 1 + (q >> 1)] >> (16 * (q & 1))) & 0xFFFFu;
            u32x4 o;
            o.x = life_bits4_to_cells(b16 & 0xFu);
            o.y = life_bits4_to_cells((b16 >> 4) & 0xFu);
            o.z = life_bits4_to_cells((b16 >> 8) & 0xFu);
            o.w = life_bits4_to_cells(b16 >> 12);
            uint8_t *dst = p.nxt + (int64_t)gi * ld + jc;
            if (jc + 15 <= gi) {
                *(u32x4 *)dst = o;
            } else {  // the chunk meets the diagonal: cells jc .. gi only
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (jc + e <= gi) dst[e] = (uint8_t)((b16 >> e) & 1u);
            }
        }
    } else {
        for (int tr = 0; tr < T; ++tr) {
            const int32_t gi = i0 + tr;
            if (gi >= n) break;
            const uint32_t wv = A[(K + tr + 1) * S::WPR + 1 + (lane >> 5)];
            if (gj <= gi) p.nxt[(int64_t)gi * ld + gj] = (uint8_t)((wv >> (lane & 31)) & 1u);
        }
    }
}

// One generation of two neighbouring 64 x 64 tiles, (bi, bj) and (bi, bj + 1),
// by one wave, bit-sliced as above, with 16-byte row moves: the window is
// 64 rows x 128 cells, so every row segment the wave loads or stores is a
// whole 128-byte line where bj is even (a 64-cell tile alone moves 64-byte
// halves, the other half belonging to the neighbouring tile and another
// wave).  The staged window (rows i0 - 1 .. i0 + 64) is kept as six words
// per row: word 0 holds cells j0 - 4 .. j0 - 1 in its top bits, words 1 to
// 4 the 128 cells, word 5 cells j0 + 128 .. j0 + 131 in its low bits.
// Only cells of the domain are written back, and with two == false only
// those of the first tile (the second then belongs to another window or
// lies outside the domain).  lds: at least LifeBits1Pair::WORDS words (ld
// a multiple of 16, 16-byte aligned grids).
struct LifeBits1Pair {
    static constexpr int R = 66;            // staged rows
    static constexpr int PR = R + 2;        // plus a zero row above and below
    static constexpr int WPR = 6;           // words per row
    static constexpr int BUF = PR * WPR;
    static constexpr int WORDS = 2 * BUF;
    static constexpr int RND = (R + 7) / 8; // rounds of 8 rows (8 lanes per row)
    static constexpr int HR = (2 * R + 63) / 64;  // rounds of 64 halo words
};

__device__ __forceinline__ void life_bits1_pair_body(const LifeTile &p, int32_t bi, int32_t bj,
                                                     bool two, uint32_t *lds)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    using S = LifeBits1Pair;
    constexpr int T = 64, WPR = S::WPR;
    uint32_t *A = lds, *B = lds + S::BUF;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t ldi = (int32_t)ld;
    const int32_t i0 = bi * T, j0 = bj * T;
    const int lane = threadIdx.x & 63;

    // loads: lane = 8 * row + chunk, chunk q of 16 cells; every address
    // clamped into the grid, values outside the domain masked after staging
    const int q = lane & 7, rr = lane >> 3;
    const int32_t col = j0 + 16 * q < ldi - 16 ? j0 + 16 * q : ldi - 16;
    u32x4 cv[S::RND];
    uint32_t hv[S::HR];
#pragma unroll
    for (int r = 0; r < S::RND; ++r) {
        const int row = 8 * r + rr;
        const int32_t gi = i0 - 1 + row;
        const int32_t gic = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
        if (r + 1 < S::RND || row < S::R)
            cv[r] = *(const u32x4 *)(p.cur + (int64_t)gic * ld + col);
        else
            cv[r] = u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int k = 0; k < S::HR; ++k) {
        const int t = lane + 64 * k;  // halo word t: row t / 2, west or east
        const int row = (t >> 1) < S::R ? (t >> 1) : S::R - 1;
        const int32_t gi = i0 - 1 + row;
        const int32_t gic = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
        int32_t hc = (t & 1) ? j0 + 2 * T : j0 - 4;
        hc = hc < 0 ? 0 : (hc > ldi - 4 ? ldi - 4 : hc);
        hv[k] = *(const uint32_t *)(p.cur + (int64_t)gic * ld + hc);
    }
    // the zero rows above and below the window
    if (lane < WPR) {
        A[lane] = 0u;
        A[(S::PR - 1) * WPR + lane] = 0u;
    }
    __builtin_amdgcn_sched_barrier(0);
    uint16_t *A16 = (uint16_t *)A;
#pragma unroll
    for (int r = 0; r < S::RND; ++r) {
        const int row = 8 * r + rr;
        if (row < S::R) {
            const uint32_t b16 = life_cells4_to_bits(cv[r].x) |
                                 (life_cells4_to_bits(cv[r].y) << 4) |
                                 (life_cells4_to_bits(cv[r].z) << 8) |
                                 (life_cells4_to_bits(cv[r].w) << 12);
            A16[((row + 1) * WPR + 1 + (q >> 1)) * 2 + (q & 1)] = (uint16_t)b16;
        }
    }
#pragma unroll
    for (int k = 0; k < S::HR; ++k) {
        const int t = lane + 64 * k;
        if (t < 2 * S::R) {
            const uint32_t hb = life_cells4_to_bits(hv[k]);
            A[((t >> 1) + 1) * WPR + ((t & 1) ? 5 : 0)] = (t & 1) ? hb : hb << 28;
        }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    // staged bits outside the domain cleared, unless the whole window
    // (cells j0 - 32 .. j0 + 159 of rows i0 - 1 .. i0 + 64) lies inside it
    const bool inner = bj >= 1 && bi - bj >= 3 && i0 + T + 1 <= n;
    if (!inner) {
        for (int idx = lane; idx < S::R * WPR; idx += 64) {
            const int row = idx / WPR, c = idx - row * WPR;
            A[(row + 1) * WPR + c] &= life_bits_mask(i0 - 1 + row, j0 - 32 + 32 * c, n);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
    // the update: words 1 .. 4 of staged rows 1 .. 64, four rows of one
    // word per lane (lane = 4 * band + word - 1)
    const int c1 = 1 + (lane & 3), r1 = 1 + 4 * (lane >> 2);
    const auto sums_at = [&](int r, uint32_t &s0, uint32_t &s1, uint32_t &h0, uint32_t &h1,
                             uint32_t &x) {
        const uint32_t *row = A + (r + 1) * WPR;
        const uint32_t w = row[c1 - 1], e = row[c1 + 1];
        x = row[c1];
        const uint32_t W = __builtin_amdgcn_alignbit(x, w, 31), E = __builtin_amdgcn_alignbit(e, x, 1);
        h0 = W ^ E;
        h1 = W & E;
        s0 = h0 ^ x;
        s1 = h1 | (x & h0);
    };
    {
        uint32_t u0, u1, m0, m1, mc, q0, q1, z0, z1, z2;
        sums_at(r1 - 1, u0, u1, z0, z1, z2);
        sums_at(r1, q0, q1, m0, m1, mc);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int r = r1 + k;
            uint32_t d0, d1, n0, n1, nc;
            sums_at(r + 1, d0, d1, n0, n1, nc);
            // 0..8 live neighbours: bit 0 t0, bit 1 x1, 4 or more h2
            const uint32_t t0 = u0 ^ d0 ^ m0;
            const uint32_t c0 = (u0 & d0) | (m0 & (u0 ^ d0));
            const uint32_t x1 = u1 ^ d1 ^ m1 ^ c0;
            const uint32_t h2 = ((u1 & d1) | (m1 & (u1 ^ d1))) | (c0 & (u1 | d1 | m1));
            B[(r + 1) * WPR + c1] = x1 & ~h2 & (t0 | mc);
            u0 = q0; u1 = q1;
            q0 = d0; q1 = d1;
            m0 = n0; m1 = n1; mc = nc;
        }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    // unpack and store: lane = 8 * row + chunk, 8 rounds of 8 rows
    const int32_t jc = j0 + 16 * q;
#pragma unroll
    for (int r0 = 0; r0 < T; r0 += 8) {
        const int tr = r0 + rr;
        const int32_t gi = i0 + tr;
        if (gi >= n) continue;
        const uint32_t b16 = (B[(tr + 2) * WPR + 1 + (q >> 1)] >> (16 * (q & 1))) & 0xFFFFu;
        if (jc > gi || (!two && q >= 4)) continue;  // above the diagonal, or not this window's
        u32x4 o;
        o.x = life_bits4_to_cells(b16 & 0xFu);
        o.y = life_bits4_to_cells((b16 >> 4) & 0xFu);
        o.z = life_bits4_to_cells((b16 >> 8) & 0xFu);
        o.w = life_bits4_to_cells(b16 >> 12);
        uint8_t *dst = p.nxt + (int64_t)gi * ld + jc;
        if (jc + 15 <= gi) {
            *(u32x4 *)dst = o;
        } else {  // the chunk meets the diagonal: cells jc .. gi only
#pragma unroll
            for (int e = 0; e < 16; ++e)
                if (jc + e <= gi) dst[e] = (uint8_t)((b16 >> e) & 1u);
        }
    }
}

// Up to 16 generations of two neighbouring 64 x 64 tiles, (bi, bj) and
// (bi, bj + 1), by one wave, bit-sliced, with 16-byte row moves.  The
// window is rows i0 - 16 .. i0 + 79 and cells j0 - 16 .. j0 + 143: five
// words per row, the 16 halo cells on each side sharing the edge words with
// the tiles (a single tile's window needs four words per row for 64 cells,
// half of two of them halo), so a generation updates 5 words of 96 rows for
// 128 cells instead of 8 for two tiles.  After g generations every cell at
// least g cells inside the window is exact (the light cone grows by one
// cell per generation), whatever the cells outside it hold: the edge words
// read across the row boundary without a test.  Cells outside the domain
// are forced dead after every generation; only cells of the domain are
// written back, and with two == false only those of the first tile.
// Lanes 0 .. 59 update: lane = 5 * band + word, band b owns
// rows 8 b .. 8 b + 7.  lds: at least LifeBits16Pair::WORDS words (ld a
// multiple of 16, 16-byte aligned grids); 1 <= gens <= 16.
struct LifeBits16Pair {
    static constexpr int K = 16;                  // halo rows and cells
    static constexpr int R = 64 + 2 * K;          // staged rows
    static constexpr int PR = R + 2;              // plus a zero row above and below
    static constexpr int WPR = 5;                 // words per row
    static constexpr int BUF = PR * WPR;
    static constexpr int WORDS = 2 * BUF + 3;     // two buffers between three zero guard words
    static constexpr int CH = 10;                 // 16-cell chunks per row
    static constexpr int NCH = R * CH;
    static constexpr int RNDS = (NCH + 63) / 64;  // load rounds, in batches
    static constexpr int BANDS = 12, RB = 8;
    static_assert(BANDS * RB == R && BANDS * WPR <= 64, "update layout");
};

__device__ __forceinline__ void life_bits16_pair_body(const LifeTile &p, int32_t bi, int32_t bj,
                                                      bool two, int gens, uint32_t *lds)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    using S = LifeBits16Pair;
    constexpr int T = 64, K = S::K, WPR = S::WPR;
    uint32_t *A = lds + 1, *B = lds + 2 + S::BUF;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t ldi = (int32_t)ld;
    const int32_t i0 = bi * T, j0 = bj * T, jw = j0 - K;
    const int lane = threadIdx.x & 63;

    if (lane < WPR) {
        A[lane] = A[(S::PR - 1) * WPR + lane] = 0u;
        B[lane] = B[(S::PR - 1) * WPR + lane] = 0u;
        if (lane < 3) lds[lane * (S::BUF + 1)] = 0u;
    }
    // staging: chunk idx = 10 * row + k (16 cells at jw + 16 k), loaded from
    // clamped addresses, NB rounds of 64 chunks per batch
    constexpr int NB = 5;
    uint16_t *A16 = (uint16_t *)A;
#pragma unroll
    for (int b0 = 0; b0 < S::RNDS; b0 += NB) {
        u32x4 v[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int idx = lane + 64 * (b0 + u);
            const int row = idx / S::CH, k = idx - row * S::CH;
            const int32_t gi = i0 - K + (row < S::R ? row : S::R - 1);
            const int32_t gic = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
            int32_t c = jw + 16 * k;
            c = c < 0 ? 0 : (c > ldi - 16 ? ldi - 16 : c);
            if (b0 + u < S::RNDS && idx < S::NCH)
                v[u] = *(const u32x4 *)(p.cur + (int64_t)gic * ld + c);
            else
                v[u] = u32x4{0u, 0u, 0u, 0u};
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int idx = lane + 64 * (b0 + u);
            if (b0 + u < S::RNDS && idx < S::NCH) {
                const int row = idx / S::CH, k = idx - row * S::CH;
                const uint32_t b16 = life_cells4_to_bits(v[u].x) |
                                     (life_cells4_to_bits(v[u].y) << 4) |
                                     (life_cells4_to_bits(v[u].z) << 8) |
                                     (life_cells4_to_bits(v[u].w) << 12);
                A16[((row + 1) * WPR + (k >> 1)) * 2 + (k & 1)] = (uint16_t)b16;
            }
        }
    }
    // domain masks, unless the window (cells j0 - 16 .. j0 + 143 of rows
    // i0 - 16 .. i0 + 79) lies inside the domain
    const int wc = lane % WPR, band = lane / WPR;
    const bool act = band < S::BANDS;
    const int rb0 = band * S::RB;
    const bool inner = bj >= 1 && bi - bj >= 3 && i0 + T + K <= n;
    uint32_t msk[S::RB];
#pragma unroll
    for (int k = 0; k < S::RB; ++k)
        msk[k] = !act ? 0u : (inner ? ~0u : life_bits_mask(i0 - K + rb0 + k, jw + 32 * wc, n));
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    if (!inner) {
        if (act) {
#pragma unroll
            for (int k = 0; k < S::RB; ++k) A[(rb0 + k + 1) * WPR + wc] &= msk[k];
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
    const auto row_sums = [&](const uint32_t *src, int r, uint32_t &s0, uint32_t &s1,
                              uint32_t &h0, uint32_t &h1, uint32_t &x) {
        const uint32_t *row = src + (r + 1) * WPR;
        const uint32_t w = row[wc - 1], e = row[wc + 1];
        x = row[wc];
        const uint32_t W = __builtin_amdgcn_alignbit(x, w, 31), E = __builtin_amdgcn_alignbit(e, x, 1);
        h0 = W ^ E;
        h1 = W & E;
        s0 = h0 ^ x;
        s1 = h1 | (x & h0);
    };
    for (int g = 0; g < gens; ++g) {
        if (act) {
            uint32_t u0, u1, m0, m1, mc, q0, q1, z0, z1, z2;
            row_sums(A, rb0 - 1, u0, u1, z0, z1, z2);
            row_sums(A, rb0, q0, q1, m0, m1, mc);
#pragma unroll
            for (int k = 0; k < S::RB; ++k) {
                const int r = rb0 + k;
                uint32_t d0, d1, n0, n1, nc;
                row_sums(A, r + 1, d0, d1, n0, n1, nc);
                // 0..8 live neighbours: bit 0 t0, bit 1 x1, 4 or more h2
                const uint32_t t0 = u0 ^ d0 ^ m0;
                const uint32_t c0 = (u0 & d0) | (m0 & (u0 ^ d0));
                const uint32_t x1 = u1 ^ d1 ^ m1 ^ c0;
                const uint32_t h2 = ((u1 & d1) | (m1 & (u1 ^ d1))) | (c0 & (u1 | d1 | m1));
                B[(r + 1) * WPR + wc] = x1 & ~h2 & (t0 | mc) & msk[k];
                u0 = q0; u1 = q1;
                q0 = d0; q1 = d1;
                m0 = n0; m1 = n1; mc = nc;
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        uint32_t *t = A;
        A = B;
        B = t;
    }
    // the tiles' cells: rows i0 .. i0 + 63 (staged K ..), chunks 1 .. 8
    const int q = lane & 7, rr = lane >> 3;
    const int ch = 1 + q;
    const int32_t jc = j0 + 16 * q;
#pragma unroll
    for (int r0 = 0; r0 < T; r0 += 8) {
        const int tr = r0 + rr;
        const int32_t gi = i0 + tr;
        if (gi >= n) continue;
        const uint32_t b16 = (A[(tr + K + 1) * WPR + (ch >> 1)] >> (16 * (ch & 1))) & 0xFFFFu;
        if (jc > gi || (!two && q >= 4)) continue;  // above the diagonal, or not this window's
        u32x4 o;
        o.x = life_bits4_to_cells(b16 & 0xFu);
        o.y = life_bits4_to_cells((b16 >> 4) & 0xFu);
        o.z = life_bits4_to_cells((b16 >> 8) & 0xFu);
        o.w = life_bits4_to_cells(b16 >> 12);
        uint8_t *dst = p.nxt + (int64_t)gi * ld + jc;
        if (jc + 15 <= gi) {
            *(u32x4 *)dst = o;
        } else {  // the chunk meets the diagonal: cells jc .. gi only
#pragma unroll
            for (int e = 0; e < 16; ++e)
                if (jc + e <= gi) dst[e] = (uint8_t)((b16 >> e) & 1u);
        }
    }
}

// lds: 2 * LifeMultiShape<TILE>::WORDS words; 256 threads; 1 <= gens <= 4;
// HOIST as for life_tile_body
template <int TILE, bool HOIST = true>
__device__ __forceinline__ void life_multi_tile_body(const LifeTile &p, int32_t bi, int32_t bj,
                                                     int gens, uint32_t *lds)
{
    using S = LifeMultiShape<TILE>;
    uint32_t *buf0 = lds, *buf1 = lds + S::WORDS;
    const int32_t n = p.n;
    const int64_t ld = p.ld;
    const int32_t i0 = bi * TILE, j0 = bj * TILE;
    const int K = kLifeMaxGen;

    // stage rows i0-K .. i0+TILE+K-1, words at columns j0-4 .. j0+TILE, with
    // a zero border around the window; unconditional loads from clamped
    // addresses, masked afterwards (as in life_tile_body)
    auto mask_of = [&](int pr, int pw) -> uint32_t {
        if (pr < 1 || pr > S::R || pw < 1 || pw > S::W) return 0u;
        return life_window_mask(i0 - K + (pr - 1), j0 - 4 + 4 * (pw - 1), n);
    };
    auto clamped = [&](int pr, int pw) -> const uint32_t * {
        int32_t gi = i0 - K + (pr - 1), gj = j0 - 4 + 4 * (pw - 1);
        gi = gi < 0 ? 0 : (gi >= n ? n - 1 : gi);
        gj = gj < 0 ? 0 : (gj > (int32_t)ld - 4 ? (int32_t)ld - 4 : gj);
        return (const uint32_t *)(p.cur + (int64_t)gi * ld + gj);
    };
    if constexpr (HOIST) {
        constexpr int IT = (S::WORDS + S::NT - 1) / S::NT;
        uint32_t raw[IT];
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int idx = threadIdx.x + u * S::NT;
            raw[u] = *clamped(idx / S::PW, idx % S::PW);
        }
#pragma unroll
        for (int u = 0; u < IT; ++u) {
            const int idx = threadIdx.x + u * S::NT;
            if (idx >= S::WORDS) break;
            buf0[idx] = raw[u] & mask_of(idx / S::PW, idx % S::PW);
            buf1[idx] = 0;
        }
    } else {
        for (int idx = threadIdx.x; idx < S::WORDS; idx += S::NT) {
            const uint32_t m = mask_of(idx / S::PW, idx % S::PW);
            buf0[idx] = m ? *clamped(idx / S::PW, idx % S::PW) & m : 0u;
            buf1[idx] = 0;
        }
    }
    __syncthreads();

    const int w = threadIdx.x % S::W;      // word column of this thread
    const int st = threadIdx.x / S::W;     // strip
    const bool active = st < S::STRIPS;
    const int r0 = st * S::SH;             // first staged row of the strip
    const int32_t gj = j0 - 4 + 4 * w;
    const uint32_t *A = buf0;
    uint32_t *B = buf1;
    for (int g = 0; g < gens; ++g) {
        if (active) {
            auto L = [A](int r, int c) { return A[(r + 1) * S::PW + (c + 1)]; };
            uint32_t hprev = life_hsum3(L(r0 - 1, w - 1), L(r0 - 1, w), L(r0 - 1, w + 1));
            uint32_t hcur = life_hsum3(L(r0, w - 1), L(r0, w), L(r0, w + 1));
            for (int k = 0; k < S::SH; ++k) {
                const int r = r0 + k;
                if (r >= S::R) break;
                const uint32_t hnext = life_hsum3(L(r + 1, w - 1), L(r + 1, w), L(r + 1, w + 1));
                const uint32_t self = L(r, w);
                const uint32_t s9 = hprev + hcur + hnext;
                uint32_t nv = life_zero_bytes(s9 ^ 0x03030303u) |
                              (life_zero_bytes(s9 ^ 0x04040404u) & self);
                nv &= life_window_mask(i0 - K + r, gj, n);  // dead outside the domain
                B[(r + 1) * S::PW + (w + 1)] = nv;
                hprev = hcur;
                hcur = hnext;
            }
        }
        __syncthreads();
        const uint32_t *t = A;
        A = B;
        B = (uint32_t *)t;
    }

    // the tile: staged rows K .. K+TILE-1, words 1 .. TILE/4
    for (int idx = threadIdx.x; idx < TILE * (TILE / 4); idx += S::NT) {
        const int tr = idx / (TILE / 4), tw = idx % (TILE / 4);
        const int32_t gi = i0 + tr, gjw = j0 + 4 * tw;
        const uint32_t v = A[(K + tr + 1) * S::PW + (tw + 2)];
        if (gi < n && gjw + 3 <= gi) {
            *(uint32_t *)(p.nxt + (int64_t)gi * ld + gjw) = v;
        } else if (gi < n && gjw <= gi) {  // the word holding the diagonal cell
            uint8_t *q = p.nxt + (int64_t)gi * ld + gjw;
            for (int b = 0; b <= gi - gjw; ++b) q[b] = (uint8_t)(v >> (8 * b));
        }
    }
}

// ---------------------------------------------------------------------------
// Euclidean distance map, direct FP32: d(i, j) = sqrt(sum_k (x_ik - x_jk)^2)
// for the strict lower triangle, tile (bi, bj) covering rows 1 + bi rho ..
// and columns bj rho .., written to out[i (i - 1) / 2 + j].  Both point blocks
// are staged in LDS dimension-major; each lane accumulates an RB x CB block.
// ---------------------------------------------------------------------------
struct EdmTile {
    int32_t n;
    int32_t d;
    int64_t ldx;
    const float *x;
    float *out;
};

template <int TILE>
struct EdmF32Shape {
    static constexpr int NT = 256;
    static constexpr int TX = 16;                  // lanes along columns
    static constexpr int TY = NT / TX;             // lanes along rows
    static constexpr int RB = TILE / TY;           // register rows per lane (contiguous)
    static constexpr int CB = TILE / TX;           // register columns per lane (stride TX)
    static constexpr int K = TILE >= 64 ? 32 : 64;  // dimensions staged per step
    // row stride of the staged blocks: a multiple of 4 so that a lane's RB
    // consecutive row values are one aligned vector read
    static constexpr int LD = TILE + 4;
    static constexpr int LDS_FLOATS = 2 * K * LD;
    static_assert(RB >= 1 && CB >= 1 && RB * TY == TILE && CB * TX == TILE, "edm tile");
    static_assert(RB == 1 || RB == 2 || RB % 4 == 0, "row block");
};

// RB consecutive floats from LDS (16-byte aligned when RB >= 4).
template <int RB>
__device__ __forceinline__ void lds_read_rows(const float *src, float (&dst)[RB])
{
    if constexpr (RB % 4 == 0) {
        typedef float f4v __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int q = 0; q < RB / 4; ++q) {
            const f4v v = *(const f4v *)(src + 4 * q);
            dst[4 * q + 0] = v.x;
            dst[4 * q + 1] = v.y;
            dst[4 * q + 2] = v.z;
            dst[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int a = 0; a < RB; ++a) dst[a] = src[a];
    }
}

// Distances of one tile of the strict lower triangle: tile (bi, bj) covers
// rows 1 + bi rho .. and columns bj rho ..; d(i, j) = sqrt(sum_k (x_ik -
// x_jk)^2) with FP32 fused multiply-adds in k order, written to the
// condensed out[i (i - 1) / 2 + j] for j < i < n.  Each lane holds an RB x CB
// block: RB consecutive rows (one vector read from LDS per step) against CB
// columns TX apart (so that the 16 lanes of a row store consecutive words).
// STAGE: how a step's coordinates reach LDS.  kEdmStageLoop: a load-store
// loop (the batched kernel, to hold its registers down).  kEdmStageScalar:
// every load of the step issued before the first is stored (clamped
// addresses, masked values), so that their latencies overlap.
// kEdmStageVec4: the same with 16-byte loads at 32-bit byte offsets from the
// base (needs d and ldx multiples of 4, a 16-byte aligned x and
// n * ldx * 4 < 2^31): a quarter of the loads and of their address
// registers.
enum { kEdmStageLoop = 0, kEdmStageScalar = 1, kEdmStageVec4 = 2 };

template <int TILE, int STAGE = kEdmStageScalar>
__device__ __forceinline__ void edm_f32_tile_body(const EdmTile &p, int32_t bi, int32_t bj,
                                                  float *lds)
{
    using S = EdmF32Shape<TILE>;
    float *XI = lds;                  // [K][LD]
    float *XJ = lds + S::K * S::LD;   // [K][LD]
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
        if constexpr (STAGE == kEdmStageVec4) {
            typedef float f4v __attribute__((ext_vector_type(4)));
            constexpr int KQ = S::K / 4;                 // vectors per staged row
            constexpr int PER = TILE * KQ / S::NT;       // vectors per lane and block
            static_assert(PER * S::NT == TILE * KQ, "staging shape");
            const char *xb = (const char *)p.x;
            const int32_t ld32 = (int32_t)ldx;
            f4v vi[PER], vj[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int idx = threadIdx.x + S::NT * u;
                const int row = idx / KQ, kq = idx % KQ;
                const int32_t k = min(k0 + 4 * kq, d - 4);
                const int32_t ri = min(ri0 + row, n - 1), rj = min(cj0 + row, n - 1);
                vi[u] = *(const f4v *)(xb + (uint32_t)((ri * ld32 + k) * 4));
                vj[u] = *(const f4v *)(xb + (uint32_t)((rj * ld32 + k) * 4));
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int idx = threadIdx.x + S::NT * u;
                const int row = idx / KQ, kq = idx % KQ;
                const bool kin = k0 + 4 * kq < d;
                const bool iin = kin && ri0 + row < n, jin = kin && cj0 + row < n;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    XI[(4 * kq + e) * S::LD + row] = iin ? vi[u][e] : 0.f;
                    XJ[(4 * kq + e) * S::LD + row] = jin ? vj[u][e] : 0.f;
                }
            }
        } else if constexpr (STAGE == kEdmStageScalar) {
            constexpr int PER = TILE * S::K / S::NT;  // staged values per lane and block
            static_assert(PER * S::NT == TILE * S::K, "staging shape");
            float vi[PER], vj[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int idx = threadIdx.x + S::NT * u;
                const int row = idx / S::K, kk = idx % S::K;
                const int32_t k = min(k0 + kk, d - 1);
                vi[u] = p.x[(int64_t)min(ri0 + row, n - 1) * ldx + k];
                vj[u] = p.x[(int64_t)min(cj0 + row, n - 1) * ldx + k];
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int idx = threadIdx.x + S::NT * u;
                const int row = idx / S::K, kk = idx % S::K;
                const bool kin = k0 + kk < d;
                XI[kk * S::LD + row] = (ri0 + row < n && kin) ? vi[u] : 0.f;
                XJ[kk * S::LD + row] = (cj0 + row < n && kin) ? vj[u] : 0.f;
            }
        } else {
            for (int idx = threadIdx.x; idx < TILE * S::K; idx += S::NT) {
                const int row = idx / S::K, kk = idx % S::K;
                const int32_t k = k0 + kk;
                const int32_t gi = ri0 + row, gj = cj0 + row;
                XI[kk * S::LD + row] = (gi < n && k < d) ? p.x[(int64_t)gi * ldx + k] : 0.f;
                XJ[kk * S::LD + row] = (gj < n && k < d) ? p.x[(int64_t)gj * ldx + k] : 0.f;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < S::K; ++kk) {
            float xa[S::RB], xb[S::CB];
            lds_read_rows<S::RB>(XI + kk * S::LD + ty * S::RB, xa);
#pragma unroll
            for (int c = 0; c < S::CB; ++c) xb[c] = XJ[kk * S::LD + tx + S::TX * c];
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
        const int32_t i = ri0 + ty * S::RB + a;
        if (i >= n) continue;
        float *orow = p.out + (int64_t)i * (i - 1) / 2;
#pragma unroll
        for (int c = 0; c < S::CB; ++c) {
            const int32_t j = cj0 + tx + S::TX * c;
            if (j < i) __builtin_nontemporal_store(__builtin_sqrtf(acc[a][c]), orow + j);
        }
    }
}

}  // namespace trimap
