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
//
// TRI_EDM_BF16X3 / TRI_EDM_BF16: d^2 = |x_i|^2 + |x_j|^2 - 2 x_i.x_j with the
// Gram term on the matrix cores.  A pre-pass centres the points on their mean
// (distances are translation invariant; centring shrinks the norms and with
// them the cancellation), splits each centred coordinate into a BF16 high
// part and a BF16 low part (hi = bf16(x), lo = bf16(x - hi)), and computes the
// norms from the same rounded operands the matrix cores see.  Each 128 x 128
// output tile is then four waves of 64 x 64, each a 2 x 2 grid of
// v_mfma_f32_32x32x16_bf16 blocks accumulating hi.hi + hi.lo + lo.hi in FP32
// (hi.hi only for TRI_EDM_BF16).  Distances whose Gram-based square falls
// below fixup_thr are recomputed directly in FP32 from the original
// coordinates, which removes the cancellation error for near-duplicates.
// The output write (4 B per pair) bounds this path.
#include "bodies.hpp"
#include "common.hpp"
#include "maps.hpp"

#include <mutex>


namespace trimap {

TileGrid plan_tile_grid(const tri_plan *p);

struct EdmArgs {
    TileGrid g;
    EdmTile t;
};

template <int MAP, int TILE, int STAGE>
__global__ void __launch_bounds__(256) k_edm_f32(EdmArgs p)
{
    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
    __shared__ __attribute__((aligned(16))) float lds[EdmF32Shape<TILE>::LDS_FLOATS];
    edm_f32_tile_body<TILE, STAGE>(p.t, bi, bj, lds);
}

template <int MAP, int STAGE>
static bool edm_f32_tile(const tri_plan *p, const EdmArgs &a, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    switch (p->tile) {
    case 16: k_edm_f32<MAP, 16, STAGE><<<grid, 256, 0, s>>>(a); return true;
    case 32: k_edm_f32<MAP, 32, STAGE><<<grid, 256, 0, s>>>(a); return true;
    case 64: k_edm_f32<MAP, 64, STAGE><<<grid, 256, 0, s>>>(a); return true;
    case 128: k_edm_f32<MAP, 128, STAGE><<<grid, 256, 0, s>>>(a); return true;
    }
    return false;
}

template <int STAGE>
static bool edm_f32_map(const tri_plan *p, const EdmArgs &a, hipStream_t s)
{
    switch (p->map) {
    case TRI_MAP_BB: return edm_f32_tile<MAP_BB, STAGE>(p, a, s);
    case TRI_MAP_RB: return edm_f32_tile<MAP_RB, STAGE>(p, a, s);
    case TRI_MAP_REC: return edm_f32_tile<MAP_REC, STAGE>(p, a, s);
    case TRI_MAP_LAMBDA: return edm_f32_tile<MAP_LAMBDA, STAGE>(p, a, s);
    }
    return false;
}

// 16-byte staging for tiles of 64 and 128 where the coordinates allow it
// (see kEdmStageVec4; measured at n = 65536, d = 128: 12.3 -> 11.4 ms at
// tile 128, where it also lowers the registers from 193 to 126 and so
// doubles the workgroups per CU; at tile 32 it is slower, 18.7 -> 21.4 ms).
static bool edm_f32(const tri_plan *p, const EdmArgs &a, hipStream_t s)
{
    const EdmTile &t = a.t;
    const bool vec4 = p->tile >= 64 && t.d % 4 == 0 && t.ldx % 4 == 0 &&
                      ((uintptr_t)t.x & 15) == 0 &&
                      (uint64_t)t.n * (uint64_t)t.ldx * 4 < (1ull << 31);
    return vec4 ? edm_f32_map<kEdmStageVec4>(p, a, s) : edm_f32_map<kEdmStageScalar>(p, a, s);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kEdmTile = 128;     // output tile of the MFMA kernel
constexpr int kColsumRows = 64;   // rows per block of the column-sum pass

// Workspace of the MFMA modes (all offsets 256-byte aligned).
//
// Up to 128 dimensions (the strip kernel) the BF16 operands are stored in
// MFMA fragment order, in groups of 32 points: for plane q (k-step s and
// part hi / lo: q = s * parts + part; then the norm step as a column
// operand, q = KP = S * parts, and as a row operand, q = KP + 1) and half h
// (dimensions 16 s + 8 h .. + 7), one 16-byte vector per point,
//   frag[((p / 32) * (KP + 2) * 2 + q * 2 + h) * 32 + p % 32],
// so that a wave's 64 lanes (32 points, two halves) read the operand of one
// 32 x 32 x 16 MFMA as 1 KiB of contiguous memory, and all operands of 32
// points form one contiguous block.  The dimensions are padded to S = 2, 4
// or 8 k-steps and the points to np (every row block of the tile grid,
// zeros beyond n).
// Above 128 dimensions the chunked kernel reads row-major hi and lo planes.
struct EdmWs {
    size_t hi, lo, norms, mean, partial, total;
    int64_t dp, nb;
    int64_t np;    // points in the fragment layout (strip kernel), else n
    int32_t S;     // k-steps of the strip kernel, 0: chunked kernel
};

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

constexpr int kStripMaxDims = 128;
// frag vectors per group of 32 points with KP operand planes
__host__ __device__ constexpr int edm_group_vecs(int KP) { return (KP + 2) * 2 * 32; }

static EdmWs edm_ws_layout(int64_t n, int64_t d)
{
    EdmWs w{};
    w.dp = (d + 15) / 16 * 16;
    w.nb = (n + kColsumRows - 1) / kColsumRows;
    size_t o = 0;
    if (w.dp <= kStripMaxDims) {
        const int64_t ks = w.dp / 16;
        w.S = ks <= 2 ? 2 : (ks <= 4 ? 4 : 8);
        w.dp = 16 * w.S;
        // rows of the last tile row reach 1 + 128 m <= n + 128
        w.np = (n + kEdmTile) / kEdmTile * kEdmTile + kEdmTile;
        // fragments: up to 2 S operand planes and two norm-step planes of
        // 32 bytes per point
        w.hi = o;  o = align256(o + (size_t)w.np * (2 * w.S + 2) * 32);
        w.lo = w.hi;
        w.norms = w.hi;
    } else {
        w.S = 0;
        w.np = n;
        w.hi = o;      o = align256(o + (size_t)n * w.dp * 2);
        w.lo = o;      o = align256(o + (size_t)n * w.dp * 2);
        w.norms = o;   o = align256(o + (size_t)n * 4);
    }
    w.mean = o;    o = align256(o + (size_t)w.dp * 4);
    w.partial = o; o = align256(o + (size_t)w.nb * w.dp * 4);
    w.total = o;
    return w;
}

// Column sums of blocks of kColsumRows rows, in row order (deterministic).
__global__ void __launch_bounds__(256) k_edm_colsum(const float *x, int32_t n, int32_t d,
                                                    int64_t ldx, int32_t dp, float *partial)
{
    const int32_t r0 = blockIdx.x * kColsumRows;
    const int32_t r1 = min(n, r0 + kColsumRows);
    for (int32_t k = threadIdx.x; k < dp; k += 256) {
        float s = 0.f;
        if (k < d)
            for (int32_t r = r0; r < r1; ++r) s += x[(int64_t)r * ldx + k];
        partial[(int64_t)blockIdx.x * dp + k] = s;
    }
}

// mean[k] = (sum over blocks of partial[b][k]) / n: one workgroup per
// dimension, a fixed-order strided sum per thread, then a fixed tree.
__global__ void __launch_bounds__(256) k_edm_mean(const float *partial, int32_t nb, int32_t n,
                                                  int32_t dp, float *mean)
{
    __shared__ float red[256];
    const int32_t k = blockIdx.x;
    float s = 0.f;
    for (int32_t b = threadIdx.x; b < nb; b += 256) s += partial[(int64_t)b * dp + k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) mean[k] = red[0] / (float)n;
}

// One wave per point: centre, split into BF16 hi/lo, and the norm of the
// rounded operands, hi.hi + 2 hi.lo (hi.hi only without the split), reduced
// across the wave in a fixed butterfly order.
template <bool SPLIT>
__global__ void __launch_bounds__(64) k_edm_split(const float *x, int32_t d, int64_t ldx,
                                                  int32_t dp, const float *mean, __bf16 *hi,
                                                  __bf16 *lo, float *norms)
{
    const int64_t row = blockIdx.x;
    float acc = 0.f;
    for (int32_t k = threadIdx.x; k < dp; k += 64) {
        float c = 0.f;
        if (k < d) c = x[row * ldx + k] - mean[k];
        const __bf16 h = (__bf16)c;
        const float hf = (float)h;
        const __bf16 l = (__bf16)(c - hf);
        const float lf = (float)l;
        hi[row * dp + k] = h;
        if (SPLIT) {
            lo[row * dp + k] = l;
            acc = __builtin_fmaf(hf, hf, __builtin_fmaf(2.f * hf, lf, acc));
        } else {
            acc = __builtin_fmaf(hf, hf, acc);
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (threadIdx.x == 0) norms[row] = acc;
}

struct EdmMfmaArgs {
    TileGrid g;
    int32_t n, d, dp;
    int64_t ldx;
    const float *x;
    const __bf16 *hi;
    const __bf16 *lo;
    const float *norms;
    float *out;
    float thr;
};

__device__ __forceinline__ float direct_d2(const float *x, int64_t ldx, int32_t d, int32_t i,
                                           int32_t j)
{
    const float *xi = x + (int64_t)i * ldx, *xj = x + (int64_t)j * ldx;
    float s = 0.f;
    // one dimension at a time: the recompute is rare (near pairs only), and
    // more loads in flight here cost the whole kernel registers
#pragma unroll 1
    for (int32_t k = 0; k < d; ++k) {
        const float df = xi[k] - xj[k];
        s = __builtin_fmaf(df, df, s);
    }
    return s;
}

// LDS staging of the operands: the tile's 128 row points and 128 column
// points, kKC dimensions at a time, rows padded so that the 16-byte operand
// reads of eight consecutive rows hit distinct banks.  The next chunk is
// loaded into registers while the matrix cores work on the current one.
constexpr int kKC = 64;                // dimensions per LDS chunk
constexpr int kRS = kKC + 8;           // operand row stride in bf16 (144 bytes)
constexpr int kPlaneBytes = kEdmTile * kRS * 2;
constexpr int kVecPerThread = kEdmTile * kKC / 8 / 256;  // 16-byte vectors per plane

// s_waitcnt immediate that waits until at most n vector memory operations
// of this wave are outstanding (vmcnt(n), 0 <= n <= 63), leaving expcnt and
// lgkmcnt at their maxima (no wait).
constexpr unsigned waitcnt_vm(unsigned n) { return (n & 0xFu) | ((n >> 4) << 14) | 0x0F70u; }

// Workgroup barrier that orders LDS traffic only: wait for this wave's LDS
// operations, then s_barrier.  Unlike __syncthreads() it does not wait for
// outstanding global stores or prefetch loads.  (A global load that feeds
// LDS is waited for by the data dependency of the LDS store.)
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0), vmcnt and expcnt untouched
    __builtin_amdgcn_s_barrier();
}

template <bool SPLIT>
struct EdmStage {
    bf16x8 ha[kVecPerThread], hb[kVecPerThread], la[kVecPerThread], lb[kVecPerThread];
};

template <bool SPLIT>
__device__ __forceinline__ void edm_stage_load(const EdmMfmaArgs &p, int32_t RW, int32_t CW,
                                               int32_t k0, EdmStage<SPLIT> &st, int tid)
{
    const int32_t n = p.n, dp = p.dp;
    const int32_t kn = min(kKC, dp - k0);
#pragma unroll
    for (int u = 0; u < kVecPerThread; ++u) {
        const int v = tid + 256 * u;
        const int row = v / (kKC / 8), c8 = (v % (kKC / 8)) * 8;
        const int32_t ra = min(RW + row, n - 1), rb = min(CW + row, n - 1);
        st.ha[u] = st.hb[u] = st.la[u] = st.lb[u] = bf16x8{};
        if (c8 < kn) {
            st.ha[u] = *(const bf16x8 *)(p.hi + (int64_t)ra * dp + k0 + c8);
            st.hb[u] = *(const bf16x8 *)(p.hi + (int64_t)rb * dp + k0 + c8);
            if (SPLIT) {
                st.la[u] = *(const bf16x8 *)(p.lo + (int64_t)ra * dp + k0 + c8);
                st.lb[u] = *(const bf16x8 *)(p.lo + (int64_t)rb * dp + k0 + c8);
            }
        }
    }
}

template <bool SPLIT>
__device__ __forceinline__ void edm_stage_store(const EdmStage<SPLIT> &st, __bf16 *sAh, __bf16 *sBh,
                                                __bf16 *sAl, __bf16 *sBl, int tid)
{
#pragma unroll
    for (int u = 0; u < kVecPerThread; ++u) {
        const int v = tid + 256 * u;
        const int row = v / (kKC / 8), c8 = (v % (kKC / 8)) * 8;
        *(bf16x8 *)&sAh[row * kRS + c8] = st.ha[u];
        *(bf16x8 *)&sBh[row * kRS + c8] = st.hb[u];
        if (SPLIT) {
            *(bf16x8 *)&sAl[row * kRS + c8] = st.la[u];
            *(bf16x8 *)&sBl[row * kRS + c8] = st.lb[u];
        }
    }
}

// One LDS chunk of the Gram products: kn dimensions (a multiple of 16) of
// the wave's 64 x 64 block as a 2 x 2 grid of 32 x 32 MFMA blocks
// (hi.hi + hi.lo + lo.hi with the split, hi.hi without).
template <bool SPLIT>
__device__ __forceinline__ void edm_mfma_chunk(f32x16 (&acc)[2][2], const __bf16 *sAh,
                                               const __bf16 *sBh, const __bf16 *sAl,
                                               const __bf16 *sBl, int32_t kn, int wr, int wc,
                                               int lr, int lk)
{
    for (int kk = 0; kk < kn; kk += 16) {
        bf16x8 Ah[2], Bh[2], Al[2], Bl[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int ia = (64 * wr + 32 * a + lr) * kRS + kk + lk;
            const int ib = (64 * wc + 32 * a + lr) * kRS + kk + lk;
            Ah[a] = *(const bf16x8 *)&sAh[ia];
            Bh[a] = *(const bf16x8 *)&sBh[ib];
            if (SPLIT) {
                Al[a] = *(const bf16x8 *)&sAl[ia];
                Bl[a] = *(const bf16x8 *)&sBl[ib];
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah[a], Bh[b], acc[a][b], 0, 0, 0);
                if (SPLIT) {
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah[a], Bl[b], acc[a][b], 0, 0, 0);
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al[a], Bh[b], acc[a][b], 0, 0, 0);
                }
            }
    }
}

// Stores a wave's 64 x 64 block of squared distances as distances.  MFMA
// layout of a 32 x 32 block: lane l holds column l % 32 and, in register
// 4 q + u, row 8 q + 4 (l / 32) + u.  ob is the start of row R0 in the
// condensed array and offsets are counted from there in 32 bits.  FULL:
// every pair is in the domain (no per-store test).
template <bool FULL>
__device__ __forceinline__ void edm_store_block(char *ob, const f32x16 (&acc)[2][2], int32_t R0,
                                                int32_t jl, int32_t n, int l)
{
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int32_t i = R0 + 32 * a + 8 * q + 4 * (l >> 5);
            uint32_t off = (uint32_t)((i - R0) * (i + R0 - 1)) / 2u + (uint32_t)jl;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    // the square root of a negative square (rounding) is NaN,
                    // which the max turns into 0
                    const float dd = fmaxf(__builtin_amdgcn_sqrtf(acc[a][b][4 * q + u]), 0.f);
                    if (FULL || (i < n && jl + 32 * b < i))
                        __builtin_nontemporal_store(dd, (float *)(ob + ((off + 32u * b) << 2)));
                }
                off += (uint32_t)i;  // start of row i + 1
                ++i;
            }
        }
}

// The distances of a wave's 64 x 64 block whose first row point is R0 and
// first column point C0 (R0 < n and C0 < R0 + 63: some pair j < i < n
// lies in it), from the Gram block in acc and the tile's norms in sN (rows
// first, then columns).
__device__ __forceinline__ void edm_epilogue(const EdmMfmaArgs &p, f32x16 (&acc)[2][2],
                                             const float *sN, int wr, int wc, int32_t R0,
                                             int32_t C0, int l)
{
    const int lr = l & 31;
    const int32_t n = p.n;
    // d^2 = |x_i|^2 + |x_j|^2 - 2 x_i.x_j, in place
    bool near = false;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 ni = *(const float4 *)&sN[64 * wr + 32 * a + 8 * q + 4 * (l >> 5)];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const float nj = sN[kEdmTile + 64 * wc + 32 * b + lr];
                f32x16 &v = acc[a][b];
                v[4 * q + 0] = __builtin_fmaf(-2.f, v[4 * q + 0], ni.x + nj);
                v[4 * q + 1] = __builtin_fmaf(-2.f, v[4 * q + 1], ni.y + nj);
                v[4 * q + 2] = __builtin_fmaf(-2.f, v[4 * q + 2], ni.z + nj);
                v[4 * q + 3] = __builtin_fmaf(-2.f, v[4 * q + 3], ni.w + nj);
                near |= (v[4 * q + 0] < p.thr) | (v[4 * q + 1] < p.thr) |
                        (v[4 * q + 2] < p.thr) | (v[4 * q + 3] < p.thr);
            }
        }
    // Row i of the condensed array starts at i (i - 1) / 2.  The wave's rows
    // lie within 64 rows of R0, so each offset from the start of row R0 fits
    // in 32 bits and every store takes the one wave-uniform base.
    char *const ob = (char *)(p.out + (uint64_t)R0 * (uint64_t)(R0 - 1) / 2);
    // every pair of the block is in the domain unless it touches the
    // diagonal or the last row
    if ((C0 + 63 < R0) && (R0 + 63 < n))
        edm_store_block<true>(ob, acc, R0, C0 + lr, n, l);
    else
        edm_store_block<false>(ob, acc, R0, C0 + lr, n, l);
    // near-duplicates (rare): recompute those squares directly in FP32 and
    // store them over the values just written (same lane, same address, the
    // same non-temporal policy)
    if (__any(near)) {
        uint64_t m = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (acc[a][b][r] < p.thr) m |= 1ull << (32 * a + 16 * b + r);
        while (m) {
            const int k = __builtin_ctzll(m);
            m &= m - 1;
            const int a = k >> 5, b = (k >> 4) & 1, r = k & 15;
            const int32_t i = R0 + 32 * a + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
            const int32_t j = C0 + 32 * b + lr;
            if (i < n && j < i)
                __builtin_nontemporal_store(
                    __builtin_amdgcn_sqrtf(direct_d2(p.x, p.ldx, p.d, i, j)),
                    (float *)(ob + (((uint32_t)((i - R0) * (i + R0 - 1)) / 2u + (uint32_t)j) << 2)));
        }
    }
}

// Distances of the wave's 64 x 64 block into the tile buffer D (row stride
// kDStride floats, tile coordinates): d^2 from the Gram block and the norms
// as in edm_epilogue, near-duplicates recomputed directly in FP32.
constexpr int kDStride = kEdmTile + 8;  // floats: rows 4 apart fall 32 banks apart

__device__ __forceinline__ void edm_distances_to_lds(const EdmMfmaArgs &p, f32x16 (&acc)[2][2],
                                                     const float *sN, int wr, int wc, int32_t R0,
                                                     int32_t C0, int l, float *D)
{
    const int lr = l & 31;
    const int32_t n = p.n;
    bool near = false;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 ni = *(const float4 *)&sN[64 * wr + 32 * a + 8 * q + 4 * (l >> 5)];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const float nj = sN[kEdmTile + 64 * wc + 32 * b + lr];
                f32x16 &v = acc[a][b];
                v[4 * q + 0] = __builtin_fmaf(-2.f, v[4 * q + 0], ni.x + nj);
                v[4 * q + 1] = __builtin_fmaf(-2.f, v[4 * q + 1], ni.y + nj);
                v[4 * q + 2] = __builtin_fmaf(-2.f, v[4 * q + 2], ni.z + nj);
                v[4 * q + 3] = __builtin_fmaf(-2.f, v[4 * q + 3], ni.w + nj);
                near |= (v[4 * q + 0] < p.thr) | (v[4 * q + 1] < p.thr) |
                        (v[4 * q + 2] < p.thr) | (v[4 * q + 3] < p.thr);
            }
        }
    float *const Dw = D + (64 * wr + 4 * (l >> 5)) * kDStride + 64 * wc + lr;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                Dw[(32 * a + 8 * (r >> 2) + (r & 3)) * kDStride + 32 * b] =
                    fmaxf(__builtin_amdgcn_sqrtf(acc[a][b][r]), 0.f);
    if (__any(near)) {
        uint64_t m = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if (acc[a][b][r] < p.thr) m |= 1ull << (32 * a + 16 * b + r);
        while (m) {
            const int k = __builtin_ctzll(m);
            m &= m - 1;
            const int a = k >> 5, b = (k >> 4) & 1, r = k & 15;
            const int dr = 32 * a + 8 * (r >> 2) + (r & 3);
            const int32_t i = R0 + dr + 4 * (l >> 5);
            const int32_t j = C0 + 32 * b + lr;
            if (i < n && j < i)
                Dw[dr * kDStride + 32 * b] = __builtin_amdgcn_sqrtf(direct_d2(p.x, p.ldx, p.d, i, j));
        }
    }
}

// Stores rows 32 w .. 32 w + 31 of the tile's distances from D (row point RW
// + row, column point CW + column).  A store covers two rows, 32 lanes with
// four consecutive pairs each: a 512-byte run of the condensed array per
// row.  Row i starts at i (i - 1) / 2, any word, hence the 4-byte aligned
// vector type.  The output is written once and not read back here:
// non-temporal stores.
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

__device__ __forceinline__ void edm_store_tile_rows(const EdmMfmaArgs &p, const float *D,
                                                    int32_t RW, int32_t CW, int w, int l)
{
    const int32_t n = p.n;
    const int q = l & 31, hl = l >> 5;
    const int32_t j0 = CW + 4 * q;
#pragma unroll
    for (int r = 0; r < 32; r += 8) {
        f32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            v[k] = *(const f32x4 *)&D[(32 * w + r + 2 * k + hl) * kDStride + 4 * q];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t i = RW + 32 * w + r + 2 * k + hl;
            if (i >= n) continue;
            float *const orow = p.out + (uint64_t)i * (uint64_t)(i - 1) / 2 + j0;
            if (j0 + 3 < i) {
                __builtin_nontemporal_store(v[k], (f32x4u *)orow);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (j0 + e < i) __builtin_nontemporal_store(v[k][e], orow + e);
            }
        }
    }
}

// One workgroup per tile of the plan's grid (every map).
template <int MAP, bool SPLIT>
__global__ void __launch_bounds__(256) k_edm_mfma(EdmMfmaArgs p)
{
    constexpr int PLANES = SPLIT ? 4 : 2;
    // the operand planes, and without the split, after the last product,
    // the tile's distances
    constexpr int kLdsBytes = SPLIT ? PLANES * kPlaneBytes : kEdmTile * kDStride * 4;
    static_assert(kEdmTile * kDStride * 4 >= PLANES * kPlaneBytes || SPLIT, "LDS layout");
    __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
    __shared__ __attribute__((aligned(16))) float sN[2 * kEdmTile];
    __bf16 *sAh = (__bf16 *)lds;
    __bf16 *sBh = (__bf16 *)(lds + kPlaneBytes);
    __bf16 *sAl = (__bf16 *)(lds + 2 * kPlaneBytes);  // split only
    __bf16 *sBl = (__bf16 *)(lds + 3 * kPlaneBytes);

    int32_t bi, bj;
    if (!tile_of_block<MAP>(p.g, bi, bj)) return;
    const int t = threadIdx.x, l = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform
    const int32_t n = p.n, dp = p.dp;
    const int32_t RW = 1 + bi * kEdmTile;  // first row point of the tile
    const int32_t CW = bj * kEdmTile;      // first column point of the tile

    EdmStage<SPLIT> st;
    edm_stage_load<SPLIT>(p, RW, CW, 0, st, t);
    // norms of the tile's row and column points
    {
        const int32_t q = t < kEdmTile ? RW + t : CW + (t - kEdmTile);
        sN[t] = p.norms[min(q, n - 1)];
    }

    const int wr = w >> 1, wc = w & 1;
    const int lr = l & 31, lk = (l >> 5) * 8;
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

    for (int32_t k0 = 0; k0 < dp; k0 += kKC) {
        const int32_t kn = min(kKC, dp - k0);  // multiple of 16
        edm_stage_store<SPLIT>(st, sAh, sBh, sAl, sBl, t);
        lds_barrier();
        if (k0 + kKC < dp) edm_stage_load<SPLIT>(p, RW, CW, k0 + kKC, st, t);  // in flight
        edm_mfma_chunk<SPLIT>(acc, sAh, sBh, sAl, sBl, kn, wr, wc, lr, lk);
        lds_barrier();
    }

    const int32_t R0 = RW + 64 * wr, C0 = CW + 64 * wc;  // this wave's 64 x 64 block
    if constexpr (SPLIT) {
        // each wave stores straight from the MFMA layout and ends
        if (R0 >= n || C0 >= R0 + 63) return;  // no pair j < i < n here (no barrier follows)
        edm_epilogue(p, acc, sN, wr, wc, R0, C0, l);
    } else {
        // distances through LDS (the planes are free after the last barrier),
        // then stored as row runs; a wave with no pair j < i < n in its block
        // only takes part in the barrier and the row stores
        float *const D = (float *)lds;
        if (R0 < n && C0 < R0 + 63) edm_distances_to_lds(p, acc, sN, wr, wc, R0, C0, l, D);
        lds_barrier();
        edm_store_tile_rows(p, D, RW, CW, w, l);
    }
}

template <int MAP>
static void edm_mfma_launch(const tri_plan *p, const EdmMfmaArgs &a, bool split, hipStream_t s)
{
    const dim3 grid(p->gx, p->gy);
    if (split)
        k_edm_mfma<MAP, true><<<grid, 256, 0, s>>>(a);
    else
        k_edm_mfma<MAP, false><<<grid, 256, 0, s>>>(a);
}

static bool edm_mfma(const tri_plan *p, const EdmMfmaArgs &a, bool split, hipStream_t s)
{
    switch (p->map) {
    case TRI_MAP_BB: edm_mfma_launch<MAP_BB>(p, a, split, s); return true;
    case TRI_MAP_RB: edm_mfma_launch<MAP_RB>(p, a, split, s); return true;
    case TRI_MAP_REC: edm_mfma_launch<MAP_REC>(p, a, split, s); return true;
    case TRI_MAP_LAMBDA: edm_mfma_launch<MAP_LAMBDA>(p, a, split, s); return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Line-aligned strip kernel of the MFMA modes (up to 128 dimensions).
//
// A workgroup (four waves) walks G consecutive tiles of the map (a strip,
// see strip_first); wave w owns rows R0 + 32 w .. + 31 of every tile and
// all of its 128 columns (four 32 x 32 MFMA blocks), so the wave's row
// operands stay in registers while the strip stays in one tile row.  The
// tile's column operands (128 points x all k-steps x both planes, 64 KiB at
// 128 dimensions, plus the norm step) are staged in LDS straight from global
// memory for all four waves, in two halves (column blocks 0, 1 and 2, 3):
// each half of the next tile is loaded as soon as every wave has issued its
// products over that half of this tile, so its loads are in flight for about
// one tile.
//
// Stores: the condensed rows start at any word, and a store that covers
// parts of two 128-byte lines costs the memory system about 1.6 times a
// whole-line store (measured).  So every store instruction writes one whole
// aligned line of one row (lanes 0..31; lanes 32..63 the row four below):
// with delta the row's misalignment (in floats) at the tile's first column,
// line k of the row covers the tile's columns 32 k - delta .. 32 k + 31 -
// delta, i.e. the last delta columns of MFMA block k - 1 and the first 32 -
// delta of block k.  Lane l takes block k's column l when l < 32 - delta and
// block k - 1's column l otherwise; the lanes then hold the line's 32
// addresses in another order, and a per-lane select is all the data
// movement.  Block -1 is the previous tile's block 3, carried in registers
// when the previous tile of the strip is the left neighbour; at a strip's
// end a tile stores its own tail.
//
// The norms enter the products through one more k-step (exact products of a
// norm part and one), so the accumulator ends holding -d^2 / 2.
// ---------------------------------------------------------------------------

// Three BF16 parts of a value: v ~ h + m + lo to about 2^-24 relative.
__device__ __forceinline__ void split3(float v, __bf16 &h, __bf16 &m, __bf16 &lo)
{
    h = (__bf16)v;
    const float r1 = v - (float)h;
    m = (__bf16)r1;
    lo = (__bf16)(r1 - (float)m);
}

// Pre-pass in fragment order: one thread per point p < np centres its
// coordinates, splits them into BF16 hi and lo (hi only for single BF16),
// and sums the norm of the rounded operands, hi.hi + 2 hi.lo, in dimension
// order.  It then writes the two planes of the norm step: as a column
// operand (dimensions 0..5: 1, 1, 1 and -n / 2 in three parts) and as a row
// operand (the three parts, then 1, 1, 1); dimensions 8..15 are zero.
// Points beyond n get zeros (their norm steps carry no norm).
template <bool SPLIT, int S>
__global__ void __launch_bounds__(256) k_edm_frag(const float *x, int32_t n, int32_t d,
                                                  int64_t ldx, int32_t np, const float *mean,
                                                  bf16x8 *frag)
{
    constexpr int P = SPLIT ? 2 : 1;
    constexpr int KP = S * P;
    const int32_t p = blockIdx.x * 256 + threadIdx.x;
    if (p >= np) return;
    const bool live = p < n;
    const int64_t grp = (int64_t)(p >> 5) * edm_group_vecs(KP) + (p & 31);
    float acc = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            bf16x8 hv, lv;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int32_t k = 16 * s + 8 * h + e;
                float c = 0.f;
                if (live && k < d) c = x[(int64_t)p * ldx + k] - mean[k];
                const __bf16 hb = (__bf16)c;
                const float hf = (float)hb;
                const __bf16 lb = (__bf16)(c - hf);
                const float lf = (float)lb;
                hv[e] = hb;
                lv[e] = lb;
                if (SPLIT) acc = __builtin_fmaf(hf, hf, __builtin_fmaf(2.f * hf, lf, acc));
                else acc = __builtin_fmaf(hf, hf, acc);
            }
            frag[grp + ((s * P) * 2 + h) * 32] = hv;
            if (SPLIT) frag[grp + ((s * P + 1) * 2 + h) * 32] = lv;
        }
    __bf16 nh, nm, nl;
    split3(-0.5f * acc, nh, nm, nl);
    const __bf16 one = (__bf16)1.f;
    bf16x8 col{}, row{};
    col[0] = one; col[1] = one; col[2] = one; col[3] = nh; col[4] = nm; col[5] = nl;
    row[0] = nh; row[1] = nm; row[2] = nl; row[3] = one; row[4] = one; row[5] = one;
    if (!live) col = row = bf16x8{};
    frag[grp + (KP * 2) * 32] = col;
    frag[grp + (KP * 2 + 1) * 32] = bf16x8{};
    frag[grp + ((KP + 1) * 2) * 32] = row;
    frag[grp + ((KP + 1) * 2 + 1) * 32] = bf16x8{};
}

// The distance from an accumulator holding -d^2 / 2: d^2 = -2 acc exactly.
// A square that rounding made negative (acc > 0) counts as near and is
// recomputed; its magnitude keeps the stored value a number.
__device__ __forceinline__ float dist_of(float acc)
{
    return __builtin_amdgcn_sqrtf(2.f * __builtin_fabsf(acc));
}

struct EdmLinesArgs {
    TileGrid g;
    StripGrid sg;
    int32_t n, d;
    int64_t ldx;
    const float *x;
    const bf16x8 *frag;
    float *out;
    float thr;  // fix-up threshold on d^2
};

template <int MAP, bool SPLIT, int S>
__global__ void __launch_bounds__(256, 2) k_edm_lines(EdmLinesArgs a)
{
    constexpr int P = SPLIT ? 2 : 1;
    constexpr int KP = S * P;                   // operand planes (k-step, hi / lo)
    constexpr int kGroup = edm_group_vecs(KP);  // frag vectors per group of 32 points
    // column operands of the tile, one array per half (blocks 2 h, 2 h + 1):
    // 16-byte vector (plane p, block 2 h + e, lane) at (p 2 + e) 64 + lane,
    // plane KP the norm step
    __shared__ bf16x8 sB0[(KP + 1) * 2 * 64];
    __shared__ bf16x8 sB1[(KP + 1) * 2 * 64];

    const int t = threadIdx.x, l = t & 63, lo = l & 31, hf = l >> 5;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int32_t n = a.n;
    const float nthr = -0.5f * a.thr;  // near: acc > -thr / 2, i.e. d^2 < thr
    // misalignment of the output array within a 128-byte line, in floats
    const uint32_t amod = (uint32_t)(((uintptr_t)a.out >> 2) & 31u);

    const uint32_t first = strip_first<MAP>(a.g, a.sg);
    int32_t bi, bj;
    int k = strip_next<MAP>(a.g, a.sg, first, 0, bi, bj);
    if (k >= a.sg.G) return;  // the whole strip maps to no tile (uniform)
    bi = __builtin_amdgcn_readfirstlane(bi);
    bj = __builtin_amdgcn_readfirstlane(bj);

    // the wave's row operands: row R0 + 32 w + (l & 31), half l >> 5, and
    // its norm step
    bf16x8 A[S][P];
    bf16x8 Ax;
    auto load_rows = [&](int32_t rbi) {
        const int32_t r0 = 1 + rbi * kEdmTile + 32 * w + lo;
        const bf16x8 *rowp = a.frag + (int64_t)(r0 >> 5) * kGroup + hf * 32 + (r0 & 31);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int pl = 0; pl < P; ++pl) A[s][pl] = rowp[(s * P + pl) * 64];
        Ax = rowp[(KP + 1) * 64];
    };
    // one half of a tile's column operands into LDS, with no register in
    // between: each plane of 32 points is 1 KiB of contiguous frag, one
    // 16-byte load per lane landing in lane order.  Wave w loads block
    // 2 h + (w & 1), the planes of parity w >> 1.
    auto stage_half = [&](bf16x8 *dst, int32_t cbj, int h) {
        const int e = w & 1;
        const bf16x8 *src = a.frag + (int64_t)(4 * cbj + 2 * h + e) * kGroup + l;
#pragma unroll
        for (int q = 0; q < (KP + 2) / 2; ++q) {
            const int p = 2 * q + (w >> 1);
            if (p <= KP)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(src + p * 64),
                    (__attribute__((address_space(3))) void *)(dst + (p * 2 + e) * 64), 16, 0, 0);
        }
    };

    // The store geometry of a tile row, the same for all its tiles (their
    // first columns are multiples of 32 floats): for the row i of register r
    // (this lane's half), bit r of wbits is set when this lane takes the
    // block to the left in every line of the row (lane >= 32 - delta, delta
    // the row's misalignment), and offw[r] = 4 (rowoff(i) + lane - 32 wrap),
    // with rowoff(i) the offset of (i, 0) from row R0's start.  Line k of the
    // tile at column CW then sits at orow + 4 CW + offw + 128 k.
    uint32_t offw[16];
    uint32_t wbits = 0;
    char *orow = nullptr;
    int32_t R0 = 0;
    auto set_rows = [&](int32_t rbi) {
        R0 = 1 + rbi * kEdmTile;
        const uint64_t TR0 = (uint64_t)R0 * (uint64_t)(R0 - 1) / 2;
        orow = (char *)(a.out + TR0);
        const uint32_t rmod = (uint32_t)(TR0 & 31u) + amod;
        wbits = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int32_t i = R0 + 32 * w + 8 * (r >> 2) + 4 * hf + (r & 3);
            const uint32_t ro = (uint32_t)((i - R0) * (i + R0 - 1)) / 2u;
            const uint32_t wrap = (uint32_t)(lo + (int32_t)((ro + rmod) & 31u) >= 32);
            offw[r] = (ro + (uint32_t)lo - 32u * wrap) << 2;
            wbits |= wrap << r;
        }
    };

    load_rows(bi);
    stage_half(sB0, bj, 0);
    stage_half(sB1, bj, 1);
    set_rows(bi);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));

    f32x16 carry{};           // distances of the previous tile's block 3
    uint32_t carry_near = 0;  // which of them are near (bit r)
    bool carry_ok = false;    // the previous tile of the strip is the left neighbour
    // Stores of whole lines are deferred into the next pass's products, a few
    // per k-step, so that every wave writes while its products run: V0, V1
    // hold two lines of the 16 rows, stored at vbase + offw + k0 / k1.
    f32x16 V0{}, V1{};
    bool vpend = false;       // V0, V1 hold lines 2, 3 of the previous tile
    char *vbase = nullptr;
    bool pfull = false;       // the previous tile was full and waited for nothing
    bool pcok = false;        // ... and deferred its line 0
    for (;;) {
        int32_t nbi = 0, nbj = 0;
        const int nk = strip_next<MAP>(a.g, a.sg, first, k + 1, nbi, nbj);
        const bool more = nk < a.sg.G;
        nbi = __builtin_amdgcn_readfirstlane(nbi);
        nbj = __builtin_amdgcn_readfirstlane(nbj);

        const int32_t CW = bj * kEdmTile;
        char *const obt = orow + 4 * (int64_t)CW;  // the tile's row R0, column 0
        // store of line k (byte offset 128 k) of the row of register r
        auto st = [&](int r, uint32_t k128, float v) {
            __builtin_nontemporal_store(v, (float *)((obt + offw[r]) + k128));
        };
        const bool tail_self = !(more && nbi == bi && nbj == bj + 1);
        const bool full = CW + kEdmTile - 1 < R0 && R0 + kEdmTile - 1 < n;
        // per-lane test of pair (row of register r, tile column jt), for
        // tiles that cross the diagonal or the last row
        auto inside = [&](int r, int32_t jt) {
            const int32_t i = R0 + 32 * w + 8 * (r >> 2) + 4 * hf + (r & 3);
            return i < n && CW + jt >= 0 && CW + jt < i;
        };

        f32x16 mid{};          // distances of block 1 (line 2 takes its tail)
        uint64_t near = 0;     // bit c 16 + r: the square is below the threshold
        bool waited = false;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            bf16x8 *const sB = pass ? sB1 : sB0;
            // This half's loads are complete in every wave.  They were issued
            // a half tile ago; younger, when the previous tile was full: its
            // 16 line 1 stores (and 16 of line 0 when deferred) and KP / 2
            // loads of the other half (the first half), or its 32 stores of
            // lines 2 and 3 (the second half).
            if (pass == 0) {
                if (pfull && pcok) __builtin_amdgcn_s_waitcnt(waitcnt_vm(32 + KP / 2));
                else if (pfull) __builtin_amdgcn_s_waitcnt(waitcnt_vm(16 + KP / 2));
                else __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
            } else {
                if (pfull) __builtin_amdgcn_s_waitcnt(waitcnt_vm(32));
                else __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
            }
            lds_barrier();
            // the deferred lines stored during this pass: lines 2, 3 of the
            // previous tile (pass 0) or lines 0 (when the carry is there)
            // and 1 of this tile (pass 1)
            const bool sv = pass ? full : vpend;
            const bool sv0 = pass ? (full && carry_ok) : vpend;
            char *const sbase = pass ? obt : vbase;
            const uint32_t k0 = pass ? 0u : 256u, k1 = pass ? 128u : 384u;
            // acc[e] = rows x column block 2 pass + e.  The column operands of
            // k-step s are read from LDS kPf k-steps ahead of their products,
            // so that the reads' latency hides behind the products in flight.
            constexpr int kPf = SPLIT ? 1 : 4;
            constexpr int kRows = 16 / S;  // deferred rows stored per k-step
            bf16x8 Bh[S][2], Bl[S][2];
            auto read_b = [&](int s) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    Bh[s][e] = sB[((s * P) * 2 + e) * 64 + l];
                    if constexpr (SPLIT) Bl[s][e] = sB[((s * P + 1) * 2 + e) * 64 + l];
                }
            };
            f32x16 acc[2];
            {
                const bf16x8 X0 = sB[(KP * 2) * 64 + l], X1 = sB[(KP * 2 + 1) * 64 + l];
#pragma unroll
                for (int s = 0; s < kPf && s < S; ++s) read_b(s);
                __builtin_amdgcn_sched_barrier(0);
                const f32x16 z{};
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ax, X0, z, 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ax, X1, z, 0, 0, 0);
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (s + kPf < S) read_b(s + kPf);
                if (sv) {
#pragma unroll
                    for (int q = 0; q < kRows; ++q) {
                        const int r = s * kRows + q;
                        if (sv0) __builtin_nontemporal_store(V0[r], (float *)((sbase + offw[r]) + k0));
                        __builtin_nontemporal_store(V1[r], (float *)((sbase + offw[r]) + k1));
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int e = 0; e < 2; ++e)
                    acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][0], Bh[s][e], acc[e], 0, 0, 0);
                if constexpr (SPLIT) {
#pragma unroll
                    for (int e = 0; e < 2; ++e)
                        acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][0], Bl[s][e], acc[e], 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 2; ++e)
                        acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][P - 1], Bh[s][e], acc[e], 0, 0, 0);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            // every wave's products over this half are issued (their LDS
            // reads done): the next tile's half may overwrite it
            lds_barrier();
            if (more) {
                if (pass == 0) stage_half(sB0, nbj, 0);
                else stage_half(sB1, nbj, 1);
            }
            {
                float mx = acc[0][0];
#pragma unroll
                for (int e = 0; e < 2; ++e)
#pragma unroll
                    for (int r = 0; r < 16; ++r) mx = fmaxf(mx, acc[e][r]);
                if (__any(mx > nthr)) {  // rare: which squares (bit c 16 + r)
                    // shifted in one at a time: no per-bit constant is held
                    uint32_t m = 0;
#pragma unroll
                    for (int e = 1; e >= 0; --e)
#pragma unroll
                        for (int r = 15; r >= 0; --r) m = (m << 1) | (uint32_t)(acc[e][r] > nthr);
                    near |= (uint64_t)m << (32 * pass);
                }
            }
            f32x16 D[2];
#pragma unroll
            for (int e = 0; e < 2; ++e)
#pragma unroll
                for (int r = 0; r < 16; ++r) D[e][r] = dist_of(acc[e][r]);

            if (pass == 0) {
                // line 0 (the carry's tail and block 0) and line 1 (blocks 0,
                // 1): deferred in a full tile (line 0 stored now when there is
                // no carry, by the lanes that do not take it)
                if (full) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const bool wrap = (wbits >> r) & 1u;
                        V0[r] = wrap ? carry[r] : D[0][r];
                        V1[r] = wrap ? D[0][r] : D[1][r];
                    }
                    if (!carry_ok) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            if (!((wbits >> r) & 1u)) st(r, 0u, V0[r]);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const bool wrap = (wbits >> r) & 1u;
                        const int32_t jt = lo - 32 * (int32_t)wrap;
                        if ((carry_ok || !wrap) && inside(r, jt)) st(r, 0u, wrap ? carry[r] : D[0][r]);
                        if (inside(r, jt + 32)) st(r, 128u, wrap ? D[0][r] : D[1][r]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                mid = D[1];
                __builtin_amdgcn_sched_barrier(0);
            } else {
                // line 4: the tile's own tail (block 3, columns 128 - delta ..)
                if (tail_self) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        if (((wbits >> r) & 1u) && (full || inside(r, 96 + lo))) st(r, 512u, D[1][r]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                if (more && nbi != bi) {
                    // a new tile row (once a strip, or where it crosses a row
                    // end): wait for its row operands here, so that the
                    // products never wait for a store
                    load_rows(nbi);
                    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                }
                // the stores below stay after these loads (the waits for the
                // loads count them)
                asm volatile("" ::: "memory");
                const bool anynear = __any((near | (carry_ok ? carry_near : 0u)) != 0);
                // lines 2 (blocks 1, 2) and 3 (blocks 2, 3): deferred into the
                // next tile's first pass when it continues this tile row and
                // no near square waits for its fix-up
                const bool defer = full && more && nbi == bi && !anynear;
                if (full) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const bool wrap = (wbits >> r) & 1u;
                        V0[r] = wrap ? mid[r] : D[0][r];
                        V1[r] = wrap ? D[0][r] : D[1][r];
                    }
                    if (!defer) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            st(r, 256u, V0[r]);
                            st(r, 384u, V1[r]);
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const bool wrap = (wbits >> r) & 1u;
                        const int32_t jt = lo - 32 * (int32_t)wrap;
                        if (inside(r, jt + 64)) st(r, 256u, wrap ? mid[r] : D[0][r]);
                        if (inside(r, jt + 96)) st(r, 384u, wrap ? D[0][r] : D[1][r]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                vpend = defer;
                vbase = obt;
                // near-duplicates (rare): recompute directly in FP32 over the
                // values just stored, the carried ones included
                if (anynear) {
                    // bits 0..63: this tile's squares; then the carried ones
                    uint64_t mk = near;
                    uint32_t mc = carry_ok ? carry_near : 0u;
                    while (mk | mc) {
                        int r, jt;
                        if (mk) {
                            const int b = __builtin_ctzll(mk);
                            mk &= mk - 1;
                            r = b & 15;
                            jt = 32 * (b >> 4) + lo;
                            // block 3's tail goes to the next tile unless this tile stores it
                            if ((b >> 4) == 3 && ((wbits >> r) & 1u) && !tail_self) continue;
                        } else {
                            r = __builtin_ctz(mc);
                            mc &= mc - 1;
                            if (!((wbits >> r) & 1u)) continue;  // not a carried value
                            jt = lo - 32;
                        }
                        if (!inside(r, jt)) continue;
                        const int32_t i = R0 + 32 * w + 8 * (r >> 2) + 4 * hf + (r & 3);
                        const uint32_t ro = (uint32_t)((i - R0) * (i + R0 - 1)) / 2u;
                        *(float *)(obt + 4u * (ro + (uint32_t)jt)) =
                            __builtin_amdgcn_sqrtf(direct_d2(a.x, a.ldx, a.d, i, CW + jt));
                    }
                    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                    waited = true;
                }
                carry = D[1];
            }
        }
        // the carry for the next tile (block 3's distances, set above)
        carry_near = (uint32_t)(near >> 48);
        // a wait in this tile (fix-up) completed everything; else the next
        // tile counts this tile's unconditional stores
        pfull = full && !waited;
        pcok = carry_ok;
        carry_ok = !tail_self;
        if (!more) break;
        if (nbi != bi) set_rows(nbi);
        k = nk;
        bi = nbi;
        bj = nbj;
    }
}

// ---------------------------------------------------------------------------
// Pipelined strip kernel of the MFMA modes (up to 128 dimensions): one
// workgroup of four waves per CU.
//
// The tiles, operands and line-aligned stores are those of k_edm_lines, with
// three differences.  The column operands of two tiles sit in LDS (2 x 68
// KiB at 128 dimensions): the next tile's are loaded while this tile's
// products run, with one barrier per tile.  A wave computes all four column
// blocks of a tile at once (64 accumulators).  And the distances, selects
// and stores of the previous tile (when it is this tile's left neighbour and
// lies wholly in the domain, the usual case along a strip) are interleaved
// with this tile's products in one instruction stream, a few rows per
// k-step, so that the vector ALU and the stores work in the shadow of the
// matrix cores (one wave per SIMD: nothing else would fill it).  Other
// tiles (first of a strip, last of a strip, diagonal or last-row tiles) take
// the same steps one after the other.
//
// Near pairs: d = sqrt(max(-2 acc, 0)) below sqrt(thr) (a square that
// rounding made negative gives 0) are recomputed directly in FP32 after the
// tile's stores.
// ---------------------------------------------------------------------------
template <int MAP, bool SPLIT, int S>
__global__ void __launch_bounds__(256, 1) k_edm_pipe(EdmLinesArgs a)
{
    constexpr int P = SPLIT ? 2 : 1;
    constexpr int KP = S * P;                   // operand planes (k-step, hi / lo)
    constexpr int kGroup = edm_group_vecs(KP);  // frag vectors per group of 32 points
    constexpr int kBuf = (KP + 1) * 4 * 64;     // vectors of one tile's column operands
    constexpr int RPS = 16 / S;                 // rows of the previous tile per k-step
    // column operands of two tiles: vector (plane p, block c, lane) of
    // buffer b at b kBuf + (p 4 + c) 64 + lane, plane KP the norm step
    __shared__ bf16x8 sB[2 * kBuf];

    const int t = threadIdx.x, l = t & 63, lo = l & 31, hf = l >> 5;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int32_t n = a.n;
    const float sthr = __builtin_sqrtf(a.thr);  // near: d < sqrt(thr)
    // misalignment of the output array within a 128-byte line, in floats
    const uint32_t amod = (uint32_t)(((uintptr_t)a.out >> 2) & 31u);

    const uint32_t first = strip_first<MAP>(a.g, a.sg);
    int32_t bi, bj;
    int k = strip_next<MAP>(a.g, a.sg, first, 0, bi, bj);
    if (k >= a.sg.G) return;  // the whole strip maps to no tile (uniform)
    bi = __builtin_amdgcn_readfirstlane(bi);
    bj = __builtin_amdgcn_readfirstlane(bj);

    // the wave's row operands: row R0 + 32 w + (l & 31), half l >> 5, and
    // its norm step
    bf16x8 A[S][P];
    bf16x8 Ax;
    auto load_rows = [&](int32_t rbi) {
        const int32_t r0 = 1 + rbi * kEdmTile + 32 * w + lo;
        const bf16x8 *rowp = a.frag + (int64_t)(r0 >> 5) * kGroup + hf * 32 + (r0 & 31);
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int pl = 0; pl < P; ++pl) A[s][pl] = rowp[(s * P + pl) * 64];
        Ax = rowp[(KP + 1) * 64];
    };
    // a tile's column operands into buffer b: wave w loads block w, every
    // plane (1 KiB of contiguous frag each, one 16-byte load per lane)
    auto stage = [&](int b, int32_t cbj) {
        const bf16x8 *src = a.frag + (int64_t)(4 * cbj + w) * kGroup + l;
#pragma unroll
        for (int p = 0; p <= KP; ++p)
            __builtin_amdgcn_global_load_lds(
                (const __attribute__((address_space(1))) void *)(src + p * 64),
                (__attribute__((address_space(3))) void *)(sB + b * kBuf + (p * 4 + w) * 64), 16, 0,
                0);
    };

    // store geometry of a tile row, as in k_edm_lines
    uint32_t offw[16];
    uint32_t wbits = 0;
    char *orow = nullptr;
    int32_t R0 = 0;
    auto set_rows = [&](int32_t rbi) {
        R0 = 1 + rbi * kEdmTile;
        const uint64_t TR0 = (uint64_t)R0 * (uint64_t)(R0 - 1) / 2;
        orow = (char *)(a.out + TR0);
        const uint32_t rmod = (uint32_t)(TR0 & 31u) + amod;
        wbits = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int32_t i = R0 + 32 * w + 8 * (r >> 2) + 4 * hf + (r & 3);
            const uint32_t ro = (uint32_t)((i - R0) * (i + R0 - 1)) / 2u;
            const uint32_t wrap = (uint32_t)(lo + (int32_t)((ro + rmod) & 31u) >= 32);
            offw[r] = (ro + (uint32_t)lo - 32u * wrap) << 2;
            wbits |= wrap << r;
        }
    };
    auto dist = [](float acc) { return __builtin_amdgcn_sqrtf(fmaxf(-2.f * acc, 0.f)); };

    // products of one k-step (or the norm step) into acc[0..3]
    auto ext_step = [&](f32x16 (&acc)[4], int b) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const f32x16 z{};
            acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ax, sB[b * kBuf + (KP * 4 + e) * 64 + l],
                                                             z, 0, 0, 0);
        }
    };

    load_rows(bi);
    set_rows(bi);
    stage(0, bj);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
    lds_barrier();

    f32x16 carry{};           // distances of the previous tile's block 3
    uint32_t carry_near = 0;  // which of them are near (bit r)
    bool carry_ok = false;    // carry holds the left neighbour's block 3
    f32x16 accP[4];           // a deferred tile's accumulators (its left neighbour's
    bool pend = false;        // epilogue runs in this tile's products)
    int buf = 0;

    // Epilogue of a tile from its accumulators, step by step (any tile):
    // distances, stores (lines 0..3, line 4 when it ends its strip's run),
    // near-pair recompute; leaves block 3 in carry and its near bits in
    // carry_near.
    auto epilogue = [&](f32x16 (&acc)[4], char *obt, int32_t CW, bool full, bool c_ok,
                        bool tail_self) {
        auto st = [&](int r, uint32_t k128, float v) {
            __builtin_nontemporal_store(v, (float *)((obt + offw[r]) + k128));
        };
        auto inside = [&](int r, int32_t jt) {
            const int32_t i = R0 + 32 * w + 8 * (r >> 2) + 4 * hf + (r & 3);
            return i < n && CW + jt >= 0 && CW + jt < i;
        };
        float mn = 3.4e38f;
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                acc[e][r] = dist(acc[e][r]);
                mn = fminf(mn, acc[e][r]);
            }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const bool wrap = (wbits >> r) & 1u;
            const float L0 = wrap ? carry[r] : acc[0][r], L1 = wrap ? acc[0][r] : acc[1][r];
            const float L2 = wrap ? acc[1][r] : acc[2][r], L3 = wrap ? acc[2][r] : acc[3][r];
            if (full) {
                if (c_ok || !wrap) st(r, 0u, L0);
                st(r, 128u, L1);
                st(r, 256u, L2);
                st(r, 384u, L3);
                if (tail_self && wrap) st(r, 512u, acc[3][r]);
            } else {
                const int32_t jt = lo - 32 * (int32_t)wrap;
                if ((c_ok || !wrap) && inside(r, jt)) st(r, 0u, L0);
                if (inside(r, jt + 32)) st(r, 128u, L1);
                if (inside(r, jt + 64)) st(r, 256u, L2);
                if (inside(r, jt + 96)) st(r, 384u, L3);
                if (tail_self && wrap && inside(r, 96 + lo)) st(r, 512u, acc[3][r]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        const uint32_t cn = c_ok ? carry_near : 0u;
        carry_near = 0;
        if (__any(mn < sthr || cn != 0u)) {
            // rare: which squares are near (bit e 16 + r), then recompute
            // them directly in FP32 over the values just stored
            uint64_t mk = 0;
#pragma unroll
            for (int e = 3; e >= 0; --e)
#pragma unroll
                for (int r = 15; r >= 0; --r) mk = (mk << 1) | (uint64_t)(acc[e][r] < sthr);
            carry_near = (uint32_t)(mk >> 48);
            uint32_t mc = cn;
            while (mk | mc) {
                int r, jt;
                if (mk) {
                    const int b = __builtin_ctzll(mk);
                    mk &= mk - 1;
                    r = b & 15;
                    jt = 32 * (b >> 4) + lo;
                    // block 3's tail goes to the next tile unless this tile stores it
                    if ((b >> 4) == 3 && ((wbits >> r) & 1u) && !tail_self) continue;
                } else {
                    r = __builtin_ctz(mc);
                    mc &= mc - 1;
                    if (!((wbits >> r) & 1u)) continue;  // not a carried value
                    jt = lo - 32;
                }
                if (!inside(r, jt)) continue;
                const int32_t i = R0 + 32 * w + 8 * (r >> 2) + 4 * hf + (r & 3);
                const uint32_t ro = (uint32_t)((i - R0) * (i + R0 - 1)) / 2u;
                *(float *)(obt + 4u * (ro + (uint32_t)jt)) =
                    __builtin_amdgcn_sqrtf(direct_d2(a.x, a.ldx, a.d, i, CW + jt));
            }
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        }
        carry = acc[3];
    };

    for (;;) {
        int32_t nbi = 0, nbj = 0;
        const int nk = strip_next<MAP>(a.g, a.sg, first, k + 1, nbi, nbj);
        const bool more = nk < a.sg.G;
        nbi = __builtin_amdgcn_readfirstlane(nbi);
        nbj = __builtin_amdgcn_readfirstlane(nbj);
        const bool right = more && nbi == bi && nbj == bj + 1;  // the next tile continues the row

        const int32_t CW = bj * kEdmTile;
        char *const obt = orow + 4 * (int64_t)CW;  // the tile's row R0, column 0
        const bool full = CW + kEdmTile - 1 < R0 && R0 + kEdmTile - 1 < n;

        // the next tile's columns into the other buffer (every wave is done
        // with it: the barrier at the end of the previous tile)
        if (more) stage(buf ^ 1, nbj);

        f32x16 acc[4];
        bool fused = false;
        if (pend) {
            // this tile's products with the left neighbour's epilogue (a
            // full tile with its carry; its stores go to obt - 512)
            fused = true;
            char *const pobt = obt - 512;
            float mn = 3.4e38f;
            bf16x8 B[2][P][4];  // [slot][part of the k-step][block]
            auto read_b = [&](int s, int slot) {
#pragma unroll
                for (int pl = 0; pl < P; ++pl)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        B[slot][pl][e] = sB[buf * kBuf + ((s * P + pl) * 4 + e) * 64 + l];
            };
            read_b(0, 0);
            ext_step(acc, buf);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int sl = s & 1;
                if (s + 1 < S) read_b(s + 1, sl ^ 1);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][0], B[sl][0][e], acc[e], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                // distances of this step's rows of the previous tile
#pragma unroll
                for (int q = 0; q < RPS; ++q) {
                    const int r = s * RPS + q;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        accP[e][r] = dist(accP[e][r]);
                        mn = fminf(mn, accP[e][r]);
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (SPLIT) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][0], B[sl][1][e], acc[e], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                }
                // their four lines
#pragma unroll
                for (int q = 0; q < RPS; ++q) {
                    const int r = s * RPS + q;
                    const bool wrap = (wbits >> r) & 1u;
                    char *const rp = pobt + offw[r];
                    __builtin_nontemporal_store(wrap ? carry[r] : accP[0][r], (float *)(rp + 0u));
                    __builtin_nontemporal_store(wrap ? accP[0][r] : accP[1][r], (float *)(rp + 128u));
                    __builtin_nontemporal_store(wrap ? accP[1][r] : accP[2][r], (float *)(rp + 256u));
                    __builtin_nontemporal_store(wrap ? accP[2][r] : accP[3][r], (float *)(rp + 384u));
                }
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (SPLIT) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][P - 1], B[sl][0][e], acc[e], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // near pairs of the previous tile (rare), after its stores
            const uint32_t cn = carry_near;
            carry_near = 0;
            if (__any(mn < sthr || cn != 0u)) {
                uint64_t mk = 0;
#pragma unroll
                for (int e = 3; e >= 0; --e)
#pragma unroll
                    for (int r = 15; r >= 0; --r) mk = (mk << 1) | (uint64_t)(accP[e][r] < sthr);
                carry_near = (uint32_t)(mk >> 48);
                uint32_t mc = cn;
                const int32_t PCW = CW - kEdmTile;
                while (mk | mc) {
                    int r, jt;
                    if (mk) {
                        const int b = __builtin_ctzll(mk);
                        mk &= mk - 1;
                        r = b & 15;
                        jt = 32 * (b >> 4) + lo;
                        if ((b >> 4) == 3 && ((wbits >> r) & 1u)) continue;  // carried on
                    } else {
                        r = __builtin_ctz(mc);
                        mc &= mc - 1;
                        if (!((wbits >> r) & 1u)) continue;
                        jt = lo - 32;
                    }
                    const int32_t i = R0 + 32 * w + 8 * (r >> 2) + 4 * hf + (r & 3);
                    const uint32_t ro = (uint32_t)((i - R0) * (i + R0 - 1)) / 2u;
                    *(float *)(pobt + 4u * (ro + (uint32_t)jt)) =
                        __builtin_amdgcn_sqrtf(direct_d2(a.x, a.ldx, a.d, i, PCW + jt));
                }
                __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
                fused = false;  // the wait drained the stores: count no younger operations
            }
            carry = accP[3];
        } else {
            ext_step(acc, buf);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                bf16x8 Bh[4], Bl[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    Bh[e] = sB[buf * kBuf + ((s * P) * 4 + e) * 64 + l];
                    if constexpr (SPLIT) Bl[e] = sB[buf * kBuf + ((s * P + 1) * 4 + e) * 64 + l];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][0], Bh[e], acc[e], 0, 0, 0);
                if constexpr (SPLIT) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][0], Bl[e], acc[e], 0, 0, 0);
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[e] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A[s][P - 1], Bh[e], acc[e], 0, 0, 0);
                }
            }
        }
        // this tile: deferred to the next tile's products when that tile
        // continues the row and this one is full with its carry; else now
        const bool defer = right && full && carry_ok;
        bool waited = false;
        if (defer) {
#pragma unroll
            for (int e = 0; e < 4; ++e) accP[e] = acc[e];
        } else {
            epilogue(acc, obt, CW, full, carry_ok, !right);
            waited = true;  // counted as such below (stores of any number)
        }
        pend = defer;
        carry_ok = right;
        if (!more) break;

        // The next tile's columns are complete in every wave, and every
        // wave is done with this tile's buffer.  A fused tile issued its 64
        // stores after those loads (so at most 63 younger operations may
        // remain); otherwise wait for everything.
        if (fused && !waited) __builtin_amdgcn_s_waitcnt(waitcnt_vm(63));
        else __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        lds_barrier();
        if (nbi != bi) {
            load_rows(nbi);
            set_rows(nbi);
            __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
        }
        k = nk;
        bi = nbi;
        bj = nbj;
        buf ^= 1;
    }
}

// Workgroups that share a group of strips (1: each workgroup's tiles are
// consecutive, so the carry passes from tile to tile).
constexpr int32_t kEdmStripGroup = 1;

// Tiles per strip: the plan's TRI_FLAG_STRIP, else enough strips for
// several rounds of the GPU's workgroup slots and strips long enough that the
// row operands loaded into registers serve several tiles.
static int32_t strip_len(const tri_plan *p)
{
    if (const int32_t f = strip_flag_len(p->flags)) return f;
    const uint64_t g = (uint64_t)p->T / 8192;
    return (int32_t)(g < 1 ? 1 : (g > 8 ? 8 : g));
}

template <int MAP, bool SPLIT, int S>
static void edm_lines_launch(const tri_plan *p, const EdmLinesArgs &a0, hipStream_t s)
{
    EdmLinesArgs a = a0;
    dim3 grid;
    a.sg = strip_grid(MAP, a.g.m, a.g.flags, a.g.T, p->gx, p->gy, strip_len(p), kEdmStripGroup, grid);
    if (p->flags & TRI_FLAG_EDM_PIPE)
        k_edm_pipe<MAP, SPLIT, S><<<grid, 256, 0, s>>>(a);
    else
        k_edm_lines<MAP, SPLIT, S><<<grid, 256, 0, s>>>(a);
}

template <bool SPLIT, int S>
static bool edm_lines_map(const tri_plan *p, const EdmLinesArgs &a, hipStream_t s)
{
    switch (p->map) {
    case TRI_MAP_BB: edm_lines_launch<MAP_BB, SPLIT, S>(p, a, s); return true;
    case TRI_MAP_RB: edm_lines_launch<MAP_RB, SPLIT, S>(p, a, s); return true;
    case TRI_MAP_REC: edm_lines_launch<MAP_REC, SPLIT, S>(p, a, s); return true;
    case TRI_MAP_LAMBDA: edm_lines_launch<MAP_LAMBDA, SPLIT, S>(p, a, s); return true;
    }
    return false;
}

template <bool SPLIT>
static bool edm_lines(const tri_plan *p, const EdmLinesArgs &a, int S, hipStream_t s)
{
    switch (S) {
    case 2: return edm_lines_map<SPLIT, 2>(p, a, s);
    case 4: return edm_lines_map<SPLIT, 4>(p, a, s);
    case 8: return edm_lines_map<SPLIT, 8>(p, a, s);
    }
    return false;
}

template <bool SPLIT>
static void edm_frag_launch(int S, const float *x, int32_t n, int32_t d, int64_t ldx, int32_t np,
                            const float *mean, bf16x8 *frag, hipStream_t s)
{
    const dim3 grid((uint32_t)((np + 255) / 256));
    switch (S) {
    case 2: k_edm_frag<SPLIT, 2><<<grid, 256, 0, s>>>(x, n, d, ldx, np, mean, frag); break;
    case 4: k_edm_frag<SPLIT, 4><<<grid, 256, 0, s>>>(x, n, d, ldx, np, mean, frag); break;
    case 8: k_edm_frag<SPLIT, 8><<<grid, 256, 0, s>>>(x, n, d, ldx, np, mean, frag); break;
    }
}

// One distance-map domain under lambda with the FP32 body (batched
// per-instance mode); false for an unsupported tile.
bool launch_edm_f32_lambda(int tile, const TileGrid &g, const EdmTile &t, hipStream_t s)
{
    EdmArgs a{g, t};
    uint32_t gx, gy;
    if (g.T <= (1ull << 24)) { gx = (uint32_t)g.T; gy = 1; }
    else { gx = 1u << 16; gy = (uint32_t)((g.T + gx - 1) / gx); }
    const dim3 grid(gx, gy);
    switch (tile) {
    case 16: k_edm_f32<MAP_LAMBDA, 16, kEdmStageScalar><<<grid, 256, 0, s>>>(a); return true;
    case 32: k_edm_f32<MAP_LAMBDA, 32, kEdmStageScalar><<<grid, 256, 0, s>>>(a); return true;
    case 64: k_edm_f32<MAP_LAMBDA, 64, kEdmStageScalar><<<grid, 256, 0, s>>>(a); return true;
    }
    return false;
}

static tri_status edm_check(const tri_plan *p, int64_t d, int mode)
{
    if (!p) return fail(TRI_E_INVAL, "tri_edm: plan is NULL");
    if (p->diag) return fail(TRI_E_INVAL, "tri_edm: the plan must exclude the diagonal");
    if (p->map == TRI_MAP_UTM) return fail(TRI_E_UNSUPPORTED, "tri_edm: UTM is not supported");
    if (d < 1 || d > 4096) return fail(TRI_E_RANGE, "tri_edm: d = %lld not in [1, 4096]", (long long)d);
    if (p->flags & TRI_FLAG_STRIP_BAND)
        return fail(TRI_E_UNSUPPORTED, "tri_edm: two-row band strips are for the elementwise kernels");
    if (mode == TRI_EDM_FP32) {
        if (p->tile != 16 && p->tile != 32 && p->tile != 64 && p->tile != 128)
            return fail(TRI_E_UNSUPPORTED, "tri_edm: FP32 mode needs tile 16, 32, 64 or 128");
        return TRI_OK;
    }
    if (mode == TRI_EDM_BF16X3 || mode == TRI_EDM_BF16) {
        if (p->tile != kEdmTile)
            return fail(TRI_E_UNSUPPORTED, "tri_edm: MFMA modes need tile %d", kEdmTile);
        return TRI_OK;
    }
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
    if (mode != TRI_EDM_FP32) *bytes = edm_ws_layout(p->n, d).total;
    return TRI_OK;
}

namespace trimap {

static tri_status edm_run(const tri_plan *p, const float *x, int64_t d, int64_t ldx, float *out,
                          int mode, float fixup_thr, void *ws, size_t ws_bytes, void *stream)
{
    tri_status st = edm_check(p, d, mode);
    if (st != TRI_OK) return st;
    if (p->n < 2) return TRI_OK;
    if (!x || !out) return fail(TRI_E_INVAL, "tri_edm: NULL buffer");
    if (ldx < d) return fail(TRI_E_INVAL, "tri_edm: ldx < d");
    if (((uintptr_t)x | (uintptr_t)out) & 3) return fail(TRI_E_INVAL, "tri_edm: unaligned buffer");
    hipStream_t s = (hipStream_t)stream;
    if (mode == TRI_EDM_FP32) {
        EdmArgs a{plan_tile_grid(p), EdmTile{(int32_t)p->n, (int32_t)d, ldx, x, out}};
        if (!edm_f32(p, a, s)) return fail(TRI_E_UNSUPPORTED, "tri_edm: tile");
        TRI_HIP(hipGetLastError());
        return TRI_OK;
    }
    if ((uintptr_t)out & 15)
        return fail(TRI_E_INVAL, "tri_edm: the MFMA modes need a 16-byte aligned output");
    const EdmWs L = edm_ws_layout(p->n, d);
    if (!ws || ws_bytes < L.total)
        return fail(TRI_E_NOMEM, "tri_edm: workspace of %zu bytes needed", L.total);
    if ((uintptr_t)ws & 255) return fail(TRI_E_INVAL, "tri_edm: workspace must be 256-byte aligned");
    if (!(fixup_thr >= 0.f)) return fail(TRI_E_INVAL, "tri_edm: fixup_thr must be >= 0");
    char *w = (char *)ws;
    __bf16 *hi = (__bf16 *)(w + L.hi), *lo = (__bf16 *)(w + L.lo);
    float *norms = (float *)(w + L.norms), *mean = (float *)(w + L.mean);
    float *partial = (float *)(w + L.partial);
    const int32_t n = (int32_t)p->n, dd = (int32_t)d, dp = (int32_t)L.dp;
    const bool split = (mode == TRI_EDM_BF16X3);
    k_edm_colsum<<<dim3((uint32_t)L.nb), 256, 0, s>>>(x, n, dd, ldx, dp, partial);
    k_edm_mean<<<dim3((uint32_t)dp), 256, 0, s>>>(partial, (int32_t)L.nb, n, dp, mean);
    if (L.S) {
        bf16x8 *frag = (bf16x8 *)(w + L.hi);
        const int32_t np = (int32_t)L.np;
        if (split) edm_frag_launch<true>(L.S, x, n, dd, ldx, np, mean, frag, s);
        else edm_frag_launch<false>(L.S, x, n, dd, ldx, np, mean, frag, s);
        TRI_HIP(hipGetLastError());
        EdmLinesArgs a{plan_tile_grid(p), StripGrid{}, n, dd, ldx, x, frag, out, fixup_thr};
        const bool ok = split ? edm_lines<true>(p, a, L.S, s) : edm_lines<false>(p, a, L.S, s);
        if (!ok) return fail(TRI_E_UNSUPPORTED, "tri_edm: map");
        TRI_HIP(hipGetLastError());
        return TRI_OK;
    }
    if (split)
        k_edm_split<true><<<dim3((uint32_t)n), 64, 0, s>>>(x, dd, ldx, dp, mean, hi, lo, norms);
    else
        k_edm_split<false><<<dim3((uint32_t)n), 64, 0, s>>>(x, dd, ldx, dp, mean, hi, lo, norms);
    TRI_HIP(hipGetLastError());
    EdmMfmaArgs a{plan_tile_grid(p), n, dd, dp, ldx, x, hi, lo, norms, out, fixup_thr};
    if (!edm_mfma(p, a, split, s)) return fail(TRI_E_UNSUPPORTED, "tri_edm: map");
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}

// Scratch of the allocation-free entry point: the MFMA modes' workspace in a
// device array of the library (one copy on every GPU the library runs on,
// held until the process ends).  In host code `scratch` names a host-side
// stand-in, never the device memory: host code uses only the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[TRI_EDM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch, looked up on the first
// call on that device and kept.
static tri_status edm_scratch(void **out)
{
    int dev = 0;
    TRI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(TRI_E_RANGE, "tri_edm_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        TRI_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(TRI_E_HIP, "tri_edm_noalloc: no device address for the scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TRI_OK;
}

}  // namespace trimap

extern "C" tri_status tri_edm(const tri_plan *p, const float *x, int64_t d, int64_t ldx,
                              float *out, int mode, float fixup_thr, void *ws, size_t ws_bytes,
                              void *stream)
{
    clear_error();
    return edm_run(p, x, d, ldx, out, mode, fixup_thr, ws, ws_bytes, stream);
}

extern "C" tri_status tri_edm_noalloc(const tri_plan *p, const float *x, int64_t d, int64_t ldx,
                                      float *out, int mode, float fixup_thr, void *stream)
{
    clear_error();
    tri_status st = edm_check(p, d, mode);
    if (st != TRI_OK) return st;
    if (mode == TRI_EDM_FP32 || p->n < 2)
        return edm_run(p, x, d, ldx, out, mode, fixup_thr, nullptr, 0, stream);
    const size_t need = edm_ws_layout(p->n, d).total;
    if (need > (size_t)TRI_EDM_NOALLOC_SCRATCH_BYTES)
        return fail(TRI_E_RANGE,
                    "tri_edm_noalloc: n = %lld, d = %lld need %zu bytes of workspace, above the "
                    "%zu-byte scratch (use tri_edm with a caller workspace)",
                    (long long)p->n, (long long)d, need, (size_t)TRI_EDM_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    st = edm_scratch(&ws);
    if (st != TRI_OK) return st;
    return edm_run(p, x, d, ldx, out, mode, fixup_thr, ws, TRI_EDM_NOALLOC_SCRATCH_BYTES, stream);
}
