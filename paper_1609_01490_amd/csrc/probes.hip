// Measurement probes: a STREAM-style add (c = a + b over 16-byte vectors, two
// reads and one write per element, the same mix as the fp32 elementwise
// body) that gives the HBM bandwidth a plain streaming kernel reaches on this
// GPU, the ceiling the triangular kernels are compared with.
#include "common.hpp"

namespace trimap {

typedef float f4p __attribute__((ext_vector_type(4)));

// Each workgroup streams a contiguous block of 4 x 256 vectors: every
// thread issues its four loads of a and of b before the first add.
constexpr int kStreamUnroll = 4;

__global__ void __launch_bounds__(256) k_stream_add(f4p *c, const f4p *a, const f4p *b,
                                                    uint64_t nvec)
{
    const uint64_t base = (uint64_t)blockIdx.x * (256 * kStreamUnroll) + threadIdx.x;
    f4p x[kStreamUnroll], y[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const uint64_t k = base + 256 * u;
        if (k < nvec) {
            x[u] = __builtin_nontemporal_load(a + k);
            y[u] = __builtin_nontemporal_load(b + k);
        }
    }
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
        const uint64_t k = base + 256 * u;
        if (k < nvec) __builtin_nontemporal_store(x[u] + y[u], c + k);
    }
}

}  // namespace trimap

using namespace trimap;

extern "C" tri_status tri_stream_add(float *c, const float *a, const float *b, int64_t count,
                                     void *stream)
{
    clear_error();
    if (count < 0 || (count > 0 && (!a || !b || !c)))
        return fail(TRI_E_INVAL, "tri_stream_add: bad arguments");
    if (count % 4 || (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15))
        return fail(TRI_E_INVAL, "tri_stream_add: count must be a multiple of 4 and buffers 16-byte aligned");
    if (count == 0) return TRI_OK;
    const uint64_t nvec = (uint64_t)count / 4;
    const uint64_t blocks = (nvec + 256 * kStreamUnroll - 1) / (256 * kStreamUnroll);
    if (blocks > kMaxWorkItems / 256) return fail(TRI_E_RANGE, "tri_stream_add: count too large");
    k_stream_add<<<dim3((uint32_t)blocks), 256, 0, (hipStream_t)stream>>>((f4p *)c, (const f4p *)a,
                                                                          (const f4p *)b, nvec);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
