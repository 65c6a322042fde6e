// Measurement probes: a STREAM-style add (c = a + b over 16-byte vectors, two
// reads and one write per element, the same mix as the fp32 elementwise
// body) that gives the HBM bandwidth a plain streaming kernel reaches on this
// GPU, the ceiling the triangular kernels are compared with.
#include "common.hpp"

namespace trimap {

typedef float f4p __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_add(f4p *c, const f4p *a, const f4p *b,
                                                    uint64_t nvec)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < nvec; k += stride) {
        const f4p x = __builtin_nontemporal_load(a + k);
        const f4p y = __builtin_nontemporal_load(b + k);
        __builtin_nontemporal_store(x + y, c + k);
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
    int dev = 0, cus = 0;
    TRI_HIP(hipGetDevice(&dev));
    TRI_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t nvec = (uint64_t)count / 4;
    const uint64_t want = (nvec + 255) / 256;
    const uint32_t grid = (uint32_t)(want < (uint64_t)cus * 16 ? want : (uint64_t)cus * 16);
    k_stream_add<<<grid, 256, 0, (hipStream_t)stream>>>((f4p *)c, (const f4p *)a,
                                                         (const f4p *)b, nvec);
    TRI_HIP(hipGetLastError());
    return TRI_OK;
}
