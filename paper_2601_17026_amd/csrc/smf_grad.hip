// Backward of the optimal surface energy (gfx950).
//
// E*(c) = min over delta-smooth surfaces h of sum_p c(p, h(p)) (Section 1.1,
// Eq. 1, feature term) is a minimum of functions that are linear in c, so
// where the optimal height of a column is unique dE*/dc(p,z) = [z == h(p)];
// where it is not, the indicator of the minimal surface is a supergradient.
// The backward pass is therefore a one-hot scatter of the incoming energy
// gradient: a pure write stream of one float per voxel.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "../../include/smf.h"

namespace smf {

// grad[b][p][z] = g[b] if z == h[b][p] else 0.  Block (bx, b) with threads
// (tx, ty): volume b = blockIdx.y, its columns taken blockDim.y at a time
// (grid-stride over blockIdx.x), and each column's heights written by the
// blockDim.x threads of one row, four consecutive heights per 16-byte store
// when K % 4 == 0.  A row of threads writes one column's contiguous 4K
// bytes and the rows of a block consecutive columns, so the stores of a
// block form one contiguous stream; no index needs a division.
__global__ __launch_bounds__(256) void k_onehot_backward(const int *__restrict__ h,
                                                         const float *__restrict__ g,
                                                         float *__restrict__ grad, int P, int K,
                                                         int quads)
{
    const int b = blockIdx.y;
    const float gb = g[b];
    const size_t vol = (size_t)b * P;
    for (int p = blockIdx.x * blockDim.y + threadIdx.y; p < P; p += gridDim.x * blockDim.y) {
        const int hz = h[vol + p];
        float *dst = grad + (vol + p) * (size_t)K;
        for (int q = threadIdx.x; q < quads; q += blockDim.x) {
            const int z0 = 4 * q;
            const float v0 = z0 == hz ? gb : 0.f;
            const float v1 = z0 + 1 == hz ? gb : 0.f;
            const float v2 = z0 + 2 == hz ? gb : 0.f;
            const float v3 = z0 + 3 == hz ? gb : 0.f;
            if ((K & 3) == 0) {
                *reinterpret_cast<float4 *>(dst + z0) = make_float4(v0, v1, v2, v3);
            } else {
                dst[z0] = v0;
                if (z0 + 1 < K) dst[z0 + 1] = v1;
                if (z0 + 2 < K) dst[z0 + 2] = v2;
                if (z0 + 3 < K) dst[z0 + 3] = v3;
            }
        }
    }
}

}  // namespace smf

extern "C" int smf_onehot_backward(const int32_t *surface_dev, const float *grad_energy_dev,
                                   float *grad_cost_dev, int32_t n, int32_t nx, int32_t ny,
                                   int32_t K, void *stream)
{
    if (!surface_dev || !grad_energy_dev || !grad_cost_dev || n < 1 || nx < 1 || ny < 1 || K < 1 ||
        n > 65535 || (long long)nx * ny > INT32_MAX)
        return SMF_ERR_ARG;
    const int P = nx * ny;
    const int quads = (K + 3) / 4;
    // a row of threads per column: the smallest power of two >= quads, at most 64
    int tx = 1;
    while (tx < quads && tx < 64) tx <<= 1;
    const int ty = 256 / tx;
    long long bx = ((long long)P + ty - 1) / ty;
    if (bx > 2048) bx = 2048;
    hipLaunchKernelGGL(smf::k_onehot_backward, dim3((unsigned)bx, (unsigned)n), dim3(tx, ty), 0,
                       (hipStream_t)stream, surface_dev, grad_energy_dev, grad_cost_dev, P, K, quads);
    return hipGetLastError() == hipSuccess ? SMF_OK : SMF_ERR_HIP;
}
