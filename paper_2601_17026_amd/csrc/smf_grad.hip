// Backward of the optimal surface energy (gfx950).
//
// E*(c) = min over delta-smooth surfaces h of sum_p c(p, h(p)) (Section 1.1,
// Eq. 1, feature term) is a minimum of functions that are linear in c, so
// where the optimal height of a column is unique dE*/dc(p,z) = [z == h(p)];
// where it is not, the indicator of the minimal surface is a supergradient.
// The backward pass is therefore a one-hot scatter of the incoming energy
// gradient: a pure write stream of one float per voxel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smf.h"

namespace smf {

// grad[b][p][z] = g[b] if z == h[b][p] else 0.  One thread writes four
// consecutive heights with one 16-byte store when the column allows it.
__global__ __launch_bounds__(256) void k_onehot_backward(const int *__restrict__ h,
                                                         const float *__restrict__ g,
                                                         float *__restrict__ grad, long long P,
                                                         int K, long long quads_per_col, int n)
{
    const long long total = (long long)n * P * quads_per_col;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const long long col = i / quads_per_col;          // b * P + p
        const int z0 = (int)(i - col * quads_per_col) * 4;
        const int b = (int)(col / P);
        const int hz = h[col];
        const float gb = g[b];
        float *dst = grad + col * K + z0;
        const float v0 = z0 == hz ? gb : 0.f;
        const float v1 = z0 + 1 == hz ? gb : 0.f;
        const float v2 = z0 + 2 == hz ? gb : 0.f;
        const float v3 = z0 + 3 == hz ? gb : 0.f;
        if ((K & 3) == 0) {
            *reinterpret_cast<float4 *>(dst) = make_float4(v0, v1, v2, v3);
        } else {
            dst[0] = v0;
            if (z0 + 1 < K) dst[1] = v1;
            if (z0 + 2 < K) dst[2] = v2;
            if (z0 + 3 < K) dst[3] = v3;
        }
    }
}

}  // namespace smf

extern "C" int smf_onehot_backward(const int32_t *surface_dev, const float *grad_energy_dev,
                                   float *grad_cost_dev, int32_t n, int32_t nx, int32_t ny,
                                   int32_t K, void *stream)
{
    if (!surface_dev || !grad_energy_dev || !grad_cost_dev || n < 1 || nx < 1 || ny < 1 || K < 1)
        return SMF_ERR_ARG;
    const long long P = (long long)nx * ny;
    const long long quads = (K + 3) / 4;
    const long long total = (long long)n * P * quads;
    long long blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(smf::k_onehot_backward, dim3((unsigned)blocks), dim3(256), 0,
                       (hipStream_t)stream, surface_dev, grad_energy_dev, grad_cost_dev, P, K,
                       quads, n);
    return hipGetLastError() == hipSuccess ? SMF_OK : SMF_ERR_HIP;
}
