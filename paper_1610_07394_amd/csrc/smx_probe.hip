// Measurement probe: the FP32 vector-ALU issue ceiling of the device, for the
// roofline of the VALU-bound kernels.  Each thread runs eight independent
// chains of fused multiply-adds (no memory traffic in the loop), enough waves
// to fill every SIMD; one store per thread keeps the chains live.  Lane
// operations per launch: blocks x 256 x iters x 64.
#include "smx_device.h"
#include "smx_internal.h"

namespace smx {

__global__ __launch_bounds__(256) void valu_probe_kernel(float *out, int iters, float b, float c) {
    float a0 = float(threadIdx.x), a1 = a0 + 1.f, a2 = a0 + 2.f, a3 = a0 + 3.f;
    float a4 = a0 + 4.f, a5 = a0 + 5.f, a6 = a0 + 6.f, a7 = a0 + 7.f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a0 = __builtin_fmaf(a0, b, c);
            a1 = __builtin_fmaf(a1, b, c);
            a2 = __builtin_fmaf(a2, b, c);
            a3 = __builtin_fmaf(a3, b, c);
            a4 = __builtin_fmaf(a4, b, c);
            a5 = __builtin_fmaf(a5, b, c);
            a6 = __builtin_fmaf(a6, b, c);
            a7 = __builtin_fmaf(a7, b, c);
        }
    }
    out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}

int launch_valu_probe(float *out, int64_t blocks, int iters, hipStream_t s) {
    hipLaunchKernelGGL(valu_probe_kernel, dim3(uint32_t(blocks)), dim3(256), 0, s, out, iters, 0.999f, 0.001f);
    return check_launch("valu probe");
}

}  // namespace smx
