// Test exports (the span search and basis exactly as the kernels use them)
// and a fill kernel for zeroing gradients (a kernel, not a memset, so that
// the call can be captured in a graph).
#include "device.hpp"
#include "launch.hpp"

#include <algorithm>

namespace nd {
namespace {
template <int D>
__global__ void k_spans(const float* U, int nk, const float* x, int nx, int32_t* spans, float* N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx) return;
    float Nb[D + 1];
    const int k = sample_basis<D>(U, nk - D - 1, x[i], Nb);
    if (spans) spans[i] = k;
    if (N) {
#pragma unroll
        for (int r = 0; r <= D; ++r) N[(size_t)i * (D + 1) + r] = Nb[r];
    }
}
__global__ void k_zero(float* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}
}  // namespace

hipError_t launch_zero(hipStream_t st, float* p, size_t n) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_spans(int p, hipStream_t st, const float* U, int nk, const float* x, int nx, int* spans,
                        float* N) {
    const dim3 grid((nx + 255) / 256);
    switch (p) {
#define C(D) case D: hipLaunchKernelGGL((k_spans<D>), grid, dim3(256), 0, st, U, nk, x, nx, spans, N); break;
        C(1) C(2) C(3) C(4) C(5) C(6) C(7)
#undef C
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace nd
