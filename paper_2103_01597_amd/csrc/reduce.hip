// Deterministic reductions over the interior of one field.  Stage 1: block
// b walks rows b, b + G, b + 2G, ... (G = REDUCE_BLOCKS) with each thread
// striding x by 256, then a fixed LDS tree; stage 2: one block combines the
// G partials in the same fixed tree.  FP64 accumulation throughout, so the
// result depends only on the data, never on timing.
#include "mhd_internal.hpp"

namespace mhd {
namespace {

__device__ __forceinline__ double nan_max(double a, double b)
{
    return (isnan(a) || isnan(b)) ? __longlong_as_double(0x7ff8000000000000LL) : (a > b ? a : b);
}
__device__ __forceinline__ double nan_min(double a, double b)
{
    return (isnan(a) || isnan(b)) ? __longlong_as_double(0x7ff8000000000000LL) : (a < b ? a : b);
}

__device__ __forceinline__ double red_init(int op)
{
    if (op == MHD_RED_MIN) return __longlong_as_double(0x7ff0000000000000LL);   // +inf
    if (op == MHD_RED_MAX) return -__longlong_as_double(0x7ff0000000000000LL);  // -inf
    return 0.0;
}
__device__ __forceinline__ double red_map(double v, int op)
{
    switch (op) {
    case MHD_RED_SUMSQ: return v * v;
    case MHD_RED_SUMEXP: return exp(v);
    case MHD_RED_NONFINITE: return isfinite(v) ? 0.0 : 1.0;
    case MHD_RED_MAXABS: return fabs(v);
    default: return v;
    }
}
__device__ __forceinline__ double red_comb(double a, double b, int op)
{
    switch (op) {
    case MHD_RED_MAXABS:
    case MHD_RED_MAX: return nan_max(a, b);
    case MHD_RED_MIN: return nan_min(a, b);
    default: return a + b;
    }
}

__device__ double block_tree(double v, int op, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h)
            sh[t] = red_comb(sh[t], sh[t + h], op);
        __syncthreads();
    }
    return sh[0];
}

template <typename E>
__global__ __launch_bounds__(256) void k_reduce_stage1(Grid g, const E* __restrict__ f, int op,
                                                       double* __restrict__ partials)
{
    __shared__ double sh[256];
    double acc = red_init(op);
    const int rows = g.ny * g.nz;
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const int j = r % g.ny, k = r / g.ny;
        const E* row = f + g.interior + k * g.mxy + j * g.mx;
        for (int x = threadIdx.x; x < g.nx; x += 256)
            acc = red_comb(acc, red_map(double(row[x]), op), op);
    }
    const double b = block_tree(acc, op, sh);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = b;
}

__global__ __launch_bounds__(256) void k_reduce_stage2(const double* __restrict__ partials,
                                                       int n, int op, double* __restrict__ out)
{
    __shared__ double sh[256];
    double acc = red_init(op);
    for (int i = threadIdx.x; i < n; i += 256)
        acc = red_comb(acc, partials[i], op);
    const double b = block_tree(acc, op, sh);
    if (threadIdx.x == 0)
        *out = b;
}

}  // namespace

hipError_t launch_reduce(const Grid& g, const void* field, int elem_size, int op,
                         double* partials, int npartials, double* result, hipStream_t st)
{
    if (elem_size == 8)
        hipLaunchKernelGGL(k_reduce_stage1<double>, dim3(npartials), dim3(256), 0, st, g,
                           (const double*)field, op, partials);
    else
        hipLaunchKernelGGL(k_reduce_stage1<float>, dim3(npartials), dim3(256), 0, st, g,
                           (const float*)field, op, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_reduce_stage2, dim3(1), dim3(256), 0, st, partials, npartials, op,
                       result);
    return hipGetLastError();
}

}  // namespace mhd
