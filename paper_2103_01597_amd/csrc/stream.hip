// Achievable HBM bandwidth: plain streaming kernels (copy and triad) whose
// rate is the practical ceiling against which the fused substep's traffic is
// judged (the paper, too, confirms its bandwidth figures by measurement,
// Section 5).
//
// Each thread moves UNROLL 16-byte vectors spaced one block apart, issuing
// all loads before any store; a launch covers the arrays with one pass.
//   copy : c[i] = a[i]              (16 B read + 16 B written per vector)
//   triad: c[i] = a[i] + s * b[i]   (32 B read + 16 B written, FP64)
// The non-temporal variants store (and load) with the non-temporal hint.
#include "mhd_internal.hpp"

namespace mhd {
namespace {

constexpr int SB_THREADS = 256;
constexpr int SB_UNROLL = 4;

template <bool TRIAD, bool NT>
__global__ __launch_bounds__(SB_THREADS) void k_stream(const double2* __restrict__ a,
                                                      const double2* __restrict__ b,
                                                      double2* __restrict__ c, int64_t n,
                                                      double s)
{
    const int64_t base = (int64_t)blockIdx.x * SB_THREADS * SB_UNROLL + threadIdx.x;
    double2 va[SB_UNROLL], vb[SB_UNROLL];
#pragma unroll
    for (int u = 0; u < SB_UNROLL; ++u) {
        const int64_t i = base + (int64_t)u * SB_THREADS;
        if (i < n) {
            if (NT) {
                va[u].x = __builtin_nontemporal_load(&a[i].x);
                va[u].y = __builtin_nontemporal_load(&a[i].y);
                if (TRIAD) {
                    vb[u].x = __builtin_nontemporal_load(&b[i].x);
                    vb[u].y = __builtin_nontemporal_load(&b[i].y);
                }
            } else {
                va[u] = a[i];
                if (TRIAD) vb[u] = b[i];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < SB_UNROLL; ++u) {
        const int64_t i = base + (int64_t)u * SB_THREADS;
        if (i < n) {
            double2 v = va[u];
            if (TRIAD) {
                v.x = fma(s, vb[u].x, v.x);
                v.y = fma(s, vb[u].y, v.y);
            }
            if (NT) {
                __builtin_nontemporal_store(v.x, &c[i].x);
                __builtin_nontemporal_store(v.y, &c[i].y);
            } else {
                c[i] = v;
            }
        }
    }
}

}  // namespace
}  // namespace mhd

extern "C" int mhd_bandwidth_probe(int32_t kind, const void* a, const void* b, void* c,
                                   int64_t bytes, void* stream)
{
    using namespace mhd;
    if (kind < MHD_BW_COPY || kind > MHD_BW_TRIAD_NT || !a || !c || bytes <= 0 || bytes % 16)
        return MHD_ERR_INVALID;
    const bool triad = kind == MHD_BW_TRIAD || kind == MHD_BW_TRIAD_NT;
    const bool nt = kind == MHD_BW_COPY_NT || kind == MHD_BW_TRIAD_NT;
    if (triad && !b) return MHD_ERR_INVALID;
    if (a == c || (triad && b == c)) return MHD_ERR_INVALID;
    const int64_t n = bytes / 16;
    const int64_t per_block = (int64_t)SB_THREADS * SB_UNROLL;
    const int64_t blocks = (n + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) return MHD_ERR_INVALID;
    const double2* pa = (const double2*)a;
    const double2* pb = (const double2*)b;
    double2* pc = (double2*)c;
    hipStream_t st = (hipStream_t)stream;
    dim3 grid((unsigned)blocks), block(SB_THREADS);
    if (!triad && !nt)
        hipLaunchKernelGGL((k_stream<false, false>), grid, block, 0, st, pa, pb, pc, n, 0.0);
    else if (!triad)
        hipLaunchKernelGGL((k_stream<false, true>), grid, block, 0, st, pa, pb, pc, n, 0.0);
    else if (!nt)
        hipLaunchKernelGGL((k_stream<true, false>), grid, block, 0, st, pa, pb, pc, n, 3.0);
    else
        hipLaunchKernelGGL((k_stream<true, true>), grid, block, 0, st, pa, pb, pc, n, 3.0);
    return hipGetLastError() == hipSuccess ? MHD_OK : MHD_ERR_DEVICE;
}
