// LDS-tiled z-marching fused RHS + RK3 kernel (placeholder until written):
// reports "not launched" so the caller falls back to the direct kernel.
#include "mhd_internal.hpp"

namespace mhd {

hipError_t launch_rk3_tiled(const Grid&, const Phys&, int, int, const void*, void*, void*, void*,
                            double, hipStream_t, bool* launched)
{
    *launched = false;
    return hipSuccess;
}

}  // namespace mhd
