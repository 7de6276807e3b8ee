// Periodic halo fill (Section 3.3): every halo cell of the padded grid
// takes the interior cell given by the mapping s' = ((s - r) mod n) + r on
// each axis.  One launch fills sides, edges and corners of all 8 fields:
// each halo cell reads its interior source directly, so no cell depends on
// another halo cell and the three regions below can run concurrently.
//
//   region Z: the 6 halo planes z < 3, z >= nz+3      (all y, all x)
//   region Y: interior planes, the 6 halo rows of y   (all x)
//   region X: interior planes and rows, the 6 halo columns of x
//
// Regions Z and Y are contiguous runs of x and coalesce; region X touches
// 6 elements per row.  Bytes per launch: 2 * 8 * elem * (M^3 - N^3).
#include "mhd_internal.hpp"

namespace mhd {
namespace {

__device__ __forceinline__ int wrap_index(int s, int n)
{
    int t = (s - R) % n;
    return (t < 0 ? t + n : t) + R;
}

template <typename E>
__global__ __launch_bounds__(256) void k_halo(Grid g, E* __restrict__ fields)
{
    const int per_field_z = 6 * g.mxy;
    const int per_field_y = g.nz * 6 * g.mx;
    const int per_field_x = g.nz * g.ny * 6;
    const int total = per_field_z + per_field_y + per_field_x;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 >= total)
        return;
    E* f = fields + (int64_t)blockIdx.y * g.fstride;

    int x, y, z, t = t0;
    if (t < per_field_z) {
        const int p = t / g.mxy;
        const int rem = t - p * g.mxy;
        y = rem / g.mx;
        x = rem - y * g.mx;
        z = p < 3 ? p : g.nz + p;
    } else if ((t -= per_field_z) < per_field_y) {
        const int row6 = 6 * g.mx;
        const int zz = t / row6;
        const int rem = t - zz * row6;
        const int r = rem / g.mx;
        x = rem - r * g.mx;
        y = r < 3 ? r : g.ny + r;
        z = R + zz;
    } else {
        t -= per_field_y;
        const int col6 = 6 * g.ny;
        const int zz = t / col6;
        const int rem = t - zz * col6;
        const int yy = rem / 6;
        const int c = rem - yy * 6;
        x = c < 3 ? c : g.nx + c;
        y = R + yy;
        z = R + zz;
    }
    const int sx = wrap_index(x, g.nx), sy = wrap_index(y, g.ny), sz = wrap_index(z, g.nz);
    f[(z * g.my + y) * g.mx + x] = f[(sz * g.my + sy) * g.mx + sx];
}

}  // namespace

hipError_t launch_halo(const Grid& g, void* fields, int elem_size, hipStream_t st)
{
    const int total = 6 * g.mxy + g.nz * 6 * g.mx + g.nz * g.ny * 6;
    dim3 block(256);
    dim3 grid((total + 255) / 256, NQ);
    if (elem_size == 8)
        hipLaunchKernelGGL(k_halo<uint64_t>, grid, block, 0, st, g, (uint64_t*)fields);
    else
        hipLaunchKernelGGL(k_halo<uint32_t>, grid, block, 0, st, g, (uint32_t*)fields);
    return hipGetLastError();
}

}  // namespace mhd
