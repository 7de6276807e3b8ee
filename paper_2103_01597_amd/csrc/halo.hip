// Periodic halo fill (Section 3.3): every halo cell of the padded grid
// takes the interior cell given by the mapping s' = ((s - r) mod n) + r on
// each axis.  One launch fills sides, edges and corners of all 8 fields:
// each halo cell reads its interior source directly, so no cell depends on
// another halo cell and the three regions below can run concurrently.
//
//   region Z: the 2r halo planes z < r, z >= nz+r     (all y, all x)
//   region Y: interior planes, the 2r halo rows of y  (all x)
//   region X: interior planes and rows, the 2r halo columns of x
//
// r is the halo width (the stencil radius, 1..4).  Regions Z and Y are
// contiguous runs of x and coalesce; region X touches 2r elements per row.
// Bytes per launch: 2 * 8 * elem * (M^3 - N^3).
#include "mhd_internal.hpp"

namespace mhd {
namespace {

__device__ __forceinline__ int wrap_index(int s, int n, int r)
{
    int t = (s - r) % n;
    return (t < 0 ? t + n : t) + r;
}

template <typename E>
__global__ __launch_bounds__(256) void k_halo(Grid g, E* __restrict__ fields)
{
    const int r = g.r, w = 2 * g.r;
    const int per_field_z = w * g.mxy;
    const int per_field_y = g.nz * w * g.mx;
    const int per_field_x = g.nz * g.ny * w;
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
        z = p < r ? p : g.nz + p;
    } else if ((t -= per_field_z) < per_field_y) {
        const int rows = w * g.mx;
        const int zz = t / rows;
        const int rem = t - zz * rows;
        const int yr = rem / g.mx;
        x = rem - yr * g.mx;
        y = yr < r ? yr : g.ny + yr;
        z = r + zz;
    } else {
        t -= per_field_y;
        const int cols = w * g.ny;
        const int zz = t / cols;
        const int rem = t - zz * cols;
        const int yy = rem / w;
        const int c = rem - yy * w;
        x = c < r ? c : g.nx + c;
        y = r + yy;
        z = r + zz;
    }
    const int sx = wrap_index(x, g.nx, r), sy = wrap_index(y, g.ny, r), sz = wrap_index(z, g.nz, r);
    f[(z * g.my + y) * g.mx + x] = f[(sz * g.my + sy) * g.mx + sx];
}

}  // namespace

hipError_t launch_halo(const Grid& g, void* fields, int elem_size, hipStream_t st)
{
    const int w = 2 * g.r;
    const int total = w * g.mxy + g.nz * w * g.mx + g.nz * g.ny * w;
    dim3 block(256);
    dim3 grid((total + 255) / 256, NQ);
    if (elem_size == 8)
        hipLaunchKernelGGL(k_halo<uint64_t>, grid, block, 0, st, g, (uint64_t*)fields);
    else
        hipLaunchKernelGGL(k_halo<uint32_t>, grid, block, 0, st, g, (uint32_t*)fields);
    return hipGetLastError();
}

}  // namespace mhd
