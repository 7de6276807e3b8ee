// Periodic halo fill (Section 3.3): every halo cell of the padded grid
// takes the interior cell given by the mapping s' = ((s - r) mod n) + r on
// each axis, r the halo width (the stencil radius, 1..4); sides, edges and
// corners of all 8 fields are filled.  Bytes per fill: 2 * 8 * elem *
// (M^3 - N^3).
#include "mhd_internal.hpp"

namespace mhd {
namespace {

__device__ __forceinline__ int wrap_index(int s, int n, int r)
{
    int t = (s - r) % n;
    return (t < 0 ? t + n : t) + r;
}

// Three launches, each reading only cells that are final when it runs:
//   X: interior planes and rows, the 2r halo columns (element copies of
//      interior cells, x wrapped);
//   Y: interior planes, the 2r halo rows, each copied whole (its halo
//      columns included, filled by X) from the wrapped interior row;
//   Z: the 2r halo planes, each copied whole from the wrapped interior plane.
// Y and Z copy whole rows and planes in units of V elements (V = 2 when the
// padded row length mx is even: every row then starts on a V-element
// boundary, so FP64 moves 16 bytes per access).
template <typename E, int V>
struct alignas(sizeof(E) * V) HVec {
    E v[V];
};

// X: a workgroup covers 32 rows of one interior plane of one field, eight
// lanes per row (lane c < 2r fills column c of the left halo, c < r, or
// column c - r of the right halo), so the row and plane come from the
// launch indices rather than from divisions.
constexpr int HX_ROWS = 32;

template <typename E>
__global__ __launch_bounds__(256) void k_halo_x(Grid g, E* __restrict__ fields)
{
    const int r = g.r, c = threadIdx.x & 7;
    const int yy = blockIdx.x * HX_ROWS + (threadIdx.x >> 3);
    if (c >= 2 * r || yy >= g.ny) return;
    E* f = fields + (int64_t)blockIdx.z * g.fstride;
    const int row = ((r + (int)blockIdx.y) * g.my + r + yy) * g.mx;
    const int dst = c < r ? c : g.nx + c;  // padded halo column
    f[row + dst] = f[row + wrap_index(dst, g.nx, r)];
}

template <typename E, int V>
__global__ __launch_bounds__(256) void k_halo_y(Grid g, E* __restrict__ fields)
{
    using Vt = HVec<E, V>;
    const int r = g.r, row_units = g.mx / V;
    const int per_plane = 2 * r * row_units;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nz * per_plane) return;
    E* f = fields + (int64_t)blockIdx.y * g.fstride;
    const int zz = t / per_plane, rem = t - zz * per_plane;
    const int yr = rem / row_units, u = rem - yr * row_units;
    const int y = yr < r ? yr : g.ny + yr;
    const int plane = (r + zz) * g.mxy;
    Vt* dst = reinterpret_cast<Vt*>(f + plane + y * g.mx);
    const Vt* src = reinterpret_cast<const Vt*>(f + plane + wrap_index(y, g.ny, r) * g.mx);
    dst[u] = src[u];
}

template <typename E, int V>
__global__ __launch_bounds__(256) void k_halo_z(Grid g, E* __restrict__ fields)
{
    using Vt = HVec<E, V>;
    const int r = g.r, plane_units = g.mxy / V;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * r * plane_units) return;
    E* f = fields + (int64_t)blockIdx.y * g.fstride;
    const int p = t / plane_units, u = t - p * plane_units;
    const int z = p < r ? p : g.nz + p;
    Vt* dst = reinterpret_cast<Vt*>(f + z * g.mxy);
    const Vt* src = reinterpret_cast<const Vt*>(f + wrap_index(z, g.nz, r) * g.mxy);
    dst[u] = src[u];
}

template <typename E, int V>
void launch_halo_typed(const Grid& g, void* fields, hipStream_t st)
{
    const int w = 2 * g.r;
    auto blocks = [](int n) { return dim3((unsigned)((n + 255) / 256), NQ); };
    hipLaunchKernelGGL(k_halo_x<E>, dim3((unsigned)((g.ny + HX_ROWS - 1) / HX_ROWS), (unsigned)g.nz, NQ),
                       dim3(256), 0, st, g, (E*)fields);
    hipLaunchKernelGGL((k_halo_y<E, V>), blocks(g.nz * w * (g.mx / V)), dim3(256), 0, st, g,
                       (E*)fields);
    hipLaunchKernelGGL((k_halo_z<E, V>), blocks(w * (g.mxy / V)), dim3(256), 0, st, g,
                       (E*)fields);
}

}  // namespace

hipError_t launch_halo(const Grid& g, void* fields, int elem_size, hipStream_t st)
{
    const bool vec = g.mx % 2 == 0;
    if (elem_size == 8) {
        if (vec) launch_halo_typed<uint64_t, 2>(g, fields, st);
        else launch_halo_typed<uint64_t, 1>(g, fields, st);
    } else {
        if (vec) launch_halo_typed<uint32_t, 2>(g, fields, st);
        else launch_halo_typed<uint32_t, 1>(g, fields, st);
    }
    return hipGetLastError();
}

}  // namespace mhd
