// Packed halo segments for the segmented (inner / outer) iteration of
// Section 3.3: the 6 side and 12 edge segments of a subdomain's r-cell
// boundary layer (corners are not read by the stencil, Section 5), packed
// into one contiguous buffer, and the reverse scatter of received segments
// into the halo.
//
// Segment d, a direction in {-1, 0, 1}^3 with one or two non-zero
// components, covers per axis a:  d_a = -1: cells [0, r),  0: [0, n_a),
// +1: [n_a - r, n_a)  of the interior (what the neighbour at offset d needs),
// and its received counterpart fills the halo cells  d_a = -1: [-r, 0),
// 0: [0, n_a), +1: [n_a, n_a + r); r is the halo width.  Within a segment the layout is
// [field][z][y][x] over the segment's extents; segments follow each other in
// the fixed order of seg_table.
#include "mhd_internal.hpp"

namespace mhd {

SegTable seg_table(const Grid& g)
{
    SegTable t{};
    int k = 0;
    int64_t off = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int nnz = (dx != 0) + (dy != 0) + (dz != 0);
                if (nnz == 0 || nnz == 3) continue;
                const int d[3] = {dx, dy, dz}, n[3] = {g.nx, g.ny, g.nz};
                int64_t cells = 1;
                for (int a = 0; a < 3; ++a) {
                    t.dir[k][a] = d[a];
                    t.len[k][a] = d[a] == 0 ? n[a] : g.r;
                    cells *= t.len[k][a];
                }
                t.off[k] = off;
                off += NQ * cells;
                ++k;
            }
    t.off[NSEG] = off;
    return t;
}

namespace {

constexpr int SEG_THREADS = 256;

// Launch geometry: per segment its first workgroup, buffer offset, extents,
// the interior start of its packed cells and of its halo cells, and the
// lanes given to one x-row of the segment (the power of two >= its x length,
// at most SEG_THREADS; a workgroup covers SEG_THREADS / lanes rows).  The
// kernel indexes it only with workgroup-uniform values, so it stays in
// scalar registers.
struct SegLaunch {
    int blk[NSEG + 1];  // blk[NSEG]: workgroups per field
    int64_t off[NSEG];
    int len[NSEG][3];
    int src[NSEG][3];
    int dst[NSEG][3];
    int lanes_log2[NSEG];
};

SegLaunch seg_launch(const Grid& g, const SegTable& t)
{
    SegLaunch L{};
    const int n[3] = {g.nx, g.ny, g.nz};
    int blocks = 0;
    for (int k = 0; k < NSEG; ++k) {
        L.blk[k] = blocks;
        L.off[k] = t.off[k];
        int lg = 0;
        while ((1 << lg) < t.len[k][0] && (1 << lg) < SEG_THREADS) ++lg;
        L.lanes_log2[k] = lg;
        const int64_t rows = (int64_t)t.len[k][1] * t.len[k][2];
        const int rows_per_block = SEG_THREADS >> lg;
        blocks += (int)((rows + rows_per_block - 1) / rows_per_block);
        for (int a = 0; a < 3; ++a) {
            const int d = t.dir[k][a];
            L.len[k][a] = t.len[k][a];
            L.src[k][a] = d == 0 ? 0 : d < 0 ? 0 : n[a] - g.r;
            L.dst[k][a] = d == 0 ? 0 : d < 0 ? -g.r : n[a];
        }
    }
    L.blk[NSEG] = blocks;
    return L;
}

// A workgroup copies whole x-rows of one segment and field (blockIdx.y is the
// field, so every index within a field fits 32 bits): each row gets
// 2^lanes_log2 consecutive lanes, which step through it, so consecutive lanes
// touch consecutive cells on both sides.  UNPACK false: boundary layer ->
// buffer, true: buffer -> halo.
template <typename T, bool UNPACK>
__global__ __launch_bounds__(SEG_THREADS) void k_segments(Grid g, SegLaunch L,
                                                           T* __restrict__ grid_fields,
                                                           T* __restrict__ buf)
{
    const int b = blockIdx.x;
    int k = 0;
#pragma unroll
    for (int j = 1; j < NSEG; ++j) k += b >= L.blk[j];
    const int lx = L.len[k][0], ly = L.len[k][1], lz = L.len[k][2];
    const int lg = L.lanes_log2[k];
    const int lanes = 1 << lg;
    const int row = (b - L.blk[k]) * (SEG_THREADS >> lg) + (threadIdx.x >> lg);
    if (row >= ly * lz) return;
    const int z = row / ly, y = row - z * ly;
    const int q = blockIdx.y;
    const int cy = (UNPACK ? L.dst[k][1] : L.src[k][1]) + y;
    const int cz = (UNPACK ? L.dst[k][2] : L.src[k][2]) + z;
    const int cx0 = UNPACK ? L.dst[k][0] : L.src[k][0];
    T* gp = grid_fields + (int64_t)q * g.fstride + g.interior + (int64_t)cz * g.mxy +
            (int64_t)cy * g.mx + cx0;
    T* bp = buf + L.off[k] + (int64_t)q * lx * ly * lz + (int64_t)row * lx;
    for (int x = threadIdx.x & (lanes - 1); x < lx; x += lanes) {
        if (UNPACK)
            gp[x] = bp[x];
        else
            bp[x] = gp[x];
    }
}

template <typename T>
void launch_typed(const Grid& g, const SegLaunch& L, T* fields, T* buf, bool unpack, hipStream_t st)
{
    const dim3 grid((unsigned)L.blk[NSEG], NQ), block(SEG_THREADS);
    if (unpack)
        hipLaunchKernelGGL((k_segments<T, true>), grid, block, 0, st, g, L, fields, buf);
    else
        hipLaunchKernelGGL((k_segments<T, false>), grid, block, 0, st, g, L, fields, buf);
}

}  // namespace

hipError_t launch_segments(const Grid& g, const SegTable& t, void* fields, void* buf,
                           int elem_size, bool unpack, hipStream_t st)
{
    const SegLaunch L = seg_launch(g, t);
    if (L.blk[NSEG] == 0) return hipSuccess;
    if (elem_size == 8)
        launch_typed(g, L, (double*)fields, (double*)buf, unpack, st);
    else
        launch_typed(g, L, (float*)fields, (float*)buf, unpack, st);
    return hipGetLastError();
}

}  // namespace mhd
