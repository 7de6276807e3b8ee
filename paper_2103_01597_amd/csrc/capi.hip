// C ABI of the MHD library (declared in include/mhd.h): argument checks,
// the context, and the host-side step driver.  Every step of the path runs
// in the HIP kernels of this library; the host only validates and launches.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "mhd_internal.hpp"

namespace mhd {
hipError_t launch_rk3_direct(const Grid& g, const Phys& P, int precision, const Box& bx, int s,
                             const void* f_in, void* f_out, void* w, void* comp, double dt,
                             hipStream_t st);
hipError_t launch_rk3_tiled(const Grid& g, const Phys& P, int precision, const Box* bx, int nbox,
                            int s, const void* f_in, void* f_out, void* w, void* comp, double dt,
                            hipStream_t st);
hipError_t launch_rk3_split(const Grid& g, const Phys& P, const Phys* P_dev, int precision,
                            const Box* bx, int nbox, int s, const void* f_in, void* f_out,
                            void* w, void* comp, double dt, hipStream_t st);
}  // namespace mhd

using namespace mhd;

// One captured step (halo + substep, three times) per starting buffer.
struct StepGraph {
    hipGraphExec_t exec = nullptr;
    const void* f0 = nullptr;
    const void* f1 = nullptr;
    const void* w = nullptr;
    const void* comp = nullptr;
    double dt = 0.0;
};

struct mhd_ctx {
    mhd_config cfg;
    mhd_layout lay;
    Grid grid;
    Phys phys;
    Phys* phys_dev;        // device copy of phys (read by the split kernel)
    SegTable seg;          // packed halo segments of this grid
    hipEvent_t ev_ready;   // segmented step: a substep's segments are packed
    hipEvent_t ev_halo;    // segmented step: its halo has been unpacked
    int device;
    double* red_partials;  // device, REDUCE_BLOCKS doubles, then 1 result
    double* red_host;      // pinned host, 1 double
    hipStream_t capture_stream;
    StepGraph graphs[2];   // indexed by the starting buffer
    bool use_graphs;
};

namespace {

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int validate(const mhd_config* c)
{
    if (!c) return MHD_ERR_INVALID;
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return MHD_ERR_INVALID;
    if (c->precision < MHD_F64 || c->precision > MHD_F32) return MHD_ERR_INVALID;
    if (c->kernel < MHD_KERNEL_TILED || c->kernel > MHD_KERNEL_AUTO) return MHD_ERR_INVALID;
    if (c->order != 2 && c->order != 4 && c->order != 6 && c->order != 8) return MHD_ERR_INVALID;
    if (!finite_pos(c->lx) || !finite_pos(c->ly) || !finite_pos(c->lz)) return MHD_ERR_INVALID;
    if (!isfinite(c->gamma) || c->gamma <= 1.0) return MHD_ERR_INVALID;
    if (!finite_pos(c->cp) || !isfinite(c->cs0) || !isfinite(c->lnrho0)) return MHD_ERR_INVALID;
    if (!isfinite(c->mu0) || c->mu0 == 0.0) return MHD_ERR_INVALID;
    const double rest[5] = {c->nu, c->zeta, c->eta, c->K, 0.0};
    for (double v : rest)
        if (!isfinite(v)) return MHD_ERR_INVALID;
    for (double v : c->bext)
        if (!isfinite(v)) return MHD_ERR_INVALID;
    if (!isfinite(c->heat) || !isfinite(c->cool)) return MHD_ERR_INVALID;
    // every padded field must be addressable with 32-bit offsets
    const int64_t mx = c->nx + c->order, my = c->ny + c->order, mz = c->nz + c->order;
    if (mx * my * mz > (int64_t)INT32_MAX - 4096) return MHD_ERR_INVALID;
    // and every padded field must be byte-addressable with 32-bit offsets
    const int64_t elem = c->precision == MHD_F64 ? 8 : 4;
    if ((mx * my * mz + 64) * elem > ((int64_t)1 << 32) - 65536) return MHD_ERR_INVALID;
    if (c->nz > 65535 || c->ny > 65535) return MHD_ERR_INVALID;
    return MHD_OK;
}

int from_hip(hipError_t e)
{
    if (e == hipSuccess) return MHD_OK;
    if (e == hipErrorOutOfMemory) return MHD_ERR_NOMEM;
    return MHD_ERR_DEVICE;
}

void drop_graph(StepGraph& gr)
{
    if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
    gr = StepGraph{};
}

// One launch of the fused kernel over up to six disjoint boxes (the direct
// kernel: one launch per box); empty boxes are dropped.
int one_substep(mhd_ctx* ctx, int s, const Box* boxes, int nbox, const void* f_in, void* f_out,
                void* w, void* comp, double dt, hipStream_t st)
{
    Box bx[6];
    int n = 0;
    for (int k = 0; k < nbox && n < 6; ++k)
        if (boxes[k].x1 > boxes[k].x0 && boxes[k].y1 > boxes[k].y0 && boxes[k].z1 > boxes[k].z0)
            bx[n++] = boxes[k];
    if (n == 0) return MHD_OK;
    const Grid& g = ctx->grid;
    const int prec = ctx->cfg.precision;
    hipError_t e = hipSuccess;
    switch (ctx->cfg.kernel) {
    case MHD_KERNEL_TILED:
        e = launch_rk3_tiled(g, ctx->phys, prec, bx, n, s, f_in, f_out, w, comp, dt, st);
        break;
    case MHD_KERNEL_SPLIT:
        e = launch_rk3_split(g, ctx->phys, ctx->phys_dev, prec, bx, n, s, f_in, f_out, w, comp,
                             dt, st);
        break;
    default:
        for (int k = 0; k < n && e == hipSuccess; ++k)
            e = launch_rk3_direct(g, ctx->phys, prec, bx[k], s, f_in, f_out, w, comp, dt, st);
        break;
    }
    return from_hip(e);
}

int one_substep(mhd_ctx* ctx, int s, const Box& bx, const void* f_in, void* f_out, void* w,
                void* comp, double dt, hipStream_t st)
{
    return one_substep(ctx, s, &bx, 1, f_in, f_out, w, comp, dt, st);
}

int one_substep(mhd_ctx* ctx, int s, const void* f_in, void* f_out, void* w, void* comp,
                double dt, hipStream_t st)
{
    return one_substep(ctx, s, full_box(ctx->grid), f_in, f_out, w, comp, dt, st);
}

// The interior split of the segmented iteration (Section 3.3): the inner box,
// which reads no halo, and the six slabs of the outer shell (z faces over the
// whole plane, then y faces, then x faces), disjoint and together the whole
// interior.  The shell is r planes thick at the z faces but a whole tile
// (OUTER_X columns, OUTER_Y rows) at the x and y faces: the fused kernels
// march in z over 32 x 8 tiles, and a slab thinner than a tile would leave
// most of each tile's lanes idle.  Empty boxes are skipped by one_substep.
constexpr int OUTER_X = 32, OUTER_Y = 8;
void inner_outer(const Grid& g, Box& inner, Box outer[6])
{
    auto lo = [](int n, int w) { return n < w ? n : w; };
    auto hi = [&](int n, int w) { return n - w > lo(n, w) ? n - w : lo(n, w); };
    const int xa = lo(g.nx, OUTER_X), xb = hi(g.nx, OUTER_X), ya = lo(g.ny, OUTER_Y),
              yb = hi(g.ny, OUTER_Y), za = lo(g.nz, g.r), zb = hi(g.nz, g.r);
    inner = Box{xa, xb, ya, yb, za, zb};
    outer[0] = Box{0, g.nx, 0, g.ny, 0, za};
    outer[1] = Box{0, g.nx, 0, g.ny, zb, g.nz};
    outer[2] = Box{0, g.nx, 0, ya, za, zb};
    outer[3] = Box{0, g.nx, yb, g.ny, za, zb};
    outer[4] = Box{0, xa, ya, yb, za, zb};
    outer[5] = Box{xb, g.nx, ya, yb, za, zb};
}

// Exchange with the periodic neighbour (on one GPU: this subdomain itself, so
// received segment k is sent segment NSEG-1-k, direction -d) and unpack, on
// `st`; the segments must already be packed into sendbuf.
int exchange_unpack(mhd_ctx* ctx, void* fields, void* sendbuf, void* recvbuf, hipStream_t st)
{
    const int es = (int)ctx->lay.elem_size;
    hipError_t e = hipSuccess;
    for (int k = 0; k < NSEG && e == hipSuccess; ++k) {
        const int src = NSEG - 1 - k;
        e = hipMemcpyAsync((char*)recvbuf + ctx->seg.off[k] * es, (char*)sendbuf + ctx->seg.off[src] * es,
                           (size_t)(ctx->seg.off[k + 1] - ctx->seg.off[k]) * es,
                           hipMemcpyDeviceToDevice, st);
    }
    if (e == hipSuccess) e = launch_segments(ctx->grid, ctx->seg, fields, recvbuf, es, true, st);
    return from_hip(e);
}

int halo_exchange(mhd_ctx* ctx, void* fields, void* sendbuf, void* recvbuf, hipStream_t st)
{
    const hipError_t e = launch_segments(ctx->grid, ctx->seg, fields, sendbuf,
                                         (int)ctx->lay.elem_size, false, st);
    if (e != hipSuccess) return from_hip(e);
    return exchange_unpack(ctx, fields, sendbuf, recvbuf, st);
}

int substep_args_ok(mhd_ctx* ctx, int32_t s, const void* f_in, const void* f_out, const void* w,
                    const void* comp, double dt)
{
    if (!ctx || !f_in || !f_out || !w) return MHD_ERR_INVALID;
    if (s < 0 || s > 2 || !isfinite(dt)) return MHD_ERR_INVALID;
    if (ctx->cfg.precision == MHD_F32C && !comp) return MHD_ERR_INVALID;
    if (f_in == f_out || f_in == w || f_out == w) return MHD_ERR_INVALID;
    if (comp && (comp == f_in || comp == f_out || comp == w)) return MHD_ERR_INVALID;
    return MHD_OK;
}

// Three substeps from buffer `cur`, each after a halo fill of its input.
int step_once(mhd_ctx* ctx, void* const f[2], int cur, void* w, void* comp, double dt,
              hipStream_t st)
{
    for (int s = 0; s < 3; ++s) {
        hipError_t e = launch_halo(ctx->grid, f[cur], (int)ctx->lay.elem_size, st);
        if (e != hipSuccess) return from_hip(e);
        int rc = one_substep(ctx, s, f[cur], f[1 - cur], w, comp, dt, st);
        if (rc != MHD_OK) return rc;
        cur ^= 1;
    }
    return MHD_OK;
}

int ensure_graph(mhd_ctx* ctx, void* const f[2], int cur, void* w, void* comp, double dt)
{
    StepGraph& gr = ctx->graphs[cur];
    if (gr.exec && gr.f0 == f[0] && gr.f1 == f[1] && gr.w == w && gr.comp == comp && gr.dt == dt)
        return MHD_OK;
    drop_graph(gr);
    hipStream_t cs = ctx->capture_stream;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return from_hip(e);
    int rc = step_once(ctx, f, cur, w, comp, dt, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (rc != MHD_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != MHD_OK ? rc : from_hip(e);
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return from_hip(e);
    gr.exec = exec;
    gr.f0 = f[0];
    gr.f1 = f[1];
    gr.w = w;
    gr.comp = comp;
    gr.dt = dt;
    return MHD_OK;
}

}  // namespace

namespace mhd {
// Read-only access to a context's geometry for the closure kernels.
const Grid* ctx_grid(const mhd_ctx* ctx) { return &ctx->grid; }
int ctx_precision(const mhd_ctx* ctx) { return ctx->cfg.precision; }
}  // namespace mhd

extern "C" {

void mhd_config_default(mhd_config* cfg, int32_t nx, int32_t ny, int32_t nz, int32_t precision)
{
    if (!cfg) return;
    memset(cfg, 0, sizeof *cfg);
    cfg->nx = nx;
    cfg->ny = ny;
    cfg->nz = nz;
    cfg->precision = precision;
    cfg->lx = cfg->ly = cfg->lz = 2.0 * M_PI;
    cfg->cs0 = 1.0;
    cfg->gamma = 5.0 / 3.0;
    cfg->cp = 1.0;
    cfg->lnrho0 = 0.0;
    cfg->mu0 = 1.0;
    cfg->nu = 5e-3;
    cfg->zeta = 0.0;
    cfg->eta = 5e-3;
    cfg->K = 5e-3;
    cfg->order = 6;
    cfg->kernel = MHD_KERNEL_AUTO;
}

const char* mhd_strerror(int status)
{
    switch (status) {
    case MHD_OK: return "ok";
    case MHD_ERR_INVALID: return "invalid argument";
    case MHD_ERR_NO_DEVICE: return "no usable HIP device";
    case MHD_ERR_DEVICE: return "HIP runtime or kernel failure";
    case MHD_ERR_NOMEM: return "out of memory";
    default: return "unknown status";
    }
}

int mhd_init(const mhd_config* cfg, mhd_ctx** out, mhd_layout* layout)
{
    if (!out || !layout) return MHD_ERR_INVALID;
    *out = nullptr;
    int rc = validate(cfg);
    if (rc != MHD_OK) return rc;

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return MHD_ERR_NO_DEVICE;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MHD_ERR_DEVICE;

    mhd_ctx* ctx = new (std::nothrow) mhd_ctx();
    if (!ctx) return MHD_ERR_NOMEM;
    ctx->cfg = *cfg;
    ctx->device = dev;

    // AUTO: the fastest kernel built for the precision and order (measured
    // at 512^3 and 256^3 on MI355X): SPLIT for FP64 at every order and for
    // the FP32 variants at order 8, TILED otherwise
    if (cfg->kernel == MHD_KERNEL_AUTO) {
        const bool split = cfg->precision == MHD_F64 || cfg->order == 8;
        ctx->cfg.kernel = split ? MHD_KERNEL_SPLIT : MHD_KERNEL_TILED;
    }
    const int r = cfg->order / 2;
    mhd_layout& L = ctx->lay;
    L.mx = cfg->nx + 2 * r;
    L.my = cfg->ny + 2 * r;
    L.mz = cfg->nz + 2 * r;
    const int64_t cells = L.mx * L.my * L.mz;
    L.field_stride = (cells + 63) / 64 * 64;
    L.elem_size = cfg->precision == MHD_F64 ? 8 : 4;
    L.interior_offset = (r * L.my + r) * L.mx + r;
    L.total_elems = NQ * L.field_stride;
    L.halo = r;
    L.kernel = ctx->cfg.kernel;

    Grid& g = ctx->grid;
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.nz = cfg->nz;
    g.mx = (int)L.mx;
    g.my = (int)L.my;
    g.mz = (int)L.mz;
    g.fstride = L.field_stride;
    g.mxy = (int)(L.mx * L.my);
    g.interior = (int)L.interior_offset;
    g.r = r;

    Phys& P = ctx->phys;
    P.inv_h[0] = cfg->nx / cfg->lx;
    P.inv_h[1] = cfg->ny / cfg->ly;
    P.inv_h[2] = cfg->nz / cfg->lz;
    P.cs0sq = cfg->cs0 * cfg->cs0;
    P.gamma = cfg->gamma;
    P.inv_cp = 1.0 / cfg->cp;
    P.lnrho0 = cfg->lnrho0;
    P.mu0 = cfg->mu0;
    P.inv_mu0 = 1.0 / cfg->mu0;
    P.nu = cfg->nu;
    P.zeta = cfg->zeta;
    P.eta = cfg->eta;
    P.K = cfg->K;
    for (int a = 0; a < 3; ++a) P.bext[a] = cfg->bext[a];
    P.gamma_m1 = cfg->gamma - 1.0;
    P.cp_gm1 = cfg->cp * (cfg->gamma - 1.0);
    P.hc = cfg->heat - cfg->cool;

    hipError_t e = hipMalloc(&ctx->red_partials, (REDUCE_BLOCKS + 1) * sizeof(double));
    ctx->seg = seg_table(ctx->grid);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_halo, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&ctx->phys_dev, sizeof(Phys));
    if (e == hipSuccess) e = hipMemcpy(ctx->phys_dev, &ctx->phys, sizeof(Phys), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->red_host, sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        rc = from_hip(e);
        mhd_finalize(ctx);
        return rc;
    }
    // capture-and-replay pays off where launch latency rivals kernel time
    ctx->use_graphs = (int64_t)cfg->nx * cfg->ny * cfg->nz <= (int64_t)128 * 128 * 128;
    *layout = L;
    *out = ctx;
    return MHD_OK;
}

void mhd_finalize(mhd_ctx* ctx)
{
    if (!ctx) return;
    for (auto& gr : ctx->graphs) drop_graph(gr);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->red_partials) (void)hipFree(ctx->red_partials);
    if (ctx->phys_dev) (void)hipFree(ctx->phys_dev);
    if (ctx->ev_ready) (void)hipEventDestroy(ctx->ev_ready);
    if (ctx->ev_halo) (void)hipEventDestroy(ctx->ev_halo);
    if (ctx->red_host) (void)hipHostFree(ctx->red_host);
    delete ctx;
}

int mhd_halo_periodic(mhd_ctx* ctx, void* fields, void* stream)
{
    if (!ctx || !fields) return MHD_ERR_INVALID;
    return from_hip(launch_halo(ctx->grid, fields, (int)ctx->lay.elem_size, (hipStream_t)stream));
}

int mhd_rk3_substep(mhd_ctx* ctx, int32_t s, const void* f_in, void* f_out, void* w, void* comp,
                    double dt, void* stream)
{
    int rc = substep_args_ok(ctx, s, f_in, f_out, w, comp, dt);
    if (rc != MHD_OK) return rc;
    if (ctx->cfg.precision != MHD_F32C) comp = nullptr;
    return one_substep(ctx, s, f_in, f_out, w, comp, dt, (hipStream_t)stream);
}

int mhd_step(mhd_ctx* ctx, void* const f[2], int32_t* cur, void* w, void* comp, double dt,
             int32_t nsteps, void* stream)
{
    if (!ctx || !f || !cur || nsteps < 0 || (*cur != 0 && *cur != 1)) return MHD_ERR_INVALID;
    int rc = substep_args_ok(ctx, 0, f[0], f[1], w, comp, dt);
    if (rc != MHD_OK) return rc;
    if (ctx->cfg.precision != MHD_F32C) comp = nullptr;
    hipStream_t st = (hipStream_t)stream;
    int c = *cur;
    for (int32_t t = 0; t < nsteps; ++t) {
        if (ctx->use_graphs) {
            rc = ensure_graph(ctx, f, c, w, comp, dt);
            if (rc != MHD_OK) return rc;
            rc = from_hip(hipGraphLaunch(ctx->graphs[c].exec, st));
        } else {
            rc = step_once(ctx, f, c, w, comp, dt, st);
        }
        if (rc != MHD_OK) return rc;
        c ^= 1;  // three swaps per step
        *cur = c;
    }
    return MHD_OK;
}

int mhd_rk3_substep_box(mhd_ctx* ctx, int32_t s, const mhd_box* box, const void* f_in,
                        void* f_out, void* w, void* comp, double dt, void* stream)
{
    int rc = substep_args_ok(ctx, s, f_in, f_out, w, comp, dt);
    if (rc != MHD_OK) return rc;
    if (!box) return MHD_ERR_INVALID;
    const Grid& g = ctx->grid;
    if (box->x0 < 0 || box->y0 < 0 || box->z0 < 0 || box->x1 > g.nx || box->y1 > g.ny ||
        box->z1 > g.nz || box->x0 > box->x1 || box->y0 > box->y1 || box->z0 > box->z1)
        return MHD_ERR_INVALID;
    if (ctx->cfg.precision != MHD_F32C) comp = nullptr;
    const Box bx{box->x0, box->x1, box->y0, box->y1, box->z0, box->z1};
    return one_substep(ctx, s, bx, f_in, f_out, w, comp, dt, (hipStream_t)stream);
}

int64_t mhd_halo_segment_elems(const mhd_ctx* ctx)
{
    if (!ctx) return -1;
    return ctx->seg.off[NSEG];
}

namespace {
bool exchange_ok(const mhd_ctx* ctx)
{
    const Grid& g = ctx->grid;
    return g.nx >= g.r && g.ny >= g.r && g.nz >= g.r;
}
}  // namespace

int mhd_halo_pack(mhd_ctx* ctx, const void* fields, void* sendbuf, void* stream)
{
    if (!ctx || !fields || !sendbuf || !exchange_ok(ctx)) return MHD_ERR_INVALID;
    return from_hip(launch_segments(ctx->grid, ctx->seg, const_cast<void*>(fields), sendbuf,
                                    (int)ctx->lay.elem_size, false, (hipStream_t)stream));
}

int mhd_halo_unpack(mhd_ctx* ctx, const void* recvbuf, void* fields, void* stream)
{
    if (!ctx || !fields || !recvbuf || !exchange_ok(ctx)) return MHD_ERR_INVALID;
    return from_hip(launch_segments(ctx->grid, ctx->seg, fields, const_cast<void*>(recvbuf),
                                    (int)ctx->lay.elem_size, true, (hipStream_t)stream));
}

int mhd_halo_exchange_self(mhd_ctx* ctx, void* fields, void* sendbuf, void* recvbuf,
                           void* stream)
{
    if (!ctx || !fields || !sendbuf || !recvbuf || sendbuf == recvbuf || !exchange_ok(ctx))
        return MHD_ERR_INVALID;
    return halo_exchange(ctx, fields, sendbuf, recvbuf, (hipStream_t)stream);
}

int mhd_step_segmented(mhd_ctx* ctx, void* const f[2], int32_t* cur, void* w, void* comp,
                       double dt, int32_t nsteps, void* sendbuf, void* recvbuf, void* stream,
                       void* comm_stream)
{
    if (!ctx || !f || !cur || nsteps < 0 || (*cur != 0 && *cur != 1)) return MHD_ERR_INVALID;
    int rc = substep_args_ok(ctx, 0, f[0], f[1], w, comp, dt);
    if (rc != MHD_OK) return rc;
    if (!sendbuf || !recvbuf || sendbuf == recvbuf || !exchange_ok(ctx)) return MHD_ERR_INVALID;
    if (ctx->cfg.precision != MHD_F32C) comp = nullptr;
    hipStream_t st = (hipStream_t)stream, cs = (hipStream_t)comm_stream;
    Box inner, outer[6];
    inner_outer(ctx->grid, inner, outer);
    int c = *cur;
    for (int32_t t = 0; t < nsteps; ++t) {
        for (int s = 0; s < 3; ++s) {
            // pack on the launch stream (so the exchange never waits behind
            // the inner box); exchange and unpack on comm_stream while the
            // inner box is updated; then the outer shell once the halo is in.
            // (Outer slabs on comm_stream, concurrent with the inner box,
            // measured no faster: the inner box's workgroups hold the CUs.)
            hipError_t e = launch_segments(ctx->grid, ctx->seg, f[c], sendbuf,
                                           (int)ctx->lay.elem_size, false, st);
            if (e == hipSuccess) e = hipEventRecord(ctx->ev_ready, st);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs, ctx->ev_ready, 0);
            if (e != hipSuccess) return from_hip(e);
            rc = exchange_unpack(ctx, f[c], sendbuf, recvbuf, cs);
            if (rc != MHD_OK) return rc;
            e = hipEventRecord(ctx->ev_halo, cs);
            if (e != hipSuccess) return from_hip(e);
            rc = one_substep(ctx, s, inner, f[c], f[1 - c], w, comp, dt, st);
            if (rc != MHD_OK) return rc;
            e = hipStreamWaitEvent(st, ctx->ev_halo, 0);
            if (e != hipSuccess) return from_hip(e);
            rc = one_substep(ctx, s, outer, 6, f[c], f[1 - c], w, comp, dt, st);
            if (rc != MHD_OK) return rc;
            c ^= 1;
        }
        *cur = c;
    }
    return MHD_OK;
}

int mhd_reduce(mhd_ctx* ctx, const void* fields, int32_t field, int32_t op, double* out_host,
               void* stream)
{
    if (!ctx || !fields || !out_host) return MHD_ERR_INVALID;
    if (field < 0 || field >= NQ || op < MHD_RED_SUM || op > MHD_RED_NONFINITE)
        return MHD_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const char* base = (const char*)fields + field * ctx->lay.field_stride * ctx->lay.elem_size;
    hipError_t e = launch_reduce(ctx->grid, base, (int)ctx->lay.elem_size, op, ctx->red_partials,
                                 REDUCE_BLOCKS, ctx->red_partials + REDUCE_BLOCKS, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->red_host, ctx->red_partials + REDUCE_BLOCKS, sizeof(double),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return from_hip(e);
    *out_host = *ctx->red_host;
    return MHD_OK;
}

}  // extern "C"
