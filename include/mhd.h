/*
 * mhd.h -- C ABI of the fused high-order MHD RK3 substep on one MI355X (gfx950).
 *
 * The operations follow Pekkila et al., "Scalable communication for
 * high-order stencil computations using CUDA-aware MPI":
 *   - the grid is the computational domain of n_i cells per axis surrounded
 *     by a halo of r cells, r the stencil radius (Section 2, Eq. 1): order
 *     k = 2r of 2, 4, 6 (the default) or 8 (Section 4);
 *   - the periodic halo mapping is s' = ((s - r) mod n) + r (Section 3.3);
 *   - the right-hand side is the non-ideal MHD system of Appendix B
 *     (Eqs. B.1-B.4, fields of Table B.1) with central differences of
 *     order 2r on the stencil set of Section 4, Eq. (stencil-fd);
 *   - time integration is Williamson's third-order low-storage (2N)
 *     Runge-Kutta scheme (Section 4); one substep is one iterative-stencil
 *     iteration and a full step is three of them (Section 5);
 *   - single and double precision are both supported (Section 3.3).
 *
 * Conventions shared by every entry point
 *   - All pointers named `fields`, `f_in`, `f_out`, `w`, `comp` are DEVICE
 *     pointers owned by the caller, laid out as described by mhd_layout
 *     (returned by mhd_init).  The library never frees them.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call except mhd_reduce is asynchronous on that stream; a fault inside
 *     a kernel surfaces at the next synchronising call (mhd_reduce or the
 *     caller's own synchronisation).
 *   - Return values are MHD_OK (0) or one of the MHD_ERR_* codes below; no
 *     C++ exception or abort crosses the ABI.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef MHD_H
#define MHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum mhd_status {
    MHD_OK = 0,
    MHD_ERR_INVALID = 1,   /* bad argument (NULL, size, precision, aliasing, substep index) */
    MHD_ERR_NO_DEVICE = 2, /* no usable HIP device */
    MHD_ERR_DEVICE = 3,    /* a HIP runtime call or an earlier kernel failed */
    MHD_ERR_NOMEM = 4      /* device or host allocation failed */
};

/* Storage / arithmetic variants (Section 3.3: single and double precision). */
enum mhd_precision {
    MHD_F64 = 0,  /* FP64 storage and arithmetic */
    MHD_F32C = 1, /* FP32 storage; FP64 second-derivative sums; the state update
                     f <- f + beta*w is Kahan-compensated with the per-cell
                     FP32 array `comp` carried across substeps and steps */
    MHD_F32 = 2   /* plain FP32 (ablation): FP32 everywhere, no compensation */
};

/* Field order of Table B.1. */
enum mhd_field {
    MHD_LNRHO = 0, MHD_UX = 1, MHD_UY = 2, MHD_UZ = 3, MHD_SS = 4,
    MHD_AX = 5, MHD_AY = 6, MHD_AZ = 7, MHD_NFIELDS = 8
};

/* Reductions over the interior of one field (diagnostics, not per step). */
enum mhd_reduce_op {
    MHD_RED_SUM = 0,      /* sum of values */
    MHD_RED_SUMSQ = 1,    /* sum of squares */
    MHD_RED_MAXABS = 2,   /* max |value| (NaN-propagating) */
    MHD_RED_MIN = 3,
    MHD_RED_MAX = 4,
    MHD_RED_SUMEXP = 5,   /* sum of exp(value): total mass for the lnrho field */
    MHD_RED_NONFINITE = 6 /* number of NaN/Inf cells, returned as a double */
};

/* ---------------------------------------------------------------- types */
/* Which fused-substep kernel runs (same results up to rounding order).
 * All three serve every order and precision.
 * AUTO: init picks the fastest for the precision and order (SPLIT for
 * MHD_F64 at every order and for MHD_F32C / MHD_F32 at order 8, TILED
 * otherwise) and reports it in mhd_layout.kernel. */
enum mhd_kernel {
    MHD_KERNEL_TILED = 0,  /* LDS-tiled z-marching kernel */
    MHD_KERNEL_DIRECT = 1, /* one thread per cell, stencil read from global memory */
    MHD_KERNEL_SPLIT = 2,  /* LDS-tiled z-march, two threads per cell splitting the
                              fields (velocity side / entropy-induction side) */
    MHD_KERNEL_AUTO = 3
};

typedef struct mhd_config {
    int32_t nx, ny, nz;   /* computational domain n_i >= 1 (interior cells per axis) */
    int32_t precision;    /* enum mhd_precision */
    int32_t kernel;       /* enum mhd_kernel */
    int32_t order;        /* stencil order k = 2r: 2, 4, 6 or 8 (Section 4); the
                             halo and the stencil radius are r = order/2 */
    double lx, ly, lz;    /* box lengths; h_i = l_i / n_i (vertex-centred cells) */
    /* Appendix B constants: adiabatic sound speed at ln rho = lnrho0, s = 0;
     * adiabatic index; heat capacity at constant pressure; reference ln rho;
     * vacuum permeability; kinematic viscosity; bulk viscosity; magnetic
     * diffusivity; radiative thermal conductivity (constant). */
    double cs0, gamma, cp, lnrho0, mu0, nu, zeta, eta, K;
    double bext[3];       /* uniform field added to curl A (zero by default) */
    double heat, cool;    /* explicit heating H and cooling C of Eq. B.3, taken
                             spatially uniform (the paper gives no model; 0 by
                             default) */
} mhd_config;

/* Geometry of every buffer the caller allocates (f, w, comp), with a halo
 * of r = order/2 cells.  Element (q, z, y, x) of the padded grid,
 * 0 <= x < mx etc., is at element index q*field_stride + (z*my + y)*mx + x;
 * interior cell (i, j, k) is at padded (i + r, j + r, k + r), i.e.
 * interior_offset + (k*my + j)*mx + i within its field.  A buffer holds
 * total_elems elements of elem_size bytes and must be at least 256-byte
 * aligned. */
typedef struct mhd_layout {
    int64_t mx, my, mz;         /* padded extents n_i + 2r */
    int64_t field_stride;       /* elements between fields (>= mx*my*mz) */
    int64_t elem_size;          /* 8 for MHD_F64, 4 otherwise */
    int64_t interior_offset;    /* (r*my + r)*mx + r */
    int64_t total_elems;        /* 8 * field_stride */
    int64_t halo;               /* r */
    int64_t kernel;             /* the fused kernel in use (enum mhd_kernel, never AUTO) */
} mhd_layout;

typedef struct mhd_ctx mhd_ctx;

/* A sub-box of the interior in interior cell indices, half-open:
 * x0 <= x < x1, y0 <= y < y1, z0 <= z < z1 (0 <= x0 <= x1 <= nx, ...). */
typedef struct mhd_box {
    int32_t x0, x1, y0, y1, z0, z1;
} mhd_box;

/* ------------------------------------------------------------ functions */

/* Fill *cfg with the defaults for an n = (nx, ny, nz) grid: l = 2*pi per
 * axis, cs0 = 1, gamma = 5/3, cp = 1, lnrho0 = 0, mu0 = 1,
 * nu = eta = 5e-3, zeta = 0, K = 5e-3, bext = 0, heat = cool = 0, order = 6,
 * kernel = MHD_KERNEL_AUTO.  Never fails. */
void mhd_config_default(mhd_config *cfg, int32_t nx, int32_t ny, int32_t nz,
                        int32_t precision);

/* Validate *cfg, bind the current HIP device and create a context.
 * Writes the buffer geometry to *layout.  *out stays NULL on failure.
 * Errors: MHD_ERR_INVALID (NULL argument, n_i < 1, a padded field of more
 * than 2^31 - 4096 cells or of 4 GiB or more (the kernels address within a
 * field with 32-bit offsets), ny or nz above 65535, non-finite or
 * non-positive lengths, gamma <= 1,
 * cp <= 0, mu0 == 0, unknown precision or kernel, order not in
 * {2, 4, 6, 8}, a kernel not built for the order and precision),
 * MHD_ERR_NO_DEVICE, MHD_ERR_DEVICE, MHD_ERR_NOMEM. */
int mhd_init(const mhd_config *cfg, mhd_ctx **out, mhd_layout *layout);

/* Release the context and its device scratch (NULL-safe). */
void mhd_finalize(mhd_ctx *ctx);

/* Static description of a status code. */
const char *mhd_strerror(int status);

/* Periodic halo fill of all 8 fields in place (Section 3.3): every halo
 * cell (x, y, z) of the padded grid receives the interior cell obtained by
 * mapping each coordinate s with ((s - r) mod n) + r, r = order/2 the halo
 * width (mhd_layout.halo); edges and corners included.
 * Errors: MHD_ERR_INVALID (NULL). */
int mhd_halo_periodic(mhd_ctx *ctx, void *fields, void *stream);

/* One RK3 substep s in {0, 1, 2} (Section 4; Appendix B):
 *   w     <- alpha_s * w + dt * RHS(f_in)   (alpha_0 = 0: w is not read)
 *   f_out <- f_in + beta_s * w
 * on the interior; alpha = (0, -5/9, -153/128), beta = (1/3, 15/16, 8/15).
 * Precondition: the halo of f_in is filled.  The halo of f_out is left
 * untouched.  For MHD_F32C the update of f_out is compensated with `comp`
 * (read and written at the interior; zero it before the first substep);
 * comp may be NULL for the other precisions.  f_in must not alias f_out,
 * w or comp.  Errors: MHD_ERR_INVALID (s out of range, NULL, aliasing,
 * non-finite dt). */
int mhd_rk3_substep(mhd_ctx *ctx, int32_t s, const void *f_in, void *f_out, void *w,
                    void *comp, double dt, void *stream);

/* nsteps full RK3 steps (Section 5: each step is three substeps), each
 * substep preceded by mhd_halo_periodic on the current buffer.  Starts
 * from f[*cur] and ping-pongs between f[0] and f[1]; on return *cur names
 * the buffer holding the result (it flips once per step).  Small grids are
 * replayed from a captured HIP graph.  Errors: as mhd_rk3_substep, and
 * MHD_ERR_INVALID for nsteps < 0 or *cur not in {0, 1}. */
int mhd_step(mhd_ctx *ctx, void *const f[2], int32_t *cur, void *w, void *comp, double dt,
             int32_t nsteps, void *stream);

/* ------------------------------------------------ segmented iteration
 * The iteration of Section 3.3 (Fig. concurrency): pack the 6 side and 12
 * edge segments of the r-cell boundary layer (corners are not needed by
 * the stencil, Section 5) into a send buffer, exchange them with the
 * neighbouring subdomains while the inner box (cells at least r from every
 * face, which read no halo) is updated, unpack the received segments into
 * the halo, then update the outer shell.  On one GPU with periodic
 * boundaries the neighbour in every direction is the subdomain itself, so
 * the exchange is a device-to-device copy of each segment to the slot of
 * the opposite direction (where several GPUs would exchange peer to peer).
 * Every entry point here requires nx, ny, nz >= r (else MHD_ERR_INVALID). */

/* Elements of one packed buffer (all 8 fields, 18 segments; bytes =
 * elements * layout.elem_size).  Segment order: directions d in
 * {-1,0,1}^3 with one or two non-zero components, z slowest then y then x;
 * each segment [field][z][y][x] over its extents (r along every non-zero
 * component of d, n along the others).  -1 for a NULL ctx. */
int64_t mhd_halo_segment_elems(const mhd_ctx *ctx);

/* Pack the boundary layer of `fields` (interior cells within r of the face
 * or edge in direction d, for every segment d) into `sendbuf` (device,
 * mhd_halo_segment_elems elements of the storage type). */
int mhd_halo_pack(mhd_ctx *ctx, const void *fields, void *sendbuf, void *stream);

/* Scatter received segments into the halo of `fields`: segment d of
 * `recvbuf` fills the halo cells beyond the face or edge in direction d. */
int mhd_halo_unpack(mhd_ctx *ctx, const void *recvbuf, void *fields, void *stream);

/* Pack, the periodic one-GPU exchange (received segment d = sent segment
 * -d) and unpack, on `stream`: afterwards every side and edge halo cell of
 * `fields` equals what mhd_halo_periodic writes there (3D corner cells are
 * not written).  sendbuf and recvbuf must differ. */
int mhd_halo_exchange_self(mhd_ctx *ctx, void *fields, void *sendbuf, void *recvbuf,
                           void *stream);

/* mhd_rk3_substep restricted to the interior cells of `box`; every other
 * cell of f_out, w and comp is left untouched.  Precondition: every cell
 * within r of the box (halo included) holds current values.  Errors: as
 * mhd_rk3_substep, and MHD_ERR_INVALID for a NULL or out-of-range box. */
int mhd_rk3_substep_box(mhd_ctx *ctx, int32_t s, const mhd_box *box, const void *f_in,
                        void *f_out, void *w, void *comp, double dt, void *stream);

/* mhd_step with the segmented iteration.  Per substep: the boundary
 * segments of the input are packed on `stream`; the exchange and unpack
 * (as mhd_halo_exchange_self) run on `comm_stream` while the inner box is
 * updated on `stream`; the six outer slabs follow on `stream`, in one launch,
 * once the halo is in.  The inner box keeps r cells from the z faces, 32 from the x faces
 * and 8 from the y faces (whole tiles of the fused kernels); on return all
 * work of `comm_stream` is ordered before the rest of `stream`.  Results are
 * identical to mhd_step's, bit for bit.  sendbuf, recvbuf: device buffers of
 * mhd_halo_segment_elems elements.  Calls on one context must not overlap.
 * Errors: as mhd_step, and MHD_ERR_INVALID for missing or equal buffers or a
 * grid below r cells. */
int mhd_step_segmented(mhd_ctx *ctx, void *const f[2], int32_t *cur, void *w, void *comp,
                       double dt, int32_t nsteps, void *sendbuf, void *recvbuf, void *stream,
                       void *comm_stream);

/* Deterministic reduction `op` (enum mhd_reduce_op) over the interior of
 * field `field` of `fields`, accumulated in FP64 in a fixed order; the
 * result is written to *out_host.  Synchronises `stream`; reports an
 * earlier asynchronous kernel fault on it as MHD_ERR_DEVICE.
 * Errors: MHD_ERR_INVALID (NULL, field or op out of range). */
int mhd_reduce(mhd_ctx *ctx, const void *fields, int32_t field, int32_t op,
               double *out_host, void *stream);

/* ------------------------------------------------------- measurement
 * Achievable HBM bandwidth, the practical ceiling beside the 8 TB/s peak
 * (Section 5 confirms bandwidth figures by measurement).  One launch of a
 * plain streaming kernel over arrays of `bytes` bytes (a multiple of 16):
 *   MHD_BW_COPY     c = a               (bytes read, bytes written)
 *   MHD_BW_TRIAD    c = a + 3 * b, FP64 (2 * bytes read, bytes written)
 * and the same with non-temporal loads and stores (_NT).  a, b, c: device
 * buffers owned by the caller, b unused by the copies; c must not alias a
 * or b.  Asynchronous on `stream`.  Errors: MHD_ERR_INVALID (unknown kind,
 * NULL, aliasing, size), MHD_ERR_DEVICE (launch failure). */
enum mhd_bandwidth_kind {
    MHD_BW_COPY = 0, MHD_BW_COPY_NT = 1, MHD_BW_TRIAD = 2, MHD_BW_TRIAD_NT = 3
};
int mhd_bandwidth_probe(int32_t kind, const void *a, const void *b, void *c, int64_t bytes,
                        void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MHD_H */
