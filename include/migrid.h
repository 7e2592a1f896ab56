/*
 * migrid — convolutional gridding and degridding on AMD Instinct MI355X
 * (gfx950).  C ABI.
 *
 * The operation (Muscat, "High-Performance Gridding For Radio
 * Interferometric Image Synthesis", 2021):
 *   records xi_p carry values F(xi_p) at continuous (u, v[, w]) positions;
 *   the Gridding Step convolves every record with an oversampled, lookup-
 *   table kernel and samples the result on an N x N uv-grid (Algorithm
 *   "General Convolutional Gridding", Section 2.3; oversampled kernel,
 *   Section 2.3.6 and the studied algorithm of Section 2.4.5).  Every
 *   polarisation of a record is gridded with the same weights (Section 1.1).
 *   Degridding is the adjoint map (the forward/backward operator pair of the
 *   major-cycle residual, Section 1.6), which the thesis names as future work
 *   (Section 9.1).
 *
 * Index rule (identical in every entry point, computed in FP64):
 *   x = coord * scale + n/2            cells, origin at the centre pixel
 *                                      (Section 2.1.2)
 *   q = floor(x * beta + 1/2)          nearest pixel of the beta-oversampled
 *                                      grid; rect is 1 on (-1/(2beta),
 *                                      1/(2beta)] (Section 2.1.4), so ties go up
 *   k_lo = floor((q - beta*S/2)/beta) + 1, footprint cells k_lo .. k_lo+S-1
 *                                      (offsets in (-S/2, S/2], Section 2.3.4)
 *   t0 = k_lo*beta - q + beta*S/2      in [1, beta]; cell k_lo+i takes table
 *                                      entry t0 + i*beta; o = t0 - 1
 *   W-projection plane: p = min(P-1, floor(|w| * inv_dw + 1/2)), support
 *   S_p, conjugated table for w < 0 (Section 1.3: gbar_{-w} = conj(gbar_w)).
 *   A record is skipped (and counted) unless uvw is finite and its whole
 *   footprint lies inside the grid (Bounded Records Assumption, Section
 *   2.3.1).  Each argument of the rule is formed in FP64 without fused
 *   multiply-add, so indices are reproducible bit for bit.
 *
 * Layouts:
 *   uvw      [nrec][3], F32 or F64, wavelengths
 *   vis      [nrec][npol] complex64 (re, im float pairs), npol in 1..4
 *   grid     [npol][nv][nu] complex64, u fastest, cell (nu/2, nv/2) is u=v=0
 *   separable taps: beta*S + 1 real values; entry t at offset
 *            (t - beta*S/2)/beta cells; the 2-D weight is T[tu] * T[tv]
 *   W-projection taps: planes concatenated; plane p is (beta*S_p+1)^2
 *            complex values, row-major [tv][tu], starting at element
 *            plane_offset[p]
 *   tap dtype: F32, F16 or BF16 (a complex tap is a pair of that type);
 *            arithmetic is always FP32.
 *
 * Ownership and streams:
 *   All array arguments are DEVICE pointers unless stated; the caller owns
 *   them and they must stay alive until the work queued on `stream` ends.
 *   Calls are asynchronous on `stream`.  Argument errors are returned
 *   synchronously before anything is queued; launch errors are returned as
 *   MG_EDEVICE.  The last error's text is available from mg_last_error()
 *   (thread-local).
 *
 * Accumulation: grid entry points ADD into `grid`; degrid entry points
 * OVERWRITE `vis_out` (skipped records get 0).
 */
#ifndef MIGRID_H
#define MIGRID_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_EINVAL = -1,        /* bad argument (checked on the host, nothing queued) */
    MG_ENOMEM = -2,        /* device allocation failed / over the serving budget */
    MG_EDEVICE = -3,       /* a HIP call or kernel launch failed */
    MG_EUNSUPPORTED = -4,  /* valid request this build does not handle */
    MG_EBUSY = -5          /* serving: no free slot */
} mg_status;

typedef enum { MG_F32 = 0, MG_F64 = 1, MG_F16 = 2, MG_BF16 = 3 } mg_dtype;

/* MG_KERNEL_WSTACK: W-stacking with the plain gridder (Section 1.7.1,
 * correction of the W-term in the (l, m)-plane; the W-handling route the
 * thesis names for its gridders, Section 9.1).  A separable kernel (support,
 * taps as for MG_KERNEL_SEPARABLE) and L = nplanes layers of spacing
 * dw = 1 / inv_dw centred on w_j = (j - (L-1)/2) dw: a record goes to layer
 *   j = floor(w inv_dw + L/2) clamped to [0, L-1]   (FP64, no contraction)
 * and is gridded onto that layer's own nu x nv grid (index rule, bounds and
 * skips per layer).  The layers' grids are stacked along v: grid and degrid
 * buffers are [npol][L][nv][nu] (the same memory as [npol][L nv][nu]), and
 * L nv must be at most 65535.  mg_compute_indices reports k_lo_v in the
 * stacked rows (j nv + k_lo_v) and plane -1.  Image with mg_wstack_imager_*. */
typedef enum { MG_KERNEL_SEPARABLE = 0, MG_KERNEL_WPROJ = 1, MG_KERNEL_WSTACK = 2 } mg_kernel_kind;

/* Grid geometry.  scale_* = cells per wavelength (= N x pixel size in rad,
 * the N*dl = 1 normalisation of Section 2.1.2).  nu, nv in [1, 65535]. */
typedef struct {
    int32_t nu, nv;
    int32_t npol;        /* 1..4 */
    int32_t beta;        /* oversampling factor >= 1, beta*S even */
    double scale_u, scale_v;
} mg_grid_desc;

/* Kernel bank.  plane_support / plane_offset are HOST arrays read during the
 * call (copied by plans).  taps is a DEVICE pointer. */
typedef struct {
    mg_kernel_kind kind;
    mg_dtype tap_dtype;            /* MG_F32, MG_F16 or MG_BF16 */
    int32_t support;               /* separable: S (1..64) */
    int32_t nplanes;               /* W-projection: number of planes (1..128);
                                      W-stacking: number of layers (1..128) */
    const int32_t *plane_support;  /* W-projection: S_p per plane (1..64) */
    const int64_t *plane_offset;   /* W-projection: first complex tap of plane p */
    double inv_dw;                 /* W-projection: 1 / plane spacing in w;
                                      W-stacking: 1 / layer spacing */
    const void *taps;              /* device: the table(s) */
    int64_t ntaps;                 /* elements in taps (real for separable,
                                      complex for W-projection, at most 2^30) */
} mg_kernel_desc;

/* Text of the status code. */
const char *mg_status_str(mg_status s);

/* Text of the last error set on this thread ("" if none). */
const char *mg_last_error(void);

/* Per-record integer indices of the index rule above, in input order
 * (parity and debugging): the nearest pixel of Section 2.1.4, the footprint
 * of Section 2.3.4 and the plane of Section 1.3, computed in FP64.  Outputs
 * are device arrays of nrec entries: k_lo_u, k_lo_v, o_u, o_v, plane (-1 for
 * a separable kernel), valid (0/1); k_lo and o are 0 for skipped records.
 * *d_nskipped (device, may be NULL) is INCREMENTED by the skipped count.
 * Errors: MG_EINVAL for a bad descriptor or a null output with nrec > 0. */
mg_status mg_compute_indices(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                             const void *uvw, mg_dtype uvw_dtype,
                             int32_t *k_lo_u, int32_t *k_lo_v, int32_t *o_u, int32_t *o_v,
                             int32_t *plane, uint8_t *valid, int64_t *d_nskipped,
                             hipStream_t stream);

/* ---- plans: index + sort once, grid / degrid many times (major cycles) ----
 *
 * mg_plan_create runs the index rule over all records and sorts the valid
 * ones on `stream` by uv tile and plane (the planes of one support class
 * share their tiles) and by cell inside each run of records (the thesis's
 * sorted record order, Section 3.2.4), and prepares the kernel bank: a
 * private copy re-laid so that the taps of each oversampling phase are
 * contiguous, plus its conjugate for W-projection.  A plan keeps no pointer
 * to uvw or to the caller's taps, so neither needs to outlive the create
 * call's stream work.  A plan is immutable after creation and may be used
 * from several streams once the creating stream's work has completed. */
typedef struct mg_plan mg_plan;

/* Bytes of device workspace a plan of these descriptors and nrec records
 * holds (its sorted record metadata and permutation, chunk and unit lists,
 * tap table and the build's temporaries).  Host-only: nothing is queued.
 * Errors: MG_EINVAL as mg_plan_create (uvw is not needed). */
mg_status mg_plan_workspace_size(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                                 size_t *bytes);

/* Builds a plan for the records uvw [nrec][3] (device).  workspace: device
 * memory of at least mg_plan_workspace_size bytes, 256-byte aligned, owned by
 * the caller, which keeps it alive (and unused by anything else) until the
 * plan is destroyed and the plan's queued work has completed; every device
 * array of the plan lives in it, so a caller's allocator accounts for all of
 * the plan's memory.  workspace == NULL: the library allocates it
 * stream-ordered on `stream` and releases it in mg_plan_destroy.
 * Errors: MG_EINVAL (bad descriptor, misaligned workspace), MG_ENOMEM,
 * MG_EUNSUPPORTED (tap table above 2^30 entries, too many buckets),
 * MG_EDEVICE; on error *plan is NULL and nothing remains allocated. */
mg_status mg_plan_create(mg_plan **plan, const mg_grid_desc *g, const mg_kernel_desc *k,
                         int64_t nrec, const void *uvw, mg_dtype uvw_dtype, void *workspace,
                         hipStream_t stream);

/* Gridding Step (Algorithm "General Convolutional Gridding", Section 2.3;
 * oversampled kernel as in the studied algorithm of Section 2.4.5), every
 * polarisation with the same weights (Section 1.1): grid += G vis.
 * vis: [nrec][npol] complex64 in the create call's record order; grid:
 * [npol][nv][nu] complex64.  Scratch (sorted visibilities, 32 B per record
 * and a few words per unit) is allocated and released stream-ordered inside
 * the call.  Errors: MG_EINVAL (null pointer), MG_ENOMEM, MG_EDEVICE. */
mg_status mg_plan_grid(const mg_plan *plan, const void *vis, void *grid, hipStream_t stream);

/* Degridding, the adjoint of the Gridding Step (the forward/backward pair of
 * the major-cycle residual, Section 1.6): vis_out = G^H grid, i.e.
 * vis_out[r][pol] = sum over the footprint of conj(weight) * grid (skipped
 * records get 0; overwritten).  Errors as mg_plan_grid. */
mg_status mg_plan_degrid(const mg_plan *plan, const void *grid, void *vis_out,
                         hipStream_t stream);

/* Number of records skipped by the Bounded Records rule (Section 2.3.1) or
 * for non-finite uvw; waits for the plan's creation work. */
mg_status mg_plan_nskipped(const mg_plan *plan, int64_t *nskipped);

/* Device bytes the plan holds (its workspace size). */
mg_status mg_plan_bytes(const mg_plan *plan, size_t *bytes);

/* Releases the plan.  A library-owned workspace is freed stream-ordered
 * after the plan's build and its last call on every stream it was used on
 * (no host or device-wide wait); a caller workspace is left to the caller. */
mg_status mg_plan_destroy(mg_plan *plan);

/* ---- one-shot calls: index + sort + grid (or degrid) in one go ----
 * The same maps as mg_plan_grid / mg_plan_degrid (Sections 2.3, 2.4.5, 1.6)
 * for one set of records.  The plan and the call's scratch are one
 * allocation, made and released stream-ordered inside the call.
 * *d_nskipped (device, may be NULL) is INCREMENTED by the skipped count.
 * Errors: MG_EINVAL, MG_ENOMEM, MG_EUNSUPPORTED, MG_EDEVICE. */
mg_status mg_grid(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                  const void *uvw, mg_dtype uvw_dtype, const void *vis, void *grid,
                  int64_t *d_nskipped, hipStream_t stream);

mg_status mg_degrid(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                    const void *uvw, mg_dtype uvw_dtype, const void *grid, void *vis_out,
                    int64_t *d_nskipped, hipStream_t stream);

/* ---- one-shot gridding that allocates nothing ----
 * For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and arguments as mg_grid, with the plan and the call's
 * scratch taken from a static device array of mg_grid_static_capacity()
 * bytes (64 MiB) inside the library, one per GPU, held until the process
 * ends.  No hipMalloc, hipFree or allocating library routine is called.
 * Calls that need more scratch than the array holds (about 44 bytes per
 * record plus the grid's bucket arrays and the tap table: roughly 1.3
 * million records on a 1024^2 grid) return MG_ENOMEM before anything is
 * queued, with the needed size in mg_last_error().  Every call on one GPU
 * uses the same array: calls that overlap on one GPU (different streams or
 * threads) race and must be ordered by the caller.  Errors otherwise as
 * mg_grid. */
mg_status mg_grid_static(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                         const void *uvw, mg_dtype uvw_dtype, const void *vis, void *grid,
                         int64_t *d_nskipped, hipStream_t stream);

/* Bytes of the static scratch of mg_grid_static. */
size_t mg_grid_static_capacity(void);

/* ---- Hybrid Gridding and column pruning ----
 *
 * Hybrid Gridding (Algorithm "The studied Hybrid Gridding Algorithm",
 * Section 2.4.4) splits the convolutional Gridding Step in one dimension:
 * along u a record is convolved with the separable kernel (S taps at the
 * integer cells, the index rule above), along v it is moved to the nearest
 * pixel of the beta-oversampled v axis, row q = floor(beta x_v + 1/2) with
 * x_v = v scale_v + nv/2 (nearest-neighbour interpolation, C_hy = C_co(u)
 * rect(v)).  Output grid: [npol][beta nv][nu] complex64, u fastest, column
 * nu/2 and row beta nv / 2 are u = v = 0.  A record is gridded if uvw is
 * finite, its u footprint lies inside [0, nu) and 0 <= q < beta nv;
 * otherwise it is skipped and counted.  Kernel: separable only, support
 * 1..32, taps F32/F16/BF16 (FP32 arithmetic).  Grid entry points ADD into
 * the grid.  A hybrid plan bins the records once by tile of the hybrid grid
 * (the Gridder then takes chunks of one tile); its memory is the caller's
 * workspace (mg_hybrid_plan_workspace_size bytes, 256-byte aligned, kept
 * alive until the plan is destroyed and its work has completed), or, with
 * workspace == NULL, a stream-ordered allocation released on the creating
 * stream by mg_hybrid_plan_destroy (calls on other streams must be ordered
 * before it).  Errors: MG_EINVAL (bad descriptor, non-separable kernel,
 * support above 32), MG_ENOMEM, MG_EDEVICE. */
typedef struct mg_hybrid_plan mg_hybrid_plan;

mg_status mg_hybrid_plan_workspace_size(const mg_grid_desc *g, const mg_kernel_desc *k,
                                        int64_t nrec, size_t *bytes);

mg_status mg_hybrid_plan_create(mg_hybrid_plan **plan, const mg_grid_desc *g,
                                const mg_kernel_desc *k, int64_t nrec, const void *uvw,
                                mg_dtype uvw_dtype, void *workspace, hipStream_t stream);

/* grid_hy += G_hy vis; vis [nrec][npol] complex64 in the create call's
 * order, grid_hy [npol][beta nv][nu] complex64.  Allocates nothing. */
mg_status mg_hybrid_plan_grid(const mg_hybrid_plan *plan, const void *vis, void *grid_hy,
                              hipStream_t stream);

/* Records skipped by the hybrid rule (waits for the plan's creation). */
mg_status mg_hybrid_plan_nskipped(const mg_hybrid_plan *plan, int64_t *nskipped);

mg_status mg_hybrid_plan_destroy(mg_hybrid_plan *plan);

/* One-shot Hybrid Gridding (bin + grid; scratch allocated and released
 * stream-ordered inside the call).  *d_nskipped (device, may be NULL) is
 * INCREMENTED by the skipped count. */
mg_status mg_hybrid_grid(const mg_grid_desc *g, const mg_kernel_desc *k, int64_t nrec,
                         const void *uvw, mg_dtype uvw_dtype, const void *vis, void *grid_hy,
                         int64_t *d_nskipped, hipStream_t stream);

/* Column pruning, the Pruning Step of Hybrid Gridding (Convolution-Based FFT
 * Pruning, Algorithm of Section 2.5.2, down every column as the Column
 * Pruner of Section 7.1; its output equation, Section 7.1.1): every column
 * of M = nrows values is circularly convolved with the pruning kernel and
 * downsampled by alpha,
 *   out[j] = sum_{s=0}^{Sz-1} sum_{a=0}^{alpha-1} c(alpha (s - Sz/2) + a)
 *            in[(alpha (j - Sz/2 + s) + a) mod M],   j < M / alpha,
 * c(d) = ztaps[d + alpha Sz/2] (DEVICE, FP32, alpha Sz + 1 entries; entry e
 * at offset (e - alpha Sz/2)/alpha output samples; the last is not used).
 * in: [npol][nrows][ncols] complex64; out: [npol][nrows/alpha][ncols]
 * complex64, OVERWRITTEN.  For Hybrid Gridding: nrows = beta nv, ncols =
 * nu, alpha = beta/2 (oversampling 2 after pruning), Sz even in 2..16.
 * Errors: MG_EINVAL (nrows not a multiple of alpha, Sz odd or above 16,
 * null pointer), MG_EDEVICE.  Allocates nothing. */
mg_status mg_prune_columns(int32_t npol, int64_t nrows, int32_t ncols, int32_t alpha,
                           int32_t support_z, const float *ztaps, const void *in, void *out,
                           hipStream_t stream);

/* ---- imaging chain: origin shift, inverse FFT, Correction Step ----
 *
 * The IFFT and Correction Steps of the studied algorithms (Section 2.4.5;
 * Section 2.4.4 for Hybrid Gridding).  For centred grids of even sizes the
 * image is the unnormalised inverse transform with e^{+j2pi}, centred,
 *   I[y][x] = sum_k G[kv][ku] exp(+j2pi((ku - nx/2)(x - nx/2)/nx
 *                                        + (kv - ny/2)(y - ny/2)/ny)),
 * times separable correctors corr_x[x] corr_y[y]. */

/* Corrector vector (device, n floats): h(l) = 1 / ((1/phases) sum_e T[e]
 * cos(2pi ((e - E/2)/beta) l) s(l)), l = (i - n/2)/n, where T is a
 * symmetric table of E + 1 = table_len values (DEVICE, FP32) whose entry e
 * lies (e - E/2)/beta cells from the centre, and s(l) = sinc(l/beta) (the
 * nearest-pixel snap onto the beta-oversampled grid) if nn_sinc, else 1.
 * Convolutional gridding (corrector h_co): T the kernel's beta S + 1 taps,
 * phases = beta.  Pruned hybrid v axis (h_pr): T the pruning kernel's
 * alpha Sz + 1 taps, phases = alpha.  Computed in FP64. */
mg_status mg_corrector(int32_t n, int32_t beta, int32_t table_len, int32_t phases,
                       int32_t nn_sinc, const float *table, float *corr, hipStream_t stream);

typedef struct mg_imager mg_imager;

/* An imager for [npol][ny][nx] grids (nx, ny even): holds a batched C2C FFT
 * plan of the platform library (which allocates its own work area).  One
 * stream at a time per imager. */
mg_status mg_imager_create(mg_imager **im, int32_t npol, int32_t nx, int32_t ny);

/* image = rows [y0, y0 + out_ny) of the centred inverse transform of grid
 * ([npol][ny][nx] complex64, device, read only), times corr_x[x] (nx
 * floats) and corr_y[y - y0] (out_ny floats), into image ([npol][out_ny][nx]
 * complex64).  work: [npol][ny][nx] complex64 scratch (may equal image when
 * y0 = 0 and out_ny = ny).  A pruned hybrid grid (2 nv rows, nu columns)
 * takes y0 = nv/2, out_ny = nv (the central half of its doubled field). */
mg_status mg_imager_exec(mg_imager *im, const void *grid, void *work, void *image,
                         const float *corr_x, const float *corr_y, int32_t y0, int32_t out_ny,
                         hipStream_t stream);

mg_status mg_imager_destroy(mg_imager *im);

/* ---- W-stacking image ----
 *
 * The image of MG_KERNEL_WSTACK grids (Section 1.7.1, correction of the
 * W-term in the (l, m)-plane): every layer's centred inverse transform (as
 * mg_imager_exec), multiplied by the inverse W-term of its layer
 *   gbar_{w_j}(l, m) = exp(+j2pi w_j (sqrt(1 - l^2 - m^2) - 1)),
 *   w_j = (j - (L-1)/2) dw,  l = (x - nx/2)/nx fov_x,  m = (y - ny/2)/ny fov_y
 * (fov = the radians the field spans, the grid's cells-per-wavelength
 * scale), summed over the layers and multiplied by corr_x[x] corr_y[y].
 * The screen phase is reduced in FP64, its sine and cosine taken in FP32. */
typedef struct mg_wstack_imager mg_wstack_imager;

/* An imager for [npol][layers][ny][nx] layer grids (nx, ny even): holds a
 * batched C2C FFT plan of the platform library (which allocates its own
 * work area).  One stream at a time per imager. */
mg_status mg_wstack_imager_create(mg_wstack_imager **im, int32_t npol, int32_t layers,
                                  int32_t nx, int32_t ny);

/* image ([npol][ny][nx] complex64) from grids ([npol][layers][ny][nx]
 * complex64, read only); work: scratch of the grids' size, distinct from
 * image; corr_x: nx floats, corr_y: ny floats (device).  dw: the layer
 * spacing (1 / inv_dw of the kernel descriptor). */
mg_status mg_wstack_imager_exec(mg_wstack_imager *im, const void *grids, void *work, void *image,
                                const float *corr_x, const float *corr_y, double fov_x,
                                double fov_y, double dw, hipStream_t stream);

mg_status mg_wstack_imager_destroy(mg_wstack_imager *im);

/* ---- kernel generation: W-projection kernel bank ----
 *
 * Plane p of the bank tabulates the GCF convolved with the transform of the
 * inverse W-term at w_p (Section 1.7.1, W-projection; the W-term g_w and
 * gbar_w = 1 / g_w of Section 1.3):
 *   K_p = F[ c(l) c(m) gbar_{w_p}(l, m) ],
 *   gbar_w(l, m) = exp(+j2pi w (sqrt(1 - l^2 - m^2) - 1)),
 * with c the image-domain taper of the separable GCF whose base_len =
 * beta*S0 + 1 symmetric FP64 taps (DEVICE) put entry t at
 * (t - beta*S0/2)/beta cells, and F the transform with exp(-j2pi(ul + vm)).
 * Discretisation: M = 2 beta S_p points per axis at beta/M field units,
 * physical direction cosine = field units x fov (the radians the uv grid's
 * field spans, i.e. its cells-per-wavelength scale); plane p keeps the
 * central beta S_p + 1 samples per axis, row (v offset) major: the layout
 * the gridders take.  The bank is normalised so its largest |tap| is 1.  At
 * w = 0 a plane is the outer product of the (zero-padded) base taps.
 * Computed in FP64 (the platform library's Z2Z FFT) and stored as out_dtype
 * (MG_F32: complex64; MG_F16 / MG_BF16: re, im pairs). */
mg_status mg_wkernel_bank_size(int32_t nplanes, const int32_t *plane_support, int32_t beta,
                               int64_t *bank_elems, size_t *workspace_bytes);

/* plane_support, plane_w: HOST [nplanes]; bank: DEVICE, bank_elems taps;
 * plane_offset: HOST output [nplanes], element offset of each plane;
 * workspace: DEVICE, at least the size mg_wkernel_bank_size reports (FP64
 * image grids and tapers), passed with its size, in use until the queued
 * work is done.  The work is queued on `stream` (no host copies, no
 * synchronisation); the FFT plans of the platform library (one per plane
 * size and device, created on first use) are kept for the life of the
 * process and shared, so builds on different streams of one device must not
 * overlap.  Errors: MG_EINVAL (sizes out of range, beta*S
 * odd or above 4096, a plane narrower than the base kernel, fov not
 * positive, non-finite w, null pointers, workspace too small), MG_EDEVICE. */
mg_status mg_wkernel_bank(int32_t nplanes, const int32_t *plane_support, const double *plane_w,
                          int32_t beta, int32_t base_len, const double *base_taps, double fov,
                          mg_dtype out_dtype, void *bank, int64_t *plane_offset, void *workspace,
                          size_t workspace_bytes, hipStream_t stream);

/* ---- serving: continuous batching of gridding jobs ----
 *
 * A server owns a pool of HIP streams (default priority) on one device and a
 * scheduler thread.  mg_server_submit queues a one-shot gridding job (the
 * same computation as mg_grid) and returns at once.  The scheduler admits
 * queued jobs in arrival order whenever a slot is free and the job's HBM
 * footprint fits the budget beside the jobs already running, and launches
 * each admitted job on the next stream, so the work of jobs that arrive
 * while others run overlaps on the device.  A job's footprint is its caller
 * buffers (uvw, vis, grid) plus the library scratch it needs; it is released
 * when the job completes.  The caller keeps every buffer of a job alive
 * until the job is done.  Jobs on different streams must not share an
 * output grid. */
typedef struct mg_server mg_server;

typedef enum { MG_JOB_QUEUED = 0, MG_JOB_RUNNING = 1, MG_JOB_DONE = 2, MG_JOB_FAILED = 3 } mg_job_state;

typedef struct {
    uint64_t submitted, admitted, completed, failed;
    uint64_t bytes_in_use, bytes_peak, budget;
    int32_t running, queued, max_running;
} mg_server_stats;

/* hbm_budget_bytes: admission budget; max_slots: jobs running at once
 * (1..1024); nstreams: streams in the pool (1..64); device: the HIP device
 * of the server (-1: the calling thread's current device).
 * Errors: MG_EINVAL, MG_EDEVICE. */
mg_status mg_server_create(mg_server **srv, size_t hbm_budget_bytes, int32_t max_slots,
                           int32_t nstreams, int32_t device);

/* Queues a job.  inputs_ready (may be NULL): an event recorded after the
 * work that produces the job's inputs; the job's stream waits for it before
 * starting, so the caller need not synchronise.  Returns MG_ENOMEM (nothing
 * queued) if the job alone exceeds the budget, MG_EINVAL for bad arguments
 * (as mg_grid), MG_EBUSY while the server shuts down.  *job_id receives the
 * job's id.  Every kernel kind of mg_grid is accepted (a W-stacking job's
 * grid holds its stacked layers, as for mg_grid). */
mg_status mg_server_submit(mg_server *srv, const mg_grid_desc *g, const mg_kernel_desc *k,
                           int64_t nrec, const void *uvw, mg_dtype uvw_dtype, const void *vis,
                           void *grid, hipEvent_t inputs_ready, uint64_t *job_id);

/* Job state; for a finished job *latency_s is the time from submission to
 * the scheduler observing completion (may be NULL).  MG_EINVAL for an
 * unknown or already released job id. */
mg_status mg_server_poll(mg_server *srv, uint64_t job_id, mg_job_state *state,
                         double *latency_s);

/* Blocks until the job finishes, then releases the job's record (its id
 * becomes unknown); returns the job's own status: MG_OK, or the status of a
 * failed launch, or MG_EDEVICE if the device reported an error for the job's
 * work. */
mg_status mg_server_wait(mg_server *srv, uint64_t job_id, double *latency_s);

mg_status mg_server_get_stats(mg_server *srv, mg_server_stats *out);

/* Waits for every queued and running job, then releases the server. */
mg_status mg_server_destroy(mg_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* MIGRID_H */
