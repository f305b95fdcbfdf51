/*
 * ibm.h -- C ABI of the MI355X (gfx950) wall-modeled immersed boundary stage.
 *
 * The stage is the per-time-step part of the simplified wall-modeled IBM of
 * Liu & Stevens (arXiv 2006.03343, §3): classify the nodes of the staggered
 * grid by the signed distance phi, model the wall stress in a band of nodes
 * next to the immersed surface (log law in a local frame), zero the stress
 * inside the body, take the divergence of the stress and force the
 * intermediate velocity inside the body.
 *
 * Conventions used by every entry point
 *  - Grid: uniform spacings dx, dy, dz (§2.4, eq. dxdydz); x and y periodic.
 *  - Fields: contiguous device arrays laid out [nz][ny][nx], x fastest, all of
 *    the context's storage dtype (float or double), owned by the caller and
 *    resident on the context's device.  Pointers are plain device addresses.
 *  - Staggering (§2.4): a "uv" node (i,j,k) sits at (i dx, j dy, (k+1/2) dz),
 *    a "w" node at (i dx, j dy, k dz).  u, v, tau_xx, tau_yy, tau_zz, tau_xy,
 *    phi_uv, dp/dx, dp/dy live on uv nodes; w, tau_xz, tau_yz, phi_w, dp/dz on
 *    w nodes.  Stress component order everywhere: 0 xx, 1 yy, 2 zz, 3 xy,
 *    4 xz, 5 yz.
 *  - Streams: ``stream`` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Per-step calls only enqueue work; they never synchronise.
 *  - Errors: every function returns 0 (IBM_OK) or a negative IBM_E_* code and
 *    then leaves a message in ibm_last_error() (thread-local).  Argument
 *    checks run before anything is enqueued; nothing is thrown across the ABI.
 *  - Ownership: the library owns the context and everything it allocates
 *    (masks, band records, run lists, reduction scratch, adjoint maps); no
 *    call keeps a caller pointer after it returns.
 */
#ifndef IBM_H
#define IBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    IBM_OK = 0,
    IBM_E_ARG = -1,          /* bad pointer, size, dtype or alignment */
    IBM_E_STATE = -2,        /* call order: a step before levelset_prepare */
    IBM_E_HIP = -3,          /* a HIP runtime call failed (message has the HIP error) */
    IBM_E_NOMEM = -4,        /* device allocation failed */
    IBM_E_RANGE = -5,        /* parameter out of range, or non-finite phi */
    IBM_E_UNSUPPORTED = -6   /* e.g. mixed precision with double storage */
};

enum { IBM_F32 = 0, IBM_F64 = 1 };                 /* storage dtype of every field */
enum { IBM_PREC_PLAIN = 0, IBM_PREC_MIXED = 1 };   /* mixed: only with IBM_F32 */
enum { IBM_GRID_UV = 0, IBM_GRID_W = 1 };

typedef struct ibm_ctx ibm_ctx;

typedef struct { int nx, ny, nz; double dx, dy, dz; } ibm_grid;

typedef struct {
    double band_width;  /* 2 phi_b, a length; §3.3 gives [dz, 1.5 dz) */
    double phi_c;       /* sample distance from the surface, >= band_width (§3.3); <= 0 -> band_width */
    double kappa;       /* von Karman constant (§2.2: 0.4) */
} ibm_params;

/* Create a context for one grid on the current HIP device.
 * dtype: IBM_F32 or IBM_F64.  precision: IBM_PREC_PLAIN, or IBM_PREC_MIXED
 * (float storage; double only for small-gradient normal normalisation, the
 * near-wall log law within one dz of the surface and the drag sums).
 * Errors: IBM_E_ARG (nx, ny, nz < 1, spacing <= 0 or not finite, or
 * nx*ny*nz > 2^31 - 1), IBM_E_UNSUPPORTED (mixed with double). */
int ibm_create(ibm_ctx** out, const ibm_grid* g, int dtype, int precision);
int ibm_destroy(ibm_ctx* c);

/* §3.1 and §3.3, computed once per geometry (the paper identifies the band
 * points at initialisation, §5): node classes of both grids, forcing flags
 * (phi <= 0), normals n = grad phi / |grad phi| at band nodes, and for every
 * band node the trilinear stencil of its sample point x + (phi_c - phi) n.
 * phi_uv, phi_w: device fields (context dtype) of the signed distance at the
 * uv and w nodes (+ fluid, - solid).  Synchronises ``stream``: it reads back
 * counts.  Errors: IBM_E_RANGE for band_width <= 0, phi_c < band_width,
 * kappa <= 0 or any non-finite phi. May be called again for a new geometry. */
int ibm_levelset_prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w,
                         const ibm_params* p, void* stream);

/* Host copies of what prepare found.  counts: uv fluid, uv band, uv solid,
 * w fluid, w band, w solid.  band_size: number of band records of a grid.
 * band_export: ascending linear indices (and, if normals != NULL, 3 doubles
 * per record: the stored normal).  mask_export: one byte per linear index,
 * bits 0-1 uv class (0 fluid, 1 band, 2 solid), bits 2-3 w class, bit 4 uv
 * node forced, bit 5 w node forced. Errors: IBM_E_STATE before prepare. */
int ibm_counts(const ibm_ctx* c, int64_t out[6]);
int ibm_band_size(const ibm_ctx* c, int grid, int64_t* n);
int ibm_band_export(const ibm_ctx* c, int grid, int32_t* idx_host, double* normals_host);
int ibm_mask_export(const ibm_ctx* c, uint8_t* mask_host);

/* §3.3 wall model, eq. bc-bottom-immersed, in place on tau[6].
 * On entry tau holds the SGS stress; on return band nodes hold the modeled
 * wall stress (uv band: xx, yy, zz, xy; w band: xz, yz), solid nodes hold 0
 * on their grid's components and fluid nodes are untouched.
 * u, v (uv nodes) and w (w nodes) are sampled at the band nodes' sample
 * points.  Roughness: the scalar z0 (0 < z0 < phi_c) when log_z0 is NULL,
 * else the per-node field log_z0 (context dtype) read at the band node.
 * stats_dev: NULL or 4 device doubles receiving [sum tau_w over uv band
 * nodes, sum tau_w over w band nodes, max |U_r| over band nodes, number of
 * band nodes].  Asynchronous on ``stream``.  Errors: IBM_E_STATE, IBM_E_ARG,
 * IBM_E_RANGE (bad z0). */
int ibm_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                    const void* log_z0, void* const tau[6], double* stats_dev, void* stream);

/* Stress divergence (§2.4 differences: second-order central in x and y,
 * periodic; staggered second-order in z, stress outside 0 <= k < nz taken as
 * 0) and direct forcing (§3.2, eq. u-*-IBM), one dense pass.
 * div[0], div[1] (uv nodes) and div[2] (w nodes) receive +div(tau); they may
 * not alias tau.  ustar[3] is updated in place: at nodes with phi <= 0 on the
 * component's own grid it becomes (3 dt / 2) gradp (gradp == NULL or an
 * entry NULL: 0); elsewhere it is untouched.  drag_dev: NULL or 3 device
 * doubles receiving D_c = dx dy dz * sum of div_c over the nodes of the
 * component's grid with phi > 0.  Asynchronous on ``stream``.
 * Errors: IBM_E_STATE, IBM_E_ARG. */
int ibm_apply(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
              const void* const gradp[3], double dt, void* const div[3], double* drag_dev,
              void* stream);

/* One stage pass in one call: ibm_wall_stress (§3.3) followed by ibm_apply
 * (§2.4 divergence, §3.2 eq. u-*-IBM forcing), with the band statistics and
 * the drag summed by one launch instead of one each.  Arguments, layouts and
 * results as for those two calls (bit for bit: the same kernels and slot
 * order); stats_dev (4 doubles) and drag_dev (3 doubles) are each nullable.
 * tau entries must be distinct and may not alias u, v, w or log_z0; div and
 * ustar as for ibm_apply.  ustar may be u, v, w themselves (the forcing runs
 * after the wall stress has read them).  Asynchronous on ``stream`` (three
 * launches).  Errors: those of ibm_wall_stress and ibm_apply. */
int ibm_stage(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
              const void* log_z0, void* const tau[6], void* const ustar[3],
              const void* const gradp[3], double dt, void* const div[3], double* stats_dev,
              double* drag_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ibm_apply
 * with its drag reduction slots (3 doubles per tile of the dense pass) in a
 * static device array of the library, 1 MiB on each GPU (held until the
 * process ends), instead of the context's.  Allocates nothing and calls no
 * allocating routine.  Same arguments, checks and results as ibm_apply (bit
 * for bit: the same kernels and slot order).  When drag_dev is given the
 * context's tile shape may have at most 43690 tiles (ibm_get_tile), else
 * IBM_E_RANGE before anything is enqueued.  Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents (each slot a call reads
 * is written by that call first): calls that overlap on one GPU -- on
 * different streams or from several host threads -- race and their drag is
 * undefined; order them on one stream.  Asynchronous on ``stream``.  Errors:
 * those of ibm_apply, IBM_E_RANGE. */
int ibm_apply_noalloc(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                      const void* const gradp[3], double dt, void* const div[3],
                      double* drag_dev, void* stream);

/* ibm_apply with the horizontal derivatives of the divergence taken
 * pseudo-spectrally, as the paper's solver does (§2.4, eq. dudx): d/dx A =
 * sum of i k A_hat exp(i k x) over the wavenumbers of the periodic x and y
 * directions, the Nyquist mode without derivative; vertical differences,
 * zero padding, forcing and drag exactly as in ibm_apply.  nx and ny must be
 * powers of two that fit one block's LDS (float: nx, ny <= 2048; double:
 * nx, ny <= 1024), else IBM_E_UNSUPPORTED.  The first call
 * on a context builds twiddle tables (synchronous).  Asynchronous on
 * ``stream`` otherwise.  Errors: those of ibm_apply, IBM_E_UNSUPPORTED. */
int ibm_apply_spectral(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                       const void* const gradp[3], double dt, void* const div[3],
                       double* drag_dev, void* stream);

/* The time advance around the stage (§2.4).  ibm_ab2_predict: eq. u-inter,
 * ustar = u + dt (3/2 rhs_now - 1/2 rhs_prev) per component (ustar may alias
 * u).  ibm_pressure_project: eqs. p-Poisson, p-Poisson-Fourier, u-t+1 and
 * p-bc.  By eq. dxdydz (dz = Lz / (nz - 1)) the w node 0 is the floor and the
 * w node nz-1 the lid; the uv layers 0 .. nz-2 are the cells between them and
 * the uv layer nz-1 lies above the lid.  Solves D G p = 2/(3 dt) D ustar on
 * the cells and returns u_out = ustar - (3 dt/2) G p and the pressure p_out
 * (on uv nodes).  D: pseudo-spectral d/dx, d/dy (Nyquist modes without
 * derivative) plus (w[k+1] - w[k]) / dz with the wall w taken as 0; G:
 * pseudo-spectral d/dx, d/dy of p on uv nodes and (p[k] - p[k-1]) / dz on the
 * interior w nodes.  On the two wall w nodes the correction is eq. p-bc's
 * wall-normal gradient 2 w* / (3 dt), so w_out = 0 there (eqs. bc-bottom-u3,
 * bc-top) whatever ustar holds; it does not enter the cells' equations.
 * Each horizontal mode is a tridiagonal system over the nz - 1 cells (Thomas,
 * its recurrences in double for either storage type; the vertical
 * differences of p that correct w are formed there in double and
 * transformed back, not taken from the stored p, whose small-wavenumber part
 * is large and nearly constant in z); a mode without horizontal wavenumber
 * (the mean and the Nyquist modes) is singular and takes p = 0 at k = 0 in
 * place of its first row, so u_out is discretely divergence-free in every
 * cell.  The layer above the lid gets p_out = 0 and keeps ustar's u, v.
 * u_out may alias ustar;
 * p_out may alias neither.  nx, ny: powers of two as for
 * ibm_apply_spectral, else IBM_E_UNSUPPORTED.  The first call allocates a
 * workspace of 3 half-spectrum complex volumes of the storage type
 * (nz x ny x (nx/2 + 1) modes, rows padded to an even count) and builds
 * twiddle tables (synchronous).  Needs a context, not a prepare.  Asynchronous on
 * ``stream`` otherwise.  Errors: IBM_E_ARG, IBM_E_RANGE (dt <= 0),
 * IBM_E_UNSUPPORTED, IBM_E_HIP. */
int ibm_ab2_predict(ibm_ctx* c, const void* const u[3], const void* const rhs_now[3],
                    const void* const rhs_prev[3], double dt, void* const ustar[3],
                    void* stream);
int ibm_pressure_project(ibm_ctx* c, const void* const ustar[3], double dt, void* const u_out[3],
                         void* p_out, void* stream);

/* Smagorinsky sub-grid stress with Mason's wall damping (§2.2, eqs.
 * t-ij-1963, nu-t, smag, smag-1): the stress field that ibm_wall_stress then
 * overwrites at band and solid nodes.  The wall distance in the damping is
 * phi of each node's own grid (phi_uv for the four uv components, phi_w for
 * xz, yz).  Strain S = (grad u + grad u^T) / 2 with central differences in x
 * and y (periodic) and the staggered vertical differences of §2.4 (velocity
 * outside 0 <= k < nz taken as 0); |S| = sqrt(2 S:S) with the components of
 * the other node set averaged from its two neighbouring planes; 1/lambda^2 =
 * 1/(cs (dx dy dz)^(1/3))^2 + 1/(kappa (phi + z0))^2, lambda = 0 where
 * phi + z0 <= 0; tau = -2 lambda^2 |S| S, all six components written.  In
 * float the reciprocal in lambda^2 and the square root are the hardware's
 * (1 ulp), in double correctly rounded.
 * z0: scalar (> 0), used when log_z0 == NULL; log_z0: per-node ln z0 field
 * or NULL.  Needs a context, not a prepare.  tau may alias no input.
 * Asynchronous on ``stream``.  Errors: IBM_E_ARG (NULL or aliased fields),
 * IBM_E_RANGE (z0, cs or kappa not finite and > 0). */
int ibm_sgs_stress(ibm_ctx* c, const void* phi_uv, const void* phi_w, const void* u,
                   const void* v, const void* w, double z0, const void* log_z0, double cs,
                   double kappa, void* const tau[6], void* stream);

/* ibm_sgs_stress and the dense pass of ibm_apply in one pass (§2.2 and §2.4,
 * eq. u-*-IBM): the Smagorinsky stress is formed on the fly and never stored.
 * The stress differentiated is, per node and node set, the band value in tau
 * where the node is a band node of its grid (ibm_wall_stress must have filled
 * tau there; tau is read nowhere else), 0 where it is solid, and the
 * Smagorinsky stress of u, v, w elsewhere -- what ibm_sgs_stress followed by
 * ibm_wall_stress leaves in tau, so div, the forcing of ustar and drag_dev are
 * those of ibm_apply on that field.  Arguments as for ibm_sgs_stress and
 * ibm_apply; needs a prepared context.  ustar, div and drag_dev are written
 * while u, v, w, phi_uv, phi_w, log_z0 and tau are read by the same launch, so
 * ustar and div may alias none of them.  Asynchronous on ``stream``.  Errors:
 * IBM_E_STATE, IBM_E_ARG (also: an x-y plane of more than (2^32 - 1) / 5
 * bytes, beyond the pass's 32-bit offsets within a block's planes),
 * IBM_E_RANGE. */
int ibm_apply_sgs(ibm_ctx* c, const void* phi_uv, const void* phi_w, const void* u,
                  const void* v, const void* w, double z0, const void* log_z0, double cs,
                  double kappa, const void* const tau[6], void* const ustar[3],
                  const void* const gradp[3], double dt, void* const div[3], double* drag_dev,
                  void* stream);

/* Chester et al.'s original wall-modeled immersed boundary method, the
 * comparison the paper improves on (§1: a near-wall model for the stresses in
 * a fluid band, linear extrapolation of the stresses into a solid band around
 * the body, SOR iterations smoothing the stress inside the body; §3.3, closing
 * paragraphs: it classifies the w and uv grid points alike).  The paper gives
 * no stencil or parameter for steps 2 and 3; these calls implement one stated
 * reading.  Both node sets take the classes fluid phi > b, fluid band
 * 0 <= phi <= b, solid band -b <= phi < 0, interior phi < -b (b = band_width
 * of ibm_levelset_prepare).
 *
 * ibm_chester_prepare: the classes, band records, solid-band records and the
 * interior node lists for this geometry.  phi_uv and phi_w must be the fields
 * given to ibm_levelset_prepare (whose forcing flags ibm_apply keeps using);
 * a later ibm_levelset_prepare discards this set-up.  nx and ny must each be 1
 * or even (red-black colouring across the periodic seams), else
 * IBM_E_UNSUPPORTED.  Synchronises ``stream``.  Errors: IBM_E_STATE (not
 * prepared), IBM_E_ARG, IBM_E_UNSUPPORTED, IBM_E_HIP, IBM_E_NOMEM.
 *
 * ibm_chester_counts: out[0..3] uv nodes per class (fluid, fluid band, solid
 * band, interior), out[4..7] w nodes.  Errors: IBM_E_STATE.
 *
 * ibm_chester_wall_stress: tau[6] holds the SGS stress on entry and leaves:
 *   1. at fluid-band nodes the wall model of ibm_wall_stress (§3.3: sample at
 *      phi_c along the normal, eq. bc-bottom-immersed, the rotated tensor;
 *      uv nodes xx, yy, zz, xy, w nodes xz, yz); every node with phi < 0 set
 *      to 0 on its node set's components; fluid nodes untouched;
 *   2. at solid-band nodes, per component of the node set, the straight line
 *      in the distance from the surface through the trilinear samples of the
 *      field of step 1 at x + (phi_c - phi) n and x + (2 phi_c - phi) n,
 *      evaluated at the node's phi;
 *   3. ``iterations`` red-black SOR sweeps (relaxation ``omega`` in (0, 2);
 *      red = even i + j + k first) of the 7-point Laplace equation with
 *      spacings dx, dy, dz (periodic in x and y, values outside 0 <= k < nz
 *      taken as 0) over the interior nodes of each node set, every other node
 *      held fixed.
 * Then ibm_apply gives the divergence, forcing and drag as for the simplified
 * stage.  z0, log_z0 and stats_dev (4 device doubles, over the fluid-band
 * nodes) as for ibm_wall_stress.  tau entries must be distinct and may not
 * alias u, v, w or log_z0.  Asynchronous on ``stream`` (2 + 2 iterations
 * launches).  Errors: IBM_E_STATE, IBM_E_ARG, IBM_E_RANGE (z0, omega). */
int ibm_chester_prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w, void* stream);
int ibm_chester_counts(const ibm_ctx* c, int64_t out[8]);
int ibm_chester_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                            const void* log_z0, void* const tau[6], double omega, int iterations,
                            double* stats_dev, void* stream);

/* Reverse mode of one stage pass with respect to u, v, w and log z0, for a
 * single velocity state that is both sampled by the wall model and forced
 * (ustar == u).  Cotangents: g_tau[6] (array or entries may be NULL = 0) of
 * the wall-modeled stress, g_div[3] of the divergence, g_ustar[3] of the
 * forced velocity, g_drag[3] (host doubles) of the drag.  Outputs gu, gv,
 * gw (overwritten) and glog_z0 (overwritten; NULL allowed, required NULL
 * when log_z0 is NULL).  The first call after a prepare builds the transposed
 * stencil map (synchronous); later calls are asynchronous on ``stream``.
 * Errors: IBM_E_STATE before prepare; IBM_E_ARG for a missing or misaligned
 * field, glog_z0 without log_z0, or 2^28 or more band records (uv and w
 * together), beyond the map's 32-bit entry offsets; IBM_E_RANGE for z0 outside
 * (0, phi_c). */
int ibm_stage_vjp(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                  const void* log_z0, const void* const g_tau[6], const void* const g_div[3],
                  const void* const g_ustar[3], const double g_drag[3], void* gu, void* gv,
                  void* gw, void* glog_z0, void* stream);

/* Tile shape of the dense pass (ibm_apply): a wave owns vx*64 nodes along x,
 * ty rows and kz planes; wpb waves per block.  vx in {1,2,4} (double: {1,2})
 * and must divide nx; ty in {1,2,4,8}; kz >= 1; wpb in 1..4.  A batch accepts
 * ty <= 2.  The shape only
 * changes speed and the summation order of the drag, never the divergence or
 * forcing values.  ibm_sgs_stress then runs on it too (one row per wave), in
 * place of a shape the autotuner chose for it.  ibm_get_tile reports the
 * dense pass's shape.  The default, from the grid size: the longest z march
 * (at most 64 planes) that still gives 1024 wave-tiles, one row per wave (two
 * in double while 1024 tiles remain), four waves per block below 2048 tiles.
 * Errors:
 * IBM_E_ARG for an unsupported shape. */
int ibm_set_tile(ibm_ctx* c, int vx, int ty, int kz, int wpb);
int ibm_get_tile(const ibm_ctx* c, int out[4]);

/* ---------------------------------------------------------------- tuning
 * Time candidate tile shapes of the dense pass on this context's prepared
 * grid (on scratch fields allocated for the call; caller data is not read)
 * and keep the fastest.  cache_path (nullable): a JSON file, one entry per
 * grid shape, dtype, precision and GPU architecture; a cached shape is reused
 * without timing unless IBM_TUNE_FORCE.  IBM_TUNE_BATCH restricts the search
 * to shapes the batched kernels accept (ty <= 2).  Without it the Smagorinsky
 * kernel of ibm_sgs_stress gets a tile of its own the same way (one row per
 * wave; cached under the key ending in "sgs"); otherwise, and after
 * ibm_set_tile, it runs on the dense pass's tile.  Synchronises ``stream``. */
enum { IBM_TUNE_FORCE = 1, IBM_TUNE_BATCH = 2 };
int ibm_autotune(ibm_ctx* c, const char* cache_path, int flags, void* stream);

/* ------------------------------------------------------------- ensembles
 * A batch advances many grids of different sizes together: one step is three
 * kernels (wall stress, dense pass, reductions) whose blocks take items of
 * work lists that span every case, captured once in a hipGraph and replayed
 * by ibm_batch_launch.  Each case computes exactly what ibm_wall_stress followed
 * by ibm_apply computes on a context with the same tile shape (bitwise). */
typedef struct ibm_batch ibm_batch;

typedef struct {
    const void *u, *v, *w;   /* sampled velocity (uv, uv, w nodes) */
    const void* log_z0;      /* per-node log z0, or NULL for the case's scalar z0 */
    void* tau[6];            /* in: SGS stress; out: wall-modeled stress */
    void* ustar[3];          /* forced in place */
    const void* gradp[3];    /* entries may be NULL (0) */
    void* div[3];            /* out: +div(tau) */
    double dt;
    double* drag_dev;        /* NULL or 3 device doubles: the case's drag (as ibm_apply) */
    double* stats_dev;       /* NULL or 4 device doubles: band statistics (as ibm_wall_stress) */
} ibm_case_io;

/* ncases contexts on the current device; grids[i] is case i's grid. */
int ibm_batch_create(ibm_batch** out, int ncases, const ibm_grid* grids, int dtype, int precision);
int ibm_batch_destroy(ibm_batch* b);
/* Prepare every case (as ibm_levelset_prepare; synchronous).  z0[i]: case i's
 * scalar roughness (0 < z0 < phi_c). Unbinds every case. */
int ibm_batch_prepare(ibm_batch* b, const void* const* phi_uv, const void* const* phi_w,
                      const ibm_params* p, const double* z0, void* stream);
/* Attach case i's caller-owned device fields.  The batch keeps the pointers:
 * they must stay valid, at the same addresses, until the batch is destroyed or
 * the case is bound again.  tau and div need 16-byte alignment when the case's
 * tile has vx > 1.  Invalidates a captured graph. */
int ibm_batch_bind(ibm_batch* b, int case_id, const ibm_case_io* io);
/* Autotune each distinct grid shape once (IBM_TUNE_BATCH) and give the shape
 * to every case of that size.  Invalidates a captured graph. */
int ibm_batch_tune(ibm_batch* b, const char* cache_path, void* stream);
/* One step without a graph (three kernel launches on ``stream``). */
int ibm_batch_run(ibm_batch* b, void* stream);
/* Record one step into a hipGraph (stream capture on ``stream``, which must be
 * a created stream, not the null stream), after every case is bound.
 * ibm_batch_launch replays it on any stream: one hipGraphLaunch per step.
 * Errors: IBM_E_STATE when a case is unbound or the graph is stale, IBM_E_ARG
 * for the null stream. */
int ibm_batch_capture(ibm_batch* b, void* stream);
int ibm_batch_launch(ibm_batch* b, void* stream);
/* The context of one case (owned by the batch): counts, masks, band lists. */
int ibm_batch_case(const ibm_batch* b, int case_id, ibm_ctx** out);

/* Message of the last failing call on this thread ("" if none). */
const char* ibm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
