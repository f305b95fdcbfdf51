/*
 * ibm_oracle.h -- plain FP64 CPU reference of the simplified wall-modeled
 * immersed boundary stage of Liu & Stevens (arXiv 2006.03343), §3.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark call it; the GPU library never does, and the
 * two share no source.  Every routine follows the paper's definitions in
 * their written order, without blocking, fusion or precomputed stencils.
 *
 * Layout: every field is a C-order double array [nz][ny][nx] (x fastest).
 * uv node (i,j,k) sits at (i dx, j dy, (k+1/2) dz); w node (i,j,k) at
 * (i dx, j dy, k dz) (§2.4: vertical staggering).  u, v, tau_xx, tau_yy,
 * tau_zz, tau_xy, phi_uv and dp/dx, dp/dy live on uv nodes; w, tau_xz,
 * tau_yz, phi_w and dp/dz on w nodes.  Stress component order everywhere:
 * 0 xx, 1 yy, 2 zz, 3 xy, 4 xz, 5 yz.
 */
#ifndef IBM_ORACLE_H
#define IBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int nx, ny, nz; double dx, dy, dz; } ora_grid;
typedef struct {
    double band_width;   /* 2 phi_b, a length */
    double phi_c;        /* sample distance from the surface, >= band_width */
    double kappa;        /* von Karman constant */
} ora_params;

enum { ORA_FLUID = 0, ORA_BAND = 1, ORA_SOLID = 2 };
enum { ORA_UV = 0, ORA_W = 1 };

/* §3.3 node classes: w grid fluid phi > phi_b, band |phi| <= phi_b, solid
 * phi < -phi_b; uv grid fluid phi > 2 phi_b, band 0 <= phi <= 2 phi_b,
 * solid phi < 0. */
int ora_uv_class(double phi, double band_width);
int ora_w_class(double phi, double band_width);

/* Mask byte per linear index: bits 0-1 uv class, bits 2-3 w class, bit 4 uv
 * node forced (phi_uv <= 0, eq. u-*-IBM), bit 5 w node forced (phi_w <= 0). */
void ora_classify(const ora_grid* g, const ora_params* p, const double* phi_uv,
                  const double* phi_w, uint8_t* mask);

/* §3.1: n = grad(phi) / |grad(phi)| at node (i,j,k) of the grid phi lives on.
 * Central differences, periodic in x and y, one-sided at k = 0 and nz-1;
 * |grad(phi)| = 0 gives n = e_z. */
void ora_normal(const ora_grid* g, const double* phi, long i, long j, long k, double n[3]);

/* Trilinear interpolation of a field living on grid ``kind`` at the physical
 * point p: periodic in x and y, vertical index coordinate clamped to
 * [0, nz-1]. */
double ora_interp(const ora_grid* g, const double* f, int kind, const double p[3]);
/* Adjoint of ora_interp: adds value * weight into each of the 8 corners. */
void ora_interp_scatter(const ora_grid* g, double* f, int kind, const double p[3], double value);

/* §3.3 wall model at one band node (i,j,k) of grid ``kind``: local frame
 * e1 = U_r/|U_r|, e3 = n, e2 = e3 x e1; tau' with tau'_13 = tau'_31 = tau_w
 * from eq. bc-bottom-immersed; rotation tau_ij = a_im a_jn tau'_mn.
 * ln_ratio = ln(phi_c / z0).  Writes the full 3x3 tensor (row-major) and, if
 * non-NULL, tau_w and |U_r|. */
void ora_local_stress(const ora_grid* g, const ora_params* p, const double* phi, int kind,
                      long i, long j, long k, const double* u, const double* v, const double* w,
                      double ln_ratio, double tau[9], double* tau_w, double* ur_mag);

/* Whole-domain wall stress.  tau[6] holds the SGS stress on entry and the
 * wall-modeled stress on return: band nodes get the wall model (uv band:
 * xx, yy, zz, xy; w band: xz, yz), solid nodes get zeros on their grid's
 * components, fluid nodes are untouched.  log_z0 may be NULL (then the
 * scalar z0 is used).  stats (may be NULL): [0] sum tau_w over uv band
 * nodes, [1] sum tau_w over w band nodes, [2] max |U_r| over band nodes,
 * [3] number of band nodes. */
void ora_wall_stress(const ora_grid* g, const ora_params* p, const double* phi_uv,
                     const double* phi_w, const double* u, const double* v, const double* w,
                     double z0, const double* log_z0, double* const tau[6], double stats[4]);

/* Stress divergence at every node (eq. dudx with second-order central
 * differences, eqs. dudz/dwdz in z; tau outside 0 <= k < nz reads as 0):
 * div[0], div[1] on uv nodes, div[2] on w nodes. */
void ora_divergence(const ora_grid* g, const double* const tau[6], double* const div[3]);
/* Transpose of ora_divergence, accumulated: gtau[c] += (D^T gdiv)[c]. */
void ora_divergence_transpose(const ora_grid* g, const double* const gdiv[3],
                              double* const gtau[6]);

/* Eq. u-*-IBM: at nodes with phi <= 0 on each component's own grid,
 * ustar = (3 dt / 2) dp; elsewhere unchanged.  gradp may be NULL (zero). */
void ora_forcing(const ora_grid* g, const double* phi_uv, const double* phi_w,
                 double* const ustar[3], const double* const gradp[3], double dt);

/* D_c = dx dy dz * sum over nodes of component c's grid with phi > 0 of
 * div_c, summed in linear-index order. */
void ora_drag(const ora_grid* g, const double* phi_uv, const double* phi_w,
              const double* const div[3], double D[3]);

/* Six class counts: uv fluid, uv band, uv solid, w fluid, w band, w solid. */
void ora_counts(const ora_grid* g, const ora_params* p, const double* phi_uv,
                const double* phi_w, int64_t counts[6]);

/* Reverse mode of (tau_out, div, ustar_ib, drag) with respect to u, v, w
 * and the per-node log z0 field, for one velocity state that is both
 * sampled by the wall model and forced (ustar = u).  g_tau entries may be
 * NULL (zero).  gu, gv, gw are overwritten; glog_z0 (NULL unless log_z0 is
 * given) is overwritten. */
void ora_stage_vjp(const ora_grid* g, const ora_params* p, const double* phi_uv,
                   const double* phi_w, const double* u, const double* v, const double* w,
                   double z0, const double* log_z0, const double* const g_tau[6],
                   const double* const g_div[3], const double* const g_ustar[3],
                   const double g_drag[3], double* gu, double* gv, double* gw, double* glog_z0);

/* §2.2 Smagorinsky sub-grid stress with Mason's wall damping, the wall
 * distance being phi (the node's own grid):
 *   S = (grad u + grad u^T) / 2 (eq. t-ij-1963) with the §2.4 differences:
 *       central in x and y (periodic), eq. dwdz for dw/dz on the uv node,
 *       eq. dudz for du/dz and dv/dz on the w node; velocity taken as 0
 *       outside 0 <= k < nz;
 *   S11, S22, S33, S12 live on uv nodes, S13, S23 on w nodes; |S| =
 *       sqrt(2 S:S) (eq. nu-t) on each node set, with the components of the
 *       other set averaged from its two nodes above and below;
 *   lambda_0 = cs (dx dy dz)^(1/3) (eq. smag), 1/lambda^2 = 1/lambda_0^2 +
 *       1/[kappa (phi + z0)]^2 (eq. smag-1, n = 2), lambda = 0 where
 *       phi + z0 <= 0; z0 is the scalar or exp(log_z0[q]);
 *   nu_t = lambda^2 |S|, tau = -2 nu_t S (eqs. nu-t, t-ij-1963).
 * Writes all six stress components. */
void ora_smagorinsky(const ora_grid* g, double cs, double kappa, const double* phi_uv,
                     const double* phi_w, const double* u, const double* v, const double* w,
                     double z0, const double* log_z0, double* const tau[6]);

/* §1: Chester et al.'s original method, the comparison the paper improves on
 * (its three steps are named in §1 and at the end of §3.3; the stencils are
 * readings, see the design notes).  Both node sets are classified alike:
 * fluid phi > b, fluid band 0 <= phi <= b, solid band -b <= phi < 0,
 * interior phi < -b (b = band_width). */
enum { ORA_CH_FLUID = 0, ORA_CH_BAND = 1, ORA_CH_SOLID_BAND = 2, ORA_CH_INTERIOR = 3 };
int ora_chester_class(double phi, double band_width);
/* counts[class] for uv nodes, counts[4 + class] for w nodes. */
void ora_chester_counts(const ora_grid* g, const ora_params* p, const double* phi_uv,
                        const double* phi_w, int64_t counts[8]);
/* Step 1: the wall model of ora_wall_stress on the fluid band of each node
 * set (uv: xx, yy, zz, xy; w: xz, yz); every node with phi < 0 gets 0 on its
 * set's components; fluid nodes untouched.  stats as in ora_wall_stress,
 * over the fluid-band nodes. */
void ora_chester_wall_stress(const ora_grid* g, const ora_params* p, const double* phi_uv,
                             const double* phi_w, const double* u, const double* v,
                             const double* w, double z0, const double* log_z0,
                             double* const tau[6], double stats[4]);
/* Step 2: linear extrapolation into the solid band.  A solid-band node x
 * with normal n (ora_normal on its set) samples each of its set's
 * components (ora_interp on its set) at the points at distances phi_c and
 * 2 phi_c from the surface along n, x + (phi_c - phi) n and
 * x + (2 phi_c - phi) n, and takes tau1 + (phi - phi_c)(tau2 - tau1)/phi_c.
 * Every value is computed from the field on entry, then written. */
void ora_chester_extrapolate(const ora_grid* g, const ora_params* p, const double* phi_uv,
                             const double* phi_w, double* const tau[6]);
/* Step 3: ``iterations`` red-black SOR sweeps with relaxation ``omega`` of
 * the Laplace equation (7-point, spacings dx, dy, dz; periodic in x and y,
 * values outside 0 <= k < nz read as 0) for each component over the interior
 * nodes of its node set, every other node held fixed.  Red = even i + j + k,
 * first; each colour is updated from the values before its half-sweep. */
void ora_chester_sor(const ora_grid* g, const ora_params* p, const double* phi_uv,
                     const double* phi_w, double omega, int iterations, double* const tau[6]);

int ora_num_threads(void);
void ora_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
