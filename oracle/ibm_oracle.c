/*
 * ibm_oracle.c -- plain FP64 CPU reference of the simplified wall-modeled
 * IBM stage (Liu & Stevens, arXiv 2006.03343, §3).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU baseline; never by the GPU library.  It is deliberately
 * literal: classes are evaluated from phi at every node, the normal and the
 * sample point are recomputed on the fly, the stress is built in an explicit
 * local frame and rotated with a full triple loop, and the divergence is
 * evaluated node by node.  OpenMP splits only the outer k loop.
 */
#include "ibm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static long pmod(long a, long n) {
    long r = a % n;
    return r < 0 ? r + n : r;
}

static long lin(const ora_grid* g, long i, long j, long k) {
    return (k * g->ny + j) * (long)g->nx + i;
}

/* value of a field at (i, j, k) with periodic x/y and zero outside 0 <= k < nz */
static double at_padded(const ora_grid* g, const double* f, long i, long j, long k) {
    if (k < 0 || k >= g->nz) return 0.0;
    return f[lin(g, pmod(i, g->nx), pmod(j, g->ny), k)];
}

int ora_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel loops (timing with one thread). */
void ora_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------- §3.3 classes */
int ora_uv_class(double phi, double band_width) {
    if (phi < 0.0) return ORA_SOLID;
    if (phi <= band_width) return ORA_BAND;
    return ORA_FLUID;
}

int ora_w_class(double phi, double band_width) {
    double phi_b = band_width / 2.0;
    if (phi < -phi_b) return ORA_SOLID;
    if (phi <= phi_b) return ORA_BAND;
    return ORA_FLUID;
}

void ora_classify(const ora_grid* g, const ora_params* p, const double* phi_uv,
                  const double* phi_w, uint8_t* mask) {
    long n = (long)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < n; ++q) {
        int m = ora_uv_class(phi_uv[q], p->band_width) | (ora_w_class(phi_w[q], p->band_width) << 2);
        if (phi_uv[q] <= 0.0) m |= 1 << 4;
        if (phi_w[q] <= 0.0) m |= 1 << 5;
        mask[q] = (uint8_t)m;
    }
}

void ora_counts(const ora_grid* g, const ora_params* p, const double* phi_uv,
                const double* phi_w, int64_t counts[6]) {
    long n = (long)g->nx * g->ny * g->nz;
    for (int c = 0; c < 6; ++c) counts[c] = 0;
    for (long q = 0; q < n; ++q) {
        counts[ora_uv_class(phi_uv[q], p->band_width)] += 1;
        counts[3 + ora_w_class(phi_w[q], p->band_width)] += 1;
    }
}

/* ------------------------------------------------------------ §3.1 normals */
void ora_normal(const ora_grid* g, const double* phi, long i, long j, long k, double n[3]) {
    double gx = (phi[lin(g, pmod(i + 1, g->nx), j, k)] - phi[lin(g, pmod(i - 1, g->nx), j, k)]) / (2.0 * g->dx);
    double gy = (phi[lin(g, i, pmod(j + 1, g->ny), k)] - phi[lin(g, i, pmod(j - 1, g->ny), k)]) / (2.0 * g->dy);
    double gz;
    if (g->nz == 1)
        gz = 0.0;
    else if (k == 0)
        gz = (phi[lin(g, i, j, 1)] - phi[lin(g, i, j, 0)]) / g->dz;
    else if (k == g->nz - 1)
        gz = (phi[lin(g, i, j, k)] - phi[lin(g, i, j, k - 1)]) / g->dz;
    else
        gz = (phi[lin(g, i, j, k + 1)] - phi[lin(g, i, j, k - 1)]) / (2.0 * g->dz);
    double mag = sqrt(gx * gx + gy * gy + gz * gz);
    if (mag == 0.0) {
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
        return;
    }
    n[0] = gx / mag; n[1] = gy / mag; n[2] = gz / mag;
}

/* ----------------------------------------------- second-order interpolation */
typedef struct { long i[2], j[2], k[2]; double wx[2], wy[2], wz[2]; } stencil;

static void make_stencil(const ora_grid* g, int kind, const double p[3], stencil* s) {
    double xi = p[0] / g->dx;
    double yi = p[1] / g->dy;
    double zi = p[2] / g->dz - (kind == ORA_UV ? 0.5 : 0.0);
    if (zi < 0.0) zi = 0.0;
    if (zi > g->nz - 1) zi = (double)(g->nz - 1);
    double fx = floor(xi), fy = floor(yi), fz = floor(zi);
    double ax = xi - fx, ay = yi - fy, az = zi - fz;
    long i0 = (long)fx, j0 = (long)fy, k0 = (long)fz;
    s->i[0] = pmod(i0, g->nx); s->i[1] = pmod(i0 + 1, g->nx);
    s->j[0] = pmod(j0, g->ny); s->j[1] = pmod(j0 + 1, g->ny);
    s->k[0] = k0; s->k[1] = (k0 + 1 > g->nz - 1) ? g->nz - 1 : k0 + 1;
    s->wx[0] = 1.0 - ax; s->wx[1] = ax;
    s->wy[0] = 1.0 - ay; s->wy[1] = ay;
    s->wz[0] = 1.0 - az; s->wz[1] = az;
}

double ora_interp(const ora_grid* g, const double* f, int kind, const double p[3]) {
    stencil s;
    make_stencil(g, kind, p, &s);
    double sum = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                sum += s.wx[a] * s.wy[b] * s.wz[c] * f[lin(g, s.i[a], s.j[b], s.k[c])];
    return sum;
}

void ora_interp_scatter(const ora_grid* g, double* f, int kind, const double p[3], double value) {
    stencil s;
    make_stencil(g, kind, p, &s);
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                f[lin(g, s.i[a], s.j[b], s.k[c])] += s.wx[a] * s.wy[b] * s.wz[c] * value;
}

/* --------------------------------------------------- §3.3 wall-stress model */
static void node_position(const ora_grid* g, int kind, long i, long j, long k, double x[3]) {
    x[0] = i * g->dx;
    x[1] = j * g->dy;
    x[2] = (k + (kind == ORA_UV ? 0.5 : 0.0)) * g->dz;
}

/* The velocity sampled for a band node: the point at distance phi_c from the
 * surface on the line through the node parallel to n. */
static void sample_point(const ora_grid* g, const ora_params* p, const double* phi, int kind,
                         long i, long j, long k, double n[3], double pt[3]) {
    double x[3];
    node_position(g, kind, i, j, k, x);
    ora_normal(g, phi, i, j, k, n);
    double shift = p->phi_c - phi[lin(g, i, j, k)];
    for (int d = 0; d < 3; ++d) pt[d] = x[d] + shift * n[d];
}

static void sampled_velocity(const ora_grid* g, const double* u, const double* v,
                             const double* w, const double pt[3], double us[3]) {
    us[0] = ora_interp(g, u, ORA_UV, pt);
    us[1] = ora_interp(g, v, ORA_UV, pt);
    us[2] = ora_interp(g, w, ORA_W, pt);
}

void ora_local_stress(const ora_grid* g, const ora_params* p, const double* phi, int kind,
                      long i, long j, long k, const double* u, const double* v, const double* w,
                      double ln_ratio, double tau[9], double* tau_w_out, double* ur_out) {
    double n[3], pt[3], us[3], ur[3];
    sample_point(g, p, phi, kind, i, j, k, n, pt);
    sampled_velocity(g, u, v, w, pt, us);
    /* tangential part U_r = u - (u.n) n */
    double un = us[0] * n[0] + us[1] * n[1] + us[2] * n[2];
    for (int d = 0; d < 3; ++d) ur[d] = us[d] - un * n[d];
    double U = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
    /* eq. bc-bottom-immersed */
    double r = p->kappa * U / ln_ratio;
    double tau_w = -(r * r);
    for (int a = 0; a < 9; ++a) tau[a] = 0.0;
    if (tau_w_out) *tau_w_out = tau_w;
    if (ur_out) *ur_out = U;
    if (U == 0.0) return;
    /* local basis: e1 along U_r, e3 = n, e2 = e3 x e1 */
    double e1[3] = {ur[0] / U, ur[1] / U, ur[2] / U};
    double e3[3] = {n[0], n[1], n[2]};
    double e2[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2],
                    e3[0] * e1[1] - e3[1] * e1[0]};
    /* a[i][m]: direction cosine between global axis i and local axis m */
    double a[3][3];
    for (int d = 0; d < 3; ++d) {
        a[d][0] = e1[d];
        a[d][1] = e2[d];
        a[d][2] = e3[d];
    }
    double tl[3][3] = {{0.0, 0.0, tau_w}, {0.0, 0.0, 0.0}, {tau_w, 0.0, 0.0}};
    for (int ii = 0; ii < 3; ++ii)
        for (int jj = 0; jj < 3; ++jj) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m)
                for (int nn = 0; nn < 3; ++nn) s += a[ii][m] * a[jj][nn] * tl[m][nn];
            tau[3 * ii + jj] = s;
        }
}

static double ln_ratio_at(const ora_params* p, double z0, const double* log_z0, long q) {
    if (log_z0) return log(p->phi_c) - log_z0[q];
    return log(p->phi_c / z0);
}

void ora_wall_stress(const ora_grid* g, const ora_params* p, const double* phi_uv,
                     const double* phi_w, const double* u, const double* v, const double* w,
                     double z0, const double* log_z0, double* const tau[6], double stats[4]) {
    long nz = g->nz;
    double* part = (double*)calloc((size_t)nz * 4, sizeof(double));
#pragma omp parallel for schedule(dynamic)
    for (long k = 0; k < nz; ++k) {
        double s_uv = 0.0, s_w = 0.0, umax = 0.0, cnt = 0.0;
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long q = lin(g, i, j, k);
                double t[9], tw, U;
                int cu = ora_uv_class(phi_uv[q], p->band_width);
                if (cu == ORA_BAND) {
                    ora_local_stress(g, p, phi_uv, ORA_UV, i, j, k, u, v, w,
                                     ln_ratio_at(p, z0, log_z0, q), t, &tw, &U);
                    tau[0][q] = t[0];      /* xx */
                    tau[1][q] = t[4];      /* yy */
                    tau[2][q] = t[8];      /* zz */
                    tau[3][q] = t[1];      /* xy */
                    s_uv += tw;
                    if (U > umax) umax = U;
                    cnt += 1.0;
                } else if (cu == ORA_SOLID) {
                    tau[0][q] = 0.0; tau[1][q] = 0.0; tau[2][q] = 0.0; tau[3][q] = 0.0;
                }
                int cw = ora_w_class(phi_w[q], p->band_width);
                if (cw == ORA_BAND) {
                    ora_local_stress(g, p, phi_w, ORA_W, i, j, k, u, v, w,
                                     ln_ratio_at(p, z0, log_z0, q), t, &tw, &U);
                    tau[4][q] = t[2];      /* xz */
                    tau[5][q] = t[5];      /* yz */
                    s_w += tw;
                    if (U > umax) umax = U;
                    cnt += 1.0;
                } else if (cw == ORA_SOLID) {
                    tau[4][q] = 0.0; tau[5][q] = 0.0;
                }
            }
        part[4 * k + 0] = s_uv;
        part[4 * k + 1] = s_w;
        part[4 * k + 2] = umax;
        part[4 * k + 3] = cnt;
    }
    if (stats) {
        stats[0] = stats[1] = stats[2] = stats[3] = 0.0;
        for (long k = 0; k < nz; ++k) {
            stats[0] += part[4 * k + 0];
            stats[1] += part[4 * k + 1];
            if (part[4 * k + 2] > stats[2]) stats[2] = part[4 * k + 2];
            stats[3] += part[4 * k + 3];
        }
    }
    free(part);
}

/* --------------------------------------------------- divergence of the stress */
void ora_divergence(const ora_grid* g, const double* const tau[6], double* const div[3]) {
    const double *txx = tau[0], *tyy = tau[1], *tzz = tau[2], *txy = tau[3], *txz = tau[4], *tyz = tau[5];
    double dx = g->dx, dy = g->dy, dz = g->dz;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long q = lin(g, i, j, k);
                /* x momentum on the uv node: d/dx txx + d/dy txy + d/dz txz (txz on w nodes k, k+1) */
                div[0][q] = (at_padded(g, txx, i + 1, j, k) - at_padded(g, txx, i - 1, j, k)) / (2.0 * dx)
                          + (at_padded(g, txy, i, j + 1, k) - at_padded(g, txy, i, j - 1, k)) / (2.0 * dy)
                          + (at_padded(g, txz, i, j, k + 1) - at_padded(g, txz, i, j, k)) / dz;
                /* y momentum on the uv node */
                div[1][q] = (at_padded(g, txy, i + 1, j, k) - at_padded(g, txy, i - 1, j, k)) / (2.0 * dx)
                          + (at_padded(g, tyy, i, j + 1, k) - at_padded(g, tyy, i, j - 1, k)) / (2.0 * dy)
                          + (at_padded(g, tyz, i, j, k + 1) - at_padded(g, tyz, i, j, k)) / dz;
                /* z momentum on the w node: tzz on uv nodes k-1, k */
                div[2][q] = (at_padded(g, txz, i + 1, j, k) - at_padded(g, txz, i - 1, j, k)) / (2.0 * dx)
                          + (at_padded(g, tyz, i, j + 1, k) - at_padded(g, tyz, i, j - 1, k)) / (2.0 * dy)
                          + (at_padded(g, tzz, i, j, k) - at_padded(g, tzz, i, j, k - 1)) / dz;
            }
}

/* Scatter form of D^T: every term c * tau[src] of div[out] sends c * gdiv[out]
 * back to tau[src].  Serial, because sources collide. */
static void add_padded(const ora_grid* g, double* f, long i, long j, long k, double val) {
    if (k < 0 || k >= g->nz) return;
    f[lin(g, pmod(i, g->nx), pmod(j, g->ny), k)] += val;
}

void ora_divergence_transpose(const ora_grid* g, const double* const gdiv[3],
                              double* const gtau[6]) {
    double *txx = gtau[0], *tyy = gtau[1], *tzz = gtau[2], *txy = gtau[3], *txz = gtau[4], *tyz = gtau[5];
    double cx = 1.0 / (2.0 * g->dx), cy = 1.0 / (2.0 * g->dy), cz = 1.0 / g->dz;
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long q = lin(g, i, j, k);
                double gx = gdiv[0][q], gy = gdiv[1][q], gz = gdiv[2][q];
                add_padded(g, txx, i + 1, j, k, cx * gx);
                add_padded(g, txx, i - 1, j, k, -cx * gx);
                add_padded(g, txy, i, j + 1, k, cy * gx);
                add_padded(g, txy, i, j - 1, k, -cy * gx);
                add_padded(g, txz, i, j, k + 1, cz * gx);
                add_padded(g, txz, i, j, k, -cz * gx);

                add_padded(g, txy, i + 1, j, k, cx * gy);
                add_padded(g, txy, i - 1, j, k, -cx * gy);
                add_padded(g, tyy, i, j + 1, k, cy * gy);
                add_padded(g, tyy, i, j - 1, k, -cy * gy);
                add_padded(g, tyz, i, j, k + 1, cz * gy);
                add_padded(g, tyz, i, j, k, -cz * gy);

                add_padded(g, txz, i + 1, j, k, cx * gz);
                add_padded(g, txz, i - 1, j, k, -cx * gz);
                add_padded(g, tyz, i, j + 1, k, cy * gz);
                add_padded(g, tyz, i, j - 1, k, -cy * gz);
                add_padded(g, tzz, i, j, k, cz * gz);
                add_padded(g, tzz, i, j, k - 1, -cz * gz);
            }
}

/* ------------------------------------------------------ §3.2 direct forcing */
void ora_forcing(const ora_grid* g, const double* phi_uv, const double* phi_w,
                 double* const ustar[3], const double* const gradp[3], double dt) {
    long n = (long)g->nx * g->ny * g->nz;
    for (long q = 0; q < n; ++q) {
        for (int c = 0; c < 3; ++c) {
            double phi = (c < 2) ? phi_uv[q] : phi_w[q];
            if (phi <= 0.0) {
                double gp = (gradp && gradp[c]) ? gradp[c][q] : 0.0;
                ustar[c][q] = 3.0 * dt / 2.0 * gp;
            }
        }
    }
}

void ora_drag(const ora_grid* g, const double* phi_uv, const double* phi_w,
              const double* const div[3], double D[3]) {
    long n = (long)g->nx * g->ny * g->nz;
    double dv = g->dx * g->dy * g->dz;
    for (int c = 0; c < 3; ++c) {
        const double* phi = (c < 2) ? phi_uv : phi_w;
        double s = 0.0;
        for (long q = 0; q < n; ++q)
            if (phi[q] > 0.0) s += div[c][q];
        D[c] = dv * s;
    }
}

/* ------------------------------------------------------------- reverse mode */
/* Reverse of ora_local_stress for the components a node of ``kind`` stores:
 * given their cotangents, accumulate into the velocity cotangents (through
 * the interpolation) and return the cotangent of ln_ratio. */
static double local_stress_reverse(const ora_grid* g, const ora_params* p, const double* phi,
                                   int kind, long i, long j, long k, const double* u,
                                   const double* v, const double* w, double ln_ratio,
                                   const double tbar[9], double* gu, double* gv, double* gw) {
    double n[3], pt[3], us[3], ur[3];
    sample_point(g, p, phi, kind, i, j, k, n, pt);
    sampled_velocity(g, u, v, w, pt, us);
    double un = us[0] * n[0] + us[1] * n[1] + us[2] * n[2];
    for (int d = 0; d < 3; ++d) ur[d] = us[d] - un * n[d];
    double U = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
    if (U == 0.0) return 0.0;   /* tau is quadratic in U_r: zero gradient there */
    double t[3] = {ur[0] / U, ur[1] / U, ur[2] / U};
    double kap = p->kappa;
    double tau_w = -(kap * U / ln_ratio) * (kap * U / ln_ratio);
    /* tau_ij = tau_w (t_i n_j + n_i t_j) */
    double tw_bar = 0.0, t_bar[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double tb = tbar[3 * a + b];
            if (tb == 0.0) continue;
            tw_bar += tb * (t[a] * n[b] + n[a] * t[b]);
            t_bar[a] += tau_w * tb * n[b];
            t_bar[b] += tau_w * tb * n[a];
        }
    /* tau_w = -(kappa U / L)^2 */
    double U_bar = tw_bar * (-2.0 * kap * kap * U / (ln_ratio * ln_ratio));
    double L_bar = tw_bar * (2.0 * kap * kap * U * U / (ln_ratio * ln_ratio * ln_ratio));
    /* t = U_r / U and U = |U_r| */
    double tdot = t[0] * t_bar[0] + t[1] * t_bar[1] + t[2] * t_bar[2];
    double ur_bar[3];
    for (int d = 0; d < 3; ++d) ur_bar[d] = (t_bar[d] - t[d] * tdot) / U + U_bar * t[d];
    /* U_r = u_s - (u_s . n) n */
    double nd = ur_bar[0] * n[0] + ur_bar[1] * n[1] + ur_bar[2] * n[2];
    double us_bar[3];
    for (int d = 0; d < 3; ++d) us_bar[d] = ur_bar[d] - nd * n[d];
    ora_interp_scatter(g, gu, ORA_UV, pt, us_bar[0]);
    ora_interp_scatter(g, gv, ORA_UV, pt, us_bar[1]);
    ora_interp_scatter(g, gw, ORA_W, pt, us_bar[2]);
    return L_bar;
}

void ora_stage_vjp(const ora_grid* g, const ora_params* p, const double* phi_uv,
                   const double* phi_w, const double* u, const double* v, const double* w,
                   double z0, const double* log_z0, const double* const g_tau[6],
                   const double* const g_div[3], const double* const g_ustar[3],
                   const double g_drag[3], double* gu, double* gv, double* gw, double* glog_z0) {
    long n = (long)g->nx * g->ny * g->nz;
    double dv = g->dx * g->dy * g->dz;
    /* 1. the drag adds dV [phi > 0] g_drag to the divergence cotangent */
    double* gd[3];
    for (int c = 0; c < 3; ++c) {
        gd[c] = (double*)malloc(sizeof(double) * (size_t)n);
        const double* phi = (c < 2) ? phi_uv : phi_w;
        for (long q = 0; q < n; ++q)
            gd[c][q] = (g_div && g_div[c] ? g_div[c][q] : 0.0) + (phi[q] > 0.0 ? dv * g_drag[c] : 0.0);
    }
    /* 2. stress cotangent = g_tau + D^T gd */
    double* gt[6];
    for (int c = 0; c < 6; ++c) {
        gt[c] = (double*)malloc(sizeof(double) * (size_t)n);
        for (long q = 0; q < n; ++q) gt[c][q] = (g_tau && g_tau[c]) ? g_tau[c][q] : 0.0;
    }
    ora_divergence_transpose(g, (const double* const*)gd, gt);
    memset(gu, 0, sizeof(double) * (size_t)n);
    memset(gv, 0, sizeof(double) * (size_t)n);
    memset(gw, 0, sizeof(double) * (size_t)n);
    if (glog_z0) memset(glog_z0, 0, sizeof(double) * (size_t)n);
    /* 3. band nodes: reverse of the wall model (only band stresses depend on u) */
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long q = lin(g, i, j, k);
                double lr = ln_ratio_at(p, z0, log_z0, q);
                if (ora_uv_class(phi_uv[q], p->band_width) == ORA_BAND) {
                    double tb[9] = {0};
                    tb[0] = gt[0][q]; tb[4] = gt[1][q]; tb[8] = gt[2][q]; tb[1] = gt[3][q];
                    double lb = local_stress_reverse(g, p, phi_uv, ORA_UV, i, j, k, u, v, w, lr, tb, gu, gv, gw);
                    if (glog_z0) glog_z0[q] += -lb;
                }
                if (ora_w_class(phi_w[q], p->band_width) == ORA_BAND) {
                    double tb[9] = {0};
                    tb[2] = gt[4][q]; tb[5] = gt[5][q];
                    double lb = local_stress_reverse(g, p, phi_w, ORA_W, i, j, k, u, v, w, lr, tb, gu, gv, gw);
                    if (glog_z0) glog_z0[q] += -lb;
                }
            }
    /* 4. forcing keeps u at unforced nodes and replaces it elsewhere */
    for (long q = 0; q < n; ++q) {
        if (phi_uv[q] > 0.0) {
            gu[q] += g_ustar && g_ustar[0] ? g_ustar[0][q] : 0.0;
            gv[q] += g_ustar && g_ustar[1] ? g_ustar[1][q] : 0.0;
        }
        if (phi_w[q] > 0.0) gw[q] += g_ustar && g_ustar[2] ? g_ustar[2][q] : 0.0;
    }
    for (int c = 0; c < 3; ++c) free(gd[c]);
    for (int c = 0; c < 6; ++c) free(gt[c]);
}

/* ----------------------------------------------- §2.2 Smagorinsky SGS stress */
static double ddx(const ora_grid* g, const double* f, long i, long j, long k) {
    return (at_padded(g, f, i + 1, j, k) - at_padded(g, f, i - 1, j, k)) / (2.0 * g->dx);
}

static double ddy(const ora_grid* g, const double* f, long i, long j, long k) {
    return (at_padded(g, f, i, j + 1, k) - at_padded(g, f, i, j - 1, k)) / (2.0 * g->dy);
}

/* S11, S22, S33, S12 on the uv node (i,j,k); zero outside 0 <= k < nz */
static void strain_uv(const ora_grid* g, const double* u, const double* v, const double* w,
                      long i, long j, long k, double s[4]) {
    if (k < 0 || k >= g->nz) {
        s[0] = s[1] = s[2] = s[3] = 0.0;
        return;
    }
    s[0] = ddx(g, u, i, j, k);
    s[1] = ddy(g, v, i, j, k);
    /* eq. dwdz: dw/dz of the w nodes k and k+1, on the uv node k between them */
    s[2] = (at_padded(g, w, i, j, k + 1) - at_padded(g, w, i, j, k)) / g->dz;
    s[3] = 0.5 * (ddy(g, u, i, j, k) + ddx(g, v, i, j, k));
}

/* S13, S23 on the w node (i,j,k); zero outside 0 <= k < nz */
static void strain_w(const ora_grid* g, const double* u, const double* v, const double* w,
                     long i, long j, long k, double s[2]) {
    if (k < 0 || k >= g->nz) {
        s[0] = s[1] = 0.0;
        return;
    }
    /* eq. dudz: du/dz of the uv nodes k-1 and k, on the w node k between them */
    const double dudz = (at_padded(g, u, i, j, k) - at_padded(g, u, i, j, k - 1)) / g->dz;
    const double dvdz = (at_padded(g, v, i, j, k) - at_padded(g, v, i, j, k - 1)) / g->dz;
    s[0] = 0.5 * (dudz + ddx(g, w, i, j, k));
    s[1] = 0.5 * (dvdz + ddy(g, w, i, j, k));
}

/* lambda^2 of eq. smag-1 with n = 2 at wall distance d */
static double mixing_length_sq(const ora_grid* g, double cs, double kappa, double d, double z0) {
    const double lambda0 = cs * cbrt(g->dx * g->dy * g->dz);
    if (!(d + z0 > 0.0)) return 0.0;
    const double wall = kappa * (d + z0);
    return 1.0 / (1.0 / (lambda0 * lambda0) + 1.0 / (wall * wall));
}

void ora_smagorinsky(const ora_grid* g, double cs, double kappa, const double* phi_uv,
                     const double* phi_w, const double* u, const double* v, const double* w,
                     double z0, const double* log_z0, double* const tau[6]) {
#pragma omp parallel for schedule(static)
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                const long q = lin(g, i, j, k);
                const double zq = log_z0 ? exp(log_z0[q]) : z0;
                double a[4], below[4], wk[2], wk1[2];
                strain_uv(g, u, v, w, i, j, k, a);
                strain_uv(g, u, v, w, i, j, k - 1, below);
                strain_w(g, u, v, w, i, j, k, wk);
                strain_w(g, u, v, w, i, j, k + 1, wk1);
                /* uv node k: S13, S23 from the w nodes k and k+1 */
                const double s13 = 0.5 * (wk[0] + wk1[0]), s23 = 0.5 * (wk[1] + wk1[1]);
                const double ss_uv = a[0] * a[0] + a[1] * a[1] + a[2] * a[2] +
                                     2.0 * (a[3] * a[3] + s13 * s13 + s23 * s23);
                const double nu_uv = mixing_length_sq(g, cs, kappa, phi_uv[q], zq) * sqrt(2.0 * ss_uv);
                for (int c = 0; c < 4; ++c) tau[c][q] = -2.0 * nu_uv * a[c];
                /* w node k: S11, S22, S33, S12 from the uv nodes k-1 and k */
                double m[4];
                for (int c = 0; c < 4; ++c) m[c] = 0.5 * (below[c] + a[c]);
                const double ss_w = m[0] * m[0] + m[1] * m[1] + m[2] * m[2] +
                                    2.0 * (m[3] * m[3] + wk[0] * wk[0] + wk[1] * wk[1]);
                const double nu_w = mixing_length_sq(g, cs, kappa, phi_w[q], zq) * sqrt(2.0 * ss_w);
                tau[4][q] = -2.0 * nu_w * wk[0];
                tau[5][q] = -2.0 * nu_w * wk[1];
            }
}

/* ------------------------------------------- §1: Chester et al.'s original */
/* The method the paper simplifies, in its three named steps (§1, §3.3's
 * closing paragraphs), with both node sets classified alike. */
int ora_chester_class(double phi, double band_width) {
    if (phi > band_width) return ORA_CH_FLUID;
    if (phi >= 0.0) return ORA_CH_BAND;
    if (phi >= -band_width) return ORA_CH_SOLID_BAND;
    return ORA_CH_INTERIOR;
}

void ora_chester_counts(const ora_grid* g, const ora_params* p, const double* phi_uv,
                        const double* phi_w, int64_t counts[8]) {
    long n = (long)g->nx * g->ny * g->nz;
    for (int c = 0; c < 8; ++c) counts[c] = 0;
    for (long q = 0; q < n; ++q) {
        counts[ora_chester_class(phi_uv[q], p->band_width)] += 1;
        counts[4 + ora_chester_class(phi_w[q], p->band_width)] += 1;
    }
}

/* Step 1: the near-wall model in the fluid band, zero inside the body. */
void ora_chester_wall_stress(const ora_grid* g, const ora_params* p, const double* phi_uv,
                             const double* phi_w, const double* u, const double* v,
                             const double* w, double z0, const double* log_z0,
                             double* const tau[6], double stats[4]) {
    long nz = g->nz;
    double* part = (double*)calloc((size_t)nz * 4, sizeof(double));
#pragma omp parallel for schedule(dynamic)
    for (long k = 0; k < nz; ++k) {
        double s_uv = 0.0, s_w = 0.0, umax = 0.0, cnt = 0.0;
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long q = lin(g, i, j, k);
                double t[9], tw, U;
                int cu = ora_chester_class(phi_uv[q], p->band_width);
                if (cu == ORA_CH_BAND) {
                    ora_local_stress(g, p, phi_uv, ORA_UV, i, j, k, u, v, w,
                                     ln_ratio_at(p, z0, log_z0, q), t, &tw, &U);
                    tau[0][q] = t[0];
                    tau[1][q] = t[4];
                    tau[2][q] = t[8];
                    tau[3][q] = t[1];
                    s_uv += tw;
                    if (U > umax) umax = U;
                    cnt += 1.0;
                } else if (cu != ORA_CH_FLUID) {
                    tau[0][q] = 0.0; tau[1][q] = 0.0; tau[2][q] = 0.0; tau[3][q] = 0.0;
                }
                int cw = ora_chester_class(phi_w[q], p->band_width);
                if (cw == ORA_CH_BAND) {
                    ora_local_stress(g, p, phi_w, ORA_W, i, j, k, u, v, w,
                                     ln_ratio_at(p, z0, log_z0, q), t, &tw, &U);
                    tau[4][q] = t[2];
                    tau[5][q] = t[5];
                    s_w += tw;
                    if (U > umax) umax = U;
                    cnt += 1.0;
                } else if (cw != ORA_CH_FLUID) {
                    tau[4][q] = 0.0; tau[5][q] = 0.0;
                }
            }
        part[4 * k + 0] = s_uv;
        part[4 * k + 1] = s_w;
        part[4 * k + 2] = umax;
        part[4 * k + 3] = cnt;
    }
    if (stats) {
        stats[0] = stats[1] = stats[2] = stats[3] = 0.0;
        for (long k = 0; k < nz; ++k) {
            stats[0] += part[4 * k + 0];
            stats[1] += part[4 * k + 1];
            if (part[4 * k + 2] > stats[2]) stats[2] = part[4 * k + 2];
            stats[3] += part[4 * k + 3];
        }
    }
    free(part);
}

/* Step 2 on the components ``f[0..nc-1]`` of one node set: every solid-band
 * node x takes the straight line, in the distance from the surface, through
 * the two samples of its own components at x + (phi_c - phi) n and
 * x + (2 phi_c - phi) n.  All values are computed from the field as it
 * stands, then written. */
static void chester_extrapolate_set(const ora_grid* g, const ora_params* p, const double* phi,
                                    int kind, double* const* f, int nc) {
    long n = (long)g->nx * g->ny * g->nz;
    long m = 0;
    for (long q = 0; q < n; ++q)
        if (ora_chester_class(phi[q], p->band_width) == ORA_CH_SOLID_BAND) ++m;
    long* idx = (long*)malloc(sizeof(long) * (size_t)(m > 0 ? m : 1));
    double* val = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * nc);
    m = 0;
    for (long q = 0; q < n; ++q)
        if (ora_chester_class(phi[q], p->band_width) == ORA_CH_SOLID_BAND) idx[m++] = q;
#pragma omp parallel for schedule(dynamic, 64)
    for (long r = 0; r < m; ++r) {
        long q = idx[r];
        long i = q % g->nx, j = (q / g->nx) % g->ny, k = q / ((long)g->nx * g->ny);
        double x[3], nrm[3], p1[3], p2[3];
        node_position(g, kind, i, j, k, x);
        ora_normal(g, phi, i, j, k, nrm);
        double d1 = p->phi_c, d2 = 2.0 * p->phi_c;
        for (int d = 0; d < 3; ++d) {
            p1[d] = x[d] + (d1 - phi[q]) * nrm[d];
            p2[d] = x[d] + (d2 - phi[q]) * nrm[d];
        }
        for (int c = 0; c < nc; ++c) {
            double t1 = ora_interp(g, f[c], kind, p1);
            double t2 = ora_interp(g, f[c], kind, p2);
            val[r * nc + c] = t1 + (phi[q] - d1) * (t2 - t1) / (d2 - d1);
        }
    }
    for (long r = 0; r < m; ++r)
        for (int c = 0; c < nc; ++c) f[c][idx[r]] = val[r * nc + c];
    free(idx);
    free(val);
}

void ora_chester_extrapolate(const ora_grid* g, const ora_params* p, const double* phi_uv,
                             const double* phi_w, double* const tau[6]) {
    double* const uvf[4] = {tau[0], tau[1], tau[2], tau[3]};
    double* const wf[2] = {tau[4], tau[5]};
    chester_extrapolate_set(g, p, phi_uv, ORA_UV, uvf, 4);
    chester_extrapolate_set(g, p, phi_w, ORA_W, wf, 2);
}

/* Step 3 on one node set: ``iterations`` red-black SOR sweeps of the 7-point
 * Laplace equation over the interior nodes (parity of i + j + k; each colour
 * from the values before its half-sweep), all other nodes held fixed. */
static void chester_sor_set(const ora_grid* g, const ora_params* p, const double* phi,
                            double* const* f, int nc, double omega, int iterations) {
    long n = (long)g->nx * g->ny * g->nz;
    const double ax = 1.0 / (g->dx * g->dx), ay = 1.0 / (g->dy * g->dy),
                 az = 1.0 / (g->dz * g->dz);
    const double diag = 2.0 * (ax + ay + az);
    /* the interior nodes of each colour, in ascending linear index */
    long* list[2];
    long m[2] = {0, 0};
    for (int colour = 0; colour < 2; ++colour)
        list[colour] = (long*)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    for (long k = 0; k < g->nz; ++k)
        for (long j = 0; j < g->ny; ++j)
            for (long i = 0; i < g->nx; ++i) {
                long q = lin(g, i, j, k);
                if (ora_chester_class(phi[q], p->band_width) != ORA_CH_INTERIOR) continue;
                int colour = (int)((i + j + k) % 2);
                list[colour][m[colour]++] = q;
            }
    double* nv = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int it = 0; it < iterations; ++it)
        for (int colour = 0; colour < 2; ++colour)
            for (int c = 0; c < nc; ++c) {
                double* a = f[c];
                const long* L = list[colour];
#pragma omp parallel for schedule(static)
                for (long r = 0; r < m[colour]; ++r) {
                    long q = L[r];
                    long i = q % g->nx, j = (q / g->nx) % g->ny, k = q / ((long)g->nx * g->ny);
                    double s = ax * (at_padded(g, a, i + 1, j, k) + at_padded(g, a, i - 1, j, k))
                             + ay * (at_padded(g, a, i, j + 1, k) + at_padded(g, a, i, j - 1, k))
                             + az * (at_padded(g, a, i, j, k + 1) + at_padded(g, a, i, j, k - 1));
                    nv[r] = (1.0 - omega) * a[q] + omega * s / diag;
                }
                for (long r = 0; r < m[colour]; ++r) a[L[r]] = nv[r];
            }
    free(nv);
    free(list[0]);
    free(list[1]);
}

void ora_chester_sor(const ora_grid* g, const ora_params* p, const double* phi_uv,
                     const double* phi_w, double omega, int iterations, double* const tau[6]) {
    double* const uvf[4] = {tau[0], tau[1], tau[2], tau[3]};
    double* const wf[2] = {tau[4], tau[5]};
    chester_sor_set(g, p, phi_uv, uvf, 4, omega, iterations);
    chester_sor_set(g, p, phi_w, wf, 2, omega, iterations);
}
