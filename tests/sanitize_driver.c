/* Calls every routine of the oracle (oracle/ibm_oracle.c) on a small ragged,
 * anisotropic grid with a tilted-plane-plus-bump level set, so a host build
 * with AddressSanitizer and UndefinedBehaviorSanitizer can check its memory
 * accesses and arithmetic.  Exit status 0 when every call returned. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ibm_oracle.h"

static uint64_t state = 0x9e3779b97f4a7c15ull;

static double urand(void) {   /* uniform in [-1, 1) */
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static double* field(long n, double scale) {
    double* f = malloc(sizeof(double) * (size_t)n);
    for (long q = 0; q < n; ++q) f[q] = scale * urand();
    return f;
}

int main(void) {
    const ora_grid g = {13, 9, 11, 0.8, 1.3, 0.9};
    const ora_params p = {1.5 * g.dz, 2.0 * g.dz, 0.4};
    const long n = (long)g.nx * g.ny * g.nz;
    double* phi_uv = malloc(sizeof(double) * (size_t)n);
    double* phi_w = malloc(sizeof(double) * (size_t)n);
    for (int k = 0; k < g.nz; ++k)
        for (int j = 0; j < g.ny; ++j)
            for (int i = 0; i < g.nx; ++i) {
                const long q = ((long)k * g.ny + j) * g.nx + i;
                const double x = i * g.dx, y = j * g.dy;
                const double zs = 2.0 + 0.2 * x - 0.1 * y + 1.5 * exp(-((x - 5) * (x - 5) + (y - 6) * (y - 6)) / 8);
                phi_uv[q] = (k + 0.5) * g.dz - zs;
                phi_w[q] = k * g.dz - zs;
            }
    double *u = field(n, 2.0), *v = field(n, 2.0), *w = field(n, 0.5), *lz = field(n, 1.0);
    for (long q = 0; q < n; ++q) lz[q] = log(1e-3) + 0.3 * lz[q];
    double* tau[6];
    double* tau2[6];
    for (int c = 0; c < 6; ++c) {
        tau[c] = field(n, 0.01);
        tau2[c] = field(n, 0.01);
    }
    uint8_t* mask = malloc((size_t)n);
    ora_classify(&g, &p, phi_uv, phi_w, mask);
    int64_t counts[6];
    ora_counts(&g, &p, phi_uv, phi_w, counts);
    double stats[4];
    ora_wall_stress(&g, &p, phi_uv, phi_w, u, v, w, 1e-3, NULL, tau, stats);
    ora_wall_stress(&g, &p, phi_uv, phi_w, u, v, w, 0.0, lz, tau2, stats);
    double* div[3];
    double* gp[3];
    double* us[3];
    for (int c = 0; c < 3; ++c) {
        div[c] = field(n, 0.0);
        gp[c] = field(n, 0.1);
        us[c] = field(n, 1.0);
    }
    ora_divergence(&g, (const double* const*)tau, div);
    double* gt[6];
    for (int c = 0; c < 6; ++c) gt[c] = field(n, 0.0);
    ora_divergence_transpose(&g, (const double* const*)div, gt);
    ora_forcing(&g, phi_uv, phi_w, us, (const double* const*)gp, 0.01);
    ora_forcing(&g, phi_uv, phi_w, us, NULL, 0.01);
    double drag[3];
    ora_drag(&g, phi_uv, phi_w, (const double* const*)div, drag);
    double nrm[3], pt[3] = {0.0, 0.0, 0.0};
    const long corners[4][3] = {{0, 0, 0}, {g.nx - 1, g.ny - 1, g.nz - 1}, {0, g.ny - 1, 1}, {5, 4, 0}};
    for (int c = 0; c < 4; ++c) {
        ora_normal(&g, phi_uv, corners[c][0], corners[c][1], corners[c][2], nrm);
        ora_normal(&g, phi_w, corners[c][0], corners[c][1], corners[c][2], nrm);
    }
    for (int t = 0; t < 64; ++t) {
        pt[0] = 1.5 * g.nx * g.dx * urand();
        pt[1] = 1.5 * g.ny * g.dy * urand();
        pt[2] = 0.5 * g.nz * g.dz * (1.0 + urand());
        (void)ora_interp(&g, u, ORA_UV, pt);
        (void)ora_interp(&g, w, ORA_W, pt);
        ora_interp_scatter(&g, gt[0], ORA_UV, pt, 1.0);
        ora_interp_scatter(&g, gt[1], ORA_W, pt, 1.0);
    }
    double *gu = field(n, 0.0), *gv = field(n, 0.0), *gw = field(n, 0.0), *glz = field(n, 0.0);
    const double gdrag[3] = {0.3, -0.2, 0.1};
    const double* gtn[6] = {NULL, gt[1], NULL, gt[3], gt[4], NULL};
    ora_stage_vjp(&g, &p, phi_uv, phi_w, u, v, w, 1e-3, NULL, gtn, (const double* const*)div,
                  (const double* const*)us, gdrag, gu, gv, gw, NULL);
    ora_stage_vjp(&g, &p, phi_uv, phi_w, u, v, w, 0.0, lz, (const double* const*)gt,
                  (const double* const*)div, (const double* const*)us, gdrag, gu, gv, gw, glz);
    ora_smagorinsky(&g, 0.16, 0.4, phi_uv, phi_w, u, v, w, 1e-3, NULL, tau);
    ora_smagorinsky(&g, 0.16, 0.4, phi_uv, phi_w, u, v, w, 0.0, lz, tau2);
    printf("oracle routines ran: counts %lld %lld %lld, drag %.6e\n", (long long)counts[0],
           (long long)counts[1], (long long)counts[2], drag[0]);
    for (int c = 0; c < 6; ++c) {
        free(tau[c]);
        free(tau2[c]);
        free(gt[c]);
    }
    for (int c = 0; c < 3; ++c) {
        free(div[c]);
        free(gp[c]);
        free(us[c]);
    }
    free(phi_uv);
    free(phi_w);
    free(u);
    free(v);
    free(w);
    free(lz);
    free(mask);
    free(gu);
    free(gv);
    free(gw);
    free(glz);
    return 0;
}
