// api.hip -- the extern "C" entry points declared in include/ibm.h: argument
// checks, context lifetime, error reporting and stream plumbing.  All numeric
// work is in the other sources.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ibm_impl.h"

namespace ibm {

// Drag slots of ibm_apply_noalloc: a static device array, one copy per GPU,
// held until the process ends.  Host code never passes ``scratch`` itself (in
// host code the name is a stand-in, not a device address): its address on
// each device is taken once, at the first ibm_create on that device, and
// kept in g_scratch.
constexpr long kScratchDoubles = 1L << 17;   // 1 MiB: 3 slots per tile, 43690 tiles
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
thread_local char g_err[512] = "";

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// With ``dev`` current: look up and keep this device's address of scratch.
int scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return IBM_OK;   // ibm_apply_noalloc will refuse
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return IBM_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = (double*)p;
    return IBM_OK;
}

double* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? IBM_E_NOMEM : IBM_E_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

size_t tsize(const ibm_ctx* c) { return c->dtype == IBM_F64 ? 8 : 4; }

namespace {

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int check_ctx(const ibm_ctx* c, bool need_prepared, const char* fn) {
    if (!c) return fail(IBM_E_ARG, "%s: context is NULL", fn);
    if (need_prepared && !c->prepared)
        return fail(IBM_E_STATE, "%s: call ibm_levelset_prepare first", fn);
    return IBM_OK;
}

int check_field(const ibm_ctx* c, const void* p, const char* fn, const char* name,
                bool vec_aligned = false) {
    if (!p) return fail(IBM_E_ARG, "%s: %s is NULL", fn, name);
    const uintptr_t a = (uintptr_t)p;
    if (a % tsize(c)) return fail(IBM_E_ARG, "%s: %s is not aligned to its element size", fn, name);
    if (vec_aligned && a % 16)
        return fail(IBM_E_ARG, "%s: %s must be 16-byte aligned", fn, name);
    return IBM_OK;
}

// True if any of the n pointers in ``outs`` equals one of the m pointers in
// ``ins`` (NULL entries ignored) or two entries of ``outs`` are equal.
bool aliases(const void* const* outs, int n, const void* const* ins, int m) {
    for (int i = 0; i < n; ++i) {
        if (!outs[i]) continue;
        for (int j = 0; j < m; ++j)
            if (ins[j] && ins[j] == outs[i]) return true;
        for (int j = i + 1; j < n; ++j)
            if (outs[j] == outs[i]) return true;
    }
    return false;
}

// Argument checks of ibm_apply and ibm_apply_noalloc; leaves the tile shape
// to launch in *cfg (one element per lane for misaligned views).
int check_apply(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                const void* const gradp[3], double dt, void* const div[3], double* drag_dev,
                const char* fn, TileCfg* cfg_out) {
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if (!tau || !ustar || !div) return fail(IBM_E_ARG, "%s: tau, ustar and div are required", fn);
    if (!std::isfinite(dt)) return fail(IBM_E_ARG, "%s: dt must be finite", fn);
    TileCfg cfg = c->cfg;
    bool vec = cfg.vx > 1;
    for (int pass = 0; pass < 2; ++pass) {
        bool ok = true;
        for (int i = 0; i < 6 && ok; ++i)
            ok = tau[i] && (uintptr_t)tau[i] % (vec ? 16 : tsize(c)) == 0;
        for (int i = 0; i < 3 && ok; ++i) ok = div[i] && (uintptr_t)div[i] % (vec ? 16 : tsize(c)) == 0;
        if (ok) break;
        if (!vec) break;
        cfg.vx = 1;   // a misaligned view: fall back to one element per lane
        vec = false;
    }
    for (int i = 0; i < 6; ++i)
        if ((rc = check_field(c, tau[i], fn, "tau[i]"))) return rc;
    for (int i = 0; i < 3; ++i) {
        if ((rc = check_field(c, div[i], fn, "div[i]"))) return rc;
        if ((rc = check_field(c, ustar[i], fn, "ustar[i]"))) return rc;
        if (gradp && gradp[i] && (rc = check_field(c, gradp[i], fn, "gradp[i]"))) return rc;
    }
    if (drag_dev && ((uintptr_t)drag_dev % 8)) return fail(IBM_E_ARG, "%s: drag_dev misaligned", fn);
    {   // one launch reads tau and gradp and writes div and ustar
        const void* ins[9] = {tau[0], tau[1], tau[2], tau[3], tau[4], tau[5],
                              gradp ? gradp[0] : nullptr, gradp ? gradp[1] : nullptr,
                              gradp ? gradp[2] : nullptr};
        const void* outs[3] = {div[0], div[1], div[2]};
        if (aliases(outs, 3, ins, 9) || aliases(outs, 3, (const void* const*)ustar, 3))
            return fail(IBM_E_ARG, "%s: div entries must be distinct and may not alias tau, gradp or ustar", fn);
        const void* us[3] = {ustar[0], ustar[1], ustar[2]};
        if (aliases(us, 3, ins, 6))
            return fail(IBM_E_ARG, "%s: ustar entries must be distinct and may not alias tau", fn);
    }
    *cfg_out = cfg;
    return IBM_OK;
}
}  // namespace
}  // namespace ibm

using namespace ibm;

extern "C" {

const char* ibm_last_error(void) { return ibm::g_err; }

int ibm_create(ibm_ctx** out, const ibm_grid* g, int dtype, int precision) {
    g_err[0] = 0;
    if (!out || !g) return fail(IBM_E_ARG, "ibm_create: NULL argument");
    *out = nullptr;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(IBM_E_ARG, "ibm_create: grid sizes must be >= 1 (got %d %d %d)", g->nx, g->ny,
                    g->nz);
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz))
        return fail(IBM_E_ARG, "ibm_create: grid spacings must be finite and > 0");
    const long n = (long)g->nx * g->ny * g->nz;
    if (n > 2147483647L) return fail(IBM_E_ARG, "ibm_create: nx*ny*nz exceeds 2^31-1");
    if (dtype != IBM_F32 && dtype != IBM_F64) return fail(IBM_E_ARG, "ibm_create: bad dtype %d", dtype);
    if (precision != IBM_PREC_PLAIN && precision != IBM_PREC_MIXED)
        return fail(IBM_E_ARG, "ibm_create: bad precision %d", precision);
    if (precision == IBM_PREC_MIXED && dtype != IBM_F32)
        return fail(IBM_E_UNSUPPORTED, "ibm_create: mixed precision needs float storage");
    ibm_ctx* c = new (std::nothrow) ibm_ctx();
    if (!c) return fail(IBM_E_NOMEM, "ibm_create: out of host memory");
    c->g = *g;
    c->dtype = dtype;
    c->precision = precision;
    c->n = n;
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDevice");
    }
    c->cfg = default_tile(c);
    const int rc = scratch_init(c->device);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return IBM_OK;
}

int ibm_destroy(ibm_ctx* c) {
    if (!c) return IBM_OK;
    DeviceScope dg(c->device);
    free_prepared(c);
    free_spectral(c);
    free_projection(c);
    (void)hipFree(c->ws_partials);
    (void)hipFree(c->ap_partials);
    delete c;
    return IBM_OK;
}

int ibm_levelset_prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w, const ibm_params* p,
                         void* stream) {
    g_err[0] = 0;
    int rc = check_ctx(c, false, "ibm_levelset_prepare");
    if (rc) return rc;
    if (!p) return fail(IBM_E_ARG, "ibm_levelset_prepare: params is NULL");
    if ((rc = check_field(c, phi_uv, "ibm_levelset_prepare", "phi_uv"))) return rc;
    if ((rc = check_field(c, phi_w, "ibm_levelset_prepare", "phi_w"))) return rc;
    ibm_params q = *p;
    if (!(q.phi_c > 0.0)) q.phi_c = q.band_width;
    if (!finite_pos(q.band_width))
        return fail(IBM_E_RANGE, "ibm_levelset_prepare: band_width must be finite and > 0");
    if (!std::isfinite(q.phi_c) || q.phi_c < q.band_width)
        return fail(IBM_E_RANGE, "ibm_levelset_prepare: phi_c must be >= band_width (phi_c >= 2 phi_b)");
    if (!finite_pos(q.kappa)) return fail(IBM_E_RANGE, "ibm_levelset_prepare: kappa must be > 0");
    DeviceScope dg(c->device);
    c->p = q;
    ++c->gen;
    rc = prepare(c, phi_uv, phi_w, (hipStream_t)stream);
    if (rc) return rc;
    return size_partials(c);
}

int ibm_counts(const ibm_ctx* c, int64_t out[6]) {
    int rc = check_ctx(c, true, "ibm_counts");
    if (rc) return rc;
    if (!out) return fail(IBM_E_ARG, "ibm_counts: out is NULL");
    for (int i = 0; i < 6; ++i) out[i] = c->counts[i];
    return IBM_OK;
}

int ibm_band_size(const ibm_ctx* c, int grid, int64_t* n) {
    int rc = check_ctx(c, true, "ibm_band_size");
    if (rc) return rc;
    if ((grid != IBM_GRID_UV && grid != IBM_GRID_W) || !n)
        return fail(IBM_E_ARG, "ibm_band_size: bad grid or NULL output");
    *n = c->rec[grid].n;
    return IBM_OK;
}

int ibm_band_export(const ibm_ctx* c, int grid, int32_t* idx_host, double* normals_host) {
    int rc = check_ctx(c, true, "ibm_band_export");
    if (rc) return rc;
    if ((grid != IBM_GRID_UV && grid != IBM_GRID_W) || !idx_host)
        return fail(IBM_E_ARG, "ibm_band_export: bad grid or NULL output");
    DeviceScope dg(c->device);
    const Records& R = c->rec[grid];
    if (R.n == 0) return IBM_OK;
    IBM_HIP(hipMemcpy(idx_host, R.q, sizeof(int32_t) * R.n, hipMemcpyDeviceToHost));
    if (normals_host) {
        std::vector<char> tmp(tsize(c) * R.n);
        for (int d = 0; d < 3; ++d) {
            IBM_HIP(hipMemcpy(tmp.data(), R.nrm[d], tmp.size(), hipMemcpyDeviceToHost));
            for (long r = 0; r < R.n; ++r)
                normals_host[3 * r + d] = c->dtype == IBM_F64 ? ((double*)tmp.data())[r]
                                                               : (double)((float*)tmp.data())[r];
        }
    }
    return IBM_OK;
}

int ibm_mask_export(const ibm_ctx* c, uint8_t* mask_host) {
    int rc = check_ctx(c, true, "ibm_mask_export");
    if (rc) return rc;
    if (!mask_host) return fail(IBM_E_ARG, "ibm_mask_export: NULL output");
    DeviceScope dg(c->device);
    IBM_HIP(hipMemcpy(mask_host, c->mask, (size_t)c->n, hipMemcpyDeviceToHost));
    return IBM_OK;
}

int ibm_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                    const void* log_z0, void* const tau[6], double* stats_dev, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_wall_stress";
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if ((rc = check_field(c, u, fn, "u")) || (rc = check_field(c, v, fn, "v")) ||
        (rc = check_field(c, w, fn, "w")))
        return rc;
    if (!tau) return fail(IBM_E_ARG, "%s: tau is NULL", fn);
    for (int i = 0; i < 6; ++i)
        if ((rc = check_field(c, tau[i], fn, "tau[i]"))) return rc;
    if (log_z0) {
        if ((rc = check_field(c, log_z0, fn, "log_z0"))) return rc;
    } else if (!(z0 > 0.0) || !(z0 < c->p.phi_c)) {
        return fail(IBM_E_RANGE, "%s: z0 must satisfy 0 < z0 < phi_c (got %g)", fn, z0);
    }
    if (stats_dev && ((uintptr_t)stats_dev % 8))
        return fail(IBM_E_ARG, "%s: stats_dev misaligned", fn);
    {   // one launch gathers u, v, w and writes tau
        const void* ins[4] = {u, v, w, log_z0};
        const void* outs[6] = {tau[0], tau[1], tau[2], tau[3], tau[4], tau[5]};
        if (aliases(outs, 6, ins, 4))
            return fail(IBM_E_ARG, "%s: tau entries must be distinct and may not alias u, v, w or log_z0", fn);
    }
    DeviceScope dg(c->device);
    return launch_wall_stress(c, u, v, w, z0, log_z0, tau, stats_dev, (hipStream_t)stream);
}

int ibm_apply(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
              const void* const gradp[3], double dt, void* const div[3], double* drag_dev,
              void* stream) {
    g_err[0] = 0;
    TileCfg cfg;
    const int rc = check_apply(c, tau, ustar, gradp, dt, div, drag_dev, "ibm_apply", &cfg);
    if (rc) return rc;
    DeviceScope dg(c->device);
    return launch_apply(c, cfg, tau, ustar, gradp, dt, div, drag_dev, (hipStream_t)stream);
}

int ibm_apply_noalloc(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                      const void* const gradp[3], double dt, void* const div[3],
                      double* drag_dev, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_apply_noalloc";
    TileCfg cfg;
    int rc = check_apply(c, tau, ustar, gradp, dt, div, drag_dev, fn, &cfg);
    if (rc) return rc;
    double* slots = nullptr;
    if (drag_dev) {
        const long need = 3 * apply_tiles(c, cfg);
        if (need > kScratchDoubles)
            return fail(IBM_E_RANGE, "%s: %ld drag slots needed (3 per tile), the static scratch "
                        "holds %ld; use ibm_apply or a tile shape with fewer tiles", fn, need,
                        kScratchDoubles);
        slots = scratch_ptr(c->device);
        if (!slots)
            return fail(IBM_E_STATE, "%s: no static scratch on device %d", fn, c->device);
    }
    DeviceScope dg(c->device);
    return launch_apply(c, cfg, tau, ustar, gradp, dt, div, drag_dev, (hipStream_t)stream, slots);
}

int ibm_stage(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
              const void* log_z0, void* const tau[6], void* const ustar[3],
              const void* const gradp[3], double dt, void* const div[3], double* stats_dev,
              double* drag_dev, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_stage";
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if ((rc = check_field(c, u, fn, "u")) || (rc = check_field(c, v, fn, "v")) ||
        (rc = check_field(c, w, fn, "w")))
        return rc;
    if (log_z0) {
        if ((rc = check_field(c, log_z0, fn, "log_z0"))) return rc;
    } else if (!(z0 > 0.0) || !(z0 < c->p.phi_c)) {
        return fail(IBM_E_RANGE, "%s: z0 must satisfy 0 < z0 < phi_c (got %g)", fn, z0);
    }
    if (stats_dev && ((uintptr_t)stats_dev % 8))
        return fail(IBM_E_ARG, "%s: stats_dev misaligned", fn);
    TileCfg cfg;
    if ((rc = check_apply(c, tau, ustar, gradp, dt, div, drag_dev, fn, &cfg))) return rc;
    {   // the wall-stress kernel gathers u, v, w and writes tau
        const void* ins[4] = {u, v, w, log_z0};
        const void* outs[6] = {tau[0], tau[1], tau[2], tau[3], tau[4], tau[5]};
        if (aliases(outs, 6, ins, 4))
            return fail(IBM_E_ARG, "%s: tau entries must be distinct and may not alias u, v, w or log_z0", fn);
    }
    DeviceScope dg(c->device);
    return launch_stage(c, cfg, u, v, w, z0, log_z0, tau, ustar, gradp, dt, div, stats_dev,
                        drag_dev, (hipStream_t)stream);
}

int ibm_apply_spectral(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                       const void* const gradp[3], double dt, void* const div[3],
                       double* drag_dev, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_apply_spectral";
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if (!tau || !ustar || !div) return fail(IBM_E_ARG, "%s: tau, ustar and div are required", fn);
    if (!std::isfinite(dt)) return fail(IBM_E_ARG, "%s: dt must be finite", fn);
    for (int i = 0; i < 6; ++i)
        if ((rc = check_field(c, tau[i], fn, "tau[i]"))) return rc;
    for (int i = 0; i < 3; ++i) {
        if ((rc = check_field(c, div[i], fn, "div[i]"))) return rc;
        if ((rc = check_field(c, ustar[i], fn, "ustar[i]"))) return rc;
        if (gradp && gradp[i] && (rc = check_field(c, gradp[i], fn, "gradp[i]"))) return rc;
        for (int j = 0; j < 6; ++j)
            if (div[i] == tau[j]) return fail(IBM_E_ARG, "%s: div may not alias tau", fn);
    }
    if (drag_dev && ((uintptr_t)drag_dev % 8)) return fail(IBM_E_ARG, "%s: drag_dev misaligned", fn);
    {   // one launch reads tau and gradp and writes div and ustar
        const void* ins[9] = {tau[0], tau[1], tau[2], tau[3], tau[4], tau[5],
                              gradp ? gradp[0] : nullptr, gradp ? gradp[1] : nullptr,
                              gradp ? gradp[2] : nullptr};
        const void* outs[3] = {div[0], div[1], div[2]};
        if (aliases(outs, 3, ins, 9) || aliases(outs, 3, (const void* const*)ustar, 3))
            return fail(IBM_E_ARG, "%s: div entries must be distinct and may not alias tau, gradp or ustar", fn);
        const void* us[3] = {ustar[0], ustar[1], ustar[2]};
        if (aliases(us, 3, ins, 6))
            return fail(IBM_E_ARG, "%s: ustar entries must be distinct and may not alias tau", fn);
    }
    DeviceScope dg(c->device);
    return launch_apply_spectral(c, tau, ustar, gradp, dt, div, drag_dev, (hipStream_t)stream);
}

int ibm_ab2_predict(ibm_ctx* c, const void* const u[3], const void* const rhs_now[3],
                    const void* const rhs_prev[3], double dt, void* const ustar[3],
                    void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_ab2_predict";
    int rc = check_ctx(c, false, fn);
    if (rc) return rc;
    if (!u || !rhs_now || !rhs_prev || !ustar) return fail(IBM_E_ARG, "%s: NULL field array", fn);
    for (int i = 0; i < 3; ++i)
        if ((rc = check_field(c, u[i], fn, "u[i]")) || (rc = check_field(c, rhs_now[i], fn, "rhs_now[i]")) ||
            (rc = check_field(c, rhs_prev[i], fn, "rhs_prev[i]")) ||
            (rc = check_field(c, ustar[i], fn, "ustar[i]")))
            return rc;
    if (!std::isfinite(dt)) return fail(IBM_E_ARG, "%s: dt must be finite", fn);
    DeviceScope dg(c->device);
    return launch_ab2(c, u, rhs_now, rhs_prev, dt, ustar, (hipStream_t)stream);
}

int ibm_pressure_project(ibm_ctx* c, const void* const ustar[3], double dt, void* const u_out[3],
                         void* p_out, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_pressure_project";
    int rc = check_ctx(c, false, fn);
    if (rc) return rc;
    if (!ustar || !u_out) return fail(IBM_E_ARG, "%s: NULL field array", fn);
    if ((rc = check_field(c, p_out, fn, "p_out"))) return rc;
    for (int i = 0; i < 3; ++i) {
        if ((rc = check_field(c, ustar[i], fn, "ustar[i]")) ||
            (rc = check_field(c, u_out[i], fn, "u_out[i]")))
            return rc;
        if (p_out == ustar[i] || p_out == u_out[i])
            return fail(IBM_E_ARG, "%s: p_out may not alias a velocity field", fn);
    }
    if (!finite_pos(dt)) return fail(IBM_E_RANGE, "%s: dt must be finite and > 0", fn);
    DeviceScope dg(c->device);
    return launch_pressure_project(c, ustar, dt, u_out, p_out, (hipStream_t)stream);
}

int ibm_sgs_stress(ibm_ctx* c, const void* phi_uv, const void* phi_w, const void* u,
                   const void* v, const void* w, double z0, const void* log_z0, double cs,
                   double kappa, void* const tau[6], void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_sgs_stress";
    int rc = check_ctx(c, false, fn);
    if (rc) return rc;
    if ((rc = check_field(c, phi_uv, fn, "phi_uv")) || (rc = check_field(c, phi_w, fn, "phi_w")) ||
        (rc = check_field(c, u, fn, "u")) || (rc = check_field(c, v, fn, "v")) ||
        (rc = check_field(c, w, fn, "w")))
        return rc;
    if (!tau) return fail(IBM_E_ARG, "%s: tau is NULL", fn);
    for (int i = 0; i < 6; ++i) {
        if ((rc = check_field(c, tau[i], fn, "tau[i]"))) return rc;
        if (tau[i] == u || tau[i] == v || tau[i] == w || tau[i] == phi_uv || tau[i] == phi_w ||
            (log_z0 && tau[i] == log_z0))
            return fail(IBM_E_ARG, "%s: tau may not alias an input", fn);
    }
    if (log_z0) {
        if ((rc = check_field(c, log_z0, fn, "log_z0"))) return rc;
    } else if (!finite_pos(z0)) {
        return fail(IBM_E_RANGE, "%s: z0 must be finite and > 0 (got %g)", fn, z0);
    }
    if (!finite_pos(cs) || !finite_pos(kappa))
        return fail(IBM_E_RANGE, "%s: cs and kappa must be finite and > 0", fn);
    TileCfg cfg = c->sgs_tuned ? c->sgs_cfg : c->cfg;
    cfg.ty = 1;
    bool vec = cfg.vx > 1;
    const void* vecs[6] = {phi_uv, phi_w, u, v, w, log_z0};
    for (const void* p : vecs) vec = vec && (!p || (uintptr_t)p % 16 == 0);
    for (int i = 0; i < 6; ++i) vec = vec && (uintptr_t)tau[i] % 16 == 0;
    if (!vec) cfg.vx = 1;   // a misaligned view: one element per lane
    DeviceScope dg(c->device);
    return launch_sgs(c, cfg, phi_uv, phi_w, u, v, w, z0, log_z0, cs, kappa, tau,
                      (hipStream_t)stream);
}

int ibm_apply_sgs(ibm_ctx* c, const void* phi_uv, const void* phi_w, const void* u,
                  const void* v, const void* w, double z0, const void* log_z0, double cs,
                  double kappa, const void* const tau[6], void* const ustar[3],
                  const void* const gradp[3], double dt, void* const div[3], double* drag_dev,
                  void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_apply_sgs";
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if ((rc = check_field(c, phi_uv, fn, "phi_uv")) || (rc = check_field(c, phi_w, fn, "phi_w")) ||
        (rc = check_field(c, u, fn, "u")) || (rc = check_field(c, v, fn, "v")) ||
        (rc = check_field(c, w, fn, "w")))
        return rc;
    if (!tau || !ustar || !div) return fail(IBM_E_ARG, "%s: tau, ustar and div are required", fn);
    if (!std::isfinite(dt)) return fail(IBM_E_ARG, "%s: dt must be finite", fn);
    if (log_z0) {
        if ((rc = check_field(c, log_z0, fn, "log_z0"))) return rc;
    } else if (!finite_pos(z0)) {
        return fail(IBM_E_RANGE, "%s: z0 must be finite and > 0 (got %g)", fn, z0);
    }
    if (!finite_pos(cs) || !finite_pos(kappa))
        return fail(IBM_E_RANGE, "%s: cs and kappa must be finite and > 0", fn);
    for (int i = 0; i < 6; ++i)
        if ((rc = check_field(c, tau[i], fn, "tau[i]"))) return rc;
    // read by the launch that writes ustar, div
    const void* ins[12] = {u, v, w, phi_uv, phi_w, log_z0,
                           tau[0], tau[1], tau[2], tau[3], tau[4], tau[5]};
    for (int i = 0; i < 3; ++i) {
        if ((rc = check_field(c, div[i], fn, "div[i]"))) return rc;
        if ((rc = check_field(c, ustar[i], fn, "ustar[i]"))) return rc;
        if (gradp && gradp[i] && (rc = check_field(c, gradp[i], fn, "gradp[i]"))) return rc;
        for (const void* p : ins)
            if (p && (p == div[i] || p == ustar[i]))
                return fail(IBM_E_ARG, "%s: ustar and div may not alias an input", fn);
    }
    if (drag_dev && ((uintptr_t)drag_dev % 8)) return fail(IBM_E_ARG, "%s: drag_dev misaligned", fn);
    DeviceScope dg(c->device);
    return launch_sgs_apply(c, phi_uv, phi_w, u, v, w, z0, log_z0, cs, kappa, tau, ustar, gradp,
                            dt, div, drag_dev, (hipStream_t)stream);
}

int ibm_chester_prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_chester_prepare";
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if ((rc = check_field(c, phi_uv, fn, "phi_uv")) || (rc = check_field(c, phi_w, fn, "phi_w")))
        return rc;
    // red-black colouring stays a two-colouring across the periodic seams
    if ((c->g.nx > 1 && c->g.nx % 2) || (c->g.ny > 1 && c->g.ny % 2))
        return fail(IBM_E_UNSUPPORTED, "%s: nx and ny must be 1 or even (got %d, %d)", fn, c->g.nx,
                    c->g.ny);
    DeviceScope dg(c->device);
    return chester_prepare(c, phi_uv, phi_w, (hipStream_t)stream);
}

int ibm_chester_counts(const ibm_ctx* c, int64_t out[8]) {
    int rc = check_ctx(c, true, "ibm_chester_counts");
    if (rc) return rc;
    if (!c->ch.built) return fail(IBM_E_STATE, "ibm_chester_counts: call ibm_chester_prepare first");
    if (!out) return fail(IBM_E_ARG, "ibm_chester_counts: out is NULL");
    for (int i = 0; i < 8; ++i) out[i] = c->ch.counts[i];
    return IBM_OK;
}

int ibm_chester_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                            const void* log_z0, void* const tau[6], double omega, int iterations,
                            double* stats_dev, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_chester_wall_stress";
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if (!c->ch.built) return fail(IBM_E_STATE, "%s: call ibm_chester_prepare first", fn);
    if ((rc = check_field(c, u, fn, "u")) || (rc = check_field(c, v, fn, "v")) ||
        (rc = check_field(c, w, fn, "w")))
        return rc;
    if (!tau) return fail(IBM_E_ARG, "%s: tau is NULL", fn);
    for (int i = 0; i < 6; ++i)
        if ((rc = check_field(c, tau[i], fn, "tau[i]"))) return rc;
    if (log_z0) {
        if ((rc = check_field(c, log_z0, fn, "log_z0"))) return rc;
    } else if (!(z0 > 0.0) || !(z0 < c->p.phi_c)) {
        return fail(IBM_E_RANGE, "%s: z0 must satisfy 0 < z0 < phi_c (got %g)", fn, z0);
    }
    if (!(omega > 0.0 && omega < 2.0))
        return fail(IBM_E_RANGE, "%s: omega must lie in (0, 2) (got %g)", fn, omega);
    if (iterations < 0) return fail(IBM_E_ARG, "%s: iterations must be >= 0", fn);
    if (stats_dev && ((uintptr_t)stats_dev % 8))
        return fail(IBM_E_ARG, "%s: stats_dev misaligned", fn);
    {
        const void* ins[4] = {u, v, w, log_z0};
        const void* outs[6] = {tau[0], tau[1], tau[2], tau[3], tau[4], tau[5]};
        if (aliases(outs, 6, ins, 4))
            return fail(IBM_E_ARG, "%s: tau entries must be distinct and may not alias u, v, w or log_z0", fn);
    }
    DeviceScope dg(c->device);
    return launch_chester_wall_stress(c, u, v, w, z0, log_z0, tau, omega, iterations, stats_dev,
                                      (hipStream_t)stream);
}

int ibm_set_tile(ibm_ctx* c, int vx, int ty, int kz, int wpb) {
    g_err[0] = 0;
    int rc = check_ctx(c, false, "ibm_set_tile");
    if (rc) return rc;
    TileCfg t;
    t.vx = vx;
    t.ty = ty;
    t.kz = kz;
    t.wpb = wpb;
    if (!tile_supported(c, t))
        return fail(IBM_E_ARG, "ibm_set_tile: unsupported shape vx=%d ty=%d kz=%d wpb=%d", vx, ty,
                    kz, wpb);
    DeviceScope dg(c->device);
    c->cfg = t;
    c->sgs_tuned = false;   // an explicit tile governs the Smagorinsky kernel too
    ++c->gen;
    return c->prepared ? size_partials(c) : IBM_OK;
}

int ibm_get_tile(const ibm_ctx* c, int out[4]) {
    int rc = check_ctx(c, false, "ibm_get_tile");
    if (rc) return rc;
    if (!out) return fail(IBM_E_ARG, "ibm_get_tile: NULL output");
    out[0] = c->cfg.vx;
    out[1] = c->cfg.ty;
    out[2] = c->cfg.kz;
    out[3] = c->cfg.wpb;
    return IBM_OK;
}

int ibm_stage_vjp(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                  const void* log_z0, const void* const g_tau[6], const void* const g_div[3],
                  const void* const g_ustar[3], const double g_drag[3], void* gu, void* gv,
                  void* gw, void* glog_z0, void* stream) {
    g_err[0] = 0;
    const char* fn = "ibm_stage_vjp";
    int rc = check_ctx(c, true, fn);
    if (rc) return rc;
    if ((rc = check_field(c, u, fn, "u")) || (rc = check_field(c, v, fn, "v")) ||
        (rc = check_field(c, w, fn, "w")) || (rc = check_field(c, gu, fn, "gu")) ||
        (rc = check_field(c, gv, fn, "gv")) || (rc = check_field(c, gw, fn, "gw")))
        return rc;
    if (!g_div || !g_ustar || !g_drag)
        return fail(IBM_E_ARG, "%s: g_div, g_ustar and g_drag are required", fn);
    for (int i = 0; i < 3; ++i) {
        if ((rc = check_field(c, g_div[i], fn, "g_div[i]"))) return rc;
        if ((rc = check_field(c, g_ustar[i], fn, "g_ustar[i]"))) return rc;
        if (!std::isfinite(g_drag[i])) return fail(IBM_E_ARG, "%s: g_drag must be finite", fn);
    }
    if (g_tau)
        for (int i = 0; i < 6; ++i)
            if (g_tau[i] && (rc = check_field(c, g_tau[i], fn, "g_tau[i]"))) return rc;
    if (log_z0) {
        if ((rc = check_field(c, log_z0, fn, "log_z0"))) return rc;
    } else {
        if (glog_z0) return fail(IBM_E_ARG, "%s: glog_z0 needs a log_z0 field", fn);
        if (!(z0 > 0.0) || !(z0 < c->p.phi_c))
            return fail(IBM_E_RANGE, "%s: z0 must satisfy 0 < z0 < phi_c (got %g)", fn, z0);
    }
    if (glog_z0 && (rc = check_field(c, glog_z0, fn, "glog_z0"))) return rc;
    {   // the gradients are written while the inputs are still read
        const void* ins[16] = {u, v, w, log_z0, g_div[0], g_div[1], g_div[2],
                               g_ustar[0], g_ustar[1], g_ustar[2]};
        if (g_tau)
            for (int i = 0; i < 6; ++i) ins[10 + i] = g_tau[i];
        const void* outs[4] = {gu, gv, gw, glog_z0};
        if (aliases(outs, 4, ins, 16))
            return fail(IBM_E_ARG, "%s: gu, gv, gw, glog_z0 must be distinct and may not alias an input", fn);
    }
    // the transposed stencil map keys a record in 29 bits and offsets its
    // eight corners per record in 32-bit signed integers
    const long nrec = c->rec[0].n + c->rec[1].n;
    if (nrec >= (1L << 28))
        return fail(IBM_E_ARG, "%s: %ld band records; the adjoint takes fewer than 2^28", fn, nrec);
    DeviceScope dg(c->device);
    return stage_vjp(c, u, v, w, z0, log_z0, g_tau, g_div, g_ustar, g_drag, gu, gv, gw, glog_z0,
                     (hipStream_t)stream);
}

}  // extern "C"
