// ibm_impl.h -- internal types of the MI355X wall-modeled IBM library.
//
// Data kept on the device per context (all owned by the library):
//  * mask    : one byte per linear index (classes of both grids + forcing flags)
//  * fmask   : forcing flags packed 2 bits per node (bit 2t: uv forced, bit 2t+1:
//              w forced) in 32-bit words, rows padded to whole words; the dense
//              pass reads 1/4 byte per node instead of the whole mask byte
//  * records : one structure-of-arrays per grid with the band nodes in ascending
//              linear index: index, unit normal, phi, and the trilinear stencil of
//              the sample point on the uv and on the w node set
//  * zsegs   : segments of kSeg consecutive linear indices holding a solid node
//              of either grid; their solid nodes' stress is zeroed each step
//  * fsegs   : segments holding a forced node (phi <= 0) of either grid; their
//              forced nodes' intermediate velocity is set each step
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ibm.h"

namespace ibm {

constexpr int kWave = 64;
constexpr int kSeg = 4096;
constexpr int kBandBlock = 256;

// Band records of one grid.  T arrays are the context's storage type.
struct Records {
    long n = 0;
    void* buf = nullptr;
    int32_t* q = nullptr;     // linear index of the band node
    int32_t* base = nullptr;  // j0 * nx + i0: lower corner column of the sample stencil
    int32_t* sx = nullptr;    // x step to the upper corner (1 or 1 - nx across the seam)
    int32_t* sy = nullptr;    // y step (nx or (1 - ny) * nx)
    int32_t* ku = nullptr;    // lower vertical index of the uv-grid stencil
    int32_t* kw = nullptr;    // lower vertical index of the w-grid stencil
    void* nrm[3] = {nullptr, nullptr, nullptr};
    void* phi = nullptr;
    void* fx = nullptr;       // fractions of the stencil
    void* fy = nullptr;
    void* fzu = nullptr;
    void* fzw = nullptr;
};

template <typename T>
struct RecView {
    long n;
    const int32_t *q, *base, *sx, *sy, *ku, *kw;
    const T *nx, *ny, *nz, *phi, *fx, *fy, *fzu, *fzw;
};

template <typename T>
inline RecView<T> view(const Records& r) {
    return RecView<T>{r.n, r.q, r.base, r.sx, r.sy, r.ku, r.kw,
                      (const T*)r.nrm[0], (const T*)r.nrm[1], (const T*)r.nrm[2],
                      (const T*)r.phi, (const T*)r.fx, (const T*)r.fy,
                      (const T*)r.fzu, (const T*)r.fzw};
}

// A segment of consecutive linear indices [q, q + len), len <= kSeg, and which
// grids hold a solid (zsegs) or forced (fsegs) node in it: bit 0 uv, bit 1 w.
struct Seg {
    int32_t q;
    int32_t len;
    int32_t sel;
    int32_t pad;
};

// Tile shape of the dense pass: a wave owns 64*vx points along x, ty rows and
// up to kz planes; wpb waves per block.
struct TileCfg {
    int vx = 4, ty = 4, kz = 16, wpb = 4;
};

// Twiddle tables of the pseudo-spectral mode (built on first use).
struct SpectralTw {
    void* twx = nullptr;   // exp(-2 pi i t / nx), t < nx, storage-type complex
    void* twy = nullptr;
};

// Workspace of the pressure projection (allocated on first use): three
// half-spectrum complex volumes of the storage type (nz x ny x (nx/2 + 1)
// modes, rows padded to an even count).
struct ProjWs {
    void* buf = nullptr;
    size_t bytes = 0;
};

// Transposed sample-stencil map for the reverse mode (built on first use).
struct AdjointMap {
    bool built = false;
    long m[2] = {0, 0};          // number of distinct touched nodes (uv grid, w grid)
    long e[2] = {0, 0};          // number of entries
    int32_t* node[2] = {nullptr, nullptr};
    int32_t* off[2] = {nullptr, nullptr};
    int32_t* rec[2] = {nullptr, nullptr};   // record index in [uv records | w records]
    void* wgt[2] = {nullptr, nullptr};      // trilinear weight of the entry's corner (storage type)
    void* rbar = nullptr;        // per-record sample-velocity cotangents, 3 x (nuv + nw)
    long nb = 0;                 // band nodes (a uv record, a w record or both)
    int32_t* brec = nullptr;     // per band node, ascending: [uv record or -1, w record or -1]
};

// Set-up of Chester et al.'s original method (built by ibm_chester_prepare).
// Both node sets are classified alike: 0 fluid (phi > b), 1 fluid band
// (0 <= phi <= b), 2 solid band (-b <= phi < 0), 3 body interior (phi < -b);
// the class byte holds the uv class in bits 0-1 and the w class in bits 2-3.
struct ChesterGeom {
    bool built = false;
    uint8_t* mask = nullptr;
    int64_t counts[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // [uv class 0..3, w class 0..3]
    Records band[2];             // fluid band: sample stencil at distance phi_c
    Records sb1[2];              // solid band: stencils at distances phi_c ...
    Records sb2[2];              // ... and 2 phi_c from the surface along the normal
    void* lists = nullptr;       // interior nodes of each node set and colour
    int32_t* inner[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    long ninner[2][2] = {{0, 0}, {0, 0}};
    void* ext = nullptr;         // extrapolated values: 4 per uv, 2 per w solid-band record
    long nzsegs = 0;
    Seg* zsegs = nullptr;        // segments holding a node with phi < 0 on either set
    double* partials = nullptr;  // statistics slots, 4 per fluid-band block
};

}  // namespace ibm

struct ibm_ctx {
    int device = 0;
    ibm_grid g{};
    int dtype = IBM_F32;
    int precision = IBM_PREC_PLAIN;
    ibm_params p{};
    bool prepared = false;
    long n = 0;
    int wrow = 0;                       // 32-bit fmask words per row
    uint8_t* mask = nullptr;
    uint32_t* fmask = nullptr;
    int64_t counts[6] = {0, 0, 0, 0, 0, 0};
    ibm::Records rec[2];
    long nzsegs = 0;
    ibm::Seg* zsegs = nullptr;
    long nfsegs = 0;
    ibm::Seg* fsegs = nullptr;
    double* ws_partials = nullptr;      // wall_stress block slots (4 per band block)
    long ws_cap = 0;                    // in doubles
    double* ap_partials = nullptr;      // apply wave slots (3 per tile)
    long ap_cap = 0;                    // in doubles
    ibm::TileCfg cfg;
    ibm::TileCfg sgs_cfg;               // the Smagorinsky kernel's tile (ty = 1) ...
    bool sgs_tuned = false;             // ... when the autotuner chose one; else cfg's
    ibm::AdjointMap adj;
    ibm::SpectralTw spec;
    ibm::ProjWs proj;
    ibm::ChesterGeom ch;
    // bumped whenever the tile shape or any prepared device buffer may change;
    // a batch compares it against the value its work tables were built with
    unsigned long gen = 0;
};

namespace ibm {

// Thread-local error message and helpers (api.hip).
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
size_t tsize(const ibm_ctx* c);

// prepare.hip
int prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w, hipStream_t s);
void free_prepared(ibm_ctx* c);

// stage.hip
int launch_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
                       const void* log_z0, void* const tau[6], double* stats, hipStream_t s);
// ``partials``: the drag slots (3 per tile) to use instead of the context's
// (NULL: the context's, sized by size_partials).
int launch_apply(ibm_ctx* c, const TileCfg& cfg, const void* const tau[6], void* const ustar[3],
                 const void* const gradp[3], double dt, void* const div[3], double* drag,
                 hipStream_t s, double* partials = nullptr);
// ibm_wall_stress then ibm_apply, with one launch for both slot sums.
int launch_stage(ibm_ctx* c, const TileCfg& cfg, const void* u, const void* v, const void* w,
                 double z0, const void* log_z0, void* const tau[6], void* const ustar[3],
                 const void* const gradp[3], double dt, void* const div[3], double* stats,
                 double* drag, hipStream_t s);
bool tile_supported(const ibm_ctx* c, const TileCfg& cfg);
TileCfg default_tile(const ibm_ctx* c);
long apply_tiles(const ibm_ctx* c, const TileCfg& cfg);
long band_blocks(const ibm_ctx* c);
// Size the reduction slots for the current geometry and tile shape.  Called
// outside launches; waits for the device before freeing a smaller buffer.
int size_partials(ibm_ctx* c);

// spectral.hip
int launch_apply_spectral(ibm_ctx* c, const void* const tau[6], void* const ustar[3],
                          const void* const gradp[3], double dt, void* const div[3],
                          double* drag, hipStream_t s);
long spectral_slots(const ibm_ctx* c);   // reduction slots (doubles) it needs
int ensure_twiddles(ibm_ctx* c);          // twiddle tables of nx and ny (first use: synchronous)
// IBM_E_UNSUPPORTED unless nx and ny are powers of two that one block's
// thread teams and LDS hold (float: <= 2048, double: <= 1024).
int spectral_check(const ibm_ctx* c);
// Dynamic LDS bytes of a 256-thread transform block for sequences of n that
// exchanges ``seqs`` sequences at once.
size_t spectral_lds_bytes(const ibm_ctx* c, int n, int seqs, int threads = 256);
void free_spectral(ibm_ctx* c);

// projection.hip
int launch_pressure_project(ibm_ctx* c, const void* const ustar[3], double dt,
                            void* const u_out[3], void* p_out, hipStream_t s);
int launch_ab2(ibm_ctx* c, const void* const u[3], const void* const rhs_now[3],
               const void* const rhs_prev[3], double dt, void* const ustar[3], hipStream_t s);
void free_projection(ibm_ctx* c);

// sgs_apply.hip
long sgs_apply_blocks(const ibm_ctx* c);   // dense blocks = drag slots / 3
int launch_sgs_apply(ibm_ctx* c, const void* phi_uv, const void* phi_w, const void* u,
                     const void* v, const void* w, double z0, const void* log_z0, double cs,
                     double kappa, const void* const tau[6], void* const ustar[3],
                     const void* const gradp[3], double dt, void* const div[3], double* drag,
                     hipStream_t s);

// sgs.hip
int launch_sgs(ibm_ctx* c, const TileCfg& cfg, const void* phi_uv, const void* phi_w,
               const void* u, const void* v, const void* w, double z0, const void* log_z0,
               double cs, double kappa, void* const tau[6], hipStream_t s);

// chester.hip
int chester_prepare(ibm_ctx* c, const void* phi_uv, const void* phi_w, hipStream_t s);
int launch_chester_wall_stress(ibm_ctx* c, const void* u, const void* v, const void* w,
                               double z0, const void* log_z0, void* const tau[6], double omega,
                               int iterations, double* stats, hipStream_t s);
void free_chester(ibm_ctx* c);

// batch.hip
int autotune(ibm_ctx* c, const char* cache_path, int flags, hipStream_t s);

// vjp.hip
int stage_vjp(ibm_ctx* c, const void* u, const void* v, const void* w, double z0,
              const void* log_z0, const void* const g_tau[6], const void* const g_div[3],
              const void* const g_ustar[3], const double g_drag[3], void* gu, void* gv, void* gw,
              void* glog_z0, hipStream_t s);
void free_adjoint(ibm_ctx* c);

// Make a device current for the duration of a call; restores the caller's.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
    DeviceScope(const DeviceScope&) = delete;
    DeviceScope& operator=(const DeviceScope&) = delete;
};

#define IBM_HIP(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return ::ibm::hip_fail(e_, #call);   \
    } while (0)

}  // namespace ibm
