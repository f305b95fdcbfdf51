// batch.hip -- an ensemble of grids of different sizes advanced together, and
// the tile autotuner.
//
// Each case of a batch is an ordinary context (prepare.hip builds its masks,
// band records and segment lists).  One step of the whole ensemble is three
// kernels -- wall stress, dense pass, finalize -- captured once in a hipGraph
// and replayed with a single hipGraphLaunch:
//   * the wall stress and the dense pass take one work item per block or per
//     wave from lists that span every case: (case, band block | solid segment)
//     for the wall stress, and for the dense pass the wave-tiles of every case
//     followed by the quarters of the forcing segments;
//   * each list of equal-role items is cut into 8 contiguous slices of equal
//     estimated cost, one per XCD (block b runs on XCD b % 8, and the blocks of
//     one XCD are dispatched in order), so each XCD's L2 sees neighbouring
//     tiles of one case at the same time and the hardware dispatcher balances
//     the waves; the forcing blocks come after every tile block, as in the
//     per-case dense pass;
//   * items call the same device functions as the per-case kernels (kernels.h)
//     with the case's own arguments and tile shape, so every value of a case is
//     bit-identical to a plain call with the same tile shape.
// No memset and no host synchronisation is inside the graph.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.h"

namespace ibm {

struct Split {
    long off[9];
};


}  // namespace ibm

struct ibm_batch {
    int device = 0;
    int dtype = IBM_F32;
    int precision = IBM_PREC_PLAIN;
    int ncases = 0;
    std::vector<ibm_ctx*> cases;
    std::vector<ibm_case_io> io;
    std::vector<char> bound;
    std::vector<double> z0;
    bool prepared = false;
    bool tables = false;
    std::vector<unsigned long> gens;  // ibm_ctx::gen of each case when the tables were built
    void* ws_tab = nullptr;        // WSArgs<T>[ncases]
    void* ap_tab = nullptr;        // ApplyArgs<T>[ncases]
    int* ws_flags = nullptr;       // per case: bit 0 mixed, bit 1 per-node log z0
    int2* ws_items = nullptr;
    int4* ap_items = nullptr;      // wave-tiles of every case, then forcing quarters
    ibm::FinJob* fin = nullptr;
    long nws = 0, nap = 0;         // items of the wall stress; of the dense pass
    long ntiles = 0;               // the dense pass's tile items (the first ntiles of ap_items)
    int nfin = 0;
    ibm::Split ws_split{}, ap_split{};   // XCD slices of the wall-stress items, of the tiles
    unsigned ws_grid = 0, ap_grid = 0;
    int ws_per_xcd = 0, ap_per_xcd = 0;  // blocks per XCD for the longest slice
    int ap_fblocks = 0;                  // forcing blocks after the tile blocks
    double* drag = nullptr;        // [ncases][3], for cases bound without drag_dev
    double* stats = nullptr;       // [ncases][4], for cases bound without stats_dev
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace ibm {
namespace {

// A work table of argument structs, read through the constant address space:
// the pointers loaded from it are then known to be global (only the host
// writes that memory), so their accesses compile to global loads and stores
// with exact wait counts instead of flat ones.  The wall-stress items use it
// (205 against 221 us per ensemble step); the dense-pass tiles keep the
// generic reference, with which their schedule measured faster (867 against
// 921 us).
// (The qualifier exists in the device compilation only; the host pass, which
// parses device code too, sees a plain pointer.)
#if defined(__HIP_DEVICE_COMPILE__)
#define IBM_CONSTANT_AS __attribute__((address_space(4)))
#else
#define IBM_CONSTANT_AS
#endif
template <typename A>
__device__ inline const IBM_CONSTANT_AS A* const_table(const A* t) {
    return (const IBM_CONSTANT_AS A*)t;
}

// One block per item: block b runs on XCD b % 8 and takes item i = b / 8 of
// that XCD's slice.
template <typename T>
__global__ void __launch_bounds__(kBandBlock) k_batch_ws(const WSArgs<T>* __restrict__ tab,
                                                         const int* __restrict__ flags,
                                                         const int2* __restrict__ items, Split sp) {
    const int x = blockIdx.x & 7;
    const long it = sp.off[x] + (blockIdx.x >> 3);
    if (it >= sp.off[x + 1]) return;
    const int2 w = items[it];
    const int cs = __builtin_amdgcn_readfirstlane(w.x);
    const int blk = __builtin_amdgcn_readfirstlane(w.y);
    const WSArgs<T> a = const_table(tab)[cs];
    switch (flags[cs]) {
        case 0: ws_block<T, false, false>(a, blk); break;
        case 1: ws_block<T, true, false>(a, blk); break;
        case 2: ws_block<T, false, true>(a, blk); break;
        default: ws_block<T, true, true>(a, blk); break;
    }
}

// The first 8 * per_xcd blocks own wave-tiles, one per wave: block b runs on
// XCD b % 8 and takes tiles 4 (b / 8) .. 4 (b / 8) + 3 of that XCD's slice.
// The blocks after them force quarters of the forcing segments, one per wave.
template <typename T, typename Acc>
__global__ void __launch_bounds__(256) k_batch_apply(const ApplyArgs<T>* __restrict__ tab,
                                                     const int4* __restrict__ items, Split sp,
                                                     int per_xcd, long nitems, int nfblocks) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntb = 8 * per_xcd;
    if ((int)blockIdx.x >= ntb) {
        for (long it = sp.off[8] + 4L * (blockIdx.x - ntb) + wv; it < nitems; it += 4L * nfblocks) {
            const int4 w = items[it];
            const int cs = __builtin_amdgcn_readfirstlane(w.x);
            const int idx = __builtin_amdgcn_readfirstlane(w.z);
            const ApplyArgs<T>& a = tab[cs];
            const Seg sg = a.fsegs[idx >> 2];
            const int off = (idx & 3) * (kSeg / 4);
            force_seg<T>(a, Seg{sg.q + off, min(kSeg / 4, sg.len - off), 0, 0}, lane, 64);
        }
        return;
    }
    const int x = blockIdx.x & 7;
    const long it = sp.off[x] + 4L * (blockIdx.x >> 3) + wv;
    if (it >= sp.off[x + 1]) return;
    const int4 w = items[it];
    const int cs = __builtin_amdgcn_readfirstlane(w.x);
    const int idx = __builtin_amdgcn_readfirstlane(w.z);
    const int shape = __builtin_amdgcn_readfirstlane(w.w);
    const ApplyArgs<T>& a = tab[cs];
    switch (shape) {
        case 11: apply_tile<T, Acc, 1, 1>(a, idx, lane); break;
        case 12: apply_tile<T, Acc, 1, 2>(a, idx, lane); break;
        case 21: apply_tile<T, Acc, 2, 1>(a, idx, lane); break;
        case 22: apply_tile<T, Acc, 2, 2>(a, idx, lane); break;
        case 41:
            if constexpr (sizeof(T) == 4) apply_tile<T, Acc, 4, 1>(a, idx, lane);
            break;
        case 42:
            if constexpr (sizeof(T) == 4) apply_tile<T, Acc, 4, 2>(a, idx, lane);
            break;
        default: break;
    }
}

__global__ void __launch_bounds__(256) k_batch_finalize(const FinJob* __restrict__ jobs) {
    const FinJob j = jobs[blockIdx.x];
    finalize_slots(j.p, j.nslots, j.nc, j.maxmask, j.scale, j.out);
}

// Cut items with the given costs into 8 contiguous slices of equal cost.
Split split_by_cost(const std::vector<double>& cost) {
    Split s;
    double total = 0.0;
    for (double c : cost) total += c;
    s.off[0] = 0;
    double acc = 0.0;
    int x = 1;
    for (size_t i = 0; i < cost.size() && x < 8; ++i) {
        acc += cost[i];
        while (x < 8 && acc >= total * x / 8.0) s.off[x++] = (long)i + 1;
    }
    while (x < 8) s.off[x++] = (long)cost.size();
    s.off[8] = (long)cost.size();
    return s;
}

void free_tables(ibm_batch* b) {
    // a replay or run of the old tables may still be in flight
    if (b->exec || b->ws_tab) (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    (void)hipFree(b->ws_tab);
    (void)hipFree(b->ap_tab);
    (void)hipFree(b->ws_flags);
    (void)hipFree(b->ws_items);
    (void)hipFree(b->ap_items);
    (void)hipFree(b->fin);
    b->ws_tab = b->ap_tab = nullptr;
    b->ws_flags = nullptr;
    b->ws_items = nullptr;
    b->ap_items = nullptr;
    b->fin = nullptr;
    b->tables = false;
}

// Blocks per XCD for the longest slice when each block takes ``per_block``
// items of its XCD's slice.
int slice_blocks(const Split& sp, int per_block) {
    long m = 0;
    for (int x = 0; x < 8; ++x) m = std::max(m, sp.off[x + 1] - sp.off[x]);
    return (int)((m + per_block - 1) / per_block);
}

template <typename T>
int build_tables(ibm_batch* b) {
    free_tables(b);
    const int n = b->ncases;
    std::vector<WSArgs<T>> ws(n);
    std::vector<ApplyArgs<T>> ap(n);
    std::vector<int> flags(n);
    std::vector<int2> wsi;
    std::vector<int4> api, fpi;   // tile items; forcing items (appended after the tiles)
    std::vector<double> wsc, apc;
    std::vector<FinJob> fin;
    for (int cs = 0; cs < n; ++cs) {
        ibm_ctx* c = b->cases[cs];
        const ibm_case_io& io = b->io[cs];
        if (c->cfg.ty > 2 || (sizeof(T) == 8 && c->cfg.vx > 2))
            return fail(IBM_E_ARG, "batch: case %d tile shape vx=%d ty=%d is not batchable (ty <= 2)",
                        cs, c->cfg.vx, c->cfg.ty);
        if (c->cfg.vx > 1) {
            // vx > 1 moves 16-byte vectors of the stress and divergence fields
            bool al = true;
            for (int i = 0; i < 6; ++i) al = al && (uintptr_t)io.tau[i] % 16 == 0;
            for (int i = 0; i < 3; ++i) al = al && (uintptr_t)io.div[i] % 16 == 0;
            if (!al)
                return fail(IBM_E_ARG, "batch: case %d: tau or div not 16-byte aligned for tile vx=%d",
                            cs, c->cfg.vx);
        }
        double* st = io.stats_dev ? io.stats_dev : b->stats + 4 * cs;
        double* dr = io.drag_dev ? io.drag_dev : b->drag + 3 * cs;
        ws[cs] = make_ws_args<T>(c, (const T*)io.u, (const T*)io.v, (const T*)io.w, b->z0[cs],
                                 (const T*)io.log_z0, io.tau, st);
        ap[cs] = make_apply_args<T>(c, c->cfg, io.tau, io.ustar, io.gradp, io.dt, io.div, dr);
        flags[cs] = (c->precision == IBM_PREC_MIXED ? 1 : 0) | (io.log_z0 ? 2 : 0);
        const long nbb = ws[cs].nb_band;
        for (long k = 0; k < nbb + c->nzsegs; ++k) {
            wsi.push_back(make_int2(cs, (int)k));
            wsc.push_back(k < nbb ? 1.0 : 2.0);    // 256 gathering records; up to kSeg zeroed nodes
        }
        std::vector<Seg> fs(c->nfsegs);
        if (c->nfsegs)
            IBM_HIP(hipMemcpy(fs.data(), c->fsegs, sizeof(Seg) * c->nfsegs, hipMemcpyDeviceToHost));
        for (long k = 0; k < c->nfsegs; ++k)
            for (int part = 0; part < 4 && part * (kSeg / 4) < fs[k].len; ++part)
                fpi.push_back(make_int4(cs, 0, (int)(4 * k + part), 0));
        const int shape = 10 * c->cfg.vx + c->cfg.ty;
        const double tile_pts = 64.0 * c->cfg.vx * c->cfg.ty * std::min(c->cfg.kz, c->g.nz);
        for (long t = 0; t < ap[cs].ntiles; ++t) {
            api.push_back(make_int4(cs, 1, (int)t, shape));
            apc.push_back(tile_pts);
        }
        fin.push_back(FinJob{c->ws_partials, nbb, 4, 1u << 2, 1.0, st});
        fin.push_back(FinJob{c->ap_partials, ap[cs].ntiles, 3, 0u, ap[cs].dv, dr});
    }
    b->nws = (long)wsi.size();
    b->ntiles = (long)api.size();
    api.insert(api.end(), fpi.begin(), fpi.end());
    b->nap = (long)api.size();
    b->nfin = (int)fin.size();
    b->gens.resize(n);
    for (int cs = 0; cs < n; ++cs) b->gens[cs] = b->cases[cs]->gen;
    b->ws_split = split_by_cost(wsc);
    b->ap_split = split_by_cost(apc);
    IBM_HIP(hipMalloc(&b->ws_tab, sizeof(WSArgs<T>) * n));
    IBM_HIP(hipMalloc(&b->ap_tab, sizeof(ApplyArgs<T>) * n));
    IBM_HIP(hipMalloc(&b->ws_flags, sizeof(int) * n));
    IBM_HIP(hipMalloc(&b->ws_items, sizeof(int2) * std::max<long>(1, b->nws)));
    IBM_HIP(hipMalloc(&b->ap_items, sizeof(int4) * std::max<long>(1, b->nap)));
    IBM_HIP(hipMalloc(&b->fin, sizeof(FinJob) * std::max(1, b->nfin)));
    IBM_HIP(hipMemcpy(b->ws_tab, ws.data(), sizeof(WSArgs<T>) * n, hipMemcpyHostToDevice));
    IBM_HIP(hipMemcpy(b->ap_tab, ap.data(), sizeof(ApplyArgs<T>) * n, hipMemcpyHostToDevice));
    IBM_HIP(hipMemcpy(b->ws_flags, flags.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    if (b->nws)
        IBM_HIP(hipMemcpy(b->ws_items, wsi.data(), sizeof(int2) * b->nws, hipMemcpyHostToDevice));
    if (b->nap)
        IBM_HIP(hipMemcpy(b->ap_items, api.data(), sizeof(int4) * b->nap, hipMemcpyHostToDevice));
    IBM_HIP(hipMemcpy(b->fin, fin.data(), sizeof(FinJob) * b->nfin, hipMemcpyHostToDevice));
    b->ws_per_xcd = slice_blocks(b->ws_split, 1);
    b->ws_grid = (unsigned)(8L * b->ws_per_xcd);
    b->ap_per_xcd = slice_blocks(b->ap_split, 4);
    const long nf = b->nap - b->ntiles;
    b->ap_fblocks = (int)std::min<long>((nf + 3) / 4, 2048);
    b->ap_grid = (unsigned)(8L * b->ap_per_xcd + b->ap_fblocks);
    if (8L * b->ap_per_xcd + b->ap_fblocks > INT32_MAX || 8L * b->ws_per_xcd > INT32_MAX)
        return fail(IBM_E_RANGE, "batch: too many work items for one launch");
    b->tables = true;
    return IBM_OK;
}

template <typename T>
int enqueue(ibm_batch* b, hipStream_t s) {
    if (b->nws)
        hipLaunchKernelGGL(k_batch_ws<T>, dim3(b->ws_grid), dim3(kBandBlock), 0, s,
                           (const WSArgs<T>*)b->ws_tab, (const int*)b->ws_flags,
                           (const int2*)b->ws_items, b->ws_split);
    if (b->nap) {
        if (b->precision == IBM_PREC_MIXED || sizeof(T) == 8)
            hipLaunchKernelGGL((k_batch_apply<T, double>), dim3(b->ap_grid), dim3(256), 0, s,
                               (const ApplyArgs<T>*)b->ap_tab, (const int4*)b->ap_items,
                               b->ap_split, b->ap_per_xcd, b->nap, b->ap_fblocks);
        else
            hipLaunchKernelGGL((k_batch_apply<T, float>), dim3(b->ap_grid), dim3(256), 0, s,
                               (const ApplyArgs<T>*)b->ap_tab, (const int4*)b->ap_items,
                               b->ap_split, b->ap_per_xcd, b->nap, b->ap_fblocks);
    }
    hipLaunchKernelGGL(k_batch_finalize, dim3(b->nfin), dim3(256), 0, s, (const FinJob*)b->fin);
    IBM_HIP(hipGetLastError());
    return IBM_OK;
}

// True when a case's tile shape or prepared buffers changed after the tables
// were built (ibm_set_tile, ibm_autotune or ibm_levelset_prepare on a case).
bool stale(const ibm_batch* b) {
    if (!b->tables) return true;
    for (int cs = 0; cs < b->ncases; ++cs)
        if (b->gens[cs] != b->cases[cs]->gen) return true;
    return false;
}

int ensure_tables(ibm_batch* b) {
    if (b->tables && !stale(b)) return IBM_OK;
    free_tables(b);
    for (int cs = 0; cs < b->ncases; ++cs)
        if (!b->bound[cs]) return fail(IBM_E_STATE, "batch: case %d is not bound", cs);
    return b->dtype == IBM_F64 ? build_tables<double>(b) : build_tables<float>(b);
}

// ------------------------------------------------------------------ autotuner
std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

// what: "plain" (the dense pass), "batch" (its batched kernel) or "sgs" (the
// Smagorinsky kernel)
std::string tune_key(const ibm_ctx* c, const char* what) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|%s|%s|%dx%dx%d|%s", arch_name(c->device).c_str(),
             c->dtype == IBM_F64 ? "f64" : "f32", c->precision == IBM_PREC_MIXED ? "mixed" : "plain",
             c->g.nx, c->g.ny, c->g.nz, what);
    return buf;
}

// The cache is a JSON object with one entry per line:
//   "gfx950|f32|mixed|512x256x256|plain": [vx, ty, kz, wpb, ms],
std::map<std::string, std::vector<double>> read_cache(const char* path) {
    std::map<std::string, std::vector<double>> m;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
        const size_t b0 = line.find('[');
        const size_t b1 = line.find(']');
        if (q1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos) continue;
        std::string key = line.substr(q0 + 1, q1 - q0 - 1);
        std::string vals = line.substr(b0 + 1, b1 - b0 - 1);
        std::replace(vals.begin(), vals.end(), ',', ' ');
        std::istringstream is(vals);
        std::vector<double> v;
        double x;
        while (is >> x) v.push_back(x);
        if (v.size() >= 4) m[key] = v;
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, std::vector<double>>& m) {
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        fprintf(f, "\"%s\": [%d, %d, %d, %d, %.6f]%s\n", kv.first.c_str(), (int)kv.second[0],
                (int)kv.second[1], (int)kv.second[2], (int)kv.second[3],
                kv.second.size() > 4 ? kv.second[4] : 0.0, ++i < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    std::rename(tmp.c_str(), path);
}

bool cached(const std::map<std::string, std::vector<double>>& m, const std::string& key, TileCfg& t) {
    auto it = m.find(key);
    if (it == m.end()) return false;
    t.vx = (int)it->second[0];
    t.ty = (int)it->second[1];
    t.kz = (int)it->second[2];
    t.wpb = (int)it->second[3];
    return true;
}

int set_cfg(ibm_ctx* c, const TileCfg& t) {
    c->cfg = t;
    ++c->gen;
    return size_partials(c);
}

}  // namespace

// Time candidate tile shapes of the dense pass on this context's grid (scratch
// fields, so caller data is untouched) and keep the fastest; outside batch
// tuning also those of the Smagorinsky kernel (one row per wave), whose best
// shape differs from the dense pass's (it reads five fields and writes six).
int autotune(ibm_ctx* c, const char* cache_path, int flags, hipStream_t s) {
    const bool batch = flags & IBM_TUNE_BATCH;
    const std::string key = tune_key(c, batch ? "batch" : "plain");
    const std::string skey = tune_key(c, "sgs");
    bool dense = true, sgs = !batch;
    if (cache_path && !(flags & IBM_TUNE_FORCE)) {
        const auto m = read_cache(cache_path);
        TileCfg t;
        if (cached(m, key, t) && tile_supported(c, t)) {
            const int rc = set_cfg(c, t);
            if (rc) return rc;
            dense = false;
        }
        if (sgs && cached(m, skey, t) && t.ty == 1 && tile_supported(c, t)) {
            c->sgs_cfg = t;
            c->sgs_tuned = true;
            sgs = false;
        }
        if (!dense && !sgs) return IBM_OK;
    }
    const size_t ts = tsize(c);
    const size_t fb = ((size_t)c->n * ts + 255) / 256 * 256;
    char* scratch = nullptr;
    IBM_HIP(hipMalloc(&scratch, 15 * fb));
    IBM_HIP(hipMemsetAsync(scratch, 0, 15 * fb, s));
    void* tau[6];
    void* us[3];
    void* dv[3];
    const void* gp[3];
    for (int i = 0; i < 6; ++i) tau[i] = scratch + i * fb;
    for (int i = 0; i < 3; ++i) {
        us[i] = scratch + (6 + i) * fb;
        dv[i] = scratch + (9 + i) * fb;
        gp[i] = scratch + (12 + i) * fb;
    }
    double* drag = nullptr;
    IBM_HIP(hipMalloc(&drag, 3 * sizeof(double)));
    hipEvent_t e0, e1;
    IBM_HIP(hipEventCreate(&e0));
    IBM_HIP(hipEventCreate(&e1));
    const TileCfg keep = c->cfg;
    TileCfg best = keep, sbest = c->cfg;
    float best_ms = 1e30f, sbest_ms = 1e30f;
    const int vxs[3] = {4, 2, 1};
    const int tys[3] = {1, 2, 4};
    const int kzs[6] = {4, 8, 16, 32, 64, 128};
    const int skzs[5] = {16, 32, 64, 128, 256};
    const int wpbs[3] = {1, 2, 4};
    int rc = IBM_OK;
    // mean of 5 launches after one untimed
    auto timed = [&](auto launch, float& ms) -> int {
        int r = launch();
        if (r) return r;
        IBM_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < 5 && r == IBM_OK; ++k) r = launch();
        if (r) return r;
        IBM_HIP(hipEventRecord(e1, s));
        IBM_HIP(hipEventSynchronize(e1));
        IBM_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms /= 5.f;
        return IBM_OK;
    };
    if (dense)
        for (int vx : vxs)
            for (int ty : tys)
                for (int kz : kzs)
                    for (int wpb : wpbs) {
                        TileCfg t;
                        t.vx = vx;
                        t.ty = ty;
                        t.kz = kz;
                        t.wpb = wpb;
                        if (!tile_supported(c, t) || (batch && ty > 2)) continue;
                        if (kz > 2 * c->g.nz && kz != kzs[0]) continue;
                        if ((rc = set_cfg(c, t))) goto done;
                        float ms = 0.f;
                        rc = timed([&] { return launch_apply(c, t, tau, us, gp, 0.01, dv, drag, s); }, ms);
                        if (rc) goto done;
                        if (ms < best_ms) {
                            best_ms = ms;
                            best = t;
                        }
                    }
    if (sgs)
        for (int vx : vxs)
            for (int kz : skzs)
                for (int wpb : wpbs) {
                    TileCfg t;
                    t.vx = vx;
                    t.ty = 1;
                    t.kz = kz;
                    t.wpb = wpb;
                    if (!tile_supported(c, t)) continue;
                    if (kz > 2 * c->g.nz && kz != skzs[0]) continue;
                    float ms = 0.f;
                    rc = timed([&] {
                        return launch_sgs(c, t, gp[0], gp[1], us[0], us[1], us[2], 1e-3, nullptr, 0.16,
                                          0.4, tau, s);
                    }, ms);
                    if (rc) goto done;
                    if (ms < sbest_ms) {
                        sbest_ms = ms;
                        sbest = t;
                    }
                }
done:
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(drag);
    (void)hipFree(scratch);
    if (rc) {
        set_cfg(c, keep);
        return rc;
    }
    if (dense) rc = set_cfg(c, best);
    if (rc == IBM_OK && sgs) {
        c->sgs_cfg = sbest;
        c->sgs_tuned = true;
    }
    if (rc == IBM_OK && cache_path) {
        auto m = read_cache(cache_path);
        if (dense) m[key] = {(double)best.vx, (double)best.ty, (double)best.kz, (double)best.wpb, best_ms};
        if (sgs) m[skey] = {(double)sbest.vx, 1.0, (double)sbest.kz, (double)sbest.wpb, sbest_ms};
        write_cache(cache_path, m);
    }
    return rc;
}

}  // namespace ibm

using namespace ibm;

namespace {

int check_batch(const ibm_batch* b, bool need_prepared, const char* fn) {
    if (!b) return fail(IBM_E_ARG, "%s: batch is NULL", fn);
    if (need_prepared && !b->prepared) return fail(IBM_E_STATE, "%s: call ibm_batch_prepare first", fn);
    return IBM_OK;
}

}  // namespace

extern "C" {

int ibm_autotune(ibm_ctx* c, const char* cache_path, int flags, void* stream) {
    if (!c) return fail(IBM_E_ARG, "ibm_autotune: context is NULL");
    if (!c->prepared) return fail(IBM_E_STATE, "ibm_autotune: call ibm_levelset_prepare first");
    DeviceScope ds(c->device);
    return autotune(c, cache_path, flags, (hipStream_t)stream);
}

int ibm_batch_create(ibm_batch** out, int ncases, const ibm_grid* grids, int dtype, int precision) {
    if (!out || !grids || ncases < 1) return fail(IBM_E_ARG, "ibm_batch_create: bad arguments");
    *out = nullptr;
    ibm_batch* b = new (std::nothrow) ibm_batch();
    if (!b) return fail(IBM_E_NOMEM, "ibm_batch_create: out of host memory");
    b->ncases = ncases;
    b->dtype = dtype;
    b->precision = precision;
    b->cases.assign(ncases, nullptr);
    b->io.assign(ncases, ibm_case_io{});
    b->bound.assign(ncases, 0);
    b->z0.assign(ncases, 0.0);
    for (int cs = 0; cs < ncases; ++cs) {
        int rc = ibm_create(&b->cases[cs], &grids[cs], dtype, precision);
        if (rc) {
            ibm_batch_destroy(b);
            return rc;
        }
    }
    b->device = b->cases[0]->device;
    DeviceScope ds(b->device);
    if (hipMalloc(&b->drag, 3 * sizeof(double) * ncases) != hipSuccess ||
        hipMalloc(&b->stats, 4 * sizeof(double) * ncases) != hipSuccess) {
        ibm_batch_destroy(b);
        return fail(IBM_E_NOMEM, "ibm_batch_create: device allocation failed");
    }
    *out = b;
    return IBM_OK;
}

int ibm_batch_destroy(ibm_batch* b) {
    if (!b) return IBM_OK;
    {
        DeviceScope ds(b->device);
        free_tables(b);
        (void)hipFree(b->drag);
        (void)hipFree(b->stats);
    }
    for (ibm_ctx* c : b->cases) ibm_destroy(c);
    delete b;
    return IBM_OK;
}

int ibm_batch_prepare(ibm_batch* b, const void* const* phi_uv, const void* const* phi_w,
                      const ibm_params* p, const double* z0, void* stream) {
    int rc = check_batch(b, false, "ibm_batch_prepare");
    if (rc) return rc;
    if (!phi_uv || !phi_w || !p || !z0) return fail(IBM_E_ARG, "ibm_batch_prepare: NULL argument");
    DeviceScope ds(b->device);
    free_tables(b);
    b->prepared = false;
    for (int cs = 0; cs < b->ncases; ++cs) {
        if ((rc = ibm_levelset_prepare(b->cases[cs], phi_uv[cs], phi_w[cs], p, stream))) return rc;
        const double pc = b->cases[cs]->p.phi_c;
        if (!(z0[cs] > 0.0) || !(z0[cs] < pc))
            return fail(IBM_E_RANGE, "ibm_batch_prepare: case %d: z0 must satisfy 0 < z0 < phi_c", cs);
        b->z0[cs] = z0[cs];
        b->bound[cs] = 0;
    }
    b->prepared = true;
    return IBM_OK;
}

int ibm_batch_bind(ibm_batch* b, int case_id, const ibm_case_io* io) {
    int rc = check_batch(b, true, "ibm_batch_bind");
    if (rc) return rc;
    if (case_id < 0 || case_id >= b->ncases || !io)
        return fail(IBM_E_ARG, "ibm_batch_bind: bad case id or NULL io");
    const size_t ts = b->dtype == IBM_F64 ? 8 : 4;
    const ibm_ctx* c = b->cases[case_id];
    const size_t al = c->cfg.vx > 1 ? 16 : ts;
    auto bad = [&](const void* p, size_t a) { return !p || ((uintptr_t)p % a) != 0; };
    if (bad(io->u, ts) || bad(io->v, ts) || bad(io->w, ts) ||
        (io->log_z0 && bad(io->log_z0, ts)))
        return fail(IBM_E_ARG, "ibm_batch_bind: case %d: velocity or log_z0 NULL or misaligned", case_id);
    for (int i = 0; i < 6; ++i)
        if (bad(io->tau[i], al)) return fail(IBM_E_ARG, "ibm_batch_bind: case %d: tau NULL or not 16-byte aligned", case_id);
    for (int i = 0; i < 3; ++i) {
        if (bad(io->div[i], al) || bad(io->ustar[i], ts))
            return fail(IBM_E_ARG, "ibm_batch_bind: case %d: div or ustar NULL or misaligned", case_id);
        if (io->gradp[i] && bad(io->gradp[i], ts))
            return fail(IBM_E_ARG, "ibm_batch_bind: case %d: gradp misaligned", case_id);
    }
    if (!std::isfinite(io->dt)) return fail(IBM_E_ARG, "ibm_batch_bind: dt must be finite");
    if (((uintptr_t)io->drag_dev % 8) || ((uintptr_t)io->stats_dev % 8))
        return fail(IBM_E_ARG, "ibm_batch_bind: drag_dev or stats_dev misaligned");
    DeviceScope ds(b->device);
    free_tables(b);
    b->io[case_id] = *io;
    b->bound[case_id] = 1;
    return IBM_OK;
}

int ibm_batch_tune(ibm_batch* b, const char* cache_path, void* stream) {
    int rc = check_batch(b, true, "ibm_batch_tune");
    if (rc) return rc;
    DeviceScope ds(b->device);
    free_tables(b);
    std::map<std::string, TileCfg> done;
    for (int cs = 0; cs < b->ncases; ++cs) {
        ibm_ctx* c = b->cases[cs];
        char key[64];
        snprintf(key, sizeof(key), "%dx%dx%d", c->g.nx, c->g.ny, c->g.nz);
        auto it = done.find(key);
        if (it != done.end()) {
            if ((rc = set_cfg(c, it->second))) return rc;
            continue;
        }
        if ((rc = autotune(c, cache_path, IBM_TUNE_BATCH, (hipStream_t)stream))) return rc;
        done[key] = c->cfg;
    }
    return IBM_OK;
}

int ibm_batch_run(ibm_batch* b, void* stream) {
    int rc = check_batch(b, true, "ibm_batch_run");
    if (rc) return rc;
    DeviceScope ds(b->device);
    if ((rc = ensure_tables(b))) return rc;
    return b->dtype == IBM_F64 ? enqueue<double>(b, (hipStream_t)stream)
                               : enqueue<float>(b, (hipStream_t)stream);
}

int ibm_batch_capture(ibm_batch* b, void* stream) {
    int rc = check_batch(b, true, "ibm_batch_capture");
    if (rc) return rc;
    DeviceScope ds(b->device);
    if ((rc = ensure_tables(b))) return rc;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(IBM_E_ARG, "ibm_batch_capture: the null stream cannot be captured; pass a created stream");
    IBM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = b->dtype == IBM_F64 ? enqueue<double>(b, s) : enqueue<float>(b, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    IBM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return IBM_OK;
}

int ibm_batch_launch(ibm_batch* b, void* stream) {
    int rc = check_batch(b, true, "ibm_batch_launch");
    if (rc) return rc;
    if (!b->exec || stale(b))
        return fail(IBM_E_STATE,
                    "ibm_batch_launch: capture the batch (again) after binding, preparing or changing a tile");
    DeviceScope ds(b->device);
    IBM_HIP(hipGraphLaunch(b->exec, (hipStream_t)stream));
    return IBM_OK;
}

int ibm_batch_case(const ibm_batch* b, int case_id, ibm_ctx** out) {
    int rc = check_batch(b, false, "ibm_batch_case");
    if (rc) return rc;
    if (case_id < 0 || case_id >= b->ncases || !out) return fail(IBM_E_ARG, "ibm_batch_case: bad case id");
    *out = b->cases[case_id];
    return IBM_OK;
}

}  // extern "C"
