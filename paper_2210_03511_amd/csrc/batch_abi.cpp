// C ABI of the batched (many-sector) path: host orchestration only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "basis.h"
#include "batch.h"
#include "tune.h"

using namespace symed;

struct ed_batch {
    std::vector<ed_basis *> secs;
    int device = 0, n_cu = 0;
    hipStream_t own = nullptr;
    size_t lds = 0;
    int apply_blocks = 0, vec_blocks = 0;
    int64_t tile_rows = 0, ntiles = 0;
    std::vector<SectorDesc> hdesc;
    SectorDesc *d_desc = nullptr;
    int64_t *d_tile0 = nullptr;
    double *d_partials = nullptr;
    int64_t partial_cap = 0;
    // Lanczos storage
    std::vector<double *> v, w, vprev, alpha, beta;
    LState *d_ls = nullptr;
    int lanczos_cap = 0;
    hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
    std::vector<void *> allocs;
    ed_batch_info_t info{};
    // launch shape: fixed, or chosen per lookup mode (tile rows, blocks per CU)
    bool autotune = true;
    int max_bpc = 1;
    int64_t choice_rows[3] = {0, 0, 0};
    int choice_bpc[3] = {0, 0, 0};
    std::string cache_path;
};

static ed_status balloc(ed_batch *b, void **p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) return fail(ED_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    b->allocs.push_back(*p);
    return ED_OK;
}

// Free an allocation of balloc that a larger one replaced (no-op for NULL).
// The caller has drained the batch's stream.
static void brelease(ed_batch *b, void *p)
{
    if (!p) return;
    for (size_t k = 0; k < b->allocs.size(); ++k)
        if (b->allocs[k] == p) {
            (void)hipFree(p);
            b->allocs.erase(b->allocs.begin() + (long)k);
            return;
        }
}

// tiles of every sector for a tile length; uploads descriptors and tile starts
static ed_status layout_tiles(ed_batch *b, int64_t tile_rows)
{
    b->info.tile_rows = (int32_t)tile_rows;
    const int n = (int)b->secs.size();
    std::vector<int64_t> tile0(n + 1, 0);
    for (int s = 0; s < n; ++s) {
        const int64_t nt = (b->secs[s]->dim + tile_rows - 1) / tile_rows;
        b->hdesc[s].tile0 = tile0[s];
        b->hdesc[s].ntiles = nt;
        tile0[s + 1] = tile0[s] + nt;
    }
    b->tile_rows = tile_rows;
    b->ntiles = tile0[n];
    // partials hold one value per tile, and one per block of the vector kernels
    const int64_t need = std::max<int64_t>(b->ntiles, b->vec_blocks);
    // nothing of the batch may be in flight while its tiling changes
    HIP_OK(hipStreamSynchronize(b->own));
    if (need > b->partial_cap) {
        double *np = nullptr;
        ed_status st = balloc(b, (void **)&np, need * sizeof(double));
        if (st != ED_OK) return st;
        brelease(b, b->d_partials);
        b->d_partials = np;
        b->partial_cap = need;
    }
    HIP_OK(hipMemcpyAsync(b->d_tile0, tile0.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, b->own));
    HIP_OK(hipMemcpyAsync(b->d_desc, b->hdesc.data(), n * sizeof(SectorDesc), hipMemcpyHostToDevice, b->own));
    HIP_OK(hipStreamSynchronize(b->own));
    for (auto &g : b->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    b->info.n_tiles = b->ntiles;
    return ED_OK;
}

// Launch shape: tiles of tile_rows rows on a persistent grid of bpc blocks
// per compute unit (captured steps hold the old shape and are dropped).
static ed_status set_shape(ed_batch *b, int64_t tile_rows, int bpc)
{
    bpc = std::max(1, std::min(bpc, b->max_bpc));
    if (tile_rows != b->tile_rows) {
        ed_status st = layout_tiles(b, tile_rows);
        if (st != ED_OK) return st;
    }
    if (bpc * b->n_cu != b->apply_blocks) {
        HIP_OK(hipStreamSynchronize(b->own));
        b->apply_blocks = bpc * b->n_cu;
        for (auto &g : b->graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    b->info.apply_blocks = b->apply_blocks;
    b->info.blocks_per_cu = bpc;
    return ED_OK;
}

// Fingerprint of a batch for the tuning cache: device, and every sector's
// shape, decompositions and table size.
static uint64_t batch_fingerprint(const ed_batch *b)
{
    uint64_t h = device_fingerprint(b->device);
    for (const ed_basis *s : b->secs) {
        const int64_t v[] = {s->dim, s->n_elements, s->T.G, s->T.N, s->T.R, s->T.A, s->T.is_complex, s->lay.bytes,
                             s->lay.rep_global};
        h = fnv1a(v, sizeof v, h);
    }
    return h;
}

static ed_status batch_apply_impl(ed_batch *b, const void *const *d_x, void *const *d_y, int32_t lookup_mode,
                                  void *stream);

// The launch shape for a lookup mode: fixed, the choice made earlier, the
// cache file's, or the fastest of the candidates timed now in that mode.
static ed_status ensure_shape(ed_batch *b, int mode)
{
    if (!b->autotune) return ED_OK;
    if (b->choice_rows[mode] > 0) return set_shape(b, b->choice_rows[mode], b->choice_bpc[mode]);
    const uint64_t fp = batch_fingerprint(b);
    int64_t rows = 0, bpc = 0;
    ed_status st;
    if (tune_cache_lookup(b->cache_path.c_str(), "batch", fp, mode, rows, bpc) && rows > 0 && bpc >= 1) {
        b->choice_rows[mode] = rows;
        b->choice_bpc[mode] = (int)bpc;
        b->info.tune_mode = mode;
        b->info.cache_hit = 1;
        b->info.n_candidates = 0;
        return set_shape(b, rows, (int)bpc);
    }
    // time one batched H.v in this mode per candidate (after a warm-up)
    const int n = (int)b->secs.size();
    std::vector<const void *> xs(n);
    std::vector<void *> ys(n);
    for (int s = 0; s < n; ++s) {
        xs[s] = b->v[s];
        ys[s] = b->w[s];
    }
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    const int64_t rows_c[] = {2048, 8192, 32768};
    std::vector<int> bpcs = {b->max_bpc};
    if (b->max_bpc > 1) bpcs.push_back(1);
    double best = 1e300;
    int64_t best_rows = rows_c[0];
    int best_bpc = b->max_bpc, k = 0;
    st = ED_OK;
    for (int64_t r : rows_c) {
        for (int c : bpcs) {
            if (st == ED_OK) st = set_shape(b, r, c);
            if (st == ED_OK) st = batch_apply_impl(b, xs.data(), ys.data(), mode, b->own);
            if (st != ED_OK) break;
            float ms = 0;
            if (hipEventRecord(e0, b->own) != hipSuccess) st = fail(ED_EDEVICE, "event");
            if (st == ED_OK) st = batch_apply_impl(b, xs.data(), ys.data(), mode, b->own);
            if (st == ED_OK && (hipEventRecord(e1, b->own) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = fail(ED_EDEVICE, "event timing");
            if (st != ED_OK) break;
            if (k < 8) {
                b->info.tune_rows[k] = (int32_t)r;
                b->info.tune_blocks[k] = c;
                b->info.tune_seconds[k] = ms / 1e3;
                ++k;
            }
            if (ms / 1e3 < best) {
                best = ms / 1e3;
                best_rows = r;
                best_bpc = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ED_OK) return st;
    b->info.n_candidates = k;
    b->info.tune_mode = mode;
    b->info.cache_hit = 0;
    b->choice_rows[mode] = best_rows;
    b->choice_bpc[mode] = best_bpc;
    (void)tune_cache_store(b->cache_path.c_str(), "batch", fp, mode, best_rows, best_bpc, best);
    return set_shape(b, best_rows, best_bpc);
}

// The tables a sector stages into LDS grow when its learned index is trained
// after the batch was made: size the batched launch for the largest, and
// drop the captured steps, which hold the old launch shape.
static ed_status fit_lds(ed_batch *b)
{
    size_t need = 0;
    for (auto *s : b->secs) need = std::max(need, (size_t)s->lay.bytes);
    if (need <= b->lds) return ED_OK;
    if (batch_prepare(need) != hipSuccess) return fail(ED_EDEVICE, "kernel attribute");
    int bpc = 0;
    if (batch_occupancy(need, &bpc) != hipSuccess || bpc < 1)
        return fail(ED_EINVAL, "batched kernel does not fit on a compute unit");
    HIP_OK(hipStreamSynchronize(b->own));
    b->lds = need;
    b->max_bpc = bpc;
    b->apply_blocks = std::min(b->apply_blocks, bpc * b->n_cu);
    b->info.apply_blocks = b->apply_blocks;
    b->info.blocks_per_cu = b->apply_blocks / b->n_cu;
    for (auto &g : b->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    return ED_OK;
}

static ed_status check_mode(const ed_batch *b, int mode)
{
    if (mode < 0 || mode > 2) return fail(ED_EINVAL, "lookup_mode must be 0, 1 or 2");
    if (mode == 2)
        for (auto *s : b->secs)
            if (!s->hashed) return fail(ED_EINVAL, "lookup_mode 2 needs the hashed table in every sector");
    if (mode == 1)
        for (auto *s : b->secs)
            if (!s->indexed) return fail(ED_EINVAL, "lookup_mode 1 needs a trained index in every sector");
    return ED_OK;
}

extern "C" {

void ed_batch_free(ed_batch *b)
{
    if (!b) return;
    for (auto &g : b->graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (void *p : b->allocs) (void)hipFree(p);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

ed_status ed_batch_apply(ed_batch *b, const void *const *d_x, void *const *d_y, int32_t lookup_mode, void *stream);

ed_status ed_batch_create(ed_basis *const *sectors, int32_t n, const ed_batch_cfg *cfg_in, void *stream,
                          ed_batch **out)
{
    if (!sectors || !out || n < 1) return fail(ED_EINVAL, "bad arguments");
    if (n > kMaxSectors) return fail(ED_EINVAL, "at most 256 sectors per batch");
    for (int k = 0; k < n; ++k)
        if (sectors[k] && sectors[k]->T.n_colors) return fail(ED_EINVAL, "batches hold spin-1/2 sectors only");
    // work queued on the caller's stream (e.g. the sectors' builds) comes first
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return fail(ED_EDEVICE, "stream");
    ed_batch_cfg cfg{};
    if (cfg_in) cfg = *cfg_in;
    ed_batch *b = new (std::nothrow) ed_batch();
    if (!b) return fail(ED_ENOMEM, "host allocation failed");
    auto cleanup = [&](ed_status s) {
        std::string m = ed_last_error();
        ed_batch_free(b);
        fail(s, m);
        return s;
    };
    b->secs.assign(sectors, sectors + n);
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess ||
        hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(ED_EDEVICE, "device query failed"));
    b->hdesc.resize(n);
    int64_t total = 0, elements = 0;
    for (int s = 0; s < n; ++s) {
        ed_basis *e = sectors[s];
        if (!e || e->dim < 1) return cleanup(fail(ED_EINVAL, "empty or NULL sector " + std::to_string(s)));
        SectorDesc &D = b->hdesc[s];
        D = SectorDesc{};
        D.p = make_params(e);
        D.pos2slot = e->d_pos2slot;
        D.cplx = e->T.is_complex ? 1 : 0;
        b->lds = std::max(b->lds, (size_t)e->lay.bytes);
        total += e->dim;
        elements += e->n_elements;
    }
    if (batch_prepare(b->lds) != hipSuccess) return cleanup(fail(ED_EDEVICE, "kernel attribute"));
    int bpc = 0;
    if (batch_occupancy(b->lds, &bpc) != hipSuccess || bpc < 1)
        return cleanup(fail(ED_EINVAL, "batched kernel does not fit on a compute unit"));
    b->apply_blocks = bpc * b->n_cu;
    b->vec_blocks = 4 * b->n_cu;
    ed_status st;
    if ((st = balloc(b, (void **)&b->d_desc, n * sizeof(SectorDesc))) != ED_OK) return cleanup(st);
    if ((st = balloc(b, (void **)&b->d_tile0, (n + 1) * sizeof(int64_t))) != ED_OK) return cleanup(st);
    // Lanczos vectors double as autotuning operands
    b->v.resize(n);
    b->w.resize(n);
    b->vprev.assign(n, nullptr);
    for (int s = 0; s < n; ++s) {
        const size_t vb = (size_t)sectors[s]->dim * sizeof(double) * (b->hdesc[s].cplx ? 2 : 1);
        if ((st = balloc(b, (void **)&b->v[s], vb)) != ED_OK) return cleanup(st);
        if ((st = balloc(b, (void **)&b->w[s], vb)) != ED_OK) return cleanup(st);
        if (b->hdesc[s].cplx && (st = balloc(b, (void **)&b->vprev[s], vb)) != ED_OK) return cleanup(st);
        if (launch_fill(b->v[s], (int64_t)(vb / 8), 1.0, b->vec_blocks, b->own) != hipSuccess)
            return cleanup(fail(ED_EDEVICE, "fill"));
        b->hdesc[s].v = b->v[s];
        b->hdesc[s].w = b->w[s];
        b->hdesc[s].vprev = b->vprev[s];
    }
    if ((st = balloc(b, (void **)&b->d_ls, n * sizeof(LState))) != ED_OK) return cleanup(st);
    for (int s = 0; s < n; ++s) b->hdesc[s].ls = b->d_ls + s;
    b->info.n_sectors = n;
    b->info.total_dim = total;
    b->info.total_elements = elements;
    // launch shape: fixed, or chosen per lookup mode at its first use
    b->max_bpc = bpc;
    b->autotune = !(cfg.tile_rows > 0 && !cfg.autotune);
    b->cache_path = cfg.cache_path ? cfg.cache_path : "";
    b->info.tune_mode = -1;
    const int64_t rows0 = cfg.tile_rows > 0 ? cfg.tile_rows : 8192;
    const int bpc0 = cfg.blocks_per_cu > 0 ? cfg.blocks_per_cu : bpc;
    if ((st = set_shape(b, rows0, bpc0)) != ED_OK) return cleanup(st);
    b->tile_rows = rows0;
    *out = b;
    return ED_OK;
}

ed_status ed_batch_info(const ed_batch *b, ed_batch_info_t *info)
{
    if (!b || !info) return fail(ED_EINVAL, "NULL argument");
    *info = b->info;
    return ED_OK;
}

ed_status ed_batch_apply(ed_batch *b, const void *const *d_x, void *const *d_y, int32_t lookup_mode, void *stream)
{
    if (!b || !d_x || !d_y) return fail(ED_EINVAL, "NULL argument");
    ed_status st = check_mode(b, lookup_mode);
    if (st != ED_OK) return st;
    if ((st = fit_lds(b)) != ED_OK) return st;
    // tuning runs on the batch's own stream: work already queued on `stream` goes first
    if (b->autotune && b->choice_rows[lookup_mode] == 0) HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    if ((st = ensure_shape(b, lookup_mode)) != ED_OK) return st;
    return batch_apply_impl(b, d_x, d_y, lookup_mode, stream);
}

}  // extern "C"

static ed_status batch_apply_impl(ed_batch *b, const void *const *d_x, void *const *d_y, int32_t lookup_mode,
                                  void *stream)
{
    ed_status st = ED_OK;
    const int n = (int)b->secs.size();
    bool changed = false;
    for (int s = 0; s < n; ++s) {
        if (!d_x[s] || !d_y[s] || d_x[s] == d_y[s]) return fail(ED_EINVAL, "bad vector pointers");
        if (b->hdesc[s].x != d_x[s] || b->hdesc[s].y != d_y[s]) changed = true;
        b->hdesc[s].x = static_cast<const double *>(d_x[s]);
        b->hdesc[s].y = static_cast<double *>(d_y[s]);
        KParams p = make_params(b->secs[s]);
        if (memcmp(&p, &b->hdesc[s].p, sizeof(KParams)) || b->hdesc[s].pos2slot != b->secs[s]->d_pos2slot)
            changed = true;
        b->hdesc[s].p = p;
        b->hdesc[s].pos2slot = b->secs[s]->d_pos2slot;
    }
    hipStream_t stm = (hipStream_t)stream;
    if (changed) HIP_OK(hipMemcpyAsync(b->d_desc, b->hdesc.data(), n * sizeof(SectorDesc), hipMemcpyHostToDevice, stm));
    HIP_OK(launch_batch_apply(b->d_desc, n, b->d_tile0, b->ntiles, b->tile_rows, 0, lookup_mode, b->d_partials,
                              b->apply_blocks, b->lds, b->vec_blocks, stm));
    if (changed) HIP_OK(hipStreamSynchronize(stm));  // the host descriptor copy must outlive the transfer
    return st;
}

extern "C" {

ed_status ed_batch_lanczos(ed_batch *b, const void *const *d_v0, int32_t n_iter, int32_t lookup_mode,
                           double *h_alpha, double *h_beta, int32_t *n_done, void *stream)
{
    if (!b || !d_v0 || !h_alpha || !h_beta || !n_done || n_iter < 1) return fail(ED_EINVAL, "bad arguments");
    ed_status st = check_mode(b, lookup_mode);
    if (st != ED_OK) return st;
    if ((st = fit_lds(b)) != ED_OK) return st;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    if ((st = ensure_shape(b, lookup_mode)) != ED_OK) return st;
    const int n = (int)b->secs.size();
    if (n_iter > b->lanczos_cap) {
        HIP_OK(hipStreamSynchronize(b->own));
        for (int s = 0; s < (int)b->alpha.size(); ++s) {
            brelease(b, b->alpha[s]);
            brelease(b, b->beta[s]);
        }
        b->alpha.assign(n, nullptr);
        b->beta.assign(n, nullptr);
        const int cap = std::max(n_iter, 256);
        for (int s = 0; s < n; ++s) {
            if ((st = balloc(b, (void **)&b->alpha[s], cap * sizeof(double))) != ED_OK) return st;
            if ((st = balloc(b, (void **)&b->beta[s], cap * sizeof(double))) != ED_OK) return st;
            b->hdesc[s].alpha = b->alpha[s];
            b->hdesc[s].beta = b->beta[s];
        }
        b->lanczos_cap = cap;
        for (auto &g : b->graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    for (int s = 0; s < n; ++s) {
        b->hdesc[s].p = make_params(b->secs[s]);
        b->hdesc[s].pos2slot = b->secs[s]->d_pos2slot;
    }
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    hipStream_t stm = b->own;
    HIP_OK(hipMemcpyAsync(b->d_desc, b->hdesc.data(), n * sizeof(SectorDesc), hipMemcpyHostToDevice, stm));
    // start vectors: v_s = v0_s / |v0_s|, w_s = vprev_s = 0 (per sector, outside the graph)
    for (int s = 0; s < n; ++s) {
        const bool c = b->hdesc[s].cplx;
        const int64_t d = b->secs[s]->dim, n2 = d * (c ? 2 : 1);
        if (!d_v0[s]) return fail(ED_EINVAL, "NULL start vector");
        HIP_OK(launch_norm2_partial(d_v0[s], d, c, b->d_partials, b->vec_blocks, stm));
        HIP_OK(launch_scale_copy(d_v0[s], b->v[s], d, c, b->d_partials, b->vec_blocks, b->vec_blocks, stm));
        HIP_OK(launch_fill(b->w[s], n2, 0.0, b->vec_blocks, stm));
        if (c) HIP_OK(launch_fill(b->vprev[s], n2, 0.0, b->vec_blocks, stm));
        HIP_OK(launch_lstate_init(b->d_ls + s, stm));
    }
    hipGraphExec_t &ge = b->graph[lookup_mode];
    if (!ge) {
        hipGraph_t g = nullptr;
        HIP_OK(hipStreamBeginCapture(stm, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_batch_step(b->d_desc, n, b->d_tile0, b->ntiles, b->tile_rows, lookup_mode,
                                         b->d_partials, b->apply_blocks, b->vec_blocks, b->lds, stm);
        hipError_t e2 = hipStreamEndCapture(stm, &g);
        if (e != hipSuccess || e2 != hipSuccess) return fail(ED_EDEVICE, "graph capture of the batched step failed");
        HIP_OK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
    }
    for (int k = 0; k < n_iter; ++k) HIP_OK(hipGraphLaunch(ge, stm));
    std::vector<LState> ls(n);
    for (int s = 0; s < n; ++s) {
        HIP_OK(hipMemcpyAsync(h_alpha + (size_t)s * n_iter, b->alpha[s], n_iter * sizeof(double),
                              hipMemcpyDeviceToHost, stm));
        HIP_OK(hipMemcpyAsync(h_beta + (size_t)s * n_iter, b->beta[s], n_iter * sizeof(double),
                              hipMemcpyDeviceToHost, stm));
    }
    HIP_OK(hipMemcpyAsync(ls.data(), b->d_ls, n * sizeof(LState), hipMemcpyDeviceToHost, stm));
    HIP_OK(hipStreamSynchronize(stm));
    bool broken = false;
    for (int s = 0; s < n; ++s) {
        n_done[s] = ls[s].broken_step >= 0 ? ls[s].broken_step + 1 : n_iter;
        broken |= ls[s].broken_step >= 0;
    }
    if (broken) {
        set_error("Lanczos breakdown in at least one sector");
        return ED_EBREAKDOWN;
    }
    return ED_OK;
}

}  // extern "C"
