// C ABI of the symed library.  Host orchestration only: every step of the
// hot path runs in the HIP kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "basis.h"
#include "launch.h"
#include "learned.h"
#include "learned_dev.h"

using namespace symed;

namespace symed {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

ed_status fail(ed_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

}  // namespace symed


ed_status dev_alloc(ed_basis *b, void **ptr, size_t bytes)
{
    if (b->mem_limit > 0 && b->bytes + (int64_t)bytes > b->mem_limit)
        return fail(ED_ENOMEM, "device memory cap exceeded (" + std::to_string(b->bytes + bytes) + " > " +
                                   std::to_string(b->mem_limit) + " bytes)");
    hipError_t e = hipMalloc(ptr, bytes ? bytes : 16);
    if (e != hipSuccess) return fail(ED_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    b->bytes += (int64_t)bytes;
    b->allocs.emplace_back(*ptr, (int64_t)bytes);
    return ED_OK;
}

void dev_release(ed_basis *b, void *ptr)
{
    if (!ptr) return;
    for (size_t k = 0; k < b->allocs.size(); ++k)
        if (b->allocs[k].first == ptr) {
            (void)hipFree(ptr);
            b->bytes -= b->allocs[k].second;
            b->allocs.erase(b->allocs.begin() + (long)k);
            return;
        }
}

ed_status TmpPool::take(void **q, size_t bytes)
{
    if (basis && basis->mem_limit > 0 && basis->bytes + (int64_t)bytes > basis->mem_limit)
        return fail(ED_ENOMEM, "device memory cap exceeded by temporaries (" + std::to_string(basis->bytes + bytes) +
                                   " > " + std::to_string(basis->mem_limit) + " bytes)");
    hipError_t e = hipMalloc(q, bytes ? bytes : 16);
    if (e != hipSuccess) return fail(ED_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    ptrs.push_back(*q);
    if (basis) {
        basis->bytes += (int64_t)bytes;
        held += (int64_t)bytes;
    }
    return ED_OK;
}

#define TAKE(pool, ptr, bytes)                                          \
    do {                                                                \
        ed_status _ts = (pool).take((void **)(ptr), (size_t)(bytes));   \
        if (_ts != ED_OK) return _ts;                                   \
    } while (0)

// Persistent grids of the apply kernel: as many blocks per compute unit as
// fit, except for a plain lookup over long Limits windows (more than 64 keys
// on average) in arrays larger than the 256 MiB last-level cache: its binary
// searches touch so many lines that a second block per compute unit only
// thrashes the caches (measured at 40 sites: 2.31 s with one block, 2.78 s
// with two; at 32 sites, where everything is cached, two blocks are faster).
static void set_grids(ed_basis *b, int blocks_per_cu)
{
    b->cfg.apply_blocks = blocks_per_cu * b->n_cu;
    b->cfg.lookup_blocks[1] = b->cfg.lookup_blocks[2] = b->cfg.apply_blocks;
    const double searched = (double)b->dim * sizeof(uint64_t) + (double)((1ull << b->pbits) + 1) * sizeof(uint32_t);
    const bool thrash = b->limits_mean_window > 64.0 && searched > 256.0 * (1 << 20);
    b->cfg.lookup_blocks[0] = (thrash ? 1 : blocks_per_cu) * b->n_cu;
}

KParams make_params(const ed_basis *b)
{
    KParams p{};
    const HostTables &T = b->T;
    p.N = T.N;
    p.R = T.R;
    p.br = T.br;
    p.A = T.A;
    p.ba = T.ba;
    p.n_pairs = (int)T.pairs.size();
    p.G = T.G;
    p.is_complex = T.is_complex ? 1 : 0;
    p.pbits = b->pbits;
    p.n_up = T.n_up;
    p.n_colors = T.n_colors;
    p.n_moves = (int)T.moves.size();
    p.maskN = (T.N == 64) ? ~0ull : ((1ull << T.N) - 1);
    p.lay = b->lay;
    p.blob = b->d_blob;
    p.reps = b->d_reps;
    p.stab = b->d_stab;
    p.limits = b->d_limits;
    p.dim = b->dim;
    p.lv.segs = static_cast<const Seg *>(b->d_segs);
    p.lv.cells = static_cast<const uint2 *>(b->d_cells);
    p.lv.n_cells = b->n_cells;
    p.lv.lg = b->lg_segs;
    p.lv.rk_W = T.N - T.n_up + 1;
    p.lv.eq_K = b->eq_K;
    p.lv.eq_invK = 1.0 / (double)b->eq_K;
    p.has_index = b->indexed ? 1 : 0;
    p.htab = b->d_htab;
    p.hslots = b->hslots;
    p.lrec = b->d_lrec;
    p.gtab = b->d_gtab;
    return p;
}

hipError_t stage_input(const ed_basis *b, int lookup_mode, const void *d_x, hipStream_t st)
{
    if (lookup_mode == 2)
        return launch_hash_values(b->d_htab, b->d_pos2slot, d_x, b->dim, b->T.is_complex, b->cfg.vec_blocks, st);
    if (lookup_mode == 1 && b->d_lrec)
        return launch_hash_values(b->d_lrec, nullptr, d_x, b->dim, b->T.is_complex, b->cfg.vec_blocks, st);
    return hipSuccess;
}

static uint64_t binom64(int n, int k)
{
    if (k < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    unsigned __int128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (unsigned)(n - k + i) / (unsigned)i;
    return (uint64_t)r;
}

extern "C" {

const char *ed_last_error(void) { return g_err.c_str(); }

const char *ed_version(void) { return "symed 0.1 (gfx950)"; }

void ed_basis_free(ed_basis *b)
{
    if (!b) return;
    for (auto &g : b->step_graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto &a : b->allocs) (void)hipFree(a.first);
    if (b->own) (void)hipStreamDestroy(b->own);
    delete b;
}

// Number of configurations with the given color counts, n! / prod counts!;
// 0 if it exceeds 2^58 (the enumeration's rank arithmetic multiplies it by n).
static uint64_t multinomial64(int n_colors, const int32_t *counts)
{
    unsigned __int128 r = 1;
    int k = 0;
    for (int c = 0; c < n_colors; ++c)
        for (int q = 1; q <= counts[c]; ++q) {
            ++k;
            r = r * (unsigned)k / (unsigned)q;   // exact: r is an integer multiple of C(k, q) here
            if (r >> 58) return 0;
        }
    return (uint64_t)r;
}

// n_colors == 0: spin-1/2 model in the sector of n_up up spins; otherwise an
// SU(n_colors) permutation model in the sector of the given color counts.
static ed_status build_impl(const ed_model *model, const ed_group *group, int32_t n_up, int n_colors,
                            const int32_t *color_counts, const ed_options *opts, hipStream_t st, ed_basis *b)
{
    auto t0 = std::chrono::steady_clock::now();
    ed_options o{};
    if (opts) o = *opts;
    ed_status s = n_colors ? build_color_tables(model, group, n_colors, color_counts, o.n_sub_rep, o.n_sub_act, b->T)
                           : build_host_tables(model, group, n_up, o.n_sub_rep, o.n_sub_act, b->T);
    if (s != ED_OK) return s;
    HostTables &T = b->T;
    b->mem_limit = o.mem_limit_bytes;
    std::vector<uint8_t> gblob;
    std::vector<uint8_t> blob = pack_blob(T, b->lay, &gblob);

    HIP_OK(hipGetDevice(&b->device));
    int lds_max = 0;
    HIP_OK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device));
    HIP_OK(hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, b->device));
    if ((int64_t)b->lay.bytes + 256 > lds_max)
        return fail(ED_EINVAL, "lookup tables (" + std::to_string(b->lay.bytes) + " B) exceed the LDS of one block (" +
                                   std::to_string(lds_max) + " B); choose other sublattice decompositions");
    HIP_OK(hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking));

    if ((s = dev_alloc(b, &b->d_blob, blob.size())) != ED_OK) return s;
    HIP_OK(hipMemcpy(b->d_blob, blob.data(), blob.size(), hipMemcpyHostToDevice));
    if (b->lay.rep_global) {
        // Rep/Sym tables too large for LDS: read through the caches
        if ((s = dev_alloc(b, &b->d_gtab, gblob.size())) != ED_OK) return s;
        HIP_OK(hipMemcpy(b->d_gtab, gblob.data(), gblob.size(), hipMemcpyHostToDevice));
    }

    KParams p = make_params(b);
    int bpc = 0, athreads = 0;
    HIP_OK(prepare_kernels(p, &bpc, &athreads));
    if (bpc < 1) return fail(ED_EINVAL, "apply kernel does not fit on a compute unit");
    b->cfg.apply_threads = athreads;
    set_grids(b, bpc);
    b->cfg.vec_blocks = 4 * b->n_cu;

    TmpPool tmp(b);  // temporaries of the build, charged to the memory cap while held
    // --- enumeration of the sector (two passes + scan) -------------------
    const int N = T.N;
    const uint64_t total = n_colors ? multinomial64(n_colors, color_counts) : binom64(N, n_up);
    if (n_colors && total == 0) return fail(ED_EINVAL, "color sector with more than 2^58 configurations");
    std::vector<uint64_t> hb(64 * 64, 0);
    for (int n = 0; n < 64; ++n)
        for (int k = 0; k < 64; ++k) hb[n * 64 + k] = binom64(n, k);
    uint64_t *d_binom = nullptr;
    TAKE(tmp, &d_binom, hb.size() * sizeof(uint64_t));
    HIP_OK(hipMemcpy(d_binom, hb.data(), hb.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    uint64_t len = std::max<uint64_t>(256, (total + (1ull << 24) - 1) >> 24);
    uint64_t n_chunks = (total + len - 1) / len;
    if (n_chunks == 0) n_chunks = 1;
    uint32_t *d_counts = nullptr;
    uint64_t *d_offsets = nullptr, *d_total = nullptr;
    uint64_t *d_scan = nullptr;
    TAKE(tmp, &d_counts, n_chunks * sizeof(uint32_t));
    TAKE(tmp, &d_offsets, n_chunks * sizeof(uint64_t));
    TAKE(tmp, &d_total, sizeof(uint64_t));
    TAKE(tmp, &d_scan, scan_tmp_words(n_chunks) * sizeof(uint64_t));
    int eblocks = (int)std::min<uint64_t>((n_chunks + 255) / 256, (uint64_t)b->n_cu * 16);
    if (eblocks < 1) eblocks = 1;
    if (n_colors)
        HIP_OK(launch_enumerate_colors(p, color_counts, n_colors, T.n_sites, total, len, n_chunks, d_counts, nullptr,
                                       nullptr, nullptr, false, eblocks, st));
    else
        HIP_OK(launch_enumerate(p, d_binom, total, len, n_chunks, d_counts, nullptr, nullptr, nullptr, false, eblocks,
                                st));
    HIP_OK(launch_scan(d_counts, d_offsets, n_chunks, d_total, d_scan, st));
    uint64_t dim = 0;
    HIP_OK(hipMemcpyAsync(&dim, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (dim >= (1ull << 32) - 1) return fail(ED_EINVAL, "sector dimension >= 2^32 is not supported");
    b->dim = (int64_t)dim;
    if ((s = dev_alloc(b, (void **)&b->d_reps, dim * sizeof(uint64_t))) != ED_OK) return s;
    if ((s = dev_alloc(b, (void **)&b->d_stab, dim * sizeof(uint16_t))) != ED_OK) return s;
    p = make_params(b);
    if (n_colors)
        HIP_OK(launch_enumerate_colors(p, color_counts, n_colors, T.n_sites, total, len, n_chunks, d_counts, d_offsets,
                                       b->d_reps, b->d_stab, true, eblocks, st));
    else
        HIP_OK(launch_enumerate(p, d_binom, total, len, n_chunks, d_counts, d_offsets, b->d_reps, b->d_stab, true,
                                eblocks, st));
    HIP_OK(hipStreamSynchronize(st));

    // --- Limits prefix table --------------------------------------------
    int pb = o.prefix_bits;
    if (pb <= 0) {
        int lg = 0;
        while (lg < 62 && (1ull << lg) < (uint64_t)std::max<int64_t>(dim, 1)) ++lg;
        pb = std::min(std::min(N, 28), std::max(4, lg + 1));
    }
    if (pb > N) pb = N;
    if (pb > 30) return fail(ED_EINVAL, "prefix_bits must be <= 30");
    b->pbits = pb;
    if ((s = dev_alloc(b, (void **)&b->d_limits, ((1ull << pb) + 1) * sizeof(uint32_t))) != ED_OK) return s;
    HIP_OK(launch_limits(b->d_reps, b->dim, N, pb, b->d_limits, st));

    // --- key-weighted Limits bucket statistics (search window of the plain lookup)
    {
        unsigned long long *d_ls = nullptr, hls[2] = {0, 0};
        TAKE(tmp, &d_ls, 2 * sizeof(unsigned long long));
        HIP_OK(hipMemsetAsync(d_ls, 0, 2 * sizeof(unsigned long long), st));
        HIP_OK(launch_limits_stats(b->d_limits, pb, d_ls, st));
        HIP_OK(hipMemcpyAsync(hls, d_ls, sizeof(hls), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        b->limits_mean_window = b->dim ? (double)hls[0] / (double)b->dim : 0.0;
        b->limits_max_window = (int64_t)hls[1];
        set_grids(b, b->cfg.apply_blocks / b->n_cu);
    }

    // --- element count ----------------------------------------------------
    p = make_params(b);
    unsigned long long *d_cnt = nullptr, cnt = 0;
    TAKE(tmp, &d_cnt, sizeof(unsigned long long));
    HIP_OK(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long), st));
    if (b->dim > 0) HIP_OK(launch_count_elements(p, d_cnt, 4 * b->n_cu, st));
    HIP_OK(hipMemcpyAsync(&cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    b->n_elements = (int64_t)cnt;
    b->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return ED_OK;
}

static ed_status build_any(const ed_model *model, const ed_group *group, int32_t n_up, int n_colors,
                           const int32_t *color_counts, const ed_options *opts, void *stream, ed_basis **out)
{
    if (!out) return fail(ED_EINVAL, "out must not be NULL");
    ed_basis *b = new (std::nothrow) ed_basis();
    if (!b) return fail(ED_ENOMEM, "host allocation failed");
    ed_status s = build_impl(model, group, n_up, n_colors, color_counts, opts, (hipStream_t)stream, b);
    if (s != ED_OK) {
        std::string msg = g_err;
        (void)hipDeviceSynchronize();  // nothing of the failed build may still run when it is freed
        ed_basis_free(b);
        g_err = msg;
        return s;
    }
    *out = b;
    return ED_OK;
}

ed_status ed_basis_build(const ed_model *model, const ed_group *group, int32_t n_up, const ed_options *opts,
                         void *stream, ed_basis **out)
{
    return build_any(model, group, n_up, 0, nullptr, opts, stream, out);
}

ed_status ed_basis_build_colors(const ed_model *model, const ed_group *group, int32_t n_colors, const int32_t *counts,
                                const ed_options *opts, void *stream, ed_basis **out)
{
    if (n_colors < 2 || n_colors > 4) return fail(ED_EINVAL, "n_colors must be in [2, 4]");
    return build_any(model, group, 0, n_colors, counts, opts, stream, out);
}

ed_status ed_basis_info(const ed_basis *b, ed_basis_info_t *info)
{
    if (!b || !info) return fail(ED_EINVAL, "NULL argument");
    ed_basis_info_t r{};
    r.dim = b->dim;
    r.is_complex = b->T.is_complex ? 1 : 0;
    r.n_sites = b->T.n_colors ? b->T.n_sites : b->T.N;
    r.n_colors = b->T.n_colors;
    r.n_elem = b->T.G;
    r.n_sub_rep = b->T.R;
    r.n_sub_act = b->T.A;
    r.prefix_bits = b->pbits;
    r.n_elements = b->n_elements;
    r.n_offdiag = b->n_elements - b->dim;
    r.bytes_device = b->bytes;
    r.table_bytes = b->lay.bytes;
    r.limits_bytes = (int64_t)(((1ull << b->pbits) + 1) * sizeof(uint32_t));
    r.index_bytes = b->indexed ? b->istats.mlp_bytes + b->istats.table_bytes : 0;
    r.index_max_err = b->indexed ? b->istats.max_err : -1;
    r.lds_resident = 1;
    r.limits_mean_window = b->limits_mean_window;
    r.limits_max_window = b->limits_max_window;
    r.apply_blocks = b->cfg.apply_blocks;
    r.apply_threads = b->cfg.apply_threads;
    r.build_seconds = b->build_seconds;
    *info = r;
    return ED_OK;
}

ed_status ed_basis_export(const ed_basis *b, uint64_t *h_reps, uint32_t *h_stab)
{
    if (!b) return fail(ED_EINVAL, "NULL basis");
    if (b->dim == 0) return ED_OK;
    if (h_reps) HIP_OK(hipMemcpy(h_reps, b->d_reps, b->dim * sizeof(uint64_t), hipMemcpyDeviceToHost));
    if (h_stab) {
        std::vector<uint16_t> tmp(b->dim);
        HIP_OK(hipMemcpy(tmp.data(), b->d_stab, b->dim * sizeof(uint16_t), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < b->dim; ++i) h_stab[i] = tmp[i];
    }
    return ED_OK;
}

ed_status ed_basis_device_reps(const ed_basis *b, const uint64_t **d_reps)
{
    if (!b || !d_reps) return fail(ED_EINVAL, "NULL argument");
    *d_reps = b->d_reps;
    return ED_OK;
}

static ed_status check_lookup(const ed_basis *b, int mode)
{
    if (mode == 0 || (mode == 1 && b->indexed) || (mode == 2 && b->hashed)) return ED_OK;
    return fail(ED_EINVAL, "lookup_mode must be 0 (plain), 1 (learned, after ed_index_train) or 2 (hashed, after "
                           "ed_hash_build)");
}

ed_status ed_apply_H(const ed_basis *b, const void *d_x, void *d_y, int32_t lookup_mode, void *stream)
{
    if (!b) return fail(ED_EINVAL, "NULL basis");
    ed_status cs = check_lookup(b, lookup_mode);
    if (cs != ED_OK) return cs;
    if (b->dim == 0) return ED_OK;
    if (!d_x || !d_y) return fail(ED_EINVAL, "NULL vector");
    if (d_x == d_y) return fail(ED_EINVAL, "x and y must not alias");
    HIP_OK(stage_input(b, lookup_mode, d_x, (hipStream_t)stream));
    KParams p = make_params(b);
    HIP_OK(launch_apply(p, b->cfg, d_x, d_y, 0, lookup_mode, nullptr, nullptr, (hipStream_t)stream));
    return ED_OK;
}

ed_status ed_lookup(const ed_basis *b, const uint64_t *d_keys, int64_t n, int64_t *d_idx, int32_t mode, void *stream)
{
    if (!b) return fail(ED_EINVAL, "NULL basis");
    ed_status cs = check_lookup(b, mode);
    if (cs != ED_OK) return cs;
    if (n < 0) return fail(ED_EINVAL, "negative count");
    if (n == 0) return ED_OK;
    if (!d_keys || !d_idx) return fail(ED_EINVAL, "NULL array");
    if (b->dim == 0) {
        std::vector<int64_t> m1(n, -1);
        HIP_OK(hipMemcpyAsync(d_idx, m1.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, (hipStream_t)stream));
        HIP_OK(hipStreamSynchronize((hipStream_t)stream));
        return ED_OK;
    }
    KParams p = make_params(b);
    HIP_OK(launch_lookup(p, d_keys, n, d_idx, mode, (hipStream_t)stream));
    return ED_OK;
}

// Vectors, scalars and alpha/beta arrays for n_iter steps; when the arrays
// grow, their first `keep` entries (steps already done) are carried over.
static ed_status lanczos_workspace(ed_basis *b, int n_iter, int keep)
{
    const bool cplx = b->T.is_complex;
    const size_t vbytes = (size_t)b->dim * sizeof(double) * (cplx ? 2 : 1);
    ed_status s;
    if (!b->d_v) {
        if ((s = dev_alloc(b, (void **)&b->d_v, vbytes)) != ED_OK) return s;
        if ((s = dev_alloc(b, (void **)&b->d_w, vbytes)) != ED_OK) return s;
        if (cplx && (s = dev_alloc(b, (void **)&b->d_vprev, vbytes)) != ED_OK) return s;
        // one partial per 64 rows of the apply kernel, one per block of the vector kernels
        const int64_t np = std::max<int64_t>((b->dim + 63) / 64, b->cfg.vec_blocks);
        if ((s = dev_alloc(b, (void **)&b->d_partials, np * sizeof(double))) != ED_OK) return s;
        if ((s = dev_alloc(b, (void **)&b->d_ls, sizeof(LState))) != ED_OK) return s;
    }
    if (n_iter > b->lanczos_cap) {
        // graphs reference the alpha/beta arrays: rebuild them
        for (auto &g : b->step_graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
        int cap = std::max(n_iter, std::max(256, 2 * b->lanczos_cap));
        double *na = nullptr, *nb = nullptr;
        if ((s = dev_alloc(b, (void **)&na, cap * sizeof(double))) != ED_OK) return s;
        if ((s = dev_alloc(b, (void **)&nb, cap * sizeof(double))) != ED_OK) return s;
        if (keep > 0 && b->d_alpha) {
            HIP_OK(hipMemcpy(na, b->d_alpha, keep * sizeof(double), hipMemcpyDeviceToDevice));
            HIP_OK(hipMemcpy(nb, b->d_beta, keep * sizeof(double), hipMemcpyDeviceToDevice));
        }
        // nothing queued may still read the old arrays (hipMemcpy above and
        // the graph launches before it ran on other streams)
        HIP_OK(hipStreamSynchronize(b->own));
        dev_release(b, b->d_alpha);
        dev_release(b, b->d_beta);
        b->d_alpha = na;
        b->d_beta = nb;
        b->lanczos_cap = cap;
    }
    return ED_OK;
}

// One Lanczos step as a kernel sequence on stream `st` (captured once).
static hipError_t enqueue_step(ed_basis *b, int mode, hipStream_t st)
{
    const bool cplx = b->T.is_complex;
    KParams p = make_params(b);
    hipError_t e;
    if ((e = stage_input(b, mode, b->d_v, st)) != hipSuccess) return e;
    if ((e = launch_apply(p, b->cfg, b->d_v, b->d_w, cplx ? 2 : 1, mode, b->d_ls, b->d_partials, st)) != hipSuccess)
        return e;
    if ((e = launch_finalize(b->d_partials, (b->dim + 63) / 64, b->d_alpha, b->d_beta, b->d_ls, 0, st)) != hipSuccess)
        return e;
    if ((e = launch_axpy_norm(b->d_w, b->d_v, b->d_vprev, b->dim, cplx, b->d_alpha, b->d_ls, b->d_partials,
                              b->cfg.vec_blocks, st)) != hipSuccess)
        return e;
    if ((e = launch_finalize(b->d_partials, b->cfg.vec_blocks, b->d_alpha, b->d_beta, b->d_ls, 1, st)) != hipSuccess)
        return e;
    if ((e = launch_rotate(b->d_v, b->d_w, b->d_vprev, b->dim, cplx, b->d_beta, b->d_ls, b->cfg.vec_blocks, st)) !=
        hipSuccess)
        return e;
    return launch_step_inc(b->d_ls, b->d_beta, st);
}

}  // extern "C"

// Workspace for n_iter steps and the captured step graph of a lookup mode.
ed_status lanczos_prepare(ed_basis *b, int n_iter, int lookup_mode, int keep)
{
    if (n_iter < 1) return fail(ED_EINVAL, "n_iter must be >= 1");
    ed_status cs = check_lookup(b, lookup_mode);
    if (cs != ED_OK) return cs;
    if (b->dim == 0) return fail(ED_EINVAL, "empty sector");
    ed_status s = lanczos_workspace(b, n_iter, keep);
    if (s != ED_OK) return s;
    hipGraphExec_t &ge = b->step_graph[lookup_mode];
    if (!ge) {
        hipStream_t st = b->own;
        hipGraph_t g = nullptr;
        HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_step(b, lookup_mode, st);
        hipError_t e2 = hipStreamEndCapture(st, &g);
        if (e != hipSuccess) return fail(ED_EDEVICE, std::string("capture: ") + hipGetErrorString(e));
        if (e2 != hipSuccess) return fail(ED_EDEVICE, std::string("end capture: ") + hipGetErrorString(e2));
        HIP_OK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
    }
    return ED_OK;
}

// Start of a run on the basis's own stream (after `stream` has drained):
// v = v0 / |v0|, w = vprev = 0, scalars reset.
ed_status lanczos_start(ed_basis *b, const void *d_v0, void *stream)
{
    const bool cplx = b->T.is_complex;
    const int64_t n2 = b->dim * (cplx ? 2 : 1);
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    hipStream_t st = b->own;
    HIP_OK(launch_norm2_partial(d_v0, b->dim, cplx, b->d_partials, b->cfg.vec_blocks, st));
    HIP_OK(launch_scale_copy(d_v0, b->d_v, b->dim, cplx, b->d_partials, b->cfg.vec_blocks, b->cfg.vec_blocks, st));
    HIP_OK(launch_fill(b->d_w, n2, 0.0, b->cfg.vec_blocks, st));
    if (cplx) HIP_OK(launch_fill(b->d_vprev, n2, 0.0, b->cfg.vec_blocks, st));
    HIP_OK(launch_lstate_init(b->d_ls, st));
    return ED_OK;
}

// Steps done + 1 .. done + n of the run on the basis's stream; alpha/beta of
// these steps to the host.  Records how far the run got.
ed_status lanczos_advance(ed_basis *b, int done, int n, int lookup_mode, double *h_alpha, double *h_beta,
                          int32_t *n_done)
{
    hipStream_t st = b->own;
    for (int k = 0; k < n; ++k) HIP_OK(hipGraphLaunch(b->step_graph[lookup_mode], st));
    LState ls{};
    HIP_OK(hipMemcpyAsync(h_alpha, b->d_alpha + done, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(h_beta, b->d_beta + done, n * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&ls, b->d_ls, sizeof(LState), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    b->lanczos_steps = done + n;
    if (ls.broken_step >= 0) {
        b->lanczos_broken = true;
        *n_done = ls.broken_step + 1 - done;
        set_error("Lanczos breakdown at step " + std::to_string(ls.broken_step));
        return ED_EBREAKDOWN;
    }
    b->lanczos_broken = false;
    *n_done = n;
    return ED_OK;
}

extern "C" {

ed_status ed_lanczos_run(const ed_basis *cb, const void *d_v0, int32_t n_iter, int32_t lookup_mode, double *h_alpha,
                         double *h_beta, int32_t *n_done, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(cb);
    if (!b || !d_v0 || !h_alpha || !h_beta || !n_done) return fail(ED_EINVAL, "NULL argument");
    b->lanczos_steps = -1;
    ed_status s = lanczos_prepare(b, n_iter, lookup_mode, 0);
    if (s != ED_OK) return s;
    if ((s = lanczos_start(b, d_v0, stream)) != ED_OK) return s;
    return lanczos_advance(b, 0, n_iter, lookup_mode, h_alpha, h_beta, n_done);
}

ed_status ed_lanczos_resume(const ed_basis *cb, int32_t n_more, int32_t lookup_mode, double *h_alpha,
                            double *h_beta, int32_t *n_done, void *stream)
{
    ed_basis *b = const_cast<ed_basis *>(cb);
    if (!b || !h_alpha || !h_beta || !n_done) return fail(ED_EINVAL, "NULL argument");
    if (n_more < 1) return fail(ED_EINVAL, "n_more must be >= 1");
    if (b->lanczos_steps < 0) return fail(ED_EINVAL, "no Lanczos run to resume on this basis");
    const int done = b->lanczos_steps;
    if (b->lanczos_broken) {
        *n_done = 0;
        set_error("the run being resumed broke down");
        return ED_EBREAKDOWN;
    }
    if ((int64_t)done + n_more > (1 << 30)) return fail(ED_EINVAL, "too many steps");
    ed_status s = lanczos_prepare(b, done + n_more, lookup_mode, done);
    if (s != ED_OK) return s;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    return lanczos_advance(b, done, n_more, lookup_mode, h_alpha, h_beta, n_done);
}

ed_status ed_hash_build(ed_basis *b, const ed_hash_cfg *cfg_in, ed_hash_stats *out, void *stream)
{
    if (!b) return fail(ED_EINVAL, "NULL basis");
    ed_hash_cfg cfg{};
    if (cfg_in) cfg = *cfg_in;
    // Default: 15 % of the slots occupied for 16-byte records (about 1.09
    // probes per lookup; at 40 sites 3.5 % faster than a quarter, for 18 GB
    // more), a quarter for the 32-byte complex records (at 36 sites a load of
    // 0.15 is 5 % slower), or the smallest load whose slot count still fits
    // in 32 bits.
    const double base = b->T.is_complex ? 0.25 : 0.15;
    const double load = cfg.load != 0.0 ? cfg.load
                                         : std::max(base, std::ceil((double)b->dim / 4.0e9 * 100.0) / 100.0);
    if (!(load >= 0.05 && load <= 0.95)) return fail(ED_EINVAL, "load must lie in [0.05, 0.95]");
    if (b->T.N >= 64) return fail(ED_EINVAL, "the hashed table needs N < 64 (all-ones marks an empty slot)");
    if (b->dim == 0) return fail(ED_EINVAL, "empty sector");
    uint64_t slots = (uint64_t)std::ceil((double)b->dim / load);
    if (slots <= (uint64_t)b->dim) slots = (uint64_t)b->dim + 1;
    if (slots >= (1ull << 32)) return fail(ED_EINVAL, "too many slots for 32-bit slot numbers");
    if (b->hashed) {
        if (slots != b->hslots) return fail(ED_EINVAL, "hashed table already built with another load");
        if (out) *out = b->hstats;
        return ED_OK;
    }
    const auto t0 = std::chrono::steady_clock::now();
    const size_t words = b->T.is_complex ? 4 : 2;
    ed_status s;
    if ((s = dev_alloc(b, (void **)&b->d_htab, slots * words * sizeof(uint64_t))) != ED_OK) return s;
    if ((s = dev_alloc(b, (void **)&b->d_pos2slot, (size_t)b->dim * sizeof(uint32_t))) != ED_OK) return s;
    unsigned long long *d_stats = nullptr;
    if ((s = dev_alloc(b, (void **)&d_stats, 2 * sizeof(unsigned long long))) != ED_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(hipMemsetAsync(d_stats, 0, 2 * sizeof(unsigned long long), st));
    HIP_OK(launch_hash_build(b->d_htab, slots, b->d_reps, b->dim, b->T.is_complex, b->d_pos2slot, d_stats,
                             4 * b->n_cu, st));
    unsigned long long h[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(h, d_stats, sizeof(h), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    b->hslots = slots;
    b->hashed = true;
    ed_hash_stats &r = b->hstats;
    r.slots = (int64_t)slots;
    r.bytes = (int64_t)(slots * words * sizeof(uint64_t) + (size_t)b->dim * sizeof(uint32_t));
    r.load = (double)b->dim / (double)slots;
    r.mean_probes = (double)h[0] / (double)b->dim;
    r.max_probes = (int64_t)h[1];
    r.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (out) *out = r;
    return ED_OK;
}

// Sturm-sequence bisection for the lowest k eigenvalues of a symmetric
// tridiagonal matrix.
static int sturm_count(const double *a, const double *b, int n, double x)
{
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < n; ++i) {
        if (q == 0.0) q = 1e-300;
        q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
        if (q < 0) ++c;
    }
    return c;
}

ed_status ed_eigenvalues(const double *alpha, const double *beta, int32_t n, int32_t k, double *evals)
{
    if (!alpha || !evals || n < 1 || k < 1 || k > n || (n > 1 && !beta))
        return fail(ED_EINVAL, "bad arguments to ed_eigenvalues");
    double lo = alpha[0], hi = alpha[0];
    for (int i = 0; i < n; ++i) {
        double r = (i > 0 ? std::fabs(beta[i - 1]) : 0.0) + (i < n - 1 ? std::fabs(beta[i]) : 0.0);
        lo = std::min(lo, alpha[i] - r);
        hi = std::max(hi, alpha[i] + r);
    }
    const double span = std::max(hi - lo, 1e-300);
    lo -= 1e-12 * span + 1e-300;
    hi += 1e-12 * span + 1e-300;
    for (int m = 0; m < k; ++m) {
        // smallest x with count(x) > m
        double l = lo, h = hi;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (l + h);
            if (mid == l || mid == h) break;
            if (sturm_count(alpha, beta, n, mid) > m) h = mid; else l = mid;
        }
        evals[m] = 0.5 * (l + h);
    }
    return ED_OK;
}

ed_status ed_index_train(ed_basis *b, const ed_index_cfg *cfg_in, ed_index_stats *out, void *stream)
{
    if (!b) return fail(ED_EINVAL, "NULL basis");
    if (b->dim < 1) return fail(ED_EINVAL, "empty sector");
    if (b->T.n_colors) return fail(ED_EINVAL, "the learned index ranks spin-1/2 configurations; not for SU(d) bases");
    ed_index_cfg cfg{};
    if (cfg_in) cfg = *cfg_in;
    const int N = b->T.N, n_up = b->T.n_up;
    // one input feature (the rank read as a fraction of the largest rank)
    const int F = 1;
    if (cfg.n_features != 0 && cfg.n_features != 1) return fail(ED_EINVAL, "the index network has one input feature");
    if (cfg.hidden != 0 && cfg.hidden != kHidden) return fail(ED_EINVAL, "hidden width must be 32");
    if (cfg.routing < 0 || cfg.routing > 2) return fail(ED_EINVAL, "routing must be 0, 1 or 2");
    const int steps = cfg.routing == 0 ? (cfg.steps > 0 ? cfg.steps : 3000) : 0;
    const int batch = cfg.batch > 0 ? cfg.batch : 8192;
    const float lr0 = cfg.lr > 0 ? cfg.lr : 1e-2f;
    int lg = cfg.log2_segments;
    if (lg <= 0) {
        // about 2048 keys per segment
        lg = 4;
        while (lg < 22 && (int64_t(1) << (lg + 11)) < b->dim) ++lg;
    }
    if (lg < 1 || lg > 24) return fail(ED_EINVAL, "log2_segments must be in [1, 24]");
    const uint32_t kpc = cfg.keys_per_cell > 0 ? (uint32_t)cfg.keys_per_cell : kKeysPerCell;
    const uint32_t win = cfg.max_window > 0 ? (uint32_t)cfg.max_window : kMaxWindow;
    if (kpc > (1u << 16)) return fail(ED_EINVAL, "keys_per_cell must be at most 65536");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = b->own;
    HIP_OK(hipStreamSynchronize((hipStream_t)stream));
    TmpPool tmp(b);  // charged to the memory cap while held
    ed_status s;

    // --- rank table and equalizer (host) -------------------------------------
    const int W = N - n_up + 1, nr = rank_table_entries(N, n_up);
    std::vector<uint64_t> hr((size_t)std::max(nr, 1), 0);
    for (int j = 0; j < n_up; ++j)
        for (int q = 0; q < W; ++q) hr[(size_t)j * W + q] = binom64(q + j, j + 1);
    // knots: ranks of the keys at positions floor(j (dim - 1) / K)
    const int K = (int)std::max<int64_t>(1, std::min<int64_t>(kEqMax, b->dim - 1));
    std::vector<uint64_t> heq(kEqBytes / 8, 0);
    double *hinvw = reinterpret_cast<double *>(heq.data() + kEqMax + 1);
    for (int j = 0; j <= K; ++j) {
        const int64_t pos = (int64_t)((double)j * (double)(b->dim - 1) / (double)K);
        uint64_t key = 0;
        HIP_OK(hipMemcpy(&key, b->d_reps + std::min<int64_t>(pos, b->dim - 1), sizeof(uint64_t),
                         hipMemcpyDeviceToHost));
        heq[j] = sz_rank(key, hr.data(), W);
        if (j > 0 && heq[j] <= heq[j - 1]) heq[j] = heq[j - 1] + 1;  // one key (dim 1): any width
    }
    for (int j = 0; j < K; ++j) hinvw[j] = 1.0 / (double)(heq[j + 1] - heq[j]);
    if (!b->d_rank && (s = dev_alloc(b, (void **)&b->d_rank, kRankMaxEntries * sizeof(uint64_t))) != ED_OK) return s;
    if (!b->d_eq && (s = dev_alloc(b, (void **)&b->d_eq, kEqBytes)) != ED_OK) return s;
    HIP_OK(hipMemcpy(b->d_rank, hr.data(), (size_t)nr * sizeof(uint64_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(b->d_eq, heq.data(), kEqBytes, hipMemcpyHostToDevice));
    const Equalizer eq{reinterpret_cast<const uint64_t *>(b->d_eq),
                       reinterpret_cast<const double *>(b->d_eq + (kEqMax + 1) * 8), K, 1.0 / (double)K};
    const RankFeat rf{b->d_rank, W, n_up, eq};

    // --- network: training on (feature, position) samples ------------------
    const int NP = mlp_param_count(F, kHidden);
    const int nb = mlp_train_blocks(batch);
    if (!b->d_params && (s = dev_alloc(b, (void **)&b->d_params, kMlpMaxParams * sizeof(float))) != ED_OK) return s;
    float *d_m = nullptr, *d_v = nullptr, *d_gpart = nullptr, *d_lpart = nullptr, *d_loss = nullptr, *d_ur = nullptr;
    TAKE(tmp, &d_m, NP * sizeof(float));
    TAKE(tmp, &d_v, NP * sizeof(float));
    TAKE(tmp, &d_gpart, (size_t)nb * NP * sizeof(float));
    TAKE(tmp, &d_lpart, (size_t)nb * sizeof(float));
    TAKE(tmp, &d_loss, sizeof(float));
    TAKE(tmp, &d_ur, 2 * sizeof(float));
    HIP_OK(hipMemsetAsync(b->d_params, 0, kMlpMaxParams * sizeof(float), st));
    HIP_OK(hipMemsetAsync(d_m, 0, NP * sizeof(float), st));
    HIP_OK(hipMemsetAsync(d_v, 0, NP * sizeof(float), st));
    HIP_OK(hipMemsetAsync(d_loss, 0, sizeof(float), st));
    float ur[2] = {0.f, 1.f};
    HIP_OK(feature_range(b->d_reps, b->dim, rf, d_ur, st));
    HIP_OK(hipMemcpyAsync(ur, d_ur, 2 * sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    // input standardization x = (u - mu) * sc maps the keys' feature range to [-1, 1]
    const float mu = 0.5f * (ur[0] + ur[1]);
    const float sc = (ur[1] > ur[0]) ? 2.0f / (ur[1] - ur[0]) : 1.0f;
    HIP_OK(mlp_init(b->d_params, F, 0x5EEDull + cfg.seed, st));
    for (int t = 0; t < steps; ++t) {
        // cosine decay to 2% of the initial rate
        const float lr = lr0 * (0.02f + 0.98f * 0.5f * (1.0f + std::cos(3.14159265f * t / steps)));
        HIP_OK(mlp_train_step(b->d_params, d_m, d_v, F, mu, sc, rf, b->d_reps, b->dim, cfg.seed, t, batch, lr, d_gpart,
                              d_lpart, d_loss, st));
    }
    float loss = 0;
    HIP_OK(hipMemcpyAsync(&loss, d_loss, sizeof(float), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    // expanded form; routing 2 replaces the network by y = u (one piece)
    std::vector<float> hp(kMlpMaxParams), block;
    HIP_OK(hipMemcpy(hp.data(), b->d_params, NP * sizeof(float), hipMemcpyDeviceToHost));
    int pieces = 1;
    if (cfg.routing == 2) {
        block.assign((size_t)pw_floats(1), 0.0f);
        block[0] = 1.0f;
        block[kPwHeader + 1] = 1.0f;   // slope
        block[kPwHeader + 2] = 0.0f;   // intercept
    } else {
        double dev = 0.0;
        pieces = expand_network(hp.data(), mu, sc, block, &dev);
        double yscale = 1.0;
        for (int q = 0; q < pieces; ++q)
            yscale = std::max(yscale, (double)std::fabs(block[kPwHeader + 2 * pieces + q]));
        if (!(dev <= 1e-4 * yscale)) return fail(ED_EDEVICE, "network expansion disagrees with the network");
    }
    // blob: the pieces at off_mlp, the equalizer and the rank table right
    // behind them (LDS)
    const size_t off_rank = (b->lay.off_mlp + block.size() * sizeof(float) + 15) & ~(size_t)15;
    if (off_rank + kEqBytes + (size_t)nr * sizeof(uint64_t) > b->lay.reserved)
        return fail(ED_EDEVICE, "network expansion, equalizer and rank table larger than their reserved space");
    // nothing may still run on the old index while it is replaced
    HIP_OK(hipDeviceSynchronize());
    unsigned char *blob = static_cast<unsigned char *>(b->d_blob);
    const float *d_pw = reinterpret_cast<const float *>(blob + b->lay.off_mlp);
    HIP_OK(hipMemcpyAsync(blob + b->lay.off_mlp, block.data(), block.size() * sizeof(float), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(blob + off_rank, heq.data(), kEqBytes, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(blob + off_rank + kEqBytes, hr.data(), (size_t)nr * sizeof(uint64_t),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));  // the host copies are about to go
    b->lay.off_rank = (uint32_t)off_rank;
    b->lay.bytes = (uint32_t)((off_rank + kEqBytes + (size_t)nr * sizeof(uint64_t) + 15) & ~(size_t)15);
    {
        int bpc = 0, athreads = 0;
        HIP_OK(prepare_kernels(make_params(b), &bpc, &athreads));
        if (bpc < 1) return fail(ED_EINVAL, "tables and network exceed the LDS of one compute unit");
        set_grids(b, bpc);
    }

    // --- segments and cells --------------------------------------------------
    const uint64_t M = 1ull << lg;
    const int kblocks = 8 * b->n_cu;
    if (b->d_segs && b->lg_segs != lg) {
        dev_release(b, b->d_segs);
        b->d_segs = nullptr;
    }
    if (!b->d_segs && (s = dev_alloc(b, &b->d_segs, M * sizeof(Seg))) != ED_OK) return s;
    uint32_t *d_cnt = nullptr, *d_factor = nullptr, *d_sizes = nullptr, *d_err = nullptr, *d_bad = nullptr,
             *d_maxwin = nullptr;
    unsigned long long *d_rmin = nullptr, *d_rmax = nullptr, *d_stats = nullptr;
    uint64_t *d_offsets = nullptr, *d_total = nullptr, *d_scan = nullptr;
    unsigned int *d_count = nullptr;
    TAKE(tmp, &d_cnt, M * sizeof(uint32_t));
    TAKE(tmp, &d_factor, M * sizeof(uint32_t));
    TAKE(tmp, &d_sizes, M * sizeof(uint32_t));
    TAKE(tmp, &d_rmin, M * sizeof(unsigned long long));
    TAKE(tmp, &d_rmax, M * sizeof(unsigned long long));
    TAKE(tmp, &d_offsets, M * sizeof(uint64_t));
    TAKE(tmp, &d_total, sizeof(uint64_t));
    TAKE(tmp, &d_scan, scan_tmp_words(M) * sizeof(uint64_t));
    TAKE(tmp, &d_err, sizeof(uint32_t));
    TAKE(tmp, &d_bad, sizeof(uint32_t));
    TAKE(tmp, &d_maxwin, sizeof(uint32_t));
    TAKE(tmp, &d_count, sizeof(unsigned int));
    TAKE(tmp, &d_stats, 5 * sizeof(unsigned long long));
    HIP_OK(hipMemsetAsync(d_cnt, 0, M * sizeof(uint32_t), st));
    HIP_OK(hipMemsetAsync(d_factor, 0, M * sizeof(uint32_t), st));
    HIP_OK(hipMemsetAsync(d_rmin, 0xff, M * sizeof(unsigned long long), st));
    HIP_OK(hipMemsetAsync(d_rmax, 0, M * sizeof(unsigned long long), st));
    HIP_OK(hipMemsetAsync(d_err, 0, sizeof(uint32_t), st));
    HIP_OK(hipMemsetAsync(d_bad, 0, sizeof(uint32_t), st));
    HIP_OK(hipMemsetAsync(d_maxwin, 0, sizeof(uint32_t), st));
    HIP_OK(hipMemsetAsync(d_stats, 0, 5 * sizeof(unsigned long long), st));
    HIP_OK(index_route(d_pw, rf, lg, b->d_reps, b->dim, d_cnt, d_rmin, d_rmax, d_err, kblocks, st));
    // cell ranges and errors; segments with too wide a window get more cells
    uint32_t *c_first = nullptr, *c_last = nullptr, *c_elo = nullptr, *c_ehi = nullptr;
    uint64_t cap = 0, total = 0;
    int rounds = 0;
    for (;; ++rounds) {
        HIP_OK(index_seg_shape(M, d_cnt, d_rmin, d_rmax, kpc, d_factor, b->d_segs, d_sizes, st));
        HIP_OK(launch_scan(d_sizes, d_offsets, M, d_total, d_scan, st));
        HIP_OK(hipMemcpyAsync(&total, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (total >= (1ull << 31)) return fail(ED_EINVAL, "cell table too large");
        HIP_OK(index_seg_setoff(b->d_segs, M, d_offsets, st));
        if (total > cap) {
            cap = total + total / 2 + 1;
            TAKE(tmp, &c_first, cap * sizeof(uint32_t));
            TAKE(tmp, &c_last, cap * sizeof(uint32_t));
            TAKE(tmp, &c_elo, cap * sizeof(uint32_t));
            TAKE(tmp, &c_ehi, cap * sizeof(uint32_t));
        }
        HIP_OK(index_cells(d_pw, rf, lg, b->d_reps, b->dim, b->d_segs, total, c_first, c_last, c_elo, c_ehi, kblocks,
                           st));
        if (rounds == kRefineRounds) break;
        unsigned int refined = 0;
        HIP_OK(hipMemsetAsync(d_count, 0, sizeof(unsigned int), st));
        HIP_OK(index_refine(M, b->d_segs, d_sizes, c_first, c_last, c_elo, c_ehi, win, kMaxRefine, d_factor, d_count,
                            st));
        HIP_OK(hipMemcpyAsync(&refined, d_count, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        if (refined == 0) break;
    }
    if (b->d_cells) {
        dev_release(b, b->d_cells);
        b->d_cells = nullptr;
        b->n_cells = 0;
    }
    if ((s = dev_alloc(b, &b->d_cells, total * sizeof(uint2))) != ED_OK) return s;
    HIP_OK(index_pack(total, c_first, c_last, c_elo, c_ehi, b->d_cells, d_bad, st));
    b->n_cells = total;
    b->lg_segs = lg;
    b->eq_K = K;
    b->mlp_F = F;
    uint32_t bad = 0, net_err = 0, max_win = 0;
    unsigned long long hst[5] = {0, 0, 0, 0, 0};
    HIP_OK(index_window_stats(d_pw, rf, lg, b->d_reps, b->dim, b->d_segs, b->d_cells, total, d_stats, d_maxwin, kblocks,
                              st));
    HIP_OK(hipMemcpyAsync(&bad, d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&net_err, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&max_win, d_maxwin, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(hst, d_stats, sizeof(hst), hipMemcpyDeviceToHost, st));
    std::vector<uint32_t> hc(M), hf(M);
    HIP_OK(hipMemcpyAsync(hc.data(), d_cnt, M * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(hf.data(), d_factor, M * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    b->indexed = false;  // until the checks below pass
    if (bad) return fail(ED_EINVAL, "a cell of the learned index covers 2^20 positions or more");
    if (hst[4] != 0) return fail(ED_EDEVICE, "learned index build: a key lies outside its recorded window");
    int64_t used = 0, refined_segs = 0;
    for (uint64_t q = 0; q < M; ++q) {
        used += hc[q] ? 1 : 0;
        refined_segs += hf[q] > 1 ? 1 : 0;
    }
    for (auto &g : b->step_graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    if (!b->d_lrec && !b->T.is_complex) {
        // records {rep, x} in basis order (real sectors): the H.v gather
        // reads x_j from the record its search ends on
        const size_t words = 2;
        if ((s = dev_alloc(b, (void **)&b->d_lrec, (size_t)b->dim * words * sizeof(uint64_t))) != ED_OK) return s;
        HIP_OK(launch_lrec_keys(b->d_lrec, b->d_reps, b->dim, b->T.is_complex, b->cfg.vec_blocks, st));
        HIP_OK(hipStreamSynchronize(st));
    }
    b->indexed = true;
    const double D = (double)b->dim;
    ed_index_stats r{};
    r.max_err = (int32_t)max_win;
    r.n_segments = (int32_t)M;
    r.final_loss = loss;
    r.mlp_max_err = (float)net_err;
    r.mlp_bytes = (int64_t)NP * sizeof(float);
    r.table_bytes = (int64_t)(M * sizeof(Seg) + total * sizeof(uint2));
    r.train_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    r.mean_window = (double)hst[0] / D;
    r.n_features = F;
    r.n_pieces = pieces;
    r.used_segments = used;
    r.feature_offset = cfg.routing == 2 ? 0.0f : mu;
    r.feature_scale = cfg.routing == 2 ? 1.0f : sc;
    r.n_cells = (int64_t)total;
    r.refined_segments = refined_segs;
    r.mean_abs_err = (double)hst[1] / D;
    r.frac_exact = (double)hst[2] / D;
    r.mean_lines = (double)hst[3] / D;
    r.lds_bytes = (int64_t)(b->lay.bytes - b->lay.off_mlp);
    r.routing = cfg.routing;
    b->istats = r;
    if (out) *out = r;
    return ED_OK;
}

ed_status ed_index_info(const ed_basis *b, ed_index_stats *out, float *h_params, int64_t cap)
{
    if (!b) return fail(ED_EINVAL, "NULL basis");
    if (!b->indexed) return fail(ED_EINVAL, "no learned index: call ed_index_train first");
    if (out) *out = b->istats;
    if (h_params) {
        const int NP = mlp_param_count(b->mlp_F, kHidden);
        if (cap < NP) return fail(ED_EINVAL, "parameter buffer too small");
        HIP_OK(hipMemcpy(h_params, b->d_params, NP * sizeof(float), hipMemcpyDeviceToHost));
    }
    return ED_OK;
}

ed_status ed_index_predict(const ed_basis *b, const uint64_t *d_keys, int64_t n, float *d_u, float *d_y, void *stream)
{
    if (!b) return fail(ED_EINVAL, "NULL basis");
    if (!b->indexed) return fail(ED_EINVAL, "no learned index: call ed_index_train first");
    if (n < 0 || (n > 0 && (!d_keys || !d_u || !d_y))) return fail(ED_EINVAL, "bad arguments");
    if (n == 0) return ED_OK;
    const float *d_pw = reinterpret_cast<const float *>(static_cast<const unsigned char *>(b->d_blob) + b->lay.off_mlp);
    const Equalizer eq{reinterpret_cast<const uint64_t *>(b->d_eq),
                       reinterpret_cast<const double *>(b->d_eq + (kEqMax + 1) * 8), b->eq_K, 1.0 / (double)b->eq_K};
    const RankFeat rf{b->d_rank, b->T.N - b->T.n_up + 1, b->T.n_up, eq};
    HIP_OK(index_predict(d_pw, rf, b->T.N, d_keys, n, d_u, d_y, (hipStream_t)stream));
    return ED_OK;
}

ed_status ed_mlp_loss_grad(int32_t n_features, const float *d_params, const float *d_X, const float *d_t, int64_t n,
                           float *d_grad, float *d_loss, void *stream)
{
    if (n_features < 1 || n_features > kMaxFeatures) return fail(ED_EINVAL, "n_features must be in [1, 8]");
    if (!d_params || !d_X || !d_t || !d_grad || !d_loss || n < 1) return fail(ED_EINVAL, "bad arguments");
    const int NP = mlp_param_count(n_features, kHidden);
    const int nb = (int)((n + 63) / 64);
    TmpPool tmp;
    float *d_gpart = nullptr, *d_lpart = nullptr;
    HIP_OK(tmp.alloc((void **)&d_gpart, (size_t)nb * NP * sizeof(float)));
    HIP_OK(tmp.alloc((void **)&d_lpart, (size_t)nb * sizeof(float)));
    hipStream_t st = (hipStream_t)stream;
    HIP_OK(mlp_loss_grad(d_params, n_features, d_X, d_t, n, d_grad, d_loss, d_gpart, d_lpart, st));
    HIP_OK(hipStreamSynchronize(st));
    return ED_OK;
}

static uint32_t sub_image_bits(const int32_t *p, int X, int b, uint32_t s)
{
    uint32_t out = 0;
    for (int q = 0; q < b; ++q)
        if ((s >> (b - 1 - q)) & 1u) out |= 1u << (b - 1 - (p[X * b + q] % b));
    return out;
}

ed_status ed_tables_inspect(const ed_model *model, const ed_group *group, int32_t n_up, int32_t n_sub,
                            uint32_t *rep_out, uint32_t *sym_off, uint32_t *sym_out, int64_t sym_cap, int64_t *n_sym,
                            uint64_t *act_out)
{
    HostTables T;
    ed_status s = validate_and_copy_group(model, group, n_up, T);
    if (s != ED_OK) return s;
    if ((s = check_stable(T, n_sub)) != ED_OK) return s;
    const int b = T.N / n_sub;
    if (b > 20) return fail(ED_EINVAL, "substates wider than 20 bits");
    std::vector<uint16_t> rep;
    std::vector<uint32_t> off, lst;
    if (b > 16) return fail(ED_EINVAL, "substates wider than 16 bits");
    build_rep_sym(T, n_sub, rep, off, lst);
    const size_t S = (size_t)1 << b;
    if (rep_out)
        for (size_t i = 0; i < rep.size(); ++i) rep_out[i] = rep[i];
    if (sym_off) std::memcpy(sym_off, off.data(), off.size() * sizeof(uint32_t));
    if (n_sym) *n_sym = (int64_t)lst.size();
    if (sym_out && (int64_t)lst.size() <= sym_cap)
        for (size_t i = 0; i < lst.size(); ++i) sym_out[i] = lst[i] >> 16;
    if (act_out) {
        for (int g = 0; g < T.G; ++g) {
            const int32_t *p = &T.sp_perm[(size_t)T.sp_of[g] * T.N];
            for (int X = 0; X < n_sub; ++X) {
                int d = p[X * b] / b;
                for (uint32_t v = 0; v < S; ++v) {
                    uint32_t img = sub_image_bits(p, X, b, v);
                    if (T.flip[g]) img ^= (uint32_t)(S - 1);
                    act_out[((size_t)g * n_sub + X) * S + v] = (uint64_t)img << (T.N - (d + 1) * b);
                }
            }
        }
    }
    return ED_OK;
}

}  // extern "C"
