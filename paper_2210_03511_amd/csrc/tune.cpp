// Autotuning: the cache file of tuned choices and the tuner of the
// sublattice decomposition pair (n_sub_rep, n_sub_act).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "basis.h"
#include "tune.h"

namespace symed {

uint64_t fnv1a(const void *data, size_t n, uint64_t h)
{
    const unsigned char *p = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

uint64_t device_fingerprint(int device)
{
    hipDeviceProp_t prop{};
    uint64_t h = fnv1a(&device, 0);
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        h = fnv1a(prop.gcnArchName, std::strlen(prop.gcnArchName), h);
        h = fnv1a(&prop.multiProcessorCount, sizeof(prop.multiProcessorCount), h);
    }
    return h;
}

bool tune_cache_lookup(const char *path, const char *kind, uint64_t fp, int mode, int64_t &a, int64_t &b)
{
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[32] = {0};
        unsigned long long h = 0;
        int ver = 0, m = -1;
        long long x = 0, y = 0;
        double sec = 0;
        if (std::sscanf(line, "symed-tune %d %31s %llx %d %lld %lld %lf", &ver, k, &h, &m, &x, &y, &sec) != 7)
            continue;
        if (ver == 1 && std::strcmp(k, kind) == 0 && h == fp && m == mode) {
            a = x;
            b = y;
            found = true;  // the last matching line wins
        }
    }
    std::fclose(f);
    return found;
}

bool tune_cache_store(const char *path, const char *kind, uint64_t fp, int mode, int64_t a, int64_t b, double seconds)
{
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "a");
    if (!f) return false;
    std::fprintf(f, "symed-tune 1 %s %016llx %d %lld %lld %.6f\n", kind, (unsigned long long)fp, mode, (long long)a,
                 (long long)b, seconds);
    return std::fclose(f) == 0;
}

}  // namespace symed

using namespace symed;

namespace {

// Fingerprint of a sector problem for the decomposition tuner.
uint64_t problem_fingerprint(const ed_model *m, const ed_group *g, int n_up, int device)
{
    uint64_t h = device_fingerprint(device);
    h = fnv1a(&m->n_sites, sizeof m->n_sites, h);
    h = fnv1a(&n_up, sizeof n_up, h);
    h = fnv1a(m->bond_sites, sizeof(int32_t) * 2 * (size_t)m->n_bonds, h);
    h = fnv1a(m->bond_J, sizeof(double) * (size_t)m->n_bonds, h);
    if (m->n_tri > 0) {
        h = fnv1a(m->tri_sites, sizeof(int32_t) * 3 * (size_t)m->n_tri, h);
        h = fnv1a(m->tri_Jchi, sizeof(double) * (size_t)m->n_tri, h);
    }
    h = fnv1a(&g->n_elem, sizeof g->n_elem, h);
    h = fnv1a(g->perm, sizeof(int32_t) * (size_t)g->n_elem * m->n_sites, h);
    h = fnv1a(g->flip, (size_t)g->n_elem, h);
    h = fnv1a(g->chi_re, sizeof(double) * (size_t)g->n_elem, h);
    if (g->chi_im) h = fnv1a(g->chi_im, sizeof(double) * (size_t)g->n_elem, h);
    return h;
}

}  // namespace

extern "C" {

ed_status ed_tune_decomposition(const ed_model *model, const ed_group *group, int32_t n_up, int32_t lookup_mode,
                                const char *cache_path, void *stream, int32_t *n_sub_rep, int32_t *n_sub_act,
                                ed_tune_report *report)
{
    if (!model || !group || !n_sub_rep || !n_sub_act) return fail(ED_EINVAL, "NULL argument");
    if (lookup_mode < 0 || lookup_mode > 2) return fail(ED_EINVAL, "lookup_mode must be 0, 1 or 2");
    HostTables T;
    ed_status s = validate_and_copy_group(model, group, n_up, T);
    if (s != ED_OK) return s;
    int device = 0;
    HIP_OK(hipGetDevice(&device));
    ed_tune_report rep{};
    const uint64_t fp = problem_fingerprint(model, group, n_up, device);
    int64_t ca = 0, cb = 0;
    if (tune_cache_lookup(cache_path, "decomposition", fp, lookup_mode, ca, cb)) {
        *n_sub_rep = (int32_t)ca;
        *n_sub_act = (int32_t)cb;
        rep.cache_hit = 1;
        if (report) *report = rep;
        return ED_OK;
    }
    // stable contiguous decompositions, then pairs R | A (finest first)
    std::vector<int> subs;
    for (int n = 1; n <= T.N; ++n)
        if (T.N % n == 0 && check_stable(T, n) == ED_OK) subs.push_back(n);
    std::vector<std::pair<int, int>> pairs;
    // within the build's limits: Rep/Sym substates of at most 16 bits, action
    // substates of at most 12 bits and at most 16 action sublattices
    for (auto ia = subs.rbegin(); ia != subs.rend(); ++ia)
        for (int r : subs)
            if (*ia % r == 0 && T.N / r <= 16 && T.N / *ia <= 12 && *ia <= 16 && pairs.size() < 16)
                pairs.emplace_back(r, *ia);
    hipStream_t st = (hipStream_t)stream;
    double best = 1e300;
    int bestR = 0, bestA = 0;
    for (const auto &pr : pairs) {
        const int k = rep.n_candidates++;
        rep.sub_rep[k] = pr.first;
        rep.sub_act[k] = pr.second;
        rep.seconds[k] = -1.0;
        ed_options o{};
        o.n_sub_rep = pr.first;
        o.n_sub_act = pr.second;
        ed_basis *b = nullptr;
        if (ed_basis_build(model, group, n_up, &o, stream, &b) != ED_OK) continue;  // refused: tables too large
        ed_status ps = ED_OK;
        if (lookup_mode == 1) ps = ed_index_train(b, nullptr, nullptr, stream);
        if (lookup_mode == 2) ps = ed_hash_build(b, nullptr, nullptr, stream);
        if (ps != ED_OK) {
            ed_basis_free(b);
            continue;
        }
        const size_t vb = (size_t)b->dim * sizeof(double) * (b->T.is_complex ? 2 : 1);
        void *x = nullptr, *y = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool ok = hipMalloc(&x, vb ? vb : 16) == hipSuccess && hipMalloc(&y, vb ? vb : 16) == hipSuccess &&
                  hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
        ok = ok && launch_fill(static_cast<double *>(x), (int64_t)(vb / 8), 1.0, b->cfg.vec_blocks, st) == hipSuccess;
        float ms = 0.0f;
        ok = ok && ed_apply_H(b, x, y, lookup_mode, stream) == ED_OK;  // warm-up
        ok = ok && hipEventRecord(e0, st) == hipSuccess && ed_apply_H(b, x, y, lookup_mode, stream) == ED_OK &&
             hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(st);
        (void)hipFree(x);
        (void)hipFree(y);
        ed_basis_free(b);
        if (!ok) return fail(ED_EDEVICE, "decomposition tuner: timing failed");
        rep.seconds[k] = ms / 1e3;
        if (ms / 1e3 < best) {
            best = ms / 1e3;
            bestR = pr.first;
            bestA = pr.second;
        }
    }
    if (bestR == 0) return fail(ED_ENOTSTABLE, "no admissible decomposition pair could be built");
    *n_sub_rep = bestR;
    *n_sub_act = bestA;
    (void)tune_cache_store(cache_path, "decomposition", fp, lookup_mode, bestR, bestA, best);
    if (report) *report = rep;
    return ED_OK;
}

}  // extern "C"
