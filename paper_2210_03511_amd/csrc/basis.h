// The library-owned state behind an ed_basis handle (private).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "launch.h"

using symed::BlobLayout;
using symed::HostTables;
using symed::LaunchCfg;
using symed::LState;

struct ed_basis {
    HostTables T;
    BlobLayout lay{};
    int device = 0;
    hipStream_t own = nullptr;
    void *d_blob = nullptr;
    uint64_t *d_reps = nullptr;
    uint16_t *d_stab = nullptr;
    uint32_t *d_limits = nullptr;
    int pbits = 0;
    double limits_mean_window = 0.0;
    int64_t limits_max_window = 0;
    int64_t dim = 0;
    int64_t n_elements = 0;
    int64_t bytes = 0;
    int64_t mem_limit = 0;
    LaunchCfg cfg{};
    int n_cu = 0;
    double build_seconds = 0.0;
    // Lanczos workspace and captured step graphs (one per lookup mode)
    double *d_v = nullptr, *d_w = nullptr, *d_vprev = nullptr, *d_partials = nullptr;
    double *d_alpha = nullptr, *d_beta = nullptr;
    LState *d_ls = nullptr;
    int lanczos_cap = 0;
    int lanczos_steps = -1;        // steps of the current run (-1: none to resume)
    bool lanczos_broken = false;
    hipGraphExec_t step_graph[3] = {nullptr, nullptr, nullptr};
    // learned index
    bool indexed = false;
    void *d_gtab = nullptr;       // Rep/Sym tables when they do not fit LDS
    uint64_t *d_lrec = nullptr;   // {rep, x} records in basis order for the learned lookup (real sectors)
    float *d_params = nullptr;
    uint64_t *d_rank = nullptr;   // rank table, device copy for the build kernels
    unsigned char *d_eq = nullptr;  // equalizer (knots, inverse widths), device copy for the build kernels
    void *d_segs = nullptr;       // Seg[2^lg_segs]
    void *d_cells = nullptr;      // uint2[n_cells]
    uint64_t n_cells = 0;
    int lg_segs = 0, eq_K = 1, mlp_F = 0;
    ed_index_stats istats{};
    // hashed staging table
    bool hashed = false;
    uint64_t *d_htab = nullptr;
    uint64_t hslots = 0;
    uint32_t *d_pos2slot = nullptr;
    ed_hash_stats hstats{};
    std::vector<std::pair<void *, int64_t>> allocs;  // every device allocation and its size
};


ed_status dev_alloc(ed_basis *b, void **ptr, size_t bytes);
// Free one allocation of dev_alloc (no-op for NULL) and stop charging it to
// the memory cap.
void dev_release(ed_basis *b, void *ptr);

// Temporary device buffers of one call, freed when the call returns (error
// returns included).  With a basis, they count against its memory cap while
// they are held: take() fails with ED_ENOMEM beyond the cap.
struct TmpPool {
    std::vector<void *> ptrs;
    ed_basis *basis = nullptr;
    int64_t held = 0;
    TmpPool() = default;
    explicit TmpPool(ed_basis *b) : basis(b) {}
    TmpPool(const TmpPool &) = delete;
    TmpPool &operator=(const TmpPool &) = delete;
    ~TmpPool()
    {
        for (void *q : ptrs) (void)hipFree(q);
        if (basis) basis->bytes -= held;
    }
    hipError_t alloc(void **q, size_t bytes)
    {
        hipError_t e = hipMalloc(q, bytes ? bytes : 16);
        if (e == hipSuccess) ptrs.push_back(*q);
        return e;
    }
    ed_status take(void **q, size_t bytes);
};
symed::KParams make_params(const ed_basis *b);
// Copy of the H.v input into the records of lookup mode 1 (basis order, real
// sectors) or 2 (hashed table); nothing otherwise.
hipError_t stage_input(const ed_basis *b, int lookup_mode, const void *d_x, hipStream_t st);
ed_status lanczos_prepare(ed_basis *b, int n_iter, int lookup_mode, int keep);
ed_status lanczos_advance(ed_basis *b, int done, int n, int lookup_mode, double *h_alpha, double *h_beta,
                          int32_t *n_done);
ed_status lanczos_start(ed_basis *b, const void *d_v0, void *stream);

#define HIP_OK(expr)                                                                             \
    do {                                                                                         \
        hipError_t _e = (expr);                                                                  \
        if (_e != hipSuccess)                                                                    \
            return symed::fail(ED_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));   \
    } while (0)
