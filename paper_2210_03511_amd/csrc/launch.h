// Host-callable launchers for the device code in kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace symed {

// Lanczos scalars kept on the device between graph replays.
struct LState {
    int32_t step;         // index of the step being computed
    int32_t broken_step;  // first step whose beta vanished (-1: none)
    double beta_prev;     // beta produced by the previous step (0 at start)
    double max_abs_alpha;
};

struct LaunchCfg {
    int apply_blocks;      // largest grid of the apply kernel (persistent, grid-stride)
    int lookup_blocks[3];  // its grid per lookup kind (plain, learned, hashed)
    int apply_threads;  // block size of the apply kernel
    int vec_blocks;     // grid of the streaming vector kernels
};

hipError_t launch_enumerate(const KParams &p, const uint64_t *d_binom, uint64_t total, uint64_t chunk_len,
                            uint64_t n_chunks, uint32_t *d_counts, const uint64_t *d_offsets, uint64_t *d_reps,
                            uint16_t *d_stab, bool write, int blocks, hipStream_t st);
// Exclusive scan of n u32 counts into u64 offsets, the total to *d_total;
// d_tmp: scan_tmp_words(n) words of device memory.  Asynchronous on st.
hipError_t launch_scan(const uint32_t *d_in, uint64_t *d_out, uint64_t n, uint64_t *d_total, uint64_t *d_tmp,
                       hipStream_t st);
uint64_t scan_tmp_words(uint64_t n);
hipError_t launch_limits(const uint64_t *d_reps, int64_t dim, int N, int pbits, uint32_t *d_limits, hipStream_t st);
hipError_t launch_limits_stats(const uint32_t *d_limits, int pbits, unsigned long long *d_stats, hipStream_t st);
hipError_t launch_count_elements(const KParams &p, unsigned long long *d_count, int blocks, hipStream_t st);
// lookup_kind: 0 plain, 1 learned, 2 hashed staging table
hipError_t launch_apply(const KParams &p, const LaunchCfg &c, const void *x, void *y, int mode, int lookup_kind,
                        const LState *ls, double *partials, hipStream_t st);
hipError_t launch_hash_build(uint64_t *tab, uint64_t slots, const uint64_t *reps, int64_t dim, bool cplx,
                             uint32_t *pos2slot, unsigned long long *d_stats, int blocks, hipStream_t st);
// x into the records: record pos2slot[i] (hashed table) or i (pos2slot null,
// the learned lookup's records in basis order).
hipError_t launch_hash_values(uint64_t *tab, const uint32_t *pos2slot, const void *x, int64_t dim, bool cplx,
                              int blocks, hipStream_t st);
// Records {rep, x} in basis order for the learned lookup: write the keys.
hipError_t launch_lrec_keys(uint64_t *rec, const uint64_t *reps, int64_t dim, bool cplx, int blocks, hipStream_t st);
hipError_t launch_lookup(const KParams &p, const uint64_t *keys, int64_t n, int64_t *idx, int mode, hipStream_t st);

// Lanczos vector ops (vectors of n real or n complex numbers)
hipError_t launch_norm2_partial(const void *v, int64_t n, bool cplx, double *partials, int blocks, hipStream_t st);
hipError_t launch_scale_copy(const void *src, void *dst, int64_t n, bool cplx, const double *partials, int nparts,
                             int blocks, hipStream_t st);
hipError_t launch_finalize(const double *partials, int64_t nparts, double *alpha, double *beta, LState *ls, int which,
                           hipStream_t st);
hipError_t launch_axpy_norm(void *w, const void *v, const void *vprev, int64_t n, bool cplx, const double *alpha,
                            const LState *ls, double *partials, int blocks, hipStream_t st);
hipError_t launch_rotate(void *v, void *w, void *vprev, int64_t n, bool cplx, const double *beta, const LState *ls,
                         int blocks, hipStream_t st);
hipError_t launch_step_inc(LState *ls, const double *beta, hipStream_t st);
hipError_t launch_fill(double *v, int64_t n, double val, int blocks, hipStream_t st);
// psi[0..n2) += coef[ls->step] * v
hipError_t launch_axpy_coef(double *psi, const double *v, int64_t n2, const double *coef, const LState *ls,
                            int blocks, hipStream_t st);
// partials[0..blocks) = Re <a|b> per block; complex: partials[blocks..2 blocks) = Im
hipError_t launch_dot(const void *a, const void *b, int64_t n, bool cplx, double *partials, int blocks, hipStream_t st);
hipError_t prepare_kernels(const KParams &p, int *apply_blocks_per_cu, int *apply_threads);
hipError_t launch_lstate_init(LState *ls, hipStream_t st);

size_t apply_lds_bytes(const KParams &p);

// SU(d) permutation models (colors.hip)
hipError_t launch_enumerate_colors(const KParams &p, const int32_t *counts, int n_colors, int n_sites, uint64_t total,
                                   uint64_t chunk_len, uint64_t n_chunks, uint32_t *d_counts,
                                   const uint64_t *d_offsets, uint64_t *d_reps, uint16_t *d_stab, bool write,
                                   int blocks, hipStream_t st);
hipError_t launch_count_colors(const KParams &p, unsigned long long *d_count, int blocks, hipStream_t st);
// lookup_kind 0 (plain) or 2 (hashed staging table)
hipError_t launch_apply_colors(const KParams &p, const LaunchCfg &c, const void *x, void *y, int mode, int lookup_kind,
                               const LState *ls, double *partials, hipStream_t st);
hipError_t prepare_color_kernels(const KParams &p, int *apply_blocks_per_cu);

}  // namespace symed
