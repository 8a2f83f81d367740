// Kernels of SU(d) permutation models: basis enumeration of a color-count
// sector and the gather-form H.v (same structure as the spin-1/2 kernels:
// persistent grid-stride rows, tables staged in LDS, one lane per row, no
// atomics).
#include <hip/hip_runtime.h>

#include <mutex>

#include "colors_dev.h"
#include "launch.h"

namespace symed {

namespace {

template <bool CPLX, int MODE, int LK>
__global__ void __launch_bounds__(kApplyThreads, 8) k_apply_colors(KParams p, const double *__restrict__ x,
                                                              double *__restrict__ y, const LState *ls,
                                                              double *partials)
{
    extern __shared__ __align__(16) unsigned char lds[];
    stage_blob(lds, p.blob, p.lay.bytes);
    const Lds L = lds_view(lds, p.lay, static_cast<const unsigned char *>(p.gtab));
    const double beta = (MODE == 1) ? ls->beta_prev : 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); i0 < p.dim; i0 += stride) {
        const int64_t i = i0 + lane;
        double part = 0.0;
        if (i < p.dim) part = apply_row_colors<CPLX, MODE, LK>(p, L, i, x, y, beta);
        if (MODE != 0) {
            part = wave_sum(part);
            if (lane == 0) partials[i0 >> 6] = part;
        }
    }
}

// Per-row element count: the diagonal plus every move that changes the row's
// representative.
__global__ void __launch_bounds__(256) k_count_colors(KParams p, unsigned long long *out)
{
    extern __shared__ __align__(16) unsigned char lds[];
    stage_blob(lds, p.blob, p.lay.bytes);
    const Lds L = lds_view(lds, p.lay, static_cast<const unsigned char *>(p.gtab));
    unsigned long long c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.dim; i += stride) {
        const uint64_t s = p.reps[i];
        c += 1;
        for (int q = 0; q < p.n_moves; ++q) c += move_target(s, L.moves[q]) != s;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, c);
}

// Chunk c covers ranks [c*len, (c+1)*len) of the color-count sector in
// ascending order; a configuration is kept iff it is its own representative
// and chi is trivial on its stabilizer, with the prefix pruning of the
// spin-1/2 enumeration (a failed prefix test on coarse sublattice X skips to
// the next configuration whose bits above that sublattice's end differ).
template <bool WRITE>
__global__ void __launch_bounds__(256) k_enumerate_colors(KParams p, ColorSector cs, uint64_t total, uint64_t len,
                                                        uint64_t n_chunks, uint32_t *counts, const uint64_t *offsets,
                                                        uint64_t *out_reps, uint16_t *out_stab)
{
    extern __shared__ __align__(16) unsigned char lds[];
    stage_blob(lds, p.blob, p.lay.bytes);
    const Lds L = lds_view(lds, p.lay, static_cast<const unsigned char *>(p.gtab));
    const int N = p.N, br = p.br;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_chunks; c += stride) {
        const uint64_t r0 = c * len;
        const uint64_t r1 = min(total, r0 + len);
        uint64_t s = color_unrank(r0, total, cs);
        const uint64_t send = (r1 < total) ? color_unrank(r1, total, cs) : kNoConfig;
        uint64_t k = WRITE ? offsets[c] : 0;
        uint32_t found = 0;
        while (s < send) {
            const int bad = rep_prefix_fail(s, p, L);
            if (bad >= 0) {
                const int sh = N - (bad + 1) * br;
                s = color_next(((s >> sh) + 1) << sh, cs);
                continue;
            }
            uint32_t stab = 0;
            bool triv = true;
            if (rep_check(s, p, L, stab, triv) && triv) {
                if (WRITE) {
                    out_reps[k] = s;
                    out_stab[k] = (uint16_t)stab;
                    ++k;
                } else {
                    ++found;
                }
            }
            s = color_next(s + 1, cs);
        }
        if (!WRITE) counts[c] = found;
    }
}

}  // namespace

hipError_t launch_enumerate_colors(const KParams &p, const int32_t *counts, int n_colors, int n_sites, uint64_t total,
                                   uint64_t chunk_len, uint64_t n_chunks, uint32_t *d_counts,
                                   const uint64_t *d_offsets, uint64_t *d_reps, uint16_t *d_stab, bool write,
                                   int blocks, hipStream_t st)
{
    ColorSector cs{};
    cs.n = n_sites;
    cs.d = n_colors;
    for (int c = 0; c < 4; ++c) cs.cnt[c] = c < n_colors ? counts[c] : 0;
    const size_t lds = p.lay.bytes;
    if (write)
        hipLaunchKernelGGL(k_enumerate_colors<true>, dim3(blocks), dim3(256), lds, st, p, cs, total, chunk_len,
                           n_chunks, d_counts, d_offsets, d_reps, d_stab);
    else
        hipLaunchKernelGGL(k_enumerate_colors<false>, dim3(blocks), dim3(256), lds, st, p, cs, total, chunk_len,
                           n_chunks, d_counts, d_offsets, d_reps, d_stab);
    return hipGetLastError();
}

hipError_t launch_count_colors(const KParams &p, unsigned long long *d_count, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_colors, dim3(blocks), dim3(256), p.lay.bytes, st, p, d_count);
    return hipGetLastError();
}

hipError_t launch_apply_colors(const KParams &p, const LaunchCfg &c, const void *x, void *y, int mode, int lookup_kind,
                               const LState *ls, double *partials, hipStream_t st)
{
    const size_t lds = apply_lds_bytes(p);
    const double *xd = static_cast<const double *>(x);
    double *yd = static_cast<double *>(y);
    dim3 g(c.lookup_blocks[lookup_kind]), b(kApplyThreads);
#define SYMED_APPLY(C, M, K) hipLaunchKernelGGL((k_apply_colors<C, M, K>), g, b, lds, st, p, xd, yd, ls, partials)
#define SYMED_APPLY_K(C, M)                                                        \
    do {                                                                           \
        if (lookup_kind == kLookupHash) SYMED_APPLY(C, M, kLookupHash);             \
        else SYMED_APPLY(C, M, kLookupPlain);                                      \
    } while (0)
    if (lookup_kind == kLookupLearned) return hipErrorInvalidValue;
    if (!p.is_complex) {
        if (mode == 0) SYMED_APPLY_K(false, 0);
        else SYMED_APPLY_K(false, 1);
    } else {
        if (mode == 0) SYMED_APPLY_K(true, 0);
        else SYMED_APPLY_K(true, 2);
    }
#undef SYMED_APPLY_K
#undef SYMED_APPLY
    return hipGetLastError();
}

hipError_t prepare_color_kernels(const KParams &p, int *apply_blocks_per_cu)
{
    const size_t lds = apply_lds_bytes(p);
    const void *ks[] = {(const void *)k_apply_colors<false, 0, 0>, (const void *)k_apply_colors<false, 1, 0>,
                        (const void *)k_apply_colors<true, 0, 0>,  (const void *)k_apply_colors<true, 2, 0>,
                        (const void *)k_apply_colors<false, 0, 2>, (const void *)k_apply_colors<false, 1, 2>,
                        (const void *)k_apply_colors<true, 0, 2>,  (const void *)k_apply_colors<true, 2, 2>,
                        (const void *)k_count_colors,              (const void *)k_enumerate_colors<false>,
                        (const void *)k_enumerate_colors<true>};
    hipError_t e;
    {
        // per-kernel limit shared by every basis of the process; it only grows
        static std::mutex mu;
        static size_t granted = 0;
        std::lock_guard<std::mutex> lock(mu);
        if (lds > granted) {
            for (const void *k : ks) {
                e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                if (e != hipSuccess) return e;
            }
            granted = lds;
        }
    }
    int nb = 0;
    const void *ka = p.is_complex ? (const void *)k_apply_colors<true, 0, 0> : (const void *)k_apply_colors<false, 0, 0>;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ka, kApplyThreads, lds);
    if (e != hipSuccess) return e;
    *apply_blocks_per_cu = nb;
    return hipSuccess;
}

}  // namespace symed
