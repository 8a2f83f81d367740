// Many symmetry sectors through one persistent launch.
//
// The rows of all sectors are cut into tiles of equal length; tile t belongs
// to the sector whose tile range contains it.  Blocks walk the tiles
// round-robin (tile t on block t mod grid); a block stages the lookup tables
// of a sector into LDS when it moves to a tile of another sector, then runs
// the same per-row gather as the single-sector kernel.  Per-tile partial
// sums of the Lanczos reductions are combined per sector in tile order, so
// every result is independent of scheduling.  One Lanczos step of all
// sectors is the launch sequence batch-apply, finalize(alpha),
// batch-axpy+norm, finalize(beta), batch-rotate, step-increment, captured
// once as a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "apply_dev.h"
#include "batch.h"

namespace symed {

namespace {

constexpr int kBatchVecThreads = 256;

__device__ __forceinline__ int sector_of(const int64_t *tile0, int nsec, int64_t t)
{
    int lo = 0, hi = nsec - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile0[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// lanczos = 0: y_s = H_s x_s.  lanczos = 1: w_s <- H_s v_s - beta_s w_s
// (real sectors) or w_s <- H_s v_s (complex sectors), partial <w|v> per tile.
// As for the single-sector kernel, the register budget allows 8 waves per
// SIMD, so two blocks share a compute unit when the tables leave room.
template <int LK>
__global__ void __launch_bounds__(kApplyThreads, 8) k_batch_apply(const SectorDesc *__restrict__ secs, int nsec,
                                                             const int64_t *__restrict__ tile0g, int64_t ntiles,
                                                             int64_t tile_rows, int lanczos, double *partials)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int64_t tile0[kMaxSectors + 1];
    __shared__ double scratch[kApplyThreads / 64];
    for (int k = threadIdx.x; k <= nsec; k += blockDim.x) tile0[k] = tile0g[k];
    __syncthreads();
    int cur = -1;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int sec = sector_of(tile0, nsec, t);
        const SectorDesc &D = secs[sec];
        const KParams p = D.p;
        if (sec != cur) {
            __syncthreads();
            stage_blob(lds, p.blob, p.lay.bytes);
            cur = sec;
        }
        const Lds L = lds_view(lds, p.lay, static_cast<const unsigned char *>(p.gtab));
        const int64_t r0 = (t - tile0[sec]) * tile_rows;
        const int64_t r1 = min(r0 + tile_rows, p.dim);
        double part = 0.0;
        const double beta = (lanczos && !D.cplx) ? D.ls->beta_prev : 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            if (!lanczos) {
                if (D.cplx) apply_row<true, 0, LK>(p, L, i, D.x, D.y, 0.0);
                else apply_row<false, 0, LK>(p, L, i, D.x, D.y, 0.0);
            } else if (D.cplx) {
                part += apply_row<true, 2, LK>(p, L, i, D.v, D.w, 0.0);
            } else {
                part += apply_row<false, 1, LK>(p, L, i, D.v, D.w, beta);
            }
        }
        if (lanczos) {
            const double s = block_sum(part, scratch);
            if (threadIdx.x == 0) partials[t] = s;
        }
    }
}

// Copy of each sector's input (x, or v in a Lanczos step) into its records,
// tile by tile: the hashed staging table (lookup kind 2, slot pos2slot[i])
// or the learned lookup's records in basis order (kind 1, slot i; real
// sectors only).
__global__ void __launch_bounds__(kBatchVecThreads) k_batch_hash_values(const SectorDesc *__restrict__ secs, int nsec,
                                                                      const int64_t *__restrict__ tile0g,
                                                                      int64_t ntiles, int64_t tile_rows, int lanczos,
                                                                      int lookup)
{
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int sec = sector_of(tile0g, nsec, t);
        const SectorDesc &D = secs[sec];
        const int64_t r0 = (t - D.tile0) * tile_rows;
        const int64_t r1 = min(r0 + tile_rows, D.p.dim);
        const double *x = lanczos ? D.v : D.x;
        const bool hashed = lookup == kLookupHash;
        uint64_t *tab = const_cast<uint64_t *>(hashed ? D.p.htab : D.p.lrec);
        if (!tab) continue;  // complex sector under the learned lookup: no records
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const uint64_t s = hashed ? (uint64_t)D.pos2slot[i] : (uint64_t)i;
            if (D.cplx) {
                tab[s * 4 + 1] = (uint64_t)__double_as_longlong(x[2 * i]);
                tab[s * 4 + 2] = (uint64_t)__double_as_longlong(x[2 * i + 1]);
            } else {
                tab[s * 2 + 1] = (uint64_t)__double_as_longlong(x[i]);
            }
        }
    }
}

// which = 0: alpha_s[step] = sum of the sector's tile partials; which = 1:
// beta_s[step] = sqrt(sum), breakdown check.  One thread per sector.
__global__ void k_batch_finalize(const SectorDesc *secs, int nsec, const double *partials, int which)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsec) return;
    const SectorDesc &D = secs[s];
    double t = 0.0;
    for (int64_t k = 0; k < D.ntiles; ++k) t += partials[D.tile0 + k];
    LState *ls = D.ls;
    const int st = ls->step;
    if (which == 0) {
        D.alpha[st] = t;
        ls->max_abs_alpha = fmax(ls->max_abs_alpha, fabs(t));
    } else {
        const double b = sqrt(fmax(t, 0.0));
        D.beta[st] = b;
        if (ls->broken_step < 0 && !(b >= 1e-14 * fmax(1.0, ls->max_abs_alpha))) ls->broken_step = st;
    }
}

// w <- w - alpha v (- beta_prev vprev for complex sectors); partial |w|^2 per tile
__global__ void __launch_bounds__(kBatchVecThreads) k_batch_axpy_norm(const SectorDesc *__restrict__ secs, int nsec,
                                                                    const int64_t *__restrict__ tile0g,
                                                                    int64_t ntiles, int64_t tile_rows,
                                                                    double *partials)
{
    __shared__ double scratch[kBatchVecThreads / 64];
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int sec = sector_of(tile0g, nsec, t);
        const SectorDesc &D = secs[sec];
        const int w2 = D.cplx ? 2 : 1;
        const int64_t r0 = (t - D.tile0) * tile_rows * w2;
        const int64_t r1 = min(r0 + tile_rows * w2, D.p.dim * w2);
        const double a = D.alpha[D.ls->step];
        const double b = D.ls->beta_prev;
        double acc = 0.0;
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            double v = D.w[i] - a * D.v[i];
            if (D.cplx) v -= b * D.vprev[i];
            D.w[i] = v;
            acc += v * v;
        }
        const double s = block_sum(acc, scratch);
        if (threadIdx.x == 0) partials[t] = s;
    }
}

// real: (v, w) <- (w / beta, v); complex: vprev <- v, v <- w / beta
__global__ void __launch_bounds__(kBatchVecThreads) k_batch_rotate(const SectorDesc *__restrict__ secs, int nsec,
                                                                 const int64_t *__restrict__ tile0g, int64_t ntiles,
                                                                 int64_t tile_rows)
{
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int sec = sector_of(tile0g, nsec, t);
        const SectorDesc &D = secs[sec];
        const int w2 = D.cplx ? 2 : 1;
        const int64_t r0 = (t - D.tile0) * tile_rows * w2;
        const int64_t r1 = min(r0 + tile_rows * w2, D.p.dim * w2);
        const LState *ls = D.ls;
        const double inv = (ls->broken_step >= 0) ? 0.0 : 1.0 / D.beta[ls->step];
        for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            const double vi = D.v[i];
            D.v[i] = D.w[i] * inv;
            if (D.cplx) D.vprev[i] = vi; else D.w[i] = vi;
        }
    }
}

__global__ void k_batch_step_inc(const SectorDesc *secs, int nsec)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsec) return;
    LState *ls = secs[s].ls;
    ls->beta_prev = (ls->broken_step >= 0) ? 0.0 : secs[s].beta[ls->step];
    ls->step += 1;
}

}  // namespace

hipError_t batch_prepare(size_t lds_bytes)
{
    // the limit only ever grows (it is shared by every batch in the process)
    static std::mutex mu;
    static size_t granted = 0;
    std::lock_guard<std::mutex> lock(mu);
    if (lds_bytes <= granted) return hipSuccess;
    const void *ks[] = {(const void *)k_batch_apply<kLookupPlain>, (const void *)k_batch_apply<kLookupLearned>,
                        (const void *)k_batch_apply<kLookupHash>};
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    granted = lds_bytes;
    return hipSuccess;
}

hipError_t batch_occupancy(size_t lds_bytes, int *blocks_per_cu)
{
    // the fewest blocks per compute unit over the lookup kinds
    const void *ks[] = {(const void *)k_batch_apply<kLookupPlain>, (const void *)k_batch_apply<kLookupLearned>,
                        (const void *)k_batch_apply<kLookupHash>};
    int best = 1 << 30;
    for (const void *k : ks) {
        int nb = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kApplyThreads, lds_bytes);
        if (e != hipSuccess) return e;
        best = std::min(best, nb);
    }
    *blocks_per_cu = best;
    return hipSuccess;
}

hipError_t launch_batch_apply(const SectorDesc *d_secs, int nsec, const int64_t *d_tile0, int64_t ntiles,
                              int64_t tile_rows, int lanczos, int lookup, double *partials, int blocks, size_t lds,
                              int vec_blocks, hipStream_t st)
{
    if (lookup == kLookupHash) {
        hipLaunchKernelGGL(k_batch_hash_values, dim3(vec_blocks), dim3(kBatchVecThreads), 0, st, d_secs, nsec,
                           d_tile0, ntiles, tile_rows, lanczos, lookup);
        hipLaunchKernelGGL(k_batch_apply<kLookupHash>, dim3(blocks), dim3(kApplyThreads), lds, st, d_secs, nsec,
                           d_tile0, ntiles, tile_rows, lanczos, partials);
    } else if (lookup == kLookupLearned) {
        hipLaunchKernelGGL(k_batch_hash_values, dim3(vec_blocks), dim3(kBatchVecThreads), 0, st, d_secs, nsec,
                           d_tile0, ntiles, tile_rows, lanczos, lookup);
        hipLaunchKernelGGL(k_batch_apply<kLookupLearned>, dim3(blocks), dim3(kApplyThreads), lds, st, d_secs, nsec,
                           d_tile0, ntiles, tile_rows, lanczos, partials);
    } else {
        hipLaunchKernelGGL(k_batch_apply<kLookupPlain>, dim3(blocks), dim3(kApplyThreads), lds, st, d_secs, nsec,
                           d_tile0, ntiles, tile_rows, lanczos, partials);
    }
    return hipGetLastError();
}

hipError_t launch_batch_step(const SectorDesc *d_secs, int nsec, const int64_t *d_tile0, int64_t ntiles,
                             int64_t tile_rows, int lookup, double *partials, int apply_blocks, int vec_blocks,
                             size_t lds, hipStream_t st)
{
    hipError_t e = launch_batch_apply(d_secs, nsec, d_tile0, ntiles, tile_rows, 1, lookup, partials, apply_blocks,
                                      lds, vec_blocks, st);
    if (e != hipSuccess) return e;
    const int fb = (nsec + 63) / 64;
    hipLaunchKernelGGL(k_batch_finalize, dim3(fb), dim3(64), 0, st, d_secs, nsec, partials, 0);
    hipLaunchKernelGGL(k_batch_axpy_norm, dim3(vec_blocks), dim3(kBatchVecThreads), 0, st, d_secs, nsec, d_tile0,
                       ntiles, tile_rows, partials);
    hipLaunchKernelGGL(k_batch_finalize, dim3(fb), dim3(64), 0, st, d_secs, nsec, partials, 1);
    hipLaunchKernelGGL(k_batch_rotate, dim3(vec_blocks), dim3(kBatchVecThreads), 0, st, d_secs, nsec, d_tile0,
                       ntiles, tile_rows);
    hipLaunchKernelGGL(k_batch_step_inc, dim3(fb), dim3(64), 0, st, d_secs, nsec);
    return hipGetLastError();
}

}  // namespace symed
