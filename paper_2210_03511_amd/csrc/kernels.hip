// Device code of the symed library (gfx950 / CDNA4, wave64).
//
// The hot path is a gather-form matrix-free H.v in a symmetry-adapted basis
// (thesis chapter on large-scale exact diagonalization):
//   row i (one lane) -> every non-branching piece on its representative ->
//   sublattice-coded representative search with the lookup tables staged in
//   LDS -> index lookup -> accumulate character x norm ratio x amplitude x x_j.
// Each output entry is written by exactly one lane: no atomics, results are
// independent of scheduling.
#include <hip/hip_runtime.h>

#include <mutex>

#include "apply_dev.h"

namespace symed {

namespace {

constexpr int kVecThreads = 256;

// mode 0: y = H x.  mode 1 (real Lanczos): w <- H v - beta_prev w, partial
// <w|v>.  mode 2 (complex Lanczos): w <- H v, partial Re<w|v>.  The partials
// are one per 64 consecutive rows (partials[i / 64]), so their sum in
// k_finalize does not depend on the grid: every grid and lookup gives the
// same Lanczos coefficients.
// At least 8 waves per SIMD (two 1024-thread blocks per CU when the tables
// leave room in LDS): the register budget is capped at 64 per lane, which
// every variant meets without spilling.  RG = 0 when the Rep/Sym tables are
// in LDS (their reads are then LDS reads, not flat loads), 1 otherwise.
template <bool CPLX, int MODE, int LK, int RG>
__global__ void __launch_bounds__(kApplyThreads, 8) k_apply(KParams p, const double *__restrict__ x,
                                                       double *__restrict__ y, const LState *ls,
                                                       double *partials)
{
    extern __shared__ __align__(16) unsigned char lds[];
    stage_blob(lds, p.blob, p.lay.bytes);
    const Lds L = lds_view_t<RG>(lds, p.lay, static_cast<const unsigned char *>(p.gtab));
    const double beta = (MODE == 1) ? ls->beta_prev : 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    // rows of one wave are 64 consecutive rows; the loop is wave-uniform
    for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x - lane); i0 < p.dim; i0 += stride) {
        const int64_t i = i0 + lane;
        double part = 0.0;
        if (i < p.dim) part = apply_row<CPLX, MODE, LK>(p, L, i, x, y, beta);
        if (MODE != 0) {
            part = wave_sum(part);
            if (lane == 0) partials[i0 >> 6] = part;
        }
    }
}

// Per-row element count: the diagonal plus every antiparallel pair with a
// non-zero merged amplitude.
template <bool CPLX>
__global__ void __launch_bounds__(256) k_count(KParams p, unsigned long long *out)
{
    extern __shared__ __align__(16) unsigned char lds[];
    stage_blob(lds, p.blob, p.lay.bytes);
    const Lds L = lds_view(lds, p.lay, static_cast<const unsigned char *>(p.gtab));
    unsigned long long c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.dim; i += stride) {
        const uint64_t s = p.reps[i];
        c += 1;
        for (int q = 0; q < p.n_pairs; ++q) {
            const PairTerm pt = L.pairs[q];
            if (__popcll(s & pt.mask) != 1) continue;
            double hre, him;
            pair_amp<CPLX>(s, pt, L, hre, him);
            if (hre != 0.0 || him != 0.0) ++c;
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, c);
}

// LK = kLookupHash: membership from the staging table, position from the
// plain lookup (the table holds no positions).
template <int LK>
__global__ void __launch_bounds__(256) k_lookup(KParams p, const uint64_t *keys, int64_t n, int64_t *idx)
{
    // the learned index's region of the blob (network, equalizer, rank table)
    __shared__ __align__(16) unsigned char sli[kLearnedLdsMax];
    if (LK == kLookupLearned) {
        const unsigned char *blob = static_cast<const unsigned char *>(p.blob) + p.lay.off_mlp;
        const uint32_t nb = p.lay.bytes - p.lay.off_mlp;
        for (uint32_t q = threadIdx.x; q < nb / 16u; q += blockDim.x)
            reinterpret_cast<uint4 *>(sli)[q] = reinterpret_cast<const uint4 *>(blob)[q];
        __syncthreads();
    }
    const LearnedLds li = learned_lds(sli, 0u, LK == kLookupLearned ? p.lay.off_rank - p.lay.off_mlp : 0u);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const uint64_t key = keys[k];
        // keys outside the N-bit range cannot be representatives
        int64_t r = -1;
        if (!(key & ~p.maskN)) {
            if (LK == kLookupHash) {
                const bool in = p.is_complex ? hash_find<true>(key, p) >= 0 : hash_find<false>(key, p) >= 0;
                r = in ? lookup<false>(key, p, li) : -1;
            } else {
                r = lookup<LK == kLookupLearned>(key, p, li);
            }
        }
        idx[k] = r;
    }
}

// Hashed staging table.  Build: every slot empty, then every
// representative inserted by linear probing from its home slot with a
// 64-bit compare-and-swap (the layout depends on the order of insertion,
// the results of H.v do not: only the slot of a record changes).
template <bool CPLX>
__global__ void __launch_bounds__(256) k_hash_clear(uint64_t *tab, uint64_t slots)
{
    constexpr int S = hash_words<CPLX>();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < (int64_t)slots; s += stride) {
        tab[s * S] = kHashEmpty;
        for (int w = 1; w < S; ++w) tab[s * S + w] = 0ull;
    }
}

template <bool CPLX>
__global__ void __launch_bounds__(256) k_hash_insert(uint64_t *tab, uint64_t slots, const uint64_t *__restrict__ reps,
                                                     int64_t dim, uint32_t *pos2slot, unsigned long long *stats)
{
    constexpr int S = hash_words<CPLX>();
    unsigned long long sum = 0, mx = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        const uint64_t key = reps[i];
        const uint64_t home = hash_home(key, slots);
        uint64_t s = home;
        for (;;) {
            const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long *>(tab + s * S),
                                                     (unsigned long long)kHashEmpty, (unsigned long long)key);
            if (old == (unsigned long long)kHashEmpty) break;
            if (++s == slots) s = 0;
        }
        pos2slot[i] = (uint32_t)s;
        const unsigned long long d = (s >= home ? s - home : s + slots - home) + 1;  // probes to reach it
        sum += d;
        mx = d > mx ? d : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o, 64);
        const unsigned long long m2 = __shfl_xor(mx, o, 64);
        mx = m2 > mx ? m2 : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(stats, sum);
        atomicMax(stats + 1, mx);
    }
}

// Keys of the learned lookup's records, in basis order (x is copied in
// before every H.v, as for the hashed table, with slot = row).
template <bool CPLX>
__global__ void __launch_bounds__(256) k_lrec_keys(uint64_t *rec, const uint64_t *__restrict__ reps, int64_t dim)
{
    constexpr int S = hash_words<CPLX>();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        rec[i * S] = reps[i];
        for (int w = 1; w < S; ++w) rec[i * S + w] = 0ull;
    }
}

// Copy of the input vector into the records (before every H.v); pos2slot
// null: record i belongs to row i.
template <bool CPLX>
__global__ void __launch_bounds__(256) k_hash_values(uint64_t *tab, const uint32_t *__restrict__ pos2slot,
                                                     const double *__restrict__ x, int64_t dim)
{
    constexpr int S = hash_words<CPLX>();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += stride) {
        const uint64_t s = pos2slot ? pos2slot[i] : (uint64_t)i;
        if (CPLX) {
            const double2 v = reinterpret_cast<const double2 *>(x)[i];
            tab[s * S + 1] = (uint64_t)__double_as_longlong(v.x);
            tab[s * S + 2] = (uint64_t)__double_as_longlong(v.y);
        } else {
            tab[s * S + 1] = (uint64_t)__double_as_longlong(x[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// basis enumeration
// ---------------------------------------------------------------------------

// k-th (0-based) N-bit integer with `ones` set bits, ascending order
__device__ uint64_t unrank(int n, int ones, uint64_t r, const uint64_t *binom)
{
    uint64_t s = 0;
    for (int pos = n - 1; pos >= 0 && ones > 0; --pos) {
        const uint64_t c = binom[pos * 64 + ones];  // integers with bit pos clear
        if (r >= c) {
            s |= 1ull << pos;
            r -= c;
            --ones;
        }
    }
    return s;
}

constexpr uint64_t kInf = ~0ull;

// smallest v >= t with popcount(v) == k and v < 2^N, else kInf
__device__ __forceinline__ uint64_t next_with_popcount(uint64_t t, int k, int N)
{
    for (;;) {
        if (t >> N) return kInf;
        const int c = __popcll(t);
        if (c == k) return t;
        if (c < k) {
            for (int q = 0; q < k - c; ++q) t |= t + 1;  // set the lowest zero bit
            return (t >> N) ? kInf : t;
        }
        t += t & (~t + 1);  // clear the lowest run of ones, carry
    }
}

// Chunk c covers ranks [c*len, (c+1)*len) of the Sz sector in ascending
// order.  A configuration is kept iff it is its own representative and chi
// is trivial on its stabilizer (algorithm "Preparation of the distributed
// and symmetrized Hilbert space", on one device).  Prefix pruning: the
// identity is in G_0, so a representative has Rep_0(s_0) = s_0 and
// Rep_X(s_X) >= s_0 for every coarse sublattice X; a failed test on X
// rejects every configuration sharing sublattices 0..X, which are skipped.
template <bool WRITE, int RG>
__global__ void __launch_bounds__(256) k_enumerate(KParams p, const uint64_t *binom, uint64_t total, uint64_t len,
                                                 uint64_t n_chunks, uint32_t *counts, const uint64_t *offsets,
                                                 uint64_t *out_reps, uint16_t *out_stab)
{
    extern __shared__ __align__(16) unsigned char lds[];
    stage_blob(lds, p.blob, p.lay.bytes);
    const Lds L = lds_view_t<RG>(lds, p.lay, static_cast<const unsigned char *>(p.gtab));
    const int N = p.N, br = p.br;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_chunks; c += stride) {
        const uint64_t r0 = c * len;
        const uint64_t r1 = min(total, r0 + len);
        uint64_t s = unrank(N, p.n_up, r0, binom);
        const uint64_t send = (r1 < total) ? unrank(N, p.n_up, r1, binom) : kInf;
        uint64_t k = WRITE ? offsets[c] : 0;
        uint32_t found = 0;
        while (s < send) {
            const int bad = rep_prefix_fail(s, p, L);
            if (bad >= 0) {
                const int sh = N - (bad + 1) * br;
                s = next_with_popcount(((s >> sh) + 1) << sh, p.n_up, N);
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
            // next configuration with the same number of up spins
            if (s == 0) break;
            const uint64_t tt = s | (s - 1);
            const uint64_t nx = (tt + 1) | (((~tt & (tt + 1)) - 1) >> (__builtin_ctzll(s) + 1));
            if ((nx >> N) || nx <= s) break;
            s = nx;
        }
        if (!WRITE) counts[c] = found;
    }
}

// exclusive scan of u32 counts into u64 offsets, 4096 elements per block
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;

__global__ void __launch_bounds__(kScanThreads) k_scan_block(const uint32_t *in, uint64_t *out, uint64_t n,
                                                           uint64_t *block_sums)
{
    __shared__ uint64_t sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanThreads * kScanPer + (uint64_t)threadIdx.x * kScanPer;
    uint64_t v[kScanPer];
    uint64_t tsum = 0;
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        tsum += v[q];
    }
    sh[threadIdx.x] = tsum;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        uint64_t t = (threadIdx.x >= (unsigned)o) ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    uint64_t run = sh[threadIdx.x] - tsum;  // exclusive prefix of this thread
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == kScanThreads - 1) block_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void __launch_bounds__(kScanThreads) k_scan_u64_block(const uint64_t *in, uint64_t *out, uint64_t n,
                                                               uint64_t *block_sums)
{
    __shared__ uint64_t sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanThreads * kScanPer + (uint64_t)threadIdx.x * kScanPer;
    uint64_t v[kScanPer];
    uint64_t tsum = 0;
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        tsum += v[q];
    }
    sh[threadIdx.x] = tsum;
    __syncthreads();
    for (int o = 1; o < kScanThreads; o <<= 1) {
        uint64_t t = (threadIdx.x >= (unsigned)o) ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    uint64_t run = sh[threadIdx.x] - tsum;
    for (int q = 0; q < kScanPer; ++q) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == kScanThreads - 1) block_sums[blockIdx.x] = sh[threadIdx.x];
}

__global__ void k_add_offsets(uint64_t *out, uint64_t n, const uint64_t *block_off)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += block_off[i / (kScanThreads * kScanPer)];
}

__global__ void k_limits(const uint64_t *reps, int64_t dim, int N, int pbits, uint32_t *limits)
{
    const uint64_t np = 1ull << pbits;
    const uint64_t pf = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pf > np) return;
    if (pf == np) {
        limits[pf] = (uint32_t)dim;
        return;
    }
    const uint64_t key = pf << (N - pbits);
    int64_t lo = 0, hi = dim;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (reps[mid] < key) lo = mid + 1; else hi = mid;
    }
    limits[pf] = (uint32_t)lo;
}

// key-weighted bucket statistics of the Limits table: sum of size^2, max size
__global__ void k_limits_stats(const uint32_t *limits, int pbits, unsigned long long *stats)
{
    const uint64_t np = 1ull << pbits;
    unsigned long long sq = 0, mx = 0;
    for (uint64_t pf = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; pf < np; pf += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long w = limits[pf + 1] - limits[pf];
        sq += w * w;
        mx = w > mx ? w : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
        sq += __shfl_xor(sq, o, 64);
        const unsigned long long t = __shfl_xor(mx, o, 64);
        mx = t > mx ? t : mx;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&stats[0], sq);
        atomicMax(&stats[1], mx);
    }
}

// ---------------------------------------------------------------------------
// Lanczos vector kernels (deterministic: fixed grid, fixed reduction order)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kVecThreads) k_norm2(const double *v, int64_t n2, double *partials)
{
    __shared__ double scratch[kVecThreads / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) acc += v[i] * v[i];
    const double t = block_sum(acc, scratch);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

__device__ __forceinline__ double sum_partials(const double *partials, int nparts)
{
    double t = 0.0;
    for (int k = 0; k < nparts; ++k) t += partials[k];
    return t;
}

__global__ void __launch_bounds__(kVecThreads) k_scale_copy(const double *src, double *dst, int64_t n2,
                                                          const double *partials, int nparts)
{
    __shared__ double inv;
    if (threadIdx.x == 0) inv = 1.0 / sqrt(sum_partials(partials, nparts));
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) dst[i] = src[i] * inv;
}

// which = 0: alpha[step] = sum; which = 1: beta[step] = sqrt(sum), breakdown
// check.  One block of kFinalizeThreads: thread t adds partials t, t + T,
// t + 2T, ... in order, then the block sum in a fixed order.
constexpr int kFinalizeThreads = 1024;

__global__ void __launch_bounds__(kFinalizeThreads) k_finalize(const double *partials, int64_t nparts, double *alpha,
                                                               double *beta, LState *ls, int which)
{
    __shared__ double scratch[kFinalizeThreads / 64];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < nparts; k += blockDim.x) acc += partials[k];
    const double t = block_sum(acc, scratch);
    if (threadIdx.x != 0) return;
    const int st = ls->step;
    if (which == 0) {
        alpha[st] = t;
        ls->max_abs_alpha = fmax(ls->max_abs_alpha, fabs(t));
    } else {
        const double b = sqrt(fmax(t, 0.0));
        beta[st] = b;
        if (ls->broken_step < 0 && !(b >= 1e-14 * fmax(1.0, ls->max_abs_alpha))) ls->broken_step = st;
    }
}

// psi <- psi + coef[step] v  (n doubles; the Ritz vector of a second
// Lanczos pass, coefficient of the current Lanczos vector)
__global__ void __launch_bounds__(kVecThreads) k_axpy_coef(double *psi, const double *v, int64_t n,
                                                         const double *coef, const LState *ls)
{
    const double c = coef[ls->step];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) psi[i] += c * v[i];
}

// per-block partials of <a|b> = sum conj(a_i) b_i: real part in partials[b],
// imaginary part (complex vectors) in partials[gridDim + b]
template <bool CPLX>
__global__ void __launch_bounds__(kVecThreads) k_dot(const double *a, const double *b, int64_t n, double *partials)
{
    __shared__ double scratch[kVecThreads / 64];
    double re = 0.0, im = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (CPLX) {
            const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
            re += ar * br + ai * bi;
            im += ar * bi - ai * br;
        } else {
            re += a[i] * b[i];
        }
    }
    const double sr = block_sum(re, scratch);
    if (threadIdx.x == 0) partials[blockIdx.x] = sr;
    if (CPLX) {
        const double si = block_sum(im, scratch);
        if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = si;
    }
}

// real: w <- w - alpha v ; complex: w <- w - alpha v - beta_prev vprev ; partial |w|^2
template <bool CPLX>
__global__ void __launch_bounds__(kVecThreads) k_axpy_norm(double *w, const double *v, const double *vprev,
                                                         int64_t n2, const double *alpha, const LState *ls,
                                                         double *partials)
{
    __shared__ double scratch[kVecThreads / 64];
    const double a = alpha[ls->step];
    const double b = ls->beta_prev;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
        double t = w[i] - a * v[i];
        if (CPLX) t -= b * vprev[i];
        w[i] = t;
        acc += t * t;
    }
    const double t = block_sum(acc, scratch);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// real: (v, w) <- (w / beta, v) ; complex: vprev <- v, v <- w / beta
template <bool CPLX>
__global__ void __launch_bounds__(kVecThreads) k_rotate(double *v, double *w, double *vprev, int64_t n2,
                                                      const double *beta, const LState *ls)
{
    const int st = ls->step;
    const bool broken = ls->broken_step >= 0;
    const double inv = broken ? 0.0 : 1.0 / beta[st];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
        const double vi = v[i];
        v[i] = w[i] * inv;
        if (CPLX) vprev[i] = vi; else w[i] = vi;
    }
}

__global__ void k_step_inc(LState *ls, const double *beta)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ls->beta_prev = (ls->broken_step >= 0) ? 0.0 : beta[ls->step];
        ls->step += 1;
    }
}

__global__ void __launch_bounds__(kVecThreads) k_fill(double *v, int64_t n, double val)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) v[i] = val;
}

__global__ void k_lstate_init(LState *ls)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ls->step = 0;
        ls->broken_step = -1;
        ls->beta_prev = 0.0;
        ls->max_abs_alpha = 0.0;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

size_t apply_lds_bytes(const KParams &p) { return (size_t)p.lay.bytes; }

hipError_t launch_enumerate(const KParams &p, const uint64_t *d_binom, uint64_t total, uint64_t chunk_len,
                            uint64_t n_chunks, uint32_t *d_counts, const uint64_t *d_offsets, uint64_t *d_reps,
                            uint16_t *d_stab, bool write, int blocks, hipStream_t st)
{
    const size_t lds = p.lay.bytes;
#define SYMED_ENUM(W, RG)                                                                                   \
    hipLaunchKernelGGL((k_enumerate<W, RG>), dim3(blocks), dim3(256), lds, st, p, d_binom, total, chunk_len, \
                       n_chunks, d_counts, d_offsets, d_reps, d_stab)
    if (p.lay.rep_global) {
        if (write) SYMED_ENUM(true, 1);
        else SYMED_ENUM(false, 1);
    } else {
        if (write) SYMED_ENUM(true, 0);
        else SYMED_ENUM(false, 0);
    }
#undef SYMED_ENUM
    return hipGetLastError();
}

uint64_t scan_tmp_words(uint64_t n)
{
    const uint64_t per = (uint64_t)kScanThreads * kScanPer;
    const uint64_t nb = n > per ? (n + per - 1) / per : 1;
    // block sums and their scanned offsets, then the next level's
    return 2 * (nb + 1) + (nb > 1 ? scan_tmp_words(nb) : 0);
}

// Exclusive scan, one level: per-block scans, then the block sums are
// scanned (recursively) and added back.  tmp holds scan_tmp_words(n) words.
template <typename T>
static hipError_t scan_level(const T *d_in, uint64_t *d_out, uint64_t n, uint64_t *d_total, uint64_t *tmp,
                             hipStream_t st)
{
    const uint64_t per = (uint64_t)kScanThreads * kScanPer;
    const uint64_t nb = n > per ? (n + per - 1) / per : 1;
    uint64_t *sums = tmp, *sums_off = tmp + nb + 1;
    if (sizeof(T) == sizeof(uint32_t))
        hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(kScanThreads), 0, st,
                           reinterpret_cast<const uint32_t *>(d_in), d_out, n, sums);
    else
        hipLaunchKernelGGL(k_scan_u64_block, dim3(nb), dim3(kScanThreads), 0, st,
                           reinterpret_cast<const uint64_t *>(d_in), d_out, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nb > 1) {
        e = scan_level<uint64_t>(sums, sums_off, nb, d_total, tmp + 2 * (nb + 1), st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_add_offsets, dim3((n + 255) / 256), dim3(256), 0, st, d_out, n, sums_off);
        return hipGetLastError();
    }
    // single block: total = sums[0]
    return hipMemcpyAsync(d_total, sums, sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
}

hipError_t launch_scan(const uint32_t *d_in, uint64_t *d_out, uint64_t n, uint64_t *d_total, uint64_t *d_tmp,
                       hipStream_t st)
{
    return scan_level<uint32_t>(d_in, d_out, n, d_total, d_tmp, st);
}

hipError_t launch_limits(const uint64_t *d_reps, int64_t dim, int N, int pbits, uint32_t *d_limits, hipStream_t st)
{
    const uint64_t n = (1ull << pbits) + 1;
    hipLaunchKernelGGL(k_limits, dim3((n + 255) / 256), dim3(256), 0, st, d_reps, dim, N, pbits, d_limits);
    return hipGetLastError();
}

hipError_t launch_limits_stats(const uint32_t *d_limits, int pbits, unsigned long long *d_stats, hipStream_t st)
{
    hipLaunchKernelGGL(k_limits_stats, dim3(1024), dim3(256), 0, st, d_limits, pbits, d_stats);
    return hipGetLastError();
}

hipError_t launch_count_elements(const KParams &p, unsigned long long *d_count, int blocks, hipStream_t st)
{
    if (p.n_colors) return launch_count_colors(p, d_count, blocks, st);
    if (p.is_complex)
        hipLaunchKernelGGL(k_count<true>, dim3(blocks), dim3(256), p.lay.bytes, st, p, d_count);
    else
        hipLaunchKernelGGL(k_count<false>, dim3(blocks), dim3(256), p.lay.bytes, st, p, d_count);
    return hipGetLastError();
}

hipError_t launch_apply(const KParams &p, const LaunchCfg &c, const void *x, void *y, int mode, int lookup_kind,
                        const LState *ls, double *partials, hipStream_t st)
{
    if (p.n_colors) return launch_apply_colors(p, c, x, y, mode, lookup_kind, ls, partials, st);
    const size_t lds = apply_lds_bytes(p);
    const double *xd = static_cast<const double *>(x);
    double *yd = static_cast<double *>(y);
    dim3 g(c.lookup_blocks[lookup_kind]), b(kApplyThreads);
#define SYMED_APPLY(C, M, K)                                                                      \
    do {                                                                                          \
        if (p.lay.rep_global) hipLaunchKernelGGL((k_apply<C, M, K, 1>), g, b, lds, st, p, xd, yd, ls, partials); \
        else hipLaunchKernelGGL((k_apply<C, M, K, 0>), g, b, lds, st, p, xd, yd, ls, partials);   \
    } while (0)
#define SYMED_APPLY_K(C, M)                                                        \
    do {                                                                           \
        if (lookup_kind == kLookupHash) SYMED_APPLY(C, M, kLookupHash);             \
        else if (lookup_kind == kLookupLearned) SYMED_APPLY(C, M, kLookupLearned);  \
        else SYMED_APPLY(C, M, kLookupPlain);                                      \
    } while (0)
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

hipError_t launch_hash_build(uint64_t *tab, uint64_t slots, const uint64_t *reps, int64_t dim, bool cplx,
                             uint32_t *pos2slot, unsigned long long *d_stats, int blocks, hipStream_t st)
{
    if (cplx) {
        hipLaunchKernelGGL(k_hash_clear<true>, dim3(blocks), dim3(256), 0, st, tab, slots);
        hipLaunchKernelGGL(k_hash_insert<true>, dim3(blocks), dim3(256), 0, st, tab, slots, reps, dim, pos2slot,
                           d_stats);
    } else {
        hipLaunchKernelGGL(k_hash_clear<false>, dim3(blocks), dim3(256), 0, st, tab, slots);
        hipLaunchKernelGGL(k_hash_insert<false>, dim3(blocks), dim3(256), 0, st, tab, slots, reps, dim, pos2slot,
                           d_stats);
    }
    return hipGetLastError();
}

hipError_t launch_hash_values(uint64_t *tab, const uint32_t *pos2slot, const void *x, int64_t dim, bool cplx,
                              int blocks, hipStream_t st)
{
    const double *xd = static_cast<const double *>(x);
    if (cplx) hipLaunchKernelGGL(k_hash_values<true>, dim3(blocks), dim3(256), 0, st, tab, pos2slot, xd, dim);
    else hipLaunchKernelGGL(k_hash_values<false>, dim3(blocks), dim3(256), 0, st, tab, pos2slot, xd, dim);
    return hipGetLastError();
}

hipError_t launch_lrec_keys(uint64_t *rec, const uint64_t *reps, int64_t dim, bool cplx, int blocks, hipStream_t st)
{
    if (cplx) hipLaunchKernelGGL(k_lrec_keys<true>, dim3(blocks), dim3(256), 0, st, rec, reps, dim);
    else hipLaunchKernelGGL(k_lrec_keys<false>, dim3(blocks), dim3(256), 0, st, rec, reps, dim);
    return hipGetLastError();
}

hipError_t launch_lookup(const KParams &p, const uint64_t *keys, int64_t n, int64_t *idx, int mode, hipStream_t st)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    if (mode == kLookupHash)
        hipLaunchKernelGGL(k_lookup<kLookupHash>, dim3((unsigned)blocks), dim3(256), 0, st, p, keys, n, idx);
    else if (mode == kLookupLearned)
        hipLaunchKernelGGL(k_lookup<kLookupLearned>, dim3((unsigned)blocks), dim3(256), 0, st, p, keys, n, idx);
    else
        hipLaunchKernelGGL(k_lookup<kLookupPlain>, dim3((unsigned)blocks), dim3(256), 0, st, p, keys, n, idx);
    return hipGetLastError();
}

hipError_t launch_norm2_partial(const void *v, int64_t n, bool cplx, double *partials, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_norm2, dim3(blocks), dim3(kVecThreads), 0, st, static_cast<const double *>(v),
                       cplx ? 2 * n : n, partials);
    return hipGetLastError();
}

hipError_t launch_scale_copy(const void *src, void *dst, int64_t n, bool cplx, const double *partials, int nparts,
                             int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale_copy, dim3(blocks), dim3(kVecThreads), 0, st, static_cast<const double *>(src),
                       static_cast<double *>(dst), cplx ? 2 * n : n, partials, nparts);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int64_t nparts, double *alpha, double *beta, LState *ls, int which,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalizeThreads), 0, st, partials, nparts, alpha, beta, ls, which);
    return hipGetLastError();
}

hipError_t launch_axpy_norm(void *w, const void *v, const void *vprev, int64_t n, bool cplx, const double *alpha,
                            const LState *ls, double *partials, int blocks, hipStream_t st)
{
    if (cplx)
        hipLaunchKernelGGL(k_axpy_norm<true>, dim3(blocks), dim3(kVecThreads), 0, st, static_cast<double *>(w),
                           static_cast<const double *>(v), static_cast<const double *>(vprev), 2 * n, alpha, ls,
                           partials);
    else
        hipLaunchKernelGGL(k_axpy_norm<false>, dim3(blocks), dim3(kVecThreads), 0, st, static_cast<double *>(w),
                           static_cast<const double *>(v), static_cast<const double *>(vprev), n, alpha, ls,
                           partials);
    return hipGetLastError();
}

hipError_t launch_rotate(void *v, void *w, void *vprev, int64_t n, bool cplx, const double *beta, const LState *ls,
                         int blocks, hipStream_t st)
{
    if (cplx)
        hipLaunchKernelGGL(k_rotate<true>, dim3(blocks), dim3(kVecThreads), 0, st, static_cast<double *>(v),
                           static_cast<double *>(w), static_cast<double *>(vprev), 2 * n, beta, ls);
    else
        hipLaunchKernelGGL(k_rotate<false>, dim3(blocks), dim3(kVecThreads), 0, st, static_cast<double *>(v),
                           static_cast<double *>(w), static_cast<double *>(vprev), n, beta, ls);
    return hipGetLastError();
}

hipError_t launch_step_inc(LState *ls, const double *beta, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, st, ls, beta);
    return hipGetLastError();
}

hipError_t launch_axpy_coef(double *psi, const double *v, int64_t n2, const double *coef, const LState *ls,
                            int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_axpy_coef, dim3(blocks), dim3(kVecThreads), 0, st, psi, v, n2, coef, ls);
    return hipGetLastError();
}

hipError_t launch_dot(const void *a, const void *b, int64_t n, bool cplx, double *partials, int blocks, hipStream_t st)
{
    const double *ad = static_cast<const double *>(a), *bd = static_cast<const double *>(b);
    if (cplx) hipLaunchKernelGGL(k_dot<true>, dim3(blocks), dim3(kVecThreads), 0, st, ad, bd, n, partials);
    else hipLaunchKernelGGL(k_dot<false>, dim3(blocks), dim3(kVecThreads), 0, st, ad, bd, n, partials);
    return hipGetLastError();
}

hipError_t launch_fill(double *v, int64_t n, double val, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kVecThreads), 0, st, v, n, val);
    return hipGetLastError();
}

// Allow the dynamic LDS the table blob needs and report how many apply blocks
// fit on one compute unit.
hipError_t prepare_kernels(const KParams &p, int *apply_blocks_per_cu, int *apply_threads)
{
    const size_t lds = apply_lds_bytes(p);
    hipError_t e;
#define SYMED_K4(RG, K)                                                                             \
    (const void *)k_apply<false, 0, K, RG>, (const void *)k_apply<false, 1, K, RG>,                   \
        (const void *)k_apply<true, 0, K, RG>, (const void *)k_apply<true, 2, K, RG>
    const void *ks[] = {SYMED_K4(0, 0), SYMED_K4(0, 1), SYMED_K4(0, 2), SYMED_K4(1, 0), SYMED_K4(1, 1),
                        SYMED_K4(1, 2), (const void *)k_count<false>, (const void *)k_count<true>,
                        (const void *)k_enumerate<false, 0>, (const void *)k_enumerate<true, 0>,
                        (const void *)k_enumerate<false, 1>, (const void *)k_enumerate<true, 1>};
#undef SYMED_K4
    {
        // the limit is per kernel, shared by every basis in the process: it
        // only ever grows, so a later basis with smaller tables cannot
        // invalidate the launches of an earlier one
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
    *apply_threads = kApplyThreads;
    if (p.n_colors) return prepare_color_kernels(p, apply_blocks_per_cu);
    int nb = 0;
    const void *ka = p.lay.rep_global
                         ? (p.is_complex ? (const void *)k_apply<true, 0, 1, 1> : (const void *)k_apply<false, 0, 1, 1>)
                         : (p.is_complex ? (const void *)k_apply<true, 0, 1, 0> : (const void *)k_apply<false, 0, 1, 0>);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ka, kApplyThreads, lds);
    if (e != hipSuccess) return e;
    *apply_blocks_per_cu = nb;
    *apply_threads = kApplyThreads;
    return hipSuccess;
}

hipError_t launch_lstate_init(LState *ls, hipStream_t st)
{
    hipLaunchKernelGGL(k_lstate_init, dim3(1), dim3(64), 0, st, ls);
    return hipGetLastError();
}

}  // namespace symed
