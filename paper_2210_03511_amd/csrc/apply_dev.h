// Device-side pieces of the H.v gather shared by the single-sector and the
// batched (many sectors, one persistent launch) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"
#include "learned_dev.h"
#include "represent.h"

namespace symed {

// Compile-time tuning knobs (block size of the H.v kernel, lookups kept in
// flight per lane).
#ifndef SYMED_APPLY_THREADS
#define SYMED_APPLY_THREADS 1024
#endif
#ifndef SYMED_KBATCH
#define SYMED_KBATCH 1
#endif
constexpr int kApplyThreads = SYMED_APPLY_THREADS;

// Copy the table blob (multiple of 16 bytes) into LDS.
__device__ __forceinline__ void stage_blob(unsigned char *lds, const void *blob, uint32_t bytes)
{
    const uint4 *s = reinterpret_cast<const uint4 *>(blob);
    uint4 *d = reinterpret_cast<uint4 *>(lds);
    for (uint32_t k = threadIdx.x; k < bytes / 16u; k += blockDim.x) d[k] = s[k];
    __syncthreads();
}

// Plain index lookup: Limits(prefix) = [begin, end) then binary search
// (thesis: "Basis" array plus "Limits" prefix map, section on distributed
// memory parallelization).  -1 if absent.
__device__ __forceinline__ int64_t lookup_plain(uint64_t key, const KParams &p)
{
    const uint64_t pf = key >> (p.N - p.pbits);
    uint32_t lo = p.limits[pf], hi = p.limits[pf + 1];
    const uint32_t end = hi;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (p.reps[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < end && p.reps[lo] == key) ? (int64_t)lo : -1;
}

// K independent lookups advanced in lockstep: every round issues the probe
// loads of all unfinished searches before comparing, so one lane keeps up
// to K dependent-load chains in flight.  valid bit k set = slot k in use.
template <int K>
__device__ __forceinline__ void lookup_plain_batch(const uint64_t (&key)[K], uint32_t valid, const KParams &p,
                                                   int64_t (&j)[K])
{
    uint32_t lo[K], hi[K], end[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (((valid >> k) & 1u) && key[k] <= p.maskN) {
            const uint64_t pf = key[k] >> (p.N - p.pbits);
            lo[k] = p.limits[pf];
            hi[k] = p.limits[pf + 1];
        } else {
            lo[k] = hi[k] = 0;
        }
        end[k] = hi[k];
    }
    for (;;) {
        uint64_t v[K];
        uint32_t mid[K];
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            mid[k] = (lo[k] + hi[k]) >> 1;
            if (lo[k] < hi[k]) {
                v[k] = p.reps[mid[k]];
                any = true;
            }
        }
        if (!any) break;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (lo[k] < hi[k]) {
                if (v[k] < key[k]) lo[k] = mid[k] + 1; else hi[k] = mid[k];
            }
    }
    uint64_t f[K];
#pragma unroll
    for (int k = 0; k < K; ++k) f[k] = (lo[k] < end[k]) ? p.reps[lo[k]] : ~key[k];
#pragma unroll
    for (int k = 0; k < K; ++k) j[k] = (lo[k] < end[k] && f[k] == key[k]) ? (int64_t)lo[k] : -1;
}

template <int K>
__device__ __forceinline__ void lookup_learned_batch(const uint64_t (&key)[K], uint32_t valid, const KParams &p,
                                                     const PwView &pw, int64_t (&j)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k)
        j[k] = ((valid >> k) & 1u) ? lookup_learned(key[k], p.reps, pw, static_cast<const Leaf *>(p.leaves), p.sub,
                                                    p.N, p.log2_leaves)
                                   : -1;
}

// Index of a representative: plain Limits + binary search, or the learned
// index (network in LDS, leaf table, bounded binary search).
template <bool LEARNED>
__device__ __forceinline__ int64_t lookup(uint64_t key, const KParams &p, const PwView &pw)
{
    if (LEARNED)
        return lookup_learned(key, p.reps, pw, static_cast<const Leaf *>(p.leaves), p.sub, p.N, p.log2_leaves);
    return lookup_plain(key, p);
}

// Amplitude <tau|H_pair|sigma> of the merged pieces flipping pair q of s
// (s antiparallel on the pair).  Real part: exchange J/2; imaginary part:
// chirality edges.
template <bool CPLX>
__device__ __forceinline__ void pair_amp(uint64_t s, const PairTerm &pt, const Lds &L, double &hre, double &him)
{
    hre = 0.5 * pt.Jsum;
    him = 0.0;
    if (CPLX) {
        for (int c = pt.chi_begin; c < pt.chi_end; ++c) {
            const ChiTerm ct = L.chis[c];
            him += (s & ct.site_bit) ? ct.c : -ct.c;
        }
        if (s & pt.lo_bit) him = -him;
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum: waves reduce by shuffles, wave results combined in
// a fixed order by thread 0.  `scratch` holds one double per wave.
__device__ __forceinline__ double block_sum(double v, double *scratch)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += scratch[k];
    return t;
}

constexpr int kBatch = SYMED_KBATCH;  // lookups in flight per lane

// Flush the pending (key, coefficient) slots: lookups in lockstep, then the
// gathers of x_j, accumulated oldest slot first (the order the pieces were
// generated), so the sum is the same as one piece at a time.
template <bool CPLX, bool LEARNED>
__device__ __forceinline__ void flush_batch(const uint64_t (&key)[kBatch], const double (&cr)[kBatch],
                                            const double (&ci)[kBatch], uint32_t valid, const KParams &p,
                                            const PwView &pw, const double *__restrict__ x, double &ar, double &ai)
{
    int64_t j[kBatch];
    if (LEARNED) lookup_learned_batch<kBatch>(key, valid, p, pw, j);
    else lookup_plain_batch<kBatch>(key, valid, p, j);
    double xr[kBatch], xi[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
        if (j[k] >= 0) {
            xr[k] = CPLX ? x[2 * j[k]] : x[j[k]];
            xi[k] = CPLX ? x[2 * j[k] + 1] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
        if (j[k] >= 0) {
            if (!CPLX) {
                ar += cr[k] * xr[k];
            } else {
                ar += cr[k] * xr[k] - ci[k] * xi[k];
                ai += cr[k] * xi[k] + ci[k] * xr[k];
            }
        }
    }
}

// One row of H.v: y_i = diag_i x_i + isq_i * sum over flipped pairs of
// coefficient * x_j (gather; only this lane writes y_i).  mode 0 writes
// y_i; mode 1 (real Lanczos) writes w_i = (H v)_i - beta w_i and returns
// w_i v_i; mode 2 (complex Lanczos) writes w_i = (H v)_i and returns
// Re(conj(w_i) v_i).
template <bool CPLX, int MODE, bool LEARNED>
__device__ __forceinline__ double apply_row(const KParams &p, const Lds &L, int64_t i, const double *__restrict__ x,
                                            double *__restrict__ y, double beta)
{
    const uint64_t s = p.reps[i];
    const double isq = L.isqrtt[p.stab[i]];
    double diag = 0.0, ar = 0.0, ai = 0.0;
    // pending pieces, oldest in slot 0
    uint64_t key[kBatch];
    double cr[kBatch], ci[kBatch];
    uint32_t valid = 0;
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
        key[k] = 0;
        cr[k] = ci[k] = 0.0;
    }
    // Pairs are taken in windows of 128: the antiparallel pairs of the window
    // are marked in a bit mask first (and the diagonal summed), then every
    // lane walks its own marked pairs in ascending order.  Lanes of a wave
    // thus stay busy while any lane has pairs left, instead of idling on the
    // parallel pairs of the others; the order of the terms is unchanged.
    for (int q0 = 0; q0 < p.n_pairs; q0 += 128) {
        const int qn = min(p.n_pairs - q0, 128);
        uint64_t m[2] = {0ull, 0ull};
        for (int q = 0; q < qn; ++q) {
            const PairTerm &pt = L.pairs[q0 + q];
            const bool anti = __popcll(s & pt.mask) == 1;
            diag += anti ? -0.25 * pt.Jsum : 0.25 * pt.Jsum;
            m[q >> 6] |= (uint64_t)anti << (q & 63);
        }
        for (int h = 0; h < 2; ++h) {
            uint64_t mm = m[h];
            while (mm) {
                const int q = q0 + 64 * h + __builtin_ctzll(mm);
                mm &= mm - 1;
                const PairTerm pt = L.pairs[q];
                double hre, him;
                pair_amp<CPLX>(s, pt, L, hre, him);
                if (hre == 0.0 && him == 0.0) continue;
                const Found f = find_rep(s ^ pt.mask, p, L);
                const double w = L.sqrtt[f.cnt];
                double kr, ki = 0.0;
                if (!CPLX) {
                    kr = L.chi[f.g] * w * hre;
                } else {
                    // chi(g) * w * conj(h)
                    const double c_r = L.chi[2 * f.g] * w, c_i = L.chi[2 * f.g + 1] * w;
                    kr = c_r * hre + c_i * him;
                    ki = c_i * hre - c_r * him;
                }
#pragma unroll
                for (int k = 0; k < kBatch - 1; ++k) {
                    key[k] = key[k + 1];
                    cr[k] = cr[k + 1];
                    ci[k] = ci[k + 1];
                }
                key[kBatch - 1] = f.rep;
                cr[kBatch - 1] = kr;
                ci[kBatch - 1] = ki;
                valid = (valid >> 1) | (1u << (kBatch - 1));
                if (valid & 1u) {
                    flush_batch<CPLX, LEARNED>(key, cr, ci, valid, p, L.pw, x, ar, ai);
                    valid = 0;
                }
            }
        }
    }
    if (valid) flush_batch<CPLX, LEARNED>(key, cr, ci, valid, p, L.pw, x, ar, ai);
    double part = 0.0;
    if (!CPLX) {
        const double xi = x[i];
        double yi = diag * xi + isq * ar;
        if (MODE == 1) {
            yi -= beta * y[i];
            part = yi * xi;
        }
        y[i] = yi;
    } else {
        const double xr = x[2 * i], xim = x[2 * i + 1];
        const double yr = diag * xr + isq * ar, yim = diag * xim + isq * ai;
        if (MODE == 2) part = yr * xr + yim * xim;
        y[2 * i] = yr;
        y[2 * i + 1] = yim;
    }
    return part;
}

}  // namespace symed
