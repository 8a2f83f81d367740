// Device-side pieces of the H.v gather shared by the single-sector and the
// batched (many sectors, one persistent launch) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.h"
#include "learned_dev.h"
#include "represent.h"

namespace symed {

// Block size of the H.v kernel (compile-time tuning knob).
#ifndef SYMED_APPLY_THREADS
#define SYMED_APPLY_THREADS 1024
#endif
constexpr int kApplyThreads = SYMED_APPLY_THREADS;

// Lookup kinds of the H.v gather.
constexpr int kLookupPlain = 0;    // Limits prefix map + binary search (the thesis's method)
constexpr int kLookupLearned = 1;  // learned index + bounded binary search
constexpr int kLookupHash = 2;     // hashed staging table of {rep, x} records

// Words per record of the hashed staging table and the empty-slot marker
// (no N-bit configuration with N < 64 equals it).
template <bool CPLX>
constexpr int hash_words() { return CPLX ? 4 : 2; }
constexpr uint64_t kHashEmpty = ~0ull;

// Home slot of a key: the 64-bit finalizer of MurmurHash3 (Appleby) as the
// mixing function, reduced to [0, slots) by a multiply-high.
__host__ __device__ __forceinline__ uint64_t hash_mix(uint64_t k)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ uint64_t hash_home(uint64_t key, uint64_t slots) { return __umul64hi(hash_mix(key), slots); }

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
    if (key > p.maskN) return -1;
    const uint64_t pf = key >> (p.N - p.pbits);
    uint32_t lo = p.limits[pf], hi = p.limits[pf + 1];
    const uint32_t end = hi;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (p.reps[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < end && p.reps[lo] == key) ? (int64_t)lo : -1;
}

// Index of a representative (ed_lookup): plain Limits + binary search, or the learned
// index (network and rank table in LDS, segment and cell tables, bounded search).
template <bool LEARNED>
__device__ __forceinline__ int64_t lookup(uint64_t key, const KParams &p, const LearnedLds &li)
{
    if (LEARNED) return lookup_learned(key, p.reps, p.lv, li, p.N, p.n_up);
    return lookup_plain(key, p);
}

// Record of key in the hashed staging table: linear probing from the home
// slot until the key or an empty slot (absent: -1).  The table always has
// an empty slot, so the probe ends.
template <bool CPLX>
__device__ __forceinline__ int64_t hash_find(uint64_t key, const KParams &p)
{
    constexpr int S = hash_words<CPLX>();
    uint64_t s = hash_home(key, p.hslots);
    for (;;) {
        const uint64_t k = p.htab[s * S];
        if (k == key) return (int64_t)s;
        if (k == kHashEmpty) return -1;
        if (++s == p.hslots) s = 0;
    }
}

// x of key from the hashed staging table; false if the key is absent.  Each
// probe reads the whole record (16 B, or both 16 B halves of a complex
// record at once), so x arrives with the key that confirms it and is not
// fetched again after the line may have left the caches.
template <bool CPLX>
__device__ __forceinline__ bool hash_get(uint64_t key, const KParams &p, double &xr, double &xi)
{
    const uint4 *rec = reinterpret_cast<const uint4 *>(p.htab);
    uint64_t s = hash_home(key, p.hslots);
    for (;;) {
        uint4 a = rec[CPLX ? 2 * s : s];
        uint4 b = make_uint4(0u, 0u, 0u, 0u);
        if (CPLX) b = rec[2 * s + 1];
        // The record's words pass through an empty statement (no code), so
        // the compiler issues the whole record as one load instead of
        // deferring the x words to a second load after the key compare.
        asm("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
        if (CPLX) asm("" : "+v"(b.x), "+v"(b.y));
        const uint64_t k = ((uint64_t)a.y << 32) | a.x;
        if (k == key) {
            xr = __hiloint2double((int)a.w, (int)a.z);
            if (CPLX) xi = __hiloint2double((int)b.y, (int)b.x);
            return true;
        }
        if (k == kHashEmpty) return false;
        if (++s == p.hslots) s = 0;
    }
}

// x of key through the learned index over the records {rep, x} kept in
// basis order (real sectors): the search in the recorded window starts at
// the predicted record, which is read whole, so when the prediction is exact
// x comes with the key that confirms it; otherwise the search compares
// record keys and the record it ends on is read whole.  false if absent.
// Targets of H.v are sector configurations (n_up up spins below bit N).
__device__ __forceinline__ bool learned_get(uint64_t key, const KParams &p, const Lds &L, double &xr)
{
    uint32_t pred, lo, hi;
    if (!learned_window(key, p.lv, L.li, pred, lo, hi)) return false;
    const uint4 *rec = reinterpret_cast<const uint4 *>(p.lrec);
    uint4 a = rec[pred];
    // whole-record load (see hash_get)
    asm("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
    uint64_t k = ((uint64_t)a.y << 32) | a.x;
    if (k != key) {
        uint32_t lo2 = lo, hi2 = hi + 1u;   // half-open
        if (k < key) lo2 = pred + 1u; else hi2 = pred;
        while (lo2 < hi2) {
            const uint32_t mid = (lo2 + hi2) >> 1;
            if (p.lrec[(uint64_t)mid * 2] < key) lo2 = mid + 1u; else hi2 = mid;
        }
        if (lo2 > hi) return false;
        a = rec[lo2];
        asm("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
        k = ((uint64_t)a.y << 32) | a.x;
        if (k != key) return false;
    }
    xr = __hiloint2double((int)a.w, (int)a.z);
    return true;
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

// One row of H.v: y_i = diag_i x_i + isq_i * sum over flipped pairs of
// coefficient * x_j (gather; only this lane writes y_i).  mode 0 writes
// y_i; mode 1 (real Lanczos) writes w_i = (H v)_i - beta w_i and returns
// w_i v_i; mode 2 (complex Lanczos) writes w_i = (H v)_i and returns
// Re(conj(w_i) v_i).  LK: kLookupPlain finds j and reads x_j from x;
// kLookupHash finds the record of the target in the hashed staging table,
// and kLookupLearned (real sectors) in the records kept in basis order; the
// record's copy of x_j sits beside the key that confirms the match.  Complex
// sectors search the learned index over the representatives and read x_j
// from x: their 32 B records would spread the search over 4x the lines.
template <bool CPLX, int MODE, int LK>
__device__ __forceinline__ double apply_row(const KParams &p, const Lds &L, int64_t i, const double *__restrict__ x,
                                            double *__restrict__ y, double beta)
{
    const uint64_t s = p.reps[i];
    const double isq = L.isqrtt[p.stab[i]];
    double diag = 0.0, ar = 0.0, ai = 0.0;
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
                double xr, xi = 0.0;
                if (LK == kLookupHash) {
                    if (!hash_get<CPLX>(f.rep, p, xr, xi)) continue;
                } else if (LK == kLookupLearned && !CPLX) {
                    if (!learned_get(f.rep, p, L, xr)) continue;
                } else {
                    const int64_t j = lookup<LK == kLookupLearned>(f.rep, p, L.li);
                    if (j < 0) continue;
                    xr = CPLX ? x[2 * j] : x[j];
                    if (CPLX) xi = x[2 * j + 1];
                }
                const double w = L.sqrtt[f.cnt];
                if (!CPLX) {
                    const double kr = L.chi[f.g] * w * hre;
                    ar += kr * xr;
                } else {
                    // chi(g) * w * conj(h)
                    const double c_r = L.chi[2 * f.g] * w, c_i = L.chi[2 * f.g + 1] * w;
                    const double kr = c_r * hre + c_i * him;
                    const double ki = c_i * hre - c_r * him;
                    ar += kr * xr - ki * xi;
                    ai += kr * xi + ki * xr;
                }
            }
        }
    }
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
