// Device side of SU(d) permutation models (d <= 4 colors, two bits per site):
// the color-count sector in ascending order, and one row of H.v.
//
// Model (thesis, chapter on SU(N) chiral spin liquids): H = J sum P_ij +
// i K sum (P_ijk - P_ijk^-1), where P_ij exchanges the colors of two sites and
// P_ijk moves the color of i to j, of j to k and of k to i.  Every term maps a
// configuration to one configuration (a non-branching term in the sense of
// section "Computations in the symmetrized basis"), so the gather of the
// spin-1/2 case carries over with moves in place of flipped pairs.
#pragma once

#include <hip/hip_runtime.h>

#include "apply_dev.h"

namespace symed {

// Color-count sector: n sites, d colors, cnt[c] sites of color c.
struct ColorSector {
    int n, d;
    int cnt[4];
};

constexpr uint64_t kNoConfig = ~0ull;

// Smallest configuration >= t of the sector (digits < d with the sector's
// color counts), kNoConfig if none.  Keys compare like the digit strings read
// from site 0, so this is the next multiset permutation in lexicographic
// order: t's digits are taken while they fit the remaining counts; at the
// first that does not (or, moving back, at an earlier position) the smallest
// larger color still available is placed and the rest filled in ascending
// order.
__host__ __device__ __forceinline__ uint64_t color_next(uint64_t t, const ColorSector &cs)
{
    const int n = cs.n;
    if (t >> (2 * n)) return kNoConfig;
    int rem[4] = {cs.cnt[0], cs.cnt[1], cs.cnt[2], cs.cnt[3]};
    int i = 0;
    for (; i < n; ++i) {
        const int dg = (int)(t >> (2 * (n - 1 - i))) & 3;
        if (dg >= cs.d || rem[dg] == 0) break;
        --rem[dg];
    }
    if (i == n) return t;
    for (int q = i; q >= 0; --q) {
        const int dg = (int)(t >> (2 * (n - 1 - q))) & 3;
        if (q < i) ++rem[dg];
        for (int c = dg + 1; c < cs.d; ++c) {
            if (rem[c] == 0) continue;
            uint64_t r = (t >> (2 * (n - q))) << (2 * (n - q));  // digits above q (2n <= 62)
            --rem[c];
            r |= (uint64_t)c << (2 * (n - 1 - q));
            int pos = q + 1;
            for (int cc = 0; cc < cs.d; ++cc)
                for (int k = 0; k < rem[cc]; ++k, ++pos) r |= (uint64_t)cc << (2 * (n - 1 - pos));
            return r;
        }
    }
    return kNoConfig;
}

// r-th (0-based) configuration of the sector in ascending order; total =
// number of configurations (multinomial n! / prod cnt[c]!).  The completions
// of a prefix with counts rem number M = (n-i)! / prod rem!, and those that
// place color c next number M rem[c] / (n-i), an exact integer (the host keeps
// total * n below 2^64).
__host__ __device__ __forceinline__ uint64_t color_unrank(uint64_t r, uint64_t total, const ColorSector &cs)
{
    const int n = cs.n;
    int rem[4] = {cs.cnt[0], cs.cnt[1], cs.cnt[2], cs.cnt[3]};
    uint64_t M = total, s = 0;
    for (int i = 0; i < n; ++i) {
        const uint64_t left = (uint64_t)(n - i);
        for (int c = 0; c < cs.d; ++c) {
            if (rem[c] == 0) continue;
            const uint64_t Mc = M * (uint64_t)rem[c] / left;
            if (r < Mc) {
                s |= (uint64_t)c << (2 * (n - 1 - i));
                --rem[c];
                M = Mc;
                break;
            }
            r -= Mc;
        }
    }
    return s;
}

// Configuration that move mv makes of s.
__host__ __device__ __forceinline__ uint64_t move_target(uint64_t s, const ColorMove &mv)
{
    const uint64_t a = (s >> mv.sh[0]) & 3u, b = (s >> mv.sh[1]) & 3u;
    if (mv.kind == 0) {
        const uint64_t x = a ^ b;
        return s ^ (x << mv.sh[0]) ^ (x << mv.sh[1]);
    }
    const uint64_t c = (s >> mv.sh[2]) & 3u;
    // kind 1: site 0 gets c, site 1 gets a, site 2 gets b; kind 2 the inverse
    const bool f = mv.kind == 1;
    const uint64_t n0 = f ? c : b, n1 = f ? a : c, n2 = f ? b : a;
    return s ^ ((a ^ n0) << mv.sh[0]) ^ ((b ^ n1) << mv.sh[1]) ^ ((c ^ n2) << mv.sh[2]);
}

// <t|H_move|s> for a move that changes s.
__host__ __device__ __forceinline__ void move_amp(const ColorMove &mv, double &hre, double &him)
{
    hre = mv.kind == 0 ? mv.amp : 0.0;
    him = mv.kind == 1 ? mv.amp : (mv.kind == 2 ? -mv.amp : 0.0);
}

// One row of H.v for an SU(d) model; modes, lookups and the write of y_i as
// in apply_row of the spin-1/2 case.  Moves are taken in windows of 128: the
// moves that change s are marked first (the exchanges that do not change it
// summed into the diagonal), then every lane walks its marked moves in
// ascending order, so the lanes of a wave stay busy together.
template <bool CPLX, int MODE, int LK>
__device__ __forceinline__ double apply_row_colors(const KParams &p, const Lds &L, int64_t i,
                                                   const double *__restrict__ x, double *__restrict__ y, double beta)
{
    const uint64_t s = p.reps[i];
    const double isq = L.isqrtt[p.stab[i]];
    double diag = 0.0, ar = 0.0, ai = 0.0;
    for (int q0 = 0; q0 < p.n_moves; q0 += 128) {
        const int qn = min(p.n_moves - q0, 128);
        uint64_t m[2] = {0ull, 0ull};
        for (int q = 0; q < qn; ++q) {
            const ColorMove mv = L.moves[q0 + q];
            const bool act = move_target(s, mv) != s;
            if (!act && mv.kind == 0) diag += mv.amp;
            m[q >> 6] |= (uint64_t)act << (q & 63);
        }
        for (int h = 0; h < 2; ++h) {
            uint64_t mm = m[h];
            while (mm) {
                const int q = q0 + 64 * h + __builtin_ctzll(mm);
                mm &= mm - 1;
                const ColorMove mv = L.moves[q];
                const Found f = find_rep(move_target(s, mv), p, L);
                double xr, xi = 0.0;
                if (LK == kLookupHash) {
                    if (!hash_get<CPLX>(f.rep, p, xr, xi)) continue;
                } else {
                    const int64_t j = lookup_plain(f.rep, p);
                    if (j < 0) continue;
                    xr = CPLX ? x[2 * j] : x[j];
                    if (CPLX) xi = x[2 * j + 1];
                }
                double hre, him;
                move_amp(mv, hre, him);
                const double w = L.sqrtt[f.cnt];
                if (!CPLX) {
                    ar += L.chi[f.g] * w * hre * xr;
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
