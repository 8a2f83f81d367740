// Sublattice-coded representative search (host and device).
//
// Shared by the H.v and enumeration kernels; also compiled for the host so
// the same code can be checked against brute force on the CPU.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "learned_dev.h"

namespace symed {

struct Lds {
    const uint2 *rent;          // per coarse substate: {Rep | count << 16, first Sym entry}
    const uint16_t *symlist;    // symmetry codes (sp << 1) | flip
    const uint16_t *atab;   // distinct SymmetryAction tables, 2^ba entries each
    const uint32_t *aent;   // [n_sp][2^aent_lg >= A]: (byte offset of the table in atab << 8) | shift of the source substate
    uint32_t aent_lg;
    const PairTerm *pairs;
    const ChiTerm *chis;
    const double *chi;
    const double *sqrtt;
    const double *isqrtt;
    const uint8_t *chione;
    const ColorMove *moves;  // SU(d) models
    LearnedLds li;  // learned index: network pieces, equalizer, rank table
};

// Views of the tables: b is the staged blob (LDS), g the buffer that holds
// the Rep/Sym tables when they are too large for LDS (L.rep_global).
// RG = 0: the Rep/Sym tables are in the blob (L.rep_global must be 0), so
// every pointer derives from b and the compiler issues LDS reads for them;
// RG = 1: decided from L.rep_global at run time (generic pointers, flat
// loads).
template <int RG>
__host__ __device__ __forceinline__ Lds lds_view_t(const unsigned char *b, const BlobLayout &L,
                                                   const unsigned char *g)
{
    Lds v;
    if (RG && L.rep_global) {
        v.rent = reinterpret_cast<const uint2 *>(g + L.g_rent);
        v.symlist = reinterpret_cast<const uint16_t *>(g + L.g_symlist);
    } else {
        v.rent = reinterpret_cast<const uint2 *>(b + L.off_rent);
        v.symlist = reinterpret_cast<const uint16_t *>(b + L.off_symlist);
    }
    v.atab = reinterpret_cast<const uint16_t *>(b + L.off_atab);
    v.aent = reinterpret_cast<const uint32_t *>(b + L.off_aent);
    v.aent_lg = L.aent_lg;
    v.pairs = reinterpret_cast<const PairTerm *>(b + L.off_pairs);
    v.chis = reinterpret_cast<const ChiTerm *>(b + L.off_chis);
    v.chi = reinterpret_cast<const double *>(b + L.off_chi);
    v.sqrtt = reinterpret_cast<const double *>(b + L.off_sqrt);
    v.isqrtt = reinterpret_cast<const double *>(b + L.off_isqrt);
    v.chione = b + L.off_chione;
    v.moves = reinterpret_cast<const ColorMove *>(b + L.off_moves);
    v.li = learned_lds(b, L.off_mlp, L.off_rank);
    return v;
}

__host__ __device__ __forceinline__ Lds lds_view(const unsigned char *b, const BlobLayout &L,
                                                 const unsigned char *g = nullptr)
{
    return lds_view_t<1>(b, L, g);
}

// Substate that a symmetry puts at fine destination d of the configuration
// t (spin flip not applied); en: the symmetry's A entries, each the byte
// offset of its table in atab (<< 8) and the right shift that brings the
// source substate of t to the low bits.
__host__ __device__ __forceinline__ uint32_t act_image(const uint32_t *en, const uint16_t *atab, uint64_t t, int d,
                                                      uint32_t ma)
{
    const uint32_t ent = en[d];
    const uint32_t ss = (uint32_t)(t >> (ent & 63u)) & ma;
    return *reinterpret_cast<const uint16_t *>(reinterpret_cast<const unsigned char *>(atab) + (ent >> 8) + 2u * ss);
}

struct Found {
    uint64_t rep;
    uint32_t g;    // code (sp << 1) | flip of a symmetry reaching the representative
    uint32_t cnt;  // number of group elements reaching the representative = |Stab|
};

// Candidate scan of find_rep in words of type V.  Every candidate maps its
// sublattice onto the most significant coarse sublattice with image MinRep,
// so the fine destinations 0..d0-1 agree for all candidates; images are
// compared from destination d0 on and a candidate is dropped at the first
// destination where it exceeds the best so far.  V = uint64_t carries the
// MinRep prefix in the image; V = uint32_t (when the W = (A - d0) * ba bits
// from destination d0 on number at most 31) carries only those bits, with
// the all-ones start value above every image, and the prefix is put back at
// the end.
template <typename V>
__host__ __device__ __forceinline__ Found scan_candidates(uint64_t t, const KParams &p, const Lds &L, uint32_t minrep,
                                                          uint32_t xm, uint2 e0)
{
    const int N = p.N, R = p.R, br = p.br, A = p.A, ba = p.ba;
    const uint32_t S = 1u << br, mr = S - 1u, ma = (1u << ba) - 1u;
    const int d0 = A / R;
    const V start = sizeof(V) == 8 ? (V)minrep : (V)0;
    V best = ~(V)0;
    uint32_t bg = 0, cnt = 0;
    bool first = true;
    while (xm) {
        const int X = __builtin_ctz(xm);
        xm &= xm - 1u;
        uint2 e = e0;
        if (!first) {
            const uint32_t s = (uint32_t)(t >> (N - (X + 1) * br)) & mr;
            e = L.rent[X * S + s];
        }
        first = false;
        const uint32_t k1 = e.y + (e.x >> 16);
        for (uint32_t k = e.y; k < k1; ++k) {
            const uint32_t e = L.symlist[k];
            const uint32_t sp = e >> 1;
            const uint32_t fm = (e & 1u) ? ma : 0u;  // spin flip complements every substate
            const uint32_t *en = L.aent + ((size_t)sp << L.aent_lg);
            V v = start;
            V bp = 0;
            int d = d0;
            for (; d < A; ++d) {
                v = (v << ba) | (V)(act_image(en, L.atab, t, d, ma) ^ fm);
                bp = best >> ((A - 1 - d) * ba);
                if (v != bp) break;
            }
            if (d == A) {
                // no destination differed: the same image as the best so far,
                // or (one fine sublattice, d0 == A) the first candidate
                if (v == best) {
                    ++cnt;
                } else {
                    best = v;
                    bg = e;
                    cnt = 1;
                }
                continue;
            }
            if (v > bp) continue;
            for (++d; d < A; ++d) v = (v << ba) | (V)(act_image(en, L.atab, t, d, ma) ^ fm);
            best = v;
            bg = e;
            cnt = 1;
        }
    }
    const uint64_t rep = sizeof(V) == 8 ? (uint64_t)best : (((uint64_t)minrep << ((A - d0) * ba)) | (uint64_t)best);
    return Found{rep, bg, cnt};
}

// Representative of t by sublattice coding (algorithm "Sublattice coding
// algorithm for finding the representative"): MinRep over the coarse
// sublattices, then every symmetry in Sym_Y of each sublattice Y attaining
// MinRep is applied through the SymmetryAction tables of the fine
// decomposition (destination-major, so the image is assembled most
// significant sublattice first).  All minimizers lie among these candidates
// and each group element is a candidate at most once, so the number of
// candidates reaching the minimum is the stabilizer size.
__host__ __device__ __forceinline__ Found find_rep(uint64_t t, const KParams &p, const Lds &L)
{
    const int N = p.N, R = p.R, br = p.br;
    const uint32_t S = 1u << br, mr = S - 1u;
    // MinRep, and in xm the coarse sublattices that attain it (R <= 16); e0
    // keeps the entry of the first of them
    uint32_t minrep = 0xffffffffu, xm = 0;
    uint2 e0 = make_uint2(0u, 0u);
    for (int X = 0; X < R; ++X) {
        uint32_t s = (uint32_t)(t >> (N - (X + 1) * br)) & mr;
        const uint2 e = L.rent[X * S + s];
        const uint32_t r = e.x & 0xffffu;
        if (r < minrep) {
            minrep = r;
            xm = 1u << X;
            e0 = e;
        } else if (r == minrep) {
            xm |= 1u << X;
        }
    }
    if ((p.A - p.A / R) * p.ba <= 31) return scan_candidates<uint32_t>(t, p, L, minrep, xm, e0);
    return scan_candidates<uint64_t>(t, p, L, minrep, xm, e0);
}

// Enumeration tests (algorithm "Preparation of the distributed and
// symmetrized Hilbert space"): the first coarse sublattice X at which s fails
// the prefix test of a representative, or -1.  The identity is in G_0, so a
// representative has Rep_0(s_0) = s_0 and Rep_X(s_X) >= s_0 for every coarse
// sublattice X; a failed test on X rejects every configuration that shares
// sublattices 0..X with s.
__host__ __device__ __forceinline__ int rep_prefix_fail(uint64_t s, const KParams &p, const Lds &L)
{
    const int N = p.N, R = p.R, br = p.br;
    const uint32_t S = 1u << br, mr = S - 1u;
    const uint32_t s0 = (uint32_t)(s >> (N - br)) & mr;
    if ((L.rent[s0].x & 0xffffu) != s0) return 0;
    for (int X = 1; X < R; ++X) {
        const uint32_t sx = (uint32_t)(s >> (N - (X + 1) * br)) & mr;
        if ((L.rent[X * S + sx].x & 0xffffu) < s0) return X;
    }
    return -1;
}

// Full test of a configuration that passed the prefix test: every symmetry
// of Sym_Y of a coarse sublattice Y with Rep_Y(s_Y) = s_0 is applied; s is a
// representative iff no image is smaller.  stab counts the images equal to
// s (the stabilizer), triv is false if chi is not 1 on one of them.
__host__ __device__ __forceinline__ bool rep_check(uint64_t s, const KParams &p, const Lds &L, uint32_t &stab,
                                                   bool &triv)
{
    const int N = p.N, R = p.R, br = p.br, A = p.A, ba = p.ba;
    const uint32_t S = 1u << br, mr = S - 1u, ma = (1u << ba) - 1u;
    const uint32_t s0 = (uint32_t)(s >> (N - br)) & mr;
    stab = 0;
    triv = true;
    for (int Y = 0; Y < R; ++Y) {
        const uint32_t sy = (uint32_t)(s >> (N - (Y + 1) * br)) & mr;
        const uint2 e = L.rent[Y * S + sy];
        if ((e.x & 0xffffu) != s0) continue;
        const uint32_t k1 = e.y + (e.x >> 16);
        for (uint32_t q = e.y; q < k1; ++q) {
            const uint32_t c = L.symlist[q];
            const uint32_t *en = L.aent + ((size_t)(c >> 1) << L.aent_lg);
            uint64_t v = 0;
            for (int d = 0; d < A; ++d) v = (v << ba) | act_image(en, L.atab, s, d, ma);
            if (c & 1u) v ^= p.maskN;
            if (v < s) return false;
            if (v == s) {
                ++stab;
                if (!L.chione[c]) triv = false;
            }
        }
    }
    return true;
}

}  // namespace symed
