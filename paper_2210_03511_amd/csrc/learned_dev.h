// Device-side learned index: the network evaluation and the bounded search.
// Shared by the index build (learned.hip) and by H.v / lookup (kernels.hip):
// both must evaluate the network bit-identically, since the recorded error
// bounds are only valid for exactly the same arithmetic.  Every floating
// point step is an explicit fmaf / fmaxf, and contraction is switched off.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace symed {

constexpr int kMaxFeatures = 8;
constexpr int kHidden = 32;
constexpr int kMlpMaxParams = kHidden * kMaxFeatures + kHidden + kHidden * kHidden + kHidden + kHidden + 1;

// Parameter layout (floats): W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3.
__host__ __device__ inline int mlp_param_count(int F, int H) { return H * F + H + H * H + H + H + 1; }

// Rank of a configuration among all N-bit configurations with the same
// number k of up spins, in ascending integer order (combinatorial number
// system): with the set bits at positions p_0 < p_1 < ... < p_{k-1},
// rank = sum_j C(p_j, j + 1).  The j-th set bit lies in [j, j + N - k], so
// the table holds C(p, j + 1) at j * W + (p - j), W = N - k + 1 (k rows).
// The key must have exactly k set bits below bit N.  Every key takes k steps.
__host__ __device__ __forceinline__ uint64_t sz_rank(uint64_t key, const uint64_t *binom, int W)
{
    uint64_t r = 0;
    int j = 0;
    while (key) {
        const int pos = __builtin_ctzll(key);
        key &= key - 1;
        r += binom[j * W + (pos - j)];
        ++j;
    }
    return r;
}

// Entries of the rank table (at most 32 * 33 for N < 64).
__host__ __device__ inline int rank_table_entries(int N, int n_up) { return n_up * (N - n_up + 1); }
constexpr int kRankMaxEntries = 32 * 33;

// Input of the network: the rank equalized by the monotone piecewise-linear
// map through K + 1 rank quantiles of the basis (knot j = rank of the key at
// position floor(j (dim - 1) / K)):
//   u = (j + (rank - knot_j) / (knot_{j+1} - knot_j)) / K  for knot_j <= rank < knot_{j+1},
// 0 below the first knot and 1 from the last one on.  Computed in float64
// from the exact rank, then rounded to float32; non-decreasing in the key.
// The representatives' ranks are far from uniform (whole ranges of leading
// substates hold none), which a 32-unit network cannot follow; after this
// normalization it models what is left.
constexpr int kEqMax = 64;   // largest K
// bytes of the equalizer in the LDS blob: knots, then inverse widths
constexpr int kEqBytes = ((2 * kEqMax + 1) * 8 + 15) & ~15;
struct Equalizer {
    const uint64_t *knot;    // K + 1 ascending ranks
    const double *invw;      // 1 / (knot_{j+1} - knot_j), K entries
    int K;
    double invK;             // 1 / K
};

__host__ __device__ __forceinline__ float equalize(uint64_t rank, const Equalizer &e)
{
#pragma clang fp contract(off)
    if (rank <= e.knot[0]) return 0.0f;
    if (rank >= e.knot[e.K]) return 1.0f;
    int lo = 0, hi = e.K - 1;  // the piece j with knot_j <= rank < knot_{j+1}
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (e.knot[mid] <= rank) lo = mid; else hi = mid - 1;
    }
    const double f = (double)(rank - e.knot[lo]) * e.invw[lo];
    return (float)(((double)lo + f) * e.invK);
}

// Hidden activation of unit j: the first half of each hidden layer uses
// relu(z) (convex), the second half min(z, 0) (concave).  Both are
// non-decreasing, so with non-negative weights the network is a
// non-decreasing function of its input, and the mix lets it bend both ways.
__host__ __device__ __forceinline__ float hidden_act(float z, int j)
{
    return (j < kHidden / 2) ? fmaxf(z, 0.0f) : fminf(z, 0.0f);
}

// y = W3 act(W2 act(W1 x + b1) + b2) + b3, fixed evaluation order.
__device__ __forceinline__ float mlp_eval(const float *__restrict__ P, int F, const float *x)
{
#pragma clang fp contract(off)
    const int H = kHidden;
    const float *W1 = P, *b1 = P + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;
    float h1[kHidden];
#pragma unroll
    for (int j = 0; j < kHidden; ++j) {
        float a = b1[j];
        for (int f = 0; f < F; ++f) a = fmaf(W1[j * F + f], x[f], a);
        h1[j] = hidden_act(a, j);
    }
    float y = b3[0];
#pragma unroll 4
    for (int k = 0; k < kHidden; ++k) {
        float a = b2[k];
#pragma unroll
        for (int j = 0; j < kHidden; ++j) a = fmaf(W2[k * H + j], h1[j], a);
        y = fmaf(W3[k], hidden_act(a, k), y);
    }
    return y;
}

// The network has one input, so it is a piecewise-linear function of u with
// at most kPwMax pieces.  After training the host expands it exactly (in
// float64) into breakpoints brk[0..n-2] (ascending) and per-piece values
// y = fmaf(slope[i], u, icpt[i]) for piece i = number of breakpoints <= u.
// The index build and every lookup evaluate the network through this
// expansion, so their arithmetic is identical.  Block layout (floats):
// header (n, 3 unused), brk[n], slope[n], icpt[n] (brk[n-1] unused), so a
// block takes 4 + 3n floats.
constexpr int kPwMax = kHidden + kHidden * (kHidden + 1) + 2;
constexpr int kPwHeader = 4;

struct PwView {
    int n;                  // pieces
    const float *brk;       // n - 1 breakpoints
    const float *slope;     // n
    const float *icpt;      // n
};

__device__ __forceinline__ float pw_eval(const PwView &w, float u)
{
#pragma clang fp contract(off)
    int lo = 0, hi = w.n - 1;  // piece index in [0, n-1]
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u < w.brk[mid]) hi = mid; else lo = mid + 1;
    }
    return fmaf(w.slope[lo], u, w.icpt[lo]);
}

__host__ __device__ __forceinline__ PwView pw_view(const float *base)
{
    PwView w;
    w.n = (int)base[0];
    w.brk = base + kPwHeader;
    w.slope = base + kPwHeader + w.n;
    w.icpt = base + kPwHeader + 2 * w.n;
    return w;
}

// floats of an expansion block with n pieces, and of the largest one
__host__ __device__ constexpr int pw_floats(int n) { return kPwHeader + 3 * n; }
constexpr int kPwFloats = pw_floats(kPwMax);

// The index below the network.  The network output y in [0, 1) picks one
// of 2^lg segments.  A segment maps the rank of a key linearly onto its
// cells (cells are allocated in proportion to the keys the network routes to
// the segment): cell c = floor(t), t = (rank - r0) * scale, and the fraction
// t - c places the key inside the cell.  A cell covers the positions
// [first, first + n) of the keys routed to it and predicts position
// first + floor((t - c) * n); elo and ehi are its recorded largest errors
// below and above the prediction (63: unbounded, the whole cell), so every
// key routed to the cell lies in [pred - elo, pred + ehi].
struct Seg {
    uint64_t r0;      // smallest rank routed here
    float scale;      // cells per unit of rank
    uint32_t cell0;   // first cell of the segment
};

constexpr uint32_t kCellNBits = 20;            // positions covered by a cell, < 2^20
constexpr uint32_t kCellErrSat = 63;           // saturated error: search the whole cell
__host__ __device__ __forceinline__ uint32_t cell_meta(uint32_t n, uint32_t elo, uint32_t ehi)
{
    const uint32_t a = elo < kCellErrSat ? elo : kCellErrSat, b = ehi < kCellErrSat ? ehi : kCellErrSat;
    return n | (a << kCellNBits) | (b << (kCellNBits + 6));
}

// Segment of a network output; the index is clamped as an integer: for
// 2^m >= 2^24 the float value of (2^m - 0.5) rounds up to 2^m.
__host__ __device__ __forceinline__ uint32_t seg_of(float y, int lg)
{
#pragma clang fp contract(off)
    const uint32_t Mi = 1u << lg;
    const float M = (float)Mi;
    float u = y * M;
    u = fminf(fmaxf(u, 0.0f), M);  // fmaxf also maps NaN to 0
    uint32_t b = (uint32_t)floorf(u);
    return b > Mi - 1u ? Mi - 1u : b;
}

// Cell of a rank in its segment (global cell number, clamped to the table)
// and the position of the key inside the cell, in [0, 1).  false: the rank
// lies below every key routed to the segment (absent).
__host__ __device__ __forceinline__ bool cell_of(uint64_t rank, const Seg &S, uint64_t n_cells, uint64_t &ci,
                                                double &frac)
{
#pragma clang fp contract(off)
    if (rank < S.r0) return false;
    const double t = (double)(rank - S.r0) * (double)S.scale;
    const double c = floor(t);
    const uint64_t cc = c < 4.0e9 ? (uint64_t)c : (uint64_t)4000000000ull;
    const uint64_t g = (uint64_t)S.cell0 + cc;
    ci = g < n_cells ? g : n_cells - 1;
    frac = t - c;
    return true;
}

// Offset of the predicted position inside a cell of n positions.
__host__ __device__ __forceinline__ uint32_t cell_offset(uint32_t n, double frac)
{
#pragma clang fp contract(off)
    const uint32_t off = (uint32_t)(frac * (double)n);
    return off > n - 1u ? n - 1u : off;
}

// Prediction and recorded window of a cell for a key at fraction frac.
__host__ __device__ __forceinline__ void cell_window(uint2 C, double frac, uint32_t &pred, uint32_t &lo, uint32_t &hi)
{
    const uint32_t n = C.y & ((1u << kCellNBits) - 1u);
    const uint32_t elo = (C.y >> kCellNBits) & 63u, ehi = C.y >> (kCellNBits + 6);
    const uint32_t off = cell_offset(n, frac);
    pred = C.x + off;
    lo = (elo == kCellErrSat || elo > off) ? C.x : pred - elo;
    hi = (ehi == kCellErrSat || ehi > n - 1u - off) ? C.x + n - 1u : pred + ehi;
}

// The network input as the index build sees it (rank table and equalizer
// in device memory).
struct RankFeat {
    const uint64_t *binom;   // rank table
    int W, n_up;
    Equalizer eq;
};

// Everything the learned lookup reads besides the LDS-staged network and
// rank table.
struct LearnedView {
    const Seg *segs;
    const uint2 *cells;
    uint64_t n_cells;
    int lg;          // log2 of the segment count
    int rk_W;        // rank table width
    int eq_K;        // equalizer pieces
    double eq_invK;
};

// The learned index's pieces in LDS: network expansion, equalizer and rank
// table, laid out at off_mlp as [pieces][equalizer, kEqBytes][rank table];
// at most kLearnedLdsMax bytes.
constexpr int kLearnedLdsMax = ((kPwFloats * 4 + 15) & ~15) + kEqBytes + kRankMaxEntries * 8;
struct LearnedLds {
    PwView pw;
    const uint64_t *knot;
    const double *invw;
    const uint64_t *rbinom;
};

__host__ __device__ __forceinline__ LearnedLds learned_lds(const unsigned char *blob, uint32_t off_mlp,
                                                         uint32_t off_eq)
{
    LearnedLds l;
    l.pw = pw_view(reinterpret_cast<const float *>(blob + off_mlp));
    l.knot = reinterpret_cast<const uint64_t *>(blob + off_eq);
    l.invw = reinterpret_cast<const double *>(blob + off_eq + (kEqMax + 1) * 8);
    l.rbinom = reinterpret_cast<const uint64_t *>(blob + off_eq + kEqBytes);
    return l;
}

// Window of the learned lookup: rank -> equalizer -> network -> segment ->
// cell -> prediction and recorded error.  false: absent without a search.
__device__ __forceinline__ bool learned_window(uint64_t key, const LearnedView &v, const LearnedLds &li,
                                               uint32_t &pred, uint32_t &lo, uint32_t &hi)
{
    const uint64_t rank = sz_rank(key, li.rbinom, v.rk_W);
    const Equalizer eq{li.knot, li.invw, v.eq_K, v.eq_invK};
    const float y = pw_eval(li.pw, equalize(rank, eq));
    const Seg S = v.segs[seg_of(y, v.lg)];
    uint64_t ci;
    double frac;
    if (!cell_of(rank, S, v.n_cells, ci, frac)) return false;
    const uint2 C = v.cells[ci];
    if ((C.y & ((1u << kCellNBits) - 1u)) == 0u) return false;
    cell_window(C, frac, pred, lo, hi);
    return true;
}

// Position of key among the sorted keys (stride S words: the representatives
// themselves, or {rep, x} records), searched in the window [lo, hi] starting
// at the prediction; -1 if absent.
template <int S>
__device__ __forceinline__ int64_t window_search(uint64_t key, const uint64_t *__restrict__ keys, uint32_t pred,
                                                 uint32_t lo, uint32_t hi)
{
    const uint64_t k0 = keys[(uint64_t)pred * S];
    if (k0 == key) return (int64_t)pred;
    uint32_t a = lo, b = hi + 1u;    // half-open [a, b)
    if (k0 < key) a = pred + 1u; else b = pred;
    while (a < b) {
        const uint32_t mid = (a + b) >> 1;
        if (keys[(uint64_t)mid * S] < key) a = mid + 1u; else b = mid;
    }
    return (a <= hi && keys[(uint64_t)a * S] == key) ? (int64_t)a : -1;
}

// Learned lookup of a position over the representatives; -1 if absent.
__device__ __forceinline__ int64_t lookup_learned(uint64_t key, const uint64_t *__restrict__ reps,
                                                 const LearnedView &v, const LearnedLds &li, int N, int n_up)
{
    if (__popcll(key) != n_up || (N < 64 && (key >> N))) return -1;
    uint32_t pred, lo, hi;
    if (!learned_window(key, v, li, pred, lo, hi)) return -1;
    return window_search<1>(key, reps, pred, lo, hi);
}

}  // namespace symed
