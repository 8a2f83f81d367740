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

// Input of the network: one monotone feature of the key, read like a
// floating-point number, u = (e + 1 + m) / (N + 1), where e is the position
// of the leading one and m in [0, 1) the next 24 bits below it.
// Representatives cluster at small values (the orbit minimum has leading
// zeros); the exponent/mantissa split spreads them over [0, 1).  u is a
// non-decreasing function of the key (IEEE rounding is monotone).
__device__ __forceinline__ float key_feature(uint64_t key, int N)
{
#pragma clang fp contract(off)
    const int e = key ? 63 - __builtin_clzll(key) : -1;
    const uint64_t mb = (e > 0) ? (key << (64 - e)) >> 40 : 0ull;  // 24 bits below the leading one
    const float m = (float)(uint32_t)mb * (1.0f / 16777216.0f);
    const float inv = 1.0f / (float)(N + 1);
    return fmaf(m, inv, (float)(e + 1) * inv);
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

// A leaf: the keys routed to it occupy positions inside [lo, hi).  The leaf
// is split into nsub buckets uniform in key space: key k falls in bucket
// floor((k - kfirst) * scale) (clamped), and sub[off + q] is the first
// position in [lo, hi) whose key falls in bucket q or later (sub[off + nsub]
// = hi).  Buckets are monotone in the key, so every key of [lo, hi) - routed
// here or not - lies in the bucket of its own value.
struct Leaf {
    uint32_t lo, hi, off, nsub;
    uint64_t kfirst;
    double scale;     // nsub / (last key - kfirst + 1)
};

__host__ __device__ __forceinline__ uint32_t leaf_bucket(const Leaf &L, uint64_t key)
{
#pragma clang fp contract(off)
    if (key <= L.kfirst) return 0u;
    const double t = (double)(key - L.kfirst) * L.scale;
    const uint32_t q = t >= (double)L.nsub ? L.nsub - 1u : (uint32_t)t;
    return q < L.nsub ? q : L.nsub - 1u;
}

// Leaf and fractional position inside the leaf from the network output y.
// The leaf index is clamped as an integer: for 2^m >= 2^24 the float value
// of (2^m - 0.5) rounds up to 2^m.
__device__ __forceinline__ void leaf_of(float y, int log2_leaves, uint32_t &b, float &frac)
{
#pragma clang fp contract(off)
    const uint32_t Mi = 1u << log2_leaves;
    const float M = (float)Mi;
    float u = y * M;
    u = fminf(fmaxf(u, 0.0f), M);  // fmaxf also maps NaN to 0
    uint32_t bi = (uint32_t)floorf(u);
    if (bi > Mi - 1u) bi = Mi - 1u;
    b = bi;
    frac = fminf(u - (float)bi, 1.0f);
}

// Learned lookup: network (expanded form) -> leaf -> key-space bucket ->
// binary search.  -1 if absent.
__device__ __forceinline__ int64_t lookup_learned(uint64_t key, const uint64_t *__restrict__ reps, const PwView &pw,
                                                 const Leaf *__restrict__ leaves, const uint32_t *__restrict__ sub,
                                                 int N, int log2_leaves)
{
    const float y = pw_eval(pw, key_feature(key, N));
    uint32_t b;
    float frac;
    leaf_of(y, log2_leaves, b, frac);
    const Leaf L = leaves[b];
    if (L.lo >= L.hi) return -1;
    const uint32_t q = leaf_bucket(L, key);
    uint32_t lo = sub[L.off + q], hi = sub[L.off + q + 1];
    const uint32_t end = hi;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (reps[mid] < key) lo = mid + 1; else hi = mid;
    }
    return (lo < end && reps[lo] == key) ? (int64_t)lo : -1;
}

}  // namespace symed
