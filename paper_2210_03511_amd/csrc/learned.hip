// Learned index over the sorted representative list: training kernels
// (forward, backward, Adam) and the exact leaf-table build.
//
// The network maps a representative to an estimate of its normalized rank;
// that estimate routes the key to one of 2^m leaves.  The network is
// monotone, so the keys routed to a leaf fill a position range [lo, hi).
// Each leaf splits its range into buckets uniform in key space and records
// where each bucket begins, so a binary search inside the key's bucket finds
// every stored key and reports absence for every other key.  Leaves whose
// largest bucket holds more than kMaxWindow keys get proportionally more
// buckets, a few rounds at most.  The plain Limits lookup remains the
// reference the learned lookup is compared with.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "learned.h"
#include "learned_dev.h"

namespace symed {

namespace {

constexpr int kTB = 64;  // samples per training block
constexpr uint32_t kMaxRefine = 1024;  // largest bucket refinement factor of a leaf

__device__ __forceinline__ uint64_t splitmix(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Deterministic initialization of the monotone network (input standardized
// to [-1, 1]): first-layer units are hinges at knots spread over [-1, 1];
// second-layer and output weights are small positive numbers.
__global__ void k_mlp_init(float *P, int F, uint64_t seed)
{
    const int H = kHidden;
    const int n = mlp_param_count(F, H);
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        const int o_b1 = H * F, o_W2 = o_b1 + H, o_b2 = o_W2 + H * H, o_W3 = o_b2 + H, o_b3 = o_W3 + H;
        const double u = (double)(splitmix(seed * 0x100000001B3ull + (uint64_t)p) >> 11) * (1.0 / 9007199254740992.0);
        if (p < o_b1) {
            P[p] = 1.0f;
        } else if (p < o_W2) {
            const int j = p - o_b1;
            P[p] = -(-1.0f + 2.0f * ((float)(j % (H / 2)) + 0.5f) / (float)(H / 2));
        } else if (p < o_b2) {
            P[p] = (float)(u * 2.0 / H);
        } else if (p < o_W3) {
            P[p] = 0.0f;
        } else if (p < o_b3) {
            P[p] = (float)(u * 2.0 / H);
        } else {
            P[p] = 0.0f;
        }
    }
}

// One block: kTB samples.  Forward with stored activations, backward of
// L = (1/2) * inv_total * sum (y - t)^2, per-block gradient sums written to
// gpart[block][param] (summed over blocks in a fixed order by k_adam).
// Sampling mode (X == nullptr): sample s draws position j = hash(seed, step,
// s) mod D and uses (key = reps[j], t = (j + 1/2) / D).  Explicit mode: X[s][F],
// T[s].
__global__ void __launch_bounds__(kTB) k_fwdbwd(const float *__restrict__ Pg, int F, float mu, float sc, int N,
                                               const uint64_t *__restrict__ reps, int64_t D, uint64_t seed,
                                               int step, const float *__restrict__ X, const float *__restrict__ T,
                                               int64_t n_total, float inv_total, float *gpart, float *lpart)
{
    const int H = kHidden;
    const int NP = mlp_param_count(F, H);
    __shared__ float sP[kMlpMaxParams];
    __shared__ float sx[kTB][kMaxFeatures];
    __shared__ float sh1[kTB][kHidden], sd1[kTB][kHidden], sh2[kTB][kHidden], sd2[kTB][kHidden];
    __shared__ float sr[kTB], sl[kTB];
    for (int p = threadIdx.x; p < NP; p += kTB) sP[p] = Pg[p];
    __syncthreads();
    const float *W1 = sP, *b1 = sP + H * F, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;

    const int64_t s = (int64_t)blockIdx.x * kTB + threadIdx.x;
    const bool valid = s < n_total;
    float x[kMaxFeatures];
    float t = 0.0f;
    if (valid) {
        if (X) {
            for (int f = 0; f < F; ++f) x[f] = X[s * F + f];
            t = T[s];
        } else {
            const uint64_t h = splitmix(seed ^ ((uint64_t)step << 32) ^ (uint64_t)s);
            const uint64_t j = h % (uint64_t)D;
            x[0] = (key_feature(reps[j], N) - mu) * sc;
            t = (float)(((double)j + 0.5) / (double)D);
        }
    } else {
        for (int f = 0; f < F; ++f) x[f] = 0.0f;
    }
    // activation derivative masks: relu units pass where z > 0, min(z,0) units where z < 0
    float z1[kHidden], h1[kHidden], z2[kHidden];
    for (int j = 0; j < H; ++j) {
        float a = b1[j];
        for (int f = 0; f < F; ++f) a = fmaf(W1[j * F + f], x[f], a);
        z1[j] = a;
        h1[j] = hidden_act(a, j);
    }
    float y = b3[0];
    for (int k = 0; k < H; ++k) {
        float a = b2[k];
        for (int j = 0; j < H; ++j) a = fmaf(W2[k * H + j], h1[j], a);
        z2[k] = a;
        sh2[threadIdx.x][k] = hidden_act(a, k);
        y = fmaf(W3[k], hidden_act(a, k), y);
    }
    const float r = valid ? (y - t) * inv_total : 0.0f;
    sl[threadIdx.x] = valid ? 0.5f * (y - t) * (y - t) * inv_total : 0.0f;
    float d2[kHidden];
    for (int k = 0; k < H; ++k) {
        const bool pass = (k < kHidden / 2) ? (z2[k] > 0.0f) : (z2[k] < 0.0f);
        d2[k] = pass ? r * W3[k] : 0.0f;
        sd2[threadIdx.x][k] = d2[k];
    }
    for (int j = 0; j < H; ++j) {
        float a = 0.0f;
        for (int k = 0; k < H; ++k) a = fmaf(d2[k], W2[k * H + j], a);
        const bool pass = (j < kHidden / 2) ? (z1[j] > 0.0f) : (z1[j] < 0.0f);
        sd1[threadIdx.x][j] = pass ? a : 0.0f;
        sh1[threadIdx.x][j] = h1[j];
    }
    for (int f = 0; f < F; ++f) sx[threadIdx.x][f] = x[f];
    sr[threadIdx.x] = r;
    __syncthreads();

    const int o_b1 = H * F, o_W2 = o_b1 + H, o_b2 = o_W2 + H * H, o_W3 = o_b2 + H, o_b3 = o_W3 + H;
    for (int p = threadIdx.x; p < NP; p += kTB) {
        float g = 0.0f;
        if (p < o_b1) {
            const int j = p / F, f = p % F;
            for (int q = 0; q < kTB; ++q) g = fmaf(sd1[q][j], sx[q][f], g);
        } else if (p < o_W2) {
            const int j = p - o_b1;
            for (int q = 0; q < kTB; ++q) g += sd1[q][j];
        } else if (p < o_b2) {
            const int k = (p - o_W2) / H, j = (p - o_W2) % H;
            for (int q = 0; q < kTB; ++q) g = fmaf(sd2[q][k], sh1[q][j], g);
        } else if (p < o_W3) {
            const int k = p - o_b2;
            for (int q = 0; q < kTB; ++q) g += sd2[q][k];
        } else if (p < o_b3) {
            const int k = p - o_W3;
            for (int q = 0; q < kTB; ++q) g = fmaf(sr[q], sh2[q][k], g);
        } else {
            for (int q = 0; q < kTB; ++q) g += sr[q];
        }
        gpart[(int64_t)blockIdx.x * NP + p] = g;
    }
    if (threadIdx.x == 0) {
        float l = 0.0f;
        for (int q = 0; q < kTB; ++q) l += sl[q];
        lpart[blockIdx.x] = l;
    }
}

// Sum the block partials in a fixed order; optionally apply one Adam step.
// monotone != 0: weights (not biases) are projected onto >= 0 after the
// step, which keeps the network non-decreasing in its input.
__global__ void k_adam(float *P, float *m, float *v, const float *gpart, const float *lpart, int nblocks, int NP,
                       float lr, float b1, float b2, float eps, int t, float *grad_out, float *loss_out, int F,
                       int monotone)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss_out) {
        float l = 0.0f;
        for (int q = 0; q < nblocks; ++q) l += lpart[q];
        *loss_out = l;
    }
    if (p >= NP) return;
    float g = 0.0f;
    for (int q = 0; q < nblocks; ++q) g += gpart[(int64_t)q * NP + p];
    if (grad_out) grad_out[p] = g;
    if (!m) return;
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.0f - powf(b1, (float)t));
    const float vh = vv / (1.0f - powf(b2, (float)t));
    float w = P[p] - lr * mh / (sqrtf(vh) + eps);
    if (monotone) {
        const int H = kHidden;
        const int o_b1 = H * F, o_W2 = o_b1 + H, o_b2 = o_W2 + H * H, o_W3 = o_b2 + H, o_b3 = o_W3 + H;
        const bool weight = p < o_b1 || (p >= o_W2 && p < o_b2) || (p >= o_W3 && p < o_b3);
        if (weight) w = fmaxf(w, 0.0f);
    }
    P[p] = w;
}

__global__ void k_leaf_init(Leaf *leaves, uint64_t M)
{
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < M; b += (uint64_t)gridDim.x * blockDim.x)
        leaves[b] = Leaf{0xffffffffu, 0u, 0u, 0u, 0ull, 0.0};
}

// position range of every leaf
__global__ void __launch_bounds__(256) k_leaf_range(const float *pwg, int N, int lg, const uint64_t *reps, int64_t D,
                                                  Leaf *leaves)
{
    __shared__ float spw[kPwFloats];
    for (int q = threadIdx.x; q < kPwFloats; q += blockDim.x) spw[q] = pwg[q];
    __syncthreads();
    const PwView pw = pw_view(spw);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t b;
        float frac;
        leaf_of(pw_eval(pw, key_feature(reps[i], N)), lg, b, frac);
        atomicMin(&leaves[b].lo, (uint32_t)i);
        atomicMax(&leaves[b].hi, (uint32_t)(i + 1));
    }
}

// key-space bucket count of each leaf: about `target` keys per bucket, at
// most one bucket per position of the range, both times the leaf's
// refinement factor (0 = 1); sizes[b] = entries of the leaf's bucket-begin
// array (nsub + 1, or 0 for an empty leaf)
__global__ void k_leaf_shape(Leaf *leaves, uint64_t M, const uint64_t *reps, uint32_t target,
                             const uint32_t *factor, uint32_t *sizes)
{
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < M; b += (uint64_t)gridDim.x * blockDim.x) {
        Leaf L = leaves[b];
        if (L.lo >= L.hi) {
            leaves[b] = Leaf{0u, 0u, 0u, 0u, 0ull, 0.0};
            sizes[b] = 0;
            continue;
        }
        const uint32_t count = L.hi - L.lo;
        const uint32_t f = (factor && factor[b]) ? factor[b] : 1u;
        uint64_t nsub = ((uint64_t)count + target - 1) / target * f;
        if (nsub < 1) nsub = 1;
        if (nsub > (uint64_t)count * f) nsub = (uint64_t)count * f;
        const uint64_t k0 = reps[L.lo], k1 = reps[L.hi - 1];
        L.kfirst = k0;
        L.nsub = (uint32_t)nsub;
        L.scale = (double)nsub / ((double)(k1 - k0) + 1.0);
        leaves[b] = L;
        sizes[b] = (uint32_t)nsub + 1;
    }
}

__global__ void k_leaf_setoff(Leaf *leaves, uint64_t M, const uint64_t *offsets)
{
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < M; b += (uint64_t)gridDim.x * blockDim.x)
        leaves[b].off = (uint32_t)offsets[b];
}

// Bucket begins, one wavefront per leaf, its lanes over the positions of the
// leaf's range [lo, hi) (whatever leaf each position is routed to: the FP32
// evaluation of the network can step back at a breakpoint, so neighbouring
// ranges may overlap): sub[off + q] = first position of [lo, hi) whose key
// lies in bucket q or later.  Position p writes the entries of the buckets
// after its predecessor's up to its own, and the last position also those
// after its own, ending with sub[off + nsub] = hi.
__global__ void __launch_bounds__(256) k_leaf_fill(const Leaf *leaves, uint64_t M, const uint64_t *reps,
                                                 uint32_t *sub)
{
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    for (uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < M; b += waves) {
        const Leaf L = leaves[b];
        if (L.lo >= L.hi) continue;
        for (uint32_t p = L.lo + lane; p < L.hi; p += 64) {
            const uint32_t q = leaf_bucket(L, reps[p]);
            const int64_t q0 = (p == L.lo) ? -1 : (int64_t)leaf_bucket(L, reps[p - 1]);
            for (int64_t r = q0 + 1; r <= (int64_t)q; ++r) sub[L.off + r] = p;
            if (p + 1 == L.hi)
                for (uint32_t r = q + 1; r <= L.nsub; ++r) sub[L.off + r] = L.hi;
        }
    }
}

// Bucket sizes, one wavefront per leaf, from the first position of each
// bucket: the sum of their squares and their maximum (stats), and the
// largest bucket of every leaf.
__global__ void __launch_bounds__(256) k_leaf_stats(const Leaf *leaves, uint64_t M, const uint64_t *reps,
                                                  const uint32_t *sub, uint32_t *leaf_max,
                                                  unsigned long long *stats)
{
    __shared__ unsigned long long ssq[256];
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    unsigned long long sq = 0, mx = 0;
    for (uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < M; b += waves) {
        const Leaf L = leaves[b];
        uint32_t lm = 0;
        if (L.lo < L.hi) {
            for (uint32_t p = L.lo + lane; p < L.hi; p += 64) {
                const uint32_t q = leaf_bucket(L, reps[p]);
                if (p != L.lo && leaf_bucket(L, reps[p - 1]) == q) continue;
                const uint32_t w = sub[L.off + q + 1] - p;
                sq += (unsigned long long)w * w;
                lm = w > lm ? w : lm;
            }
        }
        for (int o = 32; o > 0; o >>= 1) lm = max(lm, (uint32_t)__shfl_xor((int)lm, o, 64));
        if (lane == 0) leaf_max[b] = lm;
        mx = lm > mx ? lm : mx;
    }
    ssq[threadIdx.x] = sq;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) ssq[threadIdx.x] += ssq[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(&stats[0], ssq[0]);
    if (lane == 0) atomicMax(&stats[1], mx);
}

// Leaves whose largest bucket holds more than `window` keys: the
// refinement factor grows by ceil(largest / window), up to kMaxRefine in
// all; `count` receives the number of leaves refined.
__global__ void k_leaf_refine(const Leaf *leaves, uint64_t M, const uint32_t *leaf_max, uint32_t window,
                              uint32_t *factor, unsigned int *count)
{
    for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < M; b += (uint64_t)gridDim.x * blockDim.x) {
        const Leaf L = leaves[b];
        if (L.lo >= L.hi) continue;
        const uint32_t mx = leaf_max[b];
        const uint32_t f = factor[b] ? factor[b] : 1u;
        if (mx <= window || f >= kMaxRefine || L.nsub >= (1u << 22)) continue;
        factor[b] = min(kMaxRefine, f * ((mx + window - 1) / window));
        atomicAdd(count, 1u);
    }
}

// largest |network estimate * D - position| over all keys
__global__ void __launch_bounds__(256) k_net_err(const float *pwg, int N, const uint64_t *reps, int64_t D,
                                               uint32_t *net_err)
{
    __shared__ float spw[kPwFloats];
    for (int q = threadIdx.x; q < kPwFloats; q += blockDim.x) spw[q] = pwg[q];
    __syncthreads();
    const PwView pw = pw_view(spw);
    uint32_t worst = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        const float y = pw_eval(pw, key_feature(reps[i], N));
        const double dy = fabs((double)y * (double)D - (double)i);
        const uint32_t me = dy > 4.0e9 ? 0xffffffffu : (uint32_t)dy;
        worst = max(worst, me);
    }
    for (int o = 32; o > 0; o >>= 1) worst = max(worst, (uint32_t)__shfl_xor((int)worst, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(net_err, worst);
}

// u and the expanded network output for given keys (verification)
__global__ void __launch_bounds__(256) k_predict(const float *pwg, int N, const uint64_t *keys, int64_t n, float *u,
                                               float *y)
{
    __shared__ float spw[kPwFloats];
    for (int q = threadIdx.x; q < kPwFloats; q += blockDim.x) spw[q] = pwg[q];
    __syncthreads();
    const PwView pw = pw_view(spw);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float uu = key_feature(keys[i], N);
        u[i] = uu;
        y[i] = pw_eval(pw, uu);
    }
}

__global__ void k_feature_range(const uint64_t *reps, int64_t D, int N, float *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = key_feature(reps[0], N);
        out[1] = key_feature(reps[D - 1], N);
    }
}

}  // namespace

hipError_t feature_range(const uint64_t *reps, int64_t D, int N, float *d_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_feature_range, dim3(1), dim3(64), 0, st, reps, D, N, d_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

hipError_t mlp_init(float *d_params, int F, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_init, dim3(8), dim3(256), 0, st, d_params, F, seed);
    return hipGetLastError();
}

int mlp_train_blocks(int batch) { return (batch + kTB - 1) / kTB; }

hipError_t mlp_train_step(float *d_params, float *d_m, float *d_v, int F, float mu, float sc, int N,
                          const uint64_t *reps, int64_t D, uint64_t seed, int step, int batch, float lr, float *d_gpart,
                          float *d_lpart, float *d_loss, hipStream_t st)
{
    const int nb = mlp_train_blocks(batch);
    const int NP = mlp_param_count(F, kHidden);
    hipLaunchKernelGGL(k_fwdbwd, dim3(nb), dim3(kTB), 0, st, d_params, F, mu, sc, N, reps, D, seed, step, nullptr,
                       nullptr, (int64_t)batch, 1.0f / (float)batch, d_gpart, d_lpart);
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, st, d_params, d_m, d_v, d_gpart, d_lpart, nb,
                       NP, lr, 0.9f, 0.999f, 1e-8f, step + 1, nullptr, d_loss, F, 1);
    return hipGetLastError();
}

hipError_t mlp_loss_grad(const float *d_params, int F, const float *d_X, const float *d_T, int64_t n, float *d_grad,
                         float *d_loss, float *d_gpart, float *d_lpart, hipStream_t st)
{
    const int nb = (int)((n + kTB - 1) / kTB);
    const int NP = mlp_param_count(F, kHidden);
    hipLaunchKernelGGL(k_fwdbwd, dim3(nb), dim3(kTB), 0, st, d_params, F, 0.0f, 1.0f, 64, nullptr, (int64_t)1, 0ull, 0,
                       d_X, d_T, n, 1.0f / (float)n, d_gpart, d_lpart);
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, st, const_cast<float *>(d_params), nullptr,
                       nullptr, d_gpart, d_lpart, nb, NP, 0.0f, 0.0f, 0.0f, 0.0f, 1, d_grad, d_loss, F, 0);
    return hipGetLastError();
}

hipError_t leaf_ranges(const float *d_pw, int N, int lg, const uint64_t *reps, int64_t D, void *d_leaves,
                       uint32_t target, uint32_t *d_sizes, uint32_t *d_net_err, int blocks, hipStream_t st)
{
    Leaf *lv = static_cast<Leaf *>(d_leaves);
    const uint64_t M = 1ull << lg;
    hipLaunchKernelGGL(k_leaf_init, dim3(1024), dim3(256), 0, st, lv, M);
    hipLaunchKernelGGL(k_leaf_range, dim3(blocks), dim3(256), 0, st, d_pw, N, lg, reps, D, lv);
    hipLaunchKernelGGL(k_leaf_shape, dim3(1024), dim3(256), 0, st, lv, M, reps, target, nullptr, d_sizes);
    hipLaunchKernelGGL(k_net_err, dim3(blocks), dim3(256), 0, st, d_pw, N, reps, D, d_net_err);
    return hipGetLastError();
}

hipError_t leaf_reshape(void *d_leaves, int lg, const uint64_t *reps, uint32_t target, const uint32_t *d_factor,
                        uint32_t *d_sizes, hipStream_t st)
{
    Leaf *lv = static_cast<Leaf *>(d_leaves);
    const uint64_t M = 1ull << lg;
    hipLaunchKernelGGL(k_leaf_shape, dim3(1024), dim3(256), 0, st, lv, M, reps, target, d_factor, d_sizes);
    return hipGetLastError();
}

hipError_t leaf_refine(const void *d_leaves, int lg, const uint32_t *d_leaf_max, uint32_t window, uint32_t *d_factor,
                       unsigned int *d_count, hipStream_t st)
{
    const Leaf *lv = static_cast<const Leaf *>(d_leaves);
    const uint64_t M = 1ull << lg;
    hipLaunchKernelGGL(k_leaf_refine, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, st, lv, M, d_leaf_max, window,
                       d_factor, d_count);
    return hipGetLastError();
}

hipError_t leaf_buckets(void *d_leaves, int lg, const uint64_t *reps, const uint64_t *d_offsets, uint32_t *d_sub,
                        uint32_t *d_leaf_max, unsigned long long *d_stats, hipStream_t st)
{
    Leaf *lv = static_cast<Leaf *>(d_leaves);
    const uint64_t M = 1ull << lg;
    // one wavefront per leaf, at most 65536 blocks of four
    const unsigned blocks = (unsigned)std::min<uint64_t>((M + 3) / 4, 65536);
    hipLaunchKernelGGL(k_leaf_setoff, dim3(1024), dim3(256), 0, st, lv, M, d_offsets);
    hipLaunchKernelGGL(k_leaf_fill, dim3(blocks), dim3(256), 0, st, lv, M, reps, d_sub);
    hipLaunchKernelGGL(k_leaf_stats, dim3(blocks), dim3(256), 0, st, lv, M, reps, d_sub, d_leaf_max, d_stats);
    return hipGetLastError();
}

hipError_t index_predict(const float *d_pw, int N, const uint64_t *keys, int64_t n, float *u, float *y, hipStream_t st)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_predict, dim3((unsigned)blocks), dim3(256), 0, st, d_pw, N, keys, n, u, y);
    return hipGetLastError();
}

}  // namespace symed
