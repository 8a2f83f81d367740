// Learned index over the sorted representative list: training kernels
// (forward, backward, Adam) and the build of the tables below the network.
//
// The network maps the rank of a representative (among all configurations
// with its number of up spins) to an estimate of its normalized position;
// the estimate picks one of 2^lg segments.  Each segment maps ranks linearly
// onto cells, which are allocated in proportion to the keys routed to the
// segment; each cell records the position range of its keys, predicts a
// position by linear interpolation inside the cell, and records its largest
// errors below and above the prediction.  A segment whose cells need a
// window wider than the target gets four times the cells, a few rounds at
// most.  Every stored key lies in the window of its own cell, so a search
// there is exact; the plain Limits lookup remains the reference.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "learned.h"
#include "learned_dev.h"

namespace symed {

namespace {

constexpr int kTB = 64;  // samples per training block

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
__global__ void __launch_bounds__(kTB) k_fwdbwd(const float *__restrict__ Pg, int F, float mu, float sc,
                                               RankFeat rf, const uint64_t *__restrict__ reps, int64_t D, uint64_t seed,
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
            x[0] = (equalize(sz_rank(reps[j], rf.binom, rf.W), rf.eq) - mu) * sc;
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

// Stage the network pieces and the rank table into LDS.
__device__ __forceinline__ void stage_index(float *spw, uint64_t *srank, const float *pwg, const RankFeat &rf)
{
    for (int q = threadIdx.x; q < kPwFloats; q += blockDim.x) spw[q] = pwg[q];
    const int nr = rf.n_up * rf.W;
    for (int q = threadIdx.x; q < nr; q += blockDim.x) srank[q] = rf.binom[q];
    __syncthreads();
}

__device__ __forceinline__ void reduce_u64_add(unsigned long long v, unsigned long long *out)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

__device__ __forceinline__ void reduce_u32_max(uint32_t v, uint32_t *out)
{
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, v);
}

// Segment of every key: key count and rank range of each segment, and the
// largest |network estimate * D - position| (the network's own error).
__global__ void __launch_bounds__(256) k_route(const float *pwg, RankFeat rf, int lg, const uint64_t *reps, int64_t D,
                                             uint32_t *cnt, unsigned long long *rmin, unsigned long long *rmax,
                                             uint32_t *net_err)
{
    __shared__ float spw[kPwFloats];
    __shared__ uint64_t srank[kRankMaxEntries];
    stage_index(spw, srank, pwg, rf);
    const PwView pw = pw_view(spw);
    uint32_t worst = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t rank = sz_rank(reps[i], srank, rf.W);
        const float y = pw_eval(pw, equalize(rank, rf.eq));
        const uint32_t s = seg_of(y, lg);
        atomicAdd(&cnt[s], 1u);
        atomicMin(&rmin[s], (unsigned long long)rank);
        atomicMax(&rmax[s], (unsigned long long)rank);
        const double dy = fabs((double)y * (double)D - (double)i);
        worst = max(worst, dy > 4.0e9 ? 0xffffffffu : (uint32_t)dy);
    }
    reduce_u32_max(worst, net_err);
}

// Cells of every segment: about keys_per_cell keys per cell times the
// segment's refinement factor; sizes[s] = its cell count (0: no key).
__global__ void k_seg_shape(uint64_t M, const uint32_t *cnt, const unsigned long long *rmin,
                            const unsigned long long *rmax, uint32_t keys_per_cell, const uint32_t *factor, Seg *segs,
                            uint32_t *sizes)
{
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < M; s += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t n = cnt[s];
        if (n == 0) {
            segs[s] = Seg{~0ull, 0.0f, 0u};  // every rank lies below r0: absent
            sizes[s] = 0;
            continue;
        }
        const uint64_t f = factor[s] ? factor[s] : 1u;
        uint64_t nc = ((uint64_t)n + keys_per_cell - 1) / keys_per_cell * f;
        const uint64_t span = (uint64_t)(rmax[s] - rmin[s]) + 1;
        if (nc > span) nc = span;  // no more cells than ranks
        // scale rounded down, so the segment's last key stays in its last cell
        const double x = (double)nc / (double)span;
        float sf = (float)x;
        if ((double)sf > x) sf = nextafterf(sf, 0.0f);
        segs[s] = Seg{(uint64_t)rmin[s], sf, 0u};
        sizes[s] = (uint32_t)nc;
    }
}

__global__ void k_seg_setoff(Seg *segs, uint64_t M, const uint64_t *offsets)
{
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < M; s += (uint64_t)gridDim.x * blockDim.x)
        segs[s].cell0 = (uint32_t)offsets[s];
}

__global__ void k_cell_clear(uint32_t *first, uint32_t *last, uint32_t *elo, uint32_t *ehi, uint64_t n)
{
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (uint64_t)gridDim.x * blockDim.x) {
        first[c] = 0xffffffffu;
        last[c] = 0u;
        elo[c] = 0u;
        ehi[c] = 0u;
    }
}

// Cell of every key, as the lookup computes it.
__device__ __forceinline__ uint64_t key_cell(uint64_t key, const PwView &pw, const uint64_t *srank,
                                             const RankFeat &rf, int lg, const Seg *segs, uint64_t n_cells,
                                             double &frac)
{
    const uint64_t rank = sz_rank(key, srank, rf.W);
    const float y = pw_eval(pw, equalize(rank, rf.eq));
    const Seg S = segs[seg_of(y, lg)];
    uint64_t ci = 0;
    frac = 0.0;
    (void)cell_of(rank, S, n_cells, ci, frac);  // a routed key is never below its segment's r0
    return ci;
}

// Position range of the keys of every cell (pass 0), then the largest
// errors of the cell's interpolation below and above (pass 1).
template <int PASS>
__global__ void __launch_bounds__(256) k_cell_pass(const float *pwg, RankFeat rf, int lg, const uint64_t *reps,
                                                 int64_t D, const Seg *segs, uint64_t n_cells, uint32_t *first,
                                                 uint32_t *last, uint32_t *elo, uint32_t *ehi)
{
    __shared__ float spw[kPwFloats];
    __shared__ uint64_t srank[kRankMaxEntries];
    stage_index(spw, srank, pwg, rf);
    const PwView pw = pw_view(spw);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        double frac;
        const uint64_t ci = key_cell(reps[i], pw, srank, rf, lg, segs, n_cells, frac);
        if (PASS == 0) {
            atomicMin(&first[ci], (uint32_t)i);
            atomicMax(&last[ci], (uint32_t)i);
        } else {
            const uint32_t pred = first[ci] + cell_offset(last[ci] - first[ci] + 1u, frac);
            if (pred > (uint32_t)i) atomicMax(&elo[ci], pred - (uint32_t)i);
            else if (pred < (uint32_t)i) atomicMax(&ehi[ci], (uint32_t)i - pred);
        }
    }
}

// One wavefront per segment: the widest window among its cells; segments
// wider than `window` keys get four times the cells (factor up to fmax, and
// at most 2^24 cells per segment).  *count += segments refined.
__global__ void __launch_bounds__(256) k_seg_refine(uint64_t M, const Seg *segs, const uint32_t *sizes,
                                                  const uint32_t *first, const uint32_t *last, const uint32_t *elo,
                                                  const uint32_t *ehi, uint32_t window, uint32_t fmax,
                                                  uint32_t *factor, unsigned int *count)
{
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    for (uint64_t s = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; s < M; s += waves) {
        const uint32_t nc = sizes[s], c0 = segs[s].cell0;
        uint32_t w = 0;
        for (uint32_t c = lane; c < nc; c += 64) {
            const uint32_t g = c0 + c;
            if (first[g] > last[g]) continue;  // empty cell
            const uint32_t n = last[g] - first[g] + 1u;
            w = max(w, min(n, elo[g] + ehi[g] + 1u));
        }
        for (int o = 32; o > 0; o >>= 1) w = max(w, (uint32_t)__shfl_xor((int)w, o, 64));
        if (lane == 0 && w > window) {
            const uint32_t f = factor[s] ? factor[s] : 1u;
            if (f < fmax && (uint64_t)nc * 4u <= (1u << 24)) {
                factor[s] = f * 4u;
                atomicAdd(count, 1u);
            }
        }
    }
}

// Final cells {first, n | elo << 20 | ehi << 26}; *bad = 1 if a cell covers
// 2^20 positions or more.
__global__ void k_cell_pack(uint64_t n_cells, const uint32_t *first, const uint32_t *last, const uint32_t *elo,
                            const uint32_t *ehi, uint2 *cells, uint32_t *bad)
{
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_cells;
         c += (uint64_t)gridDim.x * blockDim.x) {
        if (first[c] > last[c]) {
            cells[c] = make_uint2(0u, 0u);
            continue;
        }
        const uint32_t n = last[c] - first[c] + 1u;
        if (n >= (1u << kCellNBits)) atomicMax(bad, 1u);
        cells[c] = make_uint2(first[c], cell_meta(n, elo[c], ehi[c]));
    }
}

// Windows of the finished index, key by key, as the lookup sees them:
// stats[0] = sum of window sizes, [1] = sum |prediction - position|, [2] =
// exact predictions, [3] = sum of 128-byte record lines spanned by the
// window ({rep, x} records of 16 bytes), [4] = keys outside their window
// (must be 0); max_win = largest window.
__global__ void __launch_bounds__(256) k_window_stats(const float *pwg, RankFeat rf, int lg, const uint64_t *reps,
                                                    int64_t D, const Seg *segs, const uint2 *cells, uint64_t n_cells,
                                                    unsigned long long *stats, uint32_t *max_win)
{
    __shared__ float spw[kPwFloats];
    __shared__ uint64_t srank[kRankMaxEntries];
    stage_index(spw, srank, pwg, rf);
    const PwView pw = pw_view(spw);
    unsigned long long sw = 0, se = 0, sx = 0, sl = 0, so = 0;
    uint32_t mw = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D; i += (int64_t)gridDim.x * blockDim.x) {
        double frac;
        const uint64_t ci = key_cell(reps[i], pw, srank, rf, lg, segs, n_cells, frac);
        uint32_t pred, lo, hi;
        cell_window(cells[ci], frac, pred, lo, hi);
        const uint32_t w = hi - lo + 1u;
        sw += w;
        se += pred > (uint32_t)i ? pred - (uint32_t)i : (uint32_t)i - pred;
        sx += pred == (uint32_t)i;
        sl += (hi >> 3) - (lo >> 3) + 1u;
        so += ((uint32_t)i < lo || (uint32_t)i > hi);
        mw = max(mw, w);
    }
    reduce_u64_add(sw, &stats[0]);
    reduce_u64_add(se, &stats[1]);
    reduce_u64_add(sx, &stats[2]);
    reduce_u64_add(sl, &stats[3]);
    reduce_u64_add(so, &stats[4]);
    reduce_u32_max(mw, max_win);
}

// u and the expanded network output for given keys (verification); keys
// that are not sector configurations give NaN
__global__ void __launch_bounds__(256) k_predict(const float *pwg, RankFeat rf, int N, const uint64_t *keys, int64_t n,
                                               float *u, float *y)
{
    __shared__ float spw[kPwFloats];
    __shared__ uint64_t srank[kRankMaxEntries];
    stage_index(spw, srank, pwg, rf);
    const PwView pw = pw_view(spw);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        if (__popcll(k) != rf.n_up || (N < 64 && (k >> N))) {
            u[i] = __int_as_float(0x7fc00000);
            y[i] = __int_as_float(0x7fc00000);
            continue;
        }
        const float uu = equalize(sz_rank(k, srank, rf.W), rf.eq);
        u[i] = uu;
        y[i] = pw_eval(pw, uu);
    }
}

__global__ void k_feature_range(const uint64_t *reps, int64_t D, RankFeat rf, float *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        out[0] = equalize(sz_rank(reps[0], rf.binom, rf.W), rf.eq);
        out[1] = equalize(sz_rank(reps[D - 1], rf.binom, rf.W), rf.eq);
    }
}

}  // namespace

hipError_t feature_range(const uint64_t *reps, int64_t D, const RankFeat &rf, float *d_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_feature_range, dim3(1), dim3(64), 0, st, reps, D, rf, d_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------

hipError_t mlp_init(float *d_params, int F, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_init, dim3(8), dim3(256), 0, st, d_params, F, seed);
    return hipGetLastError();
}

int mlp_train_blocks(int batch) { return (batch + kTB - 1) / kTB; }

hipError_t mlp_train_step(float *d_params, float *d_m, float *d_v, int F, float mu, float sc, const RankFeat &rf,
                          const uint64_t *reps, int64_t D, uint64_t seed, int step, int batch, float lr, float *d_gpart,
                          float *d_lpart, float *d_loss, hipStream_t st)
{
    const int nb = mlp_train_blocks(batch);
    const int NP = mlp_param_count(F, kHidden);
    hipLaunchKernelGGL(k_fwdbwd, dim3(nb), dim3(kTB), 0, st, d_params, F, mu, sc, rf, reps, D, seed, step, nullptr,
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
    hipLaunchKernelGGL(k_fwdbwd, dim3(nb), dim3(kTB), 0, st, d_params, F, 0.0f, 1.0f, RankFeat{}, nullptr,
                       (int64_t)1, 0ull, 0, d_X, d_T, n, 1.0f / (float)n, d_gpart, d_lpart);
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, st, const_cast<float *>(d_params), nullptr,
                       nullptr, d_gpart, d_lpart, nb, NP, 0.0f, 0.0f, 0.0f, 0.0f, 1, d_grad, d_loss, F, 0);
    return hipGetLastError();
}

hipError_t index_route(const float *d_pw, const RankFeat &rf, int lg, const uint64_t *reps, int64_t D, uint32_t *cnt,
                       unsigned long long *rmin, unsigned long long *rmax, uint32_t *net_err, int blocks,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_route, dim3(blocks), dim3(256), 0, st, d_pw, rf, lg, reps, D, cnt, rmin, rmax, net_err);
    return hipGetLastError();
}

hipError_t index_seg_shape(uint64_t M, const uint32_t *cnt, const unsigned long long *rmin,
                           const unsigned long long *rmax, uint32_t keys_per_cell, const uint32_t *factor, void *segs,
                           uint32_t *sizes, hipStream_t st)
{
    hipLaunchKernelGGL(k_seg_shape, dim3(1024), dim3(256), 0, st, M, cnt, rmin, rmax, keys_per_cell, factor,
                       static_cast<Seg *>(segs), sizes);
    return hipGetLastError();
}

hipError_t index_seg_setoff(void *segs, uint64_t M, const uint64_t *offsets, hipStream_t st)
{
    hipLaunchKernelGGL(k_seg_setoff, dim3(1024), dim3(256), 0, st, static_cast<Seg *>(segs), M, offsets);
    return hipGetLastError();
}

hipError_t index_cells(const float *d_pw, const RankFeat &rf, int lg, const uint64_t *reps, int64_t D, const void *segs,
                       uint64_t n_cells, uint32_t *first, uint32_t *last, uint32_t *elo, uint32_t *ehi, int blocks,
                       hipStream_t st)
{
    const Seg *sg = static_cast<const Seg *>(segs);
    hipLaunchKernelGGL(k_cell_clear, dim3(1024), dim3(256), 0, st, first, last, elo, ehi, n_cells);
    hipLaunchKernelGGL(k_cell_pass<0>, dim3(blocks), dim3(256), 0, st, d_pw, rf, lg, reps, D, sg, n_cells, first, last,
                       elo, ehi);
    hipLaunchKernelGGL(k_cell_pass<1>, dim3(blocks), dim3(256), 0, st, d_pw, rf, lg, reps, D, sg, n_cells, first, last,
                       elo, ehi);
    return hipGetLastError();
}

hipError_t index_refine(uint64_t M, const void *segs, const uint32_t *sizes, const uint32_t *first,
                        const uint32_t *last, const uint32_t *elo, const uint32_t *ehi, uint32_t window, uint32_t fmax,
                        uint32_t *factor, unsigned int *count, hipStream_t st)
{
    // one wavefront per segment, at most 65536 blocks of four
    const unsigned blocks = (unsigned)std::min<uint64_t>((M + 3) / 4, 65536);
    hipLaunchKernelGGL(k_seg_refine, dim3(blocks), dim3(256), 0, st, M, static_cast<const Seg *>(segs), sizes, first,
                       last, elo, ehi, window, fmax, factor, count);
    return hipGetLastError();
}

hipError_t index_pack(uint64_t n_cells, const uint32_t *first, const uint32_t *last, const uint32_t *elo,
                      const uint32_t *ehi, void *cells, uint32_t *bad, hipStream_t st)
{
    hipLaunchKernelGGL(k_cell_pack, dim3(1024), dim3(256), 0, st, n_cells, first, last, elo, ehi,
                       static_cast<uint2 *>(cells), bad);
    return hipGetLastError();
}

hipError_t index_window_stats(const float *d_pw, const RankFeat &rf, int lg, const uint64_t *reps, int64_t D,
                              const void *segs, const void *cells, uint64_t n_cells, unsigned long long *stats,
                              uint32_t *max_win, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL(k_window_stats, dim3(blocks), dim3(256), 0, st, d_pw, rf, lg, reps, D,
                       static_cast<const Seg *>(segs), static_cast<const uint2 *>(cells), n_cells, stats, max_win);
    return hipGetLastError();
}

hipError_t index_predict(const float *d_pw, const RankFeat &rf, int N, const uint64_t *keys, int64_t n, float *u,
                         float *y, hipStream_t st)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_predict, dim3((unsigned)blocks), dim3(256), 0, st, d_pw, rf, N, keys, n, u, y);
    return hipGetLastError();
}

}  // namespace symed
