// Host-callable launchers of the learned-index kernels (learned.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace symed {

hipError_t mlp_init(float *d_params, int F, uint64_t seed, hipStream_t st);
hipError_t feature_range(const uint64_t *reps, int64_t D, int N, float *d_out, hipStream_t st);
int mlp_train_blocks(int batch);
hipError_t mlp_train_step(float *d_params, float *d_m, float *d_v, int F, float mu, float sc, int N,
                          const uint64_t *reps, int64_t D, uint64_t seed, int step, int batch, float lr, float *d_gpart,
                          float *d_lpart, float *d_loss, hipStream_t st);
hipError_t mlp_loss_grad(const float *d_params, int F, const float *d_X, const float *d_T, int64_t n, float *d_grad,
                         float *d_loss, float *d_gpart, float *d_lpart, hipStream_t st);
hipError_t leaf_ranges(const float *d_pw, int N, int lg, const uint64_t *reps, int64_t D, void *d_leaves,
                       uint32_t target, uint32_t *d_sizes, uint32_t *d_net_err, int blocks, hipStream_t st);
// Bucket begins at d_offsets, window statistics, largest bucket per leaf.
hipError_t leaf_buckets(void *d_leaves, int lg, const uint64_t *reps, const uint64_t *d_offsets, uint32_t *d_sub,
                        uint32_t *d_leaf_max, unsigned long long *d_stats, hipStream_t st);
// Bucket counts again, with a refinement factor per leaf (0 = 1).
hipError_t leaf_reshape(void *d_leaves, int lg, const uint64_t *reps, uint32_t target, const uint32_t *d_factor,
                        uint32_t *d_sizes, hipStream_t st);
// Raise the factor of leaves whose largest bucket exceeds `window` keys;
// *d_count += leaves raised.
hipError_t leaf_refine(const void *d_leaves, int lg, const uint32_t *d_leaf_max, uint32_t window, uint32_t *d_factor,
                       unsigned int *d_count, hipStream_t st);
// Largest bucket the index build aims for (keys), and refinement rounds.
constexpr uint32_t kMaxWindow = 64;
constexpr int kRefineRounds = 6;
hipError_t index_predict(const float *d_pw, int N, const uint64_t *keys, int64_t n, float *u, float *y, hipStream_t st);

}  // namespace symed
