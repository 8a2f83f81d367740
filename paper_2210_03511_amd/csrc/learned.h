// Host-callable launchers of the learned-index kernels (learned.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "learned_dev.h"

namespace symed {

hipError_t mlp_init(float *d_params, int F, uint64_t seed, hipStream_t st);
// network inputs of the first and last representative
hipError_t feature_range(const uint64_t *reps, int64_t D, const RankFeat &rf, float *d_out, hipStream_t st);
int mlp_train_blocks(int batch);
hipError_t mlp_train_step(float *d_params, float *d_m, float *d_v, int F, float mu, float sc, const RankFeat &rf,
                          const uint64_t *reps, int64_t D, uint64_t seed, int step, int batch, float lr, float *d_gpart,
                          float *d_lpart, float *d_loss, hipStream_t st);
hipError_t mlp_loss_grad(const float *d_params, int F, const float *d_X, const float *d_T, int64_t n, float *d_grad,
                         float *d_loss, float *d_gpart, float *d_lpart, hipStream_t st);
// Index build: key count and rank range of every segment (counters cleared
// by the caller: cnt 0, rmin all ones, rmax 0), the network's largest error.
hipError_t index_route(const float *d_pw, const RankFeat &rf, int lg, const uint64_t *reps, int64_t D, uint32_t *cnt,
                       unsigned long long *rmin, unsigned long long *rmax, uint32_t *net_err, int blocks,
                       hipStream_t st);
// Segments (r0, scale) and their cell counts; factor: refinement (0 = 1).
hipError_t index_seg_shape(uint64_t M, const uint32_t *cnt, const unsigned long long *rmin,
                           const unsigned long long *rmax, uint32_t keys_per_cell, const uint32_t *factor, void *segs,
                           uint32_t *sizes, hipStream_t st);
hipError_t index_seg_setoff(void *segs, uint64_t M, const uint64_t *offsets, hipStream_t st);
// Position range and recorded errors of every cell.
hipError_t index_cells(const float *d_pw, const RankFeat &rf, int lg, const uint64_t *reps, int64_t D, const void *segs,
                       uint64_t n_cells, uint32_t *first, uint32_t *last, uint32_t *elo, uint32_t *ehi, int blocks,
                       hipStream_t st);
// Raise the factor of segments with a cell window wider than `window`.
hipError_t index_refine(uint64_t M, const void *segs, const uint32_t *sizes, const uint32_t *first,
                        const uint32_t *last, const uint32_t *elo, const uint32_t *ehi, uint32_t window, uint32_t fmax,
                        uint32_t *factor, unsigned int *count, hipStream_t st);
hipError_t index_pack(uint64_t n_cells, const uint32_t *first, const uint32_t *last, const uint32_t *elo,
                      const uint32_t *ehi, void *cells, uint32_t *bad, hipStream_t st);
// stats (5 counters, cleared by the caller) and the largest window.
hipError_t index_window_stats(const float *d_pw, const RankFeat &rf, int lg, const uint64_t *reps, int64_t D,
                              const void *segs, const void *cells, uint64_t n_cells, unsigned long long *stats,
                              uint32_t *max_win, int blocks, hipStream_t st);
hipError_t index_predict(const float *d_pw, const RankFeat &rf, int N, const uint64_t *keys, int64_t n, float *u,
                         float *y, hipStream_t st);

// Build targets: keys per cell, widest recorded window (keys), refinement
// rounds and the largest refinement factor of a segment.
constexpr uint32_t kKeysPerCell = 64;
constexpr uint32_t kMaxWindow = 16;
constexpr int kRefineRounds = 5;
constexpr uint32_t kMaxRefine = 1024;

}  // namespace symed
