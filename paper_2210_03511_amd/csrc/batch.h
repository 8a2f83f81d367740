// Descriptors and launchers of the batched (many-sector) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "launch.h"

namespace symed {

constexpr int kMaxSectors = 256;

// One sector of a batch (device-resident array of these).
struct SectorDesc {
    KParams p;
    const double *x;  // ed_batch_apply input
    double *y;        // ed_batch_apply output
    double *v, *w, *vprev;
    double *alpha, *beta;
    LState *ls;
    const uint32_t *pos2slot;  // hashed staging table: slot of each row (lookup kind 2)
    int64_t tile0;    // first tile of the sector
    int64_t ntiles;
    int32_t cplx;
    int32_t pad;
};

hipError_t batch_prepare(size_t lds_bytes);
hipError_t batch_occupancy(size_t lds_bytes, int *blocks_per_cu);
// lookup: 0 plain, 1 learned, 2 hashed staging table (for 1 and 2 the input
// vectors are copied into the sectors' records first)
hipError_t launch_batch_apply(const SectorDesc *d_secs, int nsec, const int64_t *d_tile0, int64_t ntiles,
                              int64_t tile_rows, int lanczos, int lookup, double *partials, int blocks, size_t lds,
                              int vec_blocks, hipStream_t st);
hipError_t launch_batch_step(const SectorDesc *d_secs, int nsec, const int64_t *d_tile0, int64_t ntiles,
                             int64_t tile_rows, int lookup, double *partials, int apply_blocks, int vec_blocks,
                             size_t lds, hipStream_t st);

}  // namespace symed
