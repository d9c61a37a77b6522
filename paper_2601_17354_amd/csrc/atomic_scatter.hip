// Float-atomic throughput reference for the render backward's gradient
// scatter (the index-mapped "+=" into the 2D gradient records): the same
// instruction (a float add without return into a 64-byte record of nine
// fields), issued in the same pattern as the backward's per-batch flush -
// a workgroup takes 256 consecutive targets and its threads walk the
// 256 x 9 (target, field) adds with consecutive threads on consecutive
// fields.  With the backward's own target list (the sorted pair values)
// the contention matches the backward's: each record is hit once per tile
// the Gaussian touches.  A measurement aid, not part of the method.
#include "common.hpp"

namespace {

constexpr int kTargetsPerGroup = 256;

__global__ __launch_bounds__(256) void k_atomic_scatter(float* __restrict__ records, uint32_t n_records,
                                                        const uint32_t* __restrict__ targets, uint32_t n_targets) {
    const uint32_t t0 = blockIdx.x * (uint32_t)kTargetsPerGroup;
    const uint32_t nb = min((uint32_t)kTargetsPerGroup, n_targets - t0);
    for (uint32_t idx = threadIdx.x; idx < nb * PGS_GRAD2D_FIELDS; idx += blockDim.x) {
        const uint32_t j = idx / PGS_GRAD2D_FIELDS, f = idx - j * PGS_GRAD2D_FIELDS;
        const uint32_t r = targets[t0 + j];
        if (r < n_records) unsafeAtomicAdd(&records[(size_t)r * PGS_GRAD2D_STRIDE + f], 1.0f);
    }
}

}  // namespace

extern "C" pgs_status pgs_atomic_scatter(float* records_dev, uint32_t n_records, const uint32_t* targets_dev,
                                         uint32_t n_targets, void* stream) {
    if (n_targets == 0) return PGS_OK;
    PGS_REQUIRE(records_dev && targets_dev, "pgs_atomic_scatter: null pointer");
    const uint32_t groups = (n_targets + kTargetsPerGroup - 1) / kTargetsPerGroup;
    k_atomic_scatter<<<groups, 256, 0, pgs::as_stream(stream)>>>(records_dev, n_records, targets_dev, n_targets);
    PGS_CHECK_LAUNCH("pgs_atomic_scatter");
    return PGS_OK;
}
