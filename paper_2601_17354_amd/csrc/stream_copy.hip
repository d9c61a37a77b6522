// Streaming copy used as the measured "achievable HBM bandwidth" reference
// and to calibrate hardware traffic counters against a kernel whose bytes
// are known exactly (reads n*16 B, writes n*16 B).
#include "common.hpp"

namespace {

// Each lane moves four 16-byte words 256 words apart per step, so four loads
// are in flight before the first store.
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                size_t n) {
    const size_t stride = (size_t)gridDim.x * 1024;
    for (size_t i = blockIdx.x * (size_t)1024 + threadIdx.x; i < n; i += stride) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + 256 * k < n) v[k] = src[i + 256 * k];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + 256 * k < n) dst[i + 256 * k] = v[k];
    }
}

}  // namespace

extern "C" pgs_status pgs_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream) {
    PGS_REQUIRE(bytes % 16 == 0, "pgs_stream_copy: bytes must be a multiple of 16");
    if (bytes == 0) return PGS_OK;
    PGS_REQUIRE(src_dev && dst_dev, "pgs_stream_copy: null pointer");
    PGS_REQUIRE(((uintptr_t)src_dev % 16) == 0 && ((uintptr_t)dst_dev % 16) == 0,
                "pgs_stream_copy: pointers must be 16-byte aligned");
    const size_t n = bytes / 16;
    // one 1024-word chunk per workgroup up to 65536 workgroups (measured best
    // on MI355X), grid-stride beyond that
    size_t blocks = (n + 1023) / 1024;
    if (blocks > 65536) blocks = 65536;
    k_copy16<<<(unsigned)blocks, 256, 0, pgs::as_stream(stream)>>>(static_cast<const uint4*>(src_dev),
                                                                  static_cast<uint4*>(dst_dev), n);
    PGS_CHECK_LAUNCH("pgs_stream_copy");
    return PGS_OK;
}
