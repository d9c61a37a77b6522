// Host-side helpers of the C ABI around the kernels: reading the device
// overflow flags, and recording a sequence of library calls on a stream as
// a HIP graph that can be replayed.
#include <new>

#include "common.hpp"

struct pgs_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

pgs_status hip_fail(const char* what, hipError_t e) {
    pgs::set_error("%s: %s", what, hipGetErrorString(e));
    return PGS_ERR_HIP;
}

}  // namespace

extern "C" pgs_status pgs_check_flags(const uint32_t* flags_dev, uint32_t* flags_host, void* stream) {
    PGS_REQUIRE(flags_dev && flags_host, "pgs_check_flags: null pointer");
    hipStream_t s = pgs::as_stream(stream);
    hipError_t e = hipMemcpyAsync(flags_host, flags_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail("pgs_check_flags: copy", e);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail("pgs_check_flags: synchronise", e);
    const uint32_t f = *flags_host;
    if (f & (PGS_FLAG_PAIR_OVERFLOW | PGS_FLAG_CACHE_OVERFLOW)) {
        pgs::set_error("pgs_check_flags: capacity overflow (flags 0x%x:%s%s)", f,
                       (f & PGS_FLAG_PAIR_OVERFLOW) ? " pairs" : "",
                       (f & PGS_FLAG_CACHE_OVERFLOW) ? " trace" : "");
        return PGS_ERR_CAPACITY;
    }
    return PGS_OK;
}

extern "C" pgs_status pgs_graph_begin(void* stream) {
    PGS_REQUIRE(stream != nullptr, "pgs_graph_begin: the null stream cannot be captured");
    const hipError_t e = hipStreamBeginCapture(pgs::as_stream(stream), hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail("pgs_graph_begin", e);
    return PGS_OK;
}

extern "C" pgs_status pgs_graph_end(void* stream, pgs_graph** graph_out) {
    PGS_REQUIRE(stream != nullptr && graph_out != nullptr, "pgs_graph_end: null pointer");
    *graph_out = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(pgs::as_stream(stream), &g);
    if (e != hipSuccess) return hip_fail("pgs_graph_end: end capture", e);
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail("pgs_graph_end: instantiate", e);
    }
    pgs_graph* h = new (std::nothrow) pgs_graph{g, x};
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        pgs::set_error("pgs_graph_end: out of host memory");
        return PGS_ERR_HIP;
    }
    *graph_out = h;
    return PGS_OK;
}

extern "C" pgs_status pgs_graph_launch(const pgs_graph* graph, void* stream) {
    PGS_REQUIRE(graph != nullptr, "pgs_graph_launch: null graph");
    const hipError_t e = hipGraphLaunch(graph->exec, pgs::as_stream(stream));
    if (e != hipSuccess) return hip_fail("pgs_graph_launch", e);
    return PGS_OK;
}

extern "C" void pgs_graph_destroy(pgs_graph* graph) {
    if (!graph) return;
    (void)hipGraphExecDestroy(graph->exec);
    (void)hipGraphDestroy(graph->graph);
    delete graph;
}
