// Random-gather probe: the rate of dependent random 16-byte reads the memory system sustains
// for the access pattern of a walk step (one aligned record at a hashed position of a buffer
// much larger than the Infinity Cache).  It prices the walk kernels against a measured
// random-access ceiling as well as against the streaming peak.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "saba_internal.hpp"

namespace saba {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeBlocks = 8192;

__global__ void probe_fill_kernel(int4 *__restrict__ buf, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t h = mm2_final(mm2_block(0x1234567u, (uint32_t)i));
        buf[i] = make_int4((int32_t)h, (int32_t)(h * 3u), (int32_t)(h * 5u), 0);
    }
}

// Every lane follows its own chain: position k + 1 is derived from the record read at k.
__global__ __launch_bounds__(kProbeBlock) void probe_chase_kernel(const int4 *__restrict__ buf,
                                                                  uint64_t mask, int32_t steps,
                                                                  uint32_t *__restrict__ sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t x = mm2_final(mm2_block(0x9E3779B9u, tid));
    for (int32_t s = 0; s < steps; ++s) {
        const int4 v = buf[(uint64_t)x & mask];
        x = mm2_final((uint32_t)v.x ^ (x + (uint32_t)s));
    }
    if (x == 0x5A5A5A5Au) sink[tid & 1023] = x;  // keeps the chain live
}

}  // namespace
}  // namespace saba

using namespace saba;

extern "C" int saba_probe_random_reads(int32_t log2_records, int32_t steps, double *reads_per_s,
                                       double *ms, void *stream) {
    clear_error();
    if (log2_records < 10 || log2_records > 30 || steps < 1 || steps > 4096 || !reads_per_s) {
        set_error("invalid probe arguments");
        return SABA_E_INVALID;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = (int64_t)1 << log2_records;
    DevBuf buf, sink;
    struct Guard {
        DevBuf *a, *b;
        ~Guard() {
            a->release();
            b->release();
        }
    } guard{&buf, &sink};
    SABA_TRY(buf.ensure(sizeof(int4) * (size_t)n));
    SABA_TRY(sink.ensure(sizeof(uint32_t) * 1024));
    probe_fill_kernel<<<4096, 256, 0, s>>>(buf.as<int4>(), n);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SABA_HIP_TRY(hipEventCreate(&e0));
    SABA_HIP_TRY(hipEventCreate(&e1));
    // warm-up, then the timed launch
    probe_chase_kernel<<<kProbeBlocks, kProbeBlock, 0, s>>>(buf.as<int4>(), (uint64_t)(n - 1), steps,
                                                            sink.as<uint32_t>());
    SABA_HIP_TRY(hipEventRecord(e0, s));
    probe_chase_kernel<<<kProbeBlocks, kProbeBlock, 0, s>>>(buf.as<int4>(), (uint64_t)(n - 1), steps,
                                                            sink.as<uint32_t>());
    SABA_HIP_TRY(hipEventRecord(e1, s));
    SABA_HIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    SABA_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    SABA_HIP_TRY(hipGetLastError());
    const double reads = (double)kProbeBlocks * kProbeBlock * steps;
    *reads_per_s = reads / (t * 1e-3);
    if (ms) *ms = t;
    return SABA_OK;
}
