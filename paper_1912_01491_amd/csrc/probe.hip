// Read-stream bandwidth of the device: the practical ceiling that the
// HBM-bound kernels are compared with, next to the published peak. A
// reduction over a buffer with 16-byte nontemporal loads, timed with HIP
// events over several grid sizes; the best rate is reported.
#include "lb_internal.h"

#include <algorithm>

namespace {

typedef double lb_d2v __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_read_stream(const double* a, int64_t n2, double* out) {
    double s = 0.0;
    const lb_d2v* p = (const lb_d2v*)a;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
        const lb_d2v v = __builtin_nontemporal_load((const lb_d2v __attribute__((address_space(1)))*)(p + i));
        s += v.x + v.y;
    }
    if (s == 1.0e300) out[0] = s;  // the buffer is zero: never taken, keeps the loads
}

struct Buf {
    void* p = nullptr;
    ~Buf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

int lb_impl_read_bandwidth(lb_ctx* c, size_t bytes, double* gbs) {
    hipStream_t s = c->stream;
    const int64_t n = (int64_t)(bytes / 16) * 2;  // doubles, a whole number of 16-byte pairs
    Buf buf, out;
    if (hipMalloc(&buf.p, (size_t)n * 8) != hipSuccess || hipMalloc(&out.p, 8) != hipSuccess) {
        (void)hipGetLastError();
        return lb_fail(LB_ERR_OOM, "probe buffer of %zu bytes", bytes);
    }
    LB_HIP(hipMemsetAsync(buf.p, 0, (size_t)n * 8, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LB_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return lb_fail(LB_ERR_DEVICE, "event creation failed");
    }
    double best = 0.0;
    int rc = LB_OK;
    const int reps = 5;
    for (int blocks : {1024, 2048, 4096, 8192, 32768}) {
        for (int r = 0; r < reps + 1 && !rc; ++r) {
            if (r == 1 && hipEventRecord(e0, s) != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "event record failed");
            hipLaunchKernelGGL(k_read_stream, dim3(blocks), dim3(256), 0, s, (const double*)buf.p, n / 2,
                               (double*)out.p);
            if (hipGetLastError() != hipSuccess) rc = lb_fail(LB_ERR_DEVICE, "probe launch failed");
        }
        float ms = 0.0f;
        if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = lb_fail(LB_ERR_DEVICE, "probe timing failed");
        if (rc) break;
        best = std::max(best, reps * (double)n * 8.0 / (ms * 1e-3) / 1e9);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *gbs = best;
    return LB_OK;
}
