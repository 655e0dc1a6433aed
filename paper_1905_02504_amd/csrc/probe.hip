// Benchmark helper (not part of the scheme): the attainable FP64 vector rate.
#include "rg_geom_host.hpp"
#include "rg_internal.hpp"

#include <hip/hip_runtime.h>

namespace rg {

// Sixteen independent FMA chains per lane: the attainable FP64 vector rate for
// the benchmark's roofline (not part of the scheme).  Each lane writes its sum.
__global__ __launch_bounds__(256) void fma_probe(double *__restrict__ sink, int iters)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double a[16];
#pragma unroll
    for (int j = 0; j < 16; j++) a[j] = 1e-3 * (double)(threadIdx.x + j);
    const double m = 0.9999999, c = 1e-9;
    for (int i = 0; i < iters; i++)
#pragma unroll
        for (int j = 0; j < 16; j++) a[j] = fma(a[j], m, c);
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 16; j++) s += a[j];
    sink[t] = s;
}

rg_status launch_fma_probe(double *sink, long long n_threads, int iters, void *stream)
{
    if (n_threads <= 0 || n_threads % 256 != 0 || iters <= 0) {
        set_error("fma probe: n_threads must be a positive multiple of 256 and iters positive");
        return RG_EINVAL;
    }
    fma_probe<<<(unsigned)(n_threads / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(sink, iters);
    if (hipGetLastError() != hipSuccess) {
        set_error("fma probe launch failed");
        return RG_EDEVICE;
    }
    return RG_OK;
}

}  // namespace rg
