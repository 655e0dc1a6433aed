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

// Eight independent accumulator chains of matrix-core products per wavefront:
// the attainable matrix-core rate for the benchmark's roofline (not part of
// the scheme).  kind 0: v_mfma_f64_16x16x4f64 (2048 flops each); kind 1:
// v_mfma_f32_16x16x32_bf16 (16384 flops each).  Each lane writes its sum.
typedef __bf16 probe_bf16x8 __attribute__((ext_vector_type(8)));
typedef float probe_f32x4 __attribute__((ext_vector_type(4)));
typedef double probe_f64x4 __attribute__((ext_vector_type(4)));

template <int KIND>
__global__ __launch_bounds__(256) void mfma_probe(double *__restrict__ sink, int iters)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if constexpr (KIND == 0) {
        const double a = 1e-3 * (double)(threadIdx.x % 16), b = 0.5;
        probe_f64x4 acc[8];
#pragma unroll
        for (int j = 0; j < 8; j++) acc[j] = probe_f64x4{0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < iters; i++)
#pragma unroll
            for (int j = 0; j < 8; j++) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 8; j++) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    } else {
        probe_bf16x8 a, b;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            a[e] = (__bf16)(0.001f * (float)((threadIdx.x + e) % 16));
            b[e] = (__bf16)0.5f;
        }
        probe_f32x4 acc[8];
#pragma unroll
        for (int j = 0; j < 8; j++) acc[j] = probe_f32x4{0.f, 0.f, 0.f, 0.f};
        for (int i = 0; i < iters; i++)
#pragma unroll
            for (int j = 0; j < 8; j++) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 8; j++) s += (double)(acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3]);
    }
    sink[t] = s;
}

rg_status launch_mfma_probe(double *sink, long long n_threads, int iters, int kind, void *stream)
{
    if (n_threads <= 0 || n_threads % 256 != 0 || iters <= 0 || (kind != 0 && kind != 1)) {
        set_error("mfma probe: n_threads must be a positive multiple of 256, iters positive, kind 0 or 1");
        return RG_EINVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned nb = (unsigned)(n_threads / 256);
    if (kind == 0) mfma_probe<0><<<nb, 256, 0, st>>>(sink, iters);
    else mfma_probe<1><<<nb, 256, 0, st>>>(sink, iters);
    if (hipGetLastError() != hipSuccess) {
        set_error("mfma probe launch failed");
        return RG_EDEVICE;
    }
    return RG_OK;
}

}  // namespace rg
