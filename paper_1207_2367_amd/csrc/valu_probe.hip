// Measurement probe for the roofline denominators of the evaluation
// kernel: the rounding of v_rsq_f32 and v_rsq_f64 against the exact 1/sqrt
// over [1, 4), and the sustained VALU throughput of single instruction kinds
// (FP32 FMA and MUL, FP64 FMA and ADD, v_rsq_f32, v_rsq_f64, FP64->FP32
// conversion) with 4, 8 or 16 independent chains per lane, and of FP32 and
// FP64 FMA chains interleaved (do the two kinds overlap in issue?).  Every
// buffer is sized for its grid.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cmath>
#include <vector>
#define CK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s line %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

__global__ void rsq_probe(const float *x, float *y0, float *y1, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = x[i];
    float r = __builtin_amdgcn_rsqf(v);
    y0[i] = r;
    float e = fmaf(-v * r, r, 1.0f);
    y1[i] = fmaf(0.5f * r, e, r);
}

__global__ void rsq64_probe(const double *x, double *y, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = __builtin_amdgcn_rsq(x[i]);
}

template <int K>
__global__ void fma32(float *out, float a, float b, int iters) {
    float x[K];
    for (int k = 0; k < K; ++k) x[k] = threadIdx.x * 0.001f + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = fmaf(x[k], a, b);
    }
    float s = 0; for (int k = 0; k < K; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void fma64(double *out, double a, double b, int iters) {
    double x[8];
    for (int k = 0; k < 8; ++k) x[k] = threadIdx.x * 0.001 + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fma(x[k], a, b);
    }
    double s = 0; for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void add64(double *out, double a, int iters) {
    double x[8];
    for (int k = 0; k < 8; ++k) x[k] = threadIdx.x * 0.001 + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = x[k] + a;
    }
    double s = 0; for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void rsq32(float *out, float a, int iters) {
    float x[8];
    for (int k = 0; k < 8; ++k) x[k] = 1.0f + threadIdx.x * 0.001f + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_rsqf(x[k]) + a;
    }
    float s = 0; for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void rsq64(double *out, double a, int iters) {
    double x[8];
    for (int k = 0; k < 8; ++k) x[k] = 1.0 + threadIdx.x * 0.001 + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_rsq(x[k]) + a;
    }
    double s = 0; for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
// 4 FP32 and 4 FP64 independent FMA chains interleaved: 8 lane-ops per
// iteration, as in the other kernels
__global__ void fma_mix(double *out, float af, float bf, double ad, double bd, int iters) {
    float x[4]; double y[4];
    for (int k = 0; k < 4; ++k) { x[k] = threadIdx.x * 0.001f + k; y[k] = threadIdx.x * 0.002 + k; }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 4; ++k) { x[k] = fmaf(x[k], af, bf); y[k] = fma(y[k], ad, bd); }
    }
    double s = 0; for (int k = 0; k < 4; ++k) s += x[k] + y[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void cvt_probe(float *out, double a, int iters) {
    double x[8]; float y[8];
    for (int k = 0; k < 8; ++k) { x[k] = threadIdx.x * 0.001 + k; y[k] = 0; }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) { y[k] += (float)(x[k]); x[k] = x[k] + a; }
    }
    float s = 0; for (int k = 0; k < 8; ++k) s += y[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
__global__ void mul32(float *out, float a, int iters) {
    float x[8];
    for (int k = 0; k < 8; ++k) x[k] = 1.0f + threadIdx.x * 0.001f + k;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = x[k] * a;
    }
    float s = 0; for (int k = 0; k < 8; ++k) s += x[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main() {
    int dev; CK(hipGetDevice(&dev));
    hipDeviceProp_t p; CK(hipGetDeviceProperties(&p, dev));
    printf("device %s CUs %d clock %d kHz LDS/block %zu LDS/CU(max shared per MP) %zu l2 %d\n", p.name, p.multiProcessorCount, p.clockRate, p.sharedMemPerBlock, p.maxSharedMemoryPerMultiProcessor, p.l2CacheSize);
    // rsq probe: x uniform in [1,4)
    const int n = 1 << 22;
    std::vector<float> hx(n);
    for (int i = 0; i < n; ++i) hx[i] = 1.0f + 3.0f * (float)i / n;
    float *dx, *dy0, *dy1;
    CK(hipMalloc(&dx, n * 4)); CK(hipMalloc(&dy0, n * 4)); CK(hipMalloc(&dy1, n * 4));
    CK(hipMemcpy(dx, hx.data(), n * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(rsq_probe, dim3(n / 256), dim3(256), 0, 0, dx, dy0, dy1, n);
    CK(hipGetLastError());
    std::vector<float> y0(n), y1(n);
    CK(hipMemcpy(y0.data(), dy0, n * 4, hipMemcpyDeviceToHost));
    CK(hipMemcpy(y1.data(), dy1, n * 4, hipMemcpyDeviceToHost));
    double s0 = 0, s1 = 0, m0 = 0, m1 = 0, sr = 0, mr = 0;
    for (int i = 0; i < n; ++i) {
        double ex = 1.0 / std::sqrt((double)hx[i]);
        double ulp = std::ldexp(1.0, std::ilogb((float)ex) - 23);
        double e0 = (y0[i] - ex) / ulp, e1 = (y1[i] - ex) / ulp;
        double er = ((double)(float)ex - ex) / ulp;
        s0 += e0; s1 += e1; sr += er;
        m0 = std::fmax(m0, std::fabs(e0)); m1 = std::fmax(m1, std::fabs(e1)); mr = std::fmax(mr, std::fabs(er));
    }
    printf("rsq ulp error: raw mean %.4f max %.3f | newton mean %.4f max %.3f | correctly-rounded mean %.4f max %.3f\n",
           s0 / n, m0, s1 / n, m1, sr / n, mr);
    // v_rsq_f64 on the same inputs, against a long-double reference
    {
        std::vector<double> hxd(n), hy(n);
        for (int i = 0; i < n; ++i) hxd[i] = 1.0 + 3.0 * (double)i / n + 1e-9 * (i % 7);
        double *dxd, *dyd;
        CK(hipMalloc(&dxd, n * 8)); CK(hipMalloc(&dyd, n * 8));
        CK(hipMemcpy(dxd, hxd.data(), n * 8, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(rsq64_probe, dim3(n / 256), dim3(256), 0, 0, dxd, dyd, n);
        CK(hipGetLastError());
        CK(hipMemcpy(hy.data(), dyd, n * 8, hipMemcpyDeviceToHost));
        double sm = 0, mx = 0;
        for (int i = 0; i < n; ++i) {
            const long double ex = 1.0L / std::sqrt((long double)hxd[i]);
            const double ulp = std::ldexp(1.0, std::ilogb((double)ex) - 52);
            const double e = (double)(((long double)hy[i] - ex) / ulp);
            sm += e; mx = std::fmax(mx, std::fabs(e));
        }
        printf("rsq64 ulp error: mean %.3g max %.4g (relative max %.3g)\n", sm / n, mx, mx * std::ldexp(1.0, -52));
        CK(hipFree(dxd)); CK(hipFree(dyd));
    }
    // throughput
    const int blocks = 256 * 8 * 4, threads = 256, iters = 4096;
    float *of; double *od;
    CK(hipMalloc(&of, blocks * threads * 4)); CK(hipMalloc(&od, blocks * threads * 8));
    hipEvent_t a, b; CK(hipEventCreate(&a)); CK(hipEventCreate(&b));
    auto timeit = [&](const char *name, auto launch, double flops_per_op) {
        launch(); CK(hipDeviceSynchronize());
        CK(hipEventRecord(a)); launch(); CK(hipEventRecord(b)); CK(hipEventSynchronize(b));
        float ms; CK(hipEventElapsedTime(&ms, a, b));
        double ops = (double)blocks * threads * iters * 8;
        printf("%-8s %.3f ms  %.2f T lane-ops/s  %.2f TFLOP/s\n", name, ms, ops / ms / 1e9, ops * flops_per_op / ms / 1e9);
        return 0;
    };
    timeit("fma32", [&] { hipLaunchKernelGGL(fma32<8>, dim3(blocks), dim3(threads), 0, 0, of, 0.999f, 0.001f, iters); }, 2);
    timeit("fma32x16", [&] { hipLaunchKernelGGL(fma32<16>, dim3(blocks), dim3(threads), 0, 0, of, 0.999f, 0.001f, iters / 2); }, 2);
    timeit("fma32x4", [&] { hipLaunchKernelGGL(fma32<4>, dim3(blocks), dim3(threads), 0, 0, of, 0.999f, 0.001f, iters * 2); }, 2);
    timeit("mul32", [&] { hipLaunchKernelGGL(mul32, dim3(blocks), dim3(threads), 0, 0, of, 0.999f, iters); }, 1);
    timeit("fma64", [&] { hipLaunchKernelGGL(fma64, dim3(blocks), dim3(threads), 0, 0, od, 0.999, 0.001, iters); }, 2);
    timeit("add64", [&] { hipLaunchKernelGGL(add64, dim3(blocks), dim3(threads), 0, 0, od, 0.001, iters); }, 1);
    timeit("rsq32", [&] { hipLaunchKernelGGL(rsq32, dim3(blocks), dim3(threads), 0, 0, of, 0.001f, iters); }, 1);
    timeit("rsq64", [&] { hipLaunchKernelGGL(rsq64, dim3(blocks), dim3(threads), 0, 0, od, 0.001, iters); }, 1);
    timeit("fma32|64", [&] { hipLaunchKernelGGL(fma_mix, dim3(blocks), dim3(threads), 0, 0, od, 0.999f, 0.001f, 0.999, 0.001, iters); }, 2);
    timeit("cvt+add", [&] { hipLaunchKernelGGL(cvt_probe, dim3(blocks), dim3(threads), 0, 0, of, 0.001, iters); }, 1);
    CK(hipFree(dx)); CK(hipFree(dy0)); CK(hipFree(dy1)); CK(hipFree(of)); CK(hipFree(od));
    return 0;
}
