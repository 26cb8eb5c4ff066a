// Radix-16 DFT throughput on gfx950: the VALU butterflies of the solver's
// passes (DFT<16> in psn_device.h) against a 16-point DFT as a dense complex
// matrix product on FP32 MFMA (v_mfma_f32_16x16x4f32), data resident in
// registers.  A 16-point DFT of 16 columns is [Yr; Yi] = [Fr -Fi; Fi Fr] [Xr; Xi]:
// two 16x32 by 32x16 real products, 16 MFMA instructions.  The MFMA side does
// not model the lane permutations a pass would need between stages, so it is
// an upper bound for MFMA.  Prints one line of key=value pairs.
#include "../psn_device.h"
#include <cmath>
#include <cstdio>
#include <vector>
using namespace psn;
typedef float f4 __attribute__((ext_vector_type(4)));

// A operands for one 16-point forward DFT block: lane l, k-step s (0..7):
// rows i = l % 16; stacked column c = 4 s + l / 16 of [Fr, -Fi] (Yr) and [Fi, Fr] (Yi)
__device__ void dft_A(int lane, float (&ar)[8], float (&ai)[8]) {
    const int i = lane % 16, g = lane / 16;
    for (int s = 0; s < 8; ++s) {
        const int c = 4 * s + g;            // 0..31
        const int k = c % 16;
        const double ang = -2.0 * M_PI * double(i * k % 16) / 16.0;
        const float fr = float(cos(ang)), fi = float(sin(ang));
        ar[s] = c < 16 ? fr : -fi;          // [Fr, -Fi]
        ai[s] = c < 16 ? fi : fr;           // [Fi,  Fr]
    }
}

// x[s]: lane (g = l/16, j = l%16) holds stacked row 4 s + g of column j
// (rows 0..15 real parts, 16..31 imaginary parts)
__device__ void dft16_mfma(const float (&ar)[8], const float (&ai)[8], const float (&x)[8], f4& yr, f4& yi) {
    yr = f4{0.f, 0.f, 0.f, 0.f};
    yi = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        yr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[s], x[s], yr, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[s], x[s], yi, 0, 0, 0);
    }
}

// correctness: one block of 16 DFTs; in[j][k] complex, out[j][k]
__global__ void check(const float* in, float* out) {
    const int l = threadIdx.x, g = l / 16, j = l % 16;
    float ar[8], ai[8], x[8];
    dft_A(l, ar, ai);
    for (int s = 0; s < 8; ++s) {
        const int row = 4 * s + g;          // stacked row
        x[s] = row < 16 ? in[(j * 16 + row) * 2] : in[(j * 16 + row - 16) * 2 + 1];
    }
    f4 yr, yi;
    dft16_mfma(ar, ai, x, yr, yi);
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * g + v;
        out[(j * 16 + i) * 2] = yr[v];
        out[(j * 16 + i) * 2 + 1] = yi[v];
    }
}

__global__ void bench_valu(float* sink, int iters) {
    cx<float> v[16];
    for (int k = 0; k < 16; ++k) v[k] = {float(threadIdx.x + k), float(k)};
    for (int it = 0; it < iters; ++it) {
        DFT<16, -1, float>::run(v);
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = scale(v[k], 0.0625f);
    }
    float s = 0.f;
    for (int k = 0; k < 16; ++k) s += v[k].x + v[k].y;
    if (s == 1234.5f) sink[threadIdx.x] = s;   // keeps the work alive; in bounds
}

__global__ void bench_mfma(float* sink, int iters) {
    float ar[8], ai[8], x[8];
    dft_A(threadIdx.x % 64, ar, ai);
    for (int s = 0; s < 8; ++s) x[s] = float(threadIdx.x + s);
    for (int it = 0; it < iters; ++it) {
        f4 yr, yi;
        dft16_mfma(ar, ai, x, yr, yi);
        // feed the outputs back (layout permutation not modelled)
        for (int v = 0; v < 4; ++v) { x[v] = yr[v] * 0.0625f; x[4 + v] = yi[v] * 0.0625f; }
    }
    float s = 0.f;
    for (int k = 0; k < 8; ++k) s += x[k];
    if (s == 1234.5f) sink[threadIdx.x] = s;
}

int main() {
    // correctness of the MFMA mapping
    std::vector<float> hin(16 * 16 * 2), hout(16 * 16 * 2);
    for (size_t i = 0; i < hin.size(); ++i) hin[i] = float(std::sin(0.37 * i) + 0.1 * i / hin.size());
    float *din, *dout, *sink;
    if (hipMalloc(&din, hin.size() * 4) != hipSuccess || hipMalloc(&dout, hout.size() * 4) != hipSuccess ||
        hipMalloc(&sink, 1 << 20) != hipSuccess) {
        printf("status=alloc_failed\n");
        return 1;
    }
    hipMemcpy(din, hin.data(), hin.size() * 4, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(check, dim3(1), dim3(64), 0, 0, din, dout);
    hipMemcpy(hout.data(), dout, hout.size() * 4, hipMemcpyDeviceToHost);
    double err = 0, mx = 0;
    for (int j = 0; j < 16; ++j)
        for (int k = 0; k < 16; ++k) {
            double re = 0, im = 0;
            for (int m = 0; m < 16; ++m) {
                const double a = -2 * M_PI * m * k / 16.0;
                const double xr = hin[(j * 16 + m) * 2], xi = hin[(j * 16 + m) * 2 + 1];
                re += xr * cos(a) - xi * sin(a);
                im += xr * sin(a) + xi * cos(a);
            }
            err = fmax(err, fabs(re - hout[(j * 16 + k) * 2]) + fabs(im - hout[(j * 16 + k) * 2 + 1]));
            mx = fmax(mx, fabs(re) + fabs(im));
        }
    const double rel = err / mx;
    // throughput
    const int blocks = 256 * 8, threads = 256, iters = 2000;
    hipEvent_t a, b; hipEventCreate(&a); hipEventCreate(&b);
    float ms;
    hipLaunchKernelGGL(bench_valu, dim3(blocks), dim3(threads), 0, 0, sink, 10);
    hipEventRecord(a); hipLaunchKernelGGL(bench_valu, dim3(blocks), dim3(threads), 0, 0, sink, iters); hipEventRecord(b);
    hipEventSynchronize(b); hipEventElapsedTime(&ms, a, b);
    const double dv = double(blocks) * threads * iters;          // one DFT-16 per lane per iteration
    const double valu = dv / ms * 1e3;
    hipLaunchKernelGGL(bench_mfma, dim3(blocks), dim3(threads), 0, 0, sink, 10);
    hipEventRecord(a); hipLaunchKernelGGL(bench_mfma, dim3(blocks), dim3(threads), 0, 0, sink, iters); hipEventRecord(b);
    hipEventSynchronize(b); hipEventElapsedTime(&ms, a, b);
    const double dm = double(blocks) * (threads / 64) * 16 * iters;   // 16 DFT-16 per wave per iteration
    const double mfma = dm / ms * 1e3;
    const hipError_t e = hipGetLastError();
    printf("valu_dft16_per_s=%.4e mfma_dft16_per_s=%.4e mfma_tflops=%.2f mfma_rel_err=%.3e hip_status=%d\n", valu, mfma,
           dm * 2048 / ms / 1e9, rel, int(e));
    return e == hipSuccess ? 0 : 1;
}
