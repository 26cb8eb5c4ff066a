// Kernel-spectrum build in FP64 on the device (paper section 2: the G-tensor
// and the near-zone correction; section 3: it is the setup phase).
//
//   a_j(k)   = 2 int_0^T exp(-tau_j^2 y^2) cos(kappa_k y) dy,  kappa_k = 2 pi k / (2 n h)
//   C0, C2   = int_{B_delta} (U - U_GS) dy,  int_{B_delta} |y|^2 (U - U_GS) dy
//   K(k)     = sum_j w_j a_j(k0) a_j(k1) a_j(k2) + C0 - (C2/6) |kappa|^2
//
// The mode integrals use the Gaussian's Fourier transform where the tail
// beyond T is below exp(-37) (tau T >= 6.1) and composite 16-point
// Gauss-Legendre elsewhere, with one panel per half period of the highest
// frequency plus eight; for tau T < 1 the integrand is split into cos(kappa y)
// (integral exactly 2T at k = 0 and 0 otherwise, since kappa T = pi k) plus the
// smooth remainder expm1(-tau^2 y^2) cos(kappa y).
#include "psn_device.h"
#include "psn_internal.h"

namespace psn {

constexpr double kPi = 3.14159265358979323846;

__global__ void k_modes(const double* __restrict__ tau, int n, double T, double period,
                        const double* __restrict__ glx, const double* __restrict__ glw, double* __restrict__ A) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k > n) return;
    const double t = tau[j];
    const double kap = 2.0 * kPi * double(k) / period;
    const double tT = t * T;
    double a;
    if (tT >= 6.1) {
        a = sqrt(kPi) / t * exp(-kap * kap / (4.0 * t * t));
    } else {
        const bool small = tT < 1.0;
        const int panels = n / 2 + 8;
        const double half = 0.5 * T / panels;
        double sum = 0.0;
        for (int pnl = 0; pnl < panels; ++pnl) {
            const double mid = (2 * pnl + 1) * half;
            double ps = 0.0;
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                const double y = mid + half * glx[g];
                const double ty = t * y;
                const double f = small ? expm1(-ty * ty) : exp(-ty * ty);
                ps += glw[g] * f * cos(kap * y);
            }
            sum += half * ps;
        }
        a = 2.0 * sum + ((small && k == 0) ? 2.0 * T : 0.0);
    }
    A[size_t(j) * (n + 1) + k] = a;
}

// int_0^delta r^p exp(-tau^2 r^2) dr for p = 2, 4
__device__ void radial_moments(double t, double delta, double& i2, double& i4) {
    const double x = t * delta;
    if (x < 0.5) {
        const double z = -x * x;
        double term = 1.0, s2 = 0.0, s4 = 0.0;
        for (int m = 0; m < 40; ++m) {
            s2 += term / (2 * m + 3);
            s4 += term / (2 * m + 5);
            term *= z / (m + 1);
        }
        const double d3 = delta * delta * delta;
        i2 = s2 * d3;
        i4 = s4 * d3 * delta * delta;
    } else {
        const double e = exp(-x * x), ef = erf(x), sp = sqrt(kPi);
        const double t2 = t * t;
        i2 = sp * ef / (4.0 * t2 * t) - delta * e / (2.0 * t2);
        i4 = 3.0 * sp * ef / (8.0 * t2 * t2 * t) - e * (3.0 * delta / (4.0 * t2 * t2) + delta * delta * delta / (2.0 * t2));
    }
}

__global__ void k_correction(const double* __restrict__ tau, const double* __restrict__ w, int terms, double delta,
                             double* __restrict__ out) {
    __shared__ double s2[256], s4[256];
    double a2 = 0.0, a4 = 0.0;
    for (int j = threadIdx.x; j < terms; j += blockDim.x) {
        double i2, i4;
        radial_moments(tau[j], delta, i2, i4);
        a2 += w[j] * i2;
        a4 += w[j] * i4;
    }
    s2[threadIdx.x] = a2;
    s4[threadIdx.x] = a4;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s2[threadIdx.x] += s2[threadIdx.x + h];
            s4[threadIdx.x] += s4[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = delta * delta / 2.0 - 4.0 * kPi * s2[0];
        out[1] = delta * delta * delta * delta / 4.0 - 4.0 * kPi * s4[0];
    }
}

// One workgroup per (k0~, k1~); threads run over k2 = 0..n.  A0, A1, A2 are the
// mode tables of the three axes (the same table for a cube).
template <class Kt>
__global__ void k_assemble(const double* __restrict__ A0, const double* __restrict__ A1,
                           const double* __restrict__ A2, const double* __restrict__ w, int terms, int n,
                           double p0, double p1, double p2, const double* __restrict__ Cc, double scale,
                           Kt* __restrict__ K, Kt* __restrict__ Kb) {
    extern __shared__ double cj[];
    __shared__ double edge[2];
    const int kt0 = blockIdx.x, kt1 = blockIdx.y;
    const int np1 = n + 1;
    for (int j = threadIdx.x; j < terms; j += blockDim.x)
        cj[j] = w[j] * A0[size_t(j) * np1 + kt0] * A1[size_t(j) * np1 + kt1];
    __syncthreads();
    const double C0 = Cc[0], C2 = Cc[1];
    const double b0 = 2.0 * kPi * kt0 / p0, b1 = 2.0 * kPi * kt1 / p1, b2 = 2.0 * kPi / p2;
    const double q01 = b0 * b0 + b1 * b1;
    for (int k2 = threadIdx.x; k2 <= n; k2 += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < terms; ++j) s = fma(cj[j], A2[size_t(j) * np1 + k2], s);
        const double v = s + C0 - (C2 / 6.0) * (q01 + b2 * b2 * double(k2) * k2);
        if (k2 == 0) edge[0] = v;
        else if (k2 == n) edge[1] = v;
        else K[psn_host::k_index(n, kt1, kt0, k2)] = Kt(scale * v);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        K[psn_host::k_index(n, kt1, kt0, 0)] = Kt(scale * 0.5 * (edge[0] + edge[1]));
        Kb[size_t(kt1) * np1 + kt0] = Kt(scale * 0.5 * (edge[0] - edge[1]));
    }
}

}  // namespace psn

namespace psn_host {

hipError_t launch_kernel_build(psn_plan* p, const double* d_tau, const double* d_w, int terms, const double* d_glx,
                               const double* d_glw, double* d_A, double* d_c, hipStream_t s) {
    const int n = p->n;
    const size_t tab = size_t(terms) * (n + 1);
    // one mode table per distinct axis length
    const double* A[3];
    for (int q = 0; q < 3; ++q) {
        int same = -1;
        for (int r = 0; r < q; ++r)
            if (p->T[r] == p->T[q] && p->period[r] == p->period[q]) same = r;
        if (same >= 0) {
            A[q] = A[same];
            continue;
        }
        A[q] = d_A + q * tab;
        hipLaunchKernelGGL(psn::k_modes, dim3((n + 1 + 127) / 128, terms), dim3(128), 0, s, d_tau, n, p->T[q],
                           p->period[q], d_glx, d_glw, d_A + q * tab);
    }
    hipLaunchKernelGGL(psn::k_correction, dim3(1), dim3(256), 0, s, d_tau, d_w, terms, p->delta, d_c);
    const double M = 2.0 * n;
    const double scale = 1.0 / (M * M * M);
    const size_t lds = size_t(terms) * sizeof(double);
    if (p->dtype == PSN_F32) {
        hipLaunchKernelGGL(psn::k_assemble<float>, dim3(n + 1, n + 1), dim3(256), lds, s, A[0], A[1], A[2], d_w,
                           terms, n, p->period[0], p->period[1], p->period[2], d_c, scale, static_cast<float*>(p->K),
                           static_cast<float*>(p->Kb));
    } else {
        hipLaunchKernelGGL(psn::k_assemble<double>, dim3(n + 1, n + 1), dim3(256), lds, s, A[0], A[1], A[2], d_w,
                           terms, n, p->period[0], p->period[1], p->period[2], d_c, scale,
                           static_cast<double*>(p->K), static_cast<double*>(p->Kb));
    }
    return hipGetLastError();
}

}  // namespace psn_host
