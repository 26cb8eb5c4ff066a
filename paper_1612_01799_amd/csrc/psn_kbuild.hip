// Kernel-spectrum build in FP64 on the device (paper section 2: the G-tensor
// and the near-zone correction; section 3: it is the setup phase).
//
//   a_j(k)   = 2 int_0^T exp(-tau_j^2 y^2) cos(kappa_k y) dy,  kappa_k = 2 pi k / (2 n h)
//   C0, C2   = int_{B_delta} (U - U_GS) dy,  int_{B_delta} |y|^2 (U - U_GS) dy
//   K(k)     = sum_j w_j a_j(k0) a_j(k1) a_j(k2) + C0 - (C2/6) |kappa|^2
//
// Mode integrals, by the size of tau T:
// * tau T >= 6.1: the Gaussian's Fourier transform (the tail beyond T is
//   below exp(-37) relative).
// * tau T < 1: the integrand is 1 plus expm1(-tau^2 y^2) = sum_{m>=1}
//   (-tau^2 y^2)^m / m!, so a_j(k) = 2T [k = 0] + sum_m (-tau_j^2)^m / m! M_m(k)
//   with the moments M_m(k) = 2 int_0^T y^2m cos(kappa_k y) dy, which do not
//   depend on the term.  Each summand is at most 2T (tau T)^2m / (m! (2m+1)),
//   so the series converges without cancellation; the moments are computed
//   once per frequency by composite 16-point Gauss-Legendre.
// * otherwise: composite 16-point Gauss-Legendre of the integral itself, with
//   one panel per two half periods of cos(kappa_k y) plus eight.
// The octant assembly is the product of the (k0, k1) rows sum_j over the
// terms with the (k2) columns: an FP64 GEMM on the matrix cores
// (v_mfma_f64_16x16x4f64, the row operand a_j(k0) a_j(k1) formed as it is
// fed).  On a cube the
// three axes share one mode table and K is symmetric in (k0, k1); then only
// k0 <= k1 is computed, the pair product a_j(k0) a_j(k1) is formed first (so
// both halves agree bitwise) and each value is written to both places.
#include <algorithm>

#include "psn_device.h"
#include "psn_internal.h"

namespace psn {

constexpr double kPi = 3.14159265358979323846;

typedef double psn_d4 __attribute__((ext_vector_type(4)));

constexpr int kMoments = 22;  // series terms of the tau T < 1 branch: 1/22! < 1e-21

// Panels of the composite Gauss-Legendre rule for frequency k: one per two
// half periods of cos(kappa_k y) on [0, T] plus eight.
__device__ __forceinline__ int gl_panels(int k) { return (k + 1) / 2 + 8; }

// Sum over the kPanelThreads threads of a workgroup, in a fixed order (the
// result does not depend on timing); v[] holds each thread's NV partial sums;
// red has NV * kPanelThreads doubles; the sums land in v[] of thread 0.
constexpr int kPanelThreads = 64;
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int m = 0; m < NV; ++m) red[m * kPanelThreads + tid] = v[m];
    __syncthreads();
    for (int h = kPanelThreads / 2; h > 0; h >>= 1) {
        if (tid < h) {
#pragma unroll
            for (int m = 0; m < NV; ++m) red[m * kPanelThreads + tid] += red[m * kPanelThreads + tid + h];
        }
        __syncthreads();
    }
    if (tid == 0) {
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] = red[m * kPanelThreads];
    }
}

// M_m(k) = 2 int_0^T y^2m cos(kappa_k y) dy, m = 1..kMoments, for k = 0..n;
// Mom[(m - 1) (n + 1) + k].  One workgroup per k; its threads share the panels.
__global__ void __launch_bounds__(kPanelThreads) k_moments(int n, double T, double period,
                                                           const double* __restrict__ glx,
                                                           const double* __restrict__ glw, double* __restrict__ Mom) {
    __shared__ double red[kMoments * kPanelThreads];
    const int k = blockIdx.x;
    const double kap = 2.0 * kPi * double(k) / period;
    const int panels = gl_panels(k);
    const double half = 0.5 * T / panels;
    double acc[kMoments];
#pragma unroll
    for (int m = 0; m < kMoments; ++m) acc[m] = 0.0;
    for (int pnl = threadIdx.x; pnl < panels; pnl += kPanelThreads) {
        const double mid = (2 * pnl + 1) * half;
        for (int g = 0; g < 16; ++g) {
            const double y = mid + half * glx[g];
            const double y2 = y * y;
            double f = 2.0 * half * glw[g] * cos(kap * y);
#pragma unroll
            for (int m = 0; m < kMoments; ++m) {
                f *= y2;
                acc[m] += f;
            }
        }
    }
    block_sum(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int m = 0; m < kMoments; ++m) Mom[size_t(m) * (n + 1) + k] = acc[m];
    }
}

// Terms with tau T >= 6.1 (closed form) or tau T < 1 (moment series); the
// terms in between are left to k_modes_mid.  One thread per (k, j).
__global__ void k_modes(const double* __restrict__ tau, int n, double T, double period,
                        const double* __restrict__ Mom, double* __restrict__ A) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (k > n) return;
    const double t = tau[j];
    const double kap = 2.0 * kPi * double(k) / period;
    const double tT = t * T;
    double a;
    if (tT >= 6.1) {
        a = sqrt(kPi) / t * exp(-kap * kap / (4.0 * t * t));
    } else if (tT < 1.0) {
        // 2T [k = 0] + sum_m (-tau^2)^m / m! M_m(k), smallest terms first
        double c[kMoments];
        double cm = 1.0;
        for (int m = 0; m < kMoments; ++m) {
            cm *= -t * t / double(m + 1);
            c[m] = cm;
        }
        double sum = 0.0;
        for (int m = kMoments - 1; m >= 0; --m) sum = fma(c[m], Mom[size_t(m) * (n + 1) + k], sum);
        a = sum + (k == 0 ? 2.0 * T : 0.0);
    } else {
        return;
    }
    A[size_t(j) * (n + 1) + k] = a;
}

// Terms with 1 <= tau T < 6.1, by composite Gauss-Legendre: one workgroup
// per (k, term), its threads share the panels.
__global__ void __launch_bounds__(kPanelThreads) k_modes_mid(const double* __restrict__ tau, int j0, int n, double T,
                                                             double period, const double* __restrict__ glx,
                                                             const double* __restrict__ glw, double* __restrict__ A) {
    __shared__ double red[kPanelThreads];
    const int k = blockIdx.x, j = j0 + blockIdx.y;
    const double t = tau[j];
    const double kap = 2.0 * kPi * double(k) / period;
    const int panels = gl_panels(k);
    const double half = 0.5 * T / panels;
    double sum[1] = {0.0};
    for (int pnl = threadIdx.x; pnl < panels; pnl += kPanelThreads) {
        const double mid = (2 * pnl + 1) * half;
        double ps = 0.0;
#pragma unroll
        for (int g = 0; g < 16; ++g) {
            const double y = mid + half * glx[g];
            const double ty = t * y;
            ps += glw[g] * exp(-ty * ty) * cos(kap * y);
        }
        sum[0] += half * ps;
    }
    block_sum(sum, red);
    if (threadIdx.x == 0) A[size_t(j) * (n + 1) + k] = 2.0 * sum[0];
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

// K(k0, k1, n) for every (k0, k1), FP64: the k2 = n column, which the
// octant stores folded with k2 = 0.  Kn[k1 (n + 1) + k0].
__global__ void k_edge(const double* __restrict__ A0, const double* __restrict__ A1, const double* __restrict__ A2,
                       const double* __restrict__ w, int terms, int n, double p0, double p1, double p2,
                       const double* __restrict__ Cc, double fold, double* __restrict__ Kn) {
    const int k0 = blockIdx.x * blockDim.x + threadIdx.x, k1 = blockIdx.y;
    if (k0 > n) return;
    const int np1 = n + 1;
    double s = 0.0;
    for (int j = 0; j < terms; ++j)
        s = fma(A0[size_t(j) * np1 + k0] * A1[size_t(j) * np1 + k1], w[j] * A2[size_t(j) * np1 + n], s);
    const double b0 = 2.0 * kPi * k0 / p0, b1 = 2.0 * kPi * k1 / p1, b2 = 2.0 * kPi * n / p2;
    Kn[size_t(k1) * np1 + k0] = s + fold * (Cc[0] - (Cc[1] / 6.0) * (b0 * b0 + b1 * b1 + b2 * b2));
}

// Octant assembly, k2 = 0..n-1: a workgroup of 256 threads computes a tile of
// 128 k0 x 64 k2 of one k1 plane, each thread 4 k0 x 8 k2 (k0 = k0b + r +
// 32 i, k2 = k2b + q + 8 c with q = tid % 8, r = tid / 8), so that the eight
// lanes of a k0 row write 8 consecutive k2 of the tiled octant.  The terms
// stream through LDS in chunks of 16: a_j(k0) and w_j a_j(k2).  With SYM
// (A0 == A1) only tiles with k0b <= k1 run and entries with k0 <= k1 are
// written, to (k0, k1) and (k1, k0).
constexpr int kTile0 = 128, kTile2 = 64, kChunk = 32;

template <class Kt, bool SYM>
__global__ void __launch_bounds__(256) k_gemm(const double* __restrict__ A0, const double* __restrict__ A1,
                                              const double* __restrict__ A2, const double* __restrict__ w, int terms,
                                              int n, double p0, double p1, double p2,
                                              const double* __restrict__ Cc, double fold,
                                              const double* __restrict__ Kn, double scale, Kt* __restrict__ K,
                                              Kt* __restrict__ Kb) {
    __shared__ double sa[kChunk][kTile0], sb[kChunk][kTile2], s1[kChunk];
    const int np1 = n + 1;
    const int k1 = blockIdx.z;
    const int k0b = blockIdx.y * kTile0, k2b = blockIdx.x * kTile2;
    if (SYM && k0b > k1) return;  // whole workgroup: the mirror tile covers it
    const int tid = threadIdx.x;
    // wave wv owns rows k0b + 32 wv .. +31 as two 16-row blocks, all 64 columns
    // as four 16-column blocks: eight 16 x 16 FP64 accumulators
    const int wv = tid / 64, lane = tid % 64, li = lane % 16, lg = lane / 16;
    psn_d4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[i][c] = psn_d4{0.0, 0.0, 0.0, 0.0};
    for (int j0 = 0; j0 < terms; j0 += kChunk) {
        __syncthreads();  // the previous chunk's reads are done
        for (int idx = tid; idx < kChunk * kTile0; idx += 256) {
            const int jj = idx / kTile0, c = idx % kTile0, j = j0 + jj, k0 = k0b + c;
            sa[jj][c] = (j < terms && k0 <= n) ? A0[size_t(j) * np1 + k0] : 0.0;
        }
        for (int idx = tid; idx < kChunk * kTile2; idx += 256) {
            const int jj = idx / kTile2, c = idx % kTile2, j = j0 + jj, k2 = k2b + c;
            sb[jj][c] = (j < terms && k2 < n) ? w[j] * A2[size_t(j) * np1 + k2] : 0.0;
        }
        if (tid < kChunk) s1[tid] = j0 + tid < terms ? A1[size_t(j0 + tid) * np1 + k1] : 0.0;
        __syncthreads();
        // four k-steps of four terms: lane (li, lg) gives term 4 s + lg of row
        // li (the product a_j(k0) a_j(k1)) and of column li (w_j a_j(k2))
#pragma unroll
        for (int st = 0; st < kChunk / 4; ++st) {
            const int jj = 4 * st + lg;
            const double a1 = s1[jj];
            double av[2], bv[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = sa[jj][32 * wv + 16 * i + li] * a1;
#pragma unroll
            for (int c = 0; c < 4; ++c) bv[c] = sb[jj][16 * c + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[i][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[c], acc[i][c], 0, 0, 0);
        }
    }
    // result (row lg + 4 e, column li) of each 16 x 16 block is word e of the
    // lane (the FP64 form interleaves the rows over the four lane groups)
    const double C0 = Cc[0], C2 = Cc[1];
    const double b1 = 2.0 * kPi * k1 / p1;
#pragma unroll
    for (int ie = 0; ie < 8; ++ie) {
        const int i = ie / 4, e = ie % 4;
        const int k0 = k0b + 32 * wv + 16 * i + lg + 4 * e;
        if (k0 > n || (SYM && k0 > k1)) continue;
        const double b0 = 2.0 * kPi * k0 / p0;
        const double q01 = b0 * b0 + b1 * b1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int k2 = k2b + 16 * c + li;
            if (k2 >= n) continue;
            const double b2 = 2.0 * kPi * k2 / p2;
            const double v = acc[i][c][e] + fold * (C0 - (C2 / 6.0) * (q01 + b2 * b2));
            if (k2 == 0) {
                const double e = Kn[size_t(k1) * np1 + k0];
                K[psn_host::k_index(n, k1, k0, 0)] = Kt(scale * 0.5 * (v + e));
                Kb[size_t(k1) * np1 + k0] = Kt(scale * 0.5 * (v - e));
                if (SYM && k0 != k1) {
                    K[psn_host::k_index(n, k0, k1, 0)] = Kt(scale * 0.5 * (v + e));
                    Kb[size_t(k0) * np1 + k1] = Kt(scale * 0.5 * (v - e));
                }
            } else {
                K[psn_host::k_index(n, k1, k0, k2)] = Kt(scale * v);
                if (SYM && k0 != k1) K[psn_host::k_index(n, k0, k1, k2)] = Kt(scale * v);
            }
        }
    }
}

// Octant of a grid with per-axis sizes, k_q = 0..n_q, in the k2-tiled layout
// of g_k_index: one thread per k2, sum over the terms; the padding k2 > n2 of
// the last tile is set to zero.  A_q has rows of n_q + 1.
template <class Kt>
__global__ void g_assemble(const double* __restrict__ A0, const double* __restrict__ A1,
                           const double* __restrict__ A2, const double* __restrict__ w, int terms, int n0, int n1,
                           int n2, double p0, double p1, double p2, const double* __restrict__ Cc, double fold,
                           double scale, Kt* __restrict__ K) {
    const int k2 = blockIdx.x * blockDim.x + threadIdx.x, k1 = blockIdx.y, k0 = blockIdx.z;
    if (k2 >= psn_host::g_pitch(n2)) return;
    if (k2 > n2) {
        K[psn_host::g_k_index(n0, n2, k0, k1, k2)] = Kt(0);
        return;
    }
    double s = 0.0;
    for (int j = 0; j < terms; ++j)
        s = fma(A0[size_t(j) * (n0 + 1) + k0] * A1[size_t(j) * (n1 + 1) + k1], w[j] * A2[size_t(j) * (n2 + 1) + k2],
                s);
    const double b0 = 2.0 * kPi * k0 / p0, b1 = 2.0 * kPi * k1 / p1, b2 = 2.0 * kPi * k2 / p2;
    const double v = s + fold * (Cc[0] - (Cc[1] / 6.0) * (b0 * b0 + b1 * b1 + b2 * b2));
    K[psn_host::g_k_index(n0, n2, k0, k1, k2)] = Kt(scale * v);
}

}  // namespace psn

namespace psn_host {

size_t kbuild_scratch_doubles(int n, int terms) {
    const size_t np1 = size_t(n) + 1;
    return 3 * size_t(terms) * np1 + 3 * size_t(psn::kMoments) * np1 + np1 * np1;
}

hipError_t launch_kernel_build(psn_plan* p, const double* d_tau, const double* d_w, int terms, const double* d_glx,
                               const double* d_glw, double* d_A, double* d_c, hipStream_t s) {
    const int n = p->n;
    const int nmax = std::max(p->ng[0], std::max(p->ng[1], p->ng[2]));
    const size_t np1 = size_t(nmax) + 1;
    const size_t tab = size_t(terms) * np1;
    double* d_mom = d_A + 3 * tab;                           // 3 x kMoments x (nmax+1)
    double* d_kn = d_mom + 3 * size_t(psn::kMoments) * np1;  // (n+1)^2
    // one mode table per distinct axis (length, period, points); table q has
    // rows of ng[q] + 1 entries
    const double* A[3];
    for (int q = 0; q < 3; ++q) {
        int same = -1;
        for (int r = 0; r < q; ++r)
            if (p->T[r] == p->T[q] && p->period[r] == p->period[q] && p->ng[r] == p->ng[q]) same = r;
        if (same >= 0) {
            A[q] = A[same];
            continue;
        }
        const int nq = p->ng[q];
        A[q] = d_A + q * tab;
        double* mom = d_mom + q * size_t(psn::kMoments) * np1;
        hipLaunchKernelGGL(psn::k_moments, dim3(nq + 1), dim3(psn::kPanelThreads), 0, s, nq, p->T[q], p->period[q],
                           d_glx, d_glw, mom);
        hipLaunchKernelGGL(psn::k_modes, dim3((nq + 1 + 127) / 128, terms), dim3(128), 0, s, d_tau, nq, p->T[q],
                           p->period[q], mom, d_A + q * tab);
        // the terms with 1 <= tau T < 6.1: a contiguous range (tau grows with j)
        int j0 = terms, j1 = 0;
        for (int j = 0; j < terms; ++j) {
            const double tT = p->tau[j] * p->T[q];
            if (tT >= 1.0 && tT < 6.1) {
                j0 = j < j0 ? j : j0;
                j1 = j + 1;
            }
        }
        if (j1 > j0)
            hipLaunchKernelGGL(psn::k_modes_mid, dim3(nq + 1, j1 - j0), dim3(psn::kPanelThreads), 0, s, d_tau, j0, nq,
                               p->T[q], p->period[q], d_glx, d_glw, d_A + q * tab);
    }
    hipLaunchKernelGGL(psn::k_correction, dim3(1), dim3(256), 0, s, d_tau, d_w, terms, p->delta, d_c);
    if (p->general) {
        const int n0 = p->ng[0], n1 = p->ng[1], n2 = p->ng[2];
        const double scale = 1.0 / (8.0 * double(n0) * n1 * n2);
        const dim3 g(unsigned((psn_host::g_pitch(n2) + 127) / 128), n1 + 1, n0 + 1);
        if (p->dtype == PSN_F32)
            hipLaunchKernelGGL(psn::g_assemble<float>, g, dim3(128), 0, s, A[0], A[1], A[2], d_w, terms, n0, n1, n2,
                               p->period[0], p->period[1], p->period[2], d_c, 1.0, scale, static_cast<float*>(p->K));
        else
            hipLaunchKernelGGL(psn::g_assemble<double>, g, dim3(128), 0, s, A[0], A[1], A[2], d_w, terms, n0, n1, n2,
                               p->period[0], p->period[1], p->period[2], d_c, 1.0, scale, static_cast<double*>(p->K));
        return hipGetLastError();
    }
    // the correction symbol is folded into K unless the plan adds it by the
    // Fourier series of the density (then fold = 0 leaves the G-tensor alone)
    const double fold = p->correction == PSN_CORRECTION_FOURIER ? 0.0 : 1.0;
    hipLaunchKernelGGL(psn::k_edge, dim3((n + 1 + 127) / 128, n + 1), dim3(128), 0, s, A[0], A[1], A[2], d_w, terms,
                       n, p->period[0], p->period[1], p->period[2], d_c, fold, d_kn);
    const double M = 2.0 * n;
    const double scale = 1.0 / (M * M * M);
    const bool sym = A[0] == A[1];
    const dim3 grid((n + psn::kTile2 - 1) / psn::kTile2, (n + 1 + psn::kTile0 - 1) / psn::kTile0, n + 1);
#define PSN_GEMM(KT, SYMV)                                                                                         \
    hipLaunchKernelGGL((psn::k_gemm<KT, SYMV>), grid, dim3(256), 0, s, A[0], A[1], A[2], d_w, terms, n,            \
                       p->period[0], p->period[1], p->period[2], d_c, fold, d_kn, scale, static_cast<KT*>(p->K),   \
                       static_cast<KT*>(p->Kb))
    if (p->dtype == PSN_F32) {
        if (sym) PSN_GEMM(float, true);
        else PSN_GEMM(float, false);
    } else {
        if (sym) PSN_GEMM(double, true);
        else PSN_GEMM(double, false);
    }
#undef PSN_GEMM
    return hipGetLastError();
}

}  // namespace psn_host
