// Grids with a different number of points per axis (paper section 2's
// general box, N = n0 n1 n2 points, section 3): the same convolution, run as
// five line-transform steps over plain workspaces.  Each step transforms
// lines of one axis at that axis' padded length L = 2 n_q, with the zero half
// of the input formed in registers and only the needed outputs stored:
//
//   1  axis 2, real -> complex:  rho[i0][i1][0..n2)  -> W1[i0][i1][0..n2]      (n2 + 1 outputs)
//   2  axis 1, forward:          W1[i0][0..n1)[k2]   -> W2[i0][0..2n1)[k2]
//   3  axis 0, forward, x K, inverse, in place on W2[0..n0)[k1][k2]
//   4  axis 1, inverse:          W2[i0][0..2n1)[k2]  -> W1[i0][0..n1)[k2]
//   5  axis 2, complex -> real:  W1[i0][i1][0..n2]   -> u[i0][i1][0..n2)
//
// K is the octant [k0][k1][k2] (k_q = 0..n_q, folded index min(k, 2 n_q - k)),
// scaled by 1 / (8 n0 n1 n2).  A workgroup holds B lines with the same
// element stride: consecutive lines of an axis-2 step are rows (threads run
// along a row), those of the other steps are consecutive k2 (threads of
// consecutive lines touch consecutive addresses).
#pragma once

#include "psn_device.h"
#include "psn_internal.h"

namespace psn {

template <class Real, class Io>
struct GArgs {
    const Io* rho;
    Io* u;
    cx<Real>* w1;
    cx<Real>* w2;
    const Real* K;
    const cx<Real>* tw;  // exp(-2 pi i m / 2L), m < 2L, for this step's length L
    int n0, n1, n2;
};

template <int L, class Real>
struct GCfg {
    static constexpr int E = elems_per_thread(L, sizeof(Real));
    static constexpr int T = L / E;
    static constexpr int CX = sizeof(cx<Real>);
    static constexpr int TWS = TwLds<Real>::slots(L);
    static constexpr int pick() {
        for (int b = 8; b > 1; b /= 2)
            if ((b * L + TWS) * CX <= 65536 && b * T <= 1024) return b;
        return 1;
    }
    static constexpr int B = pick();
    static constexpr size_t lds = size_t(B * L + TWS) * CX;
};

template <int L, class Real, class Io, int STEP>
__global__ void __launch_bounds__((GCfg<L, Real>::B * GCfg<L, Real>::T)) g_step(const GArgs<Real, Io> a) {
    using C = GCfg<L, Real>;
    constexpr int B = C::B, T = C::T;
    constexpr bool rows = STEP == 1 || STEP == 5;
    using Ff = TeamFFT<L, T, Real, -1, false>;
    using Fi = TeamFFT<L, T, Real, +1, STEP == 3>;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int h = n2 + 1;  // k2 per row of the workspaces
    const int c = rows ? int(threadIdx.x) / T : int(threadIdx.x) % B;
    const int t = rows ? int(threadIdx.x) % T : int(threadIdx.x) / B;
    long nlines;
    if constexpr (STEP == 1 || STEP == 5) nlines = long(n0) * n1;
    else if constexpr (STEP == 3) nlines = 2L * n1 * h;
    else nlines = long(n0) * h;
    const long line = long(blockIdx.x) * B + c;
    const bool live = line < nlines;  // a partial last workgroup still joins every barrier
    const long ln = live ? line : 0;
    TwLds<Real> tl{sb + B * L};
    tl.fill(a.tw, L, threadIdx.x, B * T);
    __syncthreads();
    LdsCols<Real> lds{sb, B, c};
    cx<Real> d[C::E];
    if constexpr (STEP == 1) {
        // real row of n2 samples, zero beyond
        const Io* x = a.rho + ln * n2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Ff::in_pos(t, e);
            d[e] = {(live && p < n2) ? Real(x[p]) : Real(0), Real(0)};
        }
        Ff::run1(d, t, tl, lds);
        cx<Real>* y = a.w1 + ln * h;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int k = Ff::out_pos(t, e);
            if (live && k <= n2) gst(y + k, d[e]);
        }
    } else if constexpr (STEP == 2) {
        const long i0 = ln / h, k2 = ln % h;
        const cx<Real>* x = a.w1 + i0 * n1 * h + k2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Ff::in_pos(t, e);
            d[e] = (live && p < n1) ? gld(x + long(p) * h) : cx<Real>{Real(0), Real(0)};
        }
        Ff::run1(d, t, tl, lds);
        cx<Real>* y = a.w2 + i0 * 2 * n1 * h + k2;
#pragma unroll
        for (int e = 0; e < C::E; ++e)
            if (live) gst(y + long(Ff::out_pos(t, e)) * h, d[e]);
    } else if constexpr (STEP == 3) {
        const long k1 = ln / h, k2 = ln % h;
        const long s0 = 2L * n1 * h;
        cx<Real>* x = a.w2 + ln;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Ff::in_pos(t, e);
            d[e] = (live && p < n0) ? gld(x + long(p) * s0) : cx<Real>{Real(0), Real(0)};
        }
        Ff::run1(d, t, tl, lds);
        const long k1f = k1 <= n1 ? k1 : 2 * n1 - k1;
        const Real* Kr = a.K + k1f * h + k2;
        const long sk0 = long(n1 + 1) * h;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int k0 = Ff::out_pos(t, e);
            const int k0f = k0 <= n0 ? k0 : 2 * n0 - k0;
            d[e] = scale(d[e], live ? Real(Kr[k0f * sk0]) : Real(0));
        }
        __syncthreads();  // the forward transform's last exchange reads are done
        Fi::run1(d, t, tl, lds);  // radices reversed: starts from the forward output layout
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Fi::out_pos(t, e);
            if (live && p < n0) gst(x + long(p) * s0, d[e]);
        }
    } else if constexpr (STEP == 4) {
        const long i0 = ln / h, k2 = ln % h;
        const cx<Real>* x = a.w2 + i0 * 2 * n1 * h + k2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) d[e] = live ? gld(x + long(Fi::in_pos(t, e)) * h) : cx<Real>{Real(0), Real(0)};
        Fi::run1(d, t, tl, lds);
        cx<Real>* y = a.w1 + i0 * n1 * h + k2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Fi::out_pos(t, e);
            if (live && p < n1) gst(y + long(p) * h, d[e]);
        }
    } else {
        // the row's spectrum is that of a real sequence: X[L - k] = conj X[k]
        const cx<Real>* x = a.w1 + ln * h;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int k = Fi::in_pos(t, e);
            cx<Real> v{Real(0), Real(0)};
            if (live) v = k <= n2 ? gld(x + k) : conj(gld(x + (L - k)));
            d[e] = v;
        }
        Fi::run1(d, t, tl, lds);
        Io* y = a.u + ln * n2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Fi::out_pos(t, e);
            if (live && p < n2) y[p] = Io(d[e].x);
        }
    }
}

template <int L, class Real, class Io, int STEP>
hipError_t launch_g_step(const GArgs<Real, Io>& a, long nlines, hipStream_t s) {
    using C = GCfg<L, Real>;
    hipLaunchKernelGGL((g_step<L, Real, Io, STEP>), dim3(unsigned((nlines + C::B - 1) / C::B)), dim3(C::B * C::T),
                       C::lds, s, a);
    return hipSuccess;
}

// dispatch on the padded length L = 2 n of a compiled size n
template <class Real, class Io, int STEP>
hipError_t g_step_n(int n, const GArgs<Real, Io>& a, long nlines, hipStream_t s) {
    switch (n) {
#define PSN_CASE(NN) \
    case NN: return launch_g_step<2 * NN, Real, Io, STEP>(a, nlines, s);
        PSN_FOR_EACH_SIZE(PSN_CASE)
#undef PSN_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psn
