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

// Per step: the axis-2 steps (1, 5) transform the real line as n2/2 packed
// pairs, a length FL = L/2 transform; the strided steps transform length L.
// B lines per workgroup: 8 where the lines and the twiddle table fit (the
// strided steps up to the 160 KB of LDS, so that they move 64-byte FP32 row
// pieces; the row steps within 64 KB, where more lines only cost occupancy).
template <int L, class Real, int STEP>
struct GCfg {
    static constexpr bool rows = STEP == 1 || STEP == 5;
    static constexpr int FL = rows ? L / 2 : L;
    static constexpr int E = elems_per_thread(FL, sizeof(Real));
    static constexpr int T = FL / E;
    static constexpr int CX = sizeof(cx<Real>);
    static constexpr int TWS = TwLds<Real>::slots(L);
    static constexpr int pick() {
        for (int b = 8; b > 1; b /= 2)
            if ((b * FL + TWS) * CX <= (rows ? 65536 : 163840) && b * T <= 1024) return b;
        return 1;
    }
    static constexpr int B = pick();
    static constexpr size_t lds = size_t(B * FL + TWS) * CX;
};

template <int L, class Real, class Io, int STEP>
__global__ void __launch_bounds__((GCfg<L, Real, STEP>::B * GCfg<L, Real, STEP>::T)) g_step(const GArgs<Real, Io> a) {
    using C = GCfg<L, Real, STEP>;
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
    // workgroups are dealt to the 8 XCDs round robin: give each XCD a
    // contiguous run of line groups (neighbours share cache lines in its L2);
    // the grid is a multiple of 8, and groups past the end leave at once
    const long grp = long(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    if (grp * B >= nlines) return;  // whole workgroup
    const long line = grp * B + c;
    const bool live = line < nlines;  // a partial last workgroup still joins every barrier
    const long ln = live ? line : 0;
    TwLds<Real> tl{sb + B * C::FL};
    tl.fill(a.tw, L, threadIdx.x, B * T);
    __syncthreads();
    LdsCols<Real> lds{sb, B, c};
    cx<Real> d[C::E];
    if constexpr (STEP == 1) {
        // Real row of n2 = FL samples, zero beyond: z_j = x_2j + i x_2j+1
        // (j < FL/2, zero beyond), Z = DFT_FL(z), then the padded spectrum
        // X[k] = E[k] + w^k O[k], w = exp(-2 pi i / L), with E and O the
        // transforms of the even and odd samples, E = (Z[k] + conj Z[FL-k])/2,
        // O = (Z[k] - conj Z[FL-k])/(2i); X[0] and X[FL] come from Z[0].
        constexpr int FL = C::FL;
        using Fh = TeamFFT<FL, T, Real, -1, false>;
        const Io* x = a.rho + ln * n2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int j = Fh::in_pos(t, e);
            d[e] = (live && j < FL / 2) ? cx<Real>{Real(x[2 * j]), Real(x[2 * j + 1])} : cx<Real>{Real(0), Real(0)};
        }
        Fh::run1(d, t, TwHalf<Real>{tl}, lds);
        __syncthreads();  // the transform's last exchange reads are done
#pragma unroll
        for (int e = 0; e < C::E; ++e) lds.put(Fh::out_pos(t, e), d[e]);
        __syncthreads();
        cx<Real>* y = a.w1 + ln * h;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int k = Fh::out_pos(t, e);
            const cx<Real> Z = lds.get(k);
            if (k == 0) {
                if (live) {
                    gst(y, cx<Real>{Z.x + Z.y, Real(0)});
                    gst(y + FL, cx<Real>{Z.x - Z.y, Real(0)});
                }
            } else {
                const cx<Real> Zr = conj(lds.get(FL - k));
                const cx<Real> Ev = scale(Z + Zr, Real(0.5));
                const cx<Real> Od = rot<-1>(scale(Z - Zr, Real(0.5)));
                if (live) gst(y + k, Ev + Od * tl(2 * k));
            }
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
        // The row's padded spectrum X[0..FL] is that of a real sequence.  The
        // inverse of length FL of Y[k] = (X[k] + conj X[FL-k])
        // + i (X[k] - conj X[FL-k]) w^-k gives z_j = u_2j + i u_2j+1; only
        // j < FL/2 lies inside the box.
        constexpr int FL = C::FL;
        using Fh = TeamFFT<FL, T, Real, +1, false>;
        const cx<Real>* x = a.w1 + ln * h;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int k = Fh::in_pos(t, e);
            cx<Real> v{Real(0), Real(0)};
            if (live) {
                const cx<Real> p = gld(x + k), q = conj(gld(x + (FL - k)));
                v = (p + q) + rot<+1>(mul_conj(p - q, tl(2 * k)));
            }
            d[e] = v;
        }
        Fh::run1(d, t, TwHalf<Real>{tl}, lds);
        Io* y = a.u + ln * n2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int j = Fh::out_pos(t, e);
            if (live && j < FL / 2) {
                y[2 * j] = Io(d[e].x);
                y[2 * j + 1] = Io(d[e].y);
            }
        }
    }
}

template <int L, class Real, class Io, int STEP>
hipError_t launch_g_step(const GArgs<Real, Io>& a, long nlines, hipStream_t s) {
    using C = GCfg<L, Real, STEP>;
    if constexpr (C::lds > 65536) {
        static const hipError_t ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&g_step<L, Real, Io, STEP>),
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, int(C::lds));
        if (ok != hipSuccess) return ok;
    }
    const long groups = (nlines + C::B - 1) / C::B;
    hipLaunchKernelGGL((g_step<L, Real, Io, STEP>), dim3(unsigned(8 * ((groups + 7) / 8))), dim3(C::B * C::T), C::lds,
                       s, a);
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
