// The five pruned passes of one solve (paper section 2: the size-8N transform
// pair of I_1 with the G-tensor multiply; section 3: its cost).
//
// Layout (C order, last index contiguous), M = 2n:
//   rho, u : [i0][i1][i2]            n^3 reals
//   W1     : [i0][i1][k2]            n^3 complex, k2 = 0..n-1
//   W2     : [i0][k1][k2]            n * M * n complex
//   K      : [k1~][k0~][k2]          (n+1)^2 * n reals, folded k~ = min(k, M-k)
//   Kb     : [k1~][k0~]              (n+1)^2 reals
// The real-to-complex transform along axis 2 gives n+1 frequencies; the two
// real ones (k2 = 0 and k2 = n) travel packed as one complex value in column
// 0 (real part: k2 = 0, imaginary part: k2 = n).  The middle pass separates
// them with the conjugate-symmetric partner (-k0, -k1) and applies their own
// kernel values: Z' = a Z(k) + b conj(Z(-k)), a = (K0+Kn)/2, b = (K0-Kn)/2.
//
// Zero padding is never formed.  A length-M transform of a line whose second
// half is zero splits into two length-n transforms: even outputs are DFT_n(x),
// odd outputs DFT_n(x * w^j) with w = exp(-2 pi i / M).  Likewise a length-M
// inverse keeping only the first n outputs is IDFT_n(even) + w^-j IDFT_n(odd).
//
//   P1  axis 2, real -> complex   rho -> W1   (two reals per complex lane)
//   P2  axis 1, forward           W1  -> W2   (n inputs, M outputs)
//   P3  axis 0, forward, x K, inverse, in place on W2 (n in, n out)
//   P4  axis 1, inverse           W2  -> W1   (M inputs, n outputs)
//   P5  axis 2, complex -> real   W1  -> u
// The 1/M^3 of the inverse transform is folded into K.
#include "psn_device.h"
#include "psn_internal.h"

namespace psn {

constexpr int kMaxLds = 65536;

constexpr int pick_cols(int N, int bmax, int sets, int cxbytes, int T) {
    for (int b = bmax; b >= 1; --b)
        if (N % b == 0 && sets * b * N * cxbytes <= kMaxLds && sets * b * T <= 1024) return b;
    return 1;
}

constexpr int rows_padded(int N) { return N + (N >> 4) + 1; }

constexpr int pick_lines(int N, int T, int cxbytes) {
    int l = 256 / T;
    if (l < 1) l = 1;
    while (l > 1 && ((N * N) % l != 0 || l * rows_padded(N) * cxbytes > kMaxLds)) l /= 2;
    return l;
}

template <int N, int DT>
struct Cfg {
    using P = Prec<DT>;
    using Real = typename P::Real;
    using Io = typename P::Io;
    using Kt = typename P::Kt;
    static constexpr int E = elems_per_thread(N);
    static constexpr int T = N / E;
    static constexpr int CX = sizeof(cx<Real>);
    static constexpr int BS = pick_cols(N, DT == DT_F32 ? 16 : 8, 1, CX, T);   // P2, P4 columns
    static constexpr int BP3 = pick_cols(N, DT == DT_F32 ? 8 : 4, 2, CX, T);   // P3 columns per set
    static constexpr int LC = pick_lines(N, T, CX);                            // P1, P5 lines
    static constexpr int NP = rows_padded(N);
};

// ------------------------------------------------------------------ P1
template <int N, int DT>
__global__ void __launch_bounds__((Cfg<N, DT>::LC * Cfg<N, DT>::T))
p1_r2c(const typename Cfg<N, DT>::Io* __restrict__ rho, Work<DT> w1,
       const cx<typename Cfg<N, DT>::Real>* __restrict__ tw) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, C::T, Real, -1, false>;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int t = threadIdx.x % C::T, ln = threadIdx.x / C::T;
    const size_t line = size_t(blockIdx.x) * C::LC + ln;
    const typename C::Io* x = rho + line * N;

    // z[j] = x[2j] + i x[2j+1]; zero for j >= n/2 (the padding)
    cx<Real> d[F::E];
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        const int pos = F::in_pos(t, e);
        if (pos < N / 2) d[e] = {Real(x[2 * pos]), Real(x[2 * pos + 1])};
        else d[e] = {Real(0), Real(0)};
    }
    LdsRows<Real> lds{sb + ln * C::NP};
    F::run(d, t, tw, lds);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < F::E; ++e) lds.put(F::out_pos(t, e), d[e]);
    __syncthreads();
    // X[k] = E[k] + w^k O[k], E = (Z[k] + conj Z[n-k])/2, O = (Z[k] - conj Z[n-k])/(2i)
#pragma unroll
    for (int q = 0; q < F::E; ++q) {
        const int k = t + C::T * q;
        const cx<Real> Z = lds.get(k);
        cx<Real> X;
        if (k == 0) {
            X = {Z.x + Z.y, Z.x - Z.y};  // (X[0], X[n]) packed
        } else {
            const cx<Real> Zr = conj(lds.get(N - k));
            const cx<Real> Ev = scale(Z + Zr, Real(0.5));
            const cx<Real> Od = rot<-1>(scale(Z - Zr, Real(0.5)));
            X = Ev + Od * tw[k];
        }
        w1.st(line * N + k, X);
    }
}

// ------------------------------------------------------------------ P2
template <int N, int DT>
__global__ void __launch_bounds__((Cfg<N, DT>::BS * Cfg<N, DT>::T))
p2_fwd(Work<DT> w1, Work<DT> w2, const cx<typename Cfg<N, DT>::Real>* __restrict__ tw) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, C::T, Real, -1, false>;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int c = threadIdx.x % C::BS, t = threadIdx.x / C::BS;
    const int k2 = blockIdx.x * C::BS + c;
    const size_t i0 = blockIdx.y;
    const size_t inb = i0 * N * N + k2;
    const size_t outb = i0 * (2 * N) * N + k2;

    cx<Real> x[F::E];
#pragma unroll
    for (int e = 0; e < F::E; ++e) x[e] = w1.ld(inb + size_t(F::in_pos(t, e)) * N);
    LdsCols<Real> lds{sb, C::BS, c};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        cx<Real> d[F::E];
#pragma unroll
        for (int e = 0; e < F::E; ++e) d[e] = p ? x[e] * tw[F::in_pos(t, e)] : x[e];
        F::run(d, t, tw, lds);
#pragma unroll
        for (int e = 0; e < F::E; ++e) w2.st(outb + size_t(2 * F::out_pos(t, e) + p) * N, d[e]);
    }
}

// ------------------------------------------------------------------ P3
template <int N, int DT>
__global__ void __launch_bounds__((2 * Cfg<N, DT>::BP3 * Cfg<N, DT>::T))
p3_conv(Work<DT> w2, const typename Cfg<N, DT>::Kt* __restrict__ K,
        const typename Cfg<N, DT>::Kt* __restrict__ Kb, const cx<typename Cfg<N, DT>::Real>* __restrict__ tw) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using Ff = TeamFFT<N, C::T, Real, -1, false>;
    using Fi = TeamFFT<N, C::T, Real, +1, true>;
    static_assert(Ff::E == Fi::E, "");
    constexpr int B = C::BP3;
    constexpr size_t s0 = size_t(2 * N) * N;  // stride of i0 in W2
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);

    const int c = threadIdx.x % B;
    const int set = (threadIdx.x / B) & 1;
    const int t = threadIdx.x / (2 * B);
    const int q = blockIdx.y;
    // sets pair k1 with -k1 (mod M); pair 0 holds the two self-conjugate rows 0 and n
    const int k1 = set == 0 ? q : (q == 0 ? N : 2 * N - q);
    const int kt1 = (q == 0) ? (set ? N : 0) : q;
    const int partner = (q == 0) ? set : 1 - set;
    const int k2 = blockIdx.x * B + c;
    const bool colzero = blockIdx.x == 0;  // workgroup-uniform
    const size_t base = size_t(k1) * N + k2;
    const typename C::Kt* Krow = K + size_t(kt1) * (N + 1) * N + k2;
    const typename C::Kt* Kbr = Kb + size_t(kt1) * (N + 1);

    cx<Real> x[Ff::E], acc[Ff::E];
#pragma unroll
    for (int e = 0; e < Ff::E; ++e) x[e] = w2.ld(base + size_t(Ff::in_pos(t, e)) * s0);
    LdsCols<Real> lds{sb + set * B, 2 * B, c};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        cx<Real> d[Ff::E];
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) d[e] = p ? x[e] * tw[Ff::in_pos(t, e)] : x[e];
        Ff::run(d, t, tw, lds);
        if (colzero) {
            __syncthreads();
            if (c == 0) {
#pragma unroll
                for (int e = 0; e < Ff::E; ++e) sb[set * N + Ff::out_pos(t, e)] = d[e];
            }
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) {
            const int m = Ff::out_pos(t, e);
            const int k0 = 2 * m + p;
            const int kt0 = k0 <= N ? k0 : 2 * N - k0;
            const Real kv = Real(Krow[size_t(kt0) * N]);
            if (colzero && c == 0) {
                const int mp = p == 0 ? (m == 0 ? 0 : N - m) : N - 1 - m;
                const cx<Real> zp = conj(sb[partner * N + mp]);
                d[e] = scale(d[e], kv) + scale(zp, Real(Kbr[kt0]));
            } else {
                d[e] = scale(d[e], kv);
            }
        }
        Fi::run(d, t, tw, lds);
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) {
            if (p == 0) acc[e] = d[e];
            else acc[e] = acc[e] + mul_conj(d[e], tw[Fi::out_pos(t, e)]);
        }
    }
#pragma unroll
    for (int e = 0; e < Ff::E; ++e) w2.st(base + size_t(Fi::out_pos(t, e)) * s0, acc[e]);
}

// ------------------------------------------------------------------ P4
template <int N, int DT>
__global__ void __launch_bounds__((Cfg<N, DT>::BS * Cfg<N, DT>::T))
p4_inv(Work<DT> w2, Work<DT> w1, const cx<typename Cfg<N, DT>::Real>* __restrict__ tw) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, C::T, Real, +1, false>;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int c = threadIdx.x % C::BS, t = threadIdx.x / C::BS;
    const int k2 = blockIdx.x * C::BS + c;
    const size_t i0 = blockIdx.y;
    const size_t inb = i0 * (2 * N) * N + k2;
    const size_t outb = i0 * N * N + k2;

    cx<Real> acc[F::E];
    LdsCols<Real> lds{sb, C::BS, c};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        cx<Real> d[F::E];
#pragma unroll
        for (int e = 0; e < F::E; ++e) d[e] = w2.ld(inb + size_t(2 * F::in_pos(t, e) + p) * N);
        F::run(d, t, tw, lds);
#pragma unroll
        for (int e = 0; e < F::E; ++e) {
            if (p == 0) acc[e] = d[e];
            else acc[e] = acc[e] + mul_conj(d[e], tw[F::out_pos(t, e)]);
        }
    }
#pragma unroll
    for (int e = 0; e < F::E; ++e) w1.st(outb + size_t(F::out_pos(t, e)) * N, acc[e]);
}

// ------------------------------------------------------------------ P5
template <int N, int DT>
__global__ void __launch_bounds__((Cfg<N, DT>::LC * Cfg<N, DT>::T))
p5_c2r(Work<DT> w1, typename Cfg<N, DT>::Io* __restrict__ u, const cx<typename Cfg<N, DT>::Real>* __restrict__ tw) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using Io = typename C::Io;
    using F = TeamFFT<N, C::T, Real, +1, false>;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int t = threadIdx.x % C::T, ln = threadIdx.x / C::T;
    const size_t line = size_t(blockIdx.x) * C::LC + ln;
    const size_t base = line * N;

    // Y[k] = (V[k] + conj V[n-k]) + i (V[k] - conj V[n-k]) w^-k; V[0], V[n] real and packed
    cx<Real> d[F::E];
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        const int pos = F::in_pos(t, e);
        if (pos == 0) {
            const cx<Real> V = w1.ld(base);
            d[e] = {V.x + V.y, V.x - V.y};
        } else {
            const cx<Real> a = w1.ld(base + pos);
            const cx<Real> b = conj(w1.ld(base + N - pos));
            d[e] = (a + b) + rot<+1>(mul_conj(a - b, tw[pos]));
        }
    }
    LdsRows<Real> lds{sb + ln * C::NP};
    F::run(d, t, tw, lds);
    // z[j] = u[2j] + i u[2j+1]; only j < n/2 lies inside the box
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        const int pos = F::out_pos(t, e);
        if (pos < N / 2) {
            u[base + 2 * pos] = Io(d[e].x);
            u[base + 2 * pos + 1] = Io(d[e].y);
        }
    }
}

// ------------------------------------------------------------------ launcher
template <int N, int DT>
hipError_t solve_n(const psn_plan* p, const void* rho_, void* u_, hipStream_t s, hipEvent_t* ev) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using Io = typename C::Io;
    using Kt = typename C::Kt;
    const Io* rho = static_cast<const Io*>(rho_);
    Io* u = static_cast<Io*>(u_);
    const cx<Real>* tw = static_cast<const cx<Real>*>(p->tw);
    const Kt* K = static_cast<const Kt*>(p->K);
    const Kt* Kb = static_cast<const Kt*>(p->Kb);
    Work<DT> w1, w2;
    if constexpr (DT == DT_SPLIT) {
        w1 = {static_cast<cx<float>*>(p->W1), static_cast<uint32_t*>(p->W1lo)};
        w2 = {static_cast<cx<float>*>(p->W2), static_cast<uint32_t*>(p->W2lo)};
    } else {
        w1 = {static_cast<cx<Real>*>(p->W1)};
        w2 = {static_cast<cx<Real>*>(p->W2)};
    }
    const size_t lds_rows = size_t(C::LC) * C::NP * C::CX;
    const size_t lds_cols = size_t(C::BS) * N * C::CX;
    const size_t lds_p3 = size_t(2) * C::BP3 * N * C::CX;

    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    };
    mark(0);
    hipLaunchKernelGGL((p1_r2c<N, DT>), dim3(N * N / C::LC), dim3(C::LC * C::T), lds_rows, s, rho, w1, tw);
    mark(1);
    hipLaunchKernelGGL((p2_fwd<N, DT>), dim3(N / C::BS, N), dim3(C::BS * C::T), lds_cols, s, w1, w2, tw);
    mark(2);
    hipLaunchKernelGGL((p3_conv<N, DT>), dim3(N / C::BP3, N), dim3(2 * C::BP3 * C::T), lds_p3, s, w2, K, Kb, tw);
    mark(3);
    hipLaunchKernelGGL((p4_inv<N, DT>), dim3(N / C::BS, N), dim3(C::BS * C::T), lds_cols, s, w2, w1, tw);
    mark(4);
    hipLaunchKernelGGL((p5_c2r<N, DT>), dim3(N * N / C::LC), dim3(C::LC * C::T), lds_rows, s, w1, u, tw);
    mark(5);
    return hipGetLastError();
}

template <int DT>
hipError_t solve_dt(const psn_plan* p, const void* rho, void* u, hipStream_t s, hipEvent_t* ev) {
    switch (p->n) {
#define PSN_CASE(NN) \
    case NN: return solve_n<NN, DT>(p, rho, u, s, ev);
        PSN_FOR_EACH_SIZE(PSN_CASE)
#undef PSN_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psn

namespace psn_host {

hipError_t launch_solve(const psn_plan* p, const void* rho, void* u, hipStream_t stream, hipEvent_t* ev) {
    switch (p->dtype) {
        case PSN_F64: return psn::solve_dt<psn::DT_F64>(p, rho, u, stream, ev);
        case PSN_F32: return psn::solve_dt<psn::DT_F32>(p, rho, u, stream, ev);
        case PSN_SPLIT: return psn::solve_dt<psn::DT_SPLIT>(p, rho, u, stream, ev);
    }
    return hipErrorInvalidValue;
}

bool size_compiled(int n) {
    switch (n) {
#define PSN_CASE(NN) \
    case NN: return true;
        PSN_FOR_EACH_SIZE(PSN_CASE)
#undef PSN_CASE
        default: return false;
    }
}

}  // namespace psn_host
