// Grids with a different number of points per axis (paper section 2's
// general box, N = n0 n1 n2 points, section 3): the same convolution, run as
// five line-transform steps over their own workspaces.  Each step transforms
// lines of one axis at that axis' padded length L = 2 n_q, with the zero half
// of the input formed in registers and only the needed outputs stored:
//
//   1  axis 2, real -> complex:  rho[i0][i1][0..n2)  -> W1[i0][i1][0..n2]      (n2 + 1 outputs)
//   2  axis 1, forward:          W1[i0][0..n1)[k2]   -> W2(i0, 0..2n1, k2)
//   3  axis 0, forward, x K, inverse, in place on W2(0..n0, k1, k2)
//   4  axis 1, inverse:          W2(i0, 0..2n1, k2)  -> W1[i0][0..n1)[k2]
//   5  axis 2, complex -> real:  W1[i0][i1][0..n2]   -> u[i0][i1][0..n2)
//
// The workspace rows hold hw = g_pitch(n2) >= n2 + 1 elements (a multiple of
// kGTile; the tail is never read into a result).  W2 is blocked over k1 and
// tiled over k2 as [k1 / KB][i0][k2 / kGTile][k1 % KB][k2 % kGTile]
// (KB = w2_k1_block(n1), dividing 2 n1): a workgroup of the axis-0 step then
// spans n0 KB rows instead of the whole array, and one of the axis-1 steps
// 2 n1 / KB runs of KB kGTile elements, consecutive k1 of its tile next to
// each other, so that its two chains' stores fill whole lines and the pages
// either step touches stay few.  K is the octant
// (k_q = 0..n_q, folded index min(k, 2 n_q - k)) scaled by 1 / (8 n0 n1 n2),
// tiled over k2 as g_k_index lays it out.  A workgroup holds B lines with
// the same element stride: consecutive lines of an axis-2 step are rows
// (threads run along a row), those of the other steps are consecutive k2 of
// one aligned tile (threads of consecutive lines touch consecutive
// addresses; lines with k2 > n2 only pad the tile).
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
    int kb;   // k1 block of W2 (a power of two)
    int kbs;  // log2 kb
};

// Every step runs transforms of length FL = L/2 = n_q.  The axis-2 steps
// (1, 5) transform the real line as n2/2 packed pairs.  The strided steps split
// the padded length-L transform of a line whose second half is zero into two
// length-n_q chains: forward, the even outputs are DFT(x) and the odd ones
// DFT(x w^p), w = exp(-2 pi i / L); the inverse that keeps the first n_q
// outputs is IDFT(even) + w^-p IDFT(odd).  The two chains of a line advance in
// lockstep through one LDS exchange.
// B lines per workgroup: for the strided steps kGTile, within the 160 KB of
// LDS (64-byte FP32 row pieces; two workgroups of eight length-512 lines
// share a CU, which measured faster than one of sixteen); for the row steps
// up to 16 and 512 threads within 80 KB, so that two workgroups share a CU
// and each fills its twiddle table for twice the rows (as P1/P5).
// The row steps keep each line as an LDS row of pitch NP (threads of a team
// walk along it; the skew of one slot per 16 and a pitch of 8 mod 32 spread a
// wave's accesses over the banks); the strided steps keep the lines as columns
// (consecutive lanes, consecutive lines), both chains side by side.  All need
// the length-FL table exp(-2 pi i m / L), m < 2 FL.  The strided steps take at
// most 8 elements per thread, so that enough waves fit beside their LDS.
template <int L, class Real, int STEP>
struct GCfg {
    static constexpr bool rows = STEP == 1 || STEP == 5;
    static constexpr int FL = L / 2;
    static constexpr int E = elems_per_thread(FL, rows ? int(sizeof(Real)) : 8);
    static constexpr int T = FL / E;
    static constexpr int CX = sizeof(cx<Real>);
    // The axis-0 step at n0 >= 512 reads its stage twiddles from per-stage
    // rows (one row per thread and stage, as P3 does at those sizes), the
    // other steps from the swizzled table.
    static constexpr bool trows = STEP == 3 && FL >= 512;
    using Ff = TeamFFT<FL, T, Real, -1, false>;
    using Fi = TeamFFT<FL, T, Real, +1, STEP == 3>;
    static constexpr int tw_slots() {
        if constexpr (trows) return Ff::rows_size() + (Ff::template same_rows<Fi>() ? 0 : Fi::rows_size());
        else return TwLds<Real>::slots(FL);
    }
    static constexpr int TWS = tw_slots();
    static constexpr int pitch() {
        int np = FL + (FL >> 4) + 1;
        while (np % 32 != 8) ++np;
        return np;
    }
    // The strided steps exchange their two chains one after the other
    // through a one-chain area (two more barriers per exchange), so that more
    // workgroups share a CU; at n_q >= 512 they ask the compiler for six
    // waves per SIMD in FP32 (at most 80 VGPRs: three workgroups) and four in
    // FP64 arithmetic (at most 128 VGPRs: two workgroups; the axis-0 step then
    // spills a few registers and still runs about 5 % faster).
    static constexpr bool seq = STEP >= 2 && STEP <= 4;
    static constexpr int min_waves = seq && FL >= 512 ? (sizeof(Real) == 4 ? 6 : 4) : 1;
    static constexpr int NP = rows ? pitch() : seq ? FL : 2 * FL;  // LDS elements per line
    static constexpr int pick() {
        if constexpr (rows) {
            for (int b = 16; b > 1; b /= 2)
                if ((b * NP + TWS) * CX <= 81920 && b * T <= 512) return b;
        } else {
            for (int b = psn_host::kGTile; b > 1; b /= 2)
                if ((b * NP + TWS) * CX <= 163840 && b * T <= 1024) return b;
        }
        return 1;
    }
    static constexpr int B = pick();
    static_assert(rows || B == psn_host::kGTile, "a strided workgroup is one whole k2 tile");
    static constexpr size_t lds = size_t(B * NP + TWS) * CX;
};

template <int L, class Real, class Io, int STEP>
__global__ void __launch_bounds__((GCfg<L, Real, STEP>::B * GCfg<L, Real, STEP>::T), (GCfg<L, Real, STEP>::min_waves))
    g_step(const GArgs<Real, Io> a) {
    using C = GCfg<L, Real, STEP>;
    constexpr int B = C::B, T = C::T;
    constexpr bool rows = STEP == 1 || STEP == 5;
    constexpr int FL = C::FL;
    using Ff = TeamFFT<FL, T, Real, -1, false>;
    using Fi = TeamFFT<FL, T, Real, +1, STEP == 3>;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int n0 = a.n0, n1 = a.n1, n2 = a.n2;
    const int h = n2 + 1;                 // k2 of the spectrum
    const long hw = psn_host::g_pitch(n2);  // elements per workspace row
    const int kb = a.kb, kbs = a.kbs;
    // offset of W2 element (i0, k1, k2)
    constexpr long KT = psn_host::kGTile;
    auto w2at = [&](long i0, long k1, long k2) {
        return (((k1 >> kbs) * n0 + i0) * (hw / KT) + k2 / KT) * (kb * KT) + (k1 & (kb - 1)) * KT + k2 % KT;
    };
    const int c = rows ? int(threadIdx.x) / T : int(threadIdx.x) % B;
    const int t = rows ? int(threadIdx.x) % T : int(threadIdx.x) / B;
    long nlines;
    if constexpr (STEP == 1 || STEP == 5) nlines = long(n0) * n1;
    else if constexpr (STEP == 3) nlines = 2L * n1 * hw;
    else nlines = long(n0) * hw;
    // workgroups are dealt to the 8 XCDs round robin: give each XCD a
    // contiguous run of line groups (neighbours share cache lines in its L2);
    // the grid is a multiple of 8, and groups past the end leave at once
    const long grp = long(blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;
    if (grp * B >= nlines) return;  // whole workgroup
    const long line = grp * B + c;
    // a partial last workgroup, and the lines of a tile past k2 = n2, still
    // join every barrier
    [[maybe_unused]] const bool live = line < nlines && (rows || line % hw < h);
    [[maybe_unused]] const long ln = live ? line : 0;
    // the length-FL table from every other entry of the step's length-L
    // table, or the twiddle rows of both transforms (taken from the same)
    TwLds<Real> tl{sb + B * C::NP};
    cx<Real>* const rows_f = sb + B * C::NP;
    cx<Real>* const rows_i = rows_f + (Ff::template same_rows<Fi>() ? 0 : Ff::rows_size());
    if constexpr (C::trows) {
        Ff::template fill_rows<1, 2>(rows_f, a.tw, threadIdx.x, B * T);
        if constexpr (!Ff::template same_rows<Fi>()) Fi::template fill_rows<1, 2>(rows_i, a.tw, threadIdx.x, B * T);
    } else {
        for (int i = threadIdx.x; i < L; i += B * T) tl.p[TwLds<Real>::at(i)] = a.tw[2 * i];
    }
    __syncthreads();
    using View = std::conditional_t<rows, LdsRows<Real>, std::conditional_t<C::seq, LdsColsSeq<Real>, LdsCols2<Real>>>;
    View lds = [&] {
        if constexpr (rows) return LdsRows<Real>{sb + c * C::NP};
        else if constexpr (C::seq) return LdsColsSeq<Real>{sb, B, c};
        else return LdsCols2<Real>{sb, B, c};
    }();
    cx<Real> d[C::E];          // the row steps' line
    cx<Real> d2[2][C::E];      // the strided steps' two chains
    if constexpr (STEP == 1) {
        // Real row of n2 = FL samples, zero beyond: z_j = x_2j + i x_2j+1
        // (j < FL/2, zero beyond), Z = DFT_FL(z), then the padded spectrum
        // X[k] = E[k] + w^k O[k], w = exp(-2 pi i / L), with E and O the
        // transforms of the even and odd samples, E = (Z[k] + conj Z[FL-k])/2,
        // O = (Z[k] - conj Z[FL-k])/(2i); X[0] and X[FL] come from Z[0].
        using Fh = TeamFFT<FL, T, Real, -1, false>;
        const Io* x = a.rho + ln * n2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int j = Fh::in_pos(t, e);
            d[e] = (live && j < FL / 2) ? cx<Real>{Real(x[2 * j]), Real(x[2 * j + 1])} : cx<Real>{Real(0), Real(0)};
        }
        Fh::run1(d, t, tl, lds);
        __syncthreads();  // the transform's last exchange reads are done
#pragma unroll
        for (int e = 0; e < C::E; ++e) lds.put(Fh::out_pos(t, e), d[e]);
        __syncthreads();
        cx<Real>* y = a.w1 + ln * hw;
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
                if (live) gst(y + k, Ev + Od * tl(k));
            }
        }
    } else if constexpr (STEP == 2) {
        const long i0 = ln / hw, k2 = ln % hw;
        const cx<Real>* x = a.w1 + i0 * n1 * hw + k2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Ff::in_pos(t, e);
            d2[0][e] = live ? gld(x + long(p) * hw) : cx<Real>{Real(0), Real(0)};
            d2[1][e] = d2[0][e] * a.tw[2 * p];
        }
        Ff::template run<2>(d2, t, tl, lds);
        // output k1 = 2m + chain.  The workgroup's 2 n1 x B outputs are one
        // tile of W2 in each of the 2 n1 / KB k1 blocks, each a run of KB B
        // elements.  Stage them in LDS in k1-major order, then store the runs,
        // two elements per lane (lanes of padding lines store padding).  The
        // exchange area holds R of the 2 n1 B values: one round with both
        // chains' area, two with the one-chain area (k1 < n1, then k1 >= n1).
        // Every lane stores for the whole workgroup: its i0 and tile come from
        // the workgroup's first line (B divides hw, and no workgroup is
        // partial), not from the lane's own line.
        const long i0w = grp * B / hw, k2w = grp * B % hw;
        const int run = kb * B;
        constexpr int rounds = C::seq ? 2 : 1;
        constexpr int K1R = 2 * FL / rounds;  // k1 per round
        constexpr int NQ = K1R / (2 * T);     // stores per lane and round, two elements each
#pragma unroll
        for (int h = 0; h < rounds; ++h) {
            __syncthreads();  // the transform's last exchange (or the last round's stores) read the area
#pragma unroll
            for (int e = 0; e < C::E; ++e) {
                const int m = Ff::out_pos(t, e);
#pragma unroll
                for (int ch = 0; ch < 2; ++ch) {
                    const int k1 = 2 * m + ch - h * K1R;
                    if (k1 >= 0 && k1 < K1R) sb[k1 * B + c] = d2[ch][e];
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NQ; ++r) {
                const int q = 2 * int(threadIdx.x) + r * 2 * B * T;  // in this round's area
                const int qg = h * K1R * B + q;                         // among the 2 n1 B outputs
                cx<Real>* y = a.w2 + w2at(i0w, long(qg >> (kbs + __builtin_ctz(B))) * kb, k2w) + (qg & (run - 1));
                if constexpr (sizeof(Real) == 4) {
                    gst2(y, sb[q], sb[q + 1]);
                } else {
                    gst(y, sb[q]);
                    gst(y + 1, sb[q + 1]);
                }
            }
        }
    } else if constexpr (STEP == 3) {
        // B divides hw, and 2 n1 hw lines are whole workgroups: a workgroup
        // holds one k1 and B columns of one aligned k2 tile, every lane
        // addresses W2 and K inside their rows (lanes past k2 = n2 work on the
        // padding), and the addresses are a workgroup-uniform base per element
        // plus one 32-bit lane offset.  The axis length n0 is the compile-time
        // FL.  Consecutive groups of one tile take k1 = 0, 2 n1 - 1, 1,
        // 2 n1 - 2, ...: each pair k1, 2 n1 - k1 shares a kernel row, and k1,
        // k1 + 1 (two groups apart) share the lines of their W2 pieces.
        constexpr int N0 = FL;
        long g = grp;
        const long sub = g % (KT / B);
        g /= KT / B;
        const long q = g % (2L * n1);
        const long k1 = q % 2 == 0 ? q / 2 : 2L * n1 - (q + 1) / 2;
        const long k2b = (g / (2L * n1)) * KT + sub * B;
        const uint32_t s0 = uint32_t(kb) * uint32_t(hw);  // i0 stride
        cx<Real>* const xu = a.w2 + w2at(0, k1, k2b);
        const uint32_t xl = (uint32_t(c) + uint32_t(t) * s0) * uint32_t(sizeof(cx<Real>));
        const uint32_t wl = uint32_t(2 * t) * uint32_t(sizeof(cx<Real>));
        cx<Real> w[C::E];  // w^p of each input position p = t + in_pos(0, e)
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p0 = Ff::in_pos(0, e);
            w[e] = gld(byte_off(sbase(a.tw + 2 * p0), wl));
            d2[0][e] = gld(byte_off(sbase(xu + size_t(p0) * s0), xl));
            d2[1][e] = d2[0][e] * w[e];
        }
        if constexpr (C::trows) Ff::template run<2>(d2, t, TwRows<Real>{rows_f}, lds);
        else Ff::template run<2>(d2, t, tl, lds);
        // kernel values of the outputs k0 = 2m + chain, m = t + out_pos(0, e),
        // at the folded index min(k0, 2 n0 - k0); the folded k0 steps by
        // kGTile.  An element whose k0 all lie on one side of n0 is a uniform
        // base plus the lane offset 2t or -2t (written as 2 (T - 1 - t)).
        const int k1f = int(k1 <= n1 ? k1 : 2 * n1 - k1);
        const Real* const Ku = a.K + psn_host::g_k_index(N0, n2, 0, k1f, int(k2b));
        const uint32_t kup = (uint32_t(2 * KT) * uint32_t(t) + uint32_t(c)) * uint32_t(sizeof(Real));
        const uint32_t kdn = (uint32_t(2 * KT) * uint32_t(T - 1 - t) + uint32_t(c)) * uint32_t(sizeof(Real));
        Real kk[2][C::E];
#pragma unroll
        for (int e = 0; e < C::E; ++e)
#pragma unroll
            for (int ch = 0; ch < 2; ++ch) {
                const int a0 = 2 * Ff::out_pos(0, e) + ch;  // k0 of lane t = 0
                if (a0 + 2 * (T - 1) <= N0) {
                    kk[ch][e] = gld(byte_off(sbase(Ku + a0 * KT), kup));
                } else if (a0 >= N0) {
                    kk[ch][e] = gld(byte_off(sbase(Ku + (2 * N0 - a0 - 2 * (T - 1)) * KT), kdn));
                } else {
                    const int k0 = a0 + 2 * t;
                    kk[ch][e] = Ku[(k0 <= N0 ? k0 : 2 * N0 - k0) * KT + c];
                }
            }
        // radices reversed: starts from the forward output layout and ends in
        // its input layout (slot e at position Ff::in_pos(t, e))
        if constexpr (C::trows) Fi::template run_scaled<2>(d2, t, TwRows<Real>{rows_i}, lds, kk);
        else Fi::template run_scaled<2>(d2, t, tl, lds, kk);
#pragma unroll
        for (int e = 0; e < C::E; ++e)
            gst(byte_off(sbase(xu + size_t(Ff::in_pos(0, e)) * s0), xl), twfma<+1>(d2[1][e], w[e], d2[0][e]));
    } else if constexpr (STEP == 4) {
        const long i0 = ln / hw, k2 = ln % hw;
        const cx<Real>* x = a.w2;  // input k1 = 2m + chain
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const long m = Fi::in_pos(t, e);
            d2[0][e] = live ? gld(x + w2at(i0, 2 * m, k2)) : cx<Real>{Real(0), Real(0)};
            d2[1][e] = live ? gld(x + w2at(i0, 2 * m + 1, k2)) : cx<Real>{Real(0), Real(0)};
        }
        Fi::template run<2>(d2, t, tl, lds);
        cx<Real>* y = a.w1 + i0 * n1 * hw + k2;
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int p = Fi::out_pos(t, e);
            if (live) gst(y + long(p) * hw, twfma<+1>(d2[1][e], a.tw[2 * p], d2[0][e]));
        }
    } else {
        // The row's padded spectrum X[0..FL] is that of a real sequence.  The
        // inverse of length FL of Y[k] = (X[k] + conj X[FL-k])
        // + i (X[k] - conj X[FL-k]) w^-k gives z_j = u_2j + i u_2j+1; only
        // j < FL/2 lies inside the box.
        // Each X[k] is loaded once, into the line's LDS row (X[FL] by its
        // first thread), and the partner X[FL-k] read back from there.
        using Fh = TeamFFT<FL, T, Real, +1, false>;
        const cx<Real>* x = a.w1 + ln * hw;
#pragma unroll
        for (int e = 0; e < C::E; ++e) d[e] = live ? gld(x + Fh::in_pos(t, e)) : cx<Real>{Real(0), Real(0)};
        const cx<Real> last = (live && t == 0) ? gld(x + FL) : cx<Real>{Real(0), Real(0)};
#pragma unroll
        for (int e = 0; e < C::E; ++e) lds.put(Fh::in_pos(t, e), d[e]);
        if (t == 0) lds.put(FL, last);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < C::E; ++e) {
            const int k = Fh::in_pos(t, e);
            const cx<Real> p = d[e], q = conj(lds.get(FL - k));
            d[e] = (p + q) + rot<+1>(mul_conj(p - q, tl(k)));
        }
        Fh::run1(d, t, tl, lds);  // its first exchange waits before reusing the row
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
