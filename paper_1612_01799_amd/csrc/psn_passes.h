// The five pruned passes of one solve (paper section 2: the size-8N transform
// pair of I_1 with the G-tensor multiply; section 3: its cost).
//
// Layout (C order, last index contiguous), M = 2n:
//   rho, u : [i0][i1][i2]            n^3 reals
//   W1     : [i0][k2/BL][i1][k2%BL]  n^3 complex, k2 = 0..n-1, tiled over k2
//            (BL = the axis-1 column tile) so that an axis-1 workgroup's
//            column block is one contiguous run
//   W2     : n * M * n complex, blocked over k1 and tiled over k2 (W2Index)
//            so that both the axis-1 passes (fixed i0, all k1) and the axis-0
//            pass (fixed k1, all i0) read and write long contiguous runs
//   K      : [k1~][k2/KT][k0~][k2%KT] (n+1)^2 * n reals, folded k~ = min(k, M-k)
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
#pragma once

#include "psn_device.h"
#include "psn_internal.h"

#include <type_traits>

namespace psn {

constexpr int kMaxLds = 65536;       // per workgroup for the one-chain passes
constexpr int kMaxLdsP3 = 163840;    // gfx950: 160 KB of LDS per workgroup

constexpr int pick_cols(int N, int bmax, int sets, int cxbytes, int T) {
    for (int b = bmax; b >= 1; --b)
        if (N % b == 0 && sets * b * N * cxbytes <= kMaxLds && sets * b * T <= 1024) return b;
    return 1;
}

constexpr int pick_cols_p3(int N, int bmax, int cxbytes, int T) {
    for (int b = bmax; b >= 1; --b)
        if (N % b == 0 && (2 * b * N + ((2 * N + 15) & ~15)) * cxbytes <= kMaxLdsP3 && b * T <= 1024) return b;
    return 1;
}

// largest P3 tile width <= bmax that fits and divides the W2 layout tile
constexpr int pick_cols_p3_div(int N, int bmax, int cxbytes, int T, int layout_tile) {
    for (int b = bmax; b >= 1; --b)
        if (N % b == 0 && layout_tile % b == 0 && (2 * b * N + ((2 * N + 15) & ~15)) * cxbytes <= kMaxLdsP3 &&
            b * T <= 1024)
            return b;
    return 1;
}

// LDS row pitch of the contiguous passes (in elements): room for the skew of
// one slot per 16, rounded to 8 mod 32 so that the rows one wave touches at
// once (8-byte elements: 4 rows per 256-byte bank sweep; 16-byte: 2 rows)
// start in different banks
constexpr int rows_padded(int N) {
    int np = N + (N >> 4) + 1;
    while (np % 32 != 8) ++np;
    return np;
}

// lines per workgroup of the contiguous passes (up to `threads` threads);
// their LDS, at most `lds` bytes, holds the lines and the 2N-entry twiddle table
constexpr int pick_lines(int N, int T, int cxbytes, int threads, int lds) {
    int l = threads / T;
    if (l < 1) l = 1;
    while (l > 1 && (N % l != 0 || (l * rows_padded(N) + ((2 * N + 15) & ~15)) * cxbytes > lds)) l /= 2;
    if (l * T < 64) {
        // halving left less than a wave (odd team sizes): any divisor of N that fits
        for (int d = threads / T; d > l; --d)
            if (N % d == 0 && (d * rows_padded(N) + ((2 * N + 15) & ~15)) * cxbytes <= lds) return d;
    }
    return l;
}
// P1 and P5: up to 512 threads and 80 KB, so that two workgroups share a CU
// (at n = 512 FP32, 16 lines instead of 8: both passes about 5 % faster)
constexpr int kMaxLdsRows = 81920;

// W2 layout, tile-major: element (i0, k1, k2) lives at
//   slot / KB * blk + (i0 * (N / BL) + k2 / BL) * (KB * BL) + (slot % KB) * BL + k2 % BL
// with slot(k1) putting rows k1 and M-k1 next to each other (rows 0 and n
// form pair 0) and blk = N * N * KB plus a small pad, so that the k1 blocks of
// one tile, otherwise a power of two apart, do not share cache sets.  So the axis-1 passes (one i0, one tile of BL columns, all k1)
// write and read runs of KB * BL contiguous elements, and the two workgroups
// of the axis-0 pass that share a kernel row (k1 and M-k1) read the two halves
// of the same 128-byte lines.  BL is the column tile of the axis-1 passes.
//
// Paired form (PAIR): two consecutive i0 of a column sit next to each other,
//   slot / KB * blk + (i0 / 2 * (N / BL) + k2 / BL) * (2 KB BL) + (slot % KB) * 2 BL + (k2 % BL) * 2 + i0 % 2,
// so a slot row of a tile holds BL columns x 2 i0 (128 bytes in FP32), the
// axis-0 pass reads one 16-byte pair per lane and whole rows per eight lanes,
// and the axis-1 passes, each workgroup handling an i0 pair, move runs of
// 2 KB BL elements.
template <int N, int BL, bool PAIR = false>
struct W2Index {
    static constexpr int KB = psn_host::w2_k1_block(N);
    static constexpr size_t blk = size_t(N) * N * KB + psn_host::kW2BlockPad;  // stride of k1 blocks
    static_assert(N % BL == 0 && (2 * N) % KB == 0, "");
    static __device__ __forceinline__ int slot(int k1) {
        if (k1 == 0) return 0;
        if (k1 == N) return 1;
        return k1 < N ? 2 * k1 : 2 * (2 * N - k1) + 1;
    }
    static __device__ __forceinline__ size_t at(int i0, int k1, int k2) {
        const int sl = slot(k1);
        if constexpr (PAIR) {
            return size_t(sl / KB) * blk + (size_t(i0 >> 1) * (N / BL) + k2 / BL) * size_t(2 * KB * BL) +
                   size_t(sl % KB) * (2 * BL) + (k2 % BL) * 2 + (i0 & 1);
        } else {
            return size_t(sl / KB) * blk + (size_t(i0) * (N / BL) + k2 / BL) * size_t(KB * BL) +
                   size_t(sl % KB) * BL + k2 % BL;
        }
    }
    // stride between consecutive i0 (PAIR: consecutive i0 pairs) at fixed (k1, k2)
    static constexpr size_t s0 = size_t(N) * KB * (PAIR ? 2 : 1);
};

// Sizes whose W2 is stored in the paired form.  The axis-0 pass then splits
// each line by decimation in time into its even and odd samples, giving four
// half-length chains per line; the axis-1 passes take an i0 pair per
// workgroup.
// FP32 only: the FP64-arithmetic precisions already move 16 bytes per lane
// and element, and their paired axis-1 passes measured slower (one 144 KB
// workgroup per CU then holds two lines per column).
template <int N, int DT>
struct PairW2 {
    static constexpr bool value = DT == DT_F32 && N >= 16 && (N & (N - 1)) == 0;
};

// W1 layout, tiled over k2: element (i0, i1, k2) lives at
//   ((i0 * (N / BL) + k2 / BL) * N + i1) * BL + k2 % BL,
// so the axis-1 passes (one i0, one tile of BL columns, all i1) move one
// contiguous block and the axis-2 passes (a few lines i1 of one i0) move
// runs of lines * BL elements.
template <int N, int BL>
struct W1Index {
    static_assert(N % BL == 0, "");
    static __device__ __forceinline__ size_t at(int i0, int i1, int k2) {
        return ((size_t(i0) * (N / BL) + k2 / BL) * N + i1) * BL + k2 % BL;
    }
};

template <int N, int DT>
struct Cfg {
    using P = Prec<DT>;
    using Real = typename P::Real;
    using Io = typename P::Io;
    using Kt = typename P::Kt;
    static constexpr int E = elems_per_thread(N, sizeof(Real));
    static constexpr int T = N / E;
    static constexpr int CX = sizeof(cx<Real>);
    static constexpr int T24 = N / elems_per_thread(N, 8);                     // P2, P4 team (two chains)
    static constexpr int BS = pick_cols_p3(N, 8, CX, T24);                     // P2, P4 columns
    static constexpr int T3 = N / elems_per_thread(N, 8);                      // P3 team (two chains)
    static constexpr int BP3 = pick_cols_p3_div(N, DT == DT_F32 ? 8 : 4, CX, T3, BS);  // P3 columns (divide BS)
    static_assert(BS % BP3 == 0, "P3 tile must lie inside the W2 layout tile");
    static constexpr int LC = pick_lines(N, T, CX, 512, kMaxLdsRows);          // P1, P5 lines
    static constexpr int NP = rows_padded(N);
};

// One launch serves up to kMaxBatch problems of the same size.  The table
// travels by value in the kernel arguments (no device copy, capturable in a
// graph); workgroup units are numbered problem-major.
constexpr int kMaxBatch = kMaxBatchHost;

// Storage of the axis-1 output W2: split precision keeps it in FP64.  The
// middle pass reads and writes W2 in narrow column tiles at large strides,
// where 12-byte elements straddle the memory's 64-byte sectors; W1, moved in
// whole tile runs by the axis passes, keeps the 12-byte form.
template <int DT>
constexpr int w2_dt() {
    return DT == DT_SPLIT ? DT_F64 : DT;
}

template <int DT>
struct Prob {
    const typename Prec<DT>::Io* rho;
    typename Prec<DT>::Io* u;
    Work<DT> w1;
    Work<w2_dt<DT>()> w2;
    const typename Prec<DT>::Kt* K;
    const typename Prec<DT>::Kt* Kb;
    const cx<typename Prec<DT>::Real>* tw;
};

template <int DT>
struct Batch {
    int count;
    Prob<DT> p[kMaxBatch];
};

// Workgroup ids are dealt to the XCDs round robin; give each XCD a contiguous
// run of units so neighbouring tiles (which may share 128-byte lines) meet in
// the same L2.
__device__ __forceinline__ int xcd_unit() {
    const int g = blockIdx.x;
    return (g % 8) * (gridDim.x / 8) + g / 8;
}

// Grid size for `units` units dealt by xcd_unit().
inline int xcd_grid(long units) { return int(8 * ((units + 7) / 8)); }

// The LC * N W1 elements of an axis-2 workgroup in tile-contiguous order:
// element j = tid + LC * T * q is line lj = j / BL % LC and column
// k = j / (BL * LC) * BL + j % BL, so consecutive threads touch consecutive W1
// addresses.  When BL divides T, k = k0 + T * q with lj and k0 fixed per thread.
template <int N, int LC, int T, int BL>
struct TileOrder {
    static constexpr bool split = T % BL == 0;
    static __device__ __forceinline__ void at(int tid, int q, int& lj, int& k0, int& off) {
        if constexpr (split) {
            lj = (tid / BL) % LC;
            k0 = (tid / (BL * LC)) * BL + tid % BL;
            off = T * q;
        } else {
            const int j = tid + LC * T * q;
            lj = (j / BL) % LC;
            k0 = (j / (BL * LC)) * BL + j % BL;
            off = 0;
        }
    }
};

// ------------------------------------------------------------------ P1
template <int N, int DT>
__global__ void __launch_bounds__((Cfg<N, DT>::LC * Cfg<N, DT>::T))
p1_r2c(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, C::T, Real, -1, false>;
    constexpr int units = N * N / C::LC;  // per problem
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;
    const Prob<DT>& P = bt.p[ug / units];
    const Work<DT>& w1 = P.w1;
    const cx<Real>* __restrict__ tw = P.tw;
    const int t = threadIdx.x % C::T, ln = threadIdx.x / C::T;
    const int line0 = (ug % units) * C::LC;  // first line of the workgroup; all share i0
    const int i0 = line0 / N, i1b = line0 % N;
    const typename C::Io* x = P.rho + (size_t(line0) + ln) * N;

    // z[j] = x[2j] + i x[2j+1]; zero for j >= n/2 (the padding)
    cx<Real> d[F::E];
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        const int pos = F::in_pos(t, e);
        if (pos < N / 2) d[e] = {Real(x[2 * pos]), Real(x[2 * pos + 1])};
        else d[e] = {Real(0), Real(0)};
    }
    TwLds<Real> tl{sb + C::LC * C::NP};
    tl.fill(tw, N, threadIdx.x, C::LC * C::T);
    LdsRows<Real> lds{sb + ln * C::NP};
    F::run1(d, t, tl, lds);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < F::E; ++e) lds.put2(t, F::out_pos(0, e), d[e]);  // out_pos(t, e) = t + out_pos(0, e)
    __syncthreads();
    // X[k] = E[k] + w^k O[k], E = (Z[k] + conj Z[n-k])/2, O = (Z[k] - conj Z[n-k])/(2i).
    // Element j of the workgroup's LC * N outputs is (line j / BS % LC,
    // k = j / (BS * LC) * BS + j % BS): consecutive threads write consecutive
    // W1 addresses.
    constexpr int BL = C::BS;
    using W1I = W1Index<N, BL>;
    using TO = TileOrder<N, C::LC, C::T, BL>;
#pragma unroll
    for (int q = 0; q < F::E; ++q) {
        int lj, k0, off;
        TO::at(int(threadIdx.x), q, lj, k0, off);
        const int k = k0 + off;
        const LdsRows<Real> row{sb + lj * C::NP};
        const cx<Real> Z = row.get2(k0, off);
        cx<Real> X;
        if (k == 0) {
            X = {Z.x + Z.y, Z.x - Z.y};  // (X[0], X[n]) packed
        } else {
            const cx<Real> Zr = conj(row.get2(N - k0, -off));
            const cx<Real> Ev = scale(Z + Zr, Real(0.5));
            const cx<Real> Od = rot<-1>(scale(Z - Zr, Real(0.5)));
            X = Ev + Od * tl(k);
        }
        w1.st(W1I::at(i0, i1b + lj, k), X);
    }
}

// ------------------------------------------------------------------ P2
// Unit = (i0, tile of B columns k2).  Both outputs of a line (DFT_n of x and
// of x w^j) are computed in lockstep from the same loads.
// LDS view of the strided passes: both chains side by side, or one at a time
template <class Real, bool SEQ>
using ChainLds = std::conditional_t<SEQ, LdsColsSeq<Real>, LdsCols2<Real>>;

template <int N, int DT, int B, int TT, bool SEQ>
__global__ void __launch_bounds__((B * TT), (SEQ && N / TT <= 8 ? 3 : 1))
p2_fwd(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, TT, Real, -1, false>;
    using WI = W2Index<N, Cfg<N, DT>::BS>;
    static_assert(B == Cfg<N, DT>::BS, "the axis-1 tile is the W2 layout tile");
    constexpr int E = F::E;
    constexpr int tiles = N / B;
    constexpr int units = N * tiles;  // per problem
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    cx<Real>* stw = sb + (SEQ ? 1 : 2) * B * N;
    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;
    const Prob<DT>& P = bt.p[ug / units];
    const Work<DT>& w1 = P.w1;
    const auto& w2 = P.w2;
    const cx<Real>* __restrict__ tw = P.tw;
    const int u = ug % units;
    const int i0 = u / tiles, tile = u % tiles;
    const int c = threadIdx.x % B, t = threadIdx.x / B;
    const int k2 = tile * B + c;
    using W1I = W1Index<N, B>;

    cx<Real> d[2][E], w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int pos = F::in_pos(t, e);
        d[0][e] = w1.ld(W1I::at(i0, pos, k2));
        w[e] = tw[pos];
    }
    TwLds<Real> tl{stw};
    tl.fill(tw, N, threadIdx.x, B * TT);  // visible after the first exchange
#pragma unroll
    for (int e = 0; e < E; ++e) d[1][e] = d[0][e] * w[e];
    ChainLds<Real, SEQ> lds{sb, B, c};
    F::template run<2>(d, t, tl, lds);
    {
        // Stage the workgroup's output in LDS in W2 order (slot-major, B columns
        // per slot), then store whole runs of KB * B elements, two consecutive
        // elements per lane.  The two-chain exchange area holds all 2N slots;
        // the one-chain area holds N, so that variant stages in two rounds.
        constexpr int KB = WI::KB, RUN = KB * B;
        constexpr int HALF = SEQ ? N : 2 * N;  // slots per round
        static_assert((HALF * B) % RUN == 0, "rounds cover whole runs");
        const size_t tile0 = WI::at(i0, 0, tile * B);  // (slot 0, column tile*B): start of block 0's run
#pragma unroll
        for (int h = 0; h < 2 * N / HALF; ++h) {
            __syncthreads();  // the last exchange's (or round's) reads are done
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int m = F::out_pos(t, e);
#pragma unroll
                for (int ch = 0; ch < 2; ++ch) {
                    const int sl = WI::slot(2 * m + ch) - h * HALF;
                    if (sl >= 0 && sl < HALF) sb[sl * B + c] = d[ch][e];
                }
            }
            __syncthreads();
            for (int g = 2 * int(threadIdx.x); g < HALF * B; g += 2 * B * TT) {
                const int gg = h * HALF * B + g;
                w2.st2(tile0 + size_t(gg / RUN) * WI::blk + gg % RUN, sb[g], sb[g + 1]);
            }
        }
    }
}

// ------------------------------------------------------------------ P3
// One workgroup = SL rows of W2 and B adjacent columns k2.  With SL = 2 the
// rows are k1 and M-k1, which share a kernel row and sit next to each other in
// the W2 layout, so each i0 is one run of 2 * B elements; with SL = 1 the two
// rows go to consecutive units instead.  The two parity chains (even and odd
// k0) of each line advance in lockstep, stored side by side in LDS, so one pair
// of barriers and one 16-byte access per element serve both.  Workgroup ids
// are dealt to the XCDs round robin; each XCD gets a contiguous run of units,
// so tiles sharing 128-byte lines and rows sharing a kernel row meet in the
// same L2.  All global loads (data, the pre/post twiddles of the odd chain and
// the kernel values) are issued before any arithmetic; the stage twiddles come
// from a copy of the table in LDS.  Column 0 (the packed k2 = 0 / k2 = n pair)
// is left to p3_col0.
template <int N>
struct P3Rows {
    static constexpr bool value = N >= 512;
};

// Minimum waves per SIMD asked of the compiler for P3.  The one-chain variant
// uses little LDS, so it asks for three waves per SIMD (six for 512-thread
// FP32 workgroups with up to 8 elements per thread: three workgroups per CU).
// FP32 keeps few values live across the forward transform (see kLean), so
// this holds up to 20 elements per thread; FP64 arithmetic only up to 8.
// Longer plans are left unbounded, where a bound would only force spills.
constexpr int p3_waves(int e, int threads, bool f32, bool seq) {
    if (!seq || e > (f32 ? 20 : 8)) return 1;
    return f32 && threads > 256 && e <= 8 ? 6 : 3;
}

template <int N, int DT, int B, int TT, int SL, bool SEQ>
__global__ void __launch_bounds__((B * TT * SL), (p3_waves(N / TT, B * TT * SL, DT == DT_F32, SEQ)))
p3_conv(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using Ff = TeamFFT<N, TT, Real, -1, false>;
    using Fi = TeamFFT<N, TT, Real, +1, true>;
    static_assert(SL == 1 || SL == 2, "one row or a row pair per workgroup");
    constexpr int E = Ff::E;
    constexpr int tiles = N / B;
    constexpr int units = (2 / SL) * N * tiles;  // per problem
    using WI = W2Index<N, Cfg<N, DT>::BS>;
    static_assert(Cfg<N, DT>::BS % B == 0, "the axis-0 tile lies inside a W2 layout tile");
    constexpr size_t s0 = WI::s0;  // stride of i0 in W2
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    cx<Real>* stw = sb + (SEQ ? 1 : 2) * B * SL * N;

    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;  // whole workgroup
    const Prob<DT>& P = bt.p[ug / units];
    const auto& w2 = P.w2;
    const typename C::Kt* __restrict__ K = P.K;
    const cx<Real>* __restrict__ tw = P.tw;
    const int u = ug % units;
    int q, tile, set;
    if constexpr (SL == 1) {
        const int item = u >> 1;
        set = u & 1;
        q = item / tiles;
        tile = item % tiles;
    } else {
        q = u / tiles;
        tile = u % tiles;
        set = (threadIdx.x / B) & 1;
    }
    const int c = threadIdx.x % B, t = threadIdx.x / (B * SL);
    const int k2 = tile * B + c;
    // Addresses: a base uniform over the workgroup (row q, column tile * B)
    // plus a 32-bit lane offset.  Row M-q sits BS elements after row q in the
    // W2 layout; its kernel row is q as well, except for the pair (0, n).
    static_assert(WI::s0 * N * sizeof(cx<double>) < (size_t(1) << 32) &&
                      size_t(N + 1) * (N + 1) * N * sizeof(double) < (size_t(1) << 32),
                  "lane byte offsets fit 32 bits");
    const size_t ub = WI::at(0, q, tile * B);
    // element e sits at the uniform base xb(e) plus the lane offset xl
    const uint32_t xl = uint32_t(c) + uint32_t(set) * Cfg<N, DT>::BS + uint32_t(t) * uint32_t(s0);
    auto xb = [&](int e) { return ub + size_t(Ff::in_pos(0, e)) * s0; };
    // Kernel values of the even and odd outputs a = 2m, b = 2m + 1 of
    // m = out_pos(t, e) = t + m0(e), at the folded index min(a, 2N - a) of
    // this lane's kernel row (plane q, or n for the set-1 row of pair 0) in the
    // tiled K layout, where the folded k0 steps by the K tile width KT.  When a
    // whole element lies on one side of n, the folded index is a constant plus
    // 2t or minus 2t: a uniform base plus one of two lane offsets.
    constexpr int KT = psn_host::k_tile(N);
    const typename C::Kt* __restrict__ Kq = K;
    const uint32_t kl = uint32_t(psn_host::k_index(N, (set != 0 && q == 0) ? N : q, 0, k2));
    const uint32_t kup = (kl + uint32_t(2 * t * KT)) * uint32_t(sizeof(typename C::Kt));
    const uint32_t kdn = (kl + uint32_t(2 * (TT - 1 - t) * KT)) * uint32_t(sizeof(typename C::Kt));
    auto kval = [&](int e, int odd) -> Real {
        const int m0 = Ff::out_pos(0, e);
        if (2 * m0 + 2 * TT - 1 <= N) return Real(gld(byte_off(sbase(Kq + (2 * m0 + odd) * KT), kup)));
        if (2 * m0 >= N) return Real(gld(byte_off(sbase(Kq + (2 * N - 2 * m0 - odd - 2 * (TT - 1)) * KT), kdn)));
        const int a = 2 * (m0 + t) + odd;
        return Real(gld(Kq + kl + uint32_t(a <= N ? a : 2 * N - a) * KT));
    };

    cx<Real> x[E], w[E];
    Real kk[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        x[e] = w2.ld(xb(e), xl);
        w[e] = tw[Ff::in_pos(t, e)];
    }
    // FP32 variants with the one-chain exchange or more than 8 elements per
    // thread keep fewer values live across the forward transform (more waves
    // fit): they load the kernel values after it and reload the twiddles w at
    // the end.  The FP64-arithmetic variants measured faster with early loads.
    constexpr bool kLean = DT == DT_F32 && (SEQ || E > 8);
    auto load_k = [&]() {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            kk[0][e] = kval(e, 0);
            kk[1][e] = kval(e, 1);
        }
    };
    if constexpr (!kLean) load_k();
    // Stage twiddles: per-stage rows of both transforms (shared when their
    // radices match) for n >= 512, where the saved index arithmetic outweighs
    // the scattered reads that fill them; else the swizzled 2N-entry table.
    constexpr bool kRows = P3Rows<N>::value;
    cx<Real>* rows_i = stw + (Ff::template same_rows<Fi>() ? 0 : Ff::rows_size());
    TwLds<Real> tl{stw};
    if constexpr (kRows) {
        Ff::fill_rows(stw, tw, threadIdx.x, B * TT * SL);  // visible after the first exchange
        if constexpr (!Ff::template same_rows<Fi>()) Fi::fill_rows(rows_i, tw, threadIdx.x, B * TT * SL);
    } else {
        tl.fill(tw, N, threadIdx.x, B * TT * SL);
    }

    cx<Real> d[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        d[0][e] = x[e];
        d[1][e] = x[e] * w[e];
    }
    ChainLds<Real, SEQ> lds{sb, B * SL, int(threadIdx.x % (B * SL))};
    if constexpr (kRows) Ff::template run<2>(d, t, TwRows<Real>{stw}, lds);
    else Ff::template run<2>(d, t, tl, lds);
    if constexpr (kLean) load_k();
    // the multiply by K is folded into the first stage of the inverse
    if constexpr (kRows) Fi::template run_scaled<2>(d, t, TwRows<Real>{rows_i}, lds, kk);
    else Fi::template run_scaled<2>(d, t, tl, lds, kk);
    if constexpr (kLean) {
#pragma unroll
        for (int e = 0; e < E; ++e) w[e] = gld(byte_off(sbase(tw + Ff::in_pos(0, e)), uint32_t(t) * uint32_t(C::CX)));
    }
    if (k2 != 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) w2.st(xb(e), xl, twfma<+1>(d[1][e], w[e], d[0][e]));
    }
}

// Column 0 of W2 carries Z = A + iB with A, B the spectra of the real k2 = 0
// and k2 = n planes.  With the partner row -k the product is
// Z' = a Z(k) + b conj(Z(-k)), a = (K0+Kn)/2 (stored in K's column 0) and
// b = (K0-Kn)/2 (stored in Kb).  A row pair is rows q and M-q (row 0 pairs
// with itself, as does row n); a workgroup holds Col0::G row pairs so that
// short lines still fill a 64-lane wave.
template <int N, int DT>
struct Col0 {
    // the team of the strided passes (at most 8 elements per thread, twice
    // the threads of the row passes' team at n = 512: 25.8 -> 22.4 us there)
    static constexpr int T = Cfg<N, DT>::T3;
    static constexpr int G = 2 * T >= 64 ? 1 : (64 / (2 * T) < N ? 64 / (2 * T) : N);  // row pairs per workgroup
    static constexpr int groups = (N + G - 1) / G;                                    // workgroups per problem
    static constexpr size_t lds = size_t(G) * 2 * N * Cfg<N, DT>::CX;
};

template <int N, int DT>
__global__ void __launch_bounds__((2 * Col0<N, DT>::T * Col0<N, DT>::G))
p3_col0(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using G0 = Col0<N, DT>;
    using Ff = TeamFFT<N, G0::T, Real, -1, false>;
    using Fi = TeamFFT<N, G0::T, Real, +1, true>;
    using WI = W2Index<N, Cfg<N, DT>::BS, PairW2<N, DT>::value>;
    extern __shared__ __align__(16) unsigned char smem[];

    if (int(blockIdx.x) >= bt.count * G0::groups) return;
    const Prob<DT>& P = bt.p[blockIdx.x / G0::groups];
    const auto& w2 = P.w2;
    const typename C::Kt* __restrict__ K = P.K;
    const typename C::Kt* __restrict__ Kb = P.Kb;
    const cx<Real>* __restrict__ tw = P.tw;
    const int g = threadIdx.x / (2 * G0::T);  // row pair within the workgroup
    const int set = threadIdx.x & 1;
    const int t = (threadIdx.x >> 1) % G0::T;
    const int qg = (blockIdx.x % G0::groups) * G0::G + g;
    const bool live = qg < N;  // the last workgroup may hold pairs past the end
    const int q = live ? qg : N - 1;
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem) + size_t(g) * 2 * N;
    const int k1 = set == 0 ? q : (q == 0 ? N : 2 * N - q);
    const int kt1 = (q == 0) ? (set ? N : 0) : q;
    const int partner = (q == 0) ? set : 1 - set;
    const typename C::Kt* Krow = K + psn_host::k_index(N, kt1, 0, 0);  // column 0 of plane kt1
    const typename C::Kt* Kbr = Kb + size_t(kt1) * (N + 1);

    cx<Real> x[Ff::E], acc[Ff::E];
#pragma unroll
    for (int e = 0; e < Ff::E; ++e) x[e] = w2.ld(WI::at(Ff::in_pos(t, e), k1, 0));
    LdsCols<Real> lds{sb + set, 2, 0};
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        cx<Real> d[Ff::E];
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) d[e] = p ? x[e] * tw[Ff::in_pos(t, e)] : x[e];
        Ff::run(d, t, tw, lds);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) sb[set * N + Ff::out_pos(t, e)] = d[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) {
            const int m = Ff::out_pos(t, e);
            const int k0 = 2 * m + p;
            const int kt0 = k0 <= N ? k0 : 2 * N - k0;
            const int mp = p == 0 ? (m == 0 ? 0 : N - m) : N - 1 - m;
            const cx<Real> zp = conj(sb[partner * N + mp]);
            d[e] = scale(d[e], Real(Krow[size_t(kt0) * psn_host::k_tile(N)])) + scale(zp, Real(Kbr[kt0]));
        }
        Fi::run(d, t, tw, lds);
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) {
            if (p == 0) acc[e] = d[e];
            else acc[e] = acc[e] + mul_conj(d[e], tw[Fi::out_pos(t, e)]);
        }
    }
    if (live) {
#pragma unroll
        for (int e = 0; e < Ff::E; ++e) w2.st(WI::at(Fi::out_pos(t, e), k1, 0), acc[e]);
    }
}

// ------------------------------------------------------------------ P4
// Unit = (i0, tile of B columns k2).  The even and odd rows of a line are
// inverted in lockstep and combined as y = y_even + w^-j y_odd.
template <int N, int DT, int B, int TT, bool SEQ>
__global__ void __launch_bounds__((B * TT), (SEQ && N / TT <= 8 ? 3 : 1))
p4_inv(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, TT, Real, +1, false>;
    using WI = W2Index<N, Cfg<N, DT>::BS>;
    static_assert(B == Cfg<N, DT>::BS, "the axis-1 tile is the W2 layout tile");
    constexpr int E = F::E;
    constexpr int tiles = N / B;
    constexpr int units = N * tiles;  // per problem
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    cx<Real>* stw = sb + (SEQ ? 1 : 2) * B * N;
    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;
    const Prob<DT>& P = bt.p[ug / units];
    const Work<DT>& w1 = P.w1;
    const auto& w2 = P.w2;
    const cx<Real>* __restrict__ tw = P.tw;
    const int u = ug % units;
    const int i0 = u / tiles, tile = u % tiles;
    const int c = threadIdx.x % B, t = threadIdx.x / B;
    const int k2 = tile * B + c;
    using W1I = W1Index<N, B>;

    cx<Real> d[2][E], w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int pos = F::in_pos(t, e);
        d[0][e] = w2.ld(WI::at(i0, 2 * pos, k2));
        d[1][e] = w2.ld(WI::at(i0, 2 * pos + 1, k2));
        w[e] = tw[F::out_pos(t, e)];
    }
    TwLds<Real> tl{stw};
    tl.fill(tw, N, threadIdx.x, B * TT);  // visible after the first exchange
    ChainLds<Real, SEQ> lds{sb, B, c};
    F::template run<2>(d, t, tl, lds);
#pragma unroll
    for (int e = 0; e < E; ++e)
        w1.st(W1I::at(i0, F::out_pos(t, e), k2), twfma<+1>(d[1][e], w[e], d[0][e]));
}

// ------------------------------------------------------------------ paired W2
// Axis-1 forward over an i0 pair: unit = (i0 pair, tile of B columns k2).
// The two lines of each column (i0 = 2p and 2p + 1) are transformed one after
// the other through the same LDS exchange area; the first one's outputs wait
// in registers.  The outputs are then staged in LDS in the paired W2 order and
// stored as whole runs of 2 KB B elements, one 16-byte (FP32) pair per lane.
// Minimum waves per SIMD asked of the compiler for the paired axis-1 passes:
// with up to 8 points per thread, two 512-thread workgroups per CU (the LDS
// allows two) need at most 128 VGPRs.
constexpr int p24p_waves(int e, bool seq) { return e > 8 ? 1 : (seq ? 3 : 4); }

template <int N, int DT, int B, int TT, bool SEQ>
__global__ void __launch_bounds__((B * TT), p24p_waves(N / TT, SEQ))
p2p_fwd(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, TT, Real, -1, false>;
    using WI = W2Index<N, C::BS, true>;
    static_assert(B == C::BS, "the axis-1 tile is the W2 layout tile");
    constexpr int E = F::E;
    constexpr int tiles = N / B;
    constexpr int units = (N / 2) * tiles;  // per problem
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    cx<Real>* stw = sb + (SEQ ? 1 : 2) * B * N;
    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;
    const Prob<DT>& P = bt.p[ug / units];
    const Work<DT>& w1 = P.w1;
    const auto& w2 = P.w2;
    const cx<Real>* __restrict__ tw = P.tw;
    const int u = ug % units;
    const int pr = u / tiles, tile = u % tiles;
    const int c = threadIdx.x % B, t = threadIdx.x / B;
    const int k2 = tile * B + c;
    using W1I = W1Index<N, B>;

    cx<Real> xa[E], xb[E], w[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int pos = F::in_pos(t, e);
        xa[e] = w1.ld(W1I::at(2 * pr, pos, k2));
        xb[e] = w1.ld(W1I::at(2 * pr + 1, pos, k2));
        w[e] = tw[pos];
    }
    TwLds<Real> tl{stw};
    tl.fill(tw, N, threadIdx.x, B * TT);  // visible after the first exchange
    ChainLds<Real, SEQ> lds{sb, B, c};
    cx<Real> ra[2][E], d[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        ra[0][e] = xa[e];
        ra[1][e] = xa[e] * w[e];
    }
    F::template run<2>(ra, t, tl, lds);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        d[0][e] = xb[e];
        d[1][e] = xb[e] * w[e];
    }
    F::template run<2>(d, t, tl, lds);
    {
        // Stage in rounds of HALF slots: element (slot, column, i0 parity) at
        // ((slot - h HALF) B + c) 2 + parity, the order of the W2 runs.
        constexpr int KB = WI::KB, RUN = 2 * KB * B;
        constexpr int HALF = SEQ ? N / 2 : N;  // slots per round
        static_assert((2 * HALF * B) % RUN == 0, "rounds cover whole runs");
        const size_t tile0 = WI::at(2 * pr, 0, tile * B);  // start of block 0's run
#pragma unroll
        for (int h = 0; h < 2 * N / HALF; ++h) {
            __syncthreads();  // the last exchange's (or round's) reads are done
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int m = F::out_pos(t, e);
#pragma unroll
                for (int ch = 0; ch < 2; ++ch) {
                    const int sl = WI::slot(2 * m + ch) - h * HALF;
                    if (sl >= 0 && sl < HALF) {
                        sb[(sl * B + c) * 2] = ra[ch][e];
                        sb[(sl * B + c) * 2 + 1] = d[ch][e];
                    }
                }
            }
            __syncthreads();
            for (int g = 2 * int(threadIdx.x); g < 2 * HALF * B; g += 2 * B * TT) {
                const int gg = h * 2 * HALF * B + g;
                w2.st2(tile0 + size_t(gg / RUN) * WI::blk + gg % RUN, sb[g], sb[g + 1]);
            }
        }
    }
}

// Axis-0 pass on the paired layout.  One workgroup = SL rows of W2 (k1 and
// M-k1 when SL = 2) and B adjacent columns.  A line x (n samples along i0)
// is split by decimation in time: with w = exp(-2 pi i / 2n) and H = n/2,
//   A = DFT_H(x[2i]),  B = DFT_H(x[2i+1]),
//   C = DFT_H(x[2i] w^2i),  D = DFT_H(x[2i+1] w^(2i+1)),
// and the padded forward transform is X[2m] = A[m] + w^2m B[m],
// X[2m + 2H] = A[m] - w^2m B[m] (likewise X[2m+1], X[2m+1+2H] from C and D).
// After the multiply by K, the inverse that keeps the first n samples splits
// by decimation in frequency into four half-length inverses whose inputs are
// P = ks A + kd w^2m B and Q = ks B + kd w^-2m A (ks, kd = sum and difference
// of the kernel values of the two outputs) for the even outputs (likewise R,
// S for the odd ones); then u[2i] = P[i] + w^-2i R[i] and
// u[2i+1] = Q[i] + w^-(2i+1) S[i].  Each lane loads and stores the pair
// (x[2i], x[2i+1]) of its column as one access; all four chains advance in
// lockstep, G of them per LDS exchange round.  Column 0 is left to p3_col0.
// Per-stage twiddle rows for the half-length transforms of the paired middle
// pass (n >= 512, where the saved index arithmetic outweighs the fill).
template <int N>
struct P3PRows {
    static constexpr bool value = N >= 512;
};
template <int N, int DT, int TT>
constexpr size_t p3p_tw_entries() {
    using Real = typename Cfg<N, DT>::Real;
    using Ff = TeamFFT<N / 2, TT, Real, -1, false>;
    using Fi = TeamFFT<N / 2, TT, Real, +1, true>;
    if constexpr (P3PRows<N>::value) return Ff::rows_size() + (Ff::template same_rows<Fi>() ? 0 : Fi::rows_size());
    else return TwLds<Real>::slots(N);
}

template <int N, int DT, int B, int TT, int SL, int G>
__global__ void __launch_bounds__((B * TT * SL), (G < 4 && DT == DT_F32 ? 2 : 1))
p3p_conv(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    constexpr int H = N / 2;
    using Ff = TeamFFT<H, TT, Real, -1, false>;
    using Fi = TeamFFT<H, TT, Real, +1, true>;
    static_assert(SL == 1 || SL == 2, "one row or a row pair per workgroup");
    static_assert(G == 4 || G == 2, "four chains exchanged all at once or two at a time");
    constexpr int E = Ff::E;
    constexpr int tiles = N / B;
    constexpr int units = (2 / SL) * N * tiles;  // per problem
    using WI = W2Index<N, C::BS, true>;
    static_assert(C::BS % B == 0, "the axis-0 tile lies inside a W2 layout tile");
    constexpr size_t sp = WI::s0;  // stride of i0 pairs in W2
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    cx<Real>* stw = sb + size_t(G) * H * B * SL;

    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;  // whole workgroup
    const Prob<DT>& P = bt.p[ug / units];
    const auto& w2 = P.w2;
    const typename C::Kt* __restrict__ K = P.K;
    const cx<Real>* __restrict__ tw = P.tw;
    const int u = ug % units;
    int q, tile, set;
    if constexpr (SL == 1) {
        const int item = u >> 1;
        set = u & 1;
        q = item / tiles;
        tile = item % tiles;
    } else {
        q = u / tiles;
        tile = u % tiles;
        set = (threadIdx.x / B) & 1;
    }
    const int c = threadIdx.x % B, t = threadIdx.x / (B * SL);
    const int k2 = tile * B + c;
    static_assert(WI::s0 * H * sizeof(cx<double>) < (size_t(1) << 32) &&
                      size_t(N + 1) * (N + 1) * N * sizeof(double) < (size_t(1) << 32),
                  "lane byte offsets fit 32 bits");
    // pair i = in_pos(t, e) of row q (set 0) or M-q (set 1, 2 BS elements on)
    const size_t ub = WI::at(0, q, tile * B);
    const uint32_t xl = uint32_t(2 * c) + uint32_t(set) * (2 * C::BS) + uint32_t(t) * uint32_t(sp);
    auto xb = [&](int e) { return ub + size_t(Ff::in_pos(0, e)) * sp; };

    cx<Real> d[4][E];
#pragma unroll
    for (int e = 0; e < E; ++e) w2.ld_pair(xb(e), xl, d[0][e], d[1][e]);
    // kernel values of outputs 2m, 2m+1 (m = out_pos(t, e) = t + m0) and of
    // their partners n - 2m, n - 2m - 1: a uniform base plus one of two lane
    // offsets in the tiled K row (plane q, or n for the set-1 row of pair 0)
    constexpr int KT = psn_host::k_tile(N);
    using Kt = typename C::Kt;
    const uint32_t kl = uint32_t(psn_host::k_index(N, (set != 0 && q == 0) ? N : q, 0, k2));
    const uint32_t kup = (kl + uint32_t(2 * t * KT)) * uint32_t(sizeof(Kt));
    const uint32_t kdn = (kl + uint32_t(2 * (TT - 1 - t) * KT)) * uint32_t(sizeof(Kt));
    auto kv = [&](int e, int odd, int mirror) -> Real {
        const int m0 = Ff::out_pos(0, e);
        if (!mirror) return Real(gld(byte_off(sbase(K + (2 * m0 + odd) * KT), kup)));
        return Real(gld(byte_off(sbase(K + (N - 2 * m0 - odd - 2 * (TT - 1)) * KT), kdn)));
    };
    // Stage twiddles of the half-length transforms: per-stage rows for
    // n >= 512 (filled from every other entry of the 2n table), else the
    // swizzled 2n table read at even entries.
    constexpr bool kRows = P3PRows<N>::value;
    TwLds<Real> tl{stw};
    cx<Real>* rows_i = stw + (Ff::template same_rows<Fi>() ? 0 : Ff::rows_size());
    if constexpr (kRows) {
        Ff::template fill_rows<1, 2>(stw, tw, threadIdx.x, B * TT * SL);  // visible after the first exchange
        if constexpr (!Ff::template same_rows<Fi>()) Fi::template fill_rows<1, 2>(rows_i, tw, threadIdx.x, B * TT * SL);
    } else {
        tl.fill(tw, N, threadIdx.x, B * TT * SL);   // visible after the first exchange
        if constexpr (Ff::S == 1) __syncthreads();  // no exchange: the combine reads the table
    }
    // pre-twiddles w^2i, w^(2i+1) of the pair this lane holds
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = Ff::in_pos(t, e);
        d[2][e] = d[0][e] * gld(tw + 2 * i);
        d[3][e] = d[1][e] * gld(tw + 2 * i + 1);
    }
    using Lds = std::conditional_t<G == 4, LdsColsN<Real, 4>, LdsColsSeq<Real, 2>>;
    Lds lds{sb, B * SL, int(threadIdx.x % (B * SL))};
    if constexpr (G == 4) lds.plane = 2 * H * B * SL;
    TwHalf<Real> th{tl};
    if constexpr (kRows) Ff::template run<4>(d, t, TwRows<Real>{stw}, lds);
    else Ff::template run<4>(d, t, th, lds);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = Ff::out_pos(t, e);
        // w^2m = exp(-2 pi i m / n)
        const cx<Real> W = kRows ? gld(byte_off(sbase(tw + 2 * Ff::out_pos(0, e)), uint32_t(2 * t * C::CX)))
                                 : tl(2 * m);
#pragma unroll
        for (int odd = 0; odd < 2; ++odd) {
            const Real k0 = kv(e, odd, 0), k1 = kv(e, odd, 1);
            const Real ks = k0 + k1, kd = k0 - k1;
            const cx<Real> a = d[2 * odd][e], b = d[2 * odd + 1][e];
            // P = ks a + (kd W) b,  Q = ks b + conj(kd W) a
            const cx<Real> kw = scale(W, kd);
            d[2 * odd][e] = {fmad(ks, a.x, fmad(kw.x, b.x, -kw.y * b.y)), fmad(ks, a.y, fmad(kw.x, b.y, kw.y * b.x))};
            d[2 * odd + 1][e] = {fmad(ks, b.x, fmad(kw.x, a.x, kw.y * a.y)), fmad(ks, b.y, fmad(kw.x, a.y, -kw.y * a.x))};
        }
    }
    if constexpr (kRows) Fi::template run<4>(d, t, TwRows<Real>{rows_i}, lds);
    else Fi::template run<4>(d, t, th, lds);
    if (k2 != 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = Fi::out_pos(t, e);
            const cx<Real> u0 = twfma<+1>(d[2][e], gld(tw + 2 * i), d[0][e]);
            const cx<Real> u1 = twfma<+1>(d[3][e], gld(tw + 2 * i + 1), d[1][e]);
            w2.st_pair(xb(e), xl, u0, u1);
        }
    }
}

// Axis-1 inverse over an i0 pair: unit = (i0 pair, tile of B columns k2).
// Each lane loads rows 2j and 2j+1 of its column as (i0 = 2p, 2p + 1) pairs;
// the two lines are inverted one after the other and combined as
// y = y_even + w^-j y_odd.
template <int N, int DT, int B, int TT, bool SEQ>
__global__ void __launch_bounds__((B * TT), p24p_waves(N / TT, SEQ))
p4p_inv(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using F = TeamFFT<N, TT, Real, +1, false>;
    using WI = W2Index<N, C::BS, true>;
    static_assert(B == C::BS, "the axis-1 tile is the W2 layout tile");
    constexpr int E = F::E;
    constexpr int tiles = N / B;
    constexpr int units = (N / 2) * tiles;  // per problem
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    cx<Real>* stw = sb + (SEQ ? 1 : 2) * B * N;
    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;
    const Prob<DT>& P = bt.p[ug / units];
    const Work<DT>& w1 = P.w1;
    const auto& w2 = P.w2;
    const cx<Real>* __restrict__ tw = P.tw;
    const int u = ug % units;
    const int pr = u / tiles, tile = u % tiles;
    const int c = threadIdx.x % B, t = threadIdx.x / B;
    const int k2 = tile * B + c;
    using W1I = W1Index<N, B>;

    cx<Real> a[2][E], b[2][E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int pos = F::in_pos(t, e);
        w2.ld_pair(WI::at(2 * pr, 2 * pos, k2), a[0][e], b[0][e]);
        w2.ld_pair(WI::at(2 * pr, 2 * pos + 1, k2), a[1][e], b[1][e]);
    }
    TwLds<Real> tl{stw};
    tl.fill(tw, N, threadIdx.x, B * TT);  // visible after the first exchange
    if constexpr (F::S == 1) __syncthreads();  // no exchange: the combine reads the table
    ChainLds<Real, SEQ> lds{sb, B, c};
    // the combine twiddles w^-j come from the LDS table (fewer live registers)
    F::template run<2>(a, t, tl, lds);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = F::out_pos(t, e);
        w1.st(W1I::at(2 * pr, j, k2), twfma<+1>(a[1][e], tl(j), a[0][e]));
    }
    F::template run<2>(b, t, tl, lds);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int j = F::out_pos(t, e);
        w1.st(W1I::at(2 * pr + 1, j, k2), twfma<+1>(b[1][e], tl(j), b[0][e]));
    }
}

// ------------------------------------------------------------------ P5
template <int N, int DT>
__global__ void __launch_bounds__((Cfg<N, DT>::LC * Cfg<N, DT>::T))
p5_c2r(const Batch<DT> bt) {
    using C = Cfg<N, DT>;
    using Real = typename C::Real;
    using Io = typename C::Io;
    using F = TeamFFT<N, C::T, Real, +1, false>;
    constexpr int units = N * N / C::LC;  // per problem
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const int ug = xcd_unit();
    if (ug >= bt.count * units) return;
    const Prob<DT>& P = bt.p[ug / units];
    const Work<DT>& w1 = P.w1;
    Io* __restrict__ u = P.u;
    const cx<Real>* __restrict__ tw = P.tw;
    const int t = threadIdx.x % C::T, ln = threadIdx.x / C::T;
    const int line0 = (ug % units) * C::LC;  // first line of the workgroup; all share i0
    const int i0 = line0 / N, i1b = line0 % N;
    const size_t base = (size_t(line0) + ln) * N;  // of this thread's line in u

    // Y[k] = (V[k] + conj V[n-k]) + i (V[k] - conj V[n-k]) w^-k; V[0], V[n] real and packed.
    // The workgroup's LC lines of W1 are read with consecutive threads on
    // consecutive addresses (element j is line j / BS % LC, k = j / (BS * LC) * BS
    // + j % BS) into the LDS rows; each line's team then takes V[k] and its
    // partner V[n-k] from there (the first exchange of the transform waits
    // before reusing the rows).
    constexpr int BL = C::BS;
    using W1I = W1Index<N, BL>;
    TwLds<Real> tl{sb + C::LC * C::NP};
    tl.fill(tw, N, threadIdx.x, C::LC * C::T);
    using TO = TileOrder<N, C::LC, C::T, BL>;
    cx<Real> d[F::E];
#pragma unroll
    for (int q = 0; q < F::E; ++q) {
        int lj, k0, off;
        TO::at(int(threadIdx.x), q, lj, k0, off);
        d[q] = w1.ld(W1I::at(i0, i1b + lj, k0 + off));
    }
#pragma unroll
    for (int q = 0; q < F::E; ++q) {
        int lj, k0, off;
        TO::at(int(threadIdx.x), q, lj, k0, off);
        LdsRows<Real>{sb + lj * C::NP}.put2(k0, off, d[q]);
    }
    __syncthreads();
    LdsRows<Real> lds{sb + ln * C::NP};
#pragma unroll
    for (int e = 0; e < F::E; ++e) {
        const int pos = F::in_pos(t, e);
        const int pc = pos - t;  // compile-time part of the position
        const cx<Real> a = lds.get2(t, pc);
        if (pos == 0) {
            d[e] = {a.x + a.y, a.x - a.y};
        } else {
            const cx<Real> b = conj(lds.get2(N - t, -pc));
            d[e] = (a + b) + rot<+1>(mul_conj(a - b, tl(pos)));
        }
    }
    F::run1(d, t, tl, lds);
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

// ------------------------------------------------------------------ Fourier-series correction
// The near-zone correction by the paper's own route (section 2: derivatives
// from the finite Fourier series of the density, one forward and one
// backward FFT of size N = n^3, section 3): z = C0 rho + (C2/6) Laplace_N(rho),
// with the Laplacian's symbol -sum_q kappa_q^2, kappa_q = 2 pi k / (n h_q) at
// the signed index k (period n h_q, the samples' own grid).  It runs after
// the axis-1 inverse, while rho is intact (also in place) and W2 is free: z
// lives in W2's memory, as n^3 complex values in C order.  Five line passes,
// each one read and one write of the volume: axis 2 forward reading rho
// itself; axis 1 forward; axis 0 forward, times the symbol
// (C0 - (C2/6) |kappa|^2) / n^3, inverse (one pass, radices reversed as in
// the middle pass of the solve); axis 1 inverse; and, after the solve's
// axis-2 pass, axis 2 inverse adding Re z to u.
template <int DT>
struct CorrProb {
    const typename Prec<DT>::Io* rho;
    typename Prec<DT>::Io* u;
    cx<typename Prec<DT>::Real>* z;
    const cx<typename Prec<DT>::Real>* tw;
    double c0, c2;   // C0 and C2 / 6
    double kq[3];    // 2 pi / (n h_q)
};
template <int DT>
struct CorrBatch {
    int count;
    CorrProb<DT> p[kMaxBatch];
};

// Length-N transforms of the real density along each axis (DIR = -1
// forward, +1 inverse, unnormalised), on its half spectrum z[i0][i1][k2],
// k2 = 0..N/2, rows padded to HZ.  Axis 2: a workgroup holds LC contiguous
// lines, one LDS row each; the forward reads a row of rho as N/2 complex
// pairs, transforms them at length N/2 and unpacks the N/2 + 1 outputs (as
// P1), the inverse packs them back and adds the row to u (as P5).  Axes 0
// and 1: a workgroup holds B adjacent lines (consecutive k2), element-major
// in LDS, so each point's B values are one contiguous run; on axis 0 the
// forward is followed in registers by the symbol and the inverse (DIR is
// ignored there).
template <int N, int DT>
struct CorrCfg {
    using Real = typename Prec<DT>::Real;
    static constexpr int CX = sizeof(cx<Real>);
    // axis 2: packed transforms of length N/2
    static constexpr int E = elems_per_thread(N / 2, sizeof(Real));
    static constexpr int T = N / 2 / E;
    static constexpr int LC = pick_lines(N / 2, T, CX, 256, kMaxLds);  // axis-2 lines
    static constexpr int NP = rows_padded(N / 2);
    // axes 0 and 1: at most 8 elements per thread (FP32 otherwise takes 16),
    // so that the three workgroups that fit a CU's LDS hold twice the waves
    static constexpr int T01 = N / elems_per_thread(N, 8);
    static constexpr int B = (N % 8 == 0 && (8 * N + TwLds<Real>::slots(N)) * CX <= 65536 && 8 * T01 <= 1024) ? 8
                             : (N % 4 == 0 && (4 * N + TwLds<Real>::slots(N)) * CX <= 65536) ? 4
                                                                                              : 1;
    static constexpr int HZ = (N / 2 + B) / B * B;  // N/2 + 1 rounded up to B
};

template <int N, int DT, int AX, int DIR>
__global__ void corr_fft(const CorrBatch<DT> cb) {
    using CC = CorrCfg<N, DT>;
    using Real = typename CC::Real;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<Real>* sb = reinterpret_cast<cx<Real>*>(smem);
    const CorrProb<DT>& P = cb.p[blockIdx.y];
    cx<Real>* __restrict__ z = P.z;
    if constexpr (AX == 2) {
        // packed length FL = N/2: z_j = x_2j + i x_2j+1, Z = DFT_FL(z),
        // X[k] = (Z[k] + conj Z[FL-k])/2 + w^k (Z[k] - conj Z[FL-k])/(2i),
        // w = exp(-2 pi i / N), X[0] and X[FL] from Z[0]; the inverse packs
        // Y[k] = (X[k] + conj X[FL-k]) + i w^-k (X[k] - conj X[FL-k]) and
        // IDFT_FL(Y)_j = u_2j + i u_2j+1
        constexpr int FL = N / 2;
        using F = TeamFFT<FL, CC::T, Real, DIR, false>;
        cx<Real> d[F::E];
        using Io = typename Prec<DT>::Io;
        const int t = threadIdx.x % CC::T, ln = threadIdx.x / CC::T;
        const size_t line = size_t(blockIdx.x) * CC::LC + ln;
        const size_t base = line * N;  // of rho and u
        cx<Real>* const zr = z + line * CC::HZ;
        // the length-FL table exp(-2 pi i m / N), m < N: every other entry of
        // the plan's length-2N table
        TwLds<Real> tl{sb + CC::LC * CC::NP};
        for (int i = threadIdx.x; i < N; i += CC::LC * CC::T) tl.p[TwLds<Real>::at(i)] = P.tw[2 * i];
        __syncthreads();
        LdsRows<Real> lds{sb + ln * CC::NP};
        if constexpr (DIR < 0) {
#pragma unroll
            for (int e = 0; e < F::E; ++e) {
                const int j = F::in_pos(t, e);
                d[e] = {Real(P.rho[base + 2 * j]), Real(P.rho[base + 2 * j + 1])};
            }
            F::run1(d, t, tl, lds);
            __syncthreads();  // the transform's last exchange reads are done
#pragma unroll
            for (int e = 0; e < F::E; ++e) lds.put(F::out_pos(t, e), d[e]);
            __syncthreads();
#pragma unroll
            for (int e = 0; e < F::E; ++e) {
                const int k = F::out_pos(t, e);
                const cx<Real> Z = lds.get(k);
                if (k == 0) {
                    gst(zr, cx<Real>{Z.x + Z.y, Real(0)});
                    gst(zr + FL, cx<Real>{Z.x - Z.y, Real(0)});
                } else {
                    const cx<Real> Zr = conj(lds.get(FL - k));
                    const cx<Real> Ev = scale(Z + Zr, Real(0.5));
                    const cx<Real> Od = rot<-1>(scale(Z - Zr, Real(0.5)));
                    gst(zr + k, Ev + Od * tl(k));
                }
            }
        } else {
            // each X[k] loaded once into the line's row (X[FL] by its first
            // thread); the partner X[FL-k] read back from there
#pragma unroll
            for (int e = 0; e < F::E; ++e) d[e] = gld(zr + F::in_pos(t, e));
            const cx<Real> last = t == 0 ? gld(zr + FL) : cx<Real>{Real(0), Real(0)};
#pragma unroll
            for (int e = 0; e < F::E; ++e) lds.put(F::in_pos(t, e), d[e]);
            if (t == 0) lds.put(FL, last);
            __syncthreads();
#pragma unroll
            for (int e = 0; e < F::E; ++e) {
                const int k = F::in_pos(t, e);
                const cx<Real> p = d[e], q = conj(lds.get(FL - k));
                d[e] = (p + q) + rot<+1>(mul_conj(p - q, tl(k)));
            }
            F::run1(d, t, tl, lds);  // its first exchange waits before reusing the row
#pragma unroll
            for (int e = 0; e < F::E; ++e) {
                const int j = F::out_pos(t, e);
                Io* __restrict__ u = P.u + base + 2 * j;
                u[0] = Io(u[0] + Io(d[e].x));
                u[1] = Io(u[1] + Io(d[e].y));
            }
        }
    } else {
        constexpr int B = CC::B, TT = CC::T01;
        using F = TeamFFT<N, TT, Real, DIR, false>;
        cx<Real> d[F::E];
        // units (line, tile of B columns k2), tiles fastest, dealt XCD-aware
        // so that neighbouring tiles (which share 128-byte lines) meet in one
        // L2; columns past k2 = N/2 transform the row padding
        constexpr int HZ = CC::HZ;
        constexpr int units = N * (HZ / B);
        const int u = xcd_unit();
        if (u >= units) return;  // whole workgroup
        const int c = threadIdx.x % B, t = threadIdx.x / B;
        const int line = u / (HZ / B), i2 = (u % (HZ / B)) * B + c;
        // axis 1: (i0 = line, pos, k2 = i2); axis 0: (pos, i1 = line, k2 = i2)
        const size_t stride = AX == 1 ? size_t(HZ) : size_t(N) * HZ;
        const size_t base = (AX == 1 ? size_t(line) * N * HZ : size_t(line) * HZ) + i2;
        TwLds<Real> tl{sb + B * N};
        tl.fill(P.tw, N, threadIdx.x, B * TT);
        __syncthreads();
#pragma unroll
        for (int e = 0; e < F::E; ++e) d[e] = gld(z + base + size_t(F::in_pos(t, e)) * stride);
        LdsCols<Real> lds{sb, B, c};
        F::run1(d, t, tl, lds);
        if constexpr (AX == 0) {
            // z *= (C0 - (C2/6) |kappa|^2) / n^3 at (k0, k1 = line, k2 = i2), then the
            // inverse with the radices reversed, which starts from this layout
            using Fi = TeamFFT<N, TT, Real, +1, true>;
            auto kap2 = [](double kq, int k) {
                const double v = kq * double(k <= N / 2 ? k : k - N);
                return v * v;
            };
            const double q12 = kap2(P.kq[1], line) + kap2(P.kq[2], i2);
            const double inv = 1.0 / (double(N) * N * N);
#pragma unroll
            for (int e = 0; e < F::E; ++e) {
                const double q = q12 + kap2(P.kq[0], F::out_pos(t, e));
                d[e] = scale(d[e], Real((P.c0 - P.c2 * q) * inv));
            }
            __syncthreads();  // the forward's last exchange reads are done
            Fi::run1(d, t, tl, lds);
#pragma unroll
            for (int e = 0; e < F::E; ++e) gst(z + base + size_t(Fi::out_pos(t, e)) * stride, d[e]);
        } else {
#pragma unroll
            for (int e = 0; e < F::E; ++e) gst(z + base + size_t(F::out_pos(t, e)) * stride, d[e]);
        }
    }
}

// ------------------------------------------------------------------ launcher
// Kernels needing more than 64 KB of dynamic LDS must say so once.
inline bool allow_lds(const void* fn, size_t bytes) {
    if (bytes <= 65536) return true;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) == hipSuccess;
}

// The correction's passes before the solve's axis-2 pass (z after the
// axis-1 inverse) and the one after it (axis-2 inverse added to u).
template <int N, int DT>
hipError_t launch_corr_z(const CorrBatch<DT>& cb, hipStream_t s) {
    using CC = CorrCfg<N, DT>;
    const size_t lds2 = (size_t(CC::LC) * CC::NP + TwLds<typename CC::Real>::slots(N / 2)) * CC::CX;
    const size_t lds01 = (size_t(CC::B) * N + TwLds<typename CC::Real>::slots(N)) * CC::CX;
    const dim3 g2(N * N / CC::LC, cb.count), g01(xcd_grid(N * (CC::HZ / CC::B)), cb.count);
    const dim3 b2(CC::LC * CC::T), b01(CC::B * CC::T01);
    hipLaunchKernelGGL((corr_fft<N, DT, 2, -1>), g2, b2, lds2, s, cb);
    hipLaunchKernelGGL((corr_fft<N, DT, 1, -1>), g01, b01, lds01, s, cb);
    hipLaunchKernelGGL((corr_fft<N, DT, 0, -1>), g01, b01, lds01, s, cb);
    hipLaunchKernelGGL((corr_fft<N, DT, 1, +1>), g01, b01, lds01, s, cb);
    return hipGetLastError();
}
template <int N, int DT>
hipError_t launch_corr_add(const CorrBatch<DT>& cb, hipStream_t s) {
    using CC = CorrCfg<N, DT>;
    const size_t lds2 = (size_t(CC::LC) * CC::NP + TwLds<typename CC::Real>::slots(N / 2)) * CC::CX;
    hipLaunchKernelGGL((corr_fft<N, DT, 2, +1>), dim3(N * N / CC::LC, cb.count), dim3(CC::LC * CC::T), lds2, s, cb);
    return hipGetLastError();
}

// ------------------------------------------------------------------ schedules
// Tile shapes of the strided passes: B adjacent columns per workgroup, TT
// threads per line.  Each pass has three compiled candidates; the autotuner
// times them once per (n, precision) and keeps the fastest.  A candidate that
// does not fit (LDS, threads, radix plan) is replaced by candidate 0.
struct TileV {
    int B, TT;
    int SL = 1;        // rows per workgroup (the axis-0 pass only)
    bool SEQ = false;  // exchange the two chains one at a time (half the LDS)
};

constexpr bool tile_ok(int N, TileV v, int cxbytes) {
    return v.B >= 1 && v.TT >= 1 && (v.SL == 1 || v.SL == 2) && N % v.B == 0 && N % v.TT == 0 &&
           v.B * v.TT * v.SL <= 1024 &&
           ((v.SEQ ? 1 : 2) * v.B * v.SL * N + ((2 * N + 15) & ~15)) * cxbytes <= kMaxLdsP3 &&
           make_plan(N, N / v.TT).n > 0 && N / v.TT <= 20;
}

constexpr TileV pick_tile(int N, TileV v, TileV dflt, int cxbytes) { return tile_ok(N, v, cxbytes) ? v : dflt; }
constexpr TileV pick_tile3(int N, TileV v, TileV dflt, int cxbytes, int layout_tile) {
    return (tile_ok(N, v, cxbytes) && layout_tile % v.B == 0) ? v : dflt;
}

template <int N, int DT>
struct Sched {
    using C = Cfg<N, DT>;
    static constexpr int e8 = elems_per_thread(N, 8), e16 = elems_per_thread(N, 4);
    static constexpr TileV d24{C::BS, C::T24}, d3{C::BP3, C::T3};
    // P2/P4 keep the W2 layout tile (B = BS); P3 tiles must divide it
    // Sizes with a factor 3 or 5 keep all odd factors in every thread, so their
    // teams are small (8 threads for a 160-point line); their second candidate
    // halves the elements per thread instead (twice the threads per line, a
    // longer radix plan).
    static constexpr int odd = N / (N & -N);
    static constexpr int eh = odd * 2;
    // (the one-chain exchange stages the W2 runs in two rounds of n slots,
    // which needs the k1 block to divide n)
    // The fourth candidate: sizes with an odd factor halve the elements per
    // thread and exchange one chain at a time; powers of two take 4 elements
    // per thread (twice the threads, one more exchange).
    static constexpr bool seq_ok = N % psn_host::w2_k1_block(N) == 0;
    static constexpr TileV v24[psn_host::kScheduleCandidates] = {
        d24, pick_tile(N, odd > 1 ? TileV{C::BS, N / eh} : TileV{C::BS, N / e16}, d24, C::CX),
        seq_ok ? pick_tile(N, {C::BS, C::T24, 1, true}, d24, C::CX) : d24,
        odd > 1 ? (seq_ok ? pick_tile(N, TileV{C::BS, N / eh, 1, true}, d24, C::CX) : d24)
                : pick_tile(N, TileV{C::BS, N / 4}, d24, C::CX)};
    // P3: one row per workgroup; the row pair k1, M-k1 per workgroup (sizes with
    // an odd factor: with the chains exchanged one at a time); one row with
    // the chains exchanged one at a time; and (odd factor) half the elements
    // per thread, or (powers of two) 4 elements per thread with the one-chain
    // exchange.  (The whole layout tile of 8 columns with the one-chain
    // exchange fits one 512-thread FP64-arithmetic workgroup per CU and
    // measured 30 % slower at n = 512.)
    static constexpr TileV v3[psn_host::kScheduleCandidates] = {
        d3,
        pick_tile3(N, odd > 1 ? TileV{C::BP3, C::T3, 2, true} : TileV{C::BP3, C::T3, 2}, d3, C::CX, C::BS),
        pick_tile3(N, {C::BP3, C::T3, 1, true}, d3, C::CX, C::BS),
        pick_tile3(N, odd > 1 ? TileV{C::BP3, N / eh} : TileV{C::BP3, N / 4, 1, true}, d3, C::CX, C::BS)};
    static_assert(tile_ok(N, d24, C::CX) && tile_ok(N, d3, C::CX), "default tiles must fit");
};

// Axis-0 tiles on the paired layout: B columns, TT threads per half line
// (n/2 points), SL rows per workgroup, G chains per LDS exchange round.
struct TileP {
    int B, TT;
    int SL = 1;
    int G = 4;
};

constexpr bool tilep_ok(int N, TileP v, int cxbytes) {
    return v.B >= 1 && v.TT >= 1 && (v.SL == 1 || v.SL == 2) && (v.G == 2 || v.G == 4) && N % v.B == 0 &&
           (N / 2) % v.TT == 0 && v.B * v.TT * v.SL <= 1024 &&
           (size_t(v.G) * (N / 2) * v.B * v.SL + ((2 * N + 15) & ~15)) * cxbytes <= size_t(kMaxLdsP3) &&
           make_plan(N / 2, N / 2 / v.TT).n > 0 && N / 2 / v.TT <= 16;
}
constexpr TileP pick_tilep(int N, TileP v, TileP dflt, int cxbytes, int layout_tile) {
    return (tilep_ok(N, v, cxbytes) && layout_tile % v.B == 0) ? v : dflt;
}

template <int N, int DT>
struct SchedP {
    using C = Cfg<N, DT>;
    static constexpr int H = N / 2;
    static constexpr int e8 = H >= 8 ? 8 : H;
    static constexpr int e4 = H >= 4 ? 4 : H;
    // eight points per chain and thread, two chains per exchange round (all
    // four at once halves the workgroups per CU and measured 45 % slower at
    // n = 512); the row pair k1, M-k1 per workgroup; four points per chain
    // (twice the threads, one more exchange); sixteen points per chain (one
    // exchange fewer, half the threads)
    static constexpr int e16 = H >= 16 ? 16 : H;
    static constexpr TileP d3{C::BP3, H / e8, 1, 2};
    static constexpr TileP v3[psn_host::kScheduleCandidates] = {
        d3, pick_tilep(N, TileP{C::BP3, H / e8, 2, 2}, d3, C::CX, C::BS),
        pick_tilep(N, TileP{C::BP3, H / e4, 1, 2}, d3, C::CX, C::BS),
        pick_tilep(N, TileP{C::BP3, H / e16, 1, 2}, d3, C::CX, C::BS)};
};

// LDS of the strided passes: the exchange area plus the stage twiddle rows
template <int N, int DT, int B, int TT, bool SEQ>
constexpr size_t lds_p24() {
    return (size_t(SEQ ? 1 : 2) * B * N + TwLds<typename Cfg<N, DT>::Real>::slots(N)) * Cfg<N, DT>::CX;
}
template <int N, int DT, int B, int TT, int SL, bool SEQ>
constexpr size_t lds_p3() {
    using Real = typename Cfg<N, DT>::Real;
    using Ff = TeamFFT<N, TT, Real, -1, false>;
    using Fi = TeamFFT<N, TT, Real, +1, true>;
    const size_t rows = P3Rows<N>::value ? Ff::rows_size() + (Ff::template same_rows<Fi>() ? 0 : Fi::rows_size())
                                         : TwLds<Real>::slots(N);
    return (size_t(SEQ ? 1 : 2) * B * SL * N + rows) * Cfg<N, DT>::CX;
}

template <int N, int DT, int I>
hipError_t launch_p2(const Batch<DT>& bt, hipStream_t s) {
    constexpr TileV v = Sched<N, DT>::v24[I];
    const size_t lds = lds_p24<N, DT, v.B, v.TT, v.SEQ>();
    static const bool ok = allow_lds(reinterpret_cast<const void*>(&p2_fwd<N, DT, v.B, v.TT, v.SEQ>), lds);
    if (!ok) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((p2_fwd<N, DT, v.B, v.TT, v.SEQ>), dim3(xcd_grid(long(bt.count) * N * (N / v.B))), dim3(v.B * v.TT),
                       lds, s, bt);
    return hipSuccess;
}

template <int N, int DT, int I>
hipError_t launch_p4(const Batch<DT>& bt, hipStream_t s) {
    constexpr TileV v = Sched<N, DT>::v24[I];
    const size_t lds = lds_p24<N, DT, v.B, v.TT, v.SEQ>();
    static const bool ok = allow_lds(reinterpret_cast<const void*>(&p4_inv<N, DT, v.B, v.TT, v.SEQ>), lds);
    if (!ok) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((p4_inv<N, DT, v.B, v.TT, v.SEQ>), dim3(xcd_grid(long(bt.count) * N * (N / v.B))), dim3(v.B * v.TT),
                       lds, s, bt);
    return hipSuccess;
}

template <int N, int DT, int I>
hipError_t launch_p3(const Batch<DT>& bt, hipStream_t s) {
    constexpr TileV v = Sched<N, DT>::v3[I];
    const size_t lds = lds_p3<N, DT, v.B, v.TT, v.SL, v.SEQ>();
    static const bool ok = allow_lds(reinterpret_cast<const void*>(&p3_conv<N, DT, v.B, v.TT, v.SL, v.SEQ>), lds);
    if (!ok) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((p3_conv<N, DT, v.B, v.TT, v.SL, v.SEQ>),
                       dim3(xcd_grid(long(bt.count) * (2 / v.SL) * N * (N / v.B))), dim3(v.B * v.TT * v.SL), lds, s,
                       bt);
    return hipSuccess;
}

// the axis-1 passes on the paired layout: the same tiles, one i0 pair per workgroup
template <int N, int DT, int I>
hipError_t launch_p2p(const Batch<DT>& bt, hipStream_t s) {
    constexpr TileV v = Sched<N, DT>::v24[I];
    const size_t lds = lds_p24<N, DT, v.B, v.TT, v.SEQ>();
    static const bool ok = allow_lds(reinterpret_cast<const void*>(&p2p_fwd<N, DT, v.B, v.TT, v.SEQ>), lds);
    if (!ok) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((p2p_fwd<N, DT, v.B, v.TT, v.SEQ>), dim3(xcd_grid(long(bt.count) * (N / 2) * (N / v.B))),
                       dim3(v.B * v.TT), lds, s, bt);
    return hipSuccess;
}

template <int N, int DT, int I>
hipError_t launch_p4p(const Batch<DT>& bt, hipStream_t s) {
    constexpr TileV v = Sched<N, DT>::v24[I];
    const size_t lds = lds_p24<N, DT, v.B, v.TT, v.SEQ>();
    static const bool ok = allow_lds(reinterpret_cast<const void*>(&p4p_inv<N, DT, v.B, v.TT, v.SEQ>), lds);
    if (!ok) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((p4p_inv<N, DT, v.B, v.TT, v.SEQ>), dim3(xcd_grid(long(bt.count) * (N / 2) * (N / v.B))),
                       dim3(v.B * v.TT), lds, s, bt);
    return hipSuccess;
}

template <int N, int DT, int I>
hipError_t launch_p3p(const Batch<DT>& bt, hipStream_t s) {
    constexpr TileP v = SchedP<N, DT>::v3[I];
    static_assert(tilep_ok(N, v, Cfg<N, DT>::CX), "paired axis-0 tile must fit");
    const size_t lds = (size_t(v.G) * (N / 2) * v.B * v.SL + p3p_tw_entries<N, DT, v.TT>()) * Cfg<N, DT>::CX;
    static const bool ok =
        allow_lds(reinterpret_cast<const void*>(&p3p_conv<N, DT, v.B, v.TT, v.SL, v.G>), lds);
    if (!ok) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((p3p_conv<N, DT, v.B, v.TT, v.SL, v.G>),
                       dim3(xcd_grid(long(bt.count) * (2 / v.SL) * N * (N / v.B))), dim3(v.B * v.TT * v.SL), lds,
                       s, bt);
    return hipSuccess;
}

template <int N, int DT>
hipError_t launch_p24(const Batch<DT>& bt, hipStream_t s, int v, bool forward) {
    if constexpr (PairW2<N, DT>::value) {
        switch (v) {
            case 1: return forward ? launch_p2p<N, DT, 1>(bt, s) : launch_p4p<N, DT, 1>(bt, s);
            case 2: return forward ? launch_p2p<N, DT, 2>(bt, s) : launch_p4p<N, DT, 2>(bt, s);
            case 3: return forward ? launch_p2p<N, DT, 3>(bt, s) : launch_p4p<N, DT, 3>(bt, s);
            default: return forward ? launch_p2p<N, DT, 0>(bt, s) : launch_p4p<N, DT, 0>(bt, s);
        }
    } else {
        switch (v) {
            case 1: return forward ? launch_p2<N, DT, 1>(bt, s) : launch_p4<N, DT, 1>(bt, s);
            case 2: return forward ? launch_p2<N, DT, 2>(bt, s) : launch_p4<N, DT, 2>(bt, s);
            case 3: return forward ? launch_p2<N, DT, 3>(bt, s) : launch_p4<N, DT, 3>(bt, s);
            default: return forward ? launch_p2<N, DT, 0>(bt, s) : launch_p4<N, DT, 0>(bt, s);
        }
    }
}

template <int N, int DT>
hipError_t launch_p3v(const Batch<DT>& bt, hipStream_t s, int v) {
    if constexpr (PairW2<N, DT>::value) {
        switch (v) {
            case 1: return launch_p3p<N, DT, 1>(bt, s);
            case 2: return launch_p3p<N, DT, 2>(bt, s);
            case 3: return launch_p3p<N, DT, 3>(bt, s);
            default: return launch_p3p<N, DT, 0>(bt, s);
        }
    } else {
        switch (v) {
            case 1: return launch_p3<N, DT, 1>(bt, s);
            case 2: return launch_p3<N, DT, 2>(bt, s);
            case 3: return launch_p3<N, DT, 3>(bt, s);
            default: return launch_p3<N, DT, 0>(bt, s);
        }
    }
}

// Enqueue the six kernels of one solve for bt.count problems of size N with
// schedule (v24 for P2/P4, v3 for P3).
// With cb (the entries whose plan adds the correction by its Fourier series),
// z is formed after the axis-1 inverse and added after the axis-2 pass
// (both counted in the last pass's event interval).
template <int N, int DT>
hipError_t solve_n(const Batch<DT>& bt, hipStream_t s, hipEvent_t* ev, int v24, int v3,
                   const CorrBatch<DT>* cb = nullptr) {
    using C = Cfg<N, DT>;
    constexpr size_t tws = TwLds<typename C::Real>::slots(N);
    const size_t lds_rows = (size_t(C::LC) * C::NP + tws) * C::CX;
    const long cnt = bt.count;
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    };
    static const bool lds_ok = allow_lds(reinterpret_cast<const void*>(&p1_r2c<N, DT>), lds_rows) &&
                               allow_lds(reinterpret_cast<const void*>(&p5_c2r<N, DT>), lds_rows);
    if (!lds_ok) return hipErrorInvalidValue;
    hipError_t e;
    mark(0);
    hipLaunchKernelGGL((p1_r2c<N, DT>), dim3(xcd_grid(cnt * N * N / C::LC)), dim3(C::LC * C::T), lds_rows, s, bt);
    mark(1);
    if ((e = launch_p24<N, DT>(bt, s, v24, true)) != hipSuccess) return e;
    mark(2);
    if ((e = launch_p3v<N, DT>(bt, s, v3)) != hipSuccess) return e;
    using G0 = Col0<N, DT>;
    hipLaunchKernelGGL((p3_col0<N, DT>), dim3(cnt * G0::groups), dim3(2 * G0::T * G0::G), G0::lds, s, bt);
    mark(3);
    if ((e = launch_p24<N, DT>(bt, s, v24, false)) != hipSuccess) return e;
    mark(4);
    if (cb && (e = launch_corr_z<N, DT>(*cb, s)) != hipSuccess) return e;
    hipLaunchKernelGGL((p5_c2r<N, DT>), dim3(xcd_grid(cnt * N * N / C::LC)), dim3(C::LC * C::T), lds_rows, s, bt);
    if (cb && (e = launch_corr_add<N, DT>(*cb, s)) != hipSuccess) return e;
    mark(5);
    return hipGetLastError();
}

// Time the candidates of the strided passes on one problem's workspace
// (contents are irrelevant to the timing) and return the fastest indices.
template <int N, int DT>
hipError_t tune_n(const Batch<DT>& bt, hipStream_t s, int* best24, int* best3) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // one timed launch sequence
    auto timed = [&](auto&& launch, float* ms) -> hipError_t {
        hipError_t le = hipEventRecord(a, s);
        if (le == hipSuccess) le = launch();
        if (le == hipSuccess) le = hipEventRecord(b, s);
        if (le == hipSuccess) le = hipEventSynchronize(b);
        if (le == hipSuccess) le = hipEventElapsedTime(ms, a, b);
        return le;
    };
    // Candidates are timed in interleaved rounds (so clock changes hit all of
    // them alike); each keeps its best time; round 0 only warms up.
    constexpr int NC = psn_host::kScheduleCandidates;
    float t24[NC], t3[NC];
    for (int v = 0; v < NC; ++v) t24[v] = t3[v] = 1e30f;
    for (int round = 0; round < 7 && e == hipSuccess; ++round) {
        for (int v = 0; v < NC && e == hipSuccess; ++v) {
            float x = 0.f, y = 0.f;
            e = timed([&] {
                    hipError_t r = launch_p24<N, DT>(bt, s, v, true);
                    return r == hipSuccess ? launch_p24<N, DT>(bt, s, v, false) : r;
                }, &x);
            if (e == hipSuccess) e = timed([&] { return launch_p3v<N, DT>(bt, s, v); }, &y);
            if (e == hipSuccess && round > 0) {
                t24[v] = x < t24[v] ? x : t24[v];
                t3[v] = y < t3[v] ? y : t3[v];
            }
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return e;
    *best24 = 0;
    *best3 = 0;
    for (int v = 1; v < NC; ++v) {
        if (t24[v] < 0.97f * t24[*best24]) *best24 = v;
        if (t3[v] < 0.97f * t3[*best3]) *best3 = v;
    }
    return hipSuccess;
}

template <int DT>
Prob<DT> prob_of(const psn_host::Slot& sl) {
    using Real = typename Prec<DT>::Real;
    using Io = typename Prec<DT>::Io;
    using Kt = typename Prec<DT>::Kt;
    Prob<DT> pr{};
    pr.rho = static_cast<const Io*>(sl.rho);
    pr.u = static_cast<Io*>(sl.u);
    if constexpr (DT == DT_SPLIT) {
        pr.w1 = {static_cast<uint32_t*>(sl.W1)};
        pr.w2 = {static_cast<cx<double>*>(sl.W2)};
    } else {
        pr.w1 = {static_cast<cx<Real>*>(sl.W1)};
        pr.w2 = {static_cast<cx<Real>*>(sl.W2)};
    }
    pr.K = static_cast<const Kt*>(sl.plan->K);
    pr.Kb = static_cast<const Kt*>(sl.plan->Kb);
    pr.tw = static_cast<const cx<Real>*>(sl.plan->tw);
    return pr;
}

template <int DT>
CorrProb<DT> corr_of(const psn_host::Slot& sl) {
    using Real = typename Prec<DT>::Real;
    using Io = typename Prec<DT>::Io;
    const psn_plan* p = sl.plan;
    CorrProb<DT> c{};
    c.rho = static_cast<const Io*>(sl.rho);
    c.u = static_cast<Io*>(sl.u);
    c.z = static_cast<cx<Real>*>(sl.W2);  // free between the axis-1 inverse and the end of the solve
    c.tw = static_cast<const cx<Real>*>(p->tw);
    c.c0 = p->C0;
    c.c2 = p->C2 / 6.0;
    for (int q = 0; q < 3; ++q) c.kq[q] = 2.0 * 3.14159265358979323846 / (double(p->n) * p->h[q]);
    return c;
}

// Slots [0, count) share n, precision and schedule (the caller groups them
// so); v24/v3 >= 0 override the plans' schedule.
template <int DT>
hipError_t solve_group(const psn_host::Slot* slots, int count, hipStream_t s, hipEvent_t* ev, int v24o = -1,
                       int v3o = -1) {
    const int v24 = v24o >= 0 ? v24o : slots[0].plan->sched24, v3 = v3o >= 0 ? v3o : slots[0].plan->sched3;
    for (int base = 0; base < count; base += kMaxBatch) {
        Batch<DT> bt{};
        CorrBatch<DT> cb{};
        bt.count = count - base < kMaxBatch ? count - base : kMaxBatch;
        for (int i = 0; i < bt.count; ++i) {
            const psn_host::Slot& sl = slots[base + i];
            bt.p[i] = prob_of<DT>(sl);
            if (sl.plan->correction == PSN_CORRECTION_FOURIER) cb.p[cb.count++] = corr_of<DT>(sl);
        }
        const CorrBatch<DT>* cbp = cb.count > 0 ? &cb : nullptr;
        hipError_t e = hipErrorInvalidValue;
        switch (slots[0].plan->n) {
#define PSN_CASE(NN) \
    case NN: e = solve_n<NN, DT>(bt, s, ev, v24, v3, cbp); break;
            PSN_FOR_EACH_SIZE(PSN_CASE)
#undef PSN_CASE
            default: break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Time the candidates on a batch group's own entries (their workspaces in
// the batch arena; contents are irrelevant to the timing): the first
// kMaxBatch of them in one launch, as the batch runs them.
template <int DT>
hipError_t tune_slots(const psn_host::Slot* slots, int count, hipStream_t s, int* best24, int* best3) {
    Batch<DT> bt{};
    bt.count = count < kMaxBatch ? count : kMaxBatch;
    for (int i = 0; i < bt.count; ++i) bt.p[i] = prob_of<DT>(slots[i]);
    switch (slots[0].plan->n) {
#define PSN_CASE(NN) \
    case NN: return tune_n<NN, DT>(bt, s, best24, best3);
        PSN_FOR_EACH_SIZE(PSN_CASE)
#undef PSN_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int DT>
hipError_t tune_plan(const psn_plan* p, hipStream_t s, int* best24, int* best3) {
    Batch<DT> bt{};
    bt.count = 1;
    bt.p[0] = prob_of<DT>(psn_host::Slot{p, nullptr, nullptr, p->W1, p->W2});
    switch (p->n) {
#define PSN_CASE(NN) \
    case NN: return tune_n<NN, DT>(bt, s, best24, best3);
        PSN_FOR_EACH_SIZE(PSN_CASE)
#undef PSN_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace psn

// Defines the per-precision entry points of one compilation unit.
#define PSN_DEFINE_PRECISION(DTV, SUFFIX)                                                                       \
    namespace psn_host {                                                                                        \
    hipError_t launch_group_##SUFFIX(const Slot* slots, int count, hipStream_t stream, hipEvent_t* ev, int v24, \
                                     int v3) {                                                                  \
        return psn::solve_group<DTV>(slots, count, stream, ev, v24, v3);                                        \
    }                                                                                                           \
    hipError_t tune_slots_##SUFFIX(const Slot* slots, int count, hipStream_t stream, int* best24, int* best3) { \
        return psn::tune_slots<DTV>(slots, count, stream, best24, best3);                                       \
    }                                                                                                           \
    hipError_t tune_##SUFFIX(const psn_plan* p, hipStream_t stream, int* best24, int* best3) {                \
        return psn::tune_plan<DTV>(p, stream, best24, best3);                                                   \
    }                                                                                                           \
    }
