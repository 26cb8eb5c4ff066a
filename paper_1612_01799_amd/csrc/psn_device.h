// Device building blocks for the pruned padded-FFT convolution on gfx950:
// complex arithmetic, in-register DFT butterflies, the register-resident
// Stockham "team" FFT, and the storage formats of the three precisions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psn {

// ----------------------------------------------------------------- complex
template <class R>
struct cx {
    R x, y;
};

template <class R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.x * s, a.y * s}; }
template <class R>
__device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.x, -a.y}; }
// a * conj(w)
template <class R>
__device__ __forceinline__ cx<R> mul_conj(cx<R> a, cx<R> w) {
    return {a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y};
}
// multiply by DIR * i  (DIR = -1 forward, +1 inverse)
template <int DIR, class R>
__device__ __forceinline__ cx<R> rot(cx<R> a) {
    if constexpr (DIR < 0) return {a.y, -a.x};
    else return {-a.y, a.x};
}
// twiddle product: a * w (forward) or a * conj(w) (inverse)
template <int DIR, class R>
__device__ __forceinline__ cx<R> twmul(cx<R> a, cx<R> w) {
    if constexpr (DIR < 0) return a * w;
    else return mul_conj(a, w);
}
template <class R>
__device__ __forceinline__ R fmad(R a, R b, R c) {
    if constexpr (sizeof(R) == 4) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}
// c + a * w (forward) or c + a * conj(w) (inverse) as four fused multiply-adds
template <int DIR, class R>
__device__ __forceinline__ cx<R> twfma(cx<R> a, cx<R> w, cx<R> c) {
    const R wy = DIR < 0 ? w.y : -w.y;
    return {fmad(a.x, w.x, fmad(-a.y, wy, c.x)), fmad(a.x, wy, fmad(a.y, w.x, c.y))};
}
// 2 a - s, the partner of s = a + b in a butterfly, by one fused multiply-add per part
template <class R>
__device__ __forceinline__ cx<R> twice_minus(cx<R> a, cx<R> s) {
    return {fmad(R(2), a.x, -s.x), fmad(R(2), a.y, -s.y)};
}

// ----------------------------------------------------------------- butterflies
// In-register DFT of length R with sign DIR: v[k] <- sum_j v[j] exp(DIR 2 pi i jk/R).
template <int R, int DIR, class T>
struct DFT;

template <int DIR, class T>
struct DFT<2, DIR, T> {
    static __device__ __forceinline__ void run(cx<T>* v) {
        cx<T> a = v[0];
        v[0] = a + v[1];
        v[1] = a - v[1];
    }
};

template <int DIR, class T>
struct DFT<4, DIR, T> {
    static __device__ __forceinline__ void run(cx<T>* v) {
        cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
        cx<T> t2 = v[1] + v[3], t3 = rot<DIR>(v[1] - v[3]);
        v[0] = t0 + t2;
        v[2] = t0 - t2;
        v[1] = t1 + t3;
        v[3] = t1 - t3;
    }
};

template <int DIR, class T>
struct DFT<3, DIR, T> {
    static __device__ __forceinline__ void run(cx<T>* v) {
        const T h = T(0.86602540378443864676);  // sin(2 pi / 3)
        cx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
        cx<T> m = v[0] - scale(t1, T(0.5));
        cx<T> s = rot<DIR>(scale(t2, h));
        v[0] = v[0] + t1;
        v[1] = m + s;
        v[2] = m - s;
    }
};

template <int DIR, class T>
struct DFT<5, DIR, T> {
    static __device__ __forceinline__ void run(cx<T>* v) {
        const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
        const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
        cx<T> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
        cx<T> a1 = v[0] + scale(t1, c1) + scale(t2, c2);
        cx<T> a2 = v[0] + scale(t1, c2) + scale(t2, c1);
        cx<T> b1 = rot<DIR>(scale(t3, s1) + scale(t4, s2));
        cx<T> b2 = rot<DIR>(scale(t3, s2) - scale(t4, s1));
        v[0] = v[0] + t1 + t2;
        v[1] = a1 + b1;
        v[4] = a1 - b1;
        v[2] = a2 + b2;
        v[3] = a2 - b2;
    }
};

// Lengths R1 * R2 with coprime R1 (a power of two) and R2 (odd), by the
// prime-factor (Good-Thomas) mapping: input n = (R2 n1 + R1 n2) mod R and
// output k = (R2 t1 k1 + R1 t2 k2) mod R, with t1 R2 = 1 (mod R1) and
// t2 R1 = 1 (mod R2), turn exp(2 pi i nk / R) into the product of
// exp(2 pi i n1 k1 / R1) and exp(2 pi i n2 k2 / R2).  So the DFT is R2 DFTs
// of length R1 followed by R1 DFTs of length R2, with no twiddle factors
// between them; both index maps are compile-time register renamings.
constexpr int mod_inverse(int a, int m) {
    for (int x = 1; x < m; ++x)
        if ((a * x) % m == 1) return x;
    return 1;
}
template <int R1, int R2, int DIR, class T>
struct PrimeFactorDFT {
    static constexpr int R = R1 * R2;
    static constexpr int t1 = mod_inverse(R2 % R1, R1), t2 = mod_inverse(R1 % R2, R2);
    static_assert((R2 * t1) % R1 == 1 % R1 && (R1 * t2) % R2 == 1, "coprime factors");
    static __device__ __forceinline__ void run(cx<T>* v) {
        cx<T> a[R2][R1];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) a[n2][n1] = v[(R2 * n1 + R1 * n2) % R];
            DFT<R1, DIR, T>::run(a[n2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            cx<T> b[R2];
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) b[n2] = a[n2][k1];
            DFT<R2, DIR, T>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) v[(R2 * t1 * k1 + R1 * t2 * k2) % R] = b[k2];
        }
    }
};
template <int DIR, class T>
struct DFT<6, DIR, T> : PrimeFactorDFT<2, 3, DIR, T> {};
template <int DIR, class T>
struct DFT<10, DIR, T> : PrimeFactorDFT<2, 5, DIR, T> {};
template <int DIR, class T>
struct DFT<12, DIR, T> : PrimeFactorDFT<4, 3, DIR, T> {};
template <int DIR, class T>
struct DFT<20, DIR, T> : PrimeFactorDFT<4, 5, DIR, T> {};

// Radix 8 as three layers of radix-2 butterflies.  The first layer pairs
// inputs j and j+4 (s = v_j + v_j+4, d = v_j - v_j+4); its variants below fold
// an input twiddle or an input scale into the butterfly with fused
// multiply-adds (d is formed as 2 v_j - s), which the layers after it share.
template <int DIR, class T>
struct DFT<8, DIR, T> {
    static __device__ __forceinline__ void finish(const cx<T> (&s)[4], const cx<T> (&d)[4], cx<T>* v) {
        const T q = T(0.70710678118654752440);
        // radix-4 on the even inputs (0, 2, 4, 6) and on the odd ones (1, 3, 5, 7)
        cx<T> a[4], b[4];
        const cx<T> ra = rot<DIR>(d[2]), rb = rot<DIR>(d[3]);
        a[0] = s[0] + s[2];
        a[2] = s[0] - s[2];
        a[1] = d[0] + ra;
        a[3] = d[0] - ra;
        b[0] = s[1] + s[3];
        b[2] = s[1] - s[3];
        b[1] = d[1] + rb;
        b[3] = d[1] - rb;
        // b[k] *= exp(DIR 2 pi i k / 8)
        b[1] = {q * (b[1].x - DIR * b[1].y), q * (b[1].y + DIR * b[1].x)};
        b[2] = rot<DIR>(b[2]);
        b[3] = {q * (-b[3].x - DIR * b[3].y), q * (-b[3].y + DIR * b[3].x)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = a[k] + b[k];
            v[k + 4] = a[k] - b[k];
        }
    }
    static __device__ __forceinline__ void run(cx<T>* v) {
        cx<T> s[4], d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[j] = v[j] + v[j + 4];
            d[j] = v[j] - v[j + 4];
        }
        finish(s, d, v);
    }
    // inputs multiplied first by w[j] (forward) or conj(w[j]) (inverse), j = 1..7
    static __device__ __forceinline__ void run_tw(cx<T>* v, const cx<T>* w) {
        cx<T> s[4], d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const cx<T> a = j == 0 ? v[0] : twmul<DIR>(v[j], w[j]);
            s[j] = twfma<DIR>(v[j + 4], w[j + 4], a);
            d[j] = twice_minus(a, s[j]);
        }
        finish(s, d, v);
    }
    // inputs multiplied first by the real k[j], j = 0..7
    static __device__ __forceinline__ void run_scaled(cx<T>* v, const T* k) {
        cx<T> s[4], d[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const cx<T> p = scale(v[j + 4], k[j + 4]);
            s[j] = {fmad(k[j], v[j].x, p.x), fmad(k[j], v[j].y, p.y)};
            d[j] = {fmad(k[j], v[j].x, -p.x), fmad(k[j], v[j].y, -p.y)};
        }
        finish(s, d, v);
    }
};

template <int DIR, class T>
struct DFT<16, DIR, T> {
    static __device__ __forceinline__ void run(cx<T>* v) {
        const T c = T(0.92387953251128675613), s = T(0.38268343236508977173);
        const T q = T(0.70710678118654752440);
        cx<T> a[4][4];
#pragma unroll
        for (int j0 = 0; j0 < 4; ++j0) {
#pragma unroll
            for (int j1 = 0; j1 < 4; ++j1) a[j0][j1] = v[j0 + 4 * j1];
            DFT<4, DIR, T>::run(a[j0]);
        }
        // a[j0][k1] *= exp(DIR 2 pi i j0 k1 / 16); the exponent j0*k1 is in {0..9}
        const T cs[10] = {T(1), c, q, s, T(0), -s, -q, -c, T(-1), -c};
        const T sn[10] = {T(0), s, q, c, T(1), c, q, s, T(0), -s};
#pragma unroll
        for (int j0 = 1; j0 < 4; ++j0) {
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) {
                const int e = j0 * k1;
                const cx<T> w = {cs[e], T(DIR) * sn[e]};
                a[j0][k1] = a[j0][k1] * w;
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            DFT<4, DIR, T>::run(b);
#pragma unroll
            for (int k0 = 0; k0 < 4; ++k0) v[k1 + 4 * k0] = b[k0];
        }
    }
};

// ----------------------------------------------------------------- radix plan
struct RadixPlan {
    int n;
    int r[16];
};

// Stages for a length-N transform with E elements per thread: odd radices
// first, each merged with a factor 4 or 2 into one prime-factor radix (20, 12,
// 10, 6) where that divides both what is left of N and E; then the largest
// power-of-two radix (<= 16) dividing both what is left of N and the
// power-of-two part of E, so each stage gives every thread a whole number of
// butterflies.
constexpr int odd_radix(int f, int rem, int E) {
    for (int p = 4; p >= 1; p /= 2)
        if (rem % (f * p) == 0 && E % (f * p) == 0) return f * p;
    return -1;
}
constexpr RadixPlan make_plan(int N, int E) {
    RadixPlan p{0, {}};
    if (N < 1 || E < 1 || N % E != 0) return RadixPlan{-1, {}};
    int rem = N;
    // every radix must divide E: a thread runs E / R butterflies of radix R per stage
    for (int f = 5; f >= 3; f -= 2) {
        while (rem % f == 0) {
            const int R = odd_radix(f, rem, E);
            if (R < 0) return RadixPlan{-1, {}};
            p.r[p.n++] = R;
            rem /= R;
        }
    }
    int e2 = E & -E;
    while (rem > 1) {
        int R = 16;
        while (R > 1 && (rem % R != 0 || e2 % R != 0)) R /= 2;
        if (R == 1) return RadixPlan{-1, {}};
        p.r[p.n++] = R;
        rem /= R;
    }
    return p;
}

// Elements per thread for a length-N line: N's odd factors, at most 15 of
// them (an odd part above 15, such as 81, keeps its largest divisor up to 9:
// radix-3 stages then fill the rest), times up to 16 (N a power of two; 8
// for 8-byte reals) or 4 (N with a factor 3 or 5) of its powers of two.
constexpr int elems_per_thread(int N, int real_bytes) {
    int odd = N;
    while (odd % 2 == 0) odd /= 2;
    int p2 = N / odd;
    int cap = odd == 1 ? (real_bytes == 8 ? 8 : 16) : 4;
    int oe = odd;
    if (oe > 15) {
        oe = 1;
        for (int d = 9; d >= 1; --d)
            if (odd % d == 0) {
                oe = d;
                break;
            }
        cap = 2;
    }
    return oe * (p2 < cap ? p2 : cap);
}

// ----------------------------------------------------------------- twiddle sources
// exp(-2 pi i m / 2N) for m in [0, 2N)
template <class Real>
struct TwGlobal {
    static constexpr bool kRows = false;
    const cx<Real>* __restrict__ p;
    __device__ __forceinline__ cx<Real> operator()(int m) const { return p[m]; }
};
// LDS copy of the table, entries permuted within aligned blocks of 16 (XOR
// swizzle, no padding): the stage twiddles one wave reads are multiples of a
// power-of-two stride apart, which would otherwise fall into one bank.
template <class Real>
struct TwLds {
    static constexpr bool kRows = false;
    cx<Real>* p;
    static constexpr int slots(int N) { return (2 * N + 15) & ~15; }
    __device__ __forceinline__ static int at(int m) { return m ^ ((m >> 4) & 15); }
    __device__ __forceinline__ cx<Real> operator()(int m) const { return p[at(m)]; }
    // cooperative copy of the 2N-entry table; visible after the next barrier
    __device__ __forceinline__ void fill(const cx<Real>* __restrict__ tw, int N, int tid, int nthreads) {
        for (int i = tid; i < 2 * N; i += nthreads) p[at(i)] = tw[i];
    }
};

// Twiddles of a half-length transform (length N/2 needs exp(-2 pi i m / N))
// from the 2N-entry table of the full length: entry 2m.
template <class Real>
struct TwHalf {
    static constexpr bool kRows = false;
    TwLds<Real> full;
    __device__ __forceinline__ cx<Real> operator()(int m) const { return full(2 * m); }
};

// Per-stage twiddle rows in LDS, laid out by TeamFFT::fill_rows: a thread
// reads all R - 1 factors of a stage from one row.
template <class Real>
struct TwRows {
    static constexpr bool kRows = true;
    const cx<Real>* p;
};

// Adapts a one-value LDS view to the cx[1] interface of TeamFFT::stage.
template <class Lds>
struct Single {
    static constexpr bool kSeq = false;
    Lds& l;
    template <class C>
    __device__ __forceinline__ void put2(int base, int off, const C (&v)[1]) { l.put2(base, off, v[0]); }
    template <class C>
    __device__ __forceinline__ void get2(int base, int off, C (&v)[1]) const { v[0] = l.get2(base, off); }
    __device__ __forceinline__ void sync() { l.sync(); }
};

// ----------------------------------------------------------------- team FFT
// A team of T threads computes one length-N transform (DIR = -1 forward,
// +1 inverse, unnormalised) with the Stockham autosort algorithm: natural
// order in and out.  Thread t holds E = N/T elements in registers.  On entry
// slot e holds input position in_pos(t, e); on exit it holds output position
// out_pos(t, e).  Between stages the team exchanges through an LDS view
// (`Lds::put/get` at a position, `Lds::sync` = workgroup barrier).
// With REV the radices run in reverse order; a REV transform's in_pos is the
// forward transform's out_pos, so a forward pass and a REV inverse pass can be
// chained in registers (used for the fused multiply of the middle pass).
template <int N, int T, class Real, int DIR, bool REV>
struct TeamFFT {
    static constexpr int E = N / T;
    static constexpr RadixPlan plan = make_plan(N, E);
    static constexpr int S = plan.n;
    static_assert(N % T == 0, "team must divide the line");
    static_assert(S > 0, "no radix plan for this size");
    static constexpr bool radices_divide_e() {
        for (int i = 0; i < S; ++i)
            if (E % plan.r[i] != 0) return false;
        return true;
    }
    static_assert(radices_divide_e(), "every radix must divide the elements per thread");

    static constexpr int radix(int i) { return REV ? plan.r[S - 1 - i] : plan.r[i]; }
    static constexpr int span(int i) {
        int ns = 1;
        for (int q = 0; q < i; ++q) ns *= radix(q);
        return ns;
    }
    static constexpr int R0 = radix(0);
    static constexpr int RL = radix(S - 1);

    // Twiddle rows: stage i (span Ns = span(i) > 1, radix R) keeps, for each
    // k < Ns, the factors exp(-2 pi i r k step / 2N), r = 1..R-1, step =
    // 2N / (Ns R), in a row of row_pitch(i) entries (odd, so that rows of
    // neighbouring k fall into different banks); the stages are packed in
    // order.  A thread's k for a stage is t % Ns or t plus a constant (see
    // row_k), so one row address per stage serves all its twiddles.
    static constexpr int row_pitch(int i) { return (radix(i) - 1) | 1; }
    static constexpr int rows_offset(int i) {
        int o = 0;
        for (int q = 1; q < i; ++q) o += span(q) * row_pitch(q);
        return o;
    }
    static constexpr int rows_size() { return rows_offset(S); }  // entries
    // true when both transforms use the same rows (same radices in the same order)
    template <class F2>
    static constexpr bool same_rows() {
        if (F2::S != S) return false;
        for (int i = 0; i < S; ++i)
            if (F2::radix(i) != radix(i)) return false;
        return true;
    }
    // cooperative fill from the 2N-entry table tw2n (global; with TS = 2,
    // every other entry of the table of a transform twice as long); visible
    // after the next barrier
    template <int I = 1, int TS = 1>
    static __device__ __forceinline__ void fill_rows(cx<Real>* rows, const cx<Real>* __restrict__ tw2n, int tid,
                                                     int nthreads) {
        if constexpr (I < S) {
            constexpr int Ns = span(I), R = radix(I), RP = row_pitch(I), step = 2 * N / (Ns * R);
            cx<Real>* row0 = rows + rows_offset(I);
            for (int idx = tid; idx < Ns * RP; idx += nthreads) {
                const int k = idx / RP, r = idx % RP + 1;
                row0[idx] = r < R ? tw2n[TS * r * k * step] : cx<Real>{Real(0), Real(0)};
            }
            fill_rows<I + 1, TS>(rows, tw2n, tid, nthreads);
        }
    }
    // k of group s of thread t in stage i, (t + T s) mod Ns, written so that
    // its t part and its s part separate where the sizes allow
    template <int Ns>
    static __device__ __forceinline__ int row_k(int t, int s) {
        if constexpr (T % Ns == 0) return t % Ns;
        else if constexpr (Ns % T == 0) return t + T * (s % (Ns / T));
        else return (t + T * s) % Ns;
    }

    static __device__ __forceinline__ int in_pos(int t, int e) {
        return t + T * (e / R0) + (e % R0) * (N / R0);
    }
    static __device__ __forceinline__ int out_pos(int t, int e) {
        return t + T * (e / RL) + (e % RL) * (N / RL);
    }

    // NC independent lines per thread advance together: one barrier pair per
    // exchange serves all of them.  `lds` stores the NC values of one position
    // together (put2/get2 of cx[NC] at position base + off, off a compile-time
    // constant); `tw(m)` returns exp(-2 pi i m / 2N).
    // ks: if not null, per-element real scales applied to the input of stage 0
    template <int I, int NC, class Lds, class Tw>
    static __device__ __forceinline__ void stage(cx<Real> (&d)[NC][E], int t, const Tw& tw, Lds& lds,
                                                 const Real (*ks)[E] = nullptr) {
        if constexpr (I < S) {
            constexpr int R = radix(I);
            constexpr int Ns = span(I);
            constexpr int twstep = 2 * N / (Ns * R);
            if constexpr (I > 0 && !Lds::kSeq) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    cx<Real> v[NC];
                    lds.get2(t, T * (e / R) + (e % R) * (N / R), v);
#pragma unroll
                    for (int c = 0; c < NC; ++c) d[c][e] = v[c];
                }
            }
#pragma unroll
            for (int s = 0; s < E / R; ++s) {
                cx<Real> w[R];
                if constexpr (Ns > 1) {
                    if constexpr (Tw::kRows) {
                        const cx<Real>* row = tw.p + rows_offset(I) + row_k<Ns>(t, s) * row_pitch(I);
#pragma unroll
                        for (int r = 1; r < R; ++r) w[r] = row[r - 1];
                    } else {
                        const int k = (t + T * s) % Ns;
#pragma unroll
                        for (int r = 1; r < R; ++r) w[r] = tw(r * k * twstep);
                    }
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    cx<Real>* v = d[c] + s * R;
                    if constexpr (Ns > 1) {
                        if constexpr (R == 8) {
                            DFT<8, DIR, Real>::run_tw(v, w);
                        } else {
#pragma unroll
                            for (int r = 1; r < R; ++r) v[r] = twmul<DIR>(v[r], w[r]);
                            DFT<R, DIR, Real>::run(v);
                        }
                    } else if (I == 0 && ks != nullptr) {
                        if constexpr (R == 8) {
                            DFT<8, DIR, Real>::run_scaled(v, ks[c] + s * R);
                        } else {
#pragma unroll
                            for (int r = 0; r < R; ++r) v[r] = scale(v[r], ks[c][s * R + r]);
                            DFT<R, DIR, Real>::run(v);
                        }
                    } else {
                        DFT<R, DIR, Real>::run(v);
                    }
                }
            }
            if constexpr (I + 1 < S) {
                // output position of slot e as (per-thread base, constant offset)
                auto put_at = [&](int e, int& base, int& off) {
                    if constexpr (T % Ns == 0) {
                        base = (t / Ns) * Ns * R + t % Ns;
                        off = T * (e / R) * R + (e % R) * Ns;
                    } else {
                        const int b = t + T * (e / R);
                        base = (b / Ns) * Ns * R + (b % Ns) + (e % R) * Ns;
                        off = 0;
                    }
                };
                if constexpr (Lds::kSeq) {
                    // G chains at a time through a G-chain buffer
                    constexpr int R2 = radix(I + 1);
                    constexpr int G = Lds::kGroup;
                    static_assert(NC % G == 0, "the chains split into whole groups");
#pragma unroll
                    for (int c0 = 0; c0 < NC; c0 += G) {
                        lds.sync();
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            int base, off;
                            put_at(e, base, off);
                            cx<Real> v[G];
#pragma unroll
                            for (int g = 0; g < G; ++g) v[g] = d[c0 + g][e];
                            lds.putg(base, off, v);
                        }
                        lds.sync();
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            cx<Real> v[G];
                            lds.getg(t, T * (e / R2) + (e % R2) * (N / R2), v);
#pragma unroll
                            for (int g = 0; g < G; ++g) d[c0 + g][e] = v[g];
                        }
                    }
                } else {
                    lds.sync();
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        cx<Real> v[NC];
#pragma unroll
                        for (int c = 0; c < NC; ++c) v[c] = d[c][e];
                        int base, off;
                        put_at(e, base, off);
                        lds.put2(base, off, v);
                    }
                    lds.sync();
                }
            }
            stage<I + 1, NC>(d, t, tw, lds);
        }
    }

    template <int NC, class Lds, class Tw>
    static __device__ __forceinline__ void run(cx<Real> (&d)[NC][E], int t, const Tw& tw, Lds& lds) {
        stage<0, NC>(d, t, tw, lds);
    }
    // the same, with the input of chain c, slot e first multiplied by the real ks[c][e]
    template <int NC, class Lds, class Tw>
    static __device__ __forceinline__ void run_scaled(cx<Real> (&d)[NC][E], int t, const Tw& tw, Lds& lds,
                                                      const Real (&ks)[NC][E]) {
        stage<0, NC>(d, t, tw, lds, ks);
    }

    // single line per thread, twiddles from a global table
    template <class Lds>
    static __device__ __forceinline__ void run(cx<Real> (&d)[E], int t, const cx<Real>* __restrict__ tw,
                                               Lds& lds) {
        TwGlobal<Real> g{tw};
        run1(d, t, g, lds);
    }

    // single line per thread, any twiddle source
    template <class Lds, class Tw>
    static __device__ __forceinline__ void run1(cx<Real> (&d)[E], int t, const Tw& tw, Lds& lds) {
        cx<Real> dd[1][E];
#pragma unroll
        for (int e = 0; e < E; ++e) dd[0][e] = d[e];
        Single<Lds> l1{lds};
        stage<0, 1>(dd, t, tw, l1);
#pragma unroll
        for (int e = 0; e < E; ++e) d[e] = dd[0][e];
    }
};

// ----------------------------------------------------------------- LDS views
// Strided passes: lines are columns of a tile, element-major, column fastest.
template <class Real>
struct LdsCols {
    static constexpr bool kSeq = false;
    cx<Real>* buf;
    int stride;  // columns per element row
    int col;
    __device__ __forceinline__ void put(int pos, cx<Real> v) { buf[pos * stride + col] = v; }
    __device__ __forceinline__ cx<Real> get(int pos) const { return buf[pos * stride + col]; }
    __device__ __forceinline__ void put2(int base, int off, cx<Real> v) { put(base + off, v); }
    __device__ __forceinline__ cx<Real> get2(int base, int off) const { return get(base + off); }
    __device__ __forceinline__ void sync() { __syncthreads(); }
};

// Strided passes, NC chains per line: element-major, column next, chain
// fastest, so one wide access moves two chains of an element (two FP32
// chains: 16 bytes).  Four chains live in two such planes (chains 0-1, then
// 2-3), so that consecutive positions stay one 2-chain row apart and the
// lanes of a wave spread over the LDS banks as with two chains.
template <class Real, int NC>
struct LdsColsN {
    static_assert(NC == 1 || NC == 2 || NC == 4, "one, two or four chains");
    static constexpr bool kSeq = false;
    static constexpr int kPlane = NC == 4 ? 2 : NC;  // chains per plane
    cx<Real>* buf;
    int stride;  // columns per element row
    int col;
    int plane = 0;  // elements per plane (four chains: positions * stride * 2)
    __device__ __forceinline__ void put(int pos, const cx<Real> (&v)[NC]) {
        cx<Real>* q = buf + kPlane * (pos * stride + col);
#pragma unroll
        for (int c = 0; c < NC; ++c) q[(c / kPlane) * plane + c % kPlane] = v[c];
    }
    __device__ __forceinline__ void get(int pos, cx<Real> (&v)[NC]) const {
        const cx<Real>* q = buf + kPlane * (pos * stride + col);
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = q[(c / kPlane) * plane + c % kPlane];
    }
    __device__ __forceinline__ void put2(int base, int off, const cx<Real> (&v)[NC]) { put(base + off, v); }
    __device__ __forceinline__ void get2(int base, int off, cx<Real> (&v)[NC]) const { get(base + off, v); }
    __device__ __forceinline__ void sync() { __syncthreads(); }
};
template <class Real>
using LdsCols2 = LdsColsN<Real, 2>;

// Strided passes, the chains of a line exchanged G at a time through a
// G-chain buffer: less LDS per column than all chains at once, two more
// barriers per exchange for each further group.
template <class Real, int G = 1>
struct LdsColsSeq {
    static constexpr bool kSeq = true;
    static constexpr int kGroup = G;
    cx<Real>* buf;
    int stride;  // columns per element row
    int col;
    __device__ __forceinline__ void putg(int base, int off, const cx<Real> (&v)[G]) {
        cx<Real>* q = buf + G * ((base + off) * stride + col);
#pragma unroll
        for (int c = 0; c < G; ++c) q[c] = v[c];
    }
    __device__ __forceinline__ void getg(int base, int off, cx<Real> (&v)[G]) const {
        const cx<Real>* q = buf + G * ((base + off) * stride + col);
#pragma unroll
        for (int c = 0; c < G; ++c) v[c] = q[c];
    }
    __device__ __forceinline__ void sync() { __syncthreads(); }
};

// Contiguous passes: one row per line, with one pad slot every 16 elements so
// strided butterfly writes spread over the banks.
template <class Real>
struct LdsRows {
    static constexpr bool kSeq = false;
    cx<Real>* buf;
    __device__ __forceinline__ static int skew(int pos) { return pos + (pos >> 4); }
    // skew(base + off) for a constant off: a multiple of 16 passes through the
    // shift exactly (base + off >= 0), so only base's skew is computed
    __device__ __forceinline__ static int skew2(int base, int off) {
        return (off % 16 == 0) ? skew(base) + off + off / 16 : skew(base + off);
    }
    __device__ __forceinline__ void put(int pos, cx<Real> v) { buf[skew(pos)] = v; }
    __device__ __forceinline__ cx<Real> get(int pos) const { return buf[skew(pos)]; }
    __device__ __forceinline__ void put2(int base, int off, cx<Real> v) { buf[skew2(base, off)] = v; }
    __device__ __forceinline__ cx<Real> get2(int base, int off) const { return buf[skew2(base, off)]; }
    __device__ __forceinline__ void sync() { __syncthreads(); }
};

// ----------------------------------------------------------------- storage
// Precision codes match psn_dtype.
enum { DT_F64 = 0, DT_F32 = 1, DT_SPLIT = 2 };

template <int DT>
struct Prec;

template <>
struct Prec<DT_F64> {
    using Real = double;  // arithmetic
    using Io = double;    // rho, u
    using Kt = double;    // kernel spectrum
};
template <>
struct Prec<DT_F32> {
    using Real = float;
    using Io = float;
    using Kt = float;
};
template <>
struct Prec<DT_SPLIT> {
    using Real = double;
    using Io = double;
    using Kt = double;
};


// Workspace of complex values between passes.
template <int DT>
struct Work;

// Global-memory load and store.  The workspace pointers reach a kernel through
// a table in its arguments, from which the compiler cannot tell their address
// space; a flat access would also count against the LDS wait counter and so
// tie the wait for an LDS exchange to outstanding HBM traffic.
#define PSN_GLOBAL __attribute__((address_space(1)))
template <class R>
using vec2 = R __attribute__((ext_vector_type(2)));
template <class R>
__device__ __forceinline__ cx<R> gld(const cx<R>* p) {
    const vec2<R> v = *(const PSN_GLOBAL vec2<R>*)(p);
    return {v.x, v.y};
}
template <class R>
__device__ __forceinline__ void gst(cx<R>* p, cx<R> v) {
    *(PSN_GLOBAL vec2<R>*)(p) = vec2<R>{v.x, v.y};
}
__device__ __forceinline__ uint32_t gld(const uint32_t* p) { return *(const PSN_GLOBAL uint32_t*)(p); }
__device__ __forceinline__ float gld(const float* p) { return *(const PSN_GLOBAL float*)(p); }
__device__ __forceinline__ double gld(const double* p) { return *(const PSN_GLOBAL double*)(p); }
// two consecutive complex floats in one 16-byte access (p 16-byte aligned)
typedef float psn_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t psn_u2 __attribute__((ext_vector_type(2)));
typedef uint32_t psn_u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void gst2(cx<float>* p, cx<float> a, cx<float> b) {
    *(PSN_GLOBAL psn_f4*)(p) = psn_f4{a.x, a.y, b.x, b.y};
}

__device__ __forceinline__ void gst(uint32_t* p, uint32_t v) { *(PSN_GLOBAL uint32_t*)(p) = v; }

// Pointer `base` advanced by `ob` bytes.  With base uniform over the wave and
// ob a 32-bit lane value, the access takes the scalar-base form: the uniform
// part stays in scalar registers and the lane part is one 32-bit register.
// `p` kept in scalar registers as an opaque value, so that the compiler does
// not move a uniform offset added to it into per-lane 64-bit address
// arithmetic.  p must be uniform over the wave.
template <class T>
__device__ __forceinline__ T* sbase(T* p) {
    asm("" : "+s"(p));
    return p;
}
template <class T>
__device__ __forceinline__ T* byte_off(T* base, uint32_t ob) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + ob);
}
template <class T>
__device__ __forceinline__ const T* byte_off(const T* base, uint32_t ob) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + ob);
}

// ld/st(i) address element i; ld/st(ub, off) address element ub + off with ub
// uniform over the wave and off a 32-bit lane offset whose byte offset also
// fits 32 bits.
template <>
struct Work<DT_F32> {
    cx<float>* p;
    __device__ __forceinline__ cx<float> ld(size_t i) const { return gld(p + i); }
    __device__ __forceinline__ void st(size_t i, cx<float> v) const { gst(p + i, v); }
    __device__ __forceinline__ cx<float> ld(size_t ub, uint32_t off) const { return gld(byte_off(sbase(p + ub), off * 8u)); }
    __device__ __forceinline__ void st(size_t ub, uint32_t off, cx<float> v) const {
        gst(byte_off(sbase(p + ub), off * 8u), v);
    }
    // elements i and i+1 (i even)
    __device__ __forceinline__ void st2(size_t i, cx<float> a, cx<float> b) const { gst2(p + i, a, b); }
    // elements ub + off and ub + off + 1 (ub + off even) in one 16-byte access
    __device__ __forceinline__ void ld_pair(size_t ub, uint32_t off, cx<float>& a, cx<float>& b) const {
        const psn_f4 v = *(const PSN_GLOBAL psn_f4*)(byte_off(sbase(p + ub), off * 8u));
        a = {v.x, v.y};
        b = {v.z, v.w};
    }
    __device__ __forceinline__ void st_pair(size_t ub, uint32_t off, cx<float> a, cx<float> b) const {
        *(PSN_GLOBAL psn_f4*)(byte_off(sbase(p + ub), off * 8u)) = psn_f4{a.x, a.y, b.x, b.y};
    }
    __device__ __forceinline__ void ld_pair(size_t i, cx<float>& a, cx<float>& b) const {
        const psn_f4 v = *(const PSN_GLOBAL psn_f4*)(p + i);
        a = {v.x, v.y};
        b = {v.z, v.w};
    }
};
template <>
struct Work<DT_F64> {
    cx<double>* p;
    __device__ __forceinline__ cx<double> ld(size_t i) const { return gld(p + i); }
    __device__ __forceinline__ void st(size_t i, cx<double> v) const { gst(p + i, v); }
    __device__ __forceinline__ cx<double> ld(size_t ub, uint32_t off) const {
        return gld(byte_off(sbase(p + ub), off * 16u));
    }
    __device__ __forceinline__ void st(size_t ub, uint32_t off, cx<double> v) const {
        gst(byte_off(sbase(p + ub), off * 16u), v);
    }
    __device__ __forceinline__ void st2(size_t i, cx<double> a, cx<double> b) const {
        gst(p + i, a);
        gst(p + i + 1, b);
    }
    __device__ __forceinline__ void ld_pair(size_t ub, uint32_t off, cx<double>& a, cx<double>& b) const {
        const cx<double>* q = byte_off(sbase(p + ub), off * 16u);
        a = gld(q);
        b = gld(q + 1);
    }
    __device__ __forceinline__ void st_pair(size_t ub, uint32_t off, cx<double> a, cx<double> b) const {
        cx<double>* q = byte_off(sbase(p + ub), off * 16u);
        gst(q, a);
        gst(q + 1, b);
    }
    __device__ __forceinline__ void ld_pair(size_t i, cx<double>& a, cx<double>& b) const {
        a = gld(p + i);
        b = gld(p + i + 1);
    }
};
// FP64 values in 6 bytes per real: each real rounded to its leading 48 bits
// (sign, exponent and 36 fraction bits: 37 significant bits, half an ulp of
// 2^-37 relative).  A complex value is one 12-byte element of three 32-bit
// words: the high words of the real and imaginary parts, then both parts'
// next 16 bits, so one access per lane moves a whole element.  Unpacking is
// a shift and a mask; no float conversions.
typedef uint32_t psn_u3 __attribute__((ext_vector_type(3)));
template <>
struct Work<DT_SPLIT> {
    uint32_t* p;  // 3 words per element
    static __device__ __forceinline__ psn_u3 pack(cx<double> v) {
        // + 2^15 rounds the kept 48 bits to nearest (a carry may reach the exponent)
        const uint64_t bx = uint64_t(__double_as_longlong(v.x)) + 0x8000u;
        const uint64_t by = uint64_t(__double_as_longlong(v.y)) + 0x8000u;
        return psn_u3{uint32_t(bx >> 32), uint32_t(by >> 32), (uint32_t(bx) >> 16) | (uint32_t(by) & 0xFFFF0000u)};
    }
    static __device__ __forceinline__ cx<double> join(psn_u3 w) {
        return {__longlong_as_double((long long)((uint64_t(w.x) << 32) | uint64_t(w.z << 16))),
                __longlong_as_double((long long)((uint64_t(w.y) << 32) | uint64_t(w.z & 0xFFFF0000u)))};
    }
    static __device__ __forceinline__ psn_u3 ld3(const uint32_t* q) { return *(const PSN_GLOBAL psn_u3*)(q); }
    static __device__ __forceinline__ void st3(uint32_t* q, psn_u3 w) { *(PSN_GLOBAL psn_u3*)(q) = w; }
    __device__ __forceinline__ cx<double> ld(size_t i) const { return join(ld3(p + 3 * i)); }
    __device__ __forceinline__ void st(size_t i, cx<double> v) const { st3(p + 3 * i, pack(v)); }
    __device__ __forceinline__ cx<double> ld(size_t ub, uint32_t off) const {
        return join(ld3(byte_off(sbase(p + 3 * ub), off * 12u)));
    }
    __device__ __forceinline__ void st(size_t ub, uint32_t off, cx<double> v) const {
        st3(byte_off(sbase(p + 3 * ub), off * 12u), pack(v));
    }
    // elements i and i+1
    __device__ __forceinline__ void st2(size_t i, cx<double> a, cx<double> b) const {
        st3(p + 3 * i, pack(a));
        st3(p + 3 * i + 3, pack(b));
    }
    __device__ __forceinline__ void ld_pair(size_t ub, uint32_t off, cx<double>& a, cx<double>& b) const {
        const uint32_t* q = byte_off(sbase(p + 3 * ub), off * 12u);
        a = join(ld3(q));
        b = join(ld3(q + 3));
    }
    __device__ __forceinline__ void st_pair(size_t ub, uint32_t off, cx<double> a, cx<double> b) const {
        uint32_t* q = byte_off(sbase(p + 3 * ub), off * 12u);
        st3(q, pack(a));
        st3(q + 3, pack(b));
    }
    __device__ __forceinline__ void ld_pair(size_t i, cx<double>& a, cx<double>& b) const {
        a = join(ld3(p + 3 * i));
        b = join(ld3(p + 3 * i + 3));
    }
};

}  // namespace psn
