/*
 * psn.h -- C ABI of the MI355X free-space Poisson solver.
 *
 * Computes u = U * rho with U(x) = 1/(4 pi |x|) on a box (the cube [-L, L]^3 or
 * a general [a0,b0] x [a1,b1] x [a2,b2]) sampled with n points per axis, or n_q
 * points on axis q (both end points included, h_q = (b_q - a_q)/(n_q - 1)), by the
 * method of Exl, "A GPU accelerated and error-controlled solver for the
 * unbounded Poisson equation in three dimensions" (arXiv 1612.01799):
 *
 *   u = crop( IFFT_2n( K * FFT_2n( pad(rho) ) ) ),
 *
 * where K is the spectrum of the Gaussian-sum approximation of U truncated to
 * [-T, T]^3 (T = n h) plus the symbol C0 - (C2/6)|kappa|^2 of the near-zone
 * correction (paper section 2, eq. approx and the G-tensor; section 3 for the
 * transform sizes).  The solve is five pruned passes over the padded (2n)^3
 * spectrum that never materialise its zero half.
 *
 * Conventions shared by every entry point
 *   - Arrays are C order [i0][i1][i2] (i2 contiguous) of n^3 reals (n0 n1 n2
 *     for a plan from psn_plan_create_grid).
 *   - rho and u are DEVICE pointers owned by the caller.  F32 plans read and
 *     write float; F64 and SPLIT plans read and write double.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Solves are
 *     enqueued asynchronously and stream-ordered; argument and state errors are
 *     returned synchronously before anything is enqueued.
 *   - No function throws; every failure is a psn_status.
 */
#ifndef PSN_H
#define PSN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psn_plan psn_plan;

/* Arithmetic of a plan.
 *   PSN_F64   FP64 arithmetic and FP64 storage everywhere.
 *   PSN_F32   FP32 arithmetic, FP32 storage, FP32 kernel spectrum.
 *   PSN_SPLIT FP64 arithmetic inside each pass; the axis-2/axis-1
 *             intermediate stored in 6 bytes per real, split into the high
 *             32-bit word of the FP64 value and the next 16 bits (the value
 *             rounded to 37 significant bits); the axis-1/axis-0 intermediate
 *             in FP64; FP64 kernel spectrum; FP64 input and output. */
typedef enum { PSN_F64 = 0, PSN_F32 = 1, PSN_SPLIT = 2 } psn_dtype;

/* How the near-zone correction I_delta ~ C0 rho + (C2/6) Laplace(rho) enters
 * (paper section 2, eq. approx and the Taylor expansion that follows it).
 *   PSN_CORRECTION_FOLDED   its symbol C0 - (C2/6)|kappa|^2 is added to the
 *                           padded kernel spectrum: no extra work per solve.
 *   PSN_CORRECTION_FOURIER  the paper's own route: the Laplacian from the
 *                           finite Fourier series of the density on its
 *                           n-point grid (period n h per axis), one forward
 *                           and one backward FFT of size N = n^3 (section 3),
 *                           added after the padded convolution with the
 *                           G-tensor alone.
 * For a resolved density the two agree far below the method's error (about
 * 1e-13 of max |u| for a Gaussian of width 1 on a 32^3 grid). */
typedef enum { PSN_CORRECTION_FOLDED = 0, PSN_CORRECTION_FOURIER = 1 } psn_correction;

typedef enum {
    PSN_OK = 0,
    PSN_EINVAL = -1,  /* bad argument: null pointer, L <= 0, tol outside [1e-15, 1e-4], bad dtype */
    PSN_ESIZE = -2,   /* n not supported: n must be even, 2n = 2^a 3^b 5^c, and compiled in */
    PSN_ENOMEM = -3,  /* device allocation failed */
    PSN_EDEVICE = -4, /* a HIP call or kernel launch failed */
    PSN_ESTATE = -5,  /* psn_solve before psn_kernel_build */
    PSN_EFIT = -6,    /* the Gaussian-sum fit missed tol on [delta, R] */
    PSN_ELIMIT = -7   /* a fixed limit of psn_solve_batched_noalloc exceeded */
} psn_status;

typedef struct {
    int n;              /* points per axis */
    int dtype;          /* psn_dtype */
    double L;           /* largest half-width of the box (lambda of section 2; the cube's L) */
    double tol;         /* requested Gaussian-sum relative tolerance eps */
    double h;           /* grid spacing of axis 0: (b0-a0)/(n-1) */
    double T;           /* kernel truncation of axis 0: n*h (half the padded period) */
    double period;      /* padded FFT period of axis 0: 2*n*h */
    double delta;       /* near-zone radius (section 3 heuristic, physical units) */
    double R;           /* largest distance the Gaussian sum must resolve: the box diagonal */
    double hs;          /* sinc-quadrature step */
    int terms;          /* number of Gaussian-sum terms (S + 1) */
    double eps_achieved;/* max |U_GS/U - 1| on the check grid */
    double C0, C2;      /* correction constants; valid once built */
    int built;          /* 1 after psn_kernel_build succeeded */
    size_t device_bytes;     /* device memory held by the plan */
    double algorithmic_bytes;/* HBM bytes one solve must move (five pruned passes) */
    double a[3], b[3];  /* the box [a0,b0] x [a1,b1] x [a2,b2] */
    double h3[3];       /* grid spacing per axis */
    double T3[3];       /* kernel truncation per axis */
    int schedule[2];    /* tile candidates of the axis-1 passes and of the axis-0 pass */
    int tuned;          /* 1 if the schedule came from the autotuner (or its cache file) */
    int device;         /* HIP device the kernel spectrum was built on; -1 before the build */
    int correction;     /* psn_correction */
    int n3[3];          /* points per axis (all n for psn_plan_create and _box) */
} psn_plan_info;

/* Create a plan for an n^3 grid on [-L, L]^3 (the solver construction of the
 * paper's section 4; setup is kept apart from solves, section 3).  Host only:
 * computes the geometry, the near-zone radius and the Gaussian-sum table, and
 * checks that table against 1/(4 pi r) on [delta, R] to `tol`.  No device work
 * and no device memory.  On success *out owns a new plan; on failure *out is
 * set to NULL.  Errors: PSN_EINVAL, PSN_ESIZE, PSN_EFIT. */
psn_status psn_plan_create(int n, double L, double tol, psn_dtype dtype, psn_plan **out);

/* As psn_plan_create for a general rectangular box [a0,b0] x [a1,b1] x [a2,b2]
 * (arrays of 3 doubles, b_q > a_q), n points per axis (section 2's general box:
 * per-axis spacing h_q = (b_q - a_q)/(n-1), per-axis factors of the G-tensor;
 * delta from the smallest axis and lambda = the largest half-width; the
 * Gaussian sum resolves distances up to the box diagonal).
 * Errors: PSN_EINVAL, PSN_ESIZE, PSN_EFIT. */
psn_status psn_plan_create_box(int n, const double *a, const double *b, double tol, psn_dtype dtype,
                               psn_plan **out);

/* As psn_plan_create_box with n[q] points on axis q (arrays of 3: the paper's
 * general box with N = n0 n1 n2 points, section 2 and section 3): spacing
 * h_q = (b_q - a_q)/(n_q - 1), per-axis mode tables, delta from
 * min_q (b_q - a_q)/(50 n_q).  Each n_q must be a supported size.  Equal sizes
 * give the same plan as psn_plan_create_box.  Otherwise the plan runs the
 * five steps on workspaces with rows of hw = n2 + 1 rounded up to a multiple
 * of 8 (W1 n0 n1 hw, W2 2 n0 n1 hw complex; split precision stores them in
 * FP64), has no tile schedules
 * (psn_plan_set_schedule: PSN_EINVAL), takes only the folded correction, and
 * psn_kernel_download fills (n0+1)(n1+1)(n2+1) values.
 * Errors: PSN_EINVAL, PSN_ESIZE, PSN_EFIT. */
psn_status psn_plan_create_grid(const int *n, const double *a, const double *b, double tol, psn_dtype dtype,
                                psn_plan **out);

/* Build the kernel spectrum on the current device (the G-tensor precomputation
 * of section 3): FP64 mode integrals, correction constants C0 and C2 and the
 * octant assembly, then conversion to the plan's storage type; also allocates
 * the solve workspace.  Then picks the tile schedule of the strided passes:
 * each has four compiled candidates, timed once per (n, precision) in the
 * process on this plan's workspace (set PSN_TUNE=0 to keep the defaults).
 * With PSN_TUNE_CACHE naming a file, a schedule recorded there for the same
 * (n, precision) is taken without timing, and a newly timed one is appended,
 * so that separate processes pick the same candidates (candidates agree only
 * within rounding, see psn_plan_set_schedule).
 * Synchronises `stream` before returning.  Idempotent.
 * Errors: PSN_EINVAL, PSN_ENOMEM, PSN_EDEVICE. */
psn_status psn_kernel_build(psn_plan *p, void *stream);

/* Enqueue one solve u = U * rho (paper eq. conv, approximated as in eq.
 * approx).  rho and u are device arrays of n^3 elements of the plan's I/O
 * type; rho == u is allowed.  The plan's workspace is shared, so calls on one
 * plan must not overlap across streams.
 * Errors: PSN_EINVAL, PSN_ESTATE, PSN_EDEVICE. */
psn_status psn_solve(psn_plan *p, const void *rho, void *u, void *stream);

/* Enqueue `count` independent solves, possibly of different sizes, as one
 * batch (many densities on one device).  This is the reuse of a set-up solver
 * for many right-hand sides (paper section 4: construction once, then any
 * number of solves without renewed setup), spread over several geometries at
 * once.  plans[i], rho[i], u[i] as for psn_solve; the same plan may appear
 * more than once.  Each entry runs in its own region of a per-device
 * workspace arena (grown on demand, which synchronises the device; held until
 * the process ends), entries of one (n, precision, schedule) share each
 * kernel launch, and the launch sequence is captured once per argument list
 * and schedule set into a HIP graph and replayed.  Before the first capture
 * of a group of two or more entries whose plans were autotuned, the schedule
 * candidates are timed once on that group's own arena entries (several
 * entries per launch can favour another candidate than one solve); with
 * PSN_TUNE=0 or PSN_TUNE_CACHE set the plans' schedules are kept.  The arena
 * is shared by all batched calls on a device, so such calls must not overlap
 * across streams.  count == 0 does nothing.
 * Errors: as psn_solve, for the first bad entry; PSN_ENOMEM if the arena
 * cannot grow. */
psn_status psn_solve_batched(int count, psn_plan *const *plans,
                             const void *const *rho, void *const *u, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * batch as psn_solve_batched, with the same results, but it allocates
 * nothing.  The workspace of every entry comes from one fixed device array of
 * 256 MiB per device, compiled into the library and held until the process
 * ends (e.g. two n = 160 FP32 entries or twelve n = 96 ones fit; one entry
 * needs about 24 n^3 bytes in FP32, 44 n^3 in SPLIT and 48 n^3 in F64).  No graph is captured:
 * the launches are enqueued on `stream` directly, entries of one
 * (n, precision, schedule) sharing each launch, under the schedule that
 * psn_solve_batched timed for such a group if it did (else the plans').  plans, rho, u as for
 * psn_solve_batched; the plans must have been built (which also looks the
 * array up on their device).  Every call on a device uses the same array, so
 * calls that overlap on one device (any streams, any plans) race; order them
 * on one stream or synchronise between them.
 * Errors: as psn_solve_batched; PSN_ELIMIT (nothing enqueued) if the entries'
 * workspace exceeds the array or count exceeds 1024. */
psn_status psn_solve_batched_noalloc(int count, psn_plan *const *plans,
                                     const void *const *rho, void *const *u, void *stream);

/* As psn_solve, but also records a HIP event on `stream` before the first
 * pass and after each of the five passes (P1 axis-2 real-to-complex, P2
 * axis-1 forward, P3 axis-0 forward x K inverse, P4 axis-1 inverse, P5 axis-2
 * complex-to-real), waits for the stream, and writes the five pass durations
 * in milliseconds to pass_ms[5].  For measurement only (it synchronises).
 * Errors: as psn_solve. */
psn_status psn_solve_timed(psn_plan *p, const void *rho, void *u, void *stream, double *pass_ms);

/* Override the tile schedule: candidate p24 (0..3) for the axis-1 passes and
 * p3 (0..3) for the axis-0 pass.  Every candidate computes the same
 * transform; results agree within rounding but not bitwise, since a
 * candidate may run another radix plan or another order of operations.  For
 * one candidate the result is bitwise reproducible.  Errors: PSN_EINVAL. */
psn_status psn_plan_set_schedule(psn_plan *p, int p24, int p3);

/* Choose how the near-zone correction enters (psn_correction); call before
 * psn_kernel_build, since the kernel spectrum differs.  With
 * PSN_CORRECTION_FOURIER a solve also runs the size-N transform pair; its
 * workspace is the plan's (or the batch entry's) own.
 * Errors: PSN_EINVAL (bad mode, or PSN_CORRECTION_FOURIER on a plan from
 * psn_plan_create_grid with unequal sizes), PSN_ESTATE (already built). */
psn_status psn_plan_set_correction(psn_plan *p, int mode);

/* Fill *info: the discretisation and error-control parameters of the paper's
 * sections 2-3 as this plan derived them (grid spacing h from the section 4
 * grid, truncation T, padded period, near-zone radius delta from the section
 * 3 heuristic, the Gaussian-sum step, term count and achieved tolerance eps,
 * the correction constants C0 and C2 once built), plus the device, memory,
 * algorithmic HBM bytes per solve and the tile schedule.  Host only.
 * Errors: PSN_EINVAL. */
psn_status psn_plan_query(const psn_plan *p, psn_plan_info *info);

/* Copy the Gaussian-sum table to host arrays tau[cap], w[cap] (section 2:
 * U_GS(r) = sum_j w_j exp(-tau_j^2 r^2)).  Returns the number of terms in
 * *terms; copies min(cap, terms) entries.  Errors: PSN_EINVAL. */
psn_status psn_plan_gs_table(const psn_plan *p, double *tau, double *w, int cap, int *terms);

/* Copy the built kernel spectrum to a host array octant[(n0+1)(n1+1)(n2+1)]
 * ((n+1)^3 on a grid of n points per axis), FP64, index [k0][k1][k2] with
 * k_q = 0..n_q the folded frequency index, in the paper's normalisation (no
 * 1/(8 n0 n1 n2) factor).  Synchronous.
 * Errors: PSN_EINVAL, PSN_ESTATE, PSN_EDEVICE. */
psn_status psn_kernel_download(const psn_plan *p, double *octant);

/* Release the plan and its device memory.  NULL is a no-op. */
void psn_plan_destroy(psn_plan *p);

/* Text of the last HIP failure seen by this library on the calling thread
 * (the failing call and HIP's message), or "" if there was none.  The
 * string stays valid until the next call into the library on this thread. */
const char *psn_last_error(void);

/* Static description of a status code. */
const char *psn_strerror(psn_status st);

/* Nonzero if n is a supported grid size (even, 2n 5-smooth, compiled in). */
int psn_size_supported(int n);

#ifdef __cplusplus
}
#endif

#endif /* PSN_H */
