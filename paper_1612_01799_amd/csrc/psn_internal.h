// Host-side plan state shared by the ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "../../include/psn.h"

// Grid sizes compiled into the library: even n with 2n = 2^a 3^b 5^c.
#define PSN_FOR_EACH_SIZE(X) \
    X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(160) X(162) X(192) X(256) X(320) X(384) X(512)

struct psn_plan {
    // geometry (section 4 grid; padded period 2nh; truncation T = nh), per axis
    int n = 0;
    double L = 0, tol = 0;  // L: largest half-width (lambda of section 2)
    psn_dtype dtype = PSN_F64;
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    double h[3] = {0, 0, 0}, T[3] = {0, 0, 0}, period[3] = {0, 0, 0};
    double delta = 0, R = 0;
    // Gaussian sum (section 2)
    double hs = 0, gs_err = 0;
    std::vector<double> tau, w;
    // device state
    int device = -1;
    bool built = false;
    double C0 = 0, C2 = 0;
    void* K = nullptr;    // [k1~][k0~][k2] k1~,k0~ in 0..n, k2 in 0..n-1 (column 0 holds (K0+Kn)/2)
    void* Kb = nullptr;   // [k1~][k0~] (K0-Kn)/2 for the packed DC/Nyquist column
    void* tw = nullptr;   // 2n twiddles exp(-2 pi i m / 2n), compute precision
    void* W1 = nullptr;   // n * n * n complex
    void* W2 = nullptr;   // n * 2n * n complex
    size_t device_bytes = 0;
    // schedule of the strided passes (candidate indices, see Sched)
    int sched24 = 0, sched3 = 0;
    bool tuned = false;
    // near-zone correction: folded into K, or added by its Fourier series
    int correction = PSN_CORRECTION_FOLDED;
    // points per axis; `general` when they differ (the five-step path, with
    // the workspace and octant layouts of g_pitch and g_k_index)
    int ng[3] = {0, 0, 0};
    bool general = false;
};

namespace psn {
// problems per launch of one pass kernel (the by-value launch table)
constexpr int kMaxBatchHost = 32;
}

namespace psn_host {

// Kernel spectrum layout: planes of (n+1) x n reals per folded k~1, each tiled
// over k2 as [k2 / KT][k~0][k2 % KT] with KT the largest of 8, 4, 2, 1 dividing
// n, so the middle pass's workgroup (one k~1, a tile of k2) reads one run.
__host__ __device__ constexpr int k_tile(int n) { return n % 8 == 0 ? 8 : n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : 1; }
__host__ __device__ constexpr size_t k_index(int n, int kt1, int kt0, int k2) {
    return (size_t(kt1) * (n / k_tile(n)) + k2 / k_tile(n)) * size_t(n + 1) * k_tile(n) + size_t(kt0) * k_tile(n) +
           k2 % k_tile(n);
}

// Grids with per-axis sizes: the k2 extent n2 + 1 of the workspaces' rows and
// of the kernel octant is padded to a multiple of kGTile, so that a workgroup
// of the strided steps (up to kGTile consecutive k2) moves whole aligned row
// pieces; the octant is tiled over k2 as [k1][k2 / kGTile][k0][k2 % kGTile],
// so that the axis-0 step's workgroup (one k1, one tile) reads one run.
constexpr int kGTile = 8;
__host__ __device__ constexpr long g_pitch(int n2) { return (long(n2) + kGTile) / kGTile * kGTile; }
__host__ __device__ constexpr size_t g_k_index(int n0, int n2, int k0, int k1, int k2) {
    return ((size_t(k1) * size_t(g_pitch(n2) / kGTile) + size_t(k2 / kGTile)) * size_t(n0 + 1) + size_t(k0)) * kGTile +
           size_t(k2 % kGTile);
}

// k1 block of the W2 layout: the largest power of two <= sqrt(2n) dividing 2n
constexpr int w2_k1_block(int n) {
    int kb = 1;
    while ((2 * kb) * (2 * kb) <= 2 * n && (2 * n) % (2 * kb) == 0) kb *= 2;
    return kb;
}
constexpr size_t kW2BlockPad = 512;  // elements between k1 blocks of W2
// complex elements of W2 (n * 2n * n plus the block pads)
constexpr size_t w2_elems(int n) {
    return size_t(2) * n * n * n + size_t(2 * n / w2_k1_block(n)) * kW2BlockPad;
}

// One problem of a solve: its plan (kernel spectrum, twiddles), its input and
// output, and the workspace it runs in (the plan's own, or a batch arena's).
struct Slot {
    const psn_plan* plan;
    const void* rho;
    void* u;
    void* W1;
    void* W2;
};

// Enqueue the passes for `count` slots that share n and precision (one launch
// per pass per 32 slots).  With `ev` non-null, ev[0] is recorded before the
// first pass and ev[i] after pass i (i = 1..5).
// v24/v3 >= 0 override the plans' schedule for this group.
hipError_t launch_group(const Slot* slots, int count, hipStream_t stream, hipEvent_t* ev = nullptr, int v24 = -1,
                        int v3 = -1);
hipError_t launch_group_f64(const Slot* slots, int count, hipStream_t stream, hipEvent_t* ev, int v24, int v3);
hipError_t launch_group_f32(const Slot* slots, int count, hipStream_t stream, hipEvent_t* ev, int v24, int v3);
hipError_t launch_group_split(const Slot* slots, int count, hipStream_t stream, hipEvent_t* ev, int v24, int v3);

// The five-step solve of a grid with per-axis sizes, one slot (FP32, or
// FP64 arithmetic and storage for F64 and split-precision plans).
hipError_t launch_general_f32(const Slot& sl, hipStream_t stream, hipEvent_t* ev);
hipError_t launch_general_f64(const Slot& sl, hipStream_t stream, hipEvent_t* ev);

// Time the schedule candidates on `count` slots sharing n and precision (the
// first kMaxBatch in one launch; synchronises `stream`); return the fastest.
hipError_t tune_slots(const Slot* slots, int count, hipStream_t stream, int* best24, int* best3);
hipError_t tune_slots_f64(const Slot* slots, int count, hipStream_t stream, int* best24, int* best3);
hipError_t tune_slots_f32(const Slot* slots, int count, hipStream_t stream, int* best24, int* best3);
hipError_t tune_slots_split(const Slot* slots, int count, hipStream_t stream, int* best24, int* best3);

// Time the compiled tile candidates of the strided passes on the plan's own
// workspace (synchronises `stream`) and return the fastest.
hipError_t tune_f64(const psn_plan* p, hipStream_t stream, int* best24, int* best3);
hipError_t tune_f32(const psn_plan* p, hipStream_t stream, int* best24, int* best3);
hipError_t tune_split(const psn_plan* p, hipStream_t stream, int* best24, int* best3);
constexpr int kScheduleCandidates = 4;

// Kernel spectrum build on the device (FP64), written into p->K / p->Kb in
// the plan's storage type, plus C0/C2 into the two doubles at d_c.
// d_A is scratch of kbuild_scratch_doubles(n, terms) doubles: three mode
// tables of terms x (n+1), three moment tables, and the k2 = n column.
size_t kbuild_scratch_doubles(int n, int terms);
hipError_t launch_kernel_build(psn_plan* p, const double* d_tau, const double* d_w, int terms,
                               const double* d_glx, const double* d_glw, double* d_A, double* d_c,
                               hipStream_t stream);

size_t elem_bytes(psn_dtype dt);        // bytes of one complex value in the compute precision (8 or 16)
size_t w1_bytes(psn_dtype dt);          // bytes of one complex element of W1 (8, 16, or 12 split)
size_t w2_bytes(psn_dtype dt);          // bytes of one complex element of W2 (8, or 16: split keeps W2 in FP64)
size_t kernel_elem_bytes(psn_dtype dt); // bytes of one real of the kernel spectrum
bool size_compiled(int n);

}  // namespace psn_host
