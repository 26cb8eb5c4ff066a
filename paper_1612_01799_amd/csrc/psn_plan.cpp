// C ABI: plan creation (geometry, near-zone radius, Gaussian-sum table and its
// self-check), device state, and the entry points declared in psn.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "psn_internal.h"

namespace {

thread_local std::string g_last_error;

// Record a failed HIP call (its name and HIP's message) and report it.
bool hip_ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    (void)hipGetLastError();
    return false;
}

constexpr double kPi = 3.14159265358979323846;

bool five_smooth(long v) {
    if (v <= 0) return false;
    for (long f : {2L, 3L, 5L})
        while (v % f == 0) v /= f;
    return v == 1;
}

// Inverse of erfc by Newton's method on log(erfc(x)) (well conditioned for
// the tiny arguments used here).
double erfcinv(double y) {
    double x = std::sqrt(-std::log(y));
    for (int it = 0; it < 100; ++it) {
        const double e = std::erfc(x);
        const double g = std::log(e) - std::log(y);
        const double dg = -2.0 / std::sqrt(kPi) * std::exp(-x * x) / e;
        const double dx = g / dg;
        x -= dx;
        if (std::fabs(dx) < 1e-16 * x) break;
    }
    return x;
}

// max over log-spaced r in [delta, R] of |4 pi r U_GS(r) - 1|.  The radii are
// split over a few host threads; each radius is summed the same way whoever
// takes it, and a maximum does not depend on the order, so the result is the
// same for any thread count.
double gs_max_rel_error(const std::vector<double>& tau, const std::vector<double>& w, double delta, double R,
                        int points) {
    const double a = std::log(delta), b = std::log(R);
    auto part = [&](int i0, int i1) {
        double worst = 0.0;
        for (int i = i0; i < i1; ++i) {
            const double r = std::exp(a + (b - a) * i / (points - 1));
            double s = 0.0;
            for (size_t j = 0; j < tau.size(); ++j) s += w[j] * std::exp(-(tau[j] * r) * (tau[j] * r));
            worst = std::fmax(worst, std::fabs(4.0 * kPi * r * s - 1.0));
        }
        return worst;
    };
    const int nt = int(std::max(1u, std::min(8u, std::thread::hardware_concurrency())));
    std::vector<double> worst(nt, 0.0);
    std::vector<std::thread> pool;
    for (int k = 1; k < nt; ++k)
        pool.emplace_back([&, k] { worst[k] = part(int(long(points) * k / nt), int(long(points) * (k + 1) / nt)); });
    worst[0] = part(0, int(long(points) / nt));
    for (auto& th : pool) th.join();
    return *std::max_element(worst.begin(), worst.end());
}

// Gaussian sum by sinc quadrature of 1/r = (2/sqrt(pi)) int exp(-r^2 e^{2t} + t) dt
// (paper section 2): tau_j = exp(j hs), w_j = hs tau_j / (2 pi^{3/2}).  The
// tolerance eps is split in quarters over the step error (the integrand is
// analytic for |Im t| < pi/4), the tail t > t_max (relative error
// erfc(r e^{t_max}) at r = delta) and the tail t < t_min (relative error
// (2/sqrt(pi)) r e^{t_min} at r = R).  The fit is then checked on [delta, R];
// on failure the step shrinks by 5 %.
bool fit_gaussian_sum(psn_plan* p) {
    const double ep = p->tol / 4.0;
    double hs = kPi * kPi / (2.0 * std::log(2.0 / ep));
    const double t_max = std::log(erfcinv(ep) / p->delta);
    const double t_min = std::log(ep * std::sqrt(kPi) / (2.0 * p->R));
    for (int attempt = 0; attempt < 20; ++attempt) {
        const long j0 = (long)std::floor(t_min / hs), j1 = (long)std::ceil(t_max / hs);
        p->tau.clear();
        p->w.clear();
        for (long j = j0; j <= j1; ++j) {
            const double tj = std::exp(double(j) * hs);
            p->tau.push_back(tj);
            p->w.push_back(hs * tj / (2.0 * std::pow(kPi, 1.5)));
        }
        p->hs = hs;
        p->gs_err = gs_max_rel_error(p->tau, p->w, p->delta, p->R, 32768);
        if (p->gs_err <= p->tol) return true;
        hs *= 0.95;
    }
    return false;
}

// 16-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_16).
void gauss_legendre16(double* x, double* wt) {
    const int m = 16;
    for (int i = 0; i < m; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (m + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= m; ++k) {
                const double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = m * (z * p0 - p1) / (z * z - 1.0);
            const double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        x[i] = z;
        wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

psn_status dev_alloc(void** ptr, size_t bytes, size_t* total) {
    if (!hip_ok(hipMalloc(ptr, bytes), "hipMalloc")) {
        *ptr = nullptr;
        return PSN_ENOMEM;
    }
    *total += bytes;
    return PSN_OK;
}

void free_device(psn_plan* p) {
    for (void** q : {&p->K, &p->Kb, &p->tw, &p->W1, &p->W2}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    p->device_bytes = 0;
    p->built = false;
}

bool is_real_dtype(int d) { return d == PSN_F64 || d == PSN_F32 || d == PSN_SPLIT; }

// Autotuned schedules, once per (n, precision) and process.  PSN_TUNE=0 keeps
// the default tiles.  PSN_TUNE_CACHE names a text file of lines
// "n precision p24 p3": a recorded schedule is taken without timing and a
// newly timed one is appended, so separate processes agree on the candidates.
std::mutex g_tune_mutex;
std::map<std::pair<int, int>, std::pair<int, int>> g_tuned;

bool tune_cache_lookup(const char* path, int n, int dt, int* b24, int* b3) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    int a, b, c, d;
    bool found = false;
    while (std::fscanf(f, "%d %d %d %d", &a, &b, &c, &d) == 4) {
        if (a == n && b == dt && c >= 0 && c < psn_host::kScheduleCandidates && d >= 0 &&
            d < psn_host::kScheduleCandidates) {
            *b24 = c;
            *b3 = d;
            found = true;  // the last record of a key wins
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_append(const char* path, int n, int dt, int b24, int b3) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d\n", n, dt, b24, b3);
    std::fclose(f);
}

psn_status tune_schedule(psn_plan* p, hipStream_t s) {
    const char* env = std::getenv("PSN_TUNE");
    if (env && env[0] == '0') return PSN_OK;
    const char* cache = std::getenv("PSN_TUNE_CACHE");
    if (cache && !cache[0]) cache = nullptr;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    const auto key = std::make_pair(p->n, int(p->dtype));
    int b24 = 0, b3 = 0;
    if (cache && tune_cache_lookup(cache, p->n, int(p->dtype), &b24, &b3)) {
        // the recorded choice wins over this process's own timing
        g_tuned[key] = std::make_pair(b24, b3);
    } else {
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            b24 = it->second.first;
            b3 = it->second.second;
        } else {
            hipError_t e = hipErrorInvalidValue;
            switch (p->dtype) {
                case PSN_F64: e = psn_host::tune_f64(p, s, &b24, &b3); break;
                case PSN_F32: e = psn_host::tune_f32(p, s, &b24, &b3); break;
                case PSN_SPLIT: e = psn_host::tune_split(p, s, &b24, &b3); break;
            }
            if (!hip_ok(e, "schedule tuning")) return PSN_EDEVICE;
            g_tuned.emplace(key, std::make_pair(b24, b3));
        }
        if (cache) tune_cache_append(cache, p->n, int(p->dtype), b24, b3);
    }
    p->sched24 = b24;
    p->sched3 = b3;
    p->tuned = true;
    return PSN_OK;
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// HBM bytes one solve must move: five passes, each one read and one write of
// its arrays (io: rho and u, s: complex intermediates per real, k: kernel
// spectrum per real)
double algorithmic_bytes(const psn_plan* p) {
    const double bio = p->dtype == PSN_F32 ? 4 : 8;
    const double bk = p->dtype == PSN_F32 ? 4 : 8;
    if (p->general) {
        // W1 = n0 n1 (n2+1) and W2 = 2 n0 n1 (n2+1) complex (FP64 storage
        // for the FP64-arithmetic precisions), K = (n0+1)(n1+1)(n2+1) reals
        const double bs = p->dtype == PSN_F32 ? 4 : 8;
        const double n0 = p->ng[0], n1 = p->ng[1], n2 = p->ng[2];
        return 2 * bio * n0 * n1 * n2 + 24 * bs * n0 * n1 * (n2 + 1) + bk * (n0 + 1) * (n1 + 1) * (n2 + 1);
    }
    // W1 (n^3 complex) is written and read twice (P1, P2, P4, P5), W2 (2 n^3
    // complex) four times (P2, P3 read and write, P4)
    const double n3 = double(p->n) * p->n * p->n, np1 = p->n + 1.0;
    const double b1 = double(psn_host::w1_bytes(p->dtype)), b2 = double(psn_host::w2_bytes(p->dtype));
    return 2 * bio * n3 + 4 * b1 * n3 + 8 * b2 * n3 + bk * np1 * np1 * np1;
}

// complex workspace elements of a grid with per-axis sizes (rows padded to
// g_pitch(n2) >= n2 + 1 elements)
size_t general_w1(const psn_plan* p) { return size_t(p->ng[0]) * p->ng[1] * psn_host::g_pitch(p->ng[2]); }
size_t general_w2(const psn_plan* p) { return 2 * general_w1(p); }
size_t general_cx(const psn_plan* p) { return p->dtype == PSN_F32 ? 8 : 16; }

size_t slot_bytes(const psn_plan* p) {
    if (p->general) return align256(general_w1(p) * general_cx(p)) + align256(general_w2(p) * general_cx(p));
    const size_t n3 = size_t(p->n) * p->n * p->n;
    const size_t w2 = psn_host::w2_elems(p->n);
    return align256(n3 * psn_host::w1_bytes(p->dtype)) + align256(w2 * psn_host::w2_bytes(p->dtype));
}

psn_host::Slot own_slot(const psn_plan* p, const void* rho, void* u) {
    return psn_host::Slot{p, rho, u, p->W1, p->W2};
}

psn_host::Slot arena_slot(const psn_plan* p, const void* rho, void* u, char* base) {
    const size_t n3 = size_t(p->n) * p->n * p->n;
    psn_host::Slot sl{p, rho, u, nullptr, nullptr};
    if (p->general) {
        sl.W1 = base;
        sl.W2 = base + align256(general_w1(p) * general_cx(p));
        return sl;
    }
    sl.W1 = base;
    sl.W2 = base + align256(n3 * psn_host::w1_bytes(p->dtype));
    return sl;
}

// Per-device state of batched solves: the workspace arena (grown on demand,
// held until the process ends) and the captured graphs keyed by the argument
// list.  Growing the arena synchronises the device.
struct BatchCache {
    void* arena = nullptr;
    size_t arena_bytes = 0;
    hipStream_t capture = nullptr;
    // branch streams and fork/join events of the capture: the (n, precision)
    // groups are spread over at most kBatchChains parallel chains, so the graph
    // lets small groups overlap large ones
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    std::map<std::vector<const void*>, hipGraphExec_t> graphs;
    // schedules timed on batch groups: (n, precision, plan schedule, entries
    // per launch) -> (axis-1 candidate, axis-0 candidate)
    std::map<std::array<int, 5>, std::pair<int, int>> group_sched;
    // A graph may still run on the stream it was launched on (any stream of
    // the caller's), so the device is drained before any is destroyed.
    void clear_graphs() {
        if (graphs.empty()) return;
        (void)hipDeviceSynchronize();
        for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
        graphs.clear();
    }
};
std::mutex g_batch_mutex;
std::map<int, BatchCache> g_batch;
// Parallel chains of a batch graph: the number of hardware queues a process
// gets by default.  A graph with more independent branches than queues runs
// some of them back to back, in an order the runtime picks.
constexpr size_t kBatchChains = 4;

// Workspace of psn_solve_batched_noalloc: a fixed device array, so that call
// makes no allocation.  Host code never passes `scratch` itself to a kernel
// (in host code the name is a host-side stand-in, not a device address); it
// uses the address hipGetSymbolAddress returns, looked up once per device with
// that device current and kept in g_scratch_ptr.  Every call on a device shares
// the array; the passes overwrite every workspace element they later read, so
// nothing needs clearing between calls.
constexpr size_t kScratchBytes = size_t(256) << 20;
constexpr int kNoAllocMaxCount = 1024;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mutex;
std::map<int, void*> g_scratch_ptr;

// Address of this device's scratch array (the current device must be `dev`).
bool scratch_ptr(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress (scratch)")) return false;
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return true;
}

}  // namespace

namespace psn_host {

hipError_t launch_group(const Slot* slots, int count, hipStream_t stream, hipEvent_t* ev, int v24, int v3) {
    if (count <= 0) return hipSuccess;
    if (slots[0].plan->general) {
        // grids with per-axis sizes: the five steps, one entry after the other
        for (int i = 0; i < count; ++i) {
            const hipError_t e = slots[i].plan->dtype == PSN_F32 ? launch_general_f32(slots[i], stream, ev)
                                                                 : launch_general_f64(slots[i], stream, ev);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    switch (slots[0].plan->dtype) {
        case PSN_F64: return launch_group_f64(slots, count, stream, ev, v24, v3);
        case PSN_F32: return launch_group_f32(slots, count, stream, ev, v24, v3);
        case PSN_SPLIT: return launch_group_split(slots, count, stream, ev, v24, v3);
    }
    return hipErrorInvalidValue;
}

hipError_t tune_slots(const Slot* slots, int count, hipStream_t stream, int* best24, int* best3) {
    switch (slots[0].plan->dtype) {
        case PSN_F64: return tune_slots_f64(slots, count, stream, best24, best3);
        case PSN_F32: return tune_slots_f32(slots, count, stream, best24, best3);
        case PSN_SPLIT: return tune_slots_split(slots, count, stream, best24, best3);
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

size_t elem_bytes(psn_dtype dt) { return dt == PSN_F64 ? 16 : 8; }
size_t w1_bytes(psn_dtype dt) { return dt == PSN_F64 ? 16 : dt == PSN_SPLIT ? 12 : 8; }
size_t w2_bytes(psn_dtype dt) { return dt == PSN_F32 ? 8 : 16; }
size_t kernel_elem_bytes(psn_dtype dt) { return dt == PSN_F32 ? 4 : 8; }

}  // namespace psn_host

extern "C" {

int psn_size_supported(int n) {
    return (n >= 4 && n % 2 == 0 && five_smooth(2L * n) && psn_host::size_compiled(n)) ? 1 : 0;
}

psn_status psn_plan_create_grid(const int* n3, const double* a, const double* b, double tol, psn_dtype dtype,
                                psn_plan** out) {
    if (!out) return PSN_EINVAL;
    *out = nullptr;
    if (!n3 || !a || !b || !is_real_dtype(dtype) || !(tol >= 1e-15 && tol <= 1e-4)) return PSN_EINVAL;
    for (int q = 0; q < 3; ++q)
        if (!std::isfinite(a[q]) || !std::isfinite(b[q]) || !(b[q] > a[q])) return PSN_EINVAL;
    for (int q = 0; q < 3; ++q)
        if (!psn_size_supported(n3[q])) return PSN_ESIZE;
    psn_plan* p = new (std::nothrow) psn_plan();
    if (!p) return PSN_ENOMEM;
    p->n = n3[0];
    p->tol = tol;
    p->dtype = dtype;
    p->general = !(n3[0] == n3[1] && n3[1] == n3[2]);
    if (p->general) p->sched24 = p->sched3 = -1;  // the five-step path has no tile schedules
    double lam = 0.0, dmin = 1e300, diag2 = 0.0;
    for (int q = 0; q < 3; ++q) {
        const double w = b[q] - a[q];
        p->ng[q] = n3[q];
        p->a[q] = a[q];
        p->b[q] = b[q];
        p->h[q] = w / (n3[q] - 1);
        p->T[q] = n3[q] * p->h[q];
        p->period[q] = 2.0 * n3[q] * p->h[q];
        lam = std::fmax(lam, 0.5 * w);
        dmin = std::fmin(dmin, w / (50.0 * n3[q]));
        diag2 += w * w;
    }
    p->L = lam;
    // section 3: delta = min_q (b_q - a_q) / (50 n_q) in the standardised
    // frame, at least 1e-3; the physical radius is lambda times that
    p->delta = lam * std::fmax(1e-3, dmin);
    // the Gaussian sum must resolve every distance between two grid points
    p->R = std::sqrt(diag2);
    if (!fit_gaussian_sum(p)) {
        delete p;
        return PSN_EFIT;
    }
    *out = p;
    return PSN_OK;
}

psn_status psn_plan_create_box(int n, const double* a, const double* b, double tol, psn_dtype dtype,
                               psn_plan** out) {
    const int n3[3] = {n, n, n};
    return psn_plan_create_grid(n3, a, b, tol, dtype, out);
}

psn_status psn_plan_create(int n, double L, double tol, psn_dtype dtype, psn_plan** out) {
    if (!out) return PSN_EINVAL;
    *out = nullptr;
    if (!(L > 0) || !std::isfinite(L)) return PSN_EINVAL;
    const double a[3] = {-L, -L, -L}, b[3] = {L, L, L};
    return psn_plan_create_box(n, a, b, tol, dtype, out);
}

psn_status psn_kernel_build(psn_plan* p, void* stream) {
    if (!p) return PSN_EINVAL;
    if (p->built) return PSN_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    g_last_error.clear();
    (void)hipGetLastError();  // drop errors left by unrelated earlier calls
    if (!hip_ok(hipGetDevice(&p->device), "hipGetDevice")) return PSN_EDEVICE;
    const size_t n = p->n, M = 2 * n;
    const size_t kb = psn_host::kernel_elem_bytes(p->dtype);
    size_t tot = 0;
    psn_status st = PSN_OK;
    const size_t cxb = p->dtype == PSN_F32 ? 8 : 16;
    if (p->general) {
        // octant tiled over k2, per-axis twiddle tables of 4 n_q entries,
        // workspaces with padded rows
        const size_t g0 = p->ng[0], g1 = p->ng[1], g2 = p->ng[2];
        if ((st = dev_alloc(&p->K, (g0 + 1) * (g1 + 1) * size_t(psn_host::g_pitch(p->ng[2])) * kb, &tot)) ||
            (st = dev_alloc(&p->Kb, kb, &tot)) || (st = dev_alloc(&p->tw, 4 * (g0 + g1 + g2) * cxb, &tot)) ||
            (st = dev_alloc(&p->W1, general_w1(p) * general_cx(p), &tot)) ||
            (st = dev_alloc(&p->W2, general_w2(p) * general_cx(p), &tot))) {
            free_device(p);
            return st;
        }
    } else if ((st = dev_alloc(&p->K, (n + 1) * (n + 1) * n * kb, &tot)) ||
               (st = dev_alloc(&p->Kb, (n + 1) * (n + 1) * kb, &tot)) || (st = dev_alloc(&p->tw, M * cxb, &tot)) ||
               (st = dev_alloc(&p->W1, n * n * n * psn_host::w1_bytes(p->dtype), &tot)) ||
               (st = dev_alloc(&p->W2, psn_host::w2_elems(p->n) * psn_host::w2_bytes(p->dtype), &tot))) {
        free_device(p);
        return st;
    }
    p->device_bytes = tot;

    // twiddles exp(-2 pi i m / M), evaluated in extended precision, rounded
    // once; a grid with per-axis sizes has one table of 4 n_q entries per axis
    // (the padded length 2 n_q needs exp(-2 pi i m / 4 n_q))
    std::vector<double> twd;
    auto table = [&](size_t len) {
        for (size_t m = 0; m < len; ++m) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)len;
            twd.push_back((double)cosl(a));
            twd.push_back((double)-sinl(a));
        }
    };
    if (p->general) {
        for (int q = 0; q < 3; ++q) table(4 * size_t(p->ng[q]));
    } else {
        table(M);
    }
    const size_t tw_entries = twd.size() / 2;
    std::vector<float> twf;
    const void* twsrc = twd.data();
    if (p->dtype == PSN_F32) {
        twf.assign(twd.begin(), twd.end());
        twsrc = twf.data();
    }
    double glx[16], glw[16];
    gauss_legendre16(glx, glw);
    const int terms = (int)p->tau.size();

    DevBuf d_tau, d_w, d_gl, d_A, d_c;
    if ((st = dev_alloc(&d_tau.p, terms * 8, &tot)) || (st = dev_alloc(&d_w.p, terms * 8, &tot)) ||
        (st = dev_alloc(&d_gl.p, 32 * 8, &tot)) || (st = dev_alloc(&d_A.p,
                                  psn_host::kbuild_scratch_doubles(std::max(p->ng[0], std::max(p->ng[1], p->ng[2])),
                                                                   terms) * 8,
                                  &tot)) ||
        (st = dev_alloc(&d_c.p, 2 * 8, &tot))) {
        free_device(p);
        return st;
    }
    std::vector<double> gl(32);
    std::memcpy(gl.data(), glx, sizeof glx);
    std::memcpy(gl.data() + 16, glw, sizeof glw);
    double cc[2] = {0, 0};
    bool ok = hip_ok(hipMemcpyAsync(p->tw, twsrc, tw_entries * cxb, hipMemcpyHostToDevice, s), "copy twiddles") &&
              hip_ok(hipMemcpyAsync(d_tau.p, p->tau.data(), terms * 8, hipMemcpyHostToDevice, s), "copy tau") &&
              hip_ok(hipMemcpyAsync(d_w.p, p->w.data(), terms * 8, hipMemcpyHostToDevice, s), "copy w") &&
              hip_ok(hipMemcpyAsync(d_gl.p, gl.data(), 32 * 8, hipMemcpyHostToDevice, s), "copy nodes");
    ok = ok && hip_ok(psn_host::launch_kernel_build(p, static_cast<double*>(d_tau.p), static_cast<double*>(d_w.p),
                                                    terms, static_cast<double*>(d_gl.p),
                                                    static_cast<double*>(d_gl.p) + 16, static_cast<double*>(d_A.p),
                                                    static_cast<double*>(d_c.p), s),
                      "kernel-spectrum launch");
    ok = ok && hip_ok(hipMemcpyAsync(cc, d_c.p, sizeof cc, hipMemcpyDeviceToHost, s), "copy C0/C2");
    ok = ok && hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (!ok) {
        free_device(p);
        return PSN_EDEVICE;
    }
    p->C0 = cc[0];
    p->C2 = cc[1];
    void* sp = nullptr;
    if (!scratch_ptr(p->device, &sp)) {  // set-up of the no-allocation batch entry point on this device
        free_device(p);
        return PSN_EDEVICE;
    }
    p->built = true;
    if (p->general) return PSN_OK;  // no tile schedules on the five-step path
    return tune_schedule(p, s);
}

psn_status psn_solve(psn_plan* p, const void* rho, void* u, void* stream) {
    if (!p || !rho || !u) return PSN_EINVAL;
    if (!p->built) return PSN_ESTATE;
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return PSN_EDEVICE;
    if (dev != p->device) return PSN_EINVAL;
    (void)hipGetLastError();
    const psn_host::Slot sl = own_slot(p, rho, u);
    if (!hip_ok(psn_host::launch_group(&sl, 1, static_cast<hipStream_t>(stream)), "solve launch"))
        return PSN_EDEVICE;
    return PSN_OK;
}

psn_status psn_solve_timed(psn_plan* p, const void* rho, void* u, void* stream, double* pass_ms) {
    if (!p || !rho || !u || !pass_ms) return PSN_EINVAL;
    if (!p->built) return PSN_ESTATE;
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return PSN_EDEVICE;
    if (dev != p->device) return PSN_EINVAL;
    (void)hipGetLastError();
    hipEvent_t ev[6] = {};
    for (auto& e : ev)
        if (!hip_ok(hipEventCreate(&e), "hipEventCreate")) {
            for (auto& f : ev)
                if (f) (void)hipEventDestroy(f);
            return PSN_EDEVICE;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const psn_host::Slot sl = own_slot(p, rho, u);
    bool ok = hip_ok(psn_host::launch_group(&sl, 1, s, ev), "solve launch") &&
              hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int i = 0; ok && i < 5; ++i) {
        float ms = 0.f;
        ok = hip_ok(hipEventElapsedTime(&ms, ev[i], ev[i + 1]), "hipEventElapsedTime");
        pass_ms[i] = ms;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return ok ? PSN_OK : PSN_EDEVICE;
}

psn_status psn_solve_batched(int count, psn_plan* const* plans, const void* const* rho, void* const* u,
                             void* stream) {
    if (count < 0 || (count > 0 && (!plans || !rho || !u))) return PSN_EINVAL;
    int dev = -1;
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !rho[i] || !u[i]) return PSN_EINVAL;
        if (!plans[i]->built) return PSN_ESTATE;
    }
    if (count == 0) return PSN_OK;
    g_last_error.clear();
    (void)hipGetLastError();
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return PSN_EDEVICE;
    for (int i = 0; i < count; ++i)
        if (plans[i]->device != dev) return PSN_EINVAL;
    std::lock_guard<std::mutex> lock(g_batch_mutex);
    BatchCache& bc = g_batch[dev];

    // workspace: one region per entry in the device's batch arena
    std::vector<size_t> off(count);
    size_t need = 0;
    for (int i = 0; i < count; ++i) {
        off[i] = need;
        need += slot_bytes(plans[i]);
    }
    if (need > bc.arena_bytes) {
        // the old arena may still be in use by earlier batches on any stream
        if (bc.arena && !hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize")) return PSN_EDEVICE;
        bc.clear_graphs();
        if (bc.arena) (void)hipFree(bc.arena);
        bc.arena = nullptr;
        bc.arena_bytes = 0;
        if (!hip_ok(hipMalloc(&bc.arena, need), "hipMalloc (batch arena)")) return PSN_ENOMEM;
        bc.arena_bytes = need;
    }

    // the launch sequence is captured once per argument list and schedule set
    // and replayed; a plan's schedule is fixed in the graph at capture
    std::vector<const void*> key;
    key.reserve(4 * count);
    for (int i = 0; i < count; ++i) {
        key.push_back(plans[i]);
        key.push_back(rho[i]);
        key.push_back(u[i]);
        key.push_back(reinterpret_cast<const void*>(
            static_cast<uintptr_t>(plans[i]->sched24 * psn_host::kScheduleCandidates + plans[i]->sched3)));
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    auto it = bc.graphs.find(key);
    if (it == bc.graphs.end()) {
        // group entries by (n, precision, schedule), keeping the order within a
        // group: a group shares each launch, so its entries share one schedule
        std::map<std::array<int, 4>, std::vector<psn_host::Slot>> groups;
        for (int i = 0; i < count; ++i) {
            const psn_plan* p = plans[i];
            groups[{p->n, int(p->dtype), p->sched24, p->sched3}].push_back(
                arena_slot(p, rho[i], u[i], static_cast<char*>(bc.arena) + off[i]));
        }
        // Chains: groups in decreasing order of HBM bytes, each appended to the
        // chain with the fewest bytes so far (longest-first list scheduling),
        // so the largest group starts at once and small ones share a chain.
        std::vector<std::pair<double, const std::vector<psn_host::Slot>*>> order;
        for (auto& g : groups)
            order.push_back({algorithmic_bytes(g.second.front().plan) * double(g.second.size()), &g.second});
        std::stable_sort(order.begin(), order.end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        const size_t nchain = std::min(order.size(), kBatchChains);
        std::vector<std::vector<const std::vector<psn_host::Slot>*>> chains(nchain);
        std::vector<double> load(nchain, 0.0);
        for (auto& o : order) {
            const size_t c = size_t(std::min_element(load.begin(), load.end()) - load.begin());
            chains[c].push_back(o.second);
            load[c] += o.first;
        }
        // Several entries sharing a launch run best under the schedule timed on
        // such a launch, which can differ from the single-solve choice: a
        // group of autotuned plans is timed once on its own arena entries (on
        // the caller's stream, after the work already queued there).  Off
        // with PSN_TUNE=0 or a PSN_TUNE_CACHE file (whose choices are kept).
        std::map<const std::vector<psn_host::Slot>*, std::pair<int, int>> gsched;
        {
            const char* env = std::getenv("PSN_TUNE");
            const char* cache = std::getenv("PSN_TUNE_CACHE");
            const bool tune = !(env && env[0] == '0') && !(cache && cache[0]);
            for (auto& g : groups) {
                const psn_plan* p0 = g.second.front().plan;
                bool all_tuned = g.second.size() >= 2;
                for (const auto& sl : g.second) all_tuned = all_tuned && sl.plan->tuned;
                if (!tune || !all_tuned) continue;
                const int per_launch = int(std::min<size_t>(g.second.size(), size_t(psn::kMaxBatchHost)));
                const std::array<int, 5> gk{p0->n, int(p0->dtype), p0->sched24, p0->sched3, per_launch};
                auto gi = bc.group_sched.find(gk);
                if (gi == bc.group_sched.end()) {
                    int b24 = 0, b3 = 0;
                    if (!hip_ok(psn_host::tune_slots(g.second.data(), int(g.second.size()), s, &b24, &b3),
                                "batch schedule tuning"))
                        return PSN_EDEVICE;
                    gi = bc.group_sched.emplace(gk, std::make_pair(b24, b3)).first;
                }
                gsched[&g.second] = gi->second;
            }
        }
        if (!bc.capture && !hip_ok(hipStreamCreateWithFlags(&bc.capture, hipStreamNonBlocking), "hipStreamCreate"))
            return PSN_EDEVICE;
        if (!bc.fork && !hip_ok(hipEventCreateWithFlags(&bc.fork, hipEventDisableTiming), "hipEventCreate"))
            return PSN_EDEVICE;
        const size_t nb = nchain - 1;  // the first chain stays on the capture stream
        while (bc.branch.size() < nb) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            if (!hip_ok(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate")) return PSN_EDEVICE;
            if (!hip_ok(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate")) {
                (void)hipStreamDestroy(st);
                return PSN_EDEVICE;
            }
            bc.branch.push_back(st);
            bc.join.push_back(ev);
        }
        if (!hip_ok(hipStreamBeginCapture(bc.capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture"))
            return PSN_EDEVICE;
        hipError_t le = hipEventRecord(bc.fork, bc.capture);
        // chains 1.. fork from the capture stream first, so that every chain
        // starts at the head of the graph
        for (size_t ci = 1; ci < nchain && le == hipSuccess; ++ci) le = hipStreamWaitEvent(bc.branch[ci - 1], bc.fork, 0);
        for (size_t ci = 0; ci < nchain && le == hipSuccess; ++ci) {
            hipStream_t st = ci == 0 ? bc.capture : bc.branch[ci - 1];
            for (const auto* g : chains[ci]) {
                if (le != hipSuccess) break;
                const auto gs = gsched.find(g);
                le = gs == gsched.end() ? psn_host::launch_group(g->data(), int(g->size()), st)
                                        : psn_host::launch_group(g->data(), int(g->size()), st, nullptr,
                                                                 gs->second.first, gs->second.second);
            }
        }
        for (size_t ci = 1; ci < nchain && le == hipSuccess; ++ci) {
            le = hipEventRecord(bc.join[ci - 1], bc.branch[ci - 1]);
            if (le == hipSuccess) le = hipStreamWaitEvent(bc.capture, bc.join[ci - 1], 0);
        }
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(bc.capture, &graph);
        if (!hip_ok(le, "batch launch (capture)") || !hip_ok(ee, "hipStreamEndCapture")) {
            if (graph) (void)hipGraphDestroy(graph);
            return PSN_EDEVICE;
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (!hip_ok(ie, "hipGraphInstantiate")) return PSN_EDEVICE;
        if (bc.graphs.size() >= 16) bc.clear_graphs();
        it = bc.graphs.emplace(key, exec).first;
    }
    if (!hip_ok(hipGraphLaunch(it->second, s), "hipGraphLaunch")) return PSN_EDEVICE;
    return PSN_OK;
}

psn_status psn_solve_batched_noalloc(int count, psn_plan* const* plans, const void* const* rho, void* const* u,
                                    void* stream) {
    if (count < 0 || (count > 0 && (!plans || !rho || !u))) return PSN_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !rho[i] || !u[i]) return PSN_EINVAL;
        if (!plans[i]->built) return PSN_ESTATE;
    }
    g_last_error.clear();
    if (count == 0) return PSN_OK;
    if (count > kNoAllocMaxCount) {
        g_last_error = "psn_solve_batched_noalloc: " + std::to_string(count) + " entries, at most " +
                       std::to_string(kNoAllocMaxCount);
        return PSN_ELIMIT;
    }
    (void)hipGetLastError();
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return PSN_EDEVICE;
    size_t need = 0;
    for (int i = 0; i < count; ++i) {
        if (plans[i]->device != dev) return PSN_EINVAL;
        need += slot_bytes(plans[i]);
    }
    if (need > kScratchBytes) {
        g_last_error = "psn_solve_batched_noalloc: the batch needs " + std::to_string(need) +
                       " workspace bytes, the fixed scratch area holds " + std::to_string(kScratchBytes);
        return PSN_ELIMIT;
    }
    void* base = nullptr;
    if (!scratch_ptr(dev, &base)) return PSN_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // Entry i's workspace starts at the sum of the earlier entries' sizes.
    // Entries sharing (n, precision, schedule) share each launch; the groups
    // run one after another on `stream`, found by repeated scans (no host or
    // device allocation).
    bool done[kNoAllocMaxCount] = {};
    psn_host::Slot group[psn::kMaxBatchHost];
    for (int i = 0; i < count; ++i) {
        if (done[i]) continue;
        const psn_plan* p0 = plans[i];
        // the schedule a batched call timed for such a group, if any (lookup only)
        int gsize = 0;
        for (int j = i; j < count; ++j) {
            const psn_plan* pj = plans[j];
            gsize += (!done[j] && pj->n == p0->n && pj->dtype == p0->dtype && pj->sched24 == p0->sched24 &&
                      pj->sched3 == p0->sched3)
                         ? 1
                         : 0;
        }
        int v24 = -1, v3 = -1;
        {
            std::lock_guard<std::mutex> lock(g_batch_mutex);
            auto bi = g_batch.find(dev);
            if (bi != g_batch.end()) {
                const std::array<int, 5> gk{p0->n, int(p0->dtype), p0->sched24, p0->sched3,
                                            std::min(gsize, psn::kMaxBatchHost)};
                auto gi = bi->second.group_sched.find(gk);
                if (gi != bi->second.group_sched.end()) {
                    v24 = gi->second.first;
                    v3 = gi->second.second;
                }
            }
        }
        size_t off = 0;
        int g = 0;
        for (int j = 0; j < count; ++j) {
            const psn_plan* pj = plans[j];
            if (j >= i && !done[j] && pj->n == p0->n && pj->dtype == p0->dtype && pj->sched24 == p0->sched24 &&
                pj->sched3 == p0->sched3) {
                group[g++] = arena_slot(pj, rho[j], u[j], static_cast<char*>(base) + off);
                done[j] = true;
                if (g == psn::kMaxBatchHost) {
                    if (!hip_ok(psn_host::launch_group(group, g, s, nullptr, v24, v3), "batch launch"))
                        return PSN_EDEVICE;
                    g = 0;
                }
            }
            off += slot_bytes(pj);
        }
        if (g > 0 && !hip_ok(psn_host::launch_group(group, g, s, nullptr, v24, v3), "batch launch"))
            return PSN_EDEVICE;
    }
    return PSN_OK;
}

psn_status psn_plan_query(const psn_plan* p, psn_plan_info* info) {
    if (!p || !info) return PSN_EINVAL;
    std::memset(info, 0, sizeof *info);
    info->n = p->n;
    info->dtype = p->dtype;
    info->L = p->L;
    info->tol = p->tol;
    info->h = p->h[0];
    info->T = p->T[0];
    info->period = p->period[0];
    info->schedule[0] = p->sched24;
    info->schedule[1] = p->sched3;
    info->tuned = p->tuned ? 1 : 0;
    info->device = p->built ? p->device : -1;
    info->correction = p->correction;
    for (int q = 0; q < 3; ++q) info->n3[q] = p->ng[q];
    for (int q = 0; q < 3; ++q) {
        info->a[q] = p->a[q];
        info->b[q] = p->b[q];
        info->h3[q] = p->h[q];
        info->T3[q] = p->T[q];
    }
    info->delta = p->delta;
    info->R = p->R;
    info->hs = p->hs;
    info->terms = (int)p->tau.size();
    info->eps_achieved = p->gs_err;
    info->C0 = p->C0;
    info->C2 = p->C2;
    info->built = p->built ? 1 : 0;
    info->device_bytes = p->device_bytes;
    info->algorithmic_bytes = algorithmic_bytes(p);
    return PSN_OK;
}

psn_status psn_plan_set_correction(psn_plan* p, int mode) {
    if (!p || (mode != PSN_CORRECTION_FOLDED && mode != PSN_CORRECTION_FOURIER)) return PSN_EINVAL;
    if (p->general && mode != PSN_CORRECTION_FOLDED) return PSN_EINVAL;
    if (p->built) return PSN_ESTATE;
    p->correction = mode;
    return PSN_OK;
}

psn_status psn_plan_set_schedule(psn_plan* p, int p24, int p3) {
    if (!p || p->general || p24 < 0 || p24 >= psn_host::kScheduleCandidates || p3 < 0 ||
        p3 >= psn_host::kScheduleCandidates)
        return PSN_EINVAL;
    p->sched24 = p24;
    p->sched3 = p3;
    p->tuned = false;
    return PSN_OK;
}

psn_status psn_plan_gs_table(const psn_plan* p, double* tau, double* w, int cap, int* terms) {
    if (!p || !terms || cap < 0 || (cap > 0 && (!tau || !w))) return PSN_EINVAL;
    const int m = (int)p->tau.size();
    *terms = m;
    for (int i = 0; i < m && i < cap; ++i) {
        tau[i] = p->tau[i];
        w[i] = p->w[i];
    }
    return PSN_OK;
}

psn_status psn_kernel_download(const psn_plan* p, double* octant) {
    if (!p || !octant) return PSN_EINVAL;
    if (!p->built) return PSN_ESTATE;
    if (p->general) {
        const int g0 = p->ng[0], g1 = p->ng[1], g2 = p->ng[2];
        const size_t kb = psn_host::kernel_elem_bytes(p->dtype);
        std::vector<unsigned char> hk(size_t(g0 + 1) * (g1 + 1) * size_t(psn_host::g_pitch(g2)) * kb);
        if (!hip_ok(hipMemcpy(hk.data(), p->K, hk.size(), hipMemcpyDeviceToHost), "copy K")) return PSN_EDEVICE;
        const double inv = 8.0 * double(g0) * g1 * g2;
        size_t i = 0;  // plain [k0][k1][k2] order
        for (int k0 = 0; k0 <= g0; ++k0)
            for (int k1 = 0; k1 <= g1; ++k1)
                for (int k2 = 0; k2 <= g2; ++k2, ++i) {
                    const size_t j = psn_host::g_k_index(g0, g2, k0, k1, k2);
                    octant[i] = (kb == 4 ? (double)reinterpret_cast<const float*>(hk.data())[j]
                                         : reinterpret_cast<const double*>(hk.data())[j]) * inv;
                }
        return PSN_OK;
    }
    const size_t n = p->n, np1 = n + 1;
    const size_t kb = psn_host::kernel_elem_bytes(p->dtype);
    std::vector<unsigned char> hk(np1 * np1 * n * kb), hb(np1 * np1 * kb);
    if (!hip_ok(hipMemcpy(hk.data(), p->K, hk.size(), hipMemcpyDeviceToHost), "copy K") ||
        !hip_ok(hipMemcpy(hb.data(), p->Kb, hb.size(), hipMemcpyDeviceToHost), "copy Kb"))
        return PSN_EDEVICE;
    auto get = [&](const std::vector<unsigned char>& v, size_t i) -> double {
        if (kb == 4) return (double)reinterpret_cast<const float*>(v.data())[i];
        return reinterpret_cast<const double*>(v.data())[i];
    };
    const double M = 2.0 * n, inv = M * M * M;
    for (size_t a = 0; a < np1; ++a)
        for (size_t b = 0; b < np1; ++b) {
            double* dst = octant + (a * np1 + b) * np1;
            const double al = get(hk, psn_host::k_index(int(n), int(b), int(a), 0)), be = get(hb, b * np1 + a);
            dst[0] = (al + be) * inv;
            dst[n] = (al - be) * inv;
            for (size_t c = 1; c < n; ++c) dst[c] = get(hk, psn_host::k_index(int(n), int(b), int(a), int(c))) * inv;
        }
    return PSN_OK;
}

void psn_plan_destroy(psn_plan* p) {
    if (!p) return;
    {
        // captured batches that reference this plan's device arrays go too
        std::lock_guard<std::mutex> lock(g_batch_mutex);
        for (auto& dc : g_batch)
            for (auto it = dc.second.graphs.begin(); it != dc.second.graphs.end();) {
                bool uses = false;
                for (size_t i = 0; i < it->first.size(); i += 4) uses |= it->first[i] == p;
                if (uses) {
                    // the graph may still be running on the caller's stream
                    (void)hipDeviceSynchronize();
                    (void)hipGraphExecDestroy(it->second);
                    it = dc.second.graphs.erase(it);
                } else {
                    ++it;
                }
            }
    }
    free_device(p);
    delete p;
}

const char* psn_last_error(void) { return g_last_error.c_str(); }

const char* psn_strerror(psn_status st) {
    switch (st) {
        case PSN_OK: return "success";
        case PSN_EINVAL: return "invalid argument";
        case PSN_ESIZE: return "unsupported grid size (n must be even, 2n 5-smooth, and compiled in)";
        case PSN_ENOMEM: return "device allocation failed";
        case PSN_EDEVICE: return "HIP call or kernel launch failed";
        case PSN_ESTATE: return "kernel spectrum not built";
        case PSN_EFIT: return "Gaussian-sum fit missed the tolerance";
        case PSN_ELIMIT: return "request exceeds a fixed limit of the no-allocation entry point";
    }
    return "unknown status";
}

}  // extern "C"
