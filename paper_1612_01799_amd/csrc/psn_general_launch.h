// Launch sequence of the five-step solve on a grid with per-axis sizes.
#pragma once

#include "psn_general.h"
#include "psn_internal.h"

namespace psn {

template <class Real, class Io>
hipError_t general_solve(const psn_host::Slot& sl, hipStream_t s, hipEvent_t* ev) {
    const psn_plan* p = sl.plan;
    const int n0 = p->ng[0], n1 = p->ng[1], n2 = p->ng[2];
    GArgs<Real, Io> a{static_cast<const Io*>(sl.rho), static_cast<Io*>(sl.u), static_cast<cx<Real>*>(sl.W1),
                      static_cast<cx<Real>*>(sl.W2), static_cast<const Real*>(p->K), nullptr, n0, n1, n2,
                      psn_host::w2_k1_block(n1), 0};
    while ((1 << a.kbs) < a.kb) ++a.kbs;
    // twiddle tables exp(-2 pi i m / 4 n_q), m < 4 n_q, one after the other
    const cx<Real>* tw = static_cast<const cx<Real>*>(p->tw);
    const cx<Real>* tw0 = tw;
    const cx<Real>* tw1 = tw + 4 * n0;
    const cx<Real>* tw2 = tw + 4 * n0 + 4 * n1;
    const long hw = psn_host::g_pitch(n2);  // workspace row: n2 + 1 spectrum entries, padded
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    };
    hipError_t e;
    mark(0);
    a.tw = tw2;
    if ((e = g_step_n<Real, Io, 1>(n2, a, long(n0) * n1, s)) != hipSuccess) return e;
    mark(1);
    a.tw = tw1;
    if ((e = g_step_n<Real, Io, 2>(n1, a, long(n0) * hw, s)) != hipSuccess) return e;
    mark(2);
    a.tw = tw0;
    if ((e = g_step_n<Real, Io, 3>(n0, a, 2L * n1 * hw, s)) != hipSuccess) return e;
    mark(3);
    a.tw = tw1;
    if ((e = g_step_n<Real, Io, 4>(n1, a, long(n0) * hw, s)) != hipSuccess) return e;
    mark(4);
    a.tw = tw2;
    if ((e = g_step_n<Real, Io, 5>(n2, a, long(n0) * n1, s)) != hipSuccess) return e;
    mark(5);
    return hipGetLastError();
}

}  // namespace psn

#define PSN_DEFINE_GENERAL(REAL, IO, SUFFIX)                                                                   \
    namespace psn_host {                                                                                       \
    hipError_t launch_general_##SUFFIX(const Slot& sl, hipStream_t stream, hipEvent_t* ev) {                  \
        return psn::general_solve<REAL, IO>(sl, stream, ev);                                                   \
    }                                                                                                          \
    }
