// Step ranges of the resident cylindrical / k_z kernels: a run may be cut
// into parts (launches) that resume from the fields in memory, so that the
// time-convergence stop can look at the partial force between them.
#pragma once

#include "device.hpp"

namespace cf {

// Steps of one launch per order: [s0[m], s1[m]) of RedOrders::steps[m].  A
// launch with s0[m] = 0 clears, kicks and starts the channel; a later one
// resumes from the fields its predecessor left in memory.
struct RedSpan {
    int s0[kMaxOrders];
    int s1[kMaxOrders];
};

// Steps of order m after d of the run's base steps (n_steps = base): all of
// them at d = base, else d * steps[m] / base rounded down (the same physical
// time to within one step of each order).
inline int red_step_at(const RedOrders& o, int m, int d, int base) {
    return d >= base ? o.steps[m] : (int)((int64_t)d * o.steps[m] / base);
}

// The part [d0, d1) of a run of `base` steps, for orders 0..n_ord-1.
inline RedSpan red_span(const RedOrders& o, int n_ord, int d0, int d1, int base) {
    RedSpan sp{};
    for (int m = 0; m < n_ord && m < kMaxOrders; ++m) {
        sp.s0[m] = red_step_at(o, m, d0, base);
        sp.s1[m] = red_step_at(o, m, d1, base);
    }
    return sp;
}

// launch_red_resident for the steps of `span` only.
template <typename T>
hipError_t launch_red_resident_span(int variant, T* fields, const ChanDev* ch, const int* slots, int nslots,
                                    const Grid2D& g, const RedOrders& ord, const RedSpan& span, const SurfTables& t,
                                    double dA, double* acc, double* gamma, int gamma_stride, hipStream_t s,
                                    int* used);

}  // namespace cf
