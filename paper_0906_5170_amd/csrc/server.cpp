// Serving: continuous batching of force-solve requests on one GPU.
//
// A scheduler thread owns a device arena (the HBM budget).  Requests wait in
// arrival order; at every tick boundary each queued request whose memory fits
// is admitted (later requests may pass an earlier one that does not fit yet):
// its tables are uploaded, its fields zeroed and kicked, and it joins the
// resident set.  A tick advances the resident requests:
//   - all 2D requests whose stress surface fits a fused tile share one fused
//     launch per polarization and advance K steps per tick (each instance
//     reads its own buffers, tables and K(t) and starts at its own step of
//     the scheduler clock);
//   - other requests (3D on the fused z-streaming step, or split kernels
//     for surfaces wider than a tile) run one after another, in channel
//     waves that bound their memory, each with its own step count.  Each
//     gets an equal share of the tick's device time, the share of one
//     fused request, as steps from its measured time per step.  A cheap 2D
//     request is thus not held to the pace of a 3D cell many times its
//     size (processor sharing in time rather than in steps);
//   - cylindrical and k_z requests (whose kernels run every step of a
//     channel in one launch) run their whole solve in one tick, on their
//     arena region and the server's stream.
// When a request has run all its steps its accumulators are copied back,
// its memory returns to the arena and waiting requests can enter.  Every
// request's arithmetic is independent of its co-residents, so a result is
// bitwise the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/casimir_fdtd.h"
#include "arena.hpp"
#include "device.hpp"
#include "plan.hpp"
#include "solver.hpp"

struct cf_problem {
    cf::Problem p;
};

namespace {

using cfi::fail;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

enum { ST_QUEUED = 0, ST_RUNNING = 1, ST_DONE = 2, ST_FAILED = 3, ST_CANCELLED = 4 };

struct Req {
    uint64_t ticket = 0;
    cf::Problem own;                  // the request's copy of the submitted problem
    const cf::Problem* prob = nullptr;   // == &own
    cf_opts opts{};
    std::vector<cf::Channel> chans;
    cfi::Staged st;
    bool fused = false;
    int variant = -1;                 // fused variant of this request
    int v3 = -1;                      // fused 3D step variant (-1: split 3D kernels)
    int v3s = -1;                     // its single-step band shape (a step without a partner in the tick)
    cfi::ConvergenceStop conv;        // time-convergence stop (single-wave requests)
    int steps_run = -1;
    int par = 0;                      // fused 3D: field array holding the current step
    int C = 0;
    size_t bytes = 0, off = 0;
    size_t o_ids, o_lut, o_ktab, o_pml, o_ch, o_slots, o_gidx, o_gw, o_uidx, o_uoff, o_usamp, o_uw, o_basis,
        o_acc, o_fa, o_fb, o_psi, o_psi2, o_idp, o_shadow, o_zr;
    std::vector<uint32_t> idp;        // fused 3D: packed material ids
    std::vector<uint8_t> ids;
    std::vector<uint8_t> lut;     // field-precision bytes
    std::vector<double> ktab, pml;
    int wave = 0;
    long long start = 0;          // fused: clock step of the current wave's step 0
    // non-fused requests keep their own step count and advance by a share of
    // device time per tick (see plan_steps)
    long long done = 0;           // steps of the current wave run
    int tick_steps = 0;           // steps in the coming tick
    double credit = 0;            // step credit carried between ticks
    double sps = 0;               // measured device seconds per step
    // cylindrical and k_z requests run as one cf_solve on their arena region
    // (their kernels take every step of a channel in one launch)
    bool whole = false;
    bool ran = false;
    std::unique_ptr<cf_problem> handle;
    std::vector<double> w_ph, w_pf, w_pc;
    cf_result w_res{};
    int state = ST_QUEUED;
    cf_status status = CF_OK;
    std::string err;
    std::vector<double> acc;
    double t_submit = 0, t_admit = 0, t_done = 0;
    bool cancel = false;
};

// A request that has reached a terminal state keeps only what its result
// needs (faces, grid, channel table, tile shapes): the copied material ids,
// interpolation tables and upload staging go.
void drop_tables(Req& r) {
    for (auto& v : r.own.ids) std::vector<uint8_t>().swap(v);
    std::vector<cf::Gather>().swap(r.own.gathers);
    r.own.gather_of.clear();
    std::vector<uint32_t>().swap(r.idp);
    std::vector<uint8_t>().swap(r.ids);
    std::vector<uint8_t>().swap(r.lut);
    std::vector<double>().swap(r.ktab);
    std::vector<double>().swap(r.pml);
    std::vector<int32_t>().swap(r.st.gidx);
    std::vector<int32_t>().swap(r.st.uidx);
    std::vector<int32_t>().swap(r.st.uoff);
    std::vector<int32_t>().swap(r.st.usamp);
    std::vector<double>().swap(r.st.gw);
    std::vector<double>().swap(r.st.uw);
    std::vector<double>().swap(r.st.basis);
    std::vector<cf::ChanDev>().swap(r.st.dev);
}

}  // namespace

struct cf_server {
    std::mutex mu;
    std::condition_variable cv;       // new work / completions
    std::thread worker;
    bool stop = false;
    int device = 0;
    int precision = CF_FP32;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char* arena_base = nullptr;
    bool own_arena = false;
    cfi::Arena arena;
    std::deque<std::shared_ptr<Req>> queue;
    std::vector<std::shared_ptr<Req>> active;
    std::map<uint64_t, std::shared_ptr<Req>> all;
    uint64_t next_ticket = 1;
    long long clock = 0;
    int parity = 0;
    int kh = 8;                       // steps per tick
    std::vector<int> prefer;          // fused variants in order of preference (same steps per launch)
    // fused group tables (server-owned device memory)
    char* group = nullptr;
    size_t group_bytes = 0, g_ch = 0, g_inst = 0, g_work = 0;
    size_t cap_ch = 0, cap_inst = 0, cap_work = 0;
    bool membership_changed = true;
    struct Launch {
        int variant, pol;
        size_t off;                   // first work item in the concatenated lists
        int n;
    };
    std::vector<Launch> launches;     // fused launches of one tick
    // tick timing: events around the fused launches and each non-fused
    // request's steps, and the fused launches' device time last tick
    std::vector<hipEvent_t> ev;
    size_t n_marks = 0;
    double group_s = 0;
    // second stream for the TE launches of the fused group (forked from and
    // joined back to the server's stream every tick); default priority
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::deque<std::vector<cf::ChanDev>> keep_ch;
    std::deque<std::vector<cf::InstDev>> keep_inst;
    std::deque<std::vector<cf::WorkItem>> keep_work;
    // statistics
    uint64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_cancelled = 0;
    double busy_s = 0;
    std::string thread_error;
};

namespace {

// Bytes of one request region and the offsets inside it.
void layout_request(const cf_server* S, Req& r) {
    const cf::Problem& p = *r.prob;
    const size_t fsz = S->precision == CF_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = cfi::align_up(off + bytes, 256);
        return at;
    };
    const cfi::Staged& st = r.st;
    r.o_ids = take((size_t)cf::kNumComp * p.ncell);
    r.o_lut = take(2 * cf::kNumComp * 256 * 2 * fsz);
    r.o_ktab = take((size_t)r.opts.n_steps * 8);
    r.o_pml = take((size_t)4 * p.nz * 8);
    r.o_ch = take(st.dev.size() * sizeof(cf::ChanDev));
    r.o_slots = take(st.slot_lists.size() * sizeof(int) + 4);
    r.o_gidx = take(st.gidx.size() * 4 + 4);
    r.o_gw = take(st.gw.size() * 8 + 8);
    r.o_uidx = take(st.uidx.size() * 4 + 4);
    r.o_uoff = take(st.uoff.size() * 4 + 4);
    r.o_usamp = take(st.usamp.size() * 4 + 4);
    r.o_uw = take(st.uw.size() * 8 + 8);
    r.o_basis = take(st.basis.size() * 8 + 8);
    r.o_acc = take((size_t)r.C * 2 * 8);
    const size_t block = (size_t)st.resident * st.ncomp * p.ncell * fsz;
    r.o_fa = take(block);
    const bool f3 = r.v3 >= 0;
    r.o_fb = r.fused || f3 ? take(block) : off;
    r.o_psi = st.psi_comp > 0 ? take((size_t)st.resident * 4 * st.psi_comp * fsz) : off;
    r.o_psi2 = st.psi_comp > 0 && f3 ? take((size_t)st.resident * 4 * st.psi_comp * fsz) : off;
    r.o_idp = f3 ? take((size_t)p.ncell * 8) : off;
    r.o_shadow = f3 && cf::f3d_steps(r.v3) == 2 ? take((size_t)st.resident * st.sbox.vol * fsz) : off;
    r.o_zr = f3 && !st.zr.empty() ? take(st.zr.size() * 4 + 8) : off;
    r.bytes = off;
}

// Stage a request: channels, tables; decide fused vs split; pick the channel
// wave size so the request fits the budget.  Returns "" or an error.
std::string prepare(cf_server* S, Req& r) {
    const cf::Problem& p = *r.prob;
    r.chans = cf::channel_table(p, r.opts.pol);
    r.C = (int)r.chans.size();
    cf_opts o = r.opts;
    o.n_subset = 0;
    o.channel_subset = nullptr;
    o.path = CF_PATH_BATCHED;
    o.flags &= ~(CF_FLAG_KEEP_GAMMA | CF_FLAG_TIME_STENCIL);
    o.max_resident = 0;
    cfi::stage(p, o, r.chans, r.st);
    r.variant = -1;
    if (p.grid.ndim == 2)
        for (int v : S->prefer)
            if (v < (int)r.st.plans.size() && r.st.plans[v].ok && r.st.shapes[v].kh == S->kh) {
                r.variant = v;
                break;
            }
    r.fused = r.variant >= 0;
    // 3D requests take the fused z-streaming step when it applies: in FP32
    // the two-step kernel (12 waves of 1 row; steps go in pairs within a clock
    // tick), else the single-step band shape of 8 waves of 1 row, else the
    // first usable one
    r.v3 = -1;
    if (p.grid.ndim == 3 && r.st.f3d) {
        cf::Grid3D g{};
        g.nx = p.nx;
        g.ny = p.ny;
        g.nz = p.nz;
        for (int a = 0; a < 3; ++a) g.per[a] = p.grid.bc[a] == CF_BC_PERIODIC;
        g.pml = p.grid.bc[2] == CF_BC_PML ? p.grid.pml_cells[2] : 0;
        auto usable = [&](int v) {
            return S->precision == CF_FP64 ? cf::f3d_usable<double>(v, g) : cf::f3d_usable<float>(v, g);
        };
        const int pref2 = 5, pref = 2;
        if (S->precision != CF_FP64 && usable(pref2) && r.st.sbox.vol > 0) r.v3 = pref2;
        if (r.v3 < 0 && usable(pref)) r.v3 = pref;
        for (int v = 0; v < cf::f3d_variants() && r.v3 < 0; ++v)
            if (usable(v) && cf::f3d_steps(v) == 1) r.v3 = v;
        r.v3s = r.v3 >= 0 && cf::f3d_steps(r.v3) == 2 ? cf::f3d_single(r.v3) : r.v3;
    }
    int R = r.opts.max_resident > 0 ? std::min(r.opts.max_resident, r.C) : r.C;
    if (r.fused) R = r.C;   // fused requests keep every channel resident
    for (;;) {
        if (R != r.st.resident) {
            o.max_resident = R;
            r.st = cfi::Staged();
            cfi::stage(p, o, r.chans, r.st);
        }
        layout_request(S, r);
        if (r.bytes <= S->arena.size() || R == 1 || r.fused) break;
        R = std::max(1, R / 2);
    }
    if (r.bytes > S->arena.size()) return "request larger than the server's memory budget";
    r.conv.on = r.opts.stop_tol > 0 && r.st.waves.size() == 1;
    r.conv.tol = r.opts.stop_tol;
    r.conv.every = r.conv.next = r.opts.stop_every > 0 ? r.opts.stop_every : 500;
    // host copies of the per-request tables
    r.ids.resize((size_t)cf::kNumComp * p.ncell);
    for (int c = 0; c < cf::kNumComp; ++c)
        std::memcpy(r.ids.data() + (size_t)c * p.ncell, p.ids[c].data(), p.ncell);
    if (r.v3 >= 0) {
        r.idp.resize((size_t)p.ncell * 2);
        for (int64_t c = 0; c < p.ncell; ++c) {
            r.idp[2 * c] = uint32_t(p.ids[CF_EX][c]) | (uint32_t(p.ids[CF_EY][c]) << 8) |
                           (uint32_t(p.ids[CF_EZ][c]) << 16) | (uint32_t(p.ids[CF_HX][c]) << 24);
            r.idp[2 * c + 1] = uint32_t(p.ids[CF_HY][c]) | (uint32_t(p.ids[CF_HZ][c]) << 8);
        }
    }
    std::vector<double> l64 = cf::coefficient_lut(p, r.opts.sigma, r.opts.courant);
    if (S->precision == CF_FP64) {
        r.lut.resize(l64.size() * 8);
        std::memcpy(r.lut.data(), l64.data(), r.lut.size());
    } else {
        std::vector<float> l32(l64.begin(), l64.end());
        r.lut.resize(l32.size() * 4);
        std::memcpy(r.lut.data(), l32.data(), r.lut.size());
    }
    r.ktab.resize(r.opts.n_steps);
    cf::kernel_table(r.opts.kernel, r.opts.sigma, r.opts.courant / p.grid.res, r.opts.n_steps, r.ktab.data());
    std::vector<double> bh, ch, be, ce;
    cf::pml_tables(p, r.opts.courant, bh, ch, be, ce);
    r.pml.clear();
    for (auto* v : {&bh, &ch, &be, &ce}) r.pml.insert(r.pml.end(), v->begin(), v->end());
    return "";
}

template <typename T>
struct Dev {
    // device views of a request region
    static cf::SurfTables tabs(char* b, const Req& r) {
        cf::SurfTables t;
        t.gidx = reinterpret_cast<const int32_t*>(b + r.o_gidx);
        t.gw = reinterpret_cast<const double*>(b + r.o_gw);
        t.uidx = reinterpret_cast<const int32_t*>(b + r.o_uidx);
        t.uoff = reinterpret_cast<const int32_t*>(b + r.o_uoff);
        t.usamp = reinterpret_cast<const int32_t*>(b + r.o_usamp);
        t.uw = reinterpret_cast<const double*>(b + r.o_uw);
        t.basis = reinterpret_cast<const double*>(b + r.o_basis);
        return t;
    }
    static cf::Grid2D grid2(char* b, const Req& r) {
        const cf::Problem& p = *r.prob;
        cf::Grid2D g{};
        g.nx = p.nx;
        g.ny = p.ny;
        g.ncell = p.ncell;
        g.perx = p.grid.bc[0] == CF_BC_PERIODIC;
        g.pery = p.grid.bc[1] == CF_BC_PERIODIC;
        for (int c = 0; c < cf::kNumComp; ++c)
            g.ids[c] = reinterpret_cast<const uint8_t*>(b + r.o_ids) + (size_t)c * p.ncell;
        return g;
    }
    static cf::Grid3D grid3(char* b, const Req& r) {
        const cf::Problem& p = *r.prob;
        cf::Grid3D g{};
        g.nx = p.nx;
        g.ny = p.ny;
        g.nz = p.nz;
        g.ncell = p.ncell;
        for (int a = 0; a < 3; ++a) g.per[a] = p.grid.bc[a] == CF_BC_PERIODIC;
        for (int c = 0; c < cf::kNumComp; ++c)
            g.ids[c] = reinterpret_cast<const uint8_t*>(b + r.o_ids) + (size_t)c * p.ncell;
        g.pml = p.grid.ndim == 3 && p.grid.bc[2] == CF_BC_PML ? p.grid.pml_cells[2] : 0;
        g.psi_comp = r.st.psi_comp;
        const double* pm = reinterpret_cast<const double*>(b + r.o_pml);
        g.pml_bh = pm;
        g.pml_ch = pm + p.nz;
        g.pml_be = pm + 2 * p.nz;
        g.pml_ce = pm + 3 * p.nz;
        g.idp = r.v3 >= 0 ? reinterpret_cast<const uint2*>(b + r.o_idp) : nullptr;
        g.zr_tab = r.v3 >= 0 && !r.st.zr.empty() ? reinterpret_cast<const int2*>(b + r.o_zr) : nullptr;
        for (int v = 0; v < 8; ++v) g.zr_off[v] = r.st.zr_off[v];
        return g;
    }
};

// Zero, kick and start one wave of a request in buffer `f`.
template <typename T>
hipError_t start_wave(cf_server* S, Req& r, T* f) {
    char* b = S->arena_base + r.off;
    hipStream_t s = S->stream;
    const cf::Problem& p = *r.prob;
    const cfi::Wave& w = r.st.waves[r.wave];
    const cf::ChanDev* dch = reinterpret_cast<const cf::ChanDev*>(b + r.o_ch);
    const int* dl = reinterpret_cast<const int*>(b + r.o_slots);
    const T* lut = reinterpret_cast<const T*>(b + r.o_lut);
    const cf::SurfTables t = Dev<T>::tabs(b, r);
    const size_t fbytes = (size_t)r.st.resident * r.st.ncomp * p.ncell * sizeof(T);
    hipError_t e;
    if ((e = hipMemsetAsync(f, 0, fbytes, s)) != hipSuccess) return e;
    if (r.fused || r.v3 >= 0) {
        // the fused kernels never write the cells they skip: zero in both arrays
        char* other = b + (reinterpret_cast<char*>(f) == b + r.o_fa ? r.o_fb : r.o_fa);
        if ((e = hipMemsetAsync(other, 0, fbytes, s)) != hipSuccess) return e;
    }
    if (r.st.psi_comp > 0 &&
        (e = hipMemsetAsync(b + r.o_psi, 0, (size_t)r.st.resident * 4 * r.st.psi_comp * sizeof(T), s)) != hipSuccess)
        return e;
    if (r.v3 >= 0 && r.st.psi_comp > 0 &&
        (e = hipMemsetAsync(b + r.o_psi2, 0, (size_t)r.st.resident * 4 * r.st.psi_comp * sizeof(T), s)) != hipSuccess)
        return e;
    r.par = 0;
    if ((e = cf::launch_kick<T>(f, dch, dl + w.all_off, w.n_all, r.st.max_uniq, t, s)) != hipSuccess) return e;
    if (p.grid.ndim == 3) {
        const cf::Grid3D g = Dev<T>::grid3(b, r);
        T* psi = r.st.psi_comp > 0 ? reinterpret_cast<T*>(b + r.o_psi) : nullptr;
        if ((e = cf::launch_h3d<T>(1, f, psi, dch, dl + w.d3_off, w.n_3d, g, lut, s)) != hipSuccess) return e;
        return cf::launch_e3d<T>(1, f, psi, dch, dl + w.d3_off, w.n_3d, g, lut, s);
    }
    const cf::Grid2D g = Dev<T>::grid2(b, r);
    if ((e = cf::launch_h2d<T>(CF_POL_TM, 1, f, dch, dl + w.tm_off, w.n_tm, g, lut, s)) != hipSuccess) return e;
    if ((e = cf::launch_h2d<T>(CF_POL_TE, 1, f, dch, dl + w.te_off, w.n_te, g, lut, s)) != hipSuccess) return e;
    if ((e = cf::launch_e2d<T>(CF_POL_TM, 1, f, dch, dl + w.tm_off, w.n_tm, g, lut, s)) != hipSuccess) return e;
    return cf::launch_e2d<T>(CF_POL_TE, 1, f, dch, dl + w.te_off, w.n_te, g, lut, s);
}

template <typename T>
hipError_t admit(cf_server* S, Req& r) {
    if (r.whole) return hipSuccess;   // cf_solve stages its own tables at run time
    char* b = S->arena_base + r.off;
    hipStream_t s = S->stream;
    const cfi::Staged& st = r.st;
    auto up = [&](size_t o, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(b + o, src, bytes, hipMemcpyHostToDevice, s);
    };
    hipError_t e;
#define UP(o, p_, n_) \
    if ((e = up(o, p_, n_)) != hipSuccess) return e
    UP(r.o_ids, r.ids.data(), r.ids.size());
    UP(r.o_lut, r.lut.data(), r.lut.size());
    UP(r.o_ktab, r.ktab.data(), r.ktab.size() * 8);
    UP(r.o_pml, r.pml.data(), r.pml.size() * 8);
    UP(r.o_ch, st.dev.data(), st.dev.size() * sizeof(cf::ChanDev));
    UP(r.o_slots, st.slot_lists.data(), st.slot_lists.size() * sizeof(int));
    UP(r.o_gidx, st.gidx.data(), st.gidx.size() * 4);
    UP(r.o_gw, st.gw.data(), st.gw.size() * 8);
    UP(r.o_uidx, st.uidx.data(), st.uidx.size() * 4);
    UP(r.o_uoff, st.uoff.data(), st.uoff.size() * 4);
    UP(r.o_usamp, st.usamp.data(), st.usamp.size() * 4);
    UP(r.o_uw, st.uw.data(), st.uw.size() * 8);
    UP(r.o_basis, st.basis.data(), st.basis.size() * 8);
    UP(r.o_idp, r.idp.data(), r.idp.size() * 4);
    if (r.v3 >= 0) UP(r.o_zr, st.zr.data(), st.zr.size() * 4);
#undef UP
    if ((e = hipMemsetAsync(b + r.o_acc, 0, (size_t)r.C * 2 * 8, s)) != hipSuccess) return e;
    r.wave = 0;
    r.start = S->clock;
    r.done = 0;
    r.credit = 0;
    r.sps = 0;
    // a fused request is kicked into the buffer the next fused launch reads
    T* f = reinterpret_cast<T*>(b + (r.fused && S->parity ? r.o_fb : r.o_fa));
    return start_wave<T>(S, r, f);
}

// Rebuild the fused group: descriptors and instances of every fused request
// and one work list per (variant, polarization) in use.
template <typename T>
hipError_t rebuild_group(cf_server* S) {
    std::vector<cf::ChanDev> ch;
    std::vector<cf::InstDev> inst;
    struct SlotTiles {
        std::vector<int> first;                          // slots
        std::vector<const std::vector<cfi::LiveTile>*> second;   // live tiles per slot
        std::vector<int> third;                          // surface tile per slot
    };
    std::map<std::pair<int, int>, SlotTiles> lists;   // (v, pol) -> slots, tiles, surface tiles
    for (auto& rp : S->active) {
        Req& r = *rp;
        if (!r.fused) continue;
        char* b = S->arena_base + r.off;
        const cf::Problem& p = *r.prob;
        const cfi::TBPlan& pl = r.st.plans[r.variant];
        const int ii = (int)inst.size();
        cf::InstDev I{};
        I.fa = b + r.o_fa;
        I.fb = b + r.o_fb;
        I.acc = reinterpret_cast<double*>(b + r.o_acc);
        I.nx = p.nx;
        I.ny = p.ny;
        I.ncell = p.ncell;
        const cf::Grid2D g = Dev<T>::grid2(b, r);
        I.perx = g.perx;
        I.pery = g.pery;
        for (int c = 0; c < cf::kNumComp; ++c) I.ids[c] = g.ids[c];
        I.lut = b + r.o_lut;
        I.base_x = pl.base_x;
        I.base_y = pl.base_y;
        I.ntx = pl.ntx;
        I.nty = pl.nty;
        I.stile = pl.stile;
        I.start = (int)r.start;
        I.nsteps = r.opts.n_steps;
        I.dt = r.opts.courant / p.grid.res;
        I.dA = std::pow(1.0 / p.grid.res, p.grid.ndim - 1);
        I.ktab = reinterpret_cast<const double*>(b + r.o_ktab);
        I.gamma = nullptr;
        I.gamma_stride = r.C;
        I.t = Dev<T>::tabs(b, r);
        inst.push_back(I);
        for (int c = 0; c < r.C; ++c) {
            cf::ChanDev d = r.st.dev[c];
            d.inst = ii;
            const int slot = (int)ch.size();
            ch.push_back(d);
            auto& l = lists[{r.variant, r.chans[c].pol}];
            l.first.push_back(slot);
            l.second.push_back(&cfi::live_tiles(pl, r.chans[c].pol));
            l.third.push_back(pl.stile);
        }
    }
    std::vector<cf::WorkItem> work;
    std::vector<cf_server::Launch> launches;
    for (auto& kv : lists) {
        std::vector<cf::WorkItem> w = cfi::make_work(kv.second.first, kv.second.second, kv.second.third);
        launches.push_back({kv.first.first, kv.first.second, work.size(), (int)w.size()});
        work.insert(work.end(), w.begin(), w.end());
    }
    if (ch.size() > S->cap_ch || inst.size() > S->cap_inst || work.size() > S->cap_work) return hipErrorOutOfMemory;
    hipStream_t s = S->stream;
    S->keep_ch.push_back(std::move(ch));
    S->keep_inst.push_back(std::move(inst));
    S->keep_work.push_back(std::move(work));
    const auto& kc = S->keep_ch.back();
    const auto& ki = S->keep_inst.back();
    const auto& kw = S->keep_work.back();
    hipError_t e;
    if (!kc.empty() && (e = hipMemcpyAsync(S->group + S->g_ch, kc.data(), kc.size() * sizeof(cf::ChanDev),
                                           hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    if (!ki.empty() && (e = hipMemcpyAsync(S->group + S->g_inst, ki.data(), ki.size() * sizeof(cf::InstDev),
                                           hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    if (!kw.empty() && (e = hipMemcpyAsync(S->group + S->g_work, kw.data(), kw.size() * sizeof(cf::WorkItem),
                                           hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    S->launches = std::move(launches);
    S->membership_changed = false;
    return hipSuccess;
}

// One tick: K steps of every resident request.
template <typename T>
hipError_t tick(cf_server* S) {
    hipStream_t s = S->stream;
    hipError_t e;
    S->n_marks = 0;
    auto mark = [&]() -> hipError_t {
        if (S->n_marks == S->ev.size()) {
            hipEvent_t x;
            const hipError_t c = hipEventCreate(&x);
            if (c != hipSuccess) return c;
            S->ev.push_back(x);
        }
        return hipEventRecord(S->ev[S->n_marks++], s);
    };
    bool any_fused = false;
    for (auto& rp : S->active) any_fused = any_fused || rp->fused;
    if ((e = mark()) != hipSuccess) return e;
    if (any_fused) {
        if (S->membership_changed && (e = rebuild_group<T>(S)) != hipSuccess) return e;
        const cf::ChanDev* gch = reinterpret_cast<const cf::ChanDev*>(S->group + S->g_ch);
        const cf::InstDev* gin = reinterpret_cast<const cf::InstDev*>(S->group + S->g_inst);
        const cf::WorkItem* gw = reinterpret_cast<const cf::WorkItem*>(S->group + S->g_work);
        // TM and TE launches on two streams: each polarization's launch tail
        // overlaps the other's (the requests' channels are independent runs)
        bool any_te = false, any_tm = false;
        for (const auto& l : S->launches) (l.pol == CF_POL_TE ? any_te : any_tm) = true;
        const bool split = any_te && any_tm && S->side;
        if (split) {
            if ((e = hipEventRecord(S->fork, s)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(S->side, S->fork, 0)) != hipSuccess) return e;
        }
        for (const auto& l : S->launches)
            if ((e = cf::launch_tb2d<T>(l.variant, l.pol, gch, gw + l.off, l.n, gin, S->kh, (int)S->clock,
                                        S->parity, split && l.pol == CF_POL_TE ? S->side : s)) != hipSuccess)
                return e;
        if (split) {
            if ((e = hipEventRecord(S->join, S->side)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, S->join, 0)) != hipSuccess) return e;
        }
    }
    if ((e = mark()) != hipSuccess) return e;
    for (auto& rp : S->active) {
        Req& r = *rp;
        if (r.fused || r.whole) continue;
        char* b = S->arena_base + r.off;
        const cf::Problem& p = *r.prob;
        const cfi::Wave& w = r.st.waves[r.wave];
        const cf::ChanDev* dch = reinterpret_cast<const cf::ChanDev*>(b + r.o_ch);
        const int* dl = reinterpret_cast<const int*>(b + r.o_slots);
        const T* lut = reinterpret_cast<const T*>(b + r.o_lut);
        const cf::SurfTables t = Dev<T>::tabs(b, r);
        T* f = reinterpret_cast<T*>(b + r.o_fa);
        T* psi = r.st.psi_comp > 0 ? reinterpret_cast<T*>(b + r.o_psi) : nullptr;
        const double* kt = reinterpret_cast<const double*>(b + r.o_ktab);
        double* acc = reinterpret_cast<double*>(b + r.o_acc);
        const double dt = r.opts.courant / p.grid.res, dA = std::pow(1.0 / p.grid.res, p.grid.ndim - 1);
        for (int k = 0; k < r.tick_steps; ++k) {
            const long long m = r.done + k;
            if (m >= r.opts.n_steps) break;
            T* cur = f;   // field array the surface is read from after this step
            if (p.grid.ndim == 3 && r.v3 >= 0) {
                const cf::Grid3D g = Dev<T>::grid3(b, r);
                T* fa = reinterpret_cast<T*>(b + r.o_fa);
                T* fb = reinterpret_cast<T*>(b + r.o_fb);
                T* pa = psi;
                T* pb = psi ? reinterpret_cast<T*>(b + r.o_psi2) : nullptr;
                T* src = r.par ? fb : fa;
                T* dst = r.par ? fa : fb;
                // steps m and m + 1 in one two-step launch when both fall in this tick
                const bool two = cf::f3d_steps(r.v3) == 2 && k + 1 < r.tick_steps && m + 1 < r.opts.n_steps;
                T* sh = reinterpret_cast<T*>(b + r.o_shadow);
                if ((e = cf::launch_f3d<T>(two ? r.v3 : r.v3s, dch, dl + w.d3_off, w.n_3d, g, lut, src, dst,
                                           r.par ? pb : pa, r.par ? pa : pb, sh, r.st.sbox, s)) != hipSuccess)
                    return e;
                if (two) {
                    if ((e = cf::launch_surface_box<T>(sh, r.st.sbox, g, dch, dl + w.all_off, w.n_all, t, kt, (int)m,
                                                       dt, dA, acc, nullptr, 0, s)) != hipSuccess)
                        return e;
                    ++k;   // the pair's second step: measured below
                }
                r.par ^= 1;
                cur = dst;
                if (two) {
                    if ((e = cf::launch_surface<T>(cur, dch, dl + w.all_off, w.n_all, t, kt, (int)m + 1, dt, dA, acc,
                                                   nullptr, 0, s)) != hipSuccess)
                        return e;
                    continue;
                }
            } else if (p.grid.ndim == 3) {
                const cf::Grid3D g = Dev<T>::grid3(b, r);
                if ((e = cf::launch_h3d<T>(0, f, psi, dch, dl + w.d3_off, w.n_3d, g, lut, s)) != hipSuccess) return e;
                if ((e = cf::launch_e3d<T>(0, f, psi, dch, dl + w.d3_off, w.n_3d, g, lut, s)) != hipSuccess) return e;
            } else {
                const cf::Grid2D g = Dev<T>::grid2(b, r);
                if ((e = cf::launch_h2d<T>(CF_POL_TM, 0, f, dch, dl + w.tm_off, w.n_tm, g, lut, s)) != hipSuccess)
                    return e;
                if ((e = cf::launch_h2d<T>(CF_POL_TE, 0, f, dch, dl + w.te_off, w.n_te, g, lut, s)) != hipSuccess)
                    return e;
                if ((e = cf::launch_e2d<T>(CF_POL_TM, 0, f, dch, dl + w.tm_off, w.n_tm, g, lut, s)) != hipSuccess)
                    return e;
                if ((e = cf::launch_e2d<T>(CF_POL_TE, 0, f, dch, dl + w.te_off, w.n_te, g, lut, s)) != hipSuccess)
                    return e;
            }
            if ((e = cf::launch_surface<T>(cur, dch, dl + w.all_off, w.n_all, t, kt, (int)m, dt, dA, acc, nullptr, 0,
                                           s)) != hipSuccess)
                return e;
        }
        if ((e = mark()) != hipSuccess) return e;
    }
    // whole-solve requests: one blocking cf_solve each (a failure fails only
    // that request)
    for (auto& rp : S->active) {
        Req& r = *rp;
        if (!r.whole || r.ran || r.cancel) continue;
        cf_opts o = r.opts;
        o.stream = s;
        r.w_res = cf_result{};
        r.w_res.per_harmonic = r.w_ph.data();
        r.w_res.per_harmonic_len = (int)r.w_ph.size();
        r.w_res.per_face = r.w_pf.data();
        r.w_res.per_face_len = (int)r.w_pf.size();
        r.w_res.per_channel = r.w_pc.data();
        r.w_res.per_channel_len = (int)r.w_pc.size();
        const cf_status st = cf_solve(r.handle.get(), &o, S->arena_base + r.off, r.bytes, &r.w_res);
        r.ran = true;
        if (st != CF_OK) {
            r.status = st;
            r.err = cf_last_error();
        }
    }
    return hipSuccess;
}

// Steps of each non-fused request in the coming tick.  Every resident
// request is entitled to the same device time per tick: the fused launches
// advance all fused requests by K steps in group_s seconds, so the share is
// group_s / (fused requests); with no fused request resident it is K steps
// of the cheapest non-fused request.  A request earns share / (its seconds
// per step) of step credit per tick.  Until its time per step is measured a
// request runs K steps.  Convergence checks fall on tick boundaries, and
// two-step 3D requests run their steps in pairs (a single step only at the
// end or before a check).
void plan_steps(cf_server* S) {
    int nf = 0;
    double min_sps = 0;
    for (auto& rp : S->active) {
        if (rp->fused) ++nf;
        else if (!rp->whole && rp->sps > 0 && (min_sps == 0 || rp->sps < min_sps)) min_sps = rp->sps;
    }
    const double share = nf > 0 ? (S->group_s > 0 ? S->group_s / nf : 0.0) : S->kh * min_sps;
    for (auto& rp : S->active) {
        Req& r = *rp;
        if (r.fused || r.whole) continue;
        const long long left = r.opts.n_steps - r.done;
        long long n = S->kh;
        if (r.sps > 0 && share > 0) {
            r.credit += share / r.sps;
            n = (long long)r.credit;
        }
        n = std::min(n, left);
        if (r.conv.on) n = std::min<long long>(n, r.conv.next - r.done);
        const bool pairs = r.v3 >= 0 && cf::f3d_steps(r.v3) == 2;
        const bool last = n == left || (r.conv.on && n == r.conv.next - r.done);
        if (pairs && n % 2 == 1 && !last) --n;
        n = std::max<long long>(n, 0);
        r.tick_steps = (int)n;
        if (r.sps > 0 && share > 0) r.credit = std::min(std::max(r.credit - n, 0.0), 2.0);
    }
}

// Device times of the tick just drained: the fused launches and each
// non-fused request's steps (events recorded by tick in this order).
void read_times(cf_server* S) {
    if (S->n_marks < 2) return;
    auto span = [&](size_t a) {
        float ms = 0;
        return hipEventElapsedTime(&ms, S->ev[a], S->ev[a + 1]) == hipSuccess ? ms * 1e-3 : -1.0;
    };
    bool any_fused = false;
    for (auto& rp : S->active) any_fused = any_fused || rp->fused;
    const double g = span(0);
    if (any_fused && g > 0) S->group_s = S->group_s > 0 ? 0.5 * (S->group_s + g) : g;
    size_t k = 1;
    for (auto& rp : S->active) {
        Req& r = *rp;
        if (r.fused || r.whole) continue;
        if (k + 1 >= S->n_marks) break;
        const double t = span(k++);
        if (r.tick_steps > 0 && t > 0) {
            const double per = t / r.tick_steps;
            r.sps = r.sps > 0 ? 0.5 * (r.sps + per) : per;
        }
    }
}

template <typename T>
void loop(cf_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // ---- admission (arrival order, later requests may pass) ----
        for (auto it = S->queue.begin(); it != S->queue.end();) {
            Req& r = **it;
            if (!r.cancel) {
                ++it;
                continue;
            }
            r.state = ST_CANCELLED;
            r.status = CF_E_CANCELLED;
            r.err = "request cancelled";
            r.t_done = now_s();
            ++S->n_cancelled;
            it = S->queue.erase(it);
            S->cv.notify_all();
        }
        std::vector<size_t> want;
        for (auto& q : S->queue) want.push_back(q->bytes);
        const auto picked = cfi::admit_pass(S->arena, want);
        std::vector<bool> taken(S->queue.size(), false);
        for (const auto& kp : picked) {
            Req& r = *S->queue[kp.first];
            taken[kp.first] = true;
            r.off = kp.second;
            r.t_admit = now_s();
            hipError_t e = admit<T>(S, r);
            if (e != hipSuccess) {
                S->thread_error = std::string("admission failed: ") + hipGetErrorString(e);
                r.state = ST_FAILED;
                r.status = CF_E_DEVICE;
                r.err = S->thread_error;
                r.t_done = now_s();
                S->arena.release(r.off, r.bytes);
                ++S->n_failed;
                S->cv.notify_all();
                continue;
            }
            r.state = ST_RUNNING;
            S->active.push_back(S->queue[kp.first]);
            if (r.fused) S->membership_changed = true;
        }
        {
            std::deque<std::shared_ptr<Req>> rest;
            for (size_t k = 0; k < S->queue.size(); ++k)
                if (!taken[k]) rest.push_back(S->queue[k]);
            S->queue.swap(rest);
        }
        if (S->active.empty() && !S->queue.empty()) {
            // nothing resident and still nothing fits: the head can never run
            Req& r = *S->queue.front();
            r.state = ST_FAILED;
            r.status = CF_E_BUDGET;
            r.err = "request does not fit the server's memory budget";
            r.t_done = now_s();
            ++S->n_failed;
            S->queue.pop_front();
            S->cv.notify_all();
            continue;
        }
        if (S->active.empty()) {
            if (S->stop) break;
            S->cv.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->stop && S->queue.empty()) break;
            continue;
        }
        // ---- one tick ----
        plan_steps(S);
        const double t0 = now_s();
        lk.unlock();
        hipError_t e = tick<T>(S);
        if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
        lk.lock();
        S->busy_s += now_s() - t0;
        if (e != hipSuccess) {
            S->thread_error = std::string("tick failed: ") + hipGetErrorString(e);
            for (auto& rp : S->active) {
                rp->state = ST_FAILED;
                rp->status = CF_E_DEVICE;
                rp->err = S->thread_error;
                rp->t_done = now_s();
                S->arena.release(rp->off, rp->bytes);
                ++S->n_failed;
            }
            S->active.clear();
            S->membership_changed = true;
            S->cv.notify_all();
            continue;
        }
        read_times(S);
        S->clock += S->kh;
        S->parity ^= 1;
        for (auto& rp : S->active)
            if (!rp->fused && !rp->whole) rp->done += rp->tick_steps;
        // the stream has drained: staged group tables are no longer read
        S->keep_ch.clear();
        S->keep_inst.clear();
        S->keep_work.clear();
        // ---- retire finished requests / start next channel waves ----
        for (auto it = S->active.begin(); it != S->active.end();) {
            Req& r = **it;
            const long long ran = r.fused ? S->clock - r.start : r.whole ? (r.ran ? r.opts.n_steps : 0) : r.done;
            bool wave_done = ran >= r.opts.n_steps;
            const long long done = std::min<long long>(ran, r.opts.n_steps);
            if (!wave_done && r.conv.on && done >= r.conv.next) {
                // time-convergence check on the accumulators (the stream has drained)
                while (r.conv.next <= done) r.conv.next += r.conv.every;
                std::vector<double> a((size_t)r.C * 2);
                if (hipMemcpyAsync(a.data(), S->arena_base + r.off + r.o_acc, a.size() * 8, hipMemcpyDeviceToHost,
                                   S->stream) == hipSuccess &&
                    hipStreamSynchronize(S->stream) == hipSuccess && r.conv.update(a, r.chans)) {
                    wave_done = true;
                    r.steps_run = (int)done;
                }
            }
            if (!wave_done && !r.cancel) {
                ++it;
                continue;
            }
            if (!r.cancel && !r.fused && r.wave + 1 < (int)r.st.waves.size()) {
                ++r.wave;
                r.start = S->clock;
                r.done = 0;
                r.credit = 0;
                hipError_t e2 = start_wave<T>(S, r, reinterpret_cast<T*>(S->arena_base + r.off + r.o_fa));
                if (e2 == hipSuccess) {
                    ++it;
                    continue;
                }
                r.status = CF_E_DEVICE;
                r.err = hipGetErrorString(e2);
            }
            if (r.cancel) {
                r.state = ST_CANCELLED;
                r.status = CF_E_CANCELLED;
                r.err = "request cancelled";
                ++S->n_cancelled;
            } else if (r.whole) {
                r.state = r.status == CF_OK ? ST_DONE : ST_FAILED;
                (r.status == CF_OK ? S->n_completed : S->n_failed)++;
            } else if (r.status == CF_OK) {
                r.acc.assign((size_t)r.C * 2, 0.0);
                hipError_t e3 = hipMemcpyAsync(r.acc.data(), S->arena_base + r.off + r.o_acc, r.acc.size() * 8,
                                               hipMemcpyDeviceToHost, S->stream);
                if (e3 == hipSuccess) e3 = hipStreamSynchronize(S->stream);
                bool finite = e3 == hipSuccess;
                for (double v : r.acc) finite = finite && std::isfinite(v);
                if (e3 != hipSuccess) {
                    r.status = CF_E_DEVICE;
                    r.err = hipGetErrorString(e3);
                } else if (!finite) {
                    r.status = CF_E_NONFINITE;
                    r.err = "a force accumulator is not finite";
                }
                r.state = r.status == CF_OK ? ST_DONE : ST_FAILED;
                (r.status == CF_OK ? S->n_completed : S->n_failed)++;
            } else {
                r.state = ST_FAILED;
                ++S->n_failed;
            }
            r.t_done = now_s();
            S->arena.release(r.off, r.bytes);
            drop_tables(r);
            if (r.fused) S->membership_changed = true;
            it = S->active.erase(it);
            S->cv.notify_all();
        }
    }
}

std::shared_ptr<Req> find(cf_server* S, uint64_t ticket) {
    auto it = S->all.find(ticket);
    return it == S->all.end() ? nullptr : it->second;
}

}  // namespace

// ---- entry points: bodies (no C linkage) -----------------------------------

static cf_status cf_server_create_impl(size_t hbm_budget_bytes, int precision, int tile_variant, void* arena, void* stream,
                           cf_server** out) {
    if (!out || hbm_budget_bytes < (size_t)1 << 20) return fail(CF_E_ARG, "bad server arguments");
    if (precision != CF_FP32 && precision != CF_FP64) return fail(CF_E_ARG, "unknown precision");
    *out = nullptr;
    std::unique_ptr<cf_server> S(new cf_server);
    S->precision = precision;
    if (hipGetDevice(&S->device) != hipSuccess) return fail(CF_E_DEVICE, "no HIP device");
    // fused variant and steps per tick
    cf::TBShape sh[cf::kMaxVariants];
    const int nv = precision == CF_FP64 ? cf::tb_variants<double>(sh, cf::kMaxVariants)
                                        : cf::tb_variants<float>(sh, cf::kMaxVariants);
    if (tile_variant < 0 || tile_variant > nv) return fail(CF_E_ARG, "tile_variant out of range");
    // default: the FP32 shape that is fastest on the piston workloads (8 waves
    // of 7 rows, 8 steps per launch), the first FP64 shape
    const int first = tile_variant > 0 ? tile_variant - 1 : (precision == CF_FP64 ? 0 : std::min(12, nv - 1));
    S->kh = sh[first].kh;
    // the preferred variant, then every other one with the same steps per
    // launch (wider tiles take surfaces the preferred one cannot hold)
    S->prefer.push_back(first);
    for (int v = 0; v < nv; ++v)
        if (v != first && sh[v].kh == S->kh) S->prefer.push_back(v);
    // fused group tables: descriptors, instances and two work lists
    S->cap_ch = 1 << 16;
    S->cap_inst = 1 << 10;
    S->cap_work = (size_t)1 << 20;
    S->g_ch = 0;
    S->g_inst = cfi::align_up(S->cap_ch * sizeof(cf::ChanDev), 256);
    S->g_work = S->g_inst + cfi::align_up(S->cap_inst * sizeof(cf::InstDev), 256);
    S->group_bytes = S->g_work + S->cap_work * sizeof(cf::WorkItem);
    if (hbm_budget_bytes <= S->group_bytes + ((size_t)1 << 20))
        return fail(CF_E_BUDGET, "budget too small for the server's tables");
    if (arena) {
        S->arena_base = static_cast<char*>(arena);
    } else {
        void* a = nullptr;
        if (hipMalloc(&a, hbm_budget_bytes) != hipSuccess) return fail(CF_E_DEVICE, "hipMalloc of the budget failed");
        S->arena_base = static_cast<char*>(a);
        S->own_arena = true;
    }
    S->group = S->arena_base;
    S->arena.reset(hbm_budget_bytes - S->group_bytes);
    S->arena_base += S->group_bytes;   // request regions follow the group tables
    if (stream) {
        S->stream = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreate(&S->stream) != hipSuccess) return fail(CF_E_DEVICE, "hipStreamCreate failed");
        S->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&S->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&S->join, hipEventDisableTiming) != hipSuccess)
        return fail(CF_E_DEVICE, "server stream setup failed");
    cf_server* raw = S.get();
    if (precision == CF_FP64) S->worker = std::thread([raw] { loop<double>(raw); });
    else S->worker = std::thread([raw] { loop<float>(raw); });
    *out = S.release();
    return CF_OK;
}

static cf_status cf_server_submit_impl(cf_server* S, cf_problem* prob, const cf_opts* o, uint64_t* ticket) {
    if (!S || !prob || !o || !ticket) return fail(CF_E_ARG, "null argument");
    if (o->precision != S->precision) return fail(CF_E_ARG, "request precision differs from the server's");
    if (o->path != CF_PATH_BATCHED) return fail(CF_E_ARG, "served requests use the batched path");
    if (o->n_subset > 0) return fail(CF_E_ARG, "served requests run every channel");
    if (prob->p.dispersive)
        return fail(CF_E_UNSUPPORTED, "problems with dispersive materials are solved with cf_solve, not served");
    if (prob->p.pml2d() && !prob->p.reduced())
        return fail(CF_E_UNSUPPORTED, "2D problems with PML layers are solved with cf_solve, not served");
    cf_status st = cf_validate(prob, o);
    if (st != CF_OK) return st;
    auto r = std::make_shared<Req>();
    r->opts = *o;
    r->t_submit = now_s();
    if (prob->p.reduced()) {
        // the caller may destroy its problem after submitting: keep a copy
        r->handle.reset(new cf_problem{prob->p});
        r->prob = &r->handle->p;
        r->whole = true;
        cf_info info;
        if ((st = cf_problem_info(r->handle.get(), o, &info)) != CF_OK) return st;
        r->C = info.n_channels;
        r->w_ph.assign(info.per_harmonic_len, 0.0);
        r->w_pf.assign(2 * r->prob->grid.ndim, 0.0);
        r->w_pc.assign(info.n_channels, 0.0);
        r->bytes = cfi::align_up(info.workspace_bytes, 256);
        if (r->bytes > S->arena.size())
            return fail(CF_E_BUDGET, "request does not fit the server's memory budget");
    } else {
        r->own = prob->p;             // the caller may destroy its problem after submitting
        r->prob = &r->own;
        // staging reads only settings fixed at creation: no lock needed
        std::string err = prepare(S, *r);
        if (!err.empty()) return fail(CF_E_BUDGET, err);
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        S->queue.push_back(r);
        S->all[r->ticket] = r;
        ++S->n_submitted;
        *ticket = r->ticket;
    }
    S->cv.notify_all();
    return CF_OK;
}

static cf_status report(cf_server* S, const std::shared_ptr<Req>& r, int* state, cf_result* out) {
    if (state) *state = r->state;
    if (r->state == ST_DONE && out) {
        const int lab = cf::harmonic_len(*r->prob);
        if (out->per_harmonic && out->per_harmonic_len < lab) return fail(CF_E_ARG, "per_harmonic too short");
        if (out->per_face && out->per_face_len < 2 * r->prob->grid.ndim) return fail(CF_E_ARG, "per_face too short");
        if (out->per_channel && out->per_channel_len < r->C) return fail(CF_E_ARG, "per_channel too short");
        if (out->gamma || out->trace) return fail(CF_E_ARG, "served requests keep no gamma or trace");
    }
    if (r->state == ST_DONE && out && r->whole) {
        const cf_result& w = r->w_res;
        auto put = [](double* dst, int len, const std::vector<double>& v) {
            if (dst) std::copy(v.begin(), v.begin() + std::min<size_t>(v.size(), (size_t)len), dst);
        };
        put(out->per_harmonic, out->per_harmonic_len, r->w_ph);
        put(out->per_face, out->per_face_len, r->w_pf);
        put(out->per_channel, out->per_channel_len, r->w_pc);
        out->force = w.force;
        out->n_channels_run = w.n_channels_run;
        out->cell_updates = w.cell_updates;
        out->device_ms = w.device_ms;
        out->stencil_ms_avg = w.stencil_ms_avg;
        out->stencil_samples = w.stencil_samples;
        out->stencil_launches = w.stencil_launches;
        out->stencil_alg_bytes = w.stencil_alg_bytes;
        out->stencil_cell_updates = w.stencil_cell_updates;
        out->fused = w.fused;
        out->tile_variant = w.tile_variant;
        out->tile_halo = w.tile_halo;
        out->n_steps_run = w.n_steps_run;
        out->advanced_cell_updates = w.advanced_cell_updates;
    } else if (r->state == ST_DONE && out) {
        cfi::StencilTiming tim;
        tim.steps_run = r->steps_run;
        tim.variant = r->variant >= 0 ? r->variant : r->v3;   // fused 2D tile or fused 3D band shape
        cf_opts o = r->opts;
        const bool ok = cfi::fill_result(*r->prob, r->chans, r->acc, {}, o, (r->t_done - r->t_admit) * 1e3, tim,
                                         r->st, out);
        if (!ok) return fail(CF_E_NONFINITE, "a force accumulator is not finite");
    }
    if (r->state == ST_FAILED || r->state == ST_CANCELLED) return fail(r->status, r->err.empty() ? "request failed" : r->err);
    cfi::clear_error();
    return CF_OK;
}

static cf_status cf_server_poll_impl(cf_server* S, uint64_t ticket, int* state, cf_result* out) {
    if (!S) return fail(CF_E_ARG, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto r = find(S, ticket);
    if (!r) return fail(CF_E_ARG, "unknown ticket");
    return report(S, r, state, out);
}

static cf_status cf_server_wait_impl(cf_server* S, uint64_t ticket, double timeout_s, int* state, cf_result* out) {
    if (!S) return fail(CF_E_ARG, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto r = find(S, ticket);
    if (!r) return fail(CF_E_ARG, "unknown ticket");
    auto pred = [&] { return r->state >= ST_DONE; };
    if (timeout_s < 0) S->cv.wait(lk, pred);
    else S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
    return report(S, r, state, out);
}

static cf_status cf_server_cancel_impl(cf_server* S, uint64_t ticket) {
    if (!S) return fail(CF_E_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto r = find(S, ticket);
        if (!r) return fail(CF_E_ARG, "unknown ticket");
        r->cancel = true;
    }
    S->cv.notify_all();
    return CF_OK;
}

static cf_status cf_server_times_impl(cf_server* S, uint64_t ticket, double* submit_s, double* admit_s, double* done_s) {
    if (!S) return fail(CF_E_ARG, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto r = find(S, ticket);
    if (!r) return fail(CF_E_ARG, "unknown ticket");
    if (submit_s) *submit_s = r->t_submit;
    if (admit_s) *admit_s = r->t_admit;
    if (done_s) *done_s = r->t_done;
    return CF_OK;
}

static cf_status cf_server_stats_impl(cf_server* S, cf_server_info* out) {
    if (!S || !out) return fail(CF_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out->submitted = S->n_submitted;
    out->completed = S->n_completed;
    out->failed = S->n_failed;
    out->cancelled = S->n_cancelled;
    out->queued = (int)S->queue.size();
    out->running = (int)S->active.size();
    out->bytes_in_use = S->arena.used();
    out->budget = S->arena.size();
    out->clock_steps = S->clock;
    out->busy_s = S->busy_s;
    out->steps_per_tick = S->kh;
    return CF_OK;
}

static cf_status cf_server_destroy_impl(cf_server* S) {
    if (!S) return CF_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto& kv : S->all) kv.second->cancel = true;
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipStreamSynchronize(S->stream);
    for (hipEvent_t x : S->ev) (void)hipEventDestroy(x);
    if (S->side) {
        (void)hipStreamSynchronize(S->side);
        (void)hipStreamDestroy(S->side);
    }
    if (S->fork) (void)hipEventDestroy(S->fork);
    if (S->join) (void)hipEventDestroy(S->join);
    if (S->own_stream) (void)hipStreamDestroy(S->stream);
    if (S->own_arena) (void)hipFree(S->group);
    delete S;
    return CF_OK;
}


// ---- the C ABI: every entry point runs its body under cfi::guarded ---------

extern "C" {

cf_status cf_server_create(size_t hbm_budget_bytes, int precision, int tile_variant, void* arena, void* stream,
                           cf_server** out) {
    return cfi::guarded([&] { return cf_server_create_impl(hbm_budget_bytes, precision, tile_variant, arena, stream, out); });
}

cf_status cf_server_submit(cf_server* S, cf_problem* prob, const cf_opts* o, uint64_t* ticket) {
    return cfi::guarded([&] { return cf_server_submit_impl(S, prob, o, ticket); });
}

cf_status cf_server_poll(cf_server* S, uint64_t ticket, int* state, cf_result* out) {
    return cfi::guarded([&] { return cf_server_poll_impl(S, ticket, state, out); });
}

cf_status cf_server_wait(cf_server* S, uint64_t ticket, double timeout_s, int* state, cf_result* out) {
    return cfi::guarded([&] { return cf_server_wait_impl(S, ticket, timeout_s, state, out); });
}

cf_status cf_server_cancel(cf_server* S, uint64_t ticket) {
    return cfi::guarded([&] { return cf_server_cancel_impl(S, ticket); });
}

cf_status cf_server_times(cf_server* S, uint64_t ticket, double* submit_s, double* admit_s, double* done_s) {
    return cfi::guarded([&] { return cf_server_times_impl(S, ticket, submit_s, admit_s, done_s); });
}

cf_status cf_server_stats(cf_server* S, cf_server_info* out) {
    return cfi::guarded([&] { return cf_server_stats_impl(S, out); });
}

cf_status cf_server_destroy(cf_server* S) {
    return cfi::guarded([&] { return cf_server_destroy_impl(S); });
}

}  // extern "C"
