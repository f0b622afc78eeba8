// C ABI of the Casimir FDTD library: problem handles, validation, workspace
// layout, table upload, the batched and plain stepping loops and the final
// reduction of the per-channel FP64 accumulators into the force.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/casimir_fdtd.h"
#include "device.hpp"
#include "plan.hpp"
#include "solver.hpp"
#include "red_span.hpp"

struct cf_problem {
    cf::Problem p;
};

namespace cfi {

thread_local std::string g_err;

cf_status fail(cf_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

cf_status fail_nothrow(cf_status code, const char* msg) noexcept {
    try {
        g_err = msg;
    } catch (...) {
        g_err.clear();
    }
    return code;
}

void clear_error() { g_err.clear(); }

#define CF_HIP(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(CF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

// Device workspace layout of one solve.
struct Layout {
    size_t ids, lut, ktab, pml, chans, slots, gidx, gw, uidx, uoff, usamp, uw, basis, acc, gamma,
        fields, fields2, psi, psi2, pml2, idp, shadow, rinv, inst, work, aux, lor, zr, total;
    size_t work_items;    // capacity of one work list
};




// Where some E component of a polarization can be nonzero: a summed-area
// table over the grid of cells whose E coefficients are not a = b = 0 (the
// fused kernel's test for waves that advance nothing).
struct ELive {
    int nx = 0, ny = 0;
    bool perx = false, pery = false;
    std::vector<int32_t> sat;   // (ny + 1) x (nx + 1) prefix sums
    int64_t box(int x0, int x1, int y0, int y1) const {   // [x0, x1) x [y0, y1) inside the grid
        const size_t W = (size_t)nx + 1;
        return (int64_t)sat[y1 * W + x1] - sat[y0 * W + x1] - sat[y1 * W + x0] + sat[y0 * W + x0];
    }
    // cells of [x0, x1) x [y0, y1) in region coordinates: periodic axes wrap,
    // others end at the grid (cells beyond it hold nothing)
    int64_t count(int x0, int x1, int y0, int y1) const {
        int xs[4], ys[4];
        const int nxs = segments(x0, x1, nx, perx, xs), nys = segments(y0, y1, ny, pery, ys);
        int64_t n = 0;
        for (int a = 0; a < nxs; ++a)
            for (int b = 0; b < nys; ++b) n += box(xs[2 * a], xs[2 * a + 1], ys[2 * b], ys[2 * b + 1]);
        return n;
    }
    // the interval [lo, hi) as at most two [begin, end) pairs inside [0, n)
    static int segments(int lo, int hi, int n, bool periodic, int* out) {
        if (hi <= lo) return 0;
        if (!periodic) {
            out[0] = std::max(lo, 0);
            out[1] = std::min(hi, n);
            return out[0] < out[1] ? 1 : 0;
        }
        if (hi - lo >= n) {
            out[0] = 0;
            out[1] = n;
            return 1;
        }
        const int a = ((lo % n) + n) % n, len = hi - lo;
        out[0] = a;
        if (a + len <= n) {
            out[1] = a + len;
            return 1;
        }
        out[1] = n;
        out[2] = 0;
        out[3] = a + len - n;
        return 2;
    }
};

ELive make_elive(const cf::Problem& p, int pol) {
    ELive e;
    e.nx = p.nx;
    e.ny = p.ny;
    e.perx = p.grid.bc[0] == CF_BC_PERIODIC;
    e.pery = p.grid.bc[1] == CF_BC_PERIODIC;
    std::vector<int> comps = pol == CF_POL_TM ? std::vector<int>{CF_EZ} : std::vector<int>{CF_EX, CF_EY};
    const size_t W = (size_t)p.nx + 1;
    e.sat.assign((size_t)(p.ny + 1) * W, 0);
    for (int y = 0; y < p.ny; ++y) {
        int32_t row = 0;
        for (int x = 0; x < p.nx; ++x) {
            const int64_t c = (int64_t)y * p.nx + x;
            bool live = false;
            for (int comp : comps) {
                const int id = p.ids[comp][c];
                live = live || (id != cf::kWallId && id < p.nmat && std::isfinite(p.eps[id]));
            }
            row += live ? 1 : 0;
            e.sat[(y + 1) * W + x + 1] = e.sat[y * W + x + 1] + row;
        }
    }
    return e;
}

TBPlan plan_tiles(const cf::Problem& p, const std::vector<cf::Channel>& chans, cf::TBShape sh,
                  const ELive* el);

std::vector<cf::Channel> selected_channels(const cf::Problem& p, const cf_opts& o, std::string* err) {
    std::vector<cf::Channel> all = cf::channel_table(p, o.pol);
    if (o.n_subset <= 0 || !o.channel_subset) return all;
    std::vector<cf::Channel> out;
    for (int k = 0; k < o.n_subset; ++k) {
        int c = o.channel_subset[k];
        if (c < 0 || c >= (int)all.size()) {
            *err = "channel_subset index out of range";
            return {};
        }
        out.push_back(all[c]);
    }
    return out;
}

// Tilings of a problem for a channel set and precision, kept per problem
// (the search over tiling origins costs tens of milliseconds on the larger
// grids, and a solve stages its problem several times).  The key is the
// problem's unique id, the precision, the polarizations run and the box of
// every surface stencil point, which decide the plans.
std::mutex g_plan_mu;
std::map<std::vector<int64_t>, std::vector<TBPlan>> g_plans;

std::vector<TBPlan> cached_plans(const cf::Problem& p, const std::vector<cf::Channel>& chans, int precision,
                                 const std::vector<cf::TBShape>& shapes) {
    int xmin = p.nx, xmax = -1, ymin = p.ny, ymax = -1, pols = 0;
    for (const auto& ch : chans) {
        pols |= ch.pol;
        const cf::Gather& g = p.gathers[p.gather_of.at({ch.face, ch.meas})];
        for (int32_t idx : g.idx) {
            xmin = std::min(xmin, idx % p.nx);
            xmax = std::max(xmax, idx % p.nx);
            ymin = std::min(ymin, idx / p.nx);
            ymax = std::max(ymax, idx / p.nx);
        }
    }
    const std::vector<int64_t> key = {(int64_t)p.uid, precision, pols, xmin, xmax, ymin, ymax};
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_plans.find(key);
        if (it != g_plans.end()) return it->second;
    }
    const ELive el[2] = {make_elive(p, CF_POL_TM), make_elive(p, CF_POL_TE)};
    std::vector<TBPlan> plans;
    for (const cf::TBShape& sh : shapes) plans.push_back(plan_tiles(p, chans, sh, el));
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_plans.size() >= 1024) g_plans.clear();
    g_plans[key] = plans;
    return plans;
}

// 3D: for every (plane z, row y), whether some E component of the row can be
// nonzero (coefficients not a = b = 0), row-major [z][y]; kept per problem
// (a scan of every cell).
std::map<uint64_t, std::vector<uint8_t>> g_erows;

std::vector<uint8_t> e_live_rows(const cf::Problem& p) {
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        auto it = g_erows.find(p.uid);
        if (it != g_erows.end()) return it->second;
    }
    std::vector<uint8_t> rows((size_t)p.nz * p.ny, 0);
    for (int c = CF_EX; c <= CF_EZ; ++c)
        for (int64_t k = 0; k < p.ncell; ++k) {
            const int id = p.ids[c][k];
            if (id != cf::kWallId && id < p.nmat && std::isfinite(p.eps[id])) rows[k / p.nx] = 1;
        }
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (g_erows.size() >= 64) g_erows.clear();
    g_erows[p.uid] = rows;
    return rows;
}

void forget_plans(uint64_t uid) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) it = (uint64_t)it->first[0] == uid ? g_plans.erase(it) : std::next(it);
    g_erows.erase(uid);
}

// Per band of each fused 3D variant, the planes [lo, hi) the band's region
// (its rows plus one halo row per step on either side) can change: E can be
// nonzero only on planes kmin..kmax where some E component of those rows has
// nonzero coefficients, H only on kmin - 1..kmax (its z difference reads the
// next plane); outside, every field stays 0 and the kernel skips the planes.
void stage_zranges(const cf::Problem& p, Staged& st) {
    const std::vector<uint8_t> rows = e_live_rows(p);
    const bool pery = p.grid.bc[1] == CF_BC_PERIODIC;
    st.zr.clear();
    std::vector<uint8_t> live(p.nz);
    for (int v = 0; v < cf::f3d_variants() && v < 8; ++v) {
        int W, B, steps;
        cf::f3d_shape(v, &W, &B, &steps);
        st.zr_off[v] = (int)(st.zr.size() / 2);
        const int band = W * B - 2 * steps;
        if (band <= 0) continue;
        const int nb = (p.ny + band - 1) / band;
        for (int b = 0; b < nb; ++b) {
            std::fill(live.begin(), live.end(), 0);
            for (int ry = 0; ry < W * B; ++ry) {
                int y = b * band - steps + ry;
                if (y < 0 || y >= p.ny) {
                    if (!pery) continue;
                    y = ((y % p.ny) + p.ny) % p.ny;
                }
                for (int z = 0; z < p.nz; ++z) live[z] |= rows[(size_t)z * p.ny + y];
            }
            int kmin = -1, kmax = -1;
            for (int z = 0; z < p.nz; ++z)
                if (live[z]) {
                    if (kmin < 0) kmin = z;
                    kmax = z;
                }
            st.zr.push_back(kmin < 0 ? 0 : std::max(kmin - 1, 0));
            st.zr.push_back(kmin < 0 ? 0 : kmax + 1);
        }
    }
}

// Build host copies of every table a solve uploads.  Channels run in waves
// of `resident` consecutive channels; channel c uses field block c % resident.
void stage(const cf::Problem& p, const cf_opts& o, const std::vector<cf::Channel>& chans, Staged& st) {
    st.chans = chans;
    st.ncomp = cf::n_comp(p);
    const int C = (int)chans.size();
    const bool plain = o.path == CF_PATH_PLAIN;
    st.resident = plain ? 1 : (o.max_resident > 0 ? std::min(o.max_resident, C) : C);
    st.resident = std::max(st.resident, 1);
    const int P = p.grid.ndim == 3 && p.grid.bc[2] == CF_BC_PML ? p.grid.pml_cells[2] : 0;
    st.psi_comp = (int64_t)2 * P * p.nx * p.ny;
    st.psi_block = 4 * st.psi_comp;
    if (p.grid.ndim == 2) {
        // in-plane CPML (split kernels): an x and a y layer array per field slot
        const int px = p.grid.bc[0] == CF_BC_PML ? p.grid.pml_cells[0] : 0;
        const int py = p.grid.bc[1] == CF_BC_PML ? p.grid.pml_cells[1] : 0;
        st.pml2d = px > 0 || py > 0;
        st.psi2d_slot = (int64_t)p.ny * 2 * px + (int64_t)2 * py * p.nx;
        st.psi_block = st.pml2d ? (int64_t)st.ncomp * st.psi2d_slot : 0;
    }
    // concatenated gather / scatter tables for every (face, comp) pair used
    std::vector<int> g_goff(p.gathers.size(), -1), g_uoff(p.gathers.size(), -1);
    auto add_gather = [&](int gi) {
        if (g_goff[gi] >= 0) return;
        const cf::Gather& g = p.gathers[gi];
        g_goff[gi] = (int)st.gidx.size();
        st.gidx.insert(st.gidx.end(), g.idx.begin(), g.idx.end());
        st.gw.insert(st.gw.end(), g.w.begin(), g.w.end());
        g_uoff[gi] = (int)st.uidx.size();
        const int base = (int)st.usamp.size();
        st.uidx.insert(st.uidx.end(), g.uidx.begin(), g.uidx.end());
        // uoff holds one entry per distinct point plus a trailing one, offsets
        // global into usamp/uw; uidx gets a pad entry to stay index-aligned.
        for (size_t k = 0; k < g.uoff.size(); ++k) st.uoff.push_back(base + g.uoff[k]);
        st.uidx.push_back(0);
        st.usamp.insert(st.usamp.end(), g.usamp.begin(), g.usamp.end());
        st.uw.insert(st.uw.end(), g.uw.begin(), g.uw.end());
    };
    std::vector<int> basis_face_off(p.faces.size());
    for (size_t f = 0; f < p.faces.size(); ++f) {
        basis_face_off[f] = (int)st.basis.size();
        st.basis.insert(st.basis.end(), p.basis[f].begin(), p.basis[f].end());
    }
    // waves: consecutive runs of `resident` channels; the split cylindrical
    // path groups the channels by azimuthal order first (one order per wave),
    // the resident cylindrical kernel takes any mix of orders
    // the resident reduced kernels carry no CPML and no polarizations
    st.red_res = p.reduced() && !plain && !(o.flags & CF_FLAG_SPLIT) && !p.dispersive && !st.pml2d;
    std::vector<std::vector<int>> wave_lists;
    std::vector<int> wave_order;
    {
        std::vector<std::vector<int>> groups;
        if (p.reduced() && !st.red_res) {
            groups.assign(p.n_orders(), {});
            for (int c = 0; c < C; ++c) groups[chans[c].order].push_back(c);
        } else {
            groups.emplace_back();
            for (int c = 0; c < C; ++c) groups[0].push_back(c);
        }
        for (size_t gi = 0; gi < groups.size(); ++gi)
            for (size_t k0 = 0; k0 < groups[gi].size(); k0 += st.resident) {
                const size_t k1 = std::min(groups[gi].size(), k0 + st.resident);
                wave_lists.emplace_back(groups[gi].begin() + k0, groups[gi].begin() + k1);
                wave_order.push_back(p.reduced() && !st.red_res ? (int)gi : -1);
            }
    }
    std::vector<int> block_of(C, 0);
    for (const auto& wl : wave_lists)
        for (size_t k = 0; k < wl.size(); ++k) block_of[wl[k]] = (int)k;
    // dispersive media: (P^m, P^{m-1}) per E slot (Cartesian: two, the TE
    // count; k_z runs: three per part) and term
    const int e_slots = p.reduced() ? 3 * (p.bloch ? 2 : 1) : 2;
    st.aux_block = p.dispersive ? (int64_t)e_slots * p.n_lor * 2 * p.ncell : 0;
    const double res = p.grid.res;
    for (int c = 0; c < C; ++c) {
        const cf::Channel& ch = chans[c];
        int gm = p.gather_of.at({ch.face, cf::gather_key(p, ch.meas, ch.order)});
        int gs = p.gather_of.at({ch.face, cf::gather_key(p, ch.src, ch.order)});
        add_gather(gm);
        add_gather(gs);
        const int blk = block_of[c];
        cf::ChanDev d{};
        d.field_off = (int64_t)blk * st.ncomp * p.ncell;
        d.psi_off = (int64_t)blk * st.psi_block;
        d.aux_off = (int64_t)blk * st.aux_block;
        d.src_off = d.field_off + (int64_t)cf::comp_slot(ch.pol, ch.src) * p.ncell;
        d.meas_off = d.field_off + (int64_t)cf::comp_slot(ch.pol, ch.meas) * p.ncell;
        d.kind = ch.kind;
        d.order = ch.order;
        d.inst = 0;
        d.pol = ch.pol;
        d.local = c;
        d.nsamp = p.gathers[gm].nsamp;
        d.P = p.gathers[gm].P;
        d.g_off = g_goff[gm];
        d.u_off = g_uoff[gs];
        d.n_uniq = (int)p.gathers[gs].uidx.size();
        d.basis_off = basis_face_off[ch.face] + ch.row * p.faces[ch.face].nsamp;
        d.meas_slot = cf::comp_slot(ch.pol, ch.meas);
        d.kick_scale = -res / (ch.kind == 0 ? p.eps_s : p.mu_s);
        if (c == 0 && (o.flags & CF_FLAG_INJECT_NAN)) d.kick_scale = std::nan("");
        st.max_uniq = std::max(st.max_uniq, d.n_uniq);
        st.dev.push_back(d);
    }
    for (size_t wi = 0; wi < wave_lists.size(); ++wi) {
        const std::vector<int>& wl = wave_lists[wi];
        Wave w{};
        w.order = wave_order[wi];
        auto add = [&](int pol, int* off, int* n) {
            *off = (int)st.slot_lists.size();
            for (int c : wl)
                if (pol == 0 || chans[c].pol == pol) st.slot_lists.push_back(c);
            *n = (int)st.slot_lists.size() - *off;
        };
        add(CF_POL_TM, &w.tm_off, &w.n_tm);
        add(CF_POL_TE, &w.te_off, &w.n_te);
        add(CF_POL_3D, &w.d3_off, &w.n_3d);
        add(0, &w.all_off, &w.n_all);
        st.waves.push_back(w);
    }
    if (p.reduced()) return;   // no fused 2D / 3D kernels for reduced problems
    if (!plain && p.grid.ndim == 3 && !(o.flags & CF_FLAG_SPLIT)) {
        cf::Grid3D g{};
        g.nx = p.nx;
        g.ny = p.ny;
        g.nz = p.nz;
        for (int a = 0; a < 3; ++a) g.per[a] = p.grid.bc[a] == CF_BC_PERIODIC;
        const int nv = cf::f3d_variants();
        auto usable = [&](int v) {
            return o.precision == CF_FP64 ? cf::f3d_usable<double>(v, g) : cf::f3d_usable<float>(v, g);
        };
        if (o.tile_variant >= 1 && o.tile_variant <= nv && usable(o.tile_variant - 1)) {
            st.f3d = true;
            st.v3d = o.tile_variant - 1;
        } else {
            for (int v = 0; v < nv; ++v) st.f3d = st.f3d || usable(v);
        }
        if (st.f3d && !st.gidx.empty()) {
            // bounding box of every surface stencil point (all gathers)
            int lo[3] = {p.nx, p.ny, p.nz}, hi[3] = {-1, -1, -1};
            for (int32_t ix : st.gidx) {
                const int c[3] = {(int)(ix % p.nx), (int)((ix / p.nx) % p.ny), (int)(ix / ((int64_t)p.nx * p.ny))};
                for (int a = 0; a < 3; ++a) {
                    lo[a] = std::min(lo[a], c[a]);
                    hi[a] = std::max(hi[a], c[a]);
                }
            }
            cf::ShadowBox& b = st.sbox;
            b.x0 = lo[0];
            b.y0 = lo[1];
            b.z0 = lo[2];
            b.bnx = hi[0] - lo[0] + 1;
            b.bny = hi[1] - lo[1] + 1;
            b.bnz = hi[2] - lo[2] + 1;
            b.vol = (int64_t)b.bnx * b.bny * b.bnz;
        }
        if (st.v3d >= 0 && cf::f3d_steps(st.v3d) == 2 && st.sbox.vol <= 0) st.v3d = cf::f3d_single(st.v3d);
        if (st.f3d) stage_zranges(p, st);
    }
    // the fused kernel carries no polarizations and no CPML: dispersive
    // problems and problems with in-plane layers take the split kernels
    if (!plain && p.grid.ndim == 2 && !(o.flags & CF_FLAG_SPLIT) && !p.dispersive && !st.pml2d) {
        cf::TBShape sh[cf::kMaxVariants];
        const int nv = o.precision == CF_FP64 ? cf::tb_variants<double>(sh, cf::kMaxVariants)
                                              : cf::tb_variants<float>(sh, cf::kMaxVariants);
        for (int v = 0; v < nv; ++v) st.shapes.push_back(sh[v]);
        st.plans = cached_plans(p, chans, o.precision, st.shapes);
        if (o.tile_variant >= 1 && o.tile_variant <= nv && st.plans[o.tile_variant - 1].ok) {
            st.variant = o.tile_variant - 1;
        } else {
            for (int v = 0; v < nv; ++v)
                if (st.plans[v].ok) {
                    st.variant = v;   // provisional: the autotuner may replace it
                    break;
                }
        }
        if (st.variant >= 0) st.tb = st.plans[st.variant];
    }
}

// ---- autotuner cache: "key variant" lines ---------------------------------

std::string tune_key(const cf::Problem& p, const cf_opts& o, int n_tm, int n_te) {
    std::ostringstream k;
    k << "2d fp" << (o.precision == CF_FP64 ? 64 : 32) << " " << p.nx << "x" << p.ny << " tm" << n_tm << " te"
      << n_te;
    return k.str();
}

bool tune_lookup(const std::string& key, int* v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) {
        g_tune_loaded = true;
        if (const char* path = std::getenv("CF_AUTOTUNE_CACHE")) {
            std::ifstream f(path);
            std::string line;
            while (std::getline(f, line)) {
                const size_t at = line.rfind(' ');
                if (at == std::string::npos) continue;
                g_tune[line.substr(0, at)] = std::atoi(line.c_str() + at + 1);
            }
        }
    }
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *v = it->second;
    return true;
}

void tune_store(const std::string& key, int v) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = v;
    if (const char* path = std::getenv("CF_AUTOTUNE_CACHE")) {
        std::ofstream f(path, std::ios::app);
        f << key << " " << v << "\n";
    }
}

// Tiling origins along one axis: every base in (-w, 0] for which the cells
// lo..hi (the surface stencil) lie in one tile of width w, with its tile
// count over 0..n-1, the tile holding lo..hi and the stencil's distance to
// the nearer edge of that tile.
struct AxisPlacement {
    int base, ntiles, stile, slack;
};

static std::vector<AxisPlacement> place_axis(int lo, int hi, int n, int w) {
    std::vector<AxisPlacement> out;
    if (hi - lo + 1 > w) return out;
    auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    for (int b = 0; b > -w; --b) {
        const int t = fdiv(lo - b, w);
        if (fdiv(hi - b, w) != t) continue;              // S straddles two tiles
        const int t0 = b + t * w;                         // first cell of S's tile
        out.push_back({b, (n - b + w - 1) / w, t, std::min(lo - t0, t0 + w - 1 - hi)});
    }
    return out;
}

// Live waves of the tiling t (base, tile counts and surface tile set) for
// polarization slot k; with fill, also its live tile list and live cells.  A
// wave is dead when its rows, and the first row above them, hold no E
// component that can be nonzero (the kernel's own test; above the region's
// top wave lie only stale rim rows).  The surface tile always runs.
static long live_waves(const cf::Problem& p, TBPlan& t, const cf::TBShape& sh, const ELive& el, int k,
                       bool fill) {
    const int RW = sh.tx + 2 * sh.kh, RH = sh.ty + 2 * sh.kh, W = RH / sh.b;
    long n = 0;
    if (fill) {
        t.live[k].clear();
        t.live_cells[k] = 0;
    }
    std::vector<char> zero(W);
    for (int tile = 0; tile < t.ntx * t.nty; ++tile) {
        const int rx0 = t.base_x + (tile % t.ntx) * sh.tx - sh.kh;
        const int ry0 = t.base_y + (tile / t.ntx) * sh.ty - sh.kh;
        for (int w = 0; w < W; ++w) zero[w] = el.count(rx0, rx0 + RW, ry0 + w * sh.b, ry0 + (w + 1) * sh.b) == 0;
        bool any = false;
        uint32_t mask = 0;
        for (int w = 0; w < W; ++w) {
            if (zero[w] && (w + 1 == W || zero[w + 1])) continue;   // advances nothing
            any = true;
            mask |= 1u << w;
            ++n;
            if (!fill) continue;
            // tile-interior cells of the wave inside the grid
            const int y0 = std::max({ry0 + w * sh.b, ry0 + sh.kh, 0});
            const int y1 = std::min({ry0 + (w + 1) * sh.b, ry0 + sh.kh + sh.ty, p.ny});
            const int x0 = std::max(rx0 + sh.kh, 0), x1 = std::min(rx0 + sh.kh + sh.tx, p.nx);
            if (y1 > y0 && x1 > x0) t.live_cells[k] += (double)(y1 - y0) * (x1 - x0);
        }
        if (!any && tile == t.stile) ++n;
        if (fill && (any || tile == t.stile)) t.live[k].push_back({tile, mask});
    }
    return n;
}

// Tiling of the fused kernel for the channels' surface stencils.  Among the
// origins that keep every stencil point in one tile, the one with the fewest
// live waves (summed over the polarizations run) is taken, then the fewest
// tiles, then the stencil most centred in its tile: first along y with x at
// its fewest-tiles origin, then along x at the chosen y.
TBPlan plan_tiles(const cf::Problem& p, const std::vector<cf::Channel>& chans, cf::TBShape sh,
                  const ELive* el) {
    TBPlan t;
    if (p.grid.ndim != 2 || p.reduced() || chans.empty()) return t;
    // the fused kernel forms the surface sum with its first four waves
    if ((sh.ty + 2 * sh.kh) / sh.b < 4) return t;
    int xmin = p.nx, xmax = -1, ymin = p.ny, ymax = -1;
    bool pol_used[2] = {false, false};
    for (const auto& ch : chans) {
        pol_used[ch.pol == CF_POL_TE ? 1 : 0] = true;
        const cf::Gather& g = p.gathers[p.gather_of.at({ch.face, ch.meas})];
        for (int32_t idx : g.idx) {
            const int x = idx % p.nx, y = idx / p.nx;
            xmin = std::min(xmin, x);
            xmax = std::max(xmax, x);
            ymin = std::min(ymin, y);
            ymax = std::max(ymax, y);
        }
    }
    const std::vector<AxisPlacement> px = place_axis(xmin, xmax, p.nx, sh.tx);
    const std::vector<AxisPlacement> py = place_axis(ymin, ymax, p.ny, sh.ty);
    if (px.empty() || py.empty()) return t;
    auto fewest = [](const std::vector<AxisPlacement>& v) {
        AxisPlacement best = v[0];
        for (const auto& a : v)
            if (a.ntiles < best.ntiles || (a.ntiles == best.ntiles && a.slack > best.slack)) best = a;
        return best;
    };
    auto set = [&](const AxisPlacement& ax, const AxisPlacement& ay) {
        t.base_x = ax.base;
        t.ntx = ax.ntiles;
        t.base_y = ay.base;
        t.nty = ay.ntiles;
        t.stile = ay.stile * t.ntx + ax.stile;
    };
    auto cost = [&]() {
        long n = 0;
        for (int k = 0; k < 2; ++k)
            if (pol_used[k]) n += live_waves(p, t, sh, el[k], k, false);
        return n;
    };
    auto better = [](long c, const AxisPlacement& a, long bc, const AxisPlacement& b) {
        if (c != bc) return c < bc;
        if (a.ntiles != b.ntiles) return a.ntiles < b.ntiles;
        return a.slack > b.slack;
    };
    AxisPlacement bx = fewest(px), by = py[0];
    long bcost = -1;
    for (const auto& ay : py) {
        set(bx, ay);
        const long c = cost();
        if (bcost < 0 || better(c, ay, bcost, by)) {
            bcost = c;
            by = ay;
        }
    }
    bcost = -1;
    AxisPlacement bx2 = bx;
    for (const auto& ax : px) {
        set(ax, by);
        const long c = cost();
        if (bcost < 0 || better(c, ax, bcost, bx2)) {
            bcost = c;
            bx2 = ax;
        }
    }
    set(bx2, by);
    t.ok = true;
    for (int k = 0; k < 2; ++k) live_waves(p, t, sh, el[k], k, true);
    return t;
}

// Work list of a fused launch: channel `slots[k]` contributes ntiles[k]
// tiles.  Each channel is assigned whole to the XCD queue with the fewest
// tiles so far; block b = 8 i + x takes item i of queue x, so every tile of
// a channel runs on XCD x (blocks are dispatched to XCDs round-robin).
std::vector<cf::WorkItem> make_work(const std::vector<int>& slots, const std::vector<const std::vector<LiveTile>*>& tiles,
                                    const std::vector<int>& stile) {
    std::vector<std::vector<cf::WorkItem>> q(8);
    std::vector<long> load(8, 0);
    for (size_t k = 0; k < slots.size(); ++k) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        const std::vector<LiveTile>& tl = *tiles[k];
        const LiveTile* s = nullptr;
        for (const LiveTile& t : tl)
            if (t.tile == stile[k]) s = &t;
        if (s) q[x].push_back({slots[k], s->tile, s->waves});
        for (const LiveTile& t : tl)
            if (t.tile != stile[k]) q[x].push_back({slots[k], t.tile, t.waves});
        load[x] += (long)tl.size();
    }
    size_t len = 0;
    for (auto& v : q) len = std::max(len, v.size());
    std::vector<cf::WorkItem> out(8 * len, cf::WorkItem{-1, 0, 0u});
    for (int x = 0; x < 8; ++x)
        for (size_t i = 0; i < q[x].size(); ++i) out[8 * i + x] = q[x][i];
    return out;
}

// Channel groups per polarization that a fused 2D solve runs on streams of
// their own (each group's work list is padded separately).  One group per
// polarization (TM and TE on two streams) took the 400x200 piston solve from
// 227 to 168 ms; two groups per polarization (four streams) measured 171 ms.
constexpr int kPolGroups = 1;

size_t work_capacity(int resident, int max_tiles) {
    return (size_t)8 * ((size_t)resident * max_tiles / 8 + kPolGroups * (max_tiles + 1));
}

Layout layout_for(const cf::Problem& p, const cf_opts& o, const Staged& st) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t fsz = o.precision == CF_FP64 ? 8 : 4;
    const size_t C = st.chans.size();
    const size_t block = (size_t)st.resident * st.ncomp * p.ncell * fsz;
    L.ids = take((size_t)cf::kNumComp * p.ncell);
    const size_t n_orders = (size_t)p.n_orders();   // reduced problems: one table per order
    L.lut = take(n_orders * 2 * cf::kNumComp * 256 * 2 * fsz);
    const int t_max = cf::max_steps(p, o);
    L.ktab = take(n_orders * (size_t)t_max * 8);
    L.pml = take((size_t)4 * p.nz * 8);
    L.chans = take(C * sizeof(cf::ChanDev));
    L.slots = take(st.slot_lists.size() * sizeof(int) + 4);
    L.gidx = take(st.gidx.size() * 4 + 4);
    L.gw = take(st.gw.size() * 8 + 8);
    L.uidx = take(st.uidx.size() * 4 + 4);
    L.uoff = take(st.uoff.size() * 4 + 4);
    L.usamp = take(st.usamp.size() * 4 + 4);
    L.uw = take(st.uw.size() * 8 + 8);
    L.basis = take(st.basis.size() * 8 + 8);
    L.acc = take(C * 2 * 8);
    L.gamma = (o.flags & CF_FLAG_KEEP_GAMMA) ? take((size_t)t_max * C * 8) : off;
    L.fields = take(block);
    L.fields2 = st.variant >= 0 || st.f3d ? take(block) : off;
    L.psi = st.psi_block > 0 ? take((size_t)st.resident * st.psi_block * fsz) : off;
    L.pml2 = st.pml2d ? take((size_t)p.n_orders() * 4 * (p.nx + p.ny) * 8) : off;   // per order: its time step
    L.psi2 = st.psi_comp > 0 && st.f3d ? take((size_t)st.resident * 4 * st.psi_comp * fsz) : off;
    L.idp = st.f3d ? take((size_t)p.ncell * 8) : st.red_res ? take((size_t)p.ncell * 4) : off;
    L.shadow = st.f3d && st.sbox.vol > 0 ? take((size_t)st.resident * st.sbox.vol * fsz) : off;
    L.rinv = p.reduced() ? take((size_t)6 * p.ny * fsz) : off;
    int max_tiles = 0;
    for (const TBPlan& pl : st.plans)
        if (pl.ok) max_tiles = std::max(max_tiles, pl.ntx * pl.nty);
    L.work_items = max_tiles ? work_capacity(st.resident, max_tiles) : 0;
    L.inst = take(sizeof(cf::InstDev));
    L.work = take(2 * L.work_items * sizeof(cf::WorkItem) + 8);
    L.aux = st.aux_block ? take((size_t)st.resident * st.aux_block * fsz) : off;
    L.zr = st.zr.empty() ? off : take(st.zr.size() * 4 + 8);
    L.lor = p.dispersive ? take((size_t)256 * cf::kLorStride(p.n_lor) * 8) : off;
    L.total = off;
    return L;
}

// Per material id: [flag, 1/eps_inf, (c1, c2, c3) per term] of the centred
// Lorentz update P^{m+1} = c1 P^m - c2 P^{m-1} + c3 E^m on the conductivity
// contour (damping sigma): c1 = (2 - (w0 dt)^2)/(1 + r), c2 = (1 - r)/(1 + r),
// c3 = d_eps (w0 dt)^2/(1 + r), r = sigma dt / 2.  Conductors and ids
// without terms have flag 0.
std::vector<double> lorentz_table(const cf::Problem& p, double sigma, double courant) {
    const int stride = cf::kLorStride(p.n_lor);
    std::vector<double> t((size_t)256 * stride, 0.0);
    const double dt = courant / p.grid.res, r = 0.5 * sigma * dt;
    for (int id = 0; id < p.nmat; ++id) {
        if (!p.has_terms(id) || !std::isfinite(p.eps[id])) continue;
        double* row = t.data() + (size_t)id * stride;
        row[0] = 1.0;
        row[1] = 1.0 / p.eps[id];
        for (int j = 0; j < p.n_lor; ++j) {
            const double de = p.lor_de[(size_t)id * p.n_lor + j], w = p.lor_w0[(size_t)id * p.n_lor + j] * dt;
            row[2 + 3 * j] = de != 0.0 ? (2.0 - w * w) / (1.0 + r) : 0.0;
            row[3 + 3 * j] = de != 0.0 ? (1.0 - r) / (1.0 + r) : 0.0;
            row[4 + 3 * j] = de * w * w / (1.0 + r);
        }
    }
    return t;
}


// Sampled HIP-event timing of field-update launches on the solve's stream.
struct Sampler {
    std::vector<hipEvent_t> ev;
    int taken = 0, seen = 0, stride = 1;
    double bytes = 0, cu = 0;
    bool on = false;
    bool begin(hipStream_t s) {
        const bool take = on && seen % stride == 0 && taken < (int)ev.size() / 2;
        if (take) (void)hipEventRecord(ev[2 * taken], s);
        return take;
    }
    void end(bool take, hipStream_t s, double launch_cu, double launch_bytes) {
        ++seen;
        if (!take) return;
        (void)hipEventRecord(ev[2 * taken + 1], s);
        ++taken;
        cu += launch_cu;
        bytes += launch_bytes;
    }
};

// Optional capture of a launch sequence into a HIP graph (CF_FLAG_GRAPH).
// The launches are captured on a private stream (the caller's stream may be
// the null stream, which cannot be captured); end() instantiates the graph
// and launches it once on the caller's stream.  Graphs and the private
// stream live until the object dies, after the caller has drained its stream.
struct GraphRun {
    bool on = false;
    hipStream_t cap = nullptr;
    std::vector<hipGraph_t> graphs;
    std::vector<hipGraphExec_t> execs;
    // stream the captured launches are issued on
    hipStream_t launch_stream(hipStream_t s) const { return on ? cap : s; }
    hipError_t begin() {
        if (!on) return hipSuccess;
        if (!cap) {
            const hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
        }
        return hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    }
    hipError_t end(hipStream_t s, hipError_t body) {
        if (!on) return body;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(cap, &g);   // the capture ends whatever the body did
        if (g) graphs.push_back(g);
        if (body != hipSuccess) return body;
        if (ec != hipSuccess) return ec;
        hipGraphExec_t x = nullptr;
        const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) return ei;
        execs.push_back(x);
        return hipGraphLaunch(x, s);
    }
    GraphRun() = default;
    GraphRun(const GraphRun&) = delete;
    GraphRun& operator=(const GraphRun&) = delete;
    ~GraphRun() {
        for (auto x : execs) (void)hipGraphExecDestroy(x);
        for (auto g : graphs) (void)hipGraphDestroy(g);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// Extra streams for the channel groups of a fused 2D solve, forked from and
// joined back to the solve's stream with events; released (after draining)
// on scope exit.  Default priority, like every stream here.
struct SideStreams {
    std::vector<hipStream_t> s;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    // n streams and their events (before any graph capture begins)
    hipError_t create(int n) {
        hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int k = 0; k < n && e == hipSuccess; ++k) {
            hipStream_t x = nullptr;
            hipEvent_t j = nullptr;
            e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
            if (e != hipSuccess) break;
            s.push_back(x);
            e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
            if (e != hipSuccess) break;
            join.push_back(j);
        }
        return e;
    }
    // the streams start after everything issued on main so far (inside a
    // capture this makes them branches of the graph)
    hipError_t open(hipStream_t main) {
        hipError_t e = hipEventRecord(fork, main);
        for (size_t k = 0; k < s.size() && e == hipSuccess; ++k) e = hipStreamWaitEvent(s[k], fork, 0);
        return e;
    }
    hipError_t close(hipStream_t main) {
        hipError_t e = hipSuccess;
        for (size_t k = 0; k < s.size() && e == hipSuccess; ++k) {
            e = hipEventRecord(join[k], s[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(main, join[k], 0);
        }
        return e;
    }
    SideStreams() = default;
    SideStreams(const SideStreams&) = delete;
    SideStreams& operator=(const SideStreams&) = delete;
    ~SideStreams() {
        for (hipStream_t x : s) {
            (void)hipStreamSynchronize(x);
            (void)hipStreamDestroy(x);
        }
        if (fork) (void)hipEventDestroy(fork);
        for (hipEvent_t j : join) (void)hipEventDestroy(j);
    }
};

// Reduced solve (cylindrical orders m, or k_z points q).  Every order has
// its own coefficient table, K(t_k) and coupling (a cylindrical order its
// own time step and step count).  Resident path: one launch
// per wave, each block carrying one channel (any order) through all its
// steps.  Split path (CF_FLAG_SPLIT, plain): waves of one order each; per
// wave clear, kick, consistent start, then per step the H and E half steps
// and the surface projection with the g-weighted accumulation.
void pml_order(const cf::Problem& p, const Layout& L, char* ws, cf::Grid2D& g, int m);

// In-plane CPML of a 2D problem (split kernels): uploads the x and y
// profiles for the time step of every order (cylindrical orders m >= 2 step
// with a smaller Courant number; the other problems have one order or one
// time step) and points the grid at order 0's and at the psi blocks
// (pml_order moves it to another order's).  tab holds the host copy until
// the solve has synchronized.
hipError_t set_pml2d(const cf::Problem& p, const cf_opts& o, const Staged& st, const Layout& L, char* ws,
                     hipStream_t s, cf::Grid2D& g, std::vector<double>& tab) {
    tab.clear();
    for (int m = 0; m < p.n_orders(); ++m)
        for (int a = 0; a < 2; ++a) cf::pml_axis_tables(p, a, cf::order_courant(p, o.courant, m), tab);
    g.psi = ws + L.psi;
    g.psi_slot = st.psi2d_slot;
    pml_order(p, L, ws, g, 0);
    return hipMemcpyAsync(ws + L.pml2, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s);
}

// Points the grid's CPML profiles at order m's (the layout of set_pml2d).
void pml_order(const cf::Problem& p, const Layout& L, char* ws, cf::Grid2D& g, int m) {
    const size_t per_axis[2] = {p.grid.bc[0] == CF_BC_PML ? 4 * (size_t)p.nx : 0,
                                p.grid.bc[1] == CF_BC_PML ? 4 * (size_t)p.ny : 0};
    const double* base = reinterpret_cast<const double*>(ws + L.pml2) + (size_t)m * (per_axis[0] + per_axis[1]);
    g.pml[0] = per_axis[0] ? p.grid.pml_cells[0] : 0;
    g.pml[1] = per_axis[1] ? p.grid.pml_cells[1] : 0;
    g.pml_tab[0] = base;
    g.pml_tab[1] = base + per_axis[0];
}

template <typename T>
cf_status run_reduced(const cf::Problem& p, const cf_opts& o, const Staged& st, const Layout& L, char* ws,
                  hipStream_t s, std::vector<double>& acc_out, std::vector<double>& gamma_out, double* device_ms,
                  StencilTiming* timing) {
    const size_t C = st.chans.size();
    const int t_max = cf::max_steps(p, o);
    std::vector<uint8_t> ids((size_t)cf::kNumComp * p.ncell);
    for (int c = 0; c < cf::kNumComp; ++c)
        std::memcpy(ids.data() + (size_t)c * p.ncell, p.ids[c].data(), p.ncell);
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    CF_HIP(up(L.ids, ids.data(), ids.size()));
    CF_HIP(up(L.chans, st.dev.data(), st.dev.size() * sizeof(cf::ChanDev)));
    CF_HIP(up(L.slots, st.slot_lists.data(), st.slot_lists.size() * sizeof(int)));
    CF_HIP(up(L.gidx, st.gidx.data(), st.gidx.size() * 4));
    CF_HIP(up(L.gw, st.gw.data(), st.gw.size() * 8));
    CF_HIP(up(L.uidx, st.uidx.data(), st.uidx.size() * 4));
    CF_HIP(up(L.uoff, st.uoff.data(), st.uoff.size() * 4));
    CF_HIP(up(L.usamp, st.usamp.data(), st.usamp.size() * 4));
    CF_HIP(up(L.uw, st.uw.data(), st.uw.size() * 8));
    CF_HIP(up(L.basis, st.basis.data(), st.basis.size() * 8));
    CF_HIP(hipMemsetAsync(ws + L.acc, 0, C * 2 * 8, s));
    const bool keep_gamma = (o.flags & CF_FLAG_KEEP_GAMMA) != 0;
    if (keep_gamma) CF_HIP(hipMemsetAsync(ws + L.gamma, 0, (size_t)t_max * C * 8, s));

    T* fields = reinterpret_cast<T*>(ws + L.fields);
    const cf::ChanDev* dch = reinterpret_cast<const cf::ChanDev*>(ws + L.chans);
    const int* dslots = reinterpret_cast<const int*>(ws + L.slots);
    const T* dlut = reinterpret_cast<const T*>(ws + L.lut);
    const double* dk = reinterpret_cast<const double*>(ws + L.ktab);
    double* dacc = reinterpret_cast<double*>(ws + L.acc);
    double* dgam = keep_gamma ? reinterpret_cast<double*>(ws + L.gamma) : nullptr;
    cf::SurfTables tabs;
    tabs.gidx = reinterpret_cast<const int32_t*>(ws + L.gidx);
    tabs.gw = reinterpret_cast<const double*>(ws + L.gw);
    tabs.uidx = reinterpret_cast<const int32_t*>(ws + L.uidx);
    tabs.uoff = reinterpret_cast<const int32_t*>(ws + L.uoff);
    tabs.usamp = reinterpret_cast<const int32_t*>(ws + L.usamp);
    tabs.uw = reinterpret_cast<const double*>(ws + L.uw);
    tabs.basis = reinterpret_cast<const double*>(ws + L.basis);
    const uint8_t* dids = reinterpret_cast<const uint8_t*>(ws + L.ids);
    cf::Grid2D g{};
    g.nx = p.nx;
    g.ny = p.ny;
    g.ncell = p.ncell;
    g.perx = p.grid.bc[0] == CF_BC_PERIODIC;
    g.pery = p.grid.bc[1] == CF_BC_PERIODIC;   // k_z problems only (the tube wall is PEC)
    for (int c = 0; c < cf::kNumComp; ++c) g.ids[c] = dids + (size_t)c * p.ncell;
    std::vector<double> lor;
    if (p.dispersive) {   // k_z runs (split kernels); every order shares the Courant number
        lor = lorentz_table(p, o.sigma, o.courant);
        CF_HIP(up(L.lor, lor.data(), lor.size() * 8));
        g.n_lor = p.n_lor;
        g.lor = reinterpret_cast<const double*>(ws + L.lor);
        g.aux = ws + L.aux;
    }
    std::vector<double> pml2_host;
    if (st.pml2d) CF_HIP(set_pml2d(p, o, st, L, ws, s, g, pml2_host));
    const size_t aux_bytes = (size_t)st.resident * st.aux_block * sizeof(T);
    const size_t psi_bytes = (size_t)st.resident * st.psi_block * sizeof(T);
    const double dA = 1.0 / p.grid.res;       // line element of the two-dimensional plane
    const size_t field_bytes = (size_t)st.resident * st.ncomp * p.ncell * sizeof(T);
    const double state_bytes = 2.0 * st.ncomp * sizeof(T);
    // per-order tables: coefficients for courant_m, K(t_k) on dt_m
    const size_t lut_len = 2 * cf::kNumComp * 256 * 2;
    cf::RedOrders ord{};
    ord.lut = dlut;
    ord.lut_stride = (int64_t)lut_len;
    ord.ktab = dk;
    ord.ktab_stride = t_max;
    const int n_ord = p.n_orders();
    std::vector<T> luts(lut_len * n_ord);
    std::vector<double> ktabs((size_t)t_max * n_ord, 0.0);
    for (int m = 0; m < n_ord; ++m) {
        const double cm = cf::order_courant(p, o.courant, m);
        ord.steps[m] = cf::order_steps(p, o, m);
        ord.dt[m] = cm / p.grid.res;
        ord.coup[m] = p.coupling(m);
        const double phi = p.bloch ? p.kxs[m] * p.nx / p.grid.res : 0.0;   // k_x L
        ord.ph_c[m] = std::cos(phi);
        ord.ph_s[m] = std::sin(phi);
        std::vector<double> l64 = cf::coefficient_lut(p, o.sigma, cm);
        std::copy(l64.begin(), l64.end(), luts.begin() + m * lut_len);
        cf::kernel_table(o.kernel, o.sigma, ord.dt[m], ord.steps[m], ktabs.data() + (size_t)m * t_max);
    }
    ord.axis = p.cyl ? 1 : 0;
    ord.cplx = p.bloch ? 1 : 0;

    CF_HIP(up(L.lut, luts.data(), luts.size() * sizeof(T)));
    CF_HIP(up(L.ktab, ktabs.data(), ktabs.size() * 8));
    // row factors in the field precision (A, B, C, D, P, Q per row):
    // cylindrical (j + 1/2, j - 1/2, 1/j, 1/(j - 1/2), j, j - 1) with row 0
    // on the axis (unused); k_z all 1
    std::vector<T> rows(6 * (size_t)p.ny, p.cyl ? T(0) : T(1));
    if (p.cyl)
        for (int j = 1; j < p.ny; ++j) {
            const T r = T(j);
            rows[6 * j + 0] = r + T(0.5);
            rows[6 * j + 1] = r - T(0.5);
            rows[6 * j + 2] = T(1) / r;
            rows[6 * j + 3] = T(1) / (r - T(0.5));
            rows[6 * j + 4] = r;
            rows[6 * j + 5] = r - T(1);
        }
    CF_HIP(up(L.rinv, rows.data(), rows.size() * sizeof(T)));
    ord.rows = ws + L.rinv;
    const T* drows = reinterpret_cast<const T*>(ws + L.rinv);
    // material ids packed in 4 bits per component for the register kernel
    // (15 = wall id), when every id fits
    std::vector<uint32_t> idw;
    if (st.red_res) {
        idw.assign(p.ncell, 0u);
        bool fits = true;
        for (int c = 0; c < cf::kNumComp && fits; ++c)
            for (int64_t k = 0; k < p.ncell; ++k) {
                const int id = p.ids[c][k];
                if (id >= 15 && id != cf::kWallId) {
                    fits = false;
                    break;
                }
                idw[k] |= uint32_t(id == cf::kWallId ? 15 : id) << (4 * c);
            }
        if (fits) {
            CF_HIP(up(L.idp, idw.data(), idw.size() * 4));
            ord.idw = reinterpret_cast<const uint32_t*>(ws + L.idp);
        }
    }

    hipEvent_t e0, e1;
    CF_HIP(hipEventCreate(&e0));
    CF_HIP(hipEventCreate(&e1));
    Sampler smp;
    smp.on = (o.flags & CF_FLAG_TIME_STENCIL) != 0;
    if (smp.on) {
        smp.ev.resize(2 * 256);
        for (auto& e : smp.ev) CF_HIP(hipEventCreate(&e));
        long total = 0;
        for (const Wave& w : st.waves) total += st.red_res ? 1 : cf::order_steps(p, o, w.order);
        smp.stride = std::max(1L, total / 200);
    }
    hipError_t err = hipSuccess;
    timing->variant = -1;     // resident variant - 1 (-1: split path)
    // time-convergence stop (resident kernels, one wave): the run goes in
    // parts of stop_every steps on the base axis (each order its share of
    // its own steps, red_step_at); F(T') is checked after each part
    cfi::ConvergenceStop conv;
    conv.on = o.stop_tol > 0 && st.waves.size() == 1 && st.red_res && o.path != CF_PATH_PLAIN;
    conv.tol = o.stop_tol;
    conv.every = conv.next = o.stop_every > 0 ? o.stop_every : 500;
    int steps_run = o.n_steps;
    std::vector<double> acc_probe;
#define STEP_OK(expr)                     \
    do {                                  \
        err = (expr);                     \
        if (err != hipSuccess) goto done; \
    } while (0)
    STEP_OK(hipEventRecord(e0, s));
    for (const Wave& w : st.waves) {
        const int* sl = dslots + w.all_off;
        if (st.red_res) {
            // one launch per part: every channel of the wave, any mix of orders
            for (int d0 = 0; d0 < o.n_steps;) {
                const int d1 = conv.on ? std::min(o.n_steps, d0 + conv.every) : o.n_steps;
                const cf::RedSpan span = cf::red_span(ord, n_ord, d0, d1, o.n_steps);
                double cu = 0;
                for (int k = 0; k < w.n_all; ++k) {
                    const int m = st.chans[st.slot_lists[w.all_off + k]].order;
                    cu += (double)p.ncell * (span.s1[m] - span.s0[m]);
                }
                const bool take = smp.begin(s);
                int used = 0;
                STEP_OK(cf::launch_red_resident_span<T>(o.tile_variant, fields, dch, sl, w.n_all, g, ord, span, tabs,
                                                        dA, dacc, dgam, (int)C, s, &used));
                smp.end(take, s, cu, cu * state_bytes);
                timing->variant = std::max(timing->variant, used - 1);
                d0 = d1;
                if (conv.on && d1 < o.n_steps) {
                    conv.next += conv.every;
                    acc_probe.assign(C * 2, 0.0);
                    STEP_OK(hipMemcpyAsync(acc_probe.data(), dacc, C * 2 * 8, hipMemcpyDeviceToHost, s));
                    STEP_OK(hipStreamSynchronize(s));
                    if (conv.update(acc_probe, st.chans)) {
                        steps_run = d1;
                        break;
                    }
                }
            }
            continue;
        }
        const int m = w.order;
        const int tm = ord.steps[m];
        const double dt = ord.dt[m];
        if (st.pml2d) pml_order(p, L, ws, g, m);
        const T* lut_m = dlut + m * lut_len;
        const double* k_m = dk + (size_t)m * t_max;
        STEP_OK(hipMemsetAsync(fields, 0, field_bytes, s));
        if (psi_bytes) STEP_OK(hipMemsetAsync(ws + L.psi, 0, psi_bytes, s));
        if (aux_bytes) STEP_OK(hipMemsetAsync(ws + L.aux, 0, aux_bytes, s));
        STEP_OK(cf::launch_kick<T>(fields, dch, sl, w.n_all, st.max_uniq, tabs, s));
        STEP_OK(cf::launch_hred<T>(1, ord.coup[m], ord.axis, fields, dch, sl, w.n_all, g, lut_m, drows, ord.ph_c[m],
                                   ord.ph_s[m], ord.cplx, s));
        STEP_OK(cf::launch_ered<T>(1, ord.coup[m], ord.axis, fields, dch, sl, w.n_all, g, lut_m, drows, ord.ph_c[m],
                                   ord.ph_s[m], ord.cplx, s));
        for (int k = 0; k < tm; ++k) {
            const bool take = smp.begin(s);
            STEP_OK(cf::launch_hred<T>(0, ord.coup[m], ord.axis, fields, dch, sl, w.n_all, g, lut_m, drows,
                                       ord.ph_c[m], ord.ph_s[m], ord.cplx, s));
            STEP_OK(cf::launch_ered<T>(0, ord.coup[m], ord.axis, fields, dch, sl, w.n_all, g, lut_m, drows,
                                       ord.ph_c[m], ord.ph_s[m], ord.cplx, s));
            const double cu = (double)w.n_all * p.ncell;
            smp.end(take, s, cu, cu * state_bytes);
            STEP_OK(cf::launch_surface<T>(fields, dch, sl, w.n_all, tabs, k_m, k, dt, dA, dacc, dgam, (int)C, s));
        }
    }
    STEP_OK(hipEventRecord(e1, s));
    STEP_OK(hipEventSynchronize(e1));
    {
        float ms = 0;
        STEP_OK(hipEventElapsedTime(&ms, e0, e1));
        *device_ms = ms;
    }
    if (smp.on) {
        double tot = 0;
        for (int k = 0; k < smp.taken; ++k) {
            float ms = 0;
            STEP_OK(hipEventElapsedTime(&ms, smp.ev[2 * k], smp.ev[2 * k + 1]));
            tot += ms;
        }
        timing->samples = smp.taken;
        timing->ms_total = tot;
        timing->bytes_total = smp.bytes;
        timing->cu_total = smp.cu;
        timing->launches = smp.seen;
    }
    timing->steps_run = steps_run;
    acc_out.assign(C * 2, 0.0);
    // copies on the solve's own stream: a non-blocking caller stream is not
    // ordered with the null stream
    STEP_OK(hipMemcpyAsync(acc_out.data(), ws + L.acc, C * 2 * 8, hipMemcpyDeviceToHost, s));
    if (keep_gamma) {
        gamma_out.assign((size_t)t_max * C, 0.0);
        STEP_OK(hipMemcpyAsync(gamma_out.data(), ws + L.gamma, gamma_out.size() * 8, hipMemcpyDeviceToHost, s));
    }
    STEP_OK(hipStreamSynchronize(s));
done:
#undef STEP_OK
    if (err != hipSuccess) (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto& e : smp.ev) (void)hipEventDestroy(e);
    if (err != hipSuccess)
        return fail(CF_E_DEVICE, std::string("device step failed: ") + hipGetErrorString(err));
    return CF_OK;
}

template <typename T>
cf_status run_solve(const cf::Problem& p, const cf_opts& o, const Staged& st, const Layout& L,
                    char* ws, hipStream_t s, std::vector<double>& acc_out, std::vector<double>& gamma_out,
                    double* device_ms, StencilTiming* timing) {
    if (p.reduced()) return run_reduced<T>(p, o, st, L, ws, s, acc_out, gamma_out, device_ms, timing);
    const size_t C = st.chans.size();
    // ---- upload tables --------------------------------------------------
    std::vector<uint8_t> ids((size_t)cf::kNumComp * p.ncell);
    for (int c = 0; c < cf::kNumComp; ++c)
        std::memcpy(ids.data() + (size_t)c * p.ncell, p.ids[c].data(), p.ncell);
    std::vector<double> lut64 = cf::coefficient_lut(p, o.sigma, o.courant);
    std::vector<T> lut(lut64.begin(), lut64.end());
    std::vector<double> ktab(o.n_steps);
    cf::kernel_table(o.kernel, o.sigma, o.courant / p.grid.res, o.n_steps, ktab.data());
    std::vector<double> bh, chh, be, ce, pml;
    cf::pml_tables(p, o.courant, bh, chh, be, ce);
    pml.insert(pml.end(), bh.begin(), bh.end());
    pml.insert(pml.end(), chh.begin(), chh.end());
    pml.insert(pml.end(), be.begin(), be.end());
    pml.insert(pml.end(), ce.begin(), ce.end());
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    CF_HIP(up(L.ids, ids.data(), ids.size()));
    CF_HIP(up(L.lut, lut.data(), lut.size() * sizeof(T)));
    CF_HIP(up(L.ktab, ktab.data(), ktab.size() * 8));
    CF_HIP(up(L.pml, pml.data(), pml.size() * 8));
    CF_HIP(up(L.chans, st.dev.data(), st.dev.size() * sizeof(cf::ChanDev)));
    CF_HIP(up(L.slots, st.slot_lists.data(), st.slot_lists.size() * sizeof(int)));
    CF_HIP(up(L.gidx, st.gidx.data(), st.gidx.size() * 4));
    CF_HIP(up(L.gw, st.gw.data(), st.gw.size() * 8));
    CF_HIP(up(L.uidx, st.uidx.data(), st.uidx.size() * 4));
    CF_HIP(up(L.uoff, st.uoff.data(), st.uoff.size() * 4));
    CF_HIP(up(L.usamp, st.usamp.data(), st.usamp.size() * 4));
    CF_HIP(up(L.uw, st.uw.data(), st.uw.size() * 8));
    CF_HIP(up(L.basis, st.basis.data(), st.basis.size() * 8));
    std::vector<uint32_t> idp;
    if (st.f3d) {
        // material ids of the six components packed per cell for the fused 3D step
        idp.resize((size_t)p.ncell * 2);
        for (int64_t c = 0; c < p.ncell; ++c) {
            idp[2 * c] = uint32_t(p.ids[CF_EX][c]) | (uint32_t(p.ids[CF_EY][c]) << 8) |
                         (uint32_t(p.ids[CF_EZ][c]) << 16) | (uint32_t(p.ids[CF_HX][c]) << 24);
            idp[2 * c + 1] = uint32_t(p.ids[CF_HY][c]) | (uint32_t(p.ids[CF_HZ][c]) << 8);
        }
        CF_HIP(up(L.idp, idp.data(), idp.size() * 4));
        if (!st.zr.empty()) CF_HIP(up(L.zr, st.zr.data(), st.zr.size() * 4));
    }
    CF_HIP(hipMemsetAsync(ws + L.acc, 0, C * 2 * 8, s));
    const bool keep_gamma = (o.flags & CF_FLAG_KEEP_GAMMA) != 0;
    if (keep_gamma) CF_HIP(hipMemsetAsync(ws + L.gamma, 0, (size_t)o.n_steps * C * 8, s));
    std::vector<double> lor;
    if (p.dispersive) {
        lor = lorentz_table(p, o.sigma, o.courant);
        CF_HIP(up(L.lor, lor.data(), lor.size() * 8));
    }

    T* fields = reinterpret_cast<T*>(ws + L.fields);
    T* psi = st.psi_block > 0 ? reinterpret_cast<T*>(ws + L.psi) : nullptr;
    const cf::ChanDev* dch = reinterpret_cast<const cf::ChanDev*>(ws + L.chans);
    const int* dslots = reinterpret_cast<const int*>(ws + L.slots);
    const T* dlut = reinterpret_cast<const T*>(ws + L.lut);
    const double* dk = reinterpret_cast<const double*>(ws + L.ktab);
    const double* dpml = reinterpret_cast<const double*>(ws + L.pml);
    double* dacc = reinterpret_cast<double*>(ws + L.acc);
    double* dgam = keep_gamma ? reinterpret_cast<double*>(ws + L.gamma) : nullptr;
    cf::SurfTables tabs;
    tabs.gidx = reinterpret_cast<const int32_t*>(ws + L.gidx);
    tabs.gw = reinterpret_cast<const double*>(ws + L.gw);
    tabs.uidx = reinterpret_cast<const int32_t*>(ws + L.uidx);
    tabs.uoff = reinterpret_cast<const int32_t*>(ws + L.uoff);
    tabs.usamp = reinterpret_cast<const int32_t*>(ws + L.usamp);
    tabs.uw = reinterpret_cast<const double*>(ws + L.uw);
    tabs.basis = reinterpret_cast<const double*>(ws + L.basis);
    const uint8_t* dids = reinterpret_cast<const uint8_t*>(ws + L.ids);
    cf::Grid2D g{};
    g.nx = p.nx;
    g.ny = p.ny;
    g.ncell = p.ncell;
    g.perx = p.grid.bc[0] == CF_BC_PERIODIC;
    g.pery = p.grid.bc[1] == CF_BC_PERIODIC;
    for (int c = 0; c < cf::kNumComp; ++c) g.ids[c] = dids + (size_t)c * p.ncell;
    if (p.dispersive) {
        g.n_lor = p.n_lor;
        g.lor = reinterpret_cast<const double*>(ws + L.lor);
        g.aux = ws + L.aux;
    }
    std::vector<double> pml2_host;
    if (st.pml2d) CF_HIP(set_pml2d(p, o, st, L, ws, s, g, pml2_host));
    const size_t aux_bytes = (size_t)st.resident * st.aux_block * sizeof(T);
    cf::Grid3D g3{};
    g3.nx = p.nx;
    g3.ny = p.ny;
    g3.nz = p.nz;
    g3.ncell = p.ncell;
    for (int a = 0; a < 3; ++a) g3.per[a] = p.grid.bc[a] == CF_BC_PERIODIC;
    for (int c = 0; c < cf::kNumComp; ++c) g3.ids[c] = g.ids[c];
    g3.pml = p.grid.ndim == 3 && p.grid.bc[2] == CF_BC_PML ? p.grid.pml_cells[2] : 0;
    g3.psi_comp = st.psi_comp;
    g3.pml_bh = dpml;
    g3.pml_ch = dpml + p.nz;
    g3.pml_be = dpml + 2 * p.nz;
    g3.pml_ce = dpml + 3 * p.nz;
    g3.idp = st.f3d ? reinterpret_cast<const uint2*>(ws + L.idp) : nullptr;
    g3.zr_tab = st.f3d && !st.zr.empty() ? reinterpret_cast<const int2*>(ws + L.zr) : nullptr;
    for (int v = 0; v < 8; ++v) g3.zr_off[v] = st.zr_off[v];
    const double dt = o.courant / p.grid.res;
    const double dA = std::pow(1.0 / p.grid.res, p.grid.ndim - 1);
    const size_t field_bytes = (size_t)st.resident * st.ncomp * p.ncell * sizeof(T);
    const size_t psi_bytes = (size_t)st.resident * st.psi_block * sizeof(T);
    const double state_bytes = 2.0 * st.ncomp * sizeof(T);   // read + write of a cell's state
    const bool three = p.grid.ndim == 3;

    hipEvent_t e0, e1;
    CF_HIP(hipEventCreate(&e0));
    CF_HIP(hipEventCreate(&e1));
    Sampler smp;
    smp.on = (o.flags & CF_FLAG_TIME_STENCIL) != 0;
    if (smp.on) {
        smp.ev.resize(2 * 256);
        for (auto& e : smp.ev) CF_HIP(hipEventCreate(&e));
        const int kh = st.variant >= 0 ? st.shapes[st.variant].kh : 1;
        const int per_wave = st.variant >= 0 ? 2 * ((o.n_steps + kh - 1) / kh) : o.n_steps;
        smp.stride = std::max(1, per_wave * (int)st.waves.size() / 200);
    }
    auto make_inst = [&](const TBPlan& pl, bool with_gamma) {
        cf::InstDev I{};
        I.fa = fields;
        I.fb = ws + L.fields2;
        I.acc = dacc;
        I.nx = p.nx;
        I.ny = p.ny;
        I.ncell = p.ncell;
        I.perx = g.perx;
        I.pery = g.pery;
        for (int c = 0; c < cf::kNumComp; ++c) I.ids[c] = g.ids[c];
        I.lut = dlut;
        I.base_x = pl.base_x;
        I.base_y = pl.base_y;
        I.ntx = pl.ntx;
        I.nty = pl.nty;
        I.stile = pl.stile;
        I.start = 0;
        I.nsteps = o.n_steps;
        I.dt = dt;
        I.dA = dA;
        I.ktab = dk;
        I.gamma = with_gamma ? dgam : nullptr;
        I.gamma_stride = (int64_t)C;
        I.t = tabs;
        return I;
    };
    cf::InstDev* dinst = reinterpret_cast<cf::InstDev*>(ws + L.inst);
    cf::WorkItem* dwork = reinterpret_cast<cf::WorkItem*>(ws + L.work);
    // sources of asynchronous uploads: kept (at stable addresses) until the
    // stream has drained
    std::deque<std::vector<cf::WorkItem>> host_work;
    std::deque<cf::InstDev> host_inst;
    // work list of one wave's channels of one polarization for plan pl
    // work list of `list` at slot_off; it must end by region_end (both in items)
    auto upload_work = [&](const int* list, int n, const TBPlan& pl, int pol, size_t slot_off,
                           size_t region_end, int* nwork) -> hipError_t {
        std::vector<int> sl(list, list + n), st(n, pl.stile);
        std::vector<const std::vector<LiveTile>*> tl(n, &live_tiles(pl, pol));
        host_work.push_back(make_work(sl, tl, st));
        *nwork = (int)host_work.back().size();
        if (slot_off + (size_t)*nwork > region_end) return hipErrorInvalidValue;
        return hipMemcpyAsync(dwork + slot_off, host_work.back().data(), *nwork * sizeof(cf::WorkItem),
                              hipMemcpyHostToDevice, s);
    };
    auto upload_inst = [&](const cf::InstDev& I) -> hipError_t {
        host_inst.push_back(I);
        return hipMemcpyAsync(dinst, &host_inst.back(), sizeof(cf::InstDev), hipMemcpyHostToDevice, s);
    };
    int variant = st.variant;
    int v3 = st.v3d;                       // fused 3D variant (autotuned below when -1)
    hipError_t err = hipSuccess;
    GraphRun graph;
    graph.on = (o.flags & CF_FLAG_GRAPH) && !smp.on && !(o.stop_tol > 0);
    // time-convergence stop (one wave of resident channels only)
    cfi::ConvergenceStop conv;
    conv.on = o.stop_tol > 0 && st.waves.size() == 1 && o.path != CF_PATH_PLAIN;
    conv.tol = o.stop_tol;
    conv.every = conv.next = o.stop_every > 0 ? o.stop_every : 500;
    int steps_run = o.n_steps;
    std::vector<double> acc_probe;
    // after `done` steps: true when the run has converged (syncs the stream)
    auto converged = [&](int done) -> bool {
        if (!conv.on || done < conv.next || done >= o.n_steps) return false;
        while (conv.next <= done) conv.next += conv.every;
        acc_probe.assign(C * 2, 0.0);
        if (hipMemcpyAsync(acc_probe.data(), dacc, C * 2 * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return false;
        if (!conv.update(acc_probe, st.chans)) return false;
        steps_run = done;
        return true;
    };
#define STEP_OK(expr)                     \
    do {                                  \
        err = (expr);                     \
        if (err != hipSuccess) goto done; \
    } while (0)
    if (variant >= 0 && o.tile_variant == 0 && !st.waves.empty()) {
        // autotune: time every applicable variant on this solve's own buffers
        // (fields, accumulators and Gamma are reset before the real run)
        const Wave& w = st.waves[0];
        const bool tm = w.n_tm >= w.n_te;
        const int n = tm ? w.n_tm : w.n_te;
        const std::string key = tune_key(p, o, w.n_tm, w.n_te);
        int cached;
        if (tune_lookup(key, &cached) && cached >= 0 && cached < (int)st.plans.size() && st.plans[cached].ok) {
            variant = cached;
        } else if (n > 0) {
            double best = 1e300;
            hipEvent_t t0, t1;
            STEP_OK(hipEventCreate(&t0));
            STEP_OK(hipEventCreate(&t1));
            for (int v = 0; v < (int)st.plans.size(); ++v) {
                if (!st.plans[v].ok) continue;
                const int kh = st.shapes[v].kh;
                int nw = 0;
                STEP_OK(upload_inst(make_inst(st.plans[v], false)));
                const int pol = tm ? CF_POL_TM : CF_POL_TE;
                STEP_OK(upload_work(st.slot_lists.data() + (tm ? w.tm_off : w.te_off), n, st.plans[v], pol, 0,
                                    L.work_items, &nw));
                STEP_OK(cf::launch_tb2d<T>(v, pol, dch, dwork, nw, dinst, kh, 0, 0, s));
                STEP_OK(hipEventRecord(t0, s));
                for (int r = 0; r < 3; ++r) STEP_OK(cf::launch_tb2d<T>(v, pol, dch, dwork, nw, dinst, kh, 0, r & 1, s));
                STEP_OK(hipEventRecord(t1, s));
                STEP_OK(hipEventSynchronize(t1));
                float ms = 0;
                STEP_OK(hipEventElapsedTime(&ms, t0, t1));
                const double per_cu = ms / (3.0 * n * (double)p.ncell * kh);
                if (per_cu < best) {
                    best = per_cu;
                    variant = v;
                }
            }
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            tune_store(key, variant);
        }
        STEP_OK(hipMemsetAsync(ws + L.acc, 0, C * 2 * 8, s));
    }
    timing->variant = variant;
    if (st.f3d && !st.waves.empty()) {
        auto usable3 = [&](int v) {
            return v >= 0 && cf::f3d_usable<T>(v, g3) && (cf::f3d_steps(v) == 1 || st.sbox.vol > 0);
        };
        const Wave& w0 = st.waves[0];
        const std::string key = tune_key(p, o, 0, w0.n_3d) + " f3d";
        int cached;
        if (v3 < 0 && tune_lookup(key, &cached) && usable3(cached)) v3 = cached;
        if (v3 < 0) {
            // time every usable variant on this solve's buffers (the fields
            // are cleared again when the first wave starts)
            STEP_OK(hipMemsetAsync(fields, 0, field_bytes, s));
            T* fb = reinterpret_cast<T*>(ws + L.fields2);
            T* pb = psi ? reinterpret_cast<T*>(ws + L.psi2) : nullptr;
            double best = 1e300;
            hipEvent_t t0, t1;
            STEP_OK(hipEventCreate(&t0));
            STEP_OK(hipEventCreate(&t1));
            T* sh = reinterpret_cast<T*>(ws + L.shadow);
            for (int v = 0; v < cf::f3d_variants(); ++v) {
                if (!usable3(v)) continue;
                const int* sl = dslots + w0.d3_off;
                STEP_OK(cf::launch_f3d<T>(v, dch, sl, w0.n_3d, g3, dlut, fields, fb, psi, pb, sh, st.sbox, s));
                STEP_OK(hipEventRecord(t0, s));
                for (int r = 0; r < 2; ++r)
                    STEP_OK(cf::launch_f3d<T>(v, dch, sl, w0.n_3d, g3, dlut, fields, fb, psi, pb, sh, st.sbox, s));
                STEP_OK(hipEventRecord(t1, s));
                STEP_OK(hipEventSynchronize(t1));
                float ms = 0;
                STEP_OK(hipEventElapsedTime(&ms, t0, t1));
                ms /= (float)cf::f3d_steps(v);      // per time step
                if (ms < best) {
                    best = ms;
                    v3 = v;
                }
            }
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            tune_store(key, v3);
        }
        timing->variant = v3;
    }
    STEP_OK(hipEventRecord(e0, s));
    for (const Wave& w : st.waves) {
        const int* s_tm = dslots + w.tm_off;
        const int* s_te = dslots + w.te_off;
        const int* s_3d = dslots + w.d3_off;
        const int* s_all = dslots + w.all_off;
        if (o.path == CF_PATH_PLAIN) {
            // plain: one channel at a time, three launches per step
            for (int k = 0; k < w.n_all; ++k) {
                const int* one = s_all + k;
                const int pol = st.chans[st.slot_lists[w.all_off + k]].pol;
                STEP_OK(hipMemsetAsync(fields, 0, field_bytes, s));
                if (psi) STEP_OK(hipMemsetAsync(psi, 0, psi_bytes, s));
                if (aux_bytes) STEP_OK(hipMemsetAsync(ws + L.aux, 0, aux_bytes, s));
                STEP_OK(cf::launch_kick<T>(fields, dch, one, 1, st.max_uniq, tabs, s));
                if (three) {
                    STEP_OK(cf::launch_h3d<T>(1, fields, psi, dch, one, 1, g3, dlut, s));
                    STEP_OK(cf::launch_e3d<T>(1, fields, psi, dch, one, 1, g3, dlut, s));
                } else {
                    STEP_OK(cf::launch_h2d<T>(pol, 1, fields, dch, one, 1, g, dlut, s));
                    STEP_OK(cf::launch_e2d<T>(pol, 1, fields, dch, one, 1, g, dlut, s));
                }
                for (int m = 0; m < o.n_steps; ++m) {
                    if (three) {
                        STEP_OK(cf::launch_h3d<T>(0, fields, psi, dch, one, 1, g3, dlut, s));
                        STEP_OK(cf::launch_e3d<T>(0, fields, psi, dch, one, 1, g3, dlut, s));
                    } else {
                        STEP_OK(cf::launch_h2d<T>(pol, 0, fields, dch, one, 1, g, dlut, s));
                        STEP_OK(cf::launch_e2d<T>(pol, 0, fields, dch, one, 1, g, dlut, s));
                    }
                    STEP_OK(cf::launch_surface<T>(fields, dch, one, 1, tabs, dk, m, dt, dA, dacc, dgam,
                                                  (int)C, s));
                }
            }
            continue;
        }
        // batched: kick and consistent start for the whole wave
        STEP_OK(hipMemsetAsync(fields, 0, field_bytes, s));
        if (psi) STEP_OK(hipMemsetAsync(psi, 0, psi_bytes, s));
        if (aux_bytes) STEP_OK(hipMemsetAsync(ws + L.aux, 0, aux_bytes, s));
        STEP_OK(cf::launch_kick<T>(fields, dch, s_all, w.n_all, st.max_uniq, tabs, s));
        if (three) {
            STEP_OK(cf::launch_h3d<T>(1, fields, psi, dch, s_3d, w.n_3d, g3, dlut, s));
            STEP_OK(cf::launch_e3d<T>(1, fields, psi, dch, s_3d, w.n_3d, g3, dlut, s));
        } else {
            STEP_OK(cf::launch_h2d<T>(CF_POL_TM, 1, fields, dch, s_tm, w.n_tm, g, dlut, s));
            STEP_OK(cf::launch_h2d<T>(CF_POL_TE, 1, fields, dch, s_te, w.n_te, g, dlut, s));
            STEP_OK(cf::launch_e2d<T>(CF_POL_TM, 1, fields, dch, s_tm, w.n_tm, g, dlut, s));
            STEP_OK(cf::launch_e2d<T>(CF_POL_TE, 1, fields, dch, s_te, w.n_te, g, dlut, s));
        }
        if (variant >= 0) {
            const TBPlan& pl = st.plans[variant];
            const int kh = st.shapes[variant].kh;
            int nw_tm = 0, nw_te = 0;
            STEP_OK(upload_inst(make_inst(pl, true)));
            // TM and TE channels, and channels among themselves, are
            // independent runs: without launch sampling or the convergence
            // stop each polarization's channels go in kPolGroups groups, each
            // with its own work list and stream (a parallel branch of the graph
            // when captured), so that the tail of one group's launch overlaps
            // the other groups' launches
            const bool split_pol = !smp.on && !conv.on && w.n_tm > 0 && w.n_te > 0;
            const int G = split_pol ? kPolGroups : 1;
            int gn[2][kPolGroups] = {}, gw[2][kPolGroups] = {};
            size_t goff[2][kPolGroups] = {};
            for (int q = 0; q < 2; ++q) {
                const int n = q == 0 ? w.n_tm : w.n_te;
                const int* list = st.slot_lists.data() + (q == 0 ? w.tm_off : w.te_off);
                size_t off = q == 0 ? 0 : L.work_items;
                for (int k = 0, first = 0; k < G; ++k) {
                    const int cnt = n / G + (k < n % G ? 1 : 0);
                    gn[q][k] = cnt;
                    goff[q][k] = off;
                    if (cnt > 0)
                        STEP_OK(upload_work(list + first, cnt, pl, q == 0 ? CF_POL_TM : CF_POL_TE, off,
                                            (q + 1) * L.work_items, &gw[q][k]));
                    off += gw[q][k];
                    first += cnt;
                }
            }
            nw_tm = gw[0][0];
            nw_te = gw[1][0];
            // cells the fused kernel skips are never written: both ping-pong
            // arrays start at zero there
            STEP_OK(hipMemsetAsync(ws + L.fields2, 0, field_bytes, s));
            SideStreams side;
            if (split_pol) STEP_OK(side.create(2 * G - 1));
            STEP_OK(graph.begin());
            const hipStream_t ls = graph.launch_stream(s);
            hipError_t fork_err = split_pol ? side.open(ls) : hipSuccess;
            const hipError_t body0 = fork_err != hipSuccess ? fork_err : [&]() -> hipError_t {
                int parity = 0;
                for (int m = 0; m < o.n_steps; m += kh) {
                    const int ks = std::min(kh, o.n_steps - m);
                    for (int q = 0; q < 2; ++q)
                        for (int k = 0; k < G; ++k) {
                            if (gn[q][k] == 0) continue;
                            // group 0 (and every group when not split) on the solve's stream
                            const int gi = q * G + k;
                            const hipStream_t ps = !split_pol || gi == 0 ? ls : side.s[gi - 1];
                            const bool take = smp.begin(ls);
                            const hipError_t e =
                                cf::launch_tb2d<T>(variant, q == 0 ? CF_POL_TM : CF_POL_TE, dch, dwork + goff[q][k],
                                                   gw[q][k], dinst, kh, m, parity, ps);
                            if (e != hipSuccess) return e;
                            const double cu = (double)gn[q][k] * p.ncell * ks;
                            smp.end(take, ls, cu, cu * state_bytes);
                        }
                    parity ^= 1;
                    if (converged(m + ks)) break;
                }
                return hipSuccess;
            }();
            hipError_t body = body0;
            if (split_pol && !side.s.empty()) {
                const hipError_t ec = side.close(ls);   // joins the branches before a capture ends
                if (body == hipSuccess) body = ec;
            }
            STEP_OK(graph.end(s, body));
        } else if (three && st.f3d) {
            // fused 3D: one launch per step, ping-pong between the two field
            // (and psi) arrays; the surface is read from the array just written
            T* fa = fields;
            T* fb = reinterpret_cast<T*>(ws + L.fields2);
            T* pa = psi;
            T* pb = psi ? reinterpret_cast<T*>(ws + L.psi2) : nullptr;
            if (pb) STEP_OK(hipMemsetAsync(pb, 0, psi_bytes, s));
            // planes the kernel skips are never written: zero in both arrays
            STEP_OK(hipMemsetAsync(fb, 0, field_bytes, s));
            T* sh = reinterpret_cast<T*>(ws + L.shadow);
            // a two-step variant takes steps in pairs (the surface of the first
            // step of a pair is read from the shadow box); an odd last step
            // runs on the single-step variant of the same band shape
            for (int m = 0; m < o.n_steps;) {
                const bool two = cf::f3d_steps(v3) == 2 && o.n_steps - m >= 2;
                const int v = two || cf::f3d_steps(v3) == 1 ? v3 : cf::f3d_single(v3);
                const bool take = smp.begin(s);
                STEP_OK(cf::launch_f3d<T>(v, dch, s_3d, w.n_3d, g3, dlut, fa, fb, pa, pb, sh, st.sbox, s));
                const double cu = (double)w.n_3d * p.ncell * (two ? 2 : 1);
                smp.end(take, s, cu, cu * state_bytes);
                if (two)
                    STEP_OK(cf::launch_surface_box<T>(sh, st.sbox, g3, dch, s_all, w.n_all, tabs, dk, m, dt, dA, dacc,
                                                      dgam, (int)C, s));
                m += two ? 2 : 1;
                STEP_OK(cf::launch_surface<T>(fb, dch, s_all, w.n_all, tabs, dk, m - 1, dt, dA, dacc, dgam, (int)C,
                                              s));
                std::swap(fa, fb);
                std::swap(pa, pb);
                if (converged(m)) break;
            }
        } else {
            for (int m = 0; m < o.n_steps; ++m) {
                const bool take = smp.begin(s);
                if (three) {
                    STEP_OK(cf::launch_h3d<T>(0, fields, psi, dch, s_3d, w.n_3d, g3, dlut, s));
                    STEP_OK(cf::launch_e3d<T>(0, fields, psi, dch, s_3d, w.n_3d, g3, dlut, s));
                } else {
                    STEP_OK(cf::launch_h2d<T>(CF_POL_TM, 0, fields, dch, s_tm, w.n_tm, g, dlut, s));
                    STEP_OK(cf::launch_h2d<T>(CF_POL_TE, 0, fields, dch, s_te, w.n_te, g, dlut, s));
                    STEP_OK(cf::launch_e2d<T>(CF_POL_TM, 0, fields, dch, s_tm, w.n_tm, g, dlut, s));
                    STEP_OK(cf::launch_e2d<T>(CF_POL_TE, 0, fields, dch, s_te, w.n_te, g, dlut, s));
                }
                const double cu = (double)w.n_all * p.ncell;
                smp.end(take, s, cu, cu * state_bytes);
                STEP_OK(cf::launch_surface<T>(fields, dch, s_all, w.n_all, tabs, dk, m, dt, dA, dacc, dgam,
                                              (int)C, s));
                if (converged(m + 1)) break;
            }
        }
    }
    STEP_OK(hipEventRecord(e1, s));
    STEP_OK(hipEventSynchronize(e1));
    {
        float ms = 0;
        STEP_OK(hipEventElapsedTime(&ms, e0, e1));
        *device_ms = ms;
    }
    if (smp.on) {
        double tot = 0;
        for (int k = 0; k < smp.taken; ++k) {
            float ms = 0;
            STEP_OK(hipEventElapsedTime(&ms, smp.ev[2 * k], smp.ev[2 * k + 1]));
            tot += ms;
        }
        timing->samples = smp.taken;
        timing->ms_total = tot;
        timing->bytes_total = smp.bytes;
        timing->cu_total = smp.cu;
        timing->launches = smp.seen;
    }
    timing->steps_run = steps_run;
    acc_out.assign(C * 2, 0.0);
    STEP_OK(hipMemcpyAsync(acc_out.data(), ws + L.acc, C * 2 * 8, hipMemcpyDeviceToHost, s));
    if (keep_gamma) {
        gamma_out.assign((size_t)o.n_steps * C, 0.0);
        STEP_OK(hipMemcpyAsync(gamma_out.data(), ws + L.gamma, gamma_out.size() * 8, hipMemcpyDeviceToHost, s));
    }
    STEP_OK(hipStreamSynchronize(s));
done:
#undef STEP_OK
    // host staging vectors die with this frame: drain the stream first
    if (err != hipSuccess) (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto& e : smp.ev) (void)hipEventDestroy(e);
    if (err != hipSuccess)
        return fail(CF_E_DEVICE, std::string("device step failed: ") + hipGetErrorString(err));
    return CF_OK;
}

// Host reduction (FP64, channel order): F = (1/pi) sum_c sign_c acc_c and
// the per-harmonic / per-face / per-channel / trace outputs.  Returns false
// when an accumulator is not finite.
bool fill_result(const cf::Problem& p, const std::vector<cf::Channel>& chans, const std::vector<double>& acc,
                 const std::vector<double>& gam, const cf_opts& o, double ms, const StencilTiming& tim,
                 const Staged& sg, cf_result* out) {
    const size_t C = chans.size();
    std::vector<double> a(C);
    bool finite = true;
    for (size_t c = 0; c < C; ++c) {
        a[c] = acc[2 * c] + acc[2 * c + 1];
        finite = finite && std::isfinite(a[c]);
    }
    double F = 0;
    for (size_t c = 0; c < C; ++c) F += chans[c].sign * a[c];
    out->force = F / M_PI;
    if (out->per_harmonic) {
        std::fill(out->per_harmonic, out->per_harmonic + out->per_harmonic_len, 0.0);
        for (size_t c = 0; c < C; ++c) out->per_harmonic[chans[c].label] += chans[c].sign * a[c] / M_PI;
    }
    if (out->per_face) {
        std::fill(out->per_face, out->per_face + out->per_face_len, 0.0);
        for (size_t c = 0; c < C; ++c)
            out->per_face[p.faces[chans[c].face].index] += chans[c].sign * a[c] / M_PI;
    }
    if (out->per_channel)
        for (size_t c = 0; c < C; ++c) out->per_channel[c] = a[c];
    if (out->gamma && !gam.empty()) std::copy(gam.begin(), gam.end(), out->gamma);
    if (out->trace && !gam.empty() && !p.reduced()) {
        std::vector<double> ktab(o.n_steps);
        const double dt = o.courant / p.grid.res;
        cf::kernel_table(o.kernel, o.sigma, dt, o.n_steps, ktab.data());
        double run = 0;
        for (int m = 0; m < o.n_steps; ++m) {
            double s = 0;
            for (size_t c = 0; c < C; ++c) s += chans[c].sign * gam[(size_t)m * C + c];
            run += dt * ktab[m] * s / M_PI;
            out->trace[m] = run;
        }
    }
    const int steps = tim.steps_run >= 0 ? tim.steps_run : o.n_steps;
    out->n_channels_run = (int)C;
    out->n_steps_run = steps;
    out->cell_updates = (double)C * (double)p.ncell * (double)steps;
    if (p.reduced()) {
        // each order runs its share of its own steps (all of them unless the
        // convergence stop ended the run after `steps` base steps)
        out->cell_updates = 0;
        for (size_t c = 0; c < C; ++c) {
            const int64_t tm = cf::order_steps(p, o, chans[c].order);
            const int64_t run = steps >= o.n_steps ? tm : (int64_t)steps * tm / o.n_steps;
            out->cell_updates += (double)p.ncell * (double)run;
        }
    }
    out->device_ms = ms;
    out->stencil_samples = tim.samples;
    out->stencil_launches = tim.launches;
    out->stencil_ms_avg = tim.samples ? tim.ms_total / tim.samples : 0.0;
    out->stencil_alg_bytes = tim.samples ? tim.bytes_total / tim.samples : 0.0;
    out->stencil_cell_updates = tim.samples ? tim.cu_total / tim.samples : 0.0;
    out->fused = tim.variant >= 0 ? 1 : 0;
    out->tile_variant = tim.variant + 1;
    out->tile_halo = tim.variant >= 0 && tim.variant < (int)sg.shapes.size() ? sg.shapes[tim.variant].kh : 0;
    out->advanced_cell_updates = out->cell_updates;
    if (tim.variant >= 0 && tim.variant < (int)sg.plans.size() && p.grid.ndim == 2 && !p.reduced()) {
        // the fused 2D kernel advances the live waves' tile interiors only
        const TBPlan& pl = sg.plans[tim.variant];
        double a = 0;
        for (size_t c = 0; c < C; ++c) a += pl.live_cells[chans[c].pol == CF_POL_TE ? 1 : 0];
        out->advanced_cell_updates = a * (double)steps;
    }
    if (tim.variant >= 0 && tim.variant < 8 && p.grid.ndim == 3 && sg.f3d && !sg.zr.empty()) {
        // the fused 3D steps advance each band's planes [z0, z1) only
        int W, B, ks;
        cf::f3d_shape(tim.variant, &W, &B, &ks);
        const int band = W * B - 2 * ks;
        if (band > 0) {
            const int nb = (p.ny + band - 1) / band;
            double cells = 0;
            for (int b = 0; b < nb; ++b) {
                const size_t k = 2 * ((size_t)sg.zr_off[tim.variant] + b);
                cells += (double)std::min(band, p.ny - b * band) * (sg.zr[k + 1] - sg.zr[k]) * p.nx;
            }
            out->advanced_cell_updates = cells * (double)C * (double)steps;
        }
    }
    return finite;
}

// ---------------------------------------------------------------------------
// Batched solve: several 2D problems advanced by one fused launch sequence.

struct BatchPlan {
    std::vector<const cf::Problem*> probs;
    std::vector<std::vector<cf::Channel>> chans;
    std::vector<Staged> st;
    std::vector<int> base;                 // first global channel slot per instance
    std::vector<cf::ChanDev> dev;          // all channels, global slots
    std::vector<int32_t> gidx, uidx, uoff, usamp;
    std::vector<double> gw, uw, basis;
    std::vector<int> all, tm, te;          // global slot lists
    std::vector<int> inst_tm_off, inst_tm_n, inst_te_off, inst_te_n;   // per instance, into `lists`
    std::vector<int> lists;                // all | tm | te | per-instance tm | per-instance te
    std::vector<size_t> ids_off, lut_off, ktab_off, field_off;
    size_t ids_bytes = 0, lut_bytes = 0, ktab_bytes = 0, field_elems = 0, work_items = 0;
    std::vector<int> variants_ok;          // variants every instance can use
    int max_uniq = 0;
    int C = 0;
};

std::string plan_batch(cf_problem* const* probs, int n, const cf_opts& o, BatchPlan& B) {
    cf_opts oo = o;
    oo.n_subset = 0;
    oo.channel_subset = nullptr;
    oo.max_resident = 0;
    oo.path = CF_PATH_BATCHED;
    oo.flags &= ~CF_FLAG_KEEP_GAMMA;
    const size_t fsz = o.precision == CF_FP64 ? 8 : 4;
    int nvar = -1;
    for (int i = 0; i < n; ++i) {
        const cf::Problem& p = probs[i]->p;
        B.probs.push_back(&p);
        B.chans.push_back(cf::channel_table(p, o.pol));
        B.st.emplace_back();
        stage(p, oo, B.chans.back(), B.st.back());
        const Staged& st = B.st.back();
        if (nvar < 0) nvar = (int)st.plans.size();
        if ((int)st.plans.size() != nvar) nvar = 0;
    }
    for (int v = 0; v < nvar; ++v) {
        bool ok = true;
        for (auto& st : B.st) ok = ok && st.plans[v].ok;
        if (ok) B.variants_ok.push_back(v);
    }
    if (B.variants_ok.empty()) return "no fused tile shape fits every problem";
    for (int i = 0; i < n; ++i) {
        const cf::Problem& p = *B.probs[i];
        const Staged& st = B.st[i];
        const int Ci = (int)B.chans[i].size();
        B.base.push_back(B.C);
        B.ids_off.push_back(B.ids_bytes);
        B.ids_bytes = align_up(B.ids_bytes + (size_t)cf::kNumComp * p.ncell, 256);
        B.lut_off.push_back(B.lut_bytes);
        B.lut_bytes = align_up(B.lut_bytes + 2 * cf::kNumComp * 256 * 2 * fsz, 256);
        B.ktab_off.push_back(B.ktab_bytes);
        B.ktab_bytes = align_up(B.ktab_bytes + (size_t)o.n_steps * 8, 256);
        B.field_off.push_back(B.field_elems);
        const int G = (int)B.gidx.size(), U = (int)B.uidx.size(), S = (int)B.usamp.size(),
                  Bo = (int)B.basis.size();
        B.gidx.insert(B.gidx.end(), st.gidx.begin(), st.gidx.end());
        B.gw.insert(B.gw.end(), st.gw.begin(), st.gw.end());
        B.uidx.insert(B.uidx.end(), st.uidx.begin(), st.uidx.end());
        for (int32_t v : st.uoff) B.uoff.push_back(v + S);
        B.usamp.insert(B.usamp.end(), st.usamp.begin(), st.usamp.end());
        B.uw.insert(B.uw.end(), st.uw.begin(), st.uw.end());
        B.basis.insert(B.basis.end(), st.basis.begin(), st.basis.end());
        for (int c = 0; c < Ci; ++c) {
            cf::ChanDev d = st.dev[c];
            d.field_off += (int64_t)B.field_elems;
            d.src_off += (int64_t)B.field_elems;
            d.meas_off += (int64_t)B.field_elems;
            d.local = B.C + c;   // the batch keeps one accumulator array and one field array
            d.g_off += G;
            d.u_off += U;
            d.basis_off += Bo;
            d.inst = i;
            B.dev.push_back(d);
            const int slot = B.C + c;
            B.all.push_back(slot);
            (B.chans[i][c].pol == CF_POL_TM ? B.tm : B.te).push_back(slot);
        }
        B.max_uniq = std::max(B.max_uniq, st.max_uniq);
        B.field_elems += (size_t)Ci * st.ncomp * p.ncell;
        B.C += Ci;
    }
    B.lists = B.all;
    B.lists.insert(B.lists.end(), B.tm.begin(), B.tm.end());
    B.lists.insert(B.lists.end(), B.te.begin(), B.te.end());
    for (int i = 0; i < n; ++i) {
        const int Ci = (int)B.chans[i].size();
        B.inst_tm_off.push_back((int)B.lists.size());
        for (int c = 0; c < Ci; ++c)
            if (B.chans[i][c].pol == CF_POL_TM) B.lists.push_back(B.base[i] + c);
        B.inst_tm_n.push_back((int)B.lists.size() - B.inst_tm_off.back());
        B.inst_te_off.push_back((int)B.lists.size());
        for (int c = 0; c < Ci; ++c)
            if (B.chans[i][c].pol == CF_POL_TE) B.lists.push_back(B.base[i] + c);
        B.inst_te_n.push_back((int)B.lists.size() - B.inst_te_off.back());
    }
    // work-list capacity for the largest variant
    size_t cap = 0;
    for (int v : B.variants_ok) {
        long tiles = 0;
        int tmax = 0;
        for (int i = 0; i < n; ++i) {
            const int t = B.st[i].plans[v].ntx * B.st[i].plans[v].nty;
            tiles += (long)t * (long)B.chans[i].size();
            tmax = std::max(tmax, t);
        }
        cap = std::max(cap, (size_t)(8 * (tiles / 8 + 2 * tmax + 1)));
    }
    B.work_items = cap;
    return "";
}

struct BatchLayout {
    size_t ids, lut, ktab, chans, lists, gidx, gw, uidx, uoff, usamp, uw, basis, acc, inst, work, fA, fB,
        total;
};

BatchLayout batch_layout(const BatchPlan& B, const cf_opts& o) {
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const size_t fsz = o.precision == CF_FP64 ? 8 : 4;
    L.ids = take(B.ids_bytes);
    L.lut = take(B.lut_bytes);
    L.ktab = take(B.ktab_bytes);
    L.chans = take(B.dev.size() * sizeof(cf::ChanDev));
    L.lists = take(B.lists.size() * sizeof(int) + 4);
    L.gidx = take(B.gidx.size() * 4 + 4);
    L.gw = take(B.gw.size() * 8 + 8);
    L.uidx = take(B.uidx.size() * 4 + 4);
    L.uoff = take(B.uoff.size() * 4 + 4);
    L.usamp = take(B.usamp.size() * 4 + 4);
    L.uw = take(B.uw.size() * 8 + 8);
    L.basis = take(B.basis.size() * 8 + 8);
    L.acc = take((size_t)B.C * 2 * 8);
    L.inst = take(B.probs.size() * sizeof(cf::InstDev));
    L.work = take(2 * B.work_items * sizeof(cf::WorkItem) + 8);
    L.fA = take(B.field_elems * fsz);
    L.fB = take(B.field_elems * fsz);
    L.total = off;
    return L;
}

template <typename T>
cf_status run_batch(const BatchPlan& B, const BatchLayout& L, const cf_opts& o, char* ws, hipStream_t s,
                    std::vector<double>& acc_out, double* device_ms, StencilTiming* timing) {
    const int n = (int)B.probs.size();
    std::deque<std::vector<uint8_t>> keep8;
    std::deque<std::vector<T>> keepT;
    std::deque<std::vector<double>> keepD;
    std::deque<std::vector<cf::WorkItem>> keepW;
    std::deque<std::vector<cf::InstDev>> keepI;
    auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    for (int i = 0; i < n; ++i) {
        const cf::Problem& p = *B.probs[i];
        keep8.emplace_back((size_t)cf::kNumComp * p.ncell);
        for (int c = 0; c < cf::kNumComp; ++c)
            std::memcpy(keep8.back().data() + (size_t)c * p.ncell, p.ids[c].data(), p.ncell);
        CF_HIP(up(L.ids + B.ids_off[i], keep8.back().data(), keep8.back().size()));
        std::vector<double> l64 = cf::coefficient_lut(p, o.sigma, o.courant);
        keepT.emplace_back(l64.begin(), l64.end());
        CF_HIP(up(L.lut + B.lut_off[i], keepT.back().data(), keepT.back().size() * sizeof(T)));
        keepD.emplace_back(o.n_steps);
        cf::kernel_table(o.kernel, o.sigma, o.courant / p.grid.res, o.n_steps, keepD.back().data());
        CF_HIP(up(L.ktab + B.ktab_off[i], keepD.back().data(), (size_t)o.n_steps * 8));
    }
    CF_HIP(up(L.chans, B.dev.data(), B.dev.size() * sizeof(cf::ChanDev)));
    CF_HIP(up(L.lists, B.lists.data(), B.lists.size() * sizeof(int)));
    CF_HIP(up(L.gidx, B.gidx.data(), B.gidx.size() * 4));
    CF_HIP(up(L.gw, B.gw.data(), B.gw.size() * 8));
    CF_HIP(up(L.uidx, B.uidx.data(), B.uidx.size() * 4));
    CF_HIP(up(L.uoff, B.uoff.data(), B.uoff.size() * 4));
    CF_HIP(up(L.usamp, B.usamp.data(), B.usamp.size() * 4));
    CF_HIP(up(L.uw, B.uw.data(), B.uw.size() * 8));
    CF_HIP(up(L.basis, B.basis.data(), B.basis.size() * 8));

    const cf::ChanDev* dch = reinterpret_cast<const cf::ChanDev*>(ws + L.chans);
    const int* dl = reinterpret_cast<const int*>(ws + L.lists);
    double* dacc = reinterpret_cast<double*>(ws + L.acc);
    cf::InstDev* dinst = reinterpret_cast<cf::InstDev*>(ws + L.inst);
    cf::WorkItem* dwork = reinterpret_cast<cf::WorkItem*>(ws + L.work);
    T* A = reinterpret_cast<T*>(ws + L.fA);
    T* Bf = reinterpret_cast<T*>(ws + L.fB);
    cf::SurfTables tabs;
    tabs.gidx = reinterpret_cast<const int32_t*>(ws + L.gidx);
    tabs.gw = reinterpret_cast<const double*>(ws + L.gw);
    tabs.uidx = reinterpret_cast<const int32_t*>(ws + L.uidx);
    tabs.uoff = reinterpret_cast<const int32_t*>(ws + L.uoff);
    tabs.usamp = reinterpret_cast<const int32_t*>(ws + L.usamp);
    tabs.uw = reinterpret_cast<const double*>(ws + L.uw);
    tabs.basis = reinterpret_cast<const double*>(ws + L.basis);
    auto grid_of = [&](int i) {
        const cf::Problem& p = *B.probs[i];
        cf::Grid2D g{};
        g.nx = p.nx;
        g.ny = p.ny;
        g.ncell = p.ncell;
        g.perx = p.grid.bc[0] == CF_BC_PERIODIC;
        g.pery = p.grid.bc[1] == CF_BC_PERIODIC;
        for (int c = 0; c < cf::kNumComp; ++c)
            g.ids[c] = reinterpret_cast<const uint8_t*>(ws + L.ids + B.ids_off[i]) + (size_t)c * p.ncell;
        return g;
    };
    auto insts_for = [&](int v) {
        std::vector<cf::InstDev> I(n);
        for (int i = 0; i < n; ++i) {
            const cf::Problem& p = *B.probs[i];
            const TBPlan& pl = B.st[i].plans[v];
            const cf::Grid2D g = grid_of(i);
            cf::InstDev& d = I[i];
            d.fa = A;
            d.fb = Bf;
            d.acc = dacc;
            d.nx = p.nx;
            d.ny = p.ny;
            d.ncell = p.ncell;
            d.perx = g.perx;
            d.pery = g.pery;
            for (int c = 0; c < cf::kNumComp; ++c) d.ids[c] = g.ids[c];
            d.lut = ws + L.lut + B.lut_off[i];
            d.base_x = pl.base_x;
            d.base_y = pl.base_y;
            d.ntx = pl.ntx;
            d.nty = pl.nty;
            d.stile = pl.stile;
            d.start = 0;
            d.nsteps = o.n_steps;
            d.dt = o.courant / p.grid.res;
            d.dA = std::pow(1.0 / p.grid.res, p.grid.ndim - 1);
            d.ktab = reinterpret_cast<const double*>(ws + L.ktab + B.ktab_off[i]);
            d.gamma = nullptr;
            d.gamma_stride = B.C;
            d.t = tabs;
        }
        return I;
    };
    auto work_for = [&](int v, const std::vector<int>& slots) {
        std::vector<const std::vector<LiveTile>*> tl;
        std::vector<int> st;
        for (int sl : slots) {
            const int i = B.dev[sl].inst;
            tl.push_back(&live_tiles(B.st[i].plans[v], B.dev[sl].pol));
            st.push_back(B.st[i].plans[v].stile);
        }
        return make_work(slots, tl, st);
    };
    const int n_tm = (int)B.tm.size(), n_te = (int)B.te.size();
    hipError_t err = hipSuccess;
    hipEvent_t e0, e1;
    CF_HIP(hipEventCreate(&e0));
    CF_HIP(hipEventCreate(&e1));
    int variant = B.variants_ok[0];
    const size_t fbytes = B.field_elems * sizeof(T);
    GraphRun graph;
    graph.on = (o.flags & CF_FLAG_GRAPH) != 0;
#define BSTEP(expr)                        \
    do {                                   \
        err = (expr);                      \
        if (err != hipSuccess) goto bdone; \
    } while (0)
    if (o.tile_variant >= 1) {
        variant = -1;
        for (int v : B.variants_ok)
            if (v == o.tile_variant - 1) variant = v;
        if (variant < 0) variant = B.variants_ok[0];
    } else if (B.variants_ok.size() > 1) {
        std::ostringstream k;
        k << "batch fp" << (sizeof(T) == 8 ? 64 : 32) << " n" << n << " ch" << B.C << " cells" << B.field_elems;
        int cached;
        if (tune_lookup(k.str(), &cached) &&
            std::find(B.variants_ok.begin(), B.variants_ok.end(), cached) != B.variants_ok.end()) {
            variant = cached;
        } else {
            double best = 1e300;
            for (int v : B.variants_ok) {
                keepI.push_back(insts_for(v));
                BSTEP(up(L.inst, keepI.back().data(), n * sizeof(cf::InstDev)));
                const std::vector<int>& sl = n_tm >= n_te ? B.tm : B.te;
                keepW.push_back(work_for(v, sl));
                BSTEP(up(L.work, keepW.back().data(), keepW.back().size() * sizeof(cf::WorkItem)));
                const int kh = B.st[0].shapes[v].kh, nw = (int)keepW.back().size();
                const int pol = n_tm >= n_te ? CF_POL_TM : CF_POL_TE;
                BSTEP(cf::launch_tb2d<T>(v, pol, dch, dwork, nw, dinst, kh, 0, 0, s));
                BSTEP(hipEventRecord(e0, s));
                for (int r = 0; r < 2; ++r) BSTEP(cf::launch_tb2d<T>(v, pol, dch, dwork, nw, dinst, kh, 0, r, s));
                BSTEP(hipEventRecord(e1, s));
                BSTEP(hipEventSynchronize(e1));
                float ms = 0;
                BSTEP(hipEventElapsedTime(&ms, e0, e1));
                const double per = ms / (2.0 * kh);
                if (per < best) {
                    best = per;
                    variant = v;
                }
            }
            tune_store(k.str(), variant);
        }
    }
    timing->variant = variant;
    {
        const int kh = B.st[0].shapes[variant].kh;
        keepI.push_back(insts_for(variant));
        BSTEP(up(L.inst, keepI.back().data(), n * sizeof(cf::InstDev)));
        keepW.push_back(work_for(variant, B.tm));
        const int nw_tm = (int)keepW.back().size();
        BSTEP(up(L.work, keepW.back().data(), nw_tm * sizeof(cf::WorkItem)));
        keepW.push_back(work_for(variant, B.te));
        const int nw_te = (int)keepW.back().size();
        BSTEP(up(L.work + B.work_items * sizeof(cf::WorkItem), keepW.back().data(), nw_te * sizeof(cf::WorkItem)));
        BSTEP(hipMemsetAsync(dacc, 0, (size_t)B.C * 2 * 8, s));
        BSTEP(hipMemsetAsync(A, 0, fbytes, s));
        BSTEP(hipMemsetAsync(Bf, 0, fbytes, s));   // cells the fused kernel skips stay zero in both arrays
        BSTEP(hipEventRecord(e0, s));
        BSTEP(cf::launch_kick<T>(A, dch, dl, B.C, B.max_uniq, tabs, s));
        for (int i = 0; i < n; ++i) {
            const cf::Grid2D g = grid_of(i);
            const T* lut = reinterpret_cast<const T*>(ws + L.lut + B.lut_off[i]);
            const int* tm = dl + B.inst_tm_off[i];
            const int* te = dl + B.inst_te_off[i];
            BSTEP(cf::launch_h2d<T>(CF_POL_TM, 1, A, dch, tm, B.inst_tm_n[i], g, lut, s));
            BSTEP(cf::launch_h2d<T>(CF_POL_TE, 1, A, dch, te, B.inst_te_n[i], g, lut, s));
            BSTEP(cf::launch_e2d<T>(CF_POL_TM, 1, A, dch, tm, B.inst_tm_n[i], g, lut, s));
            BSTEP(cf::launch_e2d<T>(CF_POL_TE, 1, A, dch, te, B.inst_te_n[i], g, lut, s));
        }
        int launches = 0;
        // the TE launches on a second stream (a parallel branch of the graph
        // when captured), so that each polarization's launch tail overlaps
        // the other's
        SideStreams side;
        const bool split_pol = n_tm > 0 && n_te > 0 && !(o.flags & CF_FLAG_TIME_STENCIL);
        if (split_pol) BSTEP(side.create(1));
        BSTEP(graph.begin());
        {
            const hipStream_t ls = graph.launch_stream(s);
            hipError_t body = split_pol ? side.open(ls) : hipSuccess;
            if (body == hipSuccess)
                body = [&]() -> hipError_t {
                    const hipStream_t ts = split_pol ? side.s[0] : ls;
                    int parity = 0;
                    for (int m = 0; m < o.n_steps; m += kh) {
                        hipError_t e = hipSuccess;
                        if (n_tm)
                            e = cf::launch_tb2d<T>(variant, CF_POL_TM, dch, dwork, nw_tm, dinst, kh, m, parity, ls);
                        if (e == hipSuccess && n_te)
                            e = cf::launch_tb2d<T>(variant, CF_POL_TE, dch, dwork + B.work_items, nw_te, dinst, kh, m,
                                                   parity, ts);
                        if (e != hipSuccess) return e;
                        launches += (n_tm > 0) + (n_te > 0);
                        parity ^= 1;
                    }
                    return hipSuccess;
                }();
            if (split_pol && !side.s.empty()) {
                const hipError_t ec = side.close(ls);   // joins the branch before the capture ends
                if (body == hipSuccess) body = ec;
            }
            BSTEP(graph.end(s, body));
        }
        timing->launches = launches;
        BSTEP(hipEventRecord(e1, s));
        BSTEP(hipEventSynchronize(e1));
        float ms = 0;
        BSTEP(hipEventElapsedTime(&ms, e0, e1));
        *device_ms = ms;
    }
    acc_out.assign((size_t)B.C * 2, 0.0);
    BSTEP(hipMemcpyAsync(acc_out.data(), dacc, (size_t)B.C * 2 * 8, hipMemcpyDeviceToHost, s));
    BSTEP(hipStreamSynchronize(s));
bdone:
#undef BSTEP
    if (err != hipSuccess) (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return fail(CF_E_DEVICE, std::string("batched device step failed: ") + hipGetErrorString(err));
    return CF_OK;
}

}  // namespace cfi

using namespace cfi;

// ---- entry points: bodies (no C linkage) -----------------------------------

static cf_status cf_problem_create_impl(const cf_grid* grid, const cf_materials* mats, const cf_surface* surf,
                            cf_problem** out) {
    if (!grid || !mats || !surf || !out) return fail(CF_E_ARG, "null argument");
    *out = nullptr;
    std::unique_ptr<cf_problem> h(new (std::nothrow) cf_problem);
    if (!h) return fail(CF_E_ARG, "out of host memory");
    std::string err = cf::build_problem(*grid, *mats, *surf, h->p);
    if (!err.empty()) {
        bool surface = err.find("surface") != std::string::npos;
        return fail(surface ? CF_E_SURFACE : CF_E_ARG, err);
    }
    *out = h.release();
    g_err.clear();
    return CF_OK;
}

static cf_status cf_problem_destroy_impl(cf_problem* p) {
    if (p) forget_plans(p->p.uid);
    delete p;
    return CF_OK;
}

static cf_status cf_validate_impl(const cf_problem* h, const cf_opts* o) {
    if (!h || !o) return fail(CF_E_ARG, "null argument");
    cf_status code;
    std::string err = cf::validate_opts(h->p, *o, &code);
    if (!err.empty()) return fail(code, err);
    if (o->n_subset > 0) {
        std::string e2;
        auto ch = selected_channels(h->p, *o, &e2);
        if (!e2.empty()) return fail(CF_E_ARG, e2);
    }
    return CF_OK;
}

static cf_status cf_problem_info_impl(const cf_problem* h, const cf_opts* o, cf_info* out) {
    cf_status st = cf_validate(h, o);
    if (st != CF_OK) return st;
    if (!out) return fail(CF_E_ARG, "null argument");
    const cf::Problem& p = h->p;
    std::string e2;
    auto all = cf::channel_table(p, o->pol);
    auto chans = selected_channels(p, *o, &e2);
    Staged sg;
    stage(p, *o, chans, sg);
    Layout L = layout_for(p, *o, sg);
    out->n_channels = (int)all.size();
    out->n_faces = (int)p.faces.size();
    out->per_harmonic_len = cf::harmonic_len(p);
    out->n_comp = cf::n_comp(p);
    out->workspace_bytes = L.total;
    out->eps_s = p.eps_s;
    out->mu_s = p.mu_s;
    out->n_steps_max = cf::max_steps(p, *o);
    return CF_OK;
}

static cf_status cf_channel_table_impl(const cf_problem* h, const cf_opts* o, int n, int* face, int* label,
                           int* kind, int* src, int* meas, double* sign) {
    cf_status st = cf_validate(h, o);
    if (st != CF_OK) return st;
    auto all = cf::channel_table(h->p, o->pol);
    if (n < (int)all.size()) return fail(CF_E_ARG, "channel arrays too short");
    for (size_t c = 0; c < all.size(); ++c) {
        if (face) face[c] = h->p.faces[all[c].face].index;
        if (label) label[c] = all[c].label;
        if (kind) kind[c] = all[c].kind;
        if (src) src[c] = all[c].src;
        if (meas) meas[c] = all[c].meas;
        if (sign) sign[c] = all[c].sign;
    }
    return CF_OK;
}

static cf_status cf_workspace_size_impl(const cf_problem* h, const cf_opts* o, size_t* bytes) {
    cf_info info;
    cf_status st = cf_problem_info(h, o, &info);
    if (st != CF_OK) return st;
    if (!bytes) return fail(CF_E_ARG, "null argument");
    *bytes = info.workspace_bytes;
    return CF_OK;
}

static cf_status cf_kernel_table_impl(int kernel, double sigma, double dt, int n, double* out) {
    if (!out || n < 0 || !(dt > 0) || !(sigma >= 0)) return fail(CF_E_ARG, "bad kernel table arguments");
    if (kernel != CF_KERNEL_GENERAL && kernel != CF_KERNEL_ZINV2D) return fail(CF_E_ARG, "unknown kernel");
    cf::kernel_table(kernel, sigma, dt, n, out);
    return CF_OK;
}

static cf_status cf_solve_impl(cf_problem* h, const cf_opts* o, void* workspace, size_t ws_bytes, cf_result* out) {
    cf_status st = cf_validate(h, o);
    if (st != CF_OK) return st;
    if (!out) return fail(CF_E_ARG, "null result");
    const cf::Problem& p = h->p;
    std::string e2;
    auto chans = selected_channels(p, *o, &e2);
    if (!e2.empty()) return fail(CF_E_ARG, e2);
    const size_t C = chans.size();
    const int lab = cf::harmonic_len(p);
    const bool keep_gamma = (o->flags & CF_FLAG_KEEP_GAMMA) != 0;
    if (out->per_harmonic && out->per_harmonic_len < lab) return fail(CF_E_ARG, "per_harmonic too short");
    if (out->per_face && out->per_face_len < 2 * p.grid.ndim) return fail(CF_E_ARG, "per_face too short");
    if (out->per_channel && out->per_channel_len < (int)C) return fail(CF_E_ARG, "per_channel too short");
    if (out->gamma && (!keep_gamma || out->gamma_len < (long long)cf::max_steps(p, *o) * (long long)C))
        return fail(CF_E_ARG, "gamma needs CF_FLAG_KEEP_GAMMA and n_steps_max*channels entries");
    if (out->trace && (!keep_gamma || out->trace_len < o->n_steps))
        return fail(CF_E_ARG, "trace needs CF_FLAG_KEEP_GAMMA and n_steps entries");
    Staged sg;
    stage(p, *o, chans, sg);
    Layout L = layout_for(p, *o, sg);
    char* ws = static_cast<char*>(workspace);
    void* owned = nullptr;
    if (!ws) {
        CF_HIP(hipMalloc(&owned, L.total));
        ws = static_cast<char*>(owned);
    } else if (ws_bytes < L.total) {
        return fail(CF_E_BUDGET, "workspace smaller than cf_workspace_size()");
    }
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    std::vector<double> acc, gam;
    double ms = 0;
    StencilTiming tim;
    cf_status rs = o->precision == CF_FP64 ? run_solve<double>(p, *o, sg, L, ws, s, acc, gam, &ms, &tim)
                                           : run_solve<float>(p, *o, sg, L, ws, s, acc, gam, &ms, &tim);
    if (owned) (void)hipFree(owned);
    if (rs != CF_OK) return rs;
    const bool finite = fill_result(p, chans, acc, gam, *o, ms, tim, sg, out);
    if (!finite) return fail(CF_E_NONFINITE, "a force accumulator is not finite");
    g_err.clear();
    return CF_OK;
}


// Reduced problems of a batch (cylindrical, k_z, Bloch) are solved
// concurrently by this many host threads, each with its own stream and
// workspace slot: one such solve runs one block per channel, often on fewer
// CUs than the chip has, so several of them share the GPU.
constexpr int kRedWorkers = 4;

static size_t ws_align(size_t b) { return (b + 255) & ~size_t(255); }

static cf_status cf_batch_workspace_size_impl(cf_problem* const* probs, int n, const cf_opts* o, size_t* bytes) {
    if (!probs || n < 1 || !o || !bytes) return fail(CF_E_ARG, "bad batch arguments");
    size_t solo = 0, red_max = 0;
    int n_red = 0;
    std::vector<cf_problem*> fused;
    for (int i = 0; i < n; ++i) {
        cf_status st = cf_validate(probs[i], o);
        if (st != CF_OK) return st;
        if (probs[i]->p.fusable2d()) fused.push_back(probs[i]);
        size_t b = 0;
        cf_opts oo = *o;
        oo.n_subset = 0;
        oo.channel_subset = nullptr;
        st = cf_workspace_size(probs[i], &oo, &b);
        if (st != CF_OK) return st;
        solo = std::max(solo, b);
        if (probs[i]->p.reduced()) {
            ++n_red;
            red_max = std::max(red_max, ws_align(b));
        }
    }
    size_t fb = 0;
    if (!fused.empty()) {
        BatchPlan B;
        if (plan_batch(fused.data(), (int)fused.size(), *o, B).empty()) fb = batch_layout(B, *o).total;
    }
    const size_t rb = n_red >= 2 ? (size_t)std::min(n_red, kRedWorkers) * red_max : 0;
    *bytes = std::max({solo, fb, rb});
    return CF_OK;
}

// Solve probs[idx[..]] concurrently (see kRedWorkers); slot k of the
// workspace is [k * slot, (k + 1) * slot).  Work already queued on the
// caller's stream finishes before any of them starts.
static cf_status solve_concurrently(cf_problem* const* probs, const std::vector<int>& idx, const cf_opts& oo,
                                    char* ws, size_t slot, cf_result* outs) {
    const int nw = std::min((int)idx.size(), kRedWorkers);
    int dev = 0;
    CF_HIP(hipGetDevice(&dev));
    hipEvent_t ready;
    CF_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ready, static_cast<hipStream_t>(oo.stream));
    if (e != hipSuccess) {
        (void)hipEventDestroy(ready);
        return fail(CF_E_DEVICE, std::string("device step failed: ") + hipGetErrorString(e));
    }
    std::atomic<int> next{0};
    std::atomic<int> solved{0};
    std::vector<cf_status> status(nw, CF_OK);
    std::vector<std::string> msg(nw);
    std::vector<std::string> setup_msg(nw);
    auto worker = [&](int k) {
        // a worker whose stream cannot be set up takes no problems; the
        // others take them all
        hipStream_t s = nullptr;
        hipError_t he = hipSetDevice(dev);
        // non-blocking (default priority): workers are not serialised
        // through the null stream
        if (he == hipSuccess) he = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (he == hipSuccess) he = hipStreamWaitEvent(s, ready, 0);
        if (he != hipSuccess) {
            setup_msg[k] = std::string("device step failed: ") + hipGetErrorString(he);
            if (s) (void)hipStreamDestroy(s);
            return;
        }
        for (int j; status[k] == CF_OK && (j = next.fetch_add(1)) < (int)idx.size();) {
            cf_opts oi = oo;
            oi.stream = s;
            const int i = idx[j];
            try {
                status[k] = cf_solve(probs[i], &oi, ws + (size_t)k * slot, slot, &outs[i]);
                if (status[k] != CF_OK) msg[k] = cf_last_error();
                else solved.fetch_add(1);
            } catch (const std::bad_alloc&) {   // nothing may escape a worker thread
                status[k] = CF_E_BUDGET;
                msg[k] = "host allocation failed";
            } catch (const std::exception& ex) {
                status[k] = CF_E_DEVICE;
                msg[k] = ex.what();
            }
        }
        (void)hipStreamDestroy(s);
    };
    std::vector<std::thread> pool;
    for (int k = 1; k < nw; ++k) {
        try {
            pool.emplace_back(worker, k);
        } catch (const std::system_error&) {   // the started workers take the rest
            break;
        }
    }
    worker(0);
    for (auto& t : pool) t.join();
    (void)hipEventDestroy(ready);
    for (int k = 0; k < nw; ++k)
        if (status[k] != CF_OK) return fail(status[k], msg[k]);
    if (solved.load() < (int)idx.size()) {
        for (int k = 0; k < nw; ++k)
            if (!setup_msg[k].empty()) return fail(CF_E_DEVICE, setup_msg[k]);
        return fail(CF_E_DEVICE, "concurrent solve left problems unsolved");
    }
    return CF_OK;
}

static cf_status cf_batch_solve_impl(cf_problem* const* probs, int n, const cf_opts* o, void* workspace, size_t ws_bytes,
                         cf_result* outs) {
    if (!probs || n < 1 || !o || !outs) return fail(CF_E_ARG, "bad batch arguments");
    cf_opts oo = *o;
    oo.n_subset = 0;
    oo.channel_subset = nullptr;
    oo.flags &= ~CF_FLAG_KEEP_GAMMA;
    for (int i = 0; i < n; ++i) {
        cf_status st = cf_validate(probs[i], &oo);
        if (st != CF_OK) return st;
    }
    // 2D problems share one fused sequence when every one fits a common tile
    std::vector<int> fused_idx;
    if (!(o->flags & CF_FLAG_SPLIT))
        for (int i = 0; i < n; ++i)
            if (probs[i]->p.fusable2d())
                fused_idx.push_back(i);
    BatchPlan B;
    if (fused_idx.size() >= 1) {
        std::vector<cf_problem*> fp;
        for (int i : fused_idx) fp.push_back(probs[i]);
        if (!plan_batch(fp.data(), (int)fp.size(), oo, B).empty()) fused_idx.clear();
    }
    std::vector<bool> done(n, false);
    if (!fused_idx.empty()) {
        BatchLayout L = batch_layout(B, oo);
        char* ws = static_cast<char*>(workspace);
        void* owned = nullptr;
        if (!ws) {
            CF_HIP(hipMalloc(&owned, L.total));
            ws = static_cast<char*>(owned);
        } else if (ws_bytes < L.total) {
            return fail(CF_E_BUDGET, "workspace smaller than cf_batch_workspace_size()");
        }
        hipStream_t s = static_cast<hipStream_t>(o->stream);
        std::vector<double> acc;
        double ms = 0;
        StencilTiming tim;
        cf_status rs = o->precision == CF_FP64 ? run_batch<double>(B, L, oo, ws, s, acc, &ms, &tim)
                                               : run_batch<float>(B, L, oo, ws, s, acc, &ms, &tim);
        if (owned) (void)hipFree(owned);
        if (rs != CF_OK) return rs;
        for (size_t k = 0; k < fused_idx.size(); ++k) {
            const int i = fused_idx[k];
            const size_t Ci = B.chans[k].size();
            std::vector<double> ai(acc.begin() + 2 * (size_t)B.base[k], acc.begin() + 2 * ((size_t)B.base[k] + Ci));
            const bool finite = fill_result(*B.probs[k], B.chans[k], ai, {}, oo, ms, tim, B.st[k], &outs[i]);
            if (!finite) return fail(CF_E_NONFINITE, "a force accumulator is not finite");
            done[i] = true;
        }
    }
    std::vector<int> red_idx;
    size_t red_max = 0;
    for (int i = 0; i < n; ++i)
        if (!done[i] && probs[i]->p.reduced()) {
            size_t b = 0;
            cf_status st = cf_workspace_size(probs[i], &oo, &b);
            if (st != CF_OK) return st;
            red_max = std::max(red_max, ws_align(b));
            red_idx.push_back(i);
        }
    if (red_idx.size() >= 2) {
        const size_t need = (size_t)std::min((int)red_idx.size(), kRedWorkers) * red_max;
        char* ws = static_cast<char*>(workspace);
        void* owned = nullptr;
        if (!ws) {
            CF_HIP(hipMalloc(&owned, need));
            ws = static_cast<char*>(owned);
        } else if (ws_bytes < need) {
            return fail(CF_E_BUDGET, "workspace smaller than cf_batch_workspace_size()");
        }
        cf_status st = solve_concurrently(probs, red_idx, oo, ws, red_max, outs);
        if (owned) (void)hipFree(owned);
        if (st != CF_OK) return st;
        for (int i : red_idx) done[i] = true;
    }
    for (int i = 0; i < n; ++i) {
        if (done[i]) continue;
        cf_status st = cf_solve(probs[i], &oo, workspace, ws_bytes, &outs[i]);
        if (st != CF_OK) return st;
    }
    g_err.clear();
    return CF_OK;
}


// ---- the C ABI: every entry point runs its body under cfi::guarded ---------

extern "C" {

const char* cf_last_error(void) { return g_err.c_str(); }

cf_status cf_problem_create(const cf_grid* grid, const cf_materials* mats, const cf_surface* surf,
                            cf_problem** out) {
    return guarded([&] { return cf_problem_create_impl(grid, mats, surf, out); });
}

cf_status cf_problem_destroy(cf_problem* p) {
    return guarded([&] { return cf_problem_destroy_impl(p); });
}

cf_status cf_validate(const cf_problem* h, const cf_opts* o) {
    return guarded([&] { return cf_validate_impl(h, o); });
}

cf_status cf_problem_info(const cf_problem* h, const cf_opts* o, cf_info* out) {
    return guarded([&] { return cf_problem_info_impl(h, o, out); });
}

cf_status cf_channel_table(const cf_problem* h, const cf_opts* o, int n, int* face, int* label, int* kind,
                           int* src, int* meas, double* sign) {
    return guarded([&] { return cf_channel_table_impl(h, o, n, face, label, kind, src, meas, sign); });
}

cf_status cf_workspace_size(const cf_problem* h, const cf_opts* o, size_t* bytes) {
    return guarded([&] { return cf_workspace_size_impl(h, o, bytes); });
}

cf_status cf_kernel_table(int kernel, double sigma, double dt, int n, double* out) {
    return guarded([&] { return cf_kernel_table_impl(kernel, sigma, dt, n, out); });
}

cf_status cf_solve(cf_problem* h, const cf_opts* o, void* workspace, size_t ws_bytes, cf_result* out) {
    return guarded([&] { return cf_solve_impl(h, o, workspace, ws_bytes, out); });
}

cf_status cf_batch_workspace_size(cf_problem* const* probs, int n, const cf_opts* o, size_t* bytes) {
    return guarded([&] { return cf_batch_workspace_size_impl(probs, n, o, bytes); });
}

cf_status cf_batch_solve(cf_problem* const* probs, int n, const cf_opts* o, void* workspace, size_t ws_bytes,
                         cf_result* outs) {
    return guarded([&] { return cf_batch_solve_impl(probs, n, o, workspace, ws_bytes, outs); });
}

}  // extern "C"
