// Host structures shared by the solve, batch and serving code of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/casimir_fdtd.h"
#include "device.hpp"
#include "plan.hpp"

namespace cfi {

cf_status fail(cf_status code, const std::string& msg);
void clear_error();
size_t align_up(size_t v, size_t a);

// Runs the body of an entry point of the C ABI so that no C++ exception
// crosses it: a failed host allocation becomes CF_E_BUDGET, any other
// exception CF_E_ARG, each with its message in cf_last_error().
cf_status fail_nothrow(cf_status code, const char* msg) noexcept;
template <class F>
cf_status guarded(F&& body) noexcept {
    try {
        return body();
    } catch (const std::bad_alloc&) {
        return fail_nothrow(CF_E_BUDGET, "host memory allocation failed");
    } catch (const std::length_error&) {
        return fail_nothrow(CF_E_BUDGET, "host array size exceeds the allocator's limit");
    } catch (const std::exception& e) {
        return fail_nothrow(CF_E_ARG, e.what());
    } catch (...) {
        return fail_nothrow(CF_E_ARG, "unknown internal error");
    }
}

// Tiling of the fused kernel: shifted so that every measured surface stencil
// point of every channel lies in one tile (the surface tile).
//
// A wave of the fused kernel whose rows, and the first row of the wave above,
// hold only E components with a = b = 0 (perfect conductor, wall, outside
// the grid) advances nothing: E stays 0 there, so does H (its curl reads only
// those rows), and the kernel skips it.  live[k] lists the tiles of
// polarization k (0 TM, 1 TE) with at least one other wave, each with the
// bit mask of its live waves (the kernel reads it from its work item); the
// rest are not launched.  live_cells[k] counts the tile-interior cells of
// those waves inside the grid (cells the kernel advances per channel and
// step).
struct LiveTile {
    int tile;
    uint32_t waves;   // bit w: wave w of the tile advances
};
struct TBPlan {
    bool ok = false;
    int base_x = 0, base_y = 0, ntx = 0, nty = 0, stile = -1;
    std::vector<LiveTile> live[2];
    double live_cells[2] = {0, 0};
};

// One wave of resident channels: index lists (into the channel table) per
// polarization and in channel order.
struct Wave {
    int tm_off, n_tm, te_off, n_te, d3_off, n_3d, all_off, n_all;
    int order;   // azimuthal order of every channel in the wave (cylindrical problems)
};

struct Staged {
    TBPlan tb;                             // plan of the chosen variant
    int variant = -1;                      // chosen fused variant (-1: not fused)
    std::vector<TBPlan> plans;             // plan per fused variant
    std::vector<cf::TBShape> shapes;
    std::vector<cf::Channel> chans;       // channels run, in output order
    std::vector<cf::ChanDev> dev;          // one descriptor per channel run
    std::vector<int> slot_lists;           // concatenated per-wave lists
    std::vector<Wave> waves;
    std::vector<int32_t> gidx, uidx, uoff, usamp;
    std::vector<double> gw, uw, basis;
    int max_uniq = 0;
    int resident = 0;                      // field blocks on the device
    int ncomp = 3;
    int64_t psi_comp = 0;                  // values per psi component (3D CPML)
    int64_t psi_block = 0;                 // CPML values per resident channel (3D, or 2D split kernels)
    int64_t psi2d_slot = 0;                // 2D CPML: values per field slot (x and y layer arrays)
    bool pml2d = false;                    // 2D problem with in-plane CPML layers (split kernels)
    bool red_res = false;                  // cylindrical waves on the resident solve kernel
    bool f3d = false;                      // 3D steps on the fused z-streaming kernel
    int v3d = -1;                          // its variant when fixed by the options (-1: autotune)
    cf::ShadowBox sbox{};                  // surface box of a 3D solve (two-step fused launches)
    int64_t aux_block = 0;                 // polarization values per resident channel (dispersive media)
    std::vector<int32_t> zr;               // fused 3D: per variant and band, the planes [lo, hi) it can change
    int zr_off[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // first band of variant v in zr (pairs)
};

struct StencilTiming {
    double ms_total = 0, bytes_total = 0, cu_total = 0;
    int samples = 0;
    int launches = 0;
    int variant = -1;
    int steps_run = -1;     // time steps run (-1: all of opts.n_steps)
};

// Time-convergence stop: every `every` steps the partial force F(T') is
// formed from the FP64 accumulators on the host; the run ends once two
// consecutive windows change it by at most tol |F(T')|.
struct ConvergenceStop {
    bool on = false;
    double tol = 0;
    int every = 500;
    int next = 500;
    int calm = 0;
    double f_prev = 0;
    bool have_prev = false;
    // F(T') from (sum, compensation) pairs and the channel signs
    bool update(const std::vector<double>& acc, const std::vector<cf::Channel>& chans) {
        double f = 0;
        for (size_t c = 0; c < chans.size(); ++c) f += chans[c].sign * (acc[2 * c] + acc[2 * c + 1]);
        f /= 3.14159265358979323846;
        const bool quiet = have_prev && std::abs(f - f_prev) <= tol * std::abs(f);
        calm = quiet ? calm + 1 : 0;
        f_prev = f;
        have_prev = true;
        return calm >= 2;
    }
};

// Stage the tables of one problem for the given channels and options.
void stage(const cf::Problem& p, const cf_opts& o, const std::vector<cf::Channel>& chans, Staged& st);
// XCD-balanced work list (see api.cpp).
// Work list of the fused 2D launch: the tiles of each slot on one XCD
// (channels balanced over the 8 XCDs, block b on XCD b mod 8), each slot's
// surface tile stile[k] first (its block does the per-step surface work, so
// it should not be left for the tail of the launch).
// tiles[k] lists the tiles slot k runs (its plan's live tiles of the slot's
// polarization).
std::vector<cf::WorkItem> make_work(const std::vector<int>& slots, const std::vector<const std::vector<LiveTile>*>& tiles,
                                    const std::vector<int>& stile);
// the live tile list of polarization pol (CF_POL_TM / CF_POL_TE) in plan pl
inline const std::vector<LiveTile>& live_tiles(const TBPlan& pl, int pol) { return pl.live[pol == CF_POL_TE ? 1 : 0]; }
// Host reduction of accumulators into a cf_result; false if not finite.
bool fill_result(const cf::Problem& p, const std::vector<cf::Channel>& chans, const std::vector<double>& acc,
                 const std::vector<double>& gam, const cf_opts& o, double ms, const StencilTiming& tim,
                 const Staged& sg, cf_result* out);

}  // namespace cfi
