// 2D Yee kernels for gfx950: TM (Ez, Hx, Hy) and TE (Ex, Ey, Hz) updates
// with the uniform conductivity sigma carried by per-kind coefficient tables,
// the delta(t) kick, the surface projection with the FP64 compensated
// g-weighted time accumulation, and the fused temporal-blocked step kernel.
//
// Layout: a channel's field block is 3 components x (ny x nx) cells, x
// fastest.  Update forms (undivided differences; a, b from the channel
// kind's table):
//   TM  Hx <- a Hx - b (Ez[j+1] - Ez[j])        Hy <- a Hy - b (Ez[i] - Ez[i+1])
//       Ez <- a Ez + b ((Hy[i] - Hy[i-1]) - (Hx[j] - Hx[j-1]))
//   TE  Hz <- a Hz - b ((Ey[i+1] - Ey[i]) - (Ex[j+1] - Ex[j]))
//       Ex <- a Ex + b (Hz[j] - Hz[j-1])         Ey <- a Ey - b (Hz[i] - Hz[i-1])
// A neighbour beyond the grid reads as 0 on a PEC wall and wraps on a
// periodic one.  Every kernel evaluates these forms through the same inline
// helpers with explicit fused multiply-adds (the library is built without
// automatic contraction), so the split, fused and plain paths produce
// bitwise-identical fields.
#include "../../include/casimir_fdtd.h"
#include "device.hpp"
#include "yee_common.hpp"

namespace cf {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int NT = 256;   // threads of the surface and fused kernels

using yee::from_next;
using yee::from_prev;
using yee::lut_ab;
using yee::Pair;
template <typename T>
__device__ __forceinline__ T yee_sub(T a, T x, T b, T d) { return yee::sub(a, x, b, d); }
template <typename T>
__device__ __forceinline__ T yee_add(T a, T x, T b, T d) { return yee::add(a, x, b, d); }
template <typename T>
__device__ __forceinline__ T yee_half(T b, T d) { return yee::half(b, d); }

using yee::neumaier;
using yee::block_surface_sum;
using yee::lorentz_step;
using yee::pml_d2;
using yee::as_global;

// ---------------------------------------------------------------------------
// split half-step kernels (one launch per half step for a batch of channels)

template <typename T, int POL, int MODE>
__global__ __launch_bounds__(BX* BY) void k_h2d(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                              const int* __restrict__ slots, Grid2D g,
                                              const T* __restrict__ lut) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 0) return;   // start: E-kind runs set H^{-1/2}
    const int tiles_x = (g.nx + BX - 1) / BX;
    const int i = (blockIdx.x % tiles_x) * BX + threadIdx.x;
    const int j = (blockIdx.x / tiles_x) * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    T* base = fields + d.field_off;
    const int64_t c = (int64_t)j * g.nx + i;
    const bool in_r = i + 1 < g.nx, in_u = j + 1 < g.ny;
    if (POL == CF_POL_TM) {
        const T* Ez = base;
        T* Hx = base + g.ncell;
        T* Hy = base + 2 * g.ncell;
        const T ez = Ez[c];
        const T ezr = in_r ? Ez[c + 1] : (g.perx ? Ez[c + 1 - g.nx] : T(0));
        const T ezu = in_u ? Ez[c + g.nx] : (g.pery ? Ez[i] : T(0));
        const T* lx = lut_ab(lut, d.kind, CF_HX, g.ids[CF_HX][c]);
        const T* ly = lut_ab(lut, d.kind, CF_HY, g.ids[CF_HY][c]);
        // the consistent start (MODE 1) stretches its curl in the CPML too
        T* psi = g.psi ? static_cast<T*>(g.psi) + d.psi_off : nullptr;
        const T dy = pml_d2(ezu - ez, g, psi, 1, 1, true, i, j);
        const T dx = pml_d2(ezr - ez, g, psi, 2, 0, true, i, j);
        if (MODE == 0) {
            Hx[c] = yee_sub(lx[0], Hx[c], lx[1], dy);
            Hy[c] = yee_sub(ly[0], Hy[c], ly[1], -dx);
        } else {
            Hx[c] = yee_half(lx[1], dy);
            Hy[c] = yee_half(ly[1], -dx);
        }
    } else {
        const T* Ex = base;
        const T* Ey = base + g.ncell;
        T* Hz = base + 2 * g.ncell;
        const T ex = Ex[c], ey = Ey[c];
        const T eyr = in_r ? Ey[c + 1] : (g.perx ? Ey[c + 1 - g.nx] : T(0));
        const T exu = in_u ? Ex[c + g.nx] : (g.pery ? Ex[i] : T(0));
        const T* lz = lut_ab(lut, d.kind, CF_HZ, g.ids[CF_HZ][c]);
        T* psi = g.psi ? static_cast<T*>(g.psi) + d.psi_off : nullptr;
        const T dx = pml_d2(eyr - ey, g, psi, 2, 0, true, i, j);
        const T dy = pml_d2(exu - ex, g, psi, 2, 1, true, i, j);
        if (MODE == 0) {
            Hz[c] = yee_sub(lz[0], Hz[c], lz[1], dx - dy);
        } else {
            Hz[c] = yee_half(lz[1], dx - dy);
        }
    }
}

template <typename T, int POL, int MODE>
__global__ __launch_bounds__(BX* BY) void k_e2d(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                              const int* __restrict__ slots, Grid2D g,
                                              const T* __restrict__ lut) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 1) return;   // start: H-kind runs set E^{+1/2}
    const int tiles_x = (g.nx + BX - 1) / BX;
    const int i = (blockIdx.x % tiles_x) * BX + threadIdx.x;
    const int j = (blockIdx.x / tiles_x) * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    T* base = fields + d.field_off;
    const int64_t c = (int64_t)j * g.nx + i;
    if (POL == CF_POL_TM) {
        T* Ez = base;
        const T* Hx = base + g.ncell;
        const T* Hy = base + 2 * g.ncell;
        const T hx = Hx[c], hy = Hy[c];
        const T hyl = i > 0 ? Hy[c - 1] : (g.perx ? Hy[c - 1 + g.nx] : T(0));
        const T hxd = j > 0 ? Hx[c - g.nx] : (g.pery ? Hx[c + (int64_t)(g.ny - 1) * g.nx] : T(0));
        const T* lz = lut_ab(lut, d.kind, CF_EZ, g.ids[CF_EZ][c]);
        T* psi = g.psi ? static_cast<T*>(g.psi) + d.psi_off : nullptr;
        const T dx = pml_d2(hy - hyl, g, psi, 0, 0, false, i, j);
        const T dy = pml_d2(hx - hxd, g, psi, 0, 1, false, i, j);
        if (MODE == 0) {
            const T ez = Ez[c];
            T e_new = yee_add(lz[0], ez, lz[1], dx - dy);
            if (g.n_lor > 0)
                e_new -= lorentz_step(g, static_cast<T*>(g.aux) + d.aux_off, 0, c, g.ids[CF_EZ][c], lz[0], ez);
            Ez[c] = e_new;
        } else {
            Ez[c] = yee_half(lz[1], dx - dy);
        }
    } else {
        T* Ex = base;
        T* Ey = base + g.ncell;
        const T* Hz = base + 2 * g.ncell;
        const T hz = Hz[c];
        const T hzd = j > 0 ? Hz[c - g.nx] : (g.pery ? Hz[c + (int64_t)(g.ny - 1) * g.nx] : T(0));
        const T hzl = i > 0 ? Hz[c - 1] : (g.perx ? Hz[c - 1 + g.nx] : T(0));
        const T* lx = lut_ab(lut, d.kind, CF_EX, g.ids[CF_EX][c]);
        const T* ly = lut_ab(lut, d.kind, CF_EY, g.ids[CF_EY][c]);
        T* psi = g.psi ? static_cast<T*>(g.psi) + d.psi_off : nullptr;
        const T dy = pml_d2(hz - hzd, g, psi, 0, 1, false, i, j);
        const T dx = pml_d2(hz - hzl, g, psi, 1, 0, false, i, j);
        if (MODE == 0) {
            const T ex = Ex[c], ey = Ey[c];
            T ex_new = yee_add(lx[0], ex, lx[1], dy);
            T ey_new = yee_sub(ly[0], ey, ly[1], dx);
            if (g.n_lor > 0) {
                T* aux = static_cast<T*>(g.aux) + d.aux_off;
                ex_new -= lorentz_step(g, aux, 0, c, g.ids[CF_EX][c], lx[0], ex);
                ey_new -= lorentz_step(g, aux, 1, c, g.ids[CF_EY][c], ly[0], ey);
            }
            Ex[c] = ex_new;
            Ey[c] = ey_new;
        } else {
            Ex[c] = yee_half(lx[1], dy);
            Ey[c] = -yee_half(ly[1], dx);
        }
    }
}

// X_src[g] = kick_scale * sum_{(s, w) at g} w f_n(s) over the distinct
// points g of the source component's interpolation stencil (adjoint W^T).
template <typename T>
__global__ void k_kick(T* __restrict__ fields, const ChanDev* __restrict__ ch, const int* __restrict__ slots,
                       SurfTables t) {
    const ChanDev d = ch[slots[blockIdx.y]];
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < d.n_uniq; u += gridDim.x * blockDim.x) {
        const int k0 = t.uoff[d.u_off + u], k1 = t.uoff[d.u_off + u + 1];
        double s = 0.0;
        for (int k = k0; k < k1; ++k) s += t.uw[k] * t.basis[d.basis_off + t.usamp[k]];
        fields[d.src_off + t.uidx[d.u_off + u]] = T(d.kick_scale * s);
    }
}

// One block per channel: Gamma = dA sum_s f_n(s) sum_p w_sp X[idx_sp] (FP64),
// then the Neumaier update of (sum, comp) += dt K(t_m) Gamma.
template <typename T>
__global__ __launch_bounds__(NT) void k_surface(const T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                                const int* __restrict__ slots, SurfTables t,
                                                const double* __restrict__ ktab, int m, double dt,
                                                double dA, double* __restrict__ acc,
                                                double* __restrict__ gamma, int gamma_stride) {
    __shared__ double red[NT / 64];
    const int slot = slots[blockIdx.x];
    const ChanDev d = ch[slot];
    const T* X = fields + d.meas_off;
    const double s = block_surface_sum(d, t, [&](int32_t idx) { return (double)X[idx]; }, red);
    if (threadIdx.x == 0) {
        const double G = dA * s;
        double sum = acc[2 * slot], comp = acc[2 * slot + 1];
        neumaier(sum, comp, (dt * ktab[m]) * G);
        acc[2 * slot] = sum;
        acc[2 * slot + 1] = comp;
        if (gamma) gamma[(int64_t)m * gamma_stride + slot] = G;
    }
}

// ---------------------------------------------------------------------------
// fused temporal-blocked kernel, register-blocked
//
// Block b works on one tile of one channel.  Its region is 64 CX columns (CX
// per lane) by W*B rows (wave w of W holds rows w*B .. w*B+B-1 of its
// columns in registers); the tile proper is the region minus a KH-cell halo on
// every side.  The block loads the region, takes `ksteps` <= KH full time
// steps and writes the tile's cells to dst.  After step s the fields are
// exact on the region shrunk by s cells on every side, so the tile stays
// exact for KH steps; the shrinking rim holds finite stale values that are
// never written back.
//
// Neighbours: along x a lane takes its neighbour lane's value with a DPP
// wave shift (no memory); along y rows of one wave are registers and the
// rows at a wave boundary go through a one-row LDS exchange per half step.
// Barriers per step: one after the E-row writes, one after the H-row writes
// (plus two around the surface staging in the surface tile).
// Coefficients come from the channel kind's table in LDS, indexed by the
// per-cell material ids held packed in registers.  Cells outside a
// non-periodic grid carry the null material (a = b = 0) and stay 0.
//
// The tiling is shifted so that every surface stencil point lies in one
// tile (g.stile); that tile's block stages the measured component in LDS
// after every step, forms Gamma with the shared block reduction, and
// carries the channel's compensated accumulator through the launch.
//
// Work: block b takes item work[b] = (channel slot, tile).  The host lays
// the list out so that b % 8, the XCD a block is dispatched to, is the same
// for every tile of a channel (halo re-reads hit that XCD's L2).  Instances
// (problems) of one launch have their own grids, tables and time origin.

// Largest channel surface (samples, stencil points per sample) whose tables
// the surface tile keeps in LDS over a launch; larger ones are read from the
// global tables after every step.  A block of a shape whose other LDS arrays
// are large keeps fewer samples, so that two blocks still fit in a CU's LDS.
// With the present shapes every fused surface fits: it lies inside one tile,
// so a face has at most 120 samples, with 2 x 2 points each.
constexpr int kSurfP = 4;
constexpr int surf_cap(int other_lds_bytes) {
    return other_lds_bytes + 512 * (kSurfP * (2 + 8) + 8) <= 80 * 1024 ? 512 : 128;
}

// Register-blocked fused kernel.  A block holds a (64 CX) x (RBW B) region
// of one channel: lane l of wave w owns columns CX l .. CX l + CX - 1 and rows
// w B .. w B + B - 1, with every field value in registers.  x neighbours come
// from the lane's own registers or, across lanes, by DPP row shifts; y
// neighbours inside a wave's band from registers, across bands through LDS
// exchange rows.  KH steps run per launch; the outer KH cells of the region
// go stale one per step, so only the interior (64 CX - 2 KH) x (RBW B - 2 KH)
// is written back.
template <typename T, int POL, int RBW, int B, int KH, bool CREG, int CX, int WPE>
__global__ __launch_bounds__(64 * RBW) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_rb2d(const ChanDev* __restrict__ ch, const WorkItem* __restrict__ work,
            const InstDev* __restrict__ insts, int kmax, int mclock, int parity) {
    constexpr int RH = RBW * B;
    constexpr int RW = 64 * CX;
    constexpr int NTB = 64 * RBW;
    constexpr int TX = RW - 2 * KH, TY = RH - 2 * KH;
    constexpr int NP = (B + 3) / 4;
    constexpr int C0 = POL == CF_POL_TM ? CF_EZ : CF_EX;
    constexpr int C1 = POL == CF_POL_TM ? CF_HX : CF_EY;
    constexpr int C2 = POL == CF_POL_TM ? CF_HY : CF_HZ;
    __shared__ Pair<T> L[3][256];
    // wave-boundary rows: E rows (read by the wave below) and H rows (read by
    // the wave above) in separate buffers, so each write is separated from
    // the previous reads of the same buffer by the other half step's barrier
    __shared__ T xe[RBW][CX][64];
    __shared__ T xh[RBW][CX][64];
    __shared__ T stage[RH * RW];     // measured component (surface tile only), [row][col j][lane]
    __shared__ double red[RBW];
    // launch-resident surface tables of the surface tile (see `staged`)
    constexpr int kSurfCap =
        surf_cap((int)(sizeof(L) + sizeof(xe) + sizeof(xh) + sizeof(stage) + sizeof(red)) + 8 * KH);
    __shared__ uint16_t s_off[kSurfCap * kSurfP];
    __shared__ double s_w[kSurfCap * kSurfP];
    __shared__ double s_b[kSurfCap];
    __shared__ double s_k[KH];

    const WorkItem wi = work[blockIdx.x];
    if (wi.slot < 0) return;
    // A wave whose band, and the band of the wave above, hold no E component
    // with a nonzero coefficient advances nothing: E is held at 0 there and H,
    // whose curl reads only those rows, keeps its value, which is 0 from the
    // start (every field there starts at 0 and the cells are never written).
    // Such a wave skips its loads, arithmetic and write-back; it still takes
    // part in the barriers and writes its (zero) exchange rows.  Above the top
    // wave lie only stale rim rows, so its own band decides.  The host's plan
    // applies this test to the material ids (live_waves) and hands the tile's
    // live waves over in the work item.
    const int slot = wi.slot, tile = wi.tile;
    const ChanDev d = ch[slot];
    const InstDev g = insts[d.inst];
    const SurfTables& t = g.t;
    const int m0 = mclock - g.start;                      // instance's own step
    const int ksteps = min(kmax, g.nsteps - m0);
    if (m0 < 0 || ksteps <= 0) return;                    // not started / finished
    const auto lut = as_global(static_cast<const T*>(g.lut));
    const auto src = as_global(static_cast<const T*>(parity ? g.fb : g.fa));
    const auto dst = as_global(static_cast<T*>(parity ? g.fa : g.fb));
    const auto acc = as_global(g.acc + 2 * d.local);
    const int tx = tile % g.ntx, ty = tile / g.ntx;
    const int rx0 = g.base_x + tx * TX - KH, ry0 = g.base_y + ty * TY - KH;
    const int tid = threadIdx.x;
    // the wave index is uniform across a wave: taken as a scalar, every row
    // index and row bound below is scalar arithmetic
    const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool live = ((wi.waves >> w) & 1u) != 0;

    // Column of the lane's cell j and row r of the wave's band in the grid
    // (wrapped on a periodic axis), or -1 beyond a non-periodic edge: the x
    // index is per lane and column, the y index uniform across the wave, so
    // each is formed once here instead of once per cell.  Cell indices fit
    // 32 bits: the library refuses larger grids.
    int col[CX], row[B];
#pragma unroll
    for (int j = 0; j < CX; ++j) {
        int gx = rx0 + lane * CX + j;
        if (gx < 0 || gx >= g.nx) gx = g.perx ? ((gx % g.nx) + g.nx) % g.nx : -1;
        col[j] = gx;
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
        int gy = ry0 + w * B + r;
        if (gy < 0 || gy >= g.ny) gy = g.pery ? ((gy % g.ny) + g.ny) % g.ny : -1;
        row[r] = __builtin_amdgcn_readfirstlane(gy);
    }
    // The channel kind's coefficient pairs of the three components, staged in
    // LDS once the cell loads below are issued too.  Every load of the
    // prologue is unconditional (a clamped index where a thread has no
    // entry), so that all of them are in flight at once.
    constexpr int NL = (3 * 256 + NTB - 1) / NTB;
    Pair<T> lv[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = min(tid + k * NTB, 3 * 256 - 1);
        const int s = i >> 8, id = i & 255;
        const int comp = s == 0 ? C0 : (s == 1 ? C1 : C2);
        const auto p = lut + (((d.kind * 6 + comp) << 8) + id) * 2;   // (a, b) of (kind, comp, id)
        lv[k].a = p[0];
        lv[k].b = p[1];
    }

    // A cell is read when its wave is live and its row and column lie in the
    // grid.  The loads of a live wave are unconditional, from the clamped
    // cell (0 for an index beyond the grid), and the null id or zero field
    // is selected after them, so that all of them are in flight at once (a
    // load under a lane mask whose byte is then shifted makes the compiler
    // wait for it inside the mask, one load after another).  The row offset
    // row[r] nx is uniform: each load takes a scalar row base and the lane's
    // column as its offset.  A skipped wave reads nothing.
    uint32_t m0p[CX][NP], m1p[CX][NP], m2p[CX][NP];
    T f0[CX][B], f1[CX][B], f2[CX][B];
    {
        constexpr uint32_t kNull4 = kNullId * 0x01010101u;
#pragma unroll
        for (int j = 0; j < CX; ++j)
#pragma unroll
            for (int q = 0; q < NP; ++q) m0p[j][q] = m1p[j][q] = m2p[j][q] = live ? 0u : kNull4;
        uint32_t b0[CX][B], b1[CX][B], b2[CX][B];
        if (live) {
            const auto I0 = as_global(g.ids[C0]), I1 = as_global(g.ids[C1]), I2 = as_global(g.ids[C2]);
            const auto S0 = src + d.field_off;
            const auto S1 = S0 + g.ncell;
            const auto S2 = S1 + g.ncell;
#pragma unroll
            for (int r = 0; r < B; ++r) {
                const int64_t ro = (int64_t)max(row[r], 0) * g.nx;
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const uint32_t cj = (uint32_t)max(col[j], 0);
                    b0[j][r] = (I0 + ro)[cj];
                    b1[j][r] = (I1 + ro)[cj];
                    b2[j][r] = (I2 + ro)[cj];
                    f0[j][r] = (S0 + ro)[cj];
                    f1[j][r] = (S1 + ro)[cj];
                    f2[j][r] = (S2 + ro)[cj];
                }
            }
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const bool in = row[r] >= 0 && col[j] >= 0;
                    m0p[j][r >> 2] |= (in ? b0[j][r] : kNullId) << (8 * (r & 3));
                    m1p[j][r >> 2] |= (in ? b1[j][r] : kNullId) << (8 * (r & 3));
                    m2p[j][r >> 2] |= (in ? b2[j][r] : kNullId) << (8 * (r & 3));
                    if (!in) f0[j][r] = f1[j][r] = f2[j][r] = T(0);
                }
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) f0[j][r] = f1[j][r] = f2[j][r] = T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = tid + k * NTB;
        if (i < 3 * 256) L[i >> 8][i & 255] = lv[k];
    }
    const bool stile = tile == g.stile;
    // The surface tile keeps its channel's surface tables in LDS for the
    // launch when they fit: the stage offset of every stencil point (its
    // grid index converted once), the weights, the basis row and K(t_m) of
    // the launch's steps.  The sum after each step then reads no global
    // memory, in the same order as the table path.
    const bool staged = stile && d.nsamp <= kSurfCap && d.P <= kSurfP;
    if (staged) {
        const int ne = d.nsamp * d.P;
        const auto gi = as_global(t.gidx) + d.g_off;
        const auto gw = as_global(t.gw) + d.g_off;
        for (int e = tid; e < ne; e += NTB) {
            const int32_t idx = gi[e];
            const int gx = idx % g.nx, gy = idx / g.nx;
            const int cx = gx - rx0;
            s_off[e] = (uint16_t)((gy - ry0) * RW + (cx % CX) * 64 + cx / CX);
            s_w[e] = gw[e];
        }
        for (int i = tid; i < d.nsamp; i += NTB) s_b[i] = as_global(t.basis)[d.basis_off + i];
        if (tid < ksteps) s_k[tid] = as_global(g.ktab)[m0 + tid];
    }
    double acc_s = 0.0, acc_c = 0.0;
    if (stile && tid == 0) {
        acc_s = acc[0];
        acc_c = acc[1];
    }
    __syncthreads();

#define CF_ID(p, j, r) ((p[j][(r) >> 2] >> (8 * ((r) & 3))) & 255u)
    // CREG: each cell's (a, b) pairs are constant over the launch and can be
    // held in registers instead of being looked up in LDS every step.
    constexpr int KJ = CREG ? CX : 1, KB = CREG ? B : 1;
    Pair<T> k0[KJ][KB], k1[KJ][KB], k2[KJ][KB];
    if constexpr (CREG) {
        if (live)
#pragma unroll
        for (int j = 0; j < CX; ++j)
#pragma unroll
            for (int r = 0; r < B; ++r) {
                k0[j % KJ][r % KB] = L[0][CF_ID(m0p, j, r)];
                k1[j % KJ][r % KB] = L[1][CF_ID(m1p, j, r)];
                k2[j % KJ][r % KB] = L[2][CF_ID(m2p, j, r)];
            }
    }
#define CF_K(s, j, r) (CREG ? k##s[(j) % KJ][(r) % KB] : L[s][CF_ID(m##s##p, j, r)])
    // Unrolled over the KH steps of a launch: a rolled loop ends every step
    // with a copy of each field into the register the next step reads.
#pragma unroll
    for (int step = 0; step < KH; ++step) {
        if (step >= ksteps) break;
        // ---- H half: needs the E row above the wave's band ----
        T e_above[CX];
#pragma unroll
        for (int j = 0; j < CX; ++j) xe[w][j][lane] = f0[j][0];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CX; ++j) e_above[j] = w + 1 < RBW ? xe[w + 1][j][lane] : f0[j][B - 1];
        if (!live) {
        } else if (POL == CF_POL_TM) {
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const T ez = f0[j][r];
                    const T ezr = j + 1 < CX ? f0[(j + 1) % CX][r] : from_next(f0[0][r]);
                    const T ezu = r + 1 < B ? f0[j][(r + 1) % B] : e_above[j];
                    const Pair<T> cx = CF_K(1, j, r), cy = CF_K(2, j, r);
                    yee::sub_into(f1[j][r], cx.a, cx.b, ezu - ez);
                    yee::sub_into(f2[j][r], cy.a, cy.b, ez - ezr);
                }
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const T ex = f0[j][r], ey = f1[j][r];
                    const T eyr = j + 1 < CX ? f1[(j + 1) % CX][r] : from_next(f1[0][r]);
                    const T exu = r + 1 < B ? f0[j][(r + 1) % B] : e_above[j];
                    const Pair<T> cz = CF_K(2, j, r);
                    yee::sub_into(f2[j][r], cz.a, cz.b, (eyr - ey) - (exu - ex));
                }
        }
        // ---- E half: needs the H row below the wave's band ----
        T h_below[CX];
#pragma unroll
        for (int j = 0; j < CX; ++j) xh[w][j][lane] = POL == CF_POL_TM ? f1[j][B - 1] : f2[j][B - 1];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CX; ++j)
            h_below[j] = w > 0 ? xh[w - 1][j][lane] : (POL == CF_POL_TM ? f1[j][0] : f2[j][0]);
        if (!live) {
        } else if (POL == CF_POL_TM) {
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const T hx = f1[j][r], hy = f2[j][r];
                    const T hyl = j > 0 ? f2[(j + CX - 1) % CX][r] : from_prev(f2[CX - 1][r]);
                    const T hxd = r > 0 ? f1[j][(r + B - 1) % B] : h_below[j];
                    const T curl = (hy - hyl) - (hx - hxd);
                    const Pair<T> cz = CF_K(0, j, r);
                    yee::add_into(f0[j][r], cz.a, cz.b, curl);
                }
        } else {
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const T hz = f2[j][r];
                    const T hzl = j > 0 ? f2[(j + CX - 1) % CX][r] : from_prev(f2[CX - 1][r]);
                    const T hzd = r > 0 ? f2[j][(r + B - 1) % B] : h_below[j];
                    const Pair<T> cx = CF_K(0, j, r), cy = CF_K(1, j, r);
                    yee::add_into(f0[j][r], cx.a, cx.b, hz - hzd);
                    yee::sub_into(f1[j][r], cy.a, cy.b, hz - hzl);
                }
        }
        if (stile) {
            const int ms = d.meas_slot;
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j)
                    stage[(w * B + r) * RW + j * 64 + lane] = ms == 0 ? f0[j][r] : (ms == 1 ? f1[j][r] : f2[j][r]);
            __syncthreads();
            double s;
            if (staged) {
                yee::wave_surface_partials_staged(
                    d.nsamp, d.P, s_off, s_w, s_b, [&](uint16_t o) { return (double)stage[o]; }, red);
                __syncthreads();
                s = tid == 0 ? yee::wave_partials_total(red) : 0.0;
            } else {
                s = block_surface_sum(
                    d, t,
                    [&](int32_t idx) {
                        const int gx = idx % g.nx, gy = idx / g.nx;
                        const int cx = gx - rx0;
                        return (double)stage[(gy - ry0) * RW + (cx % CX) * 64 + cx / CX];
                    },
                    red);
            }
            if (tid == 0) {
                const double G = g.dA * s;
                const int m = m0 + step;
                const double kt = staged ? s_k[step] : as_global(g.ktab)[m];
                neumaier(acc_s, acc_c, (g.dt * kt) * G);
                if (g.gamma) as_global(g.gamma)[(int64_t)m * g.gamma_stride + d.local] = G;
            }
            __syncthreads();
        }
    }
#undef CF_K
#undef CF_ID
    if (stile && tid == 0) {
        acc[0] = acc_s;
        acc[1] = acc_c;
    }
    if (!live) return;   // its cells are 0 in both arrays already
    const auto D0 = dst + d.field_off;
    const auto D1 = D0 + g.ncell;
    const auto D2 = D1 + g.ncell;
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const int ry = w * B + r;   // uniform: the row test is a scalar branch
        const int gy = ry0 + ry;
        if (ry < KH || ry >= KH + TY || gy < 0 || gy >= g.ny) continue;
        const int64_t ro = (int64_t)gy * g.nx;
#pragma unroll
        for (int j = 0; j < CX; ++j) {
            const int cx = lane * CX + j;
            const int gx = rx0 + cx;
            if (cx < KH || cx >= KH + TX || gx < 0 || gx >= g.nx) continue;
            (D0 + ro)[(uint32_t)gx] = f0[j][r];
            (D1 + ro)[(uint32_t)gx] = f1[j][r];
            (D2 + ro)[(uint32_t)gx] = f2[j][r];
        }
    }
}

inline dim3 grid2d(const Grid2D& g, int nslots) {
    const int tiles = ((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY);
    return dim3(tiles, nslots, 1);
}

}  // namespace

// Register-blocking variants: W waves of B rows, CX columns per lane and
// halo KH give a tile of (64 CX - 2 KH) x (W B - 2 KH) cells and at most KH
// steps per launch.  All variants evaluate the same arithmetic; the
// autotuner picks among them.  Indices are part of the ABI (tile_variant).
struct RbVariant {
    int W, B, KH;
    bool creg;   // coefficients held in registers over the launch
    int CX;
};
constexpr RbVariant kRbF32[] = {{8, 8, 8, false, 1},  {8, 8, 6, false, 1},  {8, 8, 4, false, 1},
                                {16, 4, 8, false, 1}, {8, 8, 8, true, 1},   {16, 4, 8, true, 1},
                                {8, 8, 6, true, 1},   {16, 4, 8, false, 2}, {8, 8, 8, false, 2},
                                {16, 4, 8, true, 2},  {8, 8, 8, true, 2},   {7, 8, 8, true, 1},
                                {8, 7, 8, true, 1}};
constexpr RbVariant kRbF64[] = {{8, 4, 4, false, 1}, {8, 4, 2, false, 1}, {16, 4, 4, false, 1},
                                {16, 4, 4, true, 1}, {8, 4, 4, false, 2}};

template <typename T>
static const RbVariant* rb_table(int* n) {
    if (sizeof(T) == 4) {
        *n = sizeof(kRbF32) / sizeof(kRbF32[0]);
        return kRbF32;
    }
    *n = sizeof(kRbF64) / sizeof(kRbF64[0]);
    return kRbF64;
}

template <typename T>
int tb_variants(TBShape* out, int max) {
    int n;
    const RbVariant* v = rb_table<T>(&n);
    for (int i = 0; i < n && i < max; ++i)
        out[i] = TBShape{64 * v[i].CX - 2 * v[i].KH, v[i].W * v[i].B - 2 * v[i].KH, v[i].KH, v[i].B};
    return n;
}
template int tb_variants<float>(TBShape*, int);
template int tb_variants<double>(TBShape*, int);

template <typename T>
hipError_t launch_h2d(int pol, int mode, T* fields, const ChanDev* ch, const int* slots, int nslots,
                      const Grid2D& g, const T* lut, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    dim3 grid = grid2d(g, nslots), block(BX, BY, 1);
    if (pol == CF_POL_TM) {
        if (mode == 0) hipLaunchKernelGGL((k_h2d<T, CF_POL_TM, 0>), grid, block, 0, s, fields, ch, slots, g, lut);
        else hipLaunchKernelGGL((k_h2d<T, CF_POL_TM, 1>), grid, block, 0, s, fields, ch, slots, g, lut);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_h2d<T, CF_POL_TE, 0>), grid, block, 0, s, fields, ch, slots, g, lut);
        else hipLaunchKernelGGL((k_h2d<T, CF_POL_TE, 1>), grid, block, 0, s, fields, ch, slots, g, lut);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_e2d(int pol, int mode, T* fields, const ChanDev* ch, const int* slots, int nslots,
                      const Grid2D& g, const T* lut, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    dim3 grid = grid2d(g, nslots), block(BX, BY, 1);
    if (pol == CF_POL_TM) {
        if (mode == 0) hipLaunchKernelGGL((k_e2d<T, CF_POL_TM, 0>), grid, block, 0, s, fields, ch, slots, g, lut);
        else hipLaunchKernelGGL((k_e2d<T, CF_POL_TM, 1>), grid, block, 0, s, fields, ch, slots, g, lut);
    } else {
        if (mode == 0) hipLaunchKernelGGL((k_e2d<T, CF_POL_TE, 0>), grid, block, 0, s, fields, ch, slots, g, lut);
        else hipLaunchKernelGGL((k_e2d<T, CF_POL_TE, 1>), grid, block, 0, s, fields, ch, slots, g, lut);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_kick(T* fields, const ChanDev* ch, const int* slots, int nslots, int max_uniq,
                       const SurfTables& t, hipStream_t s) {
    if (nslots <= 0 || max_uniq <= 0) return hipSuccess;
    dim3 grid((max_uniq + 255) / 256, nslots, 1);
    hipLaunchKernelGGL((k_kick<T>), grid, dim3(256), 0, s, fields, ch, slots, t);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_surface(const T* fields, const ChanDev* ch, const int* slots, int nslots,
                          const SurfTables& t, const double* ktab, int m, double dt, double dA,
                          double* acc, double* gamma, int gamma_stride, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_surface<T>), dim3(nslots), dim3(NT), 0, s, fields, ch, slots, t, ktab, m,
                       dt, dA, acc, gamma, gamma_stride);
    return hipGetLastError();
}

// waves per SIMD the register budget is sized for: the field state per lane
// is 3 B CX values of sizeof(T) bytes (plus as many coefficient pairs with
// creg).  An FP32 shape that reads its coefficients from LDS fits 6 waves
// (76 VGPRs, no spills), three 8-wave blocks per CU.
constexpr int rb_wpe(int B, bool creg, int CX, int tsize) {
    return B * CX * (tsize / 4) >= 16 ? 2 : (creg ? 3 : (tsize == 4 ? 6 : 4));
}

template <typename T, int W, int B, int KH, bool CREG, int CX>
static void rb_launch(int pol, int nwork, hipStream_t s, const ChanDev* ch, const WorkItem* work,
                      const InstDev* inst, int kmax, int m, int parity) {
    constexpr int WPE = rb_wpe(B, CREG, CX, (int)sizeof(T));
    dim3 grid(nwork), block(64 * W);
    if (pol == CF_POL_TM)
        hipLaunchKernelGGL((k_rb2d<T, CF_POL_TM, W, B, KH, CREG, CX, WPE>), grid, block, 0, s, ch, work, inst, kmax,
                           m, parity);
    else
        hipLaunchKernelGGL((k_rb2d<T, CF_POL_TE, W, B, KH, CREG, CX, WPE>), grid, block, 0, s, ch, work, inst, kmax,
                           m, parity);
}

template <typename T>
hipError_t launch_tb2d(int variant, int pol, const ChanDev* ch, const WorkItem* work, int nwork,
                       const InstDev* inst, int kmax, int m, int parity, hipStream_t s) {
    if (nwork <= 0) return hipSuccess;
    int n;
    const RbVariant* v = rb_table<T>(&n);
    if (variant < 0 || variant >= n) return hipErrorInvalidValue;
    if (kmax < 1 || kmax > v[variant].KH) return hipErrorInvalidValue;
#define CF_RB(W, B, KH, CR, CX) rb_launch<T, W, B, KH, CR, CX>(pol, nwork, s, ch, work, inst, kmax, m, parity)
    if constexpr (sizeof(T) == 4) {
        switch (variant) {
            case 0: CF_RB(8, 8, 8, false, 1); break;
            case 1: CF_RB(8, 8, 6, false, 1); break;
            case 2: CF_RB(8, 8, 4, false, 1); break;
            case 3: CF_RB(16, 4, 8, false, 1); break;
            case 4: CF_RB(8, 8, 8, true, 1); break;
            case 5: CF_RB(16, 4, 8, true, 1); break;
            case 6: CF_RB(8, 8, 6, true, 1); break;
            case 7: CF_RB(16, 4, 8, false, 2); break;
            case 8: CF_RB(8, 8, 8, false, 2); break;
            case 9: CF_RB(16, 4, 8, true, 2); break;
            case 10: CF_RB(8, 8, 8, true, 2); break;
            case 11: CF_RB(7, 8, 8, true, 1); break;
            default: CF_RB(8, 7, 8, true, 1); break;
        }
    } else {
        switch (variant) {
            case 0: CF_RB(8, 4, 4, false, 1); break;
            case 1: CF_RB(8, 4, 2, false, 1); break;
            case 2: CF_RB(16, 4, 4, false, 1); break;
            case 3: CF_RB(16, 4, 4, true, 1); break;
            default: CF_RB(8, 4, 4, false, 2); break;
        }
    }
#undef CF_RB
    return hipGetLastError();
}

#define CF_INSTANTIATE(T)                                                                               \
    template hipError_t launch_h2d<T>(int, int, T*, const ChanDev*, const int*, int, const Grid2D&,     \
                                      const T*, hipStream_t);                                           \
    template hipError_t launch_e2d<T>(int, int, T*, const ChanDev*, const int*, int, const Grid2D&,     \
                                      const T*, hipStream_t);                                           \
    template hipError_t launch_kick<T>(T*, const ChanDev*, const int*, int, int, const SurfTables&,     \
                                       hipStream_t);                                                    \
    template hipError_t launch_surface<T>(const T*, const ChanDev*, const int*, int, const SurfTables&, \
                                          const double*, int, double, double, double*, double*, int,    \
                                          hipStream_t);                                                 \
    template hipError_t launch_tb2d<T>(int, int, const ChanDev*, const WorkItem*, int, const InstDev*,    \
                                       int, int, int, hipStream_t);
CF_INSTANTIATE(float)
CF_INSTANTIATE(double)
#undef CF_INSTANTIATE

}  // namespace cf
