// 3D Yee kernels for gfx950 (Sec. III E, the full 3D computation): H and E
// half-step updates of all six components with the uniform conductivity
// sigma in the per-kind coefficient tables, periodic or PEC walls, and a
// CPML along z (Roden-Gedney, kappa = 1, alpha = 0).
//
// Layout: a channel's field block is 6 components (Ex, Ey, Ez, Hx, Hy, Hz)
// x (nz x ny x nx) cells, x fastest; a 64 x 4 thread block covers 64
// consecutive x cells of 4 y rows of one z plane (coalesced rows).
//
// Curls (undivided differences):
//   at H_a: (curl E)_x = (Ez[j+1]-Ez) - (Ey[k+1]-Ey), (curl E)_y = (Ex[k+1]-Ex) - (Ez[i+1]-Ez),
//           (curl E)_z = (Ey[i+1]-Ey) - (Ex[j+1]-Ex);   H_a <- a H_a - b (curl E)_a
//   at E_a: (curl H)_x = (Hz-Hz[j-1]) - (Hy-Hy[k-1]), (curl H)_y = (Hx-Hx[k-1]) - (Hz-Hz[i-1]),
//           (curl H)_z = (Hy-Hy[i-1]) - (Hx-Hx[j-1]);   E_a <- a E_a + b (curl H)_a
// Inside the z layers every z difference D becomes D + psi with
// psi <- b_z psi + c_z D (b_z, c_z at the updated component's z position);
// psi lives only in the two layers (2 P planes per psi component).
#include <algorithm>

#include "../../include/casimir_fdtd.h"
#include "device.hpp"
#include "yee_common.hpp"

namespace cf {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

template <typename T>
__device__ __forceinline__ T yee_sub(T a, T x, T b, T d) { return yee::sub(a, x, b, d); }
template <typename T>
__device__ __forceinline__ T yee_add(T a, T x, T b, T d) { return yee::add(a, x, b, d); }
template <typename T>
__device__ __forceinline__ T yee_half(T b, T d) { return yee::half(b, d); }
using yee::lut_ab;

// psi plane of z index k inside the layers, or -1 outside
__device__ __forceinline__ int pml_plane(int k, int nz, int P) {
    if (P <= 0) return -1;
    if (k < P) return k;
    if (k >= nz - P) return P + (k - (nz - P));
    return -1;
}

// z difference with the CPML update: psi <- b psi + c D, returns D + psi.
// The consistent start (mode 1) advances psi too: its partner field is set
// from the stretched curl, and the first step stretches it again.
template <typename T, int MODE>
__device__ __forceinline__ T zdiff(T D, T* psi, int64_t at, T b, T c) {
    if (psi == nullptr) return D;
    const T p = fma(b, psi[at], c * D);
    psi[at] = p;
    return D + p;
}

template <typename T, int MODE>
__global__ __launch_bounds__(BX* BY) void k_h3d(T* __restrict__ fields, T* __restrict__ psi_base,
                                              const ChanDev* __restrict__ ch, const int* __restrict__ slots,
                                              Grid3D g, const T* __restrict__ lut) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 0) return;   // start: E-kind runs set H^{-1/2}
    const int tiles_x = (g.nx + BX - 1) / BX, tiles_y = (g.ny + BY - 1) / BY;
    const int tile = blockIdx.x;
    const int i = (tile % tiles_x) * BX + threadIdx.x;
    const int j = ((tile / tiles_x) % tiles_y) * BY + threadIdx.y;
    const int k = tile / (tiles_x * tiles_y);
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    T* F = fields + d.field_off;
    const int64_t n = g.ncell;
    const int64_t c = ((int64_t)k * g.ny + j) * g.nx + i;
    const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
    // +1 neighbours (0 beyond a PEC/PML wall, wrapped when periodic)
    const bool rx = i + 1 < g.nx, ry = j + 1 < g.ny, rz = k + 1 < g.nz;
    const int64_t cx = rx ? c + sx : (g.per[0] ? c + sx - (int64_t)g.nx * sx : -1);
    const int64_t cy = ry ? c + sy : (g.per[1] ? c + sy - (int64_t)g.ny * sy : -1);
    const int64_t cz = rz ? c + sz : (g.per[2] ? c + sz - (int64_t)g.nz * sz : -1);
    const T* Ex = F;
    const T* Ey = F + n;
    const T* Ez = F + 2 * n;
    const T ex = Ex[c], ey = Ey[c], ez = Ez[c];
    const T ez_y = cy >= 0 ? Ez[cy] : T(0), ey_z = cz >= 0 ? Ey[cz] : T(0);
    const T ex_z = cz >= 0 ? Ex[cz] : T(0), ez_x = cx >= 0 ? Ez[cx] : T(0);
    const T ey_x = cx >= 0 ? Ey[cx] : T(0), ex_y = cy >= 0 ? Ex[cy] : T(0);
    const int plane = pml_plane(k, g.nz, g.pml);
    T* psi = (plane >= 0 && psi_base) ? psi_base + d.psi_off : nullptr;
    const int64_t pat = plane >= 0 ? ((int64_t)plane * g.ny + j) * g.nx + i : 0;
    const T bz = g.pml > 0 ? (T)g.pml_bh[k] : T(1), czz = g.pml > 0 ? (T)g.pml_ch[k] : T(0);
    // psi components: 0 Hx (dz Ey), 1 Hy (dz Ex), 2 Ex (dz Hy), 3 Ey (dz Hx)
    const T dzEy = zdiff<T, MODE>(ey_z - ey, psi, pat, bz, czz);
    const T dzEx = zdiff<T, MODE>(ex_z - ex, psi ? psi + g.psi_comp : nullptr, pat, bz, czz);
    const T curl_x = (ez_y - ez) - dzEy;
    const T curl_y = dzEx - (ez_x - ez);
    const T curl_z = (ey_x - ey) - (ex_y - ex);
    T* Hx = F + 3 * n;
    T* Hy = F + 4 * n;
    T* Hz = F + 5 * n;
    const T* lx = lut_ab(lut, d.kind, CF_HX, g.ids[CF_HX][c]);
    const T* ly = lut_ab(lut, d.kind, CF_HY, g.ids[CF_HY][c]);
    const T* lz = lut_ab(lut, d.kind, CF_HZ, g.ids[CF_HZ][c]);
    if (MODE == 0) {
        Hx[c] = yee_sub(lx[0], Hx[c], lx[1], curl_x);
        Hy[c] = yee_sub(ly[0], Hy[c], ly[1], curl_y);
        Hz[c] = yee_sub(lz[0], Hz[c], lz[1], curl_z);
    } else {
        Hx[c] = yee_half(lx[1], curl_x);
        Hy[c] = yee_half(ly[1], curl_y);
        Hz[c] = yee_half(lz[1], curl_z);
    }
}

template <typename T, int MODE>
__global__ __launch_bounds__(BX* BY) void k_e3d(T* __restrict__ fields, T* __restrict__ psi_base,
                                              const ChanDev* __restrict__ ch, const int* __restrict__ slots,
                                              Grid3D g, const T* __restrict__ lut) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 1) return;   // start: H-kind runs set E^{+1/2}
    const int tiles_x = (g.nx + BX - 1) / BX, tiles_y = (g.ny + BY - 1) / BY;
    const int tile = blockIdx.x;
    const int i = (tile % tiles_x) * BX + threadIdx.x;
    const int j = ((tile / tiles_x) % tiles_y) * BY + threadIdx.y;
    const int k = tile / (tiles_x * tiles_y);
    if (i >= g.nx || j >= g.ny || k >= g.nz) return;
    T* F = fields + d.field_off;
    const int64_t n = g.ncell;
    const int64_t c = ((int64_t)k * g.ny + j) * g.nx + i;
    const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
    // -1 neighbours (0 beyond a PEC/PML wall, wrapped when periodic)
    const int64_t cx = i > 0 ? c - sx : (g.per[0] ? c - sx + (int64_t)g.nx * sx : -1);
    const int64_t cy = j > 0 ? c - sy : (g.per[1] ? c - sy + (int64_t)g.ny * sy : -1);
    const int64_t cz = k > 0 ? c - sz : (g.per[2] ? c - sz + (int64_t)g.nz * sz : -1);
    const T* Hx = F + 3 * n;
    const T* Hy = F + 4 * n;
    const T* Hz = F + 5 * n;
    const T hx = Hx[c], hy = Hy[c], hz = Hz[c];
    const T hz_y = cy >= 0 ? Hz[cy] : T(0), hy_z = cz >= 0 ? Hy[cz] : T(0);
    const T hx_z = cz >= 0 ? Hx[cz] : T(0), hz_x = cx >= 0 ? Hz[cx] : T(0);
    const T hy_x = cx >= 0 ? Hy[cx] : T(0), hx_y = cy >= 0 ? Hx[cy] : T(0);
    const int plane = pml_plane(k, g.nz, g.pml);
    T* psi = (plane >= 0 && psi_base) ? psi_base + d.psi_off : nullptr;
    const int64_t pat = plane >= 0 ? ((int64_t)plane * g.ny + j) * g.nx + i : 0;
    const T bz = g.pml > 0 ? (T)g.pml_be[k] : T(1), czz = g.pml > 0 ? (T)g.pml_ce[k] : T(0);
    const T dzHy = zdiff<T, MODE>(hy - hy_z, psi ? psi + 2 * g.psi_comp : nullptr, pat, bz, czz);
    const T dzHx = zdiff<T, MODE>(hx - hx_z, psi ? psi + 3 * g.psi_comp : nullptr, pat, bz, czz);
    const T curl_x = (hz - hz_y) - dzHy;
    const T curl_y = dzHx - (hz - hz_x);
    const T curl_z = (hy - hy_x) - (hx - hx_y);
    T* Ex = F;
    T* Ey = F + n;
    T* Ez = F + 2 * n;
    const T* lx = lut_ab(lut, d.kind, CF_EX, g.ids[CF_EX][c]);
    const T* ly = lut_ab(lut, d.kind, CF_EY, g.ids[CF_EY][c]);
    const T* lz = lut_ab(lut, d.kind, CF_EZ, g.ids[CF_EZ][c]);
    if (MODE == 0) {
        Ex[c] = yee_add(lx[0], Ex[c], lx[1], curl_x);
        Ey[c] = yee_add(ly[0], Ey[c], ly[1], curl_y);
        Ez[c] = yee_add(lz[0], Ez[c], lz[1], curl_z);
    } else {
        Ex[c] = yee_half(lx[1], curl_x);
        Ey[c] = yee_half(ly[1], curl_y);
        Ez[c] = yee_half(lz[1], curl_z);
    }
}


// ---------------------------------------------------------------------------
// Fused 3D step: one full time step (H then E) per launch, streaming in z.
//
// Block (band b, channel slots[blockIdx.y]) owns the interior rows
// y0 .. y0 + band - 1 (y0 = b band) of every z plane, for the whole x range:
// lane l of wave w holds columns l, l + 64, .. (CX of them, so every load of
// a row is one contiguous 64-value segment) of rows w B .. w B + B - 1
// of a region that starts one row below y0 (region row 0 and row W B - 1 are
// halo rows, computed but never stored).  The block marches k = 0 .. nz - 1
// keeping E(k), E(k+1), H(k) and the new H(k-1) of its columns in registers:
//   H_new(k) needs E(k), E(k+1) and the x+1 / y+1 neighbours of E(k);
//   E_new(k) needs H_new(k), H_new(k-1) and the x-1 / y-1 neighbours of H_new(k).
// x neighbours come from the next / previous lane (DPP) or, across a
// 64-column segment, from a lane broadcast of the neighbouring register; at
// the row ends a periodic wall takes column 0 / nx - 1 (lane broadcast), a
// PEC wall reads 0.  y neighbours
// inside a wave's rows are registers, across waves one LDS row per half step.
// Reads come from src (fields and CPML psi) and writes go to dst, so the
// halo rows a block reads are never the rows a neighbouring block writes in
// the same launch.  z walls are PEC or CPML (periodic z is not handled here).
// The arithmetic of every cell is that of k_h3d followed by k_e3d.
constexpr int kF3MaxPml = 64;   // CPML layers the fused 3D step stages in LDS

// LDS of a fused 3D block (dynamic, carved in this order): the kind's
// coefficient pairs [6][256], the E exchange rows [W][2][CX][64], the H
// exchange rows [W][2][CX][64] and the CPML coefficients [4][2 kF3MaxPml].
template <typename T>
constexpr size_t f3_lds_bytes(int W, int CX) {
    return (size_t)6 * 256 * 2 * sizeof(T) + (size_t)2 * W * 2 * CX * 64 * sizeof(T) +
           (size_t)4 * 2 * kF3MaxPml * sizeof(T);
}
constexpr size_t kF3LdsMax = 160 * 1024;   // LDS of a gfx950 CU

// Logical (band, slot, chunk) of a fused 3D block.  Blocks are dispatched
// to the 8 XCDs round-robin in flat-id order; numbering the logical blocks so
// that XCD x takes a contiguous range keeps neighbouring bands of a channel
// (which read each other's halo rows) on one XCD and its L2.  The logical
// order is band, then z chunk, then channel, so each XCD takes whole channels
// and the same mix of chunks (chunks below a conductor may be short or
// empty, see f3_chunk).
struct F3Block {
    int band, slot, chunk;
};
__device__ __forceinline__ F3Block f3_block() {
    const unsigned nb = gridDim.x, nc = gridDim.z;
    const unsigned total = nb * gridDim.y * nc;
    const unsigned h = blockIdx.x + nb * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned q = total / 8, r = total % 8, x = h % 8;
    const unsigned l = x * q + min(x, r) + h / 8;
    return F3Block{(int)(l % nb), (int)(l / (nb * nc)), (int)((l / nb) % nc)};
}

// The z chunk of a block, clipped to the planes its band can change.
__device__ __forceinline__ void f3_chunk(const Grid3D& g, const int2* zr, const F3Block& b, int* z0, int* z1) {
    const int zc = (g.nz + (int)gridDim.z - 1) / (int)gridDim.z;
    *z0 = b.chunk * zc;
    *z1 = min(g.nz, *z0 + zc);
    if (zr) {
        const int2 r = zr[b.band];
        *z0 = max(*z0, r.x);
        *z1 = min(*z1, r.y);
    }
}

template <typename T, int W, int B, int CX>
__global__ __launch_bounds__(64 * W) void k_f3d(const ChanDev* __restrict__ ch, const int* __restrict__ slots,
                                                 Grid3D g, const T* __restrict__ lut, const T* __restrict__ src,
                                                 T* __restrict__ dst, const T* __restrict__ psrc,
                                                 T* __restrict__ pdst, int band, const int2* __restrict__ zr) {
    constexpr int NTB = 64 * W;
    extern __shared__ double f3_lds[];
    yee::Pair<T> (*L)[256] = reinterpret_cast<yee::Pair<T> (*)[256]>(f3_lds);   // [6][256] coefficient pairs
    char* const lds_xe = reinterpret_cast<char*>(f3_lds) + (size_t)6 * 256 * 2 * sizeof(T);
    char* const lds_xh = lds_xe + (size_t)W * 2 * CX * 64 * sizeof(T);
    T (*xe)[2][CX][64] = reinterpret_cast<T (*)[2][CX][64]>(lds_xe);   // first region row of each wave: Ez, Ex
    T (*xh)[2][CX][64] = reinterpret_cast<T (*)[2][CX][64]>(lds_xh);   // last region row of each wave: Hz, Hx
    T (*Lz)[2 * kF3MaxPml] =                                           // CPML b, c of the layer planes
        reinterpret_cast<T (*)[2 * kF3MaxPml]>(lds_xh + (size_t)W * 2 * CX * 64 * sizeof(T));
    const F3Block fb = f3_block();
    const ChanDev d = ch[slots[fb.slot]];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int yb = fb.band * band - 1;               // global y of region row 0
    for (int i = threadIdx.x; i < 6 * 256; i += NTB) {
        const int comp = i >> 8, id = i & 255;
        const T* p = lut_ab(lut, d.kind, comp, id);
        L[comp][id].a = p[0];
        L[comp][id].b = p[1];
    }
    for (int i = threadIdx.x; i < 2 * g.pml; i += NTB) {
        const int kz = i < g.pml ? i : g.nz - 2 * g.pml + i;   // psi plane i -> z index
        Lz[0][i] = (T)g.pml_bh[kz];
        Lz[1][i] = (T)g.pml_ch[kz];
        Lz[2][i] = (T)g.pml_be[kz];
        Lz[3][i] = (T)g.pml_ce[kz];
    }
    const int64_t n = g.ncell, sz = (int64_t)g.nx * g.ny;
    const T* __restrict__ S = src + d.field_off;
    T* __restrict__ D = dst + d.field_off;
    int64_t rowoff[B];
    bool rin[B], rst[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const int ry = w * B + r;
        int y = yb + ry;
        bool in = true;
        if (y < 0 || y >= g.ny) {
            if (g.per[1]) y = ((y % g.ny) + g.ny) % g.ny;
            else in = false;
        }
        rin[r] = in;
        rowoff[r] = (int64_t)y * g.nx;
        rst[r] = in && ry >= 1 && ry <= band && yb + ry < g.ny;   // stored (interior) row
    }
    bool cin[CX];
#pragma unroll
    for (int j = 0; j < CX; ++j) cin[j] = j * 64 + lane < g.nx;
    const bool perx = g.per[0] != 0;
    const int lastj = (g.nx - 1) / 64, lastl = (g.nx - 1) % 64;   // register / lane of column nx - 1
    const bool T_PSI = g.pml > 0 && psrc != nullptr;

    // z chunk of this block: planes z0 .. z1-1 are stored; a chunk that does
    // not start at 0 first marches plane z0 - 1 to obtain H_new(z0 - 1)
    // (nothing of that plane is stored)
    int z0, z1;
    f3_chunk(g, zr, fb, &z0, &z1);
    if (z0 >= z1) return;                          // whole block: before any barrier
    const int kb = z0 > 0 ? z0 - 1 : 0;
    // Loads are issued from clamped (always valid) addresses and masked only
    // where the values are taken up, one plane later for the prefetched set,
    // so the memory latency overlaps a whole plane of arithmetic.
    bool vc[B][CX];                          // cell (r, j) lies in the grid
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int j = 0; j < CX; ++j) vc[r][j] = rin[r] && cin[j];
    auto raw3 = [&](int k, int comp0, T (&a)[B][CX], T (&b)[B][CX], T (&c)[B][CX]) {
        const int64_t pk = (int64_t)min(max(k, 0), g.nz - 1) * sz;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const int64_t at = comp0 * n + (vc[r][j] ? pk + rowoff[r] + j * 64 + lane : 0);
                a[r][j] = S[at];
                b[r][j] = S[n + at];
                c[r][j] = S[2 * n + at];
            }
    };
    auto raw_ids = [&](int k, uint2 (&id)[B][CX]) {
        const int64_t pk = (int64_t)min(max(k, 0), g.nz - 1) * sz;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j)
                id[r][j] = g.idp[vc[r][j] ? pk + rowoff[r] + j * 64 + lane : 0];
    };
    auto mask3 = [&](bool kin, T (&a)[B][CX], T (&b)[B][CX], T (&c)[B][CX]) {
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const bool v = kin && vc[r][j];
                a[r][j] = v ? a[r][j] : T(0);
                b[r][j] = v ? b[r][j] : T(0);
                c[r][j] = v ? c[r][j] : T(0);
            }
    };
    // null material (kNullId, a = b = 0) for cells outside the grid
    constexpr uint32_t kNull4 = 0x01010101u * kNullId, kNull2 = 0x0101u * kNullId;

    T ex[B][CX], ey[B][CX], ez[B][CX];       // E(k)
    T ex1[B][CX], ey1[B][CX], ez1[B][CX];    // E(k+1)
    T hx[B][CX], hy[B][CX], hz[B][CX];       // H(k), then H_new(k)
    uint32_t id0[B][CX], id1[B][CX];         // material ids of plane k (Ex Ey Ez Hx | Hy Hz)
    T px[B][CX], py[B][CX];                  // H_new(k-1): Hx, Hy
    {
        uint2 i2[B][CX];
        raw3(kb, 0, ex, ey, ez);
        raw3(kb + 1, 0, ex1, ey1, ez1);
        raw3(kb, 3, hx, hy, hz);
        raw_ids(kb, i2);
        mask3(true, ex, ey, ez);
        mask3(kb + 1 < g.nz, ex1, ey1, ez1);
        mask3(true, hx, hy, hz);
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                id0[r][j] = vc[r][j] ? i2[r][j].x : kNull4;
                id1[r][j] = vc[r][j] ? i2[r][j].y : kNull2;
                px[r][j] = T(0);
                py[r][j] = T(0);
            }
    }
    __syncthreads();   // coefficient table

    for (int k = kb; k < z1; ++k) {
        const int64_t pk = (int64_t)k * sz;
        const bool warm = k < z0;                  // uniform over the block
        const int plane = pml_plane(k, g.nz, g.pml);
        const bool zp = T_PSI && plane >= 0;       // uniform
        const T bh = zp ? Lz[0][plane] : T(1), chh = zp ? Lz[1][plane] : T(0);
        const T be = zp ? Lz[2][plane] : T(1), ce = zp ? Lz[3][plane] : T(0);
        const int64_t pp = (int64_t)plane * sz;
        // this plane's psi (layer planes only), loaded before the prefetch so
        // that waiting for it does not wait for the next plane's inputs
        T ps[4][B][CX];
        if (zp) {
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const int64_t pa = d.psi_off + (vc[r][j] ? pp + rowoff[r] + j * 64 + lane : 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) ps[q][r][j] = psrc[pa + q * g.psi_comp];
                }
        }
        // next plane's inputs, issued before this plane's arithmetic
        T ex2[B][CX], ey2[B][CX], ez2[B][CX];
        T hxn[B][CX], hyn[B][CX], hzn[B][CX];
        uint2 idn[B][CX];
        raw3(k + 2, 0, ex2, ey2, ez2);
        raw3(k + 1, 3, hxn, hyn, hzn);
        raw_ids(k + 1, idn);

        // ---- H half ----
#pragma unroll
        for (int j = 0; j < CX; ++j) {
            xe[w][0][j][lane] = ez[0][j];
            xe[w][1][j][lane] = ex[0][j];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < B; ++r) {
            // x + 1 neighbours: the next lane, or lane 0 of the next register
            // for lane 63; column 0 of the row for the periodic wrap
            T nez[CX], ney[CX];
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const T a = yee::from_next(ez[r][j]), b = yee::from_next(ey[r][j]);
                const T a1 = j + 1 < CX ? yee::lane_value(ez[r][(j + 1) % CX], 0) : T(0);
                const T b1 = j + 1 < CX ? yee::lane_value(ey[r][(j + 1) % CX], 0) : T(0);
                nez[j] = lane == 63 ? a1 : a;
                ney[j] = lane == 63 ? b1 : b;
            }
            const T fez = yee::lane_value(ez[r][0], 0), fey = yee::lane_value(ey[r][0], 0);
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                T ez_y, ex_y;
                if (r + 1 < B) {
                    ez_y = ez[(r + 1) % B][j];
                    ex_y = ex[(r + 1) % B][j];
                } else if (w + 1 < W) {
                    ez_y = xe[(w + 1) % W][0][j][lane];
                    ex_y = xe[(w + 1) % W][1][j][lane];
                } else {
                    ez_y = T(0);   // last region row: halo, never stored
                    ex_y = T(0);
                }
                T ez_x = nez[j];
                T ey_x = ney[j];
                if (j * 64 + lane == g.nx - 1) {
                    ez_x = perx ? fez : T(0);
                    ey_x = perx ? fey : T(0);
                }
                T dzEy = ey1[r][j] - ey[r][j];
                T dzEx = ex1[r][j] - ex[r][j];
                if (zp && vc[r][j]) {
                    const int64_t pa = d.psi_off + pp + rowoff[r] + j * 64 + lane;
                    const T p0 = fma(bh, ps[0][r][j], chh * dzEy);
                    const T p1 = fma(bh, ps[1][r][j], chh * dzEx);
                    if (rst[r] && !warm) {
                        pdst[pa] = p0;
                        pdst[pa + g.psi_comp] = p1;
                    }
                    dzEy = dzEy + p0;
                    dzEx = dzEx + p1;
                }
                const T curl_x = (ez_y - ez[r][j]) - dzEy;
                const T curl_y = dzEx - (ez_x - ez[r][j]);
                const T curl_z = (ey_x - ey[r][j]) - (ex_y - ex[r][j]);
                const yee::Pair<T> cx = L[CF_HX][id0[r][j] >> 24];
                const yee::Pair<T> cy = L[CF_HY][id1[r][j] & 255u];
                const yee::Pair<T> cz = L[CF_HZ][(id1[r][j] >> 8) & 255u];
                const bool v = rin[r] && cin[j];
                hx[r][j] = v ? yee_sub(cx.a, hx[r][j], cx.b, curl_x) : T(0);
                hy[r][j] = v ? yee_sub(cy.a, hy[r][j], cy.b, curl_y) : T(0);
                hz[r][j] = v ? yee_sub(cz.a, hz[r][j], cz.b, curl_z) : T(0);
            }
        }

        // ---- E half (not on the warm-up plane) ----
        if (!warm) {
#pragma unroll
        for (int j = 0; j < CX; ++j) {
            xh[w][0][j][lane] = hz[B - 1][j];
            xh[w][1][j][lane] = hx[B - 1][j];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < B; ++r) {
            // x - 1 neighbours: the previous lane, or lane 63 of the previous
            // register for lane 0; column nx - 1 of the row for the periodic wrap
            T phz[CX], phy[CX];
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const T a = yee::from_prev(hz[r][j]), b = yee::from_prev(hy[r][j]);
                const T a1 = j > 0 ? yee::lane_value(hz[r][(j + CX - 1) % CX], 63) : T(0);
                const T b1 = j > 0 ? yee::lane_value(hy[r][(j + CX - 1) % CX], 63) : T(0);
                phz[j] = lane == 0 ? a1 : a;
                phy[j] = lane == 0 ? b1 : b;
            }
            T lhz = hz[r][0], lhy = hy[r][0];
#pragma unroll
            for (int j = 1; j < CX; ++j)
                if (lastj == j) {
                    lhz = hz[r][j];
                    lhy = hy[r][j];
                }
            lhz = yee::lane_value(lhz, lastl);
            lhy = yee::lane_value(lhy, lastl);
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                T hz_y, hx_y;
                if (r > 0) {
                    hz_y = hz[(r + B - 1) % B][j];
                    hx_y = hx[(r + B - 1) % B][j];
                } else if (w > 0) {
                    hz_y = xh[(w + W - 1) % W][0][j][lane];
                    hx_y = xh[(w + W - 1) % W][1][j][lane];
                } else {
                    hz_y = T(0);   // region row 0: halo, never stored
                    hx_y = T(0);
                }
                T hz_x = phz[j];
                T hy_x = phy[j];
                if (j * 64 + lane == 0) {
                    hz_x = perx ? lhz : T(0);
                    hy_x = perx ? lhy : T(0);
                }
                T dzHy = hy[r][j] - py[r][j];
                T dzHx = hx[r][j] - px[r][j];
                if (zp && vc[r][j]) {
                    const int64_t pa = d.psi_off + 2 * g.psi_comp + pp + rowoff[r] + j * 64 + lane;
                    const T p2 = fma(be, ps[2][r][j], ce * dzHy);
                    const T p3 = fma(be, ps[3][r][j], ce * dzHx);
                    if (rst[r]) {
                        pdst[pa] = p2;
                        pdst[pa + g.psi_comp] = p3;
                    }
                    dzHy = dzHy + p2;
                    dzHx = dzHx + p3;
                }
                const T curl_x = (hz[r][j] - hz_y) - dzHy;
                const T curl_y = dzHx - (hz[r][j] - hz_x);
                const T curl_z = (hy[r][j] - hy_x) - (hx[r][j] - hx_y);
                const yee::Pair<T> cx = L[CF_EX][id0[r][j] & 255u];
                const yee::Pair<T> cy = L[CF_EY][(id0[r][j] >> 8) & 255u];
                const yee::Pair<T> cz = L[CF_EZ][(id0[r][j] >> 16) & 255u];
                const T nex = yee_add(cx.a, ex[r][j], cx.b, curl_x);
                const T ney = yee_add(cy.a, ey[r][j], cy.b, curl_y);
                const T nez = yee_add(cz.a, ez[r][j], cz.b, curl_z);
                if (rst[r] && cin[j]) {
                    const int64_t at = pk + rowoff[r] + j * 64 + lane;
                    D[at] = nex;
                    D[n + at] = ney;
                    D[2 * n + at] = nez;
                    D[3 * n + at] = hx[r][j];
                    D[4 * n + at] = hy[r][j];
                    D[5 * n + at] = hz[r][j];
                }
            }
        }
        } else {
            __syncthreads();   // the xe rows of this plane are read before the next plane writes them
        }
        mask3(k + 2 < g.nz, ex2, ey2, ez2);
        mask3(true, hxn, hyn, hzn);
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                px[r][j] = hx[r][j];
                py[r][j] = hy[r][j];
                ex[r][j] = ex1[r][j];
                ey[r][j] = ey1[r][j];
                ez[r][j] = ez1[r][j];
                ex1[r][j] = ex2[r][j];
                ey1[r][j] = ey2[r][j];
                ez1[r][j] = ez2[r][j];
                hx[r][j] = hxn[r][j];
                hy[r][j] = hyn[r][j];
                hz[r][j] = hzn[r][j];
                id0[r][j] = vc[r][j] ? idn[r][j].x : kNull4;
                id1[r][j] = vc[r][j] ? idn[r][j].y : kNull2;
            }
    }
}

// ---------------------------------------------------------------------------
// Two-step fused 3D kernel: one launch takes a wave of channels from step n
// to step n + 2 in a single z march.  Iteration k advances plane k to step
// n + 1 (level 1: the single-step kernel's plane update) and then plane
// k - 1 to step n + 2 (level 2), which needs level-1 values of planes k - 1
// and k only; level-1 values stay in registers.  The region has two halo
// rows below and two above the band (each level uses up one row on either
// side), so band = W B - 4.  Level 2 keeps E(k-1), H(k-1) and the new
// Hx, Hy of plane k - 2; the CPML psi of a layer plane goes from level 1 to
// level 2 in registers and only level 2 writes psi.
//
// The surface projection of step n + 1 needs level-1 values: each block
// stores the measured component of its channel for the cells of its band
// that lie in the surface box `sb` (see ShadowBox).
//
// A z chunk z0 .. z1-1 starts level 1 at z0 - 2 and level 2 at z0 - 1 (the
// level-2 plane z0 - 1 gives only the H values E(z0) needs), so that a
// chunk stores exactly its own planes.  Below plane 0 and above nz - 1 the
// fields are 0 (PEC or CPML walls), as in the single-step kernel.
//
// Every level half writes its LDS row and passes its barrier even when its
// arithmetic is skipped (chunk edges), so the four exchanges of an iteration
// alternate between the two row buffers and every write is separated from
// the previous reads of that buffer by a barrier.  The arithmetic of every
// cell is that of k_h3d followed by k_e3d, twice.
template <typename T, int W, int B, int CX>
__global__ __launch_bounds__(64 * W) void k_f3d2(const ChanDev* __restrict__ ch, const int* __restrict__ slots,
                                                  Grid3D g, const T* __restrict__ lut, const T* __restrict__ src,
                                                  T* __restrict__ dst, const T* __restrict__ psrc,
                                                  T* __restrict__ pdst, T* __restrict__ shadow, ShadowBox sb,
                                                  int band, const int2* __restrict__ zr) {
    constexpr int NTB = 64 * W;
    extern __shared__ double f3_lds[];
    yee::Pair<T> (*L)[256] = reinterpret_cast<yee::Pair<T> (*)[256]>(f3_lds);   // [6][256] coefficient pairs
    char* const lds_xe = reinterpret_cast<char*>(f3_lds) + (size_t)6 * 256 * 2 * sizeof(T);
    char* const lds_xh = lds_xe + (size_t)W * 2 * CX * 64 * sizeof(T);
    T (*xe)[2][CX][64] = reinterpret_cast<T (*)[2][CX][64]>(lds_xe);   // first region row of each wave: Ez, Ex
    T (*xh)[2][CX][64] = reinterpret_cast<T (*)[2][CX][64]>(lds_xh);   // last region row of each wave: Hz, Hx
    T (*Lz)[2 * kF3MaxPml] =                                           // CPML b, c of the layer planes
        reinterpret_cast<T (*)[2 * kF3MaxPml]>(lds_xh + (size_t)W * 2 * CX * 64 * sizeof(T));
    const F3Block fb = f3_block();
    const ChanDev d = ch[slots[fb.slot]];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int yb = fb.band * band - 2;               // global y of region row 0
    for (int i = threadIdx.x; i < 6 * 256; i += NTB) {
        const int comp = i >> 8, id = i & 255;
        const T* p = lut_ab(lut, d.kind, comp, id);
        L[comp][id].a = p[0];
        L[comp][id].b = p[1];
    }
    for (int i = threadIdx.x; i < 2 * g.pml; i += NTB) {
        const int kz = i < g.pml ? i : g.nz - 2 * g.pml + i;
        Lz[0][i] = (T)g.pml_bh[kz];
        Lz[1][i] = (T)g.pml_ch[kz];
        Lz[2][i] = (T)g.pml_be[kz];
        Lz[3][i] = (T)g.pml_ce[kz];
    }
    const int64_t n = g.ncell, sz = (int64_t)g.nx * g.ny;
    const T* __restrict__ S = src + d.field_off;
    T* __restrict__ D = dst + d.field_off;
    T* __restrict__ SH = shadow + (d.field_off / (6 * n)) * sb.vol;
    int64_t rowoff[B], sbrow[B];
    bool rin[B], rst[B], sbr[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
        const int ry = w * B + r;
        int y = yb + ry;
        bool in = true;
        if (y < 0 || y >= g.ny) {
            if (g.per[1]) y = ((y % g.ny) + g.ny) % g.ny;
            else in = false;
        }
        rin[r] = in;
        rowoff[r] = (int64_t)y * g.nx;
        rst[r] = in && ry >= 2 && ry < 2 + band && yb + ry < g.ny;   // stored (interior) row
        sbr[r] = rst[r] && y >= sb.y0 && y < sb.y0 + sb.bny;
        sbrow[r] = (int64_t)(y - sb.y0) * sb.bnx;
    }
    bool cin[CX], sbc[CX];
#pragma unroll
    for (int j = 0; j < CX; ++j) {
        const int x = j * 64 + lane;
        cin[j] = x < g.nx;
        sbc[j] = cin[j] && x >= sb.x0 && x < sb.x0 + sb.bnx;
    }
    const bool perx = g.per[0] != 0;
    const int lastj = (g.nx - 1) / 64, lastl = (g.nx - 1) % 64;
    const bool T_PSI = g.pml > 0 && psrc != nullptr;
    const int ms = d.meas_slot;

    int z0, z1;
    f3_chunk(g, zr, fb, &z0, &z1);
    if (z0 >= z1) return;                          // whole block: before any barrier
    const int kb = max(z0 - 2, 0);                 // first level-1 plane
    const int p0 = z0 > 0 ? z0 - 1 : 0;            // first level-2 plane
    bool vc[B][CX];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int j = 0; j < CX; ++j) vc[r][j] = rin[r] && cin[j];
    auto raw3 = [&](int k, int comp0, T (&a)[B][CX], T (&b)[B][CX], T (&c)[B][CX]) {
        const int64_t pk = (int64_t)min(max(k, 0), g.nz - 1) * sz;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const int64_t at = comp0 * n + (vc[r][j] ? pk + rowoff[r] + j * 64 + lane : 0);
                a[r][j] = S[at];
                b[r][j] = S[n + at];
                c[r][j] = S[2 * n + at];
            }
    };
    auto raw_ids = [&](int k, uint2 (&id)[B][CX]) {
        const int64_t pk = (int64_t)min(max(k, 0), g.nz - 1) * sz;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j)
                id[r][j] = g.idp[vc[r][j] ? pk + rowoff[r] + j * 64 + lane : 0];
    };
    auto mask3 = [&](bool kin, T (&a)[B][CX], T (&b)[B][CX], T (&c)[B][CX]) {
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const bool v = kin && vc[r][j];
                a[r][j] = v ? a[r][j] : T(0);
                b[r][j] = v ? b[r][j] : T(0);
                c[r][j] = v ? c[r][j] : T(0);
            }
    };
    constexpr uint32_t kNull4 = 0x01010101u * kNullId, kNull2 = 0x0101u * kNullId;

    // H half on one plane: H <- a H - b curl E from E of the plane, Ex, Ey of
    // the next plane (En*) and the x+1 / y+1 neighbours; in a layer plane the
    // z differences carry psi (P0 for Hx, P1 for Hy), advanced in place.
    auto h_half = [&](bool active, const T (&Ex)[B][CX], const T (&Ey)[B][CX], const T (&Ez)[B][CX],
                      const T (&Enx)[B][CX], const T (&Eny)[B][CX], T (&Hx)[B][CX], T (&Hy)[B][CX],
                      T (&Hz)[B][CX], const uint32_t (&I0)[B][CX], const uint32_t (&I1)[B][CX], T (&P0)[B][CX],
                      T (&P1)[B][CX], bool zp, T bh, T chh) {
#pragma unroll
        for (int j = 0; j < CX; ++j) {
            xe[w][0][j][lane] = Ez[0][j];
            xe[w][1][j][lane] = Ex[0][j];
        }
        __syncthreads();
        if (!active) return;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            T nez[CX], ney[CX];
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const T a = yee::from_next(Ez[r][j]), b = yee::from_next(Ey[r][j]);
                const T a1 = j + 1 < CX ? yee::lane_value(Ez[r][(j + 1) % CX], 0) : T(0);
                const T b1 = j + 1 < CX ? yee::lane_value(Ey[r][(j + 1) % CX], 0) : T(0);
                nez[j] = lane == 63 ? a1 : a;
                ney[j] = lane == 63 ? b1 : b;
            }
            const T fez = yee::lane_value(Ez[r][0], 0), fey = yee::lane_value(Ey[r][0], 0);
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                T ez_y, ex_y;
                if (r + 1 < B) {
                    ez_y = Ez[(r + 1) % B][j];
                    ex_y = Ex[(r + 1) % B][j];
                } else if (w + 1 < W) {
                    ez_y = xe[(w + 1) % W][0][j][lane];
                    ex_y = xe[(w + 1) % W][1][j][lane];
                } else {
                    ez_y = T(0);   // last region row: halo, never stored
                    ex_y = T(0);
                }
                T ez_x = nez[j];
                T ey_x = ney[j];
                if (j * 64 + lane == g.nx - 1) {
                    ez_x = perx ? fez : T(0);
                    ey_x = perx ? fey : T(0);
                }
                T dzEy = Eny[r][j] - Ey[r][j];
                T dzEx = Enx[r][j] - Ex[r][j];
                if (zp && vc[r][j]) {
                    const T q0 = fma(bh, P0[r][j], chh * dzEy);
                    const T q1 = fma(bh, P1[r][j], chh * dzEx);
                    P0[r][j] = q0;
                    P1[r][j] = q1;
                    dzEy = dzEy + q0;
                    dzEx = dzEx + q1;
                }
                const T curl_x = (ez_y - Ez[r][j]) - dzEy;
                const T curl_y = dzEx - (ez_x - Ez[r][j]);
                const T curl_z = (ey_x - Ey[r][j]) - (ex_y - Ex[r][j]);
                const yee::Pair<T> cx = L[CF_HX][I0[r][j] >> 24];
                const yee::Pair<T> cy = L[CF_HY][I1[r][j] & 255u];
                const yee::Pair<T> cz = L[CF_HZ][(I1[r][j] >> 8) & 255u];
                const bool v = vc[r][j];
                Hx[r][j] = v ? yee_sub(cx.a, Hx[r][j], cx.b, curl_x) : T(0);
                Hy[r][j] = v ? yee_sub(cy.a, Hy[r][j], cy.b, curl_y) : T(0);
                Hz[r][j] = v ? yee_sub(cz.a, Hz[r][j], cz.b, curl_z) : T(0);
            }
        }
    };
    // E half on one plane: E <- a E + b curl H from H of the plane, Hx, Hy of
    // the previous plane (Hp*) and the x-1 / y-1 neighbours; psi P2 (Ex), P3
    // (Ey) in a layer plane.
    auto e_half = [&](bool active, T (&Ex)[B][CX], T (&Ey)[B][CX], T (&Ez)[B][CX], const T (&Hx)[B][CX],
                      const T (&Hy)[B][CX], const T (&Hz)[B][CX], const T (&Hpx)[B][CX], const T (&Hpy)[B][CX],
                      const uint32_t (&I0)[B][CX], T (&P2)[B][CX], T (&P3)[B][CX], bool zp, T be, T ce) {
#pragma unroll
        for (int j = 0; j < CX; ++j) {
            xh[w][0][j][lane] = Hz[B - 1][j];
            xh[w][1][j][lane] = Hx[B - 1][j];
        }
        __syncthreads();
        if (!active) return;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            T phz[CX], phy[CX];
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                const T a = yee::from_prev(Hz[r][j]), b = yee::from_prev(Hy[r][j]);
                const T a1 = j > 0 ? yee::lane_value(Hz[r][(j + CX - 1) % CX], 63) : T(0);
                const T b1 = j > 0 ? yee::lane_value(Hy[r][(j + CX - 1) % CX], 63) : T(0);
                phz[j] = lane == 0 ? a1 : a;
                phy[j] = lane == 0 ? b1 : b;
            }
            T lhz = Hz[r][0], lhy = Hy[r][0];
#pragma unroll
            for (int j = 1; j < CX; ++j)
                if (lastj == j) {
                    lhz = Hz[r][j];
                    lhy = Hy[r][j];
                }
            lhz = yee::lane_value(lhz, lastl);
            lhy = yee::lane_value(lhy, lastl);
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                T hz_y, hx_y;
                if (r > 0) {
                    hz_y = Hz[(r + B - 1) % B][j];
                    hx_y = Hx[(r + B - 1) % B][j];
                } else if (w > 0) {
                    hz_y = xh[(w + W - 1) % W][0][j][lane];
                    hx_y = xh[(w + W - 1) % W][1][j][lane];
                } else {
                    hz_y = T(0);   // region row 0: halo, never stored
                    hx_y = T(0);
                }
                T hz_x = phz[j];
                T hy_x = phy[j];
                if (j * 64 + lane == 0) {
                    hz_x = perx ? lhz : T(0);
                    hy_x = perx ? lhy : T(0);
                }
                T dzHy = Hy[r][j] - Hpy[r][j];
                T dzHx = Hx[r][j] - Hpx[r][j];
                if (zp && vc[r][j]) {
                    const T q2 = fma(be, P2[r][j], ce * dzHy);
                    const T q3 = fma(be, P3[r][j], ce * dzHx);
                    P2[r][j] = q2;
                    P3[r][j] = q3;
                    dzHy = dzHy + q2;
                    dzHx = dzHx + q3;
                }
                const T curl_x = (Hz[r][j] - hz_y) - dzHy;
                const T curl_y = dzHx - (Hz[r][j] - hz_x);
                const T curl_z = (Hy[r][j] - hy_x) - (Hx[r][j] - hx_y);
                const yee::Pair<T> cx = L[CF_EX][I0[r][j] & 255u];
                const yee::Pair<T> cy = L[CF_EY][(I0[r][j] >> 8) & 255u];
                const yee::Pair<T> cz = L[CF_EZ][(I0[r][j] >> 16) & 255u];
                Ex[r][j] = yee_add(cx.a, Ex[r][j], cx.b, curl_x);
                Ey[r][j] = yee_add(cy.a, Ey[r][j], cy.b, curl_y);
                Ez[r][j] = yee_add(cz.a, Ez[r][j], cz.b, curl_z);
            }
        }
    };

    T ex[B][CX], ey[B][CX], ez[B][CX];       // level 1: E(k), step n, then n + 1
    T ex1[B][CX], ey1[B][CX], ez1[B][CX];    // E(k+1), step n
    T hx[B][CX], hy[B][CX], hz[B][CX];       // H(k), step n, then n + 1
    uint32_t id0[B][CX], id1[B][CX];         // material ids of plane k (Ex Ey Ez Hx | Hy Hz)
    T fx[B][CX], fy[B][CX], fz[B][CX];       // level 2: E(k-1), step n + 1, then n + 2
    T gx[B][CX], gy[B][CX], gz[B][CX];       // H(k-1), step n + 1, then n + 2
    T qx[B][CX], qy[B][CX];                  // Hx, Hy of plane k-2 at step n + 2
    uint32_t jd0[B][CX], jd1[B][CX];         // material ids of plane k-1
    T pc[4][B][CX];                          // psi of plane k-1 after step n + 1 (layer planes)
    {
        uint2 i2[B][CX];
        raw3(kb, 0, ex, ey, ez);
        raw3(kb + 1, 0, ex1, ey1, ez1);
        raw3(kb, 3, hx, hy, hz);
        raw_ids(kb, i2);
        mask3(true, ex, ey, ez);
        mask3(kb + 1 < g.nz, ex1, ey1, ez1);
        mask3(true, hx, hy, hz);
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                id0[r][j] = vc[r][j] ? i2[r][j].x : kNull4;
                id1[r][j] = vc[r][j] ? i2[r][j].y : kNull2;
                fx[r][j] = fy[r][j] = fz[r][j] = T(0);
                gx[r][j] = gy[r][j] = gz[r][j] = T(0);
                qx[r][j] = qy[r][j] = T(0);
                jd0[r][j] = kNull4;
                jd1[r][j] = kNull2;
#pragma unroll
                for (int q = 0; q < 4; ++q) pc[q][r][j] = T(0);
            }
    }
    __syncthreads();   // coefficient tables

    for (int k = kb; k <= z1; ++k) {
        const int p = k - 1;
        const bool l1 = k < g.nz;                  // uniform over the block
        const bool l2 = p >= p0;
        const bool l2e = p >= z0;                  // level-2 E half and the stores
        const int plane1 = l1 ? pml_plane(k, g.nz, g.pml) : -1;
        const int plane2 = l2 ? pml_plane(p, g.nz, g.pml) : -1;
        const bool zp1 = T_PSI && plane1 >= 0, zp2 = T_PSI && plane2 >= 0;
        const T bh1 = zp1 ? Lz[0][plane1] : T(1), ch1 = zp1 ? Lz[1][plane1] : T(0);
        const T be1 = zp1 ? Lz[2][plane1] : T(1), ce1 = zp1 ? Lz[3][plane1] : T(0);
        const T bh2 = zp2 ? Lz[0][plane2] : T(1), ch2 = zp2 ? Lz[1][plane2] : T(0);
        const T be2 = zp2 ? Lz[2][plane2] : T(1), ce2 = zp2 ? Lz[3][plane2] : T(0);
        // psi of plane k at step n (layer planes), loaded before the prefetch
        T ps[4][B][CX];
        if (zp1) {
            const int64_t pp = (int64_t)plane1 * sz;
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    const int64_t pa = d.psi_off + (vc[r][j] ? pp + rowoff[r] + j * 64 + lane : 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) ps[q][r][j] = psrc[pa + q * g.psi_comp];
                }
        }
        // next plane's inputs, issued before this plane's arithmetic
        T ex2[B][CX], ey2[B][CX], ez2[B][CX];
        T hxn[B][CX], hyn[B][CX], hzn[B][CX];
        uint2 idn[B][CX];
        raw3(k + 2, 0, ex2, ey2, ez2);
        raw3(k + 1, 3, hxn, hyn, hzn);
        raw_ids(k + 1, idn);

        // ---- level 1 on plane k (step n -> n + 1) ----
        h_half(l1, ex, ey, ez, ex1, ey1, hx, hy, hz, id0, id1, ps[0], ps[1], zp1, bh1, ch1);
        e_half(l1, ex, ey, ez, hx, hy, hz, gx, gy, id0, ps[2], ps[3], zp1, be1, ce1);
        if (!l1) {
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) ex[r][j] = ey[r][j] = ez[r][j] = T(0);   // beyond the top wall
        }
        if (l1 && k >= z0 && k < z1 && k >= sb.z0 && k < sb.z0 + sb.bnz) {
            const int64_t zo = (int64_t)(k - sb.z0) * sb.bny * sb.bnx - sb.x0;
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j)
                    if (sbr[r] && sbc[j]) {
                        const T v = ms == 0 ? ex[r][j]
                                  : ms == 1 ? ey[r][j]
                                  : ms == 2 ? ez[r][j]
                                  : ms == 3 ? hx[r][j]
                                  : ms == 4 ? hy[r][j] : hz[r][j];
                        SH[zo + sbrow[r] + j * 64 + lane] = v;
                    }
        }

        // ---- level 2 on plane k - 1 (step n + 1 -> n + 2) ----
        h_half(l2, fx, fy, fz, ex, ey, gx, gy, gz, jd0, jd1, pc[0], pc[1], zp2, bh2, ch2);
        e_half(l2e, fx, fy, fz, gx, gy, gz, qx, qy, jd0, pc[2], pc[3], zp2, be2, ce2);
        if (l2e) {
            const int64_t pk = (int64_t)p * sz;
            const int64_t pp = (int64_t)plane2 * sz;
#pragma unroll
            for (int r = 0; r < B; ++r)
#pragma unroll
                for (int j = 0; j < CX; ++j) {
                    if (!rst[r] || !cin[j]) continue;
                    const int64_t at = pk + rowoff[r] + j * 64 + lane;
                    D[at] = fx[r][j];
                    D[n + at] = fy[r][j];
                    D[2 * n + at] = fz[r][j];
                    D[3 * n + at] = gx[r][j];
                    D[4 * n + at] = gy[r][j];
                    D[5 * n + at] = gz[r][j];
                    if (zp2) {
                        const int64_t pa = d.psi_off + pp + rowoff[r] + j * 64 + lane;
#pragma unroll
                        for (int q = 0; q < 4; ++q) pdst[pa + q * g.psi_comp] = pc[q][r][j];
                    }
                }
        }

        // ---- rotate ----
        mask3(k + 2 < g.nz, ex2, ey2, ez2);
        mask3(k + 1 < g.nz, hxn, hyn, hzn);
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int j = 0; j < CX; ++j) {
                qx[r][j] = gx[r][j];
                qy[r][j] = gy[r][j];
                fx[r][j] = ex[r][j];
                fy[r][j] = ey[r][j];
                fz[r][j] = ez[r][j];
                gx[r][j] = hx[r][j];
                gy[r][j] = hy[r][j];
                gz[r][j] = hz[r][j];
                jd0[r][j] = id0[r][j];
                jd1[r][j] = id1[r][j];
#pragma unroll
                for (int q = 0; q < 4; ++q) pc[q][r][j] = ps[q][r][j];
                ex[r][j] = ex1[r][j];
                ey[r][j] = ey1[r][j];
                ez[r][j] = ez1[r][j];
                ex1[r][j] = ex2[r][j];
                ey1[r][j] = ey2[r][j];
                ez1[r][j] = ez2[r][j];
                hx[r][j] = hxn[r][j];
                hy[r][j] = hyn[r][j];
                hz[r][j] = hzn[r][j];
                const bool v = vc[r][j] && k + 1 < g.nz;
                id0[r][j] = v ? idn[r][j].x : kNull4;
                id1[r][j] = v ? idn[r][j].y : kNull2;
            }
    }
}

// Surface projection of step m from the shadow box of a two-step launch.
template <typename T>
__global__ __launch_bounds__(yee::kSurfThreads) void k_surface_box(
    const T* __restrict__ shadow, ShadowBox sb, int nx, int ny, int64_t block_elems,
    const ChanDev* __restrict__ ch, const int* __restrict__ slots, SurfTables t, const double* __restrict__ ktab,
    int m, double dt, double dA, double* __restrict__ acc, double* __restrict__ gamma, int gamma_stride) {
    __shared__ double red[yee::kSurfThreads / 64];
    const int slot = slots[blockIdx.x];
    const ChanDev d = ch[slot];
    const T* X = shadow + (d.field_off / block_elems) * sb.vol;
    const double s = yee::block_surface_sum(
        d, t,
        [&](int32_t idx) {
            const int x = idx % nx, y = (idx / nx) % ny, z = idx / (nx * ny);
            return (double)X[((int64_t)(z - sb.z0) * sb.bny + (y - sb.y0)) * sb.bnx + (x - sb.x0)];
        },
        red);
    if (threadIdx.x == 0) {
        const double G = dA * s;
        double sum = acc[2 * slot], comp = acc[2 * slot + 1];
        yee::neumaier(sum, comp, (dt * ktab[m]) * G);
        acc[2 * slot] = sum;
        acc[2 * slot + 1] = comp;
        if (gamma) gamma[(int64_t)m * gamma_stride + slot] = G;
    }
}

// Fused 3D variants: W waves of B rows, `steps` time steps per launch
// (band = W B - 2 steps stored rows).  Indices are part of the ABI
// (tile_variant); the single-step variants come first.
struct F3Variant {
    int W, B, steps;
};
constexpr F3Variant kF3[] = {{8, 2, 1}, {16, 1, 1}, {8, 1, 1}, {12, 1, 1}, {8, 1, 2}, {12, 1, 2}};
constexpr int kNumF3 = sizeof(kF3) / sizeof(kF3[0]);

template <typename T, int W, int CX>
constexpr bool f3_fits() {
    return f3_lds_bytes<T>(W, CX) <= kF3LdsMax;
}

// LDS a block may take on the current device
inline size_t f3_device_lds() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return (size_t)v;
}

// A dynamic LDS size above 64 KB needs the kernel's attribute raised first
// (once per kernel instantiation).
template <typename K>
bool f3_lds_attr(K kernel, size_t bytes) {
    if (bytes <= 65536) return true;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes) == hipSuccess;
}

template <typename T, int W, int B, int CX, int STEPS>
hipError_t f3_launch(const ChanDev* ch, const int* slots, int nslots, const Grid3D& g, const T* lut, const T* src,
                     T* dst, const T* psrc, T* pdst, T* shadow, const ShadowBox& sb, const int2* zr,
                     hipStream_t s) {
    if constexpr (!f3_fits<T, W, CX>()) {
        return hipErrorInvalidValue;
    } else {
        const int band = W * B - 2 * STEPS;
        const int bands = (g.ny + band - 1) / band;
        // z chunks: enough blocks to fill the chip several times over, each
        // chunk at least 24 planes deep (one extra H plane per chunk)
        const long xy = (long)bands * nslots;
        int nzc = (int)std::min<long>((4096 + xy - 1) / xy, std::max(1, g.nz / 24));
        nzc = std::max(1, std::min(nzc, 65535));
        dim3 grid(bands, nslots, nzc), block(64 * W, 1, 1);
        constexpr size_t lds = f3_lds_bytes<T>(W, CX);
        if constexpr (STEPS == 1) {
            static const bool attr = f3_lds_attr(&k_f3d<T, W, B, CX>, lds);
            if (!attr) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_f3d<T, W, B, CX>), grid, block, lds, s, ch, slots, g, lut, src, dst, psrc, pdst,
                               band, zr);
        } else {
            if (shadow == nullptr || sb.vol <= 0) return hipErrorInvalidValue;
            static const bool attr = f3_lds_attr(&k_f3d2<T, W, B, CX>, lds);
            if (!attr) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_f3d2<T, W, B, CX>), grid, block, lds, s, ch, slots, g, lut, src, dst, psrc, pdst,
                               shadow, sb, band, zr);
        }
        return hipGetLastError();
    }
}

template <typename T, int W, int B, int STEPS>
hipError_t f3_dispatch_cx(int cx, const ChanDev* ch, const int* slots, int nslots, const Grid3D& g, const T* lut,
                          const T* src, T* dst, const T* psrc, T* pdst, T* sh, const ShadowBox& sb, const int2* zr,
                          hipStream_t s) {
    switch (cx) {
        case 1: return f3_launch<T, W, B, 1, STEPS>(ch, slots, nslots, g, lut, src, dst, psrc, pdst, sh, sb, zr, s);
        case 2: return f3_launch<T, W, B, 2, STEPS>(ch, slots, nslots, g, lut, src, dst, psrc, pdst, sh, sb, zr, s);
        case 3: return f3_launch<T, W, B, 3, STEPS>(ch, slots, nslots, g, lut, src, dst, psrc, pdst, sh, sb, zr, s);
        case 4: return f3_launch<T, W, B, 4, STEPS>(ch, slots, nslots, g, lut, src, dst, psrc, pdst, sh, sb, zr, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
bool f3_variant_fits(int v, int cx) {
    const size_t bytes = f3_lds_bytes<T>(kF3[v].W, cx);
    return bytes <= kF3LdsMax && bytes <= f3_device_lds();
}
}  // namespace

template <typename T>
hipError_t launch_h3d(int mode, T* fields, T* psi, const ChanDev* ch, const int* slots, int nslots,
                      const Grid3D& g, const T* lut, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    const int tiles = ((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY) * g.nz;
    dim3 grid(tiles, nslots, 1), block(BX, BY, 1);
    if (mode == 0) hipLaunchKernelGGL((k_h3d<T, 0>), grid, block, 0, s, fields, psi, ch, slots, g, lut);
    else hipLaunchKernelGGL((k_h3d<T, 1>), grid, block, 0, s, fields, psi, ch, slots, g, lut);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_e3d(int mode, T* fields, T* psi, const ChanDev* ch, const int* slots, int nslots,
                      const Grid3D& g, const T* lut, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    const int tiles = ((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY) * g.nz;
    dim3 grid(tiles, nslots, 1), block(BX, BY, 1);
    if (mode == 0) hipLaunchKernelGGL((k_e3d<T, 0>), grid, block, 0, s, fields, psi, ch, slots, g, lut);
    else hipLaunchKernelGGL((k_e3d<T, 1>), grid, block, 0, s, fields, psi, ch, slots, g, lut);
    return hipGetLastError();
}


template <typename T>
bool f3d_usable(int variant, const Grid3D& g) {
    if (variant < 0 || variant >= kNumF3) return false;
    if (g.nx < 1 || g.nx > 256 || g.per[2] || g.pml > kF3MaxPml) return false;
    const int cx = (g.nx + 63) / 64;
    return f3_variant_fits<T>(variant, cx) && g.ny >= 1;
}

int f3d_variants() { return kNumF3; }

int f3d_steps(int variant) { return variant >= 0 && variant < kNumF3 ? kF3[variant].steps : 0; }

int f3d_single(int variant) {
    if (variant < 0 || variant >= kNumF3) return -1;
    for (int v = 0; v < kNumF3; ++v)
        if (kF3[v].steps == 1 && kF3[v].W == kF3[variant].W && kF3[v].B == kF3[variant].B) return v;
    return -1;
}

template <typename T>
hipError_t launch_f3d(int variant, const ChanDev* ch, const int* slots, int nslots, const Grid3D& g, const T* lut,
                      const T* src, T* dst, const T* psrc, T* pdst, T* sh, const ShadowBox& sb, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    if (!f3d_usable<T>(variant, g)) return hipErrorInvalidValue;
    const int cx = (g.nx + 63) / 64;
    const int2* zr = g.zr_tab ? g.zr_tab + g.zr_off[variant] : nullptr;
#define CF_F3(W, B, S) f3_dispatch_cx<T, W, B, S>(cx, ch, slots, nslots, g, lut, src, dst, psrc, pdst, sh, sb, zr, s)
    switch (variant) {
        case 0: return CF_F3(8, 2, 1);
        case 1: return CF_F3(16, 1, 1);
        case 2: return CF_F3(8, 1, 1);
        case 3: return CF_F3(12, 1, 1);
        case 4: return CF_F3(8, 1, 2);
        default: return CF_F3(12, 1, 2);
    }
#undef CF_F3
}

void f3d_shape(int variant, int* w, int* b, int* steps) {
    const bool ok = variant >= 0 && variant < kNumF3;
    *w = ok ? kF3[variant].W : 0;
    *b = ok ? kF3[variant].B : 0;
    *steps = ok ? kF3[variant].steps : 0;
}

template <typename T>
hipError_t launch_surface_box(const T* shadow, const ShadowBox& sb, const Grid3D& g, const ChanDev* ch,
                              const int* slots, int nslots, const SurfTables& t, const double* ktab, int m,
                              double dt, double dA, double* acc, double* gamma, int gamma_stride, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_surface_box<T>), dim3(nslots), dim3(yee::kSurfThreads), 0, s, shadow, sb, g.nx, g.ny,
                       (int64_t)6 * g.ncell, ch, slots, t, ktab, m, dt, dA, acc, gamma, gamma_stride);
    return hipGetLastError();
}

#define CF_INSTANTIATE(T)                                                                                    \
    template hipError_t launch_h3d<T>(int, T*, T*, const ChanDev*, const int*, int, const Grid3D&, const T*, \
                                      hipStream_t);                                                          \
    template hipError_t launch_e3d<T>(int, T*, T*, const ChanDev*, const int*, int, const Grid3D&, const T*, \
                                      hipStream_t);                                                          \
    template bool f3d_usable<T>(int, const Grid3D&);                                                         \
    template hipError_t launch_f3d<T>(int, const ChanDev*, const int*, int, const Grid3D&, const T*, const T*, \
                                      T*, const T*, T*, T*, const ShadowBox&, hipStream_t);               \
    template hipError_t launch_surface_box<T>(const T*, const ShadowBox&, const Grid3D&, const ChanDev*,     \
                                              const int*, int, const SurfTables&, const double*, int, double, \
                                              double, double*, double*, int, hipStream_t);
CF_INSTANTIATE(float)
CF_INSTANTIATE(double)
#undef CF_INSTANTIATE

}  // namespace cf
