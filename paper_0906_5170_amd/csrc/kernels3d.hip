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
#include "../../include/casimir_fdtd.h"
#include "device.hpp"

namespace cf {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

template <typename T>
__device__ __forceinline__ T yee_sub(T a, T x, T b, T d) { return fma(a, x, -(b * d)); }
template <typename T>
__device__ __forceinline__ T yee_add(T a, T x, T b, T d) { return fma(a, x, b * d); }
template <typename T>
__device__ __forceinline__ T yee_half(T b, T d) { return (T(0.5) * b) * d; }

template <typename T>
__device__ __forceinline__ const T* lut_ab(const T* lut, int kind, int comp, int id) {
    return lut + (((kind * 6 + comp) << 8) + id) * 2;
}

// psi plane of z index k inside the layers, or -1 outside
__device__ __forceinline__ int pml_plane(int k, int nz, int P) {
    if (P <= 0) return -1;
    if (k < P) return k;
    if (k >= nz - P) return P + (k - (nz - P));
    return -1;
}

// z difference with the CPML update: psi <- b psi + c D, returns D + psi.
// In start mode (mode 1) psi is not advanced: the layers hold zero fields.
template <typename T, int MODE>
__device__ __forceinline__ T zdiff(T D, T* psi, int64_t at, T b, T c) {
    if (MODE == 1 || psi == nullptr) return D;
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

#define CF_INSTANTIATE(T)                                                                                    \
    template hipError_t launch_h3d<T>(int, T*, T*, const ChanDev*, const int*, int, const Grid3D&, const T*, \
                                      hipStream_t);                                                          \
    template hipError_t launch_e3d<T>(int, T*, T*, const ChanDev*, const int*, int, const Grid3D&, const T*, \
                                      hipStream_t);
CF_INSTANTIATE(float)
CF_INSTANTIATE(double)
#undef CF_INSTANTIATE

}  // namespace cf
