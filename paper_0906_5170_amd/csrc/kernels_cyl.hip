// Yee update in cylindrical coordinates for one azimuthal order m (Sec.
// III D; Appendix, harmonic expansion in cylindrical coordinates), on the
// (r, z) half plane of a cylindrically symmetric problem.
//
// Fields proportional to exp(i m phi), with E_phi, H_r, H_z carried as
// -i times their value, obey the real system
//   mu  dh_r/dt   = -[ (m/r) e_z - d_z e_phi ]
//   mu  dh_phi/dt = -[ d_z e_r - d_r e_z ]
//   mu  dh_z/dt   = -[ (1/r) d_r (r e_phi) - (m/r) e_r ]
//   eps de_r/dt   =    -(m/r) h_z - d_z h_phi
//   eps de_phi/dt =    d_z h_r - d_r h_z
//   eps de_z/dt   =    (1/r) d_r (r h_phi) + (m/r) h_r
// The axial coordinate is the grid's x (index i), the radius its y (index j):
// slots Ex = e_z, Ey = e_r, Ez = e_phi, Hx = h_z, Hy = h_r, Hz = h_phi, each
// an (nr x nz) array, z fastest.  Ey, Hx, Hz sit at r = j cells, Ex, Ez, Hy
// at r = j - 1/2 (their row 0 lies outside and stays 0).  The tube wall is
// at r = nr - 1/2: a neighbour beyond it reads 0.  Along z a neighbour beyond
// the grid reads 0 (PEC ends) or wraps (periodic).
//
// Axis (row 0 of Ey, Hx, Hz): h_z there follows the circulation of e_phi
// around the disk of radius 1/2 cell, (4 / dx) e_phi(r = 1/2), for m = 0
// and is 0 otherwise; e_r and h_phi enter no update there and are kept at
// 0 (the surface interpolation applies their axis value, the next row's
// for m = 1).
//
// Coefficients (a, b) come from the Cartesian per-kind tables built for
// this order's Courant number: x <- a x -/+ b curl, with the curls above in
// undivided form (times dx).
//
// Two drivers share the per-cell updates (so their fields agree bitwise):
// split half-step launches (one launch per half step for a batch of
// channels of one order), and the resident solve, where one block carries
// one channel through clear, kick, start and all its steps with the surface
// projection, in a single launch for channels of any mix of orders (a
// channel's block of 6 x nr x nz values stays in the L2 of its XCD).
#include "../../include/casimir_fdtd.h"
#include "device.hpp"
#include "yee_common.hpp"

namespace cf {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int kResThreads = 1024;

using yee::lut_ab;

inline dim3 grid_cyl(const Grid2D& g, int nslots) {
    const int tiles = ((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY);
    return dim3(tiles, nslots, 1);
}

// H update of cell (i, j) of the channel block F: MODE 0 h <- a h - b curl e,
// MODE 1 the consistent start h^{-1/2} = (b / 2) curl e^0.
template <typename T, int MODE>
__device__ __forceinline__ void hcyl_cell(T* __restrict__ F, const Grid2D& g, const T* __restrict__ lut, int kind,
                                          int m, int i, int j) {
    const T* Ex = F;
    const T* Ey = F + g.ncell;
    const T* Ez = F + 2 * g.ncell;
    T* Hx = F + 3 * g.ncell;
    T* Hy = F + 4 * g.ncell;
    T* Hz = F + 5 * g.ncell;
    const int64_t c = (int64_t)j * g.nx + i;
    const bool in_r = i + 1 < g.nx, in_u = j + 1 < g.ny;
    const T ezu = in_u ? Ez[c + g.nx] : T(0);
    const T* lx = lut_ab(lut, kind, CF_HX, g.ids[CF_HX][c]);
    if (j == 0) {
        // axis: h_z from the disk circulation (m = 0), h_r outside, h_phi 0
        const T cz = T(4) * ezu;
        if (MODE == 0) Hx[c] = m == 0 ? yee::sub(lx[0], Hx[c], lx[1], cz) : T(0);
        else Hx[c] = m == 0 ? yee::half(lx[1], cz) : T(0);
        Hy[c] = T(0);
        Hz[c] = T(0);
        return;
    }
    const T ex = Ex[c], ey = Ey[c], ez = Ez[c];
    const T exu = in_u ? Ex[c + g.nx] : T(0);
    const T ezr = in_r ? Ez[c + 1] : (g.perx ? Ez[c + 1 - g.nx] : T(0));
    const T eyr = in_r ? Ey[c + 1] : (g.perx ? Ey[c + 1 - g.nx] : T(0));
    const T M = T(m);
    const T r1 = T(j);                 // radius of h_z (cells)
    const T r0 = T(j) - T(0.5);        // radius of h_r
    // h_z: (1/r) d_r (r e_phi) - (m/r) e_r
    const T cz = (((r1 + T(0.5)) * ezu - r0 * ez) - M * ey) / r1;
    // h_r: (m/r) e_z - d_z e_phi
    const T cr = (M * ex) / r0 - (ezr - ez);
    // h_phi: d_z e_r - d_r e_z
    const T cp = (eyr - ey) - (exu - ex);
    const T* ly = lut_ab(lut, kind, CF_HY, g.ids[CF_HY][c]);
    const T* lz = lut_ab(lut, kind, CF_HZ, g.ids[CF_HZ][c]);
    if (MODE == 0) {
        Hx[c] = yee::sub(lx[0], Hx[c], lx[1], cz);
        Hy[c] = yee::sub(ly[0], Hy[c], ly[1], cr);
        Hz[c] = yee::sub(lz[0], Hz[c], lz[1], cp);
    } else {
        Hx[c] = yee::half(lx[1], cz);
        Hy[c] = yee::half(ly[1], cr);
        Hz[c] = yee::half(lz[1], cp);
    }
}

// E update of cell (i, j): MODE 0 e <- a e + b curl h, MODE 1 the
// consistent start e^{+1/2} = (b / 2) curl h^0.
template <typename T, int MODE>
__device__ __forceinline__ void ecyl_cell(T* __restrict__ F, const Grid2D& g, const T* __restrict__ lut, int kind,
                                          int m, int i, int j) {
    T* Ex = F;
    T* Ey = F + g.ncell;
    T* Ez = F + 2 * g.ncell;
    const T* Hx = F + 3 * g.ncell;
    const T* Hy = F + 4 * g.ncell;
    const T* Hz = F + 5 * g.ncell;
    const int64_t c = (int64_t)j * g.nx + i;
    if (j == 0) {
        // e_z, e_phi outside / on the wall id, e_r on the axis: all 0
        Ex[c] = T(0);
        Ey[c] = T(0);
        Ez[c] = T(0);
        return;
    }
    const T hx = Hx[c], hy = Hy[c], hz = Hz[c];
    const T hxd = Hx[c - g.nx], hzd = Hz[c - g.nx];
    const T hyl = i > 0 ? Hy[c - 1] : (g.perx ? Hy[c - 1 + g.nx] : T(0));
    const T hzl = i > 0 ? Hz[c - 1] : (g.perx ? Hz[c - 1 + g.nx] : T(0));
    const T M = T(m);
    const T r1 = T(j);                 // radius of e_r
    const T r0 = T(j) - T(0.5);        // radius of e_z
    // e_z: (1/r) d_r (r h_phi) + (m/r) h_r
    const T cz = ((r1 * hz - (r1 - T(1)) * hzd) + M * hy) / r0;
    // e_r: -(m/r) h_z - d_z h_phi
    const T cr = -((M * hx) / r1) - (hz - hzl);
    // e_phi: d_z h_r - d_r h_z
    const T cp = (hy - hyl) - (hx - hxd);
    const T* lx = lut_ab(lut, kind, CF_EX, g.ids[CF_EX][c]);
    const T* ly = lut_ab(lut, kind, CF_EY, g.ids[CF_EY][c]);
    const T* lz = lut_ab(lut, kind, CF_EZ, g.ids[CF_EZ][c]);
    if (MODE == 0) {
        Ex[c] = yee::add(lx[0], Ex[c], lx[1], cz);
        Ey[c] = yee::add(ly[0], Ey[c], ly[1], cr);
        Ez[c] = yee::add(lz[0], Ez[c], lz[1], cp);
    } else {
        Ex[c] = yee::half(lx[1], cz);
        Ey[c] = yee::half(ly[1], cr);
        Ez[c] = yee::half(lz[1], cp);
    }
}

template <typename T, int MODE>
__global__ __launch_bounds__(BX* BY) void k_hcyl(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                               const int* __restrict__ slots, Grid2D g,
                                               const T* __restrict__ lut, int m) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 0) return;   // start: E-kind runs set H^{-1/2}
    const int tiles_x = (g.nx + BX - 1) / BX;
    const int i = (blockIdx.x % tiles_x) * BX + threadIdx.x;
    const int j = (blockIdx.x / tiles_x) * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    hcyl_cell<T, MODE>(fields + d.field_off, g, lut, d.kind, m, i, j);
}

template <typename T, int MODE>
__global__ __launch_bounds__(BX* BY) void k_ecyl(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                               const int* __restrict__ slots, Grid2D g,
                                               const T* __restrict__ lut, int m) {
    const ChanDev d = ch[slots[blockIdx.y]];
    if (MODE == 1 && d.kind != 1) return;   // start: H-kind runs set E^{+1/2}
    const int tiles_x = (g.nx + BX - 1) / BX;
    const int i = (blockIdx.x % tiles_x) * BX + threadIdx.x;
    const int j = (blockIdx.x / tiles_x) * BY + threadIdx.y;
    if (i >= g.nx || j >= g.ny) return;
    ecyl_cell<T, MODE>(fields + d.field_off, g, lut, d.kind, m, i, j);
}

// Every cell of the grid once, block-strided: thread t takes flat cells
// t, t + kResThreads, ... (consecutive threads on consecutive z).
template <typename Body>
__device__ __forceinline__ void for_cells(const Grid2D& g, Body body) {
    const int di = kResThreads % g.nx, dj = kResThreads / g.nx;
    int i = threadIdx.x % g.nx, j = threadIdx.x / g.nx;
    while (j < g.ny) {
        body(i, j);
        i += di;
        j += dj;
        if (i >= g.nx) {
            i -= g.nx;
            ++j;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kResThreads) void k_cyl_resident(T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                                              const int* __restrict__ slots, Grid2D g, CylOrders ord,
                                                              SurfTables t, double dA, double* __restrict__ acc,
                                                              double* __restrict__ gamma, int gamma_stride) {
    __shared__ double red[yee::kSurfThreads / 64];
    const int slot = slots[blockIdx.x];
    const ChanDev d = ch[slot];
    const int m = d.order;
    const T* lut = static_cast<const T*>(ord.lut) + m * ord.lut_stride;
    const double* ktab = ord.ktab + m * ord.ktab_stride;
    const int nsteps = ord.steps[m];
    const double dt = ord.dt[m];
    T* F = fields + d.field_off;
    const int64_t nval = 6 * g.ncell;
    for (int64_t k = threadIdx.x; k < nval; k += kResThreads) F[k] = T(0);
    __syncthreads();
    // kick: the source component's surface deposit (one writer per point)
    for (int u = threadIdx.x; u < d.n_uniq; u += kResThreads) {
        const int k0 = t.uoff[d.u_off + u], k1 = t.uoff[d.u_off + u + 1];
        double s = 0.0;
        for (int k = k0; k < k1; ++k) s += t.uw[k] * t.basis[d.basis_off + t.usamp[k]];
        fields[d.src_off + t.uidx[d.u_off + u]] = T(d.kick_scale * s);
    }
    __syncthreads();
    if (d.kind == 0) for_cells(g, [&](int i, int j) { hcyl_cell<T, 1>(F, g, lut, d.kind, m, i, j); });
    else for_cells(g, [&](int i, int j) { ecyl_cell<T, 1>(F, g, lut, d.kind, m, i, j); });
    __syncthreads();
    const T* X = fields + d.meas_off;
    double sum = 0.0, comp = 0.0;
    if (threadIdx.x == 0) {
        sum = acc[2 * slot];
        comp = acc[2 * slot + 1];
    }
    for (int step = 0; step < nsteps; ++step) {
        for_cells(g, [&](int i, int j) { hcyl_cell<T, 0>(F, g, lut, d.kind, m, i, j); });
        __syncthreads();
        for_cells(g, [&](int i, int j) { ecyl_cell<T, 0>(F, g, lut, d.kind, m, i, j); });
        __syncthreads();
        // every read of X ends at the barrier inside; the next writes of the
        // fields come after it
        const double s = yee::block_surface_sum(d, t, [&](int32_t idx) { return (double)X[idx]; }, red);
        if (threadIdx.x == 0) {
            const double G = dA * s;
            yee::neumaier(sum, comp, (dt * ktab[step]) * G);
            if (gamma) gamma[(int64_t)step * gamma_stride + slot] = G;
        }
    }
    if (threadIdx.x == 0) {
        acc[2 * slot] = sum;
        acc[2 * slot + 1] = comp;
    }
}

}  // namespace

template <typename T>
hipError_t launch_hcyl(int mode, int m, T* fields, const ChanDev* ch, const int* slots, int nslots,
                       const Grid2D& g, const T* lut, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    const dim3 grid = grid_cyl(g, nslots), block(BX, BY, 1);
    if (mode == 0) hipLaunchKernelGGL((k_hcyl<T, 0>), grid, block, 0, s, fields, ch, slots, g, lut, m);
    else hipLaunchKernelGGL((k_hcyl<T, 1>), grid, block, 0, s, fields, ch, slots, g, lut, m);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ecyl(int mode, int m, T* fields, const ChanDev* ch, const int* slots, int nslots,
                       const Grid2D& g, const T* lut, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    const dim3 grid = grid_cyl(g, nslots), block(BX, BY, 1);
    if (mode == 0) hipLaunchKernelGGL((k_ecyl<T, 0>), grid, block, 0, s, fields, ch, slots, g, lut, m);
    else hipLaunchKernelGGL((k_ecyl<T, 1>), grid, block, 0, s, fields, ch, slots, g, lut, m);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cyl_resident(T* fields, const ChanDev* ch, const int* slots, int nslots, const Grid2D& g,
                               const CylOrders& ord, const SurfTables& t, double dA, double* acc, double* gamma,
                               int gamma_stride, hipStream_t s) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_cyl_resident<T>), dim3(nslots), dim3(kResThreads), 0, s, fields, ch, slots, g, ord, t, dA,
                       acc, gamma, gamma_stride);
    return hipGetLastError();
}

#define CF_CYL_INSTANTIATE(T)                                                                                   \
    template hipError_t launch_hcyl<T>(int, int, T*, const ChanDev*, const int*, int, const Grid2D&, const T*, \
                                       hipStream_t);                                                           \
    template hipError_t launch_ecyl<T>(int, int, T*, const ChanDev*, const int*, int, const Grid2D&, const T*, \
                                       hipStream_t);                                                           \
    template hipError_t launch_cyl_resident<T>(T*, const ChanDev*, const int*, int, const Grid2D&,            \
                                               const CylOrders&, const SurfTables&, double, double*, double*, \
                                               int, hipStream_t);
CF_CYL_INSTANTIATE(float)
CF_CYL_INSTANTIATE(double)
#undef CF_CYL_INSTANTIATE

}  // namespace cf
