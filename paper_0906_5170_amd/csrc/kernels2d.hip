// 2D Yee kernels for gfx950: TM (Ez, Hx, Hy) and TE (Ex, Ey, Hz) half-step
// updates with the uniform conductivity sigma carried by the per-kind
// coefficient tables, the delta(t) kick, and the surface projection with
// the FP64 compensated g-weighted time accumulation.
//
// Layout: a channel's field block is 3 components x (ny x nx) cells, x
// fastest.  A 64 x 4 thread block covers 64 consecutive x cells of 4 rows,
// so every wavefront reads and writes 64 contiguous elements per component
// (coalesced 256 B / 512 B for FP32 / FP64).  Channels run along grid.y.
//
// Update forms (undivided differences; a, b from the channel kind's table):
//   TM  Hx <- a Hx - b (Ez[j+1] - Ez[j])        Hy <- a Hy - b (Ez[i] - Ez[i+1])
//       Ez <- a Ez + b ((Hy[i] - Hy[i-1]) - (Hx[j] - Hx[j-1]))
//   TE  Hz <- a Hz - b ((Ey[i+1] - Ey[i]) - (Ex[j+1] - Ex[j]))
//       Ex <- a Ex + b (Hz[j] - Hz[j-1])         Ey <- a Ey - b (Hz[i] - Hz[i-1])
// A neighbour beyond the grid reads as 0 on a PEC wall and wraps on a
// periodic one.  The consistent start writes the partner field of the
// kicked one as +b/2 times the same curl.
#include "../../include/casimir_fdtd.h"
#include "device.hpp"

namespace cf {

namespace {

constexpr int BX = 64;
constexpr int BY = 4;

template <typename T>
__device__ __forceinline__ const T* lut_ab(const T* lut, int kind, int comp, int id) {
    return lut + (((kind * 6 + comp) << 8) + id) * 2;
}

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
        if (MODE == 0) {
            Hx[c] = lx[0] * Hx[c] - lx[1] * (ezu - ez);
            Hy[c] = ly[0] * Hy[c] - ly[1] * (ez - ezr);
        } else {
            Hx[c] = T(0.5) * lx[1] * (ezu - ez);
            Hy[c] = T(0.5) * ly[1] * (ez - ezr);
        }
    } else {
        const T* Ex = base;
        const T* Ey = base + g.ncell;
        T* Hz = base + 2 * g.ncell;
        const T ex = Ex[c], ey = Ey[c];
        const T eyr = in_r ? Ey[c + 1] : (g.perx ? Ey[c + 1 - g.nx] : T(0));
        const T exu = in_u ? Ex[c + g.nx] : (g.pery ? Ex[i] : T(0));
        const T curl = (eyr - ey) - (exu - ex);
        const T* lz = lut_ab(lut, d.kind, CF_HZ, g.ids[CF_HZ][c]);
        if (MODE == 0) {
            Hz[c] = lz[0] * Hz[c] - lz[1] * curl;
        } else {
            Hz[c] = T(0.5) * lz[1] * curl;
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
        const T curl = (hy - hyl) - (hx - hxd);
        const T* lz = lut_ab(lut, d.kind, CF_EZ, g.ids[CF_EZ][c]);
        if (MODE == 0) {
            Ez[c] = lz[0] * Ez[c] + lz[1] * curl;
        } else {
            Ez[c] = T(0.5) * lz[1] * curl;
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
        if (MODE == 0) {
            Ex[c] = lx[0] * Ex[c] + lx[1] * (hz - hzd);
            Ey[c] = ly[0] * Ey[c] - ly[1] * (hz - hzl);
        } else {
            Ex[c] = T(0.5) * lx[1] * (hz - hzd);
            Ey[c] = T(-0.5) * ly[1] * (hz - hzl);
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

// One wavefront per channel: Gamma = dA sum_s f_n(s) sum_p w_sp X[idx_sp] in
// FP64, reduced across the wave in a fixed order, then the Neumaier update of
// (sum, comp) += dt K(t_m) Gamma.
template <typename T>
__global__ __launch_bounds__(64) void k_surface(const T* __restrict__ fields, const ChanDev* __restrict__ ch,
                                                const int* __restrict__ slots, SurfTables t,
                                                const double* __restrict__ ktab, int m, double dt,
                                                double dA, double* __restrict__ acc,
                                                double* __restrict__ gamma, int gamma_stride) {
    const int slot = slots[blockIdx.x];
    const ChanDev d = ch[slot];
    const T* X = fields + d.meas_off;
    double s = 0.0;
    for (int i = threadIdx.x; i < d.nsamp; i += 64) {
        const int32_t* gi = t.gidx + d.g_off + (int64_t)i * d.P;
        const double* gw = t.gw + d.g_off + (int64_t)i * d.P;
        double v = 0.0;
        for (int p = 0; p < d.P; ++p) v += gw[p] * (double)X[gi[p]];
        s += t.basis[d.basis_off + i] * v;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (threadIdx.x == 0) {
        const double G = dA * s;
        const double term = dt * ktab[m] * G;
        double sum = acc[2 * slot], comp = acc[2 * slot + 1];
        const double nt = sum + term;
        if (fabs(sum) >= fabs(term))
            comp += (sum - nt) + term;
        else
            comp += (term - nt) + sum;
        acc[2 * slot] = nt;
        acc[2 * slot + 1] = comp;
        if (gamma) gamma[(int64_t)m * gamma_stride + slot] = G;
    }
}

inline dim3 grid2d(const Grid2D& g, int nslots) {
    const int tiles = ((g.nx + BX - 1) / BX) * ((g.ny + BY - 1) / BY);
    return dim3(tiles, nslots, 1);
}

}  // namespace

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
    hipLaunchKernelGGL((k_surface<T>), dim3(nslots), dim3(64), 0, s, fields, ch, slots, t, ktab, m,
                       dt, dA, acc, gamma, gamma_stride);
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
                                          hipStream_t);
CF_INSTANTIATE(float)
CF_INSTANTIATE(double)
#undef CF_INSTANTIATE

}  // namespace cf
