// Device helpers shared by the 2D, 3D and cylindrical kernels: the update
// forms with explicit fused multiply-adds (the library is built without
// automatic contraction, so every path that uses these evaluates bitwise the
// same arithmetic), coefficient-table addressing, cross-lane moves, and the
// surface projection with its compensated time accumulation.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace cf {
namespace yee {

// x <- a x - b d  and  x <- a x + b d
template <typename T>
__device__ __forceinline__ T sub(T a, T x, T b, T d) { return fma(a, x, -(b * d)); }
template <typename T>
__device__ __forceinline__ T add(T a, T x, T b, T d) { return fma(a, x, b * d); }
// The same two updates computed into x's own register: the final fused
// multiply-add is written as the three-source form with x as both a source
// and the destination, so a field updated under a branch (the fused kernel
// skips waves that hold only conductor) needs no copy back into its home
// register.  Bitwise the same as sub / add.
__device__ __forceinline__ void fma_into(float& x, float a, float t) {
    asm("v_fma_f32 %0, %1, %0, %2" : "+v"(x) : "v"(a), "v"(t));
}
__device__ __forceinline__ void fma_into(double& x, double a, double t) {
    asm("v_fma_f64 %0, %1, %0, %2" : "+v"(x) : "v"(a), "v"(t));
}
template <typename T>
__device__ __forceinline__ void sub_into(T& x, T a, T b, T d) { fma_into(x, a, -(b * d)); }
template <typename T>
__device__ __forceinline__ void add_into(T& x, T a, T b, T d) { fma_into(x, a, b * d); }
// partner field of the consistent start: (b / 2) d
template <typename T>
__device__ __forceinline__ T half(T b, T d) { return (T(0.5) * b) * d; }

// (a, b) of component comp, material id, channel kind in the coefficient table
template <typename T>
__device__ __forceinline__ const T* lut_ab(const T* lut, int kind, int comp, int id) {
    return lut + (((kind * 6 + comp) << 8) + id) * 2;
}

// A device pointer that reaches a kernel inside a struct read from memory is
// a generic pointer to the compiler, which then addresses it with FLAT
// instructions: those also count on the LDS/scalar counter, so every wait
// for an LDS exchange waits for them too, and each needs a 64-bit address
// in vector registers.  Every buffer the library hands its kernels is global
// device memory; the global view of such a pointer gets global instructions
// (an SGPR base with a 32-bit lane offset where the base is uniform).
template <typename T>
using gmem = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gmem<T> as_global(T* p) {
    return (gmem<T>)p;
}

template <typename T>
struct Pair {
    T a, b;
};

// Value of v held by lane l+1 (DPP wave_shl:1) / lane l-1 (wave_shr:1).  The
// lane with no neighbour (63 / 0) reads 0 (bound_ctrl).
__device__ __forceinline__ float from_next(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_prev(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_next(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_prev(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true),
                            __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true));
}

// Value of v in lane l (l uniform across the wave), broadcast to every lane.
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Undivided difference D along in-plane axis `axis` for the component in
// field slot `slot` at cell (i, j) of a 2D grid, stretched inside the CPML
// layers (Roden-Gedney with kappa = 1, alpha = 0): psi <- b psi + c D,
// returns D + psi.  Outside the layers b = 1 and c = 0, so psi stays 0 and
// the difference is returned as it is.  half: the updated component sits at
// a half-cell position along the axis.  psi: the channel's CPML block
// (part already applied), or nullptr.
template <typename T>
__device__ __forceinline__ T pml_d2(T D, const Grid2D& g, T* psi, int slot, int axis, bool half, int i, int j) {
    const int P = g.pml[axis];
    if (P == 0 || psi == nullptr) return D;
    const int n = axis == 0 ? g.nx : g.ny;
    const int q = axis == 0 ? i : j;
    if (q >= P && q < n - P) return D;
    const int qq = q < P ? q : q - (n - 2 * P);
    T* arr = psi + slot * g.psi_slot + (axis == 0 ? 0 : (int64_t)g.ny * 2 * g.pml[0]);
    const int64_t at = axis == 0 ? (int64_t)j * (2 * P) + qq : (int64_t)qq * g.nx + i;
    const double* tab = g.pml_tab[axis] + (half ? 0 : 2 * n);
    const T p = fma(T(tab[q]), arr[at], T(tab[n + q]) * D);
    arr[at] = p;
    return D + p;
}

// Dispersive media: advances the Lorentz polarizations of one E component at
// cell c (every term's pair P^m, P^{m-1} -> P^{m+1}, P^m, from E^m = e_old)
// and returns (sum P^{m+1} - a sum P^m) / eps_inf, the amount the E update
// of D = eps_inf E + sum P subtracts.  Zero for an id without terms.  aux:
// the channel's polarization block (part already applied); e_slot: the E
// component's slot in it.
template <typename T>
__device__ __forceinline__ T lorentz_step(const Grid2D& g, T* aux, int e_slot, int64_t c, int id, T a, T e_old) {
    const double* row = g.lor + (size_t)id * kLorStride(g.n_lor);
    if (row[0] == 0.0) return T(0);
    T sum_now = T(0), sum_next = T(0);
    for (int j = 0; j < g.n_lor; ++j) {
        T* pc = aux + (int64_t)((e_slot * g.n_lor + j) * 2) * g.ncell + c;
        T* pp = pc + g.ncell;
        const T cur = *pc, prev = *pp;
        const T nxt = fma(T(row[2 + 3 * j]), cur, fma(-T(row[3 + 3 * j]), prev, T(row[4 + 3 * j]) * e_old));
        sum_now += cur;
        sum_next += nxt;
        *pp = cur;
        *pc = nxt;
    }
    return (sum_next - a * sum_now) * T(row[1]);
}

// Threads that take part in a surface sum (the first kSurfThreads of the block).
constexpr int kSurfThreads = 256;

// Neumaier-compensated (sum, comp) += term.
__device__ __forceinline__ void neumaier(double& sum, double& comp, double term) {
    const double nt = sum + term;
    if (fabs(sum) >= fabs(term))
        comp += (sum - nt) + term;
    else
        comp += (term - nt) + sum;
    sum = nt;
}

// Fixed-order sum of s over a wave; lane 0 of each of the first
// kSurfThreads / 64 waves stores its wave's sum in red[wave].
__device__ __forceinline__ void wave_partial_store(double s, double* red) {
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0 && threadIdx.x < kSurfThreads) red[threadIdx.x >> 6] = s;
}

// Gamma sum of one channel by the first kSurfThreads threads of a block:
// thread t takes samples t, t + kSurfThreads, ...; sum_p w X in FP64 per
// sample, weighted by the basis row; then a fixed-order reduction over the
// wave and over the kSurfThreads / 64 waves.  Every thread of the block must
// call it (it holds a barrier); the total is returned in thread 0.
// `fetch(idx)` reads the measured component at flat grid index idx.
// First part of the sum, without a barrier: the per-wave partial sums of the
// first kSurfThreads threads land in red[0 .. kSurfThreads / 64 - 1].
template <typename Fetch>
__device__ __forceinline__ void wave_surface_partials(const ChanDev& d, const SurfTables& t, Fetch fetch,
                                                      double* red) {
    double s = 0.0;
    const int n = threadIdx.x < kSurfThreads ? d.nsamp : 0;
    for (int i = threadIdx.x; i < n; i += kSurfThreads) {
        const auto gi = as_global(t.gidx) + d.g_off + (int64_t)i * d.P;
        const auto gw = as_global(t.gw) + d.g_off + (int64_t)i * d.P;
        double v = 0.0;
        for (int p = 0; p < d.P; ++p) v += gw[p] * fetch(gi[p]);
        s += as_global(t.basis)[d.basis_off + i] * v;
    }
    wave_partial_store(s, red);
}

// The same partial sums from a launch-resident copy of the channel's tables:
// off[i P + p] is where fetch finds point p of sample i, w the weights in
// the table's order and b the basis row, so the result is bitwise that of
// wave_surface_partials.
template <typename Fetch>
__device__ __forceinline__ void wave_surface_partials_staged(int nsamp, int P, const uint16_t* off,
                                                             const double* w, const double* b, Fetch fetch,
                                                             double* red) {
    double s = 0.0;
    const int n = threadIdx.x < kSurfThreads ? nsamp : 0;
    for (int i = threadIdx.x; i < n; i += kSurfThreads) {
        double v = 0.0;
        for (int p = 0; p < P; ++p) v += w[i * P + p] * fetch(off[i * P + p]);
        s += b[i] * v;
    }
    wave_partial_store(s, red);
}

// The fixed-order total of the wave partials (after a barrier that follows
// wave_surface_partials).
__device__ __forceinline__ double wave_partials_total(const double* red) {
    return ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename Fetch>
__device__ __forceinline__ double block_surface_sum(const ChanDev& d, const SurfTables& t, Fetch fetch,
                                                    double* red) {
    wave_surface_partials(d, t, fetch, red);
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0) tot = wave_partials_total(red);
    return tot;
}

}  // namespace yee
}  // namespace cf
