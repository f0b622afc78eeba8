// Device helpers shared by the 2D and 3D kernels: the update forms with
// explicit fused multiply-adds (the library is built without automatic
// contraction, so every path that uses these evaluates bitwise the same
// arithmetic), coefficient-table addressing, and cross-lane moves.
#pragma once

#include <hip/hip_runtime.h>

namespace cf {
namespace yee {

// x <- a x - b d  and  x <- a x + b d
template <typename T>
__device__ __forceinline__ T sub(T a, T x, T b, T d) { return fma(a, x, -(b * d)); }
template <typename T>
__device__ __forceinline__ T add(T a, T x, T b, T d) { return fma(a, x, b * d); }
// partner field of the consistent start: (b / 2) d
template <typename T>
__device__ __forceinline__ T half(T b, T d) { return (T(0.5) * b) * d; }

// (a, b) of component comp, material id, channel kind in the coefficient table
template <typename T>
__device__ __forceinline__ const T* lut_ab(const T* lut, int kind, int comp, int id) {
    return lut + (((kind * 6 + comp) << 8) + id) * 2;
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

}  // namespace yee
}  // namespace cf
