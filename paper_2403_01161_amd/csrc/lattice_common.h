// D3Q19 velocity set and population storage formats, shared by the forward
// lattice kernels and the adjoint kernels.
#pragma once

#include <stdint.h>

#include <type_traits>

#include "device_common.h"

namespace ibmlb {

// f(integral_constant<int, k>) for k = B .. E-1, unrolled at compile time.
template <int B, int E, class Fn>
__device__ __forceinline__ void static_for(Fn&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// ---------------------------------------------------------------- D3Q19
// Index 0 is the rest population; 2p-1 and 2p (p = 1..9) are opposite.
constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
template <class R>
__host__ __device__ constexpr R wgt(int i) {
    return i == 0 ? R(1) / R(3) : (i <= 6 ? R(1) / R(18) : R(1) / R(36));
}

// ---------------------------------------------------------------- storage
struct SF64 { using store_t = double; using real = double; };
struct SF32 { using store_t = float; using real = float; };
struct SF16 { using store_t = _Float16; using real = float; };
struct SBF16 { using store_t = uint16_t; using real = float; };

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }
// Round to nearest even with the conversion instruction of gfx950
// (v_cvt_pk_bf16_f32); NaN stays NaN.
__device__ inline uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <class C> __device__ inline typename C::real dec(typename C::store_t v, float inv);
template <> __device__ inline double dec<SF64>(double v, float) { return v; }
template <> __device__ inline float dec<SF32>(float v, float) { return v; }
template <> __device__ inline float dec<SF16>(_Float16 v, float inv) { return float(v) * inv; }
template <> __device__ inline float dec<SBF16>(uint16_t v, float) { return bf16_to_f32(v); }

template <class C> __device__ inline typename C::store_t enc(typename C::real v, float sc);
template <> __device__ inline double enc<SF64>(double v, float) { return v; }
template <> __device__ inline float enc<SF32>(float v, float) { return v; }
template <> __device__ inline _Float16 enc<SF16>(float v, float sc) { return _Float16(v * sc); }
template <> __device__ inline uint16_t enc<SBF16>(float v, float) { return f32_to_bf16(v); }

}  // namespace ibmlb
