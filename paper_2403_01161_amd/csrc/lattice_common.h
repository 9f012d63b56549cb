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

// ---------------------------------------------------------------- MRT basis
// The orthogonal D3Q19 moment basis of d'Humieres et al. (2002), with
// c2 = |c|^2: rho; e = 19 c2 - 30; eps = (21 c2^2 - 53 c2 + 24)/2; j_a = c_a;
// q_a = (5 c2 - 9) c_a; 3p_xx = 3 c_x^2 - c2; 3pi_xx = (3 c_x^2 - c2)(3 c2 - 5);
// p_ww = c_y^2 - c_z^2; pi_ww = (c_y^2 - c_z^2)(3 c2 - 5); p_xy, p_yz, p_xz;
// m_x = (c_y^2 - c_z^2) c_x, m_y = (c_z^2 - c_x^2) c_y, m_z = (c_x^2 - c_y^2) c_z,
// in the order rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww,
// pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z. Entry (k, i) is moment k of velocity i.
__host__ __device__ constexpr int mrt_m(int k, int i) {
    const int cx = CX[i], cy = CY[i], cz = CZ[i];
    const int c2 = cx * cx + cy * cy + cz * cz;
    switch (k) {
        case 0: return 1;
        case 1: return 19 * c2 - 30;
        case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
        case 3: return cx;
        case 4: return (5 * c2 - 9) * cx;
        case 5: return cy;
        case 6: return (5 * c2 - 9) * cy;
        case 7: return cz;
        case 8: return (5 * c2 - 9) * cz;
        case 9: return 3 * cx * cx - c2;
        case 10: return (3 * cx * cx - c2) * (3 * c2 - 5);
        case 11: return cy * cy - cz * cz;
        case 12: return (cy * cy - cz * cz) * (3 * c2 - 5);
        case 13: return cx * cy;
        case 14: return cy * cz;
        case 15: return cx * cz;
        case 16: return (cy * cy - cz * cz) * cx;
        case 17: return (cz * cz - cx * cx) * cy;
        default: return (cx * cx - cy * cy) * cz;
    }
}
// Squared norm of basis row k (the basis is orthogonal: M^-1 = M^T diag(1/norm)).
__host__ __device__ constexpr int mrt_norm2(int k) {
    int s = 0;
    for (int i = 0; i < Q; ++i) s += mrt_m(k, i) * mrt_m(k, i);
    return s;
}

// Weighted moments of the basis rows, in units of 1/36 (36 w_i = 12, 2, 1):
// sum_i m_ki 36 w_i, sum_i m_ki 36 w_i c_ia and sum_i m_ki 36 w_i c_ia c_ib.
// Moment k of any field w_i (a + b.c_i + c_i^T C c_i) follows from them.
__host__ __device__ constexpr int w36(int i) { return i == 0 ? 12 : (i <= 6 ? 2 : 1); }
__host__ __device__ constexpr int cc(int i, int a) { return a == 0 ? CX[i] : (a == 1 ? CY[i] : CZ[i]); }
__host__ __device__ constexpr int mrt_w0(int k) {
    int s = 0;
    for (int i = 0; i < Q; ++i) s += mrt_m(k, i) * w36(i);
    return s;
}
__host__ __device__ constexpr int mrt_w1(int k, int a) {
    int s = 0;
    for (int i = 0; i < Q; ++i) s += mrt_m(k, i) * w36(i) * cc(i, a);
    return s;
}
__host__ __device__ constexpr int mrt_w2(int k, int a, int b) {
    int s = 0;
    for (int i = 0; i < Q; ++i) s += mrt_m(k, i) * w36(i) * cc(i, a) * cc(i, b);
    return s;
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
