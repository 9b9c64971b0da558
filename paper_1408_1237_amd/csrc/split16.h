// Split-f16 slot vectors of the FP32 / BF16 matrix-core product (kmvp.hip).
//
// Every FP32 operand v is split as v = hi + lo, hi = f16(v), lo = f16(v - hi).
// v - hi is exact in FP32 and |v - hi| <= 2^-11 |v|; rounding it to f16 (11-bit
// significand, subnormals kept) leaves |v - hi - lo| <= 2^-22 |v| (plus half an
// f16 subnormal step, 2^-25, when v - hi is below the f16 normal range): four
// times the FP32 rounding of v itself.
// An inner product a_i . b_j + c_i + e_j over D coordinates is then one over
// 3 D + 4 slots: coordinate k takes slots 3k .. 3k + 2 with (hi, hi, lo) of the
// source value and (hi, lo, hi) of the target value; slots 3D, 3D + 1 hold
// (1, 1) against the target constant (c_hi, c_lo), slots 3D + 2, 3D + 3 the
// source constant (e_hi, e_lo) against (1, 1); the rest are 0.  The Gaussian
// exponent uses no source constant (e = 0), the Matern squared distance both.
// The slots are grouped in chunks of 16 for one v_mfma_f32_32x32x16_f16, each
// chunk as two octets (slots 8w .. 8w + 7, w = 2 kc + half).
#pragma once

#include <hip/hip_runtime.h>

namespace krr {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef unsigned uintx4_t __attribute__((ext_vector_type(4)));

// 16-slot chunks of dimension D (compiled dimensions up to 48), 0 above.
constexpr int split_chunks(int D) { return D <= 48 ? (3 * D + 4 + 15) / 16 : 0; }

struct HiLo {
    _Float16 hi, lo;
};
__device__ __forceinline__ HiLo split_f16(float v) {
    const _Float16 hi = static_cast<_Float16>(v);
    return HiLo{hi, static_cast<_Float16>(v - static_cast<float>(hi))};
}
__device__ __forceinline__ unsigned f16_bits(_Float16 v) { return __builtin_bit_cast(unsigned short, v); }

// Slot s (a compile-time constant after unrolling) of a source (SOURCE) or
// target vector given the per-coordinate splits v and the two constant pairs:
// c for slots 3D, 3D + 1 and c2 for slots 3D + 2, 3D + 3 (on the source side
// c = (1, 1) and c2 = e; on the target side c = the target constant, c2 = (1, 1)
// or (0, 0)).
template <int D, bool SOURCE>
__device__ __forceinline__ _Float16 slot_value(int s, const HiLo (&v)[D], HiLo c, HiLo c2) {
    if (s < 3 * D) {
        const HiLo p = v[s / 3];
        const int kind = s % 3;
        if (SOURCE) return kind == 2 ? p.lo : p.hi;
        return kind == 1 ? p.lo : p.hi;
    }
    if (s == 3 * D) return c.hi;
    if (s == 3 * D + 1) return c.lo;
    if (s == 3 * D + 2) return c2.hi;
    if (s == 3 * D + 3) return c2.lo;
    return static_cast<_Float16>(0.f);
}

// Octet w (slots 8 w .. 8 w + 7) as one 16-byte vector.
template <int D, bool SOURCE>
__device__ __forceinline__ half8_t slot_octet(int w, const HiLo (&v)[D], HiLo c, HiLo c2) {
    uintx4_t u;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        u[e] = f16_bits(slot_value<D, SOURCE>(8 * w + 2 * e, v, c, c2)) |
               (f16_bits(slot_value<D, SOURCE>(8 * w + 2 * e + 1, v, c, c2)) << 16);
    return __builtin_bit_cast(half8_t, u);
}

constexpr float LOG2E_F = 1.44269504088896341f;
constexpr float LN2_F = 0.693147180559945309f;

}  // namespace krr
