// Split-f16 slot vectors of the FP32 / BF16 matrix-core product (kmvp.hip).
//
// Every FP32 operand v is split as v = hi + lo, hi = f16(v), lo = f16(v - hi):
// |v - hi - lo| <= 2^-24 |v| (v - hi is exact in FP32; f16 subnormals are kept).
// The folded exponent of a pair, sum_k 2 t_ik o_jk + c_i, is then an inner
// product over 3 D + 2 slots: coordinate k takes slots 3k .. 3k + 2 with
// (hi, hi, lo) of o_jk on the source side and (hi, lo, hi) of 2 t_ik on the
// target side; slots 3D and 3D + 1 hold (1, 1) and (c_hi, c_lo); the rest are 0.
// The slots are grouped in chunks of 16 for one v_mfma_f32_32x32x16_f16, each
// chunk as two octets (slots 8w .. 8w + 7, w = 2 kc + half).
#pragma once

#include <hip/hip_runtime.h>

namespace krr {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef unsigned uintx4_t __attribute__((ext_vector_type(4)));

// 16-slot chunks of dimension D (compiled dimensions up to 16), 0 above.
constexpr int split_chunks(int D) { return D <= 16 ? (3 * D + 2 + 15) / 16 : 0; }

struct HiLo {
    _Float16 hi, lo;
};
__device__ __forceinline__ HiLo split_f16(float v) {
    const _Float16 hi = static_cast<_Float16>(v);
    return HiLo{hi, static_cast<_Float16>(v - static_cast<float>(hi))};
}
__device__ __forceinline__ unsigned f16_bits(_Float16 v) { return __builtin_bit_cast(unsigned short, v); }

// Slot s (a compile-time constant after unrolling) of a source (SOURCE) or
// target vector given the per-coordinate splits v and the constant pair c.
template <int D, bool SOURCE>
__device__ __forceinline__ _Float16 slot_value(int s, const HiLo (&v)[D], HiLo c) {
    if (s < 3 * D) {
        const HiLo p = v[s / 3];
        const int kind = s % 3;
        if (SOURCE) return kind == 2 ? p.lo : p.hi;
        return kind == 1 ? p.lo : p.hi;
    }
    if (s == 3 * D) return c.hi;
    if (s == 3 * D + 1) return c.lo;
    return static_cast<_Float16>(0.f);
}

// Octet w (slots 8 w .. 8 w + 7) as one 16-byte vector.
template <int D, bool SOURCE>
__device__ __forceinline__ half8_t slot_octet(int w, const HiLo (&v)[D], HiLo c) {
    uintx4_t u;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        u[e] = f16_bits(slot_value<D, SOURCE>(8 * w + 2 * e, v, c)) |
               (f16_bits(slot_value<D, SOURCE>(8 * w + 2 * e + 1, v, c)) << 16);
    return __builtin_bit_cast(half8_t, u);
}

}  // namespace krr
