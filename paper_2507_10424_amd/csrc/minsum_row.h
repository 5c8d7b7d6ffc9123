// Check-row primitives shared by the on-chip and streaming decoders: the
// three-input XOR, the XOR of a row's words, the two smallest magnitudes of
// a row (Observation 1 of Sec. III), and the message of one edge from them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ldpc {

// Three-input XOR in one VALU instruction (v_bitop3_b32 with truth table
// 0x96 = a ^ b ^ c), which the compiler does not form from XOR chains.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// XOR of N words with ceil((N - 1) / 2) instructions: three-input XORs, and
// one two-input XOR when N is even.
template <int N> __device__ __forceinline__ uint32_t xor_all(const uint32_t *v) {
    if constexpr (N == 1) {
        return v[0];
    } else if constexpr (N == 2) {
        return v[0] ^ v[1];
    } else {
        uint32_t acc = xor3(v[0], v[1], v[2]);
#pragma unroll
        for (int k = 3; k + 1 < N; k += 2) acc = xor3(acc, v[k], v[k + 1]);
        if constexpr (N % 2 == 0) acc ^= v[N - 1];
        return acc;
    }
}

// Smallest and second smallest of N non-negative floats (min0 <= min1, equal
// on a tie): groups of three give (min3, med3); a group joins the running pair
// as min0 = min(m, gm), min1 = min3(max(m, gm), s, gs); single leftover values
// join as min0 = min(m, v), min1 = med3(m, v, s).  Inputs are never NaN or
// signalling, so the float min/max instructions are exact selections.
template <int N> __device__ __forceinline__ void min_pair(const float *a, float &m, float &s) {
    static_assert(N >= 1, "empty row");
    if constexpr (N == 1) {
        m = a[0];
        s = __builtin_inff();
    } else if constexpr (N == 2) {
        m = fminf(a[0], a[1]);
        s = fmaxf(a[0], a[1]);
    } else {
        m = fminf(fminf(a[0], a[1]), a[2]);
        s = __builtin_amdgcn_fmed3f(a[0], a[1], a[2]);
        int k = 3;
#pragma unroll
        for (; k + 3 <= N; k += 3) {
            const float gm = fminf(fminf(a[k], a[k + 1]), a[k + 2]);
            const float gs = __builtin_amdgcn_fmed3f(a[k], a[k + 1], a[k + 2]);
            s = fminf(fminf(fmaxf(m, gm), s), gs);
            m = fminf(m, gm);
        }
#pragma unroll
        for (; k < N; ++k) {
            s = __builtin_amdgcn_fmed3f(m, a[k], s);
            m = fminf(m, a[k]);
        }
    }
}

// The plain Min-Sum message of an edge from its row's two smallest
// magnitudes min0 <= min1 and K = bits(min0) + bits(min1) + (sign bit of the
// row's parity), as 32-bit integers.  Clamping x to [-min1, min1] gives
// sign(x) min(|x|, min1): magnitude min0 at the row's minimum and min1 at
// every other edge (all other |x| are >= min1).  Non-negative floats order
// like their bit patterns and a sign bit is 2^31 modulo 2^32, so K - clamp is
// the other magnitude (min1 at the minimum, min0 elsewhere) with the sign
// parity XOR sign(x): the message of Observations 1 and 2, in two
// instructions.  x must not be -0 (its sign bit is read as its sign); when
// min1 = 0 only the sign of a zero message can differ from the definition.
__device__ __forceinline__ float edge_message(float x, float min1, uint32_t K) {
    return __uint_as_float(K - __float_as_uint(__builtin_amdgcn_fmed3f(x, -min1, min1)));
}
__device__ __forceinline__ uint32_t row_word(float min0, float min1, uint32_t parity) {
    return __float_as_uint(min0) + __float_as_uint(min1) + (parity & 0x80000000u);
}

} // namespace ldpc
