// ext_bits.h -- device helpers of the bit-sliced kernels (ext_bitslice.hip,
// ext_bsk.hip): the fused AND-XOR and the in-register 32x32 bit transpose
// that turns 32 block pairs' words into bit planes and back.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qext {

__device__ __forceinline__ uint32_t bs_and_xor(uint32_t a, uint32_t b, uint32_t acc) {
    return __builtin_amdgcn_bitop3_b32(a, b, acc, 0x6A);  // (a & b) ^ acc
}

// One block-swap step of the 32x32 transpose: for rows r with bit J clear,
// the columns of row r with bit J set are exchanged with the columns of row
// r + J with bit J clear (M selects the columns with bit J clear).  Steps of
// 16 and 8 move whole bytes (one v_perm_b32 per row); the others take a
// shift and a bit select (v_bitop3_b32 0xD8: (a & ~m) | (b & m)) per row.
__device__ __forceinline__ uint32_t bs_select(uint32_t a, uint32_t b, uint32_t m) {
    return __builtin_amdgcn_bitop3_b32(a, b, m, 0xD8);
}

template <int J, uint32_t M>
__device__ __forceinline__ void transpose_step(uint32_t (&a)[32]) {
#pragma unroll
    for (int r = 0; r < 32; ++r) {
        if (r & J) continue;
        const uint32_t lo = a[r], hi = a[r + J];
        if constexpr (J == 16) {
            a[r] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);      // lo.b0 lo.b1 hi.b0 hi.b1
            a[r + J] = __builtin_amdgcn_perm(hi, lo, 0x07060302u);  // lo.b2 lo.b3 hi.b2 hi.b3
        } else if constexpr (J == 8) {
            a[r] = __builtin_amdgcn_perm(hi, lo, 0x06020400u);      // lo.b0 hi.b0 lo.b2 hi.b2
            a[r + J] = __builtin_amdgcn_perm(hi, lo, 0x07030501u);  // lo.b1 hi.b1 lo.b3 hi.b3
        } else {
            a[r] = bs_select(lo, hi << J, M << J);
            a[r + J] = bs_select(hi, lo >> J, M);
        }
    }
}

// In place: on entry bit c of a[r] is element (r, c); on exit bit r of a[c]
// is element (r, c).
__device__ __forceinline__ void transpose32(uint32_t (&a)[32]) {
    transpose_step<16, 0x0000FFFFu>(a);
    transpose_step<8, 0x00FF00FFu>(a);
    transpose_step<4, 0x0F0F0F0Fu>(a);
    transpose_step<2, 0x33333333u>(a);
    transpose_step<1, 0x55555555u>(a);
}

}  // namespace qext
