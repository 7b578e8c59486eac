// Shared pieces of the warm-start MLP kernels (mlp.hip, mlp_fused.hip):
// bfloat16 rounding, MFMA operand types, the packed parameter layout and
// the shape checks.
#pragma once

#include "common.h"

namespace dvq {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round to the nearest bfloat16, ties to even.
__device__ __forceinline__ __bf16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __builtin_bit_cast(__bf16, (unsigned short)(u >> 16));
}

// Packed float32 parameters: W1[h][d_in], b1[h], W2[h][h], b2[h],
// W3[d_out][h], b3[d_out] (row-major).
struct MlpOffsets {
    int64_t W1, b1, W2, b2, W3, b3, total;
};

__host__ __device__ inline MlpOffsets offsets(const dvq_mlp_shape& s) {
    MlpOffsets o;
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)s.hidden * s.d_in;
    o.W2 = o.b1 + s.hidden;
    o.b2 = o.W2 + (int64_t)s.hidden * s.hidden;
    o.W3 = o.b2 + s.hidden;
    o.b3 = o.W3 + (int64_t)s.d_out * s.hidden;
    o.total = o.b3 + s.d_out;
    return o;
}

inline dvq_status check_shape(const dvq_mlp_shape* s, int batch) {
    DVQ_REQUIRE(s != nullptr, "shape is NULL");
    DVQ_REQUIRE(s->d_in >= 1 && s->d_in <= 64, "d_in=%d outside 1..64", s->d_in);
    DVQ_REQUIRE(s->hidden >= 32 && s->hidden <= 512 && s->hidden % 32 == 0,
                "hidden=%d must be a multiple of 32 in 32..512", s->hidden);
    DVQ_REQUIRE(s->d_out >= 1 && s->d_out <= 512, "d_out=%d outside 1..512", s->d_out);
    DVQ_REQUIRE(batch >= 1 && batch <= 65536, "batch=%d outside 1..65536", batch);
    return DVQ_OK;
}

}  // namespace dvq
