// Host / device records of the general bilinear level (k_bilinear.hip,
// bilinear.cpp): block grids of one dimension and the coefficients each
// kernel takes as an argument.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "starmm.h"

namespace starmm {

// The g blocks of one dimension: block i starts at off[i] and holds ext[i]
// rows (ceil(dim / g) each, fewer or none at the end).
struct BlockTable {
    int64_t off[MM_BILINEAR_MAX_GRID];
    int64_t ext[MM_BILINEAR_MAX_GRID];
};

// One side's pre-addition coefficients: coef[r * g * g + p].
struct BilinearSide {
    int32_t products;
    int8_t coef[MM_BILINEAR_MAX_PRODUCTS * MM_BILINEAR_MAX_GRID * MM_BILINEAR_MAX_GRID];
};

// The post-addition coefficients: coef[c * products + r].
struct BilinearOut {
    int32_t products;
    int8_t coef[MM_BILINEAR_MAX_GRID * MM_BILINEAR_MAX_GRID * MM_BILINEAR_MAX_PRODUCTS];
};

// The leaves of one operand as k-tiled bf16 hi/lo planes: prow rows (a
// multiple of 32) of row length ldo (a multiple of 16), leaf r at
// out + r * leaf_stride, its lo plane at + lo_off.  side_b: X is B (k x n),
// read in place, the leaves being B^T operands.
hipError_t launch_bilinear_pre(int g, bool side_b, const float* X, int64_t ldx, const BlockTable& rows,
                               const BlockTable& ks, uint16_t* out, int64_t prow, int64_t ldo, int64_t leaf_stride,
                               int64_t lo_off, const BilinearSide& cf, hipStream_t st);
// C blocks += the gamma combination of the products P (leaf r at
// P + r * leaf_stride, lr x lc, row length ldp).
hipError_t launch_bilinear_post(int g, const float* P, int64_t ldp, int64_t leaf_stride, const BlockTable& rows,
                                const BlockTable& cols, float* C, int64_t ldc, int64_t lr, int64_t lc,
                                const BilinearOut& cf, hipStream_t st);

}  // namespace starmm
