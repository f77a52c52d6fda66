// Device helpers shared by the tile kernels: the recursion's tile order, the
// k-range of a slice, and the XCD-aware workgroup numbering.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace starmm {

// Slice bookkeeping passed by value to every tile kernel.
struct SliceArgs {
    int32_t levels = 0;      // log2(split_k)
    int32_t sar_levels = 0;  // low `sar_levels` bits of the slice index are SAR (temporaries)
    int32_t tk = 16;         // k-depth of a staged tile; slice boundaries fall on multiples of it
    int32_t atomic_c = 0;    // TAR levels present: slice-0 writes to C are atomic
    int64_t temp_stride = 0; // elements between temporaries
    int64_t ldt = 0;         // leading dimension of a temporary
    int32_t overwrite = 0;   // slice-0 writes C = acc instead of C (+)= acc
    int32_t batch = 1;       // independent products of equal shape (split_k must be 1 if > 1)
    int64_t stride_a = 0, stride_b = 0, stride_c = 0;  // elements between consecutive products
    int64_t temp_batch_stride = 0;  // elements between the temporaries of consecutive products
    int64_t a_plane = 0, b_plane = 0;  // pre-split planes: element offset of the lo plane from the hi plane
    // fp16 planes of scaled operands: output (r, c) is multiplied by
    // row_unscale[r] * col_unscale[c] as it is written (same for every product)
    const float* row_unscale = nullptr;
    const float* col_unscale = nullptr;
};

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber so that XCD x runs one contiguous range of logical
// workgroups: neighbours in the recursion order then share that XCD's L2.
__device__ inline int64_t xcd_logical_id(int64_t bid, int64_t total) {
    const int64_t x = bid & 7, q = bid >> 3;
    const int64_t per = total >> 3, rem = total & 7;
    return x * per + (x < rem ? x : rem) + q;
}

// The t-th output tile in the order the recursion visits C.  Square-ish
// grids split into ceil/floor halves in both dimensions, quadrants in the
// order 00, 01, 10, 11 (eq. mm-dac); a grid at least twice as tall as wide
// (or wide as tall) is halved along its long side only, so the sub-grids
// the order walks through stay square-ish for rectangular products.  Every
// sub-grid takes one contiguous range of t, so the order is a permutation
// of the tm x tn tiles.
__host__ __device__ inline void recursion_tile(int64_t t, int64_t tm, int64_t tn, int64_t* ti, int64_t* tj) {
    int64_t i0 = 0, j0 = 0;
    while (tm > 1 || tn > 1) {
        if (tm >= 2 * tn) {
            const int64_t m0 = (tm + 1) >> 1;
            if (t < m0 * tn) {
                tm = m0;
            } else {
                t -= m0 * tn; i0 += m0; tm -= m0;
            }
            continue;
        }
        if (tn >= 2 * tm) {
            const int64_t n0 = (tn + 1) >> 1;
            if (t < tm * n0) {
                tn = n0;
            } else {
                t -= tm * n0; j0 += n0; tn -= n0;
            }
            continue;
        }
        const int64_t m0 = (tm + 1) >> 1, n0 = (tn + 1) >> 1;
        const int64_t m1 = tm - m0, n1 = tn - n0;
        const int64_t q00 = m0 * n0, q01 = m0 * n1, q10 = m1 * n0;
        if (t < q00) {
            tm = m0; tn = n0;
        } else if (t < q00 + q01) {
            t -= q00; j0 += n0; tm = m0; tn = n1;
        } else if (t < q00 + q01 + q10) {
            t -= q00 + q01; i0 += m0; tm = m1; tn = n0;
        } else {
            t -= q00 + q01 + q10; i0 += m0; j0 += n0; tm = m1; tn = n1;
        }
    }
    *ti = i0;
    *tj = j0;
}

// k-range [kb, ke) of slice `sigma`: the recursion halves the k-tiles at
// each of the top `levels` levels (ceil half first), bit (levels-1-l) of
// sigma choosing the half at level l.
__device__ inline void slice_k_range(int sigma, int levels, int64_t k, int tk, int64_t* kb, int64_t* ke) {
    int64_t start = 0, nb = (k + tk - 1) / tk;
    for (int l = 0; l < levels; ++l) {
        const int bit = (sigma >> (levels - 1 - l)) & 1;
        const int64_t h0 = (nb + 1) >> 1;
        if (bit) {
            start += h0;
            nb -= h0;
        } else {
            nb = h0;
        }
    }
    int64_t b = start * tk, e = (start + nb) * tk;
    *kb = b < k ? b : k;
    *ke = e < k ? e : k;
}

}  // namespace starmm
