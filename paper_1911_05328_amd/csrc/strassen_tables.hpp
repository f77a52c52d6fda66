// Coefficient tables of one Strassen level and the block-path tables of a
// multi-level recursion.  Shared by the host orchestration and the pre/post
// addition kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace starmm {

// Operand r (0..6) of one level: A-side operand = sum_ij alpha(r,i,j) A_ij,
// B-side operand = sum_ij beta(r,i,j) B_ij, and C_ij += gamma(r,i,j) P_r.
//
// Variant 0, the seven products as printed in Sec. strassen:
//   P1 = (A00+A11)(B00+B11)  P2 = (A10+A11)B00  P3 = A00(B01-B11)
//   P4 = A11(B10-B00)        P5 = (A00+A01)B11  P6 = (A10-A00)(B00+B01)
//   P7 = (A01-A11)(B10+B11)
//   C00 = P1+P4-P5+P7, C01 = P3+P5, C10 = P2+P4, C11 = P1+P3-P2+P6.
// Variant 1, Strassen-Winograd with its pre/post sums expanded to +-1
// combinations of quadrants:
//   M1 = A00 B00, M2 = A01 B10, M3 = (A00+A01-A10-A11) B11,
//   M4 = A11 (B00-B01-B10+B11), M5 = (A10+A11)(B01-B00),
//   M6 = (A10+A11-A00)(B00-B01+B11), M7 = (A00-A10)(B11-B01);
//   C00 = M1+M2, C01 = M1+M3+M5+M6, C10 = M1-M4+M6+M7, C11 = M1+M5+M6+M7.
__host__ __device__ constexpr int strassen_alpha(int variant, int r, int i, int j) {
    constexpr signed char cl[7][4] = {{1, 0, 0, 1}, {0, 0, 1, 1}, {1, 0, 0, 0}, {0, 0, 0, 1},
                                      {1, 1, 0, 0}, {-1, 0, 1, 0}, {0, 1, 0, -1}};
    constexpr signed char wi[7][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {1, 1, -1, -1}, {0, 0, 0, 1},
                                      {0, 0, 1, 1}, {-1, 0, 1, 1}, {1, 0, -1, 0}};
    return variant == 0 ? cl[r][i * 2 + j] : wi[r][i * 2 + j];
}

__host__ __device__ constexpr int strassen_beta(int variant, int r, int i, int j) {
    constexpr signed char cl[7][4] = {{1, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, -1}, {-1, 0, 1, 0},
                                      {0, 0, 0, 1}, {1, 1, 0, 0}, {0, 0, 1, 1}};
    constexpr signed char wi[7][4] = {{1, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}, {1, -1, -1, 1},
                                      {-1, 1, 0, 0}, {1, -1, 0, 1}, {0, -1, 0, 1}};
    return variant == 0 ? cl[r][i * 2 + j] : wi[r][i * 2 + j];
}

__host__ __device__ constexpr int strassen_gamma(int variant, int r, int i, int j) {
    constexpr signed char cl[7][4] = {{1, 0, 0, 1}, {0, 0, 1, -1}, {0, 1, 0, 1}, {1, 0, 1, 0},
                                      {-1, 1, 0, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}};
    constexpr signed char wi[7][4] = {{1, 1, 1, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, -1, 0},
                                      {0, 1, 0, 1}, {0, 1, 1, 1}, {0, 0, 1, 1}};
    return variant == 0 ? cl[r][i * 2 + j] : wi[r][i * 2 + j];
}

// Block paths of a d-level halving of one dimension (d <= 3): for path p
// (bit d-1-l chooses the half at level l), the offset of its first element
// and how many of its rows exist (the rest is zero padding of odd sizes).
struct PathTable {
    int64_t off[8];
    int64_t ext[8];
};

inline PathTable make_paths(int64_t dim, int d) {
    PathTable t{};
    for (int p = 0; p < (1 << d); ++p) {
        int64_t off = 0, ext = dim, size = dim;
        for (int l = 0; l < d; ++l) {
            const int bit = (p >> (d - 1 - l)) & 1;
            const int64_t h = (size + 1) / 2;
            if (bit) {
                off += h;
                ext = ext > h ? ext - h : 0;
            } else {
                ext = ext < h ? ext : h;
            }
            size = h;
        }
        t.off[p] = off;
        t.ext[p] = ext;
    }
    return t;
}

// Depth-first rounds of a Strassen recursion: a `fix` word holds one 3-bit
// digit per level from the top (level 0 in the low bits): the product a
// depth-first level computes in this round, or 7 for a breadth-first level
// (all seven at once).
constexpr uint32_t kAllFree = 0777;

// The C blocks one depth-first round adds into: entry t packs the block's
// row index (bits 0-7) and column index (bits 8-15) on the grid of the
// depth-first levels, and bit 16 set when the product of the round's gammas
// for that block is -1.
constexpr int kMaxRoundTargets = 64;
struct RoundTargets {
    int32_t count;
    int32_t target[kMaxRoundTargets];
};

// Padded size of one dimension after d halvings.
inline int64_t leaf_dim(int64_t dim, int d) {
    for (int l = 0; l < d; ++l) dim = (dim + 1) / 2;
    return dim;
}

}  // namespace starmm
