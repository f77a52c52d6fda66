// Strassen levels (Sec. strassen) as two fused elementwise passes around a
// batched base product:
//
//  pre-add : one pass over A (and one over B) forms the operands of all 7^d
//            base products.  A thread owns one position (x, y) of a leaf
//            block, reads the 4^d source values at that position (one per
//            depth-d block of the input, zero where a level padded an odd
//            dimension), and applies the per-level linear maps S_r / T_r
//            depth-first in registers.
//  post-add: one pass over the 7^d products P forms the 4^d output blocks at
//            a position and adds them into C (C <- C + A B).
//
// Classic is the seven products as the paper prints them; Winograd is
// Strassen-Winograd written out as +-1 combinations of quadrants.  In the
// high-accuracy mode the additions run in fp64 with one rounding per leaf
// operand and one rounding per output element.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "internal.hpp"
#include "strassen_tables.hpp"
#include "tile_bf16.hpp"

namespace starmm {

namespace {

constexpr int kPreThreads = 256;

// Coefficient of quadrant (i, j) in operand r of the given side.
// SIDE 0: A (alpha); 1: B (beta); 2: B^T, whose quadrant (i, j) is B's (j, i).
template <int VAR, int SIDE>
__device__ constexpr int coef(int r, int i, int j) {
    return SIDE == 0 ? strassen_alpha(VAR, r, i, j)
                     : (SIDE == 1 ? strassen_beta(VAR, r, i, j) : strassen_beta(VAR, r, j, i));
}

// Leaf value -> output: fp32, or bf16 hi/lo planes (hi = bf16(v), lo =
// bf16(v - hi), the difference taken in T so fp64 sums keep their low bits).
template <typename T>
__device__ inline void write_leaf(float* out, int64_t idx, int64_t, T v) {
    out[idx] = (float)v;
}
template <typename T>
__device__ inline void write_leaf(uint16_t* out, int64_t idx, int64_t lo_off, T v) {
    const uint32_t h = bf16_bits((float)v);
    const T rest = v - (T)bf16_value(h);
    out[idx] = (uint16_t)h;
    out[idx + lo_off] = (uint16_t)bf16_bits((float)rest);
}

template <int D>
struct Pow2 {
    static constexpr int v = 1 << D;
};

// Depth-first pre-addition: vals is a (2^D x 2^D) block grid at one position,
// index [I * 2^D + J] with the level-1 quadrant bit most significant.
template <int D, int VAR, int SIDE, typename T>
struct PreAdd {
    template <typename O>
    __device__ static void run(const T* vals, int64_t leaf, O* out, int64_t leaf_stride, int64_t pos, int64_t lo_off) {
        constexpr int W = Pow2<D>::v, H = W / 2;
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            T sub[H * H];
#pragma unroll
            for (int I = 0; I < H; ++I)
#pragma unroll
                for (int J = 0; J < H; ++J) {
                    T s = T(0);
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            const int c = coef<VAR, SIDE>(r, i, j);
                            const T v = vals[(i * H + I) * W + (j * H + J)];
                            if (c == 1) s += v;
                            else if (c == -1) s -= v;
                        }
                    sub[I * H + J] = s;
                }
            PreAdd<D - 1, VAR, SIDE, T>::run(sub, leaf * 7 + r, out, leaf_stride, pos, lo_off);
        }
    }
};

template <int VAR, int SIDE, typename T>
struct PreAdd<0, VAR, SIDE, T> {
    template <typename O>
    __device__ static void run(const T* vals, int64_t leaf, O* out, int64_t leaf_stride, int64_t pos, int64_t lo_off) {
        write_leaf(out, leaf * leaf_stride + pos, lo_off, vals[0]);
    }
};

// Depth-first post-addition: out (2^D x 2^D) = sum_r gamma_r (x) (result of product r).
template <int D, int VAR, typename T>
struct PostAdd {
    __device__ static void run(const float* P, int64_t leaf, int64_t leaf_stride, int64_t pos, T* out) {
        constexpr int W = Pow2<D>::v, H = W / 2;
#pragma unroll
        for (int q = 0; q < W * W; ++q) out[q] = T(0);
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            T sub[H * H];
            PostAdd<D - 1, VAR, T>::run(P, leaf * 7 + r, leaf_stride, pos, sub);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int c = strassen_gamma(VAR, r, i, j);
                    if (c == 0) continue;
#pragma unroll
                    for (int I = 0; I < H; ++I)
#pragma unroll
                        for (int J = 0; J < H; ++J) {
                            T& o = out[(i * H + I) * W + (j * H + J)];
                            if (c == 1) o += sub[I * H + J];
                            else o -= sub[I * H + J];
                        }
                }
        }
    }
};

template <int VAR, typename T>
struct PostAdd<0, VAR, T> {
    __device__ static void run(const float* P, int64_t leaf, int64_t leaf_stride, int64_t pos, T* out) {
        out[0] = (T)P[leaf * leaf_stride + pos];
    }
};

// Pre-addition over one operand X (rows x cols, leading dimension ldx).
// Leaf operand (r_1..r_D) is written at out + leaf * leaf_stride, rows
// `leaf_rows` x cols `leaf_cols`: fp32 row-major with leading dimension ldo,
// or (bf16 planes) k-tiled with row length ldo = leaf_cols.  Planes are
// walked in tiled order, one element per thread, so stores stay contiguous;
// positions outside the source (padding rows, k past the operand) get 0.
template <int D, int VAR, int SIDE, typename T, typename O>
__global__ void __launch_bounds__(kPreThreads)
k_strassen_pre(const float* __restrict__ X, int64_t ldx, PathTable rows, PathTable cols, O* __restrict__ out,
               int64_t leaf_rows, int64_t leaf_cols, int64_t ldo, int64_t leaf_stride, int64_t lo_off) {
    int64_t x, y, pos;
    if constexpr (std::is_same<O, uint16_t>::value) {
        pos = (int64_t)blockIdx.x * kPreThreads + threadIdx.x;
        if (pos >= leaf_rows * ldo) return;  // leaf_rows: whole 32-row units here
        const int64_t unit = pos >> 9, ku = ldo / kPlaneKBlock;
        const int p = (int)(pos & 511), ri = p >> 4, c = ((p >> 3) & 1) ^ tiled_swz(ri);
        x = (unit / ku) * kPlaneRowBlock + ri;
        y = (unit % ku) * kPlaneKBlock + c * 8 + (p & 7);
    } else {
        const int64_t col_blocks = (leaf_cols + kPreThreads - 1) / kPreThreads;
        x = (int64_t)blockIdx.x / col_blocks;
        y = ((int64_t)blockIdx.x % col_blocks) * kPreThreads + threadIdx.x;
        if (y >= leaf_cols || x >= leaf_rows) return;
        pos = x * ldo + y;
    }
    constexpr int W = Pow2<D>::v;
    T vals[W * W];
#pragma unroll
    for (int I = 0; I < W; ++I)
#pragma unroll
        for (int J = 0; J < W; ++J) {
            const bool ok = x < rows.ext[I] && y < cols.ext[J];
            vals[I * W + J] = ok ? (T)X[(rows.off[I] + x) * ldx + cols.off[J] + y] : T(0);
        }
    PreAdd<D, VAR, SIDE, T>::run(vals, 0, out, leaf_stride, pos, lo_off);
}

template <int D, int VAR, typename T>
__global__ void __launch_bounds__(kPreThreads)
k_strassen_post(const float* __restrict__ P, int64_t ldp, int64_t leaf_stride, PathTable rows, PathTable cols,
                float* __restrict__ C, int64_t ldc, int64_t leaf_rows, int64_t leaf_cols) {
    const int64_t col_blocks = (leaf_cols + kPreThreads - 1) / kPreThreads;
    const int64_t x = (int64_t)blockIdx.x / col_blocks;
    const int64_t y = ((int64_t)blockIdx.x % col_blocks) * kPreThreads + threadIdx.x;
    if (y >= leaf_cols || x >= leaf_rows) return;
    constexpr int W = Pow2<D>::v;
    T out[W * W];
    PostAdd<D, VAR, T>::run(P, 0, leaf_stride, x * ldp + y, out);
#pragma unroll
    for (int I = 0; I < W; ++I)
#pragma unroll
        for (int J = 0; J < W; ++J) {
            if (x < rows.ext[I] && y < cols.ext[J]) {
                float* c = C + (rows.off[I] + x) * ldc + cols.off[J] + y;
                *c = (float)((T)*c + out[I * W + J]);
            }
        }
}

template <int D, int VAR, typename T, typename O>
hipError_t pre_launch(int side, const float* X, int64_t ldx, const PathTable& rows, const PathTable& cols, O* out,
                      int64_t lr, int64_t lc, int64_t ldo, int64_t ls, int64_t lo_off, hipStream_t st) {
    if constexpr (std::is_same<O, uint16_t>::value) {
        if (lc != ldo || ldo % kPlaneKBlock != 0) return hipErrorInvalidValue;
        lr = plane_rows(lr);
    }
    dim3 grid((unsigned)(std::is_same<O, uint16_t>::value ? ceil_div(lr * ldo, kPreThreads)
                                                          : ceil_div(lc, kPreThreads) * lr));
    ProfScope ps("strassen_pre", st);
    if (side == 0)
        hipLaunchKernelGGL((k_strassen_pre<D, VAR, 0, T, O>), grid, dim3(kPreThreads), 0, st, X, ldx, rows, cols, out,
                           lr, lc, ldo, ls, lo_off);
    else if (side == 1)
        hipLaunchKernelGGL((k_strassen_pre<D, VAR, 1, T, O>), grid, dim3(kPreThreads), 0, st, X, ldx, rows, cols, out,
                           lr, lc, ldo, ls, lo_off);
    else
        hipLaunchKernelGGL((k_strassen_pre<D, VAR, 2, T, O>), grid, dim3(kPreThreads), 0, st, X, ldx, rows, cols, out,
                           lr, lc, ldo, ls, lo_off);
    return hipGetLastError();
}

template <int D, int VAR, typename T>
hipError_t post_launch(const float* P, int64_t ldp, int64_t ls, const PathTable& rows, const PathTable& cols,
                       float* C, int64_t ldc, int64_t lr, int64_t lc, hipStream_t st) {
    dim3 grid((unsigned)(ceil_div(lc, kPreThreads) * lr));
    ProfScope ps("strassen_post", st);
    hipLaunchKernelGGL((k_strassen_post<D, VAR, T>), grid, dim3(kPreThreads), 0, st, P, ldp, ls, rows, cols, C, ldc,
                       lr, lc);
    return hipGetLastError();
}

template <int VAR, typename T, typename O>
hipError_t pre_depth(int d, int side, const float* X, int64_t ldx, const PathTable& rows, const PathTable& cols,
                     O* out, int64_t lr, int64_t lc, int64_t ldo, int64_t ls, int64_t lo_off, hipStream_t st) {
    switch (d) {
        case 1: return pre_launch<1, VAR, T, O>(side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off, st);
        case 2: return pre_launch<2, VAR, T, O>(side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off, st);
        default: return pre_launch<3, VAR, T, O>(side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off, st);
    }
}

template <typename O>
hipError_t pre_any(int depth, int variant, bool f64, int side, const float* X, int64_t ldx, const PathTable& rows,
                   const PathTable& cols, O* out, int64_t lr, int64_t lc, int64_t ldo, int64_t ls, int64_t lo_off,
                   hipStream_t st) {
    if (lr == 0 || lc == 0) return hipSuccess;
    if (variant == MM_STRASSEN_CLASSIC)
        return f64 ? pre_depth<MM_STRASSEN_CLASSIC, double>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls,
                                                            lo_off, st)
                   : pre_depth<MM_STRASSEN_CLASSIC, float>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls,
                                                           lo_off, st);
    return f64 ? pre_depth<MM_STRASSEN_WINOGRAD, double>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls,
                                                         lo_off, st)
               : pre_depth<MM_STRASSEN_WINOGRAD, float>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off,
                                                        st);
}

// fp32 transpose through a 64 x 64 LDS tile: XT (cols x ldt) = X^T.
__global__ void __launch_bounds__(256)
k_transpose_f32(const float* __restrict__ X, int64_t ldx, int64_t rows, int64_t cols, float* __restrict__ XT,
                int64_t ldt) {
    __shared__ float t[64][65];
    const int64_t tiles_c = (cols + 63) / 64;
    const int64_t r0 = (int64_t)(blockIdx.x / tiles_c) * 64, c0 = (int64_t)(blockIdx.x % tiles_c) * 64;
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < rows && c < cols) t[i][tx] = X[r * ldx + c];
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (r < rows && c < cols) XT[c * ldt + r] = t[tx][i];
    }
}

template <int VAR, typename T>
hipError_t post_depth(int d, const float* P, int64_t ldp, int64_t ls, const PathTable& rows, const PathTable& cols,
                      float* C, int64_t ldc, int64_t lr, int64_t lc, hipStream_t st) {
    switch (d) {
        case 1: return post_launch<1, VAR, T>(P, ldp, ls, rows, cols, C, ldc, lr, lc, st);
        case 2: return post_launch<2, VAR, T>(P, ldp, ls, rows, cols, C, ldc, lr, lc, st);
        default: return post_launch<3, VAR, T>(P, ldp, ls, rows, cols, C, ldc, lr, lc, st);
    }
}

}  // namespace

hipError_t launch_strassen_pre(int depth, int variant, bool f64, int side, const float* X, int64_t ldx,
                               const PathTable& rows, const PathTable& cols, float* out, int64_t leaf_rows,
                               int64_t leaf_cols, int64_t ldo, int64_t leaf_stride, hipStream_t st) {
    return pre_any(depth, variant, f64, side, X, ldx, rows, cols, out, leaf_rows, leaf_cols, ldo, leaf_stride, 0, st);
}

hipError_t launch_strassen_pre_planes(int depth, int variant, bool f64, int side, const float* X, int64_t ldx,
                                      const PathTable& rows, const PathTable& cols, uint16_t* out, int64_t leaf_rows,
                                      int64_t leaf_cols, int64_t ldo, int64_t leaf_stride, int64_t lo_off,
                                      hipStream_t st) {
    return pre_any(depth, variant, f64, side, X, ldx, rows, cols, out, leaf_rows, leaf_cols, ldo, leaf_stride, lo_off,
                   st);
}

hipError_t launch_transpose_f32(const float* X, int64_t ldx, int64_t rows, int64_t cols, float* XT, int64_t ldt,
                                hipStream_t st) {
    if (rows == 0 || cols == 0) return hipSuccess;
    ProfScope ps("transpose", st);
    hipLaunchKernelGGL(k_transpose_f32, dim3((unsigned)(ceil_div(rows, 64) * ceil_div(cols, 64))), dim3(256), 0, st,
                       X, ldx, rows, cols, XT, ldt);
    return hipGetLastError();
}

hipError_t launch_strassen_post(int depth, int variant, bool f64, const float* P, int64_t ldp, int64_t leaf_stride,
                                const PathTable& rows, const PathTable& cols, float* C, int64_t ldc,
                                int64_t leaf_rows, int64_t leaf_cols, hipStream_t st) {
    if (leaf_rows == 0 || leaf_cols == 0) return hipSuccess;
    if (variant == MM_STRASSEN_CLASSIC)
        return f64 ? post_depth<MM_STRASSEN_CLASSIC, double>(depth, P, ldp, leaf_stride, rows, cols, C, ldc,
                                                             leaf_rows, leaf_cols, st)
                   : post_depth<MM_STRASSEN_CLASSIC, float>(depth, P, ldp, leaf_stride, rows, cols, C, ldc, leaf_rows,
                                                            leaf_cols, st);
    return f64 ? post_depth<MM_STRASSEN_WINOGRAD, double>(depth, P, ldp, leaf_stride, rows, cols, C, ldc, leaf_rows,
                                                          leaf_cols, st)
               : post_depth<MM_STRASSEN_WINOGRAD, float>(depth, P, ldp, leaf_stride, rows, cols, C, ldc, leaf_rows,
                                                         leaf_cols, st);
}

}  // namespace starmm
