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
// Depth-first levels (SAR-Strassen, Lemma sar-strassen) reuse the same
// passes one product at a time: a `fix` word names, per level from the top
// (3 bits each), the one product a depth-first level computes in this round
// (7 = all seven, a breadth-first level).  The pre-addition then forms only
// the leaves under the fixed digits (and skips the source blocks their
// coefficients zero out); the round's post-addition combines its leaves over
// the breadth-first levels and adds the result into every C block the fixed
// digits reach, times the product of their gammas.
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

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPreThreads = 256;
// workgroup of the tiled pre-additions (one level: 4% faster than 256)
constexpr int kPreTiledThreads = 512;
constexpr int kFree = 7;  // fix digit of a breadth-first level: all seven products

// Coefficient of quadrant (i, j) in operand r of the given side.
// SIDE 0: A (alpha); 1: B (beta); 2: B^T, whose quadrant (i, j) is B's (j, i).
template <int VAR, int SIDE>
__device__ constexpr int coef(int r, int i, int j) {
    return SIDE == 0 ? strassen_alpha(VAR, r, i, j)
                     : (SIDE == 1 ? strassen_beta(VAR, r, i, j) : strassen_beta(VAR, r, j, i));
}

// Product over the fixed levels of the coefficient that source block
// (I, J) of the depth-D block grid (top-level bit most significant) has in
// the round's leaves; 0 means no leaf of the round reads the block.
template <int D, int VAR, int SIDE>
__device__ inline int fixed_coef(uint32_t fix, int I, int J) {
    int c = 1;
#pragma unroll
    for (int l = 0; l < D; ++l) {
        const int f = (int)((fix >> (3 * l)) & 7);
        if (f == kFree) continue;
        c *= coef<VAR, SIDE>(f, (I >> (D - 1 - l)) & 1, (J >> (D - 1 - l)) & 1);
    }
    return c;
}

// Leaf value -> fp32 output.
template <typename T>
__device__ inline void write_leaf(float* out, int64_t idx, int64_t, T v) {
    out[idx] = (float)v;
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
    __device__ static void run(const T* vals, int64_t leaf, O* out, int64_t leaf_stride, int64_t pos, int64_t lo_off,
                               uint32_t fix) {
        constexpr int W = Pow2<D>::v, H = W / 2;
        const int f = (int)(fix & 7);
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            if (f != kFree && r != f) continue;
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
            PreAdd<D - 1, VAR, SIDE, T>::run(sub, f == kFree ? leaf * 7 + r : leaf, out, leaf_stride, pos, lo_off,
                                             fix >> 3);
        }
    }
};

template <int VAR, int SIDE, typename T>
struct PreAdd<0, VAR, SIDE, T> {
    template <typename O>
    __device__ static void run(const T* vals, int64_t leaf, O* out, int64_t leaf_stride, int64_t pos, int64_t lo_off,
                               uint32_t) {
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

// PostAdd over 4 consecutive positions at once (out[block][position]),
// each position combined in the same order as PostAdd.
template <int D, int VAR, typename T>
struct PostAdd4 {
    __device__ static void run(const float* P, int64_t leaf, int64_t leaf_stride, int64_t pos, T (*out)[4]) {
        constexpr int W = Pow2<D>::v, H = W / 2;
#pragma unroll
        for (int q = 0; q < W * W; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) out[q][e] = T(0);
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            T sub[H * H][4];
            PostAdd4<D - 1, VAR, T>::run(P, leaf * 7 + r, leaf_stride, pos, sub);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int c = strassen_gamma(VAR, r, i, j);
                    if (c == 0) continue;
#pragma unroll
                    for (int I = 0; I < H; ++I)
#pragma unroll
                        for (int J = 0; J < H; ++J)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                T& o = out[(i * H + I) * W + (j * H + J)][e];
                                if (c == 1) o += sub[I * H + J][e];
                                else o -= sub[I * H + J][e];
                            }
                }
        }
    }
};

// (the products are read once: non-temporal loads, which measured 10%
// faster for the pass than plain ones)
template <int VAR, typename T>
struct PostAdd4<0, VAR, T> {
    __device__ static void run(const float* P, int64_t leaf, int64_t leaf_stride, int64_t pos, T (*out)[4]) {
        const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(P + leaf * leaf_stride + pos));
        out[0][0] = (T)v.x, out[0][1] = (T)v.y, out[0][2] = (T)v.z, out[0][3] = (T)v.w;
    }
};

// Pre-addition over one operand X (rows x cols, leading dimension ldx) into
// fp32 leaves: leaf operand (r_1..r_D) is written at out + leaf *
// leaf_stride, rows `leaf_rows` x cols `leaf_cols`, leading dimension ldo.
template <int D, int VAR, int SIDE, typename T, typename O>
__global__ void __launch_bounds__(kPreThreads)
k_strassen_pre(const float* __restrict__ X, int64_t ldx, PathTable rows, PathTable cols, O* __restrict__ out,
               int64_t leaf_rows, int64_t leaf_cols, int64_t ldo, int64_t leaf_stride, int64_t lo_off,
               uint32_t fix) {
    const int64_t col_blocks = (leaf_cols + kPreThreads - 1) / kPreThreads;
    const int64_t x = (int64_t)blockIdx.x / col_blocks;
    const int64_t y = ((int64_t)blockIdx.x % col_blocks) * kPreThreads + threadIdx.x;
    if (y >= leaf_cols || x >= leaf_rows) return;
    constexpr int W = Pow2<D>::v;
    T vals[W * W];
#pragma unroll
    for (int I = 0; I < W; ++I)
#pragma unroll
        for (int J = 0; J < W; ++J) {
            const bool ok = x < rows.ext[I] && y < cols.ext[J] && fixed_coef<D, VAR, SIDE>(fix, I, J) != 0;
            vals[I * W + J] = ok ? (T)X[(rows.off[I] + x) * ldx + cols.off[J] + y] : T(0);
        }
    PreAdd<D, VAR, SIDE, T>::run(vals, 0, out, leaf_stride, x * ldo + y, lo_off, fix);
}

// NV leaf values (consecutive k of one row) -> NV-element chunks of the hi
// and lo planes: hi = bf16(v), lo = bf16(v - hi) (fp16 when F16), the
// difference taken in T.
template <typename T, int NV, bool F16>
__device__ inline void write_leaf_v(uint16_t* out, int64_t idx, int64_t lo_off, const T (&v)[NV]) {
    uint32_t h[NV], l[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        if constexpr (F16) {
            h[e] = fp16_bits((float)v[e]);
            l[e] = fp16_bits((float)(v[e] - (T)fp16_value(h[e])));
        } else {
            h[e] = bf16_bits((float)v[e]);
            l[e] = bf16_bits((float)(v[e] - (T)bf16_value(h[e])));
        }
    }
    if constexpr (NV == 8) {
        *reinterpret_cast<uint4*>(out + idx) =
            make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16, h[6] | h[7] << 16);
        *reinterpret_cast<uint4*>(out + idx + lo_off) =
            make_uint4(l[0] | l[1] << 16, l[2] | l[3] << 16, l[4] | l[5] << 16, l[6] | l[7] << 16);
    } else if constexpr (NV == 4) {
        *reinterpret_cast<uint2*>(out + idx) = make_uint2(h[0] | h[1] << 16, h[2] | h[3] << 16);
        *reinterpret_cast<uint2*>(out + idx + lo_off) = make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16);
    } else if constexpr (NV == 2) {
        *reinterpret_cast<uint32_t*>(out + idx) = h[0] | h[1] << 16;
        *reinterpret_cast<uint32_t*>(out + idx + lo_off) = l[0] | l[1] << 16;
    } else {
        out[idx] = (uint16_t)h[0];
        out[idx + lo_off] = (uint16_t)l[0];
    }
}

// PreAdd over NV positions at once (vals[block][lane of the chunk]).
template <int D, int VAR, int SIDE, typename T, int NV, bool F16>
struct PreAddV {
    __device__ static void run(const T (*vals)[NV], int64_t leaf, uint16_t* out, int64_t leaf_stride, int64_t pos,
                               int64_t lo_off, uint32_t fix) {
        constexpr int W = Pow2<D>::v, H = W / 2;
        const int f = (int)(fix & 7);
#pragma unroll
        for (int r = 0; r < 7; ++r) {
            if (f != kFree && r != f) continue;
            T sub[H * H][NV];
#pragma unroll
            for (int I = 0; I < H; ++I)
#pragma unroll
                for (int J = 0; J < H; ++J)
#pragma unroll
                    for (int e = 0; e < NV; ++e) {
                        T s = T(0);
#pragma unroll
                        for (int i = 0; i < 2; ++i)
#pragma unroll
                            for (int j = 0; j < 2; ++j) {
                                const int c = coef<VAR, SIDE>(r, i, j);
                                const T v = vals[(i * H + I) * W + (j * H + J)][e];
                                if (c == 1) s += v;
                                else if (c == -1) s -= v;
                            }
                        sub[I * H + J][e] = s;
                    }
            PreAddV<D - 1, VAR, SIDE, T, NV, F16>::run(sub, f == kFree ? leaf * 7 + r : leaf, out, leaf_stride, pos,
                                                       lo_off, fix >> 3);
        }
    }
};

template <int VAR, int SIDE, typename T, int NV, bool F16>
struct PreAddV<0, VAR, SIDE, T, NV, F16> {
    __device__ static void run(const T (*vals)[NV], int64_t leaf, uint16_t* out, int64_t leaf_stride, int64_t pos,
                               int64_t lo_off, uint32_t) {
        write_leaf_v<T, NV, F16>(out, leaf * leaf_stride + pos, lo_off, vals[0]);
    }
};

// Pre-addition straight into k-tiled bf16 (or fp16) hi/lo planes (row length ldo,
// prow = leaf rows rounded up to whole 32-row units).  A thread owns NV
// consecutive tiled positions (NV consecutive k of one leaf row), so every
// store is an NV-element chunk and a wave's stores are contiguous.
// SIDE 0: X = A (rows x k).  SIDE 2: X = B (k x n) read in place, the leaves
// being B^T operands: block (I, J) of the B^T grid is B's block (J, I)
// transposed, so element (x, y) of it is X[(cols.off[J] + y) * ldx +
// rows.off[I] + x]; lanes of a wave then read runs of consecutive B columns.
// Positions outside the source (padding rows, k past the operand) get 0.
// F16: fp16 planes, every value of leaf row x multiplied by scale[x] (an exact
// power of two) before the split.
template <int D, int VAR, int SIDE, typename T, int NV, bool F16>
__global__ void __launch_bounds__(kPreTiledThreads)
k_strassen_pre_tiled(const float* __restrict__ X, int64_t ldx, PathTable rows, PathTable cols,
                     uint16_t* __restrict__ out, int64_t prow, int64_t ldo, int64_t leaf_stride, int64_t lo_off,
                     const float* __restrict__ scale, uint32_t fix) {
    int64_t pos = ((int64_t)blockIdx.x * kPreTiledThreads + threadIdx.x) * NV;
    if (pos >= prow * ldo) return;
    const int64_t ku = ldo / kPlaneKBlock;
    if constexpr (SIDE == 2) {
        // units in k-block-major order: consecutive workgroups take the
        // row blocks (32 columns of B each) of one k-block, so B is read
        // along its rows rather than down 16-row strips
        const int64_t lin = pos >> 9, nrb = prow / kPlaneRowBlock;
        pos = ((lin % nrb) * ku + lin / nrb) * 512 + (pos & 511);
    }
    const int64_t unit = pos >> 9;
    const int p = (int)(pos & 511), ri = p >> 4, c = ((p >> 3) & 1) ^ tiled_swz(ri);
    const int64_t x = (unit / ku) * kPlaneRowBlock + ri;
    const int64_t y0 = (unit % ku) * kPlaneKBlock + c * 8 + (p & 7);
    constexpr int W = Pow2<D>::v;
    T vals[W * W][NV];
#pragma unroll
    for (int I = 0; I < W; ++I)
#pragma unroll
        for (int J = 0; J < W; ++J) {
            const bool row_ok = x < rows.ext[I] && fixed_coef<D, VAR, SIDE>(fix, I, J) != 0;
            if constexpr (SIDE == 0 && NV == 8) {
                const float* src = X + (rows.off[I] + x) * ldx + cols.off[J] + y0;
                if (row_ok && y0 + 8 <= cols.ext[J] && ((uintptr_t)src & 15) == 0) {
                    const float4 a = reinterpret_cast<const float4*>(src)[0];
                    const float4 b = reinterpret_cast<const float4*>(src)[1];
                    const float f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e) vals[I * W + J][e] = (T)f[e];
                    continue;
                }
            }
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                const int64_t y = y0 + e;
                const bool ok = row_ok && y < cols.ext[J];
                const int64_t idx = SIDE == 2 ? (cols.off[J] + y) * ldx + rows.off[I] + x
                                              : (rows.off[I] + x) * ldx + cols.off[J] + y;
                vals[I * W + J][e] = ok ? (T)X[idx] : T(0);
            }
        }
    if constexpr (F16) {
        const T sc = (T)scale[x];
#pragma unroll
        for (int q = 0; q < W * W; ++q)
#pragma unroll
            for (int e = 0; e < NV; ++e) vals[q][e] *= sc;
    }
    PreAddV<D, VAR, SIDE, T, NV, F16>::run(vals, 0, out, leaf_stride, pos, lo_off, fix);
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

// k_strassen_post with a thread per 4 consecutive leaf columns: 16-byte
// loads of the products (rows padded to a multiple of 4 columns, 16-byte
// aligned) and 16-byte read-modify-writes of C where a block's columns and
// C's alignment allow, single elements elsewhere.  Same values and order.
template <int D, int VAR, typename T>
__global__ void __launch_bounds__(kPreThreads)
k_strassen_post4(const float* __restrict__ P, int64_t ldp, int64_t leaf_stride, PathTable rows, PathTable cols,
                 float* __restrict__ C, int64_t ldc, int64_t leaf_rows, int64_t leaf_cols) {
    const int64_t groups = (leaf_cols + 3) / 4;
    const int64_t col_blocks = (groups + kPreThreads - 1) / kPreThreads;
    const int64_t x = (int64_t)blockIdx.x / col_blocks;
    const int64_t y0 = (((int64_t)blockIdx.x % col_blocks) * kPreThreads + threadIdx.x) * 4;
    if (y0 >= leaf_cols || x >= leaf_rows) return;
    constexpr int W = Pow2<D>::v;
    T out[W * W][4];
    PostAdd4<D, VAR, T>::run(P, 0, leaf_stride, x * ldp + y0, out);
#pragma unroll
    for (int I = 0; I < W; ++I) {
        if (x >= rows.ext[I]) continue;
#pragma unroll
        for (int J = 0; J < W; ++J) {
            const T* o = out[I * W + J];
            float* c = C + (rows.off[I] + x) * ldc + cols.off[J] + y0;
            const int64_t ye = cols.ext[J] - y0;  // columns e < ye exist
            if (ye >= 4 && ((uintptr_t)c & 15) == 0) {
                float4 v = *reinterpret_cast<float4*>(c);
                v.x = (float)((T)v.x + o[0]), v.y = (float)((T)v.y + o[1]);
                v.z = (float)((T)v.z + o[2]), v.w = (float)((T)v.w + o[3]);
                *reinterpret_cast<float4*>(c) = v;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e < ye) c[e] = (float)((T)c[e] + o[e]);
            }
        }
    }
}

// Post-addition of one depth-first round.  The round's 7^BF products P
// (one per digit tuple of the breadth-first levels below the depth-first
// ones) are combined over those levels at one leaf position (as in
// k_strassen_post); the resulting 2^BF x 2^BF blocks are then added into
// every depth-first target: C block (I_top, J_top) of the depth-(D - BF)
// grid, times the product of the round's gammas (+1 or -1).  Blocks are
// indexed on the full depth-D path tables, top-level bit most significant.
template <int BF, int VAR, typename T>
__global__ void __launch_bounds__(kPreThreads)
k_strassen_post_round(const float* __restrict__ P, int64_t ldp, int64_t leaf_stride, PathTable rows, PathTable cols,
                      float* __restrict__ C, int64_t ldc, int64_t leaf_rows, int64_t leaf_cols, RoundTargets tg) {
    const int64_t col_blocks = (leaf_cols + kPreThreads - 1) / kPreThreads;
    const int64_t x = (int64_t)blockIdx.x / col_blocks;
    const int64_t y = ((int64_t)blockIdx.x % col_blocks) * kPreThreads + threadIdx.x;
    if (y >= leaf_cols || x >= leaf_rows) return;
    constexpr int W = Pow2<BF>::v;
    T out[W * W];
    PostAdd<BF, VAR, T>::run(P, 0, leaf_stride, x * ldp + y, out);
    for (int t = 0; t < tg.count; ++t) {
        const int itop = tg.target[t] & 0xff, jtop = (tg.target[t] >> 8) & 0xff;
        const bool neg = (tg.target[t] >> 16) & 1;
#pragma unroll
        for (int I = 0; I < W; ++I)
#pragma unroll
            for (int J = 0; J < W; ++J) {
                const int bi = itop * W + I, bj = jtop * W + J;
                if (x < rows.ext[bi] && y < cols.ext[bj]) {
                    float* c = C + (rows.off[bi] + x) * ldc + cols.off[bj] + y;
                    const T v = out[I * W + J];
                    *c = (float)(neg ? (T)*c - v : (T)*c + v);
                }
            }
    }
}

template <int BF, int VAR, typename T>
hipError_t post_round_launch(const float* P, int64_t ldp, int64_t ls, const PathTable& rows, const PathTable& cols,
                             float* C, int64_t ldc, int64_t lr, int64_t lc, const RoundTargets& tg, hipStream_t st) {
    dim3 grid((unsigned)(ceil_div(lc, kPreThreads) * lr));
    ProfScope ps("strassen_post", st);
    hipLaunchKernelGGL((k_strassen_post_round<BF, VAR, T>), grid, dim3(kPreThreads), 0, st, P, ldp, ls, rows, cols, C,
                       ldc, lr, lc, tg);
    return hipGetLastError();
}

template <int VAR, typename T>
hipError_t post_round_depth(int bf, const float* P, int64_t ldp, int64_t ls, const PathTable& rows,
                            const PathTable& cols, float* C, int64_t ldc, int64_t lr, int64_t lc,
                            const RoundTargets& tg, hipStream_t st) {
    switch (bf) {
        case 0: return post_round_launch<0, VAR, T>(P, ldp, ls, rows, cols, C, ldc, lr, lc, tg, st);
        case 1: return post_round_launch<1, VAR, T>(P, ldp, ls, rows, cols, C, ldc, lr, lc, tg, st);
        default: return post_round_launch<2, VAR, T>(P, ldp, ls, rows, cols, C, ldc, lr, lc, tg, st);
    }
}

template <int D, int VAR, typename T, typename O>
hipError_t pre_launch(int side, const float* X, int64_t ldx, const PathTable& rows, const PathTable& cols, O* out,
                      int64_t lr, int64_t lc, int64_t ldo, int64_t ls, int64_t lo_off, uint32_t fix, hipStream_t st) {
    dim3 grid((unsigned)(ceil_div(lc, kPreThreads) * lr));
    ProfScope ps("strassen_pre", st);
    if (side == 0)
        hipLaunchKernelGGL((k_strassen_pre<D, VAR, 0, T, O>), grid, dim3(kPreThreads), 0, st, X, ldx, rows, cols, out,
                           lr, lc, ldo, ls, lo_off, fix);
    else if (side == 1)
        hipLaunchKernelGGL((k_strassen_pre<D, VAR, 1, T, O>), grid, dim3(kPreThreads), 0, st, X, ldx, rows, cols, out,
                           lr, lc, ldo, ls, lo_off, fix);
    else
        hipLaunchKernelGGL((k_strassen_pre<D, VAR, 2, T, O>), grid, dim3(kPreThreads), 0, st, X, ldx, rows, cols, out,
                           lr, lc, ldo, ls, lo_off, fix);
    return hipGetLastError();
}

template <int D, int VAR, typename T>
hipError_t post_launch(const float* P, int64_t ldp, int64_t ls, const PathTable& rows, const PathTable& cols,
                       float* C, int64_t ldc, int64_t lr, int64_t lc, hipStream_t st) {
    if constexpr (D == 1) {  // (deeper levels would hold 16 blocks x 4 positions per thread)
        // 16-byte product loads stay inside each padded row
        if (ldp % 4 == 0 && ls % 4 == 0 && ldp >= round_up(lc, 4) && ((uintptr_t)P & 15) == 0) {
            dim3 grid((unsigned)(ceil_div(ceil_div(lc, 4), kPreThreads) * lr));
            ProfScope ps("strassen_post", st);
            hipLaunchKernelGGL((k_strassen_post4<D, VAR, T>), grid, dim3(kPreThreads), 0, st, P, ldp, ls, rows, cols,
                               C, ldc, lr, lc);
            return hipGetLastError();
        }
    }
    dim3 grid((unsigned)(ceil_div(lc, kPreThreads) * lr));
    ProfScope ps("strassen_post", st);
    hipLaunchKernelGGL((k_strassen_post<D, VAR, T>), grid, dim3(kPreThreads), 0, st, P, ldp, ls, rows, cols, C, ldc,
                       lr, lc);
    return hipGetLastError();
}

template <int VAR, typename T, typename O>
hipError_t pre_depth(int d, int side, const float* X, int64_t ldx, const PathTable& rows, const PathTable& cols,
                     O* out, int64_t lr, int64_t lc, int64_t ldo, int64_t ls, int64_t lo_off, uint32_t fix,
                     hipStream_t st) {
    switch (d) {
        case 1: return pre_launch<1, VAR, T, O>(side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off, fix, st);
        case 2: return pre_launch<2, VAR, T, O>(side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off, fix, st);
        default: return pre_launch<3, VAR, T, O>(side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off, fix, st);
    }
}

template <typename O>
hipError_t pre_any(int depth, int variant, bool f64, int side, const float* X, int64_t ldx, const PathTable& rows,
                   const PathTable& cols, O* out, int64_t lr, int64_t lc, int64_t ldo, int64_t ls, int64_t lo_off,
                   uint32_t fix, hipStream_t st) {
    if (lr == 0 || lc == 0) return hipSuccess;
    if (variant == MM_STRASSEN_CLASSIC)
        return f64 ? pre_depth<MM_STRASSEN_CLASSIC, double>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls,
                                                            lo_off, fix, st)
                   : pre_depth<MM_STRASSEN_CLASSIC, float>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls,
                                                           lo_off, fix, st);
    return f64 ? pre_depth<MM_STRASSEN_WINOGRAD, double>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls,
                                                         lo_off, fix, st)
               : pre_depth<MM_STRASSEN_WINOGRAD, float>(depth, side, X, ldx, rows, cols, out, lr, lc, ldo, ls, lo_off,
                                                        fix, st);
}

// Positions per thread of the tiled pre-addition: whole 16-byte chunks
// while the 4^D source values per position fit in registers.
template <int D, typename T>
constexpr int tiled_nv() {
    return D == 1 ? 8 : (D == 2 ? (sizeof(T) == 4 ? 8 : 4) : (sizeof(T) == 4 ? 2 : 1));
}

template <int D, int VAR, typename T>
hipError_t pre_tiled_launch(int side, const float* X, int64_t ldx, const PathTable& rows, const PathTable& cols,
                            uint16_t* out, int64_t prow, int64_t ldo, int64_t ls, int64_t lo_off, const float* scale,
                            uint32_t fix, hipStream_t st) {
    constexpr int NV = tiled_nv<D, T>();
    dim3 grid((unsigned)ceil_div(prow * ldo / NV, kPreTiledThreads));
    ProfScope ps("strassen_pre", st);
    const dim3 b(kPreTiledThreads);
    if (scale) {
        if (side == 0)
            hipLaunchKernelGGL((k_strassen_pre_tiled<D, VAR, 0, T, NV, true>), grid, b, 0, st, X, ldx, rows, cols, out,
                               prow, ldo, ls, lo_off, scale, fix);
        else
            hipLaunchKernelGGL((k_strassen_pre_tiled<D, VAR, 2, T, NV, true>), grid, b, 0, st, X, ldx, rows, cols, out,
                               prow, ldo, ls, lo_off, scale, fix);
    } else {
        if (side == 0)
            hipLaunchKernelGGL((k_strassen_pre_tiled<D, VAR, 0, T, NV, false>), grid, b, 0, st, X, ldx, rows, cols,
                               out, prow, ldo, ls, lo_off, scale, fix);
        else
            hipLaunchKernelGGL((k_strassen_pre_tiled<D, VAR, 2, T, NV, false>), grid, b, 0, st, X, ldx, rows, cols,
                               out, prow, ldo, ls, lo_off, scale, fix);
    }
    return hipGetLastError();
}

template <int VAR, typename T>
hipError_t pre_tiled_depth(int d, int side, const float* X, int64_t ldx, const PathTable& rows,
                           const PathTable& cols, uint16_t* out, int64_t prow, int64_t ldo, int64_t ls,
                           int64_t lo_off, const float* scale, uint32_t fix, hipStream_t st) {
    switch (d) {
        case 1:
            return pre_tiled_launch<1, VAR, T>(side, X, ldx, rows, cols, out, prow, ldo, ls, lo_off, scale, fix, st);
        case 2:
            return pre_tiled_launch<2, VAR, T>(side, X, ldx, rows, cols, out, prow, ldo, ls, lo_off, scale, fix, st);
        default:
            return pre_tiled_launch<3, VAR, T>(side, X, ldx, rows, cols, out, prow, ldo, ls, lo_off, scale, fix, st);
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
                               int64_t leaf_cols, int64_t ldo, int64_t leaf_stride, hipStream_t st, uint32_t fix) {
    return pre_any(depth, variant, f64, side, X, ldx, rows, cols, out, leaf_rows, leaf_cols, ldo, leaf_stride, 0, fix,
                   st);
}

hipError_t launch_strassen_pre_planes(int depth, int variant, bool f64, int side, const float* X, int64_t ldx,
                                      const PathTable& rows, const PathTable& cols, uint16_t* out, int64_t leaf_rows,
                                      int64_t ldo, int64_t leaf_stride, int64_t lo_off, hipStream_t st,
                                      const float* f16_scale, uint32_t fix) {
    if (leaf_rows == 0) return hipSuccess;
    if ((side != 0 && side != 2) || ldo <= 0 || ldo % kPlaneKBlock != 0) return hipErrorInvalidValue;
    const int64_t prow = plane_rows(leaf_rows);
    const float* sc = f16_scale;
    if (variant == MM_STRASSEN_CLASSIC)
        return f64 ? pre_tiled_depth<MM_STRASSEN_CLASSIC, double>(depth, side, X, ldx, rows, cols, out, prow, ldo,
                                                                  leaf_stride, lo_off, sc, fix, st)
                   : pre_tiled_depth<MM_STRASSEN_CLASSIC, float>(depth, side, X, ldx, rows, cols, out, prow, ldo,
                                                                 leaf_stride, lo_off, sc, fix, st);
    return f64 ? pre_tiled_depth<MM_STRASSEN_WINOGRAD, double>(depth, side, X, ldx, rows, cols, out, prow, ldo,
                                                               leaf_stride, lo_off, sc, fix, st)
               : pre_tiled_depth<MM_STRASSEN_WINOGRAD, float>(depth, side, X, ldx, rows, cols, out, prow, ldo,
                                                              leaf_stride, lo_off, sc, fix, st);
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

hipError_t launch_strassen_post_round(int bf_levels, int variant, bool f64, const float* P, int64_t ldp,
                                      int64_t leaf_stride, const PathTable& rows, const PathTable& cols, float* C,
                                      int64_t ldc, int64_t leaf_rows, int64_t leaf_cols, const RoundTargets& tg,
                                      hipStream_t st) {
    if (leaf_rows == 0 || leaf_cols == 0 || tg.count == 0) return hipSuccess;
    if (bf_levels < 0 || bf_levels > 2 || tg.count > kMaxRoundTargets) return hipErrorInvalidValue;
    if (variant == MM_STRASSEN_CLASSIC)
        return f64 ? post_round_depth<MM_STRASSEN_CLASSIC, double>(bf_levels, P, ldp, leaf_stride, rows, cols, C, ldc,
                                                                   leaf_rows, leaf_cols, tg, st)
                   : post_round_depth<MM_STRASSEN_CLASSIC, float>(bf_levels, P, ldp, leaf_stride, rows, cols, C, ldc,
                                                                  leaf_rows, leaf_cols, tg, st);
    return f64 ? post_round_depth<MM_STRASSEN_WINOGRAD, double>(bf_levels, P, ldp, leaf_stride, rows, cols, C, ldc,
                                                                leaf_rows, leaf_cols, tg, st)
               : post_round_depth<MM_STRASSEN_WINOGRAD, float>(bf_levels, P, ldp, leaf_stride, rows, cols, C, ldc,
                                                               leaf_rows, leaf_cols, tg, st);
}

}  // namespace starmm
