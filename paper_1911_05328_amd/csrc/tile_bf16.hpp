// Core of the bf16 MFMA base-case tile: stage A/B through LDS and accumulate
// the tile product in registers.
//   MODE 0: fp32 A, B (row-major); split into bf16 hi/lo while staging.
//   MODE 1: bf16 A, B (row-major); one product.
//   MODE 2: pre-split bf16 planes in the k-tiled layout below: A hi at Av,
//           lo at Av + a_plane (m x k, row length lda); B^T hi at Bv, lo at
//           Bv + b_plane (n x k, row length ldb).  Staging is a plain copy.
//   MODE 3: one k-tiled bf16 plane per operand (A and B^T); one product.
//   MODE 4: as MODE 2 with fp16 hi/lo planes (fp16 MFMA).
//   MODE 5: as MODE 1 with fp16 A, B (fp16 MFMA).
//           Planes (MODE 2/3) must hold zeros from k to the row length, a
//           multiple of 32 (every producer here writes that padding).
// Used by the tile kernel and by the persistent batched kernel; the caller
// owns the epilogue.
//
// k-tiled planes: a plane of R x L bf16 values (L a multiple of 16, rows
// padded to a multiple of 32) is a grid of 1 KB units, each 32 rows x 16 k:
// unit (r / 32, k / 16) starts at element 32 L (r / 32) + 512 (k / 16), and
// inside it row r % 32 holds two 16-byte k-chunks, chunk c in slot
// c ^ tiled_swz(r % 32).  A unit is byte for byte the LDS image the 256-wide
// tile wants, so one wave copies it with one 1 KB direct-to-LDS load.
//
// MFMA lane layout (v_mfma_f32_32x32x16_bf16): lane l supplies row/col l%32
// and the 8 consecutive k values 8*(l/32)..+7 of a 16-deep step;
// accumulator register i of lane l is C[8*(i/4) + 4*(l/32) + i%4][l%32].
// LDS holds both operands k-contiguous ([row][k] for A, [col][k] for B),
// rows padded to 80 bytes so 16-byte reads of 32 consecutive rows are
// conflict-free.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace starmm {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBf16BK = 32;           // k per staged tile
constexpr int kBf16Ld = kBf16BK + 8;  // LDS row stride in bf16 elements (80 bytes)

constexpr int kPlaneRowBlock = 32;  // rows per unit of a k-tiled plane
constexpr int kPlaneKBlock = 16;    // k per unit

// Slot swizzle of a unit row: 16-byte reads of 32 consecutive rows at one
// k-chunk touch every LDS bank once per 8 (and per 16) lanes.
__host__ __device__ inline int tiled_swz(int ri) { return ((ri >> 2) ^ (ri >> 3)) & 1; }

// Element offset of (r, k) in a k-tiled plane with row length ld.
__host__ __device__ inline int64_t tiled_off(int64_t r, int64_t k, int64_t ld) {
    const int ri = (int)(r & 31), c = (int)((k >> 3) & 1);
    return (r >> 5) * 32 * ld + (k >> 4) * 512 + ((ri * 2 + (c ^ tiled_swz(ri))) << 3) + (k & 7);
}

// Rows of a k-tiled plane holding r rows (whole 32-row units).
__host__ __device__ inline int64_t plane_rows_dev(int64_t r) { return (r + 31) / 32 * 32; }

// Chunk q (16 bytes, 8 k values) of a k-tiled plane in tiled order (unit
// q / 64, slot q % 64) -> its row and first k.
__device__ inline void chunk_coord(int64_t q, int64_t ld, int64_t* r, int64_t* k0) {
    const int64_t unit = q >> 6, ku = ld / kPlaneKBlock;
    const int p = (int)(q & 63), ri = p >> 1, c = (p & 1) ^ tiled_swz(ri);
    *r = (unit / ku) * kPlaneRowBlock + ri;
    *k0 = (unit % ku) * kPlaneKBlock + c * 8;
}

__device__ inline uint32_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ inline float bf16_value(uint32_t bits) { return __builtin_bit_cast(float, bits << 16); }

// 16 bytes from any address p: one aligned 16-byte load when p is 16-byte
// aligned, else the two aligned 16-byte blocks that contain [p, p+16) and a
// byte funnel-shift.  Every byte read lies in a 16-byte-aligned block that
// also holds a requested byte, so the read never reaches a page that the
// requested range does not touch.
// Operands of the tile core live in device global memory; pointers of this
// type make every access a global one even where the pointer was read from
// memory (a generic pointer would be accessed with flat instructions, whose
// completion also counts against the LDS wait counter).
template <class T>
using gptr = __attribute__((address_space(1))) T*;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte global load from a 16-byte aligned address.
__device__ inline uint4 ld16(gptr<const void> p) {
    const u32x4 v = *(gptr<const u32x4>)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ inline uint4 load16_any(gptr<const void> p) {
    const uintptr_t a = (uintptr_t)p;
    const uint32_t off = (uint32_t)(a & 15u);
    if (off == 0) return ld16(p);
    const uint4 x = ld16((gptr<const void>)(a - off)), y = ld16((gptr<const void>)(a - off + 16));
    const uint32_t w[8] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w};
    const uint32_t wo = off >> 2, sh = (off & 3u) * 8u;
    uint32_t r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t lo = w[i], hi = w[i + 1];
#pragma unroll
        for (uint32_t q = 1; q < 4; ++q)
            if (wo == q) {
                lo = w[i + q];
                hi = w[i + q + 1];
            }
        r[i] = sh ? (uint32_t)((((uint64_t)hi << 32) | lo) >> sh) : lo;
    }
    return make_uint4(r[0], r[1], r[2], r[3]);
}

// Split x into hi/lo bf16 bit patterns, each rounded to nearest even.
__device__ inline void split2(float x, uint32_t& hi, uint32_t& lo) {
    hi = bf16_bits(x);
    lo = bf16_bits(x - bf16_value(hi));
}

__device__ inline uint32_t fp16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ inline float fp16_value(uint32_t bits) { return (float)__builtin_bit_cast(_Float16, (uint16_t)bits); }

// Split x into hi/lo fp16 bit patterns, each rounded to nearest even (the
// difference x - hi is exact in fp32).
__device__ inline void split2_f16(float x, uint32_t& hi, uint32_t& lo) {
    hi = fp16_bits(x);
    lo = fp16_bits(x - fp16_value(hi));
}

// Eight values -> one 16-byte chunk of the hi plane and one of the lo plane
// (bf16, or fp16 when F16).
template <bool F16 = false>
__device__ inline void split_pack8(const float* x, uint4& hi, uint4& lo) {
    uint32_t h[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if constexpr (F16)
            split2_f16(x[e], h[e], l[e]);
        else
            split2(x[e], h[e], l[e]);
    }
    hi = make_uint4(h[0] | h[1] << 16, h[2] | h[3] << 16, h[4] | h[5] << 16, h[6] | h[7] << 16);
    lo = make_uint4(l[0] | l[1] << 16, l[2] | l[3] << 16, l[4] | l[5] << 16, l[6] | l[7] << 16);
}

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// One 32x32x16 MFMA step; the 16-byte operands hold bf16 or (F16) fp16 values.
template <bool F16>
__device__ inline f32x16 mfma32x32x16(bf16x8 a, bf16x8 b, f32x16 c) {
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

template <int BM, int BN, int WM, int WN, int MODE>
struct Bf16Tile {
    static constexpr int NT = WM * WN * 64;
    static constexpr int FM = BM / WM / 32, FN = BN / WN / 32;
    static constexpr int NP = (MODE == 1 || MODE == 3 || MODE == 5) ? 1 : 2;  // planes per operand (hi, lo)
    static constexpr bool kPlanes = MODE >= 2 && MODE <= 4;                   // operands arrive as k-tiled planes
    static constexpr bool kRow16 = MODE == 1 || MODE == 5;                    // 16-bit row-major operands
    static_assert(FM >= 1 && FN >= 1, "bad tile");
    static constexpr int kBK = kBf16BK, kLd = kBf16Ld;

    struct Smem {
        uint16_t As[2][NP][BM][kLd];
        uint16_t Bs[2][NP][BN][kLd];
    };

    // Row / column (within the tile) of accumulator element (a, b, i) of this thread.
    __device__ static int acc_row(int a, int i) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        return (wave / WN) * FM * 32 + a * 32 + (i / 4) * 8 + (lane >> 5) * 4 + (i % 4);
    }
    __device__ static int acc_col(int b) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        return (wave % WN) * FN * 32 + b * 32 + (lane & 31);
    }

    // acc = A[row0:row0+BM, kb:ke] * B[kb:ke, col0:col0+BN] (fp32 accumulation;
    // out-of-range rows/cols/k read as zero).  Av/Bv are fp32 (MODE 0) or
    // bf16 (MODE 1), row-major.  Ends with a barrier, so sm may be reused.
    // ALIGNED: every row start (and so every 16-byte chunk) is 16-byte aligned,
    // so chunks load with one vector load; otherwise through load16_any.
    template <bool ALIGNED>
    __device__ static void compute(Smem& sm, const void* __restrict__ Av, int64_t lda, const void* __restrict__ Bv,
                                   int64_t ldb, int64_t m, int64_t n, int64_t row0, int64_t col0, int64_t kb,
                                   int64_t ke, int vec_ok, f32x16 (&acc)[FM][FN], int64_t a_plane = 0,
                                   int64_t b_plane = 0) {
        auto& As = sm.As;
        auto& Bs = sm.Bs;
        const int tid = threadIdx.x;
        const int lane = tid & 63, wave = tid >> 6;
        const int wm = wave / WN, wn = wave % WN;
        const int lrow = lane & 31, half = lane >> 5;
        const gptr<const float> Af = (gptr<const float>)Av;
        const gptr<const float> Bf = (gptr<const float>)Bv;
        const gptr<const uint16_t> Ah = (gptr<const uint16_t>)Av;
        const gptr<const uint16_t> Bh = (gptr<const uint16_t>)Bv;
    #pragma unroll
        for (int a = 0; a < FM; ++a)
    #pragma unroll
            for (int b = 0; b < FN; ++b)
    #pragma unroll
                for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.0f;

        const bool rows_full = row0 + BM <= m;
        const bool cols_full = col0 + BN <= n;

        // ---- staging registers
        // MODE 0: A as float4 chunks (4 k of one row); B as pairs of float4
        //         (rows k, k+1; 4 columns), packed into k-pair words in LDS.
        // MODE 1: A as 8-bf16 chunks; B as pairs of 8-bf16 rows.
        constexpr int AW = MODE == 0 ? 4 : 8;  // elements per A chunk
        constexpr int BW = MODE == 0 ? 4 : 8;  // columns per B pair (MODE 0/1)
        constexpr int A_TOT = BM * kBK / AW;
        constexpr int B_TOT = kPlanes ? BN * kBK / 8 : BN * kBK / (2 * BW);
        constexpr int A_CH = (A_TOT + NT - 1) / NT, B_CH = (B_TOT + NT - 1) / NT;
        float ra[MODE == 0 ? A_CH : 1][4];
        float rb[MODE == 0 ? B_CH : 1][2][4];
        uint4 ha[kRow16 ? A_CH : 1];
        uint4 hb[kRow16 ? B_CH : 1][2];
        uint4 pa[kPlanes ? NP : 1][kPlanes ? A_CH : 1];  // MODE 2/3: A planes
        uint4 pb[kPlanes ? NP : 1][kPlanes ? B_CH : 1];  // MODE 2/3: B^T planes

        // MODE 2/3: one 16-byte chunk (8 k values) of a k-tiled plane, zero
        // for rows >= rows_lim.  No k check: plane rows are zero from k to
        // their length (a multiple of 32), and slice ends other than k fall
        // on 32-deep tile boundaries, so a staged k-tile never reads values
        // of another slice.
        auto load_plane = [&](gptr<const uint16_t> base, int64_t ld, int64_t row, int64_t rows_lim, int64_t gk,
                              bool fast) -> uint4 {
            // gk is a multiple of 8: the chunk is one 16-byte slot
            if (!fast && row >= rows_lim) return make_uint4(0u, 0u, 0u, 0u);
            const gptr<const uint16_t> q = base + tiled_off(row, gk, ld);
            return ALIGNED ? ld16(q) : load16_any(q);
        };

        // FAST: the whole tile is inside the matrices (interior tile, full
        // k-tile), so every chunk is loaded without a bounds check.
        auto load_tiles = [&](int64_t k0, auto fast_tag) {
            constexpr bool FAST = decltype(fast_tag)::value;
            const bool k_full = FAST || k0 + kBK <= ke;
            if constexpr (kPlanes) {
#pragma unroll
                for (int p = 0; p < NP; ++p) {
#pragma unroll
                    for (int c = 0; c < A_CH; ++c) {
                        const int idx = tid + c * NT;
                        if (A_TOT % NT != 0 && idx >= A_TOT) break;
                        const int r = idx / (kBK / 8), kc = (idx % (kBK / 8)) * 8;
                        const bool fast = FAST || (vec_ok && k_full && (rows_full || row0 + r < m));
                        pa[p][c] = load_plane(Ah + p * a_plane, lda, row0 + r, m, k0 + kc, fast);
                    }
#pragma unroll
                    for (int c = 0; c < B_CH; ++c) {
                        const int idx = tid + c * NT;
                        if (B_TOT % NT != 0 && idx >= B_TOT) break;
                        const int r = idx / (kBK / 8), kc = (idx % (kBK / 8)) * 8;
                        const bool fast = FAST || (vec_ok && k_full && (cols_full || col0 + r < n));
                        pb[p][c] = load_plane(Bh + p * b_plane, ldb, col0 + r, n, k0 + kc, fast);
                    }
                }
            } else {
    #pragma unroll
            for (int c = 0; c < A_CH; ++c) {
                const int idx = tid + c * NT;
                if (A_TOT % NT != 0 && idx >= A_TOT) break;
                const int r = idx / (kBK / AW), kc = (idx % (kBK / AW)) * AW;
                const int64_t gr = row0 + r, gk = k0 + kc;
                const bool fast = FAST || (vec_ok && k_full && (rows_full || gr < m));
                if constexpr (MODE == 0) {
                    if (fast) {
                        const uint4 v = ALIGNED ? ld16(Af + gr * lda + gk)
                                                : load16_any(Af + gr * lda + gk);
                        ra[c][0] = __builtin_bit_cast(float, v.x); ra[c][1] = __builtin_bit_cast(float, v.y);
                        ra[c][2] = __builtin_bit_cast(float, v.z); ra[c][3] = __builtin_bit_cast(float, v.w);
                    } else {
    #pragma unroll
                        for (int e = 0; e < 4; ++e) ra[c][e] = (gr < m && gk + e < ke) ? Af[gr * lda + gk + e] : 0.0f;
                    }
                } else {
                    if (fast) {
                        ha[c] = ALIGNED ? ld16(Ah + gr * lda + gk)
                                        : load16_any(Ah + gr * lda + gk);
                    } else {
                        uint16_t v[8];
    #pragma unroll
                        for (int e = 0; e < 8; ++e) v[e] = (gr < m && gk + e < ke) ? Ah[gr * lda + gk + e] : (uint16_t)0;
                        ha[c] = make_uint4(v[0] | (uint32_t)v[1] << 16, v[2] | (uint32_t)v[3] << 16,
                                           v[4] | (uint32_t)v[5] << 16, v[6] | (uint32_t)v[7] << 16);
                    }
                }
            }
    #pragma unroll
            for (int c = 0; c < B_CH; ++c) {
                const int idx = tid + c * NT;
                if (B_TOT % NT != 0 && idx >= B_TOT) break;
                const int kp = idx % (kBK / 2), nc = (idx / (kBK / 2)) * BW;
                const int64_t gk = k0 + 2 * kp, gc = col0 + nc;
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int64_t kk = gk + h;
                    const bool fast = FAST || (vec_ok && cols_full && kk < ke);
                    if constexpr (MODE == 0) {
                        if (fast) {
                            const uint4 v = ALIGNED ? ld16(Bf + kk * ldb + gc)
                                                    : load16_any(Bf + kk * ldb + gc);
                            rb[c][h][0] = __builtin_bit_cast(float, v.x); rb[c][h][1] = __builtin_bit_cast(float, v.y);
                            rb[c][h][2] = __builtin_bit_cast(float, v.z); rb[c][h][3] = __builtin_bit_cast(float, v.w);
                        } else {
    #pragma unroll
                            for (int e = 0; e < 4; ++e)
                                rb[c][h][e] = (kk < ke && gc + e < n) ? Bf[kk * ldb + gc + e] : 0.0f;
                        }
                    } else {
                        if (fast) {
                            hb[c][h] = ALIGNED ? ld16(Bh + kk * ldb + gc)
                                               : load16_any(Bh + kk * ldb + gc);
                        } else {
                            uint16_t v[8];
    #pragma unroll
                            for (int e = 0; e < 8; ++e)
                                v[e] = (kk < ke && gc + e < n) ? Bh[kk * ldb + gc + e] : (uint16_t)0;
                            hb[c][h] = make_uint4(v[0] | (uint32_t)v[1] << 16, v[2] | (uint32_t)v[3] << 16,
                                                  v[4] | (uint32_t)v[5] << 16, v[6] | (uint32_t)v[7] << 16);
                        }
                    }
                }
            }
            }
        };

        auto store_tiles = [&](int buf) {
            if constexpr (kPlanes) {
#pragma unroll
                for (int p = 0; p < NP; ++p) {
#pragma unroll
                    for (int c = 0; c < A_CH; ++c) {
                        const int idx = tid + c * NT;
                        if (A_TOT % NT != 0 && idx >= A_TOT) break;
                        *reinterpret_cast<uint4*>(&As[buf][p][idx / (kBK / 8)][(idx % (kBK / 8)) * 8]) = pa[p][c];
                    }
#pragma unroll
                    for (int c = 0; c < B_CH; ++c) {
                        const int idx = tid + c * NT;
                        if (B_TOT % NT != 0 && idx >= B_TOT) break;
                        *reinterpret_cast<uint4*>(&Bs[buf][p][idx / (kBK / 8)][(idx % (kBK / 8)) * 8]) = pb[p][c];
                    }
                }
            } else {
    #pragma unroll
            for (int c = 0; c < A_CH; ++c) {
                const int idx = tid + c * NT;
                if (A_TOT % NT != 0 && idx >= A_TOT) break;
                const int r = idx / (kBK / AW), kc = (idx % (kBK / AW)) * AW;
                if constexpr (MODE == 0) {
                    uint32_t h[4], l[4];
    #pragma unroll
                    for (int e = 0; e < 4; ++e) split2(ra[c][e], h[e], l[e]);
                    *reinterpret_cast<uint2*>(&As[buf][0][r][kc]) = make_uint2(h[0] | h[1] << 16, h[2] | h[3] << 16);
                    *reinterpret_cast<uint2*>(&As[buf][1][r][kc]) = make_uint2(l[0] | l[1] << 16, l[2] | l[3] << 16);
                } else {
                    *reinterpret_cast<uint4*>(&As[buf][0][r][kc]) = ha[c];
                }
            }
    #pragma unroll
            for (int c = 0; c < B_CH; ++c) {
                const int idx = tid + c * NT;
                if (B_TOT % NT != 0 && idx >= B_TOT) break;
                const int kp = idx % (kBK / 2), nc = (idx / (kBK / 2)) * BW;
                if constexpr (MODE == 0) {
    #pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        uint32_t h0, l0, h1, l1;
                        split2(rb[c][0][e], h0, l0);
                        split2(rb[c][1][e], h1, l1);
                        *reinterpret_cast<uint32_t*>(&Bs[buf][0][nc + e][2 * kp]) = h0 | h1 << 16;
                        *reinterpret_cast<uint32_t*>(&Bs[buf][1][nc + e][2 * kp]) = l0 | l1 << 16;
                    }
                } else {
                    const uint32_t w0[4] = {hb[c][0].x, hb[c][0].y, hb[c][0].z, hb[c][0].w};
                    const uint32_t w1[4] = {hb[c][1].x, hb[c][1].y, hb[c][1].z, hb[c][1].w};
    #pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const uint32_t lo16 = (w0[e / 2] >> (16 * (e % 2))) & 0xffffu;
                        const uint32_t hi16 = (w1[e / 2] >> (16 * (e % 2))) & 0xffffu;
                        *reinterpret_cast<uint32_t*>(&Bs[buf][0][nc + e][2 * kp]) = lo16 | hi16 << 16;
                    }
                }
            }
            }
        };

        auto mfma_step = [&](int buf, int ks) {
            bf16x8 a[NP][FM], b[NP][FN];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    a[p][i] = *reinterpret_cast<const bf16x8*>(&As[buf][p][wm * FM * 32 + i * 32 + lrow][ks + 8 * half]);
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[p][j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][p][wn * FN * 32 + j * 32 + lrow][ks + 8 * half]);
            }
            constexpr bool F16 = MODE == 4 || MODE == 5;
            if constexpr (NP == 2) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = mfma32x32x16<F16>(a[0][i], b[1][j], acc[i][j]);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = mfma32x32x16<F16>(a[1][i], b[0][j], acc[i][j]);
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma32x32x16<F16>(a[0][i], b[0][j], acc[i][j]);
        };

        // One pipelined iteration: prefetch k-tile kt+1 into registers, run the
        // two 16-deep MFMA steps of k-tile kt from LDS, stage k-tile kt+1 into
        // the other LDS buffer, barrier.
        auto iteration = [&](int64_t kt, auto fast_tag) {
            const int buf = (int)(kt & 1);
            load_tiles(kb + (kt + 1) * kBK, fast_tag);
            mfma_step(buf, 0);
            mfma_step(buf, 16);
            // Keep the staging of the next tile (which waits for its global
            // loads) after this tile's MFMAs: nothing is scheduled across.
            __builtin_amdgcn_sched_barrier(0);
            store_tiles(buf ^ 1);
            __syncthreads();
        };

        const int64_t nkt = (ke - kb + kBK - 1) / kBK;
        const int64_t nfull = (ke - kb) / kBK;  // k-tiles with all kBK columns
        if (nkt > 0 && MODE == 0) {
            // In-kernel split: conditional prefetch / staging blocks keep the
            // split's VALU work after the MFMAs of the current tile.
            load_tiles(kb, std::false_type{});
            store_tiles(0);
            __syncthreads();
            for (int64_t kt = 0; kt < nkt; ++kt) {
                const int buf = (int)(kt & 1);
                if (kt + 1 < nkt) load_tiles(kb + (kt + 1) * kBK, std::false_type{});
                mfma_step(buf, 0);
                mfma_step(buf, 16);
                if (kt + 1 < nkt) store_tiles(buf ^ 1);
                __syncthreads();
            }
        } else if (nkt > 0) {
            load_tiles(kb, std::false_type{});
            store_tiles(0);
            __syncthreads();
            int64_t kt = 0;
            // k-tiles 1..nfull-1 are full: interior tiles prefetch them unchecked
            if (MODE != 0 && rows_full && cols_full && vec_ok) {
                for (; kt + 1 < nfull; ++kt) iteration(kt, std::true_type{});
            }
            for (; kt + 1 < nkt; ++kt) iteration(kt, std::false_type{});
            mfma_step((int)(kt & 1), 0);
            mfma_step((int)(kt & 1), 16);
            __syncthreads();
        }
    }
};

}  // namespace starmm
