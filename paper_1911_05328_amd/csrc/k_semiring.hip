// Integer-semiring tile kernel ((min,+), (max,+), (max, min), Boolean): the
// base case of the flattened 8-way recursion (eq. mm-dac) on the vector
// ALUs, plus the ordered madd that merges k-slice temporaries (Fig. mm-n3,
// line "madd"; Sec. sar-mm).
//
// Exactness: (min,+) entries lie in [0, 2^30] (2^30 = +INF), so a + b <= 2^31
// fits in uint32; the accumulator starts at INF, so min(INF, sums) is already
// the saturated result.  (max,+) mirrors this in int32 on [-2^30, 0].  Masked
// (out-of-range) operands load the semiring zero, which annihilates under
// (x) and is neutral under (+).  (max, min) needs no domain: min and max
// of int32 stay int32, and INT32_MIN is its zero.  Boolean works on 0/1 with
// bitwise and / or.
//
// Checked range (MM_FLAG_CHECKED_RANGE, and every 128 tile): (min,+) entries may be negative,
// anywhere in [-2^30, 2^30].  An operand is moved into an unsigned domain as
// it is loaded: x + 2^30, with INF mapped to 0xffffffff, so a product is one
// saturating add (an INF operand saturates whatever its partner, and finite
// sums, x + y + 2^31, stay below 2^32) and (+) is still an unsigned min.  The
// result goes back as the sum minus 2^31, INF when it reaches 2^30.  (max,+)
// runs the same on negated operands (entries in [-2^30, 2^30 - 1], -2^30 =
// -INF).  Partial results, temporaries and C always hold the caller's values;
// only the inner loop sees the shifted domain.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.hpp"
#include "kcommon.hpp"

namespace starmm {

namespace {

// Kernel kinds beyond mm_semiring_kind: the checked-range variants.
constexpr int kMinPlusChecked = 101, kMaxPlusChecked = 102;

// Each semiring: the inner loop's type T, its zero, (x), (+), and the moves
// between the caller's int32 values and T (in: operands as loaded; out: the
// accumulator when the slice is done).  merge / atomic_plus / zero_out are
// (+) and its zero on the caller's values (temporaries, slots, C).
template <int SR>
struct Sem;

// Where T holds the caller's values unchanged.
template <class D, class TT>
struct SemSameDomain {
    using T = TT;
    __device__ static T in(int32_t x) { return (T)x; }
    __device__ static int32_t out(T x) { return (int32_t)x; }
    __device__ static int32_t merge(int32_t a, int32_t b) { return (int32_t)D::plus((T)a, (T)b); }
};

// (min,+) on uint32 bit patterns.
template <>
struct Sem<MM_SR_MIN_PLUS> : SemSameDomain<Sem<MM_SR_MIN_PLUS>, uint32_t> {
    static constexpr uint32_t zero = 1u << 30;
    static constexpr int32_t zero_out = 1 << 30;
    // a + b <= 2^31 never saturates here; the clamped add measured faster
    // than the plain one in the 32 and 64 tiles
    __device__ static T times(T a, T b) { return __builtin_elementwise_add_sat(a, b); }
    __device__ static T plus(T a, T b) { return a < b ? a : b; }
    __device__ static T plus3(T a, T b, T c) { return plus(plus(a, b), c); }
    __device__ static void atomic_plus(int32_t* p, int32_t v) {
        atomicMin(reinterpret_cast<unsigned int*>(p), (unsigned int)v);
    }
};

// (max,+) on int32.
template <>
struct Sem<MM_SR_MAX_PLUS> : SemSameDomain<Sem<MM_SR_MAX_PLUS>, int32_t> {
    static constexpr int32_t zero = -(1 << 30);
    static constexpr int32_t zero_out = -(1 << 30);
    __device__ static T times(T a, T b) { return a + b; }
    __device__ static T plus(T a, T b) { return a > b ? a : b; }
    __device__ static T plus3(T a, T b, T c) { return plus(plus(a, b), c); }
    __device__ static void atomic_plus(int32_t* p, int32_t v) { atomicMax(p, v); }
};

// (max, min) on int32.
template <>
struct Sem<MM_SR_MAX_MIN> : SemSameDomain<Sem<MM_SR_MAX_MIN>, int32_t> {
    static constexpr int32_t zero = INT32_MIN;
    static constexpr int32_t zero_out = INT32_MIN;
    __device__ static T times(T a, T b) { return a < b ? a : b; }
    __device__ static T plus(T a, T b) { return a > b ? a : b; }
    __device__ static T plus3(T a, T b, T c) { return plus(plus(a, b), c); }
    __device__ static void atomic_plus(int32_t* p, int32_t v) { atomicMax(p, v); }
};

// Boolean (or, and) on 0/1.
template <>
struct Sem<MM_SR_OR_AND> : SemSameDomain<Sem<MM_SR_OR_AND>, uint32_t> {
    static constexpr uint32_t zero = 0u;
    static constexpr int32_t zero_out = 0;
    __device__ static T times(T a, T b) { return a & b; }
    __device__ static T plus(T a, T b) { return a | b; }
    __device__ static T plus3(T a, T b, T c) { return a | b | c; }
    __device__ static void atomic_plus(int32_t* p, int32_t v) {
        atomicOr(reinterpret_cast<unsigned int*>(p), (unsigned int)v);
    }
};

// Checked (min,+) / (max,+): the shifted unsigned domain of the file header;
// NEG negates operands and result ((max,+) as (min,+) of the negations).
template <bool NEG>
struct SemShifted {
    using T = uint32_t;
    static constexpr int32_t kInf = 1 << 30;
    static constexpr uint32_t zero = 0xffffffffu;
    static constexpr int32_t zero_out = NEG ? -kInf : kInf;
    // (negation in unsigned arithmetic: inputs outside the domain then give
    // unspecified values rather than signed overflow)
    __device__ static T in(int32_t x) {
        const int32_t y = NEG ? (int32_t)(0u - (uint32_t)x) : x;
        return y >= kInf ? zero : (uint32_t)y + (uint32_t)kInf;
    }
    __device__ static int32_t out(T acc) {
        if (acc >= 0xc0000000u) return zero_out;  // sum >= INF, or an INF operand
        const uint32_t r = acc ^ 0x80000000u;      // acc - 2^31
        return (int32_t)(NEG ? 0u - r : r);
    }
    __device__ static T times(T a, T b) { return __builtin_elementwise_add_sat(a, b); }
    __device__ static T plus(T a, T b) { return a < b ? a : b; }
    __device__ static T plus3(T a, T b, T c) { return plus(plus(a, b), c); }
    __device__ static int32_t merge(int32_t a, int32_t b) { return NEG ? (a > b ? a : b) : (a < b ? a : b); }
    __device__ static void atomic_plus(int32_t* p, int32_t v) {
        if (NEG)
            atomicMax(p, v);
        else
            atomicMin(p, v);
    }
};

template <>
struct Sem<kMinPlusChecked> : SemShifted<false> {};
template <>
struct Sem<kMaxPlusChecked> : SemShifted<true> {};

constexpr int kBK = 16;

// One workgroup = one base-case output tile of BM x BN for one k-slice.
// Thread (ty, tx) owns TM x TN outputs: TM/4 groups of 4 rows spaced BM/(TM/4)
// apart, and likewise for columns, so LDS reads are 16-byte vectors that are
// broadcast (A) or contiguous (B) across a wavefront.
template <int SR, int BM, int BN, int TM, int TN, int KU>
struct SemTile {
    using S = Sem<SR>;
    using T = typename S::T;
    static constexpr int NTX = BN / TN, NTY = BM / TM, NT = NTX * NTY;
    static constexpr int GM = TM / 4, GN = TN / 4;      // 4-row / 4-column groups per thread
    static constexpr int SM = BM / GM, SN = BN / GN;    // spacing between groups
    static constexpr int A_CHUNKS = BM * kBK / 4 / NT;  // int4 chunks of the A tile per thread
    static constexpr int B_CHUNKS = BN * kBK / 4 / NT;
    static_assert(A_CHUNKS >= 1 && B_CHUNKS >= 1, "tile too small for the thread count");
    static_assert((TM * TN) % 4 == 0, "outputs per thread in whole 16-byte vectors");

    struct Smem {
        T As[2][kBK][BM];
        T Bs[2][kBK][BN];
    };

    // Row / column (within the tile) of this thread's output (i, j).
    __device__ static int out_row(int i) { return (i / 4) * SM + (int)(threadIdx.x / NTX) * 4 + (i % 4); }
    __device__ static int out_col(int j) { return (j / 4) * SN + (int)(threadIdx.x % NTX) * 4 + (j % 4); }

    // acc <- (+)_{l in [kb, ke)} A[row0 + i, l] (x) B[l, col0 + j] for this
    // thread's outputs, returned as the caller's int32 values (bit patterns
    // in T).  Out-of-range operands load the semiring zero.  Ends with a
    // barrier, so sm may be reused.
    __device__ static void compute(Smem& sm, const int32_t* __restrict__ A, int64_t lda,
                                   const int32_t* __restrict__ B, int64_t ldb, int64_t m, int64_t n, int64_t row0,
                                   int64_t col0, int64_t kb, int64_t ke, int vec_ok, T (&acc)[TM][TN]) {
        const int tid = threadIdx.x;
        const int tx = tid % NTX, ty = tid / NTX;
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = S::zero;

        const bool rows_full = row0 + BM <= m;
        const bool cols_full = col0 + BN <= n;
        T ra[A_CHUNKS][4], rb[B_CHUNKS][4];

        auto load_tiles = [&](int64_t k0) {
            const bool k_full = k0 + kBK <= ke;
#pragma unroll
            for (int c = 0; c < A_CHUNKS; ++c) {
                const int idx = tid + c * NT;
                const int r = idx / (kBK / 4), kc = (idx % (kBK / 4)) * 4;
                const int64_t gr = row0 + r, gk = k0 + kc;
                if (vec_ok && k_full && (rows_full || gr < m)) {
                    const int4 v = *reinterpret_cast<const int4*>(A + gr * lda + gk);
                    ra[c][0] = S::in(v.x); ra[c][1] = S::in(v.y); ra[c][2] = S::in(v.z); ra[c][3] = S::in(v.w);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        ra[c][e] = (gr < m && gk + e < ke) ? S::in(A[gr * lda + gk + e]) : S::zero;
                }
            }
#pragma unroll
            for (int c = 0; c < B_CHUNKS; ++c) {
                const int idx = tid + c * NT;
                const int r = idx / (BN / 4), nc = (idx % (BN / 4)) * 4;
                const int64_t gk = k0 + r, gc = col0 + nc;
                if (vec_ok && cols_full && gk < ke) {
                    const int4 v = *reinterpret_cast<const int4*>(B + gk * ldb + gc);
                    rb[c][0] = S::in(v.x); rb[c][1] = S::in(v.y); rb[c][2] = S::in(v.z); rb[c][3] = S::in(v.w);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rb[c][e] = (gk < ke && gc + e < n) ? S::in(B[gk * ldb + gc + e]) : S::zero;
                }
            }
        };
        auto store_tiles = [&](int buf) {
#pragma unroll
            for (int c = 0; c < A_CHUNKS; ++c) {
                const int idx = tid + c * NT;
                const int r = idx / (kBK / 4), kc = (idx % (kBK / 4)) * 4;
#pragma unroll
                for (int e = 0; e < 4; ++e) sm.As[buf][kc + e][r] = ra[c][e];
            }
#pragma unroll
            for (int c = 0; c < B_CHUNKS; ++c) {
                const int idx = tid + c * NT;
                const int r = idx / (BN / 4), nc = (idx % (BN / 4)) * 4;
                *reinterpret_cast<uint4*>(&sm.Bs[buf][r][nc]) =
                    make_uint4((uint32_t)rb[c][0], (uint32_t)rb[c][1], (uint32_t)rb[c][2], (uint32_t)rb[c][3]);
            }
        };

        const int64_t nkt = (ke - kb + kBK - 1) / kBK;
        if (nkt > 0) {
            load_tiles(kb);
            store_tiles(0);
            __syncthreads();
            for (int64_t kt = 0; kt < nkt; ++kt) {
                const int buf = (int)(kt & 1);
                if (kt + 1 < nkt) load_tiles(kb + (kt + 1) * kBK);
                // KU k-pairs unrolled: bounds how many LDS operands are in flight
#pragma unroll KU
                for (int kk = 0; kk < kBK; kk += 2) {
                    T a0[TM], a1[TM], b0[TN], b1[TN];
#pragma unroll
                    for (int g = 0; g < GM; ++g) {
                        const uint4 x0 = *reinterpret_cast<const uint4*>(&sm.As[buf][kk][g * SM + ty * 4]);
                        const uint4 x1 = *reinterpret_cast<const uint4*>(&sm.As[buf][kk + 1][g * SM + ty * 4]);
                        a0[g * 4 + 0] = (T)x0.x; a0[g * 4 + 1] = (T)x0.y; a0[g * 4 + 2] = (T)x0.z; a0[g * 4 + 3] = (T)x0.w;
                        a1[g * 4 + 0] = (T)x1.x; a1[g * 4 + 1] = (T)x1.y; a1[g * 4 + 2] = (T)x1.z; a1[g * 4 + 3] = (T)x1.w;
                    }
#pragma unroll
                    for (int g = 0; g < GN; ++g) {
                        const uint4 y0 = *reinterpret_cast<const uint4*>(&sm.Bs[buf][kk][g * SN + tx * 4]);
                        const uint4 y1 = *reinterpret_cast<const uint4*>(&sm.Bs[buf][kk + 1][g * SN + tx * 4]);
                        b0[g * 4 + 0] = (T)y0.x; b0[g * 4 + 1] = (T)y0.y; b0[g * 4 + 2] = (T)y0.z; b0[g * 4 + 3] = (T)y0.w;
                        b1[g * 4 + 0] = (T)y1.x; b1[g * 4 + 1] = (T)y1.y; b1[g * 4 + 2] = (T)y1.z; b1[g * 4 + 3] = (T)y1.w;
                    }
#pragma unroll
                    for (int i = 0; i < TM; ++i)
#pragma unroll
                        for (int j = 0; j < TN; ++j)
                            acc[i][j] = S::plus3(acc[i][j], S::times(a0[i], b0[j]), S::times(a1[i], b1[j]));
                }
                if (kt + 1 < nkt) store_tiles(buf ^ 1);
                __syncthreads();
            }
        }
        // back to the caller's values (a no-op where the domains agree)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = (T)S::out(acc[i][j]);
    }
};

template <int SR, int BM, int BN, int TM, int TN, int KU>
__global__ void __launch_bounds__((BM / TM) * (BN / TN))
k_semiring_tile(const int32_t* __restrict__ A, int64_t lda, const int32_t* __restrict__ B, int64_t ldb,
                int32_t* __restrict__ C, int64_t ldc, int32_t* __restrict__ temps, int64_t m, int64_t n,
                int64_t k, int64_t tiles_m, int64_t tiles_n, SliceArgs sa, int vec_ok) {
    using Tile = SemTile<SR, BM, BN, TM, TN, KU>;
    using S = typename Tile::S;
    using T = typename Tile::T;
    __shared__ __attribute__((aligned(16))) typename Tile::Smem sm;

    const int64_t tiles = tiles_m * tiles_n;
    const int64_t logical = xcd_logical_id(blockIdx.x, (int64_t)gridDim.x);
    const int sigma = (int)(logical / tiles);
    int64_t ti, tj;
    recursion_tile(logical % tiles, tiles_m, tiles_n, &ti, &tj);
    const int64_t row0 = ti * BM, col0 = tj * BN;
    int64_t kb, ke;
    slice_k_range(sigma, sa.levels, k, sa.tk, &kb, &ke);

    T acc[TM][TN];
    Tile::compute(sm, A, lda, B, ldb, m, n, row0, col0, kb, ke, vec_ok, acc);

    // Epilogue: slice index sigma = (TAR group g, SAR index r).  r == 0 keeps
    // the parent's storage (C); r > 0 writes its own temporary.
    const int r_sar = sigma & ((1 << sa.sar_levels) - 1);
    const int g_tar = sigma >> sa.sar_levels;
    const int per_group = (1 << sa.sar_levels) - 1;
    int32_t* dst;
    int64_t ldd;
    if (r_sar == 0) {
        dst = C;
        ldd = ldc;
    } else {
        dst = temps + (int64_t)(g_tar * per_group + r_sar - 1) * sa.temp_stride;
        ldd = sa.ldt;
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int64_t gr = row0 + Tile::out_row(i);
        if (gr >= m) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t gc = col0 + Tile::out_col(j);
            if (gc >= n) continue;
            int32_t* p = dst + gr * ldd + gc;
            if (r_sar != 0) {
                *p = (int32_t)acc[i][j];
            } else if (sa.atomic_c) {
                S::atomic_plus(p, (int32_t)acc[i][j]);
            } else {
                *p = S::merge(*p, (int32_t)acc[i][j]);
            }
        }
    }
}

// ---- persistent launch with a ring of slot groups (MM_FLAG_PERSISTENT)
//
// Items (tile, slice) are handed out in order by a device counter, tile-major
// in the recursion's tile order.  Tile t's slices write their partial
// results into slot group t mod G; the slice that arrives last (per-tile
// arrival count, in place of SAR's trylock) merges C (+)= D_0 (+) ... (+)
// D_{s-1} in slice order and passes the group to tile t + G.  A slice waits
// only while its group still belongs to tile t - G.  Every wait ends: items
// are handed out only to running workgroups, in order, so the oldest
// unmerged tile has all its slices on running workgroups and its group
// free.  The wait is still bounded (by a spin count the host scales with
// the k-depth of a slice, the longest a slice of the previous owner can still
// take); a workgroup that exceeds the bound sets the error word and leaves,
// the others then leave too, and mm_persistent_status() reports the call as
// incomplete.
struct PersistCtl {
    unsigned long long next;  // next item
    uint32_t error;           // nonzero: some wait exceeded its bound (C incomplete)
    uint32_t pad;
};

// Spins of a bounded wait: a base of ~1 s of s_sleep(8) steps, plus 256
// steps (tens of microseconds) for every k-tile of the deepest slice.
constexpr uint64_t kPersistSpinBase = uint64_t(1) << 22;
constexpr uint64_t kPersistSpinPerKTile = 256;

__global__ void __launch_bounds__(256)
k_persist_init(PersistCtl* __restrict__ ctl, unsigned long long* __restrict__ owner, uint32_t* __restrict__ arrive,
               int64_t groups) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0) {
        ctl->next = 0ull;
        ctl->error = 0u;
    }
    if (i < groups) {
        owner[i] = (unsigned long long)i;
        arrive[i] = 0u;
    }
}

template <int SR, int BM, int BN, int TM, int TN, int KU>
__global__ void __launch_bounds__((BM / TM) * (BN / TN), BM == 128 ? 3 : 1)
k_semiring_persist(const int32_t* __restrict__ A, int64_t lda, const int32_t* __restrict__ B, int64_t ldb,
                   int32_t* __restrict__ C, int64_t ldc, int64_t m, int64_t n, int64_t k, int64_t tiles_m,
                   int64_t tiles_n, int levels, int64_t groups, PersistCtl* __restrict__ ctl,
                   unsigned long long* __restrict__ owner, uint32_t* __restrict__ arrive,
                   int32_t* __restrict__ slots, int vec_ok, uint64_t spin_limit) {
    using Tile = SemTile<SR, BM, BN, TM, TN, KU>;
    using S = typename Tile::S;
    using T = typename Tile::T;
    constexpr int NT = Tile::NT;
    constexpr int64_t kSlot = (int64_t)BM * BN;
    __shared__ __attribute__((aligned(16))) typename Tile::Smem sm;
    __shared__ unsigned long long s_item;
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    const int64_t ns = int64_t(1) << levels;
    const int64_t total = tiles_m * tiles_n * ns;

    for (;;) {
        if (tid == 0) s_item = atomicAdd(&ctl->next, 1ull);
        __syncthreads();
        const int64_t item = (int64_t)s_item;
        __syncthreads();
        if (item >= total) break;
        const int64_t tile = item >> levels;
        const int sigma = (int)(item & (ns - 1));
        int64_t ti, tj;
        recursion_tile(tile, tiles_m, tiles_n, &ti, &tj);
        const int64_t row0 = ti * BM, col0 = tj * BN;
        int64_t kb, ke;
        slice_k_range(sigma, levels, k, kBK, &kb, &ke);

        T acc[TM][TN];
        Tile::compute(sm, A, lda, B, ldb, m, n, row0, col0, kb, ke, vec_ok, acc);

        if (ns > 1) {
            const int64_t g = tile % groups;
            if (tid == 0) {
                uint64_t spins = 0;
                int ok = 1;
                while (__hip_atomic_load(&owner[g], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) !=
                       (unsigned long long)tile) {
                    if (++spins > spin_limit ||
                        __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                        atomicExch(&ctl->error, 1u);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(8);
                }
                s_flag = ok;
            }
            __syncthreads();
            if (!s_flag) break;
            // this slice's partial into its slot: each thread's TM x TN values
            // contiguous, written as 16-byte vectors off one address
            int4* slot = reinterpret_cast<int4*>(slots + (g * ns + sigma) * kSlot + (int64_t)tid * (TM * TN));
#pragma unroll
            for (int v = 0; v < TM * TN / 4; ++v) {
                const int e = 4 * v;
                slot[v] = make_int4((int32_t)acc[e / TN][e % TN], (int32_t)acc[(e + 1) / TN][(e + 1) % TN],
                                    (int32_t)acc[(e + 2) / TN][(e + 2) % TN], (int32_t)acc[(e + 3) / TN][(e + 3) % TN]);
            }
            __threadfence();
            __syncthreads();
            if (tid == 0) s_flag = atomicAdd(&arrive[g], 1u) == (uint32_t)(ns - 1);
            __syncthreads();
            if (!s_flag) continue;
            __threadfence();
            // last slice in: the partials of slices 0 .. s-1, in that order
            const int32_t* base = slots + g * ns * kSlot + (int64_t)tid * (TM * TN);
#pragma unroll
            for (int v = 0; v < TM * TN / 4; ++v) {
                const int4 x = reinterpret_cast<const int4*>(base)[v];
                const int e = 4 * v;
                acc[e / TN][e % TN] = (T)x.x;
                acc[(e + 1) / TN][(e + 1) % TN] = (T)x.y;
                acc[(e + 2) / TN][(e + 2) % TN] = (T)x.z;
                acc[(e + 3) / TN][(e + 3) % TN] = (T)x.w;
            }
            for (int64_t q = 1; q < ns; ++q) {
                const int4* sl = reinterpret_cast<const int4*>(base + q * kSlot);
#pragma unroll
                for (int v = 0; v < TM * TN / 4; ++v) {
                    const int4 x = sl[v];
                    const int e = 4 * v;
                    acc[e / TN][e % TN] = (T)S::merge((int32_t)acc[e / TN][e % TN], x.x);
                    acc[(e + 1) / TN][(e + 1) % TN] = (T)S::merge((int32_t)acc[(e + 1) / TN][(e + 1) % TN], x.y);
                    acc[(e + 2) / TN][(e + 2) % TN] = (T)S::merge((int32_t)acc[(e + 2) / TN][(e + 2) % TN], x.z);
                    acc[(e + 3) / TN][(e + 3) % TN] = (T)S::merge((int32_t)acc[(e + 3) / TN][(e + 3) % TN], x.w);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < TM; ++i) {
            const int64_t gr = row0 + Tile::out_row(i);
            if (gr >= m) continue;
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int64_t gc = col0 + Tile::out_col(j);
                if (gc >= n) continue;
                int32_t* pc = C + gr * ldc + gc;
                *pc = S::merge(*pc, (int32_t)acc[i][j]);
            }
        }
        if (ns > 1) {
            // every thread has read the group's slots: pass it on
            __syncthreads();
            if (tid == 0) {
                const int64_t g = tile % groups;
                atomicExch(&arrive[g], 0u);
                __threadfence();
                __hip_atomic_store(&owner[g], (unsigned long long)(tile + groups), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// madd of the temporaries of one band: per TAR group, C-slot value (C itself
// when SAR-only, else the semiring zero) and the S-1 temporaries are reduced
// in recursion order -- pairs of neighbours first, as the nested madd of each
// recursion level would -- and written to C (atomically with TAR groups).
template <int SR, int NS>
__global__ void __launch_bounds__(256)
k_merge_i32(int32_t* __restrict__ C, int64_t ldc, const int32_t* __restrict__ temps, int64_t m, int64_t n,
            int groups, int atomic_c, int64_t temp_stride, int64_t ldt) {
    using S = Sem<SR>;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * n) return;
    const int64_t i = idx / n, j = idx % n;
    for (int g = 0; g < groups; ++g) {
        int32_t v[NS];
        v[0] = atomic_c ? S::zero_out : C[i * ldc + j];
#pragma unroll
        for (int r = 1; r < NS; ++r) v[r] = temps[(int64_t)(g * (NS - 1) + r - 1) * temp_stride + i * ldt + j];
#pragma unroll
        for (int w = 1; w < NS; w *= 2)
#pragma unroll
            for (int q = 0; q + w < NS; q += 2 * w) v[q] = S::merge(v[q], v[q + w]);
        if (atomic_c)
            S::atomic_plus(&C[i * ldc + j], v[0]);
        else
            C[i * ldc + j] = v[0];
    }
}

template <int SR, int BM, int BN, int TM, int TN, int KU>
hipError_t launch_tile_cfg(const Plan& p, int64_t m, int64_t n, int64_t k, const int32_t* A, int64_t lda,
                           const int32_t* B, int64_t ldb, int32_t* C, int64_t ldc, int32_t* temps,
                           hipStream_t st) {
    const mm_plan_info& pi = p.info;
    SliceArgs sa;
    sa.levels = pi.tar_levels + pi.sar_levels;
    sa.sar_levels = pi.sar_levels;
    sa.tk = kBK;
    sa.atomic_c = pi.tar_levels > 0;
    sa.temp_stride = p.temp_stride;
    sa.ldt = p.ldt;
    const int64_t tiles_m = ceil_div(m, BM), tiles_n = ceil_div(n, BN);
    const int64_t grid = tiles_m * tiles_n * pi.sched.split_k;
    if (grid == 0) return hipSuccess;
    const int vec_ok = (lda % 4 == 0) && (ldb % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
    ProfScope ps("semiring_tile", st);
    hipLaunchKernelGGL((k_semiring_tile<SR, BM, BN, TM, TN, KU>), dim3((unsigned)grid), dim3((BM / TM) * (BN / TN)),
                       0, st, A, lda, B, ldb, C, ldc, temps, m, n, k, tiles_m, tiles_n, sa, vec_ok);
    return hipGetLastError();
}

template <int SR>
hipError_t launch_tile_sr(const Plan& p, int64_t m, int64_t n, int64_t k, const int32_t* A, int64_t lda,
                          const int32_t* B, int64_t ldb, int32_t* C, int64_t ldc, int32_t* temps,
                          hipStream_t st) {
    switch (p.info.sched.tile) {
        case 128: return launch_tile_cfg<SR, 128, 128, 8, 8, 2>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, st);
        case 64: return launch_tile_cfg<SR, 64, 64, 4, 4, 8>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, st);
        default: return launch_tile_cfg<SR, 32, 32, 4, 4, 8>(p, m, n, k, A, lda, B, ldb, C, ldc, temps, st);
    }
}

template <int SR, int NS>
hipError_t launch_merge_ns(const Plan& p, int32_t* C, int64_t ldc, const int32_t* temps, int64_t m, int64_t n,
                           hipStream_t st) {
    const int64_t total = m * n;
    if (total == 0) return hipSuccess;
    const int groups = 1 << p.info.tar_levels;
    ProfScope ps("merge", st);
    hipLaunchKernelGGL((k_merge_i32<SR, NS>), dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, C, ldc,
                       temps, m, n, groups, (int)(p.info.tar_levels > 0), p.temp_stride, p.ldt);
    return hipGetLastError();
}

template <int SR>
hipError_t launch_merge_sr(const Plan& p, int32_t* C, int64_t ldc, const int32_t* temps, int64_t m, int64_t n,
                           hipStream_t st) {
    switch (p.info.sar_levels) {
        case 0: return hipSuccess;
        case 1: return launch_merge_ns<SR, 2>(p, C, ldc, temps, m, n, st);
        case 2: return launch_merge_ns<SR, 4>(p, C, ldc, temps, m, n, st);
        case 3: return launch_merge_ns<SR, 8>(p, C, ldc, temps, m, n, st);
        case 4: return launch_merge_ns<SR, 16>(p, C, ldc, temps, m, n, st);
        case 5: return launch_merge_ns<SR, 32>(p, C, ldc, temps, m, n, st);
        default: return launch_merge_ns<SR, 64>(p, C, ldc, temps, m, n, st);
    }
}

template <int SR, int BM, int BN, int TM, int TN, int KU>
hipError_t launch_persist_cfg(const Plan& p, int64_t m, int64_t n, int64_t k, const int32_t* A, int64_t lda,
                              const int32_t* B, int64_t ldb, int32_t* C, int64_t ldc, void* ws, hipStream_t st) {
    const int64_t tiles_m = ceil_div(m, BM), tiles_n = ceil_div(n, BN);
    const int levels = p.info.sar_levels;
    const int64_t total = tiles_m * tiles_n << levels;
    if (total == 0) return hipSuccess;
    if (!ws) return hipErrorInvalidValue;
    const int64_t groups = p.groups;
    if (levels > 0 && groups < 1) return hipErrorInvalidValue;
    char* w = static_cast<char*>(ws);
    auto* ctl = reinterpret_cast<PersistCtl*>(w);
    auto* owner = reinterpret_cast<unsigned long long*>(w + 16);
    auto* arrive = reinterpret_cast<uint32_t*>(w + 16 + 8 * groups);
    auto* slots = reinterpret_cast<int32_t*>(w + persist_ctl_bytes(groups));
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_semiring_persist<SR, BM, BN, TM, TN, KU>,
                                                         (BM / TM) * (BN / TN), 0);
    if (e != hipSuccess) return e;
    // at most half the ring's slots in flight, so that a new tile rarely
    // finds its group still taken (no cap when every tile has its own group)
    int64_t grid = std::min<int64_t>((int64_t)std::max(per_cu, 1) * cus, total);
    if (levels > 0 && groups < tiles_m * tiles_n)
        grid = std::min<int64_t>(grid, std::max<int64_t>(groups * (int64_t(1) << levels) / 2, 1));
    const int vec_ok = (lda % 4 == 0) && (ldb % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
    // the deepest slice: the ceil half at every split level
    int64_t slice_tiles = ceil_div(k, kBK);
    for (int l = 0; l < levels; ++l) slice_tiles = (slice_tiles + 1) / 2;
    const uint64_t spin_limit = kPersistSpinBase + kPersistSpinPerKTile * (uint64_t)slice_tiles;
    ProfScope ps("semiring_persist", st);
    hipLaunchKernelGGL(k_persist_init, dim3((unsigned)ceil_div(std::max<int64_t>(groups, 1), 256)), dim3(256), 0, st,
                       ctl, owner, arrive, groups);
    hipLaunchKernelGGL((k_semiring_persist<SR, BM, BN, TM, TN, KU>), dim3((unsigned)grid),
                       dim3((BM / TM) * (BN / TN)), 0, st, A, lda, B, ldb, C, ldc, m, n, k, tiles_m, tiles_n, levels,
                       std::max<int64_t>(groups, 1), ctl, owner, arrive, slots, vec_ok, spin_limit);
    return hipGetLastError();
}

template <int SR>
hipError_t launch_persist_sr(const Plan& p, int64_t m, int64_t n, int64_t k, const int32_t* A, int64_t lda,
                             const int32_t* B, int64_t ldb, int32_t* C, int64_t ldc, void* ws, hipStream_t st) {
    switch (p.info.sched.tile) {
        case 128: return launch_persist_cfg<SR, 128, 128, 8, 8, 2>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        case 64: return launch_persist_cfg<SR, 64, 64, 4, 4, 8>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        default: return launch_persist_cfg<SR, 32, 32, 4, 4, 8>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
    }
}

// The kernel kind for a semiring, the schedule's flags, the tile and the
// launch's (tile, slice) items.  A full 128-tile launch (at least the three
// workgroups per CU that fit) runs (min,+) and (max,+) in the shifted
// domain: on the narrow domain the results are the same, and that kernel
// measured 6-13% faster there (n = 4096; the shift between the global loads
// and the LDS stores moves the wait on the loads out of the unrolled
// block).  With fewer workgroups each one's latency decides, and there it
// measured slower (1024 x 1024 x 16384 unsplit: 5.1 against 3.75 ms), as
// in the 32 and 64 tiles.
constexpr int64_t kFull128Items = 3 * 256;  // three resident workgroups on each of 256 CUs

int sem_kind(mm_semiring_kind sr, int32_t flags, int32_t tile, int64_t items) {
    if ((flags & MM_FLAG_CHECKED_RANGE) || (tile == 128 && items >= kFull128Items)) {
        if (sr == MM_SR_MIN_PLUS) return kMinPlusChecked;
        if (sr == MM_SR_MAX_PLUS) return kMaxPlusChecked;
    }
    return (int)sr;
}

}  // namespace

hipError_t launch_semiring_persistent(const Plan& p, mm_semiring_kind sr, int64_t m, int64_t n, int64_t k,
                                      const int32_t* A, int64_t lda, const int32_t* B, int64_t ldb, int32_t* C,
                                      int64_t ldc, void* ws, hipStream_t st) {
    const int32_t t = p.info.sched.tile;
    const int64_t items = ceil_div(m, t) * ceil_div(n, t) * p.info.sched.split_k;
    switch (sem_kind(sr, p.info.sched.flags, t, items)) {
        case MM_SR_MIN_PLUS: return launch_persist_sr<MM_SR_MIN_PLUS>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        case MM_SR_MAX_PLUS: return launch_persist_sr<MM_SR_MAX_PLUS>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        case MM_SR_MAX_MIN: return launch_persist_sr<MM_SR_MAX_MIN>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        case MM_SR_OR_AND: return launch_persist_sr<MM_SR_OR_AND>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        case kMinPlusChecked: return launch_persist_sr<kMinPlusChecked>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        case kMaxPlusChecked: return launch_persist_sr<kMaxPlusChecked>(p, m, n, k, A, lda, B, ldb, C, ldc, ws, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_semiring_tiles(const Plan& p, mm_semiring_kind sr, int64_t m, int64_t n, int64_t k,
                                 const int32_t* A, int64_t lda, const int32_t* B, int64_t ldb, int32_t* C,
                                 int64_t ldc, int32_t* temps, int64_t band_row0, int64_t band_m,
                                 hipStream_t st) {
    (void)m;
    const int32_t* Ab = A + band_row0 * lda;
    int32_t* Cb = C + band_row0 * ldc;
    const int32_t t = p.info.sched.tile;
    const int64_t items = ceil_div(band_m, t) * ceil_div(n, t) * p.info.sched.split_k;
    switch (sem_kind(sr, p.info.sched.flags, t, items)) {
        case MM_SR_MIN_PLUS: return launch_tile_sr<MM_SR_MIN_PLUS>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, st);
        case MM_SR_MAX_PLUS: return launch_tile_sr<MM_SR_MAX_PLUS>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, st);
        case MM_SR_MAX_MIN: return launch_tile_sr<MM_SR_MAX_MIN>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, st);
        case MM_SR_OR_AND: return launch_tile_sr<MM_SR_OR_AND>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, st);
        case kMinPlusChecked: return launch_tile_sr<kMinPlusChecked>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, st);
        case kMaxPlusChecked: return launch_tile_sr<kMaxPlusChecked>(p, band_m, n, k, Ab, lda, B, ldb, Cb, ldc, temps, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_merge_i32(const Plan& p, mm_semiring_kind sr, int32_t* C, int64_t ldc, const int32_t* temps,
                            int64_t band_row0, int64_t band_m, int64_t n, hipStream_t st) {
    int32_t* Cb = C + band_row0 * ldc;
    // merges take the caller's values: every kind of a semiring agrees on
    // them, and the checked one (signed) covers the wider domain
    switch (sem_kind(sr, p.info.sched.flags, 0, 0)) {
        case MM_SR_MIN_PLUS: return launch_merge_sr<MM_SR_MIN_PLUS>(p, Cb, ldc, temps, band_m, n, st);
        case MM_SR_MAX_PLUS: return launch_merge_sr<MM_SR_MAX_PLUS>(p, Cb, ldc, temps, band_m, n, st);
        case MM_SR_MAX_MIN: return launch_merge_sr<MM_SR_MAX_MIN>(p, Cb, ldc, temps, band_m, n, st);
        case MM_SR_OR_AND: return launch_merge_sr<MM_SR_OR_AND>(p, Cb, ldc, temps, band_m, n, st);
        case kMinPlusChecked: return launch_merge_sr<kMinPlusChecked>(p, Cb, ldc, temps, band_m, n, st);
        case kMaxPlusChecked: return launch_merge_sr<kMaxPlusChecked>(p, Cb, ldc, temps, band_m, n, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace starmm
