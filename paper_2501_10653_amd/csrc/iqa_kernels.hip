// Tile-wise LISI / augLISI on gfx950: one fused streaming pass over both images.
//
// What is computed (Li, Adamek & Armour, Sec. 1-3): after the Sec. 2 clamp of
// negative pixels to zero, every N_T x N_T tile gets
//   A = sum (x'+y')/(|x'-y'|+C1),  P = sum (x'+y')|x'-y'|,  Sx = sum x',  Sy = sum y'
//   lisi = D*A/(max(Sx,Sy)+C2)  (Eq. 1),   auglisi = 1 - P/(Sx+Sy+C)  (Eq. 2).
//
// How (MI355X design, not the paper's block-per-tile shared-memory scheme):
//   * The work is HBM-bound: 8 bytes per pixel pair against ~18 VALU slots, so
//     the kernel's job is to keep enough 128-bit loads in flight and to spend
//     as few instructions as possible outside the per-pixel loop.
//   * A wave of 64 lanes is cut into groups of seg*rp lanes, one group per
//     tile: `seg` lanes stream along a tile row (seg*vec floats wide) and `rp`
//     such segments take interleaved rows.  So a wave covers 64/(seg*rp)
//     adjacent tiles, and a whole tile slice reduces inside one wave with DPP
//     lane permutations, with no LDS and no barrier.  Several waves of a
//     workgroup may share a tile's rows (combined once in LDS), and for shapes
//     with few large tiles several workgroups share them (the last of them to
//     finish combines their partials, chosen by an atomic ticket; no second
//     launch).
//   * Each lane folds `vec` adjacent pixels with plain FP32 (FMA chains) and
//     adds the block into Kahan-compensated (hi, lo) accumulators: the long
//     per-lane sums are compensated.  Across lanes the partial sums are folded
//     to one float and added plainly: every partial is non-negative, so a tree
//     of depth d adds at most d units of roundoff, relative.
//   * Loads are double-buffered: the next `unroll` rows are in flight while the
//     current ones are reduced.
//   * Every reduction has a fixed order and there are no floating-point
//     atomics, so results are bitwise reproducible and bitwise symmetric in x, y.
//   * augLISI = 1 - P/S is finalised in double-float so the subtraction keeps
//     the accuracy of the sums.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "iqa.h"
#include "iqa_internal.h"

namespace iqa {

constexpr int kWave = 64;
enum Mode : int { kLisi = 1, kAug = 2, kBoth = 3 };
// How the parts of a split tile group are added up (see split_finish).
enum SplitMode : int { kSplitNone = 0, kSplitTicket = 1, kSplitCombine = 2 };

struct KArgs {
    const float *x;
    const float *y;
    int32_t N;           // image side (row stride in floats), <= 2^17
    int32_t smode;       // split tiles: kSplitNone, kSplitTicket or kSplitCombine
    int32_t NT;          // tile side
    int32_t ns;          // tiles per side
    int32_t ngx;         // tile groups along x: ceil(ns / ht)
    int32_t log_seg;     // log2(lanes per segment)
    int32_t log_grp;     // log2(lanes per tile in a wave) = log2(seg * rp)
    int32_t ht;          // tiles per wave: 64 / (seg * rp)
    int32_t ks;          // workgroups per tile group
    int32_t rows_wave;   // tile rows per wave slice: NT / (waves * ks)
    int32_t lpt;         // column groups per tile row: NT / vec
    int32_t cpl;         // column chunks per lane: ceil(lpt / seg)
    uint32_t ngx_m;      // division multipliers for ngx and ks (see udiv)
    uint32_t ks_m;
    float D, C1, C2, C;
    float *lisi;
    float *aug;
    float *sums;
    float *ws;           // split partials: [group][ks][ht][4]
};

// ---------------------------------------------------------------------------
// Compensated FP32 arithmetic
// ---------------------------------------------------------------------------

struct CSum {
    float hi, lo;   // value = hi + lo
};

// Kahan step: add v, keeping in lo what the rounding of hi lost.
__device__ __forceinline__ void cadd(CSum &a, float v) {
    const float y = v + a.lo;
    const float t = a.hi + y;
    a.lo = y - (t - a.hi);
    a.hi = t;
}

// Exact error-free sum s + e = a + b (Knuth's TwoSum; no ordering needed).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// n / d for d > 0 (normal, finite): the hardware reciprocal estimate, then one
// correction with the exact residual n - q*d from an FMA.  Within one unit in
// the last place (almost always the correctly rounded quotient) in 4
// dependent operations; an IEEE division is a chain of about 15.
__device__ __forceinline__ float div_pos(float n, float d, float rd) {
    const float q = n * rd;
    return __builtin_fmaf(__builtin_fmaf(-q, d, n), rd, q);
}

struct Acc {
    CSum A, P, X, Y;
};

__device__ __forceinline__ Acc acc_zero() {
    return Acc{{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
}

// ---------------------------------------------------------------------------
// Lane permutations
// ---------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// All-reduce steps inside aligned lane groups.  Within a row of 16 lanes the
// partner comes from a DPP permutation: quad swaps for strides 1 and 2, then
// half-row and row mirrors for 4 and 8 (once the smaller strides have made
// each half uniform, a mirror pairs every lane with the other half).  Across
// rows, gfx950's permlane swaps exchange whole rows (16) or half-waves (32).
template <int CTRL>
__device__ __forceinline__ void dpp_add(float &v) {
    v += dpp<CTRL>(v);
}

template <int W>
__device__ __forceinline__ void permlane_swap(float &a, float &b) {
    const auto r = W == 16 ? __builtin_amdgcn_permlane16_swap(__float_as_uint(a),
                                                              __float_as_uint(b), false, false)
                           : __builtin_amdgcn_permlane32_swap(__float_as_uint(a),
                                                              __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// One swap level for a single value: with both operands equal, the two
// results are the two halves of a row pair (W = 16) or of the wave (W = 32),
// and their sum is the same on every lane.
template <int W>
__device__ __forceinline__ void swap_add(float &v) {
    float a = v, b = v;
    permlane_swap<W>(a, b);
    v = a + b;
}

// The same level for two values with two swaps instead of two pairs of
// swaps and adds.  Swapping between a and b leaves in one half of each row
// pair (or wave) a's two halves and in the other b's; one add then forms a's
// total in the first and b's in the second, with the operands in the order
// swap_add uses, so the bits are the same.  Swapping that sum with itself
// hands both totals to every lane.
template <int W>
__device__ __forceinline__ void swap_add2(float &a, float &b) {
    permlane_swap<W>(a, b);
    float t = a + b, u = t;
    permlane_swap<W>(t, u);
    a = t;
    b = u;
}

// Plain sums over aligned groups of 2^log_g lanes; every lane of a group ends
// with the same bits (each step adds the same two values).
struct Sum4 {
    float A, P, X, Y;
};

template <int MODE, typename Step>
__device__ __forceinline__ void each(Sum4 &s, Step step) {
    if constexpr ((MODE & kLisi) != 0) step(s.A);
    if constexpr ((MODE & kAug) != 0) step(s.P);
    step(s.X);
    step(s.Y);
}

template <int MODE, int W>
__device__ __forceinline__ void swap_level(Sum4 &s) {
    if constexpr (MODE == kBoth) {
        swap_add2<W>(s.A, s.P);
    } else if constexpr (MODE == kLisi) {
        swap_add<W>(s.A);
    } else {
        swap_add<W>(s.P);
    }
    swap_add2<W>(s.X, s.Y);
}

// log_g is uniform, so the level tests are scalar branches; marked likely,
// they keep the levels a group needs in one straight run of code.
template <int MODE>
__device__ __forceinline__ Sum4 group_allreduce(Sum4 s, int log_g) {
    if (__builtin_expect(log_g > 0, 1)) {
        each<MODE>(s, [](float &v) { dpp_add<0xB1>(v); });    // quad_perm [1,0,3,2]
        if (__builtin_expect(log_g > 1, 1)) {
            each<MODE>(s, [](float &v) { dpp_add<0x4E>(v); });    // quad_perm [2,3,0,1]
            if (__builtin_expect(log_g > 2, 1)) {
                each<MODE>(s, [](float &v) { dpp_add<0x141>(v); });   // row_half_mirror
                if (__builtin_expect(log_g > 3, 1)) {
                    each<MODE>(s, [](float &v) { dpp_add<0x140>(v); });   // row_mirror
                    if (__builtin_expect(log_g > 4, 1)) {
                        swap_level<MODE, 16>(s);
                        if (__builtin_expect(log_g > 5, 1)) swap_level<MODE, 32>(s);
                    }
                }
            }
        }
    }
    return s;
}

__device__ __forceinline__ Sum4 fold(const Acc &a) {
    return Sum4{a.A.hi + a.A.lo, a.P.hi + a.P.lo, a.X.hi + a.X.lo, a.Y.hi + a.Y.lo};
}

// ---------------------------------------------------------------------------
// Per-pixel work
// ---------------------------------------------------------------------------

template <int VEC> struct VecT;
template <> struct VecT<4> { using T = float4; };
template <> struct VecT<2> { using T = float2; };
template <> struct VecT<1> { using T = float; };

// Streaming loads: every input byte is read exactly once, so they carry the
// nontemporal hint and do not displace other data in the caches.
template <int VEC>
__device__ __forceinline__ typename VecT<VEC>::T vload(const float *p) {
    if constexpr (VEC == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p));
        return float4{v.x, v.y, v.z, v.w};
    } else if constexpr (VEC == 2) {
        typedef float f2 __attribute__((ext_vector_type(2)));
        const f2 v = __builtin_nontemporal_load(reinterpret_cast<const f2 *>(p));
        return float2{v.x, v.y};
    } else {
        return __builtin_nontemporal_load(p);
    }
}

// Load at a wave-uniform base plus a 32-bit per-lane byte offset, which the
// hardware adds itself (no 64-bit address arithmetic per load).
template <int VEC>
__device__ __forceinline__ typename VecT<VEC>::T vload_off(const float *base, uint32_t byte_off) {
    return vload<VEC>(reinterpret_cast<const float *>(reinterpret_cast<const char *>(base) +
                                                      byte_off));
}

template <int VEC>
__device__ __forceinline__ typename VecT<VEC>::T vzero() {
    typename VecT<VEC>::T z;
    std::memset(&z, 0, sizeof(z));
    return z;
}

template <int VEC>
__device__ __forceinline__ float velem(const typename VecT<VEC>::T &v, int e) {
    if constexpr (VEC == 1) {
        return v;
    } else {
        return reinterpret_cast<const float *>(&v)[e];
    }
}

// Per-pixel terms of VEC adjacent pixel pairs, added with plain FP32 (FMA
// chains) into a short block sum b.  A pair of zeros adds nothing.
template <int VEC, int MODE>
__device__ __forceinline__ void accumulate(const typename VecT<VEC>::T &xv,
                                           const typename VecT<VEC>::T &yv, float C1, Sum4 &b) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const float xr = velem<VEC>(xv, e);
        const float yr = velem<VEC>(yv, e);
        const float xc = xr > 0.f ? xr : 0.f;   // Sec. 2 clamp; NaN and -0 -> +0
        const float yc = yr > 0.f ? yr : 0.f;
        const float s = xc + yc;                // |x'+y'| (both non-negative)
        const float d = fabsf(xc - yc);         // |x'-y'|
        if constexpr ((MODE & kLisi) != 0) {
            const float r = __builtin_amdgcn_rcpf(d + C1);
            b.A = __builtin_fmaf(s, r, b.A);
        }
        if constexpr ((MODE & kAug) != 0) b.P = __builtin_fmaf(s, d, b.P);
        b.X = b.X + xc;
        b.Y = b.Y + yc;
    }
}

// Add a block sum into the Kahan-compensated lane accumulators.
template <int MODE>
__device__ __forceinline__ void add_block(Acc &acc, const Sum4 &b) {
    if constexpr ((MODE & kLisi) != 0) cadd(acc.A, b.A);
    if constexpr ((MODE & kAug) != 0) cadd(acc.P, b.P);
    cadd(acc.X, b.X);
    cadd(acc.Y, b.Y);
}

// ---------------------------------------------------------------------------
// Finalisation (Eq. 1, Eq. 2)
// ---------------------------------------------------------------------------

// A tile's sums reach these as plain FP32 values: each lane folded its
// compensation in before the cross-lane adds.

// Eq. 1.
__device__ __forceinline__ void finalize_lisi(const KArgs &a, int64_t t, const Sum4 &s) {
    if (!a.lisi) return;
    const float den = fmaxf(s.X, s.Y) + a.C2;
    a.lisi[t] = div_pos(a.D * s.A, den, __builtin_amdgcn_rcpf(den));
}

// Eq. 2: S = Sx + Sy + C and q = P / S in double-float, then 1 - q.
__device__ __forceinline__ void finalize_aug(const KArgs &a, int64_t t, const Sum4 &s) {
    if (!a.aug) return;
    float s1, e1;
    two_sum(s.X, s.Y, s1, e1);
    float s2, e2;
    two_sum(s1, a.C, s2, e2);
    float Sh, Sl;
    two_sum(s2, e1 + e2, Sh, Sl);
    const float rS = __builtin_amdgcn_rcpf(Sh);
    const float q1 = div_pos(s.P, Sh, rS);
    float r = __builtin_fmaf(-q1, Sh, s.P);    // remainder of P / Sh
    r = __builtin_fmaf(-q1, Sl, r);
    const float q2 = r * rS;                   // correction term: a few bits suffice
    float h, e;
    two_sum(1.0f, -q1, h, e);
    a.aug[t] = h + (e - q2);
}

__device__ __forceinline__ void store_sums(const KArgs &a, int64_t t, const Sum4 &s) {
    if (a.sums) reinterpret_cast<float4 *>(a.sums)[t] = float4{s.A, s.P, s.X, s.Y};
}

template <int MODE>
__device__ __forceinline__ void finalize(const KArgs &a, int64_t t, const Sum4 &s) {
    if constexpr ((MODE & kLisi) != 0) finalize_lisi(a, t, s);
    if constexpr ((MODE & kAug) != 0) finalize_aug(a, t, s);
    if constexpr (MODE == kBoth) store_sums(a, t, s);
}

// The dispatcher hands workgroup b to XCD b % 8, and each XCD has its own L2
// whose channels interleave on low address bits.  Renumbering so that XCD x
// gets one contiguous range of logical workgroups keeps every XCD streaming
// from all column offsets (and so from all of its L2 channels) instead of the
// one offset class that b % 8 would give it.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_remap(uint32_t b, uint32_t grid) {
    const uint32_t xcd = b % kXcds;
    const uint32_t local = b / kXcds;
    const uint32_t full = grid / kXcds;
    const uint32_t rem = grid % kXcds;
    return (int)(xcd * full + (xcd < rem ? xcd : rem) + local);
}

// Division by a divisor d fixed for the launch (1 <= d < 2^31), for numerators
// 0 <= n < 2^31, without the ~30-instruction integer division sequence: with
// l = ceil(log2 d) and m = floor(2^(31+l) / d) + 1 (< 2^32, computed on the
// host by div_magic), n / d = (n * m) >> (31 + l) exactly (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994,
// Theorem 4.2 with 31-bit numerators).  Block indices are wave-uniform, so
// this runs on the scalar unit ahead of the first load.
__device__ __forceinline__ int udiv(int n, uint32_t m, int d) {
    const uint32_t l = d > 1 ? 32u - (uint32_t)__clz((uint32_t)d - 1u) : 0u;
    return (int)(((uint64_t)(uint32_t)n * m) >> (31u + l));
}

// ---------------------------------------------------------------------------
// Timeline stamps (diagnostic launches only)
// ---------------------------------------------------------------------------
//
// The constant-rate wall clock, read once `v` has been computed: the empty
// volatile asm needs v in a register, and volatile statements keep their
// order with the clock read, so the stamp cannot move above the arithmetic
// (and the loads) that produced v.
__device__ __forceinline__ uint64_t stamp_after(float v) {
    asm volatile("" ::"v"(v));
    return wall_clock64();
}

// ---------------------------------------------------------------------------
// One wave's slice of one tile group
// ---------------------------------------------------------------------------
//
// A tile group is the ht = 64/(seg*rp) horizontally adjacent tiles one wave
// covers: tiles txg*ht .. txg*ht+ht-1 of tile row ty.  A slice is rows
// slice*rows_wave .. (slice+1)*rows_wave-1 of those tiles.  Lane L works on
// tile j = L >> log_grp, row phase k = (L >> log_seg) & (rp-1) and column
// group l = L & (seg-1): rows k, k+rp, k+2rp, ... of the slice.  Returns the
// slice's sums of tile j, the same on every lane of the tile's lane group.
template <int VEC, int U, int MODE, bool WIDE, bool TL = false>
__device__ __forceinline__ Sum4 slice_sums(const KArgs &a, int ty, int txg, int slice, int lane,
                                           uint64_t *ts = nullptr) {
    using V = typename VecT<VEC>::T;
    const int seg = 1 << a.log_seg;
    const int log_rp = a.log_grp - a.log_seg;
    const int rp = 1 << log_rp;
    const int l = lane & (seg - 1);
    const int k = (lane >> a.log_seg) & (rp - 1);
    const int j = lane >> a.log_grp;
    const int tx = txg * a.ht + j;

    int M = 0;   // rows of the tile this lane reduces: ceil((rows_wave - k) / rp)
    if (tx < a.ns && k < a.rows_wave) M = (a.rows_wave - k + rp - 1) >> log_rp;
    const int64_t col0 = (int64_t)tx * a.NT;
    // First row of the slice: uniform across the wave, so the image pointers
    // below live in scalar registers.
    const int64_t srow = (int64_t)ty * a.NT + (int64_t)slice * a.rows_wave;

    Acc acc = acc_zero();

    if constexpr (!WIDE) {
        // One column group per lane (lanes past the tile row idle).  The slice
        // spans rows_wave * N floats, which the host keeps below 2^30, so byte
        // offsets from the slice start fit in 32 bits.
        if (l >= a.lpt) M = 0;
        const float *bx = a.x + srow * a.N;
        const float *by = a.y + srow * a.N;
        uint32_t off = (uint32_t)(((int64_t)k * a.N + col0 + (int64_t)l * VEC) * 4);
        const uint32_t step = (uint32_t)((int64_t)rp * a.N * 4);
        // Full batches of U rows, double-buffered: the next batch is in flight
        // while this one is reduced.  Compensation is per batch.
        int m = 0;
        if (M >= U) {
            V ax[U], ay[U], cx[U], cy[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ax[u] = vload_off<VEC>(bx, off + u * step);
                ay[u] = vload_off<VEC>(by, off + u * step);
            }
            off += U * step;
            while (true) {
                const bool more_c = m + 2 * U <= M;
                if (more_c) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        cx[u] = vload_off<VEC>(bx, off + u * step);
                        cy[u] = vload_off<VEC>(by, off + u * step);
                    }
                    off += U * step;
                }
                {
                    Sum4 b{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int u = 0; u < U; ++u) accumulate<VEC, MODE>(ax[u], ay[u], a.C1, b);
                    add_block<MODE>(acc, b);
                    if constexpr (TL) {
                        if (m == 0) ts[0] = stamp_after(acc.X.hi);
                    }
                }
                m += U;
                if (!more_c) break;
                const bool more_a = m + 2 * U <= M;
                if (more_a) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        ax[u] = vload_off<VEC>(bx, off + u * step);
                        ay[u] = vload_off<VEC>(by, off + u * step);
                    }
                    off += U * step;
                }
                {
                    Sum4 b{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int u = 0; u < U; ++u) accumulate<VEC, MODE>(cx[u], cy[u], a.C1, b);
                    add_block<MODE>(acc, b);
                }
                m += U;
                if (!more_a) break;
            }
        }
        // Remaining rows (fewer than U), one at a time.
        for (; m < M; ++m) {
            const V xv = vload_off<VEC>(bx, off);
            const V yv = vload_off<VEC>(by, off);
            off += step;
            Sum4 b{0.f, 0.f, 0.f, 0.f};
            accumulate<VEC, MODE>(xv, yv, a.C1, b);
            add_block<MODE>(acc, b);
            if constexpr (TL) {
                if (m == 0) ts[0] = stamp_after(acc.X.hi);
            }
        }
    } else {
        // Tile rows wider than a segment: chunk q covers column group l + q*seg.
        for (int m = 0; m < M; ++m) {
            const int64_t row = srow + k + (int64_t)m * rp;
            const float *px = a.x + row * a.N + col0;
            const float *py = a.y + row * a.N + col0;
            for (int q0 = 0; q0 < a.cpl; q0 += U) {
                V xv[U], yv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cg = l + (q0 + u) * seg;
                    if (q0 + u < a.cpl && cg < a.lpt) {
                        xv[u] = vload<VEC>(px + (int64_t)cg * VEC);
                        yv[u] = vload<VEC>(py + (int64_t)cg * VEC);
                    } else {
                        xv[u] = vzero<VEC>();
                        yv[u] = vzero<VEC>();
                    }
                }
                Sum4 b{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int u = 0; u < U; ++u) accumulate<VEC, MODE>(xv[u], yv[u], a.C1, b);
                add_block<MODE>(acc, b);
                if constexpr (TL) {
                    if (m == 0 && q0 == 0) ts[0] = stamp_after(acc.X.hi);
                }
            }
        }
    }
    if constexpr (TL) ts[1] = stamp_after(acc.X.hi);

    // Sum the lanes of each tile inside the wave.
    return group_allreduce<MODE>(fold(acc), a.log_grp);
}

// Pairwise tree over the partial sums of WAVES waves (all non-negative), in a
// fixed order: the same bits wherever a tile's slices are combined.
template <int WAVES>
__device__ __forceinline__ float4 wave_tree(float4 (&v)[WAVES]) {
#pragma unroll
    for (int h = 1; h < WAVES; h *= 2) {
#pragma unroll
        for (int w = 0; w + h < WAVES; w += 2 * h) {
            v[w].x += v[w + h].x;
            v[w].y += v[w + h].y;
            v[w].z += v[w + h].z;
            v[w].w += v[w + h].w;
        }
    }
    return v[0];
}

// ---------------------------------------------------------------------------
// Split tiles: adding up the parts of a tile group
// ---------------------------------------------------------------------------
//
// With ks > 1 workgroups per tile group, every part stores its partial sums
// (one float4 per tile), and the parts are added in one of two ways:
//
//   * kSplitTicket: each part then takes a ticket from the group's counter,
//     and the part that draws the last one adds the partials and finalises,
//     within the same launch; it also sets the counter back to zero.  No part
//     waits for another.  The parts run on different XCDs, whose L2 caches
//     are not coherent with one another, so the partials travel by
//     device-coherent accesses (agent-scope atomic stores and loads, which
//     bypass the non-coherent cache levels), and only the ordering is left to
//     the counter: a part's partial stores have completed (vmcnt 0) before it
//     takes its ticket, and the last part issues its partial loads only after
//     its ticket has returned.
//   * kSplitCombine: the parts only store their partials, and combine_kernel,
//     launched right after on the same stream, adds them.
//
// The ticket costs every part a few memory round trips at its end (store
// acknowledgement, atomic); while a launch fits the GPU in one round of
// workgroups that is cheaper than a second launch, but when many rounds of
// workgroups queue behind those round trips it is not, and the host picks
// the combine launch (split_mode).
//
// Either way the partials are added the way the kernel adds pixels: lane q of
// tile j's lane group Kahan-adds parts q, q + g, q + 2g, ... (g lanes per
// tile), then the group is summed with the same fixed DPP tree.  The order
// depends neither on the mechanism nor on which part came last, so results
// are bitwise reproducible and equal between the two.
//
// Workspace: partials [group][part][ht] float4 from a.ws on, and (ticket
// mode) one 32-bit counter per group just below a.ws (group g's at
// a.ws - 4 (g + 1) bytes), in a counter region that holds nothing but
// counters.  The counters start at zero and every launch leaves the ones it
// used at zero, so a region reused by shapes of any size is all zeros between
// launches.
__host__ __device__ __forceinline__ int64_t split_partials(int64_t groups, int64_t ks, int64_t ht) {
    return groups * ks * ht;   // float4 entries
}

__device__ __forceinline__ void store_coherent(float4 *p, float4 v) {
    uint64_t *q = reinterpret_cast<uint64_t *>(p);
    const uint64_t lo = (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
    const uint64_t hi = (uint64_t)__float_as_uint(v.z) | ((uint64_t)__float_as_uint(v.w) << 32);
    __hip_atomic_store(q, lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, hi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ float4 load_coherent(const float4 *p) {
    const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
    const uint64_t lo = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t hi = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return float4{__uint_as_float((uint32_t)lo), __uint_as_float((uint32_t)(lo >> 32)),
                  __uint_as_float((uint32_t)hi), __uint_as_float((uint32_t)(hi >> 32))};
}

// Wait until this wave's vector memory operations have completed.
__device__ __forceinline__ void wait_vmem() {
    __builtin_amdgcn_s_waitcnt(/*vmcnt*/ 0 | (/*expcnt*/ 0x7 << 4) | (/*lgkmcnt*/ 0xf << 8));
}

// Add up tile group grp's parts and finalise its tiles (one wave).  COHERENT
// reads the partials with device-coherent loads (within the launch that wrote
// them), else with plain loads (a later launch).
template <int MODE, bool COHERENT>
__device__ __forceinline__ void combine_parts(const KArgs &a, int grp, int lane) {
    const float4 *ws = reinterpret_cast<const float4 *>(a.ws);
    const int64_t base = (int64_t)grp * a.ks;
    const int ty = udiv(grp, a.ngx_m, a.ngx);
    const int txg = grp - ty * a.ngx;
    // Lane group of tile j: 2^log_grp lanes; lane q of the group takes parts
    // q, q + g, ...
    const int g = 1 << a.log_grp;
    const int j = lane >> a.log_grp;
    const int q = lane & (g - 1);
    const int tx = txg * a.ht + j;
    Acc c = acc_zero();
    if (tx < a.ns) {
        for (int p = q; p < a.ks; p += g) {
            const float4 *src = ws + (base + p) * a.ht + j;
            const float4 w = COHERENT ? load_coherent(src) : *src;
            if constexpr ((MODE & kLisi) != 0) cadd(c.A, w.x);
            if constexpr ((MODE & kAug) != 0) cadd(c.P, w.y);
            cadd(c.X, w.z);
            cadd(c.Y, w.w);
        }
    }
    const Sum4 s = group_allreduce<MODE>(fold(c), a.log_grp);
    if (q == 0 && tx < a.ns) finalize<MODE>(a, (int64_t)ty * a.ns + tx, s);
}

// A part's end of a split tile group; returns whether this workgroup
// finished the group (ticket mode, last part).
template <int MODE>
__device__ __forceinline__ bool split_finish(const KArgs &a, int grp, int part, int lane, bool mine,
                                             int jt, float4 v) {
    float4 *ws = reinterpret_cast<float4 *>(a.ws);
    float4 *slot = ws + ((int64_t)grp * a.ks + part) * a.ht + jt;
    if (a.smode == kSplitCombine) {
        if (mine) *slot = v;
        return false;
    }
    if (mine) store_coherent(slot, v);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(a.ws) - 1 - grp;
    wait_vmem();                                        // partials stored before the ticket
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t ticket = 0;
    if (lane == 0) ticket = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ticket = __builtin_amdgcn_readfirstlane(ticket);    // waits for the returned value
    if (ticket != (uint32_t)(a.ks - 1)) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    combine_parts<MODE, true>(a, grp, lane);
    if (lane == 0) __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

// ---------------------------------------------------------------------------
// The tile kernel (one image pair)
// ---------------------------------------------------------------------------
//
// Grid: one workgroup of WAVES waves per (tile group, split part).  The tile
// rows are cut into WAVES*ks contiguous slices of rows_wave rows; wave w of
// part p takes slice p*WAVES + w.
//
// SPLIT kernels (ks > 1 workgroups per tile group) finish through
// split_finish; the others finalise directly, and carry no split code.
//
// With several waves and both indices wanted, a workgroup that is not split
// finishes its tiles on two waves at once: wave 0 Eq. 1 (and the sums), wave
// 1 Eq. 2, each from the same LDS tree.
//
// TL (diagnostic launches only) records, per workgroup, wall-clock stamps of
// wave 0: entry, its first batch of rows reduced (first loads back), its last
// rows reduced (last loads back), and its exit after its results are stored,
// plus the XCD and hardware slot it ran on: 8 uint64 per workgroup at
// tl[8 * blockIdx.x], written with ordinary vector stores; the split part's
// word has bit 32 set when this workgroup finished its tiles.
template <int VEC, int WAVES, int U, int MODE, bool WIDE, bool SPLIT, bool TL>
__device__ __forceinline__ void tiles_body(const KArgs &a, uint64_t *tl) {
    uint64_t ts[4] = {0, 0, 0, 0};
    if constexpr (TL) ts[0] = wall_clock64();
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const int grp = udiv(bid, a.ks_m, a.ks);
    const int part = bid - grp * a.ks;
    const int ty = udiv(grp, a.ngx_m, a.ngx);
    const int txg = grp - ty * a.ngx;

    const Sum4 s = slice_sums<VEC, U, MODE, WIDE, TL>(a, ty, txg, part * WAVES + wave, lane, ts + 1);
    constexpr bool kTwoWaveFinish = WAVES > 1 && MODE == kBoth && !SPLIT;

    // The tile this lane finishes, if any: a lane group's leader with one wave
    // per workgroup; lane j of wave 0 after the LDS combine otherwise.
    bool mine;
    int jt;
    float4 v{s.A, s.P, s.X, s.Y};
    if constexpr (WAVES == 1) {
        jt = lane >> a.log_grp;
        mine = (lane & ((1 << a.log_grp) - 1)) == 0 && txg * a.ht + jt < a.ns;
    } else {
        // Combine the waves' slices of each tile in LDS, wave order fixed.
        __shared__ float4 lds[WAVES][kWave];
        if ((lane & ((1 << a.log_grp) - 1)) == 0) lds[wave][lane >> a.log_grp] = v;
        __syncthreads();
        if (wave != 0 && !(kTwoWaveFinish && wave == 1)) return;
        jt = lane;
        mine = lane < a.ht && txg * a.ht + lane < a.ns;
        if (mine) {
            float4 w[WAVES];
#pragma unroll
            for (int i = 0; i < WAVES; ++i) w[i] = lds[i][lane];
            v = wave_tree<WAVES>(w);
        }
    }
    bool last = true;   // this workgroup finished its tiles
    if constexpr (!SPLIT) {
        const int64_t t = (int64_t)ty * a.ns + txg * a.ht + jt;
        const Sum4 r{v.x, v.y, v.z, v.w};
        if constexpr (kTwoWaveFinish) {
            if (mine && wave == 0) {
                finalize_lisi(a, t, r);
                store_sums(a, t, r);
            }
            if (mine && wave == 1) finalize_aug(a, t, r);
        } else {
            if (mine) finalize<MODE>(a, t, r);
        }
    } else {
        last = split_finish<MODE>(a, grp, part, lane, mine, jt, v);
    }
    if constexpr (TL) {
        if (wave == 0) {
            __builtin_amdgcn_s_waitcnt(0);   // every store of the wave has landed
            const uint64_t t_end = wall_clock64();
            if (lane == 0) {
                uint64_t *r = tl + (int64_t)blockIdx.x * 8;
                r[0] = ts[0];
                r[1] = ts[1];
                r[2] = ts[2];
                r[3] = t_end;
                r[4] = (uint64_t)__builtin_amdgcn_s_getreg((31 << 11) | 20);   // XCC_ID
                r[5] = (uint64_t)__builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_ID
                r[6] = (uint64_t)grp;
                r[7] = (uint64_t)part | ((uint64_t)last << 32);
            }
        }
    }
}

template <int VEC, int WAVES, int U, int MODE, bool WIDE, bool SPLIT>
__global__ __launch_bounds__(WAVES * kWave) void tiles_kernel(KArgs a) {
    tiles_body<VEC, WAVES, U, MODE, WIDE, SPLIT, false>(a, nullptr);
}

template <int VEC, int WAVES, int U, bool WIDE, bool SPLIT>
__global__ __launch_bounds__(WAVES * kWave) void tiles_kernel_tl(KArgs a, uint64_t *tl) {
    tiles_body<VEC, WAVES, U, kBoth, WIDE, SPLIT, true>(a, tl);
}

// kSplitCombine: one wave per tile group adds its parts, after the tile
// kernel on the same stream (so the partials are complete and visible).
template <int MODE>
__global__ __launch_bounds__(kWave) void combine_kernel(KArgs a) {
    combine_parts<MODE, false>(a, (int)blockIdx.x, (int)threadIdx.x);
}

// ---------------------------------------------------------------------------
// The batched kernel (many image pairs of mixed N and N_T, one launch)
// ---------------------------------------------------------------------------
//
// Each pair is described by its own geometry and by the index of its first
// work unit.  A unit is the work of one workgroup of kBatchWaves waves:
//   * a pair whose geometry has one wave per tile group (waves 1) packs
//     kBatchWaves consecutive tile groups into a unit, wave w taking the
//     unit's w-th group;
//   * a pair whose geometry has kBatchWaves waves per tile group gives each
//     tile group a unit of its own: the waves take its row slices and combine
//     them in LDS exactly as tiles_kernel does.
// A persistent grid takes units round-robin: workgroup b does units b, b + G,
// b + 2G, ... where G is the number of workgroups.  Either way a pair's
// results are bitwise equal to a single-pair launch with the same geometry
// and unroll (ksplit 1).
struct BatchDesc {
    KArgs a;
    int64_t unit_begin;
};
static_assert(sizeof(BatchDesc) <= IQA_BATCH_DESC_BYTES, "batch descriptor size");

constexpr int kBatchWaves = 4;   // waves per workgroup

// A pair whose waves split its tile groups' rows (rows_wave < NT).
__host__ __device__ __forceinline__ bool batch_coop(const KArgs &a) { return a.rows_wave != a.NT; }

// Work units of one pair.
__host__ __device__ __forceinline__ int64_t batch_units(const KArgs &a) {
    const int64_t groups = (int64_t)a.ns * a.ngx;
    return batch_coop(a) ? groups : (groups + kBatchWaves - 1) / kBatchWaves;
}

template <int U>
__device__ __forceinline__ void batch_body(const BatchDesc *descs, int count, int64_t units) {
    __shared__ float4 lds[kBatchWaves][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    for (int64_t u = xcd_remap(blockIdx.x, gridDim.x); u < units; u += gridDim.x) {
        // Binary search for the pair whose units contain u (same in every wave).
        int lo = 0, hi = count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (descs[mid].unit_begin <= u) lo = mid; else hi = mid - 1;
        }
        const int pi = __builtin_amdgcn_readfirstlane(lo);
        const KArgs a = descs[pi].a;
        // A unit outside the pair's units (a unit count or pair count that
        // does not match the table) is skipped, never read.
        const int64_t g64 = u - descs[pi].unit_begin;
        if (g64 < 0 || g64 >= batch_units(a)) continue;
        const bool leader = (lane & ((1 << a.log_grp) - 1)) == 0;
        if (!batch_coop(a)) {
            const int64_t grp64 = g64 * kBatchWaves + wave;
            if (grp64 >= (int64_t)a.ns * a.ngx) continue;
            const int grp = (int)grp64;
            const int ty = udiv(grp, a.ngx_m, a.ngx);
            const int txg = grp - ty * a.ngx;
            const Sum4 s = a.cpl > 1 ? slice_sums<4, U, kBoth, true>(a, ty, txg, 0, lane)
                                     : slice_sums<4, U, kBoth, false>(a, ty, txg, 0, lane);
            const int tx = txg * a.ht + (lane >> a.log_grp);
            if (leader && tx < a.ns) finalize<kBoth>(a, (int64_t)ty * a.ns + tx, s);
        } else {
            // Workgroup-uniform branch: every wave reaches both barriers.
            const int grp = (int)g64;
            const int ty = udiv(grp, a.ngx_m, a.ngx);
            const int txg = grp - ty * a.ngx;
            const Sum4 s = a.cpl > 1 ? slice_sums<4, U, kBoth, true>(a, ty, txg, wave, lane)
                                     : slice_sums<4, U, kBoth, false>(a, ty, txg, wave, lane);
            if (leader) lds[wave][lane >> a.log_grp] = float4{s.A, s.P, s.X, s.Y};
            __syncthreads();
            // Two waves finish the tiles at once, as in the tile kernel.
            if (wave < 2 && lane < a.ht) {
                const int txl = txg * a.ht + lane;
                if (txl < a.ns) {
                    float4 v[kBatchWaves];
#pragma unroll
                    for (int w = 0; w < kBatchWaves; ++w) v[w] = lds[w][lane];
                    const float4 t4 = wave_tree<kBatchWaves>(v);
                    const Sum4 r{t4.x, t4.y, t4.z, t4.w};
                    const int64_t t = (int64_t)ty * a.ns + txl;
                    if (wave == 0) {
                        finalize_lisi(a, t, r);
                        store_sums(a, t, r);
                    } else {
                        finalize_aug(a, t, r);
                    }
                }
            }
            __syncthreads();   // the LDS slots are reused by the next unit
        }
    }
}

// The descriptor table in device memory (any number of pairs).
template <int U>
__global__ __launch_bounds__(kBatchWaves * kWave) void batch_kernel(const BatchDesc *descs,
                                                                    int count, int64_t units) {
    batch_body<U>(descs, count, units);
}

// Up to CAP descriptors passed by value in the kernel arguments: no table to
// copy to the device before the launch.  The waves read the descriptors
// straight from the kernel-argument segment.  Instantiated for CAP = 1, 4 and
// IQA_BATCH_INLINE_MAX: a launch uses the smallest that holds its batch,
// because the host-side cost of a launch grows with its argument size.
template <int CAP>
struct InlineDescs {
    BatchDesc d[CAP];
    int64_t units;
    int32_t count;
};

template <int U, int CAP>
__global__ __launch_bounds__(kBatchWaves * kWave) void batch_kernel_inline(InlineDescs<CAP> in) {
    batch_body<U>(in.d, in.count, in.units);
}

// ---------------------------------------------------------------------------
// Hierarchical aggregation (Eq. 3, Eq. 4)
// ---------------------------------------------------------------------------
//
// Eq. 3 and Eq. 4 recover the value of a larger tile (or of the whole image)
// from its child tiles.  Both weight each child's index by its own
// denominator, which is the same as adding the children's sums A, P, Sx, Sy
// and applying Eq. 1 / Eq. 2 to the totals; that is what this kernel does,
// from the sums iqa_tiles exports.  One workgroup per parent tile: each thread
// adds a fixed stride of children with Kahan compensation, the wave and the
// workgroup then add in a fixed order, and thread 0 finalises.
struct MergeArgs {
    const float *sums_in;   // ns*ns children, 4 floats each
    int64_t ns;             // children per side
    int64_t f;              // children per parent side
    float D, C2, C;
    float *lisi;
    float *aug;
    float *sums;
};

__global__ __launch_bounds__(256) void merge_kernel(MergeArgs m) {
    const int64_t np = m.ns / m.f;
    const int64_t p = blockIdx.x;
    const int64_t py = p / np, px = p - py * np;
    const int64_t nchild = m.f * m.f;
    Acc acc = acc_zero();
    const float4 *in = reinterpret_cast<const float4 *>(m.sums_in);
    for (int64_t c = threadIdx.x; c < nchild; c += 256) {
        const int64_t cy = c / m.f, cx = c - cy * m.f;
        const float4 v = in[(py * m.f + cy) * m.ns + px * m.f + cx];
        cadd(acc.A, v.x);
        cadd(acc.P, v.y);
        cadd(acc.X, v.z);
        cadd(acc.Y, v.w);
    }
    Sum4 s = group_allreduce<kBoth>(fold(acc), 6);
    __shared__ float4 part[4];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) part[wave] = float4{s.A, s.P, s.X, s.Y};
    __syncthreads();
    if (threadIdx.x != 0) return;
    const float4 a = part[0], b = part[1], c = part[2], d = part[3];
    const Sum4 t{(a.x + b.x) + (c.x + d.x), (a.y + b.y) + (c.y + d.y),
                 (a.z + b.z) + (c.z + d.z), (a.w + b.w) + (c.w + d.w)};
    KArgs k{};
    k.D = m.D;
    k.C2 = m.C2;
    k.C = m.C;
    k.lisi = m.lisi;
    k.aug = m.aug;
    k.sums = m.sums;
    finalize<kBoth>(k, p, t);
}

// ---------------------------------------------------------------------------
// Streaming-read reference: the attainable HBM read rate on this GPU
// ---------------------------------------------------------------------------
//
// Each workgroup sums a contiguous chunk of float4s (several loads in flight
// per lane) and writes one float; the result is only there so that the loads
// cannot be removed.  Used to express the tile kernel's bandwidth as a
// fraction of what a plain read achieves.
__global__ __launch_bounds__(256) void read_ceiling_kernel(const float4 *__restrict__ src,
                                                           int64_t n4, int64_t per_block,
                                                           float *out) {
    const int64_t b0 = (int64_t)blockIdx.x * per_block;
    const int64_t b1 = b0 + per_block < n4 ? b0 + per_block : n4;
    float acc = 0.f;
    int64_t i = b0 + threadIdx.x;
    const float *f = reinterpret_cast<const float *>(src);
    for (; i + 3 * 256 < b1; i += 4 * 256) {
        const float4 a = vload<4>(f + 4 * i), b = vload<4>(f + 4 * (i + 256));
        const float4 c = vload<4>(f + 4 * (i + 512)), d = vload<4>(f + 4 * (i + 768));
        acc += (a.x + a.y + a.z + a.w) + (b.x + b.y + b.z + b.w) +
               (c.x + c.y + c.z + c.w) + (d.x + d.y + d.z + d.w);
    }
    for (; i < b1; i += 256) {
        const float4 a = vload<4>(f + 4 * i);
        acc += a.x + a.y + a.z + a.w;
    }
    for (int st = 32; st > 0; st >>= 1) acc += __shfl_xor(acc, st, kWave);
    __shared__ float part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

thread_local int g_last_hip_error = 0;

// Every launch goes through hipLaunchKernel and reports its own status (not a
// sticky error some earlier, unrelated call left behind).  The arguments take
// the kernel's own parameter types, so a mismatch does not compile.
template <typename T>
struct same_type {
    using type = T;
};

template <typename... P>
hipError_t launch_kernel(void (*fn)(P...), unsigned grid, unsigned block, hipStream_t s,
                         typename same_type<P>::type... args) {
    void *argv[] = {static_cast<void *>(&args)...};
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(grid), dim3(block), argv, 0,
                           s);
}

iqa_status hip_status(hipError_t e) {
    if (e == hipSuccess) return IQA_OK;
    g_last_hip_error = (int)e;
    return IQA_ERR_HIP;
}

using LaunchFn = hipError_t (*)(const KArgs &, uint64_t *, unsigned, hipStream_t);

template <int VEC, int WAVES, int U, int MODE, bool WIDE, bool SPLIT>
hipError_t launch_impl(const KArgs &a, uint64_t *, unsigned grid, hipStream_t s) {
    return launch_kernel(&tiles_kernel<VEC, WAVES, U, MODE, WIDE, SPLIT>, grid, WAVES * kWave, s,
                         a);
}

template <int VEC, int WAVES, int U, bool WIDE, bool SPLIT>
hipError_t launch_tl(const KArgs &a, uint64_t *tl, unsigned grid, hipStream_t s) {
    return launch_kernel(&tiles_kernel_tl<VEC, WAVES, U, WIDE, SPLIT>, grid, WAVES * kWave, s, a,
                         tl);
}

// What a launch needs, mapped onto the instantiated kernels.
struct Want {
    int mode;
    bool wide, split, tl;
};

template <int VEC, int WAVES, int U, bool WIDE, bool SPLIT>
LaunchFn pick_mode(const Want &w) {
    if (w.tl) {
        if constexpr (VEC == 4) return &launch_tl<VEC, WAVES, U, WIDE, SPLIT>;
        return nullptr;
    }
    switch (w.mode) {
        case kLisi: return &launch_impl<VEC, WAVES, U, kLisi, WIDE, SPLIT>;
        case kAug: return &launch_impl<VEC, WAVES, U, kAug, WIDE, SPLIT>;
        default: return &launch_impl<VEC, WAVES, U, kBoth, WIDE, SPLIT>;
    }
}

template <int VEC, int WAVES, int U>
LaunchFn pick_shape(const Want &w) {
    if (w.wide) {
        return w.split ? pick_mode<VEC, WAVES, U, true, true>(w)
                       : pick_mode<VEC, WAVES, U, true, false>(w);
    }
    return w.split ? pick_mode<VEC, WAVES, U, false, true>(w)
                   : pick_mode<VEC, WAVES, U, false, false>(w);
}

template <int VEC, int WAVES>
LaunchFn pick_unroll(int unroll, const Want &w) {
    switch (unroll) {
        case 4: return pick_shape<VEC, WAVES, 4>(w);
        case 8: return pick_shape<VEC, WAVES, 8>(w);
        default: return nullptr;
    }
}

// The instantiated launch shapes: waves 1/2/4/8 with unroll 4/8 and waves 16
// with unroll 4 for vec 4, and waves 1/4 with unroll 4 for the narrow vec 2
// and vec 1 paths; each with and without a row split across workgroups.
// Timeline launches exist for the vec 4 shapes, fused mode.
LaunchFn pick(const iqa_launch_cfg &c, const Want &w) {
    if (c.vec == 4) {
        switch (c.waves) {
            case 1: return pick_unroll<4, 1>(c.unroll, w);
            case 2: return pick_unroll<4, 2>(c.unroll, w);
            case 4: return pick_unroll<4, 4>(c.unroll, w);
            case 8: return pick_unroll<4, 8>(c.unroll, w);
            case 16: return c.unroll == 4 ? pick_shape<4, 16, 4>(w) : nullptr;
            default: return nullptr;
        }
    }
    if (w.tl || c.unroll != 4 || !(c.waves == 1 || c.waves == 4)) return nullptr;
    if (c.vec == 2) return c.waves == 1 ? pick_shape<2, 1, 4>(w) : pick_shape<2, 4, 4>(w);
    if (c.vec == 1) return c.waves == 1 ? pick_shape<1, 1, 4>(w) : pick_shape<1, 4, 4>(w);
    return nullptr;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int64_t v) {
    int r = 0;
    while ((int64_t(1) << r) < v) ++r;
    return r;
}
int64_t next_pow2(int64_t v) { return int64_t(1) << ilog2(v); }

// Multiplier m = floor(2^(31 + ceil(log2 d)) / d) + 1 for udiv (1 <= d < 2^31).
uint32_t div_magic(int64_t d) {
    const int l = ilog2(d);
    return (uint32_t)(((uint64_t)1 << (31 + l)) / (uint64_t)d + 1);
}

bool param_ok(float v) {
    return std::isfinite(v) && v > 0.f && std::fpclassify(v) == FP_NORMAL;
}

bool aligned(const void *p, size_t b) { return (reinterpret_cast<uintptr_t>(p) % b) == 0; }

iqa_status check_shape(int64_t N, int64_t NT) {
    if (N <= 0 || NT <= 0 || N > IQA_MAX_N || NT > N || N % NT != 0) return IQA_ERR_SHAPE;
    return IQA_OK;
}

struct Geometry {
    int64_t ns, ht, ngx, groups, grid;
    int lpt, cpl;
};

iqa_status geometry(int64_t N, int64_t NT, const iqa_launch_cfg &c, Geometry &g) {
    if (!(c.vec == 1 || c.vec == 2 || c.vec == 4) || NT % c.vec) return IQA_ERR_CONFIG;
    if (!is_pow2(c.seg) || !is_pow2(c.rp) || (int64_t)c.seg * c.rp > kWave) return IQA_ERR_CONFIG;
    if (!is_pow2(c.waves) || c.waves > 16) return IQA_ERR_CONFIG;
    if (c.ksplit < 1 || NT % ((int64_t)c.waves * c.ksplit) != 0) return IQA_ERR_CONFIG;
    if (pick(c, Want{kBoth, false, false, false}) == nullptr) return IQA_ERR_CONFIG;
    g.ns = N / NT;
    g.ht = kWave / ((int64_t)c.seg * c.rp);
    g.ngx = (g.ns + g.ht - 1) / g.ht;
    g.groups = g.ns * g.ngx;
    g.grid = g.groups * c.ksplit;
    g.lpt = (int)(NT / c.vec);
    g.cpl = (int)((g.lpt + c.seg - 1) / c.seg);
    if (g.grid > (int64_t)INT_MAX) return IQA_ERR_CONFIG;
    return IQA_OK;
}

// Built-in launch shape for (N, NT), for shapes the autotuner has not
// measured: widest aligned vector, one segment per tile row (up to a full
// wave), two row phases per wave, enough waves per workgroup that each lane
// reduces ~16 rows, and row splits across workgroups while the launch has
// fewer than ~4 waves per CU.  (The measured shapes cluster around this.)
constexpr int64_t kTargetWaves = 1024;

iqa_launch_cfg default_cfg(int64_t N, int64_t NT, const float *x, const float *y) {
    iqa_launch_cfg c{};
    c.vec = 1;
    if (NT % 2 == 0 && aligned(x, 8) && aligned(y, 8)) c.vec = 2;
    if (NT % 4 == 0 && aligned(x, 16) && aligned(y, 16)) c.vec = 4;
    const int64_t lpt = NT / c.vec;
    c.seg = (int)std::min<int64_t>(kWave, next_pow2(lpt));
    const int64_t tpw = kWave / c.seg;     // segments per wave
    const int64_t ns = N / NT;
    const int64_t rp = std::min<int64_t>(2, tpw);
    c.rp = (int)rp;
    const int64_t ht = tpw / rp;
    const int64_t groups = ns * ((ns + ht - 1) / ht);
    int64_t kw = 1;
    const int64_t kw_max = c.vec == 4 ? 16 : 4;
    while (kw < kw_max && NT % (kw * 2) == 0 && NT / (rp * kw * 2) >= 16) kw *= 2;
    if (c.vec != 4 && kw > 1) kw = (NT % 4 == 0) ? 4 : 1;
    int64_t ks = 1;
    while (groups * kw * ks < kTargetWaves && NT % (kw * ks * 2) == 0 &&
           NT / (rp * kw * ks * 2) >= 4)
        ks *= 2;
    c.waves = (int)kw;
    c.unroll = (c.vec == 4 && kw <= 8) ? 8 : 4;
    c.ksplit = (int)ks;
    return c;
}

// Tuned launch shapes.  The autotuner's measurements on gfx950 are compiled in
// (tuned_table.inc, generated by the build from the tuner's JSON cache);
// entries registered at run time take precedence.  kind 0 = single-pair
// launches, kind 1 = per-pair geometry in batches; N == 0 matches any N.
struct TunedEntry {
    int64_t N, NT;
    int kind;
    iqa_launch_cfg cfg;
};
#if __has_include("tuned_table.inc")
#include "tuned_table.inc"
#else
static const TunedEntry kTuned[] = {{-1, -1, -1, {0, 0, 0, 0, 0, 0}}};
static const int kTunedCount = 0;
static const int64_t kTunedBatchWaves = 0;
#endif

std::mutex g_tune_mutex;
std::map<std::tuple<int64_t, int64_t, int>, iqa_launch_cfg> g_tuned;

// The per-pair geometries the batch kernel can run: vec 4, no row split,
// unroll 8, and one wave per tile group or the workgroup's four waves on each.
constexpr int kBatchUnroll = 8;

bool batch_geometry_ok(const iqa_launch_cfg &c) {
    return c.vec == 4 && c.ksplit == 1 && c.unroll == kBatchUnroll &&
           (c.waves == 1 || c.waves == kBatchWaves);
}

bool tuned_lookup(int64_t N, int64_t NT, int kind, iqa_launch_cfg *out) {
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        for (int64_t n : {N, int64_t(0)}) {
            auto it = g_tuned.find(std::make_tuple(n, NT, kind));
            if (it != g_tuned.end()) {
                *out = it->second;
                return true;
            }
        }
    }
    for (int64_t n : {N, int64_t(0)}) {
        for (int i = 0; i < kTunedCount; ++i) {
            const TunedEntry &e = kTuned[i];
            if (e.N == n && e.NT == NT && e.kind == kind) {
                Geometry g{};
                if (geometry(N, NT, e.cfg, g) != IQA_OK) continue;
                if (kind != IQA_TUNE_SINGLE && !batch_geometry_ok(e.cfg)) continue;
                *out = e.cfg;
                return true;
            }
        }
    }
    return false;
}

iqa_launch_cfg pick_cfg(int64_t N, int64_t NT, const float *x, const float *y) {
    iqa_launch_cfg c;
    if (aligned(x, 16) && aligned(y, 16) && tuned_lookup(N, NT, 0, &c)) return c;
    return default_cfg(N, NT, x, y);
}

// Per-pair geometry inside a batch: vec 4, one wave per tile group, no row
// split, and as many tiles per wave as make a unit of about 64 KiB of input.

iqa_launch_cfg batch_cfg(int64_t N, int64_t NT) {
    iqa_launch_cfg c;
    if (tuned_lookup(N, NT, 1, &c)) return c;
    c.vec = 4;
    c.waves = 1;
    c.unroll = kBatchUnroll;
    c.ksplit = 1;
    const int64_t lpt = NT / 4;
    c.seg = (int)std::min<int64_t>(kWave, next_pow2(lpt));
    const int64_t tpw = kWave / c.seg;
    const int64_t want = std::max<int64_t>(1, (int64_t(64) << 10) / (8 * NT * NT));
    int64_t ht = 1;
    while (ht * 2 <= tpw && ht * 2 <= want && ht * 2 <= next_pow2(N / NT)) ht *= 2;
    c.rp = (int)(tpw / ht);
    return c;
}

// Per-pair geometry in the server's batches: its own tuned entries (chosen
// for a lone pair's latency), else the ragged-batch geometry.
iqa_launch_cfg serve_cfg(int64_t N, int64_t NT) {
    iqa_launch_cfg c;
    if (tuned_lookup(N, NT, IQA_TUNE_SERVE, &c)) return c;
    return batch_cfg(N, NT);
}

// Per (device, stream) workspace for split tiles: a counter region (ticket
// counters only) followed by a partial-sum region.  A launch uses its
// workspace from its first workgroup to its last, and launches on one stream
// run one after the other, so one buffer per stream is enough; concurrent
// streams get their own.  A new buffer is cleared on its stream before first
// use, and since each launch leaves its counters at zero, the counter region
// stays all zeros between launches whatever shapes share it.  A buffer that
// is outgrown is kept, not freed: a graph captured earlier may still launch
// kernels that use it.
struct Workspace {
    void *ptr = nullptr;
    size_t cnt_bytes = 0;    // counter region, at ptr
    size_t part_bytes = 0;   // partial-sum region, at ptr + cnt_bytes
};
std::mutex g_ws_mutex;
std::map<std::pair<int, void *>, Workspace> g_ws;
std::vector<void *> g_ws_retired;

// Split launches of at most this many workgroups (one round on gfx950's 256
// CUs at four workgroups each) add their parts by ticket, within the launch;
// larger ones store their partials and a combine launch adds them (see
// split_finish for why).
constexpr int64_t kTicketMaxGrid = 1024;

int split_mode(const Geometry &g, const iqa_launch_cfg &c) {
    if (c.ksplit <= 1) return kSplitNone;
    return g.grid <= kTicketMaxGrid ? kSplitTicket : kSplitCombine;
}

struct SplitNeed {
    size_t cnt_bytes = 0, part_bytes = 0;   // 0, 0: the launch does not split
};

SplitNeed split_need(const Geometry &g, const iqa_launch_cfg &c) {
    SplitNeed n;
    const int m = split_mode(g, c);
    if (m == kSplitNone) return n;
    if (m == kSplitTicket) n.cnt_bytes = (size_t)g.groups * sizeof(uint32_t);
    n.part_bytes = (size_t)split_partials(g.groups, c.ksplit, g.ht) * 4 * sizeof(float);
    return n;
}

size_t round_up(size_t v, size_t m) { return (v + m - 1) / m * m; }

// *part receives the partial-sum region; the counter region ends where it
// starts.  The caller holds g_ws_mutex.
iqa_status workspace_for(hipStream_t s, const SplitNeed &need, float **part) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    Workspace &w = g_ws[{dev, (void *)s}];
    if (w.cnt_bytes < need.cnt_bytes || w.part_bytes < need.part_bytes) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (s != nullptr) {
            e = hipStreamIsCapturing(s, &cs);
            if (e != hipSuccess) return hip_status(e);
        }
        if (cs != hipStreamCaptureStatusNone) return IQA_ERR_CAPTURE;
        const size_t cb = round_up(std::max(need.cnt_bytes, w.cnt_bytes), 4096);
        const size_t pb = round_up(std::max(need.part_bytes, w.part_bytes), 4096);
        void *p = nullptr;
        e = hipMalloc(&p, cb + pb);
        if (e != hipSuccess) return hip_status(e);
        e = hipMemsetAsync(p, 0, cb + pb, s);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return hip_status(e);
        }
        if (w.ptr) g_ws_retired.push_back(w.ptr);
        w.ptr = p;
        w.cnt_bytes = cb;
        w.part_bytes = pb;
    }
    *part = reinterpret_cast<float *>(static_cast<char *>(w.ptr) + w.cnt_bytes);
    return IQA_OK;
}

// Scratch of the no-allocation entry point: a fixed array in device memory,
// one copy per GPU, held until the process ends.  It starts zeroed (the
// loader clears the array), and every launch leaves its ticket counters at
// zero.  Its device address comes from hipGetSymbolAddress, once per device,
// with that device current; host code never uses the array's name otherwise.
static __device__ __align__(256) float scratch[IQA_NOALLOC_SCRATCH_BYTES / sizeof(float)];

// The first kScratchCounterBytes of the array are the counter region (the
// partial-sum region starts right after it), the rest holds partial sums.
constexpr size_t kScratchCounterBytes = 64 << 10;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// The caller holds g_scratch_mutex.
iqa_status scratch_for_current_device(float **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices) return IQA_ERR_CONFIG;
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        if (p == nullptr) return IQA_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<float *>(g_scratch_ptr[dev]);
    return IQA_OK;
}

void fill_args(KArgs &a, const float *x, const float *y, int64_t N, int64_t NT, float D,
               float C1, float C2, float C, float *lisi, float *aug, float *sums,
               const iqa_launch_cfg &c, const Geometry &g) {
    a.x = x;
    a.y = y;
    a.N = (int32_t)N;
    a.smode = kSplitNone;
    a.NT = (int32_t)NT;
    a.ns = (int32_t)g.ns;
    a.ngx = (int32_t)g.ngx;
    a.log_seg = ilog2(c.seg);
    a.log_grp = ilog2((int64_t)c.seg * c.rp);
    a.ht = (int32_t)g.ht;
    a.ks = c.ksplit;
    a.rows_wave = (int32_t)(NT / ((int64_t)c.waves * c.ksplit));
    a.lpt = g.lpt;
    a.cpl = g.cpl;
    a.ngx_m = div_magic(g.ngx);
    a.ks_m = div_magic(c.ksplit);
    a.D = D;
    a.C1 = C1;
    a.C2 = C2;
    a.C = C;
    a.lisi = lisi;
    a.aug = aug;
    a.sums = sums;
}

hipError_t launch_combine(const KArgs &a, int mode, const Geometry &g, hipStream_t s) {
    void (*fn)(KArgs) = mode == kLisi  ? &combine_kernel<kLisi>
                        : mode == kAug ? &combine_kernel<kAug>
                                       : &combine_kernel<kBoth>;
    return launch_kernel(fn, (unsigned)g.groups, kWave, s, a);
}

// Where a launch's split workspace comes from.
enum class Ws {
    kLibrary,   // the per-(device, stream) buffer, grown on demand
    kScratch,   // the fixed scratch array (no allocation; bounded size)
    kPrepare,   // only allocate the library buffer, launch nothing
};

iqa_status run(const float *x, const float *y, int64_t N, int64_t NT, float D, float C1,
               float C2, float C, float *lisi, float *aug, float *sums,
               const iqa_launch_cfg *cfg_in, void *stream, Ws ws, uint64_t *tl = nullptr) {
    iqa_launch_cfg c = cfg_in ? *cfg_in : pick_cfg(N, NT, x, y);
    Geometry g{};
    iqa_status st = geometry(N, NT, c, g);
    if (st != IQA_OK) return st;
    if (ws != Ws::kPrepare) {
        if (!aligned(x, 4 * c.vec) || !aligned(y, 4 * c.vec)) return IQA_ERR_ALIGN;
    }
    int mode = ((lisi || sums) ? kLisi : 0) | ((aug || sums) ? kAug : 0);
    if (mode == 0) mode = kBoth;
    LaunchFn fn = pick(c, Want{mode, g.cpl > 1, c.ksplit > 1, tl != nullptr});
    if (!fn) return IQA_ERR_CONFIG;
    hipStream_t s = static_cast<hipStream_t>(stream);

    KArgs a{};
    const SplitNeed need = split_need(g, c);
    // The workspace (or scratch) stays locked until the launches are
    // enqueued: a combine-mode split is two launches, and another host
    // thread's split launches on the same stream must not come between them.
    std::unique_lock<std::mutex> ws_lock(g_ws_mutex, std::defer_lock);
    std::unique_lock<std::mutex> scratch_lock(g_scratch_mutex, std::defer_lock);
    if (need.part_bytes > 0) {
        if (ws == Ws::kScratch) {
            if (need.cnt_bytes > kScratchCounterBytes ||
                need.part_bytes > IQA_NOALLOC_SCRATCH_BYTES - kScratchCounterBytes)
                return IQA_ERR_SCRATCH;
            scratch_lock.lock();
            float *base = nullptr;
            st = scratch_for_current_device(&base);
            if (st != IQA_OK) return st;
            a.ws = reinterpret_cast<float *>(reinterpret_cast<char *>(base) + kScratchCounterBytes);
        } else {
            ws_lock.lock();
            st = workspace_for(s, need, &a.ws);
            if (st != IQA_OK) return st;
        }
    }
    if (ws == Ws::kPrepare) return IQA_OK;

    fill_args(a, x, y, N, NT, D, C1, C2, C, lisi, aug, sums, c, g);
    a.smode = split_mode(g, c);
    hipError_t e = fn(a, tl, (unsigned)g.grid, s);
    if (e == hipSuccess && a.smode == kSplitCombine) e = launch_combine(a, mode, g, s);
    return hip_status(e);
}

iqa_status check_common(const float *x, const float *y, int64_t N, int64_t NT) {
    if (!x || !y) return IQA_ERR_NULL;
    iqa_status st = check_shape(N, NT);
    if (st != IQA_OK) return st;
    if (!aligned(x, 4) || !aligned(y, 4)) return IQA_ERR_ALIGN;
    return IQA_OK;
}

iqa_status check_outputs_params(float *lisi, float *auglisi, float *sums, float D, float C1,
                                float C2, float C) {
    if (!lisi && !auglisi && !sums) return IQA_ERR_NULL;
    if (!aligned(lisi, 4) || !aligned(auglisi, 4) || !aligned(sums, 16)) return IQA_ERR_ALIGN;
    const bool need_l = lisi || sums, need_a = auglisi || sums;
    if (need_l && (!param_ok(D) || !param_ok(C1) || !param_ok(C2))) return IQA_ERR_PARAM;
    if (need_a && !param_ok(C)) return IQA_ERR_PARAM;
    return IQA_OK;
}

template <int CAP>
iqa_status launch_inline(const void *descs_host, int64_t count, int64_t total_units,
                         int64_t blocks, hipStream_t s) {
    InlineDescs<CAP> in;
    std::memset(&in, 0, sizeof(in));
    std::memcpy(in.d, descs_host, (size_t)count * sizeof(BatchDesc));
    in.units = total_units;
    in.count = (int32_t)count;
    return hip_status(launch_kernel(&batch_kernel_inline<kBatchUnroll, CAP>, (unsigned)blocks,
                                    kBatchWaves * kWave, s, in));
}

}  // namespace iqa

using namespace iqa;

extern "C" {

iqa_status iqa_tiles_cfg(const float *x, const float *y, int64_t N, int64_t NT, float D,
                         float C1, float C2, float C, float *lisi, float *auglisi, float *sums,
                         const iqa_launch_cfg *cfg, void *stream) {
    iqa_status st = check_common(x, y, N, NT);
    if (st != IQA_OK) return st;
    st = check_outputs_params(lisi, auglisi, sums, D, C1, C2, C);
    if (st != IQA_OK) return st;
    return run(x, y, N, NT, D, C1, C2, C, lisi, auglisi, sums, cfg, stream, Ws::kLibrary);
}

iqa_status iqa_tiles(const float *x, const float *y, int64_t N, int64_t NT, float D, float C1,
                     float C2, float C, float *lisi, float *auglisi, float *sums, void *stream) {
    return iqa_tiles_cfg(x, y, N, NT, D, C1, C2, C, lisi, auglisi, sums, nullptr, stream);
}

iqa_status iqa_tiles_noalloc(const float *x, const float *y, int64_t N, int64_t NT, float D,
                             float C1, float C2, float C, float *lisi, float *auglisi, float *sums,
                             const iqa_launch_cfg *cfg, void *stream) {
    iqa_status st = check_common(x, y, N, NT);
    if (st != IQA_OK) return st;
    st = check_outputs_params(lisi, auglisi, sums, D, C1, C2, C);
    if (st != IQA_OK) return st;
    return run(x, y, N, NT, D, C1, C2, C, lisi, auglisi, sums, cfg, stream, Ws::kScratch);
}

iqa_status iqa_tiles_timeline(const float *x, const float *y, int64_t N, int64_t NT, float D,
                              float C1, float C2, float C, float *lisi, float *auglisi,
                              float *sums, const iqa_launch_cfg *cfg, uint64_t *stamps,
                              int64_t stamp_count, void *stream) {
    iqa_status st = check_common(x, y, N, NT);
    if (st != IQA_OK) return st;
    st = check_outputs_params(lisi, auglisi, sums, D, C1, C2, C);
    if (st != IQA_OK) return st;
    if (!stamps) return IQA_ERR_NULL;
    if (!aligned(stamps, 8)) return IQA_ERR_ALIGN;
    const iqa_launch_cfg c = cfg ? *cfg : pick_cfg(N, NT, x, y);
    Geometry g{};
    st = geometry(N, NT, c, g);
    if (st != IQA_OK) return st;
    if (stamp_count < 8 * g.grid) return IQA_ERR_SHAPE;
    return run(x, y, N, NT, D, C1, C2, C, lisi, auglisi, sums, &c, stream, Ws::kLibrary, stamps);
}

int64_t iqa_launch_workgroups(int64_t N, int64_t NT, const iqa_launch_cfg *cfg) {
    if (!cfg || check_shape(N, NT) != IQA_OK) return -1;
    Geometry g{};
    if (geometry(N, NT, *cfg, g) != IQA_OK) return -1;
    return g.grid;
}

iqa_status lisi_tiles(const float *x, const float *y, int64_t N, int64_t NT, float D, float C1,
                      float C2, float *lisi, void *stream) {
    iqa_status st = check_common(x, y, N, NT);
    if (st != IQA_OK) return st;
    if (!lisi) return IQA_ERR_NULL;
    if (!aligned(lisi, 4)) return IQA_ERR_ALIGN;
    if (!param_ok(D) || !param_ok(C1) || !param_ok(C2)) return IQA_ERR_PARAM;
    return run(x, y, N, NT, D, C1, C2, 1.0f, lisi, nullptr, nullptr, nullptr, stream,
               Ws::kLibrary);
}

iqa_status auglisi_tiles(const float *x, const float *y, int64_t N, int64_t NT, float C,
                         float *auglisi, void *stream) {
    iqa_status st = check_common(x, y, N, NT);
    if (st != IQA_OK) return st;
    if (!auglisi) return IQA_ERR_NULL;
    if (!aligned(auglisi, 4)) return IQA_ERR_ALIGN;
    if (!param_ok(C)) return IQA_ERR_PARAM;
    return run(x, y, N, NT, 1.0f, 1.0f, 1.0f, C, nullptr, auglisi, nullptr, nullptr, stream,
               Ws::kLibrary);
}

iqa_status iqa_default_cfg(int64_t N, int64_t NT, const float *x, const float *y,
                           iqa_launch_cfg *cfg) {
    if (!cfg) return IQA_ERR_NULL;
    iqa_status st = check_shape(N, NT);
    if (st != IQA_OK) return st;
    *cfg = pick_cfg(N, NT, x, y);
    return IQA_OK;
}

iqa_status iqa_check_cfg(int64_t N, int64_t NT, const iqa_launch_cfg *cfg) {
    if (!cfg) return IQA_ERR_NULL;
    iqa_status st = check_shape(N, NT);
    if (st != IQA_OK) return st;
    Geometry g{};
    return geometry(N, NT, *cfg, g);
}

iqa_status iqa_prepare(int64_t N, int64_t NT, const iqa_launch_cfg *cfg, void *stream) {
    iqa_status st = check_shape(N, NT);
    if (st != IQA_OK) return st;
    const float *probe = reinterpret_cast<const float *>(uintptr_t(256));
    return run(probe, probe, N, NT, 1.f, 1.f, 1.f, 1.f, nullptr, nullptr, nullptr, cfg, stream,
               Ws::kPrepare);
}

iqa_status iqa_tune_set(int64_t N, int64_t NT, int kind, const iqa_launch_cfg *cfg) {
    if (!cfg) return IQA_ERR_NULL;
    // N == 0 registers the entry for every image size with this tile size.
    iqa_status st = check_shape(N == 0 ? NT : N, NT);
    if (st != IQA_OK) return st;
    if (kind != IQA_TUNE_SINGLE && kind != IQA_TUNE_BATCH && kind != IQA_TUNE_SERVE)
        return IQA_ERR_CONFIG;
    Geometry g{};
    st = geometry(N == 0 ? NT : N, NT, *cfg, g);
    if (st != IQA_OK) return st;
    if (cfg->vec != 4) return IQA_ERR_CONFIG;
    if (kind != IQA_TUNE_SINGLE && !batch_geometry_ok(*cfg)) return IQA_ERR_CONFIG;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tuned[std::make_tuple(N, NT, kind)] = *cfg;
    return IQA_OK;
}

void iqa_tune_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tuned.clear();
}

int64_t iqa_batch_default_waves(void) {
    return kTunedBatchWaves > 0 ? kTunedBatchWaves : 2048;
}

iqa_status iqa_batch_cfg(int64_t N, int64_t NT, iqa_launch_cfg *cfg) {
    if (!cfg) return IQA_ERR_NULL;
    iqa_status st = check_shape(N, NT);
    if (st != IQA_OK) return st;
    if (NT % 4 != 0) return IQA_ERR_CONFIG;
    *cfg = batch_cfg(N, NT);
    return IQA_OK;
}

iqa_status iqa_serve_cfg(int64_t N, int64_t NT, iqa_launch_cfg *cfg) {
    if (!cfg) return IQA_ERR_NULL;
    iqa_status st = check_shape(N, NT);
    if (st != IQA_OK) return st;
    if (NT % 4 != 0) return IQA_ERR_CONFIG;
    *cfg = serve_cfg(N, NT);
    return IQA_OK;
}

iqa_status iqa_batch_describe(const iqa_pair *pairs, int64_t count, void *descs,
                              int64_t *total_units) {
    return iqa::describe_pairs(pairs, count, descs, total_units, IQA_TUNE_BATCH);
}

}  // extern "C"

iqa_status iqa::describe_pairs(const iqa_pair *pairs, int64_t count, void *descs,
                               int64_t *total_units, int kind) {
    if (!pairs || !descs || !total_units) return IQA_ERR_NULL;
    if (count < 1 || count > INT_MAX) return IQA_ERR_SHAPE;
    BatchDesc *out = static_cast<BatchDesc *>(descs);
    int64_t units = 0;
    for (int64_t i = 0; i < count; ++i) {
        const iqa_pair &p = pairs[i];
        iqa_status st = check_common(p.x, p.y, p.N, p.NT);
        if (st != IQA_OK) return st;
        st = check_outputs_params(p.lisi, p.auglisi, p.sums, p.D, p.C1, p.C2, p.C);
        if (st != IQA_OK) return st;
        if (p.NT % 4 != 0) return IQA_ERR_CONFIG;
        if (!aligned(p.x, 16) || !aligned(p.y, 16)) return IQA_ERR_ALIGN;
        const iqa_launch_cfg c = kind == IQA_TUNE_SERVE ? serve_cfg(p.N, p.NT) : batch_cfg(p.N, p.NT);
        Geometry g{};
        st = geometry(p.N, p.NT, c, g);
        if (st != IQA_OK) return st;
        BatchDesc d;
        std::memset(&d, 0, sizeof(d));
        // Outputs a pair does not ask for stay NULL; the batch always computes
        // all four sums, so lisi and auglisi get the constants they need.
        fill_args(d.a, p.x, p.y, p.N, p.NT, p.lisi || p.sums ? p.D : 1.f,
                  p.lisi || p.sums ? p.C1 : 1.f, p.lisi || p.sums ? p.C2 : 1.f,
                  p.auglisi || p.sums ? p.C : 1.f, p.lisi, p.auglisi, p.sums, c, g);
        d.unit_begin = units;
        units += batch_units(d.a);
        std::memcpy(out + i, &d, sizeof(d));
    }
    if (units > ((int64_t)1 << 40)) return IQA_ERR_SHAPE;
    *total_units = units;
    return IQA_OK;
}

extern "C" {

iqa_status iqa_tiles_batched(const void *descs_dev, int64_t count, int64_t total_units,
                             int64_t waves, void *stream) {
    if (!descs_dev) return IQA_ERR_NULL;
    if (count < 1 || count > INT_MAX || total_units < 1) return IQA_ERR_SHAPE;
    if (!aligned(descs_dev, 16)) return IQA_ERR_ALIGN;
    if (waves < kBatchWaves || waves % kBatchWaves != 0 || waves / kBatchWaves > INT_MAX)
        return IQA_ERR_CONFIG;
    const int64_t blocks = std::min<int64_t>(waves / kBatchWaves, total_units);
    return hip_status(launch_kernel(&batch_kernel<kBatchUnroll>, (unsigned)blocks,
                                    kBatchWaves * kWave, static_cast<hipStream_t>(stream),
                                    static_cast<const BatchDesc *>(descs_dev), (int)count,
                                    total_units));
}

iqa_status iqa_tiles_batched_inline(const void *descs_host, int64_t count, int64_t total_units,
                                    int64_t waves, void *stream) {
    if (!descs_host) return IQA_ERR_NULL;
    if (count < 1 || count > IQA_BATCH_INLINE_MAX || total_units < 1) return IQA_ERR_SHAPE;
    if (waves < kBatchWaves || waves % kBatchWaves != 0 || waves / kBatchWaves > INT_MAX)
        return IQA_ERR_CONFIG;
    // The table is on the host here, so its unit numbering is checked: pair i
    // starts where pair i - 1 ends, and the pairs cover exactly total_units.
    int64_t next = 0;
    for (int64_t i = 0; i < count; ++i) {
        BatchDesc d;
        std::memcpy(&d, static_cast<const BatchDesc *>(descs_host) + i, sizeof(d));
        if (d.unit_begin != next || d.a.ns < 1 || d.a.ngx < 1) return IQA_ERR_CONFIG;
        next += batch_units(d.a);
    }
    if (next != total_units) return IQA_ERR_CONFIG;
    const int64_t blocks = std::min<int64_t>(waves / kBatchWaves, total_units);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (count == 1) return launch_inline<1>(descs_host, count, total_units, blocks, s);
    if (count <= 4) return launch_inline<4>(descs_host, count, total_units, blocks, s);
    return launch_inline<IQA_BATCH_INLINE_MAX>(descs_host, count, total_units, blocks, s);
}

iqa_status iqa_merge_tiles(const float *sums_in, int64_t ns, int64_t f, float D, float C2,
                           float C, float *lisi, float *auglisi, float *sums_out, void *stream) {
    if (!sums_in) return IQA_ERR_NULL;
    if (ns <= 0 || f <= 0 || ns % f != 0 || ns > IQA_MAX_N) return IQA_ERR_SHAPE;
    iqa_status st = check_outputs_params(lisi, auglisi, sums_out, D, 1.f, C2, C);
    if (st != IQA_OK) return st;
    if (!aligned(sums_in, 16)) return IQA_ERR_ALIGN;
    const int64_t np = ns / f;
    if (np * np > INT_MAX) return IQA_ERR_SHAPE;
    MergeArgs m{sums_in, ns, f, D, C2, C, lisi, auglisi, sums_out};
    return hip_status(launch_kernel(&merge_kernel, (unsigned)(np * np), 256,
                                    static_cast<hipStream_t>(stream), m));
}

iqa_status iqa_read_ceiling(const float *buf, int64_t n, float *out, int64_t blocks,
                            void *stream) {
    if (!buf || !out) return IQA_ERR_NULL;
    if (n <= 0 || n % 4 != 0 || blocks <= 0 || blocks > INT_MAX) return IQA_ERR_SHAPE;
    if (!aligned(buf, 16) || !aligned(out, 4)) return IQA_ERR_ALIGN;
    const int64_t n4 = n / 4;
    const int64_t per = (n4 + blocks - 1) / blocks;
    return hip_status(launch_kernel(&read_ceiling_kernel, (unsigned)blocks, 256,
                                    static_cast<hipStream_t>(stream),
                                    reinterpret_cast<const float4 *>(buf), n4, per, out));
}

const char *iqa_status_str(int status) {
    switch (status) {
        case IQA_OK: return "IQA_OK";
        case IQA_ERR_NULL: return "IQA_ERR_NULL: a required pointer is NULL or no output was requested";
        case IQA_ERR_SHAPE: return "IQA_ERR_SHAPE: N and NT must be positive, NT must divide N, N <= 2^17";
        case IQA_ERR_ALIGN: return "IQA_ERR_ALIGN: a float pointer is not 4-byte aligned (sums: 16-byte)";
        case IQA_ERR_PARAM: return "IQA_ERR_PARAM: D, C1, C2 and C must be positive, finite, normal floats";
        case IQA_ERR_HIP: return "IQA_ERR_HIP: a HIP call or kernel launch failed";
        case IQA_ERR_CONFIG: return "IQA_ERR_CONFIG: launch configuration invalid for this shape";
        case IQA_ERR_CAPTURE: return "IQA_ERR_CAPTURE: workspace must grow while the stream is captured";
        case IQA_ERR_BUDGET: return "IQA_ERR_BUDGET: the request can never fit the server's HBM budget";
        case IQA_ERR_TIMEOUT: return "IQA_ERR_TIMEOUT: the wait ran out of time";
        case IQA_ERR_SCRATCH: return "IQA_ERR_SCRATCH: the shape needs more split scratch than iqa_tiles_noalloc holds";
        default: return "unknown iqa_status";
    }
}

int iqa_last_hip_error(void) { return g_last_hip_error; }

int iqa_version(void) { return 400; }

}  // extern "C"
