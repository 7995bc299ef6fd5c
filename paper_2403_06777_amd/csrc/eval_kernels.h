// Evaluation kernels for gfx950 (templates): evaluate a packed term program over its
// assignments and sum the terms exactly.  Each eval_w*.hip unit instantiates one form-vector
// width W, so the variants compile in parallel.
//
// Work decomposition.  The paper gives one GPU thread to each subterm row of one bitstring
// and multiplies/sums with repeated pairwise launches (Section 3.3, Appendix E).  Here a lane
// owns a whole slice of 2^g assignments instead: the high parameters are fixed by the slice
// index, the low g parameters are enumerated in Gray-code order so that one step flips one
// parameter, which XORs one wave-uniform column into the lane's form vector L.  The product
// of all factors of a term is read off popcounts of L (value classes, see the packer): a
// value class (d, r, e) and a power 2^h such that the term is 2^h * w^r sqrt2^e Q(d), with
// the exact Z[w] value of each class in a small int64 table.  Terms are summed per lane in
// int64 or int128 registers (term = table entry shifted by h), or, when that would need the
// wide int128 shift on every term, counted per class in LDS as sums of powers of two and
// multiplied by the table only when the counters are flushed.  Partial sums go lane -> wave
// -> block through shuffles and LDS; a finaliser adds the per-block partials, applies the
// constant and reduces to canonical form.  No floating point is used anywhere.
//
// Image words are read through the constant address space so that every wave-uniform read
// is a scalar load.

#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "image.h"
#include "kernels.h"
#include "zw.h"

namespace {

typedef const __attribute__((address_space(4))) uint32_t CU32;
// whole-entry reads of the image: one scalar load each, which the compiler cannot split
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef const __attribute__((address_space(4))) u32x4 CV4;
typedef const __attribute__((address_space(4))) u32x8 CV8;

__device__ __forceinline__ uint32_t popc(uint32_t x) { return (uint32_t)__builtin_popcount(x); }

__device__ __forceinline__ CU32 *const_words(const uint8_t *img) {
    return (CU32 *)(uintptr_t)img;
}

// A zero the compiler cannot see through: image reads offset by it are not hoisted out of
// loops, so masks needed only on a rare path are read there instead of occupying scalar
// registers for the whole walk.
__device__ __forceinline__ uint32_t opaque_zero() {
    uint32_t z;
    asm volatile("s_mov_b32 %0, 0" : "=s"(z));
    return z;
}

// the per-program statistic and zero masks, kept in scalar registers
template <int W>
struct Slots {
    uint32_t m[kSlots][W];
    uint32_t zm[W];
    const uint32_t *ntab;  // node table in LDS (sets with kSlotsNodeTable)
    uint32_t nmask;        // node bits of word 0
};

// the dynamic LDS of the kernels (value table or class counters, then the node table)
extern __shared__ int64_t s_dyn[];

template <int W, uint32_t SET>
__device__ __forceinline__ void load_slots(const ImgHeader &H, CU32 *wd, Slots<W> &S) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
        if (!((SET >> i) & 1u)) continue;
        CU32 *e = wd + H.off_slots + i * (W + 1);
#pragma unroll
        for (int w = 0; w < slot_words(SET, i, W); ++w) S.m[i][w] = e[1 + w];
    }
#pragma unroll
    for (int w = 0; w < W; ++w) {
        S.zm[w] = wd[H.off_zmask + w];
    }
    if (SET & kSlotsNodeTable) {
        S.ntab = reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(s_dyn) + H.ntab_lds);
        S.nmask = H.ntab_n - 1u;
    }
}

struct TermClass {
    uint32_t cls;  // value class (d, r, e) or the zero entry
    int h;         // the term is 2^h times the class value
    bool zero;
};

// ZERO: test the vanishing bits (a compile-time switch so that the walk of a program without
// such factors carries no test at all)
template <int W, uint32_t SET, bool ZERO>
__device__ __forceinline__ TermClass classify(const ImgHeader &H, const Slots<W> &S, const uint32_t (&L)[W],
                                              int phi) {
    if (SET & kSlotsNodeTable) {
        // node factors from the table; the phase slots count the linear terms
        const uint32_t e = S.ntab[L[0] & S.nmask];
        int rl = H.stat_base[STAT_R];
#pragma unroll
        for (int i = 0; i < kSlots; ++i) {
            if (!((SET >> i) & 1u)) continue;
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) c += popc(L[w] & S.m[i][w]);
            rl += (int)c * slot_weight(i);
        }
        TermClass t;
        t.zero = ZERO && (e & 1u);
        const int R = (int)(e >> 16) + rl + phi;
        const uint32_t E = (e >> 8) & 0xFFu;
        t.cls = ((((e >> 1) & 0x7Fu) << 4) | ((uint32_t)(R & 7) << 1)) | (E & 1u);
        t.h = (int)(E >> 1);
        return t;
    }
    int st[N_STATS];
#pragma unroll
    for (int s = 0; s < N_STATS; ++s) st[s] = H.stat_base[s];
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
        if ((SET >> i) & 1u) {  // compile-time: the slot belongs to this kernel's set
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < slot_words(SET, i, W); ++w) c += popc(L[w] & S.m[i][w]);
            const int wgt = slot_weight(i);
            if (wgt == 1) st[slot_stat(i)] += (int)c;
            else if (wgt == -1) st[slot_stat(i)] -= (int)c;
            else st[slot_stat(i)] += (int)c * wgt;
        }
    }
    TermClass t;
    t.zero = false;
    if (ZERO) {
        uint32_t z = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) z |= L[w] & S.zm[w];
        t.zero = z != 0u;
    }
    const int A = st[STAT_A], B = st[STAT_B];
    const int m = A < B ? A : B;
    const int E = st[STAT_E] + m;
    const int R = st[STAT_R] + 2 * m + phi;
    t.cls = (((uint32_t)(A - B + H.d_off) << 4) | ((uint32_t)(R & 7) << 1)) | (uint32_t)(E & 1);
    t.h = E >> 1;
    return t;
}

// per-lane accumulation state for the three modes
template <int ACC>
struct Acc {
    int64_t a64[4];
    i128 a128[4];
    uint32_t a32[4];  // one block's int64-mode terms, modulo 2^32 (see flush32)
    __device__ void clear() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a64[k] = 0;
            a128[k] = 0;
            a32[k] = 0;
        }
    }
    // With n node factors a term's coordinates are at most 2^n in absolute value (each factor
    // has coefficient sum 2 in the w-basis, and w^r and the linear phases only permute and
    // negate coordinates), so when n + KB <= 30 (header flag block_sum32; always so for
    // node-table programs) the 2^KB terms a lane adds in one block sum to less than 2^31: they
    // are added in 32-bit registers (one shift-and-add each) and moved to the int64 sums after
    // the block.
    static_assert(kMaxTableNodes + kMaxInnerBits < 31, "node-table blocks must fit in int32");
    __device__ void flush32() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a64[k] += (int64_t)(int32_t)a32[k];
            a32[k] = 0;
        }
    }
    // int64 mode with more terms than int64 holds (header flag block_flush128): a block's sums
    // (2^KB terms of at most 2^n per coordinate, n + KB <= 62) move to int128 after the block
    __device__ void flush128() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a128[k] += (i128)a64[k];
            a64[k] = 0;
        }
    }
};

template <int W, int ACC, uint32_t SET, bool ZERO, bool B32 = false>
__device__ __forceinline__ void add_term(const ImgHeader &H, const Slots<W> &S, const int64_t *tab,
                                         unsigned long long *cnt, const uint32_t (&L)[W], int phi, Acc<ACC> &acc) {
    const TermClass t = classify<W, SET, ZERO>(H, S, L, phi);
    if (ACC == ACC_CLASS) {
        if (!t.zero) {
            // counters are laid out [q][class]: 24-bit multiply-add (full rate)
            const uint32_t slot = __umul24((uint32_t)(t.h >> 5), H.zero_entry) + t.cls;
            atomicAdd(cnt + slot, (unsigned long long)(1u << (t.h & 31)));
        }
    } else {
        const uint32_t idx = t.zero ? H.zero_entry : t.cls;
        const longlong2 *p = reinterpret_cast<const longlong2 *>(tab + (size_t)idx * 4);
        const longlong2 v01 = p[0], v23 = p[1];
        if (ACC == ACC_I64 && B32) {
            acc.a32[0] += (uint32_t)v01.x << t.h;
            acc.a32[1] += (uint32_t)v01.y << t.h;
            acc.a32[2] += (uint32_t)v23.x << t.h;
            acc.a32[3] += (uint32_t)v23.y << t.h;
        } else if (ACC == ACC_I64) {
            acc.a64[0] += (int64_t)((uint64_t)v01.x << t.h);
            acc.a64[1] += (int64_t)((uint64_t)v01.y << t.h);
            acc.a64[2] += (int64_t)((uint64_t)v23.x << t.h);
            acc.a64[3] += (int64_t)((uint64_t)v23.y << t.h);
        } else {
            acc.a128[0] += (i128)v01.x << t.h;
            acc.a128[1] += (i128)v01.y << t.h;
            acc.a128[2] += (i128)v23.x << t.h;
            acc.a128[3] += (i128)v23.y << t.h;
        }
    }
}

// field-wise sum mod 8 of two vectors of 4-bit fields holding values 0..7, and negation mod 8
// (8 - x never borrows from the next field)
__device__ __forceinline__ uint32_t field_add(uint32_t a, uint32_t b) { return (a + b) & 0x77777777u; }
__device__ __forceinline__ uint32_t field_neg(uint32_t a) { return (0x88888888u - a) & 0x77777777u; }

// phase change (monomials) of flipping walk position i to its new value (bit i of gray).  The
// walk bits below i are fixed at a flip (bit i-1 set, lower bits clear), so only the entries of
// position i that depend on bits above i are tested; dal holds the always-firing
// slice-dependent changes of every position as 4-bit fields.
__device__ __forceinline__ int flip_phase(const ImgHeader &H, CU32 *wd, uint32_t i, uint32_t gray, uint64_t dal,
                                          uint64_t s) {
    CU32 *didx = wd + H.off_didx;
    const uint32_t e0 = didx[i], e1 = didx[i + 1];
    CU32 *de = wd + H.off_delta + 4 * e0;
    int du = (int)wd[H.off_ui + i];
    int dv = (int)((dal >> (4 * i)) & 7u);
    for (uint32_t e = e0; e < e1; ++e, de += 4) {
        const uint32_t wm = de[1];
        if ((gray & wm) != wm) continue;
        const uint64_t hm = (uint64_t)de[2] | ((uint64_t)de[3] << 32);
        const int c = (int)de[0];
        if (hm == 0) du += c;
        else dv += ((s & hm) == hm) ? c : 0;
    }
    const int dd = du + dv;
    return ((gray >> i) & 1u) ? dd : -dd;
}

// Queue of surviving terms of one wave (programs whose factors can vanish, W <= 4): an entry
// is a term's form vector and phase, padded to 4 or 8 words; terms are appended by ballot and
// prefix count and their statistics evaluated 64 at a time, so that sparse survivors do not
// leave most lanes of a wave idle.  The count is wave-uniform.
constexpr uint32_t kQueueCap = 128;  // one append (<= 64) on top of < 64 pending entries
template <int W>
constexpr bool kCompact = W <= 4;
template <int W>
constexpr int kQueueWords = W + 1;  // the form vector and the phase, packed
struct WaveQueue {
    uint32_t *q;  // this wave's kQueueCap entries in LDS
    uint32_t n;   // pending entries
};

// evaluates the last `count` (<= 64) pending entries, one per lane
template <int W, int ACC, uint32_t SET>
__device__ __forceinline__ void queue_drain(const ImgHeader &H, CU32 *wd, const int64_t *tab,
                                            unsigned long long *cnt, WaveQueue &Q, uint32_t count,
                                            Acc<ACC> &acc) {
    Slots<W> S;
    load_slots<W, SET>(H, wd + opaque_zero(), S);
    const uint32_t lane = threadIdx.x & 63u;
    Q.n -= count;
    __builtin_amdgcn_wave_barrier();
    if (lane < count) {
        const uint32_t *e = Q.q + (Q.n + lane) * kQueueWords<W>;
        uint32_t words[W + 1];
#pragma unroll
        for (int j = 0; j <= W; ++j) words[j] = e[j];
        uint32_t L[W];
#pragma unroll
        for (int w = 0; w < W; ++w) L[w] = words[w];
        add_term<W, ACC, SET, false>(H, S, tab, cnt, L, (int)words[W], acc);
    }
    __builtin_amdgcn_wave_barrier();
}

template <int W>
__device__ __forceinline__ bool words_equal(const uint32_t (&a)[W], const uint32_t (&b)[W]) {
    if (W == 1) return a[0] == b[0];
    if (W == 2) return (((uint64_t)a[1] << 32) | a[0]) == (((uint64_t)b[1] << 32) | b[0]);
    uint32_t x = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) x |= a[w] ^ b[w];
    return x == 0u;
}

// field k of a block's phase vector (NF = 2 or 4 words of 4-bit fields), for a per-lane k: a
// 64-bit half picked by bit 4 of k, then a shift (a select chain over the words would be
// turned into a stack array)
template <int NF>
__device__ __forceinline__ uint32_t field_at(const uint32_t (&fv)[NF], uint32_t k) {
    static_assert(NF == 2 || NF == 4 || NF == 8, "16, 32 or 64 fields");
    uint64_t x = (uint64_t)fv[0] | ((uint64_t)fv[1] << 32);
    if (NF >= 4) {
        const uint64_t h = (uint64_t)fv[2 % NF] | ((uint64_t)fv[3 % NF] << 32);
        x = (k & 16u) ? h : x;
    }
    if (NF == 8) {
        const uint64_t h2 = (uint64_t)fv[4 % NF] | ((uint64_t)fv[5 % NF] << 32);
        const uint64_t h3 = (uint64_t)fv[6 % NF] | ((uint64_t)fv[7 % NF] << 32);
        const uint64_t y = (k & 16u) ? h3 : h2;
        x = (k & 32u) ? y : x;
    }
    return (uint32_t)(x >> (4 * (k & 15u))) & 7u;
}

// bit i of b (8 bits) to bit 4i
__device__ __forceinline__ uint32_t spread8(uint32_t b) {
    b = (b | (b << 12)) & 0x000F000Fu;
    b = (b | (b << 6)) & 0x03030303u;
    return (b | (b << 3)) & 0x11111111u;
}

// Form monomials [e0, e1) of one group: DEG3 forms (else two), coefficient C.  Their 2^KB-bit
// patterns over a block are ANDs of the forms' patterns (a form is its bit of O xor its lambda),
// and C times each pattern is added to three bit planes (a sum mod 8 in bit-sliced form).  The
// entries are read four at a time before any is used, so that one wait covers four scalar loads.
template <int KW, int C, bool DEG3>
__device__ __forceinline__ void fm_group(CV8 *fe, uint32_t e0,
                                         uint32_t e1, uint32_t O, uint32_t (&c0)[KW], uint32_t (&c1)[KW],
                                         uint32_t (&c2)[KW]) {
    auto one = [&](const u32x8 &E) {
        const uint32_t h = E[0];
        const uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int)O, (h >> 16) & 0xFFu, 1u);
        const uint32_t m2 = (uint32_t)__builtin_amdgcn_sbfe((int)O, h >> 24, 1u);
        uint32_t P[KW];
#pragma unroll
        for (int w = 0; w < KW; ++w) P[w] = (E[2 + w] ^ m1) & (E[4 + w] ^ m2);
        if (DEG3) {
            const uint32_t m3 = (uint32_t)__builtin_amdgcn_sbfe((int)O, E[1], 1u);
#pragma unroll
            for (int w = 0; w < KW; ++w) P[w] &= E[6 + w] ^ m3;
        }
#pragma unroll
        for (int w = 0; w < KW; ++w) {
            if (C & 1) {
                const uint32_t t = c0[w] & P[w];
                c0[w] ^= P[w];
                const uint32_t u = c1[w] & t;
                c1[w] ^= t;
                c2[w] ^= u;
            }
            if (C & 2) {
                const uint32_t t = c1[w] & P[w];
                c1[w] ^= P[w];
                c2[w] ^= t;
            }
            if (C & 4) c2[w] ^= P[w];
        }
    };
    uint32_t e = e0;
    for (; e + 4 <= e1; e += 4) {
        u32x8 E[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) E[u] = fe[e + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) one(E[u]);
    }
    for (; e < e1; ++e) {
        const u32x8 E1 = fe[e];
        one(E1);
    }
}

// Adds to ft the phase of the form monomials at each of a block's 2^KB terms, as 4-bit fields
// (field k of word k / 8).  O holds the monomials' forms at the block's first term; at step k a
// form is its bit of O xor bit k of its lambda (the parity of its inner part at gray(k)).  The
// entries come in 14 groups by degree and coefficient (fm_group), and the bit planes become
// fields at the end.
template <int KB, int NF>
__device__ __forceinline__ void form_fields(const ImgHeader &H, CU32 *wd, uint32_t O, uint32_t (&ft)[NF]) {
    constexpr int KW = (1 << KB) >= 32 ? (1 << KB) / 32 : 1;  // 32-bit words of a pattern
    uint32_t c0[KW], c1[KW], c2[KW];
#pragma unroll
    for (int w = 0; w < KW; ++w) c0[w] = c1[w] = c2[w] = 0;
    CV8 *fe = reinterpret_cast<CV8 *>(wd + H.off_fmono);
    CU32 *gb = wd + H.off_fmgrp;
    fm_group<KW, 1, false>(fe, gb[0], gb[1], O, c0, c1, c2);
    fm_group<KW, 2, false>(fe, gb[1], gb[2], O, c0, c1, c2);
    fm_group<KW, 3, false>(fe, gb[2], gb[3], O, c0, c1, c2);
    fm_group<KW, 4, false>(fe, gb[3], gb[4], O, c0, c1, c2);
    fm_group<KW, 5, false>(fe, gb[4], gb[5], O, c0, c1, c2);
    fm_group<KW, 6, false>(fe, gb[5], gb[6], O, c0, c1, c2);
    fm_group<KW, 7, false>(fe, gb[6], gb[7], O, c0, c1, c2);
    fm_group<KW, 1, true>(fe, gb[7], gb[8], O, c0, c1, c2);
    fm_group<KW, 2, true>(fe, gb[8], gb[9], O, c0, c1, c2);
    fm_group<KW, 3, true>(fe, gb[9], gb[10], O, c0, c1, c2);
    fm_group<KW, 4, true>(fe, gb[10], gb[11], O, c0, c1, c2);
    fm_group<KW, 5, true>(fe, gb[11], gb[12], O, c0, c1, c2);
    fm_group<KW, 6, true>(fe, gb[12], gb[13], O, c0, c1, c2);
    fm_group<KW, 7, true>(fe, gb[13], gb[14], O, c0, c1, c2);
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        const int wi = (8 * j) / 32, sh = (8 * j) % 32;
        const uint32_t f = spread8((c0[wi] >> sh) & 0xFFu) | (spread8((c1[wi] >> sh) & 0xFFu) << 1) |
                           (spread8((c2[wi] >> sh) & 0xFFu) << 2);
        ft[j] = field_add(ft[j], f);
    }
}

// form_fields for one half of a 64-term block (steps 0..31 or 32..63), from that half's table
// (ht: two-form entries from word 0, three-form entries from word off3): the patterns' one
// word of the half, and the four field words of that half.  gb holds the 15 group bounds.
//
// A group (one coefficient C) first counts, per step, how many of its monomials are 1 there
// (mod 8, three bit planes t) with carry-save adders over four patterns at a time, so the
// patterns of a batch are independent and the planes take few dependent operations; C * t is
// then added to the block's planes c once per group.
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) { return (a & b) | (a & c) | (b & c); }

// (c0, c1, c2) += (u0, u1, u2) mod 8, bit-sliced
__device__ __forceinline__ void planes_add(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t u0, uint32_t u1,
                                           uint32_t u2) {
    const uint32_t k1 = c0 & u0;
    c0 ^= u0;
    const uint32_t k2 = maj3(c1, u1, k1);
    c1 ^= u1 ^ k1;
    c2 ^= u2 ^ k2;
}

template <int C>
__device__ __forceinline__ void planes_add_times(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t t0, uint32_t t1,
                                                 uint32_t t2) {
    // C * t mod 8 from t, 2t = (0, t0, t1) and 4t = (0, 0, t0)
    if (C & 1) planes_add(c0, c1, c2, t0, t1, t2);
    if (C & 2) planes_add(c0, c1, c2, 0u, t0, t1);
    if (C & 4) c2 ^= t0;
}

template <int C, bool DEG3>
__device__ __forceinline__ void fmh_group(const uint4 *t, uint32_t e0, uint32_t e1, uint32_t O, uint32_t &c0,
                                          uint32_t &c1, uint32_t &c2) {
    if (e0 >= e1) return;
    uint32_t t0 = 0, t1 = 0, t2 = 0;
    auto pat = [&](uint32_t j1, uint32_t j2, uint32_t j3, uint32_t l1, uint32_t l2, uint32_t l3) {
        const uint32_t m1 = (uint32_t)__builtin_amdgcn_sbfe((int)O, j1, 1u);
        const uint32_t m2 = (uint32_t)__builtin_amdgcn_sbfe((int)O, j2, 1u);
        uint32_t P = (l1 ^ m1) & (l2 ^ m2);
        if (DEG3) P &= l3 ^ (uint32_t)__builtin_amdgcn_sbfe((int)O, j3, 1u);
        return P;
    };
    auto add4 = [&](uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
        const uint32_t s1 = t0 ^ a ^ b, k1 = maj3(t0, a, b);
        t0 = s1 ^ c ^ d;
        const uint32_t k2 = maj3(s1, c, d);
        t2 ^= maj3(t1, k1, k2);
        t1 ^= k1 ^ k2;
    };
    // the groups are whole batches (padded with null entries), read from LDS with the same
    // address in every lane (broadcast reads, returned in order)
    if (DEG3) {
        for (uint32_t e = e0; e < e1; e += 4) {
            uint4 A[4], B[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                A[u] = t[2 * (e + u)];
                B[u] = t[2 * (e + u) + 1];
            }
            uint32_t P[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) P[u] = pat(A[u].x, A[u].y, A[u].z, A[u].w, B[u].x, B[u].y);
            add4(P[0], P[1], P[2], P[3]);
        }
    } else {
        for (uint32_t e = e0; e < e1; e += 8) {
            uint4 E[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) E[u] = t[e + u];
            uint32_t P[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) P[u] = pat(E[u].x, E[u].y, 0u, E[u].z, E[u].w, 0u);
            add4(P[0], P[1], P[2], P[3]);
            add4(P[4], P[5], P[6], P[7]);
        }
    }
    planes_add_times<C>(c0, c1, c2, t0, t1, t2);
}

__device__ __forceinline__ void form_fields_half(const uint4 *ht, uint32_t off3, const uint32_t (&gb)[16], uint32_t O,
                                                 uint32_t hsel, uint32_t (&ft)[8]) {
    uint32_t c0 = 0, c1 = 0, c2 = 0;
    const uint4 *t3 = ht + off3 / 4;  // three-form entries
    fmh_group<1, false>(ht, gb[0], gb[1], O, c0, c1, c2);
    fmh_group<2, false>(ht, gb[1], gb[2], O, c0, c1, c2);
    fmh_group<3, false>(ht, gb[2], gb[3], O, c0, c1, c2);
    fmh_group<4, false>(ht, gb[3], gb[4], O, c0, c1, c2);
    fmh_group<5, false>(ht, gb[4], gb[5], O, c0, c1, c2);
    fmh_group<6, false>(ht, gb[5], gb[6], O, c0, c1, c2);
    fmh_group<7, false>(ht, gb[6], gb[7], O, c0, c1, c2);
    fmh_group<1, true>(t3, gb[8], gb[9], O, c0, c1, c2);
    fmh_group<2, true>(t3, gb[9], gb[10], O, c0, c1, c2);
    fmh_group<3, true>(t3, gb[10], gb[11], O, c0, c1, c2);
    fmh_group<4, true>(t3, gb[11], gb[12], O, c0, c1, c2);
    fmh_group<5, true>(t3, gb[12], gb[13], O, c0, c1, c2);
    fmh_group<6, true>(t3, gb[13], gb[14], O, c0, c1, c2);
    fmh_group<7, true>(t3, gb[14], gb[15], O, c0, c1, c2);
    uint32_t f[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
        f[j] = spread8((c0 >> (8 * j)) & 0xFFu) | (spread8((c1 >> (8 * j)) & 0xFFu) << 1) |
               (spread8((c2 >> (8 * j)) & 0xFFu) << 2);
    if (hsel == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) ft[j] = field_add(ft[j], f[j]);
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) ft[4 + j] = field_add(ft[4 + j], f[j]);
    }
}

// phase of the form monomials at one term whose forms' values are the bits of O (short walks)
__device__ __forceinline__ int form_phase(const ImgHeader &H, CU32 *wd, uint32_t O) {
    CV8 *fe = reinterpret_cast<CV8 *>(wd + H.off_fmono);
    int ph = 0;
    for (uint32_t e = 0; e < H.n_fmono; ++e) {
        const u32x8 E = fe[e];
        const uint32_t h = E[0];
        uint32_t v = (O >> ((h >> 16) & 0xFFu)) & (O >> (h >> 24));
        if (((h >> 8) & 3u) == 3u) v &= O >> E[1];
        ph += (v & 1u) ? (int)(h & 7u) : 0;
    }
    return ph;
}

// The blocks of a slice: 2^(g - KB) blocks of 2^KB terms.  Between blocks one
// outer walk position flips (column XOR, phase change from the position's lists); inside a
// block the flip positions are compile-time constants, the inner columns sit in registers and
// the phase of each term is read from the block's vector of 4-bit fields.
// With ZERO and CQ (compacting), lanes whose slice is past the end of the range still walk
// (valid = false) and never report a surviving term, so the queue is always operated on by
// the whole wave.
// Blocks [b0, b1) of the slice are walked; L and phi hold the state of block b0's first term.
template <int W, bool MONO, int ACC, uint32_t SET, bool ZERO, bool CQ, bool ZT, bool B32 = false>
__device__ __forceinline__ void walk_blocks(const ImgHeader &H, const Slots<W> &S, CU32 *wd, const int64_t *tab,
                                            unsigned long long *cnt, uint64_t s, bool valid, uint32_t b0,
                                            uint32_t b1, uint32_t (&L)[W], int phi, uint64_t dal, uint32_t Sf,
                                            WaveQueue *Q, Acc<ACC> &acc, uint32_t half = 0) {
    constexpr int KB = inner_bits_for(W);  // inner bits of a block
    constexpr int KS = 1 << KB;             // its terms
    constexpr int NF = KS / 8;              // words of its 4-bit phase fields
    static_assert(!B32 || (ACC == ACC_I64 && !CQ), "32-bit block sums: int64 mode, walks without a queue");
    CU32 *col = wd + H.off_col;
    uint32_t ck[KB][W];
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
        for (int w = 0; w < W; ++w) ck[j][w] = col[j * W + w];
    uint32_t cz[KB][W];  // the inner columns on the vanishing bits
#pragma unroll
    for (int j = 0; j < KB; ++j)
#pragma unroll
        for (int w = 0; w < W; ++w) cz[j][w] = ck[j][w] & S.zm[w];
    // per lane: the masked start vector of a block is (L & zmv) | nvv, the never-matching
    // pattern on lanes without a slice
    uint32_t zmv[W], nvv[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        zmv[w] = valid ? S.zm[w] : 0u;
        nvv[w] = valid ? 0u : wd[H.off_never + w];
    }
    // the inner phase vectors of the current outer state (even and odd blocks)
    uint32_t v0[NF], v1[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) v0[j] = v1[j] = 0;
    if (MONO) {
        CU32 *ci = wd + H.off_inner;
#pragma unroll
        for (int j = 0; j < NF; ++j) {
            v0[j] = ci[j];
            v1[j] = ci[NF + j];
        }
        CU32 *e2 = wd + H.off_c2;
        #pragma unroll 4
        for (uint32_t e = 0; e < H.n_c2; ++e, e2 += 2 * NF + 2) {
            const uint64_t hm = (uint64_t)e2[2 * NF] | ((uint64_t)e2[2 * NF + 1] << 32);
            if ((s & hm) == hm) {
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    v0[j] = field_add(v0[j], e2[j]);
                    v1[j] = field_add(v1[j], e2[NF + j]);
                }
            }
        }
    }
    uint32_t gray = (b0 ^ (b0 >> 1)) << KB;  // walk bits at or above KB
    // the outer walk parts of the form monomials' forms at the current walk state (uniform)
    uint32_t G = 0;
    // the form monomials' padded group bounds of the half tables, read once (teams of two waves)
    uint32_t gbv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) gbv[k] = 0;
    if (MONO && H.n_fmono) {
        CU32 *gc = wd + H.off_gcol;
        for (uint32_t bits = gray; bits; bits &= bits - 1u) G ^= gc[__builtin_ctz(bits)];
        if (KB == 6 && half) {
            CU32 *gb = wd + H.off_fmh;
#pragma unroll
            for (int k = 0; k < 16; ++k) gbv[k] = gb[k];
        }
    }
    if (MONO && b0) {
        // inner-and-outer monomials already switched on at the start state
        CU32 *e3 = wd + H.off_c3all;
        #pragma unroll 4
        for (uint32_t e = 0; e < H.n_c3all; ++e, e3 += 2 * NF + 3) {
            const uint32_t om = e3[2 * NF];
            if ((gray & om) != om) continue;
            const uint64_t hm = (uint64_t)e3[2 * NF + 1] | ((uint64_t)e3[2 * NF + 2] << 32);
            if ((s & hm) == hm) {
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    v0[j] = field_add(v0[j], e3[j]);
                    v1[j] = field_add(v1[j], e3[NF + j]);
                }
            }
        }
    }
    // What the flip at the start of the next block reads (its column and its position record)
    // is loaded one block ahead, so that the scalar loads overlap the current block's work
    // instead of stalling the flip.
    CV4 *recs = reinterpret_cast<CV4 *>(wd + H.off_pos);
    uint32_t cn[W];
    // ui; flip entries [lo, hi) of word 1 (16 bits each); inner-vector entries [lo, hi) of word 2
    u32x4 rn = {0, 0, 0, 0};
    if (b0 + 1 < b1) {
        const uint32_t i = KB + (uint32_t)__builtin_ctz(b0 + 1);
#pragma unroll
        for (int w = 0; w < W; ++w) cn[w] = col[i * W + w];
        if (MONO) rn = recs[i];
    }
    for (uint32_t b = b0; b < b1; ++b) {
        if (b != b0) {
            const uint32_t i = KB + (uint32_t)__builtin_ctz(b);
            gray ^= 1u << i;
#pragma unroll
            for (int w = 0; w < W; ++w) L[w] ^= cn[w];
            const u32x4 r = rn;
            if (b + 1 < b1) {
                const uint32_t in = KB + (uint32_t)__builtin_ctz(b + 1);
#pragma unroll
                for (int w = 0; w < W; ++w) cn[w] = col[in * W + w];
                if (MONO) rn = recs[in];
            }
            if (MONO) {
                // the phase change of the flip: uniform and always-firing parts, then the
                // entries that depend on walk bits above i
                int dd = (int)r[0] + (int)((dal >> (4 * i)) & 7u);
                CV4 *de = reinterpret_cast<CV4 *>(wd + H.off_delta);
                for (uint32_t e = r[1] & 0xFFFFu; e < (r[1] >> 16); ++e) {
                    const u32x4 d = de[e];  // c, walk mask, slice mask lo, hi
                    const uint32_t c = d[0], wm = d[1], hl = d[2], hh = d[3];
                    if ((gray & wm) != wm) continue;
                    const uint64_t hm = (uint64_t)hl | ((uint64_t)hh << 32);
                    dd += ((s & hm) == hm) ? (int)c : 0;
                }
                phi += ((gray >> i) & 1u) ? dd : -dd;
                G ^= r[3];
                // inner vectors of the monomials that also need outer bits: those of position i
                // whose other outer bits are set switch on (bit i now 1) or off
                const bool on = (gray >> i) & 1u;
                CV8 *e3 = reinterpret_cast<CV8 *>(wd + H.off_c3);
                for (uint32_t e = r[2] & 0xFFFFu; e < (r[2] >> 16); ++e) {
                    // even[NF], odd[NF], other outer bits, slice mask lo, hi (4 NF words)
                    uint32_t v[4 * NF];
#pragma unroll
                    for (int h = 0; h < NF / 2; ++h) {
                        const u32x8 part = e3[(NF / 2) * e + h];
#pragma unroll
                        for (int j = 0; j < 8; ++j) v[8 * h + j] = part[j];
                    }
                    const uint32_t om = v[2 * NF], hl = v[2 * NF + 1], hh = v[2 * NF + 2];
                    if ((gray & om) != om) continue;
                    if (!on) {
#pragma unroll
                        for (int j = 0; j < 2 * NF; ++j) v[j] = field_neg(v[j]);
                    }
                    const uint64_t hm = (uint64_t)hl | ((uint64_t)hh << 32);
                    if ((s & hm) == hm) {
#pragma unroll
                        for (int j = 0; j < NF; ++j) {
                            v0[j] = field_add(v0[j], v[j]);
                            v1[j] = field_add(v1[j], v[NF + j]);
                        }
                    }
                }
            }
        }
        uint32_t fv[NF];  // the phase fields of this block's terms
#pragma unroll
        for (int j = 0; j < NF; ++j) fv[j] = 0;
        if (MONO) {
            const bool odd = b & 1u;
#pragma unroll
            for (int j = 0; j < NF; ++j) fv[j] = odd ? v1[j] : v0[j];
        }
        if (ZERO && CQ && ZT) {
            // The vanishing bits lie in word 0: a = L0 & zm is looked up in a hashed LDS table of
            // the keys P(gray(k)) & zm with the masks of their steps (no key a: no survivor), and
            // each round every lane with a survivor left appends one, while any lane has one.
            const uint32_t *zt =
                reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(tab) + H.ztab_lds);
            const uint32_t a = L[0] & S.zm[0];
            const uint4 ent = reinterpret_cast<const uint4 *>(zt)[(a * H.ztab_mult) >> H.ztab_shift];
            uint64_t hits = valid && ent.x == a ? ((uint64_t)ent.z << 32) | ent.y : 0ull;
            const uint32_t nz = 4 * ztab_slots_for(KB);  // words of the hashed table: P(gray(k)) follow
            for (;;) {
                const uint64_t m = __ballot(hits != 0u);
                if (!m) break;
                const uint32_t below =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (hits) {
                    const uint32_t k = (uint32_t)__builtin_ctzll(hits);
                    hits &= hits - 1u;
                    const uint32_t *pk = zt + nz + k * W;  // P(gray(k))
                    uint32_t words[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                    for (int w = 0; w < W; ++w) words[w] = L[w] ^ pk[w];
                    const int f = MONO ? (int)field_at<NF>(fv, k) : 0;
                    words[W] = (uint32_t)(phi + f);
                    uint32_t *e = Q->q + (Q->n + below) * kQueueWords<W>;
#pragma unroll
                    for (int j = 0; j <= W; ++j) e[j] = words[j];
                }
                Q->n += (uint32_t)__popcll(m);
                if (Q->n >= 64u) queue_drain<W, ACC, SET>(H, wd, tab, cnt, *Q, 64u, acc);
            }
            // the block's last state: gray(KS - 1) has only the top inner bit set
#pragma unroll
            for (int w = 0; w < W; ++w) L[w] ^= ck[KB - 1][w];
        } else if (ZERO && CQ) {  // !ZT
            // Term k of the block has L0 ^ P(gray(k)), P the XOR of the inner columns of the set
            // bits, and survives iff a = (L0 & zm) equals P(gray(k)) & zm.  The coordinates of a
            // in the reduced basis of those vectors are its pivot bits; a is in their span iff
            // removing the picked basis vectors leaves zero, and then y = gray(k) of one
            // surviving step follows from the basis vectors' inner-column combinations (the
            // others are y ^ the null-space combinations).
            uint32_t a[W], x[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                a[w] = (L[w] & zmv[w]) | nvv[w];
                x[w] = a[w];
            }
            uint32_t y = 0;
            CU32 *bs = wd + H.off_ibasis;
#pragma unroll
            for (int i = 0; i < KB; ++i) {  // padded with all-zero entries past the rank
                CU32 *e = bs + i * (3 + W);
                const uint32_t pw = e[0], pb = e[1], cm = e[2];
                uint32_t aw = a[0];
#pragma unroll
                for (int w = 1; w < W; ++w) aw = pw == (uint32_t)w ? a[w] : aw;
                const uint32_t m = 0u - ((aw >> pb) & 1u);
#pragma unroll
                for (int w = 0; w < W; ++w) x[w] ^= e[3 + w] & m;
                y ^= cm & m;
            }
            uint32_t zero[W];
#pragma unroll
            for (int w = 0; w < W; ++w) zero[w] = 0;
            const bool hit = words_equal<W>(x, zero);
            const uint64_t m = __ballot(hit);
            if (m) {
                // pass 2: append each lane's surviving terms (L0 ^ P(gray(k)), phase) to the queue
                const uint32_t below =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const uint32_t n_kern = KB - H.inner_rank;
                CU32 *kn = wd + H.off_ikern;
                for (uint32_t z = 0; z < (1u << n_kern); ++z) {
                    uint32_t yz = y;
                    for (uint32_t t = 0; t < n_kern; ++t)
                        if ((z >> t) & 1u) yz ^= kn[t];
                    if (hit) {
                        uint32_t k = yz;  // the step with gray(k) = yz (prefix XOR of its bits)
                        k ^= k >> 1;
                        k ^= k >> 2;
                        k ^= k >> 4;
                        uint32_t words[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                        for (int w = 0; w < W; ++w) words[w] = L[w];
#pragma unroll
                        for (int j = 0; j < KB; ++j) {
                            const uint32_t mj = 0u - ((yz >> j) & 1u);
#pragma unroll
                            for (int w = 0; w < W; ++w) words[w] ^= ck[j][w] & mj;
                        }
                        const int f = MONO ? (int)field_at<NF>(fv, k) : 0;
                        words[W] = (uint32_t)(phi + f);
                        uint32_t *e = Q->q + (Q->n + below) * kQueueWords<W>;
#pragma unroll
                        for (int j = 0; j <= W; ++j) e[j] = words[j];
                    }
                    Q->n += (uint32_t)__popcll(m);
                    if (Q->n >= 64u) queue_drain<W, ACC, SET>(H, wd, tab, cnt, *Q, 64u, acc);
                }
            }
            // the block's last state: gray(KS - 1) has only the top inner bit set
#pragma unroll
            for (int w = 0; w < W; ++w) L[w] ^= ck[KB - 1][w];
        } else if (ZERO) {
            // wide form vectors: compare with each step's value, evaluate the survivors in place
            uint32_t a[W];
#pragma unroll
            for (int w = 0; w < W; ++w) a[w] = (L[w] & zmv[w]) | nvv[w];
            uint32_t d[W];
#pragma unroll
            for (int w = 0; w < W; ++w) d[w] = opaque_zero();
            uint64_t any = 0;
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                if (k) {
#pragma unroll
                    for (int w = 0; w < W; ++w) d[w] ^= cz[__builtin_ctz(k)][w];
                }
                any |= __ballot(words_equal<W>(a, d));
            }
            if (any) {
                uint32_t Lk[W];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    Lk[w] = L[w];
                    d[w] = 0;
                }
#pragma unroll
                for (int k = 0; k < KS; ++k) {
                    if (k) {
                        const int j = __builtin_ctz(k);
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            Lk[w] ^= ck[j][w];
                            d[w] ^= cz[j][w];
                        }
                    }
                    if (words_equal<W>(a, d)) {
                        const int f = MONO ? (int)((fv[k >> 3] >> (4 * (k & 7))) & 7u) : 0;
                        add_term<W, ACC, SET, false, B32>(H, S, tab, cnt, Lk, phi + f, acc);
                    }
                }
            }
            // the block's last state: gray(KS - 1) has only the top inner bit set
#pragma unroll
            for (int w = 0; w < W; ++w) L[w] ^= ck[KB - 1][w];
        } else if (KB == 6 && half) {
            // a team of two waves shares the walk: this one evaluates half of the block's terms
            // (steps 0..31 or 32..63) with the form monomials' fields of that half only; the
            // block's last state follows as usual.  (Programs without variable monomials.)
            uint32_t L0[W];
#pragma unroll
            for (int w = 0; w < W; ++w) L0[w] = L[w];
            uint32_t ft[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            const uint32_t hsel = half - 1u;
            if (MONO && H.n_fmono)
                form_fields_half(reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(tab) + H.fmh_lds) +
                                     (16 + hsel * H.fmh_stride) / 4,
                                 H.fmh_off3, gbv,
                                 Sf ^ G ^ ((b & 1u) ? H.gcol_top : 0u), hsel, ft);
            if (hsel == 0) {
                add_term<W, ACC, SET, false, B32>(H, S, tab, cnt, L, phi + (int)(ft[0] & 7u), acc);
#pragma unroll
                for (int k = 1; k < 32; ++k) {
                    const int j = __builtin_ctz(k);
#pragma unroll
                    for (int w = 0; w < W; ++w) L[w] ^= ck[j][w];
                    add_term<W, ACC, SET, false, B32>(H, S, tab, cnt, L,
                                                     phi + (int)((ft[k >> 3] >> (4 * (k & 7))) & 7u), acc);
                }
            } else {
#pragma unroll
                for (int w = 0; w < W; ++w) L[w] ^= ck[4 % KB][w] ^ ck[5 % KB][w];  // gray(32) = 48
                add_term<W, ACC, SET, false, B32>(H, S, tab, cnt, L, phi + (int)(ft[4] & 7u), acc);
#pragma unroll
                for (int k = 33; k < 64; ++k) {
                    const int j = __builtin_ctz(k);
#pragma unroll
                    for (int w = 0; w < W; ++w) L[w] ^= ck[j % KB][w];
                    add_term<W, ACC, SET, false, B32>(H, S, tab, cnt, L,
                                                     phi + (int)((ft[(k >> 3) % NF] >> (4 * (k & 7))) & 7u), acc);
                }
            }
#pragma unroll
            for (int w = 0; w < W; ++w) L[w] = L0[w] ^ ck[KB - 1][w];
        } else {
            // with form monomials, their absolute phase at each term joins the block's fields
            // (fv itself, relative to the first term, keeps carrying phi across blocks)
            uint32_t ft[NF];
#pragma unroll
            for (int j = 0; j < NF; ++j) ft[j] = fv[j];
            if (MONO && H.n_fmono) form_fields<KB, NF>(H, wd, Sf ^ G ^ ((b & 1u) ? H.gcol_top : 0u), ft);
            add_term<W, ACC, SET, false, B32>(H, S, tab, cnt, L, phi + (MONO ? (int)(ft[0] & 7u) : 0), acc);
#pragma unroll
            for (int k = 1; k < KS; ++k) {
                const int j = __builtin_ctz(k);
#pragma unroll
                for (int w = 0; w < W; ++w) L[w] ^= ck[j][w];
                const int f = MONO ? (int)((ft[k >> 3] >> (4 * (k & 7))) & 7u) : 0;
                add_term<W, ACC, SET, false, B32>(H, S, tab, cnt, L, phi + f, acc);
            }
        }
        if (B32) acc.flush32();
        if (ACC == ACC_I64 && H.block_flush128) acc.flush128();
        if (MONO) phi += (int)(fv[NF - 1] >> 28);  // the block's last state
    }
}

// Assignments of slice s (high parameters = bits of s): blocks [b0, b1) of its walk, or with
// fewer than KB walk bits the whole walk (b0 = 0, b1 = 1).  CQ: the compacting walk of a
// program with vanishing factors and at least KB walk bits (called by the whole wave,
// valid marks the lanes with a slice); otherwise every other kind of program.
template <int W, bool MONO, int ACC, uint32_t SET, bool CQ>
__device__ __forceinline__ void run_slice(const ImgHeader &H, CU32 *wd, const int64_t *tab, unsigned long long *cnt,
                                          uint64_t s, bool valid, uint32_t b0, uint32_t b1, WaveQueue *Q,
                                          Acc<ACC> &acc, uint32_t half = 0) {
    // the compacting walk needs only the vanishing masks (the queue reads the statistic
    // masks when it evaluates terms)
    Slots<W> S;
    if (CQ) {
#pragma unroll
        for (int w = 0; w < W; ++w) S.zm[w] = wd[H.off_zmask + w];
    } else {
        load_slots<W, SET>(H, wd + opaque_zero(), S);
    }
    CU32 *col = wd + H.off_col;
    uint32_t L[W];
#pragma unroll
    for (int w = 0; w < W; ++w) L[w] = wd[H.off_cvec + w];
    // the high parameters of the slice into L, and into the form monomials' forms (S: their
    // constants and slice parts, one column of forms per slice bit)
    const bool fm = MONO && H.n_fmono;
    uint32_t Sf = fm ? H.fm_s0 : 0u;
    CU32 *scol = wd + H.off_scol - H.g;
    #pragma unroll 4
    for (uint32_t j = H.g; j < H.pe; ++j) {
        const uint32_t m = 0u - (uint32_t)((s >> (j - H.g)) & 1u);
#pragma unroll
        for (int w = 0; w < W; ++w) L[w] ^= col[j * W + w] & m;
        if (fm) Sf ^= scol[j] & m;
    }
    int phi = 0;
    uint64_t dal = 0;  // 4-bit field i: always-firing slice-dependent change at a flip of i (mod 8)
    if (MONO) {
        CU32 *mh = wd + H.off_monohi;
        #pragma unroll 4
        for (uint32_t e = 0; e < H.n_monohi; ++e, mh += 3) {
            const uint64_t hm = (uint64_t)mh[1] | ((uint64_t)mh[2] << 32);
            phi += ((s & hm) == hm) ? (int)mh[0] : 0;
        }
        CU32 *aidx = wd + H.off_aidx;
        const uint32_t n_al = aidx[H.g];  // entries of all positions (none: skip the walk)
        for (uint32_t i = 0; i < (n_al ? H.g : 0u); ++i) {
            int f = 0;
            CU32 *ae = wd + H.off_al + 3 * aidx[i];
            #pragma unroll 4
            for (uint32_t e = aidx[i]; e < aidx[i + 1]; ++e, ae += 3) {
                const uint64_t hm = (uint64_t)ae[1] | ((uint64_t)ae[2] << 32);
                f += ((s & hm) == hm) ? (int)ae[0] : 0;
            }
            dal |= (uint64_t)(f & 7) << (4 * i);
        }
    }
    // the form monomials' forms at the slice's first assignment, without their walk parts
    if (b0) {
        // the walk starts at block b0: its first state has the walk bits of gray(b0 * 2^K)
        const uint32_t t0 = b0 << inner_bits_for(W);
        const uint32_t g0 = t0 ^ (t0 >> 1);
        for (uint32_t bits = g0; bits; bits &= bits - 1u) {
            const uint32_t j = (uint32_t)__builtin_ctz(bits);
#pragma unroll
            for (int w = 0; w < W; ++w) L[w] ^= col[j * W + w];
        }
        if (MONO) {
            CU32 *mw = wd + H.off_monowalk;
            #pragma unroll 4
            for (uint32_t e = 0; e < H.n_monowalk; ++e, mw += 4) {
                const uint32_t wm = mw[1];
                if ((g0 & wm) != wm) continue;
                const uint64_t hm = (uint64_t)mw[2] | ((uint64_t)mw[3] << 32);
                phi += ((s & hm) == hm) ? (int)mw[0] : 0;
            }
        }
    }
    if (CQ) {
        // the table of surviving steps or the reduced-basis test, chosen once per slice (two
        // copies of the loop, so that neither holds the other's registers)
        if (H.ztab_bits)
            walk_blocks<W, MONO, ACC, SET, true, true, true>(H, S, wd, tab, cnt, s, valid, b0, b1, L, phi, dal, Sf, Q, acc);
        else
            walk_blocks<W, MONO, ACC, SET, true, true, false>(H, S, wd, tab, cnt, s, valid, b0, b1, L, phi, dal, Sf, Q,
                                                               acc);
        return;
    }
    if (H.g >= (uint32_t)inner_bits_for(W)) {
        // int64 node-table and node-word-0 kernels add a block's terms in 32 bits where the
        // header allows it
        constexpr bool B32_OK = ACC == ACC_I64 && (SET & (kSlotsNodeTable | kSlotsNodeWord0)) != 0;
        const bool b32 = B32_OK && H.block_sum32;
        if (!H.has_zero) {
            if (b32)
                walk_blocks<W, MONO, ACC, SET, false, false, false, B32_OK>(H, S, wd, tab, cnt, s, true, b0, b1, L, phi,
                                                                           dal, Sf, Q, acc, half);
            else
                walk_blocks<W, MONO, ACC, SET, false, false, false>(H, S, wd, tab, cnt, s, true, b0, b1, L, phi, dal, Sf,
                                                                    Q, acc, half);
        } else if (!kCompact<W>) {
            if (b32)
                walk_blocks<W, MONO, ACC, SET, true, false, false, B32_OK>(H, S, wd, tab, cnt, s, true, b0, b1, L, phi,
                                                                          dal, Sf, Q, acc);
            else
                walk_blocks<W, MONO, ACC, SET, true, false, false>(H, S, wd, tab, cnt, s, true, b0, b1, L, phi, dal, Sf, Q,
                                                                   acc);
        }
        return;
    }
    // short walks: one step at a time (form monomials evaluated per term)
    uint32_t Of = Sf;
    add_term<W, ACC, SET, true>(H, S, tab, cnt, L, phi + (fm ? form_phase(H, wd, Of) : 0), acc);
    uint32_t gray = 0;
    for (uint32_t t = 1; t < (1u << H.g); ++t) {
        const uint32_t i = (uint32_t)__builtin_ctz(t);
        gray ^= 1u << i;
#pragma unroll
        for (int w = 0; w < W; ++w) L[w] ^= col[i * W + w];
        if (MONO) phi += flip_phase(H, wd, i, gray, dal, s);
        if (fm) Of ^= wd[H.off_gcol + i];
        add_term<W, ACC, SET, true>(H, S, tab, cnt, L, phi + (fm ? form_phase(H, wd, Of) : 0), acc);
    }
}

// v moved across lanes by one DPP pattern (four 32-bit moves); lanes the pattern does not
// write, or whose source is out of range, get 0
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ i128 dpp_i128(i128 v) {
    const unsigned __int128 u = (unsigned __int128)v;
    const uint32_t p0 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROWS, BANKS, true);
    const uint32_t p1 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROWS, BANKS, true);
    const uint32_t p2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 64), CTRL, ROWS, BANKS, true);
    const uint32_t p3 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 96), CTRL, ROWS, BANKS, true);
    return (i128)((unsigned __int128)p0 | ((unsigned __int128)p1 << 32) | ((unsigned __int128)p2 << 64) |
                  ((unsigned __int128)p3 << 96));
}

// sum of v over the wave, in lane 63: windows of 4, 8 and 16 lanes within each row of 16
// (row shifts), then the rows' sums through the row broadcasts of lanes 15 and 31
__device__ __forceinline__ i128 wave_sum_to_lane63(i128 v) {
    i128 a = v + dpp_i128<0x111, 0xf, 0xf>(v);   // row_shr:1
    a += dpp_i128<0x112, 0xf, 0xf>(v);           // row_shr:2
    a += dpp_i128<0x113, 0xf, 0xf>(v);           // row_shr:3
    a += dpp_i128<0x114, 0xf, 0xe>(a);           // row_shr:4, lanes 4..15 of a row
    a += dpp_i128<0x118, 0xf, 0xc>(a);           // row_shr:8, lanes 8..15
    a += dpp_i128<0x142, 0xa, 0xf>(a);           // row_bcast:15 into rows 1 and 3
    a += dpp_i128<0x143, 0xc, 0xf>(a);           // row_bcast:31 into rows 2 and 3
    return a;
}

// sum of acc over the block (per wave by cross-lane moves, then LDS in wave order), written by
// thread 0.  Integer addition is associative, so the result does not depend on the order.
__device__ __forceinline__ void block_reduce_store(i128 (&acc)[4], Partial *out) {
    __shared__ i128 s_red[kMaxThreads / 64][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = wave_sum_to_lane63(acc[k]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s_red[wave][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        i128 tot[4] = {0, 0, 0, 0};
        for (int w = 0; w < nw; ++w)
            for (int k = 0; k < 4; ++k) tot[k] += s_red[w][k];
        for (int k = 0; k < 4; ++k) {
            out->w[2 * k] = (uint64_t)tot[k];
            out->w[2 * k + 1] = (uint64_t)((unsigned __int128)tot[k] >> 64);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ i128 load_i128(const uint64_t *w) {
    return (i128)((unsigned __int128)w[0] | ((unsigned __int128)w[1] << 64));
}

// class counters -> int128 accumulators: counter (class, q) holds sum of 2^(h - 32q) over the
// terms of that class with h >> 5 == q; its value is that times 2^(32q) times the class entry
template <int ACC>
__device__ __forceinline__ void flush_counters(const ImgHeader &H, const int64_t *__restrict__ gtab,
                                               unsigned long long *cnt, i128 (&out)[4]) {
    if (ACC != ACC_CLASS) return;
    __syncthreads();
    const uint32_t n = H.zero_entry * H.q_limbs;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const unsigned long long c = cnt[i];
        if (!c) continue;
        cnt[i] = 0;
        const uint32_t q = i / H.zero_entry, cls = i - q * H.zero_entry;
        const int64_t *v = gtab + (size_t)cls * 4;
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] += ((i128)c * (i128)v[k]) << (32 * q);
    }
    __syncthreads();
}

template <int ACC>
__device__ __forceinline__ void acc_to_i128(Acc<ACC> &acc, i128 (&out)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (ACC == ACC_I64) out[k] += (i128)acc.a64[k] + acc.a128[k];
        if (ACC == ACC_I128) out[k] += acc.a128[k];
    }
    acc.clear();
}

// shared-memory prologue of a program: value table (register modes) or zeroed counters
template <int ACC>
__device__ __forceinline__ void prepare_lds(const ImgHeader &H, const int64_t *__restrict__ gtab,
                                            int64_t *s_tab, unsigned long long *s_cnt) {
    if (ACC == ACC_CLASS) {
        const uint32_t n = H.zero_entry * H.q_limbs;
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s_cnt[i] = 0;
    } else {
        // the value table from its base entries Q(d) (r = 0, e = 0): each thread builds the 16
        // entries w^r sqrt2^e Q(d) of one d (negacyclic rotations, one product with sqrt2), so a
        // workgroup loads one entry per d instead of all of them
        const uint32_t nd = H.zero_entry / 16;
        longlong2 *t2 = reinterpret_cast<longlong2 *>(s_tab);
        for (uint32_t d = threadIdx.x; d < nd; d += blockDim.x) {
            const longlong2 *src = reinterpret_cast<const longlong2 *>(gtab + (size_t)d * 64);
            const longlong2 a = src[0], b = src[1];
            int64_t z[4] = {a.x, a.y, b.x, b.y};
            int64_t y[4] = {z[1] - z[3], z[0] + z[2], z[1] + z[3], z[2] - z[0]};  // sqrt2 z
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const size_t at = ((size_t)d * 16 + (size_t)r * 2) * 2;
                t2[at] = make_longlong2(z[0], z[1]);
                t2[at + 1] = make_longlong2(z[2], z[3]);
                t2[at + 2] = make_longlong2(y[0], y[1]);
                t2[at + 3] = make_longlong2(y[2], y[3]);
                // times w: (c0, c1, c2, c3) -> (-c3, c0, c1, c2)
                const int64_t z3 = z[3], y3 = y[3];
                z[3] = z[2];
                z[2] = z[1];
                z[1] = z[0];
                z[0] = (int64_t)(0ull - (uint64_t)z3);
                y[3] = y[2];
                y[2] = y[1];
                y[1] = y[0];
                y[0] = (int64_t)(0ull - (uint64_t)y3);
            }
        }
        if (threadIdx.x < 4) s_tab[(size_t)H.zero_entry * 4 + threadIdx.x] = 0;
    }
    const uint32_t *words = reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(gtab) - H.table_byte_off);
    if (H.ntab_n) {
        uint32_t *d = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(s_tab) + H.ntab_lds);
        for (uint32_t i = threadIdx.x; i < H.ntab_n; i += blockDim.x) d[i] = words[H.off_ntab + i];
    }
    if (H.ztab_bits) {
        const uint32_t n = 4 * ztab_slots_for(inner_bits_for(H.W)) + (1u << inner_bits_for(H.W)) * H.W;
        uint32_t *d = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(s_tab) + H.ztab_lds);
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = words[H.off_ztab + i];
    }
    if (H.off_fmh) {
        // the form monomials' half tables (16-byte aligned at both ends)
        const uint32_t n4 = (16 + 2 * H.fmh_stride) / 4;
        uint4 *d = reinterpret_cast<uint4 *>(reinterpret_cast<char *>(s_tab) + H.fmh_lds);
        const uint4 *src = reinterpret_cast<const uint4 *>(words + H.off_fmh);
        for (uint32_t i = threadIdx.x; i < n4; i += blockDim.x) d[i] = src[i];
    }
    __syncthreads();
}

// Values that are the same in every lane of the wave, kept in scalar registers (the compiler
// cannot always prove it, for instance after a 64-bit division).
__device__ __forceinline__ uint32_t uniform32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    return ((uint64_t)uniform32((uint32_t)(x >> 32)) << 32) | uniform32((uint32_t)x);
}

// Work of one range of slices.  The unit is one block of the walks of a group of 64
// consecutive slices (one slice per lane; with fewer than KB walk bits a whole walk),
// and wave w of the nw waves that share the range takes a contiguous run of units, so the waves
// differ by at most one unit and every lane of a wave is at the same block.  Lanes whose slice
// is past the end of the range do nothing (or, in the compacting walk, walk without results).
// With class counters the runs are cut into chunks of at most chunk_units units, the same
// number of chunks in every wave of the workgroup, and the counters are flushed after each.
template <int W, bool MONO, int ACC, uint32_t SET>
__device__ __forceinline__ void run_range(const ImgHeader &H, const uint8_t *img, uint64_t s_first, uint64_t s_count,
                                          uint64_t wave, uint64_t n_waves, uint64_t chunk_units, int64_t *s_tab,
                                          unsigned long long *s_cnt, uint32_t *s_queue, i128 (&out)[4]) {
    CU32 *wd = const_words(img);
    const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
    Acc<ACC> acc;
    acc.clear();
    WaveQueue Q{s_queue + (threadIdx.x >> 6) * kQueueCap * kQueueWords<W>, 0u};
    const bool blocks = H.g >= (uint32_t)inner_bits_for(W);
    const bool compact = kCompact<W> && H.has_zero && blocks;
    const uint32_t lg_nb = blocks ? H.g - inner_bits_for(W) : 0u;  // units per slice group = 2^lg_nb
    const uint64_t n_units = ((s_count + 63) >> 6) << lg_nb;
    // teams of two waves sharing every unit, each evaluating half of a block's terms (header
    // flag term_split, used when the launch holds whole teams): twice the waves for small grids
    const uint32_t T = (H.term_split == 2 && blocks && !compact && (n_waves & 1) == 0) ? 2u : 1u;
    const uint32_t half = T == 2 ? (uint32_t)(wave & 1) + 1u : 0u;
    wave >>= T - 1u;  // T is 1 or 2: a shift, not a 64-bit division
    n_waves >>= T - 1u;
    // (32-bit division when the operands fit: the 64-bit one is a long instruction sequence)
    const bool narrow = (n_units >> 32) == 0 && (n_waves >> 32) == 0;
    const uint64_t q = uniform64(narrow ? (uint64_t)((uint32_t)n_units / (uint32_t)n_waves) : n_units / n_waves);
    const uint64_t r = uniform64(n_units - q * n_waves);
    const uint64_t u_begin = uniform64(wave * q + (wave < r ? wave : r));
    const uint64_t u_end = uniform64(u_begin + q + (wave < r ? 1 : 0));
    const uint64_t most = q + (r ? 1 : 0);  // largest run of any wave
    const uint64_t chunk = ACC == ACC_CLASS && chunk_units ? chunk_units : (most ? most : 1);
    const uint64_t n_chunks = chunk == most ? (most ? 1u : 0u) : uniform64((most + chunk - 1) / chunk);
    const uint32_t lane = threadIdx.x & 63u;
    for (uint64_t c = 0; c < n_chunks; ++c) {
        const uint64_t c0 = u_begin + c * chunk;
        const uint64_t c1 = c0 + chunk < u_end ? c0 + chunk : u_end;
        for (uint64_t u = c0; u < c1;) {
            const uint64_t group = uniform64(u >> lg_nb);
            const uint32_t b0 = uniform32((uint32_t)(u & ((1ull << lg_nb) - 1)));
            const uint64_t left = c1 - u;
            const uint32_t b1 =
                uniform32((uint64_t)(1u << lg_nb) - b0 < left ? (1u << lg_nb) : b0 + (uint32_t)left);
            const uint64_t s = (group << 6) + lane;
            const bool valid = s < s_count;
            if (compact)
                run_slice<W, MONO, ACC, SET, true>(H, wd, s_tab, s_cnt, s_first + (valid ? s : 0), valid, b0,
                                                   blocks ? b1 : 1u, &Q, acc);
            else if (valid)
                run_slice<W, MONO, ACC, SET, false>(H, wd, s_tab, s_cnt, s_first + s, true, b0,
                                                    blocks ? b1 : 1u, &Q, acc, half);
            u += b1 - b0;
        }
        if (ACC == ACC_CLASS && c + 1 < n_chunks) {
            if (compact && Q.n) queue_drain<W, ACC, SET>(H, wd, s_tab, s_cnt, Q, Q.n, acc);
            flush_counters<ACC>(H, gtab, s_cnt, out);
        }
    }
    if (compact && Q.n) queue_drain<W, ACC, SET>(H, wd, s_tab, s_cnt, Q, Q.n, acc);
    if (ACC == ACC_CLASS) flush_counters<ACC>(H, gtab, s_cnt, out);
    acc_to_i128<ACC>(acc, out);
}

template <int W, bool MONO, int ACC, uint32_t SET>
__global__ __launch_bounds__(kMaxThreads) void k_eval(ImgHeader H, const uint8_t *__restrict__ img,
                                                      uint64_t s_begin, uint64_t s_count, uint64_t chunk_units,
                                                      Partial *__restrict__ partials) {
    extern __shared__ int64_t s_dyn[];
    __shared__ uint4 s_queue[kCompact<W> ? kMaxThreads / 64 * kQueueCap * kQueueWords<W> / 4 : 1];
    const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
    prepare_lds<ACC>(H, gtab, s_dyn, reinterpret_cast<unsigned long long *>(s_dyn));
    i128 out[4] = {0, 0, 0, 0};
    // wave-uniform by construction; readfirstlane tells the compiler so
    const uint64_t wave = __builtin_amdgcn_readfirstlane((uint32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    run_range<W, MONO, ACC, SET>(H, img, s_begin, s_count, wave, n_waves, chunk_units, s_dyn,
                                 reinterpret_cast<unsigned long long *>(s_dyn), reinterpret_cast<uint32_t *>(s_queue),
                                 out);
    block_reduce_store(out, partials + blockIdx.x);
}

// One workgroup per work item (slices [s_begin, s_end) of one program): the hardware dispatcher
// balances the items, and the kernel keeps the live state of the single-program kernel (a
// persistent item loop would cost registers, and with them resident waves).
template <int W, bool MONO, int ACC, uint32_t SET>
__global__ __launch_bounds__(kMaxThreads) void k_eval_batch(const ImgHeader *__restrict__ hdrs,
                                                            const uint64_t *__restrict__ imgs,
                                                            const WorkItem *__restrict__ items, uint32_t n_items,
                                                            uint64_t chunk_units, Partial *__restrict__ partials) {
    extern __shared__ int64_t s_dyn[];
    __shared__ uint4 s_queue[kCompact<W> ? kMaxThreads / 64 * kQueueCap * kQueueWords<W> / 4 : 1];
    const uint32_t it = blockIdx.x;
    if (it >= n_items) return;
    const WorkItem wi = items[it];
    const uint32_t prog = __builtin_amdgcn_readfirstlane(wi.prog);
    const ImgHeader H = hdrs[prog];
    const uint8_t *img = reinterpret_cast<const uint8_t *>(imgs[prog]);
    const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
    prepare_lds<ACC>(H, gtab, s_dyn, reinterpret_cast<unsigned long long *>(s_dyn));
    i128 out[4] = {0, 0, 0, 0};
    run_range<W, MONO, ACC, SET>(H, img, wi.s_begin, wi.s_end - wi.s_begin,
                                 __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), blockDim.x >> 6, chunk_units,
                                 s_dyn, reinterpret_cast<unsigned long long *>(s_dyn),
                                 reinterpret_cast<uint32_t *>(s_queue), out);
    block_reduce_store(out, partials + wi.out_slot);
}

template <typename K>
hipError_t set_lds(K kern, size_t lds) {
    if (lds <= 48 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <int W, bool MONO, int ACC, uint32_t SET>
hipError_t launch_eval_t(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                         Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream,
                         hipEvent_t ev_start, hipEvent_t ev_stop) {
    const size_t lds = dyn_lds_bytes(H);
    auto kern = k_eval<W, MONO, ACC, SET>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    if (ev_start || ev_stop) {
        // timed by the dispatch itself: the events take the kernel's start and end
        hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, stream, ev_start, ev_stop, 0u, H,
                              reinterpret_cast<const uint8_t *>(dimg), s_begin, s_count,
                              chunk_units_for(H, threads), partials);
    } else {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, stream, H, reinterpret_cast<const uint8_t *>(dimg),
                           s_begin, s_count, chunk_units_for(H, threads), partials);
    }
    return hipGetLastError();
}

template <int W, bool MONO, int ACC, uint32_t SET>
hipError_t launch_batch_t(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                          const WorkItem *d_items, uint32_t n_items, Partial *partials, uint32_t threads,
                          uint32_t lds_bytes, hipStream_t stream) {
    auto kern = k_eval_batch<W, MONO, ACC, SET>;
    hipError_t e = set_lds(kern, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(threads), lds_bytes, stream, d_hdrs, d_imgs, d_items, n_items,
                       chunk_units_for(H0, threads), partials);
    return hipGetLastError();
}

}  // namespace

// variant selection within one width: slot set (int128 accumulation only with the full set;
// node slots in word 0 for widths 2 to 8), accumulation mode, monomials
#define DISPATCH_A(w, m, ACC_, MENU_, CALL)                                                  \
    do {                                                                                     \
        if ((ACC_) == ACC_I128) return CALL(w, m, ACC_I128, kSlotSetAll);                    \
        if ((ACC_) == ACC_I64) {                                                             \
            if ((MENU_) == 2) return CALL(w, m, ACC_I64, kSlotSetPhase);                     \
            if ((MENU_) == 3 && w <= 8) return CALL(w, m, ACC_I64, kSlotSetPhaseLow | kNTAB);\
            if (w > 1 && w < 16 && N0_) {                                                    \
                if ((MENU_) == 1) return CALL(w, m, ACC_I64, kSlotSetNodes | kNW0);          \
                return CALL(w, m, ACC_I64, kSlotSetAll | kNW0);                              \
            }                                                                                \
            if ((MENU_) == 1) return CALL(w, m, ACC_I64, kSlotSetNodes);                     \
            return CALL(w, m, ACC_I64, kSlotSetAll);                                         \
        }                                                                                    \
        if ((MENU_) == 2) return CALL(w, m, ACC_CLASS, kSlotSetPhase);                       \
        if ((MENU_) == 3 && w <= 8) return CALL(w, m, ACC_CLASS, kSlotSetPhaseLow | kNTAB);  \
        if (w > 1 && w < 16 && N0_) {                                                        \
            if ((MENU_) == 1) return CALL(w, m, ACC_CLASS, kSlotSetNodes | kNW0);            \
            return CALL(w, m, ACC_CLASS, kSlotSetAll | kNW0);                                \
        }                                                                                    \
        if ((MENU_) == 1) return CALL(w, m, ACC_CLASS, kSlotSetNodes);                       \
        return CALL(w, m, ACC_CLASS, kSlotSetAll);                                           \
    } while (0)


#define DISPATCH_WM(w, m, ACC_, MENU_, CALL)                                                 \
    do {                                                                                     \
        if ((ACC_) > 2 || (MENU_) > 3) return hipErrorInvalidValue;                          \
        if ((MENU_) == 3 && ((ACC_) == ACC_I128 || (w) > 8)) return hipErrorInvalidValue;    \
        constexpr uint32_t kNW0 = kSlotsNodeWord0;                                           \
        constexpr uint32_t kNTAB = kSlotsNodeTable;                                          \
        DISPATCH_A(w, m, ACC_, MENU_, CALL);                                                 \
    } while (0)

template <int W, bool MONO>
hipError_t launch_eval_wm(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                          Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream,
                          hipEvent_t ev_start, hipEvent_t ev_stop) {
#define CALL_EVAL(w, m, a, set) \
    launch_eval_t<w, m, a, set>(H, dimg, s_begin, s_count, partials, blocks, threads, stream, ev_start, ev_stop)
    const bool N0_ = H.node_word0 != 0;
    DISPATCH_WM(W, MONO, H.acc, H.slot_menu, CALL_EVAL);
#undef CALL_EVAL
}

template <int W, bool MONO, int ACC, uint32_t SET>
hipError_t occupancy_t(const ImgHeader &H, uint32_t threads, int *blocks_per_cu) {
    const size_t lds = dyn_lds_bytes(H);
    auto kern = k_eval<W, MONO, ACC, SET>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, kern, (int)threads, lds);
}

template <int W, bool MONO>
hipError_t occupancy_wm(const ImgHeader &H, uint32_t threads, int *blocks_per_cu) {
#define CALL_OCC(w, m, a, set) occupancy_t<w, m, a, set>(H, threads, blocks_per_cu)
    const bool N0_ = H.node_word0 != 0;
    DISPATCH_WM(W, MONO, H.acc, H.slot_menu, CALL_OCC);
#undef CALL_OCC
}

template <int W, bool MONO>
hipError_t launch_batch_wm(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                           const WorkItem *d_items, uint32_t n_items, Partial *partials, uint32_t threads,
                           uint32_t lds_bytes, hipStream_t stream) {
#define CALL_BATCH(w, m, a, set) \
    launch_batch_t<w, m, a, set>(H0, d_hdrs, d_imgs, d_items, n_items, partials, threads, lds_bytes, stream)
    const bool N0_ = H0.node_word0 != 0;
    DISPATCH_WM(W, MONO, H0.acc, H0.slot_menu, CALL_BATCH);
#undef CALL_BATCH
}

#define INSTANTIATE_EVAL_WM(w, m)                                                                     \
    template hipError_t occupancy_wm<w, m>(const ImgHeader &, uint32_t, int *);                       \
    template hipError_t launch_eval_wm<w, m>(const ImgHeader &, const void *, uint64_t, uint64_t,     \
                                             Partial *, uint32_t, uint32_t, hipStream_t, hipEvent_t,  \
                                             hipEvent_t);                                             \
    template hipError_t launch_batch_wm<w, m>(const ImgHeader &, const ImgHeader *, const uint64_t *, \
                                              const WorkItem *, uint32_t, Partial *, uint32_t, uint32_t, \
                                              hipStream_t);
