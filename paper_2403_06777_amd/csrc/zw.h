// Exact arithmetic in Z[w], w = e^{i pi/4}, for the library (host and device).
//
// An element is c0 + c1 w + c2 w^2 + c3 w^3 with w^4 = -1.  The paper records subterm values
// as A + B sqrt2 + i (C + D sqrt2) (Section 3.3, step 5; Appendix E, Lemmas 6-7); the
// w-basis holds the same numbers with integer coordinates (A = c0, B = (c1 - c3)/2,
// C = c2, D = (c1 + c3)/2), and multiplying by w is a negacyclic rotation of the four
// coefficients, so a factor 1 + w^k needs no multiplication at all.
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#define ZW_HD __host__ __device__
#else
#define ZW_HD
#endif

typedef __int128 i128;

struct Zw {
    i128 c[4];
};

ZW_HD inline Zw zw_make(i128 a, i128 b, i128 c, i128 d) {
    Zw z;
    z.c[0] = a;
    z.c[1] = b;
    z.c[2] = c;
    z.c[3] = d;
    return z;
}

ZW_HD inline Zw zw_zero() { return zw_make(0, 0, 0, 0); }
ZW_HD inline Zw zw_one() { return zw_make(1, 0, 0, 0); }

ZW_HD inline bool zw_is_zero(const Zw &z) {
    return z.c[0] == 0 && z.c[1] == 0 && z.c[2] == 0 && z.c[3] == 0;
}

// z * w^k: each step maps (c0, c1, c2, c3) to (-c3, c0, c1, c2)
ZW_HD inline Zw zw_rot(Zw z, int k) {
    k &= 7;
    if (k & 4) {
        for (int i = 0; i < 4; ++i) z.c[i] = -z.c[i];
    }
    for (int s = 0; s < (k & 3); ++s) z = zw_make(-z.c[3], z.c[0], z.c[1], z.c[2]);
    return z;
}

// r + 1 when z = w^r exactly (one coefficient +-1, the others 0), else 0
ZW_HD inline uint32_t zw_unit_code(const Zw &z) {
    int nz = 0, at = 0;
    for (int k = 0; k < 4; ++k)
        if (z.c[k] != 0) ++nz, at = k;
    if (nz != 1 || (z.c[at] != 1 && z.c[at] != -1)) return 0;
    return (uint32_t)(at + (z.c[at] < 0 ? 4 : 0)) + 1u;
}

ZW_HD inline Zw zw_add(const Zw &a, const Zw &b) {
    return zw_make(a.c[0] + b.c[0], a.c[1] + b.c[1], a.c[2] + b.c[2], a.c[3] + b.c[3]);
}

// sqrt2 = w - w^3
ZW_HD inline Zw zw_times_sqrt2(const Zw &z) {
    return zw_make(z.c[1] - z.c[3], z.c[0] + z.c[2], z.c[1] + z.c[3], z.c[2] - z.c[0]);
}

ZW_HD inline bool zw_div_sqrt2_ok(const Zw &z) {
    return (((z.c[1] - z.c[3]) & 1) == 0) && (((z.c[0] + z.c[2]) & 1) == 0);
}

ZW_HD inline Zw zw_div_sqrt2(const Zw &z) {
    return zw_make((z.c[1] - z.c[3]) / 2, (z.c[0] + z.c[2]) / 2, (z.c[1] + z.c[3]) / 2,
                   (z.c[2] - z.c[0]) / 2);
}

// Full product with overflow detection (used only off the per-term path).
ZW_HD inline bool zw_mul_checked(const Zw &a, const Zw &b, Zw *out) {
    Zw r = zw_zero();
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) {
            i128 t;
            if (__builtin_mul_overflow(a.c[i], b.c[j], &t)) return false;
            int k = i + j;
            if (k >= 4) {
                k -= 4;
                if (__builtin_sub_overflow(r.c[k], t, &r.c[k])) return false;
            } else {
                if (__builtin_add_overflow(r.c[k], t, &r.c[k])) return false;
            }
        }
    }
    *out = r;
    return true;
}

ZW_HD inline bool zw_add_checked(const Zw &a, const Zw &b, Zw *out) {
    Zw r;
    for (int i = 0; i < 4; ++i)
        if (__builtin_add_overflow(a.c[i], b.c[i], &r.c[i])) return false;
    *out = r;
    return true;
}

// Canonical form of z * sqrt2^e: zero has e = 0; otherwise divide out sqrt2 while the
// quotient stays integral.
// Dividing by 2 = sqrt2^2 removes the common trailing zero bits of the four coefficients;
// after that at most one more sqrt2 divides z (two would mean z is even again).
ZW_HD inline int zw_ctz128(i128 v) {
    const uint64_t lo = (uint64_t)v, hi = (uint64_t)((unsigned __int128)v >> 64);
    if (lo) return __builtin_ctzll(lo);
    if (hi) return 64 + __builtin_ctzll(hi);
    return 128;
}

ZW_HD inline void zw_canonicalise(Zw *z, int32_t *e) {
    if (zw_is_zero(*z)) {
        *e = 0;
        return;
    }
    int k = 128;
    for (int i = 0; i < 4; ++i) {
        int t = zw_ctz128(z->c[i]);
        k = t < k ? t : k;
    }
    if (k) {
        for (int i = 0; i < 4; ++i) z->c[i] >>= k;
        *e += 2 * k;
    }
    if (zw_div_sqrt2_ok(*z)) {
        *z = zw_div_sqrt2(*z);
        *e += 1;
    }
}
