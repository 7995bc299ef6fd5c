// Exact comparison of real elements of Z[w] (host only), for the sampling decisions.
//
// A probability of the method is z * sqrt2^e with z real, i.e. z = a + b sqrt2 (coefficients
// (a, b, 0, -b) in the w-basis, since sqrt2 = w - w^3).  Deciding u < P(B || 0) / P(B) for a
// dyadic u = U / 2^53 is the sign of 2^53 P(B || 0) - U P(B): after bringing both terms to one
// power of sqrt2 (multiplying by sqrt2 maps a + b sqrt2 to 2b + a sqrt2) that is the sign of
// A + B sqrt2 for integers A, B, which is the sign of A when B = 0 or A, B agree, and
// otherwise the sign of A^2 - 2 B^2 taken with A's sign (sqrt2 is irrational, so that
// difference is never 0).  The integers outgrow 128 bits, hence the small big integer here.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "zw.h"

struct BigInt {
    bool neg = false;
    std::vector<uint32_t> m;  // magnitude, little-endian limbs, no leading zero limb

    bool zero() const { return m.empty(); }
    void trim() {
        while (!m.empty() && !m.back()) m.pop_back();
        if (m.empty()) neg = false;
    }
    static BigInt of(i128 v) {
        BigInt r;
        r.neg = v < 0;
        unsigned __int128 u = r.neg ? (unsigned __int128)0 - (unsigned __int128)v : (unsigned __int128)v;
        while (u) {
            r.m.push_back((uint32_t)u);
            u >>= 32;
        }
        return r;
    }
};

namespace zreal {

inline int cmp_mag(const BigInt &a, const BigInt &b) {
    if (a.m.size() != b.m.size()) return a.m.size() < b.m.size() ? -1 : 1;
    for (size_t i = a.m.size(); i-- > 0;)
        if (a.m[i] != b.m[i]) return a.m[i] < b.m[i] ? -1 : 1;
    return 0;
}

inline std::vector<uint32_t> add_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
    std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0);
    uint64_t carry = 0;
    for (size_t i = 0; i + 1 < r.size(); ++i) {
        uint64_t s = carry + (i < a.size() ? a[i] : 0) + (i < b.size() ? b[i] : 0);
        r[i] = (uint32_t)s;
        carry = s >> 32;
    }
    r.back() = (uint32_t)carry;
    return r;
}

// |a| - |b| for |a| >= |b|
inline std::vector<uint32_t> sub_mag(const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
    std::vector<uint32_t> r(a.size(), 0);
    int64_t borrow = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        int64_t d = (int64_t)a[i] - (i < b.size() ? b[i] : 0) - borrow;
        borrow = d < 0;
        r[i] = (uint32_t)(d + (borrow << 32));
    }
    return r;
}

inline BigInt add(const BigInt &a, const BigInt &b) {
    BigInt r;
    if (a.neg == b.neg) {
        r.m = add_mag(a.m, b.m);
        r.neg = a.neg;
    } else if (cmp_mag(a, b) >= 0) {
        r.m = sub_mag(a.m, b.m);
        r.neg = a.neg;
    } else {
        r.m = sub_mag(b.m, a.m);
        r.neg = b.neg;
    }
    r.trim();
    return r;
}

inline BigInt neg(BigInt a) {
    if (!a.zero()) a.neg = !a.neg;
    return a;
}

inline BigInt mul(const BigInt &a, const BigInt &b) {
    BigInt r;
    if (a.zero() || b.zero()) return r;
    r.m.assign(a.m.size() + b.m.size(), 0);
    for (size_t i = 0; i < a.m.size(); ++i) {
        uint64_t carry = 0;
        for (size_t j = 0; j < b.m.size(); ++j) {
            uint64_t t = (uint64_t)a.m[i] * b.m[j] + r.m[i + j] + carry;
            r.m[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        size_t k = i + b.m.size();
        while (carry) {
            uint64_t t = (uint64_t)r.m[k] + carry;
            r.m[k++] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    r.neg = a.neg != b.neg;
    r.trim();
    return r;
}

inline BigInt shl(const BigInt &a, unsigned bits) {
    BigInt r;
    if (a.zero()) return r;
    const unsigned limbs = bits / 32, sh = bits % 32;
    r.m.assign(a.m.size() + limbs + 1, 0);
    for (size_t i = 0; i < a.m.size(); ++i) {
        uint64_t v = (uint64_t)a.m[i] << sh;
        r.m[i + limbs] |= (uint32_t)v;
        r.m[i + limbs + 1] |= (uint32_t)(v >> 32);
    }
    r.neg = a.neg;
    r.trim();
    return r;
}

inline int sign(const BigInt &a) { return a.zero() ? 0 : (a.neg ? -1 : 1); }

// sign of A + B sqrt2
inline int sign_sqrt2(const BigInt &A, const BigInt &B) {
    const int sa = sign(A), sb = sign(B);
    if (!sb) return sa;
    if (!sa || sa == sb) return sb;
    const int d = cmp_mag(mul(A, A), shl(mul(B, B), 1));  // A^2 vs 2 B^2, never equal
    return d > 0 ? sa : sb;
}

// (a + b sqrt2) sqrt2^e
struct Real {
    BigInt a, b;
    int32_t e = 0;
};

// z must be real (c2 = 0, c3 = -c1); false otherwise
inline bool real_of(const Zw &z, int32_t e, Real *out) {
    if (z.c[2] != 0 || z.c[1] != -z.c[3]) return false;
    out->a = BigInt::of(z.c[0]);
    out->b = BigInt::of(z.c[1]);
    out->e = e;
    return true;
}

// the same number written with exponent E <= r.e
inline Real lower_to(const Real &r, int32_t E) {
    Real o;
    const unsigned d = (unsigned)(r.e - E);
    o.a = shl(r.a, d / 2);
    o.b = shl(r.b, d / 2);
    if (d & 1) {  // (a + b sqrt2) sqrt2 = 2b + a sqrt2
        BigInt t = shl(o.b, 1);
        o.b = o.a;
        o.a = t;
    }
    o.e = E;
    return o;
}

// sign of x * X - y * Y for non-negative 64-bit multipliers x, y
inline int sign_diff(uint64_t x, const Real &X, uint64_t y, const Real &Y) {
    const int32_t E = X.e < Y.e ? X.e : Y.e;
    const Real Xl = lower_to(X, E), Yl = lower_to(Y, E);
    const BigInt bx = BigInt::of((i128)x), by = BigInt::of((i128)y);
    const BigInt A = add(mul(bx, Xl.a), neg(mul(by, Yl.a)));
    const BigInt B = add(mul(bx, Xl.b), neg(mul(by, Yl.b)));
    return sign_sqrt2(A, B);
}

}  // namespace zreal
