// Device side of finishing an exact sum (shared by the finaliser kernels and the evaluation
// kernel's own finishing step): times the program's constant, the sqrt2 exponent, and the
// canonical form, written as a 72-byte result.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "zw.h"

__device__ __forceinline__ i128 fin_load_i128(const uint64_t *w) {
    return (i128)((unsigned __int128)w[0] | ((unsigned __int128)w[1] << 64));
}

// out = sum (raw), or 0 for a zero program, or c * sum * sqrt2^e in canonical form; an int128
// overflow while applying c sets RESULT_FLAG_OVERFLOW and writes zero
__device__ inline void finish_sum(const Zw &sum, const FinalArgs &A, DevResult *out) {
    uint32_t flags = 0;
    int32_t e = 0;
    Zw r = sum;
    if (A.raw) {
        flags |= RESULT_FLAG_RAW;
    } else if (A.zero) {
        r = zw_zero();
    } else {
        bool ok;
        if (A.unit) {
            // times w^u: u single negacyclic rotations, z w = (-c3, c0, c1, c2) (w^4 = -1), with
            // fixed indices only (no stack array)
            const i128 lo = (i128)((unsigned __int128)1 << 127);  // the one value without a negation
            ok = true;
            for (uint32_t t = 1; t < A.unit; ++t) {
                const i128 top = r.c[3];
                ok = ok && top != lo;
                r.c[3] = r.c[2];
                r.c[2] = r.c[1];
                r.c[1] = r.c[0];
                r.c[0] = -top;
            }
        } else {
            Zw c0;
            for (int k = 0; k < 4; ++k) c0.c[k] = fin_load_i128(A.c0 + 2 * k);
            ok = zw_mul_checked(c0, sum, &r);
        }
        if (!ok) {
            flags |= RESULT_FLAG_OVERFLOW;
            r = zw_zero();
        }
        e = A.e;
        zw_canonicalise(&r, &e);
    }
    for (int k = 0; k < 4; ++k) {
        out->w[2 * k] = (uint64_t)r.c[k];
        out->w[2 * k + 1] = (uint64_t)((unsigned __int128)r.c[k] >> 64);
    }
    out->e = e;
    out->flags = flags;
}
