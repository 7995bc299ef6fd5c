// HIP kernels for gfx950 shared by every program: the finalisers that
// add per-block partial sums, apply the program's constant and reduce to canonical form; and
// the width dispatch of the evaluation launches (the evaluation kernels themselves are
// instantiated per form-vector width in eval_w*.hip).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "final.h"
#include "image.h"
#include "kernels.h"
#include "zw.h"

namespace {

__device__ __forceinline__ i128 load_i128(const uint64_t *w) {
    return (i128)((unsigned __int128)w[0] | ((unsigned __int128)w[1] << 64));
}

// sums partials [first, first + n) and *carry (if not null), then applies the constant and
// canonicalises (thread 0)
__device__ void finalize_range(const Partial *partials, uint32_t first, uint32_t n, const FinalArgs &A,
                               DevResult *out, const Partial *carry = nullptr) {
    __shared__ i128 s_sum[kMaxThreads][4];
    i128 acc[4] = {0, 0, 0, 0};
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        for (int k = 0; k < 4; ++k) acc[k] += load_i128(partials[first + i].w + 2 * k);
    if (carry && threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) acc[k] += load_i128(carry->w + 2 * k);
    for (int k = 0; k < 4; ++k) s_sum[threadIdx.x][k] = acc[k];
    __syncthreads();
    // tree reduction over the workgroup (blockDim.x is a power of two)
    for (uint32_t half = blockDim.x / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half)
            for (int k = 0; k < 4; ++k) s_sum[threadIdx.x][k] += s_sum[threadIdx.x + half][k];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    Zw sum = zw_zero();
    for (int k = 0; k < 4; ++k) sum.c[k] = s_sum[0][k];
    finish_sum(sum, A, out);
}

__global__ __launch_bounds__(kMaxThreads) void k_finalize(const Partial *__restrict__ partials, uint32_t n,
                                                          FinalArgs args, DevResult *__restrict__ out) {
    finalize_range(partials, 0, n, args, out);
}

__global__ __launch_bounds__(kMaxThreads) void k_finalize_batch(const Partial *__restrict__ partials,
                                                                const uint32_t *__restrict__ item_first,
                                                                const uint32_t *__restrict__ item_count,
                                                                const FinalArgs *__restrict__ args,
                                                                DevResult *__restrict__ out,
                                                                const Partial *__restrict__ carry) {
    const uint32_t k = blockIdx.x;
    finalize_range(partials, item_first[k], item_count[k], args[k], out + k, carry ? carry + k : nullptr);
}

// One serving step's finaliser: program k adds its partials to its carried raw sum (slot
// slots[k] of carry, read unless flags bit 0 says its first step) and writes the result back to
// that slot as a raw sum, or, when flags bit 1 says its last step, finalises it into out[k].
__global__ __launch_bounds__(kMaxThreads) void k_serve_finalize(const Partial *__restrict__ partials,
                                                                const uint32_t *__restrict__ item_first,
                                                                const uint32_t *__restrict__ item_count,
                                                                const FinalArgs *__restrict__ args,
                                                                const uint32_t *__restrict__ slots,
                                                                const uint32_t *__restrict__ flags,
                                                                DevResult *carry, DevResult *__restrict__ out) {
    const uint32_t k = blockIdx.x;
    const uint32_t f = flags[k];
    DevResult *slot = carry + slots[k];
    FinalArgs a = args[k];
    a.raw = (f & 2u) ? 0u : 1u;
    finalize_range(partials, item_first[k], item_count[k], a, (f & 2u) ? out + k : slot,
                   (f & 1u) ? nullptr : reinterpret_cast<const Partial *>(slot));
}

// ---- marginals by summing: sum of |A|^2 over a batch of amplitudes, exactly
//
// A = z sqrt2^e with z = c0 + c1 w + c2 w^2 + c3 w^3 (canonical results of the batch), and
// |A|^2 = (a + b sqrt2) 2^e with a = c0^2 + c1^2 + c2^2 + c3^2, b = c0 c1 + c1 c2 + c2 c3 - c3 c0
// (the products c_i c_j w^(i-j) pair up as w + w^-1 = sqrt2).  Relative to a reference e_ref <= e
// every square is an integer, shifted by e - e_ref; the sums are kept in 384-bit two's
// complement integers (WIDE limbs), exact and independent of the order of the additions.
constexpr int WIDE = 6;

__device__ __forceinline__ void wide_add(uint64_t (&acc)[WIDE], const uint64_t (&v)[WIDE]) {
    uint64_t carry = 0;
#pragma unroll
    for (int i = 0; i < WIDE; ++i) {
        const uint64_t s = acc[i] + v[i];
        const uint64_t c1 = s < acc[i] ? 1u : 0u;
        const uint64_t t = s + carry;
        const uint64_t c2 = t < s ? 1u : 0u;
        acc[i] = t;
        carry = c1 | c2;
    }
}

// v = sign * (mag << shift), mag a 256-bit magnitude, shift < 384 (bits past 384 are dropped:
// the caller's bound keeps them zero)
__device__ __forceinline__ void wide_of(const uint64_t (&mag)[4], bool neg, uint32_t shift, uint64_t (&v)[WIDE]) {
#pragma unroll
    for (int i = 0; i < WIDE; ++i) v[i] = 0;
    const uint32_t q = shift >> 6, r = shift & 63u;
    for (int i = 0; i < 4; ++i) {
        const uint32_t at = q + (uint32_t)i;
        if (at < (uint32_t)WIDE) v[at] |= mag[i] << r;
        if (r && at + 1 < (uint32_t)WIDE) v[at + 1] |= mag[i] >> (64 - r);
    }
    if (neg) {  // two's complement
        uint64_t carry = 1;
#pragma unroll
        for (int i = 0; i < WIDE; ++i) {
            const uint64_t t = ~v[i] + carry;
            carry = (carry && t == 0) ? 1u : 0u;
            v[i] = t;
        }
    }
}

// |x| * |y| for int128 x, y as a 256-bit magnitude
__device__ __forceinline__ void mul_mag(unsigned __int128 x, unsigned __int128 y, uint64_t (&m)[4]) {
    const uint64_t x0 = (uint64_t)x, x1 = (uint64_t)(x >> 64), y0 = (uint64_t)y, y1 = (uint64_t)(y >> 64);
    const unsigned __int128 p00 = (unsigned __int128)x0 * y0, p01 = (unsigned __int128)x0 * y1;
    const unsigned __int128 p10 = (unsigned __int128)x1 * y0, p11 = (unsigned __int128)x1 * y1;
    const unsigned __int128 mid = (p00 >> 64) + (uint64_t)p01 + (uint64_t)p10;
    m[0] = (uint64_t)p00;
    m[1] = (uint64_t)mid;
    const unsigned __int128 hi = (mid >> 64) + (p01 >> 64) + (p10 >> 64) + (uint64_t)p11;
    m[2] = (uint64_t)hi;
    m[3] = (uint64_t)(hi >> 64) + (uint64_t)(p11 >> 64);
}

__device__ __forceinline__ void add_product(uint64_t (&acc)[WIDE], i128 x, i128 y, bool negate, uint32_t shift) {
    const bool neg = ((x < 0) != (y < 0)) != negate;
    const unsigned __int128 ux = x < 0 ? (unsigned __int128)0 - (unsigned __int128)x : (unsigned __int128)x;
    const unsigned __int128 uy = y < 0 ? (unsigned __int128)0 - (unsigned __int128)y : (unsigned __int128)y;
    uint64_t m[4], v[WIDE];
    mul_mag(ux, uy, m);
    wide_of(m, neg, shift, v);
    wide_add(acc, v);
}

// per workgroup: the sums (a, b) of its share of the n results, as 2 x WIDE limbs; flags bit 0
// is set when a result's exponent is below e_ref or its shift leaves the 384 bits
__global__ __launch_bounds__(kMaxThreads) void k_norm2_partial(const DevResult *__restrict__ res, uint32_t n,
                                                               int32_t e_ref, uint64_t *__restrict__ part,
                                                               uint32_t *flags) {
    __shared__ uint64_t s_sum[kMaxThreads][2 * WIDE];
    uint64_t a[WIDE] = {0, 0, 0, 0, 0, 0}, b[WIDE] = {0, 0, 0, 0, 0, 0};
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const DevResult r = res[i];
        i128 c[4];
        bool zero = true;
        for (int k = 0; k < 4; ++k) {
            c[k] = load_i128(r.w + 2 * k);
            zero = zero && c[k] == 0;
        }
        if (zero) continue;
        // the squares (at most 2 maxbits + 2 bits) shifted by sh, summed over at most 2^32 results,
        // stay inside the 384 bits when 2 maxbits + sh <= 348
        uint32_t maxbits = 0;
        for (int k = 0; k < 4; ++k) {
            const unsigned __int128 u = c[k] < 0 ? (unsigned __int128)0 - (unsigned __int128)c[k] : (unsigned __int128)c[k];
            const uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
            const uint32_t bits = hi ? 128u - (uint32_t)__clzll(hi) : (lo ? 64u - (uint32_t)__clzll(lo) : 0u);
            maxbits = bits > maxbits ? bits : maxbits;
        }
        const int32_t sh = r.e - e_ref;
        if (sh < 0 || 2 * (int32_t)maxbits + sh > 348) {
            atomicOr(flags, 1u);
            continue;
        }
        for (int k = 0; k < 4; ++k) add_product(a, c[k], c[k], false, (uint32_t)sh);
        add_product(b, c[0], c[1], false, (uint32_t)sh);
        add_product(b, c[1], c[2], false, (uint32_t)sh);
        add_product(b, c[2], c[3], false, (uint32_t)sh);
        add_product(b, c[3], c[0], true, (uint32_t)sh);
    }
    for (int k = 0; k < WIDE; ++k) {
        s_sum[threadIdx.x][k] = a[k];
        s_sum[threadIdx.x][WIDE + k] = b[k];
    }
    __syncthreads();
    for (uint32_t half = blockDim.x / 2; half > 0; half >>= 1) {
        if (threadIdx.x < half) {
            uint64_t x[WIDE], y[WIDE], u[WIDE], v[WIDE];
            for (int k = 0; k < WIDE; ++k) {
                x[k] = s_sum[threadIdx.x][k];
                y[k] = s_sum[threadIdx.x][WIDE + k];
                u[k] = s_sum[threadIdx.x + half][k];
                v[k] = s_sum[threadIdx.x + half][WIDE + k];
            }
            wide_add(x, u);
            wide_add(y, v);
            for (int k = 0; k < WIDE; ++k) {
                s_sum[threadIdx.x][k] = x[k];
                s_sum[threadIdx.x][WIDE + k] = y[k];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 2 * WIDE) part[(size_t)blockIdx.x * 2 * WIDE + threadIdx.x] = s_sum[0][threadIdx.x];
}

// acc (2 x WIDE limbs, device) += the sum of the n_parts partials (one workgroup)
__global__ __launch_bounds__(kMaxThreads) void k_norm2_accumulate(const uint64_t *__restrict__ part, uint32_t n_parts,
                                                                  uint64_t *acc) {
    if (threadIdx.x != 0) return;
    uint64_t a[WIDE], b[WIDE];
    for (int k = 0; k < WIDE; ++k) {
        a[k] = acc[k];
        b[k] = acc[WIDE + k];
    }
    for (uint32_t i = 0; i < n_parts; ++i) {
        uint64_t u[WIDE], v[WIDE];
        for (int k = 0; k < WIDE; ++k) {
            u[k] = part[(size_t)i * 2 * WIDE + k];
            v[k] = part[(size_t)i * 2 * WIDE + WIDE + k];
        }
        wide_add(a, u);
        wide_add(b, v);
    }
    for (int k = 0; k < WIDE; ++k) {
        acc[k] = a[k];
        acc[WIDE + k] = b[k];
    }
}

}  // namespace

hipError_t launch_norm2_sum(const DevResult *d_res, uint32_t n, int32_t e_ref, uint64_t *d_part, uint32_t n_blocks,
                            uint64_t *d_acc, uint32_t *d_flags, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm2_partial, dim3(n_blocks), dim3(kMaxThreads), 0, stream, d_res, n, e_ref, d_part,
                       d_flags);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_norm2_accumulate, dim3(1), dim3(kMaxThreads), 0, stream, d_part, n_blocks, d_acc);
    return hipGetLastError();
}

hipError_t launch_serve_finalize(const Partial *partials, const uint32_t *d_item_first, const uint32_t *d_item_count,
                                 const FinalArgs *d_args, const uint32_t *d_slots, const uint32_t *d_flags,
                                 uint32_t n_progs, DevResult *d_carry, DevResult *d_out, hipStream_t stream) {
    if (n_progs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_serve_finalize, dim3(n_progs), dim3(kMaxThreads), 0, stream, partials, d_item_first,
                       d_item_count, d_args, d_slots, d_flags, d_carry, d_out);
    return hipGetLastError();
}

size_t dyn_lds_bytes(const ImgHeader &H) {
    const size_t base = H.acc == ACC_CLASS ? (size_t)H.zero_entry * H.q_limbs * 8 : (size_t)H.table_n * 32;
    size_t end = H.ntab_n ? (size_t)H.ntab_lds + (size_t)H.ntab_n * 4 : base;
    if (H.ztab_bits) {
        const int kb = inner_bits_for(H.W);
        const size_t zwords = 4 * (size_t)ztab_slots_for(kb) + ((size_t)1 << kb) * H.W;
        end = std::max(end, (size_t)H.ztab_lds + zwords * 4);
    }
    if (H.off_fmh) end = std::max(end, (size_t)H.fmh_lds + (16 + 2 * (size_t)H.fmh_stride) * 4);
    return end;
}

uint64_t chunk_units_for(const ImgHeader &H, uint32_t threads) {
    // a unit is one block (2^KB terms) of 64 lanes, or one whole walk of 2^g terms
    const uint32_t kb = (uint32_t)inner_bits_for(H.W);
    const uint32_t lg_terms = H.g >= kb ? kb : H.g;
    const uint64_t per_unit = (uint64_t)(threads ? threads : 64) << lg_terms;  // terms per unit in a workgroup
    const uint64_t c = ((uint64_t)1 << 32) / per_unit;
    return c ? c : 1;
}

// width and monomial flag of a program select the instantiation unit
#define SWITCH_WM(H_, CALL)                                   \
    do {                                                      \
        const bool m_ = (H_).has_mono != 0;                   \
        switch ((H_).W) {                                     \
            case 1: return m_ ? CALL(1, true) : CALL(1, false);   \
            case 2: return m_ ? CALL(2, true) : CALL(2, false);   \
            case 4: return m_ ? CALL(4, true) : CALL(4, false);   \
            case 8: return m_ ? CALL(8, true) : CALL(8, false);   \
            case 16: return m_ ? CALL(16, true) : CALL(16, false); \
            default: return hipErrorInvalidValue;             \
        }                                                     \
    } while (0)

hipError_t eval_occupancy(const ImgHeader &H, uint32_t threads, int *blocks_per_cu) {
#define CALL_OCC(w, m) occupancy_wm<w, m>(H, threads, blocks_per_cu)
    SWITCH_WM(H, CALL_OCC);
#undef CALL_OCC
}

hipError_t launch_eval(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                       Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream,
                       hipEvent_t ev_start, hipEvent_t ev_stop) {
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64 || blocks == 0)
        return hipErrorInvalidValue;
    if (dyn_lds_bytes(H) > MAX_TABLE_BYTES) return hipErrorInvalidValue;
#define CALL_EVAL(w, m) \
    launch_eval_wm<w, m>(H, dimg, s_begin, s_count, partials, blocks, threads, stream, ev_start, ev_stop)
    SWITCH_WM(H, CALL_EVAL);
#undef CALL_EVAL
}

hipError_t launch_eval_batch(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                             const WorkItem *d_items, uint32_t n_items, Partial *partials, uint32_t threads,
                             uint32_t lds_bytes, hipStream_t stream) {
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64 || n_items == 0)
        return hipErrorInvalidValue;
    if (lds_bytes > MAX_TABLE_BYTES) return hipErrorInvalidValue;
#define CALL_BATCH(w, m) \
    launch_batch_wm<w, m>(H0, d_hdrs, d_imgs, d_items, n_items, partials, threads, lds_bytes, stream)
    SWITCH_WM(H0, CALL_BATCH);
#undef CALL_BATCH
}

hipError_t launch_finalize(const Partial *partials, uint32_t n, const FinalArgs &args, DevResult *out,
                           hipStream_t stream) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kMaxThreads), 0, stream, partials, n, args, out);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const Partial *partials, const uint32_t *d_item_first,
                                 const uint32_t *d_item_count, const FinalArgs *d_args, uint32_t n_progs,
                                 DevResult *d_out, hipStream_t stream, const Partial *d_carry) {
    if (n_progs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_batch, dim3(n_progs), dim3(kMaxThreads), 0, stream, partials,
                       d_item_first, d_item_count, d_args, d_out, d_carry);
    return hipGetLastError();
}

// Fixed device scratch of the allocation-free entry point (sim_eval_ranges_static): one copy per
// device, held until the process ends.  Host code never passes this name to a kernel: it is a
// host-side stand-in; static_scratch_address gives each device's own address.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_address(void **ptr) {
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}
