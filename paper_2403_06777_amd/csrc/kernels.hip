// HIP kernels for gfx950: evaluate a packed term program over its assignments and sum the
// terms exactly.
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

#include <hip/hip_runtime.h>

#include "image.h"
#include "kernels.h"
#include "zw.h"

namespace {

constexpr int kMaxThreads = 256;
typedef const __attribute__((address_space(4))) uint32_t CU32;

__device__ __forceinline__ uint32_t popc(uint32_t x) { return (uint32_t)__builtin_popcount(x); }

__device__ __forceinline__ CU32 *const_words(const uint8_t *img) {
    return (CU32 *)(uintptr_t)img;
}

// the per-program statistic masks, read once and kept in scalar registers
template <int W>
struct Slots {
    uint32_t m[kSlots][W];
};

template <int W, uint32_t SET>
__device__ __forceinline__ void load_slots(const ImgHeader &H, CU32 *wd, Slots<W> &S) {
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
        if (!((SET >> i) & 1u)) continue;
        CU32 *e = wd + H.off_slots + i * (W + 1);
#pragma unroll
        for (int w = 0; w < W; ++w) S.m[i][w] = e[1 + w];
    }
}

struct TermClass {
    uint32_t cls;  // value class (d, r, e) or the zero entry
    int h;         // the term is 2^h times the class value
    bool zero;
};

template <int W, uint32_t SET>
__device__ __forceinline__ TermClass classify(const ImgHeader &H, const Slots<W> &S, CU32 *wd,
                                              const uint32_t (&L)[W], int phi) {
    int st[N_STATS];
#pragma unroll
    for (int s = 0; s < N_STATS; ++s) st[s] = H.stat_base[s];
#pragma unroll
    for (int i = 0; i < kSlots; ++i) {
        if ((SET >> i) & 1u) {  // compile-time: the slot belongs to this kernel's set
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) c += popc(L[w] & S.m[i][w]);
            const int wgt = slot_weight(i);
            if (wgt == 1) st[slot_stat(i)] += (int)c;
            else if (wgt == -1) st[slot_stat(i)] -= (int)c;
            else st[slot_stat(i)] += (int)c * wgt;
        }
    }
    TermClass t;
    t.zero = false;
    if (H.has_zero) {
        uint32_t z = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) z |= (~L[w] & wd[H.off_z0 + w]) | (L[w] & wd[H.off_z1 + w]);
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
    __device__ void clear() {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a64[k] = 0;
            a128[k] = 0;
        }
    }
};

template <int W, int ACC, uint32_t SET>
__device__ __forceinline__ void add_term(const ImgHeader &H, const Slots<W> &S, CU32 *wd, const int64_t *tab,
                                         unsigned long long *cnt, const uint32_t (&L)[W], int phi, Acc<ACC> &acc) {
    const TermClass t = classify<W, SET>(H, S, wd, L, phi);
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
        if (ACC == ACC_I64) {
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

// all 2^g assignments of slice s (high parameters = bits of s)
template <int W, bool MONO, int ACC, uint32_t SET>
__device__ __forceinline__ void run_slice(const ImgHeader &H, const Slots<W> &S, CU32 *wd, const int64_t *tab,
                                          unsigned long long *cnt, uint64_t s, Acc<ACC> &acc) {
    CU32 *col = wd + H.off_col;
    uint32_t L[W];
#pragma unroll
    for (int w = 0; w < W; ++w) L[w] = wd[H.off_cvec + w];
    for (uint32_t j = H.g; j < H.pe; ++j) {
        const uint32_t m = 0u - (uint32_t)((s >> (j - H.g)) & 1u);
#pragma unroll
        for (int w = 0; w < W; ++w) L[w] ^= col[j * W + w] & m;
    }
    int phi = 0;
    uint64_t dal = 0;  // 4-bit field i: always-firing slice-dependent change at a flip of i (mod 8)
    if (MONO) {
        CU32 *mh = wd + H.off_monohi;
        for (uint32_t e = 0; e < H.n_monohi; ++e, mh += 3) {
            const uint64_t hm = (uint64_t)mh[1] | ((uint64_t)mh[2] << 32);
            phi += ((s & hm) == hm) ? (int)mh[0] : 0;
        }
        CU32 *aidx = wd + H.off_aidx;
        for (uint32_t i = 0; i < H.g; ++i) {
            int f = 0;
            CU32 *ae = wd + H.off_al + 3 * aidx[i];
            for (uint32_t e = aidx[i]; e < aidx[i + 1]; ++e, ae += 3) {
                const uint64_t hm = (uint64_t)ae[1] | ((uint64_t)ae[2] << 32);
                f += ((s & hm) == hm) ? (int)ae[0] : 0;
            }
            dal |= (uint64_t)(f & 7) << (4 * i);
        }
    }
    add_term<W, ACC, SET>(H, S, wd, tab, cnt, L, phi, acc);
    const uint32_t n = 1u << H.g;
    uint32_t gray = 0;
    for (uint32_t t = 1; t < n; ++t) {
        const uint32_t i = (uint32_t)__builtin_ctz(t);
        gray ^= 1u << i;
#pragma unroll
        for (int w = 0; w < W; ++w) L[w] ^= col[i * W + w];
        if (MONO) {
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
            phi += ((gray >> i) & 1u) ? dd : -dd;
        }
        add_term<W, ACC, SET>(H, S, wd, tab, cnt, L, phi, acc);
    }
}

__device__ __forceinline__ i128 shfl_xor_i128(i128 v, int mask) {
    const unsigned __int128 u = (unsigned __int128)v;
    uint32_t p0 = (uint32_t)u, p1 = (uint32_t)(u >> 32), p2 = (uint32_t)(u >> 64), p3 = (uint32_t)(u >> 96);
    p0 = (uint32_t)__shfl_xor((int)p0, mask);
    p1 = (uint32_t)__shfl_xor((int)p1, mask);
    p2 = (uint32_t)__shfl_xor((int)p2, mask);
    p3 = (uint32_t)__shfl_xor((int)p3, mask);
    const unsigned __int128 r = (unsigned __int128)p0 | ((unsigned __int128)p1 << 32) |
                                ((unsigned __int128)p2 << 64) | ((unsigned __int128)p3 << 96);
    return (i128)r;
}

// sum of acc over the block (wave shuffles, then LDS in wave order), written by thread 0.
// Integer addition is associative, so the result does not depend on the order.
__device__ __forceinline__ void block_reduce_store(i128 (&acc)[4], Partial *out) {
    __shared__ i128 s_red[kMaxThreads / 64][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off > 0; off >>= 1) acc[k] += shfl_xor_i128(acc[k], off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
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
        if (ACC == ACC_I64) out[k] += (i128)acc.a64[k];
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
        for (uint32_t i = threadIdx.x; i < H.table_n * 4; i += blockDim.x) s_tab[i] = gtab[i];
    }
    __syncthreads();
}

// Rounds of blockDim slices are uniform across the block, so counters can be flushed
// between rounds (every flush_rounds rounds keeps each counter below 2^64).
template <int W, bool MONO, int ACC, uint32_t SET>
__device__ __forceinline__ void run_range(const ImgHeader &H, const uint8_t *img, uint64_t s_first, uint64_t s_count,
                                          uint64_t lane0, uint64_t stride, uint32_t flush_rounds, int64_t *s_tab,
                                          unsigned long long *s_cnt, i128 (&out)[4]) {
    CU32 *wd = const_words(img);
    const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
    Slots<W> S;
    load_slots<W, SET>(H, wd, S);
    Acc<ACC> acc;
    acc.clear();
    uint32_t rounds = 0;
    for (uint64_t base = lane0 - threadIdx.x; base < s_count; base += stride) {
        const uint64_t s = base + threadIdx.x;
        if (s < s_count) run_slice<W, MONO, ACC, SET>(H, S, wd, s_tab, s_cnt, s_first + s, acc);
        if (ACC == ACC_CLASS && ++rounds == flush_rounds) {
            flush_counters<ACC>(H, gtab, s_cnt, out);
            rounds = 0;
        }
    }
    if (ACC == ACC_CLASS) flush_counters<ACC>(H, gtab, s_cnt, out);
    acc_to_i128<ACC>(acc, out);
}

template <int W, bool MONO, int ACC, uint32_t SET>
__global__ __launch_bounds__(kMaxThreads) void k_eval(ImgHeader H, const uint8_t *__restrict__ img,
                                                      uint64_t s_begin, uint64_t s_count, uint32_t flush_rounds,
                                                      Partial *__restrict__ partials) {
    extern __shared__ int64_t s_dyn[];
    const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
    prepare_lds<ACC>(H, gtab, s_dyn, reinterpret_cast<unsigned long long *>(s_dyn));
    i128 out[4] = {0, 0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    run_range<W, MONO, ACC, SET>(H, img, s_begin, s_count, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride,
                            flush_rounds, s_dyn, reinterpret_cast<unsigned long long *>(s_dyn), out);
    block_reduce_store(out, partials + blockIdx.x);
}

template <int W, bool MONO, int ACC, uint32_t SET>
__global__ __launch_bounds__(kMaxThreads) void k_eval_batch(const ImgHeader *__restrict__ hdrs,
                                                            const uint64_t *__restrict__ imgs,
                                                            const WorkItem *__restrict__ items, uint32_t n_items,
                                                            uint32_t *__restrict__ queue, uint32_t flush_rounds,
                                                            Partial *__restrict__ partials) {
    extern __shared__ int64_t s_dyn[];
    __shared__ uint32_t s_item;
    uint32_t loaded = 0xffffffffu;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= n_items) break;
        const WorkItem wi = items[it];
        const uint32_t prog = __builtin_amdgcn_readfirstlane(wi.prog);
        const ImgHeader H = hdrs[prog];
        const uint8_t *img = reinterpret_cast<const uint8_t *>(imgs[prog]);
        const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
        if (prog != loaded || ACC == ACC_CLASS) {
            prepare_lds<ACC>(H, gtab, s_dyn, reinterpret_cast<unsigned long long *>(s_dyn));
            loaded = prog;
        }
        i128 out[4] = {0, 0, 0, 0};
        run_range<W, MONO, ACC, SET>(H, img, wi.s_begin, wi.s_end - wi.s_begin, threadIdx.x, blockDim.x, flush_rounds,
                                s_dyn, reinterpret_cast<unsigned long long *>(s_dyn), out);
        block_reduce_store(out, partials + wi.out_slot);
    }
}

__global__ void k_reset_queue(uint32_t *queue) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0u;
}

// sums partials [first, first + n), then applies the constant and canonicalises (thread 0)
__device__ void finalize_range(const Partial *partials, uint32_t first, uint32_t n, const FinalArgs &A,
                               DevResult *out) {
    __shared__ i128 s_sum[kMaxThreads][4];
    i128 acc[4] = {0, 0, 0, 0};
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x)
        for (int k = 0; k < 4; ++k) acc[k] += load_i128(partials[first + i].w + 2 * k);
    for (int k = 0; k < 4; ++k) s_sum[threadIdx.x][k] = acc[k];
    __syncthreads();
    if (threadIdx.x != 0) return;
    Zw sum = zw_zero();
    for (uint32_t t = 0; t < blockDim.x; ++t)
        for (int k = 0; k < 4; ++k) sum.c[k] += s_sum[t][k];
    uint32_t flags = 0;
    int32_t e = 0;
    Zw r = sum;
    if (A.raw) {
        flags |= RESULT_FLAG_RAW;
    } else if (A.zero) {
        r = zw_zero();
    } else {
        Zw c0;
        for (int k = 0; k < 4; ++k) c0.c[k] = load_i128(A.c0 + 2 * k);
        if (!zw_mul_checked(c0, sum, &r)) {
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

__global__ __launch_bounds__(kMaxThreads) void k_finalize(const Partial *__restrict__ partials, uint32_t n,
                                                          FinalArgs args, DevResult *__restrict__ out) {
    finalize_range(partials, 0, n, args, out);
}

__global__ __launch_bounds__(kMaxThreads) void k_finalize_batch(const Partial *__restrict__ partials,
                                                                const uint32_t *__restrict__ item_first,
                                                                const uint32_t *__restrict__ item_count,
                                                                const FinalArgs *__restrict__ args,
                                                                DevResult *__restrict__ out) {
    const uint32_t k = blockIdx.x;
    finalize_range(partials, item_first[k], item_count[k], args[k], out + k);
}

template <typename K>
hipError_t set_lds(K kern, size_t lds) {
    if (lds <= 48 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

template <int W, bool MONO, int ACC, uint32_t SET>
hipError_t launch_eval_t(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                         Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream) {
    const size_t lds = dyn_lds_bytes(H);
    auto kern = k_eval<W, MONO, ACC, SET>;
    hipError_t e = set_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, stream, H, reinterpret_cast<const uint8_t *>(dimg),
                       s_begin, s_count, flush_rounds_for(H, threads), partials);
    return hipGetLastError();
}

template <int W, bool MONO, int ACC, uint32_t SET>
hipError_t launch_batch_t(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                          const WorkItem *d_items, uint32_t n_items, uint32_t *d_queue, Partial *partials,
                          uint32_t blocks, uint32_t threads, uint32_t lds_bytes, hipStream_t stream) {
    auto kern = k_eval_batch<W, MONO, ACC, SET>;
    hipError_t e = set_lds(kern, lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds_bytes, stream, d_hdrs, d_imgs, d_items, n_items,
                       d_queue, flush_rounds_for(H0, threads), partials);
    return hipGetLastError();
}

}  // namespace

size_t dyn_lds_bytes(const ImgHeader &H) {
    if (H.acc == ACC_CLASS) return (size_t)H.zero_entry * H.q_limbs * 8;
    return (size_t)H.table_n * 32;
}

uint32_t flush_rounds_for(const ImgHeader &H, uint32_t threads) {
    // one round adds at most threads * 2^g terms of at most 2^31 each to a counter
    const uint64_t per_round = (uint64_t)threads << H.g;
    const uint64_t r = ((uint64_t)1 << 32) / (per_round ? per_round : 1);
    return (uint32_t)(r < 1 ? 1 : (r > 0xffffffffu ? 0xffffffffu : r));
}

// variant selection: slot set (int128 accumulation only with the full set), accumulation
// mode, monomials, form-vector width
#define DISPATCH(W_, MONO_, ACC_, MENU_, CALL)                                               \
    do {                                                                                     \
        if ((ACC_) > 2 || (MENU_) > 2) return hipErrorInvalidValue;                          \
        switch (W_) {                                                                        \
            case 1: DISPATCH_M(1, MONO_, ACC_, MENU_, CALL);                                 \
            case 2: DISPATCH_M(2, MONO_, ACC_, MENU_, CALL);                                 \
            case 4: DISPATCH_M(4, MONO_, ACC_, MENU_, CALL);                                 \
            case 8: DISPATCH_M(8, MONO_, ACC_, MENU_, CALL);                                 \
            case 16: DISPATCH_M(16, MONO_, ACC_, MENU_, CALL);                               \
            default: return hipErrorInvalidValue;                                            \
        }                                                                                    \
    } while (0)
#define DISPATCH_M(w, MONO_, ACC_, MENU_, CALL)                                              \
    if (MONO_) DISPATCH_A(w, true, ACC_, MENU_, CALL);                                       \
    else DISPATCH_A(w, false, ACC_, MENU_, CALL);
#define DISPATCH_A(w, m, ACC_, MENU_, CALL)                                                  \
    do {                                                                                     \
        if ((ACC_) == ACC_I128) return CALL(w, m, ACC_I128, kSlotSetAll);                    \
        if ((ACC_) == ACC_I64) {                                                             \
            if ((MENU_) == 1) return CALL(w, m, ACC_I64, kSlotSetNodes);                     \
            if ((MENU_) == 2) return CALL(w, m, ACC_I64, kSlotSetPhase);                     \
            return CALL(w, m, ACC_I64, kSlotSetAll);                                         \
        }                                                                                    \
        if ((MENU_) == 1) return CALL(w, m, ACC_CLASS, kSlotSetNodes);                       \
        if ((MENU_) == 2) return CALL(w, m, ACC_CLASS, kSlotSetPhase);                       \
        return CALL(w, m, ACC_CLASS, kSlotSetAll);                                           \
    } while (0)

hipError_t launch_eval(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                       Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream) {
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64 || blocks == 0)
        return hipErrorInvalidValue;
    if (dyn_lds_bytes(H) > MAX_TABLE_BYTES) return hipErrorInvalidValue;
#define CALL_EVAL(w, m, a, set) \
    launch_eval_t<w, m, a, set>(H, dimg, s_begin, s_count, partials, blocks, threads, stream)
    DISPATCH(H.W, H.has_mono != 0, H.acc, H.slot_menu, CALL_EVAL);
#undef CALL_EVAL
}

hipError_t launch_eval_batch(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                             const WorkItem *d_items, uint32_t n_items, uint32_t *d_queue,
                             Partial *partials, uint32_t blocks, uint32_t threads, uint32_t lds_bytes,
                             hipStream_t stream) {
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64 || blocks == 0)
        return hipErrorInvalidValue;
    if (lds_bytes > MAX_TABLE_BYTES) return hipErrorInvalidValue;
#define CALL_BATCH(w, m, a, set) \
    launch_batch_t<w, m, a, set>(H0, d_hdrs, d_imgs, d_items, n_items, d_queue, partials, blocks, threads, \
                                 lds_bytes, stream)
    DISPATCH(H0.W, H0.has_mono != 0, H0.acc, H0.slot_menu, CALL_BATCH);
#undef CALL_BATCH
}

hipError_t launch_reset_queue(uint32_t *d_queue, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, stream, d_queue);
    return hipGetLastError();
}

hipError_t launch_finalize(const Partial *partials, uint32_t n, const FinalArgs &args, DevResult *out,
                           hipStream_t stream) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kMaxThreads), 0, stream, partials, n, args, out);
    return hipGetLastError();
}

hipError_t launch_finalize_batch(const Partial *partials, const uint32_t *d_item_first,
                                 const uint32_t *d_item_count, const FinalArgs *d_args, uint32_t n_progs,
                                 DevResult *d_out, hipStream_t stream) {
    if (n_progs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_batch, dim3(n_progs), dim3(kMaxThreads), 0, stream, partials,
                       d_item_first, d_item_count, d_args, d_out);
    return hipGetLastError();
}
