// HIP kernels for gfx950: evaluate a packed term program over its assignments and sum the
// terms exactly.
//
// Work decomposition.  The paper gives one GPU thread to each subterm row of one bitstring
// and multiplies/sums with repeated pairwise launches (Section 3.3, Appendix E).  Here a
// lane owns a whole slice of 2^g assignments instead: the high parameters are fixed by the
// slice index, the low g parameters are enumerated in Gray-code order so that one step
// flips one parameter, which XORs one wave-uniform column into the lane's form vector L.
// The product of all factors of a term is read off popcounts of L (value classes, see the
// packer) and one exact table entry w^r sqrt2^e Q(d) from LDS, shifted by sqrt2^(2h) = 2^h
// and added to four int128 accumulators.  Partial sums go wave -> block through shuffles and
// LDS, then a finaliser adds the per-block partials, applies the constant and reduces to
// canonical form.  No floating point is used anywhere.

#include <hip/hip_runtime.h>

#include "image.h"
#include "kernels.h"
#include "zw.h"

namespace {

constexpr int kMaxThreads = 256;

__device__ __forceinline__ uint32_t popc(uint32_t x) { return (uint32_t)__builtin_popcount(x); }

// one term: value classes -> table entry -> accumulate
template <int W>
__device__ __forceinline__ void eval_term(const ImgHeader &H, const uint32_t *__restrict__ wd,
                                          const int64_t *tab, const uint32_t (&L)[W], int phi,
                                          i128 (&acc)[4]) {
    int st[N_STATS];
#pragma unroll
    for (int s = 0; s < N_STATS; ++s) {
        int v = H.stat_base[s];
        const uint32_t *ent = wd + H.stat_off[s];
        const uint32_t n = H.stat_n[s];
        for (uint32_t e = 0; e < n; ++e, ent += W + 1) {
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) c += popc(L[w] & ent[1 + w]);
            v += (int)ent[0] * (int)c;
        }
        st[s] = v;
    }
    bool zero = false;
    if (H.has_zero) {
        uint32_t z = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) z |= (~L[w] & wd[H.off_z0 + w]) | (L[w] & wd[H.off_z1 + w]);
        zero = z != 0u;
    }
    const int A = st[STAT_A], B = st[STAT_B];
    const int m = A < B ? A : B;
    const int E = st[STAT_E] + m;
    const int R = st[STAT_R] + 2 * m + phi;
    uint32_t idx = ((uint32_t)(A - B + H.d_off) * 8u + (uint32_t)(R & 7)) * 2u + (uint32_t)(E & 1);
    idx = zero ? H.zero_entry : idx;
    const int h = E >> 1;
    const longlong2 *t = reinterpret_cast<const longlong2 *>(tab + (size_t)idx * 4);
    const longlong2 v01 = t[0];
    const longlong2 v23 = t[1];
    acc[0] += (i128)v01.x << h;
    acc[1] += (i128)v01.y << h;
    acc[2] += (i128)v23.x << h;
    acc[3] += (i128)v23.y << h;
}

// all 2^g assignments of slice s (high parameters = bits of s)
template <int W, bool MONO>
__device__ __forceinline__ void run_slice(const ImgHeader &H, const uint32_t *__restrict__ wd,
                                          const int64_t *tab, uint64_t s, i128 (&acc)[4]) {
    const uint32_t *col = wd + H.off_col;
    uint32_t L[W];
#pragma unroll
    for (int w = 0; w < W; ++w) L[w] = wd[H.off_cvec + w];
    for (uint32_t j = H.g; j < H.pe; ++j) {
        const uint32_t m = 0u - (uint32_t)((s >> (j - H.g)) & 1u);
#pragma unroll
        for (int w = 0; w < W; ++w) L[w] ^= col[j * W + w] & m;
    }
    int phi = 0;
    if (MONO) {
        const uint32_t *mh = wd + H.off_monohi;
        for (uint32_t e = 0; e < H.n_monohi; ++e, mh += 3) {
            const uint64_t hm = (uint64_t)mh[1] | ((uint64_t)mh[2] << 32);
            phi += ((s & hm) == hm) ? (int)mh[0] : 0;
        }
    }
    eval_term<W>(H, wd, tab, L, phi, acc);
    const uint32_t n = 1u << H.g;
    uint32_t gray = 0;
    for (uint32_t t = 1; t < n; ++t) {
        const uint32_t i = (uint32_t)__builtin_ctz(t);
        gray ^= 1u << i;
#pragma unroll
        for (int w = 0; w < W; ++w) L[w] ^= col[i * W + w];
        if (MONO) {
            const uint32_t *didx = wd + H.off_didx;
            const uint32_t e0 = didx[i], e1 = didx[i + 1];
            const uint32_t *de = wd + H.off_delta + 4 * e0;
            int du = 0, dv = 0;
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
        eval_term<W>(H, wd, tab, L, phi, acc);
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

template <int W, bool MONO>
__global__ __launch_bounds__(kMaxThreads) void k_eval(ImgHeader H, const uint8_t *__restrict__ img,
                                                      uint64_t s_begin, uint64_t s_count,
                                                      Partial *__restrict__ partials) {
    extern __shared__ int64_t s_tab[];
    const uint32_t *wd = reinterpret_cast<const uint32_t *>(img);
    const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
    for (uint32_t i = threadIdx.x; i < H.table_n * 4; i += blockDim.x) s_tab[i] = gtab[i];
    __syncthreads();
    i128 acc[4] = {0, 0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < s_count; s += stride)
        run_slice<W, MONO>(H, wd, s_tab, s_begin + s, acc);
    block_reduce_store(acc, partials + blockIdx.x);
}

template <int W, bool MONO>
__global__ __launch_bounds__(kMaxThreads) void k_eval_batch(const ImgHeader *__restrict__ hdrs,
                                                            const uint64_t *__restrict__ imgs,
                                                            const WorkItem *__restrict__ items,
                                                            uint32_t n_items, uint32_t *__restrict__ queue,
                                                            Partial *__restrict__ partials) {
    extern __shared__ int64_t s_tab[];
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
        const uint32_t *wd = reinterpret_cast<const uint32_t *>(img);
        if (prog != loaded) {
            const int64_t *gtab = reinterpret_cast<const int64_t *>(img + H.table_byte_off);
            for (uint32_t i = threadIdx.x; i < H.table_n * 4; i += blockDim.x) s_tab[i] = gtab[i];
            __syncthreads();
            loaded = prog;
        }
        i128 acc[4] = {0, 0, 0, 0};
        for (uint64_t s = wi.s_begin + threadIdx.x; s < wi.s_end; s += blockDim.x)
            run_slice<W, MONO>(H, wd, s_tab, s, acc);
        block_reduce_store(acc, partials + wi.out_slot);
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

template <int W, bool MONO>
hipError_t launch_eval_t(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                         Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream) {
    const size_t lds = (size_t)H.table_n * 32;
    auto kern = k_eval<W, MONO>;
    if (lds > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), lds, stream, H,
                       reinterpret_cast<const uint8_t *>(dimg), s_begin, s_count, partials);
    return hipGetLastError();
}

template <int W, bool MONO>
hipError_t launch_batch_t(const ImgHeader *d_hdrs, const uint64_t *d_imgs, const WorkItem *d_items,
                          uint32_t n_items, uint32_t *d_queue, Partial *partials, uint32_t blocks,
                          uint32_t threads, uint32_t table_bytes, hipStream_t stream) {
    auto kern = k_eval_batch<W, MONO>;
    if (table_bytes > 48 * 1024) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)table_bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(threads), table_bytes, stream, d_hdrs, d_imgs, d_items,
                       n_items, d_queue, partials);
    return hipGetLastError();
}

}  // namespace

#define DISPATCH_W(W_, MONO_, CALL)                                    \
    switch (W_) {                                                      \
        case 1: return MONO_ ? CALL(1, true) : CALL(1, false);        \
        case 2: return MONO_ ? CALL(2, true) : CALL(2, false);        \
        case 4: return MONO_ ? CALL(4, true) : CALL(4, false);        \
        case 8: return MONO_ ? CALL(8, true) : CALL(8, false);        \
        case 16: return MONO_ ? CALL(16, true) : CALL(16, false);     \
        default: return hipErrorInvalidValue;                          \
    }

hipError_t launch_eval(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                       Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream) {
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64 || blocks == 0)
        return hipErrorInvalidValue;
    if ((size_t)H.table_n * 32 > MAX_TABLE_BYTES) return hipErrorInvalidValue;
#define CALL_EVAL(w, m) launch_eval_t<w, m>(H, dimg, s_begin, s_count, partials, blocks, threads, stream)
    DISPATCH_W(H.W, H.has_mono != 0, CALL_EVAL)
#undef CALL_EVAL
}

hipError_t launch_eval_batch(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                             const WorkItem *d_items, uint32_t n_items, uint32_t *d_queue,
                             Partial *partials, uint32_t blocks, uint32_t threads, uint32_t table_bytes,
                             hipStream_t stream) {
    if (threads == 0 || threads > (uint32_t)kMaxThreads || threads % 64 || blocks == 0)
        return hipErrorInvalidValue;
    if (table_bytes > MAX_TABLE_BYTES) return hipErrorInvalidValue;
#define CALL_BATCH(w, m) \
    launch_batch_t<w, m>(d_hdrs, d_imgs, d_items, n_items, d_queue, partials, blocks, threads, table_bytes, stream)
    DISPATCH_W(H0.W, H0.has_mono != 0, CALL_BATCH)
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
