// Launch wrappers of the HIP kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "image.h"

// arguments of the finaliser: constant c (four int128 as lo/hi pairs), exponent, mode
struct FinalArgs {
    uint64_t c0[8];
    int32_t e;
    uint32_t raw;   // 1: write the raw sum (no constant, no canonical form)
    uint32_t zero;  // 1: the program is identically zero
    uint32_t unit;  // r + 1 when the constant is exactly w^r (a rotation, no products); 0 otherwise
};

// device result, laid out exactly like sim_zomega
struct DevResult {
    uint64_t w[8];
    int32_t e;
    uint32_t flags;  // bit 0 raw, bit 1 int128 overflow while applying the constant
};

#define RESULT_FLAG_RAW 1u
#define RESULT_FLAG_OVERFLOW 2u

// largest dynamic LDS a value table may take
#define MAX_TABLE_BYTES kMaxDynLdsBytes

// largest block of the evaluation and finalise kernels
constexpr int kMaxThreads = 256;

// dynamic LDS of a program: value table (register modes) or class counters
size_t dyn_lds_bytes(const ImgHeader &H);
// work units per wave between flushes of the class counters (every workgroup adds fewer than
// 2^32 terms of at most 2^31 each to a counter between flushes)
uint64_t chunk_units_for(const ImgHeader &H, uint32_t threads);

// ev_start / ev_stop (optional, timing events): set by the kernel's own dispatch at its start and
// end (no separate event packets on the stream)
hipError_t launch_eval(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                       Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream,
                       hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

hipError_t launch_finalize(const Partial *partials, uint32_t n, const FinalArgs &args, DevResult *out,
                           hipStream_t stream);

// multi-program launch, one workgroup per work item; all programs share W, the monomial flag,
// the accumulation mode and the slot set of `H0`; lds_bytes is the largest dyn_lds_bytes of them
hipError_t launch_eval_batch(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                             const WorkItem *d_items, uint32_t n_items, Partial *partials, uint32_t threads,
                             uint32_t lds_bytes, hipStream_t stream);

// per-program finaliser: program k sums partials [item_first[k], item_first[k] + item_count[k])
// and, when d_carry is not null, d_carry[k] (a raw sum carried over from earlier launches)
hipError_t launch_finalize_batch(const Partial *partials, const uint32_t *d_item_first,
                                 const uint32_t *d_item_count, const FinalArgs *d_args, uint32_t n_progs,
                                 DevResult *d_out, hipStream_t stream, const Partial *d_carry = nullptr);

// bytes of the file-scope device array of the allocation-free entry point, and its address on
// the current device (called once per device with that device current)
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
hipError_t static_scratch_address(void **ptr);

// serving step finaliser: program k adds carry[slots[k]] (unless flags bit 0) to its partials and
// writes the raw sum back there, or (flags bit 1) finalises it into d_out[k]
hipError_t launch_serve_finalize(const Partial *partials, const uint32_t *d_item_first, const uint32_t *d_item_count,
                                 const FinalArgs *d_args, const uint32_t *d_slots, const uint32_t *d_flags,
                                 uint32_t n_progs, DevResult *d_carry, DevResult *d_out, hipStream_t stream);

// marginals by summing: d_acc (2 x 6 uint64: the 384-bit two's complement sums a, b) += the sum
// over the n results of |A|^2 = (a + b sqrt2) 2^e relative to 2^e_ref, through n_blocks partials
// (2 x 6 uint64 each) in d_part; *d_flags bit 0 is set if an exponent is below e_ref or too far
// above it (more than 120)
hipError_t launch_norm2_sum(const DevResult *d_res, uint32_t n, int32_t e_ref, uint64_t *d_part, uint32_t n_blocks,
                            uint64_t *d_acc, uint32_t *d_flags, hipStream_t stream);

// resident blocks per compute unit of the single-program evaluation kernel of H
hipError_t eval_occupancy(const ImgHeader &H, uint32_t threads, int *blocks_per_cu);

// evaluation launches per form-vector width W (1, 2, 4, 8, 16) and monomial flag, instantiated
// in eval_w<W>_m<0|1>.hip
template <int W, bool MONO>
hipError_t occupancy_wm(const ImgHeader &H, uint32_t threads, int *blocks_per_cu);
template <int W, bool MONO>
hipError_t launch_eval_wm(const ImgHeader &H, const void *dimg, uint64_t s_begin, uint64_t s_count,
                          Partial *partials, uint32_t blocks, uint32_t threads, hipStream_t stream,
                          hipEvent_t ev_start, hipEvent_t ev_stop);
template <int W, bool MONO>
hipError_t launch_batch_wm(const ImgHeader &H0, const ImgHeader *d_hdrs, const uint64_t *d_imgs,
                           const WorkItem *d_items, uint32_t n_items, Partial *partials, uint32_t threads,
                           uint32_t lds_bytes, hipStream_t stream);
