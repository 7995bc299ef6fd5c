// C-ABI of the library: programs, single-program evaluation, ranges, batches and plans.
//
// Device memory: a program's packed image is uploaded once at creation.  Per-block partial
// sums, batch work lists and result slots of one call are laid out in one region of device
// scratch memory: the library's own per-device buffer (grown on demand, kept until the process
// ends, guarded by a per-device lock), or memory the caller owns and passes in (the *_ws entry
// points, sim_batch_prepare / sim_enqueue_batch), which the library never grows or frees.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zxpar.h"
#include "compiler.h"
#include "kernels.h"
#include "program.h"
#include "zreal.h"

struct sim_program {
    int device = 0;
    IrProgram ir;
    PackedProgram pk;
    void *dimg = nullptr;
    // the image goes up asynchronously (the device's upload stream); launches wait for this
    // event once, the first time the program is used
    hipEvent_t up_ev = nullptr;
    mutable std::atomic<bool> uploaded{false};
    double compile_seconds = 0.0;
    uint32_t t_count = 0;
    uint32_t n_constraints = 0;
    // resident blocks per compute unit of its evaluation kernel, for occ_threads threads
    // (queried once; evaluations hold the device lock)
    uint32_t occ_threads = 0;
    int occ_blocks = 0;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(call)                                                                       \
    do {                                                                                    \
        hipError_t _e = (call);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(SIM_EDEVICE, std::string(#call) + " failed: " + hipGetErrorString(_e)); \
    } while (0)

struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
};

struct DeviceState {
    bool ready = false;
    int cus = 0;
    std::mutex mu;
    DevBuf ws;                    // the library's scratch region
    std::vector<void *> ws_old;   // scratch buffers it outgrew: kept until the process ends
    DevBuf msum;                  // sim_marginal_sum: its 384-bit sums and their partials
    void *static_scratch = nullptr;  // this device's address of the fixed array (kStaticScratchBytes)
    // program images are copied on a stream of their own (non-blocking, default priority), so
    // creating a program never waits behind evaluations already enqueued on other streams
    hipStream_t upload = nullptr;
    // pipelined serving steps (sim_serve_enqueue): a ring of device regions and pinned staging
    // buffers, each reused only after the event of its previous step has completed
    static constexpr int kRing = 4;
    DevBuf ring_dev[kRing];
    void *ring_host[kRing] = {nullptr, nullptr, nullptr, nullptr};
    size_t ring_host_cap[kRing] = {0, 0, 0, 0};
    hipEvent_t ring_ev[kRing] = {nullptr, nullptr, nullptr, nullptr};
    bool ring_used[kRing] = {false, false, false, false};
    unsigned ring_next = 0;
    void *host_result = nullptr;  // pinned
    size_t host_cap = 0;
    void *host_stage = nullptr;   // pinned staging of batch layouts
    size_t host_stage_cap = 0;
    bool aux_ready = false;       // auxiliary streams (default priority) for concurrent batch groups
    hipStream_t aux[4];
    hipEvent_t ev_fork, ev_join[4];
    // evaluations enqueued without waiting (sim_enqueue_amplitude) may still use the scratch
    // above; the last of them went to pending_stream.  No event marks them: a recorded event
    // costs the GPU about as much as a tenth of a small evaluation, and a stream handle kept
    // for a later record could have been destroyed by then.
    hipStream_t pending_stream = nullptr;
    bool pending = false;
};

constexpr int kAux = 4;
// free outcomes a marginal by summing may have (2^m amplitudes, in chunks of 2^16)
constexpr size_t kMaxMarginalFree = 32;

constexpr int kMaxDevices = 64;
DeviceState g_dev[kMaxDevices];
std::mutex g_init_mu;

// waits on the host for enqueued work that may still use the device's scratch (caller holds
// D.mu): the whole device, since the stream it went to need not exist any more
int settle(DeviceState &D) {
    if (!D.pending) return SIM_OK;
    D.pending = false;
    HIP_TRY(hipSetDevice((int)(&D - g_dev)));
    HIP_TRY(hipDeviceSynchronize());
    return SIM_OK;
}

int ensure(DevBuf &b, size_t need) {
    if (b.cap >= need) return SIM_OK;
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.cap = 0;
    size_t cap = std::max<size_t>(need, 4096);
    hipError_t e = hipMalloc(&b.ptr, cap);
    if (e != hipSuccess) return fail(SIM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    b.cap = cap;
    return SIM_OK;
}

int ensure_host(DeviceState &D, size_t need) {
    if (D.host_cap >= need) return SIM_OK;
    if (D.host_result) (void)hipHostFree(D.host_result);
    D.host_result = nullptr;
    D.host_cap = 0;
    size_t cap = std::max<size_t>(need, 4096);
    hipError_t e = hipHostMalloc(&D.host_result, cap, hipHostMallocDefault);
    if (e != hipSuccess) return fail(SIM_ENOMEM, std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
    D.host_cap = cap;
    return SIM_OK;
}

int ensure_aux(DeviceState &D) {
    if (D.aux_ready) return SIM_OK;
    for (int a = 0; a < kAux; ++a) {
        HIP_TRY(hipStreamCreateWithFlags(&D.aux[a], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&D.ev_join[a], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&D.ev_fork, hipEventDisableTiming));
    D.aux_ready = true;
    return SIM_OK;
}

int init_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(SIM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_init_mu);
    DeviceState &D = g_dev[dev];
    if (D.ready) return SIM_OK;
    HIP_TRY(hipSetDevice(dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    D.cus = prop.multiProcessorCount;
    // this device's copy of the allocation-free entry point's array
    void *sp = nullptr;
    HIP_TRY(static_scratch_address(&sp));
    D.static_scratch = sp;
    HIP_TRY(hipStreamCreateWithFlags(&D.upload, hipStreamNonBlocking));
    D.ready = true;
    return SIM_OK;
}

int current_device(int *dev) {
    HIP_TRY(hipGetDevice(dev));
    return init_device(*dev);
}

FinalArgs final_args(const PackedProgram &pk, bool raw) {
    FinalArgs a;
    memset(&a, 0, sizeof a);
    for (int k = 0; k < 4; ++k) {
        a.c0[2 * k] = (uint64_t)pk.c0.c[k];
        a.c0[2 * k + 1] = (uint64_t)((unsigned __int128)pk.c0.c[k] >> 64);
    }
    a.e = pk.e;
    a.raw = raw ? 1u : 0u;
    a.zero = pk.zero ? 1u : 0u;
    a.unit = zw_unit_code(pk.c0);
    return a;
}

int to_zomega(const DevResult &r, sim_zomega *out) {
    if (r.flags & RESULT_FLAG_OVERFLOW)
        return fail(SIM_ERANGE, "int128 overflow while applying the program constant");
    for (int k = 0; k < 4; ++k) {
        out->c[k].lo = r.w[2 * k];
        out->c[k].hi = (int64_t)r.w[2 * k + 1];
    }
    out->sqrt2_exp = r.e;
    out->flags = r.flags & RESULT_FLAG_RAW ? SIM_ZOMEGA_RAW : 0u;
    return SIM_OK;
}

void zero_result(sim_zomega *out, bool raw) {
    memset(out, 0, sizeof *out);
    if (raw) out->flags = SIM_ZOMEGA_RAW;
}

uint32_t pick_threads(const sim_tuning *t) {
    uint32_t th = t && t->block_threads ? t->block_threads : 256u;
    th = std::min<uint32_t>(256u, std::max<uint32_t>(64u, th / 64 * 64));
    return th;
}

// Grid of the single-program kernel over `count` slices: by default what the chip holds at
// once (every block resident), so that the kernel's own split of the work into per-wave runs of
// blocks, not a second wave of workgroups, balances it; never more waves than work units (one
// 2^KB-term block of 64 slices, or one whole short walk of 64 slices).
int eval_grid(DeviceState &D, const sim_program *P, uint64_t count, uint32_t threads, const sim_tuning *t,
              uint32_t *blocks) {
    const ImgHeader &H = P->pk.hdr;
    uint32_t bpc = t && t->blocks_per_cu ? t->blocks_per_cu : 0u;
    if (!bpc) {
        sim_program *Pm = const_cast<sim_program *>(P);
        if (Pm->occ_threads != threads) {
            int occ = 0;
            HIP_TRY(eval_occupancy(H, threads, &occ));
            Pm->occ_blocks = std::max(1, occ);
            Pm->occ_threads = threads;
        }
        bpc = (uint32_t)Pm->occ_blocks;
    }
    const uint32_t kb = (uint32_t)inner_bits_for(H.W);
    const uint32_t lg_units = H.g >= kb ? H.g - kb : 0u;
    // a unit is taken by a team of term_split waves
    const uint64_t units = (((count + 63) / 64) << std::min<uint32_t>(lg_units, 40)) * std::max<uint32_t>(1, H.term_split);
    const uint64_t waves_per_block = threads / 64;
    const uint64_t want = (units + waves_per_block - 1) / waves_per_block;
    const uint64_t cap = (uint64_t)std::max(1, D.cus) * bpc;
    *blocks = (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
    return SIM_OK;
}

// ---- scratch regions

constexpr size_t kAlign = 256;
size_t up256(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// device memory one call lays its buffers out in
struct Region {
    char *base = nullptr;
    size_t cap = 0;
};

// The library's scratch for work on stream st, at least `need` bytes (device lock held).
// Enqueued work on another stream that may still use it is waited for on the host; on the same
// stream, stream order suffices.  A scratch that is too small is replaced by one at least
// twice its size, and the old buffer is kept, never freed: enqueued work and captured graphs
// that hold its address stay valid, and growing needs no wait.
int lib_region(DeviceState &D, size_t need, Region *R, hipStream_t st) {
    if (D.pending && D.pending_stream != st) {
        int rc = settle(D);
        if (rc) return rc;
    }
    if (D.ws.cap < need) {
        void *p = nullptr;
        const size_t cap = std::max<size_t>({need, 2 * D.ws.cap, 4096});
        hipError_t e = hipMalloc(&p, cap);
        if (e != hipSuccess) return fail(SIM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        if (D.ws.ptr) D.ws_old.push_back(D.ws.ptr);
        D.ws.ptr = p;
        D.ws.cap = cap;
    }
    R->base = (char *)D.ws.ptr;
    R->cap = D.ws.cap;
    return SIM_OK;
}

// memory the caller passed in: never grown; too small is an error
int caller_region(void *dev_scratch, size_t bytes, size_t need, Region *R) {
    if (!dev_scratch) return fail(SIM_EINVAL, "null dev_scratch");
    if (reinterpret_cast<uintptr_t>(dev_scratch) % kAlign) return fail(SIM_EINVAL, "dev_scratch must be 256-byte aligned");
    if (bytes < need)
        return fail(SIM_ERANGE, "dev_scratch holds " + std::to_string(bytes) + " bytes; the call needs " +
                                    std::to_string(need) + " (see sim_scratch_bytes)");
    R->base = (char *)dev_scratch;
    R->cap = bytes;
    return SIM_OK;
}

// a single-program evaluation: per-workgroup partials at offset 0, its result at o_res
struct SinglePlan {
    uint32_t blocks = 1, threads = 256;
    size_t o_res = 0, total = 0;
};

int plan_single(DeviceState &D, const sim_program *P, uint64_t count, const sim_tuning *t, SinglePlan *S) {
    S->threads = pick_threads(t);
    if (!(t && t->block_threads)) {
        // fewer work units (waves) than four per compute unit: one-wave workgroups, so that the
        // waves spread over every compute unit instead of filling half of them
        const ImgHeader &H = P->pk.hdr;
        const uint32_t kb = (uint32_t)inner_bits_for(H.W);
        const uint32_t lg_units = H.g >= kb ? H.g - kb : 0u;
        const uint64_t units = (((count + 63) / 64) << std::min<uint32_t>(lg_units, 40)) * std::max<uint32_t>(1, H.term_split);
        if (units < 4 * (uint64_t)std::max(1, D.cus)) S->threads = 64;
    }
    int rc = eval_grid(D, P, count, S->threads, t, &S->blocks);
    if (rc) return rc;
    S->o_res = up256((size_t)S->blocks * sizeof(Partial));
    S->total = S->o_res + up256(sizeof(DevResult));
    return SIM_OK;
}

// events created for one call and destroyed on every return path
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

int await_upload(const sim_program *P);

// Blocking evaluation of one slice range in region R (laid out by S): kernel, finaliser, copy of
// the 72-byte result to host memory (`pinned` staging of the library, or a pageable copy) and a
// wait on the stream.  Device lock held.
int eval_single(const sim_program *P, uint64_t first, uint64_t count, bool raw, const SinglePlan &S, const Region &R,
                void *pinned, hipStream_t stream, sim_zomega *out, float *kernel_ms = nullptr) {
    Partial *parts = (Partial *)R.base;
    DevResult *dres = (DevResult *)(R.base + S.o_res);
    int rc = await_upload(P);
    if (rc) return rc;
    EventPair ev;
    if (kernel_ms) {
        HIP_TRY(hipEventCreate(&ev.a));
        HIP_TRY(hipEventCreate(&ev.b));
    }
    HIP_TRY(launch_eval(P->pk.hdr, P->dimg, first, count, parts, S.blocks, S.threads, stream, ev.a, ev.b));
    HIP_TRY(launch_finalize(parts, S.blocks, final_args(P->pk, raw), dres, stream));
    DevResult r;
    HIP_TRY(hipMemcpyAsync(pinned ? pinned : (void *)&r, dres, sizeof(DevResult), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (kernel_ms) HIP_TRY(hipEventElapsedTime(kernel_ms, ev.a, ev.b));
    if (pinned) memcpy(&r, pinned, sizeof r);
    return to_zomega(r, out);
}

// one evaluation of a slice range in the library's scratch (device lock held)
int eval_range_locked(DeviceState &D, const sim_program *P, uint64_t first, uint64_t count, bool raw,
                      hipStream_t stream, const sim_tuning *t, sim_zomega *out, float *kernel_ms = nullptr) {
    SinglePlan S;
    Region R;
    int rc;
    if ((rc = plan_single(D, P, count, t, &S))) return rc;
    if ((rc = lib_region(D, S.total, &R, stream))) return rc;
    if ((rc = ensure_host(D, sizeof(DevResult)))) return rc;
    return eval_single(P, first, count, raw, S, R, D.host_result, stream, out, kernel_ms);
}

int finish_program(std::unique_ptr<sim_program> &P, sim_program **out, bool eliminate = true) {
    std::string err;
    int rc = pack_program(P->ir, 12, &P->pk, &err, eliminate);
    if (rc) return fail(rc, err);
    int dev;
    if ((rc = current_device(&dev))) return rc;
    P->device = dev;
    hipError_t e = hipMalloc(&P->dimg, P->pk.blob.size());
    if (e != hipSuccess) return fail(SIM_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    // the host blob stays alive with the program, so the copy may still be in flight on return
    const hipStream_t up = g_dev[dev].upload;
    e = hipEventCreateWithFlags(&P->up_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMemcpyAsync(P->dimg, P->pk.blob.data(), P->pk.blob.size(), hipMemcpyHostToDevice, up);
    if (e == hipSuccess) e = hipEventRecord(P->up_ev, up);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(up);
        if (P->up_ev) (void)hipEventDestroy(P->up_ev);
        (void)hipFree(P->dimg);
        P->dimg = nullptr;
        return fail(SIM_EDEVICE, std::string("program upload failed: ") + hipGetErrorString(e));
    }
    *out = P.release();
    return SIM_OK;
}

// the program's image is on the device: waits (host) for its upload the first time only.  A
// host wait rather than a stream wait keeps every launch path capturable.
int await_upload(const sim_program *P) {
    if (P->uploaded.load(std::memory_order_acquire)) return SIM_OK;
    HIP_TRY(hipEventSynchronize(P->up_ev));
    P->uploaded.store(true, std::memory_order_release);
    return SIM_OK;
}

int enter_device(const sim_program *P, DeviceState **D) {
    int rc = init_device(P->device);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(P->device));
    *D = &g_dev[P->device];
    return SIM_OK;
}

}  // namespace

extern "C" {

const char *sim_last_error(void) { return g_err.c_str(); }

int sim_init(int device) {
    int rc = init_device(device);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(device));
    return SIM_OK;
}

int sim_device_cus(void) {
    int dev;
    if (current_device(&dev)) return 0;
    return g_dev[dev].cus;
}

int sim_program_from_ir_flags(const char *ir_text, size_t len, uint32_t flags, sim_program **out) {
    if (!ir_text || !out) return fail(SIM_EINVAL, "null argument");
    if (flags & ~SIM_IR_KEEP_VANISHING) return fail(SIM_EINVAL, "unknown flags");
    std::unique_ptr<sim_program> P(new (std::nothrow) sim_program());
    if (!P) return fail(SIM_ENOMEM, "out of host memory");
    std::string err;
    if (!ir_parse(ir_text, len, &P->ir, &err)) return fail(SIM_EINVAL, err);
    return finish_program(P, out, !(flags & SIM_IR_KEEP_VANISHING));
}

int sim_program_from_ir(const char *ir_text, size_t len, sim_program **out) {
    return sim_program_from_ir_flags(ir_text, len, 0u, out);
}

int sim_compile(const char *circuit_text, size_t len, const sim_query *q, const sim_compile_opts *opts,
                sim_program **out) {
    if (!circuit_text || !q || !out) return fail(SIM_EINVAL, "null argument");
    std::unique_ptr<sim_program> P(new (std::nothrow) sim_program());
    if (!P) return fail(SIM_ENOMEM, "out of host memory");
    CompileOptions co;
    if (opts) {
        if (opts->p_cap) co.p_cap = (int)opts->p_cap;
        co.eliminate_constraints = opts->eliminate_constraints != 0;
        co.hub_params = opts->t_spiders_only == 0;
    }
    CompileStats cs;
    std::string err;
    auto t0 = std::chrono::steady_clock::now();
    int rc = compile_circuit(circuit_text, len, *q, co, &P->ir, &cs, &err);
    auto t1 = std::chrono::steady_clock::now();
    if (rc) return fail(rc, err);
    P->compile_seconds = std::chrono::duration<double>(t1 - t0).count();
    P->t_count = (uint32_t)cs.t_count;
    P->n_constraints = (uint32_t)cs.n_constraints;
    return finish_program(P, out);
}


}  // extern "C"

namespace {
void fill_info(const PackedProgram &pk, double compile_seconds, uint32_t t_count, uint32_t n_constraints,
               sim_info *out) {
    memset(out, 0, sizeof *out);
    out->n_params = (uint32_t)pk.p;
    out->n_forms = (uint32_t)pk.n_forms;
    out->n_factors = (uint32_t)pk.n_factors;
    out->n_monomials = (uint32_t)pk.n_mono;
    out->sqrt2_exp = pk.e;
    out->walk_bits = (uint32_t)pk.walk_bits;
    out->n_slices = pk.n_slices;
    out->image_bytes = pk.blob.size();
    out->log2_terms = (double)pk.p;
    out->n_eval_params = pk.hdr.pe;
    out->is_zero = pk.zero ? 1u : 0u;
    out->compile_seconds = compile_seconds;
    out->t_count = t_count;
    out->n_constraints = n_constraints;
    out->ops_per_term = pk.ops_per_term;
    out->nonzero_fraction = pk.nonzero_fraction;
    out->n_outer = (uint32_t)pk.outer;
    out->vanish_table_bits = pk.hdr.ztab_bits;
    out->n_params_given = (uint32_t)pk.p_given;
    out->n_eliminated = (uint32_t)pk.eliminated;
    out->n_form_monomials = (uint32_t)pk.n_fmono;
    out->n_mono_forms = (uint32_t)pk.n_mforms;
    out->block_sum32 = pk.hdr.block_sum32;
    out->team_waves = std::max<uint32_t>(1, pk.hdr.term_split);
}
}  // namespace

extern "C" int sim_ir_info_flags(const char *ir_text, size_t len, uint32_t flags, sim_info *out) {
    if (!ir_text || !out) return fail(SIM_EINVAL, "null argument");
    if (flags & ~SIM_IR_KEEP_VANISHING) return fail(SIM_EINVAL, "unknown flags");
    IrProgram ir;
    std::string err;
    if (!ir_parse(ir_text, len, &ir, &err)) return fail(SIM_EINVAL, err);
    PackedProgram pk;
    int rc = pack_program(ir, 12, &pk, &err, !(flags & SIM_IR_KEEP_VANISHING));
    if (rc) return fail(rc, err);
    fill_info(pk, 0.0, 0, 0, out);
    return SIM_OK;
}

extern "C" int sim_ir_info(const char *ir_text, size_t len, sim_info *out) {
    return sim_ir_info_flags(ir_text, len, 0u, out);
}

extern "C" int sim_ir_affine_layout(const char *ir_text, size_t len, uint64_t *x0, uint64_t *cols, uint32_t cap,
                                    uint32_t *p_out) {
    if (!ir_text || !x0 || !p_out) return fail(SIM_EINVAL, "null argument");
    IrProgram ir;
    std::string err;
    if (!ir_parse(ir_text, len, &ir, &err)) return fail(SIM_EINVAL, err);
    PackedProgram pk;
    int rc = pack_program(ir, 12, &pk, &err);
    if (rc) return fail(rc, err);
    *p_out = (uint32_t)pk.p;
    if (cap < (uint32_t)pk.p || (!cols && pk.p)) return fail(SIM_ERANGE, "cols buffer shorter than p");
    *x0 = pk.lay_x0;
    for (int j = 0; j < pk.p; ++j) cols[j] = pk.lay_cols[j];
    return SIM_OK;
}

extern "C" int sim_compile_to_ir(const char *circuit_text, size_t len, const sim_query *q,
                                 const sim_compile_opts *opts, char *buf, size_t cap, size_t *len_out,
                                 sim_info *info) {
    if (!circuit_text || !q) return fail(SIM_EINVAL, "null argument");
    CompileOptions co;
    if (opts) {
        if (opts->p_cap) co.p_cap = (int)opts->p_cap;
        co.eliminate_constraints = opts->eliminate_constraints != 0;
        co.hub_params = opts->t_spiders_only == 0;
    }
    CompileStats cs;
    std::string err;
    IrProgram ir;
    auto t0 = std::chrono::steady_clock::now();
    int rc = compile_circuit(circuit_text, len, *q, co, &ir, &cs, &err);
    auto t1 = std::chrono::steady_clock::now();
    if (rc) return fail(rc, err);
    std::string s = ir_print(ir);
    if (len_out) *len_out = s.size();
    if (info) {
        PackedProgram pk;
        rc = pack_program(ir, 12, &pk, &err);
        if (rc) return fail(rc, err);
        fill_info(pk, std::chrono::duration<double>(t1 - t0).count(), (uint32_t)cs.t_count,
                  (uint32_t)cs.n_constraints, info);
    }
    if (buf) {
        if (cap < s.size() + 1) return fail(SIM_ERANGE, "buffer too small for the IR text");
        memcpy(buf, s.c_str(), s.size() + 1);
    }
    return SIM_OK;
}

extern "C" {

int sim_program_info(const sim_program *P, sim_info *out) {
    if (!P || !out) return fail(SIM_EINVAL, "null argument");
    fill_info(P->pk, P->compile_seconds, P->t_count, P->n_constraints, out);
    return SIM_OK;
}

int sim_program_ir(const sim_program *P, char *buf, size_t cap, size_t *len_out) {
    if (!P) return fail(SIM_EINVAL, "null argument");
    std::string s = ir_print(P->ir);
    if (len_out) *len_out = s.size();
    if (!buf) return SIM_OK;
    if (cap < s.size() + 1) return fail(SIM_ERANGE, "buffer too small for the IR text");
    memcpy(buf, s.c_str(), s.size() + 1);
    return SIM_OK;
}

int sim_program_layout(const sim_program *P, int32_t *perm, uint32_t cap) {
    if (!P || (!perm && P->pk.p)) return fail(SIM_EINVAL, "null argument");
    if (P->pk.eliminated)
        return fail(SIM_EINVAL, "the program's vanishing conditions were eliminated: use sim_program_affine_layout");
    if (cap < (uint32_t)P->pk.p) return fail(SIM_ERANGE, "perm buffer shorter than p");
    for (int j = 0; j < P->pk.p; ++j) perm[j] = P->pk.perm[j];
    return SIM_OK;
}

int sim_program_affine_layout(const sim_program *P, uint64_t *x0, uint64_t *cols, uint32_t cap) {
    if (!P || !x0 || (!cols && P->pk.p)) return fail(SIM_EINVAL, "null argument");
    if (cap < (uint32_t)P->pk.p) return fail(SIM_ERANGE, "cols buffer shorter than p");
    *x0 = P->pk.lay_x0;
    for (int j = 0; j < P->pk.p; ++j) cols[j] = P->pk.lay_cols[j];
    return SIM_OK;
}

int sim_eval_amplitude(const sim_program *P, void *stream, sim_zomega *out) {
    if (!P || !out) return fail(SIM_EINVAL, "null argument");
    if (P->pk.zero) {
        zero_result(out, false);
        return SIM_OK;
    }
    DeviceState *D;
    int rc = enter_device(P, &D);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(D->mu);
    if ((rc = settle(*D))) return rc;
    return eval_range_locked(*D, P, 0, P->pk.n_slices, false, (hipStream_t)stream, nullptr, out);
}

int sim_eval_timed(const sim_program *P, void *stream, sim_zomega *out, float *kernel_ms) {
    if (!P || !out || !kernel_ms) return fail(SIM_EINVAL, "null argument");
    if (P->pk.zero) {
        zero_result(out, false);
        *kernel_ms = 0.f;
        return SIM_OK;
    }
    DeviceState *D;
    int rc = enter_device(P, &D);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(D->mu);
    if ((rc = settle(*D))) return rc;
    return eval_range_locked(*D, P, 0, P->pk.n_slices, false, (hipStream_t)stream, nullptr, out, kernel_ms);
}

int sim_enqueue_amplitude(const sim_program *P, void *stream, void *ev_before, void *ev_after, sim_zomega *dev_out) {
    if (!P || !dev_out) return fail(SIM_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(dev_out) % 8) return fail(SIM_EINVAL, "dev_out must be 8-byte aligned");
    DeviceState *D;
    int rc = enter_device(P, &D);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(D->mu);
    hipStream_t st = (hipStream_t)stream;
    if (P->pk.zero) {
        static const sim_zomega zero = {};
        if (D->pending && D->pending_stream != st && (rc = settle(*D))) return rc;
        if (ev_before) HIP_TRY(hipEventRecord((hipEvent_t)ev_before, st));
        if (ev_after) HIP_TRY(hipEventRecord((hipEvent_t)ev_after, st));
        HIP_TRY(hipMemcpyAsync(dev_out, &zero, sizeof zero, hipMemcpyHostToDevice, st));
        return SIM_OK;
    }
    SinglePlan S;
    Region R;
    if ((rc = plan_single(*D, P, P->pk.n_slices, nullptr, &S))) return rc;
    if ((rc = lib_region(*D, S.o_res, &R, st))) return rc;
    if ((rc = await_upload(P))) return rc;
    Partial *parts = (Partial *)R.base;
    HIP_TRY(launch_eval(P->pk.hdr, P->dimg, 0, P->pk.n_slices, parts, S.blocks, S.threads, st,
                        (hipEvent_t)ev_before, (hipEvent_t)ev_after));
    HIP_TRY(launch_finalize(parts, S.blocks, final_args(P->pk, false), reinterpret_cast<DevResult *>(dev_out), st));
    D->pending = true;
    D->pending_stream = st;
    return SIM_OK;
}

int sim_eval_range(const sim_program *P, uint64_t first_slice, uint64_t n_slices, void *stream, sim_zomega *raw) {
    if (!P || !raw) return fail(SIM_EINVAL, "null argument");
    if (first_slice > P->pk.n_slices || n_slices > P->pk.n_slices - first_slice)
        return fail(SIM_EINVAL, "slice range outside the program");
    if (P->pk.zero || n_slices == 0) {
        zero_result(raw, true);
        return SIM_OK;
    }
    DeviceState *D;
    int rc = enter_device(P, &D);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(D->mu);
    if ((rc = settle(*D))) return rc;
    return eval_range_locked(*D, P, first_slice, n_slices, true, (hipStream_t)stream, nullptr, raw);
}

int sim_raw_add(const sim_zomega *a, const sim_zomega *b, sim_zomega *out) {
    if (!a || !b || !out) return fail(SIM_EINVAL, "null argument");
    sim_zomega r;
    memset(&r, 0, sizeof r);
    for (int k = 0; k < 4; ++k) {
        i128 x = (i128)((unsigned __int128)a->c[k].lo | ((unsigned __int128)(uint64_t)a->c[k].hi << 64));
        i128 y = (i128)((unsigned __int128)b->c[k].lo | ((unsigned __int128)(uint64_t)b->c[k].hi << 64));
        i128 s;
        if (__builtin_add_overflow(x, y, &s)) return fail(SIM_ERANGE, "int128 overflow adding partials");
        r.c[k].lo = (uint64_t)s;
        r.c[k].hi = (int64_t)((unsigned __int128)s >> 64);
    }
    r.flags = SIM_ZOMEGA_RAW;
    *out = r;
    return SIM_OK;
}

int sim_finalize(const sim_program *P, const sim_zomega *raw, void *stream, sim_zomega *out) {
    if (!P || !raw || !out) return fail(SIM_EINVAL, "null argument");
    if (P->pk.zero) {
        zero_result(out, false);
        return SIM_OK;
    }
    DeviceState *D;
    int rc = enter_device(P, &D);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(D->mu);
    if ((rc = settle(*D))) return rc;
    hipStream_t st = (hipStream_t)stream;
    Region R;
    const size_t o_res = up256(sizeof(Partial));
    if ((rc = lib_region(*D, o_res + up256(sizeof(DevResult)), &R, st))) return rc;
    if ((rc = ensure_host(*D, sizeof(DevResult)))) return rc;
    Partial part;
    for (int k = 0; k < 4; ++k) {
        part.w[2 * k] = raw->c[k].lo;
        part.w[2 * k + 1] = (uint64_t)raw->c[k].hi;
    }
    HIP_TRY(hipMemcpyAsync(R.base, &part, sizeof part, hipMemcpyHostToDevice, st));
    FinalArgs fa = final_args(P->pk, false);
    HIP_TRY(launch_finalize((Partial *)R.base, 1, fa, (DevResult *)(R.base + o_res), st));
    HIP_TRY(hipMemcpyAsync(D->host_result, R.base + o_res, sizeof(DevResult), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    DevResult r;
    memcpy(&r, D->host_result, sizeof r);
    return to_zomega(r, out);
}

void sim_program_free(sim_program *P) {
    if (!P) return;
    if (P->dimg) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(P->device);
        if (P->up_ev) {
            (void)hipEventSynchronize(P->up_ev);
            (void)hipEventDestroy(P->up_ev);
        }
        (void)hipFree(P->dimg);
        (void)hipSetDevice(cur);
    }
    delete P;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

// work list of a batch: programs grouped by kernel variant (W, monomials), each program's
// slices cut into items of about 2^chunk_log2 terms
struct BatchLayout {
    struct Group {
        uint32_t W = 1, mono = 0, acc = 0;
        uint32_t item_first = 0, n_items = 0;
        uint32_t lds_bytes = 0;
        ImgHeader h0;
    };
    std::vector<Group> groups;
    std::vector<WorkItem> items;
    std::vector<ImgHeader> hdrs;
    std::vector<uint64_t> imgs;
    std::vector<uint32_t> firsts, counts;  // per program: its items
    std::vector<FinalArgs> args;
    std::vector<uint32_t> live;  // indices of programs that need the GPU
    // programs large enough to fill the GPU alone run as single-program launches (resident grid)
    // beside the work queue of the small ones; their partials follow the items'
    struct Big {
        uint32_t prog;
        uint64_t s0, count;
        uint32_t blocks, slot;
    };
    std::vector<Big> big;
    size_t n_partials = 0;
};

// terms from which a program in a batch gets its own launch
constexpr uint64_t kBigTerms = (uint64_t)1 << 26;
constexpr uint32_t kBigThreads = 256;

constexpr uint64_t kMaxItemsPerProgram = 4096;
constexpr uint32_t kMinItemLog2 = 20;

int build_layout(DeviceState &D, const sim_program *const *ps, size_t n, const uint64_t *first_slice,
                 const uint64_t *n_slices, bool raw, const sim_tuning *t, BatchLayout *L) {
    L->hdrs.resize(n);
    L->imgs.resize(n);
    L->firsts.assign(n, 0);
    L->counts.assign(n, 0);
    L->args.resize(n);
    std::vector<uint32_t> order;
    for (size_t i = 0; i < n; ++i) {
        const sim_program *P = ps[i];
        L->hdrs[i] = P->pk.hdr;
        if (int rc = await_upload(P)) return rc;
        L->imgs[i] = (uint64_t)(uintptr_t)P->dimg;
        L->args[i] = final_args(P->pk, raw);
        uint64_t cnt = n_slices ? n_slices[i] : P->pk.n_slices;
        if (P->pk.zero || !cnt) continue;
        const uint32_t lg = std::min<uint32_t>(P->pk.hdr.g, 62);
        if (cnt >= (kBigTerms >> lg)) {
            BatchLayout::Big b;
            b.prog = (uint32_t)i;
            b.s0 = first_slice ? first_slice[i] : 0;
            b.count = cnt;
            b.slot = 0;
            int rc = eval_grid(D, P, cnt, kBigThreads, nullptr, &b.blocks);
            if (rc) return rc;
            L->big.push_back(b);
            L->live.push_back((uint32_t)i);
            continue;
        }
        order.push_back((uint32_t)i);
    }
    // group by kernel variant, keep program order inside a group
    auto menu_of = [](const ImgHeader &H) { return H.acc == ACC_I128 ? 0u : H.slot_menu; };
    // the node-slots-in-word-0 variants exist for widths 2 to 8 with the node or full slot sets
    auto word0_of = [&](const ImgHeader &H) {
        return H.node_word0 && H.W > 1 && H.W < 16 && H.acc != ACC_I128 && menu_of(H) < 2 ? 1u : 0u;
    };
    auto variant = [&](uint32_t i) {
        const ImgHeader &H = ps[i]->pk.hdr;
        return (((H.W * 2 + H.has_mono) * 4 + H.acc) * 4 + menu_of(H)) * 2 + word0_of(H);
    };
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return variant(a) < variant(b); });
    for (uint32_t i : order) {
        const sim_program *P = ps[i];
        const ImgHeader &H = P->pk.hdr;
        const uint32_t menu = menu_of(H), word0 = word0_of(H);
        if (L->groups.empty() || L->groups.back().W != H.W || L->groups.back().mono != H.has_mono ||
            L->groups.back().acc != H.acc || L->groups.back().h0.slot_menu != menu ||
            L->groups.back().h0.node_word0 != word0) {
            BatchLayout::Group g;
            g.W = H.W;
            g.mono = H.has_mono;
            g.acc = H.acc;
            g.item_first = (uint32_t)L->items.size();
            g.h0 = H;
            g.h0.slot_menu = menu;
            g.h0.node_word0 = word0;
            L->groups.push_back(g);
        }
        BatchLayout::Group &g = L->groups.back();
        g.lds_bytes = std::max<uint32_t>(g.lds_bytes, (uint32_t)dyn_lds_bytes(H));
        if (H.g > g.h0.g) g.h0.g = H.g;  // flush interval follows the longest walk of the group
        uint64_t s0 = first_slice ? first_slice[i] : 0;
        uint64_t cnt = n_slices ? n_slices[i] : P->pk.n_slices;
        // slices per item: with an explicit chunk, 2^chunk_log2 terms; by default at least one
        // slice per thread of a workgroup and 2^kMinItemLog2 terms (the per-item costs of the
        // queue, the LDS set-up and the reduction stay small), and at most kMaxItemsPerProgram
        // items per program
        uint64_t per;
        if (t && t->chunk_log2) {
            per = t->chunk_log2 > H.g ? ((uint64_t)1 << std::min<uint32_t>(62, t->chunk_log2 - H.g)) : 1;
        } else {
            const uint64_t min_terms = H.g < kMinItemLog2 ? (uint64_t)1 << (kMinItemLog2 - H.g) : 1;
            per = std::max<uint64_t>(std::max<uint64_t>(256, min_terms),
                                     (cnt + kMaxItemsPerProgram - 1) / kMaxItemsPerProgram);
        }
        L->firsts[i] = (uint32_t)L->items.size();
        for (uint64_t s = 0; s < cnt; s += per) {
            WorkItem wi;
            wi.prog = i;
            wi.out_slot = (uint32_t)L->items.size();
            wi.s_begin = s0 + s;
            wi.s_end = s0 + std::min(cnt, s + per);
            L->items.push_back(wi);
        }
        L->counts[i] = (uint32_t)L->items.size() - L->firsts[i];
        g.n_items = (uint32_t)L->items.size() - g.item_first;
        L->live.push_back(i);
    }
    size_t slot = L->items.size();
    for (auto &b : L->big) {
        b.slot = (uint32_t)slot;
        L->firsts[b.prog] = b.slot;
        L->counts[b.prog] = b.blocks;
        slot += b.blocks;
    }
    L->n_partials = slot;
    if (L->n_partials > 0xffffffffu) return fail(SIM_ERANGE, "too many work items");
    return SIM_OK;
}

// enqueues the batch on `stream` (no host synchronisation); buffers must be uploaded
int enqueue_batch(DeviceState &D, const BatchLayout &L, size_t n, const sim_tuning *t, hipStream_t stream,
                  const ImgHeader *d_hdrs, const uint64_t *d_imgs, const WorkItem *d_items,
                  Partial *d_parts, const uint32_t *d_firsts, const uint32_t *d_counts, const FinalArgs *d_args,
                  DevResult *d_out, bool allow_fork = true, const Partial *d_carry = nullptr,
                  const uint32_t *d_slots = nullptr, const uint32_t *d_flags = nullptr, DevResult *d_slot_carry = nullptr) {
    const uint32_t threads = pick_threads(t);
    const size_t ng = L.groups.size();
    // kernel variants run concurrently: group k on auxiliary stream k % kAux, forked from and
    // joined back into `stream` with events (also valid under stream capture); without
    // allow_fork every launch goes to `stream`
    const bool fork = allow_fork && (ng > 1 || (ng > 0 && !L.big.empty()));
    if (fork) {
        int rc = ensure_aux(D);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(D.ev_fork, stream));
        for (int a = 0; a < kAux; ++a) HIP_TRY(hipStreamWaitEvent(D.aux[a], D.ev_fork, 0));
    }
    uint32_t gi = 0;
    for (const auto &g : L.groups) {
        hipStream_t s = fork ? D.aux[gi % kAux] : stream;
        HIP_TRY(launch_eval_batch(g.h0, d_hdrs, d_imgs, d_items + g.item_first, g.n_items, d_parts, threads,
                                  g.lds_bytes, s));
        ++gi;
    }
    // the large programs one after another on the caller's stream, beside the item groups
    for (const auto &b : L.big)
        HIP_TRY(launch_eval(L.hdrs[b.prog], (const void *)(uintptr_t)L.imgs[b.prog], b.s0, b.count,
                            d_parts + b.slot, b.blocks, kBigThreads, stream));
    if (fork) {
        for (int a = 0; a < kAux && a < (int)ng; ++a) {
            HIP_TRY(hipEventRecord(D.ev_join[a], D.aux[a]));
            HIP_TRY(hipStreamWaitEvent(stream, D.ev_join[a], 0));
        }
    }
    if (d_slots)
        HIP_TRY(launch_serve_finalize(d_parts, d_firsts, d_counts, d_args, d_slots, d_flags, (uint32_t)n, d_slot_carry,
                                      d_out, stream));
    else
        HIP_TRY(launch_finalize_batch(d_parts, d_firsts, d_counts, d_args, (uint32_t)n, d_out, stream, d_carry));
    return SIM_OK;
}

// device addresses of the pieces of a batch layout inside one region
struct LayoutPtrs {
    const ImgHeader *hdrs;
    const uint64_t *imgs;
    const WorkItem *items;
    const uint32_t *firsts, *counts;
    const FinalArgs *args;
    Partial *parts;
    DevResult *res;  // null when the results go elsewhere (sim_enqueue_batch)
};

// Byte offsets of a batch inside its region: the work layout (headers, image addresses, item
// ranges, finaliser arguments, work items: uploaded with one copy), the partials and, unless the
// caller provides device memory for them, the results.
struct BatchPlan {
    size_t o_hdrs = 0, o_imgs = 0, o_firsts = 0, o_counts = 0, o_args = 0, o_items = 0, stage = 0;
    size_t o_parts = 0, o_res = 0, total = 0;
};

size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

BatchPlan plan_batch(const BatchLayout &L, size_t n, bool results) {
    BatchPlan B;
    B.o_hdrs = 0;
    B.o_imgs = align16(B.o_hdrs + n * sizeof(ImgHeader));
    B.o_firsts = align16(B.o_imgs + n * 8);
    B.o_counts = align16(B.o_firsts + n * 4);
    B.o_args = align16(B.o_counts + n * 4);
    B.o_items = align16(B.o_args + n * sizeof(FinalArgs));
    B.stage = align16(B.o_items + L.items.size() * sizeof(WorkItem)) + 16;
    B.o_parts = up256(B.stage);
    B.o_res = up256(B.o_parts + std::max<size_t>(1, L.n_partials) * sizeof(Partial));
    B.total = results ? up256(B.o_res + std::max<size_t>(1, n) * sizeof(DevResult)) : B.o_res;
    return B;
}

void pack_stage(const BatchLayout &L, size_t n, const BatchPlan &B, char *h) {
    if (n) {
        memcpy(h + B.o_hdrs, L.hdrs.data(), n * sizeof(ImgHeader));
        memcpy(h + B.o_imgs, L.imgs.data(), n * 8);
        memcpy(h + B.o_firsts, L.firsts.data(), n * 4);
        memcpy(h + B.o_counts, L.counts.data(), n * 4);
        memcpy(h + B.o_args, L.args.data(), n * sizeof(FinalArgs));
    }
    if (!L.items.empty()) memcpy(h + B.o_items, L.items.data(), L.items.size() * sizeof(WorkItem));
}

LayoutPtrs layout_ptrs(const BatchPlan &B, const Region &R, bool results) {
    LayoutPtrs P;
    P.hdrs = (const ImgHeader *)(R.base + B.o_hdrs);
    P.imgs = (const uint64_t *)(R.base + B.o_imgs);
    P.firsts = (const uint32_t *)(R.base + B.o_firsts);
    P.counts = (const uint32_t *)(R.base + B.o_counts);
    P.args = (const FinalArgs *)(R.base + B.o_args);
    P.items = (const WorkItem *)(R.base + B.o_items);
    P.parts = (Partial *)(R.base + B.o_parts);
    P.res = results ? (DevResult *)(R.base + B.o_res) : nullptr;
    return P;
}

// Uploads the work layout into R: from the library's pinned staging (library scratch), or from
// pageable host memory that `keep` holds until the caller has waited on the stream.
int upload_stage(DeviceState &D, const BatchLayout &L, size_t n, const BatchPlan &B, const Region &R, bool lib,
                 hipStream_t st, std::vector<char> *keep) {
    char *h;
    if (lib) {
        if (D.host_stage_cap < B.stage) {
            if (D.host_stage) (void)hipHostFree(D.host_stage);
            D.host_stage = nullptr;
            D.host_stage_cap = 0;
            const size_t cap = std::max<size_t>(B.stage, 1 << 16);
            hipError_t e = hipHostMalloc(&D.host_stage, cap, hipHostMallocDefault);
            if (e != hipSuccess) return fail(SIM_ENOMEM, std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
            D.host_stage_cap = cap;
        }
        h = (char *)D.host_stage;
    } else {
        keep->assign(B.stage, 0);
        h = keep->data();
    }
    pack_stage(L, n, B, h);
    HIP_TRY(hipMemcpyAsync(R.base, h, B.stage, hipMemcpyHostToDevice, st));
    return SIM_OK;
}

int check_batch_args(const sim_program *const *ps, size_t n, int *dev) {
    if (n && !ps) return fail(SIM_EINVAL, "null program list");
    for (size_t i = 0; i < n; ++i)
        if (!ps[i]) return fail(SIM_EINVAL, "null program in batch");
    if (n) {
        *dev = ps[0]->device;
        for (size_t i = 1; i < n; ++i)
            if (ps[i]->device != *dev) return fail(SIM_EINVAL, "programs of one batch must share a device");
    } else {
        HIP_TRY(hipGetDevice(dev));
    }
    return init_device(*dev);
}

int check_ranges(const sim_program *const *ps, size_t n, const uint64_t *first, const uint64_t *count) {
    if (first && count)
        for (size_t i = 0; i < n; ++i)
            if (first[i] > ps[i]->pk.n_slices || count[i] > ps[i]->pk.n_slices - first[i])
                return fail(SIM_EINVAL, "slice range outside a program");
    return SIM_OK;
}

// A blocking batch in region R (caller memory or the file-scope array; null: the library's
// scratch): upload, kernels, finaliser, copy of the results to host memory, wait.  Device lock
// held.
int run_batch_locked(DeviceState &D, const sim_program *const *ps, size_t n, const uint64_t *first,
                     const uint64_t *count, bool raw, hipStream_t st, const sim_tuning *t, const Region *given,
                     sim_zomega *out, bool allow_fork = true) {
    int rc;
    BatchLayout L;
    if ((rc = build_layout(D, ps, n, first, count, raw, t, &L))) return rc;
    const BatchPlan B = plan_batch(L, n, true);
    Region R;
    const bool lib = given == nullptr;
    if (lib) {
        if ((rc = lib_region(D, B.total, &R, st))) return rc;
        if ((rc = ensure_host(D, std::max<size_t>(1, n) * sizeof(DevResult)))) return rc;
    } else {
        if (given->cap < B.total)
            return fail(SIM_ERANGE, "scratch holds " + std::to_string(given->cap) + " bytes; the batch needs " +
                                        std::to_string(B.total));
        R = *given;
    }
    std::vector<char> keep;
    std::vector<DevResult> host(lib ? 0 : std::max<size_t>(1, n));
    DevResult *hres = lib ? (DevResult *)D.host_result : host.data();
    if (!L.live.empty()) {
        if ((rc = upload_stage(D, L, n, B, R, lib, st, &keep))) return rc;
        const LayoutPtrs LP = layout_ptrs(B, R, true);
        if ((rc = enqueue_batch(D, L, n, t, st, LP.hdrs, LP.imgs, LP.items, LP.parts, LP.firsts, LP.counts, LP.args,
                                LP.res, allow_fork)))
            return rc;
        HIP_TRY(hipMemcpyAsync(hres, LP.res, n * sizeof(DevResult), hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<sim_zomega> res(n);
    for (size_t i = 0; i < n; ++i) {
        const sim_program *P = ps[i];
        uint64_t cnt = count ? count[i] : P->pk.n_slices;
        if (P->pk.zero || cnt == 0) {
            zero_result(&res[i], raw);
            continue;
        }
        DevResult r;
        memcpy(&r, (const char *)hres + i * sizeof(DevResult), sizeof r);
        if ((rc = to_zomega(r, &res[i]))) return rc;
    }
    for (size_t i = 0; i < n; ++i) out[i] = res[i];
    return SIM_OK;
}

int run_batch(const sim_program *const *ps, size_t n, const uint64_t *first, const uint64_t *count, bool raw,
              void *stream, const sim_tuning *t, sim_zomega *out) {
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    if ((rc = check_ranges(ps, n, first, count))) return rc;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    if ((rc = settle(D))) return rc;
    return run_batch_locked(D, ps, n, first, count, raw, (hipStream_t)stream, t, nullptr, out);
}

}  // namespace

struct sim_batch_plan {
    int device = 0;
    size_t n = 0;
    std::vector<const sim_program *> progs;
    BatchLayout L;
    sim_tuning tuning;
    bool has_tuning = false;
    DevBuf hdrs, imgs, items, parts, firsts, counts, args, result;
    void *host_result = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

int sim_eval_batch(const sim_program *const *ps, size_t n, void *stream, const sim_tuning *t, sim_zomega *out) {
    if (n && !out) return fail(SIM_EINVAL, "null output");
    return run_batch(ps, n, nullptr, nullptr, false, stream, t, out);
}

int sim_eval_outcomes(const sim_program *P, size_t n, const uint8_t *bits, void *stream, const sim_tuning *t,
                      sim_zomega *out) {
    if (!P || (n && (!bits || !out))) return fail(SIM_EINVAL, "null argument");
    const int k = P->pk.outer;
    if (k <= 0) return fail(SIM_EINVAL, "the program has no query parameters (compile an OUTCOMES query)");
    // the query parameters are the top k bits of the slice index
    const uint32_t low = (uint32_t)(P->pk.hdr.pe - P->pk.hdr.g) - (uint32_t)k;
    std::vector<const sim_program *> ps(n, P);
    std::vector<uint64_t> first(n), count(n, (uint64_t)1 << low);
    for (size_t r = 0; r < n; ++r) {
        uint64_t y = 0;
        for (int i = 0; i < k; ++i) {
            const uint8_t b = bits[r * (size_t)k + i];
            if (b > 1) return fail(SIM_EINVAL, "output bits must be 0 or 1");
            y |= (uint64_t)b << i;
        }
        first[r] = y << low;
    }
    return run_batch(ps.data(), n, first.data(), count.data(), false, stream, t, out);
}

namespace {

// a * sqrt2 with overflow detection
bool times_sqrt2_checked(const Zw &z, Zw *out) {
    Zw r;
    if (__builtin_sub_overflow(z.c[1], z.c[3], &r.c[0]) || __builtin_add_overflow(z.c[0], z.c[2], &r.c[1]) ||
        __builtin_add_overflow(z.c[1], z.c[3], &r.c[2]) || __builtin_sub_overflow(z.c[2], z.c[0], &r.c[3]))
        return false;
    *out = r;
    return true;
}

// a sqrt2^ea - b sqrt2^eb, canonical; false on int128 overflow
bool sub_scaled(Zw a, int32_t ea, Zw b, int32_t eb, Zw *out, int32_t *eo) {
    if (zw_is_zero(b)) eb = ea;
    if (zw_is_zero(a)) ea = eb;
    for (; ea > eb; --ea)
        if (!times_sqrt2_checked(a, &a)) return false;
    for (; eb > ea; --eb)
        if (!times_sqrt2_checked(b, &b)) return false;
    Zw r;
    for (int i = 0; i < 4; ++i)
        if (__builtin_sub_overflow(a.c[i], b.c[i], &r.c[i])) return false;
    int32_t e = ea;
    zw_canonicalise(&r, &e);
    *out = r;
    *eo = e;
    return true;
}

Zw zw_of(const sim_zomega &v) {
    Zw z;
    for (int k = 0; k < 4; ++k) z.c[k] = (i128)(((unsigned __int128)(uint64_t)v.c[k].hi << 64) | v.c[k].lo);
    return z;
}

sim_zomega zomega_of(const Zw &z, int32_t e) {
    sim_zomega v;
    memset(&v, 0, sizeof v);
    for (int k = 0; k < 4; ++k) {
        v.c[k].lo = (uint64_t)z.c[k];
        v.c[k].hi = (int64_t)((unsigned __int128)z.c[k] >> 64);
    }
    v.sqrt2_exp = e;
    return v;
}

}  // namespace

int sim_sample(const sim_program *const *progs, size_t K, size_t n, const uint64_t *uniforms, void *stream,
               const sim_tuning *t, uint8_t *out_bits, sim_zomega *out_prob) {
    if (!progs || (n && (!uniforms || !out_bits))) return fail(SIM_EINVAL, "null argument");
    if (K < 1 || K > 62) return fail(SIM_EINVAL, "the number of sampled qubits must be 1 .. 62");
    for (size_t k = 1; k <= K; ++k)
        if (!progs[k - 1] || progs[k - 1]->pk.outer != (int)k)
            return fail(SIM_EINVAL, "progs[" + std::to_string(k - 1) + "] must have " + std::to_string(k) +
                                        " query parameters (the prefix program of the first " +
                                        std::to_string(k) + " qubits)");
    for (size_t i = 0; i < n * K; ++i)
        if (uniforms[i] >> 53) return fail(SIM_EINVAL, "uniforms must be below 2^53");
    if (!n) return SIM_OK;
    // per sample: the bits drawn so far and their probability P(B) (canonical)
    std::vector<uint64_t> pre(n, 0);
    std::vector<Zw> pz(n, zw_one());
    std::vector<int32_t> pe(n, 0);
    std::vector<uint64_t> keys;
    std::vector<uint8_t> rows;
    std::vector<sim_zomega> res;
    std::vector<zreal::Real> p0;
    for (size_t k = 0; k < K; ++k) {
        // every distinct prefix is evaluated once: P(B || 0) for B = bits 0 .. k-1
        keys = pre;
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        const size_t nr = keys.size(), w = k + 1;
        rows.assign(nr * w, 0);
        for (size_t r = 0; r < nr; ++r)
            for (size_t j = 0; j < k; ++j) rows[r * w + j] = (uint8_t)((keys[r] >> j) & 1);
        res.resize(nr);
        int rc = sim_eval_outcomes(progs[k], nr, rows.data(), stream, t, res.data());
        if (rc) return rc;
        p0.resize(nr);
        for (size_t r = 0; r < nr; ++r)
            if (!zreal::real_of(zw_of(res[r]), res[r].sqrt2_exp, &p0[r]))
                return fail(SIM_EINVAL, "a prefix probability is not real: progs[" + std::to_string(k) +
                                            "] is not a prefix program");
        for (size_t i = 0; i < n; ++i) {
            const size_t r = (size_t)(std::lower_bound(keys.begin(), keys.end(), pre[i]) - keys.begin());
            zreal::Real pb;
            zreal::real_of(pz[i], pe[i], &pb);
            // bit k is 0 iff U / 2^53 < P(B || 0) / P(B), i.e. 2^53 P(B || 0) - U P(B) > 0
            const bool zero = zreal::sign_diff((uint64_t)1 << 53, p0[r], uniforms[i * K + k], pb) > 0;
            const Zw z0 = zw_of(res[r]);
            if (zero) {
                pz[i] = z0;
                pe[i] = res[r].sqrt2_exp;
            } else {
                pre[i] |= (uint64_t)1 << k;
                if (!sub_scaled(pz[i], pe[i], z0, res[r].sqrt2_exp, &pz[i], &pe[i]))
                    return fail(SIM_ERANGE, "a prefix probability exceeds int128");
            }
            out_bits[i * K + k] = zero ? 0 : 1;
        }
    }
    if (out_prob)
        for (size_t i = 0; i < n; ++i) out_prob[i] = zomega_of(pz[i], pe[i]);
    return SIM_OK;
}

namespace {

// canonical (a + b sqrt2) sqrt2^e as a Z[w] element (a, b, 0, -b); false if it exceeds int128
bool canonical_of(zreal::Real r, Zw *z, int32_t *e) {
    using namespace zreal;
    if (r.a.zero() && r.b.zero()) {
        *z = zw_zero();
        *e = 0;
        return true;
    }
    auto even = [](const BigInt &v) { return v.zero() || !(v.m[0] & 1); };
    auto half = [](const BigInt &v) {  // exact v / 2 of an even v
        BigInt h;
        h.neg = v.neg;
        h.m.assign(v.m.size(), 0);
        for (size_t i = 0; i < v.m.size(); ++i)
            h.m[i] = (v.m[i] >> 1) | (i + 1 < v.m.size() ? v.m[i + 1] << 31 : 0);
        h.trim();
        return h;
    };
    while (even(r.a) && even(r.b)) {  // divide by 2 = sqrt2^2
        r.a = half(r.a);
        r.b = half(r.b);
        r.e += 2;
    }
    if (even(r.a)) {  // (a + b sqrt2) / sqrt2 = b + (a / 2) sqrt2
        BigInt t = half(r.a);
        r.a = r.b;
        r.b = t;
        r.e += 1;
    }
    auto fits = [](const BigInt &v, i128 *out) {
        if (v.m.size() > 4 || (v.m.size() == 4 && (v.m[3] >> 31))) return false;
        unsigned __int128 u = 0;
        for (size_t i = v.m.size(); i-- > 0;) u = (u << 32) | v.m[i];
        *out = v.neg ? -(i128)u : (i128)u;
        return true;
    };
    i128 a, b;
    if (!fits(r.a, &a) || !fits(r.b, &b)) return false;
    *z = zw_make(a, b, 0, -b);
    *e = r.e;
    return true;
}

}  // namespace

int sim_marginal_sum(const sim_program *P, const uint8_t *pattern, void *stream, const sim_tuning *t,
                     sim_zomega *out) {
    if (!P || !pattern || !out) return fail(SIM_EINVAL, "null argument");
    const int k = P->pk.outer;
    if (k <= 0) return fail(SIM_EINVAL, "the program has no query parameters (compile an OUTCOMES query)");
    uint64_t fixed = 0;
    std::vector<int> free_pos;
    for (int i = 0; i < k; ++i) {
        if (pattern[i] == 2) free_pos.push_back(i);
        else if (pattern[i] <= 1) fixed |= (uint64_t)pattern[i] << i;
        else return fail(SIM_EINVAL, "pattern bytes must be 0, 1 or 2");
    }
    const size_t m = free_pos.size();
    if (m > kMaxMarginalFree)
        return fail(SIM_ERANGE, "at most " + std::to_string(kMaxMarginalFree) + " summed outcomes");
    if (P->pk.zero) {
        zero_result(out, false);
        return SIM_OK;
    }
    DeviceState *D;
    int rc = enter_device(P, &D);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(D->mu);
    if ((rc = settle(*D))) return rc;
    hipStream_t st = (hipStream_t)stream;
    // one slice range per string that matches the pattern (the outcomes are the top bits), in
    // chunks of at most 2^16 strings: each chunk's amplitudes stay on the device, where their
    // squares are added to two 384-bit sums (the accumulator lives in its own small buffer)
    const uint32_t low = (uint32_t)(P->pk.hdr.pe - P->pk.hdr.g) - (uint32_t)k;
    const uint64_t n = (uint64_t)1 << m;
    const uint64_t chunk = std::min<uint64_t>(n, (uint64_t)1 << 16);
    const uint32_t n_blocks = (uint32_t)std::min<uint64_t>(256, (chunk + kMaxThreads - 1) / kMaxThreads);
    const size_t acc_bytes = 2 * 6 * 8, part_off = 256;
    if ((rc = ensure(D->msum, part_off + (size_t)n_blocks * acc_bytes))) return rc;
    char *mbase = (char *)D->msum.ptr;
    {
        const std::vector<uint8_t> zeros(part_off, 0);
        HIP_TRY(hipMemcpyAsync(mbase, zeros.data(), part_off, hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    std::vector<const sim_program *> ps(chunk, P);
    std::vector<uint64_t> first(chunk), count(chunk, (uint64_t)1 << low);
    for (uint64_t c0 = 0; c0 < n; c0 += chunk) {
        const size_t nc = (size_t)std::min<uint64_t>(chunk, n - c0);
        for (size_t r = 0; r < nc; ++r) {
            uint64_t y = fixed;
            const uint64_t idx = c0 + r;
            for (size_t j = 0; j < m; ++j) y |= ((idx >> j) & 1) << free_pos[j];
            first[r] = y << low;
        }
        BatchLayout L;
        if ((rc = build_layout(*D, ps.data(), nc, first.data(), count.data(), false, t, &L))) return rc;
        const BatchPlan B = plan_batch(L, nc, true);
        Region R;
        if ((rc = lib_region(*D, B.total, &R, st))) return rc;
        if ((rc = upload_stage(*D, L, nc, B, R, true, st, nullptr))) return rc;
        const LayoutPtrs LP = layout_ptrs(B, R, true);
        if (!L.live.empty()) {
            if ((rc = enqueue_batch(*D, L, nc, t, st, LP.hdrs, LP.imgs, LP.items, LP.parts, LP.firsts, LP.counts,
                                    LP.args, LP.res)))
                return rc;
            HIP_TRY(launch_norm2_sum(LP.res, (uint32_t)nc, P->pk.e, (uint64_t *)(mbase + part_off), n_blocks,
                                     (uint64_t *)mbase, (uint32_t *)(mbase + acc_bytes), st));
        }
        // the staging buffers are reused by the next chunk
        HIP_TRY(hipStreamSynchronize(st));
    }
    uint64_t host[2 * 6 + 2];
    HIP_TRY(hipMemcpy(host, mbase, sizeof host, hipMemcpyDeviceToHost));
    if (((const uint32_t *)(host + 12))[0] & 1u)
        return fail(SIM_ERANGE, "an amplitude of the marginal leaves the 384-bit sums");
    auto big_of = [](const uint64_t *w) {  // 384-bit two's complement -> BigInt
        uint64_t v[6];
        for (int i = 0; i < 6; ++i) v[i] = w[i];
        BigInt r;
        r.neg = (v[5] >> 63) != 0;
        if (r.neg) {
            uint64_t carry = 1;
            for (int i = 0; i < 6; ++i) {
                const uint64_t x = ~v[i] + carry;
                carry = (carry && x == 0) ? 1u : 0u;
                v[i] = x;
            }
        }
        for (int i = 0; i < 6; ++i) {
            r.m.push_back((uint32_t)v[i]);
            r.m.push_back((uint32_t)(v[i] >> 32));
        }
        r.trim();
        return r;
    };
    zreal::Real acc;
    acc.a = big_of(host);
    acc.b = big_of(host + 6);
    acc.e = 2 * P->pk.e;
    Zw z = zw_zero();
    int32_t e = 0;
    if ((!acc.a.zero() || !acc.b.zero()) && !canonical_of(acc, &z, &e))
        return fail(SIM_ERANGE, "the marginal exceeds int128");
    *out = zomega_of(z, e);
    return SIM_OK;
}

int sim_eval_ranges(const sim_program *const *ps, const uint64_t *first_slice, const uint64_t *n_slices, size_t n,
                    void *stream, const sim_tuning *t, sim_zomega *raw) {
    if (n && (!raw || !first_slice || !n_slices)) return fail(SIM_EINVAL, "null argument");
    return run_batch(ps, n, first_slice, n_slices, true, stream, t, raw);
}

int sim_finalize_batch(const sim_program *const *ps, const sim_zomega *raws, size_t n, void *stream,
                       sim_zomega *out) {
    if (n && (!raws || !out)) return fail(SIM_EINVAL, "null argument");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    if (!n) return SIM_OK;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    if ((rc = settle(D))) return rc;
    hipStream_t st = (hipStream_t)stream;
    // one "item" per program whose partial is the raw sum given by the caller
    BatchLayout L;
    L.hdrs.resize(n);
    L.imgs.assign(n, 0);
    L.args.resize(n);
    L.firsts.resize(n);
    L.counts.assign(n, 1);
    for (size_t i = 0; i < n; ++i) {
        L.hdrs[i] = ps[i]->pk.hdr;
        L.args[i] = final_args(ps[i]->pk, false);
        L.firsts[i] = (uint32_t)i;
    }
    L.n_partials = n;
    const BatchPlan B = plan_batch(L, n, true);
    Region R;
    if ((rc = lib_region(D, B.total, &R, st))) return rc;
    if ((rc = ensure_host(D, n * sizeof(DevResult)))) return rc;
    if ((rc = upload_stage(D, L, n, B, R, true, st, nullptr))) return rc;
    const LayoutPtrs LP = layout_ptrs(B, R, true);
    std::vector<Partial> parts(n);
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < 4; ++k) {
            parts[i].w[2 * k] = raws[i].c[k].lo;
            parts[i].w[2 * k + 1] = (uint64_t)raws[i].c[k].hi;
        }
    HIP_TRY(hipMemcpyAsync(LP.parts, parts.data(), n * sizeof(Partial), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_finalize_batch(LP.parts, LP.firsts, LP.counts, LP.args, (uint32_t)n, LP.res, st));
    HIP_TRY(hipMemcpyAsync(D.host_result, LP.res, n * sizeof(DevResult), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<sim_zomega> res(n);
    for (size_t i = 0; i < n; ++i) {
        DevResult r;
        memcpy(&r, (const char *)D.host_result + i * sizeof(DevResult), sizeof r);
        if ((rc = to_zomega(r, &res[i]))) return rc;
    }
    for (size_t i = 0; i < n; ++i) out[i] = res[i];
    return SIM_OK;
}

void sim_batch_plan_free(sim_batch_plan *plan) {
    if (!plan) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(plan->device);
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    for (DevBuf *b : {&plan->hdrs, &plan->imgs, &plan->items, &plan->parts, &plan->firsts, &plan->counts,
                      &plan->args, &plan->result})
        if (b->ptr) (void)hipFree(b->ptr);
    if (plan->host_result) (void)hipHostFree(plan->host_result);
    (void)hipSetDevice(cur);
    delete plan;
}

int sim_batch_plan_create(const sim_program *const *ps, size_t n, const sim_tuning *t, void *stream,
                          sim_batch_plan **out) {
    if (!out) return fail(SIM_EINVAL, "null output");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    HIP_TRY(hipSetDevice(dev));
    std::unique_ptr<sim_batch_plan, void (*)(sim_batch_plan *)> plan(new sim_batch_plan(), sim_batch_plan_free);
    plan->device = dev;
    plan->n = n;
    plan->progs.assign(ps, ps + n);
    if (t) {
        plan->tuning = *t;
        plan->has_tuning = true;
    }
    // the device lock covers the layout (occupancy queries) and the capture (auxiliary streams)
    std::lock_guard<std::mutex> lk(g_dev[dev].mu);
    if ((rc = settle(g_dev[dev]))) return rc;
    if ((rc = build_layout(g_dev[dev], ps, n, nullptr, nullptr, false, t, &plan->L))) return rc;
    const BatchLayout &L = plan->L;
    hipStream_t st = (hipStream_t)stream;
    auto alloc = [&](DevBuf &b, size_t bytes) { return ensure(b, std::max<size_t>(bytes, 64)); };
    if ((rc = alloc(plan->hdrs, n * sizeof(ImgHeader))) || (rc = alloc(plan->imgs, n * 8)) ||
        (rc = alloc(plan->items, L.items.size() * sizeof(WorkItem))) ||
        (rc = alloc(plan->parts, L.n_partials * sizeof(Partial))) || (rc = alloc(plan->firsts, n * 4)) ||
        (rc = alloc(plan->counts, n * 4)) || (rc = alloc(plan->args, n * sizeof(FinalArgs))) ||
        (rc = alloc(plan->result, n * sizeof(DevResult))))
        return rc;
    HIP_TRY(hipHostMalloc(&plan->host_result, std::max<size_t>(1, n) * sizeof(DevResult), hipHostMallocDefault));
    if (n) {
        HIP_TRY(hipMemcpy(plan->hdrs.ptr, L.hdrs.data(), n * sizeof(ImgHeader), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(plan->imgs.ptr, L.imgs.data(), n * 8, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(plan->firsts.ptr, L.firsts.data(), n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(plan->counts.ptr, L.counts.data(), n * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(plan->args.ptr, L.args.data(), n * sizeof(FinalArgs), hipMemcpyHostToDevice));
    }
    if (!L.items.empty())
        HIP_TRY(hipMemcpy(plan->items.ptr, L.items.data(), L.items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    if (!L.live.empty()) {
        // capture the launch sequence once on a private stream
        hipStream_t cap;
        HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        DeviceState &D = g_dev[dev];
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = enqueue_batch(D, L, n, plan->has_tuning ? &plan->tuning : nullptr, cap,
                               (const ImgHeader *)plan->hdrs.ptr, (const uint64_t *)plan->imgs.ptr,
                               (const WorkItem *)plan->items.ptr,
                               (Partial *)plan->parts.ptr, (const uint32_t *)plan->firsts.ptr,
                               (const uint32_t *)plan->counts.ptr, (const FinalArgs *)plan->args.ptr,
                               (DevResult *)plan->result.ptr);
            if (rc == SIM_OK) {
                e = hipMemcpyAsync(plan->host_result, plan->result.ptr, n * sizeof(DevResult), hipMemcpyDeviceToHost,
                                   cap);
                if (e != hipSuccess) rc = fail(SIM_EDEVICE, std::string("hipMemcpyAsync failed: ") + hipGetErrorString(e));
            }
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(cap, &graph);
            plan->graph = graph;
            if (rc == SIM_OK && e2 != hipSuccess)
                rc = fail(SIM_EDEVICE, std::string("hipStreamEndCapture failed: ") + hipGetErrorString(e2));
        } else {
            rc = fail(SIM_EDEVICE, std::string("hipStreamBeginCapture failed: ") + hipGetErrorString(e));
        }
        (void)hipStreamDestroy(cap);
        if (rc) return rc;
        HIP_TRY(hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0));
    }
    (void)st;
    *out = plan.release();
    return SIM_OK;
}

int sim_batch_plan_run(sim_batch_plan *plan, void *stream, sim_zomega *out) {
    if (!plan || (plan->n && !out)) return fail(SIM_EINVAL, "null argument");
    HIP_TRY(hipSetDevice(plan->device));
    hipStream_t st = (hipStream_t)stream;
    if (plan->exec) {
        HIP_TRY(hipGraphLaunch(plan->exec, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    std::vector<sim_zomega> res(plan->n);
    for (size_t i = 0; i < plan->n; ++i) {
        const sim_program *P = plan->progs[i];
        if (P->pk.zero) {
            zero_result(&res[i], false);
            continue;
        }
        DevResult r;
        memcpy(&r, (const char *)plan->host_result + i * sizeof(DevResult), sizeof r);
        int rc = to_zomega(r, &res[i]);
        if (rc) return rc;
    }
    for (size_t i = 0; i < plan->n; ++i) out[i] = res[i];
    return SIM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ caller-owned scratch

namespace {

// a batch whose work layout sim_batch_prepare wrote into caller memory, by (device, address)
struct Prepared {
    uint64_t fp = 0;
    size_t n = 0;
    BatchLayout L;  // without its work items (they are on the device)
    BatchPlan B;
};
std::map<std::pair<int, uintptr_t>, Prepared> g_prepared;  // each device's entries under its lock

uint64_t batch_fingerprint(int dev, const sim_program *const *ps, size_t n, const sim_tuning *t) {
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&](uint64_t v) {
        for (int k = 0; k < 8; ++k) {
            h ^= (v >> (8 * k)) & 0xFFu;
            h *= 0x100000001b3ull;
        }
    };
    mix((uint64_t)dev);
    mix(n);
    for (size_t i = 0; i < n; ++i) {
        mix((uint64_t)(uintptr_t)ps[i]);
        mix((uint64_t)(uintptr_t)ps[i]->dimg);
    }
    const sim_tuning z = {0, 0, 0, 0};
    const sim_tuning &u = t ? *t : z;
    mix(((uint64_t)u.block_threads << 32) | u.blocks_per_cu);
    mix(((uint64_t)u.walk_bits << 32) | u.chunk_log2);
    return h;
}

// the single-program and batch needs of a set of programs (device lock held)
int scratch_need(DeviceState &D, const sim_program *const *ps, size_t n, const sim_tuning *t, size_t *need) {
    size_t m = up256(sizeof(Partial)) + up256(sizeof(DevResult));  // sim_finalize-sized calls
    for (size_t i = 0; i < n; ++i) {
        if (ps[i]->pk.zero) continue;
        SinglePlan S;
        int rc = plan_single(D, ps[i], ps[i]->pk.n_slices, t, &S);
        if (rc) return rc;
        m = std::max(m, S.total);
    }
    BatchLayout L;
    int rc = build_layout(D, ps, n, nullptr, nullptr, false, t, &L);
    if (rc) return rc;
    m = std::max(m, plan_batch(L, n, true).total);
    *need = m;
    return SIM_OK;
}

// one program in caller memory: [first, first + count) in slices
int eval_single_ws(const sim_program *P, uint64_t first, uint64_t count, bool raw, void *stream, void *dev_scratch,
                   size_t scratch_bytes, sim_zomega *out) {
    if (P->pk.zero || count == 0) {
        zero_result(out, raw);
        return SIM_OK;
    }
    DeviceState *D;
    int rc = enter_device(P, &D);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(D->mu);
    SinglePlan S;
    Region R;
    if ((rc = plan_single(*D, P, count, nullptr, &S))) return rc;
    if ((rc = caller_region(dev_scratch, scratch_bytes, S.total, &R))) return rc;
    return eval_single(P, first, count, raw, S, R, nullptr, (hipStream_t)stream, out);
}

}  // namespace

extern "C" {

int sim_scratch_bytes(const sim_program *const *ps, size_t n, const sim_tuning *t, size_t *bytes) {
    if (!bytes) return fail(SIM_EINVAL, "null argument");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    size_t need = 0;
    if ((rc = scratch_need(D, ps, n, t, &need))) return rc;
    *bytes = need;
    return SIM_OK;
}

int sim_eval_amplitude_ws(const sim_program *P, void *stream, void *dev_scratch, size_t scratch_bytes,
                          sim_zomega *out) {
    if (!P || !out) return fail(SIM_EINVAL, "null argument");
    return eval_single_ws(P, 0, P->pk.n_slices, false, stream, dev_scratch, scratch_bytes, out);
}

int sim_eval_range_ws(const sim_program *P, uint64_t first, uint64_t count, uint32_t g, void *stream,
                      void *dev_scratch, size_t scratch_bytes, sim_zomega *raw) {
    if (!P || !raw) return fail(SIM_EINVAL, "null argument");
    const uint32_t wb = (uint32_t)P->pk.walk_bits;
    if (g < wb || g > (uint32_t)P->pk.p)
        return fail(SIM_EINVAL, "g must lie between the program's walk bits (" + std::to_string(wb) + ") and p (" +
                                    std::to_string(P->pk.p) + ")");
    const uint32_t sh = g - wb;  // slices per unit: 2^sh
    const uint64_t units = P->pk.n_slices >> sh;
    if (first > units || count > units - first) return fail(SIM_EINVAL, "range outside the program");
    return eval_single_ws(P, first << sh, count << sh, true, stream, dev_scratch, scratch_bytes, raw);
}

int sim_eval_batch_ws(const sim_program *const *ps, size_t n, void *stream, void *dev_scratch, size_t scratch_bytes,
                      const sim_tuning *t, sim_zomega *out) {
    if (n && !out) return fail(SIM_EINVAL, "null output");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    Region R;
    if ((rc = caller_region(dev_scratch, scratch_bytes, 0, &R))) return rc;
    return run_batch_locked(D, ps, n, nullptr, nullptr, false, (hipStream_t)stream, t, &R, out);
}

int sim_batch_prepare(const sim_program *const *ps, size_t n, const sim_tuning *t, void *dev_scratch,
                      size_t scratch_bytes, void *stream) {
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    Prepared Pr;
    Pr.n = n;
    if ((rc = build_layout(D, ps, n, nullptr, nullptr, false, t, &Pr.L))) return rc;
    Pr.B = plan_batch(Pr.L, n, false);
    Region R;
    if ((rc = caller_region(dev_scratch, scratch_bytes, Pr.B.total, &R))) return rc;
    // the auxiliary streams of concurrent kernel variants exist before any capture
    if ((rc = ensure_aux(D))) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::vector<char> keep;
    if ((rc = upload_stage(D, Pr.L, n, Pr.B, R, false, st, &keep))) return rc;
    HIP_TRY(hipStreamSynchronize(st));
    Pr.L.items.clear();
    Pr.L.items.shrink_to_fit();
    Pr.fp = batch_fingerprint(dev, ps, n, t);
    g_prepared[{dev, reinterpret_cast<uintptr_t>(dev_scratch)}] = std::move(Pr);
    return SIM_OK;
}

int sim_enqueue_batch(const sim_program *const *ps, size_t n, void *stream, void *dev_scratch, size_t scratch_bytes,
                      const sim_tuning *t, sim_zomega *dev_out) {
    if (n && !dev_out) return fail(SIM_EINVAL, "null dev_out");
    if (reinterpret_cast<uintptr_t>(dev_out) % 8) return fail(SIM_EINVAL, "dev_out must be 8-byte aligned");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    auto it = g_prepared.find({dev, reinterpret_cast<uintptr_t>(dev_scratch)});
    if (it == g_prepared.end() || it->second.fp != batch_fingerprint(dev, ps, n, t))
        return fail(SIM_EINVAL, "dev_scratch does not hold this batch: call sim_batch_prepare with the same "
                                "programs and tuning first");
    const Prepared &Pr = it->second;
    Region R;
    if ((rc = caller_region(dev_scratch, scratch_bytes, Pr.B.total, &R))) return rc;
    if (!n) return SIM_OK;
    const LayoutPtrs LP = layout_ptrs(Pr.B, R, false);
    return enqueue_batch(D, Pr.L, n, t, (hipStream_t)stream, LP.hdrs, LP.imgs, LP.items, LP.parts, LP.firsts,
                         LP.counts, LP.args, reinterpret_cast<DevResult *>(dev_out));
}

int sim_batch_forget(void *dev_scratch) {
    int dev;
    HIP_TRY(hipGetDevice(&dev));
    int rc = init_device(dev);
    if (rc) return rc;
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    g_prepared.erase({dev, reinterpret_cast<uintptr_t>(dev_scratch)});
    return SIM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free entry point

extern "C" int sim_eval_ranges_static(const sim_program *const *ps, const uint64_t *first_slice,
                                      const uint64_t *n_slices, size_t n, void *stream, const sim_tuning *t,
                                      sim_zomega *raw) {
    if (n && (!raw || !first_slice || !n_slices)) return fail(SIM_EINVAL, "null argument");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    if ((rc = check_ranges(ps, n, first_slice, n_slices))) return rc;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    if (!D.static_scratch) return fail(SIM_EDEVICE, "the fixed scratch array has no address on this device");
    // the device lock serialises calls, and each waits for its stream before returning, so the
    // array is used by one call at a time
    std::lock_guard<std::mutex> lk(D.mu);
    Region R;
    R.base = (char *)D.static_scratch;
    R.cap = kStaticScratchBytes;
    // every launch on the caller's stream: no auxiliary streams are created
    return run_batch_locked(D, ps, n, first_slice, n_slices, true, (hipStream_t)stream, t, &R, raw, false);
}

// ------------------------------------------------------------------ serving step

extern "C" int sim_serve_step(const sim_program *const *ps, const uint64_t *first_slice, const uint64_t *n_slices,
                              const sim_zomega *carry, const uint8_t *last, size_t n, void *stream,
                              const sim_tuning *t, sim_zomega *out) {
    if (n && (!out || !first_slice || !n_slices || !last)) return fail(SIM_EINVAL, "null argument");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    if ((rc = check_ranges(ps, n, first_slice, n_slices))) return rc;
    if (carry)
        for (size_t i = 0; i < n; ++i)
            if (!(carry[i].flags & SIM_ZOMEGA_RAW)) return fail(SIM_EINVAL, "carry values must be raw partial sums");
    if (!n) return SIM_OK;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    if ((rc = settle(D))) return rc;
    hipStream_t st = (hipStream_t)stream;
    BatchLayout L;
    if ((rc = build_layout(D, ps, n, first_slice, n_slices, true, t, &L))) return rc;
    for (size_t i = 0; i < n; ++i) L.args[i].raw = last[i] ? 0u : 1u;  // finalise the requests that end here
    const BatchPlan B = plan_batch(L, n, true);
    // the carried sums follow the results in the same region
    const size_t o_carry = B.total;
    Region R;
    if ((rc = lib_region(D, o_carry + up256(n * sizeof(Partial)), &R, st))) return rc;
    if ((rc = ensure_host(D, n * sizeof(DevResult)))) return rc;
    if ((rc = upload_stage(D, L, n, B, R, true, st, nullptr))) return rc;
    std::vector<Partial> cp(n);
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < 4; ++k) {
            cp[i].w[2 * k] = carry ? carry[i].c[k].lo : 0u;
            cp[i].w[2 * k + 1] = carry ? (uint64_t)carry[i].c[k].hi : 0u;
        }
    HIP_TRY(hipMemcpyAsync(R.base + o_carry, cp.data(), n * sizeof(Partial), hipMemcpyHostToDevice, st));
    const LayoutPtrs LP = layout_ptrs(B, R, true);
    if ((rc = enqueue_batch(D, L, n, t, st, LP.hdrs, LP.imgs, LP.items, LP.parts, LP.firsts, LP.counts, LP.args,
                            LP.res, true, (const Partial *)(R.base + o_carry))))
        return rc;
    HIP_TRY(hipMemcpyAsync(D.host_result, LP.res, n * sizeof(DevResult), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::vector<sim_zomega> res(n);
    for (size_t i = 0; i < n; ++i) {
        if (ps[i]->pk.zero) {
            zero_result(&res[i], !last[i]);
            continue;
        }
        DevResult r;
        memcpy(&r, (const char *)D.host_result + i * sizeof(DevResult), sizeof r);
        if ((rc = to_zomega(r, &res[i]))) return rc;
    }
    for (size_t i = 0; i < n; ++i) out[i] = res[i];
    return SIM_OK;
}

// ------------------------------------------------------------------ pipelined serving step

extern "C" int sim_serve_enqueue(const sim_program *const *ps, const uint64_t *first_slice, const uint64_t *n_slices,
                                 const uint32_t *slots, const uint8_t *flags, size_t n, void *dev_carry,
                                 size_t n_carry_slots, void *stream, const sim_tuning *t, sim_zomega *dev_out) {
    if (n && (!first_slice || !n_slices || !slots || !flags || !dev_carry || !dev_out))
        return fail(SIM_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(dev_carry) % 8 || reinterpret_cast<uintptr_t>(dev_out) % 8)
        return fail(SIM_EINVAL, "dev_carry and dev_out must be 8-byte aligned");
    int dev, rc;
    if ((rc = check_batch_args(ps, n, &dev))) return rc;
    if ((rc = check_ranges(ps, n, first_slice, n_slices))) return rc;
    for (size_t i = 0; i < n; ++i) {
        if (slots[i] >= n_carry_slots) return fail(SIM_EINVAL, "carry slot out of range");
        if (flags[i] > 3) return fail(SIM_EINVAL, "flags must be 0 .. 3");
        for (size_t j = 0; j < i; ++j)
            if (slots[j] == slots[i]) return fail(SIM_EINVAL, "two requests of one step share a carry slot");
    }
    if (!n) return SIM_OK;
    HIP_TRY(hipSetDevice(dev));
    DeviceState &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    if ((rc = settle(D))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int r = (int)(D.ring_next++ % DeviceState::kRing);
    if (!D.ring_ev[r]) HIP_TRY(hipEventCreateWithFlags(&D.ring_ev[r], hipEventDisableTiming));
    if (D.ring_used[r]) HIP_TRY(hipEventSynchronize(D.ring_ev[r]));  // its previous step is done with it
    BatchLayout L;
    if ((rc = build_layout(D, ps, n, first_slice, n_slices, true, t, &L))) return rc;
    // programs without work (zero programs, empty ranges) still pass through the finaliser
    const BatchPlan B = plan_batch(L, n, false);
    const size_t o_slots = align16(B.stage);
    const size_t o_flags = align16(o_slots + n * 4);
    const size_t stage = align16(o_flags + n * 4);
    const size_t o_parts = up256(stage);
    const size_t total = o_parts + up256(std::max<size_t>(1, L.n_partials) * sizeof(Partial));
    if ((rc = ensure(D.ring_dev[r], total))) return rc;
    if (D.ring_host_cap[r] < stage) {
        if (D.ring_host[r]) (void)hipHostFree(D.ring_host[r]);
        D.ring_host[r] = nullptr;
        D.ring_host_cap[r] = 0;
        const size_t cap = std::max<size_t>(stage, 1 << 16);
        hipError_t e = hipHostMalloc(&D.ring_host[r], cap, hipHostMallocDefault);
        if (e != hipSuccess) return fail(SIM_ENOMEM, std::string("hipHostMalloc failed: ") + hipGetErrorString(e));
        D.ring_host_cap[r] = cap;
    }
    char *h = (char *)D.ring_host[r];
    pack_stage(L, n, B, h);
    uint32_t *hs = (uint32_t *)(h + o_slots), *hf = (uint32_t *)(h + o_flags);
    for (size_t i = 0; i < n; ++i) {
        hs[i] = slots[i];
        hf[i] = flags[i];
    }
    Region R;
    R.base = (char *)D.ring_dev[r].ptr;
    R.cap = D.ring_dev[r].cap;
    HIP_TRY(hipMemcpyAsync(R.base, h, stage, hipMemcpyHostToDevice, st));
    LayoutPtrs LP = layout_ptrs(B, R, false);
    LP.parts = (Partial *)(R.base + o_parts);
    if ((rc = enqueue_batch(D, L, n, t, st, LP.hdrs, LP.imgs, LP.items, LP.parts, LP.firsts, LP.counts, LP.args,
                            reinterpret_cast<DevResult *>(dev_out), true, nullptr, (const uint32_t *)(R.base + o_slots),
                            (const uint32_t *)(R.base + o_flags), reinterpret_cast<DevResult *>(dev_carry))))
        return rc;
    HIP_TRY(hipEventRecord(D.ring_ev[r], st));
    D.ring_used[r] = true;
    return SIM_OK;
}
