/*
 * zxpar: exact GPU evaluation of parametric ZX scalars on MI355X (gfx950).
 *
 * The method (Sutcliffe & Kissinger, "Fast Classical Simulation of Quantum Circuits via
 * Parametric Rewriting in the ZX-Calculus", QPL 2024): a Clifford+T diagram whose
 * decomposition terms differ only by pi phases is simplified once with Boolean parameters
 * (Section 3.1, Eq. 1), giving a parametric scalar (Section 3.2, Eq. 2-3) that is then
 * evaluated for every assignment of its p parameters on the GPU and summed (Section 3.3,
 * Appendix E).  Here that scalar is a "term program":
 *
 *     S = sqrt2^e * c * sum_{x in {0,1}^p} w^{phi(x)} * prod_j F_j(x),     w = e^{i pi/4},
 *
 * with F2-affine forms l(x) = const XOR parity(mask & x), node factors 1 + w^{a + b l(x)},
 * phase-pair factors (Eq. 3), and phi a Z/8 phase polynomial.  Every step is exact: values
 * live in Z[w] (four integer coefficients in the basis 1, w, w^2, w^3) with a shared power
 * of sqrt2; there is no floating point anywhere on the evaluation path.
 *
 * Conventions for every entry point:
 *   - return value: SIM_OK (0) or a negative SIM_E* code; no exception crosses the ABI;
 *   - on error, sim_last_error() returns a message for the calling thread and the output
 *     arguments are left untouched;
 *   - pointers are host pointers unless named dev_*; "stream" is a hipStream_t passed as
 *     void* (NULL = the null stream of the current device); outputs are caller-owned host
 *     memory; the call returns when the output is valid;
 *   - a sim_program is immutable after creation and owned by the library until
 *     sim_program_free; its device image lives on the device that was current when it was
 *     created, and it must be evaluated on that device;
 *   - evaluations on one device are serialised by the library (a per-device lock guards
 *     its scratch memory); programs may be created and freed from any thread.
 */
#ifndef ZXPAR_H
#define ZXPAR_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define SIM_API __attribute__((visibility("default")))
#else
#define SIM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,  /* bad argument, malformed IR or circuit text (message has the line) */
    SIM_ERANGE = -2,  /* p above the cap, or a static bound says int128 could overflow */
    SIM_ENOMEM = -3,  /* host or device allocation failed */
    SIM_EDEVICE = -4, /* a HIP call failed (message names it) */
    SIM_EBUSY = -5    /* admission refused: a memory budget would be exceeded */
};

typedef struct sim_program sim_program;

/* two's complement 128-bit integer */
typedef struct {
    uint64_t lo;
    int64_t hi;
} sim_i128;

/* value = (c[0] + c[1] w + c[2] w^2 + c[3] w^3) * sqrt2^sqrt2_exp.  Final results are in
 * canonical form: zero is all-zero with exponent 0; otherwise the coefficients are not all
 * divisible by sqrt2 (c1 = c3 and c0 = c2 mod 2 fails).  flags bit 0 = RAW: a partial sum
 * over assignments without the program's constant c and sqrt2^e (sim_eval_range). */
typedef struct {
    sim_i128 c[4];
    int32_t sqrt2_exp;
    uint32_t flags;
} sim_zomega;

#define SIM_ZOMEGA_RAW 1u
/* set by the device in an enqueued result (sim_enqueue_amplitude) whose product with the
 * program constant left int128: the value is invalid (sim_eval_amplitude returns SIM_ERANGE) */
#define SIM_ZOMEGA_OVERFLOW 2u

/* A query on a Clifford+T circuit (Section 2.2).  AMPLITUDE: <y|C|0^n> with y_i =
 * out_bits[i] (0/1 bytes, n_qubits of them).  MARGINAL: P(qubit = value) =
 * <0^n| C^dag (|value><value|_qubit (x) I) C |0^n>, the doubled diagram of Fig. 3.
 * OUTCOMES: the amplitude with every output bit y_i a Boolean parameter of the program (the
 * output effects become polar-phase spiders, Section 3.2), so one compilation serves every
 * output string (the repeated strong simulation of Section 4); out_bits is ignored and the
 * program's last n_qubits parameters are y_0 .. y_{n-1} (see sim_eval_outcomes).
 * PREFIX: the marginal of the first k = qubit qubits, P(y_0 .. y_{k-1}) =
 * <0^n| C^dag (|y><y|_{0..k-1} (x) I) C |0^n> (the doubled diagram of Fig. 3 right, the
 * k-th step of the repeated weak simulation of Appendix F), 1 <= k <= n_qubits.  With
 * out_bits NULL the k outcomes are query parameters (the program's last k parameters are
 * y_0 .. y_{k-1}, k <= 62; evaluate with sim_eval_outcomes or sim_sample); otherwise y_i =
 * out_bits[i] for i < k and the program is a plain scalar. */
enum { SIM_QUERY_AMPLITUDE = 0, SIM_QUERY_MARGINAL = 1, SIM_QUERY_OUTCOMES = 2, SIM_QUERY_PREFIX = 3 };
typedef struct {
    uint32_t kind;
    uint32_t n_qubits;
    const uint8_t *out_bits;
    uint32_t qubit;
    uint32_t value;
} sim_query;

/* p_cap: refuse (SIM_ERANGE) programs with more parameters (0 = 48).
 * eliminate_constraints: 1 (default when opts is NULL) substitutes away every parameter
 * fixed by a parity constraint of the simplified diagram (a factor that is 0 or 2), so the
 * program has p' <= p parameters and 2^p' terms; 0 keeps them as 0/2-valued factors.
 * t_spiders_only: 0 (default) lets the decomposition give a parameter to any spider, taking
 * the one that removes the most T-like spiders (itself, and its T-like neighbours of degree 1,
 * which become node factors); 1 parameterises T-like spiders only. */
typedef struct {
    uint32_t p_cap;
    uint32_t eliminate_constraints;
    uint32_t t_spiders_only;
    uint32_t reserved[5];
} sim_compile_opts;

typedef struct {
    uint32_t n_params;      /* p: terms of the program = 2^p */
    uint32_t n_forms;
    uint32_t n_factors;     /* node + pair factors after constant folding */
    uint32_t n_monomials;   /* variable monomials of phi */
    int32_t sqrt2_exp;      /* e of the program's constant */
    uint32_t walk_bits;     /* parameters enumerated inside one slice (2^walk_bits terms) */
    uint64_t n_slices;      /* 2^(p - walk_bits): the unit of sim_eval_range */
    uint64_t image_bytes;   /* device memory held by the program */
    double log2_terms;      /* p */
    uint32_t n_eval_params; /* parameters the kernel enumerates (p plus one per pair factor) */
    uint32_t is_zero;       /* the program is identically zero (a constant factor vanished) */
    double compile_seconds; /* host time spent in sim_compile (0 for IR programs) */
    uint32_t t_count;       /* T-like spiders before parameterisation (sim_compile only) */
    uint32_t n_constraints; /* parameters removed by constraint elimination */
    double ops_per_term;    /* int32 lane operations per term of the evaluation algorithm,
                               counted from the packed program (the roofline's work unit) */
    double nonzero_fraction; /* exact fraction of the 2^p assignments on which no factor
                               vanishes (only those terms reach the factor statistics) */
    uint32_t n_outer;       /* query parameters (OUTCOMES programs: n_qubits, else 0); an output
                               string costs 2^(p - n_outer) terms */
    uint32_t vanish_table_bits; /* z > 0: the vanishing factors own the low z bits of the form
                               vector and a block's surviving terms are read from a 2^z-entry
                               table; 0: found by the reduced-basis test (or nothing vanishes) */
    uint32_t n_params_given;  /* parameters of the program as given (before the elimination) */
    uint32_t n_eliminated;    /* parameters solved for by the exact elimination of the vanishing
                                 conditions: n_params = n_params_given - n_eliminated, and the
                                 2^n_params terms summed are exactly the nonzero ones' subspace */
    uint32_t n_form_monomials; /* phase monomials that the elimination turned into products of
                                 two or three affine forms */
    uint32_t n_mono_forms;    /* distinct forms of those products (at most 32) */
    uint32_t block_sum32;     /* 1: each 2^KB-term block's terms are added in 32 bits first (the
                                 node factors bound a block's sum below 2^31), then in 64 */
    uint32_t team_waves;      /* waves that share each block of the walk: 2 for small programs
                                 whose monomials are all form monomials (their per-half tables
                                 in LDS), else 1 */
} sim_info;

/* launch shape of the evaluation kernels; zero fields take the library's choice */
typedef struct {
    uint32_t block_threads;   /* 64..1024, multiple of 64 */
    uint32_t blocks_per_cu;   /* single-program grid: blocks per compute unit (0: as many as
                                 are resident at once); batches: unused */
    uint32_t walk_bits;       /* upper bound on the Gray-walk length log2 */
    uint32_t chunk_log2;      /* batch: log2 of terms per work item */
} sim_tuning;

/* Selects the device (hipSetDevice) and creates the library's state for it.  Optional:
 * every entry point initialises the current device on first use. */
SIM_API int sim_init(int device);

/* Parses a "zxir 1" term program and uploads its packed image to the current device.
 * Text layout (whitespace-separated, '#' starts a comment, sections in this order):
 *     zxir 1
 *     p <p>
 *     forms <F>   then F lines  f <const 0|1> <mask, hex; bit i = parameter x_i>
 *     nodes <N>   then N lines  n <form> <a> <b>            1 + w^{a + b l(x)}
 *     pairs <Q>   then Q lines  q <form1> <form2> <a> <b>   Eq. 3 with Psi = a pi/4 + pi l1,
 *                                                           Phi = b pi/4 + pi l2
 *     lin <K>     then K lines  l <c> <form>                phi += c l(x)
 *     mono <M>    then M lines  m <c> <d> <v_1> .. <v_d>    phi += c x_v1 .. x_vd
 *     scalar <c0> <c1> <c2> <c3> <e>                        c = c0 + c1 w + c2 w^2 + c3 w^3
 *     end
 * The text need not be NUL-terminated.  SIM_EINVAL on a malformed text (message names the
 * line), SIM_ERANGE when p > 62 or the static bound (sum of |term| over all terms) could
 * exceed int128. */
SIM_API int sim_program_from_ir(const char *ir_text, size_t len, sim_program **out);

/* sim_program_from_ir with flags: SIM_IR_KEEP_VANISHING keeps the factors that can vanish as
 * factors tested at run time instead of solving their conditions exactly (the default packs
 * the sum over the surviving affine subspace only; see sim_info.n_eliminated).  Same value
 * either way.  SIM_EINVAL on unknown flags. */
#define SIM_IR_KEEP_VANISHING 1u
SIM_API int sim_program_from_ir_flags(const char *ir_text, size_t len, uint32_t flags, sim_program **out);

/* Host-side compiler (Section 3): circuit text -> ZX diagram closed with |0^n> and the
 * query's effect -> parametric Clifford simplification with one Boolean parameter per
 * remaining T-like spider -> term program, uploaded like sim_program_from_ir.  opts may be
 * NULL.  SIM_EINVAL on a circuit or query error, SIM_ERANGE when p exceeds the cap. */
SIM_API int sim_compile(const char *circuit_text, size_t len, const sim_query *q,
                const sim_compile_opts *opts, sim_program **out);

SIM_API int sim_program_info(const sim_program *prog, sim_info *out);

/* Host only (no device needed): parses and packs an IR text and reports what
 * sim_program_from_ir would create, without uploading anything.  Same errors. */
SIM_API int sim_ir_info(const char *ir_text, size_t len, sim_info *out);

/* sim_ir_info with the flags of sim_program_from_ir_flags. */
SIM_API int sim_ir_info_flags(const char *ir_text, size_t len, uint32_t flags, sim_info *out);

/* Host only: sim_program_affine_layout of the program sim_program_from_ir would create from
 * the IR text; *p_out receives its n_params (also when cap is too small: SIM_ERANGE). */
SIM_API int sim_ir_affine_layout(const char *ir_text, size_t len, uint64_t *x0, uint64_t *cols, uint32_t cap,
                                 uint32_t *p_out);

/* Host only: runs the compiler of sim_compile and writes the resulting IR text into buf
 * (cap bytes, NUL-terminated; *len_out receives the full length, SIM_ERANGE if it does not
 * fit).  info (may be NULL) receives what sim_program_info would report. */
SIM_API int sim_compile_to_ir(const char *circuit_text, size_t len, const sim_query *q,
                      const sim_compile_opts *opts, char *buf, size_t cap, size_t *len_out,
                      sim_info *info);

/* Writes the program's IR text (as parsed or as compiled, before packing) into buf (cap
 * bytes, NUL-terminated when it fits); *len_out receives the full length.  SIM_ERANGE
 * when cap is too small (nothing written). */
SIM_API int sim_program_ir(const sim_program *prog, char *buf, size_t cap, size_t *len_out);

/* Assignment order of slices: slice s covers the 2^walk_bits assignments whose index, read
 * in the order perm[0..p-1] (bit j of the index is parameter perm[j]), lies in
 * [s << walk_bits, (s + 1) << walk_bits).  perm must hold p entries.  SIM_EINVAL for a program
 * whose vanishing conditions were eliminated (its slices are not a relabelling of the given
 * parameters' assignments): use sim_program_affine_layout. */
SIM_API int sim_program_layout(const sim_program *prog, int32_t *perm, uint32_t cap);

/* Assignments of the slice-ordered index t (0 <= t < 2^p, p = n_params; slice s covers
 * [s << walk_bits, (s + 1) << walk_bits)) as assignments of the n_params_given parameters of
 * the program as given: x(t) = *x0 XOR (XOR of cols[j] over the set bits j of t), bit i of an
 * assignment being parameter x_i.  Without elimination x0 = 0 and cols[j] = 1 << perm[j]; with
 * it (Section 5's vanishing factors solved for exactly) x(t) runs over the affine subspace on
 * which no factor vanishes, and every assignment outside it has a zero term.  cols must hold
 * n_params entries (SIM_ERANGE otherwise). */
SIM_API int sim_program_affine_layout(const sim_program *prog, uint64_t *x0, uint64_t *cols, uint32_t cap);

/* The whole hot path for one program: sum over all 2^p assignments on the GPU, times the
 * constant, in canonical form. */
SIM_API int sim_eval_amplitude(const sim_program *prog, void *stream, sim_zomega *out);

/* As sim_eval_amplitude, and *kernel_ms receives the duration of the evaluation kernel
 * alone, measured with HIP events recorded on `stream` right before and after its launch
 * (the finaliser and the result copy are outside the bracket). */
SIM_API int sim_eval_timed(const sim_program *prog, void *stream, sim_zomega *out, float *kernel_ms);

/* Raw partial sum over slices [first_slice, first_slice + n_slices) (flags = RAW): for
 * checkpoint/resume and sharding.  Partials over disjoint slices add exactly; finish with
 * sim_finalize.  "Raw" leaves out the packed program's constant: the IR's scalar times the
 * factors that the packer folds into it (factors on constant forms, factors whose two values
 * coincide, cancelling node pairs), so only finalised values compare with the IR's terms. */
SIM_API int sim_eval_range(const sim_program *prog, uint64_t first_slice, uint64_t n_slices,
                   void *stream, sim_zomega *raw);

/* Applies the program's constant and sqrt2 power to a raw sum and canonicalises it (on
 * the device). */
SIM_API int sim_finalize(const sim_program *prog, const sim_zomega *raw, void *stream, sim_zomega *out);

/* Many programs of uneven size in one launch per kernel variant (variants run concurrently):
 * work items of 2^chunk_log2 terms (default: at least 2^20), one workgroup each; programs of
 * 2^26 terms or more get a single-program launch of their own beside them.  Per-item partials
 * are summed per program in a fixed order, so each result is bit-identical to
 * sim_eval_amplitude.  t may be NULL. */
SIM_API int sim_eval_batch(const sim_program *const *progs, size_t n, void *stream,
                   const sim_tuning *t, sim_zomega *out);

/* Same as sim_eval_batch, but the launch sequence (evaluation kernels on forked streams,
 * finaliser, result copy) is captured once into a hipGraph held by the plan and replayed
 * by sim_batch_plan_run.  The plan keeps the programs' device images referenced; the
 * programs must outlive the plan. */
typedef struct sim_batch_plan sim_batch_plan;
SIM_API int sim_batch_plan_create(const sim_program *const *progs, size_t n, const sim_tuning *t,
                          void *stream, sim_batch_plan **out);
SIM_API int sim_batch_plan_run(sim_batch_plan *plan, void *stream, sim_zomega *out);
SIM_API void sim_batch_plan_free(sim_batch_plan *plan);

/* Continuous batching primitive: evaluates, in one launch, the next slice range of each
 * active request.  first_slice[i] and n_slices[i] select the range of progs[i]; the raw
 * partials are written to raw[i].  Used by the serving loop, which adds partials exactly
 * and finalises a request when its slices are done. */
SIM_API int sim_eval_ranges(const sim_program *const *progs, const uint64_t *first_slice,
                    const uint64_t *n_slices, size_t n, void *stream, const sim_tuning *t,
                    sim_zomega *raw);

/* One step of continuous batching (the serving loop's tick): for each request i, the raw sum
 * of slices [first_slice[i], first_slice[i] + n_slices[i]) of progs[i] plus carry[i] (the raw
 * sum of its earlier slices, flags RAW; carry NULL = all zero).  out[i] is that raw sum (flags
 * RAW) when last[i] is 0, else its finalised value (the constant, the sqrt2 power, canonical
 * form: what sim_finalize of the raw sum gives).  Work items of every request in one batch of
 * launches, the carried sums and the finalisation in the same finaliser launch, and one wait:
 * a request that ends in this step is answered by it.  Partial sums over disjoint slices add
 * exactly, so a request's final value does not depend on how its slices were split into steps
 * or which requests shared them. */
SIM_API int sim_serve_step(const sim_program *const *progs, const uint64_t *first_slice, const uint64_t *n_slices,
                           const sim_zomega *carry, const uint8_t *last, size_t n, void *stream,
                           const sim_tuning *t, sim_zomega *out);

/* The pipelined form of sim_serve_step: raw sums carried on the device and nothing waited for,
 * so a serving loop can enqueue its next step while the previous one runs.  dev_carry holds
 * n_carry_slots device accumulators of 72 bytes (caller-owned, 8-byte aligned); request i uses
 * slot slots[i] (distinct within a step).  flags[i] bit 0: its first step (the slot is not
 * read); bit 1: its last step.  Each request's partial sum over slices [first_slice[i],
 * first_slice[i] + n_slices[i]) plus its carried sum goes back to its slot as a raw sum, or, on
 * its last step, is finalised into dev_out[i] (caller-owned device memory, n x 72 bytes).  The
 * layout of a step goes through one of a few library staging buffers, reused once the step that
 * last used it has completed (the call waits on the host only then).  Steps on one stream run in
 * order, so a slot's sum is read by its next step after the previous one wrote it. */
SIM_API int sim_serve_enqueue(const sim_program *const *progs, const uint64_t *first_slice, const uint64_t *n_slices,
                              const uint32_t *slots, const uint8_t *flags, size_t n, void *dev_carry,
                              size_t n_carry_slots, void *stream, const sim_tuning *t, sim_zomega *dev_out);

/* Amplitudes of an OUTCOMES program (query kind SIM_QUERY_OUTCOMES) for n output strings:
 * bits holds n rows of n_outer bytes (0/1), row k = y_0 .. y_{n_outer-1}; out[k] =
 * <y|C|0^n> in canonical form, bit-identical to compiling and evaluating the AMPLITUDE query
 * for y.  The query parameters are the top bits of the slice index, so each string is one
 * contiguous slice range; all n ranges run as one batch (same kernels and launch shapes as
 * sim_eval_batch).  SIM_EINVAL if prog has no query parameters or a byte is not 0/1. */
SIM_API int sim_eval_outcomes(const sim_program *prog, size_t n, const uint8_t *bits, void *stream,
                              const sim_tuning *t, sim_zomega *out);

/* <y|C|0^n> (or the program's sum) like sim_eval_amplitude, but enqueued on stream without
 * waiting: the device writes the canonical value to dev_out (memory the caller owns and the
 * device can write, one sim_zomega, 8-byte aligned) when the stream gets there; flags bit
 * SIM_ZOMEGA_OVERFLOW marks an invalid value.  ev_before and ev_after, if not NULL, are
 * hipEvent_t created with timing that take the start and end time of the evaluation kernel
 * (not the finaliser) from its own dispatch, with no event packets of their own on the
 * stream.  Calls on one device share its scratch: an enqueued evaluation is ordered before
 * any later call on the device.  A later call on the same stream follows it in stream order; a
 * later call on another stream first waits on the host until the device is idle (so no event
 * is recorded per evaluation, and the stream may be destroyed after the call).  To capture
 * enqueued evaluations into a graph, make one call on the capture stream before the capture
 * begins, for the program needing the most scratch (the capture cannot allocate).  Scratch
 * buffers the library outgrows are kept until the process ends, so a captured graph stays
 * valid whatever is evaluated later.  For pipelines of many evaluations without a host round
 * trip between them. */
SIM_API int sim_enqueue_amplitude(const sim_program *prog, void *stream, void *ev_before, void *ev_after,
                                  sim_zomega *dev_out);

/* Repeated weak simulation (Appendix F's algorithm, with the conditional probabilities of
 * the product rule of Section 2.2).  progs[k-1] is the PREFIX program of the first k qubits
 * of one circuit, compiled with the outcomes as parameters (k = 1 .. K, K <= 62); the caller
 * guarantees they come from the same circuit.  uniforms holds n rows of K integers below
 * 2^53; sample i draws its bits in qubit order, bit k being 0 iff
 *     uniforms[i*K + k] / 2^53 < P(B || 0) / P(B),
 * B its bits 0 .. k-1 (P of the empty prefix = 1), decided exactly (no rounding).  Step k
 * evaluates P(B || 0) once per distinct prefix B among the samples, as one batch (the
 * kernels of sim_eval_outcomes).  Writes n rows of K bytes (0/1) to out_bits and, if
 * out_prob is not NULL, each sample's probability P(y_0 .. y_{K-1}) in canonical form.
 * Blocks until done.  SIM_EINVAL on bad arguments or if a program does not have k query
 * parameters or yields a non-real probability; other codes as sim_eval_outcomes. */
SIM_API int sim_sample(const sim_program *const *progs, size_t K, size_t n, const uint64_t *uniforms,
                       void *stream, const sim_tuning *t, uint8_t *out_bits, sim_zomega *out_prob);

/* Marginal by summing (Fig. 3 left): prog is an OUTCOMES program (k = n_outer query
 * parameters); pattern holds k bytes, 0 or 1 fixing y_i and 2 leaving it free.  out = the sum
 * of |<y|C|0^n>|^2 over the 2^m strings y that match (m = number of free outcomes, at most 32),
 * exactly, canonical.  The amplitudes are evaluated in batches of up to 2^16 strings (the
 * kernels of sim_eval_outcomes) and stay on the device, where their squares (in Z[sqrt2]:
 * |z|^2 = a + b sqrt2) are added to two 384-bit integer sums; only those come back.  Blocks
 * until done.  SIM_EINVAL on bad arguments, SIM_ERANGE if m > 32, an amplitude leaves the
 * 384-bit sums, or the exact sum exceeds int128 coefficients. */
SIM_API int sim_marginal_sum(const sim_program *prog, const uint8_t *pattern, void *stream,
                             const sim_tuning *t, sim_zomega *out);

/* ---- caller-owned scratch (the repeated-evaluation interface of Sections 3.3 and 4: many
 * evaluations of resident programs, the caller owning every device buffer).
 *
 * The calls below take device memory from the caller instead of the library's own scratch:
 * dev_scratch (256-byte aligned, e.g. a torch tensor's data_ptr()) of scratch_bytes bytes.
 * They never allocate or free device memory; a region that is too small gives SIM_ERANGE
 * (message: the bytes needed) and nothing is launched.  The caller must not use the region
 * for anything else while a call that uses it runs on the device.  Results are exactly those
 * of the library-scratch calls they mirror. */

/* Bytes of dev_scratch that sim_eval_amplitude_ws and sim_eval_range_ws need for any of the n
 * programs, and that sim_eval_batch_ws, sim_batch_prepare and sim_enqueue_batch need for the
 * whole set (the largest of these).  t may be NULL. */
SIM_API int sim_scratch_bytes(const sim_program *const *progs, size_t n, const sim_tuning *t, size_t *bytes);

/* sim_eval_amplitude with the partial sums in dev_scratch.  Blocks until *out is valid. */
SIM_API int sim_eval_amplitude_ws(const sim_program *prog, void *stream, void *dev_scratch, size_t scratch_bytes,
                                  sim_zomega *out);

/* Raw partial sum (flags = RAW) over the assignments of units [first, first + count), a unit
 * being 2^g consecutive assignments in slice order (sim_program_layout), with the program's
 * walk bits <= g <= p: g = walk bits is sim_eval_range; larger g splits the 2^p assignments
 * into 2^(p - g) equal shards (Section 3.3's independent terms, e.g. one per GPU).  Partials of
 * disjoint ranges add exactly (sim_raw_add); finish with sim_finalize.  SIM_EINVAL if g is out
 * of bounds or the range leaves the program.  Blocks until *raw is valid. */
SIM_API int sim_eval_range_ws(const sim_program *prog, uint64_t first, uint64_t count, uint32_t g, void *stream,
                              void *dev_scratch, size_t scratch_bytes, sim_zomega *raw);

/* sim_eval_batch with the work layout, partials and results in dev_scratch.  Blocks. */
SIM_API int sim_eval_batch_ws(const sim_program *const *progs, size_t n, void *stream, void *dev_scratch,
                              size_t scratch_bytes, const sim_tuning *t, sim_zomega *out);

/* Writes the work layout of a batch of n programs (as sim_eval_batch would run them, tuning t,
 * which may be NULL) into dev_scratch and waits for the copy; it also creates the library's
 * auxiliary streams if they do not exist yet.  After that, sim_enqueue_batch with the same
 * programs, tuning and dev_scratch may be called any number of times, including under stream
 * capture.  The library keeps a small host-side record of the prepared region (until it is
 * prepared again or sim_batch_forget); the programs must outlive it. */
SIM_API int sim_batch_prepare(const sim_program *const *progs, size_t n, const sim_tuning *t, void *dev_scratch,
                              size_t scratch_bytes, void *stream);

/* Enqueues the batch prepared in dev_scratch on stream without waiting: the device writes the
 * n canonical results to dev_out (caller-owned device memory, n sim_zomega, 8-byte aligned),
 * each bit-identical to sim_eval_amplitude.  No allocation, no host synchronisation and no
 * host memory read by the enqueued work, so a hipGraph capture of the call replays it.  The
 * kernel variants of the batch run on the library's auxiliary streams, forked from and joined
 * back into `stream` with events; while a capture holds such a call, no other call on the
 * device may run.  SIM_EINVAL if dev_scratch was not prepared for these programs and tuning. */
SIM_API int sim_enqueue_batch(const sim_program *const *progs, size_t n, void *stream, void *dev_scratch,
                              size_t scratch_bytes, const sim_tuning *t, sim_zomega *dev_out);

/* Drops the host-side record of a region prepared on the current device (no-op if none). */
SIM_API int sim_batch_forget(void *dev_scratch);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): sim_eval_ranges with the work layout, partials and results in a fixed array of
 * 4 MiB per device (a file-scope device array, its address taken once per device at set-up).
 * It calls no hipMalloc, hipFree or hipHostMalloc and creates no stream: every launch goes to
 * `stream`, and the layout and results move through pageable host copies.  The array keeps the
 * last call's contents; nothing in it has to start at zero.  Calls on one device share the
 * array: the device lock serialises them and each waits for its stream before returning, so
 * they take turns rather than overlap.  SIM_ERANGE (message: the bytes needed) when the batch
 * needs more than the array holds; other errors as sim_eval_ranges. */
SIM_API int sim_eval_ranges_static(const sim_program *const *progs, const uint64_t *first_slice,
                                   const uint64_t *n_slices, size_t n, void *stream, const sim_tuning *t,
                                   sim_zomega *raw);

/* sim_finalize for n programs in one launch: out[i] = finalised raws[i] of progs[i]. */
SIM_API int sim_finalize_batch(const sim_program *const *progs, const sim_zomega *raws, size_t n,
                               void *stream, sim_zomega *out);

/* Adds two raw partials of the same program exactly (host, int128 with overflow check). */
SIM_API int sim_raw_add(const sim_zomega *a, const sim_zomega *b, sim_zomega *out);

SIM_API void sim_program_free(sim_program *prog);

/* thread-local message of the last failing call on this thread ("" if none) */
SIM_API const char *sim_last_error(void);

/* number of compute units of the current device (0 if unknown) */
SIM_API int sim_device_cus(void);

#ifdef __cplusplus
}
#endif

#endif /* ZXPAR_H */
