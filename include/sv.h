/*
 * sv.h -- C-ABI of the MI355X (gfx950) state-vector simulator library libsv.so.
 *
 * The library applies quantum gates to a register of n qubits held as 2^n
 * complex amplitudes in GPU memory, and reduces that vector to measurement
 * probabilities and Z-string expectations.  It follows the problem statement
 * of "Simulating Quantum Computers Using OpenCL" (arXiv 1805.00988):
 *
 *   - a register of n qubits is a vector of 2^n complex amplitudes that starts
 *     in |0...0> (Sec. 2.1);
 *   - a gate is a 2x2 complex matrix [[A, B], [C, D]] applied to target qubit
 *     t, optionally controlled (Sec. 2.2, Sec. 2.3 and Alg. 1);
 *   - measurement needs the probability |psi_x|^2 of every outcome x (Sec. 2.4).
 *
 * Conventions used by every entry point:
 *   - qubit q is bit q of the amplitude index (qubit 0 least significant);
 *   - amplitudes are interleaved (re, im): float2 for SV_C64, double2 for
 *     SV_C128, amplitude x at byte offset x * sizeof(element);
 *   - a matrix U of a k-qubit gate is 2^k x 2^k, row-major, complex entries
 *     interleaved as (re, im) doubles, in HOST memory; bit j of its row/column
 *     index is the value of qubit targets[j];
 *   - a control mask selects the subspace where every masked bit is 1; the
 *     gate acts as the identity elsewhere (Sec. 2.3, controlled variant).
 *
 * Ownership: every host array argument belongs to the caller and is read
 * before the call returns.  Device buffers passed in (dev_buf, dev_out) belong
 * to the caller; the library frees only memory it allocated itself.
 *
 * Ordering: a handle is bound to one HIP stream.  Calls enqueue their kernels
 * on that stream and return without waiting, except calls that write a host
 * result (host_* arguments), which wait for it.  A handle must not be used by
 * two threads at once.
 *
 * Errors: every call validates its arguments on the host before enqueueing
 * anything.  On failure it returns a negative sv_status, leaves the state
 * unchanged and records a message readable with sv_last_error() (per thread).
 * Asynchronous device faults surface as SV_EDEVICE from the next call that
 * synchronises.  Unitarity of U is not checked; no call renormalises.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sv_state *sv_handle;

enum sv_dtype { SV_C64 = 1, SV_C128 = 2 };

enum sv_status {
    SV_OK = 0,
    SV_EINVAL = -1,       /* bad argument (qubit out of range, duplicate, NULL, ...) */
    SV_ENOMEM = -2,       /* the state (or a work buffer) does not fit in device memory */
    SV_EDEVICE = -3,      /* a HIP runtime call failed */
    SV_EUNSUPPORTED = -4  /* valid request the library does not implement */
};

/* Arithmetic of sv_apply_fused blocks.  Blocks run on the matrix cores
 * (MFMA) whenever the state is large enough to fill whole MFMA tiles (2^10
 * amplitudes for 5-qubit blocks), narrower blocks padded to 4 qubits; tiny
 * states use the vector ALUs in the same precision. */
enum sv_prec {
    SV_PREC_NATIVE = 0,     /* the state's own precision: FP32 products and sums
                               for complex64, FP64 for complex128 */
    SV_PREC_FP32 = 1,       /* FP32 matrix-core (MFMA) products, FP32 accumulate */
    SV_PREC_SPLIT_BF16 = 2  /* each FP32 operand split into bf16 hi + lo; three
                               bf16 MFMA products (hi*hi, hi*lo, lo*hi) with FP32
                               accumulate */
};

/* Named gates of an sv_op (see sv_op.kind). */
enum sv_gate_kind {
    SV_GATE_H = 1, SV_GATE_X = 2, SV_GATE_Y = 3, SV_GATE_Z = 4, SV_GATE_S = 5,
    SV_GATE_T = 6,
    SV_GATE_RX = 7, SV_GATE_RY = 8, SV_GATE_RZ = 9, /* exp(-i theta P / 2) */
    SV_GATE_U1 = 10,                                 /* diag(1, e^{i theta}) */
    SV_GATE_MATRIX = 11                              /* explicit 2x2 or 4x4 */
};

/* One gate of a circuit.  H..T follow the gate table of Sec. 1.3.2 (CNOT =
 * SV_GATE_X with one control); U1 is the phase gate of the QFT benchmark
 * (App. A).  n_targets is 1, or 2 for SV_GATE_MATRIX; matrix holds the
 * 2^k x 2^k entries for SV_GATE_MATRIX only.  param_index >= 0 replaces theta
 * by params[param_index] (parametrised gates RX RY RZ U1). */
typedef struct sv_op {
    int32_t kind;
    int32_t n_targets;
    int32_t targets[2];
    uint64_t ctrl_mask;
    int32_t param_index;
    int32_t reserved;
    double theta;
    double matrix[32];
} sv_op;

/* Bytes of an n-qubit state: 2^n * 8 (SV_C64, the paper's 64 bits per
 * amplitude, Sec. 2.1) or 2^n * 16 (SV_C128).  0 for invalid arguments. */
size_t sv_state_bytes(int n_qubits, int dtype);

/* Create a register of n_qubits (1..40) in |0...0> (Sec. 2.1).
 * dev_buf: NULL to let the library allocate the 2^n amplitudes, else a device
 * buffer of at least sv_state_bytes() bytes, 16-byte aligned, that the
 * caller keeps alive until sv_free (e.g. a torch tensor).  hip_stream: the
 * hipStream_t all work of this handle is ordered on (NULL = null stream).
 * SV_ENOMEM if the state would not fit in free device memory (checked before
 * any allocation). */
int sv_alloc(int n_qubits, int dtype, void *dev_buf, void *hip_stream, sv_handle *out);

/* Release the handle and whatever the library allocated for it. */
int sv_free(sv_handle h);

/* Set the state to the basis state |x> (x < 2^n). */
int sv_set_basis(sv_handle h, uint64_t x);

/* Rebind the handle to another HIP stream. */
int sv_set_stream(sv_handle h, void *hip_stream);

/* Wait for all work of the handle; SV_EDEVICE if a kernel failed. */
int sv_sync(sv_handle h);

/* Device pointer of the amplitudes. */
void *sv_data(sv_handle h);

/* Apply one k-qubit gate (k = 1 or 2) with optional controls: Alg. 1 of
 * Sec. 2.3 for k = 1 (every pair of amplitudes that differ only in bit
 * targets[0] is multiplied by U; with controls, only pairs whose control bits
 * are all 1), and its 4x4 analogue on the quadruples differing in bits
 * targets[0], targets[1] for k = 2.  Diagonal gates touch only the
 * amplitudes they change.  SV_EINVAL for k outside {1,2}, a target or
 * control >= n, duplicate targets, a control that is also a target, or NULL
 * pointers. */
int sv_apply_gate(sv_handle h, int k, const int *targets, uint64_t ctrl_mask, const double *U);

/* Apply a dense k-qubit block (1 <= k <= 5), typically the product of
 * several gates computed by sv_fuse: every group of 2^k amplitudes differing
 * only in the bits qubits[0..k-1] is multiplied by U (bit j <-> qubits[j]).
 * prec selects the arithmetic (enum sv_prec); SV_PREC_FP32 and
 * SV_PREC_SPLIT_BF16 require an SV_C64 state (SV_EUNSUPPORTED otherwise). */
int sv_apply_fused(sv_handle h, int k, const int *qubits, const double *U, int prec);

/* Sec. 2.4: write p_x = re^2 + im^2 for every x to dev_out (float[2^n] for
 * SV_C64, double[2^n] for SV_C128; device memory, may be NULL to skip the
 * write) and, if host_norm is not NULL, the FP64 sum of all p_x. */
int sv_probabilities(sv_handle h, void *dev_out, double *host_norm);

/* Sec. 1.3.3 (measurement in the computational basis: outcome x has
 * probability |psi_x|^2): the expectation of a diagonal observable,
 * <psi| sum_j coeffs[j] Z^{z_masks[j]} |psi> = sum_x |psi_x|^2 h(x) with
 * h(x) = sum_j coeffs[j] (-1)^popcount(x & z_masks[j]), accumulated in FP64;
 * Z^m is the product of Pauli Z on the qubits of mask m.  z_masks and coeffs
 * are n_terms host values (1 <= n_terms <= 64); *host_out (host) receives
 * the result and the call waits for it.  SV_EINVAL for NULL pointers, a
 * term count out of range or mask bits >= n. */
int sv_expectation(sv_handle h, int n_terms, const uint64_t *z_masks, const double *coeffs,
                   double *host_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): the
 * expectation of sv_expectation, computed by the same kernels, on a caller's
 * state without a handle, without any allocation and without waiting.
 * dev_amps: device pointer to the 2^n_qubits amplitudes (16-byte aligned,
 * layout as for every entry point); z_masks, coeffs: n_terms host values
 * (1 <= n_terms <= 64), read before the call returns; dev_out: device
 * pointer to one double that receives the FP64 result when the work on
 * hip_stream (NULL = null stream) reaches it.  The partial sums live in a
 * static device array of the library (64 KiB per device, held until the
 * process ends; any state size fits it, since the reduction uses at most
 * 8192 workgroups): calls that overlap on one device race, calls ordered on
 * one stream do not.  The device current at the call must be the one
 * holding dev_amps.  SV_EINVAL for NULL or misaligned pointers, n_qubits
 * outside [1, 40], an unknown dtype, n_terms outside [1, 64] or mask bits
 * >= n_qubits; SV_EDEVICE if the launch fails. */
int sv_expectation_noalloc(const void *dev_amps, int n_qubits, int dtype, int n_terms,
                           const uint64_t *z_masks, const double *coeffs, double *dev_out,
                           void *hip_stream);

/* Run a gate list on the state.  params (n_params doubles, may be NULL when
 * no op has param_index >= 0) supplies the angles of parametrised ops.
 * mode SV_RUN_PER_GATE launches one kernel per gate; SV_RUN_TILED lets the
 * scheduler group gates whose targets lie in one tile of qubits into single
 * passes through on-chip memory (a gate may move ahead of gates on other
 * qubits; each tile's qubits are chosen so that the pass and the next take
 * many gates), and stream the others.  The result is that of applying the
 * ops in order. */
enum sv_run_mode { SV_RUN_PER_GATE = 0, SV_RUN_TILED = 1 };
int sv_run(sv_handle h, const sv_op *ops, int n_ops, const double *params, int n_params,
           int mode);

/* The passes sv_run's tiled mode forms for a register of n_qubits of the
 * given dtype (host only: no state, no device call).  Gates apply in the
 * order of Sec. 2.3 (the ops in sequence); a pass may take a gate ahead of
 * gates left behind only when they share no qubit.  level 0 is the greedy
 * scheduler, 1 the lookahead, 2 the two-pass lookahead, -1 the level sv_run
 * uses for that state size.  gate_pass (n_ops ints, caller-owned) receives
 * the pass index of every op; pass_qubits (max_passes values) the qubit mask
 * of each pass's tile (bit q = qubit q), or 0 for a single gate sv_run
 * streams instead; *n_passes the pass count.  SV_EINVAL for n_qubits outside
 * [1, 40], an unknown dtype, level outside [-1, 2], NULL outputs, an invalid
 * op, or more passes than max_passes (then *n_passes still holds the
 * count). */
int sv_schedule(int n_qubits, int dtype, const sv_op *ops, int n_ops, const double *params, int n_params,
                int level, int max_passes, int *gate_pass, uint64_t *pass_qubits, int *n_passes);

/* Greedy fusion (host, FP64): walk ops in order, growing a block whose qubit
 * set (targets and controls) has at most k_max qubits; multiply each gate
 * into the block's 2^k x 2^k matrix; start a new block when a gate does not
 * fit.  Writes up to max_blocks blocks: block_k[b], block_qubits[b*5 ..]
 * (ascending, -1 padded), block_mats[b * 2*32*32 ..] (2^k x 2^k row-major
 * interleaved, leading dimension 2^k), block_gates[b] (gates absorbed).
 * *n_blocks receives the block count (SV_EINVAL if it exceeds max_blocks).
 * 1 <= k_max <= 5. */
int sv_fuse(int n_qubits, const sv_op *ops, int n_ops, const double *params, int n_params,
            int k_max, int max_blocks, int *block_k, int *block_qubits, double *block_mats,
            int *block_gates, int *n_blocks);

/* Apply the gate list through fused tile passes: the gates are first grouped
 * into passes whose qubits (targets and controls) fit one LDS tile, then the
 * gates of each pass are fused as by sv_fuse into blocks of at most k_max
 * qubits, and every block of a pass is applied, as by sv_apply_fused(prec),
 * during a single read and write of the state.  Per pass, a cost model
 * (fitted to MI355X kernel times) picks the cheapest of: blocks of at most
 * k_max qubits, blocks of at most 4 qubits (when k_max is 5), and the pass's
 * gates applied one by one as register sweeps in the state's own precision
 * (as sv_run does), so a pass never runs a fused form the model rates slower
 * than the plain one.  A diagonal gate of at most
 * four qubits may keep qubits outside the tile: they are fixed within one
 * tile, so the block holding the gate carries one matrix per value of its
 * outside qubits (at most 16) and each tile uses its own.  Only a gate's
 * qubits inside the tile count towards k_max in a block; every gate must
 * still touch at most k_max qubits (SV_EINVAL).  *n_blocks_out (may be
 * NULL) receives the number of blocks applied (passes run as plain sweeps
 * add none).  Same result as sv_run up
 * to rounding (FP32 or split-BF16 products for prec != SV_PREC_NATIVE). */
int sv_run_fused(sv_handle h, const sv_op *ops, int n_ops, const double *params, int n_params,
                 int k_max, int prec, int *n_blocks_out);

/* Autotuner of the fused path: runs the gate list once untimed and reps
 * times timed (HIP events on the handle's stream) for each candidate, each
 * run from the handle's present state, and reports the fastest: k = 0 for
 * plain tile passes (sv_run, SV_RUN_TILED), else sv_run_fused with k_max
 * = k in {4, 5} (k <= k_max, and no gate wider than k) and precision p with
 * bit p of prec_mask set (complex64: SV_PREC_FP32, SV_PREC_SPLIT_BF16;
 * complex128: SV_PREC_NATIVE).  *k_out, *prec_out receive the choice and
 * *ms_out (may be NULL) its time per run.  The state is left as it was on
 * entry; a temporary device copy of it is allocated for the duration
 * (SV_ENOMEM if it does not fit).  Plain passes are always a candidate, so
 * the choice is never slower than sv_run as measured. */
int sv_fused_tune(sv_handle h, const sv_op *ops, int n_ops, const double *params, int n_params,
                  int k_max, int prec_mask, int reps, int *k_out, int *prec_out, double *ms_out);

/* Sec. 1.3.3: outcome probabilities of measuring the k <= 6 qubits of mask
 * in the computational basis.  host_out[o] (2^k doubles, host) = sum of
 * |psi_x|^2 over the x whose mask bits spell o, where bit i of o is the
 * i-th lowest qubit of mask; FP64, fixed summation order.  The state is not
 * changed.  SV_EINVAL for an empty mask, bits >= n or more than 6 qubits. */
int sv_marginals(sv_handle h, uint64_t mask, double *host_out);

/* Sec. 1.3.3 post-measurement state: project onto the x with
 * (x & mask) == (value & mask) and divide by sqrt(p), p = the FP64
 * probability of that outcome, written to *host_prob (may be NULL).
 * SV_EINVAL (state unchanged) if p == 0 or mask has bits >= n. */
int sv_collapse(sv_handle h, uint64_t mask, uint64_t value, double *host_prob);

/* Measure the k <= 6 qubits of mask: the outcome is chosen from the
 * sv_marginals probabilities by the inverse cumulative distribution with the
 * caller's uniform u in [0, 1) (the first outcome, in outcome order, whose
 * cumulative probability exceeds u times the total), then the state
 * collapses onto it as by sv_collapse.  *host_value receives the outcome as
 * bits at the mask positions, *host_prob (may be NULL) its probability. */
int sv_measure(sv_handle h, uint64_t mask, double u, uint64_t *host_value, double *host_prob);

/* Sec. 2.4: n_samples full-register outcomes drawn from p_x = |psi_x|^2
 * without changing the state (repeated measurement of one prepared state).
 * Outcome s is the first x, in index order, whose FP64 cumulative
 * probability exceeds uniforms[s] times the total.  uniforms: n_samples host
 * doubles in [0, 1); host_out: n_samples host uint64.  0 <= n_samples <= 2^24.
 * The cumulative sums are formed per block of amplitudes, so an outcome can
 * differ from a strictly sequential sum only when the target falls within
 * rounding of a boundary between outcomes. */
int sv_sample(sv_handle h, int n_samples, const double *uniforms, uint64_t *host_out);

/* Adjoint-method gradient of L = <psi| H |psi>, H = sum_j coeffs[j] Z^{z_masks[j]},
 * psi = U_G ... U_1 psi_0 for the gate list ops with angles params.
 * On entry h must hold the circuit's output psi (as left by sv_run with the
 * same ops and params); lam is a second handle of the same size and dtype
 * used as work space.  The reverse sweep undoes one gate at a time on psi and
 * lam = H psi and accumulates dL/dtheta = 2 Re <lam| dU/dtheta |psi> for every
 * parametrised gate in FP64.  Writes L to *host_loss and the n_params
 * gradient entries to host_grad; on return h holds psi_0 as recovered by the
 * sweep.  Parametrised ops must be RX, RY, RZ or U1 (controls allowed). */
int sv_adjoint_grad(sv_handle h, sv_handle lam, const sv_op *ops, int n_ops,
                    const double *params, int n_params, int n_terms, const uint64_t *z_masks,
                    const double *coeffs, double *host_loss, double *host_grad);

/* Batches of independent circuits (one persistent launch).
 *
 * sv_batch_create compiles n_circuits circuits: circuit i acts on its own
 * register of widths[i] qubits (4..30 for SV_C64, 3..30 for SV_C128), starts
 * in |0...0> and runs ops[op_offsets[i] .. op_offsets[i+1]) (op_offsets has
 * n_circuits + 1 entries, op_offsets[0] = 0; params as in sv_run).  The
 * result of circuit i is <psi_i| Z^{z_mask} |psi_i> in FP64.  Circuits whose
 * state fits in one workgroup's LDS never touch HBM; wider ones keep their
 * state in device memory.  The whole batch is captured once as a HIP graph
 * holding one persistent kernel whose workgroups take circuits from a device
 * queue, longest first.  flags: SV_BATCH_KEEP_STATES also stores every final
 * state (for sv_batch_state).  All work is ordered on hip_stream.
 * sv_batch_run launches the graph (asynchronous); sv_batch_results waits and
 * copies the n_circuits results to host memory; sv_batch_output returns
 * their device address.  sv_batch_tune times the graph for every candidate
 * fusion width (0: the gates as given; 1 or 2: each circuit's gates
 * multiplied greedily, in circuit order, into blocks of at most 1 or 2
 * qubits, FP64 products rounded once to the state's precision), tile size
 * (LDS tile of 13, 12 or 11 qubits for complex64; 12, 11, 10 for
 * complex128), sweep width (3 or 4 register qubits, at most the narrowest
 * circuit's width) and grid (1 or 2 workgroups per CU), reps launches
 * each, and keeps the fastest; the chosen values and their time per launch
 * are written to the non-NULL outputs. */
enum sv_batch_flags { SV_BATCH_KEEP_STATES = 1 };
typedef struct sv_batch *sv_batch_handle;
int sv_batch_create(int n_circuits, const int *widths, const int64_t *op_offsets, const sv_op *ops,
                    const double *params, int n_params, int dtype, uint64_t z_mask, int flags,
                    void *hip_stream, sv_batch_handle *out);
int sv_batch_run(sv_batch_handle b);
int sv_batch_results(sv_batch_handle b, double *host_out);
void *sv_batch_output(sv_batch_handle b);
int sv_batch_state(sv_batch_handle b, int i, void *host_out);
int sv_batch_tune(sv_batch_handle b, int reps, int *tile_m, int *sweep_w, int *grid, int *fuse_w,
                  double *best_ms);
/* Rebuild the batch's program and graph for one configuration of the
 * tuner's space (tile_m in the tuner's three tile sizes, sweep_w 3 or 4 and
 * at most the narrowest circuit, grid workgroups, fuse_w 0, 1 or 2);
 * SV_EINVAL outside it. */
int sv_batch_config(sv_batch_handle b, int tile_m, int sweep_w, int grid, int fuse_w);
int sv_batch_free(sv_batch_handle b);

/* Per-launch timing of a handle's kernels, for measurement: with timing on,
 * every kernel launch of the handle is bracketed by two HIP events recorded
 * on the handle's stream.  sv_timing(h, 1) starts (and clears) a record,
 * sv_timing(h, 0) stops recording; both wait for the stream first.
 * sv_timing_read waits for the stream and writes one entry per kernel kind
 * that ran since the record was cleared: launches, summed event time and the
 * summed algorithmic HBM bytes of those launches (every amplitude a launch
 * must read and write once: 2 * bytes-per-amplitude * amplitudes touched for
 * a gate or tile pass) and their algorithmic floating-point operations (per
 * updated amplitude: 14 for a general 2x2 complex matvec, 6 for a real 2x2
 * or a diagonal, 3 on average for a phase gate, 0 for a swap, 30 for a 4x4,
 * 8 * 2^k for a k-qubit dense block).  *n_out receives the number of kinds;
 * SV_EINVAL if it exceeds cap.  Reading clears the record. */
typedef struct sv_kernel_stat {
    char name[24];
    int64_t launches;
    double total_ms;
    double bytes;  /* algorithmic HBM bytes of all launches */
    double flops;  /* algorithmic floating-point operations of all launches */
} sv_kernel_stat;
int sv_timing(sv_handle h, int enable);
int sv_timing_read(sv_handle h, sv_kernel_stat *out, int cap, int *n_out);

/* Message of the last failed call on this thread ("" if none). */
const char *sv_last_error(void);

/* Library version string. */
const char *sv_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SV_H */
