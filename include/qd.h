/*
 * qd.h - C ABI of libqd, an MI355X (gfx950) engine that applies generalized qudit gates to a dense
 * complex state vector over a mixed-radix register.
 *
 * Method: QuDiet (arXiv 2211.07918). The paper simulates a circuit by forming, per Moment, the
 * Kronecker product of the gates acting on every wire, multiplying those operators and applying
 * the product to the initial state (Sec. 3.5-3.6). libqd computes the same result gate by gate:
 * applying the Kronecker-embedded operator I (x) U (x) I of one gate to the state costs O(D d_T)
 * instead of O(D^2).
 *
 * Conventions (apply to every call):
 *   - A register is a list of qudit dimensions dims[0..n-1]; its state has D = prod dims[i]
 *     amplitudes (Sec. 2.2). The flat index is big-endian mixed radix: qudit 0 is the most
 *     significant digit, stride s_i = prod_{j>i} dims[j] (the Kronecker order of Sec. 3.3, Eq. (3),
 *     and the ket labels of the Sec. 3.9 example).
 *   - Amplitudes are interleaved (re, im): complex128 = 2 doubles, complex64 = 2 floats.
 *   - A gate acts on distinct targets t_0..t_{k-1}; its unitary U is d_T x d_T with
 *     d_T = prod dims[t_j], row-major, each entry (re, im) as two doubles (so 2*d_T*d_T doubles).
 *     Row/column index of U: t_0 is the most significant digit (the block layout of the
 *     generalized CNOT, Sec. 2.1).
 *   - Controls c_0..c_{m-1} with values v_j: the gate acts only on basis states whose digit at
 *     c_j equals v_j, and is the identity elsewhere (Sec. 2.1 generalized CNOT and multi-controlled
 *     Toffoli, which fire on d-1; here the value is explicit, 0 <= v_j < dims[c_j]).
 *
 * Ownership: every input array is copied before the call returns; the caller may free it at once.
 * Output buffers are allocated by the caller. Handles are released with the matching *_free.
 *
 * Errors: every entry point returns a status (QD_OK = 0 or a negative QD_E* code) and never
 * throws across the ABI. Arguments are validated before any device work, so a call that fails
 * validation leaves the state bit-identical. qd_last_error() returns a message for the calling
 * thread. Gate calls are asynchronous on the state's HIP stream; calls that return data to the host
 * (download, probabilities to host, norm, compare) synchronise that stream and report a deferred
 * device fault as QD_EDEVICE.
 */
#ifndef QD_H
#define QD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qd_state qd_state;
typedef struct qd_fused qd_fused;
typedef struct qd_batch qd_batch;

enum {
  QD_OK = 0,
  QD_EINVAL = -1,       /* malformed argument: null pointer, bad index, bad count           */
  QD_EDIM = -2,         /* dimension mismatch: U size != d_T, radix out of range, size mismatch */
  QD_ENOTUNITARY = -3,  /* max |U^dag U - I| > 1e-10, or a NaN/Inf entry                      */
  QD_ENOMEM = -4,       /* device or pinned allocation failed                                */
  QD_EOVERFLOW = -5,    /* D or its byte size overflows int64 / the device capacity           */
  QD_EDEVICE = -6       /* a HIP call failed, or a deferred device fault was observed         */
};

enum { QD_C128 = 0, QD_C64 = 1 };                                   /* state precision */
enum { QD_MODE_FP64_PLAIN = 0, QD_MODE_FP32_MFMA = 1, QD_MODE_BF16X3_MFMA = 2 };
enum { QD_FUSED_RENORMALIZE = 0x100 };   /* qd_apply_fused flag, OR'd into the mode */
enum { QD_FLAG_SKIP_UNITARY_CHECK = 1 };
enum { QD_GATE_X = 0, QD_GATE_Z = 1, QD_GATE_F = 2, QD_GATE_I = 3 };   /* named gates, Sec. 2.1 */
enum { QD_CLASS_DENSE = 0, QD_CLASS_MONOMIAL = 1, QD_CLASS_DIAGONAL = 2 };
enum { QD_ROUTE_DIRECT = 0, QD_ROUTE_TILED = 1, QD_ROUTE_DIAG = 2, QD_ROUTE_GENERIC = 3, QD_ROUTE_GEMM = 4 };

#define QD_MAX_QUDITS 64    /* n <= 64 */
#define QD_MAX_RADIX 256    /* 2 <= dims[i] <= 256 */
#define QD_MAX_GATE_DIM 1024 /* d_T <= 1024: the 4^5 x 4^5 five-ququart gate of Sec. 1 */
#define QD_MAX_FUSED_DIM 128 /* largest fused block qd_fuse builds */

/* One gate as data, for qd_fuse and the batched path. Pointers are read during the call only. */
typedef struct {
  int32_t k;                       /* number of targets, >= 1                                  */
  const int32_t* targets;          /* k distinct qudit indices                                 */
  int32_t m;                       /* number of controls, >= 0                                 */
  const int32_t* controls;         /* m qudit indices, disjoint from targets                   */
  const int32_t* control_values;   /* m values, 0 <= v_j < dims[c_j]                           */
  const double* U;                 /* d_T x d_T complex, row-major, interleaved (re, im) FP64  */
} qd_gate;

/* ---------------------------------------------------------------- library, register, gates */

/* Library version string (static storage). */
const char* qd_version(void);

/* Message for the last failed call on this thread (thread-local storage, valid until the next
 * failing call on the same thread). */
const char* qd_last_error(void);

/* Name of the kernel instance that the calling thread's last qd_apply_gate / qd_apply_gate_ex
 * launched, e.g. "k_slices_direct<double, 2, DenseOp<double, 2>, 1, plain>" (template arguments:
 * precision, slice size d_T after any control folded into the targets, gate operation, slices per
 * thread and the control mode plain / pred / edge), or that the last block of its last
 * qd_apply_fused launched (e.g. "k_fused_pipe<3, 6, 41, 1, true, 13312>", the template arguments
 * as rocprofv3 prints them); "" when that call launched nothing. Static thread-local storage, for
 * profiling labels; it changes no state. */
const char* qd_last_kernel(void);

/* Gate kernel launches made on a state since it was created: one per qd_apply_gate that moved
 * data, and one per pass of the density-matrix calls (a composed run of operations is one pass).
 * Host counter, no synchronisation. QD_EINVAL for a null argument. */
int qd_state_gate_launches(const qd_state* s, int64_t* out);

/* Register table (Sec. 2.2: the state has prod dims[i] entries). Host only, no device work.
 * Writes D to *D_out and the n big-endian strides to strides_out[n] (caller-allocated).
 * QD_EINVAL for n outside 1..64 or null pointers, QD_EDIM for a radix outside 2..256,
 * QD_EOVERFLOW if D overflows int64. */
int qd_register_strides(const int32_t* dims, int32_t n, int64_t* D_out, int64_t* strides_out);

/* Unitary of a named gate of Sec. 2.1 on a wire of dimension d, written to U_out
 * (2*d*d doubles, row-major, interleaved). Host only.
 *   QD_GATE_X: generalized NOT X^d_{+a}, |x> -> |(x+a) mod d>, requires 1 <= a <= d-1;
 *   QD_GATE_Z: phase-shift diag(1, w, ..., w^{d-1}), w = exp(2 pi i / d);
 *   QD_GATE_F: generalized Hadamard (1/sqrt d) [w^{jk}];
 *   QD_GATE_I: identity.
 * w^m is evaluated with m reduced mod d; quarter turns are exact. QD_EINVAL for an unknown kind
 * or a shift outside 1..d-1, QD_EDIM for d outside 2..256. */
int qd_gate_matrix(int32_t kind, int32_t d, int32_t a, double* U_out);

/* Validate one gate against a register without touching the device (the checks qd_apply_gate
 * runs first). flags: QD_FLAG_SKIP_UNITARY_CHECK skips the unitarity test. Returns QD_OK or the
 * code qd_apply_gate would return. */
int qd_validate_gate(const int32_t* dims, int32_t n, const int32_t* targets, int32_t k,
                     const int32_t* controls, const int32_t* control_values, int32_t m,
                     const double* U, uint32_t flags);

/* Structural class of a d_T x d_T unitary as the kernels see it (exact zero tests in FP64):
 * QD_CLASS_DIAGONAL (only diagonal entries non-zero), QD_CLASS_MONOMIAL (one non-zero per row and
 * column, e.g. X_{+a} and the qudit swap), else QD_CLASS_DENSE. Host only; -1 on bad arguments. */
int qd_gate_class(const double* U, int32_t dT);

/* Kernel family qd_apply_gate would launch for this gate on a state of register dims and
 * precision prec, written to *route_out (host only, no device work):
 *   QD_ROUTE_DIRECT  one slice per thread (every target stride >= the run threshold, or every
 *                    target stride >= one 128-byte line with controls inside a line that leave
 *                    lines without a matching amplitude: those lines are skipped);
 *   QD_ROUTE_TILED   slices staged in LDS (a target with a small stride);
 *   QD_ROUTE_DIAG    elementwise phases (diagonal U);
 *   QD_ROUTE_GEMM    dense 10 <= d_T <= 64 (and other monomials in that range): per tile of
 *                    slices a small complex GEMM, U and the tile in LDS;
 *   QD_ROUTE_GENERIC any d_T up to 1024 or D >= 2^32 (U in device memory).
 * Validation as in qd_apply_gate. */
int qd_gate_route(const int32_t* dims, int32_t n, int32_t prec, const int32_t* targets, int32_t k,
                  const int32_t* controls, const int32_t* control_values, int32_t m, const double* U,
                  int32_t* route_out);

/* ---------------------------------------------------------------- state vectors (Sec. 3.3) */

/* Allocate a state of the register dims[0..n-1] in device memory owned by the library and set it
 * to |0...0> (Sec. 2.2: circuits start in the computational basis state |0>; Sec. 3.2 default
 * init_states). prec is QD_C128 or QD_C64. hip_stream is the hipStream_t every call on this state
 * is ordered on (NULL = the null stream). *out receives the handle.
 * QD_ENOMEM if the device allocation fails, QD_EOVERFLOW if D * bytes-per-amplitude overflows. */
int qd_state_init(const int32_t* dims, int32_t n, int32_t prec, void* hip_stream, qd_state** out);

/* As qd_state_init, but over caller-owned device memory dev_ptr of `bytes` bytes (for instance a
 * PyTorch tensor), which must hold D amplitudes. The contents are left untouched; the library
 * never frees this memory. QD_EDIM if bytes < D * bytes-per-amplitude. */
int qd_state_wrap(const int32_t* dims, int32_t n, int32_t prec, void* dev_ptr, int64_t bytes,
                  void* hip_stream, qd_state** out);

/* Set the state to the basis state |values[0] ... values[n-1]> (Sec. 3.2 init_states: the
 * Kronecker product of one basis vector per wire, Sec. 3.3 Eq. (3)). QD_EINVAL if a value is
 * outside 0..dims[i]-1. Asynchronous. */
int qd_state_set_basis(qd_state* s, const int32_t* values);

/* Copy n = D amplitudes from host memory (interleaved, in the state's precision) into the state,
 * or out of it into host memory. QD_EDIM if n != D. Both synchronise the stream. */
int qd_state_upload(qd_state* s, const void* host_amps, int64_t n);
int qd_state_download(const qd_state* s, void* host_amps, int64_t n);

/* Queries: register size D, the register (dims_out needs room for 64 ints; *n_out receives n),
 * precision, device pointer of the amplitudes. */
int qd_state_size(const qd_state* s, int64_t* D_out);
int qd_state_dims(const qd_state* s, int32_t* dims_out, int32_t* n_out);
int qd_state_precision(const qd_state* s, int32_t* prec_out);
int qd_state_device_ptr(const qd_state* s, void** ptr_out);

/* Wait for all work queued on the state's stream; QD_EDEVICE reports a deferred fault. */
int qd_state_sync(const qd_state* s);

void qd_state_free(qd_state* s);

/* ---------------------------------------------------------------- gate application (Sec. 2.1) */

/* Apply one generalized gate in place: for every basis state whose control digits match,
 * the amplitudes over the target digits are mixed by U (U acts as I (x) U (x) I on the register,
 * the Kronecker-embedded Moment operator of Sec. 3.5). Covers X_{+a}, Z_d, F_d, the generalized
 * CNOT / multi-controlled Toffoli (targets {t}, controls with values) and any user unitary
 * (Sec. 3.4 "User Defined Gate"). Validation (before any device work): 1 <= k, k + m <= n,
 * targets distinct and in range, controls in range, distinct and disjoint from the targets,
 * 0 <= v_j < dims[c_j], d_T <= 1024, U unitary within 1e-10 (max-abs of U^dag U - I) with no
 * NaN/Inf. Codes: QD_EINVAL, QD_EDIM, QD_ENOTUNITARY. A complex64 state receives U rounded to
 * FP32. Asynchronous on the state's stream. */
int qd_apply_gate(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls,
                  const int32_t* control_values, int32_t m, const double* U);

/* qd_apply_gate with flags (QD_FLAG_SKIP_UNITARY_CHECK skips the unitarity test only). */
int qd_apply_gate_ex(qd_state* s, const int32_t* targets, int32_t k, const int32_t* controls,
                     const int32_t* control_values, int32_t m, const double* U, uint32_t flags);

/* ---------------------------------------------------------------- gate fusion (Sec. 3.6) */

/* Fusion plan, host only: the paper multiplies the Moment operators of a whole circuit into one
 * operator (Sec. 3.6); here the products are bounded to blocks whose window W (the union of the
 * members' targets and controls) keeps prod_{w in W} dims[w] <= max_block_dim
 * (2 <= max_block_dim <= 128). A block starts at the first gate not yet placed; a later gate joins
 * it if the window stays within the bound and the gate touches no qudit of a gate skipped so far
 * (so it commutes with every gate it moves ahead of); members keep their circuit order.
 * block_of_gate[g] receives the block index of gate g (caller-allocated, g entries; blocks run in
 * index order); *nblocks the number of blocks. A gate whose own qudits exceed max_block_dim is
 * QD_EDIM. */
int qd_fuse_plan(const int32_t* dims, int32_t n, const qd_gate* gates, int32_t g,
                 int32_t max_block_dim, int32_t* block_of_gate, int32_t* nblocks);

/* Plan (as qd_fuse_plan) and build every block on the GPU in FP64: block = E_last ... E_first
 * over the block's members, E_i the gate embedded in the block's window (window qudits in
 * ascending order, the first most significant). Also emits the FP32 and split-BF16 (hi, lo) copies used by qd_apply_fused.
 * Gates are validated as in qd_apply_gate. Asynchronous on hip_stream. */
int qd_fuse(const int32_t* dims, int32_t n, const qd_gate* gates, int32_t g, int32_t max_block_dim,
            void* hip_stream, qd_fused** out);
/* max_block_dim = 0 lets qd_fuse choose the fusion width: each candidate in {16, 27, 32, 36, 48,
 * 64, 81, 96, 128} is planned and costed as sum over blocks of max(8 B D / F, 16 D / H) with F
 * and H the matrix-core and HBM rates of the complex64 block kernel (defaults 40 TFLOP/s and
 * 5 TB/s); the cheapest plan is built. */

/* Number of blocks, and per block: window size k, window qudits (caller array of >= 64 ints,
 * ascending), block dimension B, first member gate and member count; qd_fused_block_gates writes
 * the member gate indices (ngates ints, ascending). */
int qd_fused_count(const qd_fused* f, int32_t* nblocks);
int qd_fused_block_info(const qd_fused* f, int32_t b, int32_t* k, int32_t* window, int32_t* B,
                        int32_t* first_gate, int32_t* ngates);
int qd_fused_block_gates(const qd_fused* f, int32_t b, int32_t* gates_out);

/* Copy block b (B x B complex FP64, row-major, interleaved) to host memory; synchronises. */
int qd_fused_download_block(const qd_fused* f, int32_t b, double* out);

/* Apply all fused blocks in order to a state whose register matches the fused circuit.
 *   QD_MODE_FP64_PLAIN: complex128 state, FP64 blocks, FP64 arithmetic;
 *   QD_MODE_FP32_MFMA: complex64 state, FP32 blocks on FP32 matrix cores, FP32 accumulation;
 *   QD_MODE_BF16X3_MFMA: complex64 state, split-BF16 products a_hi b_hi + a_hi b_lo + a_lo b_hi
 *   on BF16 matrix cores with FP32 accumulation.
 * mode may carry QD_FUSED_RENORMALIZE: after the last block the state is brought back to
 * sum |alpha|^2 = 1 (Eq. (1)) on the GPU, an FP64 reduction of ||psi||^2 (the tree of qd_norm2)
 * followed by a scaling by 1/sqrt(||psi||^2) computed in FP64 on the device, with no host wait (a
 * norm of zero or not finite leaves the state as it is). The unit norm of every circuit's state is
 * exact in exact arithmetic, so this removes only the drift that rounding of the blocks (held to
 * BF16 pairs in QD_MODE_BF16X3_MFMA) accumulates.
 * QD_EDIM if the register or precision does not match the mode, QD_EINVAL for another flag.
 * Asynchronous. */
int qd_apply_fused(qd_state* s, const qd_fused* f, int32_t mode);

void qd_fused_free(qd_fused* f);

/* ---------------------------------------------------------------- readout (Sec. 3.8) */

/* Probability of every basis state, |alpha_x|^2 computed in FP64 (Sec. 3.8 OutputMethod
 * probability; Eq. (1) normalisation). out holds D doubles; out_is_device != 0 means out is a
 * device pointer (asynchronous), else host memory (synchronises). */
int qd_probabilities(const qd_state* s, double* out, int32_t out_is_device);

/* ||psi||^2 in FP64 by a deterministic two-pass tree reduction (same result on every run).
 * Synchronises. */
int qd_norm2(const qd_state* s, double* out);

/* Both readouts of Sec. 3.8 / Eq. (1) from one pass over the state: the probabilities, as
 * qd_probabilities writes them (out: D doubles, a device pointer when out_is_device != 0, else
 * host memory), and ||psi||^2 into *norm2 (host), bitwise equal to what qd_norm2 returns (the same
 * grid, visiting order and reduction tree). QD_EINVAL for a null argument. Synchronises. */
int qd_probabilities_norm2(const qd_state* s, double* out, int32_t out_is_device, double* norm2);

/* qd_norm2 for callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the same kernels and the same fixed reduction tree, so
 * the result is bitwise equal to qd_norm2's, written as one FP64 value to out_dev, a device
 * pointer the caller owns. Asynchronous on the state's stream (no synchronisation, no host copy).
 * The reduction partials live in a static 16 KiB device array per GPU (at most 2048 partials,
 * which covers every register size; a larger grid would return QD_EINVAL) instead of a buffer the
 * library allocates; the array's device address is looked up once per GPU on the first call.
 * The call makes no hipMalloc, hipFree or other allocating call. Calls on one GPU share the array:
 * calls that can overlap in time (on different streams of the same GPU, or from several threads
 * without ordering) race and must be serialised by the caller. Every workgroup rewrites its own
 * partial, so no state carries over from one call to the next.
 * Errors: QD_EINVAL for a null argument, QD_EDEVICE if the array's address cannot be found or
 * the state's device id is 64 or above, or a launch error. */
int qd_norm2_noalloc(const qd_state* s, double* out_dev);

/* Precision diagnostics in FP64 against a complex128 reference state of the same register:
 * max_x |psi_x - ref_x|, fidelity loss 1 - |<ref|psi>|^2 (psi unnormalised) and norm drift
 * | ||psi||^2 - 1 |. s may be complex64 or complex128. Any output pointer may be NULL.
 * QD_EDIM if the registers differ or ref is not complex128. Synchronises. */
int qd_compare(const qd_state* ref64, const qd_state* s, double* max_abs, double* fid_loss,
               double* norm_drift);

/* qd_compare plus the normalised variant, written to out[0..4]:
 *   out[0] max_x |psi_x - ref_x|, out[1] 1 - |<ref|psi>|^2, out[2] | ||psi||^2 - 1 |,
 *   out[3] ||psi||^2, out[4] 1 - |<ref|psi>|^2 / ||psi||^2 (direction error only).
 * Same requirements and errors as qd_compare. Synchronises. */
int qd_compare_ex(const qd_state* ref64, const qd_state* s, double* out5);

/* Restore the normalisation of Eq. (1) (sum |alpha|^2 = 1): ||psi||^2 by the FP64 reduction of
 * qd_norm2, then every amplitude scaled by 1/sqrt(||psi||^2) in the state's precision.
 * *norm2_before (may be NULL) receives the squared norm before scaling. QD_EINVAL if the norm is
 * zero or not finite (the state is left untouched). Synchronises. */
int qd_normalize(qd_state* s, double* norm2_before);

/* ---------------------------------------------------------------- measurement (Sec. 2.2, 3.1, 3.8) */

/* Shots of a computational-basis measurement of every qudit (measure_all, Sec. 3.1; each qudit
 * returns an integer digit, Sec. 2.2): out[j] is the basis index drawn by the 64-bit random word
 * rand[j]. Outcome x has weight w_x = round(p_x 2^62), p_x = re*re + im*im in FP64 (products
 * rounded before the sum); with W = sum w_x, t = floor(rand[j] W / 2^64) and out[j] is the first x
 * whose cumulative weight exceeds t. The weights are exact integers, so a random word always
 * gives the same index, whatever the summation order. The caller supplies the random words (any
 * uniform 64-bit generator). on_device != 0: rand and out are device pointers, else host memory.
 * QD_EINVAL if the squared norm reaches 3.999 or some |alpha|^2 is not finite (weights would not
 * fit in 64 bits), or if the state is zero. Synchronises. */
int qd_sample(qd_state* s, const uint64_t* rand, int64_t shots, int64_t* out, int32_t on_device);

/* Per-qudit outcome distributions: out[o_q + v] = sum of p_x over the basis states whose digit q
 * is v, o_q = d_0 + ... + d_{q-1} (host array of d_0 + ... + d_{n-1} doubles). FP64, p as in
 * qd_sample, summed in a fixed order (repeated calls return identical values). Synchronises. */
int qd_marginals(qd_state* s, double* out);

/* The basis states that carry probability (run() output, Sec. 3.6 and Sec. 3.8): every x with
 * p_x > eps (eps >= 0; 0 lists the states of non-zero probability), in ascending order. *count
 * receives how many there are; the first min(count, max_out) are written to the host arrays that
 * are not NULL: idx (basis index), amps (amplitude in the state's precision, interleaved re, im)
 * and probs (p_x in FP64). Synchronises. */
int qd_support(qd_state* s, double eps, int64_t max_out, int64_t* idx, void* amps, double* probs,
               int64_t* count);

/* Ket label of basis index x (Sec. 3.8 OutputType print; Sec. 3.9 prints |120> for q0 = 1, q1 = 2,
 * q2 = 0): digits of qudit 0 first, side by side when every radix is at most 10, else separated by
 * commas; written NUL-terminated to buf. QD_EINVAL if x is outside the register or buf is too
 * small. Host only. */
int qd_ket_string(const int32_t* dims, int32_t n, int64_t index, char* buf, int32_t buflen);

/* ---------------------------------------------------------------- circuit front-end (Sec. 3.4, 3.5, 4) */

/* A circuit: a register and an ordered list of named gates (QD_GATE_X with shift a, QD_GATE_Z,
 * QD_GATE_F) on one target, each with zero or more controls and their values. Host only. */
typedef struct qd_circuit qd_circuit;

/* Empty circuit on dims[0..n-1]; its qudits are named q0, q1, ... QD_EINVAL / QD_EDIM as for a
 * register. */
int qd_circuit_create(const int32_t* dims, int32_t n, qd_circuit** out);

/* Append a gate. QD_EINVAL for an unknown kind, a target or control outside the register, a repeated
 * qudit, a control value outside 0..d-1 or an X shift outside 1..d-1 (the circuit is unchanged). */
int qd_circuit_add(qd_circuit* c, int32_t kind, int32_t target, int32_t a, const int32_t* controls,
                   const int32_t* control_values, int32_t m);

/* Parse a QuDiet QASM program (Sec. 4): ".qudit n", one "qudit NAME (d)" line per qudit, then the
 * gates between ".begin" and ".end": "X q [a]" (shift a, default 1), "H q", "Z q", "CX c t [a]"
 * and the extension "MCT c1 .. ck t [a]"; every control fires on d_c - 1 (Sec. 2.1). Names are
 * case-insensitive, '#' starts a comment. QD_EINVAL with the line number in qd_last_error() for
 * any malformed line, an unknown qudit or gate, a shift outside 1..d-1, a repeated qudit in one
 * gate, a count that differs from ".qudit", or a missing ".begin"/".end". */
int qd_qasm_parse(const char* text, qd_circuit** out);

/* Number of qudits and gates; either pointer may be NULL. */
int qd_circuit_size(const qd_circuit* c, int32_t* n_qudits, int64_t* n_gates);

/* The register (n values) and the name of qudit q (NUL-terminated, lowercase). */
int qd_circuit_dims(const qd_circuit* c, int32_t* dims_out);
int qd_circuit_name(const qd_circuit* c, int32_t q, char* buf, int32_t buflen);

/* Gate i: kind, target, shift (0 unless X), number of controls m, and the m controls and values
 * (arrays of at least m entries, or NULL). */
int qd_circuit_gate(const qd_circuit* c, int64_t i, int32_t* kind, int32_t* target, int32_t* a, int32_t* m,
                    int32_t* controls, int32_t* control_values);

/* Moment of every gate (Sec. 3.5): a gate moves back through the preceding Moments while all of
 * its qudits (target and controls) hold identities there, so its Moment is one past the latest
 * Moment of the earlier gates sharing a qudit (0-based). moment_out holds one int32 per gate (or
 * NULL); *depth (or NULL) receives the number of Moments. Gates of one Moment touch disjoint
 * qudits and commute. */
int qd_circuit_moments(const qd_circuit* c, int32_t* moment_out, int32_t* depth);

/* New circuit with every X of two or more controls replaced by generalized CNOTs (Sec. 3.4): for
 * controls c_1..c_k with values v_1..v_k, c_{i-1} at its marker raises c_i by 1 (i = 2..k; the
 * marker of c_1 is v_1, of c_i is v_i + 1), c_k at its marker shifts the target, then the chain is
 * undone in reverse with shifts d_{c_i} - 1. Exact on every basis state whose chained controls
 * c_2..c_k are not already at their markers (the intermediate level is free). QD_EDIM if some
 * chained control has no level v_i + 1. Other gates are copied. */
int qd_circuit_decompose(const qd_circuit* c, qd_circuit** out);

/* Apply the circuit's gates in order to a state of the same register (qd_apply_gate for each).
 * QD_EDIM if the registers differ. Asynchronous, like qd_apply_gate. */
int qd_circuit_apply(qd_state* s, const qd_circuit* c);

void qd_circuit_free(qd_circuit* c);

/* ---------------------------------------------------------------- sparse state (Sec. 3.3, 3.7) */

/* A state kept as the list of its non-zero amplitudes (complex128) with their flat indices (int64),
 * the compressed sparse column of Sec. 3.3 and the sparse backends of Sec. 3.7, updated gate by
 * gate on the GPU. The register may be far larger than any dense state (D up to 2^63 - 1); the
 * list holds at most 2^31 - 1 entries.
 *
 * Rules:
 *  - an index is present exactly when its amplitude is not exactly zero: a dense-gate output whose
 *    real and imaginary parts are both 0.0 is dropped (sparse products store no exact zeros);
 *    entries moved by a monomial gate are kept;
 *  - a monomial gate (exactly one non-zero entry in every row and column of U: X_{+a}, generalized
 *    CNOTs, Z_d, controlled phases, qudit swaps) moves each matching entry where it stands: column
 *    loc goes to the row r of its entry and the amplitude is multiplied by U[r, loc] unless that
 *    entry is exactly 1. It never changes the count and never waits on the host;
 *  - any other gate is dense: the matching entries that share every non-target digit form a slice,
 *    and the slice's d_T outputs are U times its d_T inputs (absent inputs are zero). A product
 *    u x is (ur xr - ui xi, ur xi + ui xr) and an output sums j = 0..d_T-1 in order from +0.0, each
 *    real operation rounded on its own, so results are bitwise reproducible;
 *  - list order: a monomial gate keeps every position; a dense gate keeps the non-matching entries
 *    in order and writes each slice's non-zero outputs, by increasing local row, where the slice's
 *    first entry stood.
 * Calls are asynchronous on the state's stream except where noted. Overlapping calls on one state
 * from several threads are not allowed. */
typedef struct qd_sparse qd_sparse;

/* Sparse |0...0> (one entry, amplitude 1) on dims[0..n-1]. capacity: initial entries per list
 * buffer (0 = 65536; the lists grow by themselves). QD_EINVAL / QD_EDIM / QD_EOVERFLOW as for a
 * register, QD_ENOMEM if the device allocation fails. Synchronises. */
int qd_sparse_init(const int32_t* dims, int32_t n, int64_t capacity, void* hip_stream, qd_sparse** out);

/* Replace the list by `count` host entries: idx[e] (distinct, 0..D-1) and amps[2e], amps[2e+1]
 * (finite, not both zero). QD_EINVAL otherwise (the state is unchanged). Synchronises. */
int qd_sparse_upload(qd_sparse* s, const int64_t* idx, const double* amps, int64_t count);

/* One basis state (values[i] in 0..d_i-1), amplitude 1. Synchronises. */
int qd_sparse_set_basis(qd_sparse* s, const int32_t* values);

/* Apply a (controlled) k-qudit gate: arguments and validation exactly as qd_apply_gate_ex (all
 * checks before any device work; a failed call leaves the list unchanged). A dense gate waits once
 * on the host for its slice count. */
int qd_sparse_apply_gate(qd_sparse* s, const int32_t* targets, int32_t k, const int32_t* controls,
                         const int32_t* control_values, int32_t m, const double* U, uint32_t flags);

/* Apply count gates in order (qd_gate as for qd_fuse; flags as qd_apply_gate_ex). Every gate is
 * validated before any device work. Runs of consecutive monomial gates (at most 4 targets and 8
 * controls each) are applied in one pass over the list with the entry's digits held in LDS; the
 * result is the same, bit for bit, as gate by gate. */
int qd_sparse_apply_gates(qd_sparse* s, const qd_gate* gates, int32_t count, uint32_t flags);

/* Number of entries. Synchronises. */
int qd_sparse_count(qd_sparse* s, int64_t* out);

/* Copy the list (list order) to host arrays of `cap` entries (idx: int64, amps: interleaved
 * doubles). *count receives the number of entries; QD_EINVAL if cap is smaller (nothing copied).
 * Synchronises. */
int qd_sparse_download(qd_sparse* s, int64_t* idx, double* amps, int64_t cap, int64_t* count);

/* Device addresses of the current list and its count, valid until the next qd_sparse_* call on s.
 * Synchronises. */
int qd_sparse_device_lists(qd_sparse* s, int64_t** idx, double** amps, int64_t* count);

/* Sum of |a|^2 over the entries in FP64 (fixed reduction order for a given count). Synchronises. */
int qd_sparse_norm2(qd_sparse* s, double* out);

/* |a_e|^2 per entry in list order (re^2 + im^2, each operation rounded) into out (cap entries,
 * device memory when out_is_device). QD_EINVAL if cap is smaller than the count. Synchronises. */
int qd_sparse_probabilities(qd_sparse* s, double* out, int32_t out_is_device, int64_t cap);

/* Write the state into a dense state of the same register (zeros elsewhere; rounded to complex64
 * for a QD_C64 state). QD_EDIM if the registers differ. Synchronises. */
int qd_sparse_to_dense(qd_sparse* s, qd_state* dst);

/* Entries written by gates since the state was created: a monomial gate counts its matching
 * entries, a dense gate the outputs it writes for its slices (the amplitude updates of the
 * throughput figures). Synchronises. */
int qd_sparse_updates(qd_sparse* s, int64_t* out);

/* Wait for the state's queued work. */
int qd_sparse_sync(qd_sparse* s);

/* Apply a circuit's gates in order to a sparse state of the same register (qd_sparse_apply_gate
 * for each). QD_EDIM if the registers differ. */
int qd_circuit_apply_sparse(qd_sparse* s, const qd_circuit* c);

void qd_sparse_free(qd_sparse* s);

/* ---------------------------------------------------------------- density matrices and noise (Sec. 3.1, 3.3, 7) */

/* The paper keeps states as vectors and names density matrices (Sec. 3.3) and noise models (Sec. 7)
 * as the next representations; a channel on qudits of dimensions (d_1..d_k) has Kraus matrices of
 * the size a gate on them has (Sec. 3.1). A density matrix rho over n qudits (D = prod d_i) is a
 * qd_state over the doubled register dims ++ dims: row qudits 0..n-1, column qudits n..2n-1,
 * element (x, y) at flat index x * D + y. qd_norm2, qd_state_download and the other state calls
 * see that doubled register. */

/* rho = |0..0><0..0| over dims[0..n-1] (1 <= n <= 32); prec QD_C128 or QD_C64. */
int qd_density_init(const int32_t* dims, int32_t n, int32_t prec, void* hip_stream, qd_state** out);

/* rho = psi psi^dagger for a pure state of the same register and precision. QD_EDIM / QD_EINVAL
 * otherwise. Asynchronous on rho's stream (psi's stream is drained first). */
int qd_density_from_state(qd_state* rho, const qd_state* psi);

/* rho -> G rho G^dagger for the (controlled) gate of qd_apply_gate_ex on the physical register
 * (targets and controls are 0..n-1; validation and flags as there). With G embedded on its targets
 * and controls (d_G = d_T x prod d_c), a gate with d_G <= 4 (d_G <= 3 for a dense or a monomial
 * non-diagonal U with controls) is one pass of G (x) conj(G) on (T, C, T + n, C + n); others are
 * two passes (U on T, conj(U) on T + n with controls c + n).
 * Asynchronous. */
int qd_density_apply_gate(qd_state* rho, const int32_t* targets, int32_t k, const int32_t* controls,
                          const int32_t* control_values, int32_t m, const double* U, uint32_t flags);

/* rho -> sum_k K_k rho K_k^dagger for nk Kraus operators on targets (d_T <= 32), given as nk
 * consecutive d_T x d_T row-major interleaved complex matrices (first target most significant).
 * QD_ENOTUNITARY unless max |sum_k K_k^dagger K_k - I| <= 1e-10 (QD_FLAG_SKIP_UNITARY_CHECK skips
 * the test). Applied as one pass of sum_k K_k (x) conj(K_k) on (T, T + n). Asynchronous. */
int qd_density_apply_channel(qd_state* rho, const int32_t* targets, int32_t k, const double* kraus, int32_t nk,
                             uint32_t flags);

/* Named one-qudit channels (readings; the paper defines none):
 *  QD_CHANNEL_DEPOLARIZING   rho -> (1 - p) rho + p tr(rho) I/d: sqrt(1 - p + p/d^2) I and
 *                            sqrt(p/d^2) X^a Z^b, (a, b) != (0, 0), operator a d + b (d^2 of them);
 *  QD_CHANNEL_DEPHASING      sqrt(1 - p) I and sqrt(p/(d-1)) Z^b, b = 1..d-1 (d of them);
 *  QD_CHANNEL_AMPLITUDE_DAMPING  K_0 = |0><0| + sqrt(1 - p) sum_{j>=1} |j><j|, K_j = sqrt(p) |j-1><j|
 *                            (d of them).
 * X and Z are the generalized shift and phase gates (Sec. 2.1). *nk receives the count; with out
 * != NULL and cap >= count the operators are written as for qd_density_apply_channel. Host only. */
enum { QD_CHANNEL_DEPOLARIZING = 0, QD_CHANNEL_DEPHASING = 1, QD_CHANNEL_AMPLITUDE_DAMPING = 2 };
int qd_channel_kraus(int32_t kind, int32_t d, double p, double* out, int32_t cap, int32_t* nk);

/* A sequence of density operations: QD_OP_GATE (targets, controls, control values and one d_T x d_T
 * matrix U in mats, nk = 1) or QD_OP_CHANNEL (targets, no controls, nk Kraus operators in mats). */
enum { QD_OP_GATE = 0, QD_OP_CHANNEL = 1 };
typedef struct {
  int32_t kind;
  int32_t k;
  const int32_t* targets;
  int32_t m;
  const int32_t* controls;
  const int32_t* control_values;
  int32_t nk;
  const double* mats;
} qd_density_op;

/* Apply count operations in order, as qd_density_apply_gate / qd_density_apply_channel would, with
 * every operation validated first. A run of two or more consecutive operations whose targets and
 * controls together span qudits S with prod d_S <= 4 (a gate and the channels that follow it, a
 * qubit-controlled gate on a qubit and its channel, operations on two qubits) is composed on the
 * host in FP64: each operation embedded on S (a gate as its controlled unitary, the identity
 * elsewhere), then one pass of the product superoperator on (S, S + n). Asynchronous.
 * A call that fails validation leaves rho unchanged; an allocation or launch failure in a later
 * pass of a call (QD_ENOMEM, QD_EDEVICE) can leave rho with the earlier passes applied, as can such
 * a failure in the second pass of a two-pass qd_density_apply_gate. */
int qd_density_apply_ops(qd_state* rho, const qd_density_op* ops, int32_t count, uint32_t flags);

/* tr(rho) (both parts), fixed reduction order. Synchronises. */
int qd_density_trace(qd_state* rho, double* re, double* im);

/* Re rho[x, x] for x = 0..D-1 (the outcome distribution) into out (device memory when
 * out_is_device). Synchronises. */
int qd_density_probabilities(qd_state* rho, double* out, int32_t out_is_device);

/* tr(rho^2) = sum |rho_xy|^2 (rho Hermitian). Synchronises. */
int qd_density_purity(qd_state* rho, double* out);

/* <psi|rho|psi> (the fidelity with a pure state of the same register and precision). Synchronises. */
int qd_density_fidelity(qd_state* rho, const qd_state* psi, double* out);

/* Number of physical qudits n (0 for a pure state). */
int qd_density_size(const qd_state* rho, int32_t* n_qudits);

/* ---------------------------------------------------------------- batched circuits (Sec. 3.5) */

/* nc independent registers in one device arena: circuit c has n_per[c] qudits whose dims follow
 * consecutively in dims_flat. All states start at |0...0>. prec is QD_C64 or QD_C128. */
int qd_batch_create(int32_t nc, const int32_t* n_per, const int32_t* dims_flat, int32_t prec,
                    void* hip_stream, qd_batch** out);

/* Total amplitudes in the arena and the arena offset (in amplitudes) of circuit c. */
int qd_batch_size(const qd_batch* b, int64_t* total_out);
int qd_batch_offset(const qd_batch* b, int32_t c, int64_t* off_out);

/* Reset every register to |0...0>. Asynchronous. */
int qd_batch_reset(qd_batch* b);

/* One gate layer: gate c acts on circuit c (a Moment of every circuit, Sec. 3.5). gates[c].k == 0
 * means no gate for circuit c in this layer. Supported: one target (d_t <= 8) and at most one
 * control; other shapes are QD_EINVAL. Gates are validated as in qd_apply_gate before any device
 * work. Every layer runs as one persistent launch. While capture is on, the launch is recorded
 * into the batch's graph instead of being run. */
int qd_batch_apply_layer(qd_batch* b, const qd_gate* gates);

/* nlayers layers (gates[l * nc + c] acts on circuit c in layer l; k == 0 = no gate) with the
 * gates of each circuit fused into blocks: a block takes the circuit's next gates in order while
 * it has at most `width` of them (1..8; 0 = the tuned QD_TUNE_BATCH_FUSE) and the union of their
 * qudits (targets and controls) has at most 4 qudits of total dimension in {2..9, 12, 16, 18, 24,
 * 27, 32}. A block of several gates is composed on the GPU in FP64 into one operation on that
 * union (M = U_last ... U_first, each U embedded, the identity where its control misses; cast to
 * the state's precision at the end) and applied in one pass over the state. Launch i applies every
 * circuit's i-th block, so the launch count is the most blocks of any circuit. Gates are validated
 * as in qd_batch_apply_layer before any device work. While capture is on, the launches are
 * recorded into the graph and the compositions run once, at recording (replays reuse the composed
 * blocks). */
int qd_batch_apply_layers(qd_batch* b, const qd_gate* gates, int32_t nlayers, int32_t width);

/* Tuning of the batched layer kernel by operation key (S9's gate class, d_T and stride class):
 * key = 6 g + 2 c + s with g = 0 for one gate, 1 for a composed block; c = 0 for d_T <= 4, 1 for
 * d_T 5..9, 2 for d_T 12..32; s = 0 when the operation's smallest target stride is below 16
 * amplitudes (one 128-byte line of complex64), else 1. spt is the slices per thread of that key's
 * operations: 1, 2, 4 or 8, or 0 to use QD_TUNE_BATCH_SPT_MID / _WIDE and the default rule.
 * qd_batch_autotune_layers tunes the keys that carry at least 3% of the workload's amplitude
 * updates; qd_tune_save writes every key. QD_EINVAL for a key outside 0..11 or another value. */
enum { QD_BATCH_KEYS = 12 };
int qd_batch_tune_key_set(int32_t key, int32_t spt);
int qd_batch_tune_key_get(int32_t key, int32_t* spt);

/* GPU time (ms, HIP events) of the block compositions qd_batch_apply_layers has launched since
 * the previous call (or since the batch was created). Synchronises with those compositions. */
int qd_batch_compose_ms(qd_batch* b, double* ms);

/* Fusion-width autotuner: records qd_batch_apply_layers over the given layers into a graph for
 * widths 1, 2, 3, 4, 6 and 8, times replays of each (the compositions run at recording, outside
 * the timed replays) and keeps the fastest as QD_TUNE_BATCH_FUSE; then, at that width, the slices
 * per thread of each wide slice class (QD_TUNE_BATCH_SPT_MID, then QD_TUNE_BATCH_SPT_WIDE: the
 * rule, 1, 2, 4, 8); then those of each operation key (qd_batch_tune_key_set) carrying at least 3%
 * of the amplitude updates, in decreasing share, a change kept when it gains 1%. All are saved by
 * qd_tune_save. The arena is saved and restored and a graph the caller recorded is kept. Not
 * allowed while recording. Synchronises. */
int qd_batch_autotune_layers(qd_batch* b, const qd_gate* gates, int32_t nlayers);

/* on = 1 starts recording layers into a new graph (dropping any previous one); on = 0 ends the
 * recording and instantiates the graph. */
int qd_batch_capture(qd_batch* b, int32_t on);

/* Autotuner of the batched layer kernel: times the layer `gates` (as qd_batch_apply_layer) with
 * every candidate tile shape (threads per workgroup x slices per thread) and keeps the fastest in
 * the process-wide tuning table (saved by qd_tune_save). The arena is saved and restored, so the
 * states are unchanged. Not allowed while recording. Synchronises. */
int qd_batch_autotune(qd_batch* b, const qd_gate* gates);

/* Launch the recorded graph once on the batch's stream. QD_EINVAL if none is recorded. */
int qd_batch_replay(qd_batch* b);

/* Copy the whole arena (total amplitudes, interleaved) to host memory; synchronises. */
int qd_batch_download(const qd_batch* b, void* host_amps, int64_t total);

void qd_batch_free(qd_batch* b);

/* ---------------------------------------------------------------- tuning and calibration */

/* Tile parameters the launchers use (QD_TUNE_* below): threads per workgroup (64, 128, 192 or
 * 256), slices per thread (1, 2 or 4; the batched kernel also 8), amplitudes per LDS tile (power of two, 256..4096),
 * slice columns per fused tile (32, 64, 128), the target stride below which a gate is staged
 * in LDS (QD_TUNE_RUN_MIN, 1..1024 amplitudes) and the workgroups per compute unit of the batched
 * layer kernel (QD_TUNE_BATCH_GRID: 1..63 persistent workgroups walk the tile list; 64 launches one
 * workgroup per tile), the most gates qd_batch_apply_layers composes into one operation
 * (QD_TUNE_BATCH_FUSE, 1..8) and the slices per thread of batched slices of 5..9 and of 12..32
 * amplitudes (QD_TUNE_BATCH_SPT_MID, QD_TUNE_BATCH_SPT_WIDE: 1, 2, 4 or 8; 0 keeps the rule of two
 * batches of 16 / d_T slices, at most QD_TUNE_BATCH_SPT). 0 restores the default. Process-wide,
 * host only; QD_EINVAL for an unknown parameter or a value outside its range. */
enum { QD_TUNE_DIRECT_BLOCK = 0, QD_TUNE_DIRECT_SPT = 1, QD_TUNE_TILE_BLOCK = 2,
       QD_TUNE_TILE_ELEMS = 3, QD_TUNE_DIAG_BLOCK = 4, QD_TUNE_BATCH_BLOCK = 5,
       QD_TUNE_BATCH_SPT = 6, QD_TUNE_FUSED_COLS = 7, QD_TUNE_RUN_MIN = 8, QD_TUNE_BATCH_GRID = 9,
       QD_TUNE_BATCH_FUSE = 10, QD_TUNE_BATCH_SPT_MID = 11, QD_TUNE_BATCH_SPT_WIDE = 12, QD_TUNE_COUNT = 13 };
int qd_tune_set(int32_t param, int32_t value);
int qd_tune_get(int32_t param, int32_t* value);

/* Autotuner of the gate kernels: for each stride class of the smallest target stride (1, 2-3,
 * 4-15, 16-255, 256-4095, >= 4096) present in the state's register, times a dense single-qudit gate with
 * every candidate tile shape (direct: 64/128/256 threads x 1/2/4 slices per thread; LDS tile:
 * 512..4096 amplitudes x 128/256 threads) and keeps the fastest per (precision, stride class).
 * The state's amplitudes are overwritten: pass a scratch state. Writes the table as JSON to path
 * (NULL = no file). A later qd_tune_set discards the tuned table. Synchronises. */
int qd_autotune(qd_state* scratch, const char* path);

/* Load a cache written by qd_autotune / qd_tune_save (replacing the current table). QD_EINVAL if
 * the file cannot be read or holds no valid entry. */
int qd_tune_load(const char* path);

/* Write the current tuning table (gate kernels and batched kernel) as JSON to path. */
int qd_tune_save(const char* path);

/* Device-to-device copy of `bytes` bytes with the library's streaming copy kernel, for the HBM
 * ceiling and the hardware-counter calibration. Asynchronous on hip_stream. */
int qd_stream_copy(void* dst, const void* src, int64_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* QD_H */
