/*
 * qw.h -- C ABI of libqw, the MI355X (gfx950) prefix-reuse statevector path.
 *
 * The path follows the paper's statement of the problem (Sec. I and Fig. 1,
 * Sec. III-A "Execution"): tasks of a workload share a gate prefix; the
 * prefix is executed once, the exact boundary state |psi_B> is materialised
 * as a typed artifact (Sec. IV-B, ArtifactRecord), and every task's suffix is
 * re-run from it; each continuation first passes the three legality gates of
 * Sec. IV-B (exactness, backend family, conversion rule of Table II) and is
 * otherwise refused with the structured record of the EVAL-7 example.
 *
 * Conventions for every call
 *   - Qubit q is bit q of the basis index (little-endian). A state of n
 *     qubits is 2^n complex64 amplitudes (interleaved re, im; 8 bytes each),
 *     slot s of a state starting at byte offset s * 8 * 2^n.
 *   - All device work is enqueued, in call order, on the HIP stream given to
 *     qw_ctx_create; calls return when the work is enqueued unless stated.
 *   - Every call returns a status (QW_OK = 0 on success). On failure no
 *     output is written and qw_last_error() describes the failure.
 *   - Pointers named host_* or documented as host memory are read during the
 *     call only; the library keeps no reference to them.
 *   - Not thread-safe per context: use one context per host thread.
 */
#ifndef QW_H
#define QW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status */
#define QW_OK 0
#define QW_E_INVALID_ARG 1  /* bad handle, size, index or gate              */
#define QW_E_OOM 2          /* device or pinned host allocation failed      */
#define QW_E_HIP 3          /* a HIP runtime call failed (message attached) */
#define QW_E_REFUSED 4      /* a continuation failed a legality gate; the
                               refusal record (JSON) is in qw_last_error()  */
#define QW_E_UNSUPPORTED 5  /* valid request outside what the library does  */
#define QW_E_ABANDONED 6    /* a persistent launch gave up a bounded wait
                               (QW_OPT_SPIN_LIMIT or qw_ctx_abandon); the
                               states it was computing are undefined; reported
                               by qw_ctx_sync                                */

/* ------------------------------------------------------------ gates */
/* Gate kinds. Matrices in the computational basis (|0>, |1>):
 *   X = [[0,1],[1,0]]   Y = [[0,-i],[i,0]]   Z = diag(1,-1)
 *   H = [[1,1],[1,-1]]/sqrt2   S = diag(1,i)   SDG = diag(1,-i)
 *   T = diag(1,e^{i pi/4})     TDG = diag(1,e^{-i pi/4})
 *   RX(t) = exp(-i t X/2)  RY(t) = exp(-i t Y/2)  RZ(t) = exp(-i t Z/2)
 *   P(t) = diag(1, e^{i t})
 *   CNOT: control q0, target q1: |b> -> |b xor (b_q0 << q1)>
 *   CZ:   phase -1 when bits q0 and q1 are both 1
 *   RENORM: no qubits; the state is divided by its norm (computed in FP64)
 *           at this point of the gate list.
 *   PROJ0(f) = diag(f, 0), PROJ1(f) = diag(0, f) on q0 (f = param, real):
 *           a projector onto q0 = 0 / 1 with a real factor (not unitary).
 *   MEASURE (mid-circuit Z measurement of q0, the measurement barrier of
 *           Sec. III-A's segmenter): param = u in [0, 1), the caller's
 *           uniform draw for this measurement. With S = sum_i |psi_i|^2 and
 *           S1 the same sum over the indices with bit q0 set (FP64 sums of
 *           the FP32 amplitudes, fixed order), the outcome is b = 1 if
 *           u < S1 / S (FP64), else b = 0, and the state becomes
 *           P_b psi / sqrt(S_b) (S_0 = S - S1). The outcome is recorded
 *           (qw_outcomes).
 *   RESET:  a MEASURE of q0 followed by X on q0 when b = 1 (q0 ends in |0>);
 *           param = u as for MEASURE, and the outcome is recorded.
 * A gate list with MEASURE or RESET runs in segments. A measurement commutes
 * with gates on other qubits, so a segment runs the gates up to a
 * measurement and every later gate that touches no qubit measured so far;
 * the measurements met on the way (up to 12, on distinct qubits, a RENORM or
 * a gate on a measured qubit ends the segment) are then decided together
 * from one FP64 sweep over the state: a single measurement from S and S1 as
 * above; several (all on qubits >= 8) from the FP64 masses of their 2^k
 * outcome bins, in gate order, each by the rule above applied to the masses
 * that agree with the earlier outcomes (the sequential rule, with the
 * probabilities it would see). The decisions run on the device, in FP64,
 * from the draws of the gate list: a decision kernel writes each outcome
 * and the operator that opens the next segment, one per measured qubit (the
 * projector P_b, the first with the factor 1 / sqrt of the chosen outcome's
 * mass, times X for a RESET with outcome 1), which that segment's first pass
 * applies as a real 2x2 operator read at run time. So the pass plans do not
 * depend on outcomes and no decision waits for the host: a call
 * synchronises the stream once, at its end, to collect the outcomes
 * (qw_outcomes), and a recorded graph needs no host at all
 * (qw_graph_outcomes). A state of zero norm at a measurement gives
 * QW_E_INVALID_ARG at the end of the call. */
#define QW_GATE_X 0x01
#define QW_GATE_Y 0x02
#define QW_GATE_Z 0x03
#define QW_GATE_H 0x04
#define QW_GATE_S 0x05
#define QW_GATE_SDG 0x06
#define QW_GATE_T 0x07
#define QW_GATE_TDG 0x08
#define QW_GATE_RX 0x21
#define QW_GATE_RY 0x22
#define QW_GATE_RZ 0x23
#define QW_GATE_P 0x24
#define QW_GATE_CNOT 0x41
#define QW_GATE_CZ 0x42
#define QW_GATE_RENORM 0x81
#define QW_GATE_MEASURE 0x82
#define QW_GATE_RESET 0x83
#define QW_GATE_PROJ0 0x84
#define QW_GATE_PROJ1 0x85

typedef struct qw_gate {
    uint32_t kind;     /* QW_GATE_*                                     */
    uint32_t q0;       /* qubit (control of CNOT)                       */
    uint32_t q1;       /* second qubit (target of CNOT); else ignored   */
    uint32_t reserved; /* must be 0                                     */
    double param;      /* angle of RX/RY/RZ/P in radians; u of MEASURE
                          and RESET; factor of PROJ0/PROJ1; else ignored */
} qw_gate;             /* 24 bytes */

/* ------------------------------------------------------------ artifacts */
/* Typed artifact metadata (Sec. IV-B: kind, exactness class, provenance
 * hash, producing backend family, size). */
#define QW_KIND_STATEVECTOR 1 /* STATEVECTOR_BOUNDARY_STATE */
#define QW_KIND_TABLEAU 2     /* TABLEAU_BOUNDARY_STATE     */

#define QW_EXACTNESS_UNKNOWN 0
#define QW_EXACT 1
#define QW_APPROX 2

#define QW_BACKEND_UNKNOWN 0
#define QW_BACKEND_SV 1        /* this library: MI355X_SV_C64, statevector    */
#define QW_BACKEND_STAB_ONLY 2 /* a stabilizer-only (tableau) backend family */

typedef struct qw_artifact {
    uint32_t kind;          /* QW_KIND_*                                  */
    uint32_t exactness;     /* QW_EXACT / QW_APPROX / QW_EXACTNESS_UNKNOWN */
    uint32_t backend;       /* producing backend family, QW_BACKEND_*     */
    uint32_t n_qubits;
    uint64_t bytes;         /* payload size                               */
    uint8_t provenance[32]; /* Eq. (1) fingerprint of the producing prefix */
} qw_artifact;

/* Snapshot modes. COPY: the boundary state is copied into a buffer of its
 * own (one read and one write of the state). FREEZE: the slot itself becomes
 * the artifact (no data moves) and may not be written until the snapshot is
 * freed. */
#define QW_SNAP_COPY 0
#define QW_SNAP_FREEZE 1

typedef struct qw_ctx qw_ctx;
typedef struct qw_state qw_state;
typedef struct qw_snap qw_snap; /* a boundary snapshot (artifact) */

/* One continuation: the suffix gates of a task and where its state goes. */
typedef struct qw_task {
    const qw_gate *gates;    /* host array of n_gates gates (may be NULL if 0) */
    uint64_t n_gates;
    uint32_t dst_slot;       /* slot of the destination state              */
    uint32_t reserved;       /* must be 0                                  */
    uint8_t expect_prov[32]; /* provenance the task expects of its source  */
} qw_task;

/* Optional expectation epilogue of qw_run_suffix_batch: for task k,
 * out[k] = sum_j coeff[j] <psi_k| P_j |psi_k>, P_j given by (x_mask[j],
 * z_mask[j]) as in qw_expect_pauli. Masks and coefficients are host arrays. */
typedef struct qw_reduce {
    const uint64_t *x_mask;
    const uint64_t *z_mask;
    const double *coeff;
    uint32_t n_terms;
    int32_t out_is_host;    /* 1: out is host memory (call synchronises)  */
    double *out;            /* n_tasks doubles                             */
} qw_reduce;

/* ------------------------------------------------------------ context */
/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream). The stream is not owned. The
 * context owns its plan/scratch buffers and the last-error text. */
int qw_ctx_create(int device, void *hip_stream, qw_ctx **out);
int qw_ctx_destroy(qw_ctx *ctx);
/* Text of the last error of this context ("" if none); valid until the next
 * call on it. For QW_E_REFUSED it is the refusal JSON record. */
const char *qw_last_error(const qw_ctx *ctx);
/* Block until all work enqueued by this context has finished. */
int qw_ctx_sync(qw_ctx *ctx);

/* Tunables (defaults in brackets):
 *   QW_OPT_TILE_BITS      max local bits per pass tile, 10..14 [14]
 *   QW_OPT_PROFILE        1: time every pass/reducer launch with HIP events
 *                         (read with qw_ctx_kernel_stats) [0]
 *   QW_OPT_XCD_REMAP      1: map workgroups so that the tiles of one source
 *                         state run on one XCD [1]
 *   QW_OPT_JIT            1: run gate passes of states with >= 10 qubits with
 *                         kernels generated for each pass structure and
 *                         compiled at run time with hipRTC (cached in memory,
 *                         and on disk under $QW_JIT_CACHE, default
 *                         ~/.cache/qw_jit; QW_JIT_CACHE=off disables the disk
 *                         cache); 0: interpreted pass kernels. Both forms
 *                         give bit-identical states. [1]
 *   QW_OPT_RELABEL        1: a pass may end with CNOTs whose targets are not
 *                         local to its tiles, applied as a permutation of
 *                         its store addresses (one pass fewer for CNOT
 *                         ladders); such a pass never runs in place, so each
 *                         task with one gets a second state buffer held by
 *                         the context. 0: plans without relabelling. Both
 *                         give the same state up to FP32 rounding. [1]
 *   QW_OPT_SECOND_BUFFER_CAP  bytes of second state buffers one execution
 *                         may hold; batches beyond it run in chunks
 *                         (at least one task per chunk) [16 GiB]
 *   QW_OPT_FUSED_EPILOGUE 1: in qw_run_suffix_batch with an expectation
 *                         epilogue, the Pauli terms that the tasks' common
 *                         last pass can evaluate on its own tiles (after
 *                         conjugation through its output relabelling) are
 *                         reduced inside that pass (generated kernels),
 *                         when that saves a reducer sweep over the states;
 *                         the results agree with separate reduction up to
 *                         FP32 rounding of the per-thread partial sums. [1]
 *   QW_OPT_STREAM_LOADS   1: generated pass kernels load the state with the
 *                         non-temporal cache policy, except a first pass that
 *                         reads a boundary snapshot (other tasks read it
 *                         too); 0: default policy for every load. Stores of
 *                         generated passes are always non-temporal. Results
 *                         do not depend on it [1]
 *   QW_OPT_TILE_ORDER     order in which the persistent generated kernels
 *                         (multi-phase passes, reducers) take the
 *                         (task, tile) items of a launch: the tasks of one
 *                         tile together (descriptor-major) or consecutive
 *                         tiles of one task (tile-major). 0: always
 *                         descriptor-major; 1: tile-major for passes with
 *                         output relabelling, descriptor-major otherwise;
 *                         2: tile-major for every pass and reducer launch.
 *                         Launches whose tasks all read one source state (a
 *                         shared snapshot) stay descriptor-major, so the
 *                         tasks of a tile share its reads in L2. Results do
 *                         not depend on it; on config-2-like batches mode 1
 *                         measured fastest. [1] */
#define QW_OPT_TILE_BITS 1
#define QW_OPT_PROFILE 2
#define QW_OPT_XCD_REMAP 4
#define QW_OPT_JIT 5
#define QW_OPT_RELABEL 6
#define QW_OPT_SECOND_BUFFER_CAP 7
#define QW_OPT_FUSED_EPILOGUE 8
#define QW_OPT_TILE_ORDER 9
#define QW_OPT_STREAM_LOADS 10
/*   QW_OPT_DEVICE_MEM_CAP bytes of device memory the context may hold: its
 *                         states and snapshot copies (allocated by it or
 *                         given by the caller), and its plan,
 *                         scratch, second-state and measurement buffers
 *                         (buffers handed to a recorded graph belong to the
 *                         graph); a call that would pass
 *                         it returns QW_E_OOM (each allocation is checked
 *                         before the device work that needs it; a suffix
 *                         batch refused this way may have written part of
 *                         its destination slots), and the caller may retry
 *                         with fewer slots or tasks per call. Setting it
 *                         synchronises the stream and releases the plan,
 *                         scratch, second-state and measurement buffers (they
 *                         grow again as calls need them); refused while a
 *                         graph is recorded. 0 = no cap, only the device's
 *                         own limit. [0] */
#define QW_OPT_DEVICE_MEM_CAP 11
/*   QW_OPT_LAYOUT         index layouts between the passes of one call:
 *                         the planner may permute the qubits' index bits so
 *                         that the tiles of a pass are longer contiguous
 *                         runs of the state (the state before the first and
 *                         after the last pass of a call is always in the
 *                         standard layout; a pass that changes the layout
 *                         runs out of place, like a relabelling pass, with
 *                         the second buffers of QW_OPT_SECOND_BUFFER_CAP).
 *                         0: standard layout throughout; 1: permuted
 *                         layouts when the call's states exceed 128 MiB
 *                         (smaller ones stay in the device's last-level
 *                         cache when updated in place); 2: permuted layouts
 *                         for every call. Results are bitwise the same in
 *                         every mode. [1] */
#define QW_OPT_LAYOUT 12
/*   QW_OPT_PERSISTENT     1: with generated kernels, each qw_run_suffix_batch
 *                         or qw_run_tree call runs all of its passes (every
 *                         pass index, every pass structure and, in a tree,
 *                         every level) in ONE persistent kernel launch: its
 *                         workgroups take (descriptor, tile range) claims in
 *                         order from one device counter, and a claim whose
 *                         source is still being written waits, in a bounded
 *                         poll, for the completion counter of the pass (or
 *                         parent task) that writes it. Claims only wait for
 *                         earlier claims, so the launch completes without
 *                         requiring its workgroups to be resident at once.
 *                         Calls that need a norm finalisation between
 *                         passes (noisy jumps) or interpreted kernels keep
 *                         one launch per pass structure, and so do the
 *                         passes of a single state (qw_apply_prefix,
 *                         measured segments), which have no other tasks to
 *                         fill the device between dependent passes. Results
 *                         are bitwise those of the per-pass launches. [0] */
#define QW_OPT_PERSISTENT 13
/*   QW_OPT_SPIN_LIMIT     microseconds one wait of a persistent launch may
 *                         last before it is abandoned (the launch then skips
 *                         its remaining work and qw_ctx_sync returns
 *                         QW_E_ABANDONED); 0 abandons at the first wait
 *                         that is not already satisfied. [1048576, ~1 s] */
#define QW_OPT_SPIN_LIMIT 14
/*   QW_OPT_PERSIST_CHUNK  most tiles (rows of an expectation epilogue) of one
 *                         descriptor that a workgroup of a persistent launch
 *                         takes per claim (a power of two, 1..1024); fewer
 *                         when a segment has too few claims to keep four per
 *                         workgroup. Each claim ends with a release of its
 *                         stores and a dependent claim starts with an
 *                         acquire, so larger claims synchronise less. [8] */
#define QW_OPT_PERSIST_CHUNK 15
int qw_ctx_set_option(qw_ctx *ctx, int key, int64_t value);

/* Ask the waits of running and later persistent launches of this context to
 * give up (callable from any host thread while the GPU works): they end with
 * QW_E_ABANDONED at the next qw_ctx_sync, which also withdraws the request. */
int qw_ctx_abandon(qw_ctx *ctx);

/* Per-kernel launch statistics gathered while QW_OPT_PROFILE is 1.
 * kernel: 0 = gate pass, 1 = expectation reducer, 2 = sampler, 3 = copy.
 * Writes launch count, total milliseconds and total algorithmic bytes
 * (read + write of every amplitude the launches touch). Resets on read when
 * reset != 0. Synchronises the stream. */
int qw_ctx_kernel_stats(qw_ctx *ctx, int kernel, uint64_t *launches,
                        double *total_ms, double *total_bytes, int reset);

/* ------------------------------------------------------------ states */
/* qw_state_alloc: a state of n_qubits (1..30) with n_slots slots, every
 * slot set to |0...0>. The slots hold the task states of a workload: the
 * boundary state |psi_B> that the shared prefix produces and the states
 * every task's suffix continues into (Sec. I and Fig. 1; Sec. III-A
 * "Execution": the prefix state is materialised once and reloaded for each
 * suffix), all starting from the all-zero basis state the circuits assume.
 * On a bad size, n_qubits or alignment: QW_E_INVALID_ARG; if the device
 * allocation fails: QW_E_OOM; *out is written only on success. If dev_buf is non-NULL it must be device memory of at
 * least n_slots * 8 * 2^n bytes (dev_buf_bytes), 256-byte aligned; the state
 * is then a view and the caller keeps the buffer alive until qw_state_free.
 * If dev_buf is NULL the library allocates (hipMalloc) and frees it. */
int qw_state_alloc(qw_ctx *ctx, uint32_t n_qubits, uint32_t n_slots,
                   void *dev_buf, uint64_t dev_buf_bytes, qw_state **out);
int qw_state_free(qw_state *st);
/* Set slots [first, first + count) to |0...0>. */
int qw_state_reset(qw_state *st, uint32_t first, uint32_t count);
/* Device address of slot `slot` (for copies by the caller). */
int qw_state_slot_ptr(const qw_state *st, uint32_t slot, void **dev_ptr);

/* ------------------------------------------------------------ the path */
/* qw_apply_prefix: apply `gates` (host array) in order to slot `slot`, in
 * place. This is the execution of a shared prefix (Sec. III-A, executed
 * once); the direct path calls it for a task's prefix and then its suffix,
 * so both paths cut the pass plan at the same boundary and produce bitwise
 * identical states. */
int qw_apply_prefix(qw_state *st, uint32_t slot, const qw_gate *gates,
                    uint64_t n_gates);

/* qw_snapshot: materialise slot `slot` as an immutable EXACT statevector
 * artifact (Sec. IV-B ArtifactRecord) with the given 32-byte provenance
 * (the Eq. (1) fingerprint computed by the caller). mode QW_SNAP_COPY copies
 * the state into copy_buf (device memory, >= 8 * 2^n bytes) or, if copy_buf
 * is NULL, into a buffer the library allocates; QW_SNAP_FREEZE moves no data
 * and freezes the slot. `parent` (may be NULL) links prefix-tree levels and
 * must be a snapshot of the same qubit count. Free with qw_snapshot_free
 * (which unfreezes a FREEZE slot). */
int qw_snapshot(qw_state *st, uint32_t slot, const uint8_t provenance[32],
                int mode, const qw_snap *parent, void *copy_buf,
                uint64_t copy_buf_bytes, qw_snap **out);
int qw_snapshot_free(qw_snap *snap);
int qw_snapshot_info(const qw_snap *snap, qw_artifact *out);

/* qw_run_suffix_batch: run n_tasks continuations into state `dst`.
 * src[k] is task k's boundary snapshot; src == NULL or src[k] == NULL means
 * the direct path (the suffix runs in place on dst slot tasks[k].dst_slot).
 * Before any device work every task with a snapshot passes the legality
 * gates of Sec. IV-B in order: (1) exactness (artifact must be EXACT),
 * (2) backend family (artifact produced by a known statevector family that
 * this target accepts), (3) conversion rule of Table II (statevector ->
 * statevector only), plus the artifact's qubit count and its provenance
 * against tasks[k].expect_prov. If any gate fails nothing is enqueued and
 * QW_E_REFUSED is returned with the refusal record (fields reason, detail,
 * source_kind, target_kind, source_backend, target_backend) as
 * qw_last_error(); the caller then falls back to the direct path.
 * Destination slots must be distinct and not frozen. If `epilogue` is
 * non-NULL its expectations are written for every task; part of its terms
 * may be reduced inside the batch's last pass (QW_OPT_FUSED_EPILOGUE), the
 * rest by reducer sweeps over the destination states. */
int qw_run_suffix_batch(qw_ctx *ctx, const qw_snap *const *src,
                        const qw_task *tasks, uint32_t n_tasks, qw_state *dst,
                        const qw_reduce *epilogue);

/* qw_run_tree: run a tree of continuations in one call (the prefix tree of
 * Fig. 1 and Sec. III-A, where a materialized node's state is the boundary
 * of the tasks below it). Task k starts from
 *   - the final state of task parent[k] of this call when parent[k] >= 0
 *     (parent[k] < k, so parents come first), or else
 *   - its boundary snapshot src[k] (src may be NULL), or else
 *   - its destination slot as it stands (the direct path).
 * out_prov (n_tasks x 32 bytes, required when any parent[k] >= 0) is the
 * provenance of each task's final state; a child's tasks[k].expect_prov
 * must equal its parent's, and snapshot sources pass the legality gates of
 * qw_run_suffix_batch. Destination slots must be distinct and not frozen;
 * gates may not measure or reset. A task with a parent must have gates.
 * With QW_OPT_PERSISTENT the whole tree is one kernel launch; otherwise it
 * runs level by level (a task after its parent's level). Every task's final
 * state is bitwise the one qw_run_suffix_batch would compute from the same
 * source with the same gates. No expectations: use qw_expect_pauli after. */
int qw_run_tree(qw_ctx *ctx, const qw_snap *const *src, const qw_task *tasks,
                const int32_t *parent, const uint8_t *out_prov, uint32_t n_tasks,
                qw_state *dst);

/* qw_outcomes: the measurement outcomes (0 or 1, one byte each) of the
 * MEASURE and RESET gates of the most recent qw_apply_prefix or
 * qw_run_suffix_batch on this context, task by task in task order and, within
 * a task, in gate order (a call without measurements leaves none). Writes
 * min(count, cap) bytes to out (host memory; may be NULL when cap is 0) and
 * the total to *count. The record stays until the next such call. */
int qw_outcomes(const qw_ctx *ctx, uint8_t *out, uint64_t cap, uint64_t *count);

/* qw_expect_pauli: the Pauli-sum expectation of each task state, the
 * observable of the paper's variational workloads that evaluate one
 * Hamiltonian repeatedly on many related circuits (the vqe_real and
 * param_sweep families of Sec. V). For each slot s in [first, first + count):
 *   out[s - first] = sum_j coeff[j] * Re sum_i conj(psi[i ^ x_j]) *
 *                    i^{popcount(x_j & z_j)} * (-1)^{popcount(i & z_j)} psi[i]
 * i.e. sum_j c_j <P_j> with X on the bits of x_j only, Z on bits of z_j only
 * and Y on bits set in both. Masks and coefficients are host arrays; out is
 * host memory (out_is_host = 1; the call then synchronises) or device
 * memory. Products and sums are in FP64 with a fixed reduction order, so the
 * result does not depend on batch composition. Bad slots or a NULL array
 * with n_terms > 0: QW_E_INVALID_ARG, nothing written. */
int qw_expect_pauli(const qw_state *st, uint32_t first, uint32_t count,
                    const uint64_t *x_mask, const uint64_t *z_mask,
                    const double *coeff, uint32_t n_terms, double *out,
                    int out_is_host);

/* qw_sample: `shots` Z-basis outcomes per slot: the multishot measurement
 * of the noisy_multishot family (Sec. V; Sec. VI, Q1), where one
 * materialised state is sampled for many shots instead of re-running the
 * circuit per shot. For slot first + k and shot
 * s, u = (SplitMix64(seed ^ ((task_base + k) * 2^32 + s)) >> 11) * 2^-53 and
 * the outcome is the smallest basis index i with CDF_i > u * total, where
 * CDF_i is the FP64 running sum of |psi_j|^2 over j <= i and total = CDF of
 * the last index. The running sum is accumulated as chunk prefixes (chunks
 * of 2^10 amplitudes), then sums of 64-amplitude sub-chunks, then single
 * amplitudes; where rounding leaves u * total past the mass of the located
 * chunk or sub-chunk, its last index of non-zero probability is taken. out[k * shots + s] receives the index (uint32); out is
 * host (out_is_host = 1, call synchronises) or device memory. count == 0 or
 * shots == 0: QW_OK with nothing written; bad slots or a NULL out:
 * QW_E_INVALID_ARG. */
int qw_sample(const qw_state *st, uint32_t first, uint32_t count,
              uint64_t seed, uint64_t task_base, uint32_t shots,
              uint32_t *out, int out_is_host);

/* qw_sample_noalloc: qw_sample for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same outcomes (bitwise those of qw_sample),
 * but every buffer beyond the state and `out` lives in a fixed device
 * scratch of 64 MiB (QW_NOALLOC_SCRATCH_BYTES) that the library holds on
 * each GPU it runs on until the process ends, and the call makes no device
 * or host allocation of its own. It needs 256-byte-aligned room for
 *   count pointers, 2 * count * 2^(n - 10) and count * 2^(n - 6) doubles,
 *   count doubles, and with out_is_host = 1 count * shots indices
 * (at 24 qubits about 2.3 MiB per slot: 27 slots; at 20 qubits 455); a
 * larger request returns QW_E_INVALID_ARG with the sizes in qw_last_error()
 * and enqueues nothing. Every call on a GPU uses that GPU's one scratch and
 * leaves its last contents there (nothing in it needs to start at zero):
 * calls that overlap on one GPU (other streams or contexts, other host
 * threads) race and must be ordered by the caller. While a graph is being
 * recorded it returns QW_E_UNSUPPORTED. */
#define QW_NOALLOC_SCRATCH_BYTES (64ull << 20)
int qw_sample_noalloc(const qw_state *st, uint32_t first, uint32_t count,
                      uint64_t seed, uint64_t task_base, uint32_t shots,
                      uint32_t *out, int out_is_host);

/* ------------------------------------------------------------ graphs
 * A workload's device work recorded once and replayed as one HIP graph
 * launch: the batched suffix scheduling of Sec. III-A (tasks that branch
 * from one snapshot or from a tree of snapshots, Fig. 1) without the host
 * planning, plan uploads and per-pass launches of every repetition.
 *
 * qw_graph_begin: the calls that follow on this context (qw_state_alloc,
 *   qw_state_reset, qw_apply_prefix, qw_snapshot, qw_run_suffix_batch,
 *   qw_expect_pauli, qw_sample, qw_tableau_export, the qw_mlp_* calls) are
 *   planned, checked (legality gates included) and their plans uploaded
 *   now, but their device work is recorded instead of run. The call first
 *   synchronises the context's stream. Gate lists with MEASURE and RESET
 *   record too: their decisions run on the device (qw_graph_outcomes reads
 *   the outcomes of a replay). While recording, these return
 *   QW_E_UNSUPPORTED: host outputs (out_is_host = 1 or an epilogue with
 *   out_is_host = 1), an expectation with no terms, qw_sample_noalloc,
 *   qw_ctx_sync, qw_ctx_kernel_stats, qw_snapshot_free, qw_state_free,
 *   qw_graph_launch, qw_graph_free and qw_graph_outcomes.
 *   QW_OPT_PROFILE timing is suspended. A call that fails while recording
 *   leaves the recording open; qw_graph_end then reports the failure.
 * qw_graph_end: closes the recording and returns the instantiated graph in
 *   *out. The graph owns the plan records and scratch buffers its nodes
 *   read; it does NOT own the states, snapshots and device outputs named in
 *   the recorded calls: the caller keeps them allocated (and frozen slots
 *   frozen) until qw_graph_free. On failure *out is NULL and the recording
 *   is closed.
 * qw_graph_launch: enqueues one replay on the context's stream (asynchronous).
 *   A replay performs exactly the recorded device work, in order, on the
 *   recorded buffers, so its results are bitwise those of the recorded calls
 *   run directly. Replays and direct calls of one context are ordered by
 *   its stream; they share no buffer except the caller's states and outputs.
 * qw_graph_nodes: number of nodes (kernels and copies) in the graph.
 * qw_graph_update_gates: new gates for task `task` of the `call`-th recorded
 *   gate-running call (qw_apply_prefix or qw_run_suffix_batch, counted from
 *   0 in recording order; a qw_apply_prefix has one task), e.g. the angles
 *   of the next iteration of a variational loop. The gates are planned with
 *   the context's current options and must give the recorded pass
 *   structure (same gate kinds and qubits); otherwise QW_E_INVALID_ARG and
 *   nothing changes, and the caller records the new gates afresh. The
 *   structure depends on the gate kinds and qubits, and on angle values
 *   only in degenerate cases: a fused run of one-qubit gates whose FP64
 *   product is exactly diagonal, exactly the identity or exactly a swap
 *   (e.g. an angle of exactly 0) lowers to a cheaper op or to none, and
 *   real rotations fused between two diagonal gates are rescaled to one-FMA
 *   form unless their combined scale would pass 2^96 (two or more
 *   rotations in a row, each within about 1e-9 of pi), which keeps the
 *   plain form. The call synchronises the context's stream and rewrites the
 *   op records the graph's nodes read; later replays use the new gates.
 *   The provenance of snapshots recorded in the graph is not recomputed:
 *   it stays that of the gates at recording time. MEASURE and RESET gates
 *   are refused.
 * qw_graph_free: synchronises the context's stream and releases the graph
 *   and its buffers. */
typedef struct qw_graph qw_graph;
int qw_graph_begin(qw_ctx *ctx);
int qw_graph_end(qw_ctx *ctx, qw_graph **out);
int qw_graph_launch(qw_graph *g);
int qw_graph_nodes(const qw_graph *g, uint64_t *nodes);
int qw_graph_update_gates(qw_graph *g, uint32_t call, uint32_t task, const qw_gate *gates,
                          uint64_t n_gates);
int qw_graph_free(qw_graph *g);
/* qw_graph_outcomes: the measurement outcomes (one byte each) of the
 * measured calls recorded in the graph, as written by its most recent
 * replay: call by call in recording order, within a call as qw_outcomes
 * orders them. Synchronises the context's stream; writes min(count, cap)
 * bytes to out (host) and the total to *count. If a replay measured a zero
 * state: QW_E_INVALID_ARG (the bytes are still written). */
int qw_graph_outcomes(qw_graph *g, uint8_t *out, uint64_t cap, uint64_t *count);

/* ------------------------------------------------------------ learned cost model
 * A 3-layer perceptron predicting (log direct time, log reuse time) from
 * QW_MLP_IN planner features, used by the planner's reuse decision (with
 * the analytic Eq. (2) rule as fallback; results never depend on it).
 * Layout of the FP32 parameter array (QW_MLP_PARAMS floats, device memory):
 *   W1[12][64], b1[64], W2[64][64], b2[64], W3[64][2], b3[2]
 * (row-major; W[k][j] multiplies input k into output j), ReLU after the two
 * hidden layers. Every matrix product rounds both inputs to BF16 (round to
 * nearest even) and accumulates in FP32 on the matrix cores; everything else
 * is FP32. Inputs are x[B][12] (row-major), targets t[B][2]. All pointers
 * are device pointers; work is enqueued on the ctx stream; work must hold
 * qw_mlp_workspace_floats(B) floats. */
#define QW_MLP_IN 12
#define QW_MLP_WIDTH 64
#define QW_MLP_OUT 2
#define QW_MLP_PARAMS 5122
uint64_t qw_mlp_workspace_floats(uint32_t batch);
/* y[B][2] = MLP(x). */
int qw_mlp_forward(qw_ctx *ctx, const float *params, const float *x, uint32_t batch, float *work,
                   float *y);
/* grad = dL/dparams for L = 1/(2B) sum_{b,j} (y[b][j] - t[b][j])^2 (runs the
 * forward pass into work first). Batch reductions run in a fixed order. */
int qw_mlp_backward(qw_ctx *ctx, const float *params, const float *x, const float *target,
                    uint32_t batch, float *work, float *grad);
/* qw_mlp_backward on a gathered mini-batch: batch row b is row rows[b] of
 * x and target (rows: host array of `batch` indices, each below n_rows, the
 * row count of x and target; copied during the call). Indices out of range:
 * QW_E_INVALID_ARG, nothing enqueued. The same gradient as qw_mlp_backward
 * on the gathered rows. */
int qw_mlp_backward_rows(qw_ctx *ctx, const float *params, const float *x, const float *target,
                         uint32_t n_rows, const uint32_t *rows, uint32_t batch, float *work,
                         float *grad);
/* loss[0] (device double) = L = 1/(2B) sum_{b,j} (y[b][j] - t[b][j])^2 of
 * the forward pass on the batch (which runs into work first), summed in
 * FP64 in a fixed order. */
int qw_mlp_loss(qw_ctx *ctx, const float *params, const float *x, const float *target,
                uint32_t batch, float *work, double *loss);
/* One Adam step (step counts from 1) on all QW_MLP_PARAMS parameters. */
int qw_mlp_adam(qw_ctx *ctx, float *params, const float *grad, float *m, float *v, uint32_t step,
                float lr, float beta1, float beta2, float eps);

/* ------------------------------------------------------------ host-only */
/* Legality of continuing `src` on a target of kind `target_kind` and
 * backend family `target_backend` (Sec. IV-B, Table II). Returns QW_OK when
 * the continuation is EXACT, QW_E_REFUSED otherwise and then writes the
 * refusal JSON record (NUL-terminated, truncated to cap) into json_out.
 * No device is needed. */
int qw_legality_check(const qw_artifact *src, uint32_t target_kind,
                      uint32_t target_backend, char *json_out, uint64_t cap);

/* ------------------------------------------------------------ tableau */
/* Stabilizer tableau (the STAB rows of Table II): the state of a Clifford
 * circuit as 2n rows (destabilizers, then stabilizer generators) of X bits,
 * Z bits and a sign, updated gate by gate by the rules of Aaronson and
 * Gottesman (Phys. Rev. A 70, 052328, 2004). Host memory only; no device is
 * needed except for qw_tableau_export.
 * qw_tableau_create: |0...0> on n_qubits (1..30). */
typedef struct qw_tableau qw_tableau;
int qw_tableau_create(uint32_t n_qubits, qw_tableau **out);
int qw_tableau_free(qw_tableau *tb);
/* Apply Clifford gates (X Y Z H S SDG CNOT CZ) in order. Another kind gives
 * QW_E_UNSUPPORTED and leaves the tableau unchanged; bad qubits give
 * QW_E_INVALID_ARG. */
int qw_tableau_apply(qw_tableau *tb, const qw_gate *gates, uint64_t n_gates);
/* The 2n rows: x[i], z[i] (bit q = qubit q; X where only x is set, Z where
 * only z, Y where both) and sign r[i] (1 = minus); rows n..2n-1 are the
 * stabilizer generators. Host arrays of 2n entries each. */
int qw_tableau_rows(const qw_tableau *tb, uint64_t *x, uint64_t *z, uint8_t *r);
/* Artifact record of the tableau as a boundary state (Sec. IV-B: kind
 * TABLEAU, exactness EXACT, stabilizer-only backend family), for the
 * legality check of a continuation. */
int qw_tableau_artifact(const qw_tableau *tb, const uint8_t provenance[32], qw_artifact *out);
/* qw_tableau_export: the STAB -> SV conversion of Table II (exact): writes
 * the tableau's state into slot `slot` of `st` (same qubit count; slot not
 * frozen) as 2^n complex64 amplitudes. With the generators in reduced
 * echelon form on their X bits (r of them X-type) and x0 a basis state of
 * the support, the state is 2^{-r/2} sum_c (prod_{i: c_i} g_i)|x0>, so every
 * amplitude is 0 or 2^{-r/2} times a power of i; the global phase makes the
 * amplitude at x0 real and positive. One kernel, enqueued on the state's
 * context stream. */
int qw_tableau_export(const qw_tableau *tb, qw_state *st, uint32_t slot);

/* The claim schedule of a persistent launch (QW_OPT_PERSISTENT), host only,
 * for a tree of n_tasks tasks with parent[] as in qw_run_tree, n_passes[t]
 * passes per task, and per (task, pass), task-major, the pass structure
 * kinds[] and the units units[] it sweeps (tiles, a power of two), on grid
 * workgroups with at most chunk_max units per claim. Writes JSON to json_out
 * (NUL-terminated, at most cap bytes): {"claims": C, "segments": [[claim0,
 * n_claims, desc0, n_descs, chunk, kind, tmaj, units], ...], "deps": [[dep,
 * need], ...], "descs": [[task, pass], ...]}, deps and descs in claim order
 * (dep -1: none). A first pass reads its parent's state, every other pass
 * its task's own. The launch's progress argument rests on it: every
 * dependency is a descriptor of an earlier level, so its claims all come
 * before the claims that wait for it. QW_E_INVALID_ARG (with the reason in
 * json_out) for a parent that does not precede its child or has no passes,
 * units that are not powers of two, or a buffer too small. */
int qw_persist_schedule(uint32_t n_tasks, const int32_t *parent, const uint32_t *n_passes,
                        const uint32_t *kinds, const uint32_t *units, uint32_t chunk_max,
                        uint32_t grid, char *json_out, uint64_t cap);

/* Pass plan the library would execute for `gates` on n qubits, as JSON
 * (passes, local bit sets and fused operations), for inspection. No device
 * is needed. Returns QW_E_INVALID_ARG (message in json_out) for bad gates. */
int qw_plan_describe(uint32_t n_qubits, const qw_gate *gates, uint64_t n_gates,
                     uint32_t tile_bits, char *json_out, uint64_t cap);

/* Cost of `gates` on n qubits in the analytic byte model of the planner
 * (Sec. IV-C): the number of tile passes the library would run and the HBM
 * bytes they move (each pass reads and writes the state once: 2 * 8 * 2^n
 * bytes). No device is needed. A list with MEASURE or RESET is costed as
 * its segments (each planned alone, the projector folded into the next
 * segment's first pass, or one pass of its own if that segment is empty)
 * plus one read of the state (8 * 2^n bytes, no pass) per measurement. */
int qw_plan_cost(uint32_t n_qubits, const qw_gate *gates, uint64_t n_gates, uint32_t tile_bits,
                 uint64_t *n_passes, double *bytes);

/* Generate and compile (hipRTC) the pass kernels that QW_OPT_JIT would use
 * for `gates` on n qubits with at most tile_bits local bits per pass, and
 * keep the code objects in the process cache and the disk cache, without
 * loading them on a device: a warm-up for later runs, usable where there is
 * no GPU. States below 10 qubits need no generated kernels (QW_OK). On a
 * compile failure returns QW_E_HIP with the compiler log in log (truncated
 * to cap, NUL-terminated); QW_E_INVALID_ARG for bad gates. */
int qw_jit_precompile(uint32_t n_qubits, const qw_gate *gates, uint64_t n_gates,
                      uint32_t tile_bits, char *log, uint64_t cap);

/* Same for the generated expectation reducers of the Pauli terms (x, z)
 * (the term groups and register phases that qw_expect_pauli would use). */
int qw_jit_precompile_terms(uint32_t n_qubits, const uint64_t *x, const uint64_t *z,
                            uint32_t n_terms, uint32_t tile_bits, char *log, uint64_t cap);

/* Compile (hipRTC, no GPU needed) the generated kernels that
 * qw_run_suffix_batch uses for `gates` as the suffix of a batch of hot tasks
 * with the expectation epilogue x/z[n_terms]: the passes, the last pass with
 * its fused expectation epilogue when that applies (QW_OPT_FUSED_EPILOGUE),
 * and the reducers of the remaining terms. Same arguments, log and results
 * as qw_jit_precompile / qw_jit_precompile_terms. */
int qw_jit_precompile_suffix(uint32_t n_qubits, const qw_gate *gates, uint64_t n_gates,
                             const uint64_t *x_mask, const uint64_t *z_mask, uint32_t n_terms,
                             uint32_t tile_bits, char *log, uint64_t cap);

/* Generated-kernel counters of this process: kernels compiled, kernels taken
 * from the disk cache, and seconds spent compiling. Any pointer may be NULL. */
int qw_jit_stats(uint64_t *compiled, uint64_t *disk_hits, double *compile_seconds);

/* Library version string. */
const char *qw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QW_H */
