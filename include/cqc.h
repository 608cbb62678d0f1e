/* cqc.h - reconstruction of cut-circuit output distributions on AMD MI355X (gfx950).
 *
 * A circuit cut on K wires into n_C subcircuits is reconstructed from the
 * subcircuit "entry" tensors as the sum, over the 4^K Pauli label assignments
 * of the cut wires, of Kronecker products of entries, scaled by 2^-K
 * (Tang et al., CutQC, ASPLOS '21: Section 3.1 Eq. 1 for the per-cut Pauli
 * expansion and its factor 1/2, Section 3.2.3 for the term sum of one cut,
 * Section 3.3 for 4^K products with K cuts):
 *
 *     p(x) = 2^-K * sum_{l in {I,X,Y,Z}^K} prod_c E_c[ row_c(l), x_c ]
 *
 * Conventions shared by every entry point
 *   - Global output index: x = sum_q b_q 2^(n-1-q); qubit 0 is the most
 *     significant bit (the |q_0 ... q_{n-1}> notation of Section 3.2).
 *   - Entry tensor E_c: row-major [4^k_c][2^f_c], k_c = number of cuts incident
 *     to c, f_c = output qubits of c (Eq. 7).  Row digits: labels of the cuts
 *     incident to c in ascending cut id, first cut = most significant base-4
 *     digit, I=0, X=1, Y=2, Z=3.  Column x_c: local output bit j (j = 0 most
 *     significant) is global qubit out_qubit[sum_{c'<c} f_c' + j].
 *   - Every call is asynchronous on `stream` unless stated otherwise; device
 *     buffers must stay alive until the stream has executed the call.
 *   - All validation happens on the host before anything is enqueued: on any
 *     non-zero status nothing was launched and no output was touched.
 *   - The caller owns every buffer, including the workspace; the library keeps
 *     no device allocations of its own, except the fixed workspace array of
 *     cqc_reconstruct_fd_noalloc (CQC_NOALLOC_WORKSPACE_BYTES per GPU that
 *     loads the library, held until the process ends).
 *   - Values are never clamped: negative reconstructed probabilities (possible
 *     with finite-shot entries, Section 3.2.3) are returned as they are.
 *   - Early termination (Section 4.2): a label assignment whose factor row in
 *     some E_c is entirely +0/-0 may be skipped (it is where a step's term sum
 *     is long enough for the work to matter).  With finite entries this
 *     changes nothing; with Inf/NaN in another factor the skipped product
 *     would have been NaN.
 *   - Thread safety: functions are re-entrant; concurrent calls must use
 *     distinct workspaces.
 */
#ifndef CQC_H
#define CQC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
  CQC_OK = 0,
  CQC_ERR_INVALID_ARG = 1,  /* null pointer, bad enum, out-of-range id          */
  CQC_ERR_SHAPE = 2,        /* sum f_c != n, output order not a permutation, ... */
  CQC_ERR_UNSUPPORTED = 3,  /* valid but outside the implemented limits         */
  CQC_ERR_WORKSPACE = 4,    /* workspace missing or smaller than required       */
  CQC_ERR_HIP = 5           /* a HIP runtime call failed                        */
};

typedef enum { CQC_F32 = 0, CQC_F64 = 1 } cqc_dtype;

/* Arithmetic of the term sum.
 *   FP64:   double inputs (F32 inputs are widened exactly), FP64 MFMA, FP64 accumulate.
 *   FP32:   float operands, FP32 MFMA with FP32 accumulation; the total mass
 *           and DD bin masses are summed in FP64.
 *   BF16X6: each float operand split into three bfloat16 parts (a = a0+a1+a2),
 *           the six products a_i b_j with i+j <= 2 on BF16 MFMA with FP32
 *           accumulation (Henry, Tang, Heinecke, ARITH 2019).
 *   BF16X3: the speed end of the same split: two bfloat16 parts
 *           (a = a0+a1) and the three products a_i b_j with i+j <= 1; the
 *           dropped part and product leave up to 2^-15 of |a b| per product
 *           (about 3e-5 relative, above the FP32 forms' error).
 * Steps with at most 16 terms (<= 2 shared cuts) or a one-column operand
 * run the FP32 form under both split precisions.                        */
typedef enum { CQC_PREC_FP64 = 0, CQC_PREC_FP32 = 1, CQC_PREC_BF16X6 = 2, CQC_PREC_BF16X3 = 3 } cqc_precision;

/* Limits of this implementation. */
#define CQC_MAX_SUB 16        /* subcircuits per instance                      */
#define CQC_MAX_CUTS 24       /* cut wires per instance                        */
#define CQC_MAX_K_SUB 12      /* cuts incident to one subcircuit               */
#define CQC_MAX_FD_QUBITS 40  /* n for the full-definition output (2^n values) */
#define CQC_MAX_DD_QUBITS 128 /* n for dynamic definition                      */
#define CQC_MAX_F_SUB 30      /* output qubits of one subcircuit               */

/* Cut description (the problem statement of Sections 3 and 4.1: subcircuits,
 * cut wires with an upstream measured end u and a downstream initialised end v
 * (Figure 3), and the output qubit order).  All arrays are HOST memory. */
typedef struct {
  int32_t n_qubits;          /* n: output qubits of the uncut circuit             */
  int32_t n_sub;             /* n_C                                               */
  int32_t n_cuts;            /* K                                                 */
  const int32_t *f;          /* [n_sub] output qubits of each subcircuit (Eq. 7)  */
  const int32_t *edge_up;    /* [n_cuts] upstream (measured) subcircuit of cut e  */
  const int32_t *edge_down;  /* [n_cuts] downstream (initialised) subcircuit      */
  const int32_t *out_qubit;  /* [n_qubits] concatenated over c: local bit -> qubit*/
} cqc_cut;

typedef struct {
  cqc_cut cut;
  const void *const *entries; /* HOST array [n_sub] of DEVICE pointers, E_c as above */
  void *out;                  /* DEVICE: FD output [2^n] in the output dtype        */
  double *mass;               /* DEVICE [1] or NULL: FP64 sum of the written outputs */
} cqc_instance;

/* Full-definition reconstruction (Section 4.2 "FD query"): writes all 2^n
 * probabilities of every instance, each output element written exactly once,
 * and (if mass != NULL) their FP64 sum.  n_inst > 1 reconstructs a batch of
 * independent instances in one call.  in_t is the dtype of every entry
 * tensor, out_t the dtype of every output.  workspace: DEVICE buffer of at
 * least cqc_fd_workspace_size() bytes, 256-byte aligned. */
int cqc_fd_workspace_size(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                          cqc_dtype out_t, cqc_precision prec, size_t *bytes);
int cqc_reconstruct_fd(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                       cqc_dtype out_t, cqc_precision prec, void *workspace,
                       size_t ws_bytes, hipStream_t stream);

/* cqc_reconstruct_fd without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops and
 * harnesses that forbid allocation).  Same arguments, kernels, results and
 * error behaviour as cqc_reconstruct_fd; the workspace is instead a fixed
 * 256-byte-aligned device array inside the library, of
 * CQC_NOALLOC_WORKSPACE_BYTES on each GPU (the device that `stream` runs on;
 * the current device for the null stream).  This call allocates nothing:
 * no hipMalloc/hipFree and no allocating library routine.  Its device
 * address is looked up once per device on the first call there.
 *   - A call whose cqc_fd_workspace_size() exceeds the array fails with
 *     CQC_ERR_WORKSPACE before anything is enqueued.
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents; nothing in it needs to start at zero (every byte a
 *     call reads was written earlier in that call).  Calls that overlap on
 *     one GPU (several streams, or several host threads) race on it and give
 *     undefined results: serialise them.
 *   - n_inst > 1 takes the batched path, which uploads its tables into the
 *     array and synchronises `stream` once, as cqc_batch_create does. */
#define CQC_NOALLOC_WORKSPACE_BYTES ((size_t)32 << 20)
int cqc_reconstruct_fd_noalloc(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                               cqc_dtype out_t, cqc_precision prec, hipStream_t stream);

/* Prepared batches (the batched form of cqc_reconstruct_fd).  A batch of
 * independent instances of uneven n and K is reconstructed by a fixed, small
 * number of kernel launches: one row-flag pass over every entry tensor, one
 * persistent launch per group of contraction steps of equal kernel shape (all
 * instances' intermediate contractions first, then all final ones, each
 * group drained from a cost-ordered work queue) and one pass for every FP64
 * mass.
 * cqc_batch_create validates and plans the batch (n_inst >= 2, else
 * CQC_ERR_INVALID_ARG), writes its descriptor tables into `workspace` (at
 * least cqc_fd_workspace_size() bytes for the same instances, which must stay
 * allocated and unmodified by the caller while the batch exists) and
 * synchronises `stream` once.  Entry, output and mass
 * pointers are bound at creation.  The output dtype must be the precision's
 * (F32 for FP32, F64 for FP64).
 * cqc_batch_run enqueues only kernel launches, with no host synchronisation
 * and no allocation, so it may be captured into a HIP graph and replayed.
 * Runs of one batch on different streams must not overlap.
 * cqc_batch_destroy frees the host-side handle only. */
typedef struct cqc_batch_s *cqc_batch;
int cqc_batch_create(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                     cqc_precision prec, void *workspace, size_t ws_bytes, hipStream_t stream,
                     cqc_batch *out);
int cqc_batch_run(cqc_batch batch, hipStream_t stream);
int cqc_batch_destroy(cqc_batch batch);

/* A prepared batch whose final contraction steps also evaluate a
 * cross-entropy against a target distribution (the loss the adjoint below is
 * driven by; the paper itself trains nothing).  For every output p_x of
 * instance i and the target t_x at the same position (targets[i]: DEVICE
 * [2^n_i], output dtype, global output order) the kernel that computes p_x
 * writes
 *     grads[i][x] = -t_x / p_x if p_x > 1e-30, else 0
 * (DEVICE [2^n_i], output dtype) - bitwise what cqc_xent_grad gives for the
 * same p and t - so no separate pass over p is needed.  inst[i].out may be
 * NULL: p is then not written at all.  losses: HOST array of n_inst DEVICE
 * pointers, or NULL; losses[i] (if set) receives
 *     L_i = -sum_x t_x log max(p_x, 1e-30)
 * (logarithms in the output precision - FP32 outputs: about 1e-7 relative
 * per term, the size of p's own rounding - and the terms summed in FP64 in
 * the fixed order of the mass, so L_i is bitwise reproducible).  An instance with
 * a loss must have inst[i].mass NULL; without one, inst[i].mass works as in
 * cqc_batch_create.  grads[i] may equal targets[i] (each element is read
 * before it is overwritten); no other two of the buffers may overlap.  The
 * workspace size, cqc_batch_run, cqc_batch_destroy and
 * cqc_batch_backward_create (grad_out = grads) are those of the plain batch.
 * Errors: those of cqc_batch_create; CQC_ERR_INVALID_ARG for NULL targets or
 * grads arrays or entries, or a loss together with a mass. */
int cqc_batch_create_xent(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                          cqc_precision prec, const void *const *targets, void *const *grads,
                          double *const *losses, void *workspace, size_t ws_bytes, hipStream_t stream,
                          cqc_batch *out);

/* Adjoint of a prepared batch (the gradient of Section 3.2.3's linear map;
 * the paper has no gradients): for every instance i, dL/dE_c for each entry
 * tensor from dL/dp, in a fixed small number of launches.  The forward
 * operands are the converted entries and intermediate tensors that the
 * batch's last cqc_batch_run left in the batch's workspace: a run must follow
 * a cqc_batch_run of the same batch on the same stream, with that workspace
 * unmodified in between.
 * grad_out[i]: DEVICE [2^n_i] dL/dp in global output order, dtype of the
 * batch's outputs.  grad_entries[i][c]: DEVICE, layout and dtype of instance
 * i's entry tensor c; every element is written (no accumulation).  Both are
 * bound at creation, like the batch's pointers.
 * cqc_batch_backward_create plans every instance's adjoint steps, writes its
 * tables into `workspace` (at least cqc_batch_backward_workspace_size()
 * bytes, 256-byte aligned, separate from the batch's, kept allocated and
 * unmodified while the handle exists) and synchronises `stream` once.
 * cqc_batch_backward_run enqueues only kernel launches (no host
 * synchronisation, no allocation), so it may be captured into a HIP graph
 * together with cqc_batch_run.  Results are bitwise reproducible (split-K
 * partials are added in a fixed order).  An FP64 batch runs the FP64 adjoint;
 * FP32 and split-BF16 batches run the FP32 one.
 * cqc_batch_backward_destroy frees the host-side handle only. */
typedef struct cqc_batch_bwd_s *cqc_batch_bwd;
int cqc_batch_backward_workspace_size(cqc_batch batch, size_t *bytes);
int cqc_batch_backward_create(cqc_batch batch, const void *const *grad_out,
                              void *const *const *grad_entries, void *workspace, size_t ws_bytes,
                              hipStream_t stream, cqc_batch_bwd *out);
int cqc_batch_backward_run(cqc_batch_bwd b, hipStream_t stream);
int cqc_batch_backward_destroy(cqc_batch_bwd b);

/* On-device entry construction (Sections 3.1-3.2): the entry tensor E_c of a
 * subcircuit from the measured distributions of its variants - the outgoing
 * cuts' labels pick the measurement bases and weight the measured cut bits,
 * the incoming cuts' labels combine the initialisations; several cuts
 * multiply.  form CQC_FORM_PAULI (Eq. 1 and Eq. 3), labels I, X, Y, Z:
 * measured bits +1/+1 (I) or +1/-1 (X, Y, Z; I and Z share the computational
 * basis); initialisations I: q0 + q1, X: 2 q+ - q0 - q1, Y: 2 q+i - q0 - q1,
 * Z: q0 - q1.  form CQC_FORM_EIGEN (Eq. 2), labels A1..A4: measured bits 2/0
 * (A1) and 0/2 (A2) in the computational basis, +1/-1 in the X (A3) and Y
 * (A4) bases; initialisations A1: q0, A2: q1, A3: 2 q+ - q0 - q1, A4: 2 q+i -
 * q0 - q1.  Both forms reconstruct the same distribution when every
 * subcircuit of an instance uses the same form; the eigen form has the
 * smaller term magnitudes.
 *   f         output qubits of the subcircuit (2^f columns), 0 <= f <= 30
 *   n_cuts    incident cuts k = k_in + k_out; k_in <= 3, k_out <= 4
 *   cut_kind  (host)[n_cuts]: the incident cuts in ascending cut id, 0 if the
 *             subcircuit initialises the cut qubit (incoming), 1 if it
 *             measures it (outgoing)
 *   variants  DEVICE [4^k_in][3^k_out][2^f][2^k_out], dtype in_t: for every
 *             initialisation combination (per incoming cut, in cut_kind's
 *             order: 0 |0>, 1 |1>, 2 |+>, 3 |+i>; first the most significant
 *             base-4 digit) and measurement-basis combination (per outgoing
 *             cut: 0 computational, 1 X, 2 Y; first the most significant
 *             base-3 digit), the probability or normalised shot count of
 *             every output bit string x (local order, first qubit the most
 *             significant bit) and measured cut-bit string (first outgoing
 *             cut the most significant bit)
 *   entries   DEVICE [4^k][2^f], dtype out_t, written in full: the layout
 *             cqc_reconstruct_fd takes (row = base-4 number of the labels
 *             - I=0, X=1, Y=2, Z=3, or A1..A4 = 0..3 - of the incident cuts
 *             in ascending cut id)
 *   form      cqc_entry_form
 * Sums are accumulated in FP64 and rounded once to out_t.  n_jobs launches,
 * one per job, on `stream`; no workspace, no synchronisation (graph-
 * capturable).  Validation (dtypes, sizes, cut_kind values, NULL pointers)
 * happens for every job before the first launch. */
typedef enum { CQC_FORM_PAULI = 0, CQC_FORM_EIGEN = 1 } cqc_entry_form;
typedef struct {
  int32_t f;
  int32_t n_cuts;
  const int32_t *cut_kind;
  const void *variants;
  void *entries;
  int32_t form;   /* cqc_entry_form */
} cqc_entry_job;
int cqc_build_entries(const cqc_entry_job *jobs, int32_t n_jobs, cqc_dtype in_t, cqc_dtype out_t,
                      hipStream_t stream);

/* Chi-square distance of two distributions (Eq. 16): *out = sum over i < n
 * with a_i + b_i > 0 of (a_i - b_i)^2 / (a_i + b_i), every term in FP64.
 * a, b: DEVICE [n] in dtypes a_t, b_t (e.g. a reconstruction against a
 * reference, or two DD bin landscapes).  out: DEVICE, one FP64.  workspace:
 * DEVICE, at least 8192 bytes (per-block partials), 8-byte aligned.  Two
 * launches on `stream`, no synchronisation; the addition order depends only
 * on n (not on the alignment of a and b), so the result is bitwise
 * reproducible.  n = 0 writes 0.  Errors: CQC_ERR_INVALID_ARG for an unknown
 * dtype, n < 0, NULL out, or NULL a / b with n > 0; CQC_ERR_WORKSPACE for a
 * missing or short workspace. */
int cqc_chi2(const void *a, cqc_dtype a_t, const void *b, cqc_dtype b_t, int64_t n, double *out,
             void *workspace, size_t ws_bytes, hipStream_t stream);

/* Cross-entropy of reconstructed outputs p against a target distribution t,
 * and its gradient, in one pass (the loss that drives the adjoint below):
 *     loss = -sum_x t_x log max(p_x, 1e-30)     (FP64, if loss != NULL)
 *     grad_x = -t_x / p_x if p_x > 1e-30, else 0 (the floor is flat)
 * p, t, grad: DEVICE [n] of dtype dt (grad may alias neither p nor t); the
 * floor test is made on p widened to FP64, the division in dt.  Flat buffers
 * of many instances' outputs are one call.  loss: DEVICE, one FP64, or NULL;
 * with a loss the workspace (DEVICE, >= 8192 bytes, 8-byte aligned) holds
 * per-block partials added in a fixed order (bitwise reproducible for a given
 * n).  One or two launches on `stream`.  Errors: CQC_ERR_INVALID_ARG for an
 * unknown dtype, n < 0 or NULL buffers with n > 0; CQC_ERR_WORKSPACE for a
 * loss without enough workspace. */
int cqc_xent_grad(const void *p, const void *t, cqc_dtype dt, int64_t n, void *grad, double *loss,
                  void *workspace, size_t ws_bytes, hipStream_t stream);

/* Dynamic definition (Algorithm 1, Section 4.3).
 * Recursion 1 makes `first_active` (or, if NULL, the first n_active qubits in
 * output order) active; every later recursion refines one bin produced so far
 * that is not yet expanded and still contains merged qubits (a candidate):
 * it zooms the bin's recursion's active qubits to the bin's bits and makes
 * the next n_active un-zoomed qubits in output order active.  Merged qubits
 * are summed out of the entries (FP64 accumulation) before the term sum.  Bin
 * b of a recursion has its active qubits (ascending id) as bits, first = most
 * significant.  Stops early when no candidate is left.
 * Which candidate (Section 4.3 names a depth-first search for sparse outputs
 * and a breadth-first one for dense outputs):
 *   CQC_DD_HEAVIEST  the largest FP64 mass over all recursions (Algorithm 1);
 *                    ties: lowest recursion, then lowest bin index.
 *   CQC_DD_DFS       the heaviest candidate of the most recent recursion that
 *                    has one (a single-state recursion sends the search back
 *                    up); ties: lowest bin index.  With several bins per
 *                    round: the latest round, and in it the earliest pick.
 *   CQC_DD_BFS       the heaviest candidate of the shallowest zoom depth that
 *                    has one; ties: lowest recursion, then lowest bin index.
 * Rounds: each round picks up to bins_per_round candidates, in the strategy's
 * order, from the recursions that existed when the round began (limited to
 * the first pick's depth for BFS and to its recursion for DFS; a round whose
 * candidates run out ends early), then runs all of them.  bins_per_round = 1
 * is the one-bin-per-recursion search; BFS gives the same records for every
 * bins_per_round.
 * This call is host-driven: it synchronises `stream` once per round (and once
 * per extra candidate refill) and returns after the last recursion completed.
 * For that per-round read-back of the selected bins the library keeps a small
 * pool of page-locked host buffers (hipHostMalloc, about 9 KiB each: 64
 * slots of 8 ranked bins and a mass; one per concurrently running query,
 * reused and held until the process ends); if page-locked memory cannot be
 * had, pageable memory is used with the same results. */
typedef enum { CQC_DD_HEAVIEST = 0, CQC_DD_DFS = 1, CQC_DD_BFS = 2 } cqc_dd_strategy;

typedef struct {
  int32_t n_active;          /* a: active qubits per recursion, 1..36            */
  int32_t n_recursions;      /* R >= 1                                            */
  const int32_t *first_active; /* HOST [n_active] or NULL                         */
  int32_t strategy;          /* cqc_dd_strategy                                   */
  int32_t bins_per_round;    /* 0..64; 0 means 1                                  */
  int32_t bins_f32;          /* 0: FP64 bins; 1: FP32 bins (half the memory: one
                                recursion of 2^35 bins is 128 GiB); masses, the
                                selection and the merge stay FP64            */
} cqc_dd_params;

typedef struct {
  int32_t parent_rec;        /* -1 for recursion 1                                */
  int32_t n_active;          /* active qubits of this recursion (<= a)            */
  int64_t parent_bin;        /* bin of parent_rec that this recursion refines     */
  double mass;               /* FP64 sum of this recursion's bins                 */
  int8_t role[CQC_MAX_DD_QUBITS]; /* per qubit: -2 active, -1 merged, 0/1 zoomed  */
} cqc_dd_record;

int cqc_dd_workspace_size(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                          const cqc_dd_params *p, size_t *bytes);
/* bins: DEVICE [n_recursions][2^n_active], FP64 (or FP32 with bins_f32),
 * rows past the last recursion are not written; records: HOST [n_recursions];
 * n_done: HOST, recursions run.  inst->out and inst->mass are ignored.  With
 * FP32 bins the candidates are ranked on the stored FP32 values (widened
 * exactly) and each record's mass is the FP64 sum of its stored bins. */
int cqc_reconstruct_dd(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                       const cqc_dd_params *p, void *bins, cqc_dd_record *records,
                       int32_t *n_done, void *workspace, size_t ws_bytes,
                       hipStream_t stream);

/* Device-resident dynamic definition: the same search as cqc_reconstruct_dd
 * (Algorithm 1, Section 4.3; same bins, records and masses, bit for bit) with
 * every decision taken on the device, so a query enqueues all its recursions
 * without a host round trip and can be captured in a HIP graph and replayed.
 * Each recursion's bin is picked by a kernel from per-recursion windows of
 * the best not-yet-expanded bins that top-T passes keep in the query state;
 * a window that runs out is refilled on the device.  One bin is expanded per
 * recursion: bins_per_round must be 0 or 1 (CQC_ERR_UNSUPPORTED otherwise).
 * cqc_dd_query_create validates and plans the query, binds the entries,
 * `bins` (DEVICE, as for cqc_reconstruct_dd), `records` (DEVICE
 * [n_recursions]) and `n_done` (DEVICE, one int32: the recursions run), writes
 * its tables into `workspace` (DEVICE, at least cqc_dd_query_workspace_size()
 * bytes, 256-byte aligned, kept allocated and unmodified while the query
 * exists) and synchronises `stream` once.
 * cqc_dd_query_run enqueues one complete query (only kernel launches: no
 * synchronisation, no allocation, no host read); records past n_done are
 * not written.  Runs of one query on different streams must not overlap.
 * cqc_dd_query_run_range enqueues recursions [first, first + count) only:
 * first = 0 starts a new search; first > 0 resumes the search the query's
 * workspace holds after recursion first - 1 (the bins, records and query
 * state left by earlier runs of this query must be unmodified), so a search
 * can be run in pieces and inspected in between with results equal to one
 * run.  Resuming a search that stopped early runs nothing.
 * cqc_dd_query_destroy frees the host-side handle only. */
typedef struct cqc_dd_query_s *cqc_dd_query;
int cqc_dd_query_workspace_size(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                                const cqc_dd_params *p, size_t *bytes);
int cqc_dd_query_create(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                        const cqc_dd_params *p, void *bins, cqc_dd_record *records, int32_t *n_done,
                        void *workspace, size_t ws_bytes, hipStream_t stream, cqc_dd_query *out);
int cqc_dd_query_run(cqc_dd_query q, hipStream_t stream);
int cqc_dd_query_run_range(cqc_dd_query q, int32_t first, int32_t count, hipStream_t stream);
int cqc_dd_query_destroy(cqc_dd_query q);

/* Adjoint of the FD build: given G = dL/dp (DEVICE [2^n] per instance, dtype
 * in_t), writes dL/dE_c for every subcircuit (DEVICE, same layout and dtype
 * as E_c):
 *     dL/dE_c[r, y] = 2^-K sum_{l: row_c(l)=r} sum_{x: x_c=y} G[x] prod_{c'!=c} E_c'[row_c'(l), x_c']
 * Every output element is written (not accumulated).  Reductions run in a
 * fixed order, so results are bitwise reproducible.  F32 arithmetic: FP32
 * accumulation throughout; the products of steps with three or four shared
 * cuts (inner extent of at least 16) run as the six-product BF16X6 split
 * (above), whose products keep FP32 accuracy (dropped terms below 2^-24 of
 * |a b|). */
int cqc_backward_workspace_size(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                                cqc_precision prec, size_t *bytes);
int cqc_reconstruct_backward(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                             cqc_precision prec, const void *const *grad_out,
                             void *const *const *grad_entries, void *workspace,
                             size_t ws_bytes, hipStream_t stream);

/* Eq. 14 of Section 4.1.4 for one instance, with subcircuits taken in the
 * greedy smallest-first order of Section 4.2: 4^K * sum_{c>=2} prod_{i<=c} 2^f_i
 * multiplications.  Also returns the multiply-adds of this library's plan. */
int cqc_cost(const cqc_cut *cut, double *eq14_mults, double *plan_macs);

/* Tile autotuner: times the candidate tile shapes of every contraction the
 * instance needs (on `stream`, synchronously), keeps the fastest per shape
 * class in a process-wide cache, and persists the cache to the file named by
 * the CQC_TUNE_CACHE environment variable if set.  Outputs are clobbered. */
int cqc_autotune(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                 cqc_dtype out_t, cqc_precision prec, void *workspace,
                 size_t ws_bytes, hipStream_t stream);
/* Clears the process-wide tile cache; the next plan that consults it reloads
 * the file named by CQC_TUNE_CACHE (if set).  Host only; not to be called
 * while another thread plans or tunes. */
int cqc_tune_reset(void);

/* Kernel tracing: when enabled, every kernel the library launches is
 * bracketed by HIP events on its stream; cqc_trace_read reports, per kernel
 * name, the launch count and the summed event time (ms), and resets. */
int cqc_trace_enable(int on);
int cqc_trace_read(char *names, size_t names_len, int32_t *counts, double *ms,
                   int32_t max_kernels, int32_t *n_kernels);

const char *cqc_status_string(int status);
const char *cqc_last_error_detail(void); /* thread-local, of the last failing call */
int cqc_version(void);

/* Self test of the MFMA operand/accumulator lane layouts the kernels assume:
 * runs one 16x16x4 FP32, one 16x16x4 FP64 and one 16x16x32 BF16 matrix-core
 * product on known operands (DEVICE out: 256 floats, 256 doubles, 256 floats:
 * 4096 bytes) and returns CQC_OK if launched. */
int cqc_selftest_mfma(void *out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* CQC_H */
