/*
 * mps_dmrg.h -- C ABI of the MI355X (gfx950) DMRG compression-step library.
 *
 * The library keeps a matrix product state (MPS) of n qubits, one qubit per
 * tensor, on one GPU and applies circuit layers to it with the compression
 * step of Ayral et al., "A density-matrix renormalization group algorithm for
 * simulating quantum circuits with a finite fidelity" (Sec. IV.B): the layer
 * is written as an MPO, a TEBD-like zip-up gives the initial guess, and
 * alternating two-site sweeps fit a bond-chi MPS to W|psi>, each local update
 * being F / sqrt(f) (eq:optimization) split back by a truncated SVD that keeps
 * the chi largest singular values (Sec. VI.A).  The partial fidelities f_delta
 * multiply into F~ (eq:Ftilde-sup).
 *
 * Conventions
 *   - Sites are chain positions 0..n-1; the caller applies any qubit -> site
 *     map.  Statevector index x = sum_k s_k 2^(n-1-k) (site 0 most
 *     significant), i.e. the tensor index order of the paper's Psi_{i1..iN}.
 *   - Bond k lies left of site k; bond 0 and bond n have dimension 1.
 *   - Complex numbers crossing the ABI are interleaved (re, im) doubles.
 *   - All pointers in this header are HOST pointers unless stated otherwise;
 *     every call copies what it needs and is synchronous with respect to the
 *     host: when it returns, output buffers are filled and input buffers may
 *     be reused.  Device work runs on the HIP stream given to mps_create.
 *   - A state is not thread-safe.  Distinct states may be used from distinct
 *     threads on distinct streams.
 *
 * Errors
 *   Every entry point returns an mps_status.  MPS_OK is 0, errors are
 *   negative; mps_last_error() returns a thread-local message describing the
 *   last error.  Argument errors (MPS_ERR_ARG) leave the state unchanged.
 *   Device, allocation or numerical failures inside apply_layer_dmrg mark the
 *   state invalid; every later call on it returns MPS_ERR_STATE.
 */
#ifndef MPS_DMRG_H
#define MPS_DMRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mps_state mps_state;

typedef enum {
    MPS_OK = 0,
    MPS_ERR_ARG = -1,     /* invalid argument; state unchanged               */
    MPS_ERR_OOM = -2,     /* device allocation failed                        */
    MPS_ERR_DEVICE = -3,  /* HIP / rocSOLVER error                           */
    MPS_ERR_NUMERIC = -4, /* non-finite or zero norm, fidelity out of range  */
    MPS_ERR_STATE = -5    /* the state was invalidated by an earlier failure */
} mps_status;

/* Arithmetic of the environment and local-tensor contractions.  The
 * truncation (Gram matrix, Hermitian eigensolver), the fidelity bookkeeping
 * and the stored MPS tensors are FP64 in every mode. */
typedef enum {
    MPS_FP64 = 0,   /* complex FP64 contractions on FP64 MFMA                  */
    MPS_FP32 = 1,   /* complex FP32 contractions on FP32 MFMA, FP32 environments */
    MPS_BF16X2 = 2, /* split precision: FP32 operands as two BF16 terms (hi, lo),
                       three BF16 MFMA products per real product (hh, hl, lh),
                       FP32 accumulation (relative error about 2^-16),
                       FP32 environments                                      */
    MPS_BF16X3 = 3  /* split precision: FP32 operands as three BF16 terms, six
                       BF16 MFMA products per real product, FP32 accumulation
                       (about FP32 accuracy), FP32 environments            */
} mps_precision;

/* Device-memory callbacks (optional, see mps_create).  alloc returns at least
 * `bytes` bytes of device memory of the state's GPU, aligned to 256 bytes,
 * usable in stream order on `stream` (a hipStream_t), or NULL on failure;
 * free releases a pointer alloc returned, in stream order on `stream`.  The
 * library calls them from the thread that makes the library call (for
 * apply_layer_dmrg_batched: from its worker threads, so they must be
 * thread-safe) and frees every block before mps_destroy returns.  `user` is
 * passed through.  The struct is copied by mps_create. */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, void* stream, void* user);
    void* user;
} mps_allocator;

/* One gate.  q1 = -1 for a one-qubit gate.  m holds the matrix as interleaved
 * complex128, row-major with rows = output and columns = input:
 *   one-qubit: 2x2 in m[0..7];
 *   two-qubit: 4x4 in m[0..31], row/column index 2*s_q0 + s_q1.
 * Within one layer every one-qubit gate acts before every two-qubit gate
 * (the cycle structure of Sec. V.A); one-qubit gates on the same site compose
 * in array order; two-qubit gates must act on disjoint sites; q0 > q1 is
 * allowed. */
typedef struct {
    int32_t q0;
    int32_t q1;
    double m[32];
} mps_gate;

/* Create the product state |x> (Sec. IV.A: an MPS of bond dimension 1).
 *   n_sites    number of sites, 1 <= n_sites <= 4096.
 *   init_bits  n_sites bytes, each 0 or 1; NULL means |0...0>.
 *   max_chi    largest bond dimension any later call may request (>= 1);
 *              used for argument checks only.
 *   precision  an mps_precision value.
 *   hip_stream hipStream_t to run on (NULL = the default stream).
 *   alloc      device-memory callbacks for every buffer the state and its
 *              calls use (e.g. a framework's caching allocator); NULL =
 *              hipMallocAsync / hipFreeAsync on the call's stream from the
 *              device's default memory pool.  Both function pointers must be
 *              non-NULL (MPS_ERR_ARG otherwise).
 *   out        receives the new state; the caller releases it with
 *              mps_destroy.  The state owns all of its device memory. */
mps_status mps_create(int n_sites, const uint8_t* init_bits, int max_chi,
                      int precision, void* hip_stream, const mps_allocator* alloc,
                      mps_state** out);

/* Release a state and all device memory it owns, after its streams have
 * drained: its buffers (through its allocator), its rocBLAS handle, its second
 * stream and its events.  Memory the default pool keeps cached is returned to
 * the device.  NULL is accepted. */
mps_status mps_destroy(mps_state* state);

/* One compression step (Sec. IV.B with K = 1): replace |psi> by the bond-chi
 * MPS |phi> that maximises |<phi|U|psi>|^2, U being the layer given by
 * `gates`.  The initial guess is a zip-up of the layer's MPO into |psi>
 * starting at the end of the chain that holds the orthogonality centre; then
 * n_sweeps two-site sweeps alternate direction.  Each local update keeps
 * chi' = min(chi, #{S_i^2 > 1e-12 sum_j S_j^2}) singular values of the
 * two-site tensor F and normalises it (eq:optimization); f = sum of the kept
 * S^2.  f_layer (may be NULL) receives f_delta, the f of the last update
 * (eq:fa-sup), which is also multiplied into F~.
 *   gates     n_gates records (see mps_gate), host memory, copied.
 *   chi       1 <= chi <= max_chi.
 *   n_sweeps  >= 0 (0 = zip-up only).
 * On error the state is unchanged for MPS_ERR_ARG, and invalid otherwise. */
mps_status apply_layer_dmrg(mps_state* state, const mps_gate* gates, int n_gates,
                            int chi, int n_sweeps, double* f_layer);

/* The compression step with single-site sweeps (the update rule of Sec. IV.B
 * with one free tensor, eq:optimization): the same zip-up as
 * apply_layer_dmrg (which fixes the bond dimensions, at most chi), then
 * n_sweeps passes in alternating directions over all n sites.  At site j
 * the local tensor F_j = L_{j-1} A_j W_j R_{j+1} is computed, f = |F_j|^2,
 * M = F_j / sqrt(f), and the orthogonality centre moves on by an FP64 QR of
 * M (its column space is kept: bond dimensions only shrink where a site has
 * fewer rows than columns).  f_layer receives the f of the last site of the
 * last pass.  Arguments, ownership and errors as for apply_layer_dmrg. */
mps_status apply_layer_dmrg_single_site(mps_state* state, const mps_gate* gates, int n_gates,
                                        int chi, int n_sweeps, double* f_layer);

/* Update rules of apply_layers_dmrg. */
typedef enum {
    MPS_UPDATE_TWO_SITE = 0,    /* the sweeps of apply_layer_dmrg            */
    MPS_UPDATE_SINGLE_SITE = 1  /* the sweeps of apply_layer_dmrg_single_site */
} mps_update;

/* One compression step over K = n_layers consecutive layers (Sec. IV.B with
 * K > 1; the contraction strategy of Sec. IV.B.2 with K layers between the two
 * MPS): |phi> maximises |<phi|U_K ... U_1|psi>|^2 over bond-chi MPS.  The MPO
 * of the step is the product of the K layer MPOs: its bond c carries the
 * operator-Schmidt indices of every two-qubit gate of any of the K layers
 * with min site < c <= max site, so its bond dimensions are the products of
 * the K layers' (at most 2^24).  Zip-up, sweeps, truncation and f_step are
 * those of the update rule; F~ is multiplied by the one f_step, and the layer
 * count of `fidelity` grows by K.  K = 1 is apply_layer_dmrg (update 0) or
 * apply_layer_dmrg_single_site (update 1).
 *   gates     the records of layer 1, then layer 2, ... (sum of n_gates
 *             records, host memory, copied); each layer obeys the rules of
 *             mps_gate (one-qubit gates act first, disjoint two-qubit gates).
 *   n_gates   K host ints, the record count of each layer (>= 0).
 *   n_layers  K, 1 <= K <= 64.
 *   update    an mps_update value.
 *   chi, n_sweeps, f_step as chi, n_sweeps, f_layer of apply_layer_dmrg.
 * On error the state is unchanged for MPS_ERR_ARG, and invalid otherwise. */
mps_status apply_layers_dmrg(mps_state* state, const mps_gate* gates, const int* n_gates,
                             int n_layers, int chi, int n_sweeps, int update, double* f_step);

/* apply_layers_dmrg with a cap per bond instead of one chi: every truncation
 * of bond c (between sites c-1 and c) keeps
 * min(chi_bond[c], #{S_i^2 > 1e-12 sum_j S_j^2}) values.  A grouping of the
 * qubits into tensors (Sec. IV.A with r_tau > 1, Sec. V.C) is the profile
 * that caps the bonds between groups at chi and leaves the bonds inside a
 * group uncapped: an MPS of grouped tensors with bond chi is an MPS of single
 * qubits with exactly those bond limits, and a layer whose gates stay inside
 * the groups is applied with f_delta = 1 at any chi.
 *   chi_bond  n_sites + 1 host ints; entries 1 .. n_sites - 1 must be in
 *             [1, max_chi] (the two end bonds are 1 and their entries are
 *             ignored).
 * Other arguments, ownership and errors as for apply_layers_dmrg. */
mps_status apply_layers_dmrg_bonds(mps_state* state, const mps_gate* gates, const int* n_gates,
                                   int n_layers, const int* chi_bond, int n_sweeps, int update,
                                   double* f_step);

/* Apply one layer to each of `batch` independent states (the compression
 * step above, per instance), concurrently: instances are driven by up to 8
 * host threads and run on their own streams, so give every state its own
 * stream in mps_create for the work to overlap (states sharing a stream are
 * still correct, only serialised).
 *   states   batch distinct state handles.
 *   gates    batch host pointers; gates[i] holds n_gates[i] records.
 *   chi      batch bond dimensions, 1 <= chi[i] <= max_chi of state i.
 *   f_layers batch outputs (may be NULL): f_delta of each instance.
 * The persistent tridiagonal reductions of the instances' truncations (orders
 * 129..2048) that the threads reach within about 1 ms of each other run in one
 * shared cooperative launch (up to 8 instances, 256 workgroups in total):
 * the reduction is latency-bound and an order-n matrix occupies only n / 8
 * workgroups, so concurrent instances fill the chip together.
 * Arguments of all instances are checked before any device work
 * (MPS_ERR_ARG leaves every state unchanged).  If an instance fails, the
 * first failing instance's status is returned with its message; that state
 * is invalid, the others have completed their layer. */
mps_status apply_layer_dmrg_batched(mps_state* const* states, int batch,
                                    const mps_gate* const* gates, const int* n_gates,
                                    const int* chi, int n_sweeps, double* f_layers);

/* Shared tridiagonal-reduction launches of apply_layer_dmrg_batched since the
 * library was loaded (*launches) and the reductions they carried
 * (*reductions); either pointer may be NULL. */
mps_status mps_batch_stats(int64_t* launches, int64_t* reductions);

/* The fidelity estimate F~ = prod_delta f_delta (eq:Ftilde-sup), its natural
 * logarithm, the number of layers applied and the number of two-qubit gates
 * N_2g applied; the error per gate is eps~ = 1 - F~^(1/N_2g).  Any output
 * pointer may be NULL. */
mps_status fidelity(const mps_state* state, double* F_tilde, double* log_F_tilde,
                    int* n_layers, int64_t* n_2q_gates);

/* Draw n_samples bitstrings from |phi(x)|^2 by exact sequential sampling from
 * the orthogonality centre outwards (weak simulation, Sec. II.C).  The uniform
 * number of sample j at site k is a Philox-4x32-10 draw (Salmon et al., SC'11)
 * keyed by (seed_lo, seed_hi) with counter (k, j_lo, j_hi, 0x5A4D5053), its
 * words 0 and 1 forming a 53-bit fraction; site k takes 0 when the fraction is
 * below p(0 | earlier sites).
 *   bits  host array of n_samples * ceil(n/64) uint64 words; bit (k % 64) of
 *         word (j * ceil(n/64) + k / 64) is the value of site k in sample j. */
mps_status sample(mps_state* state, int64_t n_samples, uint64_t seed, uint64_t* bits);

/* Thread-local description of the last error ("" if none). */
const char* mps_last_error(void);

/* ---- inspection (parity tests, analysis) -------------------------------- */

/* Amplitudes <x|phi> for n_strings bitstrings (n_strings * n bytes, 0/1),
 * evaluated in FP64 on the device; re_im receives 2 * n_strings doubles. */
mps_status mps_amplitude(const mps_state* state, int n_strings, const uint8_t* bits,
                         double* re_im);

/* The full statevector (n <= 26) in FP64: 2 * 2^n doubles, index as above. */
mps_status mps_to_statevector(const mps_state* state, double* re_im);

/* Bond dimensions: n + 1 ints. */
mps_status mps_bond_dims(const mps_state* state, int* dims);

/* Copy of site tensor A_site, shape (D_site, 2, D_site+1), row-major, as
 * interleaved complex128. */
mps_status mps_get_tensor(const mps_state* state, int site, double* re_im);

/* Per-update log of all layers applied so far, oldest first: partial fidelity
 * f, sum of all squared singular values of the local tensor, and the number
 * of singular values kept.  The zip-up of each layer logs one entry (f = its
 * final norm squared).  At most `cap` entries are written; *n receives the
 * total number available. */
mps_status mps_step_log(const mps_state* state, double* f, double* sum_s2,
                        int* chi_kept, int cap, int* n);

/* Conditioning of the truncations, one entry per applied step (call of
 * apply_layer_dmrg, apply_layers_dmrg, ... or one instance's layer in the
 * batched call), oldest first: the smallest separation
 * (lambda_k - lambda_{k+1}) / lambda_1 of the Gram eigenvalues (squared
 * singular values, Sec. VI.A) over the step's truncations where chi limited
 * the kept count (more than chi eigenvalues above the relative threshold
 * 1e-12); HUGE_VAL when chi limited none.  A separation near
 * rounding marks a cut inside a (nearly) degenerate set of singular values,
 * where the kept subspace is not unique.  At most `cap` entries are written;
 * *n receives the total. */
mps_status mps_cut_separations(const mps_state* state, double* sep, int cap, int* n);

/* How the truncations of this state were diagonalised since it was created:
 *   counts[0]  persistent multi-workgroup tridiagonal reduction (orders 129..2048);
 *   counts[1]  single-workgroup tridiagonal reduction (orders 2..128);
 *   counts[2]  fallbacks: rocSOLVER's dense solver after the persistent reduction
 *              was refused a cooperative launch or gave up waiting;
 *   counts[3]  rocSOLVER's dense solver by choice (order above 2048, order 1, or
 *              MPS_EIGENSOLVER=rocsolver).
 * counts: 4 host int64.  A truncation whose eigenvalues or kept eigenvectors
 * are not finite fails the call with MPS_ERR_NUMERIC instead. */
mps_status mps_eigensolver_counts(const mps_state* state, int64_t* counts);

/* <phi| Z_i Z_j |phi> (or <Z_i> when i == j) in FP64. */
mps_status mps_expect_zz(const mps_state* state, int i, int j, double* value);

/* <bra|ket> in FP64 (MPS-MPS overlap; the closed simulation mode of
 * Sec. IV.C contracts a forward and a backward MPS this way).  Both states
 * must have the same number of sites; neither is modified.  The bra's stream
 * is synchronised first; the work runs on the ket's stream and is complete
 * on return.  re, im: HOST outputs. */
mps_status mps_overlap(const mps_state* bra, const mps_state* ket, double* re, double* im);

/* <bra| U_K ... U_1 |ket> with the K = n_layers layers contracted exactly
 * between the two states: the closed simulation mode's middle part of depth
 * D2 (Sec. IV.C), between the backward MPS (bra) and the forward MPS (ket).
 * The layers follow the rules of apply_layers_dmrg (gates of layer 1, then
 * layer 2, ...; n_gates[l] records each; one-qubit gates act first in each
 * layer); they form the same MPO as a K-layer compression step, contracted
 * site by site as E_{k+1} = B_k^H (E_k A_k W_k) in FP64 (nothing truncated).
 * n_layers = 0 is mps_overlap.  MPS_ERR_ARG when an environment
 * D_bra x (MPO bond) x D_ket would exceed 2^31 complex values.  Neither state
 * is modified; the bra's stream is synchronised first and the work runs on the
 * ket's stream, complete on return.  re, im: HOST outputs. */
mps_status mps_overlap_layers(const mps_state* bra, mps_state* ket, const mps_gate* gates,
                              const int* n_gates, int n_layers, double* re, double* im);

/* ---- measurement -------------------------------------------------------- */

/* Kernel classes timed when profiling is on (hipEvents around every launch on
 * the state's stream). */
typedef enum {
    MPS_KCLASS_CONTRACT = 0,  /* complex GEMMs of the environment / local tensor */
    MPS_KCLASS_MPO = 1,       /* structured MPO application                      */
    MPS_KCLASS_GRAM = 2,      /* FP64 Gram matrices of the truncation            */
    MPS_KCLASS_EIGH = 3,      /* FP64 Hermitian eigensolver (tridiagonal divide
                                 and conquer, back-transformation, or the dense
                                 library solver)                                 */
    MPS_KCLASS_OTHER = 4,     /* conversions, reductions, small FP64 GEMMs       */
    MPS_KCLASS_TRIDIAG = 5,   /* FP64 tridiagonal reduction of the eigensolver;
                                 flops = (16/3) n^3 per order-n matrix           */
    MPS_KCLASS_COUNT = 6
} mps_kernel_class;

/* Turn per-launch timing on (1) or off (0) and reset the counters. */
mps_status mps_set_profiling(mps_state* state, int on);

/* Launch count, summed launch duration in milliseconds, summed algorithmic
 * real flops and summed algorithmic HBM bytes of one kernel class since
 * profiling was turned on.  Algorithmic flops count 8 per complex
 * multiply-add; bytes count each operand read once and each result written
 * once. */
mps_status mps_kernel_stats(const mps_state* state, int kernel_class, int64_t* launches,
                            double* total_ms, double* flops, double* bytes);

/* ---- kernel self-test ---------------------------------------------------- */

/* Run the library's complex GEMM kernel once, C = op(A) op(B), on host data:
 * the operands are copied to the device, converted to the arithmetic of
 * `precision`, multiplied by the same kernel the compression step uses, and
 * the result is copied back.  All buffers are HOST, interleaved complex128,
 * row-major:
 *   opa 0 (N): a is M x K;   opa 2 (C): a is K x M and op(A) = a^H.
 *   opb 0 (N): b is K x N;   opb 1 (T): b is N x K, op(B) = b^T;
 *   opb 2 (C): b is N x K, op(B) = b^H.
 *   c receives M x N.
 * precision MPS_BF16X3 / MPS_BF16X2 runs the split-precision product, which
 * takes opa = 0 with opb = 1 (b split as it stands) or opb = 0 (b^T split
 * straight from b, as the environment update does).  For kernel-level parity
 * tests; not used by the compression step. */
mps_status mps_kernel_selftest_cgemm(int precision, int opa, int opb, int M, int N, int K,
                                     const double* a, const double* b, double* c);

/* Run the FP64 Hermitian eigensolver of the truncation (Sec. VI.A: the kept
 * singular values are the largest eigenvalues of the Gram matrix of the
 * local tensor) once on host data.  a: n x n Hermitian, HOST, interleaved
 * complex128, row-major (only the lower triangle, row >= column, is read).
 * method 0: rocSOLVER's dense solver; method 1: the persistent tridiagonal
 * reduction kernel (n <= 2048, else method 0 is used) followed by the
 * library's tridiagonal divide and conquer (mps_kernel_selftest_stedc) and
 * the back-transformation.
 * Outputs (HOST): w[n] eigenvalues in ascending order; z[n * n] interleaved
 * complex128, column j at z[2 (i + j n)] is the eigenvector of w[j];
 * *used (may be NULL) the method that actually ran (method 1 falls back to
 * method 0 when the cooperative launch is refused or gives up waiting).
 * MPS_ERR_NUMERIC when the solver does not converge.  For kernel-level
 * parity tests; the compression step calls the same routine on the device
 * Gram matrix (choose the method with the environment variable
 * MPS_EIGENSOLVER = rocsolver | persistent, default persistent). */
mps_status mps_kernel_selftest_eigh(int n, const double* a, int method, double* w, double* z, int* used);

/* The tridiagonal eigensolver of the truncation's method 1, once on host
 * data: divide and conquer on the real symmetric tridiagonal matrix with
 * diagonal d[n] and off-diagonal e[n - 1] (HOST; e may be NULL when n = 1),
 * 1 <= n <= 2048.  The matrix splits into two halves plus a rank-one term,
 * the halves are solved recursively and each merge solves the secular
 * equation of the rank-one update, with deflation of negligible or nearly
 * coincident terms and eigenvectors from the recomputed update vector, so
 * that they are orthogonal to working accuracy.  It stands in for a
 * library tridiagonal solver in Sec. VI.A's truncated SVD (all eigenvalues
 * for the discarded weight, the vectors of the kept ones).  Outputs (HOST):
 * w[n] eigenvalues ascending; z[n * n] real, column-major, column j the
 * eigenvector of w[j].  For kernel-level parity tests. */
mps_status mps_kernel_selftest_stedc(int n, const double* d, const double* e, double* w, double* z);

/* The complex GEMM of mps_kernel_selftest_cgemm on DEVICE operands, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  It calls no
 * allocator.  The split-K partial sums that long contractions need live in a
 * library-owned static device array of 64 MiB per GPU (held until the process
 * ends); products whose partial sums exceed it (2 M N chunks FP32 values,
 * chunks = the library's split of K) fail with MPS_ERR_ARG before any work.
 *   precision  MPS_FP64 (double operands) or MPS_FP32 / MPS_BF16X2 /
 *              MPS_BF16X3 (float operands); the split precisions take
 *              opa = 0, opb = 1 only.
 *   opa, opb, M, N, K  as for mps_kernel_selftest_cgemm.
 *   a_re .. c_im  DEVICE pointers to planar (separate real and imaginary)
 *              row-major matrices with leading dimensions lda, ldb, ldc (in
 *              elements); c is overwritten.  The caller owns all of them.
 *   hip_stream stream the work is queued on (NULL = default stream); the call
 *              returns without waiting.
 * All calls on one GPU share its scratch array: calls that overlap in time on
 * that GPU (different streams or threads) race and give wrong results; calls
 * on one stream are ordered and safe.  Results equal those of
 * mps_kernel_selftest_cgemm on the same operands, bit for bit (same split of
 * K; for the split precisions the same BF16 terms, k tiles and MFMA order,
 * with each tile's operands split while they are staged instead of in one
 * pass beforehand). */
mps_status mps_cgemm_noalloc(int precision, int opa, int opb, int M, int N, int K,
                             const void* a_re, const void* a_im, int64_t lda,
                             const void* b_re, const void* b_im, int64_t ldb,
                             void* c_re, void* c_im, int64_t ldc, void* hip_stream);

/* ---- The exact state, for measuring the simulation (Sec. VI, VII) ---------
 * The brute-force statevector U|0> (the perfect state of eq:F-sup) held in
 * device memory: FP64 planar, 2^n amplitudes, chain site q is bit n-1-q of
 * the index (site 0 most significant, as in mps_to_statevector).  It needs
 * 16 * 2^n bytes (64 GiB at 32 qubits); sv_compare_mps needs twice that again
 * as scratch.  A state belongs to one thread at a time. */
typedef struct sv_state sv_state;

/* Create |x> on n_qubits qubits, 1 <= n_qubits <= 34.  init_bits: n_qubits
 * bytes of 0/1 (NULL = |0...0>).  hip_stream: stream for all its work.
 * MPS_ERR_OOM when the device cannot hold it.  Release with sv_destroy. */
mps_status sv_create(int n_qubits, const uint8_t* init_bits, void* hip_stream, sv_state** out);

/* Release a statevector.  NULL is accepted. */
mps_status sv_destroy(sv_state* sv);

/* Apply one layer (the gate records and rules of mps_gate: one-qubit gates
 * first, disjoint two-qubit gates) exactly.  The layer's one-qubit gates are
 * folded into the two-qubit gate on their qubit; the others are applied two
 * at a time.  MPS_ERR_ARG (state unchanged) for invalid gates. */
mps_status sv_apply_layer(sv_state* sv, const mps_gate* gates, int n_gates);

/* out[2t], out[2t+1] = amplitude of index indices[t] (HOST arrays; indices in
 * [0, 2^n)). */
mps_status sv_amplitudes(const sv_state* sv, int64_t count, const int64_t* indices, double* out);

/* Measure an MPS against the exact state (n_sites == n_qubits): the MPS is
 * expanded to its 2^n amplitudes phi on the device, then, with psi the exact
 * state and all sums in a fixed order,
 *   overlap[2] = <phi|psi> (re, im);
 *   *F   = |<phi|psi>|^2 (eq:F-sup);
 *   *F_B = 2^n sum_x |psi_x|^2 |phi_x|^2 - 1 (eq:FB-sup);
 *   norms[2] = <phi|phi>, <psi|psi>.
 * Any output may be NULL.  Runs on the MPS's stream after the statevector's
 * stream has drained; allocates 2 x 16 x 2^n bytes of scratch for the call. */
mps_status sv_compare_mps(const sv_state* sv, mps_state* mps, double* overlap, double* F, double* F_B,
                          double* norms);

/* Squared Schmidt values of the exact state across the cut after `cut` chain
 * sites (1 <= cut < n_qubits): the best possible MPS with bond chi at that cut
 * keeps the weight *kept = sum of the chi largest S_mu^2 (Sec. VI, the best
 * MPS; at the middle cut it gives eps_SVD), *total = sum of all S_mu^2 (the
 * norm, 1 for a unit state).  s2 (may be NULL) receives all min(2^cut,
 * 2^(n-cut)) values, largest first.  The smaller side must hold at most 14
 * qubits (MPS_ERR_ARG otherwise); the values are the eigenvalues of the FP64
 * Gram matrix of the smaller side (rocSOLVER, values only), so values below
 * about 1e-15 of the largest are not resolved.  Host outputs. */
mps_status sv_schmidt_weights(const sv_state* sv, int cut, int chi, double* kept, double* total, double* s2);

#ifdef __cplusplus
}
#endif

#endif /* MPS_DMRG_H */
