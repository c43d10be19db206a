/*
 * hyperion_mi355x.h -- C ABI of the MI355X (gfx950) sparse state-vector
 * library: the exact Hamiltonian-times-state product and the steps of
 * state-vector ADAPT-VQE that live on it.
 *
 * Paper: "High Performance Quantum Emulation for Chemistry Applications with
 * Hyperion" (arXiv 2604.01176), section "Sparse State-Vector Emulation":
 * the Hamiltonian is assembled from qubit-mapped fermionic operators, the
 * state lives in the symmetry-restricted configuration space Omega_CIk, and
 * the operations needed are the matrix-vector product, inner products and
 * the application of exponentiated fermionic operators.  ADAPT-VQE operator
 * selection by pool gradients is described in "Numerical performance".
 *
 * Conventions
 *   n = 2M qubits (M <= 16 spatial orbitals).  Qubit q < M is orbital q with
 *   spin alpha, qubit q >= M is orbital q-M with spin beta; bit set =
 *   occupied (Jordan-Wigner, |1> = occupied).
 *   A Pauli string is P(x, z) = tensor_q sigma(x_q, z_q) with sigma(0,0)=I,
 *   (1,0)=X, (0,1)=Z, (1,1)=Y; P|b> = i^{n_Y} (-1)^{popc(z&b)} |b xor x>.
 *   Sector (N_alpha, N_beta): all b with popc(alpha bits) = N_alpha and
 *   popc(beta bits) = N_beta.  Sector index
 *     idx(b) = rank(beta) * C(M, N_alpha) + rank(alpha),
 *     rank(s) = sum_{i=1..k} C(o_i, i) over set bits o_1 < ... < o_k,
 *   i.e. the position of b among all sector bitstrings in ascending order.
 *   Excitation hyp_exc{cre, ann}: qubit masks with |cre| = |ann| in {1, 2},
 *   disjoint.  tau = a+_{c1} a+_{c2} a_{a2} a_{a1} (c1 < c2, a1 < a2) or
 *   a+_c a_a; the generator is A = tau - tau^dagger (real antisymmetric).
 *
 * Buffers and streams
 *   State, gradient and scalar output buffers belong to the caller: device
 *   memory, contiguous, 8-byte aligned, FP64 (HYP_F64) or FP32 (HYP_F32)
 *   amplitudes of length hyp_sector_dim().  The library owns hyp_sector and
 *   hyp_ham objects and their device tables and frees them in *_destroy; it
 *   never frees caller memory.  `stream` is a hipStream_t (NULL = default).
 *   Every call validates all arguments before enqueuing anything; on error it
 *   has no side effects and leaves outputs untouched.  HYP_OK means
 *   validated and enqueued (asynchronous).  Scalar results are written to
 *   device memory.  Calls that use a sector's internal scratch (marked
 *   "scratch") must not overlap with each other on different streams for the
 *   same sector.  No C++ exception crosses this interface.
 */
#ifndef HYPERION_MI355X_H
#define HYPERION_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HYP_OK = 0,
  HYP_ERR_ARG = 1,          /* null pointer, bad dtype, mask bit >= n, |cre| != |ann|, overlap */
  HYP_ERR_SECTOR = 2,       /* excitation changes N_alpha or N_beta, or M > 16 */
  HYP_ERR_NONREAL = 3,      /* Pauli term with odd n_Y (imaginary for a real H) */
  HYP_ERR_NOMEM = 4,
  HYP_ERR_HIP = 5,          /* HIP runtime failure; text in hyp_last_error() */
  HYP_ERR_UNSUPPORTED = 6
} hyp_status;

typedef enum { HYP_F64 = 0, HYP_F32 = 1 } hyp_dtype;

typedef struct hyp_sector_s* hyp_sector;
typedef struct hyp_ham_s* hyp_ham;
typedef struct { uint32_t cre, ann; } hyp_exc;

/* Thread-local text of the last non-OK status of this thread. */
const char* hyp_last_error(void);

/* Sector (N_alpha, N_beta) of M spatial orbitals, the symmetry-restricted
 * configuration space Omega_CIk ("Sparse State-Vector Emulation", Table 1).
 * 1 <= M <= 16, 0 <= N <= M.  Uploads string and rank tables to the current
 * device.  *out owned by the library until hyp_sector_destroy. */
hyp_status hyp_sector_create(int n_orb, int n_alpha, int n_beta, hyp_sector* out);
hyp_status hyp_sector_destroy(hyp_sector s);
/* C(M, N_alpha) * C(M, N_beta); -1 for a NULL sector. */
int64_t hyp_sector_dim(hyp_sector s);

/* Host-side, bit-exact: sector index of each bitstring (-1 if outside the
 * sector), and its inverse (HYP_ERR_ARG for an index outside [0, dim)).
 * Host arrays of n elements. */
hyp_status hyp_sector_rank(hyp_sector s, const uint32_t* bits, int64_t n, int64_t* idx);
hyp_status hyp_sector_unrank(hyp_sector s, const int64_t* idx, int64_t n, uint32_t* bits);

/* Assemble the Hamiltonian H = sum_t c_t P(x_t, z_t) for this sector
 * ("Sparse State-Vector Emulation": H is obtained by summing the qubit-mapped
 * fermionic operators; here it stays matrix-free as an X-mask-grouped Pauli
 * table).  Host arrays of n_terms elements.  Duplicate (x, z) are summed.
 * HYP_ERR_NONREAL for a nonzero term with odd n_Y; HYP_ERR_ARG for a mask
 * bit >= 2M or n_terms < 0.  Terms that cannot connect two sector states
 * are dropped.  Two-body number-conserving Hamiltonians (every Jordan-Wigner
 * molecular Hamiltonian) use the structured gfx950 kernel; any other real
 * Pauli sum uses a generic term-by-term kernel.  Synchronous upload on
 * `stream`.  *out owned by the library until hyp_ham_destroy. */
hyp_status hyp_build_hamiltonian(hyp_sector s, const uint32_t* x_mask, const uint32_t* z_mask,
                                 const double* coeff, int64_t n_terms, void* stream,
                                 hyp_ham* out);
hyp_status hyp_ham_destroy(hyp_ham h);

/* Device-side Hamiltonian assembly ("Sparse State-Vector Emulation": the
 * Hamiltonian is assembled on the GPU by summing the contributions of the
 * individual fermionic operators after the qubit mapping).  From the
 * molecular integrals h_dev [M][M] and g_dev [M][M][M][M] (device FP64,
 * chemist's notation, row-major) and the constant e_core:
 *   H = e_core + sum_{pq s} h_pq a+_{ps} a_{qs}
 *     + 1/2 sum_{pqrs, s t} g_pqrs a+_{ps} a+_{rt} a_{st} a_{qs},
 * Jordan-Wigner with spin orbital p + s M on qubit p + s M (blocked spin
 * order), as a Pauli list sum_t c_t P(x_t, z_t) (P with Y where both bits are
 * set), equal strings merged (double-double sums; residues below 1e-14 of a
 * string's summed magnitudes are exact cancellations and dropped), sorted by
 * (x, z), i.e. grouped by X mask.  Writes min(n, cap) terms to the device
 * arrays x_dev, z_dev, c_dev and n to *n_terms (host); cap = 0 with NULL
 * outputs only counts.  HYP_ERR_ARG for M outside [1, 16] or cap < n (after
 * writing *n_terms); HYP_ERR_NONREAL when an imaginary part survives (h or g
 * not real-symmetric).  Synchronous on `stream`; scratch is allocated and
 * freed inside (about 40 bytes per expansion slot, 4.2 M slots at M = 16). */
hyp_status hyp_assemble_pauli(int n_orb, const double* h_dev, const double* g_dev, double e_core,
                              uint32_t* x_dev, uint32_t* z_dev, double* c_dev, int64_t cap,
                              int64_t* n_terms, void* stream);

/* hyp_assemble_pauli followed by hyp_build_hamiltonian on its list (the
 * X-group fold of the build runs on the host from the downloaded table).
 * n_orb must equal the sector's M.  Synchronous on `stream`. */
hyp_status hyp_build_hamiltonian_integrals(hyp_sector s, int n_orb, const double* h_dev,
                                           const double* g_dev, double e_core, void* stream,
                                           hyp_ham* out);
/* 1 if the structured kernel serves this Hamiltonian, 0 if the generic one, -1 on NULL. */
int hyp_ham_is_structured(hyp_ham h);

/* Autotuner of the H psi tile shape (the mixed pass's workgroup width, one
 * thread per alpha column): times the candidates {128,...,1024} on this
 * Hamiltonian with reps applications each (HIP events on `stream`), keeps
 * the fastest for later hyp_apply_h calls on h in that storage type (FP64
 * and FP32 keep separate widths) and returns it.  In FP64 the 768-thread
 * candidate is the compact, double-buffered mixed pass wherever its staging
 * tables exist (see hyp_set_row_staging).  Where the mixed pass runs on the
 * matrix cores (hyp_set_mixed_matrix_cores) it has no width to tune: the
 * call times that form and returns 1024.  Overwrites sigma_dev.  A
 * generic (non-structured) Hamiltonian returns 0 threads. */
hyp_status hyp_tune_apply_h(hyp_ham h, hyp_dtype dtype, const void* psi_dev, void* sigma_dev,
                            int reps, void* stream, int* best_threads, double* best_ms);

/* sigma = P_S H P_S psi (the paper's sparse matrix-vector product, computed
 * matrix-free as a pull gather: each output amplitude is written once, no
 * atomics).  psi and sigma: device, dim amplitudes of dtype, must not alias.
 * HYP_F32: FP32 storage, FP32 products, FP64 accumulation. */
hyp_status hyp_apply_h(hyp_ham h, hyp_dtype dtype, const void* psi_dev, void* sigma_dev,
                       void* stream);

/* Support skipping in hyp_apply_h and in the transition-value sweep of
 * hyp_pool_gradients (on = 1, the default; 0 = off).  The product is the
 * sparse matrix times a sparse vector of "Sparse State-Vector Emulation":
 * only amplitudes in the support of psi feed sigma, and only they enter the
 * gradients (T(tau) = sum_D s sigma[tau D] psi[D]).
 * hyp_apply_h (structured kernel): records which beta rows and alpha columns
 * of psi hold a nonzero amplitude (while transposing psi), restricts the
 * same-spin matrices to source rows in that support, drops mixed-pass source
 * rows outside it, and reduces an output row with no source row in the
 * support to its same-spin partials.  Device-side decisions only (no host
 * synchronisation), so the product can be captured in a HIP graph either
 * way.  The generic kernel always evaluates densely.
 * hyp_pool_gradients (modes 0 and 2): the row pairs and identity slices of
 * the transition values keep only source rows in psi's support; the
 * same-spin Gram blocks of a core whose slots hold no nonzero psi row are
 * zero without a product, and a Gram whose contraction range (beta rows for
 * the alpha blocks, alpha columns for the beta blocks) is at most half in the
 * support sums over the gathered support only.  These decisions are taken on
 * the device too: the sweep never waits on the host and can be captured.
 * The pair kernel (mode 1 and candidate subsets) skips pairs whose two
 * determinants both lie outside psi's row or column support.
 * Results equal the dense evaluation up to summation order.  Near the
 * Hartree-Fock state (early ADAPT iterations) both cost a small fraction of
 * the dense ones; for a dense psi the extra work is a support scan, list
 * compactions and flag writes.  Process-wide setting; HYP_ERR_ARG unless on
 * is 0 or 1. */
hyp_status hyp_set_support_skip(int on);

/* Same-spin part of hyp_apply_h with FP64 storage.  tiles = 1, 2 or 4
 * (default 2): grouped lists, where each wave takes 8 consecutive output
 * strings and 64 columns and loads every source amplitude their rows share
 * once (the union of their sources, each with the 8 rows' coefficients), and
 * a four-wave workgroup holds `tiles` neighbouring column tiles of 4 / tiles
 * consecutive groups; 0: per-row lists, one output string per wave.  Equal
 * results up to summation order.  FP32 storage always uses the per-row
 * lists.  Process-wide; HYP_ERR_ARG for other values. */
hyp_status hyp_set_same_spin_groups(int tiles);

/* Same-spin doubles of hyp_apply_h with FP64 storage through the strings'
 * cores (the paper's "Sparse State-Vector Emulation" product; the doubles
 * are 784 of the 849 same-spin entries of a row at 16 orbitals and 8
 * electrons).  Two strings joined by a same-spin double share exactly one
 * core, an (N-2)-electron string, so for each core K the doubles are a dense
 * S x S product (S = C(M - N + 2, 2) slots) of the core's rows, Y_K = W_K
 * psi_K, formed on FP64 MFMA in column bands, and each output row adds its
 * C(N, 2) cores' rows of Y in a fixed order (deterministic) beside its
 * singles and diagonal, which keep the per-row lists.  mode = 2 (default)
 * takes it where the tables were built with the Hamiltonian (every core of
 * both spins with at most 48 slots; a band of Y takes at most 20 GiB or an
 * eighth of the device memory, allocated with the Hamiltonian: 18.6 GB in
 * two bands at 32 qubits) and the FP64 state vector
 * exceeds 256 MiB, the size of the Infinity Cache, below which the grouped
 * lists are faster; 1 wherever the tables were built; 0 never (the grouped
 * or per-row lists of hyp_set_same_spin_groups).  With support skipping
 * (hyp_set_support_skip) the core path's choice is then made per spin on
 * the device: the core path where at least a quarter of the spin's strings
 * carry amplitude, the grouped lists below that (the other path's kernels
 * exit at once; no host synchronisation).  Equal results up to summation
 * order.  Process-wide; HYP_ERR_ARG unless mode is 0, 1 or 2. */
hyp_status hyp_set_same_spin_cores(int mode);

/* The alpha-beta products of hyp_apply_h and of hyp_pool_gradients on FP64
 * MFMA (the paper's "Sparse State-Vector Emulation" product and its pool
 * gradients; both storage types).  H psi: for one beta row, with its
 * beta-single source rows staged as the K x D_a matrix P (K <= 64), the
 * doubles and the beta singles' alpha dressing that empty alpha orbital e of
 * a source string are Z_e = A_e P over the source strings with e occupied
 * (A_e: 16 x K, the row's alpha-beta coefficients for the pairs (i, e) and
 * the dressing of e), each element added to its output string s = t - e + i
 * of the row held in LDS; the additions land in no fixed order, so sigma is
 * reproducible to rounding, not bit for bit.  Sweep: per target beta row,
 * X_e = A_e P^T with A_e the signed sigma values gathered at the targets,
 * added into per-workgroup partials that are summed in a fixed order
 * (reproducible bit for bit).  mode = 2 (default) takes the H psi form where
 * the output row fits LDS (D_a <= 14,000 at M <= 16) and the FP64 state
 * exceeds 64 MiB (28 qubits and up), the sweep form where its target row
 * fits and the state exceeds 256 MiB (32 qubits); 1 both wherever they fit;
 * 0 never (k_mixed / k_mixed_c and k_tdens_rows of hyp_set_row_staging,
 * bitwise reproducible).  With support skipping (hyp_set_support_skip) the
 * form is chosen per call on the device: the matrix-core one where at least
 * a quarter of psi's beta rows carry amplitude, the other below (both are
 * launched and the unchosen one exits at once; no host synchronisation, so
 * the calls stay capturable).  Process-wide; HYP_ERR_ARG unless mode is 0, 1
 * or 2. */
hyp_status hyp_set_mixed_matrix_cores(int mode);

/* Materialised sector Hamiltonian in CSR form, the paper's storage of H
 * ("Sparse State-Vector Emulation", Table 1 gives its size), kept as a
 * comparison for the matrix-free product.  Every row holds the same L
 * entries (diagonal; alpha singles and doubles; beta singles and doubles;
 * alpha-beta doubles; each column once, in that order): row_ptr[d] = d L,
 * int32 columns, FP64 values, all in device memory owned by the library.
 * hyp_csr_build: from a structured Hamiltonian (HYP_ERR_UNSUPPORTED for the
 * generic kind); HYP_ERR_NOMEM, with the byte count in hyp_last_error(),
 * when 12 bytes per nonzero plus the row pointers do not fit in free device
 * memory with a 2 GiB margin (24 qubits: 18.6 GB; 28 qubits would need
 * 478 GB).  Synchronous on `stream`.
 * hyp_csr_apply: sigma = H psi, one wave per row, FP64 accumulation (HYP_F32:
 * FP32 storage and products).  psi and sigma must not alias.
 * hyp_csr_export: synchronous copy to host arrays of dim + 1, nnz and nnz
 * elements.  hyp_csr_nnz: -1 for NULL. */
typedef struct hyp_csr_s* hyp_csr;
hyp_status hyp_csr_build(hyp_ham h, void* stream, hyp_csr* out);
hyp_status hyp_csr_apply(hyp_csr m, hyp_dtype dtype, const void* psi_dev, void* sigma_dev, void* stream);
hyp_status hyp_csr_export(hyp_csr m, int64_t* row_ptr, int32_t* col, double* val);
int64_t hyp_csr_nnz(hyp_csr m);
hyp_status hyp_csr_destroy(hyp_csr m);

/* *out_dev = <a|b> = sum_i a_i b_i with FP64 accumulation (the sparse inner
 * product / expectation value of "General Framework for Variational
 * Algorithms", E = <psi|H psi>).  out_dev: one device double.  Scratch. */
hyp_status hyp_expectation(hyp_sector s, hyp_dtype dtype, const void* a_dev, const void* b_dev,
                           double* out_dev, void* stream);

/* grad_dev[k] = 2 <sigma| A_k psi> for the n_ops generators in ops_dev
 * (device array of hyp_exc), with sigma = H psi given: the ADAPT-VQE pool
 * gradient dE/dtheta at theta = 0 of appending exp(theta A_k) ("Numerical
 * performance": the gradient over the pool selects each new operator).  FP64
 * output, FP64 accumulation.  Asynchronous and graph-capturable: nothing
 * waits on the host (scratch grows, and per-string-space tables are built,
 * on the first call for a sector size; capture after one eager call).
 * Host-side arguments are validated before anything is enqueued
 * (HYP_ERR_ARG: NULL pointer, bad dtype, n_ops outside [0, 2^24]).  The
 * excitations live in device memory and are validated there by the kernels
 * that read them with the rules of hyp_apply_excitation: an invalid one gets
 * grad_dev[k] = NaN, is never used as an index, and is recorded for
 * hyp_pool_check; the other gradients are unaffected. */
hyp_status hyp_pool_gradients(hyp_sector s, hyp_dtype dtype, const hyp_exc* ops_dev,
                              int64_t n_ops, const void* psi_dev, const void* sigma_dev,
                              double* grad_dev, void* stream);

/* hyp_pool_gradients for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the per-generator pair kernel (the strategy of candidate
 * subsets, hyp_set_sweep_mode 1) with its per-chunk partials in a static
 * per-GPU array of the library (32,768 generators x 16 chunks of doubles,
 * 4 MiB, held by every GPU the library runs on until the process ends).
 * No call allocates or frees device memory.  The first call on a device
 * takes the array's address there and uploads the binomial table (a
 * synchronous copy; later calls are asynchronous).  No support skipping:
 * every pair is evaluated.  Same arguments, output and device-side
 * excitation checks as hyp_pool_gradients; HYP_ERR_ARG also when n_ops
 * exceeds 32,768 (nothing enqueued).  Every call on one GPU shares the
 * array: calls that overlap on one GPU (several streams, or several host
 * threads) race; calls ordered on one stream do not. */
hyp_status hyp_pool_gradients_noalloc(hyp_sector s, hyp_dtype dtype, const hyp_exc* ops_dev,
                                      int64_t n_ops, const void* psi_dev, const void* sigma_dev,
                                      double* grad_dev, void* stream);

/* Waits for `stream`, then reports the first invalid excitation that
 * hyp_pool_gradients met on this device since the last report: HYP_ERR_ARG
 * or HYP_ERR_SECTOR (the largest status met), its list position in
 * hyp_last_error(), and clears the record; HYP_OK when there was none. */
hyp_status hyp_pool_check(void* stream);

/* Strategy of hyp_pool_gradients: 0 automatic (default), 1 the per-generator
 * pair kernel, 2 transition values, 3 transition values with per-stage bins.
 * The transition-value sweep computes T(tau) = sum_D s sigma[tau D] psi[D]
 * for every single and alpha-beta double excitation at once
 * (g = 2 (T(tau) - T(tau^dagger))), and the same-spin doubles from the two
 * Gram matrices sigma^T psi and sigma psi^T (FP64 GEMMs; per-device scratch of
 * C(M,N_a)^2 + C(M,N_b)^2 doubles, plus 2 dim doubles in FP32 mode).  Mode 2
 * walks the row pairs of each beta excitation with register accumulators
 * (small scratch); mode 3 bins every (beta row, stage) in LDS and needs
 * C(M,N_b) * ceil(C(M,N_a)/768) * (1 + N_b (M - N_b)) * 241 doubles of scratch
 * (27 GB at 32 qubits, refused above 40 GiB).  Automatic mode uses mode 2 when
 * n_ops covers at least a quarter of the full pool, else mode 1.
 * Process-wide setting. */
hyp_status hyp_set_sweep_mode(int mode);

/* Row staging of mode 2's kernel and of the FP64 mixed pass of hyp_apply_h
 * (a tuning and testing control, no effect on results): 0 (default) stages,
 * for FP64 state vectors whose rows are whole 16-byte blocks, only the blocks
 * of each source row that a column chunk (512 columns in the sweep, 768 in
 * the mixed pass) and its columns' single excitations reach, into two
 * alternating LDS buffers so that the next row's copy overlaps this row's
 * products.  Tables of about C(M,N_a) * 2.1 bytes: the sweep's per device,
 * for up to eight string spaces, built on the first sweep of one; the mixed
 * pass's with the Hamiltonian (hyp_build_hamiltonian), where the mixed pass
 * then defaults to 768 threads.  Falls back to whole rows where a chunk needs
 * more than 4094 blocks.  1 always stages whole rows (hyp_apply_h: calls and
 * graph captures made after the switch).  Both give the same gradients and
 * sigma bit for bit.  Process-wide; HYP_ERR_ARG unless mode is 0 or 1. */
hyp_status hyp_set_row_staging(int mode);

/* Kind of the pool generators (the paper's ADAPT-VQE description names the
 * qubit-excitation-based, QEB, pool as an example): 0 fermionic excitations
 * (default), 1 qubit excitations.  Both take the same (cre, ann) masks; a
 * qubit excitation is the product of qubit raising and lowering operators
 * without the Jordan-Wigner parity strings, so tau|D> = |tau D> with sign +1
 * wherever a fermionic excitation would carry (-1)^parity.  Applies to
 * hyp_pool_gradients, hyp_pool_gradients_batched, hyp_apply_excitation and
 * the ADAPT engine for calls made after it (an ADAPT object's captured
 * evaluation graph keeps the kind in force when it was captured; it is
 * recaptured whenever the ansatz grows).  Process-wide; HYP_ERR_ARG unless
 * kind is 0 or 1. */
hyp_status hyp_set_pool_kind(int kind);

/* psi <- exp(theta A) psi in place (the exponentiated fermionic operator):
 * on every pair (D, D' = tau D, sign s) psi_D <- cos psi_D - s sin psi_D',
 * psi_D' <- s sin psi_D + cos psi_D'; other amplitudes unchanged. */
hyp_status hyp_apply_excitation(hyp_sector s, hyp_dtype dtype, hyp_exc op, double theta,
                                void* psi_dev, void* stream);

/* psi <- exp(theta[n-1] A_{n-1}) ... exp(theta[0] A_0) psi: the state
 * preparation of an ansatz, rotations enqueued in order on `stream`.  ops and
 * theta are host arrays of n elements; every generator and angle is
 * validated (as for hyp_apply_excitation) before the first rotation is
 * enqueued, so an error leaves psi untouched. */
hyp_status hyp_apply_excitations(hyp_sector s, hyp_dtype dtype, const hyp_exc* ops, const double* theta,
                                 int64_t n, void* psi_dev, void* stream);

/* Batched pool gradients for up to 16 instances (possibly of different
 * sectors, one dtype).  Jobs whose list covers at least a quarter of their
 * sector's full pool take the transition-value sweep of hyp_pool_gradients
 * (per instance, in order on `stream`: for full pools it is several times
 * faster than any pair enumeration); the other jobs (candidate subsets) run
 * in ONE persistent launch that drains a device work queue of (instance,
 * generator, beta-chunk) items, then one fixed-order reduction per
 * generator.  With hyp_set_sweep_mode(1) every job takes the persistent
 * launch.  Results equal hyp_pool_gradients per job up to summation order.
 * Excitations are validated on the host first (device-to-host copy of every
 * ops_dev array).  Uses per-device library scratch (grow-only): concurrent
 * batched calls on one device race.  tile (persistent launch only) == NULL
 * selects {256 threads, 16 chunks, 4 workgroups per CU}. */
typedef struct {
  hyp_sector sector;
  hyp_dtype dtype;
  const hyp_exc* ops_dev;   /* device array of n_ops excitations */
  int64_t n_ops;
  const void* psi_dev;
  const void* sigma_dev;    /* sigma = H psi of this instance */
  double* grad_dev;         /* device, n_ops doubles */
} hyp_grad_job;
typedef struct {
  int32_t threads;          /* workgroup size: 64, 128, 256, 512 or 1024 */
  int32_t chunks;           /* beta-entry chunks per generator, 1..256 */
  int32_t blocks_per_cu;    /* resident workgroups per CU of the persistent grid, 1..32 */
  int32_t reserved;
} hyp_sweep_tile;
hyp_status hyp_pool_gradients_batched(const hyp_grad_job* jobs, int n_jobs,
                                      const hyp_sweep_tile* tile, void* stream);
/* Autotuner of the persistent launch: times every tile of {128,256,512} x
 * {4,8,16,32} x {2,4,8} with all jobs in that launch (reps launches each, HIP
 * events on `stream`) and returns the fastest and its mean time.  Overwrites
 * the jobs' gradient outputs. */
hyp_status hyp_tune_pool_gradients(const hyp_grad_job* jobs, int n_jobs, int reps,
                                   hyp_sweep_tile* best, double* best_ms, void* stream);

/* ------------------------------------------------------------------------
 * ADAPT-VQE driver ("Numerical performance"): starting from the Hartree-Fock
 * determinant (sector index 0), each iteration computes sigma = H psi and the
 * pool gradients, appends the operator of largest |g| (ties: the lowest pool
 * index among |g| >= max|g| (1 - tie_tol)), and re-optimises all parameters
 * with BFGS (strong-Wolfe line search) on E(theta) = <psi(theta)|H|psi(theta)>,
 * psi(theta) = exp(theta_j A_j) ... exp(theta_1 A_1) |HF>, warm-started from
 * the previous parameters with the new one at 0.  Each energy+gradient
 * evaluation (state preparation, H psi, energy, adjoint gradient) is one
 * hipGraph replay when use_graph != 0.  FP32 storage renormalises the state
 * after every preparation.  The driver owns its stream and buffers; calls are
 * synchronous and return after the iteration finished.
 * ------------------------------------------------------------------------ */
typedef struct hyp_adapt_s* hyp_adapt;
typedef struct {
  int32_t max_iter;   /* maximum ansatz length (buffer capacity), 1..4096 */
  int32_t max_bfgs;   /* BFGS iterations per ADAPT iteration */
  int32_t use_graph;  /* capture each evaluation in a hipGraph */
  int32_t recycle_hessian;  /* 1: BFGS starts from the previous iteration's inverse-Hessian estimate
                               (identity for the appended parameter); 0: from the identity */
  double tie_tol;     /* relative tie tolerance of the selection, in [0, 1) */
  double gtol;        /* BFGS stop: max_i |dE/dtheta_i| <= gtol, > 0 */
  double gmax_stop;   /* no operator is added when max|g| < gmax_stop */
} hyp_adapt_opts;
typedef struct {
  int32_t selected;   /* pool index appended, -1 if stopped on gmax_stop */
  int32_t tie_count;  /* size of the tie set */
  int32_t n_evals;    /* energy+gradient evaluations of the optimiser */
  int32_t bfgs_iters;
  int32_t converged;  /* 1 if max|dE/dtheta| <= gtol, or the line search stalled below 100 gtol */
  int32_t reserved;
  double gmax;        /* max |g| over the computed gradients */
  double energy_before;  /* E of the state the gradients were taken on */
  double energy;      /* E after optimisation */
  double grad_ms, opt_ms;  /* host wall time of the two phases */
  double grad_inf;    /* max |dE/dtheta_i| at the optimiser's last point */
} hyp_adapt_record;

/* pool: host array of n_pool validated excitations (the operator pool). */
hyp_status hyp_adapt_create(hyp_ham h, hyp_dtype dtype, const hyp_exc* pool, int64_t n_pool,
                            const hyp_adapt_opts* opts, hyp_adapt* out);
hyp_status hyp_adapt_destroy(hyp_adapt a);
/* One iteration.  cand == NULL: exact gradients of the whole pool; otherwise
 * only of the n_cand pool indices in cand (host array), and the selection
 * runs inside that set (the screened iteration). */
hyp_status hyp_adapt_iterate(hyp_adapt a, const int32_t* cand, int64_t n_cand,
                             hyp_adapt_record* rec);
/* The two halves of hyp_adapt_iterate: exact gradients of the current state
 * (whole pool or the candidates), then selection + BFGS over the stored
 * gradients.  A screen calls the first on its candidates, may call it again
 * on the whole pool (fallback), then calls the second. */
hyp_status hyp_adapt_gradients(hyp_adapt a, const int32_t* cand, int64_t n_cand,
                               hyp_adapt_record* rec);
hyp_status hyp_adapt_select_optimize(hyp_adapt a, hyp_adapt_record* rec);
/* Re-optimises all parameters of the current ansatz (BFGS warm-started from
 * the current theta) without selecting an operator; rec->selected = -1,
 * energy_before / energy / n_evals / bfgs_iters / converged / grad_inf /
 * opt_ms as for a selection.  Used to polish, in FP64, the parameters of an
 * ansatz found by an FP32 run (hyp_adapt_set_ansatz first). */
hyp_status hyp_adapt_optimize(hyp_adapt a, hyp_adapt_record* rec);
/* Pool gradients of the last iteration (host, n = pool size; NaN where not computed). */
hyp_status hyp_adapt_last_gradients(hyp_adapt a, double* grad, int64_t n);
/* Current ansatz (pool indices, parameters); with cap < length only *n is set. */
hyp_status hyp_adapt_ansatz(hyp_adapt a, int32_t* ops, double* theta, int64_t cap, int64_t* n);
hyp_status hyp_adapt_set_ansatz(hyp_adapt a, const int32_t* ops, const double* theta, int64_t n);
/* One energy+gradient evaluation at theta (host arrays of the ansatz length). */
hyp_status hyp_adapt_eval(hyp_adapt a, const double* theta, double* energy, double* grad);
/* Copy U(theta)|HF> (adapt dtype) to psi_dev. */
hyp_status hyp_adapt_state(hyp_adapt a, void* psi_dev);
/* Energy of the current ansatz replayed in FP64 (allocates two FP64 vectors). */
hyp_status hyp_adapt_energy_fp64(hyp_adapt a, double* energy);

/* ------------------------------------------------------------------------
 * Learned gradient screen (a ranking aid for ADAPT-VQE operator selection;
 * not in the paper).  Feature rows are 32 BF16 values per operator.  The MLP
 * is y = W3 relu(W2 relu(W1 f + b1) + b2) + b3 with widths 32-256-256-1;
 * W1, W2 and the activations entering the two matrix products are BF16
 * (round to nearest even) on MFMA with FP32 accumulation; masters, biases,
 * W3 and the output layer are FP32.  Parameter layout (host arrays):
 * W1[256][32], b1[256], W2[256][256], b2[256], W3[256], b3[1] (74,241 floats).
 * ------------------------------------------------------------------------ */
typedef struct hyp_mlp_s* hyp_mlp;
/* init_host: initial parameters (layout above); max_rows: largest batch or
 * scoring call. */
hyp_status hyp_mlp_create(const float* init_host, int64_t max_rows, hyp_mlp* out);
hyp_status hyp_mlp_destroy(hyp_mlp m);
hyp_status hyp_mlp_params(hyp_mlp m, float* host_out);
/* scores y_dev[n] for feature rows X_dev[n][32] (BF16 bit patterns). */
hyp_status hyp_mlp_forward(hyp_mlp m, const uint16_t* X_dev, int64_t n, float* y_dev, void* stream);
/* One Adam step (beta 0.9/0.999, eps 1e-8) on the mean squared error of a
 * batch of B rows (16 <= B <= max_rows, B % 16 == 0) against targets t_dev;
 * y_dev receives the forward scores. */
hyp_status hyp_mlp_train_step(hyp_mlp m, const uint16_t* X_dev, const float* t_dev, int64_t B,
                              float lr, float* y_dev, void* stream);
/* Full training state (host, 3 * 74,497 + 1 floats): parameters, Adam first
 * and second moments (parameter layout each), then the Adam step count.
 * set_state also refreshes the BF16 weight copies; a network restored this
 * way continues training exactly as the one it was taken from. */
hyp_status hyp_mlp_get_state(hyp_mlp m, float* host_out);
hyp_status hyp_mlp_set_state(hyp_mlp m, const float* host_in);
/* Parameter gradients of the last train step (host, parameter layout). */
hyp_status hyp_mlp_grads(hyp_mlp m, float* host_out);
/* Static feature rows (host): stat[n][32] FP32 = class one-hot (0..4),
 * spatial orbital index / (M-1) of (c1, c2, a1, a2) for doubles or (c, a)
 * for singles, -1 padding (5..8), log10(|h_ca| + 1e-12) for singles or
 * log10(|(c1 a1|c2 a2)| + 1e-12), log10(|(c1 a2|c2 a1)| + 1e-12) for doubles
 * (9, 10), M/16 (17), zeros elsewhere; qidx[n][4] the same spin-orbitals as
 * qubit indices.  h: M*M, g: M^4 chemist's-notation integrals (host). */
hyp_status hyp_screen_static(int n_orb, const hyp_exc* pool, const uint8_t* cls, int64_t n,
                             const double* h, const double* g, float* stat, int32_t* qidx);
/* <n_q> of every spin-orbital q < 2M for a sector state (occ_dev: 2M
 * doubles; work_dev: C(M, N_beta) * 17 doubles of scratch). */
hyp_status hyp_occupations(hyp_sector s, hyp_dtype dtype, const void* psi_dev, double* occ_dev,
                           double* work_dev, void* stream);
/* Feature rows: static part stat_dev[n][32] (FP32) with slots 11..14 set to
 * <n_q> of the operator's spin-orbitals qidx_dev[n][4] (-1: 0), slot 15 to
 * log10(|g_prev| + 1e-12), slot 16 to min(age, 50) / 10, and against the
 * last selected operator (last_qidx: its four qubit indices in the qidx
 * layout, host array read at the call; all -1 before the first selection):
 * slot 18 = 1 for that operator itself, 19 = shared spin-orbitals / 4,
 * 20 = shared spatial orbitals / 4, 21 = log10(|last_g| + 1e-12) (0 with no
 * selection); output BF16.  HYP_ERR_ARG: NULL, n_orb outside 1..16 or a
 * last_qidx entry outside -1..2 n_orb - 1. */
hyp_status hyp_features(const float* stat_dev, const int32_t* qidx_dev, const double* occ_dev,
                        const double* gprev_dev, const int32_t* age_dev, int64_t n, int n_orb,
                        const int32_t* last_qidx, double last_g, uint16_t* X_dev, void* stream);
/* Screen bookkeeping: for every k with g_dev[k] not NaN, gprev[k] = g[k]
 * and age[k] = 0; every other age grows by one. */
hyp_status hyp_screen_update(const double* g_dev, int64_t n, double* gprev_dev, int32_t* age_dev,
                             void* stream);
/* Base score of every operator, taken with the feature rows (before the
 * sweep that updates g_prev): base[k] = max(log10(|g_prev[k]| + 1e-12), t_floor)
 * (FP32).  The network predicts the change of the floored log gradient since
 * its last exact value; an operator's score is base + network output. */
hyp_status hyp_screen_base(const double* gprev_dev, int64_t n, float t_floor, float* base_dev, void* stream);
/* Training rows: Xo[i] = X[idx[i]] (32 BF16),
 * t[i] = max(log10(|g[idx[i]]| + 1e-12), t_floor) - base[idx[i]] (FP32;
 * base_dev NULL: no base; t_floor = -12 keeps the plain log target). */
hyp_status hyp_screen_batch(const uint16_t* X_dev, const double* g_dev, const int32_t* idx_dev,
                            int64_t m, float t_floor, const float* base_dev, uint16_t* Xo_dev, float* t_dev,
                            void* stream);
/* Operator indices sorted by descending score y + base (base_dev NULL: y);
 * stable: ties keep index order. */
hyp_status hyp_rank_scores(hyp_mlp m, const float* y_dev, const float* base_dev, int64_t n, int32_t* order_dev,
                           void* stream);

/* Kernel timing (tracing).  While enabled, every kernel the library launches
 * is bracketed by HIP events on its stream; hyp_profile_count() waits for
 * the recorded events and returns the number of distinct kernel names, and
 * hyp_profile_get(i, ...) returns the i-th name (NUL-terminated, truncated
 * to name_len), its summed device time in ms and its launch count.
 * Intended for measurement runs; enable before the calls to be timed. */
hyp_status hyp_profile_enable(int on);
hyp_status hyp_profile_reset(void);
int hyp_profile_count(void);
hyp_status hyp_profile_get(int i, char* name, int name_len, double* total_ms, int64_t* calls);

#ifdef __cplusplus
}
#endif

#endif /* HYPERION_MI355X_H */
