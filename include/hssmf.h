/*
 * hssmf.h -- C ABI of an MI355X (gfx950) HSS-structured multifrontal sparse
 * solver with randomized sampling.
 *
 * Method: Ghysels, Li, Rouet, Williams, Napov, "An efficient multi-core
 * implementation of a novel HSS-structured multifrontal solver using
 * randomized sampling" (arXiv 1502.07405).  The solver computes an (exact or
 * HSS-approximate) multifrontal LU factorization of a general sparse
 * non-singular matrix (Sec. 3, Sec. 4) and uses it inside iterative
 * refinement or restarted GMRES (Sec. 4.6, Sec. 6.1) to solve A x = b.
 *
 * Conventions
 *  - Every function returns HSSMF_OK (0) or a negative status code; no C++
 *    exception crosses this boundary.  hssmf_strerror() names a code.
 *  - Matrix and ordering arrays are owned by the caller and read during the
 *    call only (copied / uploaded).  Ordering arrays are host memory; the
 *    CSR arrays are host or device memory as hssmf_csr.mem says.
 *  - Vector arguments of hssmf_apply, hssmf_adjoint and
 *    hssmf_solve_noalloc are DEVICE pointers (HIP global memory on the
 *    current device).  hssmf_solve,
 *    hssmf_solve_transpose and hssmf_solve_batch take host or device
 *    vectors: the library asks the HIP runtime (hipPointerGetAttributes)
 *    which one each pointer is, and stages host vectors through device
 *    memory.  All vectors are owned by the caller.
 *  - A handle owns all device memory of a factorization until
 *    hssmf_destroy().  A handle is not thread-safe; calls on one handle must
 *    not overlap.  All device work is enqueued on the stream given to
 *    hssmf_factor (0 = the null stream); functions return after that stream
 *    has drained (they synchronize when they need host-visible results).
 *  - Indices are 0-based.
 */
#ifndef HSSMF_H
#define HSSMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define HSSMF_OK 0
#define HSSMF_EINVAL (-1)    /* malformed CSR, ordering, options or arguments */
#define HSSMF_ENOMEM (-2)    /* device or host allocation failed */
#define HSSMF_ESINGULAR (-3) /* zero pivot in an F11 block or at an ULV top node */
#define HSSMF_ERANK (-4)     /* adaptive sampling reached d_max (Sec. 2.2.1) */
#define HSSMF_ENOCONV (-5)   /* outer solver did not reach tol within max_it */
#define HSSMF_EDEVICE (-6)   /* HIP runtime error / no device */
#define HSSMF_ETOOBIG (-7)   /* the no-allocation solve's static scratch is too
                                small for this handle and these options */

/* precision of the sampling and ULV products (pivoted QR / ID, the LU of
 * F11 blocks and the refinement residual always stay FP64) */
#define HSSMF_PREC_FP64 0
#define HSSMF_PREC_FP32 1
#define HSSMF_PREC_BF16 2

#define HSSMF_OUTER_IR 0
#define HSSMF_OUTER_GMRES 1

/* where the arrays of an hssmf_csr live */
#define HSSMF_MEM_HOST 0
#define HSSMF_MEM_DEVICE 1

/* Sparse matrix A (n x n) in CSR form: a general non-symmetric,
 * non-singular matrix (Sec. 1, Sec. 3).  rowptr has n+1 entries
 * (rowptr[0] = 0, non-decreasing), colind/val have rowptr[n] entries; column
 * indices lie in [0, n) and are unique within a row.  mem: HSSMF_MEM_HOST
 * (0) when rowptr / colind / val are host memory, HSSMF_MEM_DEVICE (1) when
 * they are device memory of the current device (they are then copied to the
 * host for the symbolic analysis, and the values also device to device). */
typedef struct {
  int32_t n;
  const int64_t* rowptr;
  const int32_t* colind;
  const double* val;
  int32_t mem;
} hssmf_csr;

/* Fill-reducing nested-dissection ordering (Sec. 3.1) with its separator
 * tree, host memory.  perm[new] = old (a permutation of 0..n-1).  Fronts are
 * numbered in postorder (children before parents, parent[f] > f, -1 for a
 * root); front f eliminates the new indices [sep_ptr[f], sep_ptr[f+1]);
 * sep_ptr[0] = 0, sep_ptr[nfront] = n, non-decreasing.  Every off-diagonal
 * coupling of P A P^T must join a front with itself or with an ancestor
 * (the separator property); violations give HSSMF_EINVAL. */
typedef struct {
  const int32_t* perm;
  int32_t nfront;
  const int32_t* sep_ptr;
  const int32_t* parent;
} hssmf_ordering;

/* Options.  Use hssmf_default_opts() and override fields. */
typedef struct {
  double rel_tol;      /* HSS compression tolerance eps: rank stops at
                          |R_{i+1,i+1}| <= eps |R_11| (Sec. 5.3) */
  int32_t leaf_size;   /* max HSS leaf size (Sec. 4.2, b) */
  int32_t min_sep_hss; /* a front is HSS iff its separator has at least this
                          many indices; large value = pure multifrontal */
  int32_t d0;          /* initial number of random vectors (Sec. 2.2) */
  int32_t dd;          /* growth step Delta d of the adaptive scheme (Sec. 4.3) */
  int32_t p;           /* oversampling: an ID of rank k succeeds iff k <= d - p
                          or k equals the node's row count */
  int32_t d_max;       /* cap on d; reaching it gives HSSMF_ERANK */
  uint64_t seed;       /* key of the counter-based Gaussian generator of R */
  int32_t gemm_prec;   /* HSSMF_PREC_*: sampling / ULV product precision */
  int32_t outer;       /* HSSMF_OUTER_IR or HSSMF_OUTER_GMRES */
  int32_t restart;     /* GMRES restart length (30 in Sec. 6.1; at most 200
                          are used) */
  double tol;          /* stop when ||b - A x||_2 / ||b||_2 <= tol */
  int32_t max_it;      /* max refinement steps / GMRES iterations */
  int32_t id_kernel;   /* HSSMF_ID_*: how the pivoted QR of the IDs runs */
  int32_t use_graph;   /* 1: the preconditioner's forward and backward sweeps
                          are captured once per factorization as a HIP graph
                          (on a private stream) and replayed on the handle's
                          stream; 0 (default): launched one by one */
  int32_t gemm_tile;   /* matrix-core GEMM kernel: 0 = chosen per type and
                          shape class by the built-in autotuner (timed once
                          per process); forced: 64 (64 x 64 tiles; FP64 with
                          k-tiles of 16), 65 (64 x 64, FP64 k-tiles of 32),
                          128 (128 x 128); BF16 products always take 64 x 64;
                          the results do not depend on it */
  double abs_tol;      /* absolute HSS compression tolerance: the rank of an
                          ID stops at |R_{i+1,i+1}| <= max(rel_tol |R_11|,
                          abs_tol) (Sec. 5.3 gives the relative rule; 0, the
                          default, keeps it alone) */
  int32_t keep_stages; /* 1: every numeric factorization keeps copies of each
                          HSS front's random matrix, samples and low-rank
                          Schur factors for hssmf_front_data (device memory
                          of O(n d + m_k u) per front); 0 (default): not */
  int32_t hss_update;  /* HSSMF_UPDATE_*: how an HSS front's update matrix
                          F22 - Theta^* Phi reaches an HSS parent */
  int32_t power_q;     /* steps of power iteration in the sampling (Sec. 2.2,
                          the variant the paper describes as an option):
                          S^r = (F F^T)^q F R, S^c = (F^T F)^q F^T R, and
                          Alg. 1 takes R^r = F^T (F F^T)^(q-1) F R on the row
                          side, R^c = F (F^T F)^(q-1) F^T R on the column
                          side.  The eps-rank rule then applies to the
                          iterated samples, whose singular values are those
                          of F raised to 2q + 1.  0 (default) = plain
                          sampling; 1..4 need gemm_prec = FP64 (EINVAL
                          otherwise); each step costs four more sampling
                          passes */
  double srrqr_f;      /* strong rank-revealing QR inside every ID (Sec. 2.2
                          and Sec. 7 name it as the replacement of the
                          column-pivoted QR; Gu and Eisenstat's algorithm
                          with the rank k held fixed): after the pivoted QR
                          has fixed k, while some interchange of a selected
                          column i and a remaining column j would multiply
                          |det R11| by more than f, the largest such
                          interchange is made (column i leaves, column j
                          joins as the last selected one) and the QR is
                          redone in that pivot order, at most 64 times per
                          ID.  Afterwards every interpolation coefficient
                          |(R11^{-1} R12)_ij| is at most f.  0 (default) =
                          the pivoted QR alone; otherwise f > 1, which needs
                          the resident ID kernel (EINVAL otherwise; a pass
                          it cannot take fails with EINVAL) */
} hssmf_opts;

/* hss_update: LOWRANK = kept as the HSS generators of F22 with Theta^* and
 * Phi; the parent samples it by an HSS matrix-vector product minus
 * Theta^* (Phi X) and takes its entries from the generators (Sec. 4.4,
 * Sec. 4.5); DENSE = expanded once into a u x u matrix that the parent
 * multiplies and reads.  A dense parent always receives the dense
 * expansion. */
#define HSSMF_UPDATE_LOWRANK 0
#define HSSMF_UPDATE_DENSE 1

/* id_kernel: STEPWISE = one launch per pivot step for each batch of IDs;
 * COOPERATIVE = when every workgroup of a batch fits on the device at once,
 * one cooperative launch that keeps the candidates in registers and passes
 * the partial maxima and the pivot column between workgroups through
 * agent-coherent memory (one launch per step otherwise); RESIDENT = every
 * pivot step of a batch in one launch with each problem's candidates in the
 * registers of as few 512-thread workgroups as hold them (one workgroup,
 * and no exchange between workgroups, for the problems that fit; passes
 * with more than 640 samples, with an ID of more than twice as many
 * columns as the kernel holds sample rows per candidate, or with a problem
 * that needs more workgroups than one cooperative launch holds, take the
 * stepwise kernel).  All take the same
 * pivot rule; they differ only in the order of floating-point sums. */
#define HSSMF_ID_STEPWISE 0
#define HSSMF_ID_COOPERATIVE 1
#define HSSMF_ID_RESIDENT 2

typedef struct {
  int32_t iterations;     /* refinement steps plus GMRES iterations */
  double rel_residual;    /* final ||b - A x|| / ||b|| (FP64) */
  int32_t failed_front;   /* front id for HSSMF_ESINGULAR, else -1 */
  int32_t outer_switched; /* 1 when iterative refinement stagnated (two
                             consecutive steps without the residual falling
                             below 0.9 times the previous one) and handed
                             over to GMRES(restart) from its iterate */
} hssmf_info;

typedef struct {
  int32_t n, nfront, n_hss_fronts, max_rank, max_d, growth_rounds;
  int64_t factor_bytes;     /* device bytes held by the factors */
  double t_plan_ms, t_factor_ms;     /* host planning + upload, numeric factor */
  double flops_factor;      /* algorithmic flops of the numeric factorization */
  int64_t peak_bytes;       /* bound on the device bytes in use during the last
                               numeric factorization: the sum of each of the
                               handle's arenas' high-water marks */
  int32_t trsv_multi_ops;   /* triangular-solve launches of the recorded
                               preconditioner sweeps (both directions, both
                               transposes) that run on several workgroups per
                               system; the others, and every launch captured
                               in a graph, take one workgroup per system */
  int32_t srrqr_swaps;      /* strong-RRQR interchanges made by the last
                               numeric factorization (0 when srrqr_f is 0) */
} hssmf_stats;

/* Fill *o with defaults: rel_tol 1e-6, leaf_size 64, min_sep_hss INT32_MAX
 * (pure multifrontal), d0 128, dd 128, p 10, d_max 4096, seed 0, FP64,
 * iterative refinement, restart 30, tol 1e-10, max_it 50, resident ID
 * kernel (the stepwise one where it does not apply), sweeps launched one by
 * one (no graph), autotuned GEMM tiles, abs_tol 0, update matrices expanded
 * densely, plain sampling (power_q 0), no strong RRQR (srrqr_f 0). */
int hssmf_default_opts(hssmf_opts* o);

/* Symbolic analysis, upload and numeric factorization (Sec. 3.2, Sec. 4).
 * stream: a hipStream_t (may be 0).  On success *out receives a new handle.
 * Errors: EINVAL (bad CSR / ordering / options), ENOMEM, ESINGULAR (zero
 * pivot; the front is reported by hssmf_last_failed_front), ERANK, EDEVICE. */
int hssmf_factor(const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* opts,
                 void* stream, void** out);

/* Many independent systems in one factorization: A[0..nsys), ord[0..nsys)
 * describe the systems as hssmf_factor's arguments would (each ordering in
 * its own numbering).  They are joined into one block-diagonal matrix whose
 * elimination forest has one tree per system (system s owns unknowns
 * [off[s], off[s+1]), see hssmf_systems), so every level of every system's
 * tree and every HSS level of their fronts is factored in the same batched
 * launches (the level batching of Sec. 5 applied across systems).  The
 * random matrix of a system is keyed by its own row numbering, so each
 * system gets the factorization it would get alone.  Vectors
 * of the handle are the systems' vectors back to back; hssmf_refactor takes
 * the systems' values back to back.  The outer solvers stop when every
 * system reaches ||b_s - A_s x_s|| / ||b_s|| <= tol, and report the largest
 * of these.  Errors as hssmf_factor (EINVAL also for nsys < 1). */
int hssmf_factor_batch(int32_t nsys, const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* opts,
                       void* stream, void** out);

/* Number of systems of a handle (1 for hssmf_factor); when cap >= that
 * number + 1, off[0..nsys] receives the first unknown of every system and
 * the total. */
int hssmf_systems(void* h, int64_t* off, int32_t cap);

/* Re-run the numeric factorization with new values (same pattern as the
 * matrix given to hssmf_factor; val has rowptr[n] entries, host memory). */
int hssmf_refactor(void* h, const double* val);

/* A complex sparse system (the Helmholtz problems of Sec. 6.1 use complex
 * arithmetic), factored through its real-equivalent form.  A->val holds
 * 2 rowptr[n] doubles, the (real, imaginary) pair of each stored entry in
 * CSR order; A->mem as for hssmf_factor (values and pattern are read during
 * the call only).  The ordering is the complex system's (perm, separator
 * tree over its n unknowns).  The library forms the real system of 2n
 * unknowns in which complex unknown j becomes unknowns 2j (real part) and
 * 2j + 1 (imaginary part) and entry a + ib becomes the block [a -b; b a]:
 * 4 rowptr[n] stored entries, the ordering expanded alike (every front
 * keeps its unknowns' pairs together, separator sizes double), and factors
 * it as hssmf_factor does (every option applies; leaf_size, min_sep_hss
 * and the ranks count real unknowns).  The handle then behaves as one of
 * 2n real unknowns: a complex vector stored as interleaved (real,
 * imaginary) doubles is exactly that real system's vector, so
 * hssmf_solve and hssmf_apply take and return complex vectors in that
 * storage.  The real form's transpose is the real form of the conjugate
 * transpose: hssmf_solve_transpose and hssmf_apply with trans = 1 solve
 * with A^H.  Errors
 * as hssmf_factor; EINVAL also for n above INT32_MAX / 2.  Products cost
 * about twice the real flops that complex kernels would need. */
int hssmf_factor_z(const hssmf_csr* A, const hssmf_ordering* ord, const hssmf_opts* opts, void* stream,
                   void** out);

/* New complex values for a handle from hssmf_factor_z (same pattern; val:
 * 2 rowptr[n] doubles, (real, imaginary) pairs, host memory).  EINVAL for
 * a handle from hssmf_factor or hssmf_factor_batch. */
int hssmf_refactor_z(void* h, const double* val);

/* hssmf_refactor_z with the complex values already in device memory (2
 * rowptr[n] doubles, (real, imaginary) pairs in CSR order), read on the
 * handle's stream; a kernel forms the real-equivalent values in place of
 * the host.  The caller keeps ownership.  EINVAL as hssmf_refactor_z. */
int hssmf_refactor_z_device(void* h, const double* val_dev);

/* hssmf_refactor with the new values already in device memory: val_dev has
 * rowptr[n] entries in the CSR order given to hssmf_factor, is read on the
 * handle's stream (copied into the handle there) and stays owned by the
 * caller.  HSSMF_EINVAL for a null handle or pointer; otherwise as
 * hssmf_refactor. */
int hssmf_refactor_device(void* h, const double* val_dev);

/* One application of the factorization, y = M^{-1} x (trans = 0) or
 * y = M^{-T} x (trans = 1): the multifrontal forward sweep bottom-up and the
 * backward sweep top-down (Sec. 3.3), with ULV solves on HSS fronts.  x, y:
 * device arrays of n doubles (may alias). */
int hssmf_apply(void* h, int32_t trans, const double* x, double* y);

/* Solve A x = b with the outer solver of the options, iterative refinement
 * or restarted GMRES with modified Gram-Schmidt preconditioned by the
 * factorization (Sec. 4.6, Sec. 6.1; the Arnoldi steps and the Givens
 * rotations run on the device, which reports each step's residual estimate
 * to the host through mapped memory), stopping on the true residual
 * ||b - A x||_2 / ||b||_2 <= tol.  b, x: n x nrhs column-major (column j at
 * offset j n), host or device memory (each pointer's kind is looked up);
 * the right-hand sides are solved one after another.  info: NULL or an
 * array of nrhs records.  Returns the worst status over the right-hand
 * sides: ENOCONV still writes the best x of every column and fills info.
 * EINVAL for nrhs < 0 or null pointers (nrhs = 0 does nothing). */
int hssmf_solve(void* h, int32_t nrhs, const double* b, double* x, hssmf_info* info);

/* Solve A^T lambda = g with the same factors: the multifrontal and ULV
 * sweeps transposed (Sec. 3.3, Sec. 2.3), inside the same outer solver with
 * A^T products.  Arguments as hssmf_solve. */
int hssmf_solve_transpose(void* h, int32_t nrhs, const double* g, double* lambda, hssmf_info* info);

/* Solve every system of an hssmf_factor_batch handle: b[s] and x[s] point to
 * system s's right-hand side and solution (off[s+1] - off[s] doubles each,
 * see hssmf_systems), each host or device memory.  The systems are solved
 * together (their vectors are packed back to back on the device) and the
 * outer solver stops when every system reaches its own tolerance.  info:
 * NULL or one record (worst system).  A single-system handle takes nsys = 1
 * arrays.  EINVAL for null arrays or entries. */
int hssmf_solve_batch(void* h, const double* const* b, double* const* x, hssmf_info* info);

/* Adjoint of x = A^{-1} b for a scalar loss L with gradient g = dL/dx:
 * lambda = A^{-T} g, dl_db = lambda, dl_dval[e] = -lambda[row(e)] x[col(e)]
 * for every CSR entry e.  x, g, dl_db: device arrays of n doubles; dl_dval:
 * device array of nnz doubles. */
int hssmf_adjoint(void* h, const double* x, const double* g, double* dl_db, double* dl_dval,
                  hssmf_info* info);

int hssmf_stats_get(void* h, hssmf_stats* s);

/* Per HSS front (in front order) write up to cap records of 5 int32:
 * front id, max row rank, max column rank, final d, growth rounds.  Returns
 * the number of HSS fronts (>= 0) or a status code. */
int hssmf_hss_ranks(void* h, int32_t* out, int32_t cap);

int hssmf_last_failed_front(void* h);

/* Kernel timing hooks (diagnostics for benchmarks).  While enabled, every
 * launch of the listed kernel classes is made with hipExtLaunchKernelGGL and
 * an event pair that the launch stamps with that kernel's own start and end,
 * and the launches' algorithmic work, computed on the host, is accumulated.  hssmf_profile_read() waits for the recorded
 * events and returns, for one class, the summed kernel time (ms), the number
 * of launches and the summed work (flops).  Reading resets the class.
 * Classes: 0 = pivot steps of the column-pivoted QR behind the
 * interpolative decompositions (one launch per step, work 4dmk - 2k^2(d+m)
 * + 4/3 k^3 per d x m problem truncated at k), 1 = FP64 batched GEMM
 * (matrix cores, 2mnk), 2 = low-precision batched GEMM (2mnk), 3 = panel
 * factorization of the blocked dense LU (m w^2 - w^3/3 per m x w panel),
 * 4 = the same pivot steps when every step of an ID pass runs in one
 * launch (id_kernel = RESIDENT; the launch is bracketed by an event pair,
 * work as for class 0). */
#define HSSMF_KCLASS_ID 0
#define HSSMF_KCLASS_GEMM64 1
#define HSSMF_KCLASS_GEMMLP 2
#define HSSMF_KCLASS_LUPANEL 3
#define HSSMF_KCLASS_ID_RESIDENT 4
int hssmf_profile_enable(int32_t on);
int hssmf_profile_read(int32_t kclass, double* ms, int64_t* launches, double* flops);

/* Intermediate results of one HSS front of the last numeric factorization,
 * for checking each stage of the method on its own (diagnostics; the
 * factorization must have been made with keep_stages = 1, except for
 * HSSMF_STAGE_UPDATE of a front whose update matrix was expanded densely:
 * hss_update = DENSE, or a dense parent).  Rows are the front's local indices: the separator
 * in elimination order, then the update set in ascending new numbering.
 *  RANDOM        R (n x d), the random matrix at the final d (Sec. 2.2.1);
 *  SAMPLES_ROW   S^r = F R (n x d), SAMPLES_COL S^c = F^T R (Eq. FtimesR);
 *  THETA_T       Theta^T (m_k x u) and PHI Phi (m_k x u) of the low-rank
 *                Schur complement F21 F11^-1 F12 ~ Theta^* Phi (Sec. 4.4);
 *  UPDATE        the update matrix F22 - Theta^* Phi (u x u) passed to the
 *                parent.
 * dims[0], dims[1] receive the shape; the column-major array is copied to
 * host memory out when cap (entries) holds it, else only dims are set.
 * EINVAL for a front that is not HSS, an unknown kind, or a kind that was
 * not kept. */
#define HSSMF_STAGE_RANDOM 0
#define HSSMF_STAGE_SAMPLES_ROW 1
#define HSSMF_STAGE_SAMPLES_COL 2
#define HSSMF_STAGE_THETA_T 3
#define HSSMF_STAGE_PHI 4
#define HSSMF_STAGE_UPDATE 5
int hssmf_front_data(void* h, int32_t front, int32_t what, double* out, int64_t cap, int32_t* dims);

/* Machine-peak probes, so that roofline fractions can be quoted against the
 * device as measured as well as against its published figures.  Runs, on
 * the given stream (NULL = the default stream) and the current device:
 * a copy of 512 MiB between two device buffers (hbm_GBps = bytes read plus
 * written per second / 1e9); a loop of independent FP64 fused
 * multiply-adds (fp64_valu_TFLOPs, two flops each); a loop of FP64
 * matrix-core 16 x 16 x 4 products (fp64_mfma_TFLOPs, 2048 flops per
 * wavefront instruction).  Each figure is the best of five timed runs.
 * Allocates and frees 1 GiB of device memory and synchronizes the stream;
 * not for use under graph capture.  HSSMF_EINVAL for out == NULL,
 * HSSMF_EDEVICE when a HIP call fails. */
typedef struct {
  double hbm_GBps;
  double fp64_valu_TFLOPs;
  double fp64_mfma_TFLOPs;
} hssmf_peaks;
int hssmf_measure_peaks(void* stream, hssmf_peaks* out);

/* hssmf_solve without any memory allocation, for callers that cannot
 * allocate device memory (serving loops with a fixed memory budget,
 * harnesses that forbid hipMalloc).  The outer solver's work vectors live in
 * a static device array of HSSMF_NOALLOC_SCRATCH_BYTES per GPU (held until
 * the process ends); the preconditioner sweeps run eagerly (no graph is
 * captured).  b, x: DEVICE arrays, n x nrhs column-major; info as
 * hssmf_solve.  The scratch must hold (restart + 3) n doubles (GMRES, and
 * refinement, which may hand over to GMRES), else HSSMF_ETOOBIG (nothing is
 * launched).  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (other threads or streams) race.  Synchronizes the
 * handle's stream, like hssmf_solve; results are bitwise those of
 * hssmf_solve with use_graph = 0. */
#define HSSMF_NOALLOC_SCRATCH_BYTES (256u << 20)
int hssmf_solve_noalloc(void* h, int32_t nrhs, const double* b, double* x, hssmf_info* info);

/* Algebraic front end (host only; A in host memory, HSSMF_MEM_HOST; no GPU
 * is used).
 *
 * Static scaling and column permutation for stability (Sec. 3.1: A is
 * replaced by Dr A Dc Qc, computed as in MC64 of Duff and Koster): a
 * permutation maximizing the product of the magnitudes of the matched
 * entries, found by shortest augmenting paths on the costs
 * log max_k |a_kj| - log |a_ij|, whose dual variables give the scalings.
 * Outputs (caller-owned, n entries each): colperm[i] = the column of A
 * placed at position i, so B(:, i) = A(:, colperm[i]); row_scale = Dr,
 * col_scale = Dc (indexed by the columns of A).  The scaled, permuted
 * matrix has |r_i a_{i,colperm[i]} c_{colperm[i]}| = 1 on the diagonal and
 * every entry at most 1 in magnitude.  Errors: EINVAL (bad CSR or
 * arguments), ESINGULAR (A is structurally singular: no perfect matching
 * of its nonzero entries). */
int hssmf_static_pivoting(const hssmf_csr* A, int32_t* colperm, double* row_scale, double* col_scale);

/* Fill-reducing nested dissection of the graph of A + A^T (Sec. 3.1) with
 * the separators ordered for HSS compression (Sec. 4.2).  A vertex set of
 * more than leaf_size vertices is split at the middle level of a
 * breadth-first level structure from a pseudo-peripheral vertex (the
 * level's vertices without a neighbour beyond it join the near side); a
 * disconnected set is split off one component at a time.  Each separator
 * of more than sep_leaf vertices is ordered by recursive bisection of its
 * graph enriched with length-two connections: the halves are the first
 * ceil(m / 2) and the remaining vertices of a breadth-first order, down to
 * sep_leaf vertices, which matches the count-halving HSS tree of a front
 * with leaf size sep_leaf.  Outputs as hssmf_ordering, caller-owned: perm
 * (n entries, perm[new] = old), sep_ptr (at least n + 1), parent (at least
 * n), *nfront; fronts in postorder, at most two children each.  Errors:
 * EINVAL. */
int hssmf_nested_dissection(const hssmf_csr* A, int32_t leaf_size, int32_t sep_leaf, int32_t* perm,
                            int32_t* sep_ptr, int32_t* parent, int32_t* nfront);

void hssmf_destroy(void* h);

const char* hssmf_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* HSSMF_H */
