/*
 * spike.h -- C ABI of the MI355X recursive SPIKE banded solver.
 *
 * Solves A X = F and A^T X = F for an n x n banded matrix A with kl
 * subdiagonals and ku superdiagonals, given in LAPACK band storage, for any
 * number of leaf partitions p >= 1 (powers of two or not).  The method is the
 * recursive SPIKE algorithm of Spring, Polizzi and Sameh, "A Feature Complete
 * SPIKE Banded Algorithm and Solver" (arXiv:1811.03559):
 *
 *   - A = D S: D holds the p diagonal blocks A_i, S the spikes
 *     V_i = A_i^{-1} B_i and W_i = A_i^{-1} C_i (section "Central concept of
 *     SPIKE", eqs. partitioning, BandChats, spikes);
 *   - blocks 1..p-1 are factored LU and block p UL (section "Optimizing
 *     per-partition costs"), non-pivoting with diagonal boosting or with
 *     partial pivoting (section "An efficient pivoting scheme"; UL through the
 *     reversal permutation Q of eq. Qmat);
 *   - only spike tips are formed, with truncated sweeps (Table tab:sweeps);
 *   - the reduced system is solved recursively, S^[l] = D^[l] S^[l+1]
 *     (section "Recursive reduced system", eqs. RED_SYS_RECA/RED_SYS_RECB,
 *     D1Inverse, S2Inverse), here over a balanced merge tree valid for any
 *     p, or over the thread distribution of section "Flexible partitioning
 *     scheme for recursive SPIKE" for its admissible p = 2^m + r;
 *   - the transpose solve reuses the same factorisation,
 *     A^T = S^T D^T (section "Transpose solve option", eqs. gform1/gform2,
 *     ATF, sweeps_in_D, transred1/transred2).
 *
 * All device pointers are allocated by the caller.  The library never
 * allocates device memory: the factorisation lives in a caller-provided
 * workspace whose size spike_workspace_size() reports.
 *
 * Calls that take a stream are asynchronous: they validate arguments on the
 * host, enqueue kernels on the stream and return.  Numerical status (zero
 * pivots, boosts, refinement) is written on the device and read with
 * spike_info() after the stream has been synchronised.
 *
 * Return codes: 0 on success; -i when argument i is invalid (LAPACK style,
 * 1-based position in the call); SPIKE_ERR_HIP - e (e = hipError_t) when a
 * HIP runtime call or launch fails.
 */
#ifndef SPIKE_H
#define SPIKE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPIKE_ERR_HIP (-1000)

#ifndef SPIKE_API
#define SPIKE_API __attribute__((visibility("default")))
#endif

typedef struct spike_handle_s *spike_handle;

/* Options.  spike_default_opts() fills the defaults given in brackets. */
typedef struct spike_opts {
    int32_t p;          /* leaf partitions; 0 = planner's choice          [0]    */
    int32_t pivot;      /* 0 = non-pivoting LU/UL with diagonal boosting,
                           1 = partial pivoting inside each block         [0]    */
    int32_t precision;  /* 0 = FP64 throughout; 1 = FP32 block factors and
                           sweeps, FP64 reduced system, FP64 residual and
                           iterative refinement                           [0]    */
    int32_t sizing;     /* 0 = equal partitions; 1 = sizes from the paper's
                           load-balancing ratios computed from K and
                           nrhs_hint (R13, eq. R13_calculation, and
                           R12 = R13 / 2); 2 = sizes from the explicit
                           ratios r12 and r13 below.  First and last
                           partitions get n1, two-thread partitions of the
                           paper layout (tree 1) n2, split in two leaves,
                           single-thread inner partitions n3, with
                           n1 = n R12 R13 / (2 R12 R13 + x R13 + y R12),
                           n2 = n1 / R12, n3 = n1 / R13 (x two-thread, y
                           single-thread inner partitions)                [0]    */
    double K;           /* solve/factor cost constant K = K2/K1 used by
                           R13 sizing; <= 0 selects 1.0                   [0]    */
    int32_t nrhs_hint;  /* expected nrhs for R13 sizing; 0 = unknown       [0]    */
    int32_t nrhs_max;   /* largest nrhs handled in one pass; larger solves
                           are split into passes; sizes the workspace    [64]    */
    double boost_tau;   /* non-pivoting only: a pivot with |u_jj| <
                           boost_tau * ||A_i||_1 is boosted by that amount
                           (sign kept); 0 disables boosting; < 0 selects
                           sqrt(unit roundoff of the factor precision)  [-1]    */
    int32_t max_refine; /* FP64 iterative-refinement iteration cap; < 0
                           selects 6 with precision 1 and 0 (no
                           refinement) with precision 0.  A positive value
                           with precision 0 refines every solve (useful
                           after boosted pivots or for ill-conditioned A,
                           where SPIKE loses accuracy).  Refinement stops
                           at refine_tol, at the cap, on a non-finite
                           residual, or when the backward error fails to
                           halve in an iteration.  Refinement needs the
                           caller's dAB to stay valid                    [-1]    */
    double refine_tol;  /* backward-error target of refinement        [1e-13]    */
    int32_t tree;       /* shape of the reduced-system merge tree:
                           0 = balanced: at every level adjacent nodes
                           pair left to right, an odd last node carries
                           up; any p.
                           1 = the paper's flexible-threading layout
                           (distribution of threads, flexible
                           partitioning section): p = 2^m + r leaves
                           with 0 <= r <= 2^m - 2; leaves 1..2r (0-based)
                           are the halves of r inner two-thread
                           partitions, placed from the second partition
                           on, and merge first; a complete binary tree
                           then runs over the 2^m nodes.  Any other p is
                           an error (-4); with p = 0 the planner's count
                           is lowered to the nearest admissible one.  [0] */
    double r12;         /* sizing 2: n1 / n2 (> 0)                        [0]    */
    double r13;         /* sizing 2: n1 / n3 (> 0)                        [0]    */
} spike_opts;

/* Device-side status, read by spike_info() (blocking copy). */
typedef struct spike_status {
    int64_t info;       /* 0; i in [1, n]: first exactly-zero pivot at global
                           row i (1-based), boosting off or pivoting;
                           n + j, j in [1, p-1]: the interface system of
                           merge j is singular, merge j being the one
                           between partitions j and j+1 (1-based), i.e.
                           the first with an exactly-zero pivot in its
                           partial-pivoting LU                           */
    int32_t n_boosts;   /* pivots boosted during the factorisation        */
    int32_t refine_iters; /* refinement iterations of the last solve      */
    double min_abs_pivot; /* smallest |u_jj| over all blocks              */
    double berr;        /* backward error of the last refined solve, or -1 */
} spike_status;

/* Partition plan, as computed by the host planner (no device access). */
typedef struct spike_plan_info {
    int32_t p;          /* leaf partitions                                */
    int32_t levels;     /* depth of the reduced-system merge tree         */
    int32_t merges;     /* number of 2x2-block interface systems (= p-1)  */
    int64_t reduced_size; /* unknowns of the reduced system, (kl+ku)(p-1) */
    size_t workspace_bytes;
} spike_plan_info;

/* Fill *opts with the defaults above. */
SPIKE_API void spike_default_opts(spike_opts *opts);

/* Host-only planner query.  Writes the plan summary to *out and, when
 * sizes is not NULL, the p partition sizes (int64) in order.  sizes must hold
 * at least p entries when opts->p > 0, else 4096.  Touches no device.
 * Errors: -1 n < 0, -2 kl < 0, -3 ku < 0, -4 bad opts (p < 0, p > n, a
 * partition smaller than kl+ku, an unknown mode, with tree 1 a p that is
 * not 2^m + r with r <= 2^m - 2, or partial pivoting with bandwidths too wide
 * for 32-column panels in 128 KiB of LDS, i.e. when 32 (32 + max(kl,ku)) +
 * 32 (kl + ku) elements of the factor precision exceed 128 KiB: in FP64
 * with kl = ku, max(kl,ku) > 160). */
SPIKE_API int spike_plan_query(int64_t n, int32_t kl, int32_t ku, const spike_opts *opts,
                     spike_plan_info *out, int64_t *sizes);

/* Host-only query of the merge tree the planner builds for these options.
 * Writes, for each of the p - 1 interface systems in launch order (level 1
 * first), four int32: the tree level (1 = merges of leaves), the first leaf
 * a of the merged node, the interface index m (the left child spans leaves
 * a..m, the right child m+1..b) and the last leaf b.  merges must hold
 * 4 (p - 1) entries (p as reported by spike_plan_query).  Touches no
 * device.  Same errors as spike_plan_query. */
SPIKE_API int spike_plan_tree(int64_t n, int32_t kl, int32_t ku, const spike_opts *opts,
                    int32_t *merges);

/* Bytes of device workspace spike_factor() needs.  Same errors as
 * spike_plan_query. */
SPIKE_API int spike_workspace_size(int64_t n, int32_t kl, int32_t ku,
                         const spike_opts *opts, size_t *bytes);

/* Factor A (recursive SPIKE factorisation stage: block factors, spike tips,
 * recursive reduced-system factors).
 *   n, kl, ku   order and bandwidths (n >= 0, kl >= 0, ku >= 0)
 *   dAB         device, read-only: LAPACK band storage, column-major,
 *               A(i,j) at dAB[(ku + i - j) + j*ldab], ldab >= kl+ku+1.  With
 *               precision 1 the refinement residual reads dAB, so it must stay
 *               valid and unchanged until spike_destroy.
 *   opts        NULL for defaults
 *   dWork       device workspace of work_bytes >= spike_workspace_size(),
 *               256-byte aligned, owned by the caller, holding the
 *               factorisation until spike_destroy
 *   stream      HIP stream all work is enqueued on
 *   out         receives a host handle (host memory owned by the library)
 * Errors: -1..-3 as above, -4 dAB NULL, -5 ldab too small, -6 bad opts,
 * -7 dWork NULL or misaligned, -8 work_bytes too small, -10 out NULL. */
SPIKE_API int spike_factor(int64_t n, int32_t kl, int32_t ku, const double *dAB,
                 int64_t ldab, const spike_opts *opts, void *dWork,
                 size_t work_bytes, hipStream_t stream, spike_handle *out);

/* Batched factorisation: the factor stage of count systems, each as
 * spike_factor would factor it (its own n, bands, options, workspace and
 * handle), with the systems that share a kernel configuration (non-pivoting
 * factors on the matrix-core block LU, equal kl and ku, the same precision)
 * factored by common launches: one launch per kernel of the stage covers up
 * to 32 of them, so that many small systems fill the GPU together (the
 * batched form of the factorisation stage, section "Recursive SPIKE").
 * Other systems are factored one after the other on the same stream.
 *   n, kl, ku, dAB, ldab, dWork, work_bytes, out   arrays of count entries,
 *               each as the argument of the same name of spike_factor
 *   opts        array of count options, or NULL for the defaults
 * Returns 0, or the spike_factor error code of the first system with a bad
 * argument (nothing is launched and no handle is created), -11 count < 0,
 * -12 an array NULL, -1000-hipError. */
SPIKE_API int spike_factor_batch(int32_t count, const int64_t *n, const int32_t *kl, const int32_t *ku,
                                 const double *const *dAB, const int64_t *ldab, const spike_opts *opts,
                                 void *const *dWork, const size_t *work_bytes, hipStream_t stream,
                                 spike_handle *out);

/* Solve A X = F in place: dB (device, column-major n x nrhs, ldb >= n) holds
 * F on entry and X on exit.  Uses the handle's workspace; calls on one handle
 * must be ordered (same stream or synchronised).  If the factorisation
 * reported info != 0 the kernels leave dB untouched.
 * Errors: -1 bad handle, -2 nrhs < 0, -3 dB NULL (with nrhs > 0), -4 ldb < n. */
SPIKE_API int spike_solve(spike_handle h, int32_t nrhs, double *dB, int64_t ldb,
                hipStream_t stream);

/* Solve A^T X = F in place with the same factorisation (transpose S stage,
 * transpose recursive reduced system, transpose D stage).  Arguments and
 * errors as spike_solve. */
SPIKE_API int spike_solve_transpose(spike_handle h, int32_t nrhs, double *dB,
                          int64_t ldb, hipStream_t stream);

/* Copy the device status to *out (blocking device-to-host copy; synchronise
 * the factor/solve stream first).  Errors: -1 bad handle, -2 out NULL. */
SPIKE_API int spike_info(spike_handle h, spike_status *out);

/* Plan of an existing handle (host data, no device access). */
SPIKE_API int spike_handle_plan(spike_handle h, spike_plan_info *out);

/* Kernel timing (profiling aid).  spike_profile_enable(1) clears previous
 * records and, until spike_profile_enable(0), brackets every kernel launch of
 * the library with HIP events recorded on the launch stream.
 * spike_profile_report() waits for the recorded events and writes, per
 * kernel name, the number of launches and their summed duration (up to cap
 * entries; *count receives the number of distinct kernels).
 * spike_profile_only(name) restricts the brackets to launches of the kernel
 * of that name (NULL or "" for all), so that a timed loop carries the events
 * of one kernel only; it applies from the next spike_profile_enable(1).
 * Errors: -1 name longer than 47 characters. */
typedef struct spike_kernel_time {
    char name[48];
    int32_t calls;
    double total_ms;
} spike_kernel_time;

SPIKE_API int spike_profile_enable(int on);
SPIKE_API int spike_profile_only(const char *name);
SPIKE_API int spike_profile_report(spike_kernel_time *out, int cap, int *count);

/* Complex banded systems (the complex precisions of the paper's library,
 * section "Introduction": double complex, and single complex through
 * precision 1, FP32 factors with FP64 refinement).  A complex band A
 * (kl, ku) acts on interleaved unknowns like the real 2n x 2n band with
 * 2 x 2 blocks [[Re a, -Im a], [Im a, Re a]] (2 kl + 1 sub- and 2 ku + 1
 * superdiagonals), and the factorisation is the SPIKE factorisation of that
 * real band, built on the device from the complex one.  Its transpose is
 * the band of A^H, so the same factors solve A^H z = f directly and
 * A^T z = f as A^H conj(z) = conj(f).  Each row j is first multiplied by
 * the unit-modulus conj(a_jj) / |a_jj| (the factors are those of D A, D
 * unitary and diagonal), which makes the diagonal real and positive: for a
 * diagonally dominant A the non-pivoting elimination of the embedding then
 * meets no small pivots inside its 2 x 2 blocks.
 *   dAB   device complex band, LAPACK zgb layout with interleaved real and
 *         imaginary doubles: A(i,j) = dAB[2 ((ku + i - j) + j ldab)] +
 *         i dAB[2 ((ku + i - j) + j ldab) + 1], ldab >= kl + ku + 1 (in
 *         complex elements).  Read during spike_zfactor only (the
 *         refinement residual of precision 1 reads the embedded real band,
 *         which lives in dWork).
 *   opts  as spike_factor, for the real embedding (partition sizes, p,
 *         pivoting and precision refer to it: p partitions of the 2n real
 *         rows; a zero-pivot info i refers to real row i, complex row
 *         (i + 1) / 2)
 *   dWork device, work_bytes >= spike_zworkspace_size, 256-byte aligned.
 * spike_zsolve: dB device complex n x nrhs, interleaved, column-major with
 * leading dimension ldb (in complex elements, >= n), overwritten with the
 * solution of op(A) Z = F: trans 0 = A, 1 = A^T, 2 = A^H.  The handle is
 * used with spike_info and spike_destroy as usual.
 * Errors: as spike_factor / spike_solve; spike_zsolve -1 also for a handle
 * that is not complex, -5 a bad trans. */
SPIKE_API int spike_zworkspace_size(int64_t n, int32_t kl, int32_t ku, const spike_opts *opts,
                                    size_t *bytes);
SPIKE_API int spike_zfactor(int64_t n, int32_t kl, int32_t ku, const double *dAB, int64_t ldab,
                            const spike_opts *opts, void *dWork, size_t work_bytes,
                            hipStream_t stream, spike_handle *out);
SPIKE_API int spike_zsolve(spike_handle h, int32_t nrhs, double *dB, int64_t ldb, int32_t trans,
                           hipStream_t stream);

/* Restarted GMRES with the factorisation as preconditioner (a project
 * addition to the paper's boosting scheme: diagonal boosting perturbs the
 * factors, and the paper corrects with an outer iteration, section "An
 * efficient pivoting scheme"; GMRES is the Krylov form of that correction,
 * more robust than refinement when many pivots were boosted).  Solves
 * op(A) X = F in FP64 with the caller's band A (the dAB given to
 * spike_factor, which must still be valid) and the handle's factors M as a
 * right preconditioner: op(A) M^{-1} u = F, X = M^{-1} u, restarted every
 * `restart` Arnoldi steps (classical Gram-Schmidt, reorthogonalised once),
 * until the backward error ||F - op(A) X||_inf / (||op(A)||_inf ||X||_inf)
 * of every column is <= tol or max_iters steps were taken.
 *   h, nrhs, dB, ldb, trans  as spike_solve / spike_solve_transpose;
 *                            nrhs <= the handle's nrhs_max
 *   opts       NULL for the defaults [restart 30, max_iters 300, tol 1e-13]
 *   dWork      device scratch of work_bytes >= spike_krylov_workspace_size,
 *              256-byte aligned (holds the basis: about (restart + 7) n nrhs
 *              doubles)
 *   out        iterations, restarts, whether every column converged, and
 *              the final backward error (max over columns)
 * Blocks the host until done (each Arnoldi step reads its Hessenberg column).
 * Returns 0 (see out->converged), 1 when the factorisation reported
 * info != 0 (dB untouched), -1 bad handle, -2 nrhs < 0 or > nrhs_max, -3
 * dB NULL, -4 ldb < n, -6 bad opts, -7 dWork NULL or misaligned, -8
 * work_bytes too small, -11 out NULL, -1000-hipError. */
typedef struct spike_krylov_opts {
    int32_t restart;      /* basis vectors before a restart (1..500)     [30] */
    int32_t max_iters;    /* cap on Arnoldi steps over all restarts     [300] */
    double tol;           /* backward-error target                    [1e-13] */
} spike_krylov_opts;

typedef struct spike_krylov_result {
    int32_t iters;        /* Arnoldi steps taken                              */
    int32_t restarts;     /* restart cycles completed                         */
    int32_t converged;    /* 1 when every column met tol                      */
    double berr;          /* final backward error, max over columns (NaN if a
                             residual or solution became non-finite)        */
} spike_krylov_result;

SPIKE_API void spike_krylov_default_opts(spike_krylov_opts *opts);
SPIKE_API int spike_krylov_workspace_size(spike_handle h, int32_t nrhs, const spike_krylov_opts *opts,
                                          size_t *bytes);
SPIKE_API int spike_solve_gmres(spike_handle h, int32_t nrhs, double *dB, int64_t ldb, int32_t trans,
                                const spike_krylov_opts *opts, void *dWork, size_t work_bytes,
                                hipStream_t stream, spike_krylov_result *out);

/* Factorisation without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same as spike_factor, but the
 * factorisation lives in the library's own device scratch array of
 * spike_scratch_capacity() bytes (64 MiB), one copy per GPU, held from the
 * library's load until the process ends; the call allocates no device
 * memory.  Every call on one GPU shares that GPU's array: a later call
 * overwrites the factorisation an earlier handle on the same GPU points to
 * (use or destroy earlier handles first), and calls that overlap on one GPU
 * race.  The handle is used with spike_solve, spike_solve_transpose,
 * spike_info and spike_destroy as usual; with precision 1 dAB must stay
 * valid while it is used.
 * Errors: -1..-5 as spike_factor, -6 bad opts, -7 the factorisation needs
 * more than spike_scratch_capacity() bytes (spike_workspace_size reports
 * the need), -8 out NULL, -1000-hipError (the scratch address or a launch). */
SPIKE_API size_t spike_scratch_capacity(void);
SPIKE_API int spike_factor_scratch(int64_t n, int32_t kl, int32_t ku, const double *dAB,
                                   int64_t ldab, const spike_opts *opts, hipStream_t stream,
                                   spike_handle *out);

/* Instrumented sweep counts, the measurement behind Table tab:sweeps of
 * section "Optimizing per-partition costs" (full triangular sweeps per
 * partition in the factorisation and solve stages; the transpose section
 * states the transpose solve keeps the same counts).
 * spike_sweep_counting(on): while on is nonzero, every later spike_factor
 * sets up its handle to count, on the device, each triangular sweep of one
 * column set (a spike block or the right-hand sides) over one partition's
 * factors, in every kernel path (single and multiple right-hand sides,
 * pivoting or not, batched or not).  Off by default; handles keep the
 * setting they were made with.  Returns 0.
 * spike_sweep_counts(h, out) (blocking copy; synchronise first) writes 24
 * counters, out[(stage * 4 + type) * 2 + full]: stage 0 = factorisation,
 * 1 = spike_solve, 2 = spike_solve_transpose (summed over all calls on h);
 * type 0 = single partition (p = 1), 1 = first, 2 = middle, 3 = last; full
 * 1 = the sweep ran over all rows of the partition, 0 = a truncated sweep
 * over its trailing rows.  Errors: -1 bad handle, -2 out NULL, -3 h was not
 * made while counting was on. */
SPIKE_API int spike_sweep_counting(int on);
SPIKE_API int spike_sweep_counts(spike_handle h, uint64_t *out);

/* Release the host handle.  The caller may free dWork afterwards (after the
 * stream work using it has completed). */
SPIKE_API int spike_destroy(spike_handle h);

/* Batched solve stage (a project addition around the paper's solve stage:
 * the D stage, recursive reduced solve and retrieval, or their transposes).
 * For s = 0 .. count-1 solves op(A_s) X_s = F_s in place, A_s being the
 * factorisation held by hs[s], op = transpose when trans[s] != 0:
 *   hs[s]    handles from spike_factor (distinct systems may have different
 *            n, bandwidths, partitions and precision)
 *   nrhs[s]  columns of dB[s] (>= 0); ldb[s] >= max(1, n_s)
 *   dB[s]    device, column-major n_s x nrhs[s], overwritten with X_s.
 * Systems that share the kernel configuration (precision, window heights,
 * operation) run each phase of the solve as one launch over all their
 * partitions (or all their merges of one tree level), up to 32 systems per
 * launch; the others are solved one after another.  Results are bitwise those
 * of spike_solve / spike_solve_transpose on each system alone.  Systems must
 * not share workspaces or right-hand sides.  Asynchronous on `stream`.
 * Errors: -1 hs NULL or an invalid handle, -2 nrhs NULL or negative, -3 dB
 * NULL (or dB[s] NULL with work to do), -4 ldb NULL or too small, -5 trans
 * NULL, -6 count < 0, -1000-hipError on launch errors. */
SPIKE_API int spike_solve_batch(const spike_handle *hs, const int32_t *nrhs,
                                double *const *dB, const int64_t *ldb,
                                const int32_t *trans, int32_t count,
                                hipStream_t stream);

/* Solve stage captured once into a HIP graph and replayed (callers that
 * repeat the same solve on the same buffers, e.g. inside a time loop).  The
 * capture records exactly the launches of spike_solve_batch (or of one
 * spike_solve / spike_solve_transpose) with the given arguments on `stream`
 * (a non-null stream that is not already capturing); nothing runs during the
 * capture.  spike_graph_launch replays it on any stream: it reads dB[s] as F
 * and overwrites it with X, exactly like the eager call.  Handles with
 * refinement enabled are rejected (-1).  The handles, workspaces and dB
 * buffers must outlive the graph.  Errors as spike_solve_batch, plus -7 null
 * stream, -8 out NULL, -1000-hipError from capture or instantiation. */
typedef struct spike_graph_s *spike_graph;

/* Autotuner (a project addition to the load-balancing section, whose machine
 * constant K is measured here rather than assumed).  Times factorisation +
 * solve of candidate plans on the caller's matrix and device: partition
 * counts around the number of compute units and the planner's default, equal
 * sizing, each with the balanced tree and, where the count admits it, the
 * paper's 2^m + r thread layout; estimates K = (solve ms * max(kl,ku)) /
 * (factor ms * nrhs) from the fastest one and times that p again with R13
 * sizing at that K.  Blocks the host until each timing is done.  Results are
 * kept in a process-wide cache keyed by (n, kl, ku, floor(log2 nrhs),
 * precision, pivot): a later call with the same key returns the cached
 * options and timings without timing anything (out->cached = 1).
 *   dAB, ldab   the matrix (as spike_factor)
 *   nrhs        columns of the solves to tune for (>= 1)
 *   base        options to start from (NULL: defaults); p and sizing are
 *               tuned, everything else is kept
 *   dWork       workspace of work_bytes; candidates needing more are skipped
 *               (spike_autotune_workspace_size gives the size that fits all)
 *   dB, ldb     device n x nrhs scratch for the timed solves (overwritten)
 *   out         best options and their timings, K, candidates timed.
 * Errors: -1 n < 1, -2 kl < 0, -3 ku < 0, -4 dAB NULL, -5 ldab too small,
 * -6 nrhs < 1, -8 dWork NULL, -9 no candidate fits, -10 dB NULL or ldb < n,
 * -13 out NULL, or the error of a failing factor/solve. */
typedef struct spike_tune_result {
    spike_opts opts;
    double factor_ms;
    double solve_ms;
    double K;
    int32_t candidates;
    int32_t cached;     /* 1: taken from the tuning cache, nothing was timed */
} spike_tune_result;

/* The tuning cache (a project addition for serving: a tuned plan is reused
 * for every later system of the same shape).  spike_tune_cache_clear empties
 * it; spike_tune_cache_save writes it to a text file, one entry per line:
 *   n kl ku log2_nrhs precision pivot p sizing tree K nrhs_hint r12 r13
 *   factor_ms solve_ms candidates
 * and spike_tune_cache_load merges such a file into it (an entry replaces
 * one of the same key).  spike_tune_cache_size reports the entry count.
 * Errors: -1 path NULL, -2 the file cannot be opened, -3 a malformed line
 * (entries before it are kept). */
SPIKE_API int spike_tune_cache_clear(void);
SPIKE_API int spike_tune_cache_size(void);
SPIKE_API int spike_tune_cache_save(const char *path);
SPIKE_API int spike_tune_cache_load(const char *path);

SPIKE_API int spike_autotune_workspace_size(int64_t n, int32_t kl, int32_t ku,
                                            const spike_opts *base, size_t *bytes);
SPIKE_API int spike_autotune(int64_t n, int32_t kl, int32_t ku, const double *dAB,
                             int64_t ldab, int32_t nrhs, const spike_opts *base,
                             void *dWork, size_t work_bytes, double *dB,
                             int64_t ldb, hipStream_t stream,
                             spike_tune_result *out);
SPIKE_API int spike_graph_capture_batch(const spike_handle *hs,
                                        const int32_t *nrhs, double *const *dB,
                                        const int64_t *ldb, const int32_t *trans,
                                        int32_t count, hipStream_t stream,
                                        spike_graph *out);
SPIKE_API int spike_graph_capture_solve(spike_handle h, int32_t nrhs, double *dB,
                                        int64_t ldb, int32_t trans,
                                        hipStream_t stream, spike_graph *out);
SPIKE_API int spike_graph_launch(spike_graph g, hipStream_t stream);
SPIKE_API int spike_graph_destroy(spike_graph g);

/* Serving runtime (a project addition: many requests of mixed n, bandwidth
 * and nrhs on one GPU, reusing the paper's factor-once, solve-many structure
 * (factorisation reused by the transpose solve, section "Transpose solve
 * option") across requests).  The caller hands the server a device pool of
 * hbm_budget bytes (the library allocates no device memory); the server
 * carves factorisation workspaces out of it, keeps them resident per matrix id and
 * evicts idle ones least-recently-used when a new matrix needs room.  A
 * worker thread admits queued requests while request slots and pool memory
 * are free (continuous batching: requests that arrive while others run are
 * admitted as slots free up), orders all work on one matrix on that matrix's
 * stream, and launches the admitted solves of one stream as one batched
 * solve.  Results are bitwise those of factoring and solving each request
 * alone with the same options.  Admission is first-come first-served when
 * pool memory is short: a request waiting for room holds back the requests
 * queued after it.  The server's streams do not wait for the caller's: dAB
 * and dB must hold their data (synchronised) when a request is submitted,
 * and dB must not be touched until the request is done.  The numerical
 * status (info) is read once per factorisation with a synchronous copy. */
typedef struct spike_server_s *spike_server;

typedef struct spike_server_opts {
    size_t hbm_budget;    /* device bytes for resident factorisations  [16 GiB] */
    int32_t max_inflight; /* requests on the device at once              [64] */
    int32_t streams;      /* device streams work is spread over (1..16)   [4] */
    int32_t batch_window; /* solves fused into one batched launch        [32] */
    void *dpool;          /* device pool of hbm_budget bytes, 256-byte
                             aligned, allocated by the caller and kept
                             alive until spike_server_destroy returns;
                             required                                 [NULL] */
} spike_server_opts;

typedef struct spike_request {
    int64_t matrix_id;    /* caller's id of A: same id = same matrix, reuse   */
    int64_t n;
    int32_t kl, ku;
    const double *dAB;    /* device band (spike_factor layout); must stay
                             valid while the id may be (re)factored          */
    int64_t ldab;
    spike_opts opts;      /* factorisation options (first request of an id)  */
    int32_t nrhs;         /* >= 1 */
    double *dB;           /* device n x nrhs: F in, X out                    */
    int64_t ldb;
    int32_t trans;        /* != 0: solve A^T X = F                           */
} spike_request;

typedef struct spike_request_status {
    int32_t state;        /* 0 queued, 1 on the device, 2 done, 3 failed     */
    int32_t error;        /* failure code: -100 larger than the budget,
                             -101 the id is resident for a matrix of other
                             n, kl, ku or dAB; else a spike_factor or
                             spike_solve_batch code                          */
    int64_t info;         /* spike_status.info of the factorisation          */
    double latency_s;     /* submission to observed completion, -1 if open   */
} spike_request_status;

typedef struct spike_server_report {
    int64_t completed, failed, factorizations, evictions, resident;
    size_t hbm_used, hbm_high_water;
    double p50_s, p99_s, max_s;   /* latency percentiles of completed requests */
    double solves_per_s;          /* completed / (last completion - first submission) */
} spike_server_report;

SPIKE_API void spike_server_default_opts(spike_server_opts *opts);
/* Creates the server's streams and worker thread.  Errors: -1 bad options
 * (including a NULL or misaligned dpool), -2 out NULL, -1000-hipError
 * (stream creation). */
SPIKE_API int spike_server_create(const spike_server_opts *opts, spike_server *out);
/* Queue a request (non-blocking).  Errors: -1 bad server, -2 bad request,
 * -3 ticket NULL. */
SPIKE_API int spike_server_submit(spike_server s, const spike_request *req,
                                  int64_t *ticket);
/* Status without waiting / after waiting for completion.  -2 unknown ticket. */
SPIKE_API int spike_server_poll(spike_server s, int64_t ticket,
                                spike_request_status *st);
SPIKE_API int spike_server_wait(spike_server s, int64_t ticket,
                                spike_request_status *st);
/* Forget a finished request (-3 if it is not finished). */
SPIKE_API int spike_server_release(spike_server s, int64_t ticket);
/* Wait until every queued request has finished. */
SPIKE_API int spike_server_drain(spike_server s);
SPIKE_API int spike_server_stats(spike_server s, spike_server_report *out);
/* Finish queued work, release every factorisation and the pool. */
SPIKE_API int spike_server_destroy(spike_server s);

#ifdef __cplusplus
}
#endif

#endif /* SPIKE_H */
