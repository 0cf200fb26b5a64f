/*
 * dfjk.h -- C ABI of the MI355X (gfx950) density-fitted Coulomb/exchange build.
 *
 * One SCF iteration of GPU-accelerated Kohn-Sham/Hartree-Fock with density
 * fitting needs J and K from the current density.  The paper this library
 * follows (GPU4PySCF v1.0) describes the path only in words (Introduction:
 * three-centre integrals for density fitting, then tensor contractions on
 * matrix units; "Dataset and Performance": integrals kept resident in GPU
 * memory for small systems; "Limitations and Future Development / Mixed
 * Precision": single precision guided by Schwarz estimates).  The quantities
 * computed are the standard Coulomb-metric fitting formulas:
 *
 *   U_{P,mu nu} = (mu nu|P)          three-centre integrals, Schwarz screened
 *   V = (P|Q) = L L^T                metric and its Cholesky factor
 *   B = L^{-1} U                     whitened three-centre tensor
 *   c_P = sum_{mu nu} B_{P,mu nu} D_{mu nu};   J_{mu nu} = sum_P B_{P,mu nu} c_P
 *   K_{mu nu} = sum_P sum_{la si} B_{P,mu la} D_{la si} B_{P,si nu}
 *             = 2 sum_{P,i} X_{P,i mu} X_{P,i nu},  X_{P,i mu} = sum_nu B_{P,mu nu} C_{nu i}
 *   E_J = 1/2 Tr(D J),  E_K = -1/4 Tr(D K),  D = 2 C C^T when C is given.
 *
 * Conventions.  Units are Bohr and Hartree.  Every shell is one uncontracted
 * primitive; functions are unit-normalised real solid harmonics (Racah
 * normalisation) times a Gaussian, AO order follows the caller's shell order,
 * p functions are (x, y, z) and d/f functions run m = -l..l.  AO l <= 2, aux
 * l <= 3.  All matrices are row-major doubles.
 *
 * Memory.  The caller owns every device buffer (the Python binding allocates
 * them with torch); the library owns only the opaque plan (host metadata) and
 * borrows each workspace for as long as the call (or, for the resident
 * workspace, the plan) needs it.  The library never allocates device memory
 * itself.  Device pointers must come from hipMalloc (or torch) on the device
 * that is current when the call is made.
 *
 * Streams.  `stream` is a hipStream_t passed as void*; NULL is the default
 * stream.  Calls enqueue work and return; outputs are valid once the stream
 * has reached them.  dfjk_screen and dfjk_setup synchronise the stream before
 * they return (the host needs the screening result and the Cholesky status).
 *
 * Errors.  Every call returns a dfjk_status.  Arguments are validated before
 * any work is enqueued, and output buffers are left untouched when validation
 * fails.  dfjk_last_error() returns a thread-local message describing the
 * last failure on the calling thread.
 */
#ifndef DFJK_H
#define DFJK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DFJK_OK = 0,
    DFJK_E_INVALID = 1,      /* bad argument (NULL pointer, size, ...)          */
    DFJK_E_UNSUPPORTED = 2,  /* angular momentum or size beyond this version     */
    DFJK_E_NOT_POSDEF = 3,   /* metric Cholesky met a pivot <= 0 (index in msg) */
    DFJK_E_OOM = 4,          /* a workspace smaller than the size query asked    */
    DFJK_E_DEVICE = 5,       /* a HIP runtime error (HIP message in the text)    */
    DFJK_E_NO_DEVICE = 6,    /* no GPU visible                                   */
    DFJK_E_STATE = 7         /* call out of order (e.g. build before setup)      */
} dfjk_status;

typedef enum {
    DFJK_FP64 = 0,           /* every step in FP64                              */
    DFJK_MIXED_FP32 = 1,     /* X stored FP32, K on FP32 MFMA, FP64 chunk sums   */
    DFJK_MIXED_BF16X3 = 2,   /* X split into BF16 hi+lo, K = hi.hi + hi.lo +
                                lo.hi on BF16 MFMA, FP32 chunks, FP64 sums       */
    DFJK_MIXED_INT8 = 3      /* X split into five int8 slices a_0..a_4 under a
                                power-of-two scale per 256-element block of
                                each row (Ozaki scheme); K from the 15 slice
                                products a_i b_j with i + j <= 4 on int8 MFMA
                                with exact int32 sums, folded into FP64 once
                                per block.  Per product the dropped part is
                                below 2^-33 of the product of the two block
                                scales */,
    DFJK_MIXED_INT8_FAST = 4 /* the same slices, K from the 11 products with
                                i + j <= 3 and a_2 b_2 (a_4 unused; a_2 b_2,
                                a square on the diagonal, is kept so that the
                                dropped part carries no systematic sign): per
                                product the dropped part is below 2^-27 of the
                                product of the two block scales */
} dfjk_precision;

/* One basis (AO or auxiliary): nshell uncontracted shells on atoms. */
typedef struct {
    int32_t nshell;
    const int32_t *shell_atom;   /* atom index of each shell, 0 <= atom < natm */
    const int32_t *shell_l;      /* angular momentum of each shell             */
    const double *shell_exp;     /* Gaussian exponent of each shell, > 0       */
} dfjk_basis;

typedef struct {
    double schwarz_thresh;       /* keep (mu nu|P) iff Q_ab * Q_P >= thresh,
                                    Q the Schwarz factors sqrt|(ab|ab)|,
                                    sqrt (P|P); 0 keeps everything.  Default
                                    1e-14.                                    */
    int32_t aux_slab;            /* aux functions per slab of the K build
                                    (rounded up to 128): the half-transformed
                                    tensor X is formed and contracted one aux
                                    slab at a time, so its memory is
                                    nao * slab * nocc elements.  0 = automatic:
                                    the largest multiple of 128 whose
                                    slab-sized buffers (X, the expanded tensor
                                    of the density route, the second operand
                                    of dfjk_build_delta) stay within 48 GB.
                                    Negative values are DFJK_INVALID.         */
    int32_t k_tile;              /* output tile of the FP64 K contraction
                                    (syrk): 0 = dfjk_autotune's choice for the
                                    shape, else 64 where 128-wide tiles would
                                    execute over 14% more products (ragged
                                    nao), else 128; 64, 96 or 128 = that
                                    tile for every FP64 syrk of the plan.
                                    Other values are DFJK_E_INVALID.          */
} dfjk_options;

typedef struct dfjk_plan dfjk_plan;

/* Plan facts, filled by dfjk_plan_info. */
typedef struct {
    int64_t nao, naux;           /* basis sizes                                */
    int64_t naux_pad;            /* aux dimension as stored (multiple of 64)   */
    int64_t nshell_pairs;        /* AO shell pairs a >= b                      */
    int64_t sig_shell_pairs;     /* pairs surviving screening (after screen)   */
    int64_t nf;                  /* stored function pairs (after screen)       */
    int64_t triplets_kept;       /* shell triplets evaluated (after screen)    */
    int32_t stage;               /* 0 created, 1 screened, 2 set up            */
} dfjk_info;

/* Default options. */
int dfjk_options_default(dfjk_options *opt);

/* Host preparation (no device work): validates the molecule, orders the
 * auxiliary shells by angular momentum and enumerates AO shell pairs.
 * Passage: the paper's problem statement is a PySCF molecule with an AO
 * basis and an auxiliary (fitting) basis, density fitting being its
 * optimised SCF path (Introduction, contribution 1; Section 4.1 "Improved
 * Compatibility with PySCF", the density_fit example).  The paper prints no
 * data structure; the shell tables here are this library's.
 * coords: natm x 3 Bohr.  opt may be NULL (defaults).  *out receives a plan
 * that the caller releases with dfjk_plan_destroy.  Errors: DFJK_E_INVALID
 * for NULL pointers, natm < 1, an atom index out of range, an exponent <= 0
 * or a non-finite coordinate; DFJK_E_UNSUPPORTED for AO l > 2 or aux l > 3. */
int dfjk_plan_create(int32_t natm, const double *coords, const dfjk_basis *ao,
                     const dfjk_basis *aux, const dfjk_options *opt, dfjk_plan **out);

int dfjk_plan_info(const dfjk_plan *plan, dfjk_info *info);

/* The library's internal aux order: out[i] (host array of naux int32) is the
 * caller's aux function index of internal aux function i.  DFJK_EXPORT_CHOL,
 * DFJK_EXPORT_B and the whitened samples of dfjk_sample use this order. */
int dfjk_plan_aux_order(const dfjk_plan *plan, int32_t *out);

/* Schwarz screening.  Passage: the paper ties error control to the Schwarz
 * inequality |(ab|P)| <= sqrt|(ab|ab)| sqrt (P|P) (Section 5 "Limitations
 * and Future Development: Mixed Precision") and attributes the sub-quartic
 * growth of its timings to sparsity (Section 2.1 "Dataset and Performance").
 * dfjk_screen_bytes gives the size of the device scratch dfjk_screen needs;
 * dfjk_screen computes Q_ab for every AO shell pair and Q_P for every aux
 * shell on the GPU, copies them back, and keeps the pairs whose largest
 * triplet bound reaches the threshold.  Synchronises `stream`.  Errors:
 * DFJK_E_INVALID (NULL plan or scratch), DFJK_E_OOM (scratch smaller than
 * dfjk_screen_bytes), DFJK_E_DEVICE (HIP error, message attached). */
int dfjk_screen_bytes(const dfjk_plan *plan, size_t *bytes);
int dfjk_screen(dfjk_plan *plan, void *d_scratch, size_t bytes, void *stream);

/* Per-molecule setup on the resident workspace: three-centre integrals,
 * metric, its Cholesky factor, L^{-1} and the whitened tensor B.  Passage:
 * the three-centre integrals of density fitting computed on the GPU, after
 * which everything is tensor contractions (Introduction, contribution 1),
 * kept resident in GPU memory for small systems (Section 2.1 "Dataset and
 * Performance").  The fitting formulas themselves are the textbook
 * Coulomb-metric ones in the header comment; the paper prints none.  The
 * workspace stays borrowed until dfjk_plan_destroy (or the next setup) and
 * must not be touched by the caller meanwhile.  Returns DFJK_E_NOT_POSDEF
 * with the failing pivot in the message if the metric is not positive
 * definite.  Synchronises `stream`. */
int dfjk_setup_bytes(const dfjk_plan *plan, size_t *bytes);
int dfjk_setup(dfjk_plan *plan, void *d_workspace, size_t bytes, void *stream);

/* dfjk_setup of n screened plans (molecules of any sizes) in one call: the
 * pair records and three-centre integrals of all of them run in shared
 * launches, one per integral class (up to 16 molecules per launch, each
 * workgroup finding its molecule by a prefix table passed by value), then
 * each plan's metric, Cholesky factor, L^{-1} and whitening run on that
 * plan's side stream, beside the other plans' (a chain of small launches
 * each), joined back into `stream`.  Passage: as dfjk_setup; the packing of
 * several molecules into one integral launch is this library's serving form,
 * which the paper does not treat.  plans, d_workspaces, bytes: host arrays of
 * n entries, workspace i as for dfjk_setup of plan i (dfjk_setup_bytes),
 * borrowed alike.  Every plan ends bitwise as after its own dfjk_setup.  The
 * stage profiler records nothing for this call.  Errors, before anything is
 * enqueued: DFJK_E_INVALID (n < 1, a NULL array, pointer or workspace, or a
 * plan given twice), DFJK_E_STATE (a plan not screened, offloaded, or
 * screened on another device), DFJK_E_OOM (a workspace below its
 * dfjk_setup_bytes); the message names the plan.  After the work:
 * DFJK_E_NOT_POSDEF if a metric is not positive definite (the first such plan
 * is named; the other plans are set up).  Synchronises `stream`. */
int dfjk_setup_batch(int32_t n, dfjk_plan *const *plans, void *const *d_workspaces, const size_t *bytes,
                     void *stream);

/* One J/K build: J, K, E_J, E_K from the resident B and the current
 * orbitals or density, once per SCF iteration.  Passage: the tensor
 * contractions after the three-centre integrals, run on matrix units
 * (Introduction, contributions 1 and 2); the lower-precision variants follow
 * Section 5 "Limitations and Future Development: Mixed Precision".
 * Errors: DFJK_E_STATE before dfjk_setup; DFJK_E_INVALID for NULL outputs,
 * both or neither of d_C and d_D, nocc out of range or an unknown
 * precision; DFJK_E_UNSUPPORTED for the density route in a precision other
 * than FP64; DFJK_E_OOM for scratch below dfjk_build_bytes.  Nothing is
 * enqueued on failure.  Give exactly one of
 *   d_C: nao x nocc occupied orbitals (D = 2 C C^T), 1 <= nocc <= nao, or
 *   d_D: nao x nao symmetric density (nocc ignored; precision must be FP64).
 * Outputs: d_J, d_K (nao x nao, full symmetric), d_E[2] = {E_J, E_K}.
 * d_scratch must hold dfjk_build_bytes(plan, nocc, precision, d_D != NULL).
 * No host synchronisation; safe to capture in a HIP graph.  When the K build
 * needs several aux slabs (C route), the half transform of the next slab runs
 * on a second stream owned by the plan, forked from and joined back into
 * `stream`; such builds of one plan must not run concurrently on different
 * streams. */
int dfjk_build_bytes(const dfjk_plan *plan, int32_t nocc, int32_t precision,
                     int32_t with_density, size_t *bytes);
int dfjk_build(dfjk_plan *plan, const double *d_C, int32_t nocc, const double *d_D,
               int32_t precision, double *d_J, double *d_K, double *d_E,
               void *d_scratch, size_t scratch_bytes, void *stream);

/* The same build as dfjk_build, for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it takes no scratch argument and allocates nothing.  Its
 * scratch is a static device array of DFJK_STATIC_SCRATCH_BYTES (64 MiB)
 * inside the library, one per GPU, held until the process ends; the build
 * uses the widest aux slab whose scratch fits (single stream), so its J and
 * K equal dfjk_build's up to the order of the split-K sums.  Arguments,
 * outputs and errors as for dfjk_build, plus DFJK_E_OOM (nothing enqueued)
 * when even the narrowest slab needs more than the array holds (molecules
 * beyond about ten waters of the test basis); use dfjk_build there.  Every
 * call on a GPU shares that GPU's array, and nothing in it is assumed zero
 * or kept between calls: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller. */
#define DFJK_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int dfjk_build_static(dfjk_plan *plan, const double *d_C, int32_t nocc, const double *d_D, int32_t precision,
                      double *d_J, double *d_K, double *d_E, void *stream);

/* Incremental build for later SCF iterations, after the proposal of single
 * precision in later iterations (paper, "Limitations and Future Development:
 * Mixed Precision").  With D = 2 C C^T and D0 = 2 C0 C0^T,
 *   D - D0 = U W^T + W U^T,  U = C + C0,  W = C - C0,
 *   K(D) = K0 + G + G^T,     G = X_U X_W^T,
 * where K0 = K(D0) comes from an earlier FP64 dfjk_build with C0 on this plan
 * and X_U, X_W are the half-transforms of U and W.  C is first rotated onto
 * C0 (C -> C Q, Q the orthogonal polar factor of C^T C0, the orthogonal
 * Procrustes solution; D is unchanged) so that a sign flip or a rotation of
 * the occupied orbitals among themselves does not inflate W; if the rotation
 * cannot be formed to 1e-13 (C and C0 spanning different spaces), C is used
 * as given.  G is formed in
 * `precision` (its error scales with |C - C0|); J and both energies are FP64.
 * d_C, d_C0: nao x nocc; d_K0: nao x nao (read only, must not alias d_K).
 * d_scratch must hold dfjk_build_delta_bytes(plan, nocc, precision). */
int dfjk_build_delta_bytes(const dfjk_plan *plan, int32_t nocc, int32_t precision, size_t *bytes);
int dfjk_build_delta(dfjk_plan *plan, const double *d_C, const double *d_C0, int32_t nocc,
                     const double *d_K0, int32_t precision, double *d_J, double *d_K, double *d_E,
                     void *d_scratch, size_t scratch_bytes, void *stream);

/* Passage for batching: none in the paper, which runs one molecule at a
 * time; this is the serving form the library adds for many small molecules.
 * The contractions batched are those of dfjk_build (Introduction,
 * contributions 1 and 2).  Errors as for dfjk_build, per molecule, checked
 * for all n before anything is enqueued.
 * A batch of n closed-shell builds (molecules of any sizes, each with its own
 * set-up plan, all on the current device) on one stream: the same results as
 * n dfjk_build calls with d_C[i] (nao_i x nocc[i]), up to the order of the
 * split-K sums, but the K contractions of all FP64 molecules whose
 * half-transformed tensor fits one aux slab share one grouped launch (16
 * molecules per launch), with split counts chosen together to fill the chip,
 * and the split-K reductions and energies run as grouped launches too.  This
 * is the serving form for many small molecules, where per-launch overhead
 * dominates.  plans, d_C, nocc, d_J, d_K, d_E are host arrays of n entries;
 * outputs as for dfjk_build.  d_scratch must hold dfjk_build_batch_bytes
 * (per-molecule regions, 256-byte aligned, in order).  No host
 * synchronisation; safe to capture in a HIP graph.  A plan may appear more
 * than once. */
int dfjk_build_batch_bytes(int32_t n, dfjk_plan *const *plans, const int32_t *nocc, int32_t precision,
                           size_t *bytes);
int dfjk_build_batch(int32_t n, dfjk_plan *const *plans, const double *const *d_C, const int32_t *nocc,
                     int32_t precision, double *const *d_J, double *const *d_K, double *const *d_E,
                     void *d_scratch, size_t scratch_bytes, void *stream);

/* Autotuner for the K contraction of the closed-shell C-route build
 * (dfjk_build with d_C, this nocc and precision): its tile shape and split
 * count.  Candidates are half, one, two and four times the built-in split
 * count (within the contraction length) of the 128-wide output tiles and,
 * for FP64, of 64-wide tiles (which leave less of the syrk's work above the
 * diagonal or past nao).  Each runs one warm-up and three timed builds with
 * d_C on `stream` (HIP events; synchronises the stream), and the fastest is
 * kept in the plan for later builds of that shape.  Tile and split count
 * only reorder the FP64 sums of the split-K reduction, which stays fixed and
 * deterministic for a given choice.  dfjk_build_bytes may grow afterwards.
 * d_scratch must hold dfjk_autotune_bytes.  A candidate is reported as
 * 1000 * tile + split count: on return *chosen is the kept one; with
 * ncand != NULL, *ncand (capacity in, count out) candidates and their ms per
 * build are written to cand and ms (host arrays, may be NULL). */
int dfjk_autotune_bytes(const dfjk_plan *plan, int32_t nocc, int32_t precision, size_t *bytes);
int dfjk_autotune(dfjk_plan *plan, const double *d_C, int32_t nocc, int32_t precision, void *d_scratch,
                  size_t scratch_bytes, void *stream, int32_t *chosen, int32_t *ncand, int32_t *cand,
                  double *ms);

/* Precision chosen per build against an energy-error budget (paper,
 * Section 5 "Limitations and Future Development: Mixed Precision": lower
 * precision where an error estimate shows it is enough).  Runs the int8
 * C-route build, then a rigorous bound on |E_K(int8) - E_K| with E_K the
 * exact contraction of the same half-transformed tensor X, computed on the
 * device from the stored int8 digits of X and from C (Cauchy-Schwarz in the
 * seminorm of D = 2 C C^T, which is positive semidefinite):
 *   bound = 1/2 [2 sqrt(Q lambda R) + lambda R + lambda T] + F,
 *   lambda >= lambda_max(D) from |(C^T C)^16|_F^(1/16),
 *   A_s = sum over X of (a_s 2^{e - 7(s+1)})^2, T = sum_{i+j>=5} sqrt(A_i A_j),
 *   R = sum over blocks of 256 2^{2e-72} (the slices' remainders),
 *   Q = 2 |E_K(int8)| + lambda T + 2F, F the FP64 rounding of the folds.
 * E_J is FP64 in both precisions.  If bound <= budget (Eh) the int8 result
 * stands and *chosen = DFJK_MIXED_INT8; else the build is redone in FP64 and
 * *chosen = DFJK_FP64.  *bound receives the bound either way.  Outputs as for
 * dfjk_build (d_E[2] = {E_J, E_K}); chosen and bound are host pointers.
 * d_scratch must hold dfjk_build_checked_bytes(plan, nocc).  Synchronises
 * `stream` (the choice is read on the host), so it cannot be captured in a
 * HIP graph.  Errors: DFJK_E_STATE before dfjk_setup; DFJK_E_INVALID for NULL
 * pointers, nocc out of range or budget <= 0; DFJK_E_OOM for scratch below
 * the size query. */
int dfjk_build_checked_bytes(const dfjk_plan *plan, int32_t nocc, size_t *bytes);
int dfjk_build_checked(dfjk_plan *plan, const double *d_C, int32_t nocc, double budget, double *d_J,
                       double *d_K, double *d_E, void *d_scratch, size_t scratch_bytes, void *stream,
                       int32_t *chosen, double *bound);

/* The launch shape a closed-shell C-route dfjk_build with this nocc and
 * precision will use (after dfjk_screen; the autotuner's or dfjk_options'
 * choice included): shape[0] the K output tile (64 or 128), shape[1] the
 * split count of the K contraction, shape[2] aux functions per slab,
 * shape[3] the number of slabs.  shape is a host array of 4.  For profiling
 * and reporting; no device work. */
int dfjk_build_shape(const dfjk_plan *plan, int32_t nocc, int32_t precision, int32_t *shape);

/* Setup straight into host memory, for molecules whose B should not or
 * cannot be held in HBM even once (paper, Section 2.1 "Dataset and
 * Performance": integrals in host memory for large systems).  After the
 * metric, its Cholesky factor and L^-1 (as dfjk_setup), B = U L^-T is formed
 * one block of function-pair rows at a time: the three-centre integrals of
 * the block's shell pairs, then the whitening GEMM, then the block's rows of
 * every aux slab copied into h_pinned (slab-major [slab][f][plen], the layout
 * dfjk_offload writes; page-locked host memory the caller allocates and keeps
 * until dfjk_plan_destroy) on a copy stream of the plan, two row buffers so
 * the copies of one block overlap the next.  U and B are never whole in
 * device memory.  dfjk_setup_host_bytes: host_bytes for B and device_bytes
 * for the workspace with the widest row blocks whose workspace stays within
 * max_device_bytes (0: one block of every row); DFJK_E_OOM if not even one
 * shell pair's rows fit.  The workspace holds the plan's tables afterwards
 * and stays borrowed until dfjk_plan_destroy.  Later builds (C route, any
 * precision) stream B back slab by slab as after dfjk_offload.  Synchronises
 * `stream`.  Errors: DFJK_E_STATE unless the plan is screened and not yet
 * host-resident; DFJK_E_NOT_POSDEF as dfjk_setup; DFJK_E_OOM for buffers
 * below the size query. */
int dfjk_setup_host_bytes(const dfjk_plan *plan, size_t max_device_bytes, size_t *host_bytes,
                          size_t *device_bytes);
int dfjk_setup_host(dfjk_plan *plan, void *h_pinned, size_t host_bytes, void *d_workspace, size_t device_bytes,
                    void *stream);

/* Host-resident B, the paper's large-system storage (paper, Section 2.1
 * "Dataset and Performance": integrals held in host memory and moved to the
 * GPU asynchronously).  After dfjk_setup, dfjk_offload copies the whitened
 * tensor B into h_pinned (page-locked host memory the caller allocates and
 * keeps until dfjk_plan_destroy; slab-major, aux slabs of
 * dfjk_options.aux_slab functions or 1024) and the few tables later builds
 * need into d_tables (device memory the caller keeps).  Synchronises
 * `stream`.  From then on the plan no longer uses the setup workspace (the
 * caller may free it), and every dfjk_build (C route, any precision) streams
 * B slab by slab into two staging buffers of its scratch on a copy stream of
 * the plan, overlapped with the slab's J, half-transform and K work.  One
 * build at a time per plan.  dfjk_build_delta, dfjk_build_uks,
 * dfjk_build_batch and the density route return DFJK_E_UNSUPPORTED, and
 * dfjk_export, dfjk_sample and dfjk_setup DFJK_E_STATE, on such a plan. */
int dfjk_offload_bytes(const dfjk_plan *plan, size_t *host_bytes, size_t *device_bytes);
int dfjk_offload(dfjk_plan *plan, void *h_pinned, size_t host_bytes, void *d_tables,
                 size_t device_bytes, void *stream);

/* Convenience for callers that hold host arrays and want one answer: plan
 * creation, screening, setup and one build (the C or the D route, as in
 * dfjk_build) on the current device, with J, K (nao x nao) and E[2] copied
 * back to host memory before it returns.  C (nao x nocc) or D (nao x nao),
 * J, K, E are HOST pointers.  Unlike every other call, this one allocates
 * and frees its own device memory and stream, so it is not for the SCF loop
 * (use a plan there).  Errors as for the calls it makes. */
int dfjk_build_host(int32_t natm, const double *coords, const dfjk_basis *ao, const dfjk_basis *aux,
                    const dfjk_options *opt, const double *C, int32_t nocc, const double *D,
                    int32_t precision, double *J, double *K, double *E);

/* Open-shell (unrestricted) build, one of the methods the paper lists as
 * optimised for the GPU (paper, "Accelerated Functionalities", table of
 * functionalities: unrestricted SCF).  Per spin s (alpha, beta):
 *   D_s = C_s C_s^T,  K_s = sum_P B_P D_s B_P = X_s X_s^T,
 * J from D = D_a + D_b, and d_E[2] = {E_J, E_K} with
 *   E_J = 1/2 Tr(D J),  E_K = -1/2 (Tr(D_a K_a) + Tr(D_b K_b)).
 * d_Ca: nao x nocc_a, d_Cb: nao x nocc_b (0 <= nocc_b, nocc_a <= nao, at
 * least one positive; a spin with no electrons may pass NULL and gets K_s = 0).
 * The K contractions run in `precision`; J and the energies stay FP64.
 * Outputs d_J, d_Ka, d_Kb: nao x nao, full symmetric.
 * d_scratch must hold dfjk_build_uks_bytes(plan, nocc_a, nocc_b, precision). */
int dfjk_build_uks_bytes(const dfjk_plan *plan, int32_t nocc_a, int32_t nocc_b, int32_t precision,
                         size_t *bytes);
int dfjk_build_uks(dfjk_plan *plan, const double *d_Ca, int32_t nocc_a, const double *d_Cb,
                   int32_t nocc_b, int32_t precision, double *d_J, double *d_Ka, double *d_Kb,
                   double *d_E, void *d_scratch, size_t scratch_bytes, void *stream);

/* Four-centre direct J/K: the exact (unfitted) Coulomb and exchange matrices
 *   J_{mu nu} = sum_{la si} (mu nu|la si) D_{la si},
 *   K_{mu nu} = sum_{la si} (mu la|nu si) D_{la si},
 * from two-electron integrals over shell quartets, computed on the fly
 * (direct SCF: the integral path the package began with, paper,
 * Introduction; "Limitations and Future Development: Direct SCF & Other
 * Integral Schemes").  Needs a screened plan only (no dfjk_setup): a shell
 * pair is kept if Q_ab max Q_cd >= schwarz_thresh and a quartet is computed
 * iff Q_ab Q_cd >= schwarz_thresh (Schwarz bound on |(ab|cd)|).
 *
 * dfjk_direct_bytes gives the size of the pair tables; dfjk_direct_setup
 * fills them (product centres, exponents and the Hermite expansion of every
 * function pair) on the device.  The tables stay borrowed until the plan is
 * destroyed or set up again and must not be touched meanwhile.  Synchronises
 * `stream`.
 *
 * dfjk_direct_build takes exactly one of
 *   d_C: nao x nocc occupied orbitals (D = 2 C C^T), 1 <= nocc <= nao, or
 *   d_D: nao x nao symmetric density (nocc ignored),
 * and writes d_J, d_K (nao x nao, full symmetric, must not alias) and
 * d_E[2] = {E_J, E_K} = {1/2 Tr(D J), -1/4 Tr(D K)}.  FP64 throughout; K is
 * accumulated with atomics, so its last bits may differ between runs.
 * d_scratch must hold dfjk_direct_build_bytes(plan, d_D != NULL).  No host
 * synchronisation; safe to capture in a HIP graph.
 *
 * dfjk_direct_stats: kept pairs per class (s-s, p-s, p-p, d-s, d-p, d-d) in
 * pairs[6] and the number of (bra pair, ket pair) combinations that pass the
 * screen.
 *
 * Errors (nothing is enqueued on failure): DFJK_E_STATE before dfjk_screen
 * (tables) or dfjk_direct_setup (builds, stats), or on a device other than
 * the one the tables were set up on; DFJK_E_OOM when the tables or the
 * scratch are smaller than the *_bytes query; DFJK_E_INVALID for a NULL
 * pointer, both or neither of d_C and d_D, nocc out of range, or outputs
 * that alias each other (or J0, K0 below). */
int dfjk_direct_bytes(const dfjk_plan *plan, size_t *table_bytes);
int dfjk_direct_setup(dfjk_plan *plan, void *d_tables, size_t bytes, void *stream);
int dfjk_direct_stats(const dfjk_plan *plan, int64_t *pairs, int64_t *quartets);
int dfjk_direct_build_bytes(const dfjk_plan *plan, int32_t with_density, size_t *bytes);
int dfjk_direct_build(dfjk_plan *plan, const double *d_C, int32_t nocc, const double *d_D, double *d_J,
                      double *d_K, double *d_E, void *d_scratch, size_t scratch_bytes, void *stream);

/* Incremental direct J/K for later SCF iterations, after the paper's
 * Schwarz-bound error control in direct SCF ("Limitations and Future
 * Development: Mixed Precision"): with the exact J0 = J(D0), K0 = K(D0) of an
 * earlier dfjk_direct_build on this plan,
 *   J = J0 + J(D - D0),  K = K0 + K(D - D0),
 * where the increment skips every quartet whose density-weighted bound
 * Q_ab Q_cd max|D - D0| (the largest element of D - D0 over the shell blocks
 * the quartet contracts with: cd for J; bd, bc, ad, ac for K) is below
 * schwarz_thresh, so the work shrinks as D approaches D0.
 * d_D, d_D0: nao x nao symmetric; d_J0, d_K0: nao x nao (read only, must not
 * alias the outputs).  Outputs as for dfjk_direct_build, with
 * d_E = {1/2 Tr(D J), -1/4 Tr(D K)} of the full D.  d_scratch must hold
 * dfjk_direct_build_delta_bytes(plan). */
int dfjk_direct_build_delta_bytes(const dfjk_plan *plan, size_t *bytes);
int dfjk_direct_build_delta(dfjk_plan *plan, const double *d_D, const double *d_D0, const double *d_J0,
                            const double *d_K0, double *d_J, double *d_K, double *d_E, void *d_scratch,
                            size_t scratch_bytes, void *stream);

/* Diagnostics for tests (valid after setup).  Dense copies of intermediate
 * quantities in the caller's function order:
 *   DFJK_EXPORT_INT3C   (naux x nao x nao) unwhitened (mu nu|P), screened
 *                       entries 0
 *   DFJK_EXPORT_B       (naux x nao x nao) whitened B, aux index in the
 *                       internal order (B = L^{-1} U depends on the order)
 *   DFJK_EXPORT_METRIC  (naux x naux) (P|Q)
 *   DFJK_EXPORT_CHOL    (naux x naux) L, upper triangle 0, in the internal
 *                       aux order of dfjk_plan_aux_order (a Cholesky factor
 *                       depends on the order of the rows)
 * Every other aux index follows the caller's aux function order. */
typedef enum {
    DFJK_EXPORT_INT3C = 0,
    DFJK_EXPORT_B = 1,
    DFJK_EXPORT_METRIC = 2,
    DFJK_EXPORT_CHOL = 3
} dfjk_export_kind;
int dfjk_export(const dfjk_plan *plan, int32_t kind, double *d_out, void *stream);

/* Sampled values of the unwhitened (kind 0) or whitened (kind 1) tensor:
 * d_idx holds n triples (P, mu, nu), d_out receives n values.  mu, nu follow
 * the caller's AO order; P the caller's aux order for kind 0 and the internal
 * aux order (dfjk_plan_aux_order) for kind 1.  Pairs that screening dropped
 * read 0; a triple with an index out of range reads NaN. */
int dfjk_sample(const dfjk_plan *plan, int32_t kind, int64_t n, const int32_t *d_idx,
                double *d_out, void *stream);

/* Boys function F_0..F_mmax at n points (the device routine the integral
 * kernels use): d_T[n] -> d_F[n * (mmax+1)], mmax <= 16. */
int dfjk_boys(int32_t mmax, int64_t n, const double *d_T, double *d_F, void *stream);

/* Stage profiler.  With dfjk_profile(plan, 1) every later setup and build
 * records a pair of HIP events around each stage on its stream (no host
 * synchronisation).  dfjk_profile_read waits for the recorded events, writes
 * the summed milliseconds and the number of timed launches of each of the
 * DFJK_NSTAGES stages (host arrays), and clears the record.
 * dfjk_stage_name(i) names stage i ("build.K", ...).  "span.build" is a whole
 * dfjk_build (C or D route) from its first to its last launch on the caller's
 * stream: J runs on a side stream beside the half transform and K, so the
 * "build.*" stages of one build overlap and their sum exceeds the span.
 * "span.setup" is a whole dfjk_setup alike: the integrals, then the block
 * rows of L^-1, run on the side stream beside the metric and its factor, so
 * "setup.inverse" is the span of the inverse's steps, most of it beside
 * "setup.cholesky". */
#define DFJK_NSTAGES 12
int dfjk_profile(dfjk_plan *plan, int32_t on);
int dfjk_profile_read(dfjk_plan *plan, double *ms, int32_t *count);
const char *dfjk_stage_name(int32_t stage);

int dfjk_plan_destroy(dfjk_plan *plan);

/* Thread-local description of the last error on this thread ("" if none). */
const char *dfjk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DFJK_H */
