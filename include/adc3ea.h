/*
 * adc3ea.h -- C ABI of the MI355X (gfx950) DF-SS-FNO-EA-ADC(3) library.
 *
 * The method: density-fitted third-order algebraic diagrammatic construction for
 * electron attachment (non-Dyson EA-ADC, Sec. "Algebraic Diagrammatic
 * Construction (ADC) Theory", eqs 1-6) with state-specific frozen natural
 * orbitals (Sec. "State-Specific Frozen Natural Orbitals (SS-FNO)", eqs 9-17),
 * natural auxiliary functions (Sec. "Natural Auxiliary Functions (NAF)",
 * eqs 27-29) and the perturbative truncation correction (eq 30), following the
 * steps of Sec. "Computational Details".
 *
 * Conventions shared by every entry point
 *   - Energies in Hartree.  A root omega is an eigenvalue of the secular matrix
 *     M (eq 6): omega = E(N+1) - E(N); the electron affinity is -omega.
 *   - Inputs describe a closed-shell reference in its canonical orbitals:
 *     eps_occ[nocc], eps_vir[nvir] (ascending; every occupied energy below every
 *     virtual one) and the DF factor B[naux][n][n], n = nocc + nvir, row-major,
 *     occupied orbitals first, symmetric in its two orbital indices, such that
 *     (pq|rs) = sum_Q B[Q][p][q] B[Q][r][s] (eqs 25-26).
 *   - Vector space: N = nvir + nocc*nvir*nvir.  A vector is [r1[nvir], z[nocc][nvir][nvir]]:
 *     r1 the 1p amplitudes, z orthonormal doublet coordinates of the 2p1h space
 *     (x = z_S + z_A/sqrt(3) on c+_{a alpha} c+_{b beta} c_{i beta}|0>).
 *   - Pointers named *_dev are device pointers (HBM); others are host pointers.
 *     The caller owns every buffer.  Device work is ordered on `stream`; calls that
 *     return host results synchronise that stream before returning.
 *   - Errors: every call returns an adc3_status; nothing is thrown across the
 *     ABI.  adc3_last_error() returns a message for the last failing call on the
 *     calling thread.  Arguments are validated before any launch.
 *   - Workspace: device memory is taken only from the caller's workspace
 *     (size from the matching *_workspace_bytes query); too small a workspace
 *     returns ADC3_ENOMEM before any launch.
 */
#ifndef ADC3EA_H
#define ADC3EA_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ADC3_OK = 0,
    ADC3_WNOCONV = 1,     /* outputs valid, Davidson not converged within max_iter */
    ADC3_EINVAL = -1,     /* invalid argument (message says which) */
    ADC3_ENOMEM = -2,     /* workspace too small */
    ADC3_EHIP = -3,       /* HIP runtime error */
    ADC3_ENUMERIC = -4,   /* non-finite value met */
    ADC3_EUNSUP = -5      /* unsupported option */
} adc3_status;

/* Options.  adc3_default_opts() fills the defaults listed here. */
typedef struct {
    int level;            /* 2 or 3: ADC order of the final roots (default 3) */
    int max_iter;         /* Davidson iterations per solve (default 500) */
    int max_subspace;     /* Davidson subspace limit; 0 = max(8*nroots, 40) */
    int fno_correction;   /* 1: add omega_can-ADC(2) - omega_FNO-ADC(2) (eq 30); default 1 */
    int precision;        /* sigma arithmetic: 0 FP64; 1 FP32 ladder and 1p/2p1h coupling (FP32 matrix
                             cores, FP32 accumulation); 2 BF16 ladder (BF16 matrix cores, FP32
                             accumulation) and FP32 coupling.  For 1 and 2 each Davidson runs the
                             reduced-precision sigma until its noise floor, then restarts from the
                             Ritz vectors with FP64 sigma (FP64 residual correction) down to conv;
                             orthogonalisation, Rayleigh-Ritz, residual norms and every
                             eigendecomposition stay FP64.  Default 0. */
    int precond;          /* Davidson step.  0: Jacobi (diagonal) everywhere; 1: learned (needs
                             mlp_weights) in the ADC(3) solves; 2: Olsen, t = (D-theta)^-1 (r - eps x),
                             eps making t orthogonal to the Ritz vector x in the D-theta metric,
                             everywhere; 3 (default): Jacobi in the ADC(3) solves.  Under 1 and 3 the
                             ADC(2) solves, whose 2p1h block is diagonal, take the 1p block exactly:
                             t1 = (M11 - theta)^-1 r1 (through the eigendecomposition of M11),
                             t2 = r2 / (D2 - theta). */
    const float* mlp_weights; /* device, adc3_mlp_nparams() floats (see adc3_mlp_train); NULL default */
    int sigma_graphs;     /* 1: each sigma pass shape is captured once into a HIP graph and replayed
                             (needs a non-null stream; on the null stream sigma runs eagerly); default 0 */
    int ladder;           /* form of the ladder term sum_cd (ac|bd) r_cdi of the ADC(3) contexts:
                             1 stored: (ac|bd) assembled once per basis from the DF factor (eq 25) and
                               kept as its pair-symmetric and pair-antisymmetric blocks (about v^4/2
                               elements), about M v^4 flops per application of M rows;
                             2 assembled: sum_Q B^Q Z_i B^Q from the virtual block of the factor in
                               every application, 4 X M v^3 flops and no v^4 storage;
                             0 (default): stored unless the pair blocks of the canonical basis exceed
                               96 GB in FP64 (nvir > 393).  The choice holds for the whole solve. */
    double sm_x;          /* level 3: the scaled-matrix ADC of Sec. "ADC Theory" (equation after eq 5),
                             M = M_ADC(2) + sm_x (M_ADC(3) - M_ADC(2)): the third-order part of M11, the
                             second-order part of the 1p/2p1h coupling and the first-order 2p1h terms
                             scaled by sm_x; 0 gives ADC(2), 1 (default) ADC(3), 0.5 the usual choice.
                             In [0, 1].  The truncated ADC(2) solves of eq 30 are unaffected. */
    int fno_mode;         /* natural orbitals of the virtual truncation (eqs 9-16): 0 (default) state
                             specific, D^SS(k) = D^MP2 + D^EA(k) per root (eq 17); 1 ground-state MP2-FNO,
                             D^MP2 alone, one truncated basis shared by all roots (each root matched in it
                             as above) */
    double fno_keep_frac; /* > 0: keep ceil(fno_keep_frac * nvir) natural orbitals (largest occupations)
                             instead of those above fno_thresh (a percentage-of-virtuals truncation); 0
                             (default): by threshold.  In [0, 1]; > 0 runs the truncated pipeline. */
    const double* init_guess; /* device [n_guess][N] (N of the canonical basis), nullable: start vectors of
                             the canonical-basis Davidson (the ADC(level) solve without truncation, else
                             the canonical ADC(2) solve of step 3), taken before the diagonal guesses;
                             resuming from vectors_out of an unconverged run reaches the same roots */
    int n_guess;          /* number of init_guess vectors (0 default) */
    double* vectors_out;  /* device [nroots][N], nullable: the Ritz vectors of that canonical-basis solve */
    double* dyson_out;    /* device [nroots][nocc+nvir], nullable: spectral amplitudes x_kp = sum_A Y_Ak f_Ap
                             (eqs 7-8) of each reported root in the canonical MO basis (occupied first),
                             i.e. the Dyson-orbital coefficients; each vector's largest-magnitude entry made
                             positive.  See adc3_ea_spectral_amplitudes for f. */
    int lockstep;         /* Engine of Davidson solves that do not depend on each other (a build
                             addition).  adc3_ea_solve: the truncated ADC(2) solves of all roots' bases,
                             then their ADC(3) solves (all bases held at once: more workspace);
                             adc3_ea_solve_batched: the instances.
                             1: one lockstep block Davidson: each iteration of a chunk has a fixed shape
                             (one new direction per root not converged when the chunk began, those
                             converging within it zeroed) and keeps its convergence flags on the device,
                             and each solve's chunks of iterations are replayed from HIP graphs on its own
                             stream; the host reads the flags once per chunk and sets the next block.
                             Batches: the instances in waves of nstreams.  Jacobi and exact-1p steps only
                             (precond 1 and 2 keep one solve at a time).
                             2: each basis's steps (its contexts' setup and its solves, with the
                             one-at-a-time solver) on a host thread and a stream of its own: the same
                             iterations and roots as 0, one basis's setup and another's Davidson
                             overlapping on the GPU.  Batches: worker threads, as 0.
                             0: one solve at a time (batches: worker threads, one per stream).
                             -1 (default): 2 for the per-root bases of one solve when there are two or more
                             and their stored ladders take at most 96 GB together, else 0. */
} adc3_opts;

/* Per-root report of adc3_ea_solve. */
typedef struct {
    double omega;          /* reported root (corrected when SS-FNO/NAF is active) */
    double omega_uncorr;   /* ADC(3) root matched to k in the truncated basis */
    double omega_adc2_can; /* canonical ADC(2) root k (0 when no truncation ran) */
    double omega_adc2_fno; /* ADC(2) root k in the truncated basis */
    double resnorm;        /* final residual 2-norm of the ADC(3) root */
    int nvir_kept;         /* virtuals kept by SS-FNO (eq 11) */
    int naux_kept;         /* auxiliary functions kept by NAF (eq 29) */
    int iters;             /* Davidson iterations of the ADC(3) solve */
    int sigma_builds;      /* sigma vectors built by the solves of this root's basis (all phases); a solve
                              shared by several roots counts on the first of them only, so the sum over
                              the roots is the call's total */
    double omega_lowp;     /* precision 1/2: root k when the reduced-precision phase ended */
    int iters_lowp;        /* precision 1/2: Davidson iterations in the reduced-precision phase */
    double err_bound;      /* bound on |omega - the same combination of exact eigenvalues of the FP64
                              matrices|: each eigenvalue that enters omega (ADC(3) root, and with eq 30 the
                              canonical and truncated ADC(2) roots) lies within its FP64 residual 2-norm of
                              an eigenvalue of its matrix (symmetric M), so their sum bounds the error; in
                              every precision the last Davidson phase runs FP64 sigma, so it also bounds the
                              mixed-precision result's distance from the FP64 one */
    double pole_strength;  /* sum_p x_kp^2 of the root's spectral amplitudes (eq 7) */
    int sigma_builds_final; /* the part of sigma_builds made by the final-level (ADC(3) or sm-ADC) solves */
} adc3_root_report;

void adc3_default_opts(adc3_opts* opts);

/* Message of the last failing call on this thread ("" if none). */
const char* adc3_last_error(void);

/* ---------------------------------------------------------------------------
 * Full method (Sec. "Computational Details", steps 2-4f).
 *   fno_thresh > 0: per root k, build D^SS(k) = D^MP2 + D^EA-ADC(2)(k) (eq 17),
 *     keep natural orbitals with occupation > fno_thresh (eqs 9-11),
 *     recanonicalise (eqs 12-16);
 *   naf_thresh > 0: keep natural auxiliary functions with W-eigenvalue >= naf_thresh
 *     (eqs 27-29, W from the vv block of the root's truncated factor);
 *   both <= 0: plain canonical EA-ADC(level) roots.
 *   Root k of a truncated problem: the truncated ADC(2) root m whose eigenvector has
 *   the largest overlap with canonical ADC(2) eigenvector k projected into the kept
 *   orbitals (lowest m on ties), and the truncated ADC(3) root of the same index m.
 *   roots_out[k] = omega_FNO-ADC(3)(k) + omega_can-ADC(2)(k) - omega_FNO-ADC(2)(k) (eq 30).
 * Inputs eps_occ_dev, eps_vir_dev, B_dev are device pointers and are not modified.
 * roots_out[nroots] and reports[nroots] (nullable) are host arrays.
 * conv: a root is converged when its residual 2-norm and eigenvalue change are <= conv.
 * Returns ADC3_WNOCONV (outputs valid) if any solve hit max_iter.
 * ------------------------------------------------------------------------- */
size_t adc3_ea_solve_workspace_bytes(int nocc, int nvir, int naux, int nroots, const adc3_opts* opts);

int adc3_ea_solve(const double* eps_occ_dev, const double* eps_vir_dev, const double* B_dev,
                  int nocc, int nvir, int naux, int nroots,
                  double fno_thresh, double naf_thresh, double conv,
                  const adc3_opts* opts, double* roots_out, adc3_root_report* reports,
                  void* workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Ragged batches of independent instances (a build addition, not in the paper): every
 * instance is an adc3_ea_solve with its own sizes, roots and thresholds, and one set of
 * options.  The instances are spread over nstreams worker streams (<= 0: 4), each
 * driven by a host thread of the library, longest estimated work first onto the least
 * loaded worker; a worker solves its instances one after another in its own slice of
 * the workspace.  The workers start after the work already queued on `stream` and
 * `stream` waits for all of them; the call returns when every instance is done.
 * roots_out and reports (nullable) hold the instances' roots in order, nroots per
 * instance; status_out[ninst] (nullable) each instance's status.  The return value is
 * the most severe status (adc3_last_error names the first failing instance).
 * Results do not depend on nstreams.
 * ------------------------------------------------------------------------- */
typedef struct {
    const double* eps_occ;  /* device [nocc] */
    const double* eps_vir;  /* device [nvir] */
    const double* B;        /* device [naux][nocc+nvir][nocc+nvir] */
    int nocc, nvir, naux, nroots;
    double fno_thresh, naf_thresh, conv;
} adc3_instance;

size_t adc3_ea_solve_batched_workspace_bytes(const adc3_instance* inst, int ninst, const adc3_opts* opts,
                                             int nstreams);

int adc3_ea_solve_batched(const adc3_instance* inst, int ninst, const adc3_opts* opts, int nstreams,
                          double* roots_out, adc3_root_report* reports, int* status_out,
                          void* workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Secular-matrix context: integrals and intermediates of EA-ADC(level) for one
 * instance (eqs 3-5 truncated at `level`), kept in the caller's workspace.
 * The handle (host memory) is freed by adc3_ctx_destroy, which frees no device
 * memory; the workspace must stay alive while the context is used.
 * ------------------------------------------------------------------------- */
typedef struct adc3_ctx adc3_ctx;

/* Workspace for adc3_ea_setup plus everything later calls on the context take from
 * it: sigma builds, the dense-matrix hook and (nroots > 0) adc3_ea_davidson with up to
 * nroots roots and the default subspace.  Returns 0 for invalid arguments. */
size_t adc3_ea_setup_workspace_bytes(int nocc, int nvir, int naux, int level, int nroots, int precision);

/* precision 1 or 2 also keeps the reduced-precision copies (see adc3_opts.precision)
 * so that adc3_ea_sigma / adc3_ea_davidson may use them. */
int adc3_ea_setup(const double* eps_occ_dev, const double* eps_vir_dev, const double* B_dev,
                  int nocc, int nvir, int naux, int level, int precision,
                  void* workspace_dev, size_t workspace_bytes, hipStream_t stream,
                  adc3_ctx** ctx_out);

/* As adc3_ea_setup_workspace_bytes / adc3_ea_setup, with the ladder form of a level-3
 * context chosen as in adc3_opts.ladder (0 auto by nvir, 1 stored, 2 assembled from the
 * factor).  The two calls above are these with ladder = 0.  Invalid ladder: 0 bytes /
 * ADC3_EINVAL. */
size_t adc3_ea_setup_workspace_bytes_ex(int nocc, int nvir, int naux, int level, int nroots, int precision,
                                        int ladder);
int adc3_ea_setup_ex(const double* eps_occ_dev, const double* eps_vir_dev, const double* B_dev,
                     int nocc, int nvir, int naux, int level, int precision, int ladder,
                     void* workspace_dev, size_t workspace_bytes, hipStream_t stream,
                     adc3_ctx** ctx_out);

/* A level-3 context of the scaled-matrix ADC, M = M_ADC(2) + sm_x (M_ADC(3) - M_ADC(2)) (Sec. "ADC
 * Theory", equation after eq 5; see adc3_opts.sm_x), sm_x in [0, 1]; ladder and workspace as
 * adc3_ea_setup_ex with level 3. */
int adc3_ea_setup_sm(const double* eps_occ_dev, const double* eps_vir_dev, const double* B_dev,
                     int nocc, int nvir, int naux, double sm_x, int precision, int ladder,
                     void* workspace_dev, size_t workspace_bytes, hipStream_t stream, adc3_ctx** ctx_out);

void adc3_ctx_destroy(adc3_ctx* ctx);

/* Element budget for one chunk of the large setup tensors (the o*na*v^2 slices of the
 * 1p/2p1h coupling build are cut along the first virtual index to stay within it; the
 * assembled ladder's intermediate may take twice it).  n > 0 sets it for the process (takes
 * effect for contexts and workspace plans made afterwards); n <= 0 only queries.  Returns the
 * previous value.  Default 2^29 (4.3 GB of FP64). */
long long adc3_set_chunk_elems(long long n);

/* The ladder term alone, assembled from the DF factor (the form of adc3_opts.ladder = 2):
 *   C[m][a][b] = sum_cd (ac|bd) Z[m][c][d],  (ac|bd) = sum_Q Bvv[Q][a][c] Bvv[Q][b][d]  (eq 25),
 * computed as sum_Q B^Q Z_m B^Q in chunks of auxiliary functions.  Bvv_dev [naux][nvir][nvir]
 * (each block symmetric), Z_dev and C_dev [nrows][nvir][nvir], FP64, device, row-major; C is
 * overwritten.  precision 1 / 2: Bvv and Z are rounded to FP32 / BF16 and the products
 * accumulate in FP32 (C stays FP64).  The workspace holds the rounded copies and the
 * intermediate; its size sets the chunk: at least adc3_ladder_workspace_bytes (one auxiliary
 * function per chunk), naux times the intermediate part for a single chunk.  Stream-ordered,
 * asynchronous; nvir <= 1024, nrows <= 65535. */
size_t adc3_ladder_workspace_bytes(int nvir, int naux, int nrows, int precision);
int adc3_ladder_apply(const double* Bvv_dev, const double* Z_dev, double* C_dev, int nvir, int naux, int nrows,
                      int precision, void* workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* The same ladder term for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): identical arguments and results,
 * with no workspace argument.  Its scratch (the rounded copies of Bvv and Z for precision 1 / 2 and
 * the intermediate) is one static device array of ADC3_STATIC_SCRATCH_BYTES per GPU, held from the
 * library's first use on that GPU until the process ends; the call makes no allocation of any kind.
 * Shapes whose adc3_ladder_workspace_bytes exceeds ADC3_STATIC_SCRATCH_BYTES return ADC3_ENOMEM
 * before any launch.  Every call on one GPU shares that GPU's array: calls that overlap on a GPU
 * (other streams, other host threads) race and must be serialised by the caller.  Stream-ordered,
 * asynchronous. */
#define ADC3_STATIC_SCRATCH_BYTES (256u << 20)
int adc3_ladder_apply_static(const double* Bvv_dev, const double* Z_dev, double* C_dev, int nvir, int naux,
                             int nrows, int precision, hipStream_t stream);

/* Symmetric eigensolver of the natural-orbital and natural-auxiliary-function steps (Sec.
 * "Frozen Natural Orbitals", eq 9 and the recanonicalisation of eqs 12-13; Sec. "Natural
 * Auxiliary Functions", eq 28): FP64 cyclic Jacobi (n > 96: over blocks of 32 rows, each round's
 * block-pair sub-matrices diagonalised in LDS and their orthogonal factors applied to A and V).
 * A_dev[n][n] device, row-major, read only
 * (its symmetric part (A + A^T)/2 is diagonalised); w_dev[n] receives the eigenvalues in
 * ascending order, V_dev[n][n] the eigenvectors as columns (V[i][k] = component i of vector k),
 * each with its largest-magnitude component positive (first index on ties).  The workspace holds
 * a copy of A and the solver's scratch: at least adc3_eigh_workspace_bytes(n) bytes.  1 <= n <=
 * 4096.  Synchronises the stream (the sweep loop reads the off-diagonal norm back);
 * ADC3_ENUMERIC for a non-finite matrix. */
size_t adc3_eigh_workspace_bytes(int n);
int adc3_eigh(const double* A_dev, double* w_dev, double* V_dev, int n, void* workspace_dev, size_t workspace_bytes,
              hipStream_t stream);

/* The same eigensolver for nb independent matrices of one order n, as the solve uses it for the
 * natural orbitals and their recanonicalisation of all roots at once: A_dev[nb][n][n] device
 * (read only), w_dev[nb][n] (ascending per matrix), V_dev[nb][n][n] (columns, sign convention as
 * adc3_eigh).  Each matrix stops at its own convergence; the rounds of all matrices share their
 * launches.  Workspace: adc3_eigh_batched_workspace_bytes(n, nb).  1 <= n <= 4096,
 * 1 <= nb <= 65535.  Synchronises the stream; ADC3_ENUMERIC if any matrix is non-finite. */
size_t adc3_eigh_batched_workspace_bytes(int n, int nb);
int adc3_eigh_batched(const double* A_dev, double* w_dev, double* V_dev, int n, int nb, void* workspace_dev,
                      size_t workspace_bytes, hipStream_t stream);

/* Dimension N of the context's vector space. */
long long adc3_ea_dim(const adc3_ctx* ctx);

/* sigma = M r for nvec vectors (Sec. ADC theory, Davidson sigma vectors):
 * r_dev[nvec][N], sigma_dev[nvec][N] device, row-major, must not overlap.
 * precision: 0 (FP64) or the context's setup precision (as in adc3_opts). */
int adc3_ea_sigma(adc3_ctx* ctx, const double* r_dev, double* sigma_dev, int nvec, int precision,
                  hipStream_t stream);

/* Diagonal of M: diag_dev[N] device. */
int adc3_ea_diagonal(adc3_ctx* ctx, double* diag_dev, hipStream_t stream);

/* Lowest nroots eigenpairs of M by block Davidson (FP64).  omega[nroots] host;
 * vectors_dev[nroots][N] device (nullable); resnorm[nroots] host (nullable);
 * iters (host, nullable) receives the iteration count.  Returns ADC3_WNOCONV (outputs valid:
 * the current Ritz values and vectors) after max_iter iterations, ADC3_ENUMERIC for a non-finite
 * Ritz value or residual. */
int adc3_ea_davidson(adc3_ctx* ctx, int nroots, double conv, int max_iter, int max_subspace,
                     int precision, double* omega, double* vectors_dev, double* resnorm, int* iters,
                     hipStream_t stream);

/* The same with caller start vectors guess_dev[n_guess][N] (device; orthonormalised as a block and
 * taken before the diagonal guesses): resuming from the vectors of an unconverged call converges to
 * the same roots in fewer iterations.  ADC3_ENUMERIC if the guesses are linearly dependent. */
int adc3_ea_davidson_guess(adc3_ctx* ctx, int nroots, double conv, int max_iter, int max_subspace,
                           int precision, const double* guess_dev, int n_guess, double* omega,
                           double* vectors_dev, double* resnorm, int* iters, hipStream_t stream);

/* Spectral amplitudes (eqs 7-8) of nvec vectors vecs_dev[nvec][N] of the context's space (device):
 * x_dev[nvec][nocc+nvir] (device, occupied orbitals first), x_kp = sum_A Y_kA f_Ap with
 * f_Ap = <Psi~_A| c+_p |Psi0> for p of the attached electron's spin, kept through second order in the
 * 1p rows and first order in the 2p1h rows:  f_ab = delta_ab - D^MP2_ab / 2,  f_aj = -u1_ja (second-
 * order singles),  f_(iab),j = -[(S + sqrt3 A) T_ji]_ab (z coordinates), f_(iab),b' = 0.  No sign fixing. */
int adc3_ea_spectral_amplitudes(adc3_ctx* ctx, const double* vecs_dev, int nvec, double* x_dev,
                                hipStream_t stream);

/* Test hook of the error path: the next Davidson iteration >= iteration (> 0) on any context writes
 * NaN into one new sigma vector, once; that solve then returns ADC3_ENUMERIC.  0 disarms. */
void adc3_debug_inject_nan(int iteration);

/* Test hook of the multi-chunk paths of the k-major ladder kernel (the sigma ladder's minimum K-chunk
 * count, and large setup contractions run as consecutive K ranges): lowers the byte limit of one
 * chunk's operand span, 2^31 - 1 (32-bit offsets), to `bytes` (> 0) for every later call in the process;
 * 0 restores it.  Results are the same up to summation order. */
void adc3_debug_ladder_offset_limit(long long bytes);

/* Test hook: dense M (N <= 20000) into M_dev[N][ldm] device. */
int adc3_ea_dense_matrix(adc3_ctx* ctx, double* M_dev, int ldm, hipStream_t stream);

/* Test hook: copy an intermediate to a device buffer.  which: 0 = M11 [nvir][nvir],
 * 1 = U_z [nvir][nocc*nvir*nvir] (1p-2p1h block in z coordinates),
 * 2 = T [nocc][nocc][nvir][nvir] first-order amplitudes, 3 = MP2 virtual density
 * [nvir][nvir] (per spin).  count receives the element count when out_dev is NULL. */
int adc3_ea_intermediate(adc3_ctx* ctx, int which, double* out_dev, long long* count, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Learned Davidson preconditioner (a build addition, not in the paper).
 * For root theta and residual r the step is t_e = a0_e (1 + u_e), a0_e = r_e/(D_e - theta)
 * the Jacobi step, u_e = MLP(features of element e): 6 -> 256 -> 256 -> 1 with GELU
 * (tanh form).  Features: (D_e - theta)/(|theta|+1), r_e/rms(r), [e is 1p], e_a,
 * e_b (0 for 1p), e_i (0 for 1p).  Weights: float[adc3_mlp_nparams()] laid out
 * W1[6][256], b1[256], W2[256][256], b2[256], W3[256], b3[1]; W3 = b3 = 0 gives
 * exactly the Jacobi step.  Inference: one fused kernel per residual (FP32 first
 * layer, BF16 matrix-core second layer with FP32 accumulation, FP32 head).  A
 * non-finite step, a residual that grows by more than 2x in one iteration, or one that
 * has not improved on its best value by 10% in 5 iterations switches that root back
 * to Jacobi for the rest of the solve.
 * ------------------------------------------------------------------------- */
int adc3_mlp_nparams(void);

/* Replay sigma passes from captured HIP graphs on this context (see adc3_opts.sigma_graphs). */
int adc3_ea_set_sigma_graphs(adc3_ctx* ctx, int on);

/* Use the learned preconditioner in adc3_ea_davidson on this context (NULL: Jacobi).
 * weights_dev must stay valid while the context is used. */
int adc3_ea_set_preconditioner(adc3_ctx* ctx, const float* weights_dev);

/* Training data from a Jacobi-preconditioned Davidson solve on ctx.  The solve runs
 * twice (it is deterministic): the first run gives the converged vectors xf, the
 * replay records, at every iteration and for every unconverged root, one group of
 * group_size elements sampled by a hash of (seed, group, index): the features, the
 * Jacobi step a0 and the target, the part of xf outside the current subspace V,
 * xf - V (V^T xf), i.e. what the new search direction should supply.  Outputs
 * (device): feat[max_groups][group_size][6], a0[max_groups][group_size],
 * target[max_groups][group_size]; *ngroups (host) groups were written.  The
 * context must have been set up with at least nroots roots.  Returns ADC3_WNOCONV
 * if the solve did not converge. */
int adc3_mlp_collect(adc3_ctx* ctx, int nroots, double conv, int max_iter, int group_size, int max_groups,
                     unsigned long long seed, double* feat_dev, double* a0_dev, double* target_dev, int* ngroups,
                     hipStream_t stream);

/* Workspace for adc3_mlp_train / adc3_mlp_loss_grad with batch_groups groups of group_size. */
size_t adc3_mlp_workspace_bytes(int batch_groups, int group_size);

/* Mean over groups of 1 - cos^2(a, d), a = a0 (1 + u), and (grad_dev non-NULL) its
 * gradient with respect to the weights (FP64, adc3_mlp_nparams() entries).  loss: host. */
int adc3_mlp_loss_grad(const float* weights_dev, const double* feat_dev, const double* a0_dev,
                       const double* target_dev, int ngroups, int group_size, double* grad_dev, double* loss,
                       void* workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* u_dev[n] = MLP(feat_dev[n][6]) as in training: FP32 matrix cores, FP32 accumulation.
 * Workspace: adc3_mlp_workspace_bytes(1, n). */
int adc3_mlp_forward(const float* weights_dev, const double* feat_dev, long long n, double* u_dev,
                     void* workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* One preconditioning step t = P(theta) r on the context: the learned step (fused BF16
 * inference, as used inside adc3_ea_davidson) if a preconditioner is set, else the
 * Jacobi step r/(D - theta).  r_dev, t_dev: adc3_ea_dim() doubles on the device.
 * *fallback (nullable) is set to 1 if a non-finite learned step fell back to Jacobi
 * at some element. */
int adc3_ea_precondition(adc3_ctx* ctx, double theta, const double* r_dev, double* t_dev, int* fallback,
                         hipStream_t stream);

/* Adam training on the GPU (lr, beta 0.9/0.999, eps 1e-8): epochs over the groups in a
 * seeded shuffled order, batch_groups groups per step; weights_dev updated in place
 * (FP32 master weights); loss_per_epoch (host, nullable) receives the mean batch loss. */
int adc3_mlp_train(float* weights_dev, const double* feat_dev, const double* a0_dev, const double* target_dev,
                   int ngroups, int group_size, int epochs, int batch_groups, double lr, unsigned long long seed,
                   double* loss_per_epoch, void* workspace_dev, size_t workspace_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Timing (tracing aid, not part of the method).  When enabled, HIP events are
 * recorded on the launching stream around: 0 = each sigma-ladder GEMM launch
 * (with its algorithmic flops 2*(nvec*nocc)*nvir^4 and bytes), 1 = each sigma
 * build, 2 = each secular-matrix setup, 3 = each Davidson solve, 4 = each large
 * eigensolve, 5 = each reduced-precision sigma-ladder launch.  adc3_profile_enable(1) resets and starts; (0) stops.
 * adc3_profile_query synchronises the recorded events and returns the summed
 * milliseconds, the number of timed launches, and the summed flops and bytes.
 * adc3_profile_query_bound returns, for the ladder ids (0, 5), the summed roofline time of
 * the launches, each max(flops / matrix-core peak of its precision, bytes / 8 TB/s) with
 * MI355X's published peaks (FP64 78.6, FP32 157.3, BF16 2500 TFLOP/s); 0 for other ids.
 * ------------------------------------------------------------------------- */
void adc3_profile_enable(int on);
int adc3_profile_query(int kernel, double* total_ms, long long* count, double* flops, double* bytes);
int adc3_profile_query_bound(int kernel, double* bound_ms);

#ifdef __cplusplus
}
#endif
#endif /* ADC3EA_H */
