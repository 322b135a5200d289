/*
 * cpm.h -- C-ABI of libcpm, the MI355X (gfx950) constant-potential-method
 * electrode charge solve of the ELECTRODE paper (Ahrens-Iwers et al.,
 * arXiv 2203.15461).
 *
 * The problem (Sec. II.A, Eq. 2): electrode atoms i = 0..n-1 carry Gaussian
 * charges q_i of reciprocal width eta (the rho_i of Sec. III.B).  Their
 * Coulomb energy is U = 1/2 q^T A q - b^T q - v^T q, where A (the elastance
 * matrix) is fixed while the electrodes do not move, b depends on the
 * electrolyte positions and must be recomputed every step, and v = G v~
 * holds the applied potential of each atom's electrode (Sec. II.B, Eq. 5).
 * With total charge held at zero the minimiser is q = S (b + v), with
 * S = A^-1 - A^-1 e e^T A^-1 / (e^T A^-1 e) (Eqs. 3, 4, 6).  The slab
 * geometry adds the EW3DC dipole term (Eq. 10), split into an electrode part
 * that enters A and an electrolyte cross term that enters b (Eq. 12).
 *
 * Call order: cpm_create -> cpm_set_electrolyte -> cpm_build_elastance ->
 * cpm_invert -> cpm_set_potential -> (cpm_potential_vector ->
 * cpm_solve_charges)*.  Anything else returns CPM_ESTATE.
 *
 * Conventions (every entry point):
 *  - units: Angstrom, elementary charge e, volt.  b is minus the electrolyte
 *    potential at the electrode atoms (V), so that A q = b + v at the minimum.
 *  - pointers named d_* are device (HBM) pointers owned by the caller; h_*
 *    are host pointers owned by the caller.  The context owns everything it
 *    allocates (A, S and its FP32 / split-BF16 copies, u, d, k-set tables,
 *    workspaces) and frees it in cpm_destroy.
 *  - work is enqueued on the HIP stream given to cpm_create (NULL = the
 *    default stream) and is asynchronous unless stated otherwise.  A kernel
 *    fault surfaces as CPM_EHIP at the next synchronising call.
 *  - arguments are validated on the host before any device work; on error
 *    nothing is enqueued and cpm_last_error() says why.
 *  - one context per stream; contexts are not thread safe.
 */
#ifndef CPM_H
#define CPM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpm_ctx cpm_ctx;

typedef enum {
  CPM_OK = 0,
  CPM_EINVAL = 1,        /* bad argument (size, range, non-finite, non-neutral) */
  CPM_ESTATE = 2,        /* call out of order                                   */
  CPM_ENOMEM = 3,        /* device allocation failed                            */
  CPM_EHIP = 4,          /* HIP runtime error (launch, fault, copy)             */
  CPM_ENOTPD = 5,        /* A is not positive definite (Cholesky pivot <= 0)     */
  CPM_EUNSUPPORTED = 6,  /* valid request the library does not provide         */
  CPM_ENOCONV = 7        /* iteration stopped at its limit above the tolerance  */
} cpm_status;

/* Boundary geometry (Sec. II.E).  All three use the Ewald sum of the
 * Lx x Ly x Lz cell, Lz = slab_factor * h, with every periodic image within
 * rcut in real space, plus a dipole term:
 *   CPM_GEOM_SLAB_EW3DC: x, y periodic, vacuum in z (Eq. 10; (slab_factor -
 *     1) * h > rcut required); A += k_e (4 pi / V) z z^T, b -= k_e (4 pi / V) z M_z.
 *   CPM_GEOM_WIRE: periodic in z only, the x, y box extended (Eq. 11);
 *     A += k_e (2 pi / V)(x x^T + y y^T), b -= k_e (2 pi / V)(x M_x + y M_y).
 *   CPM_GEOM_3D: periodic in x, y and z with no dipole term (tin foil), the
 *     setting of the finite-field method (Sec. II.F; pass slab_factor 1 and
 *     h = the cell height, and the field potential through cpm_set_field).
 * Dipole terms use the coordinates as given (not wrapped). */
typedef enum { CPM_GEOM_SLAB_EW3DC = 0, CPM_GEOM_WIRE = 1, CPM_GEOM_3D = 2 } cpm_geom;

/* Which copies of S cpm_invert keeps (bit set).  FP64 is always kept. */
enum { CPM_STORE_F64 = 1, CPM_STORE_F32 = 2, CPM_STORE_BF16X2 = 4 };
/* cpm_invert flags: enqueue the inversion on a second stream of the context
 * and return at once; stop at the Cholesky factor instead of forming S
 * (see cpm_invert). */
enum { CPM_INVERT_ASYNC = 0x100, CPM_INVERT_FACTOR = 0x200 };

/* Solve modes for cpm_solve_charges.  The low byte picks the copy of S that
 * is streamed; CPM_SOLVE_REFINE adds one FP64 refinement step against A. */
enum {
  CPM_SOLVE_F64 = 0,
  CPM_SOLVE_F32 = 1,
  CPM_SOLVE_BF16X2 = 2,
  CPM_SOLVE_REFINE = 0x100,
  CPM_SOLVE_CCM = 0x200       /* constrained electrode charges (Eq. 7) instead of
                                 the applied potential; FP64 only, needs
                                 cpm_set_charge                                    */
};

/* Keys for cpm_get_info. */
enum {
  CPM_INFO_N = 0,             /* electrode atoms                                  */
  CPM_INFO_NK = 1,            /* half-space k-vectors |K+|                        */
  CPM_INFO_NE = 2,            /* electrodes                                       */
  CPM_INFO_S_SUM = 3,         /* s = e^T A^-1 e (e/V), after cpm_invert           */
  CPM_INFO_PIVOT = 4,         /* failing Cholesky pivot index after CPM_ENOTPD    */
  CPM_INFO_LZ = 5,            /* Ewald cell height slab_factor * h (A)            */
  CPM_INFO_KCUT = 6,          /* k-space cutoff used (1/A)                        */
  CPM_INFO_M = 7,             /* electrolyte charges                              */
  CPM_INFO_WORKSPACE = 8,     /* device bytes held by the context                 */
  CPM_INFO_NPAD = 9,          /* padded matrix order (multiple of 64)             */
  CPM_INFO_NRUNS = 10,        /* k-space runs (<= 16 consecutive k_z each)        */
  CPM_INFO_NLAYERS = 11,      /* z planes of the electrodes when <= 64 (planar    */
                              /* factorisation of the k-space projection), else 0 */
  CPM_INFO_SF_MATRIX = 12,    /* 1: FP64 structure factors run on matrix cores    */
  CPM_INFO_TUNE_BM = 13,      /* last cpm_autotune: rows of X per GEMM tile       */
  CPM_INFO_TUNE_KS = 14,      /*   ... parts the K dimension is split into        */
  CPM_INFO_TUNE_GRID = 15,    /*   ... workgroups of the persistent launch        */
  CPM_INFO_TUNE_US = 16,      /*   ... measured microseconds per product          */
  CPM_INFO_GROUP = 17,        /* configurations per launch group of              */
                              /* cpm_potential_vector (planar electrodes)         */
  CPM_INFO_CG_ITERS = 18,     /* last cpm_solve_cg: most iterations of a vector   */
  CPM_INFO_CG_RESID = 19,     /*   ... largest final |r| / |r0|                   */
  CPM_INFO_ELL_WIDTH = 20,    /* entries per row of the operator's real-space     */
                              /* part (cpm_build_operator)                        */
  CPM_INFO_NCOLS = 21,        /* (k_x, k_y) columns of the matrix-core k set      */
  CPM_INFO_BSR_BLOCKS = 22,   /* 64 x 64 blocks of the operator's real space      */
  CPM_INFO_PC_TILES = 23,     /* last cpm_solve_cg: tiles of its preconditioner   */
                              /*   (0: plain CG)                                  */
  CPM_INFO_PC_MODE = 24,      /*   ... its form: 0 none, 1 additive, 2 balancing  */
  CPM_INFO_PC_COARSE = 25,    /*   ... its coarse-space dimension                 */
  CPM_INFO_SF_FP32 = 26,      /* cpm_potential_vector with b_is_f32 forms the     */
                              /* structure factors on FP16 matrix cores with      */
                              /* split operands (2) or FP32 matrix cores (1)      */
  CPM_INFO_RS_PLANE = 27      /* 1: the real-space part of b runs the planar      */
                              /* kernel (atoms on z planes, one image within r_c) */
};

/* Method knobs; they map onto the paper's `fix electrode` keywords and the
 * Ewald solver (Sec. S-I.A). */
typedef struct {
  double Lx, Ly;        /* in-plane periodic cell (A)                               */
  double h;             /* slab height z_top - z_bot of the electrodes (A)          */
  double slab_factor;   /* Ewald cell height Lz = slab_factor * h; needs
                           (slab_factor - 1) * h > rcut                             */
  double eta;           /* Gaussian reciprocal width of electrode charges (1/A)    */
  double alpha;         /* Ewald splitting parameter (1/A)                          */
  double rcut;          /* real-space cutoff (A), strict r < rcut                   */
  double kspace_eps;    /* k_c = 2 alpha sqrt(ln(1/kspace_eps)) if kcut <= 0        */
  double kcut;          /* explicit k-space cutoff (1/A), |k| <= kcut; 0 = derive   */
  double coulomb_k;     /* e/(4 pi eps0) in V A / e; 0 = 14.399645478425668         */
  int geometry;         /* cpm_geom                                                 */
} cpm_params;

/* Create a context bound to `hip_stream` (a hipStream_t, or NULL).
 * Validates params (finite, positive, slab clearance) and builds the k set on
 * the host; no device work happens before cpm_build_elastance.  *out is NULL
 * on error. */
cpm_status cpm_create(const cpm_params* params, void* hip_stream, cpm_ctx** out);

/* Electrolyte point charges h_q[m] (e), fixed for the run.  Host pointer,
 * copied (uploaded on first device use); the charges must sum to zero within
 * 1e-10 sum|q| (the slab term of Eq. 12 assumes a neutral electrolyte), else
 * CPM_EINVAL.  m >= 0.  Call once per context (CPM_ESTATE otherwise). */
cpm_status cpm_set_electrolyte(cpm_ctx* ctx, int m, const double* h_q);

/* Assemble the n x n elastance matrix A in FP64 on the device (Eq. 2, A
 * fixed and precomputed, Sec. II.A): Ewald real space over periodic images,
 * k space over K+, Gaussian self term, background and the electrode part of
 * the slab dipole term (Eq. 12).  d_xyz: n x 3 row-major FP64 electrode
 * coordinates; d_electrode_id: n int32 ids in [0, n_e); d_diag_extra: n FP64
 * (V/e) added to the diagonal, or NULL.  Validates ids and coordinates
 * (copying them to the host once) and prepares the electrode data; returns
 * once the inputs have been read (they may then be freed).  The kernels that
 * form A itself are enqueued by the first call that needs A: cpm_invert (on
 * its own stream with CPM_INVERT_ASYNC, so the assembly overlaps b as well),
 * cpm_copy_matrix(0), cpm_apply_elastance or cpm_solve_cg. */
cpm_status cpm_build_elastance(cpm_ctx* ctx, int n, const double* d_xyz,
                               const int* d_electrode_id, int n_e,
                               const double* d_diag_extra);

/* The elastance as an operator instead of a matrix, for the
 * conjugate-gradient solve that Sec. II.A names as the alternative to
 * inverting A (and Sec. IV as future work): the same electrode set-up and
 * arguments as cpm_build_elastance, but A is never formed.  Keeps the
 * real-space and self terms as a sparse matrix (ELL: one entry per electrode
 * pair with a periodic image within r_c, at most CPM_INFO_ELL_WIDTH per
 * atom) stored as dense 64 x 64 blocks of interacting 64-atom tiles
 * (CPM_INFO_BSR_BLOCKS), and applies the k-space term through the electrode
 * planes (memory O(n x columns) for the in-plane phases).
 * Needs electrodes on at most 64 z planes and the matrix-core k set
 * (CPM_INFO_NLAYERS > 0, CPM_INFO_SF_MATRIX = 1), else CPM_EUNSUPPORTED.
 * A context holds either the dense elastance or the operator (CPM_ESTATE).
 * cpm_set_potential, cpm_set_potential_atoms and cpm_potential_vector work as
 * after cpm_invert; cpm_solve_charges does not (no S).  Synchronous. */
cpm_status cpm_build_operator(cpm_ctx* ctx, int n, const double* d_xyz,
                              const int* d_electrode_id, int n_e,
                              const double* d_diag_extra);

/* y = A x for `batch` vectors (Eq. 2's elastance applied to charges, e.g.
 * for the energy q^T A q / 2): d_x, d_y batch x n FP64 device arrays.  Uses
 * the operator of cpm_build_operator, or the dense A after
 * cpm_build_elastance.  Enqueued on the context stream. */
cpm_status cpm_apply_elastance(cpm_ctx* ctx, int batch, const double* d_x, double* d_y);

/* Conjugate-gradient solve (Sec. II.A's alternative to the inversion):
 * q minimises the energy with e^T q = 0, i.e. A q = b + v + mu e, by
 * conjugate gradients on the neutral subspace (projector I - e e^T / n),
 * starting from q = 0, in FP64, with A applied by the operator of
 * cpm_build_operator or, after cpm_build_elastance, by the dense A.
 * d_b: batch x n (FP64, or FP32 with b_is_f32 = 1); v from
 * cpm_set_potential(_atoms).  Each vector stops when |r| <= tol |r0| (r the
 * projected residual, recursively updated); at most maxit iterations.
 * Vectors run in groups of 64.  With the operator the iteration is
 * preconditioned (built on the first solve after cpm_build_operator) by a
 * two-level method over the operator's 64-atom plane tiles: the smoother
 * B = the inverses of A's 64 x 64 diagonal tile blocks, the coarse space Z =
 * per tile its constant and, for the balancing form on operators of at
 * least 128 tiles, the two in-plane offsets from the tile's centre
 * (environment CPM_CG_COARSE=1 or 3 forces 1 or 3 functions per tile),
 * Q = Z (Z^T A Z)^-1 Z^T, in the balancing form
 * M^-1 = Q + (I - Q A) B (I - A Q) (default) or the additive form
 * M^-1 = B + Q (environment CPM_CG_PRECOND=1; 0: none).  The stopping test
 * stays |r| <= tol |r0| on the unpreconditioned residual.  Operators with
 * more than 2048 tiles and the dense A run plain CG.  Blocks of 8
 * iterations replay one HIP graph, captured on first use for the current
 * buffers, tolerance and preconditioner (environment CPM_CG_GRAPH=0, a
 * capture the runtime refuses, or kernel timing: plain launches); a context
 * on the NULL stream runs the solve on an internal stream after draining the
 * NULL stream.
 * Writes d_q (batch x n FP64, the final
 * iterate projected to e^T q = 0) and, unless NULL, d_Qe (batch x n_e
 * electrode totals).  Synchronous (the host checks convergence every 8
 * iterations).  CPM_ENOCONV if some vector ended above the tolerance (the
 * outputs then hold the last iterates).  CPM_INFO_CG_ITERS and
 * CPM_INFO_CG_RESID report the iterations and residual reached. */
cpm_status cpm_solve_cg(cpm_ctx* ctx, int batch, const void* d_b, int b_is_f32, double tol,
                        int maxit, double* d_q, double* d_Qe);

/* Invert A in FP64 (blocked Cholesky A = L L^T, then A^-1 = L^-T L^-1,
 * Eq. 3), form u = A^-1 e, s = e^T u and the charge-neutral S of Eq. 4, and
 * keep the copies of S named by store_flags (CPM_STORE_*).  The assembly of
 * A left by cpm_build_elastance runs first, on the same stream.  Synchronous;
 * returns CPM_ENOTPD (pivot via CPM_INFO_PIVOT) if A is not positive
 * definite. */
/* With CPM_INVERT_ASYNC in store_flags the work runs on a second stream of
 * default priority, ordered after the work already enqueued on the context
 * stream, and the call returns without waiting: a following
 * cpm_potential_vector (which needs no inverse) overlaps it.  The first call
 * that needs the inverse -- cpm_set_potential(_atoms), cpm_solve_charges,
 * cpm_set_charge, cpm_autotune, cpm_solve_grouped, cpm_capture_step,
 * cpm_replay_step, cpm_copy_matrix/vector, cpm_get_info(S_SUM or PIVOT),
 * cpm_synchronize -- waits for it and returns CPM_ENOTPD there if a pivot
 * failed; a rebuild or another cpm_invert waits for it first. */
/* With CPM_INVERT_FACTOR (store_flags then names no copy of S) the work
 * stops at the factor: A = L L^T is kept (FP64, with the inverses of its
 * 64 x 64 diagonal blocks) and A^-1 x is formed by forward and back
 * substitution, 2 n^2 flop per vector and direction, instead of the
 * 2 n^3 / 3 flop of L^-1 and L^-T L^-1: u, s and the response S G come from
 * the solves with the n_e electrode indicators (n_e <= 16, else
 * CPM_EUNSUPPORTED), and cpm_solve_charges (CPM_SOLVE_F64 only) forms
 * S (b + v) = P A^-1 b + d with P = I - u e^T / s.  For few configurations
 * per electrode geometry this saves most of the set-up.  cpm_set_potential,
 * cpm_set_potential_atoms and cpm_set_field work as with S; calls that need
 * S itself or A^-1 (other solve modes, cpm_set_charge, cpm_autotune,
 * cpm_solve_grouped, cpm_capture_step, cpm_save, cpm_copy_matrix of A^-1 or
 * S, cpm_solve_charges_noalloc) return CPM_ESTATE. */
cpm_status cpm_invert(cpm_ctx* ctx, unsigned store_flags);

/* Applied potentials h_v_electrode[n_e] (V), one per electrode (v = G v~,
 * Eq. 5).  Sets d = S v for the solves to add.  cpm_invert keeps the
 * response S G (n x n_e, Eq. 6), so for n_e <= 16 this is one O(n n_e)
 * kernel with the potentials passed by value: nothing is copied and the
 * call does not wait (a time-varying potential costs no pass over S).
 * More electrodes: v is uploaded and d = S v streamed, synchronously.  Host
 * pointer, read before return. */
cpm_status cpm_set_potential(cpm_ctx* ctx, const double* h_v_electrode);

/* The same with one potential per electrode atom, h_v[n] (V, host memory):
 * d = S v for any v (one pass over S and a wait for the stream). */
cpm_status cpm_set_potential_atoms(cpm_ctx* ctx, const double* h_v);

/* Finite-field method (Sec. II.F, Eqs. 13-14; the `ffield` keyword of
 * Sec. S-I.A): the library forms the field potential itself.  Every atom
 * gets v_i = -dv0 zeta_i with zeta_i = z_i / Lz (Lz = slab_factor * h, the
 * z coordinates as given to cpm_build_elastance) plus 1 for the atoms of
 * electrode `bottom`, which puts the two electrodes next to each other
 * across the periodic z boundary as one conductor.  dv0 (V) is the
 * potential drop across the periodic boundary; with electrodes that do not
 * let the field through, it is the potential difference between them.
 * Needs CPM_GEOM_3D (CPM_EUNSUPPORTED otherwise) and 0 <= bottom < n_e
 * (CPM_EINVAL).  The first call after cpm_invert (or with a new `bottom`)
 * uploads zeta and forms S zeta with one pass over S; later calls with a new
 * dv0 cost one O(n) kernel and do not wait for the stream. */
cpm_status cpm_set_field(cpm_ctx* ctx, double dv0, int bottom);

/* b for `batch` electrolyte configurations (Sec. II.A: the per-step cost).
 * d_xyz: batch x m x 3 FP64 positions (row-major, snapshot-major).
 * d_b: batch x n output, FP64 (b_is_f32 = 0) or FP32 (b_is_f32 = 1, for
 * the reduced-precision solve modes).  With FP32 output the structure
 * factors run on FP16 matrix cores with split operands: every operand value
 * (phases formed in FP64, products of them in FP32) is carried as two FP16
 * numbers, hi and 2^11 (value - hi), a product as three FP16 products summed
 * in FP32 over a charge chunk (each value kept to about 2^-22 relative),
 * then in FP64; the rest of b stays FP64 until the final rounding.  b is
 * then within about 1e-6 (relative to its largest entry) of the FP64
 * result.  Switches read when a context is created: CPM_SF_F16=0 takes the
 * FP32 matrix-core kernel instead (FP32 phase tables and products, FP32
 * sums over 128 charges); CPM_SF_FP32=0 keeps FP64 structure factors.  b
 * includes the real-space erfc sum, the k-space structure-factor term and
 * the electrolyte cross term of the slab correction (Eq. 12). */
cpm_status cpm_potential_vector(cpm_ctx* ctx, int batch, const double* d_xyz,
                                void* d_b, int b_is_f32);

/* q = S (b + v) for `batch` vectors b (Eqs. 3, 4, 6), then the FP64
 * neutrality projection q -= (e^T q / s) u, and electrode totals
 * Q~ = G^T q (Eq. 7 left-hand side).  d_b: batch x n (FP64 or FP32 per
 * b_is_f32); d_q: batch x n FP64 output; d_Qe: batch x n_e FP64 output or
 * NULL.  mode: CPM_SOLVE_* (| CPM_SOLVE_REFINE).  FP64 with batch < 4 and
 * FP32 stream S once per vector (matvec); FP64 with batch >= 4 and split-BF16
 * (any batch) run Q = B S as one MFMA GEMM with rows padded to 64.  The
 * chosen copy of S must have been kept by cpm_invert, else CPM_EINVAL. */
cpm_status cpm_solve_charges(cpm_ctx* ctx, int batch, const void* d_b, int b_is_f32,
                             unsigned mode, double* d_q, double* d_Qe);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * solve as cpm_solve_charges (same arguments, modes, kernels and results),
 * with its work buffers in one fixed device array of
 * CPM_NOALLOC_SCRATCH_BYTES per GPU instead of context memory.  Nothing is
 * allocated or freed (the split-BF16 product runs without its split-K
 * option).  The array is held by every GPU the library runs on until the
 * process ends; each call clears the part it uses (a fill kernel).  Sizes:
 * the batch (rounded up to 64 for the matrix-core modes) times the padded
 * n, 5 doubles per element for the matrix-core modes, 4 otherwise, must fit
 * the array (e.g. 128 configurations at n = 2880), else CPM_EINVAL with the
 * bytes needed.  All calls on one GPU share the array: calls that overlap
 * in time on one GPU (two streams, two threads) race and must be ordered by
 * the caller.  The device's array address is looked up on the first call
 * on each device (the device current at the call). */
#define CPM_NOALLOC_SCRATCH_BYTES (16u << 20)
cpm_status cpm_solve_charges_noalloc(cpm_ctx* ctx, int batch, const void* d_b, int b_is_f32,
                                     unsigned mode, double* d_q, double* d_Qe);

/* Constrained charge method (Sec. II.C, Eq. 7): set the total charge of
 * each electrode, h_Q[n_e] (e, host memory; must sum to zero within 1e-12
 * relative, else CPM_EINVAL; n_e <= 16).  Computes U = A^-1 G and the
 * inverse of the electrode capacitance matrix C~ = G^T A^-1 G.  Later
 * cpm_solve_charges calls with CPM_SOLVE_F64 | CPM_SOLVE_CCM return
 * q = A^-1 (b + G v~) with v~ = C~^-1 (Q - G^T A^-1 b), so G^T q = Q.  Needs
 * cpm_invert (and again after every cpm_invert).  Synchronous. */
cpm_status cpm_set_charge(cpm_ctx* ctx, const double* h_Q);

/* Autotune the split-BF16 batched product Q~ = B S~ (the matrix-core solve
 * of Eqs. 3 and 6) for batches of `batch` vectors (rows padded to 64): times
 * every tile height (32, 64, 128 rows), K split (1, 2, 4) and persistent grid
 * size on this context's S, `reps` launches each, and keeps the fastest for
 * later cpm_solve_charges calls with the same padded row count.  Needs
 * cpm_invert with CPM_STORE_BF16X2.  Synchronous.  The choice changes only
 * the FP32 summation order of the product; results stay within the path's
 * tolerance.  CPM_INFO_TUNE_* report the choice. */
cpm_status cpm_autotune(cpm_ctx* ctx, int batch, int reps);

/* Solve several contexts at once (electrodes of uneven size): the same as
 * cpm_solve_charges on each of the n_ctx <= 8 contexts, with every product
 * with S~ of all contexts done in one persistent split-BF16 launch (two with
 * CPM_SOLVE_REFINE).  mode must be CPM_SOLVE_BF16X2, optionally with
 * CPM_SOLVE_REFINE (else CPM_EUNSUPPORTED).  batch, d_b, d_q and d_Qe
 * (may be NULL, or hold NULL entries) are host arrays of n_ctx entries; the
 * contexts must be distinct and share one stream.  Errors are reported on
 * ctxs[0]. */
cpm_status cpm_solve_grouped(cpm_ctx* const* ctxs, int n_ctx, const int* batch,
                             const void* const* d_b, int b_is_f32, unsigned mode,
                             double* const* d_q, double* const* d_Qe);

/* Capture one batched step -- cpm_potential_vector for `batch`
 * configurations followed by cpm_solve_charges -- for these exact buffers
 * and mode into a HIP graph held by the context, replacing any earlier
 * capture.  The context stream must not be the default stream.  Work
 * buffers are allocated before capture; the graph holds kernel launches
 * only.  Nothing runs until cpm_replay_step. */
cpm_status cpm_capture_step(cpm_ctx* ctx, int batch, const double* d_xyz, void* d_b,
                            int b_is_f32, unsigned mode, double* d_q, double* d_Qe);

/* Launch the captured step on the context stream (asynchronous).  The caller
 * refreshes d_xyz between replays (stream-ordered before the replay); the
 * results land in the d_b, d_q, d_Qe given at capture.  cpm_set_potential
 * and a same-size cpm_invert between replays are seen by the next replay.
 * Returns CPM_ESTATE without launching if the context has allocated or
 * freed device memory since the capture (an eager call with a larger batch,
 * a rebuild) or no longer keeps the copy of S the captured mode reads:
 * capture again in that case. */
cpm_status cpm_replay_step(cpm_ctx* ctx);

/* The grouped step of several contexts (electrodes of uneven size, Sec. II.B
 * and the batched solve of cpm_solve_grouped) as one HIP graph:
 * cpm_potential_vector of every context (ctxs[i]: batch[i] configurations
 * d_xyz[i] into d_b[i]), then cpm_solve_grouped over all of them (split-BF16
 * mode 0x2 or 0x102), captured from the stream the contexts share (not the
 * default stream).  Every context needs its inverse with the split-BF16
 * copy of S and its potential set; work buffers are allocated before
 * capture, the graph holds kernel launches only and is kept by ctxs[0],
 * replacing its earlier grouped capture.  Nothing runs until
 * cpm_replay_grouped. */
cpm_status cpm_capture_grouped(cpm_ctx* const* ctxs, int n_ctx, const int* batch,
                               const double* const* d_xyz, void* const* d_b, int b_is_f32,
                               unsigned mode, double* const* d_q, double* const* d_Qe);

/* Launch the graph of cpm_capture_grouped on the shared stream
 * (asynchronous); ctxs must list the captured contexts in the captured
 * order (CPM_EINVAL otherwise).  As for cpm_replay_step: new coordinates go
 * into the captured d_xyz buffers, stream-ordered before the replay, and
 * cpm_set_potential or a same-size cpm_invert between replays are seen; a
 * context that allocated or freed device memory since the capture, lost its
 * split-BF16 copy of S or holds only the factor makes the call return
 * CPM_ESTATE without launching. */
cpm_status cpm_replay_grouped(cpm_ctx* const* ctxs, int n_ctx);

/* State files: the `write_mat` / `write_inv` and `read_mat` / `read_inv`
 * keywords of Sec. S-I.A.  cpm_save writes A and, after cpm_invert, A^-1
 * (n x n row-major FP64 each) with a 256-byte header holding n, n_e, the
 * kept copies of S, s = e^T A^-1 e, the method knobs and a 64-bit
 * fingerprint of everything A depends on (knobs, electrode coordinates and
 * ids as given, diagonal term), plus a trailing checksum of the matrices.
 * The file is written under path + ".tmp" and renamed when complete.
 * Synchronous; CPM_ESTATE before cpm_build_elastance.
 *
 * cpm_load reads such a file into a context that has run
 * cpm_build_elastance for the same electrodes and knobs: a different
 * fingerprint, n or n_e, a damaged header, a wrong length or checksum
 * returns CPM_EINVAL.  A file with A only replaces the assembly (call
 * cpm_invert next); with A^-1 as well it also replaces the inversion:
 * u, s, S, the response S G and the copies of S the saving context kept are
 * formed from the stored A^-1 by the same kernels as cpm_invert, so charges
 * solved after a load equal those of the saving context bit for bit.
 * cpm_set_potential must follow.  Synchronous. */
cpm_status cpm_save(const cpm_ctx* ctx, const char* path);
cpm_status cpm_load(cpm_ctx* ctx, const char* path);

/* What a state file holds (host only; no device work). */
typedef struct {
  int n, n_e;
  int matrices;                 /* 1: A; 2: A and A^-1                            */
  unsigned store;               /* CPM_STORE_* copies kept by the saving context  */
  unsigned long long geometry_hash;
  double s_sum;                 /* e^T A^-1 e (0 with A only)                     */
  cpm_params params;            /* knobs; coulomb_k holds the k_e used            */
} cpm_file_info;

/* Read and check a state file's header and length (not the matrices'
 * checksum).  CPM_EINVAL if the file is missing, not a state file, of
 * another version, damaged or of the wrong length. */
cpm_status cpm_inspect_file(const char* path, cpm_file_info* out);

/* Copy a context matrix (n x n, row-major FP64) into caller memory d_out:
 * which = 0: A, 1: A^-1, 2: S.  Enqueued on the context stream. */
cpm_status cpm_copy_matrix(const cpm_ctx* ctx, int which, double* d_out);

/* Copy u = A^-1 e (n FP64) or d = S v (which = 1) into caller memory d_out. */
cpm_status cpm_copy_vector(const cpm_ctx* ctx, int which, double* d_out);

/* Scalar information (CPM_INFO_*). */
cpm_status cpm_get_info(const cpm_ctx* ctx, int key, double* out);

/* Kernel timing.  families = NULL or "" turns it off; "*" times every
 * kernel the library launches on the context stream; otherwise a
 * comma-separated list of kernel families (for example "structure_factor",
 * "kspace_project", "real_space_b", "matvec_f64", "gemm_f64") restricts it to
 * those.  Each timed launch is bracketed by two HIP event records and its
 * elapsed time is accumulated per family.  Every call clears the totals. */
cpm_status cpm_enable_timing(cpm_ctx* ctx, const char* families);

/* Total milliseconds and launch count of kernel family `name` recorded since
 * timing was enabled.  Synchronises the context stream.  A family that never
 * ran reports 0 and 0. */
cpm_status cpm_get_timing(cpm_ctx* ctx, const char* name, double* total_ms, long long* count);

/* Wait for all work of the context and report any pending HIP error. */
cpm_status cpm_synchronize(cpm_ctx* ctx);

/* Human-readable reason for the last non-OK status of ctx (never NULL). */
const char* cpm_last_error(const cpm_ctx* ctx);

/* Free everything the context owns.  NULL is a no-op. */
void cpm_destroy(cpm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* CPM_H */
