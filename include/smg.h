/*
 * smg.h -- adaptive multigrid for the 2D U(1) Wilson-Dirac normal equations on MI355X.
 *
 * C ABI of libsmg.so.  The library solves the normal equations
 *
 *     A x = rhs,   A = D^H D,
 *
 * of the Wilson-Dirac operator D (Introduction of Brannick, Brower, Clark, Osborn,
 * Rebbi, "Adaptive Multigrid Algorithm for the QCD Dirac-Wilson Operator",
 * arXiv:0710.3612) with conjugate gradients preconditioned by an adaptive
 * multigrid V-cycle (Multigrid and Adaptive Multigrid sections, Eqs. 2-5).
 * A caller who wants D psi = chi passes rhs = D^H chi (formed with smg_apply_D,
 * dagger = 1) and gets psi = x.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice     lx * lt sites, site s = t*lx + x, periodic; direction mu = 0 is x,
 *             mu = 1 is t.  gamma_x = sigma1, gamma_t = sigma2 (2 spins per site).
 * Operator    D psi_s = (2 + m) psi_s - 1/2 sum_mu [ (1 - gamma_mu) U_s^mu psi_{s+mu}
 *                        + (1 + gamma_mu) conj(U_{s-mu}^mu) psi_{s-mu} ].
 *             The diagonal is (d + m) with d = 2 (standard Wilson normalisation: the
 *             free operator at zero momentum is m); the paper prints (2d + m),
 *             which is this operator at mass m + 2.
 * Fermion BC  periodic in x; antiperiodic in t when params.t_antiperiodic != 0.
 * Vectors     complex128, real and imaginary parts interleaved.  A batch of
 *             nrhs fine vectors is [nrhs][lt][lx][2]; a batch of vectors on
 *             multigrid level l >= 1 is [nrhs][lt_l][lx_l][nv_{l-1}].
 * Gauge       complex128 [2][lt][lx]: gauge[mu][t][x] = U_{(x,t)}^mu, |U| = 1.
 * Pointers    "device" pointers are HIP device memory of the current device
 *             (for example the data pointer of a torch CUDA tensor); "host"
 *             pointers are ordinary host memory.  The caller owns every pointer
 *             it passes; the library never frees or retains them beyond the call.
 * Streams     `stream` is a hipStream_t (NULL = the null stream).  Everything is
 *             enqueued on it.  Calls marked ASYNC return before the work is done;
 *             all other calls synchronise the stream before returning.
 *             One handle may be used by one stream at a time.
 * Errors      every int-returning call returns SMG_OK (0), a negative error code
 *             or SMG_NOTCONV (+1, a warning).  smg_strerror() names a code and
 *             smg_last_error() describes the most recent failure of this thread.
 *             On error the outputs are unspecified and the handle stays valid.
 */
#ifndef SMG_H
#define SMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMG_MAXLEV 6

enum {
  SMG_OK = 0,
  SMG_NOTCONV = 1,      /* solve stopped at maxiter; x holds the last iterate */
  SMG_EINVAL = -1,      /* invalid argument or parameter */
  SMG_ESHAPE = -2,      /* lattice extents not divisible by the block extents */
  SMG_ENOMEM = -3,      /* device allocation failed */
  SMG_EDEVICE = -4,     /* a HIP runtime call failed */
  SMG_EBREAKDOWN = -5,  /* NaN/Inf, or <p, A p> <= 0 in a Krylov iteration */
  SMG_ESETUP = -6,      /* degenerate aggregate in Gram-Schmidt, or coarsest factorisation failed */
  SMG_EBUSY = -7        /* no free slot in a batch */
};

enum { SMG_COARSEST_DIRECT = 0, SMG_COARSEST_CG = 1 };
enum { SMG_FP64 = 0, SMG_MIXED = 1 };

/* reduced-precision storage in the FP32 V-cycle (smoother iterates, operators) */
enum { SMG_STORE_F32 = 0, SMG_STORE_BF16 = 1, SMG_STORE_F16 = 2 };

typedef struct smg_ctx* smg_handle;
typedef struct smg_batch_s* smg_batch;
typedef struct smg_group_s* smg_group;

typedef struct {
  int32_t lx, lt;                 /* fine extents, even, divisible by the product of blocks */
  double mass;                    /* m of the operator above */
  int32_t levels;                 /* L >= 1 grid levels; 1 = no coarsening (plain CG) */
  int32_t block[SMG_MAXLEV][2];   /* aggregate extents (bx, bt) of coarsening l -> l+1 */
  int32_t nv[SMG_MAXLEV];         /* near-null vectors of coarsening l (the paper's M) */
  int32_t setup_iters;            /* relaxation / V-cycle passes per candidate vector */
  int32_t smoother_steps;         /* nu: degree of the frozen minimal-residual polynomial */
  double smoother_omega;          /* under-relaxation of the MR steps (paper: 0.8) */
  int32_t t_antiperiodic;         /* 1: antiperiodic fermion BC in t */
  int32_t coarsest;               /* SMG_COARSEST_DIRECT (dense inverse) or SMG_COARSEST_CG */
  double coarsest_tol;            /* relative residual of the coarsest CG (and setup cycles) */
  int32_t coarsest_maxiter;       /* iteration cap of every coarsest CG */
  double inner_tol;               /* mixed precision: relative residual of each inner FP32 solve */
  uint64_t seed;                  /* random starts of the setup when none are passed in */
  double sa_scale;                /* smoothed aggregation: P = (I - w A) P_t with
                                     w = sa_scale / lambda_max(A) (20 power iterations from
                                     the calibration start); 0 = plain aggregation.  Applied
                                     where both block extents are >= 4 and both coarse
                                     extents >= 2 (the coarse operator stays 9-point). */
  int32_t smoother_storage;       /* mixed precision: storage of the fine-level smoother
                                     iterates in the FP32 V-cycle, SMG_STORE_F32 / _BF16 /
                                     _F16 (arithmetic stays FP32; BF16/FP16 need
                                     lx % 32 == 0 and lt % 16 == 0) */
  int32_t stop_recursive;         /* FP64 MG-CG and CG: 0 (default) = converged when the recomputed
                                     residual ||rhs - A x|| / ||rhs|| reaches tol; 1 = when CG's
                                     recursive residual does (the true one is still reported) */
  int32_t mfma_min_rhs;           /* coarse applies of at least this many right-hand sides run
                                     on the matrix cores (levels with nc <= 16: MFMA FP32 in
                                     the FP32 V-cycle; MFMA FP64, with the FP64 restriction and
                                     prolongation, in FP64); 1 = always, 0 = never.  Results
                                     differ from the vector-ALU path by rounding only, so a
                                     column's rounding in smg_solve / smg_vcycle can depend on
                                     nrhs; batches pin the choice by their capacity. */
  int32_t operator_storage;       /* mixed precision: storage of the FP32 V-cycle's coarse
                                     links (vector-ALU path; the matrix-core path keeps FP32),
                                     prolongators and coarsest dense inverse, SMG_STORE_F32 or
                                     SMG_STORE_F16 (each array scaled by a power of two so
                                     that its entries are at most 1; arithmetic stays FP32,
                                     the outer FP64 correction sets the final accuracy) */
  int32_t split_chirality;        /* 1: every aggregate is split by chirality (Adaptive Multigrid
                                     section: aggregates are subsets of variables).  The
                                     variables d of a block with d % 2 = 0 and with d % 2 = 1
                                     (on the fine lattice the spin components, gamma5 = sigma3)
                                     form two aggregates, so a coarse site carries 2 nv[l]
                                     variables, ordered 2k + chi for candidate k and chirality
                                     chi, and P maps chirality to chirality on every level.
                                     Needs nv[l] <= bx * bt * dof / 2 and 2 nv[l] <= 64.
                                     0 (default): one aggregate per block, nv[l] variables. */
  int32_t coarsest_fp64;          /* mixed precision, dense coarsest solve: 1 (default) = the FP32
                                     V-cycle applies the FP64 inverse with FP64 sums (its FP32
                                     input widened exactly, the result rounded to FP32), so the
                                     coarsest direct solve stays FP64; 0 = it applies an FP32
                                     copy of the inverse, or an FP16 copy under operator_storage
                                     SMG_STORE_F16 (a quarter of the bytes per V-cycle) */
  int32_t remass_affine;          /* 1: smg_setup and smg_setup_from_vectors also keep the mass
                                     coefficients of every coarse operator, A^(l)(m) = C2 + m C1
                                     + m^2 C0 with the prolongators fixed (three arrays of the
                                     level's link size, from the Galerkin operators at m = 0, 1,
                                     -1), and smg_derive / smg_set_mass form the coarse operators
                                     of a new mass from them in one pass over the links instead of
                                     Eq. 2.  Derived handles keep none (they derive by Eq. 2).
                                     0 (default): every mass change rebuilds by Eq. 2. */
  double nv_stop_rho;             /* > 0: adaptive number of vectors (Adaptive Multigrid section:
                                     the procedure is repeated until a V-cycle reduces a random
                                     error sufficiently).  After each appended vector of coarsening
                                     l (the first included) smg_setup measures the two-level
                                     cycle's convergence factor on the level's calibration start,
                                     (||e||_A / ||e_0||_A)^(1/s) after s = nv_stop_iters passes of
                                     e <- e - V A e, and stops adding vectors once it is <=
                                     nv_stop_rho; nv[l] is then the most the level takes and the
                                     next level carries as many variables per site as were kept
                                     (smg_level_info).  The random starts keep their full-nv
                                     layout; a shorter level uses the leading entries of its
                                     rows.  0 (default): exactly nv[l] vectors. */
  int32_t nv_stop_iters;          /* passes s of the factor above (default 3) */
} smg_params;

typedef struct {
  int32_t status;                 /* SMG_OK or SMG_NOTCONV for this right-hand side */
  int32_t iterations;             /* outer Krylov iterations (summed over refinements) */
  int32_t refinements;            /* defect-correction cycles (1 for SMG_FP64) */
  int32_t vcycles;                /* V-cycles applied */
  int64_t fine_applies;           /* applications of A on the fine lattice (2 of D/D^H each) */
  double true_relres;             /* ||rhs - A x|| / ||rhs|| recomputed in FP64 at exit */
  double seconds;                 /* wall time of the whole call */
} smg_stats;

/* Fill *p with the defaults: 2 levels of 4x4 blocks, Nv = 8, setup_iters = 5,
 * nu = 4, omega = 0.8, antiperiodic t, dense coarsest, coarsest_tol = 1e-12,
 * coarsest_maxiter = 10000, inner_tol = 1e-5, seed = 1, sa_scale = 4/3,
 * smoother_storage = SMG_STORE_F32, stop_recursive = 0, mfma_min_rhs = 16,
 * operator_storage = SMG_STORE_F32, split_chirality = 0, coarsest_fp64 = 1,
 * remass_affine = 0, nv_stop_rho = 0, nv_stop_iters = 3. */
void smg_default_params(smg_params* p);

/* Adaptive setup (Adaptive Multigrid section; recursion and reuse in Results).
 * gauge: device, complex128 [2][lt][lx] (copied; not retained).
 * randoms: device or NULL.  When given, the random starts of every coarsening,
 *   concatenated over l = 0..levels-2, each block complex128 [1 + nv[l]][n_l] with
 *   n_l the vector length of level l: row 0 starts the smoother calibration and
 *   rows 1..nv[l] start the candidate vectors.  When NULL they are drawn from
 *   params.seed by the library.
 * On success *out is a new handle owning all device memory of the hierarchy.
 * Errors: SMG_EINVAL, SMG_ESHAPE, SMG_ENOMEM, SMG_EDEVICE, SMG_ESETUP. */
int smg_setup(const double* gauge, const smg_params* params, const double* randoms,
              void* stream, smg_handle* out);

/* Hierarchy from given near-null vectors, skipping the adaptive iteration (block
 * Gram-Schmidt of the Adaptive Multigrid section, then Eq. 2 on every level).
 * vectors: device, concatenated over coarsenings, block l complex128 [nv[l]][n_l].
 * calib: device, concatenated over coarsenings, block l complex128 [n_l]; starts
 *   the smoother calibration of level l.
 * Errors as smg_setup. */
int smg_setup_from_vectors(const double* gauge, const smg_params* params, const double* vectors,
                           const double* calib, void* stream, smg_handle* out);

/* Change the mass, reusing the prolongators (Results: the setup is done at the
 * lightest mass and its vectors are reused for heavier masses).  Rebuilds every
 * coarse operator by Eq. 2 and recalibrates the smoothers from the stored
 * calibration starts.  Errors: SMG_EINVAL, SMG_EDEVICE. */
int smg_set_mass(smg_handle h, double mass, void* stream);

/* New handle for the same gauge field at another mass, reusing the prolongators of
 * h (Results section: vectors from the setup at the lightest mass serve every
 * heavier mass).  The new handle owns copies of P and of the calibration starts;
 * its coarse operators and smoothers are rebuilt for `mass`.  h is unchanged and
 * may be destroyed independently.  Errors: SMG_EINVAL, SMG_ENOMEM, SMG_EDEVICE. */
int smg_derive(smg_handle h, double mass, void* stream, smg_handle* out);

/* y = D x (dagger = 0) or y = D^H x (dagger = 1) on the fine lattice (Introduction).
 * x, y: device, complex128 [nrhs][lt][lx][2], must not overlap.  ASYNC.
 * Errors: SMG_EINVAL. */
int smg_apply_D(smg_handle h, const double* x, double* y, int32_t nrhs, int32_t dagger, void* stream);

/* y = A x = D^H D x on the fine lattice (the operator of the normal equations).
 * x, y: device, complex128 [nrhs][lt][lx][2], must not overlap.  ASYNC. */
int smg_apply_A(smg_handle h, const double* x, double* y, int32_t nrhs, void* stream);

/* y = A^(l) x on level l (0 = fine A; l >= 1 the Galerkin operator of Eq. 2).
 * x, y: device, complex128 level-l batches, must not overlap.  ASYNC. */
int smg_apply_level(smg_handle h, int32_t level, const double* x, double* y, int32_t nrhs,
                    void* stream);

/* FP64 operator of level `level` with the epilogues the V-cycle uses (Multigrid
 * section, steps 1-5; Results for the smoother), the modes of smg_level_op_f32
 * below.  Vectors are complex128 device arrays [nrhs][n_l] (xacc, aux may be
 * NULL where unused).  Coarse levels with nc <= 16 and nrhs >= mfma_min_rhs run
 * on the matrix cores (FP64 MFMA).  Errors: SMG_EINVAL.  ASYNC. */
int smg_level_op(smg_handle h, int32_t level, int32_t mode, double coef, const double* x, double* y, double* xacc,
                 const double* aux, int32_t nrhs, void* stream);

/* y = A^(l) x with the FP32 copy of the level-l operator that the mixed-precision
 * solves use (the same operator as smg_apply_level, links rounded to FP32).
 * x, y: device, complex64 (interleaved float) level-l batches.  ASYNC. */
int smg_apply_level_f32(smg_handle h, int32_t level, const float* x, float* y, int32_t nrhs, void* stream);

/* FP32 operator of level `level` with the epilogues the V-cycle uses (Multigrid
 * section, steps 1-5; Results for the smoother): mode 0: y = A_l x; mode 1 (one
 * frozen MR step): xacc += coef x and y = x - coef A_l x; mode 2 (residual):
 * y = aux - A_l x; mode 3 (the first MR step, from a zero iterate): xacc = coef x
 * and y = x - coef A_l x.  Vectors are complex64 device arrays [nrhs][n_l] (xacc,
 * aux may be NULL where unused).  Coarse levels with nc <= 16 and
 * nrhs >= mfma_min_rhs run on the matrix cores.  Errors: SMG_EINVAL. */
int smg_level_op_f32(smg_handle h, int32_t level, int32_t mode, double coef, const float* x, float* y, float* xacc,
                     const float* aux, int32_t nrhs, void* stream);

/* y = P^H x: restriction from level l to level l+1 (V-cycle step 2).  ASYNC. */
int smg_restrict(smg_handle h, int32_t level, const double* x, double* y, int32_t nrhs,
                 void* stream);

/* y = P x: prolongation from level l+1 to level l (V-cycle step 4).  ASYNC. */
int smg_prolong(smg_handle h, int32_t level, const double* x, double* y, int32_t nrhs,
                void* stream);

/* x = R b on level l < levels-1: the frozen minimal-residual polynomial smoother
 * (Results section; R = R^H).  ASYNC. */
int smg_smooth(smg_handle h, int32_t level, const double* b, double* x, int32_t nrhs,
               void* stream);

/* x = V b, one V-cycle from the finest level (Multigrid section, steps 1-5; Eq. 3
 * with the sign of its R A R^H term taken from those steps).  FP64.  ASYNC. */
int smg_vcycle(smg_handle h, const double* b, double* x, int32_t nrhs, void* stream);

/* x = V b as smg_vcycle, for callers that cannot allocate device memory during the
 * call: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The call allocates nothing (no hipMalloc, hipFree or allocator
 * callback): the per-level work vectors of the V-cycle live in one static device
 * array of 64 MiB per GPU (SMG_NOALLOC_SCRATCH_BYTES), taken when the library is
 * first used this way on that device and held until the process ends.  Every call
 * on a GPU shares that GPU's array, so calls that overlap on one GPU (any handle,
 * any stream) race: serialise them.  Nothing in the array needs to start at zero.
 * Needs levels >= 2 and SMG_COARSEST_DIRECT (the coarsest CG keeps Krylov vectors
 * of its own).  b, x: device, complex128 [nrhs][lt][lx][2], must not overlap.
 * ASYNC.  The result equals smg_vcycle's bit for bit.
 * Errors: SMG_EINVAL (bad arguments, CG coarsest, or nrhs columns whose work
 * vectors exceed the array: about 20 MB per column for a 256^2 lattice with Nv = 12). */
#define SMG_NOALLOC_SCRATCH_BYTES (64u << 20)
int smg_vcycle_noalloc(smg_handle h, const double* b, double* x, int32_t nrhs, void* stream);

/* The FP32 V-cycle of the mixed-precision solve (same steps; FP32 operators, the
 * fine smoother iterates stored as smoother_storage says): x = V b for complex64
 * device vectors [nrhs][n].  Errors: SMG_EINVAL. */
int smg_vcycle_f32(smg_handle h, const float* b, float* x, int32_t nrhs, void* stream);

/* Solve A x = rhs for nrhs independent right-hand sides with MG-CG (Results
 * section).  precision SMG_FP64: FP64 throughout.  SMG_MIXED: an FP32 MG-CG
 * (FP32 operators, smoother and coarse levels, with the storage that
 * smoother_storage and operator_storage select) inside FP64 defect correction:
 * the true residual and the solution update are FP64, and so are Gram-Schmidt
 * and the factorisation of the coarsest operator (setup); the FP32 V-cycle
 * applies the coarsest inverse in FP64 when coarsest_fp64 = 1, else from an FP32
 * or FP16 copy, or runs the coarsest CG in FP32 (SMG_COARSEST_CG).
 * rhs, x: device complex128 [nrhs][lt][lx][2]; x is overwritten (start from 0).
 * stats: host array of nrhs entries or NULL.
 * Returns SMG_OK when every column reached tol, SMG_NOTCONV when some did not,
 * SMG_EBREAKDOWN on NaN/Inf or loss of positive definiteness. */
int smg_solve(smg_handle h, const double* rhs, double* x, int32_t nrhs, double tol,
              int32_t maxiter, int32_t precision, void* stream, smg_stats* stats);

/* Plain CG on the fine A (the paper's comparison solver).  Arguments as smg_solve. */
int smg_cg(smg_handle h, const double* rhs, double* x, int32_t nrhs, double tol, int32_t maxiter,
           void* stream, smg_stats* stats);

/* Shape of level l: extents and degrees of freedom per site. */
int smg_level_info(smg_handle h, int32_t level, int32_t* lx, int32_t* lt, int32_t* dof);

/* Copy out the prolongator of coarsening l (Adaptive Multigrid section).
 * smoothed = 0: the tentative block-orthonormal P_t, device complex128 [J][k][i]
 *   with J the coarse site, k < nc the vector (nc = the dof of level l+1 from
 *   smg_level_info) and i = (wy*bx + wx)*dof_l + d for
 *   the site (Jx*bx + wx, Jt*bt + wy) of the aggregate.
 * smoothed = 1: the prolongator the V-cycle uses, [J][k][i] over the window of
 *   (bx + 2h) x (bt + 2h) sites, i = (wy*(bx+2h) + wx)*dof_l + d for the site
 *   (Jx*bx + wx - h, Jt*bt + wy - h) (periodic), h from smg_transfer_info.
 * Synchronous. */
int smg_get_prolongator(smg_handle h, int32_t level, int32_t smoothed, double* out, void* stream);

/* Halo h (0 or 1) of the V-cycle prolongator of coarsening l and its smoothed-
 * aggregation weight w (0 when P = P_t). */
int smg_transfer_info(smg_handle h, int32_t level, int32_t* halo, double* sa_weight);

/* Copy out the Galerkin operator of level l >= 1 as 9 link blocks per coarse site:
 * device complex128 [K][9][nc][nc], block index (dt+1)*3 + (dx+1) for the
 * neighbour K + (dx, dt), row = output component: (A v)_K = sum_D L[K][D] v_{K+D}.
 * Synchronous. */
int smg_get_coarse_links(smg_handle h, int32_t level, double* out, void* stream);

/* The two-level convergence factors that the adaptive stop (nv_stop_rho) measured on
 * coarsening `level`, one per vector count from 1: up to cap of them into out (host),
 * their number into *count (0 when the stop was off or the handle was not made by
 * smg_setup). */
int smg_get_setup_factors(smg_handle h, int32_t level, double* out, int32_t cap, int32_t* count);

/* Host copy of the nu smoother coefficients c_k of level l. */
int smg_get_smoother_coefs(smg_handle h, int32_t level, double* out);

/* ------------------------------------------------------------------------------
 * Continuous batching (serving).  A batch is a set of max_rhs column slots that run
 * MG-CG on the operator of handle h (Results section: the V-cycle preconditions
 * CG; the setup is amortised over many right-hand sides).  Right-hand sides are
 * admitted into free slots at any time, all running slots advance together, and
 * finished slots are harvested and reused.  Each slot keeps its own Krylov
 * scalars and is frozen on the device when it converges, so its result is bitwise
 * the same alone and in any mix.  precision SMG_FP64: FP64 MG-CG; SMG_MIXED: FP64
 * flexible CG preconditioned by the FP32 V-cycle.  A batch owns the column work
 * vectors of its slots (all levels) and lends them to h for the duration of each
 * smg_batch_step, so that destroying the batch returns them; h must not run other
 * calls while a step of one of its batches runs.
 * ------------------------------------------------------------------------------ */

/* New batch of max_rhs (1..256) slots with relative tolerance tol (true residual)
 * and per-slot iteration cap maxiter.  Every device array of the batch is carved
 * from one allocation (each array rounded to 256 bytes), so creating and
 * destroying a batch costs one call of the installed allocator each way.
 * Errors: SMG_EINVAL, SMG_ENOMEM. */
int smg_batch_create(smg_handle h, int32_t max_rhs, double tol, int32_t maxiter, int32_t precision, void* stream,
                     smg_batch* out);

/* Copy rhs (device, complex128 [lt][lx][2]) into a free slot, start its MG-CG and
 * return the slot.  Synchronous.  Errors: SMG_EBUSY (no free slot), SMG_EBREAKDOWN
 * (NaN/Inf in rhs). */
int smg_batch_admit(smg_batch b, const double* rhs, int32_t* slot, void* stream);

/* Advance every running slot by `iters` MG-CG iterations (slots that converge,
 * break down or reach maxiter stop).  Synchronous. */
int smg_batch_step(smg_batch b, int32_t iters, void* stream);

/* Per slot (host arrays of max_rhs entries, either may be NULL): done[j] = 1 when
 * slot j holds a finished right-hand side; stats[j] its status, iterations and
 * true relative residual. */
int smg_batch_poll(smg_batch b, uint8_t* done, smg_stats* stats);

/* Number of occupied and of still-running slots. */
int smg_batch_active(smg_batch b, int32_t* used, int32_t* running);

/* Copy the solution of finished slot `slot` to x (device complex128, or NULL to
 * drop it) and free the slot.  Synchronous.  Errors: SMG_EINVAL. */
int smg_batch_harvest(smg_batch b, int32_t slot, double* x, void* stream);

/* Free a slot whether or not it has finished (the other slots are unaffected). */
int smg_batch_cancel(smg_batch b, int32_t slot, void* stream);

/* Replay each iteration's device work as a captured HIP graph (enable = 1) or
 * launch it kernel by kernel (0, the default).  One graph is captured per number
 * of leading occupied slots and kept until the handle's operators change; results
 * are bitwise identical either way.  Errors: SMG_EINVAL (graphs with a CG coarsest
 * solve, which synchronises with the host). */
int smg_batch_use_graphs(smg_batch b, int32_t enable);

/* Grouped solves (Results section: many solves amortise one setup; here many
 * systems also share each launch).  A group binds nsys handles whose hierarchies
 * have one shape: the same lattice, levels, blocks, vectors per level (after an
 * adaptive stop, the counts that were kept), smoother steps (>= 2) and storage,
 * smoother_storage F32, a dense coarsest inverse of at most 4096 variables and
 * 4 <= nc <= 16 on the intermediate levels.  Masses, fields and setups may differ.
 * smg_group_solve solves A_j x_j = rhs_j for every system j with the SMG_MIXED solve,
 * system j in column j of every launch, so one launch per step serves all of them;
 * column j's arithmetic is that of smg_solve on handle j with one right-hand side,
 * so x_j equals that solve's result bit for bit.
 * rhs, x: device complex128 [nsys][lt][lx][2]; stats: host array of nsys or NULL.
 * The group runs on the first handle's context (its work vectors for nsys columns,
 * kept like a solve's) and reads every handle's operators in place: while the group
 * is used, no other call may use the first handle, and a re-mass of any handle is
 * picked up by the next group solve.  The group holds only its small tables of
 * per-system pointers, scales and smoother coefficients; destroy it before its handles.
 * Errors: SMG_EINVAL (shapes or options not supported, null arguments); the codes of
 * smg_solve.  Returns SMG_NOTCONV when some system did not reach tol. */
int smg_group_create(const smg_handle* hs, int32_t nsys, void* stream, smg_group* out);
int smg_group_solve(smg_group g, const double* rhs, double* x, double tol, int32_t maxiter, void* stream,
                    smg_stats* stats);
void smg_group_destroy(smg_group g);

/* The FP32 operator of level `level` (the one smg_level_op_f32 applies) of every
 * system of the group, system j's on column j, in one launch per step as inside
 * smg_group_solve (Eq. 2 on coarse levels, A = D^H D on the fine level): mode 0:
 * y_j = A_j x_j; mode 2 (residual): y_j = aux_j - A_j x_j.  x, y, aux: device
 * complex64 [nsys][n_l] (aux may be NULL for mode 0); column j equals
 * smg_level_op_f32 on handle j with one right-hand side bit for bit.  The same
 * rule on the first handle as for smg_group_solve.  Errors: SMG_EINVAL.  ASYNC. */
int smg_group_level_op_f32(smg_group g, int32_t level, int32_t mode, const float* x, float* y, const float* aux,
                           void* stream);

/* Device bytes held by the batch (in addition to its handle). */
int smg_batch_memory_bytes(smg_batch b, size_t* bytes);

/* Synchronises every stream that a call of the batch used (not the whole device),
 * then returns the batch's memory. */
void smg_batch_destroy(smg_batch b);

/* Device bytes held by the handle. */
int smg_memory_bytes(smg_handle h, size_t* bytes);

/* Device memory of the library.  A setup stays resident and is reused for many
 * right-hand sides and masses (Results section), so a caller that keeps many of
 * them accounts for their memory itself: every device array that a handle or a
 * batch owns comes from alloc(bytes, stream, ctx) and goes back through
 * release(ptr, bytes, stream, ctx), with `stream` the hipStream_t of the call that
 * allocated it.  alloc returns device memory of the current device aligned to at
 * least 256 bytes, or NULL (the call then fails with SMG_ENOMEM).  A handle or
 * batch keeps the allocator that was installed when it was created.  Before it
 * hands memory to release the library synchronises the device (a batch: the
 * streams its calls used), so no kernel still uses it.  Both NULL (the default)
 * restore hipMalloc / hipFree.  Pinned host memory (the convergence mirrors, and
 * a batch's read-back scratch, kept in a process-wide cache for reuse) and
 * rocBLAS's own workspace (blocked inversion of coarsest operators above 512
 * variables) are not routed.
 * Errors: SMG_EINVAL when only one of alloc and release is given. */
typedef void* (*smg_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*smg_release_fn)(void* ptr, size_t bytes, void* stream, void* ctx);
int smg_set_allocator(smg_alloc_fn alloc, smg_release_fn release, void* ctx);

/* Progress of long calls.  A setup of a large lattice runs for minutes inside one
 * call (the adaptive setup builds each level one near-null vector at a time,
 * Adaptive Multigrid section), so the library reports its steps as they finish:
 *   "calibrate"   level `level`'s smoother is calibrated (step 0, total = nv[level]);
 *   "candidate"   level `level` holds `step` of at most `total` near-null vectors
 *                 (value: the two-level factor that decided to go on when
 *                 nv_stop_rho > 0, else 0);
 *   "coarsest"    the setup is complete (level = levels - 1);
 *   "iteration"   an outer MG-CG (smg_solve, smg_cg; in SMG_MIXED the FP32 inner
 *                 solve) checked convergence after `step` of at most `total`
 *                 iterations (value: the largest recursive relative residual of the
 *                 columns still running);
 *   "refinement"  a SMG_MIXED solve finished defect-correction pass `step` (value:
 *                 the largest true relative residual after it);
 *   "coarsest-cg" a CG solve of the coarsest level (SMG_COARSEST_CG, or a setup
 *                 cycle's coarse system) took `step` iterations (most over the
 *                 columns; value: the largest relative residual reached).
 * The callback runs on the thread that made the call, between device
 * synchronisations, with no library lock held; calls on several threads may
 * report at the same time.  It must not call the library.  fn = NULL (the
 * default) turns reporting off.  Never fails. */
typedef void (*smg_progress_fn)(const char* stage, int32_t level, int32_t step, int32_t total, double value,
                                void* ctx);
int smg_set_progress(smg_progress_fn fn, void* ctx);

/* Device bytes the library will hold for a hierarchy with these parameters,
 * computed on the host from the allocation plan that the calls themselves follow
 * (no device call; every array counted rounded up to 256 bytes, as allocated):
 *   setup_bytes  smg_memory_bytes of a handle right after smg_setup or
 *                smg_setup_from_vectors (smg_derive: the same, less the mass
 *                coefficients that remass_affine keeps, 3 x 144 nc^2 bytes per
 *                coarse site of every coarse level);
 *   solve_bytes  what such a handle adds the first time it runs smg_solve with
 *                nrhs columns in `precision` (later solves of at most nrhs columns
 *                in that precision add nothing; smg_cg adds at most the SMG_FP64
 *                figure);
 *   batch_bytes  what smg_batch_create(h, max_rhs = nrhs, precision) adds on such
 *                a handle: the batch's own memory plus the handle's growth.
 * Any output may be NULL.  Errors: the parameter checks of smg_setup; SMG_EINVAL
 * for nrhs outside [1, 4096], or above 256 when batch_bytes is asked for. */
int smg_query_bytes(const smg_params* params, int32_t nrhs, int32_t precision, size_t* setup_bytes,
                    size_t* solve_bytes, size_t* batch_bytes);

void smg_destroy(smg_handle h);
const char* smg_strerror(int code);
const char* smg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SMG_H */
