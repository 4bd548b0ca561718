/*
 * hodbf.h -- C ABI of an MI355X (gfx950) library for the butterfly-accelerated
 * volume integral equation (VIE) solver of Sayed, Liu, Gomez and Yucel,
 * "A Butterfly-Accelerated Volume Integral Equation Solver for Broad Permittivity
 * and Large-Scale Electromagnetic Analysis" (IEEE TAP).
 *
 * Problem (Section II, eqs. (1)-(2), (4)-(5), scalar Helmholtz kernel, one unknown
 * per cubic voxel, collocation at voxel centres):
 *     Z(m,n) = delta_mn / eps_m - K(d_mn) kappa_n,   kappa = (eps - 1) / eps,
 *     K(d)   = (k h)^2 / (4 pi |d|) exp(-j k h |d|)   for integer voxel offsets d != 0,
 *     K(0)   = (1 + j k a) exp(-j k a) - 1,           a = h (3 / (4 pi))^(1/3),
 * i.e. k^2 times the Green's function exp(-jkR)/(4 pi R) integrated over the voxel
 * (one-point rule off the diagonal, the equal-volume sphere on it).  Z I = V is
 * solved as the right-preconditioned system of eq. (precon).
 *
 * Conventions shared by every call:
 *  - Return value: HODBF_OK (0) or a negative hodbf_status.  No C++ exception
 *    crosses this ABI.  hodbf_last_error() gives a message for the calling thread.
 *  - Vectors: complex numbers stored interleaved (re, im).  A block of nrhs vectors
 *    is column-major in the user's voxel order, element (i, q) at ptr[i + q*ld]
 *    (in complex elements), user index i = ix + nx*(iy + ny*iz), ld >= N.
 *    Vector arguments are DEVICE pointers owned by the caller.
 *  - stream: a hipStream_t (NULL = the null stream).  Calls are stream-ordered
 *    and return once the work is enqueued, except where stated.
 *  - Units: free-space wavelength 1 (k0 = 2 pi).  Lossy media have Im(eps) < 0
 *    (time factor exp(+j w t), matching the exp(-j k R) kernel).
 *  - An operator is immutable after hodbf_build: const calls on one operator may
 *    run concurrently on different streams; hodbf_free must not race with them.
 */
#ifndef HODBF_H
#define HODBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hodbf_op hodbf_op; /* opaque compressed operator (+ preconditioner) */

typedef enum {
  HODBF_OK = 0,
  HODBF_E_ARG = -1,     /* invalid argument: shape, pointer, tolerance, eps */
  HODBF_E_NOMEM = -2,   /* device allocation failed or the HBM budget is exceeded */
  HODBF_E_HIP = -3,     /* a HIP call failed */
  HODBF_E_NUMERIC = -4, /* NaN or Inf met in a residual or a factorization */
  HODBF_E_NOCONV = -5,  /* vie_solve hit max_iter; x holds the last iterate */
  HODBF_E_STATE = -6    /* the operator lacks what the call needs (no preconditioner) */
} hodbf_status;

typedef enum { HODBF_C64 = 0, HODBF_C128 = 1 } hodbf_dtype; /* complex FP32 / FP64 */

/*
 * Storage precision of the preconditioner's factors, a bit mask: every copy asked for
 * is kept (same structure, values rounded from one FP64 construction) and a solve
 * or apply can pick any of them.  Applies accumulate in FP32.
 *   FP32: complex FP32 factors, FP32 MFMA.
 *   BF16: complex BF16 factors and BF16-rounded inputs, BF16 MFMA.
 *   FP16: complex FP16 factors (each block scaled by its largest magnitude),
 *         converted to FP32 on load, FP32 MFMA.
 */
typedef enum {
  HODBF_P_NONE = 0, /* no preconditioner */
  HODBF_P_FP32 = 1,
  HODBF_P_BF16 = 2,
  HODBF_P_BOTH = 3, /* FP32 | BF16 */
  HODBF_P_FP16 = 4
} hodbf_prec;

/*
 * Build parameters.  The voxel grid, per-voxel permittivity and wavenumber state
 * the scattering problem (Section II); tol_con and tol_fact are the compression
 * and factorization tolerances chi_con and chi_fact of eq. (precon).
 */
typedef struct {
  int32_t nx, ny, nz;    /* voxel grid, N = nx*ny*nz >= 1 */
  double h;              /* voxel edge in wavelengths, > 0 */
  double k0;             /* wavenumber (2 pi for unit wavelength), > 0 */
  const double *eps_r;   /* HOST, 2N doubles (re, im), user order; copied; eps != 0 */
  double tol_con;        /* chi_con in (0, 1): ID truncation of the forward operator */
  double tol_fact;       /* chi_fact in (0, 1): ID truncation of the inverse factors */
  int32_t leaf_size;     /* leaf cluster size of T_H, 1..64 (64 recommended) */
  int32_t precond_prec;  /* hodbf_prec bit mask, 0..7 */
  int32_t precond_min_level; /* levels < this get no X_tau (0 = full Algorithm 1 form) */
  int32_t precond_dense_levels; /* d >= 0: Algorithm 1's recursion starts from the dense
                                   inverses of the diagonal blocks of the level L_H - d
                                   nodes (computed directly, FP64 on the host, stored like
                                   the other factors) instead of the leaves, so the d lowest
                                   levels are exact and applied in one launch; 0 = leaves
                                   of the tree; E_ARG if L_H - d < precond_min_level
                                   (clamped to L_H otherwise) */
  uint64_t seed;         /* row-sampling RNG seed */
  size_t hbm_budget;     /* bytes of device memory the operator may hold; 0 = unlimited */
  void *stream;          /* hipStream_t used for construction */
} hodbf_build_params;

/*
 * hodbf_build -- compress Z in HOD-BF form (Section III-A: cluster tree T_H, dense
 * leaf blocks D_tau, nested-ID butterflies for every off-diagonal sibling block) and,
 * if precond_prec != HODBF_P_NONE, its approximate inverse in the multiplicative
 * form of Algorithm 1 (Section III-B), built bottom-up on the device: D^{-1} B of each
 * level and the BF_SMW steps of Algorithm 2 each reconstructed as butterflies from
 * products with structured random vectors (BF_random_matvec), the blocks kept at
 * tol_fact, intermediate ones at 1e-2 tol_fact (the environment variable
 * HODBF_CHI_INNER, if set, overrides that tolerance).  Blocks until the operator is
 * ready.
 * *out receives a new operator owned by the caller (release with hodbf_free).
 * Errors: E_ARG (bad grid, h, k0, tolerance, leaf size, eps = 0 or non-finite),
 * E_NOMEM (allocation or hbm_budget), E_HIP, E_NUMERIC (singular diagonal block).
 */
hodbf_status hodbf_build(const hodbf_build_params *params, hodbf_op **out);

/*
 * hodbf_apply -- y = Z_con x for nrhs >= 0 vectors (Section III-A, the butterfly
 * product B^L W^L ... W^1 V^0 of eq. (butterfly_mat) for every off-diagonal block
 * plus the dense leaf blocks).  Arithmetic is complex FP32 with FP32 accumulation
 * whatever dtype is; dtype only sets the storage type of x and y.
 * x and y must not overlap.  nrhs == 0 is a no-op.
 */
hodbf_status hodbf_apply(const hodbf_op *op, int32_t nrhs, hodbf_dtype dtype,
                         const void *x, int64_t ldx, void *y, int64_t ldy, void *stream);

/*
 * hodbf_apply_noalloc -- the product of hodbf_apply (same arguments, same result bit for
 * bit) for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation.  It allocates nothing; its
 * temporaries (tree-order copies of x and y and the stage workspace, 2 * 8 N nrhs +
 * 8 nrhs * (stage rows) bytes, each part rounded up to 256) live in a static scratch
 * array of 64 MiB that every GPU the library runs on holds until the process ends.
 * E_ARG if these sizes need more than that (use fewer right-hand sides per call).
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller.
 */
hodbf_status hodbf_apply_noalloc(const hodbf_op *op, int32_t nrhs, hodbf_dtype dtype,
                                 const void *x, int64_t ldx, void *y, int64_t ldy, void *stream);

/*
 * hodbf_precond_apply -- y = P x with P ~ Z^{-1}: the dense inverses D_tau^{-1} of the
 * recursion's leaves (the tree's leaves, or the level L_H - d nodes with
 * precond_dense_levels = d) followed, level by level towards the root, by
 * z(tau) <- (I + X_tau) z(tau) (Algorithm 1 unrolled).  Uses the default arithmetic: the FP32 copy with split-BF16
 * products (see hodbf_apply_tree, which 6) if the FP32 copy is stored, else the FP16
 * copy, else the BF16 copy.  FP32 accumulation.  E_STATE if built without one.
 */
hodbf_status hodbf_precond_apply(const hodbf_op *op, int32_t nrhs, hodbf_dtype dtype,
                                 const void *x, int64_t ldx, void *y, int64_t ldy,
                                 void *stream);

/*
 * hodbf_apply_tree -- the same products on vectors already in the library's internal
 * layout: complex FP32, tree order (position t holds user index perm[t], see
 * hodbf_export selector 0), right-hand sides interleaved, element (t, q) at
 * ptr[t * nrhs + q].  which: 0 y = Z_con x; 1 y = P x with the default arithmetic;
 * 2 with the FP32 copy; 3 with the BF16 copy; 4 with the FP16 copy; 5 y = Z_con x and
 * 6 y = P x (FP32 copy), both with split-BF16 arithmetic: every FP32 factor and input
 * value is split into BF16 hi + lo parts and each product is hi hi + hi lo + lo hi on
 * BF16 MFMA with FP32 accumulation (relative error at most 2^-15 per product, about
 * 2^-18 typically, against 2^-24 for 0 and 2).  Only grouped-GEMM kernels run (no permutation), so callers that
 * keep data in tree order avoid two passes.
 * x and y must not overlap.  E_STATE if the requested factors are absent.
 */
hodbf_status hodbf_apply_tree(const hodbf_op *op, int32_t which, int32_t nrhs, const void *x,
                              void *y, void *stream);

typedef struct {
  double tol;           /* chi_sol: stop when ||b - Z x|| / ||b|| <= tol per column */
  int32_t restart;      /* GMRES restart length m, 1..200 (20 recommended) */
  int32_t max_iter;     /* cap on Arnoldi steps per column (the paper caps at 3000) */
  int32_t use_precond;  /* 0: none; 1: operator default; 8 + HODBF_P_FP32 / _BF16 / _FP16;
                           16 + HODBF_P_FP32: the FP32 copy with split-BF16 arithmetic
                           (see hodbf_apply_tree, which 6) */
  int32_t fp32_only;    /* 0 (default): once at most 16 columns are still iterating, their
                           products with Z (Arnoldi steps and true residuals) run in FP64
                           arithmetic over the FP32-stored factors; 1: every product in
                           FP32 as hodbf_apply */
} hodbf_solve_opts;

typedef struct {
  int32_t *iters;       /* HOST, nrhs: Arnoldi steps (products with Z) per column */
  int32_t *converged;   /* HOST, nrhs: 1 if the true residual met tol */
  double *relres;       /* HOST, nrhs: final true relative residual ||b - Z x|| / ||b|| */
} hodbf_solve_info;

/*
 * vie_solve -- solve Z x = b (eq. (4)) for nrhs columns with right-preconditioned
 * flexible GMRES(m), all Krylov arithmetic in complex FP64 on the device
 * (classical Gram-Schmidt applied twice, Givens rotations, true residual check),
 * products with Z and P as in hodbf_apply / hodbf_precond_apply.  b and x are
 * complex FP64 DEVICE arrays (user order, ld >= N); x is overwritten (x0 = 0).
 * Blocks until done (reads one small convergence flag per Arnoldi step).
 * info may be NULL.  E_NOCONV if any column missed tol within max_iter.
 */
hodbf_status vie_solve(const hodbf_op *op, int32_t nrhs, const void *b, int64_t ldb,
                       void *x, int64_t ldx, const hodbf_solve_opts *opts,
                       hodbf_solve_info *info, void *stream);

/*
 * hodbf_solve_workspace -- *bytes = the device memory one vie_solve with these
 * arguments allocates for its own use (Krylov basis, preconditioned basis, vectors,
 * apply workspace, reductions), for admission by memory budget.  The caller's b and x
 * are not included.  0 for nrhs = 0.  Same argument errors as vie_solve (E_ARG,
 * E_STATE for a preconditioner copy the operator lacks); touches no GPU.
 */
hodbf_status hodbf_solve_workspace(const hodbf_op *op, int32_t nrhs,
                                   const hodbf_solve_opts *opts, size_t *bytes);

/*
 * hodbf_plane_wave -- b(:, q) = exp(-j k0 dhat_q . (r - r_c)) at the voxel centres
 * r = h (i + 1/2), r_c the box centre (the plane-wave excitation of Section IV).
 * dirs: HOST, 3*nrhs doubles (unit vectors).  b: complex FP64 DEVICE, ld >= N.
 */
hodbf_status hodbf_plane_wave(const hodbf_op *op, int32_t nrhs, const double *dirs,
                              void *b, int64_t ldb, void *stream);

typedef struct {
  int64_t n;                 /* unknowns */
  int32_t levels;            /* L_H */
  int32_t leaves;            /* 2^L_H */
  int32_t max_rank;          /* largest butterfly rank of the forward operator */
  int32_t precond_max_rank;  /* largest butterfly rank of the X_tau factors */
  int64_t entries_fwd;       /* stored complex entries of Z_con (dense leaves + factors) */
  int64_t entries_pre;       /* stored complex entries of the preconditioner */
  int64_t bytes_fwd;         /* device bytes of the forward factors */
  int64_t bytes_pre;         /* device bytes of the preconditioner factors (all copies) */
  int64_t bytes_total;       /* device bytes held by the operator */
  int32_t fwd_stages;        /* grouped launches per forward apply */
  int32_t pre_stages;        /* grouped launches per preconditioner apply */
  double build_seconds;      /* wall time of the forward construction */
  double precond_seconds;    /* wall time of the preconditioner construction */
  int64_t id_count;          /* interpolative decompositions computed */
  int64_t io_rows_fwd;       /* vector rows one apply of Z_con moves: per grouped launch every
                                output row once and every distinct input row segment once
                                (blocks that read the same rows share them); one apply reads
                                and writes 8 * nrhs * io_rows_fwd vector bytes */
  int64_t io_rows_pre;       /* the same for the preconditioner */
  int64_t precond_reconstructions; /* butterfly sets rebuilt from random-vector products
                                      (Algorithm 1 line 7 and every BF_SMW step) */
  int64_t precond_sketch_cols;     /* columns of all those random-vector products */
} hodbf_stats_t;

hodbf_status hodbf_stats(const hodbf_op *op, hodbf_stats_t *st);

/*
 * hodbf_export -- copy operator internals to HOST memory for verification.
 * which: 0 perm (int32 N: tree position -> user index);
 *        1 forward block table, 2 forward factor values (complex FP32),
 *        3 preconditioner block table, 4 preconditioner values of the FP32 copy,
 *        5 of the BF16 copy, 6 of the FP16 copy (each as complex FP32, block
 *          scales applied).
 * Block tables are int64 rows of 12: kind (0 dense leaf, 1 V0, 2 W, 3 B),
 * hod level l, node i, child row ca, child col cb, butterfly level, a, b, rows m,
 * cols n, offset, lda: element (i, k) of the block is value [offset + k lda + i]
 * (complex elements; blocks that share an input are stored stacked, lda >= m).
 * Call with buf == NULL to get the size in *bytes; E_ARG if *bytes is too small.
 */
hodbf_status hodbf_export(const hodbf_op *op, int32_t which, void *buf, size_t *bytes);

void hodbf_free(hodbf_op *op);
const char *hodbf_last_error(void);

/*
 * hodbf_set_allocator -- route the library's device memory through the caller's
 * allocator (e.g. a framework's caching allocator, so one pool owns the bytes).
 * alloc(bytes, stream, ctx) returns device memory (NULL on failure, reported as
 * E_NOMEM); stream is the stream the memory is first used on, or NULL for operator
 * arenas used on any stream.  release(ptr, ctx) returns it; stream-ordered reuse is the
 * allocator's business (scratch is released after the call's last use was enqueued on
 * its stream).  Operator arenas remember the hook they were allocated with; per-call
 * workspace comes from the hook installed when the call starts and goes back to it,
 * also when the call fails; change the hook only while no call is running.
 * alloc == NULL restores hipMalloc / hipMallocAsync.  E_ARG if alloc is set and release
 * is not.  Process-wide, thread-safe.
 */
typedef void *(*hodbf_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*hodbf_free_fn)(void *ptr, void *ctx);
hodbf_status hodbf_set_allocator(hodbf_alloc_fn alloc, hodbf_free_fn release, void *ctx);

/*
 * hodbf_plan_probe -- run only the host part of the forward construction (cluster
 * tree, row sampling, interpolative decompositions) and export it, without touching
 * a GPU.  which: 0 perm (int32 N); 1 block table (as above, kind 3 rows give the
 * skeleton count in n and an offset into the skeleton list); 2 V0/W values
 * (complex FP64); 6 B-block skeleton columns (int32 tree positions).
 * For host-logic verification.  Same size protocol as hodbf_export.
 */
hodbf_status hodbf_plan_probe(const hodbf_build_params *params, int32_t which, void *buf,
                              size_t *bytes);

/*
 * hodbf_precond_probe -- run the preconditioner construction on the host only (complex
 * FP64 on the CPU, no GPU): the forward plan as hodbf_plan_probe, then Algorithm 1
 * (Section III-B) with the butterfly Sherman-Morrison-Woodbury recursion of Algorithm 2
 * and every new butterfly reconstructed from products with structured random vectors,
 * exactly the steps hodbf_build runs on the device.  For verification of that host
 * logic on small problems (N <= 65536, else E_ARG).  which: 0 perm (int32 N); 3 block
 * table (as hodbf_export 3: leaf inverses as kind 0 rows, then the X_tau butterflies);
 * 4 values (complex FP64); 7 counters (int64: reconstructions, Woodbury inversions,
 * sketch columns, interpolative decompositions, largest rank, operator products).
 * which + 16: the same exports, with every butterfly set packed into the device path's
 * grouped-GEMM programs (forward and transposed) and run by a host interpreter of them.
 * Same size protocol as hodbf_export; results are cached for the last parameter set.
 */
hodbf_status hodbf_precond_probe(const hodbf_build_params *params, int32_t which, void *buf,
                                 size_t *bytes);

#ifdef __cplusplus
}
#endif

#endif /* HODBF_H */
