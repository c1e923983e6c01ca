/*
 * msdd.h -- C ABI of the MI355X (gfx950) multilevel spectral domain
 * decomposition library.
 *
 * The library builds and applies the multilevel additive Schwarz
 * preconditioner with spectral (GenEO-type) coarse spaces of Bastian,
 * Scheichl, Seelinger and Strehlow, "Multilevel Spectral Domain
 * Decomposition", and runs preconditioned conjugate gradients with it:
 *
 *   - Sec. 2.1: the problem A x = b is SPD; the preconditioner is the additive
 *     subspace correction B = sum_i R_i^T A_i^{-1} R_i with A_i = R_i A R_i^T,
 *     over the splitting V_h = V_{h,0} + sum_{l=1..L} sum_i V_{h,l,i}.
 *   - Sec. 2.2: hierarchical decomposition. The finest level is an
 *     overlapping element partition T_{h,L,i}; coarser levels group the
 *     subdomains of the next finer level (index sets J_{l,i}); level 0 is one
 *     subdomain.
 *   - Sec. 2.3: local Neumann spaces, the partition of unity chi_{l,i}, the
 *     GEVP abar_{l,i}(w,v) = lambda b_{l,i}(w,v), the coarse space
 *     V_{h,l-1} = span{ e chi w : lambda < eta } and the Dirichlet subspaces.
 *   - Sec. 3.4: abar_{l,i} = sum over the subdomain's elements of a_tau;
 *     b_{l,i}(u,v) = abar_{l,i}(chi u, chi v).
 *   - Sec. 4.1/4.2: coarse levels work from patch matrices and a generating
 *     system whose pencil has a common kernel.
 *   - Sec. 5: CG, stopped when ||b - A x^m|| < rtol ||b - A x^0||.
 *
 * Conventions
 *   - Every function returns an int status: MSDD_OK (0) or a negative code.
 *   - Array arguments may be host or device pointers; the library detects
 *     which with hipPointerGetAttributes and copies what it keeps.  The
 *     caller keeps ownership of every array it passes.
 *   - Indices are 0-based.  Dof numbers refer to the free dofs (Dirichlet
 *     dofs are eliminated; an element-dof entry of -1 marks an eliminated dof).
 *   - A context is not thread-safe.  Several contexts may share a device.
 *     msdd_solve may be called any number of times after one msdd_setup.
 */
#ifndef MSDD_H_
#define MSDD_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MSDD_OK 0
#define MSDD_EINVAL (-1)   /* bad shape, index out of range, PoU not a partition of unity, NaN */
#define MSDD_ENOTSPD (-2)  /* a local or coarse matrix had a non-positive pivot */
#define MSDD_EEIG (-3)     /* the local eigensolver failed */
#define MSDD_ENOCONV (-4)  /* PCG reached maxit; x holds the last iterate */
#define MSDD_EDEVICE (-5)  /* HIP runtime error or missing GPU */
#define MSDD_ENOMEM (-6)   /* device allocation failed */
#define MSDD_ESTATE (-7)   /* call order violated (solve before setup, ...) */

/* precision modes */
#define MSDD_FP64 0   /* everything in double precision */
#define MSDD_MIXED 1  /* finest-level Dirichlet factorisations and their solves in the
                         preconditioner apply in single precision (on the diagonally
                         scaled matrices diag(A_i)^{-1/2} A_i diag(A_i)^{-1/2}); local
                         eigensolves, coarse levels, the coarsest factorisation, PCG
                         recurrences and inner products in double */

typedef struct msdd_ctx msdd_ctx; /* opaque; owns all device memory it allocates */

typedef struct {
  int precision;      /* MSDD_FP64 or MSDD_MIXED */
  double sigma;       /* spectral shift of the local pencil S = abar + sigma*b (> 0);
                         <= 0 selects 0.1*eta.  Eigenvalues do not depend on it. */
  double eps_reg_rel; /* coarse generating systems: eigenvectors of abar + b with an
                         eigenvalue below eps_reg_rel times the largest are treated as their
                         common kernel and removed (default 1e-12) */
  int nev_max;        /* 0 = threshold selection only; > 0 caps eigenvectors per subdomain */
  double eig_tol;     /* tolerance on the normwise backward error
                         ||b x - nu S x|| / (nu ||S|| ||x||) of the selected local
                         eigenpairs (default 1e-14).  The next pair, which only certifies
                         the count (lambda_{m+1} >= eta), is accepted at max(eig_tol, 1e-11),
                         or once its Krylov-Weinstein interval in the S inner product lies
                         entirely above eta */
  int eig_maxit;      /* iterations of the local eigensolver (default 200) */
  int block;          /* initial block size of the local eigensolver (default 16) */
  int device;         /* HIP device ordinal */
  void* stream;       /* hipStream_t to launch on; NULL = the legacy default stream */
  int verbose;        /* 1 = print phase timings to stderr */
  int geneo_rhs;      /* right-hand side of the finest-level GEVP (Sec. 3.4, eq. of the
                         three forms): 1 = b^1(u,v) = abar(chi u, chi v) (default);
                         2 = b^2 = the overlap elements' sum a-ring(chi u, chi v) (the
                         original GenEO choice; overlap elements are those that belong to
                         another subdomain too); 3 = b^3 = abar(u - chi u, v - chi v).
                         Coarse levels always use b^1 with their 0/1 masks. */
  int nev_fixed;      /* 0 = select lambda < eta on the finest level (default); > 0 = select
                         the nev_fixed smallest eigenvalues per finest-level subdomain (the
                         fixed-count form of the paper's runs); coarse levels use eta */
  double eig_tol_energy; /* tolerance on the energy residual ||S^{-1} b x - nu x||_S / nu
                         (x^T S x = 1) of the selected local eigenpairs, which bounds the
                         S-angle to the eigenvector by itself over the gap (default 1e-10;
                         0 = normwise test only).  Needed at high coefficient contrast,
                         where ||S|| is set by the high-coefficient rows and the normwise
                         test alone leaves vectors off by up to 1e-7 */
  int dirichlet_rule; /* Dirichlet subspace V_{h,L,i} of a finest subdomain among its Neumann
                         dofs: 0 = the dofs all of whose elements lie in the subdomain
                         (conforming elements; default); 1 = every Neumann dof (DG and
                         cell-centred finite volumes, Sec. 3.5: there the input's "elements"
                         are cells and faces, a basis function lives on one cell, and the
                         subdomain's element set holds only the faces interior to it, so a
                         face to a neighbour outside must not exclude the cell's dofs) */
  int eig_fp32;       /* finest-level eigensolver (Sec. 2.3 GEVP): 0 = shift-invert with the
                         FP64 factor of S = abar + sigma b (default); 1 = the factor of
                         diag(s) S diag(s), s = diag(S)^{-1/2}, in single precision, used as
                         the preconditioner of the block iteration
                         Y = X N + diag(s) M^{-1} diag(s) (B X - S X N) (N the current Ritz
                         values), with S Y formed in FP64 for the Rayleigh-Ritz step, so the
                         pairs, residuals and counts are those of the FP64 pencil; a
                         subdomain that does not certify its count within
                         min(eig_maxit, 64) iterations is solved again with the FP64
                         factor (built then); b = b^1 only (geneo_rhs = 1) */
} msdd_options;

typedef struct {
  int n_levels;           /* L + 1 */
  int64_t n[8];           /* n[l] = dimension of V_{h,l}, l = 0..L (n[L] = free dofs) */
  int32_t n_sub[8];       /* P_l, subdomains per level (n_sub[0] = 1) */
  int32_t m_max[8];       /* largest eigenvector count of a level-l subdomain */
  int32_t max_local[8];   /* largest local (Neumann / generating) space on level l */
  int32_t max_band;       /* largest half-bandwidth of a finest-level local matrix */
  int32_t eig_iters_max;  /* largest local eigensolver iteration count */
  int32_t eig_restarts;   /* subdomains re-run with a larger block */
  double eig_resid_max;   /* largest normwise backward error of a selected finest-level pair */
  double t_plan_ms;       /* host planning (index analysis) */
  double t_local_ms;      /* local matrix extraction + shifted Cholesky + Dirichlet Cholesky */
  double t_gevp_ms;       /* finest-level GEVPs (eigensolver) */
  double t_coarse_ms;     /* patch projections, coarse GEVPs, coarse factorisations */
  double t_setup_ms;      /* whole msdd_setup */
  double t_solve_ms;      /* last msdd_solve */
  int32_t pcg_iters;      /* last msdd_solve */
  double pcg_relres;      /* last msdd_solve: recurrence ||r_m|| / ||r_0|| */
  int64_t eig_iters_sum;  /* local eigensolver iterations summed over the finest-level
                             subdomains and all their passes */
  int32_t warm_started;   /* finest-level subdomains started from the network's block */
  int32_t warm_fallbacks; /* of those, re-solved from the random start (not converged) */
  int32_t eig_unconverged; /* finest-level subdomains whose eigensolver stopped without
                              certifying its count (the setup then fails with MSDD_EEIG) */
  int32_t eig_stagnated;  /* selected finest-level pairs accepted at the rounding floor:
                             Ritz value fixed to 1e-14 between iterations, residuals no
                             longer falling, backward error within 1e6 * eig_tol and energy
                             residual within 1e3 * eig_tol_energy, but one of them above its
                             tolerance */
  double eig_energy_resid_max; /* largest energy residual of a selected finest-level pair
                             (of its iterate one step before acceptance) */
  int32_t eig_fp64_fallbacks; /* eig_fp32 = 1: finest-level subdomains whose single-precision
                             factor iteration did not certify its count within
                             min(eig_maxit, 64) iterations and that were solved again
                             with the FP64 factor */
} msdd_stats_t;

/* Fill *opt with defaults. */
void msdd_default_options(msdd_options* opt);

/* Create a context on opt->device (opt may be NULL for defaults). */
int msdd_create(msdd_ctx** out, const msdd_options* opt);

/*
 * Build the multilevel preconditioner (Sec. 2.2, 2.3, 4.1, 4.2).
 *
 *  n, rowptr[n+1] (int64), col[nnz] (int32), val[nnz] (double):
 *      A on the free dofs, CSR, symmetric positive definite.
 *  n_elem, k, elem_dofs[n_elem*k] (int32, -1 = eliminated),
 *  elem_mat[n_elem*k*k] (double, row-major per element):
 *      the element matrices a_tau (Sec. 3.4); sum_tau a_tau must equal A.
 *  n_sub, sub_elem_ptr[n_sub+1] (int64), sub_elem[] (int32):
 *      the finest-level element sets T_{h,L,i} (overlap included).
 *  sub_dof_ptr[n_sub+1] (int64), sub_dof[] (int32), sub_pou[] (double):
 *      for each subdomain the free dofs of its elements (the Neumann space
 *      V-bar_{L,i}, any order, at most 2^24 per subdomain) and the partition-of-unity
 *      weight chi of each;
 *      chi must vanish off the subdomain's Dirichlet space (options.dirichlet_rule)
 *      and the weights must sum to 1 at every dof.
 *  n_levels (>= 2), parent[]: n_levels-2 concatenated maps; the first n_sub
 *      entries give each finest subdomain's level-(L-1) subdomain, the next
 *      P_{L-1} entries map level L-1 to level L-2, and so on (the sets
 *      J_{l,i} of Sec. 2.2, nonoverlapping).  NULL when n_levels == 2.
 *  eta: the threshold of the coarse space definition (lambda < eta, strict).
 *
 * Errors: MSDD_EINVAL (inputs), MSDD_ENOTSPD (last_error names the subdomain),
 * MSDD_EEIG, MSDD_EDEVICE, MSDD_ENOMEM.  A failed setup leaves the context
 * without a preconditioner.
 */
int msdd_setup(msdd_ctx* c, int64_t n, const int64_t* rowptr, const int32_t* col,
               const double* val, int32_t n_elem, int32_t k, const int32_t* elem_dofs,
               const double* elem_mat, int32_t n_sub, const int64_t* sub_elem_ptr,
               const int32_t* sub_elem, const int64_t* sub_dof_ptr, const int32_t* sub_dof,
               const double* sub_pou, int32_t n_levels, const int32_t* parent, double eta);

/*
 * Build the preconditioners of nprob independent problems in one setup (one set of
 * batched launches for all their subdomains and levels).  The arguments describe the
 * union of the problems exactly as for msdd_setup, with:
 *  prob_dof_ptr[nprob+1] (int64): problem t owns the dofs [prob_dof_ptr[t],
 *      prob_dof_ptr[t+1]); prob_dof_ptr[0] = 0, prob_dof_ptr[nprob] = n;
 *  A block diagonal over the problems; every subdomain (on every level) inside one
 *      problem; subdomains ordered by problem on every level (the parent maps number
 *      the coarse subdomains of problem 0 first, and so on);
 *  level 0 is one subdomain per problem (a dense block of A_0 per problem).
 * All problems share n_levels and eta.  Solve with msdd_solve_batch (one CG per
 * problem).  Errors as msdd_setup; MSDD_EINVAL names a violated batch rule.
 */
int msdd_setup_batch(msdd_ctx* c, int32_t nprob, const int64_t* prob_dof_ptr, int64_t n,
                     const int64_t* rowptr, const int32_t* col, const double* val,
                     int32_t n_elem, int32_t k, const int32_t* elem_dofs,
                     const double* elem_mat, int32_t n_sub, const int64_t* sub_elem_ptr,
                     const int32_t* sub_elem, const int64_t* sub_dof_ptr,
                     const int32_t* sub_dof, const double* sub_pou, int32_t n_levels,
                     const int32_t* parent, double eta);

/*
 * Solve A x = b by preconditioned CG (Sec. 5) from the initial guess in x.
 * b[n], x[n]: double, host or device.  Stops when the recurrence residual
 * satisfies ||r_m||_2 < rtol ||r_0||_2 or after maxit iterations.
 * iters, relres (may be NULL) receive the iteration count and ||r_m||/||r_0||.
 * Returns MSDD_ENOCONV if maxit was reached (x holds the last iterate).
 */
int msdd_solve(msdd_ctx* c, const double* b, double* x, double rtol, int32_t maxit,
               int32_t* iters, double* relres);

/*
 * PCG on every problem of a batch set up by msdd_setup_batch (Sec. 5), each problem
 * with its own CG scalars and stopping test.  b, x: the concatenated vectors (host
 * or device); iters[nprob], relres[nprob] (may be NULL) receive per-problem counts
 * and ||r_m|| / ||r_0||.  On a context set up by msdd_setup it equals msdd_solve.
 * Returns MSDD_ENOCONV if some problem reached maxit.
 */
int msdd_solve_batch(msdd_ctx* c, const double* b, double* x, double rtol, int32_t maxit,
                     int32_t* iters, double* relres);

/*
 * Residual history of the last msdd_solve: relres[k] = ||r_k||_2 / ||r_0||_2 for
 * k = 0..iters (recurrence residuals, Sec. 5).  Writes min(cap, iters+1) values
 * (relres may be NULL to query); *count receives iters+1 (0 before any solve).
 */
int msdd_solve_history(const msdd_ctx* c, double* relres, int32_t cap, int32_t* count);

/*
 * msdd_solve without allocating: for callers that cannot allocate device memory during
 * the call (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same computation, arguments, results and errors as msdd_solve, except:
 *  - b and x must be device pointers (MSDD_EINVAL otherwise);
 *  - the PCG work vectors (4 n doubles), chunk partial sums, per-problem CG scalars and
 *    the residual history ((maxit + 1) doubles per problem) live in a fixed device array of
 *    MSDD_NOALLOC_SCRATCH_BYTES per device (each device the library runs on holds it until
 *    the process ends); a call that needs more fails with MSDD_EINVAL (n up to about
 *    2 million dofs for one problem at maxit 1000);
 *  - the iterations are launched one by one on the context's stream (no graph is built).
 * It calls no hipMalloc or hipFree; the preconditioner's own buffers are the ones the
 * setup allocated.  Every call on a device shares that device's array: calls that overlap
 * in time on one device (from any context or thread) race and must not be made.
 */
#define MSDD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int msdd_solve_noalloc(msdd_ctx* c, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t* iters, double* relres);

/*
 * Hybrid form of the preconditioner (Sec. 2.1 subspace correction; the form the paper uses
 * with GMRES in Sec. 5): restricted additive Schwarz on the finest level (each local
 * solution weighted by the partition of unity chi before it is added), multiplicative over
 * the levels from the finest to the coarsest:
 *     z = sum_i R_i^T D_i A_i^{-1} R_i r;
 *     for l = L-1, ..., 0:  z += P_l (sum_i R_{l,i}^T A_{l,i}^{-1} R_{l,i}) P_l^T (r - A z)
 * (coarse levels: the owned blocks, which partition the level, so no weights; level 0: the
 * coarsest matrix).  Not symmetric: use it with GMRES.  Single-problem setups only
 * (MSDD_EINVAL after msdd_setup_batch).  r, z host or device, length n.
 */
int msdd_apply_hybrid(msdd_ctx* c, const double* r, double* z);

/*
 * Solve A x = b by restarted GMRES (restart >= 1 basis vectors per cycle) with the hybrid
 * form as right preconditioner, from the initial guess in x, to
 * ||b - A x^m|| < rtol ||b - A x^0|| (Sec. 5).  A cycle ends when GMRES's least-squares
 * residual meets the tolerance or after `restart` steps; b - A x^m is then recomputed and
 * the solve stops if it meets the tolerance.  After a cycle that met it only in the
 * least-squares sense, the next cycle refines from x^m, unless that cycle reduced the
 * recomputed residual by less than half (it is then at its FP64 rounding floor, about
 * u || |A| |x| + |b| ||, which exceeds 1e-8 ||b|| at coefficient contrast 1e6 on fine
 * meshes): the solve stops as converged.  maxit counts iterations over all cycles;
 * iters, relres (may be NULL) receive the count and the recomputed ||b - A x|| / ||r_0||;
 * msdd_solve_history returns the least-squares residuals.  MSDD_ENOCONV at maxit.
 * Single-problem setups only.
 */
int msdd_solve_gmres(msdd_ctx* c, const double* b, double* x, double rtol, int32_t restart,
                     int32_t maxit, int32_t* iters, double* relres);

/* z = B r: one application of the multilevel additive preconditioner. */
int msdd_apply(msdd_ctx* c, const double* r, double* z);

/* Setup statistics (sizes, iteration counts, timings). */
int msdd_stats(const msdd_ctx* c, msdd_stats_t* out);

/*
 * Introspection of the coarse spaces (for parity checks against a reference).
 * msdd_get_level_counts: m[i] = number of selected eigenvectors of level-l
 * subdomain i (l = 1..L), i = 0..P_l-1.
 * msdd_get_eigs: the selected eigenvalues lambda (ascending) of level-l
 * subdomain i plus up to n_extra more computed ones (lam must hold
 * m_i + n_extra doubles); *count receives how many were written.
 * msdd_get_basis: the coarse basis block chi w of level-l subdomain i.
 * On the finest level its rows are the subdomain's Neumann-space dofs in
 * ascending global order (rows = |V-bar_i|); on a coarse level its rows are
 * the owned coarse dofs (functions of the children, in ascending child
 * order); column-major, ld = rows.  *rows and *cols receive the shape;
 * pass basis == NULL to query it.
 */
int msdd_get_level_counts(const msdd_ctx* c, int32_t level, int32_t* m);
int msdd_get_eigs(const msdd_ctx* c, int32_t level, int32_t i, int32_t n_extra, double* lam,
                  int32_t* count);
int msdd_get_basis(const msdd_ctx* c, int32_t level, int32_t i, double* basis, int32_t* rows,
                   int32_t* cols);

/*
 * Kernel timing (HIP events recorded around each launch on the context's
 * stream).  msdd_profile(c, 1) resets the counters and enables them, 0 pauses them
 * (the counts are kept), 2 resumes without a reset.  While they are on, the PCG
 * iterations are launched one by one (not replayed as a graph).
 * msdd_profile_query returns, for kernel class id (0 <= id < MSDD_NPROF),
 * the summed duration in ms, the number of launches, and the algorithmic
 * bytes and flops of those launches (what the method must read, write and
 * compute; see each kernel's comment).  msdd_profile_name gives the class name
 * (NULL for an id out of range).
 */
#define MSDD_NPROF 19
int msdd_profile(msdd_ctx* c, int enable);
int msdd_profile_query(msdd_ctx* c, int id, double* total_ms, int64_t* launches,
                       double* alg_bytes, double* alg_flops);
const char* msdd_profile_name(int id);

/* Text of the last error of this context ("" if none). */
const char* msdd_last_error(const msdd_ctx* c);

/* Release all device memory owned by the context. */
void msdd_destroy(msdd_ctx* c);

/* Local eigensolver iterations of every finest-level subdomain in the last setup
 * (summed over its passes): iters[n_sub] (host or device). */
int msdd_get_eig_iters(const msdd_ctx* c, int32_t* iters);

/*
 * ---------------------------------------------------------------------------
 * Learned warm start of the local eigensolver.
 *
 * An extension of the method: the paper solves each local GEVP of Sec. 2.3
 * (abar w = lambda b w) from scratch.  A network msdd_net maps a subdomain's
 * coefficient features x (n_in values) to n_vec vectors on a fixed frame of n_pos
 * node positions, a three-layer perceptron with relu activations
 *     y = relu(relu(x W1 + b1) W2 + b2) W3 + b3,   y[v*n_pos + q] = vector v at q.
 * Attached with msdd_warm_start, it supplies the first n_vec columns of the start
 * block of the finest-level eigensolver; the eigensolver's backward-error test
 * judges the result exactly as for a random start, and a subdomain whose
 * warm-started iteration stops without converging is solved again from the random
 * start (cold-start fallback).  The eigenvalues and the coarse space therefore do
 * not depend on the network beyond the eigensolver tolerance.
 *
 * Training: the targets are the method's own converged eigenvectors
 * (msdd_warm_targets after a setup with collect > 0); the loss of a sample is the
 * share of its unit-norm target vectors t_1..t_m outside the span of the masked
 * output block Ys = diag(s) Y:
 *     loss = 1 - tr(C^T G^{-1} C) / m,  G = Ys^T Ys + 1e-6 I,  C = Ys^T T,
 * averaged over the batch; Adam (beta1 0.9, beta2 0.999, eps 1e-8) updates the
 * parameters.  Training runs in FP32; inference in BF16 on the matrix cores with
 * FP32 accumulation.
 * ---------------------------------------------------------------------------
 */
typedef struct msdd_net msdd_net; /* opaque; owns its device memory */

/* Create a network on `device`, launching on `stream` (hipStream_t; NULL = the legacy
 * default stream).  Weights are Glorot-uniform draws of a counter-based generator
 * seeded with `seed` (the splitmix64 finaliser of seed ^ index); biases are 0.
 * Limits: n_in, n_hidden, n_pos >= 1; 1 <= n_vec <= 16.  MSDD_EINVAL otherwise. */
int msdd_net_create(msdd_net** out, int32_t n_in, int32_t n_hidden, int32_t n_vec,
                    int32_t n_pos, uint64_t seed, int32_t device, void* stream);

/* Number of parameters: n_in*H + H + H*H + H + H*n_vec*n_pos + n_vec*n_pos (-1 for NULL). */
int64_t msdd_net_param_count(const msdd_net* net);

/* Flat FP32 parameter vector, in the order W1 (n_in x H, row-major), b1 (H),
 * W2 (H x H), b2 (H), W3 (H x n_vec*n_pos), b3 (n_vec*n_pos); host or device
 * pointer of msdd_net_param_count entries.  set also clears the Adam moments. */
int msdd_net_set_params(msdd_net* net, const float* p);
int msdd_net_get_params(const msdd_net* net, float* p);

/* Forward pass of `batch` samples: x (batch x n_in), y (batch x n_vec*n_pos), FP32
 * arrays on host or device.  mode 0: FP32 arithmetic (the training pass); mode 1:
 * inputs, weights and hidden activations rounded to BF16 (nearest even), products on
 * the matrix cores with FP32 accumulation, biases in FP32 (the pass the setup uses). */
int msdd_net_forward(msdd_net* net, int32_t batch, const float* x, float* y, int32_t mode);

/* Mean loss over the samples idx[0..batch) of a training set of n_samples samples:
 *   x_all  (n_samples x n_in)       features,
 *   tgt    (n_samples x m_cap x n_pos) target vectors (unit 2-norm on the mask),
 *   mask   (n_samples x n_pos)      1 on the sample's frame positions, 0 elsewhere,
 *   cnt    (n_samples)              targets used per sample (<= m_cap; 0 = none),
 * all host or device; 1 <= m_cap <= 16; every idx must lie in [0, n_samples).
 * loss (host, may be NULL) receives the mean loss and grad (host or device, may be
 * NULL) its gradient with respect to the flat parameter vector.  FP32. */
int msdd_net_grad(msdd_net* net, int32_t batch, const int32_t* idx, int32_t n_samples,
                  const float* x_all, const float* tgt, const float* mask, const int32_t* cnt,
                  int32_t m_cap, float* loss, float* grad);

/* One Adam step with learning rate lr > 0 on the same loss (loss may be NULL). */
int msdd_net_train_step(msdd_net* net, int32_t batch, const int32_t* idx, int32_t n_samples,
                        const float* x_all, const float* tgt, const float* mask,
                        const int32_t* cnt, int32_t m_cap, float lr, float* loss);

const char* msdd_net_last_error(const msdd_net* net);
void msdd_net_destroy(msdd_net* net);

/* Attach a warm start to the next msdd_setup / msdd_setup_batch of c (n_sub = 0
 * detaches).  n_sub must equal that setup's number of finest-level subdomains and
 * n_entries its sub_dof_ptr[n_sub].
 *   x (n_sub x n_in, host or device): features per subdomain (used when net != NULL);
 *   sub_pos[n_entries]: for each entry of that setup's sub_dof array, the frame position
 *     (0 <= pos < n_pos) of the dof, or -1 (no frame position: that row starts from
 *     the random block);
 *   net: the network (its n_in and n_pos must match; it must outlive the setup), or
 *     NULL: no warm start, the frame layout only serves collect;
 *   collect: m_cap > 0 keeps training targets, the first min(m_i + 1, m_cap) converged
 *     eigenvectors of every subdomain (m_i selected ones plus the next), for
 *     msdd_warm_targets; 1 <= m_cap <= 16.
 * The arrays are copied.  MSDD_EINVAL on size or range errors (also at setup time if
 * the setup's sizes differ). */
int msdd_warm_start(msdd_ctx* c, msdd_net* net, int32_t n_sub, int32_t n_in, const float* x,
                    int64_t n_entries, const int32_t* sub_pos, int32_t n_pos, int32_t collect);

/* Training targets of the last setup (it must have had collect = m_cap > 0):
 * tgt (n_sub x m_cap x n_pos), mask (n_sub x n_pos), cnt (n_sub); host or device. */
int msdd_warm_targets(const msdd_ctx* c, float* tgt, float* mask, int32_t* cnt);

/*
 * ---------------------------------------------------------------------------
 * Autotuner of launch shapes.
 *
 * msdd_autotune times the candidate launch shapes of the hot kernels on the data of
 * the context's last setup (its factors, block sizes and matrix; scratch vectors) and
 * keeps the fastest: solve-phase choices apply to the next msdd_solve / msdd_apply,
 * setup-phase choices to the next setup.  Results do not depend on the choices beyond
 * rounding (every candidate computes the same quantity).
 *   what: MSDD_TUNE_EIG (finest-level eigensolver: band-solve variant, row splits of
 *         the Gram and update kernels) | MSDD_TUNE_SOLVE (preconditioner apply: fine
 *         band-solve variant; CG: lanes per CSR row of the SpMV);
 *   reps: timed launches per candidate (1..100), after one untimed launch.
 * MSDD_ESTATE before a setup.  The measured times per launch are in msdd_tuning_t.
 * ---------------------------------------------------------------------------
 */
#define MSDD_TUNE_EIG 1
#define MSDD_TUNE_SOLVE 2

typedef struct {
  int32_t eig_solve;      /* 0 = by shape; 1 = rolling window, 8 columns per workgroup;
                             2 = rolling window, 16 columns; 3 = one wavefront per column;
                             4 = rolling window, 4 wavefronts of 4 columns; 5 = rolling
                             window, 8 wavefronts of 2 columns; 6 = as 5 plus 4 staging
                             wavefronts; 7 = as 4 plus 4 staging wavefronts; 8 = blocked
                             solve with per-block inverses of 64-row blocks on the
                             matrix cores (half-bandwidths up to 64); 9 = as 8 in four
                             launches, the block-diagonal products apart from the
                             block-to-block chain (by shape when available) */
  int32_t eig_splits;     /* row splits per subdomain of the Gram / update kernels:
                             0 = by size, else 1..16 */
  int32_t fine_solve;     /* 0 = by shape (1 for half-bandwidths below 64, else 2);
                             1 = rolling window; 2 = one wavefront per subdomain;
                             3 = two-sided: the rows before and after a separator of b rows
                             solved as two chains side by side, the separator through the
                             explicit inverse of its Schur complement.  Its factors are
                             built by a setup made with this choice set (every subdomain
                             must have a half-bandwidth below 64 and at least b + 65 rows,
                             and the workgroup's data must fit in LDS); otherwise the
                             by-shape choice runs */
  int32_t spmv_group;     /* lanes per CSR row: 0 = by average row length, else 4, 8, 16, 32 */
  float eig_solve_ms[10]; /* [v] for eig_solve = v (v = 1..9; 0 = not run or not
                             applicable): time per eigensolver iteration, from launches
                             with all subdomains active and with the longest-iterating
                             one alone, weighed by the last setup's iteration counts */
  float eig_splits_ms[5]; /* for 1, 2, 4, 8, 16 splits */
  float fine_solve_ms[4]; /* [v] for fine_solve = v (v = 1, 2, 3; 0 = not applicable) */
  float spmv_ms[4];       /* for 4, 8, 16, 32 lanes */
} msdd_tuning_t;

int msdd_autotune(msdd_ctx* c, int32_t what, int32_t reps);
int msdd_get_tuning(const msdd_ctx* c, msdd_tuning_t* t);
/* Set the choices (the *_ms fields are ignored); MSDD_EINVAL for values out of range. */
int msdd_set_tuning(msdd_ctx* c, const msdd_tuning_t* t);

#ifdef __cplusplus
}
#endif
#endif /* MSDD_H_ */
