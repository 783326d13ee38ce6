/*
 * mor.h -- C-ABI of the MI355X library for the localized model-order-reduction
 * finite element method (Gustafsson, Hannukainen, Kohonen: "Distributed finite
 * element solution using model order reduction").
 *
 * The calls follow the paper's problem statement (Section 6, first paragraph):
 * given a tetrahedral mesh, a decomposition into overlapping subdomains omega_i
 * with extensions omega_i^+, and a truncation rule (rank or tolerance), compute
 * the reduced solution of Problem 2.3.  The three steps of Section 6 map to
 *   mor_create         step 1 outputs consumed: submeshes and neighbour relations
 *   mor_local_basis*   step 2: optimal local bases, Q_i^T A_ii Q_i and Q_i^T f_i
 *   mor_project        step 3: memory-efficient Q^T A Q over neighbour pairs
 *   mor_solve          step 3: reduced solve and u~ = Q x
 *
 * Conventions for every entry point
 *   - Return 0 on success or a negative MOR_E* code; mor_last_error() then holds
 *     a message (per thread).  No C++ exception crosses this boundary: every
 *     entry point catches what it throws; a failed host allocation returns
 *     MOR_ENOMEM, anything else MOR_EDEVICE.  After such a failure inside the
 *     serving engine the context should only be destroyed.
 *   - Pointers documented "host" are caller-owned, read (or written) only during
 *     the call; the library copies what it keeps.  Device memory is owned by the
 *     context and released by mor_destroy.
 *   - Integer arrays are little-endian int32/int64 as typed; floating point is
 *     IEEE binary64 at the boundary.
 *   - One context is used by one host thread at a time; all device work runs in
 *     order on the stream given in mor_opts (0 = the null stream).
 */
#ifndef MOR_H
#define MOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOR_OK 0
#define MOR_EINVAL (-1)   /* bad argument, invalid mesh (det J <= 0), not a partition, bad rank/tol */
#define MOR_ENOMEM (-2)   /* device or host allocation failed, or a subdomain exceeds the HBM budget */
#define MOR_ENOTCONV (-3) /* block CG, its FP64 refinement or the eigensolver did not converge within
                             its limits */
#define MOR_ESTATE (-4)   /* call order: e.g. mor_project before every subdomain has a basis */
#define MOR_EDEVICE (-5)  /* HIP runtime error or a failed device-side check (non-SPD pivot) */

/* Arithmetic of the local reduction. */
#define MOR_FP64 0        /* FP64 block CG, FP64 everywhere (the plain comparator path) */
#define MOR_FP32_REFINE 1 /* FP32 block CG + FP64 residual refinement; FP64 Gram and eigen */
#define MOR_FP32 2        /* FP32 block CG; FP64 Gram and eigen on the FP32 solution */
#define MOR_BF16_SPLIT 3  /* FP32 block CG + FP64 residual refinement; Gram contraction X_C^T K_i X_C in
                             BF16 MFMA on hi/lo splits of both operands (hi^T hi + hi^T lo + lo^T hi),
                             FP32 accumulation; FP64 Cholesky, eigen and projections */

typedef struct mor_ctx mor_ctx;

/* Tetrahedral mesh (Section 2): P1 space on the tets, zero Dirichlet data at
 * nodes flagged in `dirichlet`.  xyz: n_nodes*3 (x,y,z per node), host.
 * tets: n_tets*4 node ids, host; every tet must have positive volume. */
typedef struct {
  int64_t n_nodes;
  int64_t n_tets;
  const double* xyz;
  const int32_t* tets;
  const uint8_t* dirichlet;
} mor_mesh;

/* Coefficient kappa per tet (the a(x) of Section 7.2, piecewise constant) and
 * nodal load values (the load vector is M * f_h, consistent mass times the P1
 * interpolant).  f_nodal == NULL means f = 1.  Host arrays. */
typedef struct {
  const double* kappa;   /* n_tets */
  const double* f_nodal; /* n_nodes or NULL */
} mor_coeff;

/* Overlapping decomposition (Section 3) as tet lists: subdomain i owns
 * ext_tets[ext_tet_ptr[i] .. ext_tet_ptr[i+1]) = the tets of omega_i^+, and
 * in_core[] flags the ones that also lie in omega_i.  Cores must overlap in
 * single element layers so that the interiors of the omega_i partition the
 * free nodes (checked: MOR_EINVAL otherwise), and omega_i must lie inside the
 * interior of omega_i^+ (extension r >= 1).  Host arrays. */
typedef struct {
  int32_t n_sub;
  const int64_t* ext_tet_ptr; /* n_sub + 1 */
  const int32_t* ext_tets;    /* ext_tet_ptr[n_sub] */
  const uint8_t* in_core;     /* ext_tet_ptr[n_sub] */
} mor_subdomains;

/* Device allocation callback: return a device pointer of at least `bytes`
 * (256-byte aligned) or NULL; `user` is alloc_user. */
typedef void* (*mor_alloc_fn)(size_t bytes, void* user);
typedef void (*mor_free_fn)(void* ptr, void* user);

typedef struct {
  int32_t precision;       /* MOR_FP64 | MOR_FP32_REFINE | MOR_FP32 | MOR_BF16_SPLIT */
  double cg_rtol;          /* inner FP32 CG stop: sqrt(r'M^-1 r / r0'M^-1 r0) <= cg_rtol per column
                              (0 = 1e-5).  With FP64 refinement a looser value (1e-4) needs fewer
                              iterations for the same refine_rtol target, at lower accuracy of the
                              singular values (up to 1.2e-7 relative instead of below 1e-7) */
  double refine_rtol;      /* FP32_REFINE: stop refinement when the FP64 residual reaches this */
  int32_t max_iter;        /* CG iteration cap per solve (MOR_ENOTCONV beyond it) */
  int32_t refine_steps;    /* FP32_REFINE, BF16_SPLIT: maximum number of FP64 residual corrections; a
                              system whose FP64 residual is still above refine_rtol after the last one
                              fails its request with MOR_ENOTCONV */
  int32_t oversample;      /* extra subspace vectors of the top-k eigensolve (0 = automatic) */
  double eig_rtol;         /* Ritz residual tolerance relative to the largest eigenvalue */
  int32_t eig_max_iter;    /* subspace iteration cap */
  int32_t cg_chunk;        /* CG iterations launched between two convergence polls */
  int32_t spmm_rows;       /* row tiles: rows per SpMM workgroup; halo tiles: largest halo (48, 64, 96, 128 or
                              176 rows of P staged in LDS) (0 = automatic) */
  int32_t spmm_vec;        /* halo tiles: 256-byte column slices per workgroup; row tiles: width in units of
                              64 columns, 1, 2 or 4 (0 = automatic) */
  int32_t spmm_kind;       /* 0 = automatic (LDS halo tiles, 128-byte slices), 1 = LDS halo tiles with 256-byte
                              column slices, 3 = LDS halo tiles with 128-byte slices, 2 = row tiles
                              (spmm_rows x spmm_vec) */
  int32_t stream_vec;      /* width of the streaming CG kernels' tiles in units of 64 columns (0 = 1) */
  int32_t stream_blocks;   /* row aggregates per streaming tile (0 = automatic) */
  int32_t use_graph;       /* capture each CG chunk in a HIP graph and replay it */
  int32_t dense_batch;     /* finished requests gathered before the dense stage runs while others
                              still iterate (0 = 16; 1 = lowest latency) */
  size_t hbm_budget_bytes; /* device bytes one batch of local reductions may use (0 = 75% of the
                              device memory free when the engine starts, as hipMemGetInfo reports
                              it: memory a caller's allocator keeps cached counts as used) */
  mor_alloc_fn dev_alloc;  /* NULL: hipMalloc */
  mor_free_fn dev_free;    /* NULL: hipFree */
  void* alloc_user;
  void* hip_stream;        /* hipStream_t all work is ordered on; NULL = null stream.  It must come from
                              the HIP runtime this library is linked against (a handle made by another
                              runtime instance in the same process, such as one bundled with a Python
                              framework, is not valid here); the library synchronizes this stream
                              before it returns results to the host or releases memory */
  int32_t host_only;       /* 1: derive the decomposition on the host only (no device memory);
                              only mor_get_sizes / mor_get_nodes / mor_get_pairs may follow */
  int32_t basis_update;    /* 1: the basis update of Section 6 step 2 after each local reduction:
                              eigendecomposition of the stitched block Q^T A_ii Q, eigenvalues below
                              update_drop * lambda_max removed, basis rescaled so the block is the
                              identity (the basis then has dim <= k_eff + 1 columns) */
  double update_drop;      /* relative eigenvalue drop of the basis update (basis_update = 1) only
                              (0 = 1e-10: only numerically dependent directions of the stitched block
                              go, in every precision mode; a larger drop can remove directions that
                              carry much of the solution's energy).  The block preconditioner of
                              reduced_solver 2 keeps every positive eigenvalue of each block */
  int32_t reduced_solver;  /* solver of the reduced system Q^T A Q x = Q^T b:
                              0 = dense FP64 Cholesky (mor_project stores the n x n matrix);
                              1 = FP64 conjugate gradients with the diagonal preconditioner, the
                                  paper's choice (end of Section 6 step 3, Section 7), on the
                                  block-sparse matrix (one dense row slab per subdomain over itself
                                  and its neighbours; no n x n storage);
                              2 = the same with each subdomain block's inverse as preconditioner
                                  (block Jacobi; blocks of at most 64 columns).  In exact arithmetic
                                  this is the paper's diagonal-preconditioned CG after its basis
                                  update (which makes the blocks the identity).  Where stitched
                                  columns are nearly dependent, use basis_update = 1, which drops
                                  those directions from the system, with reduced_solver 1 */
  double reduced_rtol;     /* reduced_solver 1, 2: stop when ||b~ - A~ x|| <= reduced_rtol ||b~|| for the
                              recurrence residual (1), or r'M^-1 r <= reduced_rtol^2 b~'M^-1 b~ (2)
                              (0 = 1e-12) */
  int32_t reduced_max_iter;/* reduced_solver 1, 2: iteration cap (0 = 20000); MOR_ENOTCONV beyond it */
  int32_t coarse;          /* 1 (default): two-level preconditioner for the block CG, the block Jacobi
                              plus an additive coarse correction, piecewise constant on runs of 8 row
                              aggregates, with the coarse matrix P^T A_II P inverted in FP64 (on the
                              48^3 workload 25-30% fewer iterations for a small dense product per
                              iteration); 0: block Jacobi only */
  int32_t box_spmm;        /* 0 (default): FP32 systems whose interior rows fill a box of a Kuhn lattice
                              (detected from the mesh: grid points, Kuhn edge offsets) use the
                              plane-streaming SpMM (timer "spmm_box"); -1: the general SpMM for every
                              system (also with spmm_kind 2) */
} mor_opts;

/* Fill `opts` with defaults (FP32_REFINE, cg_rtol 1e-5, refine_rtol 1e-8, ...). */
void mor_default_opts(mor_opts* opts);

/* Validate the inputs, derive the index sets I, B, V_i, P_i (Sections 3-4),
 * the neighbour pairs and omega_0 (Section 6, step 3), colour the elements, and
 * upload geometry and patterns.  *out receives the context. */
int mor_create(const mor_mesh* mesh, const mor_coeff* coeff, const mor_subdomains* sub,
               const mor_opts* opts, mor_ctx** out);

/* Local reduction of subdomain `sd` (Section 6, step 2; Sections 3-4): assemble
 * A_i^+ and the H1 matrices, lift the load and every interface hat function
 * (block CG on A_II), form the trace-norm weight (Schur complement of the H1
 * matrix, Lemmas 4.1-4.2) and the H1(omega_i) Gram matrix of the liftings, keep
 * the leading weighted singular modes (eq. 4.4-4.5), stitch (Definition 3.1),
 * and project A_ii and f_i.  rank > 0 keeps the top `rank` modes (widened over
 * a cluster of equal singular values); rank <= 0 keeps sigma > tol.  k_eff_out
 * (may be NULL) receives the number of lifting modes kept; sigma_out (may be
 * NULL, capacity sigma_cap) the leading computed singular values. */
int mor_local_basis(mor_ctx* ctx, int32_t sd, int32_t rank, double tol, int32_t* k_eff_out,
                    double* sigma_out, int32_t sigma_cap);

/* The same for `n` subdomains at once, batched on the device (all of them in one
 * set of launches, in waves bounded by hbm_budget_bytes).  sds: n ids, host.
 * ranks / tols: n values each, host (tols may be NULL).  k_eff_out: n, host, may
 * be NULL. */
int mor_local_basis_batch(mor_ctx* ctx, int32_t n, const int32_t* sds, const int32_t* ranks,
                          const double* tols, int32_t* k_eff_out);

/* The randomized local reduction of Section 6 ("Randomized numerical linear algebra"): the
 * sketch Qhat Rhat = R_i C_i A_II^-1 A_IB T, then the SVD of B = Qhat^T (weighted Z_i)
 * evaluated with two left solves.  The weight R_BB (S_B = R_BB^T R_BB, Lemma 4.1) is applied
 * through solves with the H1 matrix K^+ on all of omega_i^+, whose inverse has S_B^-1 as its
 * B block: the sketch is T = S_B^-1 S_i (the paper's R_BB^-1 S_i' for S_i' = R_BB^-T S_i), and
 * B B^T = W S_B^-1 W^T gives the singular values.  Every solve carries l or l + 1 right-hand
 * sides (two with A_II, two with K^+), and no M_i x M_i matrix is formed.
 * sds, ranks, tols: n values each, host (tols may be NULL), as in mor_local_basis_batch.
 * l: sketch columns, 1..64.  omega[i]: the random matrix S_i of subdomain sds[i], host, M_i x l
 * row-major with rows in the order of the subdomain's interface nodes B (ascending global id;
 * mor_get_nodes lists them after the interior nodes); read during the call only.
 * The orthonormalisation of the sketch drops directions whose K_i-Gram eigenvalue is below
 * 1e-10 of the largest; singular values are reported for the kept directions (at most l).
 * Needs FP64 solutions: precision MOR_FP64, MOR_FP32_REFINE or MOR_BF16_SPLIT (else
 * MOR_EINVAL).  k_eff_out: n, host, may be NULL. */
int mor_local_basis_sketched(mor_ctx* ctx, int32_t n, const int32_t* sds, const int32_t* ranks, const double* tols,
                             int32_t l, const double* const* omega, int32_t* k_eff_out);

/* Galerkin projection Q^T A Q of the global system (eq. 6.1) without forming A
 * or Q: diagonal blocks from the local step, off-diagonal blocks from A_0
 * assembled on omega_0 and the interface rows of neighbouring bases.  Needs
 * every subdomain reduced (MOR_ESTATE otherwise).  Stored dense (reduced_solver 0)
 * or as block-row slabs over the neighbour pairs (reduced_solver 1). */
int mor_project(mor_ctx* ctx);

/* Solve the reduced system (reduced_solver: FP64 Cholesky, or FP64 conjugate
 * gradients with the diagonal preconditioner from x = 0) and write
 * u~ = sum_i S_i Q_i x_i at every mesh node into u_out (n_nodes doubles, host;
 * zero at Dirichlet nodes).  n_reduced_out (may be NULL) receives dim of the
 * reduced space.  MOR_EDEVICE if the reduced matrix is not positive definite
 * (a Cholesky pivot, p'A~p or a diagonal entry <= 0); MOR_ENOTCONV if the
 * conjugate gradients reach reduced_max_iter first. */
int mor_solve(mor_ctx* ctx, double* u_out, int64_t* n_reduced_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): mor_solve's conjugate-gradient path (reduced_solver
 * 1 or 2) with every vector in a static device array of the library (32 MiB per device, held
 * until the process ends), so the call itself allocates nothing.  u_dev: device buffer of
 * n_nodes doubles, caller-owned, receives u~ (zero at Dirichlet nodes); n_reduced_out as in
 * mor_solve; the reduced solution is then also readable with mor_get_reduced_solution.
 * Errors: MOR_EINVAL for reduced_solver 0 or a NULL u_dev; MOR_ENOMEM when the reduced
 * dimension exceeds 699,008 unknowns (the array's capacity); MOR_ESTATE before mor_project;
 * MOR_EDEVICE if the array's address could not be found on the context's device; otherwise as
 * mor_solve.  All calls on one device share its array: calls that overlap on one device (from
 * two host threads, or on two streams) race and must be serialized by the caller. */
int mor_solve_noalloc(mor_ctx* ctx, double* u_dev, int64_t* n_reduced_out);

/* ---- serving: continuous batching of local-reduction requests ---------------
 * mor_submit queues a request for subdomain `sd` (rank/tol as in mor_local_basis,
 * precision one of MOR_FP64..MOR_BF16_SPLIT); it is admitted when device memory
 * within hbm_budget_bytes is free, joins the running block-CG launches at the
 * next chunk boundary, and completes independently of the others.  mor_poll
 * reports a request's state without driving the device: done = 1 when finished,
 * status = its result code.  mor_local_basis_batch uses the same engine. */
int mor_submit(mor_ctx* ctx, int32_t sd, int32_t rank, double tol, int32_t precision, uint64_t* ticket);
int mor_poll(mor_ctx* ctx, uint64_t ticket, int32_t* done, int32_t* status);
/* Drive the serving loop until every submitted request has finished. */
int mor_drain(mor_ctx* ctx);
/* Advance the serving loop by one tick (admission, one CG chunk, completions). */
int mor_step(mor_ctx* ctx);
/* Engine state: live (admitted) and pending requests, device bytes held by live requests,
 * the peak of that since creation, and the admission budget. */
int mor_engine_stats(mor_ctx* ctx, int32_t* live, int32_t* pending, int64_t* live_bytes, int64_t* peak_bytes,
                     int64_t* budget);

/* ---- results and diagnostics (host copies) ---------------------------------- */

/* Sizes of the index sets of subdomain sd: |P_i|, |V_i|, |I|, |B|. */
int mor_get_sizes(mor_ctx* ctx, int32_t sd, int32_t* nP, int32_t* nV, int32_t* nI, int32_t* nB);
/* Global node ids of the local ordering [P | V\P | I\V | B] (nI + nB ints). */
int mor_get_nodes(mor_ctx* ctx, int32_t sd, int32_t* out, int64_t cap);
/* Neighbour pairs (i < j) coupled through A_0 on omega_0: pairs_out receives 2 ints per pair
 * (up to cap pairs); n_pairs the total count.  Works in host_only mode. */
int mor_get_pairs(mor_ctx* ctx, int32_t* pairs_out, int64_t cap, int64_t* n_pairs);
/* Basis on V_i: (nV x dim) row-major doubles, dim = k_eff + 1: column 0 = q_0, then the
 * H1(omega_i)-orthonormal lifting modes; after the basis update (mor_opts.basis_update) the
 * dim columns of the updated basis instead.  The stitched basis is its first nP rows.
 * The last argument receives dim - 1. */
int mor_get_basis(mor_ctx* ctx, int32_t sd, double* out, int64_t cap, int32_t* k_eff);
/* The truncation of the last local reduction of sd (eq. 4.5): k_eff = lifting modes kept by the
 * rank or tolerance rule (widened over a cluster), dim = basis columns of the subdomain (k_eff + 1,
 * or fewer after the basis update of Section 6 step 2).  MOR_ESTATE before sd is reduced.  Either
 * pointer may be NULL. */
int mor_get_rank(mor_ctx* ctx, int32_t sd, int32_t* k_eff, int32_t* dim);
/* Leading singular values of the weighted lifting operator (up to cap). */
int mor_get_sigma(mor_ctx* ctx, int32_t sd, double* out, int32_t cap, int32_t* n);
/* Q_i^T A_ii Q_i (dim^2, row-major) and Q_i^T f_i (dim). */
int mor_get_local_block(mor_ctx* ctx, int32_t sd, double* Aii, double* bi, int64_t cap);
/* After mor_project: the dense reduced matrix (n x n, cap >= n*n; with reduced_solver 1
 * it is expanded from the block-row slabs on the host) and load (n). */
int mor_get_reduced(mor_ctx* ctx, double* At, double* bt, int64_t cap, int64_t* n);
/* After mor_solve: the reduced coefficient vector x (n). */
int mor_get_reduced_solution(mor_ctx* ctx, double* x, int64_t cap);
/* After mor_solve: the solver used (0 Cholesky, 1 and 2 conjugate gradients), its iterations
 * (0 for Cholesky) and the stopping quantity it reached: ||r|| / ||b~|| of the recurrence
 * residual (1), sqrt(r'M^-1 r / b~'M^-1 b~), the residual of the basis-updated system (2), or 0
 * (Cholesky).  Any pointer may be NULL. */
int mor_get_solve_info(mor_ctx* ctx, int32_t* solver, int32_t* iters, double* rel_residual);
/* Per-solve statistics of the last local reduction of sd: CG iterations of the
 * A- and H1-systems, FP64 refinement restarts (the larger of the two systems), subspace
 * iterations. */
int mor_get_stats(mor_ctx* ctx, int32_t sd, int32_t* cg_iter_a, int32_t* cg_iter_k, int32_t* refine,
                  int32_t* eig_iter);

/* Per-kernel device timing with HIP events on the library's stream.
 * name: "spmm" (the block-CG sparse product), "cg_update", "cg_direction",
 * "cg_coarse" (the coarse solve of the two-level preconditioner, flops), "coarse_setup",
 * "cg_graph" (a whole CG chunk in graph mode), "residual64",
 * "gram", "schur", "potrf", "trsm", "eig", "assemble", "project", "solve"
 * (the reduced solve; for conjugate gradients its work is 2 nnz(A~) flops per iteration).
 * Reports launches, total milliseconds and algorithmic bytes (spmm) or flops. */
int mor_timing_enable(mor_ctx* ctx, int32_t on);
int mor_timing_get(mor_ctx* ctx, const char* name, int64_t* launches, double* total_ms, double* work);
int mor_timing_reset(mor_ctx* ctx);

void mor_destroy(mor_ctx* ctx);
const char* mor_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MOR_H */
