// Internal descriptors shared by the host orchestration and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mor_host.h"

namespace mor {

constexpr int kWave = 64;
constexpr int kBlock = 256;   // threads per workgroup for every streaming kernel
constexpr int kNB = 64;       // dense tile size (Cholesky, TRSM, GEMM)

// ---------------------------------------------------------------------------------
// Element assembly.  One work item = one local tet of one subdomain (or of omega_0).
struct AsmSub {
  const int* ltet;    // 4 local node ids per local tet (-1 = Dirichlet / not in the index set)
  const int* tetg;    // global tet id per local tet
  const uint8_t* core;// 1 if the local tet lies in omega_i (nullptr: none)
  int t_begin;        // first local tet of the colour being assembled
  int t_count;        // number of local tets of that colour
  const int* rp;      // CSR over the local nodes (A+, K+ pattern)
  const int* col;
  const int* rpV;     // CSR over V_i (K_i pattern), nullptr if not assembled
  const int* colV;
  double* A;          // kappa-weighted stiffness values (nullable)
  double* K;          // H1 values: unweighted stiffness + mass (nullable)
  double* Ki;         // H1 values on omega_i over V_i (nullable)
  double* f;          // load vector M f_h (nullable)
};

// ---------------------------------------------------------------------------------
// One block-CG system: A_II X = F with F = [-A_IB | f_I] (or K_II E = -K_IB).
// Row-major dense blocks with leading dimension ld (multiple of 4), rows = nI.
struct CgSys {
  const int* rp;       // CSR over [I, B] rows; I rows list II columns first
  const int* col;
  const int* ii_end;   // end of the II part of each I row
  const float* val32;  // FP32 copy of the values
  const double* val64; // FP64 values
  const double* f;     // load on [I, B] (dense RHS column nB) or nullptr
  int nI, nB, ncols, ld;
  void* X; void* R; void* P; void* Q;  // CG scalar type
  double* X64;         // FP64 solution shadow (refinement), or nullptr
  const int* bp;       // aggregates of rows (block-Jacobi blocks): [bp[b], bp[b+1]), size <= 8
  int nblk;
  const void* minv;    // inverse of each diagonal block, 8 entries per row, CG scalar type
  // per-column state (length ld each)
  double* pq;          // p'Ap accumulator
  double* rz;          // r'M^-1 r of the current iterate
  double* rznew;       // accumulator of the updated r'M^-1 r
  double* rz0;         // reference of the current (re)start
  double* rzF;         // reference of the first right-hand side (refinement target)
  double* alpha;
  double* beta;
  int* active;         // 1 while the column iterates
  int* nactive;        // active columns of this system after the last iteration
  // LDS-halo SpMM tiling (shared by the A and K systems of a subdomain)
  const int4* htile;   // first row, rows, first halo entry, halo size
  const int* halo;
  const int* hrowp;    // per I row (+1): start of its padded II entries
  const int* hpe;      // padded II entries: CSR entry id or -1
  const uint16_t* hpp; // padded II entries: position in the tile halo
  const uint16_t* hself;
  const double* Fd;    // dense FP64 right-hand sides (nI x ld) in place of -A_IB and f, or nullptr
  double tol2;         // inner stop of this system: r'M^-1 r <= tol2 * (its value at the (re)start)
  // two-level preconditioner (rc == nullptr: block Jacobi only).  Coarse block c = aggregates
  // [8c, 8c+8); M^-1 r = (block Jacobi) r + P A_c^-1 P^T r with P piecewise constant on the blocks
  double* rc;          // P^T r: nc x ld (FP64), summed by the update / start kernels, cleared after use
  double* ec;          // A_c^-1 P^T r: nc x ld (FP64)
  int nc;
  // box form of the interior (FP32 systems on a Kuhn lattice; s16 == nullptr: none): stencil
  // coefficients (16 per row), the grid-point -> row map and the box extents
  const float* s16;
  const int* smap;
  int bx, by, bz;
};

// ---------------------------------------------------------------------------------
// Dense per-subdomain work (M x M matrices padded to MP = roundup(M, 64)).
struct DenseSub {
  int M, MP, T;        // T = MP / 64 tiles per dimension
  double* S;           // S_B, then its Cholesky factor R (upper) in place
  double* G;           // G1 = X_C^T K_i X_C
  double* W;           // R^-T G1
  double* C;           // R^-T G1 R^-1
  double* Dinv;        // T inverses of the diagonal 64x64 blocks of R
  int* info;           // non-SPD pivot report (0 = fine)
};

// Split-precision Gram: C = A^T B with A, B (k x m, row-major, FP64) carried as BF16 pairs
// hi + lo, stored transposed (m_pad x kp, k contiguous, zero padded), so that
// A^T B ~ Ahi^T Bhi + Ahi^T Blo + Alo^T Bhi on the BF16 matrix cores with FP32 accumulation.
struct SplitDesc {      // FP64 k x m (row-major, ld) -> BF16 hi/lo transposed mp x kp
  const double* X; int ldx;
  int k, m;            // valid rows (contraction index) and columns
  int kp, mp;          // padded sizes (multiples of 64)
  uint16_t *hi, *lo;
};
struct BfGramDesc {     // symmetric C (m x m, FP64, ldc) = A^T B from split operands
  int m, kp;
  const uint16_t *Ahi, *Alo, *Bhi, *Blo;   // mp x kp each, mp a multiple of 128
  double* C; int ldc;
};

struct TrsmDesc {       // right-hand side and solution of one subdomain's triangular solve
  const double* B; int ldb; int tb;   // tb: read B transposed
  double* X; int ldx;
  int ncol_tiles;
};

struct GemmDesc {
  int m, n, k;
  const double* A; int lda; int ta;
  const double* B; int ldb; int tb;
  double* C; int ldc;
  double alpha, beta;
  int sym;             // compute tiles ti <= tj only, write both triangles (beta must be 0)
  const double* skip = nullptr;   // or: output columns j with skip[j] == 0 need not be computed
};

// ---------------------------------------------------------------------------------
// launchers (mor_kernels.hip)
void launch_fill(double* p, int64_t n, double v, hipStream_t s);
void launch_fill_f(float* p, int64_t n, float v, hipStream_t s);
void launch_fill_i(int* p, int64_t n, int v, hipStream_t s);
void launch_assemble(const AsmSub* d_subs, const int* d_prefix, int nsub, int total,
                     const double* xyz, const int* tets, const double* kappa, const double* fnodal,
                     hipStream_t s);
void launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s);

// v = elements per lane (tile width 64 v columns): 1, 2 or 4 for float, 1 or 2 for double
template <typename T>
void launch_cg_init(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s);
template <typename T>
void launch_cg_spmm(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s);
template <typename T>
void launch_cg_spmm_halo(const CgSys* sys, const int4* tiles, int ntiles, int cap, int cwb, hipStream_t s);
// box interiors (FP32): tiles (system, tx | ty << 16, first column of a 32-column slice, 0)
void launch_cg_spmm_box(const CgSys* sys, const int4* tiles, int ntiles, hipStream_t s);
void launch_box_coeffs(const int* spos, const double* val, int nI, float* s16, hipStream_t s);
template <typename T>
void launch_cg_residual64(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s);
template <typename T>
void launch_cg_shadow(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s);
// block tiles: (system, first aggregate, first column); bpt aggregates per tile
template <typename T>
void launch_cg_update(const CgSys* sys, const int4* tiles, int ntiles, int bpt, int v, hipStream_t s);
template <typename T>
void launch_cg_direction(const CgSys* sys, const int4* tiles, int ntiles, int bpt, int v, hipStream_t s);
template <typename T>
void launch_cg_pstart(const CgSys* sys, const int4* tiles, int ntiles, int bpt, int v, hipStream_t s);
template <typename T>
void launch_cg_prolong(const CgSys* sys, const int4* tiles, int ntiles, int bpt, int v, hipStream_t s);
void launch_cg_coarse_dot(const CgSys* sys, const int2* cb, int ncb, int at_start, hipStream_t s);
void launch_coarse_assemble(const int* rp, const int* col, const int* ii_end, const double* v64, const int* rcb, int nI,
                            double* Ac, int ldac, hipStream_t s);
template <typename T>
void launch_block_inv(const int* rp, const int* col, const double* v64, const int* bp, int nblk, void* minv,
                      hipStream_t s);
// column blocks: (system, first column) of 256 columns
void launch_cg_alpha(const CgSys* sys, const int2* cb, int ncb, hipStream_t s);
void launch_cg_beta(const CgSys* sys, const int2* cb, int ncb, hipStream_t s);
void launch_cg_zero(const CgSys* sys, const int2* cb, int ncb, hipStream_t s);
void launch_cg_start(const CgSys* sys, const int2* cb, int ncb, int first, double tol2_outer, hipStream_t s);

void launch_to_f64_block(const float* in, int ldi, double* out, int ldo, int rows, int cols, hipStream_t s);
// randomized variant: sketch right-hand sides [-A_IB T | f | 0], [KW ; 0], P = A_BI X, and the
// whitening V diag(th^-1/2) of a small eigendecomposition
void launch_rhs_sketch(const int* rp, const int* col, const int* ii_end, const double* A, const double* f, int nI,
                       const double* T, int l, double* F, int ld, hipStream_t s);
void launch_rhs_rows(const double* KW, int nV, int c, int nI, double* F, int ld, hipStream_t s);
void launch_bi_product(const int* rp, const int* col, const double* A, int nI, int nB, int MP, const double* X, int ldx,
                       int c, double* P, hipStream_t s);
void launch_whiten(const double* V, const double* th, int s, int r, double* out, hipStream_t st);
// tiles: (descriptor, 64-row block of m_pad, 64-column block of kp)
void launch_split_bf16(const SplitDesc* d, const int4* tiles, int ntiles, hipStream_t s);
// tiles: (descriptor, ti, tj) with ti <= tj, 128 x 128 output blocks
void launch_gram_bf16(const BfGramDesc* d, const int4* tiles, int ntiles, hipStream_t s);
void launch_spmm64_rows(const int* rp, const int* col, const double* val, int nrows, int col_limit,
                        const double* X, int ldx, int ncols, double* Y, int ldy, hipStream_t s);
// use_skip: honour GemmDesc::skip
void launch_gemm(const GemmDesc* d, const int4* tiles, int ntiles, hipStream_t s, int use_skip = 0);
// k_gemm's contract on the FP32 matrix cores (FP64 operands rounded to FP32, FP32 accumulation)
void launch_gemm32(const GemmDesc* d, const int4* tiles, int ntiles, hipStream_t s, int use_skip = 0);
void launch_schur(const int* rp, const int* col, const double* Kval, int nI, int nB, const double* E, int lde,
                  double* S, int lds, hipStream_t s);
void launch_pad_identity(double* S, int M, int MP, hipStream_t s);
void launch_symmetrize(double* S, int MP, hipStream_t s);

void launch_potrf_diag(const DenseSub* d, int nsub, int p, hipStream_t s);
void launch_chol_panel(const DenseSub* d, int nsub, int p, int tmax, hipStream_t s);
void launch_chol_syrk(const DenseSub* d, int nsub, int p, int tmax, hipStream_t s);
// solve R^T X = B for every 64-column tile of every subdomain
void launch_trsm_lt(const DenseSub* d, const TrsmDesc* td, int nsub, int max_col_tiles, hipStream_t s, int p0 = 0,
                    int p1 = 1 << 30);
void launch_scale_cols(const double* U, int ldu, const double* sigma, int k, int rows, double* B, hipStream_t s);
// solve R X = B for one column tile (<= 64 columns): B, X are MP x 64 (ld 64)
void launch_trsm_un(const DenseSub* d, int nsub, double* const* Bs, double* const* Xs, hipStream_t s, int p0 = 0,
                    int p1 = 1 << 30);
void launch_copy_rect(const double* src, int lds, int trans, double* dst, int ldd, int rows, int cols, hipStream_t s);

void launch_jacobi(double* const* H, double* const* Svec, double* const* theta, const int* s_of, int nsub,
                   int smax, hipStream_t s);
void launch_ritz(double* const* Z, double* const* U, double* const* Vn, double* const* theta,
                 double* const* resid, const int* rows, const int* s_of, int nsub, int maxrows, int smax,
                 hipStream_t s);
void launch_cholinv_small(double* const* G, double* const* Rinv, const int* s_of, int nsub, int smax,
                          int* info, hipStream_t s);
void launch_random_init(double* const* V, const int* rows, const int* M_of, const int* s_of, int nsub,
                        int maxrows, int smax, uint32_t seed, hipStream_t s);

void launch_copy_col(const double* src, int lds, double* dst, int ldd, int rows, hipStream_t s);
// Where a neighbour pair's block Q_i^T A_0 Q_j and its transpose go: entry (a, b) of the block
// at out[base_ij + a ld_i + b], entry (b, a) of the transpose at out[base_ji + b ld_j + a].
// The dense reduced matrix and the block-row slabs of the sparse one are both such layouts.
struct PairOut {
  int64_t base_ij, base_ji;
  int ld_i, ld_j;
};
void launch_pair_project(const int4* trip_range, const int* trip, const double* A0, double* const* Vi,
                         const int* ldv, const int* k1, const PairOut* outs, double* out, int npairs, hipStream_t s);
// symmetrised A_ii of a [A_ii | b_i] block (k1 x (k1+1), ld) to out[base + a ldo + b]
void launch_scatter_block(const double* B, int k1, int ld, double* out, int64_t base, int64_t ldo, hipStream_t s);

// Block-sparse reduced system for the conjugate-gradient solve: the rows of subdomain i form a
// dense slab of dim_i rows over the columns of i and its neighbours.  Row r of the reduced system
// starts at val[rs[r]], has rwc[r].x entries whose global columns are ccol[rwc[r].y + k], and
// its diagonal entry at val[rs[r] + rdiag[r]].
struct RpcgDev {
  const double* val;
  const int* ccol;
  const int64_t* rs;
  const int2* rwc;
  const int* rdiag;
  const double* b; int bstride;   // load b~ (entry r at b[r * bstride])
  double *x, *r, *z, *p, *q, *dinv;
  double* sc;    // pq[3], rz[3], rr[3], rr0, rz0 (block preconditioner): ring of three per-iteration slots
  int* state;    // [0] stop flag, [1] iterations done, [2] failure (1 p'Ap <= 0, 2 diagonal <= 0)
  // block preconditioner (block = 1): row r's row of its subdomain block's pseudo-inverse starts at
  // bmv[rbm[r]]; rbd[r] = (first reduced row, size) of that block.  block = 0: the diagonal.
  const double* bmv;
  const int64_t* rbm;
  const int2* rbd;
  int block;
};
void launch_rpcg_setup(const RpcgDev& d, int n, hipStream_t s);
void launch_rpcg_iteration(const RpcgDev& d, int n, int it, double tol2, hipStream_t s);
// pseudo-inverse of each symmetric block from its eigendecomposition (vectors S: s x s row-major,
// values th descending): out = sum over th_j > drops[b] * th_0 of u_j u_j^T / th_j (s x s row-major)
void launch_block_pinv(double* const* S, double* const* th, const int* s_of, int n, const double* drops,
                       double* const* out, hipStream_t s);
void launch_reconstruct(const double* V, int nP, int k1, const double* x, const int* nodes, double* u,
                        hipStream_t s);

}  // namespace mor
