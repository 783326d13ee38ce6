// HIP kernels for gfx950 (CDNA4, wave64) of the localized model-order-reduction hot path.
//
//   element-coloured P1 assembly into CSR ........ Section 2 (Problem 2.2), Section 4 (H1 Gram
//                                                  matrices of R_i and R_BB), Section 6 step 2
//   block CG for A_II X = [-A_IB, f_I] ........... Problems 3.2-3.3, the lifting Z_i of Section 4
//   FP64 residual refinement ...................... (numerical addition; same solution)
//   Gram / Schur / Cholesky / TRSM (FP64 MFMA) ... Lemmas 4.1-4.2 and eq. 4.3-4.5
//   Jacobi eigensolver + Ritz steps ............... top-k of the weighted lifting operator
//   neighbour-pair projection, reduced solve ...... Section 6 step 3 (eq. 6.1)
//
// Streaming kernels use 256-thread workgroups (4 waves) and an XCD-aware tile order: the
// hardware hands workgroup b to XCD b % 8, so logical tile (b % 8) * ceil(G/8) + b / 8 keeps
// consecutive row blocks of one column tile on one XCD and its L2.
#include "mor_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace mor {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ int xcd_tile(int b, int ntiles) {
  const int g8 = (ntiles + 7) >> 3;
  return (b & 7) * g8 + (b >> 3);
}

static inline int xcd_grid(int ntiles) { return ((ntiles + 7) >> 3) << 3; }

// --------------------------------------------------------------------------------- fills
__global__ void k_fill(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f(float* p, int64_t n, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i(int* p, int64_t n, int v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
static inline int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}
void launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}
void launch_fill_f(float* p, int64_t n, float v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_f, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}
void launch_fill_i(int* p, int64_t n, int v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
}

__global__ void k_to_f32(const double* in, float* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) out[i] = (float)in[i];
}
void launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
}

// --------------------------------------------------------------------------------- assembly
__device__ __forceinline__ int find_slot(const int* __restrict__ rp, const int* __restrict__ col, int r, int c) {
  int lo = rp[r], hi = rp[r + 1];
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (col[mid] < c) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// One thread per tet of one colour: tets of a colour share no node, so the scatter into the
// CSR values needs no atomics and is deterministic.
__global__ __launch_bounds__(256) void k_assemble(const AsmSub* __restrict__ subs, const int* __restrict__ prefix,
                                                  int nsub, int total, const double* __restrict__ xyz,
                                                  const int* __restrict__ tets, const double* __restrict__ kappa,
                                                  const double* __restrict__ fnodal) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= total) return;
  int lo = 0, hi = nsub;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (prefix[mid] <= gid) lo = mid; else hi = mid;
  }
  const AsmSub& S = subs[lo];
  const int t = S.t_begin + (gid - prefix[lo]);
  const int g = S.tetg[t];
  int nd[4], ln[4];
  double x[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    nd[a] = tets[4 * (int64_t)g + a];
    ln[a] = S.ltet[4 * (int64_t)t + a];
#pragma unroll
    for (int d = 0; d < 3; ++d) x[a][d] = xyz[3 * (int64_t)nd[a] + d];
  }
  double e1[3], e2[3], e3[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    e1[d] = x[1][d] - x[0][d];
    e2[d] = x[2][d] - x[0][d];
    e3[d] = x[3][d] - x[0][d];
  }
  // rows of J^{-1} (J = [e1 e2 e3]) are the scaled cross products: grad(lambda_1..3)
  double c23[3] = {e2[1] * e3[2] - e2[2] * e3[1], e2[2] * e3[0] - e2[0] * e3[2], e2[0] * e3[1] - e2[1] * e3[0]};
  double c31[3] = {e3[1] * e1[2] - e3[2] * e1[1], e3[2] * e1[0] - e3[0] * e1[2], e3[0] * e1[1] - e3[1] * e1[0]};
  double c12[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  const double det = e1[0] * c23[0] + e1[1] * c23[1] + e1[2] * c23[2];
  const double inv = 1.0 / det;
  double gr[4][3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    gr[1][d] = c23[d] * inv;
    gr[2][d] = c31[d] * inv;
    gr[3][d] = c12[d] * inv;
    gr[0][d] = -(gr[1][d] + gr[2][d] + gr[3][d]);
  }
  const double vol = fabs(det) * (1.0 / 6.0);
  const double kap = kappa[g];
  const bool in_core = S.core != nullptr && S.core[t] != 0;
  double fv[4] = {1.0, 1.0, 1.0, 1.0};
  if (fnodal != nullptr) {
#pragma unroll
    for (int a = 0; a < 4; ++a) fv[a] = fnodal[nd[a]];
  }
  const double fsum = fv[0] + fv[1] + fv[2] + fv[3];
  const double m20 = vol * (1.0 / 20.0);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int ra = ln[a];
    if (ra < 0) continue;
    if (S.f) S.f[ra] += m20 * (fv[a] + fsum);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int cb = ln[b];
      if (cb < 0) continue;
      const double gg = vol * (gr[a][0] * gr[b][0] + gr[a][1] * gr[b][1] + gr[a][2] * gr[b][2]);
      const double mass = m20 * (a == b ? 2.0 : 1.0);
      if (S.A || S.K) {
        const int slot = find_slot(S.rp, S.col, ra, cb);
        if (S.A) S.A[slot] += kap * gg;
        if (S.K) S.K[slot] += gg + mass;
      }
      if (in_core && S.Ki) {
        const int slot = find_slot(S.rpV, S.colV, ra, cb);
        S.Ki[slot] += gg + mass;
      }
    }
  }
}

void launch_assemble(const AsmSub* d_subs, const int* d_prefix, int nsub, int total, const double* xyz,
                     const int* tets, const double* kappa, const double* fnodal, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_assemble, dim3((total + 255) / 256), dim3(256), 0, s, d_subs, d_prefix, nsub, total, xyz,
                     tets, kappa, fnodal);
}

// --------------------------------------------------------------------------------- block CG
// A tile = (system, first row, first column).  A wave owns 64 * V consecutive columns (V
// elements per lane) and rows wave, wave + 4, ... of the tile's row block.  The SpMM tile width
// (64 V) and rows per tile are tuned so that the rows in flight on one XCD plus the stencil halo
// of the neighbour rows stay inside that XCD's L2; the streaming kernels use wide tiles.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <int B> struct Raw;
template <> struct Raw<4> { using t = uint32_t; };
template <> struct Raw<8> { using t = u32x2; };
template <> struct Raw<16> { using t = u32x4; };

// Pointers read from descriptors are generic; casting them to the global address space lets
// the compiler emit global_load/global_store instead of flat accesses.
#define MOR_GLOBAL __attribute__((address_space(1)))
template <typename T, int V>
__device__ __forceinline__ void ld_vec(const T* p, T (&v)[V]) {
  using R = typename Raw<V * sizeof(T)>::t;
  *reinterpret_cast<R*>(v) = *((const MOR_GLOBAL R*)(p));
}
template <typename T, int V>
__device__ __forceinline__ void st_vec(T* p, const T (&v)[V]) {
  using R = typename Raw<V * sizeof(T)>::t;
  *((MOR_GLOBAL R*)(p)) = *reinterpret_cast<const R*>(v);
}
template <typename T>
__device__ __forceinline__ T gld(const T* p) { return *((const MOR_GLOBAL T*)(p)); }

// Sum a per-lane partial over the 4 waves and add it to a per-column FP64 accumulator.
template <int V>
__device__ __forceinline__ void column_reduce_add(double (*red)[64 * 4], const double (&part)[V], int c0tile, int ld,
                                                  double* __restrict__ acc) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < V; ++v) red[w][lane * V + v] = part[v];
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * V; i += 256) {
    const int c = c0tile + i;
    if (c < ld) {
      const double s = red[0][i] + red[1][i] + red[2][i] + red[3][i];
      if (s != 0.0) unsafeAtomicAdd(&acc[c], s);
    }
  }
}

// right-hand side entries of row r: a dense FP64 block when given, else the sparse columns
// -A_IB[r, :] and the load column
template <typename TT, int V>
__device__ __forceinline__ void rhs_row(const CgSys& S, int r, int c0, TT (&v)[V]) {
  if (S.Fd != nullptr) {
    const double* fr = S.Fd + (int64_t)r * S.ld + c0;
#pragma unroll
    for (int q = 0; q < V; ++q) v[q] = (TT)fr[q];
    return;
  }
#pragma unroll
  for (int q = 0; q < V; ++q) v[q] = 0;
  const int e1 = S.rp[r + 1];
  for (int e = S.ii_end[r]; e < e1; ++e) {
    const int j = S.col[e] - S.nI - c0;
    if (j >= 0 && j < V) {
#pragma unroll
      for (int q = 0; q < V; ++q)
        if (q == j) v[q] = (TT)(-S.val64[e]);
    }
  }
  if (S.f != nullptr) {
    const int j = S.nB - c0;
    if (j >= 0 && j < V) {
#pragma unroll
      for (int q = 0; q < V; ++q)
        if (q == j) v[q] = (TT)S.f[r];
    }
  }
}

#define MOR_TILE_PROLOGUE(V)                                  \
  const int t = xcd_tile(blockIdx.x, ntiles);                 \
  if (t >= ntiles) return;                                    \
  const int4 tl = tiles[t];                                   \
  const CgSys& S = sys[tl.x];                                 \
  const int lane = threadIdx.x & 63, w = wave_id();           \
  const int c0 = tl.z + lane * (V);                           \
  const bool act = c0 < S.ld;                                 \
  const int ld = S.ld;                                        \
  const int rend = min(tl.y + rb, S.nI);

template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_init(const CgSys* __restrict__ sys, const int4* __restrict__ tiles, int ntiles,
                                                 int rb) {
  MOR_TILE_PROLOGUE(V)
  if (!act) return;
  T* X = (T*)S.X; T* R = (T*)S.R;
  for (int r = tl.y + w; r < rend; r += 4) {
    T v[V], z[V];
    rhs_row<T, V>(S, r, c0, v);
#pragma unroll
    for (int q = 0; q < V; ++q) z[q] = 0;
    const int64_t o = (int64_t)r * ld + c0;
    st_vec<T, V>(R + o, v);
    st_vec<T, V>(X + o, z);
    if (S.X64 != nullptr) {
#pragma unroll
      for (int q = 0; q < V; ++q) S.X64[o + q] = 0.0;
    }
  }
}

// Q = A_II P and the per-column p'Q: the dominant, HBM-bound kernel of the lifting.
// The tile's CSR rows (column ids and values of the II block) are staged in LDS first, so each
// wave issues the neighbour-row loads of a row back to back instead of chasing the CSR in
// global memory; tiles whose rows exceed the LDS capacity read the CSR from global memory.
constexpr int kSpmmMaxRows = 64;
constexpr int kSpmmNnzCap = 1536;

// One row of Q = A P over this lane's V columns: the CSR entries come in chunks of 8; a chunk
// always issues 8 loads (entries past the row end read the row itself with weight 0) so the
// loads of a chunk go out back to back without branches or waits in between.
template <typename T, int V, typename IdxFn, typename ValFn>
__device__ __forceinline__ void spmm_row(const T* __restrict__ P, int ld, int c0, int self, int cnt, IdxFn idx,
                                         ValFn vals, T (&acc)[V]) {
  for (int e = 0; e < cnt; e += 8) {
    int cl[8];
    T a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool ok = e + k < cnt;
      cl[k] = ok ? idx(e + k) : self;
      a[k] = ok ? vals(e + k) : (T)0;
    }
    T p[8][V];
#pragma unroll
    for (int k = 0; k < 8; ++k) ld_vec<T, V>(P + (int64_t)cl[k] * ld + c0, p[k]);
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int q = 0; q < V; ++q) acc[q] += a[k] * p[k][q];
  }
}

template <typename T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  __builtin_nontemporal_store(v, (MOR_GLOBAL T*)p);
}
template <typename T>
__device__ __forceinline__ T ld_nt(const T* p) {
  return __builtin_nontemporal_load((const MOR_GLOBAL T*)p);
}

template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_spmm(const CgSys* __restrict__ sys, const int4* __restrict__ tiles, int ntiles,
                                                 int rb) {
  __shared__ double red[4][64 * 4];
  __shared__ int s_beg[kSpmmMaxRows + 1], s_off[kSpmmMaxRows + 1];
  __shared__ int s_col[kSpmmNnzCap];
  __shared__ T s_val[kSpmmNnzCap];
  MOR_TILE_PROLOGUE(V)
  const T* __restrict__ val = (sizeof(T) == 4) ? (const T*)S.val32 : (const T*)S.val64;
  const T* __restrict__ P = (const T*)S.P;
  T* __restrict__ Q = (T*)S.Q;
  const int nr = rend - tl.y;
  const int tid = threadIdx.x;
  if (tid < nr) {
    const int r = tl.y + tid;
    s_beg[tid] = gld(S.rp + r);
    s_off[tid + 1] = gld(S.ii_end + r) - s_beg[tid];
  }
  if (tid == 0) s_off[0] = 0;
  __syncthreads();
  if (tid == 0)
    for (int i = 0; i < nr; ++i) s_off[i + 1] += s_off[i];
  __syncthreads();
  const bool staged = s_off[nr] <= kSpmmNnzCap;
  if (staged) {
    for (int i = w; i < nr; i += 4) {
      const int cnt = s_off[i + 1] - s_off[i];
      for (int e = lane; e < cnt; e += 64) {
        s_col[s_off[i] + e] = gld(S.col + s_beg[i] + e);
        s_val[s_off[i] + e] = gld(val + s_beg[i] + e);
      }
    }
  }
  __syncthreads();
  double part[V];
#pragma unroll
  for (int q = 0; q < V; ++q) part[q] = 0.0;
  if (act) {
    for (int i = w; i < nr; i += 4) {
      const int r = tl.y + i;
      T acc[V];
#pragma unroll
      for (int q = 0; q < V; ++q) acc[q] = 0;
      const int cnt = s_off[i + 1] - s_off[i];
      const int so = s_off[i], gb = s_beg[i];
      if (staged)
        spmm_row<T, V>(P, ld, c0, r, cnt, [&](int e) { return s_col[so + e]; }, [&](int e) { return s_val[so + e]; }, acc);
      else
        spmm_row<T, V>(P, ld, c0, r, cnt, [&](int e) { return gld(S.col + gb + e); }, [&](int e) { return gld(val + gb + e); },
                       acc);
      const int64_t o = (int64_t)r * ld + c0;
#pragma unroll
      for (int q = 0; q < V; ++q) st_nt(Q + o + q, acc[q]);
      T pr[V];
      ld_vec<T, V>(P + o, pr);
#pragma unroll
      for (int q = 0; q < V; ++q) part[q] += (double)pr[q] * (double)acc[q];
    }
  }
  column_reduce_add<V>(red, part, tl.z, ld, S.pq);
}

// Q = A_II P through LDS.  A workgroup owns one row tile (a host-built run of whole row
// aggregates) of one system and sweeps a group of its column slices (CWB bytes of a row each); the launch lists
// (system, slice group, tile) with the tile fastest, so the workgroups resident on one XCD
// work on neighbouring tiles of the same slices at the same time.  Per slice, every P row
// the tile reads (its halo) is loaded once into LDS, 16 bytes per lane, and each wave forms its
// rows' Q entries from LDS alone: the L2/HBM reads per output row drop from one per matrix
// entry (about 15) to halo/rows (about 4), and neighbouring tiles (consecutive workgroups on one
// XCD) share the halo rows in L2.  The tile's CSR (halo offsets and values, padded to chunks of
// 8) is staged once; the next slice's loads are in flight while the current slice computes.
// FP32: one column per lane, one row per wave step; FP64: 32 columns, two rows per wave step.
template <typename T, int CAP, int CWB>
__global__ __launch_bounds__(256) void k_cg_spmm_halo(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                      int ntiles) {
  constexpr int CW = CWB / (int)sizeof(T);   // columns per slice (a slice is CWB bytes of a row)
  constexpr int RPW = 64 / CW;               // rows per wave step
  constexpr int CPC = 16 / (int)sizeof(T);   // elements per 16-byte staging chunk
  constexpr int CPR = CWB / 16;              // staging chunks per halo row
  constexpr int NST = (CAP * CPR + 255) / 256;       // staging chunks per thread
  constexpr int NZC = halo_nnz_cap(CAP);             // padded CSR entries per tile
  constexpr int NNZ = (NZC + 255) / 256;             // padded CSR entries per thread
  __shared__ __attribute__((aligned(16))) T hp[CAP * CW];
  __shared__ __attribute__((aligned(16))) T s_val[NZC];
  __shared__ __attribute__((aligned(16))) uint16_t s_off[NZC];   // halo position * CW
  __shared__ int s_p[kHaloRows + 1], s_self[kHaloRows];
  __shared__ double red[4 * 64];
  const int t = xcd_tile(blockIdx.x, ntiles);
  if (t >= ntiles) return;
  const int4 tl = tiles[t];
  const CgSys& S = sys[tl.x];
  const int4 ht = S.htile[tl.y];   // first row, rows, first halo entry, halo size
  const int ld = S.ld;
  const int cbeg = tl.z, cend = min(tl.w, ld);
  const T* __restrict__ P = (const T*)S.P;
  T* __restrict__ Q = (T*)S.Q;
  const T* __restrict__ val = (sizeof(T) == 4) ? (const T*)S.val32 : (const T*)S.val64;
  const int tid = threadIdx.x;
  const int nchunk = ht.w * CPR;
  const int pb = gld(S.hrowp + ht.x);
  const int np = gld(S.hrowp + ht.x + ht.y) - pb;   // <= NZC (host-checked)
  int64_t hoff[NST];   // element offset of each staged chunk's halo row (slice 0), -1: none
#pragma unroll
  for (int k = 0; k < NST; ++k) {
    const int i = k * 256 + tid;
    hoff[k] = i < nchunk ? (int64_t)gld(S.halo + ht.z + i / CPR) * ld + (i % CPR) * CPC : -1;
  }
#pragma unroll
  for (int k = 0; k < NNZ; ++k) {
    const int i = k * 256 + tid;
    if (i < np) {
      const int e = gld(S.hpe + pb + i);
      s_off[i] = (uint16_t)(gld(S.hpp + pb + i) * CW);
      s_val[i] = e >= 0 ? gld(val + e) : (T)0;
    }
  }
  if (tid <= ht.y) s_p[tid] = gld(S.hrowp + ht.x + tid) - pb;
  if (tid < ht.y) s_self[tid] = (int)gld(S.hself + ht.x + tid) * CW;
  u32x4 pv[NST];
  auto issue = [&](int c0) {
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      pv[k] = (u32x4){0u, 0u, 0u, 0u};
      if (hoff[k] >= 0 && c0 + ((k * 256 + tid) % CPR) * CPC < ld)
        pv[k] = *((const MOR_GLOBAL u32x4*)(P + hoff[k] + c0));
    }
  };
  issue(cbeg);
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int sub = lane / CW, col = lane % CW;
  // per-column p'Q of the previous slice: summed over the waves after the next barrier
  auto flush = [&](int cp) {
    if (tid < CW && cp + tid < ld) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w)
#pragma unroll
        for (int sb = 0; sb < RPW; ++sb) sum += red[w * 64 + sb * CW + tid];
      if (sum != 0.0) unsafeAtomicAdd(&S.pq[cp + tid], sum);
    }
  };
  for (int c0 = cbeg; c0 < cend; c0 += CW) {
    __syncthreads();   // the previous slice is done with hp; its red is complete
    if (c0 > cbeg) flush(c0 - CW);
#pragma unroll
    for (int k = 0; k < NST; ++k) {
      const int i = k * 256 + tid;
      if (i < nchunk) *reinterpret_cast<u32x4*>(&hp[(i / CPR) * CW + (i % CPR) * CPC]) = pv[k];
    }
    __syncthreads();
    if (c0 + CW < cend) issue(c0 + CW);
    const bool act = c0 + col < ld;
    double part = 0.0;
    for (int i0 = wv * RPW; i0 < ht.y; i0 += 4 * RPW) {
      const int i = i0 + sub;
      if (i < ht.y) {
        const int e0 = s_p[i], e1 = s_p[i + 1];
        T acc = 0;
        for (int e = e0; e < e1; e += 8) {
#pragma unroll
          for (int k = 0; k < 8; ++k) acc += s_val[e + k] * hp[s_off[e + k] + col];
        }
        if (act) {
          st_nt(Q + (int64_t)(ht.x + i) * ld + c0 + col, acc);
          part += (double)hp[s_self[i] + col] * (double)acc;
        }
      }
    }
    red[wv * 64 + lane] = part;
  }
  __syncthreads();
  flush(cbeg + (cend - cbeg - 1) / CW * CW);
}

// Q = A_II P for a subdomain whose interior rows fill a box of a Kuhn lattice (FP32): a
// plane-streaming stencil.  A workgroup owns an 8 x 8 footprint of the box in (x, y) and one
// 128-byte column slice, and marches along z.  Three planes of P (the footprint with a one-point
// ring, z-1, z, z+1) and two planes of stencil coefficients (16 per row, from the assembled
// matrix) sit in LDS; the loads of planes z+2 and z+3 are issued into registers before plane z
// computes, and the grid-point -> row lookups run one plane ahead of those loads, so a lookup
// never waits on a plane's loads.  Each P row of the box is fetched once per slice by the
// workgroup and shared with the neighbouring footprints (consecutive workgroups on one XCD)
// through L2.  Grid points outside the box (interface or Dirichlet nodes) read as zero, and
// their coefficients are zero.
// Each thread owns one column and one footprint row of 8 points, reading each LDS value once
// through sliding windows along x; per-column p'Q is summed over the workgroup and added once.
constexpr int kBoxF = 8;                     // footprint edge
constexpr int kBoxH = kBoxF + 2;             // with the ring
constexpr int kBoxRows = kBoxH * kBoxH;      // halo rows per plane
constexpr int kBoxChunks = kBoxRows * 8;     // 16-byte chunks of one 128-byte slice per plane
constexpr int kBoxLd = (kBoxChunks + 255) / 256;   // chunk loads per thread and plane

struct BoxRows {    // one plane's row lookups for this thread: its P chunks and its coefficient
  int r[kBoxLd];    // point, read at clamped coordinates, and which of them lie in the box (bit k:
  int rc;           // chunk k, bit kBoxLd: the point); the bits are applied where the rows are used
  unsigned in;
};
struct BoxPlane {   // one plane's loads in flight: P chunks, the coefficient chunk, its row,
  u32x4 pv[kBoxLd]; // and which of them lie in the box (bit k: chunk k, bit kBoxLd: the
  u32x4 cv;         // coefficients); the others are replaced by zeros when they reach LDS, not
  int rc;           // before, so that nothing waits for a load until its plane is stored
  unsigned ok;
};

// Grid point -> row lookup.  Branch-free: a point outside the box reads a clamped (valid) entry
// and `in` says so, so every load of a plane is issued unconditionally and the compiler can count
// them when it waits for the oldest (a load issued on one path only makes it assume the fewest
// ops after the awaited one, and drain everything in flight); the result is only used, and so
// only waited for, when the next plane's loads go out.
__device__ __forceinline__ int box_lookup(const CgSys& S, int x, int y, int z, bool& in) {
  in = (unsigned)x < (unsigned)S.bx && (unsigned)y < (unsigned)S.by && (unsigned)z < (unsigned)S.bz;
  return gld(S.smap + ((int64_t)(in ? z : 0) * S.by + (in ? y : 0)) * S.bx + (in ? x : 0));
}

__device__ __forceinline__ u32x4 box_keep(bool keep, u32x4 v) {
  return (u32x4){keep ? v.x : 0u, keep ? v.y : 0u, keep ? v.z : 0u, keep ? v.w : 0u};
}

__device__ __forceinline__ void box_rows(const CgSys& S, int x0, int y0, int z, BoxRows& q) {
  const int tid = threadIdx.x;
  unsigned in = 0;
#pragma unroll
  for (int k = 0; k < kBoxLd; ++k) {
    const int i = k * 256 + tid, hr = i < kBoxChunks ? i >> 3 : 0;
    bool b;
    q.r[k] = box_lookup(S, x0 - 1 + hr % kBoxH, y0 - 1 + hr / kBoxH, z, b);
    in |= b && i < kBoxChunks ? 1u << k : 0u;
  }
  const int pt = tid >> 2;   // coefficient point of this thread: quarter tid % 4 of its 16 values
  bool b;
  q.rc = box_lookup(S, x0 + (pt & 7), y0 + (pt >> 3), z, b);
  q.in = in | (b ? 1u << kBoxLd : 0u);
}

__device__ __forceinline__ void box_issue(const CgSys& S, const float* __restrict__ P, int c0, const BoxRows& q,
                                          BoxPlane& b) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBoxLd; ++k) {
    const int i = k * 256 + tid;   // rows outside the box read row 0 (zeroed when stored)
    const int64_t o = (q.in >> k) & 1u ? (int64_t)q.r[k] * S.ld + (i & 7) * 4 : 0;
    b.pv[k] = *((const MOR_GLOBAL u32x4*)(P + o + c0));
  }
  const bool pin = (q.in >> kBoxLd) & 1u;
  const int64_t oc = pin ? (int64_t)q.rc * kStencil + (tid & 3) * 4 : 0;
  b.cv = *((const MOR_GLOBAL u32x4*)(S.s16 + oc));
  b.rc = pin ? q.rc : -1;
  b.ok = q.in;
}

__device__ __forceinline__ void box_store(const BoxPlane& b, float (*pl)[32], float* cf, int* rid) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBoxLd; ++k) {
    const int i = k * 256 + tid;
    if (i < kBoxChunks) *reinterpret_cast<u32x4*>(&pl[i >> 3][(i & 7) * 4]) = box_keep((b.ok >> k) & 1u, b.pv[k]);
  }
  *reinterpret_cast<u32x4*>(&cf[tid * 4]) = box_keep((b.ok >> kBoxLd) & 1u, b.cv);
  if ((tid & 3) == 0) rid[tid >> 2] = b.rc;
}

__global__ __launch_bounds__(256) void k_cg_spmm_box(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                     int ntiles) {
  __shared__ __attribute__((aligned(16))) float pl[3][kBoxRows][32];
  __shared__ __attribute__((aligned(16))) float cf[2][kBoxF * kBoxF * kStencil];
  __shared__ int rid[2][kBoxF * kBoxF];
  __shared__ double red[8][32];
  const int t = xcd_tile(blockIdx.x, ntiles);
  if (t >= ntiles) return;
  const int4 tl = tiles[t];
  const CgSys& S = sys[tl.x];
  const int x0 = (tl.y & 0xffff) * kBoxF, y0 = (tl.y >> 16) * kBoxF, c0 = tl.z;
  const float* __restrict__ P = (const float*)S.P;
  float* __restrict__ Q = (float*)S.Q;
  const int ld = S.ld, nz = S.bz;
  const int tid = threadIdx.x;
  const int col = tid & 31, yy = tid >> 5;        // this thread: column c0 + col, footprint row yy
  // a slice whose columns have all converged is skipped (their alpha is 0: Q is not read)
  if (!__syncthreads_or(c0 + col < ld && S.active[c0 + col] != 0)) return;
  // P slot of plane z: (z + 3) % 3 (plane -1 is zeros); coefficient and row-id slot: z % 2
  BoxRows q, qa, qb;
  BoxPlane A, B;
  box_rows(S, x0, y0, -1, q);
  box_issue(S, P, c0, q, A);
  box_store(A, pl[2], cf[1], rid[1]);
  box_rows(S, x0, y0, 0, q);
  box_issue(S, P, c0, q, A);
  box_store(A, pl[0], cf[0], rid[0]);
  box_rows(S, x0, y0, 1, q);
  box_issue(S, P, c0, q, A);
  box_store(A, pl[1], cf[1], rid[1]);
  box_rows(S, x0, y0, 2, q);
  box_issue(S, P, c0, q, A);
  box_rows(S, x0, y0, 3, q);
  box_issue(S, P, c0, q, B);
  box_rows(S, x0, y0, 4, qa);
  __syncthreads();
  double part = 0.0;
  // one plane: Q rows of plane z from slots (lower, centre, upper); then plane z+2 from `nx`
  // into the lower slot, the rows of plane z+5 into `qn` and the loads of plane z+4 (rows in
  // `qz`) into `nx`.  The rows are looked up before the loads go out, so that waiting for them
  // (next plane) leaves those loads in flight; qa / qb alternate, so nothing in flight is copied.
  auto plane = [&](int z, BoxPlane& nx, const BoxRows& qz, BoxRows& qn) {
    const int sc = z % 3, su = (z + 1) % 3, sl = (z + 2) % 3, cs = z & 1;
    const float* cfz = cf[cs];
    // the thread's values of plane slot L at footprint row yy + dy, point xi (-1..8)
    const int hb = (yy + 1) * kBoxH + 1;
    auto V = [&](int L, int dy, int xi) { return pl[L][hb + dy * kBoxH + xi][col]; };
    // sliding windows along x: each LDS value is read once per thread (c: centre plane at rows
    // y-1 / y / y+1, u: upper plane at y / y+1, l: lower plane at y-1 / y; m / 0 / 1 = x-1 / x / x+1)
    float cmm = V(sc, -1, -1), cm0 = V(sc, -1, 0), c0m = V(sc, 0, -1), c00 = V(sc, 0, 0), cp0 = V(sc, 1, 0);
    float u00 = V(su, 0, 0), up0 = V(su, 1, 0);
    float lmm = V(sl, -1, -1), lm0 = V(sl, -1, 0), l0m = V(sl, 0, -1), l00 = V(sl, 0, 0);
#pragma unroll
    for (int x = 0; x < kBoxF; ++x) {
      const float c01 = V(sc, 0, x + 1), cp1 = V(sc, 1, x + 1), u01 = V(su, 0, x + 1), up1 = V(su, 1, x + 1);
      const float* c = cfz + (yy * kBoxF + x) * kStencil;
      float acc = c[0] * c00;
      acc += c[1] * c01;
      acc += c[2] * cp0;
      acc += c[3] * u00;
      acc += c[4] * cp1;
      acc += c[5] * u01;
      acc += c[6] * up0;
      acc += c[7] * up1;
      acc += c[8] * c0m;
      acc += c[9] * cm0;
      acc += c[10] * l00;
      acc += c[11] * cmm;
      acc += c[12] * l0m;
      acc += c[13] * lm0;
      acc += c[14] * lmm;
      // the stores stay conditional (a point outside the box has rid -1): then a wait for plane
      // z+2 also completes most of plane z+3's loads, but storing such points into spare rows,
      // which makes every count exact, took 174-186 VGPRs (two workgroups per CU) and was slower
      const int r = rid[cs][yy * kBoxF + x];
      if (r >= 0) {
        st_nt(Q + (int64_t)r * ld + c0 + col, acc);
        part += (double)c00 * (double)acc;
      }
      if (x + 1 < kBoxF) {
        c0m = c00; c00 = c01; cp0 = cp1; u00 = u01; up0 = up1;
        cmm = cm0; cm0 = V(sc, -1, x + 1);
        l0m = l00; l00 = V(sl, 0, x + 1);
        lmm = lm0; lm0 = V(sl, -1, x + 1);
      }
    }
    __syncthreads();
    box_store(nx, pl[sl], cf[cs], rid[cs]);
    __syncthreads();
    box_rows(S, x0, y0, z + 5, qn);
    box_issue(S, P, c0, qz, nx);
  };
  int z = 0;
  for (; z + 1 < nz; z += 2) {
    plane(z, A, qa, qb);
    plane(z + 1, B, qb, qa);
  }
  if (z < nz) plane(z, A, qa, qb);
  red[yy][col] = part;
  __syncthreads();
  if (tid < 32 && c0 + tid < ld) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < 8; ++w) sum += red[w][tid];
    if (sum != 0.0) unsafeAtomicAdd(&S.pq[c0 + tid], sum);
  }
}

// Stencil-ordered FP32 coefficients of a box interior from the assembled FP64 CSR values:
// s16[16 r + s] = val[spos[16 r + s]], 0 where the slot has no II entry.
__global__ void k_box_coeffs(const int* __restrict__ spos, const double* __restrict__ val, int n16, float* __restrict__ s16) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n16) return;
  const int e = spos[i];
  s16[i] = e >= 0 ? (float)val[e] : 0.0f;
}
void launch_box_coeffs(const int* spos, const double* val, int nI, float* s16, hipStream_t s) {
  const int n = nI * kStencil;
  if (n > 0) hipLaunchKernelGGL(k_box_coeffs, dim3((n + 255) / 256), dim3(256), 0, s, spos, val, n, s16);
}
void launch_cg_spmm_box(const CgSys* sys, const int4* tiles, int ntiles, hipStream_t s) {
  // xcd_tile spreads the tiles over a grid of whole groups of 8 workgroups
  if (ntiles > 0) hipLaunchKernelGGL(k_cg_spmm_box, dim3(xcd_grid(ntiles)), dim3(256), 0, s, sys, tiles, ntiles);
}

// Block-Jacobi preconditioner: z = M^-1 r with M the diagonal blocks of A_II over the row
// aggregates (at most 8 rows each).  A wave owns whole aggregates, so applying M^-1 needs no
// data beyond the rows the kernel streams anyway.
#define MOR_BLOCK_PROLOGUE(V)                                 \
  const int t = xcd_tile(blockIdx.x, ntiles);                 \
  if (t >= ntiles) return;                                    \
  const int4 tl = tiles[t];                                   \
  const CgSys& S = sys[tl.x];                                 \
  const int lane = threadIdx.x & 63, w = wave_id();           \
  const int c0 = tl.z + lane * (V);                           \
  const bool act = c0 < S.ld;                                 \
  const int ld = S.ld;                                        \
  const int bend = min(tl.y + bpt, S.nblk);

// z = row j (< nb) of the block inverse times the block's rows rr (rows past nb zero).  The row
// holds 8 entries, zero past nb, so all 8 are read without a branch; callers apply it to every j
// with the row clamped to nb - 1 (the results past nb are not used), so that no branch separates
// the reads of a block's rows and they go out together.
template <typename T, int V>
__device__ __forceinline__ void block_apply(const T* __restrict__ minv, int r0, int nb, const T (&rr)[8][V], int j,
                                            T (&z)[V]) {
  (void)nb;
#pragma unroll
  for (int q = 0; q < V; ++q) z[q] = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const T m = gld(minv + (int64_t)(r0 + j) * 8 + k);
#pragma unroll
    for (int q = 0; q < V; ++q) z[q] += m * rr[k][q];
  }
}

// Two-level preconditioner, restriction: add the column sums of an aggregate's rows (rr) to this
// thread's running sums.  The host makes the streaming tiles divide the coarse blocks, so all
// aggregates of a workgroup lie in one block; the sums leave the kernel once, after the loop
// (stores inside the loop would keep the uniform block-inverse loads off the scalar cache).
template <typename T, int V>
__device__ __forceinline__ void coarse_gather(int nb, const T (&rr)[8][V], double (&cs)[V]) {
#pragma unroll
  for (int j = 0; j < 8; ++j)
    if (j < nb) {
#pragma unroll
      for (int q = 0; q < V; ++q) cs[q] += (double)rr[j][q];
    }
}

// The per-column r'M^-1 r partial sums (added to acc) and, with the two-level preconditioner,
// the coarse block's column sums, reduced over the 4 waves (in one LDS pass when both fit).  A
// tile that covers its whole coarse block (the default tiles of 8 aggregates) stores the block's
// sums; tiles that share a block add theirs.  Every thread of the workgroup calls this.
template <int V>
__device__ __forceinline__ void reduce_rz_coarse(double (*red)[64 * 4], const double (&part)[V], const double (&cs)[V],
                                                 const CgSys& S, bool whole, int b0, int c0tile,
                                                 double* __restrict__ acc) {
  if (S.rc == nullptr) {
    column_reduce_add<V>(red, part, c0tile, S.ld, acc);
    return;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double* rc = S.rc + (int64_t)(b0 / kCoarseAgg) * S.ld;
  auto emit = [&](int i, bool rz, int c) {
    const double s = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    if (rz) {
      if (s != 0.0) unsafeAtomicAdd(&acc[c], s);
    } else if (whole) {
      rc[c] = s;
    } else if (s != 0.0) {
      unsafeAtomicAdd(&rc[c], s);
    }
  };
  if (2 * 64 * V <= 64 * 4) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      red[w][lane * V + v] = part[v];
      red[w][64 * V + lane * V + v] = cs[v];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * 64 * V; i += 256) {
      const bool rz = i < 64 * V;
      const int c = c0tile + (rz ? i : i - 64 * V);
      if (c < S.ld) emit(i, rz, c);
    }
    return;
  }
  for (int pass = 0; pass < 2; ++pass) {
    if (pass) __syncthreads();   // the first pass has finished reading red
#pragma unroll
    for (int v = 0; v < V; ++v) red[w][lane * V + v] = pass ? cs[v] : part[v];
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * V; i += 256)
      if (c0tile + i < S.ld) emit(i, pass == 0, c0tile + i);
  }
}

// P = M^-1 R and r'M^-1 r (start and restarts of the CG)
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_pstart(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                   int ntiles, int bpt) {
  __shared__ double red[4][64 * 4];
  MOR_BLOCK_PROLOGUE(V)
  const T* minv = (const T*)S.minv;
  const T* R = (const T*)S.R; T* P = (T*)S.P;
  double part[V], cs[V];
#pragma unroll
  for (int q = 0; q < V; ++q) part[q] = cs[q] = 0.0;
  if (act) {
    for (int b = tl.y + w; b < bend; b += 4) {
      const int r0 = gld(S.bp + b), nb = gld(S.bp + b + 1) - r0;
      T rr[8][V];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j < nb) ld_vec<T, V>(R + (int64_t)(r0 + j) * ld + c0, rr[j]);
        else {
#pragma unroll
          for (int q = 0; q < V; ++q) rr[j][q] = 0;
        }
      }
      if (S.rc != nullptr) coarse_gather<T, V>(nb, rr, cs);
      T zz[8][V];
#pragma unroll
      for (int j = 0; j < 8; ++j) {   // rows past nb: rr is zero, nothing is stored
        block_apply<T, V>(minv, r0, nb, rr, min(j, nb - 1), zz[j]);
#pragma unroll
        for (int q = 0; q < V; ++q) part[q] += (double)rr[j][q] * (double)zz[j][q];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < nb) st_vec<T, V>(P + (int64_t)(r0 + j) * ld + c0, zz[j]);
    }
  }
  const bool whole = tl.y % kCoarseAgg == 0 && (bend - tl.y >= kCoarseAgg || bend == S.nblk);
  reduce_rz_coarse<V>(red, part, cs, S, whole, tl.y, tl.z, S.rz);
}

// R -= alpha Q and the new r'M^-1 r
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_update(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                   int ntiles, int bpt) {
  __shared__ double red[4][64 * 4];
  MOR_BLOCK_PROLOGUE(V)
  const T* minv = (const T*)S.minv;
  T* R = (T*)S.R; const T* Q = (const T*)S.Q;
  T al[V];
  double part[V], cs[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    part[q] = cs[q] = 0.0;
    al[q] = act ? (T)S.alpha[c0 + q] : (T)0;
  }
  // (no skip of converged columns here: the tiles are short, and waiting for alpha before the
  // first loads cost more than the skipped columns saved)
  if (act) {
    for (int b = tl.y + w; b < bend; b += 4) {
      const int r0 = gld(S.bp + b), nb = gld(S.bp + b + 1) - r0;
      T rr[8][V], qq[8][V];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j < nb) {
          ld_vec<T, V>(R + (int64_t)(r0 + j) * ld + c0, rr[j]);
          ld_vec<T, V>(Q + (int64_t)(r0 + j) * ld + c0, qq[j]);
        } else {
#pragma unroll
          for (int q = 0; q < V; ++q) rr[j][q] = qq[j][q] = 0;
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int q = 0; q < V; ++q) rr[j][q] -= al[q] * qq[j][q];
      if (S.rc != nullptr) coarse_gather<T, V>(nb, rr, cs);
      // every row's block-Jacobi product before the first store: the compiler keeps the
      // (scalar) block-inverse loads after a store that may alias them, so between the rows'
      // stores they went out, and were waited for, one row at a time
#pragma unroll
      for (int j = 0; j < 8; ++j) {   // rows past nb: rr is zero and adds nothing
        T z[V];
        block_apply<T, V>(minv, r0, nb, rr, min(j, nb - 1), z);
#pragma unroll
        for (int q = 0; q < V; ++q) part[q] += (double)rr[j][q] * (double)z[q];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < nb) st_vec<T, V>(R + (int64_t)(r0 + j) * ld + c0, rr[j]);
    }
  }
  const bool whole = tl.y % kCoarseAgg == 0 && (bend - tl.y >= kCoarseAgg || bend == S.nblk);
  reduce_rz_coarse<V>(red, part, cs, S, whole, tl.y, tl.z, S.rznew);
}

// X += alpha P (the step of this iteration), then P = M^-1 R + beta P
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_direction(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                      int ntiles, int bpt) {
  MOR_BLOCK_PROLOGUE(V)
  if (!act) return;
  const T* minv = (const T*)S.minv;
  const T* R = (const T*)S.R; T* P = (T*)S.P; T* X = (T*)S.X;
  T be[V], al[V];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    be[q] = (T)S.beta[c0 + q];
    al[q] = (T)S.alpha[c0 + q];
  }
  {   // converged columns (alpha 0) keep X; their P is rebuilt at the next restart
    int any = 0;
#pragma unroll
    for (int q = 0; q < V; ++q) any |= al[q] != (T)0;
    if (!any) return;
  }
  for (int b = tl.y + w; b < bend; b += 4) {
    const int r0 = gld(S.bp + b), nb = gld(S.bp + b + 1) - r0;
    T ec[V];   // coarse correction of this aggregate's block (two-level preconditioner)
#pragma unroll
    for (int q = 0; q < V; ++q) ec[q] = 0;
    if (S.ec != nullptr) {
      const double* e = S.ec + (int64_t)(b / kCoarseAgg) * ld + c0;
#pragma unroll
      for (int q = 0; q < V; ++q) ec[q] = (T)e[q];
    }
    // the block's R, P and X rows are all loaded before any store: the compiler keeps a load
    // after a store that may alias it, so X loads between the rows' stores went out one row at
    // a time, each waited for in turn (R first: the block-Jacobi products need all its rows)
    T rr[8][V], pp[8][V], xx[8][V];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < nb) ld_vec<T, V>(R + (int64_t)(r0 + j) * ld + c0, rr[j]);
      else {
#pragma unroll
        for (int q = 0; q < V; ++q) rr[j][q] = 0;
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < nb) {
        ld_vec<T, V>(P + (int64_t)(r0 + j) * ld + c0, pp[j]);
        ld_vec<T, V>(X + (int64_t)(r0 + j) * ld + c0, xx[j]);
      } else {
#pragma unroll
        for (int q = 0; q < V; ++q) pp[j][q] = xx[j][q] = 0;
      }
    }
    T zz[8][V];   // every new direction is formed before the first store, for the same reason
#pragma unroll
    for (int j = 0; j < 8; ++j) {   // rows past nb are not stored
      block_apply<T, V>(minv, r0, nb, rr, min(j, nb - 1), zz[j]);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        xx[j][q] += al[q] * pp[j][q];
        zz[j][q] += ec[q] + be[q] * pp[j][q];
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < nb) {
        const int64_t o = (int64_t)(r0 + j) * ld + c0;
        st_vec<T, V>(X + o, xx[j]);
        st_vec<T, V>(P + o, zz[j]);
      }
    }
  }
}

// P += P_c A_c^-1 P_c^T R at a (re)start of the two-level preconditioned CG: the coarse
// correction of each aggregate's block, added to the block-Jacobi start direction
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_prolong(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                    int ntiles, int bpt) {
  MOR_BLOCK_PROLOGUE(V)
  if (!act || S.ec == nullptr) return;
  T* P = (T*)S.P;
  for (int b = tl.y + w; b < bend; b += 4) {
    const int r0 = gld(S.bp + b), nb = gld(S.bp + b + 1) - r0;
    const double* e = S.ec + (int64_t)(b / kCoarseAgg) * ld + c0;
    T ec[V];
#pragma unroll
    for (int q = 0; q < V; ++q) ec[q] = (T)e[q];
    for (int j = 0; j < nb; ++j) {
      T p[V];
      ld_vec<T, V>(P + (int64_t)(r0 + j) * ld + c0, p);
#pragma unroll
      for (int q = 0; q < V; ++q) p[q] += ec[q];
      st_vec<T, V>(P + (int64_t)(r0 + j) * ld + c0, p);
    }
  }
}

// X64 += X (accumulate a correction into the FP64 solution)
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_shadow(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                   int ntiles, int rb) {
  MOR_TILE_PROLOGUE(V)
  if (!act || S.X64 == nullptr) return;
  const T* X = (const T*)S.X;
  for (int r = tl.y + w; r < rend; r += 4) {
    const int64_t o = (int64_t)r * ld + c0;
    T x[V];
    ld_vec<T, V>(X + o, x);
#pragma unroll
    for (int q = 0; q < V; ++q) S.X64[o + q] += (double)x[q];
  }
}

// FP64 residual of the FP64 solution: R = F - A_II X64 (rounded to T), X = 0.
template <typename T, int V>
__global__ __launch_bounds__(256) void k_cg_residual64(const CgSys* __restrict__ sys, const int4* __restrict__ tiles,
                                                       int ntiles, int rb) {
  MOR_TILE_PROLOGUE(V)
  if (!act) return;
  T* X = (T*)S.X; T* R = (T*)S.R;
  for (int r = tl.y + w; r < rend; r += 4) {
    double acc[V];
    rhs_row<double, V>(S, r, c0, acc);
    const int e1 = S.ii_end[r];
    for (int e = S.rp[r]; e < e1; ++e) {
      const double a = S.val64[e];
      const double* xr = S.X64 + (int64_t)S.col[e] * ld + c0;
#pragma unroll
      for (int q = 0; q < V; ++q) acc[q] -= a * xr[q];
    }
    T rr[V], z[V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      rr[q] = (T)acc[q];
      z[q] = 0;
    }
    const int64_t o = (int64_t)r * ld + c0;
    st_vec<T, V>(R + o, rr);
    st_vec<T, V>(X + o, z);
  }
}

// Inverses of the diagonal blocks of A_II over the row aggregates (one thread per block,
// Gauss-Jordan on the SPD block padded with the identity to 8 x 8, in FP64).
template <typename T>
__global__ void k_block_inv(const int* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ v64,
                            const int* __restrict__ bp, int nblk, T* __restrict__ minv) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int r0 = bp[b], nb = bp[b + 1] - r0;
  double a[8][8], inv[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[i][j] = (i == j && i >= nb) ? 1.0 : 0.0;
      inv[i][j] = (i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (i < nb) {
      const int r = r0 + i;
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const int c = col[e] - r0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (c == j && j < nb) a[i][j] = v64[e];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double d = 1.0 / a[k][k];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[k][j] *= d;
      inv[k][j] *= d;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (i != k) {
        const double f = a[i][k];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          a[i][j] -= f * a[k][j];
          inv[i][j] -= f * inv[k][j];
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < nb)
#pragma unroll
      for (int j = 0; j < 8; ++j) minv[(int64_t)(r0 + i) * 8 + j] = (j < nb) ? (T)inv[i][j] : (T)0;
}

template <typename T>
void launch_block_inv(const int* rp, const int* col, const double* v64, const int* bp, int nblk, void* minv,
                      hipStream_t s) {
  if (nblk > 0)
    hipLaunchKernelGGL(k_block_inv<T>, dim3((nblk + 127) / 128), dim3(128), 0, s, rp, col, v64, bp, nblk, (T*)minv);
}
template void launch_block_inv<float>(const int*, const int*, const double*, const int*, int, void*, hipStream_t);
template void launch_block_inv<double>(const int*, const int*, const double*, const int*, int, void*, hipStream_t);

#define MOR_VSWITCH(T, V, KERNEL, ...)                                                                  \
  do {                                                                                                  \
    const dim3 g_(xcd_grid(ntiles)), b_(256);                                                           \
    if ((V) == 1) hipLaunchKernelGGL((KERNEL<T, 1>), g_, b_, 0, s, __VA_ARGS__);                        \
    else if ((V) == 2) hipLaunchKernelGGL((KERNEL<T, 2>), g_, b_, 0, s, __VA_ARGS__);                   \
    else if (sizeof(T) == 4) hipLaunchKernelGGL((KERNEL<T, (sizeof(T) == 4 ? 4 : 2)>), g_, b_, 0, s, __VA_ARGS__); \
  } while (0)

template <typename T>
void launch_cg_init(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_init, sys, tiles, ntiles, rb);
}
template <typename T>
void launch_cg_spmm(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_spmm, sys, tiles, ntiles, rb);
}
template <typename T, int CWB>
static void launch_halo_cap(const CgSys* sys, const int4* tiles, int ntiles, int cap, hipStream_t s) {
  const dim3 g(xcd_grid(ntiles)), b(256);
  static_assert(kHaloCaps[0] == 48 && kHaloCaps[1] == 64 && kHaloCaps[2] == 96 && kHaloCaps[3] == 128 &&
                kHaloCaps[4] == 176, "halo caps");
  if (cap <= 48) hipLaunchKernelGGL((k_cg_spmm_halo<T, 48, CWB>), g, b, 0, s, sys, tiles, ntiles);
  else if (cap <= 64) hipLaunchKernelGGL((k_cg_spmm_halo<T, 64, CWB>), g, b, 0, s, sys, tiles, ntiles);
  else if (cap <= 96) hipLaunchKernelGGL((k_cg_spmm_halo<T, 96, CWB>), g, b, 0, s, sys, tiles, ntiles);
  else if (cap <= 128) hipLaunchKernelGGL((k_cg_spmm_halo<T, 128, CWB>), g, b, 0, s, sys, tiles, ntiles);
  else hipLaunchKernelGGL((k_cg_spmm_halo<T, 176, CWB>), g, b, 0, s, sys, tiles, ntiles);
}
template <typename T>
void launch_cg_spmm_halo(const CgSys* sys, const int4* tiles, int ntiles, int cap, int cwb, hipStream_t s) {
  if (ntiles <= 0) return;
  if (cwb == 128) launch_halo_cap<T, 128>(sys, tiles, ntiles, cap, s);
  else launch_halo_cap<T, 256>(sys, tiles, ntiles, cap, s);
}
template <typename T>
void launch_cg_update(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_update, sys, tiles, ntiles, rb);
}
template <typename T>
void launch_cg_direction(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_direction, sys, tiles, ntiles, rb);
}
template <typename T>
void launch_cg_residual64(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_residual64, sys, tiles, ntiles, rb);
}
template <typename T>
void launch_cg_shadow(const CgSys* sys, const int4* tiles, int ntiles, int rb, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_shadow, sys, tiles, ntiles, rb);
}
template <typename T>
void launch_cg_pstart(const CgSys* sys, const int4* tiles, int ntiles, int bpt, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_pstart, sys, tiles, ntiles, bpt);
}
template <typename T>
void launch_cg_prolong(const CgSys* sys, const int4* tiles, int ntiles, int bpt, int v, hipStream_t s) {
  if (ntiles > 0) MOR_VSWITCH(T, v, k_cg_prolong, sys, tiles, ntiles, bpt);
}
#define MOR_INST(T)                                                                                      \
  template void launch_cg_init<T>(const CgSys*, const int4*, int, int, int, hipStream_t);       \
  template void launch_cg_spmm<T>(const CgSys*, const int4*, int, int, int, hipStream_t);       \
  template void launch_cg_spmm_halo<T>(const CgSys*, const int4*, int, int, int, hipStream_t);  \
  template void launch_cg_update<T>(const CgSys*, const int4*, int, int, int, hipStream_t);     \
  template void launch_cg_direction<T>(const CgSys*, const int4*, int, int, int, hipStream_t);  \
  template void launch_cg_residual64<T>(const CgSys*, const int4*, int, int, int, hipStream_t); \
  template void launch_cg_shadow<T>(const CgSys*, const int4*, int, int, int, hipStream_t);        \
  template void launch_cg_pstart<T>(const CgSys*, const int4*, int, int, int, hipStream_t);       \
  template void launch_cg_prolong<T>(const CgSys*, const int4*, int, int, int, hipStream_t);
MOR_INST(float)
MOR_INST(double)
#undef MOR_INST

// per-column scalars ------------------------------------------------------------------
// Launched over column blocks (system, first column) of 256 columns; every wave's columns
// belong to one system, so the active count takes one atomic per wave.
__device__ __forceinline__ void count_active_wave(int* cnt, bool active) {
  const unsigned long long m = __ballot(active);
  if ((threadIdx.x & 63) == 0 && m != 0ull) atomicAdd(cnt, (int)__popcll(m));
}

__global__ void k_cg_alpha(const CgSys* __restrict__ sys, const int2* __restrict__ cb) {
  const int2 b = cb[blockIdx.x];
  const CgSys& S = sys[b.x];
  const int j = b.y + threadIdx.x;
  if (b.y == 0 && threadIdx.x == 0) *S.nactive = 0;
  if (j >= S.ld) return;
  const double pq = S.pq[j];
  double a = 0.0;
  if (S.active[j]) {
    if (pq > 0.0) a = S.rz[j] / pq;
    else S.active[j] = 0;   // breakdown: p'Ap <= 0 cannot happen for SPD data
  }
  S.alpha[j] = a;
  S.pq[j] = 0.0;
}

__global__ void k_cg_beta(const CgSys* __restrict__ sys, const int2* __restrict__ cb) {
  const int2 b = cb[blockIdx.x];
  const CgSys& S = sys[b.x];
  const int j = b.y + threadIdx.x;
  bool still = false;
  if (j < S.ld) {
    const double rn = S.rznew[j];
    S.rznew[j] = 0.0;
    if (!S.active[j]) {
      S.beta[j] = 0.0;
    } else if (rn <= S.tol2 * S.rz0[j]) {
      S.active[j] = 0;
      S.beta[j] = 0.0;
      S.rz[j] = rn;
    } else {
      S.beta[j] = rn / S.rz[j];
      S.rz[j] = rn;
      still = true;
    }
  }
  count_active_wave(S.nactive, still);
}

// first = 1: references of a new right-hand side; first = 0: restart from an FP64 residual
// (columns already below the outer target stay frozen).
__global__ void k_cg_start(const CgSys* __restrict__ sys, const int2* __restrict__ cb, int first, double tol2_outer) {
  const int2 b = cb[blockIdx.x];
  const CgSys& S = sys[b.x];
  const int j = b.y + threadIdx.x;
  if (j >= S.ld) return;
  const double rz = S.rz[j];
  S.rz0[j] = rz;
  if (first) S.rzF[j] = rz;
  S.alpha[j] = 0.0;
  S.beta[j] = 0.0;
  S.pq[j] = 0.0;
  S.rznew[j] = 0.0;
  S.active[j] = first ? (rz > 0.0 ? 1 : 0) : ((rz > tol2_outer * S.rzF[j]) ? 1 : 0);
}
// r'M^-1 r of the two-level preconditioner, coarse part: (P^T r)' A_c^-1 (P^T r) per column,
// added to the fine part (rznew during the iteration, rz at a start); P^T r is cleared for the
// next restriction.
__global__ void k_cg_coarse_dot(const CgSys* __restrict__ sys, const int2* __restrict__ cb, int at_start) {
  const int2 b = cb[blockIdx.x];
  const CgSys& S = sys[b.x];
  const int j = b.y + threadIdx.x;
  if (S.rc == nullptr || j >= S.ld) return;
  double s = 0.0;
  for (int c = 0; c < S.nc; ++c) {
    const int64_t o = (int64_t)c * S.ld + j;
    s += S.rc[o] * S.ec[o];
    S.rc[o] = 0.0;
  }
  if (at_start) S.rz[j] += s;
  else S.rznew[j] += s;
}
void launch_cg_coarse_dot(const CgSys* sys, const int2* cb, int ncb, int at_start, hipStream_t s) {
  if (ncb > 0) hipLaunchKernelGGL(k_cg_coarse_dot, dim3(ncb), dim3(256), 0, s, sys, cb, at_start);
}

// A_c = P^T A_II P for the piecewise-constant coarse space: entry (rcb[r], rcb[c]) sums A_II[r, c]
__global__ void k_coarse_assemble(const int* __restrict__ rp, const int* __restrict__ col,
                                  const int* __restrict__ ii_end, const double* __restrict__ v64,
                                  const int* __restrict__ rcb, int nI, double* Ac, int ldac) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nI) return;
  const int cr = rcb[r];
  for (int e = rp[r]; e < ii_end[r]; ++e) unsafeAtomicAdd(&Ac[(int64_t)cr * ldac + rcb[col[e]]], v64[e]);
}
void launch_coarse_assemble(const int* rp, const int* col, const int* ii_end, const double* v64, const int* rcb, int nI,
                            double* Ac, int ldac, hipStream_t s) {
  if (nI > 0)
    hipLaunchKernelGGL(k_coarse_assemble, dim3((nI + 255) / 256), dim3(256), 0, s, rp, col, ii_end, v64, rcb, nI, Ac,
                       ldac);
}

__global__ void k_cg_count(const CgSys* __restrict__ sys, const int2* __restrict__ cb) {
  const int2 b = cb[blockIdx.x];
  const CgSys& S = sys[b.x];
  const int j = b.y + threadIdx.x;
  count_active_wave(S.nactive, j < S.ld && S.active[j] != 0);
}
__global__ void k_cg_zero(const CgSys* __restrict__ sys, const int2* __restrict__ cb) {
  const int2 b = cb[blockIdx.x];
  const CgSys& S = sys[b.x];
  const int j = b.y + threadIdx.x;
  if (b.y == 0 && threadIdx.x == 0) *S.nactive = 0;
  if (j < S.ld) S.rz[j] = 0.0;
}

void launch_cg_alpha(const CgSys* sys, const int2* cb, int ncb, hipStream_t s) {
  if (ncb > 0) hipLaunchKernelGGL(k_cg_alpha, dim3(ncb), dim3(256), 0, s, sys, cb);
}
void launch_cg_beta(const CgSys* sys, const int2* cb, int ncb, hipStream_t s) {
  if (ncb > 0) hipLaunchKernelGGL(k_cg_beta, dim3(ncb), dim3(256), 0, s, sys, cb);
}
void launch_cg_zero(const CgSys* sys, const int2* cb, int ncb, hipStream_t s) {
  if (ncb > 0) hipLaunchKernelGGL(k_cg_zero, dim3(ncb), dim3(256), 0, s, sys, cb);
}
void launch_cg_start(const CgSys* sys, const int2* cb, int ncb, int first, double tol2_outer, hipStream_t s) {
  if (ncb <= 0) return;
  hipLaunchKernelGGL(k_cg_start, dim3(ncb), dim3(256), 0, s, sys, cb, first, tol2_outer);
  hipLaunchKernelGGL(k_cg_count, dim3(ncb), dim3(256), 0, s, sys, cb);
}

// --------------------------------------------------------------------------------- FP64 helpers
__global__ void k_to_f64_block(const float* in, int ldi, double* out, int ldo, int rows, int cols) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)rows * cols;
  if (i >= n) return;
  const int r = (int)(i / cols), c = (int)(i % cols);
  out[(int64_t)r * ldo + c] = (double)in[(int64_t)r * ldi + c];
}
void launch_to_f64_block(const float* in, int ldi, double* out, int ldo, int rows, int cols, hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n > 0) hipLaunchKernelGGL(k_to_f64_block, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, ldi, out, ldo, rows, cols);
}

// Y[r, c] = sum over CSR entries of row r with column < col_limit of val * X[col, c]
__global__ __launch_bounds__(256) void k_spmm64_rows(const int* __restrict__ rp, const int* __restrict__ col,
                                                     const double* __restrict__ val, int nrows, int col_limit,
                                                     const double* __restrict__ X, int ldx, int ncols,
                                                     double* __restrict__ Y, int ldy) {
  const int r = blockIdx.x * 4 + wave_id();
  const int c = blockIdx.y * 64 + (threadIdx.x & 63);
  if (r >= nrows || c >= ncols) return;
  double acc = 0.0;
  const int e1 = rp[r + 1];
  for (int e = rp[r]; e < e1; ++e) {
    const int cc = col[e];
    if (cc < col_limit) acc += val[e] * X[(int64_t)cc * ldx + c];
  }
  Y[(int64_t)r * ldy + c] = acc;
}
void launch_spmm64_rows(const int* rp, const int* col, const double* val, int nrows, int col_limit, const double* X,
                        int ldx, int ncols, double* Y, int ldy, hipStream_t s) {
  if (nrows <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(k_spmm64_rows, dim3((nrows + 3) / 4, (ncols + 63) / 64), dim3(256), 0, s, rp, col, val, nrows,
                     col_limit, X, ldx, ncols, Y, ldy);
}

// S_B = K_BB + K_BI E (Schur complement of the H1 matrix onto B, Lemma 4.1), E = K_II^-1 (-K_IB)
__global__ __launch_bounds__(256) void k_schur(const int* __restrict__ rp, const int* __restrict__ col,
                                               const double* __restrict__ K, int nI, int nB,
                                               const double* __restrict__ E, int lde, double* __restrict__ S, int lds) {
  const int b = blockIdx.x * 4 + wave_id();
  const int c = blockIdx.y * 64 + (threadIdx.x & 63);
  if (b >= nB || c >= nB) return;
  const int r = nI + b;
  double acc = 0.0;
  const int e1 = rp[r + 1];
  for (int e = rp[r]; e < e1; ++e) {
    const int cc = col[e];
    const double a = K[e];
    if (cc < nI) acc += a * E[(int64_t)cc * lde + c];
    else if (cc - nI == c) acc += a;
  }
  S[(int64_t)b * lds + c] = acc;
}
void launch_schur(const int* rp, const int* col, const double* Kval, int nI, int nB, const double* E, int lde, double* S,
                  int lds, hipStream_t s) {
  if (nB <= 0) return;
  hipLaunchKernelGGL(k_schur, dim3((nB + 3) / 4, (nB + 63) / 64), dim3(256), 0, s, rp, col, Kval, nI, nB, E, lde, S, lds);
}

// rows/columns M..MP-1 of an MP x MP matrix become the identity
__global__ void k_pad_identity(double* S, int M, int MP) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)MP * MP;
  if (i >= n) return;
  const int r = (int)(i / MP), c = (int)(i % MP);
  if (r < M && c < M) return;
  S[i] = (r == c) ? 1.0 : 0.0;
}
void launch_pad_identity(double* S, int M, int MP, hipStream_t s) {
  if (M >= MP) return;
  const int64_t n = (int64_t)MP * MP;
  hipLaunchKernelGGL(k_pad_identity, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, M, MP);
}
__global__ void k_symmetrize(double* S, int MP) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)MP * MP;
  if (i >= n) return;
  const int r = (int)(i / MP), c = (int)(i % MP);
  if (r >= c) return;
  const double v = 0.5 * (S[(int64_t)r * MP + c] + S[(int64_t)c * MP + r]);
  S[(int64_t)r * MP + c] = v;
  S[(int64_t)c * MP + r] = v;
}
void launch_symmetrize(double* S, int MP, hipStream_t s) {
  const int64_t n = (int64_t)MP * MP;
  if (n > 0) hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S, MP);
}

// --------------------------------------------------------------------------------- FP64 MFMA tiles
// A 64 x 64 output tile per 256-thread workgroup; wave (wr, wc) owns a 32 x 32 quarter made
// of 2 x 2 blocks of v_mfma_f64_16x16x4 (A: lane -> row lane%16, k lane/16; B: lane -> col
// lane%16, k lane/16; D: lane -> col lane%16, register r -> row lane/16 + 4r).
constexpr int kLdsPad = 68;

// One thread's share of a 16-deep k-step of the A and B tiles (4 + 4 doubles, zero outside
// the matrix), loaded into registers one step ahead so that the loads are in flight while the
// matrix cores work on the current step.
template <bool TA, bool TB>
__device__ __forceinline__ void tile_fetch(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                                           int m, int n, int i0, int j0, int k0, int ke, double (&ra)[4],
                                           double (&rb)[4]) {
  const int tid = threadIdx.x;
  if (!TA) {
    const int i = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + kk + q;
      ra[q] = (i0 + i < m && k < ke) ? A[(int64_t)(i0 + i) * lda + k] : 0.0;
    }
  } else {
    const int kk = tid >> 4, i = (tid & 15) * 4;
    const int k = k0 + kk;
#pragma unroll
    for (int q = 0; q < 4; ++q) ra[q] = (i0 + i + q < m && k < ke) ? A[(int64_t)k * lda + i0 + i + q] : 0.0;
  }
  if (!TB) {
    const int kk = tid >> 4, j = (tid & 15) * 4;
    const int k = k0 + kk;
#pragma unroll
    for (int q = 0; q < 4; ++q) rb[q] = (k < ke && j0 + j + q < n) ? B[(int64_t)k * ldb + j0 + j + q] : 0.0;
  } else {
    const int j = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + kk + q;
      rb[q] = (k < ke && j0 + j < n) ? B[(int64_t)(j0 + j) * ldb + k] : 0.0;
    }
  }
}

template <bool TA, bool TB>
__device__ __forceinline__ void tile_put(const double (&ra)[4], const double (&rb)[4], double (*As)[kLdsPad],
                                         double (*Bs)[kLdsPad]) {
  const int tid = threadIdx.x;
  if (!TA) {
    const int i = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) As[kk + q][i] = ra[q];
  } else {
    const int kk = tid >> 4, i = (tid & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) As[kk][i + q] = ra[q];
  }
  if (!TB) {
    const int kk = tid >> 4, j = (tid & 15) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[kk][j + q] = rb[q];
  } else {
    const int j = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) Bs[kk + q][j] = rb[q];
  }
}

template <bool TA, bool TB>
__device__ __forceinline__ void tile_mma(const double* __restrict__ A, int lda, const double* __restrict__ B, int ldb,
                                         int m, int n, int i0, int j0, int kb, int ke, double (*As)[kLdsPad],
                                         double (*Bs)[kLdsPad], d4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  double ra[4], rb[4];
  if (kb < ke) tile_fetch<TA, TB>(A, lda, B, ldb, m, n, i0, j0, kb, ke, ra, rb);
  for (int k0 = kb; k0 < ke; k0 += 16) {
    tile_put<TA, TB>(ra, rb, As, Bs);
    __syncthreads();
    if (k0 + 16 < ke) tile_fetch<TA, TB>(A, lda, B, ldb, m, n, i0, j0, k0 + 16, ke, ra, rb);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kr = s4 * 4 + (lane >> 4);
      const double a0 = As[kr][wr * 32 + (lane & 15)];
      const double a1 = As[kr][wr * 32 + 16 + (lane & 15)];
      const double b0 = Bs[kr][wc * 32 + (lane & 15)];
      const double b1 = Bs[kr][wc * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void tile_zero(d4 (&acc)[2][2]) {
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
}

// C = alpha * acc + beta * C over the valid part of the tile
__device__ __forceinline__ void tile_store(double* C, int ldc, int m, int n, int i0, int j0, double alpha, double beta,
                                           const d4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int j = j0 + wc * 32 + b * 16 + (lane & 15);
        if (i < m && j < n) {
          double* p = C + (int64_t)i * ldc + j;
          const double v = alpha * acc[a][b][r];
          *p = (beta == 0.0) ? v : v + beta * *p;
        }
      }
}
// symmetric result: tile (ti <= tj); write (i, j) and (j, i) for i <= j inside diagonal tiles
__device__ __forceinline__ void tile_store_sym(double* C, int ldc, int m, int i0, int j0, double alpha,
                                               const d4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  const bool diag = (i0 == j0);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + (lane >> 4) + 4 * r;
        const int j = j0 + wc * 32 + b * 16 + (lane & 15);
        if (i < m && j < m && (!diag || i <= j)) {
          const double v = alpha * acc[a][b][r];
          C[(int64_t)i * ldc + j] = v;
          C[(int64_t)j * ldc + i] = v;
        }
      }
}

// With use_skip, a tile whose output columns all have skip[j] == 0 is left alone (uniform over
// the workgroup).
__device__ __forceinline__ bool gemm_tile_skipped(const GemmDesc& g, int tj, int use_skip) {
  if (!use_skip || g.skip == nullptr) return false;
  const int j = tj * 64 + (threadIdx.x & 63);
  return !__syncthreads_or(j < g.n && g.skip[j] != 0.0);
}

template <bool TA, bool TB>
__device__ void gemm_tile_body(const GemmDesc& g, int ti, int tj, double (*As)[kLdsPad], double (*Bs)[kLdsPad],
                               int use_skip) {
  if (gemm_tile_skipped(g, tj, use_skip)) return;
  d4 acc[2][2];
  tile_zero(acc);
  tile_mma<TA, TB>(g.A, g.lda, g.B, g.ldb, g.m, g.n, ti * 64, tj * 64, 0, g.k, As, Bs, acc);
  if (g.sym) tile_store_sym(g.C, g.ldc, g.m, ti * 64, tj * 64, g.alpha, acc);
  else tile_store(g.C, g.ldc, g.m, g.n, ti * 64, tj * 64, g.alpha, g.beta, acc);
}

// Tiles are listed column tile fastest and dealt round-robin over the XCDs, so that the tiles an
// XCD runs together share their A row panel in its L2 (grouping consecutive tiles on one XCD
// instead measured slower on the coarse products, whose panels do not fit in L2 either way).
__global__ __launch_bounds__(256) void k_gemm(const GemmDesc* __restrict__ descs, const int4* __restrict__ tiles,
                                              int use_skip) {
  __shared__ double As[16][kLdsPad], Bs[16][kLdsPad];
  const int4 tl = tiles[blockIdx.x];
  const GemmDesc& g = descs[tl.x];
  if (!g.ta && !g.tb) gemm_tile_body<false, false>(g, tl.y, tl.z, As, Bs, use_skip);
  else if (g.ta && !g.tb) gemm_tile_body<true, false>(g, tl.y, tl.z, As, Bs, use_skip);
  else if (!g.ta && g.tb) gemm_tile_body<false, true>(g, tl.y, tl.z, As, Bs, use_skip);
  else gemm_tile_body<true, true>(g, tl.y, tl.z, As, Bs, use_skip);
}
void launch_gemm(const GemmDesc* d, const int4* tiles, int ntiles, hipStream_t s, int use_skip) {
  if (ntiles > 0) hipLaunchKernelGGL(k_gemm, dim3(ntiles), dim3(256), 0, s, d, tiles, use_skip);
}

// ------------------------------------------------------------------------ randomized variant
// Right-hand sides of the sketch solve: F[r, j] = -(A_IB T)[r, j] for j < l (T = R_BB^-1 S, MP x
// 64, ld 64), F[r, l] = f[r] (the zero-boundary load problem), zero up to ld.  One thread per
// entry of the I x ld block.
__global__ void k_rhs_sketch(const int* __restrict__ rp, const int* __restrict__ col, const int* __restrict__ ii_end,
                             const double* __restrict__ A, const double* __restrict__ f, int nI, const double* __restrict__ T,
                             int l, double* __restrict__ F, int ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nI * ld) return;
  const int r = (int)(i / ld), j = (int)(i % ld);
  double v = 0.0;
  if (j < l) {
    for (int e = ii_end[r]; e < rp[r + 1]; ++e) v -= A[e] * T[(int64_t)(col[e] - nI) * 64 + j];
  } else if (j == l) {
    v = f[r];
  }
  F[i] = v;
}
void launch_rhs_sketch(const int* rp, const int* col, const int* ii_end, const double* A, const double* f, int nI,
                       const double* T, int l, double* F, int ld, hipStream_t s) {
  const int64_t n = (int64_t)nI * ld;
  if (n > 0)
    hipLaunchKernelGGL(k_rhs_sketch, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rp, col, ii_end, A, f, nI, T,
                       l, F, ld);
}

// F (nI x ld) = [KW ; 0]: the first nV rows take KW's first c columns (KW: nV x 64), the
// rest is zero.
__global__ void k_rhs_rows(const double* __restrict__ KW, int nV, int c, int nI, double* __restrict__ F, int ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nI * ld) return;
  const int r = (int)(i / ld), j = (int)(i % ld);
  F[i] = (r < nV && j < c) ? KW[(int64_t)r * 64 + j] : 0.0;
}
void launch_rhs_rows(const double* KW, int nV, int c, int nI, double* F, int ld, hipStream_t s) {
  const int64_t n = (int64_t)nI * ld;
  if (n > 0) hipLaunchKernelGGL(k_rhs_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, KW, nV, c, nI, F, ld);
}

// P (MP x 64) = A_BI X: row b of P is the B row nI + b of the local CSR times the I rows of X
// (nI x ldx), columns j < c; rows b >= nB and columns j >= c are zero.
__global__ void k_bi_product(const int* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ A,
                             int nI, int nB, int MP, const double* __restrict__ X, int ldx, int c, double* __restrict__ P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)MP * 64) return;
  const int b = (int)(i >> 6), j = (int)(i & 63);
  double v = 0.0;
  if (b < nB && j < c) {
    const int r = nI + b;
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
      const int cc = col[e];
      if (cc < nI) v += A[e] * X[(int64_t)cc * ldx + j];
    }
  }
  P[i] = v;
}
void launch_bi_product(const int* rp, const int* col, const double* A, int nI, int nB, int MP, const double* X, int ldx,
                       int c, double* P, hipStream_t s) {
  const int64_t n = (int64_t)MP * 64;
  hipLaunchKernelGGL(k_bi_product, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rp, col, A, nI, nB, MP, X, ldx,
                     c, P);
}

// Whitening of an eigendecomposition (V: s x s row-major, eigenvalues th descending):
// out (s x 64, ld 64) = V[:, :r] diag(th^-1/2), zero columns from r on.
__global__ void k_whiten(const double* __restrict__ V, const double* __restrict__ th, int s, int r,
                         double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s * 64) return;
  const int a = i >> 6, j = i & 63;
  out[i] = (j < r) ? V[a * s + j] / sqrt(th[j]) : 0.0;
}
void launch_whiten(const double* V, const double* th, int s, int r, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_whiten, dim3((s * 64 + 255) / 256), dim3(256), 0, st, V, th, s, r, out);
}

// ------------------------------------------------------------------------ split-precision Gram
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  const __bf16 b = (__bf16)x;   // round to nearest even
  return __builtin_bit_cast(uint16_t, b);
}
__device__ __forceinline__ float bf16_value(uint16_t u) {
  return __builtin_bit_cast(float, (uint32_t)u << 16);
}

// x = hi + lo with hi = bf16(x), lo = bf16(x - hi): a 16-bit significand in two halves.  One
// workgroup transposes a 64 x 64 block through LDS (reads along m, writes along k).
__global__ __launch_bounds__(256) void k_split_bf16(const SplitDesc* __restrict__ ds, const int4* __restrict__ tiles) {
  __shared__ uint16_t hs[64][66], ls[64][66];
  const int4 tl = tiles[blockIdx.x];
  const SplitDesc& d = ds[tl.x];
  const int a0 = tl.y * 64, v0 = tl.z * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int v = v0 + r, a = a0 + tx;
    const double x = (v < d.k && a < d.m) ? d.X[(int64_t)v * d.ldx + a] : 0.0;
    const uint16_t h = bf16_bits((float)x);
    hs[r][tx] = h;
    ls[r][tx] = bf16_bits((float)(x - (double)bf16_value(h)));
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {   // output row a0 + r, columns v0 + tx
    const int64_t o = (int64_t)(a0 + r) * d.kp + v0 + tx;
    d.hi[o] = hs[tx][r];
    d.lo[o] = ls[tx][r];
  }
}
void launch_split_bf16(const SplitDesc* d, const int4* tiles, int ntiles, hipStream_t s) {
  if (ntiles > 0) hipLaunchKernelGGL(k_split_bf16, dim3(ntiles), dim3(256), 0, s, d, tiles);
}

// C = A^T B on v_mfma_f32_16x16x32_bf16.  A workgroup owns a 128 x 128 block of C (ti <= tj)
// and each wave a 64 x 64 quarter (4 x 4 MFMA tiles).  Per 32-deep k step the workgroup stages
// the four operand tiles (A hi/lo, B hi/lo: 128 rows x 32 k each) in LDS, rows padded to 40
// elements against bank conflicts, while the next step's tiles load into registers; each wave
// then reads 16 fragments of 16 bytes and issues 48 MFMAs (three products per tile: hi x hi,
// hi x lo, lo x hi; lo x lo is below the FP32 accumulation error).  Operand layout (gfx950):
// lane l feeds row l % 16 with k = 8 (l / 16) .. + 7; accumulator element r is row
// 4 (l / 16) + r, column l % 16.
constexpr int kBfRow = 40;   // padded LDS row (bf16 elements) of a 32-deep operand tile
__global__ __launch_bounds__(256) void k_gram_bf16(const BfGramDesc* __restrict__ ds, const int4* __restrict__ tiles) {
  __shared__ __attribute__((aligned(16))) uint16_t sm[4][128 * kBfRow];   // A hi, A lo, B hi, B lo
  const int4 tl = tiles[blockIdx.x];
  const BfGramDesc& d = ds[tl.x];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int I0 = tl.y * 128, J0 = tl.z * 128;
  const uint16_t* src[4] = {d.Ahi + (int64_t)I0 * d.kp, d.Alo + (int64_t)I0 * d.kp, d.Bhi + (int64_t)J0 * d.kp,
                            d.Blo + (int64_t)J0 * d.kp};
  // staging: each operand tile is 128 rows x 64 bytes = 512 chunks of 16 bytes, 2 per thread
  const int r0 = tid >> 2, q0 = (tid & 3) * 8;   // chunks (row r0, k q0) and (row r0 + 64, k q0)
  u32x4 nx[4][2];
  auto load = [&](int v0) {
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        nx[o][h] = *((const MOR_GLOBAL u32x4*)(src[o] + (int64_t)(r0 + 64 * h) * d.kp + v0 + q0));
  };
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  const int kq = 8 * (lane >> 4), rl = lane & 15;
  load(0);
  for (int v0 = 0; v0 < d.kp; v0 += 32) {
    __syncthreads();   // the previous step is done with the LDS tiles
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int h = 0; h < 2; ++h) *reinterpret_cast<u32x4*>(&sm[o][(r0 + 64 * h) * kBfRow + q0]) = nx[o][h];
    __syncthreads();
    if (v0 + 32 < d.kp) load(v0 + 32);
    bf16x8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ra = (wr * 64 + t * 16 + rl) * kBfRow + kq, rb = (wc * 64 + t * 16 + rl) * kBfRow + kq;
      ah[t] = *reinterpret_cast<const bf16x8*>(&sm[0][ra]);
      al[t] = *reinterpret_cast<const bf16x8*>(&sm[1][ra]);
      bh[t] = *reinterpret_cast<const bf16x8*>(&sm[2][rb]);
      bl[t] = *reinterpret_cast<const bf16x8*>(&sm[3][rb]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
      }
  }
  const bool diag = tl.y == tl.z;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I0 + wr * 64 + a * 16 + 4 * (lane >> 4) + r;
        const int j = J0 + wc * 64 + b * 16 + rl;
        if (i < d.m && j < d.m && (!diag || i <= j)) {
          const double v = (double)acc[a][b][r];
          d.C[(int64_t)i * d.ldc + j] = v;
          d.C[(int64_t)j * d.ldc + i] = v;
        }
      }
}
void launch_gram_bf16(const BfGramDesc* d, const int4* tiles, int ntiles, hipStream_t s) {
  if (ntiles > 0) hipLaunchKernelGGL(k_gram_bf16, dim3(ntiles), dim3(256), 0, s, d, tiles);
}

// --------------------------------------------------------------------------------- FP32 MFMA GEMM
// k_gemm's contract (FP64 operands and result, the same descriptors and tile lists) computed on
// the FP32 matrix cores: operands rounded to FP32 as they are staged in LDS, FP32 accumulation,
// C = alpha acc + beta C in FP64.  For the coarse correction of the FP32 block CG, whose vectors
// are FP32 anyway.  v_mfma_f32_16x16x4f32 takes A and B with k-major lanes as the FP64 tile
// does, but returns D with lane -> col lane%16, register r -> row 4 (lane/16) + r.
constexpr int kLdsPad32 = 68;

template <bool TA, bool TB>
__device__ void gemm32_tile_body(const GemmDesc& g, int ti, int tj, float (*As)[kLdsPad32], float (*Bs)[kLdsPad32],
                                 int use_skip) {
  if (gemm_tile_skipped(g, tj, use_skip)) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int i0 = ti * 64, j0 = tj * 64;
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  double ra[4], rb[4];
  if (g.k > 0) tile_fetch<TA, TB>(g.A, g.lda, g.B, g.ldb, g.m, g.n, i0, j0, 0, g.k, ra, rb);
  for (int k0 = 0; k0 < g.k; k0 += 16) {
    if (!TA) {
      const int i = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[kk + q][i] = (float)ra[q];
    } else {
      const int kk = tid >> 4, i = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[kk][i + q] = (float)ra[q];
    }
    if (!TB) {
      const int kk = tid >> 4, j = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[kk][j + q] = (float)rb[q];
    } else {
      const int j = tid >> 2, kk = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[kk + q][j] = (float)rb[q];
    }
    __syncthreads();
    if (k0 + 16 < g.k) tile_fetch<TA, TB>(g.A, g.lda, g.B, g.ldb, g.m, g.n, i0, j0, k0 + 16, g.k, ra, rb);
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int kr = s4 * 4 + (lane >> 4);
      const float a0 = As[kr][wr * 32 + (lane & 15)];
      const float a1 = As[kr][wr * 32 + 16 + (lane & 15)];
      const float b0 = Bs[kr][wc * 32 + (lane & 15)];
      const float b1 = Bs[kr][wc * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + 4 * (lane >> 4) + r;
        const int j = j0 + wc * 32 + b * 16 + (lane & 15);
        if (i < g.m && j < g.n) {
          double* p = g.C + (int64_t)i * g.ldc + j;
          const double v = g.alpha * (double)acc[a][b][r];
          *p = (g.beta == 0.0) ? v : v + g.beta * *p;
        }
      }
}

__global__ __launch_bounds__(256) void k_gemm32(const GemmDesc* __restrict__ descs, const int4* __restrict__ tiles,
                                                int use_skip) {
  __shared__ float As[16][kLdsPad32], Bs[16][kLdsPad32];
  const int4 tl = tiles[blockIdx.x];
  const GemmDesc& g = descs[tl.x];
  if (!g.ta && !g.tb) gemm32_tile_body<false, false>(g, tl.y, tl.z, As, Bs, use_skip);
  else if (g.ta && !g.tb) gemm32_tile_body<true, false>(g, tl.y, tl.z, As, Bs, use_skip);
  else if (!g.ta && g.tb) gemm32_tile_body<false, true>(g, tl.y, tl.z, As, Bs, use_skip);
  else gemm32_tile_body<true, true>(g, tl.y, tl.z, As, Bs, use_skip);
}
void launch_gemm32(const GemmDesc* d, const int4* tiles, int ntiles, hipStream_t s, int use_skip) {
  if (ntiles > 0) hipLaunchKernelGGL(k_gemm32, dim3(ntiles), dim3(256), 0, s, d, tiles, use_skip);
}

// --------------------------------------------------------------------------------- Cholesky
// Right-looking blocked Cholesky S = R^T R (R upper) of every subdomain's padded S_B.
__global__ __launch_bounds__(256) void k_potrf_diag(const DenseSub* __restrict__ ds, int p) {
  const DenseSub& d = ds[blockIdx.x];
  if (p >= d.T) return;
  __shared__ double A[64][65];
  __shared__ double Ri[64][65];
  __shared__ int bad;
  const int tid = threadIdx.x;
  double* S = d.S + (int64_t)(p * 64) * d.MP + p * 64;
  for (int i = tid; i < 64 * 64; i += 256) {
    const int r = i >> 6, c = i & 63;
    A[r][c] = (r <= c) ? S[(int64_t)r * d.MP + c] : 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < 64; ++j) {
    if (tid == 0) {
      double v = A[j][j];
      if (!(v > 0.0)) {
        if (!bad) bad = p * 64 + j + 1;
        v = 1.0;
      }
      A[j][j] = sqrt(v);
    }
    __syncthreads();
    const double dj = A[j][j];
    for (int l = j + 1 + tid; l < 64; l += 256) A[j][l] /= dj;
    __syncthreads();
    const int rem = 63 - j;
    for (int idx = tid; idx < rem * rem; idx += 256) {
      const int i = j + 1 + idx / rem, l = j + 1 + idx % rem;
      if (i <= l) A[i][l] -= A[j][i] * A[j][l];
    }
    __syncthreads();
  }
  // inverse of the upper triangular R_pp, one column per thread
  if (tid < 64) {
    const int c = tid;
    for (int i = 0; i < 64; ++i) Ri[i][c] = 0.0;
    Ri[c][c] = 1.0 / A[c][c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= c; ++l) s += A[i][l] * Ri[l][c];
      Ri[i][c] = -s / A[i][i];
    }
  }
  __syncthreads();
  double* Di = d.Dinv + (int64_t)p * 64 * 64;
  for (int i = tid; i < 64 * 64; i += 256) {
    const int r = i >> 6, c = i & 63;
    S[(int64_t)r * d.MP + c] = A[r][c];
    Di[i] = Ri[r][c];
  }
  if (tid == 0 && bad && d.info[0] == 0) d.info[0] = bad;
}
void launch_potrf_diag(const DenseSub* d, int nsub, int p, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf_diag, dim3(nsub), dim3(256), 0, s, d, p);
}

// R_{p,j} = R_pp^{-T} S_{p,j} for j > p
__global__ __launch_bounds__(256) void k_chol_panel(const DenseSub* __restrict__ ds, int p) {
  __shared__ double As[16][kLdsPad], Bs[16][kLdsPad];
  const DenseSub& d = ds[blockIdx.y];
  const int j = p + 1 + blockIdx.x;
  if (j >= d.T) return;
  d4 acc[2][2];
  tile_zero(acc);
  double* Spj = d.S + (int64_t)(p * 64) * d.MP + j * 64;
  const double* Di = d.Dinv + (int64_t)p * 64 * 64;
  tile_mma<true, false>(Di, 64, Spj, d.MP, 64, 64, 0, 0, 0, 64, As, Bs, acc);
  tile_store(Spj, d.MP, 64, 64, 0, 0, 1.0, 0.0, acc);
}
void launch_chol_panel(const DenseSub* d, int nsub, int p, int tmax, hipStream_t s) {
  const int nt = tmax - p - 1;
  if (nt > 0) hipLaunchKernelGGL(k_chol_panel, dim3(nt, nsub), dim3(256), 0, s, d, p);
}

// S_{i,j} -= R_{p,i}^T R_{p,j} for p < i <= j
__global__ __launch_bounds__(256) void k_chol_syrk(const DenseSub* __restrict__ ds, int p, int nt) {
  __shared__ double As[16][kLdsPad], Bs[16][kLdsPad];
  const DenseSub& d = ds[blockIdx.y];
  const int a = blockIdx.x / nt, b = blockIdx.x % nt;
  if (a > b) return;
  const int i = p + 1 + a, j = p + 1 + b;
  if (j >= d.T) return;
  d4 acc[2][2];
  tile_zero(acc);
  const double* Rpi = d.S + (int64_t)(p * 64) * d.MP + i * 64;
  const double* Rpj = d.S + (int64_t)(p * 64) * d.MP + j * 64;
  tile_mma<true, false>(Rpi, d.MP, Rpj, d.MP, 64, 64, 0, 0, 0, 64, As, Bs, acc);
  double* Sij = d.S + (int64_t)(i * 64) * d.MP + j * 64;
  tile_store(Sij, d.MP, 64, 64, 0, 0, -1.0, 1.0, acc);
}
void launch_chol_syrk(const DenseSub* d, int nsub, int p, int tmax, hipStream_t s) {
  const int nt = tmax - p - 1;
  if (nt > 0) hipLaunchKernelGGL(k_chol_syrk, dim3(nt * nt, nsub), dim3(256), 0, s, d, p, nt);
}

// Forward substitution R^T X = B, left-looking per 64-column tile (workgroup = column tile),
// over the panels [p0, min(p1, T)): X_p = R_pp^{-T} (B_p - sum_{p0<=q<p} R_{q,p}^T X_q).  With
// p0 = 0 and p1 >= T this is the whole solve; a blocked solve passes one diagonal block at a time
// (B = X, in place) and applies the panels before it as a GEMM update.
__global__ __launch_bounds__(256) void k_trsm_lt(const DenseSub* __restrict__ ds, const TrsmDesc* __restrict__ tds,
                                                 int p0, int p1) {
  __shared__ double As[16][kLdsPad], Bs[16][kLdsPad];
  const DenseSub& d = ds[blockIdx.y];
  const TrsmDesc& td = tds[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= td.ncol_tiles) return;
  const int MP = d.MP;
  const double* Bm = td.B;
  double* X = td.X;
  const int ldb = td.ldb, ldx = td.ldx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  const int pe = min(p1, d.T);
  for (int p = p0; p < pe; ++p) {
    d4 acc[2][2];
    tile_zero(acc);
    // sum_{p0<=q<p} R_{q,p}^T X_{q,c}: A(i,k) = R[k][p*64+i], B(k,j) = X[k][c*64+j], 64 p0 <= k < 64p
    tile_mma<true, false>(d.S + p * 64, MP, X + c * 64, ldx, 64, 64, 0, 0, p0 * 64, p * 64, As, Bs, acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = p * 64 + wr * 32 + a * 16 + (lane >> 4) + 4 * r;
          const int j = c * 64 + wc * 32 + b * 16 + (lane & 15);
          const double bv = td.tb ? Bm[(int64_t)j * ldb + i] : Bm[(int64_t)i * ldb + j];
          X[(int64_t)i * ldx + j] = bv - acc[a][b][r];
        }
    __syncthreads();
    tile_zero(acc);
    tile_mma<true, false>(d.Dinv + (int64_t)p * 4096, 64, X + (int64_t)(p * 64) * ldx + c * 64, ldx, 64, 64, 0, 0, 0,
                          64, As, Bs, acc);
    tile_store(X + (int64_t)(p * 64) * ldx + c * 64, ldx, 64, 64, 0, 0, 1.0, 0.0, acc);
    __syncthreads();
  }
}
void launch_trsm_lt(const DenseSub* d, const TrsmDesc* td, int nsub, int max_col_tiles, hipStream_t s, int p0, int p1) {
  hipLaunchKernelGGL(k_trsm_lt, dim3(max_col_tiles, nsub), dim3(256), 0, s, d, td, p0, p1);
}

// B[r][j] = U[r][j] / sigma_j for j < k, 0 for k <= j < 64 (B: rows x 64)
__global__ void k_scale_cols(const double* U, int ldu, const double* sigma, int k, int rows, double* B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows * 64) return;
  const int r = (int)(i >> 6), j = (int)(i & 63);
  B[i] = (j < k) ? U[(int64_t)r * ldu + j] / sigma[j] : 0.0;
}
void launch_scale_cols(const double* U, int ldu, const double* sigma, int k, int rows, double* B, hipStream_t s) {
  const int64_t n = (int64_t)rows * 64;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, U, ldu, sigma, k, rows, B);
}

// Back substitution R X = B for one 64-column tile over the panels [p0, min(p1, T)), last
// first: X_p = R_pp^-1 (B_p - sum_{p<q<min(p1,T)} R_{p,q} X_q); B, X: MP x 64 (ld 64).  The
// blocked solve passes one diagonal block at a time, in place.
__global__ __launch_bounds__(256) void k_trsm_un(const DenseSub* __restrict__ ds, double* const* Bs_, double* const* Xs_,
                                                 int p0, int p1) {
  __shared__ double As[16][kLdsPad], Bs[16][kLdsPad];
  const int slot = blockIdx.x;
  const DenseSub& d = ds[slot];
  const double* Bm = Bs_[slot];
  double* X = Xs_[slot];
  const int MP = d.MP;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wr = w >> 1, wc = w & 1;
  const int pe = min(p1, d.T);
  for (int p = pe - 1; p >= p0; --p) {
    d4 acc[2][2];
    tile_zero(acc);
    // sum_{p<q<pe} R_{p,q} X_q : A(i,k) = R[p*64+i][k], k in [(p+1)*64, 64 pe)
    tile_mma<false, false>(d.S + (int64_t)(p * 64) * MP, MP, X, 64, 64, 64, 0, 0, (p + 1) * 64, pe * 64, As, Bs, acc);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = p * 64 + wr * 32 + a * 16 + (lane >> 4) + 4 * r;
          const int j = wc * 32 + b * 16 + (lane & 15);
          X[(int64_t)i * 64 + j] = Bm[(int64_t)i * 64 + j] - acc[a][b][r];
        }
    __syncthreads();
    tile_zero(acc);
    tile_mma<false, false>(d.Dinv + (int64_t)p * 4096, 64, X + (int64_t)(p * 64) * 64, 64, 64, 64, 0, 0, 0, 64, As, Bs,
                           acc);
    tile_store(X + (int64_t)(p * 64) * 64, 64, 64, 64, 0, 0, 1.0, 0.0, acc);
    __syncthreads();
  }
}
void launch_trsm_un(const DenseSub* d, int nsub, double* const* Bs, double* const* Xs, hipStream_t s, int p0, int p1) {
  hipLaunchKernelGGL(k_trsm_un, dim3(nsub), dim3(256), 0, s, d, Bs, Xs, p0, p1);
}

// dst[r][c] = src[r][c] (trans = 0) or src[c][r] (trans = 1) for r < rows, c < cols
__global__ void k_copy_rect(const double* __restrict__ src, int lds, int trans, double* __restrict__ dst, int ldd,
                            int rows, int cols) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / cols), c = (int)(i % cols);
    dst[(int64_t)r * ldd + c] = trans ? src[(int64_t)c * lds + r] : src[(int64_t)r * lds + c];
  }
}
void launch_copy_rect(const double* src, int lds, int trans, double* dst, int ldd, int rows, int cols, hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n <= 0) return;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_copy_rect, dim3(blocks), dim3(256), 0, s, src, lds, trans, dst, ldd, rows, cols);
}

// --------------------------------------------------------------------------------- small eigen
// Cyclic Jacobi on an s x s symmetric matrix (s <= 64) with a round-robin ordering: the s/2
// rotations of a round touch disjoint index pairs and are applied together.
__global__ __launch_bounds__(256) void k_jacobi(double* const* Hs, double* const* Ss, double* const* Ths,
                                                const int* s_of) {
  __shared__ double H[64][65];
  __shared__ double V[64][65];
  __shared__ double cs[32], sn[32];
  __shared__ int pp[32], qq[32];
  __shared__ double red[256];
  __shared__ int perm[64];
  const int slot = blockIdx.x;
  const int s = s_of[slot];
  const int n = s + (s & 1);
  const int tid = threadIdx.x;
  const double* Hg = Hs[slot];
  for (int i = tid; i < 64 * 64; i += 256) {
    const int r = i >> 6, c = i & 63;
    H[r][c] = (r < s && c < s) ? 0.5 * (Hg[r * s + c] + Hg[c * s + r]) : 0.0;
    V[r][c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = tid; i < n * n; i += 256) {
      const int r = i / n, c = i % n;
      const double v = H[r][c] * H[r][c];
      tot += v;
      if (r != c) off += v;
    }
    red[tid] = off;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (tid < st) red[tid] += red[tid + st];
      __syncthreads();
    }
    const double tots = red[0];
    __syncthreads();
    // off-diagonal Frobenius norm below 1e-14 of the whole: the eigenvalues then move by
    // O(off^2 / gap), far below rounding, where a tighter target sits under the rounding noise
    // of the rotations themselves (about n u |H|) and is never met
    if (!(offs > 1e-28 * tots)) break;
    for (int rnd = 0; rnd < n - 1; ++rnd) {
      if (tid < n / 2) {
        int p, q;
        if (tid == 0) { p = rnd; q = n - 1; }
        else { p = (rnd + tid) % (n - 1); q = (rnd - tid + n - 1) % (n - 1); }
        const double hpq = H[p][q];
        double c = 1.0, sv = 0.0;
        if (fabs(hpq) > 1e-300) {
          const double th = (H[q][q] - H[p][p]) / (2.0 * hpq);
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          sv = t * c;
        }
        cs[tid] = c; sn[tid] = sv; pp[tid] = p; qq[tid] = q;
      }
      __syncthreads();
      for (int idx = tid; idx < (n / 2) * n; idx += 256) {
        const int k = idx / n, col = idx % n;
        const int p = pp[k], q = qq[k];
        const double hp = H[p][col], hq = H[q][col];
        H[p][col] = cs[k] * hp - sn[k] * hq;
        H[q][col] = sn[k] * hp + cs[k] * hq;
      }
      __syncthreads();
      for (int idx = tid; idx < (n / 2) * n; idx += 256) {
        const int k = idx / n, row = idx % n;
        const int p = pp[k], q = qq[k];
        const double hp = H[row][p], hq = H[row][q];
        H[row][p] = cs[k] * hp - sn[k] * hq;
        H[row][q] = sn[k] * hp + cs[k] * hq;
        const double vp = V[row][p], vq = V[row][q];
        V[row][p] = cs[k] * vp - sn[k] * vq;
        V[row][q] = sn[k] * vp + cs[k] * vq;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    for (int i = 0; i < s; ++i) perm[i] = i;
    for (int i = 0; i < s; ++i) {
      int best = i;
      for (int j = i + 1; j < s; ++j)
        if (H[perm[j]][perm[j]] > H[perm[best]][perm[best]]) best = j;
      const int tmp = perm[i]; perm[i] = perm[best]; perm[best] = tmp;
    }
  }
  __syncthreads();
  double* Sg = Ss[slot];
  double* th = Ths[slot];
  for (int i = tid; i < s * s; i += 256) {
    const int r = i / s, c = i % s;
    Sg[i] = V[r][perm[c]];
  }
  for (int i = tid; i < s; i += 256) th[i] = H[perm[i]][perm[i]];
}
void launch_jacobi(double* const* H, double* const* Svec, double* const* theta, const int* s_of, int nsub, int smax,
                   hipStream_t s) {
  (void)smax;
  hipLaunchKernelGGL(k_jacobi, dim3(nsub), dim3(256), 0, s, H, Svec, theta, s_of);
}

// Ritz residuals ||C u_j - theta_j u_j||^2 with Z = C V S and U = V S, and the next iterate Z / theta.
__global__ __launch_bounds__(256) void k_ritz(double* const* Zs, double* const* Us, double* const* Vns,
                                              double* const* Ths, double* const* Res, const int* rows, const int* s_of) {
  const int slot = blockIdx.y;
  const int s = s_of[slot], nr = rows[slot];
  const int j = threadIdx.x & 63;
  const int r0 = blockIdx.x * 64;
  if (r0 >= nr || j >= s) return;
  const double th = Ths[slot][j];
  const double sc = fabs(th) > 1e-300 ? 1.0 / th : 1.0;
  const double* Z = Zs[slot];
  const double* U = Us[slot];
  double* Vn = Vns[slot];
  double part = 0.0;
  for (int r = r0 + (threadIdx.x >> 6); r < min(r0 + 64, nr); r += 4) {
    const double z = Z[(int64_t)r * s + j];
    const double e = z - th * U[(int64_t)r * s + j];
    part += e * e;
    Vn[(int64_t)r * s + j] = z * sc;
  }
  unsafeAtomicAdd(&Res[slot][j], part);
}
void launch_ritz(double* const* Z, double* const* U, double* const* Vn, double* const* theta, double* const* resid,
                 const int* rows, const int* s_of, int nsub, int maxrows, int smax, hipStream_t s) {
  (void)smax;
  hipLaunchKernelGGL(k_ritz, dim3((maxrows + 63) / 64, nsub), dim3(256), 0, s, Z, U, Vn, theta, resid, rows, s_of);
}

// G = R^T R (s x s, upper R), Rinv = R^-1; a zero or negative pivot flags info.
__global__ __launch_bounds__(256) void k_cholinv_small(double* const* Gs, double* const* Ris, const int* s_of, int* info) {
  __shared__ double A[64][65];
  __shared__ double Ri[64][65];
  const int slot = blockIdx.x;
  const int s = s_of[slot], tid = threadIdx.x;
  const double* G = Gs[slot];
  for (int i = tid; i < s * s; i += 256) {
    const int r = i / s, c = i % s;
    A[r][c] = 0.5 * (G[r * s + c] + G[c * s + r]);
  }
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    if (tid == 0) {
      double v = A[j][j];
      if (!(v > 0.0)) {
        if (info) info[slot] = j + 1;
        v = 1.0;
      }
      A[j][j] = sqrt(v);
    }
    __syncthreads();
    for (int l = j + 1 + tid; l < s; l += 256) A[j][l] /= A[j][j];
    __syncthreads();
    const int rem = s - 1 - j;
    for (int idx = tid; idx < rem * rem; idx += 256) {
      const int i = j + 1 + idx / rem, l = j + 1 + idx % rem;
      if (i <= l) A[i][l] -= A[j][i] * A[j][l];
    }
    __syncthreads();
  }
  if (tid < s) {
    const int c = tid;
    for (int i = 0; i < s; ++i) Ri[i][c] = 0.0;
    Ri[c][c] = 1.0 / A[c][c];
    for (int i = c - 1; i >= 0; --i) {
      double sum = 0.0;
      for (int l = i + 1; l <= c; ++l) sum += A[i][l] * Ri[l][c];
      Ri[i][c] = -sum / A[i][i];
    }
  }
  __syncthreads();
  double* R = Ris[slot];
  for (int i = tid; i < s * s; i += 256) R[i] = Ri[i / s][i % s];
}
void launch_cholinv_small(double* const* G, double* const* Rinv, const int* s_of, int nsub, int smax, int* info,
                          hipStream_t s) {
  (void)smax;
  hipLaunchKernelGGL(k_cholinv_small, dim3(nsub), dim3(256), 0, s, G, Rinv, s_of, info);
}

// deterministic start block: an integer hash mapped to (-1, 1) on rows < M, zero on padding rows
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}
__global__ void k_random_init(double* const* Vs, const int* rows, const int* M_of, const int* s_of, uint32_t seed) {
  const int slot = blockIdx.y;
  const int s = s_of[slot], nr = rows[slot], M = M_of[slot];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nr * s) return;
  const int r = (int)(i / s), c = (int)(i % s);
  double v = 0.0;
  if (r < M) {
    const uint32_t h = hash32(seed ^ hash32((uint32_t)r * 2654435761U + (uint32_t)c * 40503U + 12345U));
    v = ((double)h + 0.5) * (2.0 / 4294967296.0) - 1.0;
  }
  Vs[slot][i] = v;
}
void launch_random_init(double* const* V, const int* rows, const int* M_of, const int* s_of, int nsub, int maxrows,
                        int smax, uint32_t seed, hipStream_t s) {
  const int64_t n = (int64_t)maxrows * smax;
  hipLaunchKernelGGL(k_random_init, dim3((unsigned)((n + 255) / 256), nsub), dim3(256), 0, s, V, rows, M_of, s_of, seed);
}

// --------------------------------------------------------------------------------- projection
__global__ void k_copy_col(const double* src, int lds, double* dst, int ldd, int rows) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < rows) dst[(int64_t)r * ldd] = src[(int64_t)r * lds];
}
void launch_copy_col(const double* src, int lds, double* dst, int ldd, int rows, hipStream_t s) {
  if (rows > 0) hipLaunchKernelGGL(k_copy_col, dim3((rows + 255) / 256), dim3(256), 0, s, src, lds, dst, ldd, rows);
}

// Off-diagonal block of Q^T A Q for a neighbour pair (i, j): sum over the A_0 entries that
// couple P_i and P_j of a * V_i[p, :]^T V_j[q, :].  Writes the block and its transpose.
__global__ __launch_bounds__(256) void k_pair_project(const int4* __restrict__ range, const int* __restrict__ trip,
                                                      const double* __restrict__ A0, double* const* Vs,
                                                      const int* __restrict__ ldv, const int* __restrict__ k1,
                                                      const PairOut* __restrict__ outs, double* out) {
  const int4 pr = range[blockIdx.x];   // (i, j, first triplet, count)
  const int i = pr.x, j = pr.y;
  const int ki = k1[i], kj = k1[j];
  const double* Vi = Vs[i];
  const double* Vj = Vs[j];
  const int li = ldv[i], lj = ldv[j];
  const PairOut po = outs[blockIdx.x];
  for (int o = threadIdx.x; o < ki * kj; o += 256) {
    const int a = o / kj, b = o % kj;
    double acc = 0.0;
    for (int t = pr.z; t < pr.z + pr.w; ++t) {
      const int p = trip[3 * t], q = trip[3 * t + 1], sl = trip[3 * t + 2];
      acc += A0[sl] * Vi[(int64_t)p * li + a] * Vj[(int64_t)q * lj + b];
    }
    out[po.base_ij + (int64_t)a * po.ld_i + b] = acc;
    out[po.base_ji + (int64_t)b * po.ld_j + a] = acc;
  }
}
void launch_pair_project(const int4* trip_range, const int* trip, const double* A0, double* const* Vi, const int* ldv,
                         const int* k1, const PairOut* outs, double* out, int npairs, hipStream_t s) {
  if (npairs > 0)
    hipLaunchKernelGGL(k_pair_project, dim3(npairs), dim3(256), 0, s, trip_range, trip, A0, Vi, ldv, k1, outs, out);
}

// A_ii of a [A_ii | b_i] block (k1 x (k1+1), ld) into the reduced system, symmetrised
__global__ void k_scatter_block(const double* B, int k1, int ld, double* out, int64_t base, int64_t ldo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k1 * k1) return;
  const int a = i / k1, b = i % k1;
  out[base + a * ldo + b] = 0.5 * (B[a * ld + b] + B[b * ld + a]);
}
void launch_scatter_block(const double* B, int k1, int ld, double* out, int64_t base, int64_t ldo, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_block, dim3((k1 * k1 + 255) / 256), dim3(256), 0, s, B, k1, ld, out, base, ldo);
}

// ---- the reduced solve by conjugate gradients with the diagonal preconditioner (Section 6,
// step 3).  One iteration is three launches: q = A~ p with p'q; the x, r, z updates with r'z
// and r'r; the new direction.  The scalars of iteration `it` live in slot it % 3 of each ring, so
// a slot is cleared two launches before it is summed into and is never cleared while read.
// Every launch first reads the stop flag: once converged (or failed) the remaining launches of
// a chunk return at once, and x keeps the converged iterate.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ bool rpcg_stopped(const RpcgDev& d) {
  return __atomic_load_n(d.state, __ATOMIC_RELAXED) != 0;
}
// sum of one value per thread over the workgroup (256 threads), added to *dst by thread 0
__device__ __forceinline__ void block_add(double v, double* dst, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) unsafeAtomicAdd(dst, red[0] + red[1] + red[2] + red[3]);
}

// x = 0, r = b, z = D^-1 b, p = z, r'z into rz[2] (the slot "before iteration 0"), b'b into rr0
__global__ __launch_bounds__(256) void k_rpcg_init(const RpcgDev d, int n) {
  __shared__ double red[2][4];
  double rz = 0.0, rr = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const double a = d.val[d.rs[i] + d.rdiag[i]];
    if (!(a > 0.0)) atomicMax(d.state + 2, 2);
    const double di = a > 0.0 ? 1.0 / a : 0.0;
    const double bi = d.b[(int64_t)i * d.bstride];
    d.dinv[i] = di;
    d.x[i] = 0.0;
    d.r[i] = bi;
    if (!d.block) {   // the block preconditioner's z, p and r'z come from k_rpcg_prec
      d.z[i] = di * bi;
      d.p[i] = di * bi;
      rz += bi * di * bi;
    }
    rr += bi * bi;
  }
  block_add(rz, d.sc + 3 + 2, red[0]);
  block_add(rr, d.sc + 9, red[1]);
}

__global__ __launch_bounds__(256) void k_rpcg_matvec(const RpcgDev d, int n, int it) {
  __shared__ double red[4];
  if (rpcg_stopped(d)) return;
  const int c = it % 3;
  if (blockIdx.x == 0 && threadIdx.x == 0) {   // this iteration's r'z and r'r slots
    d.sc[3 + c] = 0.0;
    d.sc[6 + c] = 0.0;
  }
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);   // one wave per reduced row
  double part = 0.0;
  if (row < n) {
    const double* a = d.val + d.rs[row];
    const int2 wc = d.rwc[row];
    const int* cc = d.ccol + wc.y;
    double acc = 0.0;
    for (int k = lane; k < wc.x; k += 64) acc += a[k] * d.p[cc[k]];
    acc = wave_sum(acc);
    if (lane == 0) {
      d.q[row] = acc;
      part = acc * d.p[row];
    }
  }
  if (lane == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) unsafeAtomicAdd(d.sc + c, red[0] + red[1] + red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_rpcg_update(const RpcgDev d, int n, int it) {
  __shared__ double red[2][4];
  if (rpcg_stopped(d)) return;
  const int c = it % 3, pv = (it + 2) % 3;
  const double pq = d.sc[c];
  if (!(pq > 0.0)) {   // the same decision in every workgroup: A~ is not positive definite
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      d.state[2] = 1;
      __atomic_store_n(d.state, 1, __ATOMIC_RELAXED);
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) d.sc[(it + 1) % 3] = 0.0;   // next iteration's p'q slot
  const double al = d.sc[3 + pv] / pq;
  double rz = 0.0, rr = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    d.x[i] += al * d.p[i];
    const double ri = d.r[i] - al * d.q[i];
    d.r[i] = ri;
    if (!d.block) {   // block preconditioner: z and r'z in k_rpcg_prec
      const double zi = d.dinv[i] * ri;
      d.z[i] = zi;
      rz += ri * zi;
    }
    rr += ri * ri;
  }
  block_add(rz, d.sc + 3 + c, red[0]);
  block_add(rr, d.sc + 6 + c, red[1]);
}

__global__ __launch_bounds__(256) void k_rpcg_direction(const RpcgDev d, int n, int it, double tol2) {
  if (rpcg_stopped(d)) return;
  const int c = it % 3, pv = (it + 2) % 3;
  const bool first = blockIdx.x == 0 && threadIdx.x == 0;
  // converged: x is final.  Diagonal preconditioner: ||r|| <= rtol ||b||; block preconditioner:
  // the updated system's residual, r'M^-1 r <= rtol^2 b'M^-1 b
  const bool done = d.block ? d.sc[3 + c] <= tol2 * d.sc[10] : d.sc[6 + c] <= tol2 * d.sc[9];
  if (done) {
    if (first) {
      d.state[1] = it + 1;
      __atomic_store_n(d.state, 1, __ATOMIC_RELAXED);
    }
    return;
  }
  const double be = d.sc[3 + c] / d.sc[3 + pv];
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) d.p[i] = d.z[i] + be * d.p[i];
  if (first) d.state[1] = it + 1;
}

// z = M^-1 r with the block pseudo-inverses (each row: its block row times r over the block),
// r'z into sc[slot]; at the start also p = z
__global__ __launch_bounds__(256) void k_rpcg_prec(const RpcgDev d, int n, int slot, int set_p) {
  __shared__ double red[2][4];
  if (rpcg_stopped(d)) return;
  double part = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const int2 bd = d.rbd[i];
    const double* m = d.bmv + d.rbm[i];
    const double* rb = d.r + bd.x;
    double z = 0.0;
    for (int b = 0; b < bd.y; ++b) z += m[b] * rb[b];
    d.z[i] = z;
    if (set_p) d.p[i] = z;
    part += d.r[i] * z;
  }
  block_add(part, d.sc + slot, red[0]);
  if (set_p) block_add(part, d.sc + 10, red[1]);   // b'M^-1 b: the reference of the stopping test
}

// pseudo-inverse of each block from its eigendecomposition, one workgroup per block
__global__ __launch_bounds__(256) void k_block_pinv(double* const* Ss, double* const* Ths, const int* s_of,
                                                    const double* drops, double* const* Outs) {
  const int blk = blockIdx.x;
  const int s = s_of[blk];
  const double* S = Ss[blk];
  const double* th = Ths[blk];
  double* out = Outs[blk];
  const double thr = drops[blk] * th[0];
  for (int idx = threadIdx.x; idx < s * s; idx += 256) {
    const int a = idx / s, b = idx % s;
    double acc = 0.0;
    for (int j = 0; j < s; ++j)
      if (th[j] > thr && th[j] > 0.0) acc += S[a * s + j] * S[b * s + j] / th[j];
    out[idx] = acc;
  }
}
void launch_block_pinv(double* const* S, double* const* th, const int* s_of, int n, const double* drops,
                       double* const* out, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_block_pinv, dim3(n), dim3(256), 0, s, S, th, s_of, drops, out);
}

static int rpcg_grid(int n) { return std::max(1, std::min((n + 255) / 256, 1024)); }

void launch_rpcg_setup(const RpcgDev& d, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, s, d.sc, (int64_t)16, 0.0);
  hipLaunchKernelGGL(k_fill_i, dim3(1), dim3(256), 0, s, d.state, (int64_t)4, 0);
  hipLaunchKernelGGL(k_rpcg_init, dim3(rpcg_grid(n)), dim3(256), 0, s, d, n);
  if (d.block) hipLaunchKernelGGL(k_rpcg_prec, dim3(rpcg_grid(n)), dim3(256), 0, s, d, n, 3 + 2, 1);
}
void launch_rpcg_iteration(const RpcgDev& d, int n, int it, double tol2, hipStream_t s) {
  hipLaunchKernelGGL(k_rpcg_matvec, dim3((n + 3) / 4), dim3(256), 0, s, d, n, it);
  hipLaunchKernelGGL(k_rpcg_update, dim3(rpcg_grid(n)), dim3(256), 0, s, d, n, it);
  if (d.block) hipLaunchKernelGGL(k_rpcg_prec, dim3(rpcg_grid(n)), dim3(256), 0, s, d, n, 3 + it % 3, 0);
  hipLaunchKernelGGL(k_rpcg_direction, dim3(rpcg_grid(n)), dim3(256), 0, s, d, n, it, tol2);
}

// u~ at the owned nodes of one subdomain: u[node(p)] = V[p, :] . x_i
__global__ void k_reconstruct(const double* V, int nP, int k1, const double* x, const int* nodes, double* u) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  double acc = 0.0;
  for (int a = 0; a < k1; ++a) acc += V[(int64_t)p * k1 + a] * x[a];
  u[nodes[p]] = acc;
}
void launch_reconstruct(const double* V, int nP, int k1, const double* x, const int* nodes, double* u, hipStream_t s) {
  if (nP > 0) hipLaunchKernelGGL(k_reconstruct, dim3((nP + 255) / 256), dim3(256), 0, s, V, nP, k1, x, nodes, u);
}

}  // namespace mor
