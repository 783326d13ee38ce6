// C-ABI and device orchestration of the localized model-order-reduction hot path.
//
// mor_create            Section 6 step 1 inputs -> index sets, patterns, colouring (host C++)
// mor_local_basis_batch Section 6 step 2 for a batch of subdomains, on the device:
//   assembly (Section 2, Section 4 H1 matrices) -> block CG lifting (Problems 3.2-3.3) with
//   FP64 refinement -> G1 = Z^T K_i Z and S_B = Schur(H1, B) (Lemmas 4.1-4.2) -> R = chol(S_B),
//   C = R^-T G1 R^-1 -> top singular triplets of R_i Z R^-1 (eq. 4.4) through the eigenpairs of C
//   -> basis Z R^-1 v_j / sigma_j = R_i^-1 u_j, stitched to P_i (Definition 3.1) -> Q_i^T A_ii Q_i
// mor_project           eq. 6.1 block by block with A_0 on omega_0 (Section 6 step 3)
// mor_solve             reduced Cholesky solve, u~ = sum_i S_i Q_i x_i
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <type_traits>
#include <new>
#include <stdexcept>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/mor.h"
#include "mor_host.h"
#include "mor_internal.h"

using namespace mor;

static thread_local std::string g_err;

// Error reporting never throws: the message is dropped if it cannot be stored.
static int fail(int code, const std::string& msg) noexcept {
  try {
    g_err = msg;
  } catch (...) {
    g_err.clear();
  }
  return code;
}
static int fail(int code, const char* msg) noexcept {
  try {
    g_err.assign(msg);
  } catch (...) {
    g_err.clear();
  }
  return code;
}

// The C-ABI boundary: an exception thrown inside an entry point (a host allocation failure from
// a container, or any other) becomes an error code with a message and never crosses into C.
static int exception_code() noexcept {
  try {
    throw;
  } catch (const std::bad_alloc&) {
    return fail(MOR_ENOMEM, "host memory allocation failed");
  } catch (const std::exception& e) {
    int rc = MOR_EDEVICE;
    try {
      g_err = std::string("internal error: ") + e.what();
    } catch (...) {
      rc = fail(MOR_EDEVICE, "internal error");
    }
    return rc;
  } catch (...) {
    return fail(MOR_EDEVICE, "internal error (unknown exception)");
  }
}
#define MOR_TRY try {
#define MOR_CATCH \
  }               \
  catch (...) { return exception_code(); }

#define HIPCHK(expr)                                                                                     \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess)                                                                                \
      return fail(MOR_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_));                  \
  } while (0)

static inline int64_t rup(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

// The eigensolver's subspace holds at most 64 vectors; a truncation must end two inside it.
constexpr int kMaxRank = 62;

namespace {

struct TimerRec {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  int64_t launches = 0;
  double ms = 0.0;
  double work = 0.0;
};

struct SubDev {
  int *rp = nullptr, *col = nullptr, *ii_end = nullptr, *rpV = nullptr, *colV = nullptr, *bp = nullptr;
  int* bpL = nullptr;   // aggregates of all local rows (the K^+ systems of the randomized variant)
  int* rcbL = nullptr;  // their coarse blocks, per local row
  int *ltet = nullptr, *tetg = nullptr, *nodes = nullptr, *htile = nullptr, *halo = nullptr;
  int *hrowp = nullptr, *hpe = nullptr;
  uint16_t *hpp = nullptr, *hself = nullptr;
  uint8_t* core = nullptr;
  int* rcb = nullptr;
  int *smap = nullptr, *spos = nullptr;   // box form of the interior, or nullptr
};

struct SubResult {
  int reduced = 0;
  int k_eff = 0;
  std::vector<double> sigma;
  std::vector<double> Aii, bi;
  int dim = 0;             // basis columns: k_eff + 1, or fewer after the basis update
  int prec = MOR_FP64;     // precision mode the basis was computed in
  double* d_V = nullptr;   // nV x dim
  double* d_Pm = nullptr;  // (k+1) x (k+2): [Q^T A Q | Q^T f]
  int cg_a = 0, cg_k = 0, refine = 0, eig = 0;
};

}  // namespace

struct mor_ctx {
  mor_opts opts;
  int halo_cap = 96;   // LDS SpMM tiling: halo rows per tile (one of kHaloCaps)
  int device = 0;      // HIP device current at mor_create
  hipStream_t st = nullptr;
  HostMesh mesh;
  std::vector<double> kappa, fnodal;
  bool has_f = false;
  std::vector<HostSub> subs;
  std::vector<int64_t> ext_ptr;
  std::vector<int32_t> ext;
  std::vector<uint8_t> in_core;
  std::vector<int32_t> owner, ownpos;
  HostOmega0 om0;
  double *d_xyz = nullptr, *d_kappa = nullptr, *d_f = nullptr;
  int* d_tets = nullptr;
  std::vector<SubDev> sdev;
  SubDev om0dev;
  std::vector<SubResult> res;
  // reduced system
  int64_t n_red = 0, MPr = 0;
  std::vector<int> off;
  double *d_At = nullptr, *d_bt = nullptr, *d_x = nullptr;
  // block-sparse form (reduced_solver 1): row r of A~ is the slab entries val[rs[r] ..+ rwc[r].x)
  // at the global columns ccol[rwc[r].y ..]; rdiag[r] = position of its diagonal entry
  double* d_slab = nullptr;
  int *d_ccol = nullptr, *d_rdiag = nullptr;
  int64_t* d_rs = nullptr;
  int2* d_rwc = nullptr;
  std::vector<int> h_ccol;
  // block preconditioner (reduced_solver 2): pseudo-inverses of the subdomain blocks, per-row maps
  double* d_bmv = nullptr;
  int64_t* d_rbm = nullptr;
  int2* d_rbd = nullptr;
  std::vector<int64_t> h_rs;
  std::vector<int2> h_rwc;
  int64_t slab_len = 0;
  std::vector<double> x_host;
  int projected = 0, solved = 0;
  int solve_iters = 0;
  double solve_relres = 0.0;
  std::vector<void*> allocs;
  bool timing = false;
  std::map<std::string, TimerRec> timers;
  struct MorEngine* eng[2] = {nullptr, nullptr};   // FP32-CG and FP64-CG engines
};

// ------------------------------------------------------------------------------- memory
static void* dalloc(mor_ctx* c, size_t bytes) {
  bytes = (size_t)rup((int64_t)std::max<size_t>(bytes, 256), 256);
  void* p = nullptr;
  if (c->opts.dev_alloc) {
    p = c->opts.dev_alloc(bytes, c->opts.alloc_user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  return p;
}
static void dfree(mor_ctx* c, void* p) {
  if (!p) return;
  if (c->opts.dev_free) c->opts.dev_free(p, c->opts.alloc_user);
  else (void)hipFree(p);
}
// persistent allocation released by mor_destroy
static void* palloc(mor_ctx* c, size_t bytes) {
  void* p = dalloc(c, bytes);
  if (p) c->allocs.push_back(p);
  return p;
}
static void pfree(mor_ctx* c, void* p) {
  if (!p) return;
  auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
  if (it != c->allocs.end()) c->allocs.erase(it);
  dfree(c, p);
}
template <typename T>
static int upload(mor_ctx* c, T** dst, const T* src, size_t n) {
  *dst = (T*)palloc(c, sizeof(T) * std::max<size_t>(n, 1));
  if (!*dst) return fail(MOR_ENOMEM, "device allocation failed");
  if (n) HIPCHK(hipMemcpyAsync(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice, c->st));
  return 0;
}

// A bump allocator over one device block for the transient data of a batch.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  void* take(size_t bytes) {
    const size_t o = (size_t)rup((int64_t)used, 256);
    if (o + bytes > cap) return nullptr;
    used = o + bytes;
    return base + o;
  }
};
struct Sizer {
  size_t total = 0;
  void add(size_t bytes) { total = (size_t)rup((int64_t)total, 256) + bytes; }
};

// ------------------------------------------------------------------------------- timing
struct ScopedTimer {
  mor_ctx* c;
  const char* name;
  double work;
  hipEvent_t a = nullptr, b = nullptr;
  ScopedTimer(mor_ctx* c_, const char* n, double w) : c(c_), name(n), work(w) {
    if (c->timing) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, c->st);
    }
  }
  ~ScopedTimer() {
    if (c->timing) {
      (void)hipEventRecord(b, c->st);
      TimerRec& t = c->timers[name];
      t.ev.emplace_back(a, b);
      t.launches++;
      t.work += work;
    }
  }
};

// Host wall time of an engine phase (including its waits for the device), under its own name.
struct HostTimer {
  mor_ctx* c;
  const char* name;
  std::chrono::steady_clock::time_point t0;
  HostTimer(mor_ctx* c_, const char* n) : c(c_), name(n), t0(std::chrono::steady_clock::now()) {}
  ~HostTimer() {
    if (!c->timing) return;
    TimerRec& t = c->timers[name];
    t.ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    t.launches++;
  }
};

static void flush_timers(mor_ctx* c) {
  (void)hipStreamSynchronize(c->st);
  for (auto& kv : c->timers) {
    for (auto& e : kv.second.ev) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) kv.second.ms += ms;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    kv.second.ev.clear();
  }
}

struct MorEngine;
static int scratch_setup(int dev) noexcept;
static void engine_free(mor_ctx* c, MorEngine& e);
static void engine_delete(MorEngine* e);

// ------------------------------------------------------------------------------- C-ABI basics
extern "C" const char* mor_last_error(void) { return g_err.c_str(); }

extern "C" void mor_default_opts(mor_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = MOR_FP32_REFINE;
  o->cg_rtol = 1e-5;
  o->refine_rtol = 1e-8;
  o->max_iter = 4000;
  o->refine_steps = 3;
  o->oversample = 0;
  o->eig_rtol = 1e-10;
  o->eig_max_iter = 600;
  o->cg_chunk = 8;
  o->spmm_rows = 0;
  o->spmm_kind = 0;
  o->use_graph = 0;
  o->hbm_budget_bytes = 0;
  o->reduced_solver = 0;
  o->reduced_rtol = 1e-12;
  o->reduced_max_iter = 20000;
  o->coarse = 1;
}

// mor_create's body; `c` is the caller's handle of the context under construction, so that an
// exception can release it (every normal return has released it or handed it out already).
static int create_impl(const mor_mesh* mesh, const mor_coeff* coeff, const mor_subdomains* sub,
                       const mor_opts* opts, mor_ctx** out, mor_ctx*& c) {
  if (!mesh || !coeff || !sub || !out) return fail(MOR_EINVAL, "null argument");
  if (mesh->n_nodes <= 0 || mesh->n_tets <= 0 || !mesh->xyz || !mesh->tets || !mesh->dirichlet)
    return fail(MOR_EINVAL, "empty or incomplete mesh");
  if (!coeff->kappa) return fail(MOR_EINVAL, "kappa is required");
  if (sub->n_sub <= 0 || !sub->ext_tet_ptr || !sub->ext_tets || !sub->in_core)
    return fail(MOR_EINVAL, "empty decomposition");
  if (mesh->n_nodes > INT32_MAX || mesh->n_tets > INT32_MAX) return fail(MOR_EINVAL, "mesh too large for int32 ids");
  c = new mor_ctx();
  if (opts) c->opts = *opts;
  else mor_default_opts(&c->opts);
  if (c->opts.precision < MOR_FP64 || c->opts.precision > MOR_BF16_SPLIT) {
    delete c;
    c = nullptr;
    return fail(MOR_EINVAL, "unknown precision mode");
  }
  if (c->opts.reduced_solver < 0 || c->opts.reduced_solver > 2 || c->opts.reduced_rtol < 0 ||
      c->opts.reduced_max_iter < 0) {
    delete c;
    c = nullptr;
    return fail(MOR_EINVAL, "reduced_solver must be 0, 1 or 2, reduced_rtol and reduced_max_iter >= 0");
  }
  if (c->opts.reduced_rtol == 0) c->opts.reduced_rtol = 1e-12;
  if (c->opts.reduced_max_iter == 0) c->opts.reduced_max_iter = 20000;
  c->st = (hipStream_t)c->opts.hip_stream;
  HostMesh& m = c->mesh;
  m.n_nodes = mesh->n_nodes;
  m.n_tets = mesh->n_tets;
  m.xyz.assign(mesh->xyz, mesh->xyz + 3 * m.n_nodes);
  m.tets.assign(mesh->tets, mesh->tets + 4 * m.n_tets);
  m.dirichlet.assign(mesh->dirichlet, mesh->dirichlet + m.n_nodes);
  for (int64_t t = 0; t < m.n_tets; ++t)
    if (!(coeff->kappa[t] > 0.0)) {
      delete c;
      c = nullptr;
      return fail(MOR_EINVAL, "kappa must be positive");
    }
  c->kappa.assign(coeff->kappa, coeff->kappa + m.n_tets);
  c->has_f = coeff->f_nodal != nullptr;
  if (c->has_f) c->fnodal.assign(coeff->f_nodal, coeff->f_nodal + m.n_nodes);
  std::string err;
  if (build_mesh(m, err)) {
    delete c;
    c = nullptr;
    return fail(MOR_EINVAL, err);
  }
  const int n = sub->n_sub;
  c->ext_ptr.assign(sub->ext_tet_ptr, sub->ext_tet_ptr + n + 1);
  if (c->ext_ptr[0] != 0) {
    delete c;
    c = nullptr;
    return fail(MOR_EINVAL, "ext_tet_ptr[0] must be 0");
  }
  for (int i = 0; i < n; ++i)
    if (c->ext_ptr[i + 1] < c->ext_ptr[i]) {
      delete c;
      c = nullptr;
      return fail(MOR_EINVAL, "ext_tet_ptr must be non-decreasing");
    }
  c->ext.assign(sub->ext_tets, sub->ext_tets + c->ext_ptr[n]);
  c->in_core.assign(sub->in_core, sub->in_core + c->ext_ptr[n]);
  c->subs.resize(n);
  // halo size of the LDS SpMM tiles: spmm_rows picks one of kHaloCaps (0: 96 rows, with
  // 128-byte slices 19 KB of LDS per workgroup)
  c->halo_cap = 96;
  if (c->opts.spmm_kind != 2 && c->opts.spmm_rows > 0)
    for (int cap : kHaloCaps)
      if (cap <= c->opts.spmm_rows) c->halo_cap = cap;
  {
    // the subdomains are independent: build them on the host cores
    // (a worker catches what its subdomain throws: 2 = host allocation failure, 3 = other)
    std::vector<std::string> errs(n);
    std::vector<int> bad(n, 0);
    const int nth = std::max(1, std::min<int>(n, (int)std::thread::hardware_concurrency()));
    std::atomic<int> next{0};
    auto work = [&]() {
      for (int i = next++; i < n; i = next++) {
        try {
          bad[i] = build_sub(m, c->ext.data() + c->ext_ptr[i], c->in_core.data() + c->ext_ptr[i],
                             c->ext_ptr[i + 1] - c->ext_ptr[i], c->subs[i], errs[i], c->halo_cap);
        } catch (const std::bad_alloc&) {
          bad[i] = 2;
        } catch (...) {
          bad[i] = 3;
        }
      }
    };
    std::vector<std::thread> pool;
    pool.reserve(nth);
    for (int w = 0; w < nth; ++w) {
      try {
        pool.emplace_back(work);
      } catch (const std::system_error&) {
        break;   // no more threads: the ones started (or this thread, below) take the rest
      }
    }
    for (auto& th : pool) th.join();
    work();
    for (int i = 0; i < n; ++i)
      if (bad[i]) {
        const int b = bad[i];
        delete c;
        c = nullptr;
        if (b == 2) return fail(MOR_ENOMEM, "host memory allocation failed");
        if (b == 3) return fail(MOR_EDEVICE, "internal error while building subdomain " + std::to_string(i));
        return fail(MOR_EINVAL, "subdomain " + std::to_string(i) + ": " + errs[i]);
      }
  }
  if (build_owner(m, c->subs, c->owner, c->ownpos, err) ||
      build_omega0(m, c->subs, c->ext_ptr.data(), c->ext.data(), c->in_core.data(), c->owner, c->ownpos, c->om0, err)) {
    delete c;
    c = nullptr;
    return fail(MOR_EINVAL, err);
  }
  c->res.resize(n);
  if (c->opts.host_only) {
    *out = c;
    c = nullptr;
    return MOR_OK;
  }
  // device uploads: geometry, coefficients, patterns
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  (void)scratch_setup(c->device);   // the no-allocation solve's array (its failure surfaces there)
  int rc = 0;
  rc = rc ? rc : upload(c, &c->d_xyz, m.xyz.data(), m.xyz.size());
  rc = rc ? rc : upload(c, &c->d_tets, m.tets.data(), m.tets.size());
  rc = rc ? rc : upload(c, &c->d_kappa, c->kappa.data(), c->kappa.size());
  if (c->has_f) rc = rc ? rc : upload(c, &c->d_f, c->fnodal.data(), c->fnodal.size());
  auto up_sub = [&](const HostSub& h, SubDev& d) {
    int r = 0;
    r = r ? r : upload(c, &d.rp, h.rp.data(), h.rp.size());
    r = r ? r : upload(c, &d.col, h.col.data(), h.col.size());
    r = r ? r : upload(c, &d.ii_end, h.ii_end.data(), h.ii_end.size());
    r = r ? r : upload(c, &d.rpV, h.rpV.data(), h.rpV.size());
    r = r ? r : upload(c, &d.colV, h.colV.data(), h.colV.size());
    r = r ? r : upload(c, &d.ltet, h.ltet.data(), h.ltet.size());
    r = r ? r : upload(c, &d.tetg, h.tetg.data(), h.tetg.size());
    r = r ? r : upload(c, &d.nodes, h.nodes.data(), h.nodes.size());
    r = r ? r : upload(c, &d.core, h.core.data(), h.core.size());
    r = r ? r : upload(c, &d.bp, h.bp.data(), h.bp.size());
    r = r ? r : upload(c, &d.bpL, h.bpL.data(), h.bpL.size());
    r = r ? r : upload(c, &d.rcbL, h.rcbL.data(), h.rcbL.size());
    r = r ? r : upload(c, &d.htile, h.htile.data(), h.htile.size());
    r = r ? r : upload(c, &d.halo, h.halo.data(), h.halo.size());
    r = r ? r : upload(c, &d.hrowp, h.hrowp.data(), h.hrowp.size());
    r = r ? r : upload(c, &d.hpe, h.hpe.data(), h.hpe.size());
    r = r ? r : upload(c, &d.hpp, h.hpp.data(), h.hpp.size());
    r = r ? r : upload(c, &d.hself, h.hself.data(), h.hself.size());
    r = r ? r : upload(c, &d.rcb, h.rcb.data(), h.rcb.size());
    if (!h.smap.empty()) {
      r = r ? r : upload(c, &d.smap, h.smap.data(), h.smap.size());
      r = r ? r : upload(c, &d.spos, h.spos.data(), h.spos.size());
    }
    return r;
  };
  c->sdev.resize(n);
  for (int i = 0; i < n && !rc; ++i) rc = up_sub(c->subs[i], c->sdev[i]);
  if (!rc) rc = up_sub(c->om0.sub, c->om0dev);
  if (!rc && hipStreamSynchronize(c->st) != hipSuccess) rc = fail(MOR_EDEVICE, "upload failed");
  if (rc) {
    mor_destroy(c);
    c = nullptr;
    return rc;
  }
  *out = c;
  c = nullptr;
  return MOR_OK;
}

extern "C" int mor_create(const mor_mesh* mesh, const mor_coeff* coeff, const mor_subdomains* sub,
                          const mor_opts* opts, mor_ctx** out) {
  mor_ctx* c = nullptr;
  try {
    return create_impl(mesh, coeff, sub, opts, out, c);
  } catch (...) {
    const int rc = exception_code();
    if (c) {
      try {
        mor_destroy(c);
      } catch (...) {
      }
    }
    return rc;
  }
}

static void destroy_impl(mor_ctx* c) {
  if (c->opts.host_only) {
    delete c;
    return;
  }
  (void)hipStreamSynchronize(c->st);
  for (int k = 0; k < 2; ++k)
    if (c->eng[k]) {
      engine_free(c, *c->eng[k]);
      engine_delete(c->eng[k]);
      c->eng[k] = nullptr;
    }
  for (auto& kv : c->timers)
    for (auto& e : kv.second.ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  for (void* p : c->allocs) dfree(c, p);
  delete c;
}

extern "C" void mor_destroy(mor_ctx* c) {
  if (!c) return;
  try {
    destroy_impl(c);
  } catch (...) {
    (void)exception_code();   // nothing to return; the message stays in mor_last_error
  }
}

// ------------------------------------------------------------------------------- assembly
// Assemble the matrices of a set of subdomains (or omega_0) colour by colour.
struct AsmJob {
  const HostSub* h;
  const SubDev* d;
  double *A, *K, *Ki, *f;
};

static int assemble_batch(mor_ctx* c, const std::vector<AsmJob>& jobs) {
  const int nj = (int)jobs.size();
  const int nc = c->mesh.ncolours;
  std::vector<AsmSub> hs((size_t)nj * nc);
  std::vector<int> prefix((size_t)nj * nc + nc, 0);
  // per colour: nj descriptors and nj+1 prefix entries
  std::vector<int> pre((size_t)(nj + 1) * nc);
  for (int col = 0; col < nc; ++col) {
    pre[(size_t)col * (nj + 1)] = 0;
    for (int j = 0; j < nj; ++j) {
      const HostSub& h = *jobs[j].h;
      AsmSub& a = hs[(size_t)col * nj + j];
      a.ltet = jobs[j].d->ltet;
      a.tetg = jobs[j].d->tetg;
      a.core = jobs[j].d->core;
      a.t_begin = h.colour_ptr[col];
      a.t_count = h.colour_ptr[col + 1] - h.colour_ptr[col];
      a.rp = jobs[j].d->rp;
      a.col = jobs[j].d->col;
      a.rpV = jobs[j].d->rpV;
      a.colV = jobs[j].d->colV;
      a.A = jobs[j].A;
      a.K = jobs[j].K;
      a.Ki = jobs[j].Ki;
      a.f = jobs[j].f;
      pre[(size_t)col * (nj + 1) + j + 1] = pre[(size_t)col * (nj + 1) + j] + a.t_count;
    }
  }
  AsmSub* d_hs = (AsmSub*)dalloc(c, sizeof(AsmSub) * hs.size());
  int* d_pre = (int*)dalloc(c, sizeof(int) * pre.size());
  if (!d_hs || !d_pre) {
    dfree(c, d_hs);
    dfree(c, d_pre);
    return fail(MOR_ENOMEM, "device allocation failed (assembly descriptors)");
  }
  HIPCHK(hipMemcpyAsync(d_hs, hs.data(), sizeof(AsmSub) * hs.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(d_pre, pre.data(), sizeof(int) * pre.size(), hipMemcpyHostToDevice, c->st));
  {
    int64_t ntet = 0;
    for (auto& j : jobs) ntet += (int64_t)j.h->tetg.size();
    ScopedTimer tm(c, "assemble", (double)ntet);
    for (int col = 0; col < nc; ++col) {
      const int total = pre[(size_t)col * (nj + 1) + nj];
      launch_assemble(d_hs + (size_t)col * nj, d_pre + (size_t)col * (nj + 1), nj, total, c->d_xyz, c->d_tets,
                      c->d_kappa, c->d_f, c->st);
    }
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  dfree(c, d_hs);
  dfree(c, d_pre);
  return 0;
}

// ------------------------------------------------------------------------------- batch GEMM
struct GemmBatch {
  std::vector<GemmDesc> d;
  std::vector<int4> tiles;
  GemmDesc* dd = nullptr;
  int4* dt = nullptr;
  void add(const GemmDesc& g) {
    const int id = (int)d.size();
    d.push_back(g);
    const int tm = (g.m + 63) / 64, tn = (g.n + 63) / 64;
    for (int i = 0; i < tm; ++i)
      for (int j = 0; j < tn; ++j)
        if (!g.sym || i <= j) tiles.push_back(make_int4(id, i, j, 0));
  }
  double flops() const {
    double f = 0;
    for (auto& g : d) f += 2.0 * g.m * g.n * g.k * (g.sym ? 0.5 : 1.0);
    return f;
  }
};
static int gemm_upload(mor_ctx* c, GemmBatch& b, Arena& ar) {
  b.dd = (GemmDesc*)ar.take(sizeof(GemmDesc) * std::max<size_t>(1, b.d.size()));
  b.dt = (int4*)ar.take(sizeof(int4) * std::max<size_t>(1, b.tiles.size()));
  if (!b.dd || !b.dt) return fail(MOR_ENOMEM, "arena exhausted (gemm)");
  if (!b.d.empty()) HIPCHK(hipMemcpyAsync(b.dd, b.d.data(), sizeof(GemmDesc) * b.d.size(), hipMemcpyHostToDevice, c->st));
  if (!b.tiles.empty())
    HIPCHK(hipMemcpyAsync(b.dt, b.tiles.data(), sizeof(int4) * b.tiles.size(), hipMemcpyHostToDevice, c->st));
  return 0;
}
static void gemm_run(mor_ctx* c, const GemmBatch& b, const char* tname) {
  ScopedTimer tm(c, tname, b.flops());
  launch_gemm(b.dd, b.dt, (int)b.tiles.size(), c->st);
}
static GemmDesc gd(int m, int n, int k, const double* A, int lda, int ta, const double* B, int ldb, int tb, double* C,
                   int ldc, double alpha = 1.0, double beta = 0.0, int sym = 0) {
  GemmDesc g;
  g.m = m; g.n = n; g.k = k;
  g.A = A; g.lda = lda; g.ta = ta;
  g.B = B; g.ldb = ldb; g.tb = tb;
  g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta; g.sym = sym;
  return g;
}

// ------------------------------------------------------------------------------- blocked TRSM
// Triangular solves with a Cholesky factor R (upper, T panels of 64 rows, in DenseSub) over a
// batch.  The panel kernels solve one diagonal block of kTrsmBlk panels at a time, in place in X
// (B is copied there first), and the coupling to the other blocks is one k_gemm update per block
// (the rows below it for R^T X = B, the rows above it for R X = B): most of the flops then run
// on XCD-grouped GEMM tiles over the whole chip instead of inside the panel loop, which keeps
// one workgroup per 64-column tile busy for all T panels.
constexpr int kTrsmBlk = 8;

struct DevBuf {   // one device allocation for descriptors and tile lists, freed once the stream drains
  mor_ctx* c;
  char* p;
  Arena ar;
  DevBuf(mor_ctx* cc, size_t bytes) : c(cc), p((char*)dalloc(cc, bytes)) { ar = Arena{p, p ? bytes : 0, 0}; }
  ~DevBuf() {
    if (!p) return;
    (void)hipStreamSynchronize(c->st);
    dfree(c, p);
  }
};

static int gemm_now(mor_ctx* c, const GemmBatch& g, GemmDesc* dg, int4* dt) {
  if (g.d.empty()) return 0;
  HIPCHK(hipMemcpyAsync(dg, g.d.data(), sizeof(GemmDesc) * g.d.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(dt, g.tiles.data(), sizeof(int4) * g.tiles.size(), hipMemcpyHostToDevice, c->st));
  launch_gemm(dg, dt, (int)g.tiles.size(), c->st);
  return 0;
}

// R^T X = B for every slot i (hds[i], htd[i]; dds: the DenseSub table on the device)
static int trsm_lt_blocked(mor_ctx* c, const std::vector<DenseSub>& hds, const DenseSub* dds,
                           const std::vector<TrsmDesc>& htd) {
  hipStream_t st = c->st;
  const int ns = (int)hds.size();
  if (ns == 0) return 0;
  int tmax = 0, ctmax = 0;
  size_t tiles = 1;
  for (int i = 0; i < ns; ++i) {
    tmax = std::max(tmax, hds[i].T);
    ctmax = std::max(ctmax, htd[i].ncol_tiles);
    tiles += (size_t)std::max(hds[i].T - kTrsmBlk, 0) * htd[i].ncol_tiles;
  }
  DevBuf buf(c, sizeof(TrsmDesc) * ns + sizeof(GemmDesc) * ns + sizeof(int4) * tiles + 3 * 256);
  TrsmDesc* dip = (TrsmDesc*)buf.ar.take(sizeof(TrsmDesc) * ns);
  GemmDesc* dg = (GemmDesc*)buf.ar.take(sizeof(GemmDesc) * ns);
  int4* dt = (int4*)buf.ar.take(sizeof(int4) * tiles);
  if (!dip || !dg || !dt) return fail(MOR_ENOMEM, "device allocation failed (triangular solve)");
  std::vector<TrsmDesc> ip(ns);
  for (int i = 0; i < ns; ++i) {
    const TrsmDesc& t = htd[i];
    launch_copy_rect(t.B, t.ldb, t.tb, t.X, t.ldx, hds[i].MP, t.ncol_tiles * 64, st);
    ip[i] = TrsmDesc{t.X, t.ldx, 0, t.X, t.ldx, t.ncol_tiles};
  }
  HIPCHK(hipMemcpyAsync(dip, ip.data(), sizeof(TrsmDesc) * ns, hipMemcpyHostToDevice, st));
  for (int p0 = 0; p0 < tmax; p0 += kTrsmBlk) {
    const int p1 = p0 + kTrsmBlk;
    launch_trsm_lt(dds, dip, ns, ctmax, st, p0, p1);
    GemmBatch g;   // X[p1:, :] -= R[p0:p1, p1:]^T X[p0:p1, :]
    for (int i = 0; i < ns; ++i) {
      const DenseSub& d = hds[i];
      if (d.T <= p1) continue;
      const int ld = ip[i].ldx;
      double* X = ip[i].X;
      g.add(gd((d.T - p1) * 64, ip[i].ncol_tiles * 64, kTrsmBlk * 64, d.S + (size_t)p0 * 64 * d.MP + (size_t)p1 * 64,
               d.MP, 1, X + (size_t)p0 * 64 * ld, ld, 0, X + (size_t)p1 * 64 * ld, ld, -1.0, 1.0));
    }
    if (int rc = gemm_now(c, g, dg, dt)) return rc;
  }
  return 0;
}

// R X = B for one 64-column tile per slot (B, X: MP x 64, ld 64; host arrays of device pointers)
static int trsm_un_blocked(mor_ctx* c, const std::vector<DenseSub>& hds, const DenseSub* dds,
                           const std::vector<double*>& hB, const std::vector<double*>& hX) {
  hipStream_t st = c->st;
  const int ns = (int)hds.size();
  if (ns == 0) return 0;
  int tmax = 0;
  size_t tiles = 1;
  for (int i = 0; i < ns; ++i) {
    tmax = std::max(tmax, hds[i].T);
    tiles += (size_t)hds[i].T;
  }
  DevBuf buf(c, sizeof(double*) * ns + sizeof(GemmDesc) * ns + sizeof(int4) * tiles + 3 * 256);
  double** dX = (double**)buf.ar.take(sizeof(double*) * ns);
  GemmDesc* dg = (GemmDesc*)buf.ar.take(sizeof(GemmDesc) * ns);
  int4* dt = (int4*)buf.ar.take(sizeof(int4) * tiles);
  if (!dX || !dg || !dt) return fail(MOR_ENOMEM, "device allocation failed (triangular solve)");
  for (int i = 0; i < ns; ++i)
    if (hB[i] != hX[i]) launch_copy_rect(hB[i], 64, 0, hX[i], 64, hds[i].MP, 64, st);
  HIPCHK(hipMemcpyAsync(dX, hX.data(), sizeof(double*) * ns, hipMemcpyHostToDevice, st));
  for (int p0 = (tmax - 1) / kTrsmBlk * kTrsmBlk; p0 >= 0; p0 -= kTrsmBlk) {
    const int p1 = p0 + kTrsmBlk;
    launch_trsm_un(dds, ns, dX, dX, st, p0, p1);
    if (p0 == 0) break;
    GemmBatch g;   // X[:p0, :] -= R[:p0, p0:pe] X[p0:pe, :]
    for (int i = 0; i < ns; ++i) {
      const DenseSub& d = hds[i];
      if (d.T <= p0) continue;
      const int pe = std::min(p1, d.T);
      g.add(gd(p0 * 64, 64, (pe - p0) * 64, d.S + (size_t)p0 * 64, d.MP, 0, hX[i] + (size_t)p0 * 64 * 64, 64, 0, hX[i],
               64, -1.0, 1.0));
    }
    if (int rc = gemm_now(c, g, dg, dt)) return rc;
  }
  return 0;
}

// ------------------------------------------------------------------------------- block CG
// ------------------------------------------------------------------------------- CG tiles
struct TileCfg {
  int v = 4;    // elements per lane: tile width 64 v columns
  int rb = 32;  // rows (row tiles) or aggregates (block tiles) per tile
  int halo = 1; // SpMM only: LDS halo tiles (1) or row tiles (0)
  int g = 4;    // SpMM halo tiles: column slices per workgroup
  int cwb = 256;  // SpMM halo tiles: bytes of a row per column slice (128 or 256)
};

// ------------------------------------------------------------------------------- debug dumps
// MOR_DUMP=<dir> writes intermediate device arrays of the first slot of a dense batch.
static void dump(mor_ctx* c, const char* name, const void* dptr, size_t bytes) {
  const char* dir = getenv("MOR_DUMP");
  if (!dir || !dptr || !bytes) return;
  std::vector<char> h(bytes);
  if (hipStreamSynchronize(c->st) != hipSuccess) return;
  if (hipMemcpy(h.data(), dptr, bytes, hipMemcpyDeviceToHost) != hipSuccess) return;
  const std::string path = std::string(dir) + "/" + name + ".bin";
  FILE* f = fopen(path.c_str(), "wb");
  if (!f) return;
  fwrite(h.data(), 1, bytes, f);
  fclose(f);
}

// ------------------------------------------------------------------------------- truncation
// Number of leading singular triplets kept: top-`rank` (rank > 0) or sigma > tol, widened to
// the end of a cluster of equal singular values (relative gap <= 1e-4) so the kept span is
// well defined.
static int truncation_rank(const std::vector<double>& s, int rank, double tol, int cap) {
  const int M = (int)s.size();
  int k = 0;
  if (rank > 0) k = std::min(rank, M);
  else
    for (int j = 0; j < M; ++j) k += s[j] > tol ? 1 : 0;
  if (k == 0) return 0;
  while (k < M) {
    if (s[k - 1] <= 0.0 || (s[k - 1] - s[k]) / s[k - 1] > 1e-4) break;
    ++k;
  }
  return std::min(k, cap);
}

// ------------------------------------------------------------------------------- one request
struct Slot {
  int sd, rank, prec;
  double tol;
  bool fp32, refine;
  const HostSub* h;
  const SubDev* d;
  int M, MP, T, colsA, ldA, colsK, ldK, s, nconv;
  double *A64, *K64, *Ki64, *f;
  float *A32, *K32;
  float *s16A, *s16K;       // stencil coefficients of a box interior (FP32 systems), or nullptr
  void *minvA, *minvK;
  void *XA, *RA, *PA, *QA, *XK, *RK, *PK, *QK;
  double *XA64, *XK64;
  double* colst[2];         // per-column CG state of the two systems: 7 x ld doubles + ld ints
  double *Xc, *Ec;          // FP64 views of the solutions (converted in the FP32 mode)
  int ldXc, ldEc;
  double *Y, *S, *G, *W, *C, *Dinv;
  double *Vb, *Yb, *Ub, *Zb, *Vn, *Tb, *H, *Ss, *G2, *Rinv, *theta, *resid;
  double *Bk, *Wk, *Yf;
  uint16_t *Xh, *Xl, *Yh, *Yl;   // BF16 split (transposed) X_C and K_i X_C, MB x kpV
  int kpV, MB;                   // MB = roundup(M, 128): rows of the split operands
  // randomized variant (ls > 0 sketch columns, at most 64)
  bool box;                      // the plane-streaming SpMM serves this request's systems
  int ls, rk;                    // sketch columns; directions kept by the K_i-orthonormalisation
  double *Fd;                    // dense FP64 right-hand sides of the A solves, nI x ldA
  double *FdK;                   // dense FP64 right-hand sides [0; V] of the K^+ solves, nL x ldK
  double *q0v;                   // zero-boundary load solution on V_i
  double *Yk, *Wt, *KWt, *Vs;    // K_i Y, the K_i-orthonormal sketch basis W and K_i W (nV x 64); 64 x 64
  int* info;
  int k_eff;
  // two-level preconditioner (nc > 0): per system P^T r and A_c^-1 P^T r (nc x ld), A_c and then
  // A_c^-1 (MPc x MPc), R^-T (MPc x MPc), the Cholesky diagonal-block inverses, pivot reports
  // (per system: the K^+ system of the randomized variant has its own coarse blocks)
  int nc[2], MPc[2], Tc[2];
  double *crc[2], *cec[2], *cA[2], *cY[2], *cD[2];
  int* cinfo;
};

static void slot_shape(mor_ctx* c, Slot& q) {
  const HostSub& h = *q.h;
  q.M = h.nB;
  q.MP = (int)rup(q.M, 64);
  q.T = q.MP / 64;
  // rows of the block vectors start on 128-byte cache lines (32 FP32 / 16 FP64 columns), so
  // the column slices of the CG kernels never straddle a line they only partly use
  q.colsA = q.ls > 0 ? q.ls + 1 : h.nB + 1;   // sketch + load columns, or every interface column + load
  q.ldA = (int)rup(q.colsA, 32);
  // the K system: the H1 solve with every interface column, or (randomized variant) the K^+
  // solves on all local rows with the sketch's columns
  q.colsK = q.ls > 0 ? q.ls : h.nB;
  q.ldK = (int)rup(q.colsK, 32);
  const int p = c->opts.oversample > 0 ? c->opts.oversample : std::max(8, q.rank);
  int s = q.rank > 0 && q.ls == 0 ? std::min(64, q.rank + p) : 64;
  s = std::min(s, q.M);
  q.s = s;
  // the fewest Ritz pairs that must converge; the eigensolver raises it to the truncation
  // decision (kept pairs + the next + one) as the Ritz values settle
  q.nconv = std::max(1, std::min(s - 1, q.rank > 0 ? q.rank + 2 : 1));
  q.fp32 = q.prec != MOR_FP64;
  q.refine = q.prec == MOR_FP32_REFINE || q.prec == MOR_BF16_SPLIT;
  q.box = q.fp32 && c->opts.box_spmm >= 0 && c->opts.spmm_kind != 2 && !h.smap.empty() && q.d != nullptr &&
          q.d->smap != nullptr;
  const int nblk = (int)h.bp.size() - 1;
  const int nblkK = q.ls > 0 ? (int)h.bpL.size() - 1 : nblk;
  for (int w = 0; w < 2; ++w) {
    const int nb = w == 0 ? nblk : nblkK;
    q.nc[w] = c->opts.coarse ? (nb + kCoarseAgg - 1) / kCoarseAgg : 0;
    q.MPc[w] = (int)rup(std::max(q.nc[w], 1), 64);
    q.Tc[w] = q.MPc[w] / 64;
  }
}

// Device bytes of one request (CG blocks, dense matrices, eigensolver blocks), and the carve.
template <typename Take>
static bool slot_layout(Slot& q, Take tk) {
  const HostSub& h = *q.h;
  const size_t nnz = h.rp[h.nL], nnzV = h.rpV[h.nV];
  const size_t elt = q.fp32 ? 4 : 8;
  const int s = q.s;
  q.A64 = (double*)tk(8 * nnz); q.K64 = (double*)tk(8 * nnz); q.Ki64 = (double*)tk(8 * nnzV);
  q.f = (double*)tk(8 * (size_t)h.nL);
  q.A32 = q.fp32 ? (float*)tk(4 * nnz) : nullptr;
  q.K32 = q.fp32 ? (float*)tk(4 * nnz) : nullptr;
  const bool box = q.fp32 && q.box;
  q.s16A = box ? (float*)tk(4 * (size_t)kStencil * h.nI) : nullptr;
  q.s16K = box ? (float*)tk(4 * (size_t)kStencil * h.nI) : nullptr;
  const size_t rowsK = q.ls > 0 ? (size_t)h.nL : (size_t)h.nI;   // K^+ on all local rows, or K_II
  q.minvA = tk(elt * h.nI * 8); q.minvK = tk(elt * rowsK * 8);
  q.XA = tk(elt * h.nI * q.ldA); q.RA = tk(elt * h.nI * q.ldA);
  q.PA = tk(elt * h.nI * q.ldA); q.QA = tk(elt * h.nI * q.ldA);
  q.XK = tk(elt * rowsK * q.ldK); q.RK = tk(elt * rowsK * q.ldK);
  q.PK = tk(elt * rowsK * q.ldK); q.QK = tk(elt * rowsK * q.ldK);
  q.XA64 = q.refine ? (double*)tk(8 * (size_t)h.nI * q.ldA) : nullptr;
  q.XK64 = q.refine ? (double*)tk(8 * rowsK * q.ldK) : nullptr;
  q.colst[0] = (double*)tk(8 * 8 * (size_t)q.ldA + 64);
  q.colst[1] = (double*)tk(8 * 8 * (size_t)q.ldK + 64);
  if (q.fp32 && !q.refine) {
    q.Xc = (double*)tk(8 * (size_t)h.nV * q.ldA);
    q.Ec = (double*)tk(8 * (size_t)h.nI * q.ldK);
  } else if (q.refine) {
    q.Xc = q.XA64; q.Ec = q.XK64;
  } else {
    q.Xc = (double*)q.XA; q.Ec = (double*)q.XK;
  }
  q.ldXc = q.ldA; q.ldEc = q.ldK;
  const bool sk = q.ls > 0;
  q.Y = sk ? nullptr : (double*)tk(8 * (size_t)h.nV * q.ldK);
  q.kpV = (int)rup(std::max(h.nV, 1), 64);
  q.MB = (int)rup(q.M, 128);
  if (sk) {
    q.Fd = (double*)tk(8 * (size_t)h.nI * q.ldA);
    q.FdK = (double*)tk(8 * rowsK * q.ldK);
    q.q0v = (double*)tk(8 * (size_t)std::max(h.nV, 1));
    q.Yk = (double*)tk(8 * (size_t)h.nV * 64); q.Wt = (double*)tk(8 * (size_t)h.nV * 64);
    q.KWt = (double*)tk(8 * (size_t)h.nV * 64); q.Vs = (double*)tk(8 * 64 * 64);
  } else {
    q.Fd = q.FdK = q.q0v = q.Yk = q.Wt = q.KWt = q.Vs = nullptr;
  }
  if (q.prec == MOR_BF16_SPLIT && !sk) {
    const size_t b = 2 * (size_t)q.MB * q.kpV;
    q.Xh = (uint16_t*)tk(b); q.Xl = (uint16_t*)tk(b);
    q.Yh = (uint16_t*)tk(b); q.Yl = (uint16_t*)tk(b);
  } else {
    q.Xh = q.Xl = q.Yh = q.Yl = nullptr;
  }
  q.S = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * q.MP);   // the randomized variant forms no M x M matrix
  q.G = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * q.MP);
  q.W = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * q.MP);
  q.C = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * q.MP);
  q.Dinv = sk ? nullptr : (double*)tk(8 * (size_t)q.T * 4096);
  q.Vb = (double*)tk(8 * (size_t)q.MP * (sk ? 64 : s)); q.Yb = (double*)tk(8 * (size_t)q.MP * (sk ? 64 : s));
  q.Ub = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * s);
  q.Zb = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * s);
  q.Vn = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * s);
  q.Tb = sk ? nullptr : (double*)tk(8 * (size_t)q.MP * s);
  q.H = (double*)tk(8 * (size_t)s * s); q.Ss = (double*)tk(8 * (size_t)s * s);
  q.G2 = (double*)tk(8 * (size_t)s * s); q.Rinv = (double*)tk(8 * (size_t)s * s);
  q.theta = (double*)tk(8 * (size_t)s); q.resid = (double*)tk(8 * (size_t)s);
  q.Bk = (double*)tk(8 * (size_t)q.MP * 64); q.Wk = (double*)tk(8 * (size_t)q.MP * 64);
  q.Yf = (double*)tk(8 * (size_t)std::max(1, h.nP) * (s + 2));
  for (int w = 0; w < 2; ++w) {
    const int ld = w == 0 ? q.ldA : q.ldK;
    const bool on = q.nc[w] > 0;
    q.crc[w] = on ? (double*)tk(8 * (size_t)q.nc[w] * ld) : nullptr;
    q.cec[w] = on ? (double*)tk(8 * (size_t)q.nc[w] * ld) : nullptr;
    q.cA[w] = on ? (double*)tk(8 * (size_t)q.MPc[w] * q.MPc[w]) : nullptr;
    q.cY[w] = on ? (double*)tk(8 * (size_t)q.MPc[w] * q.MPc[w]) : nullptr;
    q.cD[w] = on ? (double*)tk(8 * (size_t)q.Tc[w] * 4096) : nullptr;
  }
  q.cinfo = q.nc[0] > 0 ? (int*)tk(128) : nullptr;
  q.info = (int*)tk(64);
  return q.info != nullptr;
}

static size_t slot_bytes(Slot& q) {
  Sizer z;
  Slot tmp = q;
  slot_layout(tmp, [&](size_t b) -> void* { z.add(b); return (void*)1; });
  return z.total + 4096;
}

// ------------------------------------------------------------------------------- engine
// Requests for local reductions flow through one engine per CG scalar type.  At each tick the
// engine admits pending requests whose memory fits the HBM budget (their assembly and CG
// start are batched), advances every system still iterating by one CG chunk in shared
// launches, restarts systems that reached the inner tolerance from an FP64 residual (FP32 +
// refinement), and runs the dense stage (Gram, Schur, Cholesky, eigensolve, basis, local
// projection) for the requests whose two solves finished.  Requests therefore join and leave
// the running block CG independently: continuous batching.
struct SysRun {
  CgSys S;
  int cnt;        // index of this system's active-column counter
  int phase;      // 0 iterating, 1 finished
  int iters, refines;
  int nnzII;
  int nhtile;     // LDS-halo SpMM tiles of the subdomain
  const double* Ainv = nullptr;   // two-level preconditioner: A_c^-1 (ldac x ldac), or nullptr
  int ldac = 0;
};

struct Live {
  uint64_t id;
  Slot q;
  char* mem = nullptr;
  size_t bytes = 0;
  SysRun sys[2];
  int status = 0;
  // randomized variant: 0 first K^+ solve, 1 sketch solve, 2 left solve, 3 second K^+ solve,
  // 4 done (small SVD, basis and projection)
  int stage = 0;
  int iters_prev = 0;                            // A-system iterations of finished solves
  std::shared_ptr<const std::vector<double>> om; // the random matrix S_i (M x l, host)
};

struct Req {
  uint64_t id;
  int sd, rank, prec;
  double tol;
  int done = 0, status = 0;
  int ls = 0;                                    // sketch columns (0: explicit SVD)
  std::shared_ptr<const std::vector<double>> om;
};

struct Launch {
  std::vector<SysRun*> sys;
  int4 *sp = nullptr, *bk = nullptr, *hs = nullptr, *bx = nullptr, *rs = nullptr;
  int nsp = 0, nbk = 0, nhs = 0, nbx = 0, nrs = 0;   // rs: row-tile SpMM of the systems without halo tiles
  int2* cb = nullptr;
  int ncb = 0;
  double spmm_bytes = 0;     // algorithmic bytes of the general (halo or row-tile) SpMM launch
  double box_bytes = 0;      // ... and of the box-interior launch
  double stream_bytes = 0;   // update + direction: 8 block-vector elements per entry
  GemmDesc* gd = nullptr;    // two-level preconditioner: A_c^-1 (P^T r) of every coarse system
  int4* gt = nullptr;
  int ngt = 0;
  double coarse_flops = 0;
};

// Inner stop of a block-CG system: FP64 systems iterate to the outer target refine_rtol; FP32
// systems (refined in FP64 or not) stop at cg_rtol.
template <typename T>
static double inner_tol2(const mor_ctx* c) {
  const double t = sizeof(T) == 8 ? c->opts.refine_rtol : (c->opts.cg_rtol > 0 ? c->opts.cg_rtol : 1e-5);
  return t * t;
}

struct MorEngine {
  int elt = 4;
  std::vector<Req> pending;
  std::vector<Live*> live;
  std::map<uint64_t, Req> finished;
  CgSys* d_sys = nullptr;
  size_t sys_cap = 0;
  int4* d_tiles = nullptr;
  size_t tiles_cap = 0;
  std::vector<CgSys> up_hs;   // the systems of the last upload (its device lists)
  Launch up_L;
  bool up_ok = false;
  // graph mode: the CG chunk captured once per system set and replayed
  hipStream_t cap_st = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<SysRun*> g_sys;
  std::vector<int64_t> g_key;
  int2* d_cb = nullptr;
  size_t cb_cap = 0;
  GemmDesc* d_gd = nullptr;
  size_t gd_cap = 0;
  int4* d_gt = nullptr;
  size_t gt_cap = 0;
  int* d_cnt = nullptr;
  int* h_cnt = nullptr;
  int cnt_cap = 0;
  std::vector<int> cnt_free;
  size_t live_bytes = 0, peak_bytes = 0, budget = 0;
  TileCfg sp, stm;
};

static uint64_t g_next_ticket = 1;

static int engine_init(mor_ctx* c, MorEngine& e, int elt) {
  e.elt = elt;
  e.cnt_cap = 8192;
  e.d_cnt = (int*)palloc(c, sizeof(int) * e.cnt_cap);
  if (!e.d_cnt) return fail(MOR_ENOMEM, "device allocation failed (engine counters)");
  HIPCHK(hipHostMalloc((void**)&e.h_cnt, sizeof(int) * e.cnt_cap));
  for (int i = e.cnt_cap - 1; i >= 0; --i) e.cnt_free.push_back(i);
  const bool fp32 = elt == 4;
  e.sp.halo = c->opts.spmm_kind != 2;
  e.sp.cwb = c->opts.spmm_kind == 1 ? 256 : 128;
  if (e.sp.halo) {
    e.sp.g = c->opts.spmm_vec > 0 ? std::min(c->opts.spmm_vec, 64) : 16;   // slices per workgroup
    e.sp.v = fp32 ? 4 : 2;   // the row kernels (init, residual, shadow)
  } else {
    e.sp.v = c->opts.spmm_vec > 0 ? c->opts.spmm_vec : 4;
    if (!fp32 && e.sp.v > 2) e.sp.v = 2;
  }
  // rows per row tile (the row kernels, and the SpMM of row-tile systems): 32 by default, so that
  // the tile lists the host rebuilds whenever the set of iterating systems changes stay short
  e.sp.rb = c->opts.spmm_rows > 0 ? std::min(c->opts.spmm_rows, 64) : 32;
  // block kernels hold 8 rows per lane; 64-column tiles measured fastest (C2, C3, C4 tuner sweeps)
  e.stm.v = c->opts.stream_vec > 0 ? c->opts.stream_vec : 1;
  if (!fp32 && e.stm.v > 2) e.stm.v = 2;
  e.stm.rb = c->opts.stream_blocks > 0 ? c->opts.stream_blocks : 8;
  // two-level preconditioner: every streaming tile lies inside one coarse block
  if (c->opts.coarse && kCoarseAgg % e.stm.rb != 0) e.stm.rb = kCoarseAgg;
  e.budget = c->opts.hbm_budget_bytes;
  if (!e.budget) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = (size_t)64 << 30;
    e.budget = fr / 4 * 3;
  }
  return 0;
}

static void engine_free(mor_ctx* c, MorEngine& e) {
  for (Live* L : e.live) {
    dfree(c, L->mem);
    delete L;
  }
  e.live.clear();
  dfree(c, e.d_sys);
  dfree(c, e.d_tiles);
  dfree(c, e.d_cb);
  dfree(c, e.d_gd);
  dfree(c, e.d_gt);
  if (e.h_cnt) (void)hipHostFree(e.h_cnt);
  e.h_cnt = nullptr;
  if (e.gexec) (void)hipGraphExecDestroy(e.gexec);
  e.gexec = nullptr;
  if (e.cap_st) (void)hipStreamDestroy(e.cap_st);
  e.cap_st = nullptr;
}

template <typename T>
static int grow(mor_ctx* c, T** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return 0;
  dfree(c, *p);
  *cap = std::max<size_t>(need + need / 2, 64);
  *p = (T*)dalloc(c, sizeof(T) * *cap);
  if (!*p) return fail(MOR_ENOMEM, "device allocation failed (engine tables)");
  return 0;
}

// Upload the systems in `list` as the device table; return tiles and column blocks over them.

static int engine_upload(mor_ctx* c, MorEngine& e, Launch& L) {
  const int n = (int)L.sys.size();
  std::vector<CgSys> hs(n);
  std::vector<int4> t;
  std::vector<int2> cb;
  for (int i = 0; i < n; ++i) hs[i] = L.sys[i]->S;
  // the same systems as the last upload: the device lists are still in place
  if (e.up_ok && L.sys == e.up_L.sys && std::memcmp(hs.data(), e.up_hs.data(), sizeof(CgSys) * n) == 0) {
    L = e.up_L;
    return 0;
  }
  e.up_ok = false;
  L.spmm_bytes = 0;
  L.box_bytes = 0;
  L.stream_bytes = 0;
  for (int i = 0; i < n; ++i) L.stream_bytes += 8.0 * e.elt * (double)hs[i].nI * hs[i].ncols;
  for (int i = 0; i < n; ++i) {   // the matrix once, P read once, Q written once
    const CgSys& S = hs[i];
    const double b = (double)L.sys[i]->nnzII * (4.0 + e.elt) + 4.0 * (S.nI + 1) + 2.0 * e.elt * (double)S.nI * S.ncols;
    (S.s16 != nullptr ? L.box_bytes : L.spmm_bytes) += b;
  }
  for (int i = 0; i < n; ++i) {
    const CgSys& S = hs[i];
    for (int c0 = 0; c0 < S.ld; c0 += 64 * e.sp.v)
      for (int r0 = 0; r0 < S.nI; r0 += e.sp.rb) t.push_back(make_int4(i, r0, c0, 0));
  }
  L.nsp = (int)t.size();
  for (int i = 0; i < n; ++i) {
    const CgSys& S = hs[i];
    for (int c0 = 0; c0 < S.ld; c0 += 64 * e.stm.v)
      for (int b0 = 0; b0 < S.nblk; b0 += e.stm.rb) t.push_back(make_int4(i, b0, c0, 0));
  }
  L.nbk = (int)t.size() - L.nsp;
  if (e.sp.halo) {
    const int gw = (e.sp.cwb / e.elt) * e.sp.g;   // columns per slice group
    for (int i = 0; i < n; ++i) {
      if (hs[i].s16 != nullptr) continue;   // served by the box kernel
      const int nt = L.sys[i]->nhtile;
      for (int c0 = 0; c0 < hs[i].ld; c0 += gw)
        for (int h = 0; h < nt; ++h) t.push_back(make_int4(i, h, c0, c0 + gw));
    }
  }
  L.nhs = (int)t.size() - L.nsp - L.nbk;
  // box interiors: (system, 32-column slice, footprint row, footprint column), the footprint
  // column fastest so that neighbouring footprints of one slice run together on one XCD
  for (int i = 0; i < n; ++i) {
    const CgSys& S = hs[i];
    if (S.s16 == nullptr) continue;
    const int ntx = (S.bx + 7) / 8, nty = (S.by + 7) / 8;
    for (int c0 = 0; c0 < S.ld; c0 += 32)
      for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) t.push_back(make_int4(i, tx | (ty << 16), c0, 0));
  }
  L.nbx = (int)t.size() - L.nsp - L.nbk - L.nhs;
  // in the halo mode, systems without halo tiles (the K^+ systems of the randomized variant)
  // take the row-tile SpMM
  if (e.sp.halo)
    for (int i = 0; i < n; ++i) {
      const CgSys& S = hs[i];
      if (S.s16 != nullptr || L.sys[i]->nhtile > 0) continue;
      for (int c0 = 0; c0 < S.ld; c0 += 64 * e.sp.v)
        for (int r0 = 0; r0 < S.nI; r0 += e.sp.rb) t.push_back(make_int4(i, r0, c0, 0));
    }
  L.nrs = (int)t.size() - L.nsp - L.nbk - L.nhs - L.nbx;
  for (int i = 0; i < n; ++i)
    for (int c0 = 0; c0 < hs[i].ld; c0 += 256) cb.push_back(make_int2(i, c0));
  L.ncb = (int)cb.size();
  GemmBatch gb;
  for (int i = 0; i < n; ++i) {
    const CgSys& S = hs[i];
    if (S.rc != nullptr) {   // converged columns (alpha 0) need no coarse correction
      GemmDesc g = gd(S.nc, S.ld, S.nc, L.sys[i]->Ainv, L.sys[i]->ldac, 0, S.rc, S.ld, 0, S.ec, S.ld);
      g.skip = S.alpha;
      gb.add(g);
    }
  }
  L.ngt = (int)gb.tiles.size();
  L.coarse_flops = gb.flops();
  if (int rc = grow(c, &e.d_sys, &e.sys_cap, (size_t)std::max(n, 1))) return rc;
  if (int rc = grow(c, &e.d_tiles, &e.tiles_cap, std::max<size_t>(t.size(), 1))) return rc;
  if (int rc = grow(c, &e.d_cb, &e.cb_cap, std::max<size_t>(cb.size(), 1))) return rc;
  if (int rc = grow(c, &e.d_gd, &e.gd_cap, std::max<size_t>(gb.d.size(), 1))) return rc;
  if (int rc = grow(c, &e.d_gt, &e.gt_cap, std::max<size_t>(gb.tiles.size(), 1))) return rc;
  if (!gb.d.empty()) HIPCHK(hipMemcpyAsync(e.d_gd, gb.d.data(), sizeof(GemmDesc) * gb.d.size(), hipMemcpyHostToDevice, c->st));
  if (!gb.tiles.empty())
    HIPCHK(hipMemcpyAsync(e.d_gt, gb.tiles.data(), sizeof(int4) * gb.tiles.size(), hipMemcpyHostToDevice, c->st));
  if (n) HIPCHK(hipMemcpyAsync(e.d_sys, hs.data(), sizeof(CgSys) * n, hipMemcpyHostToDevice, c->st));
  if (!t.empty()) HIPCHK(hipMemcpyAsync(e.d_tiles, t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice, c->st));
  if (!cb.empty()) HIPCHK(hipMemcpyAsync(e.d_cb, cb.data(), sizeof(int2) * cb.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));   // the host vectors are pageable
  L.sp = e.d_tiles;
  L.bk = e.d_tiles + L.nsp;
  L.hs = e.d_tiles + L.nsp + L.nbk;
  L.bx = e.d_tiles + L.nsp + L.nbk + L.nhs;
  L.rs = e.d_tiles + L.nsp + L.nbk + L.nhs + L.nbx;
  L.cb = e.d_cb;
  L.gd = e.d_gd;
  L.gt = e.d_gt;
  e.up_hs.swap(hs);
  e.up_L = L;
  e.up_ok = true;
  return 0;
}

static int read_counts(mor_ctx* c, MorEngine& e) {
  HIPCHK(hipMemcpyAsync(e.h_cnt, e.d_cnt, sizeof(int) * e.cnt_cap, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return 0;
}

// The coarse products A_c^-1 (P^T r): on the FP32 matrix cores for the FP32 block CG (whose
// vectors carry FP32 anyway), on the FP64 ones for the FP64 CG.
// In the iterations (in_loop) the columns that have converged (alpha 0) are skipped; at a
// (re)start every column is computed (alpha is not yet set).
template <typename T>
static void launch_coarse_gemm(const GemmDesc* d, const int4* tiles, int ntiles, hipStream_t s, int in_loop) {
  if (std::is_same<T, float>::value) launch_gemm32(d, tiles, ntiles, s, in_loop);
  else launch_gemm(d, tiles, ntiles, s, in_loop);
}

// Two-level preconditioner at a (re)start, after the block-Jacobi start direction: the coarse
// solve of the restricted residual, its part of r'M^-1 r, and its correction of P.
template <typename T>
static void coarse_start(mor_ctx* c, MorEngine& e, const Launch& L) {
  if (L.ngt == 0) return;
  hipStream_t st = c->st;
  launch_coarse_gemm<T>(L.gd, L.gt, L.ngt, st, 0);
  launch_cg_coarse_dot(e.d_sys, L.cb, L.ncb, 1, st);
  launch_cg_prolong<T>(e.d_sys, L.bk, L.nbk, e.stm.rb, e.stm.v, st);
}

// Start the CG of the listed systems from their right-hand sides (zero state, R = F,
// P = M^-1 R, per-column references); a system with a zero right-hand side is done at once.
template <typename T>
static int start_systems(mor_ctx* c, MorEngine& e, Launch& Ln) {
  hipStream_t st = c->st;
  if (Ln.sys.empty()) return 0;
  if (int rc = engine_upload(c, e, Ln)) return rc;
  launch_cg_zero(e.d_sys, Ln.cb, Ln.ncb, st);
  launch_cg_init<T>(e.d_sys, Ln.sp, Ln.nsp, e.sp.rb, e.sp.v, st);
  launch_cg_pstart<T>(e.d_sys, Ln.bk, Ln.nbk, e.stm.rb, e.stm.v, st);
  coarse_start<T>(c, e, Ln);
  launch_cg_start(e.d_sys, Ln.cb, Ln.ncb, 1, 0.0, st);
  HIPCHK(hipGetLastError());
  if (int rc = read_counts(c, e)) return rc;
  for (SysRun* R : Ln.sys) {
    R->phase = e.h_cnt[R->cnt] == 0 ? 1 : 0;
    R->iters = 0;
    R->refines = 0;
  }
  return 0;
}

// Two-level preconditioner set-up of newly admitted requests: for both systems of each,
// A_c = P^T A_II P (FP64), its Cholesky factor R, R^-T from a triangular solve against the
// identity, and A_c^-1 = (R^-T)^T R^-T, batched over the systems.  A request whose A_c is not
// positive definite fails with MOR_EDEVICE.
static int coarse_setup(mor_ctx* c, const std::vector<Live*>& adm) {
  hipStream_t st = c->st;
  std::vector<Live*> ls;
  for (Live* L : adm)
    if (L->q.nc[0] > 0) ls.push_back(L);
  if (ls.empty()) return 0;
  const int ns = 2 * (int)ls.size();
  int tmax = 0, mpmax = 0;
  for (Live* L : ls) {
    tmax = std::max(tmax, std::max(L->q.Tc[0], L->q.Tc[1]));
    mpmax = std::max(mpmax, std::max(L->q.MPc[0], L->q.MPc[1]));
  }
  std::vector<DenseSub> hds(ns);
  std::vector<TrsmDesc> htd(ns);
  GemmBatch gb;
  Sizer z;
  z.add(8 * (size_t)mpmax * mpmax);
  z.add(sizeof(DenseSub) * ns);
  z.add(sizeof(TrsmDesc) * ns);
  z.add(sizeof(GemmDesc) * ns);
  size_t tiles = 0;
  for (Live* L : ls) tiles += (size_t)L->q.Tc[0] * L->q.Tc[0] + (size_t)L->q.Tc[1] * L->q.Tc[1];
  z.add(sizeof(int4) * tiles);
  char* buf = (char*)dalloc(c, z.total + 4096);
  if (!buf) return fail(MOR_ENOMEM, "device allocation failed (coarse set-up)");
  struct G { mor_ctx* c; void* p; ~G() { (void)hipStreamSynchronize(c->st); dfree(c, p); } } guard{c, buf};
  Arena ar{buf, z.total + 4096, 0};
  double* ident = (double*)ar.take(8 * (size_t)mpmax * mpmax);
  DenseSub* dds = (DenseSub*)ar.take(sizeof(DenseSub) * ns);
  TrsmDesc* dtd = (TrsmDesc*)ar.take(sizeof(TrsmDesc) * ns);
  if (!dtd) return fail(MOR_ENOMEM, "arena exhausted (coarse set-up)");
  launch_pad_identity(ident, 0, mpmax, st);
  for (size_t i = 0; i < ls.size(); ++i) {
    Slot& q = ls[i]->q;
    const HostSub& h = *q.h;
    launch_fill_i(q.cinfo, 32, 0, st);
    for (int w = 0; w < 2; ++w) {
      const int ld = w == 0 ? q.ldA : q.ldK;
      const bool kp = w == 1 && q.ls > 0;   // K^+ on all local rows: every column, the rows' coarse blocks
      const int nc = q.nc[w], MPc = q.MPc[w], Tc = q.Tc[w];
      launch_fill(q.cA[w], (int64_t)MPc * MPc, 0.0, st);
      launch_coarse_assemble(q.d->rp, q.d->col, kp ? q.d->rp + 1 : q.d->ii_end, w == 0 ? q.A64 : q.K64,
                             kp ? q.d->rcbL : q.d->rcb, kp ? h.nL : h.nI, q.cA[w], MPc,
                             st);
      launch_pad_identity(q.cA[w], nc, MPc, st);
      launch_fill(q.crc[w], (int64_t)nc * ld, 0.0, st);
      launch_fill(q.cec[w], (int64_t)nc * ld, 0.0, st);
      hds[2 * i + w] = DenseSub{nc, MPc, Tc, q.cA[w], nullptr, nullptr, nullptr, q.cD[w], q.cinfo + 16 * w};
      htd[2 * i + w] = TrsmDesc{ident, mpmax, 0, q.cY[w], MPc, Tc};
      gb.add(gd(nc, nc, nc, q.cY[w], MPc, 1, q.cY[w], MPc, 0, q.cA[w], MPc, 1.0, 0.0, 1));
    }
  }
  if (int rc = gemm_upload(c, gb, ar)) return rc;
  HIPCHK(hipMemcpyAsync(dds, hds.data(), sizeof(DenseSub) * ns, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(dtd, htd.data(), sizeof(TrsmDesc) * ns, hipMemcpyHostToDevice, st));
  for (int p = 0; p < tmax; ++p) {
    launch_potrf_diag(dds, ns, p, st);
    launch_chol_panel(dds, ns, p, tmax, st);
    launch_chol_syrk(dds, ns, p, tmax, st);
  }
  if (int rc = trsm_lt_blocked(c, hds, dds, htd)) return rc;
  gemm_run(c, gb, "coarse_setup");
  HIPCHK(hipGetLastError());
  std::vector<int> hinfo(32 * ls.size());
  for (size_t i = 0; i < ls.size(); ++i)
    HIPCHK(hipMemcpyAsync(&hinfo[32 * i], ls[i]->q.cinfo, 128, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (size_t i = 0; i < ls.size(); ++i)
    if (hinfo[32 * i] != 0 || hinfo[32 * i + 16] != 0) {
      ls[i]->status = MOR_EDEVICE;
      g_err = "subdomain " + std::to_string(ls[i]->q.sd) + ": coarse matrix is not positive definite";
    }
  return 0;
}

// Admit pending requests that fit, assemble them and start their CG (batched).
template <typename T>
static int engine_admit(mor_ctx* c, MorEngine& e) {
  hipStream_t st = c->st;
  std::vector<Live*> adm;
  size_t k = 0;
  for (; k < e.pending.size(); ++k) {
    const Req& r = e.pending[k];
    Live* L = new Live();
    L->id = r.id;
    Slot& q = L->q;
    std::memset(&q, 0, sizeof(q));
    q.sd = r.sd; q.rank = r.rank; q.tol = r.tol; q.prec = r.prec;
    q.ls = r.ls;
    L->om = r.om;
    q.h = &c->subs[r.sd];
    q.d = &c->sdev[r.sd];
    slot_shape(c, q);
    L->bytes = slot_bytes(q);
    if (L->bytes > e.budget) {
      delete L;
      Req done = r;
      done.done = 1;
      done.status = MOR_ENOMEM;
      e.finished[r.id] = done;
      g_err = "subdomain " + std::to_string(r.sd) + " alone exceeds the HBM budget";
      continue;
    }
    if (e.live_bytes + L->bytes > e.budget || (int)e.cnt_free.size() < 2) {
      delete L;
      break;   // FIFO: wait for memory to free up
    }
    L->mem = (char*)dalloc(c, L->bytes);
    if (!L->mem) {
      delete L;
      if (e.live.empty()) return fail(MOR_ENOMEM, "device allocation failed (request)");
      break;
    }
    Arena ar{L->mem, L->bytes, 0};
    if (!slot_layout(q, [&](size_t b) { return ar.take(b); })) {
      dfree(c, L->mem);
      delete L;
      return fail(MOR_ENOMEM, "arena exhausted (request)");
    }
    e.live_bytes += L->bytes;
    e.peak_bytes = std::max(e.peak_bytes, e.live_bytes);
    adm.push_back(L);
  }
  e.pending.erase(e.pending.begin(), e.pending.begin() + k);
  if (adm.empty()) return 0;
  // assembly of the new requests (Section 2 stiffness with kappa, Section 4 H1 matrices, load)
  std::vector<AsmJob> jobs;
  for (Live* L : adm) {
    Slot& q = L->q;
    const HostSub& h = *q.h;
    launch_fill(q.A64, h.rp[h.nL], 0.0, st);
    launch_fill(q.K64, h.rp[h.nL], 0.0, st);
    launch_fill(q.Ki64, h.rpV[h.nV], 0.0, st);
    launch_fill(q.f, h.nL, 0.0, st);
    jobs.push_back({q.h, q.d, q.A64, q.K64, q.Ki64, q.f});
  }
  if (int rc = assemble_batch(c, jobs)) return rc;
  Launch Ln;
  for (Live* L : adm) {
    Slot& q = L->q;
    const HostSub& h = *q.h;
    const int nblk = (int)h.bp.size() - 1;
    if (sizeof(T) == 4) {
      launch_to_f32(q.A64, q.A32, h.rp[h.nL], st);
      launch_to_f32(q.K64, q.K32, h.rp[h.nL], st);
    }
    if (q.s16A) {
      launch_box_coeffs(q.d->spos, q.A64, h.nI, q.s16A, st);
      launch_box_coeffs(q.d->spos, q.K64, h.nI, q.s16K, st);
    }
    const bool sk = q.ls > 0;        // randomized variant: the K system is K^+ on all local rows
    const int nblkL = (int)h.bpL.size() - 1;
    launch_block_inv<T>(q.d->rp, q.d->col, q.A64, q.d->bp, nblk, q.minvA, st);
    launch_block_inv<T>(q.d->rp, q.d->col, q.K64, sk ? q.d->bpL : q.d->bp, sk ? nblkL : nblk, q.minvK, st);
    int nnzII = 0;
    for (int r = 0; r < h.nI; ++r) nnzII += h.ii_end[r] - h.rp[r];
    for (int w = 0; w < 2; ++w) {
      SysRun& R = L->sys[w];
      CgSys& S = R.S;
      std::memset(&S, 0, sizeof(S));
      S.rp = q.d->rp; S.col = q.d->col; S.ii_end = q.d->ii_end;
      S.val32 = w == 0 ? q.A32 : q.K32;
      S.val64 = w == 0 ? q.A64 : q.K64;
      S.f = w == 0 && q.ls == 0 ? q.f : nullptr;
      S.Fd = w == 0 && q.ls > 0 ? q.Fd : nullptr;
      S.nI = h.nI; S.nB = h.nB;
      S.ncols = w == 0 ? q.colsA : q.colsK;
      S.ld = w == 0 ? q.ldA : q.ldK;
      S.X = w == 0 ? q.XA : q.XK; S.R = w == 0 ? q.RA : q.RK;
      S.P = w == 0 ? q.PA : q.PK; S.Q = w == 0 ? q.QA : q.QK;
      S.X64 = w == 0 ? q.XA64 : q.XK64;
      S.tol2 = inner_tol2<T>(c);
      S.rc = q.nc[w] > 0 ? q.crc[w] : nullptr;
      S.ec = q.nc[w] > 0 ? q.cec[w] : nullptr;
      S.nc = q.nc[w];
      R.Ainv = q.nc[w] > 0 ? q.cA[w] : nullptr;
      R.ldac = q.MPc[w];
      S.bp = q.d->bp;
      S.nblk = nblk;
      S.minv = w == 0 ? q.minvA : q.minvK;
      S.htile = (const int4*)q.d->htile;
      S.halo = q.d->halo;
      S.hrowp = q.d->hrowp;
      S.hpe = q.d->hpe;
      S.hpp = q.d->hpp;
      S.hself = q.d->hself;
      R.nhtile = (int)h.htile.size() / 4;
      if (q.s16A) {
        S.s16 = w == 0 ? q.s16A : q.s16K;
        S.smap = q.d->smap;
        S.bx = h.bx; S.bz = h.bz; S.by = h.by;
      }
      if (sk && w == 1) {   // K^+ over [I, B]: every row, every column, dense right-hand sides
        S.nI = h.nL; S.nB = 0;
        S.ii_end = q.d->rp + 1;
        S.f = nullptr;
        S.Fd = q.FdK;
        S.bp = q.d->bpL;
        S.nblk = nblkL;
        S.htile = nullptr; S.halo = nullptr; S.hrowp = nullptr; S.hpe = nullptr; S.hpp = nullptr; S.hself = nullptr;
        R.nhtile = 0;
        S.s16 = nullptr; S.smap = nullptr;
      }
      double* cs = q.colst[w];
      const int ld = S.ld;
      S.pq = cs; S.rz = cs + ld; S.rznew = cs + 2 * ld; S.rz0 = cs + 3 * ld; S.rzF = cs + 4 * ld;
      S.alpha = cs + 5 * ld; S.beta = cs + 6 * ld; S.active = (int*)(cs + 7 * ld);
      R.cnt = e.cnt_free.back();
      e.cnt_free.pop_back();
      S.nactive = e.d_cnt + R.cnt;
      R.phase = 0; R.iters = 0; R.refines = 0; R.nnzII = sk && w == 1 ? h.rp[h.nL] : nnzII;
      if (w == 0 && q.ls > 0) {
        R.phase = 2;   // the sketch solve waits for T = S_B^-1 S_i (randomized variant)
        continue;
      }
      Ln.sys.push_back(&R);
    }
    if (q.ls > 0) {   // right-hand sides [0; S_i] of the first K^+ solve (S_i: M x l, host)
      // one contiguous copy into Wk (free until the sketch T lands there), then a device copy
      // into the padded rows: a strided copy from pageable memory goes row by row
      launch_fill(q.FdK, (int64_t)h.nL * q.ldK, 0.0, st);
      HIPCHK(hipMemcpyAsync(q.Wk, L->om->data(), sizeof(double) * (size_t)q.M * q.ls, hipMemcpyHostToDevice, st));
      launch_copy_rect(q.Wk, q.ls, 0, q.FdK + (size_t)h.nI * q.ldK, q.ldK, q.M, q.ls, st);
    }
  }
  if (int rc = coarse_setup(c, adm)) return rc;
  if (int rc = start_systems<T>(c, e, Ln)) return rc;
  for (Live* L : adm) e.live.push_back(L);
  return 0;
}

// One CG chunk over every system still iterating, then restarts and completions.
template <typename T>
static int engine_chunk(mor_ctx* c, MorEngine& e) {
  hipStream_t st = c->st;
  Launch La;
  for (Live* L : e.live)
    for (int w = 0; w < 2; ++w)
      if (L->sys[w].phase == 0 && !L->status) La.sys.push_back(&L->sys[w]);
  if (La.sys.empty()) return 0;
  if (int rc = engine_upload(c, e, La)) return rc;
  const int chunk = std::max(1, c->opts.cg_chunk);
  // one CG iteration over every admitted system: Q = A P and p'Q, alpha, R -= alpha Q with
  // r'M^-1 r, beta and convergence, X += alpha P and P = M^-1 R + beta P
  auto iteration = [&](hipStream_t s) {
    if (e.sp.halo)
      launch_cg_spmm_halo<T>(e.d_sys, La.hs, La.nhs, c->halo_cap, e.sp.cwb, s);
    else
      launch_cg_spmm<T>(e.d_sys, La.sp, La.nsp, e.sp.rb, e.sp.v, s);
    if (La.nrs > 0) launch_cg_spmm<T>(e.d_sys, La.rs, La.nrs, e.sp.rb, e.sp.v, s);
    launch_cg_spmm_box(e.d_sys, La.bx, La.nbx, s);
    launch_cg_alpha(e.d_sys, La.cb, La.ncb, s);
    launch_cg_update<T>(e.d_sys, La.bk, La.nbk, e.stm.rb, e.stm.v, s);
    if (La.ngt) {   // two-level preconditioner: coarse solve and its part of r'M^-1 r
      launch_coarse_gemm<T>(La.gd, La.gt, La.ngt, s, 1);
      launch_cg_coarse_dot(e.d_sys, La.cb, La.ncb, 0, s);
    }
    launch_cg_beta(e.d_sys, La.cb, La.ncb, s);
    launch_cg_direction<T>(e.d_sys, La.bk, La.nbk, e.stm.rb, e.stm.v, s);
  };
  if (c->opts.use_graph) {
    // The chunk as one HIP graph, captured on a private stream and launched on the library's
    // stream.  Its kernel arguments are the device lists of the last upload, which stay in
    // place (and are re-uploaded identically) while the set of systems is unchanged; any
    // change of systems, list addresses or sizes captures a new graph.
    const std::vector<int64_t> key = {(int64_t)e.sp.cwb, (int64_t)(intptr_t)e.d_sys, (int64_t)(intptr_t)e.d_tiles,
                                      (int64_t)(intptr_t)e.d_cb, La.nsp, La.nbk, La.nhs, La.ncb, chunk,
                                      (int64_t)(intptr_t)La.hs, (int64_t)(intptr_t)La.bk, (int64_t)(intptr_t)La.cb,
                                      (int64_t)c->halo_cap, (int64_t)(intptr_t)La.gd, (int64_t)(intptr_t)La.gt,
                                      La.ngt, (int64_t)(intptr_t)La.bx, La.nbx, (int64_t)(intptr_t)La.rs, La.nrs};
    if (!e.gexec || e.g_sys != La.sys || e.g_key != key) {
      if (e.gexec) HIPCHK(hipGraphExecDestroy(e.gexec));
      e.gexec = nullptr;
      if (!e.cap_st) HIPCHK(hipStreamCreateWithFlags(&e.cap_st, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(e.cap_st, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < chunk; ++k) iteration(e.cap_st);
      HIPCHK(hipStreamEndCapture(e.cap_st, &g));
      const hipError_t ie = hipGraphInstantiate(&e.gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        e.gexec = nullptr;
        return fail(MOR_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(ie));
      }
      e.g_sys = La.sys;
      e.g_key = key;
    }
    ScopedTimer tm(c, "cg_graph", chunk * (La.spmm_bytes + La.box_bytes + La.stream_bytes));
    HIPCHK(hipGraphLaunch(e.gexec, st));
  }
  // The SpMM timers' algorithmic bytes count the columns still iterating (converged columns need
  // no product; the box kernel skips their slices): per system the matrix once, P read and Q
  // written for the active columns, with the active count taken as the mean of the counts at
  // the start and the end of the chunk.  Added once the chunk's end count is known.
  std::vector<int> act0(La.sys.size());
  for (size_t i = 0; i < La.sys.size(); ++i) act0[i] = e.h_cnt[La.sys[i]->cnt];
  for (int k = 0; k < (c->opts.use_graph ? 0 : chunk); ++k) {
    {
      if (!e.sp.halo || La.nhs > 0 || La.nrs > 0) {
        ScopedTimer tm(c, "spmm", 0);
        if (e.sp.halo)
          launch_cg_spmm_halo<T>(e.d_sys, La.hs, La.nhs, c->halo_cap, e.sp.cwb, st);
        else
          launch_cg_spmm<T>(e.d_sys, La.sp, La.nsp, e.sp.rb, e.sp.v, st);
        if (La.nrs > 0) launch_cg_spmm<T>(e.d_sys, La.rs, La.nrs, e.sp.rb, e.sp.v, st);
      }
    }
    if (La.nbx > 0) {
      ScopedTimer tm(c, "spmm_box", 0);
      launch_cg_spmm_box(e.d_sys, La.bx, La.nbx, st);
    }
    launch_cg_alpha(e.d_sys, La.cb, La.ncb, st);
    {
      ScopedTimer tm(c, "cg_update", 0);
      launch_cg_update<T>(e.d_sys, La.bk, La.nbk, e.stm.rb, e.stm.v, st);
    }
    if (La.ngt) {   // two-level preconditioner: coarse solve and its part of r'M^-1 r
      ScopedTimer tm(c, "cg_coarse", La.coarse_flops);
      launch_coarse_gemm<T>(La.gd, La.gt, La.ngt, st, 1);
      launch_cg_coarse_dot(e.d_sys, La.cb, La.ncb, 0, st);
    }
    launch_cg_beta(e.d_sys, La.cb, La.ncb, st);
    {
      ScopedTimer tm(c, "cg_direction", 0);
      launch_cg_direction<T>(e.d_sys, La.bk, La.nbk, e.stm.rb, e.stm.v, st);
    }
  }
  HIPCHK(hipGetLastError());
  if (int rc = read_counts(c, e)) return rc;
  if (c->timing && !c->opts.use_graph) {
    double by[2] = {0.0, 0.0};   // general SpMM, box SpMM
    for (size_t i = 0; i < La.sys.size(); ++i) {
      const CgSys& S = La.sys[i]->S;
      const double act = 0.5 * (act0[i] + e.h_cnt[La.sys[i]->cnt]);
      by[S.s16 != nullptr] += chunk * ((double)La.sys[i]->nnzII * (4.0 + e.elt) + 4.0 * (S.nI + 1) +
                                       2.0 * e.elt * (double)S.nI * act);
    }
    if (c->timers.count("spmm")) c->timers["spmm"].work += by[0];
    if (c->timers.count("spmm_box")) c->timers["spmm_box"].work += by[1];
  }
  // Systems whose inner CG converged: refined systems fold X into the FP64 shadow and test the
  // FP64 residual against the outer target; those above it restart while refinement steps are
  // left, and fail with MOR_ENOTCONV after the last one.  Unrefined systems are done.
  Launch Lr;
  std::vector<SysRun*> fin;
  for (SysRun* R : La.sys) {
    R->iters += chunk;
    if (e.h_cnt[R->cnt] > 0) continue;
    if (R->S.X64 != nullptr) Lr.sys.push_back(R);
    else fin.push_back(R);
  }
  // iteration cap
  for (Live* L : e.live)
    for (int w = 0; w < 2; ++w)
      if (L->sys[w].phase == 0 && L->sys[w].iters > c->opts.max_iter && !L->status) {
        L->status = MOR_ENOTCONV;
        g_err = "block CG did not converge within max_iter";
      }
  if (!Lr.sys.empty()) {
    if (int rc = engine_upload(c, e, Lr)) return rc;
    launch_cg_shadow<T>(e.d_sys, Lr.sp, Lr.nsp, e.sp.rb, e.sp.v, st);
    launch_cg_zero(e.d_sys, Lr.cb, Lr.ncb, st);
    {
      ScopedTimer tm(c, "residual64", 0);
      launch_cg_residual64<T>(e.d_sys, Lr.sp, Lr.nsp, e.sp.rb, e.sp.v, st);
    }
    launch_cg_pstart<T>(e.d_sys, Lr.bk, Lr.nbk, e.stm.rb, e.stm.v, st);
    coarse_start<T>(c, e, Lr);
    const double outer2 = c->opts.refine_rtol * c->opts.refine_rtol;
    launch_cg_start(e.d_sys, Lr.cb, Lr.ncb, 0, outer2, st);
    HIPCHK(hipGetLastError());
    if (int rc = read_counts(c, e)) return rc;
    for (SysRun* R : Lr.sys) {
      if (e.h_cnt[R->cnt] == 0) {   // at the outer target (X holds zeros)
        R->phase = 1;
        continue;
      }
      if (R->refines >= c->opts.refine_steps) {   // corrections used up, residual still above it
        R->phase = 1;
        for (Live* L : e.live)
          if ((&L->sys[0] == R || &L->sys[1] == R) && !L->status) {
            L->status = MOR_ENOTCONV;
            g_err = "FP64 residual refinement did not reach refine_rtol within refine_steps corrections";
          }
        continue;
      }
      R->refines++;
    }
  }
  for (SysRun* R : fin) R->phase = 1;
  return 0;
}

// Dense stage of the requests whose two solves finished.
static int dense_stage(mor_ctx* c, std::vector<Live*>& done);
static int project_local(mor_ctx* c, Arena& ar, const std::vector<Slot*>& sl, const std::vector<Live*>& done,
                         int eig_iters);

// ----------------------------------------------------------------- randomized variant (f1)
// Section 6's randomized SVD with two left solves, for requests with a sketch S_i (l <= 64
// columns).  Stages, each batched over the requests that reach it:
//   after the H1 solve:  S_B, R_BB = chol(S_B), T = R_BB^-1 S_i and the sketch solve
//                        A_II X = [-A_IB T | f_I];
//   after that solve:    Y = C X[:, :l]; a K_i-orthonormal basis W of span(Y) from the
//                        eigendecomposition of Y^T K_i Y (directions below 1e-10 of the largest
//                        eigenvalue dropped), applied twice; the left solve A_II G = C^T K_i W;
//   after the left solve: B^T = R_BB^-T A_BI G (= the transpose of W^T K_i Z R_BB^-1 up to the
//                        sign of Z), the top eigenpairs of B B^T, the basis [q_0, W U_k] and the
//                        local projection.
struct StageBuf {
  mor_ctx* c;
  char* p = nullptr;
  Arena ar;
  StageBuf(mor_ctx* cc, size_t bytes) : c(cc) {
    p = (char*)dalloc(c, bytes);
    ar = Arena{p, p ? bytes : 0, 0};
  }
  ~StageBuf() {
    (void)hipStreamSynchronize(c->st);
    dfree(c, p);
  }
};

// device pointer table of one field over the slots
template <typename F>
static double** ptr_table(mor_ctx* c, Arena& ar, const std::vector<Slot*>& sl, F get) {
  std::vector<double*> h(sl.size());
  for (size_t i = 0; i < sl.size(); ++i) h[i] = get(*sl[i]);
  double** d = (double**)ar.take(sizeof(double*) * std::max<size_t>(1, h.size()));
  if (d && !h.empty()) (void)hipMemcpyAsync(d, h.data(), sizeof(double*) * h.size(), hipMemcpyHostToDevice, c->st);
  return d;
}
static int* int_table(mor_ctx* c, Arena& ar, const std::vector<int>& h) {
  int* d = (int*)ar.take(sizeof(int) * std::max<size_t>(1, h.size()));
  if (d && !h.empty()) (void)hipMemcpyAsync(d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, c->st);
  return d;
}

// eigenpairs (descending) of the symmetric s_i x s_i matrices in H, into Ss and theta
static int small_eig(mor_ctx* c, Arena& ar, const std::vector<Slot*>& sl, const std::vector<int>& s_of,
                     std::vector<std::vector<double>>& theta) {
  hipStream_t st = c->st;
  const int ns = (int)sl.size();
  double** PH = ptr_table(c, ar, sl, [](Slot& q) { return q.H; });
  double** PS = ptr_table(c, ar, sl, [](Slot& q) { return q.Ss; });
  double** PT = ptr_table(c, ar, sl, [](Slot& q) { return q.theta; });
  int* ds = int_table(c, ar, s_of);
  if (!PH || !PS || !PT || !ds) return fail(MOR_ENOMEM, "arena exhausted (small eigen)");
  launch_jacobi(PH, PS, PT, ds, ns, 64, st);
  theta.assign(ns, {});
  for (int i = 0; i < ns; ++i) {
    theta[i].resize(std::max(s_of[i], 1));
    HIPCHK(hipMemcpyAsync(theta[i].data(), sl[i]->theta, 8 * theta[i].size(), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return 0;
}
static int rank_of(const std::vector<double>& th, int s) {
  int r = 0;
  for (int j = 0; j < s; ++j) r += (th[j] > 0.0 && th[j] > 1e-10 * th[0]) ? 1 : 0;
  return r;
}

// After the first K^+ solve: the sketch T = S_B^-1 S_i is the B block of its solution; the
// sketch solve A_II X = [-A_IB T | f_I] starts.
template <typename T>
static int rsvd_after_kp1(mor_ctx* c, MorEngine& e, std::vector<Live*>& ls) {
  hipStream_t st = c->st;
  Launch Ln;
  for (Live* L : ls) {
    Slot& q = L->q;
    const HostSub& h = *q.h;
    launch_fill(q.Wk, (int64_t)q.MP * 64, 0.0, st);
    launch_copy_rect(q.Ec + (size_t)h.nI * q.ldEc, q.ldEc, 0, q.Wk, 64, q.M, q.ls, st);
    launch_rhs_sketch(q.d->rp, q.d->col, q.d->ii_end, q.A64, q.f, h.nI, q.Wk, q.ls, q.Fd, q.ldA, st);
    SysRun& R = L->sys[0];
    R.S.ncols = q.colsA;
    L->stage = 1;
    Ln.sys.push_back(&R);
  }
  return start_systems<T>(c, e, Ln);
}

template <typename T>
static int rsvd_after_sketch(mor_ctx* c, MorEngine& e, std::vector<Live*>& ls) {
  hipStream_t st = c->st;
  const int ns = (int)ls.size();
  std::vector<Slot*> sl(ns);
  size_t tiles = 0;
  for (int i = 0; i < ns; ++i) {
    sl[i] = &ls[i]->q;
    tiles += 4 * ((size_t)(sl[i]->h->nV + 63) / 64 + 2) + 8;
  }
  StageBuf buf(c, ns * (16 * sizeof(double*) + 4 * sizeof(int) + 4 * sizeof(GemmDesc)) + 4 * tiles * sizeof(int4) +
                      64 * 256);
  if (!buf.p) return fail(MOR_ENOMEM, "device allocation failed (sketch stage)");
  // Y = C X[:, :l], K_i Y and the Gram Y^T K_i Y
  GemmBatch g1;
  for (Slot* q : sl) {
    const HostSub& h = *q->h;
    launch_copy_col(q->Xc + q->ls, q->ldXc, q->q0v, 1, h.nV, st);   // q_0 (load column)
    launch_spmm64_rows(q->d->rpV, q->d->colV, q->Ki64, h.nV, h.nV, q->Xc, q->ldXc, q->ls, q->Yk, 64, st);
    g1.add(gd(q->ls, q->ls, h.nV, q->Xc, q->ldXc, 1, q->Yk, 64, 0, q->H, q->ls));
  }
  if (int rc = gemm_upload(c, g1, buf.ar)) return rc;
  gemm_run(c, g1, "sketch_gram");
  std::vector<int> s_of(ns);
  for (int i = 0; i < ns; ++i) s_of[i] = sl[i]->ls;
  std::vector<std::vector<double>> th;
  if (int rc = small_eig(c, buf.ar, sl, s_of, th)) return rc;
  // first pass: W1 = Y V diag(th^-1/2), K_i W1 = (K_i Y) V diag(th^-1/2)
  GemmBatch g2;
  std::vector<int> r1(ns);
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    r1[i] = rank_of(th[i], q.ls);
    launch_whiten(q.Ss, q.theta, q.ls, r1[i], q.Vs, st);
    g2.add(gd(h.nV, 64, q.ls, q.Xc, q.ldXc, 0, q.Vs, 64, 0, q.Wt, 64));
    g2.add(gd(h.nV, 64, q.ls, q.Yk, 64, 0, q.Vs, 64, 0, q.KWt, 64));
  }
  if (int rc = gemm_upload(c, g2, buf.ar)) return rc;
  gemm_run(c, g2, "sketch_orth");
  // second pass on W1 (its Gram is close to the identity): W = W1 V2 diag(th2^-1/2)
  GemmBatch g3;
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    g3.add(gd(r1[i], r1[i], h.nV, q.Wt, 64, 1, q.KWt, 64, 0, q.H, r1[i]));
  }
  if (int rc = gemm_upload(c, g3, buf.ar)) return rc;
  gemm_run(c, g3, "sketch_orth");
  if (int rc = small_eig(c, buf.ar, sl, r1, th)) return rc;
  GemmBatch g4;
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    q.rk = rank_of(th[i], r1[i]);
    launch_whiten(q.Ss, q.theta, r1[i], q.rk, q.Vs, st);
    g4.add(gd(h.nV, 64, r1[i], q.Wt, 64, 0, q.Vs, 64, 0, q.Yk, 64));   // W (into Yk)
  }
  if (int rc = gemm_upload(c, g4, buf.ar)) return rc;
  gemm_run(c, g4, "sketch_orth");
  Launch Ln;
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    launch_spmm64_rows(q.d->rpV, q.d->colV, q.Ki64, h.nV, h.nV, q.Yk, 64, q.rk, q.KWt, 64, st);   // K_i W
    launch_rhs_rows(q.KWt, h.nV, q.rk, h.nI, q.Fd, q.ldA, st);   // C^T K_i W
    SysRun& R = ls[i]->sys[0];
    ls[i]->iters_prev += R.iters;
    R.S.ncols = q.rk;
    ls[i]->stage = 2;
    if (q.rk < 1) {
      ls[i]->status = MOR_EDEVICE;
      g_err = "subdomain " + std::to_string(q.sd) + ": the sketch has no significant direction";
      continue;
    }
    Ln.sys.push_back(&R);
  }
  return start_systems<T>(c, e, Ln);
}

// After the left solve A_II G = C^T K_i W: V = A_BI G (M x rk, up to the sign of the lifting),
// and the second K^+ solve with right-hand sides [0; V] gives S_B^-1 V.
template <typename T>
static int rsvd_after_left(mor_ctx* c, MorEngine& e, std::vector<Live*>& ls) {
  hipStream_t st = c->st;
  Launch Ln;
  for (Live* L : ls) {
    Slot& q = L->q;
    const HostSub& h = *q.h;
    launch_bi_product(q.d->rp, q.d->col, q.A64, h.nI, h.nB, q.MP, q.Xc, q.ldXc, q.rk, q.Vb, st);
    launch_fill(q.FdK, (int64_t)h.nL * q.ldK, 0.0, st);
    launch_copy_rect(q.Vb, 64, 0, q.FdK + (size_t)h.nI * q.ldK, q.ldK, q.M, q.rk, st);
    SysRun& R = L->sys[1];
    L->iters_prev += L->sys[0].iters;
    R.S.ncols = q.rk;
    L->stage = 3;
    Ln.sys.push_back(&R);
  }
  return start_systems<T>(c, e, Ln);
}

static int rsvd_finish(mor_ctx* c, std::vector<Live*>& ls) {
  hipStream_t st = c->st;
  const int ns = (int)ls.size();
  std::vector<Slot*> sl(ns);
  size_t tiles = 0;
  for (int i = 0; i < ns; ++i) {
    sl[i] = &ls[i]->q;
    tiles += 4 * ((size_t)(sl[i]->h->nV + 63) / 64 + (sl[i]->h->nP + 63) / 64 + 4) + 8;
  }
  StageBuf buf(c, ns * (sizeof(DenseSub) + sizeof(TrsmDesc) + 16 * sizeof(double*) + 4 * sizeof(GemmDesc)) +
                      4 * tiles * sizeof(int4) + 64 * 256);
  if (!buf.p) return fail(MOR_ENOMEM, "device allocation failed (sketch stage)");
  // B B^T = V^T S_B^-1 V (B = W R_BB^-1 with V = W^T up to sign) and its eigenpairs: sigma^2 and
  // the left singular vectors U
  GemmBatch g1;
  std::vector<int> s_of(ns);
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    launch_copy_rect(q.Ec + (size_t)h.nI * q.ldEc, q.ldEc, 0, q.Yb, 64, q.M, q.rk, st);   // S_B^-1 V
    s_of[i] = q.rk;
    g1.add(gd(q.rk, q.rk, q.M, q.Vb, 64, 1, q.Yb, 64, 0, q.H, q.rk));
  }
  if (int rc = gemm_upload(c, g1, buf.ar)) return rc;
  gemm_run(c, g1, "sketch_svd");
  std::vector<std::vector<double>> th;
  if (int rc = small_eig(c, buf.ar, sl, s_of, th)) return rc;
  // truncation and the basis [q_0, W U_k]
  GemmBatch gV;
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    std::vector<double> sg(q.rk);
    for (int j = 0; j < q.rk; ++j) sg[j] = std::sqrt(std::max(th[i][j], 0.0));
    q.k_eff = truncation_rank(sg, q.rank, q.tol, std::max(q.rk - 1, 1));
    q.k_eff = std::min(q.k_eff, q.rk);
    SubResult& R = c->res[q.sd];
    R.sigma = sg;
    R.k_eff = q.k_eff;
    const int k1 = q.k_eff + 1;
    if (R.d_V) pfree(c, R.d_V);
    if (R.d_Pm) pfree(c, R.d_Pm);
    R.d_V = (double*)palloc(c, 8 * (size_t)h.nV * k1);
    R.d_Pm = (double*)palloc(c, 8 * (size_t)k1 * (k1 + 1));
    if (!R.d_V || !R.d_Pm) return fail(MOR_ENOMEM, "device allocation failed (basis)");
    launch_copy_col(q.q0v, 1, R.d_V, k1, h.nV, st);
    if (q.k_eff > 0) gV.add(gd(h.nV, q.k_eff, q.rk, q.Yk, 64, 0, q.Ss, q.rk, 0, R.d_V + 1, k1));
  }
  if (int rc = gemm_upload(c, gV, buf.ar)) return rc;
  gemm_run(c, gV, "basis");
  for (Live* L : ls) L->stage = 4;
  return project_local(c, buf.ar, sl, ls, 0);
}

template <typename T>
static int engine_tick(mor_ctx* c, MorEngine& e) {
  {
    HostTimer ht(c, "host_admit");
    if (int rc = engine_admit<T>(c, e)) return rc;
  }
  {
    HostTimer ht(c, "host_chunk");
    if (int rc = engine_chunk<T>(c, e)) return rc;
  }
  {   // randomized variant: move the requests whose current solve finished to their next stage
    HostTimer ht(c, "host_stage");
    std::vector<Live*> s1, s2, s3, s4;
    for (Live* L : e.live) {
      if (L->status || L->q.ls == 0) continue;
      if (L->stage == 0 && L->sys[1].phase == 1) s1.push_back(L);
      else if (L->stage == 1 && L->sys[0].phase == 1) s2.push_back(L);
      else if (L->stage == 2 && L->sys[0].phase == 1) s3.push_back(L);
      else if (L->stage == 3 && L->sys[1].phase == 1) s4.push_back(L);
    }
    auto run = [&](std::vector<Live*>& v, int rc) {
      if (rc)
        for (Live* L : v)
          if (!L->status) L->status = rc;
    };
    if (!s4.empty()) run(s4, rsvd_finish(c, s4));
    if (!s3.empty()) run(s3, rsvd_after_left<T>(c, e, s3));
    if (!s2.empty()) run(s2, rsvd_after_sketch<T>(c, e, s2));
    if (!s1.empty()) run(s1, rsvd_after_kp1<T>(c, e, s1));
  }
  std::vector<Live*> ready, keep;
  bool iterating = false;
  for (Live* L : e.live) {
    if (L->status) ready.push_back(L);
    else if (L->q.ls > 0 ? L->stage == 4 : (L->sys[0].phase == 1 && L->sys[1].phase == 1)) ready.push_back(L);
    else {
      keep.push_back(L);
      iterating = true;
    }
  }
  if (ready.empty()) return 0;
  // Batch the dense stage: wait for more finished requests while others still iterate,
  // unless enough are ready or pending requests wait for the memory they hold.
  const int want = c->opts.dense_batch > 0 ? c->opts.dense_batch : 16;
  bool failed = false, dense = false;
  for (Live* L : ready) {
    failed |= L->status != 0;
    dense |= L->status == 0 && L->q.ls == 0;
  }
  if (iterating && dense && !failed && (int)ready.size() < want && e.pending.empty()) return 0;
  std::vector<Live*> ok;
  for (Live* L : ready)
    if (!L->status && L->q.ls == 0) ok.push_back(L);
  int rc = 0;
  if (!ok.empty()) {
    HostTimer ht(c, "host_dense");
    rc = dense_stage(c, ok);
    if (rc)
      for (Live* L : ok)
        if (!L->status) L->status = rc;
  }
  for (Live* L : ready) {
    Req r;
    r.id = L->id;
    r.sd = L->q.sd;
    r.rank = L->q.rank;
    r.prec = L->q.prec;
    r.tol = L->q.tol;
    r.done = 1;
    r.status = L->status;
    e.finished[r.id] = r;
    for (int w = 0; w < 2; ++w) e.cnt_free.push_back(L->sys[w].cnt);
    (void)hipStreamSynchronize(c->st);
    dfree(c, L->mem);
    e.live_bytes -= L->bytes;
    delete L;
  }
  e.live = keep;
  c->projected = 0;
  c->solved = 0;
  return 0;
}

static MorEngine& engine_for(mor_ctx* c, int prec);
static int tick_all(mor_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    MorEngine* e = c->eng[k];
    if (!e || (e->pending.empty() && e->live.empty())) continue;
    const int rc = k == 0 ? engine_tick<float>(c, *e) : engine_tick<double>(c, *e);
    if (rc) return rc;
  }
  return 0;
}
static bool engines_idle(mor_ctx* c) {
  for (int k = 0; k < 2; ++k)
    if (c->eng[k] && (!c->eng[k]->pending.empty() || !c->eng[k]->live.empty())) return false;
  return true;
}

// ------------------------------------------------------------------------------- dense stage
template <typename F>
static double** ptr_table(mor_ctx* c, Arena& ar, const std::vector<Slot*>& sl, F get);
static int small_eig(mor_ctx* c, Arena& ar, const std::vector<Slot*>& sl, const std::vector<int>& s_of,
                     std::vector<std::vector<double>>& theta);

// Relative eigenvalue drop of a subdomain block (basis update, block preconditioner): update_drop
// if set, else the accuracy the basis was computed to, below which a block's directions are
// noise: the solves' target refine_rtol (at least 1e-10) for FP64 and FP64-refined bases, 1e-6
// where FP32 solves or the BF16 Gram set it.
// Relative eigenvalue below which the basis update drops a direction of the stitched block: only
// numerically dependent combinations of the stitched columns (near the rounding level of an FP64
// eigendecomposition), whatever the precision the basis came from.  A small eigenvalue measures
// a direction's energy per unit coefficient, not its accuracy: on high-contrast coefficients the
// blocks hold directions near 1e-8 of the largest that carry a large share of the solution.
static double drop_of(const mor_ctx* c, int prec) {
  (void)prec;
  if (c->opts.update_drop > 0) return c->opts.update_drop;
  return 1e-10;
}

// The basis update of Section 6, step 2, which diagonalises the diagonal blocks of the reduced
// system.  Reading (the paper defers the details to its source code): eigendecomposition
// Q^T A_ii Q = U Lambda U^T of each stitched block, eigenvalues below update_drop * lambda_max
// removed, basis Q U_r Lambda_r^-1/2 (its block is the identity) and load Lambda_r^-1/2 U_r^T
// Q^T f.  Runs on the blocks project_local left in R.Aii / R.d_Pm.
static int basis_update(mor_ctx* c, const std::vector<Slot*>& sl) {
  hipStream_t st = c->st;
  const int ns = (int)sl.size();
  size_t tiles = 0;
  for (Slot* q : sl) tiles += (size_t)(q->h->nV + 63) / 64 + 4;
  StageBuf buf(c, ns * (8 * sizeof(double*) + sizeof(int) + 8 * 64 + 4 * sizeof(GemmDesc)) + 2 * tiles * sizeof(int4) +
                      32 * 256);
  if (!buf.p) return fail(MOR_ENOMEM, "device allocation failed (basis update)");
  Arena& ar = buf.ar;
  std::vector<int> s_of(ns);
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    SubResult& R = c->res[q.sd];
    s_of[i] = R.dim;
    HIPCHK(hipMemcpyAsync(q.H, R.Aii.data(), 8 * R.Aii.size(), hipMemcpyHostToDevice, st));
  }
  std::vector<std::vector<double>> th;
  if (int rc = small_eig(c, ar, sl, s_of, th)) return rc;
  GemmBatch gV, gB;
  std::vector<double*> newV(ns), newb(ns);
  std::vector<int> r(ns);
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    SubResult& R = c->res[q.sd];
    r[i] = 0;
    const double drop = drop_of(c, q.prec);
    for (int j = 0; j < R.dim; ++j) r[i] += (th[i][j] > drop * th[i][0]) ? 1 : 0;
    r[i] = std::max(r[i], 1);
    launch_whiten(q.Ss, q.theta, R.dim, r[i], q.Bk, st);   // U_r Lambda_r^-1/2 (dim x 64)
    newV[i] = (double*)palloc(c, 8 * (size_t)h.nV * r[i]);
    newb[i] = (double*)ar.take(8 * 64);
    if (!newV[i] || !newb[i]) return fail(MOR_ENOMEM, "device allocation failed (basis update)");
    gV.add(gd(h.nV, r[i], R.dim, R.d_V, R.dim, 0, q.Bk, 64, 0, newV[i], r[i]));
    gB.add(gd(r[i], 1, R.dim, q.Bk, 64, 1, R.d_Pm + R.dim, R.dim + 1, 0, newb[i], 1));
  }
  if (int rc = gemm_upload(c, gV, ar)) return rc;
  if (int rc = gemm_upload(c, gB, ar)) return rc;
  gemm_run(c, gV, "basis_update");
  gemm_run(c, gB, "basis_update");
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    SubResult& R = c->res[q.sd];
    pfree(c, R.d_V);
    R.d_V = newV[i];
    R.dim = r[i];
    R.Aii.assign((size_t)r[i] * r[i], 0.0);
    for (int a = 0; a < r[i]; ++a) R.Aii[(size_t)a * r[i] + a] = 1.0;
    R.bi.assign(r[i], 0.0);
    HIPCHK(hipMemcpy(R.bi.data(), newb[i], 8 * r[i], hipMemcpyDeviceToHost));
    // [I | b~] for the reduced assembly
    std::vector<double> pm((size_t)r[i] * (r[i] + 1), 0.0);
    for (int a = 0; a < r[i]; ++a) {
      pm[(size_t)a * (r[i] + 1) + a] = 1.0;
      pm[(size_t)a * (r[i] + 1) + r[i]] = R.bi[a];
    }
    pfree(c, R.d_Pm);
    R.d_Pm = (double*)palloc(c, 8 * pm.size());
    if (!R.d_Pm) return fail(MOR_ENOMEM, "device allocation failed (basis update)");
    HIPCHK(hipMemcpy(R.d_Pm, pm.data(), 8 * pm.size(), hipMemcpyHostToDevice));
  }
  return 0;
}

// Local projection of finished bases (Section 6, step 2): with R.d_V = V_i (|V_i| x (k+1))
// filled, [Q^T A_PP Q | Q^T f_P] over the leading |P_i| rows, then the host copies of the
// local block and load, and the request's statistics.
static int project_local(mor_ctx* c, Arena& ar, const std::vector<Slot*>& sl, const std::vector<Live*>& done,
                         int eig_iters) {
  hipStream_t st = c->st;
  const int ns = (int)sl.size();
  GemmBatch gP;
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    SubResult& R = c->res[q.sd];
    const int k1 = q.k_eff + 1;
    launch_spmm64_rows(q.d->rp, q.d->col, q.A64, h.nP, h.nP, R.d_V, k1, k1, q.Yf, k1 + 1, st);
    launch_copy_col(q.f, 1, q.Yf + k1, k1 + 1, h.nP, st);
    gP.add(gd(k1, k1 + 1, h.nP, R.d_V, k1, 1, q.Yf, k1 + 1, 0, R.d_Pm, k1 + 1));
  }
  if (int rc = gemm_upload(c, gP, ar)) return rc;
  gemm_run(c, gP, "project_local");
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    SubResult& R = c->res[q.sd];
    const int k1 = q.k_eff + 1;
    std::vector<double> pm((size_t)k1 * (k1 + 1));
    HIPCHK(hipMemcpy(pm.data(), R.d_Pm, 8 * pm.size(), hipMemcpyDeviceToHost));
    R.Aii.assign((size_t)k1 * k1, 0.0);
    R.bi.assign(k1, 0.0);
    for (int a = 0; a < k1; ++a) {
      for (int b = 0; b < k1; ++b)
        R.Aii[(size_t)a * k1 + b] = 0.5 * (pm[(size_t)a * (k1 + 1) + b] + pm[(size_t)b * (k1 + 1) + a]);
      R.bi[a] = pm[(size_t)a * (k1 + 1) + k1];
    }
    R.dim = k1;
    R.cg_a = done[i]->sys[0].iters + done[i]->iters_prev;
    R.cg_k = done[i]->sys[1].iters;
    R.refine = std::max(done[i]->sys[0].refines, done[i]->sys[1].refines);
    R.eig = eig_iters;
    R.prec = q.prec;
    R.reduced = done[i]->status == 0;
  }
  if (c->opts.basis_update) return basis_update(c, sl);
  return 0;
}

static int dense_stage(mor_ctx* c, std::vector<Live*>& done) {
  hipStream_t st = c->st;
  const int ns = (int)done.size();
  std::vector<Slot*> sl(ns);
  for (int i = 0; i < ns; ++i) sl[i] = &done[i]->q;
  // scratch for descriptors and pointer tables of this stage
  size_t gemm_tiles = 0;
  for (Slot* q : sl) gemm_tiles += (size_t)(q->T + 2) * (q->T + 2) + 16 * (size_t)(q->T + 2) + 256;
  size_t bf_tiles = 0;   // split-precision Gram: split tiles of X_C and K_i X_C, symmetric C tiles
  for (Slot* q : sl)
    if (q->prec == MOR_BF16_SPLIT)
      bf_tiles += 2 * (size_t)(q->MB / 64) * (q->kpV / 64) + (size_t)(q->MB / 128) * (q->MB / 128 + 1) / 2;
  const size_t bytes = 2 * 8 * gemm_tiles * sizeof(int4) + 32 * ns * sizeof(GemmDesc) + ns * (sizeof(DenseSub) + 2 * sizeof(TrsmDesc)) +
                       8 * (size_t)ns * 20 + 8 * (size_t)ns * 64 + 16 * 4096 + bf_tiles * sizeof(int4) +
                       ns * (2 * sizeof(SplitDesc) + sizeof(BfGramDesc)) + 4 * 256;
  char* buf = (char*)dalloc(c, bytes);
  if (!buf) return fail(MOR_ENOMEM, "device allocation failed (dense stage)");
  struct Guard {
    mor_ctx* c; void* p;
    ~Guard() { (void)hipStreamSynchronize(c->st); dfree(c, p); }
  } guard{c, buf};
  Arena ar{buf, bytes, 0};
  int rc = 0;
  {
    Slot& q = *sl[0];
    const HostSub& h = *q.h;
    dump(c, "A64", q.A64, 8 * (size_t)h.rp[h.nL]);
    dump(c, "K64", q.K64, 8 * (size_t)h.rp[h.nL]);
    dump(c, "Ki64", q.Ki64, 8 * (size_t)h.rpV[h.nV]);
    dump(c, "f", q.f, 8 * (size_t)h.nL);
  }
  // ---- FP64 views of the solutions
  for (Slot* q : sl) {
    const HostSub& h = *q->h;
    if (q->fp32 && !q->refine) {
      launch_to_f64_block((const float*)q->XA, q->ldA, q->Xc, q->ldXc, h.nV, q->colsA, st);
      launch_to_f64_block((const float*)q->XK, q->ldK, q->Ec, q->ldEc, h.nI, q->colsK, st);
    }
  }
  // ---- G1 = X_C^T K_i X_C (lifted interface functions in the H1(omega_i) inner product)
  // (FP64 MFMA, or BF16 MFMA on hi/lo splits of both operands for MOR_BF16_SPLIT)
  GemmBatch gG;
  std::vector<SplitDesc> spd;
  std::vector<BfGramDesc> bgd;
  std::vector<int4> spt, bgt;
  double bf_flops = 0;
  for (Slot* q : sl) {
    const HostSub& h = *q->h;
    launch_fill(q->G, (int64_t)q->MP * q->MP, 0.0, st);
    launch_spmm64_rows(q->d->rpV, q->d->colV, q->Ki64, h.nV, h.nV, q->Xc, q->ldXc, q->M, q->Y, q->ldK, st);
    if (q->prec == MOR_BF16_SPLIT) {
      const int id = (int)spd.size();
      spd.push_back(SplitDesc{q->Xc, q->ldXc, h.nV, q->M, q->kpV, q->MB, q->Xh, q->Xl});
      spd.push_back(SplitDesc{q->Y, q->ldK, h.nV, q->M, q->kpV, q->MB, q->Yh, q->Yl});
      for (int t = 0; t < 2; ++t)
        for (int a = 0; a < q->MB / 64; ++a)
          for (int v = 0; v < q->kpV / 64; ++v) spt.push_back(make_int4(id + t, a, v, 0));
      const int gid = (int)bgd.size();
      bgd.push_back(BfGramDesc{q->M, q->kpV, q->Xh, q->Xl, q->Yh, q->Yl, q->G, q->MP});
      for (int i = 0; i < q->MB / 128; ++i)
        for (int j = i; j < q->MB / 128; ++j) bgt.push_back(make_int4(gid, i, j, 0));
      bf_flops += 3.0 * q->M * q->M * h.nV;   // three BF16 products over the symmetric half
    } else {
      gG.add(gd(q->M, q->M, h.nV, q->Xc, q->ldXc, 1, q->Y, q->ldK, 0, q->G, q->MP, 1.0, 0.0, 1));
    }
  }
  if ((rc = gemm_upload(c, gG, ar))) return rc;
  gemm_run(c, gG, "gram");
  if (!bgd.empty()) {
    SplitDesc* d_spd = (SplitDesc*)ar.take(sizeof(SplitDesc) * spd.size());
    BfGramDesc* d_bgd = (BfGramDesc*)ar.take(sizeof(BfGramDesc) * bgd.size());
    int4* d_spt = (int4*)ar.take(sizeof(int4) * spt.size());
    int4* d_bgt = (int4*)ar.take(sizeof(int4) * bgt.size());
    if (!d_spd || !d_bgd || !d_spt || !d_bgt) return fail(MOR_ENOMEM, "arena exhausted (bf16 gram)");
    HIPCHK(hipMemcpyAsync(d_spd, spd.data(), sizeof(SplitDesc) * spd.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_bgd, bgd.data(), sizeof(BfGramDesc) * bgd.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_spt, spt.data(), sizeof(int4) * spt.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_bgt, bgt.data(), sizeof(int4) * bgt.size(), hipMemcpyHostToDevice, st));
    {
      ScopedTimer tm(c, "gram_split", 0);
      launch_split_bf16(d_spd, d_spt, (int)spt.size(), st);
    }
    {
      ScopedTimer tm(c, "gram_bf16", bf_flops);
      launch_gram_bf16(d_bgd, d_bgt, (int)bgt.size(), st);
    }
  }
  // ---- S_B = K_BB + K_BI E (Lemma 4.1), padded with the identity
  for (Slot* q : sl) {
    const HostSub& h = *q->h;
    ScopedTimer tm(c, "schur", 0);
    launch_schur(q->d->rp, q->d->col, q->K64, h.nI, h.nB, q->Ec, q->ldEc, q->S, q->MP, st);
    launch_pad_identity(q->S, q->M, q->MP, st);
    launch_symmetrize(q->S, q->MP, st);
  }
  {
    Slot& q = *sl[0];
    const HostSub& h = *q.h;
    dump(c, "Xc", q.Xc, 8 * (size_t)h.nV * q.ldXc);
    dump(c, "Ec", q.Ec, 8 * (size_t)h.nI * q.ldEc);
    dump(c, "G", q.G, 8 * (size_t)q.MP * q.MP);
    dump(c, "S", q.S, 8 * (size_t)q.MP * q.MP);
  }
  // ---- R = chol(S_B), C = R^-T G1 R^-1
  std::vector<DenseSub> hds(ns);
  int tmax = 0;
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    hds[i] = DenseSub{q.M, q.MP, q.T, q.S, q.G, q.W, q.C, q.Dinv, q.info};
    tmax = std::max(tmax, q.T);
    launch_fill_i(q.info, 16, 0, st);
  }
  DenseSub* dds = (DenseSub*)ar.take(sizeof(DenseSub) * ns);
  TrsmDesc* dtd = (TrsmDesc*)ar.take(sizeof(TrsmDesc) * ns * 2);
  if (!dtd) return fail(MOR_ENOMEM, "arena exhausted (dense)");
  HIPCHK(hipMemcpyAsync(dds, hds.data(), sizeof(DenseSub) * ns, hipMemcpyHostToDevice, st));
  {
    double fl = 0;
    for (Slot* q : sl) fl += (double)q->MP * q->MP * q->MP / 3.0;
    ScopedTimer tm(c, "potrf", fl);
    for (int p = 0; p < tmax; ++p) {
      launch_potrf_diag(dds, ns, p, st);
      launch_chol_panel(dds, ns, p, tmax, st);
      launch_chol_syrk(dds, ns, p, tmax, st);
    }
  }
  {
    std::vector<int> hinfo(ns * 16);
    for (int i = 0; i < ns; ++i) HIPCHK(hipMemcpyAsync(&hinfo[i * 16], sl[i]->info, 64, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < ns; ++i)
      if (hinfo[i * 16] != 0) {
        done[i]->status = MOR_EDEVICE;
        g_err = "subdomain " + std::to_string(sl[i]->sd) + ": S_B is not positive definite (pivot " +
                std::to_string(hinfo[i * 16]) + ")";
      }
  }
  std::vector<TrsmDesc> htd(2 * ns);
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    htd[i] = TrsmDesc{q.G, q.MP, 0, q.W, q.MP, q.T};
    htd[ns + i] = TrsmDesc{q.W, q.MP, 1, q.C, q.MP, q.T};
  }
  HIPCHK(hipMemcpyAsync(dtd, htd.data(), sizeof(TrsmDesc) * 2 * ns, hipMemcpyHostToDevice, st));
  {
    double fl = 0;
    for (Slot* q : sl) fl += 2.0 * (double)q->MP * q->MP * q->MP;
    ScopedTimer tm(c, "trsm", fl);
    if ((rc = trsm_lt_blocked(c, hds, dds, std::vector<TrsmDesc>(htd.begin(), htd.begin() + ns)))) return rc;
    if ((rc = trsm_lt_blocked(c, hds, dds, std::vector<TrsmDesc>(htd.begin() + ns, htd.end())))) return rc;
  }
  for (Slot* q : sl) launch_symmetrize(q->C, q->MP, st);
  {
    Slot& q = *sl[0];
    dump(c, "R", q.S, 8 * (size_t)q.MP * q.MP);
    dump(c, "C", q.C, 8 * (size_t)q.MP * q.MP);
  }

  // ---- top eigenpairs of C by subspace iteration with Rayleigh-Ritz
  int smax = 0, maxrows = 0;
  std::vector<int> s_of(ns), rows_of(ns), M_of(ns);
  for (int i = 0; i < ns; ++i) {
    s_of[i] = sl[i]->s;
    rows_of[i] = sl[i]->MP;
    M_of[i] = sl[i]->M;
    smax = std::max(smax, sl[i]->s);
    maxrows = std::max(maxrows, sl[i]->MP);
  }
  int* d_s = (int*)ar.take(4 * ns);
  int* d_rows = (int*)ar.take(4 * ns);
  int* d_M = (int*)ar.take(4 * ns);
  int* d_info2 = (int*)ar.take(4 * ns);
  // pointer tables: Vb Yb Ub Zb Vn Tb H Ss G2 Rinv theta resid Bk Wk
  const int NP = 14;
  double** dptr = (double**)ar.take(sizeof(double*) * ns * NP);
  if (!dptr) return fail(MOR_ENOMEM, "arena exhausted (eig)");
  std::vector<double*> hptr((size_t)ns * NP);
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    double* v[NP] = {q.Vb, q.Yb, q.Ub, q.Zb, q.Vn, q.Tb, q.H, q.Ss, q.G2, q.Rinv, q.theta, q.resid, q.Bk, q.Wk};
    for (int k = 0; k < NP; ++k) hptr[(size_t)k * ns + i] = v[k];
  }
  HIPCHK(hipMemcpyAsync(dptr, hptr.data(), sizeof(double*) * ns * NP, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_s, s_of.data(), 4 * ns, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_rows, rows_of.data(), 4 * ns, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(d_M, M_of.data(), 4 * ns, hipMemcpyHostToDevice, st));
  launch_fill_i(d_info2, ns, 0, st);
  double** P_Zb = dptr + 3 * ns; double** P_Vn = dptr + 4 * ns; double** P_Ub = dptr + 2 * ns;
  double** P_H = dptr + 6 * ns; double** P_Ss = dptr + 7 * ns; double** P_G2 = dptr + 8 * ns;
  double** P_Ri = dptr + 9 * ns; double** P_th = dptr + 10 * ns; double** P_res = dptr + 11 * ns;
  double** P_Bk = dptr + 12 * ns; double** P_Wk = dptr + 13 * ns;
  GemmBatch gY, gH, gU, gZ, gO1a, gO1b, gO2a, gO2b;
  for (Slot* qp : sl) {
    Slot& q = *qp;
    const int s = q.s;
    gY.add(gd(q.MP, s, q.MP, q.C, q.MP, 0, q.Vb, s, 0, q.Yb, s));
    gH.add(gd(s, s, q.MP, q.Vb, s, 1, q.Yb, s, 0, q.H, s));
    gU.add(gd(q.MP, s, s, q.Vb, s, 0, q.Ss, s, 0, q.Ub, s));
    gZ.add(gd(q.MP, s, s, q.Yb, s, 0, q.Ss, s, 0, q.Zb, s));
    gO1a.add(gd(s, s, q.MP, q.Vn, s, 1, q.Vn, s, 0, q.G2, s));
    gO1b.add(gd(q.MP, s, s, q.Vn, s, 0, q.Rinv, s, 0, q.Tb, s));
    gO2a.add(gd(s, s, q.MP, q.Tb, s, 1, q.Tb, s, 0, q.G2, s));
    gO2b.add(gd(q.MP, s, s, q.Tb, s, 0, q.Rinv, s, 0, q.Vb, s));
  }
  for (GemmBatch* b : {&gY, &gH, &gU, &gZ, &gO1a, &gO1b, &gO2a, &gO2b})
    if ((rc = gemm_upload(c, *b, ar))) return rc;
  auto orth = [&]() {   // Vn -> Vb, Cholesky-QR twice
    gemm_run(c, gO1a, "eig");
    launch_cholinv_small(P_G2, P_Ri, d_s, ns, smax, d_info2, st);
    gemm_run(c, gO1b, "eig");
    gemm_run(c, gO2a, "eig");
    launch_cholinv_small(P_G2, P_Ri, d_s, ns, smax, d_info2, st);
    gemm_run(c, gO2b, "eig");
  };
  launch_random_init(P_Vn, d_rows, d_M, d_s, ns, maxrows, smax, 0x5eedu, st);
  orth();
  std::vector<double> hth((size_t)ns * 64), hres((size_t)ns * 64);
  int eig_it = 0;
  bool converged = false;
  for (; eig_it < c->opts.eig_max_iter; ++eig_it) {
    gemm_run(c, gY, "eig");
    gemm_run(c, gH, "eig");
    launch_jacobi(P_H, P_Ss, P_th, d_s, ns, smax, st);
    gemm_run(c, gU, "eig");
    gemm_run(c, gZ, "eig");
    for (Slot* q : sl) launch_fill(q->resid, q->s, 0.0, st);
    launch_ritz(P_Zb, P_Ub, P_Vn, P_th, P_res, d_rows, d_s, ns, maxrows, smax, st);
    for (int i = 0; i < ns; ++i) {
      HIPCHK(hipMemcpyAsync(&hth[(size_t)i * 64], sl[i]->theta, 8 * sl[i]->s, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(&hres[(size_t)i * 64], sl[i]->resid, 8 * sl[i]->s, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipStreamSynchronize(st));
    // Converged when every Ritz pair the truncation decision reads is accurate: the kept
    // ones and the next (the cluster/gap test), plus one, as judged on the current Ritz
    // values; a cluster that grows the decision grows the requirement.
    converged = true;
    for (int i = 0; i < ns && converged; ++i) {
      if (done[i]->status) continue;
      Slot& q = *sl[i];
      const double t0 = std::max(hth[(size_t)i * 64], 1e-300);
      std::vector<double> sg(q.s);
      for (int j = 0; j < q.s; ++j) sg[j] = std::sqrt(std::max(hth[(size_t)i * 64 + j], 0.0));
      const int need = std::min(q.s - 1, std::max(q.nconv, truncation_rank(sg, q.rank, q.tol, q.s - 1) + 2));
      for (int j = 0; j < need; ++j)
        if (!(std::sqrt(std::max(hres[(size_t)i * 64 + j], 0.0)) <= c->opts.eig_rtol * t0)) {
          converged = false;
          break;
        }
    }
    if (converged) break;
    orth();
  }
  if (!converged) return fail(MOR_ENOTCONV, "subspace iteration did not converge within eig_max_iter");

  // ---- truncation, basis Z R^-1 V_k Sigma_k^-1 (= R_i^-1 U_k), stitching, local projection
  double* d_sig = (double*)ar.take(8 * (size_t)ns * 64);
  if (!d_sig) return fail(MOR_ENOMEM, "arena exhausted (basis)");
  std::vector<double> sig_all((size_t)ns * 64, 1.0);
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    std::vector<double> sg(q.s);
    for (int j = 0; j < q.s; ++j) sg[j] = std::sqrt(std::max(hth[(size_t)i * 64 + j], 0.0));
    q.k_eff = truncation_rank(sg, q.rank, q.tol, q.s - 1);
    // the truncation must end inside the subspace (the kept modes and the next one resolved);
    // a tolerance below more singular values than that (or a cluster reaching its end) is
    // refused rather than cut short
    if (q.s < q.M && truncation_rank(sg, q.rank, q.tol, q.s) >= q.s - 1 && !done[i]->status) {
      done[i]->status = MOR_EINVAL;
      g_err = "subdomain " + std::to_string(q.sd) + ": the truncation keeps " + std::to_string(q.s - 1) +
              " or more modes, beyond what the " + std::to_string(q.s) +
              "-vector eigensolver subspace resolves (raise the tolerance or lower the rank)";
    }
    SubResult& R = c->res[q.sd];
    R.sigma = sg;
    R.k_eff = q.k_eff;
    for (int j = 0; j < q.s; ++j) sig_all[(size_t)i * 64 + j] = sg[j] > 0 ? sg[j] : 1.0;
  }
  HIPCHK(hipMemcpyAsync(d_sig, sig_all.data(), 8 * (size_t)ns * 64, hipMemcpyHostToDevice, st));
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    launch_scale_cols(q.Ub, q.s, d_sig + (size_t)i * 64, q.k_eff, q.MP, q.Bk, st);
  }
  {
    std::vector<double*> hB(ns), hW(ns);
    for (int i = 0; i < ns; ++i) {
      hB[i] = sl[i]->Bk;
      hW[i] = sl[i]->Wk;
    }
    ScopedTimer tm(c, "trsm_basis", 0);
    if ((rc = trsm_un_blocked(c, hds, dds, hB, hW))) return rc;
  }
  GemmBatch gV;
  for (int i = 0; i < ns; ++i) {
    Slot& q = *sl[i];
    const HostSub& h = *q.h;
    SubResult& R = c->res[q.sd];
    const int k1 = q.k_eff + 1;
    if (R.d_V) pfree(c, R.d_V);
    if (R.d_Pm) pfree(c, R.d_Pm);
    R.d_V = (double*)palloc(c, 8 * (size_t)h.nV * k1);
    R.d_Pm = (double*)palloc(c, 8 * (size_t)k1 * (k1 + 1));
    if (!R.d_V || !R.d_Pm) return fail(MOR_ENOMEM, "device allocation failed (basis)");
    launch_copy_col(q.Xc + q.M, q.ldXc, R.d_V, k1, h.nV, st);   // q_0 = zero-boundary load solution
    if (q.k_eff > 0) gV.add(gd(h.nV, q.k_eff, q.M, q.Xc, q.ldXc, 0, q.Wk, 64, 0, R.d_V + 1, k1));
  }
  if ((rc = gemm_upload(c, gV, ar))) return rc;
  gemm_run(c, gV, "basis");
  return project_local(c, ar, sl, done, eig_it + 1);
}

static void engine_delete(MorEngine* e) { delete e; }

static MorEngine& engine_for(mor_ctx* c, int prec) {
  const int k = prec == MOR_FP64 ? 1 : 0;
  if (!c->eng[k]) {
    c->eng[k] = new MorEngine();
    if (engine_init(c, *c->eng[k], k == 0 ? 4 : 8)) {
      // allocation failure is reported at the next tick (counters missing)
    }
  }
  return *c->eng[k];
}

static uint64_t enqueue(mor_ctx* c, int sd, int rank, double tol, int prec, int ls = 0,
                        std::shared_ptr<const std::vector<double>> om = nullptr) {
  Req r;
  r.id = g_next_ticket++;
  r.sd = sd; r.rank = rank; r.tol = tol; r.prec = prec;
  r.ls = ls;
  r.om = std::move(om);
  engine_for(c, prec).pending.push_back(r);
  return r.id;
}

static const Req* find_req(mor_ctx* c, uint64_t id, bool* pending) {
  for (int k = 0; k < 2; ++k) {
    MorEngine* e = c->eng[k];
    if (!e) continue;
    auto it = e->finished.find(id);
    if (it != e->finished.end()) {
      *pending = false;
      return &it->second;
    }
    for (const Req& r : e->pending)
      if (r.id == id) {
        *pending = true;
        return &r;
      }
    for (Live* L : e->live)
      if (L->id == id) {
        *pending = true;
        return nullptr;
      }
  }
  *pending = false;
  return nullptr;
}

extern "C" int mor_local_basis_batch(mor_ctx* c, int32_t n, const int32_t* sds, const int32_t* ranks, const double* tols,
                                     int32_t* k_eff_out) {
  MOR_TRY
  if (!c || n <= 0 || !sds || !ranks) return fail(MOR_EINVAL, "bad arguments");
  if (c->opts.host_only) return fail(MOR_ESTATE, "context was created host_only");
  std::vector<char> seen(c->subs.size(), 0);
  for (int i = 0; i < n; ++i) {
    const int sd = sds[i];
    if (sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "subdomain id out of range");
    if (seen[sd]) return fail(MOR_EINVAL, "subdomain listed twice in one batch");
    seen[sd] = 1;
    const double tol = tols ? tols[i] : 0.0;
    if (ranks[i] <= 0 && !(tol > 0.0)) return fail(MOR_EINVAL, "need rank > 0 or tol > 0");
    if (ranks[i] > kMaxRank) return fail(MOR_EINVAL, "rank above " + std::to_string(kMaxRank) +
                                                   " (the eigensolver subspace holds 64 vectors)");
  }
  std::vector<uint64_t> ids(n);
  for (int i = 0; i < n; ++i) ids[i] = enqueue(c, sds[i], ranks[i], tols ? tols[i] : 0.0, c->opts.precision);
  while (!engines_idle(c))
    if (int rc = tick_all(c)) return rc;
  int first_err = 0;
  std::string msg = g_err;
  for (int i = 0; i < n; ++i) {
    bool pend;
    const Req* r = find_req(c, ids[i], &pend);
    const int st = r ? r->status : MOR_ESTATE;
    if (st && !first_err) first_err = st;
    if (k_eff_out) k_eff_out[i] = c->res[sds[i]].k_eff;
  }
  for (int k = 0; k < 2; ++k)
    if (c->eng[k])
      for (uint64_t id : ids) c->eng[k]->finished.erase(id);
  if (first_err) return fail(first_err, msg);
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_local_basis_sketched(mor_ctx* c, int32_t n, const int32_t* sds, const int32_t* ranks,
                                        const double* tols, int32_t l, const double* const* omega,
                                        int32_t* k_eff_out) {
  MOR_TRY
  if (!c || n <= 0 || !sds || !ranks || !omega) return fail(MOR_EINVAL, "bad arguments");
  if (c->opts.host_only) return fail(MOR_ESTATE, "context was created host_only");
  if (l < 1 || l > 64) return fail(MOR_EINVAL, "sketch columns must be in 1..64");
  if (c->opts.precision == MOR_FP32)
    return fail(MOR_EINVAL, "the sketched variant needs FP64 solutions (MOR_FP64, MOR_FP32_REFINE or MOR_BF16_SPLIT)");
  std::vector<char> seen(c->subs.size(), 0);
  for (int i = 0; i < n; ++i) {
    const int sd = sds[i];
    if (sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "subdomain id out of range");
    if (seen[sd]) return fail(MOR_EINVAL, "subdomain listed twice in one batch");
    seen[sd] = 1;
    const double tol = tols ? tols[i] : 0.0;
    if (ranks[i] <= 0 && !(tol > 0.0)) return fail(MOR_EINVAL, "need rank > 0 or tol > 0");
    if (ranks[i] > kMaxRank) return fail(MOR_EINVAL, "rank above " + std::to_string(kMaxRank) +
                                                   " (the eigensolver subspace holds 64 vectors)");
    if (!omega[i]) return fail(MOR_EINVAL, "null sketch");
    if (c->subs[sd].nB < 1) return fail(MOR_EINVAL, "subdomain without interface nodes");
  }
  std::vector<uint64_t> ids(n);
  for (int i = 0; i < n; ++i) {
    const size_t M = (size_t)c->subs[sds[i]].nB;
    auto om = std::make_shared<const std::vector<double>>(omega[i], omega[i] + M * l);
    ids[i] = enqueue(c, sds[i], ranks[i], tols ? tols[i] : 0.0, c->opts.precision, l, std::move(om));
  }
  while (!engines_idle(c))
    if (int rc = tick_all(c)) return rc;
  int first_err = 0;
  std::string msg = g_err;
  for (int i = 0; i < n; ++i) {
    bool pend;
    const Req* r = find_req(c, ids[i], &pend);
    const int st = r ? r->status : MOR_ESTATE;
    if (st && !first_err) first_err = st;
    if (k_eff_out) k_eff_out[i] = c->res[sds[i]].k_eff;
  }
  for (int k = 0; k < 2; ++k)
    if (c->eng[k])
      for (uint64_t id : ids) c->eng[k]->finished.erase(id);
  if (first_err) return fail(first_err, msg);
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_local_basis(mor_ctx* c, int32_t sd, int32_t rank, double tol, int32_t* k_eff_out, double* sigma_out,
                               int32_t sigma_cap) {
  MOR_TRY
  const int rc = mor_local_basis_batch(c, 1, &sd, &rank, &tol, k_eff_out);
  if (rc) return rc;
  if (sigma_out) {
    const auto& s = c->res[sd].sigma;
    for (int j = 0; j < sigma_cap && j < (int)s.size(); ++j) sigma_out[j] = s[j];
  }
  return MOR_OK;
  MOR_CATCH
}

// ------------------------------------------------------------------------------- serving
extern "C" int mor_submit(mor_ctx* c, int32_t sd, int32_t rank, double tol, int32_t precision, uint64_t* ticket) {
  MOR_TRY
  if (!c || !ticket) return fail(MOR_EINVAL, "null argument");
  if (c->opts.host_only) return fail(MOR_ESTATE, "context was created host_only");
  if (sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "subdomain id out of range");
  if (rank <= 0 && !(tol > 0.0)) return fail(MOR_EINVAL, "need rank > 0 or tol > 0");
  if (rank > kMaxRank) return fail(MOR_EINVAL, "rank above " + std::to_string(kMaxRank) +
                                                 " (the eigensolver subspace holds 64 vectors)");
  if (precision < MOR_FP64 || precision > MOR_BF16_SPLIT) return fail(MOR_EINVAL, "unknown precision");
  *ticket = enqueue(c, sd, rank, tol, precision);
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_step(mor_ctx* c) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  return tick_all(c);
  MOR_CATCH
}

extern "C" int mor_poll(mor_ctx* c, uint64_t ticket, int32_t* done, int32_t* status) {
  MOR_TRY
  if (!c || !done || !status) return fail(MOR_EINVAL, "null argument");
  bool pend = false;
  const Req* r = find_req(c, ticket, &pend);
  if (!r && !pend) return fail(MOR_EINVAL, "unknown ticket");
  *done = (r && !pend) ? 1 : 0;
  *status = (r && !pend) ? r->status : 0;
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_drain(mor_ctx* c) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  while (!engines_idle(c))
    if (int rc = tick_all(c)) return rc;
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_engine_stats(mor_ctx* c, int32_t* live, int32_t* pending, int64_t* live_bytes, int64_t* peak_bytes,
                                int64_t* budget) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  int32_t l = 0, p = 0;
  int64_t lb = 0, pb = 0, bu = 0;
  for (int k = 0; k < 2; ++k)
    if (c->eng[k]) {
      l += (int32_t)c->eng[k]->live.size();
      p += (int32_t)c->eng[k]->pending.size();
      lb += (int64_t)c->eng[k]->live_bytes;
      pb = std::max<int64_t>(pb, (int64_t)c->eng[k]->peak_bytes);
      bu = std::max<int64_t>(bu, (int64_t)c->eng[k]->budget);
    }
  if (live) *live = l;
  if (pending) *pending = p;
  if (live_bytes) *live_bytes = lb;
  if (peak_bytes) *peak_bytes = pb;
  if (budget) *budget = bu;
  return MOR_OK;
  MOR_CATCH
}

// ------------------------------------------------------------------------------- projection
// The block preconditioner of the reduced CG (reduced_solver 2): the inverse of each subdomain's
// diagonal block Q_i^T A_ii Q_i from its eigendecomposition.  With the updated bases of Section 6
// step 2 the blocks are the identity and this CG is the paper's diagonal-preconditioned CG; on
// the un-updated system it is the same iteration in exact arithmetic, as long as nothing is dropped.
static int block_preconditioner(mor_ctx* c) {
  hipStream_t st = c->st;
  const int n = (int)c->subs.size();
  std::vector<int64_t> bo(n + 1, 0);
  std::vector<int> s_of(n);
  for (int i = 0; i < n; ++i) {
    s_of[i] = c->res[i].dim;
    if (s_of[i] > 64) return fail(MOR_EINVAL, "block preconditioner: a subdomain block has more than 64 columns");
    bo[i + 1] = bo[i] + (int64_t)s_of[i] * s_of[i];
  }
  c->d_bmv = (double*)palloc(c, 8 * (size_t)std::max<int64_t>(1, bo[n]));
  std::vector<int64_t> rbm(c->n_red);
  std::vector<int2> rbd(c->n_red);
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < s_of[i]; ++a) {
      rbm[c->off[i] + a] = bo[i] + (int64_t)a * s_of[i];
      rbd[c->off[i] + a] = make_int2(c->off[i], s_of[i]);
    }
  if (!c->d_bmv || upload(c, &c->d_rbm, rbm.data(), rbm.size()) || upload(c, &c->d_rbd, rbd.data(), rbd.size()))
    return fail(MOR_ENOMEM, "device allocation failed (block preconditioner)");
  const int64_t nth = c->off[n];
  const size_t bytes = 16 * (size_t)std::max<int64_t>(1, bo[n]) + 8 * (size_t)std::max<int64_t>(1, nth) +
                       4 * sizeof(double*) * n + 12 * (size_t)n + 8 * 256;
  char* buf = (char*)dalloc(c, bytes);
  if (!buf) return fail(MOR_ENOMEM, "device allocation failed (block preconditioner)");
  struct G { mor_ctx* c; void* p; ~G() { (void)hipStreamSynchronize(c->st); dfree(c, p); } } guard{c, buf};
  Arena ar{buf, bytes, 0};
  double* H = (double*)ar.take(8 * (size_t)std::max<int64_t>(1, bo[n]));
  double* S = (double*)ar.take(8 * (size_t)std::max<int64_t>(1, bo[n]));
  double* th = (double*)ar.take(8 * (size_t)std::max<int64_t>(1, nth));
  double** PH = (double**)ar.take(sizeof(double*) * n);
  double** PS = (double**)ar.take(sizeof(double*) * n);
  double** PT = (double**)ar.take(sizeof(double*) * n);
  double** PO = (double**)ar.take(sizeof(double*) * n);
  int* ds = (int*)ar.take(4 * (size_t)n);
  double* dd = (double*)ar.take(8 * (size_t)n);
  if (!dd) return fail(MOR_ENOMEM, "arena exhausted (block preconditioner)");
  // every positive eigenvalue is kept (an exact block inverse for SPD blocks): with directions
  // dropped, the full-space recurrence keeps their residual part and loses conjugacy at tight
  // tolerances; dropping belongs to the basis update, which removes them from the system
  std::vector<double> drops(n, 0.0);
  HIPCHK(hipMemcpyAsync(dd, drops.data(), 8 * (size_t)n, hipMemcpyHostToDevice, st));
  std::vector<double> hH((size_t)std::max<int64_t>(1, bo[n]));
  std::vector<double*> ph(n), ps(n), pt(n), po(n);
  for (int i = 0; i < n; ++i) {
    std::copy(c->res[i].Aii.begin(), c->res[i].Aii.end(), hH.begin() + bo[i]);
    ph[i] = H + bo[i];
    ps[i] = S + bo[i];
    pt[i] = th + c->off[i];
    po[i] = c->d_bmv + bo[i];
  }
  HIPCHK(hipMemcpyAsync(H, hH.data(), 8 * hH.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(PH, ph.data(), sizeof(double*) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(PS, ps.data(), sizeof(double*) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(PT, pt.data(), sizeof(double*) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(PO, po.data(), sizeof(double*) * n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ds, s_of.data(), 4 * (size_t)n, hipMemcpyHostToDevice, st));
  launch_jacobi(PH, PS, PT, ds, n, 64, st);
  launch_block_pinv(PS, PT, ds, n, dd, PO, st);
  HIPCHK(hipGetLastError());
  std::vector<double> hth((size_t)std::max<int64_t>(1, nth));
  HIPCHK(hipMemcpyAsync(hth.data(), th, 8 * hth.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i)
    if (s_of[i] > 0 && !(hth[c->off[i]] > 0.0))
      return fail(MOR_EDEVICE, "subdomain " + std::to_string(i) + ": reduced diagonal block is not positive definite");
  return MOR_OK;
}

extern "C" int mor_project(mor_ctx* c) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  if (c->opts.host_only) return fail(MOR_ESTATE, "context was created host_only");
  const int n = (int)c->subs.size();
  for (int i = 0; i < n; ++i)
    if (!c->res[i].reduced) return fail(MOR_ESTATE, "subdomain " + std::to_string(i) + " has no basis yet");
  hipStream_t st = c->st;
  const bool sparse = c->opts.reduced_solver >= 1;
  c->projected = c->solved = 0;
  c->off.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) c->off[i + 1] = c->off[i] + c->res[i].dim;
  c->n_red = c->off[n];
  c->MPr = rup(c->n_red, 64);
  const int npairs = (int)c->om0.pair_i.size();
  for (void* p : {(void*)c->d_At, (void*)c->d_bt, (void*)c->d_x, (void*)c->d_slab, (void*)c->d_ccol,
                  (void*)c->d_rdiag, (void*)c->d_rs, (void*)c->d_rwc, (void*)c->d_bmv, (void*)c->d_rbm,
                  (void*)c->d_rbd})
    pfree(c, p);
  c->d_bmv = nullptr;
  c->d_rbm = nullptr;
  c->d_rbd = nullptr;
  c->d_At = c->d_bt = c->d_x = c->d_slab = nullptr;
  c->d_ccol = c->d_rdiag = nullptr;
  c->d_rs = nullptr;
  c->d_rwc = nullptr;
  // where each block goes: dense rows of length MPr, or per-subdomain slabs over the neighbours
  std::vector<int64_t> dbase(n);   // element offset of block (i, i)
  std::vector<int64_t> dld(n);     // row length of subdomain i's rows
  std::vector<PairOut> pout(npairs);
  if (sparse) {
    std::vector<std::vector<int>> nb(n);
    for (int i = 0; i < n; ++i) nb[i].push_back(i);
    for (int p = 0; p < npairs; ++p) {
      nb[c->om0.pair_i[p]].push_back(c->om0.pair_j[p]);
      nb[c->om0.pair_j[p]].push_back(c->om0.pair_i[p]);
    }
    std::vector<std::map<int, int>> coff(n);   // column offset of neighbour j within subdomain i's slab
    std::vector<int64_t> sbase(n);
    c->h_ccol.clear();
    c->h_rs.assign(c->n_red, 0);
    c->h_rwc.assign(c->n_red, make_int2(0, 0));
    std::vector<int> rdiag(c->n_red);
    int64_t len = 0;
    for (int i = 0; i < n; ++i) {
      std::sort(nb[i].begin(), nb[i].end());
      nb[i].erase(std::unique(nb[i].begin(), nb[i].end()), nb[i].end());
      const int cbase = (int)c->h_ccol.size();
      int W = 0;
      for (int j : nb[i]) {
        coff[i][j] = W;
        for (int b = 0; b < c->res[j].dim; ++b) c->h_ccol.push_back(c->off[j] + b);
        W += c->res[j].dim;
      }
      sbase[i] = len;
      dld[i] = W;
      dbase[i] = len + coff[i][i];
      for (int a = 0; a < c->res[i].dim; ++a) {
        const int64_t r = c->off[i] + a;
        c->h_rs[r] = len + (int64_t)a * W;
        c->h_rwc[r] = make_int2(W, cbase);
        rdiag[r] = coff[i][i] + a;
      }
      len += (int64_t)c->res[i].dim * W;
    }
    if (c->h_ccol.size() > (size_t)INT32_MAX) return fail(MOR_EINVAL, "reduced system too large for int32 columns");
    c->slab_len = len;
    for (int p = 0; p < npairs; ++p) {
      const int i = c->om0.pair_i[p], j = c->om0.pair_j[p];
      pout[p] = PairOut{sbase[i] + coff[i][j], sbase[j] + coff[j][i], (int)dld[i], (int)dld[j]};
    }
    c->d_slab = (double*)palloc(c, 8 * (size_t)std::max<int64_t>(1, len));
    if (!c->d_slab) return fail(MOR_ENOMEM, "device allocation failed (reduced slabs)");
    if (upload(c, &c->d_ccol, c->h_ccol.data(), c->h_ccol.size()) ||
        upload(c, &c->d_rs, c->h_rs.data(), c->h_rs.size()) ||
        upload(c, &c->d_rwc, c->h_rwc.data(), c->h_rwc.size()) || upload(c, &c->d_rdiag, rdiag.data(), rdiag.size()))
      return fail(MOR_ENOMEM, "device allocation failed (reduced pattern)");
    HIPCHK(hipStreamSynchronize(st));   // rdiag is read by the copy
    if (c->opts.reduced_solver == 2)
      if (int rc = block_preconditioner(c)) return rc;
  } else {
    c->d_At = (double*)palloc(c, 8 * (size_t)c->MPr * c->MPr);
    if (!c->d_At) return fail(MOR_ENOMEM, "device allocation failed (reduced system)");
    for (int i = 0; i < n; ++i) {
      dbase[i] = (int64_t)c->off[i] * c->MPr + c->off[i];
      dld[i] = c->MPr;
    }
    for (int p = 0; p < npairs; ++p) {
      const int i = c->om0.pair_i[p], j = c->om0.pair_j[p];
      pout[p] = PairOut{(int64_t)c->off[i] * c->MPr + c->off[j], (int64_t)c->off[j] * c->MPr + c->off[i],
                        (int)c->MPr, (int)c->MPr};
    }
  }
  c->d_bt = (double*)palloc(c, 8 * (size_t)c->MPr * 64);
  c->d_x = (double*)palloc(c, 8 * (size_t)c->MPr * 64);
  if (!c->d_bt || !c->d_x) return fail(MOR_ENOMEM, "device allocation failed (reduced system)");
  ScopedTimer tm(c, "project", 0);
  double* out = sparse ? c->d_slab : c->d_At;
  if (sparse) {
    launch_fill(c->d_slab, c->slab_len, 0.0, st);
  } else {
    launch_fill(c->d_At, (int64_t)c->MPr * c->MPr, 0.0, st);
    launch_pad_identity(c->d_At, (int)c->n_red, (int)c->MPr, st);
  }
  launch_fill(c->d_bt, (int64_t)c->MPr * 64, 0.0, st);
  for (int i = 0; i < n; ++i) {
    const int k1 = c->res[i].dim;
    launch_scatter_block(c->res[i].d_Pm, k1, k1 + 1, out, dbase[i], dld[i], st);
    launch_copy_col(c->res[i].d_Pm + k1, k1 + 1, c->d_bt + (size_t)c->off[i] * 64, 64, k1, st);
  }
  // A_0 on omega_0, then every neighbour pair
  const HostSub& h0 = c->om0.sub;
  if (npairs > 0) {
    double* A0 = (double*)dalloc(c, 8 * (size_t)std::max(1, h0.rp[h0.nL]));
    if (!A0) return fail(MOR_ENOMEM, "device allocation failed (A_0)");
    launch_fill(A0, h0.rp[h0.nL], 0.0, st);
    std::vector<AsmJob> jobs{{&h0, &c->om0dev, A0, nullptr, nullptr, nullptr}};
    if (int rc = assemble_batch(c, jobs)) {
      dfree(c, A0);
      return rc;
    }
    std::vector<int4> range(npairs);
    for (int p = 0; p < npairs; ++p)
      range[p] = make_int4(c->om0.pair_i[p], c->om0.pair_j[p], c->om0.pair_first[p], c->om0.pair_count[p]);
    std::vector<double*> vp(n);
    std::vector<int> ldv(n), k1(n);
    for (int i = 0; i < n; ++i) {
      vp[i] = c->res[i].d_V;
      ldv[i] = k1[i] = c->res[i].dim;
    }
    const size_t bytes = sizeof(int4) * npairs + 4 * c->om0.trip.size() + sizeof(double*) * n + 4 * 2 * (size_t)n +
                         sizeof(PairOut) * npairs + 8 * 256;
    char* buf = (char*)dalloc(c, bytes);
    if (!buf) {
      dfree(c, A0);
      return fail(MOR_ENOMEM, "device allocation failed (pairs)");
    }
    Arena ar{buf, bytes, 0};
    int4* d_range = (int4*)ar.take(sizeof(int4) * npairs);
    int* d_trip = (int*)ar.take(4 * std::max<size_t>(1, c->om0.trip.size()));
    double** d_vp = (double**)ar.take(sizeof(double*) * n);
    int* d_ldv = (int*)ar.take(4 * n);
    int* d_k1 = (int*)ar.take(4 * n);
    PairOut* d_out = (PairOut*)ar.take(sizeof(PairOut) * npairs);
    if (!d_out) {
      dfree(c, buf);
      dfree(c, A0);
      return fail(MOR_ENOMEM, "arena exhausted (pairs)");
    }
    HIPCHK(hipMemcpyAsync(d_range, range.data(), sizeof(int4) * npairs, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_trip, c->om0.trip.data(), 4 * c->om0.trip.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_vp, vp.data(), sizeof(double*) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_ldv, ldv.data(), 4 * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_k1, k1.data(), 4 * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_out, pout.data(), sizeof(PairOut) * npairs, hipMemcpyHostToDevice, st));
    launch_pair_project(d_range, d_trip, A0, d_vp, d_ldv, d_k1, d_out, out, npairs, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    dfree(c, buf);
    dfree(c, A0);
  }
  HIPCHK(hipStreamSynchronize(st));
  c->x_host.assign((size_t)c->n_red, 0.0);
  c->projected = 1;
  return MOR_OK;
  MOR_CATCH
}

// u~ = sum_i S_i Q_i x_i at every mesh node from c->x_host
static int reconstruct_solution(mor_ctx* c, double* u_out) {
  hipStream_t st = c->st;
  double* du = (double*)dalloc(c, 8 * (size_t)c->mesh.n_nodes);
  double* dx = (double*)dalloc(c, 8 * (size_t)std::max<int64_t>(1, c->n_red));
  if (!du || !dx) {
    dfree(c, du);
    dfree(c, dx);
    return fail(MOR_ENOMEM, "device allocation failed (reconstruction)");
  }
  HIPCHK(hipMemcpyAsync(dx, c->x_host.data(), 8 * c->n_red, hipMemcpyHostToDevice, st));
  launch_fill(du, c->mesh.n_nodes, 0.0, st);
  for (size_t i = 0; i < c->subs.size(); ++i) {
    const int k1 = c->res[i].dim;
    launch_reconstruct(c->res[i].d_V, c->subs[i].nP, k1, dx + c->off[i], c->sdev[i].nodes, du, st);
  }
  HIPCHK(hipGetLastError());
  if (u_out) HIPCHK(hipMemcpyAsync(u_out, du, 8 * (size_t)c->mesh.n_nodes, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  dfree(c, dx);
  dfree(c, du);
  return MOR_OK;
}

// Reduced-solve vectors carved from one buffer: x, r, z, p, q, D^-1 (rup(n, 64) doubles each),
// the scalar rings and the stop state.
static size_t pcg_bytes(int64_t n) { return 8 * 6 * (size_t)rup(std::max<int64_t>(n, 1), 64) + 8 * 16 + 4 * 16 + 1024; }

static RpcgDev pcg_layout(mor_ctx* c, char* buf, size_t bytes, int n) {
  Arena ar{buf, bytes, 0};
  RpcgDev d{};
  d.val = c->d_slab;
  d.ccol = c->d_ccol;
  d.rs = c->d_rs;
  d.rwc = c->d_rwc;
  d.rdiag = c->d_rdiag;
  d.b = c->d_bt;
  d.bstride = 64;
  d.block = c->opts.reduced_solver == 2;
  d.bmv = c->d_bmv;
  d.rbm = c->d_rbm;
  d.rbd = c->d_rbd;
  double* v[6];
  for (auto& q : v) q = (double*)ar.take(8 * (size_t)rup(n, 64));
  d.x = v[0]; d.r = v[1]; d.z = v[2]; d.p = v[3]; d.q = v[4]; d.dinv = v[5];
  d.sc = (double*)ar.take(8 * 16);
  d.state = (int*)ar.take(4 * 16);
  return d;
}

// The reduced system by conjugate gradients with the diagonal preconditioner on the
// block-row slabs (end of Section 6 step 3; Section 7), from x = 0.  The iterations run in
// chunks of launches; between chunks the host reads the stop flag.  On success x is left in
// d.x on the device and copied into c->x_host (sized n by mor_project).
static int pcg_iterate(mor_ctx* c, const RpcgDev& d, int n) {
  hipStream_t st = c->st;
  c->solve_iters = 0;
  c->solve_relres = 0.0;
  const double tol2 = c->opts.reduced_rtol * c->opts.reduced_rtol;
  const int chunk = 32, cap = c->opts.reduced_max_iter;
  launch_rpcg_setup(d, n, st);
  int hs[4] = {0, 0, 0, 0};
  for (int it = 0; it < cap;) {
    const int m = std::min(chunk, cap - it);
    for (int k = 0; k < m; ++k) launch_rpcg_iteration(d, n, it + k, tol2, st);
    it += m;
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hs, d.state, sizeof(hs), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hs[0] || hs[2]) break;
  }
  if (hs[2] == 2) return fail(MOR_EDEVICE, "reduced matrix has a diagonal entry <= 0");
  if (hs[2] == 1)
    return fail(MOR_EDEVICE, "reduced matrix is not positive definite (p'Ap <= 0 at iteration " +
                                 std::to_string(hs[1] + 1) + ")");
  double sc[11];
  HIPCHK(hipMemcpyAsync(sc, d.sc, sizeof(sc), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  c->solve_iters = hs[1];
  const int last = hs[1] > 0 ? (hs[1] - 1) % 3 : 2;
  if (d.block)
    c->solve_relres = sc[10] > 0 ? std::sqrt(std::max(0.0, sc[3 + last]) / sc[10]) : 0.0;
  else
    c->solve_relres = sc[9] > 0 ? std::sqrt(std::max(0.0, sc[6 + last]) / sc[9]) : 0.0;
  if (!hs[0])
    return fail(MOR_ENOTCONV, "reduced conjugate gradients: ||r||/||b|| = " + std::to_string(c->solve_relres) +
                                  " after " + std::to_string(hs[1]) + " iterations");
  if ((int64_t)c->x_host.size() != (int64_t)n) return fail(MOR_ESTATE, "reduced solution storage not sized");
  HIPCHK(hipMemcpyAsync(c->x_host.data(), d.x, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return MOR_OK;
}

static int solve_pcg(mor_ctx* c, double* u_out, int64_t* n_reduced_out) {
  const int n = (int)c->n_red;
  std::fill(c->x_host.begin(), c->x_host.end(), 0.0);
  c->solve_iters = 0;
  c->solve_relres = 0.0;
  if (n > 0) {
    const size_t bytes = pcg_bytes(n);
    char* buf = (char*)dalloc(c, bytes);
    if (!buf) return fail(MOR_ENOMEM, "device allocation failed (reduced solve)");
    struct G { mor_ctx* c; void* p; ~G() { (void)hipStreamSynchronize(c->st); dfree(c, p); } } guard{c, buf};
    const RpcgDev d = pcg_layout(c, buf, bytes, n);
    if (!d.state) return fail(MOR_ENOMEM, "arena exhausted (reduced solve)");
    ScopedTimer tm(c, "solve", 0.0);
    const int rc = pcg_iterate(c, d, n);
    tm.work = 2.0 * (double)c->slab_len * c->solve_iters;
    if (rc) return rc;
  }
  if (int rc = reconstruct_solution(c, u_out)) return rc;
  if (n_reduced_out) *n_reduced_out = c->n_red;
  c->solved = 1;
  return MOR_OK;
}

// ---- the reduced solve without allocation ---------------------------------------------------
// A file-scope device array holds the conjugate-gradient vectors of mor_solve_noalloc, so the
// call allocates nothing.  Its address is looked up once per device, with that device current,
// when the first context is created there; host code passes that address, never the array's
// name, to kernels and copies.  Every call on a device shares the device's array.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxScratchDevices] = {};
static int g_scratch_state[kMaxScratchDevices] = {};   // 0 not looked up, 1 found, -1 lookup failed

// Look up this device's copy of `scratch` (the device must be current); 1 when available.
// Largest reduced dimension whose vectors fit the scratch (48 bytes per unknown, rounded to 64).
static int64_t noalloc_max_reduced() {
  int64_t n = (int64_t)((kNoAllocScratchBytes - 8 * 16 - 4 * 16 - 1024) / 48) / 64 * 64;
  while (n > 0 && pcg_bytes(n) > kNoAllocScratchBytes) n -= 64;
  return n;
}

static int scratch_setup(int dev) noexcept {
  if (dev < 0 || dev >= kMaxScratchDevices) return -1;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_state[dev] == 0) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_state[dev] = (e == hipSuccess && ptr != nullptr) ? 1 : -1;
    g_scratch_ptr[dev] = g_scratch_state[dev] == 1 ? ptr : nullptr;
  }
  return g_scratch_state[dev];
}

extern "C" int mor_solve_noalloc(mor_ctx* c, double* u_dev, int64_t* n_reduced_out) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  if (c->opts.host_only) return fail(MOR_ESTATE, "context was created host_only");
  if (!c->projected) return fail(MOR_ESTATE, "mor_project must run first");
  if (c->opts.reduced_solver < 1) return fail(MOR_EINVAL, "mor_solve_noalloc needs reduced_solver 1 or 2");
  if (!u_dev) return fail(MOR_EINVAL, "u_dev is required (device buffer of n_nodes doubles)");
  const int64_t n = c->n_red;
  if (n > 0 && pcg_bytes(n) > kNoAllocScratchBytes)
    return fail(MOR_ENOMEM, "reduced dimension " + std::to_string(n) + " exceeds the static scratch of " +
                                std::to_string(kNoAllocScratchBytes >> 20) + " MiB (at most " +
                                std::to_string(noalloc_max_reduced()) + " unknowns)");
  if (scratch_setup(c->device) != 1) return fail(MOR_EDEVICE, "static scratch of this device is not available");
  c->solved = 0;
  hipStream_t st = c->st;
  if (n > 0) {
    const RpcgDev d = pcg_layout(c, (char*)g_scratch_ptr[c->device], kNoAllocScratchBytes, (int)n);
    if (!d.state) return fail(MOR_ENOMEM, "static scratch exhausted (reduced solve)");
    if (int rc = pcg_iterate(c, d, (int)n)) return rc;
    launch_fill(u_dev, c->mesh.n_nodes, 0.0, st);
    for (size_t i = 0; i < c->subs.size(); ++i)
      launch_reconstruct(c->res[i].d_V, c->subs[i].nP, c->res[i].dim, d.x + c->off[i], c->sdev[i].nodes, u_dev, st);
  } else {
    std::fill(c->x_host.begin(), c->x_host.end(), 0.0);
    launch_fill(u_dev, c->mesh.n_nodes, 0.0, st);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  if (n_reduced_out) *n_reduced_out = n;
  c->solved = 1;
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_solve(mor_ctx* c, double* u_out, int64_t* n_reduced_out) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  if (c->opts.host_only) return fail(MOR_ESTATE, "context was created host_only");
  if (!c->projected) return fail(MOR_ESTATE, "mor_project must run first");
  c->solved = 0;
  if (c->opts.reduced_solver >= 1) return solve_pcg(c, u_out, n_reduced_out);
  c->solve_iters = 0;
  c->solve_relres = 0.0;
  hipStream_t st = c->st;
  const int64_t MP = c->MPr;
  const int T = (int)(MP / 64);
  const size_t bytes = 8 * (size_t)MP * MP + 8 * (size_t)T * 4096 + 64 + sizeof(DenseSub) + 2 * sizeof(TrsmDesc) +
                       2 * sizeof(double*) + 8 * (size_t)MP * 64 + 8192;
  char* buf = (char*)dalloc(c, bytes);
  if (!buf) return fail(MOR_ENOMEM, "device allocation failed (reduced solve)");
  struct G { mor_ctx* c; void* p; ~G() { (void)hipStreamSynchronize(c->st); dfree(c, p); } } guard{c, buf};
  Arena ar{buf, bytes, 0};
  double* F = (double*)ar.take(8 * (size_t)MP * MP);
  double* Di = (double*)ar.take(8 * (size_t)T * 4096);
  int* info = (int*)ar.take(64);
  DenseSub* dd = (DenseSub*)ar.take(sizeof(DenseSub));
  if (!dd) return fail(MOR_ENOMEM, "arena exhausted (reduced solve)");
  ScopedTimer tm(c, "solve", (double)MP * MP * MP / 3.0);
  HIPCHK(hipMemcpyAsync(F, c->d_At, 8 * (size_t)MP * MP, hipMemcpyDeviceToDevice, st));
  launch_fill_i(info, 16, 0, st);
  DenseSub hd{(int)c->n_red, (int)MP, T, F, nullptr, nullptr, nullptr, Di, info};
  HIPCHK(hipMemcpyAsync(dd, &hd, sizeof(hd), hipMemcpyHostToDevice, st));
  for (int p = 0; p < T; ++p) {
    launch_potrf_diag(dd, 1, p, st);
    launch_chol_panel(dd, 1, p, T, st);
    launch_chol_syrk(dd, 1, p, T, st);
  }
  int hinfo = 0;
  HIPCHK(hipMemcpyAsync(&hinfo, info, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hinfo) return fail(MOR_EDEVICE, "reduced matrix is not positive definite (pivot " + std::to_string(hinfo) + ")");
  // R^T y = b (y in d_x), then R x = y
  const TrsmDesc ht{c->d_bt, 64, 0, c->d_x, 64, 1};
  if (int rc = trsm_lt_blocked(c, {hd}, dd, {ht})) return rc;
  double* xsol = (double*)ar.take(8 * (size_t)MP * 64);
  if (!xsol) return fail(MOR_ENOMEM, "arena exhausted (reduced solve)");
  if (int rc = trsm_un_blocked(c, {hd}, dd, {c->d_x}, {xsol})) return rc;
  // x = column 0 of xsol
  std::vector<double> xs((size_t)MP * 64);
  HIPCHK(hipMemcpyAsync(xs.data(), xsol, 8 * xs.size(), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  c->x_host.assign((size_t)c->n_red, 0.0);
  for (int64_t i = 0; i < c->n_red; ++i) c->x_host[i] = xs[(size_t)i * 64];
  if (int rc = reconstruct_solution(c, u_out)) return rc;
  if (n_reduced_out) *n_reduced_out = c->n_red;
  c->solved = 1;
  return MOR_OK;
  MOR_CATCH
}

// ------------------------------------------------------------------------------- getters
extern "C" int mor_get_sizes(mor_ctx* c, int32_t sd, int32_t* nP, int32_t* nV, int32_t* nI, int32_t* nB) {
  MOR_TRY
  if (!c || sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "bad subdomain");
  const HostSub& h = c->subs[sd];
  if (nP) *nP = h.nP;
  if (nV) *nV = h.nV;
  if (nI) *nI = h.nI;
  if (nB) *nB = h.nB;
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_nodes(mor_ctx* c, int32_t sd, int32_t* out, int64_t cap) {
  MOR_TRY
  if (!c || sd < 0 || sd >= (int)c->subs.size() || !out) return fail(MOR_EINVAL, "bad arguments");
  const HostSub& h = c->subs[sd];
  if (cap < h.nL) return fail(MOR_EINVAL, "output too small");
  std::memcpy(out, h.nodes.data(), 4 * (size_t)h.nL);
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_pairs(mor_ctx* c, int32_t* out, int64_t cap, int64_t* n) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  const int64_t np = (int64_t)c->om0.pair_i.size();
  if (n) *n = np;
  if (out)
    for (int64_t p = 0; p < np && p < cap; ++p) {
      out[2 * p] = c->om0.pair_i[p];
      out[2 * p + 1] = c->om0.pair_j[p];
    }
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_basis(mor_ctx* c, int32_t sd, double* out, int64_t cap, int32_t* k_eff) {
  MOR_TRY
  if (!c || sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "bad subdomain");
  const SubResult& R = c->res[sd];
  if (!R.reduced) return fail(MOR_ESTATE, "subdomain not reduced");
  if (k_eff) *k_eff = R.dim - 1;
  const size_t n = (size_t)c->subs[sd].nV * R.dim;
  if (out) {
    if ((size_t)cap < n) return fail(MOR_EINVAL, "output too small");
    HIPCHK(hipMemcpy(out, R.d_V, 8 * n, hipMemcpyDeviceToHost));
  }
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_sigma(mor_ctx* c, int32_t sd, double* out, int32_t cap, int32_t* n) {
  MOR_TRY
  if (!c || sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "bad subdomain");
  const SubResult& R = c->res[sd];
  if (!R.reduced) return fail(MOR_ESTATE, "subdomain not reduced");
  if (n) *n = (int)R.sigma.size();
  if (out)
    for (int j = 0; j < cap && j < (int)R.sigma.size(); ++j) out[j] = R.sigma[j];
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_local_block(mor_ctx* c, int32_t sd, double* Aii, double* bi, int64_t cap) {
  MOR_TRY
  if (!c || sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "bad subdomain");
  const SubResult& R = c->res[sd];
  if (!R.reduced) return fail(MOR_ESTATE, "subdomain not reduced");
  if ((size_t)cap < R.Aii.size()) return fail(MOR_EINVAL, "output too small");
  if (Aii) std::memcpy(Aii, R.Aii.data(), 8 * R.Aii.size());
  if (bi) std::memcpy(bi, R.bi.data(), 8 * R.bi.size());
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_reduced(mor_ctx* c, double* At, double* bt, int64_t cap, int64_t* n) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  if (!c->projected) return fail(MOR_ESTATE, "mor_project must run first");
  const int64_t nr = c->n_red;
  if (n) *n = nr;
  if (At) {
    if (cap < nr * nr) return fail(MOR_EINVAL, "output too small");
    if (c->d_slab) {   // expand the block-row slabs
      std::vector<double> sl((size_t)c->slab_len);
      HIPCHK(hipMemcpy(sl.data(), c->d_slab, 8 * sl.size(), hipMemcpyDeviceToHost));
      std::fill(At, At + nr * nr, 0.0);
      for (int64_t r = 0; r < nr; ++r) {
        const int2 wc = c->h_rwc[r];
        for (int k = 0; k < wc.x; ++k) At[r * nr + c->h_ccol[wc.y + k]] = sl[c->h_rs[r] + k];
      }
    } else {
      HIPCHK(hipMemcpy2D(At, 8 * nr, c->d_At, 8 * c->MPr, 8 * nr, nr, hipMemcpyDeviceToHost));
    }
  }
  if (bt) {
    std::vector<double> b((size_t)c->MPr * 64);
    HIPCHK(hipMemcpy(b.data(), c->d_bt, 8 * b.size(), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nr; ++i) bt[i] = b[(size_t)i * 64];
  }
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_solve_info(mor_ctx* c, int32_t* solver, int32_t* iters, double* rel_residual) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  if (!c->solved) return fail(MOR_ESTATE, "mor_solve must run first");
  if (solver) *solver = c->opts.reduced_solver;
  if (iters) *iters = c->solve_iters;
  if (rel_residual) *rel_residual = c->solve_relres;
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_reduced_solution(mor_ctx* c, double* x, int64_t cap) {
  MOR_TRY
  if (!c || !x) return fail(MOR_EINVAL, "null argument");
  if (!c->solved) return fail(MOR_ESTATE, "mor_solve must run first");
  if (cap < c->n_red) return fail(MOR_EINVAL, "output too small");
  std::memcpy(x, c->x_host.data(), 8 * (size_t)c->n_red);
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_get_stats(mor_ctx* c, int32_t sd, int32_t* a, int32_t* k, int32_t* refine, int32_t* eig) {
  MOR_TRY
  if (!c || sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "bad subdomain");
  const SubResult& R = c->res[sd];
  if (a) *a = R.cg_a;
  if (k) *k = R.cg_k;
  if (refine) *refine = R.refine;
  if (eig) *eig = R.eig;
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_get_rank(mor_ctx* c, int32_t sd, int32_t* k_eff, int32_t* dim) {
  MOR_TRY
  if (!c || sd < 0 || sd >= (int)c->subs.size()) return fail(MOR_EINVAL, "bad subdomain");
  const SubResult& R = c->res[sd];
  if (!R.reduced) return fail(MOR_ESTATE, "subdomain not reduced");
  if (k_eff) *k_eff = R.k_eff;
  if (dim) *dim = R.dim;
  return MOR_OK;
  MOR_CATCH
}

extern "C" int mor_timing_enable(mor_ctx* c, int32_t on) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  c->timing = on != 0;
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_timing_get(mor_ctx* c, const char* name, int64_t* launches, double* total_ms, double* work) {
  MOR_TRY
  if (!c || !name) return fail(MOR_EINVAL, "null argument");
  flush_timers(c);
  auto it = c->timers.find(name);
  if (it == c->timers.end()) {
    if (launches) *launches = 0;
    if (total_ms) *total_ms = 0;
    if (work) *work = 0;
    return MOR_OK;
  }
  if (launches) *launches = it->second.launches;
  if (total_ms) *total_ms = it->second.ms;
  if (work) *work = it->second.work;
  return MOR_OK;
  MOR_CATCH
}
extern "C" int mor_timing_reset(mor_ctx* c) {
  MOR_TRY
  if (!c) return fail(MOR_EINVAL, "null context");
  flush_timers(c);
  c->timers.clear();
  return MOR_OK;
  MOR_CATCH
}
