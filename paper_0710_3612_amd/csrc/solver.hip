// Host driver of libsmg: the multigrid hierarchy, the V-cycle, the Krylov
// solvers, the adaptive setup and the C entry points declared in smg.h.
//
// Paper map (Brannick, Brower, Clark, Osborn, Rebbi, arXiv:0710.3612):
//   V-cycle        Multigrid section, steps 1-5 and Eq. 3 (read with -R A R^H)
//   Galerkin       Eq. 2, A^(l+1) = P^H A^(l) P
//   Setup          Adaptive Multigrid section: relaxation of a random vector
//                  (Eq. 4), then V-cycles on further random vectors, each
//                  survivor block-orthonormalised and appended; recursion.
//   Smoother       Results section: frozen nu-step under-relaxed MR polynomial
//   Outer solver   Results section: MG-CG, the V-cycle preconditions CG
//   Mass reuse     Results section: setup at one mass, vectors reused
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/smg.h"
#include "common.h"

namespace smg {

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    throw Error(e == hipErrorOutOfMemory ? SMG_ENOMEM : SMG_EDEVICE, buf);
  }
}

namespace {

thread_local std::string g_last_error;

// ---------------------------------------------------------------------------
// Device memory.  Every array a handle or a batch owns comes from the allocator
// installed by smg_set_allocator (hipMalloc when none is), is counted, and is
// released when its owner is destroyed.  A dry pool only counts: smg_query_bytes
// runs the same allocation plan through it without touching the device.
// ---------------------------------------------------------------------------
struct Allocator {
  smg_alloc_fn alloc = nullptr;
  smg_release_fn release = nullptr;
  void* ctx = nullptr;
};

std::mutex g_alloc_mu;
Allocator g_alloc;

Allocator current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}

// Progress reporting of long calls (smg_set_progress).  The callback is read under
// the lock and called outside it, on the calling thread.
std::mutex g_progress_mu;
smg_progress_fn g_progress = nullptr;
void* g_progress_ctx = nullptr;

void report(const char* stage, int level, int step, int total, double value) {
  smg_progress_fn fn;
  void* ctx;
  {
    std::lock_guard<std::mutex> lk(g_progress_mu);
    fn = g_progress;
    ctx = g_progress_ctx;
  }
  if (fn) fn(stage, level, step, total, value, ctx);
}

struct Pool {
  Allocator a = current_allocator();  // the allocator in force when the owner was created
  bool dry = false;
  const hipStream_t* stream = nullptr;  // the owner's current stream, handed to the allocator
  std::vector<void*> ptrs;
  std::vector<size_t> sizes;
  std::vector<hipStream_t> streams;
  size_t bytes = 0;
  uintptr_t fake = 4096;  // distinct, never dereferenced addresses of a dry pool
  // Arena pools (batches): every array is rounded to 256 bytes and carved from one
  // block that open_arena takes from the allocator, so that a batch costs one
  // allocation and one release instead of one per array.  A dry pool with the same
  // granularity counts the same bytes.
  size_t gran = 1;
  char* arena = nullptr;
  size_t arena_size = 0, arena_off = 0;
  // The owner has synchronised every stream that used the memory, so the release
  // needs no device-wide synchronisation.
  bool owner_synced = false;
  void* raw(size_t nb) {
    hipStream_t st = stream ? *stream : nullptr;
    void* p = nullptr;
    if (a.alloc) {
      p = a.alloc(nb, (void*)st, a.ctx);
      if (!p) throw Error(SMG_ENOMEM, "the installed allocator returned no memory for " + std::to_string(nb) + " bytes");
    } else if (hipMalloc(&p, nb) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(SMG_ENOMEM, "hipMalloc of " + std::to_string(nb) + " bytes failed");
    }
    ptrs.push_back(p);
    sizes.push_back(nb);
    streams.push_back(st);
    return p;
  }
  void open_arena(size_t total) {
    gran = 256;
    if (dry || total == 0) return;
    arena = static_cast<char*>(raw(total));
    arena_size = total;
    arena_off = 0;
  }
  template <typename T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    const size_t nb = (count * sizeof(T) + gran - 1) / gran * gran;
    if (dry) {
      bytes += nb;
      fake += (nb + 255) & ~(size_t)255;
      return reinterpret_cast<T*>(fake);
    }
    if (arena && arena_off + nb <= arena_size) {
      T* p = reinterpret_cast<T*>(arena + arena_off);
      arena_off += nb;
      bytes += nb;
      return p;
    }
    void* p = raw(nb);  // beyond the arena (or none): an array of its own
    bytes += nb;
    return static_cast<T*>(p);
  }
  ~Pool() {
    if (dry || ptrs.empty()) return;
    if (a.release) {
      // the callback may hand the memory to other users at once: nothing may still read it
      if (!owner_synced) (void)hipDeviceSynchronize();
      for (size_t i = 0; i < ptrs.size(); ++i) a.release(ptrs[i], sizes[i], (void*)streams[i], a.ctx);
    } else {
      for (void* p : ptrs) (void)hipFree(p);  // hipFree waits for the device itself
    }
  }
};

// Small pinned host blocks of the batches (read-back scratch), kept for reuse: a
// pinned allocation and its release each cost a round trip to the driver, and a
// serving loop opens and closes batches all the time.  Bounded by the largest
// number of batches alive at once.
struct PinnedCache {
  std::mutex mu;
  std::multimap<size_t, void*> free_;
  void* get(size_t nb) {
    nb = (nb + 4095) & ~(size_t)4095;
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = free_.find(nb);
      if (it != free_.end()) {
        void* p = it->second;
        free_.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    HIPCHECK(hipHostMalloc(&p, nb, hipHostMallocDefault));
    return p;
  }
  void put(void* p, size_t nb) {
    if (!p) return;
    nb = (nb + 4095) & ~(size_t)4095;
    std::lock_guard<std::mutex> lk(mu);
    free_.emplace(nb, p);
  }
};
PinnedCache g_pinned;  // never freed: the blocks live until the process ends

// One grid level in one precision.
template <typename R>
struct Level {
  int lx = 0, lt = 0, dof = 0;
  size_t n = 0;                     // vector length per right-hand side
  bool fine = false;
  const cpx<R>* U = nullptr;        // fine links (fine level only)
  double diag = 0;                  // 2 + m (fine level only)
  cpx<R>* L = nullptr;              // coarse links [9][dof][K][dof] (coarse levels)
  // transfer to the next level
  int bx = 0, bt = 0, nc = 0, ldk = 0;
  int halo = 0;                     // 1: smoothed prolongator on block + one-site ring
  double sa_w = 0;                  // smoothed-aggregation weight w of P = (I - w A) P_t
  cpx<R>* P = nullptr;              // prolongator of the V-cycle, [J][ldk][nw]
  cpx<R>* Pt = nullptr;             // tentative block-orthonormal prolongator [J][ldk][nagg]
  std::vector<double> coefs;        // smoother polynomial
  // work vectors, `cap` columns each
  int cap = 0;
  cpx<R>*b = nullptr, *x = nullptr, *r = nullptr, *t = nullptr, *tmp = nullptr;
  cpx<R>* wbuf = nullptr;           // prolongation scratch, cap * nK * nw values
  void *r_lp = nullptr, *t_lp = nullptr;  // BF16/FP16 smoother iterates (FP32 fine level), cap columns
  hfc* L16 = nullptr;               // FP16 coarse links (operator_storage F16), scaled by 1 / lscale
  float lscale = 1;
  hfc* P16 = nullptr;               // FP16 prolongator (operator_storage F16), scaled by 1 / pscale
  float pscale = 1;
  size_t nkw() const { return bx ? (size_t)(lx / bx) * (lt / bt) * (bx + 2 * halo) * (bt + 2 * halo) * dof : 0; }
};

struct Scal {
  double *bb = nullptr, *rz = nullptr, *pq = nullptr, *ab = nullptr, *rr = nullptr, *tt = nullptr;
  double* rz2 = nullptr;            // second <r,z> slot: the fused CG step reads one and writes the other
  int *active = nullptr, *bad = nullptr;
  // host-visible mirrors of rr and bad in coherent pinned memory, written by the reductions
  // themselves: the per-iteration convergence check needs a synchronisation but no copy
  double* rr_host = nullptr;
  int* bad_host = nullptr;
  int* on_host = nullptr;           // running columns of a defect correction, read by its scale kernel
  double* rr_part_host = nullptr;   // per-block partial |r|^2 of the fused FP32 CG, added up by the host
  int* act_host = nullptr;          // running columns of a Krylov solve, copied to `active` by a kernel
  int rr_part_nb = 0;               // blocks per column in rr_part_host
};

template <typename R>
struct KVecs {
  cpx<R>*r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *t = nullptr;
  cpx<R>* p2 = nullptr;             // second search-direction buffer of the fused CG step
  size_t cap = 0;                   // elements per vector
};

// Per-column operators of a grouped solve (smg_group_*), device arrays of G entries in
// the order of the group's handles: FP32 fine links and diagonals, FP64 fine links and
// diagonals (the defect correction's residual), coarse links and prolongators per
// level of the FP32 V-cycle, the smoother coefficients per level as [nu][G], and the
// coarsest inverse.
struct GroupTab {
  int G = 0;
  Grp U32, U64, M;
  std::vector<Grp> L, P;
  std::vector<const double*> coef;
};

struct Ctx {
  smg_params prm{};
  int nlev = 0;
  int mfma_pin = -1;                // -1: by mfma_min_rhs; 0 / 1: vector ALU / matrix cores
  const GroupTab* grp = nullptr;    // while a grouped solve runs on this context: its systems
  uint64_t gen = 0;                 // bumped whenever operators or coefficients change (captured graphs)
  rocblas_handle blas = nullptr;    // the calling thread's handle during a blocked coarsest inversion
  hipStream_t st = nullptr;
  Pool pool;
  z64* U64 = nullptr;
  z32* U32 = nullptr;
  std::vector<Level<double>> L64;
  std::vector<Level<float>> L32;
  bool f32_ready = false;
  std::vector<z64*> calib;          // smoother calibration start per coarsening
  // mass coefficients of the coarse operators (remass_affine): A^(l)(m) = C2 + m C1 + m^2 C0
  // for every coarse level l >= 1, the prolongators fixed (empty when not kept)
  std::vector<z64*> C0, C1, C2;
  std::vector<size_t> n_plan;       // vector length per level at the full nv (layout of the random starts)
  std::vector<std::vector<double>> factors;  // two-level factors measured by the adaptive stop, per level
  // dense inverse of the coarsest operator
  z64* Minv = nullptr;
  z32* Minv32 = nullptr;            // FP32 copy for the mixed solve's V-cycles
  hfc* Minv16 = nullptr;            // FP16 copy (operator_storage F16), scaled by 1 / mscale
  double mscale = 1;
  double* absmax_part = nullptr;    // per-block maxima for the FP16 scales
  double* cg_partial = nullptr;     // per-workgroup <p, A p> of the fused CG step
  double* rz_partial = nullptr;     // per-workgroup <r, z> of the V-cycle's last fine apply
  size_t cg_partial_cap = 0;
  // set by the FP32 CG around a V-cycle: its last fine apply also leaves the partial
  // sums of <r, z> here (vend_done tells the CG that it did)
  double* vend_partial = nullptr;
  bool vend_done = false;
  z64* colk = nullptr;
  double* piv = nullptr;
  // per-column scalars on the device: one set per CG nesting depth (the outer
  // solve and a coarsest-level CG running inside its V-cycle)
  int scal_cap = 0;
  Red red;                          // reduction scratch
  Scal sc[2];
  double *dc_down = nullptr, *dc_up = nullptr;
  int* fail = nullptr;
  double* h_scal = nullptr;         // pinned host mirrors
  int* h_int = nullptr;
  // Krylov vectors
  KVecs<double> f64, c64;
  KVecs<float> f32, c32;
  z64* r64 = nullptr;               // defect-correction residual
  z32 *b32 = nullptr, *e32 = nullptr;
  size_t dc_cap = 0;
  // setup scratch
  z64 *gX = nullptr, *gY = nullptr, *se = nullptr, *st_ = nullptr, *sz = nullptr;
  // counters
  int64_t fine_applies = 0;
  int64_t vcycles = 0;

  ~Ctx() {
    if (h_scal) (void)hipHostFree(h_scal);
    if (h_int) (void)hipHostFree(h_int);
    for (auto& s : sc) {
      if (s.rr_host) (void)hipHostFree(s.rr_host);
      if (s.bad_host) (void)hipHostFree(s.bad_host);
      if (s.on_host) (void)hipHostFree(s.on_host);
      if (s.rr_part_host) (void)hipHostFree(s.rr_part_host);
      if (s.act_host) (void)hipHostFree(s.act_host);
    }
  }
};

template <typename R>
std::vector<Level<R>>& levels_of(Ctx& c);
template <>
std::vector<Level<double>>& levels_of<double>(Ctx& c) { return c.L64; }
template <>
std::vector<Level<float>>& levels_of<float>(Ctx& c) { return c.L32; }

void sync(Ctx& c) { HIPCHECK(hipStreamSynchronize(c.st)); }
void zero(void* p, size_t bytes, hipStream_t st) { HIPCHECK(hipMemsetAsync(p, 0, bytes, st)); }

void ensure_scalars(Ctx& c, int nrhs) {
  if (nrhs <= c.scal_cap) return;
  const int cap = std::max(nrhs, 8);
  const int nb = red_blocks(c.L64[0].n);
  c.red.partial = c.pool.alloc<double>((size_t)2 * nb * cap);
  for (auto& s : c.sc) {
    s.bb = c.pool.alloc<double>(2 * cap);
    s.rz = c.pool.alloc<double>(2 * cap);
    s.rz2 = c.pool.alloc<double>(2 * cap);
    s.ab = c.pool.alloc<double>(2 * cap);
    s.rr = c.pool.alloc<double>(2 * cap);
    s.tt = c.pool.alloc<double>(2 * cap);
    s.active = c.pool.alloc<int>(cap);
    s.bad = c.pool.alloc<int>(cap);
    if (s.rr_host) (void)hipHostFree(s.rr_host);
    if (s.bad_host) (void)hipHostFree(s.bad_host);
    if (s.on_host) (void)hipHostFree(s.on_host);
    if (s.rr_part_host) (void)hipHostFree(s.rr_part_host);
    if (s.act_host) (void)hipHostFree(s.act_host);
    s.act_host = nullptr;
    s.rr_host = nullptr;
    s.bad_host = nullptr;
    s.on_host = nullptr;
    s.rr_part_host = nullptr;
    s.rr_part_nb = nb;
    if (c.pool.dry) continue;
    HIPCHECK(hipHostMalloc((void**)&s.rr_host, sizeof(double) * 2 * cap, hipHostMallocCoherent));
    HIPCHECK(hipHostMalloc((void**)&s.bad_host, sizeof(int) * cap, hipHostMallocCoherent));
    HIPCHECK(hipHostMalloc((void**)&s.on_host, sizeof(int) * cap, hipHostMallocCoherent));
    HIPCHECK(hipHostMalloc((void**)&s.rr_part_host, sizeof(double) * 2 * nb * cap, hipHostMallocCoherent));
    HIPCHECK(hipHostMalloc((void**)&s.act_host, sizeof(int) * cap, hipHostMallocCoherent));
  }
  c.dc_down = c.pool.alloc<double>(cap);
  c.dc_up = c.pool.alloc<double>(cap);
  c.scal_cap = cap;
  if (c.pool.dry) return;
  if (c.h_scal) (void)hipHostFree(c.h_scal);
  if (c.h_int) (void)hipHostFree(c.h_int);
  c.h_scal = nullptr;
  c.h_int = nullptr;
  HIPCHECK(hipHostMalloc((void**)&c.h_scal, sizeof(double) * 4 * cap, hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void**)&c.h_int, sizeof(int) * 2 * cap, hipHostMallocDefault));
}

// Column work vectors of one level for cap right-hand sides from `pool`.
template <typename R>
void alloc_level_work(Pool& pool, Level<R>& lv, int cap, int smoother_storage) {
  lv.cap = cap;
  lv.b = pool.alloc<cpx<R>>((size_t)cap * lv.n);
  lv.x = pool.alloc<cpx<R>>((size_t)cap * lv.n);
  lv.r = pool.alloc<cpx<R>>((size_t)cap * lv.n);
  lv.t = pool.alloc<cpx<R>>((size_t)cap * lv.n);
  lv.tmp = lv.fine ? pool.alloc<cpx<R>>((size_t)cap * lv.n) : nullptr;
  lv.wbuf = lv.bx ? pool.alloc<cpx<R>>((size_t)cap * lv.nkw()) : nullptr;
  lv.r_lp = lv.t_lp = nullptr;
  if (std::is_same<R, float>::value && lv.fine && smoother_storage != SMG_STORE_F32) {
    lv.r_lp = pool.alloc<uint32_t>((size_t)cap * lv.n);  // 4-byte complex entries
    lv.t_lp = pool.alloc<uint32_t>((size_t)cap * lv.n);
  }
}

template <typename R>
void check_work_geometry(const Ctx& c, const std::vector<Level<R>>& Ls) {
  if ((int)Ls.size() != c.nlev) throw Error(SMG_EINVAL, "level work requested before the levels exist");
  for (size_t l = 0; l + 1 < Ls.size(); ++l)  // every level but the coarsest transfers
    if (!(Ls[l].bx > 0 && Ls[l].nkw() > 0)) throw Error(SMG_EINVAL, "level work requested before the transfer geometry is set");
}

template <typename R>
void ensure_level_work(Ctx& c, int nrhs) {
  auto& Ls = levels_of<R>(c);
  check_work_geometry(c, Ls);
  for (auto& lv : Ls)
    if (lv.cap < nrhs) alloc_level_work<R>(c.pool, lv, nrhs, c.prm.smoother_storage);
}

// Work vectors of every level for cap columns from `pool`, with the shapes of the
// handle's levels: a batch owns such a set, so that they go when the batch goes.
template <typename R>
std::vector<Level<R>> alloc_work_set(Pool& pool, const Ctx& c, const std::vector<Level<R>>& Ls, int cap) {
  check_work_geometry(c, Ls);
  std::vector<Level<R>> w(Ls.begin(), Ls.end());
  for (auto& lv : w) alloc_level_work<R>(pool, lv, cap, c.prm.smoother_storage);
  return w;
}

// Lends the work vectors of `w` to the handle's levels for the lifetime of the loan
// (the V-cycle code reads them from the levels), swapping the handle's own back after.
template <typename R>
struct WorkLoan {
  std::vector<Level<R>>& Ls;
  std::vector<Level<R>>& w;
  void flip() {
    for (size_t l = 0; l < Ls.size() && l < w.size(); ++l) {
      auto& a = Ls[l];
      auto& o = w[l];
      std::swap(a.b, o.b);
      std::swap(a.x, o.x);
      std::swap(a.r, o.r);
      std::swap(a.t, o.t);
      std::swap(a.tmp, o.tmp);
      std::swap(a.wbuf, o.wbuf);
      std::swap(a.r_lp, o.r_lp);
      std::swap(a.t_lp, o.t_lp);
      std::swap(a.cap, o.cap);
    }
  }
  WorkLoan(std::vector<Level<R>>& L, std::vector<Level<R>>& W) : Ls(L), w(W) { flip(); }
  ~WorkLoan() { flip(); }
  WorkLoan(const WorkLoan&) = delete;
  WorkLoan& operator=(const WorkLoan&) = delete;
};

template <typename R>
void alloc_kvecs(Pool& pool, KVecs<R>& v, size_t elems) {
  if (v.cap >= elems) return;
  v.r = pool.alloc<cpx<R>>(elems);
  v.p = pool.alloc<cpx<R>>(elems);
  v.q = pool.alloc<cpx<R>>(elems);
  v.z = pool.alloc<cpx<R>>(elems);
  v.t = pool.alloc<cpx<R>>(elems);
  v.p2 = pool.alloc<cpx<R>>(elems);
  v.cap = elems;
}

template <typename R>
void ensure_kvecs(Ctx& c, KVecs<R>& v, size_t elems) {
  alloc_kvecs<R>(c.pool, v, elems);
}

// Per-workgroup partial sums of the fused FP32 CG step and of the V-cycle's last
// fine apply (nrhs columns).
void ensure_cg_partial(Ctx& c, int nrhs) {
  const int nb = cg_step_blocks<float>(c.L64[0].lx, c.L64[0].lt);
  const size_t need = (size_t)2 * nb * nrhs;
  if (nb == 0 || c.cg_partial_cap >= need) return;
  c.cg_partial = c.pool.alloc<double>(need);
  c.rz_partial = c.pool.alloc<double>(need);
  c.cg_partial_cap = need;
}

// FP64 residual and FP32 right-hand side and correction of defect correction.
void ensure_dc(Ctx& c, size_t elems) {
  if (c.dc_cap >= elems) return;
  c.r64 = c.pool.alloc<z64>(elems);
  c.b32 = c.pool.alloc<z32>(elems);
  c.e32 = c.pool.alloc<z32>(elems);
  c.dc_cap = elems;
}

// ---------------------------------------------------------------------------
// Operators.
// ---------------------------------------------------------------------------
// Coarse applies of many right-hand sides (FP32 and FP64) go to the matrix cores.
// A batch pins the choice for all its V-cycles (mfma_pin), so that a column's
// rounding does not depend on how many other columns run beside it.
bool use_mfma(const Ctx& c, int nc, int nrhs) {
  if (nc > 16) return false;
  if (c.mfma_pin >= 0) return c.mfma_pin == 1;
  return c.prm.mfma_min_rhs > 0 && nrhs >= c.prm.mfma_min_rhs;
}

// The operators of level lv in a grouped solve, with the smoother coefficients of
// step `step` (and step + 1 for the fused last two steps, modes 4 and 5).
template <typename R>
Grp group_ops(const Ctx& c, const Level<R>& lv, int mode, int step) {
  const GroupTab& t = *c.grp;
  const int l = (int)(&lv - levels_of<R>(const_cast<Ctx&>(c)).data());
  Grp g;
  if constexpr (std::is_same<R, float>::value) {
    g = lv.fine ? t.U32 : t.L[l];
  } else {
    if (!lv.fine) throw Error(SMG_EINVAL, "grouped solve: FP64 coarse levels are not grouped");
    g = t.U64;
  }
  if (mode == 1 || mode == 3 || mode == 4 || mode == 5) {
    if (step < 0 || (size_t)l >= t.coef.size()) throw Error(SMG_EINVAL, "grouped solve: smoother step not given");
    g.c = t.coef[l] + (size_t)step * t.G;
    if (mode == 4 || mode == 5) g.c2 = t.coef[l] + (size_t)(step + 1) * t.G;
  }
  return g;
}

// step: which smoother coefficient `coef` is (needed by grouped solves, whose systems
// each have their own), or -1.
template <typename R>
void apply_op(Ctx& c, Level<R>& lv, const cpx<R>* x, cpx<R>* y, int nrhs, int mode, double coef, cpx<R>* xacc,
              const cpx<R>* aux, double coef2 = 0, int step = -1) {
  const Grp g = c.grp ? group_ops<R>(c, lv, mode, step) : Grp{};
  if (lv.fine) {
    launch_normal<R>(lv.U, x, y, lv.tmp, lv.lx, lv.lt, lv.diag, nrhs, mode, coef, xacc, aux, c.st, coef2, g);
    c.fine_applies += nrhs;
    return;
  }
  if constexpr (std::is_same<R, float>::value) {
    if (!c.grp && use_mfma(c, lv.dof, nrhs)) {
      if (lv.L16)
        launch_coarse_mfma_h16(lv.L16, lv.lscale, x, y, lv.lx, lv.lt, lv.dof, nrhs, mode, coef, xacc, aux, c.st,
                               coef2);
      else
        launch_coarse_mfma(lv.L, x, y, lv.lx, lv.lt, lv.dof, nrhs, mode, coef, xacc, aux, c.st, coef2);
      return;
    }
    if (lv.L16) {
      launch_coarse_h16(lv.L16, lv.lscale, x, y, lv.lx, lv.lt, lv.dof, nrhs, mode, coef, xacc, aux, c.st, coef2, g);
      return;
    }
  } else {
    if (use_mfma(c, lv.dof, nrhs)) {
      launch_coarse_mfma64(lv.L, x, y, lv.lx, lv.lt, lv.dof, nrhs, mode, coef, xacc, aux, c.st, coef2);
      return;
    }
  }
  launch_coarse<R>(lv.L, x, y, lv.lx, lv.lt, lv.dof, nrhs, mode, coef, xacc, aux, c.st, coef2, g);
}

template <typename R>
void restrict_to(Ctx& c, Level<R>& lv, const cpx<R>* x, cpx<R>* y, int nrhs) {
  if constexpr (std::is_same<R, float>::value) {
    if (c.grp) {
      const Grp& g = c.grp->P[&lv - c.L32.data()];
      if (lv.P16)
        launch_restrict_s<hfc, z32>(lv.P16, lv.pscale, x, y, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc,
                                    lv.ldk, nrhs, c.st, g);
      else
        launch_restrict_s<z32, z32>(lv.P, 1.0f, x, y, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk,
                                    nrhs, c.st, g);
      return;
    }
    if (lv.P16) {
      launch_restrict_s<hfc, z32>(lv.P16, lv.pscale, x, y, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk,
                                  nrhs, c.st);
      return;
    }
  } else {
    if (use_mfma(c, lv.nc, nrhs)) {
      launch_restrict_mfma64(lv.P, x, y, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk, nrhs, c.st);
      return;
    }
  }
  launch_restrict<R>(lv.P, x, y, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk, nrhs, c.st);
}

template <typename R>
void prolong_from(Ctx& c, Level<R>& lv, const cpx<R>* e, cpx<R>* y, int nrhs, int mode) {
  if constexpr (std::is_same<R, float>::value) {
    if (c.grp) {
      const Grp& g = c.grp->P[&lv - c.L32.data()];
      if (lv.P16)
        launch_prolong_h16(lv.P16, lv.pscale, e, y, lv.wbuf, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc,
                           lv.ldk, nrhs, mode, c.st, g);
      else
        launch_prolong<float>(lv.P, e, y, lv.wbuf, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk, nrhs,
                              mode, c.st, false, g);
      return;
    }
    if (lv.P16) {
      launch_prolong_h16(lv.P16, lv.pscale, e, y, lv.wbuf, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk,
                         nrhs, mode, c.st);
      return;
    }
  }
  launch_prolong<R>(lv.P, e, y, lv.wbuf, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk, nrhs, mode, c.st,
                    std::is_same<R, double>::value && use_mfma(c, lv.nc, nrhs));
}

// x = R b for the frozen MR polynomial, from x = 0 (lv.r / lv.t are ping-pong buffers).
template <typename R>
void smooth(Ctx& c, Level<R>& lv, const cpx<R>* b, cpx<R>* x, int nrhs) {
  const int nu = (int)lv.coefs.size();
  if (nu == 1) {
    launch_zero(x, (size_t)nrhs * lv.n * sizeof(cpx<R>), c.st);
    launch_axpy_const<R>(x, b, lv.coefs[0], lv.n, nrhs, c.st);
    return;
  }
  const cpx<R>* cur = b;
  cpx<R>* bufs[2] = {lv.r, lv.t};
  for (int k = 0; k + 1 < nu; ++k) {
    // the first step sets x = c_0 b rather than accumulating into a cleared x; the
    // last apply also adds the final step's c_{nu-1} r_{nu-1} (no residual is written)
    const bool last = k + 2 == nu;
    const int mode = last ? (k == 0 ? 5 : 4) : (k == 0 ? 3 : 1);
    cpx<R>* nxt = bufs[k & 1];
    apply_op<R>(c, lv, cur, nxt, nrhs, mode, lv.coefs[k], x, nullptr, last ? lv.coefs[k + 1] : 0.0, k);
    cur = nxt;
  }
}

template <typename R>
void coarse_cg(Ctx& c, int l, const cpx<R>* b, cpx<R>* x, int nrhs, double tol, int maxiter);

// Coarsest solve: dense inverse (exact) or CG to coarsest_tol.
template <typename R>
void coarsest_solve(Ctx& c, int l, const cpx<R>* b, cpx<R>* x, int nrhs, bool use_cg) {
  auto& lv = levels_of<R>(c)[l];
  if (!use_cg && c.Minv && l == c.nlev - 1) {
    if constexpr (std::is_same<R, float>::value) {
      const Grp g = c.grp ? c.grp->M : Grp{};
      if (c.prm.coarsest_fp64)  // FP64 inverse and FP64 sums, the FP32 input widened exactly
        launch_dense_apply<double, float>(c.Minv, b, x, (int)lv.n, nrhs, c.st, g);
      else if (c.Minv16)
        launch_dense_apply_h16(c.Minv16, c.mscale, b, x, (int)lv.n, nrhs, c.st, g);
      else
        launch_dense_apply<float, float>(c.Minv32, b, x, (int)lv.n, nrhs, c.st, g);
    }
    else
      launch_dense_apply<double, double>(c.Minv, b, x, (int)lv.n, nrhs, c.st);
  } else
    coarse_cg<R>(c, l, b, x, nrhs, c.prm.coarsest_tol, c.prm.coarsest_maxiter);
}

template <typename S>
void vcycle_fine_lp(Ctx& c, int last, const z32* b, z32* x, int nrhs, bool use_cg);

// One V-cycle on level l (steps 1-5 of the Multigrid section); `last` is the level
// solved exactly.  b is read only; x receives V b.
template <typename R>
void vcycle(Ctx& c, int l, int last, const cpx<R>* b, cpx<R>* x, int nrhs, bool use_cg) {
  auto& Ls = levels_of<R>(c);
  if (l == last) {
    coarsest_solve<R>(c, l, b, x, nrhs, use_cg);
    return;
  }
  if constexpr (std::is_same<R, float>::value) {
    if (l == 0 && c.prm.smoother_storage == SMG_STORE_BF16) {
      vcycle_fine_lp<bfc>(c, last, b, x, nrhs, use_cg);
      return;
    }
    if (l == 0 && c.prm.smoother_storage == SMG_STORE_F16) {
      vcycle_fine_lp<hfc>(c, last, b, x, nrhs, use_cg);
      return;
    }
  }
  Level<R>& lv = Ls[l];
  Level<R>& nx = Ls[l + 1];
  const int nu = (int)lv.coefs.size();
  // 1. x = R^H b (= R b: the polynomial is real), tracking r = b - A x; the
  // first step starts from x = 0 (mode 3 writes x = c_0 b)
  const cpx<R>* cur = b;
  cpx<R>* bufs[2] = {lv.r, lv.t};
  for (int k = 0; k < nu; ++k) {
    cpx<R>* nxt = bufs[k & 1];
    apply_op<R>(c, lv, cur, nxt, nrhs, k == 0 ? 3 : 1, lv.coefs[k], x, nullptr, 0.0, k);
    cur = nxt;
  }
  // 2. r_c = P^H (b - A x)
  restrict_to<R>(c, lv, cur, nx.b, nrhs);
  // 3. e = V^(l+1) r_c
  vcycle<R>(c, l + 1, last, nx.b, nx.x, nrhs, use_cg);
  // 4. x = x + P e
  prolong_from<R>(c, lv, nx.x, x, nrhs, 1);
  // 5. x = x + R (b - A x); the last apply also adds the final step (mode 4) and, when
  // a surrounding FP32 CG asks for it, the partial sums of <b, x>
  apply_op<R>(c, lv, x, lv.r, nrhs, 2, 0.0, nullptr, b);
  cur = lv.r;
  cpx<R>* pb[2] = {lv.t, lv.r};
  if (nu == 1) launch_axpy_const<R>(x, cur, lv.coefs[0], lv.n, nrhs, c.st);
  for (int k = 0; k + 1 < nu; ++k) {
    const bool last = k + 2 == nu;
    cpx<R>* nxt = pb[k & 1];
    if constexpr (std::is_same<R, float>::value) {
      if (last && l == 0 && lv.fine && c.vend_partial) {
        launch_vcycle_end<float>(lv.U, cur, x, b, lv.lx, lv.lt, lv.diag, nrhs, lv.coefs[k], lv.coefs[k + 1],
                                 c.vend_partial, c.st, c.grp ? group_ops<float>(c, lv, 4, k) : Grp{});
        c.fine_applies += nrhs;
        c.vend_done = true;
        break;
      }
    }
    apply_op<R>(c, lv, cur, nxt, nrhs, last ? 4 : 1, lv.coefs[k], x, nullptr, last ? lv.coefs[k + 1] : 0.0, k);
    cur = nxt;
  }
  if (l == 0) c.vcycles += nrhs;
}

// The FP32 V-cycle's fine level with the smoother iterates stored as S (BF16 or
// FP16): the same steps as vcycle, with every residual iterate r_k written and
// read in S while x, b and all arithmetic stay FP32.
template <typename S>
void vcycle_fine_lp(Ctx& c, int last, const z32* b, z32* x, int nrhs, bool use_cg) {
  Level<float>& lv = c.L32[0];
  Level<float>& nx = c.L32[1];
  const int nu = (int)lv.coefs.size();
  S* bufs[2] = {static_cast<S*>(lv.r_lp), static_cast<S*>(lv.t_lp)};
  // 1. pre-smoothing from x = 0 (mode 3 writes x = c_0 b)
  launch_normal_lp<z32, S>(lv.U, b, bufs[0], lv.lx, lv.lt, lv.diag, nrhs, 3, lv.coefs[0], x, nullptr, c.st);
  const S* cur = bufs[0];
  for (int k = 1; k < nu; ++k) {
    S* nxt = bufs[k & 1];
    launch_normal_lp<S, S>(lv.U, cur, nxt, lv.lx, lv.lt, lv.diag, nrhs, 1, lv.coefs[k], x, nullptr, c.st);
    cur = nxt;
  }
  c.fine_applies += (int64_t)nrhs * nu;
  // 2. r_c = P^H (b - A x)
  if (lv.P16)
    launch_restrict_s<hfc, S>(lv.P16, lv.pscale, cur, nx.b, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc,
                              lv.ldk, nrhs, c.st);
  else
    launch_restrict_s<z32, S>(lv.P, 1.0f, cur, nx.b, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, lv.nc, lv.ldk, nrhs,
                              c.st);
  // 3. e = V^(1) r_c
  vcycle<float>(c, 1, last, nx.b, nx.x, nrhs, use_cg);
  // 4. x = x + P e
  prolong_from<float>(c, lv, nx.x, x, nrhs, 1);
  // 5. x = x + R (b - A x)
  launch_normal_lp<z32, S>(lv.U, x, bufs[0], lv.lx, lv.lt, lv.diag, nrhs, 2, 0.0, nullptr, b, c.st);
  c.fine_applies += nrhs;
  cur = bufs[0];
  S* pb[2] = {bufs[1], bufs[0]};
  if (nu == 1) launch_axpy_const_lp<S>(x, cur, lv.coefs[0], lv.n, nrhs, c.st);
  for (int k = 0; k + 1 < nu; ++k) {
    const bool last = k + 2 == nu;  // mode 4: this apply also adds the final step
    S* nxt = pb[k & 1];
    launch_normal_lp<S, S>(lv.U, cur, nxt, lv.lx, lv.lt, lv.diag, nrhs, last ? 4 : 1, lv.coefs[k], x, nullptr, c.st,
                           last ? lv.coefs[k + 1] : 0.0);
    c.fine_applies += nrhs;
    cur = nxt;
  }
  c.vcycles += nrhs;
}

// ---------------------------------------------------------------------------
// Conjugate gradients with per-column scalars on the device.  The host reads
// the residual norms for the convergence test (every iteration, or every 8th
// for the coarsest CG) and confirms convergence on the recomputed residual.
// ---------------------------------------------------------------------------
struct ColStats {
  std::vector<int> iters, status;
  std::vector<double> relres;
};

template <typename R>
// true_check: confirm convergence on the recomputed residual b - A x.  The inner
// FP32 solves of defect correction stop on the recursive residual instead: in FP32
// the recomputed residual of an ill-conditioned system has a rounding floor above
// the inner tolerance, and the outer FP64 loop checks the true residual anyway.
// bb_known: |b|^2 per column when the caller knows it (host array), else NULL and
// it is computed here.  preset: the caller has already set x = 0 and the first
// residual v.r = b.
void pcg(Ctx& c, int l, const cpx<R>* b, cpx<R>* x, int nrhs, double tol, int maxiter, bool precond, KVecs<R>& v,
         ColStats* cs, int check_interval, int depth, bool true_check = true, const double* bb_known = nullptr,
         bool preset = false) {
  auto& lv = levels_of<R>(c)[l];
  Scal& S = c.sc[depth];
  const size_t n = lv.n;
  ensure_scalars(c, nrhs);
  const size_t bytes = (size_t)nrhs * n * sizeof(cpx<R>);
  if (!bb_known) {
    launch_dot<R>(b, b, n, nrhs, c.red, S.bb, c.st, S.rr_host);
    sync(c);
  }
  std::vector<double> hbb(nrhs), rel(nrhs, 0.0);
  std::vector<int> act(nrhs, 1), its(nrhs, 0), stat(nrhs, SMG_NOTCONV);
  for (int j = 0; j < nrhs; ++j) {
    hbb[j] = bb_known ? bb_known[j] : S.rr_host[2 * j];
    if (!std::isfinite(hbb[j])) throw Error(SMG_EBREAKDOWN, "right-hand side contains NaN/Inf");
    if (!(hbb[j] > 0)) {
      act[j] = 0;
      stat[j] = SMG_OK;
    }
  }
  int nact = 0;
  for (int j = 0; j < nrhs; ++j) nact += act[j];
  // The running columns reach the device through host-visible memory and a small
  // kernel, without a synchronisation: the host writes act_host again only after the
  // next synchronisation of this stream, when that kernel has run.
  auto upload_active = [&](bool clear_bad) {
    for (int j = 0; j < nrhs; ++j) S.act_host[j] = act[j];
    launch_set_active(S.active, S.act_host, clear_bad ? S.bad : nullptr, nrhs, c.st);
  };
  if (!preset) {
    zero(x, bytes, c.st);
    HIPCHECK(hipMemcpyAsync(v.r, b, bytes, hipMemcpyDeviceToDevice, c.st));
  }
  for (int j = 0; j < nrhs; ++j) S.bad_host[j] = 0;  // no kernel of this stream is running (synchronised above)
  upload_active(true);
  auto precondition = [&](const cpx<R>* r, cpx<R>* z) {
    if (precond)
      vcycle<R>(c, l, c.nlev - 1, r, z, nrhs, c.prm.coarsest == SMG_COARSEST_CG);
    else
      HIPCHECK(hipMemcpyAsync(z, r, bytes, hipMemcpyDeviceToDevice, c.st));
  };
  // The FP32 outer solve on the fine level takes each CG step in one fused kernel:
  // p = z + beta p_old, q = A p and the partial sums of <p, q> (the search direction
  // alternates between two buffers because neighbouring workgroups read p_old).
  int fuse_nb = 0;
  if constexpr (std::is_same<R, float>::value)
    if (lv.fine) fuse_nb = cg_step_blocks<float>(lv.lx, lv.lt);
  if (fuse_nb > 0) ensure_cg_partial(c, nrhs);
  cpx<R>* p_cur = v.p;
  cpx<R>* p_alt = v.p2;
  // Fused path: <r, z> lives in one of two slots.  When the V-cycle's last fine apply
  // left its partial sums (folded), the next CG step forms beta from them, moves <r, z>
  // to the other slot and the update kernel reads it from there; otherwise a separate
  // pass forms beta and <r, z> in the current slot.
  double* rz_cur = S.rz;
  double* rz_nxt = S.rz2;
  bool folded = false;
  auto precondition_fold = [&](const cpx<R>* r, cpx<R>* z) {
    if (fuse_nb > kBetaFoldMaxBlocks) {  // too many partial sums for the CG step to add itself
      precondition(r, z);
      return false;
    }
    c.vend_partial = c.rz_partial;
    c.vend_done = false;
    precondition(r, z);
    const bool f = c.vend_done;
    c.vend_partial = nullptr;
    c.vend_done = false;
    return f;
  };
  bool first = true;  // the first CG step takes p = z (beta = 0)
  if (nact > 0) {
    if (fuse_nb > 0) {
      folded = precondition_fold(v.r, v.z);
      if (!folded) {
        launch_zero(S.ab, sizeof(double) * 2 * nrhs, c.st);
        launch_dot<R>(v.r, v.z, n, nrhs, c.red, rz_cur, c.st);
      }
    } else {
      precondition(v.r, v.z);
      HIPCHECK(hipMemcpyAsync(v.p, v.z, bytes, hipMemcpyDeviceToDevice, c.st));
      launch_dot<R>(v.r, v.z, n, nrhs, c.red, S.rz, c.st);
    }
  }
  for (int it = 1; it <= maxiter && nact > 0; ++it) {
    bool partials_kept = true;  // red still holds this iteration's |r|^2 partial sums
    if (fuse_nb > 0) {
      if constexpr (std::is_same<R, float>::value) {
        BetaFold bf;
        if (folded) bf = BetaFold{c.rz_partial, fuse_nb, first ? nullptr : rz_cur, rz_nxt, S.active};
        launch_cg_step<float>(lv.U, v.z, p_cur, p_alt, v.q, lv.lx, lv.lt, lv.diag, nrhs, S.ab, c.cg_partial, c.st,
                              bf, c.grp ? group_ops<float>(c, lv, 0, -1) : Grp{});
        c.fine_applies += nrhs;
        std::swap(p_cur, p_alt);
        if (folded) std::swap(rz_cur, rz_nxt);
        first = false;
        // alpha from the step's partial sums inside the update kernel
        launch_axpy_update_fold(x, v.r, p_cur, v.q, c.cg_partial, fuse_nb, rz_cur, S.ab, S.active, S.bad, S.bad_host,
                                n, nrhs, S.rr_part_host, c.st);
      }
    } else {
      apply_op<R>(c, lv, p_cur, v.q, nrhs, 0, 0.0, nullptr, nullptr);
      launch_dot_alpha<R>(p_cur, v.q, n, nrhs, c.red, S.rz, S.ab, S.active, S.bad, c.st, S.bad_host);
      launch_axpy_update<R>(x, v.r, p_cur, v.q, S.ab, n, nrhs, c.red, S.rr, c.st, S.rr_host);
    }
    for (int j = 0; j < nrhs; ++j) its[j] += act[j];
    if (it % check_interval == 0 || it == maxiter) {
      sync(c);  // the reductions wrote |r|^2 and the breakdown flags to S.rr_host / S.bad_host
      if (fuse_nb > 0) {  // |r|^2 from the update kernel's per-block partial sums, in block order
        const int nbp = red_blocks(n);
        for (int j = 0; j < nrhs; ++j) {
          double t = 0;
          for (int b = 0; b < nbp; ++b) t += S.rr_part_host[2 * ((size_t)j * nbp + b)];
          S.rr_host[2 * j] = t;
          S.rr_host[2 * j + 1] = 0;
        }
      }
      if (depth == 0) {  // the outer solve: largest recursive relative residual of the running columns
        double worst = 0;
        for (int j = 0; j < nrhs; ++j)
          if (act[j] && hbb[j] > 0) worst = std::max(worst, std::sqrt(std::max(S.rr_host[2 * j], 0.0) / hbb[j]));
        report("iteration", l, it, maxiter, worst);
      }
      std::vector<int> cand(nrhs, 0);
      bool any_cand = false;
      for (int j = 0; j < nrhs; ++j) {
        if (!act[j]) continue;
        if (S.bad_host[j])
          throw Error(SMG_EBREAKDOWN, "CG breakdown (<p,Ap> <= 0 or NaN) in column " + std::to_string(j));
        const double r2 = S.rr_host[2 * j];
        if (!std::isfinite(r2)) throw Error(SMG_EBREAKDOWN, "CG residual is NaN/Inf");
        if (r2 <= tol * tol * hbb[j]) {
          cand[j] = 1;
          any_cand = true;
        }
      }
      if (any_cand && !true_check) {
        for (int j = 0; j < nrhs; ++j)
          if (cand[j]) {
            act[j] = 0;
            stat[j] = SMG_OK;
            rel[j] = std::sqrt(S.rr_host[2 * j] / hbb[j]);
          }
        nact = 0;
        for (int j = 0; j < nrhs; ++j) nact += act[j];
        upload_active(false);
        if (nact == 0) break;
      } else if (any_cand) {
        // confirm on the true residual t = b - A x
        partials_kept = false;
        apply_op<R>(c, lv, x, v.t, nrhs, 2, 0.0, nullptr, b);
        launch_dot<R>(v.t, v.t, n, nrhs, c.red, S.tt, c.st);
        HIPCHECK(hipMemcpyAsync(c.h_scal, S.tt, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, c.st));
        sync(c);
        bool changed = false;
        for (int j = 0; j < nrhs; ++j) {
          if (!cand[j]) continue;
          const double tr = std::sqrt(c.h_scal[2 * j] / hbb[j]);
          if (tr <= tol) {
            act[j] = 0;
            stat[j] = SMG_OK;
            rel[j] = tr;
            changed = true;
          } else {  // replace the recursive residual by the true one and continue
            HIPCHECK(hipMemcpyAsync(v.r + (size_t)j * n, v.t + (size_t)j * n, n * sizeof(cpx<R>),
                                    hipMemcpyDeviceToDevice, c.st));
          }
        }
        if (changed) {
          nact = 0;
          for (int j = 0; j < nrhs; ++j) nact += act[j];
          upload_active(false);
        }
        if (nact == 0) break;
      }
    }
    if (fuse_nb > 0) {  // the V-cycle's last fine apply also forms the partial sums of <r, z>
      folded = precondition_fold(v.r, v.z);
      if (!folded) launch_dot_beta<R>(v.r, v.z, n, nrhs, c.red, rz_cur, S.ab, S.active, c.st);
    } else if (!precond && partials_kept) {
      // plain CG: z = r, and <r, r> is in the update's partial sums (no copy, no pass over r)
      launch_beta_partials(n, nrhs, c.red, S.rz, S.ab, S.active, c.st);
      launch_xpay<R>(v.r, p_cur, S.ab, n, nrhs, c.st);
    } else {
      precondition(v.r, v.z);
      launch_dot_beta<R>(v.r, v.z, n, nrhs, c.red, S.rz, S.ab, S.active, c.st);
      launch_xpay<R>(v.z, p_cur, S.ab, n, nrhs, c.st);
    }
  }
  if (nact > 0) {  // true residual of the columns that did not converge
    apply_op<R>(c, lv, x, v.t, nrhs, 2, 0.0, nullptr, b);
    launch_dot<R>(v.t, v.t, n, nrhs, c.red, S.tt, c.st);
    HIPCHECK(hipMemcpyAsync(c.h_scal, S.tt, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, c.st));
    sync(c);
    for (int j = 0; j < nrhs; ++j)
      if (act[j]) rel[j] = std::sqrt(c.h_scal[2 * j] / hbb[j]);
  }
  if (cs) {
    cs->iters = its;
    cs->status = stat;
    cs->relres = rel;
  }
}

template <typename R>
KVecs<R>& coarse_kvecs(Ctx& c);
template <>
KVecs<double>& coarse_kvecs<double>(Ctx& c) { return c.c64; }
template <>
KVecs<float>& coarse_kvecs<float>(Ctx& c) { return c.c32; }

// Relative residual of the coarsest CG inside FP32 V-cycles.
constexpr double kCoarseTolF32 = 1e-6;

template <typename R>
void coarse_cg(Ctx& c, int l, const cpx<R>* b, cpx<R>* x, int nrhs, double tol, int maxiter) {
  auto& lv = levels_of<R>(c)[l];
  KVecs<R>& v = coarse_kvecs<R>(c);
  ensure_kvecs<R>(c, v, (size_t)nrhs * lv.n);
  ColStats cs;
  if (std::is_same<R, float>::value) {
    // Inside the FP32 V-cycle of the mixed solve: FP32 cannot confirm a true
    // residual below ~1e-7, so stop on the recursive residual at a reachable
    // tolerance (the outer FP64 iteration corrects what the preconditioner misses).
    pcg<R>(c, l, b, x, nrhs, std::max(tol, kCoarseTolF32), maxiter, false, v, &cs, 8, 1, false);
  } else {
    pcg<R>(c, l, b, x, nrhs, tol, maxiter, false, v, &cs, 8, 1);
  }
  int most = 0;
  double worst = 0;
  for (int j = 0; j < nrhs; ++j) {
    most = std::max(most, cs.iters[j]);
    worst = std::max(worst, cs.relres[j]);
  }
  report("coarsest-cg", l, most, maxiter, worst);
}

// ---------------------------------------------------------------------------
// Hierarchy construction (FP64).
// ---------------------------------------------------------------------------
double dev_dot_re(Ctx& c, const z64* a, const z64* b, size_t n) {
  ensure_scalars(c, 1);
  launch_dot<double>(a, b, n, 1, c.red, c.sc[1].tt, c.st);
  HIPCHECK(hipMemcpyAsync(c.h_scal, c.sc[1].tt, 2 * sizeof(double), hipMemcpyDeviceToHost, c.st));
  sync(c);
  return c.h_scal[0];
}

// Smoother calibration (Results section): nu MR steps from the stored start
// vector, alpha_k = <A r, r> / <A r, A r>, frozen as c_k = omega * alpha_k.
void calibrate(Ctx& c, int l) {
  auto& lv = c.L64[l];
  lv.coefs.clear();
  HIPCHECK(hipMemcpyAsync(lv.r, c.calib[l], lv.n * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
  for (int k = 0; k < c.prm.smoother_steps; ++k) {
    apply_op<double>(c, lv, lv.r, lv.t, 1, 0, 0.0, nullptr, nullptr);
    const double qr = dev_dot_re(c, lv.t, lv.r, lv.n);
    const double qq = dev_dot_re(c, lv.t, lv.t, lv.n);
    if (!(qq > 0) || !std::isfinite(qr)) throw Error(SMG_ESETUP, "smoother calibration broke down");
    const double ck = c.prm.smoother_omega * qr / qq;
    lv.coefs.push_back(ck);
    launch_axpy_const<double>(lv.r, lv.t, -ck, lv.n, 1, c.st);
  }
}

// Set the number of vectors in use between level l and l+1.
void set_nc(Ctx& c, int l, int nc) {
  c.L64[l].nc = nc;
  auto& nx = c.L64[l + 1];
  nx.dof = nc;
  nx.n = (size_t)nx.lx * nx.lt * nc;
}

// Eq. 2 by colouring: for each colour and vector k, apply A^(l) to the sum of the
// k-th prolongator columns of that colour and restrict the image aggregate by
// aggregate; each restriction is column k of one link block.
void galerkin(Ctx& c, int l) {
  auto& lv = c.L64[l];
  auto& nx = c.L64[l + 1];
  const int nc = lv.nc;
  const int cx = lv.lx / lv.bx, ct = lv.lt / lv.bt;
  const size_t nK = (size_t)cx * ct;
  zero(nx.L, 9 * nK * nc * nc * sizeof(z64), c.st);
  const int ncx = colors_along(cx), nct = colors_along(ct);
  for (int a = 0; a < ncx; ++a)
    for (int bcol = 0; bcol < nct; ++bcol)
      for (int k = 0; k < nc; ++k) {
        launch_color_scatter(lv.P, c.gX, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, k, lv.ldk, a, bcol, c.st);
        apply_op<double>(c, lv, c.gX, c.gY, 1, 0, 0.0, nullptr, nullptr);
        launch_color_project(lv.P, c.gY, nx.L, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, lv.halo, nc, lv.ldk, k, a, bcol,
                             c.st);
      }
}

void check_fail(Ctx& c, const char* what) {
  HIPCHECK(hipMemcpyAsync(c.h_int, c.fail, sizeof(int), hipMemcpyDeviceToHost, c.st));
  sync(c);
  if (c.h_int[0]) throw Error(SMG_ESETUP, what);
}

// Smoothed aggregation for column k: P[.][k] = (I - w A) P_t[.][k], by colouring
// (the windows of one colour are disjoint, as are the supports of A P_t on them).
void smooth_column(Ctx& c, int l, int k) {
  auto& lv = c.L64[l];
  if (!lv.halo) return;
  const int ncx = colors_along(lv.lx / lv.bx), nct = colors_along(lv.lt / lv.bt);
  for (int a = 0; a < ncx; ++a)
    for (int b = 0; b < nct; ++b) {
      launch_color_scatter(lv.Pt, c.gX, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, 0, k, lv.ldk, a, b, c.st);
      apply_op<double>(c, lv, c.gX, c.gY, 1, 0, 0.0, nullptr, nullptr);
      launch_sa_extract(c.gX, c.gY, lv.P, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, k, lv.ldk, a, b, lv.sa_w, c.st);
    }
}

// Prolongator columns per candidate vector: 2 with chirality-split aggregates.
inline int cols_per_vector(const smg_params& p) { return p.split_chirality ? 2 : 1; }

// Appends candidate k: column k, or columns 2k and 2k + 1 with chirality-split aggregates.
void gs_append(Ctx& c, int l, const z64* v, int k) {
  auto& lv = c.L64[l];
  const int m = cols_per_vector(c.prm);
  zero(c.fail, sizeof(int), c.st);
  launch_gs_append((double*)lv.Pt, v, lv.lx, lv.lt, lv.dof, lv.bx, lv.bt, k, lv.ldk, m, c.fail, c.st);
  check_fail(c, "block Gram-Schmidt: candidate vector is degenerate on an aggregate");
  for (int chi = 0; chi < m; ++chi) smooth_column(c, l, m * k + chi);
}

// Smoothed-aggregation weight of level l: w = sa_scale / lambda, lambda the Rayleigh
// quotient after 20 power iterations of A^(l) from the calibration start.
void sa_weight(Ctx& c, int l) {
  auto& lv = c.L64[l];
  if (!lv.halo) return;
  HIPCHECK(hipMemcpyAsync(lv.r, c.calib[l], lv.n * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
  double lam = 0;
  for (int it = 0; it < 20; ++it) {
    apply_op<double>(c, lv, lv.r, lv.t, 1, 0, 0.0, nullptr, nullptr);
    lam = dev_dot_re(c, lv.r, lv.t, lv.n) / dev_dot_re(c, lv.r, lv.r, lv.n);
    const double nt = std::sqrt(dev_dot_re(c, lv.t, lv.t, lv.n));
    if (!(nt > 0) || !std::isfinite(lam)) throw Error(SMG_ESETUP, "power iteration for lambda_max broke down");
    HIPCHECK(hipMemcpyAsync(lv.r, lv.t, lv.n * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
    launch_scale_const<double>(lv.r, 1.0 / nt, lv.n, 1, c.st);
  }
  lv.sa_w = c.prm.sa_scale / lam;
}

// In-place inversion of a Hermitian positive definite n x n matrix by blocked
// Gauss-Jordan elimination without pivoting.  The buffer is taken column-major
// (B = M^T for the row-major M; inverting B gives inv(M)^T, i.e. inv(M) row-major).
// Per block column k (width m): P = inv(B_kk) (unblocked steps), R = P B_k*,
// B -= C R with C = B_*k and its block k zeroed, then row block k = R, column
// block k = -C P and B_kk = P.  The three products are plain GEMMs (rocBLAS).
constexpr int kGJBlock = 512;

std::mutex g_blas_mu;
std::vector<rocblas_handle> g_blas_free;

void blas_check(rocblas_status s) {
  if (s != rocblas_status_success) throw Error(SMG_EDEVICE, std::string("rocBLAS: ") + rocblas_status_to_string(s));
}

void blocked_gauss_jordan(Ctx& c, z64* B, int n) {
  // a rocBLAS handle from a process-wide pool (a handle holds device workspace of its
  // own and serves one thread at a time): as many handles as inversions ever ran at
  // once, kept until the process ends, instead of one per hierarchy
  struct Lease {
    Ctx& c;
    rocblas_handle h = nullptr;
    explicit Lease(Ctx& cc) : c(cc) {
      {
        std::lock_guard<std::mutex> lk(g_blas_mu);
        if (!g_blas_free.empty()) {
          h = g_blas_free.back();
          g_blas_free.pop_back();
        }
      }
      if (!h) blas_check(rocblas_create_handle(&h));
      c.blas = h;
    }
    ~Lease() {
      c.blas = nullptr;
      std::lock_guard<std::mutex> lk(g_blas_mu);
      g_blas_free.push_back(h);
    }
  } lease{c};
  blas_check(rocblas_set_stream(c.blas, c.st));
  const int nb = kGJBlock;
  Pool scratch;  // released after the final synchronisation below
  scratch.stream = &c.st;
  z64* C = scratch.alloc<z64>((size_t)n * nb);
  z64* R = scratch.alloc<z64>((size_t)n * nb);
  z64* P = scratch.alloc<z64>((size_t)nb * nb);
  const size_t zs = sizeof(z64);
  const rocblas_double_complex one = {1.0, 0.0}, mone = {-1.0, 0.0}, zer = {0.0, 0.0};
  auto zc = [](z64* p) { return reinterpret_cast<rocblas_double_complex*>(p); };
  for (int kb = 0; kb < n; kb += nb) {
    const int m = std::min(nb, n - kb);
    // C = B[:, kb:kb+m] (contiguous columns), P = its diagonal block, then zero that block of C
    HIPCHECK(hipMemcpyAsync(C, B + (size_t)kb * n, (size_t)n * m * zs, hipMemcpyDeviceToDevice, c.st));
    HIPCHECK(hipMemcpy2DAsync(P, m * zs, C + kb, (size_t)n * zs, m * zs, m, hipMemcpyDeviceToDevice, c.st));
    HIPCHECK(hipMemset2DAsync(C + kb, (size_t)n * zs, 0, m * zs, m, c.st));
    for (int k = 0; k < m; ++k) launch_gj_step(P, m, k, c.colk, c.piv, c.fail, c.st);
    // R = P B[kb:kb+m, :]
    blas_check(rocblas_zgemm(c.blas, rocblas_operation_none, rocblas_operation_none, m, n, m, &one, zc(P), m,
                             zc(B + kb), n, &zer, zc(R), m));
    // B -= C R (row block kb is untouched: C is zero there)
    blas_check(rocblas_zgemm(c.blas, rocblas_operation_none, rocblas_operation_none, n, n, m, &mone, zc(C), n,
                             zc(R), m, &one, zc(B), n));
    HIPCHECK(hipMemcpy2DAsync(B + kb, (size_t)n * zs, R, m * zs, m * zs, n, hipMemcpyDeviceToDevice, c.st));
    // B[:, kb:kb+m] = -C P, then its diagonal block = P
    blas_check(rocblas_zgemm(c.blas, rocblas_operation_none, rocblas_operation_none, n, m, m, &mone, zc(C), n,
                             zc(P), m, &zer, zc(B + (size_t)kb * n), n));
    HIPCHECK(hipMemcpy2DAsync(B + (size_t)kb * n + kb, (size_t)n * zs, P, m * zs, m * zs, m, hipMemcpyDeviceToDevice,
                              c.st));
  }
  HIPCHECK(hipStreamSynchronize(c.st));  // the scratch buffers are freed on return
  scratch.owner_synced = true;           // only this stream used them
}

// Dense inverse of the coarsest operator by Gauss-Jordan elimination (FP64).
void build_coarsest_inverse(Ctx& c) {
  if (c.nlev < 2 || c.prm.coarsest != SMG_COARSEST_DIRECT) return;
  auto& lv = c.L64[c.nlev - 1];
  const int n = (int)lv.n;
  if (!c.Minv) throw Error(SMG_EINVAL, "coarsest inverse not reserved");
  launch_coarse_to_dense(lv.L, c.Minv, lv.lx, lv.lt, lv.dof, c.st);
  zero(c.fail, sizeof(int), c.st);
  if (n <= kGJBlock)
    for (int k = 0; k < n; ++k) launch_gj_step(c.Minv, n, k, c.colk, c.piv, c.fail, c.st);
  else
    blocked_gauss_jordan(c, c.Minv, n);
  check_fail(c, "coarsest operator is not positive definite");
}

void scale_to_unit(Ctx& c, z64* e, size_t n) {
  const double nrm = std::sqrt(dev_dot_re(c, e, e, n));
  if (!(nrm > 0) || !std::isfinite(nrm)) throw Error(SMG_ESETUP, "candidate vector vanished or is not finite");
  launch_scale_const<double>(e, 1.0 / nrm, n, 1, c.st);
}

// Convergence factor of the current two-level cycle on level l (Adaptive Multigrid
// section: vectors are added until the V-cycle reduces a random error sufficiently):
// from the level's calibration start e, nv_stop_iters passes of e <- e - V(A e), then
// (||e||_A / ||e_0||_A)^(1 / passes).  The coarse system is solved by CG to
// coarsest_tol, as in the setup's cycles.
double two_level_factor(Ctx& c, int l) {
  auto& lv = c.L64[l];
  const size_t n = lv.n;
  const int it = c.prm.nv_stop_iters;
  HIPCHECK(hipMemcpyAsync(c.se, c.calib[l], n * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
  apply_op<double>(c, lv, c.se, c.st_, 1, 0, 0.0, nullptr, nullptr);
  const double n0 = std::sqrt(dev_dot_re(c, c.se, c.st_, n));
  for (int i = 0; i < it; ++i) {
    vcycle<double>(c, l, l + 1, c.st_, c.sz, 1, true);
    launch_axpy_const<double>(c.se, c.sz, -1.0, n, 1, c.st);
    apply_op<double>(c, lv, c.se, c.st_, 1, 0, 0.0, nullptr, nullptr);
  }
  const double e2 = dev_dot_re(c, c.se, c.st_, n);
  if (!(n0 > 0) || !std::isfinite(e2)) throw Error(SMG_ESETUP, "two-level factor: the error is not finite");
  return std::pow(std::sqrt(std::max(e2, 0.0)) / n0, 1.0 / it);
}

// Adaptive setup of coarsening l (Adaptive Multigrid section).  rnd holds the
// 1 + nv random starts of this level (row 0 was used for the calibration).
void adaptive_level(Ctx& c, int l, const z64* rnd) {
  auto& lv = c.L64[l];
  const int nv = c.prm.nv[l];
  const size_t n = lv.n;
  // first candidate: relaxation alone on A e = 0 (Eq. 4 with the frozen smoother)
  HIPCHECK(hipMemcpyAsync(c.se, rnd + n, n * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
  for (int it = 0; it < c.prm.setup_iters; ++it) {
    apply_op<double>(c, lv, c.se, c.st_, 1, 0, 0.0, nullptr, nullptr);
    smooth<double>(c, lv, c.st_, c.sz, 1);
    launch_axpy_const<double>(c.se, c.sz, -1.0, n, 1, c.st);
    scale_to_unit(c, c.se, n);
  }
  const int m = cols_per_vector(c.prm);
  set_nc(c, l, m);
  gs_append(c, l, c.se, 0);
  galerkin(c, l);
  report("candidate", l, 1, nv, 0.0);
  // at most the variables of an aggregate (fewer per site when the level above stopped early)
  const int nmax = std::min(nv, lv.bx * lv.bt * lv.dof / m);
  // further candidates: the current two-level V-cycle as error propagator; with
  // nv_stop_rho > 0 the level keeps what it has once that cycle's factor is small enough
  for (int k = 1; k <= nmax; ++k) {
    if (c.prm.nv_stop_rho > 0) {
      c.factors[l].push_back(two_level_factor(c, l));
      if (c.factors[l].back() <= c.prm.nv_stop_rho) break;
    }
    if (k == nmax) break;
    HIPCHECK(hipMemcpyAsync(c.se, rnd + (size_t)(1 + k) * n, n * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
    for (int it = 0; it < c.prm.setup_iters; ++it) {
      apply_op<double>(c, lv, c.se, c.st_, 1, 0, 0.0, nullptr, nullptr);
      vcycle<double>(c, l, l + 1, c.st_, c.sz, 1, true);
      launch_axpy_const<double>(c.se, c.sz, -1.0, n, 1, c.st);
      scale_to_unit(c, c.se, n);
    }
    gs_append(c, l, c.se, k);
    set_nc(c, l, m * (k + 1));
    galerkin(c, l);
    report("candidate", l, k + 1, nv, c.factors[l].empty() ? 0.0 : c.factors[l].back());
  }
}

void validate(const smg_params& p) {
  if (p.lx <= 0 || p.lt <= 0) throw Error(SMG_EINVAL, "lattice extents must be positive");
  if (p.levels < 1 || p.levels > SMG_MAXLEV) throw Error(SMG_EINVAL, "levels must be in [1, SMG_MAXLEV]");
  if (p.smoother_steps < 1 || p.smoother_steps > 64) throw Error(SMG_EINVAL, "smoother_steps must be in [1, 64]");
  if (!(p.smoother_omega > 0)) throw Error(SMG_EINVAL, "smoother_omega must be positive");
  if (p.setup_iters < 0) throw Error(SMG_EINVAL, "setup_iters must be >= 0");
  if (!(p.coarsest_tol > 0) || p.coarsest_maxiter < 1) throw Error(SMG_EINVAL, "bad coarsest CG settings");
  if (!std::isfinite(p.mass)) throw Error(SMG_EINVAL, "mass must be finite");
  if (p.coarsest != SMG_COARSEST_DIRECT && p.coarsest != SMG_COARSEST_CG) throw Error(SMG_EINVAL, "bad coarsest");
  if (!(p.sa_scale >= 0) || !std::isfinite(p.sa_scale)) throw Error(SMG_EINVAL, "sa_scale must be >= 0");
  if (p.smoother_storage < SMG_STORE_F32 || p.smoother_storage > SMG_STORE_F16)
    throw Error(SMG_EINVAL, "bad smoother_storage");
  if (p.operator_storage != SMG_STORE_F32 && p.operator_storage != SMG_STORE_F16)
    throw Error(SMG_EINVAL, "operator_storage must be SMG_STORE_F32 or SMG_STORE_F16");
  if (p.split_chirality != 0 && p.split_chirality != 1) throw Error(SMG_EINVAL, "split_chirality must be 0 or 1");
  if (p.coarsest_fp64 != 0 && p.coarsest_fp64 != 1) throw Error(SMG_EINVAL, "coarsest_fp64 must be 0 or 1");
  if (p.remass_affine != 0 && p.remass_affine != 1) throw Error(SMG_EINVAL, "remass_affine must be 0 or 1");
  if (!(p.nv_stop_rho >= 0) || !std::isfinite(p.nv_stop_rho)) throw Error(SMG_EINVAL, "nv_stop_rho must be >= 0");
  if (p.nv_stop_rho > 0 && (p.nv_stop_iters < 1 || p.nv_stop_iters > 100))
    throw Error(SMG_EINVAL, "nv_stop_iters must be in [1, 100]");
  const int m = p.split_chirality ? 2 : 1;
  if (p.smoother_storage != SMG_STORE_F32 && (p.levels < 2 || !normal_lp_fits(p.lx, p.lt)))
    throw Error(SMG_EINVAL, "BF16/FP16 smoother storage needs levels >= 2, lx % 32 == 0 and lt % 16 == 0");
  int lx = p.lx, lt = p.lt, dof = 2;
  for (int l = 0; l + 1 < p.levels; ++l) {
    const int bx = p.block[l][0], bt = p.block[l][1];
    if (bx < 1 || bt < 1) throw Error(SMG_EINVAL, "block extents must be positive");
    if (lx % bx || lt % bt) throw Error(SMG_ESHAPE, "lattice extent not divisible by the block extent");
    const int nv = p.nv[l];
    if (nv < 1 || m * nv > 64) throw Error(SMG_EINVAL, "nv must be in [1, 64] (in [1, 32] with split_chirality)");
    if (m * nv > bx * bt * dof) throw Error(SMG_EINVAL, "nv exceeds the variables of an aggregate");
    if (bx * bt * dof > 1024) throw Error(SMG_EINVAL, "aggregates larger than 1024 variables are not supported");
    lx /= bx;
    lt /= bt;
    dof = m * nv;
  }
  if ((size_t)p.lx * p.lt * 2 > (size_t)1 << 30) throw Error(SMG_EINVAL, "lattice too large");
}

// New context with every device array allocated.  The fermion links come from
// `gauge` (ABI layout) or are copied from `src_links` (already prepared).  A dry
// context only counts the bytes of the same allocations (neither is read).
// arena: bytes of the block that create and reserve_setup carve their arrays from
// (setup_arena_bytes), so that building a hierarchy costs one allocator call for
// them; 0: one allocation per array.  Arrays are rounded to 256 bytes either way, in
// dry (planning) contexts too.
Ctx* create(const double* gauge, const smg_params* prm, hipStream_t st, const z64* src_links = nullptr,
            bool dry = false, size_t arena = 0) {
  if ((!gauge && !src_links && !dry) || !prm) throw Error(SMG_EINVAL, "null gauge or params");
  validate(*prm);
  Ctx* c = new Ctx();
  try {
    c->pool.dry = dry;
    c->pool.stream = &c->st;
    c->pool.gran = 256;
    c->prm = *prm;
    c->st = st;
    if (!dry && arena) c->pool.open_arena(arena);
    c->nlev = prm->levels;
    const int lx = prm->lx, lt = prm->lt;
    const size_t V = (size_t)lx * lt;
    c->U64 = c->pool.alloc<z64>(2 * V);
    if (dry) {
    } else if (src_links) {
      HIPCHECK(hipMemcpyAsync(c->U64, src_links, 2 * V * sizeof(z64), hipMemcpyDeviceToDevice, st));
    } else {
      launch_prepare_links<double>((const z64*)gauge, c->U64, lx, lt, prm->t_antiperiodic, st);
    }
    c->L64.resize(c->nlev);
    c->L64[0].lx = lx;
    c->L64[0].lt = lt;
    c->L64[0].dof = 2;
    c->L64[0].n = 2 * V;
    c->L64[0].fine = true;
    c->L64[0].U = c->U64;
    c->L64[0].diag = 2.0 + prm->mass;
    size_t maxn = 2 * V;
    for (int l = 1; l < c->nlev; ++l) {
      auto& pv = c->L64[l - 1];
      auto& lv = c->L64[l];
      lv.lx = pv.lx / prm->block[l - 1][0];
      lv.lt = pv.lt / prm->block[l - 1][1];
      lv.dof = prm->nv[l - 1] * (prm->split_chirality ? 2 : 1);
      lv.n = (size_t)lv.lx * lv.lt * lv.dof;
      lv.L = c->pool.alloc<z64>(9 * (size_t)lv.lx * lv.lt * lv.dof * lv.dof);
      pv.bx = prm->block[l - 1][0];
      pv.bt = prm->block[l - 1][1];
      pv.nc = lv.dof;
      pv.ldk = lv.dof;
      pv.Pt = c->pool.alloc<z64>((size_t)lv.lx * lv.lt * lv.dof * pv.bx * pv.bt * pv.dof);
      // smoothed aggregation where the 9-point coarse stencil survives it
      pv.halo = (prm->sa_scale > 0 && pv.bx >= 4 && pv.bt >= 4 && lv.lx >= 2 && lv.lt >= 2) ? 1 : 0;
      if (pv.halo)
        pv.P = c->pool.alloc<z64>((size_t)lv.lx * lv.lt * lv.dof * (pv.bx + 2) * (pv.bt + 2) * pv.dof);
      else
        pv.P = pv.Pt;
    }
    for (auto& lv : c->L64) c->n_plan.push_back(lv.n);
    c->factors.assign(c->nlev, {});
    c->fail = c->pool.alloc<int>(4);
    ensure_scalars(*c, 1);
    ensure_level_work<double>(*c, 1);
    if (c->nlev > 1) {
      c->gX = c->pool.alloc<z64>(maxn);
      c->gY = c->pool.alloc<z64>(maxn);
      c->se = c->pool.alloc<z64>(maxn);
      c->st_ = c->pool.alloc<z64>(maxn);
      c->sz = c->pool.alloc<z64>(maxn);
    }
    return c;
  } catch (...) {
    delete c;
    throw;
  }
}

// Power-of-two scale s with max|a| / s in [0.5, 1) (1 for an all-zero array): FP16
// copies store a / s, so every stored entry is at most 1 in magnitude.
constexpr int kAbsmaxBlocks = 256;

double fp16_scale(Ctx& c, const z64* a, size_t n) {
  constexpr int kBlocks = kAbsmaxBlocks;
  launch_absmax_partial(a, n, c.absmax_part, kBlocks, c.st);
  double h[kBlocks];
  HIPCHECK(hipMemcpyAsync(h, c.absmax_part, sizeof h, hipMemcpyDeviceToHost, c.st));
  sync(c);
  double m = 0;
  for (double v : h) m = std::max(m, v);
  if (!std::isfinite(m)) throw Error(SMG_EBREAKDOWN, "operator contains NaN/Inf");
  if (!(m > 0)) return 1.0;
  int e = 0;
  std::frexp(m, &e);
  return std::ldexp(1.0, e);
}

// FP32 (and FP16) copies of the hierarchy for the mixed-precision solves: the
// arrays (alloc_f32), then their contents from the FP64 operators (ensure_f32).
void alloc_f32(Ctx& c) {
  if (!c.L32.empty()) return;
  const bool h16 = c.prm.operator_storage == SMG_STORE_F16;
  c.L32.resize(c.nlev);
  c.U32 = c.pool.alloc<z32>(c.L64[0].n);  // 2 links per site, as many as vector entries
  for (int l = 0; l < c.nlev; ++l) {
    auto& a = c.L64[l];
    auto& b = c.L32[l];
    // the shape, transfer geometry included: work buffers are sized from it
    b.lx = a.lx; b.lt = a.lt; b.dof = a.dof; b.n = a.n; b.fine = a.fine;
    b.bx = a.bx; b.bt = a.bt; b.nc = a.nc; b.ldk = a.ldk; b.halo = a.halo;
    if (a.fine) b.U = c.U32;
    if (a.L) {
      const size_t nl = 9 * (size_t)a.lx * a.lt * a.dof * a.dof;
      b.L = c.pool.alloc<z32>(nl);
      if (h16) b.L16 = c.pool.alloc<hfc>(nl);
    }
    if (a.P) {
      const size_t np = (size_t)(a.lx / a.bx) * (a.lt / a.bt) * a.ldk * (a.bx + 2 * a.halo) * (a.bt + 2 * a.halo) * a.dof;
      b.P = c.pool.alloc<z32>(np);
      if (h16) b.P16 = c.pool.alloc<hfc>(np);
    }
  }
  if (c.Minv && !c.prm.coarsest_fp64) {
    const size_t nn = c.L64[c.nlev - 1].n * c.L64[c.nlev - 1].n;
    c.Minv32 = c.pool.alloc<z32>(nn);
    if (h16) c.Minv16 = c.pool.alloc<hfc>(nn);
  }
  if (h16) c.absmax_part = c.pool.alloc<double>(kAbsmaxBlocks);
}

void ensure_f32(Ctx& c) {
  if (c.f32_ready) return;
  alloc_f32(c);
  const bool h16 = c.prm.operator_storage == SMG_STORE_F16;
  launch_links_convert<float>(c.U64, c.U32, c.L64[0].n, c.st);  // 2V links == n entries
  for (int l = 0; l < c.nlev; ++l) {
    auto& a = c.L64[l];
    auto& b = c.L32[l];
    b.lx = a.lx; b.lt = a.lt; b.dof = a.dof; b.n = a.n; b.fine = a.fine; b.diag = a.diag;
    b.bx = a.bx; b.bt = a.bt; b.nc = a.nc; b.ldk = a.ldk; b.coefs = a.coefs; b.halo = a.halo; b.sa_w = a.sa_w;
    if (a.L) {
      const size_t nl = 9 * (size_t)a.lx * a.lt * a.dof * a.dof;
      launch_links_convert<float>(a.L, b.L, nl, c.st);
      if (h16) {
        const double sc = fp16_scale(c, a.L, nl);
        b.lscale = (float)sc;
        launch_convert_h16(a.L, b.L16, nl, 1.0 / sc, c.st);
      }
    }
    if (a.P) {
      const size_t np = (size_t)(a.lx / a.bx) * (a.lt / a.bt) * a.ldk * (a.bx + 2 * a.halo) * (a.bt + 2 * a.halo) * a.dof;
      launch_links_convert<float>(a.P, b.P, np, c.st);
      if (h16) {
        const double sc = fp16_scale(c, a.P, np);
        b.pscale = (float)sc;
        launch_convert_h16(a.P, b.P16, np, 1.0 / sc, c.st);
      }
    }
  }
  if (c.Minv32) {
    const size_t nn = c.L64[c.nlev - 1].n * c.L64[c.nlev - 1].n;
    launch_links_convert<float>(c.Minv, c.Minv32, nn, c.st);
    if (h16) {
      c.mscale = fp16_scale(c, c.Minv, nn);
      launch_convert_h16(c.Minv, c.Minv16, nn, 1.0 / c.mscale, c.st);
    }
  }
  c.f32_ready = true;
  ++c.gen;
}

// Every allocation a setup makes beyond create(): the calibration start of every
// coarsening and the dense coarsest inverse with its elimination scratch.
size_t links_count(const Level<double>& lv) { return 9 * (size_t)lv.lx * lv.lt * lv.dof * lv.dof; }

void reserve_setup(Ctx& c, bool coefficients = true) {
  c.calib.assign(c.nlev, nullptr);
  for (int l = 0; l + 1 < c.nlev; ++l) c.calib[l] = c.pool.alloc<z64>(c.L64[l].n);
  if (coefficients && c.prm.remass_affine && c.nlev > 1) {
    c.C0.assign(c.nlev, nullptr);
    c.C1.assign(c.nlev, nullptr);
    c.C2.assign(c.nlev, nullptr);
    for (int l = 1; l < c.nlev; ++l) {
      const size_t nl = links_count(c.L64[l]);
      c.C0[l] = c.pool.alloc<z64>(nl);
      c.C1[l] = c.pool.alloc<z64>(nl);
      c.C2[l] = c.pool.alloc<z64>(nl);
    }
  }
  if (c.nlev > 1 && c.prm.coarsest == SMG_COARSEST_DIRECT) {
    const size_t n = c.L64[c.nlev - 1].n;
    c.Minv = c.pool.alloc<z64>(n * n);
    c.colk = c.pool.alloc<z64>(n);
    c.piv = c.pool.alloc<double>(1);
  }
}

// Bytes that create and reserve_setup(coefficients) allocate for these parameters,
// from the same calls on a dry context.
size_t setup_arena_bytes(const smg_params* prm, bool coefficients) {
  std::unique_ptr<Ctx> d(create(nullptr, prm, nullptr, nullptr, true));
  reserve_setup(*d, coefficients);
  return d->pool.bytes;
}

// Every allocation of a solve of nrhs columns in `prec` (smg_solve, smg_cg).
void reserve_solve(Ctx& c, int nrhs, int prec) {
  const size_t n = c.L64[0].n;
  const bool cg = c.nlev > 1 && c.prm.coarsest == SMG_COARSEST_CG;
  ensure_scalars(c, nrhs);
  ensure_level_work<double>(c, nrhs);
  if (prec == SMG_FP64) {
    ensure_kvecs<double>(c, c.f64, (size_t)nrhs * n);
    if (cg) ensure_kvecs<double>(c, c.c64, (size_t)nrhs * c.L64[c.nlev - 1].n);
  } else {
    alloc_f32(c);
    ensure_level_work<float>(c, nrhs);
    ensure_kvecs<float>(c, c.f32, (size_t)nrhs * n);
    ensure_dc(c, (size_t)nrhs * n);
    ensure_cg_partial(c, nrhs);
    if (cg) ensure_kvecs<float>(c, c.c32, (size_t)nrhs * c.L64[c.nlev - 1].n);
  }
}

// The handle's own growth when a batch of cap slots in `prec` is created on it.
void reserve_batch_handle(Ctx& c, int cap, int prec) {
  if (prec == SMG_MIXED) alloc_f32(c);  // the batch brings its own column work vectors
  if (c.nlev > 1 && c.prm.coarsest == SMG_COARSEST_CG) {  // the coarsest CG of the batch's V-cycles
    ensure_scalars(c, cap);
    if (prec == SMG_MIXED)
      ensure_kvecs<float>(c, c.c32, (size_t)cap * c.L64[c.nlev - 1].n);
    else
      ensure_kvecs<double>(c, c.c64, (size_t)cap * c.L64[c.nlev - 1].n);
  }
}

// Mass coefficients of every coarse operator (Results section: the vectors of one
// setup serve other masses).  D(m) = D0 + m, so A(m) = D0^H D0 + m (D0 + D0^H) + m^2
// and, with the prolongators fixed, every Galerkin operator is C2 + m C1 + m^2 C0 on
// each level.  The three coefficient arrays come from the Galerkin chain at
// m = 0, +1, -1: C2 = G(0), C1 = (G(1) - G(-1)) / 2, C0 = (G(1) + G(-1)) / 2 - G(0).
// The links of the setup mass are left as they were.
void build_mass_coefficients(Ctx& c) {
  if (c.C0.empty()) return;
  const int L = c.nlev;
  Pool keep;  // the setup mass's links, restored at the end
  keep.stream = &c.st;
  std::vector<z64*> saved(L, nullptr);
  for (int l = 1; l < L; ++l) {
    const size_t nl = links_count(c.L64[l]);
    saved[l] = keep.alloc<z64>(nl);
    HIPCHECK(hipMemcpyAsync(saved[l], c.L64[l].L, nl * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
  }
  const double diag0 = c.L64[0].diag;
  const double masses[3] = {0.0, 1.0, -1.0};
  z64** dst[3] = {c.C2.data(), c.C1.data(), c.C0.data()};  // G(0), G(1), G(-1) first
  for (int j = 0; j < 3; ++j) {
    c.L64[0].diag = 2.0 + masses[j];
    for (int l = 0; l + 1 < L; ++l) galerkin(c, l);
    for (int l = 1; l < L; ++l)
      HIPCHECK(hipMemcpyAsync(dst[j][l], c.L64[l].L, links_count(c.L64[l]) * sizeof(z64), hipMemcpyDeviceToDevice,
                              c.st));
  }
  for (int l = 1; l < L; ++l) {
    const size_t nl = links_count(c.L64[l]);
    z64* tmp = c.L64[l].L;  // holds C0 until C1 has been formed in place
    launch_lincomb3(c.C1[l], c.C0[l], c.C2[l], tmp, 0.5, 0.5, -1.0, nl, c.st);
    launch_lincomb3(c.C1[l], c.C0[l], c.C0[l], c.C1[l], 0.5, -0.5, 0.0, nl, c.st);
    HIPCHECK(hipMemcpyAsync(c.C0[l], tmp, nl * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
    HIPCHECK(hipMemcpyAsync(c.L64[l].L, saved[l], nl * sizeof(z64), hipMemcpyDeviceToDevice, c.st));
  }
  c.L64[0].diag = diag0;
  sync(c);  // the saved links are released on return
}

// Coarse operators of `dst` at its mass from the mass coefficients of `src` (the
// same prolongators): one pass over the links per level instead of Eq. 2.
void affine_links(Ctx& dst, const Ctx& src, double m) {
  for (int l = 1; l < dst.nlev; ++l)
    launch_lincomb3(src.C2[l], src.C1[l], src.C0[l], dst.L64[l].L, 1.0, m, m * m, links_count(dst.L64[l]), dst.st);
}

void finish_setup(Ctx& c) {
  build_coarsest_inverse(c);
  c.f32_ready = false;
  ++c.gen;
  sync(c);
}

// Offsets into the caller's concatenated per-level blocks, laid out at the full nv of
// every coarsening (the planned vector lengths).
size_t level_offset_randoms(const Ctx& c, int l, bool with_calib) {
  size_t off = 0;
  for (int q = 0; q < l; ++q) off += (size_t)(c.prm.nv[q] + (with_calib ? 1 : 0)) * c.n_plan[q];
  return off;
}

size_t level_offset_plain(const Ctx& c, int l) {
  size_t off = 0;
  for (int q = 0; q < l; ++q) off += c.n_plan[q];
  return off;
}

// Stable C-side view of stats.
void fill_stats(smg_stats* s, int nrhs, const ColStats& cs, int refinements, int64_t applies, int64_t vcyc,
                double secs) {
  if (!s) return;
  for (int j = 0; j < nrhs; ++j) {
    s[j].status = cs.status.empty() ? SMG_OK : cs.status[j];
    s[j].iterations = cs.iters.empty() ? 0 : cs.iters[j];
    s[j].refinements = refinements;
    s[j].vcycles = (int32_t)(vcyc / std::max(nrhs, 1));
    s[j].fine_applies = applies / std::max(nrhs, 1);
    s[j].true_relres = cs.relres.empty() ? 0.0 : cs.relres[j];
    s[j].seconds = secs;
  }
}

int fail_code(const Error& e) {
  g_last_error = e.what();
  return e.code;
}

Ctx* H(smg_handle h) {
  if (!h) throw Error(SMG_EINVAL, "null handle");
  return reinterpret_cast<Ctx*>(h);
}

int check_level(Ctx* c, int level) {
  if (level < 0 || level >= c->nlev) throw Error(SMG_EINVAL, "level out of range");
  return level;
}

void check_nrhs(int nrhs) {
  if (nrhs < 1 || nrhs > 4096) throw Error(SMG_EINVAL, "nrhs must be in [1, 4096]");
}

// ---------------------------------------------------------------------------
// Continuous batching: MG-CG over a fixed set of column slots of one handle.
// Every column keeps its own Krylov scalars and is frozen on the device when it
// converges, so a column's iterates do not depend on which other slots are busy
// or when they were admitted.  FP64: MG-CG as in smg_solve.  Mixed: FP64 flexible
// CG preconditioned by the FP32 V-cycle (defect correction's restarts do not fit
// admission at any time).
// ---------------------------------------------------------------------------
struct Batch {
  Ctx* c = nullptr;
  int cap = 0;
  double tol = 1e-10;
  int maxiter = 0;
  int prec = SMG_FP64;
  size_t n = 0;
  Pool pool;
  z64 *b = nullptr, *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *zo = nullptr,
      *t = nullptr;
  z32 *r32 = nullptr, *z32v = nullptr;
  std::vector<Level<double>> w64;  // the batch's own column work vectors of every level
  std::vector<Level<float>> w32;
  Red red;
  Scal S;
  double* rzo = nullptr;
  double* h = nullptr;  // pinned host scratch
  int* hi_ = nullptr;
  std::vector<int> used, act, its, stat, bad;
  std::vector<double> bb, rel;
  int64_t applies0 = 0;
  hipStream_t st0 = nullptr;  // stream of smg_batch_create (handed to the allocator)
  // One captured graph of an iteration's device work per number of leading slots
  // (pointers and coefficients are fixed for a given count); dropped when the
  // handle's operators change.
  bool use_graphs = false;
  std::vector<hipGraphExec_t> graphs;
  uint64_t graph_gen = 0;
  hipStream_t gs = nullptr;  // the batch's own stream: graphs cannot be captured on the null stream
  hipEvent_t ev = nullptr;
  std::vector<hipStream_t> seen;  // every stream a call of the batch enqueued work on
  void note(hipStream_t s) {
    if (std::find(seen.begin(), seen.end(), s) == seen.end()) seen.push_back(s);
  }
  void drop_graphs() {
    for (auto& g : graphs)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
  ~Batch() {
    drop_graphs();
    if (ev) (void)hipEventDestroy(ev);
    if (gs) (void)hipStreamDestroy(gs);
    g_pinned.put(h, sizeof(double) * 2 * cap);
    g_pinned.put(hi_, sizeof(int) * cap);
  }
  int hi() const {
    int m = 0;
    for (int j = 0; j < cap; ++j)
      if (used[j]) m = j + 1;
    return m;
  }
};

// Every device array of a batch of B.cap slots (B.n, B.prec set).
void batch_alloc(Batch& B) {
  const int cap = B.cap;
  const size_t e = (size_t)cap * B.n;
  B.b = B.pool.alloc<z64>(e);
  B.x = B.pool.alloc<z64>(e);
  B.r = B.pool.alloc<z64>(e);
  B.p = B.pool.alloc<z64>(e);
  B.q = B.pool.alloc<z64>(e);
  B.z = B.pool.alloc<z64>(e);
  B.t = B.pool.alloc<z64>(e);
  if (B.prec == SMG_MIXED) {
    B.zo = B.pool.alloc<z64>(e);
    B.r32 = B.pool.alloc<z32>(e);
    B.z32v = B.pool.alloc<z32>(e);
    B.rzo = B.pool.alloc<double>(2 * cap);
  }
  B.red.partial = B.pool.alloc<double>((size_t)2 * red_blocks(B.n) * cap);
  B.S.bb = B.pool.alloc<double>(2 * cap);
  B.S.rz = B.pool.alloc<double>(2 * cap);
  B.S.pq = B.pool.alloc<double>(2 * cap);
  B.S.ab = B.pool.alloc<double>(2 * cap);
  B.S.rr = B.pool.alloc<double>(2 * cap);
  B.S.tt = B.pool.alloc<double>(2 * cap);
  B.S.active = B.pool.alloc<int>(cap);
  B.S.bad = B.pool.alloc<int>(cap);
  B.w64 = alloc_work_set<double>(B.pool, *B.c, B.c->L64, cap);
  if (B.prec == SMG_MIXED) B.w32 = alloc_work_set<float>(B.pool, *B.c, B.c->L32, cap);
}

void batch_upload_active(Batch& B, hipStream_t st) {
  for (int j = 0; j < B.cap; ++j) B.hi_[j] = B.act[j];
  HIPCHECK(hipMemcpyAsync(B.S.active, B.hi_, sizeof(int) * B.cap, hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));
}

// z = M r on columns [j0, j0 + cnt) (the V-cycle; FP32 for mixed).
void batch_precondition(Batch& B, int j0, int cnt, hipStream_t st) {
  Ctx& c = *B.c;
  c.st = st;
  const size_t off = (size_t)j0 * B.n;
  if (c.nlev < 2) {
    HIPCHECK(hipMemcpyAsync(B.z + off, B.r + off, (size_t)cnt * B.n * sizeof(z64), hipMemcpyDeviceToDevice, st));
    return;
  }
  const bool cg = c.prm.coarsest == SMG_COARSEST_CG;
  struct Pin {  // restored on every exit path
    Ctx& c;
    ~Pin() { c.mfma_pin = -1; }
  } pin{c};
  c.mfma_pin = (c.prm.mfma_min_rhs > 0 && B.cap >= c.prm.mfma_min_rhs) ? 1 : 0;
  if (B.prec == SMG_FP64) {
    vcycle<double>(c, 0, c.nlev - 1, B.r + off, B.z + off, cnt, cg);
  } else {
    launch_convert<float, double>(B.r + off, B.r32 + off, (size_t)cnt * B.n, st);
    vcycle<float>(c, 0, c.nlev - 1, B.r32 + off, B.z32v + off, cnt, cg);
    launch_convert<double, float>(B.z32v + off, B.z + off, (size_t)cnt * B.n, st);
  }
}

// A slot that stops running keeps x; its r, z and p are cleared so that the
// shared V-cycle sees a zero (finite) column there.
void batch_clear(Batch& B, int j, hipStream_t st) {
  const size_t off = (size_t)j * B.n, bytes = B.n * sizeof(z64);
  zero(B.r + off, bytes, st);
  zero(B.z + off, bytes, st);
  zero(B.p + off, bytes, st);
  if (B.zo) zero(B.zo + off, bytes, st);
}

// One MG-CG iteration per step of the loop, ordered so that a fresh slot joins
// without work of its own: z = M r, beta (0 for a fresh slot, whose <r,z>_old is
// 0), p = z + beta p, q = A p, alpha, x/r update, convergence check.
// The device work of one iteration over slots [0, hi): no host synchronisation,
// memset or allocation, so it can be captured as a graph.
void batch_iter_device(Batch& B, int hi, hipStream_t st) {
  Ctx& c = *B.c;
  c.st = st;
  auto& lv = c.L64[0];
  const size_t n = B.n;
  if (B.prec == SMG_MIXED) launch_links_convert<double>(B.z, B.zo, (size_t)hi * n, st);  // z_old = z
  batch_precondition(B, 0, hi, st);
  if (B.prec == SMG_MIXED) {
    launch_dot<double>(B.r, B.z, n, hi, B.red, B.S.pq, st);
    launch_dot<double>(B.r, B.zo, n, hi, B.red, B.rzo, st);
    launch_cg_beta_flex(B.S.pq, B.rzo, B.S.rz, B.S.ab, B.S.active, hi, st);
  } else {
    launch_dot_beta<double>(B.r, B.z, n, hi, B.red, B.S.rz, B.S.ab, B.S.active, st);
  }
  launch_xpay<double>(B.z, B.p, B.S.ab, n, hi, st);
  apply_op<double>(c, lv, B.p, B.q, hi, 0, 0.0, nullptr, nullptr);
  launch_dot_alpha<double>(B.p, B.q, n, hi, B.red, B.S.rz, B.S.ab, B.S.active, B.S.bad, st);
  launch_axpy_update<double>(B.x, B.r, B.p, B.q, B.S.ab, n, hi, B.red, B.S.rr, st);
}

void batch_step(Batch& B, int iters, hipStream_t st) {
  Ctx& c = *B.c;
  c.st = st;
  auto& lv = c.L64[0];
  const size_t n = B.n;
  if (B.prec == SMG_MIXED) ensure_f32(c);
  // the V-cycle and the fine applies run on the batch's own work vectors
  WorkLoan<double> loan64(c.L64, B.w64);
  std::vector<Level<float>> none32;
  WorkLoan<float> loan32(c.L32, B.prec == SMG_MIXED ? B.w32 : none32);
  if (B.graph_gen != c.gen) {
    B.drop_graphs();
    B.graph_gen = c.gen;
  }
  for (int it = 0; it < iters; ++it) {
    const int hi = B.hi();
    int nact = 0;
    for (int j = 0; j < hi; ++j) nact += B.act[j];
    if (nact == 0) return;
    if (B.use_graphs) {
      // replay on the batch's own stream, after the caller's work on st
      HIPCHECK(hipEventRecord(B.ev, st));
      HIPCHECK(hipStreamWaitEvent(B.gs, B.ev, 0));
      hipGraphExec_t& g = B.graphs[hi];
      if (!g) {
        hipGraph_t graph = nullptr;
        HIPCHECK(hipStreamBeginCapture(B.gs, hipStreamCaptureModeThreadLocal));
        try {
          batch_iter_device(B, hi, B.gs);
        } catch (...) {
          (void)hipStreamEndCapture(B.gs, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          c.st = st;
          throw;
        }
        HIPCHECK(hipStreamEndCapture(B.gs, &graph));
        const hipError_t e = hipGraphInstantiate(&g, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHECK(e);
      }
      HIPCHECK(hipGraphLaunch(g, B.gs));
      HIPCHECK(hipMemcpyAsync(B.h, B.S.rr, sizeof(double) * 2 * hi, hipMemcpyDeviceToHost, B.gs));
      HIPCHECK(hipMemcpyAsync(B.hi_, B.S.bad, sizeof(int) * hi, hipMemcpyDeviceToHost, B.gs));
      HIPCHECK(hipStreamSynchronize(B.gs));
      c.st = st;
    } else {
      batch_iter_device(B, hi, st);
      HIPCHECK(hipMemcpyAsync(B.h, B.S.rr, sizeof(double) * 2 * hi, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipMemcpyAsync(B.hi_, B.S.bad, sizeof(int) * hi, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
    }
    bool changed = false, any_cand = false;
    std::vector<int> cand(hi, 0);
    auto stop = [&](int j, int status, double rel) {
      B.act[j] = 0;
      B.stat[j] = status;
      B.rel[j] = rel;
      batch_clear(B, j, st);
      changed = true;
    };
    for (int j = 0; j < hi; ++j) {
      if (!B.act[j]) continue;
      B.its[j] += 1;
      const double r2 = B.h[2 * j];
      if (B.hi_[j] || !std::isfinite(r2)) {
        stop(j, SMG_EBREAKDOWN, std::numeric_limits<double>::quiet_NaN());
        continue;
      }
      if (r2 <= B.tol * B.tol * B.bb[j]) {
        cand[j] = 1;
        any_cand = true;
      }
    }
    if (any_cand) {  // confirm on the true residual t = b - A x
      apply_op<double>(c, lv, B.x, B.t, hi, 2, 0.0, nullptr, B.b);
      launch_dot<double>(B.t, B.t, n, hi, B.red, B.S.tt, st);
      HIPCHECK(hipMemcpyAsync(B.h, B.S.tt, sizeof(double) * 2 * hi, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipStreamSynchronize(st));
      for (int j = 0; j < hi; ++j) {
        if (!cand[j]) continue;
        const double tr = std::sqrt(B.h[2 * j] / B.bb[j]);
        if (tr <= B.tol)
          stop(j, SMG_OK, tr);
        else
          HIPCHECK(hipMemcpyAsync(B.r + (size_t)j * n, B.t + (size_t)j * n, n * sizeof(z64), hipMemcpyDeviceToDevice,
                                  st));
      }
    }
    for (int j = 0; j < hi; ++j)
      if (B.act[j] && B.its[j] >= B.maxiter) stop(j, SMG_NOTCONV, std::sqrt(B.h[2 * j] / B.bb[j]));
    if (changed) batch_upload_active(B, st);
  }
}

Batch* BH(smg_batch b) {
  if (!b) throw Error(SMG_EINVAL, "null batch");
  return reinterpret_cast<Batch*>(b);
}

// ---------------------------------------------------------------------------
// V-cycle without allocation.  Its per-level work vectors come from one static
// device array per GPU instead of the handle's pool, so a call allocates nothing.
// The host never names the array itself: its address on each device is taken once
// with hipGetSymbolAddress, with that device current, and passed to the kernels.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = SMG_NOALLOC_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kScratchDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

unsigned char* scratch_on_current_device() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) throw Error(SMG_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHECK(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(SMG_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  return g_scratch_ptr[dev];
}

// Work vectors of every level for nrhs columns carved out of `base` (256-byte
// aligned pieces); returns the bytes they take.  With base == nullptr only counts.
size_t carve_level_work(Ctx& c, int nrhs, unsigned char* base, std::vector<Level<double>>* out) {
  size_t off = 0;
  auto take = [&](size_t elems) -> z64* {
    z64* p = base ? reinterpret_cast<z64*>(base + off) : nullptr;
    off += (elems * sizeof(z64) + 255) & ~(size_t)255;
    return p;
  };
  for (int l = 0; l < c.nlev; ++l) {
    Level<double> w = c.L64[l];
    const size_t n = (size_t)nrhs * w.n;
    w.b = take(n);
    w.x = take(n);
    w.r = take(n);
    w.t = take(n);
    w.tmp = w.fine ? take(n) : nullptr;
    w.wbuf = w.bx ? take((size_t)nrhs * w.nkw()) : nullptr;
    w.cap = nrhs;
    if (out) (*out)[l] = w;
  }
  return off;
}

}  // namespace
}  // namespace smg

using namespace smg;

#define API_BEGIN try {
#define API_END                                   \
  }                                               \
  catch (const Error& e) {                        \
    return fail_code(e);                          \
  }                                               \
  catch (const std::exception& e) {               \
    g_last_error = e.what();                      \
    return SMG_EINVAL;                            \
  }

// FP64 defect correction around FP32 MG-CG (smg_solve with SMG_MIXED, and grouped
// solves): rhs, x complex128 [nrhs][n] on the fine level; per-column results in cs.
void solve_mixed(Ctx* c, const double* rhs, double* x, int nrhs, double tol, int maxiter, ColStats& cs,
                 int& refinements) {
  const bool mg = c->nlev > 1;
  auto& lv = c->L64[0];
  const size_t n = lv.n;
  ensure_f32(*c);
  const z64* b = (const z64*)rhs;
  z64* xx = (z64*)x;
  launch_dc_start(b, c->r64, xx, (size_t)nrhs * n, c->st);  // r = b, x = 0
  std::vector<double> hbb(nrhs), rel(nrhs, 0.0), down(nrhs), up(nrhs);
  std::vector<int> act(nrhs, 1), its(nrhs, 0), stat(nrhs, SMG_NOTCONV);
  refinements = 0;
  int used = 0;
  std::vector<double> bb_inner(nrhs);
  bool first = true;
  while (true) {
    launch_dot<double>(c->r64, c->r64, n, nrhs, c->red, c->sc[1].rr, c->st, c->sc[1].rr_host);
    sync(*c);
    if (first) {  // r = b: the first norms are |b|^2
      first = false;
      for (int j = 0; j < nrhs; ++j) {
        hbb[j] = c->sc[1].rr_host[2 * j];
        if (!std::isfinite(hbb[j])) throw Error(SMG_EBREAKDOWN, "right-hand side contains NaN/Inf");
        if (!(hbb[j] > 0)) { act[j] = 0; stat[j] = SMG_OK; }
      }
    }
    int nact = 0;
    for (int j = 0; j < nrhs; ++j) {
      if (!act[j]) { down[j] = 0; up[j] = 0; continue; }
      const double rr = c->sc[1].rr_host[2 * j];
      if (!std::isfinite(rr)) throw Error(SMG_EBREAKDOWN, "defect correction residual is NaN/Inf");
      rel[j] = std::sqrt(rr / hbb[j]);
      if (rel[j] <= tol) { act[j] = 0; stat[j] = SMG_OK; down[j] = 0; up[j] = 0; continue; }
      down[j] = 1.0 / std::sqrt(rr);
      up[j] = std::sqrt(rr);
      ++nact;
    }
    if (refinements > 0) {  // true relative residual after this many passes (largest column)
      double worst = 0;
      for (int j = 0; j < nrhs; ++j) worst = std::max(worst, rel[j]);
      report("refinement", 0, refinements, maxiter, worst);
    }
    if (nact == 0 || used >= maxiter) break;
    // the same scales on the device, from the same |r|^2 and this decision (no copy)
    for (int j = 0; j < nrhs; ++j) c->sc[1].on_host[j] = down[j] != 0 ? 1 : 0;
    launch_dc_scales(c->sc[1].rr, c->sc[1].on_host, c->dc_down, c->dc_up, nrhs, c->st);
    launch_scale_down_start(c->r64, c->b32, c->f32.r, c->e32, c->dc_down, n, nrhs, c->st);
    ColStats inner;
    // The inner solve's own convergence test uses inner_tol; its limit is what is
    // left of maxiter.  Its right-hand side has unit norm in every running column.
    for (int j = 0; j < nrhs; ++j) bb_inner[j] = down[j] != 0 ? 1.0 : 0.0;
    pcg<float>(*c, 0, c->b32, c->e32, nrhs, c->prm.inner_tol, std::max(1, maxiter - used), mg, c->f32, &inner, 1, 0,
               false, bb_inner.data(), true);
    int maxit = 0;
    for (int j = 0; j < nrhs; ++j) {
      if (down[j] != 0) its[j] += inner.iters[j];
      maxit = std::max(maxit, inner.iters[j]);
    }
    used += std::max(maxit, 1);
    launch_scale_up_add(xx, c->e32, c->dc_up, n, nrhs, c->st);
    apply_op<double>(*c, lv, xx, c->r64, nrhs, 2, 0.0, nullptr, b);
    ++refinements;
  }
  cs.iters = its;
  cs.status = stat;
  cs.relres = rel;
}

// A grouped solve: independent systems of one shape (lattice, levels, vectors per
// level, storage) solved together, system j in column j of every launch of the mixed
// solve, so each launch does the work of all of them.  The first handle's context
// runs the solve (its work vectors for G columns, its stream); the per-column
// operator tables point into every handle's own arrays.
struct Group {
  std::vector<Ctx*> cs;
  std::vector<uint64_t> gens;  // each handle's operator generation when the tables were filled
  Pool pool;                   // the tables
  GroupTab tab;
  // host copies of the tables, uploaded after each fill
  std::vector<const void*> h_ptr;
  std::vector<double> h_val;
  const void** d_ptr = nullptr;
  double* d_val = nullptr;
};

Group* GH(smg_group g) {
  if (!g) throw Error(SMG_EINVAL, "null group");
  return reinterpret_cast<Group*>(g);
}

// The shape and storage a grouped solve needs every system to share.
void group_check(const Ctx& a, const Ctx& b) {
  const smg_params &p = a.prm, &q = b.prm;
  bool same = p.lx == q.lx && p.lt == q.lt && a.nlev == b.nlev && p.smoother_steps == q.smoother_steps &&
              p.operator_storage == q.operator_storage && p.smoother_storage == q.smoother_storage &&
              p.coarsest == q.coarsest && p.coarsest_fp64 == q.coarsest_fp64 && p.split_chirality == q.split_chirality;
  for (int l = 0; same && l < a.nlev; ++l) {
    const auto &x = a.L32[l], &y = b.L32[l];
    same = x.lx == y.lx && x.lt == y.lt && x.dof == y.dof && x.nc == y.nc && x.ldk == y.ldk && x.halo == y.halo &&
           x.bx == y.bx && x.bt == y.bt && x.coefs.size() == y.coefs.size() && (x.L16 == nullptr) == (y.L16 == nullptr) &&
           (x.P16 == nullptr) == (y.P16 == nullptr);
  }
  if (!same) throw Error(SMG_EINVAL, "grouped systems differ in shape, levels, vectors per level or storage");
}

// Fill the per-column tables from every handle's current operators (FP32 copies
// brought up to date first).
void group_fill(Group& g, hipStream_t st) {
  const int G = (int)g.cs.size();
  for (Ctx* c : g.cs) {
    c->st = st;
    ensure_f32(*c);
  }
  Ctx& c0 = *g.cs[0];
  const int nl = c0.nlev;
  for (Ctx* c : g.cs) group_check(c0, *c);
  // layout of the pointer table: U32, U64, M, then L per level, then P per level (G each);
  // of the value table: diag32, diag64, mscale, lscale per level, pscale per level, then
  // the coefficients of every level ([nu][G])
  const int nptr = 3 + 2 * nl, nu = (int)c0.L32[0].coefs.size();
  const int nval = 3 + 2 * nl + nl * nu;
  g.h_ptr.assign((size_t)nptr * G, nullptr);
  g.h_val.assign((size_t)nval * G, 0.0);
  auto P = [&](int slot, int j) -> const void*& { return g.h_ptr[(size_t)slot * G + j]; };
  auto V = [&](int slot, int j) -> double& { return g.h_val[(size_t)slot * G + j]; };
  for (int j = 0; j < G; ++j) {
    Ctx& c = *g.cs[j];
    P(0, j) = c.L32[0].U;
    V(0, j) = c.L32[0].diag;
    P(1, j) = c.L64[0].U;
    V(1, j) = c.L64[0].diag;
    const bool m16 = !c.prm.coarsest_fp64 && c.Minv16;
    P(2, j) = c.prm.coarsest_fp64 ? (const void*)c.Minv : (m16 ? (const void*)c.Minv16 : (const void*)c.Minv32);
    V(2, j) = m16 ? c.mscale : 1.0;
    for (int l = 0; l < nl; ++l) {
      const auto& lv = c.L32[l];
      P(3 + l, j) = lv.L16 ? (const void*)lv.L16 : (const void*)lv.L;
      V(3 + l, j) = lv.L16 ? lv.lscale : 1.0;
      P(3 + nl + l, j) = lv.P16 ? (const void*)lv.P16 : (const void*)lv.P;
      V(3 + nl + l, j) = lv.P16 ? lv.pscale : 1.0;
      for (int k = 0; k < (int)lv.coefs.size(); ++k) V(3 + 2 * nl + l * nu + k, j) = lv.coefs[k];
    }
  }
  if (!g.d_ptr) {
    g.pool.stream = &c0.st;
    g.d_ptr = reinterpret_cast<const void**>(g.pool.alloc<uint64_t>((size_t)nptr * G));
    g.d_val = g.pool.alloc<double>((size_t)nval * G);
  }
  HIPCHECK(hipMemcpyAsync(g.d_ptr, g.h_ptr.data(), g.h_ptr.size() * sizeof(void*), hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync(g.d_val, g.h_val.data(), g.h_val.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));  // the host copies may change at the next fill
  auto grp = [&](int pslot, int vslot) {
    Grp r;
    r.op = g.d_ptr + (size_t)pslot * G;
    r.s = g.d_val + (size_t)vslot * G;
    return r;
  };
  GroupTab& t = g.tab;
  t.G = G;
  t.U32 = grp(0, 0);
  t.U64 = grp(1, 1);
  t.M = grp(2, 2);
  t.L.assign(nl, Grp{});
  t.P.assign(nl, Grp{});
  t.coef.assign(nl, nullptr);
  for (int l = 0; l < nl; ++l) {
    t.L[l] = grp(3 + l, 3 + l);
    t.P[l] = grp(3 + nl + l, 3 + nl + l);
    t.coef[l] = g.d_val + (size_t)(3 + 2 * nl + l * nu) * G;
  }
  g.gens.resize(G);
  for (int j = 0; j < G; ++j) g.gens[j] = g.cs[j]->gen;
}

extern "C" {

void smg_default_params(smg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->lx = 32;
  p->lt = 32;
  p->mass = 0.1;
  p->levels = 2;
  for (int l = 0; l < SMG_MAXLEV; ++l) {
    p->block[l][0] = 4;
    p->block[l][1] = 4;
    p->nv[l] = 8;
  }
  p->setup_iters = 5;
  p->smoother_steps = 4;
  p->smoother_omega = 0.8;
  p->t_antiperiodic = 1;
  p->coarsest = SMG_COARSEST_DIRECT;
  p->coarsest_tol = 1e-12;
  p->coarsest_maxiter = 10000;
  p->inner_tol = 1e-5;
  p->seed = 1;
  p->sa_scale = 4.0 / 3.0;
  p->mfma_min_rhs = 16;
  p->operator_storage = SMG_STORE_F32;
  p->split_chirality = 0;
  p->coarsest_fp64 = 1;
  p->remass_affine = 0;
  p->nv_stop_rho = 0.0;
  p->nv_stop_iters = 3;
}

int smg_setup(const double* gauge, const smg_params* params, const double* randoms, void* stream,
              smg_handle* out) {
  API_BEGIN
  if (!out) throw Error(SMG_EINVAL, "null output handle");
  hipStream_t st = (hipStream_t)stream;
  Ctx* c = create(gauge, params, st, nullptr, false, params ? setup_arena_bytes(params, true) : 0);
  try {
    reserve_setup(*c);
    // The random starts and the Krylov vectors of the setup cycles' coarse CG live
    // only while the setup runs (released after its final synchronisation).
    Pool tmp;
    tmp.stream = &c->st;
    size_t cgmax = 0;
    for (int l = 1; l < c->nlev; ++l) cgmax = std::max(cgmax, c->L64[l].n);
    if (cgmax) alloc_kvecs<double>(tmp, c->c64, cgmax);
    for (int l = 0; l + 1 < c->nlev; ++l) {
      // n is shorter than the planned length when the level above kept fewer vectors
      // (nv_stop_rho): then the leading n entries of each given row are used
      const size_t n = c->L64[l].n, np = c->n_plan[l];
      const int nv = c->prm.nv[l];
      z64* rnd = tmp.alloc<z64>((1 + (size_t)nv) * n);
      if (randoms) {
        HIPCHECK(hipMemcpy2DAsync(rnd, n * sizeof(z64), (const z64*)randoms + level_offset_randoms(*c, l, true),
                                  np * sizeof(z64), n * sizeof(z64), 1 + (size_t)nv, hipMemcpyDeviceToDevice, st));
      } else {
        for (int row = 0; row <= nv; ++row)
          launch_random_gaussian(rnd + (size_t)row * n, n, c->prm.seed, (uint64_t)l * 4096 + row, st);
      }
      HIPCHECK(hipMemcpyAsync(c->calib[l], rnd, n * sizeof(z64), hipMemcpyDeviceToDevice, st));  // row 0
      calibrate(*c, l);
      report("calibrate", l, 0, nv, 0.0);
      sa_weight(*c, l);
      adaptive_level(*c, l, rnd);
    }
    build_mass_coefficients(*c);
    finish_setup(*c);
    report("coarsest", c->nlev - 1, 0, 0, 0.0);
    c->c64 = KVecs<double>{};
  } catch (...) {
    delete c;
    throw;
  }
  *out = reinterpret_cast<smg_handle>(c);
  return SMG_OK;
  API_END
}

int smg_setup_from_vectors(const double* gauge, const smg_params* params, const double* vectors, const double* calib,
                           void* stream, smg_handle* out) {
  API_BEGIN
  if (!out || !vectors || !calib) throw Error(SMG_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  Ctx* c = create(gauge, params, st, nullptr, false, params ? setup_arena_bytes(params, true) : 0);
  try {
    reserve_setup(*c);
    for (int l = 0; l + 1 < c->nlev; ++l) {
      const size_t n = c->L64[l].n;
      const int nv = c->prm.nv[l];
      HIPCHECK(hipMemcpyAsync(c->calib[l], (const z64*)calib + level_offset_plain(*c, l), n * sizeof(z64),
                              hipMemcpyDeviceToDevice, st));
      calibrate(*c, l);
      sa_weight(*c, l);
      const z64* vl = (const z64*)vectors + level_offset_randoms(*c, l, false);
      for (int k = 0; k < nv; ++k) gs_append(*c, l, vl + (size_t)k * n, k);
      set_nc(*c, l, nv * cols_per_vector(c->prm));
      galerkin(*c, l);
    }
    build_mass_coefficients(*c);
    finish_setup(*c);
  } catch (...) {
    delete c;
    throw;
  }
  *out = reinterpret_cast<smg_handle>(c);
  return SMG_OK;
  API_END
}

int smg_set_mass(smg_handle h, double mass, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  if (!std::isfinite(mass)) throw Error(SMG_EINVAL, "mass must be finite");
  c->st = (hipStream_t)stream;
  c->prm.mass = mass;
  c->L64[0].diag = 2.0 + mass;
  if (!c->C0.empty()) {
    affine_links(*c, *c, mass);
    for (int l = 0; l + 1 < c->nlev; ++l) calibrate(*c, l);
  } else {
    for (int l = 0; l + 1 < c->nlev; ++l) {
      calibrate(*c, l);
      galerkin(*c, l);
    }
  }
  finish_setup(*c);
  return SMG_OK;
  API_END
}

int smg_derive(smg_handle h, double mass, void* stream, smg_handle* out) {
  API_BEGIN
  Ctx* src = H(h);
  if (!out) throw Error(SMG_EINVAL, "null output handle");
  if (!std::isfinite(mass)) throw Error(SMG_EINVAL, "mass must be finite");
  hipStream_t st = (hipStream_t)stream;
  // What is read from src (links, prolongators, calibration starts) is written only
  // by the setup calls, which synchronise before they return, so src may be in use
  // on another stream meanwhile; its stream field is not touched.
  smg_params prm = src->prm;
  prm.mass = mass;
  Ctx* c = create(nullptr, &prm, st, src->U64, false, setup_arena_bytes(&prm, false));
  try {
    reserve_setup(*c, false);  // a derived handle keeps no mass coefficients of its own
    for (int l = 0; l + 1 < c->nlev; ++l) {
      auto& a = src->L64[l];
      auto& b = c->L64[l];
      const size_t np = (size_t)(a.lx / a.bx) * (a.lt / a.bt) * a.ldk * a.bx * a.bt * a.dof;
      HIPCHECK(hipMemcpyAsync(b.Pt, a.Pt, np * sizeof(z64), hipMemcpyDeviceToDevice, st));
      if (a.halo) {
        const size_t nw = (size_t)(a.lx / a.bx) * (a.lt / a.bt) * a.ldk * (a.bx + 2) * (a.bt + 2) * a.dof;
        HIPCHECK(hipMemcpyAsync(b.P, a.P, nw * sizeof(z64), hipMemcpyDeviceToDevice, st));
      }
      b.sa_w = a.sa_w;
      HIPCHECK(hipMemcpyAsync(c->calib[l], src->calib[l], a.n * sizeof(z64), hipMemcpyDeviceToDevice, st));
    }
    for (int l = 0; l + 1 < c->nlev; ++l) set_nc(*c, l, src->L64[l].nc);  // what the source's setup kept
    if (!src->C0.empty()) {
      affine_links(*c, *src, mass);
      for (int l = 0; l + 1 < c->nlev; ++l) calibrate(*c, l);
    } else {
      for (int l = 0; l + 1 < c->nlev; ++l) {
        calibrate(*c, l);
        galerkin(*c, l);
      }
    }
    finish_setup(*c);
  } catch (...) {
    delete c;
    throw;
  }
  *out = reinterpret_cast<smg_handle>(c);
  return SMG_OK;
  API_END
}

int smg_apply_D(smg_handle h, const double* x, double* y, int32_t nrhs, int32_t dagger, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_nrhs(nrhs);
  if (!x || !y) throw Error(SMG_EINVAL, "null vector");
  auto& lv = c->L64[0];
  launch_wilson<double>(lv.U, (const z64*)x, (z64*)y, lv.lx, lv.lt, lv.diag, nrhs, dagger != 0, (hipStream_t)stream);
  return SMG_OK;
  API_END
}

int smg_apply_level(smg_handle h, int32_t level, const double* x, double* y, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  check_nrhs(nrhs);
  if (!x || !y) throw Error(SMG_EINVAL, "null vector");
  c->st = (hipStream_t)stream;
  ensure_level_work<double>(*c, nrhs);
  apply_op<double>(*c, c->L64[level], (const z64*)x, (z64*)y, nrhs, 0, 0.0, nullptr, nullptr);
  return SMG_OK;
  API_END
}

int smg_level_op(smg_handle h, int32_t level, int32_t mode, double coef, const double* x, double* y, double* xacc,
                 const double* aux, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  check_nrhs(nrhs);
  if (mode < 0 || mode > 3) throw Error(SMG_EINVAL, "mode must be 0, 1, 2 or 3");
  if (!x || !y || ((mode == 1 || mode == 3) && !xacc) || (mode == 2 && !aux)) throw Error(SMG_EINVAL, "null vector");
  if (!std::isfinite(coef)) throw Error(SMG_EINVAL, "coef must be finite");
  c->st = (hipStream_t)stream;
  ensure_level_work<double>(*c, nrhs);
  apply_op<double>(*c, c->L64[level], (const z64*)x, (z64*)y, nrhs, mode, coef, (z64*)xacc, (const z64*)aux);
  return SMG_OK;
  API_END
}

int smg_apply_level_f32(smg_handle h, int32_t level, const float* x, float* y, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  check_nrhs(nrhs);
  if (!x || !y) throw Error(SMG_EINVAL, "null vector");
  c->st = (hipStream_t)stream;
  ensure_f32(*c);
  ensure_level_work<float>(*c, nrhs);
  apply_op<float>(*c, c->L32[level], (const z32*)x, (z32*)y, nrhs, 0, 0.0, nullptr, nullptr);
  return SMG_OK;
  API_END
}

int smg_level_op_f32(smg_handle h, int32_t level, int32_t mode, double coef, const float* x, float* y, float* xacc,
                     const float* aux, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  check_nrhs(nrhs);
  if (mode < 0 || mode > 3) throw Error(SMG_EINVAL, "mode must be 0, 1, 2 or 3");
  if (!x || !y || ((mode == 1 || mode == 3) && !xacc) || (mode == 2 && !aux)) throw Error(SMG_EINVAL, "null vector");
  if (!std::isfinite(coef)) throw Error(SMG_EINVAL, "coef must be finite");
  c->st = (hipStream_t)stream;
  ensure_f32(*c);
  ensure_level_work<float>(*c, nrhs);
  apply_op<float>(*c, c->L32[level], (const z32*)x, (z32*)y, nrhs, mode, coef, (z32*)xacc, (const z32*)aux);
  return SMG_OK;
  API_END
}

int smg_apply_A(smg_handle h, const double* x, double* y, int32_t nrhs, void* stream) {
  return smg_apply_level(h, 0, x, y, nrhs, stream);
}

int smg_restrict(smg_handle h, int32_t level, const double* x, double* y, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  check_nrhs(nrhs);
  if (level >= c->nlev - 1) throw Error(SMG_EINVAL, "no coarser level");
  if (!x || !y) throw Error(SMG_EINVAL, "null vector");
  c->st = (hipStream_t)stream;
  restrict_to<double>(*c, c->L64[level], (const z64*)x, (z64*)y, nrhs);
  return SMG_OK;
  API_END
}

int smg_prolong(smg_handle h, int32_t level, const double* x, double* y, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  check_nrhs(nrhs);
  if (level >= c->nlev - 1) throw Error(SMG_EINVAL, "no coarser level");
  if (!x || !y) throw Error(SMG_EINVAL, "null vector");
  c->st = (hipStream_t)stream;
  ensure_level_work<double>(*c, nrhs);
  prolong_from<double>(*c, c->L64[level], (const z64*)x, (z64*)y, nrhs, 0);
  return SMG_OK;
  API_END
}

int smg_smooth(smg_handle h, int32_t level, const double* b, double* x, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  check_nrhs(nrhs);
  if (level >= c->nlev - 1) throw Error(SMG_EINVAL, "the coarsest level has no smoother");
  if (!x || !b) throw Error(SMG_EINVAL, "null vector");
  c->st = (hipStream_t)stream;
  ensure_level_work<double>(*c, nrhs);
  smooth<double>(*c, c->L64[level], (const z64*)b, (z64*)x, nrhs);
  return SMG_OK;
  API_END
}

int smg_vcycle(smg_handle h, const double* b, double* x, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_nrhs(nrhs);
  if (!x || !b) throw Error(SMG_EINVAL, "null vector");
  c->st = (hipStream_t)stream;
  ensure_level_work<double>(*c, nrhs);
  vcycle<double>(*c, 0, c->nlev - 1, (const z64*)b, (z64*)x, nrhs, c->prm.coarsest == SMG_COARSEST_CG);
  return SMG_OK;
  API_END
}

int smg_vcycle_noalloc(smg_handle h, const double* b, double* x, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_nrhs(nrhs);
  if (!x || !b) throw Error(SMG_EINVAL, "null vector");
  if (c->nlev < 2 || c->prm.coarsest != SMG_COARSEST_DIRECT)
    throw Error(SMG_EINVAL, "smg_vcycle_noalloc needs levels >= 2 and the dense coarsest inverse");
  const size_t need = carve_level_work(*c, nrhs, nullptr, nullptr);
  if (need > kScratchBytes)
    throw Error(SMG_EINVAL, "smg_vcycle_noalloc: " + std::to_string(nrhs) + " columns need " + std::to_string(need) +
                                " bytes of work space, more than the " + std::to_string(kScratchBytes) +
                                " bytes of the static scratch array");
  unsigned char* base = scratch_on_current_device();
  std::vector<Level<double>> work(c->nlev);
  carve_level_work(*c, nrhs, base, &work);
  // the handle's own work vectors are swapped out for the call and restored on every exit
  WorkLoan<double> loan(c->L64, work);
  c->st = (hipStream_t)stream;
  vcycle<double>(*c, 0, c->nlev - 1, (const z64*)b, (z64*)x, nrhs, false);
  return SMG_OK;
  API_END
}

int smg_vcycle_f32(smg_handle h, const float* b, float* x, int32_t nrhs, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_nrhs(nrhs);
  if (!x || !b) throw Error(SMG_EINVAL, "null vector");
  c->st = (hipStream_t)stream;
  ensure_f32(*c);
  ensure_level_work<float>(*c, nrhs);
  vcycle<float>(*c, 0, c->nlev - 1, (const z32*)b, (z32*)x, nrhs, c->prm.coarsest == SMG_COARSEST_CG);
  return SMG_OK;
  API_END
}

int smg_solve(smg_handle h, const double* rhs, double* x, int32_t nrhs, double tol, int32_t maxiter,
              int32_t precision, void* stream, smg_stats* stats) {
  API_BEGIN
  const auto t0 = std::chrono::steady_clock::now();
  Ctx* c = H(h);
  check_nrhs(nrhs);
  if (!rhs || !x) throw Error(SMG_EINVAL, "null vector");
  if (!(tol > 0) || maxiter < 1) throw Error(SMG_EINVAL, "tol must be > 0 and maxiter >= 1");
  if (precision != SMG_FP64 && precision != SMG_MIXED) throw Error(SMG_EINVAL, "bad precision");
  c->st = (hipStream_t)stream;
  const int64_t fa0 = c->fine_applies, vc0 = c->vcycles;
  const bool mg = c->nlev > 1;
  auto& lv = c->L64[0];
  const size_t n = lv.n;
  ColStats cs;
  int refinements = 1;
  reserve_solve(*c, nrhs, precision);
  if (precision == SMG_FP64) {
    pcg<double>(*c, 0, (const z64*)rhs, (z64*)x, nrhs, tol, maxiter, mg, c->f64, &cs, 1, 0,
                c->prm.stop_recursive == 0);
  } else {
    solve_mixed(c, rhs, x, nrhs, tol, maxiter, cs, refinements);
  }
  sync(*c);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(stats, nrhs, cs, refinements, c->fine_applies - fa0, c->vcycles - vc0, secs);
  for (int j = 0; j < nrhs; ++j)
    if (cs.status[j] != SMG_OK) return SMG_NOTCONV;
  return SMG_OK;
  API_END
}

int smg_cg(smg_handle h, const double* rhs, double* x, int32_t nrhs, double tol, int32_t maxiter, void* stream,
           smg_stats* stats) {
  API_BEGIN
  const auto t0 = std::chrono::steady_clock::now();
  Ctx* c = H(h);
  check_nrhs(nrhs);
  if (!rhs || !x) throw Error(SMG_EINVAL, "null vector");
  if (!(tol > 0) || maxiter < 1) throw Error(SMG_EINVAL, "tol must be > 0 and maxiter >= 1");
  c->st = (hipStream_t)stream;
  const int64_t fa0 = c->fine_applies;
  reserve_solve(*c, nrhs, SMG_FP64);
  ColStats cs;
  pcg<double>(*c, 0, (const z64*)rhs, (z64*)x, nrhs, tol, maxiter, false, c->f64, &cs, 1, 0,
              c->prm.stop_recursive == 0);
  sync(*c);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(stats, nrhs, cs, 1, c->fine_applies - fa0, 0, secs);
  for (int j = 0; j < nrhs; ++j)
    if (cs.status[j] != SMG_OK) return SMG_NOTCONV;
  return SMG_OK;
  API_END
}

int smg_level_info(smg_handle h, int32_t level, int32_t* lx, int32_t* lt, int32_t* dof) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  if (lx) *lx = c->L64[level].lx;
  if (lt) *lt = c->L64[level].lt;
  if (dof) *dof = c->L64[level].dof;
  return SMG_OK;
  API_END
}

int smg_get_prolongator(smg_handle h, int32_t level, int32_t smoothed, double* out, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  if (level >= c->nlev - 1) throw Error(SMG_EINVAL, "no prolongator below the coarsest level");
  if (!out) throw Error(SMG_EINVAL, "null output");
  auto& a = c->L64[level];
  const int hh = smoothed ? a.halo : 0;
  // the device keeps ldk column slots per aggregate; the first nc are in use (fewer
  // than ldk when the adaptive stop kept fewer vectors)
  const size_t nJ = (size_t)(a.lx / a.bx) * (a.lt / a.bt);
  const size_t nw = (size_t)(a.bx + 2 * hh) * (a.bt + 2 * hh) * a.dof;
  HIPCHECK(hipMemcpy2DAsync(out, a.nc * nw * sizeof(z64), smoothed ? a.P : a.Pt, a.ldk * nw * sizeof(z64),
                            a.nc * nw * sizeof(z64), nJ, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
  return SMG_OK;
  API_END
}

int smg_transfer_info(smg_handle h, int32_t level, int32_t* halo, double* sa_weight) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  if (level >= c->nlev - 1) throw Error(SMG_EINVAL, "no prolongator below the coarsest level");
  if (halo) *halo = c->L64[level].halo;
  if (sa_weight) *sa_weight = c->L64[level].sa_w;
  return SMG_OK;
  API_END
}

int smg_get_coarse_links(smg_handle h, int32_t level, double* out, void* stream) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  if (level < 1) throw Error(SMG_EINVAL, "level 0 has no coarse links");
  if (!out) throw Error(SMG_EINVAL, "null output");
  auto& a = c->L64[level];
  launch_links_export(a.L, (z64*)out, a.lx * a.lt, a.dof, (hipStream_t)stream);
  HIPCHECK(hipStreamSynchronize((hipStream_t)stream));
  return SMG_OK;
  API_END
}

int smg_get_setup_factors(smg_handle h, int32_t level, double* out, int32_t cap, int32_t* count) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  const auto& f = c->factors[level];
  if (count) *count = (int32_t)f.size();
  if (out)
    for (int k = 0; k < std::min<int>(cap, (int)f.size()); ++k) out[k] = f[k];
  return SMG_OK;
  API_END
}

int smg_get_smoother_coefs(smg_handle h, int32_t level, double* out) {
  API_BEGIN
  Ctx* c = H(h);
  check_level(c, level);
  if (!out) throw Error(SMG_EINVAL, "null output");
  auto& a = c->L64[level];
  for (size_t k = 0; k < a.coefs.size(); ++k) out[k] = a.coefs[k];
  return SMG_OK;
  API_END
}

int smg_set_allocator(smg_alloc_fn alloc, smg_release_fn release, void* ctx) {
  API_BEGIN
  if (!alloc != !release) throw Error(SMG_EINVAL, "give both alloc and release, or neither");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc.alloc = alloc;
  g_alloc.release = release;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return SMG_OK;
  API_END
}

int smg_set_progress(smg_progress_fn fn, void* ctx) {
  API_BEGIN
  std::lock_guard<std::mutex> lk(g_progress_mu);
  g_progress = fn;
  g_progress_ctx = ctx;
  return SMG_OK;
  API_END
}

int smg_query_bytes(const smg_params* params, int32_t nrhs, int32_t precision, size_t* setup_bytes,
                    size_t* solve_bytes, size_t* batch_bytes) {
  API_BEGIN
  if (!params) throw Error(SMG_EINVAL, "null params");
  check_nrhs(nrhs);
  if (precision != SMG_FP64 && precision != SMG_MIXED) throw Error(SMG_EINVAL, "bad precision");
  if (batch_bytes && nrhs > 256) throw Error(SMG_EINVAL, "a batch has at most 256 slots");
  // the allocation plan of the real calls, run on dry contexts (no device call)
  auto planned = [&]() {
    std::unique_ptr<Ctx> c(create(nullptr, params, nullptr, nullptr, true));
    reserve_setup(*c);
    return c;
  };
  auto c0 = planned();
  const size_t setup = c0->pool.bytes;
  if (setup_bytes) *setup_bytes = setup;
  if (solve_bytes) {
    reserve_solve(*c0, nrhs, precision);
    *solve_bytes = c0->pool.bytes - setup;
  }
  if (batch_bytes) {
    auto c1 = planned();
    Batch B;
    B.pool.dry = true;
    B.pool.gran = 256;  // the arena's granularity (smg_batch_create)
    B.c = c1.get();
    B.cap = nrhs;
    B.prec = precision;
    B.n = c1->L64[0].n;
    reserve_batch_handle(*c1, nrhs, precision);
    batch_alloc(B);
    *batch_bytes = B.pool.bytes + (c1->pool.bytes - setup);
  }
  return SMG_OK;
  API_END
}

int smg_memory_bytes(smg_handle h, size_t* bytes) {
  API_BEGIN
  Ctx* c = H(h);
  if (!bytes) throw Error(SMG_EINVAL, "null output");
  *bytes = c->pool.bytes;
  return SMG_OK;
  API_END
}

int smg_group_create(const smg_handle* hs, int32_t nsys, void* stream, smg_group* out) {
  API_BEGIN
  if (!hs || !out) throw Error(SMG_EINVAL, "null handles or output");
  if (nsys < 1 || nsys > 4096) throw Error(SMG_EINVAL, "nsys must be in [1, 4096]");
  std::unique_ptr<Group> g(new Group());
  for (int j = 0; j < nsys; ++j) g->cs.push_back(H(hs[j]));
  const Ctx& c0 = *g->cs[0];
  if (c0.nlev < 2) throw Error(SMG_EINVAL, "a grouped solve needs levels >= 2");
  if (c0.prm.coarsest != SMG_COARSEST_DIRECT) throw Error(SMG_EINVAL, "a grouped solve needs the dense coarsest inverse");
  if (c0.prm.smoother_storage != SMG_STORE_F32) throw Error(SMG_EINVAL, "a grouped solve needs smoother_storage F32");
  if (c0.prm.smoother_steps < 2) throw Error(SMG_EINVAL, "a grouped solve needs smoother_steps >= 2");
  if (c0.L64[c0.nlev - 1].n > 4096) throw Error(SMG_EINVAL, "a grouped solve needs a coarsest level of <= 4096 variables");
  for (int l = 1; l + 1 < c0.nlev; ++l)
    if (c0.L64[l].dof < 4 || c0.L64[l].dof > 16) throw Error(SMG_EINVAL, "a grouped solve needs 4 <= nc <= 16");
  group_fill(*g, (hipStream_t)stream);
  *out = reinterpret_cast<smg_group>(g.release());
  return SMG_OK;
  API_END
}

int smg_group_solve(smg_group gh, const double* rhs, double* x, double tol, int32_t maxiter, void* stream,
                    smg_stats* stats) {
  API_BEGIN
  const auto t0 = std::chrono::steady_clock::now();
  Group& g = *GH(gh);
  if (!rhs || !x) throw Error(SMG_EINVAL, "null vector");
  if (!(tol > 0) || maxiter < 1) throw Error(SMG_EINVAL, "tol must be > 0 and maxiter >= 1");
  const int G = (int)g.cs.size();
  hipStream_t st = (hipStream_t)stream;
  bool stale = false;
  for (int j = 0; j < G; ++j) stale = stale || g.cs[j]->gen != g.gens[j] || !g.cs[j]->f32_ready;
  if (stale) group_fill(g, st);
  Ctx* c = g.cs[0];
  c->st = st;
  const int64_t fa0 = c->fine_applies, vc0 = c->vcycles;
  reserve_solve(*c, G, SMG_MIXED);
  struct Bind {  // the context runs ungrouped again on every exit path
    Ctx* c;
    ~Bind() { c->grp = nullptr; }
  } bind{c};
  c->grp = &g.tab;
  ColStats cs;
  int refinements = 0;
  solve_mixed(c, rhs, x, G, tol, maxiter, cs, refinements);
  sync(*c);
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  fill_stats(stats, G, cs, refinements, c->fine_applies - fa0, c->vcycles - vc0, secs);
  for (int j = 0; j < G; ++j)
    if (cs.status[j] != SMG_OK) return SMG_NOTCONV;
  return SMG_OK;
  API_END
}

int smg_group_level_op_f32(smg_group gh, int32_t level, int32_t mode, const float* x, float* y, const float* aux,
                           void* stream) {
  API_BEGIN
  Group& g = *GH(gh);
  if (mode != 0 && mode != 2) throw Error(SMG_EINVAL, "mode must be 0 or 2");
  if (!x || !y || (mode == 2 && !aux)) throw Error(SMG_EINVAL, "null vector");
  const int G = (int)g.cs.size();
  Ctx* c = g.cs[0];
  check_level(c, level);
  hipStream_t st = (hipStream_t)stream;
  bool stale = false;
  for (int j = 0; j < G; ++j) stale = stale || g.cs[j]->gen != g.gens[j] || !g.cs[j]->f32_ready;
  if (stale) group_fill(g, st);
  c->st = st;
  ensure_level_work<float>(*c, G);
  struct Bind {  // the context runs ungrouped again on every exit path
    Ctx* c;
    ~Bind() { c->grp = nullptr; }
  } bind{c};
  c->grp = &g.tab;
  apply_op<float>(*c, c->L32[level], (const z32*)x, (z32*)y, G, mode, 0.0, nullptr, (const z32*)aux);
  return SMG_OK;
  API_END
}

void smg_group_destroy(smg_group g) {
  if (!g) return;
  delete reinterpret_cast<Group*>(g);
}

int smg_batch_create(smg_handle h, int32_t max_rhs, double tol, int32_t maxiter, int32_t precision, void* stream,
                     smg_batch* out) {
  API_BEGIN
  Ctx* c = H(h);
  if (!out) throw Error(SMG_EINVAL, "null output");
  if (max_rhs < 1 || max_rhs > 256) throw Error(SMG_EINVAL, "max_rhs must be in [1, 256]");
  if (!(tol > 0) || maxiter < 1) throw Error(SMG_EINVAL, "tol must be > 0 and maxiter >= 1");
  if (precision != SMG_FP64 && precision != SMG_MIXED) throw Error(SMG_EINVAL, "bad precision");
  hipStream_t st = (hipStream_t)stream;
  c->st = st;
  Batch* B = new Batch();
  try {
    B->c = c;
    B->cap = max_rhs;
    B->tol = tol;
    B->maxiter = maxiter;
    B->prec = precision;
    B->n = c->L64[0].n;
    const size_t e = (size_t)max_rhs * B->n;
    B->pool.stream = &B->st0;
    B->st0 = st;
    B->note(st);
    reserve_batch_handle(*c, max_rhs, precision);
    {  // every array of the batch in one block, sized by the same plan on a dry pool
      Batch plan;
      plan.pool.dry = true;
      plan.pool.gran = 256;
      plan.c = c;
      plan.cap = max_rhs;
      plan.prec = precision;
      plan.n = B->n;
      batch_alloc(plan);
      B->pool.open_arena(plan.pool.bytes);
    }
    batch_alloc(*B);
    if (precision == SMG_MIXED) ensure_f32(*c);
    B->h = static_cast<double*>(g_pinned.get(sizeof(double) * 2 * max_rhs));
    B->hi_ = static_cast<int*>(g_pinned.get(sizeof(int) * max_rhs));
    // off by default: each (batch, slot count) pays a capture, and replays do not
    // shorten the iteration where the device front end bounds it (smg_batch_use_graphs)
    B->use_graphs = false;
    B->graphs.assign(max_rhs + 1, nullptr);
    B->graph_gen = c->gen;
    B->used.assign(max_rhs, 0);
    B->act.assign(max_rhs, 0);
    B->its.assign(max_rhs, 0);
    B->stat.assign(max_rhs, SMG_OK);
    B->bb.assign(max_rhs, 0.0);
    B->rel.assign(max_rhs, 0.0);
    zero(B->S.bad, sizeof(int) * max_rhs, st);
    zero(B->x, e * sizeof(z64), st);
    zero(B->p, e * sizeof(z64), st);
    zero(B->r, e * sizeof(z64), st);
    zero(B->z, e * sizeof(z64), st);
    zero(B->S.rz, sizeof(double) * 2 * max_rhs, st);
    batch_upload_active(*B, st);
  } catch (...) {
    delete B;
    throw;
  }
  *out = reinterpret_cast<smg_batch>(B);
  return SMG_OK;
  API_END
}

int smg_batch_admit(smg_batch b, const double* rhs, int32_t* slot, void* stream) {
  API_BEGIN
  Batch* B = BH(b);
  if (!rhs || !slot) throw Error(SMG_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  B->note(st);
  int s = -1;
  for (int j = 0; j < B->cap; ++j)
    if (!B->used[j]) {
      s = j;
      break;
    }
  if (s < 0) throw Error(SMG_EBUSY, "no free slot in the batch");
  const size_t n = B->n, off = (size_t)s * n;
  HIPCHECK(hipMemcpyAsync(B->b + off, rhs, n * sizeof(z64), hipMemcpyDeviceToDevice, st));
  HIPCHECK(hipMemcpyAsync(B->r + off, rhs, n * sizeof(z64), hipMemcpyDeviceToDevice, st));
  zero(B->x + off, n * sizeof(z64), st);
  zero(B->p + off, n * sizeof(z64), st);
  zero(B->S.rz + 2 * s, sizeof(double) * 2, st);
  zero(B->S.bad + s, sizeof(int), st);
  launch_dot<double>(B->b + off, B->b + off, n, 1, B->red, B->S.bb + 2 * s, st);
  HIPCHECK(hipMemcpyAsync(B->h, B->S.bb + 2 * s, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  const double bb = B->h[0];
  if (!std::isfinite(bb)) {  // leave the free slot finite for the shared V-cycle
    batch_clear(*B, s, st);
    HIPCHECK(hipStreamSynchronize(st));
    throw Error(SMG_EBREAKDOWN, "right-hand side contains NaN/Inf");
  }
  B->used[s] = 1;
  B->its[s] = 0;
  B->rel[s] = 0.0;
  B->bb[s] = bb;
  if (!(bb > 0)) {  // zero right-hand side: x = 0, done
    B->act[s] = 0;
    B->stat[s] = SMG_OK;
    zero(B->r + off, n * sizeof(z64), st);
  } else {  // joins at the next step with beta = 0 (<r,z>_old = 0)
    B->act[s] = 1;
    B->stat[s] = SMG_NOTCONV;
  }
  batch_upload_active(*B, st);
  *slot = s;
  return SMG_OK;
  API_END
}

int smg_batch_step(smg_batch b, int32_t iters, void* stream) {
  API_BEGIN
  Batch* B = BH(b);
  if (iters < 1) throw Error(SMG_EINVAL, "iters must be >= 1");
  B->note((hipStream_t)stream);
  batch_step(*B, iters, (hipStream_t)stream);
  return SMG_OK;
  API_END
}

int smg_batch_poll(smg_batch b, uint8_t* done, smg_stats* stats) {
  API_BEGIN
  Batch* B = BH(b);
  for (int j = 0; j < B->cap; ++j) {
    if (done) done[j] = (B->used[j] && !B->act[j]) ? 1 : 0;
    if (stats) {
      stats[j].status = B->used[j] ? B->stat[j] : SMG_OK;
      stats[j].iterations = B->its[j];
      stats[j].refinements = 1;
      stats[j].vcycles = B->its[j];
      stats[j].fine_applies = 0;
      stats[j].true_relres = B->rel[j];
      stats[j].seconds = 0;
    }
  }
  return SMG_OK;
  API_END
}

int smg_batch_active(smg_batch b, int32_t* used, int32_t* running) {
  API_BEGIN
  Batch* B = BH(b);
  int u = 0, a = 0;
  for (int j = 0; j < B->cap; ++j) {
    u += B->used[j];
    a += B->act[j];
  }
  if (used) *used = u;
  if (running) *running = a;
  return SMG_OK;
  API_END
}

int smg_batch_harvest(smg_batch b, int32_t slot, double* x, void* stream) {
  API_BEGIN
  Batch* B = BH(b);
  if (slot < 0 || slot >= B->cap || !B->used[slot]) throw Error(SMG_EINVAL, "slot is not in use");
  if (B->act[slot]) throw Error(SMG_EINVAL, "slot is still running");
  hipStream_t st = (hipStream_t)stream;
  B->note(st);
  if (x)
    HIPCHECK(hipMemcpyAsync(x, B->x + (size_t)slot * B->n, B->n * sizeof(z64), hipMemcpyDeviceToDevice, st));
  batch_clear(*B, slot, st);
  HIPCHECK(hipStreamSynchronize(st));
  B->used[slot] = 0;
  return SMG_OK;
  API_END
}

int smg_batch_cancel(smg_batch b, int32_t slot, void* stream) {
  API_BEGIN
  Batch* B = BH(b);
  if (slot < 0 || slot >= B->cap || !B->used[slot]) throw Error(SMG_EINVAL, "slot is not in use");
  B->used[slot] = 0;
  B->act[slot] = 0;
  B->note((hipStream_t)stream);
  batch_clear(*B, slot, (hipStream_t)stream);
  batch_upload_active(*B, (hipStream_t)stream);
  return SMG_OK;
  API_END
}

int smg_batch_use_graphs(smg_batch b, int32_t enable) {
  API_BEGIN
  Batch* B = BH(b);
  Ctx& c = *B->c;
  const bool can = c.nlev < 2 || c.prm.coarsest == SMG_COARSEST_DIRECT;
  if (enable && !can) throw Error(SMG_EINVAL, "graphs need a direct coarsest solve");
  B->drop_graphs();
  if (enable && !B->gs) {  // the batch's own stream, made when graphs are first wanted
    HIPCHECK(hipStreamCreateWithFlags(&B->gs, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&B->ev, hipEventDisableTiming));
  }
  B->use_graphs = enable != 0;
  return SMG_OK;
  API_END
}

int smg_batch_memory_bytes(smg_batch b, size_t* bytes) {
  API_BEGIN
  Batch* B = BH(b);
  if (!bytes) throw Error(SMG_EINVAL, "null output");
  *bytes = B->pool.bytes;
  return SMG_OK;
  API_END
}

void smg_batch_destroy(smg_batch b) {
  if (!b) return;
  Batch* B = reinterpret_cast<Batch*>(b);
  // only the batch's own calls touched its memory: once their streams are idle the
  // arena can go back to the allocator without waiting for the rest of the device
  for (hipStream_t s : B->seen) (void)hipStreamSynchronize(s);
  if (B->gs) (void)hipStreamSynchronize(B->gs);
  B->pool.owner_synced = true;
  delete B;
}

void smg_destroy(smg_handle h) {
  if (!h) return;
  Ctx* c = reinterpret_cast<Ctx*>(h);
  (void)hipStreamSynchronize(c->st);
  delete c;
}

const char* smg_strerror(int code) {
  switch (code) {
    case SMG_OK: return "success";
    case SMG_NOTCONV: return "not converged within maxiter";
    case SMG_EINVAL: return "invalid argument";
    case SMG_ESHAPE: return "lattice extents not divisible by the block extents";
    case SMG_ENOMEM: return "device out of memory";
    case SMG_EDEVICE: return "HIP runtime error";
    case SMG_EBREAKDOWN: return "numerical breakdown (NaN/Inf or loss of positive definiteness)";
    case SMG_ESETUP: return "setup failed (degenerate aggregate or coarsest factorisation)";
    case SMG_EBUSY: return "no free slot in the batch";
    default: return "unknown error code";
  }
}

const char* smg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
