// Internal definitions shared by the HIP kernels and the host driver of libsmg.
//
// Storage conventions (all device arrays are plain interleaved complex numbers):
//   fine vector batch     [nrhs][t][x][spin]        spin in {0,1}
//   level-l vector batch  [nrhs][t][x][dof]         dof = nv of the coarsening above
//   fine links            [mu][t][x]                fermion BC sign folded into mu=1, t=lt-1
//   prolongator           [J][k][i]                 J coarse site, k vector, i window variable
//   coarse links (device) [D][col][K][row]          D = (dt+1)*3 + (dx+1); "site-major" so that
//                                                   threads (K,row) read consecutive words
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>

namespace smg {

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
  R re, im;
};

template <typename R>
__host__ __device__ inline cpx<R> mk(R a, R b) { cpx<R> z; z.re = a; z.im = b; return z; }
template <typename R>
__host__ __device__ inline cpx<R> operator+(cpx<R> a, cpx<R> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename R>
__host__ __device__ inline cpx<R> operator-(cpx<R> a, cpx<R> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename R>
__host__ __device__ inline cpx<R> operator*(cpx<R> a, cpx<R> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename R>
__host__ __device__ inline cpx<R> operator*(R s, cpx<R> a) { return mk(s * a.re, s * a.im); }
template <typename R>
__host__ __device__ inline cpx<R> cj(cpx<R> a) { return mk(a.re, -a.im); }
// conj(a) * b
template <typename R>
__host__ __device__ inline cpx<R> cmulc(cpx<R> a, cpx<R> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
// i * a
template <typename R>
__host__ __device__ inline cpx<R> imul(cpx<R> a) { return mk(-a.im, a.re); }
template <typename R>
__host__ __device__ inline void fma_acc(cpx<R>& acc, cpx<R> a, cpx<R> b) {
  acc.re += a.re * b.re - a.im * b.im;
  acc.im += a.re * b.im + a.im * b.re;
}
// acc += a b with explicit fused multiply-adds in a fixed order: the rounding does not
// depend on how the compiler contracts the surrounding code (kernels instantiated
// for different numbers of right-hand sides give the same bits).
template <typename R>
__host__ __device__ inline void fma_acc_x(cpx<R>& acc, cpx<R> a, cpx<R> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
template <typename R>
__host__ __device__ inline void fma_acc_conj(cpx<R>& acc, cpx<R> a, cpx<R> b) {  // acc += conj(a) b
  acc.re += a.re * b.re + a.im * b.im;
  acc.im += a.re * b.im - a.im * b.re;
}
template <typename Ro, typename Ri>
__host__ __device__ inline cpx<Ro> cvt(cpx<Ri> a) { return mk((Ro)a.re, (Ro)a.im); }

using z64 = cpx<double>;
using z32 = cpx<float>;

// 4-byte complex storage for the fine-level smoother iterates of the FP32 V-cycle
// (BF16 or FP16 halves; all arithmetic stays FP32).
struct alignas(4) bfc { __bf16 re, im; };
struct alignas(4) hfc { _Float16 re, im; };

// Arithmetic value of a stored element (exact: BF16 and FP16 widen to FP32 exactly).
template <typename R>
__device__ inline cpx<R> widen(cpx<R> t) { return t; }
__device__ inline z32 widen(bfc t) { return mk((float)t.re, (float)t.im); }
__device__ inline z32 widen(hfc t) { return mk((float)t.re, (float)t.im); }
template <typename T>
__device__ inline auto ldv(const T* p, size_t i) { return widen(p[i]); }
template <typename R>
__device__ inline void stv(cpx<R>* p, size_t i, cpx<R> v) { p[i] = v; }
__device__ inline void stv(bfc* p, size_t i, z32 v) {
  bfc t;
  t.re = (__bf16)v.re;
  t.im = (__bf16)v.im;
  p[i] = t;
}
__device__ inline void stv(hfc* p, size_t i, z32 v) {
  hfc t;
  t.re = (_Float16)v.re;
  t.im = (_Float16)v.im;
  p[i] = t;
}

// Error raised inside the library and turned into a return code at the C boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPCHECK(call) ::smg::hip_check((call), #call, __FILE__, __LINE__)

constexpr int kThreads = 256;

// Epilogues of the operator applies (y = A x computed in registers, c and c2 real):
//   0: y = A x
//   1: xacc += c x ; y = x - c A x              (one frozen MR step)
//   2: y = aux - A x                            (residual)
//   3: xacc  = c x ; y = x - c A x              (first MR step, from a zero iterate)
//   4: xacc += c x + c2 (x - c A x)             (the last two MR steps; y is not written)
//   5: xacc  = c x + c2 (x - c A x)             (both steps of a two-step smoother from zero)
template <int N>
struct ModeC {
  static constexpr int v = N;
};
template <typename F>
void with_mode(int mode, F&& f) {
  switch (mode) {
    case 0: f(ModeC<0>{}); break;
    case 1: f(ModeC<1>{}); break;
    case 2: f(ModeC<2>{}); break;
    case 3: f(ModeC<3>{}); break;
    case 4: f(ModeC<4>{}); break;
    case 5: f(ModeC<5>{}); break;
    default: throw Error(-1, "unknown operator epilogue");
  }
}

inline unsigned grid_for(size_t n, int threads = kThreads, size_t cap = 1u << 20) {
  size_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Deterministic reductions use a partial count that depends only on the vector
// length, never on the batch size or on which columns are active.
inline int red_blocks(size_t n) {
  size_t b = (n + 4 * kThreads - 1) / (4 * kThreads);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All are asynchronous on `st`.
// ---------------------------------------------------------------------------

// Fine Wilson operator, links U [2][V] with the fermion BC sign already folded in.
template <typename R>
void launch_wilson(const cpx<R>* U, const cpx<R>* x, cpx<R>* y, int lx, int lt, double diag, int nrhs,
                   bool dagger, hipStream_t st);

// Per-column operators of a grouped solve: several independent systems of one shape
// advanced together, system j in column j of every launch.  Column j reads op[j] (its
// links, prolongator or coarsest inverse) and s[j] (their power-of-two scale, or the
// fine diagonal 2 + m) in place of the launch's own, and c[j], c2[j] (its smoother
// coefficients) where non-null.  op = nullptr: an ordinary launch.  Grouped launches
// take one column per workgroup, the kernels a single system uses, so column j's
// arithmetic is that of system j solved alone.
struct Grp {
  const void* const* op = nullptr;
  const double* s = nullptr;
  const double* c = nullptr;
  const double* c2 = nullptr;
};

// Fine normal operator with an epilogue.  mode:
//   0: y = A x
//   1: smoother step   xacc += c * x ;  y = x - c * A x
//   2: residual        y = b - A x           (b = aux)
// A x = D^H (D x); `tmp` holds D x ([nrhs][V][2]).
template <typename R>
void launch_normal(const cpx<R>* U, const cpx<R>* x, cpx<R>* y, cpx<R>* tmp, int lx, int lt, double diag,
                   int nrhs, int mode, double c, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st, double c2 = 0,
                   const Grp& g = Grp{});

// beta of the fused CG step formed inside the kernel (part == nullptr: read beta[rhs]).
// Every workgroup sums the nb partials of <r, z> per column in the order of the
// separate second pass; beta = <r,z> / rz_old[rhs] for an active column with a nonzero
// rz_old (else 0), beta = 0 for every column when rz_old is null (the first step).
// Workgroup 0 writes <r, z> to rz_new (rz_old where the column is not active).
constexpr int kBetaFoldMaxBlocks = 4 * kThreads;  // largest nb of a folded beta
struct BetaFold {
  const double* part = nullptr;
  int nb = 0;
  const double* rz_old = nullptr;
  double* rz_new = nullptr;
  const int* active = nullptr;
};

// The outer CG step on the fine level in one fused kernel: p = z + beta p_old (p = z
// where beta = 0), q = A p, and per workgroup <p, q> into partial[rhs][block] for
// cg_step_blocks(lx, lt) blocks (0: no fused tile fits, use the separate kernels).
template <typename R>
int cg_step_blocks(int lx, int lt);
template <typename R>
void launch_cg_step(const cpx<R>* U, const cpx<R>* z, const cpx<R>* p_old, cpx<R>* p, cpx<R>* q, int lx, int lt,
                    double diag, int nrhs, const double* beta, double* partial, hipStream_t st,
                    const BetaFold& bf = BetaFold{}, const Grp& g = Grp{});
// The last fine apply of a V-cycle with the CG dot folded in: z += c v + c2 (v - c A v)
// (the last two smoother steps) and per workgroup <r, z> into partial[rhs][block]
// (cg_step_blocks(lx, lt) blocks).
template <typename R>
void launch_vcycle_end(const cpx<R>* U, const cpx<R>* v, cpx<R>* z, const cpx<R>* r, int lx, int lt, double diag,
                       int nrhs, double c, double c2, double* partial, hipStream_t st, const Grp& g = Grp{});
// FP32 fine A with x and y stored as TI / TO (z32, bfc or hfc); fused kernel only
// (lx and lt multiples of 16).
template <typename TI, typename TO>
void launch_normal_lp(const z32* U, const TI* x, TO* y, int lx, int lt, double diag, int nrhs, int mode, double c,
                      z32* xacc, const z32* aux, hipStream_t st, double c2 = 0);
bool normal_lp_fits(int lx, int lt);
// FP32 P^H x with P stored as TP (z32, or hfc scaled by 1 / ps) and x stored as TI
// (z32, bfc or hfc).
template <typename TP, typename TI>
void launch_restrict_s(const TP* P, float ps, const TI* x, z32* y, int lx, int lt, int dof, int bx, int bt, int h,
                       int nc, int ldk, int nrhs, hipStream_t st, const Grp& g = Grp{});
// x += a y for y stored as TI.
template <typename TI>
void launch_axpy_const_lp(z32* y, const TI* x, double a, size_t n, int nrhs, hipStream_t st);
// Zero fill by a kernel (bytes a multiple of 8).
void launch_zero(void* p, size_t bytes, hipStream_t st);

// Coarse 9-point operator on level with extents (cx, ct), nc dof; links [9][nc][K][nc].
template <typename R>
void launch_coarse(const cpx<R>* L, const cpx<R>* x, cpx<R>* y, int cx, int ct, int nc, int nrhs, int mode,
                   double c, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st, double c2 = 0, const Grp& g = Grp{});
// The same with the links stored in FP16 scaled by 1 / lscale (a power of two).
void launch_coarse_h16(const hfc* L, float lscale, const z32* x, z32* y, int cx, int ct, int nc, int nrhs, int mode,
                       double c, z32* xacc, const z32* aux, hipStream_t st, double c2 = 0, const Grp& g = Grp{});
// Matrix-core (MFMA FP32) coarse apply for 1 <= nc <= 16, any number of right-hand sides.
void launch_coarse_mfma(const z32* L, const z32* x, z32* y, int cx, int ct, int nc, int nrhs, int mode, double c,
                        z32* xacc, const z32* aux, hipStream_t st, double c2 = 0);
// The same reading links stored in FP16 scaled by 1 / lscale (FP32 arithmetic).
void launch_coarse_mfma_h16(const hfc* L, float lscale, const z32* x, z32* y, int cx, int ct, int nc, int nrhs,
                            int mode, double c, z32* xacc, const z32* aux, hipStream_t st, double c2 = 0);
// FP64 multi-RHS coarse operator on the matrix cores (1 <= nc <= 16).
void launch_coarse_mfma64(const z64* L, const z64* x, z64* y, int cx, int ct, int nc, int nrhs, int mode, double c,
                          z64* xacc, const z64* aux, hipStream_t st, double c2 = 0);

// Transfer between level (lx, lt, dof) and its aggregates of (bx, bt) sites.
// P is [J][ldk][nw] (ldk >= nc vectors stored per aggregate) over windows of
// (bx + 2h) x (bt + 2h) sites: h = 0 tentative, h = 1 smoothed prolongator.
template <typename R>
void launch_restrict(const cpx<R>* P, const cpx<R>* x, cpx<R>* y, int lx, int lt, int dof, int bx, int bt, int h,
                     int nc, int ldk, int nrhs, hipStream_t st);
// FP64 restriction of many right-hand sides on the matrix cores (1 <= nc <= 16).
void launch_restrict_mfma64(const z64* P, const z64* x, z64* y, int lx, int lt, int dof, int bx, int bt, int h,
                            int nc, int ldk, int nrhs, hipStream_t st);
// mode 0: y = P e ; mode 1: y += P e.  wbuf holds nrhs * nK * nw scratch values.
// mfma (FP64 only, nc <= 16): the window phase on the matrix cores.
template <typename R>
void launch_prolong(const cpx<R>* P, const cpx<R>* e, cpx<R>* y, cpx<R>* wbuf, int lx, int lt, int dof, int bx,
                    int bt, int h, int nc, int ldk, int nrhs, int mode, hipStream_t st, bool mfma = false,
                    const Grp& g = Grp{});

// FP32 prolongation with P stored in FP16 scaled by 1 / ps.
void launch_prolong_h16(const hfc* P, float ps, const z32* e, z32* y, z32* wbuf, int lx, int lt, int dof, int bx,
                        int bt, int h, int nc, int ldk, int nrhs, int mode, hipStream_t st, const Grp& g = Grp{});

// Block Gram-Schmidt of candidate `v` as vector k of every aggregate (FP64).
void launch_gs_append(double* P, const z64* v, int lx, int lt, int dof, int bx, int bt, int k, int ldk, int m,
                      int* fail, hipStream_t st);

// Galerkin helpers: X = sum over aggregates J of colour (cxc, ctc) of P[J][k] (zero elsewhere).
void launch_color_scatter(const z64* P, z64* X, int lx, int lt, int dof, int bx, int bt, int h, int k, int ldk,
                          int cxc, int ctc, hipStream_t st);
// links[D(K)][k][K][:] = P_K^H (Y restricted to K's window), D(K) the offset of the colour's aggregate.
void launch_color_project(const z64* P, const z64* Y, z64* L, int lx, int lt, int dof, int bx, int bt, int h,
                          int nc, int ldk, int k, int cxc, int ctc, hipStream_t st);
// Smoothed aggregation: P[J][k] = (X - w Y) on the windows of colour (cxc, ctc).
void launch_sa_extract(const z64* X, const z64* Y, z64* P, int lx, int lt, int dof, int bx, int bt, int k, int ldk,
                       int cxc, int ctc, double w, hipStream_t st);
int colors_along(int extent);

// Dense coarsest operator and its inverse (FP64).
void launch_coarse_to_dense(const z64* L, z64* M, int cx, int ct, int nc, hipStream_t st);
void launch_gj_step(z64* M, int n, int k, z64* colk, double* piv, int* fail, hipStream_t st);
// Y = M X, M dense row-major n x n in precision RM, X and Y [nrhs][n].
template <typename RM, typename R>
void launch_dense_apply(const cpx<RM>* M, const cpx<R>* x, cpx<R>* y, int n, int nrhs, hipStream_t st,
                        const Grp& g = Grp{});
// FP32 y = M x with M stored in FP16 scaled by 1 / mscale (a power of two).
void launch_dense_apply_h16(const hfc* M, double mscale, const z32* x, z32* y, int n, int nrhs, hipStream_t st,
                            const Grp& g = Grp{});
// Per-block maxima of max(|re|, |im|) over n values into part[0 .. blocks).
void launch_absmax_partial(const z64* a, size_t n, double* part, int blocks, hipStream_t st);
// out = FP16(in * inv_scale).
void launch_convert_h16(const z64* in, hfc* out, size_t n, double inv_scale, hipStream_t st);

// Level-1 BLAS (batched over nrhs columns of length n).
// Scratch of the reductions: per column `nb` block partials.
struct Red {
  double* partial = nullptr;
};
template <typename R>
void launch_dot(const cpx<R>* a, const cpx<R>* b, size_t n, int nrhs, Red red, double* out, hipStream_t st,
                double* out_host = nullptr);  // out (and out_host when given)[2*rhs] = <a,b>
// <p, q> per column, then alpha = <r,z> / <p,q> (0 for inactive columns, breakdown flagged in bad and,
// when bad_host is given, in that host-visible mirror too).
template <typename R>
void launch_dot_alpha(const cpx<R>* p, const cpx<R>* q, size_t n, int nrhs, Red red, const double* rz,
                      double* alpha, const int* active, int* bad, hipStream_t st, int* bad_host = nullptr);
// <r, z>_new per column, then beta = <r,z>_new / <r,z>_old and <r,z>_old <- <r,z>_new (active columns).
template <typename R>
void launch_dot_beta(const cpx<R>* r, const cpx<R>* z, size_t n, int nrhs, Red red, double* rz, double* beta,
                     const int* active, hipStream_t st);
// beta and <r, r> of an unpreconditioned CG from the |r|^2 partial sums that the last
// launch_axpy_update of the same length left in red.
void launch_beta_partials(size_t n, int nrhs, Red red, double* rz, double* beta, const int* active,
                          hipStream_t st);
// x += alpha p, r -= alpha q and |r|^2 per column into rr (and rr_host when given).
template <typename R>
void launch_axpy_update(cpx<R>* x, cpx<R>* r, const cpx<R>* p, const cpx<R>* q, const double* alpha, size_t n,
                        int nrhs, Red red, double* rr, hipStream_t st,
                        double* rr_host = nullptr);
// x += alpha p, r -= alpha q (FP32), alpha formed in every block from the partial sums
// of <p, A p> of the fused CG step (pnb per column) and <r, z> in rz; the per-block
// partial sums of |r|^2 go to rr_part_host[rhs][red_blocks(n)] (host-visible memory,
// added up by the host after a synchronisation: no second pass)
void launch_axpy_update_fold(z32* x, z32* r, const z32* p, const z32* q, const double* ppart, int pnb,
                             const double* rz, double* alpha, const int* active, int* bad, int* bad_host, size_t n,
                             int nrhs, double* rr_part_host, hipStream_t st);
template <typename R>
void launch_xpay(const cpx<R>* z, cpx<R>* p, const double* beta, size_t n, int nrhs, hipStream_t st);
template <typename R>
void launch_axpy_const(cpx<R>* y, const cpx<R>* x, double a, size_t n, int nrhs, hipStream_t st);
template <typename R>
void launch_sub(const cpx<R>* a, const cpx<R>* b, cpx<R>* y, size_t n, int nrhs, hipStream_t st);  // y = a-b
template <typename R>
void launch_scale_cols(cpx<R>* x, const double* s, size_t n, int nrhs, hipStream_t st);  // x *= s[rhs]
template <typename R>
void launch_scale_const(cpx<R>* x, double a, size_t n, int nrhs, hipStream_t st);  // x *= a
template <typename Ro, typename Ri>
void launch_convert(const cpx<Ri>* in, cpx<Ro>* out, size_t n, hipStream_t st);
// Defect-correction scales from |r|^2 per column: down = 1/|r| and up = |r| where on[rhs]
// (host-visible memory, set by the host) is nonzero, else 0 and 0.
void launch_dc_scales(const double* rr, const int* on, double* down, double* up, int nrhs, hipStream_t st);
// out32 = in64 * s[rhs]   (defect-correction right-hand side)
void launch_scale_down(const z64* in, z32* out, const double* s, size_t n, int nrhs, hipStream_t st);
// b = s in (FP32), r0 = b and x0 = 0 in one pass (start of an inner FP32 solve)
void launch_scale_down_start(const z64* in, z32* b, z32* r0, z32* x0, const double* s, size_t n, int nrhs,
                             hipStream_t st);
// r = b and x = 0 over n complex entries (all columns of a batch: n = nrhs * length)
void launch_dc_start(const z64* b, z64* r, z64* x, size_t n, hipStream_t st);
// active[j] = act_host[j] (host-visible memory written before the launch), bad[j] = 0 if bad
void launch_set_active(int* active, const int* act_host, int* bad, int nrhs, hipStream_t st);
// x64 += s[rhs] * e32     (defect-correction update)
void launch_scale_up_add(z64* x, const z32* e, const double* s, size_t n, int nrhs, hipStream_t st);

// Scalar steps of CG, one thread per column; `active[rhs] == 0` freezes a column.
void launch_cg_alpha(const double* rz, const double* pq, double* alpha, const int* active, int* bad, int nrhs,
                     hipStream_t st);
void launch_cg_beta(const double* rz_new, double* rz, double* beta, const int* active, int nrhs, hipStream_t st);
void launch_cg_beta_flex(const double* rz_new, const double* rzo, double* rz, double* beta, const int* active,
                         int nrhs, hipStream_t st);

// Gauge relayout: U[mu][t][x] -> fermion links with the antiperiodic sign folded in.
template <typename R>
void launch_prepare_links(const z64* gauge, cpx<R>* U, int lx, int lt, int antiperiodic, hipStream_t st);

// Counter-based Gaussian vectors (when the caller supplies no random starts).
void launch_random_gaussian(z64* v, size_t n, uint64_t seed, uint64_t stream_id, hipStream_t st);

// Layout conversions of the coarse links: device [D][col][K][row] <-> export [K][D][row][col].
void launch_links_export(const z64* L, z64* out, int nK, int nc, hipStream_t st);
template <typename Ro>
void launch_links_convert(const z64* L, cpx<Ro>* out, size_t n, hipStream_t st);
// out = a X + b Y + c Z elementwise over n complex values (in place allowed)
void launch_lincomb3(const z64* X, const z64* Y, const z64* Z, z64* out, double a, double b, double c, size_t n,
                     hipStream_t st);

}  // namespace smg
