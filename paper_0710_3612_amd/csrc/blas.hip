// Level-1 vector kernels for the Krylov solvers (Multigrid section: conjugate
// gradients preconditioned by the V-cycle) and the smoother calibration.
//
// Reductions are deterministic and batch invariant: every column of a batch is
// reduced by the same fixed number of blocks (a function of the column length
// only), each block sums in a fixed order with wavefront shuffles, and a second
// pass adds the block partials in a fixed order.  (A single pass with a
// last-block finisher needs a device-scope release per block, which on gfx950
// writes back the XCD's L2 and was measured slower.)  The second pass also takes
// the CG scalar updates that follow a dot product (alpha; beta and <r,z>).  Sums are accumulated in FP64
// for FP32 vectors too.  Krylov scalars live on the device, so the CG loop needs
// no host round trip except the convergence check.
#include <algorithm>

#include "common.h"

namespace smg {

namespace {

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block (kThreads) sum of two doubles; result valid in thread 0.
__device__ inline void block_sum2(double& a, double& b) {
  __shared__ double sa[kThreads / 64], sb[kThreads / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) { sa[w] = a; sb[w] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0; b = 0;
    for (int i = 0; i < kThreads / 64; ++i) { a += sa[i]; b += sb[i]; }
  }
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_dot_partial(const cpx<R>* __restrict__ a, const cpx<R>* __restrict__ b,
                                                          size_t n, int nb, double* __restrict__ partial) {
  const size_t off = (size_t)blockIdx.y * n;
  double re = 0, im = 0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)nb * kThreads) {
    const cpx<R> u = a[off + i], v = b[off + i];
    re += (double)u.re * v.re + (double)u.im * v.im;
    im += (double)u.re * v.im - (double)u.im * v.re;
  }
  block_sum2(re, im);
  if (threadIdx.x == 0) {
    partial[2 * ((size_t)blockIdx.y * nb + blockIdx.x)] = re;
    partial[2 * ((size_t)blockIdx.y * nb + blockIdx.x) + 1] = im;
  }
}

// Second pass, one block per column: the partials in index order.  EPI 0: out =
// sum.  EPI 1 (alpha; sum = <p,q>, s = <r,z>): out = alpha, breakdown flagged in
// bad.  EPI 2 (beta; sum = <r,z>_new, s = <r,z>_old): out = beta, s <- sum.
template <int EPI>
__global__ void __launch_bounds__(kThreads) k_reduce_final(const double* __restrict__ partial, int nb,
                                                           double* __restrict__ out, double* __restrict__ s,
                                                           const int* __restrict__ active, int* __restrict__ bad,
                                                           double* __restrict__ out_host, int* __restrict__ bad_host) {
  double re = 0, im = 0;
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    re += partial[2 * ((size_t)blockIdx.x * nb + i)];
    im += partial[2 * ((size_t)blockIdx.x * nb + i) + 1];
  }
  block_sum2(re, im);
  if (threadIdx.x != 0) return;
  const int j = blockIdx.x;
  // out_host / bad_host (may be null): host-visible mirrors (coherent pinned memory) that
  // the host reads after a stream synchronisation, without a copy of its own
  if (EPI == 0) {
    out[2 * j] = re;
    out[2 * j + 1] = im;
    if (out_host) {
      out_host[2 * j] = re;
      out_host[2 * j + 1] = im;
    }
  } else if (EPI == 1) {
    double al = 0;
    bool broke = false;
    if (active[j]) {
      const double num = s[2 * j], den = re;
      if (!isfinite(num) || !isfinite(den)) {
        broke = true;
      } else if (num == 0) {
        al = 0;  // residual is exactly zero: nothing left to do in this column
      } else if (!(den > 0)) {
        broke = true;
      } else {
        al = num / den;
      }
    }
    if (broke) {
      bad[j] = 1;
      if (bad_host) bad_host[j] = 1;
    }
    out[j] = al;
  } else {
    double be = 0;
    if (active[j] && s[2 * j] != 0) be = re / s[2 * j];
    out[j] = be;
    if (active[j]) {
      s[2 * j] = re;
      s[2 * j + 1] = im;
    }
  }
}

// x += alpha p ; r -= alpha q ; partial |r|^2
template <typename R>
__global__ void __launch_bounds__(kThreads) k_axpy_update(cpx<R>* __restrict__ x, cpx<R>* __restrict__ r,
                                                          const cpx<R>* __restrict__ p, const cpx<R>* __restrict__ q,
                                                          const double* __restrict__ alpha, size_t n, int nb,
                                                          double* __restrict__ partial) {
  const size_t off = (size_t)blockIdx.y * n;
  const R a = (R)alpha[blockIdx.y];
  double rr = 0, dummy = 0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)nb * kThreads) {
    const size_t j = off + i;
    x[j] = x[j] + a * p[j];
    const cpx<R> rn = r[j] - a * q[j];
    r[j] = rn;
    rr += (double)rn.re * rn.re + (double)rn.im * rn.im;
  }
  block_sum2(rr, dummy);
  if (threadIdx.x == 0) {
    partial[2 * ((size_t)blockIdx.y * nb + blockIdx.x)] = rr;
    partial[2 * ((size_t)blockIdx.y * nb + blockIdx.x) + 1] = 0;
  }
}

// k_axpy_update with alpha formed in every block from the per-workgroup partials of
// <p, A p> (the fused CG step), in the order of k_reduce_final<1>, so alpha is the
// same in every block and equal to what that pass would give; block 0 records it
// and a breakdown.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_axpy_update_fold(cpx<R>* __restrict__ x, cpx<R>* __restrict__ r,
                                                               const cpx<R>* __restrict__ p,
                                                               const cpx<R>* __restrict__ q,
                                                               const double* __restrict__ ppart, int pnb,
                                                               const double* __restrict__ rz,
                                                               double* __restrict__ alpha, const int* __restrict__ active,
                                                               int* __restrict__ bad, int* __restrict__ bad_host,
                                                               size_t n, int nb, double* __restrict__ partial) {
  __shared__ double s_alpha;
  const int j = blockIdx.y;
  const size_t off = (size_t)j * n;
  // the thread's (at most E) elements are requested before alpha is formed: the loads
  // do not depend on it (grid-stride order, index clamped, the excess not stored)
  constexpr int E = 4;
  const bool pre = n <= (size_t)E * nb * kThreads;
  const size_t i0 = (size_t)blockIdx.x * kThreads + threadIdx.x, st = (size_t)nb * kThreads;
  cpx<R> xs[E], rs[E], ps[E], qs[E];
  if (pre) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const size_t k = off + min(i0 + e * st, n - 1);
      xs[e] = x[k];
      rs[e] = r[k];
      ps[e] = p[k];
      qs[e] = q[k];
    }
  }
  double re = 0, im = 0;
  for (int i = threadIdx.x; i < pnb; i += kThreads) {
    re += ppart[2 * ((size_t)j * pnb + i)];
    im += ppart[2 * ((size_t)j * pnb + i) + 1];
  }
  block_sum2(re, im);
  if (threadIdx.x == 0) {
    double al = 0;
    bool broke = false;
    if (active[j]) {
      const double num = rz[2 * j], den = re;
      if (!isfinite(num) || !isfinite(den)) {
        broke = true;
      } else if (num == 0) {
        al = 0;
      } else if (!(den > 0)) {
        broke = true;
      } else {
        al = num / den;
      }
    }
    if (blockIdx.x == 0) {
      if (broke) {
        bad[j] = 1;
        if (bad_host) bad_host[j] = 1;
      }
      alpha[j] = al;
    }
    s_alpha = al;
  }
  __syncthreads();
  const R a = (R)s_alpha;
  double rr = 0, dummy = 0;
  if (pre) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const size_t i = i0 + e * st;
      if (i < n) {
        x[off + i] = xs[e] + a * ps[e];
        const cpx<R> rn = rs[e] - a * qs[e];
        r[off + i] = rn;
        rr += (double)rn.re * rn.re + (double)rn.im * rn.im;
      }
    }
  } else {
    for (size_t i = i0; i < n; i += st) {
      const size_t k = off + i;
      x[k] = x[k] + a * p[k];
      const cpx<R> rn = r[k] - a * q[k];
      r[k] = rn;
      rr += (double)rn.re * rn.re + (double)rn.im * rn.im;
    }
  }
  block_sum2(rr, dummy);
  if (threadIdx.x == 0) {
    partial[2 * ((size_t)j * nb + blockIdx.x)] = rr;
    partial[2 * ((size_t)j * nb + blockIdx.x) + 1] = 0;
  }
}

template <typename R>
__global__ void k_xpay(const cpx<R>* __restrict__ z, cpx<R>* __restrict__ p, const double* __restrict__ beta,
                       size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  const R b = (R)beta[blockIdx.y];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[off + i] = z[off + i] + b * p[off + i];
}

template <typename R>
__global__ void k_axpy_const(cpx<R>* __restrict__ y, const cpx<R>* __restrict__ x, R a, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[off + i] = y[off + i] + a * x[off + i];
}

// Zero fill with a kernel (memset nodes are avoided where a caller may capture a graph).
__global__ void k_zero(unsigned long long* __restrict__ p, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

template <typename TI>
__global__ void k_axpy_const_lp(z32* __restrict__ y, const TI* __restrict__ x, float a, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[off + i] = y[off + i] + a * ldv(x, off + i);
}

template <typename R>
__global__ void k_sub(const cpx<R>* __restrict__ a, const cpx<R>* __restrict__ b, cpx<R>* __restrict__ y, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[off + i] = a[off + i] - b[off + i];
}

template <typename R>
__global__ void k_scale_cols(cpx<R>* __restrict__ x, const double* __restrict__ s, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  const R a = (R)s[blockIdx.y];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[off + i] = a * x[off + i];
}

template <typename R>
__global__ void k_scale_const(cpx<R>* x, R a, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[off + i] = a * x[off + i];
}

template <typename Ro, typename Ri>
__global__ void k_convert(const cpx<Ri>* __restrict__ in, cpx<Ro>* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = cvt<Ro>(in[i]);
}

// Defect-correction scales per column from |r|^2 (complex pairs) and the host's
// decision `on` (read from host-visible memory): a running column gets down = 1/|r|
// and up = |r|, a converged one 0 and 0.
__global__ void k_dc_scales(const double* __restrict__ rr, const int* __restrict__ on, double* __restrict__ down,
                            double* __restrict__ up, int nrhs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  const double r2 = rr[2 * j];
  down[j] = on[j] ? 1.0 / sqrt(r2) : 0.0;
  up[j] = on[j] ? sqrt(r2) : 0.0;
}

// Start of an inner FP32 solve: b = s r (rounded to FP32), its copy as the first
// residual, and the solution cleared, in one pass.
__global__ void k_scale_down_start(const z64* __restrict__ in, z32* __restrict__ b, z32* __restrict__ r0,
                                   z32* __restrict__ x0, const double* __restrict__ s, size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  const double a = s[blockIdx.y];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const z32 v = cvt<float>(a * in[off + i]);
    b[off + i] = v;
    r0[off + i] = v;
    x0[off + i] = mk(0.0f, 0.0f);
  }
}

// Start of a defect correction: r = b and x = 0 in one pass.
__global__ void k_dc_start(const z64* __restrict__ b, z64* __restrict__ r, z64* __restrict__ x, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    r[i] = b[i];
    x[i] = mk(0.0, 0.0);
  }
}

// Per-column flags of a Krylov solve from host-visible memory: active[j] = act_host[j],
// and bad[j] = 0 when bad is given.
__global__ void k_set_active(int* __restrict__ active, const int* __restrict__ act_host, int* __restrict__ bad,
                             int nrhs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  active[j] = act_host[j];
  if (bad) bad[j] = 0;
}

__global__ void k_scale_down(const z64* __restrict__ in, z32* __restrict__ out, const double* __restrict__ s,
                             size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  const double a = s[blockIdx.y];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[off + i] = cvt<float>(a * in[off + i]);
}

__global__ void k_scale_up_add(z64* __restrict__ x, const z32* __restrict__ e, const double* __restrict__ s,
                               size_t n) {
  const size_t off = (size_t)blockIdx.y * n;
  const double a = s[blockIdx.y];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[off + i] = x[off + i] + a * cvt<double>(e[off + i]);
}

// alpha = <r,z> / <p,Ap>; a column that is frozen or breaks down gets alpha = 0.
__global__ void k_cg_alpha(const double* __restrict__ rz, const double* __restrict__ pq, double* __restrict__ alpha,
                           const int* __restrict__ active, int* __restrict__ bad, int nrhs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double a = 0;
  if (active[j]) {
    const double num = rz[2 * j], den = pq[2 * j];
    if (!isfinite(num) || !isfinite(den)) {
      bad[j] = 1;
    } else if (num == 0) {
      a = 0;  // residual is exactly zero: nothing left to do in this column
    } else if (!(den > 0)) {
      bad[j] = 1;
    } else {
      a = num / den;
    }
  }
  alpha[j] = a;
}

// beta = <r,z>_new / <r,z>_old ; rz_old <- rz_new.
__global__ void k_cg_beta(const double* __restrict__ rz_new, double* __restrict__ rz, double* __restrict__ beta,
                          const int* __restrict__ active, int nrhs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double b = 0;
  if (active[j] && rz[2 * j] != 0) b = rz_new[2 * j] / rz[2 * j];
  beta[j] = b;
  if (active[j]) {
    rz[2 * j] = rz_new[2 * j];
    rz[2 * j + 1] = rz_new[2 * j + 1];
  }
}

// Flexible (Polak-Ribiere) beta = (<r,z>_new - <r_new, z_old>) / <r,z>_old; rz_old <- rz_new.
__global__ void k_cg_beta_flex(const double* __restrict__ rz_new, const double* __restrict__ rzo,
                               double* __restrict__ rz, double* __restrict__ beta, const int* __restrict__ active,
                               int nrhs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nrhs) return;
  double b = 0;
  if (active[j] && rz[2 * j] != 0) b = (rz_new[2 * j] - rzo[2 * j]) / rz[2 * j];
  beta[j] = b;
  if (active[j]) {
    rz[2 * j] = rz_new[2 * j];
    rz[2 * j + 1] = rz_new[2 * j + 1];
  }
}

inline dim3 ew_grid(size_t n, int nrhs) {
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 4096) g = 4096;
  return dim3((unsigned)g, nrhs);
}

}  // namespace

template <typename R>
void launch_dot(const cpx<R>* a, const cpx<R>* b, size_t n, int nrhs, Red red, double* out, hipStream_t st,
                double* out_host) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_dot_partial<R>), dim3(nb, nrhs), dim3(kThreads), 0, st, a, b, n, nb, red.partial);
  hipLaunchKernelGGL((k_reduce_final<0>), dim3(nrhs), dim3(kThreads), 0, st, red.partial, nb, out, nullptr, nullptr,
                     nullptr, out_host, nullptr);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_dot_alpha(const cpx<R>* p, const cpx<R>* q, size_t n, int nrhs, Red red, const double* rz,
                      double* alpha, const int* active, int* bad, hipStream_t st, int* bad_host) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_dot_partial<R>), dim3(nb, nrhs), dim3(kThreads), 0, st, p, q, n, nb, red.partial);
  hipLaunchKernelGGL((k_reduce_final<1>), dim3(nrhs), dim3(kThreads), 0, st, red.partial, nb, alpha,
                     const_cast<double*>(rz), active, bad, nullptr, bad_host);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_dot_beta(const cpx<R>* r, const cpx<R>* z, size_t n, int nrhs, Red red, double* rz, double* beta,
                     const int* active, hipStream_t st) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_dot_partial<R>), dim3(nb, nrhs), dim3(kThreads), 0, st, r, z, n, nb, red.partial);
  hipLaunchKernelGGL((k_reduce_final<2>), dim3(nrhs), dim3(kThreads), 0, st, red.partial, nb, beta, rz, active,
                     nullptr, nullptr, nullptr);
  HIPCHECK(hipGetLastError());
}

// beta = |r|^2 / <r, z>_old for an unpreconditioned CG (z = r), from the partial sums
// of |r|^2 that the last k_axpy_update left in red.partial (no pass over r).
void launch_beta_partials(size_t n, int nrhs, Red red, double* rz, double* beta, const int* active,
                          hipStream_t st) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_reduce_final<2>), dim3(nrhs), dim3(kThreads), 0, st, red.partial, nb, beta, rz, active,
                     nullptr, nullptr, nullptr);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_axpy_update(cpx<R>* x, cpx<R>* r, const cpx<R>* p, const cpx<R>* q, const double* alpha, size_t n,
                        int nrhs, Red red, double* rr, hipStream_t st, double* rr_host) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_axpy_update<R>), dim3(nb, nrhs), dim3(kThreads), 0, st, x, r, p, q, alpha, n, nb,
                     red.partial);
  hipLaunchKernelGGL((k_reduce_final<0>), dim3(nrhs), dim3(kThreads), 0, st, red.partial, nb, rr, nullptr, nullptr,
                     nullptr, rr_host, nullptr);
  HIPCHECK(hipGetLastError());
}

void launch_axpy_update_fold(z32* x, z32* r, const z32* p, const z32* q, const double* ppart, int pnb,
                             const double* rz, double* alpha, const int* active, int* bad, int* bad_host, size_t n,
                             int nrhs, double* rr_part_host, hipStream_t st) {
  const int nb = red_blocks(n);
  hipLaunchKernelGGL((k_axpy_update_fold<float>), dim3(nb, nrhs), dim3(kThreads), 0, st, x, r, p, q, ppart, pnb, rz,
                     alpha, active, bad, bad_host, n, nb, rr_part_host);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_xpay(const cpx<R>* z, cpx<R>* p, const double* beta, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_xpay<R>), ew_grid(n, nrhs), dim3(kThreads), 0, st, z, p, beta, n);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_axpy_const(cpx<R>* y, const cpx<R>* x, double a, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_axpy_const<R>), ew_grid(n, nrhs), dim3(kThreads), 0, st, y, x, (R)a, n);
  HIPCHECK(hipGetLastError());
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes % 8 != 0) throw Error(-1, "launch_zero needs a multiple of 8 bytes");
  const size_t words = bytes / 8;
  if (words == 0) return;
  const unsigned blocks = (unsigned)std::min<size_t>((words + kThreads - 1) / kThreads, 4096);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(kThreads), 0, st, static_cast<unsigned long long*>(p), words);
  HIPCHECK(hipGetLastError());
}

template <typename TI>
void launch_axpy_const_lp(z32* y, const TI* x, double a, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_axpy_const_lp<TI>), ew_grid(n, nrhs), dim3(kThreads), 0, st, y, x, (float)a, n);
  HIPCHECK(hipGetLastError());
}
template void launch_axpy_const_lp<bfc>(z32*, const bfc*, double, size_t, int, hipStream_t);
template void launch_axpy_const_lp<hfc>(z32*, const hfc*, double, size_t, int, hipStream_t);

template <typename R>
void launch_sub(const cpx<R>* a, const cpx<R>* b, cpx<R>* y, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_sub<R>), ew_grid(n, nrhs), dim3(kThreads), 0, st, a, b, y, n);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_scale_cols(cpx<R>* x, const double* s, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_cols<R>), ew_grid(n, nrhs), dim3(kThreads), 0, st, x, s, n);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_scale_const(cpx<R>* x, double a, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_scale_const<R>), ew_grid(n, nrhs), dim3(kThreads), 0, st, x, (R)a, n);
  HIPCHECK(hipGetLastError());
}

template <typename Ro, typename Ri>
void launch_convert(const cpx<Ri>* in, cpx<Ro>* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<Ro, Ri>), ew_grid(n, 1), dim3(kThreads), 0, st, in, out, n);
  HIPCHECK(hipGetLastError());
}

void launch_dc_scales(const double* rr, const int* on, double* down, double* up, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_scales, dim3((nrhs + 63) / 64), dim3(64), 0, st, rr, on, down, up, nrhs);
  HIPCHECK(hipGetLastError());
}

void launch_scale_down(const z64* in, z32* out, const double* s, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_down, ew_grid(n, nrhs), dim3(kThreads), 0, st, in, out, s, n);
  HIPCHECK(hipGetLastError());
}

void launch_scale_down_start(const z64* in, z32* b, z32* r0, z32* x0, const double* s, size_t n, int nrhs,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_scale_down_start, ew_grid(n, nrhs), dim3(kThreads), 0, st, in, b, r0, x0, s, n);
  HIPCHECK(hipGetLastError());
}

void launch_dc_start(const z64* b, z64* r, z64* x, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_start, ew_grid(n, 1), dim3(kThreads), 0, st, b, r, x, n);
  HIPCHECK(hipGetLastError());
}

void launch_set_active(int* active, const int* act_host, int* bad, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_set_active, dim3((nrhs + 63) / 64), dim3(64), 0, st, active, act_host, bad, nrhs);
  HIPCHECK(hipGetLastError());
}

void launch_scale_up_add(z64* x, const z32* e, const double* s, size_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_up_add, ew_grid(n, nrhs), dim3(kThreads), 0, st, x, e, s, n);
  HIPCHECK(hipGetLastError());
}

void launch_cg_alpha(const double* rz, const double* pq, double* alpha, const int* active, int* bad, int nrhs,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_cg_alpha, dim3((nrhs + 63) / 64), dim3(64), 0, st, rz, pq, alpha, active, bad, nrhs);
  HIPCHECK(hipGetLastError());
}

void launch_cg_beta_flex(const double* rz_new, const double* rzo, double* rz, double* beta, const int* active,
                         int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta_flex, dim3((nrhs + 63) / 64), dim3(64), 0, st, rz_new, rzo, rz, beta, active, nrhs);
  HIPCHECK(hipGetLastError());
}

void launch_cg_beta(const double* rz_new, double* rz, double* beta, const int* active, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(k_cg_beta, dim3((nrhs + 63) / 64), dim3(64), 0, st, rz_new, rz, beta, active, nrhs);
  HIPCHECK(hipGetLastError());
}

#define INST(R)                                                                                              \
  template void launch_dot<R>(const cpx<R>*, const cpx<R>*, size_t, int, Red, double*, hipStream_t, double*);          \
  template void launch_dot_alpha<R>(const cpx<R>*, const cpx<R>*, size_t, int, Red, const double*, double*,    \
                                    const int*, int*, hipStream_t, int*);                                     \
  template void launch_dot_beta<R>(const cpx<R>*, const cpx<R>*, size_t, int, Red, double*, double*,            \
                                   const int*, hipStream_t);                                                  \
  template void launch_axpy_update<R>(cpx<R>*, cpx<R>*, const cpx<R>*, const cpx<R>*, const double*, size_t,  \
                                      int, Red, double*, hipStream_t, double*);                               \
  template void launch_xpay<R>(const cpx<R>*, cpx<R>*, const double*, size_t, int, hipStream_t);              \
  template void launch_axpy_const<R>(cpx<R>*, const cpx<R>*, double, size_t, int, hipStream_t);              \
  template void launch_sub<R>(const cpx<R>*, const cpx<R>*, cpx<R>*, size_t, int, hipStream_t);              \
  template void launch_scale_cols<R>(cpx<R>*, const double*, size_t, int, hipStream_t);               \
  template void launch_scale_const<R>(cpx<R>*, double, size_t, int, hipStream_t);
INST(double)
INST(float)
#undef INST
template void launch_convert<float, double>(const z64*, z32*, size_t, hipStream_t);
template void launch_convert<double, float>(const z32*, z64*, size_t, hipStream_t);
template void launch_convert<double, double>(const z64*, z64*, size_t, hipStream_t);

}  // namespace smg
