// Fine-lattice Wilson-Dirac operator D, its adjoint and the normal operator A = D^H D
// (Introduction of the paper: the Wilson discretisation and the normal equations).
//
// Each hop carries a rank-1 spin projector, so a hop is computed as one complex
// "half spinor" h, multiplied by the link and spread back to two spins:
//   (1 - s1) psi = (psi0 - psi1) (1, -1)      (1 + s1) psi = (psi0 + psi1) (1,  1)
//   (1 - s2) psi = (psi0 + i psi1)(1, -i)     (1 + s2) psi = (psi0 - i psi1)(1,  i)
// D uses (1 - gamma) on the forward hop and (1 + gamma) on the backward hop; D^H
// swaps them (gamma -> -gamma), which is the relation D^H = s3 D s3.
//
// Memory layout: vectors [nrhs][t][x][2] complex, links [mu][t][x] with the
// antiperiodic-t sign folded into mu = 1, t = lt - 1.  One thread per site; the
// four neighbours of consecutive threads are consecutive, so every load is
// coalesced.
#include "common.h"

namespace smg {

namespace {

template <typename R, bool DAG>
__device__ inline void wilson_site(const cpx<R>* __restrict__ U, const cpx<R>* __restrict__ x, int lx, int lt,
                                   int xx, int t, R diag, cpx<R>& o0, cpx<R>& o1) {
  const int V = lx * lt;
  const int s = t * lx + xx;
  const int sxp = t * lx + (xx + 1 == lx ? 0 : xx + 1);
  const int sxm = t * lx + (xx == 0 ? lx - 1 : xx - 1);
  const int stp = (t + 1 == lt ? 0 : t + 1) * lx + xx;
  const int stm = (t == 0 ? lt - 1 : t - 1) * lx + xx;
  const R half = (R)0.5;

  const cpx<R> a0 = x[2 * s], a1 = x[2 * s + 1];
  cpx<R> s0 = mk<R>(0, 0), s1 = mk<R>(0, 0);  // sum of projected hops (before the -1/2)

  // +x: link U0_s, neighbour s+x
  {
    const cpx<R> u = U[s];
    const cpx<R> p0 = x[2 * sxp], p1 = x[2 * sxp + 1];
    if (!DAG) {  // (1 - s1): h (1, -1)
      cpx<R> h = u * (p0 - p1);
      s0 = s0 + h; s1 = s1 - h;
    } else {     // (1 + s1): h (1, 1)
      cpx<R> h = u * (p0 + p1);
      s0 = s0 + h; s1 = s1 + h;
    }
  }
  // -x: conj(U0_{s-x}), neighbour s-x
  {
    const cpx<R> u = cj(U[sxm]);
    const cpx<R> p0 = x[2 * sxm], p1 = x[2 * sxm + 1];
    if (!DAG) {  // (1 + s1)
      cpx<R> h = u * (p0 + p1);
      s0 = s0 + h; s1 = s1 + h;
    } else {     // (1 - s1)
      cpx<R> h = u * (p0 - p1);
      s0 = s0 + h; s1 = s1 - h;
    }
  }
  // +t: U1_s, neighbour s+t
  {
    const cpx<R> u = U[V + s];
    const cpx<R> p0 = x[2 * stp], p1 = x[2 * stp + 1];
    if (!DAG) {  // (1 - s2): h = p0 + i p1, spread (1, -i)
      cpx<R> h = u * (p0 + imul(p1));
      s0 = s0 + h; s1 = s1 - imul(h);
    } else {     // (1 + s2): h = p0 - i p1, spread (1, i)
      cpx<R> h = u * (p0 - imul(p1));
      s0 = s0 + h; s1 = s1 + imul(h);
    }
  }
  // -t: conj(U1_{s-t}), neighbour s-t
  {
    const cpx<R> u = cj(U[V + stm]);
    const cpx<R> p0 = x[2 * stm], p1 = x[2 * stm + 1];
    if (!DAG) {  // (1 + s2)
      cpx<R> h = u * (p0 - imul(p1));
      s0 = s0 + h; s1 = s1 + imul(h);
    } else {     // (1 - s2)
      cpx<R> h = u * (p0 + imul(p1));
      s0 = s0 + h; s1 = s1 - imul(h);
    }
  }
  o0 = diag * a0 - half * s0;
  o1 = diag * a1 - half * s1;
}

template <typename R, bool DAG>
__global__ void __launch_bounds__(kThreads) k_wilson(const cpx<R>* __restrict__ U, const cpx<R>* __restrict__ x,
                                                     cpx<R>* __restrict__ y, int lx, int lt, R diag) {
  const int V = lx * lt;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  const size_t off = (size_t)blockIdx.y * 2 * V;
  cpx<R> o0, o1;
  wilson_site<R, DAG>(U, x + off, lx, lt, s % lx, s / lx, diag, o0, o1);
  y[off + 2 * s] = o0;
  y[off + 2 * s + 1] = o1;
}

// Second pass of A = D^H (D x): t = D x is given; applies D^H with an epilogue.
template <typename R, int MODE>
__global__ void __launch_bounds__(kThreads) k_normal2(const cpx<R>* __restrict__ U, const cpx<R>* __restrict__ t,
                                                      const cpx<R>* __restrict__ x, cpx<R>* __restrict__ y, int lx,
                                                      int lt, R diag, R c, cpx<R>* __restrict__ xacc,
                                                      const cpx<R>* __restrict__ aux) {
  const int V = lx * lt;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= V) return;
  const size_t off = (size_t)blockIdx.y * 2 * V;
  cpx<R> o0, o1;
  wilson_site<R, true>(U, t + off, lx, lt, s % lx, s / lx, diag, o0, o1);
  const size_t i0 = off + 2 * s, i1 = i0 + 1;
  if (MODE == 0) {
    y[i0] = o0; y[i1] = o1;
  } else if (MODE == 1) {
    const cpx<R> v0 = x[i0], v1 = x[i1];
    xacc[i0] = xacc[i0] + c * v0;
    xacc[i1] = xacc[i1] + c * v1;
    y[i0] = v0 - c * o0;
    y[i1] = v1 - c * o1;
  } else {
    y[i0] = aux[i0] - o0;
    y[i1] = aux[i1] - o1;
  }
}

template <typename R>
__global__ void k_prepare_links(const z64* __restrict__ g, cpx<R>* __restrict__ U, int lx, int lt, int anti) {
  const int V = lx * lt;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * V) return;
  z64 u = g[i];
  const int mu = i / V, s = i % V;
  if (anti && mu == 1 && s / lx == lt - 1) u = mk(-u.re, -u.im);
  U[i] = cvt<R>(u);
}

}  // namespace

template <typename R>
void launch_wilson(const cpx<R>* U, const cpx<R>* x, cpx<R>* y, int lx, int lt, double diag, int nrhs,
                   bool dagger, hipStream_t st) {
  const int V = lx * lt;
  dim3 grid((V + kThreads - 1) / kThreads, nrhs);
  if (dagger)
    hipLaunchKernelGGL((k_wilson<R, true>), grid, dim3(kThreads), 0, st, U, x, y, lx, lt, (R)diag);
  else
    hipLaunchKernelGGL((k_wilson<R, false>), grid, dim3(kThreads), 0, st, U, x, y, lx, lt, (R)diag);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_normal(const cpx<R>* U, const cpx<R>* x, cpx<R>* y, cpx<R>* tmp, int lx, int lt, double diag,
                   int nrhs, int mode, double c, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st) {
  launch_wilson<R>(U, x, tmp, lx, lt, diag, nrhs, false, st);
  const int V = lx * lt;
  dim3 grid((V + kThreads - 1) / kThreads, nrhs);
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((k_normal2<R, 0>), grid, dim3(kThreads), 0, st, U, tmp, x, y, lx, lt, (R)diag, (R)c,
                         xacc, aux);
      break;
    case 1:
      hipLaunchKernelGGL((k_normal2<R, 1>), grid, dim3(kThreads), 0, st, U, tmp, x, y, lx, lt, (R)diag, (R)c,
                         xacc, aux);
      break;
    default:
      hipLaunchKernelGGL((k_normal2<R, 2>), grid, dim3(kThreads), 0, st, U, tmp, x, y, lx, lt, (R)diag, (R)c,
                         xacc, aux);
  }
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_prepare_links(const z64* gauge, cpx<R>* U, int lx, int lt, int antiperiodic, hipStream_t st) {
  const int n = 2 * lx * lt;
  hipLaunchKernelGGL((k_prepare_links<R>), dim3(grid_for(n)), dim3(kThreads), 0, st, gauge, U, lx, lt,
                     antiperiodic);
  HIPCHECK(hipGetLastError());
}

template void launch_wilson<double>(const z64*, const z64*, z64*, int, int, double, int, bool, hipStream_t);
template void launch_wilson<float>(const z32*, const z32*, z32*, int, int, double, int, bool, hipStream_t);
template void launch_normal<double>(const z64*, const z64*, z64*, z64*, int, int, double, int, int, double, z64*,
                                    const z64*, hipStream_t);
template void launch_normal<float>(const z32*, const z32*, z32*, z32*, int, int, double, int, int, double, z32*,
                                   const z32*, hipStream_t);
template void launch_prepare_links<double>(const z64*, z64*, int, int, int, hipStream_t);
template void launch_prepare_links<float>(const z64*, z32*, int, int, int, hipStream_t);

}  // namespace smg
