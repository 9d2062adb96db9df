// Multigrid kernels: transfer (restriction P^H and prolongation P), the 9-point
// Galerkin coarse operator, block Gram-Schmidt, the Galerkin build and the dense
// coarsest solve (Multigrid section, Eq. 2; Adaptive Multigrid section).
//
// Aggregates (Adaptive Multigrid section): the lattice of level l is cut into
// bx x bt blocks of sites; aggregate J holds every degree of freedom of its block,
// so its variables are i = ((t % bt) * bx + x % bx) * dof + d.  Column (J, k) of the
// tentative P is the k-th block-orthonormal near-null vector restricted to J; the
// smoothed P (smoothed aggregation, same section) is (I - w A) applied to it and
// lives on the block plus a one-site ring.
//
// The coarse operator A_c = P^H A P couples a coarse site only to the 3x3 box
// around it (A has reach one site in each direction and the blocks are at least
// two sites wide), so it is stored as 9 dense nc x nc link blocks per coarse site.
#include "common.h"

namespace smg {

namespace {

template <int N>
struct IntC {
  static constexpr int v = N;
};

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Aggregate windows.  Column (J, k) of the prolongator lives on the block of J
// (halo h = 0, the tentative P) or on the block plus a one-site ring (h = 1, the
// smoothed P).  Window variable i = ((wy * (bx + 2h)) + wx) * dof + d with
// wx in [0, bx + 2h) standing for x = Jx * bx + wx - h (periodic).
// accumulator of v_mfma_f64_16x16x4f64 (four FP64 values per lane)
typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ inline int win_index(int J, int i, int lx, int lt, int dof, int bx, int bt, int cx, int h) {
  const int Jt = J / cx, Jx = J - Jt * cx;
  const int wxw = bx + 2 * h;
  const int site = i / dof, d = i - site * dof;
  const int wy = site / wxw, wx = site - wy * wxw;
  int x = Jx * bx + wx - h, t = Jt * bt + wy - h;
  x = x < 0 ? x + lx : (x >= lx ? x - lx : x);
  t = t < 0 ? t + lt : (t >= lt ? t - lt : t);
  return (t * lx + x) * dof + d;
}

__device__ inline int agg_index(int J, int i, int lx, int dof, int bx, int bt, int cx) {
  return win_index(J, i, lx, 1 << 30, dof, bx, bt, cx, 0);
}

// Offsets o of fine coordinate c inside the window of block j (extent L, block b,
// halo h): o = c - j*b (mod L) within [-h, b + h).  At most one for h <= 1 when
// the coarse extent is at least 2 (no window covers the lattice twice).
__device__ inline bool win_offset(int c, int j, int b, int L, int h, int& o) {
  int v = c - j * b;
  v = ((v % L) + L) % L;           // [0, L)
  if (v < b + h) { o = v; return true; }
  if (v >= L - h) { o = v - L; return true; }
  return false;
}

// ---------------------------------------------------------------------------
// Restriction y[K][k] = sum_i conj(P[K][k][i]) x[agg(K,i)]: one wavefront per
// aggregate; the lanes walk the aggregate's variables (coalesced P rows) and the
// nc inner products are reduced across the wavefront one after the other.
// The result goes to out[k * ostride_k] (plain restriction or a column of the
// Galerkin links).
// ---------------------------------------------------------------------------
template <typename R, int NCH, typename TX = cpx<R>, int KW = 1, typename TP = cpx<R>, int NRB = 1>
__device__ inline void restrict_one(const TP* __restrict__ P, const TX* __restrict__ x, int K, int lx,
                                    int lt, int dof, int bx, int bt, int cx, int h, int nc, int ldk,
                                    cpx<R>* __restrict__ out, size_t ostride_k, int kbeg = 0, int kstep = 1,
                                    R ps = 1, int nq = 1, size_t xstride = 0, size_t ostride = 0) {
  // KW inner products per pass: their P rows are all requested before the first
  // is used (k clamped to nc - 1, window index clamped to nagg - 1; the excess
  // products are zeroed through xv and the excess results are not stored).  With
  // NRB > 1 the nq <= NRB right-hand sides x + q xstride (results at out + q ostride)
  // share every P row; each column's sums are those of NRB = 1.
  const int lane = threadIdx.x & 63;
  const int nagg = (bx + 2 * h) * (bt + 2 * h) * dof;
  cpx<R> xv[NRB][NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int i = lane + 64 * c;
    const int wi = i < nagg ? win_index(K, i, lx, lt, dof, bx, bt, cx, h) : -1;
#pragma unroll
    for (int q = 0; q < NRB; ++q)
      xv[q][c] = wi >= 0 ? ldv(x + (size_t)min(q, nq - 1) * xstride, wi) : mk<R>(0, 0);
  }
  const TP* PK = P + (size_t)K * ldk * nagg;
  for (int k0 = kbeg; k0 < nc; k0 += KW * kstep) {
    cpx<R> p[KW][NCH];
#pragma unroll
    for (int j = 0; j < KW; ++j) {
      const int k = min(k0 + j * kstep, nc - 1);
#pragma unroll
      for (int c = 0; c < NCH; ++c) p[j][c] = widen(PK[(size_t)k * nagg + min(lane + 64 * c, nagg - 1)]);
    }
#pragma unroll
    for (int q = 0; q < NRB; ++q) {
      if (q >= nq) break;
      R re[KW], im[KW];
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        re[j] = 0;
        im[j] = 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {  // explicit FMAs: the same rounding for every NRB
          re[j] = fma(p[j][c].re, xv[q][c].re, re[j]);
          re[j] = fma(p[j][c].im, xv[q][c].im, re[j]);
          im[j] = fma(p[j][c].re, xv[q][c].im, im[j]);
          im[j] = fma(-p[j][c].im, xv[q][c].re, im[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < KW; ++j) {
        re[j] = wave_sum(re[j]);
        im[j] = wave_sum(im[j]);
      }
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < KW; ++j)
          if (k0 + j * kstep < nc)
            out[(size_t)q * ostride + (size_t)(k0 + j * kstep) * ostride_k] = mk<R>(ps * re[j], ps * im[j]);
      }
    }
  }
}

// One workgroup per aggregate: wavefront w forms the inner products k = w, w+4, ...,
// KW of them per pass.
template <typename R, int NCH, typename TX = cpx<R>, int KW = 1, typename TP = cpx<R>, int NRB = 1>
__global__ void __launch_bounds__(kThreads) k_restrict(const TP* __restrict__ P, const TX* __restrict__ x,
                                                       cpx<R>* __restrict__ y, int lx, int lt, int dof, int bx,
                                                       int bt, int h, int nc, int ldk, R ps, int nrhs) {
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int K = blockIdx.x;
  if (K >= nK) return;
  const size_t n = (size_t)lx * lt * dof;
  const int r0 = blockIdx.y * NRB;
  restrict_one<R, NCH, TX, KW, TP, NRB>(P, x + r0 * n, K, lx, lt, dof, bx, bt, cx, h, nc, ldk,
                                        y + (size_t)r0 * nK * nc + (size_t)K * nc, 1, threadIdx.x >> 6,
                                        kThreads / 64, ps, min(NRB, nrhs - r0), n, (size_t)nK * nc);
}

// k_restrict with KW = the inner products of one wave (ceil(nc / 4)), at most 4 per
// pass and at most 64 words of P rows in flight per lane.
template <typename R, int NCH, typename TX, typename TP>
void launch_restrict_kw(dim3 grid, hipStream_t st, const TP* P, R ps, const TX* x, cpx<R>* y, int lx, int lt,
                        int dof, int bx, int bt, int h, int nc, int ldk, int nrhs) {
  const int cap = (int)(64 / (NCH * sizeof(cpx<R>) / sizeof(float)));
  const int q = std::min((nc + 3) / 4, std::max(cap, 1));
  // four right-hand sides share the P rows while their windows take at most 32 registers
  constexpr bool kShare = NCH * sizeof(cpx<R>) / sizeof(float) <= 8;
  const bool share = kShare && nrhs >= 4;
  if (share) grid.y = (nrhs + 3) / 4;
  auto go = [&](auto kw) {
    constexpr int KW = decltype(kw)::v;
    if constexpr (kShare) {
      if (share) {
        hipLaunchKernelGGL((k_restrict<R, NCH, TX, KW, TP, 4>), grid, dim3(kThreads), 0, st, P, x, y, lx, lt, dof, bx,
                           bt, h, nc, ldk, ps, nrhs);
        return;
      }
    }
    hipLaunchKernelGGL((k_restrict<R, NCH, TX, KW, TP, 1>), grid, dim3(kThreads), 0, st, P, x, y, lx, lt, dof, bx, bt,
                       h, nc, ldk, ps, nrhs);
  };
  if (q <= 1)
    go(IntC<1>{});
  else if (q == 2)
    go(IntC<2>{});
  else if (q == 3)
    go(IntC<3>{});
  else
    go(IntC<4>{});
}

// FP32 restriction with one wavefront per aggregate forming all NCOL >= nc inner
// products: each lane accumulates 2 * NCOL partial sums (re and im per column) over
// its window variables, with every P row requested before the first product.  A
// halving butterfly then sums them across the wavefront: at offset o each lane
// keeps half of its values and adds the other half of its partner's, so after
// log2(2 NCOL) steps (offsets 32, 16, ...) one sum is left per lane group and plain
// steps finish it.  That is 2 NCOL - 1 shuffles, where reducing each sum on its own
// takes 6 per sum.  Four aggregates per workgroup, no barrier.
template <int NCOL>
__device__ inline float butterfly_sum(float (&v)[2 * NCOL], int lane) {
  constexpr int V = 2 * NCOL;
  int o = 32;
#pragma unroll
  for (int cnt = V; cnt > 1; cnt >>= 1, o >>= 1) {
    const bool up = lane & o;
#pragma unroll
    for (int j = 0; j < cnt / 2; ++j) {
      const float send = up ? v[2 * j] : v[2 * j + 1];
      const float keep = up ? v[2 * j + 1] : v[2 * j];
      v[j] = keep + __shfl_xor(send, o, 64);
    }
  }
  float r = v[0];
  for (; o > 0; o >>= 1) r += __shfl_xor(r, o, 64);
  return r;
}

// NRB right-hand sides per wavefront (blockIdx.y takes NRB at a time): the P rows are
// read once for all of them; each column's arithmetic is the same as with NRB = 1.
template <int NCOL, int NCH, typename TX, typename TP, int NRB>
__global__ void __launch_bounds__(kThreads) k_restrict_bf(const TP* __restrict__ P, const TX* __restrict__ x,
                                                          z32* __restrict__ y, int lx, int lt, int dof, int bx,
                                                          int bt, int h, int nc, int ldk, float ps, int nrhs, Grp g) {
  if (g.op) {  // grouped (NRB = 1): this column's system
    P = static_cast<const TP*>(g.op[blockIdx.y]);
    ps = (float)g.s[blockIdx.y];
  }
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int K = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (K >= nK) return;  // whole wavefronts; the kernel has no barrier
  const int lane = threadIdx.x & 63;
  const size_t n = (size_t)lx * lt * dof;
  const int nagg = (bx + 2 * h) * (bt + 2 * h) * dof;
  const int r0 = blockIdx.y * NRB;
  const TP* PK = P + (size_t)K * ldk * nagg;
  TP pv[NCOL][NCH];
#pragma unroll
  for (int k = 0; k < NCOL; ++k)
#pragma unroll
    for (int c = 0; c < NCH; ++c) pv[k][c] = PK[(size_t)min(k, nc - 1) * nagg + min(lane + 64 * c, nagg - 1)];
  int wi[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int i = lane + 64 * c;
    wi[c] = i < nagg ? win_index(K, i, lx, lt, dof, bx, bt, cx, h) : -1;
  }
  z32 xv[NRB][NCH];  // the window of every right-hand side of the group, requested together
#pragma unroll
  for (int q = 0; q < NRB; ++q) {
    const TX* xr = x + (size_t)min(r0 + q, nrhs - 1) * n;
#pragma unroll
    for (int c = 0; c < NCH; ++c) xv[q][c] = wi[c] >= 0 ? ldv(xr, wi[c]) : mk<float>(0, 0);
  }
  // the sum left in a lane after the butterfly: bit s of its index is lane bit 5 - s
  constexpr int V = 2 * NCOL, LOGV = V == 8 ? 3 : V == 16 ? 4 : 5;
  int idx = 0;
#pragma unroll
  for (int b = 0; b < LOGV; ++b) idx |= ((lane >> (5 - b)) & 1) << b;
  const int k = idx >> 1;
#pragma unroll
  for (int q = 0; q < NRB; ++q) {
    if (r0 + q >= nrhs) break;
    float v[2 * NCOL];
#pragma unroll
    for (int kk = 0; kk < NCOL; ++kk) {
      float re = 0, im = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {  // explicit FMAs: the same rounding for every NRB
        const z32 a = widen(pv[kk][c]);
        re = fmaf(a.re, xv[q][c].re, re);
        re = fmaf(a.im, xv[q][c].im, re);
        im = fmaf(a.re, xv[q][c].im, im);
        im = fmaf(-a.im, xv[q][c].re, im);
      }
      v[2 * kk] = re;
      v[2 * kk + 1] = im;
    }
    const float r = butterfly_sum<NCOL>(v, lane);
    if ((lane & (64 / V - 1)) == 0 && k < nc)
      reinterpret_cast<float*>(y + ((size_t)(r0 + q) * nK + K) * nc)[idx] = ps * r;
  }
}

// The same for windows of more than 128 variables: one workgroup per aggregate,
// wavefront w takes the 64-variable chunks w, w + 4, ... (at most CPW of them), and
// the four butterfly results are added in wavefront order through LDS.
// NRB right-hand sides per workgroup (blockIdx.y takes NRB at a time) share the P rows.
template <int NCOL, int CPW, typename TX, typename TP, int NRB>
__global__ void __launch_bounds__(kThreads) k_restrict_bfw(const TP* __restrict__ P, const TX* __restrict__ x,
                                                           z32* __restrict__ y, int lx, int lt, int dof, int bx,
                                                           int bt, int h, int nc, int ldk, float ps, int nrhs,
                                                           Grp g) {
  if (g.op) {  // grouped (NRB = 1): this column's system
    P = static_cast<const TP*>(g.op[blockIdx.y]);
    ps = (float)g.s[blockIdx.y];
  }
  constexpr int NW = kThreads / 64, V = 2 * NCOL, LOGV = V == 8 ? 3 : V == 16 ? 4 : 5;
  __shared__ float part[NRB][NW][V];
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int K = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const size_t n = (size_t)lx * lt * dof;
  const int nagg = (bx + 2 * h) * (bt + 2 * h) * dof;
  const int r0 = blockIdx.y * NRB;
  const TP* PK = P + (size_t)K * ldk * nagg;
  TP pv[CPW][NCOL];
  z32 xv[NRB][CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int i = lane + 64 * (w + NW * j);
#pragma unroll
    for (int k = 0; k < NCOL; ++k) pv[j][k] = PK[(size_t)min(k, nc - 1) * nagg + min(i, nagg - 1)];
    const int wi = i < nagg ? win_index(K, i, lx, lt, dof, bx, bt, cx, h) : -1;
#pragma unroll
    for (int q = 0; q < NRB; ++q)
      xv[q][j] = wi >= 0 ? ldv(x + (size_t)min(r0 + q, nrhs - 1) * n, wi) : mk<float>(0, 0);
  }
  int idx = 0;
#pragma unroll
  for (int b = 0; b < LOGV; ++b) idx |= ((lane >> (5 - b)) & 1) << b;
#pragma unroll
  for (int q = 0; q < NRB; ++q) {
    float v[V];
#pragma unroll
    for (int k = 0; k < NCOL; ++k) {
      float re = 0, im = 0;
#pragma unroll
      for (int j = 0; j < CPW; ++j) {  // explicit FMAs: the same rounding for every NRB
        const z32 a = widen(pv[j][k]);
        re = fmaf(a.re, xv[q][j].re, re);
        re = fmaf(a.im, xv[q][j].im, re);
        im = fmaf(a.re, xv[q][j].im, im);
        im = fmaf(-a.im, xv[q][j].re, im);
      }
      v[2 * k] = re;
      v[2 * k + 1] = im;
    }
    const float r = butterfly_sum<NCOL>(v, lane);
    if ((lane & (64 / V - 1)) == 0) part[q][w][idx] = r;
  }
  __syncthreads();
  const int q = threadIdx.x / (2 * nc), comp = threadIdx.x - q * 2 * nc;
  if (q < NRB && r0 + q < nrhs) {
    float t = 0;
#pragma unroll
    for (int u = 0; u < NW; ++u) t += part[q][u][comp];
    reinterpret_cast<float*>(y + ((size_t)(r0 + q) * nK + K) * nc)[comp] = ps * t;
  }
}

// Prolongation y (+)= P e in two deterministic phases.
// Phase 1: per aggregate window, w[K][i] = sum_k P[K][k][i] e[K][k] (lanes walk the
// window variables, so P rows are read coalesced and e is a broadcast).
// NRB right-hand sides per thread (blockIdx.y takes NRB at a time): each P entry is
// read once for all of them; every column's sums run in the same order as with NRB = 1.
template <typename R, typename TP, int NRB>
__global__ void __launch_bounds__(kThreads) k_prolong_win(const TP* __restrict__ P, const cpx<R>* __restrict__ e,
                                                          cpx<R>* __restrict__ wbuf, int nK, int nw, int nc, int ldk,
                                                          R ps, int nrhs, Grp g) {
  if (g.op) {  // grouped (NRB = 1): this column's system
    P = static_cast<const TP*>(g.op[blockIdx.y]);
    ps = (R)g.s[blockIdx.y];
  }
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nK * nw) return;
  const int K = (int)(idx / nw), i = (int)(idx - (size_t)K * nw);
  const int r0 = blockIdx.y * NRB;
  const TP* PK = P + (size_t)K * ldk * nw + i;
  cpx<R> acc[NRB];
#pragma unroll
  for (int q = 0; q < NRB; ++q) acc[q] = mk<R>(0, 0);
  for (int k0 = 0; k0 < nc; k0 += 4) {  // four columns per group, index clamped: loads in flight together
    cpx<R> pv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) pv[j] = widen(PK[(size_t)min(k0 + j, nc - 1) * nw]);
#pragma unroll
    for (int q = 0; q < NRB; ++q) {
      const cpx<R>* eK = e + ((size_t)min(r0 + q, nrhs - 1) * nK + K) * nc;
      cpx<R> ev[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) ev[j] = eK[min(k0 + j, nc - 1)];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k0 + j < nc) fma_acc_x(acc[q], pv[j], ev[j]);
    }
  }
#pragma unroll
  for (int q = 0; q < NRB; ++q)
    if (r0 + q < nrhs) wbuf[(size_t)(r0 + q) * nK * nw + idx] = ps * acc[q];
}

// Phase 2: every fine variable sums the window values that cover it (one window
// for the tentative P, up to 2 x 2 for the smoothed one), in a fixed order.
template <typename R, int MODE>
__global__ void __launch_bounds__(kThreads) k_prolong_gather(const cpx<R>* __restrict__ wbuf, cpx<R>* __restrict__ y,
                                                             int lx, int lt, int dof, int bx, int bt, int h) {
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int wxw = bx + 2 * h;
  const int nw = wxw * (bt + 2 * h) * dof;
  const size_t n = (size_t)lx * lt * dof;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int rhs = blockIdx.y;
  const int site = (int)(idx / dof), d = (int)(idx - (size_t)site * dof);
  const int t = site / lx, x = site - t * lx;
  const cpx<R>* wb = wbuf + (size_t)rhs * nK * nw;
  const size_t o = (size_t)rhs * n + idx;
  const cpx<R> y0 = MODE == 1 ? y[o] : mk<R>(0, 0);  // requested early, added last
  cpx<R> acc = mk<R>(0, 0);
  int jts[3], njt = 0, jxs[3], njx = 0;
  for (int q = -h; q <= h; ++q) {  // distinct candidate blocks
    int jt = (t / bt + q + ct) % ct, jx = (x / bx + q + cx) % cx;
    bool dup = false;
    for (int a = 0; a < njt; ++a) dup |= (jts[a] == jt);
    if (!dup) jts[njt++] = jt;
    dup = false;
    for (int a = 0; a < njx; ++a) dup |= (jxs[a] == jx);
    if (!dup) jxs[njx++] = jx;
  }
  for (int a = 0; a < njt; ++a) {
    int ot;
    if (!win_offset(t, jts[a], bt, lt, h, ot)) continue;
    for (int b = 0; b < njx; ++b) {
      int ox;
      if (!win_offset(x, jxs[b], bx, lx, h, ox)) continue;
      acc = acc + wb[(size_t)(jts[a] * cx + jxs[b]) * nw + ((ot + h) * wxw + (ox + h)) * dof + d];
    }
  }
  y[o] = MODE == 0 ? acc : y0 + acc;
}

// Phase 2 without the general search: with h = 0 a variable lies in the window of
// its own block only; with h = 1 (both coarse extents >= 2) also in the window of
// the block before it along an axis when it is the first site of its block there
// (window coordinate b + 1) and of the block after it when it is the last (window
// coordinate 0).  Windows are visited in the order of the general kernel (blocks
// j - 1, j, j + 1 along t, then along x); four integer divisions per variable.
template <typename R, int MODE, int H>
__global__ void __launch_bounds__(kThreads) k_prolong_gather_f(const cpx<R>* __restrict__ wbuf,
                                                               cpx<R>* __restrict__ y, int lx, int lt, int dof, int bx,
                                                               int bt) {
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int wxw = bx + 2 * H;
  const int nw = wxw * (bt + 2 * H) * dof;
  const size_t n = (size_t)lx * lt * dof;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int rhs = blockIdx.y;
  const int site = (int)(idx / dof), d = (int)(idx - (size_t)site * dof);
  const int t = site / lx, x = site - t * lx;
  const int jt = t / bt, ut = t - jt * bt, jx = x / bx, ux = x - jx * bx;
  const cpx<R>* wb = wbuf + (size_t)rhs * nK * nw;
  const size_t o = (size_t)rhs * n + idx;
  const cpx<R> y0 = MODE == 1 ? y[o] : mk<R>(0, 0);  // requested early, added last
  // candidate blocks and window coordinates along each axis, in the order j - 1, j, j + 1
  int bt_[3], wt_[3], nt = 0, bx_[3], wx_[3], nx = 0;
  if (H == 1 && ut == 0) { bt_[nt] = jt == 0 ? ct - 1 : jt - 1; wt_[nt++] = bt + 1; }
  bt_[nt] = jt; wt_[nt++] = ut + H;
  if (H == 1 && ut == bt - 1) { bt_[nt] = jt == ct - 1 ? 0 : jt + 1; wt_[nt++] = 0; }
  if (H == 1 && ux == 0) { bx_[nx] = jx == 0 ? cx - 1 : jx - 1; wx_[nx] = bx + 1; ++nx; }
  bx_[nx] = jx; wx_[nx++] = ux + H;
  if (H == 1 && ux == bx - 1) { bx_[nx] = jx == cx - 1 ? 0 : jx + 1; wx_[nx] = 0; ++nx; }
  cpx<R> acc = mk<R>(0, 0);
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nx; ++b)
      acc = acc + wb[(size_t)(bt_[a] * cx + bx_[b]) * nw + (wt_[a] * wxw + wx_[b]) * dof + d];
  y[o] = MODE == 0 ? acc : y0 + acc;
}

// ---------------------------------------------------------------------------
// Coarse 9-point operator: y_K = sum_D L_{K,D} v_{K+D}.  Links are stored
// [D][col][K][row], so for a fixed (D, col) consecutive outputs (K, row) read
// consecutive words.  A workgroup owns 64 consecutive outputs; its four
// wavefronts each sum a quarter of the columns for all nine link blocks and the
// partial sums meet in LDS.  Up to NR right-hand sides share every link load.
// A wave takes its columns Q at a time and the directions DU at a time (all nine
// for one FP32 right-hand side, fewer where more registers per load are needed):
// the column index is clamped rather than branched on and the excess products are
// masked at use, so every load of a group is issued before the first wait.
// ---------------------------------------------------------------------------
template <typename R, int MODE, int NR, int Q, typename TL = cpx<R>>
__global__ void __launch_bounds__(kThreads) k_coarse(const TL* __restrict__ L, const cpx<R>* __restrict__ v,
                                                     cpx<R>* __restrict__ y, int cx, int ct, int nc, int nrhs, R c,
                                                     R c2, cpx<R>* __restrict__ xacc,
                                                     const cpx<R>* __restrict__ aux, R lscale) {
  __shared__ cpx<R> part[3][NR][64];
  const int nK = cx * ct;
  const size_t n = (size_t)nK * nc;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tid = blockIdx.x * 64 + lane;  // output index (K, row)
  const int rhs0 = blockIdx.y * NR;
  const bool live = tid < (int)n;
  const int q = (nc + 3) / 4;
  const int c0 = w * q, c1 = min(nc, c0 + q);
  cpx<R> acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = mk<R>(0, 0);
  if (live) {
    const int K = tid / nc;
    const int Kt = K / cx, Kx = K - Kt * cx;
    const int xm = Kx == 0 ? cx - 1 : Kx - 1, xp = Kx == cx - 1 ? 0 : Kx + 1;
    const int tm = Kt == 0 ? ct - 1 : Kt - 1, tp = Kt == ct - 1 ? 0 : Kt + 1;
    const cpx<R>* vr[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) vr[r] = v + (size_t)min(rhs0 + r, nrhs - 1) * n;
    constexpr int DU = NR >= 4 ? 1 : (NR == 1 && sizeof(R) == 4 ? 9 : 3);
    for (int cb = c0; cb < c1; cb += Q) {
#pragma unroll 1
      for (int D0 = 0; D0 < 9; D0 += DU) {
#pragma unroll
      for (int dd = 0; dd < DU; ++dd) {
        const int D = D0 + dd;
        const int nt = D / 3 == 0 ? tm : (D / 3 == 1 ? Kt : tp);
        const int nx = D % 3 == 0 ? xm : (D % 3 == 1 ? Kx : xp);
        const size_t vn = (size_t)(nt * cx + nx) * nc;
        const TL* LD = L + (size_t)D * nc * n + tid;
        cpx<R> l[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) l[j] = widen(LD[(size_t)min(cb + j, c1 - 1) * n]);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
#pragma unroll
          for (int j = 0; j < Q; ++j) {
            cpx<R> x = vr[r][vn + min(cb + j, c1 - 1)];
            if (cb + j >= c1 || rhs0 + r >= nrhs) x = mk<R>(0, 0);
            fma_acc(acc[r], l[j], x);
          }
        }
      }
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) part[w - 1][r][lane] = acc[r];
  }
  __syncthreads();
  if (w != 0 || !live) return;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (rhs0 + r >= nrhs) break;
    // lscale: power-of-two scale of reduced-precision links (1 otherwise): exact
    const cpx<R> sum = lscale * (acc[r] + part[0][r][lane] + part[1][r][lane] + part[2][r][lane]);
    const size_t o = (size_t)(rhs0 + r) * n + tid;
    if (MODE == 0) {
      y[o] = sum;
    } else if (MODE == 1 || MODE == 3) {
      const cpx<R> vi = v[o];
      xacc[o] = MODE == 3 ? c * vi : xacc[o] + c * vi;
      y[o] = vi - c * sum;
    } else if (MODE == 4 || MODE == 5) {
      const cpx<R> vi = v[o];
      const cpx<R> a = MODE == 5 ? c * vi : xacc[o] + c * vi;
      xacc[o] = a + c2 * (vi - c * sum);
    } else {
      y[o] = aux[o] - sum;
    }
  }
}

// k_coarse for one right-hand side (4 <= nc <= 16, one pass of Q = ceil(nc / 4) columns
// per wave) with the vector entries staged in LDS.  The workgroup's 64 outputs belong
// to at most 64 / nc + 2 sites; the nc entries of their nine neighbours are loaded
// once per workgroup, while the lanes' link loads are in flight, instead of once per
// lane (the lanes of one site then read the same LDS word).  The products, their
// order and the reduction over the waves are those of k_coarse.
constexpr int kCoarseSvMax = 9 * (64 + 2 * 16);  // 9 (64 / nc + 2) nc entries at most (4 <= nc <= 16)

template <typename R, int MODE, int Q, typename TL, bool GRP = false>
__global__ void __launch_bounds__(kThreads) k_coarse_sv(const TL* __restrict__ L, const cpx<R>* __restrict__ v,
                                                        cpx<R>* __restrict__ y, int cx, int ct, int nc, R c, R c2,
                                                        cpx<R>* __restrict__ xacc, const cpx<R>* __restrict__ aux,
                                                        R lscale, Grp g) {
  __shared__ cpx<R> part[3][64];
  __shared__ cpx<R> sv[kCoarseSvMax];
  if constexpr (GRP) {  // grouped: this column's system
    L = static_cast<const TL*>(g.op[blockIdx.y]);
    lscale = (R)g.s[blockIdx.y];
    if (g.c) c = (R)g.c[blockIdx.y];
    if (g.c2) c2 = (R)g.c2[blockIdx.y];
  }
  const int nK = cx * ct;
  const size_t n = (size_t)nK * nc;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tid = blockIdx.x * 64 + lane;  // output index (K, row)
  const bool live = tid < (int)n;
  const int tidc = live ? tid : (int)n - 1;
  const int c0 = w * Q, c1 = min(nc, c0 + Q);
  // 1. the neighbours' vector entries, [site][direction][column]: thread t < 9 * sites
  // loads the nc entries of pair t = (site, direction), requested before the link loads
  // (a wait for them then does not wait for the links issued after them)
  const int K_lo = (blockIdx.x * 64) / nc;
  const int K_hi = min((blockIdx.x * 64 + 63) / nc, nK - 1);
  const int npair = (K_hi - K_lo + 1) * 9;
  const bool stager = (int)threadIdx.x < npair;
  const int pr = stager ? (int)threadIdx.x : 0;
  const int kl = pr / 9, D0 = pr - kl * 9;
  const int Ks = K_lo + kl;
  const int Kst = Ks / cx, Ksx = Ks - Kst * cx;
  int st_t = Kst + D0 / 3 - 1, st_x = Ksx + D0 % 3 - 1;
  st_t = st_t < 0 ? ct - 1 : (st_t >= ct ? 0 : st_t);
  st_x = st_x < 0 ? cx - 1 : (st_x >= cx ? 0 : st_x);
  const cpx<R>* src = v + (size_t)blockIdx.y * n + (size_t)(st_t * cx + st_x) * nc;
  cpx<R> vs[16];
#pragma unroll
  for (int col = 0; col < 16; ++col) vs[col] = src[min(col, nc - 1)];  // pair 0 for non-stagers
  __builtin_amdgcn_sched_barrier(0);  // keeps these loads ahead of the link loads
  // 2. every link load of the lane (column clamped, excess products masked below)
  TL l[9][Q];
#pragma unroll
  for (int D = 0; D < 9; ++D)
#pragma unroll
    for (int j = 0; j < Q; ++j) l[D][j] = L[((size_t)D * nc + min(c0 + j, nc - 1)) * n + tidc];
  __builtin_amdgcn_sched_barrier(0);  // all loads issued before the staging stores
  if (stager) {
#pragma unroll
    for (int col = 0; col < 16; ++col)
      if (col < nc) sv[pr * nc + col] = vs[col];
  }
  __syncthreads();
  cpx<R> acc = mk<R>(0, 0);
  if (live) {
    const int ko = tid / nc - K_lo;  // this output's site within the staged ones
#pragma unroll
    for (int D = 0; D < 9; ++D) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        cpx<R> x = sv[(ko * 9 + D) * nc + min(c0 + j, nc - 1)];
        if (c0 + j >= c1) x = mk<R>(0, 0);
        fma_acc(acc, widen(l[D][j]), x);
      }
    }
  }
  if (w > 0) part[w - 1][lane] = acc;
  __syncthreads();
  if (w != 0 || !live) return;
  const cpx<R> sum = lscale * (acc + part[0][lane] + part[1][lane] + part[2][lane]);
  const size_t o = (size_t)blockIdx.y * n + tid;
  if (MODE == 0) {
    y[o] = sum;
  } else if (MODE == 1 || MODE == 3) {
    const cpx<R> vi = v[o];
    xacc[o] = MODE == 3 ? c * vi : xacc[o] + c * vi;
    y[o] = vi - c * sum;
  } else if (MODE == 4 || MODE == 5) {
    const cpx<R> vi = v[o];
    const cpx<R> a = MODE == 5 ? c * vi : xacc[o] + c * vi;
    xacc[o] = a + c2 * (vi - c * sum);
  } else {
    y[o] = aux[o] - sum;
  }
}

// ---------------------------------------------------------------------------
// Block Gram-Schmidt (FP64): append candidate v as vector k of every aggregate.
// One workgroup per aggregate; two passes of modified Gram-Schmidt against the
// earlier vectors, then normalisation to 1 (Adaptive Multigrid section).
// ---------------------------------------------------------------------------
__device__ inline void block_allreduce2(double& a, double& b, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();  // earlier readers of sh are done
  if (l == 0) { sh[2 * w] = a; sh[2 * w + 1] = b; }
  __syncthreads();
  a = 0; b = 0;
  for (int i = 0; i < kThreads / 64; ++i) { a += sh[2 * i]; b += sh[2 * i + 1]; }
}

// Candidate k of block J (blockIdx.x) appended to the tentative P, two passes of
// modified Gram-Schmidt.  m = 1: one aggregate per block, column k.  m = 2
// (chirality split): blockIdx.y = chi takes the variables with d % 2 = chi, is made
// orthogonal to the earlier columns of the same chirality (those of the other one
// have disjoint support) and becomes column 2k + chi, zero on the other variables.
template <int NCH>
__global__ void __launch_bounds__(kThreads) k_gs_append(z64* __restrict__ P, const z64* __restrict__ v, int lx,
                                                        int dof, int bx, int bt, int cx, int k, int ldk, int m,
                                                        int* __restrict__ fail) {
  __shared__ double sh[2 * (kThreads / 64)];
  const int J = blockIdx.x;
  const int chi = blockIdx.y;
  const int nagg = bx * bt * dof;
  z64* PJ = P + (size_t)J * ldk * nagg;
  z64 w[NCH];
  double ref = 0, dummy = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int i = threadIdx.x + kThreads * c;
    const bool mine = i < nagg && (m == 1 || (i % dof) % 2 == chi);
    w[c] = mine ? v[agg_index(J, i, lx, dof, bx, bt, cx)] : mk(0.0, 0.0);
    ref += w[c].re * w[c].re + w[c].im * w[c].im;
  }
  block_allreduce2(ref, dummy, sh);
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = chi; j < m * k; j += m) {
      const z64* u = PJ + (size_t)j * nagg;
      double re = 0, im = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int i = threadIdx.x + kThreads * c;
        if (i < nagg) {
          const z64 a = u[i];
          re += a.re * w[c].re + a.im * w[c].im;
          im += a.re * w[c].im - a.im * w[c].re;
        }
      }
      block_allreduce2(re, im, sh);
      const z64 proj = mk(re, im);
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const int i = threadIdx.x + kThreads * c;
        if (i < nagg) w[c] = w[c] - proj * u[i];
      }
    }
  }
  double nrm = 0;
#pragma unroll
  for (int c = 0; c < NCH; ++c) nrm += w[c].re * w[c].re + w[c].im * w[c].im;
  block_allreduce2(nrm, dummy, sh);
  nrm = sqrt(nrm);
  ref = sqrt(ref);
  if (!(nrm > 1e-12 * ref)) {
    if (threadIdx.x == 0) fail[0] = 1;
    nrm = 1.0;
  }
  const double inv = 1.0 / nrm;
  z64* out = PJ + (size_t)(m * k + chi) * nagg;
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const int i = threadIdx.x + kThreads * c;
    if (i < nagg) out[i] = inv * w[c];
  }
}

// ---------------------------------------------------------------------------
// Galerkin build by colouring.  Aggregates of one colour are at least three
// blocks apart (with wrap-around), so A applied to the sum of their k-th
// columns never mixes two of them on any aggregate: restricting that image to
// aggregate K gives column k of the link block L_{K, J-K} for the unique J of the
// colour within K's 3x3 box.  colour(j) = j mod 3 on the first 3*floor(c/3)
// blocks of an extent c, and a colour of its own for each remaining block.
// ---------------------------------------------------------------------------
__host__ __device__ inline int color_of(int j, int c) {
  if (c < 3) return j;
  const int base = 3 * (c / 3);
  return j < base ? j % 3 : 3 + (j - base);
}

// Offset d in {0,-1,+1} of the block of colour `col` next to block j (extent c),
// or 2 if there is none.  For c <= 2 several offsets name the same block; the
// first one found receives the whole coupling and the apply sums them.
__device__ inline int pick_offset(int j, int c, int col) {
  const int ds[3] = {0, -1, 1};
  for (int q = 0; q < 3; ++q) {
    int n = j + ds[q];
    n = n < 0 ? n + c : (n >= c ? n - c : n);
    if (color_of(n, c) == col) return ds[q];
  }
  return 2;
}

// X = sum over aggregates J of colour (cxc, ctc) of column k of P (window halo h).
// Windows of one colour are disjoint, so each fine variable takes at most one value.
__global__ void k_color_scatter(const z64* __restrict__ P, z64* __restrict__ X, int lx, int lt, int dof, int bx,
                                int bt, int h, int k, int ldk, int cxc, int ctc) {
  const size_t n = (size_t)lx * lt * dof;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int site = (int)(idx / dof), d = (int)(idx - (size_t)site * dof);
  const int t = site / lx, x = site - t * lx;
  const int cx = lx / bx, ct = lt / bt;
  const int wxw = bx + 2 * h;
  const int nw = wxw * (bt + 2 * h) * dof;
  z64 val = mk(0.0, 0.0);
  bool done = false;
  for (int qt = -h; qt <= h && !done; ++qt) {
    const int jt = (t / bt + qt + ct) % ct;
    int ot;
    if (color_of(jt, ct) != ctc || !win_offset(t, jt, bt, lt, h, ot)) continue;
    for (int qx = -h; qx <= h && !done; ++qx) {
      const int jx = (x / bx + qx + cx) % cx;
      int ox;
      if (color_of(jx, cx) != cxc || !win_offset(x, jx, bx, lx, h, ox)) continue;
      val = P[((size_t)(jt * cx + jx) * ldk + k) * nw + ((ot + h) * wxw + (ox + h)) * dof + d];
      done = true;
    }
  }
  X[idx] = val;
}

template <int NCH>
__global__ void __launch_bounds__(kThreads) k_color_project(const z64* __restrict__ P, const z64* __restrict__ Y,
                                                            z64* __restrict__ L, int lx, int lt, int dof, int bx,
                                                            int bt, int h, int nc, int ldk, int k, int cxc, int ctc) {
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int K = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (K >= nK) return;
  const int Kt = K / cx, Kx = K - Kt * cx;
  const int dx = pick_offset(Kx, cx, cxc), dt = pick_offset(Kt, ct, ctc);
  if (dx == 2 || dt == 2) return;
  const int D = (dt + 1) * 3 + (dx + 1);
  const size_t n = (size_t)nK * nc;
  // L[D][k][K][row]: row stride 1, so out = &L[D][k][K][0]
  restrict_one<double, NCH>(P, Y, K, lx, lt, dof, bx, bt, cx, h, nc, ldk,
                            L + ((size_t)D * nc + k) * n + (size_t)K * nc, 1);
}

// Smoothed aggregation: column k of P = (I - w A) P_t on the windows of colour
// (cxc, ctc), from X = the tentative columns of that colour and Y = A X.
__global__ void k_sa_extract(const z64* __restrict__ X, const z64* __restrict__ Y, z64* __restrict__ P, int lx,
                             int lt, int dof, int bx, int bt, int k, int ldk, int cxc, int ctc, double w) {
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int nw = (bx + 2) * (bt + 2) * dof;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)nK * nw) return;
  const int J = (int)(idx / nw), i = (int)(idx - (size_t)J * nw);
  const int Jt = J / cx, Jx = J - Jt * cx;
  if (color_of(Jx, cx) != cxc || color_of(Jt, ct) != ctc) return;
  const int f = win_index(J, i, lx, lt, dof, bx, bt, cx, 1);
  P[((size_t)J * ldk + k) * nw + i] = X[f] - w * Y[f];
}

// ---------------------------------------------------------------------------
// Dense coarsest operator and its inverse by Gauss-Jordan elimination (FP64).
// A^(L) is Hermitian positive definite, so no pivoting is needed.
// ---------------------------------------------------------------------------
__global__ void k_coarse_to_dense(const z64* __restrict__ L, z64* __restrict__ M, int cx, int ct, int nc) {
  const int nK = cx * ct;
  const size_t n = (size_t)nK * nc;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
  const int K = i / nc, row = i - K * nc, Kn = j / nc, col = j - Kn * nc;
  const int Kt = K / cx, Kx = K - Kt * cx;
  z64 acc = mk(0.0, 0.0);
  for (int D = 0; D < 9; ++D) {
    const int dt = D / 3 - 1, dx = D % 3 - 1;
    int nx = Kx + dx, nt = Kt + dt;
    nx = nx < 0 ? nx + cx : (nx >= cx ? nx - cx : nx);
    nt = nt < 0 ? nt + ct : (nt >= ct ? nt - ct : nt);
    if (nt * cx + nx == Kn) acc = acc + L[((size_t)D * nc + col) * n + (size_t)K * nc + row];
  }
  M[idx] = acc;
}

// Step k, part 1: save column k, record the pivot, scale row k.
__global__ void k_gj_pivot(z64* __restrict__ M, int n, int k, z64* __restrict__ colk, double* __restrict__ piv,
                           int* __restrict__ fail) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double p = M[(size_t)k * n + k].re;
  if (j == 0) {
    piv[0] = p;
    if (!(p > 0) || !isfinite(p)) fail[0] = 1;
  }
  colk[j] = M[(size_t)j * n + k];
  if (j != k) M[(size_t)k * n + j] = (1.0 / p) * M[(size_t)k * n + j];
}

// Step k, part 2: eliminate column k from every other row.
__global__ void k_gj_update(z64* __restrict__ M, int n, int k, const z64* __restrict__ colk,
                            const double* __restrict__ piv) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)n * n) return;
  const int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
  const double p = piv[0];
  if (i == k) {
    if (j == k) M[idx] = mk(1.0 / p, 0.0);
    return;
  }
  if (j == k) {
    M[idx] = (-1.0 / p) * colk[i];
  } else {
    M[idx] = M[idx] - colk[i] * M[(size_t)k * n + j];
  }
}

// ---------------------------------------------------------------------------
// Utilities.
// ---------------------------------------------------------------------------
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Complex Gaussian with Re, Im ~ N(0, 1/2): Box-Muller on two counter-based uniforms.
__global__ void k_random_gaussian(z64* __restrict__ v, size_t n, uint64_t seed, uint64_t sid) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = splitmix64(seed ^ splitmix64(sid));
  const uint64_t a = splitmix64(key + 2 * i), b = splitmix64(key + 2 * i + 1);
  const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740992.0);  // (0, 1]
  const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
  const double r = sqrt(-log(u1));
  double s, c;
  sincospi(2.0 * u2, &s, &c);
  v[i] = mk(r * c, r * s);
}

__global__ void k_links_export(const z64* __restrict__ L, z64* __restrict__ out, int nK, int nc) {
  const size_t total = (size_t)nK * 9 * nc * nc;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  // out index = ((K*9 + D)*nc + row)*nc + col
  const int col = (int)(idx % nc);
  size_t r = idx / nc;
  const int row = (int)(r % nc);
  r /= nc;
  const int D = (int)(r % 9);
  const int K = (int)(r / 9);
  const size_t n = (size_t)nK * nc;
  out[idx] = L[((size_t)D * nc + col) * n + (size_t)K * nc + row];
}

// out = a X + b Y + c Z elementwise over complex arrays (real coefficients): the
// coarse links of a mass from the mass coefficients, and those coefficients from
// the links at three masses.  In place is allowed (out equal to X, Y or Z).
__global__ void k_lincomb3(const z64* X, const z64* Y, const z64* Z, z64* out, double a, double b, double c,
                           size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const z64 x = X[i], y = Y[i], z = Z[i];
    out[i] = mk(fma(c, z.re, fma(b, y.re, a * x.re)), fma(c, z.im, fma(b, y.im, a * x.im)));
  }
}

template <typename Ro>
__global__ void k_copy_convert(const z64* __restrict__ in, cpx<Ro>* __restrict__ out, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = cvt<Ro>(in[i]);
}

// Dispatch on the number of 64-lane (or 256-thread) chunks covering an aggregate.
template <typename F>
void dispatch_chunks(int chunks, F&& f) {
  if (chunks <= 1) f(IntC<1>{});
  else if (chunks <= 2) f(IntC<2>{});
  else if (chunks <= 3) f(IntC<3>{});
  else if (chunks <= 4) f(IntC<4>{});
  else if (chunks <= 8) f(IntC<8>{});
  else if (chunks <= 16) f(IntC<16>{});
  else throw Error(-1, "aggregate too large (more than 1024 variables)");
}

}  // namespace

int colors_along(int extent) { return extent < 3 ? extent : 3 + (extent - 3 * (extent / 3)); }

template <typename R, typename TP, typename TX>
void launch_restrict_t(const TP* P, R ps, const TX* x, cpx<R>* y, int lx, int lt, int dof, int bx, int bt, int h,
                       int nc, int ldk, int nrhs, hipStream_t st, const Grp& grp = Grp{}) {
  const int nK = (lx / bx) * (lt / bt);
  const int nw = (bx + 2 * h) * (bt + 2 * h) * dof;
  if constexpr (std::is_same<R, float>::value) {
    // one wavefront per aggregate while its P rows fit in registers (at most 64 words)
    const int nch = (nw + 63) / 64, ncol = nc <= 4 ? 4 : nc <= 8 ? 8 : 16;
    if (nc <= 16 && nch <= 2 && ncol * nch * (int)(sizeof(TP) / 4) <= 64) {
      // eight right-hand sides per wavefront share its P rows once there are that many
      // (grouped: one per wavefront, each column its own P)
      const int nrb = nrhs >= 8 && !grp.op ? 8 : 1;
      dim3 g((nK + kThreads / 64 - 1) / (kThreads / 64), (nrhs + nrb - 1) / nrb);
      auto go = [&](auto ncl, auto ch) {
        if (nrb == 8)
          hipLaunchKernelGGL((k_restrict_bf<decltype(ncl)::v, decltype(ch)::v, TX, TP, 8>), g, dim3(kThreads), 0, st,
                             P, x, y, lx, lt, dof, bx, bt, h, nc, ldk, ps, nrhs, Grp{});
        else
          hipLaunchKernelGGL((k_restrict_bf<decltype(ncl)::v, decltype(ch)::v, TX, TP, 1>), g, dim3(kThreads), 0, st,
                             P, x, y, lx, lt, dof, bx, bt, h, nc, ldk, ps, nrhs, grp);
      };
      auto by_ch = [&](auto ncl) {
        if (nch == 1) go(ncl, IntC<1>{});
        else go(ncl, IntC<2>{});
      };
      if (ncol == 4) by_ch(IntC<4>{});
      else if (ncol == 8) by_ch(IntC<8>{});
      else by_ch(IntC<16>{});
      HIPCHECK(hipGetLastError());
      return;
    }
    // one workgroup per aggregate, the chunks spread over its four wavefronts
    const int cpw = (nch + kThreads / 64 - 1) / (kThreads / 64);
    if (nc <= 16 && cpw <= 3 && ncol * cpw * (int)(sizeof(TP) / 4) <= 64) {
      // four right-hand sides per workgroup share its P rows once there are that many
      const int nrb = nrhs >= 4 && !grp.op ? 4 : 1;
      dim3 g(nK, (nrhs + nrb - 1) / nrb);
      auto go = [&](auto ncl, auto cw) {
        if (nrb == 4)
          hipLaunchKernelGGL((k_restrict_bfw<decltype(ncl)::v, decltype(cw)::v, TX, TP, 4>), g, dim3(kThreads), 0, st,
                             P, x, y, lx, lt, dof, bx, bt, h, nc, ldk, ps, nrhs, Grp{});
        else
          hipLaunchKernelGGL((k_restrict_bfw<decltype(ncl)::v, decltype(cw)::v, TX, TP, 1>), g, dim3(kThreads), 0, st,
                             P, x, y, lx, lt, dof, bx, bt, h, nc, ldk, ps, nrhs, grp);
      };
      auto by_cw = [&](auto ncl) {
        if (cpw == 1) go(ncl, IntC<1>{});
        else if (cpw == 2) go(ncl, IntC<2>{});
        else go(ncl, IntC<3>{});
      };
      if (ncol == 4) by_cw(IntC<4>{});
      else if (ncol == 8) by_cw(IntC<8>{});
      else by_cw(IntC<16>{});
      HIPCHECK(hipGetLastError());
      return;
    }
  }
  if (grp.op) throw Error(-1, "grouped restriction needs the one-wavefront or one-workgroup kernel");
  dim3 grid(nK, nrhs);
  dispatch_chunks((nw + 63) / 64, [&](auto c) {
    launch_restrict_kw<R, decltype(c)::v, TX, TP>(grid, st, P, ps, x, y, lx, lt, dof, bx, bt, h, nc, ldk, nrhs);
  });
  HIPCHECK(hipGetLastError());
}

// FP64 restriction of many right-hand sides on the matrix cores (V-cycle step 2):
// per aggregate K, Y_K = P_K^H X_K with X_K the nw window variables of each
// right-hand side, a (nc x nw) x (nw x nrhs) product.  One wave owns one aggregate
// and 16 RT right-hand sides; K-step s takes window variables 4s..4s+3 through
// v_mfma_f64_16x16x4f64 (layout of k_coarse_mfma64), the conjugate transpose in the
// real embedding: Pr Xr + Pi Xi into Re Y, Pr Xi - Pi Xr into Im Y.  P_K is read
// once per 16 RT columns instead of once per column group of the vector-ALU kernel;
// the next step's operands are loaded while this step's instructions run.
template <int RT>
__global__ void __launch_bounds__(256) k_restrict_mfma64(const z64* __restrict__ P, const z64* __restrict__ x,
                                                         z64* __restrict__ y, int lx, int lt, int dof, int bx, int bt,
                                                         int h, int nc, int ldk, int nrhs) {
  const int cx = lx / bx, ct = lt / bt, nK = cx * ct;
  const int K = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K >= nK) return;  // wave-uniform, and no barrier follows
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const size_t n = (size_t)lx * lt * dof;
  const int nw = (bx + 2 * h) * (bt + 2 * h) * dof;
  const int rhs0 = blockIdx.y * 16 * RT;
  const z64* PK = P + (size_t)K * ldk * nw + (size_t)(i < nc ? i : nc - 1) * nw;
  const bool row_ok = i < nc;
  int rj[RT];
  bool rj_ok[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int r = rhs0 + 16 * rt + i;
    rj_ok[rt] = r < nrhs;
    rj[rt] = r < nrhs ? r : nrhs - 1;
  }
  auto load = [&](int st, double& pr, double& pi, z64 (&xv)[RT]) {
    const int w = 4 * st + kq;
    const bool wok = w < nw;
    const int wc = wok ? w : nw - 1;
    const z64 pv = PK[wc];
    pr = (row_ok && wok) ? pv.re : 0.0;
    pi = (row_ok && wok) ? pv.im : 0.0;
    const int wi = win_index(K, wc, lx, lt, dof, bx, bt, cx, h);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const z64 u = x[(size_t)rj[rt] * n + wi];
      const bool ok = rj_ok[rt] && wok;
      xv[rt] = mk<double>(ok ? u.re : 0.0, ok ? u.im : 0.0);
    }
  };
  doublex4 accR[RT], accI[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) accR[rt][r] = accI[rt][r] = 0.0;
  const int steps = (nw + 3) / 4;
  double pr, pi, pr2, pi2;
  z64 xv[RT], xv2[RT];
  load(0, pr, pi, xv);
  for (int st = 0; st < steps; ++st) {
    if (st + 1 < steps) load(st + 1, pr2, pi2, xv2);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      accR[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, xv[rt].re, accR[rt], 0, 0, 0);
      accI[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, xv[rt].im, accI[rt], 0, 0, 0);
      accR[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(pi, xv[rt].im, accR[rt], 0, 0, 0);
      accI[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-pi, xv[rt].re, accI[rt], 0, 0, 0);
    }
    pr = pr2;
    pi = pi2;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) xv[rt] = xv2[rt];
  }
  // lane holds right-hand side rhs0 + 16 rt + i, coarse variables 4 r + kq
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    if (!rj_ok[rt]) continue;
    z64* yr = y + ((size_t)rj[rt] * nK + K) * nc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * r + kq;
      if (k < nc) yr[k] = mk<double>(accR[rt][r], accI[rt][r]);
    }
  }
}

void launch_restrict_mfma64(const z64* P, const z64* x, z64* y, int lx, int lt, int dof, int bx, int bt, int h,
                            int nc, int ldk, int nrhs, hipStream_t st) {
  if (nc < 1 || nc > 16) throw Error(-1, "FP64 matrix-core restriction needs 1 <= nc <= 16");
  if (nrhs < 1) return;
  const int nK = (lx / bx) * (lt / bt);
  const int rt = nrhs <= 16 ? 1 : (nrhs <= 32 ? 2 : 4);
  const dim3 grid((unsigned)((nK + 3) / 4), (unsigned)((nrhs + 16 * rt - 1) / (16 * rt)));
  if (rt == 1)
    hipLaunchKernelGGL((k_restrict_mfma64<1>), grid, dim3(256), 0, st, P, x, y, lx, lt, dof, bx, bt, h, nc, ldk, nrhs);
  else if (rt == 2)
    hipLaunchKernelGGL((k_restrict_mfma64<2>), grid, dim3(256), 0, st, P, x, y, lx, lt, dof, bx, bt, h, nc, ldk, nrhs);
  else
    hipLaunchKernelGGL((k_restrict_mfma64<4>), grid, dim3(256), 0, st, P, x, y, lx, lt, dof, bx, bt, h, nc, ldk, nrhs);
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_restrict(const cpx<R>* P, const cpx<R>* x, cpx<R>* y, int lx, int lt, int dof, int bx, int bt, int h,
                     int nc, int ldk, int nrhs, hipStream_t st) {
  launch_restrict_t<R, cpx<R>, cpx<R>>(P, (R)1, x, y, lx, lt, dof, bx, bt, h, nc, ldk, nrhs, st);
}

template <typename TP, typename TI>
void launch_restrict_s(const TP* P, float ps, const TI* x, z32* y, int lx, int lt, int dof, int bx, int bt, int h,
                       int nc, int ldk, int nrhs, hipStream_t st, const Grp& g) {
  launch_restrict_t<float, TP, TI>(P, ps, x, y, lx, lt, dof, bx, bt, h, nc, ldk, nrhs, st, g);
}
#define INST_RS(TP, TI)                                                                                         \
  template void launch_restrict_s<TP, TI>(const TP*, float, const TI*, z32*, int, int, int, int, int, int, int, \
                                          int, int, hipStream_t, const Grp&);
INST_RS(z32, z32)
INST_RS(z32, bfc)
INST_RS(z32, hfc)
INST_RS(hfc, z32)
INST_RS(hfc, bfc)
INST_RS(hfc, hfc)
#undef INST_RS

// Phase 1 of the FP64 prolongation of many right-hand sides on the matrix cores:
// per aggregate K, W_K = P_K E_K (nw x nc times nc x nrhs).  One wave owns 16 window
// variables of one aggregate and 16 RT right-hand sides; K-step s takes coarse
// variables 4s..4s+3 through v_mfma_f64_16x16x4f64 (layout of k_coarse_mfma64):
// Pr Er - Pi Ei into Re W, Pr Ei + Pi Er into Im W.  W has the layout of
// k_prolong_win's, so the gather phase is shared.
template <int RT>
__global__ void __launch_bounds__(256) k_prolong_win_mfma64(const z64* __restrict__ P, const z64* __restrict__ e,
                                                            z64* __restrict__ wbuf, int nK, int nw, int nc, int ldk,
                                                            int nrhs) {
  const int ntile = (nw + 15) / 16;
  const int g = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= nK * ntile) return;  // wave-uniform, and no barrier follows
  const int K = g / ntile, tile = g - K * ntile;
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const int w = 16 * tile + i;
  const bool w_ok = w < nw;
  const z64* PK = P + (size_t)K * ldk * nw + (w_ok ? w : nw - 1);
  const int rhs0 = blockIdx.y * 16 * RT;
  int rj[RT];
  bool rj_ok[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int r = rhs0 + 16 * rt + i;
    rj_ok[rt] = r < nrhs;
    rj[rt] = r < nrhs ? r : nrhs - 1;
  }
  doublex4 accR[RT], accI[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) accR[rt][r] = accI[rt][r] = 0.0;
  for (int s = 0; s < (nc + 3) / 4; ++s) {
    const int k = 4 * s + kq;
    const bool k_ok = k < nc;
    const int kc = k_ok ? k : nc - 1;
    const z64 pv = PK[(size_t)kc * nw];
    const double pr = (w_ok && k_ok) ? pv.re : 0.0, pi = (w_ok && k_ok) ? pv.im : 0.0;
    z64 ev[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const z64 u = e[((size_t)rj[rt] * nK + K) * nc + kc];
      const bool ok = rj_ok[rt] && k_ok;
      ev[rt] = mk<double>(ok ? u.re : 0.0, ok ? u.im : 0.0);
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      accR[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, ev[rt].re, accR[rt], 0, 0, 0);
      accI[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(pr, ev[rt].im, accI[rt], 0, 0, 0);
      accR[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-pi, ev[rt].im, accR[rt], 0, 0, 0);
      accI[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(pi, ev[rt].re, accI[rt], 0, 0, 0);
    }
  }
  // lane holds right-hand side rhs0 + 16 rt + i, window variables 16 tile + 4 r + kq
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    if (!rj_ok[rt]) continue;
    z64* wr = wbuf + ((size_t)rj[rt] * nK + K) * nw;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int wv = 16 * tile + 4 * r + kq;
      if (wv < nw) wr[wv] = mk<double>(accR[rt][r], accI[rt][r]);
    }
  }
}

template <typename R, typename TP>
void launch_prolong_t(const TP* P, R ps, const cpx<R>* e, cpx<R>* y, cpx<R>* wbuf, int lx, int lt, int dof, int bx,
                      int bt, int h, int nc, int ldk, int nrhs, int mode, hipStream_t st, bool mfma = false,
                      const Grp& grp = Grp{}) {
  const int nK = (lx / bx) * (lt / bt);
  const int nw = (bx + 2 * h) * (bt + 2 * h) * dof;
  const size_t nkw = (size_t)nK * nw;
  bool win_done = false;
  if constexpr (std::is_same<R, double>::value && std::is_same<TP, z64>::value) {
    if (mfma) {  // FP64, many right-hand sides: phase 1 on the matrix cores
      if (nc < 1 || nc > 16) throw Error(-1, "FP64 matrix-core prolongation needs 1 <= nc <= 16");
      const int rt = nrhs <= 16 ? 1 : (nrhs <= 32 ? 2 : 4);
      const long waves = (long)nK * ((nw + 15) / 16);
      const dim3 g((unsigned)((waves + 3) / 4), (unsigned)((nrhs + 16 * rt - 1) / (16 * rt)));
      if (rt == 1)
        hipLaunchKernelGGL((k_prolong_win_mfma64<1>), g, dim3(256), 0, st, P, e, wbuf, nK, nw, nc, ldk, nrhs);
      else if (rt == 2)
        hipLaunchKernelGGL((k_prolong_win_mfma64<2>), g, dim3(256), 0, st, P, e, wbuf, nK, nw, nc, ldk, nrhs);
      else
        hipLaunchKernelGGL((k_prolong_win_mfma64<4>), g, dim3(256), 0, st, P, e, wbuf, nK, nw, nc, ldk, nrhs);
      win_done = true;
    }
  }
  if (win_done) {
  } else if (nrhs >= 8 && !grp.op) {  // eight right-hand sides per thread share its P entries
    hipLaunchKernelGGL((k_prolong_win<R, TP, 8>), dim3((unsigned)((nkw + kThreads - 1) / kThreads), (nrhs + 7) / 8),
                       dim3(kThreads), 0, st, P, e, wbuf, nK, nw, nc, ldk, ps, nrhs, Grp{});
  } else {  // one right-hand side per thread (grouped: each column its own P)
    hipLaunchKernelGGL((k_prolong_win<R, TP, 1>), dim3((unsigned)((nkw + kThreads - 1) / kThreads), nrhs),
                       dim3(kThreads), 0, st, P, e, wbuf, nK, nw, nc, ldk, ps, nrhs, grp);
  }
  const size_t total = (size_t)lx * lt * dof;
  dim3 grid((unsigned)((total + kThreads - 1) / kThreads), nrhs);
  // h = 1 needs both coarse extents >= 2 (then no window covers a site twice) and blocks
  // of at least 2 sites along each axis (the first and last site of a block differ)
  const bool fast = h == 0 || (h == 1 && lx / bx >= 2 && lt / bt >= 2 && bx >= 2 && bt >= 2);
  auto go = [&](auto md, auto hh) {
    constexpr int M = decltype(md)::v, HH = decltype(hh)::v;
    if (fast)
      hipLaunchKernelGGL((k_prolong_gather_f<R, M, HH>), grid, dim3(kThreads), 0, st, wbuf, y, lx, lt, dof, bx, bt);
    else
      hipLaunchKernelGGL((k_prolong_gather<R, M>), grid, dim3(kThreads), 0, st, wbuf, y, lx, lt, dof, bx, bt, h);
  };
  auto by_h = [&](auto md) {
    if (h == 0) go(md, IntC<0>{});
    else go(md, IntC<1>{});
  };
  if (mode == 0) by_h(IntC<0>{});
  else by_h(IntC<1>{});
  HIPCHECK(hipGetLastError());
}

template <typename R>
void launch_prolong(const cpx<R>* P, const cpx<R>* e, cpx<R>* y, cpx<R>* wbuf, int lx, int lt, int dof, int bx,
                    int bt, int h, int nc, int ldk, int nrhs, int mode, hipStream_t st, bool mfma, const Grp& g) {
  launch_prolong_t<R, cpx<R>>(P, (R)1, e, y, wbuf, lx, lt, dof, bx, bt, h, nc, ldk, nrhs, mode, st, mfma, g);
}

void launch_prolong_h16(const hfc* P, float ps, const z32* e, z32* y, z32* wbuf, int lx, int lt, int dof, int bx,
                        int bt, int h, int nc, int ldk, int nrhs, int mode, hipStream_t st, const Grp& g) {
  launch_prolong_t<float, hfc>(P, ps, e, y, wbuf, lx, lt, dof, bx, bt, h, nc, ldk, nrhs, mode, st, false, g);
}

template <typename R, int NR, int Q, typename TL>
void launch_coarse_q(const TL* L, R lscale, const cpx<R>* x, cpx<R>* y, int cx, int ct, int nc, int nrhs, int mode,
                     double c, double c2, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st) {
  const size_t total = (size_t)cx * ct * nc;
  dim3 grid((unsigned)((total + 63) / 64), (nrhs + NR - 1) / NR);
  with_mode(mode, [&](auto m) {
    hipLaunchKernelGGL((k_coarse<R, decltype(m)::v, NR, Q, TL>), grid, dim3(kThreads), 0, st, L, x, y, cx, ct, nc,
                       nrhs, (R)c, (R)c2, xacc, aux, lscale);
  });
  HIPCHECK(hipGetLastError());
}

// Columns per pass: a wave's share of the columns (ceil(nc / 4)) in one pass up to
// 4, in passes of 4 above.
template <typename R, int NR, typename TL>
void launch_coarse_nr(const TL* L, R lscale, const cpx<R>* x, cpx<R>* y, int cx, int ct, int nc, int nrhs, int mode,
                      double c, double c2, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st) {
  const int q = (nc + 3) / 4;
  if (q <= 2)
    launch_coarse_q<R, NR, 2, TL>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
  else if (q == 3)
    launch_coarse_q<R, NR, 3, TL>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
  else
    launch_coarse_q<R, NR, 4, TL>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
}

// ---------------------------------------------------------------------------
// Multi-RHS FP32 coarse operator on the matrix cores (Eq. 2 applied to 32
// right-hand sides at once).  For one coarse site K and one link direction D the
// complex product Y += L_{K,D} V_{K+D} (nc x nc times nc x 32) is the real GEMM
//   [Yr; Yi] += [[Lr, -Li], [Li, Lr]] [Vr; Vi]      (rows and K index padded to 32)
// done with v_mfma_f32_32x32x2f32: each instruction takes two link columns c, c+1
// (one per half-wave) against the matching rows of V; the Re half of the K index
// pairs Lr|Li with Vr, the Im half pairs -Li|Lr with Vi.  Per site that is
// 9 * 2 * ceil(nc/2) instructions of 4096 flops.  Lane layout (checked on the
// device): A[i][k] from lane i + 32k, B[k][j] from lane j + 32k, and accumulator
// r of lane l holds row 8(r/4) + 4(l/32) + r%4, column l%32.
//
// V is staged per workgroup for a TX x TT tile of sites plus a one-site ring,
// transposed to [site][c][rhs] (rows padded to 33 entries against bank
// conflicts), so the B operand is one conflict-free 8-byte LDS read per lane.
// Links stream from HBM once.  Waves take the tile's sites in turn.
// ---------------------------------------------------------------------------
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kMfmaRS = 33;  // padded LDS row (32 right-hand sides + 1)

__device__ inline int xcd_tile(int b, int nb) {
  // block b runs on XCD b % 8: hand XCD k the k-th eighth of the tiles
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// TL: link storage, z32, or hfc (FP16 scaled by 1 / lscale, a power of two: the
// links widen to FP32 exactly in registers and the sums are scaled exactly at the
// end, so the arithmetic is FP32 in both cases and the link stream is halved).
template <int MODE, int TX, int TT, int NW, int S, typename TL = z32>
__global__ void __launch_bounds__(NW * 64) k_coarse_mfma(const TL* __restrict__ L, const z32* __restrict__ v,
                                                        z32* __restrict__ y, int cx, int ct, int nc, int nrhs,
                                                        float c, float c2, z32* __restrict__ xacc,
                                                        const z32* __restrict__ aux, int pairs, float lscale) {
  // S = ceil(nc / 2): MFMA pairs per link direction and staged column pairs.  It is
  // a compile-time constant so that the loads below are straight-line code (loads
  // under branches make the compiler drain every outstanding load before an MFMA).
  constexpr int HX = TX + 2, HT = TT + 2, NS = HX * HT;
  constexpr int NT = NW * 64;
  __shared__ float2 vs[NS * 16 * kMfmaRS];
  const int nK = cx * ct;
  const size_t n = (size_t)nK * nc;
  const int rhs0 = blockIdx.y * 32;
  const int ntx = (cx + TX - 1) / TX;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % ntx) * TX, t0 = (tile / ntx) * TT;

  // ---- stage V (tile + ring) as [site][c][rhs]: item = (rhs, row, site in row, column pair),
  // consecutive items are consecutive 16-byte pairs of one right-hand side's row.  Out of
  // range items load a clamped (valid) address and are masked afterwards.
  {
    constexpr int U = 18;  // loads in flight per thread (a 4x4 tile of 16 columns: all of them)
    constexpr int items = 32 * NS * S;
    const int jmax = nrhs - rhs0 - 1;
    for (int base = threadIdx.x; base < items; base += NT * U) {
      float4 buf[U];
      int dst[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e0 = base + u * NT;
        const int e = e0 < items ? e0 : items - 1;
        const int pr = e % S;
        const int rest = e / S;
        const int site = rest % NS, j = rest / NS;
        const int ht = site / HX, hx = site - ht * HX;
        // periodic wrap; the ring of a ragged tile may reach past one period when an
        // extent is smaller than the tile
        const int gx = ((x0 + hx - 1) % cx + cx) % cx, gt = ((t0 + ht - 1) % ct + ct) % ct;
        const int jc = j <= jmax ? j : jmax;
        const z32* src = v + (size_t)(rhs0 + jc) * n + (size_t)(gt * cx + gx) * nc;
        float4 t;
        if (pairs) {
          t = *reinterpret_cast<const float4*>(src + 2 * pr);
        } else {
          const z32 a0 = src[2 * pr];
          const z32 a1 = src[min(2 * pr + 1, nc - 1)];
          t = make_float4(a0.re, a0.im, a1.re, a1.im);
        }
        const bool live = j <= jmax;
        const bool hi_ok = live && (2 * pr + 1 < nc);
        buf[u] = make_float4(live ? t.x : 0.f, live ? t.y : 0.f, hi_ok ? t.z : 0.f, hi_ok ? t.w : 0.f);
        dst[u] = e0 < items ? (site * 16 + 2 * pr) * kMfmaRS + j : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (dst[u] < 0) continue;
        vs[dst[u]] = make_float2(buf[u].x, buf[u].y);
        vs[dst[u] + kMfmaRS] = make_float2(buf[u].z, buf[u].w);
      }
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 31, h = lane >> 5;
  const int row = i & 15;
  const bool upper = i >= 16;
  const int rowc = row < nc ? row : nc - 1;  // clamped: every lane loads a valid address
  const bool row_ok = row < nc;
  // this wave's sites: valid sites of the tile, round robin over the waves
  const int vx = min(TX, cx - x0), vt = min(TT, ct - t0);
  const int nvalid = vx * vt;
  const int mine = nvalid > w ? (nvalid - w + NW - 1) / NW : 0;
  if (mine == 0) return;  // wave-uniform, and no barrier follows
  auto load_links = [&](int k, int D, TL* dst) {
    const int idx = w + k * NW;
    const int ox = idx % vx, ot = idx / vx;
    const TL* LD = L + (size_t)D * nc * n + (size_t)((t0 + ot) * cx + x0 + ox) * nc + rowc;
#pragma unroll
    for (int sp = 0; sp < S; ++sp) {
      const int cc = 2 * sp + h;
      dst[sp] = LD[(size_t)(cc < nc ? cc : nc - 1) * n];  // masked where used, not here
    }
  };
  // Links stream through a ring of three link directions held in registers, two
  // ahead of the MFMAs (occupancy is set by the LDS tile, so registers are free).
  // The sites of a wave and their nine directions are unrolled and their results
  // stay in registers until every site is done: the loop is straight-line code
  // with compile-time ring slots and no stores, so the compiler can wait for
  // exactly the loads each step needs.
  constexpr int MAXS = (TX * TT + NW - 1) / NW;
  const int last = 9 * mine - 1;
  auto load_step = [&](int q, TL* dst) {
    q = min(q, last);
    load_links(q / 9, q - 9 * (q / 9), dst);
  };
  TL lb[3][S];
  load_step(0, lb[0]);
  load_step(1, lb[1]);
  load_step(2, lb[2]);
  floatx16 acc[MAXS];
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
    if (k >= mine) continue;  // wave-uniform
    const int idx = w + k * NW;
    const int ox = idx % vx, ot = idx / vx;
    // B operands of direction D, read one direction ahead (their LDS round trip runs
    // under the previous direction's MFMAs)
    auto read_b = [&](int D, float2* bo) {
      const int dt = D / 3 - 1, dx = D % 3 - 1;
      const int ls = (ot + 1 + dt) * HX + (ox + 1 + dx);
      const float2* VB = vs + (size_t)ls * 16 * kMfmaRS + i;
#pragma unroll
      for (int sp = 0; sp < S; ++sp) bo[sp] = VB[(2 * sp + h) * kMfmaRS];
    };
    float2 b[2][S];
    read_b(0, b[0]);
#pragma unroll
    for (int D = 0; D < 9; ++D) {
      if (D + 1 < 9) read_b(D + 1, b[(D + 1) % 2]);
#pragma unroll
      for (int sp = 0; sp < S; ++sp) {
        const z32 l = widen(lb[D % 3][sp]);
        const bool ok = row_ok && (2 * sp + h < nc);
        const float a_re = ok ? (upper ? l.im : l.re) : 0.f;
        const float a_im = ok ? (upper ? l.re : -l.im) : 0.f;
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_re, b[D % 2][sp].x, acc[k], 0, 0, 0);
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_im, b[D % 2][sp].y, acc[k], 0, 0, 0);
      }
      load_step(9 * k + D + 3, lb[D % 3]);  // refill the slot just consumed
      // keep the refill here: the scheduler would otherwise sink it next to its use
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // ---- epilogue: lane holds rhs j = i, dofs 8(r/4) + 4h + r%4 (Re in r, Im in r + 8)
  const int j = i;
  if (rhs0 + j >= nrhs) return;
#pragma unroll
  for (int k = 0; k < MAXS; ++k) {
    if (k >= mine) break;
    const int idx = w + k * NW;
    const int ox = idx % vx, ot = idx / vx;
    const size_t ob = (size_t)(rhs0 + j) * n + (size_t)((t0 + ot) * cx + x0 + ox) * nc;
    const int lsc = (ot + 1) * HX + (ox + 1);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int dof = 8 * (r >> 2) + 4 * h + (r & 3);
      if (dof >= nc) continue;
      const z32 sum = lscale * mk<float>(acc[k][r], acc[k][r + 8]);  // exact: a power of two
      const size_t o = ob + dof;
      if (MODE == 0) {
        y[o] = sum;
      } else if (MODE == 1 || MODE == 3) {
        const float2 t = vs[(lsc * 16 + dof) * kMfmaRS + j];
        const z32 vi = mk<float>(t.x, t.y);
        xacc[o] = MODE == 3 ? c * vi : xacc[o] + c * vi;
        y[o] = vi - c * sum;
      } else if (MODE == 4 || MODE == 5) {
        const float2 t = vs[(lsc * 16 + dof) * kMfmaRS + j];
        const z32 vi = mk<float>(t.x, t.y);
        const z32 a = MODE == 5 ? c * vi : xacc[o] + c * vi;
        xacc[o] = a + c2 * (vi - c * sum);
      } else {
        y[o] = aux[o] - sum;
      }
    }
  }
}

// The same operator for large coarse lattices, walking down strips of rows: a
// workgroup owns a strip 4 sites wide and `seg` rows of it and keeps a rolling window
// of four rows of V (the two rows it computes and the rows above and below, 4 x 6
// sites with the ring, 101 KB of LDS) as [row slot][site][c][rhs].  Each step computes
// two rows (one site per wave) while the next two rows are requested into registers
// (24 per thread), and writes them over the two rows no longer needed between two
// barriers, so the staging of V runs under the MFMAs instead of before them.  The
// link ring continues from step to step.  A site's products, their order and the
// epilogue are those of k_coarse_mfma, so the results are bitwise the same.
constexpr int kTwRows = 2;  // rows per step

template <int MODE, int S, typename TL>
__global__ void __launch_bounds__(512) k_coarse_mfma_tw(const TL* __restrict__ L, const z32* __restrict__ v,
                                                        z32* __restrict__ y, int cx, int ct, int nc, int nrhs,
                                                        float c, float c2, z32* __restrict__ xacc,
                                                        const z32* __restrict__ aux, int pairs, float lscale,
                                                        int seg) {
  constexpr int NW = 8, TXW = 4, HX = TXW + 2, NSLOT = kTwRows + 2, NT = NW * 64;
  __shared__ float2 vs[NSLOT * HX * 16 * kMfmaRS];
  const int nK = cx * ct;
  const size_t n = (size_t)nK * nc;
  const int rhs0 = blockIdx.y * 32;
  const int ns = (cx + TXW - 1) / TXW;
  // XCD k takes a contiguous band of segments (xcd_tile), so that the strips beside a
  // strip, which read the same halo columns, run in the same L2
  const int tl = xcd_tile(blockIdx.x, gridDim.x);
  const int strip = tl % ns, segi = tl / ns;
  const int x0 = strip * TXW;
  const int r0 = segi * seg, r1 = min(ct, r0 + seg);
  const int jmax = nrhs - rhs0 - 1;
  // ---- staging of whole window rows: item = (rhs, row of the step, site in row, column
  // pair); ROWS rows are one pass of ROWS * U1 loads per thread
  constexpr int ITEMS_ROW = 32 * HX * S;
  constexpr int U1 = (ITEMS_ROW + NT - 1) / NT;  // loads per thread and row (3 for nc = 16)
  auto row_load = [&](int r, int u0, float4* buf) {  // unwrapped row r >= -1
    const int gt = ((r % ct) + ct) % ct;
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int e0 = threadIdx.x + u * NT;
      const int e = e0 < ITEMS_ROW ? e0 : ITEMS_ROW - 1;
      const int pr = e % S;
      const int rest = e / S;
      const int hx = rest % HX, j = rest / HX;
      const int gx = ((x0 + hx - 1) % cx + cx) % cx;
      const int jc = j <= jmax ? j : jmax;
      const z32* src = v + (size_t)(rhs0 + jc) * n + (size_t)(gt * cx + gx) * nc;
      float4 t;
      if (pairs) {
        t = *reinterpret_cast<const float4*>(src + 2 * pr);
      } else {
        const z32 a0 = src[2 * pr];
        const z32 a1 = src[min(2 * pr + 1, nc - 1)];
        t = make_float4(a0.re, a0.im, a1.re, a1.im);
      }
      const bool live = j <= jmax;
      const bool hi_ok = live && (2 * pr + 1 < nc);
      buf[u0 + u] = make_float4(live ? t.x : 0.f, live ? t.y : 0.f, hi_ok ? t.z : 0.f, hi_ok ? t.w : 0.f);
    }
  };
  auto row_store = [&](int r, int u0, const float4* buf) {
    const int slot = (r + NSLOT) % NSLOT;
#pragma unroll
    for (int u = 0; u < U1; ++u) {
      const int e0 = threadIdx.x + u * NT;
      if (e0 >= ITEMS_ROW) continue;
      const int pr = e0 % S;
      const int rest = e0 / S;
      const int hx = rest % HX, j = rest / HX;
      const int d = ((slot * HX + hx) * 16 + 2 * pr) * kMfmaRS + j;
      vs[d] = make_float2(buf[u0 + u].x, buf[u0 + u].y);
      vs[d + kMfmaRS] = make_float2(buf[u0 + u].z, buf[u0 + u].w);
    }
  };
  if (r0 >= ct) return;  // workgroup-uniform, before any barrier
  {  // the first window: rows r0 - 1 .. r0 + 2
    float4 fb[NSLOT * U1];
#pragma unroll
    for (int q = 0; q < NSLOT; ++q) row_load(r0 - 1 + q, q * U1, fb);
#pragma unroll
    for (int q = 0; q < NSLOT; ++q) row_store(r0 - 1 + q, q * U1, fb);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 31, h = lane >> 5;
  const int row = i & 15;
  const bool upper = i >= 16;
  const int rowc = row < nc ? row : nc - 1;  // clamped: every lane loads a valid address
  const bool row_ok = row < nc;
  const int ox = w % TXW, orow = w / TXW;  // this wave's site in every step
  const bool col_ok = x0 + ox < cx;
  const int gxs = col_ok ? x0 + ox : cx - 1;
  const int nsteps = (r1 - r0 + kTwRows - 1) / kTwRows;
  // link loads of step q / 9, direction q % 9 (rows and columns clamped to valid sites)
  auto load_step = [&](int q, TL* dst) {
    const int st = q / 9, D = q - 9 * st;
    const int gr = min(r0 + kTwRows * min(st, nsteps - 1) + orow, ct - 1);
    const TL* LD = L + (size_t)D * nc * n + (size_t)(gr * cx + gxs) * nc + rowc;
#pragma unroll
    for (int sp = 0; sp < S; ++sp) {
      const int cc = 2 * sp + h;
      dst[sp] = LD[(size_t)(cc < nc ? cc : nc - 1) * n];  // masked where used, not here
    }
  };
  TL lb[3][S];
  load_step(0, lb[0]);
  load_step(1, lb[1]);
  load_step(2, lb[2]);
  float4 nb[kTwRows * U1];
  for (int stp = 0; stp < nsteps; ++stp) {
    const int rs = r0 + kTwRows * stp;
    const bool has_next = stp + 1 < nsteps;  // uniform over the workgroup
    if (has_next) {
#pragma unroll
      for (int q = 0; q < kTwRows; ++q) row_load(rs + 2 + q + 1, q * U1, nb);  // rows rs + 3, rs + 4
    }
    __builtin_amdgcn_sched_barrier(0);
    const int trow = rs + orow;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    // B operands of direction D from the window (read one direction ahead, so that the
    // LDS round trip of the next direction runs under this direction's MFMAs)
    auto read_b = [&](int D, float2* bb) {
      const int dt = D / 3 - 1, dx = D % 3 - 1;
      const int slot = (trow + dt + NSLOT) % NSLOT;
      const float2* VB = vs + (size_t)(slot * HX + ox + 1 + dx) * 16 * kMfmaRS + i;
#pragma unroll
      for (int sp = 0; sp < S; ++sp) bb[sp] = VB[(2 * sp + h) * kMfmaRS];
    };
    float2 bb[2][S];
    read_b(0, bb[0]);
#pragma unroll
    for (int D = 0; D < 9; ++D) {
      if (D + 1 < 9) read_b(D + 1, bb[(D + 1) % 2]);
#pragma unroll
      for (int sp = 0; sp < S; ++sp) {
        const z32 l = widen(lb[D % 3][sp]);
        const bool ok = row_ok && (2 * sp + h < nc);
        const float a_re = ok ? (upper ? l.im : l.re) : 0.f;
        const float a_im = ok ? (upper ? l.re : -l.im) : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a_re, bb[D % 2][sp].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a_im, bb[D % 2][sp].y, acc, 0, 0, 0);
      }
      load_step(9 * stp + D + 3, lb[D % 3]);  // refill the slot just consumed (the next step's from D = 6)
      __builtin_amdgcn_sched_barrier(0);
    }
    // ---- epilogue: lane holds rhs j = i, dofs 8(r/4) + 4h + r%4 (Re in r, Im in r + 8)
    const int j = i;
    if (col_ok && trow < r1 && rhs0 + j < nrhs) {
      const size_t ob = (size_t)(rhs0 + j) * n + (size_t)(trow * cx + x0 + ox) * nc;
      const int lsc = ((trow + NSLOT) % NSLOT) * HX + ox + 1;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int dof = 8 * (r >> 2) + 4 * h + (r & 3);
        if (dof >= nc) continue;
        const z32 sum = lscale * mk<float>(acc[r], acc[r + 8]);  // exact: a power of two
        const size_t o = ob + dof;
        if (MODE == 0) {
          y[o] = sum;
        } else if (MODE == 1 || MODE == 3) {
          const float2 t = vs[(lsc * 16 + dof) * kMfmaRS + j];
          const z32 vi = mk<float>(t.x, t.y);
          xacc[o] = MODE == 3 ? c * vi : xacc[o] + c * vi;
          y[o] = vi - c * sum;
        } else if (MODE == 4 || MODE == 5) {
          const float2 t = vs[(lsc * 16 + dof) * kMfmaRS + j];
          const z32 vi = mk<float>(t.x, t.y);
          const z32 a = MODE == 5 ? c * vi : xacc[o] + c * vi;
          xacc[o] = a + c2 * (vi - c * sum);
        } else {
          y[o] = aux[o] - sum;
        }
      }
    }
    if (!has_next) break;
    __syncthreads();  // every wave is done with rows rs - 1 and rs
#pragma unroll
    for (int q = 0; q < kTwRows; ++q) row_store(rs + 3 + q, q * U1, nb);
    __syncthreads();
  }
}

template <int TX, int TT, int NW, int S, typename TL>
void launch_coarse_mfma_t(const TL* L, float lscale, const z32* x, z32* y, int cx, int ct, int nc, int nrhs,
                          int mode, double c, double c2, z32* xacc, const z32* aux, hipStream_t st) {
  const int tiles = ((cx + TX - 1) / TX) * ((ct + TT - 1) / TT);
  dim3 grid((unsigned)tiles, (unsigned)((nrhs + 31) / 32));
  // 16-byte loads of column pairs need an even nc and a 16-byte aligned input
  const int pairs = (nc % 2 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0) ? 1 : 0;
  with_mode(mode, [&](auto m) {
    hipLaunchKernelGGL((k_coarse_mfma<decltype(m)::v, TX, TT, NW, S, TL>), grid, dim3(NW * 64), 0, st, L, x, y, cx,
                       ct, nc, nrhs, (float)c, (float)c2, xacc, aux, pairs, lscale);
  });
  HIPCHECK(hipGetLastError());
}

template <int TX, int TT, int NW, typename TL>
void launch_coarse_mfma_s(const TL* L, float ls, const z32* x, z32* y, int cx, int ct, int nc, int nrhs, int mode,
                          double c, double c2, z32* xacc, const z32* aux, hipStream_t st) {
  switch ((nc + 1) / 2) {
    case 1: launch_coarse_mfma_t<TX, TT, NW, 1>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
    case 2: launch_coarse_mfma_t<TX, TT, NW, 2>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
    case 3: launch_coarse_mfma_t<TX, TT, NW, 3>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
    case 4: launch_coarse_mfma_t<TX, TT, NW, 4>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
    case 5: launch_coarse_mfma_t<TX, TT, NW, 5>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
    case 6: launch_coarse_mfma_t<TX, TT, NW, 6>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
    case 7: launch_coarse_mfma_t<TX, TT, NW, 7>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
    default: launch_coarse_mfma_t<TX, TT, NW, 8>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st); break;
  }
}

template <int S, typename TL>
void launch_coarse_mfma_tw_s(const TL* L, float ls, const z32* x, z32* y, int cx, int ct, int nc, int nrhs, int mode,
                             double c, double c2, z32* xacc, const z32* aux, hipStream_t st, int ns, int seg) {
  const int nseg = (ct + seg - 1) / seg;
  dim3 grid((unsigned)(ns * nseg), (unsigned)((nrhs + 31) / 32));
  const int pairs = (nc % 2 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0) ? 1 : 0;
  with_mode(mode, [&](auto m) {
    hipLaunchKernelGGL((k_coarse_mfma_tw<decltype(m)::v, S, TL>), grid, dim3(512), 0, st, L, x, y, cx, ct, nc, nrhs,
                       (float)c, (float)c2, xacc, aux, pairs, ls, seg);
  });
  HIPCHECK(hipGetLastError());
}

// Rows per workgroup of the strip-walking kernel: about one workgroup per CU (256),
// an even number; 0 when that leaves fewer than 8 rows per workgroup (the window's
// two extra rows would then cost more than the overlap saves).
int mfma_tw_seg(int cx, int ct) {
  const int ns = (cx + 3) / 4;
  const int nseg = std::max(1, 256 / ns);
  int seg = (ct + nseg - 1) / nseg;
  seg += seg & 1;
  return seg >= 8 ? seg : 0;
}

// Strips (k_coarse_mfma_tw) where every workgroup gets at least 8 rows (128^2 coarse
// sites and up: the staging of V runs under the MFMAs; 128^2 sites, 32 RHS, FP16
// links: 142 us vs 167 us for 4x4 tiles); otherwise 4x4 tiles (8 waves, 152 KB of
// LDS) where they fill the chip, and on small coarse lattices 2x2 tiles (4 waves,
// 68 KB), which give four times the workgroups (32^2 sites, 32 RHS: 14 us vs 35 us).
// All three give bitwise the same results.
template <typename TL>
void launch_coarse_mfma_l(const TL* L, float ls, const z32* x, z32* y, int cx, int ct, int nc, int nrhs, int mode,
                          double c, z32* xacc, const z32* aux, hipStream_t st, double c2) {
  if (nc < 1 || nc > 16) throw Error(-1, "matrix-core coarse apply needs 1 <= nc <= 16");
  const long tiles44 = (long)((cx + 3) / 4) * ((ct + 3) / 4);
  const int seg = tiles44 >= 256 ? mfma_tw_seg(cx, ct) : 0;
  if (seg > 0) {
    const int ns = (cx + 3) / 4;
    switch ((nc + 1) / 2) {
      case 1: launch_coarse_mfma_tw_s<1>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
      case 2: launch_coarse_mfma_tw_s<2>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
      case 3: launch_coarse_mfma_tw_s<3>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
      case 4: launch_coarse_mfma_tw_s<4>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
      case 5: launch_coarse_mfma_tw_s<5>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
      case 6: launch_coarse_mfma_tw_s<6>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
      case 7: launch_coarse_mfma_tw_s<7>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
      default: launch_coarse_mfma_tw_s<8>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, ns, seg); break;
    }
  } else if (tiles44 < 256)
    launch_coarse_mfma_s<2, 2, 4>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
  else
    launch_coarse_mfma_s<4, 4, 8>(L, ls, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
}

void launch_coarse_mfma(const z32* L, const z32* x, z32* y, int cx, int ct, int nc, int nrhs, int mode, double c,
                        z32* xacc, const z32* aux, hipStream_t st, double c2) {
  launch_coarse_mfma_l<z32>(L, 1.0f, x, y, cx, ct, nc, nrhs, mode, c, xacc, aux, st, c2);
}

void launch_coarse_mfma_h16(const hfc* L, float lscale, const z32* x, z32* y, int cx, int ct, int nc, int nrhs,
                            int mode, double c, z32* xacc, const z32* aux, hipStream_t st, double c2) {
  launch_coarse_mfma_l<hfc>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, xacc, aux, st, c2);
}

// ---------------------------------------------------------------------------
// Multi-RHS FP64 coarse operator on the matrix cores (Eq. 2 for the FP64 solves
// of many right-hand sides).  One wave computes one coarse site K for 16 RT
// right-hand sides.  For each link direction D the complex product
// Y += L_{K,D} V_{K+D} is the real GEMM [Yr; Yi] += [[Lr, -Li], [Li, Lr]] [Vr; Vi]
// done with v_mfma_f64_16x16x4f64: the output rows are the nc <= 16 variables
// (one tile for Re, one for Im), the columns 16 right-hand sides, and K-step s
// covers link columns 4s..4s+3, against Vr and then against Vi.  Lane layout:
// A[i][k] from lane i + 16k, B[k][j] from lane j + 16k, accumulator r of lane l
// holds row 4r + l/16, column l%16 (checked on the device).  Every link is loaded once per 16 RT
// right-hand sides; the neighbours' vector entries are read straight from memory
// (the eight other sites that read them run close by, so they come from L2), the
// next direction's operands while this direction's MFMAs run (a deeper ring pinned
// by sched_barrier measured 20-45% slower: fewer waves per SIMD).  FP64 MFMA has the
// FP64 vector peak of this chip; what the matrix cores save is the broadcast of
// link and vector entries across lanes that a vector-ALU kernel needs.
// Site order: each XCD takes a band of ct/8 rows (its blocks are contiguous after
// xcd_tile) and walks it in strips `strip` sites wide, row by row within a strip, so
// that the rows above and below the sites in flight are still in that XCD's L2 when
// their entries are read again (in plain row order a row of 64-RHS entries, 16 KB
// per site, outgrows the L2 before the next row needs it).  strip = 0: row order.
// ---------------------------------------------------------------------------
template <int MODE, int RT>
__global__ void __launch_bounds__(256) k_coarse_mfma64(const z64* __restrict__ L, const z64* __restrict__ v,
                                                       z64* __restrict__ y, int cx, int ct, int nc, int nrhs,
                                                       double c, double c2, z64* __restrict__ xacc,
                                                       const z64* __restrict__ aux, int strip) {
  const int nK = cx * ct;
  const size_t n = (size_t)nK * nc;
  const int g = xcd_tile(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (g >= nK) return;  // wave-uniform, and no barrier follows
  int kx, kt;
  if (strip > 0) {
    const int H = ct / 8, chunk = H * cx;
    const int band = g / chunk, q = g - band * chunk;
    const int sidx = q / (strip * H), r = q - sidx * (strip * H);
    kt = band * H + r / strip;
    kx = sidx * strip + r % strip;
  } else {
    kx = g % cx;
    kt = g / cx;
  }
  const int K = kt * cx + kx;
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const int rhs0 = blockIdx.y * 16 * RT;
  const int irow = i < nc ? i : nc - 1;  // clamped: every lane loads a valid address, masked after
  const bool row_ok = i < nc;
  int rj[RT];
  bool rj_ok[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int r = rhs0 + 16 * rt + i;
    rj_ok[rt] = r < nrhs;
    rj[rt] = r < nrhs ? r : nrhs - 1;
  }
  auto load = [&](int D, z64 (&l)[4], z64 (&b)[RT][4]) {
    const int dt = D / 3 - 1, dx = D % 3 - 1;
    const int gx = ((kx + dx) % cx + cx) % cx, gt = ((kt + dt) % ct + ct) % ct;
    const size_t nb = (size_t)(gt * cx + gx) * nc;
    const z64* LD = L + (size_t)D * nc * n + (size_t)K * nc + irow;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int col = 4 * s + kq;
      const z64 t = LD[(size_t)(col < nc ? col : nc - 1) * n];
      const bool ok = row_ok && col < nc;
      l[s] = mk<double>(ok ? t.re : 0.0, ok ? t.im : 0.0);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const z64 u = v[(size_t)rj[rt] * n + nb + (col < nc ? col : nc - 1)];
        const bool uok = rj_ok[rt] && col < nc;
        b[rt][s] = mk<double>(uok ? u.re : 0.0, uok ? u.im : 0.0);
      }
    }
  };
  doublex4 accR[RT], accI[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      accR[rt][r] = 0.0;
      accI[rt][r] = 0.0;
    }
  z64 la[4], lb[4], ba[RT][4], bb[RT][4];
  load(0, la, ba);
#pragma unroll
  for (int D = 0; D < 9; ++D) {
    z64(&l)[4] = (D & 1) ? lb : la;
    z64(&b)[RT][4] = (D & 1) ? bb : ba;
    if (D < 8) load(D + 1, (D & 1) ? la : lb, (D & 1) ? ba : bb);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        accR[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(l[s].re, b[rt][s].re, accR[rt], 0, 0, 0);
        accR[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-l[s].im, b[rt][s].im, accR[rt], 0, 0, 0);
        accI[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(l[s].im, b[rt][s].re, accI[rt], 0, 0, 0);
        accI[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(l[s].re, b[rt][s].im, accI[rt], 0, 0, 0);
      }
  }
  // ---- epilogue: lane holds right-hand side rhs0 + 16 rt + i, variables 4 r + kq
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    if (!rj_ok[rt]) continue;
    const size_t ob = (size_t)rj[rt] * n + (size_t)K * nc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int dof = 4 * r + kq;
      if (dof >= nc) continue;
      const z64 sum = mk<double>(accR[rt][r], accI[rt][r]);
      const size_t o = ob + dof;
      if (MODE == 0) {
        y[o] = sum;
      } else if (MODE == 1 || MODE == 3) {
        const z64 vi = v[o];
        xacc[o] = MODE == 3 ? c * vi : xacc[o] + c * vi;
        y[o] = vi - c * sum;
      } else if (MODE == 4 || MODE == 5) {
        const z64 vi = v[o];
        const z64 a = MODE == 5 ? c * vi : xacc[o] + c * vi;
        xacc[o] = a + c2 * (vi - c * sum);
      } else {
        y[o] = aux[o] - sum;
      }
    }
  }
}

// 16, 32 or 64 right-hand sides per wave (one link load each), by the column count.
void launch_coarse_mfma64(const z64* L, const z64* x, z64* y, int cx, int ct, int nc, int nrhs, int mode, double c,
                          z64* xacc, const z64* aux, hipStream_t st, double c2) {
  if (nc < 1 || nc > 16) throw Error(-1, "FP64 matrix-core coarse apply needs 1 <= nc <= 16");
  if (nrhs < 1) return;
  const long nK = (long)cx * ct;
  const int rt = nrhs <= 16 ? 1 : (nrhs <= 32 ? 2 : 4);
  const dim3 grid((unsigned)((nK + 3) / 4), (unsigned)((nrhs + 16 * rt - 1) / (16 * rt)));
  // strips of 16 sites where the bands and strips tile the lattice exactly (every
  // block's four sites inside one band, the bands one per XCD)
  constexpr int kStrip = 16;
  const int strip = (nK % 32 == 0 && (nK / 4) % 8 == 0 && ct % 8 == 0 && cx % kStrip == 0) ? kStrip : 0;
  with_mode(mode, [&](auto m) {
    constexpr int M = decltype(m)::v;
    if (rt == 1)
      hipLaunchKernelGGL((k_coarse_mfma64<M, 1>), grid, dim3(256), 0, st, L, x, y, cx, ct, nc, nrhs, c, c2, xacc, aux,
                         strip);
    else if (rt == 2)
      hipLaunchKernelGGL((k_coarse_mfma64<M, 2>), grid, dim3(256), 0, st, L, x, y, cx, ct, nc, nrhs, c, c2, xacc, aux,
                         strip);
    else
      hipLaunchKernelGGL((k_coarse_mfma64<M, 4>), grid, dim3(256), 0, st, L, x, y, cx, ct, nc, nrhs, c, c2, xacc, aux,
                         strip);
  });
  HIPCHECK(hipGetLastError());
}

template <typename R, typename TL>
void launch_coarse_t(const TL* L, R lscale, const cpx<R>* x, cpx<R>* y, int cx, int ct, int nc, int nrhs, int mode,
                     double c, double c2, cpx<R>* xacc, const cpx<R>* aux, hipStream_t st, const Grp& g = Grp{}) {
  // one FP32 right-hand side: vector entries staged in LDS (in FP64 the 27 link loads and
  // the staged entries need twice the registers, and the plain kernel is faster); a
  // grouped launch takes it for every column, each with its own links
  if constexpr (std::is_same<R, float>::value) {
    if ((nrhs == 1 || g.op) && nc >= 4 && nc <= 16) {
      const size_t total = (size_t)cx * ct * nc;
      const dim3 grid((unsigned)((total + 63) / 64), nrhs);
      const int q = (nc + 3) / 4;
      with_mode(mode, [&](auto m) {
        constexpr int M = decltype(m)::v;
        auto go = [&](auto qq, auto gg) {  // the grouped variant is its own instantiation
          hipLaunchKernelGGL((k_coarse_sv<R, M, decltype(qq)::v, TL, decltype(gg)::v == 1>), grid, dim3(kThreads), 0,
                             st, L, x, y, cx, ct, nc, (R)c, (R)c2, xacc, aux, lscale, g);
        };
        auto by_g = [&](auto qq) {
          if (g.op) go(qq, IntC<1>{});
          else go(qq, IntC<0>{});
        };
        if (q == 1) by_g(IntC<1>{});
        else if (q == 2) by_g(IntC<2>{});
        else if (q == 3) by_g(IntC<3>{});
        else by_g(IntC<4>{});
      });
      HIPCHECK(hipGetLastError());
      return;
    }
  }
  if (g.op) throw Error(-1, "grouped coarse operator needs FP32 and 4 <= nc <= 16");
  if (nrhs == 1)
    launch_coarse_nr<R, 1, TL>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
  else if (nrhs <= 2)
    launch_coarse_nr<R, 2, TL>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
  else if (nrhs <= 4)
    launch_coarse_nr<R, 4, TL>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
  else
    launch_coarse_nr<R, 8, TL>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st);
}

template <typename R>
void launch_coarse(const cpx<R>* L, const cpx<R>* x, cpx<R>* y, int cx, int ct, int nc, int nrhs, int mode, double c,
                   cpx<R>* xacc, const cpx<R>* aux, hipStream_t st, double c2, const Grp& g) {
  launch_coarse_t<R, cpx<R>>(L, (R)1, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, g);
}

void launch_coarse_h16(const hfc* L, float lscale, const z32* x, z32* y, int cx, int ct, int nc, int nrhs, int mode,
                       double c, z32* xacc, const z32* aux, hipStream_t st, double c2, const Grp& g) {
  launch_coarse_t<float, hfc>(L, lscale, x, y, cx, ct, nc, nrhs, mode, c, c2, xacc, aux, st, g);
}

void launch_gs_append(double* P, const z64* v, int lx, int lt, int dof, int bx, int bt, int k, int ldk, int m,
                      int* fail, hipStream_t st) {
  const int cx = lx / bx, nK = cx * (lt / bt);
  const int nagg = bx * bt * dof;
  if ((m != 1 && m != 2) || (m == 2 && dof % 2) || m * (k + 1) > ldk)
    throw Error(-1, "Gram-Schmidt append: bad split or column index");
  dispatch_chunks((nagg + kThreads - 1) / kThreads, [&](auto c) {
    hipLaunchKernelGGL((k_gs_append<decltype(c)::v>), dim3(nK, m), dim3(kThreads), 0, st, (z64*)P, v, lx, dof, bx,
                       bt, cx, k, ldk, m, fail);
  });
  HIPCHECK(hipGetLastError());
}

void launch_color_scatter(const z64* P, z64* X, int lx, int lt, int dof, int bx, int bt, int h, int k, int ldk,
                          int cxc, int ctc, hipStream_t st) {
  const size_t n = (size_t)lx * lt * dof;
  hipLaunchKernelGGL(k_color_scatter, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, P, X,
                     lx, lt, dof, bx, bt, h, k, ldk, cxc, ctc);
  HIPCHECK(hipGetLastError());
}

void launch_color_project(const z64* P, const z64* Y, z64* L, int lx, int lt, int dof, int bx, int bt, int h, int nc,
                          int ldk, int k, int cxc, int ctc, hipStream_t st) {
  const int nK = (lx / bx) * (lt / bt);
  const int nw = (bx + 2 * h) * (bt + 2 * h) * dof;
  dispatch_chunks((nw + 63) / 64, [&](auto c) {
    hipLaunchKernelGGL((k_color_project<decltype(c)::v>), dim3((nK + 3) / 4), dim3(kThreads), 0, st, P, Y, L, lx,
                       lt, dof, bx, bt, h, nc, ldk, k, cxc, ctc);
  });
  HIPCHECK(hipGetLastError());
}

void launch_sa_extract(const z64* X, const z64* Y, z64* P, int lx, int lt, int dof, int bx, int bt, int k, int ldk,
                       int cxc, int ctc, double w, hipStream_t st) {
  const size_t total = (size_t)(lx / bx) * (lt / bt) * (bx + 2) * (bt + 2) * dof;
  hipLaunchKernelGGL(k_sa_extract, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, X, Y,
                     P, lx, lt, dof, bx, bt, k, ldk, cxc, ctc, w);
  HIPCHECK(hipGetLastError());
}

void launch_coarse_to_dense(const z64* L, z64* M, int cx, int ct, int nc, hipStream_t st) {
  const size_t n = (size_t)cx * ct * nc;
  hipLaunchKernelGGL(k_coarse_to_dense, dim3((unsigned)((n * n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                     L, M, cx, ct, nc);
  HIPCHECK(hipGetLastError());
}

void launch_gj_step(z64* M, int n, int k, z64* colk, double* piv, int* fail, hipStream_t st) {
  hipLaunchKernelGGL(k_gj_pivot, dim3((n + kThreads - 1) / kThreads), dim3(kThreads), 0, st, M, n, k, colk, piv,
                     fail);
  const size_t nn = (size_t)n * n;
  hipLaunchKernelGGL(k_gj_update, dim3((unsigned)((nn + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, M, n, k,
                     colk, piv);
  HIPCHECK(hipGetLastError());
}

// Y = M X with one wavefront per (row, column): lanes take j = lane, lane + 64, ...
// and the partial sums meet in a fixed butterfly.  For coarsest operators small
// enough to stay in the caches (n <= kDenseRowsMax) this fills the chip where the
// tiled kernel would launch a few dozen workgroups.
constexpr int kDenseRowsMax = 4096;

template <typename RM, typename R, typename TM = cpx<RM>>
__global__ void __launch_bounds__(kThreads) k_dense_rows(const TM* __restrict__ M, const cpx<R>* __restrict__ x,
                                                         cpx<R>* __restrict__ y, int n, double mscale, Grp g) {
  if (g.op) {  // grouped: this column's system
    M = static_cast<const TM*>(g.op[blockIdx.y]);
    mscale = g.s[blockIdx.y];
  }
  const int row = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const cpx<R>* xb = x + (size_t)blockIdx.y * n;
  const TM* Mr = M + (size_t)row * n;
  double re = 0, im = 0;
  constexpr int U = 8;  // row segments per group: their loads are in flight together (index clamped)
  for (int j0 = lane; j0 < n; j0 += 64 * U) {
    cpx<RM> m[U];
    cpx<R> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = min(j0 + 64 * u, n - 1);
      m[u] = widen(Mr[j]);
      v[u] = xb[j];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (j0 + 64 * u >= n) v[u] = mk<R>(0, 0);  // a clamped duplicate contributes nothing
      re = fma((double)m[u].re, (double)v[u].re, re);
      re = fma(-(double)m[u].im, (double)v[u].im, re);
      im = fma((double)m[u].re, (double)v[u].im, im);
      im = fma((double)m[u].im, (double)v[u].re, im);
    }
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) y[(size_t)blockIdx.y * n + row] = mk<R>((R)(mscale * re), (R)(mscale * im));
}

// k_dense_rows for n % 4 == 0: each lane reads four consecutive entries of the row
// (and of x) per load, and up to G such quads per lane are in flight together.  A
// wave takes RW consecutive rows and loads each quad of x once for all of them.
// Every lane adds its entries of a row in increasing order and masked (clamped)
// entries add an exact zero, so a row's result does not depend on G or RW.
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
  T e[4];
};

template <typename RM, typename R, typename TM, int G, int RW>
__global__ void __launch_bounds__(kThreads) k_dense_rows4(const TM* __restrict__ M, const cpx<R>* __restrict__ x,
                                                          cpx<R>* __restrict__ y, int n, double mscale, Grp g) {
  if (g.op) {  // grouped: this column's system
    M = static_cast<const TM*>(g.op[blockIdx.y]);
    mscale = g.s[blockIdx.y];
  }
  const int row0 = (blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)) * RW;
  const int lane = threadIdx.x & 63;
  if (row0 >= n) return;
  const int nq = n / 4;
  const Quad<TM>* Mr[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) Mr[r] = reinterpret_cast<const Quad<TM>*>(M + (size_t)min(row0 + r, n - 1) * n);
  const Quad<cpx<R>>* xb = reinterpret_cast<const Quad<cpx<R>>*>(x + (size_t)blockIdx.y * n);
  double re[RW], im[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) re[r] = im[r] = 0;
  for (int q0 = lane; q0 < nq; q0 += 64 * G) {
    Quad<TM> m[RW][G];
    Quad<cpx<R>> v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int q = min(q0 + 64 * u, nq - 1);  // clamped: all loads of the group in flight together
      v[u] = xb[q];
#pragma unroll
      for (int r = 0; r < RW; ++r) m[r][u] = Mr[r][q];
    }
    __builtin_amdgcn_sched_barrier(0);  // keeps every load of the group ahead of the first product
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool dup = q0 + 64 * u >= nq;  // a clamped duplicate contributes nothing
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const cpx<R> b = dup ? mk<R>(0, 0) : v[u].e[e];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
          const cpx<RM> a = widen(m[r][u].e[e]);
          re[r] = fma((double)a.re, (double)b.re, re[r]);
          re[r] = fma(-(double)a.im, (double)b.im, re[r]);
          im[r] = fma((double)a.re, (double)b.im, im[r]);
          im[r] = fma((double)a.im, (double)b.re, im[r]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    const double sr = wave_sum(re[r]), si = wave_sum(im[r]);
    if (lane == 0 && row0 + r < n) y[(size_t)blockIdx.y * n + row0 + r] = mk<R>((R)(mscale * sr), (R)(mscale * si));
  }
}

// The kernel is chosen by n alone, so a column's result never depends on nrhs.
// Y = M X on the matrix cores, FP32 (M stored as TM: z32 or scaled hfc), for the
// large coarsest inverses (n > kDenseRowsMax).  A workgroup owns 32 rows x 32
// right-hand sides; its four waves each take a quarter of the k range (a multiple
// of 4).  The complex product uses the real embedding of the coarse matrix-core
// kernel: per complex k two v_mfma_f32_32x32x2f32, A = [Mr, -Mi] into Re Y and
// A = [Mi, Mr] into Im Y, both against B = [Xr; Xi] (lane l supplies A[l%32][l/32]
// and B[l/32][l%32]; accumulator r of lane l is row 8(r/4) + 4(l/32) + r%4, column
// l%32).  Indices past n or nrhs are clamped for the loads, the tail of the k range
// is masked by a zero factor, and the partial sums of the four waves meet in LDS in
// a fixed order.  The k split depends on n only, so a column's result does not
// depend on nrhs.
template <typename TM>
__global__ void __launch_bounds__(256) k_dense_mfma(const TM* __restrict__ M, const z32* __restrict__ x,
                                                    z32* __restrict__ y, int n, int nrhs, float mscale) {
  __shared__ float red[3][2][16][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 31, half = lane >> 5;
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const TM* Mr = M + (size_t)min(r0 + i, n - 1) * n;
  const z32* Xc = x + (size_t)min(c0 + i, nrhs - 1) * n;
  const int kw = ((n + 15) / 16) * 4;  // k per wave, a multiple of 4
  const int kb = w * kw, ke = min(n, kb + kw);
  floatx16 accR, accI;
#pragma unroll
  for (int r = 0; r < 16; ++r) accR[r] = accI[r] = 0.f;
  // blocks of U complex k pass through a ring of D register blocks: the loads of a
  // block are issued D - 1 blocks before its products
  constexpr int U = 4, D = 4;
  TM mb[D][U];
  z32 vb[D][U];
  auto load = [&](int d, int k0) {
#pragma unroll
    for (int t = 0; t < U; ++t) {
      const int k = min(k0 + t, n - 1);
      mb[d][t] = Mr[k];
      vb[d][t] = Xc[k];
    }
  };
#pragma unroll
  for (int d = 0; d + 1 < D; ++d) load(d, kb + d * U);
  for (int k4 = kb; k4 < ke; k4 += D * U) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      load((d + D - 1) % D, k4 + (d + D - 1) * U);
      __builtin_amdgcn_sched_barrier(0);  // keep the refill where it is issued
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const z32 m = widen(mb[d][t]), v = vb[d][t];
        const float am = (k4 + d * U + t < ke) ? 1.f : 0.f;
        const float a_re = am * (half ? -m.im : m.re);
        const float a_im = am * (half ? m.re : m.im);
        const float b = half ? v.im : v.re;
        accR = __builtin_amdgcn_mfma_f32_32x32x2f32(a_re, b, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f32_32x32x2f32(a_im, b, accI, 0, 0, 0);
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      red[w - 1][0][r][lane] = accR[r];
      red[w - 1][1][r][lane] = accI[r];
    }
  }
  __syncthreads();
  if (w != 0) return;
  const int col = c0 + i;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = r0 + 8 * (r / 4) + 4 * half + (r % 4);
    const float re = ((accR[r] + red[0][0][r][lane]) + red[1][0][r][lane]) + red[2][0][r][lane];
    const float im = ((accI[r] + red[0][1][r][lane]) + red[1][1][r][lane]) + red[2][1][r][lane];
    if (row < n && col < nrhs) y[(size_t)col * n + row] = mk<float>(mscale * re, mscale * im);
  }
}

// Y = M X in FP64 on the matrix cores for the large coarsest inverses (n >
// kDenseRowsMax), the FP64 counterpart of k_dense_mfma.  A workgroup owns 32 rows x
// 32 right-hand sides as 2 x 2 tiles of v_mfma_f64_16x16x4f64 (layout of
// k_coarse_mfma64: A[i][k] from lane i + 16k, B[k][j] from lane j + 16k,
// accumulator r of lane l is row 4r + l/16, column l%16); per step of 4 complex k
// the real embedding takes four instructions per tile: Mr Xr and -Mi Xi into Re Y,
// Mi Xr and Mr Xi into Im Y.  The four waves each take a quarter of the k range (a
// multiple of 4, set by n alone) and meet in LDS in a fixed order, so a column's
// result does not depend on nrhs.  Operands of a step are loaded three steps ahead.
// The vectors are FP64, or FP32 (the FP64 inverse inside the FP32 V-cycle), widened
// on load and rounded on store.
template <typename R>
__global__ void __launch_bounds__(256) k_dense_mfma64(const z64* __restrict__ M, const cpx<R>* __restrict__ x,
                                                      cpx<R>* __restrict__ y, int n, int nrhs) {
  __shared__ double red[3][8][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, kq = lane >> 4;
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const z64* Mr[2] = {M + (size_t)min(r0 + i, n - 1) * n, M + (size_t)min(r0 + 16 + i, n - 1) * n};
  const cpx<R>* Xc[2] = {x + (size_t)min(c0 + i, nrhs - 1) * n, x + (size_t)min(c0 + 16 + i, nrhs - 1) * n};
  const int kw = ((n + 15) / 16) * 4;  // k per wave, a multiple of 4
  const int kb = w * kw, ke = min(n, kb + kw);
  doublex4 acc[2][2][2];  // [row tile][rhs tile][Re, Im]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][0][r] = acc[a][b][1][r] = 0.0;
  constexpr int D = 4;  // ring of steps in flight
  z64 mb[D][2];
  cpx<R> vb[D][2];
  auto load = [&](int d, int k0) {
    const int k = min(k0 + kq, n - 1);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      mb[d][t] = Mr[t][k];
      vb[d][t] = Xc[t][k];
    }
  };
#pragma unroll
  for (int d = 0; d + 1 < D; ++d) load(d, kb + 4 * d);
  for (int k4 = kb; k4 < ke; k4 += 4 * D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      load((d + D - 1) % D, k4 + 4 * (d + D - 1));
      __builtin_amdgcn_sched_barrier(0);  // keep the refill where it is issued
      const double am = (k4 + 4 * d + kq < ke) ? 1.0 : 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double mre = am * mb[d][a].re, mim = am * mb[d][a].im;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const z64 v = mk<double>((double)vb[d][b].re, (double)vb[d][b].im);
          acc[a][b][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(mre, v.re, acc[a][b][0], 0, 0, 0);
          acc[a][b][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(-mim, v.im, acc[a][b][0], 0, 0, 0);
          acc[a][b][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(mim, v.re, acc[a][b][1], 0, 0, 0);
          acc[a][b][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(mre, v.im, acc[a][b][1], 0, 0, 0);
        }
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[w - 1][q][r][lane] = acc[q >> 2][(q >> 1) & 1][q & 1][r];
  }
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = c0 + 16 * b + i;
      const int q = 4 * a + 2 * b;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + 16 * a + 4 * r + kq;
        const double re = ((acc[a][b][0][r] + red[0][q][r][lane]) + red[1][q][r][lane]) + red[2][q][r][lane];
        const double im =
            ((acc[a][b][1][r] + red[0][q + 1][r][lane]) + red[1][q + 1][r][lane]) + red[2][q + 1][r][lane];
        if (row < n && col < nrhs) y[(size_t)col * n + row] = mk<R>((R)re, (R)im);
      }
    }
}

// mscale: power-of-two scale of a reduced-precision M (1 otherwise), applied exactly.
template <typename RM, typename R, typename TM>
void launch_dense_apply_t(const TM* M, double mscale, const cpx<R>* x, cpx<R>* y, int n, int nrhs, hipStream_t st,
                          const Grp& grp = Grp{}) {
  if (grp.op && n > kDenseRowsMax) throw Error(-1, "grouped coarsest apply needs n <= 4096");
  if (n <= kDenseRowsMax && n % 4 == 0 && sizeof(TM) <= sizeof(z32)) {
    // FP16 or FP32 M: two rows per wave share the loads of x; groups of up to six
    // quads per row keep both rows' loads in flight (about 120 registers, four waves
    // per SIMD)
    const int want = (n / 4 + 63) / 64;
    const dim3 g((n + 7) / 8, nrhs);
    if (want <= 4)
      hipLaunchKernelGGL((k_dense_rows4<RM, R, TM, 4, 2>), g, dim3(kThreads), 0, st, M, x, y, n, mscale, grp);
    else
      hipLaunchKernelGGL((k_dense_rows4<RM, R, TM, (sizeof(TM) <= sizeof(hfc) ? 6 : 4), 2>), g, dim3(kThreads), 0,
                         st, M, x, y, n, mscale, grp);
  } else if (n <= kDenseRowsMax && n % 4 == 0) {
    // quads in flight per lane: all of a row of n <= 4096 in one group where registers allow
    constexpr int W = (int)((sizeof(TM) + sizeof(cpx<R>)) / 4);  // registers per entry pair
    constexpr int GMAX = W <= 3 ? 16 : (W <= 4 ? 8 : 4);
    const int want = (n / 4 + 63) / 64;
    const dim3 g((n + 3) / 4, nrhs);
    if (want <= 4 || GMAX == 4)
      hipLaunchKernelGGL((k_dense_rows4<RM, R, TM, 4, 1>), g, dim3(kThreads), 0, st, M, x, y, n, mscale, grp);
    else if (want <= 8 || GMAX == 8)
      hipLaunchKernelGGL((k_dense_rows4<RM, R, TM, 8, 1>), g, dim3(kThreads), 0, st, M, x, y, n, mscale, grp);
    else if (want <= 12)
      hipLaunchKernelGGL((k_dense_rows4<RM, R, TM, (GMAX > 8 ? 12 : 8), 1>), g, dim3(kThreads), 0, st, M, x, y, n,
                         mscale, grp);
    else
      hipLaunchKernelGGL((k_dense_rows4<RM, R, TM, (GMAX > 8 ? 16 : 8), 1>), g, dim3(kThreads), 0, st, M, x, y, n,
                         mscale, grp);
  } else if (n <= kDenseRowsMax) {
    hipLaunchKernelGGL((k_dense_rows<RM, R, TM>), dim3((n + 3) / 4, nrhs), dim3(kThreads), 0, st, M, x, y, n, mscale, grp);
  } else if constexpr (std::is_same<R, float>::value && !std::is_same<TM, z64>::value) {
    dim3 grid((unsigned)((n + 31) / 32), (unsigned)((nrhs + 31) / 32));
    hipLaunchKernelGGL((k_dense_mfma<TM>), grid, dim3(256), 0, st, M, x, y, n, nrhs, (float)mscale);
  } else {
    static_assert(std::is_same<TM, z64>::value || std::is_same<R, float>::value,
                  "an FP32 or FP16 inverse is applied to FP32 vectors only");
    dim3 grid((unsigned)((n + 31) / 32), (unsigned)((nrhs + 31) / 32));
    hipLaunchKernelGGL((k_dense_mfma64<R>), grid, dim3(256), 0, st, M, x, y, n, nrhs);
  }
  HIPCHECK(hipGetLastError());
}

template <typename RM, typename R>
void launch_dense_apply(const cpx<RM>* M, const cpx<R>* x, cpx<R>* y, int n, int nrhs, hipStream_t st,
                        const Grp& g) {
  launch_dense_apply_t<RM, R, cpx<RM>>(M, 1.0, x, y, n, nrhs, st, g);
}

void launch_dense_apply_h16(const hfc* M, double mscale, const z32* x, z32* y, int n, int nrhs, hipStream_t st,
                            const Grp& g) {
  launch_dense_apply_t<float, float, hfc>(M, mscale, x, y, n, nrhs, st, g);
}

void launch_random_gaussian(z64* v, size_t n, uint64_t seed, uint64_t stream_id, hipStream_t st) {
  hipLaunchKernelGGL(k_random_gaussian, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, v, n,
                     seed, stream_id);
  HIPCHECK(hipGetLastError());
}

void launch_links_export(const z64* L, z64* out, int nK, int nc, hipStream_t st) {
  const size_t total = (size_t)nK * 9 * nc * nc;
  hipLaunchKernelGGL(k_links_export, dim3((unsigned)((total + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, L,
                     out, nK, nc);
  HIPCHECK(hipGetLastError());
}

template <typename Ro>
void launch_links_convert(const z64* L, cpx<Ro>* out, size_t n, hipStream_t st) {
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL((k_copy_convert<Ro>), dim3((unsigned)g), dim3(kThreads), 0, st, L, out, n);
  HIPCHECK(hipGetLastError());
}

// Largest |re| or |im| of n complex values: per-block maxima into part[0 .. blocks).
__global__ void __launch_bounds__(kThreads) k_absmax_partial(const z64* __restrict__ a, size_t n,
                                                            double* __restrict__ part) {
  __shared__ double sh[kThreads / 64];
  double m = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    m = fmax(m, fmax(fabs(a[i].re), fabs(a[i].im)));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, sh[w]);
    part[blockIdx.x] = m;
  }
}

// out = FP16(in * inv_scale) (inv_scale a power of two, so only the FP16 rounding is inexact).
__global__ void k_convert_h16(const z64* __restrict__ in, hfc* __restrict__ out, size_t n, double inv_scale) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    hfc t;
    t.re = (_Float16)(in[i].re * inv_scale);
    t.im = (_Float16)(in[i].im * inv_scale);
    out[i] = t;
  }
}

void launch_absmax_partial(const z64* a, size_t n, double* part, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_absmax_partial, dim3(blocks), dim3(kThreads), 0, st, a, n, part);
  HIPCHECK(hipGetLastError());
}

void launch_convert_h16(const z64* in, hfc* out, size_t n, double inv_scale, hipStream_t st) {
  size_t g = (n + kThreads - 1) / kThreads;
  if (g > 65536) g = 65536;
  if (g == 0) return;
  hipLaunchKernelGGL(k_convert_h16, dim3((unsigned)g), dim3(kThreads), 0, st, in, out, n, inv_scale);
  HIPCHECK(hipGetLastError());
}

void launch_lincomb3(const z64* X, const z64* Y, const z64* Z, z64* out, double a, double b, double c, size_t n,
                     hipStream_t st) {
  const size_t g = std::min<size_t>((n + kThreads - 1) / kThreads, 8192);
  if (g == 0) return;
  hipLaunchKernelGGL(k_lincomb3, dim3((unsigned)g), dim3(kThreads), 0, st, X, Y, Z, out, a, b, c, n);
  HIPCHECK(hipGetLastError());
}

#define INST(R)                                                                                                  \
  template void launch_restrict<R>(const cpx<R>*, const cpx<R>*, cpx<R>*, int, int, int, int, int, int, int, int, \
                                   int, hipStream_t);                                                            \
  template void launch_prolong<R>(const cpx<R>*, const cpx<R>*, cpx<R>*, cpx<R>*, int, int, int, int, int, int,  \
                                  int, int, int, int, hipStream_t, bool, const Grp&);                            \
  template void launch_coarse<R>(const cpx<R>*, const cpx<R>*, cpx<R>*, int, int, int, int, int, double, cpx<R>*, \
                                 const cpx<R>*, hipStream_t, double, const Grp&);                                \
  template void launch_links_convert<R>(const z64*, cpx<R>*, size_t, hipStream_t);
INST(double)
INST(float)
#undef INST
template void launch_dense_apply<double, double>(const z64*, const z64*, z64*, int, int, hipStream_t, const Grp&);
template void launch_dense_apply<float, float>(const z32*, const z32*, z32*, int, int, hipStream_t, const Grp&);
template void launch_dense_apply<double, float>(const z64*, const z32*, z32*, int, int, hipStream_t, const Grp&);

}  // namespace smg
